"""Host-side checks of the C ABI (no device calls): exported symbols, input
validation, schedules against the oracle's re-expansion, plan structure."""
import os
import re

import numpy as np
import pytest

import synth
from oracle import schedules as S
from paper_2504_17881_amd import prx as P

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    txt = open(os.path.join(ROOT, "include", "prx.h")).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(prx_[a-z0-9_]+)\s*\(", txt)))


def test_every_declared_function_is_exported():
    names = _declared()
    assert len(names) >= 35
    missing = [nm for nm in names if nm not in P.EXPORTED and not hasattr(P._lib, nm)]
    assert not missing, missing


def test_binding_names_match_abi():
    for nm in _declared():
        assert hasattr(P, nm), nm


def test_version_and_error_string():
    assert "gfx950" in P.prx_version()
    with pytest.raises(P.PrxError) as e:
        P.prx_ham_create(0, [1], [0], [1.0])
    assert e.value.status == P.PRX_ERR_INVALID
    assert "n must be" in P.prx_last_error()


@pytest.mark.parametrize("args,frag", [
    ((4, [1 << 4], [0], [1.0]), "beyond"),
    ((4, [1], [1 << 5], [1.0]), "beyond"),
    ((4, [1], [0], [float("nan")]), "non-finite"),
    ((64, [1], [0], [1.0]), "n must be"),
    ((4, [], [], []), "L must be"),
])
def test_ham_create_rejects(args, frag):
    with pytest.raises(P.PrxError) as e:
        P.prx_ham_create(*args)
    assert e.value.status == P.PRX_ERR_INVALID and frag in str(e.value)


def test_schedule_argument_checks():
    H = P.prx_ham_create(3, [1, 2], [0, 2], [0.5, -0.2])
    for bad in [lambda: P.prx_sched_trotter(H, 3, 1.0, 2),
                lambda: P.prx_sched_trotter(H, 1, 1.0, 0),
                lambda: P.prx_sched_trotter(H, 1, float("inf"), 2),
                lambda: P.prx_sched_qdrift(H, 1.0, 0, 1),
                lambda: P.prx_sched_partial(H, 3, 1.0, 1, 4, 1),
                lambda: P.prx_sched_partial(H, 1, 1.0, 1, 0, 1)]:
        with pytest.raises(P.PrxError) as e:
            bad()
        assert e.value.status == P.PRX_ERR_INVALID
    Z = P.prx_ham_create(3, [1], [0], [0.0])
    with pytest.raises(P.PrxError):
        P.prx_sched_qdrift(Z, 1.0, 4, 1)
    P.prx_ham_destroy(H)
    P.prx_ham_destroy(Z)


def test_lambda_matches_oracle():
    x, z, h = synth.jw_hamiltonian(10, 120, 5)
    H = P.prx_ham_create(10, x, z, h)
    assert P.prx_ham_lambda(H) == S.lambda_of(h)
    P.prx_ham_destroy(H)


@pytest.mark.parametrize("order", [1, 2])
@pytest.mark.parametrize("suffix", [False, True])
def test_trotter_schedule_equals_oracle(order, suffix):
    x, z, h = synth.jw_hamiltonian(12, 150, 6)
    H = P.prx_ham_create(12, x, z, h)
    s = P.prx_sched_trotter(H, order, 0.8, 3,
                            P.PRX_REORDER_SUFFIX if suffix else P.PRX_REORDER_NONE)
    n, rx, rz, rp = P.prx_sched_view(s)
    ox, oz, op = S.trotter(x, z, h, order, 0.8, 3, suffix=suffix)
    assert n == 12 and np.array_equal(rx, ox) and np.array_equal(rz, oz)
    assert np.array_equal(rp, op)
    P.prx_sched_destroy(s)
    P.prx_ham_destroy(H)


def test_qdrift_schedule_equals_oracle():
    x, z, h = synth.jw_hamiltonian(16, 500, 1016)
    H = P.prx_ham_create(16, x, z, h)
    for seed in (0, 1, 255):
        s = P.prx_sched_qdrift(H, 1.0, 2000, seed)
        _, rx, rz, rp = P.prx_sched_view(s)
        ox, oz, op = S.qdrift(x, z, h, 1.0, 2000, seed)
        assert np.array_equal(rx, ox) and np.array_equal(rz, oz) and np.array_equal(rp, op)
        P.prx_sched_destroy(s)
    P.prx_ham_destroy(H)


@pytest.mark.parametrize("suffix", [False, True])
def test_partial_schedule_equals_oracle(suffix):
    x, z, h = synth.jw_hamiltonian(14, 400, 3)
    H = P.prx_ham_create(14, x, z, h)
    s = P.prx_sched_partial(H, 40, 1.0, 3, 70, 9,
                            P.PRX_REORDER_SUFFIX if suffix else P.PRX_REORDER_NONE)
    _, rx, rz, rp = P.prx_sched_view(s)
    ox, oz, op = S.partial(x, z, h, 40, 1.0, 3, 70, 9, suffix=suffix)
    assert len(rx) == 3 * (80 + 70)
    assert np.array_equal(rx, ox) and np.array_equal(rz, oz) and np.array_equal(rp, op)
    P.prx_sched_destroy(s)
    P.prx_ham_destroy(H)


def test_from_rotations_roundtrip_and_checks():
    x, z, phi = synth.random_pauli_rotations(9, 50, 3)
    s = P.prx_sched_from_rotations(9, x, z, phi)
    n, rx, rz, rp = P.prx_sched_view(s)
    assert n == 9 and np.array_equal(rx, x) and np.array_equal(rz, z) and np.array_equal(rp, phi)
    P.prx_sched_destroy(s)
    with pytest.raises(P.PrxError):
        P.prx_sched_from_rotations(3, [8], [0], [0.1])
    with pytest.raises(P.PrxError):
        P.prx_sched_from_rotations(3, [1], [0], [float("nan")])


def test_plan_range_and_option_checks():
    x, z, phi = synth.random_pauli_rotations(10, 20, 3)
    s = P.prx_sched_from_rotations(10, x, z, phi)
    with pytest.raises(P.PrxError):
        P.prx_plan_create(s, 10, P.PRX_C64, 5, 4, P.PRX_FUSED)
    with pytest.raises(P.PrxError):
        P.prx_plan_create(s, 10, P.PRX_C64, 0, 21, P.PRX_FUSED)
    with pytest.raises(P.PrxError):
        P.prx_plan_create(s, 11, P.PRX_C64, 0, 20, P.PRX_FUSED)
    with pytest.raises(P.PrxError) as e:
        P.prx_plan_create(s, 10, P.PRX_C64, 0, 20, P.PRX_FUSED, dict(tile_qubits=9, chunk_rank=2))
    assert e.value.status == P.PRX_ERR_UNSUPPORTED
    pl = P.prx_plan_create(s, 10, P.PRX_C64, 3, 3, P.PRX_FUSED)
    assert P.prx_plan_get_info(pl)["passes"] == 0
    P.prx_plan_destroy(pl)
    # a workspace that is too small is rejected before any device call
    pl = P.prx_plan_create(s, 10, P.PRX_C128, 0, 20, P.PRX_FUSED)
    with pytest.raises(P.PrxError) as e:
        P.prx_plan_upload(pl, 256, ws_bytes=16)
    assert e.value.status == P.PRX_ERR_INVALID
    P.prx_plan_destroy(pl)
    P.prx_sched_destroy(s)


def test_plain_plan_is_one_pass_per_rotation():
    x, z, phi = synth.random_pauli_rotations(8, 30, 4)
    s = P.prx_sched_from_rotations(8, x, z, phi)
    pl = P.prx_plan_create(s, 8, P.PRX_C128, 0, 30, P.PRX_PLAIN)
    info = P.prx_plan_get_info(pl)
    assert info["passes"] == info["plain_passes"] == 30 and info["kernel_rotations"] == 30
    P.prx_plan_destroy(pl)
    P.prx_sched_destroy(s)


def test_autotune_cache_roundtrip(tmp_path):
    assert P.prx_autotune_lookup(7, P.PRX_C128) is None
    src = tmp_path / "tune.json"
    src.write_text('{\n  "gfx950/27/c64": {"tile_qubits": 12, "chunk_rank": 5, "max_fuse": 128, '
                   '"span_max": 3, "max_virtual": 2, "renorm_every": 1, "commuting": 0}\n}\n')
    P.prx_autotune_load(str(src))
    got = P.prx_autotune_lookup(27, P.PRX_C64)
    assert got["tile_qubits"] == 12 and got["chunk_rank"] == 5 and got["max_fuse"] == 128
    assert got["span_max"] == 3 and got["max_virtual"] == 2
    out = tmp_path / "out.json"
    P.prx_autotune_save(str(out))
    P.prx_autotune_load(str(out))
    assert P.prx_autotune_lookup(27, P.PRX_C64) == got
    # AUTO plans pick the cached setting up
    x, z, phi = synth.random_pauli_rotations(27, 10, 1)
    s = P.prx_sched_from_rotations(27, x, z, phi)
    pl = P.prx_plan_create(s, 27, P.PRX_C64, 0, 10, P.PRX_AUTO)
    info = P.prx_plan_get_info(pl)
    assert info["tile_qubits"] == 12 and info["chunk_rank"] == 5
    P.prx_plan_destroy(pl)
    P.prx_sched_destroy(s)
    with pytest.raises(P.PrxError):
        P.prx_autotune_load(str(tmp_path / "missing.json"))


def test_batch_create_host_checks():
    ns = [6, 8, 7]
    hams, scheds = [], []
    for i, n in enumerate(ns):
        x, z, h = synth.jw_hamiltonian(n, 30, 1000 + n)
        H = P.prx_ham_create(n, x, z, h)
        hams.append(H)
        scheds.append(P.prx_sched_qdrift(H, 1.0, 40, i))
    basis = [synth.basis_index(n) for n in ns]
    b = P.prx_batch_create(ns, scheds, P.PRX_C64, basis)
    assert P.prx_batch_workspace_bytes(b) > 0
    P.prx_batch_set_max_grid(b, 3)
    P.prx_batch_set_max_grid(b, 0)
    P.prx_batch_destroy(b)
    with pytest.raises(P.PrxError) as e:
        P.prx_batch_set_max_grid(None, 3)
    assert e.value.status == P.PRX_ERR_INVALID
    for bad_n, bad_b in [([6, 8, 5], basis), (ns, [0, 1 << 8, 0]), ([6, 9, 7], basis)]:
        with pytest.raises(P.PrxError) as e:
            P.prx_batch_create(bad_n, scheds, P.PRX_C64, bad_b)
        assert e.value.status == P.PRX_ERR_INVALID
    for s in scheds:
        P.prx_sched_destroy(s)
    for H in hams:
        P.prx_ham_destroy(H)


@pytest.mark.parametrize("dtype,B", [(P.PRX_C64, 12), (P.PRX_C128, 11)])
def test_batch_info_splits_samples_by_tile_frame(dtype, B):
    """Samples of at least B qubits are planned as tile-only plans with the
    batch's fixed options (exact commuting reorders on); the rest into span
    passes."""
    ns = [6, 10, 11, 12, 13, 14]
    hams, scheds = [], []
    for i, n in enumerate(ns):
        x, z, h = synth.jw_hamiltonian(n, 40, 1000 + n)
        H = P.prx_ham_create(n, x, z, h)
        hams.append(H)
        scheds.append(P.prx_sched_qdrift(H, 1.0, 150, i))
    basis = [synth.basis_index(n) for n in ns]
    b = P.prx_batch_create(ns, scheds, dtype, basis)
    info = P.prx_batch_get_info(b)
    P.prx_batch_destroy(b)
    assert info["samples"] == len(ns)
    assert info["tile_samples"] == sum(n >= B for n in ns)
    opts = dict(tile_qubits=B, chunk_rank=4, max_fuse=128, max_virtual=8, renorm_every=-1,
                tile_only=1, commuting=1)
    tile_passes, tile_sweeps, counts = 0, 0.0, []
    for n, s in zip(ns, scheds):
        if n < B:
            continue
        pl = P.prx_plan_create(s, n, dtype, 0, 150, P.PRX_FUSED, opts)
        k = P.prx_plan_get_info(pl)["passes"]
        P.prx_plan_destroy(pl)
        tile_passes += k
        tile_sweeps += k * 2.0 ** n
        counts.append(k)
    assert info["passes"] > tile_passes
    assert info["rounds"] >= max(counts)
    span_sweeps = info["amp_sweeps"] - tile_sweeps
    span_passes = info["passes"] - tile_passes
    small = [n for n in ns if n < B]
    # every span sample's sweeps are whole multiples of its size
    assert min(2.0 ** n for n in small) * span_passes <= span_sweeps
    assert span_sweeps <= max(2.0 ** n for n in small) * span_passes
    for s in scheds:
        P.prx_sched_destroy(s)
    for H in hams:
        P.prx_ham_destroy(H)


def test_rotation_jump_table_is_generated_from_its_script(tmp_path):
    """csrc/rot_jump_f32m4.inc is the output of csrc/gen_rot_jump.py, and
    every variant has 32 FMAs and one branch (the fixed stride the computed
    jump relies on)."""
    import importlib.util
    import shutil
    csrc = os.path.join(ROOT, "paper_2504_17881_amd", "csrc")
    shutil.copy(os.path.join(csrc, "gen_rot_jump.py"), tmp_path / "gen_rot_jump.py")
    spec = importlib.util.spec_from_file_location("gen_rot_jump", tmp_path / "gen_rot_jump.py")
    gen = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(gen)
    gen.main()
    for inc in ("rot_jump_f32m4.inc", "rot_jump_f64m4.inc"):
        with open(tmp_path / inc) as f, open(os.path.join(csrc, inc)) as g:
            assert f.read() == g.read(), inc
    f64 = gen.block("v_fma_f64")
    assert [x.replace("v_fma_f64", "v_fma_f32") for x in f64] == gen.block()
    lines = gen.block()
    start, end = lines.index("2:"), lines.index("3:")
    body = lines[start + 1:end]
    assert len(body) == 64 * 33
    for var in range(64):
        v = body[33 * var:33 * (var + 1)]
        assert all(x.startswith("v_fma_f32 ") for x in v[:32]) and v[32] == "s_branch 3f"
        # each amplitude register is written once (8 disjoint pairs)
        dst = [x.split()[1].rstrip(",") for x in v[:32]]
        assert sorted(dst) == sorted(f"%{i}" for i in range(32))
    assert lines[0] == "s_min_u32 %32, %35, 63" and gen.VARIANT_BYTES == 260
    # the threaded loop: each variant loads the next record, applies the same
    # FMAs as the table's variant, tests the count and dispatches the next
    # record itself
    with open(tmp_path / "rot_loop_f32m4.inc") as f, open(os.path.join(csrc, "rot_loop_f32m4.inc")) as g:
        assert f.read() == g.read()
    loop = gen.loop_block()
    start, end = loop.index("2:"), loop.index("9:")
    body = loop[start + 1:end]
    n = len(body) // 64
    assert len(body) == 64 * n and gen.LOOP_VARIANT_BYTES == 380
    dispatch = gen._dispatch("(2b - 1b)", "-1")
    for var in range(64):
        v = body[n * var:n * (var + 1)]
        assert v[0] == "s_load_dwordx8 s[80:87], s[76:77], 0x0"
        assert [x.replace("%[ga]", "%33").replace("%[gb]", "%34") for x in v[1:33]] == \
            gen.variant(var)[:32]
        assert v[33:36] == ["s_cmp_eq_u32 s78, 0", "s_cbranch_scc1 9f", "s_waitcnt lgkmcnt(0)"]
        assert v[36:] == dispatch
    # the diagonal variant index leaves before the jump; the count is tested
    # on entry and after every rotation
    assert dispatch.index("s_cmp_eq_u32 s88, 64") < dispatch.index("s_setpc_b64 s[90:91]")
    assert loop[3:5] == ["s_cmp_eq_u32 s78, 0", "s_cbranch_scc1 9f"]
    # the complex128 loop: same structure with both record loads and f64 FMAs
    with open(tmp_path / "rot_loop_f64m4.inc") as f, open(os.path.join(csrc, "rot_loop_f64m4.inc")) as g:
        assert f.read() == g.read()
    loop = gen.loop_block64()
    body = loop[loop.index("2:") + 1:loop.index("9:")]
    n = len(body) // 64
    assert len(body) == 64 * n and gen.LOOP64_VARIANT_BYTES == 404
    dispatch = gen._dispatch64("(2b - 1b)", "-1")
    for var in range(64):
        v = body[n * var:n * (var + 1)]
        assert v[:2] == ["s_load_dwordx8 s[80:87], s[76:77], 0x0",
                         "s_load_dwordx2 s[92:93], s[76:77], 0x20"]
        assert [x.replace("%[ga]", "%33").replace("%[gb]", "%34") for x in v[2:34]] == \
            gen.variant(var, "v_fma_f64")[:32]
        assert v[34:37] == ["s_cmp_eq_u32 s78, 0", "s_cbranch_scc1 9f", "s_waitcnt lgkmcnt(0)"]
        assert v[37:] == dispatch
    assert "s_add_u32 s76, s76, 40" in dispatch


def _code_object(tmp_path, obj_name):
    """The gfx950 code object of one built translation unit, extracted from
    its offload bundle (objects built in this tree)."""
    import subprocess
    build = os.path.join(ROOT, "paper_2504_17881_amd", "_build")
    obj = os.path.join(build, obj_name)
    src = os.path.join(ROOT, "paper_2504_17881_amd", "csrc", obj_name[:-2])
    if not os.path.exists(obj) or os.path.getmtime(obj) < os.path.getmtime(src):
        from paper_2504_17881_amd import build as pb
        pb.build()
    llvm = "/opt/rocm/llvm/bin"
    fat = tmp_path / (obj_name + ".fatbin")
    co = tmp_path / (obj_name + ".co")
    subprocess.run([f"{llvm}/llvm-objcopy", f"--dump-section=.hip_fatbin={fat}", obj,
                    str(tmp_path / "scratch.o")], check=True)
    subprocess.run([f"{llvm}/clang-offload-bundler", "--unbundle", "--type=o",
                    f"--input={fat}", "--targets=hipv4-amdgcn-amd-amdhsa--gfx950",
                    f"--output={co}"], check=True)
    out = subprocess.run([f"{llvm}/llvm-objdump", "-d", "--no-show-raw-insn", str(co)],
                         check=True, capture_output=True, text=True).stdout
    ins = []
    for line in out.splitlines():
        m = re.match(r"\s+(\S.*?)\s*//\s*([0-9A-Fa-f]+):", line)
        if m:
            ins.append((int(m.group(2), 16), m.group(1).split()[0], m.group(1)))
    return ins


def _branch_target(ins, j):
    """Target address of the SOPP branch at instruction j (simm16 in dwords,
    relative to the next instruction)."""
    off = int(ins[j][2].split()[-1], 0)
    if off >= 1 << 15:
        off -= 1 << 16
    return ins[j][0] + 4 + 4 * off


@pytest.mark.parametrize("obj_name", ["kernels.hip.o", "batch.hip.o"])
def test_rotation_jump_table_layout_in_built_code(tmp_path, obj_name):
    """Every instance of the computed jump in the built gfx950 code: the
    table starts right after s_setpc_b64 and the jump adds (table - return
    address) and stride * min(var, 63) to the return address.  In the
    jump table (stride 260) variant v is 32 eight-byte v_fma_f32 and one
    s_branch to the table's end; in the threaded loops (stride 380 at
    complex64, 404 at complex128) it is the next record's scalar load(s),
    32 FMAs, the count test with its exit, the wait and the next record's
    dispatch, whose computed jump returns to the same table, and every exit
    of the loop lands on the same address.  A different encoding size would send
    the jump into the middle of an instruction."""
    ins = _code_object(tmp_path, obj_name)
    addr = [a for a, _, _ in ins]
    at = {a: i for i, a in enumerate(addr)}
    tables = [i for i, (_, op, txt) in enumerate(ins) if op == "s_setpc_b64" and "s[90:91]" in txt]
    kinds = {260: 0, 380: 0, 404: 0}
    for i in tables:
        # preamble: s_min_u32, s_mul_i32 stride, s_getpc_b64, s_add/addc (var),
        # s_add/addc (label offset), s_setpc_b64
        pre = [op for _, op, _ in ins[i - 7:i + 1]]
        assert pre == ["s_min_u32", "s_mul_i32", "s_getpc_b64", "s_add_u32", "s_addc_u32",
                       "s_add_u32", "s_addc_u32", "s_setpc_b64"], pre
        assert ins[i - 7][2].endswith(", 63")
        stride = int(ins[i - 6][2].rsplit(",", 1)[1].strip(), 0)
        assert stride in kinds, stride
        ret = addr[i - 4]                       # s_getpc_b64 yields the next address
        off = int(ins[i - 2][2].rsplit(",", 1)[1].strip(), 0)
        if off >= 1 << 31:
            off -= 1 << 32
        if stride in (380, 404) and off < 0:
            continue                            # a variant's dispatch (checked below)
        kinds[stride] += 1
        start = addr[i + 1]
        assert ret + off == start, (hex(ret), off, hex(start))
        end = start + 64 * stride
        assert end in at
        if stride == 260:
            fma = ins[at[start]][1]             # complex64 or complex128 table
            assert fma in ("v_fma_f32", "v_fma_f64"), ins[at[start]]
            kinds[fma] = kinds.get(fma, 0) + 1
            for var in range(64):
                base = start + 260 * var
                for k in range(32):
                    j = at[base + 8 * k]
                    assert ins[j][1] == fma, (var, k, ins[j])
                j = at[base + 256]
                assert ins[j][1] == "s_branch" and _branch_target(ins, j) == end, (var, ins[j])
                assert addr[j + 1] == base + 260
            continue
        # threaded loop: the header's jump starts the table; every variant
        # is the next record's load(s), 32 FMAs, the count test with its
        # exit, the wait and a dispatch whose computed jump targets the same
        # table (complex64: stride 380, one load; complex128: 404, two)
        f64 = stride == 404
        hexits = [j for j in range(i - 40, i) if ins[j][1] == "s_cbranch_scc1"]
        assert len(hexits) == 2 and all(_branch_target(ins, j) == end for j in hexits)
        lead = 16 if f64 else 8
        for var in range(64):
            base = start + stride * var
            j = at[base]
            assert ins[j][1] == "s_load_dwordx8" and "s[80:87], s[76:77]" in ins[j][2], ins[j]
            if f64:
                assert ins[j + 1][1] == "s_load_dwordx2" and "s[92:93], s[76:77], 0x20" in ins[j + 1][2]
            for k in range(32):
                j = at[base + lead + 8 * k]
                assert ins[j][1] == ("v_fma_f64" if f64 else "v_fma_f32"), (var, k, ins[j])
            j = at[base + lead + 256]
            assert ins[j][1] == "s_cmp_eq_u32" and ins[j][2].endswith("s78, 0"), ins[j]
            assert ins[j + 1][1] == "s_cbranch_scc1" and _branch_target(ins, j + 1) == end
            assert ins[j + 2][1] == "s_waitcnt"
            assert [op for _, op, _ in ins[j + 3:j + 6]] == ["s_bfe_u32", "s_cmp_eq_u32",
                                                          "s_cbranch_scc1"]
            assert _branch_target(ins, j + 5) == end          # diagonal record: exit
            k = j + (25 if f64 else 22)
            assert [op for _, op, _ in ins[k - 7:k + 1]] == [
                "s_min_u32", "s_mul_i32", "s_getpc_b64", "s_add_u32", "s_addc_u32", "s_add_u32",
                "s_addc_u32", "s_setpc_b64"]
            assert ins[k - 7][2].endswith(", 63")
            assert int(ins[k - 6][2].rsplit(",", 1)[1].strip(), 0) == stride
            o2 = int(ins[k - 2][2].rsplit(",", 1)[1].strip(), 0)
            if o2 >= 1 << 31:
                o2 -= 1 << 32
            assert addr[k - 4] + o2 == start and ins[k - 1][2].endswith("-1")
            assert addr[k + 1] == base + stride
    assert kinds[380] >= 1 and kinds[404] >= 1, kinds
    if obj_name == "kernels.hip.o":
        assert kinds.get("v_fma_f32", 0) >= 1 and kinds.get("v_fma_f64", 0) >= 1, kinds


def test_launch_grids_stay_inside_the_work_item_range():
    """Every pass's launch (blocks x threads) stays below 2^32 work-items at
    the largest states: Z-only terms (diagonal sweeps), two-rotation spans and
    tile passes at n = 34 and 35, both precisions."""
    rng = np.random.default_rng(5)
    for n in (34, 35):
        x = [0, 0, 1 << (n - 1), (1 << (n - 1)) | 1, 3, 1 << (n - 2), 0b101]
        z = [1, (1 << n) - 1, 0, 1 << (n - 3), 0, 2, 0b111]
        phi = list(rng.uniform(-0.5, 0.5, size=len(x)))
        s = P.prx_sched_from_rotations(n, x, z, phi)
        for dt in (P.PRX_C64, P.PRX_C128):
            for kern, opts in ((P.PRX_PLAIN, None), (P.PRX_FUSED, None),
                               (P.PRX_FUSED, dict(span_max=1)), (P.PRX_FUSED, dict(span_max=2)),
                               (P.PRX_FUSED, dict(tile_qubits=10, chunk_rank=3))):
                pl = P.prx_plan_create(s, n, dt, 0, len(x), kern, opts)
                for i in range(P.prx_plan_get_info(pl)["passes"]):
                    ps = P.prx_plan_pass(pl, i)
                    assert 0 < ps["grid_blocks"] <= 1 << 22
                    assert ps["grid_blocks"] * ps["block_threads"] < 1 << 32, (n, dt, ps)
                P.prx_plan_destroy(pl)
        P.prx_sched_destroy(s)


def test_lambda_is_the_sum_of_magnitudes():
    """lambda = sum |h_l| (Methods, "Hamiltonian simulation"), pinned to exact
    values: dyadic coefficients whose magnitudes sum exactly, signs that a
    dropped absolute value would cancel, and random coefficients against
    math.fsum (correctly rounded) within the left-to-right rounding bound."""
    import math
    from oracle import schedules as S
    h = [0.5, -0.25, 0.125, -0.0625, 1.0, -2.0]
    assert S.lambda_of(h) == 3.9375
    H = P.prx_ham_create(3, [1, 2, 3, 4, 5, 6], [0] * 6, h)
    assert P.prx_ham_lambda(H) == 3.9375
    P.prx_ham_destroy(H)
    rng = np.random.default_rng(11)
    h = rng.normal(size=500) * np.exp(rng.normal(-4, 2, size=500))
    exact = math.fsum(abs(v) for v in h)
    bound = 500 * 2.0 ** -53 * exact
    assert abs(S.lambda_of(h) - exact) <= bound
    H = P.prx_ham_create(10, np.arange(1, 501) % 1024, np.zeros(500, np.uint64), h)
    assert abs(P.prx_ham_lambda(H) - exact) <= bound
    P.prx_ham_destroy(H)


def test_binding_rejects_mismatched_state_tensors():
    """The binding checks a state tensor before its address crosses the ABI:
    dtype, element count, contiguity and device (CPU tensors here stand in
    for every case; the device check comes last)."""
    import torch
    ws = torch.empty(256, dtype=torch.uint8)
    with pytest.raises(TypeError, match="does not match complex64"):
        P.prx_norm2(torch.zeros(16, dtype=torch.complex128), 4, P.PRX_C64, ws)
    with pytest.raises(TypeError, match="does not match complex128"):
        P.prx_amplitude(torch.zeros(16, dtype=torch.complex64), 4, P.PRX_C128, 0)
    with pytest.raises(ValueError, match="expected 2"):
        P.prx_amplitude(torch.zeros(8, dtype=torch.complex64), 4, P.PRX_C64, 0)
    with pytest.raises(ValueError, match="not contiguous"):
        P.prx_amplitude(torch.zeros(32, dtype=torch.complex64)[::2], 4, P.PRX_C64, 0)
    with pytest.raises(ValueError, match="not on a GPU"):
        P.prx_amplitude(torch.zeros(16, dtype=torch.complex64), 4, P.PRX_C64, 0)
    with pytest.raises(ValueError, match="psi0"):
        P.prx_overlap(torch.zeros(16, dtype=torch.complex64), 0, 4, P.PRX_C64, 0)
    s = P.prx_sched_from_rotations(4, [1], [0], [0.1])
    pl = P.prx_plan_create(s, 4, P.PRX_C128, 0, 1, P.PRX_FUSED)
    info = P.prx_plan_get_info(pl)
    assert info["n"] == 4 and info["dtype"] == P.PRX_C128
    with pytest.raises(TypeError, match="does not match complex128"):
        P.prx_plan_execute(pl, torch.zeros(16, dtype=torch.complex64), ws)
    with pytest.raises(ValueError, match="expected 2"):
        P.prx_apply_range(torch.zeros(32, dtype=torch.complex128), 4, P.PRX_C128, s, 0, 1,
                          P.PRX_FUSED, ws)
    P.prx_plan_destroy(pl)
    b = P.prx_batch_create([6, 7], [P.prx_sched_from_rotations(6, [1], [0], [0.1]),
                                    P.prx_sched_from_rotations(7, [1], [0], [0.1])],
                           P.PRX_C64, [0, 0])
    with pytest.raises(ValueError, match="sample 1"):
        P.prx_batch_upload(b, [0, torch.zeros(64, dtype=torch.complex64)], ws)
    with pytest.raises(ValueError, match="2 states for 1"):
        P.prx_batch_run([0, 0], [6], [s], P.PRX_C64, [0], ws)
    P.prx_batch_destroy(b)
    P.prx_sched_destroy(s)


def test_max_grid_caps_every_sweep_launch():
    n = 16
    x, z, phi = synth.random_pauli_rotations(n, 80, seed=4)
    s = P.prx_sched_from_rotations(n, x, z, phi)
    for kernel, opts in ((P.PRX_PLAIN, dict(max_grid=3)),
                         (P.PRX_FUSED, dict(tile_qubits=10, chunk_rank=4, max_grid=5)),
                         (P.PRX_FUSED, dict(max_grid=1 << 30))):
        pl = P.prx_plan_create(s, n, P.PRX_C64, 0, 80, kernel, opts)
        info = P.prx_plan_get_info(pl)
        cap = min(opts["max_grid"], 1 << 22)
        for i in range(info["passes"]):
            assert 1 <= P.prx_plan_pass(pl, i)["grid_blocks"] <= cap
        P.prx_plan_destroy(pl)
    P.prx_sched_destroy(s)
