"""Host interpreter of a library plan (test helper).

Executes the pass tables a plan exports (prx_plan_pass / _chunk /
_rotation) with numpy, workgroup by workgroup and coset by coset, using the
records exactly as the kernels receive them.  It shares no code with the
oracle or the HIP kernels, so agreement of all three pins the planner's
encodings (frames, bases, pivots, signs, scales) independently of the GPU.
"""
from __future__ import annotations

import math

import numpy as np

from paper_2504_17881_amd import prx as P


def _parity(a):
    return (np.bitwise_count(np.asarray(a, dtype=np.uint64)) & 1).astype(np.int64)


def _insert_zeros(t, pivots):
    t = np.asarray(t, dtype=np.uint64)
    for p in sorted(int(q) for q in pivots):
        p = np.uint64(p)
        one = np.uint64(1)
        lo = t & ((one << p) - one)
        t = ((t >> p) << (p + one)) | lo
    return t


def _xcomb(basis, m):
    X = [0] * (1 << m)
    for v in range(1, 1 << m):
        low = (v & -v).bit_length() - 1
        X[v] = X[v & (v - 1)] ^ int(basis[low])
    return X


def _apply_records(amp, recs, s0_of, m):
    """amp: list of 2^m complex arrays (same shape); recs: rotation records.

    Pair (a, b) of slot I (a without, b with bit I): a <- a + u ga s_b b, then
    b <- b + u gb s_a a with the new a (u = 1 or i, s the signs, ga and gb the
    records' tau_a and tau_b with the per-element sign s0)."""
    for r in recs:
        s0 = s0_of(r)
        ga = r["tau"] * (1.0 - 2.0 * s0)
        gb = r["tau_b"] * (1.0 - 2.0 * s0)
        unit = 1j if r["imag"] else 1.0
        zeta = r["zeta"]
        slot = r["slot"]
        if r["static_sign"] and slot != 15:
            # compiled variant: var = slot 2^m + imag 2^(m-1) + zp, tau_a
            # stored times (-1)^zeta_slot, pair sign (-1)^parity(c(v) & zp)
            var = r["var"]
            I, imag, zp = var >> m, (var >> (m - 1)) & 1, var & ((1 << (m - 1)) - 1)
            drop = lambda u: ((u >> (I + 1)) << I) | (u & ((1 << I) - 1))  # noqa: E731
            assert I == slot and imag == r["imag"] and zp == drop(zeta)
            for v in range(1 << m):
                if v >> I & 1:
                    continue
                w = v | (1 << I)
                sg = 1.0 - 2.0 * (bin(drop(v) & zp).count("1") & 1)
                amp[v] = amp[v] + unit * ga * sg * amp[w]
                amp[w] = amp[w] + unit * gb * sg * amp[v]
            continue
        if r["static_sign"]:
            assert r["var"] == m << m
        if slot == 15:
            for v in range(1 << m):
                sv = 1.0 - 2.0 * (bin(v & zeta).count("1") & 1)
                amp[v] = amp[v] + unit * ga * sv * amp[v]
            continue
        I = 1 << slot
        for v in range(1 << m):
            if v & I:
                continue
            w = v | I
            sv = 1.0 - 2.0 * (bin(v & zeta).count("1") & 1)
            sw = 1.0 - 2.0 * (bin(w & zeta).count("1") & 1)
            amp[v] = amp[v] + unit * ga * sw * amp[w]
            amp[w] = amp[w] + unit * gb * sv * amp[v]
    return amp


def _pending(fscale, m):
    """Factor of coset label v: the product of fscale over the bits set in v."""
    return [math.prod(fscale[i] for i in range(m) if v >> i & 1) for v in range(1 << m)]


def _plain(psi, n, r):
    x, z, phi = int(r["x"]), int(r["z"]), float(r["phi"])
    N = 1 << n
    k = np.arange(N, dtype=np.uint64)
    nY = bin(x & z).count("1")
    beta = (1j ** ((nY + 1) % 4)) * math.sin(phi)
    partner = k ^ np.uint64(x)
    sig_partner = 1.0 - 2.0 * _parity(partner & np.uint64(z))
    return math.cos(phi) * psi + beta * sig_partner * psi[partner]


def run_plan(plan: int, psi0: np.ndarray, n: int) -> np.ndarray:
    info = P.prx_plan_get_info(plan)
    rots = [P.prx_plan_rotation(plan, i) for i in range(info["kernel_rotations"])]
    psi = np.array(psi0, dtype=np.complex128, copy=True)
    pending = None
    for pi in range(info["passes"]):
        ps = P.prx_plan_pass(plan, pi)
        recs = rots[ps["rot_begin"]:ps["rot_begin"] + ps["rot_count"]]
        scale = ps["scale"]
        if ps["renorm_in"]:
            assert pending is not None
            scale *= pending
        if ps["kind"] == 3:
            # relabelling: index bit pos[j] of every amplitude moves to pos[dst[j]]
            assert ps["rot_count"] == 0
            pos, dst = ps["perm_pos"], ps["perm_dst"]
            assert sorted(dst) == list(range(12)) and pos == sorted(pos) and pos[:4] == [0, 1, 2, 3]
            k = np.arange(1 << n, dtype=np.uint64)
            kn = k.copy()
            for j in range(12):
                kn &= ~(np.uint64(1) << np.uint64(pos[j]))
            for j in range(12):
                bit = (k >> np.uint64(pos[j])) & np.uint64(1)
                kn |= bit << np.uint64(pos[dst[j]])
            out = np.empty_like(psi)
            out[kn.astype(np.int64)] = psi
            psi = out
            continue
        if ps["kind"] == 0:
            assert len(recs) == 1
            psi = _plain(psi, n, recs[0])
        elif ps["kind"] == 1:
            m = ps["m"]
            basis = ps["basis"][:m]
            k0 = _insert_zeros(np.arange(1 << (n - m), dtype=np.uint64), ps["pivot"][:m])
            X = _xcomb(basis, m)
            idx = [k0 ^ np.uint64(X[v]) for v in range(1 << m)]
            amp = [psi[i] for i in idx]
            amp = _apply_records(amp, recs, lambda r: _parity(k0 & np.uint64(r["zframe"])), m)
            F = _pending(ps["fscale"], m)
            for v in range(1 << m):
                psi[idx[v]] = amp[v] * (scale * F[v])
        else:
            B, b, g, m = ps["B"], ps["b"], ps["g"], ps["m"]
            nwg = 1 << (n - B)
            tb = _insert_zeros(np.arange(nwg, dtype=np.uint64), ps["tpivot"][:g])
            off = np.arange(1 << b, dtype=np.uint64)
            vcomb = [0] * (1 << g)  # XOR of the virtual masks selected by each tile of the set
            for vb in range(1, 1 << g):
                low = (vb & -vb).bit_length() - 1
                vcomb[vb] = vcomb[vb & (vb - 1)] ^ int(ps["vmask"][low])
            gidx = np.concatenate(
                [((tb ^ np.uint64(vcomb[vb]))[:, None] << np.uint64(b)) | off[None, :]
                 for vb in range(1 << g)], axis=1)  # (nwg, 2^B) global index of lds slot
            lds = psi[gidx]
            for c in range(ps["chunk_begin"], ps["chunk_begin"] + ps["chunk_count"]):
                ch = P.prx_plan_chunk(plan, c)
                k0 = np.asarray(_xcomb(ch["cvec"][:B - m], B - m), dtype=np.uint64)  # per thread
                X = _xcomb(ch["basis"][:m], m)
                idx = [k0 ^ np.uint64(X[v]) for v in range(1 << m)]
                # the threads' cosets partition the tile-set
                assert np.array_equal(np.sort(np.concatenate(idx)), np.arange(1 << B))
                amp = [lds[:, i.astype(np.int64)] for i in idx]
                crecs = rots[ch["rot_begin"]:ch["rot_begin"] + ch["rot_count"]]

                def s0_of(r, k0=k0):
                    return (_parity(k0 & np.uint64(r["zframe"]))[None, :] ^
                            _parity(tb & np.uint64(r["zhigh"]))[:, None])
                amp = _apply_records(amp, crecs, s0_of, m)
                F = _pending(ch["fscale"], m)
                for v in range(1 << m):
                    lds[:, idx[v].astype(np.int64)] = amp[v] * F[v]
            psi[gidx] = lds * scale
        if ps["norm_out"]:
            pending = 1.0 / math.sqrt(float(np.sum(np.abs(psi) ** 2)))
    return psi
