"""ctypes binding of ``libprx.so`` with the C ABI's names (include/prx.h).

Argument marshalling only: every computation runs in the library.  Device
buffers may be given as torch tensors (their ``data_ptr()`` is passed) or
as integer addresses; streams as ``torch.cuda.Stream`` objects, raw
integers, or None (the default stream).  A non-OK status raises
``PrxError`` carrying the library's message.

A state given as a tensor is checked before its address crosses the ABI:
it must be a contiguous GPU tensor of 2^n elements whose dtype matches the
prx dtype (complex64 for PRX_C64, complex128 for PRX_C128); workspaces must
be contiguous GPU tensors.  Violations raise TypeError or ValueError.
Integer addresses are passed as given.

The library must have been built (``python -m paper_2504_17881_amd.build``);
importing this module without it raises immediately.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "lib", "libprx.so")

PRX_OK, PRX_ERR_INVALID, PRX_ERR_OOM, PRX_ERR_HIP, PRX_ERR_UNSUPPORTED = 0, 1, 2, 3, 4
PRX_C64, PRX_C128 = 1, 2
PRX_PLAIN, PRX_FUSED, PRX_AUTO = 0, 1, 2
PRX_REORDER_NONE, PRX_REORDER_COMMUTING, PRX_REORDER_SUFFIX = 0, 1, 2

_STATUS = {0: "PRX_OK", 1: "PRX_ERR_INVALID", 2: "PRX_ERR_OOM", 3: "PRX_ERR_HIP",
           4: "PRX_ERR_UNSUPPORTED"}


class PrxError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{_STATUS.get(status, status)}: {msg}")
        self.status = status


if not os.path.exists(LIB_PATH):
    raise ImportError(f"{LIB_PATH} is missing: build it with "
                      "`python -m paper_2504_17881_amd.build` (no CPU fallback exists)")

# PyTorch ships its own HIP runtime (same soname).  Load it first so that
# libprx.so binds to that one runtime: device pointers and streams from torch
# are then valid in the library.
try:
    import torch  # noqa: F401
except ImportError:  # the C ABI also works without torch (raw addresses)
    torch = None

_lib = ctypes.CDLL(LIB_PATH)

_u64p = ctypes.POINTER(ctypes.c_uint64)
_dp = ctypes.POINTER(ctypes.c_double)
_vp = ctypes.c_void_p
_sz = ctypes.c_size_t


class prx_plan_opts(ctypes.Structure):
    _fields_ = [("tile_qubits", ctypes.c_int), ("chunk_rank", ctypes.c_int),
                ("max_fuse", ctypes.c_int), ("span_max", ctypes.c_int),
                ("max_virtual", ctypes.c_int), ("renorm_every", ctypes.c_int),
                ("commuting", ctypes.c_int), ("tile_only", ctypes.c_int),
                ("relabel", ctypes.c_int), ("max_grid", ctypes.c_int)]


class prx_plan_info(ctypes.Structure):
    _fields_ = [("rotations", _sz), ("kernel_rotations", _sz), ("passes", _sz),
                ("plain_passes", _sz), ("span_passes", _sz), ("tile_passes", _sz),
                ("workspace_bytes", _sz), ("mean_fuse", ctypes.c_double),
                ("tile_qubits", ctypes.c_int), ("chunk_rank", ctypes.c_int),
                ("n", ctypes.c_int), ("dtype", ctypes.c_int),
                ("relabel_passes", _sz)]


class prx_pass_info(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int), ("rot_begin", _sz), ("rot_count", _sz),
                ("chunk_begin", _sz), ("chunk_count", _sz),
                ("B", ctypes.c_int), ("b", ctypes.c_int), ("g", ctypes.c_int),
                ("m", ctypes.c_int),
                ("basis", ctypes.c_uint64 * 6), ("pivot", ctypes.c_uint32 * 6),
                ("vmask", ctypes.c_uint64 * 10), ("tpivot", ctypes.c_uint32 * 10),
                ("scale", ctypes.c_double), ("fscale", ctypes.c_double * 6),
                ("norm_out", ctypes.c_int), ("renorm_in", ctypes.c_int),
                ("grid_blocks", ctypes.c_uint), ("block_threads", ctypes.c_uint),
                ("perm_pos", ctypes.c_uint32 * 12), ("perm_dst", ctypes.c_uint32 * 12)]


class prx_chunk_info(ctypes.Structure):
    _fields_ = [("basis", ctypes.c_uint32 * 6), ("cvec", ctypes.c_uint32 * 10),
                ("fscale", ctypes.c_double * 6), ("rot_begin", _sz), ("rot_count", _sz)]


class prx_rot_info(ctypes.Structure):
    _fields_ = [("x", ctypes.c_uint64), ("z", ctypes.c_uint64), ("phi", ctypes.c_double),
                ("source", _sz), ("zframe", ctypes.c_uint64), ("zhigh", ctypes.c_uint64),
                ("slot", ctypes.c_uint32), ("imag", ctypes.c_uint32),
                ("zeta", ctypes.c_uint32), ("var", ctypes.c_uint32),
                ("static_sign", ctypes.c_uint32), ("tau", ctypes.c_double),
                ("tau_b", ctypes.c_double)]


def _sig(name, res, *args):
    f = getattr(_lib, name)
    f.restype = res
    f.argtypes = list(args)
    return f


_i = ctypes.c_int
_st = ctypes.c_int
_sig("prx_last_error", ctypes.c_char_p)
_sig("prx_version", ctypes.c_char_p)
_sig("prx_ham_create", _st, _i, _sz, _u64p, _u64p, _dp, ctypes.POINTER(_vp))
_sig("prx_ham_destroy", None, _vp)
_sig("prx_ham_lambda", _st, _vp, _dp)
_sig("prx_sched_trotter", _st, _vp, _i, ctypes.c_double, _i, _i, ctypes.POINTER(_vp))
_sig("prx_sched_qdrift", _st, _vp, ctypes.c_double, _sz, ctypes.c_uint64, ctypes.POINTER(_vp))
_sig("prx_sched_partial", _st, _vp, _sz, ctypes.c_double, _i, _sz, ctypes.c_uint64, _i,
     ctypes.POINTER(_vp))
_sig("prx_sched_from_rotations", _st, _i, _sz, _u64p, _u64p, _dp, ctypes.POINTER(_vp))
_sig("prx_sched_view", _st, _vp, ctypes.POINTER(_i), ctypes.POINTER(_sz),
     ctypes.POINTER(_u64p), ctypes.POINTER(_u64p), ctypes.POINTER(_dp))
_sig("prx_sched_destroy", None, _vp)
_sig("prx_plan_create", _st, _vp, _i, _i, _sz, _sz, _i, ctypes.POINTER(prx_plan_opts),
     ctypes.POINTER(_vp))
_sig("prx_plan_get_info", _st, _vp, ctypes.POINTER(prx_plan_info))
_sig("prx_plan_destroy", None, _vp)
_sig("prx_plan_upload", _st, _vp, _vp, _sz, _vp)
_sig("prx_plan_execute", _st, _vp, _vp, _vp, _sz, _vp)
_sig("prx_plan_execute_timed", _st, _vp, _vp, _vp, _sz, _vp, ctypes.POINTER(ctypes.c_float),
     ctypes.POINTER(ctypes.c_float))
_sig("prx_plan_pass", _st, _vp, _sz, ctypes.POINTER(prx_pass_info))
_sig("prx_plan_chunk", _st, _vp, _sz, ctypes.POINTER(prx_chunk_info))
_sig("prx_plan_rotation", _st, _vp, _sz, ctypes.POINTER(prx_rot_info))
_sig("prx_workspace_bytes", _sz, _i, _i, _vp, _i)
_sig("prx_apply_range", _st, _vp, _i, _i, _vp, _sz, _sz, _i, _vp, _sz, _vp)
_sig("prx_apply_range_static", _st, _vp, _i, _i, _vp, _sz, _sz, _i, _vp)
_sig("prx_reduce_workspace_bytes", _sz, _i)
_sig("prx_overlap", _st, _vp, _vp, _i, _i, _dp, _vp, _sz, _vp)
_sig("prx_amplitude", _st, _vp, _i, _i, ctypes.c_uint64, _dp, _vp)
_sig("prx_norm2", _st, _vp, _i, _i, _dp, _vp, _sz, _vp)
_sig("prx_renormalize", _st, _vp, _i, _i, _vp, _sz, _vp)
_sig("prx_batch_create", _st, _sz, ctypes.POINTER(_i), ctypes.POINTER(_vp), _i, _u64p,
     ctypes.POINTER(_vp))
_sig("prx_batch_workspace_bytes", _sz, _vp)
_sig("prx_batch_get_info", _st, _vp, _vp)
_sig("prx_batch_upload", _st, _vp, ctypes.POINTER(_vp), _vp, _sz, _vp)
_sig("prx_batch_execute", _st, _vp, _vp, _sz, _vp, _vp)
_sig("prx_batch_check", _st, _vp, _vp, _vp)
_sig("prx_batch_destroy", None, _vp)
_sig("prx_batch_set_max_grid", _st, _vp, ctypes.c_uint)
_sig("prx_batch_run", _st, _sz, ctypes.POINTER(_vp), ctypes.POINTER(_i), ctypes.POINTER(_vp),
     _i, _u64p, _dp, _vp, _sz, _vp)
_sig("prx_batch_graph", _st, _vp, _vp, _sz, _vp, _vp, ctypes.POINTER(_vp))
_sig("prx_plan_graph", _st, _vp, _vp, _vp, _sz, _vp, ctypes.POINTER(_vp))
_sig("prx_graph_launch", _st, _vp, _vp)
_sig("prx_graph_destroy", None, _vp)
_sig("prx_autotune", _st, _vp, _i, _i, _vp, _vp, _sz, _vp, ctypes.POINTER(prx_plan_opts),
     ctypes.POINTER(_i))
_TUNE_PROGRESS = ctypes.CFUNCTYPE(None, ctypes.POINTER(prx_plan_opts), ctypes.c_float, _vp)
_sig("prx_autotune_progress", _st, _vp, _i, _i, _vp, _vp, _sz, _vp, ctypes.POINTER(prx_plan_opts),
     ctypes.POINTER(ctypes.c_int), _TUNE_PROGRESS, _vp)
_sig("prx_autotune_save", _st, ctypes.c_char_p)
_sig("prx_autotune_load", _st, ctypes.c_char_p)
_sig("prx_autotune_lookup", _st, _i, _i, ctypes.POINTER(prx_plan_opts))

EXPORTED = sorted(n for n in dir(_lib) if n.startswith("prx_"))


def _check(st: int):
    if st != PRX_OK:
        raise PrxError(st, _lib.prx_last_error().decode(errors="replace"))


def _ptr(buf) -> int | None:
    """Device or host address of a torch tensor / numpy array / int."""
    if buf is None:
        return None
    if isinstance(buf, int):
        return buf
    if hasattr(buf, "data_ptr"):
        return buf.data_ptr()
    if isinstance(buf, np.ndarray):
        return buf.ctypes.data
    raise TypeError(f"cannot take the address of {type(buf)!r}")


_TORCH_DTYPE_NAME = {PRX_C64: "complex64", PRX_C128: "complex128"}


def _is_tensor(buf) -> bool:
    return torch is not None and isinstance(buf, torch.Tensor)


def _state(buf, n: int, dtype: int, what: str = "state") -> int:
    """Address of a state buffer after checking a torch tensor against the
    C ABI's contract: a contiguous GPU tensor of 2^n elements whose dtype is
    the prx dtype's.  Integer addresses pass unchecked (the caller vouches
    for them)."""
    if _is_tensor(buf):
        want = _TORCH_DTYPE_NAME.get(int(dtype))
        if want is None:
            raise ValueError(f"{what}: unknown prx dtype {dtype!r}")
        if buf.dtype != getattr(torch, want):
            raise TypeError(f"{what}: tensor dtype {buf.dtype} does not match {want}")
        if not 0 <= int(n) < 64 or buf.numel() != (1 << int(n)):
            raise ValueError(f"{what}: {buf.numel()} elements, expected 2^{n}")
        if not buf.is_contiguous():
            raise ValueError(f"{what}: tensor is not contiguous")
        if not buf.is_cuda:
            raise ValueError(f"{what}: tensor is not on a GPU")
        return buf.data_ptr()
    if isinstance(buf, int):
        return buf
    raise TypeError(f"{what}: expected a torch tensor or a device address, got {type(buf)!r}")


def _device_buf(buf, what: str = "workspace") -> int:
    """Address of a device workspace: a contiguous GPU tensor or an int."""
    if _is_tensor(buf):
        if not buf.is_contiguous():
            raise ValueError(f"{what}: tensor is not contiguous")
        if not buf.is_cuda:
            raise ValueError(f"{what}: tensor is not on a GPU")
        return buf.data_ptr()
    if isinstance(buf, int):
        return buf
    raise TypeError(f"{what}: expected a torch tensor or a device address, got {type(buf)!r}")


def _nbytes(buf, given=None) -> int:
    if given is not None:
        return int(given)
    if hasattr(buf, "numel") and hasattr(buf, "element_size"):
        return buf.numel() * buf.element_size()
    if isinstance(buf, np.ndarray):
        return buf.nbytes
    raise TypeError("pass the buffer size explicitly")


def _stream(stream) -> int | None:
    if stream is None:
        return None
    if isinstance(stream, int):
        return stream
    return stream.cuda_stream  # torch.cuda.Stream


def _u64(a):
    a = np.ascontiguousarray(a, dtype=np.uint64)
    return a, a.ctypes.data_as(_u64p)


def _f64(a):
    a = np.ascontiguousarray(a, dtype=np.float64)
    return a, a.ctypes.data_as(_dp)


# ------------------------------------------------------------------ errors

def prx_last_error() -> str:
    return _lib.prx_last_error().decode(errors="replace")


def prx_version() -> str:
    return _lib.prx_version().decode()


# ------------------------------------------------------------- Hamiltonian

def prx_ham_create(n: int, x, z, h) -> int:
    xa, xp = _u64(x)
    za, zp = _u64(z)
    ha, hp = _f64(h)
    if not (len(xa) == len(za) == len(ha)):
        raise ValueError("x, z, h lengths differ")
    out = _vp()
    _check(_lib.prx_ham_create(int(n), len(xa), xp, zp, hp, ctypes.byref(out)))
    return out.value


def prx_ham_destroy(ham: int) -> None:
    _lib.prx_ham_destroy(ham)


def prx_ham_lambda(ham: int) -> float:
    v = ctypes.c_double()
    _check(_lib.prx_ham_lambda(ham, ctypes.byref(v)))
    return v.value


# --------------------------------------------------------------- schedules

def prx_sched_trotter(ham: int, order: int, t: float, steps: int,
                      reorder: int = PRX_REORDER_NONE) -> int:
    out = _vp()
    _check(_lib.prx_sched_trotter(ham, order, t, steps, reorder, ctypes.byref(out)))
    return out.value


def prx_sched_qdrift(ham: int, t: float, N: int, seed: int) -> int:
    out = _vp()
    _check(_lib.prx_sched_qdrift(ham, t, N, seed, ctypes.byref(out)))
    return out.value


def prx_sched_partial(ham: int, L_det: int, t: float, steps: int, r_per_step: int,
                      seed: int, reorder: int = PRX_REORDER_NONE) -> int:
    out = _vp()
    _check(_lib.prx_sched_partial(ham, L_det, t, steps, r_per_step, seed, reorder,
                                  ctypes.byref(out)))
    return out.value


def prx_sched_from_rotations(n: int, x, z, phi) -> int:
    xa, xp = _u64(x)
    za, zp = _u64(z)
    pa, pp = _f64(phi)
    out = _vp()
    _check(_lib.prx_sched_from_rotations(int(n), len(xa), xp, zp, pp, ctypes.byref(out)))
    return out.value


def prx_sched_view(sched: int):
    """(n, x, z, phi) copied into numpy arrays."""
    n = ctypes.c_int()
    M = ctypes.c_size_t()
    xp, zp, pp = _u64p(), _u64p(), _dp()
    _check(_lib.prx_sched_view(sched, ctypes.byref(n), ctypes.byref(M), ctypes.byref(xp),
                               ctypes.byref(zp), ctypes.byref(pp)))
    m = M.value
    if m == 0:
        return n.value, np.zeros(0, np.uint64), np.zeros(0, np.uint64), np.zeros(0)
    x = np.ctypeslib.as_array(xp, shape=(m,)).copy()
    z = np.ctypeslib.as_array(zp, shape=(m,)).copy()
    p = np.ctypeslib.as_array(pp, shape=(m,)).copy()
    return n.value, x, z, p


def prx_sched_destroy(sched: int) -> None:
    _lib.prx_sched_destroy(sched)


# -------------------------------------------------------------------- plans

def _opts(opts):
    if opts is None:
        return None
    if isinstance(opts, prx_plan_opts):
        return ctypes.byref(opts)
    o = prx_plan_opts()
    for k, v in dict(opts).items():
        setattr(o, k, int(v))
    return ctypes.byref(o)


def prx_plan_create(sched: int, n: int, dtype: int, begin: int, end: int, kernel: int,
                    opts=None) -> int:
    out = _vp()
    _check(_lib.prx_plan_create(sched, n, dtype, begin, end, kernel, _opts(opts),
                                ctypes.byref(out)))
    return out.value


def prx_plan_get_info(plan: int) -> dict:
    i = prx_plan_info()
    _check(_lib.prx_plan_get_info(plan, ctypes.byref(i)))
    return {f: getattr(i, f) for f, _ in prx_plan_info._fields_}


def prx_plan_destroy(plan: int) -> None:
    _lib.prx_plan_destroy(plan)


def prx_plan_upload(plan: int, ws, stream=None, ws_bytes=None) -> None:
    _check(_lib.prx_plan_upload(plan, _device_buf(ws), _nbytes(ws, ws_bytes), _stream(stream)))


def _plan_state(plan: int, psi) -> int:
    i = prx_plan_get_info(plan)
    return _state(psi, i["n"], i["dtype"])


def prx_plan_execute(plan: int, psi, ws, stream=None, ws_bytes=None) -> None:
    _check(_lib.prx_plan_execute(plan, _plan_state(plan, psi), _device_buf(ws),
                                 _nbytes(ws, ws_bytes), _stream(stream)))


def prx_plan_execute_timed(plan: int, psi, ws, stream=None, ws_bytes=None):
    """Executes and waits; returns (pass_ms, renorm_ms) numpy float32 arrays."""
    npass = prx_plan_get_info(plan)["passes"]
    pm = np.zeros(max(npass, 1), dtype=np.float32)
    rm = np.zeros(max(npass, 1), dtype=np.float32)
    fp = ctypes.POINTER(ctypes.c_float)
    _check(_lib.prx_plan_execute_timed(plan, _plan_state(plan, psi), _device_buf(ws),
                                       _nbytes(ws, ws_bytes),
                                       _stream(stream), pm.ctypes.data_as(fp),
                                       rm.ctypes.data_as(fp)))
    return pm[:npass], rm[:npass]


def prx_plan_pass(plan: int, i: int) -> dict:
    o = prx_pass_info()
    _check(_lib.prx_plan_pass(plan, i, ctypes.byref(o)))
    d = {f: getattr(o, f) for f, _ in prx_pass_info._fields_}
    for k in ("basis", "pivot", "vmask", "tpivot", "fscale", "perm_pos", "perm_dst"):
        d[k] = list(d[k])
    return d


def prx_plan_chunk(plan: int, i: int) -> dict:
    o = prx_chunk_info()
    _check(_lib.prx_plan_chunk(plan, i, ctypes.byref(o)))
    d = {f: getattr(o, f) for f, _ in prx_chunk_info._fields_}
    d["basis"] = list(d["basis"])
    d["cvec"] = list(d["cvec"])
    d["fscale"] = list(d["fscale"])
    return d


def prx_plan_rotation(plan: int, i: int) -> dict:
    o = prx_rot_info()
    _check(_lib.prx_plan_rotation(plan, i, ctypes.byref(o)))
    return {f: getattr(o, f) for f, _ in prx_rot_info._fields_}


# ------------------------------------------------------------ apply/reduce

def prx_workspace_bytes(n: int, dtype: int, sched: int, kernel: int) -> int:
    return int(_lib.prx_workspace_bytes(n, dtype, sched, kernel))


def prx_apply_range(psi, n: int, dtype: int, sched: int, begin: int, end: int, kernel: int,
                    ws, stream=None, ws_bytes=None) -> None:
    _check(_lib.prx_apply_range(_state(psi, n, dtype), n, dtype, sched, begin, end, kernel,
                                _device_buf(ws), _nbytes(ws, ws_bytes), _stream(stream)))


PRX_STATIC_WS_BYTES = 64 << 20


def prx_apply_range_static(psi, n: int, dtype: int, sched: int, begin: int, end: int,
                           kernel: int, stream=None) -> None:
    _check(_lib.prx_apply_range_static(_state(psi, n, dtype), n, dtype, sched, begin, end,
                                       kernel, _stream(stream)))


def prx_reduce_workspace_bytes(n: int) -> int:
    return int(_lib.prx_reduce_workspace_bytes(n))


def prx_overlap(psi0, psi, n: int, dtype: int, ws, stream=None, ws_bytes=None) -> complex:
    out = (ctypes.c_double * 2)()
    _check(_lib.prx_overlap(_state(psi0, n, dtype, "psi0"), _state(psi, n, dtype), n, dtype,
                            out, _device_buf(ws), _nbytes(ws, ws_bytes), _stream(stream)))
    return complex(out[0], out[1])


def prx_amplitude(psi, n: int, dtype: int, k: int, stream=None) -> complex:
    out = (ctypes.c_double * 2)()
    _check(_lib.prx_amplitude(_state(psi, n, dtype), n, dtype, k, out, _stream(stream)))
    return complex(out[0], out[1])


def prx_norm2(psi, n: int, dtype: int, ws, stream=None, ws_bytes=None) -> float:
    v = ctypes.c_double()
    _check(_lib.prx_norm2(_state(psi, n, dtype), n, dtype, ctypes.byref(v), _device_buf(ws),
                          _nbytes(ws, ws_bytes), _stream(stream)))
    return v.value


def prx_renormalize(psi, n: int, dtype: int, ws, stream=None, ws_bytes=None) -> None:
    _check(_lib.prx_renormalize(_state(psi, n, dtype), n, dtype, _device_buf(ws),
                                _nbytes(ws, ws_bytes), _stream(stream)))


# ------------------------------------------------------------------ batches

def prx_batch_create(n_list, scheds, dtype: int, basis_idx) -> int:
    S = len(n_list)
    na = (ctypes.c_int * S)(*[int(v) for v in n_list])
    sa = (_vp * S)(*scheds)
    ba, bp = _u64(basis_idx)
    out = _vp()
    _check(_lib.prx_batch_create(S, na, sa, dtype, bp, ctypes.byref(out)))
    _BATCH_SHAPES[out.value] = ([int(v) for v in n_list], int(dtype))
    return out.value


# (qubit counts, dtype) of the live batch handles, for checking the states
# handed to prx_batch_upload
_BATCH_SHAPES: dict = {}


def _batch_states(psis, n_list, dtype) -> list:
    if len(psis) != len(n_list):
        raise ValueError(f"{len(psis)} states for {len(n_list)} samples")
    return [_state(p, n, dtype, f"state of sample {i}")
            for i, (p, n) in enumerate(zip(psis, n_list))]


def prx_batch_workspace_bytes(batch: int) -> int:
    return int(_lib.prx_batch_workspace_bytes(batch))


class prx_batch_info(ctypes.Structure):
    _fields_ = [("samples", _sz), ("tile_samples", _sz), ("rounds", _sz), ("passes", _sz),
                ("amp_sweeps", ctypes.c_double)]


def prx_batch_get_info(batch: int) -> dict:
    o = prx_batch_info()
    _check(_lib.prx_batch_get_info(batch, ctypes.byref(o)))
    return {f: getattr(o, f) for f, _ in prx_batch_info._fields_}


def prx_batch_upload(batch: int, psis, ws, stream=None, ws_bytes=None) -> None:
    shape = _BATCH_SHAPES.get(batch)
    addrs = _batch_states(psis, *shape) if shape else [_device_buf(p, "state") for p in psis]
    pa = (_vp * len(addrs))(*addrs)
    _check(_lib.prx_batch_upload(batch, pa, _device_buf(ws), _nbytes(ws, ws_bytes),
                                 _stream(stream)))


def prx_batch_execute(batch: int, ws, overlaps_dev, stream=None, ws_bytes=None) -> None:
    _check(_lib.prx_batch_execute(batch, _device_buf(ws), _nbytes(ws, ws_bytes),
                                  _device_buf(overlaps_dev, "overlaps"),
                                  _stream(stream)))


def prx_batch_set_max_grid(batch: int, max_grid: int) -> None:
    _check(_lib.prx_batch_set_max_grid(batch, int(max_grid)))


def prx_batch_check(batch: int, ws, stream=None) -> None:
    _check(_lib.prx_batch_check(batch, _device_buf(ws), _stream(stream)))


def prx_batch_destroy(batch: int) -> None:
    _BATCH_SHAPES.pop(batch, None)
    _lib.prx_batch_destroy(batch)


def prx_batch_run(psis, n_list, scheds, dtype: int, basis_idx, ws, stream=None,
                  ws_bytes=None) -> np.ndarray:
    S = len(psis)
    pa = (_vp * S)(*_batch_states(psis, n_list, dtype))
    na = (ctypes.c_int * S)(*[int(v) for v in n_list])
    sa = (_vp * S)(*scheds)
    ba, bp = _u64(basis_idx)
    out = np.zeros(2 * S, dtype=np.float64)
    _check(_lib.prx_batch_run(S, pa, na, sa, dtype, bp, out.ctypes.data_as(_dp),
                              _device_buf(ws), _nbytes(ws, ws_bytes), _stream(stream)))
    return out[0::2] + 1j * out[1::2]


def prx_batch_graph(batch: int, ws, overlaps_dev, stream, ws_bytes=None) -> int:
    out = _vp()
    _check(_lib.prx_batch_graph(batch, _device_buf(ws), _nbytes(ws, ws_bytes),
                                _device_buf(overlaps_dev, "overlaps"),
                                _stream(stream), ctypes.byref(out)))
    return out.value


def prx_plan_graph(plan: int, psi, ws, stream, ws_bytes=None) -> int:
    out = _vp()
    _check(_lib.prx_plan_graph(plan, _plan_state(plan, psi), _device_buf(ws),
                               _nbytes(ws, ws_bytes), _stream(stream), ctypes.byref(out)))
    return out.value


def prx_graph_launch(graph: int, stream=None) -> None:
    _check(_lib.prx_graph_launch(graph, _stream(stream)))


def prx_graph_destroy(graph: int) -> None:
    _lib.prx_graph_destroy(graph)


# ---------------------------------------------------------------- autotune

def prx_autotune(psi, n: int, dtype: int, sched: int, ws, stream=None, ws_bytes=None,
                 progress=None):
    """progress(opts: dict, ms: float) is called after each timed setting."""
    best = prx_plan_opts()
    trials = ctypes.c_int()
    if progress is None:
        _check(_lib.prx_autotune(_state(psi, n, dtype), n, dtype, sched, _device_buf(ws),
                                 _nbytes(ws, ws_bytes), _stream(stream), ctypes.byref(best),
                                 ctypes.byref(trials)))
    else:
        def _cb(o, ms, _user):
            progress({f: getattr(o.contents, f) for f, _ in prx_plan_opts._fields_}, float(ms))
        cb = _TUNE_PROGRESS(_cb)
        _check(_lib.prx_autotune_progress(_state(psi, n, dtype), n, dtype, sched,
                                          _device_buf(ws),
                                          _nbytes(ws, ws_bytes), _stream(stream),
                                          ctypes.byref(best), ctypes.byref(trials), cb, None))
    return {f: getattr(best, f) for f, _ in prx_plan_opts._fields_}, trials.value


def prx_autotune_progress(psi, n: int, dtype: int, sched: int, ws, progress, stream=None,
                          ws_bytes=None):
    return prx_autotune(psi, n, dtype, sched, ws, stream, ws_bytes, progress=progress)


def prx_autotune_save(path: str) -> None:
    _check(_lib.prx_autotune_save(path.encode()))


def prx_autotune_load(path: str) -> None:
    _check(_lib.prx_autotune_load(path.encode()))


def prx_autotune_lookup(n: int, dtype: int):
    o = prx_plan_opts()
    st = _lib.prx_autotune_lookup(n, dtype, ctypes.byref(o))
    if st == PRX_ERR_UNSUPPORTED:
        return None
    _check(st)
    return {f: getattr(o, f) for f, _ in prx_plan_opts._fields_}
