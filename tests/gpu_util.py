"""Device helpers for the GPU tests: torch supplies memory and streams only."""
from __future__ import annotations

import numpy as np
import torch

from paper_2504_17881_amd import prx as P


def dev():
    if not torch.cuda.is_available():
        raise RuntimeError("GPU test run without a visible GPU")
    return torch.device("cuda:0")


def tdtype(dtype):
    return torch.complex64 if dtype == P.PRX_C64 else torch.complex128


def to_dev(psi: np.ndarray, dtype) -> torch.Tensor:
    return torch.from_numpy(np.ascontiguousarray(psi)).to(dev(), dtype=tdtype(dtype))


def to_host(t: torch.Tensor) -> np.ndarray:
    torch.cuda.synchronize()
    return t.detach().to("cpu").numpy().astype(np.complex128)


def workspace(nbytes: int) -> torch.Tensor:
    return torch.empty(max(int(nbytes), 256), dtype=torch.uint8, device=dev())


def basis_state(n: int, k: int, dtype) -> torch.Tensor:
    t = torch.zeros(1 << n, dtype=tdtype(dtype), device=dev())
    t[k] = 1.0
    return t


def apply(psi: torch.Tensor, n: int, dtype, sched: int, kernel, begin=0, end=None, opts=None):
    """Plan, upload and execute [begin, end) on psi; returns the plan info."""
    if end is None:
        end = P.prx_sched_view(sched)[1].shape[0]
    pl = P.prx_plan_create(sched, n, dtype, begin, end, kernel, opts)
    info = P.prx_plan_get_info(pl)
    ws = workspace(info["workspace_bytes"])
    P.prx_plan_upload(pl, ws)
    P.prx_plan_execute(pl, psi, ws)
    torch.cuda.synchronize()
    P.prx_plan_destroy(pl)
    return info


def rel_err(a: np.ndarray, b: np.ndarray) -> float:
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def overlap(psi0: torch.Tensor, psi: torch.Tensor, n: int, dtype) -> complex:
    ws = workspace(P.prx_reduce_workspace_bytes(n))
    return P.prx_overlap(psi0, psi, n, dtype, ws)
