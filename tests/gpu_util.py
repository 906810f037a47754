"""Helpers shared by the GPU tests: device transfers and inputs computed on
both sides (the GPU library and the oracle each build their own face
coefficients and right-hand side from the same raw workload)."""
import numpy as np
import torch

import oracle
from paper_2605_30082_amd import solver as S


def dev():
    if not torch.cuda.is_available():
        raise RuntimeError("GPU tests need a HIP device")
    return torch.device("cuda", 0)


def T(a: np.ndarray) -> torch.Tensor:
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).to(dev())


def N(t: torch.Tensor) -> np.ndarray:
    torch.cuda.synchronize()
    return t.detach().cpu().numpy()


def gpu_inputs(wl):
    """Face coefficients and rhs computed by the GPU library from the raw workload."""
    beta = S.faces_from_vof(T(wl.f_drop), T(wl.f_film), wl.rho_drop, wl.rho_film, wl.rho_gas)
    b = S.divergence(T(wl.u), T(wl.v), T(wl.w), wl.h, wl.dt)
    return beta, b


def oracle_inputs(wl):
    beta = oracle.faces_from_vof(wl.f_drop, wl.f_film, wl.rho_drop, wl.rho_film, wl.rho_gas)
    b = oracle.divergence(wl.u, wl.v, wl.w, wl.h, wl.dt)
    return beta, b


def rel_l2(a, b) -> float:
    a = np.asarray(a).ravel()
    b = np.asarray(b).ravel()
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def max_rel(a, b) -> float:
    return float(np.max(np.abs(np.asarray(a) - np.asarray(b))) / np.max(np.abs(b)))


def note(msg: str) -> None:
    print(msg, flush=True)
