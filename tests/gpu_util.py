"""Helpers shared by the GPU tests: column-major device copies."""
import numpy as np
import torch


def dev(A: np.ndarray, ld: int | None = None) -> torch.Tensor:
    """Column-major FP64 device copy of A with leading dimension ld."""
    m, n = A.shape
    ld = m if ld is None else ld
    t = torch.empty((n, ld), dtype=torch.float64, device="cuda").t()[:m]
    t.copy_(torch.from_numpy(np.ascontiguousarray(A)))
    return t


def host(t: torch.Tensor) -> np.ndarray:
    return t.detach().cpu().numpy().copy()
