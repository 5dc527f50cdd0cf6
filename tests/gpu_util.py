"""Helpers for the GPU tests: numpy (Fortran) <-> column-major device tensors."""
import numpy as np
import torch

DEV = "cuda:0"


def to_dev(A: np.ndarray, ld: int | None = None, dtype=torch.float64):
    """Column-major device copy of a 2-D numpy array, leading dimension ld
    (>= rows; the padding rows hold NaN so that a read of them shows)."""
    r, c = A.shape
    ld = max(r, 1) if ld is None else ld
    base = torch.full((max(c, 1) * ld,), float("nan"), dtype=dtype, device=DEV)
    view = base.as_strided((r, c), (1, ld))
    if r and c:
        view.copy_(torch.from_numpy(np.asarray(A, dtype=np.float64)).to(dtype))
    return view


def to_host(T) -> np.ndarray:
    torch.cuda.synchronize()
    return np.asfortranarray(T.detach().to("cpu", torch.float64).numpy())


def zeros_info(k: int = 1):
    return torch.zeros(k, dtype=torch.int32, device=DEV)
