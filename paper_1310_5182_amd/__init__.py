"""Local approximate GP regression with greedy ALC designs on MI355X (gfx950).

Thin torch binding of the C ABI in include/lagp_alc.h: tensors supply device
memory, torch's current HIP stream carries the work, and every step of the
path runs in the library's HIP kernels.
"""
from __future__ import annotations

import torch

from . import _lib
from ._lib import LAGP_FP64, LAGP_MIXED, LagpError  # noqa: F401

__all__ = ["nn_pool", "alc_from_pool", "alc_predict", "PRECISIONS", "version"]

PRECISIONS = {"fp64": LAGP_FP64, "mixed": LAGP_MIXED}


def _f64(t: torch.Tensor, name: str) -> torch.Tensor:
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise ValueError(f"{name} must be a CUDA/HIP tensor")
    if t.dtype != torch.float64 or not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous float64")
    return t


def _stream(device: torch.device) -> int:
    return torch.cuda.current_stream(device).cuda_stream


def _prec(precision) -> int:
    if isinstance(precision, str):
        if precision not in PRECISIONS:
            raise ValueError(f"precision must be one of {sorted(PRECISIONS)}")
        return PRECISIONS[precision]
    return int(precision)


def version() -> str:
    return _lib.load().lagp_version().decode()


def nn_pool(X: torch.Tensor, XX: torch.Tensor, Np: int, out: torch.Tensor | None = None) -> torch.Tensor:
    """M x Np int32 pools: the Np nearest design rows of each location, sorted by (distance, index)."""
    L = _lib.load()
    X, XX = _f64(X, "X"), _f64(XX, "XX")
    M, p = XX.shape
    if X.dim() != 2 or X.shape[1] != p:
        raise ValueError("X must be N x p with the p of XX")
    if out is None:
        out = torch.empty((M, Np), dtype=torch.int32, device=X.device)
    _lib.check(L.lagp_nn_pool(X.data_ptr(), X.shape[0], p, XX.data_ptr(), M, Np, out.data_ptr(),
                              _stream(X.device)))
    return out


def _outputs(M: int, n: int, device) -> dict:
    return dict(
        mean=torch.empty(M, dtype=torch.float64, device=device),
        s2=torch.empty(M, dtype=torch.float64, device=device),
        var=torch.empty(M, dtype=torch.float64, device=device),
        sel=torch.empty((M, n), dtype=torch.int32, device=device),
        alc=torch.empty((M, n), dtype=torch.float64, device=device),
        status=torch.empty(M, dtype=torch.int32, device=device),
        guard=torch.empty(M, dtype=torch.int32, device=device),
    )


def alc_from_pool(X, Y, XX, pool, n0: int, n: int, d: float, g: float, precision="fp64",
                  out: dict | None = None) -> dict:
    """Greedy ALC local designs and predictions from given pools (M x Np int32)."""
    L = _lib.load()
    X, Y, XX = _f64(X, "X"), _f64(Y, "Y"), _f64(XX, "XX")
    if pool.dtype != torch.int32 or not pool.is_contiguous() or not pool.is_cuda:
        raise ValueError("pool must be a contiguous int32 device tensor")
    M, p = XX.shape
    Np = pool.shape[1]
    o = out if out is not None else _outputs(M, n, X.device)
    _lib.check(L.lagp_alc_from_pool(
        X.data_ptr(), Y.data_ptr(), X.shape[0], p, XX.data_ptr(), M, pool.data_ptr(), Np, n0, n,
        float(d), float(g), _prec(precision), o["mean"].data_ptr(), o["s2"].data_ptr(),
        o["var"].data_ptr(), o["sel"].data_ptr(), o["alc"].data_ptr(), o["status"].data_ptr(),
        o["guard"].data_ptr(), _stream(X.device)))
    return o


def alc_predict(X, Y, XX, n0: int, n: int, Np: int, d: float, g: float, precision="fp64",
                out: dict | None = None) -> dict:
    """The whole path: NN pools, greedy ALC designs, local predictions."""
    L = _lib.load()
    X, Y, XX = _f64(X, "X"), _f64(Y, "Y"), _f64(XX, "XX")
    M, p = XX.shape
    o = out if out is not None else _outputs(M, n, X.device)
    if "pool" not in o:
        o["pool"] = torch.empty((M, Np), dtype=torch.int32, device=X.device)
    _lib.check(L.lagp_alc_predict(
        X.data_ptr(), Y.data_ptr(), X.shape[0], p, XX.data_ptr(), M, n0, n, Np, float(d), float(g),
        _prec(precision), o["pool"].data_ptr(), o["mean"].data_ptr(), o["s2"].data_ptr(),
        o["var"].data_ptr(), o["sel"].data_ptr(), o["alc"].data_ptr(), o["status"].data_ptr(),
        o["guard"].data_ptr(), _stream(X.device)))
    return o
