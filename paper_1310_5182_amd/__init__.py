"""Local approximate GP regression with greedy ALC designs on MI355X (gfx950).

Thin torch binding of the C ABI in include/lagp_alc.h: tensors supply device
memory, torch's current HIP stream carries the work, and every step of the
path runs in the library's HIP kernels.
"""
from __future__ import annotations

import ctypes

import torch

from . import _lib
from ._lib import LAGP_FP64, LAGP_FP64_REFORM, LAGP_MIXED, LagpError  # noqa: F401

__all__ = ["nn_pool", "alc_scores", "alc_multistage", "alc_from_pool", "alc_predict", "alc_uneven_from_pool", "alc_uneven_predict", "Plan",
           "local_nll", "LocalNLL", "local_mle_d", "local_predict", "PRECISIONS", "version"]

PRECISIONS = {"fp64": LAGP_FP64, "mixed": LAGP_MIXED, "fp64_reform": LAGP_FP64_REFORM}


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


def nn_pool(X: torch.Tensor, XX: torch.Tensor, Np: int, out: torch.Tensor | None = None,
            grid: bool = False, workspace: torch.Tensor | None = None) -> torch.Tensor:
    """M x Np int32 pools: the Np nearest design rows of each location, sorted by (distance, index).

    grid: bucket the design into grid cells and stream, nearest cell first, only
    the cells that can hold a pool member (lagp_nn_pool_ws; the same pools),
    with the cells kept in `workspace` (a uint8 device tensor, allocated here if
    None or too small)."""
    L = _lib.load()
    X, XX = _f64(X, "X"), _f64(XX, "XX")
    M, p = XX.shape
    if X.dim() != 2 or X.shape[1] != p:
        raise ValueError("X must be N x p with the p of XX")
    if out is None:
        out = torch.empty((M, Np), dtype=torch.int32, device=X.device)
    if not grid:
        _lib.check(L.lagp_nn_pool(X.data_ptr(), X.shape[0], p, XX.data_ptr(), M, Np, out.data_ptr(),
                                  _stream(X.device)))
        return out
    nbytes = ctypes.c_size_t(0)
    _lib.check(L.lagp_nn_pool_workspace(X.shape[0], p, M, ctypes.byref(nbytes)))
    if workspace is None or workspace.numel() < nbytes.value:
        workspace = torch.empty(nbytes.value, dtype=torch.uint8, device=X.device)
    _lib.check(L.lagp_nn_pool_ws(X.data_ptr(), X.shape[0], p, XX.data_ptr(), M, Np, out.data_ptr(),
                                 workspace.data_ptr(), workspace.numel(), _stream(X.device)))
    return out


def alc_scores(Xj, Kinv, Xc, x, h, d: float, g: float, precision="fp64",
               out: torch.Tensor | None = None) -> torch.Tensor:
    """Scores v_j(x) - v_{j+1}(x) (eq. dxy) of every candidate row of Xc against
    the design Xj (j x p) at x, given K_j^{-1} (j x j) and h = K(X_j, x) (j):
    the paper's per-step kernel over all candidates in one launch."""
    L = _lib.load()
    Xj, Kinv, Xc, x, h = (_f64(t, nme) for t, nme in ((Xj, "Xj"), (Kinv, "Kinv"), (Xc, "Xc"), (x, "x"), (h, "h")))
    j, p = Xj.shape
    if Kinv.shape != (j, j) or Xc.dim() != 2 or Xc.shape[1] != p or x.numel() != p or h.numel() != j:
        raise ValueError("need Xj j x p, Kinv j x j, Xc Nc x p, x of p and h of j entries")
    if precision not in ("fp64", "mixed"):
        raise ValueError("precision must be 'fp64' or 'mixed'")
    if out is None:
        out = torch.empty(Xc.shape[0], dtype=torch.float64, device=Xc.device)
    _lib.check(L.lagp_alc_scores(Xj.data_ptr(), j, p, Kinv.data_ptr(), Xc.data_ptr(), Xc.shape[0], x.data_ptr(),
                                 h.data_ptr(), float(d), float(g), _prec(precision), out.data_ptr(),
                                 _stream(Xc.device)))
    return out


def _outputs(M: int, n: int, device, out: dict | None = None) -> dict:
    """The output tensors of an ALC call; entries missing from `out` are added to it."""
    o = out if out is not None else {}
    f64, i32 = torch.float64, torch.int32
    for k, shape, dt in (("mean", (M,), f64), ("s2", (M,), f64), ("var", (M,), f64), ("sel", (M, n), i32),
                         ("alc", (M, n), f64), ("alc32", (M, n), f64), ("status", (M,), i32),
                         ("guard", (M,), i32)):
        if k not in o:
            o[k] = torch.empty(shape, dtype=dt, device=device)
    return o


def alc_from_pool(X, Y, XX, pool, n0: int, n: int, d: float, g: float, precision="fp64",
                  out: dict | None = None) -> dict:
    """Greedy ALC local designs and predictions from given pools (M x Np int32)."""
    L = _lib.load()
    X, Y, XX = _f64(X, "X"), _f64(Y, "Y"), _f64(XX, "XX")
    if pool.dtype != torch.int32 or not pool.is_contiguous() or not pool.is_cuda:
        raise ValueError("pool must be a contiguous int32 device tensor")
    M, p = XX.shape
    Np = pool.shape[1]
    o = _outputs(M, n, X.device, out)
    _lib.check(L.lagp_alc_from_pool(
        X.data_ptr(), Y.data_ptr(), X.shape[0], p, XX.data_ptr(), M, pool.data_ptr(), Np, n0, n,
        float(d), float(g), _prec(precision), o["mean"].data_ptr(), o["s2"].data_ptr(),
        o["var"].data_ptr(), o["sel"].data_ptr(), o["alc"].data_ptr(), o["alc32"].data_ptr(),
        o["status"].data_ptr(), o["guard"].data_ptr(), _stream(X.device)))
    return o


def alc_predict(X, Y, XX, n0: int, n: int, Np: int, d: float, g: float, precision="fp64",
                out: dict | None = None) -> dict:
    """The whole path: NN pools, greedy ALC designs, local predictions."""
    L = _lib.load()
    X, Y, XX = _f64(X, "X"), _f64(Y, "Y"), _f64(XX, "XX")
    M, p = XX.shape
    o = _outputs(M, n, X.device, out)
    if "pool" not in o:
        o["pool"] = torch.empty((M, Np), dtype=torch.int32, device=X.device)
    _lib.check(L.lagp_alc_predict(
        X.data_ptr(), Y.data_ptr(), X.shape[0], p, XX.data_ptr(), M, n0, n, Np, float(d), float(g),
        _prec(precision), o["pool"].data_ptr(), o["mean"].data_ptr(), o["s2"].data_ptr(),
        o["var"].data_ptr(), o["sel"].data_ptr(), o["alc"].data_ptr(), o["alc32"].data_ptr(),
        o["status"].data_ptr(), o["guard"].data_ptr(), _stream(X.device)))
    return o


def _i32(t, name: str, M: int) -> int:
    if t is None:
        return 0
    if t.dtype != torch.int32 or not t.is_contiguous() or not t.is_cuda or t.numel() != M:
        raise ValueError(f"{name} must be a contiguous int32 device tensor of length M")
    return t.data_ptr()


def _d_per(t, M: int) -> int:
    if t is None:
        return 0
    if t.dtype != torch.float64 or not t.is_contiguous() or not t.is_cuda or t.numel() != M:
        raise ValueError("d_per must be a contiguous float64 device tensor of length M")
    return t.data_ptr()


def alc_uneven_from_pool(X, Y, XX, pool, n0: int, n_max: int, d: float, g: float, n_per=None,
                         Np_per=None, sel_off=None, precision="fp64", out: dict | None = None,
                         d_per=None) -> dict:
    """Greedy ALC designs with a design size n_per[m] and a pool size Np_per[m]
    of each location's own (int32 device tensors, None = n_max / the pool
    width) and optionally a lengthscale d_per[m] of its own (float64, None = d).  pool: M x Np_max from nn_pool(X, XX, Np_max).  Without sel_off,
    sel and alc are M x n_max with entries past n_per[m] set to -1 / NaN;
    with sel_off (int64, M + 1 offsets) they are flat rows, and `out` must
    supply sel and alc of length sel_off[M]."""
    L = _lib.load()
    X, Y, XX = _f64(X, "X"), _f64(Y, "Y"), _f64(XX, "XX")
    if pool.dtype != torch.int32 or not pool.is_contiguous() or not pool.is_cuda:
        raise ValueError("pool must be a contiguous int32 device tensor")
    M, p = XX.shape
    Np_max = pool.shape[1]
    dev = X.device
    if sel_off is not None:
        if sel_off.dtype != torch.int64 or not sel_off.is_contiguous() or sel_off.numel() != M + 1:
            raise ValueError("sel_off must be a contiguous int64 device tensor of length M + 1")
        if out is None or "sel" not in out or "alc" not in out:
            raise ValueError("with sel_off, out must supply flat sel (int32) and alc (float64)")
    o = _outputs(M, n_max, dev, out)
    nbytes = ctypes.c_size_t(0)
    _lib.check(L.lagp_alc_uneven_workspace(p, M, Np_max, n_max, ctypes.byref(nbytes)))
    ws = o.get("workspace")
    if ws is None or ws.numel() < nbytes.value:
        ws = o["workspace"] = torch.empty(max(nbytes.value, 1), dtype=torch.uint8, device=dev)
    _lib.check(L.lagp_alc_uneven_from_pool(
        X.data_ptr(), Y.data_ptr(), X.shape[0], p, XX.data_ptr(), M, pool.data_ptr(), Np_max, n0, n_max,
        _i32(n_per, "n_per", M), _i32(Np_per, "Np_per", M),
        sel_off.data_ptr() if sel_off is not None else 0, _d_per(d_per, M), float(d), float(g), _prec(precision),
        o["mean"].data_ptr(), o["s2"].data_ptr(), o["var"].data_ptr(), o["sel"].data_ptr(),
        o["alc"].data_ptr(), o["status"].data_ptr(), o["guard"].data_ptr(), ws.data_ptr(), ws.numel(),
        _stream(dev)))
    return o


def alc_uneven_predict(X, Y, XX, n0: int, n_max: int, Np_max: int, d: float, g: float, n_per=None,
                       Np_per=None, precision="fp64", out: dict | None = None, d_per=None) -> dict:
    """The whole path with per-location n and N': one pool of the Np_max nearest
    neighbours per location (each location uses its own prefix), then
    alc_uneven_from_pool."""
    X, XX = _f64(X, "X"), _f64(XX, "XX")
    o = out if out is not None else {}
    o["pool"] = nn_pool(X, XX, Np_max, out=o.get("pool"))
    return alc_uneven_from_pool(X, Y, XX, o["pool"], n0, n_max, d, g, n_per=n_per, Np_per=Np_per,
                                precision=precision, out=o, d_per=d_per)


class Plan:
    """The whole float64 path (NN pools of Np_max, then per-location greedy ALC
    designs and predictions) bound to fixed buffers, autotuned on these inputs
    and captured into one HIP graph.  `out` holds the pool and the outputs
    (sel and alc padded to M x n_max); `launch()` enqueues one run on torch's
    current stream.  The input tensors must stay alive as long as the plan."""

    def __init__(self, X, Y, XX, n0: int, n_max: int, Np_max: int, d: float, g: float, n_per=None,
                 Np_per=None, tune: bool = True, d_per=None):
        L = _lib.load()
        X, Y, XX = _f64(X, "X"), _f64(Y, "Y"), _f64(XX, "XX")
        M, p = XX.shape
        dev = X.device
        o = _outputs(M, n_max, dev)
        o["pool"] = torch.empty((M, Np_max), dtype=torch.int32, device=dev)
        nbytes = ctypes.c_size_t(0)
        _lib.check(L.lagp_plan_workspace(X.shape[0], p, M, Np_max, n_max, ctypes.byref(nbytes)))
        o["workspace"] = torch.empty(max(nbytes.value, 1), dtype=torch.uint8, device=dev)
        self._keep = (X, Y, XX, n_per, Np_per, d_per)
        self.out, self._dev, self._h = o, dev, ctypes.c_void_p()
        _lib.check(L.lagp_plan_create(
            X.data_ptr(), Y.data_ptr(), X.shape[0], p, XX.data_ptr(), M, n0, n_max, Np_max,
            _i32(n_per, "n_per", M), _i32(Np_per, "Np_per", M), 0, _d_per(d_per, M), float(d), float(g),
            o["pool"].data_ptr(),
            o["mean"].data_ptr(), o["s2"].data_ptr(), o["var"].data_ptr(), o["sel"].data_ptr(),
            o["alc"].data_ptr(), o["status"].data_ptr(), o["guard"].data_ptr(), o["workspace"].data_ptr(),
            o["workspace"].numel(), 0 if tune else 1, _stream(dev), ctypes.byref(self._h)))

    def launch(self) -> dict:
        _lib.check(_lib.load().lagp_plan_launch(self._h, _stream(self._dev)))
        return self.out

    def describe(self) -> str:
        buf = ctypes.create_string_buffer(2048)
        _lib.check(_lib.load().lagp_plan_describe(self._h, buf, len(buf)))
        return buf.value.decode()

    def close(self) -> None:
        if self._h:
            _lib.check(_lib.load().lagp_plan_destroy(self._h))
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:  # noqa: BLE001 - interpreter shutdown
            pass


def _sel(sel: torch.Tensor) -> torch.Tensor:
    if sel.dtype != torch.int32 or not sel.is_contiguous() or not sel.is_cuda or sel.dim() != 2:
        raise ValueError("sel must be a contiguous M x n int32 device tensor")
    return sel


def _per_loc(v, M: int, device, name: str) -> torch.Tensor:
    if isinstance(v, torch.Tensor):
        return _f64(v.reshape(M) if v.numel() == M else v, name)
    return torch.full((M,), float(v), dtype=torch.float64, device=device)


def local_nll(X, Y, sel, d, g, order: int = 0) -> dict:
    """Negative log of eq. gpk on each location's fixed design (float64).

    order 0: nll; 1: + dnll/dd, dnll/dg; 2: + d2nll/dd2.  d, g: scalars or M-vectors.
    """
    L = _lib.load()
    X, Y, sel = _f64(X, "X"), _f64(Y, "Y"), _sel(sel)
    M, n = sel.shape
    dev = X.device
    d, g = _per_loc(d, M, dev, "d"), _per_loc(g, M, dev, "g")
    out = {"nll": torch.empty(M, dtype=torch.float64, device=dev),
           "status": torch.empty(M, dtype=torch.int32, device=dev)}
    if order >= 1:
        out["dd"] = torch.empty(M, dtype=torch.float64, device=dev)
        out["dg"] = torch.empty(M, dtype=torch.float64, device=dev)
    if order >= 2:
        out["d2"] = torch.empty(M, dtype=torch.float64, device=dev)
    ptr = lambda k: out[k].data_ptr() if k in out else None  # noqa: E731
    _lib.check(L.lagp_local_nll(X.data_ptr(), Y.data_ptr(), X.shape[0], X.shape[1], sel.data_ptr(), M, n,
                                d.data_ptr(), g.data_ptr(), ptr("nll"), ptr("dd"), ptr("dg"), ptr("d2"),
                                ptr("status"), _stream(dev)))
    return out


class LocalNLL(torch.autograd.Function):
    """nll[m](d[m], g[m]) on fixed local designs; the backward is the library's
    hand-written reverse kernel (lagp_local_nll_backward)."""

    @staticmethod
    def forward(ctx, d, g, X, Y, sel):
        out = local_nll(X, Y, sel, d.detach().contiguous(), g.detach().contiguous(), order=0)
        ctx.save_for_backward(d.detach().contiguous(), g.detach().contiguous())
        ctx.data = (X, Y, sel)
        return out["nll"]

    @staticmethod
    def backward(ctx, grad_out):
        L = _lib.load()
        d, g = ctx.saved_tensors
        X, Y, sel = ctx.data
        M, n = sel.shape
        go = grad_out.contiguous().to(torch.float64)
        gd = torch.empty_like(d) if ctx.needs_input_grad[0] else None
        gg = torch.empty_like(g) if ctx.needs_input_grad[1] else None
        _lib.check(L.lagp_local_nll_backward(
            X.data_ptr(), Y.data_ptr(), X.shape[0], X.shape[1], sel.data_ptr(), M, n, d.data_ptr(),
            g.data_ptr(), go.data_ptr(), None if gd is None else gd.data_ptr(),
            None if gg is None else gg.data_ptr(), _stream(X.device)))
        return gd, gg, None, None, None


def local_mle_d(X, Y, sel, d0, g: float, dmin: float = 1e-3, dmax: float = 5.0, maxit: int = 100) -> dict:
    """Maximum-likelihood lengthscale per location (projected Newton, g fixed)."""
    L = _lib.load()
    X, Y, sel = _f64(X, "X"), _f64(Y, "Y"), _sel(sel)
    M, n = sel.shape
    dev = X.device
    d0 = _per_loc(d0, M, dev, "d0")
    out = {"d": torch.empty(M, dtype=torch.float64, device=dev),
           "nll": torch.empty(M, dtype=torch.float64, device=dev),
           "iters": torch.empty(M, dtype=torch.int32, device=dev),
           "status": torch.empty(M, dtype=torch.int32, device=dev)}
    _lib.check(L.lagp_local_mle_d(X.data_ptr(), Y.data_ptr(), X.shape[0], X.shape[1], sel.data_ptr(), M, n,
                                  d0.data_ptr(), float(g), float(dmin), float(dmax), int(maxit),
                                  out["d"].data_ptr(), out["nll"].data_ptr(), out["iters"].data_ptr(),
                                  out["status"].data_ptr(), _stream(dev)))
    return out


def local_predict(X, Y, sel, XX, d, g: float) -> dict:
    """Prediction at XX[m] on the fixed design sel[m] with lengthscale d[m] (eqs. predgp, preds2)."""
    L = _lib.load()
    X, Y, XX, sel = _f64(X, "X"), _f64(Y, "Y"), _f64(XX, "XX"), _sel(sel)
    M, n = sel.shape
    dev = X.device
    d = _per_loc(d, M, dev, "d")
    out = {k: torch.empty(M, dtype=torch.float64, device=dev) for k in ("mean", "s2", "var")}
    out["status"] = torch.empty(M, dtype=torch.int32, device=dev)
    _lib.check(L.lagp_local_predict(X.data_ptr(), Y.data_ptr(), X.shape[0], X.shape[1], sel.data_ptr(), M, n,
                                    XX.data_ptr(), d.data_ptr(), float(g), out["mean"].data_ptr(),
                                    out["s2"].data_ptr(), out["var"].data_ptr(), out["status"].data_ptr(),
                                    _stream(dev)))
    return out


def alc_multistage(X, Y, XX, n0: int, n: int, Np: int, d0: float, g: float, stages: int = 2,
                   dmin: float = 1e-3, dmax: float = 5.0, maxit: int = 100) -> dict:
    """Local designs with a lengthscale of each location's own (Fig. 1 with
    step 4): greedy ALC designs at d0 and the MLE of d on each design, then
    `stages - 1` more rounds of designs at each location's estimate and its
    MLE again; the prediction uses the last estimate on the last design.
    Returns pool, sel (M x n), d (the estimates, M), mle (last round) and
    mean, s2, var, status of the prediction."""
    X, Y, XX = _f64(X, "X"), _f64(Y, "Y"), _f64(XX, "XX")
    pool = nn_pool(X, XX, Np)
    d_est = None
    for _ in range(max(1, stages)):
        o = alc_uneven_from_pool(X, Y, XX, pool, n0, n, d0, g, d_per=d_est)
        mle = local_mle_d(X, Y, o["sel"], d0 if d_est is None else d_est, g, dmin, dmax, maxit)
        d_est = mle["d"]
    pred = local_predict(X, Y, o["sel"], XX, d_est, g)
    return dict(pool=pool, sel=o["sel"], d=d_est, mle=mle, design_status=o["status"], **pred)
