"""Local approximate GP regression with greedy ALC designs on MI355X (gfx950).

Thin torch binding of the C ABI in include/lagp_alc.h: tensors supply device
memory, torch's current HIP stream carries the work, and every step of the
path runs in the library's HIP kernels.
"""
from __future__ import annotations

import ctypes
import math

import torch

from . import _lib
from ._lib import LAGP_FP64, LAGP_FP64_REFORM, LAGP_MIXED, LagpError  # noqa: F401

__all__ = ["nn_pool", "nn_pool_static", "mspe_from_pool", "mspe_predict", "alc_scores", "alc_multistage", "alc_from_pool", "alc_predict", "alc_uneven_from_pool", "alc_uneven_predict", "Plan",
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
            grid: bool = False, workspace: torch.Tensor | None = None, group: int = 1) -> torch.Tensor:
    """M x Np int32 pools: the Np nearest design rows of each location, sorted by (distance, index).

    grid: bucket the design into grid cells and stream, nearest cell first, only
    the cells that can hold a pool member (lagp_nn_pool_ws; the same pools),
    with the cells kept in `workspace` (a uint8 device tensor, allocated here if
    None or too small); group: 2 or 4 locations per workgroup sharing the
    stream of cells (lagp_nn_pool_grouped; the same pools)."""
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
    if group == 1:
        _lib.check(L.lagp_nn_pool_ws(X.data_ptr(), X.shape[0], p, XX.data_ptr(), M, Np, out.data_ptr(),
                                     workspace.data_ptr(), workspace.numel(), _stream(X.device)))
    else:
        _lib.check(L.lagp_nn_pool_grouped(X.data_ptr(), X.shape[0], p, XX.data_ptr(), M, Np, int(group),
                                          out.data_ptr(), workspace.data_ptr(), workspace.numel(),
                                          _stream(X.device)))
    return out


def nn_pool_static(X: torch.Tensor, XX: torch.Tensor, Np: int, out: torch.Tensor | None = None) -> torch.Tensor:
    """The grid-pruned pools of nn_pool(grid=True) built in the library's static
    device scratch (lagp_nn_pool_static): the call allocates nothing when `out`
    is given.  Calls on one GPU share that scratch and must not overlap."""
    L = _lib.load()
    X, XX = _f64(X, "X"), _f64(XX, "XX")
    M, p = XX.shape
    if X.dim() != 2 or X.shape[1] != p:
        raise ValueError("X must be N x p with the p of XX")
    if out is None:
        out = torch.empty((M, Np), dtype=torch.int32, device=X.device)
    elif out.dtype != torch.int32 or tuple(out.shape) != (M, Np) or not out.is_contiguous() or out.device != X.device:
        raise ValueError("out must be a contiguous M x Np int32 tensor on the device of X")
    _lib.check(L.lagp_nn_pool_static(X.data_ptr(), X.shape[0], p, XX.data_ptr(), M, Np, out.data_ptr(),
                                     _stream(X.device)))
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


_OUT_SPECS = (("mean", torch.float64, False), ("s2", torch.float64, False), ("var", torch.float64, False),
              ("sel", torch.int32, True), ("alc", torch.float64, True), ("alc32", torch.float64, True),
              ("status", torch.int32, False), ("guard", torch.int32, False))


def _outputs(M: int, n: int, device, out: dict | None = None, rows: int | None = None) -> dict:
    """The output tensors of an ALC call; entries missing from `out` are added
    to it and given ones are checked.  Per-design outputs (sel, alc, alc32) are
    M x n, or flat of length `rows` when rows are given by offsets."""
    o = out if out is not None else {}
    for k, dt, per_design in _OUT_SPECS:
        shape = ((rows,) if rows is not None else (M, n)) if per_design else (M,)
        if k not in o:
            o[k] = torch.empty(shape, dtype=dt, device=device)
            continue
        t = o[k]
        if (not isinstance(t, torch.Tensor) or t.dtype != dt or not t.is_contiguous() or t.device != device
                or t.numel() != math.prod(shape)):
            raise ValueError(f"out[{k!r}] must be a contiguous {dt} tensor of {math.prod(shape)} elements "
                             f"on {device}")
    return o


def _check_xy(X, Y, XX):
    X, Y, XX = _f64(X, "X"), _f64(Y, "Y"), _f64(XX, "XX")
    if X.dim() != 2 or XX.dim() != 2 or X.shape[1] != XX.shape[1]:
        raise ValueError("X must be N x p and XX M x p with the same p")
    if Y.numel() != X.shape[0]:
        raise ValueError("Y must hold one response per row of X")
    if not (X.device == Y.device == XX.device):
        raise ValueError("X, Y and XX must be on one device")
    return X, Y, XX


def _pool_arg(pool, M: int, device) -> torch.Tensor:
    if (not isinstance(pool, torch.Tensor) or pool.dtype != torch.int32 or not pool.is_contiguous()
            or pool.device != device or pool.dim() != 2 or pool.shape[0] != M):
        raise ValueError("pool must be a contiguous M x Np int32 tensor on the device of X")
    return pool


def alc_from_pool(X, Y, XX, pool, n0: int, n: int, d: float, g: float, precision="fp64",
                  out: dict | None = None) -> dict:
    """Greedy ALC local designs and predictions from given pools (M x Np int32)."""
    L = _lib.load()
    X, Y, XX = _check_xy(X, Y, XX)
    M, p = XX.shape
    pool = _pool_arg(pool, M, X.device)
    Np = pool.shape[1]
    o = _outputs(M, n, X.device, out)
    _lib.check(L.lagp_alc_from_pool(
        X.data_ptr(), Y.data_ptr(), X.shape[0], p, XX.data_ptr(), M, pool.data_ptr(), Np, n0, n,
        float(d), float(g), _prec(precision), o["mean"].data_ptr(), o["s2"].data_ptr(),
        o["var"].data_ptr(), o["sel"].data_ptr(), o["alc"].data_ptr(), o["alc32"].data_ptr(),
        o["status"].data_ptr(), o["guard"].data_ptr(), _stream(X.device)))
    return o


def mspe_from_pool(X, Y, XX, pool, n0: int, n: int, d: float, g: float, out: dict | None = None,
                   workspace: torch.Tensor | None = None) -> dict:
    """Local designs by the MSPE criterion (eq. mspe, lagp_mspe_from_pool) from
    given pools, and the predictions on them; out["crit"] holds the criterion
    of each chosen point.  The workspace (uint8 device tensor) is allocated
    here if None or too small."""
    L = _lib.load()
    X, Y, XX = _check_xy(X, Y, XX)
    M, p = XX.shape
    pool = _pool_arg(pool, M, X.device)
    Np = pool.shape[1]
    o = _outputs(M, n, X.device, out)
    if "crit" not in o:
        o["crit"] = torch.empty((M, n), dtype=torch.float64, device=X.device)
    elif (o["crit"].dtype != torch.float64 or not o["crit"].is_contiguous() or o["crit"].device != X.device
          or o["crit"].numel() != M * n):
        raise ValueError(f"out['crit'] must be a contiguous float64 tensor of {M * n} elements on {X.device}")
    nbytes = ctypes.c_size_t(0)
    _lib.check(L.lagp_mspe_workspace(M, Np, n, ctypes.byref(nbytes)))
    if workspace is None or workspace.numel() < nbytes.value:
        workspace = torch.empty(max(nbytes.value, 1), dtype=torch.uint8, device=X.device)
    _lib.check(L.lagp_mspe_from_pool(
        X.data_ptr(), Y.data_ptr(), X.shape[0], p, XX.data_ptr(), M, pool.data_ptr(), Np, n0, n,
        float(d), float(g), o["mean"].data_ptr(), o["s2"].data_ptr(), o["var"].data_ptr(), o["sel"].data_ptr(),
        o["crit"].data_ptr(), o["status"].data_ptr(), workspace.data_ptr(), workspace.numel(),
        _stream(X.device)))
    o["workspace"] = workspace
    return o


def mspe_predict(X, Y, XX, n0: int, n: int, Np: int, d: float, g: float, out: dict | None = None) -> dict:
    """Grid-pruned NN pools, then MSPE designs and predictions (eq. mspe)."""
    pool = nn_pool(X, XX, Np, grid=True)
    o = mspe_from_pool(X, Y, XX, pool, n0, n, d, g, out=out)
    o["pool"] = pool
    return o


def _i32(t, name: str, M: int, device=None) -> int:
    if t is None:
        return 0
    if (not isinstance(t, torch.Tensor) or t.dtype != torch.int32 or not t.is_contiguous() or not t.is_cuda
            or t.numel() != M or (device is not None and t.device != device)):
        raise ValueError(f"{name} must be a contiguous int32 device tensor of length M")
    return t.data_ptr()


def _d_per(t, M: int, device=None) -> int:
    if t is None:
        return 0
    if (not isinstance(t, torch.Tensor) or t.dtype != torch.float64 or not t.is_contiguous() or not t.is_cuda
            or t.numel() != M or (device is not None and t.device != device)):
        raise ValueError("d_per must be a contiguous float64 device tensor of length M")
    return t.data_ptr()


def _sel_off(t, M: int, device) -> int:
    if t is None:
        return 0
    if (not isinstance(t, torch.Tensor) or t.dtype != torch.int64 or not t.is_contiguous() or t.device != device
            or t.numel() != M + 1):
        raise ValueError("sel_off must be a contiguous int64 tensor of length M + 1 on the device of X")
    return t.data_ptr()


def _d_sep(t, p: int, device) -> int:
    if t is None:
        return 0
    if (not isinstance(t, torch.Tensor) or t.dtype != torch.float64 or not t.is_contiguous() or t.device != device
            or t.numel() != p):
        raise ValueError("d_sep must be a contiguous float64 tensor of p lengthscales on the device of X")
    return t.data_ptr()


def _structs(X, Y, XX, n0, n, Np, d, g, precision, n_per, Np_per, d_per, sel_off, normalize, nn, out,
             d_sep=None):
    """lagp_problem and lagp_outputs for these tensors (the outputs dict is
    completed in place, including the pools)."""
    if nn not in ("grid", "brute"):
        raise ValueError("nn must be 'grid' or 'brute'")
    M, p = XX.shape
    dev = X.device
    rows = None
    if sel_off is not None:
        if out is None or "sel" not in out or "alc" not in out:
            raise ValueError("with sel_off, out must supply flat sel (int32) and alc (float64) rows")
        rows = out["sel"].numel()
    o = _outputs(M, n, dev, out, rows)
    if "pool" not in o:
        o["pool"] = torch.empty((M, Np), dtype=torch.int32, device=dev)
    _pool_arg(o["pool"], M, dev)
    if o["pool"].shape[1] != Np:
        raise ValueError("out['pool'] must be M x Np")
    pr = _lib.Problem()
    pr.struct_size = ctypes.sizeof(_lib.Problem)
    pr.flags = (_lib.LAGP_NORMALIZE_ALC if normalize else 0) | (_lib.LAGP_NN_BRUTE if nn == "brute" else 0)
    pr.X, pr.Y, pr.XX = X.data_ptr(), Y.data_ptr(), XX.data_ptr()
    pr.N, pr.M, pr.p, pr.n0, pr.n, pr.Np = X.shape[0], M, p, n0, n, Np
    pr.n_per, pr.Np_per = _i32(n_per, "n_per", M, dev), _i32(Np_per, "Np_per", M, dev)
    pr.d_per = _d_per(d_per, M, dev)
    pr.d_sep = _d_sep(d_sep, p, dev)
    pr.d, pr.g, pr.precision = float(d), float(g), _prec(precision)
    po = _lib.Outputs()
    po.struct_size = ctypes.sizeof(_lib.Outputs)
    for k in ("mean", "s2", "var", "sel", "alc", "alc32", "pool", "status", "guard"):
        setattr(po, k, o[k].data_ptr())
    po.sel_off = _sel_off(sel_off, M, dev)
    return pr, po, o


def _workspace(L, pr, o, dev) -> torch.Tensor:
    nbytes = ctypes.c_size_t(0)
    _lib.check(L.lagp_alc_workspace(ctypes.byref(pr), ctypes.byref(nbytes)))
    ws = o.get("workspace")
    if ws is None or ws.numel() < nbytes.value or ws.data_ptr() % 256:
        ws = o["workspace"] = torch.empty(max(nbytes.value, 1), dtype=torch.uint8, device=dev)
    return ws


def alc_predict(X, Y, XX, n0: int, n: int, Np: int, d: float, g: float, precision="fp64",
                out: dict | None = None, *, n_per=None, Np_per=None, d_per=None, sel_off=None,
                normalize: bool = False, nn: str = "grid", d_sep=None) -> dict:
    """The whole path in one call (lagp_alc_predict): NN pools, greedy ALC
    designs, local predictions.

    n, Np: the sizes of every location, or the upper bounds of n_per / Np_per
    (int32 device tensors of length M); d_per: a lengthscale per location.
    Without sel_off, sel / alc / alc32 are M x n, padded with -1 / NaN past
    n_per[m]; with sel_off (int64, M + 1 offsets), `out` must supply them as
    flat rows.  normalize: scores reported as psi_j Delta / (j - 2) (Sec. 3.1).
    nn: 'grid' (grid-pruned pools) or 'brute' (the whole design streamed); the
    pools are the same.  d_sep: p lengthscales of the separable kernel (float64
    device tensor; d is then unused).  Returns the outputs, the pools and the
    workspace."""
    L = _lib.load()
    X, Y, XX = _check_xy(X, Y, XX)
    pr, po, o = _structs(X, Y, XX, n0, n, Np, d, g, precision, n_per, Np_per, d_per, sel_off, normalize, nn,
                         out, d_sep)
    ws = _workspace(L, pr, o, X.device)
    _lib.check(L.lagp_alc_predict(ctypes.byref(pr), ctypes.byref(po), ws.data_ptr(), ws.numel(),
                                  _stream(X.device)))
    return o


def alc_uneven_from_pool(X, Y, XX, pool, n0: int, n_max: int, d: float, g: float, n_per=None,
                         Np_per=None, sel_off=None, precision="fp64", out: dict | None = None,
                         d_per=None) -> dict:
    """Greedy ALC designs with a design size n_per[m] and a pool size Np_per[m]
    of each location's own (int32 device tensors, None = n_max / the pool
    width) and optionally a lengthscale d_per[m] of its own (float64, None = d).
    pool: M x Np_max from nn_pool(X, XX, Np_max).  Without sel_off, sel and alc
    are M x n_max with entries past n_per[m] set to -1 / NaN; with sel_off
    (int64, M + 1 offsets) they are flat rows, and `out` must supply them."""
    L = _lib.load()
    X, Y, XX = _check_xy(X, Y, XX)
    M, p = XX.shape
    dev = X.device
    pool = _pool_arg(pool, M, dev)
    Np_max = pool.shape[1]
    rows = None
    if sel_off is not None:
        if out is None or "sel" not in out or "alc" not in out:
            raise ValueError("with sel_off, out must supply flat sel (int32) and alc (float64)")
        rows = out["sel"].numel()
    o = _outputs(M, n_max, dev, out, rows)
    nbytes = ctypes.c_size_t(0)
    _lib.check(L.lagp_alc_uneven_workspace(p, M, Np_max, n_max, ctypes.byref(nbytes)))
    ws = o.get("workspace")
    if ws is None or ws.numel() < nbytes.value:
        ws = o["workspace"] = torch.empty(max(nbytes.value, 1), dtype=torch.uint8, device=dev)
    _lib.check(L.lagp_alc_uneven_from_pool(
        X.data_ptr(), Y.data_ptr(), X.shape[0], p, XX.data_ptr(), M, pool.data_ptr(), Np_max, n0, n_max,
        _i32(n_per, "n_per", M, dev), _i32(Np_per, "Np_per", M, dev), _sel_off(sel_off, M, dev),
        _d_per(d_per, M, dev), float(d), float(g), _prec(precision),
        o["mean"].data_ptr(), o["s2"].data_ptr(), o["var"].data_ptr(), o["sel"].data_ptr(),
        o["alc"].data_ptr(), o["status"].data_ptr(), o["guard"].data_ptr(), ws.data_ptr(), ws.numel(),
        _stream(dev)))
    return o


def alc_uneven_predict(X, Y, XX, n0: int, n_max: int, Np_max: int, d: float, g: float, n_per=None,
                       Np_per=None, precision="fp64", out: dict | None = None, d_per=None) -> dict:
    """The whole path with per-location n and N' (alc_predict with n_per /
    Np_per / d_per): one pool of the Np_max nearest neighbours per location,
    each location using its own prefix."""
    return alc_predict(X, Y, XX, n0, n_max, Np_max, d, g, precision, out, n_per=n_per, Np_per=Np_per,
                       d_per=d_per)


class Plan:
    """alc_predict for one problem bound to fixed buffers, autotuned on these
    inputs and captured into one HIP graph (lagp_plan_create).  `out` holds the
    pools and the outputs (sel and alc padded to M x n); `launch()` enqueues one
    run on torch's current stream.  The plan keeps references to the input
    tensors, which must not be modified in place while it is used."""

    def __init__(self, X, Y, XX, n0: int, n_max: int, Np_max: int, d: float, g: float, n_per=None,
                 Np_per=None, tune: bool = True, d_per=None, precision="fp64", normalize: bool = False,
                 nn: str = "grid", d_sep=None, schedule: int | None = None):
        L = _lib.load()
        X, Y, XX = _check_xy(X, Y, XX)
        dev = X.device
        pr, po, o = _structs(X, Y, XX, n0, n_max, Np_max, d, g, precision, n_per, Np_per, d_per, None,
                             normalize, nn, None, d_sep)
        ws = _workspace(L, pr, o, dev)
        self._keep = (X, Y, XX, n_per, Np_per, d_per, d_sep)
        self.out, self._dev, self._h = o, dev, ctypes.c_void_p()
        flags = 0 if tune else _lib.LAGP_PLAN_NO_TUNE
        if schedule is not None:  # run this ALC schedule wherever it serves (LAGP_PLAN_SCHEDULE)
            if not 0 <= int(schedule) < _lib.LAGP_PLAN_SCHEDULES:
                raise ValueError(f"schedule must be in [0, {_lib.LAGP_PLAN_SCHEDULES})")
            flags |= (int(schedule) + 1) << 8
        _lib.check(L.lagp_plan_create(ctypes.byref(pr), ctypes.byref(po), ws.data_ptr(), ws.numel(),
                                      flags, _stream(dev), ctypes.byref(self._h)))

    def launch(self) -> dict:
        _lib.check(_lib.load().lagp_plan_launch(self._h, _stream(self._dev)))
        return self.out

    def describe(self) -> str:
        buf = ctypes.create_string_buffer(4096)
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


def _sel(sel: torch.Tensor, device=None) -> torch.Tensor:
    if (not isinstance(sel, torch.Tensor) or sel.dtype != torch.int32 or not sel.is_contiguous()
            or not sel.is_cuda or sel.dim() != 2 or (device is not None and sel.device != device)):
        raise ValueError("sel must be a contiguous M x n int32 tensor on the device of X")
    return sel


def _per_loc(v, M: int, device, name: str) -> torch.Tensor:
    """A parameter of every location: a scalar, a 1-element tensor (broadcast)
    or a tensor of M values; anything else is refused before any launch."""
    if isinstance(v, torch.Tensor):
        if v.numel() == M:
            t = v.reshape(M)
        elif v.numel() == 1:
            t = v.reshape(1).expand(M).contiguous()
        else:
            raise ValueError(f"{name} must be a scalar or hold one value per location (M = {M}), "
                             f"not {v.numel()}")
        if t.device != device:
            raise ValueError(f"{name} must be on the device of X")
        return _f64(t.contiguous(), name)
    return torch.full((M,), float(v), dtype=torch.float64, device=device)


def _xy(X, Y):
    X, Y = _f64(X, "X"), _f64(Y, "Y")
    if X.dim() != 2 or Y.numel() != X.shape[0] or X.device != Y.device:
        raise ValueError("X must be N x p and Y hold N responses on the same device")
    return X, Y


def local_nll(X, Y, sel, d, g, order: int = 0) -> dict:
    """Negative log of eq. gpk on each location's fixed design (float64).

    order 0: nll; 1: + dnll/dd, dnll/dg; 2: + d2nll/dd2.  d, g: scalars or M-vectors.
    """
    L = _lib.load()
    X, Y = _xy(X, Y)
    sel = _sel(sel, X.device)
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
        X, Y = _xy(X, Y)
        sel = _sel(sel, X.device)
        M = sel.shape[0]
        # d and g: M values each, or one shared value broadcast to every location
        dm = _per_loc(d.detach(), M, X.device, "d")
        gm = _per_loc(g.detach(), M, X.device, "g")
        out = local_nll(X, Y, sel, dm, gm, order=0)
        ctx.save_for_backward(dm, gm)
        ctx.shapes = (d.shape, g.shape)
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
        # a shared (broadcast) parameter receives the sum over the locations
        sd, sg = ctx.shapes
        if gd is not None and math.prod(sd) != M:
            gd = gd.sum().reshape(sd)
        elif gd is not None:
            gd = gd.reshape(sd)
        if gg is not None and math.prod(sg) != M:
            gg = gg.sum().reshape(sg)
        elif gg is not None:
            gg = gg.reshape(sg)
        return gd, gg, None, None, None


def local_mle_d(X, Y, sel, d0, g: float, dmin: float = 1e-3, dmax: float = 5.0, maxit: int = 100) -> dict:
    """Maximum-likelihood lengthscale per location (projected Newton, g fixed)."""
    L = _lib.load()
    X, Y = _xy(X, Y)
    sel = _sel(sel, X.device)
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
    X, Y, XX = _check_xy(X, Y, XX)
    sel = _sel(sel, X.device)
    M, n = sel.shape
    if XX.shape[0] != M:
        raise ValueError("XX must hold one location per row of sel")
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
