"""ctypes binding of the FP64 CPU oracle (``lagp_oracle.c``).

TEST INFRASTRUCTURE ONLY: the tests, the smoke check and the benchmark's CPU
baseline use it; the GPU library never does.  It shares no code with the GPU
path.  See ``lagp_oracle.c`` for the method and the readings of the paper.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(_HERE, "lagp_oracle.c")
LIB = os.path.join(_HERE, "liboracle.so")

STATUS = {0: "ok", 1: "init not PD", 2: "step failure", 3: "non-finite", 4: "bad forced", 5: "bad args"}

CFLAGS = ["-O2", "-std=c11", "-fopenmp", "-ffp-contract=off", "-fno-fast-math", "-fPIC", "-shared"]


def compile_c(src: str, out: str) -> str:
    subprocess.run(["gcc", *CFLAGS, src, "-o", out + ".tmp", "-lm"], check=True)
    os.replace(out + ".tmp", out)
    return out


def build(force: bool = False) -> str:
    """Compile the oracle with gcc (FP64, OpenMP, no contraction)."""
    if force or not os.path.exists(LIB) or os.path.getmtime(LIB) < os.path.getmtime(SRC):
        compile_c(SRC, LIB)
    return LIB


def _p(a):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def _i32(a):
    return None if a is None else np.ascontiguousarray(a, dtype=np.int32)


class Oracle:
    """One loaded copy of the oracle library."""

    def __init__(self, path: str):
        L = ctypes.CDLL(path)
        P = ctypes.c_void_p
        i64, i32, f64 = ctypes.c_int64, ctypes.c_int, ctypes.c_double
        L.orc_nn_pool.argtypes = [P, i64, i32, P, i64, i32, P, i32]
        L.orc_nn_pool.restype = i32
        L.orc_gp_predict.argtypes = [P, P, i32, i32, P, f64, f64, P]
        L.orc_gp_predict.restype = i32
        L.orc_gp_predict_b.argtypes = [P, P, i32, i32, P, f64, f64, P]
        L.orc_gp_predict_b.restype = i32
        L.orc_gp_predict_sep.argtypes = [P, P, i32, i32, P, P, f64, P]
        L.orc_gp_predict_sep.restype = i32
        L.orc_alc.argtypes = [P, P, i64, i32, P, i64, P, i32, P, i32, P, i32, i32, i32, f64, P, P, f64,
                              P, i32, i32, P, P, P, P, P, P, P, P, P, P, P]
        L.orc_alc.restype = i32
        L.orc_alc_scores.argtypes = [P, i32, i32, P, i64, P, f64, f64, i32, P, P, P]
        L.orc_alc_scores.restype = i32
        L.orc_max_threads.argtypes = []
        L.orc_max_threads.restype = i32
        L.orc_nll.argtypes = [P, P, i32, i32, f64, f64, P]
        L.orc_nll.restype = i32
        L.orc_mle_d.argtypes = [P, P, i32, i32, f64, f64, f64, f64, i32, P]
        L.orc_mle_d.restype = i32
        L.orc_local_mle.argtypes = [P, P, i32, P, i64, i32, P, f64, f64, f64, i32, i32, P]
        L.orc_local_mle.restype = i32
        L.orc_mspe.argtypes = [P, P, i64, i32, P, i64, P, i32, i32, i32, f64, f64, P, i32, i32,
                               P, P, P, P, P, P, P, P, P]
        L.orc_mspe.restype = i32
        self.L = L

    def nn_pool(self, X, XX, Np: int, threads: int = 0) -> np.ndarray:
        """M x Np int32: the Np nearest design rows of each location, sorted by (sq. distance, index)."""
        X, XX = _f64(X), _f64(np.atleast_2d(XX))
        M = XX.shape[0]
        pool = np.empty((M, Np), dtype=np.int32)
        rc = self.L.orc_nn_pool(_p(X), X.shape[0], X.shape[1], _p(XX), M, Np, _p(pool), threads)
        if rc:
            raise ValueError(f"orc_nn_pool: {STATUS.get(rc, rc)}")
        return pool

    def gp_predict(self, D, Yd, x, d: float, g: float) -> dict:
        """Textbook GP prediction on a fixed design (eqs. predgp, preds2)."""
        D, Yd, x = _f64(np.atleast_2d(D)), _f64(Yd), _f64(x)
        out = np.empty(5)
        rc = self.L.orc_gp_predict(_p(D), _p(Yd), D.shape[0], D.shape[1], _p(x), d, g, _p(out))
        return dict(mean=out[0], s2=out[1], var=out[2], v=out[3], psi=out[4], status=rc)

    def gp_predict_sep(self, D, Yd, x, dsep, g: float) -> dict:
        """gp_predict with the separable kernel (dsep: p lengthscales)."""
        D, Yd, x, dsep = _f64(np.atleast_2d(D)), _f64(Yd), _f64(x), _f64(dsep)
        out = np.empty(5)
        rc = self.L.orc_gp_predict_sep(_p(D), _p(Yd), D.shape[0], D.shape[1], _p(x), _p(dsep), g, _p(out))
        return dict(mean=out[0], s2=out[1], var=out[2], v=out[3], psi=out[4], status=rc)

    def gp_predict_b(self, D, Yd, x, d: float, g: float) -> dict:
        """gp_predict through K^{-1} grown row by row by the partitioned inverse
        (eq. piedef): the paper's route, for the output route noise."""
        D, Yd, x = _f64(np.atleast_2d(D)), _f64(Yd), _f64(x)
        out = np.empty(5)
        rc = self.L.orc_gp_predict_b(_p(D), _p(Yd), D.shape[0], D.shape[1], _p(x), d, g, _p(out))
        return dict(mean=out[0], s2=out[1], var=out[2], v=out[3], psi=out[4], status=rc)

    def alc(self, X, Y, XX, pool, n0: int, n: int, d: float, g: float, *, Np: int | None = None,
            n_per=None, Np_per=None, forced=None, mode_b: bool = False, threads: int = 0,
            d_per=None, dsep=None) -> dict:
        """Greedy ALC local designs and local predictions for every location
        (d_per: an own lengthscale per location, overriding d; dsep: p
        lengthscales of the separable kernel, overriding d).

        Returns arrays: sel, dsel, dmax, amax, dsecond, nu, psitraj (M x nmax),
        vtraj (M x (nmax + 1)), mean, s2, var, v, psi (M), status (M); with
        mode_b also mean_b, s2_b, var_b, v_b, psi_b (M): the prediction on the
        same design through the partitioned-inverse K_n^{-1} (eq. piedef).
        """
        X, Y, XX = _f64(X), _f64(Y), _f64(np.atleast_2d(XX))
        pool = _i32(np.atleast_2d(pool))
        M, Np_stride = pool.shape
        Np = Np_stride if Np is None else Np
        n_per, Np_per = _i32(n_per), _i32(Np_per)
        nmax = int(n_per.max()) if n_per is not None and len(n_per) else n
        forced = None if forced is None else _i32(np.atleast_2d(forced))
        if forced is not None:
            nmax = max(nmax, forced.shape[1])
            assert forced.shape == (M, nmax)
        sel = np.full((M, nmax), -1, np.int32)
        amax = np.full((M, nmax), -1, np.int32)
        dsel, dmax, dsecond, nu, psitraj = (np.full((M, nmax), np.nan) for _ in range(5))
        vtraj = np.full((M, nmax + 1), np.nan)
        pred = np.full((M, 5), np.nan)
        pred_b = np.full((M, 5), np.nan)
        status = np.zeros(M, np.int32)
        d_per = None if d_per is None else _f64(d_per)
        dsep = None if dsep is None else _f64(dsep)
        assert dsep is None or dsep.shape == (X.shape[1],)
        rc = self.L.orc_alc(_p(X), _p(Y), X.shape[0], X.shape[1], _p(XX), M, _p(pool), Np_stride,
                            _p(Np_per), Np, _p(n_per), n, nmax, n0, d, _p(d_per), _p(dsep), g, _p(forced),
                            int(mode_b),
                            threads, _p(sel), _p(dsel), _p(dmax), _p(amax), _p(dsecond), _p(nu),
                            _p(vtraj), _p(pred), _p(status), _p(psitraj), _p(pred_b))
        if rc:
            raise ValueError(f"orc_alc: {STATUS.get(rc, rc)}")
        out = dict(sel=sel, dsel=dsel, dmax=dmax, amax=amax, dsecond=dsecond, nu=nu, psitraj=psitraj,
                   vtraj=vtraj, mean=pred[:, 0], s2=pred[:, 1], var=pred[:, 2], v=pred[:, 3],
                   psi=pred[:, 4], status=status)
        if mode_b:
            for q, k in enumerate(("mean_b", "s2_b", "var_b", "v_b", "psi_b")):
                out[k] = pred_b[:, q]
        return out

    def lagp(self, X, Y, XX, n0: int, n: int, Np: int, d: float, g: float, **kw) -> dict:
        """Nearest-neighbour pool, greedy ALC design and prediction for every location."""
        pool = self.nn_pool(X, XX, Np, threads=kw.get("threads", 0))
        out = self.alc(X, Y, XX, pool, n0, n, d, g, **kw)
        out["pool"] = pool
        return out

    def max_threads(self) -> int:
        return self.L.orc_max_threads()

    def alc_scores(self, Xj, Xc, x, d: float, g: float, mode_b: bool = False) -> dict:
        """Scores v_j(x) - v_{j+1}(x) of every candidate row of Xc against the
        design Xj at x (eq. dxy): delta (Nc), with K_j^{-1} (Kinv) and
        h = K(X_j, x) as used by the paper's per-step kernel."""
        Xj, Xc, x = _f64(np.atleast_2d(Xj)), _f64(np.atleast_2d(Xc)), _f64(x)
        j, p = Xj.shape
        Kinv, h = np.empty((j, j)), np.empty(j)
        delta = np.empty(Xc.shape[0])
        rc = self.L.orc_alc_scores(_p(Xj), j, p, _p(Xc), Xc.shape[0], _p(x), d, g, int(mode_b), _p(Kinv),
                                   _p(h), _p(delta))
        if rc:
            raise ValueError(f"orc_alc_scores: {STATUS.get(rc, rc)}")
        return dict(delta=delta, Kinv=Kinv, h=h)

    def nll(self, D, Yd, d: float, g: float) -> dict:
        """Negative log of eq. gpk and its derivatives: nll, dd, dg, d2 (d2nll/dd2)."""
        D, Yd = _f64(np.atleast_2d(D)), _f64(Yd)
        out = np.empty(4)
        rc = self.L.orc_nll(_p(D), _p(Yd), D.shape[0], D.shape[1], d, g, _p(out))
        return dict(nll=out[0], dd=out[1], dg=out[2], d2=out[3], status=rc)

    def mle_d(self, D, Yd, d0: float, g: float, dmin: float = 1e-3, dmax: float = 5.0,
              maxit: int = 100) -> dict:
        """Projected-Newton maximum-likelihood lengthscale on one fixed design."""
        D, Yd = _f64(np.atleast_2d(D)), _f64(Yd)
        out = np.empty(4)
        self.L.orc_mle_d(_p(D), _p(Yd), D.shape[0], D.shape[1], d0, g, dmin, dmax, maxit, _p(out))
        return dict(d=out[0], nll=out[1], iters=int(out[2]), status=int(out[3]))

    def local_mle(self, X, Y, sel, d0, g: float, dmin: float = 1e-3, dmax: float = 5.0,
                  maxit: int = 100, threads: int = 0) -> dict:
        """mle_d for every location's design (sel: M x n design indices)."""
        X, Y = _f64(X), _f64(Y)
        sel = _i32(np.atleast_2d(sel))
        M, n = sel.shape
        d0 = _f64(np.broadcast_to(np.asarray(d0, dtype=np.float64), (M,)))
        out = np.empty((M, 4))
        self.L.orc_local_mle(_p(X), _p(Y), X.shape[1], _p(sel), M, n, _p(d0), g, dmin, dmax, maxit,
                             threads, _p(out))
        return dict(d=out[:, 0], nll=out[:, 1], iters=out[:, 2].astype(int), status=out[:, 3].astype(int))


    def mspe(self, X, Y, XX, pool, n0: int, n: int, d: float, g: float, *, forced=None, mode_b: bool = False,
             threads: int = 0) -> dict:
        """Local designs by the MSPE criterion (eq. mspe): at every step the
        candidate minimising V_j(x | x') + (d mu_j / dd)^2 / G_{j+1}.  Returns
        sel, jsel (criterion of the choice), jmin, amin (its smallest value and
        where), nu (route noise, mode_b), dmu, gsel (M x n), the prediction on
        the final design (mean, s2, var, v, psi) and status."""
        X, Y, XX = _f64(X), _f64(Y), _f64(np.atleast_2d(XX))
        pool = _i32(np.atleast_2d(pool))
        M, Np = pool.shape
        forced = None if forced is None else _i32(np.atleast_2d(forced))
        if forced is not None:
            assert forced.shape == (M, n)
        sel, amin = np.full((M, n), -1, np.int32), np.full((M, n), -1, np.int32)
        jsel, jmin, nu, dmu, gsel = (np.full((M, n), np.nan) for _ in range(5))
        pred = np.full((M, 5), np.nan)
        status = np.zeros(M, np.int32)
        rc = self.L.orc_mspe(_p(X), _p(Y), X.shape[0], X.shape[1], _p(XX), M, _p(pool), Np, n0, n, d, g,
                             _p(forced), int(mode_b), threads, _p(sel), _p(jsel), _p(jmin), _p(amin), _p(nu),
                             _p(dmu), _p(gsel), _p(pred), _p(status))
        if rc:
            raise ValueError(f"orc_mspe: {STATUS.get(rc, rc)}")
        return dict(sel=sel, jsel=jsel, jmin=jmin, amin=amin, nu=nu, dmu=dmu, gsel=gsel, mean=pred[:, 0],
                    s2=pred[:, 1], var=pred[:, 2], v=pred[:, 3], psi=pred[:, 4], status=status)


_default: Oracle | None = None


def default() -> Oracle:
    global _default
    if _default is None:
        _default = Oracle(build())
    return _default


def nn_pool(*a, **k):
    return default().nn_pool(*a, **k)


def gp_predict(*a, **k):
    return default().gp_predict(*a, **k)


def gp_predict_b(*a, **k):
    return default().gp_predict_b(*a, **k)


def alc(*a, **k):
    return default().alc(*a, **k)


def lagp(*a, **k):
    return default().lagp(*a, **k)


def alc_scores(*a, **k):
    return default().alc_scores(*a, **k)


def max_threads() -> int:
    return default().max_threads()


def nll(*a, **k):
    return default().nll(*a, **k)


def mle_d(*a, **k):
    return default().mle_d(*a, **k)


def local_mle(*a, **k):
    return default().local_mle(*a, **k)


def mspe(*a, **k):
    return default().mspe(*a, **k)
