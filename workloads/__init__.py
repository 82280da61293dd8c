"""Seeded synthetic workloads for local approximate GP regression with ALC designs.

This module only draws inputs: designs, responses, predictive sets and
per-location sizes.  It holds none of the method's arithmetic, so both the
CPU oracle (test infrastructure) and the GPU path can be fed from it.

The workloads stand in for the paper's data sets (the 2-d data of Sec. 4, the
LGBB runs of Sec. 5.1 and the 8-d benchmark function of Sec. 5.2, Table 1),
which are not available: inputs are uniform iid on the unit cube, responses
are smooth closed-form surfaces with optional Gaussian noise.

Random streams: ``numpy.random.default_rng([13105182, cfg, stream])`` with
stream 0 = design X, 1 = predictive set XX, 2 = response noise,
3 = per-location local design size n then candidate count N' (config 3).
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

SEED_ROOT = 13105182


def _rng(cfg: int, stream: int) -> np.random.Generator:
    return np.random.default_rng([SEED_ROOT, cfg, stream])


def response_sines(X: np.ndarray) -> np.ndarray:
    """sum_k sin(2*pi*x_k*(k+1)/4) over k = 1..p (1-based) plus x1*x2*x3."""
    p = X.shape[1]
    y = np.zeros(X.shape[0])
    for k in range(1, p + 1):
        y += np.sin(2.0 * math.pi * X[:, k - 1] * (k + 1) / 4.0)
    if p >= 3:
        y += X[:, 0] * X[:, 1] * X[:, 2]
    return y


def response_2d(X: np.ndarray) -> np.ndarray:
    """sin(5*x1) + cos(7*x2) + 0.5*x1*x2."""
    return np.sin(5.0 * X[:, 0]) + np.cos(7.0 * X[:, 1]) + 0.5 * X[:, 0] * X[:, 1]


def response_mle(X: np.ndarray) -> np.ndarray:
    """sin(6*x1)*cos(4*x2) + x3^2 - x4."""
    return np.sin(6.0 * X[:, 0]) * np.cos(4.0 * X[:, 1]) + X[:, 2] ** 2 - X[:, 3]


@dataclasses.dataclass
class Workload:
    """One problem instance.  Arrays are float64 / int32, C-contiguous."""

    name: str
    X: np.ndarray
    Y: np.ndarray
    XX: np.ndarray
    n0: int
    n: int
    Np: int
    d: float
    g: float
    n_per: np.ndarray | None = None
    Np_per: np.ndarray | None = None

    @property
    def N(self) -> int:
        return self.X.shape[0]

    @property
    def p(self) -> int:
        return self.X.shape[1]

    @property
    def M(self) -> int:
        return self.XX.shape[0]


# Full-size shapes of the five workloads: (N, p, M, n0, n, Np, d, g, response, noise variance).
CONFIGS = {
    1: dict(N=4000, p=2, M=100, n0=6, n=50, Np=500, d=0.1, g=1e-6, resp=response_2d, noise=0.0),
    2: dict(N=100_000, p=8, M=10_000, n0=6, n=50, Np=1000, d=0.5, g=1e-4, resp=response_sines, noise=1e-4),
    3: dict(N=200_000, p=4, M=50_000, n0=6, n=100, Np=2000, d=0.3, g=1e-5, resp=response_sines, noise=1e-4),
    4: dict(N=100_000, p=4, M=10_000, n0=6, n=50, Np=1000, d=0.2, g=1e-3, resp=response_mle, noise=1e-3),
    5: dict(N=1_000_000, p=8, M=1_000_000, n0=6, n=50, Np=1000, d=0.5, g=1e-4, resp=response_sines, noise=1e-4),
}


def make(cfg: int, N: int | None = None, M: int | None = None, **over) -> Workload:
    """Draw workload ``cfg`` (1..5).

    ``N`` and ``M`` override the design and predictive-set sizes; the
    predictive set is drawn at its full size and its first ``M`` rows kept, so
    a subsample is a prefix of the full workload.  Other keyword arguments
    override n0, n, Np, d, g.
    """
    c = dict(CONFIGS[cfg])
    full_M = c["M"]
    N = c["N"] if N is None else int(N)
    M = full_M if M is None else int(M)
    p = c["p"]
    X = _rng(cfg, 0).random((N, p))
    XX_full = _rng(cfg, 1).random((max(full_M, M), p))
    XX = np.ascontiguousarray(XX_full[:M])
    Y = c["resp"](X)
    if c["noise"] > 0:
        Y = Y + _rng(cfg, 2).normal(0.0, math.sqrt(c["noise"]), N)
    n_per = Np_per = None
    if cfg == 3:
        r = _rng(cfg, 3)
        n_full = r.integers(20, 101, max(full_M, M)).astype(np.int32)
        Np_full = r.integers(200, 2001, max(full_M, M)).astype(np.int32)
        n_per = np.ascontiguousarray(n_full[:M])
        Np_per = np.ascontiguousarray(Np_full[:M])
    w = Workload(
        name=f"config{cfg}", X=np.ascontiguousarray(X), Y=np.ascontiguousarray(Y), XX=XX,
        n0=c["n0"], n=c["n"], Np=c["Np"], d=c["d"], g=c["g"], n_per=n_per, Np_per=Np_per,
    )
    for k, v in over.items():
        setattr(w, k, v)
    return w


def uniform(seed: int, N: int, p: int, M: int, *, resp=response_sines, noise: float = 0.0) -> tuple:
    """Small ad-hoc uniform problem (X, Y, XX) for unit tests."""
    r = np.random.default_rng([SEED_ROOT, 1000 + seed])
    X = r.random((N, p))
    XX = r.random((M, p))
    Y = resp(X)
    if noise > 0:
        Y = Y + r.normal(0.0, math.sqrt(noise), N)
    return np.ascontiguousarray(X), np.ascontiguousarray(Y), np.ascontiguousarray(XX)


def lengthscales(M: int, lo: float, hi: float, seed: int = 0) -> np.ndarray:
    """A lengthscale per location, log-uniform on [lo, hi] (inputs for designs
    with each location's own d)."""
    r = np.random.default_rng([SEED_ROOT, 200, M, seed])
    return np.exp(r.uniform(np.log(lo), np.log(hi), M))


def scores_case(j: int, Nc: int, p: int, seed: int = 0, spread: float = 0.25) -> tuple:
    """One location with a design of j points and Nc candidates (the shape of
    the paper's ALC-in-isolation experiment, Sec. 4): x uniform on the unit
    cube, the design uniform in the cube of half-width `spread` around x, the
    candidates uniform on the unit cube.  Returns (Xj, Xc, x), float64."""
    r = np.random.default_rng([SEED_ROOT, 100 + p, j, seed])
    x = r.random(p)
    Xj = x + spread * (2.0 * r.random((j, p)) - 1.0)
    Xc = r.random((Nc, p))
    return Xj, Xc, x
