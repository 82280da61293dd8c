"""Comparison protocol between the GPU path and the CPU oracle.

Sequences.  Two exact-arithmetic-equivalent float64 routes can order two
near-tied candidates differently, so a selected index is compared with the
oracle *along the GPU's own prefix*: the oracle is forced through the GPU's
sequence and, at every step, the GPU's choice must score within tau_j of the
oracle's best, relatively.  tau_j = max(1e-12, 10 nu_j), where nu_j is the
oracle's own route noise at that step (its Cholesky route versus the
paper's partitioned-inverse route, eqs. piedef and dxy), i.e. a difference
the arithmetic cannot resolve.  Steps where the GPU picks another index are
counted as ties.

Outputs.  mean, s2 and var are compared on the GPU's final design with the
oracle forced through it.  Relative tolerance tau_out (1e-10 float64, 1e-4
mixed), raised only where the oracle's two float64 routes on that same design
disagree by more: 10 x the measured output route noise, i.e. the gap between
the oracle's Cholesky prediction and its prediction through the K_n^{-1}
grown by the partitioned inverse (eq. piedef), location by location.
"""
from __future__ import annotations

import numpy as np

EPS = np.finfo(np.float64).eps


def sequence_check(gpu_sel, pool, forced, n0, n_per=None, tau_floor=1e-12, nu_mult=10.0):
    """forced: oracle.alc(..., forced=gpu_sel, mode_b=True).  Returns stats; lists fails."""
    M = gpu_sel.shape[0]
    ties, fails, max_r = 0, [], 0.0
    for m in range(M):
        n = gpu_sel.shape[1] if n_per is None else int(n_per[m])
        if not np.array_equal(gpu_sel[m, :n0], pool[m, :n0]):
            fails.append((m, -1, "initial design is not the first n0 pool entries"))
            continue
        for j in range(n0, n):
            if gpu_sel[m, j] == forced["amax"][m, j]:
                continue
            dm, ds = forced["dmax"][m, j], forced["dsel"][m, j]
            r = (dm - ds) / dm
            tau = max(tau_floor, nu_mult * forced["nu"][m, j])
            ties += 1
            max_r = max(max_r, r)
            if not r <= tau:
                fails.append((m, j, r, tau))
    return dict(ties=ties, max_r=max_r, fails=fails)


def cond_bounds(X, sel, d, g):
    """kappa * eps * cond(K_n) per location (relative resolution of v); d is a
    scalar or one lengthscale per location."""
    out = np.empty(sel.shape[0])
    dv = np.broadcast_to(np.asarray(d, dtype=float), (sel.shape[0],))
    for m in range(sel.shape[0]):
        d = float(dv[m])
        D = X[sel[m]]
        r2 = np.zeros((len(D), len(D)))
        for k in range(D.shape[1]):
            t = D[:, k][:, None] - D[:, k][None, :]
            r2 = r2 + t * t
        K = np.exp(-r2 / d) + g * np.eye(len(D))
        out[m] = (1 + g) * EPS * np.linalg.cond(K)
    return out


def route_gap(forced, k, floor=0.0):
    """Relative gap between the oracle's two float64 routes for output k on the
    same design (forced must come from oracle.alc(..., mode_b=True))."""
    a, b = forced[k], forced[k + "_b"]
    return np.abs(a - b) / np.maximum(np.abs(a), floor)


def output_tolerance(forced, k, tau_out, floor=0.0, mult=10.0):
    """Per-location tolerance: tau_out, or 10x the measured route gap if larger."""
    return np.maximum(tau_out, mult * route_gap(forced, k, floor))


def output_check(gpu, forced, X, d, g, tau_out, mean_floor):
    """Relative output errors; returns (worst excess over tolerance, report)."""
    rep = {}
    worst = 0.0
    for k in ("mean", "s2", "var"):
        a, b = gpu[k], forced[k]
        floor = mean_floor if k == "mean" else 0.0
        rel = np.abs(a - b) / np.maximum(np.abs(b), floor)
        gap = route_gap(forced, k, floor)
        tol = output_tolerance(forced, k, tau_out, floor)
        assert np.all(np.isfinite(tol)), "the oracle's mode-B prediction is missing"
        rep[k] = dict(max_rel=float(np.max(rel)), max_route_gap=float(np.max(gap)),
                      n_route_limited=int(np.sum(tol > tau_out)), max_tol=float(np.max(tol)))
        worst = max(worst, float(np.max(rel / tol)))
    return worst, rep
