"""NumPy brute force for tiny inputs: every quantity from its definition with
fresh dense solves, no partitioned inverses, no Cholesky updates.

Test infrastructure.  Used to pin the oracle (and nothing else).
"""
from __future__ import annotations

import numpy as np


def sqdist_rows(A: np.ndarray, b: np.ndarray) -> np.ndarray:
    """Squared distances of the rows of A to b, summed left to right."""
    s = np.zeros(A.shape[0])
    for k in range(A.shape[1]):
        t = A[:, k] - b[k]
        s = s + t * t
    return s


def corr(A: np.ndarray, B: np.ndarray, d) -> np.ndarray:
    """exp(-||a - b||^2 / d) for all row pairs (Sec. 2.1); with d a vector of
    one lengthscale per input, the separable form exp(-sum_k (a_k - b_k)^2 / d_k)."""
    out = np.empty((A.shape[0], B.shape[0]))
    dv = np.asarray(d, dtype=float)
    for j in range(B.shape[0]):
        if dv.ndim == 0:
            out[:, j] = np.exp(-sqdist_rows(A, B[j]) / d)
        else:
            s = np.zeros(A.shape[0])
            for k in range(A.shape[1]):
                t = A[:, k] - B[j, k]
                s = s + t * t / dv[k]
            out[:, j] = np.exp(-s)
    return out


def pool(X: np.ndarray, x: np.ndarray, Np: int) -> np.ndarray:
    dist = sqdist_rows(X, x)
    order = np.lexsort((np.arange(X.shape[0]), dist))
    return order[:Np].astype(np.int32)


def v_of(D: np.ndarray, x: np.ndarray, d: float, g: float) -> float:
    """v(x) = K(x,x) - k^T K^{-1} k with K(x,x) = 1 + g (eq. newv)."""
    if D.shape[0] == 0:
        return 1.0 + g
    K = corr(D, D, d) + g * np.eye(D.shape[0])
    k = corr(D, x[None, :], d)[:, 0]
    return 1.0 + g - k @ np.linalg.solve(K, k)


def delta(D: np.ndarray, c: np.ndarray, x: np.ndarray, d: float, g: float) -> float:
    """v_j(x) - v_{j+1}(x) with c appended, from two fresh solves (eq. dxy, left side)."""
    return v_of(D, x, d, g) - v_of(np.vstack([D, c[None, :]]), x, d, g)


def predict(D: np.ndarray, Yd: np.ndarray, x: np.ndarray, d: float, g: float) -> dict:
    """Eqs. predgp and preds2 with N -> n, via numpy.linalg.solve."""
    n = D.shape[0]
    K = corr(D, D, d) + g * np.eye(n)
    k = corr(D, x[None, :], d)[:, 0]
    a = np.linalg.solve(K, Yd)
    psi = Yd @ a
    v = 1.0 + g - k @ np.linalg.solve(K, k)
    s2 = psi * v / n
    return dict(mean=k @ a, s2=s2, var=s2 * n / (n - 2) if n > 2 else np.nan, v=v, psi=psi)


def greedy(X: np.ndarray, x: np.ndarray, P: np.ndarray, n0: int, n: int, d: float, g: float):
    """Fig. 1 steps 2a-2b by brute force: returns (sel, best score per step)."""
    sel = list(P[:n0])
    best = []
    for _ in range(n0, n):
        D = X[sel]
        scores = []
        for c in P:
            if c in sel:
                continue
            scores.append((delta(D, X[c], x, d, g), -c, c))
        s, _, c = max(scores)
        sel.append(c)
        best.append(s)
    return np.array(sel, dtype=np.int32), np.array(best)


def nll(D: np.ndarray, Yd: np.ndarray, d: float, g: float) -> float:
    """Negative log of eq. gpk via numpy.linalg.slogdet and solve."""
    import math

    n = D.shape[0]
    K = corr(D, D, d) + g * np.eye(n)
    sign, logdet = np.linalg.slogdet(K)
    assert sign > 0
    psi = Yd @ np.linalg.solve(K, Yd)
    return -math.lgamma(n / 2) + n / 2 * math.log(2 * math.pi) + 0.5 * logdet + n / 2 * math.log(psi / 2)


def nll_by_quadrature(D: np.ndarray, Yd: np.ndarray, d: float, g: float) -> float:
    """-log of the marginal of N(Y; 0, tau2 K) over tau2 with prior 1/tau2, by quadrature.

    Independent of eq. gpk's closed form: the Gamma function and the
    (psi/2)^(-n/2) factor come out of the integral numerically.
    """
    import math

    from scipy import integrate

    n = D.shape[0]
    K = corr(D, D, d) + g * np.eye(n)
    sign, logdet = np.linalg.slogdet(K)
    psi = Yd @ np.linalg.solve(K, Yd)

    # substitute u = log tau2; integrand of the log-scale marginal, scaled by exp(-c)
    def log_f(u):
        t = math.exp(u)
        return -n / 2 * math.log(2 * math.pi * t) - 0.5 * logdet - psi / (2 * t)

    umode = math.log(psi / n)
    c = log_f(umode)
    val, _ = integrate.quad(lambda u: math.exp(log_f(u) - c), umode - 40, umode + 40, limit=400,
                            epsabs=0, epsrel=1e-12)
    return -(c + math.log(val))


def mu_of(D: np.ndarray, Yd: np.ndarray, x: np.ndarray, d: float, g: float) -> float:
    """Predictive mean k^T K^{-1} Y (eq. predgp) via numpy.linalg.solve."""
    K = corr(D, D, d) + g * np.eye(D.shape[0])
    return corr(D, x[None, :], d)[:, 0] @ np.linalg.solve(K, Yd)


def mspe_criterion(D: np.ndarray, Yd: np.ndarray, x: np.ndarray, c: np.ndarray, d: float, g: float) -> float:
    """J(c, x) of eq. mspe by brute force: V_j(x | c) of eq. newv from a fresh
    solve on the design with c appended, d mu_j / dd by central differences of
    the mean in d, and G_{j+1} = (tr W^2 - tr(W)^2 / (j + 1)) / 2 with
    W = K_{j+1}^{-1} dK_{j+1}/dd from numpy.linalg.solve."""
    j = D.shape[0]
    K = corr(D, D, d) + g * np.eye(j)
    psi = Yd @ np.linalg.solve(K, Yd)
    D1 = np.vstack([D, c[None, :]])
    v1 = v_of(D1, x, d, g)
    h = 1e-4 * d
    dmu = (mu_of(D, Yd, x, d + h, g) - mu_of(D, Yd, x, d - h, g)) / (2 * h)
    R2 = np.zeros((j + 1, j + 1))
    for k in range(D1.shape[1]):
        t = D1[:, k][:, None] - D1[:, k][None, :]
        R2 = R2 + t * t
    K1 = np.exp(-R2 / d) + g * np.eye(j + 1)
    W = np.linalg.solve(K1, np.exp(-R2 / d) * R2 / d ** 2)
    G = 0.5 * (np.trace(W @ W) - np.trace(W) ** 2 / (j + 1))
    return (j + 1) * psi / (j * (j - 1)) * v1 + dmu * dmu / G


def greedy_mspe(X: np.ndarray, Y: np.ndarray, x: np.ndarray, P: np.ndarray, n0: int, n: int, d: float,
                g: float):
    """Designs minimising eq. mspe by brute force: returns (sel, criterion per step)."""
    sel = list(P[:n0])
    best = []
    for _ in range(n0, n):
        D, Yd = X[sel], Y[sel]
        scores = []
        for c in P:
            if c in sel:
                continue
            scores.append((mspe_criterion(D, Yd, x, X[c], d, g), c))
        s, c = min(scores)
        sel.append(c)
        best.append(s)
    return np.array(sel, dtype=np.int32), np.array(best)
