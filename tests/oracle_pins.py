"""Pins of the CPU oracle to facts fixed by the paper and by mathematics.

Each pin takes an ``oracle.Oracle`` and raises AssertionError on a mismatch.
They are run on the real oracle (test_oracle_pins.py) and on copies with a
planted mistake (test_oracle_mutants.py), which each must trip at least one.

What pins what:
  pool_exact        - NN pool = lexsort by (squared distance, index), with ties
  greedy_brute      - scores and sequence = brute force v_j - v_{j+1} (eq. dxy)
                      from fresh dense solves (Sec. 2.2, Fig. 1)
  hand_j1           - closed form of the score with a one-point design
  tie_rule          - exact score ties go to the smallest design index
  invariants        - score >= 0, v_j non-increasing, telescoping sum
  y_independence    - selected sequence independent of Y (Sec. 2.1: the
                      variance does not depend on Y); mean linear in Y
  scale_invariance  - X -> 2X, d -> 4d leaves every kernel value bit-identical
  special_cases     - n0 = n (NN GP), N' = n (whole pool), n0 = n = N' = N
                      (full GP) reduce to the textbook GP (eqs. predgp, preds2)
  design_point      - at a design point v = 2g - g^2 (K^{-1})_ii -> 0 with g
  predict_textbook  - local prediction = eqs. predgp/preds2 via numpy.solve
  route_b           - the paper's partitioned-inverse route (eq. piedef) and the
                      literal three-term eq. dxy agree with mode A; the
                      prediction from its K_n^{-1} (mean_b, s2_b, ...) agrees
                      with mode A and with numpy.solve where K_n is well
                      conditioned (the output route noise is then ~ eps)
  predict_b         - the fixed-design prediction through the partitioned
                      inverse = numpy.solve (eqs. predgp, preds2, piedef)
  psi_trajectory    - psi_j = Y_j^T K_j^{-1} Y_j at every step (the global
                      variance estimate of the normalised score, Sec. 3.1)
                      = numpy.solve on the step's design
  forced            - evaluating a given sequence reproduces the free run
  nll_textbook      - negative log of eq. gpk = slogdet/solve form, and = the
                      marginal over the scale computed by quadrature (pins
                      the Gamma-function and (psi/2)^(-n/2) constants)
  nll_derivatives_fd- d/dd, d/dg and d2/dd2 = central finite differences
  mle_optimality    - the Newton MLE is a stationary point (or a bound with
                      the gradient pointing out) and beats a fine local grid
  mle_global        - the Newton MLE equals the global minimiser of the NLL
                      over [1e-3, 5] found by a 2000-point log grid refined by
                      golden-section search (or, where the likelihood has
                      several local minima, is reported as a local one)
  local_mle_batched - the batched MLE over many designs = the single-design
                      MLE of each gathered design
  scores_brute      - batch scores of many candidates against one design (both
                      routes) = brute force v_j - v_{j+1}; K_j^{-1} K_j = I and
                      h = K(X_j, x) from numpy; the one-point closed form
  scores_greedy     - the batch scores at a step of a greedy run reproduce that
                      step's best score and argmax
  mspe_brute        - designs by the MSPE criterion (eq. mspe) = brute force with
                      fresh solves, central differences of the mean in d and
                      numpy traces for the expected information
  mspe_parts        - the criterion splits into eq. newv's variance term, whose
                      v_j and psi_j the ALC route gives independently, plus
                      (d mu / dd)^2 / G; the partitioned-inverse route agrees
  separable_brute   - the separable kernel (one lengthscale per input, the
                      vectorised lengthscale of Sec. 3.1) = brute force with
                      fresh solves on that kernel; its prediction = numpy.solve
  separable_reduces - equal lengthscales give the isotropic designs; doubling
                      one input while quadrupling its lengthscale is exact
                      (bit-identical); an input with an enormous lengthscale
                      drops out (bit-identical to the run without it)
  per_location_d    - a lengthscale of each location's own (the second design
                      stage of Fig. 1 step 4) gives, location by location,
                      the run with that scalar lengthscale; invalid entries
                      fail only their own location
"""
from __future__ import annotations

import math

import numpy as np

import brute
import workloads


def _rel(a, b):
    a, b = np.asarray(a, float), np.asarray(b, float)
    return np.max(np.abs(a - b) / np.maximum(np.abs(b), 1e-300))


def pool_exact(orc):
    r = np.random.default_rng(7)
    base = r.random((150, 3))
    lattice = np.array([[i / 4, j / 4, k / 4] for i in range(5) for j in range(5) for k in range(3)])
    X = np.vstack([base, base[:40], lattice, base[10:20]])  # duplicates -> exact distance ties
    XX = np.vstack([r.random((6, 3)), lattice[[3, 17, 40]], base[[5, 11]]])
    for Np in (1, 37, 90, X.shape[0]):
        P = orc.nn_pool(X, XX, Np)
        for m in range(XX.shape[0]):
            want = brute.pool(X, XX[m], Np)
            assert np.array_equal(P[m], want), (Np, m)


def greedy_brute(orc):
    X, Y, XX = workloads.uniform(3, 70, 2, 4)
    d, g, n0, n, Np = 0.15, 1e-3, 3, 11, 30
    out = orc.lagp(X, Y, XX, n0, n, Np, d, g)
    assert np.all(out["status"] == 0)
    for m in range(XX.shape[0]):
        P = brute.pool(X, XX[m], Np)
        sel, best = brute.greedy(X, XX[m], P, n0, n, d, g)
        assert np.array_equal(out["sel"][m], sel), m
        assert _rel(out["dsel"][m, n0:], best) < 1e-8, m


def hand_j1(orc):
    X, Y, XX = workloads.uniform(4, 50, 2, 3)
    d, g, Np = 0.2, 1e-2, 20
    out = orc.lagp(X, Y, XX, 1, 2, Np, d, g)
    kappa = 1.0 + g

    def K(a, b):
        return math.exp(-sum((a[k] - b[k]) ** 2 for k in range(len(a))) / d)

    for m in range(XX.shape[0]):
        P = brute.pool(X, XX[m], Np)
        a = X[P[0]]
        x = XX[m]
        best, arg = -1.0, -1
        for c in P[1:]:
            s = kappa - K(X[c], a) ** 2 / kappa
            cov = K(X[c], x) - K(X[c], a) * K(a, x) / kappa
            sc = cov * cov / s
            if sc > best or (sc == best and c < arg):
                best, arg = sc, c
        assert out["amax"][m, 1] == arg
        assert abs(out["dmax"][m, 1] - best) <= 1e-12 * best


def tie_rule(orc):
    r = np.random.default_rng(11)
    A = r.random((60, 2))
    X = np.vstack([A, A])  # every point twice: rows i and i + 60
    Y = np.sin(4 * X[:, 0]) + X[:, 1]
    XX = r.random((3, 2))
    n0, n, Np = 2, 9, 40
    out = orc.lagp(X, Y, XX, n0, n, Np, 0.2, 1e-3)
    for m in range(XX.shape[0]):
        P = out["pool"][m]
        # twins are adjacent in the pool, smaller index first
        for s in range(0, Np - 1, 2):
            assert P[s] + 60 == P[s + 1] or P[s] == P[s + 1] - 60
        # twins score exactly alike while both are candidates (identical
        # coordinates give bit-identical kernel values), so the larger twin can
        # only be picked once the smaller one is in the design
        sel = list(out["sel"][m])
        for j in range(n0, n):
            if sel[j] >= 60:
                assert sel[j] - 60 in sel[:j], (m, j, sel)
        assert out["sel"][m, n0] < 60


def invariants(orc):
    W = workloads.make(2, N=3000, M=6)
    out = orc.lagp(W.X, W.Y, W.XX, W.n0, 30, 300, W.d, W.g)
    assert np.all(out["status"] == 0)
    ds = out["dsel"][:, W.n0:]
    assert np.all(ds >= 0)
    v = out["vtraj"][:, W.n0:]
    assert np.all(np.diff(v, axis=1) <= 1e-14 * v[:, :-1])
    tele = out["vtraj"][:, W.n0] - ds.sum(axis=1)
    assert _rel(out["vtraj"][:, 30], tele) < 1e-9


def y_independence(orc):
    W = workloads.make(2, N=2000, M=5)
    a = orc.lagp(W.X, W.Y, W.XX, 6, 20, 200, W.d, W.g)
    noise = np.random.default_rng(5).normal(size=W.N)
    b = orc.lagp(W.X, 3.0 * W.Y + noise, W.XX, 6, 20, 200, W.d, W.g)
    assert np.array_equal(a["sel"], b["sel"])
    c = orc.lagp(W.X, -2.5 * W.Y, W.XX, 6, 20, 200, W.d, W.g)
    assert _rel(c["mean"], -2.5 * a["mean"]) < 1e-12
    assert _rel(c["s2"], 6.25 * a["s2"]) < 1e-12


def scale_invariance(orc):
    W = workloads.make(1, N=1500, M=5)
    a = orc.lagp(W.X, W.Y, W.XX, 6, 16, 150, W.d, 1e-4)
    b = orc.lagp(2 * W.X, W.Y, 2 * W.XX, 6, 16, 150, 4 * W.d, 1e-4)
    for k in ("pool", "sel", "mean", "s2", "var"):
        assert np.array_equal(a[k], b[k]), k


def special_cases(orc):
    W = workloads.make(4, N=800, M=4)
    d, g = W.d, W.g
    n = 12
    # n0 = n: the NN GP on the first n pool points
    a = orc.lagp(W.X, W.Y, W.XX, n, n, 40, d, g)
    for m in range(W.M):
        P = brute.pool(W.X, W.XX[m], n)
        ref = brute.predict(W.X[P], W.Y[P], W.XX[m], d, g)
        assert np.array_equal(a["sel"][m], P)
        for k in ("mean", "s2", "var"):
            assert _rel(a[k][m], ref[k]) < 1e-9, k
    # N' = n: the final design is the whole pool
    b = orc.lagp(W.X, W.Y, W.XX, 4, n, n, d, g)
    for m in range(W.M):
        P = brute.pool(W.X, W.XX[m], n)
        assert sorted(b["sel"][m]) == sorted(P)
        ref = brute.predict(W.X[P], W.Y[P], W.XX[m], d, g)
        for k in ("mean", "s2"):
            assert _rel(b[k][m], ref[k]) < 1e-9, k
    # n0 = n = N' = N: the full GP
    Xs, Ys = W.X[:25], W.Y[:25]
    c = orc.lagp(Xs, Ys, W.XX, 25, 25, 25, d, g)
    for m in range(W.M):
        ref = brute.predict(Xs, Ys, W.XX[m], d, g)
        for k in ("mean", "s2", "var"):
            assert _rel(c[k][m], ref[k]) < 1e-9, k


def design_point(orc):
    X, Y, _ = workloads.uniform(6, 400, 2, 1)
    XX = X[[17, 123, 250]]
    vs = []
    for g in (1e-2, 1e-4, 1e-6):
        out = orc.lagp(X, Y, XX, 6, 14, 60, 0.5, g)
        for m, i in enumerate((17, 123, 250)):
            sel = out["sel"][m]
            assert sel[0] == i  # distance 0 comes first in the pool
            D = X[sel]
            K = brute.corr(D, D, 0.5) + g * np.eye(len(sel))
            Kinv = np.linalg.inv(K)
            want = 2 * g - g * g * Kinv[0, 0]
            assert abs(out["v"][m] - want) <= 1e-6 * want + 1e-15, (g, m)
            vs.append(out["v"][m] / g)
    assert max(vs) <= 2.0 + 1e-6


def predict_textbook(orc):
    r = np.random.default_rng(9)
    for n, p, d, g in ((5, 1, 0.3, 1e-3), (17, 3, 0.7, 1e-4), (40, 4, 0.25, 1e-5)):
        D = r.random((n, p))
        Yd = np.cos(3 * D).sum(axis=1) + r.normal(0, 0.1, n)
        x = r.random(p)
        got = orc.gp_predict(D, Yd, x, d, g)
        ref = brute.predict(D, Yd, x, d, g)
        for k in ("mean", "s2", "v", "psi"):
            assert _rel(got[k], ref[k]) < 1e-8, (n, k)
        assert _rel(got["var"], got["s2"] * n / (n - 2)) < 1e-15


def route_b(orc):
    W = workloads.make(2, N=5000, M=4)
    out = orc.lagp(W.X, W.Y, W.XX, 6, 30, 300, W.d, W.g, mode_b=True)
    nu = out["nu"][:, 6:]
    assert np.all(np.isfinite(nu))
    assert np.max(nu) < 1e-9, np.max(nu)
    # the prediction through the partitioned-inverse K_n^{-1}: equal to mode A
    # and to numpy.solve at this conditioning (cond(K_n) ~ 1e3)
    for m in range(W.M):
        ref = brute.predict(W.X[out["sel"][m]], W.Y[out["sel"][m]], W.XX[m], W.d, W.g)
        for k in ("mean", "s2", "var", "v", "psi"):
            assert _rel(out[k + "_b"][m], out[k][m]) < 1e-10, (m, k)
            assert _rel(out[k + "_b"][m], ref[k]) < 1e-9, (m, k)
    plain = orc.lagp(W.X, W.Y, W.XX, 6, 30, 300, W.d, W.g)
    assert "mean_b" not in plain


def predict_b(orc):
    r = np.random.default_rng(19)
    for n, p, d, g in ((1, 2, 0.3, 1e-2), (5, 1, 0.3, 1e-3), (17, 3, 0.7, 1e-4), (40, 4, 0.25, 1e-5)):
        D = r.random((n, p))
        Yd = np.cos(3 * D).sum(axis=1) + r.normal(0, 0.1, n)
        x = r.random(p)
        got = orc.gp_predict_b(D, Yd, x, d, g)
        ref = brute.predict(D, Yd, x, d, g)
        assert got["status"] == 0
        for k in ("mean", "s2", "v", "psi"):
            assert _rel(got[k], ref[k]) < 1e-7, (n, k)
        if n > 2:
            assert _rel(got["var"], ref["var"]) < 1e-7


def psi_trajectory(orc):
    W = workloads.make(2, N=3000, M=3)
    n0, n = 6, 20
    out = orc.lagp(W.X, W.Y, W.XX, n0, n, 200, W.d, W.g)
    for m in range(W.M):
        assert out["psitraj"][m, 0] == 0.0
        for j in (1, n0, 13, n - 1):
            D, Yd = W.X[out["sel"][m, :j]], W.Y[out["sel"][m, :j]]
            K = brute.corr(D, D, W.d) + W.g * np.eye(j)
            want = Yd @ np.linalg.solve(K, Yd)
            assert _rel(out["psitraj"][m, j], want) < 1e-9, (m, j)
        # psi of the last step's design grows by one term into the prediction's psi
        assert out["psi"][m] >= out["psitraj"][m, n - 1]


def forced(orc):
    W = workloads.make(2, N=3000, M=4)
    a = orc.lagp(W.X, W.Y, W.XX, 6, 20, 200, W.d, W.g)
    b = orc.alc(W.X, W.Y, W.XX, a["pool"], 6, 20, W.d, W.g, forced=a["sel"])
    for k in ("sel", "dsel", "dmax", "amax", "mean", "s2"):
        assert np.array_equal(a[k], b[k], equal_nan=True), k
    nn = np.ascontiguousarray(a["pool"][:, :20])
    c = orc.alc(W.X, W.Y, W.XX, a["pool"], 6, 20, W.d, W.g, forced=nn)
    assert np.all(c["dsel"][:, 6:] <= c["dmax"][:, 6:])
    for m in range(W.M):
        ref = brute.predict(W.X[nn[m]], W.Y[nn[m]], W.XX[m], W.d, W.g)
        assert _rel(c["mean"][m], ref["mean"]) < 1e-9


def nll_textbook(orc):
    r = np.random.default_rng(21)
    for n, p, d, g in ((4, 2, 0.4, 1e-2), (9, 3, 0.25, 1e-3), (30, 4, 0.2, 1e-3), (50, 4, 0.6, 1e-4)):
        D = r.random((n, p))
        Yd = np.sin(3 * D).sum(axis=1) + r.normal(0, 0.05, n)
        got = orc.nll(D, Yd, d, g)
        assert got["status"] == 0
        assert abs(got["nll"] - brute.nll(D, Yd, d, g)) <= 1e-9 * max(1.0, abs(got["nll"])), (n, got)
        if n <= 9:
            q = brute.nll_by_quadrature(D, Yd, d, g)
            assert abs(got["nll"] - q) <= 1e-8 * max(1.0, abs(q)), (n, got["nll"], q)


def nll_derivatives_fd(orc):
    r = np.random.default_rng(22)
    for n, p, d, g in ((6, 2, 0.3, 1e-2), (25, 4, 0.2, 1e-3), (50, 4, 0.7, 1e-3)):
        D = r.random((n, p))
        Yd = np.cos(4 * D).sum(axis=1) + r.normal(0, 0.03, n)
        f = orc.nll(D, Yd, d, g)
        hd, hg = 1e-5 * d, 1e-5 * g
        fdd = (orc.nll(D, Yd, d + hd, g)["nll"] - orc.nll(D, Yd, d - hd, g)["nll"]) / (2 * hd)
        fdg = (orc.nll(D, Yd, d, g + hg)["nll"] - orc.nll(D, Yd, d, g - hg)["nll"]) / (2 * hg)
        fd2 = (orc.nll(D, Yd, d + hd, g)["dd"] - orc.nll(D, Yd, d - hd, g)["dd"]) / (2 * hd)
        assert abs(fdd - f["dd"]) <= 1e-6 * max(1.0, abs(f["dd"])), (n, fdd, f["dd"])
        assert abs(fdg - f["dg"]) <= 1e-6 * max(1.0, abs(f["dg"])), (n, fdg, f["dg"])
        assert abs(fd2 - f["d2"]) <= 1e-5 * max(1.0, abs(f["d2"])), (n, fd2, f["d2"])


def mle_optimality(orc):
    W = workloads.make(4, N=4000, M=6)
    out = orc.lagp(W.X, W.Y, W.XX, 6, 30, 300, 0.2, W.g)
    dmin, dmax = 1e-3, 5.0
    for m in range(W.M):
        D, Yd = W.X[out["sel"][m]], W.Y[out["sel"][m]]
        res = orc.mle_d(D, Yd, 0.2, W.g, dmin, dmax)
        assert res["status"] == 0, res
        dh = res["d"]
        f = orc.nll(D, Yd, dh, W.g)
        if dmin < dh < dmax:
            assert abs(f["dd"]) <= 1e-6 * max(1.0, abs(f["nll"])) and f["d2"] > 0, (m, f)
        else:
            assert (dh == dmin and f["dd"] > 0) or (dh == dmax and f["dd"] < 0)
        # no point of a fine grid around the optimum does better
        for t in np.geomspace(max(dmin, dh / 1.5), min(dmax, dh * 1.5), 61):
            assert orc.nll(D, Yd, t, W.g)["nll"] >= f["nll"] - 1e-9 * abs(f["nll"])


def _golden(f, a, b, tol=1e-13):
    """Golden-section minimum of a unimodal f on [a, b] (log-d coordinates)."""
    phi = (math.sqrt(5.0) - 1.0) / 2.0
    c, e = b - phi * (b - a), a + phi * (b - a)
    fc, fe = f(c), f(e)
    while b - a > tol * max(1.0, abs(a) + abs(b)):
        if fc <= fe:
            b, e, fe = e, c, fc
            c = b - phi * (b - a)
            fc = f(c)
        else:
            a, c, fc = c, e, fe
            e = a + phi * (b - a)
            fe = f(e)
    return (a + b) / 2.0


def mle_global(orc):
    W = workloads.make(4, N=4000, M=6)
    out = orc.lagp(W.X, W.Y, W.XX, 6, 30, 300, 0.2, W.g)
    dmin, dmax = 1e-3, 5.0
    grid = np.geomspace(dmin, dmax, 2000)
    local = 0
    for m in range(W.M):
        D, Yd = W.X[out["sel"][m]], W.Y[out["sel"][m]]
        res = orc.mle_d(D, Yd, 0.2, W.g, dmin, dmax)
        assert res["status"] == 0, res
        f = np.array([brute.nll(D, Yd, t, W.g) for t in grid])
        i = int(np.argmin(f))
        if i == 0 or i == len(grid) - 1:
            d_glob = grid[i]
        else:
            u = _golden(lambda lu: brute.nll(D, Yd, math.exp(lu), W.g), math.log(grid[i - 1]),
                        math.log(grid[i + 1]))
            d_glob = math.exp(u)
        f_glob = brute.nll(D, Yd, d_glob, W.g)
        f_newton = brute.nll(D, Yd, res["d"], W.g)
        if f_newton <= f_glob + 1e-10 * max(1.0, abs(f_glob)):
            # the Newton optimum is the global one; interior optima agree in d
            if dmin < d_glob < dmax:
                assert abs(res["d"] - d_glob) <= 1e-6 * d_glob, (m, res["d"], d_glob)
            else:
                assert res["d"] == d_glob, (m, res["d"], d_glob)
        else:
            # a local minimum: it must still be one (a grid neighbourhood cannot improve it)
            local += 1
            for t in np.geomspace(res["d"] / 1.01, res["d"] * 1.01, 21):
                if dmin <= t <= dmax:
                    assert brute.nll(D, Yd, t, W.g) >= f_newton - 1e-10 * abs(f_newton)
    # the greedy designs of this workload have a single minimum in d
    assert local == 0, local


def local_mle_batched(orc):
    W = workloads.make(4, N=3000, M=5)
    out = orc.lagp(W.X, W.Y, W.XX, 6, 20, 200, 0.2, W.g)
    d0 = np.array([0.2, 0.05, 1.0, 3.0, 0.2])
    b = orc.local_mle(W.X, W.Y, out["sel"], d0, W.g, 1e-3, 5.0, 100, threads=2)
    for m in range(W.M):
        s = out["sel"][m]
        one = orc.mle_d(W.X[s], W.Y[s], float(d0[m]), W.g, 1e-3, 5.0, 100)
        for k in ("d", "nll", "iters", "status"):
            assert one[k] == b[k][m], (m, k, one[k], b[k][m])


def scores_brute(orc):
    r = np.random.default_rng(21)
    d, g = 0.3, 1e-3
    for j, p in ((1, 2), (3, 2), (7, 3), (12, 1)):
        Xj, Xc, x = r.random((j, p)), r.random((15, p)), r.random(p)
        a = orc.alc_scores(Xj, Xc, x, d, g)
        b = orc.alc_scores(Xj, Xc, x, d, g, mode_b=True)
        want = np.array([brute.delta(Xj, c, x, d, g) for c in Xc])
        assert np.all(want >= 0.0)
        # the brute force differences two variances: errors scale with the largest score
        scale = np.max(want)
        assert np.max(np.abs(a["delta"] - want)) <= 1e-9 * scale, (j, p)
        # the three terms of eq. dxy cancel: route noise grows with cond(K_j)
        assert np.max(np.abs(b["delta"] - want)) <= 1e-7 * scale, (j, p)
        K = brute.corr(Xj, Xj, d) + g * np.eye(j)
        assert np.max(np.abs(a["Kinv"] @ K - np.eye(j))) < 1e-9
        assert _rel(a["h"], brute.corr(Xj, x[None, :], d)[:, 0]) < 1e-15
        if j == 1:  # closed form with a one-point design
            kap = 1.0 + g
            kc = brute.corr(Xc, Xj, d)[:, 0]
            kx = brute.corr(Xc, x[None, :], d)[:, 0]
            hh = a["h"][0]
            cf = (kx - kc * hh / kap) ** 2 / (kap - kc * kc / kap)
            assert _rel(a["delta"], cf) < 1e-12


def scores_greedy(orc):
    W = workloads.make(2, N=3000, M=3)
    n0, n, Np = 6, 18, 120
    out = orc.lagp(W.X, W.Y, W.XX, n0, n, Np, W.d, W.g)
    for m in range(W.M):
        for j in (n0, 11, n - 1):
            design = out["sel"][m, :j]
            cand = np.setdiff1d(out["pool"][m], design)
            sc = orc.alc_scores(W.X[design], W.X[cand], W.XX[m], W.d, W.g)["delta"]
            best = np.max(sc)
            arg = int(np.min(cand[sc == best]))
            assert abs(best - out["dmax"][m, j]) <= 1e-12 * best, (m, j)
            assert arg == out["amax"][m, j], (m, j)


def per_location_d(orc):
    W = workloads.make(4, N=3000, M=5)
    n0, n, Np = 6, 16, 90
    pool = orc.nn_pool(W.X, W.XX, Np)
    dp = np.array([0.05, 0.2, 0.7, 2.0, 0.2])
    a = orc.alc(W.X, W.Y, W.XX, pool, n0, n, W.d, W.g, d_per=dp)
    for m in range(W.M):
        b = orc.alc(W.X, W.Y, W.XX[m:m + 1], pool[m:m + 1], n0, n, float(dp[m]), W.g)
        for k in ("sel", "dsel", "mean", "s2", "var", "status"):
            assert np.array_equal(a[k][m], b[k][0], equal_nan=True), (m, k)
    c = orc.alc(W.X, W.Y, W.XX, pool, n0, n, W.d, W.g, d_per=np.full(W.M, W.d))
    e = orc.alc(W.X, W.Y, W.XX, pool, n0, n, W.d, W.g)
    for k in ("sel", "dsel", "mean", "s2", "var"):
        assert np.array_equal(c[k], e[k], equal_nan=True), k
    bad = dp.copy()
    bad[1], bad[3] = 0.0, np.nan
    f = orc.alc(W.X, W.Y, W.XX, pool, n0, n, W.d, W.g, d_per=bad)
    assert list(f["status"] != 0) == [False, True, False, True, False]
    assert np.array_equal(f["sel"][[0, 2, 4]], a["sel"][[0, 2, 4]])


def mspe_brute(orc):
    X, Y, XX = workloads.uniform(8, 70, 2, 3)
    d, g, n0, n, Np = 0.15, 1e-3, 3, 9, 25
    pool = orc.nn_pool(X, XX, Np)
    out = orc.mspe(X, Y, XX, pool, n0, n, d, g)
    assert np.all(out["status"] == 0)
    for m in range(XX.shape[0]):
        sel, best = brute.greedy_mspe(X, Y, XX[m], pool[m], n0, n, d, g)
        assert np.array_equal(out["sel"][m], sel), (m, out["sel"][m], sel)
        assert _rel(out["jsel"][m, n0:], best) < 1e-7, m
        # d mu / dd against central differences of the mean
        for j in (n0, n - 1):
            D, Yd = X[out["sel"][m, :j]], Y[out["sel"][m, :j]]
            h = 1e-4 * d
            fd = (brute.mu_of(D, Yd, XX[m], d + h, g) - brute.mu_of(D, Yd, XX[m], d - h, g)) / (2 * h)
            assert abs(out["dmu"][m, j] - fd) <= 1e-7 * max(1e-3, abs(fd)), (m, j)


def mspe_parts(orc):
    W = workloads.make(4, N=3000, M=4)
    n0, n, Np = 6, 18, 120
    pool = orc.nn_pool(W.X, W.XX, Np)
    out = orc.mspe(W.X, W.Y, W.XX, pool, n0, n, 0.2, W.g, mode_b=True)
    assert np.all(out["status"] == 0)
    assert np.nanmax(out["nu"]) < 1e-8, np.nanmax(out["nu"])
    # along the MSPE sequence, the ALC route's v_j, score and psi_j rebuild the
    # variance term: J - dmu^2 / G = (j + 1) psi_j / (j (j - 1)) (v_j - Delta)
    a = orc.alc(W.X, W.Y, W.XX, pool, n0, n, 0.2, W.g, forced=out["sel"])
    for m in range(W.M):
        for j in range(n0, n):
            var_term = (j + 1) * a["psitraj"][m, j] / (j * (j - 1)) * (a["vtraj"][m, j] - a["dsel"][m, j])
            got = out["jsel"][m, j] - out["dmu"][m, j] ** 2 / out["gsel"][m, j]
            assert abs(got - var_term) <= 1e-9 * abs(out["jsel"][m, j]), (m, j)
    # every choice is the minimiser it reports
    assert np.array_equal(out["sel"][:, n0:], out["amin"][:, n0:])
    assert np.all(out["gsel"][:, n0:] > 0)


def separable_brute(orc):
    X, Y, XX = workloads.uniform(9, 90, 3, 3)
    dsep = np.array([0.05, 0.3, 1.5])
    g, n0, n, Np = 1e-3, 3, 10, 30
    pool = orc.nn_pool(X, XX, Np)
    out = orc.alc(X, Y, XX, pool, n0, n, 0.5, g, dsep=dsep)
    assert np.all(out["status"] == 0)
    for m in range(XX.shape[0]):
        sel, best = brute.greedy(X, XX[m], pool[m], n0, n, dsep, g)
        assert np.array_equal(out["sel"][m], sel), (m, out["sel"][m], sel)
        assert _rel(out["dsel"][m, n0:], best) < 1e-9, m
        ref = brute.predict(X[sel], Y[sel], XX[m], dsep, g)
        for k in ("mean", "s2", "var"):
            assert _rel(out[k][m], ref[k]) < 1e-9, (m, k)
        fixed = orc.gp_predict_sep(X[sel], Y[sel], XX[m], dsep, g)
        assert _rel(fixed["s2"], ref["s2"]) < 1e-9 and _rel(fixed["mean"], ref["mean"]) < 1e-9


def separable_reduces(orc):
    W = workloads.make(4, N=3000, M=6)
    n0, n, Np = 6, 18, 120
    pool = orc.nn_pool(W.X, W.XX, Np)
    iso = orc.alc(W.X, W.Y, W.XX, pool, n0, n, W.d, W.g)
    eq = orc.alc(W.X, W.Y, W.XX, pool, n0, n, 123.0, W.g, dsep=np.full(W.p, W.d))
    assert np.array_equal(iso["sel"], eq["sel"])
    for k in ("mean", "s2", "var"):
        assert _rel(iso[k], eq[k]) < 1e-12, k
    # input 2 doubled with its lengthscale quadrupled: every kernel value bit-identical
    dsep = np.array([0.1, 0.25, 0.4, 0.9])
    a = orc.alc(W.X, W.Y, W.XX, pool, n0, n, 1.0, W.g, dsep=dsep)
    X2, XX2, d2 = W.X.copy(), W.XX.copy(), dsep.copy()
    X2[:, 2] *= 2.0
    XX2[:, 2] *= 2.0
    d2[2] *= 4.0
    b = orc.alc(X2, W.Y, XX2, pool, n0, n, 1.0, W.g, dsep=d2)
    for k in ("sel", "dsel", "mean", "s2", "var"):
        assert np.array_equal(a[k], b[k], equal_nan=True), k
    # input 3 with an enormous lengthscale contributes exp(-t^2 / 1e300) = 1 exactly
    big = dsep.copy()
    big[3] = 1e300
    c = orc.alc(W.X, W.Y, W.XX, pool, n0, n, 1.0, W.g, dsep=big)
    e = orc.alc(np.ascontiguousarray(W.X[:, :3]), W.Y, np.ascontiguousarray(W.XX[:, :3]), pool, n0, n, 1.0,
                W.g, dsep=dsep[:3])
    for k in ("sel", "dsel", "mean", "s2", "var"):
        assert np.array_equal(c[k], e[k], equal_nan=True), k
    assert not np.array_equal(a["sel"], c["sel"])  # the input mattered before it was dropped


ALL = [pool_exact, greedy_brute, hand_j1, tie_rule, invariants, y_independence, scale_invariance,
       special_cases, design_point, predict_textbook, route_b, predict_b, psi_trajectory, forced,
       nll_textbook, nll_derivatives_fd, mle_optimality, mle_global, local_mle_batched, scores_brute,
       scores_greedy, mspe_brute, mspe_parts, separable_brute, separable_reduces, per_location_d]
