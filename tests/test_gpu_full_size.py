"""Full-size workloads in the launch configuration the bench times, checked on
sampled locations that the oracle recomputes one by one (pool, design,
prediction), plus properties that hold at any size."""
from __future__ import annotations

import json
import os

import numpy as np
import pytest

import parity
import workloads

pytestmark = [pytest.mark.gpu, pytest.mark.slow]

OUT = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "gpurun_out")
SAMPLE = 12


def _log(name, rec):
    print(f"[full] {name}: {json.dumps(rec)}", flush=True)
    os.makedirs(OUT, exist_ok=True)
    with open(os.path.join(OUT, "parity_log.jsonl"), "a") as f:
        f.write(json.dumps(dict(test=name, **rec)) + "\n")


@pytest.fixture(scope="module")
def lagp():
    import torch

    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    import paper_1310_5182_amd as lagp

    return lagp


def dev(a):
    import torch

    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def sampled_check(orc, W, g, rows, n_of, Np_of, name, tau_out=1e-10):
    """Recompute sampled locations with the oracle and apply the parity protocol."""
    X, Y = W.X, W.Y
    pool_ref = orc.nn_pool(X, W.XX[rows], int(max(Np_of(m) for m in rows)))
    ties, worst = 0, 0.0
    errs = dict(mean=0.0, s2=0.0, var=0.0)
    gaps = dict(mean=0.0, s2=0.0, var=0.0)
    for i, m in enumerate(rows):
        n, Np = n_of(m), Np_of(m)
        assert np.array_equal(g["pool"][m, :Np], pool_ref[i, :Np]), m
        sel = g["sel"][m, :n][None, :]
        f = orc.alc(X, Y, W.XX[m:m + 1], g["pool"][m:m + 1, :Np], W.n0, n, W.d, W.g, forced=sel, mode_b=True)
        seq = parity.sequence_check(sel, g["pool"][m:m + 1, :Np], f, W.n0)
        assert not seq["fails"], (m, seq["fails"])
        ties += seq["ties"]
        floor = 1e-6 * np.sqrt(np.mean(Y ** 2))
        for k in ("mean", "s2", "var"):
            b = f[k][0]
            fl = floor if k == "mean" else 0.0
            rel = abs(g[k][m] - b) / max(abs(b), fl)
            tol = float(parity.output_tolerance(f, k, tau_out, fl)[0])
            gaps[k] = max(gaps[k], float(parity.route_gap(f, k, fl)[0]))
            errs[k] = max(errs[k], rel)
            worst = max(worst, rel / tol)
    _log(name, dict(M=W.M, N=W.N, sampled=len(rows), ties=ties, worst_over_tol=worst, tau_out=tau_out,
                    max_rel=errs, max_route_gap=gaps))
    assert worst <= 1.0


def global_properties(g, n_of, M):
    st = g["status"]
    assert np.all(st == 0), np.unique(st, return_counts=True)
    for k in ("mean", "s2", "var"):
        assert np.all(np.isfinite(g[k])), k
    assert np.all(g["s2"] > 0) and np.all(g["var"] > g["s2"])
    # every design: the first n0 pool entries, then distinct pool members
    for m in range(0, M, max(1, M // 2000)):
        n = n_of(m)
        row = g["sel"][m, :n]
        assert len(np.unique(row)) == n
        assert np.array_equal(row[:6], g["pool"][m, :6])


@pytest.mark.parametrize("cfg,precision", [(2, "fp64"), (2, "mixed"), (5, "fp64"), (5, "mixed")])
def test_uniform_full_size(lagp, orc, cfg, precision):
    import torch

    W = workloads.make(cfg)
    print(f"[full] config{cfg} {precision} N={W.N} M={W.M}", flush=True)
    X, Y, XX = dev(W.X), dev(W.Y), dev(W.XX)
    if cfg == 5:
        # as timed: one tuned, graph-captured plan (launched again after creation)
        plan = lagp.Plan(X, Y, XX, W.n0, W.n, W.Np, W.d, W.g, precision=precision)
        print(f"[full] plan: {plan.describe()}", flush=True)
        o = plan.launch()
    else:
        o = lagp.alc_predict(X, Y, XX, W.n0, W.n, W.Np, W.d, W.g, precision)
    torch.cuda.synchronize()
    g = {k: v.cpu().numpy() for k, v in o.items() if k != "workspace"}
    del o
    if cfg == 5:
        plan.close()
        del plan
    global_properties(g, lambda m: W.n, W.M)
    steps = W.M * (W.n - W.n0)
    if precision == "mixed":
        # the precision split's report: float32 score of each chosen point
        # against its float64 score, and the fraction of steps redone in float64
        a32, a64 = g["alc32"][:, W.n0:], g["alc"][:, W.n0:]
        fin = np.isfinite(a32)
        e32 = np.abs(a32[fin] - a64[fin]) / a64[fin]
        _log(f"full_config{cfg}_mixed_report",
             dict(fallback_steps_frac=float(g["guard"].sum()) / steps, alc32_max_rel=float(e32.max()),
                  alc32_median_rel=float(np.median(e32)), float32_decided_frac=float(fin.mean())))
    else:
        assert np.all(g["guard"] == 0)
    rows = np.random.default_rng(cfg).choice(W.M, SAMPLE, replace=False)
    sampled_check(orc, W, g, rows, lambda m: W.n, lambda m: W.Np, f"full_config{cfg}_{precision}",
                  tau_out=1e-4 if precision == "mixed" else 1e-10)


def test_uneven_full_size(lagp, orc):
    import torch

    W = workloads.make(3)
    print(f"[full] config3 N={W.N} M={W.M}", flush=True)
    X, Y, XX = dev(W.X), dev(W.Y), dev(W.XX)
    # as timed: one tuned, graph-captured plan (launched again after creation)
    plan = lagp.Plan(X, Y, XX, W.n0, 100, 2000, W.d, W.g, n_per=dev(W.n_per), Np_per=dev(W.Np_per))
    print(f"[full] plan: {plan.describe()}", flush=True)
    o = plan.launch()
    torch.cuda.synchronize()
    g = {k: v.cpu().numpy() for k, v in o.items() if k != "workspace"}
    del o
    n_of = lambda m: int(W.n_per[m])  # noqa: E731
    Np_of = lambda m: int(W.Np_per[m])  # noqa: E731
    global_properties(g, n_of, W.M)
    for m in range(0, W.M, 997):
        assert np.all(g["sel"][m, n_of(m):] == -1)
    # the sample covers the extremes of the cost distribution
    cost = W.Np_per.astype(float) * W.n_per.astype(float) ** 2
    order = np.argsort(cost)
    rows = np.concatenate([order[:3], order[-5:], np.random.default_rng(3).choice(W.M, SAMPLE - 8, replace=False)])
    sampled_check(orc, W, g, rows, n_of, Np_of, "full_config3")
