"""The one-call entry point (lagp_alc_predict with lagp_problem / lagp_outputs)
on the GPU: the normalised scores of Fig. 3 step 9, per-location sizes in mixed
precision, row offsets, both NN variants and mixed-precision plans, against the
CPU oracle and against the other entry points."""
from __future__ import annotations

import json
import os

import numpy as np
import pytest

import parity
import workloads

pytestmark = pytest.mark.gpu

OUT = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "gpurun_out")


def _log(name, rec):
    print(f"[boundary] {name}: {json.dumps(rec)}", flush=True)
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


def host(o):
    return {k: v.cpu().numpy() for k, v in o.items() if k != "workspace"}


def run(lagp, W, precision, n_max=None, Np_max=None, n_per=None, Np_per=None, **kw):
    import torch

    o = lagp.alc_predict(dev(W.X), dev(W.Y), dev(W.XX), W.n0, n_max or W.n, Np_max or W.Np, W.d, W.g, precision,
                         n_per=None if n_per is None else dev(n_per),
                         Np_per=None if Np_per is None else dev(Np_per), **kw)
    torch.cuda.synchronize()
    return host(o)


@pytest.mark.parametrize("precision,per_location", [("fp64", False), ("mixed", False), ("fp64_reform", False),
                                                    ("fp64", True), ("mixed", True)])
def test_normalized_scores(lagp, orc, precision, per_location):
    """LAGP_NORMALIZE_ALC (Sec. 3.1, Fig. 3 step 9): the reported score of each
    added point is psi_j Delta / (j - 2); the choices do not change."""
    if per_location:
        W = workloads.make(3, N=30000, M=24)
        W.n_per = np.minimum(W.n_per, 60).astype(np.int32)
        W.Np_per = np.minimum(np.maximum(W.Np_per, W.n_per), 1000).astype(np.int32)
        n_max, Np_max, n_per, Np_per = 60, 1000, W.n_per, W.Np_per
    else:
        W = workloads.make(2, N=20000, M=24)
        W.n, W.Np = 30, 400
        n_max, Np_max, n_per, Np_per = 30, 400, None, None
    print(f"[boundary] normalize {precision} per_location={per_location}", flush=True)
    a = run(lagp, W, precision, n_max, Np_max, n_per, Np_per)
    b = run(lagp, W, precision, n_max, Np_max, n_per, Np_per, normalize=True)
    for k in ("pool", "sel", "mean", "s2", "var", "status", "guard"):
        assert np.array_equal(a[k], b[k], equal_nan=True), k
    f = orc.alc(W.X, W.Y, W.XX, a["pool"], W.n0, n_max, W.d, W.g, n_per=n_per, Np_per=Np_per, forced=a["sel"],
                mode_b=True)
    worst = 0.0
    for m in range(W.M):
        n = n_max if n_per is None else int(n_per[m])
        j = np.arange(W.n0, n)
        factor = f["psitraj"][m, j] / (j - 2)
        got = b["alc"][m, j]
        want = f["dsel"][m, j] * factor
        scale = f["dmax"][m, j] * factor
        tol = np.maximum(1e-9, 10 * f["nu"][m, j])
        worst = max(worst, float(np.max(np.abs(got - want) / scale / tol)))
        # the factor itself: psi_j of the GPU's design against the oracle's, to
        # the same resolution as the scores (the oracle's route noise)
        ratio = b["alc"][m, j] / a["alc"][m, j]
        assert np.all(np.abs(ratio - factor) / factor <= tol), m
        assert np.all(np.isnan(b["alc"][m, :W.n0]))
        if precision == "mixed":
            fin = np.isfinite(a["alc32"][m, j])
            r32 = b["alc32"][m, j][fin] / a["alc32"][m, j][fin]
            assert np.all(np.abs(r32 - factor[fin]) <= 1e-6 * factor[fin]), m
    _log(f"normalize_{precision}_{'uneven' if per_location else 'uniform'}", dict(worst_over_tol=worst))
    assert worst <= 1.0


def mixed_trusted(n, g):
    """The library's a-priori rule for float32 scores: the nugget bounds
    cond(K_j) by (j + g) / g, and float32 is used while that bound for the
    whole design times 2^-24 is at most 2^-4."""
    return (n + g) / g * 2.0 ** -24 <= 2.0 ** -4


@pytest.mark.parametrize("nugget", [1e-5, 1e-4])
def test_mixed_per_location(lagp, orc, nugget):
    """LAGP_MIXED with config-3 shapes (n in 20..100, N' in 200..2000 per
    location): locations within the mixed kernel's sizes (n <= 64, N' <= 1024)
    whose nugget keeps K_j conditioned well enough for float32 scores run in
    mixed precision, the others in float64 with all their steps counted in
    guard; every design and output against the oracle.  At config 3's own
    nugget (1e-5) no location qualifies: float32 scores lose the conditional
    variance to cancellation there."""
    W = workloads.make(3, M=60)
    W.g = nugget
    print(f"[boundary] mixed per-location M={W.M} g={nugget}", flush=True)
    g = run(lagp, W, "mixed", 100, 2000, W.n_per, W.Np_per)
    assert np.array_equal(g["pool"], orc.nn_pool(W.X, W.XX, 2000))
    assert np.all(g["status"] == 0), g["status"]
    eligible = (W.n_per <= 64) & (W.Np_per <= 1024) & mixed_trusted(W.n_per, nugget)
    if nugget < 1e-4:
        assert eligible.sum() == 0
    else:
        assert 0 < eligible.sum() < W.M
    steps = W.n_per - W.n0
    for m in np.flatnonzero(~eligible):
        assert g["guard"][m] == steps[m], m
        assert np.all(np.isnan(g["alc32"][m]))
    for m in range(W.M):
        assert np.all(g["sel"][m, W.n_per[m]:] == -1)
    forced = orc.alc(W.X, W.Y, W.XX, g["pool"], W.n0, 100, W.d, W.g, n_per=W.n_per, Np_per=W.Np_per,
                     forced=g["sel"], mode_b=True)
    seq = parity.sequence_check(g["sel"], g["pool"], forced, W.n0, n_per=W.n_per)
    mean_floor = 1e-6 * np.sqrt(np.mean(W.Y ** 2))
    worst, rep = parity.output_check(g, forced, W.X, W.d, W.g, 1e-4, mean_floor)
    # the float64 locations meet the float64 bar
    g64 = {k: g[k][~eligible] for k in ("mean", "s2", "var", "sel")}
    f64 = {k: forced[k][~eligible] for k in forced if forced[k].shape[:1] == (W.M,)}
    worst64, _ = parity.output_check(g64, f64, W.X, W.d, W.g, 1e-10, mean_floor)
    frac = float(g["guard"][eligible].sum()) / max(1.0, float(steps[eligible].sum()))
    _log(f"mixed_per_location_g{nugget:g}", dict(M=W.M, eligible=int(eligible.sum()), ties=seq["ties"],
                                    fails=len(seq["fails"]), outputs=rep, worst_over_tol=worst,
                                    worst64_over_tol=worst64, mixed_fallback_steps_frac=frac))
    assert not seq["fails"], seq["fails"][:5]
    assert worst <= 1.0 and worst64 <= 1.0


def test_row_offsets_and_nn_variants(lagp):
    """Flat rows by offsets equal the padded rows; the brute-force and
    grid-pruned pools give identical results through the one-call entry point."""
    import torch

    W = workloads.make(3, N=20000, M=16)
    n_per, Np_per = W.n_per, W.Np_per
    off = np.concatenate([[0], np.cumsum(n_per)]).astype(np.int64)
    pad = run(lagp, W, "fp64", 100, 2000, n_per, Np_per)
    brute = run(lagp, W, "fp64", 100, 2000, n_per, Np_per, nn="brute")
    for k in ("pool", "sel", "mean", "s2", "var", "alc", "status"):
        assert np.array_equal(pad[k], brute[k], equal_nan=True), k
    out = dict(sel=torch.full((int(off[-1]),), -9, dtype=torch.int32, device="cuda"),
               alc=torch.zeros(int(off[-1]), dtype=torch.float64, device="cuda"),
               alc32=torch.zeros(int(off[-1]), dtype=torch.float64, device="cuda"))
    flat = run(lagp, W, "fp64", 100, 2000, n_per, Np_per, sel_off=dev(off), out=out)
    for m in range(W.M):
        assert np.array_equal(flat["sel"][off[m]:off[m + 1]], pad["sel"][m, :n_per[m]])
        assert np.array_equal(flat["alc"][off[m]:off[m + 1]], pad["alc"][m, :n_per[m]], equal_nan=True)
    for k in ("mean", "s2", "var", "status"):
        assert np.array_equal(flat[k], pad[k], equal_nan=True), k


@pytest.mark.parametrize("case", ["config2_mixed", "config3_mixed"])
def test_mixed_plan_replays(lagp, case):
    """Plans in mixed precision (uniform, and per-location with the float64
    stand-in): every graph replay equals the eager call bit for bit."""
    import torch

    if case == "config3_mixed":
        W = workloads.make(3, N=50000, M=300)
        n_max, Np_max, n_per, Np_per = 100, 2000, dev(W.n_per), dev(W.Np_per)
    else:
        W = workloads.make(2, N=50000, M=300)
        n_max, Np_max, n_per, Np_per = 50, 1000, None, None
    X, Y, XX = dev(W.X), dev(W.Y), dev(W.XX)
    keys = ("pool", "sel", "mean", "s2", "var", "status", "guard", "alc", "alc32")
    snap = lambda o: {k: o[k].cpu().numpy().copy() for k in keys}  # noqa: E731
    eager = lagp.alc_predict(X, Y, XX, W.n0, n_max, Np_max, W.d, W.g, "mixed", n_per=n_per, Np_per=Np_per)
    torch.cuda.synchronize()
    ref = snap(eager)
    plan = lagp.Plan(X, Y, XX, W.n0, n_max, Np_max, W.d, W.g, n_per=n_per, Np_per=Np_per, precision="mixed")
    torch.cuda.synchronize()
    print(f"[boundary] plan {case}: {plan.describe()}", flush=True)
    for rep in range(3):
        for k in ("mean", "s2", "var", "alc", "alc32"):
            plan.out[k].fill_(float("nan"))
        for k in ("sel", "status", "pool", "guard"):
            plan.out[k].fill_(-5)
        lagp.alc_predict(X, Y, XX, W.n0, n_max, Np_max, W.d, W.g, "mixed", n_per=n_per, Np_per=Np_per, out=eager)
        plan.launch()
        torch.cuda.synchronize()
        got, again = snap(plan.out), snap(eager)
        for k in keys:
            assert np.array_equal(got[k], ref[k], equal_nan=True), (rep, k)
            assert np.array_equal(again[k], ref[k], equal_nan=True), (rep, k)
    plan.close()
