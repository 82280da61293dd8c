"""Local likelihood, its hand-written backward, the local MLE of d and
prediction on fixed designs: GPU (through the C ABI) against the CPU oracle."""
from __future__ import annotations

import json
import os

import numpy as np
import pytest

import workloads

pytestmark = pytest.mark.gpu

OUT = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "gpurun_out")


def _log(name, rec):
    print(f"[mle] {name}: {json.dumps(rec)}", flush=True)
    os.makedirs(OUT, exist_ok=True)
    with open(os.path.join(OUT, "mle_log.jsonl"), "a") as f:
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


def designs(orc, cfg=4, N=20000, M=24, n=50, Np=500, d0=0.2):
    """Local designs chosen by the oracle's greedy ALC (config-4 shapes)."""
    W = workloads.make(cfg, N=N, M=M)
    out = orc.lagp(W.X, W.Y, W.XX, 6, n, Np, d0, W.g)
    return W, out["sel"]


def rel(a, b, floor=1e-300):
    a, b = np.asarray(a, float), np.asarray(b, float)
    return np.abs(a - b) / np.maximum(np.abs(b), floor)


def check_d_hat(orc, W, sel, d_gpu, d_orc, ok):
    """Both sides stop when |nll'| <= 1e-10 or the step is <= 1e-10 d, so on a
    flat likelihood the stopping points may differ by about 1e-10 / nll''.
    Accept |d_gpu - d_orc| <= max(1e-6 d_orc, 1e-9 / nll''(d_orc))."""
    worst = 0.0
    for m in np.flatnonzero(ok):
        h = orc.nll(W.X[sel[m]], W.Y[sel[m]], d_orc[m], W.g)["d2"]
        tol = max(1e-6 * d_orc[m], 1e-9 / h if h > 0 else 0.0)
        err = abs(d_gpu[m] - d_orc[m])
        assert err <= tol, (m, d_gpu[m], d_orc[m], h)
        worst = max(worst, err / d_orc[m])
    return worst


@pytest.mark.parametrize("n", [1, 7, 50, 64])
def test_nll_and_derivatives(lagp, orc, n):
    import torch

    W, sel = designs(orc, n=max(n, 6), M=16)
    sel = np.ascontiguousarray(sel[:, :n])
    r = np.random.default_rng(n)
    d = r.uniform(0.05, 1.5, len(sel))
    g = r.uniform(1e-4, 1e-2, len(sel))
    print(f"[mle] nll n={n} M={len(sel)}", flush=True)
    got = lagp.local_nll(dev(W.X), dev(W.Y), dev(sel), dev(d), dev(g), order=2)
    torch.cuda.synchronize()
    got = {k: v.cpu().numpy() for k, v in got.items()}
    want = [orc.nll(W.X[s], W.Y[s], dm, gm) for s, dm, gm in zip(sel, d, g)]
    assert np.all(got["status"] == 0)
    rec = {}
    for k, tol in (("nll", 1e-10), ("dd", 1e-8), ("dg", 1e-8), ("d2", 1e-7)):
        w = np.array([x[k] for x in want])
        scale = np.maximum(np.abs(w), 1.0)
        err = float(np.max(np.abs(got[k] - w) / scale))
        rec[k] = err
        assert err <= tol, (k, err)
    _log(f"nll_n{n}", rec)


def test_backward_matches_oracle_and_finite_differences(lagp, orc):
    import torch

    W, sel = designs(orc, M=12)
    r = np.random.default_rng(3)
    d = dev(r.uniform(0.1, 1.0, len(sel))).requires_grad_(True)
    g = dev(r.uniform(1e-4, 1e-2, len(sel))).requires_grad_(True)
    X, Y, S = dev(W.X), dev(W.Y), dev(sel)
    nll = lagp.LocalNLL.apply(d, g, X, Y, S)
    w = dev(r.normal(size=len(sel)))
    (nll * w).sum().backward()
    gd, gg = d.grad.cpu().numpy(), g.grad.cpu().numpy()
    dn, gn, wn = d.detach().cpu().numpy(), g.detach().cpu().numpy(), w.cpu().numpy()
    want = [orc.nll(W.X[s], W.Y[s], dm, gm) for s, dm, gm in zip(sel, dn, gn)]
    wd = np.array([x["dd"] for x in want]) * wn
    wg = np.array([x["dg"] for x in want]) * wn
    assert np.max(rel(gd, wd, 1e-6)) < 1e-8
    assert np.max(rel(gg, wg, 1e-6)) < 1e-8
    # central differences of the GPU forward itself
    with torch.no_grad():
        hd, hg = 1e-6 * d, 1e-5 * g
        fd_d = (lagp.LocalNLL.apply(d + hd, g, X, Y, S) - lagp.LocalNLL.apply(d - hd, g, X, Y, S)) / (2 * hd)
        fd_g = (lagp.LocalNLL.apply(d, g + hg, X, Y, S) - lagp.LocalNLL.apply(d, g - hg, X, Y, S)) / (2 * hg)
    fd_d, fd_g = (fd_d * w).cpu().numpy(), (fd_g * w).cpu().numpy()
    e1 = float(np.max(rel(gd, fd_d, 1e-3)))
    e2 = float(np.max(rel(gg, fd_g, 1e-3)))
    _log("backward", dict(fd_d=e1, fd_g=e2))
    assert e1 < 1e-5 and e2 < 1e-5


def test_mle_matches_oracle(lagp, orc):
    import torch

    W, sel = designs(orc, M=32)
    d0 = 0.2
    print("[mle] mle config4-shaped M=32", flush=True)
    got = lagp.local_mle_d(dev(W.X), dev(W.Y), dev(sel), d0, W.g, 1e-3, 5.0, 100)
    torch.cuda.synchronize()
    got = {k: v.cpu().numpy() for k, v in got.items()}
    want = orc.local_mle(W.X, W.Y, sel, d0, W.g, 1e-3, 5.0, 100)
    assert np.array_equal(got["status"], want["status"])
    ok = want["status"] == 0
    e_f = float(np.max(rel(got["nll"][ok], want["nll"][ok], 1.0)))
    e_d = check_d_hat(orc, W, sel, got["d"], want["d"], ok)
    _log("mle", dict(converged=int(ok.sum()), max_rel_d=e_d, max_rel_nll=e_f,
                     iters_gpu=float(got["iters"].mean()), iters_oracle=float(want["iters"].mean())))
    assert ok.all(), want["status"]  # every design of this workload converges on both sides
    assert e_f < 1e-10


def test_predict_on_fixed_design(lagp, orc):
    import torch

    W, sel = designs(orc, M=20)
    r = np.random.default_rng(9)
    d = r.uniform(0.05, 2.0, len(sel))
    got = lagp.local_predict(dev(W.X), dev(W.Y), dev(sel), dev(W.XX), dev(d), W.g)
    torch.cuda.synchronize()
    got = {k: v.cpu().numpy() for k, v in got.items()}
    assert np.all(got["status"] == 0)
    worst, gap_max = 0.0, 0.0
    for m in range(len(sel)):
        ref = orc.gp_predict(W.X[sel[m]], W.Y[sel[m]], W.XX[m], d[m], W.g)
        # the parity protocol's output bound: 1e-10, raised only to 10x the gap
        # between the oracle's two float64 routes on this design (Cholesky vs
        # the inverse grown by the partitioned inverse, eq. piedef)
        refb = orc.gp_predict_b(W.X[sel[m]], W.Y[sel[m]], W.XX[m], d[m], W.g)
        for k in ("mean", "s2", "var"):
            gap = float(rel(refb[k], ref[k], 1e-8))
            gap_max = max(gap_max, gap)
            tol = max(1e-10, 10 * gap)
            r = rel(got[k][m], ref[k], 1e-8)
            worst = max(worst, r / tol)
            assert r < tol, (m, k, r, tol)
    _log("predict", dict(worst_over_tol=worst, max_route_gap=gap_max))


def test_config4_pipeline_subsample(lagp, orc):
    """Config 4 on 64 locations: NN pool -> ALC at d0 -> MLE of d -> prediction."""
    import torch

    W = workloads.make(4, M=64)
    X, Y, XX = dev(W.X), dev(W.Y), dev(W.XX)
    o = lagp.alc_predict(X, Y, XX, W.n0, W.n, W.Np, 0.2, W.g, "fp64")
    mle = lagp.local_mle_d(X, Y, o["sel"], 0.2, W.g, 1e-3, 5.0, 100)
    pr = lagp.local_predict(X, Y, o["sel"], XX, mle["d"], W.g)
    torch.cuda.synchronize()
    sel = o["sel"].cpu().numpy()
    ref = orc.local_mle(W.X, W.Y, sel, 0.2, W.g, 1e-3, 5.0, 100)
    dh = mle["d"].cpu().numpy()
    assert np.array_equal(mle["status"].cpu().numpy(), ref["status"])
    ok = ref["status"] == 0
    assert ok.all(), ref["status"]
    check_d_hat(orc, W, sel, dh, ref["d"], ok)
    assert np.max(rel(mle["nll"].cpu().numpy()[ok], ref["nll"][ok], 1.0)) < 1e-10
    mean = pr["mean"].cpu().numpy()
    for m in np.flatnonzero(ok):
        want = orc.gp_predict(W.X[sel[m]], W.Y[sel[m]], W.XX[m], ref["d"][m], W.g)
        assert rel(mean[m], want["mean"], 1e-6) < 1e-6
    _log("config4_pipeline", dict(M=W.M, converged=int(ok.sum()), d_min=float(dh.min()),
                                  d_max=float(dh.max()), d_median=float(np.median(dh))))


def test_bad_design_index_status(lagp):
    import torch

    W = workloads.make(4, N=2000, M=3)
    sel = np.tile(np.arange(10, dtype=np.int32), (3, 1))
    sel[1, 4] = -1
    sel[2, 9] = W.N
    out = lagp.local_nll(dev(W.X), dev(W.Y), dev(sel), 0.3, 1e-3, order=1)
    torch.cuda.synchronize()
    st = out["status"].cpu().numpy()
    assert list(st) == [0, 4, 4]
    assert np.isnan(out["nll"].cpu().numpy()[1:]).all()
