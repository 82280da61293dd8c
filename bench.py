"""Benchmark of the local approximate GP hot path on one MI355X.

One step = the whole path over one batch of predictive locations: NN
candidate pools, greedy ALC local designs (n0 -> n) and local predictions.
Default workload: N = 100,000 design points uniform on [0,1]^8, M = 10,000
predictive locations, n0 = 6, n = 50, N' = 1000, d = 0.5, g = 1e-4 (seeded
synthetic data).  `value` is predictive locations per second of the
mixed-precision path with inputs resident in HBM; the float64 path is timed
beside it.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu-baseline]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK = {"fp32_mfma": 157.3e12, "fp64_mfma": 78.6e12, "hbm": 8.0e12}


def alc_flops(n0: int, n: int, Np: int) -> float:
    """Algorithmic flops of the candidate scoring for one location: every
    step j scores the Np - j candidates at 2 j^2 flops each (the O(j^2)
    per-candidate cost of eq. dxy, Sec. 3.1)."""
    return float(sum(2.0 * (Np - j) * j * j for j in range(n0, n)))


def alc_evals(n0: int, n: int, Np: int) -> int:
    return sum(Np - j for j in range(n0, n))


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--config", type=int, default=2)
    ap.add_argument("--M", type=int, default=None, help="predictive locations (default: the config's)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-sample", type=int, default=512)
    ap.add_argument("--only", choices=["mixed", "fp64", "both"], default="both")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="only run a plain device copy of MIB MiB (HBM counter calibration)")
    args = ap.parse_args()

    if args.copy_calibration:
        import torch

        nbytes = args.copy_calibration << 20
        src = torch.ones(nbytes // 4, dtype=torch.float32, device="cuda:0")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_read": nbytes, "copy_bytes_written": nbytes, "dispatches": 3}))
        return 0

    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU only; --gpus must be 1"}))
        return 2

    import torch

    import paper_1310_5182_amd as lagp
    import workloads

    W = workloads.make(args.config, M=args.M)
    n0, n, Np, d, g = W.n0, W.n, W.Np, W.d, W.g
    print(f"[bench] workload config{args.config}: N={W.N} p={W.p} M={W.M} n0={n0} n={n} Np={Np}",
          file=sys.stderr, flush=True)
    dev = torch.device("cuda:0")
    X = torch.from_numpy(W.X).to(dev)
    Y = torch.from_numpy(W.Y).to(dev)
    XX = torch.from_numpy(W.XX).to(dev)
    M = W.M
    precs = ["mixed", "fp64"] if args.only == "both" else [args.only]
    outs = {p: None for p in precs}
    stream = torch.cuda.current_stream(dev)

    def full_step(prec):
        outs[prec] = lagp.alc_predict(X, Y, XX, n0, n, Np, d, g, prec, out=outs[prec])

    res = {}
    for prec in precs:
        for _ in range(args.warmup):
            full_step(prec)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            full_step(prec)
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t0) / args.steps
        res[prec] = dict(ms_per_step=dt * 1e3, loc_per_s=M / dt)
        print(f"[bench] {prec}: {dt * 1e3:.2f} ms/step, {M / dt:.1f} loc/s", file=sys.stderr, flush=True)

    # Per-kernel timing with HIP events on the stream the library launches on.
    pool = outs[precs[0]]["pool"]
    ev = lambda: torch.cuda.Event(enable_timing=True)  # noqa: E731
    e0, e1 = ev(), ev()
    e0.record(stream)
    for _ in range(args.steps):
        lagp.nn_pool(X, XX, Np, out=pool)
    e1.record(stream)
    torch.cuda.synchronize()
    nn_ms = e0.elapsed_time(e1) / args.steps
    alc_ms = {}
    for prec in precs:
        o = outs[prec]
        e0, e1 = ev(), ev()
        e0.record(stream)
        for _ in range(args.steps):
            lagp.alc_from_pool(X, Y, XX, pool, n0, n, d, g, prec, out=o)
        e1.record(stream)
        torch.cuda.synchronize()
        alc_ms[prec] = e0.elapsed_time(e1) / args.steps
        print(f"[bench] kernels: nn_pool {nn_ms:.3f} ms, alc[{prec}] {alc_ms[prec]:.3f} ms",
              file=sys.stderr, flush=True)

    head = "mixed" if "mixed" in precs else "fp64"
    flops = alc_flops(n0, n, Np) * M
    peak = PEAK["fp32_mfma"] if head == "mixed" else PEAK["fp64_mfma"]
    achieved = flops / (alc_ms[head] * 1e-3)
    o = outs[head]
    status = o["status"].cpu().numpy()
    guard = o["guard"].cpu().numpy()
    evals = alc_evals(n0, n, Np) * M

    cpu = None
    if not args.no_cpu_baseline:
        import oracle

        S = min(args.cpu_sample, M)
        orc = oracle.default()
        threads = orc.max_threads()
        t0 = time.perf_counter()
        orc.lagp(W.X, W.Y, W.XX[:S], n0, n, Np, d, g, threads=threads)
        dt = time.perf_counter() - t0
        cpu = dict(value=S / dt, unit="loc/s", cores=threads, kind="oracle",
                   sample=f"first {S} of the {M} locations, NN pool + ALC design + prediction, "
                          f"float64, OpenMP over locations ({dt:.1f} s wall)")
        print(f"[bench] cpu oracle: {S / dt:.1f} loc/s on {threads} threads", file=sys.stderr, flush=True)

    line = {
        "metric": "predictive locations/sec (n=50 ALC, N'=1000) mixed vs FP64; ALC evals/sec",
        "value": res[head]["loc_per_s"],
        "unit": "loc/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": res[head]["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32+f64" if head == "mixed" else "f64",
        "data": "synthetic",
        "config": {"workload": f"config{args.config}: N={W.N} p={W.p} uniform design, M={M} "
                               f"locations, n0={n0}, n={n}, N'={Np}, d={d}, g={g}",
                   "precision": head},
        "fp64_loc_per_s": res.get("fp64", {}).get("loc_per_s"),
        "mixed_over_fp64": (res["mixed"]["loc_per_s"] / res["fp64"]["loc_per_s"]) if len(precs) == 2 else None,
        "alc_evals_per_s": evals / (alc_ms[head] * 1e-3),
        "kernel_ms": {"nn_pool": nn_ms, **{f"alc_{k}": v for k, v in alc_ms.items()}},
        "guard_steps_frac": float(guard.sum()) / (M * (n - n0)),
        "status_nonzero": int(np.count_nonzero(status)),
        "roofline": {"kernel": f"alc_kernel<{'float' if head == 'mixed' else 'double'}>",
                     "bound": "mfma", "achieved": achieved / 1e12, "peak": peak / 1e12,
                     "unit": "TFLOP/s", "frac": achieved / peak, "traffic": None},
        "cpu_baseline": cpu,
    }
    print(json.dumps(line), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
