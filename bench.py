#!/usr/bin/env python3
"""HODLR2D matvec throughput on one MI355X, with time-to-1e-8 of GMRES.

Workload (one step = one Algorithm-2 matvec, the whole fast product):
  N = 2^20 points i.i.d. uniform in [-1, 1]^2 (seed 1), multiquadric
  sqrt(1 + (r / 0.1)^2) with 1e-6 added on the diagonal, leaf size 64,
  ACA tolerance 1e-10, one right-hand side uniform in [-1, 1].
The operator is built once on the GPU (Algorithm 1, reported apart), then
W warm-up and K timed FP64 matvecs run back to back on one stream.

value = algorithmic bytes of one FP64 matvec (every stored U, V and dense
value read once, plus the vectors) / measured time per matvec, in GB/s.

Also reported: FP16 / BF16 matvec rates, time-to-1e-8 of plain FP64
GMRES(50) against FP16 factors + FP64 iterative refinement on the log
kernel (N = 2^20, diagonal N, seed 2), GMRES on the multiquadric system,
the dominant kernel's roofline fraction from HIP events recorded around
each kernel inside the timed region, and the CPU oracle's matvec rate on a
bounded sample of the same recipe.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0


def log(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)


def cpu_baseline(n_sample: int = 65536, min_seconds: float = 5.0):
    """The oracle (single-threaded C, FP64) on the first recipe at N=n_sample."""
    import numpy as np

    import oracle
    from paper_2204_05536_amd import inputs

    oracle.build(force=False)
    xy, b, kern, leaf, tol = inputs.workload("mq1m", n=n_sample)
    t0 = time.perf_counter()
    O = oracle.OracleH(xy, kern, leaf, tol)
    t_build = time.perf_counter() - t0
    tab = O.il_table()
    levels = [O.level(l) for l in range(O.kappa + 1)]
    byts = 0.0
    for l, t, s, kd, k in zip(tab["level"], tab["tgt"], tab["src"], tab["kind"], tab["rank"]):
        m = levels[l]["count"][t]; n = levels[l]["count"][s]
        byts += 8.0 * (m * n if kd == 1 else k * (m + n))
    LL = levels[-1]
    nt, ns = O.near_table()
    byts += 8.0 * float(np.sum(LL["count"][nt] * LL["count"][ns]))
    byts += n_sample * (8 + 8 + 8 + 4)
    reps = 0
    t0 = time.perf_counter()
    while True:
        O.matvec(b)
        reps += 1
        el = time.perf_counter() - t0
        if el >= min_seconds and reps >= 3:
            break
    per = el / reps
    return {"value": byts / per / 1e9, "unit": "GB/s", "cores": 1, "kind": "oracle",
            "sample": f"oracle FP64 matvec on N={n_sample} points of the same recipe (uniform [-1,1]^2 seed 1, "
                      f"MQ c=0.1 +1e-6 I, leaf 64, tol 1e-10): {reps} matvecs averaged, {per * 1e3:.1f} ms each; "
                      f"oracle build {t_build:.1f} s excluded",
            "ms_per_matvec": per * 1e3}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--n", type=int, default=1 << 20)
    ap.add_argument("--no-solve", action="store_true")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-half", action="store_true")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="also run a plain 1 GiB device copy (a known-size kernel for counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (got --gpus {args.gpus}); the HODLR2D path here is single-GPU.",
              file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    from paper_2204_05536_amd import hodlr2d, inputs

    torch.cuda.set_device(0)
    xy, b, kern, leaf, tol = inputs.workload("mq1m", n=args.n)
    precs = () if args.no_half else ("fp16", "bf16")
    log(f"building N={args.n} MQ leaf={leaf} tol={tol}")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    H = hodlr2d.HODLR2D.build(torch.from_numpy(xy).cuda(), kern, leaf, tol, precs=precs)
    torch.cuda.synchronize()
    t_build = time.perf_counter() - t0
    info = H.info()
    log(f"built in {t_build:.2f} s: kappa={info['kappa']} IL={info['n_il']} dense IL={info['n_il_dense']} "
        f"max rank={info['max_rank']} alg bytes={info['alg_bytes_fp64'] / 1e9:.2f} GB")
    x = torch.from_numpy(b).cuda()
    y = torch.empty_like(x)

    def timed(prec, steps, warmup, profile):
        for _ in range(warmup):
            H.matvec(x, prec=prec, out=y)
        torch.cuda.synchronize()
        if profile:
            H.profile_read()  # clear
            H.profile_enable(True)
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        e0.record()
        for _ in range(steps):
            H.matvec(x, prec=prec, out=y)
        e1.record()
        torch.cuda.synchronize()
        prof = None
        if profile:
            H.profile_enable(False)
            prof = H.profile_read()
        return e0.elapsed_time(e1) / steps, prof

    ms, prof = timed("fp64", args.steps, args.warmup, True)
    if args.calibrate_copy:
        # an elementwise kernel that reads 1 GiB and writes 1 GiB (a plain
        # device copy may run on a DMA engine, which kernel counters miss)
        src = torch.ones(1 << 27, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            torch.mul(src, 2.0, out=dst)
        torch.cuda.synchronize()
        log("copy calibration: 3 x (1 GiB read + 1 GiB write) elementwise kernels done")
        del src, dst
    gbs = info["alg_bytes_fp64"] / (ms * 1e-3) / 1e9
    log(f"FP64 matvec {ms:.3f} ms  {gbs:.0f} GB/s  phases ms={prof['ms']}")
    # dominant kernel's roofline
    dom = max(prof["ms"], key=lambda k: prof["ms"][k])
    achieved = prof["bytes"][dom] / (prof["ms"][dom] * 1e-3) / 1e9
    roofline = {"bound": "hbm", "kernel": f"k_{dom}",
                "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS,
                "traffic": None, "alg_bytes_per_launch": prof["bytes"][dom], "avg_ms": prof["ms"][dom],
                "phases_ms": prof["ms"], "phases_alg_bytes": prof["bytes"]}
    extra = {"build_seconds": t_build, "kappa": info["kappa"], "n_il_blocks": info["n_il"],
             "n_il_dense": info["n_il_dense"], "max_rank": info["max_rank"],
             "alg_bytes_fp64": info["alg_bytes_fp64"], "matvecs_per_s": 1e3 / ms}
    # repeatable bits
    y1 = H.matvec(x).clone()
    y2 = H.matvec(x)
    extra["bitwise_repeatable"] = bool(torch.equal(y1, y2))
    if not args.no_half:
        half = {}
        for p in ("fp16", "bf16"):
            mh, ph = timed(p, args.steps, 2, True)
            yh = H.matvec(x, prec=p)
            err = float(torch.linalg.norm(yh - y1) / torch.linalg.norm(y1))
            half[p] = {"ms": mh, "GB/s": info["alg_bytes_half"] / (mh * 1e-3) / 1e9,
                       "rel_err_vs_fp64": err, "phases_ms": ph["ms"]}
            log(f"{p} matvec {mh:.3f} ms  {half[p]['GB/s']:.0f} GB/s  err {err:.2e}")
        extra["half"] = half
    if not args.no_solve:
        xs, sinfo = H.solve(x, tol=1e-8, restart=50, max_iter=100)
        extra["gmres_mq_plain"] = {k: sinfo[k] for k in ("iters", "relres", "seconds", "converged")}
        log(f"MQ GMRES(50) capped at 100 iterations: {sinfo}")
    H.close()
    del H
    torch.cuda.synchronize()
    if not args.no_solve:
        xy2, b2, kern2, leaf2, tol2 = inputs.workload("log1m", n=args.n)
        log("building log-kernel system for time-to-1e-8")
        H2 = hodlr2d.HODLR2D.build(torch.from_numpy(xy2).cuda(), kern2, leaf2, tol2, precs=("fp16",))
        bb = torch.from_numpy(b2).cuda()
        H2.solve(bb, tol=1e-8, restart=50)  # warm-up
        sol = {}
        xp, ip = H2.solve(bb, tol=1e-8, restart=50)
        sol["plain_fp64"] = {k: ip[k] for k in ("iters", "outer", "relres", "seconds", "converged")}
        xr, ir = H2.solve(bb, tol=1e-8, restart=50, mode="refine", inner_prec="fp16", inner_tol=1e-4)
        sol["refine_fp16"] = {k: ir[k] for k in ("iters", "outer", "relres", "seconds", "converged")}
        sol["refine_fp16"]["rel_diff_vs_plain"] = float(torch.linalg.norm(xr - xp) / torch.linalg.norm(xp))
        log(f"time-to-1e-8 plain {ip} refine {ir}")
        extra["time_to_1e-8_log1m"] = sol
        H2.close()
    cpu = None
    if not args.no_cpu:
        log("CPU oracle baseline")
        cpu = cpu_baseline()
        log(f"oracle {cpu['value']:.2f} GB/s")
    out = {
        "metric": "matvec GB/s + time-to-1e-8 residual at N=1M, plain FP64 vs chosen form",
        "value": gbs,
        "unit": "GB/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"HODLR2D FP64 matvec, N={args.n} uniform [-1,1]^2, multiquadric c=0.1 + 1e-6 I, "
                               f"leaf 64, ACA tol 1e-10, 1 RHS", "n": args.n, "leaf": 64, "tol": 1e-10,
                   "kernel": "mq", "parallelism": "single-gpu"},
        "roofline": roofline,
        "cpu_baseline": cpu,
        "extra": extra,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
