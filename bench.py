"""Benchmark: directional FMM matvecs per second on one MI355X.

Workload: N = 65,536 points uniform on a sphere of diameter K = 16 wavelengths
(seed 2), complex64 densities with real and imaginary parts iid N(0, 1),
one right-hand side, plan eps = 1e-4.  A step is one dfmm_apply (the whole
evaluation pass: S2M, HF-M2M, HF-M2L + L2L, LF-M2L, L2T and the near-field
sum) with inputs and outputs resident in HBM.

Prints one JSON line.  ``value`` counts only if the relative L2 error against
the float64 direct sum on 2,048 sampled targets is <= eps (reported as
``rel_l2_err``).  The roofline entry is for the dominant kernel, the grouped
M2L GEMM (HF and LF launches): algorithmic flops 8 r_in r_out per (pair, rhs)
divided by the launch time measured with HIP events on the apply stream over
the timed steps, against the FP32 matrix peak of MI355X (157.3 TFLOP/s).
The CPU baseline times the float64 oracle pass on a bounded sample of the
same geometry.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_FP32_MATRIX_TFLOPS = 157.3
CACHE_DIR = os.path.join(ROOT, ".dfmm_cache")


def cpu_baseline(pts, f, K, eps_tau, n_sample=16384):
    """Float64 oracle FMM on the first n_sample points of the same sphere (time of the pass only)."""
    import numpy as np

    from oracle.cache import oracle_opset
    from oracle.fmm import fmm_apply
    from oracle.tree import build_structure

    sub = pts[:n_sample]
    fs = f[:, :n_sample].astype(np.complex128)
    st = build_structure(sub, K)
    ops = oracle_opset(eps_tau, max(1, st.w_top))
    t0 = time.perf_counter()
    fmm_apply(st, ops, fs)
    dt = time.perf_counter() - t0
    threads = None
    try:
        from threadpoolctl import threadpool_info

        threads = max(int(x.get("num_threads", 1)) for x in threadpool_info()) if threadpool_info() else 1
    except Exception:
        threads = os.cpu_count()
    return {
        "value": n_sample * fs.shape[0] / dt,
        "unit": "matvecs/s",
        "cores": threads,
        "kind": "oracle",
        "sample": f"float64 oracle pass on the first {n_sample} points of the same K=16 sphere "
                  f"(same tree depth and skeletons), {dt:.2f} s; host has {os.cpu_count()} cores",
    }


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU only: this build has no multi-GPU path "
              "(run with --gpus 1)", file=sys.stderr)
        return 2

    import numpy as np
    import torch

    from paper_1311_4257_amd import dfmm, workloads

    pts, f, cfg = workloads.make_config("sphere16")
    K, N, nrhs, eps = cfg["K"], cfg["N"], cfg["nrhs"], cfg["eps"]
    dev = torch.device("cuda:0")
    plan = dfmm.Plan(pts, K, eps=eps, cache_dir=CACHE_DIR, device=0)
    info = plan.info()
    fd = torch.from_numpy(f.astype(np.complex64)).to(dev)
    u = torch.empty_like(fd)
    stream = torch.cuda.current_stream(dev)

    for _ in range(args.warmup):
        plan.apply(fd, u, stream)
    torch.cuda.synchronize()
    plan.set_timing(args.steps)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        plan.apply(fd, u, stream)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    stages = plan.stage_times()
    plan.set_timing(0)
    ms = (t1 - t0) * 1e3 / args.steps

    # accuracy gate against the float64 direct sum
    from oracle.kernel import direct_sum, rel_l2

    tg = workloads.sample_targets(N, cfg["n_check"], cfg["check_seed"])
    err = rel_l2(u.cpu().numpy().astype(np.complex128)[:, tg], direct_sum(pts, f, tg))

    m2l_ms = stages["hf_m2l"][0] + stages["lf_m2l"][0]
    m2l_launches = stages["hf_m2l"][1] + stages["lf_m2l"][1]
    flops_apply = (info.flops_m2l_hf + info.flops_m2l_lf) * nrhs
    achieved = flops_apply * args.steps / (m2l_ms * 1e-3) / 1e12 if m2l_ms > 0 else 0.0
    per_stage = {k: round(v[0] / args.steps, 4) for k, v in stages.items() if v[1]}

    out = {
        "metric": "FMM matvecs/s (N*nrhs/s) at 1e-4 rel err vs direct sum",
        "value": N * nrhs / (ms * 1e-3),
        "unit": "matvecs/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "sphere16: N=65536 uniform on a sphere of diameter K=16 (seed 2), "
                               "complex64 N(0,1) densities, nrhs=1, eps=1e-4",
                   "K": K, "N": N, "nrhs": nrhs, "eps": eps, "w_top": info.w_top,
                   "ranks": [int(info.rank[l]) for l in range(info.depth + 1)]},
        "rel_l2_err": err,
        "accuracy_ok": bool(err <= eps),
        "stage_ms": per_stage,
        "roofline": {
            "bound": "mfma",
            "kernel": "k_ggemm (grouped M2L, HF + LF launches)",
            "achieved": achieved,
            "peak": PEAK_FP32_MATRIX_TFLOPS,
            "unit": "TFLOP/s",
            "frac": achieved / PEAK_FP32_MATRIX_TFLOPS,
            "traffic": None,
            "flops_per_apply": flops_apply,
            "launches_per_apply": m2l_launches / max(1, args.steps),
        },
        "plan_seconds": info.plan_seconds,
    }
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(pts, f, K, 0.15 * eps)  # the library's tau for eps
    print(json.dumps(out))
    return 0


if __name__ == "__main__":
    sys.exit(main())
