"""Benchmark: directional FMM matvecs per second on one MI355X.

Workload (default): N = 262,144 points on the ellipsoid with semi-axes
(16, 8, 4) wavelengths in a K = 32 box, uniform in area (seed 3), 32
right-hand sides of complex64 densities with real and imaginary parts iid
N(0, 1) (seed 303), plan eps = 1e-4.  ``--workload sphere16`` takes the K = 16
sphere with N = 65,536 and one right-hand side instead.  A step is one
dfmm_apply (the whole evaluation pass: S2M, HF-M2M, HF-M2L + L2L, LF-M2L, L2T
and the near-field sum) with inputs and outputs resident in HBM.

Prints one JSON line.  ``value`` counts only if the relative L2 error against
the float64 direct sum on 2,048 sampled targets (every right-hand side) is
<= eps (reported as ``rel_l2_err``).  The roofline entry is for the dominant kernel, the grouped
M2L GEMM (HF and LF launches): algorithmic flops 8 r_in r_out per (pair, rhs)
divided by the launch time measured with HIP events on the apply stream over
a second run of the same number of steps (the events cost a little time, so
``value`` comes from the event-free run), against the FP32 matrix peak of
MI355X (157.3 TFLOP/s), or against 8 TB/s when the algorithmic bytes make
HBM the lower ceiling.
The algorithmic bytes of the M2L are the operators once per offset group,
every source slot read once and every target slot read and written once;
where the slot form runs (16 rhs and more) its launches also carry the L2L
terms, whose operators (once each) and parent slots (read once) are added.
The CPU baseline times the float64 oracle pass on a bounded sample of the
same geometry (the first points of the same point set: same K, same tree
depth, same right-hand sides).

``--calib-copy`` adds, after the timed steps, one 256 MiB device-to-device
copy: the calibration kernel for the FETCH_SIZE / WRITE_SIZE counters.
``--traffic-summary FETCH_DIR WRITE_DIR`` (with ``--workload``) turns the CSV
output of the two counter runs into the workload's traffic record
(profiles/m2l_traffic_<workload>.json) that later runs of that workload at its
default eps report, while the GEMM sources are unchanged.
"""
from __future__ import annotations

import argparse
import csv
import glob
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_FP32_MATRIX_TFLOPS = 157.3
PEAK_F16_MATRIX_TFLOPS = 2500.0  # dense fp16 / bf16 MFMA
PEAK_HBM_GBS = 8000.0
CACHE_DIR = os.path.join(ROOT, ".dfmm_cache")
# the M2L launch is defined by the tile engine and the operator layout built at plan time
GEMM_SOURCES = ["paper_1311_4257_amd/csrc/apply.hip", "paper_1311_4257_amd/csrc/plan.cpp"]
CALIB_BYTES = 256 << 20
# --precision -> (dfmm_options.precision, the dtype reported)
PRECISIONS = {"fp32": (0, "f32"), "fp16x3": (1, "f16x3 (hi/lo f16 products, f32 sums)"),
              "bf16x3": (2, "bf16x3 (hi/lo bf16 products, f32 sums)")}
# workload name -> (description, targets checked against the direct sum)
WORKLOADS = {
    "sphere16": ("sphere16: N=65536 uniform on a sphere of diameter K=16 (seed 2), complex64 N(0,1) "
                 "densities, nrhs=1", 2048),
    "ellipsoid32": ("ellipsoid32: N=262144 area-uniform on the ellipsoid with semi-axes (16, 8, 4) in a "
                    "K=32 box (seed 3), complex64 N(0,1) densities, nrhs=32", 2048),
}


def gemm_source_hash() -> str:
    h = hashlib.sha1()
    for rel in GEMM_SOURCES:
        with open(os.path.join(ROOT, rel), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def _counter_rows(d: str):
    """Rows (dispatch id, kernel name, counter, value) of a rocprofv3 counter-collection CSV."""
    files = sorted(glob.glob(os.path.join(d, "**", "*counter_collection.csv"), recursive=True))
    if not files:
        raise SystemExit(f"no *counter_collection.csv under {d}")
    rows = []
    with open(files[0], newline="") as fh:
        for r in csv.DictReader(fh):
            rows.append((int(r["Dispatch_Id"]), r["Kernel_Name"], r["Counter_Name"], float(r["Counter_Value"])))
    return rows


def traffic_file(workload: str) -> str:
    return os.path.join(ROOT, "profiles", f"m2l_traffic_{workload}.json")


def traffic_summary(fetch_dir: str, write_dir: str) -> dict:
    """Per-launch HBM bytes of the M2L launches of one apply, scaled by the copy calibration.

    Both counter runs execute the same command; the M2L launches taken are those
    after the last permute-in launch (the final apply), and the calibration is
    the largest device-to-device copy (CALIB_BYTES read and written)."""
    out = {"source_sha1": gemm_source_hash(), "calib_bytes": CALIB_BYTES}
    for key, d, counter in (("fetch", fetch_dir, "FETCH_SIZE"), ("write", write_dir, "WRITE_SIZE")):
        rows = [r for r in _counter_rows(d) if r[2] == counter]
        per = {}
        for disp, name, _, val in rows:
            per.setdefault(disp, [name, 0.0])[1] += val
        disp_sorted = sorted(per.items())
        last_perm = max(i for i, (_, (n, _)) in enumerate(disp_sorted) if "k_permute_in" in n)
        m2l = [v for _, (n, v) in disp_sorted[last_perm:] if "k_m2l" in n]
        copies = [v for _, (n, v) in disp_sorted if "copyBuffer" in n]
        if not m2l or not copies:
            raise SystemExit(f"{counter}: no M2L launch or no calibration copy found in {d}")
        calib_kib = max(copies)
        factor = (CALIB_BYTES / 1024.0) / calib_kib
        out[key] = {"counter": counter, "m2l_kib": m2l, "calib_kib": calib_kib, "factor": factor,
                    "bytes_per_launch": factor * 1024.0 * sum(m2l) / len(m2l)}
    out["launches"] = len(out["fetch"]["m2l_kib"])
    out["bytes_per_launch"] = out["fetch"]["bytes_per_launch"] + out["write"]["bytes_per_launch"]
    return out


def cpu_baseline(pts, f, K, eps_tau, workload, n_sample):
    """Float64 oracle FMM on the first n_sample points of the same point set (same
    K and tree depth, every right-hand side); the time of the pass only."""
    import numpy as np

    from oracle.cache import cached_taus, oracle_opset
    from oracle.fmm import fmm_apply
    from oracle.tree import build_structure

    sub = pts[:n_sample]
    fs = f[:, :n_sample].astype(np.complex128)
    st = build_structure(sub, K)
    # the oracle's skeletons at the plan's tau if they are cached, else at the
    # nearest cached tau (building them takes far longer than the timed pass)
    w_hi = max(1, st.w_top)
    have = cached_taus(w_hi)
    tau = eps_tau if (eps_tau in have or not have) else min(have, key=lambda t: abs(np.log(t / eps_tau)))
    ops = oracle_opset(tau, w_hi)
    t0 = time.perf_counter()
    fmm_apply(st, ops, fs)
    dt = time.perf_counter() - t0
    threads = None
    try:
        from threadpoolctl import threadpool_info

        threads = max(int(x.get("num_threads", 1)) for x in threadpool_info()) if threadpool_info() else 1
    except Exception:
        threads = os.cpu_count()
    model = None
    try:
        with open("/proc/cpuinfo") as fh:
            model = next((ln.split(":", 1)[1].strip() for ln in fh if ln.startswith("model name")), None)
    except OSError:
        pass
    return {
        "value": n_sample * fs.shape[0] / dt,
        "unit": "matvecs/s",
        "cores": threads,
        "cpu_model": model,
        "kind": "oracle",
        "sample": f"float64 oracle pass on the first {n_sample} of the {len(pts)} points of {workload} "
                  f"(same K={K:g}, tree depth {st.tree.D}, w_top {st.w_top}, {fs.shape[0]} rhs; the oracle's "
                  f"skeletons at tau={tau:.1e}), {dt:.2f} s; host has {os.cpu_count()} cores",
    }


def _log(msg: str) -> None:
    print(msg, file=sys.stderr, flush=True)


def serving_bench(args) -> int:
    """Continuous batching over 6 resident plans against the single-request form.

    Requests: plan uniform over the 6, nrhs uniform over {1, 4, 16}, complex64
    N(0, 1) densities (seed 505).  Both forms run the same plans (eps = 1e-4,
    float32 apply) on the same requests: first with every request queued at
    t = 0 (saturation throughput), then with Poisson arrivals at 0.5, 0.8 and
    0.95 of the single-request form's measured capacity (p50/p99 latency).
    """
    import numpy as np
    import torch

    from oracle.kernel import direct_sum, rel_l2
    from paper_1311_4257_amd import dfmm, workloads
    from paper_1311_4257_amd.serve import Request, Server, latency_stats

    dev = torch.device("cuda:0")
    eps = 1e-4 if args.eps is None else args.eps
    prec_b, dtype_b = PRECISIONS[args.precision]
    plans, bplans, names, pts_all, plan_s = [], [], [], [], []
    for name, kind, K, N, seed in workloads.SERVING_PLANS:
        pts = workloads.serving_points(kind, K, N, seed)
        t = time.perf_counter()
        plans.append(dfmm.Plan(pts, K, eps=eps, cache_dir=CACHE_DIR, device=0))
        plan_s.append(time.perf_counter() - t)
        # the batched form runs plans of its own precision (the same plans at fp32)
        bplans.append(plans[-1] if prec_b == 0 else
                      dfmm.Plan(pts, K, eps=eps, cache_dir=CACHE_DIR, device=0, precision=prec_b))
        names.append(name)
        pts_all.append(pts)
        _log(f"plan {name}: N={N} K={K:g} {plan_s[-1]:.2f} s")
    # accuracy of each plan alone against the direct sum (256 sampled targets)
    acc, acc_b = {}, {}
    for p, plan in enumerate(plans):
        f = workloads.densities(plan.N, 1, 600 + p)
        fd = torch.from_numpy(f.astype(np.complex64)).to(dev)
        tg = workloads.sample_targets(plan.N, 256, 700 + p)
        ref = direct_sum(pts_all[p], f, tg)
        acc[names[p]] = rel_l2(plan.apply(fd).cpu().numpy().astype(np.complex128)[:, tg], ref)
        acc_b[names[p]] = rel_l2(bplans[p].apply(fd).cpu().numpy().astype(np.complex128)[:, tg], ref)
        _log(f"accuracy {names[p]}: fp32 {acc[names[p]]:.2e}, batched form {acc_b[names[p]]:.2e}")

    n = args.requests
    pidx, nrhs, gaps = workloads.serving_mix(n, len(plans), 505)
    gen = torch.Generator(device=dev)
    gen.manual_seed(505)
    reqs = []
    for i in range(n):
        p, k = int(pidx[i]), int(nrhs[i])
        f = torch.complex(torch.randn((k, plans[p].N), generator=gen, device=dev),
                          torch.randn((k, plans[p].N), generator=gen, device=dev))
        reqs.append(Request(i, p, f, torch.empty_like(f), 0.0))
    work = sum(plans[r.plan].N * r.nrhs for r in reqs)
    budget = 200 << 30
    single = Server(plans, budget, mode="single")
    batched = Server(bplans, budget, max_batch_rhs=32, mode="batched")
    single.warm([1, 4, 16])
    batched.warm([1, 2, 4, 8, 16, 32])
    _log(f"warm: footprint {batched.footprint() / 2**30:.1f} GiB of {budget / 2**30:.0f} GiB")

    def run(srv, arrivals):
        for r, t in zip(reqs, arrivals):
            r.arrival, r.done = float(t), float("nan")
        span = srv.run(reqs)
        st = latency_stats(reqs)
        st["matvecs_per_s"] = work / span
        st["span_s"] = span
        st["passes"] = len(srv.batches)
        return st

    out_runs = {}
    zero = np.zeros(n)
    out_runs["saturation"] = {"single": run(single, zero), "batched": run(batched, zero)}
    _log(f"saturation: {json.dumps(out_runs['saturation'])}")
    # the same requests alone and in the mix: compare a sample of batched results
    diffs = []
    for r in reqs[:: max(1, n // 60)]:
        a = bplans[r.plan].apply(r.f)
        diffs.append(float(torch.linalg.norm(r.u - a) / torch.linalg.norm(a)))
    cap_req = n / out_runs["saturation"]["single"]["span_s"]
    loads = []
    for frac in (0.5, 0.8, 0.95):
        rate = frac * cap_req
        arr = np.cumsum(gaps) / rate
        arr -= arr[0]
        row = {"load": frac, "rate_req_per_s": rate, "single": run(single, arr), "batched": run(batched, arr)}
        loads.append(row)
        _log(f"load {frac}: {json.dumps(row)}")
    sat = out_runs["saturation"]
    line = {
        "metric": "FMM matvecs/s (N*nrhs/s) at 1e-4 rel err vs direct sum; p50/p99 serve latency",
        "value": sat["batched"]["matvecs_per_s"],
        "unit": "matvecs/s",
        "n_gpus": 1,
        "steps": n,
        "warmup": 0,
        "ms_per_step": sat["batched"]["span_s"] * 1e3 / n,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": dtype_b,
        "data": "synthetic",
        "config": {"workload": f"serving mix: {n} requests over 6 resident plans "
                               f"({', '.join(names)}), nrhs uniform over {{1, 4, 16}}, complex64 N(0,1) "
                               f"densities (seed 505), eps={eps:g}; value = continuous-batching throughput "
                               f"with every request queued at t=0",
                   "plans": [{"name": nm, "N": pl.N, "plan_s": round(ps, 3), "rel_l2_err_fp32": acc[nm],
                              "rel_l2_err_batched_form": acc_b[nm]}
                             for nm, pl, ps in zip(names, plans, plan_s)],
                   "single_form": "fp32, one request per pass, one pass at a time",
                   "batched_form": f"{args.precision}, continuous batching per plan, plans concurrent "
                                   "(the library's native request loop)",
                   "max_batch_rhs": 32, "hbm_budget_gib": budget / 2 ** 30},
        "serving": {
            "saturation": sat,
            "batched_over_single": sat["batched"]["matvecs_per_s"] / sat["single"]["matvecs_per_s"],
            "single_capacity_req_per_s": cap_req,
            "poisson_loads": loads,
            "mix_vs_alone_max_rel_diff": max(diffs),
            "footprint_gib": batched.footprint() / 2 ** 30,
        },
    }
    single.close()
    batched.close()
    print(json.dumps(line))
    return 0


def precision_study(args) -> int:
    """Error of each GEMM arithmetic against the float64 direct sum on the K = 32
    ellipsoid (N = 262,144, 8 right-hand sides, 4,096 sampled targets, seed 404)."""
    import numpy as np
    import torch

    from oracle.kernel import direct_sum, rel_l2
    from paper_1311_4257_amd import dfmm, workloads

    pts, _, cfg = workloads.make_config("ellipsoid32")
    K, N = cfg["K"], cfg["N"]
    nrhs = 8
    f = workloads.densities(N, nrhs, 404)
    tg = workloads.sample_targets(N, 4096, 404)
    t = time.perf_counter()
    ref = direct_sum(pts, f, tg)
    _log(f"direct sum on {len(tg)} targets: {time.perf_counter() - t:.1f} s")
    fd = torch.from_numpy(f.astype(np.complex64)).to("cuda:0")
    rows, u32 = {}, None
    for name in ("fp32", "fp16x3", "bf16x3"):
        prec, dtype = PRECISIONS[name]
        plan = dfmm.Plan(pts, K, eps=1e-4, cache_dir=CACHE_DIR, device=0, precision=prec)
        u = plan.apply(fd)
        torch.cuda.synchronize()
        t = time.perf_counter()
        for _ in range(args.steps):
            plan.apply(fd, u)
        torch.cuda.synchronize()
        ms = (time.perf_counter() - t) * 1e3 / args.steps
        un = u.cpu().numpy().astype(np.complex128)
        if u32 is None:
            u32 = un
        rows[name] = {"dtype": dtype, "rel_l2_err": rel_l2(un[:, tg], ref),
                      "max_rhs_rel_l2_err": max(rel_l2(un[k:k + 1, tg], ref[k:k + 1]) for k in range(nrhs)),
                      "rel_l2_diff_vs_fp32": rel_l2(un, u32), "ms_per_apply": ms,
                      "matvecs_per_s": N * nrhs / (ms * 1e-3)}
        _log(f"{name}: {json.dumps(rows[name])}")
        plan.close()
    print(json.dumps({"study": "precision", "workload": "ellipsoid32 (16, 8, 4), K=32, N=262144, nrhs=8, eps=1e-4, "
                      "4096 targets (seed 404) against the float64 direct sum", "results": rows}))
    return 0


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--calib-copy", action="store_true")
    ap.add_argument("--workload", default="ellipsoid32", choices=sorted(WORKLOADS),
                    help="the K=32 ellipsoid with 32 rhs (default, the headline line) or the K=16 sphere")
    ap.add_argument("--eps", type=float, default=None, help="plan eps (default: the workload's)")
    ap.add_argument("--leaf-max", type=int, default=0,
                    help="adaptive low-frequency tree: split boxes of width <= 1/2 holding more points "
                         "(0: the uniform tree)")
    ap.add_argument("--traffic-summary", nargs=2, metavar=("FETCH_DIR", "WRITE_DIR"))
    ap.add_argument("--serve", action="store_true", help="the serving mix instead of one workload")
    ap.add_argument("--precision", default="fp32", choices=sorted(PRECISIONS),
                    help="arithmetic of the translation GEMMs (fp32, or split 16-bit products)")
    ap.add_argument("--requests", type=int, default=2000, help="requests per serving run")
    ap.add_argument("--precision-study", action="store_true",
                    help="error per GEMM arithmetic on the K=32 ellipsoid with 8 rhs")
    args = ap.parse_args()
    if args.traffic_summary:
        rec = traffic_summary(*args.traffic_summary)
        rec["workload"] = args.workload
        with open(traffic_file(args.workload), "w") as fh:
            json.dump(rec, fh, indent=1)
        print(json.dumps(rec))
        return 0
    if args.gpus != 1:
        print("bench.py measures one GPU only: this build has no multi-GPU path "
              "(run with --gpus 1)", file=sys.stderr)
        return 2

    if args.serve:
        return serving_bench(args)
    if args.precision_study:
        return precision_study(args)

    import numpy as np
    import torch

    from paper_1311_4257_amd import dfmm, workloads

    pts, f, cfg = workloads.make_config(args.workload)
    if args.eps is not None:
        cfg["eps"] = args.eps
    K, N, nrhs, eps = cfg["K"], cfg["N"], cfg["nrhs"], cfg["eps"]
    dev = torch.device("cuda:0")
    prec, dtype = PRECISIONS[args.precision]
    plan = dfmm.Plan(pts, K, eps=eps, cache_dir=CACHE_DIR, device=0, precision=prec, leaf_max=args.leaf_max)
    info = plan.info()
    fd = torch.from_numpy(f.astype(np.complex64)).to(dev)
    u = torch.empty_like(fd)
    stream = torch.cuda.current_stream(dev)

    for _ in range(args.warmup):
        plan.apply(fd, u, stream)
    torch.cuda.synchronize()
    # the timed steps: nothing but the applies on the stream
    t0 = time.perf_counter()
    for _ in range(args.steps):
        plan.apply(fd, u, stream)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    # the same applies replayed from a HIP graph (one capture, K replays)
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        plan.apply(fd, u)
    graph.replay()
    torch.cuda.synchronize()
    tg0 = time.perf_counter()
    for _ in range(args.steps):
        graph.replay()
    torch.cuda.synchronize()
    ms_graph = (time.perf_counter() - tg0) * 1e3 / args.steps
    del graph
    # the same number of steps again with the stage events (timing-only HIP
    # events recorded on the apply stream between launches): per-kernel durations
    plan.set_timing(args.steps)
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    for _ in range(args.steps):
        plan.apply(fd, u, stream)
    torch.cuda.synchronize()
    ms_events = (time.perf_counter() - t2) * 1e3 / args.steps
    stages = plan.stage_times()
    plan.set_timing(0)
    if args.calib_copy:  # counter calibration: one plain copy of known size
        src = torch.empty(CALIB_BYTES // 4, dtype=torch.float32, device=dev).fill_(1.0)
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    ms = (t1 - t0) * 1e3 / args.steps

    # accuracy gate against the float64 direct sum
    from oracle.kernel import direct_sum, rel_l2

    tg = workloads.sample_targets(N, WORKLOADS[args.workload][1], cfg["check_seed"])
    t_ds = time.perf_counter()
    ref = direct_sum(pts, f, tg)
    t_ds = time.perf_counter() - t_ds
    err = rel_l2(u.cpu().numpy().astype(np.complex128)[:, tg], ref)

    m2l_ms = stages["hf_m2l"][0] + stages["lf_m2l"][0]
    m2l_launches = stages["hf_m2l"][1] + stages["lf_m2l"][1]
    per_apply = m2l_launches / max(1, args.steps)
    # slot form (from 16 rhs): one launch per level sums the level's M2L pairs and
    # its L2L terms into every incoming slot, and no reduction launches run
    slot_form = stages["hf_reduce"][1] == 0 and stages["lf_reduce"][1] == 0 and stages["lf_m2l"][1] > 0
    flops_apply = (info.flops_m2l_hf + info.flops_m2l_lf + (info.flops_l2l if slot_form else 0.0)) * nrhs
    bytes_apply = info.bytes_m2l_op + info.bytes_m2l_vec * nrhs
    if slot_form:  # the L2L terms' operators and parent slots
        bytes_apply += info.bytes_l2l_op + info.bytes_l2l_vec * nrhs
    sec = m2l_ms * 1e-3 / args.steps  # M2L launch time per apply
    # the bound is whichever ceiling is lower for these flops and bytes
    # a contraction is priced at the peak of its own MFMA dtype (16-bit plans: the
    # algorithmic flops, not the three hardware products per term)
    peak_mfma = PEAK_F16_MATRIX_TFLOPS if prec else PEAK_FP32_MATRIX_TFLOPS
    mfma_bound = flops_apply / (peak_mfma * 1e12) >= bytes_apply / (PEAK_HBM_GBS * 1e9)
    if mfma_bound:
        achieved, peak, unit = flops_apply / sec / 1e12, peak_mfma, "TFLOP/s"
    else:
        achieved, peak, unit = bytes_apply / sec / 1e9, PEAK_HBM_GBS, "GB/s"
    traffic = None
    tfile = traffic_file(args.workload)
    if os.path.exists(tfile):
        with open(tfile) as fh:
            rec = json.load(fh)
        # the record holds for the same GEMM sources, workload, eps, precision and
        # launch form (the counter runs use the workload's defaults)
        if rec.get("source_sha1") == gemm_source_hash() and args.eps is None and prec == 0 \
                and rec.get("launches") == round(per_apply):
            traffic = rec["bytes_per_launch"]
    per_stage = {k: round(v[0] / args.steps, 4) for k, v in stages.items() if v[1]}
    # near-field sum: point pairs (self pairs included, they contribute 0), flops
    # counted as 14 + 3 transcendentals per pair plus a complex MAC (8) per rhs
    nf_sec = stages["near_field"][0] * 1e-3 / args.steps
    nf_pairs = info.near_point_pairs
    nf_flops = nf_pairs * (17 + 8 * nrhs)
    near_kernel = "k_near_mfma" if (nrhs >= 4 and eps >= 1e-5) else "k_leaf_eval"
    near = {"kernel": f"{near_kernel} (near field, second stream, overlapping the far-field passes)",
            "point_pairs": nf_pairs, "ms": nf_sec * 1e3, "pairs_per_s": nf_pairs / nf_sec,
            "tflops": nf_flops / nf_sec / 1e12, "frac_fp32_vector_unpacked": nf_flops / nf_sec / 1e12 / 78.6,
            "frac_fp32_vector_packed": nf_flops / nf_sec / 1e12 / 157.3}

    eps_s = f"{eps:.0e}".replace("e-0", "e-")
    out = {
        "metric": f"FMM matvecs/s (N*nrhs/s) at {eps_s} rel err vs direct sum",
        "value": N * nrhs / (ms * 1e-3),
        "unit": "matvecs/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": dtype,
        "data": "synthetic",
        "config": {"workload": WORKLOADS[args.workload][0] + f", eps={eps_s}"
                               + (f", adaptive LF tree (leaf_max={args.leaf_max})" if args.leaf_max else ""),
                   "K": K, "N": N, "nrhs": nrhs, "eps": eps, "w_top": info.w_top,
                   "ranks": [int(info.rank[l]) for l in range(info.depth_max + 1)],
                   "leaves": int(info.leaves), "depth_max": int(info.depth_max)},
        "rel_l2_err": err,
        "accuracy_ok": bool(err <= eps),
        "stage_ms": per_stage,
        "ms_per_step_with_stage_events": ms_events,
        "ms_per_step_graph_replay": ms_graph,
        "roofline": {
            "bound": "mfma" if mfma_bound else "hbm",
            "kernel": ("k_m2l_slot (per level: every incoming slot sums its M2L pairs and L2L terms; "
                       "flops of both)" if slot_form else
                       "k_m2l_fused (every M2L level in one launch)" if stages["lf_m2l"][1] == 0 and per_apply == 1
                       else "k_m2l (grouped M2L GEMM, one launch per level)"),
            "achieved": achieved,
            "peak": peak,
            "unit": unit,
            "frac": achieved / peak,
            "traffic": traffic,
            "launches_per_apply": per_apply,
            "avg_launch_us": sec / max(1.0, per_apply) * 1e6,
            "flops_per_launch": flops_apply / max(1.0, per_apply),
            "alg_bytes_per_launch": bytes_apply / max(1.0, per_apply),
            "l2l_flops_per_apply": info.flops_l2l * nrhs,
            "m2m_flops_per_apply": info.flops_m2m * nrhs,
            "flops_per_level": {f"w={info.K / 2 ** l:g}": info.flops_m2l_level[l] * nrhs
                                for l in range(info.depth + 1) if info.flops_m2l_level[l] > 0},
        },
        "near_field": near,
        "plan_seconds": info.plan_seconds,
    }
    if not args.no_cpu_baseline:
        n_sample = {"sphere16": 16384, "ellipsoid32": 8192}[args.workload]
        out["cpu_baseline"] = cpu_baseline(pts, f, K, info.tau, args.workload, n_sample)
        # the float64 direct sum of the accuracy gate, on the same host
        out["cpu_baseline"]["direct_sum"] = {"targets": len(tg), "sources": N, "nrhs": nrhs,
                                             "seconds": t_ds, "pairs_per_s": len(tg) * N * nrhs / t_ds}
    print(json.dumps(out))
    return 0


if __name__ == "__main__":
    sys.exit(main())
