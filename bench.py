#!/usr/bin/env python
"""Benchmark of the near-field quadrature-correction generator on one GPU.

One step = one nfq_generate call over the whole workload: pair/work-queue
builder, patch preparation, self quadrature, adaptive near quadrature,
moments -> node weights, column indices.  Inputs (patch nodes, targets, near
lists) are resident in device memory before timing starts.

Workload: Helmholtz combined field D - ik S, k = 2 pi, unit sphere with 1280
quadratic patches at degree 4 (15 nodes, 19,200 on-surface targets), near
radius 1.25 R_j, tol 1e-8, complex128.  --workload times the generate step of
the full-size mixed-degree ellipsoid + torus (6000 patches, degrees 2..8) or
the 200,000-patch star surface (degree 6, tol 1e-9) instead.

Prints one JSON line (see the field list at the end of main()).
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "near-field target-points/s at tol 1e-8 (fwd; fwd+adjoint); % FP64 peak"
PEAK_FP64_TFLOPS = 78.6   # MI355X FP64 vector peak
# flops per kernel evaluation of the combined field (add/mul = 1, fma = 2,
# sqrt/div/sin/cos = 1), per moment of a complex-by-real MAC: 4
C_KERNEL = {"laplace": 12, "laplace_cplx": 18, "helmholtz": 40}


def kernel_flops(prob):
    if prob.k != 0:
        return C_KERNEL["helmholtz"]
    return C_KERNEL["laplace"] if prob.real_kernel else C_KERNEL["laplace_cplx"]


# workloads that bench.py can time; the first is the default bench line, the
# others are the full-size mixed-degree and 200,000-patch runs
WORKLOADS = {"cfie_sphere1280_d4": 1, "mixed_ellipsoid_torus": 2, "star200k_d6": 4}


def _oracle_rows(args):
    """Worker: whole rows (near + self blocks) of randomly chosen targets of the
    workload, oracle method mode, until `seconds` are spent.  Returns the
    number of rows done and the seconds taken."""
    seed, seconds, cfg = args
    import numpy as np
    import oracle
    from paper_2006_02545_amd import surfaces
    prob = surfaces.config(cfg)
    run = oracle.OracleRun(prob, mode=oracle.METHOD)
    order = np.random.default_rng(seed).permutation(prob.NT)
    done = 0
    t0 = time.perf_counter()
    for t in order:
        own = int(np.searchsorted(prob.node_ptr, t, side="right") - 1)
        for j in list(prob.near_patch[prob.near_row_ptr[t]:prob.near_row_ptr[t + 1]]) + [own]:
            run.pair(int(t), int(j))
        done += 1
        if time.perf_counter() - t0 >= seconds:
            break
    return done, time.perf_counter() - t0


def cpu_baseline(seconds, workers, cfg=1):
    """The oracle on the host: `workers` processes (one thread each), each on
    its own random sample of target rows for about `seconds`."""
    import multiprocessing as mp
    if workers <= 1:
        done, el = _oracle_rows((2024, seconds, cfg))
        rate = done / el
    else:
        with mp.get_context("spawn").Pool(workers) as pool:
            res = pool.map(_oracle_rows, [(2024 + i, seconds, cfg) for i in range(workers)])
        done = sum(r[0] for r in res)
        rate = sum(r[0] / r[1] for r in res)
        el = max(r[1] for r in res)
    cpu = "unknown CPU"
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    cpu = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return {"value": rate, "unit": "target-points/s", "cores": workers, "kind": "oracle",
            "sample": "%d random target rows of the same workload (near + self blocks), oracle "
                      "method mode, %d process(es) x 1 thread, %.1f s each, %s"
                      % (done, workers, el, cpu)}


# HBM traffic of the near kernel per launch on this workload, from two
# rocprofv3 --pmc passes (FETCH_SIZE, WRITE_SIZE in KiB per dispatch), scaled
# by the same counters on a plain 1 GiB copy kernel (bench.py
# --copy-calibration 1024: FETCH_SIZE reads 0.5 GiB, WRITE_SIZE 1 GiB), valid
# for the kernel sources with this digest.
TRAFFIC_RECORD = {
    "sources_sha256": "356cb9f19fe2f81c71736779fd27243997c37c3faefc319be5c16b44d664021e",
    "fetch_kib": 173119.0, "write_kib": 371788.6,
    "fetch_scale": 2.0, "write_scale": 1.0,
    # FP64 VALU wave instructions per launch (SQ_INSTS_VALU_{FMA,MUL,ADD,TRANS}_F64),
    # one rocprofv3 --pmc pass: hardware-counted flops = 64 lanes x (2 FMA + MUL
    # + ADD + TRANS)
    "fma_f64": 724992720, "mul_f64": 315824200, "add_f64": 142378440, "trans_f64": 6997280, "valu": 2007371962,
}
NEAR_SOURCES = ["near_patch.hpp", "kernels.hpp", "device.hpp", "fastmath.hpp", "koorn.hpp"]


def near_sources_digest():
    import hashlib
    h = hashlib.sha256()
    for f in NEAR_SOURCES:
        with open(os.path.join(ROOT, "paper_2006_02545_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def near_hw_flops():
    """Hardware-counted FP64 flops of one near-kernel launch, or None when the
    counters were taken on other kernel sources."""
    r = TRAFFIC_RECORD
    if r["sources_sha256"] != near_sources_digest():
        return None
    return 64.0 * (2.0 * r["fma_f64"] + r["mul_f64"] + r["add_f64"] + r["trans_f64"])


def near_traffic():
    if TRAFFIC_RECORD["sources_sha256"] != near_sources_digest():
        return None
    r = TRAFFIC_RECORD
    return (r["fetch_kib"] * r["fetch_scale"] + r["write_kib"] * r["write_scale"]) * 1024.0


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--cpu-workers", type=int, default=0,
                    help="oracle processes for cpu_baseline (default: min(16, cpu count))")
    ap.add_argument("--print-digest", action="store_true",
                    help="print the digest of the near-kernel sources and exit")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--workload", default="cfie_sphere1280_d4", choices=list(WORKLOADS),
                    help="workload to time (default: the bench line's); the others time the "
                         "generate step only")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="only run a plain device copy of MIB MiB five times (the known-size "
                         "kernel that scales the FETCH_SIZE / WRITE_SIZE counters) and exit")
    args = ap.parse_args()
    if args.print_digest:
        print(near_sources_digest())
        return
    if args.copy_calibration:
        import torch
        n = args.copy_calibration << 20
        src = torch.ones(n // 4, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(5):
            torch.mul(src, 1.0, out=dst)   # one elementwise kernel: reads n bytes, writes n
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_read": n, "copy_bytes_written": n, "launches": 5}))
        return
    if args.gpus != 1:
        print("bench.py runs on one GPU only: this build measures the generator on a single "
              "MI355X (the multi-GPU row sharding is described in DESIGN.md, not built)",
              file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2006_02545_amd import nfq, surfaces

    main_line = args.workload == "cfie_sphere1280_d4"
    prob = surfaces.config(WORKLOADS[args.workload])
    torch.cuda.set_device(0)
    ctx = nfq.Context(0)
    plan = nfq.plan_for(ctx, prob)
    col = torch.empty(plan.nnz, dtype=torch.int32, device="cuda")
    val = torch.empty(plan.nnz, dtype=torch.complex128, device="cuda")
    gen = dict(alpha=prob.alpha, beta=prob.beta, k=prob.k, tol=prob.tol, col=col, val=val)

    for _ in range(args.warmup):
        plan.generate(stats=False, **gen)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        plan.generate(stats=False, **gen)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ms = (t1 - t0) / args.steps * 1e3
    value = prob.NT / (ms * 1e-3)

    # the same generate captured once in a HIP graph and replayed (a plan of
    # its own, on the capture stream); per-replay durations from events
    graph = None
    try:
        if not main_line:
            raise StopIteration
        gs = torch.cuda.Stream()
        ctx_g = nfq.Context(0, stream=gs)
        plan_g = nfq.plan_for(ctx_g, prob)
        col_g = torch.empty_like(col)
        val_g = torch.empty_like(val)
        gen_g = dict(gen, col=col_g, val=val_g, stats=False)
        with torch.cuda.stream(gs):
            plan_g.generate(**gen_g)
        torch.cuda.synchronize()
        gr = torch.cuda.CUDAGraph()
        with torch.cuda.graph(gr, stream=gs):
            plan_g.generate(**gen_g)
        torch.cuda.synchronize()
        times = []
        for _ in range(max(10, args.steps)):
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            with torch.cuda.stream(gs):
                e0.record(gs)
                gr.replay()
                e1.record(gs)
            e1.synchronize()
            times.append(e0.elapsed_time(e1))
        times.sort()
        med = times[len(times) // 2]
        same = bool(torch.equal(val_g.view(torch.float64), val.view(torch.float64)))
        graph = {"value": prob.NT / (med * 1e-3), "unit": "target-points/s", "ms_median": med,
                 "replays": len(times), "matches_eager": same}
        del gr
    except StopIteration:        # timed on the default workload only
        graph = None
    except RuntimeError as exc:  # capture refused: report, keep the eager figures
        graph = {"error": str(exc)[:200]}

    # forward + adjoint: generate, apply and the adjoint (gradient of
    # conj(lambda)^T A sigma wrt node coordinates, k, alpha, beta)
    sig_t = torch.as_tensor(prob.sigma, dtype=torch.complex128, device="cuda")
    lam_t = torch.as_tensor(prob.lam, dtype=torch.complex128, device="cuda")
    grad = torch.empty((prob.N, 3), dtype=torch.complex128, device="cuda")
    gk = torch.empty(1, dtype=torch.complex128, device="cuda")
    dab = torch.empty(2, dtype=torch.complex128, device="cuda")

    def fwd_adj():
        plan.generate(stats=False, **gen)
        plan.apply(col, val, sig_t)
        plan.adjoint_into(prob.alpha, prob.beta, prob.k, prob.tol, sig_t, lam_t, grad, gk, dab)

    nfa = max(1, args.steps // 2) if main_line else 0
    ms_fa = None
    if nfa:
        fwd_adj()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(nfa):
            fwd_adj()
        torch.cuda.synchronize()
        ms_fa = (time.perf_counter() - t0) / nfa * 1e3

    # the plain per-pair GPU path (one wavefront per pair, no reuse of
    # subtriangle geometry across targets) on the same workload
    npp = max(1, args.steps // 2) if main_line else 0
    ms_pp = None
    if npp:
        for _ in range(2):
            plan.generate(stats=False, per_pair=True, **gen)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(npp):
            plan.generate(stats=False, per_pair=True, **gen)
        torch.cuda.synchronize()
        ms_pp = (time.perf_counter() - t0) / npp * 1e3

    # the GPU near-list builder on the same surface and targets (not part of
    # the step: the generator takes the lists as input)
    near_builder = None
    if main_line:
        args_nl = (prob.degree, prob.node_ptr, prob.xyz, prob.target_xyz, prob.node_of_target,
                   prob.eta)
        dev_args = [torch.as_tensor(a, device="cuda") if not isinstance(a, float) else a
                    for a in args_nl]
        ctx.near_lists(*dev_args)
        torch.cuda.synchronize()
        reps = 5
        t0 = time.perf_counter()
        for _ in range(reps):
            nl_rp, _, _, _ = ctx.near_lists(*dev_args)
        torch.cuda.synchronize()
        near_builder = {"ms": (time.perf_counter() - t0) / reps * 1e3,
                        "pairs": int(nl_rp[-1].item()), "reps": reps,
                        "what": "nfq_near_lists: balls, grid, count + fill + sort (two calls)"}

    # per-phase durations from HIP events recorded on the library's stream
    phases = {k: 0.0 for k in ("ms_builder", "ms_prep", "ms_self", "ms_near", "ms_weights")}
    st = None
    nrep = max(1, min(args.steps, 5))
    for _ in range(nrep):
        _, _, st = plan.generate(stats=True, timing=True, **gen)
        for k in phases:
            phases[k] += st[k] / nrep
    roofline = None
    degs = sorted(set(int(d) for d in prob.degree))
    if len(degs) == 1:
        nd = (degs[0] + 1) * (degs[0] + 2) // 2
        nq = 64
        # algorithmic flops of the adaptive near kernel (dominant): every
        # subtriangle visit of every pair evaluates the kernel at nq nodes and
        # accumulates nd complex moments
        flops_near = st["visits"] * nq * (kernel_flops(prob) + 4 * nd)
        achieved = flops_near / (phases["ms_near"] * 1e-3) / 1e12
        roofline = {"bound": "alu", "kernel": "k_near (adaptive near quadrature)",
                    "achieved": achieved, "peak": PEAK_FP64_TFLOPS, "unit": "TFLOP/s",
                    "frac": achieved / PEAK_FP64_TFLOPS,
                    "traffic": near_traffic() if main_line else None,
                    "flops_per_launch": flops_near, "ms_per_launch": phases["ms_near"]}
        if roofline["traffic"] is not None:
            roofline["hbm_gbps"] = roofline["traffic"] / (phases["ms_near"] * 1e-3) / 1e9
            roofline["hbm_frac"] = roofline["hbm_gbps"] / 8000.0
        hw = near_hw_flops() if main_line else None
        if hw is not None:
            roofline["hw_counted"] = {"flops_per_launch": hw,
                                      "tflops": hw / (phases["ms_near"] * 1e-3) / 1e12,
                                      "frac": hw / (phases["ms_near"] * 1e-3) / 1e12 / PEAK_FP64_TFLOPS}
    out = {
        "metric": METRIC,
        "value": value,
        "unit": "target-points/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "complex128",
        "data": "synthetic",
        "config": {"workload": args.workload, "patches": prob.P,
                   "degree": degs[0] if len(degs) == 1 else "%d..%d" % (degs[0], degs[-1]),
                   "targets": prob.NT, "near_pairs": int(prob.near_patch.size),
                   "kernel": "D - ik S", "k": prob.k.real, "tol": prob.tol, "eta": prob.eta,
                   "loosen": 1.0, "global_batch": prob.NT, "parallelism": "single-gpu"},
        "fwd_adjoint": None if ms_fa is None else {
            "value": prob.NT / (ms_fa * 1e-3), "unit": "target-points/s", "ms_per_step": ms_fa,
            "steps": nfa, "step": "generate + apply + adjoint (gradient wrt nodes, k, alpha, beta)"},
        "per_pair_path": None if ms_pp is None else {
            "value": prob.NT / (ms_pp * 1e-3), "unit": "target-points/s", "ms_per_step": ms_pp,
            "steps": npp},
        "graph_replay": graph,
        "near_list_builder": near_builder,
        "phase_ms": phases,
        "gen_stats": {k: st[k] for k in ("near_pairs", "self_pairs", "visits", "checks",
                                         "nonconverged", "max_level")},
        "roofline": roofline,
    }
    if not args.no_cpu_baseline:
        workers = args.cpu_workers or max(1, min(16, os.cpu_count() or 1))
        out["cpu_baseline"] = cpu_baseline(args.cpu_seconds, workers, WORKLOADS[args.workload])
    print(json.dumps(out))


if __name__ == "__main__":
    main()
