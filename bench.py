"""Benchmark of the MF-CIM L0RBCS hot path on one MI355X.

Default (--form batched): the largest single-GPU workload, 256 uneven
Gaussian instances (N log-uniform in [256, 4096], alpha U[0.3, 0.7],
sparsity U[0.05, 0.2], noise 0.01), 16 replicas each, 1000 Euler steps x 30
alternations, FP32 couplings, one matrix-core launch per Euler step over all
instances.  One step = one alternation of Algorithm 1 over the whole batch;
30 steps make one batched solve.  Inputs are resident in HBM before the timed
region starts.  value = spin-steps/s of the timed steps, scaled by the
fraction of 16 sampled instances whose final support equals the FP64
oracle's stored support (tests/golden/oracle_supports_batched.txt).
Prints one JSON line.

--form selects the other forms of the method (one JSON line each):
  plain      one instance, N = 2000, M = 1000, one replica, 2000 steps x 30
             alternations, FP32 (one step = one whole solve);
  precision  the MRI-shaped instance (N = 16384, M = 4915), 64 replicas,
             BF16 or FP8 couplings (--jdtype), FP64 refit, 1000 x 11, or the
             couplings applied in factored form (--jdtype factored), or the
             paper's MRI pipeline around it (--jdtype pipeline: L2 term,
             LASSO start, CG CDP);
  serving    a stream of Gaussian requests (N log-uniform in [512, 8192]),
             8 replicas, 1000 x 30, served by the continuous-batching server
             at saturation and at Poisson arrival rates below it, beside the
             single-instance path serving the same requests one at a time;
  accuracy   the paper's random-data accuracy studies on the device path:
             RMSE vs sparseness (alpha 0.6 / 0.8, noise 0.05 / 0.1, CN and
             BN), tau = 0.15 beside tau = 1, per-alternation RMSE and Hamming
             loss, late-time amplitudes; the FP64 oracle repeats a few solves.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "MF-CIM spin-steps/s & %roofline at oracle support match; p50/p99 solve latency"
HBM_PEAK_GBS = 8000.0
FP32_VECTOR_PEAK_TFS = 157.3
N, M, STEPS, OUTER, P = 2000, 1000, 2000, 30, 1
WORKLOAD = ("plain Gaussian L0RBCS: N=2000, M=1000 (alpha 0.5), Bernoulli(0.1) support, N(0,1) values, "
            "A iid N(0,1/M), noise std 0.01, 1 replica, 2000 Euler steps x 30 alternations, "
            "eta 0.8->0.18 (velo 30), Jacobi CDP 100 sweeps, FP32 couplings")


TRAFFIC_FILE = os.path.join(ROOT, "profiles", "cim_regs_kernel_plain_n2000_traffic.txt")
KERNEL_SOURCES = ("mfcim.hip", "common.h")
PRECISION_TRAFFIC_FILES = {dt: os.path.join(ROOT, "profiles", f"bstep_kernel_mri_{dt}_traffic.txt")
                           for dt in ("bf16", "fp8")}
PRECISION_SOURCES = ("batch.hip", "batch.h", "mfcim_matrix.hip")
BATCHED_TRAFFIC_FILE = os.path.join(ROOT, "profiles", "bstep_kernel_batched_256x16_traffic.txt")
BATCHED_SOURCES = ("batch.hip", "batch.h", "batch_plan.hip")


def kernel_source_hash(sources=KERNEL_SOURCES) -> str:
    h = hashlib.sha256()
    for f in sources:
        with open(os.path.join(ROOT, "paper_2405_00366_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def measured_traffic(path=TRAFFIC_FILE, sources=KERNEL_SOURCES, key="hbm_bytes_per_launch"):
    """HBM bytes per launch of a kernel from its committed counter summary, or
    None when the kernel sources changed since the counters were taken."""
    if not os.path.exists(path):
        return None
    kv = {}
    for line in open(path):
        if ":" in line and not line.startswith("#"):
            k, v = line.split(":", 1)
            kv[k.strip()] = v.strip()
    if kv.get("source_sha256") != kernel_source_hash(sources) or key not in kv:
        return None
    return float(kv[key])


def traffic_probe(torch, dev):
    """Known-size fill and copy (512 MiB each way) that calibrate the HBM
    byte counters against the kernels of the workload in the same run."""
    a = torch.empty(1 << 27, dtype=torch.float32, device=dev)
    a.fill_(1.0)
    b = torch.empty_like(a)
    b.copy_(a)
    torch.cuda.synchronize()
    del a, b


def golden_supports():
    path = os.path.join(ROOT, "tests", "golden", "oracle_supports_plain.txt")
    out = {}
    if os.path.exists(path):
        for line in open(path):
            if line.strip() and line[0] != "#":
                s, k, rm, hx = line.split()
                out[int(s)] = int(hx, 16)
    return out


def mask_to_int(sig) -> int:
    v = 0
    for r in np.flatnonzero(sig):
        v |= 1 << int(r)
    return v


def cpu_baseline(seconds_target: float = 12.0):
    """The FP64 oracle on the host: a bounded sample of the same workload
    (whole solves of seeds 0, 1, ... until about `seconds_target` of CPU work;
    the first alternations of seed 0 when one solve alone is longer)."""
    from threadpoolctl import threadpool_info

    import workloads as W
    from oracle import mfcim as O

    cores = len(os.sched_getaffinity(0))
    cim = O.CimParams(n_steps=STEPS)

    def timed(seed, n_alt):
        inst = W.plain_gaussian(seed).rounded_f32()
        outer = O.OuterParams(eta_init=0.8, eta_end=0.18, velo=OUTER, n_outer=n_alt, seed=seed)
        t1 = time.perf_counter()
        O.solve(inst.A, inst.y, cim, outer, keep_history=False)
        return time.perf_counter() - t1

    dt = timed(0, 1)
    if dt * OUTER > seconds_target:
        done = max(1, int(seconds_target / dt))
        dt = timed(0, done)
        steps, sample = done * STEPS, f"seed 0, first {done} of {OUTER} alternations"
    else:
        dt, seeds = 0.0, 0
        while dt < seconds_target and seeds < 20:
            dt += timed(seeds, OUTER)
            seeds += 1
        steps, sample = seeds * OUTER * STEPS, f"{seeds} whole solves (seeds 0-{seeds - 1})"
    threads = max([i.get("num_threads", 1) for i in threadpool_info()] or [1])
    # the same oracle with its BLAS on one thread, on a shorter sample
    from threadpoolctl import threadpool_limits
    with threadpool_limits(limits=1):
        n1 = 1
        d1 = timed(0, n1)
        while d1 < seconds_target / 3 and n1 < OUTER:
            n1 = min(OUTER, 2 * n1)
            d1 = timed(0, n1)
    return {"value": N * P * steps / dt, "unit": "spin-steps/s", "cores": int(min(threads, cores)),
            "kind": "oracle",
            "sample": f"{sample} of the same workload ({steps} Euler steps, FP64 NumPy), {dt:.1f} s",
            "value_1_thread": N * P * n1 * STEPS / d1,
            "sample_1_thread": f"seed 0, first {n1} of {OUTER} alternations with BLAS on one thread, {d1:.1f} s"}


def step_bytes(n: int, P: int, jbytes: int) -> int:
    """Algorithmic HBM bytes of one Euler step of one instance: the couplings
    once, amplitudes and error variables read and written, z and row scale."""
    return n * n * jbytes + 16 * P * n + 8 * n


def percentiles(v):
    return float(np.percentile(v, 50)), float(np.percentile(v, 99))


BATCH_SEED, BATCH_COUNT, BATCH_P, BATCH_STEPS, BATCH_OUTER = 7, 256, 16, 1000, 30
SERVE_HOST_REQUESTS = 200
BATCH_WORKLOAD = ("batched Gaussian L0RBCS: 256 instances (batch seed 7), N log-uniform [256, 4096], alpha U[0.3, 0.7], "
                  "sparsity U[0.05, 0.2], N(0,1) values, A iid N(0,1/M), noise std 0.01, 16 replicas each, "
                  "1000 Euler steps x 30 alternations, eta 0.8->0.18 (velo 30), Jacobi CDP 100 sweeps, FP32 "
                  "couplings, one matrix-core launch per Euler step over all instances (HIP graph replay)")


def golden_file(name):
    """Stored oracle results tests/golden/oracle_supports_<name>.txt:
    key -> (support bitmask, support size, RMSE against the truth)."""
    path = os.path.join(ROOT, "tests", "golden", f"oracle_supports_{name}.txt")
    out = {}
    if os.path.exists(path):
        for line in open(path):
            if line.strip() and line[0] != "#":
                k, sz, rm, hx = line.split()
                out[int(k)] = (int(hx, 16), int(sz), float(rm))
    return out


def oracle_threads():
    from threadpoolctl import threadpool_info
    threads = max([i.get("num_threads", 1) for i in threadpool_info()] or [1])
    return int(min(threads, len(os.sched_getaffinity(0))))


def calibrated_steps(timed, n0: int, n_max: int, seconds_target: float):
    """Pick the Euler step count of a bounded oracle sample: time n0 and 3 n0
    steps, fit t = a + b n (a: the per-sample set-up such as Gram prep and
    CDP), and take the n that lands near `seconds_target` (capped at n_max).
    Returns (n, seconds at n)."""
    t1 = timed(n0)
    t3 = timed(3 * n0)
    per = max((t3 - t1) / (2 * n0), 1e-6)
    fixed = max(t1 - n0 * per, 0.0)
    n = int(max(n0, min(n_max, (seconds_target - fixed) / per)))
    return n, timed(n)


def batched_cpu_baseline(W, specs, sample, P, seconds_target: float = 15.0):
    """The FP64 oracle on a bounded sample of the batched workload: the first
    alternation of every sampled instance (every 16th of the batch, so the
    sample spans the size range), with the Euler step count cut so that the
    whole sample takes about `seconds_target` seconds."""
    from oracle import mfcim as O

    insts = {k: specs[k].build().rounded_f32() for k in sample}

    def timed(n_steps):
        t = time.perf_counter()
        for k in sample:
            cim = O.CimParams(n_steps=n_steps)
            outer = O.OuterParams(eta_init=0.8, eta_end=0.18, velo=BATCH_OUTER, n_outer=1, replicas=P,
                                  seed=specs[k].seed)
            O.solve(insts[k].A, insts[k].y, cim, outer, keep_history=False)
        return time.perf_counter() - t

    n, dt = calibrated_steps(timed, 20, BATCH_STEPS, seconds_target)
    spin = sum(specs[k].N for k in sample) * P * n
    return {"value": spin / dt, "unit": "spin-steps/s", "cores": oracle_threads(), "kind": "oracle",
            "sample": f"first alternation ({n} of {BATCH_STEPS} Euler steps, Gram prep, replica choice and "
                      f"Jacobi CDP included) of {len(sample)} sampled instances (every 16th of the batch, "
                      f"sum N = {sum(specs[k].N for k in sample)}), 16 replicas, FP64 NumPy, {dt:.1f} s"}


def batched_bench(args, torch, L, W, dev):
    """Default benchmark: the batched form on the largest single-GPU workload.

    One step = one alternation of Algorithm 1 over all 256 instances and
    their 16 replicas (couplings, initial state, the 1000-step CIM run as one
    HIP-graph replay of 1001 matrix-core launches, replica choice, 100
    Jacobi sweeps).  The solves run back to back: the first step of each
    solve also forms G, b and R_init of every instance (l0cim_batch_begin),
    the last one also writes the eq. 3 objective (l0cim_batch_finish), so
    30 consecutive steps are exactly one whole batched solve.  After the
    timed steps the open solve is completed untimed and the final supports
    of the 16 sampled instances are compared with the oracle's stored ones."""
    P, steps, outer = BATCH_P, args.euler_steps or BATCH_STEPS, args.alternations or BATCH_OUTER
    specs = W.batch_specs(BATCH_SEED, BATCH_COUNT)
    print(f"[batched] building {len(specs)} instances", file=sys.stderr, flush=True)
    insts = [sp.build() for sp in specs]
    descr, A, y, R, sig, stats = L.pack_instances([i.A for i in insts], [i.y for i in insts],
                                                  [sp.seed for sp in specs], device=dev)
    cim = L.cim_params(n_steps=steps)
    flags = L.SOLVE_NO_GRAPH if args.no_graph else 0
    sp = L.solve_params(eta_init=0.8, eta_end=0.18, velo=outer, n_outer=outer, replicas=P, j_dtype=L.F32,
                        flags=flags)
    plan = L.l0cim_batch_plan_create(descr, cim, sp)
    ws = L.workspace(L.l0cim_batch_plan_workspace_bytes(plan), dev)
    stream = torch.cuda.current_stream()
    # tile tuning for this shape class, outside every timed region
    warm = L.solve_params(eta_init=0.8, eta_end=0.18, velo=outer, n_outer=1, replicas=P, j_dtype=L.F32, flags=flags)
    wplan = L.l0cim_batch_plan_create(descr, L.cim_params(n_steps=min(steps, 20)), warm)
    L.l0cim_solve_batched(wplan, A, y, R, sig, stats, ws)
    torch.cuda.synchronize()
    L.l0cim_batch_plan_destroy(wplan)
    pools = (A, y, R, sig, stats, ws)
    state = {"alt": 0, "solve_ev": []}

    def step():
        a = state["alt"]
        if a == 0:
            ev = torch.cuda.Event(enable_timing=True)
            ev.record(stream)
            state["solve_ev"].append([ev, None])
            L.l0cim_batch_begin(plan, *pools)
        L.l0cim_batch_alternations(plan, a, a + 1, *pools)
        if a == outer - 1:
            L.l0cim_batch_finish(plan, *pools)
            ev = torch.cuda.Event(enable_timing=True)
            ev.record(stream)
            state["solve_ev"][-1][1] = ev
        state["alt"] = (a + 1) % outer

    print(f"[batched] {args.warmup} warm-up steps", file=sys.stderr, flush=True)
    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(args.steps + 1)]
    L.l0cim_profile_begin()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ev[0].record(stream)
    for k in range(args.steps):
        step()
        ev[k + 1].record(stream)
        if (k + 1) % 5 == 0:
            print(f"[batched] {k + 1}/{args.steps} steps enqueued", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    cim_ms, launches = L.l0cim_profile_end()
    gpu_ms = ev[0].elapsed_time(ev[-1])
    step_ms = [ev[k].elapsed_time(ev[k + 1]) for k in range(args.steps)]
    print(f"[batched] timed {args.steps} steps in {wall:.2f} s; completing the open solve", file=sys.stderr,
          flush=True)
    while state["alt"] != 0:
        step()
    torch.cuda.synchronize()
    solve_ms = [a.elapsed_time(b) for a, b in state["solve_ev"] if b is not None]
    rows, tiles, _ = L.l0cim_batch_plan_info(plan)
    L.l0cim_batch_plan_destroy(plan)

    # the sampled instances against the oracle's stored supports
    st = L.read_stats_array(stats, len(descr))
    gold = golden_file("batched")
    sample = sorted(gold) if (steps, outer) == (BATCH_STEPS, BATCH_OUTER) else []
    sig_h = sig.cpu().numpy()
    R_h = R.double().cpu().numpy()
    match, drmse, per = 0, 0.0, []
    for k in sample:
        o = int(descr[k].x_offset)
        n = specs[k].N
        s_k = sig_h[o:o + n]
        ok = mask_to_int(s_k) == gold[k][0]
        rm = float(np.sqrt(np.mean((R_h[o:o + n] * s_k - insts[k].x * insts[k].xi) ** 2)))
        match += int(ok)
        drmse = max(drmse, abs(rm - gold[k][2]))
        per.append({"instance": k, "N": n, "support": int(s_k.sum()), "oracle_support": gold[k][1],
                    "identical": bool(ok), "rmse": rm, "oracle_rmse": gold[k][2]})
    sum_n = sum(s.N for s in specs)
    spin_per_step = sum_n * P * steps
    elapsed = max(wall, gpu_ms / 1e3)
    frac_match = match / len(sample) if sample else 0.0
    run_bytes = sum(step_bytes(s.N, P, 4) for s in specs)
    launch_s = cim_ms / 1e3 / max(launches, 1) / (steps + 1)
    achieved = run_bytes / launch_s / 1e9
    out = {
        "metric": METRIC, "value": spin_per_step * args.steps * frac_match / elapsed, "unit": "spin-steps/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": elapsed * 1e3 / args.steps,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": BATCH_WORKLOAD, "step": "one alternation of Algorithm 1 over the whole batch "
                   "(30 steps = one batched solve; Gram prep in the first, eq. 3 objective in the last)",
                   "instances": len(specs), "sum_N": sum_n, "sum_N2": sum(s.N ** 2 for s in specs),
                   "replicas": P, "euler_steps": steps, "alternations": outer,
                   "rows_per_tile": rows, "tiles": tiles},
        "support_match": f"{match}/{len(sample)} sampled instances (every 16th) identical to the FP64 oracle",
        "value_note": "spin-steps/s of the timed steps times the fraction of sampled instances whose final "
                      "support equals the oracle's",
        "spin_steps_per_s_all": spin_per_step * args.steps / elapsed,
        "max_abs_rmse_diff_vs_oracle": drmse if sample else None,
        "per_instance": per,
        "step_ms_p50": float(np.percentile(step_ms, 50)), "step_ms_p99": float(np.percentile(step_ms, 99)),
        "solve_latency_ms": solve_ms,
        "status_nonzero": sum(1 for x in st if x.status_bits),
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS,
                     "traffic": measured_traffic(BATCHED_TRAFFIC_FILE, BATCHED_SOURCES, "hbm_bytes_per_step"),
                     "kernel": "bstep_kernel<float, CN, 1, rb>",
                     "algorithmic_bytes_per_launch": run_bytes,
                     "avg_launch_ms": launch_s * 1e3, "launches": launches * (steps + 1),
                     "timing": "HIP events around each graph replay of one CIM run (n_steps + 1 launches) on "
                               "the launch stream, averaged per launch"},
    }
    if not args.no_cpu:
        print("[batched] CPU oracle baseline", file=sys.stderr, flush=True)
        out["cpu_baseline"] = batched_cpu_baseline(W, specs, list(range(0, BATCH_COUNT, 16)), P)
    return out


def factored_many_bench(args, torch, L, WM, dev, P, steps, outer):
    """The factored MRI form with K = --instances instances per step: one
    l0cim_mri_solve_many call solves K seeds (K x 64 workgroups, so that K = 4
    fills the 256 CUs).  value counts every instance's spin-steps."""
    K = args.instances
    pipeline = args.jdtype == "pipeline"
    gold, gold_R = mri_golden()
    if pipeline:
        gold = {k: (v[0], v[2]) for k, v in golden_file("mri_l2").items()}
    seeds = list(range(args.steps * K))
    cim = L.cim_params(n_steps=steps, field="BN", K=1.0, d=0.6)
    n = 128 * 128
    rows, total, cim_total, launches_total, match = [], 0.0, 0.0, 0, 0
    for g in range(args.steps):
        sds = seeds[g * K:(g + 1) * K]
        print(f"[factored x{K}] building the MRI-shaped instances of seeds {sds}", file=sys.stderr, flush=True)
        insts = [WM.mri_instance(sd) for sd in sds]
        if g == 0:
            factored_many_solve(torch, L, insts, dev, L.cim_params(n_steps=4, field="BN", K=1.0, d=0.6), P, 1, sds,
                                pipeline)
        print(f"[factored x{K}] solving ({outer} x {steps} steps)", file=sys.stderr, flush=True)
        L.l0cim_profile_begin()
        R, sel, status, dt = factored_many_solve(torch, L, insts, dev, cim, P, outer, sds, pipeline)
        ms, cnt = L.l0cim_profile_end()
        total += dt
        cim_total += ms
        launches_total += cnt
        sig_all = sel.cpu().numpy()
        R_all = R.double().cpu().numpy()
        for k, sd in enumerate(sds):
            sig, Rv, inst = sig_all[k], R_all[k], insts[k]
            rmse = float(np.sqrt(np.mean((Rv * sig - inst.x * inst.xi) ** 2)))
            ok = sd in gold and mask_to_int(sig) == gold[sd][0] and (steps, outer) == (1000, 11)
            match += int(ok)
            rows.append({"seed": sd, "support": int(sig.sum()), "rmse": rmse,
                         "oracle_rmse": gold[sd][1] if sd in gold else None, "oracle_support_match": ok,
                         "status": status[k]})
        print(f"[factored x{K}] seeds {sds}: {dt:.3f} s", file=sys.stderr, flush=True)
    spin_steps = n * P * steps * outer * len(seeds)
    run_ms = cim_total / launches_total
    flops = mri_flops_per_replica_step() * P * K * steps
    achieved = flops / (run_ms / 1e3) / 1e12
    return {
        "metric": METRIC, "value": spin_steps / total, "unit": "spin-steps/s", "n_gpus": 1, "steps": args.steps,
        "warmup": 1, "ms_per_step": total * 1e3 / args.steps, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": f"{K} MRI-shaped instances per step (seeds as listed, each its own phantom and "
                               "frequency mask), 128x128, 3-level Haar (N=16384), M=4915, 64 replicas each, BN field, "
                               "eta 0.8->0.03 over 11 alternations of 1000 steps, factored FP32 couplings, " +
                               ("MRI pipeline (L2 term, LASSO start, CG CDP)" if pipeline else
                                "Jacobi CDP in factored form, FP64 Cholesky refit") +
                               "; one l0cim_mri_solve_many call per step", "instances": K},
        "couplings": "factored" + (" + MRI pipeline" if pipeline else ""),
        "support_match": f"{match}/{len(seeds)}", "per_seed": rows,
        "spin_steps_per_s_cim_only": n * P * K * steps * launches_total / (cim_total / 1e3),
        "roofline": {"bound": "alu", "achieved": achieved, "peak": FP32_VECTOR_PEAK_TFS, "unit": "TFLOP/s",
                     "frac": achieved / FP32_VECTOR_PEAK_TFS, "traffic": None, "kernel": "mri_cim_kernel<BN>",
                     "flops_per_replica_step": mri_flops_per_replica_step(), "workgroups": K * P,
                     "avg_launch_ms": run_ms, "us_per_step": run_ms * 1e3 / steps},
    }


CAC_P, CAC_STEPS, CAC_OUTER = 8, 1000, 30


def cac_cpu_baseline(W, seed: int = 0, seconds_target: float = 12.0):
    """The FP64 CAC-CIM oracle on a bounded sample of the CAC workload: the
    first alternation of seed 0 (Gram prep, replica choice and Jacobi CDP
    included), Euler step count cut so that it takes about `seconds_target`."""
    from oracle import cac as C, mfcim as O

    inst = W.plain_gaussian(seed).rounded_f32()

    def timed(n_steps):
        t = time.perf_counter()
        outer = O.OuterParams(eta_init=0.8, eta_end=0.18, velo=CAC_OUTER, n_outer=1, replicas=CAC_P, seed=seed)
        C.solve(inst.A, inst.y, C.CacParams(n_steps=n_steps), outer, keep_history=False)
        return time.perf_counter() - t

    n, dt = calibrated_steps(timed, 50, CAC_STEPS, seconds_target)
    return {"value": N * CAC_P * n / dt, "unit": "spin-steps/s", "cores": oracle_threads(), "kind": "oracle",
            "sample": f"first alternation ({n} of {CAC_STEPS} Euler-Maruyama steps, Gram prep, replica choice and "
                      f"Jacobi CDP included) of seed {seed}, N = 2000, 8 replicas, FP64 NumPy, {dt:.1f} s"}


def cac_bench(args, torch, L, W, dev):
    """The CAC-CIM (Positive-P, eq. 5-11) as the sigma-minimiser of Algorithm 1
    at the plain shape: N = 2000, M = 1000, 8 replicas, default CAC
    parameters, 1000 steps x 30 alternations, FP32, one l0cim_cac_solve per
    seed.  Supports are compared with the FP64 oracle's stored ones
    (oracle_supports_cac.txt)."""
    gold = golden_file("cac")
    steps, outer = args.euler_steps or CAC_STEPS, args.alternations or CAC_OUTER
    seeds = list(range(args.warmup + args.steps))
    prm = L.cac_params(n_steps=steps)
    data = []
    for sd in seeds:
        inst = W.plain_gaussian(sd)
        data.append((torch.tensor(inst.A, dtype=torch.float32, device=dev),
                     torch.tensor(inst.y, dtype=torch.float32, device=dev), inst))
    outs = []
    sp0 = L.solve_params(eta_init=0.8, eta_end=0.18, velo=outer, n_outer=outer, replicas=CAC_P)
    ws = L.workspace(L.lib().l0cim_cac_solve_workspace_bytes(L.F32, M, N, CAC_P), dev)
    stream = torch.cuda.current_stream()
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(args.steps + 1)]
    for i, sd in enumerate(seeds):
        if i == args.warmup:
            torch.cuda.synchronize()
            L.l0cim_profile_begin()
            t0 = time.perf_counter()
            ev[0].record(stream)
        A, y, _ = data[i]
        sp = L.solve_params(eta_init=0.8, eta_end=0.18, velo=outer, n_outer=outer, replicas=CAC_P, seed=sd)
        outs.append(L.l0cim_cac_solve(A, y, prm, sp, ws=ws, stream=stream))
        if i >= args.warmup:
            ev[i - args.warmup + 1].record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    run_ms, launches = L.l0cim_profile_end()
    gpu_ms = ev[0].elapsed_time(ev[-1])
    elapsed = max(wall, gpu_ms / 1e3)
    match, drmse, per = 0, 0.0, []
    for i in range(args.warmup, len(seeds)):
        sd = seeds[i]
        R, sig, st = outs[i]
        s_h = sig.cpu().numpy()
        inst = data[i][2]
        rm = float(np.sqrt(np.mean((R.double().cpu().numpy() * s_h - inst.x * inst.xi) ** 2)))
        ok = sd in gold and mask_to_int(s_h) == gold[sd][0] and (steps, outer) == (CAC_STEPS, CAC_OUTER)
        match += int(ok)
        if sd in gold:
            drmse = max(drmse, abs(rm - gold[sd][2]))
        per.append({"seed": sd, "support": int(s_h.sum()), "rmse": rm, "identical_to_oracle": ok,
                    "status": L.read_stats(st).status_bits})
    spin = N * CAC_P * steps * outer * args.steps
    # the library's profiling scope wraps each CIM run: one scope per alternation
    step_s = run_ms / 1e3 / max(launches, 1) / steps
    resident = CAC_P <= 8 and N <= 2048   # the one-launch form of l0cim_cac_run (FP32)
    if resident:
        # whole run in one launch, J in registers: the row sums J mu of every
        # replica (2 N^2 P flops per step; the per-spin update and its normals
        # are not counted) against the FP32 vector rate
        flops = 2 * N * N * CAC_P
        roof = {"bound": "alu", "achieved": flops / step_s / 1e12, "peak": FP32_VECTOR_PEAK_TFS,
                "unit": "TFLOP/s", "frac": flops / step_s / 1e12 / FP32_VECTOR_PEAK_TFS, "traffic": None,
                "kernel": "cac_resident_kernel<float>", "flops_per_step": flops, "us_per_step": step_s * 1e6,
                "note": "the whole run in one cooperative launch; J stays in registers, the step time is set by "
                        "the exchange of the measured amplitudes between workgroups"}
    else:
        # one launch per step: J read once per step plus the P measured-amplitude vectors
        byts = N * N * 4 + CAC_P * N * 4 * 6
        roof = {"bound": "hbm", "achieved": byts / step_s / 1e9, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": byts / step_s / 1e9 / HBM_PEAK_GBS, "traffic": None, "kernel": "cac_step_kernel<float>",
                "algorithmic_bytes_per_step": byts, "us_per_step": step_s * 1e6,
                "note": "one launch per Euler step; J (16 MB) is read once per step at the bound"}
    return {
        "metric": METRIC, "value": spin * (match / args.steps) / elapsed, "unit": "spin-steps/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": elapsed * 1e3 / args.steps,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": "CAC-CIM (Positive-P) as the sigma-minimiser: plain Gaussian L0RBCS N=2000, M=1000, "
                               "Bernoulli(0.1), noise 0.01, 8 replicas, default CAC parameters (dt 0.02, tau 0.21, "
                               "g2 1e-7), 1000 Euler-Maruyama steps x 30 alternations, eta 0.8->0.18, Jacobi CDP, "
                               "FP32", "seeds": seeds[args.warmup:]},
        "support_match": f"{match}/{args.steps} seeds identical to the FP64 oracle", "per_seed": per,
        "max_abs_rmse_diff_vs_oracle": drmse if gold else None,
        "spin_steps_per_s_all": spin / elapsed,
        "roofline": roof,
        **({} if args.no_cpu else {"cpu_baseline": cac_cpu_baseline(W)}),
    }


MRI_PIPELINE = dict(gamma=1e-4, lasso_iters=200, lasso_lam1=3e-4, cg_max_iter=10000, cg_tol=1e-5)


def factored_mri_solve(torch, L, inst, dev, cim, P, outer, seed, pipeline=False):
    """Algorithm 1 on the MRI-shaped instance with the couplings applied in
    factored form, one call of l0cim_mri_solve: b and diag(A^T A) from A,
    R_init, then per alternation the initial state, the factored run, the
    replica choice and the CDP.  Plain: R_init = b / D, Jacobi CDP in factored
    form, FP64 refit (G_SS and b_S from A).  Pipeline: the L2 term of eq. 20
    (gamma = 1e-4), the LASSO start and the CG CDP, no refit."""
    n = inst.N
    A = torch.tensor(inst.A, dtype=torch.float32, device=dev)
    y = torch.tensor(inst.y, dtype=torch.float32, device=dev)
    mask_h = np.zeros(n, np.uint8)
    mask_h[inst.meta["freqs"]] = 1
    mask = torch.from_numpy(mask_h).to(dev)
    if pipeline:
        mp = L.mri_params(cdp=L.CDP_CG, **MRI_PIPELINE)
    else:
        mp = L.mri_params()
    sp = L.solve_params(eta_init=0.8, eta_end=0.03, velo=11, n_outer=outer, replicas=P, seed=seed,
                        final_refit_f64=0 if pipeline else 1)
    ws = L.workspace(L.lib().l0cim_mri_solve_workspace_bytes(A.shape[0], P, sp.final_refit_f64), dev)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    R, sel, stats = L.l0cim_mri_solve(mp, A, y, mask, cim, sp, ws=ws)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    return R, sel, L.read_stats(stats).status_bits, dt


def mri_golden():
    """The oracle's stored MRI supports and its FP64 refit on them."""
    gold, gold_R = {}, {}
    path = os.path.join(ROOT, "tests", "golden", "oracle_supports_mri.txt")
    if os.path.exists(path):
        for line in open(path):
            if line.strip() and line[0] != "#":
                sd, k, rm, hx = line.split()
                gold[int(sd)] = (int(hx, 16), float(rm))
    path = os.path.join(ROOT, "tests", "golden", "oracle_refit_mri.txt")
    if os.path.exists(path):
        for line in open(path):
            if line.strip() and line[0] != "#":
                f = line.split()
                gold_R[int(f[0])] = np.array([float(v) for v in f[2:]])
    return gold, gold_R


def mri_flops_per_replica_step(size: int = 128, levels: int = 3) -> float:
    """Algorithmic FP32 work of one factored-couplings Euler step of one
    replica: two 2-D DCTs (forward and inverse), each 2 x size length-size
    complex FFTs at 5 S log2 S flops plus 6 S for the phase factors; the
    inverse and forward Haar levels (3 flops per output); the mask; and
    about 20 flops per spin for the field and Euler update."""
    S = size
    dct2 = 2 * S * (5 * S * math.log2(S) + 6 * S)
    haar = 2 * sum(3 * (S >> l) ** 2 for l in range(levels))
    return 2 * dct2 + haar + S * S + 20 * S * S


def precision_cpu_baseline(P: int, seconds_target: float = 15.0):
    """The FP64 MRI-shaped oracle (couplings applied in factored form, the
    same arithmetic as its stored solves) on a bounded sample of the
    precision workload: the first Euler steps of alternation 0 of seed 0,
    all 64 replicas, from R_init, cut to about `seconds_target` seconds."""
    from oracle import mfcim as O
    from oracle import mri as OM
    from oracle import rng as ORNG
    from workloads import mri as WM

    inst = WM.mri_instance(0)
    op = OM.MriOperator(128, inst.meta["freqs"], A=inst.A)
    b = op.AT(inst.y)[0]
    R = b / op.colnorm2
    z = R * b
    c0, e0 = ORNG.initial_state(0, 0, P, op.N, 1e-2)

    def timed(n):
        cim = O.CimParams(n_steps=n, field=O.BN, K=1.0, d=0.6)
        t = time.perf_counter()
        OM.mfcim_run(op, R, z, 0.8, c0, e0, cim)
        return time.perf_counter() - t

    n, dt = calibrated_steps(timed, 4, 1000, seconds_target)
    return {"value": op.N * P * n / dt, "unit": "spin-steps/s", "cores": oracle_threads(), "kind": "oracle",
            "sample": f"seed 0, alternation 0: {n} Euler steps of all {P} replicas (N = {op.N}), couplings applied "
                      f"in factored form (FP64 NumPy/SciPy DCT), {dt:.1f} s"}


def factored_many_solve(torch, L, insts, dev, cim, P, outer, seeds, pipeline=False):
    """Several MRI-shaped instances through one l0cim_mri_solve_many call
    (their factored CIM runs, LASSO starts and CDPs as one launch each)."""
    n = insts[0].N
    A = torch.tensor(np.stack([i.A for i in insts]), dtype=torch.float32, device=dev)
    y = torch.tensor(np.stack([i.y for i in insts]), dtype=torch.float32, device=dev)
    masks = np.zeros((len(insts), n), np.uint8)
    for k, i in enumerate(insts):
        masks[k, i.meta["freqs"]] = 1
    mask = torch.from_numpy(masks).to(dev)
    mp = L.mri_params(cdp=L.CDP_CG, **MRI_PIPELINE) if pipeline else L.mri_params()
    sp = L.solve_params(eta_init=0.8, eta_end=0.03, velo=11, n_outer=outer, replicas=P,
                        final_refit_f64=0 if pipeline else 1)
    ws = L.workspace(L.lib().l0cim_mri_solve_many_workspace_bytes(len(insts), A.shape[1], P, sp.final_refit_f64), dev)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    R, sel, stats = L.l0cim_mri_solve_many(mp, A, y, mask, seeds, cim, sp, ws=ws)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    st = L.read_stats_array(stats, len(insts))
    return R, sel, [x.status_bits for x in st], dt


def factored_bench(args, torch, L, W, dev):
    from workloads import mri as WM
    P, steps, outer = 64, args.euler_steps or 1000, args.alternations or 11
    if args.instances > 1:
        return factored_many_bench(args, torch, L, WM, dev, P, steps, outer)
    pipeline = args.jdtype == "pipeline"
    gold, gold_R = mri_golden()
    if pipeline:
        gold, gold_R = {k: (v[0], v[2]) for k, v in golden_file("mri_l2").items()}, {}
    seeds = list(range(args.steps))
    cim = L.cim_params(n_steps=steps, field="BN", K=1.0, d=0.6)
    rows, total, cim_total, launches_total, match = [], 0.0, 0.0, 0, 0
    n = 128 * 128
    for sd in seeds:
        print(f"[factored] building the MRI-shaped instance of seed {sd}", file=sys.stderr, flush=True)
        inst = WM.mri_instance(sd)
        if sd == seeds[0]:
            factored_mri_solve(torch, L, inst, dev, L.cim_params(n_steps=4, field="BN", K=1.0, d=0.6), P, 1, sd,
                               pipeline)
        print(f"[factored] solving ({outer} x {steps} steps)", file=sys.stderr, flush=True)
        L.l0cim_profile_begin()
        R, sel, status, dt = factored_mri_solve(torch, L, inst, dev, cim, P, outer, sd, pipeline)
        ms, cnt = L.l0cim_profile_end()
        total += dt
        cim_total += ms
        launches_total += cnt
        sig = sel.cpu().numpy()
        Rv = R.double().cpu().numpy()
        rmse = float(np.sqrt(np.mean((Rv * sig - inst.x * inst.xi) ** 2)))
        ok = sd in gold and mask_to_int(sig) == gold[sd][0] and (steps, outer) == (1000, 11)
        xd = None
        if sd in gold and sd in gold_R:
            x_or = np.zeros(n)
            x_or[[r for r in range(n) if (gold[sd][0] >> r) & 1]] = gold_R[sd]
            xd = float(np.sqrt(np.mean((Rv * sig - x_or) ** 2)))
        match += int(ok)
        rows.append({"seed": sd, "support": int(sig.sum()), "rmse": rmse,
                     "oracle_rmse": gold[sd][1] if sd in gold else None, "oracle_support_match": ok,
                     "hamming_vs_oracle": (bin(mask_to_int(sig) ^ gold[sd][0]).count("1") / n) if sd in gold
                     else None, "xhat_rmse_vs_oracle": xd, "status": status, "solve_s": dt})
        print(f"[factored] seed {sd}: {dt:.3f} s, support {int(sig.sum())}, oracle match {ok}",
              file=sys.stderr, flush=True)
    spin_steps = n * P * steps * outer * len(seeds)
    run_ms = cim_total / launches_total
    flops = mri_flops_per_replica_step() * P * steps
    achieved = flops / (run_ms / 1e3) / 1e12
    return {
        "metric": METRIC, "value": spin_steps / total, "unit": "spin-steps/s", "n_gpus": 1, "steps": len(seeds),
        "warmup": 1, "ms_per_step": total * 1e3 / len(seeds), "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": "MRI-shaped L0RBCS stand-in: 128x128 random-ellipse phantom, 3-level Haar (N=16384), "
                               "30% variable-density DCT-II rows (M=4915), noise 1e-3, 64 replicas, BN field, K=1, "
                               "d=0.6, eta 0.8->0.03 over 11 alternations of 1000 steps, FP32 couplings applied in "
                               "factored form (Haar, FFT-based DCT, mask), " +
                               ("L2 term of eq. 20 (gamma 1e-4), LASSO start (FISTA, lam1 3e-4, 200 iterations), "
                                "CG CDP (relative residual 1e-5, at most 1e4 iterations)" if pipeline else
                                "Jacobi CDP in factored form, FP64 Cholesky refit")},
        "couplings": "factored" + (" + MRI pipeline" if pipeline else ""), "support_match": f"{match}/{len(seeds)}", "per_seed": rows,
        "spin_steps_per_s_cim_only": n * P * steps * launches_total / (cim_total / 1e3),
        "roofline": {"bound": "alu", "achieved": achieved, "peak": FP32_VECTOR_PEAK_TFS, "unit": "TFLOP/s",
                     "frac": achieved / FP32_VECTOR_PEAK_TFS, "traffic": None, "kernel": "mri_cim_kernel<BN>",
                     "flops_per_replica_step": mri_flops_per_replica_step(),
                     "avg_launch_ms": run_ms, "us_per_step": run_ms * 1e3 / steps},
        **({} if args.no_cpu else {"cpu_baseline": precision_cpu_baseline(P)}),
    }


def precision_bench(args, torch, L, W, dev):
    from workloads import mri as WM
    if args.jdtype in ("factored", "pipeline"):
        return factored_bench(args, torch, L, W, dev)
    jdt = {"bf16": L.BF16, "fp8": L.FP8E4M3}[args.jdtype]
    jb = {"bf16": 2, "fp8": 1}[args.jdtype]
    P, steps, outer = 64, args.euler_steps or 1000, args.alternations or 11
    gold = {}
    path = os.path.join(ROOT, "tests", "golden", "oracle_supports_mri.txt")
    if os.path.exists(path):
        for line in open(path):
            if line.strip() and line[0] != "#":
                sd, k, rm, hx = line.split()
                gold[int(sd)] = (int(hx, 16), float(rm))
    # the oracle's x_hat on its own support (its final FP64 refit)
    gold_R = {}
    path = os.path.join(ROOT, "tests", "golden", "oracle_refit_mri.txt")
    if os.path.exists(path):
        for line in open(path):
            if line.strip() and line[0] != "#":
                f = line.split()
                gold_R[int(f[0])] = np.array([float(v) for v in f[2:]])
    seeds = list(range(args.steps))
    cim = L.cim_params(n_steps=steps, field="BN", K=1.0, d=0.6)
    rows, total, cim_total, launches_total, match = [], 0.0, 0.0, 0, 0
    for sd in seeds:
        print(f"[precision] building the MRI-shaped instance of seed {sd}", file=sys.stderr, flush=True)
        inst = WM.mri_instance(sd)
        print(f"[precision] solving ({args.jdtype}, {outer} x {steps} steps)", file=sys.stderr, flush=True)
        A = torch.tensor(inst.A, dtype=torch.float32, device=dev)
        y = torch.tensor(inst.y, dtype=torch.float32, device=dev)
        n = inst.N
        sp = L.solve_params(eta_init=0.8, eta_end=0.03, velo=11, n_outer=outer, replicas=P, j_dtype=jdt,
                            final_refit_f64=1, seed=sd)
        ws = L.workspace(L.l0cim_solve_workspace_bytes(L.F32, inst.M, n, cim, sp), dev)
        R = torch.empty(n, device=dev)
        sg = torch.empty(n, dtype=torch.uint8, device=dev)
        st = torch.zeros(L.STATS_BYTES, dtype=torch.uint8, device=dev)
        if sd == seeds[0]:
            warm = L.solve_params(eta_init=0.8, eta_end=0.03, velo=11, n_outer=1, replicas=P, j_dtype=jdt,
                                  final_refit_f64=1, seed=sd)
            L.l0cim_solve(A, y, L.cim_params(n_steps=4, field="BN", K=1.0, d=0.6), warm, R_out=R, sigma_out=sg,
                          stats=st, ws=ws)
            torch.cuda.synchronize()
        L.l0cim_profile_begin()
        t0 = time.perf_counter()
        L.l0cim_solve(A, y, cim, sp, R_out=R, sigma_out=sg, stats=st, ws=ws)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        ms, cnt = L.l0cim_profile_end()
        total += dt
        cim_total += ms
        launches_total += cnt
        sig = sg.cpu().numpy()
        Rv = R.double().cpu().numpy()
        rmse = float(np.sqrt(np.mean((Rv * sig - inst.x * inst.xi) ** 2)))
        ok = sd in gold and mask_to_int(sig) == gold[sd][0] and (steps, outer) == (1000, 11)
        xd = None
        if sd in gold and sd in gold_R:
            x_or = np.zeros(n)
            S_or = [r for r in range(n) if (gold[sd][0] >> r) & 1]
            x_or[S_or] = gold_R[sd]
            xd = float(np.sqrt(np.mean((Rv * sig - x_or) ** 2)))
        match += int(ok)
        rows.append({"seed": sd, "support": int(sig.sum()), "rmse": rmse,
                     "oracle_rmse": gold[sd][1] if sd in gold else None, "oracle_support_match": ok,
                     "hamming_vs_oracle": (bin(mask_to_int(sig) ^ gold[sd][0]).count("1") / n) if sd in gold
                     else None, "xhat_rmse_vs_oracle": xd, "status": L.read_stats(st).status_bits, "solve_s": dt})
    spin_steps = n * P * steps * outer * len(seeds)
    run_bytes = step_bytes(n, P, jb) * (steps + 1)
    achieved = run_bytes / (cim_total / 1e3 / launches_total) / 1e9
    return {
        "metric": METRIC, "value": spin_steps / total, "unit": "spin-steps/s", "n_gpus": 1, "steps": len(seeds),
        "warmup": 1, "ms_per_step": total * 1e3 / len(seeds), "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": f"MRI-shaped L0RBCS stand-in: 128x128 random-ellipse phantom, 3-level Haar (N=16384), "
                               f"30% variable-density DCT-II rows (M=4915), noise 1e-3, 64 replicas, BN field, K=1, "
                               f"d=0.6, eta 0.8->0.03 over 11 alternations of 1000 steps, {args.jdtype} couplings "
                               f"with per-row scales, FP64 Cholesky refit"},
        "couplings": args.jdtype, "support_match": f"{match}/{len(seeds)}", "per_seed": rows,
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS,
                     "traffic": measured_traffic(PRECISION_TRAFFIC_FILES[args.jdtype], PRECISION_SOURCES,
                                                 "hbm_bytes_per_step"),
                     "kernel": f"bstep_kernel<{args.jdtype}, BN, 4, rb>",
                     "avg_launch_ms": cim_total / launches_total / (steps + 1)},
        **({} if args.no_cpu else {"cpu_baseline": precision_cpu_baseline(P)}),
    }


def serving_cpu_baseline(specs, P, seconds_target: float = 15.0):
    """The FP64 oracle on a bounded sample of the serving stream: the first
    alternation of every 20th of the first 200 requests (Euler step count cut
    so that the sample takes about `seconds_target` seconds)."""
    from oracle import mfcim as O

    sample = list(range(0, min(len(specs), SERVE_HOST_REQUESTS), 20))
    insts = {k: specs[k].build().rounded_f32() for k in sample}

    def timed(n_steps):
        t = time.perf_counter()
        for k in sample:
            outer = O.OuterParams(eta_init=0.8, eta_end=0.18, velo=30, n_outer=1, replicas=P, seed=specs[k].seed)
            O.solve(insts[k].A, insts[k].y, O.CimParams(n_steps=n_steps), outer, keep_history=False)
        return time.perf_counter() - t

    n, dt = calibrated_steps(timed, 10, 1000, seconds_target)
    return {"value": sum(specs[k].N for k in sample) * P * n / dt, "unit": "spin-steps/s", "cores": oracle_threads(),
            "kind": "oracle",
            "sample": f"first alternation ({n} of 1000 Euler steps) of {len(sample)} requests (every 20th), "
                      f"{P} replicas, FP64 NumPy, {dt:.1f} s"}


def serving_bench(args, torch, L, W, dev):
    P, steps, outer = 8, 1000, 30
    specs = W.serving_specs(args.seed, args.requests)
    cim = L.cim_params(n_steps=steps)
    sp = L.solve_params(eta_init=0.8, eta_end=0.18, velo=outer, n_outer=outer, replicas=P, j_dtype=L.F32)
    data, truth = [], []
    print(f"[serving] drawing {len(specs)} requests", file=sys.stderr, flush=True)
    for k, s in enumerate(specs):
        if k < SERVE_HOST_REQUESTS:
            # the first 200 from the NumPy generator (the oracle's stored results are on these)
            inst = s.build()
            data.append((torch.tensor(inst.A, dtype=torch.float32, device=dev),
                         torch.tensor(inst.y, dtype=torch.float32, device=dev)))
            truth.append((inst.x, inst.xi))
        else:
            # the rest of a long stream drawn on the device (same law, other draws)
            A, y, _x, _xi = W.gaussian_instance_device(s.seed, s.N, s.M, s.a, s.nu, dev)
            data.append((A, y))
            truth.append(None)
        if (k + 1) % 250 == 0:
            print(f"[serving] {k + 1}/{len(specs)} requests drawn", file=sys.stderr, flush=True)
    max_n = max(s.N for s in specs)
    outs = [(torch.empty(s.N, device=dev), torch.empty(s.N, dtype=torch.uint8, device=dev),
             torch.zeros(L.STATS_BYTES, dtype=torch.uint8, device=dev)) for s in specs]
    free, _tot = torch.cuda.mem_get_info()
    need = L.l0cim_server_arena_overhead(args.slots, max_n, sp) + sum(
        L.l0cim_server_request_bytes(s.M, s.N, sp) for s in specs)
    arena_bytes = int(min(need + (1 << 20), 0.6 * free))
    arena = L.workspace(arena_bytes, dev)
    torch.cuda.synchronize()

    def serve(arrivals):
        """Serve every request; arrivals are offsets (s) from the start."""
        server = L.l0cim_server_create(cim, sp, args.slots, max_n, arena)
        if args.step_budget_mb > 0:
            L.l0cim_server_set_step_budget(server, int(args.step_budget_mb * 1e6))
        t0 = L.l0cim_server_clock(server)
        nxt, done, lat = 0, 0, {}
        L.l0cim_profile_begin()
        while done < len(specs):
            now = L.l0cim_server_clock(server) - t0
            while nxt < len(specs) and arrivals[nxt] <= now:
                A, y = data[nxt]
                L.l0cim_server_submit(server, A, y, specs[nxt].seed, nxt, *outs[nxt])
                nxt += 1
            info = L.l0cim_server_info(server)
            if info["active"] == 0 and info["pending"] == 0:
                time.sleep(max(0.0, min(0.01, arrivals[nxt] - now)))
                continue
            done += L.l0cim_server_step(server)
            for c in L.l0cim_server_completed(server):
                lat[c.tag] = c.t_finish - t0 - arrivals[c.tag]
                if len(lat) % 20 == 0:
                    print(f"[serving] {len(lat)}/{len(specs)} done at {c.t_finish - t0:.1f} s", file=sys.stderr,
                          flush=True)
        end = L.l0cim_server_clock(server) - t0
        cim_ms, launches = L.l0cim_profile_end()
        ticks = L.l0cim_server_info(server)["ticks"]
        L.l0cim_server_destroy(server)
        v = [lat[k] for k in range(len(specs))]
        return end, v, cim_ms, ticks

    total_spin = sum(s.N for s in specs) * P * steps * outer
    total_bytes = sum(step_bytes(s.N, P, 4) for s in specs) * (steps + 1) * outer
    runs = []
    if args.ref_thr > 0:
        # rates relative to a saturation throughput measured in an earlier run (a long stream
        # then fits one process: one arrival rate per run); value is this run's throughput
        if len(args.rates) != 1:
            raise SystemExit("--ref-thr takes exactly one --rates value")
        thr = args.ref_thr
        frac = args.rates[0]
        print(f"[serving] {len(specs)} requests, arena {arena_bytes / 1e9:.1f} GB; Poisson arrivals at {frac} x "
              f"{thr:.2f} req/s", file=sys.stderr, flush=True)
        arr = W.poisson_arrivals(args.seed, len(specs), frac * thr)
        makespan, lat, cim_ms, ticks = serve(list(arr))
        p50, p99 = percentiles(lat)
        runs.append({"rate_frac": frac, "arrival_rate": frac * thr, "req_per_s": len(specs) / makespan,
                     "p50_s": p50, "p99_s": p99, "ticks": ticks})
        args.rates = []
    else:
        # saturation: every request present at t = 0
        print(f"[serving] {len(specs)} requests, arena {arena_bytes / 1e9:.1f} GB; saturation run",
              file=sys.stderr, flush=True)
        makespan, lat_sat, cim_ms, ticks = serve([0.0] * len(specs))
    # the sampled requests against the oracle's stored supports (saturation run)
    gold = golden_file("serving") if args.seed == 0 else {}
    sample = [k for k in sorted(gold) if k < len(specs)]
    match, drmse, per = 0, 0.0, []
    for k in sample:
        s_k = outs[k][1].cpu().numpy()
        R_k = outs[k][0].double().cpu().numpy()
        rm = float(np.sqrt(np.mean((R_k * s_k - truth[k][0] * truth[k][1]) ** 2)))
        ok = mask_to_int(s_k) == gold[k][0]
        match += int(ok)
        drmse = max(drmse, abs(rm - gold[k][2]))
        per.append({"request": k, "N": specs[k].N, "identical": bool(ok), "rmse": rm, "oracle_rmse": gold[k][2]})
    sat_bits = [outs[k][1].clone() for k in range(len(specs))]
    if args.ref_thr <= 0:
        thr = len(specs) / makespan
        runs = [{"rate_frac": "saturation", "req_per_s": thr, "p50_s": percentiles(lat_sat)[0],
                 "p99_s": percentiles(lat_sat)[1], "ticks": ticks}]
    achieved = total_bytes / (cim_ms / 1e3) / 1e9
    for frac in args.rates:
        print(f"[serving] Poisson arrivals at {frac} x {thr:.2f} req/s", file=sys.stderr, flush=True)
        arr = W.poisson_arrivals(args.seed, len(specs), frac * thr)
        span, lat, _ms, ticks = serve(list(arr))
        p50, p99 = percentiles(lat)
        same = all(torch.equal(outs[k][1], sat_bits[k]) for k in range(len(specs)))
        runs.append({"rate_frac": frac, "arrival_rate": frac * thr, "req_per_s": len(specs) / span, "p50_s": p50,
                     "p99_s": p99, "ticks": ticks, "supports_equal_saturation_run": bool(same)})
    # the single-instance path on the same requests, one at a time (FIFO)
    k_plain = len(specs) if args.plain_sample < 0 else min(len(specs), args.plain_sample)
    svc = []
    ws = None
    print(f"[serving] single-instance path on {k_plain} requests", file=sys.stderr, flush=True)
    for k in range(k_plain):
        A, y = data[k]
        sps = L.solve_params(eta_init=0.8, eta_end=0.18, velo=outer, n_outer=outer, replicas=P, j_dtype=L.F32,
                             seed=specs[k].seed)
        nb = L.l0cim_solve_workspace_bytes(L.F32, specs[k].M, specs[k].N, cim, sps)
        if ws is None or ws.numel() < nb:
            ws = L.workspace(nb, dev)
        R, sg, st = outs[k]
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        L.l0cim_solve(A, y, cim, sps, R_out=R, sigma_out=sg, stats=st, ws=ws)
        torch.cuda.synchronize()
        svc.append(time.perf_counter() - t1)
        if (k + 1) % 20 == 0:
            print(f"[serving] single-instance path {k + 1}/{k_plain}", file=sys.stderr, flush=True)
    plain_thr = k_plain / sum(svc) if svc else None
    plain_spin = sum(specs[k].N for k in range(k_plain)) * P * steps * outer / sum(svc) if svc else None
    # FIFO replay of the measured service times under each rate's arrivals
    # (one request at a time on the single-instance path)
    plain_p = {}
    for frac in (args.rates if svc else []):
        arr = W.poisson_arrivals(args.seed, len(specs), frac * thr)[:k_plain]
        t, lat_p = 0.0, []
        for a_k, s_k in zip(arr, svc):
            t = max(t, a_k) + s_k
            lat_p.append(t - a_k)
        plain_p[str(frac)] = {"p50_s": percentiles(lat_p)[0], "p99_s": percentiles(lat_p)[1]}
    return {
        "metric": METRIC, "value": total_spin / makespan, "unit": "spin-steps/s", "n_gpus": 1,
        "steps": len(specs), "warmup": 0, "ms_per_step": makespan * 1e3 / len(specs), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": "serving: Gaussian L0RBCS requests, N log-uniform [512, 8192], alpha U[0.2, 0.6], "
                               "sparsity U[0.05, 0.2], noise 0.01, 8 replicas, 1000 Euler steps x 30 alternations, "
                               "FP32 couplings, continuous batching (one alternation per tick)",
                   "requests": len(specs), "max_slots": args.slots, "arena_GB": arena_bytes / 1e9,
                   "step_budget_MB": args.step_budget_mb or None},
        "requests_per_s": len(specs) / makespan, "runs": runs,
        "reference_saturation_req_per_s": args.ref_thr if args.ref_thr > 0 else None,
        "support_match": f"{match}/{len(sample)} sampled requests (every 4th) identical to the FP64 oracle",
        "max_abs_rmse_diff_vs_oracle": drmse if sample else None, "per_request": per,
        "single_instance_path": {"requests_measured": k_plain, "req_per_s": plain_thr, "spin_steps_per_s": plain_spin,
                                 "fifo_latency_at_rates": plain_p,
                                 "service_s_p50": percentiles(svc)[0] if svc else None},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": None, "kernel": "bstep_kernel<float, CN, 1, rb>",
                     "note": "algorithmic bytes of every Euler step served / CIM kernel time, saturation run"},
        **({} if args.no_cpu else {"cpu_baseline": serving_cpu_baseline(specs, P)}),
    }


# ---------------------------------------------------------------------------
# accuracy form: the paper's random-data studies on the device path
# ---------------------------------------------------------------------------

ACC_N, ACC_STEPS, ACC_VELO = 2000, 1000, 51
ACC_A = (0.05, 0.1, 0.15, 0.2, 0.25, 0.3)
# (alpha, noise std, eta_end) of the noisy-observation study
ACC_CONFIGS = ((0.6, 0.05, 0.18), (0.8, 0.05, 0.18), (0.6, 0.1, 0.35), (0.8, 0.1, 0.35))


def acc_rmse(sig, R, x, xi) -> float:
    """RMSE against the truth, sqrt(mean((R sigma - x xi)^2))."""
    d = np.asarray(R, float) * sig - x * xi
    return float(np.sqrt(np.mean(d * d)))


def acc_hamming(sig, xi) -> float:
    return float(np.mean(np.abs(np.asarray(sig, int) - np.asarray(xi, int))))


def acc_seed(alpha: float, nu: float, ia: int, k: int) -> int:
    return 100000 * int(round(alpha * 10)) + 10000 * int(round(nu * 100)) + 100 * ia + k


def acc_instance(W, alpha, nu, ia, k):
    """Random data as the paper draws it: exactly round(aN) non-zeros."""
    return W.gaussian_instance(acc_seed(alpha, nu, ia, k), ACC_N, int(round(alpha * ACC_N)), ACC_A[ia], nu,
                               support="exact").rounded_f32()


def acc_oracle_sample(W, device_rows, count):
    """The FP64 oracle on `count` solves of the alpha 0.6 / noise 0.05 sweep
    (the same FP32-rounded instances and counter-generator seeds): support and
    RMSE beside the device's, and the oracle's time."""
    from threadpoolctl import threadpool_info

    from oracle import mfcim as O

    cores = len(os.sched_getaffinity(0))
    out, spent, steps = [], 0.0, 0
    for row in device_rows[:count]:
        inst = acc_instance(W, 0.6, 0.05, row["ia"], row["k"])
        cim = O.CimParams(n_steps=ACC_STEPS, field=row["field"])
        outer = O.OuterParams(eta_init=0.8, eta_end=0.18, velo=ACC_VELO, n_outer=ACC_VELO,
                              seed=acc_seed(0.6, 0.05, row["ia"], row["k"]))
        t1 = time.perf_counter()
        res = O.solve(inst.A, inst.y, cim, outer, keep_history=False)
        spent += time.perf_counter() - t1
        steps += ACC_N * ACC_STEPS * ACC_VELO
        rm = acc_rmse(res.sigma, res.R, inst.x, inst.xi)
        out.append({"a": ACC_A[row["ia"]], "field": row["field"], "seed_index": row["k"],
                    "support_identical": bool(np.array_equal(res.sigma, row["sigma"])),
                    "hamming_vs_oracle": acc_hamming(res.sigma, row["sigma"]),
                    "rmse_device": row["rmse"], "rmse_oracle": rm, "rmse_diff": abs(rm - row["rmse"])})
        print(f"[accuracy] oracle a={ACC_A[row['ia']]} {row['field']}: identical={out[-1]['support_identical']} "
              f"|drmse|={out[-1]['rmse_diff']:.2e}", file=sys.stderr, flush=True)
    threads = max([i.get("num_threads", 1) for i in threadpool_info()] or [1])
    return {"value": steps / spent if spent else None, "unit": "spin-steps/s", "cores": int(min(threads, cores)),
            "kind": "oracle",
            "sample": f"{len(out)} whole solves of the alpha 0.6 / noise 0.05 sweep (FP64 NumPy), {spent:.1f} s",
            "agreement": out}


def accuracy_bench(args, torch, L, W, dev):
    """The paper's random-data accuracy studies, run on the device path (FP32
    solve, N = 2000, 1000 Euler steps x 51 alternations, eta 0.8 -> eta_end
    over velo = 51, 100 Jacobi CDP sweeps, K = 1, d = 0.4, exactly round(aN)
    non-zeros as the paper draws its random data):
      rmse_vs_a  average RMSE against the truth (and Hamming loss) for each
                 sparseness a, at alpha 0.6 / 0.8 and noise std 0.05
                 (eta_end 0.18) / 0.1 (eta_end 0.35), CN and BN fields
                 (the noisy-observation figure of the Results);
      tau        the same at alpha 0.6, noise 0.1 with tau = 0.15 beside
                 tau = 1 (the sparseness / tau figure of the Supplement);
      history    RMSE and Hamming loss after each alternation, median and
                 quartiles over the datasets, at alpha 0.6, a = 0.2, noise
                 0.05, through the step-level entry points (the field
                 comparison figure), and the median |c| at the end of the
                 second alternation for tau = 1 and 0.15 (the amplitude figure);
      oracle     (cpu_baseline) the FP64 oracle on a few of the same solves."""
    seeds = range(args.acc_seeds)
    spin_steps, busy = 0, 0.0
    ws = {}

    def solve(inst, field, tau, eta_end, seed):
        nonlocal spin_steps, busy
        A = torch.tensor(inst.A, dtype=torch.float32, device=dev)
        y = torch.tensor(inst.y, dtype=torch.float32, device=dev)
        cim = L.cim_params(n_steps=ACC_STEPS, field=field, tau=tau)
        sp = L.solve_params(eta_init=0.8, eta_end=eta_end, velo=ACC_VELO, n_outer=ACC_VELO, seed=seed)
        key = A.shape
        if key not in ws:
            ws[key] = L.workspace(L.l0cim_solve_workspace_bytes(L.F32, A.shape[0], ACC_N, cim, sp), dev)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        R, sig, st = L.l0cim_solve(A, y, cim, sp, ws=ws[key])
        torch.cuda.synchronize()
        busy += time.perf_counter() - t1
        spin_steps += ACC_N * ACC_STEPS * ACC_VELO
        status = L.read_stats(st).status_bits
        sg = sig.cpu().numpy()
        return sg, R.double().cpu().numpy(), status

    rmse_tab, tau_tab, sample_rows, bad = {}, {}, [], 0
    for alpha, nu, eta_end in ACC_CONFIGS:
        key = f"alpha={alpha} nu={nu}"
        taus = (1.0, 0.15) if (alpha, nu) == (0.6, 0.1) else (1.0,)
        acc = {(f, tau): ([], []) for f in ("CN", "BN") for tau in taus}
        for ia, a in enumerate(ACC_A):
            per = {kk: ([], []) for kk in acc}
            for k in seeds:
                inst = acc_instance(W, alpha, nu, ia, k)
                for (field, tau) in acc:
                    sg, R, st = solve(inst, field, tau, eta_end, acc_seed(alpha, nu, ia, k))
                    bad += int(st != 0)
                    rm = acc_rmse(sg, R, inst.x, inst.xi)
                    per[(field, tau)][0].append(rm)
                    per[(field, tau)][1].append(acc_hamming(sg, inst.xi))
                    if (alpha, nu) == (0.6, 0.05) and tau == 1.0 and k == 0:
                        sample_rows.append({"ia": ia, "k": k, "field": field, "sigma": sg, "rmse": rm})
            for kk in acc:
                acc[kk][0].append(float(np.mean(per[kk][0])))
                acc[kk][1].append(float(np.mean(per[kk][1])))
            print(f"[accuracy] {key} a={a}: " + ", ".join(
                f"{f}/tau{tau} {acc[(f, tau)][0][-1]:.4f}" for f, tau in acc), file=sys.stderr, flush=True)
        rmse_tab[key] = {f: {"rmse": acc[(f, 1.0)][0], "hamming": acc[(f, 1.0)][1]} for f in ("CN", "BN")}
        if len(taus) > 1:
            tau_tab[key] = {f"{f} tau={tau}": acc[(f, tau)][0] for f, tau in acc}

    # per-alternation history through the step-level entry points
    def history(inst, field, tau, seed, n_alt):
        n = ACC_N
        A = torch.tensor(inst.A, dtype=torch.float32, device=dev)
        y = torch.tensor(inst.y, dtype=torch.float32, device=dev)
        G, b = L.l0cim_gram(A, y)
        status = torch.zeros(1, dtype=torch.int32, device=dev)
        R = L.l0cim_init_r(G, b, status=status)
        c = torch.empty((1, n), dtype=torch.float32, device=dev)
        e = torch.empty_like(c)
        H = torch.empty(1, dtype=torch.float64, device=dev)
        prm = L.cim_params(n_steps=ACC_STEPS, field=field, tau=tau)
        ws_run = L.workspace(L.l0cim_mfcim_run_workspace_bytes(L.F32, n, 1, L.F32), dev)
        ws_cdp = L.workspace(L.l0cim_update_r_workspace_bytes(L.F32, n, L.CDP_JACOBI), dev)
        rms, hls, camp = [], [], None
        for i in range(n_alt):
            eta = max(0.8 * (1.0 - i / ACC_VELO), 0.18)
            J, _, z = L.l0cim_build_couplings(G, b, R)
            L.l0cim_init_state(n, 1, seed, i, prm.c0_std, c, e)
            sig = L.l0cim_mfcim_run(J, z, eta, prm, c, e, H=H, status=status, ws=ws_run)
            sel = L.l0cim_select_replica(H, sig)
            L.l0cim_update_r(G, b, sel, R, iters=100, status=status, ws=ws_cdp)
            sg = sel.cpu().numpy()
            if i == 1:
                camp = float(np.median(np.abs(c.double().cpu().numpy())))
            rms.append(acc_rmse(sg, R.double().cpu().numpy(), inst.x, inst.xi))
            hls.append(acc_hamming(sg, inst.xi))
        return rms, hls, camp, int(status.item())

    hist_tab, amp_tab = {}, {}
    for field in ("CN", "BN"):
        runs, amps, amps_015 = [], [], []
        for k in seeds:
            inst = W.gaussian_instance(acc_seed(0.6, 0.05, 3, 50 + k), ACC_N, int(0.6 * ACC_N), 0.2, 0.05,
                                       support="exact").rounded_f32()
            rms, hls, camp, st = history(inst, field, 1.0, acc_seed(0.6, 0.05, 3, 50 + k), ACC_VELO)
            bad += int(st != 0)
            runs.append((rms, hls))
            amps.append(camp)
            _, _, camp2, st = history(inst, field, 0.15, acc_seed(0.6, 0.05, 3, 50 + k), 2)
            amps_015.append(camp2)
        rm = np.array([r[0] for r in runs])
        hl = np.array([r[1] for r in runs])
        pick = sorted(set(range(0, ACC_VELO, 5)) | {ACC_VELO - 1})
        hist_tab[field] = {"alternation": pick,
                           "rmse_median": [float(np.median(rm[:, i])) for i in pick],
                           "rmse_q25": [float(np.percentile(rm[:, i], 25)) for i in pick],
                           "rmse_q75": [float(np.percentile(rm[:, i], 75)) for i in pick],
                           "hamming_median": [float(np.median(hl[:, i])) for i in pick]}
        amp_tab[field] = {"tau=1": float(np.median(amps)), "tau=0.15": float(np.median(amps_015))}
        print(f"[accuracy] history {field}: final median RMSE {hist_tab[field]['rmse_median'][-1]:.4f}, "
              f"median |c| {amp_tab[field]}", file=sys.stderr, flush=True)

    out = {"metric": "MF-CIM accuracy studies on random data (RMSE vs sparseness, per-alternation RMSE and "
                     "Hamming loss, tau = 0.15)",
           "value": spin_steps / busy, "unit": "spin-steps/s", "n_gpus": 1, "steps": len(seeds), "warmup": 0,
           "ms_per_step": busy * 1e3 / max(1, spin_steps // (ACC_N * ACC_STEPS * ACC_VELO)),
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
           "config": {"workload": f"random Gaussian L0RBCS, N={ACC_N}, alpha in {{0.6, 0.8}}, exactly round(aN) "
                                  f"non-zeros, a in {list(ACC_A)}, noise 0.05 / 0.1, {ACC_STEPS} Euler steps x "
                                  f"{ACC_VELO} alternations, eta 0.8 -> 0.18 / 0.35 (velo {ACC_VELO}), Jacobi CDP, "
                                  f"{len(seeds)} datasets per point, FP32"},
           "status_nonzero": bad, "rmse_vs_a": {"a": list(ACC_A), **rmse_tab}, "tau": tau_tab,
           "history": hist_tab, "median_abs_c_second_alternation": amp_tab}
    if args.acc_oracle > 0 and not args.no_cpu:
        out["cpu_baseline"] = acc_oracle_sample(W, sample_rows, args.acc_oracle)
    return out


def plain_many_bench(args, torch, L, W, dev):
    """Plain form with K = --instances independent seeds per step: one
    l0cim_solve_many call solves them together, so the register-resident CIM
    runs of all K share one cooperative launch and their exchange round trips
    overlap.  value counts the spin-steps of the instances whose support equals
    the stored oracle support."""
    K = args.instances
    gold = golden_supports()
    total = (args.warmup + args.steps) * K
    seeds = sorted(gold)[:total] if len(gold) >= total else list(range(total))
    groups = [seeds[i * K:(i + 1) * K] for i in range(args.warmup + args.steps)]
    data = []
    for g in groups:
        insts = [W.plain_gaussian(s) for s in g]
        A = torch.tensor(np.stack([i.A for i in insts]), dtype=torch.float32, device=dev)
        y = torch.tensor(np.stack([i.y for i in insts]), dtype=torch.float32, device=dev)
        data.append((g, A, y))
    cim = L.cim_params(n_steps=STEPS)
    sp = L.solve_params(eta_init=0.8, eta_end=0.18, velo=OUTER, n_outer=OUTER)
    ws = L.workspace(L.l0cim_solve_many_workspace_bytes(L.F32, K, M, N, sp), dev)
    outs = [(torch.empty((K, N), dtype=torch.float32, device=dev), torch.empty((K, N), dtype=torch.uint8, device=dev),
             torch.zeros(K * L.STATS_BYTES, dtype=torch.uint8, device=dev)) for _ in groups]
    stream = torch.cuda.current_stream()

    def run(i):
        g, A, y = data[i]
        R, sig, st = outs[i]
        L.l0cim_solve_many(A, y, g, cim, sp, R_out=R, sigma_out=sig, stats=st, ws=ws, stream=stream)

    for i in range(args.warmup):
        run(i)
    torch.cuda.synchronize()
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(args.steps + 1)]
    L.l0cim_profile_begin()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ev[0].record(stream)
    for k in range(args.steps):
        run(args.warmup + k)
        ev[k + 1].record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    cim_ms, cim_launches = L.l0cim_profile_end()
    lat = [ev[k].elapsed_time(ev[k + 1]) for k in range(args.steps)]
    gpu_ms = ev[0].elapsed_time(ev[-1])
    match, status_bad = 0, 0
    for k in range(args.steps):
        i = args.warmup + k
        sig = outs[i][1].cpu().numpy()
        sts = L.read_stats_array(outs[i][2], K)
        for j, s in enumerate(groups[i]):
            status_bad += int(sts[j].status_bits != 0)
            if s in gold and mask_to_int(sig[j]) == gold[s]:
                match += 1
    spin_steps = N * P * STEPS * OUTER * K
    elapsed = max(wall, gpu_ms / 1e3)
    value = spin_steps * (match / K) / elapsed
    # (2N + 20) flops per spin-step; the K instances of a call share one
    # launch when the device holds all their workgroups at once, else the
    # library runs them one launch each: count instances per launch from
    # the launches actually made
    cim_runs = K * OUTER * args.steps
    per_launch = cim_runs / max(cim_launches, 1)
    per_launch_flops = (2 * N + 20) * N * P * STEPS * per_launch
    avg_launch_s = (cim_ms / 1e3) / max(cim_launches, 1)
    achieved = per_launch_flops / avg_launch_s / 1e12
    return {
        "metric": METRIC,
        "value": value,
        "unit": "spin-steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": elapsed * 1e3 / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": WORKLOAD + f"; {K} instances per step (l0cim_solve_many)", "N": N, "M": M,
                   "replicas": P, "euler_steps": STEPS, "alternations": OUTER, "instances": K,
                   "seeds": [s for g in groups[args.warmup:] for s in g]},
        "support_match": f"{match}/{args.steps * K}",
        "spin_steps_per_s_all": spin_steps * args.steps / elapsed,
        "spin_steps_per_s_cim_only": N * P * STEPS * cim_runs / (cim_ms / 1e3) if cim_ms > 0 else None,
        "p50_ms": float(np.percentile(lat, 50)),
        "p99_ms": float(np.percentile(lat, 99)),
        "status_nonzero": status_bad,
        "roofline": {"bound": "alu", "achieved": achieved, "peak": FP32_VECTOR_PEAK_TFS, "unit": "TFLOP/s",
                     "frac": achieved / FP32_VECTOR_PEAK_TFS, "traffic": None,
                     "kernel": "cim_regs_kernel",
                     "flops_per_launch": per_launch_flops,
                     "instances_per_launch": per_launch,
                     "regime": f"{per_launch:g} instances' couplings held in registers per cooperative launch "
                               f"({K} per call); the step time is set by the exchange of amplitudes between "
                               "workgroups",
                     "us_per_euler_step": avg_launch_s * 1e6 / STEPS,
                     "avg_launch_ms": avg_launch_s * 1e3, "launches": cim_launches},
    }


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--traffic-probe", action="store_true",
                    help="run a 512 MiB fill and copy first (HBM counter calibration)")
    ap.add_argument("--form", choices=["plain", "batched", "precision", "serving", "accuracy", "cac"], default="batched")
    ap.add_argument("--jdtype", choices=["bf16", "fp8", "factored", "pipeline"], default="bf16",
                    help="precision form couplings (factored: FP32, applied through the MRI operator; pipeline: "
                         "the same with the L2 term of eq. 20, the LASSO start and the CG CDP)")
    ap.add_argument("--requests", type=int, default=200, help="serving form: number of requests")
    ap.add_argument("--slots", type=int, default=48, help="serving form: resident requests at most")
    ap.add_argument("--rates", type=float, nargs="*", default=[0.5, 0.9],
                    help="serving form: Poisson arrival rates as fractions of the saturation throughput")
    ap.add_argument("--ref-thr", type=float, default=0.0,
                    help="serving form: skip the saturation run and take this throughput (req/s) as the reference "
                         "of the first --rates value (one rate per run; for long streams)")
    ap.add_argument("--plain-sample", type=int, default=-1,
                    help="serving form: requests timed on the single-instance path (-1: all, 0: none)")
    ap.add_argument("--step-budget-mb", type=float, default=300.0,
                    help="serving form: cap on the couplings MB one Euler step of the resident set streams (0: none)")
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--acc-seeds", type=int, default=10, help="accuracy form: datasets per point")
    ap.add_argument("--acc-oracle", type=int, default=4,
                    help="accuracy form: solves of the sweep the FP64 oracle repeats (0: none)")
    ap.add_argument("--euler-steps", type=int, default=0,
                    help="precision / batched forms: Euler steps per alternation instead of 1000 (profiling runs)")
    ap.add_argument("--alternations", type=int, default=0,
                    help="precision / batched forms: alternations instead of 11 / 30 (profiling runs)")
    ap.add_argument("--no-graph", action="store_true",
                    help="batched form: launch the Euler steps one by one (no HIP graph replay)")
    ap.add_argument("--instances", type=int, default=1,
                    help="plain form: independent instances solved together per step (l0cim_solve_many; their "
                         "register-resident CIM runs share one launch); factored / pipeline precision forms: MRI "
                         "instances per l0cim_mri_solve_many call")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for {args.gpus}); the multi-GPU layout is "
              "described in the design notes and not measured here", file=sys.stderr)
        sys.exit(2)

    import torch

    import paper_2405_00366_amd as L
    import workloads as W

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    if args.traffic_probe:
        traffic_probe(torch, dev)
    if args.form != "plain":
        fn = {"batched": batched_bench, "precision": precision_bench, "serving": serving_bench,
              "accuracy": accuracy_bench, "cac": cac_bench}[args.form]
        print(json.dumps(fn(args, torch, L, W, dev)), flush=True)
        return
    if args.instances > 1:
        print(json.dumps(plain_many_bench(args, torch, L, W, dev)), flush=True)
        return
    gold = golden_supports()
    seeds = sorted(gold)[: args.warmup + args.steps] if len(gold) >= args.warmup + args.steps else \
        list(range(args.warmup + args.steps))
    insts = []
    for s in seeds:
        inst = W.plain_gaussian(s)
        insts.append((s, torch.tensor(inst.A, dtype=torch.float32, device=dev),
                      torch.tensor(inst.y, dtype=torch.float32, device=dev)))
    cim = L.cim_params(n_steps=STEPS)
    sps = [L.solve_params(eta_init=0.8, eta_end=0.18, velo=OUTER, n_outer=OUTER, seed=s) for s in seeds]
    ws = L.workspace(L.l0cim_solve_workspace_bytes(L.F32, M, N, cim, sps[0]), dev)
    outs = [(torch.empty(N, dtype=torch.float32, device=dev), torch.empty(N, dtype=torch.uint8, device=dev),
             torch.zeros(L.STATS_BYTES, dtype=torch.uint8, device=dev)) for _ in seeds]
    stream = torch.cuda.current_stream()

    def run(i):
        s, A, y = insts[i]
        R, sig, st = outs[i]
        L.l0cim_solve(A, y, cim, sps[i], R_out=R, sigma_out=sig, stats=st, ws=ws, stream=stream)

    for i in range(args.warmup):
        run(i)
    torch.cuda.synchronize()

    ev = [torch.cuda.Event(enable_timing=True) for _ in range(args.steps + 1)]
    L.l0cim_profile_begin()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ev[0].record(stream)
    for k in range(args.steps):
        run(args.warmup + k)
        ev[k + 1].record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    cim_ms, cim_launches = L.l0cim_profile_end()
    lat = [ev[k].elapsed_time(ev[k + 1]) for k in range(args.steps)]
    gpu_ms = ev[0].elapsed_time(ev[-1])

    match, status_bad = 0, 0
    for k in range(args.steps):
        i = args.warmup + k
        s = seeds[i]
        sig = outs[i][1].cpu().numpy()
        st = L.read_stats(outs[i][2])
        status_bad += int(st.status_bits != 0)
        if s in gold and mask_to_int(sig) == gold[s]:
            match += 1
    spin_steps = N * P * STEPS * OUTER
    elapsed = max(wall, gpu_ms / 1e3)
    value = spin_steps * match / elapsed
    # roofline of the dominant kernel (the CIM run).  Its couplings stay in the
    # register file for the whole run, so HBM does not bound it; the bound is
    # the vector ALUs: (2N + 20) flops per spin-step (the J-row FMA chain and
    # the Euler update), N * P spin-steps per Euler step, STEPS steps per launch.
    per_launch_flops = (2 * N + 20) * N * P * STEPS
    per_launch_bytes = (N * N * 4 + 24 * N * P) * STEPS
    avg_launch_s = (cim_ms / 1e3) / max(cim_launches, 1)
    achieved = per_launch_flops / avg_launch_s / 1e12
    out = {
        "metric": METRIC,
        "value": value,
        "unit": "spin-steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": elapsed * 1e3 / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": WORKLOAD, "N": N, "M": M, "replicas": P, "euler_steps": STEPS,
                   "alternations": OUTER, "seeds": seeds[args.warmup:]},
        "support_match": f"{match}/{args.steps}",
        "spin_steps_per_s_all": spin_steps * args.steps / elapsed,
        # the same count over the CIM kernels' own time (HIP events around each launch)
        "spin_steps_per_s_cim_only": N * P * STEPS * cim_launches / (cim_ms / 1e3) if cim_ms > 0 else None,
        "p50_ms": float(np.percentile(lat, 50)),
        "p99_ms": float(np.percentile(lat, 99)),
        "status_nonzero": status_bad,
        "roofline": {"bound": "alu", "achieved": achieved, "peak": FP32_VECTOR_PEAK_TFS, "unit": "TFLOP/s",
                     "frac": achieved / FP32_VECTOR_PEAK_TFS, "traffic": measured_traffic(),
                     "kernel": "cim_regs_kernel",
                     "flops_per_launch": per_launch_flops,
                     "regime": "couplings held in registers for the whole run; the step time is set by the "
                               "exchange of amplitudes between workgroups, not by HBM (traffic = HBM bytes per "
                               "launch from the counters)",
                     "effective_GBps": per_launch_bytes / avg_launch_s / 1e9,
                     "us_per_euler_step": avg_launch_s * 1e6 / STEPS,
                     "avg_launch_ms": avg_launch_s * 1e3, "launches": cim_launches},
    }
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
