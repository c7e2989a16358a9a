#!/usr/bin/env python3
"""Benchmark: the batched fine propagator of Parareal for the Galloway-Proctor
kinematic dynamo on one MI355X, on the largest single-GPU workload.

Workload (default): Galloway-Proctor CP flow, Rm = 2000, kz = 0.57, 512 x 512
Fourier grid, complex128, T = 256 cut into 256 slices, fine SBDF2 with
dt = 5e-4 (2000 steps a slice).  The slice states come from the library's
seeded initial field and an initial coarse run.  One step = one fine time
step of all 256 slices at once, exactly as every Parareal iteration launches
it (column phase: inverse y-FFT, u x b, forward y-FFT with the 2/3 mask; row
phase: forward x-FFT, 1/N^2, spectral curl, implicit diffusion solve, SBDF
update, inverse x-FFT): 512^2 x 256 = 67.1 M mode-steps.

The sweep runs as Parareal runs it: blocked in time as the autotuner chooses
(at 512^2 groups of 2-3 slices running all their steps back to back on 3
streams), so a group's buffers stay in the memory-side last-level cache
between steps; the K timed steps are K steps of every slice.

value: fine-propagator mode-steps per second, N^2 * slices * K / (time of K
  steps); the states are resident in HBM before the timed region.
roofline: 192 B per mode-step (read and write state and history, 3
  complex128 components, full grid) over the time of one step of the sweep
  (HIP events on the launching stream), against 8 TB/s; the two kernels'
  own durations, launched over the whole batch, are reported beside it.

Other workloads: --config2 (a whole Parareal solve of the 128^2, 64-slice
workload), --parareal5 (a Parareal solve of the default workload), --batch,
--learned, --nc-sweep, --nc-sweep-gp, --table1, --work-precision.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu-baseline]
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

# the 128^2 whole-solve workload (--config2)
N, KZ, RM, T, P = 128, 0.57, 100.0, 64.0, 64
DT_FINE, DT_COARSE, N_COARSE = 2e-3, 1e-2, 64
TOL, MAX_ITER, SEED = 1e-8, 64, 200000
# the headline workload: largest single-GPU run
N5, RM5, T5, P5, DT5, SEED5 = 512, 2000.0, 256.0, 256, 5e-4, 500000
# coarse propagator of its initial coarse run (the slice states the steps
# start from): SBDF2 on 64^2 with dt = 2.5e-3, stable over [0, 256]
NC5, DTC5 = 64, 2.5e-3
ALG_BYTES_PER_MODE_STEP = 192.0    # read + write b and H, 3 x complex128, full grid
HBM_PEAK_GBS = 8000.0
CPU_WORKERS_MAX = 16               # at most a single-GPU host share of its cores
UNBLOCKED_STEPS = 5                # steps timed kernel by kernel before the blocked sweep


def box_m(n):
    return 2 * ((n - 1) // 3) + 1


def kernel_bytes(n, fields):
    """Algorithmic HBM bytes of one launch of each phase kernel (complex128):
    column phase reads T1 and writes T2 (3 M N values each); row phase reads
    T2, reads and writes state and history (3 M^2 each) and writes T1."""
    m = box_m(n)
    cols = fields * 2 * 3 * m * n * 16
    rows = fields * (2 * 3 * m * n + 4 * 3 * m * m) * 16
    return cols, rows


def _oracle_steps(job):
    """One worker of the CPU baseline: the oracle's fine SBDF2 steps on one
    seeded 512^2 field (no numerical input comes from the GPU)."""
    seed, t0, nsteps = job
    from oracle import stepper
    from synthetic import initial_field
    try:
        from threadpoolctl import threadpool_limits
        threadpool_limits(1)
    except Exception:
        pass
    b = initial_field(N5, KZ, seed, amp=1.0, kmax=40.0)
    t = time.perf_counter()
    stepper.propagate(b, "gp", RM5, KZ, t0, DT5, nsteps)
    return time.perf_counter() - t


def _one_thread():
    try:
        from threadpoolctl import threadpool_limits
        threadpool_limits(1)
    except Exception:
        pass


def _oracle_parareal_config1(workers):
    """The oracle's Parareal on the Roberts 32^2 workload (Rm = 10, kz = 1,
    T = 8 over 8 slices, fine dt = 1e-3, coarse dt = 1e-2, tol 1e-8) with
    the fine solves of each iteration on worker processes, and its serial
    fine solve, both timed."""
    import multiprocessing as mp
    from oracle import parareal as opr
    from oracle import stepper
    from synthetic import initial_field
    N1, kz1, Rm1, T1, P1, dtf1, dtc1 = 32, 1.0, 10.0, 8.0, 8, 1e-3, 1e-2
    b0 = initial_field(N1, kz1, 100000)
    F = stepper.SliceSolver("roberts", Rm1, kz1, N1, T1 / P1, dtf1)
    G = stepper.SliceSolver("roberts", Rm1, kz1, N1, T1 / P1, dtc1)
    nw = max(1, min(workers, P1))
    t0 = time.perf_counter()
    opr.serial_fine(b0, P1, T1 / P1, F)
    serial_s = time.perf_counter() - t0
    with mp.get_context("fork").Pool(nw, initializer=_one_thread) as pool:
        t0 = time.perf_counter()
        r = opr.parareal(b0, P1, T1 / P1, F, G, tol=1e-8, max_iter=P1,
                         fmap=lambda fn, xs, ts: pool.starmap(fn, zip(xs, ts)))
        par_s = time.perf_counter() - t0
    return {"workload": "Roberts Rm=10, kz=1, 32^2, T=8 over 8 slices, fine dt=1e-3, coarse "
                        "dt=1e-2, tol 1e-8", "k_con": r.k_con, "time_s": par_s,
            "serial_fine_s": serial_s, "workers": nw, "speedup": serial_s / par_s}


def cpu_baseline(budget_s=15.0):
    """The FP64 oracle's fine propagator, timed on the host's cores on a
    bounded sample of the headline workload: one seeded 512^2 field per
    worker process (as the paper's time-parallel layout gives each processor
    its own slice), each advanced by the same number of fine steps, sized to
    about `budget_s` of work a worker; and the oracle's whole Parareal on the
    small Roberts workload with its fine solves on worker processes.  Runs
    before the GPU is touched (the workers are forked)."""
    import multiprocessing as mp
    ncpu = os.cpu_count() or 1
    workers = max(1, min(ncpu, CPU_WORKERS_MAX))
    per_step = _oracle_steps((SEED5 + 999, 0.0, 1))      # one step, also warms the caches
    nsteps = max(2, min(400, int(budget_s / max(per_step, 1e-3))))
    jobs = [(SEED5 + 1000 + w, float(w), nsteps) for w in range(workers)]
    t0 = time.perf_counter()
    with mp.get_context("fork").Pool(workers) as pool:
        per = pool.map(_oracle_steps, jobs)
    wall = time.perf_counter() - t0
    done = workers * nsteps * N5 * N5
    par = _oracle_parareal_config1(workers)
    return {"value": done / wall, "unit": "fine mode-steps/s", "cores": workers,
            "host_cpu_count": ncpu, "kind": "oracle", "parareal": par,
            "sample": f"{workers} worker processes x {nsteps} fine SBDF2 steps of one seeded "
                      f"{N5}^2 field each (Rm={RM5:g}), {wall:.1f} s wall, "
                      f"{min(per):.1f}-{max(per):.1f} s a worker; a whole slice is 2000 steps"}


KERNEL_SOURCES = ("kernels.hip", "fft.hpp", "launch.hpp")
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic_gp128_p64.json")
TRAFFIC_FILE5 = os.path.join(ROOT, "profiles", "traffic_gp512_p256.json")


def kernels_digest():
    """Digest of the fine-step kernel sources (counters go stale when they change)."""
    import hashlib
    h = hashlib.sha256()
    for name in KERNEL_SOURCES:
        with open(os.path.join(ROOT, "paper_1902_00387_amd", "csrc", name), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def summarize_trace(trace_csv, steps, fields):
    """Kernel-trace summary of a blocked fine sweep (--kernel-only
    --blocked-only): per phase kernel, dispatches over `fields` slices with the
    groups' size (Grid_Size_Y) and their mean duration, and the span from the
    first start to the last end of all those dispatches divided by `steps`,
    the sweep's time a step."""
    import csv
    rows = list(csv.DictReader(open(trace_csv)))
    def kname(r):
        n = r["Kernel_Name"].split("(")[0]
        return n[5:] if n.startswith("void ") else n
    ks = [r for r in rows if kname(r).startswith(("pd::k_cols", "pd::k_rows"))]
    # the sweep's launches are the group launches after its start, the last
    # whole-batch launch of the program (the inverse-only row launch of step
    # 0; the autotuner's launches, whole-batch and grouped, come before it)
    ks.sort(key=lambda r: int(r["Start_Timestamp"]))
    last_full = max(i for i, r in enumerate(ks) if int(r["Grid_Size_Y"]) == int(fields))
    ks = ks[last_full + 1:]
    from collections import Counter
    gy = Counter(int(r["Grid_Size_Y"]) for r in ks).most_common(1)[0][0]
    ks = [r for r in ks if int(r["Grid_Size_Y"]) == gy]
    out = {"dispatches": len(ks), "kernels": {}}
    for r in ks:
        name = kname(r)
        d = out["kernels"].setdefault(name, {"calls": 0, "total_us": 0.0, "group": int(r["Grid_Size_Y"])})
        d["calls"] += 1
        d["total_us"] += (int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) * 1e-3
    for d in out["kernels"].values():
        d["mean_us"] = d["total_us"] / d["calls"]
    t0 = min(int(r["Start_Timestamp"]) for r in ks)
    t1 = max(int(r["End_Timestamp"]) for r in ks)
    out["span_ms"] = (t1 - t0) * 1e-6
    out["steps"] = int(steps)
    out["span_ms_per_step"] = out["span_ms"] / int(steps)
    out["sum_kernel_ms_per_step"] = sum(d["total_us"] for d in out["kernels"].values()) * 1e-3 / int(steps)
    return out


def summarize_pmc(fetch_csv, write_csv, out_path):
    """Per-dispatch HBM traffic of the fine step's kernels from two rocprofv3
    --pmc runs (FETCH_SIZE, WRITE_SIZE; KiB per dispatch), scaled by the same
    counters on a plain 1 GiB device copy."""
    import csv
    import statistics

    def per_kernel(path):
        # dispatches over the whole batch only (the largest grid of each
        # kernel): the autotuner's blocked-sweep candidates launch the same
        # kernels over groups of a few fields
        rows = list(csv.DictReader(open(path)))
        big = {}
        for r in rows:
            big[r["Kernel_Name"]] = max(big.get(r["Kernel_Name"], 0), int(r["Grid_Size"]))
        acc = {}
        for r in rows:
            if "copyBuffer" in r["Kernel_Name"] or int(r["Grid_Size"]) == big[r["Kernel_Name"]]:
                acc.setdefault(r["Kernel_Name"], []).append(float(r["Counter_Value"]))
        return acc
    fetch, write = per_kernel(fetch_csv), per_kernel(write_csv)
    copy_bytes = float(1 << 30)
    # the calibration copy is the program's last device copy (earlier copies
    # are the library's own state copies)
    cf = [v for k, vs in fetch.items() if "copyBuffer" in k for v in vs][-1] * 1024.0
    cw = [v for k, vs in write.items() if "copyBuffer" in k for v in vs][-1] * 1024.0
    out = {"kernels_sha256_16": kernels_digest(), "fetch_scale": copy_bytes / cf,
           "write_scale": copy_bytes / cw, "kernels": {}}
    for name in fetch:
        if "k_rows" not in name and "k_cols" not in name:
            continue
        f = statistics.median(fetch[name]) * 1024.0 * out["fetch_scale"]
        w = statistics.median(write.get(name, [0.0])) * 1024.0 * out["write_scale"]
        out["kernels"][name] = {"fetch_bytes": f, "write_bytes": w, "dispatches": len(fetch[name])}
    with open(out_path, "w") as fh:
        json.dump(out, fh, indent=1)
    return out


def measured_traffic(kernel_prefix, path=TRAFFIC_FILE):
    """HBM bytes per launch of the kernel from the committed counter summary,
    or None if the summary is missing or the kernels changed since."""
    try:
        with open(path) as fh:
            d = json.load(fh)
    except (OSError, ValueError):
        return None
    if d.get("kernels_sha256_16") != kernels_digest():
        return None
    # kernel_prefix names the leading template arguments, e.g. pd::k_rows<128,4,1>
    # for the instantiation pd::k_rows<128, 4, 1, 0>
    key = kernel_prefix.replace(" ", "").rstrip(">")
    for name, v in d["kernels"].items():
        full = name.split("(")[0].replace(" ", "")
        full = full[4:] if full.startswith("void") else full
        if full.startswith(key) and full[len(key):len(key) + 1] in (",", ">"):
            return v["fetch_bytes"] + v["write_bytes"]
    return None


def batch_workload(scale=1.0):
    """Many independent Galloway-Proctor problems of uneven size: 96 at 64^2,
    96 at 128^2 and 64 at 256^2 (times `scale`), Rm log-uniform in [10, 1000],
    kz uniform in [0.2, 1.2], T = 32 over 32 slices.  Fine steps per unit time
    ceil(2 A K / 0.2), coarse grid N/2 with ceil(2 A K_C / 0.4) steps per unit
    time (A = sqrt(3/2), K = floor((N-1)/3))."""
    from synthetic import gp_instance_params, initial_field
    counts = [(64, 96), (128, 96), (256, 64)]
    specs = []
    for N, cnt in counts:
        specs += [N] * max(1, int(round(cnt * scale)))
    rm, kz = gp_instance_params(len(specs), 300000)
    A = math.sqrt(1.5)
    out = []
    for i, N in enumerate(specs):
        K, Nc = (N - 1) // 3, N // 2
        Kc = (Nc - 1) // 3
        nf = math.ceil(2 * A * K / 0.2)
        nc = math.ceil(2 * A * Kc / 0.4)
        out.append(dict(N=N, Nc=Nc, Rm=float(rm[i]), kz=float(kz[i]), T=32.0, P=32,
                        dtf=1.0 / nf, dtc=1.0 / nc, nf=nf, seed=300000 + i))
    return out


def run_batch(args):
    import numpy as np
    import torch

    import paper_1902_00387_amd as pd
    from synthetic import initial_field
    inst = batch_workload(args.batch_scale)
    # launch shapes of each grid's step kernels, timed on a slice batch the
    # size of that grid's share of the workload (process-wide choice)
    tuned = {}
    for N in sorted({it["N"] for it in inst}):
        fields = sum(it["P"] for it in inst if it["N"] == N)
        tc = pd.Context(0)
        tc.set_problem("gp", 100.0, 0.57, N)
        tc.set_time(float(fields), fields, 1.0 / 64, 1.0 / 16, N // 2)
        tc.set_initial(torch.from_numpy(initial_field(N, 0.57, 1)).cuda())
        tc.parareal(0.0, 0)
        tuned[N] = tc.autotune(5)[0]
        tc.close()
        # the batch runs the process-wide launch shapes: make the tuned ones so
        pd.select_variant(N, *tuned[N])
    print(f"# batch autotune (rows, cols variant per N): {tuned}", file=sys.stderr, flush=True)
    b = pd.Batch(0)
    for it in inst:
        b.add("gp", it["Rm"], it["kz"], it["N"], it["T"], it["P"], it["dtf"], it["dtc"], it["Nc"],
              initial_field(it["N"], it["kz"], it["seed"]))
    print(f"# batch: {len(inst)} instances", file=sys.stderr, flush=True)
    t0 = time.perf_counter()
    st = b.run(TOL, 33, use_graph=True)   # first run builds buffers and captures the graph
    torch.cuda.synchronize()
    print(f"# batch: first run (graph capture) {time.perf_counter() - t0:.1f} s", file=sys.stderr, flush=True)
    times = []
    for i in range(max(1, args.steps)):
        t0 = time.perf_counter()
        st = b.run(TOL, 33, use_graph=True)
        torch.cuda.synchronize()
        times.append(time.perf_counter() - t0)
        print(f"# batch: timed run {i + 1}: {times[-1]:.1f} s", file=sys.stderr, flush=True)
    secs = min(times)
    reps = [b.result(i) for i in range(len(inst))]
    done_ms = 0.0
    serial_ms = 0.0
    for it, r in zip(inst, reps):
        P, nf, N = it["P"], it["nf"], it["N"]
        serial_ms += P * nf * N * N
        for k in range(1, r["iters"] + 1):
            done_ms += (P - min(k - 1, P - 1)) * nf * N * N
    kc = [r["k_con"] for r in reps]
    out = {
        "metric": "batched instances: serial-equivalent fine mode-steps/sec (Parareal to sigma<=1e-8)",
        "value": serial_ms / secs, "unit": "mode-steps/s", "n_gpus": 1,
        "status": st, "seconds": secs, "instances": len(inst),
        "fine_mode_steps_computed_per_s": done_ms / secs,
        "k_con": {"min": min(kc), "max": max(kc), "mean": float(np.mean(kc)),
                  "not_converged": int(sum(1 for k in kc if k < 0))},
        "growth_rate_range": [float(min(r["growth_rate"] for r in reps)),
                              float(max(r["growth_rate"] for r in reps))],
        "dtype": "c128", "data": "synthetic",
        "config": {"workload": f"{len(inst)} GP instances (64^2/128^2/256^2 = 3:3:2), Rm log-U[10,1000], "
                               "kz U[0.2,1.2], 32 slices, T=32, coarse N/2, tol 1e-8, HIP graph"},
        "autotune": {str(k): list(v) for k, v in tuned.items()},
    }
    b.close()
    print(json.dumps(out), flush=True)


def learned_workload():
    """Learned-versus-plain coarse propagator: Galloway-Proctor flow, Rm = 500,
    kz = 0.57, 256 x 256, T = 64 over 128 slices (slice length 0.5), fine
    SBDF2 dt = 1e-3."""
    return dict(N=256, Rm=500.0, kz=0.57, T=64.0, P=128, dtf=1e-3, seed=400000)


def coarse_choice(ctx, w, b0, fine_norm_T):
    """Largest N_C in {N/2, N/4} and Delta t in {1e-2, 5e-3, 2.5e-3} (halved
    until one passes) whose initial coarse run over [0, T] stays finite and
    within 1e3 of the fine solution's norm at T."""
    import numpy as np
    for dtc in (1e-2, 5e-3, 2.5e-3):
        for nc in (w["N"] // 2, w["N"] // 4):
            ctx.set_time(w["T"], w["P"], w["dtf"], dtc, nc)
            ctx.set_initial(b0)
            ctx.parareal(0.0, 0)
            nrm = ctx.slice_norms()
            ok = bool(np.all(np.isfinite(nrm))) and nrm[-1] <= 1e3 * fine_norm_T
            print(f"# coarse pre-check N_C={nc} dt={dtc}: |U_P|={nrm[-1]:.3e} "
                  f"(fine {fine_norm_T:.3e}) {'ok' if ok else 'rejected'}", file=sys.stderr, flush=True)
            if ok:
                return nc, dtc
    raise RuntimeError("no stable coarse propagator among the candidates")


def run_learned(args):
    """Time to sigma <= 1e-8 with the plain and the learned coarse propagator
    (plus the serial fine solve on the same GPU), and the training cost."""
    import torch

    import paper_1902_00387_amd as pd
    from synthetic import initial_field
    import numpy as np
    w = learned_workload()
    N, P, T = w["N"], w["P"], w["T"]
    nf = int(round(T / P / w["dtf"]))
    dev = torch.device("cuda:0")
    b0 = torch.from_numpy(initial_field(N, w["kz"], w["seed"])).to(dev)
    ctx = pd.Context(0)
    ctx.set_problem("gp", w["Rm"], w["kz"], N)
    ctx.set_time(T, P, w["dtf"], 1e-2, N // 2)
    # serial fine solve (slices one after another, batch 1)
    u = b0[None].clone()
    torch.cuda.synchronize()
    ts = time.perf_counter()
    for n in range(P):
        u = ctx.fine([n * T / P], u)
    torch.cuda.synchronize()
    serial_s = time.perf_counter() - ts
    fine_norm_T = float(torch.linalg.vector_norm(u).item())
    print(f"# serial fine solve {serial_s:.2f} s, |b(T)| = {fine_norm_T:.3e}", file=sys.stderr, flush=True)
    if args.lg_nc > 0:
        nc, dtc = args.lg_nc, args.lg_dtc
    else:
        nc, dtc = coarse_choice(ctx, w, b0, fine_norm_T)
    ctx.set_time(T, P, w["dtf"], dtc, nc)

    def solve(learned):
        switch = args.lg_switch if learned else 0
        ctx.set_coarse(learned and switch == 0)
        ctx.set_initial(b0)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        rep = ctx.parareal(TOL, switch if switch > 0 else P + 1)
        if switch > 0 and rep["k_con"] < 0:
            # plain G for the first iterations, then the learned propagator
            sig = list(rep["sigma"])
            ctx.set_coarse(True)
            rep = ctx.parareal_continue(TOL, P + 1)
            rep["sigma"] = sig + rep["sigma"][len(sig):]
        gam = ctx.growth_rate()
        torch.cuda.synchronize()
        return rep, gam, time.perf_counter() - t0

    solve(False)
    rp, gp, tp = solve(False)
    Up = ctx.get_slices_dev()[P].clone()
    print(f"# plain G: k_con {rp['k_con']} in {tp:.2f} s", file=sys.stderr, flush=True)
    # training pairs from the fine and coarse propagators: seeded random
    # fields (diverse inputs for a linear map) and the coarse inputs of
    # plain-G Parareal runs from two more initial fields (iteration k of a run
    # contributes U^k_n - U^{k-1}_n, n >= k)
    rng = np.random.default_rng(w["seed"] + 1)
    ctx.lg_init(4, w["seed"])
    tg = time.perf_counter()
    n_fields = args.lg_random
    for a in range(0, n_fields, 64):
        D = np.stack([initial_field(N, w["kz"], w["seed"] + 10 + i, amp=1.0,
                                    kmax=float(rng.uniform(2.0, 40.0)))
                      for i in range(a, min(a + 64, n_fields))])
        tt = rng.integers(0, P, D.shape[0]) * (T / P)
        ctx.lg_add_samples(tt, torch.from_numpy(D).to(dev))
    H = args.lg_harvest
    block = P * (H + 1) - H * (H + 1) // 2           # samples of one harvested run
    starts = []
    for r in range(2):
        ctx.set_coarse(False)
        ctx.set_initial(torch.from_numpy(initial_field(N, w["kz"], w["seed"] + 1000 + r)).to(dev))
        starts.append(n_fields + r * block)
        n_samples = ctx.lg_add_parareal_samples(H)
    torch.cuda.synchronize()
    gen_s = time.perf_counter() - tg
    print(f"# {n_samples} training pairs in {gen_s:.1f} s", file=sys.stderr, flush=True)
    steps = args.lg_steps
    if args.lg_late > 0:
        # only the differences of iterations k >= K0: the error that persists
        K0 = args.lg_late
        skip = P + (K0 - 1) * P - (K0 - 1) * K0 // 2
        tr0, trn = starts[0] + skip, block - skip
        va0, van = starts[1] + skip, min(64, block - skip)
    else:
        tr0, trn = 0, n_samples - 64
        va0, van = n_samples - 64, 64
    ttr = time.perf_counter()
    val0 = ctx.lg_loss(va0, van)
    losses = ctx.lg_train(tr0, trn, steps, 8, 1e-3, seed=5)
    val1 = ctx.lg_loss(va0, van)
    train_s = time.perf_counter() - ttr
    print(f"# training {steps} steps on {trn} pairs {train_s:.1f} s: held-out loss "
          f"{val0:.3f} -> {val1:.3f}", file=sys.stderr, flush=True)
    solve(True)
    rl, gl, tl = solve(True)
    Ul = ctx.get_slices_dev()[P]
    diff = float(torch.linalg.vector_norm(Ul - Up).item() / torch.linalg.vector_norm(Up).item())
    print(f"# learned G: k_con {rl['k_con']} in {tl:.2f} s", file=sys.stderr, flush=True)
    ctx.close()
    out = {
        "metric": "time to Parareal defect <= 1e-8, learned vs plain coarse propagator",
        "value": tl, "unit": "s", "higher_is_better": False, "n_gpus": 1,
        "dtype": "c128 fine / bf16-fp32 network", "data": "synthetic",
        "config": {"workload": "Galloway-Proctor Rm=500, kz=0.57, 256x256, T=64 over 128 slices, "
                               f"fine SBDF2 dt=1e-3 ({nf} steps a slice), coarse SBDF2 on {nc}^2 dt={dtc}, "
                               "network 4 layers width 32",
                   "N_coarse": nc, "dt_coarse": dtc},
        "plain": {"k_con": rp["k_con"], "time_s": tp, "growth_rate": gp,
                  "t_fine_s": rp["t_fine_s"], "t_coarse_s": rp["t_coarse_s"] + rp["t_coarse0_s"],
                  "sigma": rp["sigma"][:rp["iters"]]},
        "learned": {"k_con": rl["k_con"], "time_s": tl, "growth_rate": gl,
                    "plain_iterations_first": args.lg_switch,
                    "t_fine_s": rl["t_fine_s"], "t_coarse_s": rl["t_coarse_s"] + rl["t_coarse0_s"],
                    "sigma": rl["sigma"][:rl["iters"]], "final_state_reldiff_vs_plain": diff},
        "serial_fine_gpu_s": serial_s,
        "speedup_vs_serial": {"plain": serial_s / tp, "learned": serial_s / tl},
        "training": {"pairs": n_samples, "trained_on": [tr0, trn], "held_out": [va0, van],
                     "generate_s": gen_s, "train_s": train_s, "steps": steps,
                     "batch": 8, "held_out_loss": [val0, val1], "last_batch_loss": losses[-1]},
    }
    print(json.dumps(out), flush=True)


def _solve_in_pieces(ctx, tol, cap, piece, label):
    """Parareal to sigma <= tol (at most `cap` iterations) in pieces of
    `piece` iterations (pd_parareal, then pd_parareal_continue), one progress
    line a piece; returns (report of the last piece, sigma of every
    iteration, seconds)."""
    import torch
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    rep = ctx.parareal(tol, min(piece, cap))
    sig = list(rep["sigma"])
    _log(f"# {label}: iteration {rep['iters']}, sigma {sig[-1]:.3e}, {time.perf_counter() - t0:.1f} s")
    while rep["k_con"] < 0 and rep["iters"] < cap:
        rep = ctx.parareal_continue(tol, min(rep["iters"] + piece, cap))
        sig += rep["sigma"][len(sig):]
        _log(f"# {label}: iteration {rep['iters']}, sigma {sig[-1]:.3e}, "
             f"{time.perf_counter() - t0:.1f} s")
    torch.cuda.synchronize()
    return rep, sig, time.perf_counter() - t0


def run_learned5(args):
    """Learned against plain coarse propagator on the 512^2, 256-slice
    workload (Rm = 2000): time and iterations to sigma <= tol, each solve run
    in pieces of a few iterations; the network (BF16 matrix-core operands) is
    trained on the GPU on the coarse-propagator inputs of iterations k >= K0
    of a plain-G run from another seeded field."""
    import torch

    import paper_1902_00387_amd as pd
    nc, dtc, cap, tol = args.p5_nc, args.p5_dtc, args.l5_iters, args.l5_tol
    piece = 4
    ctx = pd.Context(0)
    ctx.set_problem("gp", RM5, KZ, N5)
    ctx.set_time(T5, P5, DT5, dtc, nc)
    ctx.seed_initial(SEED5, 1e-3, 4.0)
    ctx.parareal(0.0, 0)
    ctx.autotune(3)
    _log(f"# blocking {ctx.fine_blocking()}")
    b0 = ctx.get_slices_dev()[0:1].clone()
    torch.cuda.synchronize()
    ts = time.perf_counter()
    u = b0
    for n in range(P5):
        u = ctx.fine([n * T5 / P5], u)
        if n % 128 == 127:
            _log(f"# serial fine: slice {n + 1}/{P5}, {time.perf_counter() - ts:.1f} s")
    torch.cuda.synchronize()
    serial_s = time.perf_counter() - ts
    del u

    def solve(learned):
        ctx.set_coarse(False)
        ctx.seed_initial(SEED5, 1e-3, 4.0)
        if learned and args.l5_switch > 0:
            # plain G for the first iterations, then the learned propagator
            # (trained on the differences of later iterations)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            r0 = ctx.parareal(tol, args.l5_switch)
            sig0 = list(r0["sigma"])
            ctx.set_coarse(True)
            rep = r0
            sig = sig0
            while rep["k_con"] < 0 and rep["iters"] < cap:
                rep = ctx.parareal_continue(tol, min(rep["iters"] + piece, cap))
                sig += rep["sigma"][len(sig):]
                _log(f"# plain then learned G: iteration {rep['iters']}, sigma {sig[-1]:.3e}, "
                     f"{time.perf_counter() - t0:.1f} s")
            torch.cuda.synchronize()
            return rep, sig, time.perf_counter() - t0, ctx.growth_rate()
        ctx.set_coarse(learned)
        rep, sig, secs = _solve_in_pieces(ctx, tol, cap, piece, "learned G" if learned else "plain G")
        return rep, sig, secs, ctx.growth_rate()

    rp, sp, tp, gp = solve(False)
    Up = ctx.get_slices_dev()[P5].clone()
    # training pairs: the coarse inputs U^k_n - U^{k-1}_n of a plain-G run
    # from another seeded field, iterations k >= K0 (the error that persists)
    H, K0, steps = args.l5_harvest, args.lg_late, args.l5_steps
    ctx.lg_init(4, SEED5)
    tg = time.perf_counter()
    ctx.set_coarse(False)
    ctx.seed_initial(SEED5 + 1000, 1e-3, 4.0)
    n_samples = ctx.lg_add_parareal_samples(H)
    torch.cuda.synchronize()
    gen_s = time.perf_counter() - tg
    _log(f"# {n_samples} training pairs in {gen_s:.1f} s")
    skip = P5 + (K0 - 1) * P5 - (K0 - 1) * K0 // 2
    va_n = 64
    tr0, trn = skip, n_samples - skip - va_n
    va0 = n_samples - va_n
    val0 = ctx.lg_loss(va0, va_n)
    ttr = time.perf_counter()
    done = 0
    last = float("nan")
    while done < steps:
        k = min(250, steps - done)
        losses = ctx.lg_train(tr0, trn, k, 8, 1e-3, seed=5 + done)
        done += k
        last = float(losses[-1])
        _log(f"# training: {done}/{steps} steps, batch loss {last:.3f}, "
             f"{time.perf_counter() - ttr:.1f} s")
    val1 = ctx.lg_loss(va0, va_n)
    train_s = time.perf_counter() - ttr
    _log(f"# held-out loss {val0:.3f} -> {val1:.3f}")
    rl, sl, tl, gl = solve(True)
    Ul = ctx.get_slices_dev()[P5]
    diff = float(torch.linalg.vector_norm(Ul - Up).item() / torch.linalg.vector_norm(Up).item())
    ctx.close()
    out = {
        "experiment": "learned vs plain coarse propagator on the 512^2, 256-slice workload",
        "config": {"workload": "Galloway-Proctor Rm=2000, kz=0.57, 512x512, T=256 over 256 slices, "
                               f"fine SBDF2 dt=5e-4, coarse SBDF2 on {nc}^2 dt={dtc}, tol {tol:g}, "
                               "network 4 layers width 32 (BF16 operands)"},
        "plain": {"k_con": rp["k_con"], "iters": rp["iters"], "time_s": tp, "growth_rate": gp,
                  "sigma": sp},
        "learned": {"k_con": rl["k_con"], "iters": rl["iters"], "time_s": tl, "growth_rate": gl,
                    "plain_iterations_first": args.l5_switch,
                    "sigma": sl, "final_state_reldiff_vs_plain": diff},
        "serial_fine_gpu_s": serial_s,
        "training": {"pairs": n_samples, "harvest_iterations": H, "trained_on": [tr0, trn],
                     "held_out": [va0, va_n], "generate_s": gen_s, "train_s": train_s,
                     "steps": steps, "batch": 8, "held_out_loss": [val0, val1],
                     "last_batch_loss": last},
    }
    print(json.dumps(out), flush=True)


def _log(msg):
    print(msg, file=sys.stderr, flush=True)


def _serial_fine(ctx, b0, P, dT):
    """Serial fine solve on the GPU: slice after slice, batch 1; returns the
    slice-boundary norms and the seconds taken."""
    import torch
    u = b0[None].clone()
    norms = [float(torch.linalg.vector_norm(u).item())]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for n in range(P):
        u = ctx.fine([n * dT], u)
        norms.append(float(torch.linalg.vector_norm(u).item()))
    torch.cuda.synchronize()
    return norms, time.perf_counter() - t0


def _growth(norms, dT):
    """Least-squares slope of ln|U_n| over n = ceil(P/2)..P (the estimator
    pd_growth_rate uses)."""
    import numpy as np
    P = len(norms) - 1
    n = np.arange((P + 1) // 2, P + 1)
    return float(np.polyfit(n * dT, np.log(np.asarray(norms)[n]), 1)[0])


def nc_sweep_workload(args):
    """The coarse-grid sweep's workloads.  roberts: the paper's Section 5.2
    study (its speed-up-vs-N_C figure): Roberts flow, Rm = 512, kz = 2.87,
    N_F = 128 or 256 (powers of two around the paper's 160), fine ARS(4,4,3)
    with dt = 1e-2 (5e-3 on 256^2), 10 slices of length 1, tolerance 1e-5 (the
    paper's accuracy target).  gp128: the headline workload (Galloway-Proctor,
    Rm = 100, kz = 0.57, 128^2, 64 slices of length 1, fine SBDF2 dt = 2e-3,
    SBDF2 coarse propagator, tolerance 1e-8)."""
    if args.nc_sweep_gp:
        return dict(flow="gp", Rm=RM, kz=KZ, N=N, P=P, T=T, dtf=DT_FINE, scheme="sbdf2",
                    seed=SEED, tol=TOL, nc_list=(N // 4, N // 2, N),
                    dtc_cands=(2e-2, 1e-2, 5e-3, 2.5e-3))
    NF = args.nc_nf
    return dict(flow="roberts", Rm=512.0, kz=2.87, N=NF, P=10, T=10.0,
                dtf=1e-2 if NF <= 128 else 5e-3,  # largest stable ARS(4,4,3) step of the grid
                scheme="rk443", seed=500000, tol=args.nc_tol,
                nc_list=(NF // 8, NF // 4, NF // 2, NF),
                dtc_cands=(0.1, 0.05, 0.025, 0.0125, 0.00625, 0.003125))


def run_nc_sweep(args):
    """Coarse-grid sweep (nc_sweep_workload).  For every N_C the coarse step
    is the largest candidate whose coarse-only run is still as accurate at T
    as the smallest step allows (error against the serial fine solution
    within twice the smallest-step error: accuracy limited by the grid, not by
    the step).  Reported: k_con, R_f/R_c, time to solution (the library's default, pipelined, order), speed-up
    over the serial fine solve on the same GPU, and the paper's speed-up model
    (eq. speed_up) for as many processors as slices."""
    import numpy as np
    import torch

    import paper_1902_00387_amd as pd
    from synthetic import initial_field
    w = nc_sweep_workload(args)
    N, Rm, kz, P, T, tol, dtf = w["N"], w["Rm"], w["kz"], w["P"], w["T"], w["tol"], w["dtf"]
    b0 = torch.from_numpy(initial_field(N, kz, w["seed"])).cuda()
    ctx = pd.Context(0)
    ctx.set_problem(w["flow"], Rm, kz, N)
    ctx.set_time(T, P, dtf, dtf, N)
    ctx.set_scheme(w["scheme"], w["scheme"])
    u = b0[None].clone()
    ctx.fine([0.0], u)  # warm-up (first launches)
    torch.cuda.synchronize()
    ts = time.perf_counter()
    for n in range(P):
        u = ctx.fine([n * T / P], u)
    torch.cuda.synchronize()
    serial_s = time.perf_counter() - ts
    uT = u[0].cpu().numpy()
    _log(f"# serial fine {serial_s:.3f} s, |b(T)| {np.linalg.norm(uT):.3e}")
    rows = []
    for nc in w["nc_list"]:
        errs = {}
        for cand in w["dtc_cands"]:
            ctx.set_time(T, P, dtf, cand, nc)
            ctx.set_initial(b0)
            ctx.parareal(0.0, 0)
            g = ctx.get_slices()[P]
            e = float(np.linalg.norm(g - uT) / np.linalg.norm(uT))
            errs[cand] = e if np.isfinite(e) else float("inf")
        emin = min(errs.values())
        dtc = max(c for c, e in errs.items() if e <= 2.0 * emin)
        _log(f"# N_C={nc}: coarse-run errors " + ", ".join(f"{c:g}: {e:.2e}" for c, e in errs.items())
             + f" -> dt_c {dtc:g}")
        ctx.set_time(T, P, dtf, dtc, nc)
        ctx.set_initial(b0)
        ctx.parareal(tol, P + 1)  # warm-up
        ctx.set_initial(b0)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        rep = ctx.parareal(tol, P + 1)
        torch.cuda.synchronize()
        tp = time.perf_counter() - t0
        # R_f / R_c: one slice of F against one slice of G (batch 1)
        x = b0[None].clone()
        for fn in (ctx.fine, ctx.coarse):
            fn([0.0], x)
        torch.cuda.synchronize()
        tf = time.perf_counter()
        for _ in range(3):
            ctx.fine([0.0], x)
        torch.cuda.synchronize()
        tf = (time.perf_counter() - tf) / 3
        tc = time.perf_counter()
        for _ in range(3):
            ctx.coarse([0.0], x)
        torch.cuda.synchronize()
        tc = (time.perf_counter() - tc) / 3
        k = rep["k_con"]
        model = 1.0 / ((1.0 + k / P) * (tc / tf) + k / P) if k > 0 else None
        rows.append({"N_coarse": nc, "dt_coarse": dtc, "coarse_run_error": errs[dtc], "k_con": k,
                     "sigma": rep["sigma"][:rep["iters"]], "time_s": tp, "Rf_over_Rc": tf / tc,
                     "speedup_vs_serial_gpu": serial_s / tp, "model_speedup": model})
        _log(f"# N_C={nc} dt_c={dtc}: k_con {k}, {tp:.3f} s, Rf/Rc {tf / tc:.1f}, "
             f"speed-up {serial_s / tp:.2f} (model {model})")
    ctx.close()
    print(json.dumps({"experiment": "coarse grid sweep", "flow": w["flow"], "Rm": Rm, "kz": kz,
                      "N_coarse_list": [r["N_coarse"] for r in rows],
                      "N_fine": N, "dt_fine": dtf, "slices": P, "T": T, "scheme": w["scheme"],
                      "tol": tol, "model_processors": P,
                      "serial_fine_gpu_s": serial_s, "rows": rows}), flush=True)


def run_work_precision(args):
    """Work against accuracy of the fine steppers (the paper's Section 5.1
    comparison of RK111, RK222 and RK443, plus SBDF2): Galloway-Proctor,
    Rm = 300, N = 256, from t = 0 to 1; error
    = relative two-norm against ARS(4,4,3) at dt = 1.25e-4; work = explicit
    evaluations (steps x stages) and GPU time (batch 1)."""
    import torch

    import paper_1902_00387_amd as pd
    from synthetic import initial_field
    N, Rm, kz = 256, 300.0, 0.57
    b0 = torch.from_numpy(initial_field(N, kz, 600000, amp=1.0)).cuda()[None]
    ctx = pd.Context(0)
    ctx.set_problem("gp", Rm, kz, N)

    def solve(scheme, dt):
        ctx.set_scheme(scheme, scheme)
        n = int(round(1.0 / dt))
        ctx.steps([0.0], dt, n, b0)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        y = ctx.steps([0.0], dt, n, b0)
        torch.cuda.synchronize()
        return y, time.perf_counter() - t0, n
    ref, _, _ = solve("rk443", 1.25e-4)
    rn = float(torch.linalg.vector_norm(ref).item())
    rows = []
    for scheme, stages in (("sbdf2", 1), ("rk111", 1), ("rk222", 2), ("rk443", 4)):
        for dt in (1e-2, 5e-3, 2.5e-3, 1.25e-3, 6.25e-4, 2.5e-4):
            y, secs, n = solve(scheme, dt)
            err = float(torch.linalg.vector_norm(y - ref).item()) / rn
            rows.append({"scheme": scheme, "dt": dt, "evaluations": n * stages, "gpu_s": secs,
                         "rel_error": err})
            _log(f"# {scheme} dt={dt}: {n * stages} evaluations, {secs * 1e3:.1f} ms, error {err:.3e}")
    ctx.close()
    print(json.dumps({"experiment": "work-precision", "flow": "gp", "Rm": Rm, "N": N, "T": 1.0,
                      "reference": "rk443 dt=1.25e-4", "rows": rows}), flush=True)


# Table 1 rows also solved by Parareal: row -> (N_C, coarse dt); the paper's
# N_C = 8 for GP Rm = 3 is below the smallest grid here, so that row coarsens
# in time only
PARAREAL_ROWS = {2: (16, 0.1), 3: (64, 2e-2)}


def run_table1(args):
    """Growth rates of the paper's Table 1 parameter sets from serial fine
    solves on the GPU over t in [0, 50] (50 slices of length 1; growth =
    least-squares slope of ln|b| over the second half).  N_F = 160 of the
    first row becomes 256 (powers of two only); steppers ARS(4,4,3) except
    SBDF2 for the dt = 1e-4 row."""
    import torch

    import paper_1902_00387_amd as pd
    from synthetic import initial_field
    rows = [("roberts", 512.0, 2.87, 256, 5e-3, "rk443", 0.11),
            ("roberts", 4096.0, 7.5, 512, 2.5e-3, "rk443", 0.097),
            ("gp", 3.0, 0.57, 16, 5e-3, "rk443", 0.15),
            ("gp", 300.0, 0.57, 128, 1e-3, "rk443", 0.3),
            ("gp", 3000.0, 0.57, 512, 1e-4, "sbdf2", 0.3)]
    only = set(int(v) for v in args.table1_rows.split(",")) if args.table1_rows else None
    out = []
    for i, (flow, Rm, kz, N, dt, scheme, paper) in enumerate(rows):
        if only is not None and i not in only:
            continue
        T, P = 50.0, 50
        ctx = pd.Context(0)
        ctx.set_problem(flow, Rm, kz, N)
        ctx.set_time(T, P, dt, dt, N)
        ctx.set_scheme(scheme, scheme)
        b0 = torch.from_numpy(initial_field(N, kz, 700000 + i)).cuda()
        u = b0[None].clone()
        norms = [float(torch.linalg.vector_norm(u).item())]
        t0 = time.perf_counter()
        for n in range(P):
            u = ctx.fine([n * 1.0], u)
            norms.append(float(torch.linalg.vector_norm(u).item()))
            if n % 10 == 9:
                _log(f"# table1 row {i} ({flow} Rm={Rm}): slice {n + 1}/{P}, {time.perf_counter() - t0:.1f} s")
        g = _growth(norms, 1.0)
        serial_s = time.perf_counter() - t0
        row = {"flow": flow, "Rm": Rm, "kz": kz, "N": N, "dt": dt, "scheme": scheme,
               "growth_rate": g, "paper": paper, "seconds": serial_s}
        _log(f"# table1 row {i}: growth {g:.4f} (paper {paper})")
        if i in PARAREAL_ROWS:
            # the same solution by Parareal with the paper's coarse propagator
            # (ARS(4,4,3) on N_C with step dt_c) and the library's growth rate
            Nc, dtc = PARAREAL_ROWS[i]
            ctx.set_time(T, P, dt, dtc, Nc)
            ctx.set_scheme(scheme, "rk443")
            ctx.set_initial(b0)
            torch.cuda.synchronize()
            tp = time.perf_counter()
            rep = ctx.parareal(1e-8, P + 1)
            gp = ctx.growth_rate()
            torch.cuda.synchronize()
            tp = time.perf_counter() - tp
            row["parareal"] = {"N_coarse": Nc, "dt_coarse": dtc, "k_con": rep["k_con"],
                               "growth_rate": gp, "seconds": tp, "speedup_vs_serial_gpu": serial_s / tp}
            _log(f"# table1 row {i} Parareal (N_C={Nc}, dt_c={dtc}): k_con {rep['k_con']}, "
                 f"growth {gp:.4f}, {tp:.2f} s vs serial {serial_s:.2f} s")
        ctx.close()
        out.append(row)
    print(json.dumps({"experiment": "Table 1 growth rates", "T": 50.0, "rows": out}), flush=True)


def run_config2(args):
    """One step = one whole Parareal solve of the 128^2 workload: Galloway-
    Proctor, Rm = 100, kz = 0.57, T = 64 over 64 slices, fine SBDF2 dt = 2e-3
    (500 steps a slice, all slices batched), coarse SBDF2 on 64^2 with
    dt = 1e-2 (the paper's N_C = N_F/2 with the largest stable step), initial
    coarse run, iterations to sigma <= 1e-8, growth rate; value = serial-
    equivalent fine mode-steps/s."""
    import torch

    import paper_1902_00387_amd as pd
    from synthetic import initial_field
    dev = torch.device("cuda:0")
    b0 = torch.from_numpy(initial_field(N, KZ, SEED)).to(dev)
    ctx = pd.Context(0)
    ctx.set_problem("gp", RM, KZ, N)
    ctx.set_time(T, P, DT_FINE, DT_COARSE, N_COARSE)
    ctx.set_path(args.path)
    if args.pipeline >= 0:
        ctx.set_pipeline(args.pipeline, args.pipeline_spec)
    nf = int(round(T / P / DT_FINE))
    # launch shapes of the fine step's kernels, picked by timing on this device
    ctx.set_initial(b0)
    ctx.parareal(0.0, 0)
    tuned, tuned_ms = ctx.autotune(10)
    print(f"# autotune: rows variant {tuned[0]} {pd.variants(N, 0)[tuned[0]]} "
          f"{tuned_ms[0]*1e3:.1f} us, cols variant {tuned[1]} {pd.variants(N, 1)[tuned[1]]} "
          f"{tuned_ms[1]*1e3:.1f} us", file=sys.stderr, flush=True)

    def solve():
        ctx.set_initial(b0)
        rep = ctx.parareal(TOL, MAX_ITER)
        gam = ctx.growth_rate()
        return rep, gam

    if args.kernel_only:
        ctx.set_initial(b0)
        ctx.parareal(0.0, 0)
        for _ in range(max(1, args.steps)):
            ctx.profile_fine(20)
        # a plain device copy of known size (1 GiB read + 1 GiB written), to
        # calibrate profiler byte counters against
        src = torch.empty(1 << 27, dtype=torch.float64, device=dev)
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"kernel_only": True, "copy_bytes_each_way": src.numel() * 8}), flush=True)
        return

    for _ in range(args.warmup):
        rep, gam = solve()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        rep, gam = solve()
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    ms_step = elapsed / args.steps * 1e3
    serial_equiv = N * N * P * nf
    value = serial_equiv / (ms_step * 1e-3)
    print(f"# solve: k_con={rep['k_con']} sigma={rep['sigma'][-1]:.2e} gamma={gam:.6f} "
          f"{ms_step:.1f} ms/solve (fine {rep['t_fine_s']*1e3:.1f} ms, coarse "
          f"{(rep['t_coarse_s'] + rep['t_coarse0_s'])*1e3:.1f} ms)", file=sys.stderr, flush=True)

    # kernel durations on the context's stream (HIP events), fine sweep rate
    ctx.set_initial(b0)
    ctx.parareal(0.0, 0)
    ms_cols, ms_rows, ms_fstep = ctx.profile_fine(20)
    cols_b, rows_b = kernel_bytes(N, P)
    dominant = ("cols", ms_cols, cols_b) if ms_cols >= ms_rows else ("rows", ms_rows, rows_b)
    achieved = dominant[2] / (dominant[1] * 1e-3) / 1e9
    re_, rw = pd.variants(N, 0)[tuned[0]]
    rows_name = "k_rows<128,%d,%d,0,%s>" % (re_, abs(rw), "true" if rw < 0 else "false")
    dom_name = ("k_cols<128,%d,%d>" % tuple(pd.variants(N, 1)[tuned[1]]) if dominant[0] == "cols"
                else rows_name)
    fine_rate = N * N * P / (ms_fstep * 1e-3)
    alg_per_mode = (cols_b + rows_b) / (N * N * P)

    # serial fine solve on the same GPU (slices one after another, batch 1)
    u = b0[None].clone()
    torch.cuda.synchronize()
    ts = time.perf_counter()
    for n in range(P):
        u = ctx.fine([n * T / P], u)
    torch.cuda.synchronize()
    serial_s = time.perf_counter() - ts

    out = {
        "metric": "Parareal time-to-1e-8 as serial-equivalent fine mode-steps/sec (whole solve)",
        "value": value,
        "unit": "mode-steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "c128",
        "data": "synthetic (seeded Gaussian solenoidal initial field, |k|<=4, amplitude 1e-3)",
        "config": {
            "workload": "Galloway-Proctor kinematic dynamo Parareal, Rm=100, kz=0.57, 128x128, "
                        "T=64 over 64 slices, fine SBDF2 dt=2e-3, coarse SBDF2 dt=1e-2 on 64x64, "
                        "tol 1e-8",
            "N": N, "slices": P, "fine_steps_per_slice": nf, "N_coarse": N_COARSE,
            "dt_fine": DT_FINE, "dt_coarse": DT_COARSE, "tol": TOL,
        },
        "parareal": {
            "k_con": rep["k_con"], "sigma": rep["sigma"], "growth_rate": gam,
            "time_to_tol_s": ms_step * 1e-3,
            "fine_sweeps_s": rep["t_fine_s"],
            "coarse_sweeps_s": rep["t_coarse_s"] + rep["t_coarse0_s"],
            "serial_fine_gpu_s": serial_s,
            "speedup_vs_serial_fine_gpu": serial_s / (ms_step * 1e-3),
            # eq. speed_up from the report's per-stream sweep times (they
            # overlap in the pipelined schedule, so R_f and R_c are overstated)
            "Rf_over_Rc": rep["Rf_over_Rc"], "model_speedup": rep["model_speedup"],
            "model_speedup_note": "eq. speed_up with R_f / R_c from the report's summed fine and "
                                  "coarse kernel times per stream; in the pipelined schedule the "
                                  "sweeps overlap, so this overstates the measured speed-up "
                                  "(speedup_vs_serial_fine_gpu)",
        },
        "autotune": {"rows_variant": list(pd.variants(N, 0)[tuned[0]]),
                     "cols_variant": list(pd.variants(N, 1)[tuned[1]]),
                     "note": "rows: (values a lane, waves a workgroup; negative: state and history loaded with the row); cols: (values a lane, columns a workgroup)"},
        "fine_sweep": {
            "mode_steps_per_s": fine_rate,
            "ms_per_fine_step_all_slices": ms_fstep,
            "ms_cols_kernel": ms_cols, "ms_rows_kernel": ms_rows,
            "algorithmic_bytes_per_mode_step": alg_per_mode,
            "algorithmic_hbm_gbs": alg_per_mode * fine_rate / 1e9,
        },
        "roofline": {
            "bound": "hbm",
            "kernel": dom_name,
            "achieved": achieved,
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS,
            "traffic": measured_traffic("pd::" + dom_name),
            "traffic_note": "HBM bytes per launch (FETCH_SIZE + WRITE_SIZE, scaled by the same "
                            "counters on a 1 GiB copy) from profiles/traffic_gp128_p64.json; null "
                            "if the kernels changed since the counters were taken",
        },
    }
    ctx.close()
    print(json.dumps(out), flush=True)




def headline_context(pd, autotune=True):
    """The headline workload's context: slice states from the library's
    seeded initial field and an initial coarse run, launch shapes tuned on
    the 256-slice batch."""
    ctx = pd.Context(0)
    ctx.set_problem("gp", RM5, KZ, N5)
    ctx.set_time(T5, P5, DT5, DTC5, NC5)
    ctx.seed_initial(SEED5, 1e-3, 4.0)
    ctx.parareal(0.0, 0)
    tuned = ctx.autotune(3) if autotune else None
    return ctx, tuned


def _sweep_chunks(step0, n, nf):
    """(start, count) calls covering n fine steps from step0, restarting the
    slice's sweep at step 0 when it reaches its end (nf steps)."""
    out = []
    s = step0 % nf
    while n > 0:
        c = min(n, nf - s)
        out.append((s, c))
        n -= c
        s = (s + c) % nf
    return out


def run_headline(args, cpu):
    """K fine steps of all 256 slices of the 512^2 workload (module header)."""
    import torch

    import paper_1902_00387_amd as pd
    nf = int(round(T5 / P5 / DT5))
    ctx, tuned = headline_context(pd)
    (rv, cv), (mr, mc) = tuned
    _log(f"# autotune: rows {pd.variants(N5, 0)[rv]} {mr*1e3:.0f} us, cols "
         f"{pd.variants(N5, 1)[cv]} {mc*1e3:.0f} us")
    group, nstreams = ctx.fine_blocking()
    # the step's two kernels one at a time over the whole batch (unblocked)
    KS = UNBLOCKED_STEPS
    ctx.set_fine_blocking(0)
    ctx.fine_sweep_steps(0, 1)
    mk = ctx.fine_sweep_steps(1, KS, timed=True)
    ms_cols, ms_rows = mk[0] / KS, mk[1] / KS
    # the sweep as Parareal runs it (blocked in groups of fields as the
    # autotuner chose), continued from there
    ctx.set_fine_blocking(group, nstreams)
    s0 = 1 + KS
    if args.warmup > 0:
        for a, c in _sweep_chunks(s0, args.warmup, nf):
            ctx.fine_sweep_steps(a, c)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ms_all = 0.0
    for a, c in _sweep_chunks(s0 + args.warmup, args.steps, nf):
        ms_all += ctx.fine_sweep_steps(a, c, timed=True)[2]
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    K = args.steps
    modes = N5 * N5 * P5
    value = modes * K / elapsed
    step_ms = ms_all / K
    achieved = ALG_BYTES_PER_MODE_STEP * modes / (step_ms * 1e-3) / 1e9
    cols_b, rows_b = kernel_bytes(N5, P5)
    re_, rw_ = pd.variants(N5, 0)[rv]
    rname = ("k_rows_c3<512,%d>" % re_ if rw_ == 3 else
             "k_rows<512,%d,%d,0,%s>" % (re_, abs(rw_), "true" if rw_ < 0 else "false"))
    ce, ctx_ = pd.variants(N5, 1)[cv]
    cname = ("k_cols<512,%d,%d>" % (ce, ctx_) if ctx_ > 0 else "k_cols_pf<512,%d,%d>" % (ce, -ctx_))
    tr_c = measured_traffic("pd::" + cname, TRAFFIC_FILE5)
    tr_r = measured_traffic("pd::" + rname, TRAFFIC_FILE5)
    traffic = tr_c + tr_r if tr_c is not None and tr_r is not None else None
    sched = (f"blocked: groups of {group} fields on {nstreams} streams" if group > 0
             else "unblocked: every step over all 256 slices")
    _log(f"# unblocked kernels: cols {ms_cols:.3f} + rows {ms_rows:.3f} ms = "
         f"{ms_cols + ms_rows:.3f} ms a step")
    _log(f"# {K} steps, {sched}: {step_ms:.3f} ms/step (HIP events), {elapsed*1e3/K:.3f} ms/step "
         f"wall; {value:.3e} mode-steps/s; {achieved:.0f} GB/s algorithmic")
    out = {
        "metric": "fine-propagator mode-steps/sec (batched F over all slices) & HBM GB/s",
        "value": value, "unit": "mode-steps/s", "n_gpus": 1, "steps": K, "warmup": args.warmup,
        "ms_per_step": elapsed / K * 1e3, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "c128",
        "data": "synthetic (library-seeded solenoidal field |k|<=4, amplitude 1e-3, "
                "propagated by the initial coarse run)",
        "config": {"workload": "Galloway-Proctor kinematic dynamo, Rm=2000, kz=0.57, 512x512 "
                               "complex128, T=256 over 256 slices, fine SBDF2 dt=5e-4 (2000 "
                               "steps a slice); one step = one fine step of all 256 slices",
                   "N": N5, "slices": P5, "dt_fine": DT5, "fine_steps_per_slice": nf,
                   "mode_steps_per_step": modes, "schedule": sched},
        "roofline": {"bound": "hbm", "kernel": f"fine step ({cname} + {rname}), {sched}",
                     "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
                     "note": "achieved = 192 B x 67.1 M mode-steps / time of one step of the "
                             "sweep (HIP events on the launching stream around the K timed "
                             "steps; in the blocked sweep the kernels of different groups "
                             "overlap on the streams, so the step time is their joint span); "
                             "traffic = FETCH_SIZE + WRITE_SIZE of the two unblocked launches "
                             "of one step (bytes between L2 and memory, of which the memory-side "
                             "cache serves part in the blocked sweep), scaled by the same "
                             "counters on a 1 GiB copy (profiles/traffic_gp512_p256.json), null "
                             "if the kernels changed since"},
        "kernels": {
            "unblocked_steps": KS,
            "cols": {"name": cname, "ms": ms_cols, "design_bytes": cols_b,
                     "design_gbs": cols_b / (ms_cols * 1e-3) / 1e9},
            "rows": {"name": rname, "ms": ms_rows, "design_bytes": rows_b,
                     "design_gbs": rows_b / (ms_rows * 1e-3) / 1e9},
            "design_bytes_per_mode_step": (cols_b + rows_b) / modes,
            "blocked_ms_per_step": step_ms,
        },
    }
    if cpu is not None:
        out["cpu_baseline"] = cpu
    ctx.close()
    print(json.dumps(out), flush=True)


def run_c64(args):
    """The complex64 variant of the 128^2 workload (and of the 512^2 one)
    beside complex128: one batched fine step of all slices (HIP events over
    the step's two kernels; complex64 moves half the bytes), and Parareal on
    the 128^2 workload to the tolerance each number type can reach (1e-4 for
    complex64, whose defect has an FP32 rounding floor near 2e-5 here; 1e-8
    and 1e-4 for complex128)."""
    import torch

    import paper_1902_00387_amd as pd
    from synthetic import initial_field
    out = {"experiment": "complex64 variant", "fine_step": {}, "parareal_128": {}}
    for (n, rm, T_, P_, dtf, dtc, nc, seed) in ((N, RM, T, P, DT_FINE, DT_COARSE, N_COARSE, SEED),
                                               (N5, RM5, T5, P5, DT5, DTC5, NC5, SEED5)):
        for prec in ("c128", "c64"):
            ctx = pd.Context(0)
            ctx.set_problem("gp", rm, KZ, n)
            ctx.set_precision(prec)
            ctx.set_time(T_, P_, dtf, dtc, nc)
            ctx.set_initial(initial_field(n, KZ, seed))
            ctx.parareal(0.0, 0)
            # the two kernels over the whole batch, one at a time; then the
            # sweep as Parareal runs it (blocked at 512^2)
            ctx.set_fine_blocking(0)
            ctx.fine_sweep_steps(0, 3)
            ms = ctx.fine_sweep_steps(3, 20, timed=True)
            step_ms = (ms[0] + ms[1]) / 20
            ctx.set_fine_blocking(-1)
            blk = ctx.fine_sweep_steps(23, 40, timed=True)[2] / 40
            m = box_m(n)
            es = 16 if prec == "c128" else 8
            design = es / 16.0 * 48 * (4 * m * n + 4 * m * m) / (n * n)
            out["fine_step"][f"{n}_{prec}"] = {
                "slices": P_, "ms_cols": ms[0] / 20, "ms_rows": ms[1] / 20,
                "mode_steps_per_s": n * n * P_ / (step_ms * 1e-3),
                "blocking": list(ctx.fine_blocking()), "ms_step_as_swept": blk,
                "mode_steps_per_s_as_swept": n * n * P_ / (blk * 1e-3),
                "design_bytes_per_mode_step": design,
                "design_gbs": design * n * n * P_ / (step_ms * 1e-3) / 1e9}
            _log(f"# {n}^2 x {P_} {prec}: cols {ms[0]/20*1e3:.1f} + rows {ms[1]/20*1e3:.1f} us, "
                 f"{n * n * P_ / (step_ms * 1e-3):.3e} mode-steps/s; as swept (blocking "
                 f"{ctx.fine_blocking()}) {blk*1e3:.1f} us, {n * n * P_ / (blk * 1e-3):.3e}")
            ctx.close()
    b0 = initial_field(N, KZ, SEED)
    for prec, tol in (("c128", TOL), ("c128", 1e-4), ("c64", 1e-4)):
        ctx = pd.Context(0)
        ctx.set_problem("gp", RM, KZ, N)
        ctx.set_precision(prec)
        ctx.set_time(T, P, DT_FINE, DT_COARSE, N_COARSE)
        times = []
        for _ in range(3):
            ctx.set_initial(b0)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            rep = ctx.parareal(tol, MAX_ITER)
            gam = ctx.growth_rate()
            torch.cuda.synchronize()
            times.append(time.perf_counter() - t0)
        out["parareal_128"][f"{prec}_tol{tol:g}"] = {
            "k_con": rep["k_con"], "sigma": rep["sigma"][:rep["iters"]], "time_s": min(times),
            "growth_rate": gam}
        _log(f"# parareal 128^2 {prec} tol {tol:g}: k_con {rep['k_con']}, {min(times)*1e3:.1f} ms, "
             f"growth {gam:.6f}")
        ctx.close()
    print(json.dumps(out), flush=True)


def run_kernel_only5(args):
    """For profiler runs: the headline's autotune and K fine steps of all
    slices, then a plain 1 GiB device copy to calibrate byte counters."""
    import torch

    import paper_1902_00387_amd as pd
    nf = int(round(T5 / P5 / DT5))
    ctx, _ = headline_context(pd)
    if args.blocked_only:
        pass  # the autotuner's blocking, as the benchmark times it
    else:
        # whole-batch launches: one dispatch per kernel and step
        ctx.set_fine_blocking(0)
    for a, c in _sweep_chunks(0, args.warmup + args.steps, nf):
        ctx.fine_sweep_steps(a, c)
    src = torch.empty(1 << 27, dtype=torch.float64, device="cuda")
    dst = torch.empty_like(src)
    dst.copy_(src)
    torch.cuda.synchronize()
    ctx.close()
    print(json.dumps({"kernel_only": True, "steps": args.warmup + args.steps,
                      "copy_bytes_each_way": src.numel() * 8}), flush=True)


BLOCKING_CASES = (  # N, slices, Rm, fine dt, T, coarse dt (coarse grid 64^2)
    (512, 256, 2000.0, 5e-4, 256.0, 2.5e-3),
    (256, 128, 500.0, 1e-3, 64.0, 5e-3),
    (128, 64, 100.0, 2e-3, 64.0, 1e-2),
)
BLOCKING_SETTINGS = ((0, 1), (1, 3), (2, 3), (3, 3), (4, 3), (6, 3), (8, 3), (16, 3), (2, 2),
                     (3, 2), (4, 2), (8, 2), (16, 2), (32, 2), (4, 1), (8, 1))


def run_blocking_sweep(args):
    """Time a fine sweep of K steps of every slice for each fine-blocking
    setting (fields a group, streams) and each launch shape of the two phase
    kernels, on three grid/batch sizes (the slice states from the seeded field
    and an initial coarse run)."""
    import paper_1902_00387_amd as pd
    K = args.steps
    out = {"experiment": "fine-sweep blocking", "steps": K, "cases": []}
    for n, p, rm, dtf, T_, dtc in BLOCKING_CASES:
        ctx = pd.Context(0)
        ctx.set_problem("gp", rm, KZ, n)
        ctx.set_time(T_, p, dtf, dtc, 64)
        ctx.seed_initial(SEED5, 1e-3, 4.0)
        ctx.parareal(0.0, 0)
        nf = int(round(T_ / p / dtf))
        res = []
        try:
            for rv in range(len(pd.variants(n, 0))):
                for cv in range(len(pd.variants(n, 1))):
                    pd.select_variant(n, rv, cv)
                    for g, ns in BLOCKING_SETTINGS:
                        if g >= p:
                            continue
                        ctx.set_fine_blocking(g, ns)
                        ctx.fine_sweep_steps(0, 2)
                        ms = 0.0
                        for a, c in _sweep_chunks(2, K, nf):
                            ms += ctx.fine_sweep_steps(a, c, timed=True)[2]
                        r = {"rows": pd.variants(n, 0)[rv], "cols": pd.variants(n, 1)[cv],
                             "group": g, "streams": ns, "ms_per_step": ms / K,
                             "mode_steps_per_s": n * n * p / (ms / K * 1e-3)}
                        res.append(r)
                        _log(f"# {n}^2 x {p}: rows {r['rows']} cols {r['cols']} group {g} streams "
                             f"{ns}: {ms / K:.4f} ms a step")
        finally:
            pd.select_variant(n, 0, 0)
        ctx.close()
        best = min(res, key=lambda r: r["ms_per_step"])
        unb = min((r for r in res if r["group"] == 0), key=lambda r: r["ms_per_step"])
        out["cases"].append({"N": n, "slices": p, "results": res, "best": best, "best_unblocked": unb})
        _log(f"# {n}^2 x {p}: best {best}; best unblocked {unb['ms_per_step']:.4f} ms")
    print(json.dumps(out), flush=True)


def run_parareal5(args):
    """Parareal on the headline workload with the plain coarse propagator:
    time to sigma <= 1e-8 (or the iterations run) against the serial fine
    solve on the same GPU."""
    import numpy as np
    import torch

    import paper_1902_00387_amd as pd
    nc, dtc, iters = args.p5_nc, args.p5_dtc, args.p5_iters
    ctx = pd.Context(0)
    ctx.set_problem("gp", RM5, KZ, N5)
    ctx.set_time(T5, P5, DT5, dtc, nc)
    ctx.seed_initial(SEED5, 1e-3, 4.0)
    ctx.parareal(0.0, 0)
    ctx.autotune(3)
    b0 = ctx.get_slices_dev()[0:1].clone()
    # serial fine solve, slice after slice (batch 1)
    torch.cuda.synchronize()
    ts = time.perf_counter()
    u = b0
    norms = [float(torch.linalg.vector_norm(u).item())]
    for n in range(P5):
        u = ctx.fine([n * T5 / P5], u)
        norms.append(float(torch.linalg.vector_norm(u).item()))
        if n % 64 == 63:
            _log(f"# serial fine: slice {n + 1}/{P5}, {time.perf_counter() - ts:.1f} s")
    torch.cuda.synchronize()
    serial_s = time.perf_counter() - ts
    g_serial = _growth(norms, T5 / P5)
    ctx.seed_initial(SEED5, 1e-3, 4.0)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    rep = ctx.parareal(TOL, iters)
    gam = ctx.growth_rate()
    torch.cuda.synchronize()
    tp = time.perf_counter() - t0
    _log(f"# parareal N_C={nc} dt_c={dtc}: k_con {rep['k_con']} after {rep['iters']} iterations, "
         f"{tp:.1f} s vs serial {serial_s:.1f} s")
    ctx.close()
    print(json.dumps({"experiment": "Parareal on the 512^2, 256-slice workload",
                      "N_coarse": nc, "dt_coarse": dtc, "max_iter": iters, "k_con": rep["k_con"],
                      "iters": rep["iters"], "sigma": rep["sigma"], "time_s": tp,
                      "t_fine_s": rep["t_fine_s"], "t_coarse_s": rep["t_coarse_s"] + rep["t_coarse0_s"],
                      "growth_rate": gam, "serial_fine_gpu_s": serial_s,
                      "serial_growth_rate": g_serial, "speedup_vs_serial_gpu": serial_s / tp}),
          flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=None,
                    help="timed steps (default 100 fine steps; 20 solves with --config2, "
                         "1 batch run with --batch)")
    ap.add_argument("--warmup", type=int, default=None, help="untimed steps first (default 10, "
                    "5 with --config2)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--config2", action="store_true",
                    help="a whole Parareal solve of the 128^2, 64-slice workload as the step")
    ap.add_argument("--parareal5", action="store_true",
                    help="Parareal solves of the default workload (plain coarse propagator)")
    ap.add_argument("--lg-nc", type=int, default=0,
                    help="--learned: coarse grid of the base propagator (0: pre-check choice)")
    ap.add_argument("--lg-dtc", type=float, default=1e-2, help="--learned: base coarse step")
    ap.add_argument("--lg-random", type=int, default=0, help="--learned: random training fields")
    ap.add_argument("--lg-harvest", type=int, default=16,
                    help="--learned: plain-G Parareal iterations harvested per run")
    ap.add_argument("--lg-late", type=int, default=4,
                    help="--learned: train only on differences of iterations >= this (0: all)")
    ap.add_argument("--lg-steps", type=int, default=2000, help="--learned: Adam steps")
    ap.add_argument("--lg-switch", type=int, default=4,
                    help="--learned: plain G for this many iterations, then the learned one")
    ap.add_argument("--c64", action="store_true",
                    help="complex64 variant beside complex128 (fine step, 128^2 Parareal)")
    ap.add_argument("--p5-nc", type=int, default=128, help="--parareal5: coarse grid")
    ap.add_argument("--p5-dtc", type=float, default=2.5e-3, help="--parareal5: coarse step")
    ap.add_argument("--p5-iters", type=int, default=8, help="--parareal5: iteration cap")
    ap.add_argument("--kernel-only", action="store_true",
                    help="only the fine-sweep kernels (for profiler runs)")
    ap.add_argument("--learned5", action="store_true",
                    help="learned vs plain coarse propagator on the 512^2 workload")
    ap.add_argument("--l5-tol", type=float, default=1e-8, help="--learned5: defect tolerance")
    ap.add_argument("--l5-iters", type=int, default=40, help="--learned5: iteration cap")
    ap.add_argument("--l5-harvest", type=int, default=8, help="--learned5: harvested iterations")
    ap.add_argument("--l5-steps", type=int, default=2000, help="--learned5: Adam steps")
    ap.add_argument("--l5-switch", type=int, default=4,
                    help="--learned5: plain G for this many iterations, then the learned one")
    ap.add_argument("--blocking-sweep", action="store_true",
                    help="time the fine sweep for fine-blocking settings and launch shapes")
    ap.add_argument("--summarize-trace", nargs=3, metavar=("TRACE_CSV", "STEPS", "FIELDS"),
                    help="summarize a kernel trace of --kernel-only --blocked-only")
    ap.add_argument("--blocked-only", action="store_true",
                    help="--kernel-only: the blocked sweep instead of whole-batch launches")
    ap.add_argument("--batch", action="store_true",
                    help="the many-instance workload instead of the single solve")
    ap.add_argument("--batch-scale", type=float, default=1.0)
    ap.add_argument("--learned", action="store_true",
                    help="learned versus plain coarse propagator (256^2, 128 slices)")
    ap.add_argument("--nc-sweep", action="store_true", help="coarse-grid sweep (Roberts Rm=512)")
    ap.add_argument("--nc-sweep-gp", action="store_true",
                    help="coarse-grid sweep on the headline workload (GP Rm=100, 128^2)")
    ap.add_argument("--nc-tol", type=float, default=1e-5, help="defect tolerance of the sweep")
    ap.add_argument("--nc-nf", type=int, default=128, help="fine grid of the sweep (128 or 256)")
    ap.add_argument("--work-precision", action="store_true", help="SBDF2 vs ARS(4,4,3) work-precision")
    ap.add_argument("--table1", action="store_true", help="growth rates of the paper's Table 1 sets")
    ap.add_argument("--table1-rows", default="", help="comma-separated row indices (default all)")
    ap.add_argument("--path", type=int, default=-1, help="fine launch path (-1 auto)")
    ap.add_argument("--pipeline", type=int, default=-1,
                    help="slice chunks of pipelined Parareal (0/1 off, -1 library default)")
    ap.add_argument("--pipeline-spec", type=int, default=2,
                    help="pipelined: 0 hold the last chunk, 1 start all early, 2 predict")
    ap.add_argument("--summarize-pmc", nargs=3, metavar=("FETCH_CSV", "WRITE_CSV", "OUT_JSON"),
                    help="write the HBM traffic summary from two rocprofv3 --pmc runs")
    args = ap.parse_args()
    if args.summarize_pmc:
        print(json.dumps(summarize_pmc(*args.summarize_pmc)))
        return
    if args.summarize_trace:
        print(json.dumps(summarize_trace(*args.summarize_trace), indent=1))
        return
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for {args.gpus}): the Parareal "
              "path here is single-GPU (slices would shard across GPUs in contiguous blocks).", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import paper_1902_00387_amd as pd  # noqa: F401  (loads the library; no GPU use yet)

    default = not (args.batch or args.learned or args.nc_sweep or args.nc_sweep_gp or
                   args.work_precision or args.table1 or args.config2 or args.parareal5 or
                   args.kernel_only or args.c64 or args.blocking_sweep or args.learned5)
    if args.steps is None:
        args.steps = 1 if args.batch else 20 if args.config2 or args.kernel_only else 100
    if args.warmup is None:
        args.warmup = 5 if args.config2 or args.kernel_only else 10
    # the CPU baseline forks its workers before anything touches the GPU
    cpu = cpu_baseline() if default and not args.no_cpu_baseline else None
    if cpu is not None:
        _log(f"# cpu baseline: {cpu['value']:.3e} mode-steps/s on {cpu['cores']} workers")
    assert torch.cuda.is_available(), "bench.py needs a GPU"
    if args.batch:
        run_batch(args)
        return
    if args.learned:
        run_learned(args)
        return
    if args.nc_sweep or args.nc_sweep_gp:
        run_nc_sweep(args)
        return
    if args.work_precision:
        run_work_precision(args)
        return
    if args.table1:
        run_table1(args)
        return
    if args.config2:
        run_config2(args)
        return
    if args.kernel_only:
        run_kernel_only5(args)
        return
    if args.c64:
        run_c64(args)
        return
    if args.parareal5:
        run_parareal5(args)
        return
    if args.blocking_sweep:
        run_blocking_sweep(args)
        return
    if args.learned5:
        run_learned5(args)
        return
    run_headline(args, cpu)


if __name__ == "__main__":
    main()
