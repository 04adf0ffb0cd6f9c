"""Benchmark of the per-cell chemistry integration on one MI355X.

Default workload (``--workload flame64``): the plain FP64 GPU integrator on
the 64^3 flame field (262,144 cells, 9-species / 21-reaction synthetic
mechanism, dt = 1e-6 s, rtol 1e-8, atol 1e-12), in the autotuned launch
configuration (schedule -2 after chem_autotune on the field, outside the
timed region; the line reports the tuner's whole measured table; --schedule
fixes one instead).  One step = one call of
chem_integrate over all cells, starting from the same pristine field
(restored by a device-to-device copy inside the step, so the copy is timed
too).  Prints ONE JSON line: the metric, the roofline of the integrator
kernel (algorithmic flops from the per-cell counters over the kernel time
from HIP events on the launch stream), HBM traffic from the committed
profiler summary when it was taken on the same kernel sources, and the CPU
oracle timed on the host cores.  The same line carries, under "surrogate",
the metric's second half: the learned surrogate with per-cell fallback on
the 256x128x128 flame field (4,194,304 cells, 35 species, dt = 1e-5 s),
trained in the run on 2,097,152 integrator-labelled states for 20 epochs,
with its fused-forward MFMA roofline, the fallback fraction, the plain GPU
integrator on a seeded sample of the same cells, and max |dT| against the
oracle on a seeded 65,536-cell subset (the oracle's CPU rate from the same
run); --no-surrogate leaves it out.

Other workloads (``--workload``):
  cells4096  4,096 cells, 9 species, dt = 1e-6 (the parity case);
  zones128   128^3 = 2,097,152 cells of the 35-species mechanism, 60 % cold /
             10 % flame front / 30 % burnt, dt = 1e-5, FP32 Jacobian/LU with
             FP64 residuals and state, wave-per-cell schedule;
  laplacian128  implicit Laplacian assembly (Algorithm 1) + ldu -> CSR
             conversion on a graded 128^3 box (HBM roofline);
  species_nets  the paper's per-species networks (one 1600-800-400 network
             per species, grouped BF16 MFMA products) against the single
             512-256-128 network, both trained on the same integrator-
             labelled states of the 9-species mechanism (dt = 1e-6) and
             served on flame64: forward TFLOP/s, served step, fallback and
             max |dT| against the plain GPU integrator and the oracle;
  props_tgv  the Thermo field kernels on one GPU's share of the 256^3 TGV
             mesh (256x128x128 = 4,194,304 cells, 9 species): T from h by
             Newton from the previous step's T, then mixture-averaged
             viscosity, conductivity and diffusion coefficients;
  surrogate  the learned surrogate with per-cell fallback on the 256x128x128
             flame field (4,194,304 cells, 35 species, dt = 1e-5): training
             states labelled by the GPU integrator, training on the GPU, then
             timed inference steps against the plain integrator on the same
             cells and the oracle on a sample.  --field flame256 serves the
             256^3 field (16,777,216 cells) and --graph replays the captured
             step; the plain integrator then runs on a seeded sample.  With
             --evolve the timed steps advance the field (no restore inside the
             step), the network is first trained further on the states it
             visits itself (three rollout rounds, each labelled by the
             integrator), and the fallback count and the drift against the
             plain integrator, advanced in step on a seeded sample of cells,
             are reported after every step.
"""
from __future__ import annotations

import argparse
import glob
import hashlib
import json
import os
import sys
import tempfile
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "chemistry cell-steps/sec at dt=1e-6 s: plain FP64 vs surrogate; max |dT| vs oracle"
FP64_PEAK_TFLOPS = 78.6          # MI355X FP64 vector, dense (FP32 without packing runs at the same rate)
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic.txt")


def algorithmic_flops(K: int, R: int, counters: np.ndarray) -> dict:
    """FP64 flops of the integrator's algorithm, from per-cell operation counts.

    counters: (6, n) rows nst, nfe, nje, nni, netf, ncfn.  Per-operation
    counts follow the definitions (add/sub/mul/div = 1, fused multiply-add = 2,
    exp/log/pow/sqrt = 20), not the instructions a kernel happens to issue:
      rhs   = 40 K + 60 R + 28     (thermo 29K + log, mixture 7K, per reaction
                                    2 exp + ~20, ODE assembly 4K)
      jac   = 37 K + 115 R + 10 K^2 + 40 K
      lu    = N(N-1)/2 + (N-1)N(2N-1)/3 + 2 N^2   (factor + forming I - gamma J)
      solve = 2 N^2 - N + 10 N + 20  (triangular solves + residual, norm, update)
      step  = 21 N + 60               (predict, correct, weights, error norm, eta)
    """
    N = K + 1
    f_rhs = 40 * K + 60 * R + 28
    f_jac = 37 * K + 115 * R + 10 * K * K + 40 * K
    f_lu = N * (N - 1) // 2 + (N - 1) * N * (2 * N - 1) // 3 + 2 * N * N
    f_solve = 2 * N * N - N + 10 * N + 20
    f_step = 21 * N + 60
    nst, nfe, nje, nni = (counters[i].astype(np.float64).sum() for i in range(4))
    total = nfe * f_rhs + nje * (f_jac + f_lu) + nni * f_solve + nst * f_step
    return {"total": float(total), "per_rhs": f_rhs, "per_jac": f_jac, "per_lu": f_lu,
            "per_solve": f_solve, "per_step": f_step}


def kernel_sources_sha() -> str:
    """Digest of every source the integrator kernels are built from."""
    h = hashlib.sha256()
    files = sorted(glob.glob(os.path.join(ROOT, "paper_2312_13513_amd", "csrc", "*")))
    files.append(os.path.join(ROOT, "paper_2312_13513_amd", "codegen.py"))
    for f in files:
        if os.path.isfile(f):
            h.update(os.path.basename(f).encode())
            with open(f, "rb") as fh:
                h.update(fh.read())
    return h.hexdigest()[:16]


def traffic_for(workload: str, kernel: str):
    """HBM bytes per launch recorded by the profiler for this workload and
    kernel, if the record was taken on the current kernel sources."""
    if not os.path.exists(TRAFFIC_FILE):
        return None
    sha = kernel_sources_sha()
    for line in open(TRAFFIC_FILE):
        parts = line.split()
        if len(parts) >= 5 and not line.startswith("#") and parts[0] == workload and parts[1] == kernel \
                and parts[2] == sha:
            return float(parts[3]) + float(parts[4])
    return None


def kernel_name(mech, schedule: int, precision: int, n: int) -> str:
    lt = "float" if precision == 1 else "double"
    if schedule < 0:   # the library's own choice
        schedule = 0 if (mech.variant.startswith("specialised:") and precision == 0) else (2 if mech.N <= 16 else 1)
    if schedule == 2:   # refreshes deferred from 65,536 cells on
        return f"bdf_tile_kernel<{12 if mech.N <= 12 else 16},{lt},true,{'true' if n >= 65536 else 'false'}>"
    if schedule == 1 or precision == 1 or (mech.variant == "table" and mech.K > 9):
        np_rows = 16 if mech.N <= 16 else (40 if mech.N <= 40 else 64)
        return f"bdf_wave_kernel<{np_rows},{lt},true>"
    if mech.variant.startswith("specialised:"):
        return f"bdf_queue_kernel<GenMech_{mech.variant.split(':')[1]}>"
    return f"bdf_queue_kernel<TableMech<{mech.K}>>"


def cpu_model() -> str:
    """The host CPU's model name (first /proc/cpuinfo entry)."""
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def progress(msg: str) -> None:
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def mech_file(name: str):
    from chemgen.mechanism import standard_mechanism
    mpy = standard_mechanism(name)
    path = os.path.join(tempfile.mkdtemp(), f"{name}.mech")
    mpy.write(path)
    return mpy, path


def time_oracle(path, field, target_s: float, max_cells: int):
    """The oracle on a seeded sample of the field, repeated until target_s."""
    import oracle
    from chemgen.fields import seeded_sample
    om = oracle.OracleMech(path)
    idx = seeded_sample(field.n, min(max_cells, field.n), seed=5)
    reps, total, used, out = 0, 0.0, 0, None
    while total < target_s or reps == 0:
        t1 = time.perf_counter()
        res = om.integrate(field.T[idx], field.p[idx], field.Y[:, idx], field.dt)
        total += time.perf_counter() - t1
        reps += 1
        used = res[4]
        out = res
    return idx, out, reps * idx.size / total, used, reps, total


def time_oracle_one_thread(path, field, target_s: float, max_cells: int):
    """The oracle on one host thread (a per-core rate), a seeded sample."""
    import oracle
    from chemgen.fields import seeded_sample
    om = oracle.OracleMech(path)
    idx = seeded_sample(field.n, min(max_cells, field.n), seed=6)
    cells, total = 0, 0.0
    while total < target_s or cells == 0:
        t1 = time.perf_counter()
        om.integrate(field.T[idx], field.p[idx], field.Y[:, idx], field.dt, nthreads=1)
        total += time.perf_counter() - t1
        cells += idx.size
    return cells / total, int(idx.size), total


def run_integrator(args, workload: str):
    import torch

    from chemgen import fields as F
    from paper_2312_13513_amd import chem

    if workload == "flame64":
        mname, make, precision, schedule = "M9", F.flame64, 0, -2
        desc = "flame64: 262,144 cells (64^3 smooth flame field), synthetic 9-species/21-reaction mechanism"
    elif workload == "cells4096":
        mname, make, precision, schedule = "M9", F.cells4096, 0, -1
        desc = "cells4096: 4,096 cells, T U[900,2200] K, Y Dirichlet(1), 9-species/21-reaction mechanism"
    else:
        mname, make, precision, schedule = "M35", F.zones128, 1, 1
        desc = ("zones128: 2,097,152 cells (128^3; 60% cold, 10% flame front, 30% burnt), synthetic "
                "35-species/200-reaction mechanism, FP32 Jacobian/LU with FP64 residuals and state")
    mpy, path = mech_file(mname)
    field = make(mpy)
    if args.shuffle:
        # the same cells in a seeded random order: no spatial clustering of
        # the stiff zone (the load-balance contrast to the clustered field)
        perm = np.random.default_rng(17).permutation(field.n)
        field.T, field.p, field.Y = field.T[perm], field.p[perm], np.ascontiguousarray(field.Y[:, perm])
        if field.zone is not None:
            field.zone = field.zone[perm]
        if field.c is not None:
            field.c = field.c[perm]
        desc += "; cells in a seeded random order"
    dev = torch.device("cuda:0")
    mech = chem.Mechanism(path, 0)
    n, K, R = field.n, mpy.K, mpy.R
    opts = chem.chem_default_opts()
    if args.schedule is not None:
        schedule = args.schedule
    opts.precision = precision
    opts.schedule = schedule
    T0 = torch.tensor(field.T, dtype=torch.float64, device=dev)
    p0 = torch.tensor(field.p, dtype=torch.float64, device=dev)
    Y0 = torch.tensor(field.Y, dtype=torch.float64, device=dev)
    tune = None
    if schedule == -2:
        # launch configuration measured on this field (not timed); the steps
        # below then run the tuned choice
        t_tune = time.perf_counter()
        best, use_lpt, best_ms = mech.autotune(T0, p0, Y0, field.dt, opts=opts)
        table = mech.autotune_results()
        schedule = best.schedule
        tune = {"chosen": {"schedule": best.schedule, "jac_batch": best.jac_batch,
                           "waves_per_simd": best.waves_per_simd, "lpt": int(use_lpt), "ms": best_ms},
                "sample_cells": min(n, 262144), "tuning_s": time.perf_counter() - t_tune,
                "table": [{k: (round(v, 4) if k == "ms" else v) for k, v in e.items()} for e in table]}
        progress(f"autotune: schedule {best.schedule} jac_batch {best.jac_batch} waves/SIMD "
                 f"{best.waves_per_simd} lpt {int(use_lpt)} {best_ms:.3f} ms")
    T, Y = T0.clone(), Y0.clone()
    status = torch.zeros(n, dtype=torch.int32, device=dev)
    counters = torch.zeros(6 * n, dtype=torch.int32, device=dev)
    stream = torch.cuda.current_stream()

    def step(ev=None):
        T.copy_(T0)
        Y.copy_(Y0)
        if ev is not None:
            ev[0].record(stream)
        mech.integrate(T, p0, Y, field.dt, opts=opts, status=status, counters=counters, stream=stream)
        if ev is not None:
            ev[1].record(stream)

    for _ in range(args.warmup):
        step()
    events = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
              for _ in range(args.steps)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(args.steps):
        step(events[k])
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    avg_kern_s = float(np.mean([a.elapsed_time(b) for a, b in events])) * 1e-3

    st = status.cpu().numpy()
    cnt = counters.cpu().numpy().reshape(6, n)
    Tg, Yg = T.cpu().numpy(), Y.cpu().numpy()
    fl = algorithmic_flops(K, R, cnt)
    achieved = fl["total"] / avg_kern_s / 1e12
    kname = kernel_name(mech, schedule, precision, n)
    traffic = traffic_for(workload, kname)
    result = {
        "metric": METRIC,
        "value": n * args.steps / wall,
        "unit": "cell-steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": wall / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if precision == 0 else "f64+f32",
        "data": "synthetic",
        "config": {"workload": f"{desc}, dt={field.dt:g} s, rtol 1e-8, atol 1e-12",
                   "ncells": n, "species": K, "reactions": R, "dt": field.dt,
                   "schedule": ("tile: 16 lanes per cell, 4 cells per wave" if kname.startswith("bdf_tile") else
                                "wave per cell" if kname.startswith("bdf_wave") else
                                "thread per cell, mechanism compiled in")},
        "roofline": {"bound": "alu", "achieved": achieved, "peak": FP64_PEAK_TFLOPS, "unit": "TFLOP/s",
                     "frac": achieved / FP64_PEAK_TFLOPS, "traffic": traffic, "kernel": kname,
                     "kernel_ms": avg_kern_s * 1e3, "flops_per_launch": fl["total"],
                     "sources": kernel_sources_sha()},
        "substeps": {"mean": float(cnt[0].mean()), "max": int(cnt[0].max()), "p50": float(np.median(cnt[0])),
                     "rhs_per_cell": float(cnt[1].mean()), "jac_per_cell": float(cnt[2].mean())},
        "status_ok_frac": float(np.mean(st == 0)),
    }
    if tune is not None:
        result["autotune"] = tune
    if field.zone is not None:
        result["substeps"]["per_zone_mean"] = {name: float(cnt[0][field.zone == z].mean())
                                               for z, name in enumerate(("cold", "front", "burnt"))}
    if not args.no_cpu_baseline:
        max_cells = args.cpu_sample or (field.n if mname == "M9" else 16384)
        idx, (To, Yo, so, co, _), rate, used, reps, total = time_oracle(path, field, args.cpu_seconds, max_cells)
        result["cpu_baseline"] = {
            "value": rate, "unit": "cell-steps/s", "cores": int(used), "kind": "oracle", "cpu": cpu_model(),
            "sample": f"{idx.size} cells of the same field ({'all' if idx.size == n else 'seeded sample'}), "
                      f"{reps} pass(es), {total:.2f} s wall on {used} threads of {os.cpu_count()} host CPUs"}
        result["max_dT_vs_oracle"] = float(np.abs(Tg[idx] - To).max())
        result["max_dY_vs_oracle"] = float(np.abs(Yg[:, idx] - Yo).max())
        result["steps_equal_frac"] = float(np.mean(cnt[0][idx] == co[:, 0]))
        r1, m1, t1 = time_oracle_one_thread(path, field, min(3.0, args.cpu_seconds), 4096 if mname == "M9" else 256)
        result["cpu_baseline"]["one_thread"] = {"value": r1, "unit": "cell-steps/s",
                                                "sample": f"{m1} cells (seeded sample), {t1:.2f} s on 1 thread"}
    mech.close()
    return result


def run_surrogate(args, nested: bool = False):
    """The surrogate workload.  nested: the compact object the default
    benchmark line carries beside the plain integrator (no evolving state,
    no graph; plain integrator and oracle on seeded samples)."""
    import torch

    from chemgen import fields as F
    from chemgen.surrogate_data import epoch_orders, flame_like_states, init_params, network_dims, \
        trajectory_starts
    from paper_2312_13513_amd import chem

    dev = torch.device("cuda:0")
    mpy, path = mech_file("M35")
    mech = chem.Mechanism(path, 0)
    dt, K = 1e-5, mpy.K

    def t(a, dtype=torch.float64):
        return torch.tensor(np.ascontiguousarray(a), dtype=dtype, device=dev)

    log = {}
    # ---- training data: flame-like states and integrator trajectories, labelled on the GPU
    t0 = time.perf_counter()
    n_half = args.train_samples // 2
    T1, p1, Y1 = flame_like_states(mpy, n_half, seed=7)
    n_traj = max(2, n_half // args.traj_steps)
    # trajectories from cold unburnt mixtures and from flame-like states
    T2, p2, Y2 = trajectory_starts(mpy, n_traj // 2, seed=8)
    T3, p3, Y3 = flame_like_states(mpy, n_traj - n_traj // 2, seed=9)
    T2, p2, Y2 = np.concatenate([T2, T3]), np.concatenate([p2, p3]), np.concatenate([Y2, Y3], axis=1)
    Tt, pt, Yt = t(T2), t(p2), t(Y2)
    Ts, Ys = [], []
    for _ in range(args.traj_steps):
        mech.integrate(Tt, pt, Yt, dt)
        Ts.append(Tt.clone())
        Ys.append(Yt.clone())
    Td = torch.cat([t(T1)] + Ts)
    pd = torch.cat([t(p1), t(np.full(n_traj * args.traj_steps, p2[0]))])
    Yd = torch.cat([t(Y1)] + Ys, dim=1).contiguous()
    del Ts, Ys
    Yn = Yd.clone()
    Tn = Td.clone()
    mech.integrate(Tn, pd, Yn, dt)
    torch.cuda.synchronize()
    n_train = Td.shape[0]
    log["label_s"] = time.perf_counter() - t0
    progress(f"labelled {n_train} training states in {log['label_s']:.1f} s")
    # ---- training on the GPU
    t0 = time.perf_counter()
    surr = chem.Surrogate(mech, 512, 256, 128)
    surr.set_params(init_params(network_dims(K), 9))
    surr.fit_norm(Td, pd, Yd, Yn, dt)
    order = t(epoch_orders(n_train, args.epochs, 10), torch.int32)
    losses = surr.train(Td, pd, Yd, Yn, epochs=args.epochs, batch=4096, lr0=1e-3, lr1=1e-5, order=order)
    log["train_s"] = time.perf_counter() - t0
    progress(f"trained {args.epochs} epochs in {log['train_s']:.1f} s")
    del order
    # ---- rollout rounds (data aggregation, DAgger): the trained surrogate
    # advances fresh flame-like states for several flow steps, feeding on its
    # own output (with its checks and fallback, as served); every state it
    # visits is labelled by one step of the GPU integrator and added to the
    # training set, which the network is then trained on further
    log["rollout"] = []
    for r in range(args.rollout_rounds):
        # round r rolls out half as many cells for twice as many steps as
        # round r - 1 (the same number of visited states): later rounds reach
        # the states a long served run drifts into
        t0 = time.perf_counter()
        r_cells, r_steps = max(64, args.rollout_cells >> r), args.rollout_steps << r
        T4, p4, Y4 = flame_like_states(mpy, r_cells, seed=20 + r)
        Tr, pr, Yr = t(T4), t(p4), t(Y4)
        vis_T, vis_Y = [], []
        fb_cnt = torch.zeros(1, dtype=torch.int64, device=dev)
        fbs = []
        for _ in range(r_steps):
            surr.infer(Tr, pr, Yr, dt, fallback_count=fb_cnt)
            vis_T.append(Tr.clone())
            vis_Y.append(Yr.clone())
            fbs.append(fb_cnt.clone())
        Tv = torch.cat(vis_T)
        Yv = torch.cat(vis_Y, dim=1).contiguous()
        pv = t(np.full(Tv.shape[0], p4[0]))
        del vis_T, vis_Y
        Tvn, Yvn = Tv.clone(), Yv.clone()
        mech.integrate(Tvn, pv, Yvn, dt)
        Td, pd = torch.cat([Td, Tv]), torch.cat([pd, pv])
        Yd, Yn = torch.cat([Yd, Yv], dim=1).contiguous(), torch.cat([Yn, Yvn], dim=1).contiguous()
        del Tv, Yv, Tvn, Yvn, pv
        n_train = Td.shape[0]
        order = t(epoch_orders(n_train, args.rollout_epochs, 40 + r), torch.int32)
        l2 = surr.train(Td, pd, Yd, Yn, epochs=args.rollout_epochs, batch=4096, lr0=3e-4, lr1=1e-5, order=order)
        del order
        rollout_fb = [int(x.item()) for x in fbs]
        log["rollout"].append({"round": r + 1, "cells": r_cells, "steps": r_steps, "visited_states": r_cells * r_steps,
                               "fallback_per_step": rollout_fb, "loss_first": float(l2[0]),
                               "loss_last": float(l2[-1]), "s": time.perf_counter() - t0})
        progress(f"rollout round {r + 1}: fallback per step {rollout_fb}, {n_train} states, "
                 f"loss {l2[0]:.4g} -> {l2[-1]:.4g}, {time.perf_counter() - t0:.1f} s")
    del Td, pd, Yd, Yn, Tn
    torch.cuda.empty_cache()
    # ---- the served field
    field = F.flame256x128x128(mpy) if args.field == "flame256x128x128" else F.flame256(mpy)
    n = field.n
    T0, p0, Y0 = t(field.T), t(field.p), t(field.Y)
    progress(f"served field {field.name}: {n} cells")
    T, Y = T0.clone(), Y0.clone()
    mask = torch.zeros(n, dtype=torch.int32, device=dev)
    cnt = torch.zeros(1, dtype=torch.int64, device=dev)
    stream = torch.cuda.current_stream()

    evolve = args.evolve

    def step(ev=None):
        if not evolve:
            T.copy_(T0)
            Y.copy_(Y0)
        if ev is not None:
            ev[0].record(stream)
        surr.infer(T, p0, Y, dt, mask=mask, fallback_count=cnt, stream=stream)
        if ev is not None:
            ev[1].record(stream)

    for _ in range(max(args.warmup, 1)):
        step()
    events = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
              for _ in range(args.steps)]
    graph = None
    if args.graph:
        # the whole flow step (restore + surrogate + fallback) as one HIP graph
        side = torch.cuda.Stream()
        side.wait_stream(torch.cuda.current_stream())
        graph = torch.cuda.CUDAGraph()
        with torch.cuda.stream(side):
            with torch.cuda.graph(graph, stream=side):
                if not evolve:
                    T.copy_(T0)
                    Y.copy_(Y0)
                surr.infer(T, p0, Y, dt, mask=mask, fallback_count=cnt, stream=side)
        torch.cuda.synchronize()
        graph.replay()
    torch.cuda.synchronize()
    if evolve:
        # the plain integrator advances a seeded sample of the same cells
        # over the same flow steps, in step with the served field (cells are
        # independent): drift and fallback are recorded after every step
        from chemgen.fields import seeded_sample
        didx = seeded_sample(n, min(args.drift_cells, n), seed=13)
        di = torch.tensor(didx, dtype=torch.int64, device=dev)
        Td, Yd, pd = T[di].clone(), Y[:, di].contiguous(), p0[di].contiguous()
        per_step = []
    t0 = time.perf_counter()
    for k in range(args.steps):
        if graph is not None:
            events[k][0].record(stream)
            graph.replay()
            events[k][1].record(stream)
        else:
            step(events[k])
        if evolve:
            mech.integrate(Td, pd, Yd, dt)
            dTk = (T[di] - Td).abs()
            per_step.append({"step": k + 1, "fallback_cells": int(cnt.item()),
                             "max_dT": float(dTk.max().item()), "mean_abs_dT": float(dTk.mean().item()),
                             "max_dY": float((Y[:, di] - Yd).abs().max().item())})
            if k % 10 == 9 or k == args.steps - 1:
                progress(f"step {k + 1}: {per_step[-1]['fallback_cells']} fallback cells, drift max|dT| "
                         f"{per_step[-1]['max_dT']:.3f} K, {time.perf_counter() - t0:.1f} s")
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    kern_ms = float(np.mean([a.elapsed_time(b) for a, b in events]))
    if evolve:
        # the drift check ran between the steps: the rate is the served
        # steps' own time (HIP events around each step)
        wall = kern_ms * 1e-3 * args.steps
    progress(f"{args.steps} timed surrogate steps: {wall / args.steps * 1e3:.2f} ms per step")
    drift = None
    if evolve:
        drift = {"steps": args.steps, "cells": int(didx.size), "per_step": per_step,
                 "max_fallback_frac": max(x["fallback_cells"] for x in per_step) / n,
                 "max_dT": max(x["max_dT"] for x in per_step),
                 "max_dY": max(x["max_dY"] for x in per_step)}
        progress(f"drift over {args.steps} steps on {didx.size} cells: max|dT| {drift['max_dT']:.3f} K, "
                 f"largest fallback fraction {drift['max_fallback_frac']:.2e}")
        # one step from the pristine field for the single-step accuracy below
        T.copy_(T0)
        Y.copy_(Y0)
        surr.infer(T, p0, Y, dt, mask=mask, fallback_count=cnt, stream=stream)
        torch.cuda.synchronize()
    Ts_, Ys_ = T.cpu().numpy(), Y.cpu().numpy()
    nfb = int(cnt.item())
    # forward pass alone, on one inference pass of rows (2,097,152): algorithmic
    # MFMA flops over its time
    X = torch.zeros((min(n, args.fwd_rows), 64), dtype=torch.int16, device=dev)
    out = torch.zeros((X.shape[0], surr.nout_pad), dtype=torch.float32, device=dev)
    surr.encode(T0[:X.shape[0]], p0[:X.shape[0]], Y0[:, :X.shape[0]].contiguous(), X)
    surr.forward(X, out)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(10):
        surr.forward(X, out)
    e1.record(stream)
    torch.cuda.synchronize()
    fwd_ms = e0.elapsed_time(e1) / 10
    fwd_flops = 2.0 * X.shape[0] * ((K + 2) * 512 + 512 * 256 + 256 * 128 + 128 * K)
    # ---- plain integrator on the same cells (one timed step; a seeded
    # sample of the cells when the field is larger than --plain-cells)
    from chemgen.fields import seeded_sample
    pidx = np.arange(n) if n <= args.plain_cells else seeded_sample(n, args.plain_cells, seed=11)
    Tp, Yp = t(field.T[pidx]), t(field.Y[:, pidx])
    pp = t(field.p[pidx])
    opts = chem.chem_default_opts()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    mech.integrate(Tp, pp, Yp, dt, opts=opts)
    torch.cuda.synchronize()
    plain_s = time.perf_counter() - t0
    progress(f"plain integrator on {pidx.size} cells: {plain_s:.2f} s")
    Tp_ = Tp.cpu().numpy()
    n_plain = pidx.size
    result = {
        "metric": METRIC, "value": n * args.steps / wall, "unit": "cell-steps/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": wall / args.steps * 1e3,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "bf16+f64",
        "data": "synthetic",
        "config": {"workload": f"surrogate + fallback: {field.name} ({n} cells), synthetic 35-species/200-reaction "
                               f"mechanism, dt=1e-5 s; MLP 37-512-256-128-35 GELU, BF16 MFMA, trained on "
                               f"{n_train} integrator-labelled states for {args.epochs} epochs",
                   "ncells": n, "species": K, "dt": dt},
        "roofline": {"bound": "mfma", "achieved": fwd_flops / (fwd_ms * 1e-3) / 1e12, "peak": 2500.0,
                     "unit": "TFLOP/s", "frac": fwd_flops / (fwd_ms * 1e-3) / 1e12 / 2500.0,
                     "traffic": traffic_for("surrogate", "mlp_forward_kernel"),
                     "kernel": "mlp_forward_kernel (fused forward, 4 layers)", "kernel_ms": fwd_ms,
                     "rows": int(X.shape[0])},
        "fallback_frac": nfb / n,
        "surrogate_step_ms": kern_ms,
        "plain_gpu": {"value": n_plain / plain_s, "unit": "cell-steps/s", "cells": int(n_plain),
                      "ms": plain_s * 1e3},
        "speedup_vs_plain_gpu": (n * args.steps / wall) / (n_plain / plain_s),
        "max_dT_vs_plain_gpu": float(np.abs(Ts_[pidx] - Tp_).max()),
        "graph": bool(args.graph),
        "evolving_state": bool(evolve),
        "drift": drift,
        "train": {"samples": n_train, "epochs": args.epochs, "loss_first": float(losses[0]),
                  "loss_last": float(losses[-1]), "label_s": log["label_s"], "train_s": log["train_s"],
                  "rollout_rounds": log["rollout"]},
    }
    if not args.no_cpu_baseline:
        # the oracle on a seeded uniform subset of the served cells: the
        # accuracy check and the CPU rate in one run
        idx, (To, Yo, so, co, _), rate, used, reps, total = time_oracle(path, field, 0.0,
                                                                        args.surr_oracle_cells)
        result["cpu_baseline"] = {
            "value": rate, "unit": "cell-steps/s", "cores": int(used), "kind": "oracle", "cpu": cpu_model(),
            "sample": f"{idx.size} cells of the same field (seeded uniform subset), {reps} pass(es), "
                      f"{total:.2f} s wall on {used} threads of {os.cpu_count()} host CPUs"}
        result["max_dT_vs_oracle"] = float(np.abs(Ts_[idx] - To).max())
        result["max_dY_vs_oracle"] = float(np.abs(Ys_[:, idx] - Yo).max())
        result["oracle_cells"] = int(idx.size)
        progress(f"oracle on {idx.size} served cells: max|dT| {result['max_dT_vs_oracle']:.3f} K, {total:.1f} s")
    surr.close()
    mech.close()
    if nested:
        keep = ("value", "unit", "ms_per_step", "dtype", "config", "roofline", "fallback_frac", "surrogate_step_ms",
                "plain_gpu", "speedup_vs_plain_gpu", "max_dT_vs_plain_gpu", "cpu_baseline", "max_dT_vs_oracle",
                "max_dY_vs_oracle", "oracle_cells", "train")
        result = {k: result[k] for k in keep if k in result}
        result["metric"] = "surrogate + fallback cell-steps/sec at dt=1e-5 s; max |dT| vs oracle"
    return result


def run_laplacian(args):
    """Implicit Laplacian assembly on a graded 128^3 box (2,097,152 cells,
    6,242,304 internal faces, six patches, three fixed-value).  One step = the
    direct CSR assembly (chem_ldu_laplacian_csr); the ldu path (Algorithm 1
    with an atomic diagonal, then the ldu -> CSR conversion) is timed beside
    it.  HBM rooflines with the algorithmic bytes of every array read or
    written once."""
    import torch

    from chemgen.mesh import box_mesh, laplacian_fields
    from paper_2312_13513_amd import chem

    m = box_mesh(128, 128, 128, grading=(2.0, 1.0, 0.5))
    gc, gb, pb = laplacian_fields(m, 7)
    dev = torch.device("cuda:0")
    t = lambda a: torch.tensor(a, dtype=torch.float64, device=dev)
    g = chem.LduMesh(m)
    gct, gbt, pbt = t(gc), t(gb), t(pb)
    e = lambda n: torch.empty(n, dtype=torch.float64, device=dev)
    lo, up, dg, ic, bc = e(m.nfaces), e(m.nfaces), e(m.ncells), e(m.nbfaces), e(m.nbfaces)
    val, rhs = e(g.nnz), e(m.ncells)
    stream = torch.cuda.current_stream()

    def step(ev=None):
        if ev is not None:
            ev[0].record(stream)
        g.laplacian(gct, gbt, pbt, lo, up, dg, ic, bc, stream=stream)
        if ev is not None:
            ev[1].record(stream)
        g.to_csr(lo, up, dg, ic, bc, val, rhs, stream=stream)
        if ev is not None:
            ev[2].record(stream)

    def direct(ev=None):
        if ev is not None:
            ev[0].record(stream)
        g.laplacian_csr(gct, gbt, pbt, val, rhs, stream=stream)
        if ev is not None:
            ev[1].record(stream)

    def timed(fn, nev):
        for _ in range(args.warmup):
            fn()
        evs = [tuple(torch.cuda.Event(enable_timing=True) for _ in range(nev)) for _ in range(args.steps)]
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for k in range(args.steps):
            fn(evs[k])
        torch.cuda.synchronize()
        return time.perf_counter() - t0, evs

    # the step: the direct CSR assembly (what a solver consumes); the two-pass
    # ldu assembly with atomics (Algorithm 1 as printed) + conversion beside it
    wall, events = timed(direct, 2)
    dir_s = float(np.mean([a.elapsed_time(b) for a, b in events])) * 1e-3
    wall2, events2 = timed(step, 3)
    asm_s = float(np.mean([a.elapsed_time(b) for a, b, _ in events2])) * 1e-3
    csr_s = float(np.mean([b.elapsed_time(c) for _, b, c in events2])) * 1e-3
    nf, nc, nb = m.nfaces, m.ncells, m.nbfaces
    bytes_asm = nf * 48 + nc * 16 + nb * 48
    bytes_csr = nf * 40 + nc * 32 + nb * 20
    # direct: the face pass reads each face's two cells and geometry and
    # writes its coefficient; the entry pass reads every entry's face slot
    # and writes its value, reads the coefficients; per cell gamma, row_ptr,
    # bnd_ptr and the rhs write; boundary faces' index, type and data.  Every
    # array counted once.
    nnz = g.nnz
    bytes_dir = nf * (8 + 24 + 8 + 8) + nnz * (4 + 8) + nc * (8 + 4 + 4 + 8) + nb * (4 + 4 + 32)
    result = {
        "metric": "implicit Laplacian assembly into CSR, cells/s",
        "value": nc * args.steps / wall, "unit": "cells/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": wall / args.steps * 1e3, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": "laplacian128: graded 128^3 box, gamma smooth seeded field, 3 fixed-value and 3 "
                               "zero-gradient patches", "ncells": nc, "faces": nf, "boundary_faces": nb,
                   "csr_entries": nnz},
        "roofline": {"bound": "hbm", "achieved": bytes_dir / dir_s / 1e9, "peak": 8000.0, "unit": "GB/s",
                     "frac": bytes_dir / dir_s / 1e9 / 8000.0,
                     "traffic": traffic_for("laplacian128", "face_coeff_kernel+csr_assemble_entries_kernel"),
                     "kernel": "face_coeff_kernel + csr_assemble_entries_kernel (direct CSR assembly)",
                     "kernel_ms": dir_s * 1e3, "bytes_per_launch": bytes_dir},
        "ldu_path": {"cells_per_s": nc * args.steps / wall2, "ms_per_step": wall2 / args.steps * 1e3,
                     "assembly": {"kernel": "ldu_internal_kernel (atomic diagonal) + patch kernels",
                                  "achieved_GBps": bytes_asm / asm_s / 1e9, "frac": bytes_asm / asm_s / 1e9 / 8000.0,
                                  "ms": asm_s * 1e3, "bytes_per_launch": bytes_asm},
                     "conversion": {"achieved_GBps": bytes_csr / csr_s / 1e9, "frac": bytes_csr / csr_s / 1e9 / 8000.0,
                                    "ms": csr_s * 1e3, "bytes_per_launch": bytes_csr}},
    }
    if not args.no_cpu_baseline:
        from oracle import laplacian as L
        t1 = time.perf_counter()
        reps = 0
        while True:
            lo_o, up_o, dg_o, ic_o, bc_o = L.assemble(m, gc, gb, pb)
            L.to_csr(m, lo_o, up_o, dg_o, ic_o, bc_o)
            reps += 1
            if time.perf_counter() - t1 > min(args.cpu_seconds, 20.0):
                break
        cpu = time.perf_counter() - t1
        result["cpu_baseline"] = {"value": nc * reps / cpu, "unit": "cells/s", "cores": 1, "kind": "oracle",
                                  "cpu": cpu_model(), "sample": f"the whole mesh, {reps} pass(es), {cpu:.2f} s "
                                                                "(numpy, one thread)"}
        result["max_rel_diff_upper_vs_oracle"] = float(np.max(np.abs(up.cpu().numpy() - up_o) / np.abs(up_o)))
        rp_o, col_o, val_o, rhs_o = L.to_csr(m, lo_o, up_o, dg_o, ic_o, bc_o)
        result["max_abs_diff_csr_vs_oracle"] = float(np.max(np.abs(val.cpu().numpy() - val_o)))
    g.close()
    return result


def run_species(args):
    """Per-species networks (Section 2) vs one network, each trained on
    the same states for the same epochs, served on flame64 through the same
    checks and fallback.  One step = chem_surrogate_infer over the field from
    the pristine state (restored by a device copy inside the step)."""
    import torch

    from chemgen import fields as F
    from chemgen.surrogate_data import (epoch_orders, flame_like_states, init_params, init_species_params,
                                        network_dims, trajectory_starts)
    from paper_2312_13513_amd import chem

    dev = torch.device("cuda:0")
    mpy, path = mech_file("M9")
    mech = chem.Mechanism(path, 0)
    dt, K = 1e-6, mpy.K
    t = lambda a, dtype=torch.float64: torch.tensor(np.ascontiguousarray(a), dtype=dtype, device=dev)
    n_samples = min(args.train_samples, 524288)
    n_half = n_samples // 2
    T1, p1, Y1 = flame_like_states(mpy, n_half, seed=7)
    n_traj = max(2, n_half // args.traj_steps)
    T2, p2, Y2 = trajectory_starts(mpy, n_traj // 2, seed=8)
    T3, p3, Y3 = flame_like_states(mpy, n_traj - n_traj // 2, seed=9)
    T2, p2, Y2 = np.concatenate([T2, T3]), np.concatenate([p2, p3]), np.concatenate([Y2, Y3], axis=1)
    Tt, pt, Yt = t(T2), t(p2), t(Y2)
    Ts, Ys = [], []
    for _ in range(args.traj_steps):
        mech.integrate(Tt, pt, Yt, dt)
        Ts.append(Tt.clone())
        Ys.append(Yt.clone())
    Td = torch.cat([t(T1)] + Ts)
    pd = torch.cat([t(p1), t(np.full(n_traj * args.traj_steps, p2[0]))])
    Yd = torch.cat([t(Y1)] + Ys, dim=1).contiguous()
    del Ts, Ys
    Yn, Tn = Yd.clone(), Td.clone()
    mech.integrate(Tn, pd, Yn, dt)
    torch.cuda.synchronize()
    n_train = Td.shape[0]
    progress(f"species_nets: labelled {n_train} states")
    field = F.flame64(mpy)
    n = field.n
    T0, p0, Y0 = t(field.T), t(field.p), t(field.Y)
    # the reference: the plain FP64 integrator on the whole field
    Tp, Yp = T0.clone(), Y0.clone()
    mech.integrate(Tp, p0, Yp, dt)
    Tp_ = Tp.cpu().numpy()
    stream = torch.cuda.current_stream()
    nets = {"single": ((512, 256, 128), False), "species": ((1600, 800, 400), True)}
    out = {}
    for name, (h, per_species) in nets.items():
        s = chem.Surrogate(mech, *h, per_species=per_species)
        s.set_params(init_species_params(K, h, 11) if per_species else init_params(network_dims(K, *h), 11))
        s.fit_norm(Td, pd, Yd, Yn, dt)
        order = t(epoch_orders(n_train, args.epochs, 12), torch.int32)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        losses = s.train(Td, pd, Yd, Yn, epochs=args.epochs, batch=4096, lr0=1e-3, lr1=1e-5, order=order)
        torch.cuda.synchronize()
        train_s = time.perf_counter() - t0
        del order
        progress(f"species_nets: {name} trained in {train_s:.1f} s, loss {losses[0]:.4g} -> {losses[-1]:.4g}")
        # forward alone on the field's encoded rows
        X = torch.zeros((n, 64), dtype=torch.int16, device=dev)
        s.encode(T0, p0, Y0, X)
        o = torch.zeros((n, s.nout_pad), dtype=torch.float32, device=dev)
        for _ in range(2):
            s.forward(X, o)
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
        ev[0].record(stream)
        for _ in range(args.steps):
            s.forward(X, o)
        ev[1].record(stream)
        torch.cuda.synchronize()
        fwd_s = ev[0].elapsed_time(ev[1]) * 1e-3 / args.steps
        hh = (K + 2, *h)
        per_net = 2 * (hh[0] * hh[1] + hh[1] * hh[2] + hh[2] * hh[3])
        flops = n * (K * (per_net + 2 * hh[3]) if per_species else per_net + 2 * hh[3] * K)
        del X, o
        # served steps
        T, Y = T0.clone(), Y0.clone()
        cnt = torch.zeros(1, dtype=torch.int64, device=dev)

        def step(e=None):
            T.copy_(T0)
            Y.copy_(Y0)
            if e is not None:
                e[0].record(stream)
            s.infer(T, p0, Y, dt, fallback_count=cnt, stream=stream)
            if e is not None:
                e[1].record(stream)

        for _ in range(args.warmup):
            step()
        evs = [tuple(torch.cuda.Event(enable_timing=True) for _ in range(2)) for _ in range(args.steps)]
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for k in range(args.steps):
            step(evs[k])
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        step_ms = float(np.mean([a.elapsed_time(b) for a, b in evs]))
        Ts_ = T.cpu().numpy()
        out[name] = {
            "hidden": list(h), "networks": K if per_species else 1, "params": s.nparams,
            "served_cell_steps_per_s": n * args.steps / wall, "ms_per_step": wall / args.steps * 1e3,
            "infer_ms": step_ms, "fallback_cells": int(cnt.item()),
            "forward": {"ms": fwd_s * 1e3, "flops_per_cell": flops / n, "achieved_TFLOPs": flops / fwd_s / 1e12,
                        "frac_of_bf16_peak": flops / fwd_s / 2.5e15},
            "max_dT_vs_plain_gpu": float(np.abs(Ts_ - Tp_).max()),
            "mean_dT_vs_plain_gpu": float(np.abs(Ts_ - Tp_).mean()),
            "train": {"samples": n_train, "epochs": args.epochs, "s": train_s, "loss_first": float(losses[0]),
                      "loss_last": float(losses[-1])},
        }
        progress(f"species_nets: {name}: {out[name]['infer_ms']:.2f} ms/step, forward {fwd_s * 1e3:.3f} ms "
                 f"({flops / fwd_s / 1e12:.0f} TFLOP/s), fallback {out[name]['fallback_cells']}, "
                 f"max|dT| {out[name]['max_dT_vs_plain_gpu']:.3f} K")
        s.close()
    sp = out["species"]
    result = {
        "metric": "per-species vs single-network surrogate on flame64 (9 species, dt = 1e-6 s), served cell-steps/s",
        "value": sp["served_cell_steps_per_s"], "unit": "cell-steps/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": sp["ms_per_step"], "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "bf16", "data": "synthetic",
        "config": {"workload": "species_nets: flame64 (262,144 cells, 9 species), both networks trained on the same "
                               f"{n_train} integrator-labelled states for {args.epochs} epochs",
                   "ncells": n},
        "roofline": {"bound": "mfma", "achieved": sp["forward"]["achieved_TFLOPs"], "peak": 2500.0,
                     "unit": "TFLOP/s", "frac": sp["forward"]["frac_of_bf16_peak"], "traffic": None,
                     "kernel": "gemm_bf16_kernel (grouped, one group per species)"},
        "species": sp, "single": out["single"],
    }
    mech.close()
    return result


def props_flops(K: int) -> dict:
    """Algorithmic FP64 flops per cell of the property kernels (add, mul,
    div = 1, fused multiply-add = 2, log and sqrt = 20), from the
    definitions:
      transport  composition 5K + 2; per species the two ln T quartics
                 (8 each), T^(1/4) |P|, 1/s_k, T^(1/2) Q, X/lam and the two
                 sums (25 K); Wilke 7 K^2 (t = 1 + s_k c1 / s_j, t^2 c2,
                 X_j times it) plus 5 K; the K(K-1)/2 diffusion pairs
                 13 each (quartic, reciprocal, two products into the sums)
                 plus 8 K; log T and two square roots 60
      T from h   per Newton step 22 K + 10 (cp and h quartics, a6/T, the
                 sums, the step and the clamp), plus K for Y R / W."""
    pairs = K * (K - 1) // 2
    return {"transport": 7 * K * K + 13 * pairs + 38 * K + 62, "newton_step": 22 * K + 10, "newton_setup": K}


def run_props(args):
    """The Thermo field kernels on the TGV share: one step = restore the
    previous step's temperature (a device copy, timed), T from h by Newton
    (chem_T_from_h, cp out), then the transport properties at the new T
    (chem_transport_field: mu, lam and D).  h is the mixture enthalpy at the
    field's T (chem_mixture_h_cp, outside the timed region)."""
    import torch

    from chemgen.fields import newton_guess, seeded_sample, tgv_share
    from chemgen.transport import transport_fits
    from paper_2312_13513_amd import chem

    mech_obj, path = mech_file("M9")
    f = tgv_share(mech_obj)
    n, K = f.n, mech_obj.K
    fits = transport_fits(mech_obj, 9)
    guess = newton_guess(f.T, 12)
    m = chem.Mechanism(path)
    m.set_transport(*fits)
    dev = torch.device("cuda:0")
    t = lambda a: torch.tensor(np.ascontiguousarray(a), dtype=torch.float64, device=dev)
    Td, pd, Yd, Tg = t(f.T), t(f.p), t(f.Y), t(guess)
    h = torch.empty(n, dtype=torch.float64, device=dev)
    m.mixture_h_cp(Td, Yd, h, None)
    T = torch.empty_like(h)
    cp, mu, lam = torch.empty_like(h), torch.empty_like(h), torch.empty_like(h)
    D = torch.empty((K, n), dtype=torch.float64, device=dev)
    its = torch.empty(n, dtype=torch.int32, device=dev)
    stream = torch.cuda.current_stream()

    def step(ev=None):
        T.copy_(Tg)
        if ev is not None:
            ev[0].record(stream)
        m.T_from_h(h, Yd, T, cp, None, stream=stream)
        if ev is not None:
            ev[1].record(stream)
        m.transport(T, pd, Yd, mu, lam, D, stream=stream)
        if ev is not None:
            ev[2].record(stream)

    progress(f"props_tgv: {n} cells, K = {K}")
    for _ in range(args.warmup):
        step()
    evs = [tuple(torch.cuda.Event(enable_timing=True) for _ in range(3)) for _ in range(args.steps)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(args.steps):
        step(evs[k])
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    newton_s = float(np.mean([a.elapsed_time(b) for a, b, _ in evs])) * 1e-3
    trans_s = float(np.mean([b.elapsed_time(c) for _, b, c in evs])) * 1e-3
    # Newton steps taken (a separate call with the counts, outside the timing)
    T.copy_(Tg)
    m.T_from_h(h, Yd, T, None, its, stream=stream)
    torch.cuda.synchronize()
    steps_mean = float(its.double().mean().item())
    fl = props_flops(K)
    flops_tr = fl["transport"] * n
    flops_nw = (fl["newton_step"] * steps_mean + fl["newton_setup"]) * n
    bytes_tr = n * 8 * (K + 2) * 2            # T, p, Y in; mu, lam, D out
    bytes_nw = n * 8 * (K + 4)                # h, T, Y in; T, cp out
    peak_f = FP64_PEAK_TFLOPS * 1e12

    def roof(flops, nbytes, secs, kernel):
        t_hbm, t_alu = nbytes / 8e12, flops / peak_f
        if t_hbm >= t_alu:
            return {"bound": "hbm", "achieved": nbytes / secs / 1e9, "peak": 8000.0, "unit": "GB/s",
                    "frac": nbytes / secs / 8e12, "traffic": traffic_for("props_tgv", kernel), "kernel": kernel,
                    "kernel_ms": secs * 1e3, "bytes_per_launch": nbytes, "flops_per_launch": flops,
                    "fp64_frac": flops / secs / peak_f}
        return {"bound": "alu", "achieved": flops / secs / 1e12, "peak": FP64_PEAK_TFLOPS, "unit": "TFLOP/s",
                "frac": flops / secs / peak_f, "traffic": traffic_for("props_tgv", kernel), "kernel": kernel,
                "kernel_ms": secs * 1e3, "bytes_per_launch": nbytes, "flops_per_launch": flops,
                "hbm_frac": nbytes / secs / 8e12}

    # the library's kernel bound for K species (exact when K equals it)
    km = next(b for b in (9, 12, 16, 20, 24, 36, 48, 64) if K <= b)
    ex = "true" if km == K else "false"
    r_tr = roof(flops_tr, bytes_tr, trans_s, f"transport_kernel<{km},true,3,{ex}>")
    r_nw = roof(flops_nw, bytes_nw, newton_s, f"t_from_h_kernel<{km},{ex}>")
    dominant = r_tr if trans_s >= newton_s else r_nw
    result = {
        "metric": "thermo/transport field properties (T from h, mu, lambda, D), cells/s",
        "value": n * args.steps / wall, "unit": "cells/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": wall / args.steps * 1e3, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": "props_tgv: 256x128x128 = 4,194,304-cell flame field (one GPU's share of the "
                               "256^3 TGV mesh on four GPUs), 9 species, Newton from T + U(-20, 20) K, seeded "
                               "Lennard-Jones transport fits", "ncells": n, "species": K},
        "roofline": dominant,
        "kernels": {"t_from_h": r_nw, "transport": r_tr},
        "newton_steps_mean": steps_mean,
    }
    if not args.no_cpu_baseline:
        from oracle import OracleMech
        from oracle import transport as TR
        om = OracleMech(path)
        ns = args.cpu_sample or 1000000
        idx = seeded_sample(n, ns, 17)
        Ys, Ts, ps = f.Y[:, idx], f.T[idx], f.p[idx]
        h_s = h.cpu().numpy()[idx]
        t1 = time.perf_counter()
        T_o, cp_o, _ = TR.thermo_field(om, h_s, Ys, guess[idx])
        mu_o, lam_o, D_o = TR.transport(*fits, mech_obj.molar_masses(), T_o, ps, Ys)
        cpu = time.perf_counter() - t1
        result["cpu_baseline"] = {"value": idx.size / cpu, "unit": "cells/s", "cores": 1, "kind": "oracle",
                                  "cpu": cpu_model(), "sample": f"{idx.size} seeded cells of the field, one pass, "
                                                                f"{cpu:.2f} s (C Newton per cell, numpy transport, "
                                                                "one thread)"}
        Tgpu = T.cpu().numpy()[idx]
        result["max_abs_dT_vs_oracle"] = float(np.max(np.abs(Tgpu - T_o)))
        result["max_rel_dmu_vs_oracle"] = float(np.max(np.abs(mu.cpu().numpy()[idx] / mu_o - 1)))
        result["max_rel_dD_vs_oracle"] = float(np.max(np.abs(D.cpu().numpy()[:, idx] / D_o - 1)))
    m.close()
    return result


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="flame64",
                    choices=("flame64", "cells4096", "zones128", "surrogate", "laplacian128", "props_tgv",
                             "species_nets"))
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--schedule", type=int, default=None, choices=(-2, -1, 0, 1, 2),
                    help="integrator workloads: -2 autotuned (flame64 default), -1 library choice, 0 thread, "
                         "1 wave, 2 tile per cell")
    ap.add_argument("--cpu-sample", type=int, default=0, help="cells for the oracle timing (0 = workload default)")
    ap.add_argument("--cpu-seconds", type=float, default=10.0, help="repeat the oracle sample until this long")
    ap.add_argument("--train-samples", type=int, default=2 * 1024 * 1024)
    ap.add_argument("--traj-steps", type=int, default=64)
    ap.add_argument("--epochs", type=int, default=20)
    ap.add_argument("--field", default="flame256x128x128", choices=("flame256x128x128", "flame256"))
    ap.add_argument("--graph", action="store_true", help="surrogate: replay the step as one captured HIP graph")
    ap.add_argument("--evolve", action="store_true",
                    help="surrogate: timed steps advance the field (no restore); the drift against the plain "
                         "integrator over the same steps is reported on a seeded sample")
    ap.add_argument("--drift-cells", type=int, default=16384, help="surrogate --evolve: cells of the drift check")
    ap.add_argument("--rollout-rounds", type=int, default=None,
                    help="surrogate: rounds of rollout data aggregation after the first training "
                         "(default 3 with --evolve, else 0: the single-step workload trains on 2M states, "
                         "20 epochs)")
    ap.add_argument("--rollout-cells", type=int, default=65536, help="surrogate: flame-like states per rollout")
    ap.add_argument("--rollout-steps", type=int, default=32, help="surrogate: flow steps of each rollout")
    ap.add_argument("--rollout-epochs", type=int, default=10, help="surrogate: epochs after each rollout")
    ap.add_argument("--shuffle", action="store_true",
                    help="integrator workloads: the field's cells in a seeded random order")
    ap.add_argument("--plain-cells", type=int, default=262144,
                    help="surrogate: cells of the plain-integrator comparison (a seeded sample when fewer)")
    ap.add_argument("--surr-oracle-cells", type=int, default=65536,
                    help="surrogate: seeded subset of served cells integrated by the oracle (accuracy, CPU rate)")
    ap.add_argument("--fwd-rows", type=int, default=2097152, help="surrogate: rows of the timed forward launch")
    ap.add_argument("--no-surrogate", action="store_true",
                    help="default workload: leave out the surrogate leg")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a plain device copy of 512 MiB three times (scales the HBM "
                         "byte counters of a profiler run)")
    args = ap.parse_args()
    if args.rollout_rounds is None:
        args.rollout_rounds = 3 if args.evolve else 0
    if args.copy_calibration:
        import torch
        src = torch.ones(64 << 20, dtype=torch.float64, device="cuda:0")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_per_dispatch": src.numel() * 8, "dispatches": 3}))
        return
    if args.gpus != 1:
        print(f"bench.py: this benchmark runs on one GPU only (asked for {args.gpus}); the per-cell "
              "chemistry shards trivially across GPUs but no multi-GPU path is built", file=sys.stderr)
        sys.exit(2)
    if args.workload == "surrogate":
        result = run_surrogate(args)
    elif args.workload == "laplacian128":
        result = run_laplacian(args)
    elif args.workload == "props_tgv":
        result = run_props(args)
    elif args.workload == "species_nets":
        result = run_species(args)
    else:
        result = run_integrator(args, args.workload)
        if args.workload == "flame64" and not args.no_surrogate:
            # the metric's second half: the surrogate with per-cell fallback on
            # the 4,194,304-cell field, trained in this run
            import torch
            torch.cuda.empty_cache()
            result["surrogate"] = run_surrogate(args, nested=True)
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
