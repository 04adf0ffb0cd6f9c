"""Benchmark: chemistry cell-steps/s of the plain FP64 GPU integrator on the
64^3 flame field (262,144 cells, 9-species / 21-reaction synthetic mechanism,
dt = 1e-6 s, rtol 1e-8, atol 1e-12).

One step = one call of chem_integrate over all cells, starting from the same
pristine field (restored by a device-to-device copy inside the step, so the
copy is timed too).  Prints ONE JSON line with the metric, the roofline of the
integrator kernel (algorithmic FP64 flops from the per-cell counters, kernel
time from HIP events on the launch stream) and the CPU oracle timed on the
host cores.
"""
from __future__ import annotations

import argparse
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
FP64_PEAK_TFLOPS = 78.6          # MI355X FP64 vector, dense
TRANSCENDENTAL_FLOPS = 20        # exp / log / pow / sqrt counted as 20 flops


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


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-sample", type=int, default=0,
                    help="cells for the oracle timing (0 = the whole field)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a plain device copy of 512 MiB three times (scales the HBM "
                         "byte counters of a profiler run)")
    args = ap.parse_args()
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
        print(f"bench.py: this build runs on one GPU only (asked for {args.gpus}); the per-cell "
              "chemistry shards trivially across GPUs but no multi-GPU path is built", file=sys.stderr)
        sys.exit(2)

    import torch

    from chemgen.fields import flame64
    from chemgen.mechanism import standard_mechanism
    from paper_2312_13513_amd import chem

    dev = torch.device("cuda:0")
    mech_py = standard_mechanism("M9")
    field = flame64(mech_py)
    n, K, R = field.n, mech_py.K, mech_py.R
    tmp = tempfile.mkdtemp()
    mech_path = os.path.join(tmp, "M9.mech")
    mech_py.write(mech_path)
    mech = chem.Mechanism(mech_path, 0)

    T0 = torch.tensor(field.T, dtype=torch.float64, device=dev)
    p0 = torch.tensor(field.p, dtype=torch.float64, device=dev)
    Y0 = torch.tensor(field.Y, dtype=torch.float64, device=dev)
    T, Y = T0.clone(), Y0.clone()
    status = torch.zeros(n, dtype=torch.int32, device=dev)
    counters = torch.zeros(6 * n, dtype=torch.int32, device=dev)
    opts = chem.chem_default_opts()
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
    torch.cuda.synchronize()
    events = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
              for _ in range(args.steps)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(args.steps):
        step(events[k])
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    kern_ms = [a.elapsed_time(b) for a, b in events]
    avg_kern_s = float(np.mean(kern_ms)) * 1e-3

    st = status.cpu().numpy()
    cnt = counters.cpu().numpy().reshape(6, n)
    Tg, Yg = T.cpu().numpy(), Y.cpu().numpy()
    fl = algorithmic_flops(K, R, cnt)
    achieved = fl["total"] / avg_kern_s / 1e12
    value = n * args.steps / wall

    result = {
        "metric": METRIC,
        "value": value,
        "unit": "cell-steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": wall / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "flame64: 262,144 cells (64^3 smooth flame field), synthetic "
                               "9-species/21-reaction mechanism, dt=1e-6 s, rtol 1e-8, atol 1e-12, "
                               "plain FP64 BDF, one thread per cell",
                   "ncells": n, "species": K, "reactions": R, "dt": field.dt},
        "roofline": {"bound": "alu", "achieved": achieved, "peak": FP64_PEAK_TFLOPS,
                     "unit": "TFLOP/s", "frac": achieved / FP64_PEAK_TFLOPS, "traffic": None,
                     "kernel": "bdf_thread_kernel<9>", "kernel_ms": avg_kern_s * 1e3,
                     "flops_per_launch": fl["total"]},
        "substeps": {"mean": float(cnt[0].mean()), "max": int(cnt[0].max()),
                     "p50": float(np.median(cnt[0])), "rhs_per_cell": float(cnt[1].mean()),
                     "jac_per_cell": float(cnt[2].mean())},
        "status_ok_frac": float(np.mean(st == 0)),
    }

    if not args.no_cpu_baseline:
        import oracle
        om = oracle.OracleMech(mech_path)
        if args.cpu_sample and args.cpu_sample < n:
            from chemgen.fields import seeded_sample
            idx = seeded_sample(n, args.cpu_sample, seed=5)
        else:
            idx = np.arange(n)
        t1 = time.perf_counter()
        To, Yo, so, co, used = om.integrate(field.T[idx], field.p[idx], field.Y[:, idx], field.dt)
        tc = time.perf_counter() - t1
        result["cpu_baseline"] = {
            "value": idx.size / tc, "unit": "cell-steps/s", "cores": int(used), "kind": "oracle",
            "sample": f"{idx.size} cells of the same field ({'all' if idx.size == n else 'seeded sample'}), "
                      f"one flow step, {tc:.2f} s wall on {used} threads of {os.cpu_count()} host CPUs"}
        result["max_dT_vs_oracle"] = float(np.abs(Tg[idx] - To).max())
        result["max_dY_vs_oracle"] = float(np.abs(Yg[:, idx] - Yo).max())
        result["steps_equal_frac"] = float(np.mean(cnt[0][idx] == co[:, 0]))
    mech.close()
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
