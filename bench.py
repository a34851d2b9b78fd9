"""Throughput of the whole hot path on one MI355X.

A step is one fmm_build_tree + fmm_traverse + fmm_evaluate over a seeded
synthetic particle set already resident in HBM (the FMM particles/s metric).
Prints one JSON line.  ``--gpus`` above 1 is rejected: this build runs on one
GPU.

The JSON carries, beside the throughput:
  roofline      the dominant kernel (the batched M2L GEMM) against FP32 MFMA
                peak: algorithmic flops 2 (p+1)^4 per M2L pair it handles, over
                its average duration measured with HIP events on the library's
                stream during a separate timed pass
  accuracy      relative L2 error of potential and field on seeded targets
                against the FP64 direct sum of the oracle
  cpu_baseline  the oracle (FP64 CPU, all host threads) timed on a bounded
                sample of the same workload
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

PEAK_FP32_MFMA = 157.3e12


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="uniform1m_p10")
    ap.add_argument("--n", type=int, default=None, help="override particle count")
    ap.add_argument("--policy", type=int, default=0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-sample", type=int, default=65536)
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU; --gpus must be 1"}))
        sys.exit(2)

    import torch

    import synth
    from paper_1108_5815_amd import FMM

    x, y, z, q, tg, w = synth.make_workload(args.workload, args.n)
    n, p, theta, ncrit = w["n"], w["p"], w["theta"], w["ncrit"]
    dev = "cuda:0"
    dt = torch.float32
    X, Y, Z, Q = (torch.tensor(a, dtype=dt, device=dev) for a in (x, y, z, q))
    f = FMM(0)
    phi = torch.empty(n, dtype=dt, device=dev)
    E = torch.empty((3, n), dtype=dt, device=dev)

    tune_s = None
    train = None
    if args.policy == 2:
        # one-time kernel pre-calculation, reported separately from the steps
        t0 = time.perf_counter()
        f.tune(p)
        tune_s = time.perf_counter() - t0
    if args.policy == 3:
        # one-time generation of timing records and training of the cost model
        t0 = time.perf_counter()
        loss = f.costmodel_train(p, theta, epochs=3000, seed=7)
        train = {"seconds": time.perf_counter() - t0, "final_loss_log2": loss,
                 "records": int(f.costmodel_records()[1].size)}

    def step():
        f.build_tree(X, Y, Z, Q, ncrit)
        f.traverse(p, theta, args.policy)
        f.evaluate(out=(phi, E))

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ms = (t1 - t0) * 1e3 / args.steps
    value = n / (ms * 1e-3)
    sizes = f.sizes()

    # per-phase and dominant-kernel timing (separate pass, events on the library stream)
    f.set_timing(True)
    reps = max(3, min(args.steps, 10))
    acc_t = {}
    for _ in range(reps):
        step()
        for k, v in f.timings().items():
            acc_t[k] = acc_t.get(k, 0.0) + v / reps
    f.set_timing(False)
    torch.cuda.synchronize()
    m2l_flops = 2.0 * (p + 1) ** 4 * gemm_pairs(f)
    gemm_ms = acc_t.get("m2l_gemm", 0.0)
    achieved = m2l_flops / (gemm_ms * 1e-3) if gemm_ms > 0 else 0.0

    out = {
        "metric": "FMM particles/sec at <=1e-5 rel L2 potential error",
        "value": value,
        "unit": "particles/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": args.workload, "n": n, "p": p, "theta": theta, "ncrit": ncrit,
                   "policy": ["fmm", "treecode", "hybrid_timed", "hybrid_mlp"][args.policy],
                   "precision": "fp32", "distribution": w["dist"]},
        "sizes": sizes,
        "m2l_split": dict(zip(("batched", "general"), f.m2l_split())),
        "phase_ms": {k: round(v, 4) for k, v in acc_t.items()},
        "tuning": None if tune_s is None else {"seconds": tune_s, "unit_costs_ns": f.costs().tolist()},
        "cost_model_training": train,
        "roofline": {"kernel": "k_m2l_gemm", "bound": "mfma", "achieved": achieved / 1e12,
                     "peak": PEAK_FP32_MFMA / 1e12, "unit": "TFLOP/s", "frac": achieved / PEAK_FP32_MFMA,
                     "traffic": None, "flops_per_launch": m2l_flops, "avg_ms": gemm_ms},
    }
    # accuracy on the seeded targets (FP64 direct sum of the oracle) and the CPU baseline
    if not args.no_cpu_baseline:
        out.update(cpu_leg(x, y, z, q, tg, w, phi, E, args))
    print(json.dumps(out))


def gemm_pairs(f) -> int:
    """M2L pairs handled by the batched GEMM = all M2L pairs minus the general ones."""
    from paper_1108_5815_amd.binding import lib  # noqa: F401
    return f.sizes()["m2l"] - f.general_pairs()


def cpu_leg(x, y, z, q, tg, w, phi, E, args):
    import oracle
    import synth
    xs, ys, zs, qs = (np.asarray(a, dtype=np.float32).astype(np.float64) for a in (x, y, z, q))
    t0 = time.perf_counter()
    pd, Ed = oracle.direct(xs, ys, zs, qs, tg)
    t_direct = time.perf_counter() - t0
    ph = phi.double().cpu().numpy()[tg]
    Eg = E.double().cpu().numpy().T[tg]
    acc = {"accuracy": {"phi_rel_l2": oracle.rel_l2(ph, pd), "E_rel_l2": oracle.rel_l2(Eg, Ed),
                        "targets": int(tg.size), "reference": "FP64 direct sum (oracle)"}}
    # bounded sample: the oracle FMM on the first `cpu_sample` points of the same generator
    ns = min(args.cpu_sample, w["n"])
    xs2, ys2, zs2, qs2, _, w2 = synth.make_workload(args.workload, ns)
    t0 = time.perf_counter()
    oracle.fmm(xs2, ys2, zs2, qs2, w["p"], w["theta"], w["ncrit"])
    t_fmm = time.perf_counter() - t0
    acc["cpu_baseline"] = {"value": ns / t_fmm, "unit": "particles/s", "cores": oracle.num_threads(),
                           "kind": "oracle",
                           "sample": f"oracle FP64 FMM on {ns} points of the same distribution and "
                                     f"parameters ({t_fmm:.1f} s); direct-sum reference on "
                                     f"{tg.size} targets took {t_direct:.1f} s"}
    return acc


if __name__ == "__main__":
    main()
