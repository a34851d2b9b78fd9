"""Throughput of the whole hot path on one MI355X.

A step is one fmm_build_tree + fmm_traverse + fmm_evaluate over a seeded
synthetic particle set already resident in HBM (FMM particles/s).  The
default compares two forms of the method on the same workload (4,194,304
Plummer points, p = 10, theta = 0.4, ncrit = 64):

  value (learned + mixed): interaction kinds chosen by the learned cost
        model, same-level M2L in split-BF16 on the matrix cores;
  plain: interaction kinds chosen from the timed kernel pre-calculation,
        FP32 everywhere.

Both are checked against the FP64 direct sum on the workload's seeded
targets (the metric is quoted at <= 1e-5 relative L2 potential error).
One-time tuning and training are timed separately, outside the steps.

The JSON line also carries:
  roofline      the dominant kernel of the measured form (P2P against the
                FP32 vector peak with 20 flops per particle pair, or the
                M2L GEMM against the matrix-core peak of its precision with
                2 (p+1)^4 flops per pair), timed with HIP events on the
                library's stream in a separate pass
  cpu_baseline  the oracle (FP64 CPU, all host threads) on a bounded sample
                of the same workload
``--gpus`` above 1 is rejected: this build runs on one GPU.
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

PEAK = {"fp32_vector": 157.3e12, "fp32_mfma": 157.3e12, "bf16_mfma": 2.5e15}
POLICIES = ["fmm", "treecode", "hybrid_timed", "hybrid_mlp"]
PRECISIONS = ["fp32", "split_bf16"]


def run_form(f, X, Y, Z, Q, phi, E, w, policy, precision, steps, warmup):
    n, p, theta, ncrit = w["n"], w["p"], w["theta"], w["ncrit"]
    import torch
    prep = {}
    if policy == 2:
        t0 = time.perf_counter()
        f.tune(p, precision)
        prep = {"tuning_s": time.perf_counter() - t0, "unit_costs_ns": f.costs().tolist()}
    elif policy == 3:
        t0 = time.perf_counter()
        loss = f.costmodel_train(p, theta, epochs=3000, seed=7, precision=precision)
        prep = {"training_s": time.perf_counter() - t0, "final_loss_log2": loss,
                "records": int(f.costmodel_records()[1].size)}

    def step():
        f.build_tree(X, Y, Z, Q, ncrit)
        f.traverse(p, theta, policy)
        f.evaluate(precision, out=(phi, E))

    for _ in range(warmup):
        step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        step()
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1e3 / steps
    # per-phase times with events on the library's stream (separate pass)
    f.set_timing(True)
    reps = max(3, min(steps, 5))
    ph = {}
    for _ in range(reps):
        step()
        for k, v in f.timings().items():
            ph[k] = ph.get(k, 0.0) + v / reps
    f.set_timing(False)
    torch.cuda.synchronize()
    sizes = f.sizes()
    batched, general = f.m2l_split()
    work = f.work()
    return {"ms_per_step": ms, "value": n / (ms * 1e-3), "phase_ms": {k: round(v, 4) for k, v in ph.items()},
            "sizes": sizes, "m2l_split": {"batched": batched, "general": general}, "work": work,
            "policy": POLICIES[policy], "precision": PRECISIONS[precision], "prep": prep}


def roofline(res, p, precision):
    ph = res["phase_ms"]
    p2p_flops = 20.0 * res["work"]["p2p_particle_pairs"]
    m2l_flops = 2.0 * (p + 1) ** 4 * res["m2l_split"]["batched"]
    k_p2p = {"kernel": "k_p2p", "bound": "alu", "achieved": p2p_flops / (ph["p2p"] * 1e-3) / 1e12,
             "peak": PEAK["fp32_vector"] / 1e12, "unit": "TFLOP/s", "avg_ms": ph["p2p"],
             "flops_per_launch": p2p_flops}
    peak_m2l = PEAK["bf16_mfma"] if precision == 1 else PEAK["fp32_mfma"]
    k_m2l = {"kernel": "k_m2l_bf16" if precision == 1 else "k_m2l_gemm", "bound": "mfma",
             "achieved": m2l_flops / (ph["m2l_gemm"] * 1e-3) / 1e12 if ph["m2l_gemm"] > 0 else 0.0,
             "peak": peak_m2l / 1e12, "unit": "TFLOP/s", "avg_ms": ph["m2l_gemm"], "flops_per_launch": m2l_flops}
    for k in (k_p2p, k_m2l):
        k["frac"] = k["achieved"] / k["peak"]
        k["traffic"] = None
    dom = k_p2p if ph["p2p"] >= ph["m2l_gemm"] else k_m2l
    other = k_m2l if dom is k_p2p else k_p2p
    out = dict(dom)
    out["other"] = other
    return out


def accuracy(x, y, z, q, tg, phi, E):
    import oracle
    xs, ys, zs, qs = (np.asarray(a, dtype=np.float32).astype(np.float64) for a in (x, y, z, q))
    pd, Ed = oracle.direct(xs, ys, zs, qs, tg)
    ph = phi.double().cpu().numpy()[tg]
    Eg = E.double().cpu().numpy().T[tg]
    return {"phi_rel_l2": oracle.rel_l2(ph, pd), "E_rel_l2": oracle.rel_l2(Eg, Ed), "targets": int(tg.size),
            "reference": "FP64 direct sum (oracle)"}


def cpu_baseline(w, workload, sample):
    import oracle
    import synth
    ns = min(sample, w["n"])
    xs, ys, zs, qs, _, _ = synth.make_workload(workload, ns)
    xs, ys, zs, qs = (np.asarray(a, dtype=np.float32).astype(np.float64) for a in (xs, ys, zs, qs))
    t0 = time.perf_counter()
    oracle.fmm(xs, ys, zs, qs, w["p"], w["theta"], w["ncrit"])
    t = time.perf_counter() - t0
    return {"value": ns / t, "unit": "particles/s", "cores": oracle.num_threads(), "kind": "oracle",
            "sample": f"oracle FP64 FMM (FMM policy) on the first {ns} points of the same generator, "
                      f"same p, theta, ncrit ({t:.1f} s)"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="plummer4m_p10")
    ap.add_argument("--n", type=int, default=None, help="override particle count")
    ap.add_argument("--policy", type=int, default=3, help="0 fmm, 1 treecode, 2 timed hybrid, 3 learned hybrid")
    ap.add_argument("--precision", type=int, default=1, help="0 fp32, 1 split-bf16 M2L")
    ap.add_argument("--no-plain", action="store_true", help="skip the plain (timed FP32) comparison")
    ap.add_argument("--no-cpu-baseline", action="store_true", help="skip the oracle legs (accuracy, CPU timing)")
    ap.add_argument("--cpu-sample", type=int, default=16384)
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU; --gpus must be 1"}))
        sys.exit(2)

    import torch

    import synth
    from paper_1108_5815_amd import FMM

    x, y, z, q, tg, w = synth.make_workload(args.workload, args.n)
    n, p = w["n"], w["p"]
    dev = "cuda:0"
    X, Y, Z, Q = (torch.tensor(a, dtype=torch.float32, device=dev) for a in (x, y, z, q))
    f = FMM(0)
    phi = torch.empty(n, dtype=torch.float32, device=dev)
    E = torch.empty((3, n), dtype=torch.float32, device=dev)

    main_res = run_form(f, X, Y, Z, Q, phi, E, w, args.policy, args.precision, args.steps, args.warmup)
    acc_main = None if args.no_cpu_baseline else accuracy(x, y, z, q, tg, phi, E)
    plain = None
    if not args.no_plain and (args.policy, args.precision) != (2, 0):
        plain = run_form(f, X, Y, Z, Q, phi, E, w, 2, 0, args.steps, args.warmup)
        if not args.no_cpu_baseline:
            plain["accuracy"] = accuracy(x, y, z, q, tg, phi, E)
        plain["speedup_of_value"] = main_res["value"] / plain["value"]

    out = {
        "metric": "FMM particles/sec at <=1e-5 rel L2 potential error; learned+mixed vs plain",
        "value": main_res["value"],
        "unit": "particles/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": main_res["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32+bf16" if args.precision == 1 else "f32",
        "data": "synthetic",
        "config": {"workload": args.workload, "n": n, "p": p, "theta": w["theta"], "ncrit": w["ncrit"],
                   "distribution": w["dist"], "policy": main_res["policy"], "precision": main_res["precision"]},
        "accuracy": acc_main,
        "form": main_res,
        "plain": plain,
        "roofline": roofline(main_res, p, args.precision),
    }
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(w, args.workload, args.cpu_sample)
    print(json.dumps(out))


if __name__ == "__main__":
    main()
