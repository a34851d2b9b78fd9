"""Throughput of the whole hot path on one MI355X.

A step is one fmm_build_tree + fmm_traverse + fmm_evaluate over a seeded
synthetic particle set already resident in HBM (FMM particles/s).  The
default compares two forms of the method on the same workload (4,194,304
Plummer points, p = 10, theta = 0.4, ncrit = 64):

  value (learned + mixed): interaction kinds chosen by the learned cost
        model, same-level M2L in split-BF16 on the matrix cores;
  plain: interaction kinds chosen from the timed kernel pre-calculation,
        FP32 everywhere;
  timed_bf16: the timed kernel pre-calculation on split-BF16 timings with
        split-BF16 M2L (the network judged against the timed tuner at equal
        precision).

The learned model is the library's, trained on the GPU by its own kernels
(fmm_costmodel_train); by default the model saved for this device, order,
theta and precision under paper_1108_5815_amd/costmodels/ is loaded (so that
runs and profiles see the same lists), else one is trained (--train forces
training; --save-costmodel keeps it).

Both are checked against the FP64 direct sum on the workload's seeded
targets (the metric is quoted at <= 1e-5 relative L2 potential error).
One-time tuning and training are timed separately, outside the steps.

The JSON line also carries:
  roofline      the dominant kernel of the measured form (P2P against the
                FP32 vector peak with 20 flops per particle pair, or the
                M2L GEMM kernel against the matrix-core peak of its precision
                with 2 (p+1)^4 flops per pair), timed with HIP events around
                the kernel on the library's stream in a separate pass that
                runs every kernel in order (no concurrent near field); the
                figures under the tuned, concurrent schedule are in_step
  cpu_baseline  the oracle (FP64 CPU) timed on the host: its FMM on a
                262,144-point sample of the workload (all host threads) and
                on 16,384 points (one thread), and its direct sum on the
                workload's targets (all threads; 100 of them on one thread)
``--workload batch256_p8`` times the batch form instead: 256 independent
instances of uneven size in one fmm_evaluate_batch per step, beside the same
instances evaluated one after another.
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


def costmodel_file(w, precision):
    """The committed model of this device for (p, theta, precision)."""
    import torch
    pr = torch.cuda.get_device_properties(0)
    arch = pr.gcnArchName.split(":")[0]
    return os.path.join(ROOT, "paper_1108_5815_amd", "costmodels",
                        f"{arch}_{pr.multi_processor_count}cu_p{w['p']}_theta{w['theta']}_"
                        f"{PRECISIONS[precision]}.txt")


def prepare_costmodel(f, w, precision, args):
    p, theta = w["p"], w["theta"]
    path = args.costmodel or costmodel_file(w, precision)
    if not args.train and os.path.exists(path):
        t0 = time.perf_counter()
        f.costmodel_load(path, p, precision)
        meta = dict(l.split(" ", 1) for l in open(path).read().split("\n")[:8] if " " in l)
        return {"costmodel": "loaded", "path": os.path.relpath(path, ROOT), "load_s": time.perf_counter() - t0,
                "trained_on": meta.get("device"), "training_s": float.fromhex(meta["training_seconds"])
                if meta.get("training_seconds", "nan") not in ("nan", "-nan") else None,
                "final_loss_log2": float.fromhex(meta["loss"]) if meta.get("loss", "nan") not in ("nan", "-nan")
                else None, "records": int(meta.get("records", 0))}
    t0 = time.perf_counter()
    loss = f.costmodel_train(p, theta, epochs=6000, seed=7, precision=precision)
    prep = {"costmodel": "trained", "training_s": time.perf_counter() - t0, "final_loss_log2": loss,
            "records": int(f.costmodel_records()[1].size)}
    if args.save_costmodel:
        f.costmodel_save(args.save_costmodel)
        prep["saved"] = args.save_costmodel
    return prep


def run_form(f, X, Y, Z, Q, phi, E, w, policy, precision, steps, warmup, args):
    n, p, theta, ncrit = w["n"], w["p"], w["theta"], w["ncrit"]
    import torch
    prep = {}
    if policy == 2:
        t0 = time.perf_counter()
        f.tune(p, precision)
        prep = {"tuning_s": time.perf_counter() - t0, "unit_costs_ns": f.costs().tolist()}
    elif policy == 3:
        prep = prepare_costmodel(f, w, precision, args)

    def step():
        f.build_tree(X, Y, Z, Q, ncrit)
        f.traverse(p, theta, policy)
        f.evaluate(precision, out=(phi, E))

    # tile shapes and schedule for this workload (the library's autotuner)
    f.build_tree(X, Y, Z, Q, ncrit)
    f.traverse(p, theta, policy)
    t0 = time.perf_counter()
    prep["tile_config"] = f.autotune(precision, reps=2)
    prep["autotune_s"] = time.perf_counter() - t0
    for _ in range(warmup):
        step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        step()
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1e3 / steps
    reps = max(3, min(steps, 5))

    def phases():
        f.set_timing(True)
        ph = {}
        for _ in range(reps):
            step()
            for k, v in f.timings().items():
                ph[k] = ph.get(k, 0.0) + v / reps
        f.set_timing(False)
        torch.cuda.synchronize()
        return {k: round(v, 4) for k, v in ph.items()}

    # per-phase times with events on the library's stream (separate passes):
    # under the tuned schedule (the steps'), then with every kernel in order,
    # so that each kernel's own duration is taken alone
    sched = prep["tile_config"]["schedule"]
    ph_step = phases()
    f.set_overlap(0)
    ph_alone = phases()
    f.set_overlap(sched)
    sizes = f.sizes()
    batched, general = f.m2l_split()
    work = f.work()
    return {"ms_per_step": ms, "value": n / (ms * 1e-3), "phase_ms": ph_alone, "phase_ms_in_step": ph_step,
            "sizes": sizes, "m2l_split": {"batched": batched, "general": general}, "work": work,
            "gemm_shape": f.gemm_shape(),
            "policy": POLICIES[policy], "precision": PRECISIONS[precision], "prep": prep}


# sources a kernel's recorded traffic depends on (the GEMM kernels' slot
# groups are set in k_m2l_gemm.hip)
KERNEL_SOURCES = {"k_m2l_bf16": ("k_m2l_bf16.hip", "k_m2l_gemm.hip"), "k_m2l_gemm": ("k_m2l_gemm.hip",),
                  "k_p2p": ("k_p2p.hip",)}


def measured_traffic(kernel, workload):
    """HBM bytes per launch from the committed hardware-counter summary
    (profiles/fmm_<workload>_traffic.md), or None when there is none or the
    kernel's sources changed since the counters were taken (the recorded key is
    the SHA-256 of those source files, concatenated in order)."""
    import hashlib
    path = os.path.join(ROOT, "profiles", f"fmm_{workload}_traffic.md")
    if kernel not in KERNEL_SOURCES or not os.path.exists(path):
        return None
    h = hashlib.sha256()
    for f in KERNEL_SOURCES[kernel]:
        h.update(open(os.path.join(ROOT, "paper_1108_5815_amd", "csrc", f), "rb").read())
    sha = h.hexdigest()[:12]
    for line in open(path):
        t = line.split()
        if len(t) == 5 and t[0] == "traffic_per_launch" and t[1] == kernel:
            kv = dict(x.split("=", 1) for x in t[2:])
            if kv.get("workload") == workload and kv.get("sha") == sha:
                return int(kv["bytes"])
    return None


def roofline(res, p, precision, workload=None):
    """Dominant kernel of the form against its peak: algorithmic flops of one
    launch over the launch's event-timed duration with every kernel in order
    (in_step: the same under the tuned, concurrent schedule)."""
    def kernels(ph):
        p2p_flops = 20.0 * res["work"]["p2p_particle_pairs"]
        m2l_flops = 2.0 * (p + 1) ** 4 * res["m2l_split"]["batched"]
        k_p2p = {"kernel": "k_p2p", "bound": "alu", "achieved": p2p_flops / (ph["p2p"] * 1e-3) / 1e12,
                 "peak": PEAK["fp32_vector"] / 1e12, "unit": "TFLOP/s", "avg_ms": ph["p2p"],
                 "flops_per_launch": p2p_flops}
        peak_m2l = PEAK["bf16_mfma"] if precision == 1 else PEAK["fp32_mfma"]
        tk = ph.get("m2l_gemm_kernel", 0.0)
        k_m2l = {"kernel": "k_m2l_bf16" if precision == 1 else "k_m2l_gemm", "bound": "mfma",
                 "achieved": m2l_flops / (tk * 1e-3) / 1e12 if tk > 0 else 0.0,
                 "peak": peak_m2l / 1e12, "unit": "TFLOP/s", "avg_ms": tk, "flops_per_launch": m2l_flops,
                 "batched_m2l_pairs": res["m2l_split"]["batched"]}
        for k in (k_p2p, k_m2l):
            k["frac"] = k["achieved"] / k["peak"]
        return k_p2p, k_m2l

    k_p2p, k_m2l = kernels(res["phase_ms"])
    s_p2p, s_m2l = kernels(res["phase_ms_in_step"])
    for k in (k_p2p, k_m2l):
        k["traffic"] = measured_traffic(k["kernel"], workload) if workload else None
    k_p2p["in_step"] = {x: s_p2p[x] for x in ("achieved", "avg_ms", "frac")}
    k_m2l["in_step"] = {x: s_m2l[x] for x in ("achieved", "avg_ms", "frac")}
    dom = k_p2p if k_p2p["avg_ms"] >= k_m2l["avg_ms"] else k_m2l
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


def run_batch(args):
    """Batch workload: one step = fmm_evaluate_batch over every instance (one
    forest, each phase one pass over all instances); compared with the same
    instances evaluated one after another through the single-instance calls."""
    import torch

    import synth
    from paper_1108_5815_amd import FMM
    x, y, z, q, off, kinds, tg, w = synth.make_batch(args.workload, args.n_inst)
    if args.p is not None:
        w["p"] = args.p
    n, p, theta, ncrit = w["n"], w["p"], w["theta"], w["ncrit"]
    dev = "cuda:0"
    X, Y, Z, Q = (torch.tensor(a, dtype=torch.float32, device=dev) for a in (x, y, z, q))
    phi = torch.empty(n, dtype=torch.float32, device=dev)
    E = torch.empty((3, n), dtype=torch.float32, device=dev)
    f = FMM(0)
    prep = {}
    if args.policy == 2:
        f.tune(p, args.precision)
        prep["unit_costs_ns"] = f.costs().tolist()
    elif args.policy == 3:
        prep.update(prepare_costmodel(f, w, args.precision, args))

    def step():
        f.evaluate_batch(off, X, Y, Z, Q, ncrit, p, theta, args.policy, args.precision, out=(phi, E))

    f.build_tree_batch(off, X, Y, Z, Q, ncrit)
    f.traverse(p, theta, args.policy)
    prep["tile_config"] = f.autotune(args.precision, reps=2)
    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step()
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1e3 / args.steps
    def phases():
        f.set_timing(True)
        ph = {}
        for _ in range(3):
            step()
            for k, v in f.timings().items():
                ph[k] = ph.get(k, 0.0) + v / 3
        f.set_timing(False)
        torch.cuda.synchronize()
        return {k: round(v, 4) for k, v in ph.items()}

    sched = prep["tile_config"]["schedule"]
    ph_step = phases()
    f.set_overlap(0)
    ph_alone = phases()
    f.set_overlap(sched)
    res = {"ms_per_step": ms, "value": n / (ms * 1e-3), "phase_ms": ph_alone, "phase_ms_in_step": ph_step,
           "sizes": f.sizes(), "m2l_split": dict(zip(("batched", "general"), f.m2l_split())), "work": f.work(),
           "gemm_shape": f.gemm_shape(),
           "policy": POLICIES[args.policy], "precision": PRECISIONS[args.precision], "prep": prep}
    # the same instances one by one (single-instance calls, one context)
    g = FMM(0)
    if args.policy == 2:
        g.set_costs(*f.costs())
    elif args.policy == 3:
        g.costmodel_set_weights(f.costmodel_weights())
    views = [(int(off[k]), int(off[k + 1])) for k in range(len(off) - 1)]

    def loop():
        for b, e in views:
            g.build_tree(X[b:e], Y[b:e], Z[b:e], Q[b:e], ncrit)
            g.traverse(p, theta, args.policy)
            g.evaluate(args.precision, out=(phi[b:e], E[:, b:e]))

    loop()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    reps = max(1, min(args.steps, 3))
    for _ in range(reps):
        loop()
    torch.cuda.synchronize()
    ms_loop = (time.perf_counter() - t0) * 1e3 / reps
    res["one_by_one"] = {"ms_per_step": ms_loop, "value": n / (ms_loop * 1e-3),
                         "speedup_of_batch": ms_loop / ms}
    step()
    acc = None
    if not args.no_cpu_baseline:
        import oracle
        xs, ys, zs, qs = (np.asarray(a, dtype=np.float32).astype(np.float64) for a in (x, y, z, q))
        ph_ = phi.double().cpu().numpy()
        Eg = E.double().cpu().numpy().T
        num = den = nE = dE = 0.0
        for b, e in views:
            t = tg[(tg >= b) & (tg < e)] - b
            pd, Ed = oracle.direct(xs[b:e], ys[b:e], zs[b:e], qs[b:e], t)
            num += float(np.sum((ph_[b + t] - pd) ** 2))
            den += float(np.sum(pd ** 2))
            nE += float(np.sum((Eg[b + t] - Ed) ** 2))
            dE += float(np.sum(Ed ** 2))
        acc = {"phi_rel_l2": (num / den) ** 0.5, "E_rel_l2": (nE / dE) ** 0.5, "targets": int(tg.size),
               "reference": "FP64 direct sum of each instance (oracle)"}
    out = {
        "metric": "FMM particles/sec over a batch of independent instances",
        "value": res["value"], "unit": "particles/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": ms, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32+bf16" if args.precision == 1 else "f32", "data": "synthetic",
        "config": {"workload": args.workload, "n_inst": int(len(off) - 1), "n": n, "p": p, "theta": theta,
                   "ncrit": ncrit, "policy": res["policy"], "precision": res["precision"]},
        "accuracy": acc, "form": res, "roofline": roofline(res, p, args.precision, args.workload),
    }
    if not args.no_cpu_baseline:
        import oracle
        ns, k, t = 0, 0, 0.0
        while ns < args.cpu_sample and k < len(views):
            b, e = views[k]
            xs_, ys_, zs_, qs_ = (np.asarray(a[b:e], dtype=np.float32).astype(np.float64) for a in (x, y, z, q))
            t0 = time.perf_counter()
            oracle.fmm(xs_, ys_, zs_, qs_, p, theta, ncrit)
            t += time.perf_counter() - t0
            ns += e - b
            k += 1
        out["cpu_baseline"] = {"value": ns / t, "unit": "particles/s", "cores": oracle.num_threads(),
                               "kind": "oracle",
                               "sample": f"oracle FP64 FMM on the first {k} instances ({ns} points, {t:.1f} s)"}
    print(json.dumps(out))


def cpu_baseline(w, workload, sample, x, y, z, q, tg):
    """The oracle on the host cores: FMM particles/s on a bounded sample of the
    workload (all threads, the reported value; and one thread on 16,384
    points), and its direct sum on the workload's seeded targets."""
    import oracle
    import synth
    cores = oracle.num_threads()

    def ora_fmm(m):
        xs, ys, zs, qs, _, _ = synth.make_workload(workload, m)
        xs, ys, zs, qs = (np.asarray(a, dtype=np.float32).astype(np.float64) for a in (xs, ys, zs, qs))
        t0 = time.perf_counter()
        oracle.fmm(xs, ys, zs, qs, w["p"], w["theta"], w["ncrit"])
        return time.perf_counter() - t0

    ns = min(sample, w["n"])
    t_all = ora_fmm(ns)
    xs, ys, zs, qs = (np.asarray(a, dtype=np.float32).astype(np.float64) for a in (x, y, z, q))
    t0 = time.perf_counter()
    oracle.direct(xs, ys, zs, qs, tg)
    t_dir = time.perf_counter() - t0
    oracle.set_threads(1)
    try:
        n1 = min(16384, w["n"])
        t_one = ora_fmm(n1)
        tg1 = tg[:100]
        t0 = time.perf_counter()
        oracle.direct(xs, ys, zs, qs, tg1)
        t_dir1 = time.perf_counter() - t0
    finally:
        oracle.set_threads(cores)
    n = w["n"]
    return {"value": ns / t_all, "unit": "particles/s", "cores": cores, "kind": "oracle",
            "sample": f"oracle FP64 FMM (FMM policy) on the first {ns} points of the same generator, same p, "
                      f"theta, ncrit: {t_all:.1f} s on {cores} threads",
            "one_thread": {"value": n1 / t_one, "unit": "particles/s",
                           "sample": f"oracle FMM on the first {n1} points, 1 thread: {t_one:.1f} s"},
            "direct_sum": {"pairs_per_s": n * tg.size / t_dir, "targets": int(tg.size), "seconds": t_dir,
                           "threads": cores,
                           "one_thread_pairs_per_s": n * tg1.size / t_dir1,
                           "note": "FP64 O(N) sum per target over all N sources (the accuracy reference)"}}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="plummer4m_p10")
    ap.add_argument("--n", type=int, default=None, help="override particle count")
    ap.add_argument("--n-inst", type=int, default=None, help="batch workloads: first n instances only")
    ap.add_argument("--p", type=int, default=None, help="override the workload's expansion order")
    ap.add_argument("--policy", type=int, default=3, help="0 fmm, 1 treecode, 2 timed hybrid, 3 learned hybrid")
    ap.add_argument("--precision", type=int, default=1, help="0 fp32, 1 split-bf16 M2L")
    ap.add_argument("--no-plain", action="store_true", help="skip the plain (timed FP32) comparison")
    ap.add_argument("--no-cpu-baseline", action="store_true", help="skip the oracle legs (accuracy, CPU timing)")
    ap.add_argument("--cpu-sample", type=int, default=262144)
    ap.add_argument("--costmodel", default=None, help="cost-model file to load (default: the committed one for "
                    "this device, p, theta and precision, if any)")
    ap.add_argument("--train", action="store_true", help="train the cost model even if a saved one exists")
    ap.add_argument("--save-costmodel", default=None, help="save the trained cost model to this file")
    ap.add_argument("--no-timed-bf16", action="store_true", help="skip the timed split-BF16 comparison")
    ap.add_argument("--copy-probe-mib", type=int, default=0,
                    help="before the steps, copy this many MiB with one elementwise kernel (the reference "
                         "launch that scales hardware byte counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU; --gpus must be 1"}))
        sys.exit(2)

    import torch

    import synth
    from paper_1108_5815_amd import FMM

    if args.copy_probe_mib > 0:
        a = torch.ones(args.copy_probe_mib * 262144, dtype=torch.float32, device="cuda:0")
        b = torch.empty_like(a)
        torch.mul(a, 1.0, out=b)
        torch.cuda.synchronize()
        del a, b
    if synth.WORKLOADS[args.workload]["dist"] == "batch":
        run_batch(args)
        return
    x, y, z, q, tg, w = synth.make_workload(args.workload, args.n)
    if args.p is not None:
        w["p"] = args.p
    n, p = w["n"], w["p"]
    dev = "cuda:0"
    X, Y, Z, Q = (torch.tensor(a, dtype=torch.float32, device=dev) for a in (x, y, z, q))
    f = FMM(0)
    phi = torch.empty(n, dtype=torch.float32, device=dev)
    E = torch.empty((3, n), dtype=torch.float32, device=dev)

    main_res = run_form(f, X, Y, Z, Q, phi, E, w, args.policy, args.precision, args.steps, args.warmup, args)
    acc_main = None if args.no_cpu_baseline else accuracy(x, y, z, q, tg, phi, E)
    plain = None
    if not args.no_plain and (args.policy, args.precision) != (2, 0):
        plain = run_form(f, X, Y, Z, Q, phi, E, w, 2, 0, args.steps, args.warmup, args)
        if not args.no_cpu_baseline:
            plain["accuracy"] = accuracy(x, y, z, q, tg, phi, E)
        plain["speedup_of_value"] = main_res["value"] / plain["value"]
    timed_bf16 = None
    if not args.no_plain and not args.no_timed_bf16 and (args.policy, args.precision) == (3, 1):
        timed_bf16 = run_form(f, X, Y, Z, Q, phi, E, w, 2, 1, args.steps, args.warmup, args)
        if not args.no_cpu_baseline:
            timed_bf16["accuracy"] = accuracy(x, y, z, q, tg, phi, E)
        timed_bf16["speedup_of_value"] = main_res["value"] / timed_bf16["value"]

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
        "timed_bf16": timed_bf16,
        "roofline": roofline(main_res, p, args.precision, args.workload),
    }
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(w, args.workload, args.cpu_sample, x, y, z, q, tg)
    print(json.dumps(out))


if __name__ == "__main__":
    main()
