"""Named synthetic workloads (sizes, distributions and method parameters).

Each entry gives the particle distribution, its size, the charge law, the
expansion order p, the acceptance parameter theta, the leaf capacity ncrit,
the arithmetic precision and how many seeded direct-sum targets the accuracy
check uses.  Seeds: positions use ``seed``, charges ``100 + seed``, target
samples ``200 + seed``.
"""
from __future__ import annotations

import numpy as np

WORKLOADS = {
    # small FP64 case: 16,384 uniform points, checked against the full direct sum
    "uniform16k_p6": dict(dist="cube", n=16384, charges="uniform", p=6, theta=0.5,
                          ncrit=64, dtype="f64", n_targets=16384, seed=1),
    # 1,048,576 uniform points, FP32 particles, p=10
    "uniform1m_p10": dict(dist="cube", n=1048576, charges="uniform", p=10, theta=0.5,
                          ncrit=64, dtype="f32", n_targets=1000, seed=2),
    # 4,194,304 Plummer points (a=1, r<=20), equal masses, theta=0.4, p=10
    "plummer4m_p10": dict(dist="plummer", n=4194304, charges="equal", p=10, theta=0.4,
                          ncrit=64, dtype="f32", n_targets=1000, seed=3),
    # 16,777,216 Plummer points, p=12, theta=0.4
    "plummer16m_p12": dict(dist="plummer", n=16777216, charges="equal", p=12, theta=0.4,
                           ncrit=64, dtype="f32", n_targets=2000, seed=5),
    # 256 independent instances, sizes log-uniform in [1024, 262144], each
    # uniform or Plummer (50/50), charges uniform in [-1, 1], p=8, theta=0.5
    "batch256_p8": dict(dist="batch", n_inst=256, charges="uniform", p=8, theta=0.5,
                        ncrit=64, dtype="f32", n_targets=8, seed=4),
}


def make_workload(name: str, n: int | None = None):
    """Return (x, y, z, q, targets, params) in float64 for a named workload.

    ``n`` overrides the size (same distribution and seeds) for scaled-down runs.
    """
    from . import (charges_equal, charges_uniform, plummer, target_sample,
                   uniform_cube)
    w = dict(WORKLOADS[name])
    if n is not None:
        w["n"] = int(n)
    n = w["n"]
    seed = w["seed"]
    if w["dist"] == "cube":
        x, y, z = uniform_cube(n, seed)
    elif w["dist"] == "plummer":
        x, y, z = plummer(n, seed)
    else:
        raise ValueError(w["dist"])
    q = charges_uniform(n, 100 + seed) if w["charges"] == "uniform" else charges_equal(n)
    nt = min(w["n_targets"], n)
    tg = np.arange(n, dtype=np.int64) if nt == n else target_sample(n, nt, 200 + seed)
    return x, y, z, q, tg, w


def make_batch(name: str, n_inst: int | None = None):
    """Return (x, y, z, q, offsets, kinds, targets, params) for a batch workload.

    Instance k has batch_sizes(...)[0][k] particles, uniform in the unit cube
    (kind 0) or Plummer (kind 1); positions use seed 10000 + 100 * seed + k,
    charges (uniform in [-1, 1)) 20000 + 100 * seed + k.  ``targets`` holds
    n_targets seeded indices per instance (global indices, for direct-sum
    checks).  ``n_inst`` takes the first n_inst instances of the same draw.
    """
    from . import batch_sizes, charges_uniform, plummer, target_sample, uniform_cube
    w = dict(WORKLOADS[name])
    if w["dist"] != "batch":
        raise ValueError(name)
    sizes, kinds = batch_sizes(w["n_inst"], w["seed"])
    if n_inst is not None:
        sizes, kinds = sizes[:n_inst], kinds[:n_inst]
        w["n_inst"] = int(n_inst)
    xs, ys, zs, qs, tgs = [], [], [], [], []
    offsets = np.zeros(sizes.size + 1, dtype=np.int64)
    for k, (nk, kind) in enumerate(zip(sizes.tolist(), kinds.tolist())):
        ps = 10000 + 100 * w["seed"] + k
        x, y, z = uniform_cube(nk, ps) if kind == 0 else plummer(nk, ps)
        xs.append(x)
        ys.append(y)
        zs.append(z)
        qs.append(charges_uniform(nk, 20000 + 100 * w["seed"] + k))
        tgs.append(offsets[k] + target_sample(nk, w["n_targets"], 30000 + 100 * w["seed"] + k))
        offsets[k + 1] = offsets[k] + nk
    w["n"] = int(offsets[-1])
    cat = np.concatenate
    return cat(xs), cat(ys), cat(zs), cat(qs), offsets, kinds, cat(tgs), w
