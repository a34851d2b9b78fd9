"""Targets that differ from the sources (fmm_build_tree_ts): a target tree and
a source tree in one cube, traversed from the pair of roots ("Dual tree
traversal"), against the oracle's two-tree method; and the random spherical
shell of the paper's policy experiment ("Results")."""
import numpy as np
import pytest

import oracle as ora
import synth

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _f32(a):
    return np.asarray(a, np.float32).astype(np.float64)


def _dev(a, dt=torch.float32):
    return torch.tensor(np.ascontiguousarray(a), dtype=dt, device="cuda:0")


def ts_sets(nt, ns, seed):
    """Targets uniform in a cube around and inside the unit sphere, sources on
    the sphere (the paper's shell) with charges in [-1, 1]."""
    t = np.stack(synth.uniform_cube(nt, seed), 1) * 2.4 - 1.2
    s = np.stack(synth.sphere_shell(ns, seed + 1), 1)
    q = synth.charges_uniform(ns, seed + 2)
    return _f32(t), _f32(s), _f32(q)


def gpu_ts(t, s, q, p, theta, ncrit, policy=0, costs=None, precision=0):
    from paper_1108_5815_amd import FMM
    f = FMM(0)
    f.build_tree_ts([_dev(t[:, d]) for d in range(3)], [_dev(s[:, d]) for d in range(3)], _dev(q), ncrit)
    if costs is not None:
        f.set_costs(*costs)
    f.traverse(p, theta, policy)
    phi, E = f.evaluate(precision, out_dtype=torch.float64)
    torch.cuda.synchronize()
    return f, phi.cpu().numpy(), E.cpu().numpy().T


def cell_key(c, i):
    """(is-source-tree, level, prefix) of cell i: a name independent of numbering."""
    return (int(c["begin"][i] >= c["nt"]), int(c["level"][i]), int(c["prefix"][i]))


def canon_named(lists, c):
    t, s = lists
    return sorted((cell_key(c, a), cell_key(c, b)) for a, b in zip(t, s))


@pytest.mark.parametrize("policy,costs", [(0, None), (1, None), (2, (40.0, 2.0, 1.0))],
                         ids=["fmm", "treecode", "hybrid"])
def test_ts_trees_lists_values(policy, costs):
    t, s, q = ts_sets(7000, 9000, 81)
    nt = t.shape[0]
    f, phi, E = gpu_ts(t, s, q, 10, 0.5, 32, policy, costs)
    tr = ora.Tree.targets_sources(t, s, 32)
    # keys and permutation of the two sets (targets first), cells
    kg, pg = f.keys()
    ko, po = tr.keys()
    assert np.array_equal(kg, ko) and np.array_equal(pg.astype(np.int64), po)
    cg, co = f.cells(), tr.cells()
    for k in ("level", "prefix", "begin", "end", "parent", "first_child", "nchild", "radius_h"):
        assert np.array_equal(cg[k].astype(np.int64), co[k].astype(np.int64)), k
    tr.traverse(0.5, policy, costs or (0, 0, 0))
    lo = tr.lists()
    cg["nt"] = co["nt"] = nt
    for k in (0, 1, 2):
        assert canon_named(f.list(k), cg) == canon_named(lo[k], co), k
    po_, Eo = tr.evaluate(10, q)
    assert ora.rel_l2(phi, po_) < 1e-5 and ora.rel_l2(E, Eo) < 1e-4
    pd, Ed = ora.direct_st(s, q, t)
    assert ora.rel_l2(phi, pd) < 1e-4


def test_ts_same_points_as_one_set():
    """Targets equal to the sources: the two-tree evaluation gives the
    one-tree values (self pairs skipped as coincident points)."""
    from paper_1108_5815_amd import FMM
    x, y, z = (_f32(a) for a in synth.plummer(20000, 82))
    q = _f32(synth.charges_uniform(20000, 182))
    P = np.stack([x, y, z], 1)
    _, phi2, E2 = gpu_ts(P, P, q, 8, 0.5, 32, 0, None, 1)
    f = FMM(0)
    f.build_tree(_dev(x), _dev(y), _dev(z), _dev(q), 32)
    f.traverse(8, 0.5, 0)
    phi1, E1 = f.evaluate(1, out_dtype=torch.float64)
    assert ora.rel_l2(phi2, phi1.cpu().numpy()) < 1e-6
    assert ora.rel_l2(E2, E1.cpu().numpy().T) < 1e-6


def test_ts_coincident_and_empty_sides():
    t, s, q = ts_sets(500, 800, 83)
    t[:50] = s[:50]                       # targets sitting on sources
    _, phi, E = gpu_ts(t, s, q, 8, 0.5, 16)
    pd, Ed = ora.direct_st(s, q, t)
    assert np.all(np.isfinite(phi)) and ora.rel_l2(phi, pd) < 1e-4
    _, phi0, E0 = gpu_ts(t, s[:0], q[:0], 8, 0.5, 16)
    assert np.all(phi0 == 0) and np.all(E0 == 0)
    f, phi1, _ = gpu_ts(t[:0], s, q, 8, 0.5, 16)
    assert phi1.size == 0 and f.sizes()["m2l"] == 0


def test_shell_policy_counts():
    """The paper's shell experiment ("Results": 1e5 points on a random
    spherical shell, N_crit = 20, theta = 0.5): cell pairs of each kind under
    the treecode, the FMM and the timed hybrid (unit costs from this GPU's
    kernel pre-calculation).  The paper's CPU counts: treecode cell-particle
    : particle-particle about 5 : 1, FMM cell-cell : particle-particle about
    3 : 1, hybrid particle-particle : cell-cell about 2 : 1.  Here the
    treecode shares the dual traversal (it pairs cells of both trees and only
    swaps the far-field kind), so its cell-particle count equals the FMM's
    cell-cell count; the paper's treecode walks the source tree per target
    leaf, which gives more cell-particle pairs.  The FMM ratio is the paper's
    to within a third, and the hybrid, with this GPU's unit costs, leans
    further to particle-particle sums than the CPU's 2 : 1."""
    from paper_1108_5815_amd import FMM
    x, y, z = (_f32(a) for a in synth.sphere_shell(100000, 84))
    q = _f32(synth.charges_uniform(100000, 184))
    f = FMM(0)
    f.tune(8)
    t = [_dev(a) for a in (x, y, z, q)]
    counts = {}
    for name, pol, p in (("treecode", 1, 5), ("fmm", 0, 8), ("hybrid", 2, 8)):
        f.build_tree(*t, 20)
        f.traverse(p, 0.5, pol)
        counts[name] = f.sizes()
    print("shell 1e5, ncrit 20:", counts, "unit costs", f.costs())
    tc, fm, hy = counts["treecode"], counts["fmm"], counts["hybrid"]
    assert tc["m2l"] == 0 and fm["m2p"] == 0
    # the same criterion and tree: the far pairs are shared out, the near ones identical
    assert tc["p2p"] == fm["p2p"] and tc["m2p"] == fm["m2l"]
    assert 2 * fm["p2p"] < fm["m2l"] < 4 * fm["p2p"]
    assert hy["p2p"] > 2 * hy["m2l"]
    print("ratios: treecode M2P/P2P %.2f, FMM M2L/P2P %.2f, hybrid P2P/M2L %.2f"
          % (tc["m2p"] / tc["p2p"], fm["m2l"] / fm["p2p"], hy["p2p"] / max(hy["m2l"], 1)))
