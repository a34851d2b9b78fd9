"""GPU parity of batches: many independent instances evaluated as one forest.

Every instance of a batch must get exactly what a build of that instance by
itself gets: its own bounding cube, Morton keys and permutation, cells and
interaction lists (bit-exact against the oracle run on the instance alone),
and potentials and fields equal to the single-instance GPU result and within
the parity tolerances of the oracle's FMM.  Instances are seeded synthetic
sets of uneven size (``synth.make_batch``): uniform-cube or Plummer, charges
uniform in [-1, 1].
"""
import numpy as np
import pytest

import oracle as ora
import synth

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def f32(a):
    return np.asarray(a, dtype=np.float32).astype(np.float64)


def small_batch():
    """Five instances: uniform, empty, Plummer, a single particle, a coincident block."""
    parts, kinds = [], []
    x, y, z = synth.uniform_cube(3000, 41)
    parts.append((x, y, z, synth.charges_uniform(3000, 141)))
    parts.append((np.zeros(0), np.zeros(0), np.zeros(0), np.zeros(0)))
    x, y, z = synth.plummer(5000, 42)
    parts.append((x, y, z, synth.charges_uniform(5000, 142)))
    parts.append((np.array([0.3]), np.array([0.2]), np.array([0.1]), np.array([1.0])))
    x, y, z = synth.uniform_cube(2000, 43)
    x[10:200] = x[5]; y[10:200] = y[5]; z[10:200] = z[5]
    parts.append((x + 5.0, y - 3.0, z, synth.charges_uniform(2000, 143)))
    off = np.zeros(len(parts) + 1, dtype=np.int64)
    for k, p in enumerate(parts):
        off[k + 1] = off[k] + p[0].size
    cat = [f32(np.concatenate([p[d] for p in parts])) for d in range(4)]
    return cat, off


def dev(a):
    return torch.tensor(a, dtype=torch.float32, device="cuda:0")


def local_cells(cg, b, e):
    """Cells of the instance owning sorted positions [b, e), renumbered locally."""
    sel = np.nonzero((cg["begin"] >= b) & (cg["end"] <= e) & (cg["end"] > cg["begin"]))[0]
    loc = -np.ones(cg["level"].size, np.int64)
    loc[sel] = np.arange(sel.size)
    return sel, loc


def canon(t, s):
    o = np.lexsort((s, t))
    return np.stack([t[o], s[o]], axis=1)


@pytest.mark.parametrize("policy,costs", [(0, None), (1, None), (2, (40.0, 2.0, 1.0))],
                         ids=["fmm", "treecode", "hybrid"])
def test_forest_matches_instances_bitexact(policy, costs):
    from paper_1108_5815_amd import FMM
    (x, y, z, q), off = small_batch()
    f = FMM(0)
    f.build_tree_batch(off, dev(x), dev(y), dev(z), dev(q), 32)
    if costs:
        f.set_costs(*costs)
    f.traverse(6, 0.5, policy)
    kg, pg = f.keys()
    cg = f.cells()
    lists = {k: f.list(k) for k in (0, 1, 2)}
    boxes = f.bboxes(len(off) - 1)
    total_cells = 0
    for k in range(len(off) - 1):
        b, e = int(off[k]), int(off[k + 1])
        if e == b:
            assert np.array_equal(boxes[k], [0, 0, 0, 1])
            continue
        tr = ora.Tree(x[b:e], y[b:e], z[b:e], 32)
        lo, side = tr.bbox()
        assert np.array_equal(boxes[k, :3], lo) and boxes[k, 3] == side
        ko, po = tr.keys()
        assert np.array_equal(kg[b:e], ko)
        assert np.array_equal(pg[b:e].astype(np.int64) - b, po)
        sel, loc = local_cells(cg, b, e)
        co = tr.cells()
        assert sel.size == tr.ncell
        total_cells += sel.size
        for key in ("level", "prefix", "nchild", "radius_h"):
            assert np.array_equal(cg[key][sel].astype(np.int64), co[key].astype(np.int64)), key
        assert np.array_equal(cg["begin"][sel].astype(np.int64) - b, co["begin"])
        assert np.array_equal(cg["end"][sel].astype(np.int64) - b, co["end"])
        par = cg["parent"][sel]
        assert np.array_equal(np.where(par >= 0, loc[np.maximum(par, 0)], -1), co["parent"])
        assert np.array_equal(cg["centre_h"][sel].astype(np.int64), co["centre_h"])
        tr.traverse(0.5, policy, costs or (0, 0, 0))
        lo_ = tr.lists()
        for kind in (0, 1, 2):
            tg, sg = lists[kind]
            m = (loc[tg] >= 0)
            assert np.all(loc[sg[m]] >= 0)          # no pair crosses instances
            assert np.array_equal(canon(loc[tg[m]], loc[sg[m]]), canon(*lo_[kind])), (k, kind)
    assert total_cells == f.sizes()["cells"]


def test_forest_values_equal_single_instance_runs():
    """Same lists, same kernels, same summation order: identical results."""
    from paper_1108_5815_amd import FMM
    (x, y, z, q), off = small_batch()
    f = FMM(0)
    phi, E = f.evaluate_batch(off, dev(x), dev(y), dev(z), dev(q), 32, 8, 0.5, out_dtype=torch.float64)
    phi, E = phi.cpu().numpy(), E.cpu().numpy().T
    for k in range(len(off) - 1):
        b, e = int(off[k]), int(off[k + 1])
        if e == b:
            continue
        g = FMM(0)
        g.build_tree(dev(x[b:e]), dev(y[b:e]), dev(z[b:e]), dev(q[b:e]), 32)
        g.traverse(8, 0.5, 0)
        p1, E1 = g.evaluate(out_dtype=torch.float64)
        assert np.array_equal(phi[b:e], p1.cpu().numpy()), k
        assert np.array_equal(E[b:e], E1.cpu().numpy().T), k
        if e - b > 1:
            po, Eo, _ = ora.fmm(x[b:e], y[b:e], z[b:e], q[b:e], 8, 0.5, 32)
            assert ora.rel_l2(phi[b:e], po) < 1e-5 and ora.rel_l2(E[b:e], Eo) < 1e-4
        else:
            assert phi[b] == 0.0 and np.all(E[b] == 0.0)


def test_batch_split_bf16_and_hybrid():
    from paper_1108_5815_amd import FMM
    x, y, z, q, off, kinds, tg, w = synth.make_batch("batch256_p8", n_inst=12)
    x, y, z, q = (f32(a) for a in (x, y, z, q))
    f = FMM(0)
    f.set_costs(0.5, 0.3, 0.001)
    phi, E = f.evaluate_batch(off, dev(x), dev(y), dev(z), dev(q), 64, 8, 0.5, policy=2, precision=1,
                              out_dtype=torch.float64)
    phi, E = phi.cpu().numpy(), E.cpu().numpy().T
    for k in (0, 3, 7):
        b, e = int(off[k]), int(off[k + 1])
        po, Eo, _ = ora.fmm(x[b:e], y[b:e], z[b:e], q[b:e], 8, 0.5, 64, 2, (0.5, 0.3, 0.001))
        assert ora.rel_l2(phi[b:e], po) < 1e-5 and ora.rel_l2(E[b:e], Eo) < 1e-4


def test_batch_errors():
    from paper_1108_5815_amd import FMM, FMMError
    f = FMM(0)
    x = dev(np.linspace(0, 1, 100))
    for off in ([0, 50, 40, 100], [1, 50, 100], [0, 50, 99]):
        with pytest.raises((FMMError, ValueError)):
            f.build_tree_batch(off, x, x, x, x, 16)
    bad = x.clone()
    bad[70] = float("nan")
    with pytest.raises(FMMError) as e:
        f.build_tree_batch([0, 50, 100], bad, x, x, x, 16)
    assert e.value.status == 1
    f.build_tree_batch([0, 0, 0], x[:0], x[:0], x[:0], x[:0], 16)   # all instances empty
    f.traverse(6, 0.5, 0)
    phi, E = f.evaluate()
    assert phi.numel() == 0


def test_full_batch256_p8_sampled():
    """256 instances (9,416,653 particles), p = 8, theta = 0.5, ncrit = 64:
    8 seeded targets per instance against the FP64 direct sum of that instance,
    and the batch equal to single runs on three instances."""
    from paper_1108_5815_amd import FMM
    x, y, z, q, off, kinds, tg, w = synth.make_batch("batch256_p8")
    x, y, z, q = (f32(a) for a in (x, y, z, q))
    f = FMM(0)
    phi, E = f.evaluate_batch(off, dev(x), dev(y), dev(z), dev(q), 64, 8, 0.5)
    phi, E = phi.double().cpu().numpy(), E.double().cpu().numpy().T
    num = den = numE = denE = 0.0
    for k in range(len(off) - 1):
        b, e = int(off[k]), int(off[k + 1])
        t = tg[(tg >= b) & (tg < e)] - b
        pd, Ed = ora.direct(x[b:e], y[b:e], z[b:e], q[b:e], t)
        num += np.sum((phi[b + t] - pd) ** 2)
        den += np.sum(pd ** 2)
        numE += np.sum((E[b + t] - Ed) ** 2)
        denE += np.sum(Ed ** 2)
    ep, eE = np.sqrt(num / den), np.sqrt(numE / denE)
    print(f"batch256 p8: phi rel L2 {ep:.3e}  E rel L2 {eE:.3e}")
    assert ep < 1e-4 and eE < 1e-3
    for k in (0, 100, 255):
        b, e = int(off[k]), int(off[k + 1])
        g = FMM(0)
        g.build_tree(dev(x[b:e]), dev(y[b:e]), dev(z[b:e]), dev(q[b:e]), 64)
        g.traverse(8, 0.5, 0)
        p1, _ = g.evaluate()
        assert np.array_equal(phi[b:e], p1.double().cpu().numpy()), k


def test_autotune_choices_and_accuracy():
    """The autotuner picks a tile shape per leaf-size class and a schedule; the
    tuned evaluation stays within the parity bar of the oracle."""
    from paper_1108_5815_amd import FMM
    x, y, z, q, off, kinds, tg, w = synth.make_batch("batch256_p8", n_inst=10)
    x, y, z, q = (f32(a) for a in (x, y, z, q))
    f = FMM(0)
    f.build_tree_batch(off, dev(x), dev(y), dev(z), dev(q), 64)
    f.traverse(8, 0.5, 0)
    cfg = f.autotune(0, reps=2)
    assert all(t in (1, 2, 4, -1, -2, -4) for t in cfg["p2p_targets_per_lane"])
    phi, E = f.evaluate(out_dtype=torch.float64)
    phi, E = phi.cpu().numpy(), E.cpu().numpy().T
    for k in (1, 4):
        b, e = int(off[k]), int(off[k + 1])
        po, Eo, _ = ora.fmm(x[b:e], y[b:e], z[b:e], q[b:e], 8, 0.5, 64)
        assert ora.rel_l2(phi[b:e], po) < 1e-5 and ora.rel_l2(E[b:e], Eo) < 1e-4
    for tpl in ([-1] * 4, [-4] * 4, [1, 1, 1, 1], [2, 2, 2, 2], [4, 4, 4, 4]):
        f.set_tile_config(tpl)
        p2, _ = f.evaluate(out_dtype=torch.float64)
        assert ora.rel_l2(p2.cpu().numpy(), phi) < 1e-6
