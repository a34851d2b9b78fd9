"""Integer parity at the full sizes of the two single-GPU workloads, and the
headline form under test.

- uniform1m_p10 (1,048,576 uniform points, FP32, p = 10, theta = 0.5,
  ncrit = 64) and plummer4m_p10 (4,194,304 Plummer points, theta = 0.4):
  Morton keys, permutation, every cell field and the three lists of the FMM
  policy bit-exact against the oracle, element by element.
- plummer4m_p10 under the learned policy (trained on the GPU by the library):
  the lists bit-exact against the oracle traversal reading the same choice
  table; then the learned + split-BF16 evaluation (the headline form) against
  the FP64 direct sum on the workload's 1,000 seeded targets.
Lists are compared as sorted 64-bit keys target * ncell + source.
"""
import numpy as np
import pytest

import oracle as ora
import synth

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _f32(a):
    return np.asarray(a, np.float32).astype(np.float64)


def _keys(t, s, ncell):
    k = np.asarray(t, np.int64) * ncell + np.asarray(s, np.int64)
    k.sort()
    return k


def _build(workload):
    from paper_1108_5815_amd import FMM
    x, y, z, q, tg, w = synth.make_workload(workload)
    x, y, z, q = (_f32(a) for a in (x, y, z, q))
    f = FMM(0)
    f.build_tree(*(torch.tensor(a, dtype=torch.float32, device="cuda:0") for a in (x, y, z, q)), w["ncrit"])
    tr = ora.Tree(x, y, z, w["ncrit"])
    return f, tr, (x, y, z, q, tg, w)


def _tree_parity(f, tr):
    lo_o, side_o = tr.bbox()
    lo_g, side_g = f.bbox()
    assert np.array_equal(lo_o, lo_g) and side_o == side_g
    kg, pg = f.keys()
    ko, po = tr.keys()
    assert np.array_equal(kg, ko)
    assert np.array_equal(pg.astype(np.int64), po)
    del kg, ko, pg, po
    cg, co = f.cells(), tr.cells()
    assert f.sizes()["cells"] == tr.ncell
    for k in ("level", "prefix", "begin", "end", "parent", "first_child", "nchild", "radius_h"):
        assert np.array_equal(cg[k].astype(np.int64), co[k].astype(np.int64)), k
    assert np.array_equal(cg["centre_h"].astype(np.int64), co["centre_h"])


def _list_parity(f, lo, ncell):
    for k in (0, 1, 2):
        tg, sg = f.list(k)
        assert tg.size == lo[k][0].size, k
        assert np.all(np.diff(tg) >= 0)        # grouped by target
        assert np.array_equal(_keys(tg, sg, ncell), _keys(*lo[k], ncell)), k


@pytest.mark.parametrize("workload", ["uniform1m_p10", "plummer4m_p10"])
def test_full_size_keys_cells_lists_fmm_policy(workload):
    f, tr, (x, y, z, q, tg, w) = _build(workload)
    _tree_parity(f, tr)
    f.traverse(w["p"], w["theta"], 0)
    tr.traverse(w["theta"], 0)
    lo = tr.lists()
    print(workload, "cells", tr.ncell, "lists", [lo[k][0].size for k in (0, 1, 2)])
    _list_parity(f, lo, tr.ncell)


def test_plummer4m_learned_lists_and_headline_accuracy():
    from paper_1108_5815_amd import PREC_SPLIT_BF16
    f, tr, (x, y, z, q, tg, w) = _build("plummer4m_p10")
    p, theta = w["p"], w["theta"]
    f.costmodel_train(p, theta, epochs=6000, seed=7, precision=PREC_SPLIT_BF16)
    f.build_tree(*(torch.tensor(a, dtype=torch.float32, device="cuda:0") for a in (x, y, z, q)), w["ncrit"])
    f.traverse(p, theta, 3)
    table = f.costmodel_table(p, theta)
    tr.traverse_table(theta, table)
    lo = tr.lists()
    print("learned lists", [lo[k][0].size for k in (0, 1, 2)])
    _list_parity(f, lo, tr.ncell)
    # the trained network's choices stay within reach of the timed ones: its
    # particle-particle and cell-particle work is at most twice the timed policy's
    learned_work = f.work()
    f.tune(p, PREC_SPLIT_BF16)
    f.traverse(p, theta, 2)
    timed_work = f.work()
    print("work learned", learned_work, "timed", timed_work)
    assert learned_work["p2p_particle_pairs"] <= 2 * timed_work["p2p_particle_pairs"]
    assert learned_work["m2p_targets"] <= 2 * timed_work["m2p_targets"] + 1000000
    f.traverse(p, theta, 3)
    phi, E = f.evaluate(PREC_SPLIT_BF16, out_dtype=torch.float64)
    torch.cuda.synchronize()
    pd, Ed = ora.direct(x, y, z, q, tg)
    ep = ora.rel_l2(phi.cpu().numpy()[tg], pd)
    eE = ora.rel_l2(E.cpu().numpy().T[tg], Ed)
    print(f"plummer4m p10 learned + split-bf16: phi rel L2 {ep:.3e}  E rel L2 {eE:.3e}")
    assert ep < 1e-5 and eE < 1e-4
