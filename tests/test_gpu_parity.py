"""GPU parity: the HIP library (through its C-ABI) against the FP64 oracle.

Integer results (Morton keys, permutation, cells, interaction lists) must be
bit-exact.  Potentials and fields must match the oracle's FMM on the same
lists within 1e-5 (potential) and 1e-4 (field) relative L2 at p = 10; at the
full 1,048,576-particle size the check is against the FP64 direct sum on
1,000 seeded targets.  Inputs are seeded synthetic sets (``synth``).
"""
import numpy as np
import pytest

import oracle as ora
import synth

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _fmm():
    from paper_1108_5815_amd import FMM
    return FMM(0)


def as_input(a, dtype):
    """The exact values both sides see: rounded to the GPU input dtype, then FP64."""
    return np.asarray(a, dtype=np.float32 if dtype == torch.float32 else np.float64).astype(np.float64)


def gpu_run(x, y, z, q, p, theta, ncrit, policy=0, costs=None, dtype=torch.float32, out_dtype=torch.float64):
    f = _fmm()
    t = [torch.tensor(a, dtype=dtype, device="cuda:0") for a in (x, y, z, q)]
    f.build_tree(*t, ncrit)
    if costs is not None:
        f.set_costs(*costs)
    f.traverse(p, theta, policy)
    phi, E = f.evaluate(out_dtype=out_dtype)
    torch.cuda.synchronize()
    return f, phi.double().cpu().numpy(), E.double().cpu().numpy().T


def canon(t, s):
    o = np.lexsort((s, t))
    return np.stack([t[o], s[o]], axis=1)


def cases():
    out = []
    x, y, z = synth.uniform_cube(16384, 1)
    out.append(("uniform16k_f64", x, y, z, synth.charges_uniform(16384, 101), torch.float64, 64))
    x, y, z = synth.uniform_cube(20001, 2)
    out.append(("uniform20001_f32", x, y, z, synth.charges_uniform(20001, 102), torch.float32, 32))
    x, y, z = synth.plummer(30000, 3)
    out.append(("plummer30k_f32", x, y, z, synth.charges_equal(30000), torch.float32, 16))
    x, y, z = synth.uniform_cube(5000, 4)
    x[100:400] = x[7]; y[100:400] = y[7]; z[100:400] = z[7]   # coincident block deeper than ncrit
    out.append(("dupes5000_f32", x, y, z, synth.charges_uniform(5000, 104), torch.float32, 24))
    return out


CASES = cases()


@pytest.mark.parametrize("case", CASES, ids=[c[0] for c in CASES])
def test_keys_cells_bitexact(case):
    name, x, y, z, q, dt, ncrit = case
    xs, ys, zs = (as_input(a, dt) for a in (x, y, z))
    f = _fmm()
    f.build_tree(*(torch.tensor(a, dtype=dt, device="cuda:0") for a in (x, y, z, q)), ncrit)
    tr = ora.Tree(xs, ys, zs, ncrit)
    lo_o, side_o = tr.bbox()
    lo_g, side_g = f.bbox()
    assert np.array_equal(lo_o, lo_g) and side_o == side_g
    kg, pg = f.keys()
    ko, po = tr.keys()
    assert np.array_equal(kg, ko)
    assert np.array_equal(pg.astype(np.int64), po)
    cg, co = f.cells(), tr.cells()
    assert f.sizes()["cells"] == tr.ncell
    for k in ("level", "prefix", "begin", "end", "parent", "first_child", "nchild", "radius_h"):
        assert np.array_equal(cg[k].astype(np.int64), co[k].astype(np.int64)), k
    assert np.array_equal(cg["centre_h"].astype(np.int64), co["centre_h"])


@pytest.mark.parametrize("policy,costs", [(0, None), (1, None), (2, (40.0, 2.0, 1.0)), (2, (1e6, 1e6, 1.0))],
                         ids=["fmm", "treecode", "hybrid", "hybrid_p2p"])
@pytest.mark.parametrize("theta", [0.5, 0.4])
@pytest.mark.parametrize("case", CASES[1:3], ids=[c[0] for c in CASES[1:3]])
def test_lists_bitexact(case, theta, policy, costs):
    name, x, y, z, q, dt, ncrit = case
    xs, ys, zs = (as_input(a, dt) for a in (x, y, z))
    f = _fmm()
    f.build_tree(*(torch.tensor(a, dtype=dt, device="cuda:0") for a in (x, y, z, q)), ncrit)
    if costs is not None:
        f.set_costs(*costs)
    f.traverse(6, theta, policy)
    tr = ora.Tree(xs, ys, zs, ncrit)
    tr.traverse(theta, policy, costs or (0, 0, 0))
    lo = tr.lists()
    for k in (0, 1, 2):
        tg, sg = f.list(k)
        assert np.all(np.diff(tg) >= 0)      # grouped by target
        assert np.array_equal(canon(tg, sg), canon(*lo[k])), k


def test_values_uniform16k_p6_fp64_inputs():
    """16,384 uniform points, p = 6, theta = 0.5, ncrit = 64, FP64 inputs: against
    the oracle's FMM on the same lists and against the full direct sum."""
    x, y, z, q, tg, w = synth.make_workload("uniform16k_p6")
    _, phi, E = gpu_run(x, y, z, q, 6, 0.5, 64, dtype=torch.float64)
    po, Eo, _ = ora.fmm(x, y, z, q, 6, 0.5, 64)
    assert ora.rel_l2(phi, po) < 1e-5 and ora.rel_l2(E, Eo) < 1e-4
    pd, Ed = ora.direct(x, y, z, q)
    # the method's own truncation error at p = 6 (oracle 1.1e-4 / 1.4e-4)
    assert ora.rel_l2(phi, pd) < 2e-4 and ora.rel_l2(E, Ed) < 3e-4


@pytest.mark.parametrize("policy,costs", [(0, None), (1, None), (2, (40.0, 2.0, 1.0))],
                         ids=["fmm", "treecode", "hybrid"])
def test_values_p10_uniform(policy, costs):
    n = 24000
    x, y, z = (as_input(a, torch.float32) for a in synth.uniform_cube(n, 12))
    q = as_input(synth.charges_uniform(n, 112), torch.float32)
    _, phi, E = gpu_run(x, y, z, q, 10, 0.5, 48, policy, costs)
    po, Eo, _ = ora.fmm(x, y, z, q, 10, 0.5, 48, policy, costs or (0, 0, 0))
    assert ora.rel_l2(phi, po) < 1e-5 and ora.rel_l2(E, Eo) < 1e-4


@pytest.mark.parametrize("theta", [0.5, 0.4])
def test_values_p10_plummer_adaptive(theta):
    """Adaptive tree with mixed-level pairs (general M2L path) and equal masses."""
    n = 6000
    x, y, z = (as_input(a, torch.float32) for a in synth.plummer(n, 13))
    q = as_input(synth.charges_equal(n), torch.float32)
    _, phi, E = gpu_run(x, y, z, q, 10, theta, 16)
    po, Eo, _ = ora.fmm(x, y, z, q, 10, theta, 16)
    assert ora.rel_l2(phi, po) < 1e-5 and ora.rel_l2(E, Eo) < 1e-4


@pytest.mark.parametrize("p", [13, 16])
def test_values_high_order(p):
    """Orders above the split-BF16 range: p = 13 runs the FP32 GEMM at storage
    width 256; p = 16 (storage 320, no matrix-core tiling) sends every M2L
    pair through the per-pair kernel."""
    n = 8000
    x, y, z = (as_input(a, torch.float32) for a in synth.plummer(n, 17))
    q = as_input(synth.charges_uniform(n, 117), torch.float32)
    f, phi, E = gpu_run(x, y, z, q, p, 0.5, 32)
    batched, general = f.m2l_split()
    if p == 16:
        assert batched == 0 and general > 0
    else:
        assert batched > 0
    po, Eo, _ = ora.fmm(x, y, z, q, p, 0.5, 32)
    assert ora.rel_l2(phi, po) < 1e-5 and ora.rel_l2(E, Eo) < 1e-4


def deep_pair_set(seed=71, n=3000, ncl=3000, delta=1e-3, side=2e-5):
    """A uniform set in [0, 1]^3 (corners included, so the cube is exact) with
    the cell [0, 1/4)^3 thinned to a leaf, and a tight cluster just beyond the
    acceptance distance of that leaf at theta = 0.5: the leaf meets the
    cluster's cells only after about ten more splits of the cluster side, so
    the M2L list holds pairs whose levels differ by more than 8."""
    x, y, z = synth.uniform_cube(n, seed)
    u = synth.uniform_cube(ncl, seed + 1)
    gx = 0.375 + 0.25 * delta + side * (u[0] - 0.5)
    gy = 0.125 + side * (u[1] - 0.5)
    gz = 0.125 + side * (u[2] - 0.5)
    keep = ~((x < 0.25) & (y < 0.25) & (z < 0.25)) | (np.arange(n) % 8 == 0)
    X = np.concatenate([x[keep], [0.0, 1.0], gx])
    Y = np.concatenate([y[keep], [0.0, 1.0], gy])
    Z = np.concatenate([z[keep], [0.0, 1.0], gz])
    return X, Y, Z


def test_m2l_pairs_beyond_the_class_key():
    """Cell-cell pairs whose level difference exceeds 8 do not fit the class
    key of the batched mixed-level path and take the per-pair kernel: lists
    bit-exact and values against the oracle's FMM on the same lists."""
    x, y, z = (as_input(a, torch.float32) for a in deep_pair_set())
    n = x.size
    q = as_input(synth.charges_uniform(n, 171), torch.float32)
    f, phi, E = gpu_run(x, y, z, q, 10, 0.5, 64)
    po, Eo, tr = ora.fmm(x, y, z, q, 10, 0.5, 64)
    c = tr.cells()
    a, b = tr.lists()[0]
    d = np.abs(c["level"][a] - c["level"][b])
    assert (d > 8).sum() > 50
    tg, sg = f.list(0)
    assert np.array_equal(canon(tg, sg), canon(a, b))
    assert ora.rel_l2(phi, po) < 1e-5 and ora.rel_l2(E, Eo) < 1e-4


def to_real_scaled(C, p, r, sign):
    """oracle complex coefficients -> library real layout, scaled by r^(sign*n + (sign>0))"""
    K = (p + 1) ** 2
    out = np.zeros((C.shape[0], K))
    for n in range(p + 1):
        sc = r ** (-n) if sign < 0 else r ** (n + 1)
        out[:, n * n] = C[:, ora.cidx(n, 0)].real * sc
        for m in range(1, n + 1):
            out[:, n * n + 2 * m - 1] = C[:, ora.cidx(n, m)].real * sc
            out[:, n * n + 2 * m] = C[:, ora.cidx(n, m)].imag * sc
    return out


def test_expansions_match_oracle():
    n = 8000
    x, y, z = (as_input(a, torch.float32) for a in synth.plummer(n, 14))
    q = as_input(synth.charges_uniform(n, 114), torch.float32)
    f, _, _ = gpu_run(x, y, z, q, 8, 0.5, 20)
    Mg, Lg = f.expansions()
    _, _, tr = ora.fmm(x, y, z, q, 8, 0.5, 20)
    Mo, Lo = tr.expansions()
    r = tr.cells()["radius"]
    Mref = to_real_scaled(Mo, 8, r, -1)
    Lref = to_real_scaled(Lo, 8, r, +1)
    assert np.abs(Mg - Mref).max() <= 1e-5 * np.abs(Mref).max()
    assert np.abs(Lg - Lref).max() <= 1e-5 * np.abs(Lref).max()


def test_deterministic_repeat():
    x, y, z = synth.plummer(20000, 15)
    q = synth.charges_uniform(20000, 115)
    _, a, Ea = gpu_run(x, y, z, q, 8, 0.4, 32)
    _, b, Eb = gpu_run(x, y, z, q, 8, 0.4, 32)
    assert np.array_equal(a, b) and np.array_equal(Ea, Eb)


@pytest.mark.parametrize("n", [1, 2, 17, 64, 65, 1000, 4097])
def test_small_and_ragged_sizes(n):
    x, y, z = (as_input(a, torch.float32) for a in synth.uniform_cube(n, 16))
    q = as_input(synth.charges_uniform(n, 116), torch.float32)
    _, phi, E = gpu_run(x, y, z, q, 10, 0.5, 64)
    pd, Ed = ora.direct(x, y, z, q)
    if n == 1:
        assert phi[0] == 0.0 and np.all(E == 0.0)
        return
    po, Eo, _ = ora.fmm(x, y, z, q, 10, 0.5, 64)
    assert ora.rel_l2(phi, po) < 1e-5 and ora.rel_l2(E, Eo) < 1e-4


def test_all_points_coincident():
    n = 300
    x = np.full(n, 0.5)
    q = as_input(synth.charges_uniform(n, 117), torch.float32)
    _, phi, E = gpu_run(x, x, x, q, 6, 0.5, 16)
    assert np.all(phi == 0.0) and np.all(E == 0.0)


def test_empty_input_is_noop():
    from paper_1108_5815_amd import FMM
    f = FMM(0)
    e = torch.empty(0, device="cuda:0")
    f.build_tree(e, e, e, e, 16)
    f.traverse(6, 0.5, 0)
    phi, E = f.evaluate()
    assert phi.numel() == 0 and f.sizes()["cells"] == 0


def test_error_paths():
    from paper_1108_5815_amd import FMM, FMMError
    f = FMM(0)
    x = torch.rand(100, device="cuda:0")
    with pytest.raises(FMMError) as e:
        f.traverse(6, 0.5, 0)
    assert e.value.status == 4
    with pytest.raises(FMMError) as e:
        f.build_tree(x, x, x, x, 0)
    assert e.value.status == 1
    bad = x.clone()
    bad[5] = float("nan")
    with pytest.raises(FMMError) as e:
        f.build_tree(bad, x, x, x, 16)
    assert e.value.status == 1
    f.build_tree(x, x, x, x, 16)
    for p, th in ((17, 0.5), (-1, 0.5), (6, 0.0), (6, 1.0)):
        with pytest.raises(FMMError) as e:
            f.traverse(p, th, 0)
        assert e.value.status == 1
    with pytest.raises(FMMError) as e:
        f.traverse(6, 0.5, 2)        # timed hybrid without unit costs
    assert e.value.status == 4
    f.traverse(6, 0.5, 0)            # the context is still usable
    phi, E = f.evaluate()
    assert torch.isfinite(phi).all()


def test_full_size_uniform_1m_p10_sampled():
    """1,048,576 uniform points, FP32, p = 10, theta = 0.5, ncrit = 64 (the bench
    configuration): 1,000 seeded targets against the FP64 direct sum."""
    x, y, z, q, tg, w = synth.make_workload("uniform1m_p10")
    xs, ys, zs, qs = (as_input(a, torch.float32) for a in (x, y, z, q))
    f, phi, E = gpu_run(xs, ys, zs, qs, 10, 0.5, 64)
    pd, Ed = ora.direct(xs, ys, zs, qs, tg)
    ep, eE = ora.rel_l2(phi[tg], pd), ora.rel_l2(E[tg], Ed)
    print(f"uniform1m p10: phi rel L2 {ep:.3e}  E rel L2 {eE:.3e}")
    assert ep < 1e-5 and eE < 1e-4


def test_schedules_are_identical():
    """P2P in order, or on the second stream from the start or after the upward pass: same bits."""
    from paper_1108_5815_amd import FMM
    x, y, z = synth.plummer(30000, 17)
    q = synth.charges_uniform(30000, 117)
    t = [torch.tensor(a, dtype=torch.float32, device="cuda:0") for a in (x, y, z, q)]
    out = []
    for sched in (0, 1, 2):
        f = FMM(0)
        f.set_overlap(sched)
        f.build_tree(*t, 32)
        f.traverse(8, 0.5, 0)
        phi, E = f.evaluate()
        torch.cuda.synchronize()
        out.append((phi.cpu().numpy(), E.cpu().numpy()))
    for k in (1, 2):
        assert np.array_equal(out[0][0], out[k][0]) and np.array_equal(out[0][1], out[k][1])


def test_large_sort_stable_permutation():
    """34,000,001 points (the radix sort's longest tiles, a ragged last tile) with
    a block of 40,000 coincident points spanning several tiles: the sorted keys
    are the oracle's keys of the permuted points, non-decreasing, the
    permutation is one, and equal keys keep their input order."""
    n = 34_000_001
    x, y, z = synth.uniform_cube(n, 31)
    x[100_000:140_000] = x[7]; y[100_000:140_000] = y[7]; z[100_000:140_000] = z[7]
    q = np.ones(n)
    xs, ys, zs = (as_input(a, torch.float32) for a in (x, y, z))
    f = _fmm()
    f.build_tree(*(torch.tensor(a, dtype=torch.float32, device="cuda:0") for a in (x, y, z, q)), 64)
    torch.cuda.synchronize()
    lo, side = ora.bbox(xs, ys, zs)
    ko = ora.morton(xs, ys, zs, lo, side)
    del xs, ys, zs
    kg, pg = f.keys()
    assert np.array_equal(np.bincount(pg, minlength=n), np.ones(n, dtype=np.int64))
    assert np.array_equal(kg, ko[pg])
    assert np.all(kg[1:] >= kg[:-1])
    tie = kg[1:] == kg[:-1]
    assert tie.sum() >= 39_999
    assert np.all(pg[1:][tie] > pg[:-1][tie])
