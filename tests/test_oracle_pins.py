"""Pins of the FP64 oracle to facts outside itself.

Each test checks the oracle against something the paper or mathematics fixes:
brute force on tiny inputs, library routines, closed forms, exact identities,
error bounds and invariants.  A dropped term, a wrong sign or index or a
transposed operand anywhere in the oracle breaks at least one of them.
"""
import json
import math
import os

import numpy as np
import pytest
from scipy.special import eval_legendre, lpmv

import synth

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def spread3(v: int) -> int:
    """21-bit value spread to every third bit by the classic magic-number masks."""
    v &= 0x1FFFFF
    v = (v | (v << 32)) & 0x1F00000000FFFF
    v = (v | (v << 16)) & 0x1F0000FF0000FF
    v = (v | (v << 8)) & 0x100F00F00F00F00F
    v = (v | (v << 4)) & 0x10C30C30C30C30C3
    v = (v | (v << 2)) & 0x1249249249249249
    return v


def sph(v):
    r = np.linalg.norm(v)
    return r, math.acos(v[2] / r), math.atan2(v[1], v[0])


# ---------------------------------------------------------------- keys / sort / tree
def test_interleave_matches_magic_spread(ora):
    rng = np.random.default_rng(5)
    for _ in range(200):
        qx, qy, qz = (int(t) for t in rng.integers(0, 1 << 21, 3))
        assert ora.interleave(qx, qy, qz) == spread3(qx) | (spread3(qy) << 1) | (spread3(qz) << 2)
    top = (1 << 21) - 1
    assert ora.interleave(top, top, top) == (1 << 63) - 1
    assert ora.interleave(1, 0, 0) == 1 and ora.interleave(0, 1, 0) == 2 and ora.interleave(0, 0, 1) == 4


def test_quantisation_of_grid_points(ora):
    # points at i/7 of the unit cube: bbox lo=0, side=1; q = floor(i/7 * 2^21), clamped
    g = np.arange(8) / 7.0
    X, Y, Z = np.meshgrid(g, g, g, indexing="ij")
    x, y, z = X.ravel(), Y.ravel(), Z.ravel()
    lo, side = ora.bbox(x, y, z)
    assert np.all(lo == 0.0) and side == 1.0
    keys = ora.morton(x, y, z, lo, side)
    for a in range(0, x.size, 37):
        qs = [min((1 << 21) - 1, math.floor(c * 2097152.0)) for c in (x[a], y[a], z[a])]
        assert int(keys[a]) == spread3(qs[0]) | (spread3(qs[1]) << 1) | (spread3(qs[2]) << 2)


def test_degenerate_bbox(ora):
    x = np.full(5, 0.25)
    lo, side = ora.bbox(x, x, x)
    assert side == 1.0 and np.all(lo == 0.25)
    assert np.all(ora.morton(x, x, x, lo, side) == 0)


def test_sort_is_stable_argsort(ora):
    x, y, z = synth.uniform_cube(3000, 11)
    # duplicate some points so equal keys occur
    x[1000:1100] = x[0]; y[1000:1100] = y[0]; z[1000:1100] = z[0]
    t = ora.Tree(x, y, z, 16)
    k, perm = t.keys()
    lo, side = ora.bbox(x, y, z)
    raw = ora.morton(x, y, z, lo, side)
    ref = np.argsort(raw, kind="stable")
    assert np.array_equal(perm, ref)
    assert np.array_equal(k, raw[ref])
    assert np.array_equal(np.sort(perm), np.arange(3000))


@pytest.mark.parametrize("dist,n,ncrit", [("cube", 4000, 16), ("plummer", 6000, 10), ("cube", 50, 64)])
def test_tree_invariants(ora, dist, n, ncrit):
    if dist == "cube":
        x, y, z = synth.uniform_cube(n, 3)
    else:
        x, y, z = synth.plummer(n, 3)
    t = ora.Tree(x, y, z, ncrit)
    c = t.cells()
    keys, _ = t.keys()
    nc = t.ncell
    assert c["begin"][0] == 0 and c["end"][0] == n and c["parent"][0] == -1
    # breadth-first: level non-decreasing, keys increasing within a level
    assert np.all(np.diff(c["level"]) >= 0)
    for L in np.unique(c["level"]):
        sel = np.nonzero(c["level"] == L)[0]
        assert np.all(np.diff(c["begin"][sel]) > 0)
    for i in range(nc):
        cnt = c["end"][i] - c["begin"][i]
        assert cnt > 0
        L = int(c["level"][i])
        # every particle lies in its cell: key prefix equals the cell prefix
        sh = np.uint64(3 * (21 - L))
        pre = keys[c["begin"][i]:c["end"][i]] >> sh
        assert np.all(pre == c["prefix"][i])
        if c["nchild"][i] == 0:
            assert cnt <= ncrit or L == 21
        else:
            assert cnt > ncrit
            ch = np.arange(c["first_child"][i], c["first_child"][i] + c["nchild"][i])
            assert np.all(c["parent"][ch] == i)
            assert c["begin"][ch[0]] == c["begin"][i] and c["end"][ch[-1]] == c["end"][i]
            assert np.all(c["end"][ch[:-1]] == c["begin"][ch[1:]])
            assert np.all(c["level"][ch] == L + 1)
        # integer geometry: radius = half side, centre = (2*anchor+1)*radius
        assert c["radius_h"][i] == 1 << (21 - L)
        assert np.all(c["centre_h"][i] % (2 * c["radius_h"][i]) == c["radius_h"][i])


def test_coincident_points_stop_at_level_21(ora):
    x = np.concatenate([np.full(40, 0.5), synth.uniform(1, 0, 10)])
    y = np.concatenate([np.full(40, 0.5), synth.uniform(1, 1, 10)])
    z = np.concatenate([np.full(40, 0.5), synth.uniform(1, 2, 10)])
    t = ora.Tree(x, y, z, 8)
    c = t.cells()
    big = np.nonzero((c["end"] - c["begin"] >= 40) & (c["nchild"] == 0))[0]
    assert big.size == 1 and c["level"][big[0]] == 21


# ---------------------------------------------------------------- traversal
def coverage(t, lists, n):
    """count[i, j] = number of emitted interactions covering target i and source j."""
    c = t.cells()
    cnt = np.zeros((n, n), dtype=np.int64)
    for k in (0, 1, 2):
        tt, ss = lists[k]
        for a, b in zip(tt, ss):
            cnt[c["begin"][a]:c["end"][a], c["begin"][b]:c["end"][b]] += 1
    return cnt


@pytest.mark.parametrize("policy,costs", [(0, (0, 0, 0)), (1, (0, 0, 0)), (2, (50.0, 4.0, 1.0)), (2, (1e9, 1e9, 1.0))])
@pytest.mark.parametrize("theta", [0.5, 0.4, 0.7])
def test_coverage_exactly_once(ora, policy, costs, theta):
    x, y, z = synth.plummer(700, 21)
    t = ora.Tree(x, y, z, 6)
    t.traverse(theta, policy, costs)
    L = t.lists()
    cnt = coverage(t, L, 700)
    assert np.all(cnt == 1)
    c = t.cells()
    leaf = c["nchild"] == 0
    th2 = theta * theta
    # accepted pairs satisfy the criterion; P2P pairs either fail it between leaves or were chosen
    for k in (0, 1, 2):
        for a, b in zip(*L[k]):
            R2 = float(np.sum((c["centre_h"][a] - c["centre_h"][b]) ** 2))
            rr = float(c["radius_h"][a] + c["radius_h"][b])
            acc = rr * rr <= th2 * R2
            if k != 2:
                assert acc
            else:
                assert acc or (leaf[a] and leaf[b])
    if policy == 0:
        assert L[1][0].size == 0
    if policy == 1:
        assert L[0][0].size == 0


def _mac_accepts(c, a, b, theta):
    R2 = float(np.sum((c["centre_h"][a] - c["centre_h"][b]) ** 2))
    rr = float(c["radius_h"][a] + c["radius_h"][b])
    return rr * rr <= theta * theta * R2


@pytest.mark.parametrize("policy,costs", [(0, (0, 0, 0)), (2, (50.0, 4.0, 1.0))])
@pytest.mark.parametrize("theta", [0.5, 0.4])
def test_split_the_larger_cell_on_adaptive_tree(ora, policy, costs, theta):
    """The paper's dual traversal splits the larger cell of each pair that
    fails the criterion ("Dual tree traversal"); with cubes, larger = lower
    level, both on a tie, and a leaf cannot split.  Two consequences checked on
    an adaptive tree with many level differences:
    - every emitted pair has equal levels, or its larger (lower-level) cell is
      a leaf (a larger non-leaf cell is never kept while the smaller splits);
    - every emitted pair other than the root pair has a parent pair, one split
      away (each split side replaced by its parent cell), that failed the
      criterion, is not a pair of leaves, and whose split sides are exactly
      the lower-level non-leaf cells (both at equal levels).
    Splitting only one cell on a tie fails both checks.  (With ties split
    both, two non-leaf cells of a visited pair always have equal levels, so
    "larger" only ever decides between a leaf and a non-leaf cell.)"""
    x, y, z = synth.plummer(5000, 33)
    t = ora.Tree(x, y, z, 8)
    t.traverse(theta, policy, costs)
    L = t.lists()
    c = t.cells()
    lev, par = c["level"].astype(np.int64), c["parent"].astype(np.int64)
    leaf = c["nchild"] == 0
    ctr, rad = c["centre_h"].astype(np.float64), c["radius_h"].astype(np.float64)
    pairs = np.concatenate([np.stack(L[k], axis=1) for k in (0, 1, 2)]).astype(np.int64)
    a, b = pairs[:, 0], pairs[:, 1]
    neq = lev[a] != lev[b]
    big = np.where(lev[a] < lev[b], a, b)
    assert np.all(leaf[big[neq]])
    unequal = int(neq.sum())
    keep = ~((a == 0) & (b == 0))
    a, b = a[keep], b[keep]

    def consistent(pa, pb, how_a, how_b):
        """Candidate parents (pa, pb) whose rule splits exactly the given sides."""
        valid = (pa >= 0) & (pb >= 0)
        pa_, pb_ = np.where(valid, pa, 0), np.where(valid, pb, 0)
        R2 = np.sum((ctr[pa_] - ctr[pb_]) ** 2, axis=1)
        rr = rad[pa_] + rad[pb_]
        fails = ~(rr * rr <= theta * theta * R2)
        sa = ~leaf[pa_] & (leaf[pb_] | (lev[pa_] <= lev[pb_]))
        sb = ~leaf[pb_] & (leaf[pa_] | (lev[pb_] <= lev[pa_]))
        return valid & fails & ~(leaf[pa_] & leaf[pb_]) & (sa == how_a) & (sb == how_b)

    ok = consistent(par[a], par[b], True, True) | consistent(par[a], b, True, False) | \
        consistent(a, par[b], False, True)
    assert np.all(ok), pairs[keep][~ok][:5]
    assert unequal > 100       # the tree really mixes levels


def grid_points(m):
    g = np.arange(m) / (m - 1.0)
    X, Y, Z = np.meshgrid(g, g, g, indexing="ij")
    return X.ravel(), Y.ravel(), Z.ravel()


@pytest.mark.parametrize("theta,near,far,margin", [(0.5, 27, 189, 3), (0.4, 81, 567, 5)])
def test_full_tree_neighbour_counts(ora, theta, near, far, margin):
    """theta = 0.5 is equivalent to the 3x3x3 neighbour list ("Results"):
    interior leaves have 27 particle-particle partners and interior cells 189
    cell-cell partners; theta = 0.4 gives the |d|^2 <= 6 list (81) and 567."""
    x, y, z = grid_points(16)   # one point per level-4 cell
    t = ora.Tree(x, y, z, 1)
    c = t.cells()
    assert t.ncell == 1 + 8 + 64 + 512 + 4096
    t.traverse(theta, 0)
    L = t.lists()
    p2p = np.bincount(L[2][0], minlength=t.ncell)
    m2l = np.bincount(L[0][0], minlength=t.ncell)
    a = c["centre_h"] // c["radius_h"][:, None]  # odd integers: 2*anchor + 1
    anchor = (a - 1) // 2
    lev = c["level"]
    side = 1 << lev
    lo_ok = np.all(anchor >= margin, axis=1)
    hi_ok = np.all(anchor <= side[:, None] - 1 - margin, axis=1)
    interior4 = (lev == 4) & lo_ok & hi_ok
    assert interior4.sum() > 0
    assert np.all(p2p[interior4] == near)
    assert np.all(m2l[interior4] == far)
    assert m2l.max() == far
    # same-level only: every M2L pair joins cells of one level
    assert np.all(lev[L[0][0]] == lev[L[0][1]])


def test_paper_facts_fixture(ora):
    with open(os.path.join(GOLDEN, "paper_facts.json")) as f:
        facts = json.load(f)
    assert facts["theta_half_neighbour_list"]["near"] == 27
    assert facts["theta_half_neighbour_list"]["far"] == 189


# ---------------------------------------------------------------- harmonics
def test_ylm_low_orders_and_scipy(ora):
    rng = np.random.default_rng(2)
    for _ in range(10):
        a, b = rng.uniform(0, math.pi), rng.uniform(-math.pi, math.pi)
        Y = ora.ylm(12, a, b)
        assert abs(Y[ora.cidx(0, 0)] - 1) < 1e-15
        assert abs(Y[ora.cidx(1, 0)] - math.cos(a)) < 1e-15
        assert abs(Y[ora.cidx(1, 1)] - math.sin(a) * np.exp(1j * b) / math.sqrt(2)) < 1e-15
        for n in range(13):
            for m in range(-n, n + 1):
                am = abs(m)
                # scipy's lpmv carries the Condon-Shortley phase (-1)^m
                ref = (-1) ** am * lpmv(am, n, math.cos(a)) * math.sqrt(
                    math.factorial(n - am) / math.factorial(n + am)) * np.exp(1j * m * b)
                assert abs(Y[ora.cidx(n, m)] - ref) < 1e-12 * max(1.0, abs(ref))


def test_addition_theorem(ora):
    rng = np.random.default_rng(3)
    for _ in range(5):
        u = rng.normal(size=3); u /= np.linalg.norm(u)
        v = rng.normal(size=3); v /= np.linalg.norm(v)
        _, a1, b1 = sph(u)
        _, a2, b2 = sph(v)
        Y1, Y2 = ora.ylm(10, a1, b1), ora.ylm(10, a2, b2)
        for n in range(11):
            s = sum(Y1[ora.cidx(n, -m)] * Y2[ora.cidx(n, m)] for m in range(-n, n + 1))
            assert abs(s - eval_legendre(n, float(u @ v))) < 1e-13


# ---------------------------------------------------------------- expansions
def charges_in_ball(k, c, a, seed):
    rng = np.random.default_rng(seed)
    d = rng.normal(size=(k, 3))
    d /= np.linalg.norm(d, axis=1)[:, None]
    d *= a * rng.uniform(0, 1, size=(k, 1)) ** (1 / 3)
    return np.asarray(c) + d, rng.uniform(-1, 1, size=k)


def test_single_charge_at_centre(ora):
    c = np.array([0.3, -0.2, 0.1])
    M = ora.p2m(8, c, c[None, :], np.array([2.5]))
    x = np.array([1.7, 0.4, -0.9])
    r = np.linalg.norm(x - c)
    assert abs(ora.mp_series(8, M, c, x) - 2.5 / r) < 1e-15 * 2.5 / r * 10
    phi, e = ora.m2p(8, M, c, x)
    assert abs(phi - 2.5 / r) < 1e-14
    assert np.allclose(e, 2.5 * (x - c) / r ** 3, rtol=1e-13, atol=0)


@pytest.mark.parametrize("p", [2, 5, 9, 14])
def test_multipole_error_bound(ora, p):
    """|phi - phi_p| <= A / (r - a) (a / r)^(p+1) (Greengard-Rokhlin theorem 3.2)."""
    c = np.zeros(3)
    a = 0.5
    src, q = charges_in_ball(30, c, a, 7)
    M = ora.p2m(p, c, src, q)
    A = np.abs(q).sum()
    rng = np.random.default_rng(8)
    for _ in range(20):
        d = rng.normal(size=3)
        x = d / np.linalg.norm(d) * rng.uniform(1.2, 3.0)
        r = np.linalg.norm(x)
        exact, _ = ora.direct_st(src, q, x[None, :])
        bound = A / (r - a) * (a / r) ** (p + 1)
        assert abs(ora.mp_series(p, M, c, x) - exact[0]) <= bound * (1 + 1e-9) + 1e-14
        phi, _ = ora.m2p(p, M, c, x)
        assert abs(phi - exact[0]) <= bound * (1 + 1e-9) + 1e-14


def test_m2p_gradient_is_minus_field(ora):
    src, q = charges_in_ball(20, np.zeros(3), 0.4, 9)
    M = ora.p2m(24, np.zeros(3), src, q)
    x = np.array([1.3, -1.1, 0.8])
    _, e = ora.m2p(24, M, np.zeros(3), x)
    _, Eex = ora.direct_st(src, q, x[None, :])
    assert np.allclose(e, Eex[0], rtol=1e-10, atol=1e-13)


def test_m2m_equals_direct_p2m(ora):
    """Translating a child's multipole to the parent centre reproduces the parent
    P2M exactly for the truncated series (degree j only needs degrees <= j)."""
    pc = np.array([0.1, 0.2, 0.3])
    cc = pc + np.array([0.25, -0.25, 0.25])
    src, q = charges_in_ball(25, cc, 0.2, 10)
    for p in (4, 10):
        Mc = ora.p2m(p, cc, src, q)
        Mp = ora.p2m(p, pc, src, q)
        Mt = ora.m2m(p, Mc, cc - pc)
        assert np.max(np.abs(Mt - Mp)) < 1e-13 * np.max(np.abs(Mp))


def test_l2l_is_exact_recentring(ora):
    rng = np.random.default_rng(11)
    p = 9
    K = ora.ncoef(p)
    Lc = rng.normal(size=K) + 1j * rng.normal(size=K)
    # a local expansion of a real field: L_n^{-m} = conj(L_n^m), L_n^0 real
    for n in range(p + 1):
        Lc[ora.cidx(n, 0)] = Lc[ora.cidx(n, 0)].real
        for m in range(1, n + 1):
            Lc[ora.cidx(n, -m)] = np.conj(Lc[ora.cidx(n, m)])
    old = np.array([0.0, 0.0, 0.0])
    new = np.array([0.12, -0.07, 0.05])
    Ln = ora.l2l(p, Lc, old - new)
    for _ in range(10):
        x = new + rng.normal(size=3) * 0.1
        v1 = ora.local_series(p, Lc, old, x)
        v2 = ora.local_series(p, Ln, new, x)
        assert abs(v1 - v2) < 1e-13 * max(1, abs(v1))
        phi, e = ora.l2p(p, Lc, old, x)
        assert abs(phi - v1) < 1e-13 * max(1, abs(v1))
        # gradient by central differences of the series value
        h = 1e-5
        g = np.array([(ora.local_series(p, Lc, old, x + h * d) - ora.local_series(p, Lc, old, x - h * d)) / (2 * h)
                      for d in np.eye(3)])
        assert np.allclose(-e, g, rtol=1e-7, atol=1e-7)


def test_m2l_converges_geometrically(ora):
    """Far cluster -> local expansion -> evaluation approaches the direct value
    geometrically in p and reaches FP64 rounding at high order."""
    sc = np.array([2.0, 1.0, -1.0])
    src, q = charges_in_ball(30, sc, 0.3, 12)
    tc = np.zeros(3)
    tx = tc + np.random.default_rng(13).normal(size=(8, 3)) * 0.15
    ex_phi, ex_E = ora.direct_st(src, q, tx)
    errs = []
    for p in (2, 4, 8, 12, 18, 24):
        M = ora.p2m(p, sc, src, q)
        L = ora.m2l(p, M, sc - tc)
        ph = np.array([ora.l2p(p, L, tc, x)[0] for x in tx])
        E = np.array([ora.l2p(p, L, tc, x)[1] for x in tx])
        errs.append((np.abs(ph - ex_phi).max() / np.abs(ex_phi).max(), np.abs(E - ex_E).max() / np.abs(ex_E).max()))
    errs = np.array(errs)
    assert np.all(np.diff(np.log(errs[:4, 0])) < -1.0)
    assert errs[-1, 0] < 1e-13 and errs[-1, 1] < 1e-12


# ---------------------------------------------------------------- direct sum
def test_direct_newton_third_law_and_two_body(ora):
    x, y, z = synth.uniform_cube(2000, 4)
    q = synth.charges_uniform(2000, 104)
    phi, E = ora.direct(x, y, z, q)
    net = (q[:, None] * E).sum(axis=0)
    assert np.linalg.norm(net) < 1e-12 * np.abs(q[:, None] * E).sum()
    # sum_i q_i phi_i is symmetric in the pair order: reversing indices gives the same value
    phi_r, _ = ora.direct(x[::-1], y[::-1], z[::-1], q[::-1])
    assert abs((q * phi).sum() - (q[::-1] * phi_r).sum()) < 1e-10 * np.abs(q * phi).sum()
    # two bodies: closed form
    xs = np.array([0.0, 3.0]); zs = np.zeros(2); qs = np.array([2.0, -1.0])
    p2, E2 = ora.direct(xs, np.array([0.0, 4.0]), zs, qs)
    assert p2[0] == -1.0 / 5.0 and p2[1] == 2.0 / 5.0
    assert np.allclose(E2[0], -1.0 * np.array([-3.0, -4.0, 0.0]) / 125.0, rtol=1e-15)


def test_direct_coincident_points_skipped(ora):
    x = np.array([0.0, 0.0, 1.0]); y = np.zeros(3); z = np.zeros(3); q = np.array([1.0, 5.0, 2.0])
    phi, E = ora.direct(x, y, z, q)
    assert phi[0] == 2.0 and phi[1] == 2.0 and phi[2] == 6.0


def test_direct_scale_covariance(ora):
    x, y, z = synth.uniform_cube(500, 6)
    q = synth.charges_uniform(500, 106)
    phi, E = ora.direct(x, y, z, q)
    phi2, E2 = ora.direct(8 * x, 8 * y, 8 * z, q)
    assert np.array_equal(phi2, phi / 8) and np.array_equal(E2, E / 64)


def test_direct_field_is_minus_gradient(ora):
    src = np.stack(synth.uniform_cube(300, 7), axis=1)
    q = synth.charges_uniform(300, 107)
    xt = np.array([[0.41, 0.52, 0.33]])
    _, E = ora.direct_st(src, q, xt)
    h = 1e-6
    g = [(ora.direct_st(src, q, xt + h * d)[0][0] - ora.direct_st(src, q, xt - h * d)[0][0]) / (2 * h)
         for d in np.eye(3)]
    assert np.allclose(-np.array(g), E[0], rtol=1e-6)


# ---------------------------------------------------------------- whole method
def test_fmm_single_leaf_is_direct(ora):
    x, y, z = synth.uniform_cube(50, 8)
    q = synth.charges_uniform(50, 108)
    phi, E, t = ora.fmm(x, y, z, q, 6, 0.5, 64)
    assert t.ncell == 1
    pd, Ed = ora.direct(x, y, z, q)
    # same sums in a different order: equal up to FP64 rounding
    assert np.abs(phi - pd).max() < 1e-13 * np.abs(pd).max()
    assert np.abs(E - Ed).max() < 1e-13 * np.abs(Ed).max()


def test_fmm_error_falls_geometrically_with_p(ora):
    x, y, z = synth.uniform_cube(4096, 9)
    q = synth.charges_uniform(4096, 109)
    pd, Ed = ora.direct(x, y, z, q)
    e = []
    for p in (2, 4, 6, 8, 10):
        phi, E, _ = ora.fmm(x, y, z, q, p, 0.5, 32)
        e.append((ora.rel_l2(phi, pd), ora.rel_l2(E, Ed)))
    e = np.array(e)
    assert np.all(np.diff(np.log10(e[:, 0])) < -0.5)
    assert np.all(np.diff(np.log10(e[:, 1])) < -0.4)
    # "p = 10 gives 4 significant digits in the potential" (introduction to treecodes & FMM)
    assert e[-1, 0] < 1e-4
    # high order and small theta approach FP64 rounding
    phi, E, _ = ora.fmm(x, y, z, q, 20, 0.3, 32)
    assert ora.rel_l2(phi, pd) < 1e-11


def test_fmm_policies_agree_with_direct(ora):
    x, y, z = synth.plummer(3000, 10)
    q = synth.charges_uniform(3000, 110)
    pd, Ed = ora.direct(x, y, z, q)
    for pol, costs in ((0, (0, 0, 0)), (1, (0, 0, 0)), (2, (100.0, 3.0, 1.0))):
        phi, E, _ = ora.fmm(x, y, z, q, 10, 0.4, 16, pol, costs)
        assert ora.rel_l2(phi, pd) < 2e-5 and ora.rel_l2(E, Ed) < 1e-5


def test_fmm_scale_covariance(ora):
    x, y, z = synth.plummer(2000, 12)
    q = synth.charges_uniform(2000, 112)
    phi, E, t = ora.fmm(x, y, z, q, 6, 0.5, 16)
    phi2, E2, t2 = ora.fmm(4 * x, 4 * y, 4 * z, q, 6, 0.5, 16)
    k1, p1 = t.keys()
    k2, p2 = t2.keys()
    assert np.array_equal(k1, k2) and np.array_equal(p1, p2)
    L1, L2 = t.lists(), t2.lists()
    for k in (0, 1, 2):
        assert np.array_equal(L1[k][0], L2[k][0]) and np.array_equal(L1[k][1], L2[k][1])
    assert np.allclose(phi2, phi / 4, rtol=1e-13, atol=0)
    assert np.allclose(E2, E / 16, rtol=1e-12, atol=1e-14 * np.abs(E).max())


# ---------------------------------------------------------------- targets != sources
def _ts_sets(nt=600, ns=800, seed=41):
    t = np.stack(synth.uniform_cube(nt, seed), 1) * 1.6 - 0.3        # overlaps the shell and its inside
    s = np.stack(synth.sphere_shell(ns, seed + 1), 1)
    q = synth.charges_uniform(ns, seed + 2)
    return t, s, q


@pytest.mark.parametrize("policy,costs", [(0, (0, 0, 0)), (1, (0, 0, 0)), (2, (50.0, 4.0, 1.0))])
@pytest.mark.parametrize("theta", [0.5, 0.4])
def test_ts_coverage_exactly_once(ora, policy, costs, theta):
    """Separate target and source trees ("Dual tree traversal"): every
    (target, source) particle pair is covered by exactly one emitted
    interaction, every list pairs a target-tree cell with a source-tree cell,
    and accepted pairs satisfy the criterion."""
    t, s, q = _ts_sets()
    tr = ora.Tree.targets_sources(t, s, 6)
    tr.traverse(theta, policy, costs)
    L = tr.lists()
    c = tr.cells()
    nt, ns = t.shape[0], s.shape[0]
    is_t = c["begin"] < nt
    cnt = np.zeros((nt, ns), np.int64)
    for k in (0, 1, 2):
        for a, b in zip(*L[k]):
            assert is_t[a] and not is_t[b]
            if k != 2:
                assert _mac_accepts(c, a, b, theta)
            cnt[c["begin"][a]:c["end"][a], c["begin"][b] - nt:c["end"][b] - nt] += 1
    assert np.all(cnt == 1)


def test_ts_values_against_direct_and_same_set(ora):
    """The potential and field at the targets due to the sources match the
    direct sum within the method's error, the error falls with p, and with the
    targets equal to the sources the two-tree evaluation equals the one-tree
    evaluation bit for bit."""
    t, s, q = _ts_sets(1500, 2000, 5)
    pd, Ed = ora.direct_st(s, q, t)
    errs = []
    for p in (4, 8, 12):
        tr = ora.Tree.targets_sources(t, s, 16)
        tr.traverse(0.5, 0)
        phi, E = tr.evaluate(p, q)
        errs.append(ora.rel_l2(phi, pd))
        if p == 12:
            assert ora.rel_l2(phi, pd) < 1e-6 and ora.rel_l2(E, Ed) < 1e-5
    assert errs[0] > errs[1] > errs[2]
    x, y, z = synth.plummer(3000, 7)
    qq = synth.charges_uniform(3000, 8)
    P = np.stack([x, y, z], 1)
    two = ora.Tree.targets_sources(P, P, 16)
    two.traverse(0.5, 0)
    ph2, E2 = two.evaluate(8, qq)
    po, Eo, _ = ora.fmm(x, y, z, qq, 8, 0.5, 16)
    assert np.array_equal(ph2, po) and np.array_equal(E2, Eo)


def test_ts_empty_sides(ora):
    t, s, q = _ts_sets(50, 70)
    none = ora.Tree.targets_sources(t, s[:0], 8)
    none.traverse(0.5, 0)
    phi, E = none.evaluate(6, q[:0])
    assert phi.size == 50 and np.all(phi == 0) and np.all(E == 0)
    only_src = ora.Tree.targets_sources(t[:0], s, 8)
    only_src.traverse(0.5, 0)
    assert all(only_src.lists()[k][0].size == 0 for k in (0, 1, 2))
