"""Pins of the oracle's Cartesian (Taylor) expansions, the family the hybrid
method switches to at low accuracy ("Hybrid treecode/FMM algorithm").

- Taylor coefficients a_n(R) of 1/|R| against closed forms of the first
  derivatives, the Legendre generating function (sum over |n| = d of
  a_n(R) h^n = (-|h|)^d P_d(cos g) / |R|^(d+1)), and Laplace's equation
  (the trace of every coefficient tensor vanishes);
- M2M equals a direct P2M about the new centre; L2L is an exact re-centring;
- the degree-n Cartesian multipole term equals the degree-n spherical one
  (the contraction with derivatives of 1/r keeps only the harmonic part), so
  Cartesian and spherical M2P of the same order agree to rounding;
- M2L + L2P and M2P converge to the direct sum; the full evaluation equals
  the direct sum for a single leaf and its error falls with p.
"""
import numpy as np
import pytest
from scipy.special import eval_legendre

import synth


def _multi(P):
    for n in range(P + 1):
        for a in range(n, -1, -1):
            for b in range(n - a, -1, -1):
                yield n, a, b, n - a - b


def test_taylor_closed_forms(ora):
    R = np.array([0.7, -1.1, 0.45])
    r = np.linalg.norm(R)
    a = ora.cart_taylor(3, R)
    assert a[ora.cart_index(0, 0, 0)] == pytest.approx(1 / r, rel=1e-15)
    for d in range(3):
        e = [0, 0, 0]
        e[d] = 1
        assert a[ora.cart_index(*e)] == pytest.approx(-R[d] / r ** 3, rel=1e-14)
    # d2/dx dy (1/r) = 3 x y / r^5 (a_(1,1,0) = that / (1! 1!))
    assert a[ora.cart_index(1, 1, 0)] == pytest.approx(3 * R[0] * R[1] / r ** 5, rel=1e-14)
    # d2/dx2 (1/r) / 2! = (3 x^2 - r^2) / (2 r^5)
    assert a[ora.cart_index(2, 0, 0)] == pytest.approx((3 * R[0] ** 2 - r ** 2) / (2 * r ** 5), rel=1e-14)
    assert ora.cart_count(3) == 20 and ora.cart_index(0, 0, 3) == 19


@pytest.mark.parametrize("seed", [1, 2, 3])
def test_taylor_legendre_generating_function(ora, seed):
    rng = np.random.default_rng(seed)
    R = rng.normal(size=3) * 2
    h = rng.normal(size=3)
    P = 12
    a = ora.cart_taylor(P, R)
    r, hn = np.linalg.norm(R), np.linalg.norm(h)
    cg = R @ h / (r * hn)
    for d in range(P + 1):
        s = sum(a[ora.cart_index(i, j, k)] * h[0] ** i * h[1] ** j * h[2] ** k
                for n, i, j, k in _multi(P) if n == d)
        ref = (-hn) ** d * eval_legendre(d, cg) / r ** (d + 1)
        assert s == pytest.approx(ref, rel=1e-11, abs=1e-14 * abs(ref) + 1e-300)


def test_taylor_trace_free(ora):
    """Laplace: sum_i (k_i + 1)(k_i + 2) a_{k + 2 e_i} = 0 for every k."""
    R = np.array([-0.4, 0.9, 1.3])
    P = 10
    a = ora.cart_taylor(P, R)
    for n, i, j, k in _multi(P - 2):
        t = ((i + 1) * (i + 2) * a[ora.cart_index(i + 2, j, k)] + (j + 1) * (j + 2) * a[ora.cart_index(i, j + 2, k)]
             + (k + 1) * (k + 2) * a[ora.cart_index(i, j, k + 2)])
        scale = max(abs(a[ora.cart_index(i + 2, j, k)]), 1e-300)
        assert abs(t) <= 1e-11 * scale * 10


def _cluster(n, seed, centre, size):
    x, y, z = synth.uniform_cube(n, seed)
    xyz = (np.stack([x, y, z], 1) - 0.5) * size + centre
    return xyz, synth.charges_uniform(n, seed + 100)


def test_m2m_equals_direct_p2m_and_l2l_is_exact(ora):
    p = 7
    xyz, q = _cluster(40, 3, np.array([0.2, 0.1, -0.3]), 0.5)
    c1 = np.array([0.25, 0.05, -0.2])
    c2 = np.array([0.0, 0.0, 0.0])
    M1 = ora.cart_p2m(p, c1, xyz, q)
    M2 = ora.cart_p2m(p, c2, xyz, q)
    assert np.abs(ora.cart_m2m(p, M1, c2 - c1) - M2).max() <= 1e-13 * np.abs(M2).max()
    L = np.random.default_rng(5).normal(size=ora.cart_count(p))
    t1, t2 = np.array([0.0, 0.1, 0.2]), np.array([0.13, -0.07, 0.25])
    L2 = ora.cart_l2l(p, L, t2 - t1)
    for x in np.random.default_rng(6).uniform(-0.3, 0.3, (5, 3)):
        a, ea = ora.cart_l2p(p, L, t1, x)
        b, eb = ora.cart_l2p(p, L2, t2, x)
        assert b == pytest.approx(a, rel=1e-12, abs=1e-12)
        assert np.allclose(ea, eb, rtol=1e-11, atol=1e-11)


@pytest.mark.parametrize("p", [2, 5, 9])
def test_cartesian_m2p_equals_spherical_m2p(ora, p):
    xyz, q = _cluster(30, 7, np.zeros(3), 0.6)
    c = np.zeros(3)
    Mc = ora.cart_p2m(p, c, xyz, q)
    Ms = ora.p2m(p, c, xyz, q)
    for x in (np.array([2.0, 0.3, -0.5]), np.array([-0.4, -1.7, 1.1])):
        a, ea = ora.cart_m2p(p, Mc, c, x)
        b, eb = ora.m2p(p, Ms, c, x)
        assert a == pytest.approx(b, rel=1e-12)
        assert np.allclose(ea, eb, rtol=1e-11, atol=1e-13 * np.abs(eb).max())


def test_m2l_l2p_and_m2p_converge_to_direct(ora):
    xyz, q = _cluster(50, 11, np.zeros(3), 1.0)
    s = np.zeros(3)
    t = np.array([3.0, 1.0, -0.5])
    tx = (np.random.default_rng(12).uniform(-0.5, 0.5, (6, 3))) + t
    pd, Ed = ora.direct_st(xyz, q, tx)
    e_prev = np.inf
    for p in (2, 4, 6, 8, 10):
        M = ora.cart_p2m(p, s, xyz, q)
        L = ora.cart_m2l(p, M, t - s)
        ph = np.array([ora.cart_l2p(p, L, t, x)[0] for x in tx])
        pm = np.array([ora.cart_m2p(p, M, s, x)[0] for x in tx])
        e = ora.rel_l2(ph, pd)
        assert e < e_prev
        e_prev = e
        assert ora.rel_l2(pm, pd) < 10 * (0.5 * np.sqrt(3) / 2.5) ** (p + 1)
    assert e_prev < 1e-5


def test_full_cartesian_fmm(ora):
    x, y, z = synth.plummer(4000, 13)
    q = synth.charges_uniform(4000, 113)
    pd, Ed = ora.direct(x, y, z, q)
    one = ora.Tree(x[:50], y[:50], z[:50], 64)
    one.traverse(0.5, 0)
    ph1, E1 = one.evaluate_cart(4, q[:50])
    p1, e1 = ora.direct(x[:50], y[:50], z[:50], q[:50])
    assert ora.rel_l2(ph1, p1) < 1e-14 and ora.rel_l2(E1, e1) < 1e-14
    t = ora.Tree(x, y, z, 16)
    t.traverse(0.5, 0)
    errs = [ora.rel_l2(t.evaluate_cart(p, q)[0], pd) for p in (2, 4, 6, 8)]
    assert all(a > b for a, b in zip(errs, errs[1:]))
    # treecode lists (cell-particle and particle-particle only): the Cartesian
    # and spherical evaluations are the same truncated series
    t.traverse(0.5, 1)
    ph, E = t.evaluate_cart(8, q)
    ps, Es = t.evaluate(8, q)
    assert ora.rel_l2(ph, ps) < 1e-12 and ora.rel_l2(E, Es) < 1e-11
    # hybrid lists (all three kinds): the Cartesian error is the spherical
    # one's within the looser triangular truncation of Cartesian M2L
    t.traverse(0.5, 2, (50.0, 4.0, 1.0))
    for p in (6, 10):
        ec = ora.rel_l2(t.evaluate_cart(p, q)[0], pd)
        es = ora.rel_l2(t.evaluate(p, q)[0], pd)
        assert es <= ec < 1.5 * es
