"""The graded split-BF16 reading, checked on the oracle's FP64 expansions.

The split-BF16 form forms each FP32 product of the same-level M2L from BF16
halves, a = a_hi + a_lo, graded by multipole degree: coefficient index k < 32
(degrees 0-5) takes a_hi b_hi + a_hi b_lo + a_lo b_hi, 32 <= k < 48 drops
a_lo b_hi, k >= 48 keeps a_hi b_hi alone (a = operator entry, b = multipole
coefficient).  The reading rests on the decay of the expansion's terms with
degree ("Hierarchical N-body algorithms": the truncation error falls
geometrically with the order): a product's share of the local expansion falls
with the multipole degree, so coarser products there hold a small share of the
result.  Here the M2L operator of one well-separated same-level pair (offsets
accepted at theta = 0.4) is built column by column from the oracle, the
products are emulated in BF16 halves of the FP32 operands, and the potential of
the resulting local expansion is compared with the FP64 one: grading must add
almost nothing to the full three-product split, while two products everywhere,
or the tiers inverted (low degrees coarse), must be far worse.  Parity of the
GPU kernel itself is checked on the GPU (tests/test_gpu_bf16.py).
"""
import numpy as np
import pytest


def bf16(x):
    """Round FP32 values to BF16 (round to nearest even), returned as FP32."""
    x = np.asarray(x, np.float32)
    u = x.view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFF0000
    return u.astype(np.uint32).view(np.float32)


def split(x):
    x = np.asarray(x, np.float32)
    h = bf16(x)
    return h.astype(np.float64), bf16(x - h).astype(np.float64)


def product(a, b, tier):
    ah, al = split(a)
    bh, bl = split(b)
    if tier == 3:
        return ah * bh + ah * bl + al * bh
    if tier == 2:
        return ah * bh + ah * bl
    return ah * bh


def emulated_m2l(T, M, tiers):
    """L = T M with every real product formed by the tier of its multipole index."""
    Tr, Ti = T.real.astype(np.float32), T.imag.astype(np.float32)
    Mr, Mi = M.real.astype(np.float32), M.imag.astype(np.float32)
    L = np.zeros(T.shape[0], np.complex128)
    for k in range(T.shape[1]):
        t = tiers[k]
        L += (product(Tr[:, k], Mr[k], t) - product(Ti[:, k], Mi[k], t)) + 1j * (
            product(Tr[:, k], Mi[k], t) + product(Ti[:, k], Mr[k], t))
    return L


@pytest.mark.parametrize("offset,charges", [((3, 0, 0), "equal"), ((2, 2, 0), "signed"), ((2, 2, 2), "signed"),
                                            ((5, 0, 0), "equal")])
def test_graded_split_adds_almost_nothing(ora, offset, charges):
    p = 10
    K = ora.ncoef(p)
    rng = np.random.default_rng(sum(offset) * 7 + len(charges))
    sc = np.zeros(3)
    tc = 2.0 * np.array(offset, float)          # cells of half side 1, offset in cell sides
    assert 0.4 ** 2 * np.dot(offset, offset) >= 1.0  # accepted at theta = 0.4
    src = rng.uniform(-1, 1, size=(200, 3))
    q = np.ones(200) if charges == "equal" else rng.uniform(-1, 1, 200)
    M = ora.p2m(p, sc, src, q)
    T = np.zeros((K, K), np.complex128)
    for k in range(K):
        e = np.zeros(K, np.complex128)
        e[k] = 1.0
        T[:, k] = ora.m2l(p, e, sc - tc)
    L = T @ M
    assert np.allclose(L, ora.m2l(p, M, sc - tc), rtol=1e-10, atol=1e-14 * np.abs(L).max())
    tx = tc + rng.uniform(-1, 1, size=(64, 3))
    ref = np.array([ora.local_series(p, L, tc, x) for x in tx])

    def err(tiers):
        v = np.array([ora.local_series(p, emulated_m2l(T, M, tiers), tc, x) for x in tx])
        return float(np.sqrt(np.sum((v - ref) ** 2) / np.sum(ref ** 2)))

    k = np.arange(K)
    e3 = err(np.full(K, 3))
    eg = err(np.where(k < 32, 3, np.where(k < 48, 2, 1)))
    e2 = err(np.full(K, 2))
    einv = err(np.where(k < 32, 1, 3))
    print(offset, charges, "three %.2e graded %.2e two %.2e inverted %.2e" % (e3, eg, e2, einv))
    assert eg < 1e-5
    assert eg <= 1.1 * e3 + 1e-9
    assert e2 > 30 * eg and einv > 30 * eg
