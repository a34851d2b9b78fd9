"""Seeded synthetic inputs shared by the oracle tests, the GPU tests and the bench.

This module holds no arithmetic of the fast multipole method: it only draws
particle positions, charges, target samples and batch sizes.  Every draw is a
pure function of (seed, stream, counter), so any slice of any array can be
regenerated independently and the same numbers feed both the oracle and the
HIP path.

Generator: SplitMix64 (Steele, Lea and Flood, "Fast splittable pseudorandom
number generators", OOPSLA 2014) in its counter form.  The state of draw ``i``
of a stream is ``base + (i + 1) * GAMMA`` (mod 2**64) and the output is the
SplitMix64 finaliser applied to that state.  ``base`` is the finaliser applied
to ``seed * GAMMA ^ (stream << 48)``.  A uniform double in [0, 1) keeps the
top 53 bits: ``(bits >> 11) * 2**-53``.

Workloads follow the particle sets the paper evaluates on (random points in a
cube; random points on a spherical shell) plus a Plummer sphere for the
adaptive case.
"""
from __future__ import annotations

import math

import numpy as np

GAMMA = np.uint64(0x9E3779B97F4A7C15)
_M1 = np.uint64(0xBF58476D1CE4E5B9)
_M2 = np.uint64(0x94D049BB133111EB)

# stream ids (one independent sequence per purpose)
S_X, S_Y, S_Z, S_Q, S_PERM, S_SIZE, S_KIND = 0, 1, 2, 3, 4, 5, 6


def _mix(z: np.ndarray) -> np.ndarray:
    with np.errstate(over="ignore"):
        z = (z ^ (z >> np.uint64(30))) * _M1
        z = (z ^ (z >> np.uint64(27))) * _M2
        return z ^ (z >> np.uint64(31))


def bits(seed: int, stream: int, start: int, count: int) -> np.ndarray:
    """64-bit draws ``start .. start+count-1`` of (seed, stream)."""
    with np.errstate(over="ignore"):
        s = np.array([(int(seed) * int(GAMMA)) % (1 << 64)], dtype=np.uint64)
        s ^= np.uint64((int(stream) & 0xFFFF) << 48)
        base = _mix(s)[0]
        ctr = np.arange(start + 1, start + count + 1, dtype=np.uint64)
        return _mix(base + ctr * GAMMA)


def uniform(seed: int, stream: int, count: int, start: int = 0) -> np.ndarray:
    """Doubles in [0, 1): the top 53 bits of each draw times 2**-53."""
    b = bits(seed, stream, start, count)
    return (b >> np.uint64(11)).astype(np.float64) * (2.0 ** -53)


def uniform_cube(n: int, seed: int):
    """n points uniform in the unit cube [0, 1)^3 (float64)."""
    return (uniform(seed, S_X, n), uniform(seed, S_Y, n), uniform(seed, S_Z, n))


def plummer(n: int, seed: int, a: float = 1.0, rmax: float = 20.0):
    """n points of a Plummer sphere of scale radius ``a``, truncated at ``rmax * a``.

    Radius from the inverse cumulative mass: X ~ U(0,1), r = a (X^(-2/3) - 1)^(-1/2);
    candidates with r > rmax * a are rejected and the next candidate is taken.
    Direction: cos(polar) = 2u - 1, azimuth = 2 pi u'.  (Aarseth, Henon and
    Wielen 1974 sampling.)
    """
    xs = np.empty(n)
    ys = np.empty(n)
    zs = np.empty(n)
    filled = 0
    cursor = 0
    while filled < n:
        m = max(1024, int((n - filled) * 1.05) + 64)
        X = uniform(seed, S_X, m, cursor)
        u = uniform(seed, S_Y, m, cursor)
        v = uniform(seed, S_Z, m, cursor)
        cursor += m
        with np.errstate(divide="ignore", invalid="ignore"):
            r = a / np.sqrt(X ** (-2.0 / 3.0) - 1.0)
        r = np.where(X == 0.0, 0.0, r)
        keep = np.isfinite(r) & (r <= rmax * a)
        r, u, v = r[keep], u[keep], v[keep]
        take = min(n - filled, r.size)
        r, u, v = r[:take], u[:take], v[:take]
        ct = 2.0 * u - 1.0
        st = np.sqrt(np.maximum(0.0, 1.0 - ct * ct))
        ph = 2.0 * math.pi * v
        xs[filled:filled + take] = r * st * np.cos(ph)
        ys[filled:filled + take] = r * st * np.sin(ph)
        zs[filled:filled + take] = r * ct
        filled += take
    return xs, ys, zs


def sphere_shell(n: int, seed: int, radius: float = 1.0):
    """n points uniform on a sphere surface (the paper's spherical-shell test)."""
    u = uniform(seed, S_X, n)
    v = uniform(seed, S_Y, n)
    ct = 2.0 * u - 1.0
    st = np.sqrt(np.maximum(0.0, 1.0 - ct * ct))
    ph = 2.0 * math.pi * v
    return radius * st * np.cos(ph), radius * st * np.sin(ph), radius * ct


def charges_uniform(n: int, seed: int) -> np.ndarray:
    """Charges uniform in [-1, 1)."""
    return 2.0 * uniform(seed, S_Q, n) - 1.0


def charges_equal(n: int) -> np.ndarray:
    """Equal masses 1/n."""
    return np.full(n, 1.0 / n)


def target_sample(n: int, k: int, seed: int) -> np.ndarray:
    """k distinct indices of range(n): the first k slots of a partial Fisher-Yates shuffle."""
    k = min(k, n)
    u = uniform(seed, S_PERM, k)
    idx = np.arange(n, dtype=np.int64)
    for i in range(k):
        j = i + int(u[i] * (n - i))
        idx[i], idx[j] = idx[j], idx[i]
    return np.sort(idx[:k])


def batch_sizes(n_inst: int, seed: int, lo: int = 1024, hi: int = 262144):
    """Instance sizes log-uniform in [lo, hi] and a 50/50 kind draw (0 cube, 1 Plummer)."""
    u = uniform(seed, S_SIZE, n_inst)
    sizes = np.floor(np.exp(math.log(lo) + u * (math.log(hi) - math.log(lo)))).astype(np.int64)
    sizes = np.clip(sizes, lo, hi)
    kinds = (uniform(seed, S_KIND, n_inst) < 0.5).astype(np.int64)
    return sizes, kinds


from .workloads import WORKLOADS, make_batch, make_workload  # noqa: E402,F401
