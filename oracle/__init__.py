"""Python access to the FP64 CPU oracle (``fmm_oracle.c``).

TEST INFRASTRUCTURE ONLY: imported by ``tests/``, ``__graft_entry__.smoke()``
and the CPU-baseline leg of ``bench.py``; never by the library.  It shares no
code with the HIP path.

Functions mirror the C entry points and take/return numpy float64 arrays.
Expansion coefficients use full complex storage, index ``n*n + n + m`` for
``m = -n..n``, in the normalisation of Greengard & Rokhlin (Acta Numerica
1997): ``Y_n^m = sqrt((n-|m|)!/(n+|m|)!) P_n^|m|(cos a) e^{i m b}``, with
``P_n^m`` free of the Condon-Shortley phase.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "fmm_oracle.c")
_SRC_MLP = os.path.join(_HERE, "mlp_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

M2L, M2P, P2P = 0, 1, 2
POLICY_FMM, POLICY_TREECODE, POLICY_HYBRID = 0, 1, 2


def build(force: bool = False) -> str:
    """Compile the oracle with gcc (plain C99, OpenMP, no FMA contraction)."""
    stale = not os.path.exists(_LIB) or any(os.path.getmtime(_LIB) < os.path.getmtime(s) for s in (_SRC, _SRC_MLP))
    if force or stale:
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=gnu99", "-fopenmp", "-ffp-contract=off",
                               "-fcx-limited-range", "-fPIC", "-shared", _SRC, _SRC_MLP, "-o", tmp, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


_lib = None

D = ctypes.POINTER(ctypes.c_double)
I64 = ctypes.c_int64


def lib():
    global _lib
    if _lib is None:
        build()
        L = ctypes.CDLL(_LIB)
        vp = ctypes.c_void_p
        L.ora_build.restype = vp
        L.ora_build.argtypes = [I64, vp, vp, vp, ctypes.c_int32]
        L.ora_build_ts.restype = vp
        L.ora_build_ts.argtypes = [I64, vp, vp, vp, I64, ctypes.c_int32]
        L.ora_ncells.restype = I64
        L.ora_ncells.argtypes = [vp]
        L.ora_list_size.restype = I64
        L.ora_list_size.argtypes = [vp, ctypes.c_int]
        L.ora_traverse.argtypes = [vp, ctypes.c_double, ctypes.c_int, vp]
        L.ora_get_list.argtypes = [vp, ctypes.c_int, vp, vp]
        L.ora_get_keys.argtypes = [vp, vp, vp]
        L.ora_get_bbox.argtypes = [vp, vp, vp]
        L.ora_get_cells.argtypes = [vp] + [vp] * 11
        L.ora_evaluate.argtypes = [vp, ctypes.c_int, vp, vp, vp, vp, vp]
        L.ora_get_expansions.argtypes = [vp, vp, vp]
        L.ora_free.argtypes = [vp]
        L.ora_direct.argtypes = [I64, vp, vp, vp, vp, I64, vp, vp, vp, vp, vp]
        L.ora_direct_st.argtypes = [I64, vp, vp, vp, vp, I64, vp, vp, vp, vp, vp, vp, vp]
        L.ora_ylm.argtypes = [ctypes.c_int, ctypes.c_double, ctypes.c_double, vp]
        L.ora_p2m.argtypes = [ctypes.c_int, vp, I64, vp, vp, vp, vp, vp]
        L.ora_m2m.argtypes = [ctypes.c_int, vp, vp, vp]
        L.ora_m2l.argtypes = [ctypes.c_int, ctypes.c_int, vp, vp, vp]
        L.ora_l2l.argtypes = [ctypes.c_int, ctypes.c_int, vp, vp, vp]
        L.ora_l2p.argtypes = [ctypes.c_int, vp, vp, vp, vp, vp]
        L.ora_m2p.argtypes = [ctypes.c_int, vp, vp, vp, vp, vp]
        L.ora_mp_series.restype = ctypes.c_double
        L.ora_mp_series.argtypes = [ctypes.c_int, vp, vp, vp]
        L.ora_local_series.restype = ctypes.c_double
        L.ora_local_series.argtypes = [ctypes.c_int, vp, vp, vp]
        L.ora_bbox.argtypes = [I64, vp, vp, vp, vp, vp]
        L.ora_morton.argtypes = [I64, vp, vp, vp, vp, ctypes.c_double, vp]
        L.ora_num_threads.restype = ctypes.c_int
        L.ora_set_threads.argtypes = [ctypes.c_int]
        L.ora_traverse_table.argtypes = [vp, ctypes.c_double, vp]
        L.ora_mlp_forward.argtypes = [vp, vp, vp]
        L.ora_mlp_loss_grad.argtypes = [vp, ctypes.c_int, vp, vp, vp, vp, vp]
        L.ora_mlp_table64.argtypes = [vp, ctypes.c_int, ctypes.c_double, vp, vp, vp]
        L.ora_cart_count.restype = ctypes.c_int
        L.ora_cart_count.argtypes = [ctypes.c_int]
        L.ora_cart_index.restype = ctypes.c_int
        L.ora_cart_index.argtypes = [ctypes.c_int] * 3
        L.ora_cart_taylor.argtypes = [ctypes.c_int, vp, vp]
        L.ora_cart_p2m.argtypes = [ctypes.c_int, vp, I64, vp, vp, vp, vp, vp]
        L.ora_cart_m2m.argtypes = [ctypes.c_int, vp, vp, vp]
        L.ora_cart_m2l.argtypes = [ctypes.c_int, vp, vp, vp]
        L.ora_cart_l2l.argtypes = [ctypes.c_int, vp, vp, vp]
        L.ora_cart_l2p.argtypes = [ctypes.c_int, vp, vp, vp, vp, vp]
        L.ora_cart_m2p.argtypes = [ctypes.c_int, vp, vp, vp, vp, vp]
        L.ora_evaluate_cart.argtypes = [vp, ctypes.c_int, vp, vp, vp, vp, vp]
        L.ora_get_expansions_cart.argtypes = [vp, vp, vp]
        L.ora_interleave.restype = ctypes.c_uint64
        L.ora_interleave.argtypes = [ctypes.c_uint64] * 3
        _lib = L
    return _lib


def num_threads() -> int:
    return int(lib().ora_num_threads())


def set_threads(n: int) -> None:
    """Threads of the oracle's OpenMP loops from now on."""
    lib().ora_set_threads(int(n))


def _p(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


def _f64(a) -> np.ndarray:
    return np.ascontiguousarray(a, dtype=np.float64)


def ncoef(p: int) -> int:
    return (p + 1) * (p + 1)


def cidx(n: int, m: int) -> int:
    return n * n + n + m


# ---------------------------------------------------------------- direct sum
def direct(x, y, z, q, targets=None):
    """(phi, E) at ``targets`` (indices; default all) by O(N^2) summation."""
    x, y, z, q = map(_f64, (x, y, z, q))
    n = x.size
    tg = np.arange(n, dtype=np.int64) if targets is None else np.ascontiguousarray(targets, dtype=np.int64)
    nt = tg.size
    phi, ex, ey, ez = (np.zeros(nt) for _ in range(4))
    lib().ora_direct(n, _p(x), _p(y), _p(z), _p(q), nt, _p(tg), _p(phi), _p(ex), _p(ey), _p(ez))
    return phi, np.stack([ex, ey, ez], axis=1)


def direct_st(src_xyz, sq, tgt_xyz):
    """(phi, E) at explicit target points from explicit sources."""
    sx, sy, sz = (_f64(src_xyz[:, d]) for d in range(3))
    tx, ty, tz = (_f64(tgt_xyz[:, d]) for d in range(3))
    sq = _f64(sq)
    nt = tx.size
    phi, ex, ey, ez = (np.zeros(nt) for _ in range(4))
    lib().ora_direct_st(sx.size, _p(sx), _p(sy), _p(sz), _p(sq), nt, _p(tx), _p(ty), _p(tz),
                        _p(phi), _p(ex), _p(ey), _p(ez))
    return phi, np.stack([ex, ey, ez], axis=1)


# ---------------------------------------------------------------- keys
def bbox(x, y, z):
    x, y, z = map(_f64, (x, y, z))
    lo = np.zeros(3)
    side = np.zeros(1)
    lib().ora_bbox(x.size, _p(x), _p(y), _p(z), _p(lo), _p(side))
    return lo, float(side[0])


def morton(x, y, z, lo, side):
    x, y, z = map(_f64, (x, y, z))
    lo = _f64(lo)
    key = np.zeros(x.size, dtype=np.uint64)
    lib().ora_morton(x.size, _p(x), _p(y), _p(z), _p(lo), float(side), _p(key))
    return key


def interleave(qx: int, qy: int, qz: int) -> int:
    return int(lib().ora_interleave(qx, qy, qz))


# ---------------------------------------------------------------- harmonics / operators
def ylm(P: int, alpha: float, beta: float) -> np.ndarray:
    Y = np.zeros(ncoef(P), dtype=np.complex128)
    lib().ora_ylm(P, float(alpha), float(beta), _p(Y))
    return Y


def p2m(p, centre, xyz, q):
    xyz = np.asarray(xyz, dtype=np.float64)
    x, y, z = (_f64(xyz[:, d]) for d in range(3))
    q = _f64(q)
    c = _f64(centre)
    M = np.zeros(ncoef(p), dtype=np.complex128)
    lib().ora_p2m(p, _p(c), x.size, _p(x), _p(y), _p(z), _p(q), _p(M))
    return M


def m2m(p, O, Q):
    O = np.ascontiguousarray(O, dtype=np.complex128)
    out = np.zeros(ncoef(p), dtype=np.complex128)
    lib().ora_m2m(p, _p(O), _p(_f64(Q)), _p(out))
    return out


def m2l(p, O, Q, pl=None):
    pl = p if pl is None else pl
    O = np.ascontiguousarray(O, dtype=np.complex128)
    out = np.zeros(ncoef(pl), dtype=np.complex128)
    lib().ora_m2l(p, pl, _p(O), _p(_f64(Q)), _p(out))
    return out


def l2l(p, O, Q, pl=None):
    pl = p if pl is None else pl
    O = np.ascontiguousarray(O, dtype=np.complex128)
    out = np.zeros(ncoef(pl), dtype=np.complex128)
    lib().ora_l2l(p, pl, _p(O), _p(_f64(Q)), _p(out))
    return out


def l2p(p, L, centre, x):
    L = np.ascontiguousarray(L, dtype=np.complex128)
    phi = np.zeros(1)
    e = np.zeros(3)
    lib().ora_l2p(p, _p(L), _p(_f64(centre)), _p(_f64(x)), _p(phi), _p(e))
    return float(phi[0]), e


def m2p(p, M, centre, x):
    M = np.ascontiguousarray(M, dtype=np.complex128)
    phi = np.zeros(1)
    e = np.zeros(3)
    lib().ora_m2p(p, _p(M), _p(_f64(centre)), _p(_f64(x)), _p(phi), _p(e))
    return float(phi[0]), e


def mp_series(p, M, centre, x) -> float:
    M = np.ascontiguousarray(M, dtype=np.complex128)
    return float(lib().ora_mp_series(p, _p(M), _p(_f64(centre)), _p(_f64(x))))


def local_series(p, L, centre, x) -> float:
    L = np.ascontiguousarray(L, dtype=np.complex128)
    return float(lib().ora_local_series(p, _p(L), _p(_f64(centre)), _p(_f64(x))))


# ---------------------------------------------------------------- Cartesian expansions
def cart_count(p: int) -> int:
    """Coefficients of a Cartesian expansion of order p: multi-indices |k| <= p."""
    return int(lib().ora_cart_count(int(p)))


def cart_index(a: int, b: int, c: int) -> int:
    """Position of multi-index (a, b, c) in the graded order."""
    return int(lib().ora_cart_index(int(a), int(b), int(c)))


def cart_taylor(P: int, R) -> np.ndarray:
    """a_n(R) = (1/n!) d^n (1/|R|) for |n| <= P."""
    a = np.zeros(cart_count(P))
    lib().ora_cart_taylor(int(P), _p(_f64(R)), _p(a))
    return a


def cart_p2m(p, centre, xyz, q):
    xyz = np.asarray(xyz, dtype=np.float64)
    x, y, z = (_f64(xyz[:, d]) for d in range(3))
    M = np.zeros(cart_count(p))
    lib().ora_cart_p2m(int(p), _p(_f64(centre)), x.size, _p(x), _p(y), _p(z), _p(_f64(q)), _p(M))
    return M


def cart_m2m(p, M, d):
    """M re-centred by d = new centre - old centre."""
    out = np.zeros(cart_count(p))
    lib().ora_cart_m2m(int(p), _p(_f64(M)), _p(_f64(d)), _p(out))
    return out


def cart_m2l(p, M, R):
    """Local about t of the multipole M about s, R = t - s."""
    out = np.zeros(cart_count(p))
    lib().ora_cart_m2l(int(p), _p(_f64(M)), _p(_f64(R)), _p(out))
    return out


def cart_l2l(p, L, d):
    """L re-centred by d = new centre - old centre."""
    out = np.zeros(cart_count(p))
    lib().ora_cart_l2l(int(p), _p(_f64(L)), _p(_f64(d)), _p(out))
    return out


def cart_l2p(p, L, centre, x):
    phi = np.zeros(1)
    e = np.zeros(3)
    lib().ora_cart_l2p(int(p), _p(_f64(L)), _p(_f64(centre)), _p(_f64(x)), _p(phi), _p(e))
    return float(phi[0]), e


def cart_m2p(p, M, centre, x):
    phi = np.zeros(1)
    e = np.zeros(3)
    lib().ora_cart_m2p(int(p), _p(_f64(M)), _p(_f64(centre)), _p(_f64(x)), _p(phi), _p(e))
    return float(phi[0]), e


# ---------------------------------------------------------------- full method
class Tree:
    """Tree, lists and evaluation of one particle set (handle over the C oracle)."""

    def __init__(self, x, y, z, ncrit: int, n_targets: int = -1):
        """One set (n_targets = -1), or targets = the first n_targets points
        and sources = the rest, as two trees in one cube."""
        self.x, self.y, self.z = map(_f64, (x, y, z))
        self.n = self.x.size
        self.ncrit = int(ncrit)
        self.nt = int(n_targets)
        if self.nt < 0:
            self.h = lib().ora_build(self.n, _p(self.x), _p(self.y), _p(self.z), self.ncrit)
        else:
            self.h = lib().ora_build_ts(self.n, _p(self.x), _p(self.y), _p(self.z), self.nt, self.ncrit)
        self.ncell = int(lib().ora_ncells(self.h))
        self.p = None

    @classmethod
    def targets_sources(cls, targets, sources, ncrit: int):
        """Trees of distinct target and source points (each an (n, 3) array)."""
        t = np.asarray(targets, np.float64).reshape(-1, 3)
        s = np.asarray(sources, np.float64).reshape(-1, 3)
        a = np.concatenate([t, s])
        return cls(a[:, 0], a[:, 1], a[:, 2], ncrit, n_targets=t.shape[0])

    def __del__(self):
        h = getattr(self, "h", None)
        if h:
            lib().ora_free(h)
            self.h = None

    def keys(self):
        k = np.zeros(self.n, dtype=np.uint64)
        perm = np.zeros(self.n, dtype=np.int64)
        lib().ora_get_keys(self.h, _p(k), _p(perm))
        return k, perm

    def bbox(self):
        lo = np.zeros(3)
        side = np.zeros(1)
        lib().ora_get_bbox(self.h, _p(lo), _p(side))
        return lo, float(side[0])

    def cells(self) -> dict:
        c = self.ncell
        out = dict(level=np.zeros(c, np.int32), prefix=np.zeros(c, np.uint64),
                   begin=np.zeros(c, np.int32), end=np.zeros(c, np.int32),
                   parent=np.zeros(c, np.int32), first_child=np.zeros(c, np.int32),
                   nchild=np.zeros(c, np.int32), centre_h=np.zeros((c, 3), np.int64),
                   radius_h=np.zeros(c, np.int64), centre=np.zeros((c, 3)), radius=np.zeros(c))
        lib().ora_get_cells(self.h, *(_p(out[k]) for k in
                                      ("level", "prefix", "begin", "end", "parent", "first_child",
                                       "nchild", "centre_h", "radius_h", "centre", "radius")))
        return out

    def traverse(self, theta: float, policy: int = POLICY_FMM, costs=(0.0, 0.0, 0.0)):
        cst = _f64(costs)
        lib().ora_traverse(self.h, float(theta), int(policy), _p(cst))

    def traverse_table(self, theta: float, table):
        """Traversal whose accepted pairs take the kind given by a cost-model choice table."""
        self._table = np.ascontiguousarray(table, np.uint8).ravel()
        lib().ora_traverse_table(self.h, float(theta), _p(self._table))

    def lists(self) -> dict:
        out = {}
        for k in (M2L, M2P, P2P):
            m = int(lib().ora_list_size(self.h, k))
            t = np.zeros(m, np.int32)
            s = np.zeros(m, np.int32)
            if m:
                lib().ora_get_list(self.h, k, _p(t), _p(s))
            out[k] = (t, s)
        return out

    def evaluate(self, p: int, q):
        """(phi, E) of every particle; with separate sets q holds the sources'
        charges and the result is the targets'."""
        q = _f64(q)
        nout = self.n if self.nt < 0 else self.nt
        phi, ex, ey, ez = (np.zeros(nout) for _ in range(4))
        lib().ora_evaluate(self.h, int(p), _p(q), _p(phi), _p(ex), _p(ey), _p(ez))
        self.p = int(p)
        return phi, np.stack([ex, ey, ez], axis=1)

    def evaluate_cart(self, p: int, q):
        """As evaluate, with Cartesian (Taylor) expansions of order p."""
        q = _f64(q)
        nout = self.n if self.nt < 0 else self.nt
        phi, ex, ey, ez = (np.zeros(nout) for _ in range(4))
        lib().ora_evaluate_cart(self.h, int(p), _p(q), _p(phi), _p(ex), _p(ey), _p(ez))
        self.pc = int(p)
        return phi, np.stack([ex, ey, ez], axis=1)

    def expansions_cart(self):
        """Cartesian multipoles M_k = sum q (s - x)^k and locals of every cell
        (graded order, cart_index) after evaluate_cart."""
        K = cart_count(self.pc)
        M = np.zeros(self.ncell * K)
        L = np.zeros(self.ncell * K)
        lib().ora_get_expansions_cart(self.h, _p(M), _p(L))
        return M.reshape(self.ncell, K), L.reshape(self.ncell, K)

    def expansions(self):
        K = ncoef(self.p)
        M = np.zeros(self.ncell * K, dtype=np.complex128)
        L = np.zeros(self.ncell * K, dtype=np.complex128)
        lib().ora_get_expansions(self.h, _p(M), _p(L))
        return M.reshape(self.ncell, K), L.reshape(self.ncell, K)


def fmm(x, y, z, q, p, theta, ncrit, policy=POLICY_FMM, costs=(0.0, 0.0, 0.0)):
    """Whole oracle FMM: returns (phi, E, tree)."""
    t = Tree(x, y, z, ncrit)
    t.traverse(theta, policy, costs)
    phi, E = t.evaluate(p, q)
    return phi, E, t


def rel_l2(a, b) -> float:
    """Relative L2 error ||a - b|| / ||b|| over all components."""
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    return float(np.linalg.norm((a - b).ravel()) / np.linalg.norm(b.ravel()))


# ---------------------------------------------------------------- learned cost model
MLP_PARAMS = 4803


def mlp_forward(w, f):
    w = _f64(w)
    f = _f64(f)
    y = np.zeros(3)
    lib().ora_mlp_forward(_p(w), _p(f), _p(y))
    return y


def mlp_loss_grad(w, feat, kind, tgt):
    w = _f64(w)
    feat = _f64(feat)
    kind = np.ascontiguousarray(kind, np.int32)
    tgt = _f64(tgt)
    loss = np.zeros(1)
    g = np.zeros(MLP_PARAMS)
    lib().ora_mlp_loss_grad(_p(w), kind.size, _p(feat), _p(kind), _p(tgt), _p(loss), _p(g))
    return float(loss[0]), g


def mlp_table64(w, p, theta):
    """(choices, margin, bound), each [9,81,81,4]: the FP64 least-time kind over
    the quantised feature grid, the gap between the two least outputs, and a
    bound on the FP32 evaluation error of the outputs."""
    w = _f64(w)
    tab = np.zeros(9 * 81 * 81 * 4, np.uint8)
    mar = np.zeros(9 * 81 * 81 * 4)
    bnd = np.zeros(9 * 81 * 81 * 4)
    lib().ora_mlp_table64(_p(w), int(p), float(theta), _p(tab), _p(mar), _p(bnd))
    sh = (9, 81, 81, 4)
    return tab.reshape(sh), mar.reshape(sh), bnd.reshape(sh)
