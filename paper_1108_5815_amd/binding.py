"""ctypes binding of ``libfmm.so``; names follow the C entry points of ``include/fmm.h``.

The library must have been built (``python -m paper_1108_5815_amd.build``); a
missing library raises instead of falling back to anything else.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "libfmm.so")

POLICY_FMM, POLICY_TREECODE, POLICY_HYBRID_TIMED, POLICY_HYBRID_MLP = 0, 1, 2, 3
EXPANSION_SPHERICAL, EXPANSION_CARTESIAN, EXPANSION_AUTO = 0, 1, 2
M2L_CLASS_DENSE, M2L_CLASS_ROTATION, M2L_PAIR_DENSE, M2L_PAIR_ROTATION = 0, 1, 2, 3
PREC_FP32, PREC_SPLIT_BF16 = 0, 1
F32, F64 = 0, 1
LIST_M2L, LIST_M2P, LIST_P2P = 0, 1, 2
MLP_PARAMS = 4803
MLP_TABLE = 9 * 81 * 81 * 4

_STATUS = {0: "OK", 1: "INVALID_ARG", 2: "OUT_OF_MEMORY", 3: "DEVICE", 4: "STATE", 5: "UNSUPPORTED"}

_lib = None


def library_path() -> str:
    return _LIB_PATH


class FMMError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"{_STATUS.get(status, status)}: {message}")
        self.status = status


def lib():
    """Load libfmm.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB_PATH):
        raise RuntimeError(f"{_LIB_PATH} is missing: build it with `python -m paper_1108_5815_amd.build`")
    L = ctypes.CDLL(_LIB_PATH)
    vp, i32, i64, dbl = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_double
    sig = {
        "fmm_create": ([ctypes.POINTER(vp), ctypes.c_int, vp], ctypes.c_int),
        "fmm_destroy": ([vp], None),
        "fmm_last_error": ([vp], ctypes.c_char_p),
        "fmm_set_stream": ([vp, vp], ctypes.c_int),
        "fmm_build_tree": ([vp, i64, ctypes.c_int, vp, vp, vp, vp, i32], ctypes.c_int),
        "fmm_build_tree_batch": ([vp, i32, vp, ctypes.c_int, vp, vp, vp, vp, i32], ctypes.c_int),
        "fmm_build_tree_ts": ([vp, ctypes.c_int, i64, vp, vp, vp, i64, vp, vp, vp, vp, i32], ctypes.c_int),
        "fmm_evaluate_batch": ([vp, i32, vp, ctypes.c_int, vp, vp, vp, vp, i32, i32, dbl, i32, i32, i32,
                                vp, vp, vp, vp], ctypes.c_int),
        "fmm_get_bboxes": ([vp, i32, vp], ctypes.c_int),
        "fmm_traverse": ([vp, i32, dbl, i32], ctypes.c_int),
        "fmm_evaluate": ([vp, i32, i32, vp, vp, vp, vp], ctypes.c_int),
        "fmm_set_costs": ([vp, dbl, dbl, dbl], ctypes.c_int),
        "fmm_get_costs": ([vp, vp], ctypes.c_int),
        "fmm_tune": ([vp, i32, i32], ctypes.c_int),
        "fmm_get_sizes": ([vp, vp, vp, vp, vp], ctypes.c_int),
        "fmm_costmodel_train": ([vp, i32, dbl, i32, i32, ctypes.c_uint64, vp], ctypes.c_int),
        "fmm_costmodel_fit": ([vp, i32, vp, vp, vp, i32, dbl, ctypes.c_uint64, vp], ctypes.c_int),
        "fmm_costmodel_records": ([vp, i32, vp, vp, vp, vp], ctypes.c_int),
        "fmm_costmodel_get_weights": ([vp, vp], ctypes.c_int),
        "fmm_costmodel_set_weights": ([vp, vp], ctypes.c_int),
        "fmm_costmodel_loss_grad": ([vp, vp, i32, vp, vp, vp, vp, vp], ctypes.c_int),
        "fmm_costmodel_table": ([vp, i32, dbl, vp], ctypes.c_int),
        "fmm_get_bbox": ([vp, vp, vp], ctypes.c_int),
        "fmm_get_m2l_split": ([vp, vp, vp], ctypes.c_int),
        "fmm_get_work": ([vp, vp, vp], ctypes.c_int),
        "fmm_get_gemm_shape": ([vp, vp, vp, vp], ctypes.c_int),
        "fmm_get_keys": ([vp, vp, vp], ctypes.c_int),
        "fmm_get_cells": ([vp] + [vp] * 9, ctypes.c_int),
        "fmm_get_list": ([vp, i32, vp, vp], ctypes.c_int),
        "fmm_get_expansions": ([vp, vp, vp], ctypes.c_int),
        "fmm_get_timings": ([vp, vp, i32, vp], ctypes.c_int),
        "fmm_set_timing": ([vp, i32], ctypes.c_int),
        "fmm_set_overlap": ([vp, i32], ctypes.c_int),
        "fmm_autotune": ([vp, i32, i32], ctypes.c_int),
        "fmm_get_tile_config": ([vp, vp, vp], ctypes.c_int),
        "fmm_set_tile_config": ([vp, vp], ctypes.c_int),
        "fmm_set_allocator": ([vp, vp, vp, vp], ctypes.c_int),
        "fmm_costmodel_save": ([vp, ctypes.c_char_p], ctypes.c_int),
        "fmm_costmodel_load": ([vp, ctypes.c_char_p, i32, i32], ctypes.c_int),
        "fmm_m2l_slots": ([i32, dbl, vp, vp], ctypes.c_int),
        "fmm_set_expansion": ([vp, i32, i32], ctypes.c_int),
        "fmm_set_m2l_kernel": ([vp, i32], ctypes.c_int),
        "fmm_get_m2l_kernel": ([vp, vp], ctypes.c_int),
        "fmm_set_m2l_tile": ([vp, i32], ctypes.c_int),
        "fmm_validate": ([vp], ctypes.c_int),
        "fmm_get_m2l_tile": ([vp, vp], ctypes.c_int),
        "fmm_get_expansion": ([vp, vp], ctypes.c_int),
        "fmm_evaluate_noalloc": ([vp, i32, i32, vp, vp, vp, vp], ctypes.c_int),
    }
    for name, (args, res) in sig.items():
        f = getattr(L, name)
        f.argtypes = args
        f.restype = res
    _lib = L
    return L


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


ALLOC_FN = ctypes.CFUNCTYPE(ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p)
FREE_FN = ctypes.CFUNCTYPE(None, ctypes.c_void_p, ctypes.c_void_p)


def m2l_slots(p: int, theta: float):
    """(slots per octant class, 1 if the batched same-level GEMM is used) for (p, theta); no device needed."""
    j, b = ctypes.c_int32(), ctypes.c_int32()
    st = lib().fmm_m2l_slots(int(p), float(theta), ctypes.byref(j), ctypes.byref(b))
    if st != 0:
        raise FMMError(st, "fmm_m2l_slots failed")
    return j.value, b.value


class FMM:
    """One context of the library on one device and stream."""

    def __init__(self, device: int = 0, stream=None):
        import torch
        self._torch = torch
        self.device = int(device)
        if stream is None:
            stream = torch.cuda.current_stream(self.device).cuda_stream
        h = ctypes.c_void_p()
        st = lib().fmm_create(ctypes.byref(h), self.device, ctypes.c_void_p(stream))
        if st != 0:
            raise FMMError(st, "fmm_create failed")
        self.h = h
        self.n = 0
        self.p = None

    def close(self):
        if getattr(self, "h", None):
            lib().fmm_destroy(self.h)
            self.h = None
        self._hooks = None

    def set_allocator(self, alloc=None, free=None):
        """Route the context's device buffers through alloc(nbytes) -> int
        pointer (0 on failure) and free(ptr); None for both restores hipMalloc."""
        if alloc is None and free is None:
            self._ck(lib().fmm_set_allocator(self.h, None, None, None))
            return
        a = ALLOC_FN(lambda nbytes, user: int(alloc(int(nbytes))) or None)
        f = FREE_FN(lambda ptr, user: free(int(ptr)))
        self._ck(lib().fmm_set_allocator(self.h, ctypes.cast(a, ctypes.c_void_p), ctypes.cast(f, ctypes.c_void_p),
                                         None))
        # the library keeps the raw function pointers: hold the trampolines
        # (and any earlier ones, whose buffers are still released through them)
        if getattr(self, "_hooks", None) is None:
            self._hooks = []
        self._hooks.append((a, f))

    def use_torch_allocator(self):
        """Allocate the context's device buffers from torch's caching allocator
        on the context's device and the current stream."""
        t = self._torch
        dev = self.device
        self.set_allocator(lambda n: t.cuda.caching_allocator_alloc(n, dev),
                           lambda ptr: t.cuda.caching_allocator_delete(ptr))

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _ck(self, st):
        if st != 0:
            msg = lib().fmm_last_error(self.h)
            raise FMMError(st, msg.decode() if msg else "")

    # ------------------------------------------------------------ method
    def build_tree(self, x, y, z, q, ncrit: int):
        dt = self._check_inputs(x, y, z, q)
        self.n = x.numel()
        self.n_all = self.n
        self._ck(lib().fmm_build_tree(self.h, self.n, dt, x.data_ptr(), y.data_ptr(), z.data_ptr(),
                                      q.data_ptr(), int(ncrit)))

    def build_tree_ts(self, targets, sources, q, ncrit: int):
        """Target tree over targets = (tx, ty, tz) and source tree over
        sources = (sx, sy, sz) with charges q, in one cube; evaluate then
        returns the targets' potential and field."""
        tx, ty, tz = targets
        sx, sy, sz = sources
        dt = self._check_inputs(tx, ty, tz, tx)
        if sx.numel() > 0:
            if self._check_inputs(sx, sy, sz, q) != dt:
                raise ValueError("targets and sources must share one dtype")
        nt, ns = tx.numel(), sx.numel()
        self.n = nt
        self._ck(lib().fmm_build_tree_ts(self.h, dt, nt, tx.data_ptr(), ty.data_ptr(), tz.data_ptr(), ns,
                                         sx.data_ptr(), sy.data_ptr(), sz.data_ptr(), q.data_ptr(), int(ncrit)))
        self.n_all = nt + ns

    def _check_inputs(self, x, y, z, q):
        t = self._torch
        dt = x.dtype
        if dt not in (t.float32, t.float64):
            raise TypeError("positions must be float32 or float64")
        for a in (x, y, z, q):
            if a.dtype != dt or not a.is_cuda or not a.is_contiguous() or a.numel() != x.numel():
                raise ValueError("x, y, z, q must be contiguous device tensors of one dtype and length")
        return F64 if dt == t.float64 else F32

    @staticmethod
    def _offsets(offsets, n):
        off = np.ascontiguousarray(np.asarray(offsets, dtype=np.int64))
        if off.ndim != 1 or off.size < 2 or off[-1] != n:
            raise ValueError("offsets must hold n_inst + 1 values ending at the particle count")
        return off

    def build_tree_batch(self, offsets, x, y, z, q, ncrit: int):
        """Forest of independent instances: instance k owns particles
        [offsets[k], offsets[k+1])."""
        dt = self._check_inputs(x, y, z, q)
        off = self._offsets(offsets, x.numel())
        self.n = x.numel()
        self.n_all = self.n
        self._ck(lib().fmm_build_tree_batch(self.h, off.size - 1, _ptr(off), dt, x.data_ptr(), y.data_ptr(),
                                            z.data_ptr(), q.data_ptr(), int(ncrit)))
        self.n_inst = off.size - 1

    def evaluate_batch(self, offsets, x, y, z, q, ncrit: int, p: int, theta: float, policy: int = POLICY_FMM,
                       precision: int = PREC_FP32, out_dtype=None, out=None):
        """Build, traverse and evaluate a batch in one call; (phi, E) in input order."""
        t = self._torch
        dt = self._check_inputs(x, y, z, q)
        off = self._offsets(offsets, x.numel())
        n = x.numel()
        if out is None:
            od = t.float32 if out_dtype is None else out_dtype
            phi = t.empty(n, dtype=od, device=f"cuda:{self.device}")
            E = t.empty((3, n), dtype=od, device=f"cuda:{self.device}")
        else:
            phi, E = out
        od = F64 if phi.dtype == t.float64 else F32
        self.n = n
        self.n_all = n
        self._ck(lib().fmm_evaluate_batch(self.h, off.size - 1, _ptr(off), dt, x.data_ptr(), y.data_ptr(),
                                          z.data_ptr(), q.data_ptr(), int(ncrit), int(p), float(theta),
                                          int(policy), int(precision), od, phi.data_ptr(), E[0].data_ptr(),
                                          E[1].data_ptr(), E[2].data_ptr()))
        self.n_inst = off.size - 1
        self.p = int(p)
        return phi, E

    def bboxes(self, n_inst: int):
        out = np.zeros((n_inst, 4))
        self._ck(lib().fmm_get_bboxes(self.h, int(n_inst), _ptr(out)))
        return out

    def traverse(self, p: int, theta: float, policy: int = POLICY_FMM):
        self._ck(lib().fmm_traverse(self.h, int(p), float(theta), int(policy)))
        self.p = int(p)

    def evaluate(self, precision: int = PREC_FP32, out_dtype=None, out=None):
        """Returns (phi, E) as device tensors in the input particle order."""
        t = self._torch
        if out is None:
            od = t.float32 if out_dtype is None else out_dtype
            phi = t.empty(self.n, dtype=od, device=f"cuda:{self.device}")
            E = t.empty((3, self.n), dtype=od, device=f"cuda:{self.device}")
        else:
            phi, E = out
        od = F64 if phi.dtype == t.float64 else F32
        self._ck(lib().fmm_evaluate(self.h, int(precision), od, phi.data_ptr(), E[0].data_ptr(),
                                    E[1].data_ptr(), E[2].data_ptr()))
        return phi, E

    def evaluate_noalloc(self, precision: int = PREC_FP32, out=None):
        """fmm_evaluate on the library's fixed per-device work area (no
        allocation inside the call); the caller passes the outputs (phi, E)."""
        t = self._torch
        phi, E = out
        od = F64 if phi.dtype == t.float64 else F32
        self._ck(lib().fmm_evaluate_noalloc(self.h, int(precision), od, phi.data_ptr(), E[0].data_ptr(),
                                            E[1].data_ptr(), E[2].data_ptr()))
        return phi, E

    def set_expansion(self, expansion: int, auto_cartesian_max_p: int = 3):
        """Expansion family of the following traversals (EXPANSION_*); with
        EXPANSION_AUTO the Cartesian family is taken for p <= auto_cartesian_max_p."""
        self._ck(lib().fmm_set_expansion(self.h, int(expansion), int(auto_cartesian_max_p)))

    def set_m2l_kernel(self, kind: int):
        """Kernel of the M2L pairs outside the same-level GEMM (M2L_*)."""
        self._ck(lib().fmm_set_m2l_kernel(self.h, int(kind)))

    def m2l_kernel(self) -> int:
        v = ctypes.c_int32()
        self._ck(lib().fmm_get_m2l_kernel(self.h, ctypes.byref(v)))
        return v.value

    def set_m2l_tile(self, cols: int):
        """Targets per M2L GEMM tile (0, 64 or 128); used from the next traverse."""
        self._ck(lib().fmm_set_m2l_tile(self.h, int(cols)))

    def m2l_tile(self) -> int:
        v = ctypes.c_int32()
        self._ck(lib().fmm_get_m2l_tile(self.h, ctypes.byref(v)))
        return int(v.value)

    def validate(self):
        """Check the tree, lists and GEMM tables on host copies (raises FMMError)."""
        self._ck(lib().fmm_validate(self.h))

    def expansion(self) -> int:
        """Family of the last traversal (EXPANSION_SPHERICAL or EXPANSION_CARTESIAN)."""
        v = ctypes.c_int32()
        self._ck(lib().fmm_get_expansion(self.h, ctypes.byref(v)))
        return v.value

    def set_costs(self, c_m2l: float, c_m2p: float, c_p2p: float):
        self._ck(lib().fmm_set_costs(self.h, float(c_m2l), float(c_m2p), float(c_p2p)))

    def costs(self):
        out = np.zeros(3)
        self._ck(lib().fmm_get_costs(self.h, _ptr(out)))
        return out

    def tune(self, p: int, precision: int = PREC_FP32):
        self._ck(lib().fmm_tune(self.h, int(p), int(precision)))

    # ------------------------------------------------------------ learned cost model
    def costmodel_train(self, p: int, theta: float, epochs: int = 6000, seed: int = 1,
                        precision: int = PREC_FP32) -> float:
        loss = ctypes.c_double()
        self._ck(lib().fmm_costmodel_train(self.h, int(p), float(theta), int(precision), int(epochs), int(seed),
                                           ctypes.byref(loss)))
        return loss.value

    def costmodel_fit(self, features, kinds, targets, epochs=2000, lr=3e-3, seed=1) -> float:
        f = np.ascontiguousarray(features, np.float32)
        k = np.ascontiguousarray(kinds, np.int32)
        t = np.ascontiguousarray(targets, np.float32)
        loss = ctypes.c_double()
        self._ck(lib().fmm_costmodel_fit(self.h, k.size, _ptr(f), _ptr(k), _ptr(t), int(epochs), float(lr),
                                         int(seed), ctypes.byref(loss)))
        return loss.value

    def costmodel_records(self):
        cnt = ctypes.c_int32()
        self._ck(lib().fmm_costmodel_records(self.h, 0, ctypes.byref(cnt), None, None, None))
        m = cnt.value
        f = np.zeros((m, 6), np.float32)
        k = np.zeros(m, np.int32)
        t = np.zeros(m, np.float32)
        self._ck(lib().fmm_costmodel_records(self.h, m, ctypes.byref(cnt), _ptr(f), _ptr(k), _ptr(t)))
        return f, k, t

    def costmodel_weights(self):
        w = np.zeros(MLP_PARAMS, np.float32)
        self._ck(lib().fmm_costmodel_get_weights(self.h, _ptr(w)))
        return w

    def costmodel_set_weights(self, w):
        w = np.ascontiguousarray(w, np.float32)
        assert w.size == MLP_PARAMS
        self._ck(lib().fmm_costmodel_set_weights(self.h, _ptr(w)))

    def costmodel_loss_grad(self, w, features, kinds, targets):
        w = np.ascontiguousarray(w, np.float32)
        f = np.ascontiguousarray(features, np.float32)
        k = np.ascontiguousarray(kinds, np.int32)
        t = np.ascontiguousarray(targets, np.float32)
        loss = np.zeros(1, np.float32)
        g = np.zeros(MLP_PARAMS, np.float32)
        self._ck(lib().fmm_costmodel_loss_grad(self.h, _ptr(w), k.size, _ptr(f), _ptr(k), _ptr(t), _ptr(loss),
                                               _ptr(g)))
        return float(loss[0]), g

    def costmodel_save(self, path: str):
        self._ck(lib().fmm_costmodel_save(self.h, os.fsencode(path)))

    def costmodel_load(self, path: str, p: int = -1, precision: int = -1):
        """Load a saved model; p / precision = -1 accept any order / precision."""
        self._ck(lib().fmm_costmodel_load(self.h, os.fsencode(path), int(p), int(precision)))

    def costmodel_table(self, p: int, theta: float):
        tab = np.zeros(MLP_TABLE, np.uint8)
        self._ck(lib().fmm_costmodel_table(self.h, int(p), float(theta), _ptr(tab)))
        return tab.reshape(9, 81, 81, 4)

    def set_timing(self, on: bool):
        self._ck(lib().fmm_set_timing(self.h, 1 if on else 0))

    def set_overlap(self, schedule):
        """0 in order; 1 P2P concurrent from the start; 2 (default) P2P concurrent after the upward pass.
        True means 2, False 0."""
        sc = (2 if schedule else 0) if isinstance(schedule, bool) else int(schedule)
        self._ck(lib().fmm_set_overlap(self.h, sc))

    def autotune(self, precision: int = PREC_FP32, reps: int = 3):
        """Pick P2P tile shapes per leaf-size class, the M2L kernel kind and GEMM
        tile width, and the schedule, by timing."""
        self._ck(lib().fmm_autotune(self.h, int(precision), int(reps)))
        return self.tile_config()

    def tile_config(self) -> dict:
        tpl = np.zeros(4, np.int32)
        ov = ctypes.c_int32()
        self._ck(lib().fmm_get_tile_config(self.h, _ptr(tpl), ctypes.byref(ov)))
        return {"p2p_targets_per_lane": tpl.tolist(), "schedule": int(ov.value), "m2l_kernel": self.m2l_kernel(),
                "m2l_tile": self.m2l_tile()}

    def set_tile_config(self, tpl):
        a = np.ascontiguousarray(np.asarray(tpl, dtype=np.int32))
        self._ck(lib().fmm_set_tile_config(self.h, _ptr(a)))

    # ------------------------------------------------------------ introspection
    def sizes(self):
        v = [ctypes.c_int64() for _ in range(4)]
        self._ck(lib().fmm_get_sizes(self.h, *(ctypes.byref(a) for a in v)))
        return dict(cells=v[0].value, m2l=v[1].value, m2p=v[2].value, p2p=v[3].value)

    def m2l_split(self):
        a, b = ctypes.c_int64(), ctypes.c_int64()
        self._ck(lib().fmm_get_m2l_split(self.h, ctypes.byref(a), ctypes.byref(b)))
        return a.value, b.value

    def gemm_shape(self) -> dict:
        t, sl, a = ctypes.c_int64(), ctypes.c_int64(), ctypes.c_int64()
        self._ck(lib().fmm_get_gemm_shape(self.h, ctypes.byref(t), ctypes.byref(sl), ctypes.byref(a)))
        return {"tiles": t.value, "slots": sl.value, "active_slots": a.value}

    def work(self):
        a, b = ctypes.c_int64(), ctypes.c_int64()
        self._ck(lib().fmm_get_work(self.h, ctypes.byref(a), ctypes.byref(b)))
        return dict(p2p_particle_pairs=a.value, m2p_targets=b.value)

    def general_pairs(self) -> int:
        return self.m2l_split()[1]

    def bbox(self):
        lo = np.zeros(3)
        side = np.zeros(1)
        self._ck(lib().fmm_get_bbox(self.h, _ptr(lo), _ptr(side)))
        return lo, float(side[0])

    def keys(self):
        n = getattr(self, "n_all", self.n)
        k = np.zeros(n, dtype=np.uint64)
        perm = np.zeros(n, dtype=np.int32)
        self._ck(lib().fmm_get_keys(self.h, _ptr(k), _ptr(perm)))
        return k, perm

    def cells(self) -> dict:
        c = self.sizes()["cells"]
        out = dict(level=np.zeros(c, np.int32), prefix=np.zeros(c, np.uint64), begin=np.zeros(c, np.int32),
                   end=np.zeros(c, np.int32), parent=np.zeros(c, np.int32), first_child=np.zeros(c, np.int32),
                   nchild=np.zeros(c, np.int32), centre_h=np.zeros((c, 3), np.int32),
                   radius_h=np.zeros(c, np.int32))
        self._ck(lib().fmm_get_cells(self.h, *(_ptr(out[k]) for k in
                                              ("level", "prefix", "begin", "end", "parent", "first_child",
                                               "nchild", "centre_h", "radius_h"))))
        return out

    def list(self, kind: int):
        m = self.sizes()[{0: "m2l", 1: "m2p", 2: "p2p"}[kind]]
        t = np.zeros(m, np.int32)
        s = np.zeros(m, np.int32)
        self._ck(lib().fmm_get_list(self.h, int(kind), _ptr(t), _ptr(s)))
        return t, s

    def expansions(self):
        c = self.sizes()["cells"]
        p = self.p
        K = (p + 1) * (p + 2) * (p + 3) // 6 if self.expansion() == EXPANSION_CARTESIAN else (p + 1) ** 2
        M = np.zeros(c * K, np.float32)
        L = np.zeros(c * K, np.float32)
        self._ck(lib().fmm_get_expansions(self.h, _ptr(M), _ptr(L)))
        return M.reshape(c, K), L.reshape(c, K)

    def timings(self) -> dict:
        ms = np.zeros(12)
        cnt = ctypes.c_int32()
        self._ck(lib().fmm_get_timings(self.h, _ptr(ms), 12, ctypes.byref(cnt)))
        names = ["keys", "sort", "tree", "traverse", "lists", "p2m_m2m", "m2l_gemm", "m2l_general", "l2l", "p2p",
                 "far_final", "m2l_gemm_kernel"]
        return dict(zip(names, ms[:cnt.value].tolist()))
