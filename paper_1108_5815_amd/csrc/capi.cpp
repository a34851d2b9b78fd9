// capi.cpp -- context, device buffers and phase orchestration behind fmm.h.
//
// Phases (paper: tree construction, dual tree traversal, kernel evaluation;
// "Results"): build_tree = bounding cube -> Morton keys -> stable radix sort
// -> permuted points -> adaptive octree level by level -> geometry;
// traverse = frontier expansion level by level -> lists grouped by target ->
// batching of same-level M2L; evaluate = P2M -> M2M (bottom-up) -> M2L
// (GEMM + general) -> L2L (top-down) -> P2P -> L2P + M2P + final sum.
// Everything runs on the context's stream; the host reads back only sizes
// (one small copy per tree level and per traversal level).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <stdexcept>
#include <string>
#include <vector>

#include "../../include/fmm.h"
#include "fmm_internal.h"
#include "host_ops.h"

using namespace fmm;

namespace {

struct Buf {
    void* p = nullptr;
    size_t cap = 0;
    fmm_free_fn release = nullptr;  // the routine of the allocator that gave p (null: hipFree)
    void* user = nullptr;
};

enum { PH_KEYS, PH_SORT, PH_TREE, PH_TRAV, PH_LISTS, PH_UP, PH_M2L, PH_M2LG, PH_DOWN, PH_P2P, PH_FAR, PH_N };

}  // namespace

struct fmm_ctx_s {
    int device = 0;
    hipStream_t stream = nullptr;
    std::string err;
    std::vector<Buf*> bufs;
    // caller's device-memory hook (null: hipMalloc / hipFree)
    fmm_alloc_fn ualloc = nullptr;
    fmm_free_fn ufree = nullptr;
    void* uuser = nullptr;

    // timing
    bool timing = false;
    hipEvent_t ev[PH_N + 1] = {};
    double ms[PH_N] = {};
    hipEvent_t ev_gk[2] = {};  // around the same-level GEMM kernel itself
    double ms_gemm_kernel = 0;

    // near field on a second stream, concurrent with the far-field chain:
    // 0 in order, 1 from the start of the evaluation, 2 after the upward pass
    int schedule = 2;
    hipStream_t s2 = nullptr;
    hipEvent_t e_fork = nullptr, e_join = nullptr, e_p2p0 = nullptr, e_p2p1 = nullptr;

    // particles and tree
    int64_t n = 0;
    int dtype = 0;
    int32_t ncrit = 0;
    double lo[3] = {0, 0, 0}, side = 1;  // instance 0's bounding cube
    bool built = false, traversed = false;
    // targets != sources: the input's first n_targets particles (instance 0)
    // are the targets, the rest (instance 1) the sources, in one shared cube;
    // -1 when targets and sources are the same particles
    int64_t n_targets = -1;
    Buf ts_stage, tleaves;
    int32_t ntleaf = 0;
    // batch: instance offsets, frames, roots (cells [0, nroot))
    std::vector<int64_t> hseg;
    std::vector<Frame> frames;
    int32_t nroot = 0;
    Buf d_seg, d_bt, d_pb, d_box, d_frame, inst, bsort;
    // leaves grouped by P2P size class, and the tile shape (targets per lane) of each class
    Buf leaves_cls, lkey, lval, lkey2, lval2;
    int32_t leaf_cls[kLeafClasses + 1] = {};
    int p2p_tpl[kLeafClasses] = {4, 4, 4, 4};
    int32_t ncell = 0, nleaf = 0;
    std::vector<int32_t> lvl;  // cells of level L: [lvl[L], lvl[L+1])
    int tree_levels = 0;       // levels the last build needed (its first empty level)
    int gemm_nt = 0;           // M2L GEMM targets per tile asked for (0: the width's default)
    int trav_levels = 0;       // frontier levels the last traversal needed
    int64_t trav_cap[4] = {0, 0, 0, 0};  // pair capacities of the three lists and the frontier
    Buf keys, keys2, idx, idx2, pts, ws, small;
    Buf c_begin, c_end, c_parent, c_child, c_nchild, c_level, c_prefix, c_geo, c_ctr, leaves, tmp1, tmp2;

    // expansion family: requested (FMM_EXPANSION_*), the order up to which
    // FMM_EXPANSION_AUTO takes the Cartesian family, and the family of the
    // last traversal (kFamilySpherical or kFamilyCartesian)
    int expansion = 0, auto_cart_max_p = 3, fam = kFamilySpherical;
    HostTables ht_cart;
    int tables_p = -1, tables_fam = -1;

    // traversal
    int p = -1;
    double theta = 0;
    int policy = 0;
    double costs[3] = {0, 0, 0};
    bool costs_set = false;
    Buf fr0, fr1, cnt, off4;
    Buf raw[3], tgt[3], src[3], off[3];
    int64_t nlist[3] = {0, 0, 0};
    Buf tgt2, src2;

    // same-level M2L batching
    M2LPlan plan;
    Buf d_slot, d_offid, d_T, d_Thi, d_Tlo;
    bool plan_bf16 = false;
    Buf inner, leafpos;  // non-leaf cells in cell order; leaves before each cell
    Buf m2pflag;         // per leaf: cell-particle sources on the leaf or an ancestor
    Buf m2lslot;         // per cell-cell pair: its GEMM slot or -1
    Buf tbounds;         // tree build: octant boundaries of the cells of a level
    Buf has_fast, rkey, rval, rkey2, rval2, rowof, gather, gathercol, gtg, gsr, goff, tact, tnact, m2l_part, Msplit, nbucket, kinds;
    // pairs outside the same-level tables, batched by class
    ClsPlan cp;
    Buf ckey, ckey2, cval, cval2, chead, choff, cstart, cpos, csrcs, cnt_t, ctbase, ctile, cT, cskip, cls_part;
    bool m2l_sorted = false;
    GemmPlan gp{};
    int ntiles = 0;
    int64_t nrows = 0;
    int64_t ngeneral = 0;
    bool gemm_on = false;

    // operator tables
    HostTables ht;
    Buf d_m2m, d_l2l, d_w, d_g, d_h, d_rc, d_wrot;
    // M2L of the cell pairs outside the same-level GEMM (FMM_M2L_*)
    int m2l_kind = 0;

    // learned cost model: weights, Adam moments, training records, choice table
    Buf d_mlp, d_mlp_m, d_mlp_v, d_grad, d_grad_rec, d_loss_rec, d_feat, d_kind, d_tgt, d_table;
    bool mlp_ready = false;
    // what the model was trained for (-1 / NaN where unknown)
    int cm_p = -1, cm_precision = -1, cm_records = 0;
    double cm_theta = -1, cm_loss = NAN, cm_seconds = NAN;
    int mlp_version = 0, table_version = -1, table_p = -1, costs_version = 0, table_costs_version = -1;
    double table_theta = -1;
    std::vector<float> rec_feat, rec_tgt;
    std::vector<int32_t> rec_kind;

    // expansions and near-field partials
    Buf M, L, nearb;

    // kernel pre-calculation inputs/outputs
    Buf tune_pts, tune_out, at_out, d_lvl, d_trav;

    // pinned host staging
    void* host = nullptr;
    // per-level counts written by the scan kernels straight into mapped,
    // coherent host memory (the host only synchronises: no copy launch)

    fmm_ctx_s() {
        Buf* all[] = {&keys, &keys2, &idx, &idx2, &pts, &ws, &small, &c_begin, &c_end, &c_parent, &c_child,
                      &c_nchild, &c_level, &c_prefix, &c_geo, &c_ctr, &leaves, &tmp1, &tmp2, &fr0, &fr1,
                      &cnt, &off4, &raw[0], &raw[1], &raw[2], &tgt[0], &tgt[1], &tgt[2], &src[0], &src[1],
                      &src[2], &off[0], &off[1], &off[2], &tgt2, &src2, &d_slot, &d_offid, &d_T, &has_fast,
                      &rkey, &rval, &rkey2, &rval2, &rowof, &gather, &gathercol, &gtg, &gsr, &goff, &d_m2m, &d_l2l, &d_w, &d_g,
                      &d_h, &d_rc, &d_mlp, &M, &L, &nearb, &tune_pts, &tune_out, &d_mlp_m, &d_mlp_v,
                      &d_grad, &d_grad_rec, &d_loss_rec, &d_feat, &d_kind, &d_tgt, &d_table, &d_Thi, &d_Tlo,
                      &d_seg, &d_bt, &d_pb, &d_box, &d_frame, &inst, &bsort, &tact, &tnact,
                      &leaves_cls, &inner, &leafpos, &m2pflag, &m2lslot, &tbounds, &lkey, &lval, &lkey2, &lval2, &at_out, &m2l_part, &Msplit, &nbucket, &kinds, &ckey, &ckey2, &cval, &cval2,
                      &chead, &choff, &cstart, &cpos, &csrcs, &cnt_t, &ctbase, &ctile, &cT, &cskip, &cls_part,
                      &ts_stage, &tleaves, &d_wrot, &d_lvl, &d_trav};
        for (Buf* b : all) bufs.push_back(b);
    }
};

namespace {

struct Fail {
    fmm_status st;
    std::string msg;
};

[[noreturn]] void fail(fmm_status st, const std::string& m) { throw Fail{st, m}; }

void ck(hipError_t e, const char* what) {
    if (e != hipSuccess) fail(FMM_ERR_DEVICE, std::string(what) + ": " + hipGetErrorString(e));
}

void check_launch(const char* what) { ck(hipGetLastError(), what); }

// device memory through the caller's hook, or hipMalloc
void dev_alloc(fmm_ctx c, Buf& b, size_t nb) {
    void* np = nullptr;
    if (c->ualloc) {
        np = c->ualloc(nb, c->uuser);
        if (!np) fail(FMM_ERR_OUT_OF_MEMORY, "the allocator hook returned no memory for " + std::to_string(nb) + " bytes");
        b.release = c->ufree;
        b.user = c->uuser;
    } else {
        hipError_t e = hipMalloc(&np, nb);
        if (e != hipSuccess) {
            (void)hipGetLastError();
            fail(FMM_ERR_OUT_OF_MEMORY, "device allocation of " + std::to_string(nb) + " bytes failed");
        }
        b.release = nullptr;
        b.user = nullptr;
    }
    b.p = np;
    b.cap = nb;
}

// release a buffer with the routine that allocated it (the stream must have passed every use)
void dev_release(Buf& b) {
    if (b.p) {
        if (b.release) b.release(b.p, b.user);
        else (void)hipFree(b.p);
    }
    b.p = nullptr;
    b.cap = 0;
    b.release = nullptr;
    b.user = nullptr;
}

// grow-only device buffer; contents are not preserved
template <class T>
T* need(fmm_ctx c, Buf& b, size_t count) {
    size_t bytes = std::max<size_t>(count * sizeof(T), 256);
    if (b.cap >= bytes) return (T*)b.p;
    if (b.p) {
        ck(hipStreamSynchronize(c->stream), "sync");
        dev_release(b);
    }
    dev_alloc(c, b, bytes + bytes / 4);
    return (T*)b.p;
}

// grow-only buffer that keeps its first `keep` bytes
template <class T>
T* need_keep(fmm_ctx c, Buf& b, size_t count, size_t keep_count) {
    size_t bytes = std::max<size_t>(count * sizeof(T), 256);
    if (b.cap >= bytes) return (T*)b.p;
    Buf nbuf;
    dev_alloc(c, nbuf, bytes + bytes / 2);
    if (b.p && keep_count)
        ck(hipMemcpyAsync(nbuf.p, b.p, keep_count * sizeof(T), hipMemcpyDeviceToDevice, c->stream), "copy");
    if (b.p) {
        ck(hipStreamSynchronize(c->stream), "sync");
        dev_release(b);
    }
    b = nbuf;
    return (T*)b.p;
}

void* host_stage(fmm_ctx c) {
    if (!c->host) ck(hipHostMalloc(&c->host, 1 << 16, hipHostMallocDefault), "hipHostMalloc");
    return c->host;
}

template <class T>
void to_host(fmm_ctx c, T* dst, const void* src, size_t count) {
    if (count == 0) return;
    ck(hipMemcpyAsync(dst, src, count * sizeof(T), hipMemcpyDeviceToHost, c->stream), "D2H");
    ck(hipStreamSynchronize(c->stream), "sync");
}

template <class T>
void to_dev(fmm_ctx c, void* dst, const T* src, size_t count) {
    if (count == 0) return;
    ck(hipMemcpyAsync(dst, src, count * sizeof(T), hipMemcpyHostToDevice, c->stream), "H2D");
    ck(hipStreamSynchronize(c->stream), "sync");
}

CellArrays cells_of(fmm_ctx c) {
    CellArrays a;
    a.begin = (int32_t*)c->c_begin.p;
    a.end = (int32_t*)c->c_end.p;
    a.parent = (int32_t*)c->c_parent.p;
    a.child = (int32_t*)c->c_child.p;
    a.nchild = (int32_t*)c->c_nchild.p;
    a.level = (int32_t*)c->c_level.p;
    a.prefix = (uint64_t*)c->c_prefix.p;
    a.geo = (int4*)c->c_geo.p;
    a.ctr = (double4*)c->c_ctr.p;
    return a;
}

void ensure_cells(fmm_ctx c, size_t count, size_t keep) {
    need_keep<int32_t>(c, c->c_begin, count, keep);
    need_keep<int32_t>(c, c->c_end, count, keep);
    need_keep<int32_t>(c, c->c_parent, count, keep);
    need_keep<int32_t>(c, c->c_child, count, keep);
    need_keep<int32_t>(c, c->c_nchild, count, keep);
    need_keep<int32_t>(c, c->c_level, count, keep);
    need_keep<uint64_t>(c, c->c_prefix, count, keep);
}

void mark(fmm_ctx c, int ph) {
    if (c->timing) ck(hipEventRecord(c->ev[ph], c->stream), "event");
}

Tables tables_of(fmm_ctx c) {
    Tables t;
    t.m2m = (const float*)c->d_m2m.p;
    t.l2l = (const float*)c->d_l2l.p;
    t.wm2l = (const float*)c->d_w.p;
    t.gl2p = (const float*)c->d_g.p;
    t.hm2p = (const float*)c->d_h.p;
    t.rcoef = (const float*)c->d_rc.p;
    t.wax = (const float*)c->d_wrot.p;
    return t;
}

// coefficients per cell and row stride of the current family and order
int c_k(fmm_ctx c) { return c->fam == kFamilyCartesian ? (c->p + 1) * (c->p + 2) * (c->p + 3) / 6 : ncoef(c->p); }
int c_kp(fmm_ctx c) { return c->fam == kFamilyCartesian ? kpad_cart(c->p) : kpad(c->p); }

template <class F>
fmm_status guarded(fmm_ctx c, F f) {
    if (!c) return FMM_ERR_INVALID_ARG;
    c->err.clear();
    try {
        ck(hipSetDevice(c->device), "hipSetDevice");
        f();
        return FMM_OK;
    } catch (const Fail& e) {
        c->err = e.msg;
        return e.st;
    } catch (const std::bad_alloc&) {
        c->err = "host allocation failed";
        return FMM_ERR_OUT_OF_MEMORY;
    } catch (const std::exception& e) {
        c->err = e.what();
        return FMM_ERR_INVALID_ARG;
    }
}

int bits_for(int64_t v) {
    int b = 1;
    while (b < 32 && ((int64_t)1 << b) <= v) b++;
    return b;
}

// ------------------------------------------------------------------ build
// Build the forest of a batch: instance k owns input particles
// [hseg[k], hseg[k+1]) (host array of nseg + 1 offsets); a single problem is
// the batch of one.  Each instance gets its own bounding cube, keys relative
// to it, and its own root; the sort orders by (instance, key, input index).
void build_forest_impl(fmm_ctx c, int32_t nseg, const int64_t* hseg, int dtype, const void* x, const void* y,
                       const void* z, const void* q, int32_t ncrit, bool shared_frame = false) {
    if (nseg < 1 || !hseg) fail(FMM_ERR_INVALID_ARG, "need at least one instance");
    if (hseg[0] != 0) fail(FMM_ERR_INVALID_ARG, "offsets[0] must be 0");
    for (int32_t k = 0; k < nseg; k++)
        if (hseg[k + 1] < hseg[k]) fail(FMM_ERR_INVALID_ARG, "offsets must be non-decreasing");
    const int64_t n = hseg[nseg];
    if (n < 0 || n >= ((int64_t)1 << 31)) fail(FMM_ERR_INVALID_ARG, "n out of range");
    if (ncrit < 1) fail(FMM_ERR_INVALID_ARG, "ncrit must be >= 1");
    if (dtype != FMM_F32 && dtype != FMM_F64) fail(FMM_ERR_INVALID_ARG, "dtype must be FMM_F32 or FMM_F64");
    if (n > 0 && (!x || !y || !z || !q)) fail(FMM_ERR_INVALID_ARG, "null input pointer");
    c->built = false;
    c->traversed = false;
    c->n_targets = -1;
    c->ntleaf = 0;
    c->n = n;
    c->dtype = dtype;
    c->ncrit = ncrit;
    c->ncell = 0;
    c->nleaf = 0;
    c->nroot = 0;
    c->lvl.assign(1, 0);
    c->hseg.assign(hseg, hseg + nseg + 1);
    c->frames.assign(nseg, Frame{0, 0, 0, 1, 2097152.0, 1.0 / 4194304.0, 0, 0});
    c->lo[0] = c->lo[1] = c->lo[2] = 0;
    c->side = 1;
    if (n == 0) {
        c->built = true;
        return;
    }
    hipStream_t s = c->stream;
    mark(c, PH_KEYS);
    // bounding cube per instance: blocks of at most `chunk` particles
    const int64_t chunk = std::max<int64_t>(4096, (n + 1023) / 1024);
    std::vector<int64_t> bt;
    std::vector<int32_t> pb(nseg + 1, 0);
    for (int32_t k = 0; k < nseg; k++) {
        pb[k] = (int32_t)(bt.size() / 2);
        for (int64_t i = hseg[k]; i < hseg[k + 1]; i += chunk) {
            bt.push_back(i);
            bt.push_back(std::min(i + chunk, hseg[k + 1]));
        }
    }
    pb[nseg] = (int32_t)(bt.size() / 2);
    const int nblk = pb[nseg];
    int64_t* dseg = need<int64_t>(c, c->d_seg, nseg + 1);
    to_dev(c, dseg, hseg, nseg + 1);
    int64_t* dbt = need<int64_t>(c, c->d_bt, bt.size());
    to_dev(c, dbt, bt.data(), bt.size());
    int32_t* dpb = need<int32_t>(c, c->d_pb, nseg + 1);
    to_dev(c, dpb, pb.data(), nseg + 1);
    size_t wsb = std::max({sort_ws_bytes(n), scan_ws_bytes(n), (size_t)nblk * 6 * sizeof(double) + 256});
    void* ws = need<char>(c, c->ws, wsb);
    double* d6 = need<double>(c, c->small, 32);
    uint32_t* dbad = (uint32_t*)(d6 + 8);
    double* box = need<double>(c, c->d_box, (size_t)nseg * 6);
    bbox(x, y, z, dtype, dbt, nblk, dpb, nseg, (double*)ws, box, dbad, s);
    check_launch("bbox");
    std::vector<double> hb((size_t)nseg * 6);
    to_host<double>(c, hb.data(), box, hb.size());
    uint32_t bad = 0;
    to_host<uint32_t>(c, &bad, dbad, 1);
    if (bad) fail(FMM_ERR_INVALID_ARG, "non-finite coordinate in input");
    if (shared_frame) {
        // one cube around every instance's points: their cells then compare geometrically
        bool any = false;
        double lo[3] = {0, 0, 0}, hi[3] = {0, 0, 0};
        for (int32_t k = 0; k < nseg; k++) {
            if (hseg[k + 1] == hseg[k]) continue;
            for (int d = 0; d < 3; d++) {
                lo[d] = any ? std::min(lo[d], hb[k * 6 + d]) : hb[k * 6 + d];
                hi[d] = any ? std::max(hi[d], hb[k * 6 + 3 + d]) : hb[k * 6 + 3 + d];
            }
            any = true;
        }
        for (int32_t k = 0; k < nseg; k++)
            for (int d = 0; d < 3; d++) {
                hb[k * 6 + d] = lo[d];
                hb[k * 6 + 3 + d] = hi[d];
            }
    }
    for (int32_t k = 0; k < nseg; k++) {
        if (hseg[k + 1] == hseg[k]) continue;
        Frame& f = c->frames[k];
        double sd = 0;
        for (int d = 0; d < 3; d++) {
            double e = hb[k * 6 + 3 + d] - hb[k * 6 + d];
            if (e > sd) sd = e;
        }
        if (sd == 0.0) sd = 1.0;
        f.lox = hb[k * 6 + 0];
        f.loy = hb[k * 6 + 1];
        f.loz = hb[k * 6 + 2];
        f.side = sd;
        f.scale = 2097152.0 / sd;
        f.h = sd / 4194304.0;
    }
    {
        const Frame& f0 = c->frames[0];
        c->lo[0] = f0.lox;
        c->lo[1] = f0.loy;
        c->lo[2] = f0.loz;
        c->side = f0.side;
    }
    Frame* dfr = need<Frame>(c, c->d_frame, nseg);
    to_dev(c, dfr, c->frames.data(), nseg);
    uint64_t* keys = need<uint64_t>(c, c->keys, n);
    uint64_t* keys2 = need<uint64_t>(c, c->keys2, n);
    uint32_t* idx = need<uint32_t>(c, c->idx, n);
    uint32_t* idx2 = need<uint32_t>(c, c->idx2, n);
    uint32_t* inst = nseg > 1 ? need<uint32_t>(c, c->inst, n) : nullptr;
    morton_keys(x, y, z, dtype, n, dseg, nseg, dfr, keys, idx, inst, s);
    check_launch("morton");
    mark(c, PH_SORT);
    sort_u64(keys, idx, keys2, idx2, n, 0, 63, ws, s);
    if (nseg > 1) {
        uint32_t* ik = need<uint32_t>(c, c->bsort, 4 * (size_t)n);
        uint32_t *iv = ik + n, *ik2 = ik + 2 * n, *iv2 = ik + 3 * n;
        inst_keys(idx, inst, n, ik, iv, s);
        sort_u32(ik, iv, ik2, iv2, n, 0, bits_for(nseg - 1), ws, s);
        gather_sorted(keys, idx, iv, n, keys2, idx2, s);
        std::swap(c->keys, c->keys2);
        std::swap(c->idx, c->idx2);
        keys = (uint64_t*)c->keys.p;
        idx = (uint32_t*)c->idx.p;
    }
    check_launch("sort");
    float4* pts = need<float4>(c, c->pts, n);
    permute_points(x, y, z, q, dtype, n, idx, pts, s);
    check_launch("permute");
    mark(c, PH_TREE);
    // one root per non-empty instance, in instance order
    std::vector<int32_t> rb, re;
    for (int32_t k = 0; k < nseg; k++)
        if (hseg[k + 1] > hseg[k]) {
            rb.push_back((int32_t)hseg[k]);
            re.push_back((int32_t)hseg[k + 1]);
        }
    const int32_t nroot = (int32_t)rb.size();
    c->nroot = nroot;
    // Levels run back to back on the device: each level's bounds and its
    // count of new cells stay in device memory, and the host reads them once
    // per window of levels (as many as the previous build needed, else 6).
    // A level that would pass the cell capacity stops the tree; the arrays
    // then grow and the build runs again.
    size_t cap = std::max<size_t>(c->c_begin.cap / sizeof(int32_t),
                                  (size_t)std::max<int64_t>(1024, 4 * n / std::max(ncrit, 1) + 1024) + nroot);
    int32_t* dl = need<int32_t>(c, c->d_lvl, kMaxLevel + 8);  // level starts [0, kMaxLevel + 3), new-cell count, overflow
    uint32_t* dnnew = (uint32_t*)(dl + kMaxLevel + 4);
    uint32_t* dovf = dnnew + 1;
    std::vector<int32_t> hl(kMaxLevel + 8, 0);
    if (scan_dev_ws_bytes() > c->ws.cap) {
        ws = need<char>(c, c->ws, scan_dev_ws_bytes());
        d6 = (double*)c->small.p;
    }
    int lstar = 0;  // first empty level
    for (;;) {
        if (cap > (size_t)INT32_MAX) fail(FMM_ERR_UNSUPPORTED, "more than 2^31 cells");
        ensure_cells(c, cap, 0);
        {
            std::vector<int32_t> neg(nroot, -1), zero(nroot, 0);
            std::vector<uint64_t> z64(nroot, 0);
            to_dev(c, c->c_begin.p, rb.data(), nroot);
            to_dev(c, c->c_end.p, re.data(), nroot);
            to_dev(c, c->c_parent.p, neg.data(), nroot);
            to_dev(c, c->c_level.p, zero.data(), nroot);
            to_dev(c, c->c_child.p, neg.data(), nroot);
            to_dev(c, c->c_nchild.p, zero.data(), nroot);
            to_dev(c, c->c_prefix.p, z64.data(), nroot);
            std::vector<int32_t> h0(kMaxLevel + 8, 0);
            h0[1] = nroot;
            to_dev(c, dl, h0.data(), h0.size());
        }
        uint32_t* nsplit = need<uint32_t>(c, c->tmp1, cap + 1);
        uint32_t* choff = need<uint32_t>(c, c->tmp2, cap + 1);
        int32_t* tbnd = need<int32_t>(c, c->tbounds, cap * 7 + 1);
        const CellArrays ca = cells_of(c);
        int window = c->tree_levels > 0 ? c->tree_levels : 6;
        int L = 0;
        lstar = 0;
        while (lstar == 0) {
            for (int k = 0; k < window && L <= kMaxLevel; k++, L++) {
                tree_count(keys, ca, dl, L, ncrit, nsplit, tbnd, (int32_t)cap, s);
                scan_u32_dev(nsplit, choff, dnnew, DevCount{(const uint32_t*)(dl + L + 1), (const uint32_t*)(dl + L)},
                             c->ws.p, s);
                tree_emit(ca, dl, L, nsplit, choff, dnnew, tbnd, (int32_t)cap, dovf, s);
            }
            check_launch("tree levels");
            to_host<int32_t>(c, hl.data(), dl, hl.size());
            if (hl[kMaxLevel + 5] != 0) break;  // overflow
            // levels [0, L) are done; the new cells of the last are [hl[L], hl[L + 1])
            if (hl[L + 1] == hl[L]) {
                lstar = 1;
                while (hl[lstar + 1] != hl[lstar]) lstar++;
            }
            window = 6;
        }
        if (lstar > 0) break;
        cap *= 2;
    }
    c->tree_levels = lstar;
    c->lvl.assign(hl.begin(), hl.begin() + lstar + 1);
    const int32_t total = hl[lstar];
    c->ncell = total;
    need<int4>(c, c->c_geo, total);
    need<double4>(c, c->c_ctr, total);
    cell_geometry(cells_of(c), total, (const int64_t*)c->d_seg.p, nseg, (const Frame*)c->d_frame.p, s);
    check_launch("geometry");
    // leaves in cell order
    uint32_t* flag = need<uint32_t>(c, c->tmp1, total + 1);
    uint32_t* pos = need<uint32_t>(c, c->leafpos, total + 1);  // kept: the level translations read it
    if (scan_ws_bytes(total) > c->ws.cap) {
        ws = need<char>(c, c->ws, scan_ws_bytes(total));
        d6 = (double*)c->small.p;
    }
    leaf_flags(cells_of(c), total, flag, s);
    scan_u32(flag, pos, (uint32_t*)(d6 + 12), total, ws, s);
    int32_t* lv = need<int32_t>(c, c->leaves, total);
    int32_t* inr = need<int32_t>(c, c->inner, total);
    leaf_write(cells_of(c), total, pos, lv, inr, s);
    check_launch("leaves");
    uint32_t* hh = (uint32_t*)host_stage(c);
    to_host<uint32_t>(c, hh, d6 + 12, 1);
    c->nleaf = (int32_t)hh[0];
    {
        // leaves grouped by P2P size class (cell order within a class)
        const int32_t nl = c->nleaf;
        uint32_t* lk = need<uint32_t>(c, c->lkey, nl);
        uint32_t* lvv = need<uint32_t>(c, c->lval, nl);
        uint32_t* lk2 = need<uint32_t>(c, c->lkey2, nl);
        uint32_t* lv2 = need<uint32_t>(c, c->lval2, nl);
        if (sort_ws_bytes(nl) > c->ws.cap) {
            ws = need<char>(c, c->ws, sort_ws_bytes(nl));
            d6 = (double*)c->small.p;
        }
        leaf_class_keys(cells_of(c), lv, nl, lk, lvv, s);
        sort_u32(lk, lvv, lk2, lv2, nl, 0, 8, ws, s);
        int32_t* d9 = (int32_t*)(d6 + 20);
        class_bounds(lk, nl, 0, d9, s);
        check_launch("leaf classes");
        int32_t h9[9];
        to_host<int32_t>(c, h9, d9, 9);
        for (int k = 0; k <= kLeafClasses; k++) c->leaf_cls[k] = h9[k];
        int32_t* lc = need<int32_t>(c, c->leaves_cls, nl);
        ck(hipMemcpyAsync(lc, lvv, (size_t)nl * sizeof(int32_t), hipMemcpyDeviceToDevice, s), "copy");
    }
    mark(c, PH_TRAV);
    c->built = true;
}

void build_tree_impl(fmm_ctx c, int64_t n, int dtype, const void* x, const void* y, const void* z,
                     const void* q, int32_t ncrit) {
    if (n < 0 || n >= ((int64_t)1 << 31)) fail(FMM_ERR_INVALID_ARG, "n out of range");
    const int64_t seg[2] = {0, n};
    build_forest_impl(c, 1, seg, dtype, x, y, z, q, ncrit);
}

// ------------------------------------------------------------------ traverse
void upload_tables(fmm_ctx c, int p) {
    HostTables& t = c->fam == kFamilyCartesian ? c->ht_cart : c->ht;
    if (t.p != p) {
        if (c->fam == kFamilyCartesian) build_tables_cart(p, t);
        else build_tables(p, t);
    }
    // the device tables hold one family at a time
    if (c->tables_p == p && c->tables_fam == c->fam) return;
    to_dev(c, need<float>(c, c->d_m2m, t.m2m.size()), t.m2m.data(), t.m2m.size());
    to_dev(c, need<float>(c, c->d_l2l, t.l2l.size()), t.l2l.data(), t.l2l.size());
    to_dev(c, need<float>(c, c->d_w, t.wm2l.size()), t.wm2l.data(), t.wm2l.size());
    to_dev(c, need<float>(c, c->d_g, t.gl2p.size()), t.gl2p.data(), t.gl2p.size());
    to_dev(c, need<float>(c, c->d_h, t.hm2p.size()), t.hm2p.data(), t.hm2p.size());
    to_dev(c, need<float>(c, c->d_rc, t.rcoef.size()), t.rcoef.data(), t.rcoef.size());
    to_dev(c, need<float>(c, c->d_wrot, t.wrot.size()), t.wrot.data(), t.wrot.size());
    c->tables_p = p;
    c->tables_fam = c->fam;
}

void upload_plan(fmm_ctx c, int p, double theta) {
    const bool cart = c->fam == kFamilyCartesian;
    if (c->plan.p == p && c->plan.theta == theta && c->plan.cartesian == cart) return;
    build_m2l_plan(p, theta, c->plan, cart);
    M2LPlan& pl = c->plan;
    to_dev(c, need<int32_t>(c, c->d_slot, pl.slot_of.size()), pl.slot_of.data(), pl.slot_of.size());
    to_dev(c, need<int32_t>(c, c->d_offid, pl.offid.size()), pl.offid.data(), pl.offid.size());
    to_dev(c, need<float>(c, c->d_T, pl.T.size()), pl.T.data(), pl.T.size());
    c->plan_bf16 = false;
}

// split-BF16 copies of the same-level operators, made on first use
void upload_plan_bf16(fmm_ctx c) {
    if (c->plan_bf16) return;
    std::vector<uint16_t> hi, lo;
    split_bf16_kblocked(c->plan.T, c->plan.offsets.size(), c->plan.cartesian ? kpad_cart(c->plan.p) : kpad(c->plan.p),
                        hi, lo);
    to_dev(c, need<uint16_t>(c, c->d_Thi, hi.size()), hi.data(), hi.size());
    to_dev(c, need<uint16_t>(c, c->d_Tlo, lo.size()), lo.data(), lo.size());
    c->plan_bf16 = true;
}

// The M2L pairs outside the same-level tables (CSR by target in gtg / gsr /
// goff) keyed by class, sorted, and given one operator per class.
void build_classes(fmm_ctx c, int p) {
    c->cp = ClsPlan{};
    // the per-pair kinds take every pair outside the same-level GEMM one by one
    if (c->fam == kFamilySpherical && (c->m2l_kind == FMM_M2L_PAIR_DENSE || c->m2l_kind == FMM_M2L_PAIR_ROTATION))
        return;
    const int64_t ng = c->ngeneral;
    const int KP = c_kp(c);
    const int NT = cls_tile_cols(KP);
    if (ng <= 0 || NT <= 0) return;
    hipStream_t s = c->stream;
    CellArrays ca = cells_of(c);
    uint64_t* keys = need<uint64_t>(c, c->ckey, ng);
    uint64_t* keys2 = need<uint64_t>(c, c->ckey2, ng);
    uint32_t* cv = need<uint32_t>(c, c->cval, ng);
    uint32_t* cv2 = need<uint32_t>(c, c->cval2, ng);
    cls_keys((uint32_t*)c->gtg.p, (uint32_t*)c->gsr.p, ng, ca, keys, cv, s);
    size_t wsn = std::max(sort_ws_bytes(ng), scan_ws_bytes(ng));
    void* ws = wsn > c->ws.cap ? need<char>(c, c->ws, wsn) : c->ws.p;
    double* d6 = (double*)c->small.p;
    sort_u64(keys, cv, keys2, cv2, ng, 0, 64, ws, s);
    uint32_t* head = need<uint32_t>(c, c->chead, ng + 1);
    uint32_t* hoff = need<uint32_t>(c, c->choff, ng + 1);
    cls_heads(keys, ng, head, s);
    scan_u32(head, hoff, (uint32_t*)(d6 + 12), ng, ws, s);
    check_launch("m2l classes: keys");
    uint32_t ncls = 0;
    to_host<uint32_t>(c, &ncls, d6 + 12, 1);
    if (ncls == 0) return;
    int32_t* start = need<int32_t>(c, c->cstart, (size_t)ncls + 1);
    int32_t* pos = need<int32_t>(c, c->cpos, ng);
    uint32_t* srcs = need<uint32_t>(c, c->csrcs, ng);
    cls_index(head, hoff, ng, cv, (uint32_t*)c->gsr.p, start, pos, srcs, s);
    cls_end(keys, ng, start, (int32_t)ncls, s);
    uint32_t* nt = need<uint32_t>(c, c->cnt_t, (size_t)ncls + 1);
    uint32_t* tb = need<uint32_t>(c, c->ctbase, (size_t)ncls + 1);
    cls_ntiles(start, (int32_t)ncls, NT, nt, s);
    if (scan_ws_bytes(ncls) > c->ws.cap) {
        ws = need<char>(c, c->ws, scan_ws_bytes(ncls));
        d6 = (double*)c->small.p;
    }
    scan_u32(nt, tb, (uint32_t*)(d6 + 12), ncls, ws, s);
    check_launch("m2l classes: tiles");
    uint32_t ntiles = 0;
    int32_t nb = 0;
    to_host<uint32_t>(c, &ntiles, d6 + 12, 1);
    to_host<int32_t>(c, &nb, start + ncls, 1);
    int32_t* tile_cls = need<int32_t>(c, c->ctile, std::max<size_t>(ntiles, 1));
    cls_tiles(nt, tb, (int32_t)ncls, tile_cls, s);
    float* T = need<float>(c, c->cT, (size_t)ncls * KP * KP);
    fill_zero(T, (size_t)ncls * KP * KP * sizeof(float), s);
    if (c->fam == kFamilyCartesian) cls_ops_cart(keys, start, (int32_t)ncls, p, KP, T, s);
    else cls_ops(keys, start, (int32_t)ncls, p, KP, (const float*)c->d_w.p, T, s);
    if (nb < ng) cls_skip(pos, ng, nb, need<uint8_t>(c, c->cskip, ng), s);
    check_launch("m2l classes: operators");
    ClsPlan& cp = c->cp;
    cp.ncls = (int32_t)ncls;
    cp.ntiles = (int32_t)ntiles;
    cp.nbatched = nb;
    cp.tile_cls = tile_cls;
    cp.tbase = tb;
    cp.start = start;
    cp.srcs = srcs;
    cp.pos = pos;
}

// GEMM tiles of tc targets over the rows of the M2L GEMM (rows sorted by
// class and density in rval, class bounds in gp.class_row0): the row -> tile
// map, the gather table and each tile's used slots.  Run by the traversal,
// and again by the autotuner for another tile width on the same lists.
void gemm_tiles(fmm_ctx c, int tc) {
    hipStream_t s = c->stream;
    const int J = c->gp.J;
    const int32_t nc = c->ncell;
    int tiles = 0;
    for (int k = 0; k < 9; k++) {
        c->gp.class_tile0[k] = tiles;
        if (k < 8) tiles += (c->gp.class_row0[k + 1] - c->gp.class_row0[k] + tc - 1) / tc;
    }
    c->gp.ntiles = tiles;
    c->gp.nt = tc;
    c->ntiles = tiles;
    int32_t* ro = need<int32_t>(c, c->rowof, nc);
    fill_i32(ro, -1, nc, s);
    rows_inverse((const uint32_t*)c->rval.p, c->nrows, c->gp, tc, ro, s);
    const int64_t ngather = (int64_t)tiles * tc * J;
    const int Jp = (J + 3) & ~3;  // column rows of the fill table, 16-byte aligned
    const int64_t ncol = (int64_t)tiles * tc * Jp;
    int32_t* gcol = need<int32_t>(c, c->gathercol, (size_t)std::max<int64_t>(ncol, 1));
    int32_t* ga = need<int32_t>(c, c->gather, (size_t)std::max<int64_t>(ngather, 1));
    fill_i32(gcol, -1, ncol, s);
    m2l_fill_gather((const int2*)c->raw[0].p, (const int16_t*)c->m2lslot.p, c->nlist[0], ro, Jp, gcol, s);
    check_launch("m2l gather");
    int32_t* act = need<int32_t>(c, c->tact, (size_t)std::max(tiles, 1) * J);
    int32_t* nact = need<int32_t>(c, c->tnact, (size_t)std::max(tiles, 1));
    c->gp.act = act;
    c->gp.nact = nact;
    tile_transpose(gcol, c->gp, tc, Jp, tiles, ga, act, nact, s);
    check_launch("m2l tile slots");
}

void traverse_impl(fmm_ctx c, int32_t p, double theta, int32_t policy) {
    if (!c->built) fail(FMM_ERR_STATE, "fmm_traverse before fmm_build_tree");
    if (p < 0 || p > FMM_P_MAX) fail(FMM_ERR_INVALID_ARG, "p out of range");
    if (!(theta > 0.0 && theta < 1.0)) fail(FMM_ERR_INVALID_ARG, "theta must lie in (0, 1)");
    if (policy < 0 || policy > 3) fail(FMM_ERR_INVALID_ARG, "unknown policy");
    if (policy == FMM_POLICY_HYBRID_TIMED && !c->costs_set)
        fail(FMM_ERR_STATE, "timed hybrid needs unit costs (fmm_tune or fmm_set_costs)");
    // the timed pre-calculation stands in for a learned model that is missing
    if (policy == FMM_POLICY_HYBRID_MLP && !c->mlp_ready) {
        if (!c->costs_set) fail(FMM_ERR_STATE, "learned hybrid needs a trained cost model (or unit costs to fall back on)");
        policy = FMM_POLICY_HYBRID_TIMED;
    }
    // expansion family: spherical harmonics, or the Cartesian Taylor series
    // the hybrid method switches to at low accuracy ("Hybrid treecode/FMM
    // algorithm"): asked for, or chosen by order under FMM_EXPANSION_AUTO
    int fam = kFamilySpherical;
    if (c->expansion == FMM_EXPANSION_CARTESIAN) {
        if (p > kMaxPCart) fail(FMM_ERR_UNSUPPORTED, "Cartesian expansions are implemented for p <= 6");
        fam = kFamilyCartesian;
    } else if (c->expansion == FMM_EXPANSION_AUTO && p <= c->auto_cart_max_p && p <= kMaxPCart) {
        fam = kFamilyCartesian;
    }
    c->traversed = false;
    c->fam = fam;
    c->p = p;
    c->theta = theta;
    c->policy = policy;
    for (int k = 0; k < 3; k++) c->nlist[k] = 0;
    hipStream_t s = c->stream;
    upload_tables(c, p);
    int32_t nc = c->ncell;
    if (nc == 0) {
        c->traversed = true;
        return;
    }
    TravParams tp;
    tp.theta2 = theta * theta;
    tp.theta = theta;
    tp.policy = policy;
    tp.c_m2l = c->costs[0];
    tp.c_p2p = c->costs[2];
    tp.c_m2p = c->costs[1];
    tp.mlp_table = nullptr;
    tp.nbucket = nullptr;
    if (policy == FMM_POLICY_HYBRID_MLP) {
        if (c->table_p != p || c->table_theta != theta || c->table_version != c->mlp_version ||
            c->table_costs_version != c->costs_version) {
            mlp_table((const float*)c->d_mlp.p, p, (float)theta, c->costs_set ? c->costs : nullptr,
                      need<uint8_t>(c, c->d_table, kMlpTable), s);
            check_launch("cost model table");
            c->table_p = p;
            c->table_theta = theta;
            c->table_version = c->mlp_version;
            c->table_costs_version = c->costs_version;
        }
        tp.mlp_table = (const uint8_t*)c->d_table.p;
        uint8_t* nb = need<uint8_t>(c, c->nbucket, nc);
        cell_buckets(cells_of(c), nc, nb, s);
        tp.nbucket = nb;
    }
    // the learned policy reads both tables in every classification
    if (policy == FMM_POLICY_HYBRID_MLP && (!tp.mlp_table || !tp.nbucket))
        fail(FMM_ERR_STATE, "learned traversal without its choice table or count buckets");
    CellArrays ca = cells_of(c);
    void* ws = c->ws.p;
    double* d6 = (double*)c->small.p;
    // one (root, root) pair per instance: a root that is a leaf interacts with
    // itself directly, any other starts the frontier
    const int32_t nr = c->nroot;
    std::vector<int32_t> rch(nr);
    to_host<int32_t>(c, rch.data(), c->c_nchild.p, nr);
    std::vector<int2> self, start;
    if (c->n_targets < 0) {
        for (int32_t r = 0; r < nr; r++) (rch[r] == 0 ? self : start).push_back(make_int2(r, r));
    } else if (nr == 2) {
        // (target root, source root); the cube is shared, so the pair never
        // passes the criterion: two leaves interact directly, else split
        (rch[0] == 0 && rch[1] == 0 ? self : start).push_back(make_int2(0, 1));
    }
    // Frontier levels run back to back on the device: the frontier size, the
    // lists' running totals and the overflow bits stay in device memory, and
    // the host reads them once per window of levels (as many as the previous
    // traversal needed, else the bound 2 (levels) + 2: every level raises the
    // sum of a pair's two cell levels).  A list or frontier that would pass
    // its capacity ends the traversal; the buffers then grow and it runs
    // again.
    int64_t* cap = c->trav_cap;
    if (cap[0] == 0) {
        const int64_t per = std::min<int64_t>(m2l_plan_slots(theta), 4096) + 64;
        for (int k = 0; k < 3; k++) cap[k] = std::max<int64_t>(1 << 16, per * nc);
        cap[3] = std::max<int64_t>(1 << 16, 16 * nc);
    }
    uint32_t* dt = need<uint32_t>(c, c->d_trav, 16);  // totals[3], frontier size, overflow, levels; scan total at 8
    uint4* dadd = (uint4*)(dt + 8);
    if (scan_dev_ws_bytes() > c->ws.cap) {
        ws = need<char>(c, c->ws, scan_dev_ws_bytes());
        d6 = (double*)c->small.p;
    }
    uint32_t h[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    for (;;) {
        cap[2] = std::max<int64_t>(cap[2], (int64_t)self.size());
        cap[3] = std::max<int64_t>(cap[3], (int64_t)start.size());
        int2* lists[3];
        for (int k = 0; k < 3; k++) lists[k] = need<int2>(c, c->raw[k], cap[k] + 1);
        int2* fa = need<int2>(c, c->fr0, cap[3] + 1);
        int2* fb = need<int2>(c, c->fr1, cap[3] + 1);
        uint4* cnt = need<uint4>(c, c->cnt, cap[3] + 1);
        uint4* off = need<uint4>(c, c->off4, cap[3] + 1);
        uint4* kinds = need<uint4>(c, c->kinds, cap[3] + 1);
        if (!self.empty()) to_dev(c, lists[2], self.data(), self.size());
        if (!start.empty()) to_dev(c, fa, start.data(), start.size());
        const uint32_t h0[8] = {0, 0, (uint32_t)self.size(), (uint32_t)start.size(), 0, 0, 0, 0};
        to_dev(c, dt, h0, 8);
        const TravCaps tcap{cap[0], cap[1], cap[2], cap[3]};
        int window = c->trav_levels > 0 ? c->trav_levels : 2 * std::max(c->tree_levels, 1) + 2;
        for (;;) {
            for (int k = 0; k < window; k++) {
                trav_count(fa, dt + 3, cap[3], ca, tp, cnt, kinds, s);
                scan_u32x4_dev(cnt, off, dadd, DevCount{dt + 3, nullptr}, c->ws.p, s);
                trav_emit(fa, dt + 3, cap[3], ca, kinds, off, dt, dadd, tcap, lists[0], lists[1], lists[2], fb, dt + 4,
                          dt + 5, s);
                std::swap(fa, fb);
            }
            check_launch("traverse");
            to_host<uint32_t>(c, h, dt, 8);
            if (h[4] != 0 || h[3] == 0) break;
            window = 4;
        }
        if (h[4] == 0) break;
        for (int k = 0; k < 4; k++)
            if (h[4] & (1u << k)) cap[k] *= 2;
    }
    for (int k = 0; k < 3; k++) c->nlist[k] = h[k];
    c->trav_levels = (int)h[5];
    mark(c, PH_LISTS);
    int bits = bits_for(nc);
    // split + stable sort by target + CSR offsets
    auto sort_into = [&](const int2* raw, int64_t m, Buf& TG, Buf& SR, Buf& OF) {
        uint32_t* tg = need<uint32_t>(c, TG, m + 1);
        uint32_t* sr = need<uint32_t>(c, SR, m + 1);
        int32_t* of = need<int32_t>(c, OF, (size_t)nc + 1);
        if (m > 0) {
            size_t wsn = sort_ws_bytes(m);
            if (wsn > c->ws.cap) ws = need<char>(c, c->ws, wsn);
            uint32_t* tg2 = need<uint32_t>(c, c->tgt2, m);
            uint32_t* sr2 = need<uint32_t>(c, c->src2, m);
            if (raw) split_pairs(raw, m, tg, sr, s);
            sort_u32(tg, sr, tg2, sr2, m, 0, bits, ws, s);
        }
        csr_offsets(tg, m, nc, of, s);
        check_launch("lists");
    };
    // cell-particle and particle-particle lists: the kernels walk them by target
    sort_into((int2*)c->raw[1].p, c->nlist[1], c->tgt[1], c->src[1], c->off[1]);
    sort_into((int2*)c->raw[2].p, c->nlist[2], c->tgt[2], c->src[2], c->off[2]);
    // cell-cell list: kept in emission order; same-level pairs go to the GEMM
    // gather table, the rest are compacted and grouped by target
    c->m2l_sorted = false;
    // the per-pair slot is stored in 16 bits and the gather table grows with
    // the slot count: small theta sends every cell-cell pair to the class path
    c->gemm_on = m2l_gemm_supported_kp(c_kp(c)) && c->nlist[0] > 0 && m2l_plan_slots(theta) <= kGemmMaxSlots;
    c->ntiles = 0;
    c->nrows = 0;
    c->ngeneral = 0;
    int64_t nm = c->nlist[0];
    const int2* pr0 = (const int2*)c->raw[0].p;  // cell-cell pairs as emitted
    int16_t* slot16 = need<int16_t>(c, c->m2lslot, nm + 1);  // per pair: GEMM slot, -1 outside the tables
    if (c->gemm_on) {
        upload_plan(c, p, theta);
        if (m2l_bf16_supported_kp(c_kp(c))) upload_plan_bf16(c);
        int R = c->plan.R, J = c->plan.J;
        uint32_t* hf = need<uint32_t>(c, c->has_fast, nc);
        fill_zero(hf, (size_t)nc * 4, s);
        m2l_mark_targets(pr0, nm, ca, (int32_t*)c->d_slot.p, R, hf, slot16, s);
        uint32_t* rk = need<uint32_t>(c, c->rkey, nc);
        uint32_t* rv = need<uint32_t>(c, c->rval, nc);
        uint32_t* rk2 = need<uint32_t>(c, c->rkey2, nc);
        uint32_t* rv2 = need<uint32_t>(c, c->rval2, nc);
        row_class_keys(hf, ca, nc, J, rk, rv, s);
        size_t wsn = sort_ws_bytes(nc);
        if (wsn > c->ws.cap) ws = need<char>(c, c->ws, wsn);
        sort_u32(rk, rv, rk2, rv2, nc, 0, kRowMissBits + 4, ws, s);
        int32_t* d9 = (int32_t*)(d6 + 20);
        class_bounds(rk, nc, kRowMissBits, d9, s);
        check_launch("m2l classes");
        int32_t* h9 = (int32_t*)host_stage(c);
        to_host<int32_t>(c, h9, d9, 9);
        for (int k = 0; k < 9; k++) c->gp.class_row0[k] = h9[k];
        c->gp.J = J;
        c->gp.G = gemm_slot_groups(J);
        if (J / c->gp.G + 1 > kGemmMaxGroupSlots) fail(FMM_ERR_UNSUPPORTED, "M2L slot groups exceed the staged size");
        c->gp.nrows = h9[8];
        c->nrows = h9[8];
        const int kp = c_kp(c);
        gemm_tiles(c, gemm_tile_width_ok(kp, c->gemm_nt) ? c->gemm_nt : gemm_tile_cols_kp(kp));
    } else if (nm > 0) {
        fill_i32((int32_t*)slot16, -1, (nm + 1) / 2, s);  // two -1 slots per word
    }
    // pairs outside the GEMM tables, compacted in list order
    const int64_t nct = compact_tiles(nm);
    uint32_t* tcnt = need<uint32_t>(c, c->tgt2, (size_t)2 * nct + 2);
    uint32_t* tbase = tcnt + nct + 1;
    if (nm > 0) {
        size_t wsg = scan_ws_bytes(nct);
        if (wsg > c->ws.cap) ws = need<char>(c, c->ws, wsg);
        flag_counts(slot16, nm, tcnt, s);
        scan_u32(tcnt, tbase, (uint32_t*)(d6 + 12), nct, ws, s);
        uint32_t* hg = (uint32_t*)host_stage(c);
        to_host<uint32_t>(c, hg, d6 + 12, 1);
        c->ngeneral = hg[0];
    }
    {
        int64_t ng = c->ngeneral;
        uint32_t* gt = need<uint32_t>(c, c->gtg, ng + 1);
        uint32_t* gs = need<uint32_t>(c, c->gsr, ng + 1);
        if (ng > 0) compact_pairs(pr0, slot16, tbase, nm, gt, gs, s);
        sort_into(nullptr, ng, c->gtg, c->gsr, c->goff);
    }
    build_classes(c, p);
    ck(hipStreamSynchronize(s), "sync");
    c->traversed = true;
}

// Whether every particle pair of P2P must skip r = 0: FP64 inputs (distinct
// points can round to one FP32 point), and distinct target and source sets
// (a target may coincide with a source, in any pair of leaves).  Otherwise
// only a leaf with itself can hold coincident points.
// P2P tile shapes: t targets per lane on the vector ALUs (t = 1, 2, 4), or
// -t for the matrix-core form
bool p2p_shape_ok(int t) { return t == 1 || t == 2 || t == 4 || t == -1 || t == -2 || t == -4; }

int p2p_guard_all(fmm_ctx c) { return (c->dtype == FMM_F64 || c->n_targets >= 0) ? 1 : 0; }

// P2P over the leaves of each size class with that class's tile shape
void run_p2p(fmm_ctx c, double4* near, hipStream_t st) {
    for (int k = 0; k < kLeafClasses; k++) {
        const int32_t b = c->leaf_cls[k], e = c->leaf_cls[k + 1];
        if (e <= b) continue;
        p2p((float4*)c->pts.p, cells_of(c), (int32_t*)c->leaves_cls.p + b, e - b, (int32_t*)c->off[2].p,
            (uint32_t*)c->src[2].p, p2p_guard_all(c), c->p2p_tpl[k], near, st);
    }
    check_launch("p2p");
}

// ------------------------------------------------------------------ evaluate
// Work buffers of one evaluation (beyond the context's tree, lists and
// tables): expansions, near-field partials, per-group GEMM partials, split
// multipoles, class partials and the cell-particle flags.
struct EvalBufs {
    float* M = nullptr;         // (ncell + 1) * KP: multipoles and one all-zero row
    float* L = nullptr;         // ncell * KP
    double4* near = nullptr;    // n
    float* part = nullptr;      // G * nrows * KP (batched GEMM)
    uint4* Msplit = nullptr;    // (ncell + 1) * KP / 4 (split-BF16 batched GEMM)
    float* cls_part = nullptr;  // nbatched * KP (class-batched pairs)
    uint8_t* m2pflag = nullptr; // max(nleaf, 1)
};

enum { EB_M, EB_L, EB_NEAR, EB_PART, EB_MSPLIT, EB_CLS, EB_FLAG, EB_N };

// bytes of each work buffer for an evaluation at `precision` (0 = not used)
void eval_sizes(fmm_ctx c, int precision, size_t* b) {
    const size_t KP = (size_t)c_kp(c), nc = (size_t)c->ncell;
    const bool gemm = c->gemm_on && c->ntiles > 0;
    b[EB_M] = (nc + 1) * KP * sizeof(float);
    b[EB_L] = nc * KP * sizeof(float);
    b[EB_NEAR] = (size_t)c->n * sizeof(double4);
    b[EB_PART] = gemm ? (size_t)c->gp.G * c->gp.nrows * KP * sizeof(float) : 0;
    b[EB_MSPLIT] = gemm && precision == FMM_PREC_SPLIT_BF16 ? (nc + 1) * KP * sizeof(float) : 0;
    b[EB_CLS] = c->cp.ntiles > 0 ? (size_t)c->cp.nbatched * KP * sizeof(float) : 0;
    b[EB_FLAG] = (size_t)std::max(c->nleaf, 1);
}

void check_evaluate_args(fmm_ctx c, int32_t precision, int32_t out_dtype, void* phi, void* ex, void* ey, void* ez) {
    if (!c->traversed) fail(FMM_ERR_STATE, "fmm_evaluate before fmm_traverse");
    if (precision != FMM_PREC_FP32 && precision != FMM_PREC_SPLIT_BF16)
        fail(FMM_ERR_INVALID_ARG, "precision must be FMM_PREC_FP32 or FMM_PREC_SPLIT_BF16");
    if (precision == FMM_PREC_SPLIT_BF16 && !m2l_bf16_supported_kp(c_kp(c)))
        fail(FMM_ERR_UNSUPPORTED, "split-BF16 M2L is implemented for storage widths up to 192 (spherical p <= 12)");
    if (out_dtype != FMM_F32 && out_dtype != FMM_F64) fail(FMM_ERR_INVALID_ARG, "out_dtype must be F32 or F64");
    // one output per particle, or per target when targets and sources differ
    const int64_t nout = c->n_targets >= 0 ? c->n_targets : c->n;
    if (nout > 0 && (!phi || !ex || !ey || !ez)) fail(FMM_ERR_INVALID_ARG, "null output pointer");
}

// The evaluation proper on the given work buffers; `in_order` runs every
// kernel on the context stream (no second stream).
void evaluate_on(fmm_ctx c, int32_t precision, int32_t out_dtype, void* phi, void* ex, void* ey, void* ez,
                 const EvalBufs& eb, bool in_order) {
    hipStream_t s = c->stream;
    const int p = c->p, KP = c_kp(c), K = c_k(c), fam = c->fam;
    int32_t nc = c->ncell;
    CellArrays ca = cells_of(c);
    Tables tb = tables_of(c);
    // one extra, all-zero multipole row (index nc): the M2L GEMM reads it for absent sources
    float* M = eb.M;
    fill_zero(M + (size_t)nc * KP, (size_t)KP * sizeof(float), s);
    c->gp.zcell = nc;
    float* L = eb.L;
    double4* nr = eb.near;
    // P2P depends only on the tree and its list: under a concurrent schedule it
    // runs on the second stream (forked at the start, or after the upward
    // pass) while the expansions are formed and translated, and the final sum
    // waits for it
    const int sched = (c->nleaf > 0 && !in_order) ? c->schedule : 0;
    auto fork_p2p = [&] {
        if (!c->s2) {
            ck(hipStreamCreateWithFlags(&c->s2, hipStreamNonBlocking), "hipStreamCreate");
            for (hipEvent_t* e : {&c->e_fork, &c->e_join, &c->e_p2p0, &c->e_p2p1})
                ck(hipEventCreate(e), "hipEventCreate");
        }
        ck(hipEventRecord(c->e_fork, s), "event");
        ck(hipStreamWaitEvent(c->s2, c->e_fork, 0), "wait");
        if (c->timing) ck(hipEventRecord(c->e_p2p0, c->s2), "event");
        run_p2p(c, nr, c->s2);
        if (c->timing) ck(hipEventRecord(c->e_p2p1, c->s2), "event");
        ck(hipEventRecord(c->e_join, c->s2), "event");
    };
    if (sched == 1) fork_p2p();
    mark(c, PH_UP);
    p2m((float4*)c->pts.p, ca, (int32_t*)c->leaves.p, c->nleaf, fam, p, KP, tb.rcoef, M, s);
    int nlev = (int)c->lvl.size() - 1;
    const int32_t* inr = (const int32_t*)c->inner.p;
    const uint32_t* lpos = (const uint32_t*)c->leafpos.p;
    for (int Lv = nlev - 2; Lv >= 0; Lv--)
        m2m(ca, inr, lpos, c->lvl[Lv], c->lvl[Lv + 1], c->ncell, c->nleaf, K, KP, tb, M, s);
    check_launch("upward");
    if (sched == 2) fork_p2p();
    fill_zero(L, (size_t)nc * KP * sizeof(float), s);
    mark(c, PH_M2L);
    if (c->gemm_on && c->ntiles > 0)
    {
        float* part = eb.part;
        hipEvent_t g0 = c->timing ? c->ev_gk[0] : nullptr, g1 = c->timing ? c->ev_gk[1] : nullptr;
        if (precision == FMM_PREC_SPLIT_BF16)
            m2l_gemm_bf16((uint16_t*)c->d_Thi.p, (uint16_t*)c->d_Tlo.p, (int32_t*)c->d_offid.p, (int32_t*)c->gather.p,
                          (uint32_t*)c->rval.p, c->gp, K, KP, M, nc, eb.Msplit, part, L, s, g0, g1);
        else
            m2l_gemm((float*)c->d_T.p, (int32_t*)c->d_offid.p, (int32_t*)c->gather.p, (uint32_t*)c->rval.p, c->gp, K,
                     KP, M, part, L, s, g0, g1);
    }
    mark(c, PH_M2LG);
    if (c->cp.ntiles > 0) {
        ClsPlan cp = c->cp;
        cp.zcell = nc;
        float* part2 = eb.cls_part;
        m2l_cls((const float*)c->cT.p, cp, K, KP, M, part2, (int32_t*)c->goff.p, nc, L, s);
    }
    if (c->ngeneral > c->cp.nbatched) {
        const uint8_t* skip = c->cp.nbatched > 0 ? (const uint8_t*)c->cskip.p : nullptr;
        if (fam == kFamilyCartesian)
            m2l_general_cart((int32_t*)c->goff.p, (uint32_t*)c->gsr.p, ca, nc, p, KP, M, L, skip, s);
        else if (c->m2l_kind == FMM_M2L_CLASS_ROTATION || c->m2l_kind == FMM_M2L_PAIR_ROTATION)
            m2l_rotation((int32_t*)c->goff.p, (uint32_t*)c->gsr.p, ca, nc, p, KP, tb.wax, M, L, skip, s);
        else
            m2l_general((int32_t*)c->goff.p, (uint32_t*)c->gsr.p, ca, nc, p, KP, tb, M, L, skip, s);
    }
    check_launch("m2l");
    mark(c, PH_DOWN);
    for (int Lv = 0; Lv + 1 < nlev; Lv++)
        l2l(ca, inr, lpos, c->lvl[Lv], c->lvl[Lv + 1], c->ncell, c->nleaf, K, KP, tb, L, s);
    check_launch("downward");
    mark(c, PH_P2P);
    if (sched) {
        ck(hipStreamWaitEvent(s, c->e_join, 0), "wait");
    } else {
        run_p2p(c, nr, s);
    }
    mark(c, PH_FAR);
    uint8_t* mflag = eb.m2pflag;
    // the outputs are the targets': with distinct sets, only the target tree's leaves
    const bool ts = c->n_targets >= 0;
    far_final((float4*)c->pts.p, (uint32_t*)c->idx.p, ca, ts ? (int32_t*)c->tleaves.p : (int32_t*)c->leaves.p,
              ts ? c->ntleaf : c->nleaf, mflag, (int32_t*)c->off[1].p,
              (uint32_t*)c->src[1].p, c->nlist[1], fam, p, KP, tb, M, L, nr, out_dtype, phi, ex, ey, ez, s);
    check_launch("far field");
    mark(c, PH_N);
    if (c->timing) {
        ck(hipEventSynchronize(c->ev[PH_N]), "event sync");
        for (int k = PH_UP; k < PH_N; k++) {
            float t = 0;
            ck(hipEventElapsedTime(&t, c->ev[k], c->ev[k + 1]), "elapsed");
            c->ms[k] = t;
        }
        if (sched) {
            // the P2P kernel's own duration on the second stream
            float t = 0;
            ck(hipEventElapsedTime(&t, c->e_p2p0, c->e_p2p1), "elapsed");
            c->ms[PH_P2P] = t;
        }
        c->ms_gemm_kernel = 0;
        if (c->gemm_on && c->ntiles > 0) {
            float t = 0;
            ck(hipEventElapsedTime(&t, c->ev_gk[0], c->ev_gk[1]), "elapsed");
            c->ms_gemm_kernel = t;
        }
    }
}

// fmm_evaluate: work buffers held by the context (grown as needed)
void evaluate_impl(fmm_ctx c, int32_t precision, int32_t out_dtype, void* phi, void* ex, void* ey, void* ez) {
    check_evaluate_args(c, precision, out_dtype, phi, ex, ey, ez);
    if (c->n == 0) return;
    size_t b[EB_N];
    eval_sizes(c, precision, b);
    EvalBufs eb;
    eb.M = need<float>(c, c->M, b[EB_M] / 4);
    eb.L = need<float>(c, c->L, b[EB_L] / 4);
    eb.near = need<double4>(c, c->nearb, c->n);
    if (b[EB_PART]) eb.part = need<float>(c, c->m2l_part, b[EB_PART] / 4);
    if (b[EB_MSPLIT]) eb.Msplit = need<uint4>(c, c->Msplit, b[EB_MSPLIT] / 16);
    if (b[EB_CLS]) eb.cls_part = need<float>(c, c->cls_part, b[EB_CLS] / 4);
    eb.m2pflag = need<uint8_t>(c, c->m2pflag, b[EB_FLAG]);
    evaluate_on(c, precision, out_dtype, phi, ex, ey, ez, eb, false);
}

}  // namespace

// ================================================================== C-ABI
extern "C" {

fmm_status fmm_create(fmm_ctx* out, int device, void* hip_stream) {
    if (!out) return FMM_ERR_INVALID_ARG;
    *out = nullptr;
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || device < 0 || device >= ndev) {
        (void)hipGetLastError();
        return ndev == 0 ? FMM_ERR_DEVICE : FMM_ERR_INVALID_ARG;
    }
    fmm_ctx c = new (std::nothrow) fmm_ctx_s();
    if (!c) return FMM_ERR_OUT_OF_MEMORY;
    c->device = device;
    c->stream = (hipStream_t)hip_stream;
    fmm_status st = guarded(c, [&] {
        for (int k = 0; k <= PH_N; k++) ck(hipEventCreate(&c->ev[k]), "hipEventCreate");
        for (int k = 0; k < 2; k++) ck(hipEventCreate(&c->ev_gk[k]), "hipEventCreate");
        // the device address of the fixed work area of fmm_evaluate_noalloc
        ck(noalloc_setup(device), "work area of the no-allocation evaluation");
    });
    if (st != FMM_OK) {
        fmm_destroy(c);
        return st;
    }
    *out = c;
    return FMM_OK;
}

void fmm_destroy(fmm_ctx c) {
    if (!c) return;
    (void)hipSetDevice(c->device);
    if (c->stream) (void)hipStreamSynchronize(c->stream);
    else (void)hipDeviceSynchronize();
    for (Buf* b : c->bufs) dev_release(*b);
    for (int k = 0; k <= PH_N; k++)
        if (c->ev[k]) (void)hipEventDestroy(c->ev[k]);
    for (int k = 0; k < 2; k++)
        if (c->ev_gk[k]) (void)hipEventDestroy(c->ev_gk[k]);
    if (c->s2) {
        (void)hipStreamSynchronize(c->s2);
        (void)hipStreamDestroy(c->s2);
    }
    for (hipEvent_t e : {c->e_fork, c->e_join, c->e_p2p0, c->e_p2p1})
        if (e) (void)hipEventDestroy(e);
    if (c->host) (void)hipHostFree(c->host);
    delete c;
}

const char* fmm_last_error(fmm_ctx c) { return c ? c->err.c_str() : "null context"; }

fmm_status fmm_set_stream(fmm_ctx c, void* hip_stream) {
    return guarded(c, [&] { c->stream = (hipStream_t)hip_stream; });
}

namespace {
void build_timings(fmm_ctx c) {
    if (c->timing && c->n > 0) {
        ck(hipEventRecord(c->ev[PH_TRAV], c->stream), "event");
        ck(hipEventSynchronize(c->ev[PH_TRAV]), "event sync");
        for (int k = PH_KEYS; k < PH_TRAV; k++) {
            float t = 0;
            ck(hipEventElapsedTime(&t, c->ev[k], c->ev[k + 1]), "elapsed");
            c->ms[k] = t;
        }
    }
}
}  // namespace

fmm_status fmm_build_tree(fmm_ctx c, int64_t n, int dtype, const void* x, const void* y, const void* z,
                          const void* q, int32_t ncrit) {
    return guarded(c, [&] {
        build_tree_impl(c, n, dtype, x, y, z, q, ncrit);
        build_timings(c);
    });
}

// Target tree and source tree in one cube (targets first, with zero charge).
void build_tree_ts_impl(fmm_ctx c, int dtype, int64_t n_targets, const void* tx, const void* ty, const void* tz,
                        int64_t n_sources, const void* sx, const void* sy, const void* sz, const void* q,
                        int32_t ncrit) {
    if (n_targets < 0 || n_sources < 0 || n_targets + n_sources >= ((int64_t)1 << 31))
        fail(FMM_ERR_INVALID_ARG, "particle counts out of range");
    if (dtype != FMM_F32 && dtype != FMM_F64) fail(FMM_ERR_INVALID_ARG, "dtype must be FMM_F32 or FMM_F64");
    if ((n_targets > 0 && (!tx || !ty || !tz)) || (n_sources > 0 && (!sx || !sy || !sz || !q)))
        fail(FMM_ERR_INVALID_ARG, "null input pointer");
    const int64_t n = n_targets + n_sources;
    const size_t es = dtype == FMM_F64 ? 8 : 4;
    // the two sets side by side (targets first), targets with zero charge
    char* st = need<char>(c, c->ts_stage, 4 * (size_t)std::max<int64_t>(n, 1) * es);
    char* X[4] = {st, st + n * es, st + 2 * n * es, st + 3 * n * es};
    const void* T[3] = {tx, ty, tz};
    const void* S[4] = {sx, sy, sz, q};
    for (int d = 0; d < 3; d++) {
        if (n_targets > 0) ck(hipMemcpyAsync(X[d], T[d], n_targets * es, hipMemcpyDeviceToDevice, c->stream), "copy");
        if (n_sources > 0)
            ck(hipMemcpyAsync(X[d] + n_targets * es, S[d], n_sources * es, hipMemcpyDeviceToDevice, c->stream),
               "copy");
    }
    if (n_targets > 0) fill_zero(X[3], n_targets * es, c->stream);
    if (n_sources > 0)
        ck(hipMemcpyAsync(X[3] + n_targets * es, q, n_sources * es, hipMemcpyDeviceToDevice, c->stream), "copy");
    const int64_t seg[3] = {0, n_targets, n};
    build_forest_impl(c, 2, seg, dtype, X[0], X[1], X[2], X[3], ncrit, true);
    c->n_targets = n_targets;
    // the leaves holding targets, for the final sum
    const int32_t nl = c->nleaf;
    int32_t* tl = need<int32_t>(c, c->tleaves, std::max(nl, 1));
    c->ntleaf = 0;
    if (nl > 0 && n_targets > 0) {
        uint32_t* flag = need<uint32_t>(c, c->tmp1, nl + 1);
        uint32_t* pos = need<uint32_t>(c, c->tmp2, nl + 1);
        size_t wsn = scan_ws_bytes(nl);
        void* ws = wsn > c->ws.cap ? need<char>(c, c->ws, wsn) : c->ws.p;
        double* d6 = (double*)c->small.p;
        target_leaf_flags(cells_of(c), (const int32_t*)c->leaves.p, nl, (int32_t)n_targets, flag, c->stream);
        scan_u32(flag, pos, (uint32_t*)(d6 + 12), nl, ws, c->stream);
        target_leaf_write((const int32_t*)c->leaves.p, flag, pos, nl, tl, c->stream);
        check_launch("target leaves");
        uint32_t cnt = 0;
        to_host<uint32_t>(c, &cnt, d6 + 12, 1);
        c->ntleaf = (int32_t)cnt;
    }
}

fmm_status fmm_build_tree_ts(fmm_ctx c, int dtype, int64_t n_targets, const void* tx, const void* ty,
                             const void* tz, int64_t n_sources, const void* sx, const void* sy, const void* sz,
                             const void* q, int32_t ncrit) {
    return guarded(c, [&] {
        build_tree_ts_impl(c, dtype, n_targets, tx, ty, tz, n_sources, sx, sy, sz, q, ncrit);
        build_timings(c);
    });
}

fmm_status fmm_build_tree_batch(fmm_ctx c, int32_t n_inst, const int64_t* offsets, int dtype, const void* x,
                                const void* y, const void* z, const void* q, int32_t ncrit) {
    return guarded(c, [&] {
        build_forest_impl(c, n_inst, offsets, dtype, x, y, z, q, ncrit);
        build_timings(c);
    });
}

fmm_status fmm_evaluate_batch(fmm_ctx c, int32_t n_inst, const int64_t* offsets, int dtype, const void* x,
                              const void* y, const void* z, const void* q, int32_t ncrit, int32_t p, double theta,
                              int32_t policy, int32_t precision, int32_t out_dtype, void* phi, void* ex, void* ey,
                              void* ez) {
    fmm_status st = fmm_build_tree_batch(c, n_inst, offsets, dtype, x, y, z, q, ncrit);
    if (st == FMM_OK) st = fmm_traverse(c, p, theta, policy);
    if (st == FMM_OK) st = fmm_evaluate(c, precision, out_dtype, phi, ex, ey, ez);
    return st;
}

fmm_status fmm_traverse(fmm_ctx c, int32_t p, double theta, int32_t policy) {
    return guarded(c, [&] {
        if (c->timing) ck(hipEventRecord(c->ev[PH_TRAV], c->stream), "event");
        traverse_impl(c, p, theta, policy);
        if (c->timing && c->n > 0) {
            ck(hipEventRecord(c->ev[PH_UP], c->stream), "event");
            ck(hipEventSynchronize(c->ev[PH_UP]), "event sync");
            float t = 0;
            ck(hipEventElapsedTime(&t, c->ev[PH_TRAV], c->ev[PH_LISTS]), "elapsed");
            c->ms[PH_TRAV] = t;
            ck(hipEventElapsedTime(&t, c->ev[PH_LISTS], c->ev[PH_UP]), "elapsed");
            c->ms[PH_LISTS] = t;
        }
    });
}

fmm_status fmm_evaluate(fmm_ctx c, int32_t precision, int32_t out_dtype, void* phi, void* ex, void* ey,
                        void* ez) {
    return guarded(c, [&] { evaluate_impl(c, precision, out_dtype, phi, ex, ey, ez); });
}

fmm_status fmm_evaluate_noalloc(fmm_ctx c, int32_t precision, int32_t out_dtype, void* phi, void* ex, void* ey,
                                void* ez) {
    return guarded(c, [&] {
        check_evaluate_args(c, precision, out_dtype, phi, ex, ey, ez);
        if (c->n == 0) return;
        char* area = (char*)noalloc_area(c->device);
        if (!area) fail(FMM_ERR_DEVICE, "no work area on this device");
        size_t b[EB_N], off[EB_N], total = 0;
        eval_sizes(c, precision, b);
        for (int k = 0; k < EB_N; k++) {
            off[k] = total;
            total += (b[k] + 255) / 256 * 256;
        }
        if (total > kNoAllocScratchBytes)
            fail(FMM_ERR_INVALID_ARG, "this evaluation needs " + std::to_string(total) +
                                          " bytes of work space; fmm_evaluate_noalloc holds " +
                                          std::to_string(kNoAllocScratchBytes) + " (use fmm_evaluate)");
        EvalBufs eb;
        eb.M = (float*)(area + off[EB_M]);
        eb.L = (float*)(area + off[EB_L]);
        eb.near = (double4*)(area + off[EB_NEAR]);
        eb.part = b[EB_PART] ? (float*)(area + off[EB_PART]) : nullptr;
        eb.Msplit = b[EB_MSPLIT] ? (uint4*)(area + off[EB_MSPLIT]) : nullptr;
        eb.cls_part = b[EB_CLS] ? (float*)(area + off[EB_CLS]) : nullptr;
        eb.m2pflag = (uint8_t*)(area + off[EB_FLAG]);
        evaluate_on(c, precision, out_dtype, phi, ex, ey, ez, eb, true);
    });
}

fmm_status fmm_set_expansion(fmm_ctx c, int32_t expansion, int32_t auto_cartesian_max_p) {
    return guarded(c, [&] {
        if (expansion < FMM_EXPANSION_SPHERICAL || expansion > FMM_EXPANSION_AUTO)
            fail(FMM_ERR_INVALID_ARG, "unknown expansion family");
        if (expansion == FMM_EXPANSION_AUTO && (auto_cartesian_max_p < -1 || auto_cartesian_max_p > kMaxPCart))
            fail(FMM_ERR_INVALID_ARG, "the Cartesian range of FMM_EXPANSION_AUTO must lie in [-1, 6]");
        c->expansion = expansion;
        if (expansion == FMM_EXPANSION_AUTO) c->auto_cart_max_p = auto_cartesian_max_p;
    });
}

fmm_status fmm_set_m2l_kernel(fmm_ctx c, int32_t kind) {
    return guarded(c, [&] {
        if (kind < FMM_M2L_CLASS_DENSE || kind > FMM_M2L_PAIR_ROTATION) fail(FMM_ERR_INVALID_ARG, "unknown M2L kind");
        const bool rebuild = c->traversed && c->m2l_kind != kind;
        c->m2l_kind = kind;
        // the class batching of the current lists follows the new kind
        if (rebuild) build_classes(c, c->p);
    });
}

fmm_status fmm_get_m2l_kernel(fmm_ctx c, int32_t* kind) {
    return guarded(c, [&] {
        if (!kind) fail(FMM_ERR_INVALID_ARG, "null pointer");
        *kind = c->m2l_kind;
    });
}

fmm_status fmm_get_expansion(fmm_ctx c, int32_t* family) {
    return guarded(c, [&] {
        if (!family) fail(FMM_ERR_INVALID_ARG, "null pointer");
        if (!c->traversed) fail(FMM_ERR_STATE, "no traversal");
        *family = c->fam == kFamilyCartesian ? FMM_EXPANSION_CARTESIAN : FMM_EXPANSION_SPHERICAL;
    });
}

fmm_status fmm_set_costs(fmm_ctx c, double c_m2l, double c_m2p, double c_p2p) {
    return guarded(c, [&] {
        if (!(c_m2l > 0) || !(c_m2p > 0) || !(c_p2p > 0)) fail(FMM_ERR_INVALID_ARG, "unit costs must be > 0");
        c->costs[0] = c_m2l;
        c->costs[1] = c_m2p;
        c->costs[2] = c_p2p;
        c->costs_set = true;
        c->costs_version++;
    });
}

fmm_status fmm_get_costs(fmm_ctx c, double* costs3) {
    return guarded(c, [&] {
        if (!costs3) fail(FMM_ERR_INVALID_ARG, "null pointer");
        if (!c->costs_set) fail(FMM_ERR_STATE, "no unit costs yet");
        for (int k = 0; k < 3; k++) costs3[k] = c->costs[k];
    });
}

// Kernel pre-calculation ("Kernel pre-calculation"): every kernel is run on
// artificial coordinates and charges (and the multipoles they produce) in a
// private context with event timing, and the unit costs are the measured
// times divided by the work units: M2L pairs of the batched GEMM, target
// particles of M2P pairs, particle pairs of P2P.  The instance is large
// enough to fill the GPU, because small pre-tests mispredict on a GPU
// ("Results").
fmm_status fmm_tune(fmm_ctx c, int32_t p, int32_t precision) {
    return guarded(c, [&] {
        if (p < 0 || p > FMM_P_MAX) fail(FMM_ERR_INVALID_ARG, "p out of range");
        if (precision != FMM_PREC_FP32 && precision != FMM_PREC_SPLIT_BF16)
            fail(FMM_ERR_UNSUPPORTED, "tuning is implemented for FP32 and split-BF16");
        const int64_t n = 1 << 19;
        const int32_t ncrit = 32;
        const double theta = 0.5;
        float* pts = need<float>(c, c->tune_pts, (size_t)4 * n);
        artificial_points(n, 12345, pts, pts + n, pts + 2 * n, pts + 3 * n, c->stream);
        float* out = need<float>(c, c->tune_out, (size_t)4 * n);
        check_launch("artificial points");
        fmm_ctx t = nullptr;
        fmm_status st = fmm_create(&t, c->device, c->stream);
        if (st != FMM_OK) fail(st, "calibration context");
        struct Del {
            fmm_ctx t;
            ~Del() { fmm_destroy(t); }
        } del{t};
        t->ualloc = c->ualloc;
        t->ufree = c->ufree;
        t->uuser = c->uuser;
        t->expansion = c->expansion;
        t->auto_cart_max_p = c->auto_cart_max_p;
        t->timing = true;
        t->schedule = 0;  // each kernel timed alone
        double tm[2][PH_N] = {};
        int64_t units[3] = {0, 0, 0};
        for (int pol = 0; pol < 2; pol++) {
            build_tree_impl(t, n, FMM_F32, pts, pts + n, pts + 2 * n, pts + 3 * n, ncrit);
            traverse_impl(t, p, theta, pol == 0 ? FMM_POLICY_FMM : FMM_POLICY_TREECODE);
            for (int rep = 0; rep < 3; rep++) {
                evaluate_impl(t, precision, FMM_F32, out, out + n, out + 2 * n, out + 3 * n);
                if (rep > 0)
                    for (int k = 0; k < PH_N; k++) tm[pol][k] += t->ms[k] / 2;
            }
            // work units from the lists and the cells' particle counts
            std::vector<int32_t> b(t->ncell), e(t->ncell);
            to_host<int32_t>(t, b.data(), t->c_begin.p, t->ncell);
            to_host<int32_t>(t, e.data(), t->c_end.p, t->ncell);
            int kind = pol == 0 ? 2 : 1;
            int64_t m = t->nlist[kind];
            std::vector<uint32_t> tg(m), sr(m);
            to_host<uint32_t>(t, tg.data(), t->tgt[kind].p, m);
            to_host<uint32_t>(t, sr.data(), t->src[kind].p, m);
            int64_t u = 0;
            for (int64_t i = 0; i < m; i++) {
                int64_t nt = e[tg[i]] - b[tg[i]], ns = e[sr[i]] - b[sr[i]];
                u += kind == 2 ? nt * ns : nt;
            }
            if (pol == 0) {
                units[0] = t->nlist[0] - t->ngeneral;
                units[2] = u;
            } else {
                units[1] = u;
            }
        }
        if (units[0] <= 0 || units[1] <= 0 || units[2] <= 0) fail(FMM_ERR_DEVICE, "calibration produced no work");
        // ms -> ns per unit
        double c_m2l = tm[0][PH_M2L] * 1e6 / (double)units[0];
        double c_p2p = tm[0][PH_P2P] * 1e6 / (double)units[2];
        double c_m2p = std::max(tm[1][PH_FAR] - tm[0][PH_FAR], 1e-6) * 1e6 / (double)units[1];
        c->costs[0] = c_m2l;
        c->costs[1] = c_m2p;
        c->costs[2] = c_p2p;
        c->costs_set = true;
        c->costs_version++;
    });
}

// ---------------------------------------------------------------- learned cost model
static void mlp_features(float* f, int dl, double nt, double ns, int p, double theta) {
    f[0] = (float)dl / 2.f;
    f[1] = (float)(std::log2(nt) / 8.0);
    f[2] = (float)(std::log2(ns) / 8.0);
    f[3] = (float)p / 10.f;
    f[4] = 0.875f;  // pairs near the acceptance boundary: the last bin of the table
    f[5] = (float)theta;
}

// Timing records generated by the method itself: clustered artificial
// particle sets whose leaves all hold `per` particles give homogeneous pair
// batches; the FMM policy times same-level M2L (GEMM) and P2P per cell pair,
// the treecode policy M2P per cell pair, and a set whose lower half is one
// level deeper times the mixed-level M2L pairs of its interface.  Target and
// source sets on one lattice with different leaf sizes (a target tree and a
// source tree) time P2P off the diagonal n_t != n_s (an M2P evaluation reads
// only the source's multipole, so its cost does not depend on n_s).
static void gen_records(fmm_ctx c, int p, double theta, int precision, uint64_t seed) {
    c->rec_feat.clear();
    c->rec_kind.clear();
    c->rec_tgt.clear();
    fmm_ctx t = nullptr;
    fmm_status st = fmm_create(&t, c->device, c->stream);
    if (st != FMM_OK) fail(st, "calibration context");
    struct Del {
        fmm_ctx t;
        ~Del() { fmm_destroy(t); }
    } del{t};
    t->ualloc = c->ualloc;
    t->ufree = c->ufree;
    t->uuser = c->uuser;
    t->expansion = c->expansion;
    t->auto_cart_max_p = c->auto_cart_max_p;
    t->timing = true;
    t->schedule = 0;  // each kernel timed alone
    // leaf sizes measured: up to 128 particles, where a set of at most 2^19
    // particles still has 4096 leaves to fill the GPU (larger leaves would
    // time a nearly idle device); larger sizes follow the work scaling below
    const int pers[] = {2, 4, 8, 16, 32, 64, 128};
    const int NS = (int)(sizeof(pers) / sizeof(pers[0]));
    // one measurement: log2 ns per cell pair (NaN = not measured)
    struct Meas {
        double v = NAN;
    };
    // diagonal (n_t = n_s): same-level M2L, mixed-level M2L, M2P, P2P per leaf size
    std::vector<Meas> Tm2l(NS), Tgen(NS), Tm2p(NS), Tp2p(NS);
    // off the diagonal, targets pers[i] and sources pers[j]: P2P at [i NS + j]
    // (M2P's stay unmeasured: its cost does not depend on n_s)
    std::vector<Meas> Om2p(NS * NS), Op2p(NS * NS);
    auto lg = [](double ms, int64_t units) { return units > 0 && ms > 0 ? std::log2(ms * 1e6 / (double)units) : NAN; };
    auto meas = [](double v, int) { return Meas{v}; };
    // a warm-up evaluation, then the mean of `reps` timed ones
    auto timed = [&](int policy, double* tm, int reps) {
        traverse_impl(t, p, theta, policy);
        float* out = need<float>(c, c->tune_out, (size_t)4 * t->n);
        for (int k = 0; k < PH_N; k++) tm[k] = 0;
        for (int rep = 0; rep <= reps; rep++) {
            evaluate_impl(t, precision, FMM_F32, out, out + t->n, out + 2 * t->n, out + 3 * t->n);
            if (rep > 0)
                for (int k = 0; k < PH_N; k++) tm[k] += t->ms[k] / reps;
        }
    };
    // lattice level for a set of 2^(3L) leaves of `per` particles (plus another of per2)
    auto level_for = [](int per, int per2, int64_t cap) {
        int L = 7;
        while (L > 1 && ((int64_t)1 << (3 * L)) * (per + per2) > cap) L--;
        return L;
    };
    for (int si = 0; si < NS; si++) {
        const int per = pers[si];
        const int L = level_for(per, 0, (int64_t)1 << 19);
        int64_t n = clustered_points(L, per, per, seed, nullptr, nullptr, nullptr, nullptr, c->stream);
        float* pts = need<float>(c, c->tune_pts, (size_t)4 * n);
        clustered_points(L, per, per, seed, pts, pts + n, pts + 2 * n, pts + 3 * n, c->stream);
        check_launch("clustered points");
        build_tree_impl(t, n, FMM_F32, pts, pts + n, pts + 2 * n, pts + 3 * n, per);
        double tf[PH_N], tt[PH_N];
        timed(FMM_POLICY_FMM, tf, 2);
        Tm2l[si] = meas(lg(tf[PH_M2L], t->nlist[0] - t->ngeneral), 0);
        Tp2p[si] = meas(lg(tf[PH_P2P], t->nlist[2]), 2);
        timed(FMM_POLICY_TREECODE, tt, 1);  // M2P-heavy lists: one timed run is ample work
        Tm2p[si] = meas(lg(tt[PH_FAR] - tf[PH_FAR], t->nlist[1]), 1);
        // mixed levels: the lower half one level deeper
        int L2 = L;
        while (L2 > 1 && ((int64_t)1 << (3 * L2 - 1)) * 9 * per > ((int64_t)1 << 20)) L2--;
        int64_t n2 = clustered_points(L2, per, 8 * per, seed + 1, nullptr, nullptr, nullptr, nullptr, c->stream);
        pts = need<float>(c, c->tune_pts, (size_t)4 * n2);
        clustered_points(L2, per, 8 * per, seed + 1, pts, pts + n2, pts + 2 * n2, pts + 3 * n2, c->stream);
        check_launch("clustered points");
        build_tree_impl(t, n2, FMM_F32, pts, pts + n2, pts + 2 * n2, pts + 3 * n2, per);
        timed(FMM_POLICY_FMM, tf, 2);
        Tgen[si] = meas(lg(tf[PH_M2LG], t->ngeneral), 0);
        // off the diagonal: targets with `per` per leaf, sources with 4x fewer
        // or more on the same lattice; a leaf size ncrit in [max, 8 min) stops
        // both trees at that lattice.  Two trees pay costs one tree does not
        // (every particle pair guarded against r = 0), so the same two-tree
        // run at n_s = n_t anchors them: a record is the one-tree diagonal
        // cost times the measured two-tree ratio.
        double ts_diag[1] = {NAN};  // two-tree log2 P2P cost at n_s = n_t
        for (int sj : {si, si - 2, si + 2}) {
            if (sj < 0 || sj >= NS) continue;
            const int ps = pers[sj];
            const int Lo = level_for(per, ps, (int64_t)1 << 19);
            const int64_t nt = clustered_points(Lo, per, per, seed + 2, nullptr, nullptr, nullptr, nullptr, c->stream);
            const int64_t ns = clustered_points(Lo, ps, ps, seed + 3, nullptr, nullptr, nullptr, nullptr, c->stream);
            float* tp = need<float>(c, c->tune_pts, (size_t)4 * (nt + ns));
            float* sp = tp + 4 * nt;
            clustered_points(Lo, per, per, seed + 2, tp, tp + nt, tp + 2 * nt, tp + 3 * nt, c->stream);
            clustered_points(Lo, ps, ps, seed + 3, sp, sp + ns, sp + 2 * ns, sp + 3 * ns, c->stream);
            check_launch("clustered points");
            build_tree_ts_impl(t, FMM_F32, nt, tp, tp + nt, tp + 2 * nt, ns, sp, sp + ns, sp + 2 * ns, sp + 3 * ns,
                               std::max(per, ps));
            timed(FMM_POLICY_FMM, tf, 2);
            Meas mp2p = meas(lg(tf[PH_P2P], t->nlist[2]), 2);
            if (sj == si) {
                ts_diag[0] = mp2p.v;
                continue;
            }
            mp2p.v += Tp2p[si].v - ts_diag[0];
            Op2p[si * NS + sj] = mp2p;
        }
    }
    // Records over the whole feature grid the traversal asks about: log2 n_t
    // and log2 n_s in 0..20, the level differences, two distance-ratio bins.
    // Measured: the diagonal (n_t = n_s, equal levels; mixed levels for M2L)
    // and P2P at n_s = n_t / 4 and 4 n_t (anchored as above).  The
    // rest follows from how each kernel's work scales, stated here as the
    // model's invariances: no kernel's work depends on the distance ratio;
    // M2L's does not depend on the particle counts, nor M2P's on n_s; at
    // fixed n_t, P2P's log cost is linear in log n_s between the measured
    // points n_t / 4, n_t and 4 n_t (the measured slope on each side), and
    // beyond them grows as n_s (slope 1); outside the measured leaf sizes
    // P2P's and M2P's costs grow as n_t (and P2P's as n_s) from the nearest
    // measured size, and below it the per-pair overheads dominate (the
    // smallest measured costs stand).  The network is thus anchored wherever
    // the table is read instead of extrapolating (left alone there, it once
    // sent cells of a million particles to particle-particle sums).
    auto nearest = [&](const std::vector<Meas>& T, int i) {
        for (int d = 0; d < NS; d++) {
            if (i - d >= 0 && std::isfinite(T[i - d].v)) return T[i - d];
            if (i + d < NS && std::isfinite(T[i + d].v)) return T[i + d];
        }
        return Meas{};
    };
    const int lb = (int)std::lround(std::log2((double)pers[0]));
    const int lt = (int)std::lround(std::log2((double)pers[NS - 1]));
    // log2 cost of a cell pair with 2^a targets and 2^b sources, kind P2P
    // (p2p = true) or M2P, from the diagonal D and the off-diagonal points O
    auto cost = [&](const std::vector<Meas>& D, const std::vector<Meas>& O, int a, int b, bool p2p) {
        const int ca = std::min(std::max(a, lb), lt), i = ca - lb;
        const double d = nearest(D, i).v;
        const int db = b - ca;                          // log2 n_s - log2 n_t at the measured size
        const int near = std::max(-2, std::min(2, db)); // within the measured points
        double v = d;
        if (near != 0) {
            const int j = i + (near > 0 ? 2 : -2);
            double o = (j >= 0 && j < NS) ? O[i * NS + j].v : NAN;
            if (!std::isfinite(o)) o = p2p ? d + (near > 0 ? 2.0 : -2.0) * 0.5 : d;
            v = d + (o - d) * std::abs(near) / 2.0;
        }
        if (p2p) v += (double)(db - near);           // beyond: work ~ n_s
        if (a > lt) v += (double)(a - lt);            // larger target cells: work ~ n_t
        return v;
    };
    auto emit = [&](int dl, int a, int b, int kind, double v) {
        if (!std::isfinite(v)) return;
        for (int bq : {0, kMlpBq - 1}) {
            float f[6];
            mlp_features(f, dl, std::ldexp(1.0, a), std::ldexp(1.0, b), p, theta);
            f[4] = ((float)bq + 0.5f) / (float)kMlpBq;
            c->rec_feat.insert(c->rec_feat.end(), f, f + 6);
            c->rec_kind.push_back(kind);
            c->rec_tgt.push_back((float)v);
        }
    };
    const int dls[] = {-4, -2, -1, 0, 1, 2, 4};
    for (int a = 0; a <= 20; a++)
        for (int b = 0; b <= 20; b++)
            for (int dl : dls) {
                const int i = std::min(std::max(a, lb), lt) - lb;
                emit(dl, a, b, 0, (dl == 0 ? nearest(Tm2l, i) : nearest(Tgen, i)).v);
                emit(dl, a, b, 1, cost(Tm2p, Om2p, a, b, false));
                emit(dl, a, b, 2, cost(Tp2p, Op2p, a, b, true));
            }
}

static void mlp_init(std::vector<float>& w, uint64_t seed, float out_bias) {
    w.assign(kMlpParams, 0.f);
    uint64_t s = seed;
    auto uni = [&]() {
        s += 0x9E3779B97F4A7C15ull;
        uint64_t z = s;
        z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
        z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
        z ^= z >> 31;
        return (double)(z >> 11) * (1.0 / 9007199254740992.0) * 2.0 - 1.0;
    };
    const int H = 64, F = 6;
    for (int i = 0; i < H * F; i++) w[i] = (float)(uni() * std::sqrt(6.0 / F));
    for (int i = 0; i < H * H; i++) w[H * F + H + i] = (float)(uni() * std::sqrt(6.0 / H));
    for (int i = 0; i < 3 * H; i++) w[H * F + H + H * H + H + i] = (float)(uni() * std::sqrt(6.0 / H));
    for (int j = 0; j < 3; j++) w[kMlpParams - 3 + j] = out_bias;
}

static double mlp_fit(fmm_ctx c, int B, const float* feat, const int32_t* kind, const float* tgt, int epochs,
                      double lr, uint64_t seed) {
    if (B <= 0) fail(FMM_ERR_INVALID_ARG, "no training records");
    for (int r = 0; r < B; r++)
        if (kind[r] < 0 || kind[r] > 2) fail(FMM_ERR_INVALID_ARG, "record kind out of range");
    double mean = 0;
    for (int r = 0; r < B; r++) mean += tgt[r] / B;
    std::vector<float> w;
    mlp_init(w, seed, (float)mean);
    float* dw = need<float>(c, c->d_mlp, kMlpParams);
    float* dm = need<float>(c, c->d_mlp_m, kMlpParams);
    float* dv = need<float>(c, c->d_mlp_v, kMlpParams);
    float* dg = need<float>(c, c->d_grad, kMlpParams + 4);
    float* dgr = need<float>(c, c->d_grad_rec, (size_t)B * kMlpParams);
    float* dlr = need<float>(c, c->d_loss_rec, B);
    float* df = need<float>(c, c->d_feat, (size_t)B * 6);
    int32_t* dk = need<int32_t>(c, c->d_kind, B);
    float* dt = need<float>(c, c->d_tgt, B);
    to_dev(c, dw, w.data(), kMlpParams);
    fill_zero(dm, kMlpParams * 4, c->stream);
    fill_zero(dv, kMlpParams * 4, c->stream);
    to_dev(c, df, feat, (size_t)B * 6);
    to_dev(c, dk, kind, B);
    to_dev(c, dt, tgt, B);
    // Adam with a cosine-decayed step: lr at the first epoch, lr / 20 at the last
    for (int e = 1; e <= epochs; e++) {
        const double decay = 0.05 + 0.95 * 0.5 * (1.0 + std::cos(M_PI * (double)(e - 1) / (double)epochs));
        mlp_grad(dw, df, dk, dt, B, dgr, dlr, dg, dg + kMlpParams, c->stream);
        mlp_adam(dw, dm, dv, dg, e, (float)(lr * decay), c->stream);
    }
    mlp_grad(dw, df, dk, dt, B, dgr, dlr, dg, dg + kMlpParams, c->stream);
    check_launch("cost model training");
    float loss = 0;
    to_host<float>(c, &loss, dg + kMlpParams, 1);
    c->mlp_ready = true;
    c->mlp_version++;
    return loss;
}

fmm_status fmm_costmodel_train(fmm_ctx c, int32_t p, double theta, int32_t precision, int32_t epochs,
                               uint64_t seed, double* final_loss) {
    return guarded(c, [&] {
        if (p < 0 || p > FMM_P_MAX) fail(FMM_ERR_INVALID_ARG, "p out of range");
        if (!(theta > 0.0 && theta < 1.0)) fail(FMM_ERR_INVALID_ARG, "theta must lie in (0, 1)");
        if (epochs < 1) fail(FMM_ERR_INVALID_ARG, "epochs must be >= 1");
        if (precision != FMM_PREC_FP32 && precision != FMM_PREC_SPLIT_BF16)
            fail(FMM_ERR_UNSUPPORTED, "training is implemented for FP32 and split-BF16");
        if (precision == FMM_PREC_SPLIT_BF16 && !m2l_bf16_supported(p))
            fail(FMM_ERR_UNSUPPORTED, "split-BF16 M2L is implemented for p <= 12");
        auto t0 = std::chrono::steady_clock::now();
        gen_records(c, p, theta, precision, seed);
        double l = mlp_fit(c, (int)c->rec_kind.size(), c->rec_feat.data(), c->rec_kind.data(), c->rec_tgt.data(),
                           epochs, 3e-2, seed);
        c->cm_p = p;
        c->cm_theta = theta;
        c->cm_precision = precision;
        c->cm_loss = l;
        c->cm_records = (int)c->rec_kind.size();
        c->cm_seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
        if (final_loss) *final_loss = l;
    });
}

fmm_status fmm_costmodel_fit(fmm_ctx c, int32_t n_rec, const float* features, const int32_t* kinds,
                             const float* targets, int32_t epochs, double lr, uint64_t seed, double* final_loss) {
    return guarded(c, [&] {
        if (n_rec < 1 || !features || !kinds || !targets) fail(FMM_ERR_INVALID_ARG, "bad records");
        if (epochs < 1 || !(lr > 0)) fail(FMM_ERR_INVALID_ARG, "bad optimiser settings");
        double l = mlp_fit(c, n_rec, features, kinds, targets, epochs, lr, seed);
        c->cm_p = -1;
        c->cm_theta = -1;
        c->cm_precision = -1;
        c->cm_loss = l;
        c->cm_records = n_rec;
        c->cm_seconds = NAN;
        if (final_loss) *final_loss = l;
    });
}

fmm_status fmm_costmodel_records(fmm_ctx c, int32_t cap, int32_t* count, float* features, int32_t* kinds,
                                 float* targets) {
    return guarded(c, [&] {
        int32_t m = (int32_t)c->rec_kind.size();
        if (count) *count = m;
        int32_t k = std::min(cap, m);
        for (int32_t i = 0; i < k; i++) {
            if (features)
                for (int j = 0; j < 6; j++) features[6 * i + j] = c->rec_feat[6 * i + j];
            if (kinds) kinds[i] = c->rec_kind[i];
            if (targets) targets[i] = c->rec_tgt[i];
        }
    });
}

fmm_status fmm_costmodel_get_weights(fmm_ctx c, float* w) {
    return guarded(c, [&] {
        if (!w) fail(FMM_ERR_INVALID_ARG, "null pointer");
        if (!c->mlp_ready) fail(FMM_ERR_STATE, "no cost model");
        to_host<float>(c, w, c->d_mlp.p, kMlpParams);
    });
}

fmm_status fmm_costmodel_set_weights(fmm_ctx c, const float* w) {
    return guarded(c, [&] {
        if (!w) fail(FMM_ERR_INVALID_ARG, "null pointer");
        for (int i = 0; i < kMlpParams; i++)
            if (!std::isfinite(w[i])) fail(FMM_ERR_INVALID_ARG, "non-finite weight");
        to_dev(c, need<float>(c, c->d_mlp, kMlpParams), w, kMlpParams);
        c->mlp_ready = true;
        c->mlp_version++;
        c->cm_p = -1;
        c->cm_theta = -1;
        c->cm_precision = -1;
        c->cm_loss = NAN;
        c->cm_records = 0;
        c->cm_seconds = NAN;
    });
}

namespace {
// the device a cost model was timed on: architecture and compute-unit count
std::string device_key(int device) {
    hipDeviceProp_t prop;
    ck(hipGetDeviceProperties(&prop, device), "hipGetDeviceProperties");
    std::string arch = prop.gcnArchName;
    size_t colon = arch.find(':');
    if (colon != std::string::npos) arch = arch.substr(0, colon);
    return arch + "/" + std::to_string(prop.multiProcessorCount) + "cu";
}

const char kModelMagic[] = "fmm-costmodel";
const int kModelVersion = 1;
}  // namespace

fmm_status fmm_costmodel_save(fmm_ctx c, const char* path) {
    return guarded(c, [&] {
        if (!path) fail(FMM_ERR_INVALID_ARG, "null path");
        if (!c->mlp_ready) fail(FMM_ERR_STATE, "no cost model");
        std::vector<float> w(kMlpParams);
        to_host<float>(c, w.data(), c->d_mlp.p, kMlpParams);
        std::string tmp = std::string(path) + ".tmp";
        FILE* f = std::fopen(tmp.c_str(), "w");
        if (!f) fail(FMM_ERR_DEVICE, std::string("cannot write ") + path);
        std::fprintf(f, "%s %d\n", kModelMagic, kModelVersion);
        std::fprintf(f, "device %s\n", device_key(c->device).c_str());
        std::fprintf(f, "p %d\ntheta %a\nprecision %d\n", c->cm_p, c->cm_theta, c->cm_precision);
        std::fprintf(f, "loss %a\nrecords %d\ntraining_seconds %a\n", c->cm_loss, c->cm_records, c->cm_seconds);
        if (c->costs_set) std::fprintf(f, "costs %a %a %a\n", c->costs[0], c->costs[1], c->costs[2]);
        else std::fprintf(f, "costs none\n");
        std::fprintf(f, "p2p_tpl");
        for (int k = 0; k < kLeafClasses; k++) std::fprintf(f, " %d", c->p2p_tpl[k]);
        std::fprintf(f, "\nschedule %d\nm2l_kernel %d\nm2l_tile %d\nweights %d\n", c->schedule, c->m2l_kind, c->gemm_nt,
                     kMlpParams);
        for (int i = 0; i < kMlpParams; i++) std::fprintf(f, "%a%c", (double)w[i], (i % 8 == 7) ? '\n' : ' ');
        std::fprintf(f, "\nend\n");
        bool ok = std::ferror(f) == 0;
        ok = (std::fclose(f) == 0) && ok;
        if (!ok || std::rename(tmp.c_str(), path) != 0) {
            std::remove(tmp.c_str());
            fail(FMM_ERR_DEVICE, std::string("cannot write ") + path);
        }
    });
}

fmm_status fmm_costmodel_load(fmm_ctx c, const char* path, int32_t p, int32_t precision) {
    return guarded(c, [&] {
        if (!path) fail(FMM_ERR_INVALID_ARG, "null path");
        FILE* f = std::fopen(path, "r");
        if (!f) fail(FMM_ERR_INVALID_ARG, std::string("cannot read ") + path);
        struct Close {
            FILE* f;
            ~Close() { std::fclose(f); }
        } cl{f};
        auto bad = [&](const char* what) { fail(FMM_ERR_INVALID_ARG, std::string(path) + ": " + what); };
        char word[64], dev[256];
        int ver = 0;
        if (std::fscanf(f, "%63s %d", word, &ver) != 2 || std::strcmp(word, kModelMagic) != 0) bad("not a cost model");
        if (ver != kModelVersion) bad("unsupported format version");
        if (std::fscanf(f, " device %255s", dev) != 1) bad("missing device");
        int mp = -1, mprec = -1, nrec = 0, nw = 0, sched = 0;
        double mth = -1, loss = NAN, secs = NAN;
        if (std::fscanf(f, " p %d theta %la precision %d loss %la records %d training_seconds %la", &mp, &mth, &mprec,
                        &loss, &nrec, &secs) != 6)
            bad("malformed header");
        double cst[3] = {0, 0, 0};
        bool has_costs = false;
        char cw[32];
        if (std::fscanf(f, " costs %31s", cw) != 1) bad("missing costs");
        if (std::strcmp(cw, "none") != 0) {
            cst[0] = std::strtod(cw, nullptr);
            if (std::fscanf(f, "%la %la", &cst[1], &cst[2]) != 2) bad("malformed costs");
            has_costs = true;
            for (double v : cst)
                if (!(v > 0) || !std::isfinite(v)) bad("unit costs must be > 0");
        }
        int tpl[kLeafClasses];
        if (std::fscanf(f, " p2p_tpl") != 0) bad("missing tile shapes");
        for (int k = 0; k < kLeafClasses; k++)
            if (std::fscanf(f, "%d", &tpl[k]) != 1 || !p2p_shape_ok(tpl[k])) bad("bad tile shapes");
        if (std::fscanf(f, " schedule %d", &sched) != 1 || sched < 0 || sched > 2) bad("bad schedule");
        // the M2L kind line is optional (files written before it existed lack it)
        int mkind = -1, mtile = -1;
        if (std::fscanf(f, " %63s", word) != 1) bad("truncated file");
        if (std::strcmp(word, "m2l_kernel") == 0) {
            if (std::fscanf(f, "%d", &mkind) != 1 || mkind < FMM_M2L_CLASS_DENSE || mkind > FMM_M2L_PAIR_ROTATION)
                bad("bad M2L kernel");
            if (std::fscanf(f, " %63s", word) != 1) bad("truncated file");
        }
        if (std::strcmp(word, "m2l_tile") == 0) {
            if (std::fscanf(f, "%d", &mtile) != 1 || (mtile != 0 && mtile != 64 && mtile != 128)) bad("bad M2L tile");
            if (std::fscanf(f, " %63s", word) != 1) bad("truncated file");
        }
        if (std::strcmp(word, "weights") != 0 || std::fscanf(f, "%d", &nw) != 1) bad("missing weights");
        if (nw != kMlpParams) bad("weight count does not match this network");
        std::vector<float> w(kMlpParams);
        for (int i = 0; i < kMlpParams; i++) {
            double v;
            if (std::fscanf(f, "%la", &v) != 1 || !std::isfinite(v)) bad("malformed weights");
            w[i] = (float)v;
        }
        if (std::fscanf(f, " %63s", word) != 1 || std::strcmp(word, "end") != 0) bad("truncated file");
        const std::string here = device_key(c->device);
        if (here != dev) bad((std::string("trained on ") + dev + ", this device is " + here).c_str());
        if (p >= 0 && p != mp) bad(("trained for p = " + std::to_string(mp) + ", not " + std::to_string(p)).c_str());
        if (precision >= 0 && precision != mprec)
            bad(("trained for precision " + std::to_string(mprec) + ", not " + std::to_string(precision)).c_str());
        to_dev(c, need<float>(c, c->d_mlp, kMlpParams), w.data(), kMlpParams);
        c->mlp_ready = true;
        c->mlp_version++;
        c->cm_p = mp;
        c->cm_theta = mth;
        c->cm_precision = mprec;
        c->cm_loss = loss;
        c->cm_records = nrec;
        c->cm_seconds = secs;
        if (has_costs) {
            for (int k = 0; k < 3; k++) c->costs[k] = cst[k];
            c->costs_set = true;
            c->costs_version++;
        }
        for (int k = 0; k < kLeafClasses; k++) c->p2p_tpl[k] = tpl[k];
        c->schedule = sched;
        if (mkind >= 0) c->m2l_kind = mkind;
        if (mtile >= 0) c->gemm_nt = mtile;
    });
}

fmm_status fmm_set_allocator(fmm_ctx c, fmm_alloc_fn alloc, fmm_free_fn free_fn, void* user) {
    return guarded(c, [&] {
        if ((alloc == nullptr) != (free_fn == nullptr)) fail(FMM_ERR_INVALID_ARG, "set both routines or neither");
        c->ualloc = alloc;
        c->ufree = free_fn;
        c->uuser = alloc ? user : nullptr;
    });
}

fmm_status fmm_m2l_slots(int32_t p, double theta, int32_t* slots, int32_t* batched) {
    if (p < 0 || p > FMM_P_MAX || !(theta > 0.0 && theta < 1.0)) return FMM_ERR_INVALID_ARG;
    try {
        const int J = m2l_plan_slots(theta);
        if (slots) *slots = J;
        if (batched) *batched = (m2l_gemm_supported(p) && J <= kGemmMaxSlots) ? 1 : 0;
    } catch (...) {
        return FMM_ERR_OUT_OF_MEMORY;
    }
    return FMM_OK;
}

fmm_status fmm_costmodel_loss_grad(fmm_ctx c, const float* w, int32_t n_rec, const float* features,
                                   const int32_t* kinds, const float* targets, float* loss, float* grad) {
    return guarded(c, [&] {
        if (!w || n_rec < 1 || !features || !kinds || !targets) fail(FMM_ERR_INVALID_ARG, "bad arguments");
        for (int r = 0; r < n_rec; r++)
            if (kinds[r] < 0 || kinds[r] > 2) fail(FMM_ERR_INVALID_ARG, "record kind out of range");
        const int B = n_rec;
        float* dw = need<float>(c, c->tune_out, kMlpParams);
        float* dg = need<float>(c, c->d_grad, kMlpParams + 4);
        float* dgr = need<float>(c, c->d_grad_rec, (size_t)B * kMlpParams);
        float* dlr = need<float>(c, c->d_loss_rec, B);
        float* df = need<float>(c, c->d_feat, (size_t)B * 6);
        int32_t* dk = need<int32_t>(c, c->d_kind, B);
        float* dt = need<float>(c, c->d_tgt, B);
        to_dev(c, dw, w, kMlpParams);
        to_dev(c, df, features, (size_t)B * 6);
        to_dev(c, dk, kinds, B);
        to_dev(c, dt, targets, B);
        mlp_grad(dw, df, dk, dt, B, dgr, dlr, dg, dg + kMlpParams, c->stream);
        check_launch("cost model gradient");
        if (grad) to_host<float>(c, grad, dg, kMlpParams);
        if (loss) to_host<float>(c, loss, dg + kMlpParams, 1);
    });
}

fmm_status fmm_costmodel_table(fmm_ctx c, int32_t p, double theta, uint8_t* table) {
    return guarded(c, [&] {
        if (!table) fail(FMM_ERR_INVALID_ARG, "null pointer");
        if (!c->mlp_ready) fail(FMM_ERR_STATE, "no cost model");
        if (p < 0 || p > FMM_P_MAX || !(theta > 0.0 && theta < 1.0)) fail(FMM_ERR_INVALID_ARG, "bad p or theta");
        uint8_t* d = need<uint8_t>(c, c->d_table, kMlpTable);
        mlp_table((const float*)c->d_mlp.p, p, (float)theta, c->costs_set ? c->costs : nullptr, d, c->stream);
        check_launch("cost model table");
        c->table_p = p;
        c->table_theta = theta;
        c->table_version = c->mlp_version;
        c->table_costs_version = c->costs_version;
        to_host<uint8_t>(c, table, d, kMlpTable);
    });
}

fmm_status fmm_get_sizes(fmm_ctx c, int64_t* n_cells, int64_t* n_m2l, int64_t* n_m2p, int64_t* n_p2p) {
    return guarded(c, [&] {
        if (n_cells) *n_cells = c->built ? c->ncell : 0;
        if (n_m2l) *n_m2l = c->traversed ? c->nlist[0] : 0;
        if (n_m2p) *n_m2p = c->traversed ? c->nlist[1] : 0;
        if (n_p2p) *n_p2p = c->traversed ? c->nlist[2] : 0;
    });
}

fmm_status fmm_get_work(fmm_ctx c, int64_t* p2p_particle_pairs, int64_t* m2p_targets) {
    return guarded(c, [&] {
        if (!c->traversed) fail(FMM_ERR_STATE, "no traversal");
        uint64_t* d = (uint64_t*)need<double>(c, c->small, 32) + 28;
        uint64_t h[2] = {0, 0};
        if (p2p_particle_pairs) {
            pair_work((uint32_t*)c->tgt[2].p, (uint32_t*)c->src[2].p, c->nlist[2], cells_of(c), 1, d, c->stream);
            check_launch("work count");
            to_host<uint64_t>(c, h, d, 1);
            *p2p_particle_pairs = (int64_t)h[0];
        }
        if (m2p_targets) {
            pair_work((uint32_t*)c->tgt[1].p, (uint32_t*)c->src[1].p, c->nlist[1], cells_of(c), 0, d, c->stream);
            check_launch("work count");
            to_host<uint64_t>(c, h + 1, d, 1);
            *m2p_targets = (int64_t)h[1];
        }
    });
}

fmm_status fmm_get_m2l_split(fmm_ctx c, int64_t* n_batched, int64_t* n_general) {
    return guarded(c, [&] {
        if (!c->traversed) fail(FMM_ERR_STATE, "no traversal");
        if (n_batched) *n_batched = c->nlist[0] - c->ngeneral;
        if (n_general) *n_general = c->ngeneral;
    });
}

fmm_status fmm_get_bbox(fmm_ctx c, double* lo3, double* side) {
    return guarded(c, [&] {
        if (!c->built) fail(FMM_ERR_STATE, "no tree");
        if (!lo3 || !side) fail(FMM_ERR_INVALID_ARG, "null pointer");
        for (int d = 0; d < 3; d++) lo3[d] = c->lo[d];
        *side = c->side;
    });
}

fmm_status fmm_get_gemm_shape(fmm_ctx c, int64_t* tiles, int64_t* slots, int64_t* active_slots) {
    return guarded(c, [&] {
        if (!c->traversed) fail(FMM_ERR_STATE, "no traversal");
        const int64_t nt = c->gemm_on ? c->ntiles : 0;
        int64_t a = 0;
        if (nt > 0) {
            std::vector<int32_t> h(nt);
            to_host<int32_t>(c, h.data(), c->tnact.p, nt);
            for (int32_t v : h) a += v;
        }
        if (tiles) *tiles = nt;
        if (slots) *slots = nt * (c->gemm_on ? c->gp.J : 0);
        if (active_slots) *active_slots = a;
    });
}

fmm_status fmm_get_bboxes(fmm_ctx c, int32_t n_inst, double* lo_side) {
    return guarded(c, [&] {
        if (!c->built) fail(FMM_ERR_STATE, "no tree");
        if (!lo_side || n_inst < 0 || (size_t)n_inst > c->frames.size()) fail(FMM_ERR_INVALID_ARG, "bad n_inst");
        for (int32_t k = 0; k < n_inst; k++) {
            const Frame& f = c->frames[k];
            lo_side[4 * k + 0] = f.lox;
            lo_side[4 * k + 1] = f.loy;
            lo_side[4 * k + 2] = f.loz;
            lo_side[4 * k + 3] = f.side;
        }
    });
}

fmm_status fmm_get_keys(fmm_ctx c, uint64_t* keys, int32_t* perm) {
    return guarded(c, [&] {
        if (!c->built) fail(FMM_ERR_STATE, "no tree");
        if (c->n == 0) return;
        if (keys) to_host<uint64_t>(c, keys, c->keys.p, c->n);
        if (perm) to_host<int32_t>(c, perm, c->idx.p, c->n);
    });
}

fmm_status fmm_get_cells(fmm_ctx c, int32_t* level, uint64_t* prefix, int32_t* begin, int32_t* end, int32_t* parent,
                         int32_t* first_child, int32_t* nchild, int32_t* centre_h, int32_t* radius_h) {
    return guarded(c, [&] {
        if (!c->built) fail(FMM_ERR_STATE, "no tree");
        size_t m = c->ncell;
        if (m == 0) return;
        if (level) to_host<int32_t>(c, level, c->c_level.p, m);
        if (prefix) to_host<uint64_t>(c, prefix, c->c_prefix.p, m);
        if (begin) to_host<int32_t>(c, begin, c->c_begin.p, m);
        if (end) to_host<int32_t>(c, end, c->c_end.p, m);
        if (parent) to_host<int32_t>(c, parent, c->c_parent.p, m);
        if (first_child) to_host<int32_t>(c, first_child, c->c_child.p, m);
        if (nchild) to_host<int32_t>(c, nchild, c->c_nchild.p, m);
        if (centre_h || radius_h) {
            std::vector<int4> g(m);
            to_host<int4>(c, g.data(), c->c_geo.p, m);
            for (size_t i = 0; i < m; i++) {
                if (centre_h) {
                    centre_h[3 * i] = g[i].x;
                    centre_h[3 * i + 1] = g[i].y;
                    centre_h[3 * i + 2] = g[i].z;
                }
                if (radius_h) radius_h[i] = g[i].w;
            }
        }
    });
}

// Consistency checks of the context's tree, lists and GEMM tables on host
// copies (a debugging aid: every index the kernels follow is checked against
// the array it indexes).
fmm_status fmm_validate(fmm_ctx c) {
    return guarded(c, [&] {
        if (!c->built) fail(FMM_ERR_STATE, "no tree");
        const int64_t n = c->n;
        const int32_t nc = c->ncell;
        auto bad = [&](const std::string& what) { fail(FMM_ERR_STATE, ("validate: " + what).c_str()); };
        // the permutation and, for one instance, the key order
        if (n > 0) {
            std::vector<uint32_t> idx(n);
            std::vector<uint64_t> key(n);
            to_host<uint32_t>(c, idx.data(), c->idx.p, n);
            to_host<uint64_t>(c, key.data(), c->keys.p, n);
            std::vector<uint8_t> seen(n, 0);
            for (int64_t i = 0; i < n; i++) {
                if (idx[i] >= (uint64_t)n || seen[idx[i]]) bad("permutation is not a permutation");
                seen[idx[i]] = 1;
            }
            if (c->hseg.size() == 2)
                for (int64_t i = 1; i < n; i++)
                    if (key[i] < key[i - 1]) bad("keys out of order at " + std::to_string(i));
        }
        std::vector<int32_t> b(nc), e(nc), par(nc), ch(nc), nch(nc), lev(nc);
        if (nc > 0) {
            to_host<int32_t>(c, b.data(), c->c_begin.p, nc);
            to_host<int32_t>(c, e.data(), c->c_end.p, nc);
            to_host<int32_t>(c, par.data(), c->c_parent.p, nc);
            to_host<int32_t>(c, ch.data(), c->c_child.p, nc);
            to_host<int32_t>(c, nch.data(), c->c_nchild.p, nc);
            to_host<int32_t>(c, lev.data(), c->c_level.p, nc);
        }
        int32_t leaves = 0;
        for (int32_t i = 0; i < nc; i++) {
            const std::string at = " (cell " + std::to_string(i) + ")";
            if (!(0 <= b[i] && b[i] < e[i] && e[i] <= n)) bad("empty or out-of-range particle range" + at);
            if (lev[i] < 0 || lev[i] > kMaxLevel) bad("level out of range" + at);
            if (i < c->nroot) {
                if (par[i] != -1 || lev[i] != 0) bad("root with a parent or a level" + at);
            } else if (par[i] < 0 || par[i] >= i || lev[i] != lev[par[i]] + 1) {
                bad("parent not an earlier cell one level up" + at);
            }
            if (nch[i] < 0 || nch[i] > 8) bad("child count out of range" + at);
            if (nch[i] == 0) {
                leaves++;
                continue;
            }
            if (ch[i] <= i || (int64_t)ch[i] + nch[i] > nc) bad("children out of range" + at);
            int32_t at_p = b[i];
            for (int32_t k = ch[i]; k < ch[i] + nch[i]; k++) {
                if (par[k] != i || b[k] != at_p) bad("children do not partition the parent" + at);
                at_p = e[k];
            }
            if (at_p != e[i]) bad("children do not cover the parent" + at);
        }
        if (leaves != c->nleaf) bad("leaf count " + std::to_string(leaves) + " != " + std::to_string(c->nleaf));
        if (!c->traversed) return;
        for (int k = 0; k < 3; k++) {
            const int64_t m = c->nlist[k];
            if (m == 0) continue;
            std::vector<int2> pr(m);
            to_host<int2>(c, pr.data(), c->raw[k].p, m);
            for (int64_t i = 0; i < m; i++)
                if (pr[i].x < 0 || pr[i].x >= nc || pr[i].y < 0 || pr[i].y >= nc)
                    bad("list " + std::to_string(k) + " pair " + std::to_string(i) + " out of range");
            if (k == 0) continue;
            std::vector<uint32_t> tg(m);
            std::vector<int32_t> of((size_t)nc + 1);
            to_host<uint32_t>(c, tg.data(), c->tgt[k].p, m);
            to_host<int32_t>(c, of.data(), c->off[k].p, (size_t)nc + 1);
            for (int64_t i = 1; i < m; i++)
                if (tg[i] < tg[i - 1]) bad("list " + std::to_string(k) + " not grouped by target");
            if (of[0] != 0 || of[nc] != m) bad("list " + std::to_string(k) + " offsets do not span the list");
            for (int32_t i = 0; i < nc; i++)
                if (of[i] > of[i + 1]) bad("list " + std::to_string(k) + " offsets not monotone");
        }
        if (c->gemm_on && c->gp.ntiles > 0) {
            const int64_t ng = (int64_t)c->gp.ntiles * c->gp.nt * c->gp.J;
            std::vector<int32_t> ga(ng);
            to_host<int32_t>(c, ga.data(), c->gather.p, ng);
            for (int64_t i = 0; i < ng; i++)
                if (ga[i] < -1 || ga[i] >= nc) bad("gather entry out of range");
            for (int k = 0; k < 8; k++)
                if (c->gp.class_row0[k] > c->gp.class_row0[k + 1]) bad("GEMM class rows not monotone");
            if (c->gp.class_row0[8] != c->gp.nrows || c->gp.nrows > nc) bad("GEMM rows out of range");
        }
    });
}

fmm_status fmm_get_list(fmm_ctx c, int32_t kind, int32_t* tgt, int32_t* src) {
    return guarded(c, [&] {
        if (!c->traversed) fail(FMM_ERR_STATE, "no traversal");
        if (kind < 0 || kind > 2) fail(FMM_ERR_INVALID_ARG, "unknown list kind");
        size_t m = c->nlist[kind];
        if (m == 0) return;
        if (kind == 0 && !c->m2l_sorted) {
            // the cell-cell list is grouped by target only on request
            void* ws = need<char>(c, c->ws, std::max(sort_ws_bytes(m), c->ws.cap));
            uint32_t* tg = need<uint32_t>(c, c->tgt[0], m + 1);
            uint32_t* sr = need<uint32_t>(c, c->src[0], m + 1);
            split_pairs((int2*)c->raw[0].p, m, tg, sr, c->stream);
            sort_u32(tg, sr, need<uint32_t>(c, c->tgt2, m), need<uint32_t>(c, c->src2, m), m, 0,
                     bits_for(c->ncell), ws, c->stream);
            check_launch("sort list");
            c->m2l_sorted = true;
        }
        if (tgt) to_host<int32_t>(c, tgt, c->tgt[kind].p, m);
        if (src) to_host<int32_t>(c, src, c->src[kind].p, m);
    });
}

fmm_status fmm_get_expansions(fmm_ctx c, float* mp, float* lc) {
    return guarded(c, [&] {
        if (!c->traversed || !c->M.p) fail(FMM_ERR_STATE, "no evaluation");
        int K = c_k(c), KP = c_kp(c);
        size_t m = c->ncell;
        std::vector<float> tmp(m * KP);
        if (mp) {
            to_host<float>(c, tmp.data(), c->M.p, m * KP);
            for (size_t i = 0; i < m; i++) std::memcpy(mp + i * K, tmp.data() + i * KP, K * sizeof(float));
        }
        if (lc) {
            to_host<float>(c, tmp.data(), c->L.p, m * KP);
            for (size_t i = 0; i < m; i++) std::memcpy(lc + i * K, tmp.data() + i * KP, K * sizeof(float));
        }
    });
}

fmm_status fmm_get_timings(fmm_ctx c, double* ms, int32_t cap, int32_t* count) {
    return guarded(c, [&] {
        if (!ms && cap > 0) fail(FMM_ERR_INVALID_ARG, "null pointer");
        int k = std::min<int>(cap, PH_N + 1);
        for (int i = 0; i < k; i++) ms[i] = i < PH_N ? c->ms[i] : c->ms_gemm_kernel;
        if (count) *count = k;
    });
}

fmm_status fmm_autotune(fmm_ctx c, int32_t precision, int32_t reps) {
    return guarded(c, [&] {
        if (!c->traversed) fail(FMM_ERR_STATE, "fmm_autotune before fmm_traverse");
        if (c->n == 0) return;
        reps = std::max(1, std::min(reps, 1000));
        hipStream_t s = c->stream;
        struct Ev {
            hipEvent_t a = nullptr, b = nullptr;
            ~Ev() {
                if (a) (void)hipEventDestroy(a);
                if (b) (void)hipEventDestroy(b);
            }
        } ev;
        ck(hipEventCreate(&ev.a), "hipEventCreate");
        ck(hipEventCreate(&ev.b), "hipEventCreate");
        auto timed = [&](auto&& work) {
            work();
            ck(hipEventRecord(ev.a, s), "event");
            for (int r = 0; r < reps; r++) work();
            ck(hipEventRecord(ev.b, s), "event");
            ck(hipEventSynchronize(ev.b), "event sync");
            float t = 0;
            ck(hipEventElapsedTime(&t, ev.a, ev.b), "elapsed");
            return (double)t / reps;
        };
        // tile shape per leaf-size class: targets per lane of the P2P kernel
        double4* nr = need<double4>(c, c->nearb, c->n);
        for (int k = 0; k < kLeafClasses; k++) {
            const int32_t b = c->leaf_cls[k], e = c->leaf_cls[k + 1];
            if (e <= b) continue;
            double best = INFINITY;
            for (int tpl : {1, 2, 4, -1, -2, -4}) {
                double t = timed([&] {
                    p2p((float4*)c->pts.p, cells_of(c), (int32_t*)c->leaves_cls.p + b, e - b, (int32_t*)c->off[2].p,
                        (uint32_t*)c->src[2].p, p2p_guard_all(c), tpl, nr, s);
                    check_launch("p2p");
                });
                if (t < best) {
                    best = t;
                    c->p2p_tpl[k] = tpl;
                }
            }
        }
        float* o = need<float>(c, c->at_out, (size_t)4 * c->n);
        const bool timing = c->timing;
        c->timing = false;
        // kernel of the M2L pairs outside the same-level GEMM: class-batched
        // matrix-core products or one pair at a time, dense or by rotation
        if (c->ngeneral > 0 && c->fam == kFamilySpherical) {
            double bestk = INFINITY;
            int pick = c->m2l_kind;
            for (int kind = FMM_M2L_CLASS_DENSE; kind <= FMM_M2L_PAIR_ROTATION; kind++) {
                c->m2l_kind = kind;
                build_classes(c, c->p);
                double t = timed([&] { evaluate_impl(c, precision, FMM_F32, o, o + c->n, o + 2 * c->n, o + 3 * c->n); });
                if (t < bestk) {
                    bestk = t;
                    pick = kind;
                }
            }
            c->m2l_kind = pick;
            build_classes(c, c->p);
        }
        // targets per tile of the same-level M2L GEMM (where the storage
        // width has more than one tiling; the tables are rebuilt on the same
        // lists for each) and schedule, timed together: how well the GEMM
        // shares the chip with a concurrent P2P depends on its tile
        std::vector<int> widths{0};  // 0: the current tables only
        if (c->gemm_on && c->gp.ntiles > 0 && gemm_tile_width_ok(c_kp(c), 64) && gemm_tile_width_ok(c_kp(c), 128))
            widths = {64, 128};
        double best = INFINITY;
        int pick = 0, pick_nt = 0;
        for (int nt : widths) {
            if (nt != 0 && nt != c->gp.nt) gemm_tiles(c, nt);
            for (int sc = 0; sc < 3; sc++) {
                c->schedule = sc;
                double t = timed([&] { evaluate_impl(c, precision, FMM_F32, o, o + c->n, o + 2 * c->n, o + 3 * c->n); });
                if (t < best) {
                    best = t;
                    pick = sc;
                    pick_nt = nt;
                }
            }
        }
        if (pick_nt != 0) {
            if (pick_nt != c->gp.nt) gemm_tiles(c, pick_nt);
            c->gemm_nt = pick_nt;
        }
        c->timing = timing;
        c->schedule = pick;
    });
}

fmm_status fmm_set_m2l_tile(fmm_ctx c, int32_t cols) {
    return guarded(c, [&] {
        if (cols != 0 && cols != 64 && cols != 128) fail(FMM_ERR_INVALID_ARG, "M2L tile width must be 0, 64 or 128");
        c->gemm_nt = cols;
    });
}

fmm_status fmm_get_m2l_tile(fmm_ctx c, int32_t* cols) {
    return guarded(c, [&] {
        if (!cols) fail(FMM_ERR_INVALID_ARG, "null pointer");
        *cols = c->gemm_on && c->gp.ntiles > 0 ? c->gp.nt : c->gemm_nt;
    });
}

fmm_status fmm_get_tile_config(fmm_ctx c, int32_t* p2p_tpl, int32_t* overlap) {
    return guarded(c, [&] {
        if (p2p_tpl)
            for (int k = 0; k < kLeafClasses; k++) p2p_tpl[k] = c->p2p_tpl[k];
        if (overlap) *overlap = c->schedule;
    });
}

fmm_status fmm_set_tile_config(fmm_ctx c, const int32_t* p2p_tpl) {
    return guarded(c, [&] {
        if (!p2p_tpl) fail(FMM_ERR_INVALID_ARG, "null pointer");
        for (int k = 0; k < kLeafClasses; k++)
            if (!p2p_shape_ok(p2p_tpl[k]))
                fail(FMM_ERR_INVALID_ARG, "P2P tile shape must be 1, 2 or 4 (vector ALUs) or -1, -2, -4 (matrix cores)");
        for (int k = 0; k < kLeafClasses; k++) c->p2p_tpl[k] = p2p_tpl[k];
    });
}

fmm_status fmm_set_overlap(fmm_ctx c, int32_t schedule) {
    return guarded(c, [&] {
        if (schedule < 0 || schedule > 2) fail(FMM_ERR_INVALID_ARG, "schedule must be 0, 1 or 2");
        c->schedule = schedule;
    });
}

fmm_status fmm_set_timing(fmm_ctx c, int32_t enabled) {
    return guarded(c, [&] { c->timing = enabled != 0; });
}

}  // extern "C"
