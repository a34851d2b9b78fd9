// fmm_internal.h -- device data layout and kernel launchers of the gfx950 FMM.
//
// Layout in HBM (all arrays indexed by sorted particle k or cell c):
//   pts[k]      float4 (x, y, z, q) in Morton order, FP32
//   keys[k]     uint64 Morton key;  perm[k] original index
//   cells       SoA: begin, end, parent, child (first child or -1), nchild,
//               level (int32), prefix (uint64), geo (int4: half-grid centre
//               x,y,z and half side r), ctr (double4: physical centre, r)
//   expansions  M[c][KP], L[c][KP] FP32, KP = (p+1)^2 rounded up to 32 with
//               zero padding; degree n at offset n*n as
//               [Re c_n^0, Re c_n^1, Im c_n^1, ..., Re c_n^n, Im c_n^n],
//               Greengard-Rokhlin normalisation, M scaled by r^-n, L by r^(n+1)
//   lists       (target, source) int32 pairs grouped by target; CSR offsets
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

#include "host_ops.h"

namespace fmm {

constexpr int kMaxP = 16;
constexpr int kMaxLevel = 21;
// expansion families: spherical harmonics (any p <= kMaxP) and Cartesian
// Taylor series (p <= kMaxPCart; cart.h)
constexpr int kFamilySpherical = 0, kFamilyCartesian = 1;
constexpr int kMaxPCart = 6;

struct CellArrays {
    int32_t* begin;
    int32_t* end;
    int32_t* parent;
    int32_t* child;
    int32_t* nchild;
    int32_t* level;
    uint64_t* prefix;
    int4* geo;       // half-grid centre (x, y, z) and half side r
    double4* ctr;    // physical centre (x, y, z) and half side r
};

inline int ncoef(int p) { return (p + 1) * (p + 1); }

// ------------------------------------------------------------------ utilities
// Exclusive prefix sums.  `total` (device, may be null) receives the sum.
size_t scan_ws_bytes(int64_t n);
void scan_u32(const uint32_t* in, uint32_t* out, uint32_t* total, int64_t n, void* ws,
              hipStream_t s);
void scan_u32x4(const uint4* in, uint4* out, uint4* total, int64_t n, void* ws, hipStream_t s);
// An element count held in device memory, *hi - *lo (lo may be null), written
// by an earlier kernel on the same stream.
struct DevCount {
    const uint32_t* hi;
    const uint32_t* lo;
    __device__ int64_t get() const { return (int64_t)*hi - (lo ? (int64_t)*lo : 0); }
};
// Exclusive scans of a device-held count of elements (at most the capacity of
// in/out); the total goes to *total (device).  Workspace: scan_dev_ws_bytes().
size_t scan_dev_ws_bytes();
void scan_u32_dev(const uint32_t* in, uint32_t* out, uint32_t* total, DevCount n, void* ws, hipStream_t s);
void scan_u32x4_dev(const uint4* in, uint4* out, uint4* total, DevCount n, void* ws, hipStream_t s);

// Stable LSD radix sort on key bits [bit0, bit1), 8 bits per pass.  Result in
// (keys_a, vals_a) on return; (keys_b, vals_b) is scratch of the same size.
size_t sort_ws_bytes(int64_t n);
void sort_u64(uint64_t* keys_a, uint32_t* vals_a, uint64_t* keys_b, uint32_t* vals_b, int64_t n,
              int bit0, int bit1, void* ws, hipStream_t s);
void sort_u32(uint32_t* keys_a, uint32_t* vals_a, uint32_t* keys_b, uint32_t* vals_b, int64_t n,
              int bit0, int bit1, void* ws, hipStream_t s);

void fill_i32(int32_t* p, int32_t v, int64_t n, hipStream_t s);
// zero `bytes` (a multiple of 4) from p (4-byte aligned) with a kernel, not a
// memset node, so that a captured graph replays it like any other launch
void fill_zero(void* p, size_t bytes, hipStream_t s);
// artificial particles for the kernel pre-calculation: uniform in [0,1)^3, charges +-1
void artificial_points(int64_t n, uint64_t seed, float* x, float* y, float* z, float* q, hipStream_t s);
void iota_u32(uint32_t* p, int64_t n, hipStream_t s);

// work area of fmm_evaluate_noalloc: one fixed array per device (k_noalloc.hip)
constexpr size_t kNoAllocScratchBytes = (size_t)64 << 20;
// look up this device's copy of the array (the device must be current)
hipError_t noalloc_setup(int device);
// its device address, or null before noalloc_setup succeeded on the device
void* noalloc_area(int device);

// ------------------------------------------------------------------ tree
// A batch of independent instances: instance k owns particles [seg[k],
// seg[k+1]) of the input (and, after the sort, of the sorted order).  Its
// frame is its bounding cube: lower corner, side, the 21-bit quantisation
// scale 2^21 / side and the half-grid unit side / 2^22.
struct Frame {
    double lox, loy, loz, side, scale, h, pad0, pad1;
};
// bbox: block b reduces particles [bt[2b], bt[2b+1]); instance k's blocks are
// [pb[k], pb[k+1]); out[6k..6k+6) = {lo x,y,z, hi x,y,z}; part holds 6 doubles
// per block; bad = count of non-finite values
void bbox(const void* x, const void* y, const void* z, int dtype, const int64_t* bt, int nblk,
          const int32_t* pb, int nseg, double* part, double* out, uint32_t* bad, hipStream_t s);
// keys from each particle's instance frame; inst (may be null) = instance of particle i
void morton_keys(const void* x, const void* y, const void* z, int dtype, int64_t n, const int64_t* seg, int nseg,
                 const Frame* fr, uint64_t* keys, uint32_t* idx, uint32_t* inst, hipStream_t s);
// batch sort, second pass: ik[k] = instance of the k-th key-sorted particle, iv[k] = k
void inst_keys(const uint32_t* idx, const uint32_t* inst, int64_t n, uint32_t* ik, uint32_t* iv, hipStream_t s);
void gather_sorted(const uint64_t* keys, const uint32_t* idx, const uint32_t* perm, int64_t n, uint64_t* keys2,
                   uint32_t* idx2, hipStream_t s);
void permute_points(const void* x, const void* y, const void* z, const void* q, int dtype,
                    int64_t n, const uint32_t* idx, float4* pts, hipStream_t s);
// one level of the adaptive tree: cells [c0, c1) = [lvl[L], lvl[L+1]) at
// level L, bounds read from device memory.  nsplit[c-c0] = number of
// children of cell c (0 if it does not split).
// bounds: [c1 - c0][7] octant boundaries of the cells that split (scratch);
// cap = cell capacity (every level is narrower)
void tree_count(const uint64_t* keys, CellArrays cells, const int32_t* lvl, int L, int32_t ncrit,
                uint32_t* nsplit, int32_t* bounds, int32_t cap, hipStream_t s);
// child_off = exclusive scan of nsplit, *nnew its total; children get ids
// c1 + child_off[c-c0]; writes lvl[L+2]; sets *ovf (and splits nothing) if
// the level would pass cap cells
void tree_emit(CellArrays cells, int32_t* lvl, int L, const uint32_t* nsplit, const uint32_t* child_off,
               const uint32_t* nnew, const int32_t* bounds, int32_t cap, uint32_t* ovf, hipStream_t s);
void cell_geometry(CellArrays cells, int32_t ncell, const int64_t* seg, int nseg, const Frame* fr, hipStream_t s);

// sum over (tgt, src) pairs of n_t * n_s (both = 1) or n_t (both = 0) into *out (device)
void pair_work(const uint32_t* tgt, const uint32_t* src, int64_t n, CellArrays cells, int both, uint64_t* out,
               hipStream_t s);

// ------------------------------------------------------------------ learned cost model
constexpr int kMlpParams = 6 * 64 + 64 + 64 * 64 + 64 + 3 * 64 + 3;  // 4803
// quantised feature grid read by the traversal: level difference in
// [-kMlpDl, kMlpDl], log2 of each particle count in steps of 1/kMlpNsub up to
// 2^20, and kMlpBq bins of ((r_t + r_s)/R)/theta in (0, 1]
constexpr int kMlpDl = 4, kMlpNsub = 4, kMlpBn = 20 * kMlpNsub + 1, kMlpBq = 4;
constexpr int kMlpTable = (2 * kMlpDl + 1) * kMlpBn * kMlpBn * kMlpBq;
constexpr int kMlpChunk = 32;  // training records per workgroup (partial gradients per chunk)
void mlp_grad(const float* w, const float* feat, const int32_t* kind, const float* tgt, int B, float* grad_rec,
              float* loss_rec, float* grad, float* loss, hipStream_t s);
void mlp_adam(float* w, float* m, float* v, const float* g, int step, float lr, hipStream_t s);
// returns the particle count; writes the particles if x is not null
int64_t clustered_points(int L, int per, int per_lo, uint64_t seed, float* x, float* y, float* z, float* q,
                         hipStream_t s);
// costs (may be null): timed unit costs for the entries whose two least
// predictions lie within kMlpFallbackMargin log2 units of each other
constexpr float kMlpFallbackMargin = 0.125f;
void mlp_table(const float* w, int p, float theta, const double* costs, uint8_t* table, hipStream_t s);

// ------------------------------------------------------------------ traversal
struct TravParams {
    double theta2;
    double theta;
    int policy;
    double c_m2l, c_m2p, c_p2p;
    const uint8_t* mlp_table;  // learned choices over the quantised feature grid, or null
    const uint8_t* nbucket;    // per cell: quantised log2 of its particle count (learned policy)
};
// per cell: the particle-count bucket of the learned cost model's feature grid
void cell_buckets(CellArrays cells, int32_t ncell, uint8_t* nbucket, hipStream_t s);
// per frontier pair: counts of new (M2L, M2P, P2P, SPLIT) pairs, and the kind
// of each child pair (2 bits each, at most 64 children, in emission order)
// The frontier size *nf, the lists' running totals tot[0..2] and the overflow
// bits live in device memory; cap_frontier sizes the fixed grids.
void trav_count(const int2* frontier, const uint32_t* nf, int64_t cap_frontier, CellArrays cells, TravParams tp,
                uint4* cnt, uint4* kinds, hipStream_t s);
// capacities of the three lists and of the next frontier, in pairs
struct TravCaps {
    int64_t m2l, m2p, p2p, next;
};
// emit at tot[k] + the scan offsets (total *add), then tot += *add, *nf =
// the next frontier's size and *levels += 1 if the frontier was not empty; an
// overflow sets bits in *ovf, writes nothing and sets *nf = 0
void trav_emit(const int2* frontier, uint32_t* nf, int64_t cap_frontier, CellArrays cells, const uint4* kinds,
               const uint4* off, uint32_t* tot, const uint4* add, TravCaps caps, int2* m2l, int2* m2p, int2* p2p,
               int2* next, uint32_t* ovf, uint32_t* levels, hipStream_t s);
void split_pairs(const int2* pairs, int64_t n, uint32_t* tgt, uint32_t* src, hipStream_t s);
// offsets[c] = first index in the sorted target array with target >= c, c in [0, ncell]
void csr_offsets(const uint32_t* tgt_sorted, int64_t n, int32_t ncell, int32_t* offsets,
                 hipStream_t s);

struct GemmPlan;

// M2L same-level batching: classify each M2L pair (emission order; the
// pairs as emitted, (target, source)); slot: per pair, its slot or -1.
//   slot_of   lookup table [8][(2R+1)^3] (offset -> slot or -1)
//   rowof     [ncell] tile * NT + column of the target's GEMM row, or -1
//   gather    [ntiles][NT][Jp] source cell or -1, as filled (per tile and
//             column, the column's slots contiguous, rows of Jp = J rounded
//             up to a multiple of 4; absent entries stay -1); tile_transpose
//             turns it into the GEMM's [ntiles][J][NT]
void m2l_mark_targets(const int2* pairs, int64_t n, CellArrays cells, const int32_t* slot_of, int R,
                      uint32_t* has_fast, int16_t* slot, hipStream_t s);
void m2l_fill_gather(const int2* pairs, const int16_t* slot, int64_t n, const int32_t* rowof, int32_t rowlen,
                     int32_t* gcol, hipStream_t s);
// row keys of the M2L GEMM: (octant class << kRowMissBits) | missing slots
// (densest first); cells without same-level pairs get class 8
constexpr int kRowMissBits = 10;
constexpr uint32_t kRowMissMax = (1u << kRowMissBits) - 1;
void row_class_keys(const uint32_t* nfast, CellArrays cells, int32_t ncell, int32_t J, uint32_t* key,
                    uint32_t* val, hipStream_t s);
// rowof[rowcell[r]] = tile * NT + column of GEMM row r (plan's class tables set)
void rows_inverse(const uint32_t* rowcell, int64_t nrows, GemmPlan plan, int NT, int32_t* rowof, hipStream_t s);
// keep the pairs whose slot is -1 (outside the GEMM tables), in order: they
// are counted per tile of 4096 (flag_counts, compact_tiles(n) counts), tbase =
// exclusive scan of the counts, then compact_pairs writes each tile's pairs
// from its base
int64_t compact_tiles(int64_t n);
void flag_counts(const int16_t* slot, int64_t n, uint32_t* cnt, hipStream_t s);
void compact_pairs(const int2* pairs, const int16_t* slot, const uint32_t* tbase, int64_t n, uint32_t* otgt,
                   uint32_t* osrc, hipStream_t s);
// out9[c] = first index of the sorted class keys with key >= c, c = 0..8
// out9[c] = first index whose key >> shift is >= c, c = 0..8
void class_bounds(const uint32_t* key_sorted, int64_t n, int shift, int32_t* out9, hipStream_t s);
// leaf cells (nchild == 0) in cell order; flag/pos are scratch of ncell entries
void leaf_flags(CellArrays cells, int32_t ncell, uint32_t* flag, hipStream_t s);
// targets != sources: flag[i] = 1 for the leaves (of the list) holding
// sorted particles below nt; out[pos[i]] = leaves[i] for the flagged ones
void target_leaf_flags(CellArrays cells, const int32_t* leaves, int32_t nleaf, int32_t nt, uint32_t* flag,
                       hipStream_t s);
void target_leaf_write(const int32_t* leaves, const uint32_t* flag, const uint32_t* pos, int32_t nleaf, int32_t* out,
                       hipStream_t s);
// leaves[pos[i]] = i for leaves, inner[i - pos[i]] = i for the other cells
void leaf_write(CellArrays cells, int32_t ncell, const uint32_t* pos, int32_t* leaves, int32_t* inner,
                hipStream_t s);

// ------------------------------------------------------------------ expansions
struct Tables {
    // all device pointers, FP32
    const float* m2m;    // [8][K][K] k-major (input index major)
    const float* l2l;    // [8][K][K] k-major
    const float* wm2l;   // [(p+1)(p+2)/2][K]  general M2L weights, (j,k) x (n, m+n)
    const float* gl2p;   // [2][K] gradient weights of L2P, (k) x (n, m+n)
    const float* hm2p;   // [2][K] gradient weights of M2P
    const float* rcoef;  // recurrence constants, see expansions kernels
    const float* wax;    // [p+1][p+1][p+1] axial M2L weights of the rotation-based M2L
};
void p2m(const float4* pts, CellArrays cells, const int32_t* leaves, int32_t nleaves, int family, int p,
         int KP, const float* rc, float* M, hipStream_t s);
// One level of octant translations: the parents are the non-leaf cells of
// cells [c0, c1) (one tree level), listed in `inner` (non-leaf cells in cell
// order); leafpos[i] = number of leaves among cells [0, i) (i < ncell), nleaf
// in all.  m2m: parents' multipoles from their children; l2l: children's
// locals += translated parent local.
// (K coefficients per cell, row stride KP)
void m2m(CellArrays cells, const int32_t* inner, const uint32_t* leafpos, int32_t c0, int32_t c1, int32_t ncell,
         int32_t nleaf, int K, int KP, Tables t, float* M, hipStream_t s);
void l2l(CellArrays cells, const int32_t* inner, const uint32_t* leafpos, int32_t c0, int32_t c1, int32_t ncell,
         int32_t nleaf, int K, int KP, Tables t, float* L, hipStream_t s);
// M2L of the pairs outside the batched GEMM, given as a CSR list by target,
// one pair at a time (pairs with skip[a] != 0 are left out; skip may be null)
void m2l_general(const int32_t* goff, const uint32_t* gsrc, CellArrays cells, int32_t ncell, int p, int KP,
                 Tables t, const float* M, float* L, const uint8_t* skip, hipStream_t s);

// The same pairs batched by class (level difference, integer offset): see k_m2l_cls.hip.
struct ClsPlan {
    int32_t ncls = 0, ntiles = 0, nbatched = 0, zcell = 0;
    const int32_t* tile_cls = nullptr;  // class of each tile
    const uint32_t* tbase = nullptr;    // first tile of each class
    const int32_t* start = nullptr;     // first sorted pair of each class, start[ncls] = nbatched
    const uint32_t* srcs = nullptr;     // source cell of each sorted pair
    const int32_t* pos = nullptr;       // sorted position of each pair of the list
};
int cls_tile_cols(int KP);
// key of each pair (class, or all ones when the offset does not fit); val = pair index
void cls_keys(const uint32_t* gt, const uint32_t* gs, int64_t ng, CellArrays cells, uint64_t* key, uint32_t* val,
              hipStream_t s);
void cls_heads(const uint64_t* key, int64_t n, uint32_t* head, hipStream_t s);
void cls_index(const uint32_t* head, const uint32_t* hoff, int64_t n, const uint32_t* val, const uint32_t* gs,
               int32_t* start, int32_t* pos, uint32_t* srcs, hipStream_t s);
// start[ncls] = first pair whose key does not fit (or n)
void cls_end(const uint64_t* key, int64_t n, int32_t* start, int32_t ncls, hipStream_t s);
void cls_ntiles(const int32_t* start, int32_t ncls, int NT, uint32_t* nt, hipStream_t s);
void cls_tiles(const uint32_t* nt, const uint32_t* tbase, int32_t ncls, int32_t* tile_cls, hipStream_t s);
// operators of all classes into T (ncls x KP x KP, zeroed beforehand)
void cls_ops(const uint64_t* key, const int32_t* start, int32_t ncls, int p, int KP, const float* W, float* T,
             hipStream_t s);
void cls_skip(const int32_t* pos, int64_t ng, int32_t nbatched, uint8_t* skip, hipStream_t s);
// the class GEMMs into part (nbatched x KP) and the per-target sums into L
void m2l_cls(const float* T, const ClsPlan& cp, int K, int KP, const float* M, float* part, const int32_t* goff,
             int32_t ncell, float* L, hipStream_t s);
// m2pflag: scratch of nleaves bytes; n_m2p: cell-particle pairs in the list;
// near is updated in place for the leaves with cell-particle sources
void far_final(const float4* pts, const uint32_t* perm, CellArrays cells, const int32_t* leaves,
               int32_t nleaves, uint8_t* m2pflag, const int32_t* m2p_off, const uint32_t* m2p_src, int64_t n_m2p,
               int family, int p, int KP, Tables t, const float* M, const float* L, double4* near, int out_dtype,
               void* phi, void* ex, void* ey, void* ez, hipStream_t s);
void p2p(const float4* pts, CellArrays cells, const int32_t* leaves, int32_t nleaves,
         const int32_t* p2p_off, const uint32_t* p2p_src, int guard_all, int tpl, double4* near,
         hipStream_t s);
// P2P size class of each leaf (0: <= 8, 1: <= 16, 2: <= 32, 3: more targets), val = the leaf's cell
void leaf_class_keys(CellArrays cells, const int32_t* leaves, int32_t nleaf, uint32_t* key, uint32_t* val,
                     hipStream_t s);
constexpr int kLeafClasses = 4;

// same-level M2L on MFMA: L[rowcell[r]] = sum_j T[offid[class][j]] * M[gather[r][j]]
struct GemmPlan {
    int32_t class_row0[9];   // rows of class c: [class_row0[c], class_row0[c+1])
    int32_t class_tile0[9];  // first tile of class c
    int32_t J;               // slots per class
    const int32_t* act;      // per tile: the slots some row uses ([tile][J], in slot order)
    const int32_t* nact;     // per tile: how many
    int32_t G;               // slot groups per tile (a multiple of 8: group g runs on XCD g mod 8)
    int32_t ntiles;          // tiles
    int32_t nrows;           // rows (targets) over all classes
    int32_t zcell;           // a cell index whose multipole row is all zero (absent sources read it)
    int32_t nt;              // targets per tile (gemm_tile_cols_kp, or another width gemm_tile_width_ok accepts)
};
// whether the GEMM kernels at storage width KP have a tiling of nt targets
// per tile (64 or 128 at width 128; the default width elsewhere)
bool gemm_tile_width_ok(int KP, int nt);
// slot groups for J slots per class, a multiple of 8 (group g runs on XCD
// g mod 8): fewer groups mean fewer partial rows to write and sum, smaller
// ones keep each group's operators near one XCD's L2; at most 79 slots a
// group (71 at theta = 0.4, G = 8)
int gemm_slot_groups(int J);
// a group holds at most J / G + 1 slots (80 with G = 8 ceil(J / 632)); the GEMM
// kernels stage a group's slots and operator ids in LDS arrays of this size
constexpr int kGemmMaxGroupSlots = 80;
// split-BF16 GEMM, by K step (16 multipole coefficients each): steps below
// kBf16FullSteps (k < 32, degrees 0-5) take all three BF16 products, steps
// below kBf16TwoSteps (k < 48) drop a_lo b_hi, and the rest (k >= 48,
// degrees 6 and up) keep a_hi b_hi alone
constexpr int kBf16FullSteps = 2;
constexpr int kBf16TwoSteps = 3;
// lo blocks (8 coefficients each) of a split multipole row that any product reads
constexpr int kBf16LoBlocks = 2 * kBf16TwoSteps;
// gather[tile][J][NT] from the filled gcol[tile][NT][Jp] (Jp: J rounded up
// to a multiple of 4, the padding -1), and act[tile * J + k], k < nact[tile]:
// the slots of tile `tile` that some row uses; NT (the tile width from
// gemm_tile_cols) is 64 or 128
void tile_transpose(const int32_t* gcol, GemmPlan plan, int NT, int Jp, int ntiles, int32_t* gather, int32_t* act,
                    int32_t* nact, hipStream_t s);
// part: G * nrows * KP floats of per-group partial locals, summed into L in group order
// e0, e1 (may be null): events recorded just before and after the GEMM kernel
// itself (without the group sum), for its own duration
void m2l_gemm(const float* T, const int32_t* offid, const int32_t* gather, const uint32_t* rowcell,
              GemmPlan plan, int K, int KP, const float* M, float* part, float* L, hipStream_t s,
              hipEvent_t e0 = nullptr, hipEvent_t e1 = nullptr);
bool m2l_gemm_supported(int p);
bool m2l_gemm_supported_kp(int KP);  // by storage width
// split-BF16 variant (Thi/Tlo: k-blocked BF16 halves of the operators)
// Ms: scratch of (ncell + 1) * split_row_blocks(KP) * 16 bytes (at most
// KP * 4 bytes a row) for the split multipoles
void m2l_gemm_bf16(const uint16_t* Thi, const uint16_t* Tlo, const int32_t* offid, const int32_t* gather,
                   const uint32_t* rowcell, GemmPlan plan, int K, int KP, const float* M, int64_t ncell, uint4* Ms,
                   float* part, float* L, hipStream_t s, hipEvent_t e0 = nullptr, hipEvent_t e1 = nullptr);
// L[rowcell[r]][k] = sum over g in order of part[g][r][k], k < K
void m2l_reduce_groups(const float* part, GemmPlan plan, const uint32_t* rowcell, int KP, int K, float* L,
                       hipStream_t s);
bool m2l_bf16_supported(int p);
bool m2l_bf16_supported_kp(int KP);
int split_row_blocks(int KP);  // 16-byte blocks per split multipole row (0: unsupported width)
int gemm_tile_cols(int p);  // targets per GEMM tile for order p
int gemm_tile_cols_kp(int KP);  // the same by storage width

// M2L of the same pairs as m2l_general, one pair at a time through a
// rotation to the offset's axis (k_m2l_rot.hip; spherical family)
void m2l_rotation(const int32_t* goff, const uint32_t* gsrc, CellArrays cells, int32_t ncell, int p, int KP,
                  const float* Wax, const float* M, float* L, const uint8_t* skip, hipStream_t s);

// Cartesian counterparts of cls_ops and m2l_general (k_cart.hip)
void cls_ops_cart(const uint64_t* key, const int32_t* start, int32_t ncls, int p, int KP, float* T, hipStream_t s);
void m2l_general_cart(const int32_t* goff, const uint32_t* gsrc, CellArrays cells, int32_t ncell, int p, int KP,
                      const float* M, float* L, const uint8_t* skip, hipStream_t s);

}  // namespace fmm
