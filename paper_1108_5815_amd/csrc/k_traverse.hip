// k_traverse.hip -- dual tree traversal as a level-synchronous frontier.
//
// Paper ("Dual tree traversal"): a stack holds (target, source) cell pairs;
// a popped pair has its larger cell split, each new pair is tested with the
// acceptance criterion ("Results": theta = (r_t + r_s)/R), accepted pairs
// interact, pairs of leaves that fail become particle-particle sums, and the
// rest are pushed again.  The children of a pair depend only on that pair,
// so the set of emitted interactions does not depend on the order in which
// pairs are processed.  Here every pair of the current frontier is expanded
// at once: one pass counts the new pairs of each kind, a scan places them,
// a second pass writes them; the order is deterministic (frontier order,
// then child order).  The counting pass records the kind of every child pair
// (2 bits each) so the writing pass does not classify again.
//
// Readings fixed here and in the oracle: r = half side of the cube, R between
// cube centres, accept iff (r_t + r_s)^2 <= theta^2 R^2 (integer half-grid
// geometry, one FP64 product), split the cell of lower level (both when
// levels are equal), only accepted pairs choose an interaction kind.
#include "fmm_internal.h"

#include <algorithm>

#pragma clang fp contract(off)

namespace fmm {
namespace {

enum { KIND_M2L = 0, KIND_M2P = 1, KIND_P2P = 2, KIND_SPLIT = 3 };

__device__ inline bool is_leaf(const CellArrays& c, int32_t i) { return c.nchild[i] == 0; }

__device__ inline int classify(const CellArrays& c, int32_t t, int32_t s, const TravParams& tp) {
    int4 gt = c.geo[t], gs = c.geo[s];
    int64_t dx = (int64_t)gt.x - gs.x, dy = (int64_t)gt.y - gs.y, dz = (int64_t)gt.z - gs.z;
    int64_t R2 = dx * dx + dy * dy + dz * dz;
    int64_t rr = (int64_t)gt.w + gs.w;
    if ((double)(rr * rr) <= __dmul_rn(tp.theta2, (double)R2)) {
        if (tp.policy == 0) return KIND_M2L;
        if (tp.policy == 1) return KIND_M2P;
        double nt = (double)(c.end[t] - c.begin[t]);
        double ns = (double)(c.end[s] - c.begin[s]);
        if (tp.policy == 3) {
            // learned choice, read from the network's evaluation over the
            // quantised features of the pair (count buckets precomputed per cell)
            int dl = c.level[s] - c.level[t];
            dl = dl < -kMlpDl ? -kMlpDl : (dl > kMlpDl ? kMlpDl : dl);
            const int bt = tp.nbucket[t], bs = tp.nbucket[s];
            double ratio = sqrt((double)(rr * rr) / (double)R2) / tp.theta;
            int bq = (int)(ratio * kMlpBq);
            bq = bq < 0 ? 0 : (bq >= kMlpBq ? kMlpBq - 1 : bq);
            return tp.mlp_table[(((dl + kMlpDl) * kMlpBn + bt) * kMlpBn + bs) * kMlpBq + bq];
        }
        double c0 = tp.c_m2l;
        double c1 = __dmul_rn(tp.c_m2p, nt);
        double c2 = __dmul_rn(__dmul_rn(tp.c_p2p, nt), ns);
        int k = KIND_M2L;
        double best = c0;
        if (c1 < best) { best = c1; k = KIND_M2P; }
        if (c2 < best) k = KIND_P2P;
        return k;
    }
    if (is_leaf(c, t) && is_leaf(c, s)) return KIND_P2P;
    return KIND_SPLIT;
}

__device__ inline void split_ranges(const CellArrays& c, int32_t T, int32_t S, int32_t& t0, int32_t& t1,
                                    int32_t& s0, int32_t& s1) {
    bool lt = is_leaf(c, T), ls = is_leaf(c, S);
    int vt = c.level[T], vs = c.level[S];
    bool splitT = !lt && (ls || vt <= vs);
    bool splitS = !ls && (lt || vs <= vt);
    t0 = splitT ? c.child[T] : T;
    t1 = splitT ? c.child[T] + c.nchild[T] : T + 1;
    s0 = splitS ? c.child[S] : S;
    s1 = splitS ? c.child[S] + c.nchild[S] : S + 1;
}

// quantised log2 of each cell's particle count: rint(kMlpNsub log2 n) clamped to the grid
__global__ void k_cell_buckets(CellArrays c, int32_t ncell, uint8_t* __restrict__ nb) {
    int32_t i = (int32_t)(blockIdx.x * blockDim.x + threadIdx.x);
    if (i >= ncell) return;
    int b = (int)rint(kMlpNsub * log2((double)(c.end[i] - c.begin[i])));
    nb[i] = (uint8_t)(b < 0 ? 0 : (b >= kMlpBn ? kMlpBn - 1 : b));
}

// Count and emit work on the child pairs of a wave's 16 frontier entries,
// flattened (entry by entry, child order) and taken 64 at a time, one child
// pair per lane: an entry has 64 children when both cells split and 8 or
// fewer when only one does, so one entry per lane left most of the child
// loop serial and its stores scattered.  Kinds are kept per entry as two
// 64-bit masks (bit q of `lo`/`hi` = low/high bit of child q's kind); a
// child's place in its kind's output is its entry's offset plus the number
// of earlier children of the same kind, so the emitted order is frontier
// order, then child order, as before.
constexpr int kEPW = 16;  // frontier entries per wave

struct EntryRanges {
    int32_t t0[kEPW], ns[kEPW], s0[kEPW], pre[kEPW + 1];
    uint32_t mns[kEPW];  // ceil(2^16 / ns): q / ns = (q * mns) >> 16 for q < 64, ns <= 8
};

// entry ranges of the wave's frontier entries f0 .. f0+kEPW-1 into LDS;
// returns the number of child pairs of the wave
__device__ inline int wave_entries(const int2* __restrict__ fr, int64_t nf, int64_t f0, const CellArrays& c,
                                   EntryRanges& er, int lane) {
    const int64_t f = f0 + lane;
    int nch = 0;
    if (lane < kEPW && f < nf) {
        const int2 pr = fr[f];
        int32_t t0, t1, s0, s1;
        split_ranges(c, pr.x, pr.y, t0, t1, s0, s1);
        er.t0[lane] = t0;
        er.s0[lane] = s0;
        er.ns[lane] = s1 - s0;
        er.mns[lane] = (65536u + (uint32_t)(s1 - s0) - 1u) / (uint32_t)(s1 - s0);
        nch = (t1 - t0) * (s1 - s0);
    }
    int incl = nch;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        const int u = __shfl_up(incl, d, 64);
        if (lane >= d) incl += u;
    }
    if (lane < kEPW) er.pre[lane + 1] = incl;
    if (lane == 0) er.pre[0] = 0;
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    return __shfl(incl, 63, 64);
}

// entry (0..kEPW-1) holding flattened child c of the wave (last e with pre[e] <= c)
__device__ inline int entry_of(const EntryRanges& er, int c) {
    int lo = 0, hi = kEPW;
#pragma unroll
    for (int it = 0; (1 << it) < kEPW; it++) {
        const int mid = (lo + hi) >> 1;
        if (er.pre[mid] <= c) lo = mid;
        else hi = mid;
    }
    return lo;
}

// The frontier holds *nfp entries (device memory); each wave takes kEPW of
// them at a time, striding over the grid.
__global__ __launch_bounds__(256) void k_trav_count(const int2* __restrict__ fr, const uint32_t* __restrict__ nfp,
                                                    CellArrays c, TravParams tp, uint4* __restrict__ cnt,
                                                    uint4* __restrict__ kinds) {
    __shared__ EntryRanges s_er[4];
    __shared__ uint32_t s_n[4][kEPW][4];
    __shared__ unsigned long long s_lo[4][kEPW], s_hi[4][kEPW];
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int64_t nf = *nfp;
    const int64_t step = (int64_t)gridDim.x * 4 * kEPW;
    // wave-uniform loop; no block barrier below
    for (int64_t f0 = ((int64_t)blockIdx.x * 4 + w) * kEPW; f0 < nf; f0 += step) {
        EntryRanges& er = s_er[w];
        if (lane < kEPW) {
#pragma unroll
            for (int k = 0; k < 4; k++) s_n[w][lane][k] = 0;
            s_lo[w][lane] = 0;
            s_hi[w][lane] = 0;
        }
        const int total = wave_entries(fr, nf, f0, c, er, lane);
        for (int r0 = 0; r0 < total; r0 += 64) {
            const int ch = r0 + lane;
            const bool valid = ch < total;
            int e = 0, q = 0, k = 0;
            if (valid) {
                e = entry_of(er, ch);
                q = ch - er.pre[e];
                const int qt = (int)(((uint32_t)q * er.mns[e]) >> 16);
                k = classify(c, er.t0[e] + qt, er.s0[e] + (q - qt * er.ns[e]), tp);
            }
            // kinds of the round by ballot; the first lane of each entry in the
            // round folds its entry's lanes into the entry's counts and masks
            const uint64_t mv = __ballot(valid), m1 = __ballot(valid && (k & 1)), m2 = __ballot(valid && (k & 2));
            if (valid && (q == 0 || lane == 0)) {
                const int last = min(63, er.pre[e + 1] - r0 - 1);
                const uint64_t upto = last == 63 ? ~0ull : ((1ull << (last + 1)) - 1ull);
                const uint64_t rng = upto & ~((1ull << lane) - 1ull);
                const uint64_t lo = m1 & rng, hi = m2 & rng, all = mv & rng;
                s_n[w][e][KIND_M2L] += (uint32_t)__popcll(all & ~lo & ~hi);
                s_n[w][e][KIND_M2P] += (uint32_t)__popcll(lo & ~hi);
                s_n[w][e][KIND_P2P] += (uint32_t)__popcll(~lo & hi);
                s_n[w][e][KIND_SPLIT] += (uint32_t)__popcll(lo & hi);
                s_lo[w][e] |= (lo >> lane) << q;
                s_hi[w][e] |= (hi >> lane) << q;
            }
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        const int64_t f = f0 + lane;
        if (lane < kEPW && f < nf) {
            cnt[f] = make_uint4(s_n[w][lane][0], s_n[w][lane][1], s_n[w][lane][2], s_n[w][lane][3]);
            const unsigned long long lo = s_lo[w][lane], hi = s_hi[w][lane];
            kinds[f] = make_uint4((uint32_t)lo, (uint32_t)(lo >> 32), (uint32_t)hi, (uint32_t)(hi >> 32));
        }
        // the wave's LDS is reset and refilled by its next group of entries
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    }
}

// Children of the frontier's *nfp entries to the three lists (at their
// running totals tot[0..2]) and the next frontier, at the offsets of the
// scan whose total is *add.  If a list or the next frontier would pass its
// capacity, nothing is written and the overflow bits are set (1, 2, 4: the
// lists; 8: the frontier).
__global__ __launch_bounds__(256) void k_trav_emit(const int2* __restrict__ fr, const uint32_t* __restrict__ nfp,
                                                   CellArrays c, const uint4* __restrict__ kinds,
                                                   const uint4* __restrict__ off, const uint32_t* __restrict__ tot,
                                                   const uint4* __restrict__ add, TravCaps caps,
                                                   int2* __restrict__ m2l, int2* __restrict__ m2p,
                                                   int2* __restrict__ p2p, int2* __restrict__ next,
                                                   uint32_t* __restrict__ ovf) {
    __shared__ EntryRanges s_er[4];
    __shared__ unsigned long long s_lo[4][kEPW], s_hi[4][kEPW];
    __shared__ uint4 s_off[4][kEPW];
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int64_t nf = *nfp;
    const uint4 a = *add;
    const int64_t b0 = tot[0], b1 = tot[1], b2 = tot[2];
    const uint32_t bits = (b0 + a.x > caps.m2l ? 1u : 0u) | (b1 + a.y > caps.m2p ? 2u : 0u) |
                          (b2 + a.z > caps.p2p ? 4u : 0u) | ((int64_t)a.w > caps.next ? 8u : 0u);
    if (bits) {
        if (blockIdx.x == 0 && threadIdx.x == 0) *ovf |= bits;
        return;
    }
    const int64_t step = (int64_t)gridDim.x * 4 * kEPW;
    // wave-uniform loop; no block barrier below
    for (int64_t f0 = ((int64_t)blockIdx.x * 4 + w) * kEPW; f0 < nf; f0 += step) {
        EntryRanges& er = s_er[w];
        {
            const int64_t f = f0 + lane;
            if (lane < kEPW && f < nf) {
                const uint4 kw = kinds[f];
                s_lo[w][lane] = (unsigned long long)kw.x | ((unsigned long long)kw.y << 32);
                s_hi[w][lane] = (unsigned long long)kw.z | ((unsigned long long)kw.w << 32);
                s_off[w][lane] = off[f];
            }
        }
        const int total = wave_entries(fr, nf, f0, c, er, lane);
        for (int r0 = 0; r0 < total; r0 += 64) {
            const int ch = r0 + lane;
            if (ch < total) {
                const int e = entry_of(er, ch);
                const int q = ch - er.pre[e];
                const int ns = er.ns[e];
                const int qt = q / ns;
                const int2 v = make_int2(er.t0[e] + qt, er.s0[e] + (q - qt * ns));
                const unsigned long long lo = s_lo[w][e], hi = s_hi[w][e];
                const int k = (int)((lo >> q) & 1ull) | ((int)((hi >> q) & 1ull) << 1);
                const unsigned long long same = ((k & 1) ? lo : ~lo) & ((k & 2) ? hi : ~hi);
                const uint32_t rank = (uint32_t)__popcll(same & ((1ull << q) - 1ull));
                const uint4 o = s_off[w][e];
                if (k == KIND_M2L) m2l[b0 + o.x + rank] = v;
                else if (k == KIND_M2P) m2p[b1 + o.y + rank] = v;
                else if (k == KIND_P2P) p2p[b2 + o.z + rank] = v;
                else next[(int64_t)o.w + rank] = v;
            }
        }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    }
}

// after an emit: running totals += the level's counts, frontier size = its
// split pairs (0 after an overflow, which ends the traversal)
__global__ void k_trav_advance(uint32_t* __restrict__ tot, const uint4* __restrict__ add, uint32_t* __restrict__ nf,
                               const uint32_t* __restrict__ ovf, uint32_t* __restrict__ levels) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    const uint4 a = *add;
    if (*ovf) {
        *nf = 0;
        return;
    }
    if (*nf > 0) *levels += 1u;
    tot[0] += a.x;
    tot[1] += a.y;
    tot[2] += a.z;
    *nf = a.w;
}

__global__ void k_split_pairs(const int2* __restrict__ pairs, int64_t n, uint32_t* __restrict__ tgt,
                              uint32_t* __restrict__ src) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    int2 v = pairs[i];
    tgt[i] = (uint32_t)v.x;
    src[i] = (uint32_t)v.y;
}

__global__ void k_csr(const uint32_t* __restrict__ tgt, int64_t n, int32_t ncell, int32_t* __restrict__ off) {
    int32_t c = (int32_t)(blockIdx.x * blockDim.x + threadIdx.x);
    if (c > ncell) return;
    int64_t lo = 0, hi = n;
    while (lo < hi) {
        int64_t mid = (lo + hi) >> 1;
        if ((int32_t)tgt[mid] < c) lo = mid + 1;
        else hi = mid;
    }
    off[c] = (int32_t)lo;
}

// slot of a same-level pair in its target's offset class, or -1.  Everything
// comes from the two cells' half-grid geometry (centre and half side
// r = 2^(21 - level)): equal levels are equal r, the root is r = 2^21, and
// the target's octant within its parent is bit 1 of its centre / r per axis
// (centre / r = 2 a + 1 for cell index a), so a pair reads two 16-byte cell
// records and the table, each without waiting for another.
__device__ inline int32_t fast_slot(const CellArrays& c, int32_t t, int32_t s, const int32_t* slot_of, int R) {
    const int4 gt = c.geo[t], gs = c.geo[s];
    const int32_t side = max(2 * gt.w, 1);
    const int32_t ox = (gs.x - gt.x) / side, oy = (gs.y - gt.y) / side, oz = (gs.z - gt.z) / side;
    const bool ok = gt.w < (1 << kMaxLevel) && gs.w == gt.w && ox >= -R && ox <= R && oy >= -R && oy <= R &&
                    oz >= -R && oz <= R;
    const int W = 2 * R + 1;
    const int sh = __builtin_ctz((unsigned)max(gt.w, 1)) + 1;
    const int cls = ((gt.x >> sh) & 1) | (((gt.y >> sh) & 1) << 1) | (((gt.z >> sh) & 1) << 2);
    const size_t at = ok ? (size_t)cls * W * W * W + ((size_t)(ox + R) * W + (oy + R)) * W + (oz + R) : 0;
    const int32_t sl = slot_of[at];
    return ok ? sl : -1;
}

// Same-level pairs per target, and the slot of every pair (-1 outside the
// tables) for the gather fill.  Pairs come in emission order, where the
// children of one frontier pair sit side by side, so a wave first sums its
// runs of equal targets (segmented scan over the lanes) and adds each run
// with one atomic (integer: the counts do not depend on timing).
__global__ __launch_bounds__(256) void k_mark_targets(const int2* __restrict__ pairs, int64_t n, CellArrays c,
                                                      const int32_t* __restrict__ slot_of, int R,
                                                      uint32_t* __restrict__ nfast, int16_t* __restrict__ slot) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int lane = threadIdx.x & 63;
    int32_t t = -1;
    int v = 0;
    if (i < n) {
        const int2 pr = pairs[i];
        t = pr.x;
        const int32_t sl = fast_slot(c, t, pr.y, slot_of, R);
        slot[i] = (int16_t)sl;
        v = sl >= 0 ? 1 : 0;
    }
    const int32_t tp = __shfl_up(t, 1, 64);
    int flag = (lane == 0 || tp != t) ? 1 : 0;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        const int v2 = __shfl_up(v, d, 64), f2 = __shfl_up(flag, d, 64);
        if (lane >= d) {
            if (!flag) v += v2;
            flag |= f2;
        }
    }
    const int32_t tn = __shfl_down(t, 1, 64);
    const bool tail = lane == 63 || tn != t;
    if (tail && t >= 0 && v > 0) atomicAdd(&nfast[t], (uint32_t)v);
}

// gcol[(tile * NT + column) * rowlen + slot] = source of each same-level pair
__global__ void k_fill_gather(const int2* __restrict__ pairs, const int16_t* __restrict__ slot, int64_t n,
                              const int32_t* __restrict__ rowof, int32_t rowlen, int32_t* __restrict__ gcol) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int32_t sl = slot[i];
    const int2 pr = pairs[i];  // read with the slot: almost every pair is in the tables
    if (sl >= 0) {
        const int32_t pr_row = rowof[pr.x];  // tile * NT + column
        gcol[(int64_t)pr_row * rowlen + sl] = pr.y;
    }
}

// Rows of the M2L GEMM: cells with same-level pairs, keyed by octant class and,
// within a class, by density in buckets of 32 missing slots (densest first);
// the sort is stable, so a bucket keeps cell order (level by level, key
// order), where neighbouring rows miss similar slots: full rows share tiles,
// sparse rows do not spread zero columns over dense tiles, and a tile's
// active slots stay few (4% fewer than sorting by the exact count).
__global__ void k_row_class_keys(const uint32_t* __restrict__ nfast, CellArrays c, int32_t ncell, int32_t J,
                                 uint32_t* __restrict__ key, uint32_t* __restrict__ val) {
    int32_t i = (int32_t)(blockIdx.x * blockDim.x + threadIdx.x);
    if (i >= ncell) return;
    const uint32_t n = nfast[i];
    const uint32_t miss = n >= (uint32_t)J ? 0u : (uint32_t)J - n;
    key[i] = n ? ((uint32_t)(c.prefix[i] & 7u) << kRowMissBits) | ((miss < kRowMissMax ? miss : kRowMissMax) >> 5)
               : (8u << kRowMissBits);
    val[i] = (uint32_t)i;
}

// rowof[cell of row r] = tile * NT + column of row r in its tile (tiles hold
// NT consecutive rows of one class; the last tile of a class may be short)
__global__ void k_rows_inverse(const uint32_t* __restrict__ rowcell, int64_t nrows, GemmPlan plan, int NT,
                               int32_t* __restrict__ rowof) {
    int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= nrows) return;
    int cls = 0;
    while (cls < 7 && r >= plan.class_row0[cls + 1]) cls++;
    const int32_t local = (int32_t)r - plan.class_row0[cls];
    const int32_t tile = plan.class_tile0[cls] + local / NT;
    rowof[rowcell[r]] = tile * NT + local % NT;
}

// Gather table of each GEMM tile (NT consecutive rows of one octant class)
// from column order ([NT][Jp], as the fill writes it, Jp = J rounded up to a
// multiple of 4: the pairs one split parent pair emits for one target are
// neighbouring slots of its column) to slot order ([J][NT], as the GEMM
// reads it: a slot's NT sources in one read), through LDS in chunks of 64
// slots, both sides in 16-byte accesses; and the tile's active slots (at
// least one column holds a source), in slot order.  The GEMM runs over these
// only; a slot no row uses would add a zero block.
__global__ __launch_bounds__(256) void k_tile_transpose(const int32_t* __restrict__ gcol, GemmPlan plan, int NT,
                                                        int Jp, int32_t* __restrict__ gather,
                                                        int32_t* __restrict__ act, int32_t* __restrict__ nact) {
    __shared__ int32_t blk[128][65];  // [column][slot of the chunk], padded against bank conflicts
    __shared__ uint8_t used[64];
    const int tile = blockIdx.x;
    const int J = plan.J;
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const uint64_t below = lane == 0 ? 0ull : (~0ull >> (64 - lane));
    const int32_t* src = gcol + (size_t)tile * NT * Jp;
    int32_t* dst = gather + (size_t)tile * J * NT;
    const int NT4 = NT >> 2;
    int base = 0;  // meaningful in wave 0, which compacts
    for (int j0 = 0; j0 < J; j0 += 64) {
        const int nj = min(64, J - j0);
        // read: 16 quads of slots per column (a quad past Jp reads as absent)
        for (int e = threadIdx.x; e < NT * 16; e += 256) {
            const int c = e >> 4, q4 = (e & 15) << 2;
            int4 v = make_int4(-1, -1, -1, -1);
            if (j0 + q4 < Jp) v = *reinterpret_cast<const int4*>(src + (size_t)c * Jp + j0 + q4);
            blk[c][q4] = v.x;
            blk[c][q4 + 1] = v.y;
            blk[c][q4 + 2] = v.z;
            blk[c][q4 + 3] = v.w;
        }
        __syncthreads();
        // write: per slot of the chunk, NT / 4 quads of columns
        for (int e = threadIdx.x; e < nj * NT4; e += 256) {
            const int jj = e / NT4, c4 = (e - jj * NT4) << 2;
            *reinterpret_cast<int4*>(dst + (size_t)(j0 + jj) * NT + c4) =
                make_int4(blk[c4][jj], blk[c4 + 1][jj], blk[c4 + 2][jj], blk[c4 + 3][jj]);
        }
        for (int jj = w; jj < 64; jj += 4) {
            bool a = false;
            for (int c = lane; c < NT; c += 64) a = a || blk[c][jj] >= 0;
            const uint64_t m = __ballot(a);
            if (lane == 0) used[jj] = (jj < nj && m != 0ull) ? 1 : 0;
        }
        __syncthreads();
        if (w == 0) {
            const bool a = used[lane] != 0;
            const uint64_t m = __ballot(a);
            if (a) act[(size_t)tile * J + base + __popcll(m & below)] = j0 + lane;
            base += __popcll(m);
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) nact[tile] = base;
}

inline unsigned grid(int64_t n, int b = 256) { return (unsigned)((n + b - 1) / b); }

}  // namespace

void cell_buckets(CellArrays cells, int32_t ncell, uint8_t* nbucket, hipStream_t s) {
    if (ncell <= 0) return;
    k_cell_buckets<<<grid(ncell), 256, 0, s>>>(cells, ncell, nbucket);
}

// fixed grids sized for the frontier's capacity
static unsigned trav_blocks(int64_t cap_frontier) {
    return (unsigned)std::max<int64_t>(1, std::min<int64_t>((cap_frontier + 4 * kEPW - 1) / (4 * kEPW), 4096));
}

void trav_count(const int2* frontier, const uint32_t* nf, int64_t cap_frontier, CellArrays cells, TravParams tp,
                uint4* cnt, uint4* kinds, hipStream_t s) {
    k_trav_count<<<trav_blocks(cap_frontier), 256, 0, s>>>(frontier, nf, cells, tp, cnt, kinds);
}

void trav_emit(const int2* frontier, uint32_t* nf, int64_t cap_frontier, CellArrays cells, const uint4* kinds,
               const uint4* off, uint32_t* tot, const uint4* add, TravCaps caps, int2* m2l, int2* m2p, int2* p2p,
               int2* next, uint32_t* ovf, uint32_t* levels, hipStream_t s) {
    k_trav_emit<<<trav_blocks(cap_frontier), 256, 0, s>>>(frontier, nf, cells, kinds, off, tot, add, caps, m2l, m2p,
                                                          p2p, next, ovf);
    k_trav_advance<<<1, 64, 0, s>>>(tot, add, nf, ovf, levels);
}

void split_pairs(const int2* pairs, int64_t n, uint32_t* tgt, uint32_t* src, hipStream_t s) {
    if (n <= 0) return;
    k_split_pairs<<<grid(n), 256, 0, s>>>(pairs, n, tgt, src);
}

void csr_offsets(const uint32_t* tgt_sorted, int64_t n, int32_t ncell, int32_t* offsets, hipStream_t s) {
    k_csr<<<grid((int64_t)ncell + 1), 256, 0, s>>>(tgt_sorted, n, ncell, offsets);
}

void m2l_mark_targets(const int2* pairs, int64_t n, CellArrays cells, const int32_t* slot_of, int R,
                      uint32_t* has_fast, int16_t* slot, hipStream_t s) {
    if (n <= 0) return;
    k_mark_targets<<<grid(n), 256, 0, s>>>(pairs, n, cells, slot_of, R, has_fast, slot);
}

void tile_transpose(const int32_t* gcol, GemmPlan plan, int NT, int Jp, int ntiles, int32_t* gather, int32_t* act,
                    int32_t* nact, hipStream_t s) {
    if (ntiles <= 0) return;
    k_tile_transpose<<<ntiles, 256, 0, s>>>(gcol, plan, NT, Jp, gather, act, nact);
}

void m2l_fill_gather(const int2* pairs, const int16_t* slot, int64_t n, const int32_t* rowof, int32_t rowlen,
                     int32_t* gcol, hipStream_t s) {
    if (n <= 0) return;
    k_fill_gather<<<grid(n), 256, 0, s>>>(pairs, slot, n, rowof, rowlen, gcol);
}

void row_class_keys(const uint32_t* nfast, CellArrays cells, int32_t ncell, int32_t J, uint32_t* key, uint32_t* val,
                    hipStream_t s) {
    if (ncell <= 0) return;
    k_row_class_keys<<<grid(ncell), 256, 0, s>>>(nfast, cells, ncell, J, key, val);
}

void rows_inverse(const uint32_t* rowcell, int64_t nrows, GemmPlan plan, int NT, int32_t* rowof, hipStream_t s) {
    if (nrows <= 0) return;
    k_rows_inverse<<<grid(nrows), 256, 0, s>>>(rowcell, nrows, plan, NT, rowof);
}

}  // namespace fmm

namespace fmm {
namespace {

__global__ void k_class_bounds(const uint32_t* __restrict__ key, int64_t n, int shift, int32_t* __restrict__ out9) {
    int c = threadIdx.x;
    if (c > 8) return;
    int64_t lo = 0, hi = n;
    while (lo < hi) {
        int64_t mid = (lo + hi) >> 1;
        if ((key[mid] >> shift) < (uint32_t)c) lo = mid + 1;
        else hi = mid;
    }
    out9[c] = (int32_t)lo;
}

__global__ void k_leaf_flags(CellArrays c, int32_t ncell, uint32_t* __restrict__ flag) {
    int32_t i = (int32_t)(blockIdx.x * blockDim.x + threadIdx.x);
    if (i < ncell) flag[i] = c.nchild[i] == 0 ? 1u : 0u;
}

__global__ void k_leaf_write(CellArrays c, int32_t ncell, const uint32_t* __restrict__ pos,
                             int32_t* __restrict__ leaves, int32_t* __restrict__ inner) {
    int32_t i = (int32_t)(blockIdx.x * blockDim.x + threadIdx.x);
    if (i >= ncell) return;
    if (c.nchild[i] == 0) leaves[pos[i]] = i;
    else inner[i - (int32_t)pos[i]] = i;
}

// leaves holding target particles (sorted positions below nt)
__global__ void k_target_leaf_flags(CellArrays c, const int32_t* __restrict__ leaves, int32_t nleaf, int32_t nt,
                                    uint32_t* __restrict__ flag) {
    int32_t i = (int32_t)(blockIdx.x * blockDim.x + threadIdx.x);
    if (i < nleaf) flag[i] = c.begin[leaves[i]] < nt ? 1u : 0u;
}

__global__ void k_target_leaf_write(const int32_t* __restrict__ leaves, const uint32_t* __restrict__ flag,
                                    const uint32_t* __restrict__ pos, int32_t nleaf, int32_t* __restrict__ out) {
    int32_t i = (int32_t)(blockIdx.x * blockDim.x + threadIdx.x);
    if (i < nleaf && flag[i]) out[pos[i]] = leaves[i];
}

}  // namespace

void target_leaf_flags(CellArrays cells, const int32_t* leaves, int32_t nleaf, int32_t nt, uint32_t* flag,
                       hipStream_t s) {
    if (nleaf <= 0) return;
    k_target_leaf_flags<<<(nleaf + 255) / 256, 256, 0, s>>>(cells, leaves, nleaf, nt, flag);
}

void target_leaf_write(const int32_t* leaves, const uint32_t* flag, const uint32_t* pos, int32_t nleaf, int32_t* out,
                       hipStream_t s) {
    if (nleaf <= 0) return;
    k_target_leaf_write<<<(nleaf + 255) / 256, 256, 0, s>>>(leaves, flag, pos, nleaf, out);
}

void class_bounds(const uint32_t* key_sorted, int64_t n, int shift, int32_t* out9, hipStream_t s) {
    k_class_bounds<<<1, 64, 0, s>>>(key_sorted, n, shift, out9);
}

void leaf_flags(CellArrays cells, int32_t ncell, uint32_t* flag, hipStream_t s) {
    if (ncell <= 0) return;
    k_leaf_flags<<<(ncell + 255) / 256, 256, 0, s>>>(cells, ncell, flag);
}

void leaf_write(CellArrays cells, int32_t ncell, const uint32_t* pos, int32_t* leaves, int32_t* inner,
                hipStream_t s) {
    if (ncell <= 0) return;
    k_leaf_write<<<(ncell + 255) / 256, 256, 0, s>>>(cells, ncell, pos, leaves, inner);
}

}  // namespace fmm

namespace fmm {
namespace {

// flags in tiles of kCompactTile = 4 waves x 16 rounds x 64 lanes, in order
constexpr int kCompactTile = 4096;

// a pair is kept when its slot is -1 (outside the tables)
__device__ inline uint32_t wave_flag_count(const int16_t* __restrict__ flag, int64_t n, int64_t base, int lane) {
    uint32_t c = 0;
    for (int r = 0; r < 16; r++) {
        const int64_t g = base + r * 64 + lane;
        c += (uint32_t)__popcll(__ballot(g < n && flag[g] < 0));
    }
    return c;
}

__global__ __launch_bounds__(256) void k_flag_counts(const int16_t* __restrict__ flag, int64_t n,
                                                     uint32_t* __restrict__ cnt) {
    __shared__ uint32_t wsum[4];
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const uint32_t c = wave_flag_count(flag, n, (int64_t)blockIdx.x * kCompactTile + w * 1024, lane);
    if (lane == 0) wsum[w] = c;
    __syncthreads();
    if (threadIdx.x == 0) cnt[blockIdx.x] = wsum[0] + wsum[1] + wsum[2] + wsum[3];
}

// flagged pairs of each tile written from the tile's base, in index order
__global__ __launch_bounds__(256) void k_compact_pairs(const int2* __restrict__ pairs,
                                                       const int16_t* __restrict__ flag, const uint32_t* __restrict__ tbase,
                                                       int64_t n, uint32_t* __restrict__ otgt,
                                                       uint32_t* __restrict__ osrc) {
    __shared__ uint32_t wsum[4];
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int64_t base = (int64_t)blockIdx.x * kCompactTile + w * 1024;
    const uint32_t c = wave_flag_count(flag, n, base, lane);
    if (lane == 0) wsum[w] = c;
    __syncthreads();
    uint32_t off = tbase[blockIdx.x];
    for (int q = 0; q < w; q++) off += wsum[q];
    const uint64_t lt = lane == 0 ? 0ull : (~0ull >> (64 - lane));
    for (int r = 0; r < 16; r++) {
        const int64_t g = base + r * 64 + lane;
        const bool f = g < n && flag[g] < 0;
        const uint64_t m = __ballot(f);
        if (f) {
            const uint32_t pos = off + (uint32_t)__popcll(m & lt);
            const int2 pr = pairs[g];
            otgt[pos] = (uint32_t)pr.x;
            osrc[pos] = (uint32_t)pr.y;
        }
        off += (uint32_t)__popcll(m);
    }
}

}  // namespace

int64_t compact_tiles(int64_t n) { return (n + kCompactTile - 1) / kCompactTile; }

void flag_counts(const int16_t* flag, int64_t n, uint32_t* cnt, hipStream_t s) {
    if (n <= 0) return;
    k_flag_counts<<<(unsigned)compact_tiles(n), 256, 0, s>>>(flag, n, cnt);
}

void compact_pairs(const int2* pairs, const int16_t* flag, const uint32_t* tbase, int64_t n, uint32_t* otgt,
                   uint32_t* osrc, hipStream_t s) {
    if (n <= 0) return;
    k_compact_pairs<<<(unsigned)compact_tiles(n), 256, 0, s>>>(pairs, flag, tbase, n, otgt, osrc);
}

}  // namespace fmm
