// k_util.hip -- device-wide exclusive scans and a stable LSD radix sort.
//
// Scan: reduce tiles -> scan tile sums in one workgroup -> scan within tiles.
// Radix sort: digits of at most 11 bits, the key bits spread evenly over the
// passes (18-bit cell keys: 2 passes of 9); per tile a digit histogram, a
// scan of the digit-major histogram table, then a stable scatter in which
// each wave ranks its 64 keys per round with one ballot per digit bit (lanes
// holding the same digit form a mask; rank = popcount of the lower lanes of
// that mask).  Tiles are 4096
// keys: 4 waves x 16 rounds x 64 lanes, processed in index order, so equal
// digits keep their input order.
#include "fmm_internal.h"

namespace fmm {
namespace {

constexpr int SB = 256;          // scan threads per block
constexpr int SI = 8;            // items per thread
constexpr int ST = SB * SI;      // items per tile

__device__ inline uint32_t wave_incl_u32(uint32_t v, int lane) {
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        uint32_t t = __shfl_up(v, d, 64);
        if (lane >= d) v += t;
    }
    return v;
}

struct U1 {
    uint32_t a;
};

template <class T>
struct Ops;

template <>
struct Ops<uint32_t> {
    static constexpr int C = 1;
    __device__ static uint32_t get(const uint32_t& v, int) { return v; }
    __device__ static void set(uint32_t& v, int, uint32_t x) { v = x; }
};

template <>
struct Ops<uint4> {
    static constexpr int C = 4;
    __device__ static uint32_t get(const uint4& v, int c) {
        return c == 0 ? v.x : c == 1 ? v.y : c == 2 ? v.z : v.w;
    }
    __device__ static void set(uint4& v, int c, uint32_t x) {
        if (c == 0) v.x = x;
        else if (c == 1) v.y = x;
        else if (c == 2) v.z = x;
        else v.w = x;
    }
};

// block-wide exclusive scan of one u32 per thread (SB threads); returns the
// exclusive prefix and writes the block total into *tot (all threads).
__device__ inline uint32_t block_excl_u32(uint32_t v, uint32_t* lds, uint32_t* tot) {
    int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    uint32_t inc = wave_incl_u32(v, lane);
    if (lane == 63) lds[w] = inc;
    __syncthreads();
    uint32_t pre = 0, all = 0;
#pragma unroll
    for (int i = 0; i < SB / 64; i++) {
        uint32_t t = lds[i];
        if (i < w) pre += t;
        all += t;
    }
    __syncthreads();
    *tot = all;
    return pre + inc - v;
}

template <class T>
__global__ void k_scan_reduce(const T* __restrict__ in, int64_t n, T* __restrict__ part) {
    __shared__ uint32_t lds[SB / 64];
    int64_t base = (int64_t)blockIdx.x * ST;
    T out;
    for (int c = 0; c < Ops<T>::C; c++) {
        uint32_t acc = 0;
        for (int i = threadIdx.x; i < ST; i += SB) {
            int64_t g = base + i;
            if (g < n) acc += Ops<T>::get(in[g], c);
        }
        uint32_t tot;
        block_excl_u32(acc, lds, &tot);
        Ops<T>::set(out, c, tot);
    }
    if (threadIdx.x == 0) part[blockIdx.x] = out;
}

// one workgroup of SB threads scans the nb tile sums in place (exclusive)
template <class T>
__global__ void k_scan_partials(T* part, int64_t nb, T* total) {
    __shared__ uint32_t lds[SB / 64];
    uint32_t carries[Ops<T>::C];
    for (int c = 0; c < Ops<T>::C; c++) {
        uint32_t carry = 0;
        for (int64_t b0 = 0; b0 < nb; b0 += SB) {
            int64_t g = b0 + threadIdx.x;
            uint32_t v = g < nb ? Ops<T>::get(part[g], c) : 0u;
            uint32_t tot;
            uint32_t ex = block_excl_u32(v, lds, &tot);
            if (g < nb) {
                T t = part[g];
                Ops<T>::set(t, c, ex + carry);
                part[g] = t;
            }
            carry += tot;
        }
        carries[c] = carry;
        __syncthreads();
    }
    // one store of the totals (total may be mapped host memory)
    if (threadIdx.x == 0 && total) {
        T t;
        for (int c = 0; c < Ops<T>::C; c++) Ops<T>::set(t, c, carries[c]);
        *total = t;
    }
}

template <class T>
__global__ void k_scan_down(const T* __restrict__ in, T* __restrict__ out, int64_t n,
                            const T* __restrict__ part) {
    __shared__ uint32_t lds[SB / 64];
    int64_t base = (int64_t)blockIdx.x * ST + (int64_t)threadIdx.x * SI;
    T v[SI];
#pragma unroll
    for (int j = 0; j < SI; j++) {
        int64_t g = base + j;
        if (g < n) v[j] = in[g];
        else
            for (int c = 0; c < Ops<T>::C; c++) Ops<T>::set(v[j], c, 0u);
    }
    T pb = part[blockIdx.x];
    T res[SI];
    for (int c = 0; c < Ops<T>::C; c++) {
        uint32_t s = 0;
#pragma unroll
        for (int j = 0; j < SI; j++) s += Ops<T>::get(v[j], c);
        uint32_t tot;
        uint32_t run = block_excl_u32(s, lds, &tot) + Ops<T>::get(pb, c);
#pragma unroll
        for (int j = 0; j < SI; j++) {
            Ops<T>::set(res[j], c, run);
            run += Ops<T>::get(v[j], c);
        }
    }
#pragma unroll
    for (int j = 0; j < SI; j++) {
        int64_t g = base + j;
        if (g < n) out[g] = res[j];
    }
}

template <class T>
void scan_impl(const T* in, T* out, T* total, int64_t n, void* ws, hipStream_t s) {
    if (n <= 0) {
        if (total) hipMemsetAsync(total, 0, sizeof(T), s);
        return;
    }
    int64_t nb = (n + ST - 1) / ST;
    T* part = (T*)ws;
    k_scan_reduce<T><<<(unsigned)nb, SB, 0, s>>>(in, n, part);
    k_scan_partials<T><<<1, SB, 0, s>>>(part, nb, total);
    k_scan_down<T><<<(unsigned)nb, SB, 0, s>>>(in, out, n, part);
}

// ------------------------------------------------------------------ radix sort
constexpr int RB = 256;
constexpr int RW = RB / 64;
constexpr int RR = 16;       // rounds of 64 keys per wave for small and medium sorts
constexpr int RRmax = 64;    // for large sorts
constexpr int RT = RB * RR;  // smallest tile (sizes the workspace)
constexpr int kMaxDigitBits = 11;
constexpr int kRsBatch = 8;  // rounds whose keys are loaded together (divides RR)

// Rounds per wave: each block writes (hist) and reads (scatter) one count per
// digit, strided by the number of blocks, so large sorts take longer tiles to
// keep those scattered accesses few, while keeping >= 2048 blocks.
int rs_rounds(int64_t n) {
    int rr = RR;
    while (rr < RRmax && n >= (int64_t)RB * rr * 2 * 2048) rr *= 2;
    return rr;
}

// digit of `w` bits at `shift`, counted in 2^DB buckets (w <= DB)
template <class K>
__device__ inline uint32_t digit_of(K k, int shift, uint32_t mask) {
    return (uint32_t)(k >> shift) & mask;
}

// Adds a wave's digits to the counts h[]: the lanes hold consecutive keys
// (valid lanes first), and keys often repeat in runs (pairs of one target
// sit side by side), so each run of equal digits adds its length with one
// atomic from its first lane instead of one conflicting atomic per lane.
__device__ inline void add_digit_runs(uint32_t* h, uint32_t d, bool valid, int lane) {
    const uint32_t prev = __shfl_up(d, 1, 64);
    const bool head = valid && (lane == 0 || prev != d);
    const uint64_t heads = __ballot(head);
    const uint64_t vmask = __ballot(valid);
    if (head) {
        const uint64_t above = heads & ~((2ull << lane) - 1ull);
        const int end = above ? __builtin_ctzll(above) : __popcll(vmask);
        atomicAdd(&h[d], (uint32_t)(end - lane));
    }
}

template <class K, int DB>
__global__ void k_rs_hist(const K* __restrict__ keys, int64_t n, int shift, uint32_t mask,
                          uint32_t* __restrict__ ghist, int64_t nb, int rr) {
    constexpr int ND = 1 << DB;
    __shared__ uint32_t h[ND];
    for (int d = threadIdx.x; d < ND; d += RB) h[d] = 0;
    __syncthreads();
    const int tile = RB * rr;
    int64_t base = (int64_t)blockIdx.x * tile;
    const int lane = threadIdx.x & 63;
    for (int i0 = threadIdx.x; i0 < tile; i0 += RB * kRsBatch) {
        K kb[kRsBatch];
#pragma unroll
        for (int j = 0; j < kRsBatch; j++) {
            const int64_t g = base + i0 + j * RB;
            kb[j] = g < n ? keys[g] : K(0);
        }
#pragma unroll
        for (int j = 0; j < kRsBatch; j++) {
            const bool valid = base + i0 + j * RB < n;
            add_digit_runs(h, valid ? digit_of(kb[j], shift, mask) : 0u, valid, lane);
        }
    }
    __syncthreads();
    for (int d = threadIdx.x; d < ND; d += RB) ghist[(int64_t)d * nb + blockIdx.x] = h[d];
}

template <class K, int DB>
__global__ void k_rs_scatter(const K* __restrict__ kin, const uint32_t* __restrict__ vin,
                             K* __restrict__ kout, uint32_t* __restrict__ vout, int64_t n,
                             int shift, uint32_t mask, const uint32_t* __restrict__ goff, int64_t nb, int rr) {
    constexpr int ND = 1 << DB;
    __shared__ uint32_t wc[RW][ND];
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
    for (int i = threadIdx.x; i < RW * ND; i += RB) (&wc[0][0])[i] = 0;
    __syncthreads();
    const int64_t wbase = (int64_t)blockIdx.x * (RB * rr) + (int64_t)w * (rr * 64);
    for (int r0 = 0; r0 < rr; r0 += kRsBatch) {
        K kb[kRsBatch];
#pragma unroll
        for (int j = 0; j < kRsBatch; j++) {
            const int64_t g = wbase + (r0 + j) * 64 + lane;
            kb[j] = g < n ? kin[g] : K(0);
        }
#pragma unroll
        for (int j = 0; j < kRsBatch; j++) {
            const bool valid = wbase + (r0 + j) * 64 + lane < n;
            add_digit_runs(wc[w], valid ? digit_of(kb[j], shift, mask) : 0u, valid, lane);
        }
    }
    __syncthreads();
    for (int d = threadIdx.x; d < ND; d += RB) {
        uint32_t run = goff[(int64_t)d * nb + blockIdx.x];
        for (int ww = 0; ww < RW; ww++) {
            uint32_t c = wc[ww][d];
            wc[ww][d] = run;
            run += c;
        }
    }
    __syncthreads();
    const uint64_t lt = (lane == 0) ? 0ull : ((~0ull) >> (64 - lane));
    for (int r0 = 0; r0 < rr; r0 += kRsBatch) {
        K kb[kRsBatch];
        uint32_t vb[kRsBatch];
#pragma unroll
        for (int j = 0; j < kRsBatch; j++) {
            const int64_t g = wbase + (r0 + j) * 64 + lane;
            kb[j] = g < n ? kin[g] : K(0);
            vb[j] = g < n ? vin[g] : 0u;
        }
#pragma unroll
        for (int j = 0; j < kRsBatch; j++) {
            const bool valid = wbase + (r0 + j) * 64 + lane < n;
            const K k = kb[j];
            const uint32_t v = vb[j];
            const uint32_t d = valid ? digit_of(k, shift, mask) : 0u;
            uint64_t same = __ballot(valid);
#pragma unroll
            for (int b = 0; b < DB; b++) {
                bool bit = (d >> b) & 1u;
                uint64_t bb = __ballot(valid && bit);
                same &= bit ? bb : ~bb;
            }
            uint32_t rank = (uint32_t)__popcll(same & lt);
            uint32_t basev = valid ? wc[w][d] : 0u;
            if (valid) {
                kout[basev + rank] = k;
                vout[basev + rank] = v;
            }
            bool leader = valid && ((same >> lane) == 1ull);
            if (leader) wc[w][d] = basev + (uint32_t)__popcll(same);
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
            __builtin_amdgcn_wave_barrier();
        }
    }
}

template <class K, int DB>
void rs_pass(const K* ki, const uint32_t* vi, K* ko, uint32_t* vo, int64_t n, int sh, int w, int64_t nb, int rr,
             uint32_t* ghist, uint32_t* goff, void* sws, hipStream_t s) {
    const uint32_t mask = (1u << w) - 1u;
    k_rs_hist<K, DB><<<(unsigned)nb, RB, 0, s>>>(ki, n, sh, mask, ghist, nb, rr);
    scan_impl<uint32_t>(ghist, goff, nullptr, (int64_t)(1 << DB) * nb, sws, s);
    k_rs_scatter<K, DB><<<(unsigned)nb, RB, 0, s>>>(ki, vi, ko, vo, n, sh, mask, goff, nb, rr);
}

// LSD passes of at most kMaxDigitBits bits, the bits spread evenly over them
template <class K>
void sort_impl(K* ka, uint32_t* va, K* kb, uint32_t* vb, int64_t n, int bit0, int bit1, void* ws,
               hipStream_t s) {
    if (n <= 1 || bit1 <= bit0) return;
    const int rr = rs_rounds(n);
    const int64_t nb = (n + (int64_t)RB * rr - 1) / ((int64_t)RB * rr);
    uint32_t* ghist = (uint32_t*)ws;
    uint32_t* goff = ghist + ((size_t)1 << kMaxDigitBits) * nb;
    void* sws = goff + ((size_t)1 << kMaxDigitBits) * nb;
    K *ki = ka, *ko = kb;
    uint32_t *vi = va, *vo = vb;
    const int bits = bit1 - bit0;
    const int passes = (bits + kMaxDigitBits - 1) / kMaxDigitBits;
    int sh = bit0;
    for (int ps = 0; ps < passes; ps++) {
        const int w = (bit1 - sh + (passes - ps) - 1) / (passes - ps);  // ceil(remaining / passes left)
        switch (w <= 6 ? 6 : w) {
            case 6: rs_pass<K, 6>(ki, vi, ko, vo, n, sh, w, nb, rr, ghist, goff, sws, s); break;
            case 7: rs_pass<K, 7>(ki, vi, ko, vo, n, sh, w, nb, rr, ghist, goff, sws, s); break;
            case 8: rs_pass<K, 8>(ki, vi, ko, vo, n, sh, w, nb, rr, ghist, goff, sws, s); break;
            case 9: rs_pass<K, 9>(ki, vi, ko, vo, n, sh, w, nb, rr, ghist, goff, sws, s); break;
            case 10: rs_pass<K, 10>(ki, vi, ko, vo, n, sh, w, nb, rr, ghist, goff, sws, s); break;
            default: rs_pass<K, 11>(ki, vi, ko, vo, n, sh, w, nb, rr, ghist, goff, sws, s); break;
        }
        sh += w;
        K* tk = ki; ki = ko; ko = tk;
        uint32_t* tv = vi; vi = vo; vo = tv;
    }
    if (passes & 1) {
        hipMemcpyAsync(ka, ki, n * sizeof(K), hipMemcpyDeviceToDevice, s);
        hipMemcpyAsync(va, vi, n * sizeof(uint32_t), hipMemcpyDeviceToDevice, s);
    }
}


// Scans over a count held in device memory (written by an earlier kernel on
// the stream, so the host launches them without reading it): a fixed grid of
// SG workgroups, each taking a contiguous run of tiles.
constexpr int SG = 256;

template <class T>
__global__ void k_scand_reduce(const T* __restrict__ in, DevCount cnt, T* __restrict__ part) {
    __shared__ uint32_t lds[SB / 64];
    const int64_t n = cnt.get();
    const int64_t ntile = (n + ST - 1) / ST, per = (ntile + SG - 1) / SG;
    const int64_t g0 = (int64_t)blockIdx.x * per * ST, g1 = min(g0 + per * ST, n);
    T out;
    for (int c = 0; c < Ops<T>::C; c++) {
        uint32_t acc = 0;
        for (int64_t g = g0 + threadIdx.x; g < g1; g += SB) acc += Ops<T>::get(in[g], c);
        uint32_t tot;
        block_excl_u32(acc, lds, &tot);
        Ops<T>::set(out, c, tot);
    }
    if (threadIdx.x == 0) part[blockIdx.x] = out;
}

template <class T>
__global__ void k_scand_down(const T* __restrict__ in, T* __restrict__ out, DevCount cnt,
                             const T* __restrict__ part) {
    __shared__ uint32_t lds[SB / 64];
    const int64_t n = cnt.get();
    const int64_t ntile = (n + ST - 1) / ST, per = (ntile + SG - 1) / SG;
    const int64_t t0 = (int64_t)blockIdx.x * per, t1 = min(t0 + per, ntile);
    uint32_t carry[Ops<T>::C];
    const T pb = part[blockIdx.x];
    for (int c = 0; c < Ops<T>::C; c++) carry[c] = Ops<T>::get(pb, c);
    for (int64_t tile = t0; tile < t1; tile++) {  // uniform over the workgroup
        const int64_t base = tile * ST + (int64_t)threadIdx.x * SI;
        T v[SI], res[SI];
#pragma unroll
        for (int j = 0; j < SI; j++) {
            const int64_t g = base + j;
            if (g < n) v[j] = in[g];
            else
                for (int c = 0; c < Ops<T>::C; c++) Ops<T>::set(v[j], c, 0u);
        }
        for (int c = 0; c < Ops<T>::C; c++) {
            uint32_t sum = 0;
#pragma unroll
            for (int j = 0; j < SI; j++) sum += Ops<T>::get(v[j], c);
            uint32_t tot;
            uint32_t run = block_excl_u32(sum, lds, &tot) + carry[c];
#pragma unroll
            for (int j = 0; j < SI; j++) {
                Ops<T>::set(res[j], c, run);
                run += Ops<T>::get(v[j], c);
            }
            carry[c] += tot;
        }
#pragma unroll
        for (int j = 0; j < SI; j++) {
            const int64_t g = base + j;
            if (g < n) out[g] = res[j];
        }
    }
}

template <class T>
void scand_impl(const T* in, T* out, T* total, DevCount n, void* ws, hipStream_t s) {
    T* part = (T*)ws;
    k_scand_reduce<T><<<SG, SB, 0, s>>>(in, n, part);
    k_scan_partials<T><<<1, SB, 0, s>>>(part, SG, total);
    k_scand_down<T><<<SG, SB, 0, s>>>(in, out, n, part);
}

__global__ void k_fill_i32(int32_t* p, int32_t v, int64_t n) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

// words [0, n4) as 16-byte stores from the first 16-byte boundary, the
// words before it (head) and after the last whole vector one by one
__global__ void k_zero(uint32_t* p, int64_t n, int64_t head) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t nv = (n - head) / 4;
    if (i < nv) {
        uint4 z = make_uint4(0, 0, 0, 0);
        *(uint4*)(p + head + 4 * i) = z;
    }
    if (i < head) p[i] = 0;
    const int64_t tail = head + 4 * nv;
    if (i < n - tail) p[tail + i] = 0;
}

__global__ void k_iota_u32(uint32_t* p, int64_t n) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = (uint32_t)i;
}

}  // namespace

size_t scan_ws_bytes(int64_t n) {
    int64_t nb = (n + ST - 1) / ST + 1;
    return (size_t)nb * sizeof(uint4) + 256;
}

void scan_u32(const uint32_t* in, uint32_t* out, uint32_t* total, int64_t n, void* ws,
              hipStream_t s) {
    scan_impl<uint32_t>(in, out, total, n, ws, s);
}

void scan_u32x4(const uint4* in, uint4* out, uint4* total, int64_t n, void* ws, hipStream_t s) {
    scan_impl<uint4>(in, out, total, n, ws, s);
}

size_t scan_dev_ws_bytes() { return (size_t)SG * sizeof(uint4) + 256; }

void scan_u32_dev(const uint32_t* in, uint32_t* out, uint32_t* total, DevCount n, void* ws, hipStream_t s) {
    scand_impl<uint32_t>(in, out, total, n, ws, s);
}

void scan_u32x4_dev(const uint4* in, uint4* out, uint4* total, DevCount n, void* ws, hipStream_t s) {
    scand_impl<uint4>(in, out, total, n, ws, s);
}

size_t sort_ws_bytes(int64_t n) {
    int64_t nb = (n + RT - 1) / RT + 1;
    const int64_t nd = (int64_t)1 << kMaxDigitBits;
    return (size_t)2 * nd * nb * sizeof(uint32_t) + scan_ws_bytes(nd * nb) + 256;
}

void sort_u64(uint64_t* ka, uint32_t* va, uint64_t* kb, uint32_t* vb, int64_t n, int bit0,
              int bit1, void* ws, hipStream_t s) {
    sort_impl<uint64_t>(ka, va, kb, vb, n, bit0, bit1, ws, s);
}

void sort_u32(uint32_t* ka, uint32_t* va, uint32_t* kb, uint32_t* vb, int64_t n, int bit0,
              int bit1, void* ws, hipStream_t s) {
    sort_impl<uint32_t>(ka, va, kb, vb, n, bit0, bit1, ws, s);
}

void fill_i32(int32_t* p, int32_t v, int64_t n, hipStream_t s) {
    if (n <= 0) return;
    k_fill_i32<<<(unsigned)((n + 255) / 256), 256, 0, s>>>(p, v, n);
}

void fill_zero(void* p, size_t bytes, hipStream_t s) {
    const int64_t n = (int64_t)(bytes / 4);
    if (n <= 0) return;
    int64_t head = (int64_t)((16 - ((uintptr_t)p & 15)) & 15) / 4;
    if (head > n) head = n;
    const int64_t threads = std::max<int64_t>((n - head) / 4, 4);
    k_zero<<<(unsigned)((threads + 255) / 256), 256, 0, s>>>((uint32_t*)p, n, head);
}

void iota_u32(uint32_t* p, int64_t n, hipStream_t s) {
    if (n <= 0) return;
    k_iota_u32<<<(unsigned)((n + 255) / 256), 256, 0, s>>>(p, n);
}

}  // namespace fmm

namespace fmm {
namespace {

__device__ inline uint64_t mix64(uint64_t z) {
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

// Artificial coordinates (uniform in the unit cube) and charges (+-1) for the
// kernel pre-calculation: a SplitMix64 finaliser of (seed, index, component).
__global__ void k_artificial(int64_t n, uint64_t seed, float* __restrict__ x, float* __restrict__ y,
                             float* __restrict__ z, float* __restrict__ q) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    uint64_t b = seed * 0x9E3779B97F4A7C15ull + (uint64_t)i * 4;
    x[i] = (float)(mix64(b + 1) >> 40) * (1.0f / 16777216.0f);
    y[i] = (float)(mix64(b + 2) >> 40) * (1.0f / 16777216.0f);
    z[i] = (float)(mix64(b + 3) >> 40) * (1.0f / 16777216.0f);
    q[i] = (mix64(b + 4) >> 63) ? 1.f : -1.f;
}

}  // namespace

void artificial_points(int64_t n, uint64_t seed, float* x, float* y, float* z, float* q, hipStream_t s) {
    if (n <= 0) return;
    k_artificial<<<(unsigned)((n + 255) / 256), 256, 0, s>>>(n, seed, x, y, z, q);
}

}  // namespace fmm
