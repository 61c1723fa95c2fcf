// Periodic cell sort of a run's particles (gfx950).
//
// Reorders (s, w) by the cell of the particle's left node,
// key = clamp(floor(s - 1), -1, ng - 1) + 1 in [0, ng], the same index the
// gather and the deposit use, so that neighbouring lanes work on
// neighbouring cells.  The sort is a stable counting sort, so the order it
// produces depends only on the particles (never on timing), and every later
// result stays deterministic:
//   1. count:   segment s (seg particles) counts its keys in LDS and stores
//               them key-major, table[key * nseg + s];
//   2. scan:    one exclusive prefix sum over the whole table gives the
//               first destination of (key, segment) in the sorted order;
//   3. scatter: each wavefront of a segment's workgroup takes a contiguous
//               quarter of the segment, recounts it, and places its
//               particles in input order (lanes with equal keys are ranked
//               by lane within a 64-particle group, groups in order);
//   4. swap:    the descriptor's particle arrays and their alternates trade
//               places, so captured launches pick up the sorted arrays.
// The physics is unchanged: a step treats every particle independently and
// the fixed-point deposit does not depend on order.
#include <algorithm>

#include "pic_internal.h"

namespace pic1d {

namespace {

constexpr int kSortBlock = 256;                 // 4 wavefronts
constexpr int kSortWaves = kSortBlock / 64;
constexpr int kScanBlock = 256;
constexpr int kScanItems = 16;                  // consecutive elements per thread
constexpr int kScanTile = kScanBlock * kScanItems;
constexpr int kTopBlock = 1024;
constexpr int kKeyBits = 14;                    // keys <= kMaxNg = 2^13
constexpr int kScatterRing = 4;                 // 64-particle groups in flight per wavefront in the scatter

template <typename T>
__device__ __forceinline__ int cell_key(T s, int ng) {
    const int j = min(max((int)__builtin_floor(s - T(1)), -1), ng - 1);
    return j + 1;
}

__device__ __forceinline__ int lane_id() { return (int)(threadIdx.x & 63); }

// Active lanes whose key equals this lane's key.
__device__ __forceinline__ unsigned long long match_key(int key) {
    const unsigned long long act = __ballot(1);
    const int k0 = __builtin_amdgcn_readfirstlane(key);
    const unsigned long long same = __ballot(key == k0);
    if (same == act) return act;                // common after a sort: one key per group
    unsigned long long peers = act;
#pragma unroll
    for (int b = 0; b < kKeyBits; ++b) {
        const bool bit = (key >> b) & 1;
        const unsigned long long m = __ballot(bit);
        peers &= bit ? m : ~m;
    }
    return peers;
}

// h[key] += 1 for every active lane, one LDS atomic per distinct key when
// the group shares the first lane's key.
__device__ __forceinline__ void count_key(uint32_t *h, int key) {
    const int k0 = __builtin_amdgcn_readfirstlane(key);
    const unsigned long long same = __ballot(key == k0);
    if (key == k0) {
        if (lane_id() == __builtin_ctzll(same)) atomicAdd(h + k0, (uint32_t)__popcll(same));
    } else {
        atomicAdd(h + key, 1u);
    }
}

// Segment of workgroup b: workgroups are dispatched to the device's 8 XCDs
// in turn (b mod 8), so consecutive segments, which share the lines of the
// key-major count table, go to workgroups of one XCD, whose L2 then holds
// whole lines.  A bijection of [0, nseg) for any nseg: XCD x takes a
// contiguous range of nseg / 8 segments (one more for the first nseg mod 8).
constexpr int kXcds = 8;
__device__ __forceinline__ int segment_of(int b, int nseg) {
    const int x = b % kXcds, local = b / kXcds;
    const int full = nseg / kXcds, rem = nseg % kXcds;
    return x < rem ? x * (full + 1) + local : rem * (full + 1) + (x - rem) * full + local;
}

// Particle arrays as global-memory pointers: the descriptor holds generic
// ones, whose accesses the compiler would issue as flat operations, which
// every LDS wait in the scatter loop would also wait for.
#define GLOBAL_AS __attribute__((address_space(1)))

// 16-byte vectors of the particle state (4 FP32 or 2 FP64 values).
template <typename T>
struct Vec16;
template <>
struct Vec16<float> {
    typedef float __attribute__((ext_vector_type(4))) type;
    static constexpr int n = 4;
};
template <>
struct Vec16<double> {
    typedef double __attribute__((ext_vector_type(2))) type;
    static constexpr int n = 2;
};

// h[key] += 1 for the keys of u[i0, i1), counted by `nthr` threads (thread
// `tid` of them) in 16-byte vectors, kCountVecs per thread in flight, then
// the last partial vector one value per thread.  Counting does not depend on
// order, so a thread may take any values.  i0 must be a multiple of the
// vector width (the particle arrays start 256-byte aligned).
constexpr int kCountVecs = 4;
template <typename T>
__device__ __forceinline__ void count_range(uint32_t *h, const GLOBAL_AS T *u, int64_t i0, int64_t i1, int tid,
                                            int nthr, int ng) {
    using V = typename Vec16<T>::type;
    constexpr int VEC = Vec16<T>::n;
    const int64_t nv = (i1 - i0) / VEC;               // whole vectors
    const GLOBAL_AS V *uv = (const GLOBAL_AS V *)(u + i0);
    for (int64_t v0 = tid; v0 < nv; v0 += (int64_t)nthr * kCountVecs) {
        V buf[kCountVecs];
#pragma unroll
        for (int q = 0; q < kCountVecs; ++q) {
            const int64_t v = v0 + (int64_t)q * nthr;
            if (v < nv) buf[q] = uv[v];
        }
#pragma unroll
        for (int q = 0; q < kCountVecs; ++q) {
            if (v0 + (int64_t)q * nthr < nv) {
#pragma unroll
                for (int j = 0; j < VEC; ++j) count_key(h, cell_key(buf[q][j], ng));
            }
        }
    }
    for (int64_t i = i0 + nv * VEC + tid; i < i1; i += nthr) count_key(h, cell_key(u[i], ng));
}

template <typename T>
__global__ __launch_bounds__(kSortBlock) void sort_count_kernel(const RunDev *R, int seg, int nseg,
                                                                uint32_t *table) {
    extern __shared__ uint32_t h[];             // [ng + 1]
    const int ng = R->ng;
    const int64_t np = R->np;
    const GLOBAL_AS T *u = (const GLOBAL_AS T *)R->u;
    for (int k = threadIdx.x; k <= ng; k += kSortBlock) h[k] = 0;
    __syncthreads();
    const int s = segment_of((int)blockIdx.x, nseg);
    const int64_t b0 = (int64_t)s * seg, b1 = min(np, b0 + seg);   // seg: a multiple of 1024
    count_range<T>(h, u, b0, b1, (int)threadIdx.x, kSortBlock, ng);
    __syncthreads();
    for (int k = threadIdx.x; k <= ng; k += kSortBlock) table[(size_t)k * nseg + s] = h[k];
}

// Exclusive scan of v over the 256 threads of a block, in thread order.
__device__ __forceinline__ uint32_t block_exclusive_scan(uint32_t v, uint32_t *red, uint32_t *total) {
    const int lane = lane_id(), wv = threadIdx.x >> 6;
    uint32_t inc = v;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const uint32_t t = __shfl_up(inc, o);
        if (lane >= o) inc += t;
    }
    if (lane == 63) red[wv] = inc;
    __syncthreads();
    uint32_t off = 0, tot = 0;
    for (int k = 0; k < kScanBlock / 64; ++k) {
        if (k < wv) off += red[k];
        tot += red[k];
    }
    __syncthreads();
    *total = tot;
    return off + inc - v;
}

__global__ __launch_bounds__(kScanBlock) void scan_reduce_kernel(const uint32_t *a, int64_t n, uint32_t *bsum) {
    __shared__ uint32_t red[kScanBlock / 64];
    const int64_t b0 = (int64_t)blockIdx.x * kScanTile;
    uint32_t v = 0;
#pragma unroll
    for (int i = 0; i < kScanItems; ++i) {
        const int64_t k = b0 + (int64_t)i * kScanBlock + threadIdx.x;
        if (k < n) v += a[k];
    }
    uint32_t tot;
    (void)block_exclusive_scan(v, red, &tot);
    if (threadIdx.x == 0) bsum[blockIdx.x] = tot;
}

// Exclusive scan of the block sums in place (one workgroup).
__global__ __launch_bounds__(kTopBlock) void scan_top_kernel(uint32_t *bsum, int nb) {
    __shared__ uint32_t red[kTopBlock / 64];
    const int lane = lane_id(), wv = threadIdx.x >> 6;
    uint32_t carry = 0;
    for (int base = 0; base < nb; base += kTopBlock) {
        const int k = base + threadIdx.x;
        const uint32_t v = k < nb ? bsum[k] : 0u;
        uint32_t inc = v;
#pragma unroll
        for (int o = 1; o < 64; o <<= 1) {
            const uint32_t t = __shfl_up(inc, o);
            if (lane >= o) inc += t;
        }
        if (lane == 63) red[wv] = inc;
        __syncthreads();
        uint32_t off = 0, tot = 0;
        for (int q = 0; q < kTopBlock / 64; ++q) {
            if (q < wv) off += red[q];
            tot += red[q];
        }
        __syncthreads();
        if (k < nb) bsum[k] = carry + off + inc - v;
        carry += tot;
    }
}

// Each thread's kScanItems consecutive entries move as 16-byte vectors when
// they are all inside the table (the table starts 256-byte aligned and b0 is
// a multiple of kScanItems), one by one at its end.
__global__ __launch_bounds__(kScanBlock) void scan_down_kernel(uint32_t *a, int64_t n, const uint32_t *bsum) {
    typedef uint32_t __attribute__((ext_vector_type(4))) u32x4;
    static_assert(kScanItems % 4 == 0, "whole vectors per thread");
    __shared__ uint32_t red[kScanBlock / 64];
    const int64_t b0 = (int64_t)blockIdx.x * kScanTile + (int64_t)threadIdx.x * kScanItems;
    const bool whole = b0 + kScanItems <= n;
    uint32_t v[kScanItems];
    if (whole) {
#pragma unroll
        for (int q = 0; q < kScanItems / 4; ++q) {
            const u32x4 t = *(const u32x4 *)(a + b0 + 4 * q);
#pragma unroll
            for (int j = 0; j < 4; ++j) v[4 * q + j] = t[j];
        }
    } else {
#pragma unroll
        for (int i = 0; i < kScanItems; ++i) v[i] = b0 + i < n ? a[b0 + i] : 0u;
    }
    uint32_t sum = 0;
#pragma unroll
    for (int i = 0; i < kScanItems; ++i) sum += v[i];
    uint32_t tot;
    uint32_t run = bsum[blockIdx.x] + block_exclusive_scan(sum, red, &tot);
    uint32_t out[kScanItems];
#pragma unroll
    for (int i = 0; i < kScanItems; ++i) {
        out[i] = run;
        run += v[i];
    }
    if (whole) {
#pragma unroll
        for (int q = 0; q < kScanItems / 4; ++q)
            *(u32x4 *)(a + b0 + 4 * q) = u32x4{out[4 * q], out[4 * q + 1], out[4 * q + 2], out[4 * q + 3]};
    } else {
#pragma unroll
        for (int i = 0; i < kScanItems; ++i)
            if (b0 + i < n) a[b0 + i] = out[i];
    }
}

// Place one 64-particle group (lanes with `valid` set) in input order: lanes
// with equal keys are ranked by lane, after the wavefront's earlier
// particles of that key (`mine`).  A destination outside [0, np), which the
// count and the scan make impossible, goes to the last slot instead (memory
// stays in bounds) and sets `bad`; the store is issued for every valid lane,
// so the loop's memory operations do not depend on the data.
template <typename T>
__device__ __forceinline__ void place_group(T su, T sw, uint32_t *mine, GLOBAL_AS T *uo, GLOBAL_AS T *wo,
                                            int64_t np, int ng, int lane, uint32_t &bad) {
    const int key = cell_key(su, ng);
    const unsigned long long peers = match_key(key);
    const int leader = __builtin_ctzll(peers);
    const uint32_t rank = (uint32_t)__popcll(peers & ((1ull << lane) - 1ull));
    uint32_t base = 0;
    if (lane == leader) {
        base = mine[key];
        mine[key] = base + (uint32_t)__popcll(peers);
    }
    base = (uint32_t)__shfl((int)base, leader);
    const uint32_t dst = base + rank;
    const bool ok = dst < (uint64_t)np;
    bad |= ok ? 0u : 1u;
    const int64_t d = ok ? (int64_t)dst : np - 1;
    uo[d] = su;
    wo[d] = sw;
}

template <typename T>
__global__ __launch_bounds__(kSortBlock) void sort_scatter_kernel(RunDev *R, int seg, int nseg,
                                                                  const uint32_t *offs) {
    extern __shared__ uint32_t cw[];            // [kSortWaves][ng + 1]
    const int ng = R->ng, nk = ng + 1;
    const int64_t np = R->np;
    const GLOBAL_AS T *u = (const GLOBAL_AS T *)R->u;
    const GLOBAL_AS T *w = (const GLOBAL_AS T *)R->w;
    GLOBAL_AS T *uo = (GLOBAL_AS T *)R->u_alt;
    GLOBAL_AS T *wo = (GLOBAL_AS T *)R->w_alt;
    const int s = segment_of((int)blockIdx.x, nseg), wave = threadIdx.x >> 6, lane = lane_id();
    const int64_t b0 = (int64_t)s * seg, b1 = min(np, b0 + seg);
    const int64_t sub = (b1 - b0 + kSortBlock - 1) / kSortBlock * 64;    // per wavefront, multiple of 64
    const int64_t w0 = min(b1, b0 + wave * sub), w1 = min(b1, w0 + sub);
    uint32_t *mine = cw + wave * nk;
    for (int k = threadIdx.x; k < kSortWaves * nk; k += kSortBlock) cw[k] = 0;
    __syncthreads();
    count_range<T>(mine, u, w0, w1, lane, 64, ng);   // w0 - b0: a multiple of 64
    __syncthreads();
    // first destination of (key, wavefront): the segment's offset plus the
    // counts of the earlier wavefronts
    for (int k = threadIdx.x; k < nk; k += kSortBlock) {
        uint32_t run = offs[(size_t)k * nseg + s];
        for (int v = 0; v < kSortWaves; ++v) {
            const uint32_t c = cw[v * nk + k];
            cw[v * nk + k] = run;
            run += c;
        }
    }
    __syncthreads();
    // Groups of 64 consecutive particles in input order, kScatterRing of
    // them in registers: group g is placed from set g mod kScatterRing, which
    // is refilled with group g + kScatterRing at once (addresses past the
    // wavefront's range are clamped into it, so every load is issued), so
    // the loads of the next groups are in flight while one is placed.  Whole
    // rounds of whole groups run without data-dependent branches around
    // memory operations; the rest, from the same registers, lane by lane.
    uint32_t bad = 0;
    if (w1 > w0) {
        const int64_t ngroups = (w1 - w0 + 63) / 64, nfull = (w1 - w0) / 64;
        const int64_t last = w1 - 1;
        T bu[kScatterRing], bw[kScatterRing];
#pragma unroll
        for (int d = 0; d < kScatterRing; ++d) {
            const int64_t i = min(w0 + d * 64 + lane, last);
            bu[d] = u[i];
            bw[d] = w[i];
        }
        const int64_t rounds = nfull / kScatterRing;
        for (int64_t r = 0; r < rounds; ++r) {
#pragma unroll
            for (int d = 0; d < kScatterRing; ++d) {
                const int64_t i = w0 + (r * kScatterRing + d) * 64 + lane;
                const T su = bu[d], sw = bw[d];
                const int64_t ahead = min(i + 64 * kScatterRing, last);
                bu[d] = u[ahead];
                bw[d] = w[ahead];
                place_group<T>(su, sw, mine, uo, wo, np, ng, lane, bad);
            }
        }
#pragma unroll
        for (int d = 0; d < kScatterRing; ++d) {
            const int64_t g = rounds * kScatterRing + d;
            if (g < ngroups) {
                const int64_t i = w0 + g * 64 + lane;
                if (i < w1) place_group<T>(bu[d], bw[d], mine, uo, wo, np, ng, lane, bad);
            }
        }
    }
    if (bad) atomicOr(&R->flags, 4u);
}

__global__ void sort_swap_kernel(RunDev *R) {
    if (threadIdx.x == 0) {
        void *t = R->u;
        R->u = R->u_alt;
        R->u_alt = t;
        t = R->w;
        R->w = R->w_alt;
        R->w_alt = t;
        R->sort_swap ^= 1;
    }
}

size_t align256(size_t b) { return (b + 255) & ~(size_t)255; }

}  // namespace

SortPlan sort_plan(int64_t np, int ng) {
    SortPlan p{};
    const int64_t per = (np + kMaxSortSegments - 1) / kMaxSortSegments;
    p.seg = (int)std::max<int64_t>(4096, (per + 1023) / 1024 * 1024);
    p.nseg = (int)((np + p.seg - 1) / p.seg);
    p.table_len = (int64_t)(ng + 1) * p.nseg;
    p.nblk = (int)((p.table_len + kScanTile - 1) / kScanTile);
    return p;
}

size_t sort_scratch_bytes(int64_t np, int ng) {
    const SortPlan p = sort_plan(np, ng);
    return align256((size_t)p.table_len * 4) + align256((size_t)p.nblk * 4);
}

hipError_t sort_prepare() {
    const size_t lds = (size_t)kSortWaves * (kMaxNg + 1) * sizeof(uint32_t);
    hipError_t e = hipFuncSetAttribute((const void *)sort_scatter_kernel<float>,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
    return hipFuncSetAttribute((const void *)sort_scatter_kernel<double>,
                               hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
}

hipError_t launch_sort(RunDev *R, int64_t np, int ng, int precision, void *scratch, hipStream_t stream) {
    if (np < 1 || ng < 2 || ng > kMaxNg || !scratch) return hipErrorInvalidValue;
    const SortPlan p = sort_plan(np, ng);
    uint32_t *table = (uint32_t *)scratch;
    uint32_t *bsum = (uint32_t *)((char *)scratch + align256((size_t)p.table_len * 4));
    const size_t lds_count = (size_t)(ng + 1) * sizeof(uint32_t);
    const size_t lds_scatter = (size_t)kSortWaves * lds_count;
    int seg = p.seg, nseg = p.nseg, nb = p.nblk;
    int64_t n = p.table_len;
    void *cargs[] = {(void *)&R, (void *)&seg, (void *)&nseg, (void *)&table};
    const void *count = precision ? (const void *)sort_count_kernel<double> : (const void *)sort_count_kernel<float>;
    hipError_t e = hipLaunchKernel(count, dim3(nseg), dim3(kSortBlock), cargs, lds_count, stream);
    if (e != hipSuccess) return e;
    void *rargs[] = {(void *)&table, (void *)&n, (void *)&bsum};
    e = hipLaunchKernel((const void *)scan_reduce_kernel, dim3(nb), dim3(kScanBlock), rargs, 0, stream);
    if (e != hipSuccess) return e;
    void *targs[] = {(void *)&bsum, (void *)&nb};
    e = hipLaunchKernel((const void *)scan_top_kernel, dim3(1), dim3(kTopBlock), targs, 0, stream);
    if (e != hipSuccess) return e;
    e = hipLaunchKernel((const void *)scan_down_kernel, dim3(nb), dim3(kScanBlock), rargs, 0, stream);
    if (e != hipSuccess) return e;
    const void *scatter =
        precision ? (const void *)sort_scatter_kernel<double> : (const void *)sort_scatter_kernel<float>;
    void *sargs[] = {(void *)&R, (void *)&seg, (void *)&nseg, (void *)&table};
    e = hipLaunchKernel(scatter, dim3(nseg), dim3(kSortBlock), sargs, lds_scatter, stream);
    if (e != hipSuccess) return e;
    void *wargs[] = {(void *)&R};
    return hipLaunchKernel((const void *)sort_swap_kernel, dim3(1), dim3(64), wargs, 0, stream);
}

}  // namespace pic1d
