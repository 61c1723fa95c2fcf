// Device kernels of the 1D electrostatic PIC step (gfx950).
//
// A step is two launches on one stream:
//   step_kernel (particle pass): gather E^n (Sec. 2.3) -> kick (Sec. 2.1) ->
//     drift + periodic wrap (Sec. 2.1) -> exact fixed-point charge deposit
//     (Sec. 2.3) into a workgroup-private int64 grid in LDS -> merge into the
//     run's global grid with 64-bit atomics, plus per-tile FP64 partial sums
//     of the diagnostics;
//   solve_kernel (pic_solve.hip, one workgroup per run): the periodic
//     Poisson problem and the central-difference field (Sec. 2.2) in FP64,
//     writing E^{n+1}, the gather table for the next step and the step's
//     diagnostics.
// The kernel boundary orders the merge before the solve, so no device-wide
// fence or completion counter is needed.

// Particles are independent within a step, so they are sharded by index
// (tiles of `tile` particles, one tile per wavefront at a time) instead of by
// domain; the grid reduction replaces the paper's ghost-cell exchange and the
// solve replaces its distributed CG.  All per-run reductions use fixed
// orders that depend only on the run's (np, ng, tile), never on the launch
// shape (block size, unroll, grid, batch membership), so a run gives
// bit-identical results alone or batched with others.
//
// Stored position: s = x/dx + 1/2 in [1/2, ng + 1/2).  Then t = s - 1 =
// x/dx - 1/2 (the position measured from node 0, nodes at (g + 1/2) dx) is
// exact, and so are j = floor(t) and the fraction f = t - j; in FP32,
// f 2^32 is an integer, so the fixed-point deposit needs no 64-bit
// arithmetic.  The host reads positions back as s - 1/2 (also exact).
#include "pic_internal.h"

namespace pic1d {

namespace {

#define GLOBAL_AS __attribute__((address_space(1)))

typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef double f64x2 __attribute__((ext_vector_type(2)));

template <typename T> struct Vec;
template <> struct Vec<float> { using type = f32x4; static constexpr int n = 4; };
template <> struct Vec<double> { using type = f64x2; static constexpr int n = 2; };

// Streaming accesses to particle arrays, global address space.  NT marks
// them non-temporal (each particle is touched once per step); without it they
// are ordinary cached accesses, which let a particle state smaller than the
// device's last-level cache stay there from one step to the next.
template <typename V, bool NT>
__device__ __forceinline__ V load_stream(const void *p) {
    if constexpr (NT) return __builtin_nontemporal_load((const GLOBAL_AS V *)p);
    else return *(const GLOBAL_AS V *)p;
}
template <typename V, bool NT>
__device__ __forceinline__ void store_stream(void *p, V v) {
    if constexpr (NT) __builtin_nontemporal_store(v, (GLOBAL_AS V *)p);
    else *(GLOBAL_AS V *)p = v;
}

__device__ __forceinline__ float fma_t(float a, float b, float c) { return __builtin_fmaf(a, b, c); }
__device__ __forceinline__ double fma_t(double a, double b, double c) { return __builtin_fma(a, b, c); }

// 32-bit fraction F = floor(f 2^32) of a cell fraction f in [0, 1).
// FP32: f is a multiple of 2^-24, so f 2^32 is an exact integer.
__device__ __forceinline__ uint32_t frac32(float f) { return (uint32_t)(f * 4294967296.0f); }
__device__ __forceinline__ uint32_t frac32(double f) { return (uint32_t)(f * 4294967296.0); }


// Per-particle stages.  Conventions:
//   s, w : stored position (x/dx + 1/2) and velocity w = v dt/dx
//   Et   : gather table in LDS, Et[g+1] = E_g scaled to the change of w per
//          step, with ghosts Et[0] = E_{ng-1} and Et[ng+1] = E_0
//   Sl   : workgroup-private int64 grid in LDS, node g at Sl[g+1], ghosts
//          Sl[0] (node -1 = ng-1) and Sl[ng+1] (node ng = 0)
// Node indices are clamped to [-1, ng-1] so no value of s can address
// outside the tables.

// Field at the particle from the two nearest nodes (Sec. 2.3):
// (1-f) E_j + f E_{j+1} with j = floor(x/dx - 1/2), f the fraction.
template <typename T>
__device__ __forceinline__ T gather(T s, const T *Et, int ng) {
    const T t = s - T(1);
    const T jf = __builtin_floor(t);
    const T f = t - jf;
    const int j = min(max((int)jf, -1), ng - 1);
    const T El = Et[j + 1];
    const T Er = Et[j + 2];
    return fma_t(f, Er - El, El);
}

// Leapfrog kick and drift with periodic wrap (Sec. 2.1).
template <typename T>
__device__ __forceinline__ void push(T &s, T &w, T Ep, T ngf, T hi, uint32_t &flags) {
    w = w + Ep;                                   // v^{n+1/2} = v^{n-1/2} + qm E dt
    T sn = s + w;                                 // x^{n+1} = x^n + v^{n+1/2} dt
    sn = sn + (sn < T(0.5) ? ngf : (sn >= hi ? -ngf : T(0)));
    if (!(sn >= T(0.5) && sn < hi)) {             // rare: rounding to the end, |w| >= ng, NaN
        if (sn == hi) {
            sn = T(0.5);
        } else if (!__builtin_isfinite(sn)) {
            sn = T(0.5);
            flags |= 1u;
        } else {
            sn = sn - ngf * __builtin_floor((sn - T(0.5)) / ngf);
            if (!(sn >= T(0.5) && sn < hi)) sn = T(0.5);
            flags |= 2u;
        }
    }
    s = sn;
}

// Add the lane's pair (2^32 - F at node j, F at node j + 1) to the LDS
// grid.  Plain LDS atomics also when many lanes share a node (cell-ordered
// particles, quiet starts): on gfx950 a wavefront's same-address LDS
// atomics cost about as much as a wavefront pre-reduction, measured on
// sorted and unsorted runs, so the pass keeps the shorter code.
__device__ __forceinline__ void deposit_pair(int j, uint32_t F, unsigned long long *Sl) {
    unsigned long long *p = Sl + (j + 1);
    atomicAdd(p, (1ull << 32) - (unsigned long long)F);
    atomicAdd(p + 1, (unsigned long long)F);
}

// Exact fixed-point charge deposit (Sec. 2.3 weights): with
// U' = floor((x/dx - 1/2) 2^32) = j 2^32 + F, node j gets 2^32 - F and node
// j+1 gets F.  Also accumulates the diagnostics sums w^2 and w.
template <typename T>
__device__ __forceinline__ void deposit(T s, T w, unsigned long long *Sl, int ng, double &a1,
                                        double &a2) {
    const double wn = (double)w;
    a1 = __builtin_fma(wn, wn, a1);
    a2 += wn;
    const T t = s - T(1);
    const T jf = __builtin_floor(t);
    const uint32_t F = frac32(t - jf);
    const int j = min(max((int)jf, -1), ng - 1);
    deposit_pair(j, F, Sl);
}



// The run's gather table into LDS: Et[g + 1] = tab[g], with the ghosts
// Et[0] = tab[ng - 1] and Et[ng + 1] = tab[0].  The table (at most 64 KB,
// 256-byte aligned) is read as 16-byte vectors in rounds of kTableRound
// vectors per thread, every load of a round issued before any LDS write, so
// a round costs one memory round trip (one per table in FP32 at 640 threads
// and ng 8192, instead of one per element per thread).
constexpr int kTableRound = 4;
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));

template <typename T, int BLOCK>
__device__ __forceinline__ void fill_table(const T *tab, T *Et, int ng) {
    constexpr int PER = 16 / sizeof(T);            // table entries per vector
    const int nvec = ng / PER;
    const GLOBAL_AS u32x4 *src = (const GLOBAL_AS u32x4 *)tab;
    const GLOBAL_AS T *gtab = (const GLOBAL_AS T *)tab;
    T lo = T(0), hi = T(0);
    if (threadIdx.x == 0) {
        lo = gtab[ng - 1];
        hi = gtab[0];
    }
    for (int base = 0; base < nvec; base += BLOCK * kTableRound) {
        u32x4 buf[kTableRound];
#pragma unroll
        for (int k = 0; k < kTableRound; ++k) {
            const int i = base + k * BLOCK + (int)threadIdx.x;
            if (i < nvec) buf[k] = src[i];
        }
#pragma unroll
        for (int k = 0; k < kTableRound; ++k) {
            const int i = base + k * BLOCK + (int)threadIdx.x;
            if (i < nvec) {
                T vals[PER];
                __builtin_memcpy(vals, &buf[k], 16);
#pragma unroll
                for (int e = 0; e < PER; ++e) Et[1 + i * PER + e] = vals[e];
            }
        }
    }
    for (int g = nvec * PER + (int)threadIdx.x; g < ng; g += BLOCK) Et[g + 1] = gtab[g];
    if (threadIdx.x == 0) {
        Et[0] = lo;
        Et[ng + 1] = hi;
    }
}

// Issue the loads of one block: UNROLL vectors of VEC particles per lane,
// lane-contiguous so each load instruction covers 64*VEC particles.
template <typename V, int VEC, int UNROLL, bool NT>
__device__ __forceinline__ void load_block(const void *U, const void *W, int64_t base, int lane,
                                           V (&u)[UNROLL], V (&w)[UNROLL]) {
    using T = decltype(u[0][0] + 0);
#pragma unroll
    for (int k = 0; k < UNROLL; ++k) {
        const int64_t i = base + (int64_t)(k * 64 + lane) * VEC;
        u[k] = load_stream<V, NT>((const T *)U + i);
        w[k] = load_stream<V, NT>((const T *)W + i);
    }
}

// Push and deposit one loaded block, then store it back.  All gathers of the
// block are issued first (one LDS wait per block), then the pushes, deposits
// and stores; the accumulation order per lane is the particle order.
template <typename T, typename V, int VEC, int UNROLL, bool PUSH, bool NT>
__device__ __forceinline__ void run_block(void *U, void *W, int64_t base, int lane, V (&u)[UNROLL],
                                          V (&w)[UNROLL], const T *Et, unsigned long long *Sl, int ng,
                                          T ngf, T hi, double &a1, double &a2, uint32_t &flags) {
    if (PUSH) {
        T Ep[UNROLL][VEC];
#pragma unroll
        for (int k = 0; k < UNROLL; ++k)
#pragma unroll
            for (int e = 0; e < VEC; ++e) Ep[k][e] = gather(u[k][e], Et, ng);
#pragma unroll
        for (int k = 0; k < UNROLL; ++k) {
#pragma unroll
            for (int e = 0; e < VEC; ++e) {
                T sv = u[k][e], wv = w[k][e];
                push(sv, wv, Ep[k][e], ngf, hi, flags);
                u[k][e] = sv;
                w[k][e] = wv;
            }
        }
    }
#pragma unroll
    for (int k = 0; k < UNROLL; ++k)
#pragma unroll
        for (int e = 0; e < VEC; ++e) deposit(u[k][e], w[k][e], Sl, ng, a1, a2);
    if (PUSH) {
#pragma unroll
        for (int k = 0; k < UNROLL; ++k) {
            const int64_t i = base + (int64_t)(k * 64 + lane) * VEC;
            store_stream<V, NT>((T *)U + i, u[k]);
            store_stream<V, NT>((T *)W + i, w[k]);
        }
    }
}

// The same stages for one particle (ragged tile ends).
template <typename T, bool PUSH>
__device__ __forceinline__ void run_one(T *U, T *W, int64_t q, const T *Et, unsigned long long *Sl,
                                        int ng, T ngf, T hi, double &a1, double &a2, uint32_t &flags) {
    T sv = U[q], wv = W[q];
    if (PUSH) push(sv, wv, gather(sv, Et, ng), ngf, hi, flags);
    deposit(sv, wv, Sl, ng, a1, a2);
    if (PUSH) {
        U[q] = sv;
        W[q] = wv;
    }
}

// All tiles [tb, te) of run R.  Tile t of a run owns the block units
// (kUnit particles each) t, t + ntiles, t + 2 ntiles, ...: the wavefronts of
// the device, each on its own tile, sweep neighbouring units together.
// Wavefronts take tiles one at a time from an LDS counter, so they finish a
// chunk together whatever the tile count.  Each lane handles UNROLL vectors
// of VEC particles per iteration, all loads issued before any compute; a
// lane's particles are accumulated in index order for every UNROLL, so the
// tile partial sums depend only on the run.  The deposits stay in the
// private grid Sl (merged by the caller); the caller has put the run's gather
// table into Et (the barrier below orders it before every gather).
template <typename T, int BLOCK, int UNROLL, bool PUSH, bool NT>
__device__ void process_chunk(RunDev *R, int tb, int te, int tstride, unsigned long long *Sl, T *Et,
                              int *next_tile) {
    using V = typename Vec<T>::type;
    constexpr int VEC = Vec<T>::n;
    constexpr int PER = 64 * VEC * UNROLL;
    constexpr int SPB = kUnit / PER;                 // sub-blocks per block unit
    static_assert(kUnit % PER == 0, "a block unit holds whole sub-blocks");
    // Register sets in the load pipeline: three at one vector per lane
    // (96 VGPRs, five waves per SIMD), two when the sub-blocks are wider
    // (a third measured no faster and spills at 1024 threads).  Four sets
    // at one vector cost a wave per SIMD and measured slower.
    constexpr int DEPTH = UNROLL == 1 ? 3 : 2;
    const int ng = R->ng;
    const int64_t np = R->np;
    const int ntiles = R->ntiles;
    T *U = (T *)R->u;
    T *W = (T *)R->w;
    double *part = R->tile_part;
    const T ngf = (T)ng;
    const T hi = ngf + T(0.5);
    if (threadIdx.x == 0) *next_tile = 0;
    __syncthreads();
    const int lane = threadIdx.x & 63;
    uint32_t flags = 0;
    const int64_t nfull = np / kUnit;                // full block units of the run
    const bool ragged = nfull * (int64_t)kUnit < np;
    for (;;) {
        int k = 0;
        if (lane == 0) k = atomicAdd(next_tile, 1);
        const int t = tb + __builtin_amdgcn_readfirstlane(k) * tstride;
        if (t >= te) break;
        double a1 = 0.0, a2 = 0.0;
        // Full units of the tile in sub-blocks of PER particles,
        // software-pipelined over DEPTH register sets: sub-block i lives in
        // set i mod DEPTH, and its loads are issued DEPTH - 1 sub-blocks
        // before it is processed and stored, so a wave has that many loads
        // in flight and never waits for its own stores.  Rounds of DEPTH
        // sub-blocks; the last round skips the loads past the tile's end
        // (a wave-uniform branch: re-reading the last sub-block instead
        // measured 1% slower on short tiles).
        const int64_t nunits = t < nfull ? (nfull - 1 - t) / ntiles + 1 : 0;
        const int64_t nb = nunits * SPB;
        auto sub = [&](int64_t q) -> int64_t {
            return ((int64_t)t + (q / SPB) * ntiles) * kUnit + (q % SPB) * PER;
        };
        V bu[DEPTH][UNROLL], bw[DEPTH][UNROLL];
        if (nb > 0) {
#pragma unroll
            for (int d = 0; d < DEPTH - 1; ++d)
                load_block<V, VEC, UNROLL, NT>(U, W, sub(min((int64_t)d, nb - 1)), lane, bu[d], bw[d]);
        }
        const int64_t nrounds = nb / DEPTH;
        for (int64_t q = 0; q < nrounds; ++q) {
#pragma unroll
            for (int d = 0; d < DEPTH; ++d) {
                const int64_t ahead = q * DEPTH + d + DEPTH - 1;
                if (ahead < nb)
                    load_block<V, VEC, UNROLL, NT>(U, W, sub(ahead), lane, bu[(d + DEPTH - 1) % DEPTH],
                                                   bw[(d + DEPTH - 1) % DEPTH]);
                run_block<T, V, VEC, UNROLL, PUSH, NT>(U, W, sub(q * DEPTH + d), lane, bu[d], bw[d], Et, Sl, ng,
                                                       ngf, hi, a1, a2, flags);
            }
        }
        const int64_t rest = nb - nrounds * DEPTH;
#pragma unroll
        for (int d = 0; d < DEPTH - 1; ++d)
            if (d < rest)
                run_block<T, V, VEC, UNROLL, PUSH, NT>(U, W, sub(nrounds * DEPTH + d), lane, bu[d], bw[d], Et, Sl,
                                                       ng, ngf, hi, a1, a2, flags);
        // The run's partial last unit belongs to tile nfull mod ntiles: same
        // per-lane order as a full unit; whole vectors where they fit, then
        // single particles.
        if (ragged && nfull % ntiles == t) {
            for (int64_t base = nfull * kUnit; base < np; base += PER) {
                for (int k = 0; k < UNROLL; ++k) {
                    const int64_t i = base + (int64_t)(k * 64 + lane) * VEC;
                    if (i + VEC <= np) {
                        V vu[1], vw[1];
                        vu[0] = load_stream<V, NT>(U + i);
                        vw[0] = load_stream<V, NT>(W + i);
                        run_block<T, V, VEC, 1, PUSH, NT>(U, W, i - (int64_t)lane * VEC, lane, vu, vw, Et, Sl, ng,
                                                          ngf, hi, a1, a2, flags);
                    } else {
                        for (int e = 0; e < VEC; ++e) {
                            const int64_t q = i + e;
                            if (q < np) run_one<T, PUSH>(U, W, q, Et, Sl, ng, ngf, hi, a1, a2, flags);
                        }
                    }
                }
            }
        }
        a1 = wave_sum(a1);
        a2 = wave_sum(a2);
        if (lane == 0) {
            f64x2 pt;
            pt.x = a1;
            pt.y = a2;
            *reinterpret_cast<f64x2 *>(part + kPartCols * (size_t)t) = pt;
        }
    }
    if (flags) atomicOr(&R->flags, flags);
    __syncthreads();
}

// Merge the private grid into the run's grid S[ng] with 64-bit atomics,
// folding the two ghost nodes, and clear it.  No fence: the solve runs in
// the next launch, after the kernel boundary has made every merge visible.
// Starting at a workgroup-dependent rotation spreads concurrent merges over
// addresses.
template <int BLOCK>
__device__ void merge_grid(unsigned long long *S, int ng, int rot_seed, unsigned long long *Sl) {
    const int rot = (int)(((unsigned)rot_seed * 97u) % (unsigned)ng);
    for (int k = threadIdx.x; k < ng; k += BLOCK) {
        int c = k + rot;
        if (c >= ng) c -= ng;
        unsigned long long v = Sl[c + 1];
        Sl[c + 1] = 0ull;
        if (c == 0) {
            v += Sl[ng + 1];
            Sl[ng + 1] = 0ull;
        }
        if (c == ng - 1) {
            v += Sl[0];
            Sl[0] = 0ull;
        }
        if (v) atomicAdd(S + c, v);
    }
    __syncthreads();
}

// Particle pass.  Single run (items == nullptr): workgroup b takes an
// even share of the run's tiles, or (order 1) every grid-th tile.  Batch:
// workgroups take work items (chunks of some run's tiles, each chunk every
// nchunks-th tile, largest first): workgroup b item b, then the next
// ones from the shared queue until it is empty (see WorkQueue).  Any
// workgroup may take any chunk: nothing a chunk computes depends on who
// computes it (per-tile partials, integer grid sums).  A workgroup merges
// its private grid when it moves to another run and when it is done, so
// chunks of one run in a row cost one table load and one merge.
template <typename T, int BLOCK, int UNROLL, bool PUSH, bool NT>
__global__ __launch_bounds__(BLOCK) void step_kernel(RunDev *runs, const WorkItem *items, WorkQueue *queue,
                                                    int ng_lds, int order, const T *table0) {
    extern __shared__ unsigned long long lds[];
    __shared__ uint32_t s_item;
    __shared__ int s_tile;
    unsigned long long *Sl = lds;
    T *Et = reinterpret_cast<T *>(lds + ng_lds + 2);
    for (int g = threadIdx.x; g < ng_lds + 2; g += BLOCK) Sl[g] = 0ull;
    const uint32_t nitems = items ? queue->nitems : 1u;
    const uint32_t grid = gridDim.x;
    int prev_run = -1;
    int table_run = -1;                               // the run whose gather table Et holds
    unsigned long long *S_pend = nullptr;             // grid of prev_run, merged when the run changes
    int ng_pend = 0, rot_pend = 0;
    for (uint32_t round = 0;; ++round) {
        uint32_t it = round;                          // single run: one chunk per workgroup
        if (items && round == 0) {
            it = blockIdx.x;                          // first item: no queue traffic
        } else if (items) {
            // No more items than workgroups: every item was a first item and
            // nothing is queued, so no workgroup draws a ticket (a returning
            // atomic on one address at every workgroup's end) and `next`
            // stays 0 for the next launch.
            if (nitems <= grid) break;
            if (threadIdx.x == 0) {
                // Tickets 0, 1, ... map to items grid, grid + 1, ...; every
                // workgroup draws exactly one ticket past the list and
                // stops, so the holder of the last ticket, nitems - 1, knows
                // that no other workgroup touches `next` again.
                const uint32_t t = atomicAdd(&queue->next, 1u);
                if (t == nitems - 1u) atomicExch(&queue->next, 0u);
                s_item = grid + t;
            }
            __syncthreads();
            it = s_item;
            __syncthreads();                          // s_item is rewritten next round
        }
        if (it >= nitems) break;
        int r = 0, tb, te, chunk, nchunks, tstride = 1, ngt;
        const T *tab;
        if (items) {
            const WorkItem wi = items[it];
            r = wi.run;
            tb = wi.tile_begin;
            te = wi.tile_end;
            chunk = wi.chunk;
            nchunks = wi.nchunks;
            ngt = wi.ng;
            tstride = wi.tstride;
            tab = (const T *)wi.table;
        } else {
            ngt = ng_lds;
            tab = table0;
            const int64_t nt = runs[0].ntiles;
            if (order) {                              // tiles b, b + grid, b + 2 grid, ...
                tb = blockIdx.x;
                te = (int)nt;
                tstride = gridDim.x;
            } else {                                  // an even share of consecutive tiles
                tb = (int)(nt * blockIdx.x / gridDim.x);
                te = (int)(nt * (blockIdx.x + 1) / gridDim.x);
            }
            chunk = blockIdx.x;
            nchunks = gridDim.x;
        }
        // The gather table's address and size come with the item (or the
        // launch), so its loads start at once, beside those of the run
        // descriptor below instead of after them.  Consecutive fills are
        // separated by the barriers of the queue (or of process_chunk).
        if (PUSH && r != table_run && ngt <= ng_lds) {
            fill_table<T, BLOCK>(tab, Et, ngt);
            table_run = r;
        }
        RunDev *R = runs + r;
        // the prologue (initial deposit) runs whatever the step target, even 0
        if (!(PUSH && R->step >= R->step_target) && R->ng <= ng_lds) {
            // deposit d = step + 1 (the prologue's: 0) goes to S01[d & 1]; this
            // chunk clears its share of the other buffer, deposit d - 1, which
            // the previous launch's solve has read
            const int dep = PUSH ? (int)((R->step + 1) & 1) : 0;
            unsigned long long *Sclr = R->S01[dep ^ 1];
            const int ngr = R->ng;
            if (te > tb) {
                if (r != prev_run) {
                    // A new run: the previous run's grid goes out first (chunks
                    // of one run in a row share the private grid and the table).
                    if (prev_run >= 0) merge_grid<BLOCK>(S_pend, ng_pend, rot_pend, Sl);
                    S_pend = R->S01[dep];
                    ng_pend = ngr;
                    rot_pend = chunk;
                }
                process_chunk<T, BLOCK, UNROLL, PUSH, NT>(R, tb, te, tstride, Sl, Et, &s_tile);
                prev_run = r;
            }
            const int g1 = (int)((int64_t)ngr * (chunk + 1) / nchunks);
            for (int g = (int)((int64_t)ngr * chunk / nchunks) + (int)threadIdx.x; g < g1; g += BLOCK)
                Sclr[g] = 0ull;
        }
    }
    if (prev_run >= 0) merge_grid<BLOCK>(S_pend, ng_pend, rot_pend, Sl);
}


// The prologue (initial deposit, no stores) always reads non-temporally.
template <typename T, int BLOCK, int UNROLL, bool PUSH>
const void *kernel_ptr(bool cached) {
    if constexpr (!PUSH) {
        (void)cached;
        return (const void *)step_kernel<T, BLOCK, UNROLL, PUSH, true>;
    } else {
        return cached ? (const void *)step_kernel<T, BLOCK, UNROLL, PUSH, false>
                      : (const void *)step_kernel<T, BLOCK, UNROLL, PUSH, true>;
    }
}

template <typename T, int BLOCK, bool PUSH>
const void *kernel_unroll(int unroll, bool cached) {
    if constexpr (!PUSH) {
        (void)unroll;
        return kernel_ptr<T, BLOCK, 1, PUSH>(cached);
    } else {
        switch (unroll) {
            case 1: return kernel_ptr<T, BLOCK, 1, PUSH>(cached);
            case 2: return kernel_ptr<T, BLOCK, 2, PUSH>(cached);
            case 4: return kernel_ptr<T, BLOCK, 4, PUSH>(cached);
            default: return nullptr;
        }
    }
}

template <typename T, bool PUSH>
const void *kernel_for(int block, int unroll, bool cached) {
    switch (block) {
        case 256: return kernel_unroll<T, 256, PUSH>(unroll, cached);
        case 512: return kernel_unroll<T, 512, PUSH>(unroll, cached);
        case 640: return kernel_unroll<T, 640, PUSH>(unroll, cached);
        case 768: return kernel_unroll<T, 768, PUSH>(unroll, cached);
        case 1024: return kernel_unroll<T, 1024, PUSH>(unroll, cached);
        default: return nullptr;
    }
}

const void *kernel_select(const LaunchShape &ls, int precision, bool push) {
    if (ls.cached != 0 && ls.cached != 1) return nullptr;
    const bool c = ls.cached != 0;
    if (precision == 0)
        return push ? kernel_for<float, true>(ls.block, ls.unroll, c) : kernel_for<float, false>(ls.block, 1, c);
    return push ? kernel_for<double, true>(ls.block, ls.unroll, c) : kernel_for<double, false>(ls.block, 1, c);
}

}  // namespace

size_t step_lds_bytes(int precision, int ng_lds) {
    return (size_t)(ng_lds + 2) *
           (sizeof(unsigned long long) + (precision ? sizeof(double) : sizeof(float)));
}

hipError_t step_prepare(const LaunchShape &ls, int precision) {
    for (int push = 0; push < 2; ++push) {
        const void *fn = kernel_select(ls, precision, push != 0);
        if (!fn) return hipErrorInvalidValue;
        hipError_t e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize,
                                           (int)step_lds_bytes(precision, kMaxNg));
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

hipError_t launch_particles(RunDev *runs, const WorkItem *items, WorkQueue *queue, const void *table, int grid,
                            const LaunchShape &ls, int ng_lds, int precision, int prologue,
                            hipStream_t stream) {
    if (grid <= 0 || ng_lds <= 0 || ng_lds > kMaxNg || (items && !queue)) return hipErrorInvalidValue;
    if (!items && !table && prologue == 0) return hipErrorInvalidValue;
    const void *fn = kernel_select(ls, precision, prologue == 0);
    if (!fn) return hipErrorInvalidValue;
    int order = ls.order;
    void *args[] = {(void *)&runs, (void *)&items, (void *)&queue, (void *)&ng_lds, (void *)&order, (void *)&table};
    return hipLaunchKernel(fn, dim3(grid), dim3(ls.block), args, step_lds_bytes(precision, ng_lds),
                           stream);
}

hipError_t launch_step(RunDev *runs, const WorkItem *items, WorkQueue *queue, const void *table, int grid,
                       const LaunchShape &ls, int ng_lds, int precision, int prologue, const int32_t *slots,
                       int nsolve, hipStream_t stream, const StepEvents *ev) {
    if (nsolve <= 0) return hipErrorInvalidValue;
    hipError_t e;
    if (ev && (e = hipEventRecord(ev->e0, stream)) != hipSuccess) return e;
    e = launch_particles(runs, items, queue, table, grid, ls, ng_lds, precision, prologue, stream);
    if (e != hipSuccess) return e;
    if (ev && (e = hipEventRecord(ev->e1, stream)) != hipSuccess) return e;
    e = launch_solve(runs, slots, nsolve, prologue, ng_lds, stream);
    if (e != hipSuccess) return e;
    if (ev) return hipEventRecord(ev->e2, stream);
    return hipSuccess;
}

int step_occupancy(const LaunchShape &ls, int ng_lds, int precision) {
    int n = 0;
    const void *fn = kernel_select(ls, precision, true);
    if (!fn) return 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, fn, ls.block,
                                                     step_lds_bytes(precision, ng_lds)) != hipSuccess)
        return 1;
    return n > 0 ? n : 1;
}

}  // namespace pic1d
