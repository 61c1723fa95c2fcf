// Device kernels of the 1D electrostatic PIC step (gfx950).
//
// One launch of step_kernel advances every scheduled run by one step:
//   gather E^n (Sec. 2.3) -> kick (Sec. 2.1) -> drift + periodic wrap
//   (Sec. 2.1) -> exact fixed-point charge deposit (Sec. 2.3) into a
//   workgroup-private int64 grid in LDS -> merge into the run's global grid
//   with 64-bit atomics -> the last workgroup to finish a run solves the
//   periodic Poisson problem and forms the central-difference field
//   (Sec. 2.2) in FP64, writing E^{n+1} and the step's diagnostics.
//
// Particles are independent within a step, so they are sharded by index
// (tiles of `tile` particles, one tile per wavefront at a time) instead of by
// domain; the grid reduction replaces the paper's ghost-cell exchange and the
// solve replaces its distributed CG.  All per-run reductions use fixed
// orders that depend only on the run's (np, ng, tile), never on the launch
// shape, so a run gives identical results alone or batched with others.
#include "pic_internal.h"

namespace pic1d {

namespace {

#define GLOBAL_AS __attribute__((address_space(1)))

typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef double f64x2 __attribute__((ext_vector_type(2)));

template <typename T> struct Vec;
template <> struct Vec<float> { using type = f32x4; static constexpr int n = 4; };
template <> struct Vec<double> { using type = f64x2; static constexpr int n = 2; };

// Streaming accesses to particle arrays: global address space, non-temporal
// (each particle is touched once per step).
template <typename V>
__device__ __forceinline__ V load_stream(const void *p) {
    return __builtin_nontemporal_load((const GLOBAL_AS V *)p);
}
template <typename V>
__device__ __forceinline__ void store_stream(void *p, V v) {
    __builtin_nontemporal_store(v, (GLOBAL_AS V *)p);
}

template <typename T>
__device__ __forceinline__ T fma_t(T a, T b, T c);
template <> __device__ __forceinline__ float fma_t<float>(float a, float b, float c) {
    return __builtin_fmaf(a, b, c);
}
template <> __device__ __forceinline__ double fma_t<double>(double a, double b, double c) {
    return __builtin_fma(a, b, c);
}

// Fixed-point index of a position u = x/dx (the exact deposit rule): with
// U = floor(u 2^32) and U' = U - 2^31 (the half-cell shift from cell edges to
// nodes at (g + 1/2) dx), the left node is j = floor(U' / 2^32) and the
// 32-bit fraction is F = U' - j 2^32.  Evaluated without 64-bit integers:
//   u >= 1/2: t = u - 1/2 is exact (1/2 is a multiple of ulp(u)), so is
//             t - floor(t), and F = (t - floor(t)) 2^32 truncated;
//   u <  1/2: j = -1 and F = floor(u 2^32) + 2^31 (u 2^32 is exact).
// Also returns the gather weight f of node j+1 (= F 2^-32 up to rounding).
// j is clamped to [-1, ng-1] so that a corrupt position cannot index outside
// the grid.
template <typename T>
__device__ __forceinline__ void fixed_index(T u, int ng, int &j, uint32_t &F, T &f) {
    const T t = u - T(0.5);
    const T jf = __builtin_floor(t);
    const T fr = t - jf;
    const bool upper = u >= T(0.5);
    const uint32_t F_hi = (uint32_t)(fr * T(4294967296.0));
    const uint32_t F_lo = (uint32_t)(u * T(4294967296.0)) + 0x80000000u;
    F = upper ? F_hi : F_lo;
    j = upper ? min((int)jf, ng - 1) : -1;
    f = upper ? fr : u + T(0.5);
}

template <typename T> __device__ __forceinline__ const T *gather_table(const RunDev *R);
template <> __device__ __forceinline__ const float *gather_table<float>(const RunDev *R) {
    return R->Ehat;
}
template <> __device__ __forceinline__ const double *gather_table<double>(const RunDev *R) {
    return R->Ehat64;
}

template <typename T>
__device__ __forceinline__ bool inside(T u, T ngf) { return u >= T(0) && u < ngf; }

// One particle through gather, kick, drift, wrap and deposit.
// Es: gather table in LDS (E scaled to the change of w per step).
// Sl: workgroup-private int64 grid in LDS.
// a0, a1, a2: running sums of w_old^2, w_new^2, w_new for the diagnostics.
template <typename T, bool PUSH>
__device__ __forceinline__ void particle(T &u, T &w, const T *Es, unsigned long long *Sl, int ng,
                                         T ngf, double &a0, double &a1, double &a2,
                                         uint32_t &flags) {
    int j;
    uint32_t F;
    T f;
    if (PUSH) {
        fixed_index(u, ng, j, F, f);
        const int jl = j < 0 ? ng - 1 : j;
        const int jr = j + 1 >= ng ? 0 : j + 1;
        const T El = Es[jl];
        const T Ep = fma_t<T>(f, Es[jr] - El, El);    // (1-f) E_j + f E_{j+1}
        const double wo = (double)w;
        a0 = __builtin_fma(wo, wo, a0);
        w = w + Ep;                                   // v^{n+1/2} = v^{n-1/2} + qm E dt
        T un = u + w;                                 // x^{n+1} = x^n + v^{n+1/2} dt
        un = un + (un < T(0) ? ngf : (un >= ngf ? -ngf : T(0)));
        if (!inside(un, ngf)) {                       // rare: rounding to ng, |w| >= ng, NaN
            if (un == ngf) {
                un = T(0);
            } else if (!__builtin_isfinite(un)) {
                un = T(0);
                flags |= 1u;
            } else {
                un = un - ngf * __builtin_floor(un / ngf);
                if (!inside(un, ngf)) un = T(0);
                flags |= 2u;
            }
        }
        u = un;
    }
    const double wn = (double)w;
    a1 = __builtin_fma(wn, wn, a1);
    a2 += wn;
    fixed_index(u, ng, j, F, f);
    const int jl = j < 0 ? ng - 1 : j;
    const int jr = j + 1 >= ng ? 0 : j + 1;
    atomicAdd(&Sl[jl], (1ull << 32) - (unsigned long long)F);
    atomicAdd(&Sl[jr], (unsigned long long)F);
}

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
    return v;
}

__device__ __forceinline__ long long wave_sum(long long v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
    return v;
}

// Block-wide sums in a fixed order (butterfly inside each wavefront, then the
// wavefront totals in index order); every thread gets the same value.
template <int BLOCK, typename V>
__device__ V block_sum(V v, V *red) {
    v = wave_sum(v);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
    __syncthreads();
    V s = 0;
    for (int k = 0; k < BLOCK / 64; ++k) s += red[k];
    __syncthreads();
    return s;
}

// Exclusive prefix sum over threads in index order.
template <int BLOCK>
__device__ double block_exclusive_scan(double v, double *red) {
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    double inc = v;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        double t = __shfl_up(inc, o);
        if (lane >= o) inc += t;
    }
    double exc = __shfl_up(inc, 1);
    if (lane == 0) exc = 0.0;
    if (lane == 63) red[wv] = inc;
    __syncthreads();
    double off = 0.0;
    for (int k = 0; k < wv; ++k) off += red[k];
    __syncthreads();
    return off + exc;
}

// Periodic Poisson solve of one run by one workgroup (Sec. 2.2).
// The face field F_{g+1/2} = -(phi_{g+1} - phi_g)/dx satisfies
// F_{g+1/2} - F_{g-1/2} = (rho_g - mean rho) dx, so it is a prefix sum;
// periodicity of phi sets sum_g F_{g+1/2} = 0; the central-difference node
// field is E_g = (F_{g-1/2} + F_{g+1/2}) / 2.  D: LDS scratch of ng doubles
// (all zero on entry and on return).
template <int BLOCK>
__device__ __noinline__ void solve_run(RunDev *R, double *D, double *red, long long *redi,
                                       bool prologue) {
    const int ng = R->ng;
    const int tid = threadIdx.x;
    unsigned long long *S = R->S;
    unsigned long long *S_last = R->S_last;
    long long tot = 0;
    for (int g = tid; g < ng; g += BLOCK) {
        unsigned long long s = __hip_atomic_load(S + g, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        S[g] = 0ull;
        S_last[g] = s;
        tot += (long long)s;
        D[g] = (double)s;
    }
    tot = block_sum<BLOCK>(tot, redi);           // exact: sum_g S_g
    const double meanS = (double)tot / (double)ng;
    const double scale = R->qfac * R->dx;        // face-field change per unit of S
    const int seg = (ng + BLOCK - 1) / BLOCK;
    const int g0 = min(tid * seg, ng), g1 = min(g0 + seg, ng);
    double acc = 0.0;
    for (int g = g0; g < g1; ++g) {
        acc += (D[g] - meanS) * scale;
        D[g] = acc;
    }
    const double off = block_exclusive_scan<BLOCK>(acc, red);
    double csum = 0.0;
    for (int g = g0; g < g1; ++g) {
        double fv = D[g] + off;
        D[g] = fv;
        csum += fv;
    }
    const double C = -block_sum<BLOCK>(csum, red) / (double)ng;   // syncs: D complete
    const double ecoef = R->ecoef;
    float *Ehat = R->Ehat;
    double *Ehat64 = R->Ehat64;
    double *E64 = R->E64;
    double we = 0.0;
    for (int g = tid; g < ng; g += BLOCK) {
        double left = D[g == 0 ? ng - 1 : g - 1];
        double E = 0.5 * (left + D[g]) + C;
        E64[g] = E;
        double eh = E * ecoef;
        Ehat[g] = (float)eh;
        if (Ehat64) Ehat64[g] = eh;
        we += E * E;
    }
    we = 0.5 * R->dx * block_sum<BLOCK>(we, red);
    double a0 = 0.0, a1 = 0.0, a2 = 0.0;
    const double *part = R->tile_part;
    const int ntiles = R->ntiles;
    for (int t = tid; t < ntiles; t += BLOCK) {
        a0 += __hip_atomic_load(part + kPartCols * t + 0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        a1 += __hip_atomic_load(part + kPartCols * t + 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        a2 += __hip_atomic_load(part + kPartCols * t + 2, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    a0 = block_sum<BLOCK>(a0, red);
    a1 = block_sum<BLOCK>(a1, red);
    a2 = block_sum<BLOCK>(a2, red);
    if (tid == 0) {
        const double kc = R->kcoef, pc = R->pcoef;
        if (!prologue) {
            const int64_t n = R->step;
            if (n < R->hist_cap) {
                double *row = R->hist + (size_t)kHistCols * (size_t)n;
                row[0] = 0.5 * kc * (a0 + a1);   // KE^n, time-centred
                row[1] = R->field_now;           // W_E^n of the field this step gathered
                row[2] = pc * a2;                // P^{n+1/2}
                row[3] = kc * a1;                // K^{n+1/2}
            }
            R->step = n + 1;
        }
        R->kinetic_now = kc * a1;
        R->momentum_now = pc * a2;
        R->field_now = we;
        R->charge_now = (int64_t)tot;
        R->counter = 0u;
    }
    for (int g = tid; g < ng; g += BLOCK) D[g] = 0.0;
    __syncthreads();
}

// All tiles [tb, te) of run R: wavefront k of the block takes tiles
// tb + k, tb + k + nwaves, ...; each lane streams VEC particles per
// iteration, with the next iteration's loads issued before the current
// particles are processed.
template <typename T, int BLOCK, bool PUSH>
__device__ void process_chunk(RunDev *R, int tb, int te, bool load_table, unsigned long long *Sl,
                              T *Es, double *red, long long *redi, int *s_last) {
    using V = typename Vec<T>::type;
    constexpr int VEC = Vec<T>::n;
    constexpr int STRIDE = 64 * VEC;
    const int ng = R->ng;
    const int64_t np = R->np;
    const int tile = R->tile;
    T *U = (T *)R->u;
    T *W = (T *)R->w;
    double *part = R->tile_part;
    const T ngf = (T)ng;
    if (PUSH && load_table) {
        const T *tab = gather_table<T>(R);
        for (int g = threadIdx.x; g < ng; g += BLOCK) Es[g] = tab[g];
    }
    __syncthreads();
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    uint32_t flags = 0;
    for (int t = tb + wave; t < te; t += BLOCK / 64) {
        const int64_t p0 = (int64_t)t * tile;
        const int64_t p1 = min(p0 + (int64_t)tile, np);
        double a0 = 0.0, a1 = 0.0, a2 = 0.0;
        int64_t i = p0 + (int64_t)lane * VEC;
        V un, wn;
        if (i + VEC <= p1) {
            un = load_stream<V>(U + i);
            wn = load_stream<V>(W + i);
        }
        for (; i < p1; i += STRIDE) {
            if (i + VEC <= p1) {
                V uu = un, ww = wn;
                const int64_t inext = i + STRIDE;
                if (inext + VEC <= p1) {
                    un = load_stream<V>(U + inext);
                    wn = load_stream<V>(W + inext);
                }
#pragma unroll
                for (int k = 0; k < VEC; ++k) {
                    T uk = uu[k], wk = ww[k];
                    particle<T, PUSH>(uk, wk, Es, Sl, ng, ngf, a0, a1, a2, flags);
                    uu[k] = uk;
                    ww[k] = wk;
                }
                if (PUSH) {
                    store_stream<V>(U + i, uu);
                    store_stream<V>(W + i, ww);
                }
            } else {
                for (int64_t q = i; q < p1; ++q) {
                    T uu = U[q], ww = W[q];
                    particle<T, PUSH>(uu, ww, Es, Sl, ng, ngf, a0, a1, a2, flags);
                    if (PUSH) {
                        U[q] = uu;
                        W[q] = ww;
                    }
                }
            }
        }
        a0 = wave_sum(a0);
        a1 = wave_sum(a1);
        a2 = wave_sum(a2);
        if (lane == 0) {
            double *pp = part + (size_t)kPartCols * (size_t)t;
            pp[0] = a0;
            pp[1] = a1;
            pp[2] = a2;
        }
    }
    if (flags) atomicOr(&R->flags, flags);
    __syncthreads();
    // Merge the private grid into the run's grid.  Start at a block-dependent
    // rotation so that concurrent flushes hit different addresses.
    unsigned long long *S = R->S;
    const int rot = (int)(((unsigned)blockIdx.x * 97u) % (unsigned)ng);
    for (int k = threadIdx.x; k < ng; k += BLOCK) {
        int g = k + rot;
        if (g >= ng) g -= ng;
        const unsigned long long v = Sl[g];
        if (v) {
            atomicAdd(S + g, v);
            Sl[g] = 0ull;
        }
    }
    __threadfence();
    __syncthreads();
    if (threadIdx.x == 0) {
        const uint32_t n = (uint32_t)(te - tb);
        const uint32_t prev = atomicAdd(&R->counter, n);
        *s_last = (prev + n == (uint32_t)R->ntiles) ? 1 : 0;
    }
    __syncthreads();
    if (*s_last) {
        __threadfence();
        solve_run<BLOCK>(R, reinterpret_cast<double *>(Sl), red, redi, !PUSH);
    }
}

template <typename T, int BLOCK, bool PUSH>
__global__ __launch_bounds__(BLOCK, 6) void step_kernel(RunDev *runs, const WorkItem *items,
                                                        const int32_t *wg_begin, int ng_lds) {
    extern __shared__ unsigned long long lds[];
    __shared__ double red[BLOCK / 64];
    __shared__ long long redi[BLOCK / 64];
    __shared__ int s_last;
    unsigned long long *Sl = lds;
    T *Es = reinterpret_cast<T *>(lds + ng_lds);
    for (int g = threadIdx.x; g < ng_lds; g += BLOCK) Sl[g] = 0ull;
    int ib = 0, ie = 1;
    if (items) {
        ib = wg_begin[blockIdx.x];
        ie = wg_begin[blockIdx.x + 1];
    }
    int prev_run = -1;
    for (int it = ib; it < ie; ++it) {
        int r, tb, te;
        if (items) {
            const WorkItem wi = items[it];
            r = wi.run;
            tb = wi.tile_begin;
            te = wi.tile_end;
        } else {
            r = 0;
            const int64_t nt = runs[0].ntiles;
            tb = (int)(nt * blockIdx.x / gridDim.x);
            te = (int)(nt * (blockIdx.x + 1) / gridDim.x);
        }
        RunDev *R = runs + r;
        if (te <= tb || R->step >= R->step_target || R->ng > ng_lds) continue;
        process_chunk<T, BLOCK, PUSH>(R, tb, te, r != prev_run, Sl, Es, red, redi, &s_last);
        prev_run = r;
    }
}

template <typename T, int BLOCK, bool PUSH>
const void *kernel_ptr() {
    return (const void *)step_kernel<T, BLOCK, PUSH>;
}

template <typename T, bool PUSH>
const void *kernel_for(int block) {
    switch (block) {
        case 256: return kernel_ptr<T, 256, PUSH>();
        case 512: return kernel_ptr<T, 512, PUSH>();
        case 1024: return kernel_ptr<T, 1024, PUSH>();
        default: return nullptr;
    }
}

const void *kernel_select(int block, int precision, bool push) {
    if (precision == 0) return push ? kernel_for<float, true>(block) : kernel_for<float, false>(block);
    return push ? kernel_for<double, true>(block) : kernel_for<double, false>(block);
}

}  // namespace

size_t step_lds_bytes(int precision, int ng_lds) {
    return (size_t)ng_lds * (sizeof(unsigned long long) + (precision ? sizeof(double) : sizeof(float)));
}

hipError_t step_prepare(int block, int precision) {
    for (int push = 0; push < 2; ++push) {
        const void *fn = kernel_select(block, precision, push != 0);
        if (!fn) return hipErrorInvalidValue;
        hipError_t e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize,
                                           (int)step_lds_bytes(precision, kMaxNg));
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

hipError_t launch_step(RunDev *runs, const WorkItem *items, const int32_t *wg_begin, int grid,
                       int block, int ng_lds, int precision, int prologue, hipStream_t stream) {
    if (grid <= 0 || ng_lds <= 0 || ng_lds > kMaxNg) return hipErrorInvalidValue;
    const void *fn = kernel_select(block, precision, prologue == 0);
    if (!fn) return hipErrorInvalidValue;
    void *args[] = {(void *)&runs, (void *)&items, (void *)&wg_begin, (void *)&ng_lds};
    return hipLaunchKernel(fn, dim3(grid), dim3(block), args, step_lds_bytes(precision, ng_lds),
                           stream);
}

int step_occupancy(int block, int ng_lds, int precision) {
    int n = 0;
    const void *fn = kernel_select(block, precision, true);
    if (!fn) return 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, fn, block,
                                                     step_lds_bytes(precision, ng_lds)) != hipSuccess)
        return 1;
    return n > 0 ? n : 1;
}

}  // namespace pic1d
