// Field solve of the PIC step (gfx950): the second launch of every step.
//
// Two workgroups per run (idle and finished runs return at once).  The
// field workgroup reads the fixed-point charge sums S the particle pass
// merged (the next step's pass clears them), solves the periodic three-point
// Poisson problem (Sec. 2.2) exactly, or with the paper's fixed-iteration CG
// when the run asks for it, forms the central-difference node field, and
// writes E^{n+1} in FP64, the gather table for the next particle pass and
// the per-wavefront sums of E^2.  The diagnostics workgroup, beside it on
// another CU, sums the per-tile partials of the particle pass and records
// the step's diagnostics.  Neither reads what the other writes in the same
// launch.  Every reduction is a fixed-order sum over the workgroup's
// threads, so the results depend only on the run.
#include "pic_internal.h"

namespace pic1d {

namespace {

typedef double f64x2 __attribute__((ext_vector_type(2)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

constexpr int kMaxSolveThreads = 1024;  // largest solve workgroup

// Threads that work on a run's solve: a function of ng alone (so results
// depend only on the run), at least 256 and enough that every thread owns
// at most 8 nodes.  A launch covering several runs uses the largest; the
// extra waves of smaller runs only take part in the barriers.
__host__ __device__ __forceinline__ int solve_threads(int ng) {
    const int t = (ng + 8 * 64 - 1) / (8 * 64) * 64;
    return t < 256 ? 256 : (t > kMaxSolveThreads ? kMaxSolveThreads : t);
}


// Block reductions.  Each one writes its wavefront totals to one of two
// alternating LDS buffers and needs a single barrier: the next reduction
// writes the other buffer, and the one after that (the same buffer again)
// runs only after every thread has passed the next reduction's barrier, so
// after every read of this one.  `par` selects the buffer and must follow
// the same sequence in every thread.
constexpr int kRedSlots = kMaxSolveThreads / 64;
constexpr int kSolvePer = 8;     // nodes per thread at most: ng <= 8 solve_threads(ng)
constexpr int kPartBatch = 8;    // tile partials per thread loaded with the nodes

// Sum over the first nthr threads in a fixed order (butterfly inside each
// wavefront, then wavefront totals in index order); every thread gets the
// value.  All threads of the block must call it.
// v of lane i - 1 (lane 0: fill) and of lane i + 1 (lane 63: fill).
__device__ __forceinline__ double lane_prev(double v, double fill) {
    const int lo = __builtin_amdgcn_update_dpp(__double2loint(fill), __double2loint(v), 0x138, 0xf, 0xf, false);
    const int hi = __builtin_amdgcn_update_dpp(__double2hiint(fill), __double2hiint(v), 0x138, 0xf, 0xf, false);
    return __hiloint2double(hi, lo);
}
__device__ __forceinline__ double lane_next(double v, double fill) {
    const int lo = __builtin_amdgcn_update_dpp(__double2loint(fill), __double2loint(v), 0x130, 0xf, 0xf, false);
    const int hi = __builtin_amdgcn_update_dpp(__double2hiint(fill), __double2hiint(v), 0x130, 0xf, 0xf, false);
    return __hiloint2double(hi, lo);
}

// The first `nw` wavefront totals of a reduction, summed in slot order.
// Slots are read four at a time (one LDS round trip per four; slots past nw
// are read but not added), then added in order.
template <typename V>
__device__ __forceinline__ V sum_slots(const V *red, int nw) {
    V s = 0;
#pragma unroll
    for (int k0 = 0; k0 < kRedSlots; k0 += 4) {
        if (k0 < nw) {
            V vals[4];
#pragma unroll
            for (int k = 0; k < 4; ++k) vals[k] = red[k0 + k];
#pragma unroll
            for (int k = 0; k < 4; ++k)
                if (k0 + k < nw) s += vals[k];
        }
    }
    return s;
}

template <typename V>
__device__ V solve_sum(V v, V *red2, int &par, int nthr) {
    V *red = red2 + kRedSlots * par;
    par ^= 1;
    v = wave_sum(v);
    if ((threadIdx.x & 63) == 0 && (int)threadIdx.x < nthr) red[threadIdx.x >> 6] = v;
    __syncthreads();
    return sum_slots(red, nthr >> 6);
}

// The exact integer sum of `ti` (INT) and the sums of `a` and `b` (AB) over
// the first nthr threads, each in the order of solve_sum, with a single
// barrier: the wavefront totals go to slots of their own (ti_red, ab_red),
// which no other reduction of the workgroup uses.  Every thread gets the
// values.
template <bool INT, bool AB>
__device__ void solve_sums(long long &ti, double &a, double &b, long long *ti_red, double *ab_red, int nthr) {
    long long wt = 0;
    double wa = 0.0, wb = 0.0;
    if constexpr (INT) wt = wave_sum(ti);
    if constexpr (AB) {
        wa = wave_sum(a);
        wb = wave_sum(b);
    }
    if ((threadIdx.x & 63) == 0 && (int)threadIdx.x < nthr) {
        if constexpr (INT) ti_red[threadIdx.x >> 6] = wt;
        if constexpr (AB) {
            ab_red[threadIdx.x >> 6] = wa;
            ab_red[kRedSlots + (threadIdx.x >> 6)] = wb;
        }
    }
    __syncthreads();
    if constexpr (INT) ti = sum_slots(ti_red, nthr >> 6);
    if constexpr (AB) {
        a = sum_slots(ab_red, nthr >> 6);
        b = sum_slots(ab_red + kRedSlots, nthr >> 6);
    }
}

// Exclusive prefix sum over the first nthr threads in index order.  Inside a
// wavefront: an inclusive scan of each row of 16 lanes by DPP row shifts
// (1, 2, 4, 8; lanes shifted in from outside the row add zero), then the
// totals of rows 0 and 2 broadcast into rows 1 and 3 and the total of
// rows 0-1 into rows 2-3 (DPP row broadcasts), then a shift by one lane.
// Then the wavefront totals (lane 63) of lower wavefronts, in order.
template <int CTRL, int ROWS>
__device__ __forceinline__ double dpp_scan_term(double v) {
    const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(v), CTRL, ROWS, 0xf, true);
    const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(v), CTRL, ROWS, 0xf, true);
    return __hiloint2double(hi, lo);
}

__device__ double solve_exclusive_scan(double v, double *red2, int &par, int nthr) {
    double *red = red2 + kRedSlots * par;
    par ^= 1;
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    double inc = v;
    inc += dpp_scan_term<0x111, 0xf>(inc);     // row_shr:1
    inc += dpp_scan_term<0x112, 0xf>(inc);     // row_shr:2
    inc += dpp_scan_term<0x114, 0xf>(inc);     // row_shr:4
    inc += dpp_scan_term<0x118, 0xf>(inc);     // row_shr:8
    inc += dpp_scan_term<0x142, 0xa>(inc);     // row_bcast:15 into rows 1 and 3
    inc += dpp_scan_term<0x143, 0xc>(inc);     // row_bcast:31 into rows 2 and 3
    double exc = lane_prev(inc, 0.0);          // wave_shr:1, lane 0 gets 0
    if (lane == 63 && (int)threadIdx.x < nthr) red[wv] = inc;
    __syncthreads();
    const double off = sum_slots(red, min(wv, nthr / 64));
    return off + exc;
}

// The descriptor fields the solve reads, loaded together at its start.  A
// field read after the solve's first global store would be a fresh memory
// round trip (the store might alias the descriptor, so the compiler cannot
// keep it in a register); taken by value here they cost one.
struct SolveView {
    const unsigned long long *S, *S_alt;   // the deposit to read (see solve_kernel), the other buffer
    float *Ehat;
    double *Ehat64, *E64;
    int64_t step, step_target;
    double dx, qfac, ecoef;
    int ng, solver, cg_iters;
};

__device__ __forceinline__ SolveView solve_view(const RunDev *R) {
    SolveView v;
    v.S = R->S01[0];
    v.S_alt = R->S01[1];
    v.Ehat = R->Ehat;
    v.Ehat64 = R->Ehat64;
    v.E64 = R->E64;
    v.step = R->step;
    v.step_target = R->step_target;
    v.dx = R->dx;
    v.qfac = R->qfac;
    v.ecoef = R->ecoef;
    v.ng = R->ng;
    v.solver = R->solver;
    v.cg_iters = R->cg_iters;
    return v;
}

// The paper's field solver (Sec. 2.2, Sec. 3.3): matrix-free conjugate
// gradient on the three-point system with the potential at node 0 held at
// zero (its row is the identity, its residual zero), started from zero and
// run for a fixed number of iterations, then the central-difference field.
// Each thread owns up to kCgPer strided nodes and keeps their potential,
// residual and A d in registers; the dot products are sums in a fixed
// order.  On entry D[g] holds S_g; on exit D[g] holds E_g.
constexpr int kCgPer = 8;   // nodes per thread: ng <= 8 solve_threads(ng)
constexpr int kCgWaveMaxNg = 64 * kCgPer;   // grids one wavefront solves alone

// One node's row of the CG system applied to d: the identity at node 0,
// d_{g-1} - 2 d_g + d_{g+1} elsewhere, with d_ng = 0 beyond the last node.
__device__ __forceinline__ double cg_row(int g, int ng, double left, double mid, double right) {
    if (g == 0) return mid;
    return left - 2.0 * mid + (g + 1 < ng ? right : 0.0);
}

// The direction update d <- beta d + r (every thread that needs a value of
// d, its own or a neighbour's, forms it with this same expression).
__device__ __forceinline__ double cg_next_d(double beta, double d, double r) { return __builtin_fma(beta, d, r); }

// The CG on one wavefront, for ng <= 512: lane l owns nodes l, l + 64, ...;
// the neighbours across the ends of a row of 64 nodes come from lanes 63
// and 0 of the adjacent rows (readlane), so no LDS or barrier is needed.
__device__ __forceinline__ void cg_paper_wave(const SolveView &V, double *D, double meanS) {
    const int ng = V.ng, lane = threadIdx.x & 63;
    const double dx = V.dx, qf = V.qfac;
    double ph[kCgPer], r[kCgPer], d[kCgPer];
    double rr = 0.0;
#pragma unroll
    for (int k = 0; k < kCgPer; ++k) {
        const int g = k * 64 + lane;
        ph[k] = 0.0;
        r[k] = (g > 0 && g < ng) ? -(qf * (D[g] - meanS)) * dx * dx : 0.0;
        d[k] = r[k];
        rr += r[k] * r[k];
    }
    rr = wave_sum(rr);
    const int rows = (ng + 63) >> 6;                   // rows of 64 nodes that hold nodes
    if (__builtin_sqrt(rr) > 1e-16) {
        const int iters = V.cg_iters;
        for (int it = 0; it < iters; ++it) {
            double z[kCgPer];
            double zd = 0.0;
#pragma unroll
            for (int k = 0; k < kCgPer; ++k) {
                z[k] = 0.0;
                if (k < rows) {                                                          // uniform
                    const int g = k * 64 + lane;
                    const double below = k > 0 ? lane_read(d[k - 1], 63) : 0.0;            // node 64 k - 1
                    const double above = k + 1 < rows ? lane_read(d[k + 1], 0) : 0.0;      // node 64 (k + 1)
                    const double left = lane_prev(d[k], below), right = lane_next(d[k], above);
                    if (g < ng) {
                        z[k] = cg_row(g, ng, left, d[k], right);
                        zd += z[k] * d[k];
                    }
                }
            }
            zd = wave_sum(zd);
            if (zd == 0.0) break;
            const double alpha = rr / zd;
            double rn = 0.0;
#pragma unroll
            for (int k = 0; k < kCgPer; ++k) {
                const int g = k * 64 + lane;
                if (g < ng) {
                    ph[k] += alpha * d[k];
                    r[k] -= alpha * z[k];
                    rn += r[k] * r[k];
                }
            }
            rn = wave_sum(rn);
            const double beta = rn / rr;
#pragma unroll
            for (int k = 0; k < kCgPer; ++k) {
                const int g = k * 64 + lane;
                if (g < ng) d[k] = cg_next_d(beta, d[k], r[k]);
            }
            rr = rn;
        }
    }
    __builtin_amdgcn_wave_barrier();
#pragma unroll
    for (int k = 0; k < kCgPer; ++k) {
        const int g = k * 64 + lane;
        if (g < ng) D[g] = ph[k];
    }
    __builtin_amdgcn_wave_barrier();
    double e[kCgPer];
#pragma unroll
    for (int k = 0; k < kCgPer; ++k) {
        const int g = k * 64 + lane;
        if (g < ng) {
            const double right = D[g + 1 < ng ? g + 1 : 0];
            const double left = D[g == 0 ? ng - 1 : g - 1];
            e[k] = -(right - left) / (2.0 * dx);
        }
    }
    __builtin_amdgcn_wave_barrier();
#pragma unroll
    for (int k = 0; k < kCgPer; ++k) {
        const int g = k * 64 + lane;
        if (g < ng) D[g] = e[k];
    }
}

// The workgroup CG (ng > 512): thread tid owns nodes tid, tid + nthr, ...
// with the potential, residual and A d in registers and the direction d in
// LDS for the stencil (three barriers per iteration: the direction update
// and the two dot products).  Keeping d in registers as well, with DPP
// shifts inside a wavefront and an LDS exchange at its ends, measured
// slower here (12-22% at ng 2048-8192) than these conflict-free LDS reads.
__device__ __forceinline__ void cg_paper(const SolveView &V, double *D, double *red, int &par, double meanS,
                                         int nthr) {
    if (V.ng <= kCgWaveMaxNg) {
        if (threadIdx.x < 64) cg_paper_wave(V, D, meanS);
        __syncthreads();                              // D: E_g, for every wavefront
        return;
    }
    const int ng = V.ng, tid = threadIdx.x;
    const bool worker = tid < nthr;
    const double dx = V.dx, qf = V.qfac;
    double ph[kCgPer], r[kCgPer], z[kCgPer];
    double rr = 0.0;
#pragma unroll
    for (int k = 0; k < kCgPer; ++k) {
        const int g = k * nthr + tid;
        ph[k] = 0.0;
        z[k] = 0.0;
        // rho_g = rho0 + (Q/dx) 2^-32 S_g = (Q/dx) 2^-32 (S_g - mean S): the
        // run is neutral, sum_g S_g = np 2^32 exactly
        r[k] = (worker && g > 0 && g < ng) ? -(qf * (D[g] - meanS)) * dx * dx : 0.0;
        rr += r[k] * r[k];
    }
#pragma unroll
    for (int k = 0; k < kCgPer; ++k) {
        const int g = k * nthr + tid;
        if (worker && g < ng) D[g] = r[k];            // d = r (own nodes only)
    }
    rr = solve_sum(rr, red, par, nthr);                          // syncs: d complete
    if (__builtin_sqrt(rr) > 1e-16) {
        const int iters = V.cg_iters;
        for (int it = 0; it < iters; ++it) {
            double zd = 0.0;
#pragma unroll
            for (int k = 0; k < kCgPer; ++k) {
                const int g = k * nthr + tid;
                if (worker && g < ng) {
                    double zk;
                    if (g == 0) {
                        zk = D[0];
                    } else {
                        const double right = g + 1 < ng ? D[g + 1] : 0.0;
                        zk = D[g - 1] - 2.0 * D[g] + right;
                    }
                    z[k] = zk;
                    zd += zk * D[g];
                }
            }
            zd = solve_sum(zd, red, par, nthr);
            if (zd == 0.0) break;
            const double alpha = rr / zd;
            double rn = 0.0;
#pragma unroll
            for (int k = 0; k < kCgPer; ++k) {
                const int g = k * nthr + tid;
                if (worker && g < ng) {
                    ph[k] += alpha * D[g];
                    r[k] -= alpha * z[k];
                    rn += r[k] * r[k];
                }
            }
            rn = solve_sum(rn, red, par, nthr);                  // also: every read of d is done
            const double beta = rn / rr;
#pragma unroll
            for (int k = 0; k < kCgPer; ++k) {
                const int g = k * nthr + tid;
                if (worker && g < ng) D[g] = beta * D[g] + r[k];
            }
            __syncthreads();
            rr = rn;
        }
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < kCgPer; ++k) {
        const int g = k * nthr + tid;
        if (worker && g < ng) D[g] = ph[k];
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < kCgPer; ++k) {
        const int g = k * nthr + tid;
        if (worker && g < ng) {
            const double right = D[g + 1 < ng ? g + 1 : 0];
            const double left = D[g == 0 ? ng - 1 : g - 1];
            z[k] = -(right - left) / (2.0 * dx);
        }
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < kCgPer; ++k) {
        const int g = k * nthr + tid;
        if (worker && g < ng) D[g] = z[k];
    }
    __syncthreads();
}

// Periodic Poisson solve of one run by one workgroup (Sec. 2.2), computed by
// its first solve_threads(ng) threads whatever the block size.
// The face field F_{g+1/2} = -(phi_{g+1} - phi_g)/dx satisfies
// F_{g+1/2} - F_{g-1/2} = (rho_g - mean rho) dx, so it is a prefix sum;
// periodicity of phi sets sum_g F_{g+1/2} = 0; the central-difference node
// field is E_g = (F_{g-1/2} + F_{g+1/2}) / 2.  D: LDS scratch of
// kSolveLds doubles.  The exact solve runs a serial prefix sum over each
// thread's contiguous segment of nodes, so it stores node g at dpad(g) (one
// spare slot after every 8 nodes): the threads of a wavefront then hit
// distinct LDS banks instead of a few.  The CG indexes D by node.
constexpr int kSolveLds = kMaxNg + kMaxNg / 8;
__device__ __forceinline__ int dpad(int g) { return g + (g >> 3); }

__device__ __forceinline__ void solve_field(RunDev *R, const SolveView &V, double *D, double *red, long long *redi,
                                            double *red3, bool prologue) {
    const int ng = V.ng;
    const int tid = threadIdx.x;
    const int nthr = solve_threads(ng);
    const bool worker = tid < nthr;
    int par = 0;                                   // reduction buffers (see solve_sum)
    const unsigned long long *S = V.S;
    const bool cg = V.solver == 1;
    // Plain loads: this runs in the launch after the deposit, so the kernel
    // boundary orders them after every workgroup's merge into S.  Every
    // thread owns at most kSolvePer nodes (g = tid + k nthr, see
    // solve_threads), and the loads of all of them are issued before any is
    // used: one memory round trip for the solve's input.  The sum keeps the
    // strided order g = tid, tid + nthr, ...
    unsigned long long sv[kSolvePer];
#pragma unroll
    for (int k = 0; k < kSolvePer; ++k) {
        const int g = tid + k * nthr;
        sv[k] = worker && g < ng ? S[g] : 0ull;
    }
    long long tot = 0;
#pragma unroll
    for (int k = 0; k < kSolvePer; ++k) {
        const int g = tid + k * nthr;
        if (worker && g < ng) {
            tot += (long long)sv[k];
            D[cg ? g : dpad(g)] = (double)sv[k];
        }
    }
    // exact sum_g S_g (and the barrier after which D holds every S_g)
    double unused_a = 0.0, unused_b = 0.0;
    solve_sums<true, false>(tot, unused_a, unused_b, redi, red3, nthr);
    const double meanS = (double)tot / (double)ng;
    const double ecoef = V.ecoef;
    float *Ehat = V.Ehat;
    double *Ehat64 = V.Ehat64;
    double *E64 = V.E64;
    double we = 0.0;
    if (cg) {
        __syncthreads();                          // D holds every S_g
        cg_paper(V, D, red, par, meanS, nthr);               // D: E_g
        if (worker) {
            for (int g = tid; g < ng; g += nthr) {
                const double E = D[g];
                E64[g] = E;
                const double eh = E * ecoef;
                Ehat[g] = (float)eh;
                if (Ehat64) Ehat64[g] = eh;
                we += E * E;
            }
        }
    } else {
        // Each thread owns the contiguous nodes [g0, g1) (at most kSolvePer):
        // their S_g are read from LDS at once, the face values are formed in
        // registers, and only the segment's last one goes back to LDS (slot
        // g1 - 1), where the next thread's first node finds its left face.
        const double scale = V.qfac * V.dx;       // face-field change per unit of S
        const int seg = (ng + nthr - 1) / nthr;
        const int g0 = worker ? min(tid * seg, ng) : ng, g1 = min(g0 + seg, ng);
        const int n = g1 - g0;
        double f[kSolvePer];
#pragma unroll
        for (int j = 0; j < kSolvePer; ++j) f[j] = j < n ? D[dpad(g0 + j)] : 0.0;
        double acc = 0.0;
#pragma unroll
        for (int j = 0; j < kSolvePer; ++j) {
            if (j < n) {
                acc += (f[j] - meanS) * scale;
                f[j] = acc;
            }
        }
        const double off = solve_exclusive_scan(acc, red, par, nthr);
        double csum = 0.0;
#pragma unroll
        for (int j = 0; j < kSolvePer; ++j) {
            if (j < n) {
                f[j] += off;
                csum += f[j];
            }
        }
        // every thread read its segment before the scan's barrier
        if (n > 0) D[dpad(g1 - 1)] = f[n - 1];
        const double C = -solve_sum(csum, red, par, nthr) / (double)ng;   // syncs: last faces in D
        if (n > 0) {
            double left = D[dpad(g0 == 0 ? ng - 1 : g0 - 1)];
            double e[kSolvePer];
#pragma unroll
            for (int j = 0; j < kSolvePer; ++j) {
                e[j] = 0.5 * (left + f[j]) + C;
                left = f[j];
            }
            if (n == kSolvePer) {
                // a full segment: 16-byte stores (g0 is a multiple of 8)
#pragma unroll
                for (int j = 0; j < kSolvePer; j += 2) {
                    f64x2 ev, hv;
                    ev.x = e[j];
                    ev.y = e[j + 1];
                    hv.x = e[j] * ecoef;
                    hv.y = e[j + 1] * ecoef;
                    *reinterpret_cast<f64x2 *>(E64 + g0 + j) = ev;
                    if (Ehat64) *reinterpret_cast<f64x2 *>(Ehat64 + g0 + j) = hv;
                }
#pragma unroll
                for (int j = 0; j < kSolvePer; j += 4) {
                    f32x4 tv;
                    tv.x = (float)(e[j] * ecoef);
                    tv.y = (float)(e[j + 1] * ecoef);
                    tv.z = (float)(e[j + 2] * ecoef);
                    tv.w = (float)(e[j + 3] * ecoef);
                    *reinterpret_cast<f32x4 *>(Ehat + g0 + j) = tv;
                }
            } else {
#pragma unroll
                for (int j = 0; j < kSolvePer; ++j) {
                    if (j < n) {
                        E64[g0 + j] = e[j];
                        const double eh = e[j] * ecoef;
                        Ehat[g0 + j] = (float)eh;
                        if (Ehat64) Ehat64[g0 + j] = eh;
                    }
                }
            }
#pragma unroll
            for (int j = 0; j < kSolvePer; ++j)
                if (j < n) we += e[j] * e[j];
        }
    }
    // W_E of this field, E^m (m = 0 for the prologue, else step + 1), as one
    // sum per wavefront: the reader (the next step's diagnostics workgroup,
    // or the host) adds them in wavefront order, no barrier here
    const double wsum = wave_sum(we);
    const int m_par = prologue ? 0 : (int)((V.step + 1) & 1);
    if ((tid & 63) == 0 && worker) R->field_part[m_par][tid >> 6] = wsum;
    if (tid == 0) {
        if (!prologue) R->step = V.step + 1;
        R->charge_now = (int64_t)tot;
    }
}

// The diagnostics of a step from the per-tile partial sums of the particle
// pass (sum of w^2 and of w per tile, in tile order t = tid, tid + nthr, ...)
// and the field energy the previous field solve left: the history row of
// step n (KE^n time-centred, W_E^n of the gathered field, P^{n+1/2},
// K^{n+1/2}) and the run's current kinetic energy and momentum.
__device__ __forceinline__ void solve_diag(RunDev *R, long long *redi, double *red3, bool prologue) {
    const int64_t n = R->diag_step;
    if (!prologue && n >= R->step_target) return;
    const int ng = R->ng;
    const int tid = threadIdx.x;
    const int nthr = solve_threads(ng);
    const bool worker = tid < nthr;
    const double *part = R->tile_part;
    const int ntiles = R->ntiles;
    double a1 = 0.0, a2 = 0.0;
    if (worker) {
        for (int t0 = tid; t0 < ntiles; t0 += nthr * kPartBatch) {
            f64x2 pv[kPartBatch];
#pragma unroll
            for (int k = 0; k < kPartBatch; ++k) {
                const int t = t0 + k * nthr;
                pv[k] = t < ntiles ? *reinterpret_cast<const f64x2 *>(part + kPartCols * t) : f64x2{0.0, 0.0};
            }
#pragma unroll
            for (int k = 0; k < kPartBatch; ++k) {
                a1 += pv[k].x;
                a2 += pv[k].y;
            }
        }
    }
    long long unused = 0;
    solve_sums<false, true>(unused, a1, a2, redi, red3, nthr);
    if (tid == 0) {
        const double kc = R->kcoef, pc = R->pcoef;
        const double k_new = kc * a1;
        if (!prologue) {
            if (n < R->hist_cap) {
                // W_E^n: the sums of the solve that produced E^n, in order
                const double *fp = R->field_part[n & 1];
                double w = 0.0;
                for (int k = 0; k < kFieldParts; ++k) w += fp[k];
                double *row = R->hist + (size_t)kHistCols * (size_t)n;
                row[0] = 0.5 * (R->kinetic_now + k_new);   // KE^n, time-centred
                row[1] = 0.5 * R->dx * w;                  // W_E^n of the gathered field
                row[2] = pc * a2;                          // P^{n+1/2}
                row[3] = k_new;                            // K^{n+1/2}
            }
            R->diag_step = n + 1;
        }
        R->kinetic_now = k_new;
        R->momentum_now = pc * a2;
    }
}

// Second launch of a step: workgroups 2b and 2b + 1 handle run
// runs[slots[b]] (slots null: runs[b]), the first solving for E^{n+1}, the
// second recording the diagnostics; a slot of -1 and runs that are idle or
// finished return at once.
__global__ __launch_bounds__(kMaxSolveThreads) void solve_kernel(RunDev *runs, const int32_t *slots, int prologue) {
    __shared__ double D[kSolveLds];
    __shared__ double red[2 * kRedSlots];
    __shared__ long long redi[kRedSlots];
    __shared__ double red3[2 * kRedSlots];
    const int b = (int)(blockIdx.x >> 1);
    const int slot = slots ? slots[b] : b;
    if (slot < 0) return;
    RunDev *R = runs + slot;
    if (blockIdx.x & 1) {
        solve_diag(R, redi, red3, prologue != 0);
        return;
    }
    SolveView V = solve_view(R);
    if (!prologue && V.step >= V.step_target) return;
    // this launch's deposit d (0 for the prologue, step + 1 otherwise) is in
    // S01[d & 1] (selected here: a select inside solve_run costs scratch)
    if (!prologue && ((V.step + 1) & 1)) V.S = V.S_alt;
    solve_field(R, V, D, red, redi, red3, prologue != 0);
}

}  // namespace

hipError_t launch_solve(RunDev *runs, const int32_t *slots, int nsolve, int prologue, int ng_max,
                        hipStream_t stream) {
    if (nsolve <= 0 || ng_max < 2 || ng_max > kMaxNg) return hipErrorInvalidValue;
    void *args[] = {(void *)&runs, (void *)&slots, (void *)&prologue};
    return hipLaunchKernel((const void *)solve_kernel, dim3(2 * nsolve), dim3(solve_threads(ng_max)), args, 0,
                           stream);
}

}  // namespace pic1d
