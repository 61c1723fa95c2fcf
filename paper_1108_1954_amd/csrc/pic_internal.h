// Internal declarations shared by the device kernels (pic_kernels.hip) and
// the host runtime (pic_runtime.hip).  Not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <functional>
#include <string>

namespace pic1d {

constexpr int kMaxNg = 8192;
constexpr int kHistCols = 4;
constexpr int kPartCols = 2;     // per tile: sum w_new^2, sum w_new
constexpr int kWave = 64;
constexpr int kFieldParts = 16;  // wavefronts of the largest field-solve workgroup (1024 threads)

// Device-resident descriptor of one run.  Lives in device memory; the
// kernels update step/counter/flags and the "now" diagnostics.
struct RunDev {
    void *u, *w;                 // state: s = x/dx + 1/2 in [1/2, ng + 1/2), w = v dt/dx
    void *u_alt, *w_alt;         // cell-sort destination (ping-pong), may be null
    // [ng] fixed-point charge sums, two buffers: deposit d (d = 0 at
    // creation, n + 1 in step n) goes to S01[d & 1]; the pass of step n clears
    // S01[n & 1] (deposit n, consumed by the previous solve), so after N steps
    // S01[N & 1] holds the latest deposit and S01[(N + 1) & 1] is zero.
    unsigned long long *S01[2];
    float *Ehat;                 // [ng] gather table  E qm dt^2 / dx   (FP32)
    double *Ehat64;              // [ng] same table in FP64 (FP64 state), may be null
    double *E64;                 // [ng] node field (FP64)
    double *tile_part;           // [ntiles][kPartCols]
    double *hist;                // [hist_cap][kHistCols]
    void *sort_scratch;          // cell-sort count table and block sums, may be null
    int64_t np;
    int64_t hist_cap;
    int64_t step;                // steps completed (field solves; read by the particle pass)
    int64_t diag_step;           // steps whose diagnostics are recorded (equals step between launches)
    int64_t step_target;         // no further steps once step == step_target
    int32_t ng;
    int32_t tile;                // particles per tile (multiple of kUnit)
    int32_t ntiles;
    int32_t precision;           // 0 = FP32 state, 1 = FP64 state
    int32_t solver;              // 0 = exact prefix-sum solve, 1 = the paper's CG
    uint32_t flags;              // PIC_FLAG_* bits
    double dx;
    double qfac;                 // Q / (dx 2^32): density per unit of S
    double ecoef;                // qm dt^2 / dx: E -> change of w per step
    double kcoef;                // (m/2) (dx/dt)^2: sum w^2 -> kinetic energy
    double pcoef;                // m dx/dt: sum w -> momentum
    // W_E of the field E^m is dx/2 times the sum, in index order, of
    // field_part[m & 1][0 .. kFieldParts) (one entry per wavefront of the
    // field solve, zero beyond its wavefronts), written by the solve that
    // produces E^m
    double field_part[2][kFieldParts];
    double kinetic_now;          // (m/2) sum v^2 of the current velocities
    double momentum_now;
    int64_t charge_now;          // sum_g S_g of the current positions
    int32_t sort_swap;           // 1 when the sorted copy lives in u_alt/w_alt
    int32_t cg_iters;            // CG iterations (solver 1)
};

// One unit of schedule: tiles tile_begin, tile_begin + tstride, ... below
// tile_end of run `run`, which is chunk `chunk` of the run's `nchunks`
// chunks in this launch; `ng` and `table` repeat the run's grid size and
// gather-table address (fixed for the run's life) so the pass can load the
// table without the run descriptor.
struct WorkItem {
    int32_t run;
    int32_t tile_begin;
    int32_t tile_end;
    int32_t chunk;
    int32_t nchunks;
    int32_t ng;
    int32_t tstride;
    int32_t pad_;
    const void *table;
};

// Work queue of a batched particle pass (device memory): workgroup b takes
// item b first, then items grid, grid + 1, ... in list order through the
// ticket counter `next`; the workgroup that draws the launch's last ticket
// resets it to 0 for the next launch.  With nitems <= grid nothing is queued
// and no workgroup draws (`next` stays 0).
struct WorkQueue {
    uint32_t next;
    uint32_t nitems;
    uint32_t pad_[2];
};

// Particles per block unit: tile t of a run owns units t, t + ntiles, ...
// Tiles are whole units.
constexpr int kUnit = 1024;

// Launch shape of the step kernel (chosen per run by the autotuner):
// threads per workgroup, particle vectors per lane per iteration, the tile
// order of single runs and the cache policy of the particle accesses.
struct LaunchShape {
    int block = 512;
    int unroll = 2;
    // Single runs: 0 gives workgroup b the contiguous tiles
    // [ntiles b / grid, ntiles (b + 1) / grid), 1 the tiles b, b + grid, ...
    // (the device's wavefronts then work on neighbouring tiles spread over all
    // CUs, which HBM serves faster when every wavefront has several tiles).
    // The tiles themselves, and so the results, are the same.  Batches use
    // their work list.
    int order = 0;
    // 0: non-temporal particle loads and stores; 1: ordinary cached ones
    // (faster when the particle state fits the last-level cache and stays
    // there between steps).  Results are the same.
    int cached = 0;
};

// Kernel launchers (pic_kernels.hip).  launch_step enqueues one step on
// `stream` as two launches: the particle pass, then the field solve.
//   items == nullptr: single run `runs[0]`, tiles split over `grid`
//   workgroups in the shape's tile order, `table` its gather table (Ehat,
//   or Ehat64 for the FP64 state; may be null for the prologue) and ng_lds
//   its ng.  Otherwise the workgroups take items[0 .. queue->nitems)
//   through the queue (`table` unused).
//   The solve launch has nsolve workgroups; workgroup b solves
//   runs[slots[b]] (slots == nullptr: runs[b]); a slot of -1, idle and
//   finished runs return at once.
//   prologue != 0: deposit + solve only (creation), no push.
//   ev (optional): events recorded before the particle pass (e0), between
//   the two launches (e1) and after the solve (e2).
struct StepEvents {
    hipEvent_t e0, e1, e2;
};
hipError_t launch_step(RunDev *runs, const WorkItem *items, WorkQueue *queue, const void *table,
                       int grid, const LaunchShape &shape, int ng_lds, int precision, int prologue,
                       const int32_t *slots, int nsolve, hipStream_t stream, const StepEvents *ev = nullptr);

// The solve launch alone (pic_solve.hip): nsolve workgroups, workgroup b
// solves runs[slots[b]] (or runs[b]); ng_max bounds the ng of every run in
// the launch.
hipError_t launch_solve(RunDev *runs, const int32_t *slots, int nsolve, int prologue, int ng_max,
                        hipStream_t stream);

// The particle pass alone (used by the autotuner on saved state).
hipError_t launch_particles(RunDev *runs, const WorkItem *items, WorkQueue *queue, const void *table,
                            int grid, const LaunchShape &shape, int ng_lds, int precision,
                            int prologue, hipStream_t stream);

// Allow the step kernels of this shape/precision the LDS they need (called
// once before the first launch and before any graph capture).
hipError_t step_prepare(const LaunchShape &shape, int precision);

// Largest resident workgroups per CU for the step kernel.
int step_occupancy(const LaunchShape &shape, int ng_lds, int precision);

// Dynamic LDS of one workgroup: the int64 grid plus the gather table, each
// with two ghost nodes.
size_t step_lds_bytes(int precision, int ng_lds);

// Cell sort (pic_sort.hip).  A run of np particles is split into nseg
// segments of seg particles (nseg <= kMaxSortSegments); the count table has
// (ng + 1) * nseg entries, scanned in blocks of nblk.
constexpr int kMaxSortSegments = 1024;
struct SortPlan {
    int seg, nseg, nblk;
    int64_t table_len;
};
SortPlan sort_plan(int64_t np, int ng);
size_t sort_scratch_bytes(int64_t np, int ng);
// Allow the scatter kernel its LDS (once, before any launch or capture).
hipError_t sort_prepare();
// Enqueue a stable sort of run R's particles by cell into its alternate
// arrays, then swap the arrays in the descriptor (device side).
hipError_t launch_sort(RunDev *R, int64_t np, int ng, int precision, void *scratch, hipStream_t stream);

// Device-side loader (pic_loader.hip): particle i gets x0 = L u_i,
// x = wrap(x0 + amp sin(k x0)), v = v0 (-1)^i (two beams) or v0, plus
// vth n_i, with u_i and n_i drawn from SplitMix64 streams whose bases are
// given; stored in engine units like the host conversion.
struct LoaderArgs {
    double L, dt, amp, k, v0, vth;
    unsigned long long base_pos, base_v1, base_v2, base_sign;
    int32_t beams, lattice;
};
unsigned long long loader_stream_base(unsigned long long seed, int stream);

// Phase-space binning (pic_phase.hip): bins of (x, v) as described there.
constexpr int kMaxPhaseBins = 16384;
struct PhaseArgs {
    double xs, w_lo, w_bin;
    int32_t nx, nv;
};
hipError_t launch_phase(const void *u, const void *w, int64_t np, int precision, const PhaseArgs &a,
                        unsigned *counts, unsigned long long *outside, int cus, hipStream_t stream);
hipError_t launch_loader(void *u, void *w, int64_t np, int ng, int precision, const LoaderArgs &a, int cus,
                         hipStream_t stream);
// Fixed device scratch of the allocation-free phase-space call (pic_phase.hip):
// its size, its address on the current device (resolved once per device),
// and a fill kernel that zeroes `bytes` (a multiple of 4) at `p`.
constexpr size_t kPhaseScratchBytes = 8 + sizeof(unsigned) * kMaxPhaseBins;
hipError_t phase_scratch(void **out);
hipError_t launch_zero(void *p, size_t bytes, hipStream_t stream);

// Bandwidth reference (pic_probe.hip): swap two device arrays of nvec
// 16-byte vectors (the particle pass's bytes, nothing else).
hipError_t launch_swap(void *a, void *b, int64_t nvec, int cus, bool cached, hipStream_t stream);

// Autotuner (pic_tune.hip).  tune_key names a size class; tune_lookup finds
// a cached shape; tune_shapes times `launch(shape)` (one particle pass on
// saved state, after an untimed `prepare(shape)`) for every candidate (with
// `orders`, in both tile orders) and caches and returns the choice; *best
// holds the incumbent on entry.
std::string tune_key(const char *kind, int precision, int ng, int64_t np);
bool tune_lookup(const std::string &key, LaunchShape *out);
hipError_t tune_shapes(const std::string &key, int precision, bool orders, hipStream_t stream,
                       const std::function<hipError_t(const LaunchShape &)> &prepare,
                       const std::function<hipError_t(const LaunchShape &)> &launch, LaunchShape *best);

// ---------------------------------------------- wavefront FP64 sums --
// (device helpers shared by the particle pass and the solve)

// v of lane `lane ^ 1`, `lane ^ 2`, and of the mirrored lane in its half
// row (i <-> 7 - i) and row (i <-> 15 - i): DPP moves, no LDS.
template <int CTRL>
__device__ __forceinline__ double dpp_move(double v) {
    const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(v), CTRL, 0xf, 0xf, false);
    const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(v), CTRL, 0xf, 0xf, false);
    return __hiloint2double(hi, lo);
}
__device__ __forceinline__ double lane_read(double v, int lane) {
    const int lo = __builtin_amdgcn_readlane(__double2loint(v), lane);
    const int hi = __builtin_amdgcn_readlane(__double2hiint(v), lane);
    return __hiloint2double(hi, lo);
}

// Sum over the 64 lanes in a fixed order, the same value in every lane:
// pairs, quads, half rows and rows of 16 by DPP moves (a + b and b + a are
// the same double, so every lane of a row holds the same row sum), then
// the four row sums in lane order.
__device__ __forceinline__ double wave_sum(double v) {
    v += dpp_move<0xB1>(v);    // quad_perm [1,0,3,2]
    v += dpp_move<0x4E>(v);    // quad_perm [2,3,0,1]
    v += dpp_move<0x141>(v);   // row_half_mirror
    v += dpp_move<0x140>(v);   // row_mirror
    return ((lane_read(v, 0) + lane_read(v, 16)) + lane_read(v, 32)) + lane_read(v, 48);
}

// Integer sum over the 64 lanes (exact in any order), with the same DPP
// moves of the two 32-bit halves (data movement only) and the same lane
// reads.  Both overloads live here so that no scope hides one of them from a
// caller of the other.
template <int CTRL>
__device__ __forceinline__ long long dpp_move(long long v) {
    const int lo = __builtin_amdgcn_update_dpp(0, (int)(unsigned)(unsigned long long)v, CTRL, 0xf, 0xf, false);
    const int hi = __builtin_amdgcn_update_dpp(0, (int)(unsigned)((unsigned long long)v >> 32), CTRL, 0xf, 0xf,
                                               false);
    return (long long)(((unsigned long long)(unsigned)hi << 32) | (unsigned)lo);
}
__device__ __forceinline__ long long lane_read(long long v, int lane) {
    const unsigned lo = __builtin_amdgcn_readlane((int)(unsigned)(unsigned long long)v, lane);
    const unsigned hi = __builtin_amdgcn_readlane((int)(unsigned)((unsigned long long)v >> 32), lane);
    return (long long)(((unsigned long long)hi << 32) | lo);
}
__device__ __forceinline__ long long wave_sum(long long v) {
    v += dpp_move<0xB1>(v);
    v += dpp_move<0x4E>(v);
    v += dpp_move<0x141>(v);
    v += dpp_move<0x140>(v);
    return ((lane_read(v, 0) + lane_read(v, 16)) + lane_read(v, 32)) + lane_read(v, 48);
}


}  // namespace pic1d
