// Host runtime of the PIC engine: parameter validation, device layout,
// run lifecycle, graph replay, and the batched engine (device arena
// allocator, run table, LPT work schedule, continuous admission).
// Implements the C ABI declared in include/pic.h.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <functional>
#include <map>
#include <mutex>
#include <string>
#include <unordered_map>
#include <vector>

#include "pic.h"
#include "pic_internal.h"

using namespace pic1d;

// ------------------------------------------------------------------ errors --

static thread_local std::string g_err;

static pic_status fail(pic_status st, const char *fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
    return st;
}

#define HIP_TRY(expr)                                                                      \
    do {                                                                                   \
        hipError_t e_ = (expr);                                                            \
        if (e_ != hipSuccess)                                                              \
            return fail(PIC_EDEVICE, "%s failed: %s", #expr, hipGetErrorString(e_));       \
    } while (0)

extern "C" const char *pic_last_error(void) { return g_err.c_str(); }
extern "C" const char *pic_version(void) { return "pic1d-gfx950 1.0"; }

// ------------------------------------------------------------ device info --

namespace {

struct DeviceInfo {
    int cus = 256;
    LaunchShape shape;     // default launch shape
    bool forced = false;   // shape set through PIC1D_BLOCK / PIC1D_UNROLL / PIC1D_TILE_ORDER / PIC1D_CACHED
    bool autotune = true;  // PIC1D_AUTOTUNE=0 turns the autotuner off
};

DeviceInfo device_info() {
    DeviceInfo d;
    int dev = 0;
    if (hipGetDevice(&dev) == hipSuccess) {
        int n = 0;
        if (hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess && n > 0)
            d.cus = n;
    }
    d.shape.block = 1024;
    d.shape.unroll = 1;
    if (const char *b = getenv("PIC1D_BLOCK")) {
        int v = atoi(b);
        if (v == 256 || v == 512 || v == 640 || v == 768 || v == 1024) {
            d.shape.block = v;
            d.forced = true;
        }
    }
    if (const char *u = getenv("PIC1D_UNROLL")) {
        int v = atoi(u);
        if (v == 1 || v == 2 || v == 4) {
            d.shape.unroll = v;
            d.forced = true;
        }
    }
    if (const char *o = getenv("PIC1D_TILE_ORDER")) {
        d.shape.order = atoi(o) != 0 ? 1 : 0;
        d.forced = true;
    }
    if (const char *c = getenv("PIC1D_CACHED")) {
        d.shape.cached = atoi(c) != 0 ? 1 : 0;
        d.forced = true;
    }
    if (const char *a = getenv("PIC1D_AUTOTUNE")) d.autotune = atoi(a) != 0;
    return d;
}

pic_status validate(const pic_params *p) {
    if (!p) return fail(PIC_EINVAL, "params is NULL");
    if (!(std::isfinite(p->L) && p->L > 0)) return fail(PIC_EINVAL, "L must be finite and > 0 (got %g)", p->L);
    if (p->ng < 2 || p->ng > PIC_MAX_NG)
        return fail(PIC_EINVAL, "ng must be in [2, %d] (got %d)", PIC_MAX_NG, p->ng);
    if (p->np < 1 || p->np >= (int64_t)1 << 31)
        return fail(PIC_EINVAL, "np must be in [1, 2^31) (got %lld)", (long long)p->np);
    if (!(std::isfinite(p->dt) && p->dt > 0)) return fail(PIC_EINVAL, "dt must be finite and > 0");
    if (!(std::isfinite(p->qm) && p->qm != 0)) return fail(PIC_EINVAL, "qm must be finite and nonzero");
    if (!(std::isfinite(p->rho0) && p->rho0 > 0)) return fail(PIC_EINVAL, "rho0 must be finite and > 0");
    if (p->precision != PIC_FP32 && p->precision != PIC_FP64)
        return fail(PIC_EINVAL, "precision must be PIC_FP32 or PIC_FP64");
    if (p->tile < 0 || p->tile % kUnit != 0 || p->tile > (1 << 20))
        return fail(PIC_EINVAL, "tile must be 0 or a multiple of %d up to 2^20 (got %d)", kUnit, p->tile);
    if (p->history_cap < 0) return fail(PIC_EINVAL, "history_cap must be >= 0");
    if (p->solver != PIC_SOLVE_EXACT && p->solver != PIC_SOLVE_CG_PAPER)
        return fail(PIC_EINVAL, "solver must be PIC_SOLVE_EXACT or PIC_SOLVE_CG_PAPER (got %d)", p->solver);
    if (p->cg_iters < 0 || p->cg_iters > 100000) return fail(PIC_EINVAL, "cg_iters must be in [0, 100000]");
    if (p->sort_every < PIC_SORT_AUTO)
        return fail(PIC_EINVAL, "sort_every must be >= 0 or PIC_SORT_AUTO (got %d)", p->sort_every);
    return PIC_OK;
}

// Default particles per tile: a pure function of np, so that every launch
// shape and schedule sees the same tiles (and the same diagnostic summation
// order).  About 8192 tiles per run, so that a large single run gives the
// device's wavefronts several tiles each (with the round-robin tile order
// the autotuner can then pick, HBM serves the pass faster); at least 2048
// particles from 1M particles on (fewer per-tile start-ups when many runs
// share the device), at least 1024 and at most 16384 (whole block units).
int default_tile(int64_t np) {
    const int64_t per = (np + 8191) / 8192;
    int64_t t = (per + kUnit - 1) / kUnit * kUnit;
    t = std::max<int64_t>(t, np >= ((int64_t)1 << 20) ? 2 * kUnit : kUnit);
    return (int)std::min<int64_t>(16384, t);
}

size_t align_up(size_t v, size_t a) { return (v + a - 1) / a * a; }

// Bytes after a single run's layout that hold its device descriptor.
constexpr size_t kDescBytes = (sizeof(RunDev) + 255) / 256 * 256;

struct Layout {
    size_t u, w, u_alt, w_alt, sort, S0, S1, Ehat, Ehat64, E64, part, hist, total;
    int tile, ntiles;
    size_t esize;
    bool sorting;         // alternate particle arrays and sort scratch present
};

Layout make_layout(const pic_params *p) {
    Layout L{};
    L.esize = p->precision == PIC_FP64 ? 8 : 4;
    L.tile = p->tile > 0 ? p->tile : default_tile(p->np);
    L.ntiles = (int)((p->np + L.tile - 1) / L.tile);
    const size_t np_pad = align_up((size_t)p->np, 64);
    size_t off = 0;
    auto take = [&](size_t bytes) {
        size_t at = off;
        off = align_up(off + bytes, 256);
        return at;
    };
    L.u = take(np_pad * L.esize);
    L.w = take(np_pad * L.esize);
    L.sorting = p->sort_every > 0 || p->sort_every == PIC_SORT_AUTO;
    if (L.sorting) {
        L.u_alt = take(np_pad * L.esize);
        L.w_alt = take(np_pad * L.esize);
        L.sort = take(sort_scratch_bytes(p->np, p->ng));
    }
    L.S0 = take((size_t)p->ng * 8);
    L.S1 = take((size_t)p->ng * 8);
    L.Ehat = take((size_t)p->ng * 4);
    L.Ehat64 = take((size_t)p->ng * 8);
    L.E64 = take((size_t)p->ng * 8);
    L.part = take((size_t)L.ntiles * kPartCols * 8);
    L.hist = take((size_t)std::max<int64_t>(p->history_cap, 1) * kHistCols * 8);
    L.total = off;
    return L;
}

}  // namespace

// --------------------------------------------------------------- the run --

struct pic_run {
    pic_params p{};
    Layout lay{};
    char *base = nullptr;       // device memory of the run
    bool owns_mem = false;
    hipStream_t stream = nullptr;
    RunDev host{};              // host mirror of the descriptor (pointers, constants)
    RunDev *dev = nullptr;      // device descriptor (owned by the run or a batch slot)
    bool owns_dev = false;
    bool error = false;
    bool batch_member = false;
    // Batch members: reads go through the batch's own non-blocking stream,
    // and a run reported complete (settled) is read without waiting for the
    // batch's queued launches, which no longer touch it.
    hipStream_t io_stream = nullptr;
    bool settled = false;
    LaunchShape shape;
    int grid = 1;
    double Q = 0, m = 0, dx = 0;
    // Steps enqueued so far, and whether the particle arrays have traded
    // places with their alternates (an odd number of cell sorts enqueued).
    int64_t issued = 0;
    bool swapped = false;
    void *cur_u() const { return swapped ? host.u_alt : host.u; }
    void *cur_w() const { return swapped ? host.w_alt : host.w; }
    int sort_every() const { return lay.sorting && p.sort_every > 0 ? p.sort_every : 0; }
    // graph replay cache
    hipGraphExec_t graph = nullptr;       // graph_steps steps
    hipGraphExec_t graph_sort = nullptr;  // cell sort + graph_steps steps
    int graph_steps = 0;
};

// The run's gather table in its state precision (fixed for the run's life:
// the cell sort moves particles, not the field), passed to the particle pass
// so that it loads the table without waiting for the run descriptor.
const void *gather_table_of(const pic_run *r) {
    return r->p.precision ? (const void *)r->host.Ehat64 : (const void *)r->host.Ehat;
}

extern "C" pic_status pic_footprint(const pic_params *params, size_t *bytes) {
    pic_status st = validate(params);
    if (st != PIC_OK) return st;
    if (!bytes) return fail(PIC_EINVAL, "bytes is NULL");
    *bytes = make_layout(params).total + kDescBytes;   // + the device descriptor
    return PIC_OK;
}

namespace {

pic_status check_particles(const pic_params *p, const double *x0, const double *v) {
    if (!x0 || !v) return fail(PIC_EINVAL, "x0 and v_mhalf must not be NULL");
    const double vmax_ok = p->L / p->dt;
    for (int64_t i = 0; i < p->np; ++i) {
        if (!(x0[i] >= 0.0 && x0[i] < p->L))
            return fail(PIC_EINVAL, "x0[%lld] = %.17g outside [0, L)", (long long)i, x0[i]);
        if (!(std::fabs(v[i]) < vmax_ok))
            return fail(PIC_EINVAL, "v_mhalf[%lld] = %g: need finite |v| dt < L", (long long)i, v[i]);
    }
    return PIC_OK;
}

// A device loader's parameters.  The normal deviates come from 53-bit
// uniforms, so |n| <= sqrt(-2 ln 2^-53) < 8.58 and |v| <= |v0| + 8.58 vth:
// the single-wrap contract |v| dt < L is checked on that bound.
pic_status check_loader(const pic_params *p, const pic_loader *ld) {
    if (!ld) return fail(PIC_EINVAL, "loader is NULL");
    if (ld->pos_stream < 0 || ld->vel_stream < 0 || ld->pos_stream > (1 << 30) || ld->vel_stream > (1 << 30))
        return fail(PIC_EINVAL, "loader streams must be in [0, 2^30]");
    if (ld->beams != PIC_BEAMS_ONE && ld->beams != PIC_BEAMS_ALTERNATE && ld->beams != PIC_BEAMS_RANDOM)
        return fail(PIC_EINVAL, "loader beams must be PIC_BEAMS_ONE, _ALTERNATE or _RANDOM");
    if (ld->lattice != 0 && ld->lattice != 1) return fail(PIC_EINVAL, "loader lattice must be 0 or 1");
    if (!(std::isfinite(ld->amp) && std::isfinite(ld->k) && std::isfinite(ld->v0) && std::isfinite(ld->vth) &&
          ld->vth >= 0))
        return fail(PIC_EINVAL, "loader amp, k, v0 must be finite and vth finite and >= 0");
    if (!((std::fabs(ld->v0) + 8.58 * ld->vth) * p->dt < p->L))
        return fail(PIC_EINVAL, "loader velocities can exceed L/dt (need (|v0| + 8.58 vth) dt < L)");
    return PIC_OK;
}

LoaderArgs loader_args(const pic_params *p, const pic_loader *ld) {
    LoaderArgs a{};
    a.L = p->L;
    a.dt = p->dt;
    a.amp = ld->amp;
    a.k = ld->k;
    a.v0 = ld->v0;
    a.vth = ld->vth;
    a.base_pos = loader_stream_base(ld->seed, ld->pos_stream);
    a.base_v1 = loader_stream_base(ld->seed, ld->vel_stream);
    a.base_v2 = loader_stream_base(ld->seed, ld->vel_stream + 1);
    a.base_sign = loader_stream_base(ld->seed, ld->vel_stream + 2);
    a.beams = ld->beams;
    a.lattice = ld->lattice;
    return a;
}

// Fill the descriptor constants (normalisation of Sec. 2 / Appendix A):
// Q = sign(qm) rho0 L / np, m = Q/qm, ecoef = qm dt^2/dx, ...
void fill_constants(pic_run *r) {
    const pic_params &p = r->p;
    r->dx = p.L / p.ng;
    r->Q = (p.qm < 0 ? -1.0 : 1.0) * p.rho0 * p.L / (double)p.np;
    r->m = r->Q / p.qm;
    RunDev &h = r->host;
    h.np = p.np;
    h.ng = p.ng;
    h.hist_cap = p.history_cap;
    h.step = 0;
    h.diag_step = 0;
    h.step_target = INT64_MAX;
    h.tile = r->lay.tile;
    h.ntiles = r->lay.ntiles;
    h.precision = p.precision;
    h.solver = p.solver;
    h.cg_iters = p.cg_iters > 0 ? p.cg_iters : 150;
    h.flags = 0;
    h.dx = r->dx;
    h.qfac = r->Q / (r->dx * 4294967296.0);
    h.ecoef = p.qm * p.dt * p.dt / r->dx;
    const double vs = r->dx / p.dt;     // w -> v
    h.kcoef = 0.5 * r->m * vs * vs;
    h.pcoef = r->m * vs;
}

void carve(pic_run *r) {
    char *b = r->base;
    const Layout &L = r->lay;
    RunDev &h = r->host;
    h.u = b + L.u;
    h.w = b + L.w;
    h.u_alt = L.sorting ? b + L.u_alt : nullptr;
    h.w_alt = L.sorting ? b + L.w_alt : nullptr;
    h.S01[0] = (unsigned long long *)(b + L.S0);
    h.S01[1] = (unsigned long long *)(b + L.S1);
    h.Ehat = (float *)(b + L.Ehat);
    h.Ehat64 = r->p.precision == PIC_FP64 ? (double *)(b + L.Ehat64) : nullptr;
    h.E64 = (double *)(b + L.E64);
    h.tile_part = (double *)(b + L.part);
    h.hist = (double *)(b + L.hist);
    h.sort_scratch = L.sorting ? b + L.sort : nullptr;
    h.sort_swap = 0;
}

// Convert host FP64 particles to engine units: the stored position is
// s = x/dx + 1/2 in [1/2, ng + 1/2) (rounded once to the state precision; a
// value that rounds up to ng + 1/2 is the same point as x = 0) and the
// velocity w = v dt/dx.  `u` and `w` receive np elements of the state type.
void convert_particles(const pic_run *r, const double *x0, const double *v, void *u, void *w) {
    const pic_params &p = r->p;
    const double wscale = p.dt / r->dx;
    const size_t n = (size_t)p.np;
    if (p.precision == PIC_FP32) {
        float *uo = (float *)u, *wo = (float *)w;
        const float hi = (float)p.ng + 0.5f;
        for (size_t i = 0; i < n; ++i) {
            float si = (float)(x0[i] / r->dx + 0.5);
            if (!(si < hi)) si = 0.5f;
            uo[i] = si;
            wo[i] = (float)(v[i] * wscale);
        }
    } else {
        double *uo = (double *)u, *wo = (double *)w;
        const double hi = (double)p.ng + 0.5;
        for (size_t i = 0; i < n; ++i) {
            double si = x0[i] / r->dx + 0.5;
            if (!(si < hi)) si = 0.5;
            uo[i] = si;
            wo[i] = v[i] * wscale;
        }
    }
}

// Convert and upload a single run's particles (synchronous).
pic_status upload_particles(pic_run *r, const double *x0, const double *v) {
    const size_t bytes = (size_t)r->p.np * r->lay.esize;
    std::vector<char> u(bytes), w(bytes);
    convert_particles(r, x0, v, u.data(), w.data());
    HIP_TRY(hipMemcpyAsync(r->host.u, u.data(), bytes, hipMemcpyHostToDevice, r->stream));
    HIP_TRY(hipMemcpyAsync(r->host.w, w.data(), bytes, hipMemcpyHostToDevice, r->stream));
    HIP_TRY(hipStreamSynchronize(r->stream));
    return PIC_OK;
}

// Queue, on the run's stream: zero the grids, publish the descriptor from
// `desc` (host memory that stays valid until the copy has run) and run the
// prologue (deposit of x^0 and solve for E^0).  Nothing waits.
pic_status queue_device_init(pic_run *r, const RunDev *desc) {
    HIP_TRY(hipMemsetAsync(r->host.S01[0], 0, (size_t)r->p.ng * 8, r->stream));
    HIP_TRY(hipMemsetAsync(r->host.S01[1], 0, (size_t)r->p.ng * 8, r->stream));
    HIP_TRY(hipMemsetAsync(r->host.tile_part, 0, (size_t)r->lay.ntiles * kPartCols * 8, r->stream));
    HIP_TRY(hipMemcpyAsync(r->dev, desc, sizeof(RunDev), hipMemcpyHostToDevice, r->stream));
    HIP_TRY(step_prepare(r->shape, r->p.precision));
    HIP_TRY(launch_step(r->dev, nullptr, nullptr, gather_table_of(r), r->grid, r->shape, r->p.ng, r->p.precision, 1, nullptr,
                        1, r->stream));
    return PIC_OK;
}

// Device state of a single run, synchronously.
pic_status init_device_state(pic_run *r) {
    pic_status st = queue_device_init(r, &r->host);
    if (st != PIC_OK) return st;
    HIP_TRY(hipStreamSynchronize(r->stream));
    return PIC_OK;
}

// Bytes of a run's state that trial passes change: the particle arrays and
// both charge-sum buffers.
size_t state_bytes(const pic_run *r) { return 2 * (size_t)r->p.np * r->lay.esize + 2 * (size_t)r->p.ng * 8; }

// Copy a run's state (state_bytes) to/from a scratch buffer: autotuning runs
// real particle passes on the run's own state and then puts it back (those
// passes deposit into one charge-sum buffer and clear the other); the tile
// partials they write are rewritten by the next real pass.
pic_status save_particles(const pic_run *r, char *dst, bool restore) {
    const size_t bytes = (size_t)r->p.np * r->lay.esize, sb = (size_t)r->p.ng * 8;
    char *u = (char *)r->cur_u(), *w = (char *)r->cur_w();
    char *s0 = (char *)r->host.S01[0], *s1 = (char *)r->host.S01[1];
    if (restore) {
        HIP_TRY(hipMemcpyAsync(u, dst, bytes, hipMemcpyDeviceToDevice, r->stream));
        HIP_TRY(hipMemcpyAsync(w, dst + bytes, bytes, hipMemcpyDeviceToDevice, r->stream));
        HIP_TRY(hipMemcpyAsync(s0, dst + 2 * bytes, sb, hipMemcpyDeviceToDevice, r->stream));
        HIP_TRY(hipMemcpyAsync(s1, dst + 2 * bytes + sb, sb, hipMemcpyDeviceToDevice, r->stream));
        HIP_TRY(hipMemsetAsync(&r->dev->flags, 0, sizeof(uint32_t), r->stream));
    } else {
        HIP_TRY(hipMemcpyAsync(dst, u, bytes, hipMemcpyDeviceToDevice, r->stream));
        HIP_TRY(hipMemcpyAsync(dst + bytes, w, bytes, hipMemcpyDeviceToDevice, r->stream));
        HIP_TRY(hipMemcpyAsync(dst + 2 * bytes, s0, sb, hipMemcpyDeviceToDevice, r->stream));
        HIP_TRY(hipMemcpyAsync(dst + 2 * bytes + sb, s1, sb, hipMemcpyDeviceToDevice, r->stream));
    }
    return PIC_OK;
}

// Workgroups of a single run's particle pass: enough to give each wavefront
// a tile, at least 16K particles per workgroup (fewer workgroups merging into
// the same grid for small runs), at most what is resident at once.
int single_run_grid(const pic_run *r, const LaunchShape &shape, int cus) {
    const int occ = step_occupancy(shape, r->p.ng, r->p.precision);
    const int waves = shape.block / 64;
    int64_t want = (r->lay.ntiles + waves - 1) / waves;
    want = std::min<int64_t>(want, (r->p.np + 16383) / 16384);
    return (int)std::max<int64_t>(1, std::min<int64_t>(want, (int64_t)cus * occ));
}

// Launch shape of a run: forced by the environment, else cached or tuned
// for the run's size class, else the default.
pic_status choose_shape(pic_run *r, const DeviceInfo &d) {
    LaunchShape shape = d.shape;
    if (!d.forced && d.autotune) {
        const std::string key = tune_key("run", r->p.precision, r->p.ng, r->p.np);
        if (!tune_lookup(key, &shape)) {
            char *tmp = nullptr;
            const size_t bytes = state_bytes(r);
            if (hipMalloc((void **)&tmp, bytes) != hipSuccess)
                return fail(PIC_ENOMEM, "autotune scratch of %zu bytes", bytes);
            pic_status st = save_particles(r, tmp, false);
            hipError_t te = hipSuccess;
            if (st == PIC_OK) {
                const int cus = d.cus;
                te = tune_shapes(
                    key, r->p.precision, true, r->stream, [](const LaunchShape &) { return hipSuccess; },
                    [r, cus](const LaunchShape &s) {
                        return launch_particles(r->dev, nullptr, nullptr, gather_table_of(r), single_run_grid(r, s, cus), s, r->p.ng,
                                                r->p.precision, 0, r->stream);
                    },
                    &shape);
                st = save_particles(r, tmp, true);
            }
            hipError_t se = hipStreamSynchronize(r->stream);
            (void)hipFree(tmp);
            if (st != PIC_OK) return st;
            if (te != hipSuccess) return fail(PIC_EDEVICE, "autotune: %s", hipGetErrorString(te));
            if (se != hipSuccess) return fail(PIC_EDEVICE, "autotune: %s", hipGetErrorString(se));
        }
    }
    r->shape = shape;
    HIP_TRY(step_prepare(r->shape, r->p.precision));
    r->grid = single_run_grid(r, r->shape, d.cus);
    return PIC_OK;
}

// Cell-sort period of a run created with PIC_SORT_AUTO: the particle pass
// timed on the state as loaded, the sort, and the pass on the sorted state
// (kReps passes each, HIP events on the run's stream), all on a saved copy
// of the state that is put back afterwards.  Sort every
// K = ceil(2 t_sort / (t_unsorted - t_sorted)) steps (twice the steps the
// sort takes to pay for itself) if sorting makes the pass faster, else never.
pic_status choose_sort_period(pic_run *r) {
    constexpr int kReps = 3;
    char *tmp = nullptr;
    const size_t bytes = state_bytes(r);
    if (hipMalloc((void **)&tmp, bytes) != hipSuccess)
        return fail(PIC_ENOMEM, "sort-period trial scratch of %zu bytes", bytes);
    hipEvent_t ev[4] = {};
    hipError_t e = hipSuccess;
    for (int i = 0; i < 4 && e == hipSuccess; ++i) e = hipEventCreate(&ev[i]);
    pic_status st = e == hipSuccess ? save_particles(r, tmp, false) : PIC_OK;
    auto pass = [r]() {
        return launch_particles(r->dev, nullptr, nullptr, gather_table_of(r), r->grid, r->shape, r->p.ng, r->p.precision, 0,
                                r->stream);
    };
    float t_u = 0, t_sort = 0, t_s = 0;
    if (e == hipSuccess && st == PIC_OK) {
        e = pass();                                                      // warm-up
        if (e == hipSuccess) e = hipEventRecord(ev[0], r->stream);
        for (int k = 0; k < kReps && e == hipSuccess; ++k) e = pass();
        if (e == hipSuccess) e = hipEventRecord(ev[1], r->stream);
        if (e == hipSuccess) st = save_particles(r, tmp, true);          // back to the loaded order
        if (e == hipSuccess && st == PIC_OK) e = hipEventRecord(ev[2], r->stream);
        if (e == hipSuccess && st == PIC_OK)
            e = launch_sort(r->dev, r->p.np, r->p.ng, r->p.precision, r->host.sort_scratch, r->stream);
        if (e == hipSuccess && st == PIC_OK) {
            r->swapped = !r->swapped;                                    // the sort swapped the arrays
            e = hipEventRecord(ev[3], r->stream);
        }
        if (e == hipSuccess && st == PIC_OK) {
            e = hipEventSynchronize(ev[3]);
            if (e == hipSuccess) e = hipEventElapsedTime(&t_u, ev[0], ev[1]);
            if (e == hipSuccess) e = hipEventElapsedTime(&t_sort, ev[2], ev[3]);
        }
        if (e == hipSuccess && st == PIC_OK) e = hipEventRecord(ev[0], r->stream);
        for (int k = 0; k < kReps && e == hipSuccess && st == PIC_OK; ++k) e = pass();
        if (e == hipSuccess && st == PIC_OK) e = hipEventRecord(ev[1], r->stream);
        if (e == hipSuccess && st == PIC_OK) e = hipEventSynchronize(ev[1]);
        if (e == hipSuccess && st == PIC_OK) e = hipEventElapsedTime(&t_s, ev[0], ev[1]);
        // the loaded state again, now in the arrays the sort made current
        if (e == hipSuccess && st == PIC_OK) st = save_particles(r, tmp, true);
    }
    const hipError_t se = hipStreamSynchronize(r->stream);
    for (hipEvent_t x : ev)
        if (x) (void)hipEventDestroy(x);
    (void)hipFree(tmp);
    if (st != PIC_OK) return st;
    if (e != hipSuccess) return fail(PIC_EDEVICE, "sort-period trial: %s", hipGetErrorString(e));
    if (se != hipSuccess) return fail(PIC_EDEVICE, "sort-period trial: %s", hipGetErrorString(se));
    t_u /= kReps;
    t_s /= kReps;
    int k = 0;
    if (t_s < t_u) {
        const double steps = std::ceil(2.0 * (double)t_sort / (double)(t_u - t_s));
        k = (int)std::max(1.0, std::min(steps, (double)(1 << 20)));
    }
    r->p.sort_every = k;
    return PIC_OK;
}

pic_status check_run(pic_run *r) {
    if (!r) return fail(PIC_EINVAL, "run is NULL");
    if (r->error) return fail(PIC_ESTATE, "run is in an error state after an earlier device error");
    return PIC_OK;
}

// Capture `count` launches made by `launch(stream)` into an executable graph.
// Capture runs on a private non-blocking stream (the caller's stream may be
// the legacy default stream, which cannot be captured); the graph is later
// launched on the caller's stream.
template <typename F>
pic_status capture_graph(F launch, int count, hipGraphExec_t *exec) {
    hipStream_t cs = nullptr;
    HIP_TRY(hipStreamCreateWithFlags(&cs, hipStreamNonBlocking));
    hipGraph_t g = nullptr;
    hipError_t be = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
    hipError_t le = hipSuccess;
    if (be == hipSuccess) {
        for (int k = 0; k < count && le == hipSuccess; ++k) le = launch(cs);
    }
    hipError_t ce = be == hipSuccess ? hipStreamEndCapture(cs, &g) : be;
    (void)hipStreamDestroy(cs);
    if (le != hipSuccess || ce != hipSuccess) {
        if (g) (void)hipGraphDestroy(g);
        return fail(PIC_EDEVICE, "graph capture failed: %s",
                    hipGetErrorString(le != hipSuccess ? le : ce));
    }
    hipError_t ie = hipGraphInstantiate(exec, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (ie != hipSuccess) return fail(PIC_EDEVICE, "graph instantiate: %s", hipGetErrorString(ie));
    return PIC_OK;
}

pic_status sync_run(pic_run *r) {
    if (r->settled) return PIC_OK;
    hipError_t e = hipStreamSynchronize(r->stream);
    if (e != hipSuccess) {
        r->error = true;
        return fail(PIC_EDEVICE, "device error: %s", hipGetErrorString(e));
    }
    return PIC_OK;
}

// Device-to-host copy for the read calls (after sync_run).
hipError_t dev_read(const pic_run *r, void *dst, const void *src, size_t bytes) {
    if (!r->io_stream) return hipMemcpy(dst, src, bytes, hipMemcpyDeviceToHost);
    hipError_t e = hipMemcpyAsync(dst, src, bytes, hipMemcpyDeviceToHost, r->io_stream);
    return e != hipSuccess ? e : hipStreamSynchronize(r->io_stream);
}

}  // namespace

namespace {

// Common part of pic_create and pic_create_loaded: memory, descriptor,
// particles (by `fill`, enqueued on the run's stream), initial deposit and
// solve, launch shape.
pic_status create_run(const pic_params *params, void *dev_mem, size_t dev_bytes, void *stream,
                      const std::function<pic_status(pic_run *)> &fill, pic_run **out) {
    pic_run *r = new pic_run();
    r->p = *params;
    r->lay = make_layout(params);
    r->stream = (hipStream_t)stream;
    const size_t need = r->lay.total + kDescBytes;
    if (dev_mem) {
        if ((uintptr_t)dev_mem % 256 != 0) {
            delete r;
            return fail(PIC_EINVAL, "dev_mem must be 256-byte aligned");
        }
        if (dev_bytes < need) {
            delete r;
            return fail(PIC_ENOMEM, "dev_bytes %zu < footprint %zu", dev_bytes, need);
        }
        r->base = (char *)dev_mem;
    } else {
        void *p = nullptr;
        if (hipMalloc(&p, need) != hipSuccess) {
            delete r;
            return fail(PIC_ENOMEM, "hipMalloc of %zu bytes failed", need);
        }
        r->base = (char *)p;
        r->owns_mem = true;
    }
    r->dev = (RunDev *)(r->base + r->lay.total);
    DeviceInfo d = device_info();
    if (r->lay.sorting && sort_prepare() != hipSuccess) {
        if (r->owns_mem) (void)hipFree(r->base);
        delete r;
        return fail(PIC_EDEVICE, "cell-sort kernel setup failed");
    }
    r->shape = d.shape;
    fill_constants(r);
    carve(r);
    r->grid = single_run_grid(r, r->shape, d.cus);
    pic_status st = fill(r);
    if (st == PIC_OK) st = init_device_state(r);
    if (st == PIC_OK) st = choose_shape(r, d);
    if (st == PIC_OK && r->p.sort_every == PIC_SORT_AUTO) st = choose_sort_period(r);
    if (st != PIC_OK) {
        std::string msg = g_err;
        (void)hipStreamSynchronize(r->stream);
        if (r->owns_mem) (void)hipFree(r->base);
        delete r;
        g_err = msg;
        return st;
    }
    *out = r;
    return PIC_OK;
}

}  // namespace

extern "C" pic_status pic_create(const pic_params *params, const double *x0, const double *v_mhalf,
                                 void *dev_mem, size_t dev_bytes, void *stream, pic_run **out) {
    pic_status st = validate(params);
    if (st != PIC_OK) return st;
    if (!out) return fail(PIC_EINVAL, "out is NULL");
    *out = nullptr;
    st = check_particles(params, x0, v_mhalf);
    if (st != PIC_OK) return st;
    return create_run(params, dev_mem, dev_bytes, stream,
                      [x0, v_mhalf](pic_run *r) { return upload_particles(r, x0, v_mhalf); }, out);
}

extern "C" pic_status pic_create_loaded(const pic_params *params, const pic_loader *loader, void *dev_mem,
                                        size_t dev_bytes, void *stream, pic_run **out) {
    pic_status st = validate(params);
    if (st != PIC_OK) return st;
    if (!out) return fail(PIC_EINVAL, "out is NULL");
    *out = nullptr;
    st = check_loader(params, loader);
    if (st != PIC_OK) return st;
    const LoaderArgs a = loader_args(params, loader);
    return create_run(params, dev_mem, dev_bytes, stream,
                      [&a](pic_run *r) {
                          HIP_TRY(launch_loader(r->host.u, r->host.w, r->p.np, r->p.ng, r->p.precision, a,
                                                device_info().cus, r->stream));
                          return PIC_OK;
                      },
                      out);
}

namespace {

// True when the cell sort is due before the next step: every sort_every
// steps, counted from creation (never before the first step).
bool sort_due(const pic_run *r) {
    const int k = r->sort_every();
    return k > 0 && r->issued > 0 && r->issued % k == 0;
}

// Enqueue the next step of a single run (preceded by the cell sort when due).
pic_status enqueue_step(pic_run *r, const StepEvents *ev = nullptr) {
    hipError_t e = hipSuccess;
    if (sort_due(r)) {
        e = launch_sort(r->dev, r->p.np, r->p.ng, r->p.precision, r->host.sort_scratch, r->stream);
        if (e == hipSuccess) r->swapped = !r->swapped;
    }
    if (e == hipSuccess)
        e = launch_step(r->dev, nullptr, nullptr, gather_table_of(r), r->grid, r->shape, r->p.ng, r->p.precision, 0, nullptr, 1,
                        r->stream, ev);
    if (e != hipSuccess) {
        r->error = true;
        return fail(PIC_EDEVICE, "step launch failed: %s", hipGetErrorString(e));
    }
    ++r->issued;
    return PIC_OK;
}

}  // namespace

extern "C" pic_status pic_sort_period(pic_run *r, int32_t *k) {
    pic_status st = check_run(r);
    if (st != PIC_OK) return st;
    if (!k) return fail(PIC_EINVAL, "k is NULL");
    *k = r->sort_every();
    return PIC_OK;
}

extern "C" pic_status pic_sort(pic_run *r) {
    pic_status st = check_run(r);
    if (st != PIC_OK) return st;
    if (r->batch_member) return fail(PIC_ESTATE, "batch members are sorted by the batch");
    if (!r->lay.sorting) return fail(PIC_ESTATE, "run was created without cell sorting (sort_every = 0)");
    hipError_t e = launch_sort(r->dev, r->p.np, r->p.ng, r->p.precision, r->host.sort_scratch, r->stream);
    if (e != hipSuccess) {
        r->error = true;
        return fail(PIC_EDEVICE, "sort launch failed: %s", hipGetErrorString(e));
    }
    r->swapped = !r->swapped;
    return PIC_OK;
}

extern "C" pic_status pic_step(pic_run *r, int64_t nsteps) {
    pic_status st = check_run(r);
    if (st != PIC_OK) return st;
    if (r->batch_member) return fail(PIC_ESTATE, "batch members are stepped with pic_batch_step");
    if (nsteps < 0) return fail(PIC_EINVAL, "nsteps must be >= 0");
    for (int64_t s = 0; s < nsteps && st == PIC_OK; ++s) st = enqueue_step(r);
    return st;
}

extern "C" pic_status pic_step_graph(pic_run *r, int64_t nsteps, int32_t graph_steps) {
    pic_status st = check_run(r);
    if (st != PIC_OK) return st;
    if (r->batch_member) return fail(PIC_ESTATE, "batch members are stepped with pic_batch_step");
    if (nsteps < 0 || graph_steps < 1 || graph_steps > 4096)
        return fail(PIC_EINVAL, "need nsteps >= 0 and graph_steps in [1, 4096]");
    const int G = graph_steps, K = r->sort_every();
    if (r->graph_steps != G) {
        if (r->graph) (void)hipGraphExecDestroy(r->graph);
        if (r->graph_sort) (void)hipGraphExecDestroy(r->graph_sort);
        r->graph = r->graph_sort = nullptr;
        r->graph_steps = G;
    }
    // Two graphs: G steps, and (with the cell sort) a sort followed by G
    // steps.  A graph is replayed only where no sort falls inside it.
    const pic_run *rc = r;
    auto step_launch = [rc](hipStream_t s) {
        return launch_step(rc->dev, nullptr, nullptr, gather_table_of(rc), rc->grid, rc->shape, rc->p.ng, rc->p.precision, 0, nullptr, 1,
                           s);
    };
    int64_t left = nsteps;
    while (left > 0) {
        const bool due = sort_due(r);
        // steps until the next sort after this point
        const int64_t room = K > 0 ? K - (due ? 0 : r->issued % K) : INT64_MAX;
        if (left >= G && (due ? K >= G : room >= G)) {
            hipGraphExec_t *gx = due ? &r->graph_sort : &r->graph;
            if (!*gx) {
                int first = 1;
                st = capture_graph(
                    [&](hipStream_t s) {
                        hipError_t e = hipSuccess;
                        if (due && first)
                            e = launch_sort(rc->dev, rc->p.np, rc->p.ng, rc->p.precision, rc->host.sort_scratch, s);
                        first = 0;
                        return e == hipSuccess ? step_launch(s) : e;
                    },
                    G, gx);
                if (st != PIC_OK) return st;
            }
            HIP_TRY(hipGraphLaunch(*gx, r->stream));
            if (due) r->swapped = !r->swapped;
            r->issued += G;
            left -= G;
        } else {
            st = enqueue_step(r);
            if (st != PIC_OK) return st;
            --left;
        }
    }
    return PIC_OK;
}

namespace {

// Launch `n` steps with events around each launch and average the durations.
template <typename F>
pic_status profiled_steps(F launch, hipStream_t stream, int64_t n, double *ms_particle,
                          double *ms_solve) {
    std::vector<StepEvents> evs((size_t)n);
    for (auto &e : evs) {
        HIP_TRY(hipEventCreate(&e.e0));
        HIP_TRY(hipEventCreate(&e.e1));
        HIP_TRY(hipEventCreate(&e.e2));
    }
    pic_status st = PIC_OK;
    for (int64_t i = 0; i < n && st == PIC_OK; ++i) st = launch(&evs[(size_t)i]);
    hipError_t se = hipStreamSynchronize(stream);
    double a = 0, b = 0;
    for (auto &e : evs) {
        float t1 = 0, t2 = 0;
        if (st == PIC_OK && se == hipSuccess) {
            (void)hipEventElapsedTime(&t1, e.e0, e.e1);
            (void)hipEventElapsedTime(&t2, e.e1, e.e2);
        }
        a += t1;
        b += t2;
        (void)hipEventDestroy(e.e0);
        (void)hipEventDestroy(e.e1);
        (void)hipEventDestroy(e.e2);
    }
    if (st != PIC_OK) return st;
    if (se != hipSuccess) return fail(PIC_EDEVICE, "device error: %s", hipGetErrorString(se));
    if (ms_particle) *ms_particle = a / (double)n;
    if (ms_solve) *ms_solve = b / (double)n;
    return PIC_OK;
}

}  // namespace

extern "C" pic_status pic_step_profiled(pic_run *r, int64_t nsteps, double *ms_particle,
                                        double *ms_solve) {
    pic_status st = check_run(r);
    if (st != PIC_OK) return st;
    if (r->batch_member) return fail(PIC_ESTATE, "batch members are stepped with pic_batch_step");
    if (nsteps < 1) return fail(PIC_EINVAL, "nsteps must be >= 1");
    st = profiled_steps(
        [r](const StepEvents *ev) { return enqueue_step(r, ev); },
        r->stream, nsteps, ms_particle, ms_solve);
    if (st == PIC_EDEVICE) r->error = true;
    return st;
}

extern "C" pic_status pic_bandwidth_probe(void *a, void *b, int64_t n, int32_t reps, int32_t cached,
                                          void *stream, double *ms) {
    if (!a || !b || !ms) return fail(PIC_EINVAL, "a, b and ms must not be NULL");
    if (n < 4 || n % 4 != 0 || reps < 1 || (uintptr_t)a % 16 || (uintptr_t)b % 16)
        return fail(PIC_EINVAL, "need n a positive multiple of 4, reps >= 1, 16-byte aligned arrays");
    if (cached != 0 && cached != 1) return fail(PIC_EINVAL, "cached must be 0 or 1 (got %d)", cached);
    hipStream_t s = (hipStream_t)stream;
    const int cus = device_info().cus;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    HIP_TRY(hipEventCreate(&e0));
    hipError_t e = hipEventCreate(&e1);
    if (e == hipSuccess) e = launch_swap(a, b, n / 4, cus, cached != 0, s);       // warm-up
    if (e == hipSuccess) e = hipEventRecord(e0, s);
    for (int k = 0; k < reps && e == hipSuccess; ++k) e = launch_swap(a, b, n / 4, cus, cached != 0, s);
    if (e == hipSuccess) e = hipEventRecord(e1, s);
    if (e == hipSuccess) e = hipEventSynchronize(e1);
    float t = 0;
    if (e == hipSuccess) e = hipEventElapsedTime(&t, e0, e1);
    (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    if (e != hipSuccess) return fail(PIC_EDEVICE, "bandwidth probe: %s", hipGetErrorString(e));
    *ms = (double)t / reps;
    return PIC_OK;
}

extern "C" pic_status pic_diagnostics(pic_run *r, pic_diag *diag, double *rho_out, double *E_out,
                                      int32_t ng_cap) {
    pic_status st = check_run(r);
    if (st != PIC_OK) return st;
    if (!diag) return fail(PIC_EINVAL, "diag is NULL");
    if ((rho_out || E_out) && ng_cap < r->p.ng) return fail(PIC_EINVAL, "ng_cap < ng");
    st = sync_run(r);
    if (st != PIC_OK) return st;
    RunDev d;
    HIP_TRY(dev_read(r, &d, r->dev, sizeof d));
    diag->step = d.step;
    diag->time = (double)d.step * r->p.dt;
    diag->kinetic = d.kinetic_now;
    {
        // the field solve's per-wavefront sums of E^2, added in the same
        // order as the device adds them for the history
        double w = 0.0;
        for (int k = 0; k < kFieldParts; ++k) w += d.field_part[d.step & 1][k];
        diag->field = 0.5 * d.dx * w;
    }
    diag->momentum = d.momentum_now;
    diag->charge_fixed_sum = d.charge_now;
    diag->net_charge = r->p.rho0 * r->p.L + r->Q * ((double)d.charge_now / 4294967296.0);
    diag->flags = d.flags;
    diag->pad_ = 0;
    if (rho_out) {
        std::vector<unsigned long long> S((size_t)r->p.ng);
        HIP_TRY(dev_read(r, S.data(), r->host.S01[d.step & 1], S.size() * 8));
        const double qdx = r->Q / r->dx;
        for (int g = 0; g < r->p.ng; ++g)
            rho_out[g] = r->p.rho0 + qdx * ((double)S[g] / 4294967296.0);
    }
    if (E_out) HIP_TRY(dev_read(r, E_out, r->host.E64, (size_t)r->p.ng * 8));
    return PIC_OK;
}

extern "C" pic_status pic_read_raw(pic_run *r, void *u, void *w, int64_t cap) {
    pic_status st = check_run(r);
    if (st != PIC_OK) return st;
    if (cap < r->p.np) return fail(PIC_EINVAL, "cap %lld < np %lld", (long long)cap, (long long)r->p.np);
    st = sync_run(r);
    if (st != PIC_OK) return st;
    const size_t n = (size_t)r->p.np;
    const size_t bytes = n * r->lay.esize;
    if (u) {
        HIP_TRY(dev_read(r, u, r->cur_u(), bytes));
        // stored s = u + 1/2 with s >= 1/2: s - 1/2 is exact in either precision
        if (r->p.precision == PIC_FP32) {
            float *f = (float *)u;
            for (size_t i = 0; i < n; ++i) f[i] -= 0.5f;
        } else {
            double *d = (double *)u;
            for (size_t i = 0; i < n; ++i) d[i] -= 0.5;
        }
    }
    if (w) HIP_TRY(dev_read(r, w, r->cur_w(), bytes));
    return PIC_OK;
}

extern "C" pic_status pic_read_particles(pic_run *r, double *x, double *v, int64_t cap) {
    pic_status st = check_run(r);
    if (st != PIC_OK) return st;
    if (cap < r->p.np) return fail(PIC_EINVAL, "cap %lld < np %lld", (long long)cap, (long long)r->p.np);
    const size_t n = (size_t)r->p.np;
    const double vs = r->dx / r->p.dt;
    if (r->p.precision == PIC_FP32) {
        std::vector<float> u(n), w(n);
        st = pic_read_raw(r, u.data(), w.data(), cap);
        if (st != PIC_OK) return st;
        for (size_t i = 0; i < n; ++i) {
            if (x) x[i] = (double)u[i] * r->dx;
            if (v) v[i] = (double)w[i] * vs;
        }
    } else {
        std::vector<double> u(n), w(n);
        st = pic_read_raw(r, u.data(), w.data(), cap);
        if (st != PIC_OK) return st;
        for (size_t i = 0; i < n; ++i) {
            if (x) x[i] = u[i] * r->dx;
            if (v) v[i] = w[i] * vs;
        }
    }
    return PIC_OK;
}

extern "C" pic_status pic_read_grid(pic_run *r, int64_t *S, double *E, float *Ehat, int32_t cap) {
    pic_status st = check_run(r);
    if (st != PIC_OK) return st;
    if (cap < r->p.ng) return fail(PIC_EINVAL, "cap %d < ng %d", cap, r->p.ng);
    st = sync_run(r);
    if (st != PIC_OK) return st;
    const size_t ng = (size_t)r->p.ng;
    if (S) {
        int64_t steps = 0;                            // the latest deposit is in S01[steps & 1]
        HIP_TRY(dev_read(r, &steps, &r->dev->step, sizeof steps));
        HIP_TRY(dev_read(r, S, r->host.S01[steps & 1], ng * 8));
    }
    if (E) HIP_TRY(dev_read(r, E, r->host.E64, ng * 8));
    if (Ehat) HIP_TRY(dev_read(r, Ehat, r->host.Ehat, ng * 4));
    return PIC_OK;
}

namespace {

// Phase-space image of a run into host counts.  `fixed` is the device scratch
// to bin into (the allocation-free call), or null: then the call allocates
// its scratch and frees it again.
pic_status phase_space(pic_run *r, int32_t nx, int32_t nv, double vmin, double vmax, uint32_t *counts,
                       int64_t *outside, void *fixed) {
    pic_status st = check_run(r);
    if (st != PIC_OK) return st;
    if (!counts) return fail(PIC_EINVAL, "counts is NULL");
    if (nx < 1 || nv < 1 || (int64_t)nx * nv > kMaxPhaseBins)
        return fail(PIC_EINVAL, "need nx, nv >= 1 and nx nv <= %d (got %d x %d)", kMaxPhaseBins, nx, nv);
    if (!(std::isfinite(vmin) && std::isfinite(vmax) && vmin < vmax))
        return fail(PIC_EINVAL, "need finite vmin < vmax");
    st = sync_run(r);
    if (st != PIC_OK) return st;
    PhaseArgs a{};
    a.nx = nx;
    a.nv = nv;
    a.xs = (double)nx / (double)r->p.ng;
    const double c = r->p.dt / r->dx;
    a.w_lo = vmin * c;
    a.w_bin = (double)nv / ((vmax - vmin) * c);
    if (!(std::isfinite(a.w_lo) && std::isfinite(a.w_bin) && a.w_bin > 0))
        return fail(PIC_EINVAL, "velocity range too wide or too narrow for the bins");
    // The scratch: the outside counter, then the bins.
    const size_t nbins = (size_t)nx * nv;
    const size_t bytes = 8 + nbins * sizeof(uint32_t);
    void *buf = fixed;
    if (!buf) HIP_TRY(hipMalloc(&buf, bytes));
    unsigned long long *out_dev = (unsigned long long *)buf;
    unsigned *counts_dev = (unsigned *)((char *)buf + 8);
    unsigned long long out_host = 0;
    hipError_t e = launch_zero(buf, bytes, r->stream);
    if (e == hipSuccess)
        e = launch_phase(r->cur_u(), r->cur_w(), r->p.np, r->p.precision, a, counts_dev, out_dev,
                         device_info().cus, r->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(r->stream);
    if (e == hipSuccess) e = hipMemcpy(counts, counts_dev, nbins * sizeof(uint32_t), hipMemcpyDeviceToHost);
    if (e == hipSuccess) e = hipMemcpy(&out_host, out_dev, 8, hipMemcpyDeviceToHost);
    if (!fixed) {
        const hipError_t ef = hipFree(buf);
        if (e == hipSuccess) e = ef;
    }
    if (e != hipSuccess) {
        r->error = true;
        return fail(PIC_EDEVICE, "phase-space binning failed: %s", hipGetErrorString(e));
    }
    if (outside) *outside = (int64_t)out_host;
    return PIC_OK;
}

}  // namespace

extern "C" pic_status pic_phase_space(pic_run *r, int32_t nx, int32_t nv, double vmin, double vmax,
                                      uint32_t *counts, int64_t *outside) {
    return phase_space(r, nx, nv, vmin, vmax, counts, outside, nullptr);
}

extern "C" pic_status pic_phase_space_noalloc(pic_run *r, int32_t nx, int32_t nv, double vmin, double vmax,
                                              uint32_t *counts, int64_t *outside) {
    pic_status st = check_run(r);
    if (st != PIC_OK) return st;
    if (nx < 1 || nv < 1 || (int64_t)nx * nv > kMaxPhaseBins)
        return fail(PIC_EINVAL, "pic_phase_space_noalloc: nx nv = %lld exceeds its fixed scratch of %d bins",
                    (long long)nx * nv, kMaxPhaseBins);
    void *fixed = nullptr;
    const hipError_t e = phase_scratch(&fixed);
    if (e != hipSuccess)
        return fail(PIC_EDEVICE, "pic_phase_space_noalloc: scratch address: %s", hipGetErrorString(e));
    return phase_space(r, nx, nv, vmin, vmax, counts, outside, fixed);
}

extern "C" pic_status pic_read_history(pic_run *r, int64_t first, int64_t count, double *rows) {
    pic_status st = check_run(r);
    if (st != PIC_OK) return st;
    st = sync_run(r);
    if (st != PIC_OK) return st;
    RunDev d;
    HIP_TRY(dev_read(r, &d, r->dev, sizeof d));
    const int64_t avail = std::min<int64_t>(d.step, r->p.history_cap);
    if (first < 0 || count < 0 || first + count > avail)
        return fail(PIC_EINVAL, "history rows [%lld, %lld) outside the %lld available",
                    (long long)first, (long long)(first + count), (long long)avail);
    if (count == 0) return PIC_OK;
    if (!rows) return fail(PIC_EINVAL, "rows is NULL");
    HIP_TRY(dev_read(r, rows, r->host.hist + (size_t)first * kHistCols,
                      (size_t)count * kHistCols * 8));
    return PIC_OK;
}

extern "C" pic_status pic_destroy(pic_run *r) {
    if (!r) return PIC_OK;
    if (r->batch_member) return fail(PIC_ESTATE, "batch members are released with pic_batch_release");
    hipError_t e = hipStreamSynchronize(r->stream);
    if (r->graph) (void)hipGraphExecDestroy(r->graph);
    if (r->graph_sort) (void)hipGraphExecDestroy(r->graph_sort);
    if (r->owns_mem) (void)hipFree(r->base);
    delete r;
    if (e != hipSuccess) return fail(PIC_EDEVICE, "device error at destroy: %s", hipGetErrorString(e));
    return PIC_OK;
}

// ============================================================ batched engine

namespace {

// First-fit allocator over a device arena, 256-byte granules, coalescing.
class Arena {
  public:
    void reset(size_t bytes) {
        free_.clear();
        size_ = bytes / 256 * 256;
        if (size_) free_[0] = size_;
        used_ = 0;
    }
    bool alloc(size_t bytes, size_t *off) {
        bytes = align_up(std::max<size_t>(bytes, 1), 256);
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second >= bytes) {
                *off = it->first;
                size_t rest = it->second - bytes;
                size_t at = it->first + bytes;
                free_.erase(it);
                if (rest) free_[at] = rest;
                used_ += bytes;
                return true;
            }
        }
        return false;
    }
    void release(size_t off, size_t bytes) {
        bytes = align_up(std::max<size_t>(bytes, 1), 256);
        used_ -= bytes;
        auto it = free_.emplace(off, bytes).first;
        auto nx = std::next(it);
        if (nx != free_.end() && it->first + it->second == nx->first) {
            it->second += nx->second;
            free_.erase(nx);
        }
        if (it != free_.begin()) {
            auto pv = std::prev(it);
            if (pv->first + pv->second == it->first) {
                pv->second += it->second;
                free_.erase(it);
            }
        }
    }
    size_t used() const { return used_; }
    size_t size() const { return size_; }

  private:
    std::map<size_t, size_t> free_;
    size_t size_ = 0, used_ = 0;
};

struct Member {
    int64_t id;
    int slot;
    pic_run *run;          // view (descriptor lives in the batch's run table)
    size_t off, bytes;     // arena span
    int64_t nsteps;        // steps requested
    int64_t launch_done;   // batch launch index after which the run is complete
    int64_t admit_seq = 0; // completion mark recorded after its prologue
    int64_t admit_launch = 0;  // batch launches issued before it joined
    bool reported = false;
};

// Pinned host buffer that carries one admission's converted particles and
// descriptor to the device; reusable once `done` (recorded after the
// copies) has completed.
struct Staging {
    char *host = nullptr;
    size_t bytes = 0;
    hipEvent_t done = nullptr;
    bool busy = false;
};

constexpr size_t kStagingKeep = (size_t)1 << 30;   // idle pinned bytes kept for reuse

}  // namespace

struct pic_batch {
    pic_batch_config cfg{};
    hipStream_t stream = nullptr;
    hipStream_t io_stream = nullptr;  // reads of members (non-blocking, default priority)
    char *arena_base = nullptr;
    bool owns_arena = false;
    Arena arena;
    RunDev *table = nullptr;          // device run table [max_runs]
    WorkItem *items_dev = nullptr;    // device work list
    WorkQueue *queue_dev = nullptr;   // device work queue of the particle pass
    WorkItem *items_host = nullptr;   // pinned staging
    WorkQueue *queue_host = nullptr;
    // Slots the solve launch covers: the unfinished members' slots in slot
    // order, padded with -1 to nsolve, a power of two (so that a captured
    // graph changes only when that bucket does, not at every arrival).
    int32_t *slots_dev = nullptr;
    int32_t *slots_host = nullptr;    // pinned staging
    int nsolve = 1;
    hipEvent_t staged = nullptr;      // staging buffers free again
    int item_cap = 0;
    int grid = 0, grid_max = 0, cus = 256;
    LaunchShape shape;
    bool shape_forced = false, autotune = true;
    std::string tuned_key;                 // size class the shape was chosen for
    std::vector<int> free_slots;
    std::map<int64_t, Member> members;
    int64_t next_id = 1;
    int64_t launches = 0;             // batch step launches issued
    bool dirty = true;                // work list needs a rebuild
    // Captured step graphs, one per solve-launch size (nsolve): switching
    // between sizes as runs come and go replays a graph captured before.
    std::map<int, hipGraphExec_t> graphs;
    // Completion marks: events recorded on the batch stream after launches
    // and admissions, in order; `seq` numbers them.
    struct Mark {
        int64_t launches, seq;
        hipEvent_t ev;
    };
    std::vector<Mark> marks;
    int64_t mark_seq = 0;             // marks recorded
    int64_t seq_complete = 0;         // marks known complete
    int64_t launches_complete = 0;
    std::vector<Staging> staging;     // admission staging pool
    RunDev *idle_host = nullptr;      // pinned idle descriptor (copied into released slots)
    bool error = false;
};

namespace {

// Persistent workgroups of the batch's particle pass for a launch shape: the
// configured count, else every CU at the shape's occupancy.
int batch_grid(const pic_batch *b, const LaunchShape &s) {
    return b->cfg.grid_blocks > 0 ? b->cfg.grid_blocks : b->cus * step_occupancy(s, b->cfg.ng_max, PIC_FP32);
}

pic_status batch_check(pic_batch *b) {
    if (!b) return fail(PIC_EINVAL, "batch is NULL");
    if (b->error) return fail(PIC_ESTATE, "batch is in an error state after a device error");
    return PIC_OK;
}

// Work list of the batched particle pass: each unfinished run is split into
// chunks (whole tiles, dealt round robin), listed largest first; the
// persistent workgroups take them in that order from the device queue,
// which balances the load as it goes (longest-processing-time first).
pic_status rebuild_schedule(pic_batch *b) {
    struct Chunk {
        int slot, tb, te, index, count;
        int64_t work;
        const pic_run *run;
        int stride;
    };
    std::vector<Chunk> chunks;
    int64_t total = 0;
    for (auto &kv : b->members) {
        const Member &m = kv.second;
        if (m.launch_done <= b->launches) continue;   // finished: no work
        total += m.run->p.np;
    }
    const int64_t target = std::max<int64_t>(1, total / std::max(1, 2 * b->grid));
    // at least a tile for every wavefront of the workgroup that takes a chunk
    const int min_tiles = std::max(1, b->shape.block / 64);
    // A run's chunks: about `target` particles each (so that the queue
    // balances the launch), never fewer tiles than wavefronts per workgroup
    // (so that small batches keep every wavefront busy).  A run with tiles
    // enough for max(kFrontChunks, its share by size) chunks of a tile per
    // wavefront or more gets that many, and its tiles are dealt to its K chunks round
    // robin (chunk c: tiles c, c + K, ...); the K chunks sit together in the
    // list, so the K workgroups that take them sweep the run side by side:
    // HBM serves such a front faster than workgroups that each stream a
    // block of their own.  Other runs are cut into chunks of consecutive
    // tiles.
    constexpr int kFrontChunks = 8;
    for (auto &kv : b->members) {
        const Member &m = kv.second;
        if (m.launch_done <= b->launches) continue;
        const int tile = m.run->lay.tile, nt = m.run->lay.ntiles;
        const int64_t by_size = (m.run->p.np + target - 1) / target;
        const int64_t K = std::max<int64_t>(by_size, kFrontChunks);
        if ((int64_t)nt >= K * min_tiles) {
            for (int c = 0; c < (int)K; ++c)
                chunks.push_back({m.slot, c, nt, c, (int)K, m.run->p.np / K + 4 * m.run->p.ng, m.run, (int)K});
            continue;
        }
        const int per = (int)std::max<int64_t>(min_tiles, (target + tile - 1) / tile);
        const int count = (nt + per - 1) / per;
        for (int c = 0, t0 = 0; t0 < nt; ++c, t0 += per) {
            const int t1 = std::min(nt, t0 + per);
            // particles of tiles [t0, t1): whole tiles except the run's last
            const int64_t w = std::min<int64_t>((int64_t)t1 * tile, m.run->p.np) - (int64_t)t0 * tile;
            chunks.push_back({m.slot, t0, t1, c, count, w + 4 * m.run->p.ng, m.run, 1});
        }
    }
    if ((int)chunks.size() > b->item_cap)
        return fail(PIC_ENOMEM, "work list of %zu chunks exceeds capacity %d", chunks.size(), b->item_cap);
    std::sort(chunks.begin(), chunks.end(), [](const Chunk &a, const Chunk &c) {
        if (a.work != c.work) return a.work > c.work;
        if (a.slot != c.slot) return a.slot < c.slot;
        return a.tb < c.tb;
    });
    HIP_TRY(hipEventSynchronize(b->staged));
    // the solve launch's slot list
    int nact = 0;
    for (auto &kv : b->members)
        if (kv.second.launch_done > b->launches) b->slots_host[nact++] = kv.second.slot;
    std::sort(b->slots_host, b->slots_host + nact);
    int bucket = 1;
    while (bucket < nact) bucket <<= 1;
    for (int k = nact; k < bucket; ++k) b->slots_host[k] = -1;
    b->nsolve = bucket;                                // selects the graph with that solve grid
    HIP_TRY(hipMemcpyAsync(b->slots_dev, b->slots_host, sizeof(int32_t) * (size_t)bucket, hipMemcpyHostToDevice,
                           b->stream));
    const int n = (int)chunks.size();
    for (int k = 0; k < n; ++k) {
        const Chunk &c = chunks[(size_t)k];
        b->items_host[k] = {c.slot, c.tb, c.te, c.index, c.count, c.run->p.ng, c.stride, 0, gather_table_of(c.run)};
    }
    // The previous launch left next = 0; this copy is ordered after it.
    *b->queue_host = WorkQueue{0u, (uint32_t)n, {0u, 0u}};
    HIP_TRY(hipMemcpyAsync(b->queue_dev, b->queue_host, sizeof(WorkQueue), hipMemcpyHostToDevice, b->stream));
    if (n) HIP_TRY(hipMemcpyAsync(b->items_dev, b->items_host, sizeof(WorkItem) * (size_t)n,
                                  hipMemcpyHostToDevice, b->stream));
    HIP_TRY(hipEventRecord(b->staged, b->stream));
    b->dirty = false;
    return PIC_OK;
}

int64_t next_completion(const pic_batch *b) {
    int64_t best = INT64_MAX;
    for (auto &kv : b->members)
        if (kv.second.launch_done > b->launches) best = std::min(best, kv.second.launch_done);
    return best;
}

// Cell sorts of batch members: a member that sorts every K steps is sorted
// before its steps K+1, 2K+1, ... (counted from its admission), i.e. before
// the batch launch that follows launch admit_launch + nK.
bool member_sort_due(const Member &m, int64_t launches) {
    const int k = m.run->sort_every();
    const int64_t n = launches - m.admit_launch;
    return k > 0 && n > 0 && n % k == 0 && launches < m.launch_done;
}

// Batch launch count of the next sort point after `launches` (INT64_MAX if none).
int64_t next_sort_point(const pic_batch *b) {
    int64_t best = INT64_MAX;
    for (auto &kv : b->members) {
        const Member &m = kv.second;
        const int k = m.run->sort_every();
        if (k <= 0 || m.launch_done <= b->launches) continue;
        const int64_t n = b->launches - m.admit_launch;
        const int64_t at = m.admit_launch + (n / k + 1) * k;
        if (at < m.launch_done) best = std::min(best, at);
    }
    return best;
}

pic_status enqueue_member_sorts(pic_batch *b) {
    for (auto &kv : b->members) {
        Member &m = kv.second;
        if (!member_sort_due(m, b->launches)) continue;
        pic_run *r = m.run;
        hipError_t e = launch_sort(r->dev, r->p.np, r->p.ng, PIC_FP32, r->host.sort_scratch, b->stream);
        if (e != hipSuccess) {
            b->error = true;
            return fail(PIC_EDEVICE, "cell sort launch failed: %s", hipGetErrorString(e));
        }
        r->swapped = !r->swapped;
    }
    return PIC_OK;
}

// One batch step (particle pass, then the solve launch over the active
// slots) on `stream`.
hipError_t batch_launch(const pic_batch *b, hipStream_t stream, const StepEvents *ev = nullptr) {
    return launch_step(b->table, b->items_dev, b->queue_dev, nullptr, b->grid, b->shape, b->cfg.ng_max, PIC_FP32, 0,
                       b->slots_dev, b->nsolve, stream, ev);
}

pic_status ensure_graph(pic_batch *b) {
    if (b->cfg.graph_steps <= 1 || b->graphs.count(b->nsolve)) return PIC_OK;
    const pic_batch *bc = b;
    hipGraphExec_t exec = nullptr;
    pic_status st = capture_graph([bc](hipStream_t s) { return batch_launch(bc, s); }, b->cfg.graph_steps, &exec);
    if (st == PIC_OK) b->graphs[b->nsolve] = exec;
    return st;
}

pic_status add_mark(pic_batch *b) {
    hipEvent_t ev;
    HIP_TRY(hipEventCreateWithFlags(&ev, hipEventDisableTiming));
    HIP_TRY(hipEventRecord(ev, b->stream));
    b->marks.push_back({b->launches, ++b->mark_seq, ev});
    return PIC_OK;
}

void harvest_marks(pic_batch *b) {
    size_t k = 0;
    for (; k < b->marks.size(); ++k) {
        hipError_t q = hipEventQuery(b->marks[k].ev);
        if (q == hipErrorNotReady) break;
        if (q != hipSuccess) {
            b->error = true;
            break;
        }
        b->launches_complete = std::max(b->launches_complete, b->marks[k].launches);
        b->seq_complete = b->marks[k].seq;
        (void)hipEventDestroy(b->marks[k].ev);
    }
    b->marks.erase(b->marks.begin(), b->marks.begin() + (long)k);
}

void reap_staging(pic_batch *b) {
    for (Staging &g : b->staging)
        if (g.busy && hipEventQuery(g.done) == hipSuccess) g.busy = false;
}

// Index of an idle staging buffer of at least `need` bytes, allocating one
// (power-of-two size, >= 1 MiB) when none is free.  Idle buffers beyond
// kStagingKeep bytes are returned to the system first.
pic_status get_staging(pic_batch *b, size_t need, size_t *index) {
    reap_staging(b);
    size_t best = SIZE_MAX;
    for (size_t i = 0; i < b->staging.size(); ++i) {
        const Staging &g = b->staging[i];
        if (!g.busy && g.bytes >= need && (best == SIZE_MAX || g.bytes < b->staging[best].bytes)) best = i;
    }
    if (best != SIZE_MAX) {
        *index = best;
        return PIC_OK;
    }
    size_t idle = 0;
    for (const Staging &g : b->staging)
        if (!g.busy) idle += g.bytes;
    for (size_t i = 0; i < b->staging.size() && idle + need > kStagingKeep;) {
        Staging &g = b->staging[i];
        if (g.busy) {
            ++i;
            continue;
        }
        idle -= g.bytes;
        (void)hipHostFree(g.host);
        (void)hipEventDestroy(g.done);
        b->staging.erase(b->staging.begin() + (long)i);
    }
    Staging g;
    g.bytes = (size_t)1 << 20;
    while (g.bytes < need) g.bytes <<= 1;
    if (hipHostMalloc((void **)&g.host, g.bytes) != hipSuccess)
        return fail(PIC_ENOMEM, "pinned staging buffer of %zu bytes", g.bytes);
    if (hipEventCreateWithFlags(&g.done, hipEventDisableTiming) != hipSuccess) {
        (void)hipHostFree(g.host);
        return fail(PIC_EDEVICE, "event creation failed");
    }
    b->staging.push_back(g);
    *index = b->staging.size() - 1;
    return PIC_OK;
}

}  // namespace

extern "C" pic_status pic_batch_create(const pic_batch_config *cfg, void *stream, pic_batch **out) {
    if (!cfg || !out) return fail(PIC_EINVAL, "cfg and out must not be NULL");
    *out = nullptr;
    if (cfg->max_runs < 1 || cfg->max_runs > 65536) return fail(PIC_EINVAL, "max_runs must be in [1, 65536]");
    if (cfg->ng_max < 2 || cfg->ng_max > PIC_MAX_NG) return fail(PIC_EINVAL, "ng_max must be in [2, %d]", PIC_MAX_NG);
    if (cfg->graph_steps < 0 || cfg->graph_steps > 4096) return fail(PIC_EINVAL, "graph_steps must be in [0, 4096]");
    if (cfg->hbm_budget < 4096) return fail(PIC_EINVAL, "hbm_budget too small");
    if (cfg->arena && (uintptr_t)cfg->arena % 256) return fail(PIC_EINVAL, "arena must be 256-byte aligned");
    pic_batch *b = new pic_batch();
    b->cfg = *cfg;
    b->stream = (hipStream_t)stream;
    DeviceInfo d = device_info();
    b->shape = d.shape;
    b->shape_forced = d.forced || cfg->grid_blocks > 0;
    b->autotune = d.autotune;
    b->cus = d.cus;
    hipError_t e = step_prepare(b->shape, PIC_FP32);
    if (e == hipSuccess) e = sort_prepare();
    if (e != hipSuccess) {
        delete b;
        return fail(PIC_EDEVICE, "kernel setup: %s", hipGetErrorString(e));
    }
    const int occ = step_occupancy(b->shape, cfg->ng_max, PIC_FP32);
    b->grid = cfg->grid_blocks > 0 ? cfg->grid_blocks : d.cus * occ;
    b->grid_max = std::max(b->grid, d.cus * 16);      // room for any tuned shape
    b->item_cap = 4 * b->grid_max + 16 * cfg->max_runs;
    bool ok = true;
    if (cfg->arena) {
        b->arena_base = (char *)cfg->arena;
    } else {
        ok = hipMalloc((void **)&b->arena_base, cfg->hbm_budget) == hipSuccess;
        b->owns_arena = ok;
    }
    ok = ok && hipMalloc((void **)&b->table, sizeof(RunDev) * (size_t)cfg->max_runs) == hipSuccess;
    ok = ok && hipMalloc((void **)&b->items_dev, sizeof(WorkItem) * (size_t)b->item_cap) == hipSuccess;
    ok = ok && hipMalloc((void **)&b->queue_dev, sizeof(WorkQueue)) == hipSuccess;
    ok = ok && hipHostMalloc((void **)&b->items_host, sizeof(WorkItem) * (size_t)b->item_cap) == hipSuccess;
    ok = ok && hipHostMalloc((void **)&b->queue_host, sizeof(WorkQueue)) == hipSuccess;
    // the slot list is padded to a power of two: room for the next one up
    size_t slot_cap = 1;
    while (slot_cap < (size_t)cfg->max_runs) slot_cap <<= 1;
    ok = ok && hipMalloc((void **)&b->slots_dev, sizeof(int32_t) * slot_cap) == hipSuccess;
    ok = ok && hipHostMalloc((void **)&b->slots_host, sizeof(int32_t) * slot_cap) == hipSuccess;
    ok = ok && hipEventCreateWithFlags(&b->staged, hipEventDisableTiming) == hipSuccess;
    ok = ok && hipHostMalloc((void **)&b->idle_host, sizeof(RunDev)) == hipSuccess;
    ok = ok && hipStreamCreateWithFlags(&b->io_stream, hipStreamNonBlocking) == hipSuccess;
    if (!ok) {
        pic_batch_destroy(b);
        return fail(PIC_ENOMEM, "batch allocation failed");
    }
    b->arena.reset(cfg->hbm_budget);
    for (int s = cfg->max_runs - 1; s >= 0; --s) b->free_slots.push_back(s);
    {
        // Every slot starts idle (step == step_target): the solve launch
        // covers all slots and returns at once for idle ones.
        std::vector<RunDev> idle((size_t)cfg->max_runs);
        for (RunDev &d : idle) {
            d = RunDev{};
            d.ng = 2;
        }
        *b->idle_host = idle[0];
        if (hipMemcpy(b->table, idle.data(), sizeof(RunDev) * idle.size(), hipMemcpyHostToDevice) !=
            hipSuccess) {
            pic_batch_destroy(b);
            return fail(PIC_EDEVICE, "run table initialisation failed");
        }
    }
    if (hipEventRecord(b->staged, b->stream) != hipSuccess) {
        pic_batch_destroy(b);
        return fail(PIC_EDEVICE, "event record failed");
    }
    pic_status st = rebuild_schedule(b);
    if (st != PIC_OK) {
        std::string msg = g_err;
        pic_batch_destroy(b);
        g_err = msg;
        return st;
    }
    *out = b;
    return PIC_OK;
}

namespace {

// Admission: host particles (x0, v_mhalf) converted into pinned staging and
// uploaded, or (ld) drawn on the device; then grid clearing, descriptor and
// the initial deposit and solve, all queued on the batch stream.
pic_status admit_run(pic_batch *b, const pic_params *params, const double *x0, const double *v_mhalf,
                     const LoaderArgs *ld, int64_t nsteps, int64_t *run_id) {
    pic_status st = batch_check(b);
    if (st != PIC_OK) return st;
    st = validate(params);
    if (st != PIC_OK) return st;
    if (!run_id) return fail(PIC_EINVAL, "run_id is NULL");
    if (nsteps < 0) return fail(PIC_EINVAL, "nsteps must be >= 0");
    if (params->precision != PIC_FP32) return fail(PIC_EINVAL, "batched runs use PIC_FP32 state");
    if (params->sort_every == PIC_SORT_AUTO)
        return fail(PIC_EINVAL, "batched runs take sort_every >= 0 (PIC_SORT_AUTO is for single runs)");
    if (params->ng > b->cfg.ng_max) return fail(PIC_EINVAL, "ng %d exceeds the batch's ng_max %d", params->ng, b->cfg.ng_max);
    if (b->free_slots.empty()) return fail(PIC_EBUDGET, "run table full (%d runs)", b->cfg.max_runs);
    if (!ld) {
        st = check_particles(params, x0, v_mhalf);
        if (st != PIC_OK) return st;
    }
    Layout lay = make_layout(params);
    size_t off = 0;
    if (!b->arena.alloc(lay.total, &off))
        return fail(PIC_EBUDGET, "run needs %zu bytes; arena has %zu of %zu in use", lay.total,
                    b->arena.used(), b->arena.size());
    pic_run *r = new pic_run();
    r->p = *params;
    r->lay = lay;
    r->stream = b->stream;
    r->io_stream = b->io_stream;
    r->base = b->arena_base + off;
    r->batch_member = true;
    r->shape = b->shape;
    const int slot = b->free_slots.back();
    b->free_slots.pop_back();
    r->dev = b->table + slot;
    fill_constants(r);
    carve(r);
    r->host.step_target = nsteps;
    r->grid = single_run_grid(r, r->shape, b->cus);
    // Convert into pinned staging and queue upload, grid clearing,
    // descriptor and prologue on the batch stream; the host does not wait.
    const size_t desc_bytes = kDescBytes;
    const size_t part_bytes = ld ? 0 : (size_t)params->np * lay.esize;
    size_t gi = 0;
    st = get_staging(b, desc_bytes + 2 * part_bytes, &gi);
    if (st == PIC_OK) {
        Staging &g = b->staging[gi];
        if (!ld) convert_particles(r, x0, v_mhalf, g.host + desc_bytes, g.host + desc_bytes + part_bytes);
        std::memcpy(g.host, &r->host, sizeof(RunDev));
        g.busy = true;   // from here on the buffer may be read by queued copies
        hipError_t e;
        if (ld) {
            e = launch_loader(r->host.u, r->host.w, params->np, params->ng, PIC_FP32, *ld, b->cus, b->stream);
        } else {
            e = hipMemcpyAsync(r->host.u, g.host + desc_bytes, part_bytes, hipMemcpyHostToDevice, b->stream);
            if (e == hipSuccess)
                e = hipMemcpyAsync(r->host.w, g.host + desc_bytes + part_bytes, part_bytes, hipMemcpyHostToDevice,
                                   b->stream);
        }
        if (e == hipSuccess) {
            st = queue_device_init(r, (const RunDev *)g.host);
            if (st != PIC_OK) e = hipErrorUnknown;
        }
        if (e == hipSuccess) e = hipEventRecord(g.done, b->stream);
        if (e != hipSuccess) {
            // work may be half queued on the stream: the batch cannot continue
            b->error = true;
            if (st == PIC_OK) st = fail(PIC_EDEVICE, "admission upload: %s", hipGetErrorString(e));
        }
    }
    if (st != PIC_OK) {
        std::string msg = g_err;
        if (!b->error) {
            b->arena.release(off, lay.total);
            b->free_slots.push_back(slot);
        }
        delete r;
        g_err = msg;
        return st;
    }
    Member m;
    m.id = b->next_id++;
    m.slot = slot;
    m.run = r;
    m.off = off;
    m.bytes = lay.total;
    m.nsteps = nsteps;
    m.launch_done = b->launches + nsteps;
    m.admit_launch = b->launches;
    st = add_mark(b);
    if (st != PIC_OK) {
        b->error = true;
        delete r;
        return st;
    }
    m.admit_seq = b->mark_seq;
    b->members[m.id] = m;
    b->dirty = true;
    *run_id = m.id;
    return PIC_OK;
}

}  // namespace

extern "C" pic_status pic_batch_admit(pic_batch *b, const pic_params *params, const double *x0,
                                      const double *v_mhalf, int64_t nsteps, int64_t *run_id) {
    return admit_run(b, params, x0, v_mhalf, nullptr, nsteps, run_id);
}

extern "C" pic_status pic_batch_admit_loaded(pic_batch *b, const pic_params *params, const pic_loader *loader,
                                             int64_t nsteps, int64_t *run_id) {
    pic_status st = batch_check(b);
    if (st != PIC_OK) return st;
    st = validate(params);
    if (st != PIC_OK) return st;
    st = check_loader(params, loader);
    if (st != PIC_OK) return st;
    const LoaderArgs a = loader_args(params, loader);
    return admit_run(b, params, nullptr, nullptr, &a, nsteps, run_id);
}

namespace {

// Launch shape of the batch's particle pass for the current membership:
// cached or tuned per size class (largest grid, total particles); tuning
// runs particle passes on the members' own state and restores it.
pic_status batch_choose_shape(pic_batch *b) {
    if (b->shape_forced || !b->autotune) return PIC_OK;
    int64_t total = 0;
    std::vector<pic_run *> live;
    for (auto &kv : b->members)
        if (kv.second.launch_done > b->launches) {
            total += kv.second.run->p.np;
            live.push_back(kv.second.run);
        }
    if (live.empty()) return PIC_OK;
    const std::string key = tune_key("batch", PIC_FP32, b->cfg.ng_max, total);
    if (key == b->tuned_key) return PIC_OK;
    const int old_grid = b->grid;              // what the captured graph launches
    const LaunchShape old_shape = b->shape;
    LaunchShape shape = b->shape;
    if (!tune_lookup(key, &shape)) {
        size_t bytes = 0;
        for (pic_run *r : live) bytes += state_bytes(r);
        char *tmp = nullptr;
        if (hipMalloc((void **)&tmp, bytes) != hipSuccess)
            return fail(PIC_ENOMEM, "autotune scratch of %zu bytes", bytes);
        pic_status st = PIC_OK;
        size_t off = 0;
        for (pic_run *r : live) {
            if (st == PIC_OK) st = save_particles(r, tmp + off, false);
            off += state_bytes(r);
        }
        hipError_t te = hipSuccess;
        if (st == PIC_OK) {
            // the schedule depends on the shape (grid and chunk sizes): it is
            // rebuilt before each timed launch, outside the timing
            te = tune_shapes(
                key, PIC_FP32, false, b->stream,
                [b](const LaunchShape &s) {
                    b->shape = s;
                    b->grid = batch_grid(b, s);
                    return rebuild_schedule(b) == PIC_OK ? hipSuccess : hipErrorInvalidValue;
                },
                [b](const LaunchShape &s) {
                    return launch_particles(b->table, b->items_dev, b->queue_dev, nullptr, b->grid, s, b->cfg.ng_max,
                                            PIC_FP32, 0, b->stream);
                },
                &shape);
            off = 0;
            for (pic_run *r : live) {
                pic_status rs = save_particles(r, tmp + off, true);
                if (st == PIC_OK) st = rs;
                off += state_bytes(r);
            }
        }
        hipError_t se = hipStreamSynchronize(b->stream);
        (void)hipFree(tmp);
        if (st != PIC_OK) return st;
        if (te != hipSuccess) return fail(PIC_EDEVICE, "batch autotune: %s", hipGetErrorString(te));
        if (se != hipSuccess) return fail(PIC_EDEVICE, "batch autotune: %s", hipGetErrorString(se));
    }
    b->shape = shape;
    HIP_TRY(step_prepare(b->shape, PIC_FP32));
    b->grid = batch_grid(b, b->shape);
    b->tuned_key = key;
    // Tuning launches change the work list; the graph only has to go when
    // the launch itself (shape or grid) changed.
    b->dirty = true;
    if (b->grid != old_grid || old_shape.block != shape.block || old_shape.unroll != shape.unroll) {
        for (auto &g : b->graphs) (void)hipGraphExecDestroy(g.second);
        b->graphs.clear();
    }
    return PIC_OK;
}

// Advance the batch by up to `nsteps` launches.  With `evs`, no graph is used
// and each launch is bracketed by a StepEvents entry appended to *evs.
pic_status batch_advance(pic_batch *b, int64_t nsteps, std::vector<StepEvents> *evs) {
    int64_t left = nsteps;
    while (left > 0) {
        const int64_t nc = next_completion(b);
        if (nc == INT64_MAX) break;                      // nothing left to run
        if (b->dirty) {
            pic_status st = batch_choose_shape(b);
            if (st == PIC_OK) st = rebuild_schedule(b);
            if (st != PIC_OK) return st;
        }
        pic_status sst = enqueue_member_sorts(b);
        if (sst != PIC_OK) return sst;
        // launches before membership changes or the next cell sort
        int64_t k = std::min({left, nc - b->launches, next_sort_point(b) - b->launches});
        const int G = b->cfg.graph_steps;
        if (!evs && G > 1) {
            // captured on the first step call (also a short one), so later
            // calls only replay
            pic_status st = ensure_graph(b);
            if (st != PIC_OK) return st;
        }
        if (!evs && G > 1 && k >= G) {
            while (k >= G) {
                HIP_TRY(hipGraphLaunch(b->graphs.at(b->nsolve), b->stream));
                b->launches += G;
                left -= G;
                k -= G;
            }
        }
        for (; k > 0; --k, --left) {
            const StepEvents *ev = nullptr;
            if (evs) {
                StepEvents e{};
                HIP_TRY(hipEventCreate(&e.e0));
                HIP_TRY(hipEventCreate(&e.e1));
                HIP_TRY(hipEventCreate(&e.e2));
                evs->push_back(e);
                ev = &evs->back();
            }
            hipError_t le = batch_launch(b, b->stream, ev);
            if (le != hipSuccess) {
                b->error = true;
                return fail(PIC_EDEVICE, "batch step launch failed: %s", hipGetErrorString(le));
            }
            b->launches += 1;
        }
        if (b->launches >= nc) b->dirty = true;          // some run just finished
        pic_status st = add_mark(b);
        if (st != PIC_OK) return st;
    }
    return PIC_OK;
}

}  // namespace

extern "C" pic_status pic_batch_step(pic_batch *b, int64_t nsteps) {
    pic_status st = batch_check(b);
    if (st != PIC_OK) return st;
    if (nsteps < 0) return fail(PIC_EINVAL, "nsteps must be >= 0");
    return batch_advance(b, nsteps, nullptr);
}

extern "C" pic_status pic_batch_step_profiled(pic_batch *b, int64_t nsteps, double *ms_particle,
                                              double *ms_solve) {
    pic_status st = batch_check(b);
    if (st != PIC_OK) return st;
    if (nsteps < 1) return fail(PIC_EINVAL, "nsteps must be >= 1");
    std::vector<StepEvents> evs;
    evs.reserve((size_t)nsteps);
    st = batch_advance(b, nsteps, &evs);
    hipError_t se = hipStreamSynchronize(b->stream);
    double a = 0, c = 0;
    for (auto &e : evs) {
        float t1 = 0, t2 = 0;
        if (st == PIC_OK && se == hipSuccess) {
            (void)hipEventElapsedTime(&t1, e.e0, e.e1);
            (void)hipEventElapsedTime(&t2, e.e1, e.e2);
        }
        a += t1;
        c += t2;
        (void)hipEventDestroy(e.e0);
        (void)hipEventDestroy(e.e1);
        (void)hipEventDestroy(e.e2);
    }
    if (st != PIC_OK) return st;
    if (se != hipSuccess) {
        b->error = true;
        return fail(PIC_EDEVICE, "device error: %s", hipGetErrorString(se));
    }
    if (evs.empty()) return fail(PIC_ESTATE, "no unfinished runs to step");
    if (ms_particle) *ms_particle = a / (double)evs.size();
    if (ms_solve) *ms_solve = c / (double)evs.size();
    return PIC_OK;
}

extern "C" pic_status pic_batch_poll(pic_batch *b, int64_t *done_ids, int32_t cap, int32_t *n_done) {
    pic_status st = batch_check(b);
    if (st != PIC_OK) return st;
    if (!n_done || (cap > 0 && !done_ids)) return fail(PIC_EINVAL, "bad output arguments");
    harvest_marks(b);
    reap_staging(b);
    if (b->error) return fail(PIC_EDEVICE, "device error in batch work");
    int32_t n = 0;
    for (auto &kv : b->members) {
        Member &m = kv.second;
        // complete: its last launch and its admission (prologue) have run
        if (m.reported || m.launch_done > b->launches_complete || m.admit_seq > b->seq_complete) continue;
        if (n >= cap) break;
        done_ids[n++] = m.id;
        m.reported = true;
        m.run->settled = true;
    }
    *n_done = n;
    return PIC_OK;
}

extern "C" pic_status pic_batch_run(pic_batch *b, int64_t run_id, pic_run **view) {
    pic_status st = batch_check(b);
    if (st != PIC_OK) return st;
    if (!view) return fail(PIC_EINVAL, "view is NULL");
    auto it = b->members.find(run_id);
    if (it == b->members.end()) return fail(PIC_EINVAL, "unknown run id %lld", (long long)run_id);
    *view = it->second.run;
    return PIC_OK;
}

extern "C" pic_status pic_batch_diagnostics(pic_batch *b, int64_t run_id, pic_diag *diag) {
    pic_run *view = nullptr;
    pic_status st = pic_batch_run(b, run_id, &view);
    if (st != PIC_OK) return st;
    if (!diag) return fail(PIC_EINVAL, "diag is NULL");
    st = pic_diagnostics(view, diag, nullptr, nullptr, 0);
    if (st == PIC_EDEVICE) b->error = true;
    return st;
}

extern "C" pic_status pic_batch_release(pic_batch *b, int64_t run_id) {
    if (!b) return fail(PIC_EINVAL, "batch is NULL");
    auto it = b->members.find(run_id);
    if (it == b->members.end()) return fail(PIC_EINVAL, "unknown run id %lld", (long long)run_id);
    if (b->error) return fail(PIC_ESTATE, "batch is in an error state after a device error");
    // No wait: everything that reads the slot or the arena span was queued
    // on the batch stream before anything that can reuse them.
    Member m = it->second;
    b->members.erase(it);
    // Park the slot: a descriptor whose step equals its target does no work.
    hipError_t e = hipMemcpyAsync(b->table + m.slot, b->idle_host, sizeof(RunDev), hipMemcpyHostToDevice,
                                  b->stream);
    delete m.run;
    if (e != hipSuccess) {
        b->error = true;
        return fail(PIC_EDEVICE, "release: %s", hipGetErrorString(e));
    }
    b->arena.release(m.off, m.bytes);
    b->free_slots.push_back(m.slot);
    b->dirty = true;
    return PIC_OK;
}

extern "C" pic_status pic_batch_usage(pic_batch *b, size_t *used, size_t *free_bytes, int32_t *nruns) {
    if (!b) return fail(PIC_EINVAL, "batch is NULL");
    if (used) *used = b->arena.used();
    if (free_bytes) *free_bytes = b->arena.size() - b->arena.used();
    if (nruns) *nruns = (int32_t)b->members.size();
    return PIC_OK;
}

extern "C" pic_status pic_batch_destroy(pic_batch *b) {
    if (!b) return PIC_OK;
    hipError_t e = hipStreamSynchronize(b->stream);
    for (auto &kv : b->members) delete kv.second.run;
    for (auto &mk : b->marks) (void)hipEventDestroy(mk.ev);
    for (Staging &g : b->staging) {
        (void)hipHostFree(g.host);
        (void)hipEventDestroy(g.done);
    }
    if (b->idle_host) (void)hipHostFree(b->idle_host);
    if (b->io_stream) (void)hipStreamDestroy(b->io_stream);
    for (auto &g : b->graphs) (void)hipGraphExecDestroy(g.second);
    if (b->staged) (void)hipEventDestroy(b->staged);
    if (b->items_host) (void)hipHostFree(b->items_host);
    if (b->queue_host) (void)hipHostFree(b->queue_host);
    if (b->slots_host) (void)hipHostFree(b->slots_host);
    if (b->slots_dev) (void)hipFree(b->slots_dev);
    if (b->items_dev) (void)hipFree(b->items_dev);
    if (b->queue_dev) (void)hipFree(b->queue_dev);
    if (b->table) (void)hipFree(b->table);
    if (b->owns_arena && b->arena_base) (void)hipFree(b->arena_base);
    delete b;
    if (e != hipSuccess) return fail(PIC_EDEVICE, "device error at destroy: %s", hipGetErrorString(e));
    return PIC_OK;
}
