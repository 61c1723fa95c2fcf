// Launch-shape autotuner of the particle pass.
//
// The particle pass is timed with HIP events for every candidate shape
// (threads per workgroup x particle vectors per lane per iteration x the
// cache policy of the particle accesses, and for single runs x the order in
// which workgroups take tiles) on the caller's real state, five launches
// each, interleaved across candidates, each timed launch right after an
// untimed one of the same candidate (so a cached candidate finds the caches
// as its own steps leave them), and scored by the median; the incumbent
// shape stays unless another is at
// least 2% faster; the caller saves the particle arrays before and
// restores them after, so tuning leaves no trace in the results (which do
// not depend on the shape in any case: tiles and summation orders are fixed
// by the run alone).  Winners are cached per key (device, precision, grid
// size class, particle-count class) in memory and, when PIC1D_TUNE_CACHE
// names a file, across processes.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdio>
#include <cstdlib>
#include <fstream>
#include <map>
#include <mutex>
#include <sstream>
#include <string>
#include <vector>

#include "pic_internal.h"

namespace pic1d {

namespace {

std::mutex g_mu;
std::map<std::string, LaunchShape> g_cache;
bool g_loaded = false;

const char *cache_path() { return getenv("PIC1D_TUNE_CACHE"); }

void load_file_locked() {
    if (g_loaded) return;
    g_loaded = true;
    const char *path = cache_path();
    if (!path) return;
    std::ifstream in(path);
    std::string line;
    while (std::getline(in, line)) {
        // key block unroll order cached ms: lines of another form are skipped
        std::istringstream ls(line);
        std::string key, extra;
        LaunchShape s;
        double ms = 0;
        if ((ls >> key >> s.block >> s.unroll >> s.order >> s.cached >> ms) && !(ls >> extra))
            g_cache[key] = s;
    }
}

void append_file_locked(const std::string &key, const LaunchShape &s, double ms) {
    const char *path = cache_path();
    if (!path) return;
    std::ofstream out(path, std::ios::app);
    out << key << ' ' << s.block << ' ' << s.unroll << ' ' << s.order << ' ' << s.cached << ' ' << ms << '\n';
}

int log2_ceil(int64_t v) {
    int b = 0;
    while (((int64_t)1 << b) < v && b < 62) ++b;
    return b;
}

}  // namespace

std::string tune_key(const char *kind, int precision, int ng, int64_t np) {
    static std::string dev;
    if (dev.empty()) {
        int d = 0;
        hipDeviceProp_t prop;
        if (hipGetDevice(&d) == hipSuccess && hipGetDeviceProperties(&prop, d) == hipSuccess)
            dev = std::string(prop.gcnArchName) + "-" + std::to_string(prop.multiProcessorCount) + "cu";
        else
            dev = "unknown";
        for (char &c : dev)
            if (c == ' ' || c == ':') c = '_';
    }
    std::ostringstream k;
    k << dev << '|' << kind << "|p" << precision << "|ng" << log2_ceil(ng) << "|np" << log2_ceil(np);
    return k.str();
}

bool tune_lookup(const std::string &key, LaunchShape *out) {
    std::lock_guard<std::mutex> g(g_mu);
    load_file_locked();
    auto it = g_cache.find(key);
    if (it == g_cache.end()) return false;
    *out = it->second;
    return true;
}

hipError_t tune_shapes(const std::string &key, int precision, bool orders, hipStream_t stream,
                       const std::function<hipError_t(const LaunchShape &)> &prepare,
                       const std::function<hipError_t(const LaunchShape &)> &launch, LaunchShape *best) {
    // intermediate sizes: 640 threads fit two workgroups per CU at five
    // waves per SIMD, 768 one of twelve waves; each wins on some workloads
    static const int kBlocks[] = {256, 512, 640, 768, 1024};
    static const int kUnrolls[] = {1, 2, 4};
    constexpr int kMaxCand = 60;                      // x 2 cache policies x 2 tile orders (single runs)
    constexpr int kRounds = 5;
    // A challenger must beat the incumbent (the shape passed in) by this
    // fraction of its time: shapes within noise of each other do not flip
    // from one process to the next.
    constexpr double kMargin = 0.02;
    LaunchShape cand[kMaxCand];
    int nc = 0;
    for (int cached = 0; cached < 2; ++cached)
        for (int ord = 0; ord < (orders ? 2 : 1); ++ord)
            for (int blk : kBlocks)
                for (int un : kUnrolls) {
                    cand[nc].block = blk;
                    cand[nc].unroll = un;
                    cand[nc].order = ord;
                    cand[nc].cached = cached;
                    ++nc;
                }
    const int kCand = nc;
    hipEvent_t ev[2 * kMaxCand] = {};
    hipError_t err = hipSuccess;
    for (int i = 0; i < 2 * kCand && err == hipSuccess; ++i) err = hipEventCreate(&ev[i]);
    std::vector<float> t((size_t)kCand * kRounds, 0.0f);
    // round 0 warms every candidate up; in rounds 1..kRounds the second of
    // each candidate's two launches is timed, on its own, the candidates
    // interleaved so that drift of the device's clocks affects them alike;
    // prepare() runs outside the timing
    for (int round = 0; round <= kRounds && err == hipSuccess; ++round) {
        for (int c = 0; c < kCand && err == hipSuccess; ++c) {
            if ((err = step_prepare(cand[c], precision)) != hipSuccess) break;
            if ((err = prepare(cand[c])) != hipSuccess) break;
            if ((err = launch(cand[c])) != hipSuccess) break;
            if (round > 0 && (err = hipEventRecord(ev[2 * c], stream)) != hipSuccess) break;
            if ((err = launch(cand[c])) != hipSuccess) break;
            if (round > 0 && (err = hipEventRecord(ev[2 * c + 1], stream)) != hipSuccess) break;
            if (round > 0) {
                if ((err = hipEventSynchronize(ev[2 * c + 1])) != hipSuccess) break;
                float ms = 0;
                if ((err = hipEventElapsedTime(&ms, ev[2 * c], ev[2 * c + 1])) != hipSuccess) break;
                t[(size_t)c * kRounds + (round - 1)] = ms;
            }
        }
    }
    for (hipEvent_t e : ev)
        if (e) (void)hipEventDestroy(e);
    if (err != hipSuccess) return err;
    double med[kMaxCand];
    int incumbent = -1, fastest = 0;
    for (int c = 0; c < kCand; ++c) {
        std::vector<float> v(t.begin() + (long)c * kRounds, t.begin() + (long)(c + 1) * kRounds);
        std::sort(v.begin(), v.end());
        med[c] = v[kRounds / 2];
        if (cand[c].block == best->block && cand[c].unroll == best->unroll && cand[c].order == best->order &&
            cand[c].cached == best->cached)
            incumbent = c;
        if (med[c] < med[fastest]) fastest = c;
    }
    int pick = fastest;
    if (incumbent >= 0 && !(med[fastest] < (1.0 - kMargin) * med[incumbent])) pick = incumbent;
    *best = cand[pick];
    std::lock_guard<std::mutex> g(g_mu);
    load_file_locked();
    g_cache[key] = cand[pick];
    append_file_locked(key, cand[pick], med[pick]);
    return hipSuccess;
}

}  // namespace pic1d
