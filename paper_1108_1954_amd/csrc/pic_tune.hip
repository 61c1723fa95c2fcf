// Launch-shape autotuner of the particle pass.
//
// The particle pass is timed with HIP events for every candidate shape
// (threads per workgroup x particle vectors per lane per iteration) on the
// caller's real state; the caller saves the particle arrays before and
// restores them after, so tuning leaves no trace in the results (which do
// not depend on the shape in any case: tiles and summation orders are fixed
// by the run alone).  Winners are cached per key (device, precision, grid
// size class, particle-count class) in memory and, when PIC1D_TUNE_CACHE
// names a file, across processes.
#include <hip/hip_runtime.h>

#include <cstdio>
#include <cstdlib>
#include <fstream>
#include <map>
#include <mutex>
#include <sstream>
#include <string>

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
        std::istringstream ls(line);
        std::string key;
        LaunchShape s;
        if (ls >> key >> s.block >> s.unroll) g_cache[key] = s;
    }
}

void append_file_locked(const std::string &key, const LaunchShape &s, double ms) {
    const char *path = cache_path();
    if (!path) return;
    std::ofstream out(path, std::ios::app);
    out << key << ' ' << s.block << ' ' << s.unroll << ' ' << ms << '\n';
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

hipError_t tune_shapes(const std::string &key, int precision, hipStream_t stream,
                       const std::function<hipError_t(const LaunchShape &)> &launch, LaunchShape *best) {
    // intermediate sizes: 640 threads fit two workgroups per CU at five
    // waves per SIMD, 768 one of twelve waves; each wins on some workloads
    static const int kBlocks[] = {256, 512, 640, 768, 1024};
    static const int kUnrolls[] = {1, 2, 4};
    constexpr int kReps = 3;
    hipEvent_t e0, e1;
    hipError_t err = hipEventCreate(&e0);
    if (err != hipSuccess) return err;
    if ((err = hipEventCreate(&e1)) != hipSuccess) {
        (void)hipEventDestroy(e0);
        return err;
    }
    double best_ms = 1e30;
    LaunchShape winner = *best;
    for (int blk : kBlocks) {
        for (int un : kUnrolls) {
            LaunchShape s;
            s.block = blk;
            s.unroll = un;
            if ((err = step_prepare(s, precision)) != hipSuccess) break;
            if ((err = launch(s)) != hipSuccess) break;           // warm-up
            if ((err = hipEventRecord(e0, stream)) != hipSuccess) break;
            for (int r = 0; r < kReps && err == hipSuccess; ++r) err = launch(s);
            if (err != hipSuccess) break;
            if ((err = hipEventRecord(e1, stream)) != hipSuccess) break;
            if ((err = hipEventSynchronize(e1)) != hipSuccess) break;
            float ms = 0;
            if ((err = hipEventElapsedTime(&ms, e0, e1)) != hipSuccess) break;
            if (ms / kReps < best_ms) {
                best_ms = ms / kReps;
                winner = s;
            }
        }
        if (err != hipSuccess) break;
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (err != hipSuccess) return err;
    *best = winner;
    std::lock_guard<std::mutex> g(g_mu);
    load_file_locked();
    g_cache[key] = winner;
    append_file_locked(key, winner, best_ms);
    return hipSuccess;
}

}  // namespace pic1d
