// Phase-space density of a run's particles (gfx950): the (x, v) plane of
// the paper's two-stream figure (Sec. 4), binned on the device so that a
// snapshot of 10^8 particles leaves the GPU as a small integer image.
//
// Bins, from the stored state s = x/dx + 1/2 and w = v dt/dx in FP64:
//   ix = floor((s - 1/2) xs),  xs = nx / ng, clamped to nx - 1;
//   y  = (w - w_lo) w_bin,     counted in row iv = floor(y) iff 0 <= y < nv,
// otherwise in `outside`.  s - 1/2 is exact, and each bin index comes from
// one subtraction and one product (no contraction), so a host holding the
// same state and constants finds the same bins.
#include <algorithm>
#include <mutex>
#include <unordered_map>

#include "pic_internal.h"

namespace pic1d {

// Device scratch of the allocation-free call (pic_phase_space_noalloc): the
// outside counter (8 bytes) and then up to kMaxPhaseBins 32-bit bins.  One
// copy per GPU, alive until the process ends; every call on a GPU shares it.
// Host code never passes this name to a kernel or a copy: it is a host-side
// stand-in, and the GPU address comes from phase_scratch().
static __device__ __align__(256) unsigned char scratch[kPhaseScratchBytes];

namespace {

std::mutex g_scratch_mu;
std::unordered_map<int, void *> g_scratch_ptr;   // device -> address of `scratch` there

__global__ __launch_bounds__(256) void zero_words(unsigned *__restrict__ p, int n) {
    for (int i = blockIdx.x * 256 + threadIdx.x; i < n; i += gridDim.x * 256) p[i] = 0u;
}

template <typename T>
__global__ __launch_bounds__(256) void phase_kernel(const T *__restrict__ U, const T *__restrict__ W, int64_t np,
                                                    PhaseArgs a, unsigned *__restrict__ counts,
                                                    unsigned long long *__restrict__ outside) {
#pragma clang fp contract(off)
    extern __shared__ unsigned hist[];
    const int nbins = a.nx * a.nv;
    for (int b = threadIdx.x; b < nbins; b += blockDim.x) hist[b] = 0;
    __syncthreads();
    const double nvf = (double)a.nv;
    unsigned out = 0;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < np; i += stride) {
        const double u = (double)U[i] - 0.5;
        const double y = ((double)W[i] - a.w_lo) * a.w_bin;
        if (y >= 0.0 && y < nvf) {
            const int ix = min((int)(u * a.xs), a.nx - 1);
            atomicAdd(&hist[(int)y * a.nx + ix], 1u);
        } else {
            ++out;
        }
    }
    __syncthreads();
    for (int b = threadIdx.x; b < nbins; b += blockDim.x)
        if (hist[b]) atomicAdd(&counts[b], hist[b]);
    for (int off = 32; off > 0; off >>= 1) out += __shfl_xor(out, off);
    if ((threadIdx.x & 63) == 0 && out) atomicAdd(outside, (unsigned long long)out);
}

}  // namespace

hipError_t phase_scratch(void **out) {
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    auto it = g_scratch_ptr.find(dev);
    if (it == g_scratch_ptr.end()) {
        void *p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        if (!p) return hipErrorInvalidSymbol;
        it = g_scratch_ptr.emplace(dev, p).first;
    }
    *out = it->second;
    return hipSuccess;
}

hipError_t launch_zero(void *p, size_t bytes, hipStream_t stream) {
    if (!p || bytes % 4 != 0) return hipErrorInvalidValue;
    const int n = (int)(bytes / 4);
    if (n == 0) return hipSuccess;
    const int grid = std::min(64, (n + 255) / 256);
    unsigned *w = (unsigned *)p;
    void *args[] = {&w, (void *)&n};
    return hipLaunchKernel((const void *)zero_words, dim3(grid), dim3(256), args, 0, stream);
}

hipError_t launch_phase(const void *u, const void *w, int64_t np, int precision, const PhaseArgs &a,
                        unsigned *counts, unsigned long long *outside, int cus, hipStream_t stream) {
    const int nbins = a.nx * a.nv;
    if (np < 1 || a.nx < 1 || a.nv < 1 || nbins > kMaxPhaseBins || !u || !w || !counts || !outside)
        return hipErrorInvalidValue;
    const int grid = (int)std::min<int64_t>((np + 255) / 256, (int64_t)cus * 8);
    const size_t lds = (size_t)nbins * sizeof(unsigned);
    PhaseArgs args_copy = a;
    void *args[] = {(void *)&u, (void *)&w, (void *)&np, (void *)&args_copy, (void *)&counts, (void *)&outside};
    const void *fn = precision ? (const void *)phase_kernel<double> : (const void *)phase_kernel<float>;
    return hipLaunchKernel(fn, dim3(grid), dim3(256), args, lds, stream);
}

}  // namespace pic1d
