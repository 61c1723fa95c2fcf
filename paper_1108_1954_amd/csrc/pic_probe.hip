// Achievable-bandwidth reference for the particle pass (gfx950).
//
// The particle pass reads two FP32 arrays and writes both back in place,
// 16 bytes per particle per step.  This kernel moves exactly those bytes with
// nothing else: it swaps the contents of two device arrays with 16-byte
// loads and stores, non-temporal or ordinary cached ones (the pass's two
// cache policies), four vectors per lane in flight, grid-stride over all
// CUs.  Its rate is the bandwidth that this access pattern can reach on the
// device, the reference the pass's roofline fraction is read against.  It
// computes nothing of the method.
#include <algorithm>

#include "pic_internal.h"

namespace pic1d {

namespace {

#define GLOBAL_AS __attribute__((address_space(1)))
typedef float f32x4 __attribute__((ext_vector_type(4)));

constexpr int kProbeBlock = 256;
constexpr int kProbeUnroll = 4;

template <bool NT>
__device__ __forceinline__ f32x4 probe_load(const f32x4 *p) {
    if constexpr (NT) return __builtin_nontemporal_load((const GLOBAL_AS f32x4 *)p);
    else return *(const GLOBAL_AS f32x4 *)p;
}
template <bool NT>
__device__ __forceinline__ void probe_store(f32x4 *p, f32x4 v) {
    if constexpr (NT) __builtin_nontemporal_store(v, (GLOBAL_AS f32x4 *)p);
    else *(GLOBAL_AS f32x4 *)p = v;
}

template <bool NT>
__global__ __launch_bounds__(kProbeBlock) void swap_kernel(f32x4 *a, f32x4 *b, int64_t nvec) {
    const int64_t stride = (int64_t)gridDim.x * kProbeBlock * kProbeUnroll;
    for (int64_t base = (int64_t)blockIdx.x * kProbeBlock * kProbeUnroll + threadIdx.x; base < nvec;
         base += stride) {
        f32x4 va[kProbeUnroll], vb[kProbeUnroll];
#pragma unroll
        for (int k = 0; k < kProbeUnroll; ++k) {
            const int64_t i = base + (int64_t)k * kProbeBlock;
            if (i < nvec) {
                va[k] = probe_load<NT>(a + i);
                vb[k] = probe_load<NT>(b + i);
            }
        }
#pragma unroll
        for (int k = 0; k < kProbeUnroll; ++k) {
            const int64_t i = base + (int64_t)k * kProbeBlock;
            if (i < nvec) {
                probe_store<NT>(a + i, vb[k]);
                probe_store<NT>(b + i, va[k]);
            }
        }
    }
}

}  // namespace

hipError_t launch_swap(void *a, void *b, int64_t nvec, int cus, bool cached, hipStream_t stream) {
    if (nvec < 1 || !a || !b) return hipErrorInvalidValue;
    const int64_t want = (nvec + kProbeBlock * kProbeUnroll - 1) / (kProbeBlock * kProbeUnroll);
    const int grid = (int)std::max<int64_t>(1, std::min<int64_t>(want, (int64_t)cus * 8));
    void *args[] = {&a, &b, &nvec};
    const void *fn = cached ? (const void *)swap_kernel<false> : (const void *)swap_kernel<true>;
    return hipLaunchKernel(fn, dim3(grid), dim3(kProbeBlock), args, 0, stream);
}

}  // namespace pic1d
