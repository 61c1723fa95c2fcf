// Achievable-bandwidth reference for the particle pass (gfx950).
//
// The particle pass reads two FP32 arrays and writes both back in place,
// 16 bytes per particle per step.  This kernel moves exactly those bytes with
// nothing else: it swaps the contents of two device arrays with 16-byte
// non-temporal loads and stores, four vectors per lane in flight, grid-stride
// over all CUs.  Its rate is the HBM bandwidth that this access pattern can
// reach on the device, the reference the pass's roofline fraction is read
// against.  It computes nothing of the method.
#include <algorithm>

#include "pic_internal.h"

namespace pic1d {

namespace {

#define GLOBAL_AS __attribute__((address_space(1)))
typedef float f32x4 __attribute__((ext_vector_type(4)));

constexpr int kProbeBlock = 256;
constexpr int kProbeUnroll = 4;

__global__ __launch_bounds__(kProbeBlock) void swap_kernel(f32x4 *a, f32x4 *b, int64_t nvec) {
    const int64_t stride = (int64_t)gridDim.x * kProbeBlock * kProbeUnroll;
    for (int64_t base = (int64_t)blockIdx.x * kProbeBlock * kProbeUnroll + threadIdx.x; base < nvec;
         base += stride) {
        f32x4 va[kProbeUnroll], vb[kProbeUnroll];
#pragma unroll
        for (int k = 0; k < kProbeUnroll; ++k) {
            const int64_t i = base + (int64_t)k * kProbeBlock;
            if (i < nvec) {
                va[k] = __builtin_nontemporal_load((const GLOBAL_AS f32x4 *)(a + i));
                vb[k] = __builtin_nontemporal_load((const GLOBAL_AS f32x4 *)(b + i));
            }
        }
#pragma unroll
        for (int k = 0; k < kProbeUnroll; ++k) {
            const int64_t i = base + (int64_t)k * kProbeBlock;
            if (i < nvec) {
                __builtin_nontemporal_store(vb[k], (GLOBAL_AS f32x4 *)(a + i));
                __builtin_nontemporal_store(va[k], (GLOBAL_AS f32x4 *)(b + i));
            }
        }
    }
}

}  // namespace

hipError_t launch_swap(void *a, void *b, int64_t nvec, int cus, hipStream_t stream) {
    if (nvec < 1 || !a || !b) return hipErrorInvalidValue;
    const int64_t want = (nvec + kProbeBlock * kProbeUnroll - 1) / (kProbeBlock * kProbeUnroll);
    const int grid = (int)std::max<int64_t>(1, std::min<int64_t>(want, (int64_t)cus * 8));
    void *args[] = {&a, &b, &nvec};
    return hipLaunchKernel((const void *)swap_kernel, dim3(grid), dim3(kProbeBlock), args, 0, stream);
}

}  // namespace pic1d
