// Device-side particle loader (gfx950): draws a run's initial particles on
// the GPU instead of converting and uploading host arrays.
//
// Random numbers are SplitMix64 (Steele, Lea and Flood, OOPSLA 2014) used as
// a counter-based generator: draw i of stream s is the SplitMix64 output
// for the counter base(seed, s) + (i + 1) * gamma, so every particle is
// drawn independently and in any order, and the host can reproduce any
// draw.  Uniforms are the top 53 bits times 2^-53; normals are Box-Muller
// from the draws i of two consecutive streams.
//
// Particle i: x0 = L u_i (positions' stream) or the lattice (i + 1/2) L/np,
// x = x0 + amp sin(k x0) wrapped into [0, L); v = s_i v0 + vth n_i with the
// beam sign s_i: 1, alternating by index, or + when a uniform of the third
// velocity stream is below 1/2.
// Stored as s = x/dx + 1/2 and w = v dt/dx, rounded once to the state
// precision, exactly as the host conversion does.
#include <algorithm>

#include "pic.h"
#include "pic_internal.h"

namespace pic1d {

namespace {

constexpr unsigned long long kGamma = 0x9E3779B97F4A7C15ull;

__host__ __device__ __forceinline__ unsigned long long mix64(unsigned long long z) {
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

__device__ __forceinline__ double uniform53(unsigned long long base, long long i) {
    const unsigned long long r = mix64(base + (unsigned long long)(i + 1) * kGamma);
    return (double)(r >> 11) * (1.0 / 9007199254740992.0);
}

template <typename T>
__global__ __launch_bounds__(256) void load_kernel(T *U, T *W, int64_t np, int ng, LoaderArgs a) {
    const double L = a.L, dx = L / ng, wscale = a.dt / dx, spacing = L / (double)np;
    const T hi = (T)ng + T(0.5);
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < np; i += stride) {
        const double x0 = a.lattice ? ((double)i + 0.5) * spacing : L * uniform53(a.base_pos, i);
        double x = a.amp != 0.0 ? x0 + a.amp * sin(a.k * x0) : x0;
        x = x - L * __builtin_floor(x / L);
        if (x >= L) x = 0.0;
        double v = a.v0;
        if (a.beams == PIC_BEAMS_ALTERNATE && (i & 1)) v = -a.v0;
        if (a.beams == PIC_BEAMS_RANDOM && !(uniform53(a.base_sign, i) < 0.5)) v = -a.v0;
        if (a.vth != 0.0) {
            const double u1 = uniform53(a.base_v1, i), u2 = uniform53(a.base_v2, i);
            v += a.vth * (sqrt(-2.0 * log1p(-u1)) * cos(6.283185307179586 * u2));
        }
        T s = (T)(x / dx + 0.5);
        if (!(s < hi)) s = T(0.5);
        U[i] = s;
        W[i] = (T)(v * wscale);
    }
}

}  // namespace

unsigned long long loader_stream_base(unsigned long long seed, int stream) {
    return mix64(seed * 0x100000001B3ull + (unsigned long long)stream * 0x9E37ull + 1ull);
}

hipError_t launch_loader(void *u, void *w, int64_t np, int ng, int precision, const LoaderArgs &a, int cus,
                         hipStream_t stream) {
    if (np < 1 || ng < 2 || !u || !w) return hipErrorInvalidValue;
    const int64_t want = (np + 255) / 256;
    const int grid = (int)std::min<int64_t>(want, (int64_t)cus * 16);
    LoaderArgs args_copy = a;
    void *args[] = {(void *)&u, (void *)&w, (void *)&np, (void *)&ng, (void *)&args_copy};
    const void *fn = precision ? (const void *)load_kernel<double> : (const void *)load_kernel<float>;
    return hipLaunchKernel(fn, dim3(grid), dim3(256), args, 0, stream);
}

}  // namespace pic1d
