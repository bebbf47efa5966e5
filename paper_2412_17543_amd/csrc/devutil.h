// Device helpers shared by the HIP sources of the library (internal).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace bddc {
namespace dev {

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int m = 32; m >= 1; m >>= 1) v += __shfl_xor(v, m);
    return v;
}

__device__ __forceinline__ float wave_sum(float v) {
#pragma unroll
    for (int m = 32; m >= 1; m >>= 1) v += __shfl_xor(v, m);
    return v;
}

// Sum over the block (every thread gets the result); sh holds >= 16 doubles.
__device__ __forceinline__ double block_sum(double v, double *sh) {
    v = wave_sum(v);
    const int w = threadIdx.x >> 6, l = threadIdx.x & 63, nw = blockDim.x >> 6;
    __syncthreads();
    if (l == 0) sh[w] = v;
    __syncthreads();
    double t = 0.0;
    for (int i = 0; i < nw; ++i) t += sh[i];
    __syncthreads();
    return t;
}

// Sum of p[i * st], i < n, by one wave in a fixed order (lane-strided partial
// sums, then a butterfly): every wave that calls it gets the same value.
__device__ __forceinline__ double wave_sum_strided(const double *p, int n, int st) {
    const int l = threadIdx.x & 63;
    double s = 0.0;
    for (int i = l; i < n; i += 64) s += p[(size_t)i * st];
    return wave_sum(s);
}

__device__ __forceinline__ float bf16_to_f32(uint32_t h) { return __uint_as_float(h << 16); }

// Q1 reference stiffness on the unit cube: 1/3 on the diagonal, 0 between
// vertices differing in one coordinate, -1/12 otherwise.
__device__ __forceinline__ double kref_entry(int v, int w) {
    const int nd = __popc(v ^ w);
    return nd == 0 ? (1.0 / 3.0) : (nd == 1 ? 0.0 : (-1.0 / 12.0));
}

}  // namespace dev
}  // namespace bddc
