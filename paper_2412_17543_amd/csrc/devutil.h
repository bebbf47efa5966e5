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

// Per-thread part of a contiguous sum: element i goes to thread i % nthr,
// four independent accumulators so that the loads are issued together.
__device__ __forceinline__ double strided_part(const double *p, int n, int t, int nthr) {
    double s0 = 0.0, s1 = 0.0, s2 = 0.0, s3 = 0.0;
    int i = t;
    for (; i + 3 * nthr < n; i += 4 * nthr) {
        s0 += p[i];
        s1 += p[i + nthr];
        s2 += p[i + 2 * nthr];
        s3 += p[i + 3 * nthr];
    }
    for (; i < n; i += nthr) s0 += p[i];
    return (s0 + s1) + (s2 + s3);
}

// Sum of p[0..n) by one wave in a fixed order: every wave that calls it gets
// the same value.
__device__ __forceinline__ double wave_sum_contig(const double *p, int n) {
    return wave_sum(strided_part(p, n, threadIdx.x & 63, 64));
}

// Sum of p[0..n) by the whole block in a fixed order (every thread gets it).
__device__ __forceinline__ double block_sum_contig(const double *p, int n, double *sh) {
    return block_sum(strided_part(p, n, threadIdx.x, blockDim.x), sh);
}

// Block-wide sums of the per-thread values acc[0..ncol) (ncol <= NC, a block
// of exactly 256 threads): 16 columns at a time are transposed through LDS
// (lds: 16 * 256 doubles), thread (u, j) adds the entries j, j + 16, ... of
// column u (consecutive lanes read consecutive words) and a four-step
// butterfly finishes; res[q] (LDS, NC doubles) receives column q.  Fixed
// order; every thread may read res after the call.
template <int NC>
__device__ __forceinline__ void block_sum_cols(const double (&acc)[NC], int ncol, double *lds, double *res) {
    const int t = threadIdx.x, u = t >> 4, j = t & 15;
#pragma unroll
    for (int q0 = 0; q0 < NC; q0 += 16) {
        if (q0 < ncol) {
#pragma unroll
            for (int v = 0; v < 16; ++v)
                if (q0 + v < NC) lds[v * 256 + t] = acc[q0 + v < NC ? q0 + v : 0];
            __syncthreads();
            double s = 0.0;
#pragma unroll
            for (int i = 0; i < 16; ++i) s += lds[u * 256 + i * 16 + j];
            s += __shfl_xor(s, 8);
            s += __shfl_xor(s, 4);
            s += __shfl_xor(s, 2);
            s += __shfl_xor(s, 1);
            if (j == 0 && q0 + u < ncol) res[q0 + u] = s;
            __syncthreads();
        }
    }
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
