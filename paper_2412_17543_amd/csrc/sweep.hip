// Batched symmetric sweeps of the setup (local interior eliminations and
// Schur complements, Section 3.1; constrained-Neumann saddle inverses,
// eq. localCorr; face Schur complements of the adaptive step, Section 3.3;
// dense coarse inverses, Section 3.2), in panels of 16 pivots with the
// trailing update on the matrix cores.
//
// Sweeping a set P of pivots of a symmetric matrix A = [A_PP A_PQ; A_QP A_QQ]
// replaces it by
//     [ -A_PP^{-1}        A_PP^{-1} A_PQ                 ]
//     [ A_QP A_PP^{-1}    A_QQ - A_QP A_PP^{-1} A_PQ     ]
// and sweeping P1 then P2 equals sweeping P1 u P2 (the one-pivot sweep is the
// case |P| = 1).  So after sweeping the interior pivots, the interior block
// holds -K_II^{-1} and the interface block the Schur complement; after
// sweeping all pivots the matrix holds -A^{-1}.  Per panel of b <= 16
// pivots (every pivot checked for its expected sign):
//   k_panel_prep   (one block per matrix) sweeps the b x b block in LDS,
//                  forms U = A(P, :) and X = A_PP^{-1} U (zero on P's own
//                  columns) into a panel buffer and writes the panel's rows
//                  and columns of the result;
//   k_panel_update (64 x 64 tiles) A <- A - U^T X with
//                  v_mfma_f64_16x16x4f64; U and X vanish on P's columns, so
//                  the panel's rows and columns are left as written.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <vector>

#include "internal.h"
#include "kernels.h"

namespace bddc {

namespace {

constexpr int PB = 16;              // pivots per panel
constexpr int TS = 64;              // edge of a trailing-update tile (4 waves x 16 rows)
typedef double dvec4 __attribute__((ext_vector_type(4)));

__global__ void __launch_bounds__(256) k_panel_prep(const SweepDesc *descs, const int64_t *boff, int step,
                                                    double *buf, int *status) {
    __shared__ double P[PB][PB + 1];
    const SweepDesc d = descs[blockIdx.x];
    const int p0 = d.p0 + PB * step;
    if (p0 >= d.p1) return;
    const int b = min(PB, d.p1 - p0), n = d.n;
    const int64_t ld = d.ld;
    double *U = buf + boff[blockIdx.x];
    double *X = U + (int64_t)PB * n;
    const int t = threadIdx.x, r = t >> 4, c = t & 15;
    P[r][c] = (r < b && c < b) ? d.A[(p0 + r) * ld + p0 + c] : 0.0;
    __syncthreads();
    bool ok = true;
    for (int k = 0; k < b; ++k) {
        const double piv = P[k][k];
        ok = ok && (p0 + k < d.pos_end ? piv > 0.0 : piv < 0.0) && isfinite(piv);
        const double inv = 1.0 / piv;
        const double v = P[r][c], rk = P[r][k], kc = P[k][c];
        __syncthreads();
        if (r < b && c < b) P[r][c] = (r == k) ? (c == k ? -inv : kc * inv) : (c == k ? rk * inv : v - rk * kc * inv);
        __syncthreads();
    }
    if (!ok && t == 0) atomicMax(status, 1);
    // P now holds -A_PP^{-1}; column j of the panel rows: u = A(P, j),
    // x = A_PP^{-1} u = -P u
    for (int j = t; j < n; j += blockDim.x) {
        const bool own = j >= p0 && j < p0 + b;
        double u[PB], x[PB];
#pragma unroll
        for (int k = 0; k < PB; ++k) u[k] = (!own && k < b) ? d.A[(p0 + k) * ld + j] : 0.0;
#pragma unroll
        for (int q = 0; q < PB; ++q) {
            double s = 0.0;
#pragma unroll
            for (int k = 0; k < PB; ++k) s -= P[q][k] * u[k];
            x[q] = q < b ? s : 0.0;
        }
#pragma unroll
        for (int k = 0; k < PB; ++k) {
            U[(int64_t)k * n + j] = u[k];
            X[(int64_t)k * n + j] = x[k];
        }
#pragma unroll
        for (int q = 0; q < PB; ++q)
            if (q < b) d.A[(p0 + q) * ld + j] = own ? P[q][j - p0] : x[q];
        if (!own) {
#pragma unroll
            for (int q = 0; q < PB; ++q)
                if (q < b) d.A[(int64_t)j * ld + p0 + q] = x[q];
        }
    }
}

// A <- A - U^T X over one 64 x 64 tile: wave w takes rows I0 + 16 w .. + 15
// and the four 16-column tiles.  Operand layout of v_mfma_f64_16x16x4f64:
// A[i][k] and B[k][j] in lane i (j) + 16 k, result (i, j) in lane
// j + 16 (i % 4), register i / 4.
__global__ void __launch_bounds__(256) k_panel_update(const SweepDesc *descs, const int64_t *boff, int step,
                                                      const double *buf) {
    const SweepDesc d = descs[blockIdx.y];
    const int p0 = d.p0 + PB * step;
    if (p0 >= d.p1) return;
    const int n = d.n, T = (n + TS - 1) / TS;
    if ((int)blockIdx.x >= T * T) return;
    const int64_t ld = d.ld;
    const int I0 = ((int)blockIdx.x / T) * TS, J0 = ((int)blockIdx.x % T) * TS;
    const double *U = buf + boff[blockIdx.y];
    const double *X = U + (int64_t)PB * n;
    const int w = threadIdx.x >> 6, L = threadIdx.x & 63, li = L & 15, lk = L >> 4;
    const int ia = I0 + 16 * w + li;
    dvec4 acc[4];
#pragma unroll
    for (int tc = 0; tc < 4; ++tc) {
        const int col = J0 + 16 * tc + li;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int row = I0 + 16 * w + lk + 4 * q;
            acc[tc][q] = (row < n && col < n) ? d.A[row * ld + col] : 0.0;
        }
    }
#pragma unroll
    for (int s = 0; s < PB / 4; ++s) {
        const int k = 4 * s + lk;
        const double a = ia < n ? -U[(int64_t)k * n + ia] : 0.0;
#pragma unroll
        for (int tc = 0; tc < 4; ++tc) {
            const int col = J0 + 16 * tc + li;
            const double bv = col < n ? X[(int64_t)k * n + col] : 0.0;
            acc[tc] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, bv, acc[tc], 0, 0, 0);
        }
    }
#pragma unroll
    for (int tc = 0; tc < 4; ++tc) {
        const int col = J0 + 16 * tc + li;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int row = I0 + 16 * w + lk + 4 * q;
            if (row < n && col < n) d.A[row * ld + col] = acc[tc][q];
        }
    }
}

}  // namespace

int64_t sweep_panel_doubles(const std::vector<SweepDesc> &h, std::vector<int64_t> &off) {
    off.assign(h.size(), 0);
    int64_t total = 0;
    for (size_t i = 0; i < h.size(); ++i) {
        off[i] = total;
        total += 2 * (int64_t)PB * std::max(h[i].n, 1);
    }
    return std::max<int64_t>(total, 1);
}

void launch_sweep_blocked(const SweepDesc *d, const int64_t *d_off, const std::vector<SweepDesc> &h, double *buf,
                          int *status, hipStream_t s) {
    int steps = 0, tiles = 1;
    for (const SweepDesc &x : h) {
        steps = std::max(steps, (x.p1 - x.p0 + PB - 1) / PB);
        const int T = (x.n + TS - 1) / TS;
        tiles = std::max(tiles, T * T);
    }
    const int count = (int)h.size();
    constexpr int YMAX = 65535;
    for (int st = 0; st < steps; ++st) {
        for (int c0 = 0; c0 < count; c0 += YMAX) {
            const int cn = std::min(YMAX, count - c0);
            hipLaunchKernelGGL(k_panel_prep, dim3(cn), dim3(256), 0, s, d + c0, d_off + c0, st, buf, status);
            hipLaunchKernelGGL(k_panel_update, dim3(tiles, cn), dim3(256), 0, s, d + c0, d_off + c0, st,
                               (const double *)buf);
        }
    }
}

}  // namespace bddc
