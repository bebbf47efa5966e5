// gfx950 kernels of the BDDC / deflated-PCG solver outside the iteration.
//
// Setup (run once): local Q1 assembly, batched in-place sweeps (Gauss-Jordan
// elimination of a chosen pivot range of a symmetric matrix), saddle-point
// matrices of the constrained Neumann problems, tile packing of the symmetric
// operators, coarse matrices.  Once per right-hand side: condensation to the
// interface and interior recovery (Section 3.1), recycling products (Section
// 4.2) and the adjoint element gradient.  The kernels of one iteration are in
// hot.hip.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "devutil.h"
#include "internal.h"
#include "kernels.h"

namespace bddc {

using dev::block_sum;
using dev::kref_entry;


// ---------------------------------------------------------------------------
// setup: local assembly K_i = sum_e c_e h Kref (Section 2), dense row-major
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(256) k_assemble(const AsmDesc *descs) {
    const AsmDesc d = descs[blockIdx.x];
    const size_t nn = (size_t)d.nloc * d.nloc;
    for (size_t t = threadIdx.x; t < nn; t += blockDim.x) d.K[t] = 0.0;
    __syncthreads();
    for (int a = threadIdx.x; a < d.nloc; a += blockDim.x) {
        double *Ka = d.K + (size_t)a * d.nloc;
        for (int t = d.inc_ptr[a]; t < d.inc_ptr[a + 1]; ++t) {
            const int e = d.inc_e[t], v = d.inc_v[t];
            const double c = d.elem_c[e];
            for (int w = 0; w < 8; ++w) {
                const int b = d.elem_loc[e * 8 + w];
                if (b >= 0) Ka[b] += c * kref_entry(v, w);
            }
        }
    }
}

// ---------------------------------------------------------------------------
// setup: Schur complement onto the last m = n - p entries of a permuted copy
// of S (symmetric positive semi-definite, positive definite on the p leading
// entries), for the adaptive face selection: k_face_gather copies S(perm,
// perm) into the work matrix and its trailing block into `keep`; the leading
// p pivots are then swept (sweep.hip), which leaves the Schur complement in
// the trailing block, copied into `hat` by k_face_hat.  One block per face.
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(256) k_face_gather(const FaceSchurDesc *descs) {
    const FaceSchurDesc d = descs[blockIdx.x];
    const int n = d.n, p = d.p, m = n - p;
    const int w = threadIdx.x >> 6, l = threadIdx.x & 63, nw = blockDim.x >> 6;
    for (int i = w; i < n; i += nw) {
        const double *src = d.S + (size_t)d.perm[i] * d.ld;
        for (int j = l; j < n; j += 64) d.work[(size_t)i * n + j] = src[d.perm[j]];
    }
    for (int e = threadIdx.x; e < m * m; e += blockDim.x)
        d.keep[e] = d.S[(size_t)d.perm[p + e / m] * d.ld + d.perm[p + e % m]];
}

__global__ void __launch_bounds__(256) k_face_hat(const FaceSchurDesc *descs) {
    const FaceSchurDesc d = descs[blockIdx.x];
    const int n = d.n, p = d.p, m = n - p;
    for (int e = threadIdx.x; e < m * m; e += blockDim.x) d.hat[e] = d.work[(size_t)(p + e / m) * n + p + e % m];
}

// ---------------------------------------------------------------------------
// setup: saddle matrix [S + C^T Om C, C^T; C, 0] of eq. localCorr in Schur form.
// The augmentation C^T Om C does not change the (1,1) and (1,2) blocks of the
// inverse on the constrained subspace and makes the leading block SPD for
// floating subdomains; om_r = mean(diag S) / ||c_r||^2.
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(256) k_build_saddle(const SaddleDesc *descs) {
    __shared__ double red[16];
    const SaddleDesc d = descs[blockIdx.x];
    const int N = d.nB + d.nc;
    double s = 0.0;
    for (int i = threadIdx.x; i < d.nB; i += blockDim.x) s += d.S[(size_t)i * d.ldS + i];
    s = block_sum(s, red);
    const double sbar = d.nB > 0 ? s / d.nB : 1.0;
    const int w = threadIdx.x >> 6, l = threadIdx.x & 63, nw = blockDim.x >> 6;
    for (int i = w; i < N; i += nw)
        for (int j = l; j < N; j += 64)
            d.M[(size_t)i * d.ldM + j] = (i < d.nB && j < d.nB) ? d.S[(size_t)i * d.ldS + j] : 0.0;
    __syncthreads();
    for (int r = 0; r < d.nc; ++r) {
        const int p0 = d.cptr[r], m = d.cptr[r + 1] - p0;
        double nrm2 = 0.0;
        for (int t = 0; t < m; ++t) nrm2 += d.cval[p0 + t] * d.cval[p0 + t];
        const double om = sbar / nrm2;
        for (int t = threadIdx.x; t < m * m; t += blockDim.x) {
            const int a = t / m, b = t - a * m;
            d.M[(size_t)d.ccol[p0 + a] * d.ldM + d.ccol[p0 + b]] += om * d.cval[p0 + a] * d.cval[p0 + b];
        }
        for (int t = threadIdx.x; t < m; t += blockDim.x) {
            d.M[(size_t)(d.nB + r) * d.ldM + d.ccol[p0 + t]] = d.cval[p0 + t];
            d.M[(size_t)d.ccol[p0 + t] * d.ldM + d.nB + r] = d.cval[p0 + t];
        }
        __syncthreads();
    }
}


// ---------------------------------------------------------------------------
// setup: pack a symmetric n x n block in the slot layout
// of tile_rows / strip_len: 16x16 tiles (element order of tile_index), tile
// row I holding (I, I..nt-1), zero past n; then, with a strip, the ragged
// tail rows, row-major.  Value = sign * src[i][j] * D[i] * D[j].  With
// phr >= 0 the coarse basis sign * phi[i][q] * D[i] is written column-major
// (nc rows of phi_ld(n) values, zero past n) for the coarse restriction and
// the prolongation.
// ---------------------------------------------------------------------------
__device__ __forceinline__ void store_conv(double *p, double v) { *p = v; }
__device__ __forceinline__ void store_conv(float *p, double v) { *p = (float)v; }
__device__ __forceinline__ void store_conv(uint16_t *p, double v) {
    // round-to-nearest-even float32 -> bfloat16
    const float f = (float)v;
    const uint32_t u = __float_as_uint(f);
    const uint32_t r = u + 0x7fffu + ((u >> 16) & 1u);
    *p = (uint16_t)(r >> 16);
}

template <typename T>
__global__ void __launch_bounds__(256) k_pack(const PackDesc *descs, T *dst, T *phir) {
    const PackDesc d = descs[blockIdx.x];
    const int nt = tile_rows(d.n), n0 = nt * TILE;
    auto node = [&](int gi, int gj) {
        double v = d.sign * d.src[(size_t)gi * d.ld + gj];
        if (d.D) v *= d.D[gi] * d.D[gj];
        return v;
    };
    int64_t base = 0;
    for (int I = 0; I < nt; ++I) {
        const int nrow = nt - I;
        for (int e = threadIdx.x; e < nrow * 256; e += blockDim.x) {
            const int q = e >> 8, r = (e >> 4) & 15, c = e & 15;
            const int gi = I * TILE + r, gj = (I + q) * TILE + c;
            const double v = (gi < d.n && gj < d.n) ? node(gi, gj) : 0.0;
            store_conv(dst + d.dst + (base + q) * 256 + tile_index(r, c, (int)sizeof(T)), v);
        }
        base += nrow;
    }
    T *sp = dst + d.dst + base * 256;
    for (int64_t e = threadIdx.x; e < strip_len(d.n); e += blockDim.x) {
        const int r = (int)(e / d.n), k = (int)(e - (int64_t)r * d.n);
        store_conv(sp + e, node(n0 + r, k));
    }
    if (d.phr >= 0 && d.phi) {
        const int ld = phi_ld(d.n);
        for (int64_t e = threadIdx.x; e < (int64_t)d.nc * ld; e += blockDim.x) {
            const int q = (int)(e / ld), gi = (int)(e - (int64_t)q * ld);
            double v = 0.0;
            if (gi < d.n) {
                v = d.sign * d.phi[(size_t)gi * d.ldphi + q];
                if (d.D) v *= d.D[gi];
            }
            store_conv(phir + d.phr + e, v);
        }
    }
}


// setup: the upper triangle of a symmetric n x n row-major matrix (sign
// folded in) as 64 x 64 row-major blocks (I, J >= I), zero past n
__global__ void __launch_bounds__(256) k_pack_symblk(const double *M, int64_t ldm, int n, int nb, const int32_t *bI,
                                                     double sign, double *B) {
    const int b = blockIdx.x, I = bI[b], J = I + (b - (I * nb - I * (I - 1) / 2));
    for (int e = threadIdx.x; e < 4096; e += blockDim.x) {
        const int gi = 64 * I + (e >> 6), gj = 64 * J + (e & 63);
        B[(int64_t)b * 4096 + e] = (gi < n && gj < n) ? sign * M[(int64_t)gi * ldm + gj] : 0.0;
    }
}

// ---------------------------------------------------------------------------
// setup: K_C = Phi^T S Phi (coarse element matrices, eq. coarse_problem)
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(256) k_ptsp(const PtspDesc *descs) {
    const PtspDesc d = descs[blockIdx.x];
    for (int64_t t = threadIdx.x; t < (int64_t)d.n * d.nc; t += blockDim.x) {
        const int i = (int)(t / d.nc), a = (int)(t - (int64_t)i * d.nc);
        double s = 0.0;
        for (int j = 0; j < d.n; ++j) s += d.S[(size_t)i * d.ldS + j] * d.Phi[(size_t)j * d.ldPhi + a];
        d.X[t] = d.phisign * s;
    }
    __syncthreads();
    for (int t = threadIdx.x; t < d.nc * d.nc; t += blockDim.x) {
        const int a = t / d.nc, b = t - a * d.nc;
        if (b < a) continue;
        double s = 0.0;
        for (int i = 0; i < d.n; ++i) s += d.Phi[(size_t)i * d.ldPhi + a] * d.X[(size_t)i * d.nc + b];
        s *= d.phisign;
        d.out[a * d.nc + b] = s;
        d.out[b * d.nc + a] = s;
    }
}

// dense copy with scaling (setup: N2, Phi2 extraction)
__global__ void __launch_bounds__(256) k_dense_copy(const DenseCopyDesc *descs) {
    const DenseCopyDesc d = descs[blockIdx.x];
    for (int64_t t = threadIdx.x; t < (int64_t)d.rows * d.cols; t += blockDim.x) {
        const int r = (int)(t / d.cols), c = (int)(t - (int64_t)r * d.cols);
        double v = d.sign * d.src[(size_t)r * d.ld + c];
        if (d.Drow) v *= d.Drow[r];
        if (d.Dcol) v *= d.Dcol[c];
        d.dst[(size_t)r * d.ldd + c] = v;
    }
}

// out[t] = sum_{k in [ptr[t], ptr[t+1])} src[idx[k]]
__global__ void __launch_bounds__(256) k_gather_sum(int64_t n, const int32_t *ptr, const int32_t *idx,
                                                    const double *src, double *out) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n) return;
    double s = 0.0;
    for (int k = ptr[t]; k < ptr[t + 1]; ++k) s += src[idx[k]];
    out[t] = s;
}


// ---------------------------------------------------------------------------
// condensation and interior recovery (Section 3.1) with the packed interior
// inverses (products in hot.hip's k_symv) and the sparse couplings K_IB, K_BI
// ---------------------------------------------------------------------------
// One block per subdomain: y_I summed from its work items into LDS, then
// t_k = sum_a K_BI[k][a] y_I[a] for the interface rows.
__global__ void __launch_bounds__(256) k_cond_local(CondArgs a) {
    extern __shared__ double yI[];
    const int i = blockIdx.x;
    const int nI = a.nI[i], nB = a.nB[i], C = a.nchunk[i];
    const double *yp = a.ypart + a.pb[i];
    for (int k = threadIdx.x; k < nI; k += blockDim.x) {
        double s = 0.0;
        for (int q = 0; q < C; ++q) s += yp[(int64_t)q * nI + k];
        yI[k] = s;
    }
    __syncthreads();
    const int boff = a.b_off[i];
    for (int k = threadIdx.x; k < nB; k += blockDim.x) {
        double s = 0.0;
        for (int e = a.kbi_ptr[boff + k]; e < a.kbi_ptr[boff + k + 1]; ++e) s += a.kbi_val[e] * yI[a.kbi_col[e]];
        a.t[boff + k] = s;
    }
}

// b = F_G - sum_i R_i^T t_i (grid-stride); per-block ||b||^2 partials
__global__ void __launch_bounds__(256) k_cond_asm(CondAsmArgs a) {
    __shared__ double red[16];
    double bb = 0.0;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; g < a.n; g += stride) {
        double s = a.F[a.gamma[g]];
        for (int k = a.ptr[g]; k < a.ptr[g + 1]; ++k) s -= a.loc[a.idx[k]];
        a.b[g] = s;
        bb += s * s;
    }
    bb = block_sum(bb, red);
    if (threadIdx.x == 0) a.part[blockIdx.x] = bb;
}

// One block per subdomain: out[nodesI] = F_I - K_IB x_B (the interior
// right-hand side of the recovery, written at the subdomain's own nodes).
__global__ void __launch_bounds__(256) k_rec_rhs(RecArgs a) {
    extern __shared__ double xB[];
    const int i = blockIdx.x;
    const int nI = a.nI[i], nB = a.nB[i];
    const int boff = a.b_off[i], ioff = a.i_off[i];
    for (int k = threadIdx.x; k < nB; k += blockDim.x) xB[k] = a.x[a.gB[boff + k]];
    __syncthreads();
    for (int r = threadIdx.x; r < nI; r += blockDim.x) {
        const int node = a.nodesI[ioff + r];
        double s = a.F[node];
        for (int e = a.kib_ptr[ioff + r]; e < a.kib_ptr[ioff + r + 1]; ++e) s -= a.kib_val[e] * xB[a.kib_col[e]];
        a.out[node] = s;
    }
}

// u[nodesI] = x_I summed from the interior product's work items.
__global__ void __launch_bounds__(256) k_rec_out(RecArgs a) {
    const int i = blockIdx.x;
    const int nI = a.nI[i], C = a.nchunk[i], ioff = a.i_off[i];
    const double *yp = a.ypart + a.pb[i];
    for (int r = threadIdx.x; r < nI; r += blockDim.x) {
        double s = 0.0;
        for (int q = 0; q < C; ++q) s += yp[(int64_t)q * nI + r];
        a.u[a.nodesI[ioff + r]] = s;
    }
}

__global__ void __launch_bounds__(256) k_scatter_gamma(int n, const int32_t *gamma, const double *x, double *u) {
    const int g = blockIdx.x * blockDim.x + threadIdx.x;
    if (g < n) u[gamma[g]] = x[g];
}

// ---------------------------------------------------------------------------
// recycling (Section 4.2) on the matrix cores, v_mfma_f64_16x16x4f64 (lane
// layout: A[i][k] and B[k][j] in lane i (j) + 16 k; result (i, j) in lane
// j + 16 (i % 4), register i / 4).
//
// k_recycle_gemm: out[:, c] = sum_q V[:, q] Y[q][c] with V = [V1, V2]
// column-major (leading dimension ld); blockIdx.y selects [W, P] or
// [AW, AP].  Each wave takes 16 rows and forms out^T = Y^T V^T for them, 16
// columns per tile (NT tiles): the B operand is 16 consecutive rows of one
// column of V (one coalesced load per lane and step of 4 columns), the A
// operand entries of Y (a few KB, read through the cache), and each result
// register holds 16 consecutive rows of one output column.
// ---------------------------------------------------------------------------
typedef double dvec4 __attribute__((ext_vector_type(4)));

template <int NT>
__global__ void __launch_bounds__(256) k_recycle_gemm(GemmArgs a) {
    const int y = blockIdx.y;
    const double *V1 = a.V1[y], *V2 = a.V2[y];
    const int w = threadIdx.x >> 6, L = threadIdx.x & 63, li = L & 15, lk = L >> 4;
    const int64_t r0 = ((int64_t)blockIdx.x * 4 + w) * 16;
    if (r0 >= a.n) return;                           // (the whole wave)
    const int64_t row = r0 + li;
    const bool rok = row < a.n;
    const int m = a.k1 + a.k2;
    dvec4 acc[NT];
#pragma unroll
    for (int t = 0; t < NT; ++t) acc[t] = dvec4{0.0, 0.0, 0.0, 0.0};
    // B operands GQ steps (4 GQ columns of V) at a time, all requested before
    // the first is used
    constexpr int GQ = 8;
    for (int q1 = 0; q1 < m; q1 += 4 * GQ) {
        double b[GQ];
#pragma unroll
        for (int u = 0; u < GQ; ++u) {
            const int q = q1 + 4 * u + lk;
            b[u] = (q < m && rok) ? (q < a.k1 ? V1 + (int64_t)q * a.ld : V2 + (int64_t)(q - a.k1) * a.ld)[row] : 0.0;
        }
#pragma unroll
        for (int u = 0; u < GQ; ++u) {
            const int q = q1 + 4 * u + lk;
#pragma unroll
            for (int t = 0; t < NT; ++t) {
                const int c = 16 * t + li;
                const double av = (q < m && c < a.ncol) ? a.Y[(int64_t)q * a.ldy + c] : 0.0;
                acc[t] = __builtin_amdgcn_mfma_f64_16x16x4f64(av, b[u], acc[t], 0, 0, 0);
            }
        }
    }
    if (!rok) return;
    double *out = a.out[y];
#pragma unroll
    for (int t = 0; t < NT; ++t)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int c = 16 * t + lk + 4 * r;
            if (c < a.ncol) out[(int64_t)c * a.ld + row] = acc[t][r];
        }
}

// ---------------------------------------------------------------------------
// Gram product X^T Y (k x k2, both <= 64) of two column-major blocks (n x k
// and n x k2): per-block partials part[(p k2 + q) nblocks + block].  A block takes
// consecutive chunks of GRAM_ROWS rows, stages both blocks of the chunk in
// LDS (coalesced column loads), and each of its 4 waves multiplies its 16
// rows of the chunk on the matrix cores into all T x T output tiles
// (T = ceil(k / 16)); the waves' sums are added in wave order at the end.
// ---------------------------------------------------------------------------
constexpr int GRAM_ROWS = 64;
template <int T>
__global__ void __launch_bounds__(256, T <= 3 ? 2 : 1) k_gram(GramArgs a) {
    __shared__ double xs[16 * T][GRAM_ROWS + 1];
    __shared__ double ys[16 * T][GRAM_ROWS + 1];
    const int k = a.k, k2 = a.k2;
    const int w = threadIdx.x >> 6, L = threadIdx.x & 63, li = L & 15, lk = L >> 4;
    const int64_t per = (a.n + gridDim.x - 1) / gridDim.x;
    const int64_t g0 = (int64_t)blockIdx.x * per, g1 = min((int64_t)a.n, g0 + per);
    dvec4 acc[T][T];
#pragma unroll
    for (int p = 0; p < T; ++p)
#pragma unroll
        for (int q = 0; q < T; ++q) acc[p][q] = dvec4{0.0, 0.0, 0.0, 0.0};
    // a chunk's entries (4 T per thread and block) are all requested before
    // any is stored, and the next chunk's while the current one is multiplied
    constexpr int PER = GRAM_ROWS * 16 * T / 256;
    double vx[PER], vy[PER];
    auto fetch = [&](int64_t s0) {
        const int nr = (int)min((int64_t)GRAM_ROWS, g1 - s0);
#pragma unroll
        for (int u = 0; u < PER; ++u) {
            const int t = threadIdx.x + 256 * u, rr = t % GRAM_ROWS, c = t / GRAM_ROWS;
            vx[u] = rr < nr && c < k ? a.X[(int64_t)c * a.ld + s0 + rr] : 0.0;
            vy[u] = rr < nr && c < k2 ? a.Y[(int64_t)c * a.ld + s0 + rr] : 0.0;
        }
    };
    if (g0 < g1) fetch(g0);
    for (int64_t s0 = g0; s0 < g1; s0 += GRAM_ROWS) {
        __syncthreads();
#pragma unroll
        for (int u = 0; u < PER; ++u) {
            const int t = threadIdx.x + 256 * u, rr = t % GRAM_ROWS, c = t / GRAM_ROWS;
            xs[c][rr] = vx[u];
            ys[c][rr] = vy[u];
        }
        __syncthreads();
        if (s0 + GRAM_ROWS < g1) fetch(s0 + GRAM_ROWS);
#pragma unroll
        for (int s = 0; s < 4; ++s) {
            const int rr = 16 * w + 4 * s + lk;
            double av[T], bv[T];
#pragma unroll
            for (int p = 0; p < T; ++p) {
                av[p] = xs[16 * p + li][rr];
                bv[p] = ys[16 * p + li][rr];
            }
#pragma unroll
            for (int p = 0; p < T; ++p)
#pragma unroll
                for (int q = 0; q < T; ++q) acc[p][q] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[p], bv[q], acc[p][q], 0, 0, 0);
        }
    }
    // waves' sums in wave order through LDS (xs reused: 16 T x 16 T <= its size)
    double *sum = &xs[0][0];
    for (int wv = 0; wv < 4; ++wv) {
        __syncthreads();
        if (w == wv) {
#pragma unroll
            for (int p = 0; p < T; ++p)
#pragma unroll
                for (int q = 0; q < T; ++q)
#pragma unroll
                    for (int r = 0; r < 4; ++r) {
                        const int i = 16 * p + lk + 4 * r, j = 16 * q + li;
                        const double v = acc[p][q][r];
                        sum[i * 16 * T + j] = wv == 0 ? v : sum[i * 16 * T + j] + v;
                    }
        }
    }
    __syncthreads();
    for (int e = threadIdx.x; e < k * k2; e += blockDim.x) {
        const int i = e / k2, j = e % k2;
        a.part[(int64_t)e * gridDim.x + blockIdx.x] = sum[i * 16 * T + j];
    }
}

// adjoint: g_e = - c_e h sum_k lam_{k,e}^T Kref u_{k,e}
__global__ void __launch_bounds__(256) k_elem_grad(GradArgs a) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= a.n_elem) return;
    if (a.keep && !a.keep[e]) { a.grad[e] = 0.0; return; }
    const int64_t ex = e % a.nx, ey = (e / a.nx) % a.ny, ez = e / ((int64_t)a.nx * a.ny);
    const int64_t n1x = a.nx + 1, n1y = a.ny + 1;
    int64_t nd[8];
    for (int v = 0; v < 8; ++v)
        nd[v] = (ex + (v & 1)) + n1x * ((ey + ((v >> 1) & 1)) + n1y * (ez + ((v >> 2) & 1)));
    double s = 0.0;
    for (int k = 0; k < a.n_rhs; ++k) {
        const double *lam = a.lam + (size_t)k * a.n_nodes;
        const double *u = a.u + (size_t)k * a.n_nodes;
        double lv[8], uv[8];
        for (int v = 0; v < 8; ++v) {
            const bool fr = a.free_node[nd[v]] != 0;
            lv[v] = fr ? lam[nd[v]] : 0.0;
            uv[v] = fr ? u[nd[v]] : 0.0;
        }
        for (int v = 0; v < 8; ++v) {
            double t = 0.0;
            for (int w = 0; w < 8; ++w) t += kref_entry(v, w) * uv[w];
            s += lv[v] * t;
        }
    }
    a.grad[e] = -a.coefh[e] * s;
}

__global__ void __launch_bounds__(256) k_copy(int64_t n, const double *src, double *dst) {
    const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (g < n) dst[g] = src[g];
}

__global__ void __launch_bounds__(256) k_fill(int64_t n, double v, double *dst) {
    const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (g < n) dst[g] = v;
}

// ---------------------------------------------------------------------------
// control block and deflation-basis bookkeeping on the device
// ---------------------------------------------------------------------------
__global__ void k_ctl_init(Ctl *c, double rtol2, int record, const RecState *st, int32_t *hflag, double *hprog,
                           int iter_stop) {
    if (threadIdx.x != 0) return;
    Ctl h{};
    h.rtol2 = rtol2;
    h.iter_stop = iter_stop;
    h.record = record;
    h.k = st ? st->k : 0;
    h.hflag = hflag;
    h.hprog = hprog;
    *c = h;
}

__global__ void k_set_done(Ctl *c, int v) {
    if (threadIdx.x == 0) c->done = v;
}

__global__ void k_resume(Ctl *c, int iter_stop) {
    if (threadIdx.x == 0) {
        c->done = 0;
        c->iter_stop = iter_stop;
    }
}

__global__ void k_set_state(RecState *st, int k, int ok) {
    if (threadIdx.x == 0) { st->k = k; st->ok = ok; }
}

// One wave: symmetrise the new W^T A W and invert it in LDS by a symmetric
// Gauss-Jordan sweep of all pivots (lane t owns row t; after the sweep the
// matrix holds -(W^T A W)^{-1}).  Every pivot of a symmetric positive
// definite matrix is positive (it is a diagonal entry of a Schur
// complement), so state->ok = 1 exactly when the matrix is positive definite
// (Section 4.1: W^T A W must be invertible for the projection of
// eq. projectionQ).  k <= RMAX = 64.
__global__ void __launch_bounds__(64) k_chol_inv(CholArgs a) {
    __shared__ double A[RMAX][RMAX + 1];
    __shared__ double row[RMAX];
    const int k = a.k, t = threadIdx.x;
    // lane t reads row t (all loads issued before any store), then the
    // symmetric part is formed in LDS
    if (t < k) {
        double v[RMAX];
#pragma unroll
        for (int j = 0; j < RMAX; ++j) v[j] = j < k ? a.waw[t * k + j] : 0.0;
#pragma unroll
        for (int j = 0; j < RMAX; ++j) A[t][j] = v[j];
    }
    __syncthreads();
    {
        double v[RMAX];
#pragma unroll
        for (int j = 0; j < RMAX; ++j) v[j] = (t < k) ? 0.5 * (A[t][j] + A[j][t]) : 0.0;
        __syncthreads();
        if (t < k) {
#pragma unroll
            for (int j = 0; j < RMAX; ++j) A[t][j] = v[j];
#pragma unroll
            for (int j = 0; j < RMAX; ++j)
                if (j < k) a.waw_sym[t * k + j] = v[j];
        }
    }
    __syncthreads();
    for (int p = 0; p < k; ++p) {
        if (t < k) row[t] = A[p][t];
        __syncthreads();
        const double piv = row[p];
        if (!(piv > 0.0 && isfinite(piv))) {     // the same value in every lane
            if (t == 0) a.state->ok = 0;
            return;
        }
        const double inv = 1.0 / piv;
        if (t < k) {
            if (t == p) {
                for (int j = 0; j < k; ++j) A[p][j] = (j == p) ? -inv : row[j] * inv;
            } else {
                const double f = row[t] * inv;     // A(t, p) = A(p, t) by symmetry
                for (int j = 0; j < k; ++j) A[t][j] = (j == p) ? f : A[t][j] - f * row[j];
            }
        }
        __syncthreads();
    }
    if (t < k) {
#pragma unroll
        for (int j = 0; j < RMAX; ++j)
            if (j < k) a.inv[t * k + j] = -0.5 * (A[t][j] + A[j][t]);
    }
    if (t == 0) a.state->ok = 1;
}

// The new basis was written over W and A W; its (W^T A W)^{-1} (and
// (W^T W)^{-1}) replace the old ones when the Cholesky succeeded.  Otherwise
// the basis is dropped: the size returns to the null-space columns, whose
// block of both inverses is 1.
__global__ void __launch_bounds__(256) k_commit(CommitArgs a) {
    if (a.state->ok) {
        for (int e = threadIdx.x; e < a.ncol * a.ncol; e += blockDim.x) {
            a.inv[e] = a.inv_new[e];
            if (a.ww_new) a.ww[e] = a.ww_new[e];
        }
        if (threadIdx.x == 0) a.state->k = a.ncol;
    } else if (threadIdx.x == 0) {
        a.state->k = a.nullc;
        if (a.nullc) {
            a.inv[0] = 1.0;
            if (a.ww) a.ww[0] = 1.0;
        }
    }
}

// A <- A + coef e e^T (n x n, leading dimension ld)
__global__ void __launch_bounds__(256) k_rank1(double *A, int64_t ld, int n, const double *e, double coef) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= (int64_t)n * n) return;
    const int i = (int)(t / n), j = (int)(t % n);
    A[i * ld + j] += coef * e[i] * e[j];
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------
static inline unsigned nblk(int64_t n, int b) { return (unsigned)((n + b - 1) / b); }

void launch_rank1(double *A, int64_t ld, int n, const double *e, double coef, hipStream_t s) {
    if (n > 0) hipLaunchKernelGGL(k_rank1, dim3(nblk((int64_t)n * n, 256)), dim3(256), 0, s, A, ld, n, e, coef);
}
void launch_assemble(const AsmDesc *d, int n, hipStream_t s) {
    hipLaunchKernelGGL(k_assemble, dim3(n), dim3(256), 0, s, d);
}
void launch_face_schur(const FaceSchurDesc *d, const std::vector<FaceSchurDesc> &h, SweepDesc *d_sw, int64_t *d_off,
                       double *panel, int *status, hipStream_t s) {
    const int n = (int)h.size();
    if (n <= 0) return;
    std::vector<SweepDesc> sw(n);
    for (int q = 0; q < n; ++q) sw[q] = SweepDesc{h[q].work, h[q].n, h[q].n, 0, h[q].p, h[q].p};
    std::vector<int64_t> off;
    sweep_panel_doubles(sw, off);
    // (synchronous: the host vectors end with this call; the caller waits for
    // the previous batch before reusing the buffers)
    (void)hipMemcpy(d_sw, sw.data(), n * sizeof(SweepDesc), hipMemcpyHostToDevice);
    (void)hipMemcpy(d_off, off.data(), n * sizeof(int64_t), hipMemcpyHostToDevice);
    hipLaunchKernelGGL(k_face_gather, dim3(n), dim3(256), 0, s, d);
    launch_sweep_blocked(d_sw, d_off, sw, panel, status, s);
    hipLaunchKernelGGL(k_face_hat, dim3(n), dim3(256), 0, s, d);
}
void launch_build_saddle(const SaddleDesc *d, int n, hipStream_t s) {
    hipLaunchKernelGGL(k_build_saddle, dim3(n), dim3(256), 0, s, d);
}
void launch_pack(const PackDesc *d, int n, int prec, void *dst, void *phir, hipStream_t s) {
    if (prec == 64) hipLaunchKernelGGL(k_pack<double>, dim3(n), dim3(256), 0, s, d, (double *)dst, (double *)phir);
    else if (prec == 32) hipLaunchKernelGGL(k_pack<float>, dim3(n), dim3(256), 0, s, d, (float *)dst, (float *)phir);
    else hipLaunchKernelGGL(k_pack<uint16_t>, dim3(n), dim3(256), 0, s, d, (uint16_t *)dst, (uint16_t *)phir);
}
void launch_pack_symblk(const double *M, int64_t ldm, int n, int nb, const int32_t *bI, double sign, double *B,
                        hipStream_t s) {
    if (nb > 0) hipLaunchKernelGGL(k_pack_symblk, dim3(nb * (nb + 1) / 2), dim3(256), 0, s, M, ldm, n, nb, bI, sign, B);
}
void launch_ptsp(const PtspDesc *d, int n, hipStream_t s) {
    hipLaunchKernelGGL(k_ptsp, dim3(n), dim3(256), 0, s, d);
}
void launch_dense_copy(const DenseCopyDesc *d, int n, hipStream_t s) {
    hipLaunchKernelGGL(k_dense_copy, dim3(n), dim3(256), 0, s, d);
}
void launch_gather_sum(int64_t n, const int32_t *ptr, const int32_t *idx, const double *src, double *out, hipStream_t s) {
    if (n > 0) hipLaunchKernelGGL(k_gather_sum, dim3(nblk(n, 256)), dim3(256), 0, s, n, ptr, idx, src, out);
}
void launch_cond_local(const CondArgs &a, int nsub, int max_nI, hipStream_t s) {
    hipLaunchKernelGGL(k_cond_local, dim3(nsub), dim3(256), (size_t)std::max(1, max_nI) * 8, s, a);
}
void launch_cond_asm(const CondAsmArgs &a, int grid, hipStream_t s) {
    hipLaunchKernelGGL(k_cond_asm, dim3(grid), dim3(256), 0, s, a);
}
void launch_rec_rhs(const RecArgs &a, int nsub, int max_nB, hipStream_t s) {
    hipLaunchKernelGGL(k_rec_rhs, dim3(nsub), dim3(256), (size_t)std::max(1, max_nB) * 8, s, a);
}
void launch_rec_out(const RecArgs &a, int nsub, hipStream_t s) {
    hipLaunchKernelGGL(k_rec_out, dim3(nsub), dim3(256), 0, s, a);
}
void launch_scatter_gamma(int n, const int32_t *gamma, const double *x, double *u, hipStream_t s) {
    if (n > 0) hipLaunchKernelGGL(k_scatter_gamma, dim3(nblk(n, 256)), dim3(256), 0, s, n, gamma, x, u);
}
void launch_recycle_gemm(const GemmArgs &a, hipStream_t s, int ny) {
    if (a.n <= 0) return;
    const dim3 grid(nblk(a.n, 64), ny);               // 64 rows per block
    if (a.ncol <= 16) hipLaunchKernelGGL(k_recycle_gemm<1>, grid, dim3(256), 0, s, a);
    else if (a.ncol <= 32) hipLaunchKernelGGL(k_recycle_gemm<2>, grid, dim3(256), 0, s, a);
    else if (a.ncol <= 48) hipLaunchKernelGGL(k_recycle_gemm<3>, grid, dim3(256), 0, s, a);
    else hipLaunchKernelGGL(k_recycle_gemm<4>, grid, dim3(256), 0, s, a);
}
void launch_gram(const GramArgs &a0, int nblocks, hipStream_t s) {
    GramArgs a = a0;
    if (a.k2 <= 0) a.k2 = a.k;
    const int km = std::max(a.k, a.k2);
    if (km <= 16) hipLaunchKernelGGL(k_gram<1>, dim3(nblocks), dim3(256), 0, s, a);
    else if (km <= 32) hipLaunchKernelGGL(k_gram<2>, dim3(nblocks), dim3(256), 0, s, a);
    else if (km <= 48) hipLaunchKernelGGL(k_gram<3>, dim3(nblocks), dim3(256), 0, s, a);
    else hipLaunchKernelGGL(k_gram<4>, dim3(nblocks), dim3(256), 0, s, a);
}
void launch_elem_grad(const GradArgs &a, hipStream_t s) {
    if (a.n_elem > 0) hipLaunchKernelGGL(k_elem_grad, dim3(nblk(a.n_elem, 256)), dim3(256), 0, s, a);
}
void launch_copy(int64_t n, const double *src, double *dst, hipStream_t s) {
    if (n > 0) hipLaunchKernelGGL(k_copy, dim3(nblk(n, 256)), dim3(256), 0, s, n, src, dst);
}
void launch_fill(int64_t n, double v, double *dst, hipStream_t s) {
    if (n > 0) hipLaunchKernelGGL(k_fill, dim3(nblk(n, 256)), dim3(256), 0, s, n, v, dst);
}

void launch_ctl_init(Ctl *ctl, double rtol2, int record, const RecState *state, int32_t *hflag, double *hprog,
                     int iter_stop, hipStream_t s) {
    hipLaunchKernelGGL(k_ctl_init, dim3(1), dim3(64), 0, s, ctl, rtol2, record, state, hflag, hprog, iter_stop);
}
void launch_resume(Ctl *ctl, int iter_stop, hipStream_t s) {
    hipLaunchKernelGGL(k_resume, dim3(1), dim3(64), 0, s, ctl, iter_stop);
}
void launch_set_done(Ctl *ctl, int v, hipStream_t s) {
    hipLaunchKernelGGL(k_set_done, dim3(1), dim3(64), 0, s, ctl, v);
}
void launch_set_state(RecState *state, int k, int ok, hipStream_t s) {
    hipLaunchKernelGGL(k_set_state, dim3(1), dim3(64), 0, s, state, k, ok);
}
void launch_chol_inv(const CholArgs &a, hipStream_t s) {
    hipLaunchKernelGGL(k_chol_inv, dim3(1), dim3(64), 0, s, a);
}
void launch_commit(const CommitArgs &a, hipStream_t s) {
    hipLaunchKernelGGL(k_commit, dim3(1), dim3(256), 0, s, a);
}

}  // namespace bddc
