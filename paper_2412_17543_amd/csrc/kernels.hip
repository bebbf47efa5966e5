// gfx950 kernels of the BDDC / deflated-PCG solver.
//
// Setup (run once): local Q1 assembly, batched in-place sweeps (Gauss-Jordan
// elimination of a chosen pivot range of a symmetric matrix), saddle-point
// matrices of the constrained Neumann problems, tile packing of symmetric
// operators.  Iteration (hot path): a tiled symmetric matrix-vector product
// with LDS-staged gathers for the Schur complements S_i and the Neumann
// operators N_i (+ coarse bases Phi_i), deterministic owner-computes
// assembly fused with the PCG updates and reductions, the coarse phases of
// two/three-level BDDC, and the deflation projection.
//
// Reductions are deterministic: each block writes one partial, the last block
// to finish (atomic ticket) sums the partials in index order.
#include <hip/hip_runtime.h>

#include "internal.h"
#include "kernels.h"

namespace bddc {

// ---------------------------------------------------------------------------
// helpers
// ---------------------------------------------------------------------------
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int m = 32; m >= 1; m >>= 1) v += __shfl_xor(v, m);
    return v;
}

// Sum over the block; the result is returned to every thread.
__device__ double block_sum(double v, double *sh) {
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

// Atomic ticket: true in exactly one block, the last one to arrive.  Callers
// write their partial before and read all partials after.
__device__ bool last_block(unsigned int *cnt) {
    __shared__ int is_last;
    __threadfence();
    __syncthreads();
    if (threadIdx.x == 0) {
        unsigned int prev = atomicAdd(cnt, 1u);
        is_last = (prev == gridDim.x - 1) ? 1 : 0;
        if (is_last) atomicExch(cnt, 0u);
    }
    __syncthreads();
    if (is_last) __threadfence();
    return is_last != 0;
}

// Deterministic sum of n partials (stride st) by one block.
__device__ double sum_partials(const double *p, int n, int st, double *sh) {
    double s = 0.0;
    for (int i = threadIdx.x; i < n; i += blockDim.x) s += p[(size_t)i * st];
    return block_sum(s, sh);
}

__device__ __forceinline__ double kref_entry(int v, int w) {
    int nd = __popc(v ^ w);
    return nd == 0 ? (1.0 / 3.0) : (nd == 1 ? 0.0 : (-1.0 / 12.0));
}

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
// setup: batched sweep of pivots [p0, p1) of symmetric row-major matrices.
// After sweeping a pivot set P the matrix holds
//   [ -A_PP^{-1}         A_PP^{-1} A_PQ            ]
//   [ A_QP A_PP^{-1}     A_QQ - A_QP A_PP^{-1} A_PQ ]
// i.e. interior elimination gives -K_II^{-1}, T = K_BI K_II^{-1} and S.
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(1024) k_sweep(const SweepDesc *descs, int *status) {
    extern __shared__ double row[];
    const SweepDesc d = descs[blockIdx.x];
    const int n = d.n, ld = d.ld;
    const int w = threadIdx.x >> 6, l = threadIdx.x & 63, nw = blockDim.x >> 6;
    for (int k = d.p0; k < d.p1; ++k) {
        const double *Ak = d.A + (size_t)k * ld;
        for (int j = threadIdx.x; j < n; j += blockDim.x) row[j] = Ak[j];
        __syncthreads();
        const double piv = row[k];
        const bool ok = (k < d.pos_end ? piv > 0.0 : piv < 0.0) && isfinite(piv);
        if (!ok) {
            if (threadIdx.x == 0) atomicMax(status, 1);
            return;
        }
        const double inv = 1.0 / piv;
        for (int i = w; i < n; i += nw) {
            double *Ai = d.A + (size_t)i * ld;
            if (i == k) {
                for (int j = l; j < n; j += 64) Ai[j] = (j == k) ? -inv : row[j] * inv;
            } else {
                const double ri = row[i] * inv;
                for (int j = l; j < n; j += 64) Ai[j] = (j == k) ? ri : Ai[j] - ri * row[j];
            }
        }
        __syncthreads();
    }
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
// setup: pack a symmetric n x n block (+ an n x nc block) into 16x16 tiles.
// Tile row I holds tiles (I, I..nt-1) then (I, nt..nt+ntc-1); each tile is
// row-major.  Value = sign * src[i][j] * D[i] * D[j]  (Phi block: * D[i]).
// ---------------------------------------------------------------------------
__device__ __forceinline__ void store_conv(double *p, double v) { *p = v; }
__device__ __forceinline__ void store_conv(float *p, double v) { *p = (float)v; }
__device__ __forceinline__ void store_conv(uint16_t *p, double v) {
    // round-to-nearest-even float32 -> bfloat16
    float f = (float)v;
    uint32_t u = __float_as_uint(f);
    uint32_t r = u + 0x7fffu + ((u >> 16) & 1u);
    *p = (uint16_t)(r >> 16);
}

template <typename T>
__global__ void __launch_bounds__(256) k_pack(const PackDesc *descs, T *dst) {
    const PackDesc d = descs[blockIdx.x];
    const int nt = (d.n + TILE - 1) / TILE, ntc = (d.nc + TILE - 1) / TILE;
    int64_t base = 0;
    for (int I = 0; I < nt; ++I) {
        const int nrow = nt - I + ntc;
        for (int e = threadIdx.x; e < nrow * 256; e += blockDim.x) {
            const int q = e >> 8, r = (e >> 4) & 15, c = e & 15;
            const int J = I + q;
            const int gi = I * TILE + r;
            double v = 0.0;
            if (J < nt) {
                const int gj = J * TILE + c;
                if (gi < d.n && gj < d.n) {
                    v = d.sign * d.src[(size_t)gi * d.ld + gj];
                    if (d.D) v *= d.D[gi] * d.D[gj];
                }
            } else {
                const int gq = (J - nt) * TILE + c;
                if (gi < d.n && gq < d.nc) {
                    v = d.sign * d.phi[(size_t)gi * d.ldphi + gq];
                    if (d.D) v *= d.D[gi];
                }
            }
            store_conv(dst + d.dst + (base + q) * 256 + r * 16 + c, v);
        }
        base += nrow;
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
// hot path: batched tiled symmetric matrix-vector product with gather
//   y_i = Op_i x_i,  x_i = x[gB_i]   (one work-group per subdomain)
//   c_i = Phi_i^T x_i                (optional extra tile columns)
// FP64 tiles: lane l holds rows l/8 and l/8+8, columns 2(l%8), 2(l%8)+1.
// FP32/BF16 tiles: lane l holds row l/4, columns 4(l%4)..4(l%4)+3.
// Row sums of a tile-row are kept in registers and flushed once per row;
// column (transposed) sums are butterfly-reduced per tile into a per-wave LDS
// accumulator, so the result is deterministic.
// ---------------------------------------------------------------------------
template <typename T>
struct TileTraits;
template <>
struct TileTraits<double> {
    using acc = double;
};
template <>
struct TileTraits<float> {
    using acc = float;
};
template <>
struct TileTraits<uint16_t> {
    using acc = float;
};

__device__ __forceinline__ float bf2f(uint32_t h) { return __uint_as_float(h << 16); }

typedef double dvec2 __attribute__((ext_vector_type(2)));
typedef float fvec4 __attribute__((ext_vector_type(4)));
typedef unsigned int uvec2 __attribute__((ext_vector_type(2)));

template <typename T, int NW, int U>
__global__ void __launch_bounds__(NW * 64) k_symv(SymvArgs a) {
    using ACC = typename TileTraits<T>::acc;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    if (a.ctl && a.gated && a.ctl->done) return;
    const int sub = blockIdx.x;
    const int n = a.nB[sub];
    const int nt = (n + TILE - 1) / TILE;
    const int ncs = a.nc ? a.nc[sub] : 0;
    const int ntc = a.nc ? (ncs + TILE - 1) / TILE : 0;
    const int npad = nt * TILE;
    ACC *xs = reinterpret_cast<ACC *>(smem_raw);
    ACC *yw = xs + npad;
    ACC *cw = yw + NW * npad;
    const int tid = threadIdx.x, w = tid >> 6, l = tid & 63;
    const int boff = a.b_off[sub];
    for (int k = tid; k < npad; k += NW * 64) xs[k] = k < n ? (ACC)a.x[a.gB[boff + k]] : (ACC)0;
    for (int k = tid; k < NW * npad; k += NW * 64) yw[k] = (ACC)0;
    for (int k = tid; k < NW * ntc * TILE; k += NW * 64) cw[k] = (ACC)0;
    __syncthreads();

    const T *tb = reinterpret_cast<const T *>(a.tiles) + a.t_off[sub];
    const int64_t ntiles = (int64_t)nt * (nt + 1) / 2 + (int64_t)nt * ntc;
    const int64_t t0 = ntiles * w / NW, t1 = ntiles * (w + 1) / NW;
    int I = 0;
    int64_t rs = 0;
    while (I < nt && rs + (nt - I + ntc) <= t0) { rs += nt - I + ntc; ++I; }
    int J = I + (int)(t0 - rs);
    ACC *myy = yw + w * npad;
    ACC *myc = cw + w * ntc * TILE;

    if constexpr (sizeof(T) == 8) {
        const int r0 = l >> 3, c0 = 2 * (l & 7);
        ACC ra = 0, rb = 0;
        for (int64_t t = t0; t < t1; t += U) {
            dvec2 va[U], vb[U];
#pragma unroll
            for (int u = 0; u < U; ++u) {
                if (t + u < t1) {
                    const dvec2 *tp = reinterpret_cast<const dvec2 *>(tb + (t + u) * 256);
                    va[u] = __builtin_nontemporal_load(tp + l);
                    vb[u] = __builtin_nontemporal_load(tp + 64 + l);
                }
            }
#pragma unroll
            for (int u = 0; u < U; ++u) {
                if (t + u >= t1) break;
                const double v00 = va[u].x, v01 = va[u].y, v10 = vb[u].x, v11 = vb[u].y;
                const double xi0 = xs[I * TILE + r0], xi1 = xs[I * TILE + r0 + 8];
                if (J < nt) {
                    const double xj0 = xs[J * TILE + c0], xj1 = xs[J * TILE + c0 + 1];
                    ra += v00 * xj0 + v01 * xj1;
                    rb += v10 * xj0 + v11 * xj1;
                }
                if (J != I) {
                    double s0 = v00 * xi0 + v10 * xi1;
                    double s1 = v01 * xi0 + v11 * xi1;
                    s0 += __shfl_xor(s0, 8); s1 += __shfl_xor(s1, 8);
                    s0 += __shfl_xor(s0, 16); s1 += __shfl_xor(s1, 16);
                    s0 += __shfl_xor(s0, 32); s1 += __shfl_xor(s1, 32);
                    if (l < 8) {
                        ACC *dst = (J < nt) ? (myy + J * TILE + c0) : (myc + (J - nt) * TILE + c0);
                        dst[0] += s0;
                        dst[1] += s1;
                    }
                }
                if (++J == nt + ntc) {
                    ra += __shfl_xor(ra, 1); rb += __shfl_xor(rb, 1);
                    ra += __shfl_xor(ra, 2); rb += __shfl_xor(rb, 2);
                    ra += __shfl_xor(ra, 4); rb += __shfl_xor(rb, 4);
                    if ((l & 7) == 0) { myy[I * TILE + r0] += ra; myy[I * TILE + r0 + 8] += rb; }
                    ra = 0; rb = 0;
                    ++I;
                    J = I;
                }
            }
        }
        if (t1 > t0 && J != I) {   // flush a partially processed tile row
            ra += __shfl_xor(ra, 1); rb += __shfl_xor(rb, 1);
            ra += __shfl_xor(ra, 2); rb += __shfl_xor(rb, 2);
            ra += __shfl_xor(ra, 4); rb += __shfl_xor(rb, 4);
            if ((l & 7) == 0) { myy[I * TILE + r0] += ra; myy[I * TILE + r0 + 8] += rb; }
        }
    } else {
        const int r0 = l >> 2, c0 = 4 * (l & 3);
        ACC ra = 0;
        for (int64_t t = t0; t < t1; t += U) {
            float v[U][4];
#pragma unroll
            for (int u = 0; u < U; ++u) {
                if (t + u < t1) {
                    if constexpr (sizeof(T) == 4) {
                        const fvec4 q = __builtin_nontemporal_load(reinterpret_cast<const fvec4 *>(tb + (t + u) * 256) + l);
                        v[u][0] = q.x; v[u][1] = q.y; v[u][2] = q.z; v[u][3] = q.w;
                    } else {
                        const uvec2 q = __builtin_nontemporal_load(reinterpret_cast<const uvec2 *>(tb + (t + u) * 256) + l);
                        v[u][0] = bf2f(q.x & 0xffffu); v[u][1] = bf2f(q.x >> 16);
                        v[u][2] = bf2f(q.y & 0xffffu); v[u][3] = bf2f(q.y >> 16);
                    }
                }
            }
#pragma unroll
            for (int u = 0; u < U; ++u) {
                if (t + u >= t1) break;
                const float xi = xs[I * TILE + r0];
                if (J < nt) {
                    const float *xj = xs + J * TILE + c0;
                    ra += v[u][0] * xj[0] + v[u][1] * xj[1] + v[u][2] * xj[2] + v[u][3] * xj[3];
                }
                if (J != I) {
                    float s[4];
#pragma unroll
                    for (int q = 0; q < 4; ++q) {
                        s[q] = v[u][q] * xi;
                        s[q] += __shfl_xor(s[q], 4);
                        s[q] += __shfl_xor(s[q], 8);
                        s[q] += __shfl_xor(s[q], 16);
                        s[q] += __shfl_xor(s[q], 32);
                    }
                    if (l < 4) {
                        ACC *dst = (J < nt) ? (myy + J * TILE + c0) : (myc + (J - nt) * TILE + c0);
#pragma unroll
                        for (int q = 0; q < 4; ++q) dst[q] += s[q];
                    }
                }
                if (++J == nt + ntc) {
                    ra += __shfl_xor(ra, 1);
                    ra += __shfl_xor(ra, 2);
                    if ((l & 3) == 0) myy[I * TILE + r0] += ra;
                    ra = 0;
                    ++I;
                    J = I;
                }
            }
        }
        if (t1 > t0 && J != I) {
            ra += __shfl_xor(ra, 1);
            ra += __shfl_xor(ra, 2);
            if ((l & 3) == 0) myy[I * TILE + r0] += ra;
        }
    }
    __syncthreads();

    __shared__ double red[16];
    double dot = 0.0;
    for (int k = tid; k < n; k += NW * 64) {
        ACC s = 0;
        for (int q = 0; q < NW; ++q) s += yw[q * npad + k];
        const double yd = (double)s;
        a.y[boff + k] = yd;
        dot += (double)xs[k] * yd;
    }
    if (ncs) {
        const int coff = a.c_off[sub];
        for (int k = tid; k < ncs; k += NW * 64) {
            ACC s = 0;
            for (int q = 0; q < NW; ++q) s += cw[q * ntc * TILE + k];
            a.c[coff + k] = (double)s;
        }
    }
    if (!a.partial) return;
    dot = block_sum(dot, red);
    if (tid == 0) a.partial[sub] = dot;
    if (!last_block(&a.ctl->cnt[CNT_SYMV])) return;
    const double pAp = sum_partials(a.partial, gridDim.x, 1, red);
    if (tid == 0) {
        Ctl *c = a.ctl;
        c->pAp = pAp;
        if (a.mode == 1) {
            const double alpha = c->rho / pAp;
            c->alpha = alpha;
            if (!(pAp > 0.0) || !isfinite(alpha)) { c->status = BDDC_EBREAKDOWN; c->done = 1; }
            if (a.d_hist && c->j < a.hist_cap) { a.d_hist[c->j] = pAp; a.a_hist[c->j] = alpha; }
        }
    }
}

// ---------------------------------------------------------------------------
// hot path: assemble q = sum_i R_i^T q_i and do the PCG update (Alg. 1,
// lines 10-11): x += alpha p, r -= alpha q; ||r||^2; stopping test (Section 5).
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(256) k_update(UpdArgs a) {
    __shared__ double red[16];
    Ctl *c = a.ctl;
    if (c->done) return;
    const int g = blockIdx.x * blockDim.x + threadIdx.x;
    const double alpha = c->alpha;
    const int j = c->j;
    double rr = 0.0;
    if (g < a.n) {
        double q = 0.0;
        for (int k = a.ptr[g]; k < a.ptr[g + 1]; ++k) q += a.loc[a.idx[k]];
        const double xi = a.x[g] + alpha * a.p[g];
        const double ri = a.r[g] - alpha * q;
        a.x[g] = xi;
        a.r[g] = ri;
        rr = ri * ri;
        if (a.AP && c->record && j < a.cap) a.AP[(size_t)j * a.ld + g] = q;
    }
    rr = block_sum(rr, red);
    if (threadIdx.x == 0) a.partial[blockIdx.x] = rr;
    if (!last_block(&c->cnt[CNT_UPD])) return;
    const double tot = sum_partials(a.partial, gridDim.x, 1, red);
    if (threadIdx.x == 0) {
        c->rr = tot;
        c->j = j + 1;
        c->iter += 1;
        if (a.res_hist && c->iter < a.hist_cap) a.res_hist[c->iter] = tot;
        if (!isfinite(tot)) { c->status = BDDC_EBREAKDOWN; c->done = 1; }
        else if (tot < c->rtol2 * c->denom2) c->done = 1;
        else if (c->iter >= a.max_it) { c->status = BDDC_ENOTCONV; c->done = 1; }
    }
}

// ---------------------------------------------------------------------------
// hot path: z = sum_i R_i^T D_i w_i (eq. averaging_subdomain_solves, weights
// folded into the operators), rho = r^T z, t = (AW)^T z, then beta (Alg. 1,
// line 14) and mu = (W^T A W)^{-1} t (line 15) by the last block.
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(256) k_zasm(ZasmArgs a) {
    __shared__ double red[16];
    __shared__ double wred[4][RMAX + 1];
    Ctl *c = a.ctl;
    if (a.gated && c->done) return;
    const int g = blockIdx.x * blockDim.x + threadIdx.x;
    const int k = c->k;
    double z = 0.0;
    if (g < a.n) {
        for (int t = a.ptr[g]; t < a.ptr[g + 1]; ++t) z += a.loc[a.idx[t]];
        a.z[g] = z;
    }
    if (!a.partial) return;
    const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
    const int st = RMAX + 1;
    for (int col = 0; col <= k; ++col) {
        double v = 0.0;
        if (g < a.n) v = (col == 0) ? a.r[g] * z : a.AW[(size_t)(col - 1) * a.ld + g] * z;
        v = wave_sum(v);
        if (l == 0) wred[w][col] = v;
    }
    __syncthreads();
    if (threadIdx.x <= k) {
        double s = 0.0;
        for (int q = 0; q < (int)(blockDim.x >> 6); ++q) s += wred[q][threadIdx.x];
        a.partial[(size_t)blockIdx.x * st + threadIdx.x] = s;
    }
    if (!last_block(&c->cnt[CNT_ZASM])) return;
    __shared__ double tot[RMAX + 1];
    for (int col = 0; col <= k; ++col) {
        const double s = sum_partials(a.partial + col, gridDim.x, st, red);
        if (threadIdx.x == 0) tot[col] = s;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        const int j = c->j;
        const double rho = tot[0];
        double beta = 0.0;
        if (!a.first) {
            beta = rho / c->rho;
            if (a.b_hist && j >= 1 && j - 1 < a.hist_cap) a.b_hist[j - 1] = beta;
        }
        c->beta = beta;
        c->rho = rho;
        if (!(rho > 0.0) || !isfinite(rho)) { c->status = BDDC_EBREAKDOWN; c->done = 1; }
        if (a.rho_hist && j < a.hist_cap) a.rho_hist[j] = rho;
        // mu = (W^T A W)^{-1} t with the lower Cholesky factor Lc (k x k, row-major)
        double y[RMAX];
        for (int i = 0; i < k; ++i) {
            double s = tot[1 + i];
            for (int q = 0; q < i; ++q) s -= a.Lc[i * k + q] * y[q];
            y[i] = s / a.Lc[i * k + i];
        }
        for (int i = k - 1; i >= 0; --i) {
            double s = y[i];
            for (int q = i + 1; q < k; ++q) s -= a.Lc[q * k + i] * y[q];
            y[i] = s / a.Lc[i * k + i];
        }
        for (int i = 0; i < k; ++i) {
            c->mu[i] = y[i];
            if (a.mu_hist && j < a.hist_cap) a.mu_hist[(size_t)j * RMAX + i] = y[i];
        }
    }
}

// p = z + beta p - W mu  (Alg. 1, line 16; line 7 with beta = 0)
__global__ void __launch_bounds__(256) k_pupd(PupdArgs a) {
    Ctl *c = a.ctl;
    if (c->done) return;
    const int g = blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= a.n) return;
    const int k = c->k;
    double p = a.z[g] + c->beta * a.p[g];
    for (int q = 0; q < k; ++q) p -= a.W[(size_t)q * a.ld + g] * c->mu[q];
    a.p[g] = p;
    if (a.P && c->record && c->j < a.cap) a.P[(size_t)c->j * a.ld + g] = p;
}

// ---------------------------------------------------------------------------
// initial residual, deflated initial guess (Alg. 1, lines 3-4) and true residual
// ---------------------------------------------------------------------------
// mode 0: r = b - sum loc; ||r||^2 and W^T r partials; last block: gamma
//         (-> ctl->mu) when k > 0, else r0 statistics and the stopping test.
// mode 1: true residual: t = b - sum loc written to out; ||t||^2 -> true_rr.
__global__ void __launch_bounds__(256) k_resid(ResidArgs a) {
    __shared__ double red[16];
    __shared__ double wred[4][RMAX + 1];
    Ctl *c = a.ctl;
    const int g = blockIdx.x * blockDim.x + threadIdx.x;
    const int k = a.mode == 0 ? c->k : 0;
    double r = 0.0;
    if (g < a.n) {
        double q = 0.0;
        for (int t = a.ptr[g]; t < a.ptr[g + 1]; ++t) q += a.loc[a.idx[t]];
        r = a.b[g] - q;
        a.out[g] = r;
    }
    const int w = threadIdx.x >> 6, l = threadIdx.x & 63, st = RMAX + 1;
    for (int col = 0; col <= k; ++col) {
        double v = 0.0;
        if (g < a.n) v = (col == 0) ? r * r : a.W[(size_t)(col - 1) * a.ld + g] * r;
        v = wave_sum(v);
        if (l == 0) wred[w][col] = v;
    }
    __syncthreads();
    if (threadIdx.x <= k) {
        double s = 0.0;
        for (int q = 0; q < (int)(blockDim.x >> 6); ++q) s += wred[q][threadIdx.x];
        a.partial[(size_t)blockIdx.x * st + threadIdx.x] = s;
    }
    if (!last_block(&c->cnt[CNT_RES])) return;
    __shared__ double tot[RMAX + 1];
    for (int col = 0; col <= k; ++col) {
        const double s = sum_partials(a.partial + col, gridDim.x, st, red);
        if (threadIdx.x == 0) tot[col] = s;
    }
    __syncthreads();
    if (threadIdx.x != 0) return;
    if (a.mode == 1) { c->true_rr = tot[0]; return; }
    if (k == 0) {
        c->r0r0 = tot[0];
        c->denom2 = (a.stop_rule == 0) ? c->bb : tot[0];
        c->done = (tot[0] < c->rtol2 * c->denom2 || c->bb == 0.0) ? 1 : 0;
        return;
    }
    double y[RMAX];
    for (int i = 0; i < k; ++i) {
        double s = tot[1 + i];
        for (int q = 0; q < i; ++q) s -= a.Lc[i * k + q] * y[q];
        y[i] = s / a.Lc[i * k + i];
    }
    for (int i = k - 1; i >= 0; --i) {
        double s = y[i];
        for (int q = i + 1; q < k; ++q) s -= a.Lc[q * k + i] * y[q];
        y[i] = s / a.Lc[i * k + i];
    }
    for (int i = 0; i < k; ++i) c->mu[i] = y[i];
}

// x += W gamma; r -= AW gamma  (= b - A x_0); ||r||^2; stopping test on r_0
__global__ void __launch_bounds__(256) k_defl_init(DeflArgs a) {
    __shared__ double red[16];
    Ctl *c = a.ctl;
    const int g = blockIdx.x * blockDim.x + threadIdx.x;
    const int k = c->k;
    double rr = 0.0;
    if (g < a.n) {
        double x = a.x[g], r = a.r[g];
        for (int q = 0; q < k; ++q) {
            x += a.W[(size_t)q * a.ld + g] * c->mu[q];
            r -= a.AW[(size_t)q * a.ld + g] * c->mu[q];
        }
        a.x[g] = x;
        a.r[g] = r;
        rr = r * r;
    }
    rr = block_sum(rr, red);
    if (threadIdx.x == 0) a.partial[blockIdx.x] = rr;
    if (!last_block(&c->cnt[CNT_DEFL])) return;
    const double tot = sum_partials(a.partial, gridDim.x, 1, red);
    if (threadIdx.x == 0) {
        c->r0r0 = tot;
        c->denom2 = (a.stop_rule == 0) ? c->bb : tot;
        c->done = (tot < c->rtol2 * c->denom2 || c->bb == 0.0) ? 1 : 0;
    }
}

// ---------------------------------------------------------------------------
// condensation b = F_G - sum_i R_i^T T_i F_I and interior recovery (Section 3.1)
// on the swept local matrices [-K_II^{-1}, T_i^T; T_i, S_i]
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(256) k_cond_local(CondArgs a) {
    extern __shared__ double fI[];
    const int i = blockIdx.x;
    const int nI = a.nI[i], nloc = nI + a.nB[i];
    const double *K = a.K + a.k_off[i];
    const int ioff = a.i_off[i];
    for (int k = threadIdx.x; k < nI; k += blockDim.x) fI[k] = a.F[a.nodesI[ioff + k]];
    __syncthreads();
    for (int r = threadIdx.x; r < nloc; r += blockDim.x) {
        double s = 0.0;
        for (int k = 0; k < nI; ++k) s += K[(size_t)k * nloc + r] * fI[k];
        if (r < nI) a.yI[ioff + r] = -s;
        else a.t[a.b_off[i] + r - nI] = s;
    }
}

__global__ void __launch_bounds__(256) k_cond_asm(CondAsmArgs a) {
    __shared__ double red[16];
    const int g = blockIdx.x * blockDim.x + threadIdx.x;
    double bb = 0.0;
    if (g < a.n) {
        double s = a.F[a.gamma[g]];
        for (int k = a.ptr[g]; k < a.ptr[g + 1]; ++k) s -= a.loc[a.idx[k]];
        a.b[g] = s;
        bb = s * s;
    }
    bb = block_sum(bb, red);
    if (threadIdx.x == 0) a.partial[blockIdx.x] = bb;
    if (!last_block(&a.ctl->cnt[CNT_COND])) return;
    const double tot = sum_partials(a.partial, gridDim.x, 1, red);
    if (threadIdx.x == 0) a.ctl->bb = tot;
}

__global__ void __launch_bounds__(256) k_recover(RecArgs a) {
    extern __shared__ double xB[];
    const int i = blockIdx.x;
    const int nI = a.nI[i], nB = a.nB[i], nloc = nI + nB;
    const double *K = a.K + a.k_off[i];
    const int boff = a.b_off[i], ioff = a.i_off[i];
    for (int k = threadIdx.x; k < nB; k += blockDim.x) xB[k] = a.x[a.gB[boff + k]];
    __syncthreads();
    for (int r = threadIdx.x; r < nI; r += blockDim.x) {
        double s = a.yI[ioff + r];
        for (int k = 0; k < nB; ++k) s -= K[(size_t)(nI + k) * nloc + r] * xB[k];
        a.u[a.nodesI[ioff + r]] = s;
    }
}

__global__ void __launch_bounds__(256) k_scatter_gamma(int n, const int32_t *gamma, const double *x, double *u) {
    const int g = blockIdx.x * blockDim.x + threadIdx.x;
    if (g < n) u[gamma[g]] = x[g];
}

// ---------------------------------------------------------------------------
// coarse levels
// ---------------------------------------------------------------------------
// Level-2 phase A (one block per subregion): gather the coarse residual of
// the subregion's coarse DOFs, interior pre-solve v_I = K_II^{-1} r_I and its
// interface coupling t = K_BI K_II^{-1} r_I.
__global__ void __launch_bounds__(256) k_l2_a(L2Args a) {
    extern __shared__ double rL[];
    if (a.ctl->done) return;
    const int j = blockIdx.x;
    const int nL = a.nL[j], nI = a.nI2[j], nB = nL - nI;
    const int loff = a.L_off[j];
    for (int q = threadIdx.x; q < nL; q += blockDim.x) {
        const int cdof = a.L[loff + q];
        double s = 0.0;
        for (int k = a.cptr[cdof]; k < a.cptr[cdof + 1]; ++k) s += a.locc[a.cidx_asm[k]];
        rL[q] = s;
    }
    __syncthreads();
    const double *K = a.K2 + a.K2_off[j];
    const int i2 = a.I2_off[j], b2 = a.B2_off[j];
    for (int q = threadIdx.x; q < nL; q += blockDim.x) {
        double s = 0.0;
        for (int b = 0; b < nI; ++b) s += K[(size_t)q * nL + b] * rL[b];
        if (q < nI) a.vI2[i2 + q] = -s;
        else { a.t2[b2 + q - nI] = s; a.rB2[b2 + q - nI] = rL[q]; }
    }
    (void)nB;
}

// Level-2 phase B (one block per subregion): interface residual
// g = r_G - sum_j R_j^T t_j, then u = D N D g and c3 = (D Phi)^T g.
__global__ void __launch_bounds__(256) k_l2_b(L2Args a) {
    extern __shared__ double gs[];
    if (a.ctl->done) return;
    const int j = blockIdx.x;
    const int nB = a.nL[j] - a.nI2[j];
    const int b2 = a.B2_off[j];
    for (int k = threadIdx.x; k < nB; k += blockDim.x) {
        const int gi = a.g2[b2 + k];
        double s = a.rB2[b2 + k];
        for (int t = a.asm2_ptr[gi]; t < a.asm2_ptr[gi + 1]; ++t) s -= a.t2[a.asm2_idx[t]];
        gs[k] = s;
    }
    __syncthreads();
    const double *N = a.N2 + a.N2_off[j];
    for (int k = threadIdx.x; k < nB; k += blockDim.x) {
        double s = 0.0;
        for (int q = 0; q < nB; ++q) s += N[(size_t)k * nB + q] * gs[q];
        a.u2[b2 + k] = s;
    }
    const int nc3 = a.nc3[j], c3o = a.C3_off[j];
    const double *Ph = a.Phi2 + a.P2_off[j];
    for (int q = threadIdx.x; q < nc3; q += blockDim.x) {
        double s = 0.0;
        for (int k = 0; k < nB; ++k) s += Ph[(size_t)k * nc3 + q] * gs[k];
        a.c3loc[c3o + q] = s;
    }
}

// Dense coarse solve u = (-Kneg) r with Kneg = -K^{-1} (swept); r gathered
// from local contributions (level-3 of three levels, or K_C of two levels).
__global__ void __launch_bounds__(256) k_coarse_solve(CoarseArgs a) {
    extern __shared__ double rs[];
    if (a.ctl->done) return;
    for (int q = threadIdx.x; q < a.n; q += blockDim.x) {
        double s = 0.0;
        for (int k = a.ptr[q]; k < a.ptr[q + 1]; ++k) s += a.loc[a.idx[k]];
        rs[q] = s;
    }
    __syncthreads();
    const int r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= a.n) return;
    double s = 0.0;
    for (int q = 0; q < a.n; ++q) s += a.Kneg[(size_t)q * a.n + r] * rs[q];
    a.u[r] = -s;
}

// Prolongation (one block per level-1 subdomain): obtain the coarse solution
// on the subdomain's coarse DOFs (directly for two levels; for three levels
// by assembling the level-2 interface solution of its subregion and the
// interior post-correction x_I = v_I - T^T x_G), then u_i += (D Phi_i) u_C.
template <typename T>
__global__ void __launch_bounds__(256) k_prolong(ProlArgs a) {
    extern __shared__ double sm[];
    if (a.ctl->done) return;
    const int i = blockIdx.x;
    const int nc = a.nc[i], coff = a.c_off[i];
    double *uC = sm;                 // nc
    if (!a.three) {
        for (int q = threadIdx.x; q < nc; q += blockDim.x) uC[q] = a.uCg[a.cidx[coff + q]];
    } else {
        const int j = a.sr_of_sub[i];
        const int nL = a.nL[j], nI = a.nI2[j], nB = nL - nI;
        double *uL = sm + nc;        // nL
        const int b2 = a.B2_off[j];
        for (int k = threadIdx.x; k < nB; k += blockDim.x) {
            const int gi = a.g2[b2 + k];
            double s = 0.0;
            for (int t = a.asm2_ptr[gi]; t < a.asm2_ptr[gi + 1]; ++t) {
                const int pos = a.asm2_idx[t];
                const int jj = a.pos_sr[pos];
                const int kk = pos - a.B2_off[jj];
                const int n3j = a.nc3[jj];
                const double *ph = a.Phi2 + a.P2_off[jj] + (size_t)kk * n3j;
                const int32_t *c3 = a.c3 + a.C3_off[jj];
                double v = a.u2[pos];
                for (int q = 0; q < n3j; ++q) v += ph[q] * a.u3[c3[q]];
                s += v;
            }
            uL[nI + k] = s;
        }
        __syncthreads();
        const double *K = a.K2 + a.K2_off[j];
        const int i2 = a.I2_off[j];
        for (int q = threadIdx.x; q < nI; q += blockDim.x) {
            double s = a.vI2[i2 + q];
            for (int k = 0; k < nB; ++k) s -= K[(size_t)(nI + k) * nL + q] * uL[nI + k];
            uL[q] = s;
        }
        __syncthreads();
        for (int q = threadIdx.x; q < nc; q += blockDim.x) uC[q] = uL[a.cL[coff + q]];
    }
    __syncthreads();
    const int n = a.nB[i], nt = (n + TILE - 1) / TILE;
    const T *tb = reinterpret_cast<const T *>(a.tiles) + a.t_off[i];
    const int boff = a.b_off[i];
    for (int k = threadIdx.x; k < n; k += blockDim.x) {
        const int I = k >> 4, r = k & 15;
        const int64_t rowoff = (int64_t)I * (nt + ((nc + TILE - 1) / TILE)) - (int64_t)I * (I - 1) / 2 + (nt - I);
        double s = 0.0;
        for (int q = 0; q < nc; ++q) {
            const T *tp = tb + (rowoff + (q >> 4)) * 256 + r * 16 + (q & 15);
            double v;
            if constexpr (sizeof(T) == 8) v = *tp;
            else if constexpr (sizeof(T) == 4) v = (double)*tp;
            else v = (double)bf2f((uint32_t)*tp);
            s += v * uC[q];
        }
        a.locu[boff + k] += s;
    }
}

// ---------------------------------------------------------------------------
// recycling: out[:, c] = sum_q V[:, q] Y[q][c] for two blocks [W, P] (and
// [AW, AP]), column-major with leading dimension ld
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(256) k_recycle_gemm(GemmArgs a) {
    const int g = blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= a.n) return;
    for (int c0 = 0; c0 < a.ncol; c0 += 8) {
        double acc[8] = {0, 0, 0, 0, 0, 0, 0, 0};
        for (int q = 0; q < a.k1 + a.k2; ++q) {
            const double v = q < a.k1 ? a.V1[(size_t)q * a.ld + g] : a.V2[(size_t)(q - a.k1) * a.ld + g];
            const double *y = a.Y + (size_t)q * a.ldy + c0;
#pragma unroll
            for (int c = 0; c < 8; ++c) acc[c] += v * y[c];
        }
#pragma unroll
        for (int c = 0; c < 8; ++c)
            if (c0 + c < a.ncol) a.out[(size_t)(c0 + c) * a.ld + g] = acc[c];
    }
}

// G = X^T Y (k x k) with X, Y column-major n x k; deterministic two-stage sum
__global__ void __launch_bounds__(256) k_gram(GramArgs a) {
    __shared__ double red[16];
    const int k = a.k;
    const int64_t per = (a.n + gridDim.x - 1) / gridDim.x;
    const int64_t g0 = (int64_t)blockIdx.x * per, g1 = min((int64_t)a.n, g0 + per);
    for (int pq = 0; pq < k * k; ++pq) {
        const int p = pq / k, q = pq - p * k;
        if (q < p) continue;
        double s = 0.0;
        for (int64_t g = g0 + threadIdx.x; g < g1; g += blockDim.x)
            s += a.X[(size_t)p * a.ld + g] * a.Y[(size_t)q * a.ld + g];
        s = block_sum(s, red);
        if (threadIdx.x == 0) a.partial[(size_t)blockIdx.x * k * k + pq] = s;
    }
    if (!last_block(&a.ctl->cnt[CNT_GRAM])) return;
    for (int pq = 0; pq < k * k; ++pq) {
        const int p = pq / k, q = pq - p * k;
        if (q < p) continue;
        const double s = sum_partials(a.partial + pq, gridDim.x, k * k, red);
        if (threadIdx.x == 0) { a.out[p * k + q] = s; a.out[q * k + p] = s; }
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

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------
static inline unsigned nblk(int64_t n, int b) { return (unsigned)((n + b - 1) / b); }

void launch_assemble(const AsmDesc *d, int n, hipStream_t s) {
    hipLaunchKernelGGL(k_assemble, dim3(n), dim3(256), 0, s, d);
}
void launch_sweep(const SweepDesc *d, int n, int maxn, int *status, hipStream_t s) {
    hipLaunchKernelGGL(k_sweep, dim3(n), dim3(1024), (size_t)maxn * sizeof(double), s, d, status);
}
void set_sweep_smem_limit(size_t bytes) {
    if (bytes > 65536) hipFuncSetAttribute((const void *)k_sweep, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
}
void launch_build_saddle(const SaddleDesc *d, int n, hipStream_t s) {
    hipLaunchKernelGGL(k_build_saddle, dim3(n), dim3(256), 0, s, d);
}
void launch_pack(const PackDesc *d, int n, int prec, void *dst, hipStream_t s) {
    if (prec == 64) hipLaunchKernelGGL(k_pack<double>, dim3(n), dim3(256), 0, s, d, (double *)dst);
    else if (prec == 32) hipLaunchKernelGGL(k_pack<float>, dim3(n), dim3(256), 0, s, d, (float *)dst);
    else hipLaunchKernelGGL(k_pack<uint16_t>, dim3(n), dim3(256), 0, s, d, (uint16_t *)dst);
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

constexpr int SYMV_NW = 8;
constexpr int SYMV_U = 4;
size_t symv_smem(int prec, int max_nt, int max_ntc) {
    const size_t acc = prec == 64 ? 8 : 4;
    return acc * ((size_t)max_nt * TILE * (1 + SYMV_NW) + (size_t)SYMV_NW * max_ntc * TILE);
}
void launch_symv(const SymvArgs &a, int prec, int nsub, size_t smem, hipStream_t s) {
    if (prec == 64)
        hipLaunchKernelGGL((k_symv<double, SYMV_NW, SYMV_U>), dim3(nsub), dim3(SYMV_NW * 64), smem, s, a);
    else if (prec == 32)
        hipLaunchKernelGGL((k_symv<float, SYMV_NW, SYMV_U>), dim3(nsub), dim3(SYMV_NW * 64), smem, s, a);
    else
        hipLaunchKernelGGL((k_symv<uint16_t, SYMV_NW, SYMV_U>), dim3(nsub), dim3(SYMV_NW * 64), smem, s, a);
}
void set_symv_smem_limit(size_t bytes) {
    hipFuncSetAttribute((const void *)k_symv<double, SYMV_NW, SYMV_U>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
    hipFuncSetAttribute((const void *)k_symv<float, SYMV_NW, SYMV_U>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
    hipFuncSetAttribute((const void *)k_symv<uint16_t, SYMV_NW, SYMV_U>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
}
void launch_update(const UpdArgs &a, hipStream_t s) {
    hipLaunchKernelGGL(k_update, dim3(nblk(a.n, 256)), dim3(256), 0, s, a);
}
void launch_zasm(const ZasmArgs &a, hipStream_t s) {
    hipLaunchKernelGGL(k_zasm, dim3(nblk(a.n, 256)), dim3(256), 0, s, a);
}
void launch_pupd(const PupdArgs &a, hipStream_t s) {
    hipLaunchKernelGGL(k_pupd, dim3(nblk(a.n, 256)), dim3(256), 0, s, a);
}
void launch_resid(const ResidArgs &a, hipStream_t s) {
    hipLaunchKernelGGL(k_resid, dim3(nblk(a.n, 256)), dim3(256), 0, s, a);
}
void launch_defl_init(const DeflArgs &a, hipStream_t s) {
    hipLaunchKernelGGL(k_defl_init, dim3(nblk(a.n, 256)), dim3(256), 0, s, a);
}
void launch_cond_local(const CondArgs &a, int nsub, int max_nI, hipStream_t s) {
    hipLaunchKernelGGL(k_cond_local, dim3(nsub), dim3(256), (size_t)max_nI * 8, s, a);
}
void launch_cond_asm(const CondAsmArgs &a, hipStream_t s) {
    hipLaunchKernelGGL(k_cond_asm, dim3(nblk(a.n, 256)), dim3(256), 0, s, a);
}
void launch_recover(const RecArgs &a, int nsub, int max_nB, hipStream_t s) {
    hipLaunchKernelGGL(k_recover, dim3(nsub), dim3(256), (size_t)max_nB * 8, s, a);
}
void launch_scatter_gamma(int n, const int32_t *gamma, const double *x, double *u, hipStream_t s) {
    hipLaunchKernelGGL(k_scatter_gamma, dim3(nblk(n, 256)), dim3(256), 0, s, n, gamma, x, u);
}
void launch_l2_a(const L2Args &a, int nsr, int max_nL, hipStream_t s) {
    hipLaunchKernelGGL(k_l2_a, dim3(nsr), dim3(256), (size_t)max_nL * 8, s, a);
}
void launch_l2_b(const L2Args &a, int nsr, int max_nL, hipStream_t s) {
    hipLaunchKernelGGL(k_l2_b, dim3(nsr), dim3(256), (size_t)max_nL * 8, s, a);
}
void launch_coarse_solve(const CoarseArgs &a, hipStream_t s) {
    hipLaunchKernelGGL(k_coarse_solve, dim3(nblk(a.n, 256)), dim3(256), (size_t)a.n * 8, s, a);
}
void launch_prolong(const ProlArgs &a, int prec, int nsub, size_t smem, hipStream_t s) {
    if (prec == 64) hipLaunchKernelGGL(k_prolong<double>, dim3(nsub), dim3(256), smem, s, a);
    else if (prec == 32) hipLaunchKernelGGL(k_prolong<float>, dim3(nsub), dim3(256), smem, s, a);
    else hipLaunchKernelGGL(k_prolong<uint16_t>, dim3(nsub), dim3(256), smem, s, a);
}
void launch_recycle_gemm(const GemmArgs &a, hipStream_t s) {
    hipLaunchKernelGGL(k_recycle_gemm, dim3(nblk(a.n, 256)), dim3(256), 0, s, a);
}
void launch_gram(const GramArgs &a, int nblocks, hipStream_t s) {
    hipLaunchKernelGGL(k_gram, dim3(nblocks), dim3(256), 0, s, a);
}
void launch_elem_grad(const GradArgs &a, hipStream_t s) {
    hipLaunchKernelGGL(k_elem_grad, dim3(nblk(a.n_elem, 256)), dim3(256), 0, s, a);
}
void launch_copy(int64_t n, const double *src, double *dst, hipStream_t s) {
    if (n > 0) hipLaunchKernelGGL(k_copy, dim3(nblk(n, 256)), dim3(256), 0, s, n, src, dst);
}

}  // namespace bddc
