// gfx950 kernels of one deflated-PCG iteration (Algorithm 1) preconditioned
// by two- or three-level BDDC (Section 3.2), on the interface problem of
// Section 3.1.
//
// One iteration is a fixed chain of kernels that can be captured once as a
// graph and replayed:
//   k_symv (S)   q_i = S_i p_i                      Alg. 1 line 9 (A p)
//   k_update     alpha, x += alpha p, r -= alpha q  lines 9-11
//   k_symv (N)   stopping test (Section 5); u_i = D N_i D r_i and the
//                coarse residual partials c_i = (D Phi_i)^T r_i
//   coarse       k_coarse_dense (two levels, or three levels in explicit form);
//                three levels as a chain: k_l2_a, k_l2_b, level 3 by the
//                dense product, k_l2_d
//   k_prolong    w_i = u_i + D Phi_i u_C            eq. averaging_subdomain_solves
//   k_zasm       z = sum_i R_i^T w_i, r^T z, (AW)^T z   line 13
//   k_pupd       beta, mu, p = z + beta p - W mu    lines 14-16
// A converged or failed solve sets ctl->done; every later kernel returns at
// once, so replaying more iterations than needed is harmless.
//
// Reductions never cross blocks inside a kernel: a producer writes one
// partial per block (or per work item), column by column, and every block of
// the consuming kernel sums them in index order, so all blocks see bitwise
// the same scalars and every run gives the same result.
#include <hip/hip_runtime.h>

#include "devutil.h"
#include "internal.h"
#include "kernels.h"

namespace bddc {

using dev::block_sum;
using dev::block_sum_cols;
using dev::block_sum_contig;
using dev::wave_sum;
using dev::wave_sum_contig;

namespace {

template <typename T>
struct Acc {
    using type = double;
};
template <>
struct Acc<float> {
    using type = float;
};
template <>
struct Acc<uint16_t> {
    using type = float;
};

typedef unsigned int uvec2 __attribute__((ext_vector_type(2)));

typedef unsigned int uvec4 __attribute__((ext_vector_type(4)));

// Buffer resource over `bytes` bytes from p (raw, unswizzled): loads past the
// end return zero without a memory access.
__device__ __forceinline__ __amdgpu_buffer_rsrc_t tile_rsrc(const void *p, int bytes) {
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void *>(p), 0, bytes, 0x00020000);
}
constexpr int LOAD_NT = 2;          // non-temporal: each tile is read once per product

// Element i of a float64 array through a buffer resource of `n` elements:
// zero past the end, without a memory access.  A fixed-count loop of such
// loads needs no per-element condition, so the loads are all issued before
// the first wait.  Byte offsets below 2^31.
__device__ __forceinline__ __amdgpu_buffer_rsrc_t vec_rsrc(const double *p, int64_t n) {
    return tile_rsrc(p, (int)(n * 8));
}
__device__ __forceinline__ double ld_rc(__amdgpu_buffer_rsrc_t r, int64_t i) {
    const uvec2 v = __builtin_amdgcn_raw_buffer_load_b64(r, (int)(i * 8), 0, 0);
    return __hiloint2double(v.y, v.x);
}

// The four values lane l holds of a 16x16 tile: rows 4*(l/16)+i, column l%16
// (element order of tile_index); tile t of the resource (the whole offset is
// in the vector operand, which is what the range check sees).  settle() waits for
// a fragment that is not going to be used (a loop exit), so that no path
// reaches the loop head with its load outstanding.
template <typename T>
struct Frag;
template <>
struct Frag<double> {
    uvec4 a, b;
    __device__ __forceinline__ void load(__amdgpu_buffer_rsrc_t r, int t, int l) {
        a = __builtin_amdgcn_raw_buffer_load_b128(r, t * 2048 + l * 16, 0, LOAD_NT);
        b = __builtin_amdgcn_raw_buffer_load_b128(r, t * 2048 + 1024 + l * 16, 0, LOAD_NT);
    }
    __device__ __forceinline__ void settle() const { asm volatile("" ::"v"(a), "v"(b)); }
    __device__ __forceinline__ void get(double v[4]) const {
        v[0] = __hiloint2double(a.y, a.x); v[1] = __hiloint2double(a.w, a.z);
        v[2] = __hiloint2double(b.y, b.x); v[3] = __hiloint2double(b.w, b.z);
    }
};
template <>
struct Frag<float> {
    uvec4 a;
    __device__ __forceinline__ void load(__amdgpu_buffer_rsrc_t r, int t, int l) {
        a = __builtin_amdgcn_raw_buffer_load_b128(r, t * 1024 + l * 16, 0, LOAD_NT);
    }
    __device__ __forceinline__ void settle() const { asm volatile("" ::"v"(a)); }
    __device__ __forceinline__ void get(float v[4]) const {
        v[0] = __uint_as_float(a.x); v[1] = __uint_as_float(a.y);
        v[2] = __uint_as_float(a.z); v[3] = __uint_as_float(a.w);
    }
};
template <>
struct Frag<uint16_t> {
    uvec2 a;
    __device__ __forceinline__ void load(__amdgpu_buffer_rsrc_t r, int t, int l) {
        a = __builtin_amdgcn_raw_buffer_load_b64(r, t * 512 + l * 8, 0, LOAD_NT);
    }
    __device__ __forceinline__ void settle() const { asm volatile("" ::"v"(a)); }
    __device__ __forceinline__ void get(float v[4]) const {
        v[0] = dev::bf16_to_f32(a.x & 0xffffu);
        v[1] = dev::bf16_to_f32(a.x >> 16);
        v[2] = dev::bf16_to_f32(a.y & 0xffffu);
        v[3] = dev::bf16_to_f32(a.y >> 16);
    }
};

// Cross-lane moves without LDS: DPP within rows of 16 lanes, and the gfx950
// row-swap permutes across rows.  Every lane of the wave must be active.
template <int CTRL>
__device__ __forceinline__ float dpp(float v) {
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), CTRL, 0xf, 0xf, false));
}
template <int CTRL>
__device__ __forceinline__ double dpp(double v) {
    const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(v), CTRL, 0xf, 0xf, false);
    const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(v), CTRL, 0xf, 0xf, false);
    return __hiloint2double(hi, lo);
}
constexpr int DPP_XOR1 = 0xB1;      // quad_perm [1,0,3,2]
constexpr int DPP_XOR2 = 0x4E;      // quad_perm [2,3,0,1]
constexpr int DPP_HALF_MIRROR = 0x141;  // lane i <-> i ^ 7 within 8 lanes
constexpr int DPP_ROR8 = 0x128;     // lane i <-> i ^ 8 within 16 lanes

// v + v[l ^ 16] and then + [l ^ 32]: the sum over the four lanes l % 16 + 16 g.
__device__ __forceinline__ float col_sum4(float v) {
    auto p = __builtin_amdgcn_permlane16_swap(__float_as_uint(v), __float_as_uint(v), false, false);
    v = __uint_as_float(p[0]) + __uint_as_float(p[1]);
    auto q = __builtin_amdgcn_permlane32_swap(__float_as_uint(v), __float_as_uint(v), false, false);
    return __uint_as_float(q[0]) + __uint_as_float(q[1]);
}
__device__ __forceinline__ double col_sum4(double v) {
    auto pl = __builtin_amdgcn_permlane16_swap(__double2loint(v), __double2loint(v), false, false);
    auto ph = __builtin_amdgcn_permlane16_swap(__double2hiint(v), __double2hiint(v), false, false);
    v = __hiloint2double(ph[0], pl[0]) + __hiloint2double(ph[1], pl[1]);
    auto ql = __builtin_amdgcn_permlane32_swap(__double2loint(v), __double2loint(v), false, false);
    auto qh = __builtin_amdgcn_permlane32_swap(__double2hiint(v), __double2hiint(v), false, false);
    return __hiloint2double(qh[0], ql[0]) + __hiloint2double(qh[1], ql[1]);
}

// Sums of ra[0..3] over the 16 lanes of a row of the wave, by exchange:
// lanes with bit 3 set keep rows 2, 3 and pass rows 0, 1 to lane ^ 8 (and
// the converse), then bit 2 halves again against the mirrored lane, and two
// quad swaps finish.  Returns, in every lane, the full sum of ra[cl >> 2].
template <typename A>
__device__ __forceinline__ A row_sum4(const A (&ra)[4], int cl) {
    const bool b3 = (cl & 8) != 0, b2 = (cl & 4) != 0;
    A k0 = b3 ? ra[2] : ra[0], k1 = b3 ? ra[3] : ra[1];
    const A s0 = b3 ? ra[0] : ra[2], s1 = b3 ? ra[1] : ra[3];
    k0 += dpp<DPP_ROR8>(s0);
    k1 += dpp<DPP_ROR8>(s1);
    A m = b2 ? k1 : k0;
    const A sd = b2 ? k0 : k1;
    m += dpp<DPP_HALF_MIRROR>(sd);
    m += dpp<DPP_XOR1>(m);
    m += dpp<DPP_XOR2>(m);
    return m;
}

__device__ __forceinline__ double to_d(double v) { return v; }
__device__ __forceinline__ double to_d(float v) { return (double)v; }
__device__ __forceinline__ double to_d(uint16_t v) { return (double)dev::bf16_to_f32(v); }

// Sum of the partial products listed for assembled entry t (fixed order).
__device__ __forceinline__ double gather_sum(const Gather &G, int64_t t) {
    const int e0 = G.ptr[t], e1 = G.ptr[t + 1];
    double s = 0.0;
    int e = e0;
    for (; e + 3 < e1; e += 4) {
        const double a0 = G.part[G.idx[e]], a1 = G.part[G.idx[e + 1]];
        const double a2 = G.part[G.idx[e + 2]], a3 = G.part[G.idx[e + 3]];
        s += a0; s += a1; s += a2; s += a3;
    }
    for (; e < e1; ++e) s += G.part[G.idx[e]];
    return s;
}

// Stopping test of Section 5 (eq. stopping_rhs, or eq. stopping_residual with
// stop_rule 1) on the residual whose per-block ||r||^2 partials are in
// rr_part.  first: the first test of a solve, on r_0 (zero iterations
// allowed); otherwise after the residual update, `iter` loop passes done.
// Every block evaluates it identically; block 0 records the outcome.
__device__ bool stop_eval(Ctl *c, const double *rr_part, int rr_n, const double *bb_part, int bb_n, bool first,
                          int stop_rule, int max_it, int iter, double *res_hist, int hist_cap) {
    __shared__ int s_stop;
    if (threadIdx.x < 64) {
        const double rr = wave_sum_contig(rr_part, rr_n);
        double bb = 0.0, denom2;
        if (first) {
            bb = wave_sum_contig(bb_part, bb_n);
            denom2 = stop_rule == 0 ? bb : rr;
        } else {
            denom2 = c->denom2;
        }
        const bool conv = (first && bb == 0.0) || rr < c->rtol2 * denom2;
        const bool bad = !isfinite(rr);
        const bool maxed = !first && iter >= max_it;
        const bool run_end = !first && iter >= c->iter_stop;   // restart_every: end of a run
        const bool stop = conv || bad || maxed || run_end;
        if (threadIdx.x == 0) {
            s_stop = stop ? 1 : 0;
            if (blockIdx.x == 0) {
                c->rr = rr;
                if (first) {
                    c->bb = bb;
                    c->r0r0 = rr;
                    c->denom2 = denom2;
                    if (bb == 0.0) c->zero_rhs = 1;
                } else {
                    c->iter = iter;
                }
                if (res_hist && iter < hist_cap) res_hist[iter] = rr;
                if (c->hprog) {
                    volatile double *hp = c->hprog;
                    hp[0] = rr;
                    hp[1] = denom2;
                    hp[2] = (double)iter;
                }
                if (bad) c->status = BDDC_EBREAKDOWN;
                else if (!conv && maxed) c->status = BDDC_ENOTCONV;
                if (stop) ctl_finish(c);
            }
        }
    }
    __syncthreads();
    return s_stop != 0;
}

// The test at the start of the preconditioner's product (direction j not yet
// advanced).  While the basis is recording and `defer` is set, the test is
// left to k_pupd instead, so that the last pass also produces z = M^{-1} r,
// which the harmonic-Ritz matrices need (Section 4.2).
__device__ bool stop_test(const SymvArgs &a) {
    Ctl *c = a.ctl;
    const bool first = a.test == 2;
    return stop_eval(c, a.rr_part, a.rr_n, a.bb_part, a.bb_n, first, a.stop_rule, a.max_it, first ? 0 : c->j + 1,
                     a.res_hist, a.hist_cap);
}

// ctl->done read once per block (a block of the kernel that sets it may be
// running meanwhile): every thread gets the same answer.
__device__ bool block_done(const Ctl *c) {
    __shared__ int s_done;
    if (threadIdx.x == 0) s_done = c->done;
    __syncthreads();
    return s_done != 0;
}

// y_r = sum_{q < ncol} M[q * ldm + r] x[q] for r in [r0, r1) (M read column
// by column, i.e. the transposed access of a row-major symmetric matrix, so
// consecutive lanes read consecutive addresses).  The NW waves of the block
// split the columns; lanes take the rows; partial sums are added in wave
// order by wave 0, which calls store(r, y_r).  x is in LDS.
template <int NW, typename F>
__device__ __forceinline__ void cm_matvec(const double *M, int64_t ldm, int r0, int r1, int ncol, const double *x,
                                          double (*part)[64], F store) {
    const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
    const int q0 = (int)((int64_t)ncol * w / NW), q1 = (int)((int64_t)ncol * (w + 1) / NW);
    for (int rb = r0; rb < r1; rb += 64) {
        const int r = rb + l;
        double s = 0.0;
        if (r < r1) {
#pragma unroll 8
            for (int q = q0; q < q1; ++q) s += M[(int64_t)q * ldm + r] * x[q];
        }
        part[w][l] = s;
        __syncthreads();
        if (w == 0 && r < r1) {
            double t = 0.0;
#pragma unroll
            for (int q = 0; q < NW; ++q) t += part[q][l];
            store(r, t);
        }
        __syncthreads();
    }
}

}  // namespace

// registers for at least 6 waves per SIMD (4 with four float64 tiles in flight)
// A segment record, read through the constant address space: the index is
// block-uniform, so these become scalar loads.
__device__ __forceinline__ SymvItem load_item(const SymvItem *items, int i) {
    typedef const __attribute__((address_space(4))) int32_t CInt;
    CInt *q = (CInt *)(items + i);
    return SymvItem{q[0], q[1], q[2], q[3], q[4], q[5], q[6], q[7], q[8], q[9], q[10], q[11]};
}

template <typename T, int U>
constexpr int symv_waves_per_simd() { return (sizeof(T) == 8 && U == 4) ? 4 : 6; }

// Dot product, in float64 and entry order, of the V = 16 / sizeof(T) entries
// of one 16-byte vector with V consecutive values of x.
template <typename T, typename X>
__device__ __forceinline__ double dot16(const uvec4 &v, const X *x) {
    if constexpr (sizeof(T) == 8) {
        return __hiloint2double(v.y, v.x) * (double)x[0] + __hiloint2double(v.w, v.z) * (double)x[1];
    } else if constexpr (sizeof(T) == 4) {
        return (((double)__uint_as_float(v.x) * (double)x[0] + (double)__uint_as_float(v.y) * (double)x[1]) +
                (double)__uint_as_float(v.z) * (double)x[2]) +
               (double)__uint_as_float(v.w) * (double)x[3];
    } else {
        const unsigned int u[4] = {v.x, v.y, v.z, v.w};
        double s = 0.0;
#pragma unroll
        for (int h = 0; h < 4; ++h) {
            s += (double)dev::bf16_to_f32((uint16_t)(u[h] & 0xffffu)) * (double)x[2 * h];
            s += (double)dev::bf16_to_f32((uint16_t)(u[h] >> 16)) * (double)x[2 * h + 1];
        }
        return s;
    }
}

// Coarse restriction c_i = (D Phi_i)^T x_i of subdomain `sub` (n rows), with
// x_i staged in LDS (zero past n to a multiple of 16), for the DOFs q = c,
// c + C, ... of segment c of the subdomain's C (so that a split subdomain
// shares the work): wave w takes the w-th, (w + NW)-th, ... of those DOFs,
// QB of them at a time; a lane dots the 16-byte
// pieces V l, V l + 64 V, ... of each DOF's column-major row with x, JM
// pieces per round trip, and the wave's sum (fixed order) is the partial.
// Pieces of DOFs past nc_i read as zero through the range check (t past
// the segment's count gives q >= nc_i).
template <typename T, int NW, typename X>
__device__ __forceinline__ void coarse_tail(const SymvArgs &a, int sub, int c, int n, const X *xs, int wu, int l) {
    constexpr int V = 16 / (int)sizeof(T), W = 64 * V, QB = sizeof(T) == 2 ? 1 : 2, JM = 2;
    const int C = a.op.nchunk[sub], nci = a.nc[sub], ld = phi_ld(n);
    const int nq = nci > c ? (nci - c + C - 1) / C : 0;   // this segment's DOFs
    const __amdgpu_buffer_rsrc_t pr =
        tile_rsrc(reinterpret_cast<const T *>(a.phir) + a.phr_off[sub], nci * ld * (int)sizeof(T));
    double *cp = a.cpart + a.c_off[sub];
    for (int t0 = wu; t0 < nq; t0 += NW * QB) {
        double acc[QB];
#pragma unroll
        for (int qi = 0; qi < QB; ++qi) acc[qi] = 0.0;
        for (int p0 = V * l; p0 < ld; p0 += JM * W) {
            uvec4 f[QB][JM];
#pragma unroll
            for (int qi = 0; qi < QB; ++qi)
#pragma unroll
                for (int jj = 0; jj < JM; ++jj)
                    f[qi][jj] = p0 + jj * W < ld ? __builtin_amdgcn_raw_buffer_load_b128(
                                                       pr, ((c + C * (t0 + NW * qi)) * ld + p0 + jj * W) * (int)sizeof(T),
                                                       0, 0)
                                                 : uvec4{0u, 0u, 0u, 0u};
#pragma unroll
            for (int qi = 0; qi < QB; ++qi)
#pragma unroll
                for (int jj = 0; jj < JM; ++jj)
                    if (p0 + jj * W < ld) acc[qi] += dot16<T>(f[qi][jj], xs + p0 + jj * W);
        }
#pragma unroll
        for (int qi = 0; qi < QB; ++qi) {
            const double s = wave_sum(acc[qi]);
            const int t = t0 + NW * qi;
            if (l == 0 && t < nq) cp[c + C * t] = s;
        }
    }
}

// Name tags of the three operator batches (the kernel is the same; only the
// Neumann batch makes the stopping test and the coarse restriction).
struct OpSchur { static constexpr bool neumann = false; };
struct OpNeumann { static constexpr bool neumann = true; };
struct OpInterior { static constexpr bool neumann = false; };

template <typename T, int NW, int U, typename OP>
__global__ void __launch_bounds__(NW * 64, (symv_waves_per_simd<T, U>())) k_symv(SymvArgs a) {
    using ACC = typename Acc<T>::type;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    __shared__ double red[16];
    constexpr int NT = NW * 64;
    constexpr int GATHER_PER_THREAD = NT >= 512 ? 1 : 512 / NT;
    constexpr int SR = 4;           // strip rows per pass (registers)
    // the first pass requested with the gathered values where registers allow
    // (not beside the stopping test's registers in the float64 Neumann batch)
    constexpr bool STRIP_EARLY = sizeof(T) == 2 || (sizeof(T) == 4 && U == 2) || (sizeof(T) == 8 && U == 4 && !OP::neumann);
    const int tid = threadIdx.x, w = tid >> 6, l = tid & 63, g4 = 4 * (l >> 4), cl = l & 15;
    const int wu = __builtin_amdgcn_readfirstlane(w);     // wave-uniform control flow
    // Segment records are block-uniform: read through the constant address
    // space (scalar loads).  The first one is in flight during the control
    // check; the gather indices and first tile stage of a segment are issued
    // as soon as its record is there (before the stopping test for the first
    // segment), then gathered values, then the second stage, in this order,
    // so that waiting for the values never waits for the second stage (loads
    // complete in issue order).  Three round trips before the first tile is
    // used.
    SymvItem it = load_item(a.op.items, blockIdx.x);
    if (a.gated && block_done(a.ctl)) return;
    const bool test_here = OP::neumann && a.test && !(a.defer && a.ctl->record);

    // Tiles past w1 read as zero without a memory access (resource over tiles
    // [t, w1) for the stage starting at tile t), so the loads of the next U
    // tiles are issued unconditionally while the current U are used; two
    // register sets in turn, so that no copy waits for a load.
    double dot = 0.0;
    // the block's segments (consecutive pieces of the global tile sequence,
    // each inside one subdomain), one after the other
    for (bool first = true;; first = false) {
        const int n = it.n;
        const T *tb = reinterpret_cast<const T *>(a.op.tiles) + (int64_t)it.tile * 256;
        const int32_t *gb = a.op.gB + it.x_off;
        const int ntf = it.ntf;     // tile rows
        const int ntl = it.ntl;     // the tiles; a strip's slots follow
        // the waves split the segment's tiles; the segment holding slot ntl
        // also takes the ragged tail's strip (after its tiles)
        const int span = max(min(it.t1, ntl) - it.t0, 0);
        const bool strip_here = it.strip && it.t0 <= ntl && ntl < it.t1;
        const int w0 = it.t0 + (int)((int64_t)span * wu / NW);
        const int w1 = it.t0 + (int)((int64_t)span * (wu + 1) / NW);
        auto stage = [&](int t) {
            return tile_rsrc(tb + (int64_t)t * 256, max(w1 - t, 0) * 256 * (int)sizeof(T));
        };
        int gi[GATHER_PER_THREAD];
    #pragma unroll
        for (int j = 0; j < GATHER_PER_THREAD; ++j) gi[j] = gb[min(tid + j * NT, max(n - 1, 0))];
        asm volatile("" ::: "memory");                        // (keeps those loads first)
        Frag<T> fa[U], fb[U];
    #pragma unroll
        for (int u = 0; u < U; ++u) fa[u].load(stage(w0), u, l);
        if (first && test_here && stop_test(a)) return;
        const int npad = ((n + TILE - 1) / TILE) * TILE;
        ACC *xs = reinterpret_cast<ACC *>(smem_raw);
        ACC *yw = xs + npad;
        double xv[GATHER_PER_THREAD];
    #pragma unroll
        for (int j = 0; j < GATHER_PER_THREAD; ++j) xv[j] = a.x[gi[j]];
        asm volatile("" ::: "memory");                        // (the gathered values before fb)
        // the strip segment: its first SR rows at column tid, requested before
        // the second tile stage and applied right after the staging below
        const int rem = n % TILE, n0 = n - rem;
        const T *sp = tb + (int64_t)ntl * 256;
        T sv[SR];
        if (STRIP_EARLY && strip_here) {
    #pragma unroll
            for (int r = 0; r < SR; ++r) sv[r] = (r < rem && tid < n) ? sp[(int64_t)r * n + tid] : (T)0;
        }
        asm volatile("" ::: "memory");
    #pragma unroll
        for (int u = 0; u < U; ++u) fb[u].load(stage(w0 + U), u, l);
    #pragma unroll
        for (int j = 0; j < GATHER_PER_THREAD; ++j) {
            const int k = tid + j * NT;
            if (k < npad) xs[k] = k < n ? (ACC)xv[j] : (ACC)0;
        }
        if (npad > GATHER_PER_THREAD * NT) {   // long interfaces: indices through 32-bit offsets
            const __amdgpu_buffer_rsrc_t gr = tile_rsrc(gb, n * 4);
            for (int k = tid + GATHER_PER_THREAD * NT; k < npad; k += NT)
                xs[k] = k < n ? (ACC)a.x[(int)__builtin_amdgcn_raw_buffer_load_b32(gr, k * 4, 0, 0)] : (ACC)0;
        }
        for (int k = tid; k < NW * npad; k += NT) yw[k] = (ACC)0;
        __syncthreads();

        ACC *myy = yw + wu * npad;
        // Ragged tail rows n0 + r (r < n % 16), stored whole: rows r0..r0+SR-1 at
        // column k = k0 + tid (entries v, zero past the strip).  The thread
        // adds S[n0+r][k] x[n0+r] into y_k (columns below n0); the products
        // S[n0+r][k] x_k are summed over the wave and added into y_(n0+r).
        // Every addition goes into the thread's own wave's partials, in a
        // fixed order.
        auto strip_rows = [&](int k0, int r0, const T (&v)[SR]) {
            const int k = k0 + tid;
            const ACC xk = k < n ? xs[k] : (ACC)0;
            ACC t = (ACC)0;
    #pragma unroll
            for (int r = 0; r < SR; ++r) {
                if (r0 + r < rem) {
                    const ACC vr = (ACC)to_d(v[r]);
                    t += vr * xs[n0 + r0 + r];
                    const ACC sr = wave_sum(vr * xk);
                    if (l == 0) myy[n0 + r0 + r] += sr;
                }
            }
            if (k < n0) myy[k] += t;
        };
        if (STRIP_EARLY && strip_here) strip_rows(0, 0, sv);
        if (w0 >= w1) {
    #pragma unroll
            for (int u = 0; u < U; ++u) { fa[u].settle(); fb[u].settle(); }
        } else {
            int I = 0, rs = 0;
            while (rs + (ntf - I) <= w0) { rs += ntf - I; ++I; }
            int J = I + (w0 - rs);
            ACC xi[4], ra[4];
    #pragma unroll
            for (int q = 0; q < 4; ++q) { xi[q] = xs[I * TILE + g4 + q]; ra[q] = (ACC)0; }
            // Every fragment is used arithmetically on every path (a tile past
            // w1 reads as zero and only its bookkeeping is skipped), so no path
            // leaves a load outstanding when its registers are loaded again.
            auto use = [&](const Frag<T> (&f)[U], int t) {
    #pragma unroll
                for (int u = 0; u < U; ++u) {
                    const bool live = t + u < w1;
                    ACC v[4];
                    f[u].get(v);
                    // no direct part past the range (J < ntf holds for a live
                    // tile; the test keeps the float64 Schur variants free of spills)
                    const ACC xj = (live && J < ntf) ? xs[J * TILE + cl] : (ACC)0;
    #pragma unroll
                    for (int q = 0; q < 4; ++q) ra[q] += v[q] * xj;
                    const ACC s = col_sum4(v[0] * xi[0] + v[1] * xi[1] + v[2] * xi[2] + v[3] * xi[3]);
                    if (!live) continue;
                    if (J != I && l < 16) myy[J * TILE + cl] += s;
                    if (++J == ntf) {
                        const ACC m = row_sum4(ra, cl);
                        if ((cl & 3) == 0) myy[I * TILE + g4 + (cl >> 2)] += m;
    #pragma unroll
                        for (int q = 0; q < 4; ++q) ra[q] = (ACC)0;
                        ++I;
                        J = I;
                        if (I < ntf) {
    #pragma unroll
                            for (int q = 0; q < 4; ++q) xi[q] = xs[I * TILE + g4 + q];
                        }
                    }
                }
            };
            // fa holds tiles [t, t + U), fb the next U (both issued above)
            for (int t = w0;;) {
                use(fa, t);
                t += U;
                if (t >= w1) {
    #pragma unroll
                    for (int u = 0; u < U; ++u) fb[u].settle();
                    break;
                }
    #pragma unroll
                for (int u = 0; u < U; ++u) fa[u].load(stage(t + U), u, l);
                use(fb, t);
                t += U;
                if (t >= w1) {
    #pragma unroll
                    for (int u = 0; u < U; ++u) fa[u].settle();
                    break;
                }
    #pragma unroll
                for (int u = 0; u < U; ++u) fb[u].load(stage(t + U), u, l);
            }
            if (J != I) {   // flush a partly processed tile row
                const ACC m = row_sum4(ra, cl);
                if ((cl & 3) == 0) myy[I * TILE + g4 + (cl >> 2)] += m;
            }
        }
        if (strip_here) {   // the rest of the strip (more than SR rows, or columns past NT)
            for (int k0 = 0; k0 < n; k0 += NT) {
                for (int r0 = 0; r0 < rem; r0 += SR) {
                    if (STRIP_EARLY && k0 == 0 && r0 == 0) continue;
                    T v[SR];
    #pragma unroll
                    for (int r = 0; r < SR; ++r)
                        v[r] = (r0 + r < rem && k0 + tid < n) ? sp[(int64_t)(r0 + r) * n + k0 + tid] : (T)0;
                    strip_rows(k0, r0, v);
                }
            }
        }
        __syncthreads();

        double *yp = a.ypart + it.yoff;
        for (int k = tid; k < n; k += NW * 64) {
            ACC s = (ACC)0;
    #pragma unroll
            for (int q = 0; q < NW; ++q) s += yw[q * npad + k];
            const double y = (double)s;
            yp[k] = y;
            dot += (double)xs[k] * y;
        }
        if constexpr (OP::neumann) {   // this segment's share of the coarse restriction
            if (a.cpart) coarse_tail<T, NW>(a, it.sub, it.chunk, n, xs, wu, l);
        }
        __syncthreads();   // LDS is reused by the next segment
        if (it.next < 0) break;
        it = load_item(a.op.items, it.next);
    }
    if (a.dot) {
        dot = block_sum(dot, red);
        if (threadIdx.x == 0) a.dot[blockIdx.x] = dot;
    }
}

// ---------------------------------------------------------------------------
// Alg. 1 lines 9-11: alpha = rho_j / p^T A p (every block sums the per-item
// partials of the Schur product), q = sum_i R_i^T q_i, x += alpha p,
// r -= alpha q; per-block ||r||^2; the product is kept as AP_j for recycling.
// ---------------------------------------------------------------------------
// Operands of nodes gb, gb + stride, ..., UN of them: q from its partial
// products (in list order, as gather_sum adds them), x, p, r.  The pointer,
// index and partial loads of all UN nodes are issued together (three round
// trips for the group instead of three per node).
constexpr int UPD_SLOTS = 8;        // partials per node fetched in the first pass
template <int UPD_UN>
__device__ __forceinline__ void upd_load(const UpdArgs &a, int64_t gb, int64_t stride, double (&q)[UPD_UN],
                                         double (&xv)[UPD_UN], double (&pv)[UPD_UN], double (&rv)[UPD_UN]) {
    int e0[UPD_UN], e1[UPD_UN];
#pragma unroll
    for (int u = 0; u < UPD_UN; ++u) {
        const int64_t g = gb + u * stride;
        const bool ok = g < a.n;
        e0[u] = ok ? a.q.ptr[g] : 0;
        e1[u] = ok ? a.q.ptr[g + 1] : 0;
        xv[u] = ok ? a.x[g] : 0.0;
        pv[u] = ok ? a.p[g] : 0.0;
        rv[u] = ok ? a.r[g] : 0.0;
    }
    int id[UPD_UN][UPD_SLOTS];
#pragma unroll
    for (int u = 0; u < UPD_UN; ++u)
#pragma unroll
        for (int m = 0; m < UPD_SLOTS; ++m) id[u][m] = e0[u] + m < e1[u] ? a.q.idx[e0[u] + m] : -1;
#pragma unroll
    for (int u = 0; u < UPD_UN; ++u) {
        double v[UPD_SLOTS];
#pragma unroll
        for (int m = 0; m < UPD_SLOTS; ++m) v[m] = id[u][m] >= 0 ? a.q.part[id[u][m]] : 0.0;
        double sum = 0.0;
#pragma unroll
        for (int m = 0; m < UPD_SLOTS; ++m)
            if (id[u][m] >= 0) sum += v[m];
        for (int e = e0[u] + UPD_SLOTS; e < e1[u]; ++e) sum += a.q.part[a.q.idx[e]];
        q[u] = sum;
    }
}

// UPD_UN nodes per pass: 4 when every thread has several nodes, else 1
template <int UPD_UN>
__global__ void __launch_bounds__(256) k_update(UpdArgs a) {
    __shared__ double red[16];
    Ctl *c = a.ctl;
    if (c->done) return;
    const int j = c->j;
    const int64_t g0 = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    // the operands of this thread's first nodes do not depend on alpha: their
    // loads are issued before the reduction
    double q[UPD_UN], xv[UPD_UN], pv[UPD_UN], rv[UPD_UN];
    upd_load<UPD_UN>(a, g0, stride, q, xv, pv, rv);
    const double pAp = block_sum_contig(a.dot, a.dot_n, red);
    const double alpha = (j < a.hist_cap ? a.rho_hist[j] : 0.0) / pAp;
    const bool bad = !(pAp > 0.0) || !isfinite(alpha) || j >= a.hist_cap;
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        c->pAp = pAp;
        c->alpha = alpha;
        if (j < a.hist_cap) { a.d_hist[j] = pAp; a.a_hist[j] = alpha; }
        if (bad) { c->status = BDDC_EBREAKDOWN; ctl_finish(c); }
    }
    if (bad) return;
    const bool rec = a.AP && c->record && j < a.cap;
    double rr = 0.0;
    for (int64_t gb = g0; gb < a.n; gb += UPD_UN * stride) {
        if (gb != g0) upd_load<UPD_UN>(a, gb, stride, q, xv, pv, rv);
#pragma unroll
        for (int u = 0; u < UPD_UN; ++u) {
            const int64_t g = gb + u * stride;
            if (g < a.n) {
                const double xi = xv[u] + alpha * pv[u];
                const double ri = rv[u] - alpha * q[u];
                a.x[g] = xi;
                a.r[g] = ri;
                rr += ri * ri;
                if (rec) a.AP[(int64_t)j * a.ld + g] = q[u];
            }
        }
    }
    rr = block_sum(rr, red);
    if (threadIdx.x == 0) a.rr_part[blockIdx.x] = rr;
}

// ---------------------------------------------------------------------------
// Coarse prolongation (eq. averaging_subdomain_solves), one block per
// subdomain: w_i = u_i + (D Phi_i) u_C|_i, u_i summed from the partial
// products of the Neumann operator's work items.
// ---------------------------------------------------------------------------
// Element i of a T array through a buffer resource (zero past its end).
template <typename T>
__device__ __forceinline__ double ld_rc_as(__amdgpu_buffer_rsrc_t r, int i);
template <>
__device__ __forceinline__ double ld_rc_as<double>(__amdgpu_buffer_rsrc_t r, int i) { return ld_rc(r, i); }
template <>
__device__ __forceinline__ double ld_rc_as<float>(__amdgpu_buffer_rsrc_t r, int i) {
    return (double)__uint_as_float(__builtin_amdgcn_raw_buffer_load_b32(r, i * 4, 0, 0));
}
template <>
__device__ __forceinline__ double ld_rc_as<uint16_t>(__amdgpu_buffer_rsrc_t r, int i) {
    return (double)dev::bf16_to_f32(__builtin_amdgcn_raw_buffer_load_b16(r, i * 2, 0, 0));
}

// Coarse residual partials c_i = (D Phi_i)^T R_i x of every subdomain (the
// right-hand side of eq. coarse_problem) for several columns at once (the
// block products; a single-vector Neumann product computes them itself):
// one block per subdomain, one float64 partial per (column, local coarse
// DOF).  D Phi_i is stored
// column-major, so each coarse DOF's entries are one contiguous row: wave w
// takes the DOFs w, w + 4, ...; a lane holds 16-byte pieces of QB of them
// (JM pieces each per round trip, the first requested before the gather of
// x), dots them with the gathered x staged in LDS (zero past n), and the
// wave's sum gives the partial (a fixed order: the result does not depend
// on timing).  Pieces of DOFs past nc_i read as zero through the range check.
template <typename T>
__global__ void __launch_bounds__(256) k_crest(CrestArgs a) {
    constexpr int V = 16 / (int)sizeof(T), W = 64 * V, QB = 4, JM = 2;
    extern __shared__ double xs[];          // [cols][XL]
    if (a.ctl->done) return;
    const int i = blockIdx.x, n = a.nB[i], nci = a.nc[i];
    if (nci == 0) return;
    const int ld = phi_ld(n), J = (ld + W - 1) / W, XL = J * W;   // pieces per DOF row, staged length
    const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6), l = threadIdx.x & 63;
    const int32_t *gb = a.gB + a.b_off[i];
    const __amdgpu_buffer_rsrc_t pr =
        tile_rsrc(reinterpret_cast<const T *>(a.phir) + a.phr_off[i], nci * ld * (int)sizeof(T));
    uvec4 f[QB][JM];
    auto issue = [&](int q0, int jb) {
#pragma unroll
        for (int qi = 0; qi < QB; ++qi)
#pragma unroll
            for (int jj = 0; jj < JM; ++jj)
                f[qi][jj] = jb + jj < J ? __builtin_amdgcn_raw_buffer_load_b128(
                                              pr, ((q0 + 4 * qi) * ld + (jb + jj) * W + V * l) * (int)sizeof(T), 0, 0)
                                        : uvec4{0u, 0u, 0u, 0u};
    };
    issue(w, 0);
    bool held = true;                       // f holds (DOFs from w, pieces 0..JM-1)
    for (int c0 = 0; c0 < a.ncols; c0 += a.cols) {
        const int cg = min(a.cols, a.ncols - c0);
        __syncthreads();                    // the previous columns are used
        for (int e = threadIdx.x; e < cg * XL; e += 256) {
            const int cc = e / XL, k = e - cc * XL;
            xs[e] = k < n ? a.X[(int64_t)(c0 + cc) * a.ldx + gb[k]] : 0.0;
        }
        __syncthreads();
        for (int q0 = w; q0 < nci; q0 += 4 * QB) {
            for (int cc = 0; cc < cg; ++cc) {
                double acc[QB];
#pragma unroll
                for (int qi = 0; qi < QB; ++qi) acc[qi] = 0.0;
                for (int jb = 0; jb < J; jb += JM) {
                    if (!held) issue(q0, jb);
                    held = false;
#pragma unroll
                    for (int qi = 0; qi < QB; ++qi)
#pragma unroll
                        for (int jj = 0; jj < JM; ++jj)
                            if (jb + jj < J) acc[qi] += dot16<T>(f[qi][jj], xs + cc * XL + (jb + jj) * W + V * l);
                }
#pragma unroll
                for (int qi = 0; qi < QB; ++qi) {
                    const double s = wave_sum(acc[qi]);
                    const int q = q0 + 4 * qi;
                    if (l == 0 && q < nci) a.part[(int64_t)(c0 + cc) * a.cs + a.c_off[i] + q] = s;
                }
            }
        }
    }
    // a wave without DOFs leaves its first requests unused: none outstanding at exit
#pragma unroll
    for (int qi = 0; qi < QB; ++qi)
#pragma unroll
        for (int jj = 0; jj < JM; ++jj) asm volatile("" ::"v"(f[qi][jj]));
}

template <typename T>
__global__ void __launch_bounds__(256) k_prolong(ProlArgs a) {
    extern __shared__ double uCl[];
    constexpr int PF = 16, CF = 4;      // basis entries / partials of a row requested early
    if (a.gated && a.ctl->done) return;
    {
        const int64_t col = blockIdx.y;  // one column per grid row (block products)
        a.upart += col * a.cs_u;
        if (a.uC) a.uC += col * a.cs_uC;
        a.wloc += col * a.cs_w;
    }
    // 512 rows of one subdomain per block (large subdomains take several)
    const int i = a.ch_sub[blockIdx.x], r0 = a.ch_row[blockIdx.x];
    const int n = a.nB[i], C = a.nchunk[i];
    const int nci = a.uC ? a.nc[i] : 0, ld = phi_ld(n);
    const int32_t *ci = a.cidx + a.c_off[i];
    const T *ph = reinterpret_cast<const T *>(a.phir) + a.phr_off[i];   // column-major, rows of ld
    const double *up = a.upart + a.pb[i];
    double *wl = a.wloc + a.b_off[i];
    // The first CF partial sums and PF basis entries of this thread's first
    // two rows do not depend on u_C: they are requested before its gather,
    // through range-checked loads (no conditions; entries past the
    // subdomain's arrays read as zero, other rows' entries are not used).
    // Consecutive threads read consecutive entries of each basis column.
    const __amdgpu_buffer_rsrc_t ur = vec_rsrc(up, (int64_t)C * n);
    const __amdgpu_buffer_rsrc_t pr = tile_rsrc(ph, nci * ld * (int)sizeof(T));
    const int k0 = r0 + threadIdx.x, k1 = r0 + threadIdx.x + 256;
    double u0[CF], u1[CF], pr0[PF], pr1[PF];
#pragma unroll
    for (int cc = 0; cc < CF; ++cc) {
        u0[cc] = ld_rc(ur, cc * n + k0);
        u1[cc] = ld_rc(ur, cc * n + k1);
    }
#pragma unroll
    for (int q = 0; q < PF; ++q) {
        pr0[q] = ld_rc_as<T>(pr, q * ld + k0);
        pr1[q] = ld_rc_as<T>(pr, q * ld + k1);
    }
    for (int q = threadIdx.x; q < nci; q += blockDim.x) uCl[q] = a.uC[ci[q]];
    __syncthreads();
    // w = sum of the partials, then the basis terms, in column order
    auto row = [&](int k, const double (&u)[CF], const double (&r)[PF]) {
        double w = 0.0;
        for (int cc = 0; cc < C; ++cc) w += cc < CF ? u[cc] : up[(int64_t)cc * n + k];
#pragma unroll
        for (int q = 0; q < PF; ++q)
            if (q < nci) w += r[q] * uCl[q];
#pragma unroll 8
        for (int q = PF; q < nci; ++q) w += to_d(ph[(int64_t)q * ld + k]) * uCl[q];
        wl[k] = w;
    };
    if (k0 < n) row(k0, u0, pr0);
    if (k1 < n) row(k1, u1, pr1);
}

// ---------------------------------------------------------------------------
// Alg. 1 line 13, assembly: z = sum_i R_i^T w_i (weights folded into the
// stored operators).  Per-block partials of r^T z and (AW)^T z (line 15),
// column-major.  With `advance`, block 0 moves the direction index to j + 1
// (no block of this kernel reads it).
// ---------------------------------------------------------------------------
template <int KM>
__global__ void __launch_bounds__(256) k_zasm(ZasmArgs a) {
    __shared__ double lds[16 * 256];
    __shared__ double res[KM + 1];
    Ctl *c = a.ctl;
    if (a.gated && c->done) return;
    if (a.advance && blockIdx.x == 0 && blockIdx.y == 0 && threadIdx.x == 0) c->j = c->j + 1;
    {
        const int64_t col = blockIdx.y;  // one column per grid row (block products; no partials)
        a.w.part += col * a.cs_w;
        a.r += col * a.cs_r;
        a.z += col * a.cs_z;
    }
    const int k = a.part ? c->k : 0;
    double acc[KM + 1];
#pragma unroll
    for (int q = 0; q <= KM; ++q) acc[q] = 0.0;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    const __amdgpu_buffer_rsrc_t awr = vec_rsrc(a.AW, (int64_t)k * a.ld);
    for (int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; g < a.n; g += stride) {
        // the node's (AW) and r entries are requested with its gather, not
        // after the store of z (which the compiler may not move them past)
        double aw[KM > 0 ? KM : 1], rg = 0.0;
        if (a.part) {
            rg = a.r[g];
#pragma unroll
            for (int q = 0; q < KM; ++q) aw[q] = ld_rc(awr, (int64_t)q * a.ld + g);
        }
        const double z = gather_sum(a.w, g);
        a.z[g] = z;
        if (a.part) {
            acc[0] += rg * z;
#pragma unroll
            for (int q = 0; q < KM; ++q) acc[1 + q] += aw[q] * z;
        }
    }
    if (!a.part) return;
    block_sum_cols<KM + 1>(acc, k + 1, lds, res);
    if (threadIdx.x <= k) a.part[(int64_t)threadIdx.x * gridDim.x + blockIdx.x] = res[threadIdx.x];
}

// ---------------------------------------------------------------------------
// Alg. 1 lines 14-16 (line 7 when `first`): every block sums the k_zasm
// partials into rho = r^T z and t = (AW)^T z, mu = (W^T A W)^{-1} t,
// beta = rho / rho_prev; p = z + beta p - W mu.  Block 0 records rho, beta,
// mu for the recycling step.  `hist_only` records without updating p (the
// extra preconditioner application after convergence).
// ---------------------------------------------------------------------------
template <int KM>
__global__ void __launch_bounds__(256) k_pupd(PupdArgs a) {
    __shared__ double lds[16 * 256];
    __shared__ double tv[KM + 1];
    __shared__ double mu[RMAX];
    __shared__ double wawi[KM > 0 ? KM * KM : 1];
    Ctl *c = a.ctl;
    if (a.gated && c->done) return;
    const int k = c->k, j = c->j;
    // the stopping test deferred from the preconditioner's product (while
    // recording): on a stop, record rho and mu of this z and leave p alone
    bool hist_only = a.hist_only;
    if (a.test && c->record) {
        const bool first = a.test == 2;
        if (stop_eval(c, a.rr_part, a.rr_n, a.bb_part, a.bb_n, first, a.stop_rule, a.max_it, first ? 0 : j,
                      a.res_hist, a.hist_cap))
            hist_only = true;
    }
    const int64_t g0 = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    double z0 = 0.0, p0 = 0.0, w0[KM > 0 ? KM : 1];
    {
        double acc[KM + 1];
#pragma unroll
        for (int q = 0; q <= KM; ++q) acc[q] = 0.0;
        const __amdgpu_buffer_rsrc_t zr = vec_rsrc(a.zpart, (int64_t)(k + 1) * a.zpart_n);
        for (int b = threadIdx.x; b < a.zpart_n; b += blockDim.x) {
#pragma unroll
            for (int q = 0; q <= KM; ++q) acc[q] += ld_rc(zr, (int64_t)q * a.zpart_n + b);
        }
        // the operands of this thread's first node do not depend on beta and
        // mu: their loads overlap the reductions (columns q >= k read as zero
        // through the range check, so every load is unconditional)
        if (!hist_only && g0 < a.n) {
            z0 = a.z[g0];
            p0 = a.p[g0];
            const __amdgpu_buffer_rsrc_t wr = vec_rsrc(a.W, (int64_t)k * a.ld);
#pragma unroll
            for (int q = 0; q < KM; ++q) w0[q] = ld_rc(wr, (int64_t)q * a.ld + g0);
        }
        for (int e = threadIdx.x; e < k * k; e += blockDim.x) wawi[e] = a.WAWinv[e];
        block_sum_cols<KM + 1>(acc, k + 1, lds, tv);
    }
    // (block_sum_cols ends with a barrier: wawi is complete)
    if (threadIdx.x < k) {
        double s = 0.0;
        for (int q = 0; q < k; ++q) s += wawi[threadIdx.x * k + q] * tv[1 + q];
        mu[threadIdx.x] = s;
    }
    __syncthreads();
    const double rho = tv[0];
    const double beta = a.first ? 0.0 : rho / a.rho_hist[j - 1];
    const bool bad = !(rho > 0.0) || !isfinite(rho) || !isfinite(beta);
    if (blockIdx.x == 0) {
        if (threadIdx.x == 0) {
            if (j < a.hist_cap) a.rho_hist[j] = rho;
            if (!a.first && j >= 1 && j - 1 < a.hist_cap) a.b_hist[j - 1] = beta;
            if (bad && !hist_only) { c->status = BDDC_EBREAKDOWN; ctl_finish(c); }
        }
        if (threadIdx.x < k && j < a.hist_cap) a.mu_hist[(int64_t)j * RMAX + threadIdx.x] = mu[threadIdx.x];
    }
    if (hist_only || bad) return;
    const bool rec = a.P && c->record && j < a.cap;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    if (g0 < a.n) {
        double p = z0 + beta * p0;
#pragma unroll
        for (int q = 0; q < KM; ++q)
            if (q < k) p -= w0[q] * mu[q];
        a.p[g0] = p;
        if (rec) a.P[(int64_t)j * a.ld + g0] = p;
    }
    // the other nodes the same way: all KM loads of a node issued at once
    // (columns q >= k read as zero without an access), same summation order
    const __amdgpu_buffer_rsrc_t wr = vec_rsrc(a.W, (int64_t)k * a.ld);
    for (int64_t g = g0 + stride; g < a.n; g += stride) {
        double w[KM > 0 ? KM : 1];
#pragma unroll
        for (int q = 0; q < KM; ++q) w[q] = ld_rc(wr, (int64_t)q * a.ld + g);
        double p = a.z[g] + beta * a.p[g];
#pragma unroll
        for (int q = 0; q < KM; ++q)
            if (q < k) p -= w[q] * mu[q];
        a.p[g] = p;
        if (rec) a.P[(int64_t)j * a.ld + g] = p;
    }
}

// ---------------------------------------------------------------------------
// out = b - sum_i R_i^T q_i (initial or true residual; out = the assembled
// product when b is null); per-block partials (column-major) of ||out||^2
// and, with want_wtr, of W^T out (Alg. 1 line 3).
// ---------------------------------------------------------------------------
template <int KM>
__global__ void __launch_bounds__(256) k_resid(ResidArgs a) {
    __shared__ double lds[16 * 256];
    __shared__ double res[KM + 1];
    const int k = a.want_wtr ? a.ctl->k : 0;
    double acc[KM + 1];
#pragma unroll
    for (int q = 0; q <= KM; ++q) acc[q] = 0.0;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; g < a.n; g += stride) {
        const double q = gather_sum(a.q, g);
        const double r = a.b ? a.b[g] - q : q;
        a.out[g] = r;
        acc[0] += r * r;
        const __amdgpu_buffer_rsrc_t wr = vec_rsrc(a.W, (int64_t)k * a.ld);
#pragma unroll
        for (int q2 = 0; q2 < KM; ++q2) acc[1 + q2] += ld_rc(wr, (int64_t)q2 * a.ld + g) * r;
    }
    block_sum_cols<KM + 1>(acc, k + 1, lds, res);
    if (threadIdx.x <= k) a.part[(int64_t)threadIdx.x * gridDim.x + blockIdx.x] = res[threadIdx.x];
}

// Alg. 1 lines 3-4: gamma = (W^T A W)^{-1} W^T r (every block, from the
// k_resid partials); x += W gamma; r -= AW gamma (= b - A x_0); ||r||^2.
template <int KM>
__global__ void __launch_bounds__(256) k_defl_init(DeflArgs a) {
    __shared__ double lds[16 * 256];
    __shared__ double tv[KM + 1];
    __shared__ double gam[RMAX];
    __shared__ double red[16];
    const int k = a.ctl->k;
    {
        double acc[KM + 1];
#pragma unroll
        for (int q = 0; q <= KM; ++q) acc[q] = 0.0;
        const __amdgpu_buffer_rsrc_t wr = vec_rsrc(a.wpart, (int64_t)(k + 1) * a.wpart_n);
        for (int b = threadIdx.x; b < a.wpart_n; b += blockDim.x) {
#pragma unroll
            for (int q = 0; q <= KM; ++q) acc[q] += ld_rc(wr, (int64_t)q * a.wpart_n + b);
        }
        block_sum_cols<KM + 1>(acc, k + 1, lds, tv);
    }
    for (int e = threadIdx.x; e < k * k; e += blockDim.x) lds[e] = a.WAWinv[e];
    __syncthreads();
    if (threadIdx.x < k) {
        double s = 0.0;
        for (int q = 0; q < k; ++q) s += lds[threadIdx.x * k + q] * tv[1 + q];
        gam[threadIdx.x] = s;
    }
    __syncthreads();
    double rr = 0.0;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; g < a.n; g += stride) {
        double x = a.x[g], r = a.r[g];
        for (int q = 0; q < k; ++q) {
            x += a.W[(int64_t)q * a.ld + g] * gam[q];
            r -= a.AW[(int64_t)q * a.ld + g] * gam[q];
        }
        a.x[g] = x;
        a.r[g] = r;
        rr += r * r;
    }
    rr = block_sum(rr, red);
    if (threadIdx.x == 0) a.rr_part[blockIdx.x] = rr;
}

// out[c] = sum_b part[c * n + b] (column-major partials), one block per column
// Re-orthogonalisation (Alg. 1, optional line after the residual update):
// k_wtr writes per-block W^T r partials; k_reorth sums them in every block
// (fixed order), gamma = (W^T W)^{-1} W^T r, r -= W gamma and per-block
// ||r||^2 partials that replace the update's for the stopping test.
template <int KM>
__global__ void __launch_bounds__(256) k_wtr(ReorthArgs a) {
    __shared__ double lds[16 * 256];
    __shared__ double res[KM > 0 ? KM : 1];
    if (a.ctl->done) return;
    const int k = a.ctl->k;
    if (k == 0) return;
    double acc[KM > 0 ? KM : 1];
#pragma unroll
    for (int q = 0; q < KM; ++q) acc[q] = 0.0;
    const __amdgpu_buffer_rsrc_t wr = vec_rsrc(a.W, (int64_t)k * a.ld);
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; g < a.n; g += stride) {
        const double r = a.r[g];
#pragma unroll
        for (int q = 0; q < KM; ++q) acc[q] += ld_rc(wr, (int64_t)q * a.ld + g) * r;
    }
    block_sum_cols<KM>(acc, k, lds, res);
    if (threadIdx.x < k) a.part[(int64_t)threadIdx.x * gridDim.x + blockIdx.x] = res[threadIdx.x];
}

template <int KM>
__global__ void __launch_bounds__(256) k_reorth(ReorthArgs a) {
    __shared__ double lds[16 * 256];
    __shared__ double tv[KM > 0 ? KM : 1], gam[KM > 0 ? KM : 1];
    __shared__ double red[16];
    if (a.ctl->done) return;
    const int k = a.ctl->k;
    if (k == 0) return;
    {
        double acc[KM > 0 ? KM : 1];
#pragma unroll
        for (int q = 0; q < KM; ++q) acc[q] = 0.0;
        const __amdgpu_buffer_rsrc_t pr = vec_rsrc(a.part, (int64_t)k * gridDim.x);
        for (int b = threadIdx.x; b < (int)gridDim.x; b += blockDim.x) {
#pragma unroll
            for (int q = 0; q < KM; ++q) acc[q] += ld_rc(pr, (int64_t)q * gridDim.x + b);
        }
        block_sum_cols<KM>(acc, k, lds, tv);
    }
    if (threadIdx.x < k) {
        double s = 0.0;
        for (int q = 0; q < k; ++q) s += a.WWinv[threadIdx.x * k + q] * tv[q];
        gam[threadIdx.x] = s;
    }
    __syncthreads();
    double rr = 0.0;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; g < a.n; g += stride) {
        double r = a.r[g];
        for (int q = 0; q < k; ++q) r -= a.W[(int64_t)q * a.ld + g] * gam[q];
        a.r[g] = r;
        rr += r * r;
    }
    rr = block_sum(rr, red);
    if (threadIdx.x == 0) a.rr_part[blockIdx.x] = rr;
}

__global__ void __launch_bounds__(256) k_reduce(ReduceArgs a) {
    __shared__ double red[16];
    const int c = blockIdx.x;
    const double s = block_sum_contig(a.part + (int64_t)c * a.n, a.n, red);
    if (threadIdx.x == 0) a.out[c] = s;
}

// ---------------------------------------------------------------------------
// coarse problem (eq. coarse_problem); three levels: the multilevel paragraph
// of Section 3.2, subdomains acting as the elements of subregions.  Every
// matrix here is symmetric and row-major; products read it column by column.
// ---------------------------------------------------------------------------
// Two levels: r_C = sum_i R_Ci^T c_i, u_C = K_C^{-1} r_C with the dense
// inverse (stored negated by the sweep); block b computes rows [64b, 64b+64).
// r_C assembled once from the coarse partials (fixed order).
__device__ __forceinline__ void coarse_cols(CoarseDenseArgs &a) {
    const int64_t col = blockIdx.y;     // one column per grid row (block products)
    a.rc.part += col * a.cs_rc;
    a.r += col * a.cs_r;
    a.u += col * a.cs_u;
}

__global__ void __launch_bounds__(256) k_coarse_rhs(CoarseDenseArgs a) {
    if (a.ctl->done) return;
    coarse_cols(a);
    const int q = blockIdx.x * blockDim.x + threadIdx.x;
    if (q < a.n) a.r[q] = gather_sum(a.rc, q);
}

// Dense coarse product u_C = sign * M r_C (row-major M, rows padded with
// zeros to the even length ldm): each wave takes one row of the block's
// ROWS, lanes striding over the columns in 16-byte pieces, four pieces per
// round (8 rows per block above 4096 columns, where the staged r_C limits the
// blocks per compute unit, else 4).  The first CD_PRE rounds of the row do not depend on r_C and are
// requested before r_C is staged in LDS; the staging issues all of a
// thread's loads before waiting for any.  Loads past the row read as zero
// through the buffer range check, and the staged copy is zero past n.
constexpr int CD_PRE = 4;           // rounds of 512 columns requested up front
__host__ __device__ inline int coarse_dense_staged(int ldm) {
    return ((max(ldm, 512 * CD_PRE) + 511) / 512) * 512;
}
template <int ROWS>
__global__ void __launch_bounds__(ROWS * 64) k_coarse_dense(CoarseDenseArgs a) {
    extern __shared__ double rs[];
    if (a.ctl->done) return;
    coarse_cols(a);
    const int n = a.n, ldm = (int)a.ldm;
    const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
    const int row = blockIdx.x * ROWS + w;
    const bool live = row < n;
    const __amdgpu_buffer_rsrc_t mr = tile_rsrc(a.M + (int64_t)(live ? row : 0) * ldm, live ? ldm * 8 : 0);
    uvec4 pre[4 * CD_PRE];
#pragma unroll
    for (int u = 0; u < 4 * CD_PRE; ++u) pre[u] = __builtin_amdgcn_raw_buffer_load_b128(mr, (2 * l + 128 * u) * 8, 0, 0);
    const int nr = coarse_dense_staged(ldm);
    const __amdgpu_buffer_rsrc_t rr = vec_rsrc(a.r, n);
    constexpr int NT = ROWS * 64;
    for (int q0 = 0; q0 < nr; q0 += 8 * NT) {
        double v[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) v[u] = ld_rc(rr, q0 + u * NT + (int)threadIdx.x);
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const int q = q0 + u * NT + (int)threadIdx.x;
            if (q < nr) rs[q] = v[u];
        }
    }
    __syncthreads();
    double s[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int i = 0; i < CD_PRE; ++i) {
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int col = 2 * l + 512 * i + 128 * u;
            const uvec4 v = pre[4 * i + u];
            s[u] += __hiloint2double(v.y, v.x) * rs[col] + __hiloint2double(v.w, v.z) * rs[col + 1];
        }
    }
    for (int c0 = 512 * CD_PRE; c0 < ldm; c0 += 512) {
        uvec4 v[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) v[u] = __builtin_amdgcn_raw_buffer_load_b128(mr, (2 * l + c0 + 128 * u) * 8, 0, 0);
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int col = 2 * l + c0 + 128 * u;
            s[u] += __hiloint2double(v[u].y, v[u].x) * rs[col] + __hiloint2double(v[u].w, v[u].z) * rs[col + 1];
        }
    }
    const double t = wave_sum((s[0] + s[1]) + (s[2] + s[3]));
    if (live && l == 0) a.u[row] = a.sign * t;
}

// Level-3 coarse product with the upper triangle of the (symmetric) inverse
// in 64 x 64 blocks: half the bytes of the full matrix.  One block of
// threads per matrix block (I, J); thread t takes row i = t / 4, columns
// 16 (t % 4) .. + 15 (a wave reads 16 whole rows, 8 KB in one piece).  The
// row part B x_J is summed over the quad of the row; for J > I the column
// part B^T x_I over the 16 rows of the wave (row rotations within 16 lanes,
// then the row-swap permutes) and the 4 waves in order.
constexpr int DPP_ROR4 = 0x124;     // row_ror:4 within 16 lanes
__device__ __forceinline__ int symblk_start(int I, int nb) { return I * nb - I * (I - 1) / 2; }

__global__ void __launch_bounds__(256) k_symblk(SymBlkArgs a) {
    __shared__ double colw[4][64];
    __shared__ double xsh[128];     // x_J, then x_I
    if (a.ctl->done) return;
    const int b = blockIdx.x;
    const int t = threadIdx.x, i = t >> 2, q = t & 3, w = t >> 6, l = t & 63;
    const double2 *rp = reinterpret_cast<const double2 *>(a.B + (int64_t)b * 4096 + i * 64 + 16 * q);
    double2 v[8];
#pragma unroll
    for (int k = 0; k < 8; ++k) v[k] = rp[k];
    const int I = a.bI[b], J = I + (b - symblk_start(I, a.nb));
    // x_J and x_I staged once (range-checked loads: zero past n, no branch)
    const __amdgpu_buffer_rsrc_t rr = vec_rsrc(a.r, a.n);
    if (t < 128) xsh[t] = ld_rc(rr, t < 64 ? 64 * J + t : 64 * I + t - 64);
    __syncthreads();
    double xj[16];
#pragma unroll
    for (int c = 0; c < 16; ++c) xj[c] = xsh[16 * q + c];
    const double xi = xsh[64 + i];
    double s = 0.0;
#pragma unroll
    for (int k = 0; k < 8; ++k) s += v[k].x * xj[2 * k] + v[k].y * xj[2 * k + 1];
    s += dpp<DPP_XOR1>(s);
    s += dpp<DPP_XOR2>(s);
    if (q == 0) a.part[(int64_t)b * 128 + i] = s;
    if (J == I) return;             // (block-uniform) a diagonal block holds both triangles
    double cs[16];
#pragma unroll
    for (int k = 0; k < 8; ++k) { cs[2 * k] = v[k].x * xi; cs[2 * k + 1] = v[k].y * xi; }
#pragma unroll
    for (int k = 0; k < 16; ++k) {
        double u = cs[k] + dpp<DPP_ROR4>(cs[k]);
        u += dpp<DPP_ROR8>(u);
        cs[k] = col_sum4(u);        // the wave's 16 rows of column 16 q + k
    }
    if (l < 4) {
#pragma unroll
        for (int k = 0; k < 16; ++k) colw[w][16 * q + k] = cs[k];
    }
    __syncthreads();
    if (t < 64) a.part[(int64_t)b * 128 + 64 + t] = ((colw[0][t] + colw[1][t]) + colw[2][t]) + colw[3][t];
}

// u on the rows of panel P: the column sums of blocks (I, P), I < P, then the
// row sums of blocks (P, J), J >= P, split over 4 waves and added in order.
__global__ void __launch_bounds__(256) k_symblk_sum(SymBlkArgs a) {
    __shared__ double red[4][64];
    if (a.ctl->done) return;
    const int P = blockIdx.x, t = threadIdx.x, i = t & 63, sq = t >> 6, nb = a.nb;
    // 8 terms of the thread requested at a time (past the last term: an index
    // past the buffer, which reads as zero), added in increasing order
    const int64_t np = (int64_t)nb * (nb + 1) / 2 * 128;
    const __amdgpu_buffer_rsrc_t pr = vec_rsrc(a.part, np);
    double acc = 0.0;
    for (int k0 = sq; k0 < nb; k0 += 32) {
        double v[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const int k = k0 + 4 * u;
            const int64_t e = k >= nb ? np
                            : k < P ? (int64_t)(symblk_start(k, nb) + P - k) * 128 + 64 + i
                                    : (int64_t)(symblk_start(P, nb) + k - P) * 128 + i;
            v[u] = ld_rc(pr, e);
        }
#pragma unroll
        for (int u = 0; u < 8; ++u) acc += v[u];
    }
    red[sq][i] = acc;
    __syncthreads();
    const int g = 64 * P + t;
    if (t < 64 && g < a.n) a.u[g] = ((red[0][t] + red[1][t]) + red[2][t]) + red[3][t];
}

__device__ __forceinline__ void l2_cols(L2Args &a) {
    const int64_t col = blockIdx.y;     // one column per grid row (block products)
    a.rc.part += col * a.cs_rc;
    a.vI2 += col * a.cs_vI2;
    a.t2 += col * a.cs_t2;
    a.rB2 += col * a.cs_rB2;
    a.u2 += col * a.cs_u2;
    a.c3loc += col * a.cs_c3loc;
    a.u3 += col * a.cs_u3;
    a.uC += col * a.cs_uC;
}

// Level 2, phase A (one block per subregion): the subregion's coarse
// residual r_L, interior pre-solve v_I = K_II^{-1} r_I and its interface
// coupling t = K_BI K_II^{-1} r_I (from the swept subregion matrix).
__global__ void __launch_bounds__(256) k_l2_a(L2Args a) {
    extern __shared__ double rL[];
    __shared__ double part[4][64];
    if (a.ctl->done) return;
    l2_cols(a);
    const int j = blockIdx.x;
    const int nL = a.nL[j], nI = a.nI2[j];
    const int loff = a.L_off[j];
    for (int q = threadIdx.x; q < nL; q += blockDim.x) rL[q] = gather_sum(a.rc, a.L[loff + q]);
    __syncthreads();
    double *vI2 = a.vI2 + a.I2_off[j], *t2 = a.t2 + a.B2_off[j], *rB2 = a.rB2 + a.B2_off[j];
    cm_matvec<4>(a.K2 + a.K2_off[j], nL, 0, nL, nI, rL, part, [&](int q, double y) {
        if (q < nI) vI2[q] = -y;
        else { t2[q - nI] = y; rB2[q - nI] = rL[q]; }
    });
}

// Level 2, phase B (one block per subregion): level-2 interface residual
// g = r_G - sum_j R_j^T t_j, then u = (D N D) g and c3 = (D Phi)^T g.
__global__ void __launch_bounds__(256) k_l2_b(L2Args a) {
    extern __shared__ double gs[];
    __shared__ double part[4][64];
    if (a.ctl->done) return;
    l2_cols(a);
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
    double *u2 = a.u2 + b2, *c3 = a.c3loc + a.C3_off[j];
    cm_matvec<4>(a.N2 + a.N2_off[j], nB, 0, nB, nB, gs, part, [&](int k, double y) { u2[k] = y; });
    cm_matvec<4>(a.Phi2 + a.P2_off[j], a.nc3[j], 0, a.nc3[j], nB, gs, part, [&](int q, double y) { c3[q] = y; });
}

// Level 2, phase D (one block per subregion): level-2 interface solution
// x_G = sum_j R_j^T (u_j + (D Phi_j) u3) on the subregion's interface and the
// interior post-correction x_I = v_I - T^T x_G give the level-1 coarse
// solution u_C on the coarse DOFs of the subregion (every subregion sharing
// an interface DOF computes the same value in the same order; its owner
// writes it) for the prolongation, k_prolong.
__global__ void __launch_bounds__(256) k_l2_d(L2Args a) {
    extern __shared__ double sm[];
    __shared__ double part[4][64];
    if (a.ctl->done) return;
    l2_cols(a);
    double *uCL = sm;                 // nL: x_I then x_G
    const int j = blockIdx.x;
    const int nL = a.nL[j], nI = a.nI2[j], nB = nL - nI;
    const int b2 = a.B2_off[j];
    for (int k = threadIdx.x; k < nB; k += blockDim.x) {
        const int gi = a.g2[b2 + k];
        double s = 0.0;
        for (int t = a.asm2_ptr[gi]; t < a.asm2_ptr[gi + 1]; ++t) {
            const int pos = a.asm2_idx[t];
            const double *ph = a.Phi2 + a.ph_off[pos];
            const int32_t *c3 = a.c3 + a.c3o[pos];
            const int n3j = a.n3p[pos];
            double v = a.u2[pos];
#pragma unroll 8
            for (int q = 0; q < n3j; ++q) v += ph[q] * a.u3[c3[q]];
            s += v;
        }
        uCL[nI + k] = s;
    }
    __syncthreads();
    const double *vI2 = a.vI2 + a.I2_off[j];
    cm_matvec<4>(a.K2 + a.K2_off[j] + (int64_t)nI * nL, nL, 0, nI, nB, uCL + nI, part,
                 [&](int q, double y) { uCL[q] = vI2[q] - y; });
    // cm_matvec ends with a barrier: uCL is complete
    for (int q = threadIdx.x; q < nL; q += blockDim.x)
        if (q < nI || a.own2[b2 + q - nI]) a.uC[a.L[a.L_off[j] + q]] = uCL[q];
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------
size_t symv_smem(int prec, int nw, int max_nt) {
    const size_t acc = prec == 64 ? 8 : 4;
    return acc * (size_t)max_nt * TILE * (1 + nw);
}

template <typename T, typename OP>
static int set_limit_t(size_t bytes) {
    const void *f[4] = {(const void *)k_symv<T, 4, 2, OP>, (const void *)k_symv<T, 4, 4, OP>,
                        (const void *)k_symv<T, 8, 2, OP>, (const void *)k_symv<T, 8, 4, OP>};
    for (const void *p : f)
        if (hipFuncSetAttribute(p, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes) != hipSuccess) return -1;
    return 0;
}

int set_symv_smem_limit(size_t bytes) {
    if (set_limit_t<double, OpSchur>(bytes) || set_limit_t<double, OpInterior>(bytes) ||
        set_limit_t<double, OpNeumann>(bytes) || set_limit_t<float, OpNeumann>(bytes) ||
        set_limit_t<uint16_t, OpNeumann>(bytes))
        return -1;
    return 0;
}

template <typename T, typename OP>
static void launch_symv_t(const SymvArgs &a, SymvCfg cfg, size_t smem, hipStream_t s) {
    const dim3 grid(a.op.n_blocks);
    if (cfg.nw == 8) {
        if (cfg.unroll == 4) hipLaunchKernelGGL((k_symv<T, 8, 4, OP>), grid, dim3(512), smem, s, a);
        else hipLaunchKernelGGL((k_symv<T, 8, 2, OP>), grid, dim3(512), smem, s, a);
    } else {
        if (cfg.unroll == 4) hipLaunchKernelGGL((k_symv<T, 4, 4, OP>), grid, dim3(256), smem, s, a);
        else hipLaunchKernelGGL((k_symv<T, 4, 2, OP>), grid, dim3(256), smem, s, a);
    }
}

// The Schur and interior operators are float64 only; the Neumann operators
// come in the three storage precisions.
void launch_symv(const SymvArgs &a, SymvOp op, int prec, SymvCfg cfg, size_t smem, hipStream_t s) {
    if (a.op.n_blocks <= 0) return;
    if (op == SYMV_SCHUR) launch_symv_t<double, OpSchur>(a, cfg, smem, s);
    else if (op == SYMV_INTERIOR) launch_symv_t<double, OpInterior>(a, cfg, smem, s);
    else if (prec == 64) launch_symv_t<double, OpNeumann>(a, cfg, smem, s);
    else if (prec == 32) launch_symv_t<float, OpNeumann>(a, cfg, smem, s);
    else launch_symv_t<uint16_t, OpNeumann>(a, cfg, smem, s);
}

void launch_update(const UpdArgs &a, int grid, hipStream_t s) {
    if (a.n > (int64_t)grid * 256 * 2) hipLaunchKernelGGL(k_update<4>, dim3(grid), dim3(256), 0, s, a);
    else hipLaunchKernelGGL(k_update<1>, dim3(grid), dim3(256), 0, s, a);
}

// staged length of the gathered x of the restriction for interfaces of up
// to max_nB entries (whole 16-byte pieces of a wave)
static int crest_xl(int prec, int max_nB) {
    const int W = 64 * (128 / prec);
    return (phi_ld(std::max(1, max_nB)) + W - 1) / W * W;
}
// columns staged at a time: up to 4096 values (32 KiB of LDS)
int crest_cols(int prec, int max_nB, int ncols) {
    return std::max(1, std::min(ncols, 4096 / crest_xl(prec, max_nB)));
}

void launch_crest(const CrestArgs &a, int prec, int nsub, int max_nB, hipStream_t s) {
    if (nsub <= 0 || a.ncols <= 0) return;
    const size_t smem = (size_t)a.cols * crest_xl(prec, max_nB) * 8;
    if (prec == 64) hipLaunchKernelGGL(k_crest<double>, dim3(nsub), dim3(256), smem, s, a);
    else if (prec == 32) hipLaunchKernelGGL(k_crest<float>, dim3(nsub), dim3(256), smem, s, a);
    else hipLaunchKernelGGL(k_crest<uint16_t>, dim3(nsub), dim3(256), smem, s, a);
}

void launch_prolong(const ProlArgs &a, int prec, int nblocks, int max_nc, hipStream_t s, int ncols) {
    const size_t smem = (size_t)std::max(1, max_nc) * 8;
    const dim3 grid(nblocks, ncols);
    if (prec == 64) hipLaunchKernelGGL(k_prolong<double>, grid, dim3(256), smem, s, a);
    else if (prec == 32) hipLaunchKernelGGL(k_prolong<float>, grid, dim3(256), smem, s, a);
    else hipLaunchKernelGGL(k_prolong<uint16_t>, grid, dim3(256), smem, s, a);
}

int kmax_bucket(int k) { return k == 0 ? 0 : k <= 8 ? 8 : k <= 16 ? 16 : k <= 32 ? 32 : k <= 48 ? 48 : 64; }

void launch_zasm(const ZasmArgs &a, int kmax, int grid, hipStream_t s, int ncols) {
    switch (kmax) {
        case 0: hipLaunchKernelGGL(k_zasm<0>, dim3(grid, ncols), dim3(256), 0, s, a); break;
        case 8: hipLaunchKernelGGL(k_zasm<8>, dim3(grid, ncols), dim3(256), 0, s, a); break;
        case 16: hipLaunchKernelGGL(k_zasm<16>, dim3(grid, ncols), dim3(256), 0, s, a); break;
        case 32: hipLaunchKernelGGL(k_zasm<32>, dim3(grid, ncols), dim3(256), 0, s, a); break;
        case 48: hipLaunchKernelGGL(k_zasm<48>, dim3(grid, ncols), dim3(256), 0, s, a); break;
        default: hipLaunchKernelGGL(k_zasm<64>, dim3(grid, ncols), dim3(256), 0, s, a); break;
    }
}

void launch_pupd(const PupdArgs &a, int kmax, int grid, hipStream_t s) {
    switch (kmax) {
        case 0: hipLaunchKernelGGL(k_pupd<0>, dim3(grid), dim3(256), 0, s, a); break;
        case 8: hipLaunchKernelGGL(k_pupd<8>, dim3(grid), dim3(256), 0, s, a); break;
        case 16: hipLaunchKernelGGL(k_pupd<16>, dim3(grid), dim3(256), 0, s, a); break;
        case 32: hipLaunchKernelGGL(k_pupd<32>, dim3(grid), dim3(256), 0, s, a); break;
        case 48: hipLaunchKernelGGL(k_pupd<48>, dim3(grid), dim3(256), 0, s, a); break;
        default: hipLaunchKernelGGL(k_pupd<64>, dim3(grid), dim3(256), 0, s, a); break;
    }
}

void launch_resid(const ResidArgs &a, int kmax, int grid, hipStream_t s) {
    switch (kmax) {
        case 0: hipLaunchKernelGGL(k_resid<0>, dim3(grid), dim3(256), 0, s, a); break;
        case 8: hipLaunchKernelGGL(k_resid<8>, dim3(grid), dim3(256), 0, s, a); break;
        case 16: hipLaunchKernelGGL(k_resid<16>, dim3(grid), dim3(256), 0, s, a); break;
        case 32: hipLaunchKernelGGL(k_resid<32>, dim3(grid), dim3(256), 0, s, a); break;
        case 48: hipLaunchKernelGGL(k_resid<48>, dim3(grid), dim3(256), 0, s, a); break;
        default: hipLaunchKernelGGL(k_resid<64>, dim3(grid), dim3(256), 0, s, a); break;
    }
}

void launch_defl_init(const DeflArgs &a, int kmax, int grid, hipStream_t s) {
    switch (kmax) {
        case 0: hipLaunchKernelGGL(k_defl_init<0>, dim3(grid), dim3(256), 0, s, a); break;
        case 8: hipLaunchKernelGGL(k_defl_init<8>, dim3(grid), dim3(256), 0, s, a); break;
        case 16: hipLaunchKernelGGL(k_defl_init<16>, dim3(grid), dim3(256), 0, s, a); break;
        case 32: hipLaunchKernelGGL(k_defl_init<32>, dim3(grid), dim3(256), 0, s, a); break;
        case 48: hipLaunchKernelGGL(k_defl_init<48>, dim3(grid), dim3(256), 0, s, a); break;
        default: hipLaunchKernelGGL(k_defl_init<64>, dim3(grid), dim3(256), 0, s, a); break;
    }
}

void launch_reorth(const ReorthArgs &a, int kmax, int grid, hipStream_t s) {
    switch (kmax) {
        case 0: break;
        case 8:
            hipLaunchKernelGGL(k_wtr<8>, dim3(grid), dim3(256), 0, s, a);
            hipLaunchKernelGGL(k_reorth<8>, dim3(grid), dim3(256), 0, s, a);
            break;
        case 16:
            hipLaunchKernelGGL(k_wtr<16>, dim3(grid), dim3(256), 0, s, a);
            hipLaunchKernelGGL(k_reorth<16>, dim3(grid), dim3(256), 0, s, a);
            break;
        case 32:
            hipLaunchKernelGGL(k_wtr<32>, dim3(grid), dim3(256), 0, s, a);
            hipLaunchKernelGGL(k_reorth<32>, dim3(grid), dim3(256), 0, s, a);
            break;
        case 48:
            hipLaunchKernelGGL(k_wtr<48>, dim3(grid), dim3(256), 0, s, a);
            hipLaunchKernelGGL(k_reorth<48>, dim3(grid), dim3(256), 0, s, a);
            break;
        default:
            hipLaunchKernelGGL(k_wtr<64>, dim3(grid), dim3(256), 0, s, a);
            hipLaunchKernelGGL(k_reorth<64>, dim3(grid), dim3(256), 0, s, a);
            break;
    }
}

void launch_reduce(const ReduceArgs &a, hipStream_t s) {
    if (a.ncol > 0) hipLaunchKernelGGL(k_reduce, dim3(a.ncol), dim3(256), 0, s, a);
}

void launch_coarse_dense(const CoarseDenseArgs &a, hipStream_t s, int ncols) {
    if (a.n <= 0) return;
    hipLaunchKernelGGL(k_coarse_rhs, dim3((a.n + 255) / 256, ncols), dim3(256), 0, s, a);
    const size_t smem = (size_t)coarse_dense_staged((int)a.ldm) * 8;
    if (a.n > 4096) hipLaunchKernelGGL(k_coarse_dense<8>, dim3((a.n + 7) / 8, ncols), dim3(512), smem, s, a);
    else hipLaunchKernelGGL(k_coarse_dense<4>, dim3((a.n + 3) / 4, ncols), dim3(256), smem, s, a);
}

void launch_coarse_symblk(const CoarseDenseArgs &g, const SymBlkArgs &a, hipStream_t s) {
    if (a.n <= 0) return;
    hipLaunchKernelGGL(k_coarse_rhs, dim3((g.n + 255) / 256), dim3(256), 0, s, g);
    hipLaunchKernelGGL(k_symblk, dim3(a.nb * (a.nb + 1) / 2), dim3(256), 0, s, a);
    hipLaunchKernelGGL(k_symblk_sum, dim3(a.nb), dim3(256), 0, s, a);
}

void launch_l2_a(const L2Args &a, int nsr, int max_nL, hipStream_t s, int ncols) {
    hipLaunchKernelGGL(k_l2_a, dim3(nsr, ncols), dim3(256), (size_t)max_nL * 8, s, a);
}
void launch_l2_b(const L2Args &a, int nsr, int max_nL, hipStream_t s, int ncols) {
    hipLaunchKernelGGL(k_l2_b, dim3(nsr, ncols), dim3(256), (size_t)max_nL * 8, s, a);
}
size_t l2_d_smem(int max_nL) { return (size_t)std::max(1, max_nL) * 8; }

int set_l2_d_smem_limit(size_t bytes) {
    if (bytes <= 65536) return 0;
    return hipFuncSetAttribute((const void *)k_l2_d, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes) == hipSuccess
               ? 0 : -1;
}

void launch_l2_d(const L2Args &a, int nsr, size_t smem, hipStream_t s, int ncols) {
    hipLaunchKernelGGL(k_l2_d, dim3(nsr, ncols), dim3(256), smem, s, a);
}

}  // namespace bddc
