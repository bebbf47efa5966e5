// Block products of the block adjoint and of grouped condensation (several
// right-hand sides at once): the batched symmetric products y_i = S_i x_i
// (Schur), u_i = D N_i D g_i (Neumann, eq. localCorr) or K_II^{-1} b_i
// (interior), 16 columns at a time, on the matrix cores, and the assembly of
// the per-subdomain results.
//
// k_symm: one block per (subdomain, 16-column chunk), 4 waves; a wave keeps
// PF tiles in flight (a fixed ring of load slots, reissued on every step).  The block
// stages X_i (n x 16) in LDS, then walks the packed upper-triangle tiles one
// tile row I at a time; inside a row, wave w takes the tiles q = w, w + 4, ...
// (J = I + q):
//   row part    Y_I += T X_J          (accumulated in the wave's registers)
//   column part Y_J += T^T X_I, J > I (added to LDS; each J once per row)
// After the row the waves' row parts are added into Y_I in wave order, so
// every entry is summed in a fixed order (the product is reproducible bit by
// bit).  A short ragged tail stored as a strip after the tiles (uses_strip)
// follows as one more tile row.  A tile is loaded once (two 16-byte loads
// per lane, the layout of tile_index), written to the wave's LDS slot in
// row-major order and read
// back as MFMA operands: v_mfma_f64_16x16x4f64 takes A[i][k] and B[k][j] in
// lane i (j) + 16 k and returns (i, j) in lane j + 16 (i % 4), register i / 4.
#include <hip/hip_runtime.h>

#include "internal.h"
#include "kernels.h"

namespace bddc {

namespace {

typedef double dvec4 __attribute__((ext_vector_type(4)));
typedef double dvec2 __attribute__((ext_vector_type(2)));

constexpr int XS = 17;              // LDS row stride (doubles) of X, Y and a tile
constexpr int PF = 8;               // tiles each wave has in flight (one wave per SIMD: registers to spare)

// Workgroup barrier that orders LDS only: the tile loads in flight are not
// waited for (a plain __syncthreads() would drain them at every row end).
__device__ __forceinline__ void lds_barrier() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
    __builtin_amdgcn_s_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

__device__ __forceinline__ void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

typedef unsigned int uvec4 __attribute__((ext_vector_type(4)));

// Raw buffer over `bytes` bytes from p: loads at or past the end return zero
// without a memory access.
__device__ __forceinline__ __amdgpu_buffer_rsrc_t raw_rsrc(const void *p, int64_t bytes) {
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void *>(p), 0, (int)min(bytes, (int64_t)INT32_MAX), 0x00020000);
}

// The tiles of one wave in order: rows I = 0, 1, ... and in row I the tiles
// q = w, w + 4, ... (nt - I of them); `tile` is the index in the
// subdomain's packed sequence, past the end once the wave has no more.
struct TileSeq {
    int I, q, nt, w;
    int64_t base;
    __device__ void norm() {
        while (I < nt && q >= nt - I) { base += nt - I; ++I; q = w; }
    }
    __device__ void next() { q += 4; norm(); }
    __device__ int64_t tile(int64_t total) const { return I < nt ? base + q : total; }
};

__global__ void __launch_bounds__(256) k_symm(BlockSymvArgs a) {
    extern __shared__ __align__(16) double sm[];
    // the column chunks of one subdomain are adjacent blocks: they run at the
    // same time, so the second reads the tiles from the shared cache
    const int nch = (a.ncols + 15) / 16;
    const BlockItem it = a.items[blockIdx.x / nch];
    const int c0 = 16 * (int)(blockIdx.x % nch);
    const int n = it.n;
    const int nt = tile_rows(n), npad = 16 * ((n + 15) / 16);   // nt: tile rows (without a strip's rows)
    const int64_t total = full_tiles(n);
    double *xs = sm;                                   // npad x 16 (stride XS)
    double *ys = xs + (size_t)npad * XS;               // npad x 16
    double *ts = ys + (size_t)npad * XS;               // 4 tiles of 16 x 16
    double *red = ts + 4 * 16 * XS;                    // 4 x 256
    const int tid = threadIdx.x, w = tid >> 6, L = tid & 63, li = L & 15, lk = L >> 4;
    const int wu = __builtin_amdgcn_readfirstlane(w);
    const int32_t *gb = a.gB + it.xoff;
    // the wave's first PF tiles are requested before anything else
    const __amdgpu_buffer_rsrc_t rs = raw_rsrc(a.tiles + it.tile * 256, total * 2048);
    TileSeq ld{0, wu, nt, wu, 0};
    ld.norm();
    uvec4 fa[PF], fb[PF];
#pragma unroll
    for (int d = 0; d < PF; ++d) {
        const int off = (int)ld.tile(total) * 2048 + L * 16;
        fa[d] = __builtin_amdgcn_raw_buffer_load_b128(rs, off, 0, 0);
        fb[d] = __builtin_amdgcn_raw_buffer_load_b128(rs, off + 1024, 0, 0);
        ld.next();
    }
    // X_i: 8 entries per thread at a time, all index loads before the gathers
    for (int e0 = tid; e0 < 16 * npad; e0 += 256 * 8) {
        int gi[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const int e = e0 + 256 * u, cc = e / npad, k = e - cc * npad;
            gi[u] = (e < 16 * npad && k < n && c0 + cc < a.ncols) ? gb[k] : -1;
        }
        double v[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const int e = e0 + 256 * u, cc = e / npad;
            v[u] = gi[u] >= 0 ? a.X[(int64_t)(c0 + cc) * a.ldx + gi[u]] : 0.0;
        }
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const int e = e0 + 256 * u, cc = e / npad, k = e - cc * npad;
            if (e < 16 * npad) xs[k * XS + cc] = v[u];
        }
    }
    for (int e = tid; e < npad * XS; e += 256) ys[e] = 0.0;
    __syncthreads();
    double *tw = ts + w * 16 * XS;
    dvec4 racc = {0.0, 0.0, 0.0, 0.0};
    int rows_done = 0;
    // end of row I: the waves' row parts into Y_I in wave order (every wave
    // passes here once per row, in row order)
    auto row_end = [&](int I) {
#pragma unroll
        for (int r = 0; r < 4; ++r) red[w * 256 + (4 * r + lk) * 16 + li] = racc[r];
        lds_barrier();
        {
            const int row = tid >> 4, col = tid & 15;
            ys[(16 * I + row) * XS + col] += ((red[tid] + red[256 + tid]) + red[512 + tid]) + red[768 + tid];
        }
        lds_barrier();
        racc = dvec4{0.0, 0.0, 0.0, 0.0};
    };
    TileSeq cur{0, wu, nt, wu, 0};
    cur.norm();
    // one tile from ring slot d, whose load is then reissued for the tile PF
    // places later (slots are never copied, so no wait but for slot d's own load)
    auto step = [&](uvec4 &sa, uvec4 &sb) {
        const bool valid = cur.I < nt;                 // (wave-uniform)
        const int I = cur.I, J = cur.I + cur.q;
        if (valid) {
            while (rows_done < I) row_end(rows_done++);
            tw[(4 * lk + 0) * XS + li] = __hiloint2double(sa.y, sa.x);
            tw[(4 * lk + 1) * XS + li] = __hiloint2double(sa.w, sa.z);
            tw[(4 * lk + 2) * XS + li] = __hiloint2double(sb.y, sb.x);
            tw[(4 * lk + 3) * XS + li] = __hiloint2double(sb.w, sb.z);
        }
        // reissued on every step (past the end: a zero read, no access), so
        // that the count of loads in flight is the same on every path
        const int off = (int)ld.tile(total) * 2048 + L * 16;
        sa = __builtin_amdgcn_raw_buffer_load_b128(rs, off, 0, 0);
        sb = __builtin_amdgcn_raw_buffer_load_b128(rs, off + 1024, 0, 0);
        ld.next();
        if (!valid) return;
        wave_sync();
#pragma unroll
        for (int s = 0; s < 4; ++s)
            racc = __builtin_amdgcn_mfma_f64_16x16x4f64(tw[li * XS + 4 * s + lk],
                                                        xs[(16 * J + 4 * s + lk) * XS + li], racc, 0, 0, 0);
        if (J > I) {
            dvec4 cacc = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
            for (int s = 0; s < 4; ++s)
                cacc = __builtin_amdgcn_mfma_f64_16x16x4f64(tw[(4 * s + lk) * XS + li],
                                                            xs[(16 * I + 4 * s + lk) * XS + li], cacc, 0, 0, 0);
#pragma unroll
            for (int r = 0; r < 4; ++r) ys[(16 * J + 4 * r + lk) * XS + li] += cacc[r];
        }
        wave_sync();
        cur.next();
    };
    while (cur.I < nt) {
#pragma unroll
        for (int d = 0; d < PF; ++d) step(fa[d], fb[d]);
    }
    while (rows_done < nt) row_end(rows_done++);
    // loads issued past the wave's last tile read nothing; make sure none is
    // outstanding at exit
#pragma unroll
    for (int d = 0; d < PF; ++d) asm volatile("" ::"v"(fa[d]), "v"(fb[d]));
    // The ragged tail rows n0 + r, r < rem, stored whole as a row-major strip
    // after the tiles: one more tile row, whose 16-column chunks are the
    // chunks q < nt (row part and column part, as for a tile) and the corner
    // q = nt (the full rem x rem block: row part only).  Wave w takes the
    // chunks q = w, w + 4, ...; a chunk's rows of Y belong to that wave alone.
    const int rem = uses_strip(n) ? n % 16 : 0;
    if (rem > 0) {
        const int n0 = 16 * nt, nq = nt + 1;
        const double *sp = a.tiles + (it.tile + total) * 256;
        constexpr int G = 4;        // chunks whose entries are requested together
        for (int q0 = wu; q0 < nq; q0 += 4 * G) {
            double v[G][4];
#pragma unroll
            for (int g = 0; g < G; ++g) {
                const int q = q0 + 4 * g;
                const int cb = q < nt ? 16 * q : n0;
                const int cv = q < nt ? 16 : rem;
#pragma unroll
                for (int s = 0; s < 4; ++s) {
                    const int r = 4 * lk + s;
                    v[g][s] = (q < nq && r < rem && li < cv) ? sp[(int64_t)r * n + cb + li] : 0.0;
                }
            }
#pragma unroll
            for (int g = 0; g < G; ++g) {
                const int q = q0 + 4 * g;
                if (q >= nq) break;                        // (wave-uniform)
#pragma unroll
                for (int s = 0; s < 4; ++s) tw[(4 * lk + s) * XS + li] = v[g][s];
                wave_sync();
                // row part: Y_rag += T X_q (the corner: X rows n0..)
#pragma unroll
                for (int s = 0; s < 4; ++s)
                    racc = __builtin_amdgcn_mfma_f64_16x16x4f64(tw[li * XS + 4 * s + lk],
                                                                xs[(16 * q + 4 * s + lk) * XS + li], racc, 0, 0, 0);
                if (q != nt) {          // column part: Y_q += T^T X_rag
                    dvec4 cacc = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
                    for (int s = 0; s < 4; ++s)
                        cacc = __builtin_amdgcn_mfma_f64_16x16x4f64(tw[(4 * s + lk) * XS + li],
                                                                    xs[(n0 + 4 * s + lk) * XS + li], cacc, 0, 0, 0);
#pragma unroll
                    for (int r = 0; r < 4; ++r) ys[(16 * q + 4 * r + lk) * XS + li] += cacc[r];
                }
                wave_sync();
            }
        }
        row_end(nt);                // the waves' row parts into Y rows n0.. in wave order
    }
    for (int e = tid; e < 16 * n; e += 256) {
        const int cc = e / n, k = e - cc * n, col = c0 + cc;
        if (col < a.ncols) a.ypart[(int64_t)col * a.ylen + it.xoff + k] = ys[k * XS + cc];
    }
}

// out[g + col ldo] = sum of part[col plen + idx[e]], e in [ptr[g], ptr[g+1])
__global__ void __launch_bounds__(256) k_gather_block(int n, const int32_t *ptr, const int32_t *idx,
                                                      const double *part, int64_t plen, double *out, int64_t ldo,
                                                      int ncols) {
    const int g = blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= n) return;
    const int e0 = ptr[g], e1 = ptr[g + 1];
    for (int col = blockIdx.y; col < ncols; col += gridDim.y) {
        const double *p = part + (int64_t)col * plen;
        double s = 0.0;
        for (int e = e0; e < e1; ++e) s += p[idx[e]];
        out[g + (int64_t)col * ldo] = s;
    }
}

}  // namespace

size_t symm_smem_bytes(int max_n) {
    const int npad = 16 * ((max_n + 15) / 16);
    return sizeof(double) * ((size_t)2 * npad * XS + 4 * 16 * XS + 4 * 256);
}

int set_symm_smem_limit(size_t bytes) {
    return hipFuncSetAttribute((const void *)k_symm, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes) !=
                   hipSuccess
               ? 1
               : 0;
}

void launch_symm(const BlockSymvArgs &a, int nsub, size_t smem, hipStream_t s) {
    if (nsub <= 0 || a.ncols <= 0) return;
    hipLaunchKernelGGL(k_symm, dim3(nsub * ((a.ncols + 15) / 16)), dim3(256), smem, s, a);
}

void launch_gather_block(int n, const int32_t *ptr, const int32_t *idx, const double *part, int64_t plen, double *out,
                         int64_t ldo, int ncols, hipStream_t s) {
    if (n <= 0 || ncols <= 0) return;
    hipLaunchKernelGGL(k_gather_block, dim3((n + 255) / 256, std::min(ncols, 8)), dim3(256), 0, s, n, ptr, idx, part,
                       plen, out, ldo, ncols);
}

}  // namespace bddc
