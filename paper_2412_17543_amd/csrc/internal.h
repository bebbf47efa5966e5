// Internal declarations of the BDDC / deflated-PCG library (not part of the ABI).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

#include "bddc.h"

namespace bddc {

constexpr int TILE = 16;          // symmetric operators are stored as 16x16 tiles

// Packed symmetric operator of n rows in slots of 256 entries: 16-row tile
// rows, tile row I holding the tiles (I, I..nt-1) of the upper triangle.  A
// short ragged tail (n % 16 = 1..8 rows, n <= 512) is stored after the
// nt = n / 16 full tile rows as a row-major strip of its whole rows, padded
// to whole slots: its tile column would be mostly zero padding.  Otherwise
// the last tile row and column are zero-padded (nt = ceil(n / 16)) -- a long
// strip would cost the product more round trips than its padding costs bytes.
__host__ __device__ inline bool uses_strip(int n) {
    const int rem = n % TILE;
    return rem != 0 && rem <= 8 && n <= 512;
}
__host__ __device__ inline int tile_rows(int n) { return uses_strip(n) ? n / TILE : (n + TILE - 1) / TILE; }
__host__ __device__ inline int full_tiles(int n) {
    const int nt = tile_rows(n);
    return nt * (nt + 1) / 2;
}
__host__ __device__ inline int64_t strip_len(int n) { return uses_strip(n) ? (int64_t)(n % TILE) * n : 0; }
__host__ __device__ inline int64_t op_slots(int n) { return full_tiles(n) + (strip_len(n) + 255) / 256; }
// Row length of the column-major D Phi_i (n_c rows of n entries, zero to a
// multiple of 8 entries: 16-byte aligned rows in every storage precision).
__host__ __device__ inline int phi_ld(int n) { return (n + 7) & ~7; }
// zeroed bytes after every packed tile array: the product kernel's prefetch
// of up to 8 tiles past a work range stays inside the allocation
constexpr int64_t TILE_TAIL_BYTES = 8 * 256 * 8;
constexpr int RMAX = 64;          // largest deflation basis supported
constexpr int VGRID = 512;        // blocks of the grid-stride vector kernels (max)

// ---------------------------------------------------------------------------
// host-side structure built from mesh + partition (partition.cpp)
// ---------------------------------------------------------------------------
struct CoarseDof {
    int kind;                      // 0 corner, 1 face, 2 edge, 3 adaptive face row
    std::vector<int64_t> nodes;    // free nodes (sorted)
    std::vector<int32_t> subs;     // subdomains sharing it (sorted)
    std::vector<double> wts;       // row over `nodes`; empty: the average 1/|nodes|
};

struct SubHost {
    int nI = 0, nB = 0, nloc = 0;
    std::vector<int32_t> nodes;     // local free nodes: interior (sorted) then interface (sorted)
    std::vector<int32_t> gB;        // interface local k -> global interface index
    std::vector<int32_t> elem;      // element ids
    std::vector<int32_t> elem_loc;  // 8 local indices per element (-1: not a free node)
    std::vector<double> elem_c;     // coefficient * h per element
    std::vector<int32_t> inc_ptr, inc_e, inc_v;  // local node -> (element slot, vertex)
    std::vector<double> wB;         // interface weights D_i
    std::vector<int32_t> cidx;      // global coarse DOFs of this subdomain (ascending)
    std::vector<int32_t> c_ptr, c_col;  // constraint rows over interface-local indices
    std::vector<double> c_val;
};

struct SubregionHost {
    std::vector<int32_t> subs;      // member subdomains
    std::vector<int32_t> L;         // level-1 coarse DOFs: interior then interface
    int nI = 0, nB = 0;
    std::vector<int32_t> g2;        // interface local -> level-2 interface index
    std::vector<double> w;          // card weights on the interface
    std::vector<int32_t> c3;        // level-3 DOFs (ascending)
    std::vector<int32_t> c_ptr, c_col;
    std::vector<double> c_val;
};

struct Structure {
    int nx = 0, ny = 0, nz = 0;
    double h = 0;
    int64_t n_nodes = 0, n_elem = 0;
    std::vector<uint8_t> free_node;
    std::vector<int32_t> gamma;        // interface node ids (ascending)
    int n_sub = 0;
    std::vector<SubHost> sub;
    std::vector<CoarseDof> coarse;
    int n_corner = 0, n_face = 0, n_edge = 0, n_adaptive = 0;
    // level 2 (three-level BDDC)
    bool three = false;
    int n_sr = 0;
    std::vector<SubregionHost> sr;
    std::vector<int32_t> gamma2;       // level-1 coarse ids on the level-2 interface
    std::vector<std::vector<int32_t>> dof3_members;  // level-3 DOF -> level-1 coarse ids
    std::vector<std::vector<int32_t>> dof3_subs;     // level-3 DOF -> subregions
    std::vector<std::vector<double>> dof3_wts;       // its weights on those coarse ids
    std::vector<int8_t> dof3_kind;                   // 0 corner, 1 face, 3 level-1 adaptive row, 4 level-2 adaptive row
    int n3 = 0, n3_corner = 0, n3_face = 0, n3_adaptive = 0;
};

// A level-3 DOF added by the adaptive selection at level 2.
struct Level3Dof {
    std::vector<int32_t> members;   // level-1 coarse ids (a level-2 face)
    std::vector<double> wts;
    std::vector<int32_t> subs;      // the two subregions
};

int build_structure(const bddc_mesh *m, const bddc_partition *p, const double *coef,
                    const bddc_opts *o, Structure &st, std::string &err);
int constraint_rows(Structure &st, std::string &err);
int build_level2(Structure &st, const bddc_partition *p, std::string &err);
int add_coarse_dofs(Structure &st, const bddc_partition *p, const std::vector<CoarseDof> &extra, std::string &err);
int add_level3_dofs(Structure &st, const std::vector<Level3Dof> &extra, std::string &err);

// static device scratch of the allocation-free entry point (noalloc.hip)
int64_t noalloc_scratch_doubles();
int noalloc_scratch(double **out, std::string &err);

// host dense helpers (hostla.cpp)
bool cholesky(std::vector<double> &a, int n);                       // in place, lower
void chol_solve(const std::vector<double> &l, int n, double *x);
void sym_eig(std::vector<double> a, int n, std::vector<double> &w, std::vector<double> &v);

// ---------------------------------------------------------------------------
// device-side descriptors
// ---------------------------------------------------------------------------
struct SweepDesc {
    double *A;     // row-major symmetric matrix
    int n, ld;
    int p0, p1;    // pivots [p0, p1) are swept
    int pos_end;   // pivots < pos_end must be > 0, others < 0
};

struct SaddleDesc {
    const double *S; int ldS;      // nB x nB block
    int nB, nc;
    const int32_t *cptr, *ccol; const double *cval;  // constraint CSR (nc rows)
    double *M; int ldM;            // (nB+nc)^2 output
};

struct PackDesc {
    const double *src; int ld;     // n x n symmetric block
    int n;
    double sign;
    const double *D;               // nullable row/col scaling
    const double *phi; int ldphi;  // nullable n x nc coarse basis (scaled by D rows)
    int nc;
    int64_t dst;                   // element offset of the first tile
    int64_t phr;                   // element offset of the column-major
                                   // (D-scaled) coarse basis, or -1
};

struct PtspDesc {                  // K_C = Phi^T S Phi
    const double *S; int ldS;
    const double *Phi; int ldPhi;  // Phi stored in rows of a swept saddle matrix
    double phisign;
    int n, nc;
    double *X;                     // scratch n x nc
    double *out;                   // nc x nc
};

struct DenseCopyDesc {             // out[r][c] = sign * D[r] * src[r][c] (* D[c] when sym)
    const double *src; int ld;
    int rows, cols;
    double sign;
    const double *Drow, *Dcol;
    double *dst; int ldd;
};

// Control block of one solve, in device memory.  Every kernel of the
// iteration reads it at its start; a field is written (by block 0) only by a
// kernel none of whose other blocks read that field, so no block ever sees a
// half-updated control state.
struct Ctl {
    double rr;              // ||r_j||^2 of the last stopping test
    double bb;              // ||b||^2 of the condensed right-hand side
    double r0r0;            // ||r_0||^2
    double denom2;          // squared denominator of the stopping test
    double rtol2;           // squared relative tolerance
    double true_rr;         // ||b - A x||^2 after the loop
    double pAp, alpha;      // last p^T A p and alpha (diagnostics)
    int32_t done;           // 1: converged or failed; later kernels return at once
    int32_t iter;           // loop passes done (products with A inside the loop)
    int32_t status;         // 0 or BDDC_ENOTCONV / BDDC_EBREAKDOWN
    int32_t j;              // index of the current search direction p_j
    int32_t k;              // deflation columns in use
    int32_t record;         // store P, AP for recycling
    int32_t zero_rhs;       // b == 0: the solution is x = 0
    int32_t pfirst;         // 1: the next search direction starts a cycle (beta = 0)
    int32_t iter_stop;      // the run ends (without error) once iter reaches this
    int32_t *hflag;         // pinned host word set to 1 together with `done`
    double *hprog;          // pinned host doubles: ||r||^2 of the last test, its
                            // denominator, the iteration (read by the host to decide
                            // whether to queue another graph)
};

// Deflation-basis state kept on the device between solves: the columns in
// use and the outcome of the last basis update (1: committed).
struct RecState {
    int32_t k, ok;
};

// Marks the solve finished; the host polls hflag instead of copying ctl.
__device__ inline void ctl_finish(Ctl *c) {
    c->done = 1;
    if (c->hflag) *reinterpret_cast<volatile int32_t *>(c->hflag) = 1;
}

// Element index of entry (r, c) inside a 16x16 operator tile.  Lane
// l = 16 (r / 4) + c of a wave holds rows 4 (l / 16) .. + 3 of column l % 16;
// float64 tiles are stored as two 1 KB halves (rows i = 0,1 then 2,3 of every
// lane), float32 and bfloat16 tiles as 4 consecutive values per lane, so each
// wave-wide load is one contiguous, fully used block.
__host__ __device__ inline int tile_index(int r, int c, int elem_bytes) {
    const int l = 16 * (r >> 2) + c, i = r & 3;
    return elem_bytes == 8 ? ((i >> 1) * 128 + l * 2 + (i & 1)) : (l * 4 + i);
}

}  // namespace bddc
