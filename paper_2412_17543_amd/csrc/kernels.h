// Kernel argument structs and launchers (kernels.hip: setup and per-solve
// kernels; hot.hip: the kernels of one deflated-PCG iteration).
#pragma once

#include "internal.h"

namespace bddc {

// ============================================================ setup kernels
// Schur complement of one subdomain's interface Schur complement S onto a
// subset of its interface entries (adaptive face selection, Section 3.3):
// W = S(perm, perm) with the p entries to eliminate first; keep = W(p:, p:)
// before and hat = W(p:, p:) after eliminating them (m = n - p).
struct FaceSchurDesc {
    const double *S; int ld;
    const int32_t *perm; int n, p;
    double *work;                  // n x n scratch
    double *hat, *keep;            // m x m each, row-major
};

struct AsmDesc {
    const int32_t *elem_loc; const double *elem_c;
    const int32_t *inc_ptr, *inc_e, *inc_v;
    int nloc;
    double *K;
};

// ======================================================== operator products
// One segment of a batched symmetric product: tiles [t0, t1) of the packed
// tile sequence of one subdomain, whose tiles start at tile `tile` of the
// operator array; the subdomain has n rows, and its input entries are
// x[gB[x_off + k]], k < n.  The segment writes its partial products to
// ypart[yoff + k].  Item b is the first
// segment of block b, `next` the index of the block's next one (-1: none);
// an empty item (t0 == t1, n == 0) does nothing.  All that a block needs to
// start a segment is in this one record.
struct SymvItem {
    int32_t tile, t0, t1, n;
    int32_t x_off, yoff, next;
    int32_t ntf, ntl, strip;        // the subdomain's tile rows, tiles, 1 if its tail is a strip
    int32_t sub, chunk;             // the subdomain, and this segment's index among its segments
};

// A batch of packed symmetric operators in the slot layout of tile_rows and
// strip_len: the tiles, then, for a short ragged tail, the strip of its
// rows.  The
// concatenated slot sequence of all subdomains is cut into n_blocks ranges,
// one per block, and each range into segments inside single subdomains; the
// segment holding a subdomain's first strip slot also applies the strip.  Segment c of
// subdomain i writes its partial products to ypart[pb[i] + c * nB[i] + k].
struct OpDev {
    const void *tiles;
    const int64_t *t_off;
    const int32_t *nB, *b_off, *gB;
    const SymvItem *items;          // n_blocks first segments, then the others
    int n_blocks;
    const int32_t *nchunk, *pb;
};

// Assembled entry t is the sum of part[idx[e]] for e in [ptr[t], ptr[t+1]):
// the partial products of all work items of all owners, in a fixed order.
struct Gather {
    const int32_t *ptr, *idx;
    const double *part;
};

struct SymvArgs {
    OpDev op;
    const double *x;                // global interface vector
    double *ypart;
    double *dot;                    // nullable: per-item x_i^T y_i partials
    // Neumann batch with a coarse space: segment c of the C segments of
    // subdomain i also writes the DOFs q = c, c + C, ... of c_i = (D Phi_i)^T
    // x_i to cpart[c_off[i] + q] (nullable)
    double *cpart;
    const void *phir;               // D Phi_i, column-major (rows of phi_ld(n) entries), local precision
    const int64_t *phr_off;
    const int32_t *nc, *c_off;
    Ctl *ctl;
    int gated;                      // return when ctl->done
    // stopping test made at the start (Section 5), on the residual whose
    // per-block ||r||^2 partials the previous kernel wrote
    int test;                       // 0 none, 1 in the loop, 2 on r_0 (first)
    int defer;                      // leave the test to k_pupd while ctl->record
    int stop_rule, max_it;
    const double *rr_part; int rr_n;
    const double *bb_part; int bb_n;
    double *res_hist; int hist_cap;
};

struct UpdArgs {                    // Alg. 1, lines 9-11
    int n;
    Gather q;                       // q = A p from the Schur partials
    const double *p;
    double *x, *r;
    double *AP; int64_t ld; int cap;
    const double *dot; int dot_n;   // p^T A p partials
    double *rr_part;
    Ctl *ctl;
    double *d_hist, *a_hist;
    const double *rho_hist;
    int hist_cap;
};

struct CrestArgs {                  // c_i = (D Phi_i)^T R_i x (right-hand side of eq. coarse_problem)
    Ctl *ctl;                       // returns when ctl->done
    const int32_t *nB, *b_off, *gB, *nc, *c_off;
    const void *phir;               // D Phi_i, column-major (rows of phi_ld(n) entries), local precision
    const int64_t *phr_off;
    const double *X; int64_t ldx;   // ncols columns of the interface vector
    double *part; int64_t cs;       // partial of column j, DOF q of subdomain i: part[j * cs + c_off[i] + q]
    int ncols;
    int cols;                       // columns whose gathered x is staged in LDS at a time
};

struct ProlArgs {                   // w_i = u_i + D Phi_i u_C (eq. averaging_subdomain_solves)
    Ctl *ctl;
    int gated;
    const int32_t *nB, *b_off, *nc, *c_off, *cidx;
    const int32_t *nchunk, *pb;     // Neumann work items per subdomain, partial bases
    const double *upart;
    const void *phir;               // D Phi_i, column-major (rows of phi_ld(n) entries), local precision
    const int64_t *phr_off;
    const double *uC;               // level-1 coarse solution (nullable: no coarse space)
    double *wloc;
    const int32_t *ch_sub, *ch_row; // block b: subdomain ch_sub[b], rows ch_row[b] .. +511
    int64_t cs_u, cs_uC, cs_w;      // several columns (blockIdx.y): strides of upart, uC, wloc
};

struct ZasmArgs {                   // z = sum_i R_i^T w_i, rho, (AW)^T z
    int n;
    Gather w;
    const double *r;
    double *z;
    const double *AW; int64_t ld;
    double *part;                   // nullable: (r^T z, (AW)^T z) per block, column-major
    Ctl *ctl;
    int gated, advance;
    int64_t cs_w, cs_r, cs_z;       // several columns (blockIdx.y; no partials): strides
};

struct PupdArgs {                   // Alg. 1, lines 14-16 (line 7 when first)
    int n;
    const double *z;
    double *p;
    const double *W; int64_t ld;
    double *P; int cap;
    const double *zpart; int zpart_n;
    const double *WAWinv;
    Ctl *ctl;
    int first, hist_only, gated;
    double *rho_hist, *b_hist, *mu_hist; int hist_cap;
    // stopping test deferred from the preconditioner's product while the
    // basis is recording (0 none, 1 in the loop, 2 on r_0)
    int test, stop_rule, max_it;
    const double *rr_part; int rr_n;
    const double *bb_part; int bb_n;
    double *res_hist;
};

struct ResidArgs {                  // out = b - sum of the Schur partials
    int n, want_wtr;
    Gather q;
    const double *b;
    double *out;
    const double *W; int64_t ld;
    Ctl *ctl;
    double *part;                   // (||out||^2, W^T out) per block, column-major
};

struct DeflArgs {                   // Alg. 1, lines 3-4
    int n;
    double *x, *r;
    const double *W, *AW; int64_t ld;
    const double *wpart; int wpart_n;
    const double *WAWinv;
    double *rr_part;
    Ctl *ctl;
};

struct ReorthArgs {                 // Alg. 1 optional line: r -= W (W^T W)^{-1} W^T r
    int n;
    double *r;
    const double *W; int64_t ld;
    const double *WWinv;            // (W^T W)^{-1}, k x k
    double *part;                   // W^T r per block, column-major (k columns x grid)
    double *rr_part;                // ||r||^2 per block after the projection
    Ctl *ctl;
};

struct ReduceArgs {                 // out[c] = sum_b part[c * n + b]
    const double *part;
    int n, ncol;
    double *out;
};

// ============================================================ coarse levels
// u_C = sign * M r_C with a dense row-major n x n matrix M (r_C assembled by
// a first kernel, the product by a second): two levels,
// M = -K_C^{-1} (sign -1); three levels in explicit form, M = the level-2
// BDDC operator assembled at setup (sign +1); level 3 of the three-level
// chain, M = -K_3^{-1} (sign -1).
struct CoarseDenseArgs {
    Ctl *ctl;
    int n;
    Gather rc;                      // r_C from the coarse partials
    double *r;                      // assembled r_C (n)
    const double *M; int64_t ldm;   // rows padded to an even length (16-byte aligned)
    double sign;
    double *u;
    int64_t cs_rc, cs_r, cs_u;      // several columns (blockIdx.y): strides of rc.part, r, u
};

// Symmetric product u = K r with the upper triangle of K in 64 x 64 blocks
// (I, J >= I), each row-major and zero past n; block (I, J) has index
// I nb - I (I - 1) / 2 + J - I and bI[b] = I.  Per block: 64 row sums, then
// (J > I) 64 column sums, in part[128 b ...]; a second pass adds them.
struct SymBlkArgs {
    Ctl *ctl;
    int n, nb;                      // order, 64-row panels
    const double *B;
    const int32_t *bI;
    const double *r;
    double *part;
    double *u;
};

struct L2Args {
    Ctl *ctl;
    Gather rc;                      // level-1 coarse residual from the coarse partials
    const int32_t *nL, *nI2, *L_off, *L, *I2_off, *B2_off, *g2;
    const int64_t *K2_off; const double *K2;   // swept subregion matrices
    double *vI2, *t2, *rB2;
    const int32_t *asm2_ptr, *asm2_idx;        // level-2 interface DOF -> B2 positions
    const int64_t *N2_off; const double *N2;
    const int64_t *P2_off; const double *Phi2;
    const int32_t *nc3, *C3_off, *c3;
    double *u2, *c3loc;
    const int32_t *pos_sr;
    const uint8_t *own2;
    const double *u3;
    double *uC;
    // level-2 interface positions: offset of the position's D Phi row and
    // of its subregion's level-3 DOF list, level-3 DOFs of that subregion
    const int64_t *ph_off;
    const int32_t *c3o, *n3p;
    int n3, max_nL;
    // several columns (blockIdx.y): strides of rc.part and the per-column buffers
    int64_t cs_rc, cs_vI2, cs_t2, cs_rB2, cs_u2, cs_c3loc, cs_u3, cs_uC;
};


// ====================================================== per-solve kernels
struct CondArgs {                   // t_i = K_BI y_I, y_I from the interior-product partials
    const int32_t *nI, *nB, *i_off, *b_off;
    const int32_t *nchunk, *pb;
    const double *ypart;
    const int32_t *kbi_ptr, *kbi_col;   // interface rows (b_off based), interior columns
    const double *kbi_val;
    double *t;
};

struct CondAsmArgs {
    int n;
    const int32_t *gamma, *ptr, *idx;
    const double *F, *loc;
    double *b, *part;
};

struct RecArgs {                    // out[nodesI] = F_I - K_IB x_B; then u[nodesI] = y_I
    const int32_t *nI, *nB, *i_off, *b_off, *nodesI, *gB;
    const double *x, *F;
    const int32_t *kib_ptr, *kib_col;   // interior rows (i_off based), interface columns
    const double *kib_val;
    double *out;
    const int32_t *nchunk, *pb;
    const double *ypart;
    double *u;
};

// Two products of the same shape (blockIdx.y picks one): out[y] = [V1[y], V2[y]] Y.
struct GemmArgs {
    int n;
    int64_t ld;
    const double *V1[2]; int k1;
    const double *V2[2]; int k2;
    const double *Y; int ncol, ldy;
    double *out[2];
};

struct GramArgs {
    int n, k;
    int64_t ld;
    int k2;                         // columns of Y (0: k)
    const double *X, *Y;
    double *part;
};

struct CholArgs {                   // new W^T A W: Cholesky, inverse, commit flag
    int k;
    const double *waw;              // k x k Gram product (row-major)
    double *waw_sym;                // symmetrised copy for the host
    double *inv;                    // k x k inverse (written when SPD)
    RecState *state;
};

struct CommitArgs {                 // the new basis's inverse when state->ok, else the basis dropped
    int ncol;
    int nullc;                      // leading null-space columns kept on a drop (0 or 1)
    const double *inv_new;
    double *inv;
    const double *ww_new;           // nullable: (W^T W)^{-1} of the new basis
    double *ww;
    RecState *state;
};

struct GradArgs {
    int64_t n_elem, n_nodes;
    int nx, ny, nz, n_rhs;
    const uint8_t *keep, *free_node;
    const double *coefh, *lam, *u;
    double *grad;
};

// setup (kernels.hip)
void launch_assemble(const AsmDesc *d, int n, hipStream_t s);
void launch_rank1(double *A, int64_t ld, int n, const double *e, double coef, hipStream_t s);
// batched symmetric sweeps in panels of 16 pivots (sweep.hip): the panel
// buffer holds 2 x 16 x n doubles per matrix at the offsets the sizing call
// returns; pivots below pos_end must be positive, the others negative
int64_t sweep_panel_doubles(const std::vector<SweepDesc> &h, std::vector<int64_t> &off);
void launch_sweep_blocked(const SweepDesc *d, const int64_t *d_off, const std::vector<SweepDesc> &h, double *buf,
                          int *status, hipStream_t s);
// face Schur complements (adaptive step): gather S(perm, perm) into work and
// its trailing block into keep, sweep the leading p pivots (d_sw, d_off and
// panel sized for the batch by the caller), trailing block into hat
void launch_face_schur(const FaceSchurDesc *d, const std::vector<FaceSchurDesc> &h, SweepDesc *d_sw, int64_t *d_off,
                       double *panel, int *status, hipStream_t s);
void launch_build_saddle(const SaddleDesc *d, int n, hipStream_t s);
void launch_pack(const PackDesc *d, int n, int prec, void *dst, void *phir, hipStream_t s);
void launch_ptsp(const PtspDesc *d, int n, hipStream_t s);
void launch_dense_copy(const DenseCopyDesc *d, int n, hipStream_t s);
void launch_gather_sum(int64_t n, const int32_t *ptr, const int32_t *idx, const double *src, double *out, hipStream_t s);
// per solve (kernels.hip)
void launch_cond_local(const CondArgs &a, int nsub, int max_nI, hipStream_t s);
void launch_cond_asm(const CondAsmArgs &a, int grid, hipStream_t s);
void launch_rec_rhs(const RecArgs &a, int nsub, int max_nB, hipStream_t s);
void launch_rec_out(const RecArgs &a, int nsub, hipStream_t s);
void launch_scatter_gamma(int n, const int32_t *gamma, const double *x, double *u, hipStream_t s);
void launch_recycle_gemm(const GemmArgs &a, hipStream_t s, int ny = 2);   // ny: outputs (1 or 2)
void launch_gram(const GramArgs &a, int nblocks, hipStream_t s);

// ============================================================ block products (block.hip)
struct BlockItem {                  // one subdomain of a block product
    int64_t tile;                   // its first tile (in tiles) in the packed operator
    int32_t n;                      // rows
    int32_t xoff;                   // offset in the local interface (or interior) arrays
};
struct BlockSymvArgs {
    const double *tiles;            // float64 tiles
    const BlockItem *items;
    const int32_t *gB;              // local interface position -> interface index
    const double *X; int64_t ldx; int ncols;   // input block, column-major
    double *ypart; int64_t ylen;    // y of subdomain i, column c: ypart[c ylen + xoff_i + k]
};
size_t symm_smem_bytes(int max_n);
int set_symm_smem_limit(size_t bytes);
void launch_symm(const BlockSymvArgs &a, int nsub, size_t smem, hipStream_t s);
void launch_gather_block(int n, const int32_t *ptr, const int32_t *idx, const double *part, int64_t plen, double *out,
                         int64_t ldo, int ncols, hipStream_t s);
void launch_elem_grad(const GradArgs &a, hipStream_t s);
void launch_copy(int64_t n, const double *src, double *dst, hipStream_t s);
void launch_fill(int64_t n, double v, double *dst, hipStream_t s);
void launch_ctl_init(Ctl *ctl, double rtol2, int record, const RecState *state, int32_t *hflag, double *hprog,
                     int iter_stop, hipStream_t s);
// clear `done` and set the iteration at which the next run ends
void launch_resume(Ctl *ctl, int iter_stop, hipStream_t s);
void launch_set_done(Ctl *ctl, int v, hipStream_t s);
void launch_set_state(RecState *state, int k, int ok, hipStream_t s);
void launch_chol_inv(const CholArgs &a, hipStream_t s);
void launch_commit(const CommitArgs &a, hipStream_t s);
// iteration (hot.hip)
struct SymvCfg {
    int nw;                         // waves per block: 4 or 8
    int unroll;                     // tiles in flight per wave: 2 or 4
};
// which batch of operators a product streams: the three get kernels of
// their own name (k_symv<T, waves, tiles in flight, OpSchur | OpNeumann |
// OpInterior>) so that profiles time them apart
enum SymvOp { SYMV_SCHUR = 0, SYMV_NEUMANN = 1, SYMV_INTERIOR = 2 };
size_t symv_smem(int prec, int nw, int max_nt);
int set_symv_smem_limit(size_t bytes);
void launch_symv(const SymvArgs &a, SymvOp op, int prec, SymvCfg cfg, size_t smem, hipStream_t s);
void launch_update(const UpdArgs &a, int grid, hipStream_t s);
void launch_crest(const CrestArgs &a, int prec, int nsub, int max_nB, hipStream_t s);
int crest_cols(int prec, int max_nB, int ncols);
void launch_prolong(const ProlArgs &a, int prec, int nblocks, int max_nc, hipStream_t s, int ncols = 1);
void launch_zasm(const ZasmArgs &a, int kmax, int grid, hipStream_t s, int ncols = 1);
void launch_pupd(const PupdArgs &a, int kmax, int grid, hipStream_t s);
void launch_resid(const ResidArgs &a, int kmax, int grid, hipStream_t s);
void launch_defl_init(const DeflArgs &a, int kmax, int grid, hipStream_t s);
void launch_reduce(const ReduceArgs &a, hipStream_t s);
void launch_reorth(const ReorthArgs &a, int kmax, int grid, hipStream_t s);
void launch_coarse_dense(const CoarseDenseArgs &a, hipStream_t s, int ncols = 1);
// u = K r for the block layout of SymBlkArgs (r first gathered like the dense form's)
void launch_coarse_symblk(const CoarseDenseArgs &g, const SymBlkArgs &a, hipStream_t s);
void launch_pack_symblk(const double *M, int64_t ldm, int n, int nb, const int32_t *bI, double sign, double *B,
                        hipStream_t s);
void launch_l2_a(const L2Args &a, int nsr, int max_nL, hipStream_t s, int ncols = 1);
void launch_l2_b(const L2Args &a, int nsr, int max_nL, hipStream_t s, int ncols = 1);
size_t l2_d_smem(int max_nL);
int set_l2_d_smem_limit(size_t bytes);
void launch_l2_d(const L2Args &a, int nsr, size_t smem, hipStream_t s, int ncols = 1);
// deflation-column bucket of the templated reductions (0, 8, 16, 32, 64)
int kmax_bucket(int k);

}  // namespace bddc
