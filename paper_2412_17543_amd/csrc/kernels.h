// Kernel argument structs and launchers (kernels.hip).
#pragma once

#include "internal.h"

namespace bddc {

struct AsmDesc {
    const int32_t *elem_loc; const double *elem_c;
    const int32_t *inc_ptr, *inc_e, *inc_v;
    int nloc;
    double *K;
};

struct SymvArgs {
    const void *tiles;
    const int64_t *t_off;
    const int32_t *nB, *b_off, *gB;
    const int32_t *nc, *c_off;     // nullable: coarse-basis tile columns
    const double *x;
    double *y, *c;
    double *partial;               // nullable: no reduction
    Ctl *ctl;
    int mode;                      // 1: alpha = rho / pAp
    int gated;                     // skip when ctl->done
    double *d_hist, *a_hist;
    int hist_cap;
};

struct UpdArgs {
    int n;
    const int32_t *ptr, *idx;
    const double *loc, *p;
    double *x, *r;
    double *AP; int64_t ld; int cap;
    double *partial;
    Ctl *ctl;
    double *res_hist; int hist_cap;
    int max_it;
};

struct ZasmArgs {
    int n;
    const int32_t *ptr, *idx;
    const double *loc, *r;
    double *z;
    const double *AW; int64_t ld;
    const double *Lc;
    double *partial;
    Ctl *ctl;
    int first, gated;
    double *rho_hist, *b_hist, *mu_hist; int hist_cap;
};

struct PupdArgs {
    int n;
    const double *z;
    double *p;
    const double *W; int64_t ld;
    double *P; int cap;
    Ctl *ctl;
};

struct ResidArgs {
    int n, mode, stop_rule;
    const int32_t *ptr, *idx;
    const double *loc, *b;
    double *out;
    const double *W; int64_t ld;
    const double *Lc;
    double *partial;
    Ctl *ctl;
};

struct DeflArgs {
    int n, stop_rule;
    double *x, *r;
    const double *W, *AW; int64_t ld;
    double *partial;
    Ctl *ctl;
};

struct CondArgs {
    const int32_t *nI, *nB, *i_off, *b_off, *nodesI;
    const int64_t *k_off;
    const double *K, *F;
    double *yI, *t;
};

struct CondAsmArgs {
    int n;
    const int32_t *gamma, *ptr, *idx;
    const double *F, *loc;
    double *b, *partial;
    Ctl *ctl;
};

struct RecArgs {
    const int32_t *nI, *nB, *i_off, *b_off, *nodesI, *gB;
    const int64_t *k_off;
    const double *K, *x, *yI;
    double *u;
};

struct L2Args {
    Ctl *ctl;
    const int32_t *nL, *nI2, *L_off, *L, *I2_off, *B2_off, *g2;
    const int32_t *cptr, *cidx_asm;      // level-1 coarse DOF -> positions in locc
    const double *locc;
    const int64_t *K2_off; const double *K2;   // swept subregion matrices
    double *vI2, *t2, *rB2;
    const int32_t *asm2_ptr, *asm2_idx;  // level-2 interface DOF -> positions in the B2 arrays
    const int64_t *N2_off; const double *N2;
    const int64_t *P2_off; const double *Phi2;
    const int32_t *nc3, *C3_off;
    double *u2, *c3loc;
};

struct CoarseArgs {
    Ctl *ctl;
    int n;
    const int32_t *ptr, *idx;
    const double *loc;
    const double *Kneg;
    double *u;
};

struct ProlArgs {
    Ctl *ctl;
    int three;
    const int32_t *nB, *b_off, *nc, *c_off, *cidx, *cL;
    const void *tiles; const int64_t *t_off;
    const double *uCg;
    // three-level data
    const int32_t *sr_of_sub, *nL, *nI2, *I2_off, *B2_off, *g2, *asm2_ptr, *asm2_idx, *pos_sr;
    const int32_t *nc3, *C3_off, *c3;
    const int64_t *K2_off, *P2_off;
    const double *K2, *Phi2, *u2, *u3, *vI2;
    double *locu;
};

struct GemmArgs {
    int n;
    int64_t ld;
    const double *V1; int k1;
    const double *V2; int k2;
    const double *Y; int ncol, ldy;
    double *out;
};

struct GramArgs {
    int n, k;
    int64_t ld;
    const double *X, *Y;
    double *partial, *out;
    Ctl *ctl;
};

struct GradArgs {
    int64_t n_elem, n_nodes;
    int nx, ny, nz, n_rhs;
    const uint8_t *keep, *free_node;
    const double *coefh, *lam, *u;
    double *grad;
};

void launch_assemble(const AsmDesc *d, int n, hipStream_t s);
void launch_sweep(const SweepDesc *d, int n, int maxn, int *status, hipStream_t s);
void set_sweep_smem_limit(size_t bytes);
void launch_build_saddle(const SaddleDesc *d, int n, hipStream_t s);
void launch_pack(const PackDesc *d, int n, int prec, void *dst, hipStream_t s);
void launch_ptsp(const PtspDesc *d, int n, hipStream_t s);
void launch_dense_copy(const DenseCopyDesc *d, int n, hipStream_t s);
void launch_gather_sum(int64_t n, const int32_t *ptr, const int32_t *idx, const double *src, double *out, hipStream_t s);
size_t symv_smem(int prec, int max_nt, int max_ntc);
void set_symv_smem_limit(size_t bytes);
void launch_symv(const SymvArgs &a, int prec, int nsub, size_t smem, hipStream_t s);
void launch_update(const UpdArgs &a, hipStream_t s);
void launch_zasm(const ZasmArgs &a, hipStream_t s);
void launch_pupd(const PupdArgs &a, hipStream_t s);
void launch_resid(const ResidArgs &a, hipStream_t s);
void launch_defl_init(const DeflArgs &a, hipStream_t s);
void launch_cond_local(const CondArgs &a, int nsub, int max_nI, hipStream_t s);
void launch_cond_asm(const CondAsmArgs &a, hipStream_t s);
void launch_recover(const RecArgs &a, int nsub, int max_nB, hipStream_t s);
void launch_scatter_gamma(int n, const int32_t *gamma, const double *x, double *u, hipStream_t s);
void launch_l2_a(const L2Args &a, int nsr, int max_nL, hipStream_t s);
void launch_l2_b(const L2Args &a, int nsr, int max_nL, hipStream_t s);
void launch_coarse_solve(const CoarseArgs &a, hipStream_t s);
void launch_prolong(const ProlArgs &a, int prec, int nsub, size_t smem, hipStream_t s);
void launch_recycle_gemm(const GemmArgs &a, hipStream_t s);
void launch_gram(const GramArgs &a, int nblocks, hipStream_t s);
void launch_elem_grad(const GradArgs &a, hipStream_t s);
void launch_copy(int64_t n, const double *src, double *dst, hipStream_t s);

}  // namespace bddc
