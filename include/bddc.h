/*
 * bddc.h -- C ABI of the MI355X (gfx950) deflated-PCG / three-level BDDC solver.
 *
 * Solves a sequence of systems K u_k = F_k that share one SPD matrix K, the
 * Q1 (trilinear) discretisation of -div(c grad u) on a structured box with a
 * Dirichlet part of the boundary (Hanek, Papez & Sistek, arXiv 2412.17543,
 * Section 2: the pressure-corrector Poisson system with a fixed matrix and a
 * new right-hand side each time step).  Each system is reduced to the
 * interface between subdomains (Section 3.1, eq. Sug), solved by deflated
 * PCG (Section 4.1, Algorithm 1) preconditioned by two- or three-level BDDC
 * (Section 3.2, eqs. averaging_subdomain_solves, coarse_problem, localCorr),
 * with the deflation basis recycled from earlier solves (Section 4.2, eqs.
 * harmonicRitz and harmritzstopcrit), and the interior unknowns recovered.
 *
 * Conventions shared by every entry point
 *   - mesh: nx*ny*nz hexahedra of size h; node (ix,iy,iz) has index
 *     ix + (nx+1)*(iy + (ny+1)*iz), element (ex,ey,ez) has index
 *     ex + nx*(ey + ny*ez), element vertex v = a + 2b + 4c at offset (a,b,c).
 *   - nodal vectors are float64, length n_nodes = (nx+1)(ny+1)(nz+1), in that
 *     node order.  Entries at Dirichlet nodes and at nodes touched by no kept
 *     element are ignored on input and written as 0 on output.
 *   - "device" pointers are HIP device memory on the current device; "host"
 *     pointers are ordinary host memory.  The caller owns every buffer it
 *     passes; bddc_setup copies what it needs and the context owns all
 *     operators and the recycling state.
 *   - all GPU work is enqueued on the stream given to bddc_setup; a context is
 *     not thread-safe.  Entry points that return host results synchronise that
 *     stream before returning.
 *   - return value: 0 on success, a negative BDDC_E* code on failure; the
 *     message of the last failure of the calling thread is bddc_last_error().
 *     On failure no output is guaranteed except where stated.
 */
#ifndef BDDC_H
#define BDDC_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* error codes */
#define BDDC_OK          0
#define BDDC_EINVAL     -1   /* bad argument (sizes, null pointers, options)       */
#define BDDC_ENOMEM     -2   /* device or host allocation failed                   */
#define BDDC_EHIP       -3   /* a HIP runtime call failed                          */
#define BDDC_ESINGULAR  -4   /* a local, coarse or deflation matrix is singular    */
#define BDDC_ENOTCONV   -5   /* max_it reached without meeting the tolerance       */
#define BDDC_EBREAKDOWN -6   /* r^T z <= 0, p^T A p <= 0 or a NaN in the iteration */

/* constraint bit mask (Section 3.2: corners, face and edge averages) */
#define BDDC_CORNERS 1
#define BDDC_FACES   2
#define BDDC_EDGES   4

typedef struct bddc_ctx bddc_ctx;   /* opaque, owned by the library */

/* Structured box mesh.  h is the element size (the box is [0, nx*h] x ...). */
typedef struct {
    int32_t nx, ny, nz;
    double h;
    const uint8_t *elem_keep;       /* host, n_elem, nullable: 0 removes an element (holes) */
    const uint8_t *node_dirichlet;  /* host, n_nodes, nullable: default = nodes with ix == nx */
} bddc_mesh;

/* Element partition (Section 3.1: non-overlapping subdomains along element
 * boundaries) and, for three levels, the grouping of subdomains into
 * subregions (Section 3.2, multilevel paragraph).  Subdomains must be
 * connected through faces; removed elements carry any value. */
typedef struct {
    int32_t n_sub;
    const int32_t *elem_to_sub;      /* host, n_elem, values in [0, n_sub)          */
    int32_t n_subregion;             /* 0 -> two-level BDDC                          */
    const int32_t *sub_to_subregion; /* host, n_sub, values in [0, n_subregion)      */
} bddc_partition;

typedef struct {
    int32_t constraints;     /* BDDC_CORNERS | BDDC_FACES (| BDDC_EDGES)               */
    int32_t weights;         /* 0: card (1/multiplicity), 1: diag (stiffness diagonal) */
    int32_t local_prec;      /* storage of the constrained-Neumann operators N_i and
                                coarse bases Phi_i: 64 (float64), 32 (float32, float32
                                accumulation), 16 (bfloat16, float32 accumulation).
                                The Schur products, residuals, dot products, coarse
                                levels and deflation stay float64.                   */
    int32_t recycle_R;       /* maximal deflation-basis size R, 0 = plain PCG          */
    int32_t recycle_strategy;/* 4 = B4 (largest harmonic Ritz values, default),
                                3 = B3 (smallest), 2 = B2 (last R directions),
                                1 = B1 (first R directions)                          */
    double  ritz_freeze_tol; /* eq. harmritzstopcrit threshold (paper: 1e-5)            */
    int32_t stop_rule;       /* 0: ||r_k||/||b|| (eq. stopping_rhs), 1: ||r_k||/||r_0|| */
    int32_t init_guess;      /* 0: previous solution (default), 1: zero                 */
    int32_t max_it;          /* per right-hand side, e.g. 1000                          */
    int32_t save_cap;        /* max search directions stored per solve for recycling   */
    int32_t use_graph;       /* iterations launched in groups of two, queued ahead of
                                an asynchronous poll of the convergence flag:
                                2 (default) kernel by kernel into the stream;
                                1 as replays of a hipGraph captured once;
                                0: one iteration at a time with a host check after
                                every iteration (plain form); other values EINVAL    */
    int32_t autotune;        /* 1 (default): time a few work-list sizes, waves per
                                block and tiles in flight of the two batched operator
                                products at setup and keep the fastest; 0: fixed     */
    int32_t coarse_form;     /* three levels only: how the level-2 BDDC approximation
                                of K_C^{-1} is applied.  1: the subregion chain of
                                Section 3.2 (level-2 solves, level-3 coarse solve,
                                level-2 correction) at every application; 2: that
                                same linear operator assembled once at setup, column
                                by column through the chain, into a dense nC x nC
                                matrix applied as one product (nC <= 8192, else
                                EINVAL); 0 (default): 2 when nC <= 4096, else 1     */
    int32_t product_cfg[8];  /* optional fixed configuration of the two batched
                                products, Schur then Neumann: blocks per compute
                                unit, work split (1: blocks inside one subdomain,
                                0: equal ranges of the tile sequence), waves per
                                block (4 or 8), tiles in flight per wave (2 or 4).
                                A product whose first entry is 0 is autotuned (or
                                takes the default without autotuning).         */
    int32_t reorth;          /* 1: after every residual update, r -= W (W^T W)^{-1} W^T r
                                (Alg. 1, optional re-orthogonalisation); 0: off  */
    int32_t adapt_max_per_face; /* adaptive coarse space (Section 3.3): at most this
                                many new rows per face (paper: 10)                */
    double  adapt_tau;       /* > 0: enrich every level-1 face with the eigenvectors
                                of eq. eig-matrix whose eigenvalue exceeds tau
                                (rows from eq. c-def restricted to the face);
                                <= 0: off (default)                              */
    int32_t local_prec_set;  /* further storage precisions of N_i and Phi_i to build
                                at setup, from the same float64 solves, for
                                bddc_set_local_prec: bit mask 1 float64, 2 float32,
                                4 bfloat16 (local_prec is always built); 0 default */
    int32_t coef_log;        /* 1: coef holds log-coefficients theta_e and the element
                                coefficient is c_e = exp(theta_e); 0 (default): coef
                                holds c_e itself                                   */
    int32_t restart_every;   /* > 0: end a run of Algorithm 1 after this many passes
                                without convergence; the true residual then replaces
                                the recursive one and the iteration restarts from
                                line 5 (as after a residual replacement; not in the
                                paper).  0 (default): off                         */
    double  adapt2_tau;      /* three levels: > 0 enriches every level-2 face (coarse
                                DOFs shared by two subregions) in the same way, with
                                subregions as the subdomains, the subregion Schur
                                complements as A_s and the level-3 DOFs they share in
                                Pi (Section 3.3 applied to the coarse problem); the
                                rows become level-3 DOFs; <= 0: off (default)    */
    int32_t adapt2_max_per_face; /* at most this many rows per level-2 face (10)  */
    int32_t adapt_lobpcg_it; /* > 0: the face pencils (both levels) by LOBPCG for
                                the adapt_max_per_face largest pairs, at most this
                                many iterations (the paper's limit: 15); their Ritz
                                values are lower bounds of the pencil's eigenvalues.
                                0 (default): every pencil solved exactly (dense)  */
} bddc_opts;

/* Fills *o with the defaults: corners+faces, diag weights, float64 local
 * operators (and no other precision), R = 0, B4, freeze 1e-5, ||r||/||b||,
 * previous-solution guess, max_it 1000, save_cap 256, iterations queued
 * kernel by kernel ahead of the convergence poll (use_graph 2), autotuned
 * products, automatic coarse form, no adaptive faces at either level. */
void bddc_default_opts(bddc_opts *o);

/*
 * bddc_setup -- build the preconditioner and every operator of the solve.
 *   mesh, part, opts : host structs (see above).
 *   coef             : host or device, n_elem float64 element coefficients
 *                      c_e > 0 (element matrix c_e * h * Kref, Section 2), or
 *                      their logarithms when opts->coef_log is set.
 *   hip_stream       : hipStream_t (NULL = default stream) used for all work.
 *   out              : receives the new context.
 * Computes, all on the device: local matrices K_i, interior elimination and
 * the interface Schur complements S_i (Section 3.1), the constrained-Neumann
 * operators N_i and coarse bases Phi_i of eq. localCorr, the coarse matrices
 * of eq. coarse_problem and, for three levels, the subregion operators and
 * the dense level-3 inverse.  Errors: EINVAL (sizes, partition values,
 * non-positive coefficients), ESINGULAR (a subdomain without enough
 * constraints), ENOMEM, EHIP.
 */
int bddc_setup(const bddc_mesh *mesh, const bddc_partition *part, const double *coef,
               const bddc_opts *opts, void *hip_stream, bddc_ctx **out);

/*
 * dpcg_solve -- solve K u_k = F_k for k = 0..n_rhs-1 in order.
 *   rhs_seq     : device, n_rhs x n_nodes float64 load vectors F_k (row k contiguous).
 *   rtol        : relative tolerance of the stopping rule (Section 5).
 *   x_seq       : device, n_rhs x n_nodes float64 output u_k.
 *   iters       : host, n_rhs int32 (nullable): PCG iterations of each solve.
 *   true_relres : host, n_rhs float64 (nullable): ||b - A x||/||b|| of the
 *                 interface problem at exit, recomputed in float64.
 * Each solve condenses F_k to the interface, runs Algorithm 1 from the
 * previous solution with the current deflation basis, recovers the interior
 * and, unless the basis is frozen, calls recycle_update.  With n_rhs > 1 the
 * interior products of condensation and recovery run for up to 16 right-hand
 * sides per pass over the interior operators: a group is condensed before its
 * first solve and its interiors recovered after its last (same results; the
 * first such call allocates the group buffers, about 1.8 GB at 192^3, unless
 * an interior is too large for the block product's LDS staging).  On
 * ENOTCONV the outputs of the failing solve hold the last iterate and iters =
 * max_it; later right-hand sides are not solved.
 */
int dpcg_solve(bddc_ctx *ctx, const double *rhs_seq, int32_t n_rhs, double rtol,
               double *x_seq, int32_t *iters, double *true_relres);

/*
 * recycle_update -- rebuild the deflation basis from the last solve
 * (Section 4.2): V = [W, P], small matrices V^T A V and V^T A M^{-1} A V from
 * the solve's own scalars, generalized eigenproblem, keep R vectors (B4:
 * largest harmonic Ritz values), W <- V Y, A W <- [A W, A P] Y, W^T A W by a
 * float64 Gram product, freeze test of eq. harmritzstopcrit.  dpcg_solve
 * calls it after every solve; calling it again without a new solve is a no-op.
 * The new basis is computed over the old one; when its W^T A W is not
 * positive definite the update is refused and the recycled columns are
 * dropped (counted by bddc_solve_info).
 */
int recycle_update(bddc_ctx *ctx);

/* Forget the deflation basis and the previous solution (W = empty, x_prev = 0). */
int bddc_reset_recycle(bddc_ctx *ctx);

/*
 * bddc_adjoint_grad -- gradient of a loss L(u_0..u_{n-1}) given dL/du_k.
 *   dLdu_seq      : device, n_rhs x n_nodes, dL/du_k.
 *   u_seq         : device, n_rhs x n_nodes, the forward solutions u_k.
 *   rtol          : tolerance of the adjoint solves.
 *   grad_logcoef  : device, n_elem float64 output dL/dtheta_e for c_e = exp(theta_e):
 *                   - sum_k c_e h lambda_{k,e}^T Kref u_{k,e}.
 *   grad_rhs_seq  : device, n_rhs x n_nodes output dL/dF_k = lambda_k = K^{-1} dL/du_k.
 * The adjoint systems use the same preconditioner and the current deflation
 * basis without updating it (K is symmetric).
 */
int bddc_adjoint_grad(bddc_ctx *ctx, const double *dLdu_seq, int32_t n_rhs, const double *u_seq,
                      double rtol, double *grad_logcoef, double *grad_rhs_seq);

/*
 * bddc_adjoint_grad_block -- bddc_adjoint_grad with the n_rhs adjoint
 * systems (Appendix-B step 1 of the gradient: same BDDC, same current
 * deflation basis W) solved together as one block: block deflated PCG in the
 * breakdown-free form (an orthonormal search block whose linearly dependent
 * directions are dropped; every direction A-orthogonal to W as in
 * Algorithm 1; x_{-1} = 0), stopping when every column meets the stopping
 * rule of the options (eq. stopping_rhs or stopping_residual) at rtol.  The
 * Schur and Neumann products of a block read each operator tile once per 16
 * columns on the matrix cores.  Not in the paper: an extension for the
 * adjoint right-hand sides, which are all known at once.
 * Arguments as bddc_adjoint_grad; iters: host int32, block iterations
 * (nullable).  Needs n_rhs <= 32, the float64 Neumann operators (local_prec
 * 64 or local_prec_set bit 1), a problem with Dirichlet nodes, and every
 * subdomain interface small enough for the block product's LDS (about 540
 * nodes); otherwise EINVAL.  Errors: ENOTCONV (outputs hold the last
 * iterate), EBREAKDOWN, ENOMEM, EHIP.
 */
int bddc_adjoint_grad_block(bddc_ctx *ctx, const double *dLdu_seq, int32_t n_rhs, const double *u_seq, double rtol,
                            double *grad_logcoef, double *grad_rhs_seq, int32_t *iters);

/* ----- single operator applications on interface vectors (for testing) -----
 * Interface vectors are float64 device arrays of length bddc_info(...)[1] in
 * increasing node order of the interface nodes (free nodes shared by >= 2
 * subdomains). */

/* q = A p, the interface Schur complement product (Section 3.1, eq. Sug). */
int bddc_apply_schur(bddc_ctx *ctx, const double *p, double *q);
/*
 * bddc_apply_schur_noalloc -- q = A p like bddc_apply_schur, for callers that
 * cannot allocate device memory (code under HIP graph capture, tight serving
 * loops, harnesses that forbid hipMalloc): it allocates nothing.  Its
 * partial products live in a static device array of the library (8 MiB,
 * 2^20 doubles, one per GPU, held until the process ends) instead of context
 * memory; a context whose Schur product needs more (the partial products of
 * all its work items, i.e. the sum over subdomains of work items times
 * interface size, plus one double per vector block) is rejected with EINVAL.  Every call on one GPU shares that GPU's array and
 * leaves its contents behind (nothing in it has to start at zero): calls that
 * overlap on one GPU, from any stream or thread, race.  p, q: device, length
 * n_gamma.  Synchronises the context's stream.  Errors: EINVAL, EHIP.
 */
int bddc_apply_schur_noalloc(bddc_ctx *ctx, const double *p, double *q);
/* z = M^{-1} r, one BDDC application (eqs. averaging_subdomain_solves,
 * coarse_problem, localCorr; three levels when subregions were given). */
int bddc_apply_precond(bddc_ctx *ctx, const double *r, double *z);
/* b = F_Gamma - sum_i R_i^T K_BI K_II^{-1} F_I  (Section 3.1), F nodal. */
int bddc_condense(bddc_ctx *ctx, const double *F, double *b);

/*
 * bddc_info -- sizes, host int64 array of at least 16 entries:
 *  [0] n_nodes [1] n_gamma (interface size) [2] n_sub [3] n_coarse (level-1)
 *  [4] corners [5] faces [6] edges [7] level-2 interface [8] level-2 interior
 *  [9] level-3 size [10] deflation columns now [11] frozen (0/1)
 *  [12] bytes of the Schur operators [13] bytes of the Neumann operators
 *  in use [14] max nB [15] device bytes held now
 */
int bddc_info(const bddc_ctx *ctx, int64_t *info);

/*
 * bddc_adaptive_stats -- outcome of the adaptive face selection at setup,
 * host float64 out[4]: faces examined, rows added (coarse DOFs of kind
 * "adaptive"), largest face eigenvalue of eq. eig-matrix before enrichment,
 * seconds spent.  All zero when adapt_tau <= 0.
 */
int bddc_adaptive_stats(const bddc_ctx *ctx, double *out);
/* The same four figures for the level-2 faces (opts->adapt2_tau). */
int bddc_adaptive2_stats(const bddc_ctx *ctx, double *out);

/*
 * bddc_face_constraints -- one face problem of the adaptive selection in the
 * jump space of its m shared nodes (host float64; no device work; exported so
 * the computation can be checked on its own).  Row-major m x m inputs in the
 * order of the shared nodes: Hs, Ht the Schur complements of S_s, S_t onto
 * them, Ks, Kt the blocks S_s, S_t on them; Ds, Dt the interface weights;
 * floating_s/t: subdomain without Dirichlet nodes; B (nb x m) the rows of the
 * coarse DOFs s and t share; fpos (nf) the face's own nodes among the shared
 * ones.  Out: lam (capacity m) the eigenvalues of eq. eig-matrix, descending,
 * and n_lam of them; rows (capacity max_rows x nf) the new rows (orthonormal,
 * against the face average too) of the eigenvalues above tau, n_rows of them.
 * Errors: EINVAL (sizes), ESINGULAR (no Cholesky of H_s + H_t).
 */
int bddc_face_constraints(int32_t m, const double *Hs, const double *Ht, const double *Ks, const double *Kt,
                          const double *Ds, const double *Dt, int32_t floating_s, int32_t floating_t, int32_t nb,
                          const double *B, int32_t nf, const int32_t *fpos, double tau, int32_t max_rows,
                          double *lam, int32_t *n_lam, double *rows, int32_t *n_rows);
/* bddc_face_constraints with the largest max_rows pairs found by LOBPCG (at
 * most max_it >= 1 iterations, starting block of cosines of spread
 * frequencies, Rayleigh-Ritz on [X, R, P] in a B-orthonormalised basis):
 * lam (capacity max(max_rows, 1)) holds its Ritz values, descending; iters
 * (nullable) the iterations taken.  Errors as bddc_face_constraints. */
int bddc_face_constraints_lobpcg(int32_t m, const double *Hs, const double *Ht, const double *Ks, const double *Kt,
                                 const double *Ds, const double *Dt, int32_t floating_s, int32_t floating_t, int32_t nb,
                                 const double *B, int32_t nf, const int32_t *fpos, double tau, int32_t max_rows,
                                 int32_t max_it, double *lam, int32_t *n_lam, double *rows, int32_t *n_rows,
                                 int32_t *iters);

/* Interface node ids (host int64 out[n_gamma]) in interface-vector order. */
int bddc_interface_nodes(const bddc_ctx *ctx, int64_t *out);

/*
 * bddc_stats -- per-kernel device time accumulated with HIP events while
 * enabled (bddc_enable_timing: 0 off, 1 every class, otherwise a bit mask of
 * the classes to time, bit k = class k).  While timing is enabled the
 * iteration is launched kernel by kernel (no graph) so that every launch can
 * be bracketed by events.  out (host float64[3*n]) receives,
 * for kernel class k: total milliseconds, launch count, algorithmic bytes per
 * launch (packed upper triangle of the symmetric operators + coarse bases +
 * gathered input, its index and the output).
 * Classes: 0 Schur product, 1 preconditioner local product, 2 coarse levels,
 * 3 vector updates/reductions, 4 condensation/recovery, 5 recycle.
 */
int bddc_enable_timing(bddc_ctx *ctx, int32_t enable);
int bddc_stats(const bddc_ctx *ctx, double *out, int32_t n);

/*
 * bddc_tuning -- configuration of the two batched operator products (host
 * float64[14]): for the Schur operators then the Neumann operators, kernel
 * blocks, blocks per compute unit requested, work split (1: every block
 * inside one subdomain, 0: equal ranges of the whole tile sequence), waves
 * per block, tiles in flight per wave, fastest tuning launch in
 * microseconds (0 without autotuning), tiles.
 */
int bddc_tuning(const bddc_ctx *ctx, double *out);

/*
 * bddc_time_products -- measurement helper: `reps` back-to-back launches of
 * the batched Schur product and then of the batched Neumann product (the
 * configuration the solve uses, input x = the current interface iterate),
 * timed with HIP events on the context's stream.  out (host float64[4]):
 * Schur microseconds per launch, Schur algorithmic bytes per launch,
 * Neumann microseconds per launch, Neumann algorithmic bytes per launch.
 * Overwrites the products' partial buffers only.  Errors: EINVAL, EHIP.
 */
int bddc_time_products(bddc_ctx *ctx, int32_t reps, double *out);

/*
 * bddc_set_local_prec -- make another storage precision of the
 * constrained-Neumann operators N_i and coarse bases Phi_i the one the
 * preconditioner applies (the float64 and mixed forms of Section 3.2's
 * local solves on one set of operators).  prec: 64, 32 or 16; it must have
 * been built at setup (local_prec or local_prec_set).  The Neumann product is
 * re-tuned when autotune is on; the deflation basis and the previous solution
 * are kept.  Synchronises the stream.  Errors: EINVAL (precision not built).
 */
int bddc_set_local_prec(bddc_ctx *ctx, int32_t prec);

/*
 * bddc_set_launch -- how the following solves launch their work (the
 * batching forms of one set of operators): use_graph as in bddc_opts (2
 * queued ahead of the convergence poll, 1 graph replays, 0 plain: a host
 * check after every iteration); product_cfg (host int32[8], nullable: keep
 * the current ones) as in bddc_opts, except that a product whose first entry
 * is 0 keeps its configuration and one whose first entry is negative takes
 * the untuned default.  Synchronises the stream.
 * Errors: EINVAL (values), ENOMEM.
 */
int bddc_set_launch(bddc_ctx *ctx, int32_t use_graph, const int32_t *product_cfg);

/*
 * bddc_time_kernels -- measurement helper: `reps` back-to-back launches of
 * each of the following, timed with HIP events on the context's stream
 * (inputs: the current interface iterate and residual; only scratch buffers
 * are overwritten).  out (host float64[n], n <= 12) receives pairs
 * (microseconds per launch, algorithmic bytes per launch):
 *   [0,1]  batched Schur product (Section 3.1, A p)
 *   [2,3]  batched constrained-Neumann product (local part of eq. localCorr,
 *          with the coarse restriction (D Phi_i)^T r_i of eq. coarse_problem)
 *   [4,5]  batched interior product K_II^{-1} v (condensation, recovery)
 *   [6,7]  one whole preconditioner application z = M^{-1} r: the Neumann
 *          product, the coarse levels, prolongation and assembly
 *          (eqs. averaging_subdomain_solves, coarse_problem, localCorr)
 *   [8,9]  the coarse levels alone (from the restriction's partials)
 *   [10,11] prolongation and assembly alone
 * Algorithmic bytes are those the method must move (operators in their
 * stored precision, packed; gathered vectors and index lists once).
 * Errors: EINVAL, EHIP.
 */
int bddc_time_kernels(bddc_ctx *ctx, int32_t reps, double *out, int32_t n);

/*
 * bddc_solve_info -- recycling and memory state, host int64 out[n] (n <= 10):
 *  [0] recycling steps run (one per solve until frozen)  [1] of them refused
 *  (the new W^T A W not positive definite: the new basis, computed over the
 *  old one, is dropped and the next update starts from the stored directions)
 *  [2] basis frozen (eq. harmritzstopcrit, 0/1)  [3] the update at which it
 *  froze, counted from 1 like the solves (-1: not frozen)  [4] residual
 *  replacements in the last solve  [5] first search direction of the run the
 *  last update used (those after the last replacement)  [6] deflation
 *  columns  [7] device bytes held now  [8] most device bytes held at once
 *  [9] local precision in use.
 */
int bddc_solve_info(const bddc_ctx *ctx, int64_t *out, int32_t n);

/* Theta (selected harmonic Ritz values, host float64[R]) of the last update. */
int bddc_ritz_values(const bddc_ctx *ctx, double *theta, int32_t cap, int32_t *count);

void bddc_destroy(bddc_ctx *ctx);
const char *bddc_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* BDDC_H */
