// C ABI of the solver: setup, deflated PCG over a right-hand-side sequence,
// Krylov subspace recycling, adjoint gradient (see include/bddc.h).
#include <algorithm>
#include <cmath>
#include <cstddef>
#include <cstdio>
#include <cstring>
#include <map>
#include <numeric>

#include "internal.h"
#include "adaptive.h"
#include "kernels.h"

using namespace bddc;

namespace {

thread_local std::string g_err;

int fail(int code, const std::string &msg) {
    g_err = msg;
    return code;
}

#define HIPCHK(x)                                                                        \
    do {                                                                                 \
        hipError_t e_ = (x);                                                             \
        if (e_ != hipSuccess)                                                            \
            return fail(BDDC_EHIP, std::string(#x) + ": " + hipGetErrorString(e_));     \
    } while (0)

enum { TK_SCHUR = 0, TK_PREC, TK_COARSE, TK_VEC, TK_COND, TK_REC, TK_N };

constexpr int GRAPH_ITERS = 2;     // iterations per queued group (and per captured graph)
constexpr int GRAPH_INFLIGHT = 2;  // groups queued ahead of the convergence poll

// Host view of one batch of operators and its work list.
struct OpHost {
    OpDev dev{};
    int prec = 64;
    SymvCfg cfg{4, 2};
    int bpc = 6;                    // product blocks per compute unit
    bool per_sub = true;            // blocks inside single subdomains (else balanced ranges)
    float tuned_us = 0.f;           // fastest tuning launch
    size_t smem = 0;
    int64_t n_tiles = 0;
    double bytes = 0;               // algorithmic bytes of one product
    bool interior = false;          // interior operators (sizes nI, no gather lists)
    std::vector<int32_t> nchunk;    // per subdomain
    int32_t *d_items = nullptr, *d_nchunk = nullptr, *d_pb = nullptr;
    double *d_ypart = nullptr;
    int64_t ypart_len = 0;          // allocated length of the partial buffer
    int64_t ylen = 0;               // partial entries the current work list writes
    // flat gather list: interface node -> y partials
    int32_t *d_yptr = nullptr, *d_yidx = nullptr;
};

// Pinned host block filled by the per-solve synchronisation.
struct SyncBuf {
    Ctl ctl;
    RecState rs;
    double waw[RMAX * RMAX];
};

// Basis update enqueued but not yet confirmed by the device.
struct Pending {
    bool active = false;
    int k = 0;
    bool freeze = false;
    std::vector<double> GWW, theta;
};

}  // namespace

struct bddc_ctx {
    hipStream_t stream = nullptr;
    hipStream_t cap_stream = nullptr;
    bddc_opts opts{};
    Structure st;
    int prec = 64;
    int n_gamma = 0, n_sub = 0, nC = 0;
    int64_t n_nodes = 0;
    std::map<void *, size_t> allocs; // live device allocations and their sizes
    size_t dev_bytes = 0;           // bytes held now
    size_t dev_peak = 0;            // most bytes held at once
    size_t bytes_S = 0, bytes_N = 0;
    int n_cu = 256;
    bool allow8 = true;             // 8-wave product blocks fit in LDS

    // level 1
    int32_t *d_nB = nullptr, *d_nI = nullptr, *d_b_off = nullptr, *d_i_off = nullptr, *d_nc = nullptr,
            *d_c_off = nullptr, *d_gB = nullptr, *d_nodesI = nullptr, *d_cidx = nullptr, *d_gamma = nullptr,
            *d_pos_sub = nullptr;
    int64_t *d_k_off = nullptr, *d_s_off = nullptr, *d_phr_off = nullptr;
    int32_t *d_pch_sub = nullptr, *d_pch_row = nullptr;   // prolongation blocks: subdomain, first row
    int n_pch = 0;
    double *d_K = nullptr, *d_S = nullptr, *d_KC = nullptr;
    void *d_N = nullptr, *d_phir = nullptr;      // Neumann operators in use (local precision c->prec)
    void *d_Nx[3] = {}, *d_phirx[3] = {};        // the storage precisions built: float64, float32, bfloat16
    int prec_built = 0;                          // bit mask of those: 1 float64, 2 float32, 4 bfloat16
    int32_t *d_asm_ptr = nullptr, *d_asm_idx = nullptr, *d_casm_ptr = nullptr, *d_casm_idx = nullptr;
    double *d_crest = nullptr;                   // coarse restriction partials, one per (subdomain, coarse DOF)
    int max_nI = 0, max_nB = 0, max_nc = 0, max_nt = 0, max_ntI = 0;
    // condensation of up to CBLK right-hand sides per pass over the interior
    // tiles (k_symm): per-column partials, condensed b and ||b||^2 partials
    int cblk_state = 0;             // 0 not set up, 1 ready, -1 unavailable (LDS)
    size_t cblk_smem = 0;
    int64_t cblk_ylen = 0;
    BlockItem *d_cblk_items = nullptr;
    int32_t *d_cblk_ones = nullptr;
    double *d_cblk_y = nullptr, *d_cblk_b = nullptr, *d_cblk_bbp = nullptr;
    double *d_cblk_x = nullptr, *d_cblk_t = nullptr;   // interface solutions, recovery right-hand sides
    std::vector<int32_t> h_nB, h_nI, h_nc, h_b_off, h_c_off, h_pos_sub;
    std::vector<int32_t> h_asm_ptr, h_asm_idx, h_casm_ptr, h_casm_idx;
    OpHost opS, opN, opI;           // Schur, Neumann, interior inverse K_II^{-1}
    int64_t *d_ki_off = nullptr;
    double *d_KI = nullptr;         // packed K_II^{-1} tiles
    int32_t *d_kib_ptr = nullptr, *d_kib_col = nullptr, *d_kbi_ptr = nullptr, *d_kbi_col = nullptr;
    double *d_kib_val = nullptr, *d_kbi_val = nullptr, *d_tmpN = nullptr;
    // iteration vectors
    int vgrid = 1;
    double *d_b = nullptr, *d_x = nullptr, *d_r = nullptr, *d_z = nullptr, *d_p = nullptr, *d_tmp = nullptr;
    double *d_locq = nullptr, *d_wloc = nullptr;
    double *d_rr = nullptr, *d_bbp = nullptr, *d_zp = nullptr, *d_wp = nullptr, *d_dotS = nullptr, *d_gp = nullptr;
    // coarse
    bool three = false;
    double *d_KCinv = nullptr, *d_uC = nullptr;
    int nsr = 0, n3 = 0, max_nL = 0, ld3 = 0;
    int32_t *d_nL = nullptr, *d_nI2 = nullptr, *d_L_off = nullptr, *d_L = nullptr, *d_I2_off = nullptr,
            *d_B2_off = nullptr, *d_g2 = nullptr, *d_asm2_ptr = nullptr, *d_asm2_idx = nullptr,
            *d_pos_sr = nullptr, *d_nc3 = nullptr, *d_C3_off = nullptr, *d_c3 = nullptr,
            *d_asm3_ptr = nullptr, *d_asm3_idx = nullptr;
    uint8_t *d_own2 = nullptr;
    int64_t *d_ph_off2 = nullptr;
    int32_t *d_c3o = nullptr, *d_n3p = nullptr;
    size_t smem_l2d = 0;
    bool coarse_dense = false;      // u_C from one dense product (two levels, or explicit form)
    // dense coarse operator, row-major nC x nC with rows of ldm (even)
    // entries: -K_C^{-1} (two levels) or the explicit level-2 BDDC operator
    double *d_Mc = nullptr, *d_rC = nullptr;
    int64_t ldm = 0;
    int64_t *d_K2_off = nullptr, *d_N2_off = nullptr, *d_P2_off = nullptr;
    // level-3 inverse also as its upper triangle in 64 x 64 blocks (large levels)
    int nb3 = 0;
    double *d_K3s = nullptr, *d_K3part = nullptr;
    int32_t *d_K3bI = nullptr;
    double *d_K2 = nullptr, *d_N2 = nullptr, *d_Phi2 = nullptr, *d_K3inv = nullptr, *d_r3 = nullptr, *d_vI2 = nullptr,
           *d_t2 = nullptr, *d_rB2 = nullptr, *d_u2 = nullptr, *d_c3loc = nullptr, *d_u3 = nullptr;
    // deflation / recycling
    int R = 0, k = 0, save_cap = 0, kmax = 0;
    // pure Neumann problem (no Dirichlet node): column 0 of W is the constant
    // interface vector w0 = 1 / sqrt(n_gamma), with w0 itself as its "A W"
    // column, and the recycled columns follow it
    int nullc = 0;
    int64_t ld = 0;
    double *d_W = nullptr, *d_AW = nullptr, *d_P = nullptr, *d_AP = nullptr;
    double *d_WAWinv = nullptr, *d_Y = nullptr, *d_WAWnew = nullptr, *d_WAWsym = nullptr, *d_invnew = nullptr;
    // re-orthogonalisation: (W^T W)^{-1} of the basis in use and of the new one,
    // W^T r partials, a scratch state for the Cholesky of W^T W
    double *d_WWinv = nullptr, *d_WWnew = nullptr, *d_WWsym = nullptr, *d_WWinvnew = nullptr, *d_rop = nullptr;
    RecState *d_state2 = nullptr;
    RecState *d_state = nullptr;
    std::vector<double> WAW, GWW, theta;
    bool frozen = false;
    int freeze_step = -1, n_updates = 0, update_refused = 0, gram_nb = 1;
    Pending pend;
    // histories of the last solve
    int hist_cap = 0;
    double *d_ahist = nullptr, *d_dhist = nullptr, *d_rhohist = nullptr, *d_bhist = nullptr, *d_muhist = nullptr,
           *d_reshist = nullptr;
    // control
    Ctl *d_ctl = nullptr, *h_ctl = nullptr;
    SyncBuf *h_sync = nullptr;      // pinned
    double *h_hist = nullptr;       // pinned: alpha, d, rho (hist_cap each), mu (hist_cap x RMAX)
    SyncBuf *d_sync = nullptr;      // device image of SyncBuf (holds d_ctl, d_state, d_WAWsym)
    bool pre_schur = false;         // A x of the next solve's initial residual already enqueued
    AdaptStats adapt;               // adaptive face selection at setup
    AdaptStats adapt2;              // the same at level 2
    double *d_hblk = nullptr;       // device image of h_hist (holds the four histories)
    double *h_Y = nullptr;          // pinned staging of the recycling coefficients
    int hcopy = 0;
    int32_t *h_flags = nullptr;     // pinned, device-mapped: [0] convergence word
    int32_t *d_hflag = nullptr;     // device address of h_flags[0]
    double *h_prog = nullptr;       // pinned, device-mapped: last ||r||^2, its denominator, iteration
    double *d_hprog = nullptr;      // device address of h_prog
    double rtol2_run = 0.0;         // squared tolerance of the running solve
    int32_t *d_status = nullptr;
    bool have_solve = false, have_hist = false;
    int last_iters = 0, last_restarts = 0, last_status = 0;
    int seg_start = 0;              // first direction after the last residual replacement
    // graph of GRAPH_ITERS iterations (use_graph 1)
    hipGraph_t graph = nullptr;
    hipGraphExec_t gexec = nullptr;
    hipEvent_t gev[GRAPH_INFLIGHT + 1] = {};
    hipEvent_t sync_ev = nullptr;   // recorded after the copies of a solve's synchronisation
    // element data for the adjoint gradient
    double *d_coefh = nullptr;
    uint8_t *d_keep = nullptr, *d_free = nullptr;
    // timing
    bool timing = false;
    int timing_mask = 0;
    std::vector<std::pair<int, std::pair<hipEvent_t, hipEvent_t>>> pending;
    std::vector<hipEvent_t> ev_pool;
    double t_ms[TK_N] = {0}, t_cnt[TK_N] = {0}, t_bytes[TK_N] = {0};
};

namespace {

template <typename T>
int dalloc(bddc_ctx *c, T **p, size_t count) {
    *p = nullptr;
    if (count == 0) count = 1;
    void *q = nullptr;
    hipError_t e = hipMalloc(&q, count * sizeof(T));
    if (e != hipSuccess) return fail(BDDC_ENOMEM, "hipMalloc of " + std::to_string(count * sizeof(T)) + " bytes failed");
    c->allocs[q] = count * sizeof(T);
    c->dev_bytes += count * sizeof(T);
    c->dev_peak = std::max(c->dev_peak, c->dev_bytes);
    *p = (T *)q;
    return 0;
}

// A packed tile array of `count` elements followed by TILE_TAIL_BYTES zeroed
// bytes.
template <typename T>
int dalloc_tiles(bddc_ctx *c, T **p, size_t count) {
    const size_t tail = (TILE_TAIL_BYTES + sizeof(T) - 1) / sizeof(T);
    int rc = dalloc(c, p, count + tail);
    if (rc) return rc;
    if (hipMemset(*p + count, 0, tail * sizeof(T)) != hipSuccess) return fail(BDDC_EHIP, "hipMemset failed");
    return 0;
}

template <typename T>
int dupload(bddc_ctx *c, T **p, const std::vector<T> &v) {
    int rc = dalloc(c, p, v.size());
    if (rc) return rc;
    if (!v.empty()) HIPCHK(hipMemcpyAsync(*p, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice, c->stream));
    return 0;
}

void dfree(bddc_ctx *c, void *p) {
    if (!p) return;
    auto it = c->allocs.find(p);
    if (it != c->allocs.end()) {
        c->dev_bytes -= it->second;
        c->allocs.erase(it);
    }
    (void)hipFree(p);
}

// Batched symmetric sweeps (sweep.hip) of the matrices `h` (device copies of
// the descriptors and the panel buffer are made here and freed after the
// stream has finished them).
int run_sweeps(bddc_ctx *c, const std::vector<SweepDesc> &h) {
    if (h.empty()) return 0;
    std::vector<int64_t> off;
    const int64_t nbuf = sweep_panel_doubles(h, off);
    SweepDesc *dd = nullptr;
    int64_t *doff = nullptr;
    double *buf = nullptr;
    int rc;
    if ((rc = dupload(c, &dd, h)) || (rc = dupload(c, &doff, off)) || (rc = dalloc(c, &buf, (size_t)nbuf))) return rc;
    launch_sweep_blocked(dd, doff, h, buf, c->d_status, c->stream);
    HIPCHK(hipStreamSynchronize(c->stream));
    dfree(c, dd); dfree(c, doff); dfree(c, buf);
    return 0;
}

// CSR from (target, source) pairs; stable in insertion order
void build_csr(int64_t ntarget, const std::vector<std::pair<int64_t, int32_t>> &pairs, std::vector<int32_t> &ptr,
               std::vector<int32_t> &idx) {
    ptr.assign(ntarget + 1, 0);
    for (auto &p : pairs) ptr[p.first + 1]++;
    for (int64_t t = 0; t < ntarget; ++t) ptr[t + 1] += ptr[t];
    idx.resize(pairs.size());
    std::vector<int32_t> fill(ptr.begin(), ptr.end() - 1);
    for (auto &p : pairs) idx[fill[p.first]++] = p.second;
}


// slot of a storage precision in d_Nx / d_phirx (-1: not a storage precision)
int prec_slot(int prec) { return prec == 64 ? 0 : prec == 32 ? 1 : prec == 16 ? 2 : -1; }

// Algorithmic bytes of one batched product (Schur or Neumann, prec = the
// operator's storage precision): packed upper triangle, gathered input and
// its index, output; with `coarse` (Neumann with a coarse space) also D Phi_i
// and the coarse partials of the restriction.
double product_bytes(const bddc_ctx *c, int prec, bool coarse) {
    const double eb = prec / 8.0;
    double bytes = 0.0;
    for (int i = 0; i < c->n_sub; ++i) {
        const double n = c->h_nB[i], nci = coarse ? c->h_nc[i] : 0;
        bytes += (n * (n + 1) / 2 + n * nci) * eb + n * (8 + 4 + 8) + nci * 8;
    }
    return bytes;
}

// Algorithmic bytes of the coarse levels of one preconditioner application:
// the gather of r_C from the coarse partials, and the dense coarse operator; or, for the subregion
// chain, the level-2 blocks each phase reads (interior columns of the swept
// subregion matrix, N and Phi of the level-2 interface, Phi again and the
// interior-interface block for the correction), the level-3 inverse and the
// coarse vectors.
double coarse_bytes(const bddc_ctx *c) {
    if (c->nC == 0) return 0.0;
    double cp = 0.0;   // coarse partials gathered into r_C: index + value
    for (int i = 0; i < c->n_sub; ++i) cp += c->h_nc[i] * 12.0;
    const double vec = c->nC * (4.0 + 8.0 + 8.0);
    if (c->coarse_dense) return (double)c->nC * c->ldm * 8.0 + cp + vec + c->nC * 8.0;
    const double n3 = c->n3;
    double b = cp + vec + (c->d_K3s ? n3 * (n3 + 1) / 2 * 8.0 : n3 * c->ld3 * 8.0);
    for (const SubregionHost &r : c->st.sr) {
        const double nL = (double)r.L.size(), nI = r.nI, nB = r.nB, n3 = (double)r.c3.size();
        b += (nL * nI + nB * nB + nB * n3 + nB * n3 + nI * nB) * 8.0 + nL * (4.0 + 8.0);
    }
    return b;
}

// Algorithmic bytes of the prolongation and the assembly of z = M^{-1} r:
// Neumann partials, D Phi_i rows, gathered u_C entries, the local w_i written
// and read back, the assembly lists and z.
double prolong_bytes(const bddc_ctx *c) {
    const double eN = c->prec / 8.0;
    double b = 0.0;
    for (int i = 0; i < c->n_sub; ++i) {
        const double n = c->h_nB[i], nci = c->nC > 0 ? c->h_nc[i] : 0;
        b += c->opN.nchunk[i] * n * 8.0 + n * nci * eN + nci * 12.0 + n * 8.0;   // k_prolong
        b += n * (4.0 + 8.0);                                                   // assembly entries
    }
    return b + (c->n_gamma + 1) * 4.0 + c->n_gamma * 8.0;
}

// -------------------------------------------------------------------- timing
hipEvent_t get_event(bddc_ctx *c) {
    if (!c->ev_pool.empty()) {
        hipEvent_t e = c->ev_pool.back();
        c->ev_pool.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    (void)hipEventCreate(&e);
    return e;
}
struct TScope {
    bddc_ctx *c;
    int k;
    hipEvent_t a = nullptr;
    bool on;
    TScope(bddc_ctx *c_, int k_) : c(c_), k(k_), on(c_->timing && ((c_->timing_mask >> k_) & 1)) {
        if (on) { a = get_event(c); (void)hipEventRecord(a, c->stream); }
    }
    ~TScope() {
        if (on) {
            hipEvent_t b = get_event(c);
            (void)hipEventRecord(b, c->stream);
            c->pending.push_back({k, {a, b}});
        }
    }
};
void flush_timing(bddc_ctx *c) {
    for (auto &p : c->pending) {
        float ms = 0;
        (void)hipEventElapsedTime(&ms, p.second.first, p.second.second);
        c->t_ms[p.first] += ms;
        c->t_cnt[p.first] += 1;
        c->ev_pool.push_back(p.second.first);
        c->ev_pool.push_back(p.second.second);
    }
    c->pending.clear();
}

// ------------------------------------------------------------- work lists
// Split the work of a batched product over `nblocks` blocks and lay out the
// partial buffers (one partial vector per segment).  Work is counted in the
// operators' 256-entry slots (tiles, then the strip of the ragged tail rows).
// Balanced: the concatenated slot sequence of all subdomains is cut into nblocks equal
// ranges, each range into segments inside single subdomains (a block may
// span subdomains).  Per subdomain: every subdomain is cut into about
// tiles / (total / nblocks) equal segments, one block each (a block never
// spans subdomains; the block count follows the rounding).
int build_worklist(bddc_ctx *c, OpHost &op, int nblocks, bool per_sub) {
    const int nsub = c->n_sub;
    struct Seg { int k; int64_t t0, t1; int32_t c; };
    std::vector<std::vector<Seg>> blk;   // segments of every block, in order
    std::vector<int32_t> nch(nsub, 0), pb(nsub), xoff(nsub + 1, 0);
    int64_t ylen = 0;
    const std::vector<int32_t> &sizes = op.interior ? c->h_nI : c->h_nB;
    std::vector<int64_t> start(nsub + 1, 0);
    for (int i = 0; i < nsub; ++i) {
        start[i + 1] = start[i] + op_slots(sizes[i]);
        xoff[i + 1] = xoff[i] + sizes[i];
    }
    const int64_t total = start[nsub];
    if (total > INT32_MAX) return fail(BDDC_EINVAL, "operator tile count exceeds int32 indexing");
    if (per_sub) {
        const int64_t target = std::max<int64_t>(1, (total + nblocks - 1) / nblocks);
        for (int k = 0; k < nsub; ++k) {
            const int64_t nt = start[k + 1] - start[k];
            if (nt == 0) continue;
            const int C = (int)std::min<int64_t>(nt, std::max<int64_t>(1, (nt + target / 2) / target));
            for (int q = 0; q < C; ++q) blk.push_back({Seg{k, nt * q / C, nt * (q + 1) / C, nch[k]++}});
        }
        nblocks = (int)blk.size();
        // longest items first: the blocks that start after the first round
        // are the short ones, which fill the compute units left idle early
        std::stable_sort(blk.begin(), blk.end(), [](const std::vector<Seg> &x, const std::vector<Seg> &y) {
            return x[0].t1 - x[0].t0 > y[0].t1 - y[0].t0;
        });
        // XCD-aware order: consecutive blocks go to the 8 XCDs in turn, each
        // with its own L2.  Subdomain indices, like the interface numbering,
        // run through the domain in slabs, so inside every run of equal
        // length block p takes a subdomain of slab p mod 8 where one is left:
        // each XCD then gathers its inputs from about an eighth of the
        // interface vector.  (The results do not depend on the order.)
        constexpr int NX = 8;
        for (size_t r0 = 0; r0 < blk.size();) {
            const int64_t len = blk[r0][0].t1 - blk[r0][0].t0;
            size_t r1 = r0;
            while (r1 < blk.size() && blk[r1][0].t1 - blk[r1][0].t0 == len) ++r1;
            std::vector<std::vector<std::vector<Seg>>> slab(NX);
            for (size_t p = r0; p < r1; ++p) slab[(int64_t)blk[p][0].k * NX / nsub].push_back(blk[p]);
            std::vector<size_t> next(NX, 0);
            for (size_t p = r0; p < r1; ++p) {
                int g = (int)(p % NX);
                while (next[g] == slab[g].size()) g = (g + 1) % NX;   // (some slab has one left)
                blk[p] = slab[g][next[g]++];
            }
            r0 = r1;
        }
    } else {
        blk.resize(nblocks);
        int i = 0;
        for (int b = 0; b < nblocks; ++b) {
            const int64_t g0 = total * b / nblocks, g1 = total * (b + 1) / nblocks;
            while (i < nsub && start[i + 1] <= g0) ++i;
            for (int k = i; k < nsub && start[k] < g1; ++k) {
                const int64_t t0 = std::max(g0, start[k]) - start[k], t1 = std::min(g1, start[k + 1]) - start[k];
                if (t1 > t0) blk[b].push_back(Seg{k, t0, t1, nch[k]++});
            }
        }
    }
    for (int k = 0; k < nsub; ++k) {
        pb[k] = (int32_t)ylen;
        ylen += (int64_t)nch[k] * sizes[k];
    }
    if (ylen > INT32_MAX) return fail(BDDC_EINVAL, "operator partial buffers exceed int32 indexing");
    // block b's first segment at index b, its others appended and chained
    std::vector<SymvItem> items(std::max(nblocks, 1), SymvItem{0, 0, 0, 0, 0, 0, -1, 0, 0, 0, 0, 0});
    auto record = [&](const Seg &g) {
        const int n = sizes[g.k];
        return SymvItem{(int32_t)start[g.k], (int32_t)g.t0, (int32_t)g.t1, n, xoff[g.k], pb[g.k] + g.c * n, -1,
                        tile_rows(n), full_tiles(n), uses_strip(n) ? 1 : 0, g.k, g.c};
    };
    for (int b = 0; b < nblocks; ++b) {
        int prev = b;
        for (size_t q = 0; q < blk[b].size(); ++q) {
            if (q == 0) {
                items[b] = record(blk[b][0]);
            } else {
                items[prev].next = (int32_t)items.size();
                prev = (int)items.size();
                items.push_back(record(blk[b][q]));
            }
        }
    }
    dfree(c, op.d_items); dfree(c, op.d_nchunk); dfree(c, op.d_pb);
    std::vector<int32_t> raw(items.size() * (sizeof(SymvItem) / 4));
    std::memcpy(raw.data(), items.data(), items.size() * sizeof(SymvItem));
    int rc;
    if ((rc = dupload(c, &op.d_items, raw)) || (rc = dupload(c, &op.d_nchunk, nch)) || (rc = dupload(c, &op.d_pb, pb)))
        return rc;
    if (ylen > op.ypart_len) {
        dfree(c, op.d_ypart);
        if ((rc = dalloc(c, &op.d_ypart, (size_t)ylen))) return rc;
        op.ypart_len = ylen;
    }
    op.nchunk = nch;
    op.ylen = ylen;
    op.dev.items = reinterpret_cast<const SymvItem *>(op.d_items);
    op.dev.n_blocks = total > 0 ? nblocks : 0;
    op.dev.nchunk = op.d_nchunk;
    op.dev.pb = op.d_pb;
    if (op.interior) return 0;      // interior entries have one owner: no lists
    // flat gather lists, owners in assembly order, items in increasing order
    {
        std::vector<int32_t> ptr(c->n_gamma + 1, 0), idx;
        idx.reserve(ylen);
        for (int g = 0; g < c->n_gamma; ++g) {
            for (int e = c->h_asm_ptr[g]; e < c->h_asm_ptr[g + 1]; ++e) {
                const int pos = c->h_asm_idx[e];
                const int i = c->h_pos_sub[pos];
                const int k = pos - c->h_b_off[i];
                for (int q = 0; q < nch[i]; ++q) idx.push_back(pb[i] + q * c->h_nB[i] + k);
            }
            ptr[g + 1] = (int32_t)idx.size();
        }
        dfree(c, op.d_yptr); dfree(c, op.d_yidx);
        if ((rc = dupload(c, &op.d_yptr, ptr)) || (rc = dupload(c, &op.d_yidx, idx))) return rc;
    }
    return 0;
}

// ------------------------------------------------------------- sub-steps
int sync_ctl(bddc_ctx *c) {
    HIPCHK(hipMemcpyAsync(c->h_ctl, c->d_ctl, sizeof(Ctl), hipMemcpyDeviceToHost, c->stream));
    HIPCHK(hipStreamSynchronize(c->stream));
    return 0;
}

Gather gather_of(const OpHost &op) { return Gather{op.d_yptr, op.d_yidx, op.d_ypart}; }

// Schur products y_i = S_i x_i of every subdomain (partials in opS); with
// `dot`, per-item x_i^T y_i partials for p^T A p.
void run_schur(bddc_ctx *c, const double *x, bool gated, bool dot) {
    TScope ts(c, TK_SCHUR);
    SymvArgs a{};
    a.op = c->opS.dev;
    a.x = x;
    a.ypart = c->opS.d_ypart;
    a.dot = dot ? c->d_dotS : nullptr;
    a.ctl = c->d_ctl;
    a.gated = gated ? 1 : 0;
    launch_symv(a, SYMV_SCHUR, 64, c->opS.cfg, c->opS.smem, c->stream);
}

// Arguments of the level-2/3 kernels with the level-1 coarse residual taken
// from `rc`.
L2Args l2_args(const bddc_ctx *c, const Gather &rc) {
    L2Args l{};
    l.ctl = c->d_ctl;
    l.rc = rc;
    l.nL = c->d_nL; l.nI2 = c->d_nI2; l.L_off = c->d_L_off; l.L = c->d_L; l.I2_off = c->d_I2_off;
    l.B2_off = c->d_B2_off; l.g2 = c->d_g2;
    l.K2_off = c->d_K2_off; l.K2 = c->d_K2; l.vI2 = c->d_vI2; l.t2 = c->d_t2; l.rB2 = c->d_rB2;
    l.asm2_ptr = c->d_asm2_ptr; l.asm2_idx = c->d_asm2_idx; l.N2_off = c->d_N2_off; l.N2 = c->d_N2;
    l.P2_off = c->d_P2_off; l.Phi2 = c->d_Phi2; l.nc3 = c->d_nc3; l.C3_off = c->d_C3_off; l.c3 = c->d_c3;
    l.u2 = c->d_u2; l.c3loc = c->d_c3loc; l.pos_sr = c->d_pos_sr; l.own2 = c->d_own2; l.u3 = c->d_u3;
    l.uC = c->d_uC;
    l.ph_off = c->d_ph_off2; l.c3o = c->d_c3o; l.n3p = c->d_n3p; l.n3 = c->n3; l.max_nL = c->max_nL;
    return l;
}

// Level-2 BDDC applied to the level-1 coarse residual (Section 3.2,
// multilevel paragraph): subregion pre-solves, level-2 interface residual
// and local solves, level-3 coarse solve, level-2 correction into u_C.
void run_l2_chain(const bddc_ctx *c, const L2Args &l, hipStream_t st) {
    launch_l2_a(l, c->nsr, c->max_nL, st);
    launch_l2_b(l, c->nsr, c->max_nL, st);
    // level 3: r3 = sum of the subregion contributions, u3 = K3^{-1} r3 with
    // the inverse's upper triangle in blocks, or the dense inverse (stored
    // negated, rows padded to ld3)
    CoarseDenseArgs l3{};
    l3.ctl = c->d_ctl; l3.n = c->n3; l3.rc = Gather{c->d_asm3_ptr, c->d_asm3_idx, c->d_c3loc}; l3.r = c->d_r3;
    l3.M = c->d_K3inv; l3.ldm = c->ld3; l3.sign = -1.0; l3.u = c->d_u3;
    if (c->d_K3s) {
        SymBlkArgs sb{};
        sb.ctl = c->d_ctl; sb.n = c->n3; sb.nb = c->nb3; sb.B = c->d_K3s; sb.bI = c->d_K3bI; sb.r = c->d_r3;
        sb.part = c->d_K3part; sb.u = c->d_u3;
        launch_coarse_symblk(l3, sb, st);
    } else {
        launch_coarse_dense(l3, st);
    }
    launch_l2_d(l, c->nsr, c->smem_l2d, st);
}

void run_coarse(bddc_ctx *c, hipStream_t st);
void run_prolong_assemble(bddc_ctx *c, const double *r, double *z, bool gated, bool advance, bool reduce);

// Coarse restriction of a single-vector Neumann product: the first segment
// of every subdomain writes c_i = (D Phi_i)^T x_i (none without a coarse space).
void set_restriction(const bddc_ctx *c, SymvArgs &a) {
    if (c->nC == 0) return;
    a.cpart = c->d_crest;
    a.phir = c->d_phir; a.phr_off = c->d_phr_off;
    a.nc = c->d_nc; a.c_off = c->d_c_off;
}

// One BDDC application on r: local constrained-Neumann products, the coarse
// levels, assembly of z with the coarse prolongation and the (r^T z,
// (AW)^T z) partials.  test: stopping test at the start (0 none, 1 in the
// loop, 2 first test of a solve).
void run_precond(bddc_ctx *c, const double *r, double *z, int test, bool gated, bool advance, bool reduce) {
    {
        TScope ts(c, TK_PREC);
        SymvArgs a{};
        a.op = c->opN.dev;
        a.x = r;
        a.ypart = c->opN.d_ypart;
        a.ctl = c->d_ctl;
        a.gated = gated ? 1 : 0;
        a.test = test;
        a.defer = test ? 1 : 0;          // k_pupd tests instead while the basis records
        a.stop_rule = c->opts.stop_rule;
        a.max_it = c->opts.max_it;
        a.rr_part = c->d_rr; a.rr_n = c->vgrid;
        a.bb_part = c->d_bbp; a.bb_n = c->vgrid;
        a.res_hist = c->d_reshist; a.hist_cap = c->hist_cap;
        set_restriction(c, a);
        launch_symv(a, SYMV_NEUMANN, c->prec, c->opN.cfg, c->opN.smem, c->stream);
    }
    run_coarse(c, c->stream);
    run_prolong_assemble(c, r, z, gated, advance, reduce);
}

// Coarse levels of one BDDC application on stream st: the coarse residual
// r_C = sum_i R_Ci^T c_i from the partials of the Neumann product, then u_C
// (eq. coarse_problem; three levels as in Section 3.2).
void run_coarse(bddc_ctx *c, hipStream_t st) {
    if (c->nC == 0) return;
    TScope ts(c, TK_COARSE);
    const Gather rc{c->d_casm_ptr, c->d_casm_idx, c->d_crest};
    if (c->coarse_dense) {
        CoarseDenseArgs ca{};
        ca.ctl = c->d_ctl; ca.n = c->nC; ca.rc = rc; ca.r = c->d_rC;
        ca.M = c->d_Mc; ca.ldm = c->ldm;
        ca.sign = c->three ? 1.0 : -1.0;
        ca.u = c->d_uC;
        launch_coarse_dense(ca, st);
    } else {
        run_l2_chain(c, l2_args(c, rc), st);
    }
}

// Prolongation w_i = u_i + D Phi_i u_C and assembly z = sum_i R_i^T w_i
// (eq. averaging_subdomain_solves), with the (r^T z, (AW)^T z) partials when
// `reduce` is set.
void run_prolong_assemble(bddc_ctx *c, const double *r, double *z, bool gated, bool advance, bool reduce) {
    {
        TScope ts(c, TK_VEC);
        ProlArgs pa{};
        pa.ctl = c->d_ctl; pa.gated = gated ? 1 : 0;
        pa.nB = c->d_nB; pa.b_off = c->d_b_off; pa.nc = c->d_nc; pa.c_off = c->d_c_off; pa.cidx = c->d_cidx;
        pa.nchunk = c->opN.d_nchunk; pa.pb = c->opN.d_pb; pa.upart = c->opN.d_ypart;
        pa.phir = c->d_phir; pa.phr_off = c->d_phr_off;
        pa.uC = c->nC > 0 ? c->d_uC : nullptr;
        pa.wloc = c->d_wloc;
        pa.ch_sub = c->d_pch_sub; pa.ch_row = c->d_pch_row;
        launch_prolong(pa, c->prec, c->n_pch, c->max_nc, c->stream);
        ZasmArgs a{};
        a.n = c->n_gamma;
        a.w.ptr = c->d_asm_ptr; a.w.idx = c->d_asm_idx; a.w.part = c->d_wloc;
        a.r = r; a.z = z;
        a.AW = c->d_AW; a.ld = c->ld;
        a.part = reduce ? c->d_zp : nullptr;
        a.ctl = c->d_ctl;
        a.gated = gated ? 1 : 0;
        a.advance = advance ? 1 : 0;
        launch_zasm(a, c->kmax, c->vgrid, c->stream);
    }
}

void run_pupd(bddc_ctx *c, bool first, bool hist_only, bool gated, int test) {
    TScope ts(c, TK_VEC);
    PupdArgs a{};
    a.n = c->n_gamma; a.z = c->d_z; a.p = c->d_p; a.W = c->d_W; a.ld = c->ld;
    a.P = c->d_P; a.cap = c->save_cap;
    a.zpart = c->d_zp; a.zpart_n = c->vgrid;
    a.WAWinv = c->d_WAWinv;
    a.ctl = c->d_ctl;
    a.first = first ? 1 : 0; a.hist_only = hist_only ? 1 : 0; a.gated = gated ? 1 : 0;
    a.rho_hist = c->d_rhohist; a.b_hist = c->d_bhist; a.mu_hist = c->d_muhist; a.hist_cap = c->hist_cap;
    a.test = test; a.stop_rule = c->opts.stop_rule; a.max_it = c->opts.max_it;
    a.rr_part = c->d_rr; a.rr_n = c->vgrid; a.bb_part = c->d_bbp; a.bb_n = c->vgrid;
    a.res_hist = c->d_reshist;
    launch_pupd(a, c->kmax, c->vgrid, c->stream);
}

// Alg. 1, optional re-orthogonalisation of the updated residual.
void run_reorth(bddc_ctx *c) {
    TScope ts(c, TK_VEC);
    ReorthArgs a{};
    a.n = c->n_gamma; a.r = c->d_r; a.W = c->d_W; a.ld = c->ld; a.WWinv = c->d_WWinv;
    a.part = c->d_rop; a.rr_part = c->d_rr; a.ctl = c->d_ctl;
    launch_reorth(a, c->kmax, c->vgrid, c->stream);
}

void run_update(bddc_ctx *c) {
    TScope ts(c, TK_VEC);
    UpdArgs a{};
    a.n = c->n_gamma;
    a.q = gather_of(c->opS);
    a.p = c->d_p; a.x = c->d_x; a.r = c->d_r;
    a.AP = c->d_AP; a.ld = c->ld; a.cap = c->save_cap;
    a.dot = c->d_dotS; a.dot_n = c->opS.dev.n_blocks;
    a.rr_part = c->d_rr;
    a.ctl = c->d_ctl;
    a.d_hist = c->d_dhist; a.a_hist = c->d_ahist; a.rho_hist = c->d_rhohist; a.hist_cap = c->hist_cap;
    launch_update(a, c->vgrid, c->stream);
}

// out = b - (sum of the Schur partials); per-block ||out||^2 into d_rr and,
// with want_wtr, (||out||^2, W^T out) into d_wp.
void run_resid(bddc_ctx *c, double *out, bool want_wtr) {
    TScope ts(c, TK_VEC);
    ResidArgs a{};
    a.n = c->n_gamma; a.want_wtr = want_wtr ? 1 : 0;
    a.q = gather_of(c->opS);
    a.b = c->d_b; a.out = out;
    a.W = c->d_W; a.ld = c->ld;
    a.ctl = c->d_ctl;
    a.part = c->d_wp;
    launch_resid(a, want_wtr ? c->kmax : 0, c->vgrid, c->stream);
}

// One iteration of Algorithm 1 (lines 9-16), every kernel gated by ctl->done.
void enqueue_iteration(bddc_ctx *c) {
    run_schur(c, c->d_p, true, true);                    // line 9: A p_j, p_j^T A p_j
    run_update(c);                                       // lines 9-11
    if (c->opts.reorth && c->R + c->nullc > 0) run_reorth(c);   // optional line
    run_precond(c, c->d_r, c->d_z, 1, true, true, true); // stopping test, line 13
    run_pupd(c, false, false, true, 1);                  // lines 14-16 (the test while recording)
}

int capture_graph(bddc_ctx *c) {
    if (c->gexec) return 0;
    hipStream_t keep = c->stream;
    const bool tkeep = c->timing;
    c->timing = false;
    c->stream = c->cap_stream;
    hipError_t e = hipStreamBeginCapture(c->stream, hipStreamCaptureModeRelaxed);
    if (e == hipSuccess) {
        for (int it = 0; it < GRAPH_ITERS; ++it) enqueue_iteration(c);
        e = hipStreamEndCapture(c->stream, &c->graph);
    }
    c->stream = keep;
    c->timing = tkeep;
    if (e != hipSuccess) return fail(BDDC_EHIP, std::string("graph capture: ") + hipGetErrorString(e));
    HIPCHK(hipGraphInstantiate(&c->gexec, c->graph, nullptr, nullptr, 0));
    return 0;
}

// Iterate until ctl->done: groups of GRAPH_ITERS iterations, GRAPH_INFLIGHT
// groups queued ahead of the convergence check, which reads the pinned word
// the kernels set together with ctl->done; a group is either launched kernel
// by kernel into the stream (use_graph 2, the default) or one replay of the
// captured graph (use_graph 1: each replay starts 10-14 us after the previous
// one ends on this stack, against none between directly queued kernels).
// use_graph 0 (plain form): one iteration at a time with a host check after
// each.
int run_loop(bddc_ctx *c) {
    const int max_launch = c->opts.max_it + 2;
    if (c->opts.use_graph && !c->timing) {
        const bool graph = c->opts.use_graph == 1;
        if (graph) {
            int rc = capture_graph(c);
            if (rc) return rc;
        }
        volatile int32_t *flag = c->h_flags;
        volatile const double *prog = c->h_prog;
        int launched = 0, polled = 0;
        const int cap = max_launch / GRAPH_ITERS + GRAPH_INFLIGHT + 1;
        double last_rr = -1.0, last_it = -1.0, rate = 0.0;
        auto wait_one = [&]() -> int {
            const int ps = polled % (GRAPH_INFLIGHT + 1);
            HIPCHK(hipEventSynchronize(c->gev[ps]));
            ++polled;
            return 0;
        };
        while (true) {
            const int slot = launched % (GRAPH_INFLIGHT + 1);
            if (graph) HIPCHK(hipGraphLaunch(c->gexec, c->stream));
            else
                for (int it = 0; it < GRAPH_ITERS; ++it) enqueue_iteration(c);
            HIPCHK(hipEventRecord(c->gev[slot], c->stream));
            ++launched;
            if (launched - polled >= GRAPH_INFLIGHT || launched >= cap) {
                if (int rc = wait_one()) return rc;
                if (*flag) break;
                if (launched >= cap) break;   // every kernel stops at max_it by itself
                // The residual after the polled group and its decay per
                // iteration predict whether the groups still queued reach the
                // tolerance; if so, wait for them before queuing another (a
                // group queued past convergence costs its launches for nothing).
                const double rr = prog[0], den = prog[1], it = prog[2];
                if (last_it >= 0.0 && it > last_it && rr > 0.0 && last_rr > 0.0 && rr < last_rr)
                    rate = std::pow(rr / last_rr, 1.0 / (it - last_it));
                last_rr = rr;
                last_it = it;
                if (rate > 0.0 && rate < 1.0 && rr > 0.0 && den > 0.0) {
                    const double need = std::log(c->rtol2_run * den / rr) / std::log(rate);
                    if (need <= (double)(launched - polled) * GRAPH_ITERS) {
                        while (polled < launched && !*flag)
                            if (int rc = wait_one()) return rc;
                        if (*flag) break;
                    }
                }
            }
        }
        return 0;
    }
    for (int it = 0; it < max_launch; ++it) {
        enqueue_iteration(c);
        int rc = sync_ctl(c);
        if (rc) return rc;
        if (c->h_ctl->done) break;
    }
    return 0;
}

// y_I = K_II^{-1} v_I for every subdomain, v gathered from the nodal vector
// at the interior nodes (partial products in opI)
void run_interior(bddc_ctx *c, const double *v) {
    SymvArgs a{};
    a.op = c->opI.dev;
    a.x = v;
    a.ypart = c->opI.d_ypart;
    a.ctl = c->d_ctl;
    launch_symv(a, SYMV_INTERIOR, 64, c->opI.cfg, c->opI.smem, c->stream);
}

// Condensation (Section 3.1): y_I = K_II^{-1} F_I, t_i = K_BI y_I,
// b = F_G - sum_i R_i^T t_i, per-block ||b||^2 partials.
void run_condense(bddc_ctx *c, const double *F) {
    TScope ts(c, TK_COND);
    run_interior(c, F);
    CondArgs a{};
    a.nI = c->d_nI; a.nB = c->d_nB; a.i_off = c->d_i_off; a.b_off = c->d_b_off;
    a.nchunk = c->opI.d_nchunk; a.pb = c->opI.d_pb; a.ypart = c->opI.d_ypart;
    a.kbi_ptr = c->d_kbi_ptr; a.kbi_col = c->d_kbi_col; a.kbi_val = c->d_kbi_val; a.t = c->d_locq;
    launch_cond_local(a, c->n_sub, c->max_nI, c->stream);
    CondAsmArgs b{};
    b.n = c->n_gamma; b.gamma = c->d_gamma; b.ptr = c->d_asm_ptr; b.idx = c->d_asm_idx; b.F = F; b.loc = c->d_locq;
    b.b = c->d_b; b.part = c->d_bbp;
    launch_cond_asm(b, c->vgrid, c->stream);
}

constexpr int CBLK = 16;            // right-hand sides condensed per pass over the interior tiles

// The buffers of the block condensation, allocated on first use; unavailable
// when an interior is too large for the block product's LDS staging.
int cblk_setup(bddc_ctx *c) {
    if (c->cblk_state) return 0;
    const int nsub = c->n_sub;
    c->cblk_smem = symm_smem_bytes(c->max_nI);
    if (c->cblk_smem > 160 * 1024) { c->cblk_state = -1; return 0; }
    std::vector<BlockItem> items(nsub);
    std::vector<int32_t> ones(nsub, 1);
    int64_t slot = 0, y = 0;
    for (int i = 0; i < nsub; ++i) {
        items[i] = BlockItem{slot, c->h_nI[i], (int32_t)y};
        slot += op_slots(c->h_nI[i]);
        y += c->h_nI[i];
    }
    if (y > INT32_MAX) { c->cblk_state = -1; return 0; }
    c->cblk_ylen = std::max<int64_t>(1, y);
    int rc;
    if ((rc = dupload(c, &c->d_cblk_items, items)) || (rc = dupload(c, &c->d_cblk_ones, ones)) ||
        (rc = dalloc(c, &c->d_cblk_y, (size_t)c->cblk_ylen * CBLK)) ||
        (rc = dalloc(c, &c->d_cblk_b, (size_t)c->ld * CBLK)) ||
        (rc = dalloc(c, &c->d_cblk_bbp, (size_t)c->vgrid * CBLK)) ||
        (rc = dalloc(c, &c->d_cblk_x, (size_t)c->ld * CBLK)) ||
        (rc = dalloc(c, &c->d_cblk_t, (size_t)c->n_nodes * CBLK)))
        return rc;
    c->cblk_state = 1;
    return 0;
}

// Condensation (Section 3.1) of the g <= CBLK right-hand sides F[0..g) (rows
// of n_nodes): y_I = K_II^{-1} F_I for all of them in one pass over the
// interior tiles, then t_i = K_BI y_I and b per column, into the group buffers.
int run_condense_block(bddc_ctx *c, const double *F, int g) {
    TScope ts(c, TK_COND);
    if (set_symm_smem_limit(c->cblk_smem)) return fail(BDDC_EHIP, "hipFuncSetAttribute (block product LDS) failed");
    BlockSymvArgs a{};
    a.tiles = c->d_KI; a.items = c->d_cblk_items; a.gB = c->d_nodesI;
    a.X = F; a.ldx = c->n_nodes; a.ncols = g;
    a.ypart = c->d_cblk_y; a.ylen = c->cblk_ylen;
    launch_symm(a, c->n_sub, c->cblk_smem, c->stream);
    for (int q = 0; q < g; ++q) {
        CondArgs ca{};
        ca.nI = c->d_nI; ca.nB = c->d_nB; ca.i_off = c->d_i_off; ca.b_off = c->d_b_off;
        ca.nchunk = c->d_cblk_ones; ca.pb = c->d_i_off; ca.ypart = c->d_cblk_y + (size_t)q * c->cblk_ylen;
        ca.kbi_ptr = c->d_kbi_ptr; ca.kbi_col = c->d_kbi_col; ca.kbi_val = c->d_kbi_val; ca.t = c->d_locq;
        launch_cond_local(ca, c->n_sub, c->max_nI, c->stream);
        CondAsmArgs b{};
        b.n = c->n_gamma; b.gamma = c->d_gamma; b.ptr = c->d_asm_ptr; b.idx = c->d_asm_idx;
        b.F = F + (size_t)q * c->n_nodes; b.loc = c->d_locq;
        b.b = c->d_cblk_b + (size_t)q * c->ld; b.part = c->d_cblk_bbp + (size_t)q * c->vgrid;
        launch_cond_asm(b, c->vgrid, c->stream);
    }
    return 0;
}

// b and its ||b||^2 partials of column q of the condensed group
void take_condensed(bddc_ctx *c, int q) {
    launch_copy(c->n_gamma, c->d_cblk_b + (size_t)q * c->ld, c->d_b, c->stream);
    launch_copy(c->vgrid, c->d_cblk_bbp + (size_t)q * c->vgrid, c->d_bbp, c->stream);
}

// Interior recovery (Section 3.1) of g <= CBLK solutions at once: for each
// column q, F[q] (rows of n_nodes) and the interface solution in column q of
// d_cblk_x give K_IB x_B; x_I = K_II^{-1} (F_I - K_IB x_B) for all columns in
// one pass over the interior tiles; u[q] = (x_I, x_G).
int run_recover_block(bddc_ctx *c, const double *F, double *u, int g) {
    TScope ts(c, TK_COND);
    RecArgs a{};
    a.nI = c->d_nI; a.nB = c->d_nB; a.i_off = c->d_i_off; a.b_off = c->d_b_off; a.nodesI = c->d_nodesI;
    a.gB = c->d_gB;
    a.kib_ptr = c->d_kib_ptr; a.kib_col = c->d_kib_col; a.kib_val = c->d_kib_val;
    a.nchunk = c->d_cblk_ones; a.pb = c->d_i_off;
    for (int q = 0; q < g; ++q) {
        a.x = c->d_cblk_x + (size_t)q * c->ld; a.F = F + (size_t)q * c->n_nodes;
        a.out = c->d_cblk_t + (size_t)q * c->n_nodes;
        launch_rec_rhs(a, c->n_sub, c->max_nB, c->stream);
    }
    if (set_symm_smem_limit(c->cblk_smem)) return fail(BDDC_EHIP, "hipFuncSetAttribute (block product LDS) failed");
    BlockSymvArgs b{};
    b.tiles = c->d_KI; b.items = c->d_cblk_items; b.gB = c->d_nodesI;
    b.X = c->d_cblk_t; b.ldx = c->n_nodes; b.ncols = g;
    b.ypart = c->d_cblk_y; b.ylen = c->cblk_ylen;
    launch_symm(b, c->n_sub, c->cblk_smem, c->stream);
    for (int q = 0; q < g; ++q) {
        double *uq = u + (size_t)q * c->n_nodes;
        a.ypart = c->d_cblk_y + (size_t)q * c->cblk_ylen; a.u = uq;
        launch_fill(c->n_nodes, 0.0, uq, c->stream);
        launch_rec_out(a, c->n_sub, c->stream);
        launch_scatter_gamma(c->n_gamma, c->d_gamma, c->d_cblk_x + (size_t)q * c->ld, uq, c->stream);
    }
    return 0;
}

// Interior recovery (Section 3.1): x_I = K_II^{-1} (F_I - K_IB x_B), u = (x_I, x_G).
int run_recover(bddc_ctx *c, const double *F, double *u) {
    TScope ts(c, TK_COND);
    RecArgs a{};
    a.nI = c->d_nI; a.nB = c->d_nB; a.i_off = c->d_i_off; a.b_off = c->d_b_off; a.nodesI = c->d_nodesI;
    a.gB = c->d_gB; a.x = c->d_x; a.F = F;
    a.kib_ptr = c->d_kib_ptr; a.kib_col = c->d_kib_col; a.kib_val = c->d_kib_val; a.out = c->d_tmpN;
    a.nchunk = c->opI.d_nchunk; a.pb = c->opI.d_pb; a.ypart = c->opI.d_ypart; a.u = u;
    launch_rec_rhs(a, c->n_sub, c->max_nB, c->stream);
    run_interior(c, c->d_tmpN);
    launch_fill(c->n_nodes, 0.0, u, c->stream);
    launch_rec_out(a, c->n_sub, c->stream);
    launch_scatter_gamma(c->n_gamma, c->d_gamma, c->d_x, u, c->stream);
    return 0;
}

// ||b - A x||^2 of the interface problem into ctl->true_rr (and out = b - A x)
void run_true_residual(bddc_ctx *c, double *out) {
    run_schur(c, c->d_x, false, false);
    run_resid(c, out, false);
    ReduceArgs r{};
    r.part = c->d_wp; r.n = c->vgrid; r.ncol = 1; r.out = &c->d_ctl->true_rr;
    launch_reduce(r, c->stream);
}

// A basis update was enqueued after the previous solve; the device committed
// it only if the new W^T A W was positive definite.  Adopt its outcome.
void resolve_pending(bddc_ctx *c) {
    if (!c->pend.active) return;
    c->pend.active = false;
    const SyncBuf &h = *c->h_sync;
    if (h.rs.ok) {
        const int k = c->pend.k;
        c->k = k;
        c->WAW.assign(h.waw, h.waw + (size_t)k * k);
        c->GWW = c->pend.GWW;
        c->theta = c->pend.theta;
        if (c->pend.freeze) {
            c->frozen = true;
            c->freeze_step = c->n_updates;
        }
    } else {
        // W^T A W of the new basis not positive definite: it was written over
        // the old one, so the recycled columns are dropped
        c->update_refused++;
        c->k = c->nullc;
        c->WAW.assign(c->nullc, 1.0);
        c->GWW.clear();
        c->theta.clear();
    }
}

// The one host synchronisation of a solve: control block, deflation state
// and, when recording, the scalar histories of the solve.  end_sync_issue
// enqueues the copies and an event after them; work enqueued after that
// keeps the device busy while end_sync_wait waits for the event only.
int end_sync_issue(bddc_ctx *c, bool hist) {
    const size_t waw = c->pend.active ? (size_t)c->pend.k * c->pend.k * sizeof(double) : 0;
    HIPCHK(hipMemcpyAsync(c->h_sync, c->d_sync, offsetof(SyncBuf, waw) + waw, hipMemcpyDeviceToHost, c->stream));
    if (hist) {   // alpha, d and rho (the first hcopy of each), then mu
        const size_t n = (size_t)c->hcopy, cap = (size_t)c->hist_cap;
        HIPCHK(hipMemcpyAsync(c->h_hist, c->d_hblk, (2 * cap + n) * sizeof(double), hipMemcpyDeviceToHost, c->stream));
        HIPCHK(hipMemcpyAsync(c->h_hist + 3 * cap, c->d_muhist, n * RMAX * sizeof(double), hipMemcpyDeviceToHost,
                              c->stream));
    }
    HIPCHK(hipEventRecord(c->sync_ev, c->stream));
    return 0;
}

int end_sync_wait(bddc_ctx *c) {
    HIPCHK(hipEventSynchronize(c->sync_ev));
    *c->h_ctl = c->h_sync->ctl;
    resolve_pending(c);
    return 0;
}

// One right-hand side: condense (unless already done), Algorithm 1 from
// x_prev, recover.  The stream is synchronised once, after the loop.
// u null: the interior recovery is left to the caller (block recovery).
int solve_one(bddc_ctx *c, const double *F, double *u, double rtol, bool recycle, bool condensed, int *iters,
              double *relres) {
    const bool record = recycle && c->R > 0 && !c->frozen;
    const int strat = c->opts.recycle_strategy;
    const bool want_hist = record && (strat == 3 || strat == 4);
    *c->h_flags = 0;
    c->rtol2_run = rtol * rtol;
    const int every = c->opts.restart_every;
    launch_ctl_init(c->d_ctl, rtol * rtol, record ? 1 : 0, c->R + c->nullc > 0 ? c->d_state : nullptr, c->d_hflag,
                    c->d_hprog,
                    every > 0 ? every : INT32_MAX, c->stream);
    if (!condensed) run_condense(c, F);                  // b, ||b||^2 partials
    if (!c->pre_schur) {
        if (c->opts.init_guess == 1) launch_fill(c->n_gamma, 0.0, c->d_x, c->stream);
        run_schur(c, c->d_x, false, false);              // r = b - A x_{-1}
    }
    c->pre_schur = false;
    run_resid(c, c->d_r, c->R + c->nullc > 0);
    {
        TScope ts(c, TK_VEC);
        DeflArgs d{};                                     // Alg. 1 lines 3-4 (k = 0: ||r||^2 only)
        d.n = c->n_gamma; d.x = c->d_x; d.r = c->d_r; d.W = c->d_W; d.AW = c->d_AW; d.ld = c->ld;
        d.wpart = c->d_wp; d.wpart_n = c->vgrid; d.WAWinv = c->d_WAWinv; d.rr_part = c->d_rr; d.ctl = c->d_ctl;
        launch_defl_init(d, c->kmax, c->vgrid, c->stream);
    }
    run_precond(c, c->d_r, c->d_z, 2, false, false, true);  // first test, lines 5-6
    run_pupd(c, true, false, true, 2);                      // line 7 (the first test while recording)
    int restarts = 0, rc, seg_start = 0;
    bool recovered = false;
    while (true) {
        if ((rc = run_loop(c))) return rc;
        run_true_residual(c, c->d_tmp);                  // float64 ||b - A x||
        // while recording, the loop's last pass applied M^{-1} to r_l before
        // its (deferred) stopping test and recorded rho_l, mu_l (Section 4.2)
        const bool hist = want_hist;
        // interior recovery from this x, enqueued behind the synchronisation's
        // copies so that the device works while the host waits (done again if
        // the solve goes on or x is reset)
        if ((rc = end_sync_issue(c, hist))) return rc;
        if (u && (rc = run_recover(c, F, u))) return rc;
        recovered = true;
        if ((rc = end_sync_wait(c))) return rc;
        const Ctl &h = *c->h_ctl;
        if (h.zero_rhs) {
            launch_fill(c->n_gamma, 0.0, c->d_x, c->stream);
            recovered = false;
        }
        if (h.status != 0 || h.zero_rhs) break;
        if (h.true_rr < h.rtol2 * h.denom2 || h.iter >= c->opts.max_it) break;
        // residual replacement, then continue from line 5 (iterations keep
        // counting); only the directions from here on are recycled
        ++restarts;
        seg_start = h.j;
        recovered = false;
        launch_copy(c->n_gamma, c->d_tmp, c->d_r, c->stream);
        launch_resume(c->d_ctl, every > 0 && h.iter < INT32_MAX - every ? h.iter + every : INT32_MAX, c->stream);
        // (while recording, the loop's last pass has advanced the direction index)
        run_precond(c, c->d_r, c->d_z, 0, false, !record, true);
        run_pupd(c, true, false, true, 0);
        *c->h_flags = 0;
    }
    const Ctl h = *c->h_ctl;
    c->last_iters = h.iter;
    c->last_restarts = restarts;
    c->seg_start = seg_start;
    c->last_status = h.status;
    c->have_solve = true;
    c->have_hist = want_hist;
    if (iters) *iters = h.iter;
    if (relres) *relres = (h.bb > 0 && !h.zero_rhs) ? std::sqrt(h.true_rr / h.bb) : 0.0;
    if (u && !recovered && (rc = run_recover(c, F, u))) return rc;
    if (h.status == BDDC_EBREAKDOWN) return fail(BDDC_EBREAKDOWN, "PCG breakdown (r^T z <= 0, p^T A p <= 0 or NaN)");
    if (h.status == BDDC_ENOTCONV) return fail(BDDC_ENOTCONV, "max_it reached");
    return 0;
}

// W <- [W, P] Y, AW <- [AW, AP] Y in place (each row of the product reads
// only the same row of its operands, and every wave reads its rows before
// writing them), then on the device: Gram W^T A W of the new basis, Cholesky
// and inverse, and the commit of the inverse when it is positive definite
// (else the basis is dropped).  Nothing here waits for the device; the
// outcome is adopted at the next synchronisation (resolve_pending).
int apply_basis(bddc_ctx *c, const std::vector<double> &Y, int m, int ncol, const std::vector<double> &gww,
                const std::vector<double> &theta, bool freeze, int j0) {
    // (Y: m = recycled columns + stored directions rows, ncol recycled columns)
    const int ldy = (ncol + 7) / 8 * 8;
    std::memset(c->h_Y, 0, (size_t)m * ldy * sizeof(double));
    for (int q = 0; q < m; ++q)
        for (int j = 0; j < ncol; ++j) c->h_Y[(size_t)q * ldy + j] = Y[(size_t)q * ncol + j];
    HIPCHK(hipMemcpyAsync(c->d_Y, c->h_Y, (size_t)m * ldy * sizeof(double), hipMemcpyHostToDevice, c->stream));
    // recycled columns only: a pure Neumann problem's constant column 0 stays
    // in place in W, A W and the new buffers (set at setup)
    const int nc0 = c->nullc, k1 = c->k - nc0, l = m - k1;
    const size_t o0 = (size_t)nc0 * c->ld;
    GemmArgs g{};
    g.n = c->n_gamma; g.ld = c->ld; g.Y = c->d_Y; g.ncol = ncol; g.ldy = ldy;
    g.k1 = k1; g.k2 = l;
    g.V1[0] = c->d_W + o0; g.V2[0] = c->d_P + (size_t)j0 * c->ld; g.out[0] = c->d_W + o0;
    g.V1[1] = c->d_AW + o0; g.V2[1] = c->d_AP + (size_t)j0 * c->ld; g.out[1] = c->d_AW + o0;
    launch_recycle_gemm(g, c->stream);
    ncol += nc0;                    // the Gram product, Cholesky and commit cover all columns
    const int nb = c->gram_nb;
    GramArgs gr{};
    gr.n = c->n_gamma; gr.k = ncol; gr.ld = c->ld; gr.X = c->d_W; gr.Y = c->d_AW; gr.part = c->d_gp;
    launch_gram(gr, nb, c->stream);
    ReduceArgs r{};
    r.part = c->d_gp; r.n = nb; r.ncol = ncol * ncol; r.out = c->d_WAWnew;
    launch_reduce(r, c->stream);
    CholArgs ch{};
    ch.k = ncol; ch.waw = c->d_WAWnew; ch.waw_sym = c->d_WAWsym; ch.inv = c->d_invnew; ch.state = c->d_state;
    launch_chol_inv(ch, c->stream);
    if (c->opts.reorth) {   // (W^T W)^{-1} of the new basis
        GramArgs gw{};
        gw.n = c->n_gamma; gw.k = ncol; gw.ld = c->ld; gw.X = c->d_W; gw.Y = c->d_W; gw.part = c->d_gp;
        launch_gram(gw, nb, c->stream);
        ReduceArgs rw{};
        rw.part = c->d_gp; rw.n = nb; rw.ncol = ncol * ncol; rw.out = c->d_WWnew;
        launch_reduce(rw, c->stream);
        CholArgs cw{};
        cw.k = ncol; cw.waw = c->d_WWnew; cw.waw_sym = c->d_WWsym; cw.inv = c->d_WWinvnew; cw.state = c->d_state2;
        launch_chol_inv(cw, c->stream);
    }
    CommitArgs cm{};
    cm.ncol = ncol; cm.nullc = nc0;
    cm.inv_new = c->d_invnew; cm.inv = c->d_WAWinv; cm.state = c->d_state;
    if (c->opts.reorth) { cm.ww_new = c->d_WWinvnew; cm.ww = c->d_WWinv; }
    launch_commit(cm, c->stream);
    c->pend.active = true;
    c->pend.k = ncol;
    c->pend.GWW = gww;
    c->pend.theta = theta;
    c->pend.freeze = freeze;
    return 0;
}

// Recycling step after a solve (Section 4.2): B1/B2 select stored search
// directions; B3/B4 solve the harmonic-Ritz problem (eq. harmonicRitz) on
// V = [W, P] with the small matrices formed from the solve's own scalars,
// keep the R smallest (B3) or largest (B4) values, and test eq.
// harmritzstopcrit for freezing the basis.
int do_recycle(bddc_ctx *c) {
    if (c->R == 0 || c->frozen || !c->have_solve) return 0;
    c->have_solve = false;
    if (c->last_status != 0) return 0;
    const int strat = c->opts.recycle_strategy;
    // the directions of one unbroken run: those after the last residual
    // replacement (all of them without one), as many as were stored
    const int j0 = c->seg_start;
    const int l = std::max(0, std::min(c->last_iters, c->save_cap) - j0);
    // the recycled columns of W (after the constant one of a pure Neumann problem)
    const int nc0 = c->nullc, kt = c->k, k = kt - nc0, m = k + l;
    auto waw = [&](int i, int j) { return c->WAW[(size_t)(i + nc0) * kt + j + nc0]; };
    c->n_updates++;
    if (strat == 1 || strat == 2) {
        // B1: first R search directions; B2: sliding window of the last R
        std::vector<int> cols;
        if (strat == 1) {
            if (k >= c->R) return 0;
            for (int q = 0; q < std::min(m, c->R); ++q) cols.push_back(q);
        } else {
            for (int q = std::max(0, m - c->R); q < m; ++q) cols.push_back(q);
        }
        const int ncol = (int)cols.size();
        if (ncol == 0) return 0;
        std::vector<double> Y((size_t)m * ncol, 0.0);
        for (int j = 0; j < ncol; ++j) Y[(size_t)cols[j] * ncol + j] = 1.0;
        return apply_basis(c, Y, m, ncol, std::vector<double>(), std::vector<double>(), false, j0);
    }
    if (m == 0 || !c->have_hist) return 0;
    // scalars of the last solve
    const size_t hn = (size_t)c->hist_cap;
    const double *al = c->h_hist + j0, *dd = c->h_hist + hn + j0, *rho = c->h_hist + 2 * hn + j0,
                 *mu = c->h_hist + 3 * hn + (size_t)j0 * RMAX + nc0;
    // F = V^T A V = blockdiag(W^T A W, diag(d)) and G = V^T A M^{-1} A V from the
    // recurrences of Algorithm 1: M^{-1} A p_j = (z_j - z_{j+1}) / alpha_j
    std::vector<double> F((size_t)m * m, 0.0), G((size_t)m * m, 0.0);
    for (int i = 0; i < k; ++i)
        for (int j = 0; j < k; ++j) {
            F[(size_t)i * m + j] = waw(i, j);
            G[(size_t)i * m + j] = c->GWW[(size_t)i * k + j];
        }
    for (int j = 0; j < l; ++j) {
        const double beta = rho[j + 1] / rho[j];
        F[(size_t)(k + j) * m + k + j] = dd[j];
        G[(size_t)(k + j) * m + k + j] = dd[j] * (1.0 + beta) / al[j];
        if (j > 0) {
            const double off = -dd[j - 1] * dd[j] / rho[j - 1];
            G[(size_t)(k + j - 1) * m + k + j] = off;
            G[(size_t)(k + j) * m + k + j - 1] = off;
        }
        for (int i = 0; i < k; ++i) {
            double s = 0.0;
            for (int q = 0; q < k; ++q)
                s += waw(i, q) * (mu[(size_t)j * RMAX + q] - mu[(size_t)(j + 1) * RMAX + q]);
            s /= al[j];
            G[(size_t)i * m + k + j] = s;
            G[(size_t)(k + j) * m + i] = s;
        }
    }
    for (size_t e = 0; e < G.size(); ++e)
        if (!std::isfinite(G[e]) || !std::isfinite(F[e])) return 0;   // keep the basis
    // generalized eigenproblem G y = theta F y: F = U diag(lam) U^T, directions
    // with lam < 1e-12 max dropped, T = U lam^{-1/2}, H = T^T G T.  F is block
    // diagonal (W^T A W, then diag(d)): its eigenpairs are those of W^T A W
    // and (d_j, unit vectors).
    std::vector<double> lam(m, 0.0), U((size_t)m * m, 0.0);
    if (k > 0) {
        std::vector<double> Fw((size_t)k * k), lw, Uw;
        for (int i = 0; i < k; ++i)
            for (int j = 0; j < k; ++j) Fw[(size_t)i * k + j] = F[(size_t)i * m + j];
        sym_eig(Fw, k, lw, Uw);
        for (int j = 0; j < k; ++j) {
            lam[j] = lw[j];
            for (int i = 0; i < k; ++i) U[(size_t)i * m + j] = Uw[(size_t)i * k + j];
        }
    }
    for (int j = k; j < m; ++j) {
        lam[j] = F[(size_t)j * m + j];
        U[(size_t)j * m + j] = 1.0;
    }
    const double lmax = *std::max_element(lam.begin(), lam.end());
    std::vector<int> keep;
    for (int i = 0; i < m; ++i)
        if (lam[i] > 1e-12 * lmax) keep.push_back(i);
    const int mk = (int)keep.size();
    if (mk == 0) return 0;
    std::vector<double> T((size_t)m * mk);
    for (int q = 0; q < m; ++q)
        for (int j = 0; j < mk; ++j) T[(size_t)q * mk + j] = U[(size_t)q * m + keep[j]] / std::sqrt(lam[keep[j]]);
    std::vector<double> GT((size_t)m * mk, 0.0), H((size_t)mk * mk, 0.0);
    for (int q = 0; q < m; ++q)
        for (int j = 0; j < mk; ++j) {
            double s = 0.0;
            for (int t = 0; t < m; ++t) s += G[(size_t)q * m + t] * T[(size_t)t * mk + j];
            GT[(size_t)q * mk + j] = s;
        }
    for (int i = 0; i < mk; ++i)
        for (int j = 0; j < mk; ++j) {
            double s = 0.0;
            for (int q = 0; q < m; ++q) s += T[(size_t)q * mk + i] * GT[(size_t)q * mk + j];
            H[(size_t)i * mk + j] = s;
        }
    for (int i = 0; i < mk; ++i)
        for (int j = i + 1; j < mk; ++j) H[(size_t)i * mk + j] = H[(size_t)j * mk + i] = 0.5 * (H[(size_t)i * mk + j] + H[(size_t)j * mk + i]);
    std::vector<double> th, Z;
    sym_eig(H, mk, th, Z);
    std::vector<int> ord(mk);
    std::iota(ord.begin(), ord.end(), 0);
    if (strat == 4) std::reverse(ord.begin(), ord.end());   // descending for B4
    const int ncol = std::min(c->R, mk);
    std::vector<double> Y((size_t)m * ncol, 0.0), thsel(ncol);
    for (int j = 0; j < ncol; ++j) {
        thsel[j] = th[ord[j]];
        for (int q = 0; q < m; ++q) {
            double s = 0.0;
            for (int t = 0; t < mk; ++t) s += T[(size_t)q * mk + t] * Z[(size_t)t * mk + ord[j]];
            Y[(size_t)q * ncol + j] = s;
        }
    }
    // G_WW of the new basis: Y^T (G Y)
    std::vector<double> GY((size_t)m * ncol, 0.0), gww((size_t)ncol * ncol, 0.0);
    for (int q = 0; q < m; ++q)
        for (int r = 0; r < m; ++r) {
            const double g = G[(size_t)q * m + r];
            for (int j = 0; j < ncol; ++j) GY[(size_t)q * ncol + j] += g * Y[(size_t)r * ncol + j];
        }
    for (int q = 0; q < m; ++q)
        for (int i = 0; i < ncol; ++i) {
            const double y = Y[(size_t)q * ncol + i];
            for (int j = 0; j < ncol; ++j) gww[(size_t)i * ncol + j] += y * GY[(size_t)q * ncol + j];
        }
    // freeze test (eq. harmritzstopcrit) on the sorted selected values
    bool freeze = false;
    if ((int)c->theta.size() == c->R && ncol == c->R) {
        double num = 0.0, den = 0.0;
        for (int j = 0; j < ncol; ++j) {
            num += (thsel[j] - c->theta[j]) * (thsel[j] - c->theta[j]);
            den += thsel[j] * thsel[j];
        }
        freeze = std::sqrt(num) <= c->opts.ritz_freeze_tol * std::sqrt(den);
    }
    return apply_basis(c, Y, m, ncol, gww, thsel, freeze, j0);
}

// Wait for the device and adopt a pending basis update (end of a sequence).
int settle(bddc_ctx *c) {
    if (c->R > 0 && c->pend.active)
        HIPCHK(hipMemcpyAsync(c->h_sync, c->d_sync, offsetof(SyncBuf, waw) + (size_t)c->pend.k * c->pend.k * sizeof(double),
                              hipMemcpyDeviceToHost, c->stream));
    HIPCHK(hipStreamSynchronize(c->stream));
    resolve_pending(c);
    return 0;
}

}  // namespace


// ======================================================================== ABI
extern "C" {

void bddc_default_opts(bddc_opts *o) {
    std::memset(o, 0, sizeof(*o));
    o->constraints = BDDC_CORNERS | BDDC_FACES;
    o->weights = 1;
    o->local_prec = 64;
    o->recycle_R = 0;
    o->recycle_strategy = 4;
    o->ritz_freeze_tol = 1e-5;
    o->stop_rule = 0;
    o->init_guess = 0;
    o->max_it = 1000;
    o->save_cap = 256;
    o->use_graph = 2;
    o->autotune = 1;
    o->coarse_form = 0;
    o->adapt_max_per_face = 10;
    o->adapt_tau = 0.0;
    o->local_prec_set = 0;
    o->coef_log = 0;
    o->restart_every = 0;
    o->adapt2_tau = 0.0;
    o->adapt2_max_per_face = 10;
    o->adapt_lobpcg_it = 0;
}

const char *bddc_last_error(void) { return g_err.c_str(); }

}  // extern "C"

namespace {

// Pure Neumann problem: column 0 of W (and of A W, by the reading that it
// enters the projections with the Euclidean inner product) is the constant
// interface vector w0 = 1/sqrt(n_gamma), its block of W^T A W (and W^T W) is
// 1, and the basis holds it alone after setup and after a reset.
void init_null_column(bddc_ctx *c) {
    if (!c->nullc) return;
    const double v = 1.0 / std::sqrt((double)c->n_gamma);
    for (double *w : {c->d_W, c->d_AW})
        if (w) launch_fill(c->n_gamma, v, w, c->stream);
    launch_fill(1, 1.0, c->d_WAWinv, c->stream);
    launch_fill(1, 1.0, c->d_WWinv, c->stream);
    if (c->d_state) launch_set_state(c->d_state, 1, 1, c->stream);
    c->k = 1;
    c->WAW.assign(1, 1.0);
}

// Values of the level-1 coarse DOFs on the constant function 1 (the null
// vector of the coarse matrix of a pure Neumann problem): 1 for corners and
// averages, the sum of the weights for weighted rows (0 for the adaptive
// rows, which are orthogonal to the face average).
// Gather lists of the subregion matrices K2_j = sum over the member
// subdomains i of K_Ci (dense nL_j x nL_j at K2_off[j], ids in SubregionHost::L
// order): entry -> positions in the packed K_Ci.
void k2_csr(const Structure &st, const std::vector<int32_t> &nc, const std::vector<int64_t> &kc_off,
            const std::vector<int64_t> &K2_off, std::vector<int32_t> &ptr, std::vector<int32_t> &idx) {
    std::vector<std::pair<int64_t, int32_t>> pr;
    std::vector<int32_t> pos(st.coarse.size(), -1);
    for (int j = 0; j < st.n_sr; ++j) {
        const auto &L = st.sr[j].L;
        const int64_t nL = (int64_t)L.size();
        for (size_t a = 0; a < L.size(); ++a) pos[L[a]] = (int32_t)a;
        for (int32_t i : st.sr[j].subs)
            for (int qa = 0; qa < nc[i]; ++qa)
                for (int qb = 0; qb < nc[i]; ++qb)
                    pr.push_back({K2_off[j] + (int64_t)pos[st.sub[i].cidx[qa]] * nL + pos[st.sub[i].cidx[qb]],
                                  (int32_t)(kc_off[i] + qa * nc[i] + qb)});
        for (size_t a = 0; a < L.size(); ++a) pos[L[a]] = -1;
    }
    build_csr(K2_off[st.n_sr], pr, ptr, idx);
}

// Adaptivity at level 2: the subregion Schur complements on the device
// (assemble K2_j, sweep its interior coarse DOFs), the face pencils on the
// host, the new rows appended to the level-3 DOFs.
int adapt_level2(bddc_ctx *c, const std::vector<int32_t> &nc, const std::vector<int64_t> &kc_off) {
    Structure &st = c->st;
    const int nsr = st.n_sr;
    hipStream_t s = c->stream;
    std::vector<int64_t> K2_off(nsr + 1, 0);
    for (int j = 0; j < nsr; ++j) K2_off[j + 1] = K2_off[j] + (int64_t)st.sr[j].L.size() * st.sr[j].L.size();
    std::vector<int32_t> ptr, idx;
    k2_csr(st, nc, kc_off, K2_off, ptr, idx);
    int32_t *dp = nullptr, *di = nullptr;
    double *dK = nullptr;
    int rc;
    if ((rc = dupload(c, &dp, ptr)) || (rc = dupload(c, &di, idx)) ||
        (rc = dalloc(c, &dK, (size_t)std::max<int64_t>(1, K2_off[nsr]))))
        return rc;
    launch_gather_sum(K2_off[nsr], dp, di, c->d_KC, dK, s);
    std::vector<SweepDesc> sw(nsr);
    for (int j = 0; j < nsr; ++j) {
        const int n = (int)st.sr[j].L.size();
        sw[j] = SweepDesc{dK + K2_off[j], n, n, 0, st.sr[j].nI, n};
    }
    if ((rc = run_sweeps(c, sw))) return rc;
    std::vector<double> h((size_t)K2_off[nsr]);
    HIPCHK(hipMemcpyAsync(h.data(), dK, h.size() * sizeof(double), hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    dfree(c, dp); dfree(c, di); dfree(c, dK);
    int32_t st_h = 0;
    HIPCHK(hipMemcpy(&st_h, c->d_status, sizeof(int32_t), hipMemcpyDeviceToHost));
    if (st_h) return fail(BDDC_ESINGULAR, "non-positive pivot in a subregion interior elimination");
    std::vector<std::vector<double>> S2(nsr);
    std::vector<char> floating(nsr, 1);
    for (int j = 0; j < nsr; ++j) {
        const SubregionHost &r = st.sr[j];
        const int n = (int)r.L.size();
        S2[j].resize((size_t)r.nB * r.nB);
        for (int a = 0; a < r.nB; ++a)
            for (int b = 0; b < r.nB; ++b)
                S2[j][(size_t)a * r.nB + b] = h[K2_off[j] + (int64_t)(r.nI + a) * n + r.nI + b];
        for (int32_t i : r.subs)
            for (int32_t l : st.sub[i].elem_loc)
                if (l < 0) floating[j] = 0;
    }
    std::vector<Level3Dof> extra;
    std::string err;
    if ((rc = adaptive_level2(st, S2, floating, c->opts.adapt2_tau, std::max(0, c->opts.adapt2_max_per_face),
                              c->opts.adapt_lobpcg_it, extra, c->adapt2, err)) ||
        (rc = add_level3_dofs(st, extra, err)))
        return fail(rc, err);
    return 0;
}

std::vector<double> coarse_null_vector(const Structure &st) {
    std::vector<double> e(st.coarse.size(), 1.0);
    for (size_t q = 0; q < st.coarse.size(); ++q) {
        const CoarseDof &d = st.coarse[q];
        if (d.wts.empty()) continue;
        double s = 0.0;
        for (double w : d.wts) s += w;
        e[q] = s;
    }
    return e;
}

// Mean of the diagonal of an n x n matrix with leading dimension ld.
double diag_mean(const double *A, int n, int64_t ld, int &rc) {
    std::vector<double> d((size_t)std::max(n, 1));
    rc = 0;
    if (n == 0) return 1.0;
    if (hipMemcpy2D(d.data(), sizeof(double), A, (size_t)(ld + 1) * sizeof(double), sizeof(double), n,
                    hipMemcpyDeviceToHost) != hipSuccess) {
        rc = fail(BDDC_EHIP, "hipMemcpy2D of a coarse diagonal failed");
        return 1.0;
    }
    double s = 0.0;
    for (double x : d) s += x;
    return s / n;
}

// Inverse of a semidefinite coarsest matrix K with null vector e (pure
// Neumann problem), in the sweep's sign convention: the sweep of K + a e e^T
// (a = mean diagonal / e^T e) leaves -(K + a e e^T)^{-1}; adding
// e e^T / (a (e^T e)^2) gives -K^+, since (K + a e e^T)^{-1} and K^+ agree on
// e's complement and (K + a e e^T)^{-1} e = e / (a e^T e).
int sweep_semidefinite(bddc_ctx *c, double *A, int n, int64_t ld, const std::vector<double> &e) {
    double ee = 0.0;
    for (double x : e) ee += x * x;
    if (n == 0 || !(ee > 0.0)) return fail(BDDC_ESINGULAR, "semidefinite coarse matrix without a null vector");
    int rc;
    const double a = diag_mean(A, n, ld, rc) / ee;
    if (rc) return rc;
    double *de;
    if ((rc = dupload(c, &de, e))) return rc;
    launch_rank1(A, ld, n, de, a, c->stream);
    if ((rc = run_sweeps(c, {SweepDesc{A, n, (int)ld, 0, n, n}}))) return rc;
    launch_rank1(A, ld, n, de, 1.0 / (a * ee * ee), c->stream);
    HIPCHK(hipStreamSynchronize(c->stream));
    dfree(c, de);
    return 0;
}

// Product blocks for `per_cu` blocks per compute unit, at most one per 16
// tiles.
int product_blocks(const bddc_ctx *c, int64_t total_tiles, int per_cu) {
    return (int)std::max<int64_t>(1, std::min<int64_t>((int64_t)c->n_cu * per_cu, (total_tiles + 15) / 16));
}

int setup_operators(bddc_ctx *c) {
    const int nsub = c->n_sub;
    OpHost *ops[2] = {&c->opS, &c->opN};
    for (int w = 0; w < 2; ++w) {
        OpHost &op = *ops[w];
        const bool isN = w == 1;
        op.prec = isN ? c->prec : 64;
        op.dev.tiles = isN ? c->d_N : (const void *)c->d_S;
        op.dev.t_off = c->d_s_off;   // the two batches share the layout
        op.dev.nB = c->d_nB;
        op.dev.b_off = c->d_b_off;
        op.dev.gB = c->d_gB;
        op.n_tiles = 0;
        for (int i = 0; i < nsub; ++i) op.n_tiles += op_slots(c->h_nB[i]);
        op.bytes = product_bytes(c, op.prec, isN && c->nC > 0);
        op.cfg = SymvCfg{4, 2};
        op.smem = symv_smem(op.prec, op.cfg.nw, c->max_nt);
        int rc = build_worklist(c, op, product_blocks(c, op.n_tiles, op.bpc), op.per_sub);
        if (rc) return rc;
    }
    // (LDS accumulators are float64 for a float64 Neumann batch, else float32)
    const int pw = (c->prec_built & 1) ? 64 : 32;
    const size_t need4 = std::max(symv_smem(64, 4, c->max_nt), symv_smem(pw, 4, c->max_nt));
    const size_t need8 = std::max(symv_smem(64, 8, c->max_nt), symv_smem(pw, 8, c->max_nt));
    if (need4 > 160 * 1024) return fail(BDDC_EINVAL, "a subdomain interface is too large for the LDS-staged products");
    c->allow8 = need8 <= 160 * 1024;
    if (set_symv_smem_limit(c->allow8 ? need8 : need4)) return fail(BDDC_EHIP, "hipFuncSetAttribute (dynamic LDS) failed");
    c->t_bytes[TK_SCHUR] = c->opS.bytes;
    c->t_bytes[TK_PREC] = c->opN.bytes;
    return 0;
}

// Interior inverses K_II^{-1} packed like the other symmetric operators, and
// the sparse couplings K_IB (interior rows) and K_BI (interface rows) from
// the element matrices c_e h Kref (Section 2), for condensation and recovery.
int setup_interior(bddc_ctx *c, const std::vector<int64_t> &k_off) {
    const int nsub = c->n_sub;
    const Structure &st = c->st;
    std::vector<int64_t> ki_off(nsub + 1, 0);
    for (int i = 0; i < nsub; ++i) ki_off[i + 1] = ki_off[i] + op_slots(c->h_nI[i]) * 256;
    int rc;
    if ((rc = dupload(c, &c->d_ki_off, ki_off)) || (rc = dalloc_tiles(c, &c->d_KI, (size_t)std::max<int64_t>(1, ki_off[nsub]))))
        return rc;
    std::vector<PackDesc> pk;
    for (int i = 0; i < nsub; ++i) {
        if (c->h_nI[i] == 0) continue;
        const int nl = st.sub[i].nloc;
        pk.push_back(PackDesc{c->d_K + k_off[i], nl, c->h_nI[i], -1.0, nullptr, nullptr, 0, 0, ki_off[i], -1});
    }
    if (!pk.empty()) {
        PackDesc *dpk;
        if ((rc = dupload(c, &dpk, pk))) return rc;
        launch_pack(dpk, (int)pk.size(), 64, c->d_KI, nullptr, c->stream);
        HIPCHK(hipStreamSynchronize(c->stream));
        dfree(c, dpk);
    }
    // K_IB from the element matrices; Kref: 1/3 on the diagonal, 0 between
    // vertices differing in one coordinate, -1/12 otherwise
    std::vector<int32_t> ib_ptr(1, 0), ib_col, bi_ptr(1, 0), bi_col;
    std::vector<double> ib_val, bi_val;
    for (int i = 0; i < nsub; ++i) {
        const SubHost &sh = st.sub[i];
        const int nI = sh.nI, nB = sh.nB;
        std::vector<std::map<int, double>> rows(nI), cols(nB);
        for (size_t t = 0; t < sh.elem.size(); ++t) {
            for (int v = 0; v < 8; ++v) {
                const int a = sh.elem_loc[t * 8 + v];
                if (a < 0 || a >= nI) continue;
                for (int w = 0; w < 8; ++w) {
                    const int b = sh.elem_loc[t * 8 + w];
                    if (b < nI) continue;
                    const int nd = __builtin_popcount(v ^ w);
                    if (nd == 1) continue;
                    const double kv = sh.elem_c[t] * (nd == 0 ? 1.0 / 3.0 : -1.0 / 12.0);
                    rows[a][b - nI] += kv;
                    cols[b - nI][a] += kv;
                }
            }
        }
        for (int a = 0; a < nI; ++a) {
            for (auto &e : rows[a]) { ib_col.push_back(e.first); ib_val.push_back(e.second); }
            ib_ptr.push_back((int32_t)ib_col.size());
        }
        for (int k = 0; k < nB; ++k) {
            for (auto &e : cols[k]) { bi_col.push_back(e.first); bi_val.push_back(e.second); }
            bi_ptr.push_back((int32_t)bi_col.size());
        }
    }
    if ((rc = dupload(c, &c->d_kib_ptr, ib_ptr)) || (rc = dupload(c, &c->d_kib_col, ib_col)) ||
        (rc = dupload(c, &c->d_kib_val, ib_val)) || (rc = dupload(c, &c->d_kbi_ptr, bi_ptr)) ||
        (rc = dupload(c, &c->d_kbi_col, bi_col)) || (rc = dupload(c, &c->d_kbi_val, bi_val)) ||
        (rc = dalloc(c, &c->d_tmpN, (size_t)c->n_nodes)))
        return rc;
    OpHost &op = c->opI;
    op.interior = true;
    op.prec = 64;
    op.dev.tiles = c->d_KI;
    op.dev.t_off = c->d_ki_off;
    op.dev.nB = c->d_nI;
    op.dev.b_off = c->d_i_off;
    op.dev.gB = c->d_nodesI;
    op.n_tiles = ki_off[nsub] / 256;
    op.cfg = SymvCfg{4, 2};
    int max_ntI = 0;
    for (int i = 0; i < nsub; ++i) max_ntI = std::max(max_ntI, (c->h_nI[i] + TILE - 1) / TILE);
    if (symv_smem(64, 4, max_ntI) > 160 * 1024) return fail(BDDC_EINVAL, "a subdomain interior is too large for the LDS-staged products");
    c->max_ntI = max_ntI;
    op.smem = symv_smem(64, 4, max_ntI);
    if (c->allow8 && symv_smem(64, 8, max_ntI) > 160 * 1024) c->allow8 = false;
    const int nwmax = c->allow8 ? 8 : 4;
    const size_t lim = std::max(symv_smem(64, nwmax, std::max(c->max_nt, max_ntI)),
                                symv_smem((c->prec_built & 1) ? 64 : 32, nwmax, c->max_nt));
    if (set_symv_smem_limit(lim)) return fail(BDDC_EHIP, "hipFuncSetAttribute (dynamic LDS) failed");
    HIPCHK(hipMemsetAsync(c->d_tmpN, 0, (size_t)c->n_nodes * sizeof(double), c->stream));
    return build_worklist(c, op, product_blocks(c, op.n_tiles, op.bpc), op.per_sub);
}

// Tile-level autotuning of the two batched products on the operators just
// built: work-list granularity (items per compute unit), waves per block and
// tiles in flight per wave; the fastest of a few timed launches is kept.
int tune_operators(bddc_ctx *c, int mask = 7) {
    hipEvent_t e0 = nullptr, e1 = nullptr;
    HIPCHK(hipEventCreate(&e0));
    HIPCHK(hipEventCreate(&e1));
    int rc = 0;
    const int bpcs[7] = {1, 2, 3, 4, 5, 6, 8};
    OpHost *ops[3] = {&c->opS, &c->opN, &c->opI};
    for (int w = 0; w < 3 && rc == 0; ++w) {
        OpHost &op = *ops[w];
        if (op.dev.n_blocks == 0 || !((mask >> w) & 1)) continue;
        const int mnt = op.interior ? c->max_ntI : c->max_nt;
        float best = 1e30f;
        int best_bpc = op.bpc;
        bool best_ps = op.per_sub;
        SymvCfg best_cfg{4, 2};
        // times `reps` launches of a configuration (after 2 untimed ones)
        auto time_cfg = [&](int bpc, bool ps, SymvCfg cfg, int reps, float &ms) -> int {
            int r0 = build_worklist(c, op, product_blocks(c, op.n_tiles, bpc), ps);
            if (r0) return r0;
            const size_t smem = symv_smem(op.prec, cfg.nw, mnt);
            SymvArgs a{};
            a.op = op.dev; a.x = op.interior ? c->d_tmpN : c->d_x; a.ypart = op.d_ypart;
            a.ctl = c->d_ctl;
            if (w == 1) set_restriction(c, a);
            for (int r = 0; r < 2; ++r) launch_symv(a, (SymvOp)w, op.prec, cfg, smem, c->stream);
            HIPCHK(hipEventRecord(e0, c->stream));
            for (int r = 0; r < reps; ++r) launch_symv(a, (SymvOp)w, op.prec, cfg, smem, c->stream);
            HIPCHK(hipEventRecord(e1, c->stream));
            HIPCHK(hipEventSynchronize(e1));
            HIPCHK(hipEventElapsedTime(&ms, e0, e1));
            ms /= reps;
            return 0;
        };
        struct Cand { float ms; int bpc; bool ps; SymvCfg cfg; };
        std::vector<Cand> cand;
        for (int trial = 0; trial < 14 && rc == 0; ++trial) {
            const bool ps = trial >= 7;
            const int bpc = bpcs[trial % 7];
            for (int nw : {4, 8}) {
                if (nw == 8 && !c->allow8) continue;
                for (int u : {2, 4}) {
                    float ms = 0.f;
                    if ((rc = time_cfg(bpc, ps, SymvCfg{nw, u}, 4, ms))) break;
                    cand.push_back(Cand{ms, bpc, ps, SymvCfg{nw, u}});
                }
                if (rc) break;
            }
        }
        // the four fastest, timed again in turn over two rounds (a single
        // short timing can be off by several percent); the lowest total wins
        if (rc == 0 && !cand.empty()) {
            std::stable_sort(cand.begin(), cand.end(), [](const Cand &x, const Cand &y) { return x.ms < y.ms; });
            const size_t nk = std::min<size_t>(4, cand.size());
            std::vector<float> tot(nk, 0.f);
            for (int round = 0; round < 2 && rc == 0; ++round)
                for (size_t k = 0; k < nk && rc == 0; ++k) {
                    float ms = 0.f;
                    if ((rc = time_cfg(cand[k].bpc, cand[k].ps, cand[k].cfg, 6, ms))) break;
                    tot[k] += ms;
                }
            size_t kb = 0;
            for (size_t k = 1; k < nk; ++k)
                if (tot[k] < tot[kb]) kb = k;
            best = tot[kb] / 2 * 4;       // (kept in the unit of four launches)
            best_bpc = cand[kb].bpc; best_ps = cand[kb].ps; best_cfg = cand[kb].cfg;
        }
        if (rc == 0) rc = build_worklist(c, op, product_blocks(c, op.n_tiles, best_bpc), best_ps);
        op.cfg = best_cfg;
        op.bpc = best_bpc;
        op.per_sub = best_ps;
        op.smem = symv_smem(op.prec, best_cfg.nw, mnt);
        op.tuned_us = best * 1e3f / 4;
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    return rc;
}

// Row-major copy of an nC x nC matrix (given column-major when `transpose`)
// with rows padded to an even length, and the r_C buffer of the dense product.
int upload_dense_coarse(bddc_ctx *c, const std::vector<double> &h, bool transpose) {
    const int n = c->nC;
    c->ldm = (n + 1) & ~1;
    std::vector<double> t((size_t)n * c->ldm, 0.0);
    for (int r = 0; r < n; ++r)
        for (int q = 0; q < n; ++q)
            t[(size_t)r * c->ldm + q] = transpose ? h[(size_t)q * n + r] : h[(size_t)r * n + q];
    int rc;
    if ((rc = dupload(c, &c->d_Mc, t)) || (rc = dalloc(c, &c->d_rC, (size_t)std::max(1, n)))) return rc;
    return 0;
}

// The level-2 BDDC approximation of K_C^{-1} is a fixed linear operator: its
// columns are the level-2/3 chain applied to the unit vectors e_q (rc reads
// the coarse residual from one dense vector), stored row-major.
int build_explicit_coarse(bddc_ctx *c) {
    const int n = c->nC;
    hipStream_t s = c->stream;
    std::vector<int32_t> ptr(n + 1), idx(n);
    for (int q = 0; q <= n; ++q) ptr[q] = q;
    for (int q = 0; q < n; ++q) idx[q] = q;
    int32_t *dp, *di;
    double *de, *dcol;
    int rc;
    if ((rc = dupload(c, &dp, ptr)) || (rc = dupload(c, &di, idx)) || (rc = dalloc(c, &de, (size_t)n)) ||
        (rc = dalloc(c, &dcol, (size_t)n * n)))
        return rc;
    launch_fill(n, 0.0, de, s);
    launch_set_done(c->d_ctl, 0, s);
    const L2Args l = l2_args(c, Gather{dp, di, de});
    for (int q = 0; q < n; ++q) {
        launch_fill(1, 1.0, de + q, s);
        run_l2_chain(c, l, s);
        launch_copy(n, c->d_uC, dcol + (int64_t)q * n, s);
        launch_fill(1, 0.0, de + q, s);
    }
    HIPCHK(hipStreamSynchronize(s));
    std::vector<double> h((size_t)n * n);
    HIPCHK(hipMemcpy(h.data(), dcol, h.size() * sizeof(double), hipMemcpyDeviceToHost));
    dfree(c, dp); dfree(c, di); dfree(c, de); dfree(c, dcol);
    return upload_dense_coarse(c, h, true);
}

int setup_impl(bddc_ctx *c, const bddc_mesh *mesh, const bddc_partition *part, const double *coef) {
    Structure &st = c->st;
    std::string err;
    int rc = build_structure(mesh, part, coef, &c->opts, st, err);
    if (rc) return fail(rc, err);
    hipStream_t s = c->stream;
    // pure Neumann problem: no kept element touches a Dirichlet node
    if (mesh->node_dirichlet) {
        bool any = false;
        const int64_t n1x = mesh->nx + 1, n1y = mesh->ny + 1;
        for (int64_t e = 0; e < st.n_elem && !any; ++e) {
            if (mesh->elem_keep && !mesh->elem_keep[e]) continue;
            const int64_t ex = e % mesh->nx, ey = (e / mesh->nx) % mesh->ny, ez = e / ((int64_t)mesh->nx * mesh->ny);
            for (int v = 0; v < 8 && !any; ++v)
                any = mesh->node_dirichlet[(ex + (v & 1)) + n1x * ((ey + ((v >> 1) & 1)) + n1y * (ez + (v >> 2)))] != 0;
        }
        c->nullc = any ? 0 : 1;
    }
    {
        int dev = 0;
        HIPCHK(hipGetDevice(&dev));
        int ncu = 0;
        HIPCHK(hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev));
        c->n_cu = std::max(1, ncu);
        double *sp = nullptr;      // resolve this device's static scratch now
        if (int rc2 = noalloc_scratch(&sp, err)) return fail(rc2, err);
    }
    {
        const int nsub = st.n_sub;
        std::vector<int64_t> k_off(nsub + 1, 0);
        std::vector<int32_t> nI(nsub);
        int max_nloc = 0;
        for (int i = 0; i < nsub; ++i) {
            const SubHost &sh = st.sub[i];
            nI[i] = sh.nI;
            k_off[i + 1] = k_off[i] + (int64_t)sh.nloc * sh.nloc;
            max_nloc = std::max(max_nloc, sh.nloc);
        }
        // -------------------------------------------------- local assembly
        // K_i from the element matrices, then the interior elimination that
        // leaves S_i in the interface block (before the coarse DOFs are final:
        // adaptive face rows need S_i)
        std::vector<int32_t> eloc, incp, ince, incv;
        std::vector<double> ec;
        std::vector<int64_t> e_off(nsub + 1, 0), ip_off(nsub + 1, 0), ie_off(nsub + 1, 0);
        for (int i = 0; i < nsub; ++i) {
            const SubHost &sh = st.sub[i];
            e_off[i + 1] = e_off[i] + (int64_t)sh.elem.size();
            ip_off[i + 1] = ip_off[i] + sh.nloc + 1;
            ie_off[i + 1] = ie_off[i] + (int64_t)sh.inc_e.size();
            eloc.insert(eloc.end(), sh.elem_loc.begin(), sh.elem_loc.end());
            ec.insert(ec.end(), sh.elem_c.begin(), sh.elem_c.end());
            incp.insert(incp.end(), sh.inc_ptr.begin(), sh.inc_ptr.end());
            ince.insert(ince.end(), sh.inc_e.begin(), sh.inc_e.end());
            incv.insert(incv.end(), sh.inc_v.begin(), sh.inc_v.end());
        }
        int32_t *d_eloc, *d_incp, *d_ince, *d_incv;
        double *d_ec;
        if ((rc = dupload(c, &d_eloc, eloc)) || (rc = dupload(c, &d_ec, ec)) || (rc = dupload(c, &d_incp, incp)) ||
            (rc = dupload(c, &d_ince, ince)) || (rc = dupload(c, &d_incv, incv)))
            return rc;
        if ((rc = dalloc(c, &c->d_K, (size_t)k_off[nsub]))) return rc;
        if ((rc = dalloc(c, &c->d_status, 1))) return rc;
        HIPCHK(hipMemsetAsync(c->d_status, 0, sizeof(int32_t), s));
        {
            std::vector<AsmDesc> ad(nsub);
            for (int i = 0; i < nsub; ++i) {
                ad[i].elem_loc = d_eloc + e_off[i] * 8;
                ad[i].elem_c = d_ec + e_off[i];
                ad[i].inc_ptr = d_incp + ip_off[i];
                ad[i].inc_e = d_ince + ie_off[i];
                ad[i].inc_v = d_incv + ie_off[i];
                ad[i].nloc = st.sub[i].nloc;
                ad[i].K = c->d_K + k_off[i];
            }
            AsmDesc *dd;
            if ((rc = dupload(c, &dd, ad))) return rc;
            launch_assemble(dd, nsub, s);
            // interior elimination: sweep the interior pivots of every K_i
            std::vector<SweepDesc> sd(nsub);
            for (int i = 0; i < nsub; ++i)
                sd[i] = SweepDesc{c->d_K + k_off[i], st.sub[i].nloc, st.sub[i].nloc, 0, nI[i], st.sub[i].nloc};
            if ((rc = run_sweeps(c, sd))) return rc;
            dfree(c, dd);
        }
        dfree(c, d_eloc); dfree(c, d_incp); dfree(c, d_ince); dfree(c, d_incv);
        if (c->opts.adapt_tau > 0) {
            // Section 3.3: enrich the level-1 faces, then every later step
            // works with the enlarged coarse space
            std::vector<CoarseDof> extra;
            AdaptStats as;
            if ((rc = adaptive_faces(st, c->d_K, k_off, c->opts.adapt_tau, std::max(0, c->opts.adapt_max_per_face),
                                     c->opts.adapt_lobpcg_it,
                                     c->d_status, s, extra, as, err)))
                return fail(rc, err);
            if ((rc = add_coarse_dofs(st, part, extra, err))) return fail(rc, err);
            c->adapt = as;
        }
    }
    c->n_sub = st.n_sub;
    c->n_gamma = (int)st.gamma.size();
    c->nC = (int)st.coarse.size();
    c->n_nodes = st.n_nodes;
    c->prec = c->opts.local_prec;
    c->prec_built = (1 << prec_slot(c->prec)) | (c->opts.local_prec_set & 7);
    const int nsub = c->n_sub;
    const int eN = c->prec / 8;   // bytes per element of the local Neumann operators

    // -------------------------------------------------- level-1 metadata
    std::vector<int32_t> nI(nsub), nB(nsub), nc(nsub), i_off(nsub + 1, 0), b_off(nsub + 1, 0), c_off(nsub + 1, 0);
    std::vector<int64_t> k_off(nsub + 1, 0), s_off(nsub + 1, 0), kc_off(nsub + 1, 0),
        m_off(nsub + 1, 0), x_off(nsub + 1, 0), phr_off(nsub + 1, 0);
    std::vector<int32_t> gB, nodesI, cidx, pos_sub;
    for (int i = 0; i < nsub; ++i) {
        const SubHost &sh = st.sub[i];
        nI[i] = sh.nI; nB[i] = sh.nB; nc[i] = (int)sh.cidx.size();
        if (sh.nB == 0) return fail(BDDC_EINVAL, "subdomain " + std::to_string(i) + " has no interface");
        i_off[i + 1] = i_off[i] + sh.nI;
        b_off[i + 1] = b_off[i] + sh.nB;
        c_off[i + 1] = c_off[i] + nc[i];
        k_off[i + 1] = k_off[i] + (int64_t)sh.nloc * sh.nloc;
        s_off[i + 1] = s_off[i] + op_slots(sh.nB) * 256;
        kc_off[i + 1] = kc_off[i] + (int64_t)nc[i] * nc[i];
        m_off[i + 1] = m_off[i] + (int64_t)(sh.nB + nc[i]) * (sh.nB + nc[i]);
        x_off[i + 1] = x_off[i] + (int64_t)sh.nB * nc[i];
        phr_off[i + 1] = phr_off[i] + (int64_t)phi_ld(sh.nB) * nc[i];
        gB.insert(gB.end(), sh.gB.begin(), sh.gB.end());
        nodesI.insert(nodesI.end(), sh.nodes.begin(), sh.nodes.begin() + sh.nI);
        cidx.insert(cidx.end(), sh.cidx.begin(), sh.cidx.end());
        pos_sub.insert(pos_sub.end(), sh.nB, i);
        c->max_nI = std::max(c->max_nI, sh.nI);
        c->max_nB = std::max(c->max_nB, sh.nB);
        c->max_nc = std::max(c->max_nc, nc[i]);
        c->max_nt = std::max(c->max_nt, (sh.nB + TILE - 1) / TILE);
    }
    if (b_off[nsub] > INT32_MAX / 2) return fail(BDDC_EINVAL, "too many local interface entries");
    {   // prolongation blocks: 512 interface rows of one subdomain each
        std::vector<int32_t> ch_sub, ch_row;
        for (int i = 0; i < nsub; ++i)
            for (int r = 0; r == 0 || r < nB[i]; r += 512) { ch_sub.push_back(i); ch_row.push_back(r); }
        c->n_pch = (int)ch_sub.size();
        if ((rc = dupload(c, &c->d_pch_sub, ch_sub)) || (rc = dupload(c, &c->d_pch_row, ch_row))) return rc;
    }
    c->h_nB = nB; c->h_nI = nI; c->h_nc = nc; c->h_pos_sub = pos_sub;
    c->h_b_off.assign(b_off.begin(), b_off.end() - 1);
    c->h_c_off.assign(c_off.begin(), c_off.end() - 1);
    if ((rc = dupload(c, &c->d_nI, nI)) || (rc = dupload(c, &c->d_nB, nB)) || (rc = dupload(c, &c->d_nc, nc)) ||
        (rc = dupload(c, &c->d_i_off, i_off)) || (rc = dupload(c, &c->d_b_off, b_off)) ||
        (rc = dupload(c, &c->d_c_off, c_off)) || (rc = dupload(c, &c->d_k_off, k_off)) ||
        (rc = dupload(c, &c->d_s_off, s_off)) ||
        (rc = dupload(c, &c->d_phr_off, phr_off)) || (rc = dupload(c, &c->d_gB, gB)) ||
        (rc = dupload(c, &c->d_nodesI, nodesI)) || (rc = dupload(c, &c->d_cidx, cidx)) ||
        (rc = dupload(c, &c->d_gamma, st.gamma)) || (rc = dupload(c, &c->d_pos_sub, pos_sub)))
        return rc;
    // interface assembly lists (owner-computes, ordered by subdomain)
    {
        std::vector<std::pair<int64_t, int32_t>> pr;
        for (int i = 0; i < nsub; ++i)
            for (int k = 0; k < nB[i]; ++k) pr.push_back({st.sub[i].gB[k], b_off[i] + k});
        std::vector<int32_t> ptr, idx;
        build_csr(c->n_gamma, pr, ptr, idx);
        if ((rc = dupload(c, &c->d_asm_ptr, ptr)) || (rc = dupload(c, &c->d_asm_idx, idx))) return rc;
        c->h_asm_ptr = ptr; c->h_asm_idx = idx;
        pr.clear();
        for (int i = 0; i < nsub; ++i)
            for (int q = 0; q < nc[i]; ++q) pr.push_back({st.sub[i].cidx[q], c_off[i] + q});
        build_csr(c->nC, pr, ptr, idx);
        if ((rc = dupload(c, &c->d_casm_ptr, ptr)) || (rc = dupload(c, &c->d_casm_idx, idx))) return rc;
        c->h_casm_ptr = ptr; c->h_casm_idx = idx;
        if ((rc = dalloc(c, &c->d_crest, (size_t)std::max(1, c_off[nsub])))) return rc;
    }

    // -------------------------------------------------- constrained Neumann operators
    std::vector<int32_t> cptr, ccol;
    std::vector<double> cval, wB;
    std::vector<int64_t> cp_off(nsub + 1, 0), cc_off(nsub + 1, 0);
    for (int i = 0; i < nsub; ++i) {
        const SubHost &sh = st.sub[i];
        cp_off[i + 1] = cp_off[i] + (int64_t)sh.c_ptr.size();
        cc_off[i + 1] = cc_off[i] + (int64_t)sh.c_col.size();
        cptr.insert(cptr.end(), sh.c_ptr.begin(), sh.c_ptr.end());
        ccol.insert(ccol.end(), sh.c_col.begin(), sh.c_col.end());
        cval.insert(cval.end(), sh.c_val.begin(), sh.c_val.end());
        wB.insert(wB.end(), sh.wB.begin(), sh.wB.end());
    }
    int32_t *d_cptr, *d_ccol;
    double *d_cval, *d_wB, *d_M, *d_X;
    if ((rc = dupload(c, &d_cptr, cptr)) || (rc = dupload(c, &d_ccol, ccol)) || (rc = dupload(c, &d_cval, cval)) ||
        (rc = dupload(c, &d_wB, wB)) || (rc = dalloc(c, &d_M, (size_t)m_off[nsub])) ||
        (rc = dalloc(c, &d_X, (size_t)x_off[nsub])))
        return rc;
    {
        std::vector<SaddleDesc> sd(nsub);
        std::vector<SweepDesc> wd(nsub);
        for (int i = 0; i < nsub; ++i) {
            const int nl = st.sub[i].nloc, N = nB[i] + nc[i];
            sd[i] = SaddleDesc{c->d_K + k_off[i] + (int64_t)nI[i] * nl + nI[i], nl, nB[i], nc[i],
                               d_cptr + cp_off[i], d_ccol + cc_off[i], d_cval + cc_off[i], d_M + m_off[i], N};
            wd[i] = SweepDesc{d_M + m_off[i], N, N, 0, N, nB[i]};
        }
        SaddleDesc *dsd;
        if ((rc = dupload(c, &dsd, sd))) return rc;
        launch_build_saddle(dsd, nsub, s);
        if ((rc = run_sweeps(c, wd))) return rc;
        // tiles: S_i (float64) and D N_i D (local precision) in the same
        // layout, plus the column-major D Phi_i for the coarse restriction and
        // the prolongation
        c->bytes_S = (size_t)s_off[nsub] * 8;
        c->bytes_N = (size_t)s_off[nsub] * eN;
        if ((rc = dalloc_tiles(c, &c->d_S, (size_t)s_off[nsub]))) return rc;
        for (int p : {64, 32, 16}) {
            if (!((c->prec_built >> prec_slot(p)) & 1)) continue;
            const int e = p / 8, q = prec_slot(p);
            if ((rc = dalloc_tiles(c, (char **)&c->d_Nx[q], (size_t)s_off[nsub] * e)) ||
                (rc = dalloc(c, (char **)&c->d_phirx[q], (size_t)std::max<int64_t>(1, phr_off[nsub]) * e)))
                return rc;
        }
        c->d_N = c->d_Nx[prec_slot(c->prec)];
        c->d_phir = c->d_phirx[prec_slot(c->prec)];
        std::vector<PackDesc> ps(nsub), pn(nsub);
        std::vector<PtspDesc> pt(nsub);
        for (int i = 0; i < nsub; ++i) {
            const int nl = st.sub[i].nloc, N = nB[i] + nc[i];
            const double *Sblk = c->d_K + k_off[i] + (int64_t)nI[i] * nl + nI[i];
            ps[i] = PackDesc{Sblk, nl, nB[i], 1.0, nullptr, nullptr, 0, 0, s_off[i], -1};
            pn[i] = PackDesc{d_M + m_off[i], N, nB[i], -1.0, d_wB + b_off[i], d_M + m_off[i] + nB[i], N, nc[i], s_off[i],
                             phr_off[i]};
            pt[i] = PtspDesc{Sblk, nl, d_M + m_off[i] + nB[i], N, -1.0, nB[i], nc[i], d_X + x_off[i], nullptr};
        }
        if ((rc = dalloc(c, &c->d_KC, (size_t)std::max<int64_t>(1, kc_off[nsub])))) return rc;
        for (int i = 0; i < nsub; ++i) pt[i].out = c->d_KC + kc_off[i];
        PackDesc *dps, *dpn;
        PtspDesc *dpt;
        if ((rc = dupload(c, &dps, ps)) || (rc = dupload(c, &dpn, pn)) || (rc = dupload(c, &dpt, pt))) return rc;
        launch_pack(dps, nsub, 64, c->d_S, nullptr, s);
        for (int p : {64, 32, 16})   // each storage precision from the same float64 solves
            if ((c->prec_built >> prec_slot(p)) & 1) launch_pack(dpn, nsub, p, c->d_Nx[prec_slot(p)], c->d_phirx[prec_slot(p)], s);
        launch_ptsp(dpt, nsub, s);
        HIPCHK(hipStreamSynchronize(s));
        dfree(c, dsd); dfree(c, dps); dfree(c, dpn); dfree(c, dpt);
    }
    dfree(c, d_M); dfree(c, d_X); dfree(c, d_cptr); dfree(c, d_ccol); dfree(c, d_cval); dfree(c, d_wB);
    {
        int32_t st_h = 0;
        HIPCHK(hipMemcpy(&st_h, c->d_status, sizeof(int32_t), hipMemcpyDeviceToHost));
        if (st_h) return fail(BDDC_ESINGULAR, "non-positive pivot in a local elimination (floating subdomain without constraints?)");
    }
    if ((rc = setup_operators(c))) return rc;
    if ((rc = setup_interior(c, k_off))) return rc;
    dfree(c, c->d_K);   // the swept local matrices are not used after setup
    c->d_K = nullptr;

    // -------------------------------------------------- coarse levels
    c->three = st.three;
    if ((rc = dalloc(c, &c->d_uC, (size_t)std::max(1, c->nC)))) return rc;
    if (!c->three) {
        const int n = c->nC;
        if ((size_t)n * 8 > 160 * 1024) return fail(BDDC_EINVAL, "two-level coarse problem too large for the dense solve; use subregions");
        if ((size_t)n * 8 > 65536) return fail(BDDC_EINVAL, "two-level coarse problem above 8192 DOFs; use subregions");
        std::vector<std::pair<int64_t, int32_t>> pr;
        for (int i = 0; i < nsub; ++i)
            for (int a = 0; a < nc[i]; ++a)
                for (int b = 0; b < nc[i]; ++b)
                    pr.push_back({(int64_t)st.sub[i].cidx[a] * n + st.sub[i].cidx[b], (int32_t)(kc_off[i] + a * nc[i] + b)});
        std::vector<int32_t> ptr, idx;
        build_csr((int64_t)n * n, pr, ptr, idx);
        int32_t *dp, *di;
        if ((rc = dupload(c, &dp, ptr)) || (rc = dupload(c, &di, idx)) || (rc = dalloc(c, &c->d_KCinv, (size_t)std::max(1, n * n))))
            return rc;
        launch_gather_sum((int64_t)n * n, dp, di, c->d_KC, c->d_KCinv, s);
        if (n > 0 && c->nullc) {
            if ((rc = sweep_semidefinite(c, c->d_KCinv, n, n, coarse_null_vector(st)))) return rc;
        } else if (n > 0 && (rc = run_sweeps(c, {SweepDesc{c->d_KCinv, n, n, 0, n, n}}))) {
            return rc;
        }
        HIPCHK(hipStreamSynchronize(s));
        dfree(c, dp); dfree(c, di);
        if (n > 0) {
            std::vector<double> h((size_t)n * n);
            HIPCHK(hipMemcpy(h.data(), c->d_KCinv, h.size() * sizeof(double), hipMemcpyDeviceToHost));
            if ((rc = upload_dense_coarse(c, h, false))) return rc;
        }
        dfree(c, c->d_KCinv);
        c->d_KCinv = nullptr;
    } else {
        if (c->opts.adapt2_tau > 0 && (rc = adapt_level2(c, nc, kc_off))) return rc;
        const int nsr = st.n_sr;
        c->nsr = nsr;
        c->n3 = st.n3;
        if ((size_t)c->n3 * 8 > 65536) return fail(BDDC_EINVAL, "level-3 coarse problem above 8192 DOFs");
        std::vector<int32_t> nL(nsr), nI2(nsr), nc3(nsr), L_off(nsr + 1, 0), I2_off(nsr + 1, 0), B2_off(nsr + 1, 0),
            C3_off(nsr + 1, 0), Lall, g2all, c3all, pos_sr;
        std::vector<int64_t> K2_off(nsr + 1, 0), N2_off(nsr + 1, 0), P2_off(nsr + 1, 0), M2_off(nsr + 1, 0),
            K3_off(nsr + 1, 0);
        std::vector<double> w2all;
        for (int j = 0; j < nsr; ++j) {
            const SubregionHost &r = st.sr[j];
            nL[j] = (int)r.L.size(); nI2[j] = r.nI; nc3[j] = (int)r.c3.size();
            L_off[j + 1] = L_off[j] + nL[j];
            I2_off[j + 1] = I2_off[j] + r.nI;
            B2_off[j + 1] = B2_off[j] + r.nB;
            C3_off[j + 1] = C3_off[j] + nc3[j];
            K2_off[j + 1] = K2_off[j] + (int64_t)nL[j] * nL[j];
            N2_off[j + 1] = N2_off[j] + (int64_t)r.nB * r.nB;
            P2_off[j + 1] = P2_off[j] + (int64_t)r.nB * nc3[j];
            M2_off[j + 1] = M2_off[j] + (int64_t)(r.nB + nc3[j]) * (r.nB + nc3[j]);
            K3_off[j + 1] = K3_off[j] + (int64_t)nc3[j] * nc3[j];
            Lall.insert(Lall.end(), r.L.begin(), r.L.end());
            g2all.insert(g2all.end(), r.g2.begin(), r.g2.end());
            c3all.insert(c3all.end(), r.c3.begin(), r.c3.end());
            w2all.insert(w2all.end(), r.w.begin(), r.w.end());
            for (int k = 0; k < r.nB; ++k) pos_sr.push_back(j);
            c->max_nL = std::max(c->max_nL, nL[j]);
        }
        if ((size_t)c->max_nL * 8 > 65536) return fail(BDDC_EINVAL, "a subregion has too many coarse DOFs");
        {
            // per level-2 interface position: its D Phi row and level-3 DOF list
            std::vector<int64_t> ph_off2(B2_off[nsr]);
            std::vector<int32_t> c3o(B2_off[nsr]), n3p(B2_off[nsr]);
            for (int j = 0; j < nsr; ++j) {
                for (int k = 0; k < st.sr[j].nB; ++k) {
                    ph_off2[B2_off[j] + k] = P2_off[j] + (int64_t)k * nc3[j];
                    c3o[B2_off[j] + k] = C3_off[j];
                    n3p[B2_off[j] + k] = nc3[j];
                }
            }
            if ((rc = dupload(c, &c->d_ph_off2, ph_off2)) || (rc = dupload(c, &c->d_c3o, c3o)) ||
                (rc = dupload(c, &c->d_n3p, n3p)))
                return rc;
            c->smem_l2d = l2_d_smem(c->max_nL);
            if (set_l2_d_smem_limit(c->smem_l2d)) return fail(BDDC_EHIP, "hipFuncSetAttribute (dynamic LDS) failed");
        }
        if ((rc = dupload(c, &c->d_nL, nL)) || (rc = dupload(c, &c->d_nI2, nI2)) || (rc = dupload(c, &c->d_nc3, nc3)) ||
            (rc = dupload(c, &c->d_L_off, L_off)) || (rc = dupload(c, &c->d_I2_off, I2_off)) ||
            (rc = dupload(c, &c->d_B2_off, B2_off)) || (rc = dupload(c, &c->d_C3_off, C3_off)) ||
            (rc = dupload(c, &c->d_L, Lall)) || (rc = dupload(c, &c->d_g2, g2all)) || (rc = dupload(c, &c->d_c3, c3all)) ||
            (rc = dupload(c, &c->d_pos_sr, pos_sr)) || (rc = dupload(c, &c->d_K2_off, K2_off)) ||
            (rc = dupload(c, &c->d_N2_off, N2_off)) || (rc = dupload(c, &c->d_P2_off, P2_off)))
            return rc;
        // level-2 interface assembly lists, owners, level-3 lists
        {
            std::vector<std::pair<int64_t, int32_t>> pr;
            for (int j = 0; j < nsr; ++j)
                for (int k = 0; k < st.sr[j].nB; ++k) pr.push_back({st.sr[j].g2[k], B2_off[j] + k});
            std::vector<int32_t> ptr, idx;
            build_csr((int64_t)st.gamma2.size(), pr, ptr, idx);
            std::vector<uint8_t> own2(B2_off[nsr], 0);
            for (size_t gi = 0; gi + 1 < ptr.size(); ++gi)
                if (ptr[gi + 1] > ptr[gi]) own2[idx[ptr[gi]]] = 1;
            if ((rc = dupload(c, &c->d_asm2_ptr, ptr)) || (rc = dupload(c, &c->d_asm2_idx, idx)) ||
                (rc = dupload(c, &c->d_own2, own2)))
                return rc;
            pr.clear();
            for (int j = 0; j < nsr; ++j)
                for (int q = 0; q < nc3[j]; ++q) pr.push_back({st.sr[j].c3[q], C3_off[j] + q});
            build_csr(c->n3, pr, ptr, idx);
            if ((rc = dupload(c, &c->d_asm3_ptr, ptr)) || (rc = dupload(c, &c->d_asm3_idx, idx))) return rc;
        }
        // K2_j = sum over member subdomains of K_Ci (subdomains as elements)
        {
            std::vector<int32_t> ptr, idx;
            k2_csr(st, nc, kc_off, K2_off, ptr, idx);
            int32_t *dp, *di;
            if ((rc = dupload(c, &dp, ptr)) || (rc = dupload(c, &di, idx)) || (rc = dalloc(c, &c->d_K2, (size_t)K2_off[nsr])))
                return rc;
            launch_gather_sum(K2_off[nsr], dp, di, c->d_KC, c->d_K2, s);
            HIPCHK(hipStreamSynchronize(s));
            dfree(c, dp); dfree(c, di);
        }
        // sweep the level-2 interior pivots, then the level-2 saddle problems
        std::vector<int32_t> cptr2, ccol2;
        std::vector<double> cval2;
        std::vector<int64_t> cp2(nsr + 1, 0), cc2(nsr + 1, 0);
        for (int j = 0; j < nsr; ++j) {
            const SubregionHost &r = st.sr[j];
            cp2[j + 1] = cp2[j] + (int64_t)r.c_ptr.size();
            cc2[j + 1] = cc2[j] + (int64_t)r.c_col.size();
            cptr2.insert(cptr2.end(), r.c_ptr.begin(), r.c_ptr.end());
            ccol2.insert(ccol2.end(), r.c_col.begin(), r.c_col.end());
            cval2.insert(cval2.end(), r.c_val.begin(), r.c_val.end());
        }
        int32_t *d_cptr2, *d_ccol2;
        double *d_cval2, *d_w2, *d_M2, *d_X2, *d_K3loc;
        if ((rc = dupload(c, &d_cptr2, cptr2)) || (rc = dupload(c, &d_ccol2, ccol2)) || (rc = dupload(c, &d_cval2, cval2)) ||
            (rc = dupload(c, &d_w2, w2all)) || (rc = dalloc(c, &d_M2, (size_t)M2_off[nsr])) ||
            (rc = dalloc(c, &d_X2, (size_t)P2_off[nsr])) || (rc = dalloc(c, &d_K3loc, (size_t)K3_off[nsr])) ||
            (rc = dalloc(c, &c->d_N2, (size_t)N2_off[nsr])) || (rc = dalloc(c, &c->d_Phi2, (size_t)P2_off[nsr])))
            return rc;
        {
            std::vector<SweepDesc> s1(nsr), s2(nsr);
            std::vector<SaddleDesc> sd(nsr);
            std::vector<DenseCopyDesc> cn(nsr), cp(nsr);
            std::vector<PtspDesc> pt(nsr);
            for (int j = 0; j < nsr; ++j) {
                const int n = nL[j], i2 = nI2[j], b = n - i2, N = b + nc3[j];
                double *Kj = c->d_K2 + K2_off[j];
                const double *Sj = Kj + (int64_t)i2 * n + i2;
                s1[j] = SweepDesc{Kj, n, n, 0, i2, n};
                sd[j] = SaddleDesc{Sj, n, b, nc3[j], d_cptr2 + cp2[j], d_ccol2 + cc2[j], d_cval2 + cc2[j], d_M2 + M2_off[j], N};
                s2[j] = SweepDesc{d_M2 + M2_off[j], N, N, 0, N, b};
                cn[j] = DenseCopyDesc{d_M2 + M2_off[j], N, b, b, -1.0, d_w2 + B2_off[j], d_w2 + B2_off[j], c->d_N2 + N2_off[j], b};
                cp[j] = DenseCopyDesc{d_M2 + M2_off[j] + b, N, b, nc3[j], -1.0, d_w2 + B2_off[j], nullptr, c->d_Phi2 + P2_off[j], nc3[j]};
                pt[j] = PtspDesc{Sj, n, d_M2 + M2_off[j] + b, N, -1.0, b, nc3[j], d_X2 + P2_off[j], d_K3loc + K3_off[j]};
            }
            SaddleDesc *dsd;
            DenseCopyDesc *dcn, *dcp;
            PtspDesc *dpt;
            if ((rc = dupload(c, &dsd, sd)) || (rc = dupload(c, &dcn, cn)) || (rc = dupload(c, &dcp, cp)) ||
                (rc = dupload(c, &dpt, pt)))
                return rc;
            if ((rc = run_sweeps(c, s1))) return rc;
            launch_build_saddle(dsd, nsr, s);
            if ((rc = run_sweeps(c, s2))) return rc;
            launch_dense_copy(dcn, nsr, s);
            launch_dense_copy(dcp, nsr, s);
            launch_ptsp(dpt, nsr, s);
            HIPCHK(hipStreamSynchronize(s));
            dfree(c, dsd); dfree(c, dcn); dfree(c, dcp); dfree(c, dpt);
        }
        // level 3: assemble and invert (dense)
        {
            const int n = c->n3;
            const int ld = c->ld3 = (n + 1) & ~1;      // rows padded to an even length (zero)
            std::vector<std::pair<int64_t, int32_t>> pr;
            for (int j = 0; j < nsr; ++j)
                for (int a = 0; a < nc3[j]; ++a)
                    for (int b = 0; b < nc3[j]; ++b)
                        pr.push_back({(int64_t)st.sr[j].c3[a] * ld + st.sr[j].c3[b], (int32_t)(K3_off[j] + a * nc3[j] + b)});
            std::vector<int32_t> ptr, idx;
            build_csr((int64_t)n * ld, pr, ptr, idx);
            int32_t *dp, *di;
            if ((rc = dupload(c, &dp, ptr)) || (rc = dupload(c, &di, idx)) ||
                (rc = dalloc(c, &c->d_K3inv, (size_t)std::max<int64_t>(1, (int64_t)n * ld))) ||
                (rc = dalloc(c, &c->d_r3, (size_t)std::max(1, n))))
                return rc;
            launch_gather_sum((int64_t)n * ld, dp, di, d_K3loc, c->d_K3inv, s);
            if (n > 0 && c->nullc) {
                // the level-3 values of the constant: its level-1 values under the level-3 rows
                const std::vector<double> e1 = coarse_null_vector(st);
                std::vector<double> e3(n, 0.0);
                for (int m3 = 0; m3 < n; ++m3)
                    for (size_t q = 0; q < st.dof3_members[m3].size(); ++q)
                        e3[m3] += st.dof3_wts[m3][q] * e1[st.dof3_members[m3][q]];
                if ((rc = sweep_semidefinite(c, c->d_K3inv, n, ld, e3))) return rc;
            } else if (n > 0 && (rc = run_sweeps(c, {SweepDesc{c->d_K3inv, n, ld, 0, n, n}}))) {
                return rc;
            }
            // large levels: the upper triangle in 64 x 64 blocks for the
            // single-vector product (half the bytes per application)
            if (n >= 512) {
                const int nb = (n + 63) / 64;
                const int64_t nbt = (int64_t)nb * (nb + 1) / 2;
                std::vector<int32_t> bI;
                bI.reserve(nbt);
                for (int I = 0; I < nb; ++I)
                    for (int J = I; J < nb; ++J) bI.push_back(I);
                c->nb3 = nb;
                if ((rc = dupload(c, &c->d_K3bI, bI)) || (rc = dalloc(c, &c->d_K3s, (size_t)nbt * 4096)) ||
                    (rc = dalloc(c, &c->d_K3part, (size_t)nbt * 128)))
                    return rc;
                launch_pack_symblk(c->d_K3inv, ld, n, nb, c->d_K3bI, -1.0, c->d_K3s, s);
            }
            HIPCHK(hipStreamSynchronize(s));
            dfree(c, dp); dfree(c, di);
        }
        dfree(c, d_cptr2); dfree(c, d_ccol2); dfree(c, d_cval2); dfree(c, d_w2); dfree(c, d_M2); dfree(c, d_X2);
        dfree(c, d_K3loc);
        if ((rc = dalloc(c, &c->d_vI2, (size_t)I2_off[nsr])) || (rc = dalloc(c, &c->d_t2, (size_t)B2_off[nsr])) ||
            (rc = dalloc(c, &c->d_rB2, (size_t)B2_off[nsr])) || (rc = dalloc(c, &c->d_u2, (size_t)B2_off[nsr])) ||
            (rc = dalloc(c, &c->d_c3loc, (size_t)C3_off[nsr])) || (rc = dalloc(c, &c->d_u3, (size_t)std::max(1, c->n3))))
            return rc;
    }
    {
        int32_t st_h = 0;
        HIPCHK(hipMemcpy(&st_h, c->d_status, sizeof(int32_t), hipMemcpyDeviceToHost));
        if (st_h) return fail(BDDC_ESINGULAR, "non-positive pivot in a coarse-level elimination");
    }

    // -------------------------------------------------- iteration storage
    const int ng = c->n_gamma;
    c->ld = ng;
    c->R = c->opts.recycle_R;
    if (c->R + c->nullc > RMAX) return fail(BDDC_EINVAL, "recycle_R plus the constant column exceeds 64");
    c->kmax = kmax_bucket(c->R + c->nullc);
    c->save_cap = c->R > 0 ? c->opts.save_cap : 0;
    c->hist_cap = c->opts.max_it + 2;
    c->vgrid = std::max(1, std::min(VGRID, (ng + 255) / 256));
    const int gram_nb = std::max(1, std::min(512, (ng + 127) / 128));
    c->gram_nb = gram_nb;
    c->hcopy = std::min(c->hist_cap, c->save_cap + 2);
    if ((rc = dalloc(c, &c->d_b, ng)) || (rc = dalloc(c, &c->d_x, ng)) || (rc = dalloc(c, &c->d_r, ng)) ||
        (rc = dalloc(c, &c->d_z, ng)) || (rc = dalloc(c, &c->d_p, ng)) || (rc = dalloc(c, &c->d_tmp, ng)) ||
        (rc = dalloc(c, &c->d_locq, (size_t)b_off[nsub])) || (rc = dalloc(c, &c->d_wloc, (size_t)b_off[nsub])) ||
        (rc = dalloc(c, &c->d_rr, (size_t)c->vgrid)) || (rc = dalloc(c, &c->d_bbp, (size_t)c->vgrid)) ||
        (rc = dalloc(c, &c->d_zp, (size_t)c->vgrid * (RMAX + 1))) ||
        (rc = dalloc(c, &c->d_wp, (size_t)c->vgrid * (RMAX + 1))) ||
        (rc = dalloc(c, &c->d_gp, (size_t)gram_nb * RMAX * RMAX)) ||
        (rc = dalloc(c, &c->d_sync, 1)) || (rc = dalloc(c, &c->d_hblk, (size_t)c->hist_cap * (3 + RMAX))) ||
        (rc = dalloc(c, &c->d_bhist, c->hist_cap)) || (rc = dalloc(c, &c->d_reshist, c->hist_cap)) ||
        (rc = dalloc(c, &c->d_WAWinv, RMAX * RMAX)) || (rc = dalloc(c, &c->d_WAWnew, RMAX * RMAX)) ||
        (rc = dalloc(c, &c->d_invnew, RMAX * RMAX)) ||
        (rc = dalloc(c, &c->d_WWinv, RMAX * RMAX)) || (rc = dalloc(c, &c->d_WWnew, RMAX * RMAX)) ||
        (rc = dalloc(c, &c->d_WWsym, RMAX * RMAX)) || (rc = dalloc(c, &c->d_WWinvnew, RMAX * RMAX)) ||
        (rc = dalloc(c, &c->d_rop, (size_t)RMAX * VGRID)) || (rc = dalloc(c, &c->d_state2, 1)))
        return rc;
    // control block, deflation state and W^T A W of a pending update side by
    // side (the layout of the pinned SyncBuf: one copy per synchronisation);
    // alpha, d, rho and mu histories in one block of the pinned h_hist layout
    c->d_ctl = &c->d_sync->ctl;
    c->d_state = &c->d_sync->rs;
    c->d_WAWsym = c->d_sync->waw;
    c->d_ahist = c->d_hblk;
    c->d_dhist = c->d_hblk + c->hist_cap;
    c->d_rhohist = c->d_hblk + 2 * (size_t)c->hist_cap;
    c->d_muhist = c->d_hblk + 3 * (size_t)c->hist_cap;
    HIPCHK(hipMemsetAsync(c->d_x, 0, ng * sizeof(double), s));
    HIPCHK(hipMemsetAsync(c->d_p, 0, ng * sizeof(double), s));
    HIPCHK(hipMemsetAsync(c->d_ctl, 0, sizeof(Ctl), s));
    HIPCHK(hipMemsetAsync(c->d_state, 0, sizeof(RecState), s));
    HIPCHK(hipHostMalloc((void **)&c->h_ctl, sizeof(Ctl), hipHostMallocDefault));
    HIPCHK(hipHostMalloc((void **)&c->h_sync, sizeof(SyncBuf), hipHostMallocDefault));
    HIPCHK(hipHostMalloc((void **)&c->h_hist, sizeof(double) * (size_t)c->hist_cap * (3 + RMAX), hipHostMallocDefault));
    HIPCHK(hipHostMalloc((void **)&c->h_flags, sizeof(int32_t) * 4, hipHostMallocMapped));
    HIPCHK(hipHostGetDevicePointer((void **)&c->d_hflag, c->h_flags, 0));
    c->h_flags[0] = 0;
    HIPCHK(hipHostMalloc((void **)&c->h_prog, sizeof(double) * 4, hipHostMallocMapped));
    HIPCHK(hipHostGetDevicePointer((void **)&c->d_hprog, c->h_prog, 0));
    for (int q = 0; q < 4; ++q) c->h_prog[q] = 0.0;
    {
        // W, AW always exist (k = 0 columns are never read); the recycling
        // buffers only with R > 0
        const size_t cols = (size_t)std::max(1, c->R + c->nullc);
        // (+ RMAX: the recycling product reads up to 64 entries past a row)
        const int ymax = std::max((c->R + c->save_cap) * ((c->R + 7) / 8 * 8), RMAX * RMAX) + RMAX;
        if ((rc = dalloc(c, &c->d_W, cols * ng)) || (rc = dalloc(c, &c->d_AW, cols * ng)) ||
            (rc = dalloc(c, &c->d_Y, (size_t)ymax)))
            return rc;
        HIPCHK(hipHostMalloc((void **)&c->h_Y, sizeof(double) * (size_t)ymax, hipHostMallocDefault));
        if (c->R > 0 && ((rc = dalloc(c, &c->d_P, (size_t)std::max(1, c->save_cap) * ng)) ||
                         (rc = dalloc(c, &c->d_AP, (size_t)std::max(1, c->save_cap) * ng))))
            return rc;
    }
    // coarse form: one dense product for two levels; for three levels the
    // explicit operator when the coarse space is small enough (option)
    c->coarse_dense = !c->three;
    if (c->three && c->nC > 0) {
        const int form = c->opts.coarse_form;
        if (form < 0 || form > 2) return fail(BDDC_EINVAL, "coarse_form must be 0, 1 or 2");
        if (form == 2 && c->nC > 8192) return fail(BDDC_EINVAL, "explicit coarse operator above 8192 DOFs");
        if (form == 2 || (form == 0 && c->nC <= 4096)) {
            if ((rc = build_explicit_coarse(c))) return rc;
            c->coarse_dense = true;
        }
    }
    init_null_column(c);
    if (c->opts.autotune && (rc = tune_operators(c))) return rc;
    {   // pinned configurations
        OpHost *ops[2] = {&c->opS, &c->opN};
        for (int w = 0; w < 2; ++w) {
            const int32_t *pc = c->opts.product_cfg + 4 * w;
            if (pc[0] <= 0) continue;
            if ((pc[2] != 4 && pc[2] != 8) || (pc[3] != 2 && pc[3] != 4) || (pc[2] == 8 && !c->allow8))
                return fail(BDDC_EINVAL, "product_cfg: waves must be 4 or 8 (8 when it fits), tiles in flight 2 or 4");
            OpHost &op = *ops[w];
            op.bpc = pc[0];
            op.per_sub = pc[1] != 0;
            op.cfg = SymvCfg{pc[2], pc[3]};
            op.smem = symv_smem(op.prec, op.cfg.nw, c->max_nt);
            op.tuned_us = 0.f;
            if ((rc = build_worklist(c, op, product_blocks(c, op.n_tiles, op.bpc), op.per_sub))) return rc;
        }
    }
    if ((rc = dalloc(c, &c->d_dotS, (size_t)std::max(1, c->opS.dev.n_blocks)))) return rc;
    HIPCHK(hipStreamCreateWithFlags(&c->cap_stream, hipStreamNonBlocking));
    for (auto &e : c->gev) HIPCHK(hipEventCreateWithFlags(&e, hipEventDisableTiming));
    HIPCHK(hipEventCreateWithFlags(&c->sync_ev, hipEventDisableTiming));
    // element data for the adjoint gradient
    {
        std::vector<double> ch(st.n_elem, 0.0);
        std::vector<uint8_t> keep(st.n_elem, 1);
        for (int64_t e = 0; e < st.n_elem; ++e) {
            const bool kept = !mesh->elem_keep || mesh->elem_keep[e];
            ch[e] = kept ? coef[e] * st.h : 0.0;
            keep[e] = kept ? 1 : 0;
        }
        if ((rc = dupload(c, &c->d_coefh, ch)) || (rc = dupload(c, &c->d_keep, keep)) ||
            (rc = dupload(c, &c->d_free, st.free_node)))
            return rc;
    }
    HIPCHK(hipStreamSynchronize(s));
    return 0;
}

// ------------------------------------------------------------- block adjoint
// The adjoint systems of a sequence solved together: block deflated PCG in
// the breakdown-free form (an orthonormal search block P whose dependent
// directions are dropped), every direction A-orthogonal to W as in
// Algorithm 1.  The n x s block products (Schur, Neumann with the coarse
// rows) read every tile once for 16 columns (k_symm); the coarse levels, the
// prolongation and the assembly run on the single-vector kernels with one
// grid row per column; the s x s algebra is on the host (three
// synchronisations per iteration).
constexpr int BMAX = 32;            // columns of one block solve

struct BlockWork {
    BlockItem *items = nullptr;     // one per subdomain (the Schur and Neumann tiles share the layout)
    int32_t *ones = nullptr;
    double *B = nullptr, *X = nullptr, *R = nullptr, *Z = nullptr, *P = nullptr, *Q = nullptr;
    double *yS = nullptr, *yN = nullptr, *cN = nullptr, *gp = nullptr, *gout = nullptr, *coef = nullptr;
    double *h = nullptr;             // pinned: 4 Gram results, then 6 coefficient slots
    // per-column buffers of the coarse levels and the prolongation
    double *rC = nullptr, *uC = nullptr, *wloc = nullptr, *vI2 = nullptr, *t2 = nullptr, *rB2 = nullptr,
           *u2 = nullptr, *c3loc = nullptr, *u3 = nullptr, *r3 = nullptr;
    int64_t i2len = 1, b2len = 1, c3len = 1, n3len = 1, nclen = 1;
    int64_t ylen = 0, clen = 0;
    size_t smem = 0;
    static constexpr int GSZ = 64 * 64, CSZ = 96 * 64;
};

void free_block(bddc_ctx *c, BlockWork &b) {
    dfree(c, b.items); dfree(c, b.ones);
    dfree(c, b.B); dfree(c, b.X); dfree(c, b.R); dfree(c, b.Z); dfree(c, b.P); dfree(c, b.Q);
    dfree(c, b.yS); dfree(c, b.yN); dfree(c, b.cN); dfree(c, b.gp); dfree(c, b.gout); dfree(c, b.coef);
    dfree(c, b.rC); dfree(c, b.uC); dfree(c, b.wloc); dfree(c, b.vI2); dfree(c, b.t2); dfree(c, b.rB2);
    dfree(c, b.u2); dfree(c, b.c3loc); dfree(c, b.u3); dfree(c, b.r3);
    if (b.h) (void)hipHostFree(b.h);
    b = BlockWork{};
}

int alloc_block(bddc_ctx *c, BlockWork &b) {
    const int nsub = c->n_sub;
    std::vector<BlockItem> is(nsub);
    int64_t ts = 0;
    for (int i = 0; i < nsub; ++i) {
        is[i] = BlockItem{ts, c->h_nB[i], c->h_b_off[i]};
        ts += op_slots(c->h_nB[i]);
    }
    b.ylen = std::max<int64_t>(1, (int64_t)c->h_b_off[nsub - 1] + c->h_nB[nsub - 1]);
    b.clen = std::max<int64_t>(1, (int64_t)c->h_c_off[nsub - 1] + c->h_nc[nsub - 1]);
    const size_t nv = (size_t)c->ld * BMAX;
    int rc;
    std::vector<int32_t> ones(nsub, 1);
    if ((rc = dupload(c, &b.items, is)) || (rc = dupload(c, &b.ones, ones)) ||
        (rc = dalloc(c, &b.B, nv)) || (rc = dalloc(c, &b.X, nv)) || (rc = dalloc(c, &b.R, nv)) ||
        (rc = dalloc(c, &b.Z, nv)) || (rc = dalloc(c, &b.P, nv)) || (rc = dalloc(c, &b.Q, nv)) ||
        (rc = dalloc(c, &b.yS, (size_t)b.ylen * BMAX)) || (rc = dalloc(c, &b.yN, (size_t)b.ylen * BMAX)) ||
        (rc = dalloc(c, &b.cN, (size_t)b.clen * BMAX)) ||
        (rc = dalloc(c, &b.gp, (size_t)c->gram_nb * BlockWork::GSZ)) ||
        (rc = dalloc(c, &b.gout, (size_t)4 * BlockWork::GSZ)) || (rc = dalloc(c, &b.coef, (size_t)6 * BlockWork::CSZ)))
        return rc;
    if (hipHostMalloc((void **)&b.h, sizeof(double) * (4 * BlockWork::GSZ + 6 * BlockWork::CSZ)) != hipSuccess)
        return fail(BDDC_ENOMEM, "hipHostMalloc failed (block adjoint)");
    b.nclen = std::max(1, c->nC);
    if (c->three) {
        int64_t i2 = 0, b2 = 0, c3 = 0;
        for (const SubregionHost &r : c->st.sr) { i2 += r.nI; b2 += r.nB; c3 += (int64_t)r.c3.size(); }
        b.i2len = std::max<int64_t>(1, i2);
        b.b2len = std::max<int64_t>(1, b2);
        b.c3len = std::max<int64_t>(1, c3);
        b.n3len = std::max(1, c->n3);
    }
    if ((rc = dalloc(c, &b.rC, (size_t)b.nclen * BMAX)) || (rc = dalloc(c, &b.uC, (size_t)b.nclen * BMAX)) ||
        (rc = dalloc(c, &b.wloc, (size_t)b.ylen * BMAX)) || (rc = dalloc(c, &b.vI2, (size_t)b.i2len * BMAX)) ||
        (rc = dalloc(c, &b.t2, (size_t)b.b2len * BMAX)) || (rc = dalloc(c, &b.rB2, (size_t)b.b2len * BMAX)) ||
        (rc = dalloc(c, &b.u2, (size_t)b.b2len * BMAX)) || (rc = dalloc(c, &b.c3loc, (size_t)b.c3len * BMAX)) ||
        (rc = dalloc(c, &b.u3, (size_t)b.n3len * BMAX)) || (rc = dalloc(c, &b.r3, (size_t)b.n3len * BMAX)))
        return rc;
    // partial slots that no kernel writes (none with one chunk per subdomain) stay zero
    launch_fill((int64_t)b.ylen * BMAX, 0.0, b.yN, c->stream);
    launch_fill((int64_t)b.clen * BMAX, 0.0, b.cN, c->stream);
    b.smem = symm_smem_bytes(c->max_nB);
    return 0;
}

// X^T Y (kx x ky, row-major) into Gram slot `slot` (device), copy to the
// pinned host slot; the caller synchronises.
void block_gram(bddc_ctx *c, BlockWork &b, const double *X, int kx, const double *Y, int ky, int slot) {
    if (kx <= 0 || ky <= 0) return;
    GramArgs g{};
    g.n = c->n_gamma; g.k = kx; g.k2 = ky; g.ld = c->ld; g.X = X; g.Y = Y; g.part = b.gp;
    launch_gram(g, c->gram_nb, c->stream);
    ReduceArgs r{};
    r.part = b.gp; r.n = c->gram_nb; r.ncol = kx * ky; r.out = b.gout + (size_t)slot * BlockWork::GSZ;
    launch_reduce(r, c->stream);
    (void)hipMemcpyAsync(b.h + (size_t)slot * BlockWork::GSZ, r.out, sizeof(double) * kx * ky, hipMemcpyDeviceToHost,
                         c->stream);
}

// out = [V1, V2] Y (Y: (k1 + k2) x ncol row-major, host, coefficient slot
// `slot`); out may be V1 (each wave reads its rows before writing them).
int block_gemm(bddc_ctx *c, BlockWork &b, const double *V1, int k1, const double *V2, int k2,
               const std::vector<double> &Y, int ncol, double *out, int slot) {
    if (ncol <= 0) return 0;
    double *hy = b.h + 4 * BlockWork::GSZ + (size_t)slot * BlockWork::CSZ;
    double *dy = b.coef + (size_t)slot * BlockWork::CSZ;
    std::copy(Y.begin(), Y.end(), hy);
    HIPCHK(hipMemcpyAsync(dy, hy, sizeof(double) * Y.size(), hipMemcpyHostToDevice, c->stream));
    GemmArgs g{};
    g.n = c->n_gamma; g.ld = c->ld;
    g.V1[0] = V1; g.k1 = k1; g.V2[0] = V2 ? V2 : V1; g.k2 = k2;
    g.Y = dy; g.ncol = ncol; g.ldy = ncol; g.out[0] = out;
    launch_recycle_gemm(g, c->stream, 1);
    return 0;
}

void block_A(bddc_ctx *c, BlockWork &b, const double *X, int ncols, double *out) {
    TScope ts(c, TK_SCHUR);
    BlockSymvArgs a{};
    a.tiles = c->d_S; a.items = b.items; a.gB = c->d_gB; a.X = X; a.ldx = c->ld; a.ncols = ncols;
    a.ypart = b.yS; a.ylen = b.ylen;
    launch_symm(a, c->n_sub, b.smem, c->stream);
    launch_gather_block(c->n_gamma, c->d_asm_ptr, c->d_asm_idx, b.yS, b.ylen, out, c->ld, ncols, c->stream);
}

// The coarse levels of block_M on stream st: restriction of all columns,
// then the coarse problems (one grid row per column).
void block_coarse(bddc_ctx *c, BlockWork &b, const double *R, int ncols, hipStream_t st) {
    TScope ts(c, TK_COARSE);
    CrestArgs ra{};
    ra.ctl = c->d_ctl;
    ra.nB = c->d_nB; ra.b_off = c->d_b_off; ra.gB = c->d_gB; ra.nc = c->d_nc; ra.c_off = c->d_c_off;
    ra.phir = c->d_phirx[prec_slot(64)]; ra.phr_off = c->d_phr_off;
    ra.X = R; ra.ldx = c->ld; ra.part = b.cN; ra.cs = b.clen; ra.ncols = ncols;
    ra.cols = crest_cols(64, c->max_nB, ncols);
    launch_crest(ra, 64, c->n_sub, c->max_nB, st);
    const Gather rc{c->d_casm_ptr, c->d_casm_idx, b.cN};
    if (c->coarse_dense) {
        CoarseDenseArgs ca{};
        ca.ctl = c->d_ctl; ca.n = c->nC; ca.rc = rc; ca.r = b.rC; ca.M = c->d_Mc; ca.ldm = c->ldm;
        ca.sign = c->three ? 1.0 : -1.0; ca.u = b.uC;
        ca.cs_rc = b.clen; ca.cs_r = b.nclen; ca.cs_u = b.nclen;
        launch_coarse_dense(ca, st, ncols);
    } else {
        L2Args l = l2_args(c, rc);
        l.vI2 = b.vI2; l.t2 = b.t2; l.rB2 = b.rB2; l.u2 = b.u2; l.c3loc = b.c3loc; l.u3 = b.u3; l.uC = b.uC;
        l.cs_rc = b.clen; l.cs_vI2 = b.i2len; l.cs_t2 = b.b2len; l.cs_rB2 = b.b2len; l.cs_u2 = b.b2len;
        l.cs_c3loc = b.c3len; l.cs_u3 = b.n3len; l.cs_uC = b.nclen;
        launch_l2_a(l, c->nsr, c->max_nL, st, ncols);
        launch_l2_b(l, c->nsr, c->max_nL, st, ncols);
        CoarseDenseArgs l3{};
        l3.ctl = c->d_ctl; l3.n = c->n3; l3.rc = Gather{c->d_asm3_ptr, c->d_asm3_idx, b.c3loc}; l3.r = b.r3;
        l3.M = c->d_K3inv; l3.ldm = c->ld3; l3.sign = -1.0; l3.u = b.u3;
        l3.cs_rc = b.c3len; l3.cs_r = b.n3len; l3.cs_u = b.n3len;
        launch_coarse_dense(l3, st, ncols);
        launch_l2_d(l, c->nsr, c->smem_l2d, st, ncols);
    }
}

// BDDC on ncols columns of R (stride ld) into Z: the block products of the
// float64 Neumann operators, then the coarse levels, prolongation and
// assembly with the single-vector kernels, one grid row per column.
void block_M(bddc_ctx *c, BlockWork &b, const double *R, int ncols, double *Z) {
    {
        TScope ts(c, TK_PREC);
        BlockSymvArgs a{};
        a.tiles = (const double *)c->d_Nx[prec_slot(64)]; a.items = b.items; a.gB = c->d_gB; a.X = R; a.ldx = c->ld;
        a.ncols = ncols; a.ypart = b.yN; a.ylen = b.ylen;
        launch_symm(a, c->n_sub, b.smem, c->stream);
    }
    if (c->nC > 0) block_coarse(c, b, R, ncols, c->stream);
    TScope ts(c, TK_VEC);
    ProlArgs pa{};
    pa.ctl = c->d_ctl; pa.gated = 0;
    pa.nB = c->d_nB; pa.b_off = c->d_b_off; pa.nc = c->d_nc; pa.c_off = c->d_c_off; pa.cidx = c->d_cidx;
    pa.nchunk = b.ones; pa.pb = c->d_b_off; pa.upart = b.yN;
    pa.phir = c->d_phirx[prec_slot(64)]; pa.phr_off = c->d_phr_off;
    pa.uC = c->nC > 0 ? b.uC : nullptr;
    pa.wloc = b.wloc;
    pa.ch_sub = c->d_pch_sub; pa.ch_row = c->d_pch_row;
    pa.cs_u = b.ylen; pa.cs_uC = b.nclen; pa.cs_w = b.ylen;
    launch_prolong(pa, 64, c->n_pch, c->max_nc, c->stream, ncols);
    ZasmArgs za{};
    za.n = c->n_gamma;
    za.w = Gather{c->d_asm_ptr, c->d_asm_idx, b.wloc};
    za.r = R; za.z = Z; za.AW = c->d_AW; za.ld = c->ld; za.part = nullptr;
    za.ctl = c->d_ctl; za.gated = 0; za.advance = 0;
    za.cs_w = b.ylen; za.cs_r = c->ld; za.cs_z = c->ld;
    launch_zasm(za, c->kmax, c->vgrid, c->stream, ncols);
}

// X = G^{-1} Bm for a k x k SPD G (row-major) and k x m Bm; false if G is not SPD
bool spd_solve(std::vector<double> G, int k, const double *Bm, int m, std::vector<double> &X) {
    X.assign((size_t)k * m, 0.0);
    if (k == 0) return true;
    for (int i = 0; i < k; ++i)
        for (int j = i + 1; j < k; ++j) G[(size_t)i * k + j] = G[(size_t)j * k + i] = 0.5 * (G[(size_t)i * k + j] + G[(size_t)j * k + i]);
    if (!cholesky(G, k)) return false;
    std::vector<double> col(k);
    for (int j = 0; j < m; ++j) {
        for (int i = 0; i < k; ++i) col[i] = Bm[(size_t)i * m + j];
        chol_solve(G, k, col.data());
        for (int i = 0; i < k; ++i) X[(size_t)i * m + j] = col[i];
    }
    return true;
}

// [I; C] as a (k + r) x k coefficient matrix (identity on the first block)
std::vector<double> stack_identity(int k, const std::vector<double> &C, int r, double sign) {
    std::vector<double> Y((size_t)(k + r) * k, 0.0);
    for (int i = 0; i < k; ++i) Y[(size_t)i * k + i] = 1.0;
    for (int q = 0; q < r; ++q)
        for (int j = 0; j < k; ++j) Y[(size_t)(k + q) * k + j] = sign * C[(size_t)q * k + j];
    return Y;
}



int block_solve(bddc_ctx *c, BlockWork &b, int s, double rtol, int *iters_out) {
    const int m = c->k;                               // deflation columns (the current basis)
    const int ld = c->ld;
    std::vector<double> WAW(c->WAW.begin(), c->WAW.end()), T, Cm;
    int rc;
    // X_0 = W (W^T A W)^{-1} W^T B, R_0 = B - A W (...)
    launch_fill((int64_t)ld * s, 0.0, b.X, c->stream);
    launch_copy((int64_t)ld * s, b.B, b.R, c->stream);
    block_gram(c, b, b.B, s, b.B, s, 0);
    if (m > 0) block_gram(c, b, c->d_W, m, b.B, s, 1);
    HIPCHK(hipStreamSynchronize(c->stream));
    std::vector<double> bb(s), r0(s);
    for (int j = 0; j < s; ++j) bb[j] = b.h[(size_t)j * s + j];
    if (m > 0) {
        if (!spd_solve(WAW, m, b.h + BlockWork::GSZ, s, T)) return fail(BDDC_EBREAKDOWN, "W^T A W not positive definite");
        if ((rc = block_gemm(c, b, c->d_W, m, nullptr, 0, T, s, b.X, 0))) return rc;
        std::vector<double> Y = stack_identity(s, T, m, -1.0);
        if ((rc = block_gemm(c, b, b.R, s, c->d_AW, m, Y, s, b.R, 1))) return rc;
    }
    int r = 0, it = 0;                                // columns of P
    const int stop_r0 = c->opts.stop_rule == 1;
    std::vector<double> Gpq;
    for (;;) {
        // residual norms, Z = M^{-1} R and its products with Q and A W
        block_gram(c, b, b.R, s, b.R, s, 0);
        block_M(c, b, b.R, s, b.Z);
        if (m > 0) block_gram(c, b, c->d_AW, m, b.Z, s, 1);
        if (r > 0) block_gram(c, b, b.Q, r, b.Z, s, 2);
        HIPCHK(hipStreamSynchronize(c->stream));
        bool done = true;
        for (int j = 0; j < s; ++j) {
            const double rr = b.h[(size_t)j * s + j];
            if (it == 0) r0[j] = rr;
            const double den = stop_r0 ? r0[j] : bb[j];
            if (!(rr <= rtol * rtol * den)) done = false;
            if (!std::isfinite(rr)) return fail(BDDC_EBREAKDOWN, "block PCG: non-finite residual");
        }
        if (done) break;
        if (it >= c->opts.max_it) { *iters_out = it; return fail(BDDC_ENOTCONV, "max_it reached (block adjoint)"); }
        // Y = Z - W (W^T A W)^{-1} (A W)^T Z - P (P^T Q)^{-1} Q^T Z
        if (m > 0) {
            if (!spd_solve(WAW, m, b.h + BlockWork::GSZ, s, T)) return fail(BDDC_EBREAKDOWN, "W^T A W not positive definite");
            if ((rc = block_gemm(c, b, b.Z, s, c->d_W, m, stack_identity(s, T, m, -1.0), s, b.Z, 0))) return rc;
        }
        if (r > 0) {
            if (!spd_solve(Gpq, r, b.h + 2 * BlockWork::GSZ, s, T)) return fail(BDDC_EBREAKDOWN, "P^T A P not positive definite");
            if ((rc = block_gemm(c, b, b.Z, s, b.P, r, stack_identity(s, T, r, -1.0), s, b.Z, 1))) return rc;
        }
        // P = orth(Y): eigenvectors of Y^T Y above 1e-12 of the largest eigenvalue
        block_gram(c, b, b.Z, s, b.Z, s, 3);
        HIPCHK(hipStreamSynchronize(c->stream));
        {
            std::vector<double> G(b.h + 3 * BlockWork::GSZ, b.h + 3 * BlockWork::GSZ + (size_t)s * s), lam, V;
            for (int i = 0; i < s; ++i)
                for (int j = i + 1; j < s; ++j) G[(size_t)i * s + j] = G[(size_t)j * s + i] = 0.5 * (G[(size_t)i * s + j] + G[(size_t)j * s + i]);
            sym_eig(G, s, lam, V);
            const double top = lam.empty() ? 0.0 : lam[s - 1];
            std::vector<int> keep;
            for (int q = 0; q < s; ++q)
                if (top > 0.0 && lam[q] > 1e-12 * top) keep.push_back(q);
            r = (int)keep.size();
            if (r == 0) { *iters_out = it; return fail(BDDC_EBREAKDOWN, "block PCG: empty search block"); }
            Cm.assign((size_t)s * r, 0.0);
            for (int i = 0; i < s; ++i)
                for (int q = 0; q < r; ++q) Cm[(size_t)i * r + q] = V[(size_t)i * s + keep[q]] / std::sqrt(lam[keep[q]]);
        }
        if ((rc = block_gemm(c, b, b.Z, s, nullptr, 0, Cm, r, b.P, 2))) return rc;
        // Q = A P; alpha = (P^T Q)^{-1} P^T R
        block_A(c, b, b.P, r, b.Q);
        block_gram(c, b, b.P, r, b.Q, r, 0);
        block_gram(c, b, b.P, r, b.R, s, 1);
        HIPCHK(hipStreamSynchronize(c->stream));
        Gpq.assign(b.h, b.h + (size_t)r * r);
        std::vector<double> alpha;
        if (!spd_solve(Gpq, r, b.h + BlockWork::GSZ, s, alpha)) return fail(BDDC_EBREAKDOWN, "P^T A P not positive definite");
        if ((rc = block_gemm(c, b, b.X, s, b.P, r, stack_identity(s, alpha, r, 1.0), s, b.X, 3)) ||
            (rc = block_gemm(c, b, b.R, s, b.Q, r, stack_identity(s, alpha, r, -1.0), s, b.R, 4)))
            return rc;
        ++it;
    }
    *iters_out = it;
    return 0;
}

}  // namespace

extern "C" {

int bddc_setup(const bddc_mesh *mesh, const bddc_partition *part, const double *coef, const bddc_opts *opts,
               void *hip_stream, bddc_ctx **out) {
    if (!mesh || !part || !coef || !out) return fail(BDDC_EINVAL, "null argument");
    *out = nullptr;
    bddc_ctx *c = new bddc_ctx();
    c->stream = (hipStream_t)hip_stream;
    if (opts) c->opts = *opts;
    else bddc_default_opts(&c->opts);
    const bddc_opts &o = c->opts;
    if (o.local_prec != 64 && o.local_prec != 32 && o.local_prec != 16) { delete c; return fail(BDDC_EINVAL, "local_prec must be 64, 32 or 16"); }
    if (o.recycle_R < 0 || o.recycle_R > RMAX) { delete c; return fail(BDDC_EINVAL, "recycle_R out of range [0, 64]"); }
    if (o.recycle_strategy < 1 || o.recycle_strategy > 4) { delete c; return fail(BDDC_EINVAL, "recycle_strategy must be 1..4"); }
    if (o.max_it <= 0 || o.max_it > 100000 || o.save_cap < 0 || o.save_cap > 4096) { delete c; return fail(BDDC_EINVAL, "bad max_it or save_cap"); }
    if (o.use_graph < 0 || o.use_graph > 2) { delete c; return fail(BDDC_EINVAL, "use_graph must be 0, 1 or 2"); }
    if (!(o.constraints & (BDDC_CORNERS | BDDC_FACES | BDDC_EDGES))) { delete c; return fail(BDDC_EINVAL, "no constraints"); }
    if (mesh->nx <= 0 || mesh->ny <= 0 || mesh->nz <= 0) { delete c; return fail(BDDC_EINVAL, "mesh sizes must be positive"); }
    // element coefficients on the host (copied from device memory when given
    // there), as c_e = exp(theta_e) when they are log-coefficients
    const int64_t n_elem = (int64_t)mesh->nx * mesh->ny * mesh->nz;
    std::vector<double> coef_h((size_t)n_elem);
    {
        hipPointerAttribute_t attr{};
        const bool on_device = hipPointerGetAttributes(&attr, coef) == hipSuccess && attr.type == hipMemoryTypeDevice;
        (void)hipGetLastError();   // a plain host pointer may leave an error behind
        if (on_device) {
            if (hipMemcpy(coef_h.data(), coef, (size_t)n_elem * sizeof(double), hipMemcpyDeviceToHost) != hipSuccess) {
                delete c;
                return fail(BDDC_EHIP, "copy of the device coefficients failed");
            }
        } else {
            std::memcpy(coef_h.data(), coef, (size_t)n_elem * sizeof(double));
        }
        if (o.coef_log)
            for (double &v : coef_h) v = std::exp(v);
    }
    int rc = setup_impl(c, mesh, part, coef_h.data());
    if (rc) {
        std::string keep = g_err;
        bddc_destroy(c);
        g_err = keep;
        return rc;
    }
    *out = c;
    return 0;
}

int dpcg_solve(bddc_ctx *c, const double *rhs_seq, int32_t n_rhs, double rtol, double *x_seq, int32_t *iters,
               double *true_relres) {
    if (!c || (!rhs_seq && n_rhs > 0) || (!x_seq && n_rhs > 0) || n_rhs < 0 || !(rtol > 0))
        return fail(BDDC_EINVAL, "bad dpcg_solve argument");
    bool condensed = false;
    c->pre_schur = false;
    // several right-hand sides: condensed CBLK at a time in one pass over the
    // interior tiles, and their interiors recovered likewise after the group's
    // last solve (the results are those of the one-at-a-time forms)
    if (n_rhs > 1) {
        int rc = cblk_setup(c);
        if (rc) return rc;
    }
    const bool blk = n_rhs > 1 && c->cblk_state == 1;
    int g0 = 0, gn = 0;                 // the condensed group: right-hand sides [g0, g0 + gn)
    for (int k = 0; k < n_rhs; ++k) {
        int it = 0;
        double rr = 0.0;
        if (blk) {
            if (k >= g0 + gn) {
                g0 = k;
                gn = std::min(CBLK, n_rhs - k);
                if (int rc = run_condense_block(c, rhs_seq + (size_t)k * c->n_nodes, gn)) return rc;
            }
            take_condensed(c, k - g0);
            condensed = true;
        }
        int rc = solve_one(c, rhs_seq + (size_t)k * c->n_nodes, blk ? nullptr : x_seq + (size_t)k * c->n_nodes, rtol,
                           true, condensed, &it, &rr);
        if (iters) iters[k] = it;
        if (true_relres) true_relres[k] = rr;
        if (blk) {   // the group's interiors are recovered together after its last solve (or a failure)
            launch_copy(c->n_gamma, c->d_x, c->d_cblk_x + (size_t)(k - g0) * c->ld, c->stream);
            if (rc || k == g0 + gn - 1) {
                const int r2 = run_recover_block(c, rhs_seq + (size_t)g0 * c->n_nodes, x_seq + (size_t)g0 * c->n_nodes,
                                                 k - g0 + 1);
                if (!rc) rc = r2;
            }
        }
        if (rc) { (void)settle(c); if (c->timing) flush_timing(c); return rc; }
        // the next right-hand side is condensed while the host solves the
        // small recycling eigenproblem
        condensed = k + 1 < n_rhs;
        if (condensed) {
            if (!blk) run_condense(c, rhs_seq + (size_t)(k + 1) * c->n_nodes);
            // A x_{-1} of the next initial residual does not depend on the
            // deflation basis.  With the previous solution as x_{-1} it is the
            // product the true residual just formed, still in the Schur
            // partials (nothing in between writes them); otherwise it runs
            // here, ahead of the basis update
            if (c->opts.init_guess == 1) {
                launch_fill(c->n_gamma, 0.0, c->d_x, c->stream);
                run_schur(c, c->d_x, false, false);
            } else if (c->h_ctl->zero_rhs) {
                run_schur(c, c->d_x, false, false);    // x was reset to 0 after that product
            }
            c->pre_schur = true;
        }
        {
            TScope ts(c, TK_REC);
            rc = do_recycle(c);
        }
        if (rc) { c->pre_schur = false; (void)settle(c); if (c->timing) flush_timing(c); return rc; }
    }
    c->pre_schur = false;
    int rc = settle(c);
    if (c->timing) flush_timing(c);
    return rc;
}

int recycle_update(bddc_ctx *c) {
    if (!c) return fail(BDDC_EINVAL, "null context");
    int rc = do_recycle(c);
    if (rc) return rc;
    return settle(c);
}

int bddc_reset_recycle(bddc_ctx *c) {
    if (!c) return fail(BDDC_EINVAL, "null context");
    c->k = 0;
    c->WAW.clear();
    c->GWW.clear();
    c->theta.clear();
    c->frozen = false;
    c->freeze_step = -1;
    c->n_updates = 0;
    c->update_refused = 0;
    c->have_solve = false;
    c->last_restarts = 0;
    c->seg_start = 0;
    c->pend = Pending();
    launch_fill(c->n_gamma, 0.0, c->d_x, c->stream);
    if (c->d_state) launch_set_state(c->d_state, 0, 1, c->stream);
    init_null_column(c);
    HIPCHK(hipStreamSynchronize(c->stream));
    return 0;
}

int bddc_adjoint_grad_block(bddc_ctx *c, const double *dLdu_seq, int32_t n_rhs, const double *u_seq, double rtol,
                            double *grad_logcoef, double *grad_rhs_seq, int32_t *iters) {
    if (!c || !dLdu_seq || !u_seq || !grad_logcoef || !grad_rhs_seq || n_rhs < 0 || !(rtol > 0))
        return fail(BDDC_EINVAL, "bad bddc_adjoint_grad_block argument");
    if (n_rhs > BMAX) return fail(BDDC_EINVAL, "bddc_adjoint_grad_block: at most 32 right-hand sides");
    if (c->nullc) return fail(BDDC_EINVAL, "bddc_adjoint_grad_block: not for the pure Neumann problem");
    if (!(c->prec_built & 1))
        return fail(BDDC_EINVAL, "bddc_adjoint_grad_block: needs the float64 Neumann operators (local_prec 64 or local_prec_set bit 1)");
    if (symm_smem_bytes(c->max_nB) > 160 * 1024)
        return fail(BDDC_EINVAL, "bddc_adjoint_grad_block: a subdomain interface is too large for the block product");
    if (iters) *iters = 0;
    if (n_rhs == 0) {
        launch_fill(c->st.n_elem, 0.0, grad_logcoef, c->stream);
        HIPCHK(hipStreamSynchronize(c->stream));
        return 0;
    }
    // adopt a basis update still pending from the last forward solve
    if (c->pend.active) {
        int rc0;
        if ((rc0 = end_sync_issue(c, false)) || (rc0 = end_sync_wait(c))) return rc0;
    }
    if (set_symm_smem_limit(symm_smem_bytes(c->max_nB))) return fail(BDDC_EHIP, "hipFuncSetAttribute (block product LDS) failed");
    BlockWork b;
    int rc = alloc_block(c, b);
    double *xsave = nullptr;
    if (!rc) rc = dalloc(c, &xsave, c->n_gamma);
    if (rc) { free_block(c, b); return rc; }
    launch_copy(c->n_gamma, c->d_x, xsave, c->stream);
    launch_set_done(c->d_ctl, 0, c->stream);
    // condensation and recovery: CBLK right-hand sides per pass over the
    // interior operators when the block product can stage them
    if (n_rhs > 1 && (rc = cblk_setup(c))) { dfree(c, xsave); free_block(c, b); return rc; }
    const bool grouped = n_rhs > 1 && c->cblk_state == 1;
    for (int g0 = 0; g0 < n_rhs; g0 += CBLK) {
        const int gn = std::min(CBLK, n_rhs - g0);
        if (grouped && (rc = run_condense_block(c, dLdu_seq + (size_t)g0 * c->n_nodes, gn))) break;
        for (int q = 0; q < gn; ++q) {
            const int k = g0 + q;
            if (!grouped) run_condense(c, dLdu_seq + (size_t)k * c->n_nodes);
            launch_copy(c->n_gamma, grouped ? c->d_cblk_b + (size_t)q * c->ld : c->d_b, b.B + (size_t)k * c->ld,
                        c->stream);
        }
    }
    if (rc) { launch_copy(c->n_gamma, xsave, c->d_x, c->stream); (void)hipStreamSynchronize(c->stream); dfree(c, xsave); free_block(c, b); return rc; }
    // (set_symm_smem_limit again: the grouped condensation set its own)
    if (set_symm_smem_limit(symm_smem_bytes(c->max_nB))) rc = fail(BDDC_EHIP, "hipFuncSetAttribute (block product LDS) failed");
    int it = 0;
    if (!rc) rc = block_solve(c, b, n_rhs, rtol, &it);
    if (iters) *iters = it;
    if (rc == 0 || rc == BDDC_ENOTCONV) {
        for (int g0 = 0; g0 < n_rhs; g0 += CBLK) {
            const int gn = std::min(CBLK, n_rhs - g0);
            if (grouped) {
                for (int q = 0; q < gn; ++q)
                    launch_copy(c->n_gamma, b.X + (size_t)(g0 + q) * c->ld, c->d_cblk_x + (size_t)q * c->ld, c->stream);
                int r2 = run_recover_block(c, dLdu_seq + (size_t)g0 * c->n_nodes, grad_rhs_seq + (size_t)g0 * c->n_nodes, gn);
                if (r2 && (rc == 0 || rc == BDDC_ENOTCONV)) rc = r2;
            } else {
                for (int q = 0; q < gn; ++q) {
                    const int k = g0 + q;
                    launch_copy(c->n_gamma, b.X + (size_t)k * c->ld, c->d_x, c->stream);
                    run_recover(c, dLdu_seq + (size_t)k * c->n_nodes, grad_rhs_seq + (size_t)k * c->n_nodes);
                }
            }
        }
        GradArgs g{};
        g.n_elem = c->st.n_elem; g.n_nodes = c->n_nodes; g.nx = c->st.nx; g.ny = c->st.ny; g.nz = c->st.nz;
        g.n_rhs = n_rhs; g.keep = c->d_keep; g.free_node = c->d_free; g.coefh = c->d_coefh;
        g.lam = grad_rhs_seq; g.u = u_seq; g.grad = grad_logcoef;
        launch_elem_grad(g, c->stream);
    }
    launch_copy(c->n_gamma, xsave, c->d_x, c->stream);
    c->have_solve = false;
    (void)hipStreamSynchronize(c->stream);
    dfree(c, xsave);
    free_block(c, b);
    return rc;
}

int bddc_adjoint_grad(bddc_ctx *c, const double *dLdu_seq, int32_t n_rhs, const double *u_seq, double rtol,
                      double *grad_logcoef, double *grad_rhs_seq) {
    if (!c || !dLdu_seq || !u_seq || !grad_logcoef || !grad_rhs_seq || n_rhs < 0 || !(rtol > 0))
        return fail(BDDC_EINVAL, "bad bddc_adjoint_grad argument");
    // the forward sequence keeps its own previous solution
    double *xsave = nullptr;
    int rc = dalloc(c, &xsave, c->n_gamma);
    if (rc) return rc;
    launch_copy(c->n_gamma, c->d_x, xsave, c->stream);
    launch_fill(c->n_gamma, 0.0, c->d_x, c->stream);
    // condensation and recovery grouped as in dpcg_solve
    if (n_rhs > 1 && (rc = cblk_setup(c))) { dfree(c, xsave); return rc; }
    const bool grouped = n_rhs > 1 && c->cblk_state == 1;
    for (int g0 = 0; g0 < n_rhs && rc == 0; g0 += CBLK) {
        const int gn = std::min(CBLK, n_rhs - g0);
        if (grouped && (rc = run_condense_block(c, dLdu_seq + (size_t)g0 * c->n_nodes, gn))) break;
        int k = g0;
        for (; k < g0 + gn && rc == 0; ++k) {
            if (grouped) take_condensed(c, k - g0);
            rc = solve_one(c, dLdu_seq + (size_t)k * c->n_nodes, grouped ? nullptr : grad_rhs_seq + (size_t)k * c->n_nodes,
                           rtol, false, grouped, nullptr, nullptr);
            if (grouped) launch_copy(c->n_gamma, c->d_x, c->d_cblk_x + (size_t)(k - g0) * c->ld, c->stream);
        }
        if (grouped) {
            const int r2 = run_recover_block(c, dLdu_seq + (size_t)g0 * c->n_nodes, grad_rhs_seq + (size_t)g0 * c->n_nodes,
                                             k - g0);
            if (!rc) rc = r2;
        }
    }
    c->have_solve = false;
    launch_copy(c->n_gamma, xsave, c->d_x, c->stream);
    if (rc == 0) {
        GradArgs g{};
        g.n_elem = c->st.n_elem; g.n_nodes = c->n_nodes; g.nx = c->st.nx; g.ny = c->st.ny; g.nz = c->st.nz;
        g.n_rhs = n_rhs; g.keep = c->d_keep; g.free_node = c->d_free; g.coefh = c->d_coefh;
        g.lam = grad_rhs_seq; g.u = u_seq; g.grad = grad_logcoef;
        launch_elem_grad(g, c->stream);
    }
    (void)hipStreamSynchronize(c->stream);
    dfree(c, xsave);
    return rc;
}

int bddc_apply_schur(bddc_ctx *c, const double *p, double *q) {
    if (!c || !p || !q) return fail(BDDC_EINVAL, "null argument");
    run_schur(c, p, false, false);
    ResidArgs a{};
    a.n = c->n_gamma; a.want_wtr = 0; a.q = gather_of(c->opS); a.b = nullptr; a.out = q;
    a.W = c->d_W; a.ld = c->ld; a.ctl = c->d_ctl; a.part = c->d_wp;
    launch_resid(a, 0, c->vgrid, c->stream);
    HIPCHK(hipStreamSynchronize(c->stream));
    return 0;
}

int bddc_apply_schur_noalloc(bddc_ctx *c, const double *p, double *q) {
    if (!c || !p || !q) return fail(BDDC_EINVAL, "null argument");
    double *sp = nullptr;
    std::string err;
    if (int rc = noalloc_scratch(&sp, err)) return fail(rc, err);
    const int64_t need = c->opS.ylen + c->vgrid;
    if (need > noalloc_scratch_doubles())
        return fail(BDDC_EINVAL, "bddc_apply_schur_noalloc: this context's Schur product needs " + std::to_string(need) +
                                     " doubles of scratch; the static array holds " +
                                     std::to_string(noalloc_scratch_doubles()) + " (use bddc_apply_schur)");
    // the same kernels as bddc_apply_schur, with the partial products and the
    // per-block norm partials in the static array
    SymvArgs a{};
    a.op = c->opS.dev;
    a.x = p;
    a.ypart = sp;
    a.ctl = c->d_ctl;
    launch_symv(a, SYMV_SCHUR, 64, c->opS.cfg, c->opS.smem, c->stream);
    ResidArgs r{};
    r.n = c->n_gamma; r.want_wtr = 0; r.q = Gather{c->opS.d_yptr, c->opS.d_yidx, sp}; r.b = nullptr; r.out = q;
    r.W = c->d_W; r.ld = c->ld; r.ctl = c->d_ctl; r.part = sp + c->opS.ylen;
    launch_resid(r, 0, c->vgrid, c->stream);
    HIPCHK(hipStreamSynchronize(c->stream));
    return 0;
}

int bddc_apply_precond(bddc_ctx *c, const double *r, double *z) {
    if (!c || !r || !z) return fail(BDDC_EINVAL, "null argument");
    launch_set_done(c->d_ctl, 0, c->stream);
    run_precond(c, r, z, 0, false, false, false);
    HIPCHK(hipStreamSynchronize(c->stream));
    return 0;
}

int bddc_condense(bddc_ctx *c, const double *F, double *b) {
    if (!c || !F || !b) return fail(BDDC_EINVAL, "null argument");
    run_condense(c, F);
    launch_copy(c->n_gamma, c->d_b, b, c->stream);
    HIPCHK(hipStreamSynchronize(c->stream));
    return 0;
}

int bddc_info(const bddc_ctx *c, int64_t *info) {
    if (!c || !info) return fail(BDDC_EINVAL, "null argument");
    info[0] = c->n_nodes;
    info[1] = c->n_gamma;
    info[2] = c->n_sub;
    info[3] = c->nC;
    info[4] = c->st.n_corner;
    info[5] = c->st.n_face;
    info[6] = c->st.n_edge;
    info[7] = c->three ? (int64_t)c->st.gamma2.size() : 0;
    info[8] = c->three ? (int64_t)(c->nC - c->st.gamma2.size()) : 0;
    info[9] = c->three ? c->n3 : c->nC;
    info[10] = c->k;
    info[11] = c->frozen ? 1 : 0;
    info[12] = (int64_t)c->bytes_S;
    info[13] = (int64_t)c->bytes_N;
    info[14] = c->max_nB;
    info[15] = (int64_t)c->dev_bytes;
    return 0;
}

int bddc_adaptive_stats(const bddc_ctx *c, double *out) {
    if (!c || !out) return fail(BDDC_EINVAL, "null argument");
    out[0] = c->adapt.faces;
    out[1] = c->adapt.added;
    out[2] = c->adapt.lam_max;
    out[3] = c->adapt.seconds;
    return 0;
}

int bddc_adaptive2_stats(const bddc_ctx *c, double *out) {
    if (!c || !out) return fail(BDDC_EINVAL, "null argument");
    out[0] = c->adapt2.faces;
    out[1] = c->adapt2.added;
    out[2] = c->adapt2.lam_max;
    out[3] = c->adapt2.seconds;
    return 0;
}

int bddc_face_constraints(int32_t m, const double *Hs, const double *Ht, const double *Ks, const double *Kt,
                          const double *Ds, const double *Dt, int32_t floating_s, int32_t floating_t, int32_t nb,
                          const double *B, int32_t nf, const int32_t *fpos, double tau, int32_t max_rows,
                          double *lam, int32_t *n_lam, double *rows, int32_t *n_rows) {
    if (m < 0 || nb < 0 || nf < 0 || max_rows < 0 || !n_lam || !n_rows || (m > 0 && (!Hs || !Ht || !Ks || !Kt || !Ds || !Dt || !lam)) ||
        (nb > 0 && !B) || (nf > 0 && !fpos) || (max_rows > 0 && nf > 0 && !rows))
        return fail(BDDC_EINVAL, "bad bddc_face_constraints argument");
    for (int q = 0; q < nf; ++q)
        if (fpos[q] < 0 || fpos[q] >= m) return fail(BDDC_EINVAL, "face position out of range");
    FaceInput in{m, Hs, Ht, Ks, Kt, Ds, Dt, floating_s != 0, floating_t != 0, nb, B, nf, fpos};
    FaceOutput out;
    int rc = face_rows(in, tau, max_rows, out);
    if (rc) return fail(rc, "face problem: no Cholesky factor of H_s + H_t");
    *n_lam = (int32_t)out.lam.size();
    for (size_t i = 0; i < out.lam.size(); ++i) lam[i] = out.lam[i];
    *n_rows = (int32_t)out.rows.size();
    for (size_t r = 0; r < out.rows.size(); ++r)
        for (int q = 0; q < nf; ++q) rows[r * nf + q] = out.rows[r][q];
    return 0;
}

int bddc_face_constraints_lobpcg(int32_t m, const double *Hs, const double *Ht, const double *Ks, const double *Kt,
                                 const double *Ds, const double *Dt, int32_t floating_s, int32_t floating_t, int32_t nb,
                                 const double *B, int32_t nf, const int32_t *fpos, double tau, int32_t max_rows,
                                 int32_t max_it, double *lam, int32_t *n_lam, double *rows, int32_t *n_rows,
                                 int32_t *iters) {
    if (m < 0 || nb < 0 || nf < 0 || max_rows < 0 || max_it < 1 || !n_lam || !n_rows ||
        (m > 0 && (!Hs || !Ht || !Ks || !Kt || !Ds || !Dt || !lam)) || (nb > 0 && !B) || (nf > 0 && !fpos) ||
        (max_rows > 0 && nf > 0 && !rows))
        return fail(BDDC_EINVAL, "bad bddc_face_constraints_lobpcg argument");
    for (int q = 0; q < nf; ++q)
        if (fpos[q] < 0 || fpos[q] >= m) return fail(BDDC_EINVAL, "face position out of range");
    FaceInput in{m, Hs, Ht, Ks, Kt, Ds, Dt, floating_s != 0, floating_t != 0, nb, B, nf, fpos};
    FaceOutput out;
    int its = 0;
    int rc = face_rows(in, tau, max_rows, out, max_it, &its);
    if (rc) return fail(rc, "face problem: no Cholesky factor of H_s + H_t");
    if (iters) *iters = its;
    *n_lam = (int32_t)out.lam.size();
    for (size_t i = 0; i < out.lam.size(); ++i) lam[i] = out.lam[i];
    *n_rows = (int32_t)out.rows.size();
    for (size_t r = 0; r < out.rows.size(); ++r)
        for (int q = 0; q < nf; ++q) rows[r * nf + q] = out.rows[r][q];
    return 0;
}

int bddc_interface_nodes(const bddc_ctx *c, int64_t *out) {
    if (!c || !out) return fail(BDDC_EINVAL, "null argument");
    for (int g = 0; g < c->n_gamma; ++g) out[g] = c->st.gamma[g];
    return 0;
}

int bddc_enable_timing(bddc_ctx *c, int32_t enable) {
    if (!c) return fail(BDDC_EINVAL, "null context");
    // enable: bit k times kernel class k (1 = all classes)
    c->timing = enable != 0;
    c->timing_mask = enable == 1 ? 0x3f : (enable & 0x3f);
    for (int k = 0; k < TK_N; ++k) c->t_ms[k] = c->t_cnt[k] = 0;
    return 0;
}

int bddc_stats(const bddc_ctx *c, double *out, int32_t n) {
    if (!c || !out) return fail(BDDC_EINVAL, "null argument");
    for (int k = 0; k < n && k < TK_N; ++k) {
        out[3 * k] = c->t_ms[k];
        out[3 * k + 1] = c->t_cnt[k];
        out[3 * k + 2] = c->t_bytes[k];
    }
    return 0;
}

int bddc_time_products(bddc_ctx *c, int32_t reps, double *out) {
    if (!c || !out || reps <= 0) return fail(BDDC_EINVAL, "null argument or reps <= 0");
    hipEvent_t e0 = nullptr, e1 = nullptr;
    HIPCHK(hipEventCreate(&e0));
    HIPCHK(hipEventCreate(&e1));
    const OpHost *ops[2] = {&c->opS, &c->opN};
    int rc = 0;
    for (int w = 0; w < 2 && rc == 0; ++w) {
        const OpHost &op = *ops[w];
        SymvArgs a{};
        a.op = op.dev; a.x = c->d_x; a.ypart = op.d_ypart; a.ctl = c->d_ctl;
        if (w == 1) set_restriction(c, a);
        launch_symv(a, (SymvOp)w, op.prec, op.cfg, op.smem, c->stream);   // warm
        hipError_t e = hipEventRecord(e0, c->stream);
        for (int r = 0; r < reps && e == hipSuccess; ++r) launch_symv(a, (SymvOp)w, op.prec, op.cfg, op.smem, c->stream);
        if (e == hipSuccess) e = hipEventRecord(e1, c->stream);
        if (e == hipSuccess) e = hipEventSynchronize(e1);
        float ms = 0.f;
        if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
        if (e != hipSuccess) rc = fail(BDDC_EHIP, std::string("timing: ") + hipGetErrorString(e));
        out[2 * w] = 1e3 * ms / reps;
        out[2 * w + 1] = op.bytes;
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    return rc;
}

int bddc_set_local_prec(bddc_ctx *c, int32_t prec) {
    if (!c) return fail(BDDC_EINVAL, "null argument");
    const int q = prec_slot(prec);
    if (q < 0 || !((c->prec_built >> q) & 1) || !c->d_Nx[q])
        return fail(BDDC_EINVAL, "local precision " + std::to_string(prec) + " was not built at setup (local_prec_set)");
    if (prec == c->prec) return 0;
    HIPCHK(hipStreamSynchronize(c->stream));
    c->prec = prec;
    c->d_N = c->d_Nx[q];
    c->d_phir = c->d_phirx[q];
    OpHost &op = c->opN;
    op.prec = prec;
    op.dev.tiles = c->d_N;
    op.bytes = product_bytes(c, prec, c->nC > 0);
    c->bytes_N = (size_t)op.n_tiles * 256 * (size_t)(prec / 8);
    c->t_bytes[TK_PREC] = op.bytes;
    op.smem = symv_smem(prec, op.cfg.nw, c->max_nt);
    if (c->opts.autotune) {
        int rc = tune_operators(c, 2);
        if (rc) return rc;
    }
    if (c->gexec) {   // the captured iteration launches the other precision's kernel
        (void)hipGraphExecDestroy(c->gexec);
        c->gexec = nullptr;
    }
    if (c->graph) {
        (void)hipGraphDestroy(c->graph);
        c->graph = nullptr;
    }
    HIPCHK(hipStreamSynchronize(c->stream));
    return 0;
}

int bddc_set_launch(bddc_ctx *c, int32_t use_graph, const int32_t *product_cfg) {
    if (!c) return fail(BDDC_EINVAL, "null argument");
    if (use_graph < 0 || use_graph > 2) return fail(BDDC_EINVAL, "use_graph must be 0, 1 or 2");
    HIPCHK(hipStreamSynchronize(c->stream));
    if (product_cfg) {
        OpHost *ops[2] = {&c->opS, &c->opN};
        for (int w = 0; w < 2; ++w) {
            const int32_t *pc = product_cfg + 4 * w;
            OpHost &op = *ops[w];
            if (pc[0] == 0) continue;   // keep this product's configuration
            if (pc[0] > 0) {
                if ((pc[2] != 4 && pc[2] != 8) || (pc[3] != 2 && pc[3] != 4) || (pc[2] == 8 && !c->allow8))
                    return fail(BDDC_EINVAL, "product_cfg: waves must be 4 or 8 (8 when it fits), tiles in flight 2 or 4");
                op.bpc = pc[0];
                op.per_sub = pc[1] != 0;
                op.cfg = SymvCfg{pc[2], pc[3]};
            } else {   // negative: the untuned default
                op.bpc = 6;
                op.per_sub = true;
                op.cfg = SymvCfg{4, 2};
            }
            op.smem = symv_smem(op.prec, op.cfg.nw, c->max_nt);
            op.tuned_us = 0.f;
            if (int rc = build_worklist(c, op, product_blocks(c, op.n_tiles, op.bpc), op.per_sub)) return rc;
        }
        if (c->opS.dev.n_blocks > 0) {
            dfree(c, c->d_dotS);
            if (int rc = dalloc(c, &c->d_dotS, (size_t)c->opS.dev.n_blocks)) return rc;
        }
    }
    c->opts.use_graph = use_graph;
    if (c->gexec) {   // the captured iteration holds the old kernels and buffers
        (void)hipGraphExecDestroy(c->gexec);
        c->gexec = nullptr;
    }
    if (c->graph) {
        (void)hipGraphDestroy(c->graph);
        c->graph = nullptr;
    }
    HIPCHK(hipStreamSynchronize(c->stream));
    return 0;
}

int bddc_time_kernels(bddc_ctx *c, int32_t reps, double *out, int32_t n) {
    if (!c || !out || reps <= 0 || n < 0) return fail(BDDC_EINVAL, "null argument, reps <= 0 or n < 0");
    hipEvent_t e0 = nullptr, e1 = nullptr;
    HIPCHK(hipEventCreate(&e0));
    HIPCHK(hipEventCreate(&e1));
    int rc = 0;
    double res[12] = {0};
    auto timed = [&](int slot, double bytes, auto &&launch) {
        if (rc) return;
        launch();   // warm
        hipError_t e = hipEventRecord(e0, c->stream);
        for (int r = 0; r < reps && e == hipSuccess; ++r) launch();
        if (e == hipSuccess) e = hipEventRecord(e1, c->stream);
        if (e == hipSuccess) e = hipEventSynchronize(e1);
        float ms = 0.f;
        if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
        if (e != hipSuccess) rc = fail(BDDC_EHIP, std::string("timing: ") + hipGetErrorString(e));
        res[2 * slot] = 1e3 * ms / reps;
        res[2 * slot + 1] = bytes;
    };
    const bool tk = c->timing;
    c->timing = false;
    launch_set_done(c->d_ctl, 0, c->stream);
    const OpHost *ops[3] = {&c->opS, &c->opN, &c->opI};
    for (int w = 0; w < 3; ++w) {
        const OpHost &op = *ops[w];
        SymvArgs a{};
        a.op = op.dev; a.x = w == 2 ? c->d_tmpN : c->d_x; a.ypart = op.d_ypart; a.ctl = c->d_ctl;
        if (w == 1) set_restriction(c, a);
        double bytes = op.bytes;
        if (w == 2) {   // packed K_II^{-1}, gathered input and index, output
            bytes = 0.0;
            for (int i = 0; i < c->n_sub; ++i) {
                const double m = c->h_nI[i];
                bytes += m * (m + 1) / 2 * 8.0 + m * (8 + 4 + 8);
            }
        }
        timed(w, bytes, [&] { launch_symv(a, (SymvOp)w, op.prec, op.cfg, op.smem, c->stream); });
    }
    const double cb = coarse_bytes(c), pb = prolong_bytes(c);
    timed(3, c->opN.bytes + cb + pb, [&] { run_precond(c, c->d_r, c->d_tmp, 0, false, false, false); });
    timed(4, cb, [&] { run_coarse(c, c->stream); });
    timed(5, pb, [&] { run_prolong_assemble(c, c->d_r, c->d_tmp, false, false, false); });
    c->timing = tk;
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    for (int k = 0; k < n && k < 12; ++k) out[k] = res[k];
    return rc;
}

int bddc_solve_info(const bddc_ctx *c, int64_t *out, int32_t n) {
    if (!c || !out || n < 0) return fail(BDDC_EINVAL, "null argument or n < 0");
    const int64_t v[10] = {c->n_updates - c->update_refused, c->update_refused, c->frozen ? 1 : 0,
                           c->frozen ? c->freeze_step : -1, c->last_restarts, c->seg_start, c->k,
                           (int64_t)c->dev_bytes, (int64_t)c->dev_peak, c->prec};
    for (int k = 0; k < n && k < 10; ++k) out[k] = v[k];
    return 0;
}

int bddc_tuning(const bddc_ctx *c, double *out) {
    if (!c || !out) return fail(BDDC_EINVAL, "null argument");
    const OpHost *ops[2] = {&c->opS, &c->opN};
    for (int w = 0; w < 2; ++w) {
        double *o = out + 7 * w;
        o[0] = ops[w]->dev.n_blocks;
        o[1] = ops[w]->bpc;
        o[2] = ops[w]->per_sub ? 1.0 : 0.0;
        o[3] = ops[w]->cfg.nw;
        o[4] = ops[w]->cfg.unroll;
        o[5] = ops[w]->tuned_us;
        o[6] = (double)ops[w]->n_tiles;
    }
    return 0;
}

int bddc_ritz_values(const bddc_ctx *c, double *theta, int32_t cap, int32_t *count) {
    if (!c || !count) return fail(BDDC_EINVAL, "null argument");
    *count = (int32_t)c->theta.size();
    for (int i = 0; i < *count && i < cap && theta; ++i) theta[i] = c->theta[i];
    return 0;
}

void bddc_destroy(bddc_ctx *c) {
    if (!c) return;
    if (c->stream) (void)hipStreamSynchronize(c->stream);
    else (void)hipDeviceSynchronize();
    if (c->gexec) (void)hipGraphExecDestroy(c->gexec);
    if (c->graph) (void)hipGraphDestroy(c->graph);
    for (auto &e : c->gev)
        if (e) (void)hipEventDestroy(e);
    if (c->sync_ev) (void)hipEventDestroy(c->sync_ev);
    if (c->cap_stream) (void)hipStreamDestroy(c->cap_stream);
    for (auto &a : c->allocs) (void)hipFree(a.first);
    c->allocs.clear();
    if (c->h_ctl) (void)hipHostFree(c->h_ctl);
    if (c->h_sync) (void)hipHostFree(c->h_sync);
    if (c->h_hist) (void)hipHostFree(c->h_hist);
    if (c->h_Y) (void)hipHostFree(c->h_Y);
    if (c->h_flags) (void)hipHostFree(c->h_flags);
    if (c->h_prog) (void)hipHostFree(c->h_prog);
    for (auto &p : c->pending) { (void)hipEventDestroy(p.second.first); (void)hipEventDestroy(p.second.second); }
    for (auto e : c->ev_pool) (void)hipEventDestroy(e);
    delete c;
}

}  // extern "C"
