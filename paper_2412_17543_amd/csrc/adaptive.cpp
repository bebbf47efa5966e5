// Adaptive selection of face coarse DOFs (Section 3.3, eqs. eig-matrix,
// global-S, c-def), worked in the jump space of each face.
//
// For a face shared by subdomains s and t let G be the free nodes both
// interfaces contain (the face, its edges and corners; m of them).  The
// averaging E_st changes only entries on G, where (I - E) w is
// (a j, -b j) with the jump j = w_s - w_t and a = D_t / (D_s + D_t),
// b = D_s / (D_s + D_t).  The projection Pi (shared coarse DOFs agree) keeps
// exactly the pairs whose jump satisfies B j = 0, B the rows of those DOFs.
// So, with j restricted to null(B) (orthonormal basis Z),
//   left  side: j^T L j,  L = diag(a) S_s(G,G) diag(a) + diag(b) S_t(G,G) diag(b);
//   right side: the least energy w_s^T S_s w_s + w_t^T S_t w_t of a pair with
//               that jump, j^T P j with P = H_s - H_s (H_s + H_t)^+ H_s, where
//               H_s, H_t are the Schur complements of S_s, S_t onto G (the
//               device computes them, k_face_schur);
// and eq. eig-matrix becomes the m-sized pencil Z^T L Z y = lambda Z^T P Z y.
// The covector of eq. c-def is c = (g, -g) on G with g = Z Z^T L j, zero
// elsewhere; its entries on the face's own nodes become the new row.  The
// null space of the right-hand matrix is dropped below 1e-12 of its largest
// eigenvalue; rows are orthonormalised against the face average and the
// face's earlier rows and dropped below 1e-8 of the face part's norm.
#include <algorithm>
#include <atomic>
#include <chrono>
#include <cmath>
#include <cstring>
#include <thread>

#include "adaptive.h"
#include "kernels.h"

namespace bddc {

int adaptive_faces(const Structure &st, const double *d_K, const std::vector<int64_t> &k_off, double tau,
                   int max_per_face, int lobpcg_it, int32_t *d_status, hipStream_t s, std::vector<CoarseDof> &extra,
                   AdaptStats &stats, std::string &err) {
    const auto t0 = std::chrono::steady_clock::now();
    extra.clear();
    stats = AdaptStats{};
    struct Face {
        int c, s, t, m;
        std::vector<int32_t> ps, pt, fpos;   // shared nodes in s, t interface order; face nodes in G order
        std::vector<int64_t> G;              // shared node ids (ascending)
    };
    std::vector<Face> faces;
    for (int c = 0; c < (int)st.coarse.size(); ++c) {
        const CoarseDof &d = st.coarse[c];
        if (d.kind != 1 || d.subs.size() != 2) continue;
        Face f;
        f.c = c; f.s = d.subs[0]; f.t = d.subs[1];
        const SubHost &a = st.sub[f.s], &b = st.sub[f.t];
        int i = 0, j = 0;
        while (i < a.nB && j < b.nB) {
            const int32_t na = a.nodes[a.nI + i], nb = b.nodes[b.nI + j];
            if (na == nb) { f.ps.push_back(i); f.pt.push_back(j); f.G.push_back(na); ++i; ++j; }
            else if (na < nb) ++i;
            else ++j;
        }
        f.m = (int)f.G.size();
        for (int64_t n : d.nodes) {
            auto it = std::lower_bound(f.G.begin(), f.G.end(), n);
            if (it == f.G.end() || *it != n) { err = "face node outside the shared nodes"; return BDDC_EINVAL; }
            f.fpos.push_back((int32_t)(it - f.G.begin()));
        }
        faces.push_back(std::move(f));
    }
    stats.faces = (int)faces.size();
    if (faces.empty()) return BDDC_OK;
    std::vector<char> floating(st.n_sub, 1);
    for (int i = 0; i < st.n_sub; ++i)
        for (int32_t l : st.sub[i].elem_loc)
            if (l < 0) { floating[i] = 0; break; }

    // device: H and S(G, G) for both sides of every face, in batches that
    // bound the scratch to about 2 GiB
    std::vector<std::vector<double>> Hh(faces.size() * 2), Kh(faces.size() * 2);
    size_t max_nB = 1;
    for (const auto &sh : st.sub) max_nB = std::max(max_nB, (size_t)sh.nB);
    const size_t per_job = max_nB * max_nB;
    const size_t batch = std::max<size_t>(1, std::min<size_t>(faces.size() * 2, (size_t(2) << 30) / (per_job * 8)));
    double *d_work = nullptr, *d_out = nullptr, *d_panel = nullptr;
    int32_t *d_perm = nullptr;
    FaceSchurDesc *d_desc = nullptr;
    SweepDesc *d_sw = nullptr;
    int64_t *d_off = nullptr;
    auto cleanup = [&]() {
        if (d_work) (void)hipFree(d_work);
        if (d_out) (void)hipFree(d_out);
        if (d_perm) (void)hipFree(d_perm);
        if (d_desc) (void)hipFree(d_desc);
        if (d_panel) (void)hipFree(d_panel);
        if (d_sw) (void)hipFree(d_sw);
        if (d_off) (void)hipFree(d_off);
    };
    size_t max_m = 1;
    for (const auto &f : faces) max_m = std::max(max_m, (size_t)f.m);
    if (hipMalloc(&d_work, batch * per_job * 8) != hipSuccess || hipMalloc(&d_out, batch * 2 * max_m * max_m * 8) != hipSuccess ||
        hipMalloc(&d_perm, batch * max_nB * 4) != hipSuccess || hipMalloc(&d_desc, batch * sizeof(FaceSchurDesc)) != hipSuccess ||
        hipMalloc(&d_panel, batch * 32 * max_nB * 8) != hipSuccess || hipMalloc(&d_sw, batch * sizeof(SweepDesc)) != hipSuccess ||
        hipMalloc(&d_off, batch * sizeof(int64_t)) != hipSuccess) {
        cleanup();
        err = "hipMalloc failed for the adaptive face problems";
        return BDDC_ENOMEM;
    }
    std::vector<int32_t> perm(batch * max_nB);
    std::vector<FaceSchurDesc> desc(batch);
    std::vector<double> hout(batch * 2 * max_m * max_m);
    const size_t njobs = faces.size() * 2;
    for (size_t j0 = 0; j0 < njobs; j0 += batch) {
        const size_t nj = std::min(batch, njobs - j0);
        for (size_t q = 0; q < nj; ++q) {
            const Face &f = faces[(j0 + q) / 2];
            const bool side_t = (j0 + q) % 2;
            const int sub = side_t ? f.t : f.s;
            const SubHost &sh = st.sub[sub];
            const std::vector<int32_t> &pg = side_t ? f.pt : f.ps;
            std::vector<char> inG(sh.nB, 0);
            for (int32_t k : pg) inG[k] = 1;
            int32_t *pp = &perm[q * max_nB];
            int w = 0;
            for (int k = 0; k < sh.nB; ++k)
                if (!inG[k]) pp[w++] = k;
            for (int32_t k : pg) pp[w++] = k;
            const int nl = sh.nloc;
            desc[q] = FaceSchurDesc{d_K + k_off[sub] + (int64_t)sh.nI * nl + sh.nI, nl, d_perm + q * max_nB, sh.nB,
                                    sh.nB - f.m, d_work + q * per_job, d_out + q * 2 * max_m * max_m,
                                    d_out + q * 2 * max_m * max_m + max_m * max_m};
        }
        if (hipMemcpyAsync(d_perm, perm.data(), nj * max_nB * 4, hipMemcpyHostToDevice, s) != hipSuccess ||
            hipMemcpyAsync(d_desc, desc.data(), nj * sizeof(FaceSchurDesc), hipMemcpyHostToDevice, s) != hipSuccess) {
            cleanup();
            err = "hipMemcpy failed";
            return BDDC_EHIP;
        }
        launch_face_schur(d_desc, std::vector<FaceSchurDesc>(desc.begin(), desc.begin() + nj), d_sw, d_off, d_panel,
                          d_status, s);
        if (hipMemcpyAsync(hout.data(), d_out, nj * 2 * max_m * max_m * 8, hipMemcpyDeviceToHost, s) != hipSuccess ||
            hipStreamSynchronize(s) != hipSuccess) {
            cleanup();
            err = "face Schur complements failed";
            return BDDC_EHIP;
        }
        for (size_t q = 0; q < nj; ++q) {
            const int m = faces[(j0 + q) / 2].m;
            const double *o = &hout[q * 2 * max_m * max_m];
            Hh[j0 + q].assign(o, o + (size_t)m * m);
            Kh[j0 + q].assign(o + max_m * max_m, o + max_m * max_m + (size_t)m * m);
        }
    }
    cleanup();
    int32_t status = 0;
    if (hipMemcpy(&status, d_status, sizeof(int32_t), hipMemcpyDeviceToHost) != hipSuccess) { err = "hipMemcpy failed"; return BDDC_EHIP; }
    if (status) { err = "non-positive pivot in a face Schur complement"; return BDDC_ESINGULAR; }

    // host: the face pencils, several faces at a time
    std::vector<FaceOutput> res(faces.size());
    std::vector<int> rcs(faces.size(), 0);
    std::atomic<size_t> next{0};
    auto worker = [&]() {
        for (size_t fi = next++; fi < faces.size(); fi = next++) {
            const Face &f = faces[fi];
            const SubHost &a = st.sub[f.s], &b = st.sub[f.t];
            std::vector<double> Ds(f.m), Dt(f.m), B;
            for (int k = 0; k < f.m; ++k) { Ds[k] = a.wB[f.ps[k]]; Dt[k] = b.wB[f.pt[k]]; }
            int nb = 0;
            for (int32_t c : a.cidx) {
                const CoarseDof &d = st.coarse[c];
                if (!std::binary_search(d.subs.begin(), d.subs.end(), f.t)) continue;
                std::vector<double> rw(f.m, 0.0);
                for (size_t q = 0; q < d.nodes.size(); ++q) {
                    auto it = std::lower_bound(f.G.begin(), f.G.end(), d.nodes[q]);
                    if (it == f.G.end() || *it != d.nodes[q]) { rcs[fi] = BDDC_EINVAL; break; }
                    rw[it - f.G.begin()] = d.wts.empty() ? 1.0 / (double)d.nodes.size() : d.wts[q];
                }
                if (rcs[fi]) break;
                B.insert(B.end(), rw.begin(), rw.end());
                ++nb;
            }
            if (rcs[fi]) continue;
            FaceInput in{f.m, Hh[2 * fi].data(), Hh[2 * fi + 1].data(), Kh[2 * fi].data(), Kh[2 * fi + 1].data(),
                         Ds.data(), Dt.data(), floating[f.s] != 0, floating[f.t] != 0, nb, B.data(),
                         (int)f.fpos.size(), f.fpos.data()};
            rcs[fi] = face_rows(in, tau, max_per_face, res[fi], lobpcg_it);
        }
    };
    const unsigned nth = std::max(1u, std::min(16u, std::thread::hardware_concurrency()));
    std::vector<std::thread> pool;
    for (unsigned q = 1; q < nth; ++q) pool.emplace_back(worker);
    worker();
    for (auto &th : pool) th.join();
    for (size_t fi = 0; fi < faces.size(); ++fi) {
        if (rcs[fi]) { err = "singular face problem"; return rcs[fi]; }
        const Face &f = faces[fi];
        if (!res[fi].lam.empty()) stats.lam_max = std::max(stats.lam_max, res[fi].lam[0]);
        for (const auto &row : res[fi].rows) {
            CoarseDof d;
            d.kind = 3;
            d.nodes = st.coarse[f.c].nodes;
            d.subs = st.coarse[f.c].subs;
            d.wts = row;
            extra.push_back(d);
        }
    }
    stats.added = (int)extra.size();
    stats.seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    return BDDC_OK;
}

}  // namespace bddc

namespace bddc {

// Adaptivity at level 2 (Section 3.3 on the coarse problem of the multilevel
// method): subregions in the role of subdomains, level-1 coarse DOFs in the
// role of nodes, the subregion Schur complements S2_j (K2_j with its interior
// coarse DOFs eliminated) in the role of S_i, the level-2 card weights as D,
// and the level-3 DOFs that two subregions share as the constraints of Pi.
// Every level-2 face gets the jump-space pencil above; its rows (over the
// face's coarse DOFs) become level-3 DOFs of the two subregions.
int adaptive_level2(const Structure &st, const std::vector<std::vector<double>> &S2,
                    const std::vector<char> &floating, double tau, int max_per_face, int lobpcg_it,
                    std::vector<Level3Dof> &extra, AdaptStats &stats, std::string &err) {
    const auto t0 = std::chrono::steady_clock::now();
    extra.clear();
    stats = AdaptStats{};
    std::vector<int32_t> faces;
    for (int m3 = 0; m3 < st.n3; ++m3)
        if (st.dof3_kind[m3] == 1 && st.dof3_subs[m3].size() == 2) faces.push_back(m3);
    stats.faces = (int)faces.size();
    std::vector<FaceOutput> res(faces.size());
    std::vector<int> rcs(faces.size(), 0);
    std::atomic<size_t> next{0};
    // H = S(G,G) - S(G,O) S(O,O)^{-1} S(O,G) of one side, O = the rest of its interface
    auto side = [&](int j, const std::vector<int32_t> &pg, std::vector<double> &H, std::vector<double> &K) -> bool {
        const SubregionHost &r = st.sr[j];
        const int n = r.nB, m = (int)pg.size();
        const double *S = S2[j].data();
        std::vector<char> inG(n, 0);
        for (int32_t k : pg) inG[k] = 1;
        std::vector<int32_t> po;
        for (int k = 0; k < n; ++k)
            if (!inG[k]) po.push_back(k);
        const int no = (int)po.size();
        K.assign((size_t)m * m, 0.0);
        for (int a = 0; a < m; ++a)
            for (int b = 0; b < m; ++b) K[(size_t)a * m + b] = S[(size_t)pg[a] * n + pg[b]];
        H = K;
        if (no == 0) return true;
        std::vector<double> Loo((size_t)no * no);
        for (int a = 0; a < no; ++a)
            for (int b = 0; b < no; ++b) Loo[(size_t)a * no + b] = S[(size_t)po[a] * n + po[b]];
        if (!cholesky(Loo, no)) return false;
        std::vector<double> X((size_t)no * m), col(no);
        for (int b = 0; b < m; ++b) {
            for (int a = 0; a < no; ++a) col[a] = S[(size_t)po[a] * n + pg[b]];
            chol_solve(Loo, no, col.data());
            for (int a = 0; a < no; ++a) X[(size_t)a * m + b] = col[a];
        }
        for (int a = 0; a < m; ++a)
            for (int b = 0; b < m; ++b) {
                double t = 0.0;
                for (int q = 0; q < no; ++q) t += S[(size_t)pg[a] * n + po[q]] * X[(size_t)q * m + b];
                H[(size_t)a * m + b] -= t;
            }
        for (int a = 0; a < m; ++a)
            for (int b = a + 1; b < m; ++b) {
                const double v = 0.5 * (H[(size_t)a * m + b] + H[(size_t)b * m + a]);
                H[(size_t)a * m + b] = H[(size_t)b * m + a] = v;
            }
        return true;
    };
    auto worker = [&]() {
        for (size_t fi = next++; fi < faces.size(); fi = next++) {
            const int m3 = faces[fi];
            const int j = st.dof3_subs[m3][0], k = st.dof3_subs[m3][1];
            const SubregionHost &a = st.sr[j], &b = st.sr[k];
            std::vector<int32_t> ps, pt, G;          // shared coarse ids, ascending
            for (int p = 0, q = 0; p < a.nB && q < b.nB;) {
                const int32_t ca = a.L[a.nI + p], cb = b.L[b.nI + q];
                if (ca == cb) { ps.push_back(p++); pt.push_back(q++); G.push_back(ca); }
                else if (ca < cb) ++p;
                else ++q;
            }
            const int m = (int)G.size();
            auto pos = [&](int32_t cid) {
                auto it = std::lower_bound(G.begin(), G.end(), cid);
                return (it == G.end() || *it != cid) ? -1 : (int)(it - G.begin());
            };
            std::vector<int32_t> fpos;
            for (int32_t cid : st.dof3_members[m3]) fpos.push_back(pos(cid));
            std::vector<double> Ds(m), Dt(m), B, Hs, Ht, Ks, Kt;
            for (int q = 0; q < m; ++q) { Ds[q] = a.w[ps[q]]; Dt[q] = b.w[pt[q]]; }
            int nb = 0;
            for (int32_t d3 : a.c3) {
                if (!std::binary_search(b.c3.begin(), b.c3.end(), d3)) continue;
                std::vector<double> rw(m, 0.0);
                const auto &mem = st.dof3_members[d3];
                for (size_t q = 0; q < mem.size(); ++q) {
                    const int p = pos(mem[q]);
                    if (p < 0) { rcs[fi] = BDDC_EINVAL; break; }
                    rw[p] = st.dof3_wts[d3][q];
                }
                if (rcs[fi]) break;
                B.insert(B.end(), rw.begin(), rw.end());
                ++nb;
            }
            if (rcs[fi] || std::count(fpos.begin(), fpos.end(), -1)) { rcs[fi] = BDDC_EINVAL; continue; }
            if (!side(j, ps, Hs, Ks) || !side(k, pt, Ht, Kt)) { rcs[fi] = BDDC_ESINGULAR; continue; }
            FaceInput in{m, Hs.data(), Ht.data(), Ks.data(), Kt.data(), Ds.data(), Dt.data(), floating[j] != 0,
                         floating[k] != 0, nb, B.data(), (int)fpos.size(), fpos.data()};
            rcs[fi] = face_rows(in, tau, max_per_face, res[fi], lobpcg_it);
        }
    };
    const unsigned nth = std::max(1u, std::min(16u, std::thread::hardware_concurrency()));
    std::vector<std::thread> pool;
    for (unsigned q = 1; q < nth; ++q) pool.emplace_back(worker);
    worker();
    for (auto &th : pool) th.join();
    for (size_t fi = 0; fi < faces.size(); ++fi) {
        if (rcs[fi]) {
            err = rcs[fi] == BDDC_EINVAL ? "level-2 face constraint outside the shared coarse DOFs"
                                         : "singular level-2 face problem";
            return rcs[fi];
        }
        if (!res[fi].lam.empty()) stats.lam_max = std::max(stats.lam_max, res[fi].lam[0]);
        const int m3 = faces[fi];
        for (const auto &row : res[fi].rows) extra.push_back(Level3Dof{st.dof3_members[m3], row, st.dof3_subs[m3]});
    }
    stats.added = (int)extra.size();
    stats.seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    return BDDC_OK;
}

}  // namespace bddc
