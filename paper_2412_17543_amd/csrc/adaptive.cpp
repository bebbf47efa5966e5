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

namespace {

// Orthonormal basis of {x in R^m : B x = 0}, B (r x m, row-major) of full
// row rank: Householder QR of B^T, Z = the last m - r columns of Q.
std::vector<double> null_basis(const std::vector<double> &B, int r, int m) {
    std::vector<double> A((size_t)m * r);            // B^T, column-major by reflector
    for (int i = 0; i < r; ++i)
        for (int k = 0; k < m; ++k) A[(size_t)i * m + k] = B[(size_t)i * m + k];
    std::vector<std::vector<double>> vs;
    for (int i = 0; i < r && i < m; ++i) {
        double *a = &A[(size_t)i * m];
        double nx = 0.0;
        for (int k = i; k < m; ++k) nx += a[k] * a[k];
        nx = std::sqrt(nx);
        std::vector<double> v(m, 0.0);
        if (nx > 0.0) {
            const double alpha = a[i] > 0 ? -nx : nx;
            for (int k = i; k < m; ++k) v[k] = a[k];
            v[i] -= alpha;
            double nv = 0.0;
            for (int k = i; k < m; ++k) nv += v[k] * v[k];
            nv = std::sqrt(nv);
            if (nv > 0.0)
                for (int k = i; k < m; ++k) v[k] /= nv;
        }
        // apply H = I - 2 v v^T to the remaining columns
        for (int q = i + 1; q < r; ++q) {
            double *aq = &A[(size_t)q * m];
            double t = 0.0;
            for (int k = i; k < m; ++k) t += v[k] * aq[k];
            for (int k = i; k < m; ++k) aq[k] -= 2.0 * t * v[k];
        }
        vs.push_back(v);
    }
    const int nz = m - (int)vs.size();
    std::vector<double> Z((size_t)m * nz, 0.0);      // row-major m x nz
    for (int c = 0; c < nz; ++c) {
        std::vector<double> x(m, 0.0);
        x[(int)vs.size() + c] = 1.0;
        for (int i = (int)vs.size() - 1; i >= 0; --i) {  // Q e = H_1 ... H_r e
            const std::vector<double> &v = vs[i];
            double t = 0.0;
            for (int k = i; k < m; ++k) t += v[k] * x[k];
            for (int k = i; k < m; ++k) x[k] -= 2.0 * t * v[k];
        }
        for (int k = 0; k < m; ++k) Z[(size_t)k * nz + c] = x[k];
    }
    return Z;
}

// C = A^T B (A: p x q, B: p x r, row-major) -> q x r
std::vector<double> atb(const std::vector<double> &A, const std::vector<double> &B, int p, int q, int r) {
    std::vector<double> C((size_t)q * r, 0.0);
    for (int k = 0; k < p; ++k)
        for (int i = 0; i < q; ++i) {
            const double a = A[(size_t)k * q + i];
            if (a == 0.0) continue;
            for (int j = 0; j < r; ++j) C[(size_t)i * r + j] += a * B[(size_t)k * r + j];
        }
    return C;
}

// C = A B (A: p x q, B: q x r) -> p x r
std::vector<double> ab(const std::vector<double> &A, const std::vector<double> &B, int p, int q, int r) {
    std::vector<double> C((size_t)p * r, 0.0);
    for (int i = 0; i < p; ++i)
        for (int k = 0; k < q; ++k) {
            const double a = A[(size_t)i * q + k];
            if (a == 0.0) continue;
            for (int j = 0; j < r; ++j) C[(size_t)i * r + j] += a * B[(size_t)k * r + j];
        }
    return C;
}

}  // namespace

int face_rows(const FaceInput &in, double tau, int max_rows, FaceOutput &out) {
    const int m = in.m;
    out.lam.clear();
    out.rows.clear();
    if (m == 0) return 0;
    // left-hand matrix of the jump
    std::vector<double> L((size_t)m * m);
    std::vector<double> a(m), b(m);
    for (int k = 0; k < m; ++k) {
        const double s = in.Ds[k] + in.Dt[k];
        a[k] = in.Dt[k] / s;
        b[k] = in.Ds[k] / s;
    }
    for (int i = 0; i < m; ++i)
        for (int j = 0; j < m; ++j)
            L[(size_t)i * m + j] = a[i] * a[j] * in.Ks[(size_t)i * m + j] + b[i] * b[j] * in.Kt[(size_t)i * m + j];
    // right-hand matrix: P = H_s - H_s (H_s + H_t)^+ H_s; the sum is singular
    // only when both subdomains float (null space: constants), where the
    // consistent systems are solved with (H_s + H_t + eps 1 1^T)
    std::vector<double> Gm((size_t)m * m);
    double tr = 0.0;
    for (int e = 0; e < m * m; ++e) Gm[e] = in.Hs[e] + in.Ht[e];
    for (int k = 0; k < m; ++k) tr += Gm[(size_t)k * m + k];
    if (in.float_s && in.float_t) {
        const double eps = tr / ((double)m * m);
        for (int e = 0; e < m * m; ++e) Gm[e] += eps;
    }
    if (!cholesky(Gm, m)) return BDDC_ESINGULAR;
    std::vector<double> X((size_t)m * m);           // X = G^{-1} H_s, column by column
    {
        std::vector<double> col(m);
        for (int j = 0; j < m; ++j) {
            for (int i = 0; i < m; ++i) col[i] = in.Hs[(size_t)i * m + j];
            chol_solve(Gm, m, col.data());
            for (int i = 0; i < m; ++i) X[(size_t)i * m + j] = col[i];
        }
    }
    std::vector<double> P = ab(std::vector<double>(in.Hs, in.Hs + (size_t)m * m), X, m, m, m);
    for (int e = 0; e < m * m; ++e) P[e] = in.Hs[e] - P[e];
    for (int i = 0; i < m; ++i)
        for (int j = i + 1; j < m; ++j) {
            const double v = 0.5 * (P[(size_t)i * m + j] + P[(size_t)j * m + i]);
            P[(size_t)i * m + j] = P[(size_t)j * m + i] = v;
        }
    // jumps that keep the shared coarse DOFs continuous
    const int r = in.nb;
    const std::vector<double> Z = null_basis(std::vector<double>(in.B, in.B + (size_t)r * m), r, m);
    const int nz = m - std::min(r, m);
    if (nz == 0) return 0;
    std::vector<double> Lr = atb(Z, ab(L, Z, m, m, nz), m, nz, nz);
    std::vector<double> Pr = atb(Z, ab(P, Z, m, m, nz), m, nz, nz);
    std::vector<double> mu, V;
    sym_eig(Pr, nz, mu, V);
    const double mumax = *std::max_element(mu.begin(), mu.end());
    std::vector<int> keep;
    for (int i = 0; i < nz; ++i)
        if (mu[i] > 1e-12 * mumax) keep.push_back(i);
    const int nk = (int)keep.size();
    if (nk == 0) return 0;
    std::vector<double> T((size_t)nz * nk);
    for (int q = 0; q < nz; ++q)
        for (int j = 0; j < nk; ++j) T[(size_t)q * nk + j] = V[(size_t)q * nz + keep[j]] / std::sqrt(mu[keep[j]]);
    std::vector<double> H = atb(T, ab(Lr, T, nz, nz, nk), nz, nk, nk);
    for (int i = 0; i < nk; ++i)
        for (int j = i + 1; j < nk; ++j) {
            const double v = 0.5 * (H[(size_t)i * nk + j] + H[(size_t)j * nk + i]);
            H[(size_t)i * nk + j] = H[(size_t)j * nk + i] = v;
        }
    std::vector<double> lam, Y;
    sym_eig(H, nk, lam, Y);
    for (int i = nk - 1; i >= 0; --i) out.lam.push_back(lam[i]);
    // rows from the largest eigenvalues above tau
    const std::vector<double> ZT = ab(Z, T, m, nz, nk);            // m x nk
    std::vector<std::vector<double>> basis;
    {
        std::vector<double> avg(in.nf, 1.0 / std::sqrt((double)std::max(in.nf, 1)));
        basis.push_back(avg);
    }
    for (int i = nk - 1; i >= 0 && (int)out.rows.size() < max_rows; --i) {
        if (!(lam[i] > tau)) break;
        std::vector<double> y(m, 0.0), Ly(m, 0.0), zt(nz, 0.0), g(m, 0.0);
        for (int k = 0; k < m; ++k)
            for (int j = 0; j < nk; ++j) y[k] += ZT[(size_t)k * nk + j] * Y[(size_t)j * nk + i];
        for (int k = 0; k < m; ++k)
            for (int q = 0; q < m; ++q) Ly[k] += L[(size_t)k * m + q] * y[q];
        for (int c = 0; c < nz; ++c)
            for (int k = 0; k < m; ++k) zt[c] += Z[(size_t)k * nz + c] * Ly[k];
        for (int k = 0; k < m; ++k)
            for (int c = 0; c < nz; ++c) g[k] += Z[(size_t)k * nz + c] * zt[c];
        std::vector<double> row(in.nf);
        double n0 = 0.0;
        for (int q = 0; q < in.nf; ++q) {
            row[q] = g[in.fpos[q]];
            n0 += row[q] * row[q];
        }
        n0 = std::sqrt(n0);
        if (n0 == 0.0) continue;
        for (int pass = 0; pass < 2; ++pass)
            for (const auto &bv : basis) {
                double t = 0.0;
                for (int q = 0; q < in.nf; ++q) t += bv[q] * row[q];
                for (int q = 0; q < in.nf; ++q) row[q] -= t * bv[q];
            }
        double n1 = 0.0;
        for (double v : row) n1 += v * v;
        n1 = std::sqrt(n1);
        if (n1 < 1e-8 * n0) continue;
        for (double &v : row) v /= n1;
        basis.push_back(row);
        out.rows.push_back(row);
    }
    return 0;
}

int adaptive_faces(const Structure &st, const double *d_K, const std::vector<int64_t> &k_off, double tau,
                   int max_per_face, int32_t *d_status, hipStream_t s, std::vector<CoarseDof> &extra,
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
    double *d_work = nullptr, *d_out = nullptr;
    int32_t *d_perm = nullptr;
    FaceSchurDesc *d_desc = nullptr;
    auto cleanup = [&]() {
        if (d_work) (void)hipFree(d_work);
        if (d_out) (void)hipFree(d_out);
        if (d_perm) (void)hipFree(d_perm);
        if (d_desc) (void)hipFree(d_desc);
    };
    size_t max_m = 1;
    for (const auto &f : faces) max_m = std::max(max_m, (size_t)f.m);
    if (hipMalloc(&d_work, batch * per_job * 8) != hipSuccess || hipMalloc(&d_out, batch * 2 * max_m * max_m * 8) != hipSuccess ||
        hipMalloc(&d_perm, batch * max_nB * 4) != hipSuccess || hipMalloc(&d_desc, batch * sizeof(FaceSchurDesc)) != hipSuccess) {
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
        int maxn = 1;
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
            maxn = std::max(maxn, sh.nB);
        }
        if (hipMemcpyAsync(d_perm, perm.data(), nj * max_nB * 4, hipMemcpyHostToDevice, s) != hipSuccess ||
            hipMemcpyAsync(d_desc, desc.data(), nj * sizeof(FaceSchurDesc), hipMemcpyHostToDevice, s) != hipSuccess) {
            cleanup();
            err = "hipMemcpy failed";
            return BDDC_EHIP;
        }
        launch_face_schur(d_desc, (int)nj, maxn, d_status, s);
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
            rcs[fi] = face_rows(in, tau, max_per_face, res[fi]);
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
