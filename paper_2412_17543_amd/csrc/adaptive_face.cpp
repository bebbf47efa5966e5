// Adaptive selection of face coarse DOFs (Section 3.3): one face problem
// in the jump space of its shared nodes (host code, float64).  The reduction
// is stated in adaptive.cpp.
#include <algorithm>
#include <cmath>
#include <vector>

#include "adaptive.h"

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

// Rayleigh-Ritz of the pencil (A, B) (n x n, row-major, A symmetric, B
// symmetric positive semidefinite) on the span of the s columns of S (n x s,
// row-major): the basis is made B-orthonormal through the eigenvectors of
// S^T B S, dropping directions below 1e-12 of its largest eigenvalue; the
// k largest Ritz values go to theta (descending) and their coefficient
// vectors to C (s x kk, column q for theta[q]).  Returns kk <= k.
int rayleigh_ritz(const std::vector<double> &A, const std::vector<double> &B, int n, const std::vector<double> &S,
                  int s, int k, std::vector<double> &theta, std::vector<double> &C) {
    const std::vector<double> GA = atb(S, ab(A, S, n, n, s), n, s, s);
    std::vector<double> GB = atb(S, ab(B, S, n, n, s), n, s, s);
    for (int i = 0; i < s; ++i)
        for (int j = i + 1; j < s; ++j) GB[(size_t)i * s + j] = GB[(size_t)j * s + i] = 0.5 * (GB[(size_t)i * s + j] + GB[(size_t)j * s + i]);
    std::vector<double> g, V;
    sym_eig(GB, s, g, V);
    const double gmax = s > 0 ? g[s - 1] : 0.0;
    std::vector<int> keep;
    for (int q = 0; q < s; ++q)
        if (gmax > 0.0 && g[q] > 1e-12 * gmax) keep.push_back(q);
    const int r = (int)keep.size();
    std::vector<double> T((size_t)s * r);
    for (int i = 0; i < s; ++i)
        for (int q = 0; q < r; ++q) T[(size_t)i * r + q] = V[(size_t)i * s + keep[q]] / std::sqrt(g[keep[q]]);
    std::vector<double> H = atb(T, ab(GA, T, s, s, r), s, r, r);
    for (int i = 0; i < r; ++i)
        for (int j = i + 1; j < r; ++j) H[(size_t)i * r + j] = H[(size_t)j * r + i] = 0.5 * (H[(size_t)i * r + j] + H[(size_t)j * r + i]);
    std::vector<double> h, Y;
    sym_eig(H, r, h, Y);
    const int kk = std::min(k, r);
    theta.assign(kk, 0.0);
    C.assign((size_t)s * kk, 0.0);
    for (int q = 0; q < kk; ++q) {
        const int e = r - 1 - q;
        theta[q] = h[e];
        for (int i = 0; i < s; ++i) {
            double v = 0.0;
            for (int t = 0; t < r; ++t) v += T[(size_t)i * r + t] * Y[(size_t)t * r + e];
            C[(size_t)i * kk + q] = v;
        }
    }
    return kk;
}

// The k largest eigenpairs of A x = theta B x by LOBPCG (Knyazev, 2001):
// every iteration is a Rayleigh-Ritz step on [X, R, P] (current vectors,
// their residuals A X - B X Theta, the previous directions), X the k best Ritz
// vectors, P their part from [R, P].  Starting block: cosines of spread
// frequencies; stops when every residual is below tol (|A x| + |theta| |B x|)
// or after max_it iterations.  theta descending, X (n x kk, row-major).
int lobpcg_top(const std::vector<double> &A, const std::vector<double> &B, int n, int k, int max_it, double tol,
               std::vector<double> &theta, std::vector<double> &X, int &iters) {
    k = std::min(k, n);
    iters = 0;
    if (k <= 0) { theta.clear(); X.clear(); return 0; }
    std::vector<double> S((size_t)n * k), C;
    for (int j = 0; j < k; ++j) {
        const double f = 1.0 + (double)j * (double)(n - 1) / (double)k;
        for (int i = 0; i < n; ++i) S[(size_t)i * k + j] = std::cos(M_PI * (i + 0.5) * f / n);
    }
    int kk = rayleigh_ritz(A, B, n, S, k, k, theta, C);
    X = ab(S, C, n, k, kk);
    std::vector<double> P;
    int np = 0;
    for (int it = 0; it < max_it && kk > 0; ++it) {
        const std::vector<double> AX = ab(A, X, n, n, kk), BX = ab(B, X, n, n, kk);
        std::vector<double> R((size_t)n * kk);
        bool done = true;
        for (int j = 0; j < kk; ++j) {
            double rn = 0.0, an = 0.0, bn = 0.0;
            for (int i = 0; i < n; ++i) {
                const double v = AX[(size_t)i * kk + j] - theta[j] * BX[(size_t)i * kk + j];
                R[(size_t)i * kk + j] = v;
                rn += v * v;
                an += AX[(size_t)i * kk + j] * AX[(size_t)i * kk + j];
                bn += BX[(size_t)i * kk + j] * BX[(size_t)i * kk + j];
            }
            if (std::sqrt(rn) > tol * (std::sqrt(an) + std::fabs(theta[j]) * std::sqrt(bn))) done = false;
            if (rn > 0.0)
                for (int i = 0; i < n; ++i) R[(size_t)i * kk + j] /= std::sqrt(rn);
        }
        if (done) break;
        const int s = kk + kk + np;
        S.assign((size_t)n * s, 0.0);
        for (int i = 0; i < n; ++i) {
            for (int j = 0; j < kk; ++j) S[(size_t)i * s + j] = X[(size_t)i * kk + j];
            for (int j = 0; j < kk; ++j) S[(size_t)i * s + kk + j] = R[(size_t)i * kk + j];
            for (int j = 0; j < np; ++j) S[(size_t)i * s + 2 * kk + j] = P[(size_t)i * np + j];
        }
        const int k2 = rayleigh_ritz(A, B, n, S, s, k, theta, C);
        if (k2 == 0) break;
        X = ab(S, C, n, s, k2);
        // P: the new vectors' components along [R, P]
        std::vector<double> Pn((size_t)n * k2, 0.0);
        for (int i = 0; i < n; ++i)
            for (int q = 0; q < k2; ++q) {
                double v = 0.0;
                for (int t = kk; t < s; ++t) v += S[(size_t)i * s + t] * C[(size_t)t * k2 + q];
                Pn[(size_t)i * k2 + q] = v;
            }
        for (int q = 0; q < k2; ++q) {                 // unit columns (their scale is free)
            double nn = 0.0;
            for (int i = 0; i < n; ++i) nn += Pn[(size_t)i * k2 + q] * Pn[(size_t)i * k2 + q];
            if (nn > 0.0)
                for (int i = 0; i < n; ++i) Pn[(size_t)i * k2 + q] /= std::sqrt(nn);
        }
        P.swap(Pn);
        np = k2;
        kk = k2;
        iters = it + 1;
    }
    return kk;
}

}  // namespace

int face_rows(const FaceInput &in, double tau, int max_rows, FaceOutput &out, int lobpcg_it, int *lobpcg_iters) {
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
    // eigenpairs, largest first: vectors y (jumps over the m shared nodes)
    int npair = 0;
    std::vector<double> Yv;                            // m x npair, row-major
    if (lobpcg_it > 0) {
        // LOBPCG for the max_rows largest pairs (Section 3.3: at most 10 per
        // face and 15 iterations in the paper)
        std::vector<double> th, Xc;
        int its = 0;
        npair = lobpcg_top(Lr, Pr, nz, std::max(1, max_rows), lobpcg_it, 1e-10, th, Xc, its);
        if (lobpcg_iters) *lobpcg_iters = its;
        out.lam = th;
        Yv = ab(Z, Xc, m, nz, npair);
    } else {
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
        // the vectors (a dropped row makes the next pair a candidate)
        const std::vector<double> ZT = ab(Z, T, m, nz, nk);            // m x nk
        npair = max_rows > 0 ? nk : 0;
        Yv.assign((size_t)m * npair, 0.0);
        for (int q = 0; q < npair; ++q) {
            const int i = nk - 1 - q;
            for (int k = 0; k < m; ++k) {
                double v = 0.0;
                for (int j = 0; j < nk; ++j) v += ZT[(size_t)k * nk + j] * Y[(size_t)j * nk + i];
                Yv[(size_t)k * npair + q] = v;
            }
        }
    }
    std::vector<std::vector<double>> basis;
    {
        std::vector<double> avg(in.nf, 1.0 / std::sqrt((double)std::max(in.nf, 1)));
        basis.push_back(avg);
    }
    for (int pi = 0; pi < npair && (int)out.rows.size() < max_rows; ++pi) {
        if (!(out.lam[pi] > tau)) break;
        std::vector<double> y(m, 0.0), Ly(m, 0.0), zt(nz, 0.0), g(m, 0.0);
        for (int k = 0; k < m; ++k) y[k] = Yv[(size_t)k * npair + pi];
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

}  // namespace bddc
