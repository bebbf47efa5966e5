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

}  // namespace bddc
