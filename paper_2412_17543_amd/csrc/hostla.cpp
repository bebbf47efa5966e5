// Small dense float64 linear algebra on the host: the R x R deflation Cholesky
// factor and the (R+l)-sized generalized eigenproblem of the recycling step
// (Section 4.2, eq. harmonicRitz).  Sizes are at most a few hundred.
#include <algorithm>
#include <cmath>

#include "internal.h"

namespace bddc {

// In-place lower Cholesky of a row-major n x n SPD matrix; false if not SPD.
bool cholesky(std::vector<double> &a, int n) {
    for (int j = 0; j < n; ++j) {
        double d = a[j * n + j];
        for (int k = 0; k < j; ++k) d -= a[j * n + k] * a[j * n + k];
        if (!(d > 0) || !std::isfinite(d)) return false;
        d = std::sqrt(d);
        a[j * n + j] = d;
        for (int i = j + 1; i < n; ++i) {
            double s = a[i * n + j];
            for (int k = 0; k < j; ++k) s -= a[i * n + k] * a[j * n + k];
            a[i * n + j] = s / d;
        }
        for (int i = 0; i < j; ++i) a[i * n + j] = 0.0;
    }
    return true;
}

void chol_solve(const std::vector<double> &l, int n, double *x) {
    for (int i = 0; i < n; ++i) {
        double s = x[i];
        for (int k = 0; k < i; ++k) s -= l[i * n + k] * x[k];
        x[i] = s / l[i * n + i];
    }
    for (int i = n - 1; i >= 0; --i) {
        double s = x[i];
        for (int k = i + 1; k < n; ++k) s -= l[k * n + i] * x[k];
        x[i] = s / l[i * n + i];
    }
}

// Symmetric eigendecomposition (Golub & Van Loan, Sections 8.3.1-8.3.3):
// Householder reduction to tridiagonal form with the orthogonal factor
// accumulated, then implicit QR steps with the Wilkinson shift on the
// unreduced trailing block until every subdiagonal entry is negligible.
// a: row-major symmetric n x n.  w: eigenvalues ascending; v: row-major,
// column j is the unit eigenvector of w[j].
void sym_eig(std::vector<double> a, int n, std::vector<double> &w, std::vector<double> &v) {
    auto A = [&](int i, int j) -> double & { return a[(size_t)i * n + j]; };
    v.assign((size_t)n * n, 0.0);
    auto Q = [&](int i, int j) -> double & { return v[(size_t)i * n + j]; };
    for (int i = 0; i < n; ++i) Q(i, i) = 1.0;
    // --- A = Q T Q^T, T tridiagonal: reflector H_k = I - 2 u u^T on k+1..n-1
    std::vector<double> u(n), p(n), wv(n);
    for (int k = 0; k + 2 < n; ++k) {
        double nx = 0.0;
        for (int i = k + 1; i < n; ++i) nx += A(i, k) * A(i, k);
        nx = std::sqrt(nx);
        if (nx == 0.0) continue;
        const double alpha = A(k + 1, k) > 0 ? -nx : nx;
        for (int i = k + 1; i < n; ++i) u[i] = A(i, k);
        u[k + 1] -= alpha;
        double nu = 0.0;
        for (int i = k + 1; i < n; ++i) nu += u[i] * u[i];
        nu = std::sqrt(nu);
        if (nu == 0.0) continue;
        for (int i = k + 1; i < n; ++i) u[i] /= nu;
        // A_sub <- H A_sub H = A_sub - 2 (u w^T + w u^T), w = A_sub u - (u^T A_sub u) u
        double upu = 0.0;
        for (int i = k + 1; i < n; ++i) {
            double t = 0.0;
            for (int j = k + 1; j < n; ++j) t += A(i, j) * u[j];
            p[i] = t;
            upu += u[i] * t;
        }
        for (int i = k + 1; i < n; ++i) wv[i] = p[i] - upu * u[i];
        for (int i = k + 1; i < n; ++i)
            for (int j = k + 1; j < n; ++j) A(i, j) -= 2.0 * (u[i] * wv[j] + wv[i] * u[j]);
        // column / row k: H x = alpha e_1
        A(k + 1, k) = A(k, k + 1) = alpha;
        for (int i = k + 2; i < n; ++i) A(i, k) = A(k, i) = 0.0;
        // Q <- Q H
        for (int i = 0; i < n; ++i) {
            double t = 0.0;
            for (int j = k + 1; j < n; ++j) t += Q(i, j) * u[j];
            for (int j = k + 1; j < n; ++j) Q(i, j) -= 2.0 * t * u[j];
        }
    }
    // --- implicit symmetric QR with Wilkinson shift on T (kept in `a`:
    // tridiagonal plus the bulge of the current step); the rotations act on
    // the rows of qt = Q^T
    const double eps = 2.220446049250313e-16;
    std::vector<double> qt((size_t)n * n);
    for (int i = 0; i < n; ++i)
        for (int j = 0; j < n; ++j) qt[(size_t)j * n + i] = Q(i, j);
    // rotation G(k, k+1) = [c s; -s c]: T <- G^T T G on the band, Q <- Q G
    auto rotate = [&](int k, int lo, int hi, double c, double s) {
        const int j0 = std::max(lo, k - 1), j1 = std::min(hi, k + 2);
        for (int j = j0; j <= j1; ++j) {       // columns k, k+1
            const double x = A(j, k), y = A(j, k + 1);
            A(j, k) = c * x - s * y;
            A(j, k + 1) = s * x + c * y;
        }
        for (int j = j0; j <= j1; ++j) {       // rows k, k+1
            const double x = A(k, j), y = A(k + 1, j);
            A(k, j) = c * x - s * y;
            A(k + 1, j) = s * x + c * y;
        }
        double *qk = &qt[(size_t)k * n], *qk1 = &qt[(size_t)(k + 1) * n];
        for (int i = 0; i < n; ++i) {
            const double x = qk[i], y = qk1[i];
            qk[i] = c * x - s * y;
            qk1[i] = s * x + c * y;
        }
    };
    // c, s with [c s; -s c]^T [x; z] = [r; 0]
    auto givens = [](double x, double z, double &c, double &s) {
        if (z == 0.0) { c = 1.0; s = 0.0; return; }
        if (std::fabs(z) > std::fabs(x)) {
            const double t = -x / z;
            s = 1.0 / std::sqrt(1.0 + t * t);
            c = s * t;
        } else {
            const double t = -z / x;
            c = 1.0 / std::sqrt(1.0 + t * t);
            s = c * t;
        }
    };
    int hi = n - 1;
    for (int guard = 0; hi > 0 && guard < 60 * n; ++guard) {
        for (int i = 0; i < hi; ++i)
            if (std::fabs(A(i + 1, i)) <= eps * (std::fabs(A(i, i)) + std::fabs(A(i + 1, i + 1))))
                A(i + 1, i) = A(i, i + 1) = 0.0;
        while (hi > 0 && A(hi, hi - 1) == 0.0) --hi;   // trailing diagonal part
        if (hi == 0) break;
        int lo = hi - 1;
        while (lo > 0 && A(lo, lo - 1) != 0.0) --lo;    // unreduced block [lo, hi]
        const double d = 0.5 * (A(hi - 1, hi - 1) - A(hi, hi));
        const double e = A(hi, hi - 1);
        const double mu = A(hi, hi) - e * e / (d + (d >= 0 ? 1.0 : -1.0) * std::sqrt(d * d + e * e));
        double x = A(lo, lo) - mu, z = A(lo + 1, lo);
        for (int k = lo; k < hi; ++k) {
            double c, s;
            givens(x, z, c, s);
            rotate(k, lo, hi, c, s);
            if (k > lo) A(k + 1, k - 1) = A(k - 1, k + 1) = 0.0;   // the chased bulge
            if (k + 1 < hi) {
                x = A(k + 1, k);
                z = A(k + 2, k);
            }
        }
    }
    std::vector<int> ord(n);
    for (int i = 0; i < n; ++i) ord[i] = i;
    std::sort(ord.begin(), ord.end(), [&](int x, int y) { return A(x, x) < A(y, y); });
    w.resize(n);
    std::vector<double> vs((size_t)n * n);
    for (int j = 0; j < n; ++j) {
        w[j] = A(ord[j], ord[j]);
        for (int i = 0; i < n; ++i) vs[(size_t)i * n + j] = qt[(size_t)ord[j] * n + i];
    }
    v.swap(vs);
}

}  // namespace bddc
