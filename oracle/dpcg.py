"""Deflated preconditioned conjugate gradients (Section 4.1, Algorithm 1).

Steps, in the order and notation of Algorithm 1 (W may have zero columns, in
which case this is plain PCG):
    x_0 = x_{-1} + W (W^T A W)^{-1} W^T (b - A x_{-1})
    r_0 = b - A x_0
    z_0 = M^{-1} r_0
    mu_0 = (W^T A W)^{-1} W^T A z_0,   p_0 = z_0 - W mu_0
    for j = 1, 2, ...:
        alpha_{j-1} = r_{j-1}^T z_{j-1} / p_{j-1}^T A p_{j-1}
        x_j = x_{j-1} + alpha_{j-1} p_{j-1}
        r_j = r_{j-1} - alpha_{j-1} A p_{j-1}
        [optional: r_j -= W (W^T W)^{-1} W^T r_j]     (re-orthogonalisation)
        z_j = M^{-1} r_j
        beta_{j-1} = r_j^T z_j / r_{j-1}^T z_{j-1}
        mu_j = (W^T A W)^{-1} W^T A z_j
        p_j = z_j + beta_{j-1} p_{j-1} - W mu_j

Stopping (Section 5): ||r_j|| / ||b|| < tol (eq. stopping_rhs, the default) or
||r_j|| / ||r_0|| < tol (eq. stopping_residual).  Reading used here: r_j is the
recursively updated residual of the interface problem; the test is made on r_0
before the loop (zero iterations allowed) and after each residual update; the
iteration count is the number of loop passes (= products with A inside the
loop).  After exit the true residual b - A x is evaluated; if it does not meet
the tolerance the residual is replaced by it and the iteration continues
(counted), up to max_it.

Recycling after a residual replacement (a reading: Section 4.2 keeps "some of"
the search vectors and never meets a replacement): ``seg_start`` is the index of
the first search direction after the last replacement, so that the directions
offered for recycling, P[seg_start:], come from one unbroken run of Algorithm 1
with the same W.

``null_vec`` (Section 4.1, closing paragraph: for a semidefinite A with a
known null space, a basis vector of it is added as a column of W).  Reading:
such a column w0 (A w0 = 0) enters the projections of Algorithm 1 with the
Euclidean inner product, i.e. its "A W" column is w0 itself, so that
W^T A W stays nonsingular, mu_0 = w0^T z / w0^T w0 and every search direction
(and, from a guess orthogonal to it, the iterate) stays orthogonal to w0; the
other columns of W must be orthogonal to w0.

``restart_every`` (not in the paper; 0 = off) ends a run after that many
passes without convergence: the true residual is then evaluated and, unless it
meets the tolerance, replaces the recursive one and the iteration restarts
from line 5, as after a residual replacement.
"""
from __future__ import annotations

import numpy as np


def dpcg(apply_A, apply_M, b, x_init=None, W=None, rtol=1e-8, max_it=1000,
         stop="rhs", reorth=False, record=True, restart_every=0, null_vec=None):
    n = b.size
    if W is None:
        W = np.zeros((n, 0))
    AW = np.column_stack([apply_A(W[:, c]) for c in range(W.shape[1])]) if W.shape[1] else np.zeros((n, 0))
    if null_vec is not None:
        W = np.column_stack([null_vec, W])
        AW = np.column_stack([null_vec, AW])
    k = W.shape[1]
    WAW = W.T @ AW
    WAW = 0.5 * (WAW + WAW.T)

    def solve_small(v):
        return np.linalg.solve(WAW, v) if k else np.zeros(0)

    out = dict(alpha=[], beta=[], rho=[], d=[], mu=[], relres=[], P=[], AP=[],
               wtr=[], wtap=[], restarts=0, seg_start=0)
    nb = np.linalg.norm(b)
    x = np.zeros(n) if x_init is None else np.asarray(x_init, dtype=np.float64).copy()
    if nb == 0.0:
        out.update(x=np.zeros(n), iters=0, true_relres=0.0, r0norm=0.0)
        return out
    r = b - apply_A(x)
    if k:
        x = x + W @ solve_small(W.T @ r)                        # line 3
    r = b - apply_A(x)                                            # line 4
    r0n = np.linalg.norm(r)
    out["r0norm"] = r0n
    denom = nb if stop == "rhs" else r0n
    it = 0

    def converged(rr):
        return denom == 0.0 or np.linalg.norm(rr) / denom < rtol

    def start(rr):
        z = apply_M(rr)                                           # line 5
        mu = solve_small(AW.T @ z)                                # line 6
        p = z - W @ mu if k else z.copy()                         # line 7
        return z, mu, p

    out["relres"].append(np.linalg.norm(r) / nb)
    done = converged(r)
    while True:
        if not done:
            z, mu, p = start(r)
            rho = r @ z
            out["rho"].append(rho)
            out["mu"].append(mu)
            run_start = it
            while it < max_it:
                Ap = apply_A(p)
                d = p @ Ap
                alpha = rho / d                                   # line 9
                if record:
                    out["P"].append(p.copy())
                    out["AP"].append(Ap.copy())
                out["alpha"].append(alpha)
                out["d"].append(d)
                x = x + alpha * p                                 # line 10
                r = r - alpha * Ap                                # line 11
                if reorth and k:
                    r = r - W @ np.linalg.solve(W.T @ W, W.T @ r)  # line 12
                it += 1
                out["relres"].append(np.linalg.norm(r) / nb)
                if k:
                    # rounding in W^T r stays at eps*||r_0||, so normalise by ||r_0||
                    out["wtr"].append(np.linalg.norm(W.T @ r) / (np.linalg.norm(W) * r0n))
                    out["wtap"].append(np.linalg.norm(AW.T @ p) / (np.linalg.norm(AW) * np.linalg.norm(p)))
                if converged(r) or 0 < restart_every <= it - run_start:
                    break
                z = apply_M(r)                                    # line 13
                rho_new = r @ z
                beta = rho_new / rho                              # line 14
                mu = solve_small(AW.T @ z)                        # line 15
                p = z + beta * p - (W @ mu if k else 0.0)         # line 16
                out["beta"].append(beta)
                out["rho"].append(rho_new)
                out["mu"].append(mu)
                rho = rho_new
        true_r = b - apply_A(x)
        tr = np.linalg.norm(true_r) / nb
        if converged(true_r) or it >= max_it:
            break
        r = true_r                                                # residual replacement
        out["restarts"] += 1
        out["seg_start"] = len(out["alpha"])
        done = False
    out.update(x=x, iters=it, true_relres=tr)
    return out


def lanczos_ritz(alpha, beta):
    """Eigenvalues of the CG Lanczos tridiagonal T (Ritz values of M^{-1}A).

    T_jj = 1/alpha_j + beta_{j-1}/alpha_{j-1},  T_{j,j+1} = sqrt(beta_j)/alpha_j.
    """
    m = len(alpha)
    if m == 0:
        return np.zeros(0)
    T = np.zeros((m, m))
    for j in range(m):
        T[j, j] = 1.0 / alpha[j] + (beta[j - 1] / alpha[j - 1] if j > 0 else 0.0)
        if j + 1 < m:
            T[j, j + 1] = T[j + 1, j] = np.sqrt(beta[j]) / alpha[j]
    return np.linalg.eigvalsh(T)
