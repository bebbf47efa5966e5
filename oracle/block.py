"""Block deflated PCG: several right-hand sides with one matrix solved
together (the adjoint systems of the gradient, K lambda_k = dL/du_k, all with
the same BDDC and the same deflation basis).

Oracle code (test infrastructure only): dense float64 NumPy, nothing shared
with the GPU library.

The paper solves one system at a time (Algorithm 1); solving the s adjoint
systems of a sequence as one block is this project's extension, so the
method is taken from the block CG literature: O'Leary's block conjugate
gradients, in the breakdown-free form of Ji and Li (2017), which keeps the
search block P orthonormal and drops directions that have become linearly
dependent (columns that converged), combined with the deflation of
Algorithm 1 (every search direction A-orthogonal to W):

  X_0 = W (W^T A W)^{-1} W^T B          (x_{-1} = 0; Alg. 1 with a block)
  R_0 = B - A X_0
  P_{-1} = empty
  for i = 0, 1, ...
      stop when every column has ||r_j|| <= rtol ||b_j||   (eq. stopping_rhs)
      Z   = M^{-1} R_i
      Z  <- Z - W (W^T A W)^{-1} (A W)^T Z              (deflation)
      Y   = Z - P_{i-1} (P_{i-1}^T Q_{i-1})^{-1} Q_{i-1}^T Z    (block beta)
      P_i = orth(Y): the eigenvectors of Y^T Y with eigenvalue above
            1e-12 of the largest, scaled to an orthonormal basis of range(Y)
      Q_i = A P_i
      alpha = (P_i^T Q_i)^{-1} P_i^T R_i
      X_{i+1} = X_i + P_i alpha;  R_{i+1} = R_i - Q_i alpha

With one right-hand side this is PCG with its directions normalised, so the
iterates are those of Algorithm 1.
"""
from __future__ import annotations

import numpy as np


def orth(Y, drop=1e-12):
    """Orthonormal basis of range(Y) from the eigen-decomposition of Y^T Y
    (eigenvalues below `drop` times the largest are dropped)."""
    G = Y.T @ Y
    lam, V = np.linalg.eigh(0.5 * (G + G.T))
    if lam.size == 0 or lam[-1] <= 0:
        return Y[:, :0]
    keep = lam > drop * lam[-1]
    return Y @ (V[:, keep] / np.sqrt(lam[keep]))


def block_dpcg(apply_A, apply_M, B, W=None, rtol=1e-8, max_it=1000):
    """Solve A X = B (n x s).  apply_A / apply_M act on n x k blocks.
    Returns dict(x, iters, relres (recursive, per column), ranks (columns of
    P per iteration))."""
    n, s = B.shape
    if W is None:
        W = np.zeros((n, 0))
    AW = apply_A(W) if W.shape[1] else np.zeros((n, 0))
    WAW = W.T @ AW
    X = np.zeros((n, s))
    R = B.copy()
    if W.shape[1]:
        X = W @ np.linalg.solve(WAW, W.T @ B)
        R = B - apply_A(X)
    bn = np.linalg.norm(B, axis=0)
    P = np.zeros((n, 0))
    Q = np.zeros((n, 0))
    ranks = []
    it = 0
    while True:
        rn = np.linalg.norm(R, axis=0)
        if np.all(rn <= rtol * bn) or it >= max_it:
            break
        Z = apply_M(R)
        if W.shape[1]:
            Z = Z - W @ np.linalg.solve(WAW, AW.T @ Z)
        if P.shape[1]:
            Z = Z - P @ np.linalg.solve(P.T @ Q, Q.T @ Z)
        P = orth(Z)
        ranks.append(P.shape[1])
        if P.shape[1] == 0:
            break
        Q = apply_A(P)
        alpha = np.linalg.solve(P.T @ Q, P.T @ R)
        X = X + P @ alpha
        R = R - Q @ alpha
        it += 1
    return dict(x=X, iters=it, relres=np.linalg.norm(R, axis=0) / np.where(bn > 0, bn, 1.0), ranks=ranks)


def adjoint_block(solver, dLdu, rtol=1e-10, max_it=1000):
    """The adjoint solves of Appendix B step 1 as one block on an
    ``OracleSolver`` (its BDDC and current deflation basis): condense every
    dL/du_k, solve the block, recover the interiors.  Returns (lambda
    (s x n_nodes), iterations)."""
    ss = solver.ss
    if solver.null_vec is not None:
        raise ValueError("the block adjoint is not defined here for the pure Neumann problem")
    Bc = np.column_stack([ss.condense(g) for g in dLdu])
    W = solver.rec.basis(ss.n_gamma)
    A = lambda V: np.column_stack([ss.apply_A(v) for v in V.T]) if V.shape[1] else V
    M = lambda V: np.column_stack([solver.M.apply(v) for v in V.T]) if V.shape[1] else V
    res = block_dpcg(A, M, Bc, W if W.shape[1] else None, rtol, max_it)
    lam = np.array([ss.recover(res["x"][:, k], g) for k, g in enumerate(dLdu)])
    return lam, res
