"""Adaptive selection of face coarse degrees of freedom (Section 3.3, eqs.
eig-matrix, global-S and c-def).

Oracle code (test infrastructure only): dense FP64, written from the paper's
definitions; nothing here is shared with the GPU library.

For a face glob shared by subdomains s and t, the unknowns of the pair are
w = (w_s, w_t), the interface unknowns of both subdomains in their own order,
and
  A_st  = blockdiag(S_s, S_t), the local Schur complements (eq. global-S);
  E_st  = the averaging that makes the pair continuous: on every free node
          shared by s and t both copies are replaced by
          (D_s w_s + D_t w_t) / (D_s + D_t); every other unknown is kept;
  Pi    = the orthogonal projector onto the pairs whose initial coarse DOFs
          shared by s and t (corners, face averages, earlier adaptive rows)
          take equal values on both sides.
The pencil  Pi (I-E)^T A (I-E) Pi w = lambda Pi A Pi w  (eq. eig-matrix) is
solved on range(Pi) with the null space of Pi A Pi removed (directions whose
eigenvalue of the reduced right-hand matrix is below 1e-12 of its largest).
Every eigenvector with lambda > tau, largest first and at most
`max_per_face` of them, gives the covector c = w^T Pi (I-E)^T A (I-E) Pi
(eq. c-def).  Its entries on the s-copies of the face's free nodes (c is
antisymmetric on shared nodes, c_t = -c_s) are orthonormalised against the
face's existing rows (Gram-Schmidt, twice) and become one new coarse DOF of
both s and t; a row whose norm after the projection is below 1e-8 of the
norm of the face part is dropped.  The same functions serve level 2 (the
coarse problem's faces between subregions; bddc.Level2), with subregions as
the subdomains and coarse DOFs as the nodes.

Section 3.3 leaves Pi, E_st and the restriction of c to its reference; the
reading above is the one the GPU library implements as well.
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as sla


def pair_maps(ss, s, t):
    """Positions of the nodes shared by s and t in both interface lists."""
    ns, nt = ss.sub[s]["nodes_B"], ss.sub[t]["nodes_B"]
    shared = np.intersect1d(ns, nt)
    ps = np.searchsorted(ns, shared)
    pt = np.searchsorted(nt, shared)
    return shared, ps, pt


def averaging_matrix(ss, D, s, t):
    """E_st over the pair's unknowns (n_s + n_t square)."""
    ns, nt = ss.sub[s]["nodes_B"].size, ss.sub[t]["nodes_B"].size
    _, ps, pt = pair_maps(ss, s, t)
    E = np.eye(ns + nt)
    ds, dt = D[s][ps], D[t][pt]
    ws, wt = ds / (ds + dt), dt / (ds + dt)
    for k in range(ps.size):
        i, j = ps[k], ns + pt[k]
        E[i, i], E[i, j] = ws[k], wt[k]
        E[j, i], E[j, j] = ws[k], wt[k]
    return E


def shared_constraints(ss, dofs, s, t):
    """Rows B with B w = 0 iff every coarse DOF shared by s and t agrees."""
    ns, nt = ss.sub[s]["nodes_B"], ss.sub[t]["nodes_B"]
    rows = []
    for d in dofs:
        if s in d["subs"] and t in d["subs"]:
            r = np.zeros(ns.size + nt.size)
            r[np.searchsorted(ns, d["nodes"])] += d["wts"]
            r[ns.size + np.searchsorted(nt, d["nodes"])] -= d["wts"]
            rows.append(r)
    return np.array(rows).reshape(len(rows), ns.size + nt.size)


def face_pencil(ss, D, dofs, s, t, S_dense):
    """Return (Q, L, R): Q an orthonormal basis of range(Pi) and the reduced
    matrices L = Q^T (I-E)^T A (I-E) Q, R = Q^T A Q of eq. eig-matrix."""
    A = sla.block_diag(S_dense[s], S_dense[t])
    E = averaging_matrix(ss, D, s, t)
    B = shared_constraints(ss, dofs, s, t)
    Q = sla.null_space(B) if B.shape[0] else np.eye(A.shape[0])
    J = (np.eye(A.shape[0]) - E) @ Q
    L = J.T @ A @ J
    R = Q.T @ A @ Q
    return Q, 0.5 * (L + L.T), 0.5 * (R + R.T)


def face_eigen(ss, D, dofs, s, t, S_dense, drop_tol=1e-12):
    """Eigenpairs of eq. eig-matrix on range(Pi) minus the null space of the
    right-hand matrix: (lambda descending, w in the pair space as columns)."""
    Q, L, R = face_pencil(ss, D, dofs, s, t, S_dense)
    mu, V = np.linalg.eigh(R)
    keep = mu > drop_tol * mu.max()
    T = V[:, keep] / np.sqrt(mu[keep])
    lam, Y = np.linalg.eigh(T.T @ L @ T)
    order = np.argsort(lam)[::-1]
    return lam[order], Q @ (T @ Y[:, order])


def constraint_covector(ss, D, dofs, s, t, S_dense, w):
    """c = w^T Pi (I-E)^T A (I-E) Pi (eq. c-def) for a pair vector w."""
    A = sla.block_diag(S_dense[s], S_dense[t])
    E = averaging_matrix(ss, D, s, t)
    B = shared_constraints(ss, dofs, s, t)
    n = A.shape[0]
    if B.shape[0]:
        Pi = np.eye(n) - B.T @ np.linalg.solve(B @ B.T, B)
    else:
        Pi = np.eye(n)
    J = (np.eye(n) - E) @ Pi
    return (J.T @ A @ J).T @ w


def adaptive_dofs(ss, D, dofs, tau, max_per_face=10, S_dense=None):
    """New coarse DOFs for every face of `dofs` (the list is not changed).

    Returns (new DOFs, per-face records (s, t, eigenvalues descending, rows
    added)).
    """
    if S_dense is None:
        S_dense = [ss.dense_S(i) for i in range(ss.n_sub)]
    new, info = [], []
    for d in dofs:
        if d["kind"] != "face":
            continue
        s, t = d["subs"]
        lam, W = face_eigen(ss, D, dofs, s, t, S_dense)
        ns = ss.sub[s]["nodes_B"]
        fpos = np.searchsorted(ns, d["nodes"])
        basis = [d["wts"] / np.linalg.norm(d["wts"])]
        added = 0
        for ell in range(min(max_per_face, lam.size)):
            if not lam[ell] > tau:
                break
            c = constraint_covector(ss, D, dofs, s, t, S_dense, W[:, ell])
            row = c[fpos].copy()
            nrm = np.linalg.norm(row)
            if nrm == 0.0:
                continue
            for _ in range(2):
                for b in basis:
                    row -= (b @ row) * b
            if np.linalg.norm(row) < 1e-8 * nrm:
                continue
            row /= np.linalg.norm(row)
            basis.append(row)
            new.append(dict(kind="adaptive", nodes=d["nodes"].copy(), wts=row, subs=d["subs"]))
            added += 1
        info.append(dict(s=s, t=t, lam=lam, added=added))
    return new, info
