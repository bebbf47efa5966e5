"""Q1 (trilinear) discretisation of the pressure-corrector Poisson problem.

The paper discretises the pressure with the Q1 part of Taylor-Hood Q2-Q1
hexahedra (Section 2) and solves K x = f with K SPD once a Dirichlet part of the
boundary exists (Section 2, the algebraic-system equation and the remark that K
is SPD for a non-empty outflow part).  Here the domain is the unit cube, the
Dirichlet ("outflow") part is the face x = 1 and every other face is Neumann.

The element matrix of -div(c grad u) on a cube of side h is c*h*Kref, with Kref
the unit-cube Q1 stiffness: 1/3 on the diagonal, 0 between vertices that differ
in one coordinate, -1/12 between vertices that differ in two or three.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp

import workload


def kref() -> np.ndarray:
    """8x8 unit-cube Q1 stiffness matrix, vertex v = a + 2b + 4c."""
    by_ndiff = {0: 1.0 / 3.0, 1: 0.0, 2: -1.0 / 12.0, 3: -1.0 / 12.0}
    K = np.empty((8, 8))
    for v in range(8):
        for w in range(8):
            K[v, w] = by_ndiff[bin(v ^ w).count("1")]
    return K


def dirichlet_mask(nx: int) -> np.ndarray:
    """Nodes on the face x = 1 (the outflow boundary with u = 0)."""
    n = np.arange(workload.n_nodes(nx))
    return (n % (nx + 1)) == nx


def used_nodes(nx: int, elem_keep: np.ndarray | None) -> np.ndarray:
    """Boolean mask of nodes touched by at least one kept element."""
    en = workload.element_nodes(nx)
    if elem_keep is not None:
        en = en[elem_keep.astype(bool)]
    m = np.zeros(workload.n_nodes(nx), dtype=bool)
    m[en.ravel()] = True
    return m


def assemble(nx: int, coef: np.ndarray, elem_keep: np.ndarray | None = None,
             elems: np.ndarray | None = None) -> sp.csr_matrix:
    """Global stiffness over ALL nodes (no boundary condition applied).

    K = sum_e coef_e * h * Kref scattered to the element's 8 nodes.  ``elems``
    restricts the sum to a subset of element indices (used for subdomain
    matrices K_i, Section 3.2: "local matrix assembled from elements in the
    i-th subdomain").
    """
    h = 1.0 / nx
    en_all = workload.element_nodes(nx)
    sel = np.arange(nx ** 3)
    if elem_keep is not None:
        sel = sel[elem_keep.astype(bool)[sel]]
    if elems is not None:
        sel = np.intersect1d(sel, elems)
    en = en_all[sel]
    K0 = kref()
    rows = np.repeat(en, 8, axis=1).ravel()
    cols = np.tile(en, (1, 8)).ravel()
    vals = (coef[sel][:, None] * h * K0.ravel()[None, :]).ravel()
    n = workload.n_nodes(nx)
    return sp.coo_matrix((vals, (rows, cols)), shape=(n, n)).tocsr()


def free_nodes(nx: int, elem_keep: np.ndarray | None = None,
               dirichlet: np.ndarray | None = None) -> np.ndarray:
    """Indices of unknowns: nodes used by kept elements, minus Dirichlet nodes."""
    d = dirichlet_mask(nx) if dirichlet is None else dirichlet.astype(bool)
    return np.flatnonzero(used_nodes(nx, elem_keep) & ~d)


def direct_solve(nx: int, coef: np.ndarray, F: np.ndarray, elem_keep=None, dirichlet=None) -> np.ndarray:
    """Plain definition of the result: u = K^{-1} F on the free nodes, 0 elsewhere."""
    import scipy.sparse.linalg as spla
    K = assemble(nx, coef, elem_keep)
    fr = free_nodes(nx, elem_keep, dirichlet)
    Kff = K[fr][:, fr].tocsc()
    u = np.zeros(workload.n_nodes(nx))
    F = np.atleast_2d(F)
    lu = spla.splu(Kff)
    out = np.zeros((F.shape[0], u.size))
    for k in range(F.shape[0]):
        out[k, fr] = lu.solve(F[k, fr])
    return out
