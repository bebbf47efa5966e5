"""Adjoint gradient of a least-squares loss over a right-hand-side sequence.

Not a passage of the paper: the differentiated form of the same solve.  With
K(theta) = sum_e exp(theta_e) h Kref (scattered, Dirichlet rows removed),
u_k = K^{-1} F_k and L = sum_k ||u_k - t_k||^2 over the free nodes,
    lambda_k = K^{-1} dL/du_k = K^{-1} 2 (u_k - t_k)          (K is symmetric)
    dL/dtheta_e = - sum_k exp(theta_e) h lambda_{k,e}^T Kref u_{k,e}
    dL/dF_k = lambda_k.
Plain definition: every solve is a sparse direct solve of the global system.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse.linalg as spla

import workload
from . import q1


def element_gradient(nx, coef, lam, u, elem_keep=None):
    """g_e = - coef_e h sum_k lam_{k,e}^T Kref u_{k,e} (lam, u: (n_rhs, n_nodes), 0 off free nodes)."""
    h = 1.0 / nx
    en = workload.element_nodes(nx)
    K0 = q1.kref()
    g = np.zeros(nx ** 3)
    for k in range(lam.shape[0]):
        g -= coef * h * np.einsum("ev,vw,ew->e", lam[k][en], K0, u[k][en])
    if elem_keep is not None:
        g[~elem_keep.astype(bool)] = 0.0
    return g


def loss_and_grad(nx, theta, Fseq, targets, elem_keep=None):
    coef = np.exp(theta)
    K = q1.assemble(nx, coef, elem_keep)
    fr = q1.free_nodes(nx, elem_keep)
    lu = spla.splu(K[fr][:, fr].tocsc())
    n = workload.n_nodes(nx)
    U = np.zeros((len(Fseq), n))
    LAM = np.zeros_like(U)
    L = 0.0
    for k, F in enumerate(Fseq):
        U[k, fr] = lu.solve(F[fr])
        res = U[k, fr] - targets[k][fr]
        L += res @ res
        LAM[k, fr] = lu.solve(2.0 * res)
    return L, element_gradient(nx, coef, LAM, U, elem_keep), LAM, U


def loss(nx, theta, Fseq, targets, elem_keep=None):
    return loss_and_grad(nx, theta, Fseq, targets, elem_keep)[0]
