"""Iterative substructuring (Section 3.1, eq. Sug).

The mesh is split into non-overlapping subdomains along element boundaries.
Unknowns touched by elements of exactly one subdomain are *interior*; unknowns
shared by several subdomains form the interface Gamma.  The global problem is
reduced to A x_Gamma = b with A the Schur complement of the interior unknowns;
A is never formed, only applied (Section 3.1: "only multiplications of vectors
by A are needed").

With K_i the matrix assembled from the elements of subdomain i over its local
free nodes, split into interior (I) and interface (B) blocks,
    S_i = K_BB - K_BI K_II^{-1} K_IB,     A = sum_i R_i^T S_i R_i,
    b   = F_Gamma - sum_i R_i^T K_BI K_II^{-1} F_I,
    x_I = K_II^{-1} (F_I - K_IB x_B)   (interior recovery).
``F`` is the assembled global load vector; interior rows of F belong to one
subdomain only, so the reduction above is exactly block elimination of the
global system.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

import workload
from . import q1


class Substructuring:
    """Interior/interface split and the interface Schur complement operator."""

    def __init__(self, nx, elem_to_sub, coef, elem_keep=None, dirichlet=None):
        self.nx = nx
        self.h = 1.0 / nx
        self.n_nodes = workload.n_nodes(nx)
        self.coef = np.asarray(coef, dtype=np.float64)
        keep = np.ones(nx ** 3, bool) if elem_keep is None else elem_keep.astype(bool)
        self.keep = keep
        self.dir = q1.dirichlet_mask(nx) if dirichlet is None else dirichlet.astype(bool)
        self.used = q1.used_nodes(nx, elem_keep)
        self.free = self.used & ~self.dir
        e2s = np.asarray(elem_to_sub)
        self.e2s = e2s
        self.n_sub = int(e2s[keep].max()) + 1
        en = workload.element_nodes(nx)
        self.en = en

        # S(n): set of subdomains whose elements touch node n (all used nodes)
        ke = np.flatnonzero(keep)
        pairs = np.unique(np.stack([en[ke].ravel(), np.repeat(e2s[ke], 8)], axis=1), axis=0)
        self.node_subs = [()] * self.n_nodes
        starts = np.flatnonzero(np.r_[True, pairs[1:, 0] != pairs[:-1, 0]])
        ends = np.r_[starts[1:], len(pairs)]
        for s, t in zip(starts, ends):
            self.node_subs[pairs[s, 0]] = tuple(int(v) for v in pairs[s:t, 1])
        self.mult = np.array([len(t) for t in self.node_subs])

        # global interface numbering: sorted node ids
        self.gamma = np.flatnonzero(self.free & (self.mult >= 2))
        self.n_gamma = self.gamma.size
        self.g_of_node = -np.ones(self.n_nodes, dtype=np.int64)
        self.g_of_node[self.gamma] = np.arange(self.n_gamma)

        K0 = q1.kref()
        self.sub = []
        for i in range(self.n_sub):
            elems = ke[e2s[ke] == i]
            loc_all = np.unique(en[elems].ravel())
            loc = loc_all[self.free[loc_all]]            # local free nodes, sorted
            pos = -np.ones(self.n_nodes, dtype=np.int64)
            pos[loc] = np.arange(loc.size)
            eloc = pos[en[elems]]                          # -1 for Dirichlet vertices
            rows = np.repeat(eloc, 8, axis=1).ravel()
            cols = np.tile(eloc, (1, 8)).ravel()
            vals = (self.coef[elems][:, None] * self.h * K0.ravel()[None, :]).ravel()
            ok = (rows >= 0) & (cols >= 0)
            Ki = sp.coo_matrix((vals[ok], (rows[ok], cols[ok])), shape=(loc.size, loc.size)).tocsc()
            isB = self.mult[loc] >= 2
            Bpos = np.flatnonzero(isB)
            Ipos = np.flatnonzero(~isB)
            d = dict(elems=elems, loc=loc, K=Ki, Bpos=Bpos, Ipos=Ipos,
                     nodes_B=loc[Bpos], nodes_I=loc[Ipos], gB=self.g_of_node[loc[Bpos]])
            d["KII"] = Ki[Ipos][:, Ipos].tocsc()
            d["KIB"] = Ki[Ipos][:, Bpos].tocsc()
            d["KBI"] = Ki[Bpos][:, Ipos].tocsc()
            d["KBB"] = Ki[Bpos][:, Bpos].tocsc()
            d["luII"] = spla.splu(d["KII"]) if Ipos.size else None
            self.sub.append(d)

    # -- Section 3.1: products with A only -----------------------------------
    def _kii_solve(self, d, v):
        if d["luII"] is None:
            return np.zeros(0)
        return d["luII"].solve(np.asarray(v, dtype=np.float64))

    def apply_S_local(self, i, xb):
        d = self.sub[i]
        y = d["KBB"] @ xb
        if d["Ipos"].size:
            y = y - d["KBI"] @ self._kii_solve(d, d["KIB"] @ xb)
        return y

    def apply_A(self, x):
        """A x = sum_i R_i^T S_i R_i x (Section 3.1, eq. Sug)."""
        y = np.zeros(self.n_gamma)
        for i, d in enumerate(self.sub):
            y[d["gB"]] += self.apply_S_local(i, x[d["gB"]])
        return y

    def condense(self, F):
        """b = F_Gamma - sum_i R_i^T K_BI K_II^{-1} F_I."""
        b = F[self.gamma].astype(np.float64).copy()
        for d in self.sub:
            if d["Ipos"].size:
                b[d["gB"]] -= d["KBI"] @ self._kii_solve(d, F[d["nodes_I"]])
        return b

    def recover(self, x, F):
        """Full nodal solution from the interface part: x_I = K_II^{-1}(F_I - K_IB x_B)."""
        u = np.zeros(self.n_nodes)
        u[self.gamma] = x
        for d in self.sub:
            if d["Ipos"].size:
                u[d["nodes_I"]] = self._kii_solve(d, F[d["nodes_I"]] - d["KIB"] @ x[d["gB"]])
        return u

    # -- dense forms, for brute-force checks on tiny meshes -------------------
    def dense_S(self, i):
        d = self.sub[i]
        KBB = d["KBB"].toarray()
        if not d["Ipos"].size:
            return KBB
        return KBB - d["KBI"].toarray() @ np.linalg.solve(d["KII"].toarray(), d["KIB"].toarray())

    def dense_A(self):
        A = np.zeros((self.n_gamma, self.n_gamma))
        for i, d in enumerate(self.sub):
            A[np.ix_(d["gB"], d["gB"])] += self.dense_S(i)
        return A
