"""Two- and three-level BDDC preconditioner (Section 3.2).

One application maps an interface residual r to
    z = sum_i R_i^T D_i R_Bi (u_i + Phi_i R_Ci u_C)          (eq. averaging_subdomain_solves)
where
    K_C u_C = sum_i R_Ci^T Phi_i^T R_Bi^T D_i R_i r            (eq. coarse_problem)
    [K_i C_i^T; C_i 0] [u_i; mu_i] = [R_Bi^T D_i R_i r; 0]   (eq. localCorr)
K_i is the subdomain matrix over all its local unknowns (interior included),
C_i the constraint matrix of the subdomain's coarse DOFs, Phi_i the local coarse
basis (the constrained energy-minimising functions with C_i Phi_i = I),
K_C = sum_i R_Ci^T Phi_i^T K_i Phi_i R_Ci, and D_i the interface weights.

Coarse DOFs (Section 3.2: function values at selected interface nodes, averages
over faces).  The paper leaves the corner rule to the library; the reading used
here (also used by the GPU library, implemented independently):
  * S(n) = set of subdomains whose (kept) elements touch node n, for every node,
    Dirichlet nodes included;
  * a glob is a connected set (6-neighbour) of nodes with |S| >= 2 and equal S;
  * a face is a glob with |S| = 2; its coarse DOF is the arithmetic mean over its
    free nodes;
  * a free node with |S| >= 3 is a corner iff (its glob is a single node or it
    has at most one axis neighbour in its glob) and no axis neighbour m has
    S(m) a strict superset of S(n).
Weights (Section 3.2): 'card' = 1/|S(n)|, 'diag' = K_i(n,n)/sum_j K_j(n,n).

Three levels (Section 3.2, multilevel paragraph: the coarse problem is itself
preconditioned by BDDC with subdomains acting as elements).  The paper defers
the details to its reference; the reading used here:
  * the "elements" are the subdomains with element matrices K_Ci;
  * subdomains are grouped into subregions (given); S2(c) = subregions of the
    subdomains that share coarse DOF c; |S2| = 1 -> level-2 interior,
    |S2| >= 2 -> level-2 interface;
  * level-2 globs: level-2 interface DOFs with equal S2, connected through
    shared subdomains; faces (|S2| = 2) get an arithmetic-average constraint;
    corners are level-1 corners with |S2| >= 3 that pass the same endpoint /
    no-strict-superset test, neighbours being coarse DOFs sharing a subdomain;
  * level-2 weights are 'card' (1/|S2|); the level-3 problem is solved exactly
    (dense Cholesky);
  * adaptivity at level 2 (optional; Section 3.3 applied to the coarse
    problem, as adaptive multilevel BDDC does on every level): every level-2
    face (a glob shared by two subregions) gets the pencil of eq. eig-matrix
    with subregions in the role of subdomains, A_st built from the subregion
    Schur complements S2_j = K2_j / K2_j(interior) on the level-2 interface,
    the level-2 'card' weights in E_st and the shared level-3 DOFs in Pi; the
    rows of eq. c-def (same selection, restriction to the face and
    orthonormalisation as at level 1) become level-3 DOFs of kind
    "adaptive2", appended after the initial ones, each shared by the two
    subregions with the row's entries as weights;
  * one application: interior pre-solve, interface residual, level-2 BDDC on
    the interface, interior post-correction (harmonic extension).

Pure Neumann problem (no Dirichlet node; Section 2, the semidefinite case of
eq. systems, and Section 4.1, its closing paragraph): K, A and the coarsest
matrix (K_C for two levels, the level-3 matrix for three) are semidefinite,
their null spaces spanned by the constant function; the local constrained
problems stay nonsingular.  Reading: the coarsest problem is solved with the
Moore-Penrose pseudo-inverse (its plain definition), which is what a singular
coarse solve on consistent data needs; the constant itself is handled by the
deflation basis (dpcg.py).
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as sla
import scipy.sparse as sp
import scipy.sparse.csgraph as csg
import scipy.sparse.linalg as spla


# ---------------------------------------------------------------------------
# level-1 globs and coarse degrees of freedom
# ---------------------------------------------------------------------------

def node_globs(ss):
    """Return (glob id per node (-1 if |S|<2), key id per node) using 6-connectivity."""
    nx = ss.nx
    n1 = nx + 1
    n = ss.n_nodes
    keys = {}
    key = -np.ones(n, dtype=np.int64)
    for v in range(n):
        t = ss.node_subs[v]
        if len(t) >= 2:
            key[v] = keys.setdefault(t, len(keys))
    on = key >= 0
    idx = np.arange(n)
    ix, iy, iz = idx % n1, (idx // n1) % n1, idx // (n1 * n1)
    rows, cols = [], []
    for stride, coord in ((1, ix), (n1, iy), (n1 * n1, iz)):
        a = idx[(coord < nx)]
        b = a + stride
        m = on[a] & on[b] & (key[a] == key[b])
        rows.append(a[m])
        cols.append(b[m])
    r = np.concatenate(rows)
    c = np.concatenate(cols)
    G = sp.coo_matrix((np.ones(r.size), (r, c)), shape=(n, n))
    _, lab = csg.connected_components(G, directed=False)
    glob = np.where(on, lab, -1)
    # renumber globs compactly
    uniq = np.unique(glob[on])
    remap = -np.ones(glob.max() + 1 if glob.max() >= 0 else 1, dtype=np.int64)
    remap[uniq] = np.arange(uniq.size)
    glob = np.where(on, remap[np.maximum(glob, 0)], -1)
    return glob, key


def axis_neighbours(nx, v):
    n1 = nx + 1
    ix, iy, iz = v % n1, (v // n1) % n1, v // (n1 * n1)
    out = []
    if ix > 0: out.append(v - 1)
    if ix < nx: out.append(v + 1)
    if iy > 0: out.append(v - n1)
    if iy < nx: out.append(v + n1)
    if iz > 0: out.append(v - n1 * n1)
    if iz < nx: out.append(v + n1 * n1)
    return out


def coarse_dofs(ss, constraints=("corners", "faces"), all_corners=False):
    """List of coarse DOFs: dict(kind, nodes (free), wts, subs).

    ``all_corners`` turns every free interface node into a corner (a special
    case in which BDDC reproduces A^{-1} exactly).
    """
    dofs = []
    if all_corners:
        for v in ss.gamma:
            dofs.append(dict(kind="corner", nodes=np.array([v]), wts=np.array([1.0]),
                             subs=ss.node_subs[v]))
        return dofs
    glob, _ = node_globs(ss)
    ng = glob.max() + 1
    members = [[] for _ in range(ng)]
    for v in np.flatnonzero(glob >= 0):
        members[glob[v]].append(v)
    if "corners" in constraints:
        for v in ss.gamma:
            S = set(ss.node_subs[v])
            if len(S) < 3:
                continue
            g = glob[v]
            nb = axis_neighbours(ss.nx, v)
            in_glob = sum(1 for m in nb if glob[m] == g)
            if not (len(members[g]) == 1 or in_glob <= 1):
                continue
            if any(S < set(ss.node_subs[m]) for m in nb):
                continue
            dofs.append(dict(kind="corner", nodes=np.array([v]), wts=np.array([1.0]),
                             subs=ss.node_subs[v]))
    if "faces" in constraints:
        for g in range(ng):
            v0 = members[g][0]
            if len(ss.node_subs[v0]) != 2:
                continue
            fr = np.array(sorted(v for v in members[g] if ss.free[v]))
            if fr.size == 0:
                continue
            dofs.append(dict(kind="face", nodes=fr, wts=np.full(fr.size, 1.0 / fr.size),
                             subs=ss.node_subs[v0]))
    if "edges" in constraints:
        corner_nodes = {int(d["nodes"][0]) for d in dofs if d["kind"] == "corner"}
        for g in range(ng):
            v0 = members[g][0]
            if len(ss.node_subs[v0]) < 3:
                continue
            fr = np.array(sorted(v for v in members[g] if ss.free[v] and v not in corner_nodes))
            if fr.size < 2:
                continue
            dofs.append(dict(kind="edge", nodes=fr, wts=np.full(fr.size, 1.0 / fr.size),
                             subs=ss.node_subs[v0]))
    return dofs


def weights(ss, kind="diag"):
    """Per-subdomain interface weights D_i (partition of unity on Gamma)."""
    D = []
    if kind == "card":
        for d in ss.sub:
            D.append(1.0 / ss.mult[d["nodes_B"]])
        return D
    tot = np.zeros(ss.n_nodes)
    diags = []
    for d in ss.sub:
        kd = d["K"].diagonal()[d["Bpos"]]
        diags.append(kd)
        np.add.at(tot, d["nodes_B"], kd)
    for d, kd in zip(ss.sub, diags):
        D.append(kd / tot[d["nodes_B"]])
    return D


# ---------------------------------------------------------------------------
# generic "constrained local problem" used at levels 1 and 2
# ---------------------------------------------------------------------------

class _LocalSaddle:
    """[K C^T; C 0] over all local unknowns; constraints act on interface rows.

    Solves eq. localCorr for a right-hand side on the interface and returns the
    interface part of u; also gives the coarse basis Phi (RHS [0; I]).
    """

    def __init__(self, K, Bpos, C_B, dense=False):
        nloc = K.shape[0]
        nc = C_B.shape[0]
        Cfull = np.zeros((nc, nloc))
        Cfull[:, Bpos] = C_B
        self.Bpos = Bpos
        self.nloc = nloc
        self.nc = nc
        if dense:
            Kd = K if isinstance(K, np.ndarray) else K.toarray()
            M = np.block([[Kd, Cfull.T], [Cfull, np.zeros((nc, nc))]])
            self._lu = sla.lu_factor(M)
            self._solve = lambda rhs: sla.lu_solve(self._lu, rhs)
        else:
            M = sp.bmat([[sp.csc_matrix(K), sp.csc_matrix(Cfull.T)],
                         [sp.csc_matrix(Cfull), None]], format="csc")
            lu = spla.splu(M)
            self._solve = lambda rhs: lu.solve(np.asarray(rhs, dtype=np.float64))
        E = np.zeros((nloc + nc, max(nc, 1)))
        if nc:
            E[nloc:, :] = np.eye(nc)
            sol = self._solve(E[:, :nc]) if nc > 1 else self._solve(E[:, 0])[:, None]
            self.Phi_full = sol[:nloc, :]
        else:
            self.Phi_full = np.zeros((nloc, 0))
        self.Phi = self.Phi_full[Bpos, :]
        Kd = K if isinstance(K, np.ndarray) else K
        self.KC = self.Phi_full.T @ (Kd @ self.Phi_full) if nc else np.zeros((0, 0))

    def neumann(self, g):
        rhs = np.zeros(self.nloc + self.nc)
        rhs[self.Bpos] = g
        return self._solve(rhs)[self.Bpos]


# ---------------------------------------------------------------------------
# level 2 (coarse problem preconditioned by BDDC over subregions)
# ---------------------------------------------------------------------------

def level2_schur(K, B, I):
    """K(B, B) - K(B, I) K(I, I)^{-1} K(I, B), dense."""
    S = K[np.ix_(B, B)]
    if I.size:
        S = S - K[np.ix_(B, I)] @ np.linalg.solve(K[np.ix_(I, I)], K[np.ix_(I, B)])
    return S


class Level2:
    """M_2^{-1} approximating K_C^{-1}: BDDC with subdomains as elements."""

    def __init__(self, n_coarse, S1, is_corner, KC_loc, cidx, sub_to_subregion, is_adaptive=None, singular=False,
                 adaptive2=None):
        self.nC = n_coarse
        s2r = np.asarray(sub_to_subregion)
        self.n_sr = int(s2r.max()) + 1
        S2 = [tuple(sorted({int(s2r[i]) for i in S1[c]})) for c in range(n_coarse)]
        self.S2 = S2
        mult2 = np.array([len(t) for t in S2])
        # subregion-local DOF sets and assembled subregion matrices K2_j
        subs_of = [np.flatnonzero(s2r == j) for j in range(self.n_sr)]
        self.L = []
        self.K2 = []
        for j in range(self.n_sr):
            Lj = np.array(sorted({int(c) for i in subs_of[j] for c in cidx[i]}), dtype=np.int64)
            pos = {int(c): k for k, c in enumerate(Lj)}
            Kj = np.zeros((Lj.size, Lj.size))
            for i in subs_of[j]:
                p = np.array([pos[int(c)] for c in cidx[i]], dtype=np.int64)
                Kj[np.ix_(p, p)] += KC_loc[i]
            self.L.append(Lj)
            self.K2.append(Kj)
        # level-2 interface numbering and globs
        self.gamma2 = np.flatnonzero(mult2 >= 2)
        self.g2 = -np.ones(n_coarse, dtype=np.int64)
        self.g2[self.gamma2] = np.arange(self.gamma2.size)
        # incidence coarse DOF x subdomain -> neighbour relation (share a subdomain)
        n_sub = len(cidx)
        rows = np.concatenate([np.asarray(cidx[i]) for i in range(n_sub)]) if n_sub else np.zeros(0, int)
        cols = np.concatenate([np.full(len(cidx[i]), i) for i in range(n_sub)]) if n_sub else np.zeros(0, int)
        Bm = sp.csr_matrix((np.ones(rows.size), (rows, cols)), shape=(n_coarse, n_sub))
        Adj = (Bm @ Bm.T).tocsr()
        Adj.setdiag(0)
        Adj.eliminate_zeros()
        self.adj = Adj
        # adaptive face rows (Section 3.3) stay out of the level-2 globs: each
        # one on the level-2 interface is a level-3 unknown of its own, so the
        # operator does not depend on the rows' signs or on their basis
        adaptive = np.zeros(n_coarse, bool) if is_adaptive is None else np.asarray(is_adaptive, bool)
        keyid = {}
        key = -np.ones(n_coarse, dtype=np.int64)
        for c in self.gamma2:
            if not adaptive[c]:
                key[c] = keyid.setdefault(S2[c], len(keyid))
        Ac = Adj.tocoo()
        m = (key[Ac.row] >= 0) & (key[Ac.row] == key[Ac.col])
        Gg = sp.coo_matrix((np.ones(m.sum()), (Ac.row[m], Ac.col[m])), shape=(n_coarse, n_coarse))
        _, lab = csg.connected_components(Gg, directed=False)
        glob = np.where(key >= 0, lab, -1)
        members = {}
        for c in self.gamma2:
            if not adaptive[c]:
                members.setdefault(int(glob[c]), []).append(int(c))
        # level-2 coarse DOFs (level-3 unknowns)
        dofs3 = []
        for c in self.gamma2:
            if not is_corner[c] or mult2[c] < 3:
                continue
            nb = Adj.indices[Adj.indptr[c]:Adj.indptr[c + 1]]
            g = glob[c]
            in_glob = sum(1 for mm in nb if glob[mm] == g)
            if not (len(members[int(g)]) == 1 or in_glob <= 1):
                continue
            if any(set(S2[c]) < set(S2[mm]) for mm in nb):
                continue
            dofs3.append(dict(kind="corner", dofs=np.array([c]), wts=np.array([1.0]), subs=S2[c]))
        for c in self.gamma2:
            if adaptive[c]:
                dofs3.append(dict(kind="adaptive", dofs=np.array([c]), wts=np.array([1.0]), subs=S2[c]))
        for g, mem in members.items():
            if len(S2[mem[0]]) != 2:
                continue
            mem = np.array(sorted(mem))
            dofs3.append(dict(kind="face", dofs=mem, wts=np.full(mem.size, 1.0 / mem.size), subs=S2[mem[0]]))
        self.adapt2_info = []
        if adaptive2 is not None:
            new, self.adapt2_info = self._adaptive_level2(dofs3, mult2, *adaptive2)
            dofs3 = dofs3 + new
        self.dofs3 = dofs3
        self.n3 = len(dofs3)
        # per-subregion split, constraints, local saddle problems
        self.loc = []
        K3 = np.zeros((self.n3, self.n3))
        for j in range(self.n_sr):
            Lj = self.L[j]
            isB = mult2[Lj] >= 2
            Bpos = np.flatnonzero(isB)
            Ipos = np.flatnonzero(~isB)
            posB = {int(Lj[k]): t for t, k in enumerate(Bpos)}
            c3 = [k for k, d in enumerate(dofs3) if j in d["subs"]]
            C = np.zeros((len(c3), Bpos.size))
            for r, k in enumerate(c3):
                for c, w in zip(dofs3[k]["dofs"], dofs3[k]["wts"]):
                    C[r, posB[int(c)]] = w
            Kj = self.K2[j]
            sad = _LocalSaddle(Kj, Bpos, C, dense=True)
            D = 1.0 / mult2[Lj[Bpos]]
            d = dict(Bpos=Bpos, Ipos=Ipos, g2=self.g2[Lj[Bpos]], I_dofs=Lj[Ipos], B_dofs=Lj[Bpos],
                     KII=Kj[np.ix_(Ipos, Ipos)], KIB=Kj[np.ix_(Ipos, Bpos)], KBI=Kj[np.ix_(Bpos, Ipos)],
                     sad=sad, c3=np.array(c3, dtype=np.int64), D=D)
            d["KII_cho"] = sla.cho_factor(d["KII"]) if Ipos.size else None
            if len(c3):
                K3[np.ix_(d["c3"], d["c3"])] += sad.KC
            self.loc.append(d)
        self.K3 = K3
        self.singular = singular
        if singular:
            self.K3_pinv = np.linalg.pinv(K3, rcond=1e-10, hermitian=True) if self.n3 else None
        else:
            self.K3_cho = sla.cho_factor(K3) if self.n3 else None

    def _adaptive_level2(self, dofs3, mult2, tau, per_face):
        """Level-3 DOFs from the level-2 face pencils (eqs. eig-matrix, c-def
        with subregions as the subdomains)."""
        from types import SimpleNamespace

        from .adaptive import adaptive_dofs
        subs, D2, S2 = [], [], []
        for j in range(self.n_sr):
            Lj, Kj = self.L[j], self.K2[j]
            isB = mult2[Lj] >= 2
            B, I = np.flatnonzero(isB), np.flatnonzero(~isB)
            S = level2_schur(Kj, B, I)
            subs.append({"nodes_B": Lj[B]})                  # ascending coarse DOF ids
            D2.append(1.0 / mult2[Lj[B]])
            S2.append(0.5 * (S + S.T))
        view = SimpleNamespace(sub=subs)
        dv = [dict(kind=d["kind"], nodes=d["dofs"], wts=d["wts"], subs=d["subs"]) for d in dofs3]
        new, info = adaptive_dofs(view, D2, dv, tau, per_face, S_dense=S2)
        self.S2_dense, self.D2 = S2, D2
        return [dict(kind="adaptive2", dofs=d["nodes"], wts=d["wts"], subs=d["subs"]) for d in new], info

    def _kii(self, d, v):
        return sla.cho_solve(d["KII_cho"], v) if d["KII_cho"] is not None else np.zeros(0)

    def apply(self, rC):
        """u_C = M_2^{-1} r_C: pre-solve, interface BDDC with exact level 3, post-correction."""
        vI = []
        g = rC[self.gamma2].copy()
        for d in self.loc:                                   # 1. interior pre-solve
            v = self._kii(d, rC[d["I_dofs"]])
            vI.append(v)
            if v.size:
                g[d["g2"]] -= d["KBI"] @ v                   # 2. interface residual
        r3 = np.zeros(self.n3)                               # 3. level-2 BDDC on the interface
        us = []
        for d in self.loc:
            gj = d["D"] * g[d["g2"]]
            us.append(d["sad"].neumann(gj))
            if d["c3"].size:
                r3[d["c3"]] += d["sad"].Phi.T @ gj
        if not self.n3:
            u3 = np.zeros(0)
        else:
            u3 = self.K3_pinv @ r3 if self.singular else sla.cho_solve(self.K3_cho, r3)
        xG = np.zeros(self.gamma2.size)
        for d, u in zip(self.loc, us):
            w = u + (d["sad"].Phi @ u3[d["c3"]] if d["c3"].size else 0.0)
            xG[d["g2"]] += d["D"] * w
        uC = np.zeros(self.nC)
        uC[self.gamma2] = xG
        for d, v in zip(self.loc, vI):                       # 4. interior post-correction
            if v.size:
                uC[d["I_dofs"]] = v - self._kii(d, d["KIB"] @ xG[d["g2"]])
        return uC


# ---------------------------------------------------------------------------
# the preconditioner
# ---------------------------------------------------------------------------

class BDDC:
    """M^{-1} of Section 3.2 on the interface problem of a ``Substructuring``."""

    def __init__(self, ss, weight_kind="diag", constraints=("corners", "faces"),
                 sub_to_subregion=None, all_corners=False, adaptive=None, adaptive2=None):
        self.ss = ss
        self.dofs = coarse_dofs(ss, constraints, all_corners)
        self.D = weights(ss, weight_kind)
        self.adapt_info = []
        if adaptive is not None:
            # Section 3.3: face DOFs from eq. eig-matrix, appended after the
            # initial ones (adaptive = (tau, at most this many per face))
            from .adaptive import adaptive_dofs
            tau, per_face = adaptive
            new, self.adapt_info = adaptive_dofs(ss, self.D, self.dofs, tau, per_face)
            self.dofs = self.dofs + new
        self.nC = len(self.dofs)
        # per-subdomain constraints and local saddle problems (eq. localCorr)
        self.cidx = []
        self.loc = []
        S1 = [d["subs"] for d in self.dofs]
        is_corner = np.array([d["kind"] == "corner" for d in self.dofs], dtype=bool)
        is_adaptive = np.array([d["kind"] == "adaptive" for d in self.dofs], dtype=bool)
        for i, d in enumerate(ss.sub):
            posB = {int(v): k for k, v in enumerate(d["nodes_B"])}
            ci = [k for k, cd in enumerate(self.dofs) if i in cd["subs"]]
            C = np.zeros((len(ci), d["Bpos"].size))
            for r, k in enumerate(ci):
                for v, w in zip(self.dofs[k]["nodes"], self.dofs[k]["wts"]):
                    C[r, posB[int(v)]] = w
            self.cidx.append(np.array(ci, dtype=np.int64))
            self.loc.append(_LocalSaddle(d["K"], d["Bpos"], C))
        KC_loc = [s.KC for s in self.loc]
        self.three_level = sub_to_subregion is not None
        # no Dirichlet node: the constant function has zero energy
        self.singular = not bool((ss.used & ss.dir).any())
        if self.three_level:
            self.level2 = Level2(self.nC, S1, is_corner, KC_loc, self.cidx, sub_to_subregion, is_adaptive,
                                 self.singular, adaptive2)
        else:
            KC = np.zeros((self.nC, self.nC))
            for i, s in enumerate(self.loc):
                KC[np.ix_(self.cidx[i], self.cidx[i])] += s.KC
            self.KC = KC
            if self.singular:
                self.KC_pinv = np.linalg.pinv(KC, rcond=1e-10, hermitian=True) if self.nC else None
            else:
                self.KC_cho = sla.cho_factor(KC) if self.nC else None

    def coarse_solve(self, rC):
        if self.three_level:
            return self.level2.apply(rC)
        if not self.nC:
            return np.zeros(0)
        return self.KC_pinv @ rC if self.singular else sla.cho_solve(self.KC_cho, rC)

    def apply(self, r):
        """z = M^{-1} r (eqs. averaging_subdomain_solves, coarse_problem, localCorr)."""
        ss = self.ss
        rC = np.zeros(self.nC)
        us = []
        for i, d in enumerate(ss.sub):
            g = self.D[i] * r[d["gB"]]
            us.append(self.loc[i].neumann(g))
            if self.cidx[i].size:
                rC[self.cidx[i]] += self.loc[i].Phi.T @ g
        uC = self.coarse_solve(rC)
        z = np.zeros(ss.n_gamma)
        for i, d in enumerate(ss.sub):
            w = us[i] + (self.loc[i].Phi @ uC[self.cidx[i]] if self.cidx[i].size else 0.0)
            z[d["gB"]] += self.D[i] * w
        return z

    def counts(self):
        kinds = [d["kind"] for d in self.dofs]
        return dict(corners=kinds.count("corner"), faces=kinds.count("face"), edges=kinds.count("edge"),
                    adaptive=kinds.count("adaptive"))
