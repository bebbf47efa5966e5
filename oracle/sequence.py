"""A sequence of systems K x^{(k)} = F^{(k)} with one matrix (Section 2, Section 4.2).

For each right-hand side: condense to the interface (Section 3.1), run
deflated PCG (Algorithm 1) from the previous interface solution (the paper's
"x^prev" initial guess, Section 6.1) with the current deflation basis, recover
the interior unknowns, then update the basis (Section 4.2 recycling loop).
"""
from __future__ import annotations

import numpy as np

from .bddc import BDDC
from .dpcg import dpcg
from .recycle import Recycler
from .substructure import Substructuring


class OracleSolver:
    def __init__(self, nx, elem_to_sub, coef, elem_keep=None, sub_to_subregion=None,
                 weight_kind="diag", constraints=("corners", "faces"), R=0, strategy="B4",
                 freeze_tol=1e-5, stop="rhs", init_guess="prev", all_corners=False, reorth=False,
                 adaptive=None, restart_every=0, dirichlet=None, adaptive2=None):
        self.ss = Substructuring(nx, elem_to_sub, coef, elem_keep, dirichlet)
        self.M = BDDC(self.ss, weight_kind, constraints, sub_to_subregion, all_corners, adaptive, adaptive2)
        self.rec = Recycler(R, strategy, freeze_tol)
        self.stop = stop
        self.init_guess = init_guess
        self.reorth = reorth
        self.restart_every = restart_every
        self.x_prev = np.zeros(self.ss.n_gamma)
        # pure Neumann (Section 4.1): the constant interface vector joins W
        self.null_vec = None
        if self.M.singular:
            self.null_vec = np.ones(self.ss.n_gamma) / np.sqrt(self.ss.n_gamma)

    def reset(self):
        self.rec = Recycler(self.rec.R, self.rec.strategy, self.rec.freeze_tol)
        self.x_prev = np.zeros(self.ss.n_gamma)

    def solve(self, F, rtol=1e-8, max_it=1000, update=True):
        ss = self.ss
        b = ss.condense(F)
        W = self.rec.basis(ss.n_gamma)
        x0 = self.x_prev if self.init_guess == "prev" else np.zeros(ss.n_gamma)
        res = dpcg(ss.apply_A, self.M.apply, b, x0, W, rtol, max_it, self.stop, reorth=self.reorth,
                   restart_every=self.restart_every, null_vec=self.null_vec)
        self.x_prev = res["x"]
        if update:
            Ps = res["P"][res["seg_start"]:]            # the run after the last replacement
            P = np.column_stack(Ps) if Ps else np.zeros((ss.n_gamma, 0))
            self.rec.update(P, ss.apply_A, self.M.apply)
        res["u"] = ss.recover(res["x"], F)
        res["b"] = b
        return res

    def solve_sequence(self, Fseq, rtol=1e-8, max_it=1000):
        us, its, rr = [], [], []
        for F in Fseq:
            r = self.solve(F, rtol, max_it)
            us.append(r["u"])
            its.append(r["iters"])
            rr.append(r["true_relres"])
        return np.array(us), np.array(its), np.array(rr)
