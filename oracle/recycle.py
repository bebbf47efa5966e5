"""Deflation basis by Krylov subspace recycling (Section 4.2).

Strategies (Table "bases"):
  B1  first R search vectors of the sequence, then fixed;
  B2  sliding window of the last R search vectors;
  B3  harmonic Ritz vectors of the R smallest harmonic Ritz values;
  B4  harmonic Ritz vectors of the R largest harmonic Ritz values (the paper's
      choice for BDDC, whose spectrum is bounded below by 1).

For B3/B4, with V = [W, P] (previous basis and the search directions p_j that
were multiplied by A in the last solve), the harmonic Ritz problem is
    V^T A M^{-1} A V y = theta V^T A V y                (eq. harmonicRitz)
Here both small matrices are formed EXPLICITLY: A and M^{-1} are applied to
every column (the paper builds them at low cost from quantities of the solve;
the explicit form is the plain definition and is used to check the cheap one).
Basis freezing follows eq. harmritzstopcrit with tolerance 1e-5 on the sorted
selected values.

Readings: (i) if dim V <= R every harmonic Ritz vector is kept; (ii) F = V^T A V
is eigen-decomposed first and directions with eigenvalue below 1e-12 * max are
dropped before the generalized problem is reduced to a standard one; (iii)
theta is sorted descending (B4) or ascending (B3) and compared elementwise
with the previous selection only when both have R entries; (iv) when the test
passes the newly computed basis is kept and no further updates are made.
"""
from __future__ import annotations

import numpy as np


def select(theta, R, strategy):
    """Indices of the harmonic Ritz values kept (Section 4.2, paragraphs B3 and
    B4): the R largest for B4, the R smallest for B3, ordered from the kept end
    of the spectrum (descending for B4, ascending for B3); all of them when
    there are at most R."""
    order = np.argsort(-theta, kind="stable") if strategy == "B4" else np.argsort(theta, kind="stable")
    return order[:R]


def ritz_change(theta_new, theta_old):
    """Left-hand side of eq. harmritzstopcrit: the 2-norm of the change of the
    selected (sorted) harmonic Ritz values relative to the 2-norm of the new
    ones."""
    return np.linalg.norm(theta_new - theta_old) / np.linalg.norm(theta_new)


class Recycler:
    def __init__(self, R, strategy="B4", freeze_tol=1e-5, drop_tol=1e-12):
        self.R = int(R)
        self.strategy = strategy
        self.freeze_tol = freeze_tol
        self.drop_tol = drop_tol
        self.W = None
        self.theta = None
        self.frozen = False
        self.freeze_step = None
        self.step = 0
        self.history = []

    def basis(self, n):
        if self.W is None or self.R == 0:
            return np.zeros((n, 0))
        return self.W

    @staticmethod
    def harmonic_ritz(V, apply_A, apply_M, drop_tol=1e-12):
        """Solve V^T A M^{-1} A V y = theta V^T A V y with explicit small matrices."""
        AV = np.column_stack([apply_A(V[:, c]) for c in range(V.shape[1])])
        MAV = np.column_stack([apply_M(AV[:, c]) for c in range(V.shape[1])])
        F = V.T @ AV
        G = AV.T @ MAV
        F = 0.5 * (F + F.T)
        G = 0.5 * (G + G.T)
        lam, U = np.linalg.eigh(F)
        keep = lam > drop_tol * lam.max()
        T = U[:, keep] / np.sqrt(lam[keep])
        theta, Z = np.linalg.eigh(T.T @ G @ T)
        return theta, T @ Z, F, G

    def update(self, P, apply_A, apply_M):
        """Build W^{(i)} after a solve whose search directions are the columns of P."""
        self.step += 1
        if self.R == 0 or self.frozen:
            return
        n = P.shape[0]
        W = self.basis(n)
        if self.strategy == "B1":
            if W.shape[1] < self.R:
                self.W = np.column_stack([W, P])[:, : self.R]
            return
        if self.strategy == "B2":
            self.W = np.column_stack([W, P])[:, -self.R:]
            return
        V = np.column_stack([W, P])
        if V.shape[1] == 0:
            return
        theta, Y, _, _ = self.harmonic_ritz(V, apply_A, apply_M, self.drop_tol)
        sel = select(theta, self.R, self.strategy)
        th = theta[sel]
        self.W = V @ Y[:, sel]
        self.history.append(th.copy())
        if self.theta is not None and th.size == self.R and self.theta.size == self.R:
            if ritz_change(th, self.theta) <= self.freeze_tol:
                self.frozen = True
                self.freeze_step = self.step
        self.theta = th
