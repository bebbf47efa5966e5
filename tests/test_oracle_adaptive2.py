"""Pins of the oracle's adaptivity at level 2 (Section 3.3 applied to the
coarse problem of the multilevel method, Section 3.2), with two subregions so
that every shared coarse DOF lies on the one level-2 face:

* the largest eigenvalue of M_2^{-1} K_C (the level-2 BDDC approximation of
  the coarse inverse, built column by column from its application: interior
  pre-solve, interface BDDC, exact level 3, harmonic post-correction) equals
  max(1, largest eigenvalue of the level-2 face pencil) -- the two-subdomain
  identity of BDDC, here with subregions as the subdomains and the K_Ci as
  elements -- before and after enrichment;
* once the selected rows are constraints, the largest eigenvalue of the same
  pencil is at most tau (Courant-Fischer on the constrained space);
* an infinite threshold adds nothing; M^{-1} stays symmetric with
  lambda_min >= 1 and the three-level spectrum's top comes down.
"""
import numpy as np
import pytest

import workload
from oracle import adaptive as ad
from oracle.bddc import BDDC, Level2
from oracle.substructure import Substructuring


def two_subregion_problem(nx=16, sub=4, sigma=2.0, seed=11):
    coef = np.exp(sigma * np.random.default_rng(seed).standard_normal(nx ** 3))
    ss = Substructuring(nx, workload.cube_partition(nx, sub), coef)
    m = nx // sub
    s = np.arange(m ** 3)
    s2r = ((s % m) >= m // 2).astype(np.int32)        # x < 1/2 | x > 1/2
    return ss, s2r


def coarse_matrices(M):
    """Dense K_C and M_2^{-1} (the latter applied to unit vectors)."""
    nC = M.nC
    KC = np.zeros((nC, nC))
    for i, s in enumerate(M.loc):
        KC[np.ix_(M.cidx[i], M.cidx[i])] += s.KC
    M2 = np.column_stack([M.level2.apply(e) for e in np.eye(nC)])
    return KC, M2


def level2_face(M):
    L2 = M.level2
    faces = [d for d in L2.dofs3 if d["kind"] == "face"]
    assert len(faces) == 1 and tuple(faces[0]["subs"]) == (0, 1)
    return faces[0]


def face_lambda(M, dofs3):
    from types import SimpleNamespace
    L2 = M.level2
    view = SimpleNamespace(sub=[{"nodes_B": L2.L[j][np.isin(L2.L[j], L2.gamma2)]} for j in range(2)])
    dv = [dict(kind=d["kind"], nodes=d["dofs"], wts=d["wts"], subs=d["subs"]) for d in dofs3]
    S2 = [L2.S2_dense[j] for j in range(2)]
    lam, _ = ad.face_eigen(view, L2.D2, dv, 0, 1, S2)
    return lam


def test_face_eigenvalue_is_the_coarse_condition_number():
    ss, s2r = two_subregion_problem()
    M0 = BDDC(ss, "diag", sub_to_subregion=s2r, adaptive2=(np.inf, 10))
    assert len(M0.level2.dofs3) == len(BDDC(ss, "diag", sub_to_subregion=s2r).level2.dofs3)
    level2_face(M0)
    lam0 = face_lambda(M0, M0.level2.dofs3)
    KC, M2 = coarse_matrices(M0)
    mu = np.sort(np.linalg.eigvals(M2 @ KC).real)
    assert mu[0] >= 1 - 1e-9
    np.testing.assert_allclose(mu[-1], max(1.0, lam0[0]), rtol=1e-8)
    assert lam0[0] > 1.5                       # the coefficients make the pencil non-trivial
    tau = 0.5 * (1.0 + lam0[0])
    M1 = BDDC(ss, "diag", sub_to_subregion=s2r, adaptive2=(tau, 1000))
    added = [d for d in M1.level2.dofs3 if d["kind"] == "adaptive2"]
    assert len(added) == np.sum(lam0 > tau) >= 1
    assert all(tuple(d["subs"]) == (0, 1) for d in added)
    lam1 = face_lambda(M1, M1.level2.dofs3)
    assert lam1[0] <= tau * (1 + 1e-8)          # Courant-Fischer
    KC1, M21 = coarse_matrices(M1)
    np.testing.assert_allclose(KC1, KC, rtol=0, atol=1e-12 * np.abs(KC).max())
    mu1 = np.sort(np.linalg.eigvals(M21 @ KC1).real)
    np.testing.assert_allclose(mu1[-1], max(1.0, lam1[0]), rtol=1e-8)


def test_infinite_threshold_keeps_the_operator():
    ss, s2r = two_subregion_problem()
    r = np.random.default_rng(2).standard_normal(ss.n_gamma)
    a = BDDC(ss, "diag", sub_to_subregion=s2r).apply(r)
    b = BDDC(ss, "diag", sub_to_subregion=s2r, adaptive2=(np.inf, 10)).apply(r)
    np.testing.assert_array_equal(a, b)


def test_three_level_spectrum_with_level2_rows():
    ss, s2r = two_subregion_problem()
    A = ss.dense_A()
    n = ss.n_gamma

    def spec(M):
        Minv = np.column_stack([M.apply(e) for e in np.eye(n)])
        assert np.abs(Minv - Minv.T).max() <= 1e-11 * np.abs(Minv).max()
        return np.sort(np.linalg.eigvals(Minv @ A).real)
    lam_plain = spec(BDDC(ss, "diag", sub_to_subregion=s2r))
    M = BDDC(ss, "diag", sub_to_subregion=s2r, adaptive2=(1.5, 1000))
    assert any(d["kind"] == "adaptive2" for d in M.level2.dofs3)
    lam = spec(M)
    assert lam[0] >= 1 - 1e-10
    assert lam[-1] < lam_plain[-1]
