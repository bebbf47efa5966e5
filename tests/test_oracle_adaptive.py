"""Pins of the oracle's adaptive face constraints (Section 3.3, eqs. eig-matrix
and c-def) against facts that do not depend on the oracle's own code:

* the averaging E_st is a projection that fixes continuous pairs, Pi's range is
  the null space of the shared-DOF rows;
* a threshold no eigenvalue exceeds adds nothing and leaves M^{-1} unchanged;
* two subdomains (every shared node lies on the one face, so no part of c is
  dropped): once the selected rows are constraints, the largest eigenvalue of
  the same pencil is at most tau (Courant-Fischer on the constrained space);
* lambda_min(M^{-1}A) >= 1 still holds (Section 3.2) and the largest
  eigenvalue obeys the two-subdomain bound (1 + sqrt(tau))^2 of
  ||E w|| <= ||w|| + ||(I - E) w||; enrichment lowers the condition number.
"""
import numpy as np
import pytest

import workload
from oracle import adaptive as ad
from oracle.bddc import BDDC, coarse_dofs, weights
from oracle.substructure import Substructuring


def channel_problem(nx=6, contrast=1e4, right=1.0):
    """Two subdomains (x < 1/2, x > 1/2) crossed by four stiff channels along x;
    coefficients of the right half scaled by `right`."""
    c = workload.element_centroids(nx)
    e = np.arange(nx ** 3)
    ey, ez = (e // nx) % nx, e // (nx * nx)
    coef = np.where(np.isin(ey, (1, nx - 2)) & np.isin(ez, (1, nx - 2)), contrast, 1.0)
    e2s = (c[:, 0] > 0.5).astype(np.int32)
    return Substructuring(nx, e2s, coef * np.where(e2s == 1, right, 1.0))


def dense_spectrum(ss, M):
    A = ss.dense_A()
    n = ss.n_gamma
    Minv = np.column_stack([M.apply(np.eye(n)[:, j]) for j in range(n)])
    lam = np.linalg.eigvals(Minv @ A).real
    return np.sort(lam)


def test_pencil_pieces():
    ss = channel_problem()
    D = weights(ss, "diag")
    dofs = coarse_dofs(ss)
    E = ad.averaging_matrix(ss, D, 0, 1)
    np.testing.assert_allclose(E @ E, E, atol=1e-14)
    # a continuous pair (equal values on shared nodes) is fixed by E
    shared, ps, pt = ad.pair_maps(ss, 0, 1)
    ns = ss.sub[0]["nodes_B"].size
    g = np.random.default_rng(0).standard_normal(ss.n_nodes)
    w = np.concatenate([g[ss.sub[0]["nodes_B"]], g[ss.sub[1]["nodes_B"]]])
    np.testing.assert_allclose(E @ w, w, atol=1e-14)
    assert shared.size == ps.size == pt.size and shared.size > 0
    B = ad.shared_constraints(ss, dofs, 0, 1)
    Q, L, R = ad.face_pencil(ss, D, dofs, 0, 1, [ss.dense_S(i) for i in range(2)])
    np.testing.assert_allclose(B @ Q, 0, atol=1e-13)
    np.testing.assert_allclose(Q.T @ Q, np.eye(Q.shape[1]), atol=1e-13)
    assert Q.shape[1] == 2 * ns - B.shape[0]


def test_infinite_threshold_adds_nothing():
    ss = channel_problem()
    M0 = BDDC(ss)
    M1 = BDDC(ss, adaptive=(np.inf, 10))
    assert M1.counts()["adaptive"] == 0 and len(M1.adapt_info) == 1
    r = np.random.default_rng(1).standard_normal(ss.n_gamma)
    np.testing.assert_array_equal(M0.apply(r), M1.apply(r))


@pytest.mark.parametrize("tau", [2.0, 5.0])
def test_two_subdomain_face_bound(tau):
    ss = channel_problem()
    D = weights(ss, "diag")
    dofs = coarse_dofs(ss)
    S = [ss.dense_S(i) for i in range(2)]
    lam0, W = ad.face_eigen(ss, D, dofs, 0, 1, S)
    assert lam0[0] > tau                      # the channels make the pencil non-trivial
    new, info = ad.adaptive_dofs(ss, D, dofs, tau, max_per_face=1000, S_dense=S)
    assert info[0]["added"] == np.sum(lam0 > tau) == len(new)
    lam1, _ = ad.face_eigen(ss, D, dofs + new, 0, 1, S)
    assert lam1[0] <= tau * (1 + 1e-8)
    # c is antisymmetric on the shared nodes and zero elsewhere
    c = ad.constraint_covector(ss, D, dofs, 0, 1, S, W[:, 0])
    shared, ps, pt = ad.pair_maps(ss, 0, 1)
    ns = ss.sub[0]["nodes_B"].size
    np.testing.assert_allclose(c[ps], -c[ns + pt], atol=1e-10 * np.abs(c).max())
    other = np.setdiff1d(np.arange(c.size), np.concatenate([ps, ns + pt]))
    np.testing.assert_allclose(c[other], 0, atol=1e-10 * np.abs(c).max())


def test_two_subdomain_spectrum():
    ss = channel_problem()
    tau = 3.0
    lam_plain = dense_spectrum(ss, BDDC(ss))
    M = BDDC(ss, adaptive=(tau, 1000))
    lam = dense_spectrum(ss, M)
    assert M.counts()["adaptive"] > 0
    assert lam[0] >= 1 - 1e-10
    assert lam[-1] <= (1 + np.sqrt(tau)) ** 2 * (1 + 1e-8)
    assert lam[-1] < 0.5 * lam_plain[-1]


def test_two_subdomain_face_eigenvalue_is_the_condition_number():
    # with two subdomains the largest eigenvalue of the face pencil and that of
    # the dense M^{-1} A (built from the saddle-point solves, a separate
    # computation) coincide, before and after enrichment (unequal halves, so
    # that the weights differ from 1/2)
    ss = channel_problem(right=0.1)
    D = weights(ss, "diag")
    dofs = coarse_dofs(ss)
    S = [ss.dense_S(i) for i in range(2)]
    lam0, _ = ad.face_eigen(ss, D, dofs, 0, 1, S)
    np.testing.assert_allclose(dense_spectrum(ss, BDDC(ss))[-1], lam0[0], rtol=1e-8)
    M = BDDC(ss, adaptive=(100.0, 1000))
    lam1, _ = ad.face_eigen(ss, D, M.dofs, 0, 1, S)
    assert 1 <= M.counts()["adaptive"] < np.sum(lam0 > 1.5)
    np.testing.assert_allclose(dense_spectrum(ss, M)[-1], max(1.0, lam1[0]), rtol=1e-8)


def test_eight_subdomains_lognormal():
    s = workload.workload("tiny")
    coef = np.exp(2.0 * np.random.default_rng(5).standard_normal(s["nx"] ** 3))
    ss = Substructuring(s["nx"], s["elem_to_sub"], coef)
    lam_plain = dense_spectrum(ss, BDDC(ss))
    M = BDDC(ss, adaptive=(4.0, 10))
    lam = dense_spectrum(ss, M)
    assert M.counts()["adaptive"] > 0
    assert lam[0] >= 1 - 1e-10
    assert lam[-1] / lam[0] < lam_plain[-1] / lam_plain[0]


def test_three_levels_with_enriched_faces():
    # 4^3 subdomains in 2^3 subregions, log-normal coefficients: the enriched
    # level-1 faces join their face globs at level 2; M^{-1} stays symmetric
    # with lambda_min >= 1 and the spread shrinks
    from tests.test_oracle_bddc import _problem, _rand_coef, _spectrum
    ss, s2r = _problem(16, 4, _rand_coef(16, 2.5, seed=7), group=2)
    M0 = BDDC(ss, sub_to_subregion=s2r)
    M = BDDC(ss, sub_to_subregion=s2r, adaptive=(10.0, 10))
    assert M.counts()["adaptive"] > 0
    _, _, lam0 = _spectrum(ss, M0)
    _, Minv, lam = _spectrum(ss, M)
    assert np.abs(Minv - Minv.T).max() <= 1e-12 * np.abs(Minv).max()
    assert lam[0] >= 1 - 1e-10
    assert lam[-1] < lam0[-1]


def test_three_level_operator_depends_only_on_the_rows_span(monkeypatch):
    # reading of the level-2 treatment of adaptive rows: each row on the
    # level-2 interface is a level-3 unknown of its own, so M^{-1} must not
    # change when a row's sign is flipped or two rows of one face are
    # rotated into each other (same span)
    from tests.test_oracle_bddc import _problem, _rand_coef
    ss, s2r = _problem(16, 4, _rand_coef(16, 2.5, seed=7), group=2)
    orig = ad.adaptive_dofs
    M0 = BDDC(ss, sub_to_subregion=s2r, adaptive=(4.0, 10))
    new0, _ = orig(ss, weights(ss, "diag"), coarse_dofs(ss), 4.0, 10)
    by_face = {}
    for k, d in enumerate(new0):
        by_face.setdefault(tuple(d["nodes"]), []).append(k)
    pair = next(v for v in by_face.values() if len(v) >= 2)

    def mixed(*a, **kw):
        new, info = orig(*a, **kw)
        new = [dict(d) for d in new]
        new[0]["wts"] = -new[0]["wts"]
        c, s_ = np.cos(0.7), np.sin(0.7)
        i, j = pair[0], pair[1]
        wi, wj = new[i]["wts"].copy(), new[j]["wts"].copy()
        new[i]["wts"], new[j]["wts"] = c * wi + s_ * wj, -s_ * wi + c * wj
        return new, info
    monkeypatch.setattr(ad, "adaptive_dofs", mixed)
    M1 = BDDC(ss, sub_to_subregion=s2r, adaptive=(4.0, 10))
    assert M1.counts()["adaptive"] == M0.counts()["adaptive"] >= 2
    rng = np.random.default_rng(3)
    for _ in range(3):
        r = rng.standard_normal(ss.n_gamma)
        a, b = M0.apply(r), M1.apply(r)
        assert np.abs(a - b).max() <= 1e-10 * np.abs(a).max()
