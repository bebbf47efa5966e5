"""Pins of the oracle's substructuring and BDDC against brute force and theory."""
import numpy as np
import pytest

import workload
from oracle import q1
from oracle.bddc import BDDC, coarse_dofs
from oracle.substructure import Substructuring


def _problem(nx=8, sub=4, coef=None, group=0):
    e2s = workload.cube_partition(nx, sub)
    c = np.ones(nx ** 3) if coef is None else coef
    ss = Substructuring(nx, e2s, c)
    s2r = workload.cube_subregions(nx // sub, group) if group else None
    return ss, s2r


def _rand_coef(nx, sigma=1.0, seed=3):
    return np.exp(sigma * np.random.default_rng(seed).standard_normal(nx ** 3))


def _dense(op, n):
    return np.column_stack([op(e) for e in np.eye(n)])


# ---------------------------------------------------------------- substructuring

def test_schur_equals_global_elimination():
    nx = 8
    coef = _rand_coef(nx)
    ss, _ = _problem(nx, 4, coef)
    K = q1.assemble(nx, coef).toarray()
    fr = q1.free_nodes(nx)
    G = ss.gamma
    I = np.setdiff1d(fr, G)
    A_ref = K[np.ix_(G, G)] - K[np.ix_(G, I)] @ np.linalg.solve(K[np.ix_(I, I)], K[np.ix_(I, G)])
    np.testing.assert_allclose(ss.dense_A(), A_ref, rtol=0, atol=1e-13 * np.abs(A_ref).max())
    x = np.random.default_rng(0).standard_normal(ss.n_gamma)
    np.testing.assert_allclose(ss.apply_A(x), A_ref @ x, atol=1e-12 * np.abs(A_ref @ x).max())


def test_condense_solve_recover_equals_direct():
    nx = 8
    coef = _rand_coef(nx)
    ss, _ = _problem(nx, 4, coef)
    F = workload.rhs_sequence(nx, 1)[0]
    A = ss.dense_A()
    xg = np.linalg.solve(A, ss.condense(F))
    u = ss.recover(xg, F)
    ud = q1.direct_solve(nx, coef, F)[0]
    np.testing.assert_allclose(u, ud, atol=1e-12 * np.abs(ud).max())


def test_interface_size_structured():
    ss, _ = _problem(16, 8)
    assert ss.n_gamma == 784          # 3 planes of 17x17 nodes minus x=1 and overlaps
    for d in ss.sub:                   # a 8^3 subdomain touching the outflow face
        assert d["Bpos"].size in (200, 217)


# ---------------------------------------------------------------- coarse DOFs

def test_corner_and_face_counts_cube_lattice():
    # m^3 cube subdomains, Dirichlet face x=1: corners are lattice points shared by >= 3
    # subdomains and not on x=1: (m-1)^3 interior + 5 (m-1)^2 on the Neumann faces;
    # faces: 3 (m-1) m^2.
    for nx, sub in ((16, 8), (16, 4), (24, 8)):
        ss, _ = _problem(nx, sub)
        m = nx // sub
        dofs = coarse_dofs(ss)
        kinds = [d["kind"] for d in dofs]
        assert kinds.count("corner") == (m - 1) ** 3 + 5 * (m - 1) ** 2
        assert kinds.count("face") == 3 * (m - 1) * m * m


def test_corner_positions_c16():
    ss, _ = _problem(16, 8)
    corners = sorted(int(d["nodes"][0]) for d in coarse_dofs(ss) if d["kind"] == "corner")
    n1 = 17
    expect = sorted(x + n1 * (y + n1 * z) for (x, y, z) in
                    [(8, 8, 8), (8, 8, 0), (8, 8, 16), (8, 0, 8), (8, 16, 8), (0, 8, 8)])
    assert corners == expect
    faces = [d for d in coarse_dofs(ss) if d["kind"] == "face"]
    sizes = sorted(d["nodes"].size for d in faces)
    # faces normal to x: 8x8 free nodes incl. the Neumann boundary rows; faces normal to y/z
    # that touch x = 1 lose the Dirichlet column
    assert min(sizes) >= 49 and max(sizes) <= 64


# ---------------------------------------------------------------- BDDC pins

@pytest.mark.parametrize("kind", ["diag", "card"])
def test_partition_of_unity(kind):
    nx = 8
    ss, _ = _problem(nx, 4, _rand_coef(nx))
    M = BDDC(ss, kind)
    tot = np.zeros(ss.n_gamma)
    for i, d in enumerate(ss.sub):
        tot[d["gB"]] += M.D[i]
    np.testing.assert_allclose(tot, 1.0, atol=1e-14)


def test_diag_equals_card_for_unit_coefficient():
    ss, _ = _problem(8, 4)
    Md, Mc = BDDC(ss, "diag"), BDDC(ss, "card")
    for a, b in zip(Md.D, Mc.D):
        np.testing.assert_allclose(a, b, atol=1e-15)


def test_coarse_basis_satisfies_constraints():
    nx = 8
    ss, _ = _problem(nx, 4, _rand_coef(nx))
    M = BDDC(ss)
    for i in range(len(ss.sub)):
        loc = M.loc[i]
        # C_i Phi_i = I: rebuild C_i from the coarse DOF definitions
        posB = {int(v): k for k, v in enumerate(ss.sub[i]["nodes_B"])}
        C = np.zeros((M.cidx[i].size, ss.sub[i]["Bpos"].size))
        for r, k in enumerate(M.cidx[i]):
            for v, w in zip(M.dofs[k]["nodes"], M.dofs[k]["wts"]):
                C[r, posB[int(v)]] = w
        np.testing.assert_allclose(C @ loc.Phi, np.eye(M.cidx[i].size), atol=1e-12)
        # K_Ci equals Phi^T S_i Phi with S_i from dense elimination (interior is harmonic)
        S = ss.dense_S(i)
        np.testing.assert_allclose(loc.KC, loc.Phi.T @ S @ loc.Phi, rtol=1e-10, atol=1e-14)


def _spectrum(ss, M):
    A = ss.dense_A()
    Minv = _dense(M.apply, ss.n_gamma)
    return A, Minv, np.sort(np.linalg.eigvals(Minv @ A).real)


@pytest.mark.parametrize("three", [False, True])
def test_preconditioner_symmetric_and_lambda_min_ge_1(three):
    nx, sub = (16, 4) if three else (8, 4)
    coef = _rand_coef(nx, 0.7)
    ss, s2r = _problem(nx, sub, coef, group=2 if three else 0)
    M = BDDC(ss, "diag", sub_to_subregion=s2r)
    A, Minv, lam = _spectrum(ss, M)
    assert np.abs(Minv - Minv.T).max() <= 1e-12 * np.abs(Minv).max()
    assert lam[0] >= 1.0 - 1e-10, lam[:3]
    assert np.linalg.eigvalsh(0.5 * (Minv + Minv.T))[0] > 0


def test_three_level_coarse_is_spectrally_larger():
    # level-2 BDDC satisfies M_2^{-1} >= K_C^{-1}: eigenvalues of M_2^{-1} K_C are >= 1
    nx, sub = 16, 4
    ss, s2r = _problem(nx, sub, _rand_coef(nx, 0.5), group=2)
    M3 = BDDC(ss, sub_to_subregion=s2r)
    M2 = BDDC(ss)
    KC = M2.KC
    M2inv = _dense(M3.level2.apply, M3.nC)
    ev = np.sort(np.linalg.eigvals(M2inv @ KC).real)
    assert ev[0] >= 1 - 1e-10
    # so the three-level spectrum lies above the two-level one
    _, _, l3 = _spectrum(ss, M3)
    _, _, l2 = _spectrum(ss, M2)
    assert l3[-1] >= l2[-1] - 1e-10


def test_level2_counts_subregion_lattice():
    # 4^3 subdomains in 2^3 subregions: level-3 unknowns = 6 corners + 12 faces (like a
    # two-level 2x2x2 problem one level up)
    ss, s2r = _problem(16, 4, group=2)
    M = BDDC(ss, sub_to_subregion=s2r)
    kinds = [d["kind"] for d in M.level2.dofs3]
    assert kinds.count("corner") == 6 and kinds.count("face") == 12


def test_all_corners_gives_exact_inverse():
    nx = 8
    ss, _ = _problem(nx, 4, _rand_coef(nx))
    M = BDDC(ss, all_corners=True)
    A = ss.dense_A()
    Minv = _dense(M.apply, ss.n_gamma)
    np.testing.assert_allclose(Minv @ A, np.eye(ss.n_gamma), atol=1e-9)
