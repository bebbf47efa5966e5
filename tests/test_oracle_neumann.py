"""Pins of the pure Neumann case (Section 2: K only semidefinite without an
outflow part, its null space the constants; Section 4.1, closing paragraph:
the constant vector is added to the deflation basis).

Checked against facts fixed by the mathematics:
  * the constant function is in the null space of K, of the interface Schur
    complement A and of the coarse matrix (the coarse basis reproduces it);
  * with a consistent right-hand side the solution is unique up to a
    constant: the oracle's DPCG/BDDC solution differs from the minimum-norm
    solution of K u = F (dense, on a small mesh) by a constant only;
  * the iteration stays orthogonal to the constant interface vector (it is
    in W), and on the complement of the constants BDDC keeps
    lambda_min(M^{-1} A) >= 1 (two and three levels).
"""
import numpy as np
import pytest

import workload
from oracle import q1
from oracle.bddc import BDDC
from oracle.dpcg import dpcg
from oracle.sequence import OracleSolver
from oracle.substructure import Substructuring


def _setup(name):
    s = workload.workload(name)
    ss = Substructuring(s["nx"], s["elem_to_sub"], s["coef"], dirichlet=s["node_dirichlet"].astype(bool))
    M = BDDC(ss, sub_to_subregion=s["sub_to_subregion"])
    return s, ss, M


@pytest.mark.parametrize("name", ["c16n", "tiny3n"])
def test_null_space_is_the_constant(name):
    s, ss, M = _setup(name)
    assert M.singular
    one = np.ones(ss.n_gamma)
    assert np.abs(ss.apply_A(one)).max() < 1e-12 * np.abs(ss.apply_A(np.arange(ss.n_gamma, dtype=float))).max()
    K = q1.assemble(s["nx"], s["coef"])
    assert np.abs(K @ np.ones(K.shape[0])).max() < 1e-13
    if not M.three_level:
        assert np.abs(M.KC @ np.ones(M.nC)).max() < 1e-12 * np.abs(M.KC).max()


@pytest.mark.parametrize("name", ["c16n", "tiny3n"])
def test_solution_unique_up_to_a_constant(name):
    s, ss, M = _setup(name)
    nx = s["nx"]
    F = workload.consistent_neumann(nx, workload.rhs_sequence(nx, 2))
    assert np.abs(F.sum(axis=1)).max() < 1e-13 * np.abs(F).sum()
    o = OracleSolver(nx, s["elem_to_sub"], s["coef"], sub_to_subregion=s["sub_to_subregion"], R=4,
                     dirichlet=s["node_dirichlet"].astype(bool))
    us, its, rr = o.solve_sequence(F, 1e-10)
    assert (rr < 1e-10).all()
    Kd = q1.assemble(nx, s["coef"]).toarray()
    for k in range(2):
        ud = np.linalg.lstsq(Kd, F[k], rcond=None)[0]          # minimum-norm solution
        d = us[k] - ud
        assert np.abs(d - d.mean()).max() < 1e-8 * np.abs(ud).max()
        assert np.abs(Kd @ us[k] - F[k]).max() < 1e-8 * np.abs(F[k]).max()
    # the iterate never leaves the complement of the constant interface vector
    b = ss.condense(F[1])
    res = dpcg(ss.apply_A, M.apply, b, rtol=1e-10, null_vec=o.null_vec)
    assert abs(res["x"].sum()) < 1e-10 * np.abs(res["x"]).sum()
    P = np.column_stack(res["P"])
    assert np.abs(P.sum(axis=0)).max() < 1e-10 * np.abs(P).max() * ss.n_gamma ** 0.5


@pytest.mark.parametrize("name", ["c16n", "tiny3n"])
def test_bddc_bound_on_the_complement_of_the_constant(name):
    s, ss, M = _setup(name)
    n = ss.n_gamma
    A = ss.dense_A()
    Minv = np.column_stack([M.apply(e) for e in np.eye(n)])
    Minv = 0.5 * (Minv + Minv.T)
    Z = np.linalg.qr(np.column_stack([np.ones(n), np.random.default_rng(0).standard_normal((n, n - 1))]))[0][:, 1:]
    # eigenvalues of M^{-1} A on the complement: the pencil (Z^T A Z, Z^T M Z)
    # written through M^{-1}: eig of (Z^T Minv Z)(Z^T A Z) restricted
    lam = np.sort(np.linalg.eigvals((Z.T @ Minv @ Z) @ (Z.T @ A @ Z)).real)
    assert lam[0] >= 1.0 - 1e-8 and lam[-1] < 100
