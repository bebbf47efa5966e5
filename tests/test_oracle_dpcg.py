"""Pins of Algorithm 1 (deflated PCG) and of harmonic-Ritz recycling."""
import numpy as np
import pytest
import scipy.sparse.linalg as spla

import workload
from oracle.bddc import BDDC
from oracle.dpcg import dpcg, lanczos_ritz
from oracle.recycle import Recycler
from oracle.sequence import OracleSolver
from oracle.substructure import Substructuring


def _spd(n, cond=1e3, seed=0):
    g = np.random.default_rng(seed)
    Q, _ = np.linalg.qr(g.standard_normal((n, n)))
    lam = np.geomspace(1.0, cond, n)
    return (Q * lam) @ Q.T


@pytest.fixture(scope="module")
def c16():
    s = workload.workload("c16")
    ss = Substructuring(s["nx"], s["elem_to_sub"], s["coef"])
    M = BDDC(ss)
    F = workload.rhs_sequence(s["nx"], 2)
    return ss, M, F


def test_plain_pcg_matches_scipy_cg(c16):
    ss, M, F = c16
    b = ss.condense(F[0])
    res = dpcg(ss.apply_A, M.apply, b, rtol=1e-10)
    n = ss.n_gamma
    Aop = spla.LinearOperator((n, n), matvec=ss.apply_A)
    Mop = spla.LinearOperator((n, n), matvec=M.apply)
    count = [0]
    x, info = spla.cg(Aop, b, M=Mop, rtol=1e-10, atol=0.0, maxiter=200,
                      callback=lambda xk: count.__setitem__(0, count[0] + 1))
    assert info == 0
    assert abs(res["iters"] - count[0]) <= 1
    np.testing.assert_allclose(res["x"], x, atol=1e-8 * np.abs(x).max())


def test_dense_problem_solution():
    n = 60
    A = _spd(n)
    Minv = np.linalg.inv(A + 0.3 * np.diag(np.diag(A)))
    b = np.random.default_rng(1).standard_normal(n)
    res = dpcg(lambda v: A @ v, lambda v: Minv @ v, b, rtol=1e-12)
    np.testing.assert_allclose(res["x"], np.linalg.solve(A, b), rtol=1e-9)


def test_solution_in_span_w_takes_zero_iterations():
    n = 50
    A = _spd(n)
    g = np.random.default_rng(2)
    xs = g.standard_normal(n)
    W = np.column_stack([xs, g.standard_normal((n, 3))])
    res = dpcg(lambda v: A @ v, lambda v: v, A @ xs, W=W, rtol=1e-10)
    assert res["iters"] == 0
    np.testing.assert_allclose(res["x"], xs, rtol=1e-10)


def test_deflation_invariants(c16):
    ss, M, F = c16
    g = np.random.default_rng(5)
    W = g.standard_normal((ss.n_gamma, 4))
    res = dpcg(ss.apply_A, M.apply, ss.condense(F[0]), W=W, rtol=1e-10)
    assert max(res["wtr"]) < 1e-10          # W^T r_j = 0
    assert max(res["wtap"]) < 1e-10         # W^T A p_j = 0
    P = np.column_stack(res["P"])
    AP = np.column_stack(res["AP"])
    G = P.T @ AP
    off = G - np.diag(np.diag(G))
    assert np.abs(off).max() < 1e-6 * np.abs(np.diag(G)).max()


def test_reorthogonalisation_projects_residual(c16):
    # optional line of Alg. 1: after r -= W (W^T W)^{-1} W^T r the residual is
    # orthogonal to range(W) to rounding at every step (the recurrence alone
    # only keeps W^T r small), and the iteration still converges to A^{-1} b
    ss, M, F = c16
    g = np.random.default_rng(7)
    W = g.standard_normal((ss.n_gamma, 5))
    b = ss.condense(F[1])
    plain = dpcg(ss.apply_A, M.apply, b, W=W, rtol=1e-10)
    ro = dpcg(ss.apply_A, M.apply, b, W=W, rtol=1e-10, reorth=True)
    assert max(ro["wtr"]) < 1e-14
    assert max(ro["wtr"]) <= max(plain["wtr"])
    assert abs(ro["iters"] - plain["iters"]) <= 1
    np.testing.assert_allclose(ro["x"], plain["x"], atol=1e-8 * np.abs(plain["x"]).max())
    n = 60
    A = _spd(n, cond=1e6, seed=3)
    Wd = g.standard_normal((n, 6))
    bd = g.standard_normal(n)
    rd = dpcg(lambda v: A @ v, lambda v: v, bd, W=Wd, rtol=1e-11, reorth=True)
    np.testing.assert_allclose(rd["x"], np.linalg.solve(A, bd), rtol=1e-7)


def test_w_empty_is_plain_pcg(c16):
    ss, M, F = c16
    b = ss.condense(F[1])
    r1 = dpcg(ss.apply_A, M.apply, b, W=np.zeros((ss.n_gamma, 0)), rtol=1e-9)
    r2 = dpcg(ss.apply_A, M.apply, b, W=None, rtol=1e-9)
    assert r1["iters"] == r2["iters"]
    np.testing.assert_array_equal(r1["x"], r2["x"])


def test_stopping_rules_zero_guess_coincide(c16):
    ss, M, F = c16
    b = ss.condense(F[0])
    a = dpcg(ss.apply_A, M.apply, b, rtol=1e-8, stop="rhs")
    c = dpcg(ss.apply_A, M.apply, b, rtol=1e-8, stop="r0")
    assert a["iters"] == c["iters"]
    # from a good initial guess the ||b|| rule stops earlier (Section 5)
    x0 = a["x"] + 1e-7 * np.random.default_rng(0).standard_normal(b.size)
    a2 = dpcg(ss.apply_A, M.apply, b, x0, rtol=1e-8, stop="rhs")
    c2 = dpcg(ss.apply_A, M.apply, b, x0, rtol=1e-8, stop="r0")
    assert a2["iters"] < c2["iters"]


def test_zero_rhs():
    res = dpcg(lambda v: 2 * v, lambda v: v, np.zeros(5))
    assert res["iters"] == 0 and not res["x"].any()


def test_lanczos_ritz_values_bounded_below_by_one(c16):
    # Section 3.2: lambda_min(M^{-1} A) >= 1 for BDDC; CG Ritz values lie in the spectrum
    ss, M, F = c16
    res = dpcg(ss.apply_A, M.apply, ss.condense(F[0]), rtol=1e-12)
    th = lanczos_ritz(res["alpha"], res["beta"])
    assert th[0] >= 1 - 1e-8 and th[-1] < 50


# ---------------------------------------------------------------- harmonic Ritz

def test_harmonic_ritz_values_inside_spectrum():
    n = 40
    A = _spd(n, 1e2, 3)
    B = _spd(n, 10, 4)
    Minv = np.linalg.inv(B)
    lam = np.sort(np.linalg.eigvals(Minv @ A).real)
    V = np.random.default_rng(7).standard_normal((n, 12))
    th, Y, F, G = Recycler.harmonic_ritz(V, lambda v: A @ v, lambda v: Minv @ v)
    assert th.min() >= lam[0] - 1e-9 and th.max() <= lam[-1] + 1e-9
    # Y is F-orthonormal and diagonalises G
    np.testing.assert_allclose(Y.T @ F @ Y, np.eye(Y.shape[1]), atol=1e-9)
    np.testing.assert_allclose(Y.T @ G @ Y, np.diag(th), atol=1e-9)


def test_harmonic_ritz_exact_on_invariant_subspace():
    n = 30
    A = _spd(n, 50, 8)
    B = _spd(n, 5, 9)
    Minv = np.linalg.inv(B)
    lam, X = np.linalg.eig(Minv @ A)
    idx = np.argsort(lam.real)[-5:]
    V = X[:, idx].real @ np.random.default_rng(3).standard_normal((5, 5))
    th, *_ = Recycler.harmonic_ritz(V, lambda v: A @ v, lambda v: Minv @ v)
    np.testing.assert_allclose(np.sort(th), np.sort(lam[idx].real), rtol=1e-9)


def test_cheap_harmonic_ritz_matrices_equal_explicit(c16):
    """Low-cost construction from the solve's own scalars equals explicit formation.

    With W^T A P = 0 and A-orthogonal p_j, F = blockdiag(W^T A W, diag(d_j)); the
    P-P block of G is tridiagonal with G_jj = d_j (1 + beta_j) / alpha_j and
    G_{j-1,j} = -d_{j-1} d_j / rho_{j-1}; G_WP[:, j] = W^T A W (mu_j - mu_{j+1}) / alpha_j
    (M^{-1} A p_j = (z_j - z_{j+1}) / alpha_j from the residual update of Algorithm 1).
    """
    ss, M, F = c16
    g = np.random.default_rng(11)
    W = g.standard_normal((ss.n_gamma, 3))
    res = dpcg(ss.apply_A, M.apply, ss.condense(F[0]), W=W, rtol=1e-9)
    l = res["iters"]
    # one more preconditioner application gives z_l, rho_l, mu_l (needed for the last column)
    AW = np.column_stack([ss.apply_A(W[:, c]) for c in range(3)])
    WAW = W.T @ AW
    b = ss.condense(F[0])
    x = res["x"]
    P = np.column_stack(res["P"])
    AP = np.column_stack(res["AP"])
    # recover r_l from the recursion: r_l = r_0 - sum alpha_j A p_j
    r = b - ss.apply_A(res["x"] - sum(a * P[:, j] for j, a in enumerate(res["alpha"])))
    r = r - AP @ np.array(res["alpha"])
    zl = M.apply(r)
    rho = list(res["rho"]) + [r @ zl]
    mu = list(res["mu"]) + [np.linalg.solve(WAW, AW.T @ zl)]
    alpha, d = np.array(res["alpha"]), np.array(res["d"])
    beta = np.array(rho[1:]) / np.array(rho[:-1])
    V = np.column_stack([W, P])
    _, _, Fx, Gx = Recycler.harmonic_ritz(V, ss.apply_A, M.apply)
    Gpp = np.zeros((l, l))
    for j in range(l):
        Gpp[j, j] = d[j] * (1 + beta[j]) / alpha[j]
        if j:
            Gpp[j - 1, j] = Gpp[j, j - 1] = -d[j - 1] * d[j] / rho[j - 1]
    Gwp = np.column_stack([WAW @ (mu[j] - mu[j + 1]) / alpha[j] for j in range(l)])
    scale = np.abs(Gx).max()
    np.testing.assert_allclose(Gx[3:, 3:], Gpp, atol=1e-10 * scale)
    np.testing.assert_allclose(Gx[:3, 3:], Gwp, atol=1e-10 * scale)
    np.testing.assert_allclose(Fx[:3, 3:], 0, atol=1e-10 * np.abs(Fx).max())
    np.testing.assert_allclose(np.diag(Fx)[3:], d, rtol=1e-10)


def test_b4_recycling_reduces_iterations():
    s = workload.workload("c16")
    F = workload.rhs_sequence(16, 6)
    base = OracleSolver(16, s["elem_to_sub"], s["coef"], R=0)
    _, it0, _ = base.solve_sequence(F, 1e-10)
    rec = OracleSolver(16, s["elem_to_sub"], s["coef"], R=10, strategy="B4")
    _, it1, rr = rec.solve_sequence(F, 1e-10)
    assert it1[0] == it0[0]                 # first solve has no basis yet
    assert it1[2:].sum() < it0[2:].sum()    # deflating the largest harmonic Ritz values helps
    assert (rr < 1e-10).all()


@pytest.mark.parametrize("strategy", ["B1", "B2", "B3"])
def test_other_strategies_solve_correctly(strategy):
    s = workload.workload("c16")
    F = workload.rhs_sequence(16, 4)
    o = OracleSolver(16, s["elem_to_sub"], s["coef"], R=8, strategy=strategy)
    us, its, rr = o.solve_sequence(F, 1e-10)
    assert (rr < 1e-10).all()
    assert o.rec.W.shape[1] == 8 or strategy == "B1" and o.rec.W.shape[1] <= 8
