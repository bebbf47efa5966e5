"""Pins of the recycling selection (Section 4.2, paragraphs B3/B4) and of the
basis-freeze criterion (eq. harmritzstopcrit).

These check the oracle against facts fixed by the mathematics, not against
itself:
  * on an invariant subspace of M^{-1} A the harmonic Ritz pairs are exact
    eigenpairs, so B4 must return the eigenvectors of the R largest
    eigenvalues (B3 those of the R smallest);
  * deflating the B4 basis from a few solves lowers the top of the spectrum
    of the deflated preconditioned operator, while its bottom stays >= 1;
  * with M = I and A diagonal, the harmonic Ritz values of a coordinate
    subspace are the diagonal entries, so scaling A by (1 + delta) changes
    them by a known relative amount: the criterion must fire exactly when
    the 2-norm of the change over the 2-norm of the NEW values is <= 1e-5;
  * repeating a right-hand side gives a solve with zero iterations, so the
    second basis is built from the first one alone: the values repeat and
    the basis freezes at that update.
"""
import numpy as np
import pytest
import scipy.linalg as sla

import workload
from oracle.bddc import BDDC
from oracle.dpcg import dpcg
from oracle.recycle import Recycler, ritz_change, select
from oracle.sequence import OracleSolver
from oracle.substructure import Substructuring


def _spd(n, lo, hi, seed):
    g = np.random.default_rng(seed)
    Q, _ = np.linalg.qr(g.standard_normal((n, n)))
    return (Q * np.geomspace(lo, hi, n)) @ Q.T


def _invariant_case(seed=0):
    n = 40
    A = _spd(n, 1.0, 1e2, seed)
    Minv = np.linalg.inv(_spd(n, 1.0, 8.0, seed + 1))
    lam, X = np.linalg.eig(Minv @ A)
    lam, X = lam.real, X.real
    order = np.argsort(lam)
    lo, hi = order[:3], order[-3:]
    mix = np.random.default_rng(seed + 2).standard_normal((6, 6))
    V = np.column_stack([X[:, hi], X[:, lo]]) @ mix     # invariant, eigenvectors mixed
    return A, Minv, lam, X, lo, hi, V


@pytest.mark.parametrize("strategy", ["B4", "B3"])
def test_selection_on_invariant_subspace(strategy):
    A, Minv, lam, X, lo, hi, V = _invariant_case()
    rec = Recycler(3, strategy)
    rec.update(V, lambda v: A @ v, lambda v: Minv @ v)
    want = hi if strategy == "B4" else lo
    ang = sla.subspace_angles(rec.W, X[:, want])
    assert ang.max() < 1e-8
    ref = np.sort(lam[want])[::-1] if strategy == "B4" else np.sort(lam[want])
    np.testing.assert_allclose(rec.theta, ref, rtol=1e-10)


def test_select_orders_from_the_kept_end():
    th = np.array([1.3, 4.0, 1.0, 2.5, 1.1])
    assert list(select(th, 3, "B4")) == [1, 3, 0]
    assert list(select(th, 3, "B3")) == [2, 4, 0]
    assert list(select(th, 9, "B4")) == [1, 3, 0, 4, 2]


def _deflated_spectrum(A, Minv, W):
    """Nonzero eigenvalues of Q M^{-1} Q^T A with Q = I - W (W^T A W)^{-1} W^T A:
    the operator deflated PCG iterates with (p = Q z, Algorithm 1 line 16)."""
    n = A.shape[0]
    Q = np.eye(n) - W @ np.linalg.solve(W.T @ A @ W, W.T @ A)
    ev = np.sort(np.linalg.eigvals(Q @ Minv @ Q.T @ A).real)
    return ev[ev > 1e-8 * ev.max()]


@pytest.fixture(scope="module")
def tiny_dense():
    s = workload.workload("tiny")
    ss = Substructuring(s["nx"], s["elem_to_sub"], s["coef"])
    M = BDDC(ss)
    A = ss.dense_A()
    Minv = np.column_stack([M.apply(e) for e in np.eye(ss.n_gamma)])
    return s, ss, M, A, 0.5 * (Minv + Minv.T)


def test_b4_lowers_the_top_of_the_deflated_spectrum(tiny_dense):
    # Section 4.2, paragraph B4: BDDC puts the bottom of the spectrum at 1, so
    # deflating the largest harmonic Ritz vectors shrinks the spread from above
    s, ss, M, A, Minv = tiny_dense
    lam = np.sort(np.linalg.eigvals(Minv @ A).real)
    F = workload.rhs_sequence(s["nx"], 4)
    o = OracleSolver(s["nx"], s["elem_to_sub"], s["coef"], R=3, strategy="B4")
    o.solve_sequence(F, 1e-10)
    ev = _deflated_spectrum(A, Minv, o.rec.W)
    assert ev.min() >= 1.0 - 1e-8
    assert ev.max() < lam[-1] - 0.25 * (lam[-1] - 1.0)
    # the selected values approximate the top of the spectrum
    assert o.rec.theta.max() > lam[-1] - 1e-2 * (lam[-1] - 1.0)
    # B3 deflates near 1 and leaves the top where it was
    o3 = OracleSolver(s["nx"], s["elem_to_sub"], s["coef"], R=3, strategy="B3")
    o3.solve_sequence(F, 1e-10)
    assert _deflated_spectrum(A, Minv, o3.rec.W).max() > lam[-1] - 0.01 * (lam[-1] - 1.0)


# ------------------------------------------------------------ freeze criterion

LAM = np.array([10.0, 9.0, 8.0, 2.0, 1.5, 1.2, 1.1, 1.05, 1.0])


def _two_updates(scale2, R=3, first_cols=3):
    """First update from e_0..e_{first_cols-1} with A = diag(LAM), second from
    e_3, e_4 with A = diag(LAM * scale2) (M = I in both)."""
    n = LAM.size
    I = np.eye(n)
    rec = Recycler(R, "B4")
    A1 = np.diag(LAM)
    rec.update(I[:, :first_cols], lambda v: A1 @ v, lambda v: v)
    A2 = np.diag(LAM * scale2)
    rec.update(I[:, 3:5], lambda v: A2 @ v, lambda v: v)
    return rec


def test_harmonic_ritz_values_of_a_coordinate_subspace():
    rec = _two_updates(np.ones(LAM.size))
    np.testing.assert_allclose(rec.history[0], [10.0, 9.0, 8.0], rtol=1e-13)
    np.testing.assert_allclose(rec.history[1], [10.0, 9.0, 8.0], rtol=1e-13)
    assert rec.frozen and rec.freeze_step == 2


@pytest.mark.parametrize("delta,frozen", [
    # uniform scaling: change / ||theta_new|| = delta / (1 + delta)
    (1.000005e-5, True),     # 0.999995e-5: fires (it would not against ||theta_old||)
    (1.00002e-5, False),     # 1.00001e-5: does not fire
    (0.5e-5, True),
    (3e-5, False),
])
def test_freeze_threshold_uniform_scaling(delta, frozen):
    rec = _two_updates(np.full(LAM.size, 1.0 + delta))
    lhs = delta / (1.0 + delta)
    assert abs(ritz_change(rec.history[1], rec.history[0]) - lhs) < 1e-9 * lhs
    assert rec.frozen is frozen
    assert rec.freeze_step == (2 if frozen else None)


@pytest.mark.parametrize("delta,frozen", [
    # only the largest value moves: change 10 delta, ||theta_new||_2 ~ 15.65,
    # so the 2-norm ratio is ~0.639 delta (max-norm ratio ~delta, 1-norm ~0.37 delta)
    (1.2e-5, True),          # 2-norm 0.77e-5 fires; a max-norm ratio (1.2e-5) would not
    (2.0e-5, False),         # 2-norm 1.28e-5 does not; a 1-norm ratio (0.74e-5) would
])
def test_freeze_threshold_uses_two_norms(delta, frozen):
    sc = np.ones(LAM.size)
    sc[0] = 1.0 + delta
    rec = _two_updates(sc)
    th1 = np.array([10.0 * (1 + delta), 9.0, 8.0])
    lhs = 10.0 * delta / np.linalg.norm(th1)
    assert abs(ritz_change(rec.history[1], rec.history[0]) - lhs) < 1e-8 * lhs
    assert rec.frozen is frozen


def test_no_freeze_before_the_basis_is_full():
    # first basis has 2 < R columns: the criterion is not evaluated
    rec = _two_updates(np.ones(LAM.size), first_cols=2)
    assert not rec.frozen
    assert rec.history[0].size == 2 and rec.history[1].size == 3


def test_frozen_basis_is_not_updated():
    rec = _two_updates(np.ones(LAM.size))
    W = rec.W.copy()
    A = np.diag(LAM)
    rec.update(np.eye(LAM.size)[:, 5:8], lambda v: A @ v, lambda v: v)
    np.testing.assert_array_equal(rec.W, W)
    assert len(rec.history) == 2 and rec.step == 3


def test_repeated_rhs_freezes_at_the_zero_iteration_solve():
    # F_2 solved twice: from the previous solution the second solve takes zero
    # iterations, V = W, the harmonic Ritz values repeat and the basis freezes
    s = workload.workload("c16")
    F = workload.rhs_sequence(16, 4)
    seq = np.stack([F[0], F[1], F[2], F[2], F[3]])
    o = OracleSolver(16, s["elem_to_sub"], s["coef"], R=4, strategy="B4")
    us, its, rr = o.solve_sequence(seq, 1e-10)
    assert its[3] == 0
    assert o.rec.frozen and o.rec.freeze_step == 4
    assert ritz_change(o.rec.history[3], o.rec.history[2]) < 1e-10
    assert all(ritz_change(o.rec.history[j], o.rec.history[j - 1]) > 1e-5 for j in (1, 2))
    assert (rr < 1e-10).all()
    # the frozen basis is the one built at the freeze
    W = o.rec.W.copy()
    o.solve(F[3], 1e-10)
    np.testing.assert_array_equal(o.rec.W, W)


def test_directions_after_a_residual_replacement_form_one_run():
    # Reading: after a residual replacement only the directions of the last
    # unbroken run are offered for recycling.  Force a replacement with an
    # operator carrying a symmetric rank-one error of 1e-3 during five loop
    # products (the recursive residual then converges while the true one has
    # not); the run after the replacement must obey the recurrences the
    # low-cost harmonic-Ritz matrices are built from (checked against explicit
    # formation), while the last direction before it is not linked to the
    # first one after it by them.  Plain PCG (W empty): a perturbed product
    # also moves W^T r off zero, which a deflated run cannot undo.
    s = workload.workload("c16")
    ss = Substructuring(16, s["elem_to_sub"], s["coef"])
    M = BDDC(ss)
    b = ss.condense(workload.rhs_sequence(16, 1)[0])
    nA = np.abs(ss.apply_A(np.ones(ss.n_gamma))).max()
    u = np.random.default_rng(4).standard_normal(ss.n_gamma)
    u /= np.linalg.norm(u)
    calls = [0]

    def apply_A(v):
        # calls 1-2: the initial residuals; 3 on: the loop
        calls[0] += 1
        y = ss.apply_A(v)
        return y + 1e-3 * nA * (u @ v) * u if 6 <= calls[0] <= 10 else y
    res = dpcg(apply_A, M.apply, b, rtol=1e-10)
    assert res["restarts"] == 1 and 0 < res["seg_start"] <= res["iters"] - 2
    assert res["true_relres"] < 1e-10
    j0, l = res["seg_start"], res["iters"]
    P = np.column_stack(res["P"][j0:])
    # z_l, rho_l after the exit (one more preconditioner application)
    r = b - ss.apply_A(res["x"])
    rho = list(res["rho"][j0:l]) + [r @ M.apply(r)]
    alpha, d = np.array(res["alpha"][j0:]), np.array(res["d"][j0:])
    beta = np.array(rho[1:]) / np.array(rho[:-1])
    m = l - j0
    _, _, Fx, Gx = Recycler.harmonic_ritz(P, ss.apply_A, M.apply)
    Gpp = np.zeros((m, m))
    for j in range(m):
        Gpp[j, j] = d[j] * (1 + beta[j]) / alpha[j]
        if j:
            Gpp[j - 1, j] = Gpp[j, j - 1] = -d[j - 1] * d[j] / rho[j - 1]
    scale = np.abs(Gx).max()
    np.testing.assert_allclose(Gx, Gpp, atol=1e-9 * scale)
    np.testing.assert_allclose(np.diag(Fx), d, rtol=1e-9)
    # across the replacement: the recurrence would predict the coupling
    # -d_{j0-1} d_{j0} / rho_{j0-1} between the two directions; it is not there
    Pall = np.column_stack(res["P"][j0 - 1:j0 + 1])
    _, _, _, G2 = Recycler.harmonic_ritz(Pall, ss.apply_A, M.apply)
    pred = -res["d"][j0 - 1] * res["d"][j0] / res["rho"][j0 - 1]
    assert abs(G2[0, 1] - pred) > 1e-3 * abs(pred)


def test_restart_every_reaches_the_same_solution():
    # restart_every longer than any solve changes nothing; a short one ends
    # runs early (counted restarts, the last run offered for recycling) and
    # still meets the tolerance with the true residual
    s = workload.workload("c16")
    F = workload.rhs_sequence(16, 3)
    ref = OracleSolver(16, s["elem_to_sub"], s["coef"], R=4)
    long_ = OracleSolver(16, s["elem_to_sub"], s["coef"], R=4, restart_every=500)
    short = OracleSolver(16, s["elem_to_sub"], s["coef"], R=4, restart_every=5)
    for k in range(3):
        a, b, c = ref.solve(F[k], 1e-10), long_.solve(F[k], 1e-10), short.solve(F[k], 1e-10)
        assert a["iters"] == b["iters"] and b["restarts"] == 0
        np.testing.assert_array_equal(a["x"], b["x"])
        assert c["restarts"] == (c["iters"] - 1) // 5 and c["seg_start"] == 5 * c["restarts"]
        assert c["true_relres"] < 1e-10
        np.testing.assert_allclose(c["u"], a["u"], atol=1e-8 * np.abs(a["u"]).max())
