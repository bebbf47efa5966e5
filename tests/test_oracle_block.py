"""Pins of the oracle's block deflated PCG (the block adjoint) against facts
that do not depend on its own code:

* one right-hand side: the iterates are those of Algorithm 1 (oracle.dpcg,
  written separately), with and without a deflation basis;
* every column of the block solution is the sparse direct solution to the
  tolerance (the plain definition);
* repeated and zero columns: the dependent directions are dropped and the
  block still converges, equal columns giving equal solutions;
* the adjoint gradient from the block (Appendix B) equals the one from the
  direct solves.
"""
import numpy as np

import workload
from oracle import adjoint, block, q1
from oracle.dpcg import dpcg
from oracle.sequence import OracleSolver


def _tiny3(R=0, n_prev=0):
    s = workload.workload("tiny3")
    coef = np.exp(0.7 * np.random.default_rng(3).standard_normal(16 ** 3))
    o = OracleSolver(16, s["elem_to_sub"], coef, sub_to_subregion=s["sub_to_subregion"], R=R)
    if n_prev:
        o.solve_sequence(workload.rhs_sequence(16, n_prev), 1e-10)
    return o, coef


def _ops(o):
    A = lambda V: np.column_stack([o.ss.apply_A(v) for v in V.T]) if V.shape[1] else V
    M = lambda V: np.column_stack([o.M.apply(v) for v in V.T]) if V.shape[1] else V
    return A, M


def test_one_column_is_algorithm_1():
    for R, n_prev in ((0, 0), (6, 3)):
        o, _ = _tiny3(R, n_prev)
        A, M = _ops(o)
        W = o.rec.basis(o.ss.n_gamma)
        b = o.ss.condense(workload.rhs_sequence(16, 1, first=7)[0])
        ref = dpcg(o.ss.apply_A, o.M.apply, b, None, W if W.shape[1] else None, 1e-10, 500, "rhs", record=False)
        res = block.block_dpcg(A, M, b[:, None], W if W.shape[1] else None, 1e-10)
        assert res["iters"] == ref["iters"], (res["iters"], ref["iters"], R)
        np.testing.assert_allclose(res["x"][:, 0], ref["x"], rtol=0, atol=1e-9 * np.abs(ref["x"]).max())


def test_columns_equal_direct_solves():
    o, coef = _tiny3(6, 3)
    A, M = _ops(o)
    F = workload.rhs_sequence(16, 5, first=11)
    B = np.column_stack([o.ss.condense(f) for f in F])
    res = block.block_dpcg(A, M, B, o.rec.basis(o.ss.n_gamma), 1e-11)
    U = q1.direct_solve(16, coef, F)
    assert res["iters"] < 60 and max(res["ranks"]) == 5
    for k in range(5):
        x = o.ss.recover(res["x"][:, k], F[k])
        assert np.abs(x - U[k]).max() <= 1e-9 * np.abs(U[k]).max()


def test_dependent_columns_are_dropped():
    o, _ = _tiny3()
    A, M = _ops(o)
    F = workload.rhs_sequence(16, 2, first=3)
    b0, b1 = (o.ss.condense(f) for f in F)
    B = np.column_stack([b0, b1, b0, np.zeros_like(b0), b0 + 2 * b1])
    res = block.block_dpcg(A, M, B, None, 1e-10)
    assert res["ranks"][0] == 2                  # rank of the block
    np.testing.assert_allclose(res["x"][:, 2], res["x"][:, 0], rtol=0, atol=1e-12 * np.abs(res["x"]).max())
    assert np.all(res["x"][:, 3] == 0.0)
    one = block.block_dpcg(A, M, b0[:, None], None, 1e-10)
    np.testing.assert_allclose(res["x"][:, 0], one["x"][:, 0], rtol=0, atol=1e-8 * np.abs(one["x"]).max())


def test_block_adjoint_gradient_matches_direct():
    nx = 16
    o, coef = _tiny3(6, 3)
    F = workload.rhs_sequence(nx, 4, first=20)
    T = q1.direct_solve(nx, np.exp(0.5 * np.random.default_rng(9).standard_normal(nx ** 3)), F)
    L, g_ref, lam_ref, U = adjoint.loss_and_grad(nx, np.log(coef), F, T)
    lam, res = block.adjoint_block(o, 2.0 * (U - T), rtol=1e-12)
    assert np.abs(lam - lam_ref).max() <= 1e-9 * np.abs(lam_ref).max()
    g = adjoint.element_gradient(nx, coef, lam, U)
    assert np.abs(g - g_ref).max() <= 1e-8 * np.abs(g_ref).max()
