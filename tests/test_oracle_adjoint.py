"""Pins of the adjoint gradient against central finite differences and an identity."""
import numpy as np

import workload
from oracle import adjoint, q1


def _setup(nx=8, n_rhs=3):
    F = workload.rhs_sequence(nx, n_rhs)
    g = np.random.default_rng(4)
    theta_t = 0.5 * g.standard_normal(nx ** 3)
    T = q1.direct_solve(nx, np.exp(theta_t), F)
    theta = 0.3 * g.standard_normal(nx ** 3)
    return F, T, theta


def test_gradient_matches_central_differences():
    nx = 8
    F, T, theta = _setup(nx)
    L, g, lam, U = adjoint.loss_and_grad(nx, theta, F, T)
    # step 1e-4: truncation O(eps^2) ~ 1e-8; at 1e-6 the rounding of the solves
    # (~1e-13 L) divided by 2 eps dominates
    eps = 1e-4
    idx = np.random.default_rng(1).choice(nx ** 3, 12, replace=False)
    fd = []
    for e in idx:
        tp, tm = theta.copy(), theta.copy()
        tp[e] += eps
        tm[e] -= eps
        fd.append((adjoint.loss(nx, tp, F, T) - adjoint.loss(nx, tm, F, T)) / (2 * eps))
    fd = np.array(fd)
    err = np.abs(g[idx] - fd) / np.maximum(np.abs(fd), 1e-3 * np.abs(fd).max())
    assert err.max() < 1e-5, err


def test_gradient_scaling_identity():
    # K(theta + t 1) = e^t K(theta)  =>  sum_e dL/dtheta_e = - sum_k lambda_k^T F_k
    nx = 8
    F, T, theta = _setup(nx)
    L, g, lam, U = adjoint.loss_and_grad(nx, theta, F, T)
    fr = q1.free_nodes(nx)
    rhs = -sum(lam[k, fr] @ F[k, fr] for k in range(len(F)))
    assert abs(g.sum() - rhs) <= 1e-10 * abs(rhs)


def test_rhs_gradient_is_adjoint():
    # L is quadratic in F: a central difference along any direction is exact to roundoff
    nx = 8
    F, T, theta = _setup(nx)
    L, g, lam, U = adjoint.loss_and_grad(nx, theta, F, T)
    d = np.random.default_rng(2).standard_normal(F.shape)
    eps = 1e-3 * np.abs(F).max()
    Lp = adjoint.loss(nx, theta, F + eps * d, T)
    Lm = adjoint.loss(nx, theta, F - eps * d, T)
    fr = q1.free_nodes(nx)
    np.testing.assert_allclose((Lp - Lm) / (2 * eps), (lam[:, fr] * d[:, fr]).sum(), rtol=1e-7)


def test_central_difference_step_floor_16():
    # Why the finite-difference checks use a step of 1e-4: with sparse direct
    # solves (the oracle's most accurate path) L carries a rounding error
    # e_L ~ 1e-14 L, which a central difference of step s turns into an error
    # e_L / s in dL/dtheta_e, while the truncation error is O(s^2).  Per
    # element, dL/dtheta_e is ~1e-3 L at most, so at s = 1e-6 the rounding
    # term alone reaches ~1e-5..1e-3 of the largest entry, and at s = 1e-4 it
    # drops a hundredfold while the truncation error (~1e-8) stays far below.
    nx = 16
    F = workload.rhs_sequence(nx, 3)
    g = np.random.default_rng(4)
    T = q1.direct_solve(nx, np.exp(0.5 * g.standard_normal(nx ** 3)), F)
    theta = 0.3 * g.standard_normal(nx ** 3)
    L, grad, lam, U = adjoint.loss_and_grad(nx, theta, F, T)
    idx = workload.rng("fd").choice(nx ** 3, 20, replace=False)

    def fd(eps):
        out = []
        for e in idx:
            tp, tm = theta.copy(), theta.copy()
            tp[e] += eps
            tm[e] -= eps
            out.append((adjoint.loss(nx, tp, F, T) - adjoint.loss(nx, tm, F, T)) / (2 * eps))
        out = np.array(out)
        return np.abs(grad[idx] - out) / np.maximum(np.abs(out), 1e-3 * np.abs(out).max())
    e6, e4 = fd(1e-6), fd(1e-4)
    assert e4.max() < 1e-5, e4
    assert e6.max() > 10 * e4.max()      # the rounding floor at 1e-6
