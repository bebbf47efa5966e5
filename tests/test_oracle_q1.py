"""Pins of the oracle's Q1 discretisation against mathematics, not against itself."""
import numpy as np
import pytest

import workload
from oracle import q1


def _quadrature_kref():
    """Unit-cube Q1 stiffness by 3-point Gauss quadrature of grad(phi_v).grad(phi_w)."""
    xg, wg = np.polynomial.legendre.leggauss(3)
    xg = 0.5 * (xg + 1.0)
    wg = 0.5 * wg
    K = np.zeros((8, 8))
    for i, x in enumerate(xg):
        for j, y in enumerate(xg):
            for k, z in enumerate(xg):
                grads = []
                for v in range(8):
                    a, b, c = v & 1, (v >> 1) & 1, (v >> 2) & 1
                    fx = x if a else 1 - x
                    fy = y if b else 1 - y
                    fz = z if c else 1 - z
                    dx = 1.0 if a else -1.0
                    dy = 1.0 if b else -1.0
                    dz = 1.0 if c else -1.0
                    grads.append([dx * fy * fz, fx * dy * fz, fx * fy * dz])
                g = np.array(grads)
                K += wg[i] * wg[j] * wg[k] * g @ g.T
    return K


def test_kref_matches_quadrature():
    np.testing.assert_allclose(q1.kref(), _quadrature_kref(), atol=1e-15)


def test_kref_kernel_is_constants():
    K = q1.kref()
    np.testing.assert_allclose(K, K.T)
    np.testing.assert_allclose(K.sum(axis=1), 0.0, atol=1e-15)
    ev = np.linalg.eigvalsh(K)
    assert abs(ev[0]) < 1e-14 and ev[1] > 1e-3


def test_assembled_interior_stencil():
    # interior node of an 8^3 mesh: centre 8h/3, axis 0, face-diagonal -h/6, body-diagonal -h/12
    nx = 8
    h = 1.0 / nx
    K = q1.assemble(nx, np.ones(nx ** 3)).tocsr()
    n1 = nx + 1
    v = 4 + n1 * (4 + n1 * 4)
    row = K.getrow(v).toarray().ravel()
    expect = {}
    for dx in (-1, 0, 1):
        for dy in (-1, 0, 1):
            for dz in (-1, 0, 1):
                nd = abs(dx) + abs(dy) + abs(dz)
                expect[v + dx + n1 * (dy + n1 * dz)] = {0: 8 * h / 3, 1: 0.0, 2: -h / 6, 3: -h / 12}[nd]
    for u, val in expect.items():
        assert row[u] == pytest.approx(val, abs=1e-15)
    assert np.count_nonzero(np.abs(row) > 1e-16) == 1 + 12 + 8
    assert abs(row.sum()) < 1e-14


def test_coefficient_scales_element():
    nx = 4
    c = np.ones(nx ** 3)
    c[5] = 7.0
    K1 = q1.assemble(nx, np.ones(nx ** 3))
    K7 = q1.assemble(nx, c)
    en = workload.element_nodes(nx)[5]
    D = (K7 - K1).toarray()
    np.testing.assert_allclose(D[np.ix_(en, en)], 6.0 * q1.kref() / nx, atol=1e-15)
    D[np.ix_(en, en)] = 0
    assert np.abs(D).max() < 1e-15


def test_spd_after_dirichlet():
    nx = 4
    K = q1.assemble(nx, np.ones(nx ** 3)).toarray()
    fr = q1.free_nodes(nx)
    ev = np.linalg.eigvalsh(K[np.ix_(fr, fr)])
    assert ev[0] > 1e-6


@pytest.mark.slow
def test_manufactured_solution_converges():
    # u = cos(pi x/2) cos(pi y) cos(pi z): u = 0 at x = 1, du/dn = 0 on the other faces,
    # -Lap u = (pi^2/4 + 2 pi^2) u.  Nodal error must drop ~4x per halving of h.
    errs = []
    for nx in (8, 16, 32):
        x = workload.node_coords(nx)
        u = np.cos(np.pi * x[:, 0] / 2) * np.cos(np.pi * x[:, 1]) * np.cos(np.pi * x[:, 2])
        f = (9 * np.pi ** 2 / 4) * u
        F = workload.consistent_load(nx, f)
        uh = q1.direct_solve(nx, np.ones(nx ** 3), F)[0]
        fr = q1.free_nodes(nx)
        errs.append(np.abs(uh[fr] - u[fr]).max())
    r1, r2 = errs[0] / errs[1], errs[1] / errs[2]
    assert 3.3 < r1 < 4.7 and 3.3 < r2 < 4.7, errs
