"""GPU test at the full 192^3 size (13,824 subdomains of 8^3, three levels with
1,728 subregions, adaptive faces at tau 10, float32 Neumann operators, R = 40),
where the oracle cannot run whole.  Checked instead, on two right-hand sides:

* the coarse-space sizes against their closed forms for an m^3 lattice of
  cube subdomains with the x = 1 face Dirichlet (m = 24; subregions m/2):
  corners (m-1)^3 + 5 (m-1)^2, faces 3 (m-1) m^2, level-3 unknowns the same
  counts one level up, and every face examined by the adaptive step;
* the true interface residual below rtol (recomputed in float64 by the solver);
* the nodal residual (K u - F)_n at 2,000 sampled free nodes, each row of K
  formed here from the element matrices c_e h Kref (no library code): at most
  10 rtol ||F||_2, and at sampled interior nodes (one subdomain) at rounding
  level, since the interior is solved directly.
"""
import numpy as np
import pytest

import workload

pytestmark = pytest.mark.gpu


def _torch():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def _kref():
    from oracle.q1 import kref
    return kref()


def _row_times(nx, coef, u, n, K0):
    """(K u)_n from the (up to 8) elements around node n."""
    n1 = nx + 1
    ix, iy, iz = n % n1, (n // n1) % n1, n // (n1 * n1)
    h = 1.0 / nx
    s = 0.0
    for ez in (iz - 1, iz):
        for ey in (iy - 1, iy):
            for ex in (ix - 1, ix):
                if min(ex, ey, ez) < 0 or max(ex, ey, ez) >= nx:
                    continue
                e = ex + nx * (ey + nx * ez)
                vn = (ix - ex) + 2 * (iy - ey) + 4 * (iz - ez)
                for v in range(8):
                    a, b, c = v & 1, (v >> 1) & 1, v >> 2
                    m = (ex + a) + n1 * ((ey + b) + n1 * (ez + c))
                    s += coef[e] * h * K0[vn, v] * u[m]
    return s


def test_192_adaptive_three_level_two_rhs():
    torch = _torch()
    from paper_2412_17543_amd.solver import Solver
    s = workload.workload("c192")
    nx, m = 192, 24
    print("[gpu] 192^3 inputs", flush=True)
    F = workload.rhs_sequence(nx, 2)
    print("[gpu] 192^3 setup", flush=True)
    g = Solver(nx, s["elem_to_sub"], s["coef"], sub_to_subregion=s["sub_to_subregion"], R=s["R"],
               local_prec=32, adapt_tau=10.0, adapt_max_per_face=10)
    info, ad = g.info(), g.adaptive_stats()
    print("[gpu] 192^3", info, ad, flush=True)
    corners = lambda k: (k - 1) ** 3 + 5 * (k - 1) ** 2
    faces = lambda k: 3 * (k - 1) * k * k
    assert info["corners"] == corners(m) and info["faces"] == faces(m)
    assert ad["faces"] == faces(m)
    assert info["n_coarse"] == corners(m) + faces(m) + ad["added"]
    if ad["added"] == 0:
        assert info["level3"] == corners(m // 2) + faces(m // 2)
    rtol = 1e-8
    U, its, rr = g.solve_sequence(torch.tensor(F, device="cuda"), rtol)
    print("[gpu] 192^3 iters %s true relres %s" % (its.tolist(), rr.tolist()), flush=True)
    assert np.all(rr < rtol)
    K0 = _kref()
    rng = np.random.default_rng(0)
    free = np.flatnonzero(np.arange(workload.n_nodes(nx)) % (nx + 1) != nx)
    for k in range(2):
        u = U[k].cpu().numpy()
        nodes = rng.choice(free, 2000, replace=False)
        res = np.array([_row_times(nx, s["coef"], u, int(n), K0) - F[k, n] for n in nodes])
        assert np.abs(res).max() <= 10 * rtol * np.linalg.norm(F[k])
        # nodes strictly inside subdomain 0 (element block [0, 8)^3): interior of one subdomain
        inner = [(a + 1) + (nx + 1) * ((b + 1) + (nx + 1) * (c + 1)) for a, b, c in rng.integers(0, 7, (50, 3))]
        res_i = np.array([_row_times(nx, s["coef"], u, int(n), K0) - F[k, n] for n in inner])
        assert np.abs(res_i).max() <= 1e-12 * np.abs(F[k]).max() + 1e-12 * np.abs(u).max()
