"""GPU parity of the pure Neumann problem (no Dirichlet node, K semidefinite
with the constants as null space; Section 2 and Section 4.1, closing
paragraph) against the oracle: the library detects it from an all-zero
Dirichlet mask, solves the coarsest problem with the pseudo-inverse and keeps
the constant interface vector as column 0 of the deflation basis (the
recycled columns follow it).  float64 at rtol 1e-10: iterations +-1,
solutions (both normalised by the iteration: interface mean zero) to 1e-9."""
import numpy as np
import pytest

import workload

pytestmark = pytest.mark.gpu


def _torch():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


@pytest.mark.parametrize("name,R", [("c16n", 0), ("c16n", 4), ("tiny3n", 4)])
def test_pure_neumann_sequence_matches_oracle(name, R):
    torch = _torch()
    from oracle import q1
    from oracle.sequence import OracleSolver
    from paper_2412_17543_amd.solver import Solver
    s = workload.workload(name)
    nx = s["nx"]
    F = workload.consistent_neumann(nx, workload.rhs_sequence(nx, 4))
    print("[gpu] pure Neumann %s R=%d" % (name, R), flush=True)
    g = Solver(nx, s["elem_to_sub"], s["coef"], sub_to_subregion=s["sub_to_subregion"],
               node_dirichlet=s["node_dirichlet"], R=R)
    U, its, rr = g.solve_sequence(torch.tensor(F, device="cuda"), 1e-10)
    o = OracleSolver(nx, s["elem_to_sub"], s["coef"], sub_to_subregion=s["sub_to_subregion"], R=R,
                     dirichlet=s["node_dirichlet"].astype(bool))
    uo, ito, rro = o.solve_sequence(F, 1e-10)
    print("[gpu] iters", its.tolist(), ito.tolist(), flush=True)
    assert np.all(np.abs(its - ito) <= 1)
    assert np.all(rr < 1e-10)
    K = q1.assemble(nx, s["coef"])
    for k in range(len(F)):
        u = U[k].cpu().numpy()
        assert np.abs(u - uo[k]).max() <= 1e-9 * np.abs(uo[k]).max()
        assert np.abs(K @ u - F[k]).max() <= 1e-8 * np.abs(F[k]).max()
    info = g.solve_info()
    assert info["deflation_cols"] == 1 + (o.rec.W.shape[1] if R else 0)


def test_pure_neumann_preconditioner_parity():
    torch = _torch()
    from oracle.bddc import BDDC
    from oracle.substructure import Substructuring
    from paper_2412_17543_amd.solver import Solver
    for name in ("c16n", "tiny3n"):
        s = workload.workload(name)
        g = Solver(s["nx"], s["elem_to_sub"], s["coef"], sub_to_subregion=s["sub_to_subregion"],
                   node_dirichlet=s["node_dirichlet"])
        ss = Substructuring(s["nx"], s["elem_to_sub"], s["coef"], dirichlet=s["node_dirichlet"].astype(bool))
        M = BDDC(ss, sub_to_subregion=s["sub_to_subregion"])
        r = np.random.default_rng(3).standard_normal(ss.n_gamma)
        r -= r.mean()                                   # a consistent residual
        z = g.apply_precond(torch.tensor(r, device="cuda")).cpu().numpy()
        zo = M.apply(r)
        print("[gpu] %s M^-1 r rel diff %.2e" % (name, np.abs(z - zo).max() / np.abs(zo).max()), flush=True)
        assert np.abs(z - zo).max() <= 1e-9 * np.abs(zo).max()
