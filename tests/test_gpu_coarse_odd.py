"""GPU parity of the dense coarse product when the coarse dimension is odd
(its rows padded to an even length in device memory): the uneven holed
partition, two levels, with corners only (69 coarse DOFs) and with corners
and edges (131), against the oracle's BDDC and solves (preconditioner to
1e-9 relative, iterations within +-1, solutions to 1e-9 at rtol 1e-10)."""
import numpy as np
import pytest

import workload

pytestmark = pytest.mark.gpu


def _torch():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def _rel(a, b):
    return np.abs(np.asarray(a) - np.asarray(b)).max() / max(np.abs(np.asarray(b)).max(), 1e-300)


@pytest.mark.parametrize("cons,nc", [(("corners",), 69), (("corners", "edges"), 131)])
def test_odd_coarse_dimension_matches_oracle(cons, nc):
    torch = _torch()
    from oracle.sequence import OracleSolver
    from paper_2412_17543_amd.solver import Solver
    s = workload.workload("c3s")
    print("[gpu] c3s two-level constraints %s" % (cons,), flush=True)
    g = Solver(s["nx"], s["elem_to_sub"], s["coef"], elem_keep=s["elem_keep"], constraints=cons)
    assert g.info()["n_coarse"] == nc
    o = OracleSolver(s["nx"], s["elem_to_sub"], s["coef"], elem_keep=s["elem_keep"], constraints=cons)
    rng = np.random.default_rng(5)
    for _ in range(2):
        r = rng.standard_normal(o.ss.n_gamma)
        z = g.apply_precond(torch.tensor(r, device="cuda")).cpu().numpy()
        assert _rel(z, o.M.apply(r)) < 1e-9
    F = workload.rhs_sequence(s["nx"], 2, s["elem_keep"])
    U, its, rr = g.solve_sequence(torch.tensor(F, device="cuda"), 1e-10)
    uo, ito, _ = o.solve_sequence(F, 1e-10)
    print("[gpu] iters gpu %s oracle %s" % (its.tolist(), ito.tolist()), flush=True)
    assert np.all(np.abs(its - ito) <= 1)
    assert np.all(rr < 1e-10)
    for k in range(len(F)):
        assert _rel(U[k].cpu().numpy(), uo[k]) <= 1e-9


@pytest.mark.parametrize("cons", [("corners", "faces"), ("corners",)])
def test_three_level_chain_matches_oracle(cons):
    """Three levels applied as the subregion chain (level 3 through the same
    dense product on the padded K_3^{-1}; 3 level-3 DOFs here, an odd count)."""
    torch = _torch()
    from oracle.sequence import OracleSolver
    from paper_2412_17543_amd.solver import Solver
    s = workload.workload("c3s")
    g = Solver(s["nx"], s["elem_to_sub"], s["coef"], sub_to_subregion=s["sub_to_subregion"],
               elem_keep=s["elem_keep"], constraints=cons, coarse_form="chain")
    print("[gpu] c3s three-level chain %s: %s" % (cons, g.info()), flush=True)
    o = OracleSolver(s["nx"], s["elem_to_sub"], s["coef"], sub_to_subregion=s["sub_to_subregion"],
                     elem_keep=s["elem_keep"], constraints=cons)
    rng = np.random.default_rng(6)
    for _ in range(2):
        r = rng.standard_normal(o.ss.n_gamma)
        z = g.apply_precond(torch.tensor(r, device="cuda")).cpu().numpy()
        assert _rel(z, o.M.apply(r)) < 1e-9
