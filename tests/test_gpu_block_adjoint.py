"""GPU tests of the block adjoint (bddc_adjoint_grad_block: the adjoint
systems of Appendix B solved together by block deflated PCG) through the C
ABI, against the oracle:

* 16^3 three levels with a recycled basis W (R = 6 after three forward
  solves), 5 right-hand sides at rtol 1e-10 (above the floor that rounding
  in the deflated start, a residual part along W that directions
  A-orthogonal to W cannot remove, puts near 1e-11 here): block iterations
  within +-1 of
  the oracle's block PCG (oracle/block.py, same method and stopping rule),
  every adjoint solution lambda_k within 1e-9 of the oracle's, the gradient
  within 1e-8 of the oracle's direct-solve gradient;
* dependent right-hand sides (a repeated column, a zero column, a
  combination): the dropped directions leave the solutions equal to the
  independent ones (1e-9) and the zero column's lambda zero;
* 96^3, 1,728 subdomains, 20 right-hand sides: the block gradient equals the
  column-by-column gradient of bddc_adjoint_grad (1e-8) and satisfies
  sum_e dL/dtheta_e = -sum_k lambda_k^T F_k (1e-8).
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


def _rel(a, b):
    a, b = np.asarray(a), np.asarray(b)
    return np.abs(a - b).max() / max(np.abs(b).max(), 1e-300)


def _tiny3_pair(R=6, n_prev=3):
    from oracle.sequence import OracleSolver
    from paper_2412_17543_amd.solver import Solver
    s = workload.workload("tiny3")
    coef = np.exp(0.7 * np.random.default_rng(3).standard_normal(16 ** 3))
    print("[gpu] block adjoint setup tiny3 R %d" % R, flush=True)
    g = Solver(16, s["elem_to_sub"], coef, sub_to_subregion=s["sub_to_subregion"], R=R)
    o = OracleSolver(16, s["elem_to_sub"], coef, sub_to_subregion=s["sub_to_subregion"], R=R)
    return s, coef, g, o


def test_block_adjoint_matches_oracle_with_basis():
    torch = _torch()
    from oracle import adjoint, block
    s, coef, g, o = _tiny3_pair()
    Fp = workload.rhs_sequence(16, 3)
    g.solve_sequence(torch.tensor(Fp, device="cuda"), 1e-10)
    o.solve_sequence(Fp, 1e-10)
    assert o.rec.basis(o.ss.n_gamma).shape[1] > 0
    F = workload.rhs_sequence(16, 5, first=20)
    T = 0.9 * workload.rhs_sequence(16, 5, first=40)
    Lo, go, lam_d, U = adjoint.loss_and_grad(16, np.log(coef), F, T)
    dLdu = 2.0 * (U - T)
    lam_o, res = block.adjoint_block(o, dLdu, rtol=1e-10)
    print("[gpu] block adjoint (oracle) iterations %d ranks %s" % (res["iters"], res["ranks"][:3]), flush=True)
    grad, lam, it = g.adjoint_grad_block(torch.tensor(dLdu, device="cuda"), torch.tensor(U, device="cuda"), 1e-10)
    lam = lam.cpu().numpy()
    print("[gpu] block adjoint iterations gpu %d oracle %d, lambda rel %.2e" % (it, res["iters"], _rel(lam, lam_o)),
          flush=True)
    assert abs(it - res["iters"]) <= 1
    assert _rel(lam, lam_o) <= 1e-9
    assert _rel(grad.cpu().numpy(), go) <= 1e-8


def test_block_adjoint_dependent_columns():
    torch = _torch()
    s, coef, g, o = _tiny3_pair(R=0)
    F = workload.rhs_sequence(16, 2, first=5)
    G = np.stack([F[0], F[1], F[0], np.zeros_like(F[0]), F[0] + 2.0 * F[1]])
    U = np.zeros_like(G)
    _, lam, it = g.adjoint_grad_block(torch.tensor(G, device="cuda"), torch.tensor(U, device="cuda"), 1e-11)
    _, lam2, it2 = g.adjoint_grad_block(torch.tensor(G[:2], device="cuda"), torch.tensor(U[:2], device="cuda"), 1e-11)
    lam, lam2 = lam.cpu().numpy(), lam2.cpu().numpy()
    print("[gpu] dependent columns: iterations %d (independent pair %d)" % (it, it2), flush=True)
    assert _rel(lam[0], lam2[0]) <= 1e-9 and _rel(lam[1], lam2[1]) <= 1e-9
    assert _rel(lam[2], lam2[0]) <= 1e-9
    assert np.all(lam[3] == 0.0)
    assert _rel(lam[4], lam2[0] + 2.0 * lam2[1]) <= 1e-9


def test_block_adjoint_c96_equals_column_by_column():
    torch = _torch()
    from paper_2412_17543_amd.solver import Solver
    s = workload.workload("c96")
    print("[gpu] setup c96 for the block adjoint", flush=True)
    g = Solver(96, s["elem_to_sub"], s["coef"], sub_to_subregion=s["sub_to_subregion"], R=s["R"])
    F = torch.tensor(workload.rhs_sequence(96, 20), device="cuda")
    U, its, rr = g.solve_sequence(F, 1e-10)
    t = U * (1.0 + 0.1 * torch.tensor(workload.rng("target", 96).standard_normal(U.shape), device="cuda"))
    dLdu = 2.0 * (U - t)
    torch.cuda.synchronize()
    import time
    t0 = time.perf_counter()
    g1, lam1 = g.adjoint_grad(dLdu, U, 1e-12)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    g2, lam2, it = g.adjoint_grad_block(dLdu, U, 1e-12)
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    print("[gpu] c96 adjoint 20 rhs: column by column %.3f s, block %.3f s (%d block iterations)"
          % (t1 - t0, t2 - t1, it), flush=True)
    assert _rel(g2.cpu().numpy(), g1.cpu().numpy()) <= 1e-8
    assert _rel(lam2.cpu().numpy(), lam1.cpu().numpy()) <= 1e-8
    lhs = float(g2.sum().item())
    rhs = -float((lam2 * F).sum().item())
    assert abs(lhs - rhs) <= 1e-8 * abs(rhs)


def test_block_adjoint_rejects_too_many_columns():
    torch = _torch()
    from paper_2412_17543_amd._lib import BddcError
    s, coef, g, o = _tiny3_pair(R=0)
    G = torch.zeros((33, g.n_nodes), dtype=torch.float64, device="cuda")
    with pytest.raises(BddcError):
        g.adjoint_grad_block(G, G, 1e-10)
