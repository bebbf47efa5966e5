"""GPU tests of the solver's forms and options, through the C ABI, against the oracle.

Tolerances (same reasoning as test_gpu_parity.py):
  * graph-replayed and kernel-by-kernel iterations launch the same kernels in
    the same order on the same work lists: bitwise identical results;
  * options with an oracle counterpart (recycling strategies, stopping rule,
    zero initial guess, card weights, edge constraints) at rtol 1e-10:
    iterations within +-1, solution within 1e-9 relative;
  * bfloat16 local Neumann operators (float32 accumulation) at rtol 1e-8:
    the true float64 residual meets the tolerance and the solution is within
    1e-7 of the converged oracle solution;
  * adjoint gradient: solves at rtol 1e-12, gradient within 1e-8 of the
    oracle's direct-solve gradient (which the oracle tests pin to central
    differences), plus a direct finite-difference check through GPU solves;
  * three-level coarse operator applied through the subregion chain or as the
    explicit matrix assembled from it: the same linear operator up to
    rounding (1e-12 relative on M r, both within 1e-9 of the oracle).
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


def _solver(name, **kw):
    from paper_2412_17543_amd.solver import Solver
    s = workload.workload(name)
    coef = kw.pop("coef", s["coef"])
    print("[gpu] setup %s %s" % (name, sorted(kw)), flush=True)
    return Solver(s["nx"], s["elem_to_sub"], coef, sub_to_subregion=s["sub_to_subregion"], **kw)


def _oracle(name, **kw):
    from oracle.sequence import OracleSolver
    s = workload.workload(name)
    coef = kw.pop("coef", s["coef"])
    return OracleSolver(s["nx"], s["elem_to_sub"], coef, sub_to_subregion=s["sub_to_subregion"], **kw)


def _rel(a, b):
    a, b = np.asarray(a), np.asarray(b)
    return np.abs(a - b).max() / max(np.abs(b).max(), 1e-300)


@pytest.mark.parametrize("name,R", [("c16", 6), ("tiny3", 8)])
def test_launch_forms_agree_bitwise(name, R):
    """Queued stream launches (the default), graph replays and the plain
    kernel-by-kernel form run the same kernels in the same order."""
    torch = _torch()
    s = workload.workload(name)
    F = torch.tensor(workload.rhs_sequence(s["nx"], 4), device="cuda")
    # fixed work lists: the autotuner may pick different ones per context,
    # which changes the (deterministic) summation order
    U0, it0, _ = _solver(name, R=R, use_graph="plain", autotune=False).solve_sequence(F, 1e-10)
    for form in ("queued", "graph"):
        U1, it1, _ = _solver(name, R=R, use_graph=form, autotune=False).solve_sequence(F, 1e-10)
        np.testing.assert_array_equal(it1, it0)
        assert torch.equal(U1, U0), form


def test_repeated_sequence_is_bitwise_reproducible():
    torch = _torch()
    F = torch.tensor(workload.rhs_sequence(16, 4), device="cuda")
    g = _solver("c16", R=6)
    U1, it1, _ = g.solve_sequence(F, 1e-10)
    g.reset_recycle()
    U2, it2, _ = g.solve_sequence(F, 1e-10)
    np.testing.assert_array_equal(it1, it2)
    assert torch.equal(U1, U2)


def test_fixed_configuration_matches_autotuned():
    torch = _torch()
    F = torch.tensor(workload.rhs_sequence(16, 3), device="cuda")
    U1, it1, _ = _solver("tiny3", R=4, autotune=True).solve_sequence(F, 1e-10)
    U2, it2, _ = _solver("tiny3", R=4, autotune=False).solve_sequence(F, 1e-10)
    assert np.all(np.abs(it1 - it2) <= 1)
    for k in range(F.shape[0]):
        assert _rel(U1[k].cpu().numpy(), U2[k].cpu().numpy()) <= 1e-9


@pytest.mark.parametrize("strategy", ["B1", "B2", "B3"])
def test_recycling_strategies_match_oracle(strategy):
    torch = _torch()
    F = workload.rhs_sequence(16, 5)
    U, its, rr = _solver("c16", R=6, strategy=strategy).solve_sequence(torch.tensor(F, device="cuda"), 1e-10)
    uo, ito, _ = _oracle("c16", R=6, strategy=strategy).solve_sequence(F, 1e-10)
    print("[gpu] %s iters gpu %s oracle %s" % (strategy, its.tolist(), ito.tolist()), flush=True)
    assert np.all(np.abs(its - ito) <= 1)
    assert np.all(rr < 1e-10)
    for k in range(len(F)):
        assert _rel(U[k].cpu().numpy(), uo[k]) <= 1e-9


def test_residual_stopping_rule_and_zero_guess_match_oracle():
    torch = _torch()
    F = workload.rhs_sequence(16, 4)
    U, its, rr = _solver("tiny3", R=4, stop_rule="r0", init_guess="zero").solve_sequence(
        torch.tensor(F, device="cuda"), 1e-10)
    uo, ito, _ = _oracle("tiny3", R=4, stop="r0", init_guess="zero").solve_sequence(F, 1e-10)
    print("[gpu] r0/zero iters gpu %s oracle %s" % (its.tolist(), ito.tolist()), flush=True)
    assert np.all(np.abs(its - ito) <= 1)
    for k in range(len(F)):
        assert _rel(U[k].cpu().numpy(), uo[k]) <= 1e-9


def test_card_weights_edges_and_coefficients_precond_parity():
    torch = _torch()
    coef = workload.lognormal_coef(16 ** 3, 0.5)
    kw = dict(coef=coef, weights="card", constraints=("corners", "faces", "edges"))
    g = _solver("tiny3", **kw)
    from oracle.sequence import OracleSolver
    s = workload.workload("tiny3")
    o = OracleSolver(s["nx"], s["elem_to_sub"], coef, sub_to_subregion=s["sub_to_subregion"],
                     weight_kind="card", constraints=("corners", "faces", "edges"))
    info = g.info()
    assert info["edges"] == o.M.counts()["edges"]
    rng = np.random.default_rng(5)
    for _ in range(2):
        r = rng.standard_normal(o.ss.n_gamma)
        z = g.apply_precond(torch.tensor(r, device="cuda")).cpu().numpy()
        assert _rel(z, o.M.apply(r)) < 1e-9
        p = rng.standard_normal(o.ss.n_gamma)
        q = g.apply_schur(torch.tensor(p, device="cuda")).cpu().numpy()
        assert _rel(q, o.ss.apply_A(p)) < 1e-12


def test_bf16_neumann_operators_c16():
    torch = _torch()
    F = workload.rhs_sequence(16, 4)
    U, its, rr = _solver("c16", local_prec=16).solve_sequence(torch.tensor(F, device="cuda"), 1e-8)
    _, it64, _ = _solver("c16").solve_sequence(torch.tensor(F, device="cuda"), 1e-8)
    uo = _oracle("c16").solve_sequence(F, 1e-12)[0]
    print("[gpu] bf16 iters %s fp64 %s" % (its.tolist(), it64.tolist()), flush=True)
    assert np.all(rr < 1e-8)
    for k in range(len(F)):
        assert _rel(U[k].cpu().numpy(), uo[k]) <= 1e-7


def test_zero_rhs_and_iteration_limit():
    torch = _torch()
    from paper_2412_17543_amd._lib import BddcError
    g = _solver("c16", R=4)
    F = torch.zeros(2, workload.n_nodes(16), dtype=torch.float64, device="cuda")
    U, its, rr = g.solve_sequence(F, 1e-8)
    assert np.all(its == 0) and float(U.abs().max()) == 0.0
    g2 = _solver("c16", max_it=2)
    Fr = torch.tensor(workload.rhs_sequence(16, 1), device="cuda")
    with pytest.raises(BddcError) as e:
        g2.solve_sequence(Fr, 1e-12)
    assert "ENOTCONV" in str(e.value)


def _adjoint_problem(nx=16, n_rhs=3):
    from oracle import q1
    F = workload.rhs_sequence(nx, n_rhs)
    g = np.random.default_rng(4)
    theta_t = 0.5 * g.standard_normal(nx ** 3)
    T = q1.direct_solve(nx, np.exp(theta_t), F)
    theta = 0.3 * g.standard_normal(nx ** 3)
    return F, T, theta


def _gpu_loss_and_grad(torch, theta, F, T, R=4, rtol=1e-12):
    from paper_2412_17543_amd.solver import DPCGSolveFn
    s = workload.workload("c16")
    th = torch.tensor(theta, device="cuda", requires_grad=True)
    Ft = torch.tensor(F, device="cuda", requires_grad=True)
    spec = dict(nx=16, elem_to_sub=s["elem_to_sub"], R=R, rtol=rtol, autotune=False)
    U = DPCGSolveFn.apply(th, Ft, spec)
    L = ((U - torch.tensor(T, device="cuda")) ** 2).sum()
    L.backward()
    return L.item(), th.grad.cpu().numpy(), Ft.grad.cpu().numpy()


def test_adjoint_gradient_matches_oracle():
    torch = _torch()
    from oracle import adjoint
    F, T, theta = _adjoint_problem()
    L, g, gF = _gpu_loss_and_grad(torch, theta, F, T)
    Lo, go, lam, _ = adjoint.loss_and_grad(16, theta, F, T)
    assert abs(L - Lo) <= 1e-9 * Lo
    assert _rel(g, go) <= 1e-8
    assert _rel(gF, lam) <= 1e-8


def _fd_err(fd, g):
    """|g - FD| / max(|FD|, 1e-3 max |FD|), the per-entry measure of the
    finite-difference checks."""
    return np.abs(g - fd) / np.maximum(np.abs(fd), 1e-3 * np.abs(fd).max())


def test_adjoint_gradient_50_elements_central_differences():
    # 50 seeded element indices of the 16^3 mesh (2x2x2 subdomains, two
    # levels), every solve at rtol 1e-13; central differences of step 1e-4:
    # at 1e-6 the rounding of L alone puts even direct-solve differences
    # 5e-4 off (the CPU pin of the step), at 1e-4 truncation (O(1e-8)) and
    # rounding stay below 1e-5; each entry must agree to 1e-5
    torch = _torch()
    F, T, theta = _adjoint_problem()
    rtol = 1e-13
    L, g, _ = _gpu_loss_and_grad(torch, theta, F, T, R=0, rtol=rtol)
    eps = 1e-4
    idx = workload.rng("fd").choice(16 ** 3, 50, replace=False)
    fd = []
    for e in idx:
        tp, tm = theta.copy(), theta.copy()
        tp[e] += eps
        tm[e] -= eps
        Lp = _gpu_loss_and_grad(torch, tp, F, T, R=0, rtol=rtol)[0]
        Lm = _gpu_loss_and_grad(torch, tm, F, T, R=0, rtol=rtol)[0]
        fd.append((Lp - Lm) / (2 * eps))
    err = _fd_err(np.array(fd), g[idx])
    print("[gpu] per-element FD errors: max %.2e median %.2e" % (err.max(), np.median(err)), flush=True)
    assert err.max() <= 1e-5


def test_adjoint_gradient_50_random_directions():
    # directional central differences (step 1e-4) along 50 seeded random unit
    # directions in the space of element log-coefficients (16^3), each
    # direction to 1e-5
    torch = _torch()
    F, T, theta = _adjoint_problem()
    rtol = 1e-13
    L, g, _ = _gpu_loss_and_grad(torch, theta, F, T, R=0, rtol=rtol)
    eps = 1e-4
    rng = workload.rng("fd", 1)
    fd, gv = [], []
    for _ in range(50):
        v = rng.standard_normal(theta.size)
        v /= np.linalg.norm(v)
        Lp = _gpu_loss_and_grad(torch, theta + eps * v, F, T, R=0, rtol=rtol)[0]
        Lm = _gpu_loss_and_grad(torch, theta - eps * v, F, T, R=0, rtol=rtol)[0]
        fd.append((Lp - Lm) / (2 * eps))
        gv.append(g @ v)
    err = _fd_err(np.array(fd), np.array(gv))
    print("[gpu] directional FD errors: max %.2e median %.2e" % (err.max(), np.median(err)), flush=True)
    assert err.max() <= 1e-5


def test_adjoint_rhs_gradient_10_directions():
    # L is quadratic in F: a central difference along any direction is exact
    # up to rounding, so a large step is used and the agreement is tight
    torch = _torch()
    F, T, theta = _adjoint_problem()
    L, g, gF = _gpu_loss_and_grad(torch, theta, F, T, R=4, rtol=1e-13)
    rng = workload.rng("fd", 2)
    free = (np.arange(F.shape[1]) % 17) != 16
    for _ in range(10):
        d = rng.standard_normal(F.shape) * free
        eps = 1e-2 * np.abs(F).max() / np.abs(d).max()
        Lp = _gpu_loss_and_grad(torch, theta, F + eps * d, T, R=4, rtol=1e-13)[0]
        Lm = _gpu_loss_and_grad(torch, theta, F - eps * d, T, R=4, rtol=1e-13)[0]
        fd = (Lp - Lm) / (2 * eps)
        an = float((gF * d).sum())
        assert abs(fd - an) <= 1e-8 * abs(an), (fd, an)


def _hole_solver(name, **kw):
    from paper_2412_17543_amd.solver import Solver
    s = workload.workload(name)
    print("[gpu] setup %s %s" % (name, sorted(kw)), flush=True)
    return Solver(s["nx"], s["elem_to_sub"], s["coef"], sub_to_subregion=s["sub_to_subregion"],
                  elem_keep=s["elem_keep"], **kw)


@pytest.mark.parametrize("prec", [64, 32])
def test_uneven_partition_with_hole_matches_oracle(prec):
    # jittered RCB subdomains of very different sizes around a spherical hole,
    # log-normal coefficients, three levels, recycling
    torch = _torch()
    from oracle.sequence import OracleSolver
    s = workload.workload("c3s")
    F = workload.rhs_sequence(s["nx"], 3, s["elem_keep"])
    rtol = 1e-10 if prec == 64 else 1e-8
    U, its, rr = _hole_solver("c3s", R=6, local_prec=prec).solve_sequence(torch.tensor(F, device="cuda"), rtol)
    o = OracleSolver(s["nx"], s["elem_to_sub"], s["coef"], elem_keep=s["elem_keep"],
                     sub_to_subregion=s["sub_to_subregion"], R=6)
    uo, ito, _ = o.solve_sequence(F, 1e-10 if prec == 64 else 1e-12)
    print("[gpu] c3s fp%d iters gpu %s oracle %s" % (prec, its.tolist(), ito.tolist()), flush=True)
    assert np.all(rr < rtol)
    if prec == 64:
        assert np.all(np.abs(its - ito) <= 1)
    for k in range(len(F)):
        assert _rel(U[k].cpu().numpy(), uo[k]) <= (1e-9 if prec == 64 else 1e-7)


@pytest.mark.parametrize("name", ["tiny3", "c3s"])
def test_explicit_three_level_operator_matches_subregion_chain(name):
    torch = _torch()
    from oracle.sequence import OracleSolver
    s = workload.workload(name)
    mk = _hole_solver if name == "c3s" else _solver
    gc = mk(name, coarse_form="chain")
    ge = mk(name, coarse_form="explicit")
    o = OracleSolver(s["nx"], s["elem_to_sub"], s["coef"], elem_keep=s["elem_keep"],
                     sub_to_subregion=s["sub_to_subregion"])
    rng = np.random.default_rng(11)
    for _ in range(2):
        r = rng.standard_normal(o.ss.n_gamma)
        zc = gc.apply_precond(torch.tensor(r, device="cuda")).cpu().numpy()
        ze = ge.apply_precond(torch.tensor(r, device="cuda")).cpu().numpy()
        zo = o.M.apply(r)
        assert _rel(ze, zc) < 1e-12
        assert _rel(zc, zo) < 1e-9 and _rel(ze, zo) < 1e-9
    F = workload.rhs_sequence(s["nx"], 2, s["elem_keep"])
    Ft = torch.tensor(F, device="cuda")
    Uc, itc, _ = gc.solve_sequence(Ft, 1e-10)
    Ue, ite, _ = ge.solve_sequence(Ft, 1e-10)
    assert np.all(np.abs(itc - ite) <= 1)
    for k in range(len(F)):
        assert _rel(Ue[k].cpu().numpy(), Uc[k].cpu().numpy()) <= 1e-9


def test_pinned_product_configuration():
    torch = _torch()
    from paper_2412_17543_amd._lib import BddcError
    pin = [3, 0, 4, 2, 2, 1, 4, 4]       # Schur: balanced ranges; Neumann: per-subdomain
    g = _solver("tiny3", R=4, product_cfg=pin)
    t = g.tuning()
    assert (t["schur"]["blocks_per_cu"], t["schur"]["per_subdomain"], t["schur"]["waves"], t["schur"]["unroll"]) == (3, 0, 4, 2)
    assert (t["neumann"]["per_subdomain"], t["neumann"]["waves"], t["neumann"]["unroll"]) == (1, 4, 4)
    F = workload.rhs_sequence(16, 3)
    U, its, _ = g.solve_sequence(torch.tensor(F, device="cuda"), 1e-10)
    uo, ito, _ = _oracle("tiny3", R=4).solve_sequence(F, 1e-10)
    assert np.all(np.abs(its - ito) <= 1)
    for k in range(len(F)):
        assert _rel(U[k].cpu().numpy(), uo[k]) <= 1e-9
    with pytest.raises(BddcError):
        _solver("tiny3", product_cfg=[2, 1, 5, 2, 0, 0, 0, 0])


@pytest.mark.parametrize("name,nsub,pin_n", [("tiny3", 64, [8, 0, 4, 2]), ("c16", 8, [8, 1, 8, 4]),
                                              ("c16", 8, [8, 0, 8, 4])])
def test_split_neumann_products_restrict_once(name, nsub, pin_n):
    """The coarse restriction c_i = (D Phi_i)^T r_i is formed by the first
    work segment of each subdomain inside the Neumann product.  With many
    small blocks (balanced ranges, or several chunks per subdomain) every
    subdomain is split over blocks, and the preconditioner must still match
    the oracle's (eqs. averaging_subdomain_solves, coarse_problem); the
    float32 operators (another tail variant) agree to their precision."""
    torch = _torch()
    pin = [3, 1, 4, 2] + pin_n
    g = _solver(name, product_cfg=pin, local_prec_set=(32,))
    t = g.tuning()["neumann"]
    assert (t["per_subdomain"], t["waves"], t["unroll"]) == tuple(pin_n[1:])
    assert t["blocks"] > nsub                    # more blocks than subdomains
    o = _oracle(name)
    rng = np.random.default_rng(5)
    for _ in range(2):
        r = rng.standard_normal(o.ss.n_gamma)
        z = g.apply_precond(torch.tensor(r, device="cuda")).cpu().numpy()
        assert _rel(z, o.M.apply(r)) < 1e-9
        g.set_local_prec(32)
        z32 = g.apply_precond(torch.tensor(r, device="cuda")).cpu().numpy()
        g.set_local_prec(64)
        assert _rel(z32, z) < 1e-5


def test_reorthogonalisation_matches_oracle():
    torch = _torch()
    F = workload.rhs_sequence(16, 5)
    U, its, rr = _solver("tiny3", R=6, reorth=True).solve_sequence(torch.tensor(F, device="cuda"), 1e-10)
    uo, ito, _ = _oracle("tiny3", R=6, reorth=True).solve_sequence(F, 1e-10)
    print("[gpu] reorth iters gpu %s oracle %s" % (its.tolist(), ito.tolist()), flush=True)
    assert np.all(np.abs(its - ito) <= 1)
    assert np.all(rr < 1e-10)
    for k in range(len(F)):
        assert _rel(U[k].cpu().numpy(), uo[k]) <= 1e-9
