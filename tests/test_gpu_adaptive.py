"""GPU tests of the adaptive coarse space (Section 3.3) through the C ABI,
against the oracle's pair-space reading of eqs. eig-matrix and c-def.

The new rows are unique only up to their span (equal eigenvalues, signs), but
BDDC depends on the constraint rows only through the space of functions whose
coarse DOFs are continuous; so the preconditioners must agree as linear
operators (1e-9 relative on M r) and the solves as in the other parity tests
(rtol 1e-10: iterations within +-1, solution within 1e-9).
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


def _pair(name, coef, tau, **kw):
    from oracle.sequence import OracleSolver
    from paper_2412_17543_amd.solver import Solver
    s = workload.workload(name)
    keep = s.get("elem_keep")
    print("[gpu] adaptive setup %s tau %g" % (name, tau), flush=True)
    g = Solver(s["nx"], s["elem_to_sub"], coef, sub_to_subregion=s["sub_to_subregion"], elem_keep=keep,
               adapt_tau=tau, **kw)
    o = OracleSolver(s["nx"], s["elem_to_sub"], coef, sub_to_subregion=s["sub_to_subregion"], elem_keep=keep,
                     adaptive=(tau, 10), R=kw.get("R", 0))
    return s, g, o


def _precond_parity(torch, g, o, n=2):
    rng = np.random.default_rng(11)
    for _ in range(n):
        r = rng.standard_normal(o.ss.n_gamma)
        z = g.apply_precond(torch.tensor(r, device="cuda")).cpu().numpy()
        assert _rel(z, o.M.apply(r)) < 1e-9


def test_three_level_enriched_faces_match_oracle():
    torch = _torch()
    coef = np.exp(2.5 * np.random.default_rng(7).standard_normal(16 ** 3))
    s, g, o = _pair("tiny3", coef, 10.0)
    st = g.adaptive_stats()
    print("[gpu] tiny3 adaptive", st, o.M.counts(), flush=True)
    assert st["added"] == o.M.counts()["adaptive"] > 0
    assert st["faces"] == len(o.M.adapt_info)
    np.testing.assert_allclose(st["lam_max"], max(i["lam"][0] for i in o.M.adapt_info), rtol=1e-8)
    assert g.info()["n_coarse"] == o.M.nC
    _precond_parity(torch, g, o)


def test_two_level_enriched_sequence_matches_oracle():
    torch = _torch()
    coef = np.exp(2.0 * np.random.default_rng(5).standard_normal(8 ** 3))
    s, g, o = _pair("tiny", coef, 2.0, R=4)
    assert g.adaptive_stats()["added"] == o.M.counts()["adaptive"] > 0
    _precond_parity(torch, g, o)
    F = workload.rhs_sequence(8, 3)
    U, its, rr = g.solve_sequence(torch.tensor(F, device="cuda"), 1e-10)
    uo, ito, _ = o.solve_sequence(F, 1e-10)
    print("[gpu] tiny adaptive iters gpu %s oracle %s" % (its.tolist(), ito.tolist()), flush=True)
    assert np.all(np.abs(its - ito) <= 1)
    assert np.all(rr < 1e-10)
    for k in range(len(F)):
        assert _rel(U[k].cpu().numpy(), uo[k]) <= 1e-9


def test_uneven_partition_with_hole_enriched():
    torch = _torch()
    s = workload.workload("c3s")
    coef = s["coef"] * np.exp(1.5 * np.random.default_rng(3).standard_normal(s["nx"] ** 3))
    s, g, o = _pair("c3s", coef, 4.0)
    st = g.adaptive_stats()
    print("[gpu] c3s adaptive", st, o.M.counts(), flush=True)
    assert st["added"] == o.M.counts()["adaptive"] > 0
    _precond_parity(torch, g, o)


def test_threshold_above_every_eigenvalue_changes_nothing():
    torch = _torch()
    from paper_2412_17543_amd.solver import Solver
    s = workload.workload("tiny")
    coef = np.exp(np.random.default_rng(2).standard_normal(8 ** 3))
    g0 = Solver(s["nx"], s["elem_to_sub"], coef)
    g1 = Solver(s["nx"], s["elem_to_sub"], coef, adapt_tau=1e12)
    assert g1.adaptive_stats()["added"] == 0 and g1.adaptive_stats()["faces"] == 12
    r = torch.tensor(np.random.default_rng(4).standard_normal(g0.n_gamma), device="cuda")
    assert _rel(g1.apply_precond(r).cpu().numpy(), g0.apply_precond(r).cpu().numpy()) < 1e-14


def _level2_pair(e2s, coef, s2r, nx, tau2, tau1=0.0, R=0):
    from oracle.sequence import OracleSolver
    from paper_2412_17543_amd.solver import Solver
    print("[gpu] level-2 adaptive setup nx %d tau2 %g tau1 %g" % (nx, tau2, tau1), flush=True)
    g = Solver(nx, e2s, coef, sub_to_subregion=s2r, adapt_tau=tau1, adapt2_tau=tau2, R=R)
    o = OracleSolver(nx, e2s, coef, sub_to_subregion=s2r, adaptive=(tau1, 10) if tau1 > 0 else None,
                     adaptive2=(tau2, 10), R=R)
    return g, o


def _level2_counts_match(g, o):
    st = g.adaptive2_stats()
    info = o.M.level2.adapt2_info
    added = sum(d["kind"] == "adaptive2" for d in o.M.level2.dofs3)
    print("[gpu] level-2 adaptive", st, "oracle added", added, "n3", o.M.level2.n3, flush=True)
    assert st["faces"] == len(info)
    assert st["added"] == added > 0
    np.testing.assert_allclose(st["lam_max"], max(i["lam"][0] for i in info), rtol=1e-8)
    assert g.info()["level3"] == o.M.level2.n3


def test_level2_faces_two_subregions_match_oracle():
    torch = _torch()
    from tests.test_oracle_adaptive2 import two_subregion_problem
    ss, s2r = two_subregion_problem()
    g, o = _level2_pair(workload.cube_partition(16, 4), ss.coef, s2r, 16, 2.5, R=4)
    _level2_counts_match(g, o)
    _precond_parity(torch, g, o)
    F = workload.rhs_sequence(16, 3)
    U, its, rr = g.solve_sequence(torch.tensor(F, device="cuda"), 1e-10)
    uo, ito, _ = o.solve_sequence(F, 1e-10)
    print("[gpu] two-subregion level-2 iters gpu %s oracle %s" % (its.tolist(), ito.tolist()), flush=True)
    assert np.all(np.abs(its - ito) <= 1)
    for k in range(len(F)):
        assert _rel(U[k].cpu().numpy(), uo[k]) <= 1e-9


def test_level2_faces_with_level1_rows_match_oracle():
    # eight subregions, both levels enriched: the level-1 rows on the level-2
    # interface are level-3 DOFs of their own and enter the level-2 pencils' Pi
    torch = _torch()
    s = workload.workload("tiny3")
    coef = np.exp(2.5 * np.random.default_rng(7).standard_normal(16 ** 3))
    g, o = _level2_pair(s["elem_to_sub"], coef, s["sub_to_subregion"], 16, 2.0, tau1=10.0)
    assert g.adaptive_stats()["added"] == o.M.counts()["adaptive"] > 0
    _level2_counts_match(g, o)
    _precond_parity(torch, g, o)


def test_lobpcg_face_solver():
    # the face pencils by LOBPCG: run to convergence the preconditioner is the
    # exact-pencil one (oracle, 1e-7 on M r); with the paper's cap of 15
    # iterations the Ritz values are lower bounds, so no more rows are added
    # and the solves still converge to the tolerance
    torch = _torch()
    from oracle.sequence import OracleSolver
    from paper_2412_17543_amd.solver import Solver
    s = workload.workload("c16")
    coef = np.exp(2.0 * np.random.default_rng(5).standard_normal(16 ** 3))
    o = OracleSolver(16, s["elem_to_sub"], coef, adaptive=(2.0, 10), R=0)
    print("[gpu] lobpcg face solver setups", flush=True)
    ge = Solver(16, s["elem_to_sub"], coef, adapt_tau=2.0)
    gc = Solver(16, s["elem_to_sub"], coef, adapt_tau=2.0, adapt_lobpcg_it=500)
    g15 = Solver(16, s["elem_to_sub"], coef, adapt_tau=2.0, adapt_lobpcg_it=15)
    se, sc, s15 = ge.adaptive_stats(), gc.adaptive_stats(), g15.adaptive_stats()
    print("[gpu] lobpcg stats exact %s converged %s capped %s oracle %d" % (se, sc, s15, o.M.counts()["adaptive"]),
          flush=True)
    assert se["added"] == sc["added"] == o.M.counts()["adaptive"] > 0
    np.testing.assert_allclose(sc["lam_max"], se["lam_max"], rtol=1e-8)
    assert s15["added"] <= se["added"] and s15["lam_max"] <= se["lam_max"] * (1 + 1e-10)
    rng = np.random.default_rng(11)
    for _ in range(2):
        r = rng.standard_normal(o.ss.n_gamma)
        z = gc.apply_precond(torch.tensor(r, device="cuda")).cpu().numpy()
        assert _rel(z, o.M.apply(r)) < 1e-7
    F = torch.tensor(workload.rhs_sequence(16, 3), device="cuda")
    _, it_e, _ = ge.solve_sequence(F, 1e-10)
    _, it_15, rr = g15.solve_sequence(F, 1e-10)
    print("[gpu] lobpcg iterations exact %s capped %s" % (it_e.tolist(), it_15.tolist()), flush=True)
    assert np.all(rr < 1e-10) and np.all(it_15 <= it_e + 2)


def test_level2_faces_pure_neumann_match_oracle():
    # no Dirichlet node: every subregion floats, so both sides of every
    # level-2 face pencil are singular (the constant in the null space)
    torch = _torch()
    from oracle.bddc import BDDC
    from oracle.substructure import Substructuring
    from paper_2412_17543_amd.solver import Solver
    s = workload.workload("tiny3n")
    print("[gpu] level-2 adaptive, pure Neumann", flush=True)
    g = Solver(s["nx"], s["elem_to_sub"], s["coef"], sub_to_subregion=s["sub_to_subregion"],
               node_dirichlet=s["node_dirichlet"], adapt2_tau=2.0)
    ss = Substructuring(s["nx"], s["elem_to_sub"], s["coef"], dirichlet=s["node_dirichlet"].astype(bool))
    M = BDDC(ss, sub_to_subregion=s["sub_to_subregion"], adaptive2=(2.0, 10))
    added = sum(d["kind"] == "adaptive2" for d in M.level2.dofs3)
    st = g.adaptive2_stats()
    assert M.singular and st["added"] == added > 0 and g.info()["level3"] == M.level2.n3
    np.testing.assert_allclose(st["lam_max"], max(i["lam"][0] for i in M.level2.adapt2_info), rtol=1e-8)
    rng = np.random.default_rng(3)
    for _ in range(2):
        r = rng.standard_normal(ss.n_gamma)
        r -= r.mean()                                   # a consistent residual
        z = g.apply_precond(torch.tensor(r, device="cuda")).cpu().numpy()
        assert _rel(z, M.apply(r)) < 1e-9


def test_level2_faces_by_lobpcg_match_the_exact_pencils():
    # both levels enriched with the pencils solved by LOBPCG run to
    # convergence: the same rows (up to their span) as the exact solve
    torch = _torch()
    s = workload.workload("tiny3")
    coef = np.exp(2.5 * np.random.default_rng(7).standard_normal(16 ** 3))
    g, o = _level2_pair(s["elem_to_sub"], coef, s["sub_to_subregion"], 16, 2.0, tau1=10.0)
    from paper_2412_17543_amd.solver import Solver
    gl = Solver(16, s["elem_to_sub"], coef, sub_to_subregion=s["sub_to_subregion"], adapt_tau=10.0,
                adapt2_tau=2.0, adapt_lobpcg_it=500)
    assert gl.adaptive_stats()["added"] == g.adaptive_stats()["added"]
    assert gl.adaptive2_stats()["added"] == g.adaptive2_stats()["added"] > 0
    assert gl.info()["level3"] == o.M.level2.n3
    rng = np.random.default_rng(5)
    for _ in range(2):
        r = rng.standard_normal(o.ss.n_gamma)
        z = gl.apply_precond(torch.tensor(r, device="cuda")).cpu().numpy()
        assert _rel(z, o.M.apply(r)) < 1e-7
