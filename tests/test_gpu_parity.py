"""GPU parity: the HIP path through the C ABI against the FP64 CPU oracle.

Tolerances:
  * operator applications (Schur product, condensation): 1e-12 relative --
    both sides compute the same sums in float64, only the order differs;
  * preconditioner: 1e-9 relative -- the GPU inverts dense local saddle
    matrices by Gauss-Jordan, the oracle factors sparse ones by LU; local
    condition numbers up to ~1e6 bound the difference;
  * full solves in float64 at rtol 1e-10: solution relative error <= 1e-9 and
    iteration counts within +-1;
  * mixed precision (float32 local Neumann operators) at rtol 1e-8: solution
    error <= 1e-7 and at most 10% (+1) more iterations than float64.
"""
import json
import os

import numpy as np
import pytest

import workload

pytestmark = pytest.mark.gpu

HERE = os.path.dirname(os.path.abspath(__file__))


def _torch():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def _solver(name, **kw):
    from paper_2412_17543_amd.solver import Solver
    s = workload.workload(name)
    print("[gpu] setup %s %s" % (name, kw), flush=True)
    return Solver(s["nx"], s["elem_to_sub"], s["coef"], sub_to_subregion=s["sub_to_subregion"], **kw)


_ORACLES = {}


def _oracle(name, **kw):
    from oracle.sequence import OracleSolver
    key = (name, tuple(sorted(kw.items())))
    if key not in _ORACLES:
        s = workload.workload(name)
        _ORACLES[key] = OracleSolver(s["nx"], s["elem_to_sub"], s["coef"],
                                     sub_to_subregion=s["sub_to_subregion"], **kw)
    return _ORACLES[key]


def _rel(a, b):
    return np.abs(np.asarray(a) - np.asarray(b)).max() / max(np.abs(np.asarray(b)).max(), 1e-300)


@pytest.mark.parametrize("name", ["tiny", "c16", "tiny3"])
def test_structure_matches_oracle(name):
    _torch()
    g = _solver(name)
    o = _oracle(name)
    info = g.info()
    cnt = o.M.counts()
    assert info["n_gamma"] == o.ss.n_gamma
    assert (info["corners"], info["faces"]) == (cnt["corners"], cnt["faces"])
    np.testing.assert_array_equal(g.interface_nodes(), o.ss.gamma)
    if o.M.three_level:
        L2 = o.M.level2
        assert info["level2_interface"] == L2.gamma2.size
        assert info["level3"] == L2.n3


@pytest.mark.parametrize("name", ["tiny", "c16", "tiny3"])
def test_schur_and_condense_parity(name):
    torch = _torch()
    g = _solver(name)
    o = _oracle(name)
    rng = np.random.default_rng(1)
    for _ in range(3):
        p = rng.standard_normal(o.ss.n_gamma)
        q = g.apply_schur(torch.tensor(p, device="cuda")).cpu().numpy()
        assert _rel(q, o.ss.apply_A(p)) < 1e-12
    F = workload.rhs_sequence(o.ss.nx, 1)[0]
    b = g.condense(torch.tensor(F, device="cuda")).cpu().numpy()
    assert _rel(b, o.ss.condense(F)) < 1e-12


@pytest.mark.parametrize("name", ["tiny", "c16", "tiny3"])
def test_preconditioner_parity(name):
    torch = _torch()
    g = _solver(name)
    o = _oracle(name)
    rng = np.random.default_rng(2)
    for _ in range(3):
        r = rng.standard_normal(o.ss.n_gamma)
        z = g.apply_precond(torch.tensor(r, device="cuda")).cpu().numpy()
        assert _rel(z, o.M.apply(r)) < 1e-9


def test_preconditioner_is_deterministic():
    torch = _torch()
    g = _solver("tiny3")
    r = torch.tensor(np.random.default_rng(3).standard_normal(g.n_gamma), device="cuda")
    z1 = g.apply_precond(r).cpu().numpy()
    z2 = g.apply_precond(r).cpu().numpy()
    np.testing.assert_array_equal(z1, z2)


@pytest.mark.parametrize("name,R", [("c16", 0), ("tiny3", 0), ("c16", 6), ("tiny3", 8)])
def test_fp64_sequence_parity(name, R):
    torch = _torch()
    s = workload.workload(name)
    n_rhs = 5
    F = workload.rhs_sequence(s["nx"], n_rhs)
    g = _solver(name, R=R)
    U, its, rr = g.solve_sequence(torch.tensor(F, device="cuda"), 1e-10)
    o = _oracle(name, R=R)
    o.reset()
    uo, ito, rro = o.solve_sequence(F, 1e-10)
    print("[gpu] iters gpu", its.tolist(), "oracle", ito.tolist(), flush=True)
    assert np.all(np.abs(its - ito) <= 1), (its, ito)
    assert np.all(rr < 1e-10)
    for k in range(n_rhs):
        assert _rel(U[k].cpu().numpy(), uo[k]) <= 1e-9


def test_mixed_fp32_c16():
    torch = _torch()
    F = workload.rhs_sequence(16, 6)
    g64 = _solver("c16")
    _, it64, _ = g64.solve_sequence(torch.tensor(F, device="cuda"), 1e-8)
    g32 = _solver("c16", local_prec=32)
    U, it32, rr = g32.solve_sequence(torch.tensor(F, device="cuda"), 1e-8)
    ud = _oracle("c16").solve_sequence(F, 1e-12)[0]
    assert np.all(rr < 1e-8)
    assert it32.sum() <= 1.1 * it64.sum() + 1, (it32, it64)
    for k in range(len(F)):
        assert _rel(U[k].cpu().numpy(), ud[k]) <= 1e-7


def test_c64_sampled_against_golden():
    torch = _torch()
    gold = json.load(open(os.path.join(HERE, "golden", "c64_oracle.json")))
    rec = gold["rtol_1e-10"]
    n = gold["n_rhs"]
    F = workload.rhs_sequence(64, n)
    g = _solver("c64", R=gold["R"])
    info = g.info()
    assert (info["n_gamma"], info["corners"], info["faces"]) == (gold["n_gamma"], gold["corners"], gold["faces"])
    assert (info["level2_interface"], info["level2_interior"], info["level3"]) == (
        gold["level2_interface"], gold["level2_interior"], gold["level3"])
    U, its, rr = g.solve_sequence(torch.tensor(F, device="cuda"), 1e-10)
    print("[gpu] c64 iters gpu", its.tolist(), "oracle", rec["iters"], flush=True)
    idx = np.array(gold["sample_nodes"])
    for k in range(n):
        u = U[k].cpu().numpy()
        assert abs(int(its[k]) - rec["iters"][k]) <= 1
        assert abs(np.linalg.norm(u) - rec["u_norm2"][k]) <= 1e-9 * rec["u_norm2"][k]
        assert np.abs(u[idx] - np.array(rec["u_sample"][k])).max() <= 1e-9 * np.abs(u).max()
