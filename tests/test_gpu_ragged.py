"""GPU parity on a partition whose interfaces cover every form of the packed
operator layout: a one-element subdomain at a corner of the cube (interface
of 7 nodes: no full 16-row tile, the whole operator is the ragged-tail
strip; one interior node) carved out of a 2 x 2 x 2 partition of 8^3
(interfaces of 52 to 68 nodes: ragged tails of 4 rows stored as strips and
of 13 rows as zero-padded tiles; interiors of 48 to 64 nodes, two sizes
without a tail, one with an 8-row strip).  Against the FP64
oracle: Schur products (1e-12), preconditioner (1e-9), an FP64 sequence with
a recycled basis (iterations +-1, solutions 1e-9); and the block products of
the block adjoint (16-column tiles on the matrix cores) against the
column-by-column adjoint (1e-9).  Also: a 20-right-hand-side call (interior
condensation and recovery grouped 16 + 4 per pass over the interior tiles)
against 20 one-right-hand-side calls (iterations +-1, solutions 1e-9).
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


def ragged_partition():
    nx = 8
    part = workload.cube_partition(nx, 4)
    c = workload.element_centroids(nx)
    corner = np.all(c < 1.0 / nx, axis=1)
    assert corner.sum() == 1
    part = part.copy()
    part[corner] = part.max() + 1
    return nx, part


_PAIR = {}


def _pair(R):
    if R not in _PAIR:
        from oracle.sequence import OracleSolver
        from paper_2412_17543_amd.solver import Solver
        nx, part = ragged_partition()
        coef = np.ones(nx ** 3)
        print("[gpu] setup ragged partition R %d" % R, flush=True)
        _PAIR[R] = (Solver(nx, part, coef, R=R), OracleSolver(nx, part, coef, R=R))
    return _PAIR[R]


def test_interface_sizes_cover_the_layout():
    _torch()
    g, o = _pair(0)
    nb = np.array([d["Bpos"].size for d in o.ss.sub])
    print("[gpu] ragged interface sizes", nb.tolist(), flush=True)
    assert nb.min() < 16 and np.any(nb % 16 > 4) and g.n_gamma == o.ss.n_gamma


def test_ragged_schur_and_preconditioner():
    torch = _torch()
    g, o = _pair(0)
    rng = np.random.default_rng(11)
    for _ in range(3):
        p = rng.standard_normal(o.ss.n_gamma)
        q = g.apply_schur(torch.tensor(p, device="cuda")).cpu().numpy()
        assert _rel(q, o.ss.apply_A(p)) < 1e-12
        z = g.apply_precond(torch.tensor(p, device="cuda")).cpu().numpy()
        assert _rel(z, o.M.apply(p)) < 1e-9


def test_ragged_sequence_with_basis():
    torch = _torch()
    g, o = _pair(4)
    F = workload.rhs_sequence(8, 5)
    U, its, rr = g.solve_sequence(torch.tensor(F, device="cuda"), 1e-10)
    o.reset()
    uo, ito, _ = o.solve_sequence(F, 1e-10)
    print("[gpu] ragged iters gpu", its.tolist(), "oracle", ito.tolist(), flush=True)
    assert np.all(np.abs(its - ito) <= 1)
    assert np.all(rr < 1e-10)
    for k in range(len(F)):
        assert _rel(U[k].cpu().numpy(), uo[k]) <= 1e-9


def test_ragged_block_adjoint_equals_column_by_column():
    torch = _torch()
    g, o = _pair(0)
    F = torch.tensor(workload.rhs_sequence(8, 3), device="cuda")
    U, _, _ = g.solve_sequence(F, 1e-12)
    dLdu = 2.0 * (U - 0.9 * U.flip(0))
    g1, lam1 = g.adjoint_grad(dLdu, U, 1e-12)
    g2, lam2, it = g.adjoint_grad_block(dLdu, U, 1e-12)
    print("[gpu] ragged block adjoint: %d block iterations" % it, flush=True)
    assert _rel(lam2.cpu().numpy(), lam1.cpu().numpy()) <= 1e-9
    assert _rel(g2.cpu().numpy(), g1.cpu().numpy()) <= 1e-9


def test_grouped_condensation_and_recovery_equal_one_at_a_time():
    # one call with 20 right-hand sides condenses and recovers them in groups
    # of 16 and 4 (block products over the interior tiles); 20 calls of one
    # right-hand side take the one-vector path; same recycling sequence
    torch = _torch()
    from paper_2412_17543_amd.solver import Solver
    s = workload.workload("tiny3")
    F = torch.tensor(workload.rhs_sequence(16, 20), device="cuda")
    g1 = Solver(16, s["elem_to_sub"], s["coef"], sub_to_subregion=s["sub_to_subregion"], R=4)
    U1, it1, rr1 = g1.solve_sequence(F, 1e-10)
    g2 = Solver(16, s["elem_to_sub"], s["coef"], sub_to_subregion=s["sub_to_subregion"], R=4)
    res = [g2.solve_sequence(F[k:k + 1], 1e-10) for k in range(20)]
    U2 = torch.cat([r[0] for r in res])
    it2 = np.concatenate([r[1] for r in res])
    print("[gpu] grouped iterations", it1.tolist(), "one at a time", it2.tolist(), flush=True)
    assert np.all(np.abs(it1 - it2) <= 1)
    assert _rel(U1.cpu().numpy(), U2.cpu().numpy()) <= 1e-9
