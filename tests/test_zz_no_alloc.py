"""The allocation-free Schur product against the allocating one, through the
C ABI: bitwise equal (the same kernels, the same work lists, only the partial
buffer differs), on two calls in a row with the second on a smaller problem,
then the rejection of a work list larger than the static array."""
import ctypes

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
    print("[gpu] setup %s %s" % (name, kw), flush=True)
    return Solver(s["nx"], s["elem_to_sub"], s["coef"], sub_to_subregion=s["sub_to_subregion"], **kw)


def _noalloc(g, p):
    from paper_2412_17543_amd._lib import check
    q = p.new_empty(p.shape)
    check(g.lib.bddc_apply_schur_noalloc(g.ctx, ctypes.c_void_p(p.data_ptr()), ctypes.c_void_p(q.data_ptr())))
    return q


def test_noalloc_schur_matches_allocating_entry_point():
    torch = _torch()
    rng = np.random.default_rng(11)
    for name in ("c64", "c16"):          # the second call on a smaller problem
        g = _solver(name)
        p = torch.tensor(rng.standard_normal(g.n_gamma), device="cuda")
        q_ref = g.apply_schur(p)
        q = _noalloc(g, p)
        print("[gpu] %s n_gamma %d max |diff| %.3e" % (name, g.n_gamma, float((q - q_ref).abs().max())), flush=True)
        assert torch.equal(q, q_ref)
        # again, after the other entry point ran on the same data
        assert torch.equal(_noalloc(g, p), q_ref)


def test_noalloc_schur_rejects_work_lists_beyond_the_array():
    # 96^3 with the product split into equal ranges over 8 blocks per compute
    # unit: about 3,800 work items of ~358 partials each, 1.35M doubles, more
    # than the 2^20 the static array holds
    torch = _torch()
    from paper_2412_17543_amd._lib import BddcError
    g = _solver("c96", autotune=False, product_cfg=[8, 0, 8, 4, 0, 0, 0, 0])
    p = torch.ones(g.n_gamma, dtype=torch.float64, device="cuda")
    with pytest.raises(BddcError) as e:
        _noalloc(g, p)
    assert "EINVAL" in str(e.value) and "static array holds 1048576" in str(e.value)
