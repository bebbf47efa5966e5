"""The oracle still reproduces the stored C1-sized (16^3) results and the closed-form counts."""
import json
import os

import numpy as np
import pytest

import workload
from oracle.sequence import OracleSolver

HERE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def test_c16_golden_iterations():
    g = json.load(open(os.path.join(HERE, "c16_oracle.json")))
    # closed form for a 2x2x2 cube partition with the x=1 face Dirichlet:
    # 1 interior + 5 face lattice corners, 12 faces, 3 interface planes of 17^2 nodes
    # minus the x=1 column and the 2*17+... overlaps = 784
    assert (g["corners"], g["faces"], g["n_gamma"]) == (6, 12, 784)
    s = workload.workload("c16")
    o = OracleSolver(16, s["elem_to_sub"], s["coef"])
    F = workload.rhs_sequence(16, 3)
    idx = np.array(g["sample_nodes"])
    for k in range(3):
        r = o.solve(F[k], 1e-8)
        assert r["iters"] == g["rtol_1e-08"]["iters"][k]
        np.testing.assert_allclose(r["u"][idx], g["rtol_1e-08"]["u_sample"][k], rtol=0,
                                   atol=1e-12 * np.abs(r["u"]).max())


def test_c64_golden_counts():
    p = os.path.join(HERE, "c64_oracle.json")
    if not os.path.exists(p):
        pytest.skip("c64 golden not generated")
    g = json.load(open(p))
    m = 8
    assert g["corners"] == (m - 1) ** 3 + 5 * (m - 1) ** 2
    assert g["faces"] == 3 * (m - 1) * m * m
    assert g["n_gamma"] == 78652
    assert g["level3"] == (4 - 1) ** 3 + 5 * (4 - 1) ** 2 + 3 * (4 - 1) * 4 * 4


def test_rcb_workload_is_face_connected_and_grouped():
    # the uneven-batching inputs: every subdomain one face-connected piece of
    # kept elements, subregions of equal count, removed elements excluded
    import numpy as np
    s = workload.workload("c3s")
    keep, part = s["elem_keep"], s["elem_to_sub"]
    assert s["n_sub"] == 24 and (keep == 0).sum() > 0
    lab = workload._face_components(24, part.astype(np.int64), keep)
    assert int(lab.max()) + 1 == 24
    assert np.all(np.bincount(s["sub_to_subregion"]) == 8)
    assert np.all(np.bincount(part[keep.astype(bool)], minlength=24) > 0)
