"""Plant plausible mistakes in the oracle (on the CPU) and check that a pin fails.

Each planted bug is a monkeypatch of one oracle function; the pin that should
catch it is re-run and must raise.
"""
import numpy as np
import pytest

from oracle import adaptive, bddc, q1
from tests import test_oracle_adaptive as ta
from tests import test_oracle_bddc as tb
from tests import test_oracle_q1 as tq


def test_wrong_kref_entry_is_caught(monkeypatch):
    orig = q1.kref

    def bad():
        K = orig()
        K[0, 7] = K[7, 0] = 0.0          # dropped body-diagonal coupling
        return K
    monkeypatch.setattr(q1, "kref", bad)
    with pytest.raises(AssertionError):
        tq.test_kref_matches_quadrature()
    with pytest.raises(AssertionError):
        tq.test_kref_kernel_is_constants()


def test_unnormalised_weights_are_caught(monkeypatch):
    orig = bddc.weights
    monkeypatch.setattr(bddc, "weights", lambda ss, kind="diag": [np.ones_like(d) for d in orig(ss, kind)])
    with pytest.raises(AssertionError):
        tb.test_partition_of_unity("diag")


def test_dropped_coarse_correction_is_caught(monkeypatch):
    monkeypatch.setattr(bddc.BDDC, "coarse_solve", lambda self, rC: np.zeros_like(rC))
    with pytest.raises(AssertionError):
        tb.test_all_corners_gives_exact_inverse()


def test_transposed_coarse_basis_is_caught(monkeypatch):
    orig_init = bddc._LocalSaddle.__init__

    def bad_init(self, *a, **k):
        orig_init(self, *a, **k)
        self.Phi = self.Phi[::-1, :].copy()   # wrong row order of Phi_i
    monkeypatch.setattr(bddc._LocalSaddle, "__init__", bad_init)
    with pytest.raises(AssertionError):
        tb.test_coarse_basis_satisfies_constraints()


def test_dropped_interior_correction_is_caught(monkeypatch):
    from oracle.substructure import Substructuring
    # S_i = K_BB without the - K_BI K_II^{-1} K_IB term
    monkeypatch.setattr(Substructuring, "apply_S_local", lambda self, i, xb: self.sub[i]["KBB"] @ xb)
    with pytest.raises(AssertionError):
        tb.test_schur_equals_global_elimination()


def test_unweighted_pair_average_is_caught(monkeypatch):
    # E_st with plain (1/2, 1/2) averaging instead of the D weights
    orig = adaptive.averaging_matrix
    monkeypatch.setattr(adaptive, "averaging_matrix",
                        lambda ss, D, s, t: orig(ss, [np.ones_like(d) for d in D], s, t))
    with pytest.raises(AssertionError):
        ta.test_two_subdomain_face_eigenvalue_is_the_condition_number()


def test_missing_projection_is_caught(monkeypatch):
    # Pi left out of the pencil (shared coarse DOFs not enforced)
    monkeypatch.setattr(adaptive, "shared_constraints",
                        lambda ss, dofs, s, t: np.zeros((0, ss.sub[s]["nodes_B"].size + ss.sub[t]["nodes_B"].size)))
    with pytest.raises(AssertionError):
        ta.test_two_subdomain_face_eigenvalue_is_the_condition_number()


def test_wrong_side_of_the_pencil_is_caught(monkeypatch):
    # E in place of I - E on the left-hand side of eq. eig-matrix
    orig = adaptive.averaging_matrix
    monkeypatch.setattr(adaptive, "averaging_matrix",
                        lambda ss, D, s, t: np.eye(orig(ss, D, s, t).shape[0]) - orig(ss, D, s, t))
    with pytest.raises(AssertionError):
        ta.test_two_subdomain_face_bound(2.0)


# ------------------------------------------------ recycling (Section 4.2)

def test_b3_b4_swap_is_caught(monkeypatch):
    from oracle import recycle
    from tests import test_oracle_recycle_pins as tr
    orig = recycle.select
    monkeypatch.setattr(recycle, "select",
                        lambda theta, R, strategy: orig(theta, R, "B3" if strategy == "B4" else "B4"))
    with pytest.raises(AssertionError):
        tr.test_selection_on_invariant_subspace("B4")


def _freeze_pins(tr):
    tr.test_freeze_threshold_uniform_scaling(1.000005e-5, True)
    tr.test_freeze_threshold_uniform_scaling(1.00002e-5, False)
    tr.test_freeze_threshold_uses_two_norms(1.2e-5, True)
    tr.test_freeze_threshold_uses_two_norms(2.0e-5, False)


@pytest.mark.parametrize("mistake", ["old_denominator", "max_norm", "one_norm", "unsorted"])
def test_freeze_criterion_mistakes_are_caught(monkeypatch, mistake):
    from oracle import recycle
    from tests import test_oracle_recycle_pins as tr
    if mistake == "old_denominator":
        bad = lambda a, b: np.linalg.norm(a - b) / np.linalg.norm(b)
    elif mistake == "max_norm":
        bad = lambda a, b: np.abs(a - b).max() / np.abs(a).max()
    elif mistake == "one_norm":
        bad = lambda a, b: np.abs(a - b).sum() / np.abs(a).sum()
    else:   # new values compared in the opposite order to the stored ones
        bad = lambda a, b: np.linalg.norm(a[::-1] - b) / np.linalg.norm(a)
    monkeypatch.setattr(recycle, "ritz_change", bad)
    with pytest.raises(AssertionError):
        _freeze_pins(tr)


def test_level2_schur_without_interior_elimination_is_caught(monkeypatch):
    from tests import test_oracle_adaptive2 as t2
    monkeypatch.setattr(bddc, "level2_schur", lambda K, B, I: K[np.ix_(B, B)])
    with pytest.raises(AssertionError):
        t2.test_face_eigenvalue_is_the_coarse_condition_number()


def test_level2_rows_restricted_to_the_wrong_side_are_caught(monkeypatch):
    # c restricted to the t-copies (c_t = -c_s) flips each row's sign only,
    # which the span ignores; restricting to a shifted set of positions does not
    from tests import test_oracle_adaptive2 as t2
    orig = adaptive.adaptive_dofs

    def bad(*a, **k):
        new, info = orig(*a, **k)
        for d in new:
            d["wts"] = np.roll(d["wts"], 1)
        return new, info
    monkeypatch.setattr(adaptive, "adaptive_dofs", bad)
    with pytest.raises(AssertionError):
        t2.test_face_eigenvalue_is_the_coarse_condition_number()


def test_block_beta_with_wrong_sign_is_caught(monkeypatch):
    from oracle import block
    from tests import test_oracle_block as tbk
    orig = block.orth
    src = block.block_dpcg

    def bad_block(apply_A, apply_M, B, W=None, rtol=1e-8, max_it=1000):
        n, s = B.shape
        X = np.zeros((n, s)); R = B.copy(); P = np.zeros((n, 0)); Q = np.zeros((n, 0))
        bn = np.linalg.norm(B, axis=0); it = 0; ranks = []
        if W is not None and W.shape[1]:
            return src(apply_A, apply_M, B, W, rtol, max_it)
        while it < max_it and not np.all(np.linalg.norm(R, axis=0) <= rtol * bn):
            Z = apply_M(R)
            if P.shape[1]:
                Z = Z + P @ np.linalg.solve(P.T @ Q, Q.T @ Z)     # planted: + instead of -
            P = orig(Z); ranks.append(P.shape[1])
            Q = apply_A(P)
            alpha = np.linalg.solve(P.T @ Q, P.T @ R)
            X = X + P @ alpha; R = R - Q @ alpha; it += 1
        return dict(x=X, iters=it, relres=None, ranks=ranks)
    monkeypatch.setattr(block, "block_dpcg", bad_block)
    with pytest.raises(AssertionError):
        tbk.test_one_column_is_algorithm_1()
