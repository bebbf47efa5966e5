"""Write the stored expected values under tests/golden/ from the CPU oracle only.

    python tests/golden/make_golden.py [c16] [c64]

The paper prints no worked example, so every stored value here is either a
closed-form count (stated with its derivation in the JSON) or an oracle
result written by this script.  It imports only ``oracle`` and ``workload``.
"""
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import workload  # noqa: E402
from oracle.sequence import OracleSolver  # noqa: E402

N_SAMPLE = 256


def sample_nodes(nx, n=N_SAMPLE):
    return np.sort(workload.rng("misc", 7).choice(workload.n_nodes(nx), n, replace=False))


def run(name, n_rhs, rtols):
    s = workload.workload(name)
    out = dict(name=name, nx=s["nx"], n_rhs=n_rhs, R=s["R"], strategy="B4",
               levels=3 if s["n_subregion"] else 2, weights="diag", constraints="corners+faces",
               stop="||r||/||b||", init_guess="previous solution")
    F = workload.rhs_sequence(s["nx"], n_rhs)
    idx = sample_nodes(s["nx"])
    out["sample_nodes"] = idx.tolist()
    for rtol in rtols:
        t = time.time()
        o = OracleSolver(s["nx"], s["elem_to_sub"], s["coef"], sub_to_subregion=s["sub_to_subregion"], R=s["R"])
        if "n_gamma" not in out:
            out["n_gamma"] = int(o.ss.n_gamma)
            out.update(o.M.counts())
            if o.M.three_level:
                L2 = o.M.level2
                out["level2_interface"] = int(L2.gamma2.size)
                out["level2_interior"] = int(o.M.nC - L2.gamma2.size)
                out["level3"] = int(L2.n3)
        rec = dict(iters=[], true_relres=[], u_norm2=[], u_sample=[], theta=[])
        for k in range(n_rhs):
            r = o.solve(F[k], rtol)
            rec["iters"].append(int(r["iters"]))
            rec["true_relres"].append(float(r["true_relres"]))
            rec["u_norm2"].append(float(np.linalg.norm(r["u"])))
            rec["u_sample"].append(r["u"][idx].tolist())
            rec["theta"].append(None if o.rec.theta is None else o.rec.theta.tolist())
        rec["seconds"] = time.time() - t
        out["rtol_%g" % rtol] = rec
        print(name, rtol, rec["iters"], "%.1fs" % rec["seconds"], flush=True)
    with open(os.path.join(HERE, "%s_oracle.json" % name), "w") as f:
        json.dump(out, f, indent=1)


def run_full(name, n_rhs, rtol, tag):
    """Every nodal value of the first n_rhs solutions (compressed .npz), with
    iterations, true residuals and the recycling history."""
    from oracle.recycle import ritz_change
    s = workload.workload(name)
    F = workload.rhs_sequence(s["nx"], n_rhs, s["elem_keep"])
    t = time.time()
    o = OracleSolver(s["nx"], s["elem_to_sub"], s["coef"], elem_keep=s["elem_keep"],
                     sub_to_subregion=s["sub_to_subregion"], R=s["R"])
    U, its, rr = [], [], []
    for k in range(n_rhs):
        r = o.solve(F[k], rtol)
        U.append(r["u"])
        its.append(r["iters"])
        rr.append(r["true_relres"])
        print(name, k, r["iters"], "%.1fs" % (time.time() - t), flush=True)
    hist = o.rec.history
    change = [ritz_change(hist[j], hist[j - 1]) if hist[j].size == hist[j - 1].size == s["R"] else -1.0
              for j in range(1, len(hist))]
    np.savez_compressed(os.path.join(HERE, "%s_%s.npz" % (name, tag)), u=np.array(U), iters=np.array(its),
                        true_relres=np.array(rr), rtol=rtol, R=s["R"],
                        freeze_step=-1 if o.rec.freeze_step is None else o.rec.freeze_step,
                        ritz_change=np.array(change), n_gamma=o.ss.n_gamma, seconds=time.time() - t)


def run_sequence(name, n_rhs, rtol, tag):
    """The whole sequence: iterations, freeze step, relative change of the
    selected harmonic Ritz values at every update, norms and 256 sampled
    nodal values of every solution."""
    from oracle.recycle import ritz_change
    s = workload.workload(name)
    F = workload.rhs_sequence(s["nx"], n_rhs, s["elem_keep"])
    idx = sample_nodes(s["nx"])
    t = time.time()
    o = OracleSolver(s["nx"], s["elem_to_sub"], s["coef"], elem_keep=s["elem_keep"],
                     sub_to_subregion=s["sub_to_subregion"], R=s["R"])
    its, rr, un, us = [], [], [], []
    for k in range(n_rhs):
        r = o.solve(F[k], rtol)
        its.append(r["iters"])
        rr.append(r["true_relres"])
        un.append(np.linalg.norm(r["u"]))
        us.append(r["u"][idx])
        print(name, k, r["iters"], o.rec.frozen, "%.1fs" % (time.time() - t), flush=True)
    hist = o.rec.history
    change = [ritz_change(hist[j], hist[j - 1]) if hist[j].size == hist[j - 1].size == s["R"] else -1.0
              for j in range(1, len(hist))]
    theta = np.full((len(hist), s["R"]), np.nan)     # selected values of every update (NaN: fewer)
    for j, h in enumerate(hist):
        theta[j, :h.size] = h
    np.savez_compressed(os.path.join(HERE, "%s_%s.npz" % (name, tag)), iters=np.array(its), theta=theta,
                        true_relres=np.array(rr), u_norm2=np.array(un), u_sample=np.array(us), sample_nodes=idx,
                        rtol=rtol, R=s["R"], freeze_step=-1 if o.rec.freeze_step is None else o.rec.freeze_step,
                        ritz_change=np.array(change), seconds=time.time() - t)


if __name__ == "__main__":
    which = sys.argv[1:] or ["c16", "c64"]
    if "c16" in which:
        run("c16", 10, (1e-8, 1e-10))
    if "c64" in which:
        run("c64", 5, (1e-10, 1e-8))
    if "c64full" in which:          # every node, 5 right-hand sides, float64 parity tolerance
        run_full("c64", 5, 1e-10, "full5")
    if "c64seq" in which:           # the 50-step sequence of the benchmark, to its freeze
        run_sequence("c64", 50, 1e-8, "seq50")
    if "c3full" in which:           # holed cube, 400 uneven subdomains
        run_full("c3", 5, 1e-10, "full5")
    if "c96full" in which:          # 96^3 prefix of the differentiation workload
        run_full("c96", 2, 1e-10, "full2")
