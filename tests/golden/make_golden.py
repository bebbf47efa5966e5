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


if __name__ == "__main__":
    which = sys.argv[1:] or ["c16", "c64"]
    if "c16" in which:
        run("c16", 10, (1e-8, 1e-10))
    if "c64" in which:
        run("c64", 5, (1e-10, 1e-8))
