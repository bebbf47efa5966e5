#!/usr/bin/env python
"""Throughput of the deflated-PCG / three-level BDDC sequence solve on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W]

Workload (synthetic, seeded): Q1 Poisson on the unit cube, 64^3 elements
(274,625 nodes), Dirichlet u = 0 on x = 1, unit coefficient, 8^3 = 512 cube
subdomains of 8^3 elements, three-level BDDC (subregions of 2x2x2
subdomains, corners + face averages, diag weights), deflated PCG with a
20-vector basis recycled by B4 harmonic Ritz vectors, previous-solution
initial guess, ||r||/||b|| < 1e-8, a 50-step drifting-Gaussian right-hand-side
sequence.  One step = one 50-RHS sequence from an empty basis (setup
excluded); value = right-hand sides solved per second in float64.  The same
line reports the mixed form (float32 local Neumann operators) on the same
sequence, the roofline of the dominant kernel and the oracle on the host CPU.
"""
import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0   # MI355X HBM3E
WORKLOADS = {
    "c64": "Q1 Poisson 64^3 elements (274,625 nodes), 512 subdomains of 8^3, three-level BDDC (64 subregions), "
           "deflated PCG B4 R=20, 50 drifting-Gaussian right-hand sides, rtol 1e-8",
    "c3": "Q1 Poisson 64^3 elements minus a sphere of radius 0.15, 400 jittered-RCB subdomains of uneven size, "
          "log-normal coefficients (sigma 0.5), three-level BDDC (50 subregions), deflated PCG B4 R=20, "
          "50 drifting-Gaussian right-hand sides, rtol 1e-8",
    "c96": "Q1 Poisson 96^3 elements (912,673 nodes), 1,728 subdomains of 8^3, three-level BDDC (216 subregions), "
           "deflated PCG B4 R=20, 20 drifting-Gaussian right-hand sides, rtol 1e-8 (adjoint: 20 more solves)",
}


def kernel_hash():
    """Hash of the sources of the product kernel (traffic figures are only
    used while it is unchanged)."""
    h = hashlib.sha256()
    for f in ("hot.hip", "devutil.h", "kernels.h", "internal.h"):
        h.update(open(os.path.join(ROOT, "paper_2412_17543_amd", "csrc", f), "rb").read())
    return h.hexdigest()[:16]


def its_fmt(its):
    return "%d-%d(%.1f)" % (min(its), max(its), sum(its) / len(its))


def pin_of(tuning):
    """The 8-entry product configuration of a tuning report."""
    out = []
    for k in ("schur", "neumann"):
        t = tuning[k]
        out += [int(t["blocks_per_cu"]), int(t["per_subdomain"]), int(t["waves"]), int(t["unroll"])]
    return out


def run_form(torch, Solver, s, F, rtol, steps, warmup, local_prec, timing, use_graph=True, pin=None, autotune=True):
    t0 = time.perf_counter()
    g = Solver(s["nx"], s["elem_to_sub"], s["coef"], sub_to_subregion=s["sub_to_subregion"],
               elem_keep=s["elem_keep"], R=s["R"], local_prec=local_prec, use_graph=use_graph, product_cfg=pin,
               autotune=autotune)
    torch.cuda.synchronize()
    setup_s = time.perf_counter() - t0
    for _ in range(warmup):
        g.reset_recycle()
        g.solve_sequence(F, rtol)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        g.reset_recycle()
        U, its, rr = g.solve_sequence(F, rtol)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    st = None
    if timing:
        # one more sequence, launched kernel by kernel with HIP events around
        # every operator product (queued launches cannot be bracketed per kernel)
        g.enable_timing(True, ("schur", "precond_local"))
        g.reset_recycle()
        g.solve_sequence(F, rtol)
        torch.cuda.synchronize()
        st = g.stats()
        g.enable_timing(False)
    info = g.info()
    prod = g.time_products(20) if timing else None
    return dict(g=g, U=U, its=its, rr=rr, elapsed=el, setup_s=setup_s, stats=st, info=info, tuning=g.tuning(),
                products=prod)


def cpu_baseline(s, F_np, n_sample):
    from threadpoolctl import threadpool_limits

    from oracle.sequence import OracleSolver
    with threadpool_limits(1):
        o = OracleSolver(s["nx"], s["elem_to_sub"], s["coef"], elem_keep=s["elem_keep"],
                         sub_to_subregion=s["sub_to_subregion"], R=s["R"])
        t0 = time.perf_counter()
        for k in range(n_sample):
            o.solve(F_np[k], 1e-8)
        el = time.perf_counter() - t0
    return dict(value=n_sample / el, unit="solves/s", cores=1, kind="oracle",
                sample="first %d right-hand sides of the same sequence (oracle setup excluded, "
                       "as on the GPU), float64 NumPy/SciPy, one thread" % n_sample)


def _rhs_chunk(job):
    import workload
    nx, first, n = job
    return workload.rhs_sequence(nx, n, None, first=first)


def run_large(args):
    """192^3 (13,824 subdomains): the float32-Neumann form with adaptive faces
    and R = 40, on the leading right-hand sides of the sequence."""
    from concurrent.futures import ProcessPoolExecutor

    import workload
    s = workload.workload("c192")
    n_rhs = args.n_rhs or s["n_rhs"]
    t0 = time.perf_counter()
    chunk = max(1, (n_rhs + 15) // 16)
    jobs = [(s["nx"], k, min(chunk, n_rhs - k)) for k in range(0, n_rhs, chunk)]
    # worker processes (CPU only) are started before this process touches the GPU
    with ProcessPoolExecutor(max_workers=min(16, len(jobs))) as ex:
        parts = list(ex.map(_rhs_chunk, jobs))
    import torch

    from paper_2412_17543_amd.solver import Solver
    F = torch.cat([torch.tensor(a, device="cuda") for a in parts])
    del parts
    torch.cuda.synchronize()
    gen_s = time.perf_counter() - t0
    print("[bench] c192: %d right-hand sides generated in %.1f s" % (n_rhs, gen_s), file=sys.stderr, flush=True)
    t0 = time.perf_counter()
    g = Solver(s["nx"], s["elem_to_sub"], s["coef"], sub_to_subregion=s["sub_to_subregion"], R=s["R"],
               local_prec=32, adapt_tau=10.0, adapt_max_per_face=10)
    torch.cuda.synchronize()
    setup_s = time.perf_counter() - t0
    print("[bench] c192: setup %.1f s" % setup_s, file=sys.stderr, flush=True)
    for _ in range(args.warmup):
        g.reset_recycle()
        g.solve_sequence(F, args.rtol)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        g.reset_recycle()
        U, its, rr = g.solve_sequence(F, args.rtol)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    info = g.info()
    line = {
        "metric": "solves/s to FP64 rtol 1e-8, BDDC-DPCG with adaptive faces, 1 GPU",
        "value": round(n_rhs * args.steps / el, 3),
        "unit": "solves/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": round(1e3 * el / args.steps, 3),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64 (float32 Neumann operators)", "data": "synthetic",
        "config": {"workload": "Q1 Poisson 192^3 elements (7,189,057 nodes), 13,824 subdomains of 8^3, three-level "
                               "BDDC (1,728 subregions), adaptive faces tau 10 (at most 10 per face), float32 N_i "
                               "and Phi_i, deflated PCG B4 R=40, drifting-Gaussian right-hand sides, rtol 1e-8",
                   "n_rhs": n_rhs, "n_gamma": info["n_gamma"], "rtol": args.rtol},
        "iters": its_fmt(its.tolist()),
        "max_true_relres": float(rr.max()),
        "s_per_sequence": round(el / args.steps, 4),
        "setup_s": round(setup_s, 2),
        "adaptive": g.adaptive_stats(),
        "coarse": {k: info[k] for k in ("n_coarse", "corners", "faces", "level2_interface", "level3")},
        "device_gb": round(info["device_bytes"] / 1e9, 2),
        "rhs_generation_s": round(gen_s, 1),
        "tuning": g.tuning(),
    }
    print(json.dumps(line), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--rtol", type=float, default=1e-8)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-mixed", action="store_true")
    ap.add_argument("--no-plain", action="store_true", help="skip the plain (kernel-by-kernel) FP64 form")
    ap.add_argument("--cpu-sample", type=int, default=2)
    ap.add_argument("--workload", default="c64", choices=("c64", "c3", "c96", "c192"),
                    help="c64: 64^3 cube lattice (the headline configuration); c3: 64^3 with a spherical "
                         "hole, 400 uneven RCB subdomains, log-normal coefficients; c192: 192^3, 13,824 "
                         "subdomains, adaptive faces (tau 10), float32 Neumann operators, R = 40 (its own "
                         "line: the float32 form only)")
    ap.add_argument("--n-rhs", type=int, default=0, help="use the first N right-hand sides of the sequence")
    ap.add_argument("--no-bf16", action="store_true", help="skip the bfloat16 Neumann-operator form")
    ap.add_argument("--adjoint", action="store_true",
                    help="also time the adjoint gradient of L = sum_k ||u_k - t_k||^2 (t_k = 0.9 u_k): one adjoint "
                         "solve per right-hand side with the recycled basis, and the element gradient")
    ap.add_argument("--pin", default=None,
                    help="fixed product configuration of the float64 form: 8 comma-separated integers "
                         "(Schur then Neumann: blocks per CU, per-subdomain split, waves, tiles in flight)")
    ap.add_argument("--roofline-only", action="store_true",
                    help="set up, run one sequence, then only the timed product launches and a 256 MiB device copy "
                         "(for hardware-counter passes: the copy calibrates FETCH_SIZE/WRITE_SIZE)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures the single-GPU path only (one process, one MI355X); "
              "--gpus %d is not supported" % args.gpus, file=sys.stderr)
        sys.exit(2)

    if args.workload == "c192":
        return run_large(args)

    import numpy as np
    import torch

    import workload
    from paper_2412_17543_amd.solver import Solver

    s = workload.workload(args.workload)
    F_np = workload.rhs_sequence(s["nx"], s["n_rhs"], s["elem_keep"])
    F = torch.tensor(F_np, device="cuda")       # inputs resident in HBM before timing
    torch.cuda.synchronize()
    n_rhs = F.shape[0]
    # product configuration: --pin, else the one the counter passes measured
    # (profiles/traffic_<workload>.json, while the kernel sources are
    # unchanged), else the autotuner's choice
    traffic_file = os.path.join(ROOT, "profiles", "traffic_%s.json" % args.workload)
    traffic_rec = None
    if os.path.exists(traffic_file):
        t = json.load(open(traffic_file))
        if t.get("kernel_hash") == kernel_hash():
            traffic_rec = t
    pin_source = "autotuned"
    if args.pin:
        pin, pin_source = [int(v) for v in args.pin.split(",")], "command line"
    elif traffic_rec is not None and not args.roofline_only:
        pin, pin_source = [int(v) for v in traffic_rec["pin"].split(",")], "profiles/traffic_%s.json" % args.workload
    else:
        pin = None
    if args.roofline_only:
        g = Solver(s["nx"], s["elem_to_sub"], s["coef"], sub_to_subregion=s["sub_to_subregion"],
                   elem_keep=s["elem_keep"], R=s["R"], product_cfg=pin)
        pr = g.time_products(20)
        src = torch.ones(32 << 20, dtype=torch.float64, device="cuda")     # 256 MiB
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"products": pr, "copy_bytes_each_way": src.numel() * 8, "kernel_hash": kernel_hash(),
                          "tuning": g.tuning()}), flush=True)
        return

    f64 = run_form(torch, Solver, s, F, args.rtol, args.steps, args.warmup, 64, True, pin=pin)
    value = n_rhs * args.steps / f64["elapsed"]
    st = f64["stats"]
    pr = f64["products"]
    # dominant kernel: the batched product with the longer launch, timed by
    # back-to-back launches right after the timed region
    dom = max(("schur", "neumann"), key=lambda k: pr[k]["us"])
    avg_us = pr[dom]["us"]
    achieved = pr[dom]["bytes"] / (avg_us * 1e-6) / 1e9
    traffic = None
    if traffic_rec is not None and traffic_rec["pin"] == ",".join(str(v) for v in pin_of(f64["tuning"])):
        traffic = traffic_rec["kernels"][dom]["bytes_per_launch"]
    line = {
        "metric": "solves/s to FP64 rtol 1e-8 + HBM GB/s, mixed vs FP64 BDDC-DPCG, 1 GPU",
        "value": round(value, 3),
        "unit": "solves/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(1e3 * f64["elapsed"] / args.steps, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": WORKLOADS[args.workload],
                   "n_rhs": n_rhs, "n_gamma": f64["info"]["n_gamma"], "rtol": args.rtol},
        "iters": its_fmt(f64["its"].tolist()),
        "basis": {"columns": int(f64["info"]["deflation_cols"]), "frozen": bool(f64["info"]["frozen"])},
        "max_true_relres": float(f64["rr"].max()),
        "s_per_sequence": round(f64["elapsed"] / args.steps, 4),
        "setup_s": round(f64["setup_s"], 3),
        "roofline": {"bound": "hbm", "kernel": "k_symv<double> (" + ("Schur S_i" if dom == "schur" else "Neumann N_i") + ")",
                     "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic,
                     "avg_launch_us": round(avg_us, 2), "algorithmic_bytes_per_launch": pr[dom]["bytes"],
                     "other_product": {k: {"avg_launch_us": round(v["us"], 2),
                                           "GB/s": round(v["bytes"] / (v["us"] * 1e-6) / 1e9, 1)}
                                       for k, v in pr.items() if k != dom}},
        "kernel_ms_per_sequence_eager": {k: round(v["ms"], 3) for k, v in st.items() if v["count"]},
        "tuning": f64["tuning"],
        "pin": ",".join(str(v) for v in pin_of(f64["tuning"])),
        "pin_source": pin_source,
    }
    plain_value = None
    if not args.no_plain:
        # the plain FP64 GPU form: kernels launched one by one with a host check
        # after every iteration, default product configuration (no autotuning)
        pl = run_form(torch, Solver, s, F, args.rtol, args.steps, args.warmup, 64, False, use_graph=False,
                      autotune=False)
        plain_value = n_rhs * args.steps / pl["elapsed"]
        line["fp64_plain"] = {"value": round(plain_value, 3), "unit": "solves/s", "iters": its_fmt(pl["its"].tolist()),
                              "max_true_relres": float(pl["rr"].max())}
    if not args.no_mixed:
        mx = run_form(torch, Solver, s, F, args.rtol, args.steps, args.warmup, 32, False)
        ud = f64["U"]
        err = max(float(((mx["U"][k] - ud[k]).abs().max() / ud[k].abs().max()).item()) for k in range(n_rhs))
        mv = n_rhs * args.steps / mx["elapsed"]
        line["mixed_fp32"] = {"value": round(mv, 3), "unit": "solves/s", "iters": its_fmt(mx["its"].tolist()),
                              "max_true_relres": float(mx["rr"].max()), "max_rel_diff_vs_fp64": err,
                              "speedup_vs_fp64": round(mv / value, 3)}
        if plain_value:
            line["mixed_fp32"]["speedup_vs_plain_fp64"] = round(mv / plain_value, 3)
    if not args.no_bf16 and not args.no_mixed:
        bf = run_form(torch, Solver, s, F, args.rtol, args.steps, args.warmup, 16, False)
        ud = f64["U"]
        err = max(float(((bf["U"][k] - ud[k]).abs().max() / ud[k].abs().max()).item()) for k in range(n_rhs))
        bv = n_rhs * args.steps / bf["elapsed"]
        line["mixed_bf16"] = {"value": round(bv, 3), "unit": "solves/s", "iters": its_fmt(bf["its"].tolist()),
                              "max_true_relres": float(bf["rr"].max()), "max_rel_diff_vs_fp64": err,
                              "speedup_vs_fp64": round(bv / value, 3)}
        if plain_value:
            line["mixed_bf16"]["speedup_vs_plain_fp64"] = round(bv / plain_value, 3)
    if args.adjoint:
        g = f64["g"]
        U = f64["U"]
        dLdu = 2.0 * (U - 0.9 * U)
        g.adjoint_grad(dLdu, U, args.rtol)          # warm-up
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            grad, gF = g.adjoint_grad(dLdu, U, args.rtol)
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
        line["adjoint"] = {"value": round(n_rhs * args.steps / el, 3), "unit": "adjoint solves/s",
                           "s_per_sequence": round(el / args.steps, 4),
                           "grad_norm": float(grad.norm().item())}
    if not args.no_cpu_baseline:
        line["cpu_baseline"] = cpu_baseline(s, F_np, args.cpu_sample)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
