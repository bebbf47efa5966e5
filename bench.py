#!/usr/bin/env python
"""Throughput of the deflated-PCG / three-level BDDC sequence solve on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload c192|c64|c3|c96]

Default workload (synthetic, seeded): Q1 Poisson on the unit cube, 192^3
elements (7,189,057 nodes), Dirichlet u = 0 on x = 1, unit coefficient,
24^3 = 13,824 cube subdomains of 8^3 elements, three-level BDDC (1,728
subregions of 2x2x2 subdomains), adaptive face constraints (tau = 10, at most
10 per face), deflated PCG with a 40-vector basis recycled by B4 harmonic
Ritz vectors, previous-solution initial guess, ||r||/||b|| < 1e-8, a
200-step drifting-Gaussian right-hand-side sequence.

One step = 10 consecutive right-hand sides of that sequence, solved with the
recycling state carried from step to step, so 20 steps are the whole
200-step sequence from an empty basis (warm-up steps run the sequence's first
right-hand sides, then the basis is reset).  Setup is excluded; inputs are in
HBM before timing.  `value` = right-hand sides solved per second in the
configuration's own form: float32 local Neumann operators (N_i, Phi_i),
everything else float64.  The same line reports the float64 form, the
bfloat16 form and the plain float64 form (kernel by kernel, host check after
every iteration, untuned products) on the same operators and sequence, the
roofline of the dominant kernel and of the preconditioner application, and
the oracle on the host CPU.

Other workloads (their own lines): c64 (64^3, 512 subdomains, R = 20, 50 RHS,
float64), c3 (64^3 with a spherical hole, 400 uneven subdomains, log-normal
coefficients, float32 Neumann operators), c96 (96^3, 1,728 subdomains, 20 RHS,
float64; --adjoint times the adjoint gradient too).  For these a step is the
whole sequence.
"""
import argparse
import hashlib
import json
import os
import subprocess
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0   # MI355X HBM3E
METRIC = "solves/s to FP64 rtol 1e-8 + HBM GB/s, mixed vs FP64 BDDC-DPCG, 1 GPU"
WORKLOADS = {
    "c192": dict(desc="Q1 Poisson 192^3 elements (7,189,057 nodes), 13,824 subdomains of 8^3, three-level BDDC "
                      "(1,728 subregions), adaptive faces tau 10 (at most 10 per face), deflated PCG B4 R=40, "
                      "200 drifting-Gaussian right-hand sides, rtol 1e-8",
                 prec=32, step_rhs=10, adapt=True, launch="graph"),
    "c64": dict(desc="Q1 Poisson 64^3 elements (274,625 nodes), 512 subdomains of 8^3, three-level BDDC "
                     "(64 subregions), deflated PCG B4 R=20, 50 drifting-Gaussian right-hand sides, rtol 1e-8",
                prec=64, step_rhs=0, adapt=False),
    "c3": dict(desc="Q1 Poisson 64^3 elements minus a sphere of radius 0.15, 400 jittered-RCB subdomains of uneven "
                    "size, log-normal coefficients (sigma 0.5), three-level BDDC (50 subregions), deflated PCG B4 "
                    "R=20, 50 drifting-Gaussian right-hand sides, rtol 1e-8",
               prec=32, step_rhs=0, adapt=False),
    "c96": dict(desc="Q1 Poisson 96^3 elements (912,673 nodes), 1,728 subdomains of 8^3, three-level BDDC "
                     "(216 subregions), deflated PCG B4 R=20, 20 drifting-Gaussian right-hand sides, rtol 1e-8",
                prec=64, step_rhs=0, adapt=False),
}
PREC_NAME = {64: "f64", 32: "f32", 16: "bf16"}
# the oracle sample standing in for the 192^3 problem: a 32^3 block of the
# same 8^3 subdomains (64 of them, 8 subregions), same options
CPU_SAMPLE_NX = 32


def kernel_hash():
    """Hash of the product kernel's source (hot.hip up to the end of k_symv,
    devutil.h, internal.h): traffic figures are only used while it is
    unchanged."""
    h = hashlib.sha256()
    hot = open(os.path.join(ROOT, "paper_2412_17543_amd", "csrc", "hot.hip"), "rb").read()
    h.update(hot[: hot.index(b"// Operands of nodes gb")])
    for f in ("devutil.h", "internal.h"):
        h.update(open(os.path.join(ROOT, "paper_2412_17543_amd", "csrc", f), "rb").read())
    return h.hexdigest()[:16]


def its_fmt(its):
    return "%d-%d(%.1f)" % (min(its), max(its), sum(its) / len(its))


def gbs(k):
    return k["bytes"] / (k["us"] * 1e-6) / 1e9


def _rhs_chunk(job):
    import workload
    nx, first, n, keep = job
    return workload.rhs_sequence(nx, n, keep, first=first)


def make_rhs(s, n_rhs):
    """The sequence's load vectors on the host (worker processes for large
    meshes; they are started before this process touches the GPU)."""
    import numpy as np

    import workload
    if s["nx"] < 128:
        return workload.rhs_sequence(s["nx"], n_rhs, s["elem_keep"])
    from concurrent.futures import ProcessPoolExecutor
    workers = max(1, min(16, len(os.sched_getaffinity(0)), n_rhs))
    out = np.empty((n_rhs, workload.n_nodes(s["nx"])))
    jobs = [(s["nx"], k, 1, s["elem_keep"]) for k in range(n_rhs)]
    with ProcessPoolExecutor(max_workers=workers) as ex:
        for k, f in enumerate(ex.map(_rhs_chunk, jobs, chunksize=1)):
            out[k] = f[0]
    return out


def cpu_baseline(name, s, n_gpu_subs, budget_s=20.0):
    """The oracle as it stands (float64 NumPy/SciPy, BLAS threads on every
    core this process may use), setup excluded, timed on a bounded sample."""
    import numpy as np
    from threadpoolctl import threadpool_info

    import workload
    from oracle.sequence import OracleSolver
    cores = len(os.sched_getaffinity(0))
    try:
        model = [l.split(":", 1)[1].strip() for l in subprocess.run(["lscpu"], capture_output=True, text=True)
                 .stdout.splitlines() if l.startswith("Model name")][0]
    except Exception:
        model = "unknown"
    if name == "c192":
        # the oracle's setup of the whole 192^3 problem (13,824 sparse local
        # solvers built in Python loops) does not finish in bounded time: the
        # sample is a 32^3 block of the same subdomains, levels and options
        nx = CPU_SAMPLE_NX
        m = nx // 8
        o = OracleSolver(nx, workload.cube_partition(nx, 8), np.ones(nx ** 3),
                         sub_to_subregion=workload.cube_subregions(m, 2), R=s["R"])
        F = workload.rhs_sequence(nx, 40)
        n_sub = m ** 3
    else:
        o = OracleSolver(s["nx"], s["elem_to_sub"], s["coef"], elem_keep=s["elem_keep"],
                         sub_to_subregion=s["sub_to_subregion"], R=s["R"])
        F = workload.rhs_sequence(s["nx"], min(s["n_rhs"], 40), s["elem_keep"])
        n_sub = n_gpu_subs
    its = []
    t0 = time.perf_counter()
    for k in range(F.shape[0]):
        its.append(o.solve(F[k], 1e-8)["iters"])
        if time.perf_counter() - t0 > budget_s:
            break
    el = time.perf_counter() - t0
    n = len(its)
    scale = n_sub / n_gpu_subs
    threads = max([t.get("num_threads", 1) for t in threadpool_info()] + [1])
    if name == "c192":
        sample = ("oracle (setup excluded) on the first %d right-hand sides of the same generator on a 32^3-element "
                  "block: 64 subdomains of 8^3, 8 subregions, R = %d, rtol 1e-8, iterations %s; %.2f solves/s "
                  "there, scaled by 64/13,824 subdomains (the oracle's work per iteration is a loop over subdomains). "
                  "Adaptive selection is left out of the sample: at tau = 10 it adds no constraint on this "
                  "unit-coefficient workload (largest face eigenvalue below 2)" % (n, s["R"], its_fmt(its), n / el))
    else:
        sample = ("oracle (setup excluded) on the first %d right-hand sides of the same sequence, rtol 1e-8, "
                  "iterations %s" % (n, its_fmt(its)))
    return dict(value=n / el * scale, unit="solves/s", cores=cores, kind="oracle", sample=sample,
                seconds=round(el, 2), cpu_model=model, blas_threads=threads)


def roofline_of(k):
    """roofline entry of one timed kernel (bddc_time_kernels)."""
    a = gbs(k)
    return dict(achieved=round(a, 1), frac=round(a / HBM_PEAK_GBS, 4), avg_launch_us=round(k["us"], 2),
                algorithmic_bytes_per_launch=k["bytes"])


def run_form(torch, g, F, rtol, steps, warmup, step_rhs, keep_u):
    """Warm-up, reset, then `steps` timed steps; a step is `step_rhs`
    consecutive right-hand sides of the sequence (recycling state carried
    over; back at the start of the sequence with a reset)."""
    n_rhs = F.shape[0]
    spc = max(1, n_rhs // step_rhs)          # steps per sequence

    def step(i):
        j = i % spc
        if j == 0:
            g.reset_recycle()
        return g.solve_sequence(F[j * step_rhs:(j + 1) * step_rhs], rtol)

    for i in range(warmup):
        step(i)
    torch.cuda.synchronize()
    its, rrs, us = [], [], []
    t0 = time.perf_counter()
    for i in range(steps):
        U, it, rr = step(i)
        its += it.tolist()
        rrs += rr.tolist()
        if keep_u and i < spc:
            us.append(U)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    info = g.solve_info()
    out = dict(value=round(step_rhs * steps / el, 3), unit="solves/s", ms_per_step=round(1e3 * el / steps, 3),
               iters=its_fmt(its), max_true_relres=max(rrs),
               basis={"columns": info["deflation_cols"], "frozen": bool(info["frozen"]),
                      "freeze_step": info["freeze_step"]})
    return out, (torch.cat(us) if keep_u and us else None), its


def run_roofline_only(args, s, spec):
    """Set up, then only the timed kernel launches and a 256 MiB device copy
    (for hardware-counter passes: the copy calibrates FETCH_SIZE/WRITE_SIZE)."""
    import torch

    from paper_2412_17543_amd.solver import Solver
    g = Solver(s["nx"], s["elem_to_sub"], s["coef"], sub_to_subregion=s["sub_to_subregion"],
               elem_keep=s["elem_keep"], R=s["R"], local_prec=spec["prec"],
               adapt_tau=10.0 if spec["adapt"] else 0.0, adapt_max_per_face=10)
    if args.pin:
        g.set_launch(True, [int(v) for v in args.pin.split(",")])
    kt = g.time_kernels(20)
    src = torch.ones(32 << 20, dtype=torch.float64, device="cuda")     # 256 MiB
    dst = torch.empty_like(src)
    dst.copy_(src)
    torch.cuda.synchronize()
    print(json.dumps({"kernels": kt, "copy_bytes_each_way": src.numel() * 8, "kernel_hash": kernel_hash(),
                      "tuning": g.tuning()}), flush=True)


def run_study(args):
    """The paper's parameter studies on synthetic sequences, one JSON line:
    stopping rule x initial guess without recycling (Tab. no_recycling),
    the recycling strategies B1-B4 at R = 20 (Tab. recycling_cases), the
    basis size R for B4 (Tab. recycling_base), and the adaptive threshold tau
    with card/diag weights (Tab. recycling_case2), plus two rows with the
    level-2 faces enriched as well.  Each row: iterations as
    min-max(avg), seconds per right-hand side and per iteration (float64,
    queued launches), setup seconds; the coarse space for the tau study."""
    import numpy as np
    import torch

    import workload
    from paper_2412_17543_amd.solver import Solver
    name = args.workload if args.workload != "c192" else ("c3" if args.study == "tau" else "c64")
    s = workload.workload(name)
    F = torch.tensor(make_rhs(s, args.n_rhs or s["n_rhs"]), device="cuda")
    n_rhs = F.shape[0]
    if args.study == "stopping":
        cases = [dict(stop_rule=r, init_guess=gs, R=0) for r in ("r0", "rhs") for gs in ("zero", "prev")]
    elif args.study == "strategies":
        cases = [dict(R=0)] + [dict(R=20, strategy=b) for b in ("B1", "B2", "B3", "B4")]
    elif args.study == "rsweep":
        cases = [dict(R=r, strategy="B4") for r in (0, 5, 10, 20, 40, 60)]
    else:
        cases = [dict(R=20, adapt_tau=t, weights=w) for w in ("card", "diag") for t in (0.0, 10.0, 5.0, 3.0, 2.0)]
        cases += [dict(R=20, adapt_tau=3.0, weights="diag", adapt2_tau=t2) for t2 in (3.0, 2.0)]
    rows = []
    for kw in cases:
        t0 = time.perf_counter()
        g = Solver(s["nx"], s["elem_to_sub"], s["coef"], sub_to_subregion=s["sub_to_subregion"],
                   elem_keep=s["elem_keep"], **kw)
        torch.cuda.synchronize()
        setup = time.perf_counter() - t0
        g.solve_sequence(F, args.rtol)                   # warm-up
        g.reset_recycle()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        U, its, rr = g.solve_sequence(F, args.rtol)
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
        info = g.info()
        row = dict(kw, iters=its_fmt(its.tolist()), iters_first=int(its[0]), s_per_rhs=round(el / n_rhs, 5),
                   s_per_iteration=round(el / max(1, int(its.sum())), 6), setup_s=round(setup, 2),
                   max_true_relres=float(rr.max()), frozen=bool(info["frozen"]), n_coarse=info["n_coarse"])
        if kw.get("adapt_tau", 0) > 0:
            row["adaptive"] = g.adaptive_stats()
        if kw.get("adapt2_tau", 0) > 0:
            row["adaptive_level2"] = g.adaptive2_stats()
            row["n_level3"] = info["level3"]
        rows.append(row)
        print("[study] %s" % row, file=sys.stderr, flush=True)
        g.close()
    print(json.dumps({"study": args.study, "workload": WORKLOADS[name]["desc"], "n_rhs": n_rhs, "rtol": args.rtol,
                      "rows": rows}), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--rtol", type=float, default=1e-8)
    ap.add_argument("--workload", default="c192", choices=tuple(WORKLOADS))
    ap.add_argument("--n-rhs", type=int, default=0, help="use the first N right-hand sides of the sequence")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-mixed", action="store_true", help="only the float64 forms")
    ap.add_argument("--no-bf16", action="store_true", help="skip the bfloat16 Neumann-operator form")
    ap.add_argument("--no-plain", action="store_true", help="skip the plain (kernel-by-kernel) float64 form")
    ap.add_argument("--adjoint", action="store_true",
                    help="also time the adjoint gradient of L = sum_k ||u_k - t_k||^2 (t_k = 0.9 u_k)")
    ap.add_argument("--pin", default=None,
                    help="fixed product configuration: 8 comma-separated integers (Schur then Neumann: blocks per "
                         "CU, per-subdomain split, waves, tiles in flight); a 0 first entry keeps that product tuned")
    ap.add_argument("--roofline-only", action="store_true")
    ap.add_argument("--launch", default=None, choices=("queued", "graph"),
                    help="launch form of the timed iterations (default: the workload's)")
    ap.add_argument("--adapt2-tau", type=float, default=0.0,
                    help="also enrich the level-2 faces with this threshold (0: off)")
    ap.add_argument("--study", default=None, choices=("stopping", "strategies", "rsweep", "tau"),
                    help="a parameter study instead of the benchmark line (64^3 sequence; tau: holed cube)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures the single-GPU path only (one process, one MI355X); "
              "--gpus %d is not supported" % args.gpus, file=sys.stderr)
        sys.exit(2)

    if args.study:
        return run_study(args)
    import workload
    spec = WORKLOADS[args.workload]
    s = workload.workload(args.workload)
    if args.roofline_only:
        return run_roofline_only(args, s, spec)
    n_rhs = args.n_rhs or s["n_rhs"]
    step_rhs = spec["step_rhs"] or n_rhs
    n_rhs = max(step_rhs, n_rhs // step_rhs * step_rhs)
    t0 = time.perf_counter()
    F_np = make_rhs(s, n_rhs)
    gen_s = time.perf_counter() - t0
    print("[bench] %s: %d right-hand sides generated in %.1f s" % (args.workload, n_rhs, gen_s),
          file=sys.stderr, flush=True)

    import torch

    from paper_2412_17543_amd.solver import Solver
    F = torch.tensor(F_np, device="cuda")       # inputs resident in HBM before timing
    del F_np
    torch.cuda.synchronize()
    head = spec["prec"]
    others = [p for p in (64, 32, 16) if p != head and not (p != 64 and args.no_mixed)
              and not (p == 16 and args.no_bf16)]
    if args.no_mixed:
        head = 64
        others = []
    t0 = time.perf_counter()
    g = Solver(s["nx"], s["elem_to_sub"], s["coef"], sub_to_subregion=s["sub_to_subregion"],
               elem_keep=s["elem_keep"], R=s["R"], local_prec=head, local_prec_set=others,
               adapt_tau=10.0 if spec["adapt"] else 0.0, adapt_max_per_face=10,
               adapt2_tau=args.adapt2_tau, adapt2_max_per_face=10)
    torch.cuda.synchronize()
    setup_s = time.perf_counter() - t0
    print("[bench] setup %.1f s" % setup_s, file=sys.stderr, flush=True)
    # the Schur product's configuration: --pin, else the one the hardware
    # counter passes measured (profiles/traffic_<workload>.json, while the
    # kernel sources are unchanged), else the autotuner's
    traffic_rec, pin_source = None, "autotuned"
    tf = os.path.join(ROOT, "profiles", "traffic_%s.json" % args.workload)
    if os.path.exists(tf):
        t = json.load(open(tf))
        if t.get("kernel_hash") == kernel_hash():
            traffic_rec = t
    if args.pin:
        g.set_launch(True, [int(v) for v in args.pin.split(",")])
        pin_source = "command line"
    elif traffic_rec is not None:
        g.set_launch(True, list(traffic_rec["cfg"]) + [0, 0, 0, 0])
        pin_source = "profiles/traffic_%s.json" % args.workload
    info = g.info()

    # iterations queued kernel by kernel, or replays of a captured hipGraph
    launch = args.launch or spec.get("launch", "queued")
    g.set_launch(launch)
    forms, Us = {}, {}
    order = [head] + [p for p in others if p == 64] + [p for p in others if p != 64]
    for p in order:
        g.set_local_prec(p)
        res, Us[p], its = run_form(torch, g, F, args.rtol, args.steps, args.warmup, step_rhs, keep_u=True)
        res["kernels"] = {k: roofline_of(v) for k, v in g.time_kernels(20).items()}
        res["tuning"] = g.tuning()
        forms[p] = res
        print("[bench] %s form: %.2f solves/s, iterations %s" % (PREC_NAME[p], res["value"], res["iters"]),
              file=sys.stderr, flush=True)
    if 64 in Us and Us[64] is not None:
        U64 = Us[64]
        for p in order:
            if p != 64 and Us[p] is not None:
                forms[p]["max_rel_diff_vs_fp64"] = float(max(
                    ((Us[p][k] - U64[k]).abs().max() / U64[k].abs().max()).item() for k in range(U64.shape[0])))
    del Us
    plain = None
    if not args.no_plain and 64 in order:
        # the plain float64 form: kernels one by one with a host check after
        # every iteration, untuned default product configuration
        g.set_local_prec(64)
        g.set_launch("plain", [-1] * 8)
        plain, _, _ = run_form(torch, g, F, args.rtol, args.steps, args.warmup, step_rhs, keep_u=False)
        print("[bench] plain f64 form: %.2f solves/s" % plain["value"], file=sys.stderr, flush=True)
    hf = forms[head]
    k = hf["kernels"]
    dom = max(("schur", "neumann"), key=lambda n: k[n]["avg_launch_us"])
    dk = k[dom]
    traffic = None
    if traffic_rec is not None:
        t = traffic_rec
        tun = hf["tuning"]["schur" if dom == "schur" else "neumann"]
        cfg = [int(tun[x]) for x in ("blocks_per_cu", "per_subdomain", "waves", "unroll")]
        if t.get("kernel") == dom and t.get("cfg") == cfg and t.get("prec") == (64 if dom == "schur" else head):
            traffic = t["bytes_per_launch"]
    kname = ("k_symv<double, %d, %d, OpSchur>" if dom == "schur" else "k_symv<%s, %%d, %%d, OpNeumann>" %
             {64: "double", 32: "float", 16: "unsigned short"}[head])
    tun = hf["tuning"][dom]
    kname = kname % (int(tun["waves"]), int(tun["unroll"]))
    line = {
        "metric": METRIC,
        "value": hf["value"],
        "unit": "solves/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": hf["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if head == 64 else "f64+%s" % PREC_NAME[head],
        "data": "synthetic",
        "config": {"workload": spec["desc"], "form": "%s N_i and Phi_i storage, float64 elsewhere" % PREC_NAME[head],
                   "n_rhs": n_rhs, "rhs_per_step": step_rhs, "n_gamma": info["n_gamma"],
                   "n_coarse": info["n_coarse"], "rtol": args.rtol, "launch": launch},
        "iters": hf["iters"],
        "basis": hf["basis"],
        "max_true_relres": hf["max_true_relres"],
        "setup_s": round(setup_s, 2),
        "pin_source": pin_source,
        "roofline": {"bound": "hbm", "kernel": kname, "achieved": dk["achieved"], "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": dk["frac"], "traffic": traffic, "avg_launch_us": dk["avg_launch_us"],
                     "algorithmic_bytes_per_launch": dk["algorithmic_bytes_per_launch"],
                     "precond_apply": dict(k["precond"], peak=HBM_PEAK_GBS),
                     "kernels": k},
        "forms": {},
        "rhs_generation_s": round(gen_s, 1),
        "device_peak_gb": round(g.solve_info()["device_peak_bytes"] / 1e9, 2),
        "device_held_gb": round(g.solve_info()["device_bytes"] / 1e9, 2),
    }
    if spec["adapt"]:
        line["adaptive"] = g.adaptive_stats()
    if args.adapt2_tau > 0:
        line["adaptive_level2"] = dict(g.adaptive2_stats(), tau=args.adapt2_tau, level3=info["level3"])
    for p in order:
        f = dict(forms[p])
        f.pop("kernels")
        f["precond_apply"] = forms[p]["kernels"]["precond"]
        f["products"] = {n: forms[p]["kernels"][n] for n in ("schur", "neumann")}
        if 64 in forms:
            f["speedup_vs_fp64"] = round(forms[p]["value"] / forms[64]["value"], 3)
        if plain:
            f["speedup_vs_plain_fp64"] = round(forms[p]["value"] / plain["value"], 3)
        line["forms"][PREC_NAME[p]] = f
    if plain:
        line["forms"]["f64_plain"] = plain
    if args.adjoint:
        if 64 in order:
            g.set_local_prec(64)
        g.set_launch(True)
        U, its, rr = g.solve_sequence(F, args.rtol)
        dLdu = 2.0 * (U - 0.9 * U)
        g.adjoint_grad(dLdu, U, args.rtol)          # warm-up
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        reps = max(1, args.steps // max(1, n_rhs // step_rhs))
        for _ in range(reps):
            grad, gF = g.adjoint_grad(dLdu, U, args.rtol)
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
        line["adjoint"] = {"value": round(n_rhs * reps / el, 3), "unit": "adjoint solves/s",
                           "s_per_sequence": round(el / reps, 4), "grad_norm": float(grad.norm().item())}
        # the same adjoint systems solved as blocks of at most 32 columns
        chunks = [(k, min(n_rhs, k + 32)) for k in range(0, n_rhs, 32)]

        def block_grad():
            total, its = None, []
            for k0, k1 in chunks:
                gk, _, it = g.adjoint_grad_block(dLdu[k0:k1], U[k0:k1], args.rtol)
                total = gk if total is None else total + gk
                its.append(it)
            return total, its
        block_grad()                                # warm-up
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            gb, bits = block_grad()
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
        line["adjoint"]["block"] = {"value": round(n_rhs * reps / el, 3), "unit": "adjoint solves/s",
                                    "s_per_sequence": round(el / reps, 4), "block_iterations": bits,
                                    "max_rel_diff_vs_column_by_column":
                                        float(((gb - grad).abs().max() / grad.abs().max()).item())}
    if not args.no_cpu_baseline:
        line["cpu_baseline"] = cpu_baseline(args.workload, s, info["n_sub"])
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
