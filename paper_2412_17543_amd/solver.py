"""Python front end: a solver object over the C ABI, and an autograd Function.

PyTorch provides device memory and the stream; every step of setup, solve,
recycling and gradient runs in the library's HIP kernels.
"""
from __future__ import annotations

import ctypes

import numpy as np
import torch

from . import _lib
from ._lib import check

WEIGHTS = {"card": 0, "diag": 1}
STRATEGY = {"B1": 1, "B2": 2, "B3": 3, "B4": 4}


def _ptr(t: torch.Tensor) -> int:
    return t.data_ptr()


class Solver:
    """Deflated PCG with two/three-level BDDC on a structured Q1 box.

    Parameters mirror ``bddc_setup``: element partition (and optional
    subdomain->subregion grouping for three levels), element coefficients,
    optional element keep mask (holes) and Dirichlet node mask.  ``use_graph``
    selects how iterations are launched: "queued" (or True, the default:
    kernels queued ahead of an asynchronous convergence poll), "graph" (the
    same with replays of a captured hipGraph) or "plain" (or False: a host
    check after every iteration).
    """

    def __init__(self, nx, elem_to_sub, coef, sub_to_subregion=None, elem_keep=None,
                 node_dirichlet=None, ny=None, nz=None, R=0, strategy="B4", local_prec=64,
                 weights="diag", constraints=("corners", "faces"), stop_rule="rhs",
                 init_guess="prev", max_it=1000, save_cap=256, freeze_tol=1e-5,
                 use_graph=True, autotune=True, coarse_form="auto", product_cfg=None, reorth=False,
                 adapt_tau=0.0, adapt_max_per_face=10, local_prec_set=(), coef_log=False, restart_every=0,
                 adapt2_tau=0.0, adapt2_max_per_face=10, adapt_lobpcg_it=0,
                 device="cuda", stream=None):
        lib = _lib.load()
        self.lib = lib
        self.device = torch.device(device)
        if self.device.type != "cuda":
            raise RuntimeError("the BDDC library runs on the GPU only")
        if self.device.index is None:
            self.device = torch.device("cuda", torch.cuda.current_device())
        ny = nx if ny is None else ny
        nz = nx if nz is None else nz
        self.nx, self.ny, self.nz = nx, ny, nz
        self.n_elem = nx * ny * nz
        self.n_nodes = (nx + 1) * (ny + 1) * (nz + 1)
        self._e2s = np.ascontiguousarray(elem_to_sub, dtype=np.int32)
        if isinstance(coef, torch.Tensor):
            self._coef = coef.detach().to(dtype=torch.float64).contiguous()
        else:
            self._coef = np.ascontiguousarray(coef, dtype=np.float64)
        self._s2r = None if sub_to_subregion is None else np.ascontiguousarray(sub_to_subregion, dtype=np.int32)
        self._keep = None if elem_keep is None else np.ascontiguousarray(elem_keep, dtype=np.uint8)
        self._dir = None if node_dirichlet is None else np.ascontiguousarray(node_dirichlet, dtype=np.uint8)
        n_coef = self._coef.numel() if isinstance(self._coef, torch.Tensor) else self._coef.size
        assert self._e2s.size == self.n_elem and n_coef == self.n_elem
        mesh = _lib.Mesh(nx, ny, nz, 1.0 / nx,
                         None if self._keep is None else self._keep.ctypes.data,
                         None if self._dir is None else self._dir.ctypes.data)
        kept = self._e2s if self._keep is None else self._e2s[self._keep.astype(bool)]
        n_sub = int(kept.max()) + 1
        n_sr = 0 if self._s2r is None else int(self._s2r.max()) + 1
        part = _lib.Partition(n_sub, self._e2s.ctypes.data, n_sr,
                              None if self._s2r is None else self._s2r.ctypes.data)
        o = _lib.Opts()
        lib.bddc_default_opts(ctypes.byref(o))
        cmask = 0
        for c in constraints:
            cmask |= {"corners": 1, "faces": 2, "edges": 4}[c]
        o.constraints = cmask
        o.weights = WEIGHTS[weights]
        o.local_prec = {64: 64, 32: 32, 16: 16, "fp64": 64, "fp32": 32, "bf16": 16}[local_prec]
        o.recycle_R = R
        o.recycle_strategy = STRATEGY[strategy] if isinstance(strategy, str) else int(strategy)
        o.ritz_freeze_tol = freeze_tol
        o.stop_rule = {"rhs": 0, "r0": 1}[stop_rule]
        o.init_guess = {"prev": 0, "zero": 1}[init_guess]
        o.max_it = max_it
        o.save_cap = save_cap
        o.use_graph = {True: 2, False: 0, "queued": 2, "graph": 1, "plain": 0}[use_graph]
        o.autotune = 1 if autotune else 0
        o.coarse_form = {"auto": 0, "chain": 1, "explicit": 2}[coarse_form]
        o.reorth = 1 if reorth else 0
        o.adapt_tau = float(adapt_tau)
        o.adapt_max_per_face = int(adapt_max_per_face)
        o.local_prec_set = sum({64: 1, 32: 2, 16: 4}[p] for p in local_prec_set)
        o.coef_log = 1 if coef_log else 0
        o.restart_every = int(restart_every)
        o.adapt2_tau = float(adapt2_tau)
        o.adapt2_max_per_face = int(adapt2_max_per_face)
        o.adapt_lobpcg_it = int(adapt_lobpcg_it)
        if product_cfg is not None:
            assert len(product_cfg) == 8
            for i, v in enumerate(product_cfg):
                o.product_cfg[i] = int(v)
        self.opts = o
        torch.cuda.set_device(self.device)
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        ctx = ctypes.c_void_p()
        coef_ptr = self._coef.data_ptr() if isinstance(self._coef, torch.Tensor) else self._coef.ctypes.data
        check(lib.bddc_setup(ctypes.byref(mesh), ctypes.byref(part), coef_ptr,
                             ctypes.byref(o), ctypes.c_void_p(self.stream.cuda_stream), ctypes.byref(ctx)))
        self.ctx = ctx
        self.n_gamma = self.info()["n_gamma"]

    # ------------------------------------------------------------------ info
    INFO_KEYS = ("n_nodes", "n_gamma", "n_sub", "n_coarse", "corners", "faces", "edges",
                 "level2_interface", "level2_interior", "level3", "deflation_cols", "frozen",
                 "bytes_S", "bytes_N", "max_nB", "device_bytes")

    def info(self) -> dict:
        a = (ctypes.c_int64 * 16)()
        check(self.lib.bddc_info(self.ctx, a))
        return dict(zip(self.INFO_KEYS, list(a)))

    def adaptive_stats(self) -> dict:
        """Adaptive face selection at setup (Section 3.3): faces examined, rows
        added, largest face eigenvalue before enrichment, seconds."""
        a = (ctypes.c_double * 4)()
        check(self.lib.bddc_adaptive_stats(self.ctx, a))
        return dict(faces=int(a[0]), added=int(a[1]), lam_max=float(a[2]), seconds=float(a[3]))

    def adaptive2_stats(self) -> dict:
        """The same for the level-2 faces (three levels, adapt2_tau > 0)."""
        a = (ctypes.c_double * 4)()
        check(self.lib.bddc_adaptive2_stats(self.ctx, a))
        return dict(faces=int(a[0]), added=int(a[1]), lam_max=float(a[2]), seconds=float(a[3]))

    def interface_nodes(self) -> np.ndarray:
        a = (ctypes.c_int64 * self.n_gamma)()
        check(self.lib.bddc_interface_nodes(self.ctx, a))
        return np.frombuffer(a, dtype=np.int64).copy()

    def ritz_values(self) -> np.ndarray:
        buf = (ctypes.c_double * 64)()
        cnt = ctypes.c_int32()
        check(self.lib.bddc_ritz_values(self.ctx, buf, 64, ctypes.byref(cnt)))
        return np.frombuffer(buf, dtype=np.float64)[: cnt.value].copy()

    SOLVE_INFO_KEYS = ("recycle_steps", "refused", "frozen", "freeze_step", "replacements", "run_start",
                       "deflation_cols", "device_bytes", "device_peak_bytes", "local_prec")

    def solve_info(self) -> dict:
        """Recycling and memory state (bddc_solve_info)."""
        a = (ctypes.c_int64 * 10)()
        check(self.lib.bddc_solve_info(self.ctx, a, 10))
        return dict(zip(self.SOLVE_INFO_KEYS, list(a)))

    def set_local_prec(self, prec):
        """Apply the Neumann operators in another storage precision built at setup."""
        check(self.lib.bddc_set_local_prec(self.ctx, {64: 64, 32: 32, 16: 16, "fp64": 64, "fp32": 32,
                                                      "bf16": 16}[prec]))

    def set_launch(self, use_graph=True, product_cfg=None):
        """Launch form of later solves ("queued"/True, "graph", "plain"/False)
        and optionally the product configuration (8 ints; a product whose
        first entry is 0 keeps its configuration, negative: the untuned
        default)."""
        ug = {True: 2, False: 0, "queued": 2, "graph": 1, "plain": 0}[use_graph]
        cfg = None
        if product_cfg is not None:
            assert len(product_cfg) == 8
            cfg = (ctypes.c_int32 * 8)(*[int(v) for v in product_cfg])
        check(self.lib.bddc_set_launch(self.ctx, ug, cfg))

    KERNEL_KEYS = ("schur", "neumann", "interior", "precond", "coarse", "prolong_assemble")

    def time_kernels(self, reps=20) -> dict:
        """Back-to-back launches timed with HIP events (bddc_time_kernels):
        microseconds and algorithmic bytes per launch of the three batched
        products, one preconditioner application and its coarse and
        prolongation/assembly parts."""
        a = (ctypes.c_double * 12)()
        check(self.lib.bddc_time_kernels(self.ctx, reps, a, 12))
        return {k: {"us": a[2 * i], "bytes": a[2 * i + 1]} for i, k in enumerate(self.KERNEL_KEYS)}

    TUNING_KEYS = ("blocks", "blocks_per_cu", "per_subdomain", "waves", "unroll", "best_us", "tiles")

    def tuning(self) -> dict:
        """Configuration chosen for the Schur and Neumann products."""
        a = (ctypes.c_double * 14)()
        check(self.lib.bddc_tuning(self.ctx, a))
        v = list(a)
        return {"schur": dict(zip(self.TUNING_KEYS, v[:7])), "neumann": dict(zip(self.TUNING_KEYS, v[7:]))}

    def time_products(self, reps=20) -> dict:
        """Back-to-back launches of the Schur and Neumann products timed with
        HIP events: microseconds and algorithmic bytes per launch."""
        a = (ctypes.c_double * 4)()
        check(self.lib.bddc_time_products(self.ctx, reps, a))
        return {"schur": {"us": a[0], "bytes": a[1]}, "neumann": {"us": a[2], "bytes": a[3]}}

    def enable_timing(self, on=True, classes=None):
        """Time kernel classes with HIP events (classes: iterable of STAT_KEYS)."""
        mask = 0 if not on else (1 if classes is None else
                                 sum(1 << self.STAT_KEYS.index(k) for k in classes) | 64)
        check(self.lib.bddc_enable_timing(self.ctx, mask))

    STAT_KEYS = ("schur", "precond_local", "coarse", "vector", "condense_recover", "recycle")

    def stats(self) -> dict:
        a = (ctypes.c_double * 18)()
        check(self.lib.bddc_stats(self.ctx, a, 6))
        v = np.frombuffer(a, dtype=np.float64)
        return {k: dict(ms=v[3 * i], count=int(v[3 * i + 1]), bytes=v[3 * i + 2])
                for i, k in enumerate(self.STAT_KEYS)}

    # --------------------------------------------------------------- solving
    def _dev(self, x, shape=None) -> torch.Tensor:
        t = torch.as_tensor(x, dtype=torch.float64, device=self.device)
        t = t.contiguous()
        if shape is not None:
            t = t.reshape(shape)
        return t

    def solve_sequence(self, rhs, rtol=1e-8):
        """rhs: (n_rhs, n_nodes) load vectors.  Returns (u, iters, true_relres)."""
        F = self._dev(rhs)
        if F.dim() == 1:
            F = F[None]
        n = F.shape[0]
        assert F.shape[1] == self.n_nodes
        U = torch.empty_like(F)
        its = np.zeros(n, dtype=np.int32)
        rr = np.zeros(n, dtype=np.float64)
        check(self.lib.dpcg_solve(self.ctx, _ptr(F), n, rtol, _ptr(U),
                                  its.ctypes.data, rr.ctypes.data))
        return U, its, rr

    def reset_recycle(self):
        check(self.lib.bddc_reset_recycle(self.ctx))

    def recycle_update(self):
        check(self.lib.recycle_update(self.ctx))

    def apply_schur(self, p):
        p = self._dev(p)
        q = torch.empty_like(p)
        check(self.lib.bddc_apply_schur(self.ctx, _ptr(p), _ptr(q)))
        return q

    def apply_precond(self, r):
        r = self._dev(r)
        z = torch.empty_like(r)
        check(self.lib.bddc_apply_precond(self.ctx, _ptr(r), _ptr(z)))
        return z

    def condense(self, F):
        F = self._dev(F)
        b = torch.empty(self.n_gamma, dtype=torch.float64, device=self.device)
        check(self.lib.bddc_condense(self.ctx, _ptr(F), _ptr(b)))
        return b

    def adjoint_grad(self, dLdu, u, rtol=1e-10):
        dLdu = self._dev(dLdu)
        u = self._dev(u)
        if dLdu.dim() == 1:
            dLdu, u = dLdu[None], u[None]
        g = torch.empty(self.n_elem, dtype=torch.float64, device=self.device)
        gF = torch.empty_like(dLdu)
        check(self.lib.bddc_adjoint_grad(self.ctx, _ptr(dLdu), dLdu.shape[0], _ptr(u), rtol,
                                         _ptr(g), _ptr(gF)))
        return g, gF

    def adjoint_grad_block(self, dLdu, u, rtol=1e-10):
        """adjoint_grad with the adjoint systems solved as one block
        (bddc_adjoint_grad_block).  Returns (grad, dL/dF, block iterations)."""
        dLdu = self._dev(dLdu)
        u = self._dev(u)
        if dLdu.dim() == 1:
            dLdu, u = dLdu[None], u[None]
        g = torch.empty(self.n_elem, dtype=torch.float64, device=self.device)
        gF = torch.empty_like(dLdu)
        it = ctypes.c_int32(0)
        check(self.lib.bddc_adjoint_grad_block(self.ctx, _ptr(dLdu), dLdu.shape[0], _ptr(u), rtol,
                                               _ptr(g), _ptr(gF), ctypes.byref(it)))
        return g, gF, it.value

    def close(self):
        if getattr(self, "ctx", None):
            self.lib.bddc_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class DPCGSolveFn(torch.autograd.Function):
    """u_seq = K(exp(theta))^{-1} F_seq with an adjoint backward.

    forward(theta, F, spec) builds the solver for the coefficients exp(theta)
    (``spec`` holds nx, partition and options) and solves the sequence;
    backward solves K lambda_k = dL/du_k with the same preconditioner and
    recycled basis (K is symmetric) and forms dL/dtheta_e in one kernel.
    """

    @staticmethod
    def forward(ctx, theta, F, spec):
        s = dict(spec)
        rtol = s.pop("rtol", 1e-10)
        solver = Solver(coef=theta.detach(), coef_log=True, **s)
        U, its, rr = solver.solve_sequence(F.detach(), rtol)
        ctx.solver = solver
        ctx.rtol = rtol
        ctx.save_for_backward(U)
        ctx.iters = its
        return U

    @staticmethod
    def backward(ctx, dU):
        (U,) = ctx.saved_tensors
        g, gF = ctx.solver.adjoint_grad(dU.contiguous(), U, ctx.rtol)
        ctx.solver.close()
        return g, gF, None
