"""Python binding of the lqgrid C ABI (include/lqgrid.h).

Argument marshalling only: every step of the solve runs in the HIP kernels of
liblqgrid.so.  PyTorch provides device memory (the problem arrays, outputs
and the workspace are torch tensors on the GPU) and the current HIP stream.
If the library is not built the binding raises; there is no CPU fallback.
"""
from __future__ import annotations

import ctypes
import os
from ctypes import POINTER, byref, c_double, c_int, c_longlong, c_size_t, c_void_p

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "liblqgrid.so")

OK, EINVAL, ENOTSPD, EBREAKDOWN, ENOCONV, EWORKSPACE, EHIP, EUNSUPPORTED = range(8)
FP64, FP32_REFINE = 0, 1
OP_DELTA, OP_XI, OP_OMEGA, OP_PHI_SOLVE, OP_PRECOND, OP_NODE_PRECOND = range(6)
PRECOND_NBJM, PRECOND_NODE_TEMPORAL, PRECOND_NONE = range(3)
OP_F32 = 16   # or-ed into an operator code: run the FP32 kernels
PROF_DELTA, PROF_PHI_SOLVE, PROF_RHS, PROF_UPDATE = range(4)


class ProblemDesc(ctypes.Structure):
    _fields_ = [("K", c_int), ("N", c_int), ("T", c_int), ("n", c_int),
                ("m", c_int), ("A", c_void_p), ("A_nbr", c_void_p),
                ("B", c_void_p), ("Q", c_void_p), ("R", c_void_p),
                ("QT", c_void_p), ("n_node", c_void_p), ("m_node", c_void_p),
                ("time_varying", c_int)]


class Boundary(ctypes.Structure):
    _fields_ = [("alpha_lo", c_void_p), ("alpha_hi", c_void_p),
                ("beta_lo", c_void_p), ("beta_hi", c_void_p)]


class SolveOpts(ctypes.Structure):
    _fields_ = [("outer_S", c_int), ("inner_L", c_int), ("tol", c_double),
                ("max_iter", c_int), ("precision", c_int),
                ("inner_tol", c_double), ("check_every", c_int),
                ("warm_fallback", c_int), ("preconditioner", c_int)]


class WsNetDesc(ctypes.Structure):
    _fields_ = [("K", c_int), ("N", c_int), ("n", c_int), ("m", c_int),
                ("T", c_int), ("layers", c_int)]


class Info(ctypes.Structure):
    _fields_ = [("status", c_int), ("iterations", c_int),
                ("refinements", c_int), ("restarts", c_int),
                ("rel_kkt_residual", c_double), ("rel_res_inf", c_double),
                ("seconds", c_double), ("warm_start_used", c_int)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


_lib = None


def load(path: str = LIB_PATH):
    """Load liblqgrid.so (built by paper_2304_04980_amd.build)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(
            f"{path} is missing: build it with `python -m paper_2304_04980_amd.build`"
            " (the solver has no fallback path)")
    # One HIP runtime per process: torch ships its own libamdhip64.so.7.
    # Importing torch first makes the library's libamdhip64.so.7 dependency
    # resolve (by SONAME) to the copy torch already mapped; loading ours first
    # would map a second runtime that cannot open the device torch holds.
    import torch  # noqa: F401
    L = ctypes.CDLL(path)
    L.lqgrid_default_opts.argtypes = [POINTER(SolveOpts)]
    L.lqgrid_default_opts.restype = None
    L.lqgrid_workspace_bytes.argtypes = [POINTER(ProblemDesc), POINTER(SolveOpts)]
    L.lqgrid_workspace_bytes.restype = c_size_t
    L.lqgrid_setup.argtypes = [POINTER(ProblemDesc), c_void_p, c_size_t,
                               c_void_p, POINTER(c_void_p)]
    L.lqgrid_setup.restype = c_int
    L.lqgrid_factor.argtypes = [c_void_p]
    L.lqgrid_factor.restype = c_int
    L.lqgrid_pcg_solve.argtypes = [c_void_p, c_void_p, POINTER(SolveOpts),
                                   c_void_p, c_void_p, c_void_p, c_void_p,
                                   POINTER(Info)]
    L.lqgrid_pcg_solve.restype = c_int
    L.lqgrid_pcg_solve_bc.argtypes = [c_void_p, c_void_p, POINTER(Boundary),
                                      POINTER(SolveOpts), c_void_p, c_void_p, c_void_p,
                                      c_void_p, POINTER(Info)]
    L.lqgrid_pcg_solve_bc.restype = c_int
    L.lqgrid_batch_workspace_bytes.argtypes = [c_int, POINTER(ProblemDesc),
                                               POINTER(SolveOpts)]
    L.lqgrid_batch_workspace_bytes.restype = c_size_t
    L.lqgrid_batch_solve.argtypes = [c_int, POINTER(ProblemDesc),
                                     POINTER(c_void_p), POINTER(SolveOpts),
                                     POINTER(c_void_p), c_void_p, c_size_t,
                                     c_void_p, POINTER(Info)]
    L.lqgrid_batch_solve.restype = c_int
    L.lqgrid_apply_operator.argtypes = [c_void_p, c_int, c_int, c_int,
                                        c_void_p, c_void_p]
    L.lqgrid_apply_operator.restype = c_int
    L.lqgrid_profile_enable.argtypes = [c_void_p, c_int]
    L.lqgrid_profile_enable.restype = c_int
    L.lqgrid_profile_read.argtypes = [c_void_p, c_int, POINTER(c_longlong),
                                      POINTER(c_double)]
    L.lqgrid_profile_read.restype = c_int
    L.lqgrid_destroy.argtypes = [c_void_p]
    L.lqgrid_destroy.restype = None
    L.lqgrid_status_string.argtypes = [c_int]
    L.lqgrid_status_string.restype = ctypes.c_char_p
    L.lqgrid_abi_version.argtypes = []
    L.lqgrid_abi_version.restype = c_int
    L.lqgrid_last_error.argtypes = []
    L.lqgrid_last_error.restype = ctypes.c_char_p
    W = POINTER(WsNetDesc)
    L.lqgrid_wsnet_param_count.argtypes = [W]
    L.lqgrid_wsnet_param_count.restype = c_size_t
    L.lqgrid_wsnet_sample_bytes.argtypes = [W, c_int]
    L.lqgrid_wsnet_sample_bytes.restype = c_size_t
    L.lqgrid_wsnet_workspace_bytes.argtypes = [W, c_int]
    L.lqgrid_wsnet_workspace_bytes.restype = c_size_t
    L.lqgrid_wsnet_features.argtypes = [W, POINTER(ProblemDesc), c_void_p, c_void_p,
                                        c_void_p]
    L.lqgrid_wsnet_features.restype = c_int
    L.lqgrid_wsnet_targets.argtypes = [W, c_void_p, c_void_p, c_void_p, c_size_t,
                                       c_void_p]
    L.lqgrid_wsnet_targets.restype = c_int
    L.lqgrid_wsnet_forward.argtypes = [W, c_int, c_void_p, c_void_p, c_void_p,
                                       c_void_p, c_void_p, c_size_t, c_void_p]
    L.lqgrid_wsnet_forward.restype = c_int
    L.lqgrid_wsnet_gradient.argtypes = [W, c_int, c_void_p, c_void_p, c_void_p,
                                        c_void_p, c_void_p, POINTER(c_double),
                                        c_void_p, c_size_t, c_void_p]
    L.lqgrid_wsnet_gradient.restype = c_int
    L.lqgrid_wsnet_backward.argtypes = [W, c_int, c_void_p, c_void_p, c_void_p, c_void_p,
                                        c_void_p, c_void_p, c_size_t, c_void_p]
    L.lqgrid_wsnet_backward.restype = c_int
    L.lqgrid_wsnet_adam.argtypes = [W, c_void_p, c_void_p, c_void_p, c_int,
                                    ctypes.c_float, c_void_p]
    L.lqgrid_wsnet_adam.restype = c_int
    L.lqgrid_wsnet_predict.argtypes = [W, c_void_p, c_void_p, c_void_p, c_void_p,
                                       c_size_t, c_void_p]
    L.lqgrid_wsnet_predict.restype = c_int
    L.lqgrid_nbjm_solve.argtypes = [c_void_p, c_void_p, POINTER(SolveOpts), c_void_p,
                                    c_void_p, c_void_p, POINTER(Info)]
    L.lqgrid_nbjm_solve.restype = c_int
    L.lqgrid_condition_estimate.argtypes = [c_void_p, c_void_p, c_int, c_int, c_int,
                                            c_double, c_int, POINTER(c_double),
                                            POINTER(c_double), POINTER(c_double),
                                            POINTER(c_int)]
    L.lqgrid_condition_estimate.restype = c_int
    L.lqgrid_noalloc_capacity.argtypes = []
    L.lqgrid_noalloc_capacity.restype = c_size_t
    L.lqgrid_solve_noalloc.argtypes = [POINTER(ProblemDesc), c_void_p, POINTER(SolveOpts),
                                       c_void_p, c_void_p, c_void_p, c_void_p,
                                       POINTER(Info)]
    L.lqgrid_solve_noalloc.restype = c_int
    _lib = L
    return L


EXPORTED = ["lqgrid_default_opts", "lqgrid_workspace_bytes", "lqgrid_setup",
            "lqgrid_factor", "lqgrid_pcg_solve", "lqgrid_batch_workspace_bytes",
            "lqgrid_batch_solve", "lqgrid_apply_operator",
            "lqgrid_profile_enable", "lqgrid_profile_read", "lqgrid_destroy",
            "lqgrid_status_string", "lqgrid_abi_version", "lqgrid_last_error",
            "lqgrid_wsnet_param_count", "lqgrid_wsnet_sample_bytes",
            "lqgrid_wsnet_workspace_bytes", "lqgrid_wsnet_features",
            "lqgrid_wsnet_targets", "lqgrid_wsnet_forward", "lqgrid_wsnet_gradient",
            "lqgrid_wsnet_adam", "lqgrid_wsnet_predict", "lqgrid_noalloc_capacity",
            "lqgrid_solve_noalloc", "lqgrid_nbjm_solve", "lqgrid_condition_estimate",
            "lqgrid_pcg_solve_bc", "lqgrid_wsnet_backward"]


class LqgridError(RuntimeError):
    def __init__(self, status, where):
        L = load()
        msg = L.lqgrid_status_string(status).decode()
        if status == EHIP:
            msg += " [" + L.lqgrid_last_error().decode() + "]"
        super().__init__(f"{where}: {msg} (status {status})")
        self.status = status


def default_opts(**kw) -> SolveOpts:
    o = SolveOpts()
    load().lqgrid_default_opts(byref(o))
    for k, v in kw.items():
        setattr(o, k, v)
    return o


def _ptr(t):
    return None if t is None else c_void_p(t.data_ptr())


def _stream():
    import torch
    return c_void_p(torch.cuda.current_stream().cuda_stream)


def workspace_bytes(K, N, T, n, m, time_varying=False, node_temporal=False) -> int:
    d = ProblemDesc(K, N, T, n, m, None, None, None, None, None, None, None, None,
                    1 if time_varying else 0)
    o = default_opts(preconditioner=PRECOND_NODE_TEMPORAL) if node_temporal else None
    return load().lqgrid_workspace_bytes(byref(d), byref(o) if o is not None else None)


def problem_desc(K, N, T, n, m, A, A_nbr, B, Q, R, QT=None, n_node=None,
                 m_node=None, time_varying=False) -> ProblemDesc:
    """Tensors must be contiguous float64 (sizes: int32) CUDA tensors in the
    header's layouts; the caller keeps them alive while the setup work runs."""
    return ProblemDesc(K, N, T, n, m, _ptr(A), _ptr(A_nbr), _ptr(B), _ptr(Q),
                       _ptr(R), _ptr(QT), _ptr(n_node), _ptr(m_node),
                       1 if time_varying else 0)


class Context:
    """One problem: lqgrid_setup + lqgrid_factor, then any number of
    lqgrid_pcg_solve calls (e.g. for different initial states)."""

    def __init__(self, problem, device="cuda", factor=True, workspace=None,
                 arrays=None, node_temporal=False):
        """problem: an lqgrid_synth.Problem (numpy arrays, copied to the
        device) or, with ``arrays``, just the dims of device-resident tensors.
        workspace: optional preallocated uint8 CUDA tensor, reused as is.
        node_temporal: size the workspace for the node-temporal preconditioner
        too (PRECOND_NODE_TEMPORAL)."""
        import torch
        self.L = load()
        p = problem
        self.dims = (p.K, p.N, p.T, p.n, p.m)
        f64 = dict(dtype=torch.float64, device=device)
        if arrays is None:
            arrays = {k: torch.as_tensor(getattr(p, k)).to(**f64).contiguous()
                      for k in ("A", "A_nbr", "B", "Q", "R", "QT")}
            for k in ("n_node", "m_node"):
                v = getattr(p, k, None)
                if v is not None:
                    arrays[k] = torch.as_tensor(v).to(dtype=torch.int32,
                                                      device=device).contiguous()
        self.arrays = arrays
        a = self.arrays
        self.desc = problem_desc(*self.dims, a["A"], a["A_nbr"], a["B"], a["Q"],
                                 a["R"], a["QT"], a.get("n_node"), a.get("m_node"),
                                 getattr(p, "time_varying", False))
        wo = default_opts(preconditioner=PRECOND_NODE_TEMPORAL) if node_temporal else None
        nbytes = self.L.lqgrid_workspace_bytes(byref(self.desc),
                                               byref(wo) if wo is not None else None)
        if nbytes == 0:
            raise LqgridError(EINVAL, "lqgrid_workspace_bytes")
        # 256-byte alignment: torch's caching allocator returns 512-byte
        # aligned blocks for fresh allocations
        if workspace is None or workspace.numel() < nbytes + 256:
            workspace = torch.empty(nbytes + 256, dtype=torch.uint8, device=device)
        self.workspace = workspace
        base = self.workspace.data_ptr()
        self.ws_ptr = (base + 255) // 256 * 256
        self.ws_bytes = nbytes
        ctx = c_void_p()
        st = self.L.lqgrid_setup(byref(self.desc), c_void_p(self.ws_ptr),
                                 self.ws_bytes, _stream(), byref(ctx))
        if st != OK:
            raise LqgridError(st, "lqgrid_setup")
        self.ctx = ctx
        if factor:
            self.factor()

    def factor(self):
        st = self.L.lqgrid_factor(self.ctx)
        if st != OK:
            raise LqgridError(st, "lqgrid_factor")

    def solve(self, x0, opts: SolveOpts | None = None, delta_init=None,
              want_primal=False, out=None, raise_on_error=True, out_x=None,
              out_u=None, boundary=None):
        """x0: [N][K][n] float64 CUDA tensor (or array).  Returns
        (delta [T+1][N][K][n], x or None, u or None, info dict).  out, out_x,
        out_u: optional preallocated outputs (out_x / out_u imply
        want_primal).  boundary: optional dict (or object with attributes)
        alpha_lo, alpha_hi, beta_lo, beta_hi of known boundary states
        (lqgrid_pcg_solve_bc)."""
        import torch
        K, N, T, n, m = self.dims
        dev = self.arrays["A"].device
        x0 = torch.as_tensor(x0).to(dtype=torch.float64, device=dev).contiguous()
        if opts is None:
            opts = default_opts()
        delta = out if out is not None else torch.empty((T + 1, N, K, n), dtype=torch.float64, device=dev)
        x, u = out_x, out_u
        if want_primal and x is None:
            x = torch.empty((T + 1, N, K, n), dtype=torch.float64, device=dev)
        if want_primal and u is None:
            u = torch.empty((T, N, K, m), dtype=torch.float64, device=dev)
        di = None
        if delta_init is not None:
            di = torch.as_tensor(delta_init).to(dtype=torch.float64, device=dev).contiguous()
        info = Info()
        if boundary is None:
            st = self.L.lqgrid_pcg_solve(self.ctx, _ptr(x0), byref(opts), _ptr(di),
                                         _ptr(delta), _ptr(x), _ptr(u), byref(info))
        else:
            keep = {}
            for k in ("alpha_lo", "alpha_hi", "beta_lo", "beta_hi"):
                v = boundary.get(k) if isinstance(boundary, dict) else getattr(boundary, k, None)
                if v is not None:
                    keep[k] = torch.as_tensor(v).to(dtype=torch.float64, device=dev).contiguous()
            bc = Boundary(*[_ptr(keep.get(k)) for k in ("alpha_lo", "alpha_hi",
                                                        "beta_lo", "beta_hi")])
            st = self.L.lqgrid_pcg_solve_bc(self.ctx, _ptr(x0), byref(bc), byref(opts),
                                            _ptr(di), _ptr(delta), _ptr(x), _ptr(u),
                                            byref(info))
            torch.cuda.current_stream().synchronize()
            del keep
        if st != OK and raise_on_error:
            raise LqgridError(st, "lqgrid_pcg_solve")
        return delta, x, u, info.as_dict()

    def nbjm_solve(self, x0, opts: SolveOpts | None = None, want_primal=False,
                   raise_on_error=True):
        """Standalone NBJM (lqgrid_nbjm_solve).  Returns (delta, x or None,
        u or None, info dict); info["iterations"] counts outer sweeps."""
        import torch
        K, N, T, n, m = self.dims
        dev = self.arrays["A"].device
        x0 = torch.as_tensor(x0).to(dtype=torch.float64, device=dev).contiguous()
        opts = default_opts() if opts is None else opts
        delta = torch.empty((T + 1, N, K, n), dtype=torch.float64, device=dev)
        x = u = None
        if want_primal:
            x = torch.empty((T + 1, N, K, n), dtype=torch.float64, device=dev)
            u = torch.empty((T, N, K, m), dtype=torch.float64, device=dev)
        info = Info()
        st = self.L.lqgrid_nbjm_solve(self.ctx, _ptr(x0), byref(opts), _ptr(delta),
                                      _ptr(x), _ptr(u), byref(info))
        if st != OK and raise_on_error:
            raise LqgridError(st, "lqgrid_nbjm_solve")
        return delta, x, u, info.as_dict()

    def condition_estimate(self, x0, preconditioned=True, S=2, L=2, tol=1e-10,
                           max_iter=0):
        """lqgrid_condition_estimate: dict with kappa, lambda_min, lambda_max,
        iterations of the Lanczos estimate from one run of Algorithm 1.
        preconditioned: True / 1 (NBJM), 2 (node temporal), False / 0 (none)."""
        import torch
        dev = self.arrays["A"].device
        x0 = torch.as_tensor(x0).to(dtype=torch.float64, device=dev).contiguous()
        k, lo, hi, it = c_double(), c_double(), c_double(), c_int()
        mode = int(preconditioned) if not isinstance(preconditioned, bool) else int(preconditioned)
        st = self.L.lqgrid_condition_estimate(self.ctx, _ptr(x0), mode,
                                              S, L, tol, max_iter, byref(k), byref(lo),
                                              byref(hi), byref(it))
        if st != OK:
            raise LqgridError(st, "lqgrid_condition_estimate")
        return dict(kappa=k.value, lambda_min=lo.value, lambda_max=hi.value,
                    iterations=it.value)

    def apply(self, op, vec, S=2, L=2):
        import torch
        dev = self.arrays["A"].device
        vin = torch.as_tensor(vec).to(dtype=torch.float64, device=dev).contiguous()
        out = torch.empty_like(vin)
        st = self.L.lqgrid_apply_operator(self.ctx, op, S, L, _ptr(vin), _ptr(out))
        if st != OK:
            raise LqgridError(st, "lqgrid_apply_operator")
        torch.cuda.current_stream().synchronize()
        return out

    def profile_enable(self, on=True, stride=1):
        """Time every stride-th launch of each hot kernel with HIP events."""
        self.L.lqgrid_profile_enable(self.ctx, max(1, int(stride)) if on else 0)

    def profile_read(self, kernel):
        n = c_longlong()
        ms = c_double()
        self.L.lqgrid_profile_read(self.ctx, kernel, byref(n), byref(ms))
        return n.value, ms.value

    def close(self):
        if getattr(self, "ctx", None):
            self.L.lqgrid_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Batch:
    """Inputs, outputs and workspace of one lqgrid_batch_solve, resident on
    the device so that repeated solves time only the library call."""

    def __init__(self, problems, x0s=None, device="cuda", opts: SolveOpts | None = None):
        import torch
        self.L = load()
        f64 = dict(dtype=torch.float64, device=device)
        P = len(problems)
        self.P = P
        self.keep = []
        self.arrays, self.x0s = [], []
        self.descs = (ProblemDesc * P)()
        self.x0p = (c_void_p * P)()
        self.outp = (c_void_p * P)()
        self.outs = []
        for k, p in enumerate(problems):
            a = {nm: torch.as_tensor(getattr(p, nm)).to(**f64).contiguous()
                 for nm in ("A", "A_nbr", "B", "Q", "R", "QT")}
            self.keep.append(a)
            self.descs[k] = problem_desc(p.K, p.N, p.T, p.n, p.m, a["A"], a["A_nbr"],
                                         a["B"], a["Q"], a["R"], a["QT"])
            x0 = torch.as_tensor(p.x0 if x0s is None else x0s[k]).to(**f64).contiguous()
            self.keep.append(x0)
            self.arrays.append(a)
            self.x0s.append(x0)
            self.x0p[k] = x0.data_ptr()
            o = torch.empty((p.T + 1, p.N, p.K, p.n), **f64)
            self.outs.append(o)
            self.outp[k] = o.data_ptr()
        self.opts = default_opts() if opts is None else opts
        self.nbytes = self.L.lqgrid_batch_workspace_bytes(P, self.descs, byref(self.opts))
        if self.nbytes == 0:
            raise LqgridError(EINVAL, "lqgrid_batch_workspace_bytes")
        self.ws = torch.empty(self.nbytes + 256, dtype=torch.uint8, device=device)
        self.wp = (self.ws.data_ptr() + 255) // 256 * 256

    def solve(self, opts: SolveOpts | None = None):
        """Returns (list of delta tensors [T+1][N][K][n], list of info dicts,
        overall status)."""
        o = self.opts if opts is None else opts
        infos = (Info * self.P)()
        st = self.L.lqgrid_batch_solve(self.P, self.descs, self.x0p, byref(o), self.outp,
                                       c_void_p(self.wp), self.nbytes, _stream(), infos)
        return self.outs, [i.as_dict() for i in infos], st


def solve_noalloc(desc: ProblemDesc, x0, opts: SolveOpts, delta, x=None, u=None):
    """lqgrid_solve_noalloc: setup + factor + solve in the library's static
    device scratch (no workspace, no allocation).  desc holds device arrays;
    x0, delta, x, u are device tensors.  Returns (status, info dict)."""
    info = Info()
    st = load().lqgrid_solve_noalloc(byref(desc), _ptr(x0), byref(opts), _ptr(delta),
                                     _ptr(x), _ptr(u), _stream(), byref(info))
    return st, info.as_dict()


def batch_solve(problems, x0s=None, opts: SolveOpts | None = None, device="cuda"):
    """lqgrid_batch_solve over a list of problems sharing n."""
    return Batch(problems, x0s, device, opts).solve()


class WarmNet:
    """The warm-start network of one problem size: FP32 parameters and Adam
    moments on the device, plus the calls of the lqgrid_wsnet_* entry
    points.  Training data are arrays of per-problem feature and target
    samples (see features() and targets())."""

    def __init__(self, K, N, n, m, T, layers=6, device="cuda", params=None, seed=0):
        import numpy as np
        import torch
        self.L = load()
        self.desc = WsNetDesc(K, N, n, m, T, layers)
        self.count = self.L.lqgrid_wsnet_param_count(byref(self.desc))
        if self.count == 0:
            raise LqgridError(EINVAL, "lqgrid_wsnet_param_count")
        self.device = device
        self.feat_bytes = self.L.lqgrid_wsnet_sample_bytes(byref(self.desc), 0)
        self.tgt_bytes = self.L.lqgrid_wsnet_sample_bytes(byref(self.desc), 1)
        if params is None:
            params = self.init_params(seed)
        self.params = torch.as_tensor(np.asarray(params, dtype=np.float32)).to(device).contiguous()
        self.moments = torch.zeros(2 * self.count, dtype=torch.float32, device=device)
        self.step = 0
        self._ws = {}

    def layer_shapes(self):
        """[(W shape (64, 3, 3, cin), b shape (64,))] per layer."""
        return [((64, 3, 3, 32 if l == 0 else 64), (64,)) for l in range(self.desc.layers)]

    def init_params(self, seed):
        """He-normal weights (fan-in of the real input channels), zero biases;
        the last layer scaled by 0.1 so that the first predictions are small."""
        import numpy as np
        rng = np.random.default_rng(seed)
        d = self.desc
        cin_real = d.n + d.n * d.n + d.n * d.m
        out = []
        for l, (ws, bs) in enumerate(self.layer_shapes()):
            fan = 9 * (cin_real if l == 0 else 64)
            W = rng.standard_normal(ws) * np.sqrt(2.0 / fan)
            if l == 0:
                W[..., cin_real:] = 0.0
            if l == d.layers - 1:
                W *= 0.1
            out += [W.ravel(), np.zeros(bs)]
        return np.concatenate(out).astype(np.float32)

    def unflatten(self, flat):
        """List of (W, b) numpy arrays from a flat parameter vector."""
        import numpy as np
        flat = np.asarray(flat, dtype=np.float64)
        out, off = [], 0
        for ws, bs in self.layer_shapes():
            nw = int(np.prod(ws))
            out.append((flat[off:off + nw].reshape(ws), flat[off + nw:off + nw + 64].copy()))
            off += nw + 64
        return out

    def workspace(self, batch):
        import torch
        if batch not in self._ws:
            nb = self.L.lqgrid_wsnet_workspace_bytes(byref(self.desc), batch)
            t = torch.empty(nb + 256, dtype=torch.uint8, device=self.device)
            self._ws[batch] = (t, (t.data_ptr() + 255) // 256 * 256, nb)
        return self._ws[batch][1:]

    def alloc_features(self, count):
        import torch
        return torch.empty((count, self.feat_bytes // 2), dtype=torch.bfloat16,
                           device=self.device)

    def alloc_targets(self, count):
        import torch
        return torch.empty((count, self.tgt_bytes // 4), dtype=torch.float32,
                           device=self.device)

    def features(self, desc: ProblemDesc, x0, out):
        """Write the features of one problem (device arrays in desc) into the
        sample tensor `out` (a row of alloc_features)."""
        st = self.L.lqgrid_wsnet_features(byref(self.desc), byref(desc), _ptr(x0),
                                          _ptr(out), _stream())
        if st != OK:
            raise LqgridError(st, "lqgrid_wsnet_features")

    def targets(self, delta, out):
        wp, nb = self.workspace(1)
        st = self.L.lqgrid_wsnet_targets(byref(self.desc), _ptr(delta), _ptr(out),
                                         c_void_p(wp), nb, _stream())
        if st != OK:
            raise LqgridError(st, "lqgrid_wsnet_targets")

    def forward(self, feats, index=None, params=None):
        import torch
        batch = feats.shape[0] if index is None else index.numel()
        wp, nb = self.workspace(batch)
        P = self.desc.K * self.desc.N
        out = torch.empty((batch, P, 64), dtype=torch.float32, device=self.device)
        p = self.params if params is None else params
        st = self.L.lqgrid_wsnet_forward(byref(self.desc), batch, _ptr(feats), _ptr(index),
                                         _ptr(p), _ptr(out), c_void_p(wp), nb, _stream())
        if st != OK:
            raise LqgridError(st, "lqgrid_wsnet_forward")
        return out

    def gradient(self, feats, tgts, index, grad=None, params=None):
        """(loss, grad) of the batch index (device int32 tensor)."""
        import torch
        batch = index.numel()
        wp, nb = self.workspace(batch)
        if grad is None:
            grad = torch.empty(self.count, dtype=torch.float32, device=self.device)
        p = self.params if params is None else params
        loss = c_double()
        st = self.L.lqgrid_wsnet_gradient(byref(self.desc), batch, _ptr(feats), _ptr(tgts),
                                          _ptr(index), _ptr(p), _ptr(grad), byref(loss),
                                          c_void_p(wp), nb, _stream())
        if st != OK:
            raise LqgridError(st, "lqgrid_wsnet_gradient")
        return loss.value, grad

    def backward(self, feats, index, dout, grad=None, params=None):
        """Parameter gradient for a given output gradient dout
        ([batch][K N][64] FP32 device tensor)."""
        import torch
        batch = index.numel()
        wp, nb = self.workspace(batch)
        if grad is None:
            grad = torch.empty(self.count, dtype=torch.float32, device=self.device)
        p = self.params if params is None else params
        st = self.L.lqgrid_wsnet_backward(byref(self.desc), batch, _ptr(feats), _ptr(index),
                                          _ptr(p), _ptr(dout), _ptr(grad), c_void_p(wp), nb,
                                          _stream())
        if st != OK:
            raise LqgridError(st, "lqgrid_wsnet_backward")
        return grad

    def adam(self, grad, lr):
        self.step += 1
        st = self.L.lqgrid_wsnet_adam(byref(self.desc), _ptr(self.params), _ptr(grad),
                                      _ptr(self.moments), self.step, lr, _stream())
        if st != OK:
            raise LqgridError(st, "lqgrid_wsnet_adam")

    def predict(self, feat, out=None):
        """delta_init [T+1][N][K][n] (FP64) for one problem's features."""
        import torch
        d = self.desc
        wp, nb = self.workspace(1)
        if out is None:
            out = torch.empty((d.T + 1, d.N, d.K, d.n), dtype=torch.float64,
                              device=self.device)
        st = self.L.lqgrid_wsnet_predict(byref(self.desc), _ptr(feat), _ptr(self.params),
                                         _ptr(out), c_void_p(wp), nb, _stream())
        if st != OK:
            raise LqgridError(st, "lqgrid_wsnet_predict")
        return out

    def save(self, path):
        import numpy as np
        d = self.desc
        np.savez(path, params=self.params.cpu().numpy(),
                 dims=np.array([d.K, d.N, d.n, d.m, d.T, d.layers]))

    @classmethod
    def load_file(cls, path, device="cuda"):
        import numpy as np
        z = np.load(path)
        K, N, n, m, T, layers = (int(v) for v in z["dims"])
        return cls(K, N, n, m, T, layers, device=device, params=z["params"])
