"""Python face of the C ABI: a Plan holding the resident level hierarchy.

Tensors are torch float64 (float32 for the float32 diagnostic passes) CUDA
tensors of shape (N+1, N+1, N+1) (two-dimensional plans: (N+1, N+1)),
C-contiguous, on the plan's device.  Every
array argument is checked on the host (shape, dtype, device, layout) before
anything is launched; PyTorch only supplies device memory and the stream.
"""
import ctypes as C
from dataclasses import dataclass

import torch

from . import _abi

_PREC = {"fp64": _abi.DMGS_FP64, "fp32-in-fp64": _abi.DMGS_FP32_IN_FP64, "mixed": _abi.DMGS_FP32_IN_FP64}
_FACE = {"arith": _abi.DMGS_FACE_ARITH, "harmonic": _abi.DMGS_FACE_HARMONIC}
_SMOOTHER = {"rbgs": _abi.DMGS_RBGS, "wjacobi": _abi.DMGS_WJACOBI}


@dataclass
class Options:
    N: int
    precision: str = "fp64"          # "fp64" | "fp32-in-fp64"
    rtol: float = 1e-10
    max_cycles: int = 200
    fixed_cycles: int = 0
    nu_pre: int = 2
    nu_post: int = 2
    face_mean: str = "arith"
    h: float = 1.0
    bc_value: float = 0.0
    ir_inner_cycles: int = 8          # float32 V-cycles per refinement step (the most, when adaptive)
    ir_adaptive: bool = True          # later steps run the V-cycles the observed contraction predicts
    smoother: str = "rbgs"            # "rbgs" (red-black Gauss-Seidel) | "wjacobi" (weighted Jacobi, 6/7)
    adjoint_schedule: bool = False    # pull-back repeats the last forward solve's V-cycle schedule
    ndim: int = 3                     # 3: (N+1)^3 grids, 7-point operator; 2: (N+1)^2 grids, 5-point operator
    shape: tuple = None               # 3D: cells per axis (nx, ny, nz) of a general grid (default (N, N, N))
    spacing: tuple = None             # 3D: spacing per axis (hx, hy, hz) (default h on every axis)

    def to_c(self):
        o = _abi.default_options(self.N)
        o.precision = _PREC[self.precision]
        o.rtol = float(self.rtol)
        o.max_cycles = int(self.max_cycles)
        o.fixed_cycles = int(self.fixed_cycles)
        o.nu_pre, o.nu_post = int(self.nu_pre), int(self.nu_post)
        o.face_mean = _FACE[self.face_mean]
        o.h, o.bc_value = float(self.h), float(self.bc_value)
        o.ir_inner_cycles = int(self.ir_inner_cycles)
        o.ir_adaptive = 1 if self.ir_adaptive else 0
        o.smoother = _SMOOTHER[self.smoother]
        o.adjoint_schedule = 1 if self.adjoint_schedule else 0
        o.ndim = int(self.ndim)
        if self.shape is not None:
            o.n[0], o.n[1], o.n[2] = (int(c) for c in self.shape)
        if self.spacing is not None:
            o.h_axis[0], o.h_axis[1], o.h_axis[2] = (float(v) for v in self.spacing)
        return o

    @property
    def cells(self):
        """Cells per axis of the finest level."""
        if self.shape is not None:
            return tuple(int(c) for c in self.shape)
        return (self.N,) * self.ndim


def workspace_bytes(opts: Options, forward_vjp=False) -> int:
    """Device bytes of a plan; forward_vjp: including the second work set
    that Plan.forward_vjp allocates on first use."""
    o = opts.to_c()
    f = _abi.lib().dmgs_forward_vjp_workspace_bytes if forward_vjp else _abi.lib().dmgs_workspace_bytes
    return int(f(C.byref(o)))


def stream_copy(src, dst):
    """Library's plain streaming copy src -> dst (same-size CUDA tensors);
    returns the event-timed milliseconds."""
    import torch
    assert src.is_cuda and dst.is_cuda and src.nbytes == dst.nbytes and src.is_contiguous() and dst.is_contiguous()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    st = _abi.lib().dmgs_debug_stream_copy(C.c_void_p(src.data_ptr()), C.c_void_p(dst.data_ptr()), src.nbytes,
                                           _stream(src.device))
    e1.record()
    if st != _abi.DMGS_OK:
        raise _abi.DMGSError(st, "dmgs_debug_stream_copy")
    e1.synchronize()
    return e0.elapsed_time(e1)


def _stream(device):
    return C.c_void_p(torch.cuda.current_stream(device).cuda_stream)


def _solve_once(fn, where, opts: Options, D, mua, q, out=None, check=True):
    shape = tuple(c + 1 for c in opts.cells)
    dev = q.device
    for name, t in (("D", D), ("mua", mua), ("q", q)) + ((("out", out),) if out is not None else ()):
        if (not isinstance(t, torch.Tensor) or t.dtype != torch.float64 or t.device != dev or not t.is_cuda
                or tuple(t.shape) != shape or not t.is_contiguous()):
            raise ValueError("%s must be a contiguous float64 CUDA tensor of shape %s on %s" % (name, shape, dev))
    rho = torch.empty(shape, dtype=torch.float64, device=dev) if out is None else out
    o = opts.to_c()
    info = _abi.Info()
    with torch.cuda.device(dev):
        st = fn(C.byref(o), C.c_void_p(D.data_ptr()), C.c_void_p(mua.data_ptr()), C.c_void_p(q.data_ptr()),
                C.c_void_p(rho.data_ptr()), C.byref(info), _stream(dev))
    if check and st != _abi.DMGS_OK:
        raise _abi.DMGSError(st, where, info.as_dict())
    return rho, dict(info.as_dict(), status=st)


def solve_once(opts: Options, D, mua, q, out=None, check=True):
    """dmgs_solve_once: a plan created, used for one forward solve and
    destroyed."""
    return _solve_once(_abi.lib().dmgs_solve_once, "dmgs_solve_once", opts, D, mua, q, out, check)


def solve_once_noalloc(opts: Options, D, mua, q, out=None, check=True):
    """dmgs_solve_once_noalloc: the same solve in the library's static scratch
    array, with no device allocation (pass `out` to allocate nothing here
    either)."""
    return _solve_once(_abi.lib().dmgs_solve_once_noalloc, "dmgs_solve_once_noalloc", opts, D, mua, q, out, check)


class Plan:
    def __init__(self, opts: Options, device=None):
        self.opts = opts
        self.N = opts.N
        self.device = torch.device("cuda", torch.cuda.current_device() if device is None else torch.device(device).index or 0)
        self._c = opts.to_c()
        self._h = C.c_void_p()
        with torch.cuda.device(self.device):
            st = _abi.lib().dmgs_plan_create(C.byref(self._c), C.byref(self._h))
        if st != _abi.DMGS_OK:
            raise _abi.DMGSError(st, "dmgs_plan_create")
        self.levels = _abi.lib().dmgs_plan_levels(self._h)
        self.level_N = [_abi.lib().dmgs_plan_level_n(self._h, k) for k in range(self.levels)]
        self.level_shape = []
        for k in range(self.levels):
            n3 = (C.c_int32 * 3)()
            _abi.lib().dmgs_plan_level_shape(self._h, k, n3)
            self.level_shape.append(tuple(int(n3[a]) for a in range(opts.ndim)))
        self.bytes = workspace_bytes(opts)

    def close(self):
        if getattr(self, "_h", None) and self._h.value:
            _abi.lib().dmgs_plan_destroy(self._h)
            self._h = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # ---- argument checks ------------------------------------------------------------
    def _shape(self, k=0):
        return tuple(c + 1 for c in self.level_shape[k])

    def _arr(self, t, name, k=0, dtype=torch.float64, optional=False):
        if t is None:
            if optional:
                return None
            raise ValueError("%s is required" % name)
        if not isinstance(t, torch.Tensor):
            raise TypeError("%s must be a torch tensor" % name)
        if t.dtype != dtype or t.device != self.device or tuple(t.shape) != self._shape(k) or not t.is_contiguous():
            raise ValueError("%s must be a contiguous %s tensor of shape %s on %s (got %s %s %s)"
                             % (name, dtype, self._shape(k), self.device, t.dtype, tuple(t.shape), t.device))
        return C.c_void_p(t.data_ptr())

    def _empty(self, k=0, dtype=torch.float64):
        return torch.empty(self._shape(k), dtype=dtype, device=self.device)

    def _call(self, fn, where, *args, info=None, check=True):
        with torch.cuda.device(self.device):
            st = fn(self._h, *args)
        if check and st != _abi.DMGS_OK:
            raise _abi.DMGSError(st, where, info.as_dict() if info is not None else None)
        return st

    # ---- solver ---------------------------------------------------------------------
    def set_coefficients(self, D, mua):
        self._call(_abi.lib().dmgs_set_coefficients, "dmgs_set_coefficients", self._arr(D, "D"),
                   self._arr(mua, "mua"), _stream(self.device))

    def set_log_coefficients(self, logD, logmua):
        self._call(_abi.lib().dmgs_set_log_coefficients, "dmgs_set_log_coefficients", self._arr(logD, "logD"),
                   self._arr(logmua, "logmua"), _stream(self.device))

    def forward(self, q, out=None, check=True):
        rho = self._empty() if out is None else out
        info = _abi.Info()
        self._call(_abi.lib().dmgs_forward, "dmgs_forward", self._arr(q, "q"), self._arr(rho, "rho"),
                   C.byref(info), _stream(self.device), info=info, check=check)
        return rho, info.as_dict()

    def jvp(self, rho, dq=None, dlogD=None, dlogmua=None, out=None, check=True):
        drho = self._empty() if out is None else out
        info = _abi.Info()
        self._call(_abi.lib().dmgs_jvp, "dmgs_jvp", self._arr(rho, "rho"), self._arr(dq, "dq", optional=True),
                   self._arr(dlogD, "dlogD", optional=True), self._arr(dlogmua, "dlogmua", optional=True),
                   self._arr(drho, "drho"), C.byref(info), _stream(self.device), info=info, check=check)
        return drho, info.as_dict()

    def vjp(self, rho, rhobar, coef_grads=True, out=None, check=True):
        if out is None:
            qbar = self._empty()
            gD = self._empty() if coef_grads else None
            gmu = self._empty() if coef_grads else None
        else:
            qbar, gD, gmu = out
        info = _abi.Info()
        self._call(_abi.lib().dmgs_vjp, "dmgs_vjp", self._arr(rho, "rho"), self._arr(rhobar, "rhobar"),
                   self._arr(qbar, "qbar"), self._arr(gD, "logD_bar", optional=True),
                   self._arr(gmu, "logmua_bar", optional=True), C.byref(info), _stream(self.device),
                   info=info, check=check)
        return (qbar, gD, gmu), info.as_dict()

    def vjp_unrolled(self, q, rhobar, coef_grads=True):
        """rho = S_n q and the exact derivative of the n-cycle map pulled back
        from rhobar: (rho, (qbar, logD_bar, logmua_bar)), info
        (dmgs_vjp_unrolled; fixed-cycle float64 3D plans)."""
        rho, qbar = self._empty(), self._empty()
        gD = self._empty() if coef_grads else None
        gmu = self._empty() if coef_grads else None
        info = _abi.Info()
        self._call(_abi.lib().dmgs_vjp_unrolled, "dmgs_vjp_unrolled", self._arr(q, "q"), self._arr(rhobar, "rhobar"),
                   self._arr(rho, "rho"), self._arr(qbar, "qbar"), self._arr(gD, "logD_bar", optional=True),
                   self._arr(gmu, "logmua_bar", optional=True), C.byref(info), _stream(self.device), info=info)
        return (rho, (qbar, gD, gmu)), info.as_dict()

    def noise_weights(self, Le, mask, rel=0.05, floor=0.01):
        """Inverse noise variances of the noise model with the edge mask
        (dmgs_noise_weights)."""
        w = self._empty()
        self._call(_abi.lib().dmgs_noise_weights, "dmgs_noise_weights", self._arr(Le, "Le"), int(mask), float(rel),
                   float(floor), self._arr(w, "w"), _stream(self.device))
        return w

    def likelihood_grad(self, q, d, w, coef_grads=True, check=True):
        """rho = S q, {"H", "chi2", "nvox"} and (qbar, logD_bar, logmua_bar)
        = the gradient of H (dmgs_likelihood_grad).  Returns (rho, value,
        grads), info_fwd, info_vjp."""
        rho, qbar = self._empty(), self._empty()
        gD = self._empty() if coef_grads else None
        gmu = self._empty() if coef_grads else None
        value = (C.c_double * 3)()
        info_f, info_a = _abi.Info(), _abi.Info()
        st = self._call(_abi.lib().dmgs_likelihood_grad, "dmgs_likelihood_grad", self._arr(q, "q"), self._arr(d, "d"),
                        self._arr(w, "w"), self._arr(rho, "rho"), self._arr(qbar, "qbar"),
                        self._arr(gD, "logD_bar", optional=True), self._arr(gmu, "logmua_bar", optional=True),
                        value, C.byref(info_f), C.byref(info_a), _stream(self.device), check=False)
        if check and st != _abi.DMGS_OK:
            bad = info_f if info_f.status != _abi.DMGS_OK else info_a
            raise _abi.DMGSError(st, "dmgs_likelihood_grad", bad.as_dict())
        val = {"H": value[0], "chi2": value[1], "nvox": int(value[2])}
        return (rho, val, (qbar, gD, gmu)), info_f.as_dict(), info_a.as_dict()

    def forward_vjp(self, q, rhobar, coef_grads=True, out=None, check=True):
        """rho = S q and the VJP at rho with cotangent rhobar, the two solves
        running concurrently (dmgs_forward_vjp).  Returns (rho, (qbar,
        logD_bar, logmua_bar)), info_fwd, info_vjp."""
        if out is None:
            rho, qbar = self._empty(), self._empty()
            gD = self._empty() if coef_grads else None
            gmu = self._empty() if coef_grads else None
        else:
            rho, qbar, gD, gmu = out
        info_f, info_a = _abi.Info(), _abi.Info()
        st = self._call(_abi.lib().dmgs_forward_vjp, "dmgs_forward_vjp", self._arr(q, "q"),
                        self._arr(rhobar, "rhobar"), self._arr(rho, "rho"), self._arr(qbar, "qbar"),
                        self._arr(gD, "logD_bar", optional=True), self._arr(gmu, "logmua_bar", optional=True),
                        C.byref(info_f), C.byref(info_a), _stream(self.device), check=False)
        if check and st != _abi.DMGS_OK:
            bad = info_f if info_f.status != _abi.DMGS_OK else info_a
            raise _abi.DMGSError(st, "dmgs_forward_vjp", bad.as_dict())
        return (rho, (qbar, gD, gmu)), info_f.as_dict(), info_a.as_dict()

    # ---- kernel timing ----------------------------------------------------------------
    def timing(self, enable=True, stride=1):
        """Enable (and reset) or disable per-class timing of finest-level
        launches; stride n times one launch in n of each class (totals are
        scaled to all launches)."""
        self._call(_abi.lib().dmgs_timing_enable, "dmgs_timing_enable", max(1, int(stride)) if enable else 0)

    def trace(self, order=0):
        """Residual history of the last solve of this cycle order (0: forward
        or push-forward, 1: pull-back) as [(cycles, vcycles, rel_residual)];
        the plan must have been created with DMGS_TRACE=1."""
        count = C.c_int32(0)
        self._call(_abi.lib().dmgs_trace_read, "dmgs_trace_read", int(order), 0, None, None, None, C.byref(count))
        n = count.value
        steps, vc, rel = (C.c_int32 * max(n, 1))(), (C.c_int32 * max(n, 1))(), (C.c_double * max(n, 1))()
        self._call(_abi.lib().dmgs_trace_read, "dmgs_trace_read", int(order), n, steps, vc, rel, C.byref(count))
        return [(steps[i], vc[i], rel[i]) for i in range(n)]

    def timing_read(self):
        """{class: {"launches", "ms", "bytes"}} accumulated since timing was enabled."""
        out = {}
        for c, name in enumerate(_abi.KERNEL_CLASSES):
            n, ms, b = C.c_int64(0), C.c_double(0.0), C.c_double(0.0)
            self._call(_abi.lib().dmgs_timing_read, "dmgs_timing_read", c, C.byref(n), C.byref(ms), C.byref(b))
            out[name] = {"launches": n.value, "ms": ms.value, "bytes": b.value}
        return out

    # ---- diagnostic passes (parity tests) -------------------------------------------
    def debug_apply(self, k, u, fp32=False):
        dt = torch.float32 if fp32 else torch.float64
        out = self._empty(k, dt)
        self._call(_abi.lib().dmgs_debug_apply, "dmgs_debug_apply", int(k), int(fp32), self._arr(u, "u", k, dt),
                   self._arr(out, "out", k, dt), _stream(self.device))
        return out

    def debug_level_coefficients(self, k):
        D, mu = self._empty(k), self._empty(k)
        self._call(_abi.lib().dmgs_debug_level_coefficients, "dmgs_debug_level_coefficients", int(k),
                   self._arr(D, "D", k), self._arr(mu, "mua", k), _stream(self.device))
        return D, mu

    def debug_pre(self, k, u_in, q, order=0, fp32=False):
        dt = torch.float32 if fp32 else torch.float64
        u_out, qc = self._empty(k, dt), self._empty(k + 1, dt)
        uin = None if u_in is None else self._arr(u_in, "u_in", k, dt)   # None: start from zero
        self._call(_abi.lib().dmgs_debug_pre, "dmgs_debug_pre", int(k), int(fp32), int(order),
                   uin, self._arr(q, "q", k, dt), self._arr(u_out, "u_out", k, dt),
                   self._arr(qc, "qc", k + 1, dt), _stream(self.device))
        return u_out, qc

    def debug_post(self, k, u_in, ec, q, order=0, fp32=False):
        dt = torch.float32 if fp32 else torch.float64
        u_out = self._empty(k, dt)
        self._call(_abi.lib().dmgs_debug_post, "dmgs_debug_post", int(k), int(fp32), int(order),
                   self._arr(u_in, "u_in", k, dt), self._arr(ec, "ec", k + 1, dt), self._arr(q, "q", k, dt),
                   self._arr(u_out, "u_out", k, dt), _stream(self.device))
        return u_out

    def debug_coarsest(self, q, fp32=False):
        k = self.levels - 1
        dt = torch.float32 if fp32 else torch.float64
        u = self._empty(k, dt)
        self._call(_abi.lib().dmgs_debug_coarsest, "dmgs_debug_coarsest", int(fp32), self._arr(q, "q", k, dt),
                   self._arr(u, "u", k, dt), _stream(self.device))
        return u

    def debug_cycles(self, q, u, ncycles, order=0):
        u = u.clone()
        self._call(_abi.lib().dmgs_debug_cycles, "dmgs_debug_cycles", int(order), int(ncycles),
                   self._arr(q, "q"), self._arr(u, "u"), _stream(self.device))
        return u


class Batch:
    """Grouped execution of forward + push-forward / pull-back requests
    (dmgs_batch_*): each tick() advances every active request by one
    refinement step in grouped launches and synchronises the stream once.

    add(plan, mode, q, ...) enqueues a request on a plan that serves no other
    request of the batch; tick() returns the requests that finished, as
    dicts with the request's tag, status, infos and output tensors.  The
    batch keeps every request's tensors alive until it is reported.  Results
    are bitwise those of Plan.forward followed by Plan.jvp / Plan.vjp."""

    def __init__(self, device=None):
        self.device = torch.device("cuda", torch.cuda.current_device() if device is None else torch.device(device).index or 0)
        self._h = C.c_void_p()
        with torch.cuda.device(self.device):
            st = _abi.lib().dmgs_batch_create(C.byref(self._h))
        if st != _abi.DMGS_OK:
            raise _abi.DMGSError(st, "dmgs_batch_create")
        self._live = {}
        self._next_tag = 0

    def close(self):
        if getattr(self, "_h", None) and self._h.value:
            _abi.lib().dmgs_batch_destroy(self._h)
            self._h = C.c_void_p()
        self._live = {}

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def add(self, plan, mode, q, dq=None, dlogD=None, dlogmua=None, rhobar=None, coef_grads=True, tag=None):
        """mode "jvp": rho = S q and drho = S(dq - A' rho); mode "vjp": rho = S q,
        qbar = S^T rhobar and, with coef_grads, the log-coefficient gradients."""
        if plan.device != self.device:
            raise ValueError("the plan lives on another device")
        tag = self._next_tag if tag is None else int(tag)
        self._next_tag = max(self._next_tag, tag) + 1
        rho = plan._empty()
        out = {"rho": rho}
        if mode == "jvp":
            out["drho"] = plan._empty()
            ins = (plan._arr(dq, "dq", optional=True), plan._arr(dlogD, "dlogD", optional=True),
                   plan._arr(dlogmua, "dlogmua", optional=True))
            outs = (plan._arr(out["drho"], "drho"), None, None)
            m = _abi.DMGS_BATCH_JVP
        elif mode == "vjp":
            out["qbar"] = plan._empty()
            if coef_grads:
                out["logD_bar"], out["logmua_bar"] = plan._empty(), plan._empty()
            ins = (plan._arr(rhobar, "rhobar"), None, None)
            outs = (plan._arr(out["qbar"], "qbar"), plan._arr(out.get("logD_bar"), "logD_bar", optional=True),
                    plan._arr(out.get("logmua_bar"), "logmua_bar", optional=True))
            m = _abi.DMGS_BATCH_VJP
        else:
            raise ValueError("mode must be 'jvp' or 'vjp'")
        with torch.cuda.device(self.device):
            st = _abi.lib().dmgs_batch_add(self._h, plan._h, m, plan._arr(q, "q"), *ins, plan._arr(rho, "rho"), *outs,
                                           C.c_int64(tag))
        if st != _abi.DMGS_OK:
            raise _abi.DMGSError(st, "dmgs_batch_add")
        # inputs and outputs stay referenced until the request is reported
        self._live[tag] = {"plan": plan, "mode": mode, "keep": (q, dq, dlogD, dlogmua, rhobar), "out": out}
        return tag

    def pending(self):
        return _abi.lib().dmgs_batch_pending(self._h)

    def tick(self, stream=None):
        n = max(1, len(self._live))
        tags = (C.c_int64 * n)()
        status = (C.c_int32 * n)()
        inf = (_abi.Info * n)()
        ins = (_abi.Info * n)()
        count = C.c_int32(0)
        st_ptr = _stream(self.device) if stream is None else C.c_void_p(stream.cuda_stream)
        with torch.cuda.device(self.device):
            st = _abi.lib().dmgs_batch_tick(self._h, st_ptr, n, tags, status, inf, ins, C.byref(count))
        if st != _abi.DMGS_OK:
            raise _abi.DMGSError(st, "dmgs_batch_tick")
        done = []
        for i in range(count.value):
            rec = self._live.pop(int(tags[i]))
            done.append({"tag": int(tags[i]), "status": int(status[i]), "info_fwd": inf[i].as_dict(),
                         "info_second": ins[i].as_dict(), "mode": rec["mode"], **rec["out"]})
        return done

    def stats(self):
        t, l, r = C.c_int64(), C.c_int64(), C.c_int64()
        _abi.lib().dmgs_batch_stats(self._h, C.byref(t), C.byref(l), C.byref(r))
        return {"ticks": t.value, "launches": l.value, "recorded": r.value}

    def run(self, stream=None):
        """Tick until every request has been reported; returns them all."""
        out = []
        while self.pending():
            out.extend(self.tick(stream))
        return out
