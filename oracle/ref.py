"""ctypes view of the FP64 CPU oracle (oracle/dmgs_ref.c).

TEST INFRASTRUCTURE ONLY: the checker that the GPU library is compared
against.  Only tests/, the smoke entry point and the CPU-baseline leg of the
benchmark import this module; the GPU library never does.

All arrays are float64 numpy arrays of shape (N+1, N+1, N+1), x slowest, z
fastest.  Status codes: 0 ok, 1 invalid, 2 out of memory, 3 not converged,
4 non-finite.
"""
import ctypes as C
import os

import numpy as np

from . import build_oracle

_lib = None
_DP = C.POINTER(C.c_double)


def lib():
    global _lib
    if _lib is None:
        path = build_oracle.build(force=False)
        L = C.CDLL(path)
        vp, i, d = C.c_void_p, C.c_int, C.c_double
        ip = C.POINTER(C.c_int)
        sig = {
            "ref_num_levels_for": (i, [i]),
            "ref_hier_create": (vp, [i, d, d, i, _DP, _DP, ip]),
            "ref_hier_destroy": (None, [vp]),
            "ref_levels": (i, [vp]),
            "ref_level_N": (i, [vp, i]),
            "ref_level_coef": (None, [vp, i, _DP, _DP]),
            "ref_coarsen_field": (None, [i, _DP, _DP]),
            "ref_apply": (None, [vp, i, _DP, _DP]),
            "ref_gs_half": (None, [vp, i, i, _DP, _DP]),
            "ref_defect": (None, [vp, i, _DP, _DP, _DP]),
            "ref_restrict": (None, [i, _DP, _DP]),
            "ref_prolong_add": (None, [i, _DP, _DP]),
            "ref_exact_solve": (i, [vp, i, _DP, _DP]),
            "ref_exact_solve_adj": (i, [vp, i, _DP, _DP]),
            "ref_cycles": (None, [vp, _DP, _DP, i, i, i, i]),
            "ref_gs_half_adj": (None, [vp, i, i, _DP, _DP]),
            "ref_defect_adj": (None, [vp, i, _DP, _DP, _DP]),
            "ref_tangent_rhs": (None, [vp, _DP, _DP, _DP, _DP, _DP]),
            "ref_coef_grads": (None, [vp, _DP, _DP, _DP, _DP]),
            "ref_forward": (i, [vp, _DP, _DP, i, i, d, i, i, ip, _DP]),
            "ref_forward_history": (i, [vp, _DP, _DP, i, i, d, i, ip, _DP, _DP]),
            "ref_jvp": (i, [vp, _DP, _DP, _DP, _DP, _DP, i, i, d, i, i, ip, _DP]),
            "ref_vjp": (i, [vp, _DP, _DP, _DP, _DP, _DP, i, i, d, i, i, ip, _DP]),
            "ref_pullback_br": (i, [vp, _DP, _DP, i, i, d, i, i, ip, _DP]),
            "ref_set_smoother": (None, [vp, i, d]),
            "ref_wj_sweep": (None, [vp, i, _DP, _DP]),
            "ref_wj_sweep_adj": (None, [vp, i, _DP, _DP]),
        }
        for name, (res, args) in sig.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def _p(a):
    if a is None:
        return None
    assert a.dtype == np.float64 and a.flags["C_CONTIGUOUS"], "oracle arrays are C-contiguous float64"
    return a.ctypes.data_as(_DP)


def num_levels(N):
    return lib().ref_num_levels_for(int(N))


class OracleError(RuntimeError):
    def __init__(self, status, what):
        super().__init__("%s: oracle status %d" % (what, status))
        self.status = status


class Hierarchy:
    """Coefficient hierarchy of rediscretised operators on all levels."""

    def __init__(self, D, mua, h=1.0, bc=0.0, face_mean="arith", smoother="rbgs", omega=6.0 / 7.0):
        D = np.ascontiguousarray(D, dtype=np.float64)
        mua = np.ascontiguousarray(mua, dtype=np.float64)
        assert D.ndim == 3 and D.shape[0] == D.shape[1] == D.shape[2] and D.shape == mua.shape
        self.N = D.shape[0] - 1
        self.h, self.bc = float(h), float(bc)
        self.face_mean = face_mean
        st = C.c_int(0)
        self._h = lib().ref_hier_create(self.N, self.h, self.bc, 1 if face_mean == "harmonic" else 0,
                                        _p(D), _p(mua), C.byref(st))
        if not self._h:
            raise OracleError(st.value, "ref_hier_create")
        self.L = lib().ref_levels(self._h)
        self.Ns = [lib().ref_level_N(self._h, k) for k in range(self.L)]
        assert smoother in ("rbgs", "wjacobi")
        self.smoother, self.omega = smoother, float(omega)
        lib().ref_set_smoother(self._h, 1 if smoother == "wjacobi" else 0, self.omega)

    def __del__(self):
        if getattr(self, "_h", None):
            lib().ref_hier_destroy(self._h)
            self._h = None

    def zeros(self, k=0):
        n = self.Ns[k] + 1
        return np.zeros((n, n, n))

    def level_coef(self, k):
        D, mu = self.zeros(k), self.zeros(k)
        lib().ref_level_coef(self._h, k, _p(D), _p(mu))
        return D, mu

    # ---- single steps on level k -------------------------------------------------
    def apply(self, k, u):
        out = self.zeros(k)
        lib().ref_apply(self._h, k, _p(np.ascontiguousarray(u, np.float64)), _p(out))
        return out

    def gs_half(self, k, colour, u, q):
        u = np.array(u, dtype=np.float64, copy=True)
        lib().ref_gs_half(self._h, k, int(colour), _p(u), _p(np.ascontiguousarray(q, np.float64)))
        return u

    def wj_sweep(self, k, u, q):
        u = np.array(u, dtype=np.float64, copy=True)
        lib().ref_wj_sweep(self._h, k, _p(u), _p(np.ascontiguousarray(q, np.float64)))
        return u

    def wj_sweep_adj(self, k, ubar, qbar):
        ubar = np.array(ubar, dtype=np.float64, copy=True)
        qbar = np.array(qbar, dtype=np.float64, copy=True)
        lib().ref_wj_sweep_adj(self._h, k, _p(ubar), _p(qbar))
        return ubar, qbar

    def defect(self, k, u, q):
        r = self.zeros(k)
        lib().ref_defect(self._h, k, _p(np.ascontiguousarray(u, np.float64)),
                         _p(np.ascontiguousarray(q, np.float64)), _p(r))
        return r

    def restrict(self, k, r):
        qc = self.zeros(k + 1)
        lib().ref_restrict(self.Ns[k], _p(np.ascontiguousarray(r, np.float64)), _p(qc))
        return qc

    def prolong_add(self, k, ec, u):
        u = np.array(u, dtype=np.float64, copy=True)
        lib().ref_prolong_add(self.Ns[k], _p(np.ascontiguousarray(ec, np.float64)), _p(u))
        return u

    def exact_solve(self, k, q, u=None):
        u = self.zeros(k) if u is None else np.array(u, dtype=np.float64, copy=True)
        st = lib().ref_exact_solve(self._h, k, _p(np.ascontiguousarray(q, np.float64)), _p(u))
        if st:
            raise OracleError(st, "ref_exact_solve")
        return u

    def gs_half_adj(self, k, colour, ubar, qbar):
        ubar = np.array(ubar, dtype=np.float64, copy=True)
        qbar = np.array(qbar, dtype=np.float64, copy=True)
        lib().ref_gs_half_adj(self._h, k, int(colour), _p(ubar), _p(qbar))
        return ubar, qbar

    def defect_adj(self, k, rbar, ubar, qbar):
        ubar = np.array(ubar, dtype=np.float64, copy=True)
        qbar = np.array(qbar, dtype=np.float64, copy=True)
        lib().ref_defect_adj(self._h, k, _p(np.ascontiguousarray(rbar, np.float64)), _p(ubar), _p(qbar))
        return ubar, qbar

    def cycles(self, q, u, n, order=0, nu1=2, nu2=2):
        u = np.array(u, dtype=np.float64, copy=True)
        lib().ref_cycles(self._h, _p(np.ascontiguousarray(q, np.float64)), _p(u), int(n), int(order),
                         int(nu1), int(nu2))
        return u

    # ---- solves -----------------------------------------------------------------
    def forward(self, q, rtol=1e-10, max_cycles=200, fixed_cycles=0, nu1=2, nu2=2, check=True):
        rho = self.zeros()
        cyc, rel = C.c_int(0), C.c_double(0.0)
        st = lib().ref_forward(self._h, _p(np.ascontiguousarray(q, np.float64)), _p(rho), nu1, nu2,
                               float(rtol), int(max_cycles), int(fixed_cycles), C.byref(cyc), C.byref(rel))
        if check and st:
            raise OracleError(st, "ref_forward")
        return rho, {"cycles": cyc.value, "rel_residual": rel.value, "status": st}

    def forward_history(self, q, rtol=1e-10, max_cycles=60, nu1=2, nu2=2):
        rho = self.zeros()
        hist = np.zeros(max_cycles)
        cyc, rel = C.c_int(0), C.c_double(0.0)
        st = lib().ref_forward_history(self._h, _p(np.ascontiguousarray(q, np.float64)), _p(rho), nu1, nu2,
                                       float(rtol), int(max_cycles), C.byref(cyc), C.byref(rel), _p(hist))
        return rho, hist[:cyc.value], st

    def jvp(self, rho, dq, dlogD=None, dlogmua=None, rtol=1e-10, max_cycles=200, fixed_cycles=0,
            nu1=2, nu2=2, check=True):
        z = self.zeros()
        dq = z if dq is None else np.ascontiguousarray(dq, np.float64)
        dlogD = z if dlogD is None else np.ascontiguousarray(dlogD, np.float64)
        dlogmua = z if dlogmua is None else np.ascontiguousarray(dlogmua, np.float64)
        drho = self.zeros()
        cyc, rel = C.c_int(0), C.c_double(0.0)
        st = lib().ref_jvp(self._h, _p(np.ascontiguousarray(rho, np.float64)), _p(dq), _p(dlogD), _p(dlogmua),
                           _p(drho), nu1, nu2, float(rtol), int(max_cycles), int(fixed_cycles),
                           C.byref(cyc), C.byref(rel))
        if check and st:
            raise OracleError(st, "ref_jvp")
        return drho, {"cycles": cyc.value, "rel_residual": rel.value, "status": st}

    def vjp(self, rho, rhobar, rtol=1e-10, max_cycles=200, fixed_cycles=0, nu1=2, nu2=2, check=True):
        qbar, gD, gmu = self.zeros(), self.zeros(), self.zeros()
        cyc, rel = C.c_int(0), C.c_double(0.0)
        st = lib().ref_vjp(self._h, _p(np.ascontiguousarray(rho, np.float64)),
                           _p(np.ascontiguousarray(rhobar, np.float64)), _p(qbar), _p(gD), _p(gmu),
                           nu1, nu2, float(rtol), int(max_cycles), int(fixed_cycles), C.byref(cyc), C.byref(rel))
        if check and st:
            raise OracleError(st, "ref_vjp")
        return (qbar, gD, gmu), {"cycles": cyc.value, "rel_residual": rel.value, "status": st}

    def pullback_br(self, rhobar, rtol=1e-10, max_cycles=200, fixed_cycles=0, nu1=2, nu2=2, check=True):
        qbar = self.zeros()
        cyc, rel = C.c_int(0), C.c_double(0.0)
        st = lib().ref_pullback_br(self._h, _p(np.ascontiguousarray(rhobar, np.float64)), _p(qbar), nu1, nu2,
                                   float(rtol), int(max_cycles), int(fixed_cycles), C.byref(cyc), C.byref(rel))
        if check and st:
            raise OracleError(st, "ref_pullback_br")
        return qbar, {"cycles": cyc.value, "rel_residual": rel.value, "status": st}

    def tangent_rhs(self, rho, dq, dlogD, dlogmua):
        out = self.zeros()
        lib().ref_tangent_rhs(self._h, *[_p(np.ascontiguousarray(a, np.float64)) for a in (rho, dq, dlogD, dlogmua)],
                              _p(out))
        return out

    def coef_grads(self, rho, qbar):
        gD, gmu = self.zeros(), self.zeros()
        lib().ref_coef_grads(self._h, _p(np.ascontiguousarray(rho, np.float64)),
                             _p(np.ascontiguousarray(qbar, np.float64)), _p(gD), _p(gmu))
        return gD, gmu


def coarsen_field(f):
    f = np.ascontiguousarray(f, np.float64)
    Nf = f.shape[0] - 1
    n = Nf // 2 + 1
    out = np.zeros((n, n, n))
    lib().ref_coarsen_field(Nf, _p(f), _p(out))
    return out
