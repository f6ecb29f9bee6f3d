"""ctypes binding of the C ABI in include/dmgs.h (argument marshalling only).

Loads paper_2608_00760_amd/csrc/libdmgs.so; there is no fallback: when the
library is missing every call raises.
"""
import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "csrc", "libdmgs.so")

DMGS_OK, DMGS_ERR_INVALID, DMGS_ERR_OOM, DMGS_ERR_NOT_CONVERGED = 0, 1, 2, 3
DMGS_ERR_NONFINITE, DMGS_ERR_HIP, DMGS_ERR_BUDGET = 4, 5, 6
DMGS_FP64, DMGS_FP32_IN_FP64 = 0, 1
DMGS_RBGS, DMGS_WJACOBI = 0, 1
DMGS_FACE_ARITH, DMGS_FACE_HARMONIC = 0, 1
DMGS_NOALLOC_SCRATCH_BYTES = 144 << 20


class Options(C.Structure):
    _fields_ = [("n", C.c_int32 * 3), ("precision", C.c_int32), ("smoother", C.c_int32),
                ("nu_pre", C.c_int32), ("nu_post", C.c_int32), ("max_cycles", C.c_int32),
                ("fixed_cycles", C.c_int32), ("face_mean", C.c_int32), ("h", C.c_double),
                ("bc_value", C.c_double), ("rtol", C.c_double), ("ir_inner_cycles", C.c_int32),
                ("ir_adaptive", C.c_int32), ("adjoint_schedule", C.c_int32), ("ndim", C.c_int32),
                ("h_axis", C.c_double * 3)]


class Info(C.Structure):
    _fields_ = [("cycles", C.c_int32), ("status", C.c_int32), ("rel_residual", C.c_double),
                ("device_ms", C.c_double), ("vcycles", C.c_int32), ("reserved", C.c_int32)]

    def as_dict(self):
        return {"cycles": self.cycles, "status": self.status, "rel_residual": self.rel_residual,
                "device_ms": self.device_ms, "vcycles": self.vcycles}


# name -> (restype, argtypes); the exported symbols of include/dmgs.h
_vp, _i, _d = C.c_void_p, C.c_int, C.c_double
SIGNATURES = {
    "dmgs_default_options": (None, [C.c_int32, C.POINTER(Options)]),
    "dmgs_workspace_bytes": (C.c_size_t, [C.POINTER(Options)]),
    "dmgs_forward_vjp_workspace_bytes": (C.c_size_t, [C.POINTER(Options)]),
    "dmgs_plan_create": (_i, [C.POINTER(Options), C.POINTER(_vp)]),
    "dmgs_plan_destroy": (_i, [_vp]),
    "dmgs_plan_levels": (_i, [_vp]),
    "dmgs_plan_level_n": (_i, [_vp, _i]),
    "dmgs_plan_level_shape": (_i, [_vp, _i, C.POINTER(C.c_int32)]),
    "dmgs_set_coefficients": (_i, [_vp, _vp, _vp, _vp]),
    "dmgs_set_log_coefficients": (_i, [_vp, _vp, _vp, _vp]),
    "dmgs_forward": (_i, [_vp, _vp, _vp, C.POINTER(Info), _vp]),
    "dmgs_jvp": (_i, [_vp, _vp, _vp, _vp, _vp, _vp, C.POINTER(Info), _vp]),
    "dmgs_vjp": (_i, [_vp, _vp, _vp, _vp, _vp, _vp, C.POINTER(Info), _vp]),
    "dmgs_forward_vjp": (_i, [_vp, _vp, _vp, _vp, _vp, _vp, _vp, C.POINTER(Info), C.POINTER(Info), _vp]),
    "dmgs_solve_once": (_i, [C.POINTER(Options), _vp, _vp, _vp, _vp, C.POINTER(Info), _vp]),
    "dmgs_solve_once_noalloc": (_i, [C.POINTER(Options), _vp, _vp, _vp, _vp, C.POINTER(Info), _vp]),
    "dmgs_noise_weights": (_i, [_vp, _vp, C.c_int32, C.c_double, C.c_double, _vp, _vp]),
    "dmgs_vjp_unrolled": (_i, [_vp, _vp, _vp, _vp, _vp, _vp, _vp, C.POINTER(Info), _vp]),
    "dmgs_likelihood_grad": (_i, [_vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp, C.POINTER(C.c_double), C.POINTER(Info),
                                  C.POINTER(Info), _vp]),
    "dmgs_status_string": (C.c_char_p, [_i]),
    "dmgs_last_error": (C.c_char_p, []),
    "dmgs_debug_apply": (_i, [_vp, _i, _i, _vp, _vp, _vp]),
    "dmgs_debug_level_coefficients": (_i, [_vp, _i, _vp, _vp, _vp]),
    "dmgs_debug_pre": (_i, [_vp, _i, _i, _i, _vp, _vp, _vp, _vp, _vp]),
    "dmgs_debug_post": (_i, [_vp, _i, _i, _i, _vp, _vp, _vp, _vp, _vp]),
    "dmgs_debug_coarsest": (_i, [_vp, _i, _vp, _vp, _vp]),
    "dmgs_debug_cycles": (_i, [_vp, _i, _i, _vp, _vp, _vp]),
    "dmgs_debug_stream_copy": (_i, [_vp, _vp, C.c_size_t, _vp]),
    "dmgs_timing_enable": (_i, [_vp, _i]),
    "dmgs_timing_read": (_i, [_vp, _i, C.POINTER(C.c_int64), C.POINTER(C.c_double), C.POINTER(C.c_double)]),
    "dmgs_trace_read": (_i, [_vp, C.c_int32, C.c_int32, C.POINTER(C.c_int32), C.POINTER(C.c_int32),
                             C.POINTER(C.c_double), C.POINTER(C.c_int32)]),
    "dmgs_batch_create": (_i, [C.POINTER(_vp)]),
    "dmgs_batch_destroy": (_i, [_vp]),
    "dmgs_batch_add": (_i, [_vp, _vp, C.c_int32, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp, C.c_int64]),
    "dmgs_batch_pending": (_i, [_vp]),
    "dmgs_batch_tick": (_i, [_vp, _vp, C.c_int32, C.POINTER(C.c_int64), C.POINTER(C.c_int32), C.POINTER(Info),
                             C.POINTER(Info), C.POINTER(C.c_int32)]),
    "dmgs_batch_stats": (_i, [_vp, C.POINTER(C.c_int64), C.POINTER(C.c_int64), C.POINTER(C.c_int64)]),
}

DMGS_BATCH_JVP, DMGS_BATCH_VJP = 0, 1

KERNEL_CLASSES = ["smooth", "defect_restrict", "prolong", "residual", "update", "coef", "grad"]

_lib = None


class DMGSError(RuntimeError):
    def __init__(self, status, where, info=None):
        msg = "%s failed: %s (%d): %s" % (where, status_string(status), status, last_error())
        super().__init__(msg)
        self.status = status
        self.info = info


def lib():
    """The loaded HIP library; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError("HIP library %s is not built (run __graft_entry__.build())" % LIB_PATH)
        L = C.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def status_string(s):
    return lib().dmgs_status_string(int(s)).decode()


def last_error():
    return lib().dmgs_last_error().decode()


def default_options(N):
    o = Options()
    lib().dmgs_default_options(int(N), C.byref(o))
    return o
