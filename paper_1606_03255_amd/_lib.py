"""ctypes binding of ``libflt.so`` (the C ABI declared in ``include/flt.h``).

Argument marshalling only: every transform step runs in the library's HIP
kernels.  Importing this module fails loudly if the library is not built.
"""
import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libflt.so")

FLT_C64 = 1
FLT_C128 = 2
FLT_FLAG_HOST_ONLY = 1
FLT_FLAG_NFFT_ONLY = 2
FLT_FLAG_GRAPH = 4
FLT_FLAG_AUTOTUNE = 8
FLT_FLAG_TUNE_FORWARD = 16
FLT_NOALLOC_MAX_BYTES = 128 << 20

ERRORS = {
    0: "FLT_OK", -1: "FLT_EINVAL", -2: "FLT_EDOMAIN", -3: "FLT_EPRECISION", -4: "FLT_ENOWORKSPACE",
    -5: "FLT_EHIP", -6: "FLT_ESTATE", -7: "FLT_ENOMEM", -8: "FLT_ERANGE",
}

# every symbol include/flt.h declares
EXPORTS = (
    "flt_plan_create", "flt_plan_create_policy", "flt_plan_create_batch", "flt_plan_destroy", "flt_plan_info", "flt_plan_band", "flt_plan_node_bands",
    "flt_plan_workspace_size", "flt_plan_set_workspace", "flt_forward", "flt_derivative", "flt_adjoint",
    "flt_forward_derivative", "flt_forward_noalloc", "flt_profile_forward", "flt_profile_adjoint", "flt_strerror", "flt_last_hip_error",
    "flt_laplace_plan_create", "flt_laplace_plan_create_kernel", "flt_laplace_plan_info", "flt_laplace_forward",
    "flt_laplace_plan_destroy",
    "flt_xi_plan_create", "flt_xi_plan_info", "flt_xi_forward", "flt_xi_transposed", "flt_xi_adjoint",
    "flt_xi_plan_destroy",
)


class FltInfo(ctypes.Structure):
    _fields_ = [
        ("N", ctypes.c_int64), ("M", ctypes.c_int64),
        ("dtype", ctypes.c_int32), ("q", ctypes.c_int32), ("D", ctypes.c_int32), ("n_xi", ctypes.c_int32),
        ("mw", ctypes.c_int32), ("num_bands", ctypes.c_int32),
        ("eps", ctypes.c_double), ("eps_K", ctypes.c_double), ("eps_A", ctypes.c_double),
        ("y1", ctypes.c_double), ("nodes_z0", ctypes.c_int64), ("workspace_bytes", ctypes.c_size_t),
        ("bytes_forward", ctypes.c_double), ("flops_forward", ctypes.c_double), ("direct_scale", ctypes.c_double),
        ("forward_scratch_bytes", ctypes.c_size_t),
        ("passB_blocks", ctypes.c_int32),
        ("pad", ctypes.c_int32),
    ]


class FltBandInfo(ctypes.Structure):
    _fields_ = [
        ("m", ctypes.c_int32), ("q", ctypes.c_int32), ("ell_lo", ctypes.c_int32), ("ell_hi", ctypes.c_int32),
        ("K", ctypes.c_int64), ("n", ctypes.c_int64), ("k0", ctypes.c_int64), ("nodes", ctypes.c_int64),
        ("passes", ctypes.c_int32), ("direct", ctypes.c_int32), ("cells", ctypes.c_int64),
    ]


class FltLaplaceInfo(ctypes.Structure):
    _fields_ = [
        ("N", ctypes.c_int64), ("M", ctypes.c_int64),
        ("dtype", ctypes.c_int32), ("q", ctypes.c_int32), ("levels", ctypes.c_int32), ("kernel", ctypes.c_int32),
        ("eps", ctypes.c_double), ("y1", ctypes.c_double), ("xi1", ctypes.c_double),
    ]


class FltXiInfo(ctypes.Structure):
    _fields_ = [
        ("N", ctypes.c_int64), ("M", ctypes.c_int64),
        ("dtype", ctypes.c_int32), ("q", ctypes.c_int32), ("mw1", ctypes.c_int32), ("num_bands", ctypes.c_int32),
        ("inner_instances", ctypes.c_int32), ("inner_mw", ctypes.c_int32),
        ("eps", ctypes.c_double), ("eps_w", ctypes.c_double), ("eps_in", ctypes.c_double),
        ("sigma_min", ctypes.c_double), ("amp", ctypes.c_double),
        ("inner_coefficients", ctypes.c_int64), ("inner_nodes", ctypes.c_int64),
        ("inner_workspace_bytes", ctypes.c_size_t),
    ]


class FltError(RuntimeError):
    def __init__(self, code, where):
        self.code = code
        msg = "%s failed: %s (%d)" % (where, ERRORS.get(code, "?"), code)
        if code == -5 and _lib is not None:
            msg += ", hipError %d" % _lib.flt_last_hip_error()
        super().__init__(msg)


_lib = None


def load():
    """Load libflt.so from the package directory (raises if absent)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError("libflt.so is not built; run `python -m paper_1606_03255_amd.build` "
                          "(the transform has no CPU fallback)")
    lib = ctypes.CDLL(LIB_PATH)
    vp = ctypes.c_void_p
    P = ctypes.POINTER
    lib.flt_plan_create.argtypes = [P(vp), ctypes.c_int64, ctypes.c_int64, P(ctypes.c_double), ctypes.c_double,
                                    ctypes.c_int, ctypes.c_uint32]
    lib.flt_plan_create_policy.argtypes = [P(vp), ctypes.c_int64, ctypes.c_int64, P(ctypes.c_double),
                                           ctypes.c_double, ctypes.c_int, ctypes.c_uint32, ctypes.c_double]
    lib.flt_plan_create_batch.argtypes = [P(vp), ctypes.c_int32, P(ctypes.c_int64), P(ctypes.c_int64),
                                          P(ctypes.c_double), ctypes.c_double, ctypes.c_int, ctypes.c_uint32]
    lib.flt_plan_destroy.argtypes = [vp]
    lib.flt_plan_destroy.restype = None
    lib.flt_plan_info.argtypes = [vp, P(FltInfo)]
    lib.flt_plan_band.argtypes = [vp, ctypes.c_int32, P(FltBandInfo)]
    lib.flt_plan_node_bands.argtypes = [vp, P(ctypes.c_int32)]
    lib.flt_plan_workspace_size.argtypes = [vp, P(ctypes.c_size_t)]
    lib.flt_plan_set_workspace.argtypes = [vp, vp, ctypes.c_size_t]
    for name in ("flt_forward", "flt_derivative", "flt_adjoint"):
        getattr(lib, name).argtypes = [vp, vp, vp, vp]
    lib.flt_forward_derivative.argtypes = [vp, vp, vp, vp, vp]
    lib.flt_forward_noalloc.argtypes = [vp, vp, vp, vp]
    lib.flt_laplace_plan_create.argtypes = [P(vp), ctypes.c_int64, P(ctypes.c_double), ctypes.c_int64,
                                            P(ctypes.c_double), ctypes.c_double, ctypes.c_int, ctypes.c_uint32]
    lib.flt_laplace_plan_create_kernel.argtypes = [P(vp), ctypes.c_int32, ctypes.c_int64, P(ctypes.c_double),
                                                   ctypes.c_int64, P(ctypes.c_double), ctypes.c_double, ctypes.c_int,
                                                   ctypes.c_uint32]
    lib.flt_laplace_plan_info.argtypes = [vp, P(FltLaplaceInfo)]
    lib.flt_laplace_forward.argtypes = [vp, vp, vp, vp]
    lib.flt_laplace_plan_destroy.argtypes = [vp]
    lib.flt_laplace_plan_destroy.restype = None
    lib.flt_xi_plan_create.argtypes = [P(vp), ctypes.c_int64, P(ctypes.c_double), ctypes.c_int64,
                                       P(ctypes.c_double), ctypes.c_double, ctypes.c_int, ctypes.c_uint32]
    lib.flt_xi_plan_info.argtypes = [vp, P(FltXiInfo)]
    for name in ("flt_xi_forward", "flt_xi_transposed", "flt_xi_adjoint"):
        getattr(lib, name).argtypes = [vp, vp, vp, vp]
    lib.flt_xi_plan_destroy.argtypes = [vp]
    lib.flt_xi_plan_destroy.restype = None
    lib.flt_profile_forward.argtypes = [vp, vp, vp, vp, P(ctypes.c_double)]
    lib.flt_profile_adjoint.argtypes = [vp, vp, vp, vp, P(ctypes.c_double)]
    lib.flt_strerror.argtypes = [ctypes.c_int]
    lib.flt_strerror.restype = ctypes.c_char_p
    lib.flt_last_hip_error.argtypes = []
    _lib = lib
    return lib


def check(code, where):
    if code != 0:
        raise FltError(code, where)
