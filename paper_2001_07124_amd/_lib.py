"""ctypes declarations of the C ABI in include/rhosvd.h (argument marshalling only).

The shared library is loaded lazily, after torch, so that it binds to the HIP
runtime torch already loaded.  A missing library raises: there is no CPU
fallback anywhere in the product path.
"""
import ctypes
import os
import threading

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "librhosvd.so")

MAX_ORDER = 16
MAX_K = 128

OK, EINVAL, ENOMEM, EHIP, ENUMERIC, EBUSY, EUNSUPPORTED, ESCRATCH = range(8)
NOALLOC_SCRATCH_BYTES = 64 << 20
F32, F64 = 0, 1
RP_HOSVD, R_STHOSVD, RP_HOOI, R_PET = 0, 1, 2, 3
PREC_F64, PREC_F32, PREC_BF16, PREC_FP8 = 0, 1, 2, 3
FLAG_K_CAPPED, FLAG_CQR_SHIFTED, FLAG_EVD_NOCONV, FLAG_QR_HOUSEHOLDER = 0x1, 0x2, 0x4, 0x8
FLAG_E_EXPLICIT = 0x10
OPT_EXPLICIT_ERROR = 0x1
OPT_KR_SKETCH = 0x2
REQ_QUEUED, REQ_RUNNING, REQ_DONE = 0, 1, 2
OPTION_KERNELS = 1
KERNELS_AUTO, KERNELS_TILED = 0, 1


class Tensor(ctypes.Structure):
    _fields_ = [("order", ctypes.c_int32), ("dims", ctypes.POINTER(ctypes.c_int64)),
                ("dtype", ctypes.c_int32), ("data", ctypes.c_void_p)]


class Params(ctypes.Structure):
    _fields_ = [("algo", ctypes.c_int32), ("ranks", ctypes.POINTER(ctypes.c_int32)),
                ("oversample", ctypes.c_int32), ("power_iters", ctypes.c_int32),
                ("seed", ctypes.c_uint64), ("mode_order", ctypes.POINTER(ctypes.c_int32)),
                ("precision", ctypes.c_int32), ("flags", ctypes.c_uint32)]


class AdaptiveParams(ctypes.Structure):
    _fields_ = [("eps", ctypes.c_double), ("kmax", ctypes.c_int32), ("power_iters", ctypes.c_int32),
                ("seed", ctypes.c_uint64), ("precision", ctypes.c_int32), ("flags", ctypes.c_uint32)]


class Report(ctypes.Structure):
    _fields_ = [("norm_x2", ctypes.c_double), ("norm_core2", ctypes.c_double),
                ("order", ctypes.c_int32), ("k_used", ctypes.c_int32 * MAX_ORDER),
                ("flags", ctypes.c_uint32),
                ("sigma", (ctypes.c_double * MAX_K) * MAX_ORDER),
                ("resid2", ctypes.c_double)]


class Output(ctypes.Structure):
    _fields_ = [("core", ctypes.c_void_p), ("factors", ctypes.POINTER(ctypes.c_void_p)),
                ("report", ctypes.c_void_p)]


_lock = threading.Lock()
_lib = None

_P, _I32, _I64, _U64, _SZ = (ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_uint64,
                             ctypes.c_size_t)
_DP = ctypes.POINTER(ctypes.c_double)

_PROTOS = {
    "rhosvd_status_string": (ctypes.c_char_p, [_I32]),
    "rhosvd_last_hip_error": (_I32, []),
    "rhosvd_create": (_I32, [ctypes.POINTER(_P), _I32]),
    "rhosvd_destroy": (None, [_P]),
    "rhosvd_set_option": (_I32, [_P, _I32, _I64]),
    "rhosvd_workspace_size": (_I32, [ctypes.POINTER(Tensor), ctypes.POINTER(Params),
                                     ctypes.POINTER(_SZ)]),
    "rhosvd_decompose": (_I32, [_P, ctypes.POINTER(Tensor), ctypes.POINTER(Params), _P, _SZ,
                                ctypes.POINTER(Output), _P]),
    "rhosvd_decompose_noalloc": (_I32, [_P, ctypes.POINTER(Tensor), ctypes.POINTER(Params),
                                        ctypes.POINTER(Output), _P]),
    "rhosvd_adaptive_workspace_size": (_I32, [ctypes.POINTER(Tensor), ctypes.POINTER(AdaptiveParams),
                                              ctypes.POINTER(_SZ)]),
    "rhosvd_decompose_adaptive": (_I32, [_P, ctypes.POINTER(Tensor), ctypes.POINTER(AdaptiveParams),
                                         _P, _SZ, ctypes.POINTER(Output), ctypes.POINTER(_I32),
                                         ctypes.POINTER(_I32), _P]),
    "rhosvd_batch_create": (_I32, [_P, _I32, ctypes.POINTER(Tensor), ctypes.POINTER(Params),
                                   ctypes.POINTER(Output), ctypes.POINTER(_P), ctypes.POINTER(_SZ)]),
    "rhosvd_batch_bind": (_I32, [_P, _P, _SZ, _I32, _P]),
    "rhosvd_batch_run": (_I32, [_P, _I32, _P]),
    "rhosvd_batch_launches": (_I32, [_P]),
    "rhosvd_batch_destroy": (None, [_P]),
    "rhosvd_server_create": (_I32, [_P, _I32, _P, _SZ, _I32, ctypes.POINTER(_P)]),
    "rhosvd_server_submit": (_I32, [_P, ctypes.POINTER(Tensor), ctypes.POINTER(Params),
                                    ctypes.POINTER(Output), ctypes.POINTER(_U64)]),
    "rhosvd_server_poll": (_I32, [_P, _U64, ctypes.POINTER(_I32), _DP]),
    "rhosvd_server_release": (_I32, [_P, _U64]),
    "rhosvd_server_drain": (_I32, [_P]),
    "rhosvd_server_destroy": (None, [_P]),
    "rhosvd_report_rel_error": (ctypes.c_double, [ctypes.POINTER(Report)]),
    "rhosvd_omega_fill": (_I32, [_P, _U64, _I32, _I32, _I64, _I32, _I32, _P, _P]),
    "rhosvd_sketch": (_I32, [_P, _P, _I32, _I32, _I64, _I64, _I64, _I32, _U64, _I32, _I32, _P, _P,
                             _P, _SZ, _P]),
    "rhosvd_sketch_kr": (_I32, [_P, _P, _I32, _I32, _I64, _I64, _I64, _I32, _P, _P, _I32, _P, _P,
                                _P, _SZ, _P]),
    "rhosvd_sketch_all": (_I32, [_P, _P, _I32, _I32, _P, _P, _U64, _I32, _P, _P, _P, _SZ, _P]),
    "rhosvd_sketch_all_workspace_size": (_SZ, [_I32, _P, _P, _I32]),
    "rhosvd_power": (_I32, [_P, _P, _I32, _I32, _I64, _I64, _I64, _I32, _P, _P, _P, _SZ, _P]),
    "rhosvd_ttm": (_I32, [_P, _P, _I32, _I32, _I64, _I64, _I64, _I32, _P, _P, _P, _P, _P, _SZ, _P]),
    "rhosvd_truncate_rotated": (_I32, [_P, _I32, _P, _I32, _I64, _P, _I32, _P, _P]),
    "rhosvd_orthonormalize": (_I32, [_P, _P, _I64, _I32, _I32, _P, _P, _P, _P]),
    "rhosvd_sym_evd": (_I32, [_P, _P, _I32, _P, _P, _P, _P]),
    "rhosvd_step_workspace_size": (_SZ, [_I64, _I32, _I64]),
}


def exported_names():
    return sorted(_PROTOS)


def load(require_torch=True):
    """Load librhosvd.so (after torch) and declare every prototype."""
    global _lib
    with _lock:
        if _lib is not None:
            return _lib
        if require_torch:
            import torch  # noqa: F401  (bind to the HIP runtime torch loads)
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(
                "librhosvd.so is not built; run `python -m paper_2001_07124_amd.build` "
                "(the HIP library is required: there is no CPU fallback)")
        lib = ctypes.CDLL(LIB_PATH)
        missing = []
        for name, (res, args) in _PROTOS.items():
            try:
                fn = getattr(lib, name)
            except AttributeError:
                missing.append(name)     # a stale build: only calls of it fail
                continue
            fn.restype = res
            fn.argtypes = args
        if missing:
            import warnings
            warnings.warn(f"librhosvd.so lacks {missing}; rebuild it", RuntimeWarning)
        _lib = lib
        return lib


class RhosvdError(RuntimeError):
    def __init__(self, status, where):
        lib = _lib
        msg = lib.rhosvd_status_string(status).decode() if lib else str(status)
        extra = ""
        if status == EHIP and lib:
            extra = f" (hip error {lib.rhosvd_last_hip_error()})"
        super().__init__(f"{where}: {msg}{extra}")
        self.status = status


def check(status, where):
    if status != OK:
        raise RhosvdError(status, where)
