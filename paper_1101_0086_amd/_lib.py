"""ctypes binding of libmpa.so (include/mpa.h): argument marshalling only.

Every step of the propagation runs in the library's HIP kernels.  Loading
fails loudly if the library has not been built; there is no fallback path.
"""
from __future__ import annotations

import ctypes as C
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libmpa.so")

MPA_OK = 0
MPA_EINVAL = -1
MPA_ENOMEM = -2
MPA_EDEVICE = -3
MPA_EALIGN = -4
MPA_EHALO = -5
MPA_ENONFINITE = -6
MPA_EDIVERGE = -7
MPA_EUNSUPPORTED = -8

MPA_C64 = 0
MPA_C128 = 1

MPA_WAVEFRONT = 0
MPA_NODE_PARALLEL = 1

MPA_SHIFT_AUTO = -(1 << 31)

# symbols declared in include/mpa.h
EXPORTED = ("mpa_plan_create", "mpa_plan_destroy", "mpa_plan_get_info", "mpa_plan_validate",
            "mpa_step", "mpa_propagate", "mpa_batch_plan_validate", "mpa_batch_plan_create",
            "mpa_batch_plan_destroy", "mpa_batch_get_info", "mpa_batch_propagate",
            "mpa_graph_capture", "mpa_batch_graph_capture", "mpa_graph_launch", "mpa_graph_destroy",
            "ss_plan_create", "ss_plan_destroy", "ss_plan_propagate", "ss_propagate", "mpa_status_string", "mpa_last_error_detail",
            "mpa_checkpoint_count", "mpa_propagate_checkpointed", "mpa_adjoint", "mpa_adjoint_keep_inputs",
            "mpa_batch_checkpoint_count", "mpa_batch_propagate_checkpointed", "mpa_batch_adjoint",
            "mpa_batch_adjoint_keep_inputs",
            "mpa_propagate_noalloc", "mpa_check_field", "mpa_picard_residuals")


class mpa_map(C.Structure):
    _fields_ = [("n_seg", C.c_int32), ("seg_len", C.POINTER(C.c_double)),
                ("beta2", C.POINTER(C.c_double)), ("beta3", C.POINTER(C.c_double)),
                ("sigma", C.POINTER(C.c_double)), ("gamma", C.c_double), ("z_amp", C.c_double),
                ("raman_g0", C.c_double), ("raman_alpha", C.c_double)]


class mpa_params(C.Structure):
    _fields_ = [("n", C.c_int64), ("dt", C.c_double), ("L", C.c_double), ("M", C.c_int32),
                ("n_iter", C.c_int32), ("block", C.c_int32), ("halo", C.c_int32),
                ("precision", C.c_int32), ("omega_band", C.c_double), ("schedule", C.c_int32),
                ("shift", C.c_int32)]


class mpa_batch_desc(C.Structure):
    _fields_ = [("count", C.c_int32), ("n", C.POINTER(C.c_int64)), ("sigma_scale", C.POINTER(C.c_double))]


class mpa_plan_info(C.Structure):
    _fields_ = [("n", C.c_int64), ("block", C.c_int32), ("halo", C.c_int32),
                ("core", C.c_int32), ("n_blocks", C.c_int32), ("threads_per_block", C.c_int32),
                ("table_bytes", C.c_int64), ("workspace_bytes", C.c_int64), ("shift", C.c_int32)]


class MPAError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"{message} (status {status})")
        self.status = status


_lib = None


def lib() -> C.CDLL:
    """The loaded library (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    # torch carries its own HIP runtime; importing it first makes libmpa.so
    # bind to that same runtime (one HIP runtime per process) instead of
    # loading a second copy from the system ROCm.
    import torch  # noqa: F401
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with "
                          "`python -c 'import __graft_entry__ as g; g.build()'`")
    h = C.CDLL(LIB_PATH)
    vp, dp = C.c_void_p, C.c_double
    h.mpa_plan_create.argtypes = [C.POINTER(mpa_params), C.POINTER(mpa_map), C.c_int, C.POINTER(vp)]
    h.mpa_plan_destroy.argtypes = [vp]
    h.mpa_plan_get_info.argtypes = [vp, C.POINTER(mpa_plan_info)]
    h.mpa_plan_validate.argtypes = [C.POINTER(mpa_params), C.POINTER(mpa_map)]
    h.mpa_step.argtypes = [vp, vp, dp, vp]
    h.mpa_propagate.argtypes = [vp, vp, dp, dp, vp]
    h.mpa_propagate_noalloc.argtypes = [C.POINTER(mpa_params), C.POINTER(mpa_map), vp, dp, dp, vp]
    h.mpa_check_field.argtypes = [vp, vp, vp]
    h.mpa_picard_residuals.argtypes = [vp, vp, dp, C.POINTER(C.c_double), vp]
    h.mpa_batch_plan_validate.argtypes = [C.POINTER(mpa_params), C.POINTER(mpa_map), C.POINTER(mpa_batch_desc)]
    h.mpa_batch_plan_create.argtypes = [C.POINTER(mpa_params), C.POINTER(mpa_map), C.POINTER(mpa_batch_desc),
                                        C.c_int, C.POINTER(vp)]
    h.mpa_batch_plan_destroy.argtypes = [vp]
    h.mpa_batch_get_info.argtypes = [vp, C.POINTER(C.c_int64), C.POINTER(C.c_int32)]
    h.mpa_batch_propagate.argtypes = [vp, vp, dp, dp, vp]
    h.mpa_graph_capture.argtypes = [vp, vp, dp, dp, C.POINTER(vp)]
    h.mpa_batch_graph_capture.argtypes = [vp, vp, dp, dp, C.POINTER(vp)]
    h.mpa_graph_launch.argtypes = [vp, vp]
    h.mpa_graph_destroy.argtypes = [vp]
    h.ss_plan_create.argtypes = [C.POINTER(mpa_map), C.c_int64, dp, dp, C.c_int32, C.c_int, C.POINTER(vp)]
    h.ss_plan_destroy.argtypes = [vp]
    h.ss_plan_propagate.argtypes = [vp, vp, dp, dp, vp]
    h.ss_propagate.argtypes = [C.POINTER(mpa_map), C.c_int64, dp, dp, C.c_int32, vp, dp, dp, vp]
    h.mpa_checkpoint_count.argtypes = [vp, dp, dp, C.POINTER(C.c_int64)]
    h.mpa_propagate_checkpointed.argtypes = [vp, vp, dp, dp, vp, vp]
    h.mpa_adjoint.argtypes = [vp, vp, vp, dp, dp, vp, C.c_int64, vp]
    h.mpa_batch_checkpoint_count.argtypes = [vp, dp, dp, C.POINTER(C.c_int64)]
    h.mpa_batch_propagate_checkpointed.argtypes = [vp, vp, dp, dp, vp, vp]
    h.mpa_batch_adjoint.argtypes = [vp, vp, vp, dp, dp, vp, C.c_int64, vp]
    h.mpa_adjoint_keep_inputs.argtypes = [vp, C.c_int64]
    h.mpa_batch_adjoint_keep_inputs.argtypes = [vp, C.c_int64]
    h.mpa_status_string.argtypes = [C.c_int]
    h.mpa_status_string.restype = C.c_char_p
    h.mpa_last_error_detail.argtypes = [C.c_char_p, C.c_int]
    for name in EXPORTED:
        if name not in ("mpa_status_string",):
            getattr(h, name).restype = C.c_int
    _lib = h
    return h


def check(status: int) -> None:
    if status != MPA_OK:
        buf = C.create_string_buffer(1024)
        lib().mpa_last_error_detail(buf, 1024)
        raise MPAError(status, buf.value.decode() or lib().mpa_status_string(status).decode())


class MapStruct:
    """Keeps the ctypes arrays of an mpa_map alive."""

    def __init__(self, dmmap):
        n = len(dmmap.seg_len)
        arr = C.c_double * n
        self._a = [arr(*map(float, getattr(dmmap, f))) for f in ("seg_len", "beta2", "beta3", "sigma")]
        self.s = mpa_map(n, self._a[0], self._a[1], self._a[2], self._a[3],
                         float(dmmap.gamma), float(dmmap.z_amp),
                         float(getattr(dmmap, "raman_g0", 0.0)), float(getattr(dmmap, "raman_alpha", 0.0)))


def make_params(n, dt, L, M, n_iter, block=0, halo=0, precision=MPA_C64, omega_band=0.0,
                schedule=MPA_WAVEFRONT, shift=0):
    return mpa_params(int(n), float(dt), float(L), int(M), int(n_iter), int(block), int(halo),
                      int(precision), float(omega_band), int(schedule), int(shift))


class BatchDesc:
    """Keeps the ctypes arrays of an mpa_batch_desc alive."""

    def __init__(self, ns, sigma_scale=None):
        k = len(ns)
        self._n = (C.c_int64 * k)(*[int(v) for v in ns])
        self._s = (C.c_double * k)(*[float(v) for v in sigma_scale]) if sigma_scale is not None else None
        self.s = mpa_batch_desc(k, self._n, self._s if self._s is not None else None)
