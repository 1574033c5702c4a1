"""MI355X (gfx950) implementation of the massively parallel algorithm (MPA)
for dispersion-managed WDM fibre links, with a split-step comparator.

Python entry points wrap the C ABI of ``libmpa.so`` (include/mpa.h); fields
are torch tensors on the GPU (complex64 for the FP32 path, complex128 for the
FP64 path) and work runs on torch's current HIP stream.
"""
from __future__ import annotations

import ctypes as C

from . import _lib
from ._lib import MPA_C64, MPA_C128, MPA_NODE_PARALLEL, MPA_SHIFT_AUTO, MPA_WAVEFRONT, MPAError

__all__ = ["MPAPlan", "MPABatchPlan", "Graph", "SSPlan", "MPA_C64", "MPA_C128", "MPA_WAVEFRONT",
           "MPA_NODE_PARALLEL", "MPA_SHIFT_AUTO", "MPAError", "validate", "propagate_noalloc", "ss_propagate"]


def _stream_handle(torch, device):
    return C.c_void_p(torch.cuda.current_stream(device).cuda_stream)


def _check_field(field, precision, n):
    import torch
    want = torch.complex64 if precision == MPA_C64 else torch.complex128
    if not field.is_cuda or field.dtype != want or not field.is_contiguous() or field.numel() != n:
        raise ValueError(f"field must be a contiguous {want} CUDA tensor of {n} samples")
    return torch


def validate(n, dt, dmmap, L, M, n_iter, block=0, halo=0, precision=MPA_C64, omega_band=0.0,
             schedule=MPA_WAVEFRONT, shift=0):
    """Host-only check of a plan's parameters; raises MPAError if invalid."""
    p = _lib.make_params(n, dt, L, M, n_iter, block, halo, precision, omega_band, schedule, shift)
    m = _lib.MapStruct(dmmap)
    _lib.check(_lib.lib().mpa_plan_validate(C.byref(p), C.byref(m.s)))


def propagate_noalloc(field, dt, dmmap, L, M, n_iter, z0, z1, block=0, halo=0, precision=MPA_C64,
                      omega_band=0.0, shift=0):
    """mpa_propagate_noalloc: the march without a plan and without device
    allocation, in place on `field` (its length is N), on the field's device
    and torch's current stream."""
    import torch
    if not field.is_cuda:
        raise ValueError("field must be a CUDA tensor")
    _check_field(field, precision, field.numel())
    p = _lib.make_params(field.numel(), dt, L, M, n_iter, block, halo, precision, omega_band, shift=shift)
    m = _lib.MapStruct(dmmap)
    with torch.cuda.device(field.device):
        _lib.check(_lib.lib().mpa_propagate_noalloc(C.byref(p), C.byref(m.s), C.c_void_p(field.data_ptr()),
                                                    float(z0), float(z1), _stream_handle(torch, field.device)))
    return field


class MPAPlan:
    """mpa_plan_create / mpa_step / mpa_propagate."""

    def __init__(self, n, dt, dmmap, L, M, n_iter, block=0, halo=0, precision=MPA_C64,
                 omega_band=0.0, device=0, schedule=MPA_WAVEFRONT, shift=0):
        self.n, self.precision, self.device = int(n), int(precision), int(device)
        self.L = float(L)
        self.n_seg = len(dmmap.seg_len)
        self.coefficients = tuple(tuple(float(v) for v in getattr(dmmap, f)) for f in ("sigma", "beta2", "beta3"))
        p = _lib.make_params(n, dt, L, M, n_iter, block, halo, precision, omega_band, schedule, shift)
        m = _lib.MapStruct(dmmap)
        h = C.c_void_p()
        _lib.check(_lib.lib().mpa_plan_create(C.byref(p), C.byref(m.s), int(device), C.byref(h)))
        self._h = h

    def info(self):
        i = _lib.mpa_plan_info()
        _lib.check(_lib.lib().mpa_plan_get_info(self._h, C.byref(i)))
        return {f: getattr(i, f) for f, _ in i._fields_}

    def step(self, field, z0):
        torch = _check_field(field, self.precision, self.n)
        _lib.check(_lib.lib().mpa_step(self._h, C.c_void_p(field.data_ptr()), float(z0),
                                       _stream_handle(torch, field.device)))
        return field

    def propagate(self, field, z0, z1):
        torch = _check_field(field, self.precision, self.n)
        _lib.check(_lib.lib().mpa_propagate(self._h, C.c_void_p(field.data_ptr()), float(z0),
                                            float(z1), _stream_handle(torch, field.device)))
        return field

    def check_field(self, field):
        """mpa_check_field: raises MPAError (MPA_ENONFINITE) if the field holds NaN or Inf."""
        torch = _check_field(field, self.precision, self.n)
        _lib.check(_lib.lib().mpa_check_field(self._h, C.c_void_p(field.data_ptr()),
                                              _stream_handle(torch, field.device)))

    def picard_residuals(self, field, z0, n_iter):
        """mpa_picard_residuals: (status, residuals) of the long step at z0;
        status is MPA_OK, MPA_EDIVERGE or MPA_ENONFINITE (other errors raise)."""
        torch = _check_field(field, self.precision, self.n)
        r = (C.c_double * n_iter)()
        st = _lib.lib().mpa_picard_residuals(self._h, C.c_void_p(field.data_ptr()), float(z0), r,
                                             _stream_handle(torch, field.device))
        if st not in (_lib.MPA_OK, _lib.MPA_EDIVERGE, _lib.MPA_ENONFINITE):
            _lib.check(st)
        return st, list(r)

    def checkpoint_count(self, z0, z1):
        c = C.c_int64()
        _lib.check(_lib.lib().mpa_checkpoint_count(self._h, float(z0), float(z1), C.byref(c)))
        return c.value

    def propagate_checkpointed(self, field, z0, z1):
        """mpa_propagate_checkpointed: marches `field` in place and returns the
        checkpoints (one field per map period segment of [z0, z1])."""
        torch = _check_field(field, self.precision, self.n)
        k = self.checkpoint_count(z0, z1)
        ckpt = torch.empty((k, self.n), dtype=field.dtype, device=field.device)
        _lib.check(_lib.lib().mpa_propagate_checkpointed(
            self._h, C.c_void_p(field.data_ptr()), float(z0), float(z1),
            C.c_void_p(ckpt.data_ptr() if k else 0), _stream_handle(torch, field.device)))
        return ckpt

    def keep_inputs(self, max_bytes):
        """mpa_adjoint_keep_inputs: propagate_checkpointed keeps every long
        step's input when they fit in `max_bytes` (0: none), and adjoint over
        the same range and checkpoints reverses from them."""
        _lib.check(_lib.lib().mpa_adjoint_keep_inputs(self._h, int(max_bytes)))

    def adjoint(self, checkpoints, grad, z0, z1, store_steps=0):
        """mpa_adjoint: turns G(A(z1)) in `grad` into G(A(z0)) in place and
        returns dl/d(sigma, beta2, beta3) per span as a (3, n_seg) FP64 tensor
        on the field's device."""
        torch = _check_field(grad, self.precision, self.n)
        k = self.checkpoint_count(z0, z1)
        if checkpoints.shape != (k, self.n) or checkpoints.dtype != grad.dtype or not checkpoints.is_contiguous():
            raise ValueError(f"checkpoints must be a contiguous ({k}, {self.n}) {grad.dtype} tensor")
        pg = torch.empty((3, self.n_seg), dtype=torch.float64, device=grad.device)
        _lib.check(_lib.lib().mpa_adjoint(
            self._h, C.c_void_p(checkpoints.data_ptr() if k else 0), C.c_void_p(grad.data_ptr()),
            float(z0), float(z1), C.c_void_p(pg.data_ptr()), int(store_steps),
            _stream_handle(torch, grad.device)))
        return pg

    def close(self):
        if getattr(self, "_h", None):
            _lib.lib().mpa_plan_destroy(self._h)
            self._h = None

    __del__ = close


class Graph:
    """An executable HIP graph of captured launches (mpa_graph_*)."""

    def __init__(self, handle, device):
        self._h, self.device = handle, device

    def launch(self):
        import torch
        _lib.check(_lib.lib().mpa_graph_launch(self._h, _stream_handle(torch, self.device)))

    def close(self):
        if getattr(self, "_h", None):
            _lib.lib().mpa_graph_destroy(self._h)
            self._h = None

    __del__ = close


def _capture_propagate(self, field, z0, z1):
    _check_field(field, self.precision, self.n)
    h = C.c_void_p()
    _lib.check(_lib.lib().mpa_graph_capture(self._h, C.c_void_p(field.data_ptr()), float(z0),
                                            float(z1), C.byref(h)))
    return Graph(h, field.device)


MPAPlan.capture = _capture_propagate


class MPABatchPlan:
    """mpa_batch_plan_create / mpa_batch_propagate: many fields of different
    lengths (each a power of two >= block) marched by one launch per long
    step.  Fields are concatenated in one tensor; use :meth:`split` to view
    the instances."""

    def __init__(self, ns, dt, dmmap, L, M, n_iter, block, halo, precision=MPA_C64,
                 omega_band=0.0, sigma_scale=None, device=0, shift=0):
        self.ns = [int(v) for v in ns]
        self.n = sum(self.ns)
        self.precision, self.device = int(precision), int(device)
        self.n_seg = len(dmmap.seg_len)
        self.coefficients = tuple(tuple(float(v) for v in getattr(dmmap, f)) for f in ("sigma", "beta2", "beta3"))
        p = _lib.make_params(max(self.ns), dt, L, M, n_iter, block, halo, precision, omega_band, shift=shift)
        m = _lib.MapStruct(dmmap)
        d = _lib.BatchDesc(self.ns, sigma_scale)
        h = C.c_void_p()
        _lib.check(_lib.lib().mpa_batch_plan_create(C.byref(p), C.byref(m.s), C.byref(d.s),
                                                    int(device), C.byref(h)))
        self._h = h

    def info(self):
        total, items = C.c_int64(), C.c_int32()
        _lib.check(_lib.lib().mpa_batch_get_info(self._h, C.byref(total), C.byref(items)))
        return {"total_samples": total.value, "work_items": items.value}

    def split(self, fields):
        out, o = [], 0
        for k in self.ns:
            out.append(fields[o:o + k])
            o += k
        return out

    def propagate(self, fields, z0, z1):
        torch = _check_field(fields, self.precision, self.n)
        _lib.check(_lib.lib().mpa_batch_propagate(self._h, C.c_void_p(fields.data_ptr()), float(z0),
                                                  float(z1), _stream_handle(torch, fields.device)))
        return fields

    def checkpoint_count(self, z0, z1):
        c = C.c_int64()
        _lib.check(_lib.lib().mpa_batch_checkpoint_count(self._h, float(z0), float(z1), C.byref(c)))
        return c.value

    def propagate_checkpointed(self, fields, z0, z1):
        """mpa_batch_propagate_checkpointed: marches the concatenated `fields`
        in place and returns the checkpoints (k, total samples)."""
        torch = _check_field(fields, self.precision, self.n)
        k = self.checkpoint_count(z0, z1)
        ckpt = torch.empty((k, self.n), dtype=fields.dtype, device=fields.device)
        _lib.check(_lib.lib().mpa_batch_propagate_checkpointed(
            self._h, C.c_void_p(fields.data_ptr()), float(z0), float(z1),
            C.c_void_p(ckpt.data_ptr() if k else 0), _stream_handle(torch, fields.device)))
        return ckpt

    def keep_inputs(self, max_bytes):
        """mpa_batch_adjoint_keep_inputs (see MPAPlan.keep_inputs)."""
        _lib.check(_lib.lib().mpa_batch_adjoint_keep_inputs(self._h, int(max_bytes)))

    def adjoint(self, checkpoints, grads, z0, z1, store_steps=0):
        """mpa_batch_adjoint: turns G(A(z1)) of every instance (concatenated in
        `grads`) into G(A(z0)) in place and returns the derivatives of the loss
        with respect to the shared (sigma, beta2, beta3) per span, (3, n_seg) FP64."""
        torch = _check_field(grads, self.precision, self.n)
        k = self.checkpoint_count(z0, z1)
        if checkpoints.shape != (k, self.n) or checkpoints.dtype != grads.dtype or not checkpoints.is_contiguous():
            raise ValueError(f"checkpoints must be a contiguous ({k}, {self.n}) {grads.dtype} tensor")
        pg = torch.empty((3, self.n_seg), dtype=torch.float64, device=grads.device)
        _lib.check(_lib.lib().mpa_batch_adjoint(
            self._h, C.c_void_p(checkpoints.data_ptr() if k else 0), C.c_void_p(grads.data_ptr()),
            float(z0), float(z1), C.c_void_p(pg.data_ptr()), int(store_steps),
            _stream_handle(torch, grads.device)))
        return pg

    def capture(self, fields, z0, z1):
        _check_field(fields, self.precision, self.n)
        h = C.c_void_p()
        _lib.check(_lib.lib().mpa_batch_graph_capture(self._h, C.c_void_p(fields.data_ptr()), float(z0),
                                                      float(z1), C.byref(h)))
        return Graph(h, fields.device)

    def close(self):
        if getattr(self, "_h", None):
            _lib.lib().mpa_batch_plan_destroy(self._h)
            self._h = None

    __del__ = close


def ss_propagate(field, dt, dmmap, dz, z0, z1):
    """ss_propagate (Eq. 4) without a plan: the library builds the tables on
    the field's device, runs on torch's current stream, waits for it and
    frees them.  `field`: contiguous complex64 (MPA_C64) or complex128
    (MPA_C128) CUDA tensor, updated in place."""
    import torch
    prec = MPA_C64 if field.dtype == torch.complex64 else MPA_C128
    _check_field(field, prec, field.numel())
    m = _lib.MapStruct(dmmap)
    with torch.cuda.device(field.device):
        _lib.check(_lib.lib().ss_propagate(C.byref(m.s), int(field.numel()), float(dt), float(dz), int(prec),
                                           C.c_void_p(field.data_ptr()), float(z0), float(z1),
                                           _stream_handle(torch, field.device)))
    return field


class SSPlan:
    """ss_plan_create / ss_plan_propagate (Eq. 4)."""

    def __init__(self, n, dt, dmmap, dz, precision=MPA_C64, device=0):
        self.n, self.precision = int(n), int(precision)
        m = _lib.MapStruct(dmmap)
        h = C.c_void_p()
        _lib.check(_lib.lib().ss_plan_create(C.byref(m.s), int(n), float(dt), float(dz),
                                             int(precision), int(device), C.byref(h)))
        self._h = h

    def propagate(self, field, z0, z1):
        torch = _check_field(field, self.precision, self.n)
        _lib.check(_lib.lib().ss_plan_propagate(self._h, C.c_void_p(field.data_ptr()), float(z0),
                                                float(z1), _stream_handle(torch, field.device)))
        return field

    def close(self):
        if getattr(self, "_h", None):
            _lib.lib().ss_plan_destroy(self._h)
            self._h = None

    __del__ = close
