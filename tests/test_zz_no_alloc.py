"""mpa_propagate_noalloc (no plan, no device allocation: tables and the
march's second field in the library's per-device static scratch) against
mpa_propagate on a plan of the same parameters, through the C ABI: two
calls in a row, the second on a smaller field with another block size and
precision, then a third on a one-window field; the tolerances of the
oracle parity tests (FP32 1e-5, FP64 1e-10 relative L2); sizes beyond the
scratch and unsupported options are rejected before any device work."""
import ctypes as C

import numpy as np
import pytest

from tests.gpu_util import TOL_F32, TOL_F64, rel_l2, say, to_dev, to_host
from workloads import WORKLOADS, Grid, dm_map, wdm_field

pytestmark = pytest.mark.gpu

TOL = {0: TOL_F32, 1: TOL_F64}


def _pair(a, dt, dmmap, L, M, nit, block, halo, prec, band, z0, z1, shift=0):
    import paper_1101_0086_amd as P
    x = to_dev(a, prec)
    P.propagate_noalloc(x, dt, dmmap, L, M, nit, z0, z1, block, halo, prec, band, shift)
    got = to_host(x)
    plan = P.MPAPlan(a.size, dt, dmmap, L, M, nit, block, halo, prec, band, shift=shift)
    y = to_dev(a, prec)
    plan.propagate(y, z0, z1)
    ref = to_host(y)
    plan.close()
    return got, ref


def test_noalloc_matches_plan_march_on_successive_calls():
    w = WORKLOADS["wdm8_n262144_f32"]
    s = w.mpa
    a = w.field()
    # first call: the 2^18-mode bench field, 4096-blocks, across the span change at z = 0.5
    z0 = 0.5 - 5 * s.L
    say("noalloc 2^18 FP32", z0)
    got, ref = _pair(a, w.grid.dt, w.dmmap, s.L, s.M, s.n_iter, s.block, s.halo, 0, s.omega_band, z0,
                     z0 + 11 * s.L)
    assert rel_l2(got, ref) < TOL[0]
    # second call: a smaller field (2^15 modes), 1024-blocks with a window shift, FP64,
    # across an amplifier (the scratch keeps the first call's larger contents)
    dt = 10.0 / 1024
    b = wdm_field(Grid(1 << 15, dt), 32, 8, "ook", np.random.default_rng(5))
    L = 0.5 / 12000
    say("noalloc 2^15 FP64 shifted")
    got, ref = _pair(b, dt, dm_map(beta3=0.1), L, 2, 2, 1024, 128, 1, 145.0, 1.0 - 3 * L, 1.0 + 4 * L, shift=3)
    assert rel_l2(got, ref) < TOL[1]
    # third call: one 4096-mode window (the small FP64 workload), an odd number of
    # long steps (the result is copied back from the scratch field)
    v = WORKLOADS["dm1ch_n4096_f64"]
    say("noalloc full window")
    got, ref = _pair(v.field(), v.grid.dt, v.dmmap, v.mpa.L, v.mpa.M, v.mpa.n_iter, 0, 0, 1, 0.0, 0.4, 0.75)
    assert rel_l2(got, ref) < TOL[1]


def test_noalloc_rejections():
    from paper_1101_0086_amd import _lib as L
    from workloads.wdm import DMMap
    w = WORKLOADS["wdm8_n262144_f32"]
    s = w.mpa
    m = L.MapStruct(w.dmmap)
    lib = L.lib()

    def call(n, dmmap=None, **kw):
        base = dict(n=n, dt=w.grid.dt, L=s.L, M=s.M, n_iter=s.n_iter, block=s.block, halo=s.halo, precision=0,
                    omega_band=s.omega_band)
        base.update(kw)
        p = L.make_params(**base)
        mm = L.MapStruct(dmmap) if dmmap is not None else m
        return lib.mpa_propagate_noalloc(C.byref(p), C.byref(mm.s), C.c_void_p(1), 0.0, s.L, None)

    assert call(1 << 23) == L.MPA_EINVAL                          # 64 MiB field alone fills the scratch
    assert call(1 << 22, precision=1) == L.MPA_EINVAL
    raman = DMMap(**{**w.dmmap.__dict__, "raman_g0": 0.2, "raman_alpha": 3.0})
    assert call(1 << 18, dmmap=raman) == L.MPA_EUNSUPPORTED
    assert call(1 << 18, schedule=L.MPA_NODE_PARALLEL) == L.MPA_EUNSUPPORTED
    assert call(1 << 13, block=0, halo=0, L=0.05, M=16) == L.MPA_EUNSUPPORTED   # full window above 4096
    p = L.make_params(1 << 18, w.grid.dt, s.L, s.M, s.n_iter, s.block, s.halo, 0, s.omega_band)
    assert lib.mpa_propagate_noalloc(C.byref(p), C.byref(m.s), None, 0.0, s.L, None) == L.MPA_EINVAL
