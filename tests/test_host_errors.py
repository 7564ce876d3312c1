"""Argument checks of the C ABI that return before any GPU work: they run on
the host without a GPU (the library loads; nothing reaches the HIP runtime)."""
import ctypes
import os

import numpy as np
import pytest

from paper_2105_01865_amd import ch

LIB = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))),
                   "paper_2105_01865_amd", "libch.so")
pytestmark = pytest.mark.skipif(not os.path.exists(LIB), reason="libch.so not built")

OK, EINVAL, EUNSUPPORTED, EHANDLE = 0, -1, -4, -6


def _zf(n):
    return np.linspace(0.0, 1.0, n + 1)


def _interp(fine=(32, 32, 32), nc=(8, 8, 8), zf=None, prec=ch.CH_FP64):
    nx, ny, nz = fine
    g = ch.Grid(nx, ny, nz, 1.0 / nx)
    z = np.ascontiguousarray(_zf(nc[2]) if zf is None else zf, dtype=np.float64)
    h = ctypes.c_void_p()
    st = ch.lib().ch_interp_create(ctypes.byref(g), nc[0], nc[1], nc[2],
                                   z.ctypes.data_as(ch._PD), prec, ctypes.byref(h))
    return st, h


def test_interp_create_rejects_bad_meshes():
    assert _interp(prec=7)[0] == EINVAL
    assert _interp(nc=(3, 8, 8))[0] == EINVAL                   # fewer than 4 coarse cells
    bad = _zf(8)
    bad[0] = 0.1
    assert _interp(zf=bad)[0] == EINVAL                         # zf must start at 0
    bad = _zf(8)
    bad[3], bad[4] = bad[4], bad[3]
    assert _interp(zf=bad)[0] == EINVAL                         # zf must increase
    assert _interp(nc=(9000, 8, 8), prec=ch.CH_FP32)[0] == EUNSUPPORTED
    assert _interp(nc=(5000, 8, 8))[0] == EUNSUPPORTED          # 4096 in double
    assert _interp(fine=(8, 70000, 40000))[0] == EINVAL        # 32-bit item counts


def test_poisson_create_rejects_bad_meshes():
    h = ctypes.c_void_p()
    L = ch.lib()
    g = ch.Grid(1, 16, 16, 0.1)
    assert L.ch_poisson_create(ctypes.byref(g), 1, ch.CH_FP64, ctypes.byref(h)) == EINVAL
    g = ch.Grid(16, 16, 16, 0.0)
    assert L.ch_poisson_create(ctypes.byref(g), 0, ch.CH_FP64, ctypes.byref(h)) == EINVAL
    g = ch.Grid(16, 16, 16, 0.1)
    assert L.ch_poisson_create(ctypes.byref(g), 0, 5, ctypes.byref(h)) == EINVAL
    g = ch.Grid(4096, 4096, 4096, 1e-3)
    assert L.ch_poisson_create(ctypes.byref(g), 1, ch.CH_FP32, ctypes.byref(h)) == EUNSUPPORTED
    # under 2^31 cells, but an FP64 plane of 24000^2 cells is over 4 GiB
    g = ch.Grid(24000, 24000, 2, 1e-3)
    assert L.ch_poisson_create(ctypes.byref(g), 1, ch.CH_FP64, ctypes.byref(h)) == EUNSUPPORTED
    assert "4 GiB" in L.ch_last_error().decode()
    assert h.value is None


def test_calls_on_null_handles_report_a_bad_handle():
    L = ch.lib()
    n = ctypes.c_int64()
    assert L.ch_drops(None, 0.5, 0, ctypes.byref(n), None, None) == EHANDLE
    assert L.ch_batch_drops(None, 0, 0.5, 0, ctypes.byref(n), None, None) == EHANDLE
    t = ch.Tune()
    assert L.ch_autotune(None, None, None, None, 1e-4, 1, ctypes.byref(t)) == EHANDLE
    assert L.ch_batch_autotune(None, None, None, None, 1e-4, 1, ctypes.byref(t)) == EHANDLE
    assert L.ch_pressure_step(None, None, 1.0, 1.0, 1e-3, None, None, None, None, None) == EHANDLE
    assert L.ch_poisson_solve(None, None, None) == EHANDLE
    out = (ctypes.c_double * 3)()
    assert L.ch_interp_closure(None, out) == EHANDLE
    assert L.ch_interp_project_c(None, None, None) == EHANDLE
    assert L.ch_interp_set_solenoidal(None, 1) == EHANDLE
    assert "handle" in L.ch_last_error().decode()
    L.ch_poisson_destroy(None)      # NULL-safe
    L.ch_interp_destroy(None)


def test_create_rejects_bad_parameters_before_any_allocation():
    L = ch.lib()
    h = ctypes.c_void_p()
    g = ch.Grid(16, 16, 16, 1.0 / 16)
    cn = ctypes.c_double(-1.0)
    pe = ctypes.c_double(14.4)
    assert L.ch_create(ctypes.byref(g), cn, pe, None, None, None, ctypes.byref(h)) == EINVAL
    o = ch.make_opts(precision="fp32")
    o.kappa = float("nan")
    assert L.ch_create(ctypes.byref(g), 0.0625, 14.4, None, None, ctypes.byref(o),
                       ctypes.byref(h)) == EINVAL
    assert h.value is None
    for bad in (-1e-4, float("inf"), float("nan")):
        o = ch.make_opts(dt_hint=bad)
        assert L.ch_create(ctypes.byref(g), 0.0625, 14.4, None, None, ctypes.byref(o),
                           ctypes.byref(h)) == EINVAL
        assert "dt_hint" in L.ch_last_error().decode()
        assert h.value is None


def test_noalloc_mass_checks_arguments_before_any_gpu_call():
    L = ch.lib()
    fake = ctypes.c_void_p(0x1000)
    assert L.ch_mass_field_noalloc(fake, 0, 4, 4, 0.1, ch.CH_FP64, None, fake) == EINVAL
    assert L.ch_mass_field_noalloc(None, 4, 4, 4, 0.1, ch.CH_FP64, None, fake) == EINVAL
    assert L.ch_mass_field_noalloc(fake, 4, 4, 4, float("nan"), ch.CH_FP64, None, fake) == EINVAL
    # 2^32 cells is the limit of the scratch array's partial sums
    assert L.ch_mass_field_noalloc(fake, 4096, 4096, 257, 0.1, ch.CH_FP32, None, fake) == EINVAL
    assert "limit" in L.ch_last_error().decode()
