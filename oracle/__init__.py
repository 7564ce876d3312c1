"""FP64 CPU oracle of the Cahn-Hilliard update (arXiv 2105.01865).

TEST INFRASTRUCTURE.  Only the test-suite, ``__graft_entry__.smoke()`` and
the CPU-baseline leg of ``bench.py`` may import this package.  It wraps the
plain C implementation in ``ch_oracle.c`` / ``interp_oracle.c`` (built with
gcc into ``liboracle.so``) with ctypes, taking and returning numpy arrays of
shape (nz, ny, nx), x fastest, float64.  It shares no code with the GPU
library.

Boundary codes: 0 = periodic, 1 = no-flux (even reflection of C, zero normal
velocity on the wall faces).  Face-velocity arrays have n_d faces along their
own axis when that axis is periodic and n_d + 1 when it is no-flux.
"""
import ctypes
import os

import numpy as np

from . import build as _build
from . import pressure   # noqa: F401  (split-density pressure step, numpy)

PERIODIC = 0
NOFLUX = 1
PSI_DOUBLE_WELL = (0.0, 0.5, -1.5, 1.0)   # psi'(C) = C^3 - 1.5 C^2 + 0.5 C (eq-ch)

_lib = None
_D = ctypes.POINTER(ctypes.c_double)
_I64 = ctypes.POINTER(ctypes.c_int64)
_INT = ctypes.POINTER(ctypes.c_int)


def lib():
    global _lib
    if _lib is None:
        path = os.environ.get("CH_ORACLE_LIB", _build.TARGET)
        if path == _build.TARGET and not os.path.exists(path):
            _build.build()
        L = ctypes.CDLL(path)
        L.oracle_psi_prime.restype = ctypes.c_double
        L.oracle_psi_prime.argtypes = [ctypes.c_double, _D]
        L.oracle_weno5.restype = ctypes.c_double
        L.oracle_weno5.argtypes = [ctypes.c_double] * 6
        L.oracle_advection.argtypes = [_I64, _INT, ctypes.c_double, ctypes.c_double,
                                       _D, _D, _D, _D, _D]
        L.oracle_lap_mu.argtypes = [_I64, _INT, ctypes.c_double, _D, _D, _D]
        L.oracle_biharm.argtypes = [_I64, _INT, ctypes.c_double, ctypes.c_double,
                                    ctypes.c_double, _D, _D]
        L.oracle_biharm25.argtypes = [_I64, _INT, ctypes.c_double, ctypes.c_double, _D, _D]
        L.oracle_explicit.argtypes = [_I64, _INT, ctypes.c_double, ctypes.c_double, _D,
                                      ctypes.c_double, _D, _D, _D, _D, _D]
        L.oracle_line_solve.restype = ctypes.c_int
        L.oracle_line_solve.argtypes = [ctypes.c_int64, ctypes.c_double, ctypes.c_int, _D, _D]
        L.oracle_step.restype = ctypes.c_int
        L.oracle_step.argtypes = [_I64, _INT, ctypes.c_double, ctypes.c_double,
                                  ctypes.c_double, _D, ctypes.c_double, ctypes.c_double,
                                  _D, _D, _D, _D, ctypes.c_double, ctypes.c_int]
        L.oracle_step_explicit25.restype = ctypes.c_int
        L.oracle_step_explicit25.argtypes = [_I64, _INT, ctypes.c_double, ctypes.c_double,
                                             ctypes.c_double, _D, ctypes.c_double, _D,
                                             _D, _D, _D, ctypes.c_double, ctypes.c_int]
        L.oracle_threads.restype = ctypes.c_int
        L.oracle_threads.argtypes = []
        L.oracle_set_threads.restype = None
        L.oracle_set_threads.argtypes = [ctypes.c_int]
        L.oracle_mass.restype = ctypes.c_double
        L.oracle_mass.argtypes = [ctypes.c_int64, ctypes.c_double, _D]
        L.oracle_hermite_stencil.argtypes = [ctypes.c_int64, _D, ctypes.c_double, ctypes.c_int,
                                             ctypes.c_double, _I64, _D]
        L.oracle_interp_velocity.restype = ctypes.c_int
        L.oracle_interp_velocity.argtypes = [_I64, _D, _D, _D, _D, _I64, _D, _D, _D]
        L.oracle_solenoidal_velocity.restype = ctypes.c_int
        L.oracle_solenoidal_velocity.argtypes = [_I64, _D, _D, _D, _D, _I64, _D, _D, _D, _D]
        L.oracle_project_c.restype = ctypes.c_int
        L.oracle_label_drops.restype = ctypes.c_int64
        L.oracle_label_drops.argtypes = [_I64, _INT, _D, ctypes.c_double, _I64]
        L.oracle_project_c.argtypes = [_I64, _D, _I64, _D, _D]
        _lib = L
    return _lib


def _dp(a):
    return a.ctypes.data_as(_D)


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def _dims(C):
    nz, ny, nx = C.shape
    return (ctypes.c_int64 * 3)(nx, ny, nz)


def _bc(bc):
    return (ctypes.c_int * 3)(*[int(b) for b in bc])


def _check_vel(C, u, v, w, bc):
    nz, ny, nx = C.shape
    fx = nx if bc[0] == PERIODIC else nx + 1
    fy = ny if bc[1] == PERIODIC else ny + 1
    fz = nz if bc[2] == PERIODIC else nz + 1
    assert u.shape == (nz, ny, fx), (u.shape, (nz, ny, fx))
    assert v.shape == (nz, fy, nx), (v.shape, (nz, fy, nx))
    assert w.shape == (fz, ny, nx), (w.shape, (fz, ny, nx))


def psi_prime(C, psi=PSI_DOUBLE_WELL):
    p = (ctypes.c_double * 4)(*psi)
    return lib().oracle_psi_prime(float(C), p)


def weno5(a, b, c, d, e, eps=1e-6):
    return lib().oracle_weno5(float(a), float(b), float(c), float(d), float(e), float(eps))


def advection(C, u, v, w, h, bc=(0, 0, 0), eps=1e-6):
    """div(u C) per cell."""
    C, u, v, w = map(_f64, (C, u, v, w))
    _check_vel(C, u, v, w, bc)
    out = np.empty_like(C)
    lib().oracle_advection(_dims(C), _bc(bc), h, eps, _dp(C), _dp(u), _dp(v), _dp(w), _dp(out))
    return out


def lap_mu(C, h, bc=(0, 0, 0), psi=PSI_DOUBLE_WELL):
    """7-point Laplacian of psi'(C)."""
    C = _f64(C)
    out = np.empty_like(C)
    lib().oracle_lap_mu(_dims(C), _bc(bc), h, (ctypes.c_double * 4)(*psi), _dp(C), _dp(out))
    return out


def biharm(C, h, Cn, kappa=4.0, bc=(0, 0, 0)):
    """New-scheme biharmonic sum_d A_d C (eq-a3d; kappa = 2 gives eq-a2d)."""
    C = _f64(C)
    out = np.empty_like(C)
    lib().oracle_biharm(_dims(C), _bc(bc), h, Cn, kappa, _dp(C), _dp(out))
    return out


def biharm25(C, h, Cn, bc=(0, 0, 0)):
    """Standard 25-point biharmonic Cn^2 lap_h^2 C (eq-disbi in 3-D)."""
    C = _f64(C)
    out = np.empty_like(C)
    lib().oracle_biharm25(_dims(C), _bc(bc), h, Cn, _dp(C), _dp(out))
    return out


def explicit(C, u, v, w, h, Pe, bc=(0, 0, 0), psi=PSI_DOUBLE_WELL, eps=1e-6):
    """E = -div(u C) + lap psi'(C) / Pe."""
    C, u, v, w = map(_f64, (C, u, v, w))
    _check_vel(C, u, v, w, bc)
    out = np.empty_like(C)
    lib().oracle_explicit(_dims(C), _bc(bc), h, Pe, (ctypes.c_double * 4)(*psi), eps,
                          _dp(C), _dp(u), _dp(v), _dp(w), _dp(out))
    return out


def line_solve(b, r, bc=PERIODIC):
    """Solve (I + r D4) y = b on one line."""
    b = _f64(b)
    y = np.empty_like(b)
    rc = lib().oracle_line_solve(b.size, r, int(bc), _dp(b), _dp(y))
    if rc:
        raise RuntimeError("oracle_line_solve failed")
    return y


def step(C, u, v, w, h, Cn, Pe, dt, nsteps=1, bc=(0, 0, 0), kappa=4.0,
         psi=PSI_DOUBLE_WELL, eps=1e-6):
    """nsteps RK3/CN/AF steps; returns the new C (input untouched)."""
    C = np.array(C, dtype=np.float64, order="C", copy=True)
    u, v, w = map(_f64, (u, v, w))
    _check_vel(C, u, v, w, bc)
    rc = lib().oracle_step(_dims(C), _bc(bc), h, Cn, Pe, (ctypes.c_double * 4)(*psi),
                           kappa, eps, _dp(C), _dp(u), _dp(v), _dp(w), dt, int(nsteps))
    if rc:
        raise RuntimeError("oracle_step failed")
    return C


def step_explicit25(C, u, v, w, h, Cn, Pe, dt, nsteps=1, bc=(0, 0, 0),
                    psi=PSI_DOUBLE_WELL, eps=1e-6):
    """nsteps RK3 steps with the explicit 25-point biharmonic (no solves)."""
    C = np.array(C, dtype=np.float64, order="C", copy=True)
    u, v, w = map(_f64, (u, v, w))
    _check_vel(C, u, v, w, bc)
    rc = lib().oracle_step_explicit25(_dims(C), _bc(bc), h, Cn, Pe,
                                      (ctypes.c_double * 4)(*psi), eps, _dp(C),
                                      _dp(u), _dp(v), _dp(w), dt, int(nsteps))
    if rc:
        raise RuntimeError("oracle_step_explicit25 failed")
    return C


def threads():
    """Threads the oracle's parallel loops use."""
    return lib().oracle_threads()


def set_threads(n):
    """Threads for the oracle's parallel loops from now on (0: one per
    processor)."""
    lib().oracle_set_threads(int(n))


def mass(C, h):
    """h^3 sum C, pairwise in a fixed order."""
    C = _f64(C)
    return lib().oracle_mass(C.size, h, _dp(C))


AX_PERIODIC, AX_WALL_EVEN, AX_WALL_ODD = 0, 1, 2


def hermite_stencil(s, L, kind, t):
    """Four source indices and weights interpolating at coordinate t."""
    s = _f64(s)
    idx = (ctypes.c_int64 * 4)()
    wt = (ctypes.c_double * 4)()
    lib().oracle_hermite_stencil(s.size, _dp(s), L, int(kind), float(t), idx, wt)
    return np.array(idx[:], dtype=np.int64), np.array(wt[:])


def interp_velocity(zf, uc, vc, wc, nf):
    """Coarse stretched-z staggered velocity -> fine uniform staggered velocity.

    zf: coarse z faces (ncz+1,) from 0 to 1; uc, vc: (ncz, ncy, ncx);
    wc: (ncz+1, ncy, ncx); nf = (nfx, nfy, nfz).  Returns uf, vf (nfz, nfy, nfx)
    and wf (nfz+1, nfy, nfx).
    """
    zf, uc, vc, wc = map(_f64, (zf, uc, vc, wc))
    ncz, ncy, ncx = uc.shape
    assert vc.shape == uc.shape and wc.shape == (ncz + 1, ncy, ncx) and zf.shape == (ncz + 1,)
    nfx, nfy, nfz = nf
    uf = np.empty((nfz, nfy, nfx))
    vf = np.empty((nfz, nfy, nfx))
    wf = np.empty((nfz + 1, nfy, nfx))
    rc = lib().oracle_interp_velocity((ctypes.c_int64 * 3)(ncx, ncy, ncz), _dp(zf), _dp(uc),
                                      _dp(vc), _dp(wc), (ctypes.c_int64 * 3)(nfx, nfy, nfz),
                                      _dp(uf), _dp(vf), _dp(wf))
    if rc:
        raise RuntimeError("oracle_interp_velocity failed")
    return uf, vf, wf


def solenoidal_velocity(zf, uc, vc, wc, nf):
    """The solenoidal variant of the transfer (sec. 3.4): coarse normal
    gradients interpolated to the fine cell centres, each component
    integrated along its direction from its reference plane (u on x = 0, v on
    y = 0, w = 0 on the bottom wall; the top wall stays 0).  Shapes as in
    interp_velocity.  Returns uf, vf, wf and the largest |closure sum| of the
    x, y and z lines."""
    zf, uc, vc, wc = map(_f64, (zf, uc, vc, wc))
    ncz, ncy, ncx = uc.shape
    assert vc.shape == uc.shape and wc.shape == (ncz + 1, ncy, ncx) and zf.shape == (ncz + 1,)
    nfx, nfy, nfz = nf
    uf = np.empty((nfz, nfy, nfx))
    vf = np.empty((nfz, nfy, nfx))
    wf = np.empty((nfz + 1, nfy, nfx))
    resid = np.zeros(3)
    rc = lib().oracle_solenoidal_velocity((ctypes.c_int64 * 3)(ncx, ncy, ncz), _dp(zf), _dp(uc),
                                          _dp(vc), _dp(wc), (ctypes.c_int64 * 3)(nfx, nfy, nfz),
                                          _dp(uf), _dp(vf), _dp(wf), _dp(resid))
    if rc:
        raise RuntimeError("oracle_solenoidal_velocity failed")
    return uf, vf, wf, resid


def project_c(Cf, zf, nc):
    """Back-coupling of C (sec. 3.4): fine cell-centred C -> coarse cell
    centres (ncx, ncy, ncz) of the stretched mesh with faces zf."""
    Cf, zf = _f64(Cf), _f64(zf)
    nfz, nfy, nfx = Cf.shape
    ncx, ncy, ncz = nc
    assert zf.shape == (ncz + 1,)
    Cc = np.empty((ncz, ncy, ncx))
    rc = lib().oracle_project_c((ctypes.c_int64 * 3)(nfx, nfy, nfz), _dp(Cf),
                                (ctypes.c_int64 * 3)(ncx, ncy, ncz), _dp(zf), _dp(Cc))
    if rc:
        raise RuntimeError("oracle_project_c failed")
    return Cc


def label_drops(C, thr=0.5, bc=(PERIODIC, PERIODIC, PERIODIC)):
    """Drops of C (nz, ny, nx): face-connected cells with C >= thr, periodic
    axes wrapping.  Returns (label, ndrops): label[p] is the smallest linear
    index of p's drop, -1 below the threshold."""
    C = _f64(C)
    label = np.empty(C.shape, dtype=np.int64)
    nd = lib().oracle_label_drops(_dims(C), _bc(bc), _dp(C), float(thr),
                                  label.ctypes.data_as(_I64))
    if nd < 0:
        raise RuntimeError("oracle_label_drops failed")
    return label, int(nd)


def drop_volumes(label, h):
    """(root, cells, V, D) of every drop, sorted by root (the smallest linear
    index), with V = h^3 cells and D from (4 pi / 3)(D/2)^3 = V."""
    roots, cells = np.unique(label[label >= 0], return_counts=True)
    V = cells * h ** 3
    D = np.cbrt(6.0 * V / np.pi)
    return roots, cells, V, D
