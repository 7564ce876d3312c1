"""Python binding of libch (include/ch.h): argument marshalling only.

Every step of the Cahn-Hilliard update runs in the library's HIP kernels;
this module checks shapes and dtypes on the host, passes raw device
pointers of torch tensors, and orders the library's stream after torch's
current stream (and back).  It raises if libch.so is not built -- there is
no fallback.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np
import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libch.so")

CH_PERIODIC, CH_NOFLUX = 0, 1
CH_FP64, CH_FP32 = 0, 1
SOLVE = {"auto": 0, "fp64": 1, "native": 2}
STATUS = {0: "CH_OK", -1: "CH_EINVAL", -2: "CH_ENOMEM", -3: "CH_EHIP", -4: "CH_EUNSUPPORTED",
          -5: "CH_ENONFINITE", -6: "CH_EHANDLE"}
KERNELS = {"x": 0, "y": 1, "z": 2, "interp": 3}


class CHError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{STATUS.get(status, status)}: {msg}")
        self.status = status


class Grid(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int64), ("ny", ctypes.c_int64), ("nz", ctypes.c_int64),
                ("h", ctypes.c_double)]


class Psi(ctypes.Structure):
    _fields_ = [("c", ctypes.c_double * 4)]


class BC(ctypes.Structure):
    _fields_ = [("x", ctypes.c_int), ("y", ctypes.c_int), ("z", ctypes.c_int)]


class Opts(ctypes.Structure):
    _fields_ = [("precision", ctypes.c_int), ("kappa", ctypes.c_double),
                ("weno_eps", ctypes.c_double), ("solve_fp64", ctypes.c_int),
                ("use_graph", ctypes.c_int), ("x_rows", ctypes.c_int),
                ("seg_len", ctypes.c_int), ("waves_yz", ctypes.c_int),
                ("z_chunk", ctypes.c_int), ("x_general", ctypes.c_int),
                ("dt_hint", ctypes.c_double)]


_lib = None
_VP = ctypes.c_void_p
_I = ctypes.c_int
_D = ctypes.c_double
_PD = ctypes.POINTER(ctypes.c_double)
_PI64 = ctypes.POINTER(ctypes.c_int64)

# name -> (restype, argtypes); kept in the order of include/ch.h
class Tune(ctypes.Structure):
    _fields_ = [("x_rows", ctypes.c_int), ("z_chunk", ctypes.c_int),
                ("ms_per_step", ctypes.c_double), ("auto_ms_per_step", ctypes.c_double),
                ("candidates", ctypes.c_int), ("seg_len", ctypes.c_int)]


def _tune_dict(t):
    return {"x_rows": t.x_rows, "z_chunk": t.z_chunk, "ms_per_step": t.ms_per_step,
            "auto_ms_per_step": t.auto_ms_per_step, "candidates": t.candidates,
            "seg_len": t.seg_len}


SIGNATURES = {
    "ch_default_opts": (None, [ctypes.POINTER(Opts)]),
    "ch_create": (_I, [ctypes.POINTER(Grid), _D, _D, ctypes.POINTER(Psi), ctypes.POINTER(BC),
                       ctypes.POINTER(Opts), ctypes.POINTER(_VP)]),
    "ch_set_stream": (_I, [_VP, _VP]),
    "ch_set_field": (_I, [_VP, _VP, _I]),
    "ch_get_field": (_I, [_VP, _VP, _I]),
    "ch_step": (_I, [_VP, _VP, _VP, _VP, _D, _I]),
    "ch_step_explicit25": (_I, [_VP, _VP, _VP, _VP, _D, _I]),
    "ch_mass": (_I, [_VP, _PD]),
    "ch_mass_field_noalloc": (_I, [_VP, ctypes.c_int64, ctypes.c_int64, ctypes.c_int64, _D, _I,
                                   _VP, _VP]),
    "ch_check_velocity": (_I, [_VP, _VP, _VP, _VP]),
    "ch_destroy": (None, [_VP]),
    "ch_last_error": (ctypes.c_char_p, []),
    "ch_batch_create": (_I, [_I, ctypes.POINTER(Grid), _PD, _PD, ctypes.POINTER(Psi),
                             ctypes.POINTER(BC), ctypes.POINTER(Opts), ctypes.POINTER(_VP)]),
    "ch_batch_field_offsets": (_I, [_VP, _PI64, _PI64, _PI64, _PI64, _PI64]),
    "ch_batch_set_stream": (_I, [_VP, _VP]),
    "ch_batch_set_field": (_I, [_VP, _VP, _I]),
    "ch_batch_get_field": (_I, [_VP, _VP, _I]),
    "ch_batch_step": (_I, [_VP, _VP, _VP, _VP, _D, _I]),
    "ch_batch_mass": (_I, [_VP, _PD]),
    "ch_batch_destroy": (None, [_VP]),
    "ch_interp_create": (_I, [ctypes.POINTER(Grid), ctypes.c_int64, ctypes.c_int64,
                              ctypes.c_int64, _PD, _I, ctypes.POINTER(_VP)]),
    "ch_interp_set_stream": (_I, [_VP, _VP]),
    "ch_interp_apply": (_I, [_VP, _VP, _VP, _VP, _VP, _VP, _VP]),
    "ch_interp_destroy": (None, [_VP]),
    "ch_autotune": (_I, [_VP, _VP, _VP, _VP, _D, _I, ctypes.POINTER(Tune)]),
    "ch_batch_autotune": (_I, [_VP, _VP, _VP, _VP, _D, _I, ctypes.POINTER(Tune)]),
    "ch_drops": (_I, [_VP, _D, ctypes.c_int64, ctypes.POINTER(ctypes.c_int64),
                      ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(ctypes.c_int64)]),
    "ch_batch_drops": (_I, [_VP, _I, _D, ctypes.c_int64, ctypes.POINTER(ctypes.c_int64),
                            ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(ctypes.c_int64)]),
    "ch_poisson_create": (_I, [ctypes.POINTER(Grid), _I, _I, ctypes.POINTER(_VP)]),
    "ch_poisson_set_stream": (_I, [_VP, _VP]),
    "ch_poisson_solve": (_I, [_VP, _VP, _VP]),
    "ch_pressure_step": (_I, [_VP, _VP, _D, _D, _D, _VP, _VP, _VP, _VP, _VP]),
    "ch_poisson_destroy": (None, [_VP]),
    "ch_interp_set_solenoidal": (_I, [_VP, _I]),
    "ch_interp_closure": (_I, [_VP, ctypes.POINTER(_D)]),
    "ch_interp_project_c": (_I, [_VP, _VP, _VP]),
    "ch_step_multires": (_I, [_VP, _VP, _VP, _VP, _VP, _D, _I]),
    "ch_profile_enable": (_I, [_VP, _I]),
    "ch_profile_read": (_I, [_VP, _I, _PD, _PI64]),
    "ch_batch_profile_enable": (_I, [_VP, _I]),
    "ch_batch_profile_read": (_I, [_VP, _I, _PD, _PI64]),
    "ch_get_config": (_I, [_VP, ctypes.POINTER(ctypes.c_int)]),
    "ch_get_x_program": (_I, [_VP, ctypes.POINTER(ctypes.c_int)]),
    "ch_batch_get_x_program": (_I, [_VP, ctypes.POINTER(ctypes.c_int)]),
}

# x-pass program kinds reported by ch_get_x_program
X_PROGRAMS = {0: "general", 1: "row", 2: "row, several rows per task", 3: "segmented",
              4: "row, one launch per row mode (two or three)"}


def lib():
    """Load libch.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is not built: run `python -m "
                               "paper_2105_01865_amd.build` (there is no CPU fallback)")
        L = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def _check(status):
    if status != 0:
        raise CHError(status, lib().ch_last_error().decode())


def _dtype(precision):
    return torch.float64 if precision == CH_FP64 else torch.float32


def _prec(p):
    if p in ("fp64", "f64", CH_FP64, torch.float64):
        return CH_FP64
    if p in ("fp32", "f32", CH_FP32, torch.float32):
        return CH_FP32
    raise ValueError(f"unknown precision {p!r}")


def make_opts(precision="fp64", kappa=4.0, weno_eps=1e-6, solve="auto", use_graph=True,
              x_rows=0, seg_len=0, waves_yz=0, z_chunk=0, dt_hint=0.0, x_general=False):
    o = Opts()
    lib().ch_default_opts(ctypes.byref(o))
    o.precision = _prec(precision)
    o.kappa = kappa
    o.weno_eps = weno_eps
    o.solve_fp64 = SOLVE[solve]
    o.use_graph = 1 if use_graph else 0
    o.x_rows, o.seg_len, o.waves_yz, o.z_chunk = x_rows, seg_len, waves_yz, z_chunk
    o.dt_hint = float(dt_hint)
    o.x_general = 1 if x_general else 0
    return o


def mass_field_noalloc(C, h, out, stream=None):
    """ch_mass_field_noalloc: h^3 sum C of the CUDA tensor C (nz, ny, nx),
    FP64 or FP32, written to the one-element float64 CUDA tensor `out` on
    `stream` (the current stream if None), without allocating."""
    if C.dim() != 3:
        raise ValueError("C must be (nz, ny, nx)")
    prec = _prec(C.dtype)
    p = _dev_tensor(C, C.dtype, tuple(C.shape), "C")
    if not (isinstance(out, torch.Tensor) and out.is_cuda and out.dtype == torch.float64
            and out.numel() >= 1):
        raise ValueError("out must be a float64 CUDA tensor")
    st = stream if stream is not None else torch.cuda.current_stream()
    nz, ny, nx = C.shape
    _check(lib().ch_mass_field_noalloc(p, nx, ny, nz, float(h), prec,
                                       ctypes.c_void_p(st.cuda_stream),
                                       ctypes.c_void_p(out.data_ptr())))


def _dev_tensor(t, dtype, shape, name):
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise ValueError(f"{name} must be a CUDA tensor")
    if t.dtype != dtype:
        raise ValueError(f"{name} has dtype {t.dtype}, expected {dtype}")
    if tuple(t.shape) != tuple(shape):
        raise ValueError(f"{name} has shape {tuple(t.shape)}, expected {tuple(shape)}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    return ctypes.c_void_p(t.data_ptr())


def _host_tensor(t, dtype, shape, name):
    if not isinstance(t, torch.Tensor) or t.device.type != "cpu":
        raise ValueError(f"{name} must be a CPU tensor")
    if t.dtype != dtype:
        raise ValueError(f"{name} has dtype {t.dtype}, expected {dtype}")
    if tuple(t.shape) != tuple(shape):
        raise ValueError(f"{name} has shape {tuple(t.shape)}, expected {tuple(shape)}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    return ctypes.c_void_p(t.data_ptr())


def _drops_call(fn, args, cap):
    """Run ch_drops / ch_batch_drops, growing the host arrays once if the
    box has more than `cap` drops.  Returns (root, cells) int64 arrays."""
    while True:
        nd = ctypes.c_int64()
        root = np.zeros(max(cap, 1), dtype=np.int64)
        cells = np.zeros(max(cap, 1), dtype=np.int64)
        P64 = ctypes.POINTER(ctypes.c_int64)
        _check(fn(*args, cap, ctypes.byref(nd), root.ctypes.data_as(P64),
                  cells.ctypes.data_as(P64)))
        if nd.value <= cap:
            return root[:nd.value], cells[:nd.value]
        cap = nd.value


class _StreamMixin:
    """Orders the library's stream after torch's current stream and back."""

    def _enter(self):
        if self.stream is not None:
            self.stream.wait_stream(torch.cuda.current_stream())

    def _leave(self):
        if self.stream is not None:
            torch.cuda.current_stream().wait_stream(self.stream)


class State(_StreamMixin):
    """One box: C of shape (nz, ny, nx) on the current device."""

    def __init__(self, shape, h, Cn, Pe, psi=None, bc=(0, 0, 0), stream=None, **opts):
        nz, ny, nx = shape
        self.shape = (nz, ny, nx)
        self.bc = tuple(int(b) for b in bc)
        self.h = float(h)
        self.opts = make_opts(**opts)
        self.dtype = _dtype(self.opts.precision)
        g = Grid(nx, ny, nz, h)
        p = Psi((ctypes.c_double * 4)(*psi)) if psi is not None else None
        b = BC(*self.bc)
        handle = ctypes.c_void_p()
        _check(lib().ch_create(ctypes.byref(g), Cn, Pe, ctypes.byref(p) if p else None,
                               ctypes.byref(b), ctypes.byref(self.opts), ctypes.byref(handle)))
        self._h = handle
        self.stream = None
        self.set_stream(stream)

    # faces per axis
    def vel_shapes(self):
        nz, ny, nx = self.shape
        fx = nx + (self.bc[0] == CH_NOFLUX)
        fy = ny + (self.bc[1] == CH_NOFLUX)
        fz = nz + (self.bc[2] == CH_NOFLUX)
        return (nz, ny, fx), (nz, fy, nx), (fz, ny, nx)

    def set_stream(self, stream):
        self.stream = stream
        _check(lib().ch_set_stream(self._h, ctypes.c_void_p(stream.cuda_stream if stream else 0)))

    def set_field(self, C):
        if isinstance(C, np.ndarray):
            C = torch.from_numpy(np.ascontiguousarray(C)).to(device="cuda", dtype=self.dtype)
        ptr = _dev_tensor(C, self.dtype, self.shape, "C")
        self._enter()
        _check(lib().ch_set_field(self._h, ptr, 1))
        self._leave()
        torch.cuda.current_stream().synchronize()

    def get_field(self):
        out = torch.empty(self.shape, dtype=self.dtype, device="cuda")
        self._enter()
        _check(lib().ch_get_field(self._h, ctypes.c_void_p(out.data_ptr()), 1))
        self._leave()
        return out

    def set_field_host(self, C):
        """Copy C in from host memory (a CPU tensor; pinned memory copies
        fastest).  Returns once the copy is done."""
        ptr = _host_tensor(C, self.dtype, self.shape, "C")
        self._enter()
        _check(lib().ch_set_field(self._h, ptr, 0))
        self._leave()

    def get_field_host(self, out=None):
        """Copy C out into host memory (`out`, or a new pinned CPU tensor)."""
        if out is None:
            out = torch.empty(self.shape, dtype=self.dtype, pin_memory=True)
        ptr = _host_tensor(out, self.dtype, self.shape, "out")
        self._enter()
        _check(lib().ch_get_field(self._h, ptr, 0))
        self._leave()
        return out

    def step(self, u, v, w, dt, nsteps=1):
        su, sv, sw = self.vel_shapes()
        pu = _dev_tensor(u, self.dtype, su, "u")
        pv = _dev_tensor(v, self.dtype, sv, "v")
        pw = _dev_tensor(w, self.dtype, sw, "w")
        self._enter()
        _check(lib().ch_step(self._h, pu, pv, pw, float(dt), int(nsteps)))
        self._leave()

    def step_explicit25(self, u, v, w, dt, nsteps=1):
        """Steps of the explicit 25-point scheme (no line solves)."""
        su, sv, sw = self.vel_shapes()
        pu = _dev_tensor(u, self.dtype, su, "u")
        pv = _dev_tensor(v, self.dtype, sv, "v")
        pw = _dev_tensor(w, self.dtype, sw, "w")
        self._enter()
        _check(lib().ch_step_explicit25(self._h, pu, pv, pw, float(dt), int(nsteps)))
        self._leave()

    def step_multires(self, interp, uc, vc, wc, dt, nsteps=1):
        self._enter()
        _check(lib().ch_step_multires(self._h, interp._h, *interp._coarse_ptrs(uc, vc, wc),
                                      float(dt), int(nsteps)))
        self._leave()

    def mass(self):
        out = ctypes.c_double()
        self._enter()
        _check(lib().ch_mass(self._h, ctypes.byref(out)))
        return out.value

    def autotune(self, u, v, w, dt, steps=5):
        """Time the candidate launch plans, keep the fastest (C is restored)."""
        su, sv, sw = self.vel_shapes()
        t = Tune()
        self._enter()
        _check(lib().ch_autotune(self._h, _dev_tensor(u, self.dtype, su, "u"),
                                 _dev_tensor(v, self.dtype, sv, "v"),
                                 _dev_tensor(w, self.dtype, sw, "w"), float(dt), int(steps),
                                 ctypes.byref(t)))
        return _tune_dict(t)

    def drops(self, threshold=0.5, cap=4096):
        """(root, cells) of every drop (face-connected cells with
        C >= threshold), sorted by root; V = h^3 cells."""
        self._enter()
        return _drops_call(lib().ch_drops, (self._h, float(threshold)), cap)

    def check_velocity(self, u, v, w):
        su, sv, sw = self.vel_shapes()
        self._enter()
        _check(lib().ch_check_velocity(self._h, _dev_tensor(u, self.dtype, su, "u"),
                                       _dev_tensor(v, self.dtype, sv, "v"),
                                       _dev_tensor(w, self.dtype, sw, "w")))

    def profile(self, on=True):
        _check(lib().ch_profile_enable(self._h, 1 if on else 0))

    def profile_read(self, kernel):
        ms = ctypes.c_double()
        n = ctypes.c_int64()
        _check(lib().ch_profile_read(self._h, KERNELS.get(kernel, kernel), ctypes.byref(ms),
                                     ctypes.byref(n)))
        return ms.value, n.value

    def config(self):
        cfg = (ctypes.c_int * 8)()
        _check(lib().ch_get_config(self._h, cfg))
        return dict(x_rows=cfg[0], seg=cfg[1], yz_threads=cfg[2], tw=list(cfg[3:6]),
                    acc64=bool(cfg[6]), z_chunk=cfg[7])

    def x_program(self):
        """The x-pass program of the current plan (a key of X_PROGRAMS)."""
        k = ctypes.c_int()
        _check(lib().ch_get_x_program(self._h, ctypes.byref(k)))
        return k.value

    def close(self):
        if getattr(self, "_h", None):
            lib().ch_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Batch(_StreamMixin):
    """Independent boxes advanced together; fields are packed 1-D tensors."""

    def __init__(self, shapes, hs, Cns, Pes, bcs=None, stream=None, **opts):
        n = len(shapes)
        self.shapes = [tuple(s) for s in shapes]
        self.bcs = [tuple(b) for b in (bcs or [(0, 0, 0)] * n)]
        self.opts = make_opts(**opts)
        self.dtype = _dtype(self.opts.precision)
        grids = (Grid * n)(*[Grid(s[2], s[1], s[0], h) for s, h in zip(self.shapes, hs)])
        cn = (ctypes.c_double * n)(*Cns)
        pe = (ctypes.c_double * n)(*Pes)
        bc = (BC * n)(*[BC(*b) for b in self.bcs])
        handle = ctypes.c_void_p()
        _check(lib().ch_batch_create(n, grids, cn, pe, None, bc, ctypes.byref(self.opts),
                                     ctypes.byref(handle)))
        self._h = handle
        self.nbox = n
        offs = [(ctypes.c_int64 * n)() for _ in range(4)]
        tot = (ctypes.c_int64 * 4)()
        _check(lib().ch_batch_field_offsets(self._h, *offs, tot))
        self.c_off, self.u_off, self.v_off, self.w_off = ([int(x) for x in o] for o in offs)
        self.totals = [int(x) for x in tot]
        self.stream = None
        self.set_stream(stream)

    def set_stream(self, stream):
        self.stream = stream
        _check(lib().ch_batch_set_stream(self._h,
                                         ctypes.c_void_p(stream.cuda_stream if stream else 0)))

    def vel_shapes(self, b):
        nz, ny, nx = self.shapes[b]
        bc = self.bcs[b]
        return ((nz, ny, nx + (bc[0] == 1)), (nz, ny + (bc[1] == 1), nx),
                (nz + (bc[2] == 1), ny, nx))

    def pack(self, arrays, which):
        """Pack per-box arrays (numpy or torch) into one device tensor."""
        tot = self.totals["cuvw".index(which)]
        out = torch.empty(tot, dtype=self.dtype, device="cuda")
        offs = {"c": self.c_off, "u": self.u_off, "v": self.v_off, "w": self.w_off}[which]
        for o, a in zip(offs, arrays):
            t = torch.as_tensor(np.ascontiguousarray(a) if isinstance(a, np.ndarray) else a)
            t = t.to(device="cuda", dtype=self.dtype).reshape(-1)
            out[o:o + t.numel()] = t
        return out

    def unpack(self, packed):
        return [packed[o:o + int(np.prod(s))].reshape(s) for o, s in zip(self.c_off, self.shapes)]

    def set_field(self, C_packed):
        ptr = _dev_tensor(C_packed, self.dtype, (self.totals[0],), "C")
        self._enter()
        _check(lib().ch_batch_set_field(self._h, ptr, 1))
        self._leave()
        torch.cuda.current_stream().synchronize()

    def get_field(self):
        out = torch.empty(self.totals[0], dtype=self.dtype, device="cuda")
        self._enter()
        _check(lib().ch_batch_get_field(self._h, ctypes.c_void_p(out.data_ptr()), 1))
        self._leave()
        return out

    def set_field_host(self, C_packed):
        """Copy the packed C in from host memory; returns once it is done."""
        ptr = _host_tensor(C_packed, self.dtype, (self.totals[0],), "C")
        self._enter()
        _check(lib().ch_batch_set_field(self._h, ptr, 0))
        self._leave()

    def get_field_host(self, out=None):
        """Copy the packed C out into host memory (`out`, or a new pinned tensor)."""
        if out is None:
            out = torch.empty(self.totals[0], dtype=self.dtype, pin_memory=True)
        ptr = _host_tensor(out, self.dtype, (self.totals[0],), "out")
        self._enter()
        _check(lib().ch_batch_get_field(self._h, ptr, 0))
        self._leave()
        return out

    def step(self, u, v, w, dt, nsteps=1):
        pu = _dev_tensor(u, self.dtype, (self.totals[1],), "u")
        pv = _dev_tensor(v, self.dtype, (self.totals[2],), "v")
        pw = _dev_tensor(w, self.dtype, (self.totals[3],), "w")
        self._enter()
        _check(lib().ch_batch_step(self._h, pu, pv, pw, float(dt), int(nsteps)))
        self._leave()

    def autotune(self, u, v, w, dt, steps=5):
        """Time the candidate launch plans on the packed velocity, keep the
        fastest (C is restored)."""
        t = Tune()
        self._enter()
        _check(lib().ch_batch_autotune(self._h, _dev_tensor(u, self.dtype, (self.totals[1],), "u"),
                                       _dev_tensor(v, self.dtype, (self.totals[2],), "v"),
                                       _dev_tensor(w, self.dtype, (self.totals[3],), "w"),
                                       float(dt), int(steps), ctypes.byref(t)))
        return _tune_dict(t)

    def drops(self, box, threshold=0.5, cap=4096):
        """(root, cells) of the drops of box `box`, sorted by root."""
        self._enter()
        return _drops_call(lib().ch_batch_drops, (self._h, int(box), float(threshold)), cap)

    def mass(self):
        out = (ctypes.c_double * self.nbox)()
        self._enter()
        _check(lib().ch_batch_mass(self._h, out))
        return [float(x) for x in out]

    def profile(self, on=True):
        _check(lib().ch_batch_profile_enable(self._h, 1 if on else 0))

    def profile_read(self, kernel):
        ms = ctypes.c_double()
        n = ctypes.c_int64()
        _check(lib().ch_batch_profile_read(self._h, KERNELS.get(kernel, kernel),
                                           ctypes.byref(ms), ctypes.byref(n)))
        return ms.value, n.value

    def x_program(self):
        """The x-pass program of the current plan (a key of X_PROGRAMS)."""
        k = ctypes.c_int()
        _check(lib().ch_batch_get_x_program(self._h, ctypes.byref(k)))
        return k.value

    def close(self):
        if getattr(self, "_h", None):
            lib().ch_batch_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Interp:
    """Coarse stretched-z velocity -> fine uniform faces (multiple resolution),
    and fine C -> coarse cell centres.  With solenoidal=True the velocity is
    transferred through its normal gradients and integrated from reference
    planes (ch_interp_set_solenoidal)."""

    def __init__(self, fine_shape, h, coarse_shape, zf, precision="fp64", stream=None,
                 solenoidal=False):
        nz, ny, nx = fine_shape
        ncz, ncy, ncx = coarse_shape
        self.fine_shape = tuple(fine_shape)
        self.coarse_shape = tuple(coarse_shape)
        self.dtype = _dtype(_prec(precision))
        zf = np.ascontiguousarray(zf, dtype=np.float64)
        if zf.shape != (ncz + 1,):
            raise ValueError("zf must have ncz + 1 entries")
        g = Grid(nx, ny, nz, h)
        handle = ctypes.c_void_p()
        _check(lib().ch_interp_create(ctypes.byref(g), ncx, ncy, ncz,
                                      zf.ctypes.data_as(_PD), _prec(precision),
                                      ctypes.byref(handle)))
        self._h = handle
        self.stream = stream
        _check(lib().ch_interp_set_stream(self._h,
                                          ctypes.c_void_p(stream.cuda_stream if stream else 0)))
        if solenoidal:
            self.set_solenoidal(True)

    def set_solenoidal(self, on):
        _check(lib().ch_interp_set_solenoidal(self._h, 1 if on else 0))

    def closure(self):
        """Largest |closure sum| of the x, y and z lines of the last solenoidal
        transfer (waits for the handle's stream)."""
        out = (ctypes.c_double * 3)()
        _check(lib().ch_interp_closure(self._h, out))
        return tuple(out)

    def _coarse_ptrs(self, uc, vc, wc):
        ncz, ncy, ncx = self.coarse_shape
        return (_dev_tensor(uc, self.dtype, (ncz, ncy, ncx), "uc"),
                _dev_tensor(vc, self.dtype, (ncz, ncy, ncx), "vc"),
                _dev_tensor(wc, self.dtype, (ncz + 1, ncy, ncx), "wc"))

    def apply(self, uc, vc, wc, out=None):
        """Fine (u, v, w); `out` may hold three preallocated tensors."""
        nz, ny, nx = self.fine_shape
        if out is None:
            out = (torch.empty((nz, ny, nx), dtype=self.dtype, device="cuda"),
                   torch.empty((nz, ny, nx), dtype=self.dtype, device="cuda"),
                   torch.empty((nz + 1, ny, nx), dtype=self.dtype, device="cuda"))
        u, v, w = out
        ptrs = (_dev_tensor(u, self.dtype, (nz, ny, nx), "u"),
                _dev_tensor(v, self.dtype, (nz, ny, nx), "v"),
                _dev_tensor(w, self.dtype, (nz + 1, ny, nx), "w"))
        if self.stream is not None:
            self.stream.wait_stream(torch.cuda.current_stream())
        _check(lib().ch_interp_apply(self._h, *self._coarse_ptrs(uc, vc, wc), *ptrs))
        if self.stream is not None:
            torch.cuda.current_stream().wait_stream(self.stream)
        return u, v, w

    def project_c(self, Cf, out=None):
        """Fine cell-centred C (nz, ny, nx) -> coarse cell centres (ncz, ncy, ncx)."""
        if out is None:
            out = torch.empty(self.coarse_shape, dtype=self.dtype, device="cuda")
        src = _dev_tensor(Cf, self.dtype, self.fine_shape, "Cf")
        dst = _dev_tensor(out, self.dtype, self.coarse_shape, "Cc")
        if self.stream is not None:
            self.stream.wait_stream(torch.cuda.current_stream())
        _check(lib().ch_interp_project_c(self._h, src, dst))
        if self.stream is not None:
            torch.cuda.current_stream().wait_stream(self.stream)
        return out

    def close(self):
        if getattr(self, "_h", None):
            lib().ch_interp_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Poisson(_StreamMixin):
    """Split-density pressure step on an (nz, ny, nx) cell mesh of spacing h,
    periodic in x and y, z periodic or between walls (z_walls)."""

    def __init__(self, shape, h, z_walls=False, precision="fp64", stream=None):
        nz, ny, nx = shape
        self.shape = tuple(shape)
        self.z_walls = bool(z_walls)
        self.dtype = _dtype(_prec(precision))
        g = Grid(nx, ny, nz, h)
        handle = ctypes.c_void_p()
        _check(lib().ch_poisson_create(ctypes.byref(g), 1 if z_walls else 0, _prec(precision),
                                       ctypes.byref(handle)))
        self._h = handle
        self.stream = stream
        _check(lib().ch_poisson_set_stream(self._h,
                                           ctypes.c_void_p(stream.cuda_stream if stream else 0)))

    def w_shape(self):
        nz, ny, nx = self.shape
        return (nz + 1, ny, nx) if self.z_walls else self.shape

    def solve(self, rhs, out=None):
        """Zero-mean P with lap P = rhs - mean(rhs)."""
        if out is None:
            out = torch.empty(self.shape, dtype=self.dtype, device="cuda")
        a = _dev_tensor(rhs, self.dtype, self.shape, "rhs")
        b = _dev_tensor(out, self.dtype, self.shape, "P")
        self._enter()
        _check(lib().ch_poisson_solve(self._h, a, b))
        self._leave()
        return out

    def step(self, C, u, v, w, P, Pold, rho1, rho2, dt):
        """In place: u, v, w <- u^{l+1}; P <- P^{l+1}; Pold <- P^l."""
        ptrs = [_dev_tensor(C, self.dtype, self.shape, "C"),
                _dev_tensor(u, self.dtype, self.shape, "u"),
                _dev_tensor(v, self.dtype, self.shape, "v"),
                _dev_tensor(w, self.dtype, self.w_shape(), "w"),
                _dev_tensor(P, self.dtype, self.shape, "P"),
                _dev_tensor(Pold, self.dtype, self.shape, "Pold")]
        self._enter()
        _check(lib().ch_pressure_step(self._h, ptrs[0], float(rho1), float(rho2), float(dt),
                                      *ptrs[1:]))
        self._leave()

    def close(self):
        if getattr(self, "_h", None):
            lib().ch_poisson_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
