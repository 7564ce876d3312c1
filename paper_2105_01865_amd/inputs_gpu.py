"""Seeded synthetic inputs built on the GPU with torch, for boxes too large
for the host generator (the 1536^3 workload: one field is 13.5 GiB in single
precision).

The recipe is that of `inputs.py`: drops placed by its host rejection sampler
and given the same tanh profile (combined by max); the velocity is the
staggered discrete curl of a random-phase vector potential whose spectrum
gives E(k) ~ k^slope on kmin <= |k| <= kmax, scaled to the requested rms.
Only the random numbers differ (torch's counter-based generator on the GPU
instead of numpy's PCG64).  Like `inputs.py`, this module holds none of the
method's arithmetic.
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np
import torch

from . import inputs


@dataclass
class LargeWorkload:
    name: str
    shape: tuple          # (nz, ny, nx)
    h: float
    Cn: float
    Pe: float
    dt: float
    nsteps: int
    C: torch.Tensor       # device tensors
    u: torch.Tensor
    v: torch.Tensor
    w: torch.Tensor
    centres: np.ndarray   # drops (physical units, x y z)
    radii: np.ndarray

    @property
    def points(self):
        nz, ny, nx = self.shape
        return nx * ny * nz


def drop_field(shape, h, Cn, centres, radii, dtype=torch.float32, device="cuda"):
    """C = 1/2 [1 - tanh((r - R) / (2 sqrt(2) Cn))] around each drop (periodic
    minimum-image distance), drops combined by max, evaluated on a bounding
    cube of R + 12 profile widths like the host generator."""
    nz, ny, nx = shape
    C = torch.zeros(shape, dtype=dtype, device=device)
    width = 2.0 * math.sqrt(2.0) * Cn

    def axis(n, cc, ext):
        coord = (torch.arange(n, device=device, dtype=torch.float64) + 0.5) * h
        d = coord - cc
        L = n * h
        d = d - L * torch.round(d / L)
        sel = torch.nonzero(d.abs() <= ext).flatten()
        return sel, d[sel]

    for c, R in zip(centres, radii):
        ext = R + 12.0 * width
        ix, dx = axis(nx, c[0], ext)
        iy, dy = axis(ny, c[1], ext)
        iz, dz = axis(nz, c[2], ext)
        if ix.numel() == 0 or iy.numel() == 0 or iz.numel() == 0:
            continue
        r = torch.sqrt(dz[:, None, None] ** 2 + dy[None, :, None] ** 2 + dx[None, None, :] ** 2)
        val = (0.5 * (1.0 - torch.tanh((r - R) / width))).to(dtype)
        sel = (iz[:, None, None], iy[None, :, None], ix[None, None, :])
        C[sel] = torch.maximum(C[sel], val)
    return C


def _potential(gen, shape, kmin, kmax, slope, device):
    """One component of the random-phase vector potential (single precision)."""
    nz, ny, nx = shape
    kk = torch.arange(-kmax, kmax + 1, device=device, dtype=torch.float64)
    kr = torch.arange(0, kmax + 1, device=device, dtype=torch.float64)
    K = torch.sqrt(kk[:, None, None] ** 2 + kk[None, :, None] ** 2 + kr[None, None, :] ** 2)
    band = (K >= kmin) & (K <= kmax)
    amp = torch.zeros_like(K)
    Kb = K[band]
    amp[band] = torch.sqrt(Kb ** slope / (4.0 * math.pi * Kb ** 2)) / Kb
    re = torch.randn(K.shape, generator=gen, device=device, dtype=torch.float64)
    im = torch.randn(K.shape, generator=gen, device=device, dtype=torch.float64)
    small = (amp * torch.complex(re, im)).to(torch.complex64)
    spec = torch.zeros((nz, ny, nx // 2 + 1), dtype=torch.complex64, device=device)
    iz = torch.remainder(kk.long(), nz)
    iy = torch.remainder(kk.long(), ny)
    spec[iz[:, None, None], iy[None, :, None], kr.long()[None, None, :]] = small
    A = torch.fft.irfftn(spec, s=shape, dim=(0, 1, 2))
    del spec
    return A


def random_solenoidal(gen, shape, h, kmin, kmax, slope=-5.0 / 3.0, rms=1.0, device="cuda"):
    """u = dAz/dy - dAy/dz, v = dAx/dz - dAz/dx, w = dAy/dx - dAx/dy with
    forward differences on the periodic staggered mesh (zero discrete
    divergence), scaled so that sqrt(<u^2 + v^2 + w^2>/3) = rms.  The three
    potential components are made one at a time to bound the memory."""
    def d(a, dim):
        return (torch.roll(a, -1, dims=dim) - a) / h

    A = _potential(gen, shape, kmin, kmax, slope, device)          # Ax
    v = d(A, 0)
    w = -d(A, 1)
    del A
    A = _potential(gen, shape, kmin, kmax, slope, device)          # Ay
    u = -d(A, 0)
    w += d(A, 2)
    del A
    A = _potential(gen, shape, kmin, kmax, slope, device)          # Az
    u += d(A, 1)
    v -= d(A, 2)
    del A
    ms = sum(float(torch.sum(x * x, dtype=torch.float64)) for x in (u, v, w))
    s = math.sqrt(ms / (3.0 * u.numel()))
    for x in (u, v, w):
        x.mul_(rms / s)
    return u, v, w


def large_workload(n: int | None = None, device="cuda", dtype=torch.float32):
    """The 1536^3 periodic box: 4000 drops R ~ U[4,20] h (placement by the
    host sampler, seed of the 1536^3 workload), k^-5/3 field on 1 <= |k| <= 48 with
    rms 1; dt = 1e-4 unless the advective bound sum_d max|u_d| dt / h <= 0.8
    needs less.  `n` shrinks the edge (drops scale with the volume)."""
    n = n or 1536
    h = 1.0 / n
    shape = (n, n, n)
    Cn = h
    seed = inputs.seed_for(4)
    rng = np.random.default_rng(seed)
    ndrops = 4000 if n >= 1536 else max(1, int(4000 * (n / 1536) ** 3))
    cen, rad = inputs.place_drops(rng, ndrops, 4, 20, shape, h)
    gen = torch.Generator(device=device)
    gen.manual_seed(seed)
    u, v, w = random_solenoidal(gen, shape, h, 1, min(48, n // 3), device=device)
    umax = sum(float(x.abs().max()) for x in (u, v, w))
    dt = 1e-4 if umax * 1e-4 / h <= 0.8 else 0.8 * h / umax
    u, v, w = (x.to(dtype) for x in (u, v, w))
    C = drop_field(shape, h, Cn, cen, rad, dtype=dtype, device=device)
    return LargeWorkload("large-4000-drops", shape, h, Cn, 0.9 / Cn, dt, 200, C, u, v, w,
                         cen, rad)
