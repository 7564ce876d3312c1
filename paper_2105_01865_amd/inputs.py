"""Seeded synthetic inputs for the Cahn-Hilliard update.

This module only builds input fields (drop-laden C and prescribed velocity
fields) with numpy; it holds none of the method's arithmetic.  Both the CPU
oracle and the GPU library consume what it returns.

The fields stand in for the drop-laden turbulent flows of the paper's
Rayleigh-Benard runs (sec. 4.3: hundreds to about a thousand drops, from
about ten cells across up to a radius of 0.23 H, interface width of order
the mesh size).  No dataset is involved.

Conventions: arrays are (nz, ny, nx), x fastest, float64.  The domain is
[0,1)^3, h = 1/n.  C is cell-centred.  u lives on x faces (face i is the low
face of cell i), v on y faces, w on z faces; an axis with no-flux walls has
n + 1 faces along it (the first and last are the walls, where the normal
velocity is zero).
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

SEED_BASE = 210501865


def seed_for(config: int, box: int = 0) -> int:
    return SEED_BASE + 1000 * config + box


# --------------------------------------------------------------------------
# drops
# --------------------------------------------------------------------------
def place_drops(rng, count, rmin, rmax, shape, h, walls_z=False, gap_cells=4.0,
                max_tries=10000):
    """Sequential rejection placement of non-overlapping spheres.

    Radii uniform in [rmin, rmax] (in units of h); centres uniform in the box.
    Minimum-image distance between centres >= R_i + R_j + gap; with walls in z
    the centre keeps R + gap from each wall.  Returns (centres (m,3) in
    physical units (x, y, z), radii (m,) physical); m <= count.
    """
    nz, ny, nx = shape
    L = np.array([nx * h, ny * h, nz * h])
    gap = gap_cells * h
    cen = np.zeros((count, 3))
    rad = np.zeros(count)
    m = 0
    for _ in range(count):
        R = rng.uniform(rmin, rmax) * h
        for _try in range(max_tries):
            c = rng.uniform(0.0, 1.0, size=3) * L
            if walls_z:
                lo, hi = R + gap, L[2] - R - gap
                if hi <= lo:
                    continue
                c[2] = lo + (hi - lo) * rng.uniform()
            d = c[None, :] - cen[:m]
            d[:, 0] -= L[0] * np.round(d[:, 0] / L[0])
            d[:, 1] -= L[1] * np.round(d[:, 1] / L[1])
            if not walls_z:
                d[:, 2] -= L[2] * np.round(d[:, 2] / L[2])
            if m == 0 or np.all(np.sqrt((d * d).sum(axis=1)) >= R + rad[:m] + gap):
                cen[m] = c
                rad[m] = R
                m += 1
                break
    return cen[:m].copy(), rad[:m].copy()


def drop_field(shape, h, Cn, centres, radii, walls_z=False):
    """C = 1/2 [1 - tanh((r - R) / (2 sqrt(2) Cn))], C = 1 inside; drops by max.

    r is the minimum-image distance (periodic axes only).
    """
    nz, ny, nx = shape
    L = np.array([nx * h, ny * h, nz * h])
    x = (np.arange(nx) + 0.5) * h
    y = (np.arange(ny) + 0.5) * h
    z = (np.arange(nz) + 0.5) * h
    C = np.zeros(shape)
    width = 2.0 * math.sqrt(2.0) * Cn
    for c, R in zip(centres, radii):
        # restrict to a bounding box of R + 12 widths (tanh saturates well before)
        ext = R + 12.0 * width

        def axis_sel(coord, cc, Ld, periodic):
            d = coord - cc
            if periodic:
                d = d - Ld * np.round(d / Ld)
            sel = np.abs(d) <= ext
            return np.nonzero(sel)[0], d[sel]

        ix, dx = axis_sel(x, c[0], L[0], True)
        iy, dy = axis_sel(y, c[1], L[1], True)
        iz, dz = axis_sel(z, c[2], L[2], not walls_z)
        if ix.size == 0 or iy.size == 0 or iz.size == 0:
            continue
        r = np.sqrt(dz[:, None, None] ** 2 + dy[None, :, None] ** 2 + dx[None, None, :] ** 2)
        val = 0.5 * (1.0 - np.tanh((r - R) / width))
        sub = C[np.ix_(iz, iy, ix)]
        C[np.ix_(iz, iy, ix)] = np.maximum(sub, val)
    return C


# --------------------------------------------------------------------------
# velocity fields on the staggered mesh
# --------------------------------------------------------------------------
def abc_velocity(shape, h, A, B, Cc):
    """Steady ABC flow sampled on the faces.

    u = A sin 2 pi z + C cos 2 pi y, v = B sin 2 pi x + A cos 2 pi z,
    w = C sin 2 pi y + B cos 2 pi x.  u does not depend on x, v not on y and
    w not on z, so the staggered divergence vanishes exactly.
    """
    nz, ny, nx = shape
    xc = (np.arange(nx) + 0.5) * h
    yc = (np.arange(ny) + 0.5) * h
    zc = (np.arange(nz) + 0.5) * h
    tp = 2.0 * math.pi
    u = (A * np.sin(tp * zc)[:, None, None] + Cc * np.cos(tp * yc)[None, :, None]) \
        * np.ones((1, 1, nx))
    v = (B * np.sin(tp * xc)[None, None, :] + A * np.cos(tp * zc)[:, None, None]) \
        * np.ones((1, ny, 1))
    w = (Cc * np.sin(tp * yc)[None, :, None] + B * np.cos(tp * xc)[None, None, :]) \
        * np.ones((nz, 1, 1))
    return np.ascontiguousarray(u), np.ascontiguousarray(v), np.ascontiguousarray(w)


def _random_potential(rng, shape, kmin, kmax, slope):
    """Random-phase real field whose Fourier amplitudes give, after one curl,
    a velocity energy spectrum E(k) ~ k^slope on kmin <= |k| <= kmax."""
    nz, ny, nx = shape
    kx = np.fft.rfftfreq(nx, 1.0 / nx)
    ky = np.fft.fftfreq(ny, 1.0 / ny)
    kz = np.fft.fftfreq(nz, 1.0 / nz)
    K = np.sqrt(kz[:, None, None] ** 2 + ky[None, :, None] ** 2 + kx[None, None, :] ** 2)
    band = (K >= kmin) & (K <= kmax)
    amp = np.zeros_like(K)
    # |u_hat|^2 ~ E(k) / (4 pi k^2), and |u_hat| = k |A_hat|
    amp[band] = np.sqrt(K[band] ** slope / (4.0 * math.pi * K[band] ** 2)) / K[band]
    spec = amp * (rng.standard_normal(K.shape) + 1j * rng.standard_normal(K.shape))
    return np.fft.irfftn(spec, s=shape, axes=(0, 1, 2))


def curl_velocity(Ax, Ay, Az, h):
    """Staggered discrete curl of an edge-located vector potential on a
    periodic uniform mesh; the result has zero staggered divergence.

    Az at (i, j, k+1/2), Ay at (i, j+1/2, k), Ax at (i+1/2, j, k) (array index
    (k, j, i) of the lower corner).  u at the x face (i, j+1/2, k+1/2) etc.
    """
    def d(a, axis):  # forward difference a[m+1] - a[m] along axis (0=z,1=y,2=x)
        return (np.roll(a, -1, axis=axis) - a) / h
    u = d(Az, 1) - d(Ay, 0)
    v = d(Ax, 0) - d(Az, 2)
    w = d(Ay, 2) - d(Ax, 1)
    return u, v, w


def random_solenoidal(rng, shape, h, kmin=1, kmax=16, slope=-5.0 / 3.0, rms=1.0):
    """Frozen random-phase divergence-free field with E(k) ~ k^slope,
    scaled so that sqrt(<u^2 + v^2 + w^2> / 3) = rms."""
    Ax = _random_potential(rng, shape, kmin, kmax, slope)
    Ay = _random_potential(rng, shape, kmin, kmax, slope)
    Az = _random_potential(rng, shape, kmin, kmax, slope)
    u, v, w = curl_velocity(Ax, Ay, Az, h)
    s = math.sqrt((np.mean(u * u) + np.mean(v * v) + np.mean(w * w)) / 3.0)
    return u * (rms / s), v * (rms / s), w * (rms / s)


def staggered_divergence(u, v, w, h, bc=(0, 0, 0)):
    """Discrete divergence per cell (for the generator's own checks)."""
    def dd(a, axis, periodic):
        if periodic:
            return (np.roll(a, -1, axis=axis) - a) / h
        sl_hi = [slice(None)] * 3
        sl_lo = [slice(None)] * 3
        sl_hi[axis] = slice(1, None)
        sl_lo[axis] = slice(0, -1)
        return (a[tuple(sl_hi)] - a[tuple(sl_lo)]) / h
    return dd(u, 2, bc[0] == 0) + dd(v, 1, bc[1] == 0) + dd(w, 0, bc[2] == 0)


def wall_velocity(rng, shape, bc, h, smooth=2):
    """Divergence-free staggered velocity on a uniform mesh with no-flux
    walls on any axis (bc = (bx, by, bz), 1 = walls): the discrete curl of an
    edge-located vector potential whose components tangential to each wall
    vanish on it, so the wall-normal velocity is zero there.

    A potential component lives on the mesh nodes along the axes it is not
    aligned with (n + 1 nodes along a walled axis, n along a periodic one)
    and on the cell centres along its own axis.  The random potentials are
    smoothed by `smooth` passes of a three-point average along every axis.
    Returns u (nz, ny, fx), v (nz, fy, nx), w (fz, ny, nx), f = n (+1 with
    walls).
    """
    nz, ny, nx = shape
    nodes = [n + 1 if b else n for n, b in zip((nx, ny, nz), bc)]   # x, y, z

    def field(sz, sy, sx):
        a = rng.normal(size=(sz, sy, sx))
        for _ in range(smooth):
            for axis in range(3):
                a = (np.roll(a, 1, axis) + 2.0 * a + np.roll(a, -1, axis)) / 4.0
        return a

    Ax = field(nodes[2], nodes[1], nx)
    Ay = field(nodes[2], ny, nodes[0])
    Az = field(nz, nodes[1], nodes[0])
    if bc[0]:
        Ay[:, :, 0] = Ay[:, :, -1] = 0.0
        Az[:, :, 0] = Az[:, :, -1] = 0.0
    if bc[1]:
        Ax[:, 0, :] = Ax[:, -1, :] = 0.0
        Az[:, 0, :] = Az[:, -1, :] = 0.0
    if bc[2]:
        Ax[0] = Ax[-1] = 0.0
        Ay[0] = Ay[-1] = 0.0

    def d(a, axis, walled):
        # node-to-centre difference: forward neighbour, wrapped when periodic
        if walled:
            hi = [slice(None)] * 3
            lo = [slice(None)] * 3
            hi[axis] = slice(1, None)
            lo[axis] = slice(0, -1)
            return (a[tuple(hi)] - a[tuple(lo)]) / h
        return (np.roll(a, -1, axis=axis) - a) / h

    u = d(Az, 1, bc[1]) - d(Ay, 0, bc[2])
    v = d(Ax, 0, bc[2]) - d(Az, 2, bc[0])
    w = d(Ay, 2, bc[0]) - d(Ax, 1, bc[1])
    return u, v, w


def stretched_faces(n, alpha=2.0):
    """Face positions z_k = 1/2 [1 + tanh(alpha (2k/n - 1)) / tanh(alpha)],
    k = 0..n, clustered towards both walls."""
    k = np.arange(n + 1)
    z = 0.5 * (1.0 + np.tanh(alpha * (2.0 * k / n - 1.0)) / math.tanh(alpha))
    z[0], z[-1] = 0.0, 1.0
    return z


def coarse_wall_velocity(rng, shape, zf, kmax=16, slope=-5.0 / 3.0, rms=1.0, nmodes_z=24):
    """Divergence-free velocity on a coarse mesh, uniform and periodic in x
    and y, stretched in z between walls at z = 0 and 1 (faces zf).

    Discrete curl of a vector potential whose x and y components vanish on
    the walls (a sine series in z), so w = 0 on the walls.  Returns
    uc, vc (ncz, ncy, ncx) and wc (ncz+1, ncy, ncx).
    """
    ncz, ncy, ncx = shape
    hx, hy = 1.0 / ncx, 1.0 / ncy
    zc = 0.5 * (zf[:-1] + zf[1:])
    dz = np.diff(zf)
    kx = np.fft.fftfreq(ncx, 1.0 / ncx)
    ky = np.fft.fftfreq(ncy, 1.0 / ncy)

    def potential(zpts, sine):
        out = np.zeros((zpts.size, ncy, ncx))
        for m in range(1, nmodes_z + 1):
            kz = 0.5 * m
            K = np.sqrt(kz ** 2 + ky[:, None] ** 2 + kx[None, :] ** 2)
            band = (K >= 1.0) & (K <= kmax)
            amp = np.zeros_like(K)
            amp[band] = np.sqrt(K[band] ** slope / (4.0 * math.pi * K[band] ** 2)) / K[band]
            spec = amp * (rng.standard_normal(K.shape) + 1j * rng.standard_normal(K.shape))
            plane = np.real(np.fft.ifft2(spec)) * (ncx * ncy) ** 0.5
            prof = np.sin(math.pi * m * zpts) if sine else np.cos(math.pi * m * zpts)
            out += prof[:, None, None] * plane[None, :, :]
        return out

    Ax = potential(zf, True)    # at (i+1/2, j, z faces), zero on the walls
    Ay = potential(zf, True)    # at (i, j+1/2, z faces)
    Az = potential(zc, False)   # at (i, j, z centres)

    def dx(a):
        return (np.roll(a, -1, axis=2) - a) / hx

    def dy(a):
        return (np.roll(a, -1, axis=1) - a) / hy

    def dzf(a):  # z-face array -> centre difference over the cell
        return (a[1:] - a[:-1]) / dz[:, None, None]

    uc = dy(Az) - dzf(Ay)
    vc = dzf(Ax) - dx(Az)
    wc = dx(Ay) - dy(Ax)
    s = math.sqrt((np.mean(uc * uc) + np.mean(vc * vc) + np.mean(wc[1:-1] ** 2)) / 3.0)
    uc, vc, wc = uc * (rms / s), vc * (rms / s), wc * (rms / s)
    wc[0] = 0.0
    wc[-1] = 0.0
    return uc, vc, wc


def stretched_divergence(uc, vc, wc, zf):
    ncz, ncy, ncx = uc.shape
    dz = np.diff(zf)
    return ((np.roll(uc, -1, axis=2) - uc) * ncx + (np.roll(vc, -1, axis=1) - vc) * ncy
            + (wc[1:] - wc[:-1]) / dz[:, None, None])


# --------------------------------------------------------------------------
# the workloads
# --------------------------------------------------------------------------
@dataclass
class Workload:
    name: str
    shape: tuple           # (nz, ny, nx)
    h: float
    Cn: float
    Pe: float
    dt: float
    nsteps: int
    bc: tuple              # (bx, by, bz): 0 periodic, 1 no-flux
    C: np.ndarray
    u: np.ndarray = None
    v: np.ndarray = None
    w: np.ndarray = None
    coarse: dict = field(default_factory=dict)   # multiple-resolution source
    ndrops: int = 0

    @property
    def points(self):
        nz, ny, nx = self.shape
        return nx * ny * nz


def _cfl_dt(dt, u, v, w, h, limit=0.8):
    s = (np.abs(u).max() + np.abs(v).max() + np.abs(w).max()) * dt / h
    return dt if s <= limit else dt * limit / s


def make_workload(config: int, n: int | None = None, seed: int | None = None, box: int = 0):
    """The five workloads of the project, optionally shrunk to edge n.

    1: one drop R = 8h in a periodic box, ABC flow A = B = C = 0.1, dt = 1e-4
    2: 64 drops R ~ U[6,16] h, k^-5/3 field 1 <= k <= 16, rms 1, dt = 1e-4
    3: fine mesh with no-flux walls in z, 1000 drops R ~ U[4,12] h; velocity
       from a coarse mesh (n/2 x n/2 x 3n/8, tanh-stretched in z), interpolated
    4: 4000 drops R ~ U[4,20] h, k^-5/3 field up to k = 48
    5: one box of the batched ensemble (edge from {48,...,192}, 1-20 drops,
       ABC with amplitudes U[0.05, 0.2])
    """
    rng = np.random.default_rng(seed if seed is not None else seed_for(config, box))
    if config == 1:
        n = n or 32
        h = 1.0 / n
        shape = (n, n, n)
        Cn = h
        C = drop_field(shape, h, Cn, np.array([[0.5, 0.5, 0.5]]), np.array([8 * h]))
        u, v, w = abc_velocity(shape, h, 0.1, 0.1, 0.1)
        return Workload("drop-in-ABC-flow", shape, h, Cn, 0.9 / Cn, 1e-4, 100, (0, 0, 0),
                        C, u, v, w, ndrops=1)
    if config == 2:
        n = n or 256
        h = 1.0 / n
        shape = (n, n, n)
        Cn = h
        ndrops = 64 if n >= 256 else max(1, int(64 * (n / 256) ** 3))
        cen, rad = place_drops(rng, ndrops, 6, 16, shape, h)
        C = drop_field(shape, h, Cn, cen, rad)
        u, v, w = random_solenoidal(rng, shape, h, 1, min(16, n // 3), rms=1.0)
        return Workload("64-drops-kolmogorov-field", shape, h, Cn, 0.9 / Cn, 1e-4, 1000,
                        (0, 0, 0), C, u, v, w, ndrops=len(rad))
    if config == 3:
        n = n or 512
        h = 1.0 / n
        shape = (n, n, n)
        Cn = h
        ndrops = 1000 if n >= 512 else max(1, int(1000 * (n / 512) ** 3))
        cen, rad = place_drops(rng, ndrops, 4, 12, shape, h, walls_z=True)
        C = drop_field(shape, h, Cn, cen, rad, walls_z=True)
        ncx, ncy, ncz = n // 2, n // 2, (3 * n) // 8
        zf = stretched_faces(ncz, 2.0)
        uc, vc, wc = coarse_wall_velocity(rng, (ncz, ncy, ncx), zf, kmax=min(16, ncx // 3))
        # dt: 1e-4 unless the fine-mesh CFL bound needs less
        umax = max(np.abs(uc).max(), np.abs(vc).max(), np.abs(wc).max())
        dt = min(1e-4, 0.8 * h / (3.0 * umax))
        return Workload("multires-walls-1000-drops", shape, h, Cn, 0.9 / Cn, dt, 500,
                        (0, 0, 1), C, coarse=dict(zf=zf, uc=uc, vc=vc, wc=wc),
                        ndrops=len(rad))
    if config == 4:
        n = n or 1536
        h = 1.0 / n
        shape = (n, n, n)
        Cn = h
        ndrops = 4000 if n >= 1536 else max(1, int(4000 * (n / 1536) ** 3))
        cen, rad = place_drops(rng, ndrops, 4, 20, shape, h)
        C = drop_field(shape, h, Cn, cen, rad)
        u, v, w = random_solenoidal(rng, shape, h, 1, min(48, n // 3), rms=1.0)
        dt = _cfl_dt(1e-4, u, v, w, h)
        return Workload("large-4000-drops", shape, h, Cn, 0.9 / Cn, dt, 200, (0, 0, 0),
                        C, u, v, w, ndrops=len(rad))
    if config == 5:
        edges = [48, 64, 96, 128, 160, 192]
        n = n or int(edges[rng.integers(len(edges))])
        h = 1.0 / n
        shape = (n, n, n)
        Cn = h
        cnt = int(rng.integers(1, 21))
        cen, rad = place_drops(rng, cnt, 4, 12, shape, h)
        C = drop_field(shape, h, Cn, cen, rad)
        A, B, Cc = rng.uniform(0.05, 0.2, size=3)
        u, v, w = abc_velocity(shape, h, A, B, Cc)
        return Workload(f"ensemble-box-{box}", shape, h, Cn, 0.9 / Cn, 1e-4, 1000, (0, 0, 0),
                        C, u, v, w, ndrops=len(rad))
    raise ValueError(f"unknown config {config}")


def large_subbox(n_sub=256, n_big=1536):
    """The error reference of the 1536^3 workload: a 256^3 periodic box with
    the same h = 1/1536, holding the drops of the 1536^3 workload that lie
    inside the sub-box [0, 256 h)^3 (their centres at least R + 4 h from its
    faces, so the sub-box's own wrap does not cut them), in a k^-5/3 field
    made of the modes that are periodic on the sub-box: wavenumbers 6 to 48
    of the big box are 1 to 8 of the sub-box.  Its rms is the share of the
    big field's energy those modes carry (shell energies ~ k^-5/3).  The
    phases are the sub-box's own (seed of the 1536^3 workload, box 1).
    dt is left to the caller (the 1536^3 run's)."""
    h = 1.0 / n_big
    rng = np.random.default_rng(seed_for(4))
    cen, rad = place_drops(rng, 4000, 4, 20, (n_big,) * 3, h)
    L = n_sub * h
    gap = 4 * h
    inside = np.all((cen >= rad[:, None] + gap) & (cen <= L - rad[:, None] - gap), axis=1)
    cen, rad = cen[inside], rad[inside]
    shape = (n_sub,) * 3
    C = drop_field(shape, h, h, cen, rad)
    ratio = n_big // n_sub
    kmax_big = 48
    ks = np.arange(1, kmax_big + 1, dtype=np.float64)
    share = math.sqrt((ks[ks >= ratio] ** (-5.0 / 3.0)).sum() / (ks ** (-5.0 / 3.0)).sum())
    rng = np.random.default_rng(seed_for(4, box=1))
    u, v, w = random_solenoidal(rng, shape, h, 1, kmax_big // ratio, rms=share)
    return Workload("large-subbox", shape, h, h, 0.9 / h, 1e-4, 200, (0, 0, 0), C, u, v, w,
                    ndrops=len(rad))


def ensemble(nbox=48, n_override=None):
    """The batched ensemble: nbox independent periodic boxes."""
    return [make_workload(5, n=n_override, box=b) for b in range(nbox)]
