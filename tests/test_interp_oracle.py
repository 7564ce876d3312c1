"""Pins of the oracle's coarse-to-fine velocity interpolation (sec. 3.4,
multiple-resolution meshes): cubic Hermite in each direction, four source
points per direction."""
import math

import numpy as np
import pytest

import oracle
from paper_2105_01865_amd import inputs


def test_stencil_interpolates_nodes_and_sums_to_one():
    s = inputs.stretched_faces(24, 2.0)
    zc = 0.5 * (s[:-1] + s[1:])
    for kind, pts in ((oracle.AX_WALL_EVEN, zc), (oracle.AX_PERIODIC, np.arange(16) / 16.0)):
        for i, t in enumerate(pts):
            idx, wt = oracle.hermite_stencil(pts, 1.0, kind, t)
            assert abs(wt.sum() - 1.0) < 1e-14
            # at a node the interpolant returns that node's value
            val = np.zeros(len(pts))
            val[i] = 1.0
            assert abs((wt * val[idx]).sum() - 1.0) < 1e-14
        for t in np.linspace(0.001, 0.999, 37):
            idx, wt = oracle.hermite_stencil(pts, 1.0, kind, t)
            assert abs(wt.sum() - 1.0) < 1e-13


def test_linear_exact_on_stretched_axis_and_quadratic_exact_on_uniform_axis():
    s = inputs.stretched_faces(20, 2.0)
    zc = 0.5 * (s[:-1] + s[1:])
    for t in np.linspace(zc[2], zc[-3], 29):
        idx, wt = oracle.hermite_stencil(zc, 1.0, oracle.AX_WALL_EVEN, t)
        f = 0.3 + 2.0 * zc
        assert abs((wt * f[idx]).sum() - (0.3 + 2.0 * t)) < 1e-13
    x = np.arange(16) / 16.0
    for t in np.linspace(0.2, 0.8, 13):
        idx, wt = oracle.hermite_stencil(x, 1.0, oracle.AX_PERIODIC, t)
        f = 1.0 - x + 3.0 * x * x
        assert abs((wt * f[idx]).sum() - (1.0 - t + 3.0 * t * t)) < 1e-13


def _analytic(nc, ncz, alpha=2.0):
    zf = inputs.stretched_faces(ncz, alpha)
    zc = 0.5 * (zf[:-1] + zf[1:])
    xf = np.arange(nc) / nc
    xc = (np.arange(nc) + 0.5) / nc
    tp = 2 * math.pi
    fu = lambda x, y, z: np.sin(tp * x) * np.cos(tp * y) * np.cos(math.pi * z)
    fv = lambda x, y, z: np.cos(tp * x + 0.3) * np.sin(tp * y) * np.cos(math.pi * z)
    fw = lambda x, y, z: np.cos(tp * (x - y)) * np.sin(math.pi * z)
    grid = lambda gx, gy, gz: np.meshgrid(gz, gy, gx, indexing="ij")[::-1]
    X, Y, Z = grid(xf, xc, zc)
    uc = fu(X, Y, Z)
    X, Y, Z = grid(xc, xf, zc)
    vc = fv(X, Y, Z)
    X, Y, Z = grid(xc, xc, zf)
    wc = fw(X, Y, Z)
    wc[0] = wc[-1] = 0.0   # the wall-normal velocity vanishes on the walls
    return zf, uc, vc, wc, (fu, fv, fw)


def _fine_exact(fns, nf):
    fu, fv, fw = fns
    f = np.arange(nf) / nf
    c = (np.arange(nf) + 0.5) / nf
    ff = np.arange(nf + 1) / nf
    grid = lambda gx, gy, gz: np.meshgrid(gz, gy, gx, indexing="ij")[::-1]
    return fu(*grid(f, c, c)), fv(*grid(c, f, c)), fw(*grid(c, c, ff))


def test_interpolation_converges_and_respects_walls():
    errs = []
    for nc in (8, 16, 32):
        zf, uc, vc, wc, fns = _analytic(nc, (3 * nc) // 4)
        nf = 2 * nc
        uf, vf, wf = oracle.interp_velocity(zf, uc, vc, wc, (nf, nf, nf))
        eu, ev, ew = _fine_exact(fns, nf)
        errs.append(max(np.abs(uf - eu).max(), np.abs(vf - ev).max(), np.abs(wf - ew).max()))
        assert np.abs(wf[0]).max() == 0.0 and np.abs(wf[-1]).max() == 0.0
    rates = [math.log2(errs[i] / errs[i + 1]) for i in range(2)]
    assert min(rates) > 2.0, (errs, rates)


def test_interpolation_at_coincident_nodes_copies_the_source():
    # fine x faces at even indices coincide with the coarse x faces
    zf, uc, vc, wc, _ = _analytic(8, 6)
    uf, vf, wf = oracle.interp_velocity(zf, uc, vc, wc, (16, 16, 16))
    # u at fine x face 2i equals the coarse u interpolated only in y and z;
    # check the x direction alone with a field constant in y and z
    uc2 = np.broadcast_to(uc[:1, :1, :], uc.shape).copy()
    uf2, _, _ = oracle.interp_velocity(zf, uc2, vc, wc, (16, 16, 16))
    np.testing.assert_allclose(uf2[:, :, ::2], np.broadcast_to(uc2[0, 0, :], (16, 16, 8)),
                               atol=1e-14)


@pytest.mark.parametrize("kind", ["even", "odd"])
def test_reflection_beyond_the_walls_is_accurate_near_both_walls(kind):
    zf = inputs.stretched_faces(32, 2.0)
    if kind == "even":   # tangential component at cell centres, even about the walls
        pts, ax, f = 0.5 * (zf[:-1] + zf[1:]), oracle.AX_WALL_EVEN, lambda z: np.cos(np.pi * z)
    else:                # wall-normal component on faces, odd about the walls
        pts, ax, f = zf, oracle.AX_WALL_ODD, lambda z: np.sin(np.pi * z)
    vals = f(pts)
    if kind == "odd":
        vals[0] = vals[-1] = 0.0
    for t in np.concatenate([np.linspace(0.0, pts[2], 9), np.linspace(pts[-3], 1.0, 9)]):
        idx, wt = oracle.hermite_stencil(pts, 1.0, ax, t)
        # cubic Hermite error: small against the local cell width cubed
        dz = zf[1] - zf[0]
        assert abs((wt * vals[idx]).sum() - f(t)) < 0.05 * dz ** 2 * np.pi ** 2


# ---- the solenoidal variant and the back-projection of C (sec. 3.4) ----

def _fine_div(uf, vf, wf):
    nz, ny, nx = uf.shape
    return ((np.roll(uf, -1, axis=2) - uf) * nx + (np.roll(vf, -1, axis=1) - vf) * ny
            + (wf[1:] - wf[:-1]) * nz)


def test_solenoidal_transfer_keeps_the_fine_field_divergence_free():
    """A coarse field that is a discrete curl (exactly divergence-free on the
    stretched staggered mesh) gives a fine field whose discrete divergence
    is zero to rounding in every cell but the top layer (where the z line's
    closure sum is left); with a refinement ratio of 2 the periodic x and y
    lines close to rounding too."""
    nc, zf = (10, 8, 8), inputs.stretched_faces(10, 2.0)
    uc, vc, wc = inputs.coarse_wall_velocity(np.random.default_rng(5), nc, zf, kmax=3,
                                             nmodes_z=5)
    ncz, ncy, ncx = nc
    cdiv = ((np.roll(uc, -1, axis=2) - uc) * ncx + (np.roll(vc, -1, axis=1) - vc) * ncy
            + (wc[1:] - wc[:-1]) / np.diff(zf)[:, None, None])
    scale = max(np.abs(uc).max(), np.abs(vc).max(), np.abs(wc).max())
    assert np.abs(cdiv).max() < 1e-11 * scale * ncx
    nf = (16, 16, 20)
    uf, vf, wf, resid = oracle.solenoidal_velocity(zf, uc, vc, wc, nf)
    div = _fine_div(uf, vf, wf)
    tol = 1e-11 * scale * max(nf)
    assert np.abs(div[:-1]).max() < tol, np.abs(div[:-1]).max()
    assert resid[0] < 1e-12 * scale and resid[1] < 1e-12 * scale
    # the top layer carries exactly the z closure sum (per unit height)
    top = np.abs(div[-1]).max()
    assert abs(top - resid[2] * nf[2]) <= 1e-9 * max(1.0, top)
    assert np.all(wf[0] == 0.0) and np.all(wf[-1] == 0.0)
    # the plain transfer does not have this property
    ud, vd, wd = oracle.interp_velocity(zf, uc, vc, wc, nf)
    assert np.abs(_fine_div(ud, vd, wd)[:-1]).max() > 1e3 * tol


def test_solenoidal_transfer_reference_planes_and_x_independent_u():
    nc, zf = (6, 8, 8), inputs.stretched_faces(6, 2.0)
    uc, vc, wc = inputs.coarse_wall_velocity(np.random.default_rng(6), nc, zf, kmax=3,
                                             nmodes_z=4)
    nf = (16, 16, 12)
    uf, vf, _, _ = oracle.solenoidal_velocity(zf, uc, vc, wc, nf)
    ud, vd, _ = oracle.interp_velocity(zf, uc, vc, wc, nf)
    # the reference planes are the plain transfer on the low faces, bitwise
    assert np.array_equal(uf[:, :, 0], ud[:, :, 0])
    assert np.array_equal(vf[:, 0, :], vd[:, 0, :])
    # a u constant along x has no x gradient: every x face repeats face 0
    uc2 = np.broadcast_to(uc[:, :, :1], uc.shape).copy()
    uf2, _, _, r = oracle.solenoidal_velocity(zf, uc2, vc, wc, nf)
    assert np.array_equal(uf2, np.broadcast_to(uf2[:, :, :1], uf2.shape))
    assert r[0] == 0.0


def test_solenoidal_transfer_converges_on_a_smooth_field():
    errs = []
    for nc in (8, 16, 32):
        zf, uc, vc, wc, fns = _analytic(nc, (3 * nc) // 4)
        nf = 2 * nc
        uf, vf, wf, _ = oracle.solenoidal_velocity(zf, uc, vc, wc, (nf, nf, nf))
        eu, ev, ew = _fine_exact(fns, nf)
        errs.append(max(np.abs(uf - eu).max(), np.abs(vf - ev).max(), np.abs(wf - ew).max()))
    rates = [math.log2(errs[i] / errs[i + 1]) for i in range(2)]
    assert min(rates) > 1.8, (errs, rates)


def test_projection_of_c_is_the_identity_on_coincident_meshes_and_exact_on_constants():
    rng = np.random.default_rng(8)
    n = 12
    zf = np.arange(n + 1) / n
    Cf = rng.standard_normal((n, n, n))
    Cc = oracle.project_c(Cf, zf, (n, n, n))
    np.testing.assert_allclose(Cc, Cf, rtol=0, atol=1e-14)
    zf2 = inputs.stretched_faces(10, 2.0)
    Cc2 = oracle.project_c(np.full((24, 16, 20), 0.37), zf2, (8, 8, 10))
    np.testing.assert_allclose(Cc2, 0.37, rtol=0, atol=1e-14)


def test_projection_of_c_converges():
    f = lambda x, y, z: np.cos(2 * math.pi * x) * np.sin(2 * math.pi * y + 0.4) * np.cos(math.pi * z)
    errs = []
    for nf in (16, 32, 64):
        c = (np.arange(nf) + 0.5) / nf
        Z, Y, X = np.meshgrid(c, c, c, indexing="ij")
        nc = nf // 2
        zf = inputs.stretched_faces((3 * nc) // 4, 2.0)
        Cc = oracle.project_c(f(X, Y, Z), zf, (nc, nc, (3 * nc) // 4))
        xc = (np.arange(nc) + 0.5) / nc
        zc = 0.5 * (zf[:-1] + zf[1:])
        Zc, Yc, Xc = np.meshgrid(zc, xc, xc, indexing="ij")
        errs.append(np.abs(Cc - f(Xc, Yc, Zc)).max())
    rates = [math.log2(errs[i] / errs[i + 1]) for i in range(2)]
    assert min(rates) > 2.5, (errs, rates)
