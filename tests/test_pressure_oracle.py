"""Pins of the oracle's split-density pressure step (sec. 3.2: eq-split,
eq-newpoi, eq-u) and its fast Poisson solve.

The Laplacian and divergence used to check the oracle are written here
directly as stencils with explicit ghost cells, not through the oracle's
face operators."""
import math

import numpy as np
import pytest

import oracle
from oracle import pressure as pr
from paper_2105_01865_amd import inputs


def lap_ref(P, h, zwalls):
    """7-point Laplacian with periodic x, y and, between walls, ghost planes
    equal to the wall-adjacent planes (dP/dz = 0)."""
    out = (np.roll(P, 1, 2) + np.roll(P, -1, 2) + np.roll(P, 1, 1) + np.roll(P, -1, 1)
           - 4.0 * P) / h ** 2
    if zwalls:
        Q = np.concatenate([P[:1], P, P[-1:]], axis=0)
        return out + (Q[2:] - 2.0 * Q[1:-1] + Q[:-2]) / h ** 2
    return out + (np.roll(P, 1, 0) + np.roll(P, -1, 0) - 2.0 * P) / h ** 2


def div_ref(u, v, w, h):
    """Cell divergence; w has nz faces (periodic) or nz + 1 (walls)."""
    d = (np.roll(u, -1, 2) - u + np.roll(v, -1, 1) - v) / h
    if w.shape[0] == u.shape[0] + 1:
        return d + (w[1:] - w[:-1]) / h
    return d + (np.roll(w, -1, 0) - w) / h


@pytest.mark.parametrize("shape", [(8, 12, 10), (9, 8, 16), (12, 6, 8)])
@pytest.mark.parametrize("zwalls", [False, True])
def test_poisson_solves_the_7_point_laplacian(shape, zwalls):
    rng = np.random.default_rng(51)
    h = 1.0 / shape[2]
    rhs = rng.standard_normal(shape)
    P = pr.poisson(rhs, h, zwalls)
    assert abs(P.mean()) < 1e-12 * np.abs(P).max()
    res = lap_ref(P, h, zwalls) - (rhs - rhs.mean())
    assert np.abs(res).max() < 1e-10 * np.abs(rhs).max()


@pytest.mark.parametrize("zwalls", [False, True])
def test_poisson_recovers_a_manufactured_field(zwalls):
    n = 16
    h = 1.0 / n
    c = (np.arange(n) + 0.5) * h
    Z, Y, X = np.meshgrid(c, c, c, indexing="ij")
    P0 = np.cos(2 * math.pi * X) * np.sin(2 * math.pi * Y + 0.3) * np.cos(math.pi * Z) + 0.2 * Z
    P0 -= P0.mean()
    P = pr.poisson(lap_ref(P0, h, zwalls), h, zwalls)
    np.testing.assert_allclose(P, P0, rtol=0, atol=1e-11)


def _inputs(shape, zwalls, seed):
    rng = np.random.default_rng(seed)
    nz, ny, nx = shape
    C = rng.uniform(-0.1, 1.1, shape)
    u = rng.standard_normal(shape)
    v = rng.standard_normal(shape)
    w = rng.standard_normal((nz + 1, ny, nx) if zwalls else shape)
    if zwalls:
        w[0] = w[-1] = 0.0
    P = rng.standard_normal(shape)
    Pold = rng.standard_normal(shape)
    return C, u, v, w, P, Pold


@pytest.mark.parametrize("zwalls", [False, True])
def test_updated_velocity_is_divergence_free_for_any_density_and_pressure_history(zwalls):
    """div u^{l+1} = div u* - dt [lap P^{l+1}/rho2 + div((1/rho - 1/rho2) grad Phat)],
    and eq-newpoi makes that zero whatever rho, P^l and P^{l-1} are."""
    shape = (10, 12, 14)
    h = 1.0 / 14
    C, u, v, w, P, Pold = _inputs(shape, zwalls, 52)
    un, vn, wn, Pn, Pl = pr.pressure_step(C, u, v, w, P, Pold, h, 1e-3, 1000.0, 1.0, zwalls)
    d0 = np.abs(div_ref(u, v, w, h)).max()
    assert np.abs(div_ref(un, vn, wn, h)).max() < 1e-10 * d0
    assert np.array_equal(Pl, P)
    if zwalls:
        assert np.all(wn[0] == 0.0) and np.all(wn[-1] == 0.0)


def _solenoidal(shape, zwalls, seed):
    rng = np.random.default_rng(seed)
    nz, ny, nx = shape
    if zwalls:
        zf = np.arange(nz + 1) / nz
        return inputs.coarse_wall_velocity(rng, shape, zf, kmax=3, nmodes_z=4)
    return inputs.random_solenoidal(rng, shape, 1.0 / nx, kmin=1, kmax=3)


@pytest.mark.parametrize("zwalls", [False, True])
def test_heavy_phase_everywhere_gives_the_closed_form(zwalls):
    """C = 1 (rho = rho1 everywhere) with a divergence-free u*: eq-newpoi
    gives lap P^{l+1} = (1 - rho2/rho1) lap Phat, so P^{l+1} is
    (1 - rho2/rho1)(2 P^l - P^{l-1}) up to its mean, and eq-u leaves u*
    unchanged.  (A cube, so the divergence-free generators' unit-box
    spacings equal h on every axis.)"""
    shape = (12, 12, 12)
    h = 1.0 / 12
    _, _, _, _, P, Pold = _inputs(shape, zwalls, 53)
    u, v, w = _solenoidal(shape, zwalls, 54)
    rho1, rho2 = 50.0, 2.0
    un, vn, wn, Pn, _ = pr.pressure_step(np.ones(shape), u, v, w, P, Pold, h, 1e-3, rho1, rho2,
                                         zwalls)
    Phat = 2.0 * P - Pold
    expect = (1.0 - rho2 / rho1) * (Phat - Phat.mean())
    np.testing.assert_allclose(Pn, expect, rtol=0, atol=1e-10 * np.abs(expect).max())
    for a, b in ((un, u), (vn, v), (wn, w)):
        np.testing.assert_allclose(a, b, rtol=0, atol=1e-10 * np.abs(b).max())


@pytest.mark.parametrize("zwalls", [False, True])
def test_light_phase_everywhere_is_the_plain_projection(zwalls):
    """C = 0 (rho = rho2): the explicit part vanishes, P^{l+1} does not
    depend on the pressure history and u^{l+1} = u* - dt grad P^{l+1}/rho2
    with lap P^{l+1} = (rho2/dt) div u*."""
    shape = (8, 10, 12)
    h = 1.0 / 12
    C, u, v, w, P, Pold = _inputs(shape, zwalls, 55)
    C[:] = 0.0
    dt, rho2 = 2e-3, 1.5
    r1 = pr.pressure_step(C, u, v, w, P, Pold, h, dt, 900.0, rho2, zwalls)
    r2 = pr.pressure_step(C, u, v, w, 3.0 * P, -Pold, h, dt, 900.0, rho2, zwalls)
    np.testing.assert_allclose(r1[3], r2[3], rtol=0, atol=1e-9 * np.abs(r1[3]).max())
    res = lap_ref(r1[3], h, zwalls) - (rho2 / dt) * div_ref(u, v, w, h)
    assert np.abs(res).max() < 1e-9 * np.abs(rho2 / dt * div_ref(u, v, w, h)).max()
    gx = (r1[3] - np.roll(r1[3], 1, 2)) / h
    np.testing.assert_allclose(r1[0], u - dt * gx / rho2, rtol=0, atol=1e-12 * np.abs(u).max())


def test_density_of_the_phases_and_clipping():
    C = np.array([-0.2, 0.0, 0.25, 0.5, 1.0, 1.3])
    np.testing.assert_allclose(pr.density(C, 10.0, 2.0), [2.0, 2.0, 4.0, 6.0, 10.0, 10.0],
                               rtol=0, atol=1e-15)


@pytest.mark.parametrize("zwalls", [False, True])
def test_new_pressure_solves_eq_newpoi_with_face_means(zwalls):
    """lap P^{l+1} equals the right-hand side of eq-newpoi assembled here
    cell by cell: the density of face i along x is the mean of cells i-1 and
    i, the explicit flux (1 - rho2/rho_f)(Phat_i - Phat_{i-1})/h."""
    shape = (8, 10, 12)
    h = 1.0 / 12
    C, u, v, w, P, Pold = _inputs(shape, zwalls, 56)
    rho1, rho2, dt = 20.0, 1.0, 1e-3
    _, _, _, Pn, _ = pr.pressure_step(C, u, v, w, P, Pold, h, dt, rho1, rho2, zwalls)
    rho = rho2 + (rho1 - rho2) * np.clip(C, 0, 1)
    Ph = 2.0 * P - Pold
    rhs = (rho2 / dt) * div_ref(u, v, w, h)
    for ax in (2, 1, 0):
        if ax == 0 and zwalls:
            rf = 0.5 * (rho[1:] + rho[:-1])                 # interior z faces 1 .. nz-1
            fl = (1.0 - rho2 / rf) * (Ph[1:] - Ph[:-1]) / h
            z = np.zeros_like(Ph[:1])
            fl = np.concatenate([z, fl, z])
            rhs += (fl[1:] - fl[:-1]) / h
        else:
            rf = 0.5 * (rho + np.roll(rho, 1, ax))
            fl = (1.0 - rho2 / rf) * (Ph - np.roll(Ph, 1, ax)) / h
            rhs += (np.roll(fl, -1, ax) - fl) / h
    res = lap_ref(Pn, h, zwalls) - (rhs - rhs.mean())
    assert np.abs(res).max() < 1e-9 * np.abs(rhs).max()
