"""Checks of the seeded synthetic input generators."""
import math

import numpy as np
import pytest

from paper_2105_01865_amd import inputs


def test_abc_field_is_exactly_solenoidal():
    u, v, w = inputs.abc_velocity((16, 12, 20), 1 / 16, 0.1, 0.2, 0.15)
    assert np.abs(inputs.staggered_divergence(u, v, w, 1 / 16)).max() == 0.0


def test_random_field_is_solenoidal_with_unit_rms_and_k53_spectrum():
    rng = np.random.default_rng(1)
    n = 64
    h = 1.0 / n
    u, v, w = inputs.random_solenoidal(rng, (n, n, n), h, 1, 16)
    assert np.abs(inputs.staggered_divergence(u, v, w, h)).max() < 1e-11
    rms = math.sqrt((np.mean(u * u) + np.mean(v * v) + np.mean(w * w)) / 3)
    assert abs(rms - 1.0) < 1e-12
    # shell-averaged spectrum slope over the band (loose: random phases)
    uh = np.fft.fftn(u)
    vh = np.fft.fftn(v)
    wh = np.fft.fftn(w)
    k = np.fft.fftfreq(n, 1 / n)
    K = np.sqrt(k[:, None, None] ** 2 + k[None, :, None] ** 2 + k[None, None, :] ** 2)
    E = np.abs(uh) ** 2 + np.abs(vh) ** 2 + np.abs(wh) ** 2
    shells = np.arange(2, 15)
    Es = np.array([E[(K >= s - 0.5) & (K < s + 0.5)].sum() for s in shells])
    slope = np.polyfit(np.log(shells), np.log(Es), 1)[0]
    assert -2.3 < slope < -1.1, slope
    assert E[K > 20].sum() < 1e-3 * E.sum()


def test_wall_field_is_solenoidal_with_zero_wall_velocity():
    rng = np.random.default_rng(2)
    zf = inputs.stretched_faces(24, 2.0)
    uc, vc, wc = inputs.coarse_wall_velocity(rng, (24, 32, 32), zf, kmax=8)
    assert np.abs(inputs.stretched_divergence(uc, vc, wc, zf)).max() < 1e-10
    assert np.all(wc[0] == 0) and np.all(wc[-1] == 0)
    assert zf[0] == 0.0 and zf[-1] == 1.0 and np.all(np.diff(zf) > 0)
    # clustered at the walls
    assert np.diff(zf)[0] < np.diff(zf)[12] / 2


def test_drops_do_not_overlap_and_profile_is_tanh():
    rng = np.random.default_rng(3)
    shape = (48, 48, 48)
    h = 1 / 48
    cen, rad = inputs.place_drops(rng, 12, 4, 8, shape, h)
    for i in range(len(rad)):
        for j in range(i):
            d = cen[i] - cen[j]
            d -= np.round(d)
            assert np.sqrt((d * d).sum()) >= rad[i] + rad[j] + 4 * h - 1e-12
    C = inputs.drop_field(shape, h, h, cen[:1], rad[:1])
    assert C.max() <= 1.0 and C.min() >= 0.0
    # C = 1/2 on the sphere R (sampled along x through the centre)
    c = cen[0]
    x = (np.arange(48) + 0.5) * h
    prof = C[int(c[2] / h), int(c[1] / h), :]
    assert prof.max() > 0.9


def test_seeds_are_reproducible():
    a = inputs.make_workload(2, n=32)
    b = inputs.make_workload(2, n=32)
    np.testing.assert_array_equal(a.C, b.C)
    np.testing.assert_array_equal(a.u, b.u)
    c = inputs.make_workload(5, box=3)
    d = inputs.make_workload(5, box=3)
    assert c.shape == d.shape and c.shape[0] in (48, 64, 96, 128, 160, 192)
    np.testing.assert_array_equal(c.C, d.C)


def test_32cube_workload_matches_its_description():
    w = inputs.make_workload(1)
    assert w.shape == (32, 32, 32) and w.h == 1 / 32 and w.Cn == w.h
    assert abs(w.Pe - 0.9 / w.Cn) < 1e-12 and w.dt == 1e-4 and w.nsteps == 100
    # one sphere of radius 8h at the centre: C ~ 1/2 at distance 8h
    assert w.C[16, 16, 16] > 0.99 and w.C[0, 0, 0] < 1e-3
