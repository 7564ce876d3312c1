"""The windowed oracle (tests/windowed.py) reproduces the whole-box oracle at
the centre of its window, at the parameters of the 1536^3 workload."""
import numpy as np
import pytest

import oracle
from paper_2105_01865_amd import inputs
from tests.windowed import periodic_window, window_step


@pytest.mark.parametrize("lo", [(84, 80, 90),      # window across the periodic wrap
                                (10, 20, 5)])
def test_window_centre_matches_whole_box(lo):
    n, W, c0, cw = 96, 64, 24, 16
    h = 1.0 / 1536
    rng = np.random.default_rng(4096)
    shape = (n, n, n)
    cen, rad = inputs.place_drops(rng, 12, 4, 20, shape, h)
    C = inputs.drop_field(shape, h, h, cen, rad)
    u, v, w = inputs.random_solenoidal(rng, shape, h, 1, 16)
    umax = np.abs(u).max() + np.abs(v).max() + np.abs(w).max()
    dt = min(1e-4, 0.8 * h / umax)
    full = oracle.step(C, u, v, w, h, h, 0.9 / h, dt, 1)
    sub = window_step(C, u, v, w, lo, W, h, h, 0.9 / h, dt, 1)
    got = sub[c0:c0 + cw, c0:c0 + cw, c0:c0 + cw]
    ref = periodic_window(full, tuple(l + c0 for l in lo), cw)
    assert np.abs(got - ref).max() <= 1e-12 * np.abs(ref).max()
    # and the margin matters: a window's cells next to its faces are wrong
    edge = sub[0:2]
    ref_edge = periodic_window(full, lo, W)[0:2]
    assert np.abs(edge - ref_edge).max() > 1e-9
