"""Pins of the library's own transfer stencils (sec. 3.4: a tensor product of
1-D cubic Hermite interpolants, four source points per direction, the
stencil built once per transfer).  The tables come from ch_plan.h, compiled
for the host with sanitizers; they are checked against what the
interpolant must satisfy, and then against the oracle's independently
written stencils."""
import math

import numpy as np
import pytest

import oracle
from paper_2105_01865_amd import inputs
from tests.harness_util import lib_stencils

PERIODIC, MIRROR, ANTI = 0, 1, 2


def _value(st, f):
    idx, w = st
    return (w * f[idx]).sum(axis=1)


def _axes():
    zf = inputs.stretched_faces(24, 2.0)
    zc = 0.5 * (zf[:-1] + zf[1:])
    return dict(uniform_faces=np.arange(16) / 16.0, uniform_centres=(np.arange(16) + 0.5) / 16.0,
                stretched_centres=zc, stretched_faces=zf)


@pytest.mark.parametrize("name,kind", [("uniform_faces", PERIODIC), ("uniform_centres", PERIODIC),
                                       ("stretched_centres", MIRROR)])
def test_partition_of_unity_and_nodes(name, kind):
    s = _axes()[name]
    t = np.concatenate([s, np.linspace(0.0, 1.0 - 1e-12, 41)])
    st = lib_stencils(kind, s, t)
    assert st is not None
    # constants are reproduced everywhere, across the wrap and the walls
    assert np.abs(st[1].sum(axis=1) - 1.0).max() < 1e-14
    # at a node the interpolant takes that node's value and nothing else
    idx, w = st
    for i in range(len(s)):
        f = np.zeros(len(s))
        f[i] = 1.0
        assert abs(_value((idx[i:i + 1], w[i:i + 1]), f)[0] - 1.0) < 1e-15
        assert np.abs(w[i]).sum() - 1.0 < 1e-15


def test_linear_exact_on_stretched_axis():
    s = _axes()["stretched_centres"]
    # targets whose four points are stored points (no wall image)
    t = np.linspace(s[1], s[-2] - 1e-12, 57)
    st = lib_stencils(MIRROR, s, t)
    f = 0.3 - 2.0 * s
    assert np.abs(_value(st, f) - (0.3 - 2.0 * t)).max() < 1e-13
    # a chord slope on a stretched axis is not exact for a quadratic
    g = s * s
    assert np.abs(_value(st, g) - t * t).max() > 1e-6


def test_quadratic_exact_on_uniform_axis_and_cubic_not():
    s = np.arange(32) / 32.0
    t = np.linspace(s[1], s[-3], 61)
    st = lib_stencils(PERIODIC, s, t)
    q = lambda x: 1.0 - x + 3.0 * x * x
    assert np.abs(_value(st, q(s)) - q(t)).max() < 1e-13
    c = lambda x: x ** 3
    assert np.abs(_value(st, c(s)) - c(t)).max() > 1e-7


def test_periodic_wrap_is_a_shift():
    # a periodic interpolant commutes with shifts by whole cells: the
    # stencil at t + j/n is the one at t with every index moved by j
    n = 12
    s = (np.arange(n) + 0.5) / n
    t = np.array([0.01, 0.3, 0.77])
    base = lib_stencils(PERIODIC, s, t)
    for j in (1, 5, 11):
        moved = lib_stencils(PERIODIC, s, (t + j / n) % 1.0)
        assert np.array_equal(moved[0], (base[0] + j) % n)
        assert np.abs(moved[1] - base[1]).max() < 1e-13


def test_odd_axis_zero_at_walls_and_exact_through_them():
    zf = _axes()["stretched_faces"]
    rng = np.random.default_rng(3)
    f = rng.normal(size=zf.size)
    f[0] = f[-1] = 0.0
    st = lib_stencils(ANTI, zf, np.array([0.0, 1.0]))
    assert np.abs(_value(st, f)).max() == 0.0
    # a function odd about the bottom wall (and one odd about the top) is
    # continued by itself, so the stencils reaching past that wall stay
    # exact for it when it is linear
    t = np.linspace(0.0, zf[2], 9)
    st = lib_stencils(ANTI, zf, t)
    assert np.abs(_value(st, 2.5 * zf) - 2.5 * t).max() < 1e-13
    t = np.linspace(zf[-3], 1.0 - 1e-12, 9)
    st = lib_stencils(ANTI, zf, t)
    assert np.abs(_value(st, 1.0 - zf) - (1.0 - t)).max() < 1e-13


def test_mirror_axis_even_through_walls():
    # data even about the bottom wall: the stencils reaching past it see the
    # same values a longer axis would hold there, so s^2 interpolates as on
    # the symmetric axis built out explicitly
    zc = _axes()["stretched_centres"]
    sym = np.concatenate([-zc[::-1], zc])           # the axis continued by hand
    t = np.linspace(1e-9, zc[1], 7)
    st = lib_stencils(MIRROR, zc, t)
    g = lambda x: np.cos(3.0 * x)                    # even about 0
    got = _value(st, g(zc))
    # the same interpolant on the hand-built symmetric axis, from its stored
    # points only (no image needed at these targets)
    ref = _value(lib_stencils(MIRROR, (sym + 1.0) / 2.0, (t + 1.0) / 2.0), g(sym))
    assert np.abs(got - ref).max() < 1e-14


def test_converges_third_order_on_smooth_periodic_data():
    errs = []
    for n in (16, 32, 64, 128):
        s = (np.arange(n) + 0.5) / n
        t = np.linspace(0.0, 1.0, 301, endpoint=False)
        st = lib_stencils(PERIODIC, s, t)
        f = lambda x: np.sin(2 * math.pi * x) + 0.3 * np.cos(6 * math.pi * x)
        errs.append(np.abs(_value(st, f(s)) - f(t)).max())
    rates = [math.log2(errs[i] / errs[i + 1]) for i in range(3)]
    assert min(rates) > 2.8


def test_refuses_a_target_the_axis_cannot_bracket():
    # a two-point mirrored axis has four points in all; a target needs a
    # full window of four around its interval
    assert lib_stencils(MIRROR, np.array([0.25, 0.75]), np.array([0.5])) is not None
    assert lib_stencils(MIRROR, np.array([0.5]), np.array([0.5])) is None


@pytest.mark.parametrize("name,kind,okind", [
    ("uniform_faces", PERIODIC, oracle.AX_PERIODIC), ("uniform_centres", PERIODIC, oracle.AX_PERIODIC),
    ("stretched_centres", MIRROR, oracle.AX_WALL_EVEN), ("stretched_faces", ANTI, oracle.AX_WALL_ODD)])
def test_agrees_with_the_oracle_stencils(name, kind, okind):
    s = _axes()[name]
    t = np.concatenate([np.linspace(0.0, 1.0, 97), np.arange(40) / 40.0 + 1e-3])
    t = t[t < 1.0] if kind == PERIODIC else t
    idx, w = lib_stencils(kind, s, t)
    for q, tq in enumerate(t):
        oi, ow = oracle.hermite_stencil(s, 1.0, okind, tq)
        # the same source value gets the same total weight
        a = np.zeros(len(s))
        b = np.zeros(len(s))
        np.add.at(a, idx[q], w[q])
        np.add.at(b, oi, ow)
        assert np.abs(a - b).max() < 1e-15
