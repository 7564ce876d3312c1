"""Pins of the oracle's drop diagnostics (sec. 4: drop volumes, the
effective diameter D with (4 pi / 3)(D/2)^3 = V, the PDF of D/H): drops are
face-connected cells with C >= 1/2, periodic axes wrapping.

The labelling is checked against scipy.ndimage.label (an independent
implementation; face connectivity is its default), on periodic fields by
labelling a 3 x 3 x 3 tiling; and on drops of known geometry."""
import math

import numpy as np
import pytest
from scipy import ndimage

import oracle
from paper_2105_01865_amd import inputs

W, P = oracle.NOFLUX, oracle.PERIODIC


def _same_partition(a, b):
    """Label arrays a, b (-1 / 0 = background) induce the same partition."""
    fa, fb = a >= 0, b > 0
    if not np.array_equal(fa, fb):
        return False
    pairs = set(zip(a[fa].tolist(), b[fb].tolist()))
    return len(pairs) == len(set(a[fa].tolist())) == len(set(b[fb].tolist()))


@pytest.mark.parametrize("shape,p", [((7, 9, 11), 0.3), ((12, 5, 8), 0.45), ((6, 6, 6), 0.2)])
def test_labelling_matches_scipy_between_walls(shape, p):
    rng = np.random.default_rng(31)
    C = (rng.random(shape) < p).astype(float)
    lab, nd = oracle.label_drops(C, 0.5, bc=(W, W, W))
    ref, nref = ndimage.label(C >= 0.5)
    assert nd == nref
    assert _same_partition(lab, ref)


def _torus_partition(C, bc):
    """Label the 3 x 3 x 3 tiling (tiling only the periodic axes) with scipy,
    then join the wrapped cells of every tiled component: any path on the
    torus splits into pieces that cross each seam at most once, and each
    such piece lies within the tiling."""
    shape = C.shape
    reps = tuple(3 if b == P else 1 for b in (bc[2], bc[1], bc[0]))
    big, _ = ndimage.label(np.tile(C, reps) >= 0.5)
    parent = list(range(C.size))

    def find(a):
        while parent[a] != a:
            parent[a] = parent[parent[a]]
            a = parent[a]
        return a

    zz, yy, xx = np.nonzero(big)
    wrapped = np.ravel_multi_index((zz % shape[0], yy % shape[1], xx % shape[2]), shape)
    first = {}
    for lab, w in zip(big[zz, yy, xx].tolist(), wrapped.tolist()):
        if lab in first:
            ra, rb = find(first[lab]), find(w)
            if ra != rb:
                parent[max(ra, rb)] = min(ra, rb)
        else:
            first[lab] = w
    out = np.zeros(C.size, dtype=np.int64)
    fg = (C >= 0.5).ravel()
    for i in np.flatnonzero(fg):
        out[i] = find(i) + 1
    return out.reshape(shape)


@pytest.mark.parametrize("bc", [(P, P, P), (P, P, W), (W, P, P)])
@pytest.mark.parametrize("p", [0.22, 0.4])
def test_labelling_matches_scipy_on_a_tiling_for_periodic_axes(bc, p):
    rng = np.random.default_rng(32)
    C = (rng.random((10, 12, 14)) < p).astype(float)
    ref = _torus_partition(C, bc)
    lab, nd = oracle.label_drops(C, 0.5, bc=bc)
    assert _same_partition(lab, ref)
    assert nd == len(set(lab[lab >= 0].tolist()))
    # the same field between walls splits at least as finely
    _, n_walls = oracle.label_drops(C, 0.5, bc=(W, W, W))
    assert n_walls >= nd


def test_labels_are_the_smallest_index_of_each_drop_and_walls_do_not_connect():
    rng = np.random.default_rng(33)
    C = (rng.random((8, 9, 10)) < 0.35).astype(float)
    lab, nd = oracle.label_drops(C, 0.5, bc=(P, W, P))
    flat = lab.ravel()
    for r in np.unique(flat[flat >= 0]):
        members = np.flatnonzero(flat == r)
        assert members.min() == r
    # a slab touching both walls of a wall axis stays one drop per slab,
    # and the two wall layers do not join across the wall
    C2 = np.zeros((6, 8, 5))
    C2[:, 0, :] = 1.0
    C2[:, -1, :] = 1.0
    _, n_wall = oracle.label_drops(C2, 0.5, bc=(P, W, P))
    _, n_per = oracle.label_drops(C2, 0.5, bc=(P, P, P))
    assert (n_wall, n_per) == (2, 1)


def test_threshold_is_inclusive_and_a_single_cell_is_a_drop():
    C = np.zeros((5, 5, 5))
    C[2, 2, 2] = 0.5
    C[0, 0, 0] = 0.5 - 1e-12
    lab, nd = oracle.label_drops(C, 0.5)
    assert nd == 1 and lab[2, 2, 2] == (2 * 5 + 2) * 5 + 2 and lab[0, 0, 0] == -1
    # a cell exactly at the threshold joins the drop it touches
    C[1, 1, 1] = 1.0
    C[1, 1, 2] = 0.5
    C[1, 2, 1] = 0.5
    lab, nd = oracle.label_drops(C, 0.5)
    r = (1 * 5 + 1) * 5 + 1
    assert nd == 2 and lab[1, 1, 2] == r and lab[1, 2, 1] == r


def test_drop_volumes_and_effective_diameters_of_spheres():
    """Spheres of radius R (tanh profile) placed across the periodic corner:
    one drop each, V = h^3 #cells equal to the cells inside the C = 1/2
    surface, and D = (6V/pi)^(1/3) within a cell of 2R."""
    n = 48
    h = 1.0 / n
    centres = np.array([[0.02, 0.97, 0.5], [0.5, 0.5, 0.02], [0.7, 0.3, 0.6]])
    radii = np.array([8.0, 6.0, 10.0]) * h
    C = inputs.drop_field((n, n, n), h, h, centres, radii)
    lab, nd = oracle.label_drops(C, 0.5)
    assert nd == 3
    roots, cells, V, D = oracle.drop_volumes(lab, h)
    assert cells.sum() == np.count_nonzero(C >= 0.5)
    # match drops to spheres by a member cell near each centre
    for c, R in zip(centres, radii):
        idx = tuple(int(q / h) % n for q in (c[2], c[1], c[0]))
        k = np.searchsorted(roots, lab[idx])
        assert roots[k] == lab[idx]
        assert abs(D[k] - 2 * R) < 1.5 * h, (D[k], 2 * R)
        assert abs(V[k] - 4.0 / 3.0 * math.pi * R ** 3) < 0.12 * 4.0 / 3.0 * math.pi * R ** 3
