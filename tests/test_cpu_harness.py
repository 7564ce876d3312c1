"""The device code of libch, run on the CPU by the harness in
tests/cpu_harness (AddressSanitizer + UBSan, exact LDS sizes), against the
FP64 oracle.  This checks the kernels' indexing, halos, segments, the
chunked line recurrences and the batch layout without a GPU."""
import math

import numpy as np
import pytest

import oracle
from paper_2105_01865_amd import inputs
from tests.harness_util import run_emu


def _box(shape, bc=(0, 0, 0), seed=0, amp=1.0, drops=True):
    rng = np.random.default_rng(seed)
    nz, ny, nx = shape
    h = 1.0 / max(shape)
    if drops:
        cen, rad = inputs.place_drops(rng, 3, 2, 4, shape, h, walls_z=bc[2] == 1, gap_cells=1)
        C = inputs.drop_field(shape, h, h, cen, rad, walls_z=bc[2] == 1)
        C = C + 0.02 * rng.normal(size=shape)
    else:
        C = 0.5 + 0.3 * rng.normal(size=shape)
    if bc == (0, 0, 0):
        Ax, Ay, Az = (rng.normal(size=shape) for _ in range(3))
        u, v, w = inputs.curl_velocity(Ax, Ay, Az, h)
    elif bc == (0, 0, 1):
        zf = np.arange(nz + 1) / nz
        u, v, w = inputs.coarse_wall_velocity(rng, shape, zf, kmax=3, nmodes_z=3)
    elif bc == (1, 0, 1):
        # walls in x and z: a stream function on the x-z cell corners that
        # vanishes on the walls; v depends on x and z only
        xf = np.arange(nx + 1) / nx
        zf = np.arange(nz + 1) / nz
        psi = sum(rng.normal() * np.outer(np.sin(m * np.pi * zf), np.sin(q * np.pi * xf))
                  for m in (1, 2) for q in (1, 3))                       # (nz+1, nx+1)
        u = np.repeat(((psi[1:, :] - psi[:-1, :]) / h)[:, None, :], ny, axis=1)
        w = np.repeat((-(psi[:, 1:] - psi[:, :-1]) / h)[:, None, :], ny, axis=1)
        v = np.repeat(rng.normal(size=(nz, 1, nx)), ny, axis=1)
    else:
        u, v, w = inputs.wall_velocity(rng, shape, bc, h)
    s = amp / max(np.abs(u).max(), np.abs(v).max(), np.abs(w).max())
    return dict(C=C, u=u * s, v=v * s, w=w * s, h=h, Cn=h, Pe=0.9 / h, bc=bc)


def _oracle(b, dt, nsteps, kappa=4.0):
    return oracle.step(b["C"], b["u"], b["v"], b["w"], b["h"], b["Cn"], b["Pe"], dt, nsteps,
                       bc=b["bc"], kappa=kappa)


def _rel(a, b):
    return np.abs(a - b).max() / np.abs(b).max()


def test_32cube_fp64_matches_oracle():
    wl = inputs.make_workload(1)
    b = dict(C=wl.C, u=wl.u, v=wl.v, w=wl.w, h=wl.h, Cn=wl.Cn, Pe=wl.Pe, bc=(0, 0, 0))
    (C1,), (m,), plan = run_emu([b], wl.dt, 2)
    ref = _oracle(b, wl.dt, 2)
    assert _rel(C1, ref) < 1e-12
    assert _rel(C1 - wl.C, ref - wl.C) < 1e-10      # the increment itself
    assert abs(m - oracle.mass(ref, wl.h)) < 1e-13 * abs(m)


@pytest.mark.parametrize("zc", [1, 3, 7])
@pytest.mark.parametrize("shape,bc", [((20, 12, 16), (0, 0, 0)), ((16, 9, 24), (0, 0, 1)),
                                      ((12, 16, 8), (1, 0, 1)), ((1, 24, 16), (0, 0, 0)),
                                      ((16, 20, 1), (0, 0, 0)), ((12, 1, 16), (0, 0, 1))])
def test_fp64_matches_oracle_ragged_and_walls(shape, bc, zc):
    b = _box(shape, bc=bc, seed=1, amp=2.0)
    dt = 2e-4
    # odd row counts, ragged z chunks and short segments force ragged tiles,
    # partial marches and segmented lines
    out, masses, plan = run_emu([b], dt, 2, x_rows=3, seg=5, waves=3, z_chunk=zc)
    assert plan["z_chunk"] == zc
    ref = _oracle(b, dt, 2)
    assert _rel(out[0], ref) < 1e-12
    assert plan["ntask"][1] > 0


@pytest.mark.parametrize("zc", [1, 4])
@pytest.mark.parametrize("shape,bc,opts", [
    ((10, 12, 17), (1, 0, 0), dict(x_rows=3, seg=5)),     # x walls, odd nx
    ((9, 13, 16), (0, 1, 0), dict(x_rows=2, seg=4)),      # y walls, tiles touching them
    ((11, 10, 9), (1, 1, 1), {}),                         # walls everywhere
    ((12, 9, 8), (1, 0, 0), dict(x_rows=4)),              # x walls, the shortest x line
    ((10, 9, 1), (1, 1, 0), dict(x_rows=3)),              # degenerate x with x walls
    ((8, 11, 13), (1, 1, 0), dict(x_rows=5, seg=3, waves=2)),
    ((14, 8, 1), (0, 1, 1), {}),                          # degenerate x between y walls
    ((1, 12, 10), (1, 1, 0), {}),                         # degenerate z
])
def test_fp64_matches_oracle_walls_in_x_and_y(shape, bc, opts, zc):
    """No-flux walls along x and y: the wall face flux, the reflected x halo
    (also where every column of the tile is a halo column), the y-wall top
    face, segmented lines reaching a wall."""
    b = _box(shape, bc=bc, seed=17, amp=2.0, drops=min(shape) > 4)
    dt = 2e-4
    out, masses, plan = run_emu([b], dt, 2, z_chunk=zc, **opts)
    ref = _oracle(b, dt, 2)
    assert _rel(out[0], ref) < 1e-12
    assert abs(masses[0] - oracle.mass(ref, b["h"])) < 1e-12 * abs(masses[0])
    out32, _, _ = run_emu([b], dt, 2, prec=1, z_chunk=zc, **opts)
    assert _rel(out32[0], ref) < 2e-6


@pytest.mark.parametrize("shape,bc,zc", [((60, 10, 32), (0, 0, 0), 24), ((50, 9, 24), (0, 0, 1), 20)])
def test_fp64_long_marches(shape, bc, zc):
    # more planes per task than the automatic plan takes (the autotuner's
    # 20 and 24), ragged last march
    b = _box(shape, bc=bc, seed=7, amp=2.0)
    out, _, plan = run_emu([b], 2e-4, 2, z_chunk=zc, x_rows=1)
    assert plan["z_chunk"] == zc
    assert _rel(out[0], _oracle(b, 2e-4, 2)) < 1e-12


def test_fp64_large_dt_needs_long_warmup():
    b = _box((16, 16, 16), seed=2, amp=0.5, drops=False)
    dt = 0.05          # r >> 1: long recurrence warm-up, wrapping the line
    out, _, plan = run_emu([b], dt, 1)
    assert plan["tw_max"] > 16
    ref = _oracle(b, dt, 1)
    assert _rel(out[0], ref) < 1e-12


def test_kappa3_and_default_plan():
    b = _box((24, 24, 24), seed=3)
    out, _, plan = run_emu([b], 1e-4, 1, kappa=3.0)
    ref = _oracle(b, 1e-4, 1, kappa=3.0)
    assert _rel(out[0], ref) < 1e-12


@pytest.mark.parametrize("solve", [0, 1, 2])
def test_fp32_close_to_fp64_oracle(solve):
    b = _box((16, 16, 16), seed=4, amp=1.0)
    out, _, plan = run_emu([b], 2e-4, 3, prec=1, solve=solve)
    ref = _oracle(b, 2e-4, 3)
    assert plan["acc64"] == (1 if solve == 1 else 0)
    assert _rel(out[0], ref) < 2e-6


def test_batch_equals_single_boxes_bitwise():
    boxes = [_box((16, 16, 16), seed=5), _box((8, 12, 24), seed=6), _box((24, 8, 8), seed=7)]
    dt = 3e-4
    batch, bm, _ = run_emu(boxes, dt, 2)
    for b, got, m in zip(boxes, batch, bm):
        (single,), (sm,), _ = run_emu([b], dt, 2)
        assert np.array_equal(got, single)
        assert m == sm
        assert _rel(got, _oracle(b, dt, 2)) < 1e-12


def test_long_x_lines_two_cells_per_thread():
    # x lines longer than one work-group: each thread owns two cells
    b = _box((8, 9, 1100), seed=12, amp=1.0, drops=False)
    out, _, plan = run_emu([b], 2e-4, 1, z_chunk=3)
    assert _rel(out[0], _oracle(b, 2e-4, 1)) < 1e-12


@pytest.mark.parametrize("zc", [1, 3])
@pytest.mark.parametrize("shape,bc", [((20, 12, 16), (0, 0, 0)), ((16, 9, 24), (0, 0, 1)),
                                      ((12, 16, 8), (1, 0, 1)), ((1, 24, 16), (0, 0, 0)),
                                      ((8, 8, 1100), (0, 0, 0))])
def test_explicit25_matches_oracle(shape, bc, zc):
    """The explicit 25-point mode of the x-pass program (no solves, mixed
    second differences, C + RHS written out) against the oracle's explicit
    scheme, including walls, a degenerate axis and two cells per thread."""
    b = _box(shape, bc=bc, seed=11)
    dt = 1e-4 if shape[2] < 1000 else 2e-6       # below the explicit limit
    ref = oracle.step_explicit25(b["C"], b["u"], b["v"], b["w"], b["h"], b["Cn"], b["Pe"], dt,
                                 2, bc=bc)
    out, masses, plan = run_emu([b], dt, 2, mode=1, z_chunk=zc)
    assert plan["x_rows"] == 1
    assert _rel(out[0], ref) < 1e-12
    assert _rel(out[0] - b["C"], ref - b["C"]) < 1e-9
    assert abs(masses[0] - oracle.mass(ref, b["h"])) < 1e-12 * abs(masses[0])
    out32, _, _ = run_emu([b], dt, 2, prec=1, mode=1, z_chunk=zc)
    assert _rel(out32[0], ref) < 2e-6


@pytest.mark.parametrize("shape,bc,zc", [
    ((12, 10, 16), (0, 0, 0), 5),      # 16 of 64 threads live, ragged march
    ((9, 11, 70), (0, 0, 1), 4),       # two waves, the second partly idle
    ((10, 12, 17), (1, 0, 0), 3),      # x walls: the wall face, reflected halo columns
    ((9, 13, 16), (0, 1, 0), 4),       # y walls: reflected halo rows, the wall face ny
    ((11, 10, 9), (1, 1, 1), 2),
    ((8, 1, 24), (0, 0, 0), 3),        # degenerate y
    ((1, 9, 20), (0, 1, 0), 1),        # degenerate z
    ((14, 8, 8), (1, 1, 0), 7),        # the shortest x line
])
def test_row_program_equals_the_general_one(shape, bc, zc):
    """The row x program (one cell per thread, the y stencil in registers;
    as many rows per task as fill the group) and the general one give the
    same bits, and both the oracle's step."""
    b = _box(shape, bc=bc, seed=23, amp=2.0, drops=min(shape) > 4)
    dt = 2e-4
    ref = _oracle(b, dt, 2)
    for prec, solve, tol in ((0, 0, 1e-12), (1, 0, 2e-6), (1, 1, 2e-6)):
        out = {}
        for xg in (0, 1):
            o, m, plan = run_emu([b], dt, 2, prec=prec, solve=solve, x_rows=1, z_chunk=zc,
                                 x_general=xg)
            assert (plan["xrow"] > 0) == (xg == 0)
            out[xg] = (o[0], m[0])
        assert np.array_equal(out[0][0], out[1][0])
        assert out[0][1] == out[1][1]
        assert _rel(out[0][0], ref) < tol


@pytest.mark.parametrize("x_rows", [1, 2])
def test_row_program_in_a_batch(x_rows):
    # boxes of different widths in one launch: the narrow ones take several
    # rows per task (ragged last tasks), the widest one or two
    boxes = [_box((16, 12, 40), seed=31), _box((10, 9, 8), seed=32, bc=(0, 0, 0)),
             _box((12, 14, 33), seed=33), _box((9, 9, 13), seed=34, bc=(0, 1, 1))]
    dt = 3e-4
    got, masses, plan = run_emu(boxes, dt, 2, x_rows=x_rows)
    # the 40- and 33-wide boxes take one row per task at x_rows 1: two launches
    assert plan["xrow"] == (4 if x_rows == 1 else 2)
    gen, _, _ = run_emu(boxes, dt, 2, x_rows=x_rows, x_general=1)
    for a, g, b in zip(got, gen, boxes):
        assert np.array_equal(a, g)
        assert _rel(a, _oracle(b, dt, 2)) < 1e-12


@pytest.mark.parametrize("boxes,x_rows,xrm", [
    # rows of whole waves: 3 rows of 64 per task, the last task one row (two
    # idle waves); 2 rows of 128 with y and z walls, the last task one row
    ([((12, 10, 64), (0, 0, 0))], 3, [2]),
    ([((9, 9, 128), (0, 1, 1))], 2, [2]),
    # a batch: the 256-wide box one row per task, the 64- and 128-wide ones
    # several rows of whole waves in groups of 256 threads (two launches)
    ([((8, 8, 256), (0, 0, 0)), ((10, 9, 64), (0, 0, 1)), ((8, 11, 128), (0, 0, 0))], 0,
     [0, 2]),
    # a 48-wide box among them: four rows in groups of 192 threads with
    # per-thread row offsets, a launch of its own (three launches)
    ([((8, 8, 256), (0, 0, 0)), ((10, 9, 48), (0, 0, 0)), ((8, 11, 128), (0, 0, 0))], 0,
     [0, 1, 2]),
])
def test_wave_rows(boxes, x_rows, xrm):
    """Several rows per task whose rows are whole waves (the row offsets
    uniform per wave) give the bits of the general program, and the
    oracle's step."""
    bs = [_box(sh, bc=bc, seed=71 + i, amp=2.0) for i, (sh, bc) in enumerate(boxes)]
    dt = 2e-4
    for prec, tol in ((0, 1e-12), (1, 2e-6)):
        got, _, plan = run_emu(bs, dt, 2, prec=prec, x_rows=x_rows)
        assert plan["xrm"] == xrm
        gen, _, _ = run_emu(bs, dt, 2, prec=prec, x_rows=x_rows, x_general=1)
        for a, g, b in zip(got, gen, bs):
            assert np.array_equal(a, g)
            assert _rel(a, _oracle(b, dt, 2)) < tol


def test_launches_per_row_mode_with_their_own_group_size():
    """An ensemble-like batch (x extents 48 .. 192) in the automatic plan:
    one launch per row mode, each box in 192 or 256 threads, whichever
    leaves fewer idle: 160- and 192-cell boxes one row in 192 threads, 48-
    and 96-cell boxes 4 and 2 rows in 192 (per-thread row offsets), 64- and
    128-cell boxes rows of whole waves in 256.  The bits are the general
    program's."""
    widths = (48, 64, 96, 128, 160, 192)
    bs = [_box((8, 9, nx), seed=80 + i, amp=1.5, drops=False) for i, nx in enumerate(widths)]
    dt = 2e-4
    got, _, plan = run_emu(bs, dt, 1, prec=0)
    assert plan["xrow"] == 4 and plan["nxl"] == 3
    assert plan["xrm"] == [0, 1, 2] and plan["nth"] == [192, 192, 256]
    gen, _, _ = run_emu(bs, dt, 1, prec=0, x_general=1)
    for a, g, b in zip(got, gen, bs):
        assert np.array_equal(a, g)
        assert _rel(a, _oracle(b, dt, 1)) < 1e-12


@pytest.mark.parametrize("prec", [0, 1])
def test_launch_plan_does_not_change_the_bits(prec):
    """Every face flux is formed from the same differences whatever the tile:
    rows per task, planes per task, segment length and the x program leave
    the result bit for bit the same."""
    b = _box((18, 13, 24), bc=(0, 0, 1), seed=41, amp=2.0)
    dt = 2e-4
    ref, _, _ = run_emu([b], dt, 2, prec=prec, x_rows=1, z_chunk=18)
    for opts in (dict(x_rows=1, z_chunk=4), dict(x_rows=1, z_chunk=5, x_general=1),
                 dict(x_rows=3, z_chunk=7, seg=5), dict(x_rows=2, z_chunk=1, waves=2)):
        got, _, _ = run_emu([b], dt, 2, prec=prec, **opts)
        assert np.array_equal(got[0], ref[0]), opts


@pytest.mark.parametrize("prec,solve", [(0, 0), (1, 0), (1, 1)])
@pytest.mark.parametrize("shape,bc,opts", [
    ((20, 24, 64), (0, 0, 0), dict(seg=7)),          # full 32-column tasks, short segments
    ((19, 17, 96), (0, 1, 1), dict(seg=11, waves=2)),  # walls in y and z, 2 waves per task
    ((12, 9, 40), (0, 0, 1), {}),                     # 32 + 8 columns: one full task, one partial
])
def test_line_fast_path_equals_the_elementwise_path(shape, bc, opts, prec, solve):
    """The y/z passes' 16-byte path (rows straight into LDS, vector
    write-back) against the element-wise path, bit for bit, and the oracle."""
    b = _box(shape, bc=bc, seed=51, amp=2.0)
    dt = 2e-4
    fast, mf, _ = run_emu([b], dt, 2, prec=prec, solve=solve, **opts)
    slow, ms, _ = run_emu([b], dt, 2, prec=prec, solve=solve, line_vec=False, **opts)
    assert np.array_equal(fast[0], slow[0]) and mf == ms
    assert _rel(fast[0], _oracle(b, dt, 2)) < (1e-12 if prec == 0 else 2e-6)


@pytest.mark.parametrize("prec", [0, 1])
@pytest.mark.parametrize("shape,dt,zc", [
    ((8, 8, 1100), 2e-6, 0),       # five segments of 220
    ((9, 8, 1093), 4e-5, 3),       # long warm-ups: shorter, more segments, ragged last one
    ((8, 1, 1200), 1e-6, 2),       # degenerate y
])
def test_segmented_program_for_long_lines(shape, dt, zc, prec):
    """x lines longer than a work-group (periodic x): one row and one x
    segment per task, solved from computed warm-ups, E double-buffered; against
    the oracle and the general program (two cells per thread)."""
    b = _box(shape, seed=61, amp=1.0, drops=False)
    ref = _oracle(b, dt, 2)
    seg, ms, plan = run_emu([b], dt, 2, prec=prec, z_chunk=zc)
    assert plan["xrow"] == 3
    gen, mg, plan_g = run_emu([b], dt, 2, prec=prec, z_chunk=zc, x_general=1)
    assert plan_g["xrow"] == 0
    tol = 1e-12 if prec == 0 else 2e-6
    assert _rel(seg[0], ref) < tol and _rel(gen[0], ref) < tol
    if prec == 0:
        assert _rel(seg[0], gen[0]) < 1e-13
        assert abs(ms[0] - oracle.mass(ref, b["h"])) < 1e-12 * abs(ms[0])


def test_long_lines_with_x_walls_take_the_general_program():
    b = _box((8, 8, 1100), bc=(1, 0, 0), seed=62, amp=1.0, drops=False)
    out, _, plan = run_emu([b], 2e-6, 1)
    assert plan["xrow"] == 0
    assert _rel(out[0], _oracle(b, 2e-6, 1)) < 1e-12
