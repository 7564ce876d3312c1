"""GPU parity of libch against the FP64 CPU oracle, through the C ABI.

FP64 bar: relative L-infinity error of C after one step <= 1e-12 (the
tolerance of the project's stated target).  FP32 bar: derived from the
arithmetic (see the design notes): <= 5e-6 relative after a few steps.
"""
import ctypes
import math
import sys

import numpy as np
import pytest
import torch

import oracle
from paper_2105_01865_amd import ch, inputs

pytestmark = pytest.mark.gpu

TOL64 = 1e-12


@pytest.fixture(autouse=True)
def _gpu():
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    yield
    torch.cuda.synchronize()


def dev(a, dtype=torch.float64):
    return torch.from_numpy(np.ascontiguousarray(a)).to(device="cuda", dtype=dtype)


def rel(a, b):
    return float(np.abs(a - b).max() / np.abs(b).max())


def _case(shape, bc=(0, 0, 0), seed=0, amp=1.0):
    rng = np.random.default_rng(seed)
    nz, ny, nx = shape
    h = 1.0 / max(shape)
    cen, rad = inputs.place_drops(rng, 4, 2, 5, shape, h, walls_z=bc[2] == 1, gap_cells=1)
    C = inputs.drop_field(shape, h, h, cen, rad, walls_z=bc[2] == 1)
    C = C + 0.01 * rng.normal(size=shape)
    if bc == (0, 0, 0):
        u, v, w = inputs.curl_velocity(*(rng.normal(size=shape) for _ in range(3)), h)
    elif bc == (0, 0, 1):
        u, v, w = inputs.coarse_wall_velocity(rng, shape, np.arange(nz + 1) / nz, kmax=4,
                                              nmodes_z=4)
    else:
        u, v, w = inputs.wall_velocity(rng, shape, bc, h)
    s = amp / max(np.abs(u).max(), np.abs(v).max(), np.abs(w).max())
    return C, u * s, v * s, w * s, h


def run_gpu(C, u, v, w, h, Cn, Pe, dt, nsteps, bc=(0, 0, 0), precision="fp64", stream=True,
            **opts):
    print(f"[gpu] shape={C.shape} bc={bc} prec={precision} dt={dt} n={nsteps} {opts}",
          flush=True)
    dt_ = torch.float64 if precision == "fp64" else torch.float32
    st = torch.cuda.Stream() if stream else None
    s = ch.State(C.shape, h, Cn, Pe, bc=bc, precision=precision, stream=st, **opts)
    s.set_field(dev(C, dt_))
    s.step(dev(u, dt_), dev(v, dt_), dev(w, dt_), dt, nsteps)
    out = s.get_field().double().cpu().numpy()
    cfg = s.config()
    s.close()
    return out, cfg


def test_32cube_fp64_one_step_and_ten_steps():
    wl = inputs.make_workload(1)
    for n, tol in ((1, TOL64), (10, 1e-11)):
        got, _ = run_gpu(wl.C, wl.u, wl.v, wl.w, wl.h, wl.Cn, wl.Pe, wl.dt, n)
        ref = oracle.step(wl.C, wl.u, wl.v, wl.w, wl.h, wl.Cn, wl.Pe, wl.dt, n)
        print(f"  steps={n} rel Linf={rel(got, ref):.3e} dC rel={rel(got - wl.C, ref - wl.C):.3e}")
        assert rel(got, ref) <= tol
    assert rel(got - wl.C, ref - wl.C) <= 1e-9


@pytest.mark.parametrize("shape,bc,opts", [
    ((20, 12, 16), (0, 0, 0), dict(x_rows=3, seg_len=5, waves_yz=3)),
    ((16, 9, 24), (0, 0, 1), dict(x_rows=5, seg_len=7)),
    ((1, 24, 40), (0, 0, 0), {}),
    ((16, 20, 1), (0, 0, 0), {}),                      # degenerate x: every column is its own halo
    ((16, 20, 1), (0, 0, 0), dict(x_rows=3, z_chunk=3)),
    ((12, 1, 16), (0, 0, 1), {}),                      # degenerate y
    ((48, 48, 48), (0, 0, 0), {}),
    ((40, 33, 72), (0, 0, 1), {}),
    ((96, 96, 96), (0, 0, 0), {}),
    ((96, 96, 96), (0, 0, 0), dict(x_rows=2, z_chunk=5)),
    ((8, 9, 1100), (0, 0, 0), dict(z_chunk=3)),
    # no-flux walls along x and y: wall faces, reflected x halos, the y-wall
    # top face, segments and tiles touching the walls
    ((10, 12, 17), (1, 0, 0), dict(x_rows=3, seg_len=5)),
    ((9, 13, 16), (0, 1, 0), dict(x_rows=2, seg_len=4)),
    ((11, 10, 9), (1, 1, 1), {}),
    ((12, 9, 8), (1, 0, 0), dict(x_rows=4, z_chunk=4)),
    ((10, 9, 1), (1, 1, 0), dict(x_rows=3)),
    ((8, 11, 13), (1, 1, 0), dict(x_rows=5, seg_len=3, waves_yz=2)),
    ((40, 33, 72), (1, 1, 1), {}),
    ((64, 48, 56), (1, 1, 0), dict(x_rows=2, z_chunk=5)),
    # several rows per task, each of whole waves (row offsets uniform per
    # wave): a last task of fewer rows (idle waves), 512-thread groups, walls
    ((12, 9, 128), (0, 0, 0), dict(x_rows=2, z_chunk=5)),
    ((12, 9, 256), (0, 0, 0), dict(x_rows=2, z_chunk=4)),
    ((10, 11, 64), (0, 1, 1), dict(x_rows=3, z_chunk=4)),
    ((9, 10, 128), (1, 1, 0), dict(x_rows=2, z_chunk=3)),
])
def test_fp64_parity_tiles_walls_ragged(shape, bc, opts):
    C, u, v, w, h = _case(shape, bc, seed=sum(shape), amp=2.0)
    dt = 2e-4
    got, cfg = run_gpu(C, u, v, w, h, h, 0.9 / h, dt, 1, bc=bc, **opts)
    ref = oracle.step(C, u, v, w, h, h, 0.9 / h, dt, 1, bc=bc)
    print(f"  cfg={cfg} rel={rel(got, ref):.3e}")
    assert rel(got, ref) <= TOL64
    if bc[0] or bc[1] or shape[2] % 64 == 0 and opts.get("x_rows", 1) > 1:
        # FP32 storage in the same launch shapes
        got32, _ = run_gpu(C, u, v, w, h, h, 0.9 / h, dt, 1, bc=bc, precision="fp32", **opts)
        print(f"  fp32 rel={rel(got32, ref):.3e}")
        assert rel(got32, ref) <= 5e-6


def test_x_program_reported():
    """ch_get_x_program names the x program of the plan (the same arithmetic
    in all of them): general, row, several rows per task, segmented."""
    cases = [((8, 8, 256), {}, 1), ((8, 12, 24), {}, 2), ((8, 8, 1100), {}, 3),
             ((8, 8, 256), dict(x_general=True), 0)]
    for shape, opts, kind in cases:
        C, u, v, w, h = _case(shape, seed=7)
        s = ch.State(shape, h, h, 0.9 / h, stream=torch.cuda.Stream(), **opts)
        with pytest.raises(ch.CHError):
            s.x_program()   # no plan before the first step
        s.set_field(dev(C))
        s.step(dev(u), dev(v), dev(w), 1e-6, 1)
        assert s.x_program() == kind, (shape, opts)
        s.close()


def test_fp64_parity_large_dt_long_warmup():
    C, u, v, w, h = _case((32, 32, 32), seed=3, amp=0.5)
    got, cfg = run_gpu(C, u, v, w, h, h, 0.9 / h, 0.02, 1)
    ref = oracle.step(C, u, v, w, h, h, 0.9 / h, 0.02, 1)
    assert cfg["tw"][0] > 20
    assert rel(got, ref) <= TOL64


def test_fp64_parity_kappa3():
    C, u, v, w, h = _case((24, 24, 24), seed=4)
    got, _ = run_gpu(C, u, v, w, h, h, 0.9 / h, 1e-4, 1, kappa=3.0)
    ref = oracle.step(C, u, v, w, h, h, 0.9 / h, 1e-4, 1, kappa=3.0)
    assert rel(got, ref) <= TOL64


@pytest.mark.parametrize("solve", ["auto", "fp64", "native"])
def test_fp32_against_fp64_oracle(solve):
    C, u, v, w, h = _case((32, 32, 32), seed=5)
    got, cfg = run_gpu(C, u, v, w, h, h, 0.9 / h, 1e-4, 5, precision="fp32", solve=solve)
    ref = oracle.step(C, u, v, w, h, h, 0.9 / h, 1e-4, 5)
    print(f"  fp32 solve={solve} rel={rel(got, ref):.3e} cfg={cfg}")
    assert rel(got, ref) <= 5e-6


def test_graph_replay_matches_direct_launches():
    C, u, v, w, h = _case((32, 24, 40), seed=6)
    a, _ = run_gpu(C, u, v, w, h, h, 0.9 / h, 1e-4, 7, stream=True, use_graph=True)
    b, _ = run_gpu(C, u, v, w, h, h, 0.9 / h, 1e-4, 7, stream=True, use_graph=False)
    c, _ = run_gpu(C, u, v, w, h, h, 0.9 / h, 1e-4, 7, stream=False)
    assert np.array_equal(a, b) and np.array_equal(a, c)
    # replays interleaved with eager work and synchronisation
    st = torch.cuda.Stream()
    s = ch.State(C.shape, h, h, 0.9 / h, stream=st)
    s.set_field(dev(C))
    U, V, W = dev(u), dev(v), dev(w)
    for _ in range(7):
        s.step(U, V, W, 1e-4, 1)
        junk = torch.randn(1000, device="cuda").sum()
        torch.cuda.synchronize()
    assert np.array_equal(s.get_field().cpu().numpy(), a)
    s.close()


def test_mass_conservation_fp64_and_fp32():
    C, u, v, w, h = _case((48, 40, 32), seed=7, amp=3.0)
    for prec, tol in (("fp64", 1e-13), ("fp32", 1e-6)):
        dt_ = torch.float64 if prec == "fp64" else torch.float32
        s = ch.State(C.shape, h, h, 0.9 / h, precision=prec)
        s.set_field(dev(C, dt_))
        m0 = s.mass()
        s.step(dev(u, dt_), dev(v, dt_), dev(w, dt_), 2e-4, 30)
        m1 = s.mass()
        print(f"  {prec} mass drift {abs(m1 - m0) / m0:.3e}")
        assert abs(m1 - m0) <= tol * abs(m0)
        if prec == "fp64":
            assert abs(m0 - oracle.mass(C, h)) <= 1e-14 * abs(m0)
        s.close()


def test_batch_equals_single_boxes_bitwise():
    cases = [_case((32, 32, 32), seed=8), _case((24, 16, 48), seed=9),
             _case((16, 40, 24), seed=10)]
    shapes = [c[0].shape for c in cases]
    hs = [c[4] for c in cases]
    st = torch.cuda.Stream()
    b = ch.Batch(shapes, hs, hs, [0.9 / h for h in hs], stream=st)
    b.set_field(b.pack([c[0] for c in cases], "c"))
    b.step(b.pack([c[1] for c in cases], "u"), b.pack([c[2] for c in cases], "v"),
           b.pack([c[3] for c in cases], "w"), 1e-4, 3)
    outs = [o.cpu().numpy() for o in b.unpack(b.get_field())]
    masses = b.mass()
    b.close()
    for (C, u, v, w, h), got, m in zip(cases, outs, masses):
        single, _ = run_gpu(C, u, v, w, h, h, 0.9 / h, 1e-4, 3)
        assert np.array_equal(got, single)
        ref = oracle.step(C, u, v, w, h, h, 0.9 / h, 1e-4, 3)
        assert rel(got, ref) <= 1e-11
        assert abs(m - oracle.mass(ref, h)) <= 1e-12 * abs(m)


def test_batch_in_two_launches_with_rows_of_whole_waves():
    """A batch whose x pass is two launches: the 256-cell-wide box one row
    per task, the 64- and 128-cell-wide boxes several rows per task whose
    rows are whole waves (row offsets uniform per wave).  Each box equals its
    single-box run bit for bit and the oracle's steps."""
    cases = [_case((16, 12, 256), seed=21), _case((12, 10, 64), bc=(0, 0, 1), seed=22),
             _case((10, 9, 128), seed=23)]
    bcs = [(0, 0, 0), (0, 0, 1), (0, 0, 0)]
    shapes = [c[0].shape for c in cases]
    hs = [c[4] for c in cases]
    for prec, tol in (("fp64", 1e-11), ("fp32", 5e-6)):
        print(f"[gpu] two-launch batch with wave rows, {prec}", flush=True)
        st = torch.cuda.Stream()
        b = ch.Batch(shapes, hs, hs, [0.9 / h for h in hs], bcs=bcs, precision=prec, stream=st)
        b.set_field(b.pack([c[0] for c in cases], "c"))
        b.step(b.pack([c[1] for c in cases], "u"), b.pack([c[2] for c in cases], "v"),
               b.pack([c[3] for c in cases], "w"), 1e-4, 2)
        assert b.x_program() == 4
        outs = [o.double().cpu().numpy() for o in b.unpack(b.get_field())]
        b.close()
        for (C, u, v, w, h), bc, got in zip(cases, bcs, outs):
            single, _ = run_gpu(C, u, v, w, h, h, 0.9 / h, 1e-4, 2, bc=bc, precision=prec)
            assert np.array_equal(got, single)
            ref = oracle.step(C, u, v, w, h, h, 0.9 / h, 1e-4, 2, bc=bc)
            assert rel(got, ref) <= tol


def test_checkpoint_resume_is_bitwise():
    C, u, v, w, h = _case((32, 32, 32), seed=11)
    full, _ = run_gpu(C, u, v, w, h, h, 0.9 / h, 1e-4, 6)
    s = ch.State(C.shape, h, h, 0.9 / h)
    s.set_field(dev(C))
    U, V, W = dev(u), dev(v), dev(w)
    s.step(U, V, W, 1e-4, 4)
    saved = s.get_field().clone()
    s.close()
    s2 = ch.State(C.shape, h, h, 0.9 / h)
    s2.set_field(saved)
    s2.step(U, V, W, 1e-4, 2)
    assert np.array_equal(s2.get_field().cpu().numpy(), full)
    s2.close()


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_host_memory_fields_single_box(prec):
    """C copied in and out through host memory (on_device = 0), from pinned and
    from pageable tensors: the round trip returns C bit for bit, and steps
    from a host copy equal steps from a device copy bit for bit."""
    C, u, v, w, h = _case((12, 10, 36), seed=21)
    dt_ = torch.float64 if prec == "fp64" else torch.float32
    ref, _ = run_gpu(C, u, v, w, h, h, 0.9 / h, 1e-4, 2, precision=prec)
    U, V, W = dev(u, dt_), dev(v, dt_), dev(w, dt_)
    for pinned in (True, False):
        print(f"[gpu] host fields {C.shape} {prec} pinned={pinned}", flush=True)
        hC = torch.from_numpy(C).to(dt_)
        hC = hC.pin_memory() if pinned else hC.contiguous()
        s = ch.State(C.shape, h, h, 0.9 / h, precision=prec, stream=torch.cuda.Stream())
        s.set_field_host(hC)
        assert torch.equal(s.get_field_host(), hC)
        out = torch.empty(C.shape, dtype=dt_)              # pageable
        assert torch.equal(s.get_field_host(out), hC)
        s.step(U, V, W, 1e-4, 2)
        got = s.get_field_host(out).double().numpy()
        s.close()
        assert np.array_equal(got, ref)
    with pytest.raises(ValueError, match="CPU tensor"):
        s = ch.State(C.shape, h, h, 0.9 / h, precision=prec)
        try:
            s.set_field_host(dev(C, dt_))
        finally:
            s.close()


def test_host_memory_fields_batch():
    cases = [_case((16, 16, 16), seed=22), _case((12, 8, 24), seed=23)]
    shapes = [c[0].shape for c in cases]
    hs = [c[4] for c in cases]
    b = ch.Batch(shapes, hs, hs, [0.9 / h for h in hs], stream=torch.cuda.Stream())
    packed = b.pack([c[0] for c in cases], "c")
    U, V, W = (b.pack([c[k] for c in cases], "uvw"[k - 1]) for k in (1, 2, 3))
    print(f"[gpu] host fields batch {shapes}", flush=True)
    b.set_field(packed)
    b.step(U, V, W, 1e-4, 2)
    ref = b.get_field().cpu()
    hC = packed.cpu().pin_memory()
    b.set_field_host(hC)
    assert torch.equal(b.get_field_host(), hC)
    b.step(U, V, W, 1e-4, 2)
    assert torch.equal(b.get_field_host(), ref)
    b.close()


def test_error_paths():
    with pytest.raises(ch.CHError, match="EINVAL"):
        ch.State((4, 16, 16), 0.1, 0.1, 1.0)          # 4 cells on an axis
    with pytest.raises(ch.CHError, match="EINVAL"):
        ch.State((16, 16, 16), 0.1, -1.0, 1.0)        # Cn <= 0
    s = ch.State((16, 16, 16), 1 / 16, 1 / 16, 14.4)
    z = torch.zeros((16, 16, 16), dtype=torch.float64, device="cuda")
    with pytest.raises(ch.CHError, match="EINVAL"):
        s.step(z, z, z, -1e-4)
    with pytest.raises(ch.CHError, match="EINVAL"):
        s.step(z, z, z, float("nan"))
    with pytest.raises(ValueError):
        s.step(z.float(), z, z, 1e-4)                  # wrong dtype, caught on the host
    bad = z.clone()
    bad[3, 4, 5] = float("inf")
    with pytest.raises(ch.CHError, match="ENONFINITE"):
        s.check_velocity(bad, z, z)
    s.check_velocity(z, z, z)
    h = s._h
    s.close()
    assert ch.lib().ch_step(h, z.data_ptr(), z.data_ptr(), z.data_ptr(), 1e-4, 1) == -6
    # a live handle of another kind is rejected like a destroyed one
    L = ch.lib()
    g = ch.Grid(32, 32, 32, 1 / 32)
    zf = np.ascontiguousarray(np.linspace(0.0, 1.0, 9))
    ip = ctypes.c_void_p()
    assert L.ch_interp_create(ctypes.byref(g), 8, 8, 8, zf.ctypes.data_as(ch._PD), ch.CH_FP64,
                              ctypes.byref(ip)) == 0
    pp = ctypes.c_void_p()
    assert L.ch_poisson_create(ctypes.byref(g), 1, ch.CH_FP64, ctypes.byref(pp)) == 0
    bt = ch.Batch([(16, 16, 16)], [1 / 16], [1 / 16], [14.4])
    live = ch.State((16, 16, 16), 1 / 16, 1 / 16, 14.4)
    m = ctypes.c_double()
    for foreign in (ip, pp, bt._h):
        assert L.ch_step(foreign, z.data_ptr(), z.data_ptr(), z.data_ptr(), 1e-4, 1) == -6
        assert L.ch_mass(foreign, ctypes.byref(m)) == -6
        assert "handle" in L.ch_last_error().decode()
    for foreign in (ip, pp, live._h):
        assert L.ch_batch_step(foreign, z.data_ptr(), z.data_ptr(), z.data_ptr(), 1e-4, 1) == -6
    assert L.ch_interp_apply(pp, z.data_ptr(), z.data_ptr(), z.data_ptr(), z.data_ptr(),
                             z.data_ptr(), z.data_ptr()) == -6
    assert L.ch_poisson_solve(ip, z.data_ptr(), z.data_ptr()) == -6
    # destroying through a handle of the wrong kind does nothing; the right
    # kind still works afterwards
    L.ch_destroy(ip)
    L.ch_batch_destroy(pp)
    live.step(z, z, z, 1e-4, 1)
    L.ch_interp_destroy(ip)
    L.ch_poisson_destroy(pp)
    bt.close()
    live.close()
    # a no-flux wall with a non-zero normal velocity is reported
    s = ch.State((16, 16, 16), 1 / 16, 1 / 16, 14.4, bc=(0, 0, 1))
    w = torch.zeros((17, 16, 16), dtype=torch.float64, device="cuda")
    w[0, 2, 2] = 1.0
    with pytest.raises(ch.CHError, match="EINVAL"):
        s.check_velocity(z, z, w)
    s.close()


def test_dt_hint_plans_at_creation_and_steps_alike():
    """ch_opts.dt_hint plans the recurrences and launches at creation; the
    steps are the same bits as those of a state planned at its first step."""
    C, u, v, w, h = _case((24, 20, 28), seed=31)
    dt = 3e-4
    a = ch.State(C.shape, h, h, 0.9 / h, dt_hint=dt)
    assert a.config()["tw"][0] > 0          # planned before any step
    b = ch.State(C.shape, h, h, 0.9 / h)
    for s in (a, b):
        s.set_field(dev(C))
        s.step(dev(u), dev(v), dev(w), dt, 2)
    assert torch.equal(a.get_field(), b.get_field())
    a.close()
    b.close()


def test_256cube_full_size_fp64_one_step_against_oracle():
    """The 256^3 workload in the launch configuration the benchmark times
    (default plan, graph replay on a stream), one step against the oracle."""
    wl = inputs.make_workload(2)
    got, cfg = run_gpu(wl.C, wl.u, wl.v, wl.w, wl.h, wl.Cn, wl.Pe, wl.dt, 1)
    ref = oracle.step(wl.C, wl.u, wl.v, wl.w, wl.h, wl.Cn, wl.Pe, wl.dt, 1)
    print(f"  256^3 cfg={cfg} rel={rel(got, ref):.3e} dC={rel(got - wl.C, ref - wl.C):.3e}")
    assert rel(got, ref) <= TOL64
    # FP32 in the same configuration: close to the oracle
    got32, _ = run_gpu(wl.C, wl.u, wl.v, wl.w, wl.h, wl.Cn, wl.Pe, wl.dt, 1, precision="fp32")
    print(f"  256^3 fp32 rel={rel(got32, ref):.3e}")
    assert rel(got32, ref) <= 5e-6


def test_48box_ensemble_sampled_boxes_against_oracle():
    """The whole 48-box ensemble (about 1.2e8 points) in one batch, in the
    launch configuration the benchmark times: every box conserves its mass,
    and one box of every edge (48 to 192) matches the oracle."""
    E = inputs.ensemble(48)
    shapes = [w.shape for w in E]
    hs = [w.h for w in E]
    pick = []
    for edge in (48, 64, 96, 128, 160, 192):
        pick.append(next(i for i, w in enumerate(E) if w.shape[0] == edge))
    refs = {i: oracle.step(E[i].C, E[i].u, E[i].v, E[i].w, E[i].h, E[i].Cn, E[i].Pe, 1e-4, 1)
            for i in pick}
    for prec, tol in (("fp64", TOL64), ("fp32", 5e-6)):
        print(f"[gpu] ensemble of {len(E)} boxes, {prec}", flush=True)
        st = torch.cuda.Stream()
        b = ch.Batch(shapes, hs, [w.Cn for w in E], [w.Pe for w in E], stream=st,
                     precision=prec)
        b.set_field(b.pack([w.C for w in E], "c"))
        m0 = b.mass()
        b.step(b.pack([w.u for w in E], "u"), b.pack([w.v for w in E], "v"),
               b.pack([w.w for w in E], "w"), 1e-4, 1)
        m1 = b.mass()
        outs = b.unpack(b.get_field())
        b.close()
        drift = max(abs(a - c) / abs(a) for a, c in zip(m0, m1))
        print(f"  max mass drift {drift:.2e}")
        assert drift <= (1e-13 if prec == "fp64" else 1e-6)
        for i in pick:
            e = rel(outs[i].double().cpu().numpy(), refs[i])
            print(f"  box {i} edge {shapes[i][0]}: rel {e:.2e}")
            assert e <= tol


def test_explicit25_against_oracle():
    """The explicit 25-point scheme (no line solves) against the oracle's:
    the 32^3 box, a walled ragged box, FP32, and the 256^3 box at full size."""
    wl = inputs.make_workload(1)
    cases = [(wl.C, wl.u, wl.v, wl.w, wl.h, (0, 0, 0), 1e-4, 2)]
    C, u, v, w, h = _case((16, 9, 24), bc=(0, 0, 1), seed=21)
    cases.append((C, u, v, w, h, (0, 0, 1), 1e-4, 2))
    for C, u, v, w, h, bc, dt, n in cases:
        ref = oracle.step_explicit25(C, u, v, w, h, h, 0.9 / h, dt, n, bc=bc)
        for prec, tol in (("fp64", TOL64 * n), ("fp32", 5e-6)):
            print(f"[gpu] explicit25 shape={C.shape} bc={bc} {prec}", flush=True)
            dt_ = torch.float64 if prec == "fp64" else torch.float32
            s = ch.State(C.shape, h, h, 0.9 / h, bc=bc, precision=prec, stream=torch.cuda.Stream())
            s.set_field(dev(C, dt_))
            s.step_explicit25(dev(u, dt_), dev(v, dt_), dev(w, dt_), dt, n)
            got = s.get_field().double().cpu().numpy()
            s.close()
            print(f"  rel {rel(got, ref):.2e}")
            assert rel(got, ref) <= tol
    wl = inputs.make_workload(2)
    ref = oracle.step_explicit25(wl.C, wl.u, wl.v, wl.w, wl.h, wl.Cn, wl.Pe, 5e-5, 1)
    s = ch.State(wl.shape, wl.h, wl.Cn, wl.Pe, stream=torch.cuda.Stream())
    s.set_field(dev(wl.C))
    s.step_explicit25(dev(wl.u), dev(wl.v), dev(wl.w), 5e-5, 1)
    got = s.get_field().cpu().numpy()
    s.close()
    print(f"  256^3 explicit25 rel {rel(got, ref):.2e}")
    assert rel(got, ref) <= TOL64


def test_explicit_and_implicit_steps_interleave():
    """Explicit steps trade the state's buffers; implicit steps after them
    (captured and replayed as graphs) must still use the right ones."""
    C, u, v, w, h = _case((24, 16, 32), seed=22)
    Pe, dt = 0.9 / h, 1e-4
    ref = oracle.step(C, u, v, w, h, h, Pe, dt, 2)
    ref = oracle.step_explicit25(ref, u, v, w, h, h, Pe, dt, 1)
    ref = oracle.step(ref, u, v, w, h, h, Pe, dt, 2)
    st = torch.cuda.Stream()
    s = ch.State(C.shape, h, h, Pe, stream=st)
    s.set_field(dev(C))
    U, V, W = dev(u), dev(v), dev(w)
    s.step(U, V, W, dt, 2)
    s.step_explicit25(U, V, W, dt, 1)
    s.step(U, V, W, dt, 2)
    got = s.get_field().cpu().numpy()
    s.close()
    assert rel(got, ref) <= 5 * TOL64


@pytest.mark.parametrize("axis", [0, 2])
@pytest.mark.parametrize("kappa", [4.0, 3.0])
def test_flat_interface_equilibrium_stays_on_the_gpu(axis, kappa):
    """The scheme's discrete flat-interface equilibrium (a slab, Newton-solved
    on one periodic line) extruded along the other two axes, u = 0: 20 steps
    at dt = 1e-3 leave it in place to 1e-12 (FP64); FP32 storage keeps it to
    within its own rounding (1e-6)."""
    from tests.test_oracle_pins import _flat_equilibrium
    n = 64
    h = 1.0 / n
    prof = _flat_equilibrium(n, h, h, kappa)
    shape = (n, 16, 24) if axis == 0 else (16, 24, n)
    C = np.broadcast_to(prof[:, None, None] if axis == 0 else prof[None, None, :],
                        shape).copy()
    zero = np.zeros_like(C)
    for prec, tol in (("fp64", 1e-12), ("fp32", 1e-6)):
        print(f"[gpu] flat interface along axis {axis}, kappa {kappa}, {prec}", flush=True)
        got, _ = run_gpu(C, zero, zero, zero, h, h, 0.9 / h, 1e-3, 20, precision=prec,
                         kappa=kappa)
        ref = C if prec == "fp64" else C.astype(np.float32).astype(np.float64)
        d = float(np.abs(got - ref).max())
        print(f"  max |dC| {d:.2e}")
        assert d <= tol


def test_autotune_restores_c_and_the_tuned_plan_matches_the_oracle():
    # 136 rows in y: the segment candidates 128 and 64 split the y lines
    # (with ragged last segments), so the tuned plan may be a segmented one
    C, u, v, w, h = _case((32, 136, 48), seed=21)
    st = torch.cuda.Stream()
    s = ch.State(C.shape, h, h, 0.9 / h, stream=st)
    s.set_field(dev(C))
    U, V, W = dev(u), dev(v), dev(w)
    print("[gpu] autotune (32, 136, 48)", flush=True)
    t = s.autotune(U, V, W, 1e-4, steps=2)
    print(f"  {t}")
    assert t["candidates"] >= 2 and 0.0 < t["ms_per_step"] <= t["auto_ms_per_step"]
    assert np.array_equal(s.get_field().cpu().numpy(), C)
    cfg = s.config()
    assert (cfg["x_rows"], cfg["z_chunk"], cfg["seg"]) == (t["x_rows"], t["z_chunk"], t["seg_len"])
    s.step(U, V, W, 1e-4, 3)
    got = s.get_field().cpu().numpy()
    s.close()
    ref = oracle.step(C, u, v, w, h, h, 0.9 / h, 1e-4, 3)
    assert rel(got, ref) <= 3e-12
    same, _ = run_gpu(C, u, v, w, h, h, 0.9 / h, 1e-4, 3, x_rows=t["x_rows"],
                      z_chunk=t["z_chunk"], seg_len=t["seg_len"])
    assert np.array_equal(got, same)


def test_batch_autotune_restores_c_and_steps_like_the_oracle():
    cases = [_case((32, 32, 32), seed=22), _case((24, 16, 48), seed=23)]
    shapes = [c[0].shape for c in cases]
    hs = [c[4] for c in cases]
    st = torch.cuda.Stream()
    b = ch.Batch(shapes, hs, hs, [0.9 / h for h in hs], stream=st)
    C0 = b.pack([c[0] for c in cases], "c")
    b.set_field(C0)
    U, V, W = (b.pack([c[i] for c in cases], f) for i, f in ((1, "u"), (2, "v"), (3, "w")))
    print("[gpu] batch autotune", flush=True)
    t = b.autotune(U, V, W, 1e-4, steps=2)
    print(f"  {t}")
    assert torch.equal(b.get_field(), C0)
    b.step(U, V, W, 1e-4, 2)
    outs = [o.cpu().numpy() for o in b.unpack(b.get_field())]
    b.close()
    for (C, u, v, w, h), got in zip(cases, outs):
        assert rel(got, oracle.step(C, u, v, w, h, h, 0.9 / h, 1e-4, 2)) <= 2e-12
