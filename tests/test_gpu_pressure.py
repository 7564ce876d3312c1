"""GPU parity of the split-density pressure step (sec. 3.2: eq-split,
eq-newpoi, eq-u) and its fast Poisson solve against the numpy oracle,
through the C ABI.

Bars: FP64 1e-12 of the largest value of each field (transforms and a
tridiagonal or spectral solve in another order than the oracle's dense
solves; measured about 1e-15); FP32 1e-5 for the solve and 5e-6 for the
whole step (single-precision transforms, measured up to 2e-6 and 4e-7);
the pressure history (Pold <- P^l) is copied exactly."""
import numpy as np
import pytest
import torch

from oracle import pressure as pr

pytestmark = pytest.mark.gpu


def dev(a, dt_=torch.float64):
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda", dt_)


def relmax(a, b):
    return float(np.abs(a - b).max() / max(np.abs(b).max(), 1e-300))


def _inputs(shape, zwalls, seed):
    rng = np.random.default_rng(seed)
    nz, ny, nx = shape
    C = rng.uniform(-0.1, 1.1, shape)
    u = rng.standard_normal(shape)
    v = rng.standard_normal(shape)
    w = rng.standard_normal((nz + 1, ny, nx) if zwalls else shape)
    if zwalls:
        w[0] = w[-1] = 0.0
    return C, u, v, w, rng.standard_normal(shape), rng.standard_normal(shape)


@pytest.mark.parametrize("shape", [(8, 12, 10), (9, 8, 16), (12, 6, 8), (32, 64, 48),
                                   (10, 7, 15),    # odd y and x extents
                                   (2, 8, 8), (3, 6, 10)])   # one row each side of the middle
@pytest.mark.parametrize("zwalls", [False, True])
def test_poisson_solve_matches_oracle(shape, zwalls):
    from paper_2105_01865_amd import ch
    rng = np.random.default_rng(61)
    h = 1.0 / shape[2]
    rhs = rng.standard_normal(shape)
    ref = pr.poisson(rhs, h, zwalls)
    for prec, dt_, tol in (("fp64", torch.float64, 1e-12), ("fp32", torch.float32, 1e-5)):
        print(f"[gpu] poisson {shape} walls={zwalls} {prec}", flush=True)
        st = torch.cuda.Stream()
        p = ch.Poisson(shape, h, z_walls=zwalls, precision=prec, stream=st)
        got = p.solve(dev(rhs, dt_)).double().cpu().numpy()
        p.close()
        e = relmax(got, ref)
        print(f"  rel {e:.2e}")
        assert e <= tol


@pytest.mark.parametrize("shape", [(8, 12, 10), (16, 16, 16), (9, 10, 24), (11, 9, 13)])
@pytest.mark.parametrize("zwalls", [False, True])
def test_pressure_step_matches_oracle(shape, zwalls):
    from paper_2105_01865_amd import ch
    h = 1.0 / shape[2]
    C, u, v, w, P, Pold = _inputs(shape, zwalls, 62)
    rho1, rho2, dt = 1000.0, 1.0, 1e-3
    ref = pr.pressure_step(C, u, v, w, P, Pold, h, dt, rho1, rho2, zwalls)
    for prec, dt_, tol in (("fp64", torch.float64, 1e-12), ("fp32", torch.float32, 5e-6)):
        print(f"[gpu] pressure step {shape} walls={zwalls} {prec}", flush=True)
        st = torch.cuda.Stream()
        p = ch.Poisson(shape, h, z_walls=zwalls, precision=prec, stream=st)
        T = [dev(a, dt_) for a in (C, u, v, w, P, Pold)]
        Pin = T[4].clone()
        p.step(*T, rho1, rho2, dt)
        torch.cuda.synchronize()
        p.close()
        got = [t.double().cpu().numpy() for t in T[1:]]
        for name, g, r in zip(("u", "v", "w", "P"), got[:4], ref[:4]):
            e = relmax(g, r)
            print(f"  {name}: rel {e:.2e}")
            assert e <= tol
        assert torch.equal(T[5], Pin)
        if zwalls:
            assert np.all(got[2][0] == 0.0) and np.all(got[2][-1] == 0.0)


def test_divergence_free_at_128_cubed_with_a_density_ratio_of_1000():
    from paper_2105_01865_amd import ch
    n = 128
    h = 1.0 / n
    C, u, v, w, P, Pold = _inputs((n, n, n), True, 63)
    print(f"[gpu] pressure step {n}^3 walls, rho1/rho2 = 1000", flush=True)
    st = torch.cuda.Stream()
    p = ch.Poisson((n, n, n), h, z_walls=True, stream=st)
    T = [dev(a) for a in (C, u, v, w, P, Pold)]
    p.step(*T, 1000.0, 1.0, 1e-3)
    torch.cuda.synchronize()
    p.close()
    un, vn, wn = (t.cpu().numpy() for t in T[1:4])
    d0 = ((np.roll(u, -1, 2) - u + np.roll(v, -1, 1) - v) + (w[1:] - w[:-1])) / h
    d1 = ((np.roll(un, -1, 2) - un + np.roll(vn, -1, 1) - vn) + (wn[1:] - wn[:-1])) / h
    print(f"  max |div| before {np.abs(d0).max():.2e}, after {np.abs(d1).max():.2e}")
    assert np.abs(d1).max() <= 1e-10 * np.abs(d0).max()
