"""GPU parity of the multiple-resolution path (sec. 3.4) against the oracle:
the coarse stretched-z velocity transferred to the fine faces, and whole
steps that transfer the velocity before every step (the config-3 path).

Bars: the transfer is a fixed linear combination of coarse values, so FP64
agrees with the oracle to a few ulp of the largest velocity (1e-13 relative
L-infinity); FP32 weights and sums leave <= 2e-6.  Steps: 1e-12 relative per
step in FP64, as for the uniform-velocity path.
"""
import numpy as np
import pytest
import torch

import oracle
from paper_2105_01865_amd import ch, inputs

pytestmark = pytest.mark.gpu


def dev(a, dtype=torch.float64):
    return torch.from_numpy(np.ascontiguousarray(a)).to(device="cuda", dtype=dtype)


def rel(a, b):
    return float(np.abs(a - b).max() / max(np.abs(b).max(), 1e-300))


def _coarse(seed, nc, alpha=2.0):
    ncz, ncy, ncx = nc
    rng = np.random.default_rng(seed)
    zf = inputs.stretched_faces(ncz, alpha)
    uc, vc, wc = inputs.coarse_wall_velocity(rng, nc, zf, kmax=max(1, min(6, ncx // 3)),
                                             nmodes_z=min(8, ncz))
    return zf, uc, vc, wc


@pytest.mark.parametrize("fine,nc", [((32, 32, 32), (12, 16, 16)),       # config 3, shrunk
                                     ((36, 40, 48), (10, 16, 20)),       # uneven ratios
                                     ((24, 24, 24), (24, 24, 24))])      # same counts
def test_transfer_matches_oracle(fine, nc):
    nz, ny, nx = fine
    zf, uc, vc, wc = _coarse(7, nc)
    ref = oracle.interp_velocity(zf, uc, vc, wc, (nx, ny, nz))
    for prec, dt_, tol in (("fp64", torch.float64, 1e-13), ("fp32", torch.float32, 2e-6)):
        print(f"[gpu] transfer fine={fine} coarse={nc} {prec}", flush=True)
        st = torch.cuda.Stream()
        ip = ch.Interp(fine, 1.0 / nx, nc, zf, precision=prec, stream=st)
        got = ip.apply(dev(uc, dt_), dev(vc, dt_), dev(wc, dt_))
        torch.cuda.synchronize()
        for name, g, r in zip("uvw", got, ref):
            e = rel(g.double().cpu().numpy(), r)
            print(f"  {name}: rel {e:.2e}")
            assert e <= tol
        # the wall faces carry exactly zero normal velocity
        w = got[2].double().cpu().numpy()
        assert np.all(w[0] == 0.0) and np.all(w[-1] == 0.0)
        ip.close()


def test_multires_steps_match_oracle():
    """Config 3 shrunk to a 32^3 fine mesh (walls in z, 16 x 16 x 12 coarse
    velocity): three steps, each transferring the velocity first."""
    wl = inputs.make_workload(3, n=32)
    nz, ny, nx = wl.shape
    zf, uc, vc, wc = (wl.coarse[k] for k in ("zf", "uc", "vc", "wc"))
    nsteps = 3
    uf, vf, wf = oracle.interp_velocity(zf, uc, vc, wc, (nx, ny, nz))
    ref = oracle.step(wl.C, uf, vf, wf, wl.h, wl.Cn, wl.Pe, wl.dt, nsteps, bc=wl.bc)
    print(f"[gpu] multires {wl.shape} bc={wl.bc} dt={wl.dt} n={nsteps}", flush=True)
    st = torch.cuda.Stream()
    s = ch.State(wl.shape, wl.h, wl.Cn, wl.Pe, bc=wl.bc, stream=st)
    ip = ch.Interp(wl.shape, wl.h, uc.shape, zf, precision="fp64", stream=st)
    s.set_field(dev(wl.C))
    s.step_multires(ip, dev(uc), dev(vc), dev(wc), wl.dt, nsteps)
    got = s.get_field().cpu().numpy()
    m = s.mass()
    s.close()
    ip.close()
    e = rel(got, ref)
    print(f"  rel {e:.3e}, mass rel {abs(m - oracle.mass(ref, wl.h)) / abs(m):.2e}")
    assert e <= 1e-12 * nsteps
    assert abs(m - oracle.mass(wl.C, wl.h)) / abs(m) <= 1e-13
