"""The 1536^3 periodic box in single precision (3.6e9 points, one GPU's share
at the paper's scale) at full size, in the library's default plan: one step,
then sampled parity against the oracle on periodic windows (tests/windowed.py)
and mass conservation of the whole box.

Bars: single-precision storage and stencils, 5e-6 relative L-infinity
against the FP64 oracle on the window centres (the bar of the smaller FP32
parity tests); the FP64 mass sum of the FP32 field drifts by <= 1e-6.
"""
import numpy as np
import pytest
import torch

from paper_2105_01865_amd import ch, inputs_gpu
from tests.windowed import periodic_window, window_step

pytestmark = pytest.mark.gpu

W, C0, CW = 64, 24, 16     # window, offset and size of the compared centre


def test_large_box_fp32_one_step_sampled_windows():
    print("[gpu] generating the 1536^3 workload on the device", flush=True)
    wl = inputs_gpu.large_workload()
    n = wl.shape[0]
    # windows centred on drop interfaces: the first drop, the drop nearest the
    # periodic corner (its window wraps), and a seeded random drop
    rng = np.random.default_rng(1536)
    corner = np.minimum(wl.centres, 1.0 - wl.centres)
    picks = [0, int(np.argmin((corner ** 2).sum(axis=1))), int(rng.integers(len(wl.radii)))]
    los = []
    for i in picks:
        c, R = wl.centres[i], wl.radii[i]
        p = (c[2], c[1], c[0] + R)          # a point of the interface, (z, y, x)
        los.append(tuple((int(q / wl.h) - C0 - CW // 2) % n for q in p))
    refs = []
    for lo in los:
        sub = window_step(wl.C, wl.u, wl.v, wl.w, lo, W, wl.h, wl.Cn, wl.Pe, wl.dt, 1)
        refs.append(sub[C0:C0 + CW, C0:C0 + CW, C0:C0 + CW])
    print(f"[gpu] 1536^3 fp32 one step, dt={wl.dt:.3e}, {len(wl.radii)} drops", flush=True)
    st = torch.cuda.Stream()
    s = ch.State(wl.shape, wl.h, wl.Cn, wl.Pe, precision="fp32", stream=st)
    s.set_field(wl.C)
    m0 = s.mass()
    s.step(wl.u, wl.v, wl.w, wl.dt, 1)
    m1 = s.mass()
    cfg = s.config()
    got = s.get_field()
    s.close()
    print(f"  plan {cfg}; mass drift {abs(m1 - m0) / abs(m0):.2e}")
    assert abs(m1 - m0) <= 1e-6 * abs(m0)
    for lo, ref in zip(los, refs):
        g = periodic_window(got, tuple((l + C0) % n for l in lo), CW)
        e = float(np.abs(g - ref).max() / np.abs(ref).max())
        print(f"  window at {lo}: max |C| {np.abs(ref).max():.3f}, rel {e:.2e}")
        assert e <= 5e-6
