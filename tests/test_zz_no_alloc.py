"""The allocation-free mass (ch_mass_field_noalloc) against ch_mass, through
the C ABI: the same fixed-order FP64 sum, so the same bits, on two calls in a
row (the second with a smaller field, which reuses the library's scratch
array), in both precisions."""
import ctypes

import numpy as np
import pytest
import torch

from paper_2105_01865_amd import ch, inputs

pytestmark = pytest.mark.gpu


def _field(shape, seed, dtype):
    rng = np.random.default_rng(seed)
    h = 1.0 / max(shape)
    cen, rad = inputs.place_drops(rng, 3, 2, 5, shape, h, gap_cells=1)
    C = inputs.drop_field(shape, h, h, cen, rad) + 0.01 * rng.normal(size=shape)
    return torch.from_numpy(C).to("cuda", dtype), h


def _ch_mass(C, h, prec):
    s = ch.State(tuple(C.shape), h, h, 0.9 / h, precision=prec)
    s.set_field(C)
    m = s.mass()
    s.close()
    return m


@pytest.mark.parametrize("prec,dtype", [("fp64", torch.float64), ("fp32", torch.float32)])
def test_noalloc_mass_matches_ch_mass_on_two_calls(prec, dtype):
    L = ch.lib()
    stream = torch.cuda.Stream()
    out = torch.full((2,), float("nan"), dtype=torch.float64, device="cuda")
    # two calls in a row: a field spanning many blocks, then a smaller ragged one
    for k, shape in enumerate([(96, 80, 112), (17, 23, 31)]):
        C, h = _field(shape, 40 + k, dtype)
        torch.cuda.synchronize()
        print(f"[gpu] noalloc mass {prec} shape={shape}", flush=True)
        nz, ny, nx = shape
        pc = ch.CH_FP64 if prec == "fp64" else ch.CH_FP32
        st = L.ch_mass_field_noalloc(ctypes.c_void_p(C.data_ptr()), nx, ny, nz, h, pc,
                                     ctypes.c_void_p(stream.cuda_stream),
                                     ctypes.c_void_p(out.data_ptr() + 8 * k))
        assert st == 0, L.ch_last_error().decode()
        stream.synchronize()
        got = float(out[k].item())
        ref = _ch_mass(C, h, prec)
        print(f"  noalloc {got!r} ch_mass {ref!r}", flush=True)
        assert got == ref
    # the binding's wrapper gives the same value
    m = torch.zeros(1, dtype=torch.float64, device="cuda")
    ch.mass_field_noalloc(C, h, m, stream=stream)
    stream.synchronize()
    assert float(m.item()) == ref


def test_noalloc_mass_rejects_bad_arguments():
    L = ch.lib()
    x = torch.zeros(8, dtype=torch.float64, device="cuda")
    p = ctypes.c_void_p(x.data_ptr())
    assert L.ch_mass_field_noalloc(p, 0, 2, 2, 0.1, ch.CH_FP64, None, p) == -1
    assert L.ch_mass_field_noalloc(p, 2, 2, 2, -0.1, ch.CH_FP64, None, p) == -1
    assert L.ch_mass_field_noalloc(p, 2, 2, 2, 0.1, 9, None, p) == -1
    assert L.ch_mass_field_noalloc(None, 2, 2, 2, 0.1, ch.CH_FP64, None, p) == -1
    # more cells than the scratch array's partial sums cover
    assert L.ch_mass_field_noalloc(p, 2048, 2048, 1025, 0.1, ch.CH_FP32, None, p) == -1
    assert "limit" in L.ch_last_error().decode()
