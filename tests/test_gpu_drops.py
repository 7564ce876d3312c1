"""GPU drop labelling (the drop-size diagnostics of sec. 4) against the
oracle's flood fill, through the C ABI.

Bar: labels decide integers, so the (root, cells) lists must be equal
exactly; both sides compare C with the threshold in the state's precision
(the FP32 field is handed to the oracle converted exactly to FP64)."""
import numpy as np
import pytest
import torch

import oracle
from paper_2105_01865_amd import ch, inputs

pytestmark = pytest.mark.gpu


def _state(C, bc=(0, 0, 0), precision="fp64"):
    dt_ = torch.float64 if precision == "fp64" else torch.float32
    nz, ny, nx = C.shape
    h = 1.0 / nx
    st = torch.cuda.Stream()
    s = ch.State(C.shape, h, h, 0.9 / h, bc=bc, precision=precision, stream=st)
    s.set_field(torch.from_numpy(np.ascontiguousarray(C)).to("cuda", dt_))
    return s


def _oracle_list(C, bc, thr=0.5):
    lab, nd = oracle.label_drops(C, thr, bc=bc)
    roots, cells, _, _ = oracle.drop_volumes(lab, 1.0)
    assert len(roots) == nd
    return roots, cells


@pytest.mark.parametrize("shape,p,bc", [((8, 8, 8), 0.3, (0, 0, 0)),
                                        ((12, 9, 20), 0.25, (0, 0, 1)),
                                        ((10, 16, 8), 0.35, (1, 0, 1)),
                                        ((16, 16, 16), 0.6, (0, 0, 0)),     # one giant drop
                                        ((33, 17, 65), 0.3, (0, 1, 0))])
def test_random_fields_match_oracle(shape, p, bc):
    rng = np.random.default_rng(41)
    C = rng.random(shape) * (rng.random(shape) < p) + 0.49 * (rng.random(shape) < 0.1)
    for prec in ("fp64", "fp32"):
        print(f"[gpu] drops random {shape} p={p} bc={bc} {prec}", flush=True)
        Cp = C if prec == "fp64" else C.astype(np.float32).astype(np.float64)
        s = _state(Cp, bc, prec)
        roots, cells = s.drops(0.5, cap=8)   # also grows the host arrays
        s.close()
        r_ref, c_ref = _oracle_list(Cp, bc)
        print(f"  {len(roots)} drops, largest {cells.max() if len(cells) else 0}")
        assert np.array_equal(roots, r_ref) and np.array_equal(cells, c_ref)


def test_edge_fields():
    shape = (8, 10, 12)
    for C, expect in ((np.zeros(shape), 0), (np.ones(shape), 1), (np.full(shape, 0.5), 1),
                      (np.full(shape, 0.5 - 1e-9), 0)):
        s = _state(C)
        roots, cells = s.drops(0.5)
        s.close()
        assert len(roots) == expect
        if expect:
            assert roots[0] == 0 and cells[0] == C.size


def test_workload_field_at_full_size_matches_oracle():
    """The 256^3 bench field (64 drops) and the same field after 20 FP32 and
    FP64 steps."""
    wl = inputs.make_workload(2)
    print(f"[gpu] drops on the {wl.shape} workload", flush=True)
    s = _state(wl.C)
    roots, cells = s.drops()
    r_ref, c_ref = _oracle_list(wl.C, (0, 0, 0))
    assert np.array_equal(roots, r_ref) and np.array_equal(cells, c_ref)
    print(f"  initial: {len(roots)} drops")
    U, V, W = (torch.from_numpy(a).to("cuda") for a in (wl.u, wl.v, wl.w))
    s.step(U, V, W, wl.dt, 20)
    C64 = s.get_field().cpu().numpy()
    roots, cells = s.drops()
    s.close()
    r_ref, c_ref = _oracle_list(C64, (0, 0, 0))
    assert np.array_equal(roots, r_ref) and np.array_equal(cells, c_ref)
    print(f"  after 20 FP64 steps: {len(roots)} drops")


def test_batch_boxes_match_oracle():
    rng = np.random.default_rng(43)
    shapes = [(16, 24, 8), (12, 12, 40)]
    fields = [rng.random(sh) * (rng.random(sh) < 0.3) for sh in shapes]
    hs = [1.0 / sh[2] for sh in shapes]
    st = torch.cuda.Stream()
    b = ch.Batch(shapes, hs, hs, [0.9 / h for h in hs], bcs=[(0, 0, 0), (0, 0, 1)], stream=st)
    b.set_field(b.pack([torch.from_numpy(f).cuda() for f in fields], "c"))
    for k, (f, bc) in enumerate(zip(fields, [(0, 0, 0), (0, 0, 1)])):
        roots, cells = b.drops(k)
        r_ref, c_ref = _oracle_list(f, bc)
        assert np.array_equal(roots, r_ref) and np.array_equal(cells, c_ref)
    b.close()
