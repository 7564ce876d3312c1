"""Sampled parity at sizes the whole-box oracle cannot take: the oracle steps
a periodic window cut around a sample point, and its central cells are
compared with the full result there.

Why the centre is right: within one substage the explicit terms reach 3
cells, and each directional line-solve factor has an inverse whose taps
decay geometrically, by |z| per cell (the root of the factorised symbol;
|z| < 0.35 at the workloads' parameters).  The wrong values that periodic
wrapping puts at the window's faces therefore reach the centre, a margin of
m cells away, only at relative size ~ |z|^(m - 9) after the three substages.
`tests/test_windowed_oracle.py` checks this against the whole-box oracle.
"""
import numpy as np

import oracle


def window_index(shape, lo, W):
    return [(lo[d] + np.arange(W)) % shape[d] for d in range(3)]


def periodic_window(a, lo, W):
    """Window of W^3 cells (or faces) starting at lo = (z0, y0, x0), wrapped."""
    iz, iy, ix = window_index(a.shape, lo, W)
    if hasattr(a, "cpu"):            # a device tensor: gather there, copy the window
        import torch
        dev = a.device
        t = a[torch.as_tensor(iz, device=dev)[:, None, None],
              torch.as_tensor(iy, device=dev)[None, :, None],
              torch.as_tensor(ix, device=dev)[None, None, :]]
        return np.ascontiguousarray(t.double().cpu().numpy())
    return np.ascontiguousarray(np.asarray(a, dtype=np.float64)[np.ix_(iz, iy, ix)])


def window_step(C, u, v, w, lo, W, h, Cn, Pe, dt, nsteps=1):
    """The oracle's step on the periodic window (fields of a periodic box)."""
    return oracle.step(*(periodic_window(x, lo, W) for x in (C, u, v, w)), h, Cn, Pe, dt,
                       nsteps)
