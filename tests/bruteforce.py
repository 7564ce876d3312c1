"""Independent dense numpy implementation of one CH step, for tiny grids.

Used only to pin the C oracle.  It is written separately from the oracle:
ghosts come from numpy's ``wrap``/``symmetric`` padding, the advection is
vectorised over whole arrays, and the approximately factorised implicit
operator is formed as a dense Kronecker product
(I + r Az) (x) (I + r Ay) (x) (I + r Ax) and solved in one dense solve, with
the 1-D matrices built as a circulant (periodic) or as the square of the
Neumann second-difference matrix (no-flux).
"""
import numpy as np


def _pad(C, bc, g):
    modes = ["wrap" if b == 0 else "symmetric" for b in bc]   # (x, y, z)
    out = C
    for axis, mode in zip((2, 1, 0), modes):
        pw = [(0, 0)] * 3
        pw[axis] = (g, g)
        out = np.pad(out, pw, mode=mode)
    return out


def _weno(a, b, c, d, e, eps):
    q0 = (2 * a - 7 * b + 11 * c) / 6
    q1 = (-b + 5 * c + 2 * d) / 6
    q2 = (2 * c + 5 * d - e) / 6
    s0 = 13 / 12 * (a - 2 * b + c) ** 2 + 0.25 * (a - 4 * b + 3 * c) ** 2
    s1 = 13 / 12 * (b - 2 * c + d) ** 2 + 0.25 * (b - d) ** 2
    s2 = 13 / 12 * (c - 2 * d + e) ** 2 + 0.25 * (3 * c - 4 * d + e) ** 2
    w0 = 0.1 / (eps + s0) ** 2
    w1 = 0.6 / (eps + s1) ** 2
    w2 = 0.3 / (eps + s2) ** 2
    return (w0 * q0 + w1 * q1 + w2 * q2) / (w0 + w1 + w2)


def _take(P, axis, start, n):
    sl = [slice(3, -3)] * 3
    sl[axis] = slice(start, start + n)
    return P[tuple(sl)]


def advection(C, vel, h, bc, eps=1e-6):
    P = _pad(C, bc, 3)
    out = np.zeros_like(C)
    for d, axis in ((0, 2), (1, 1), (2, 0)):
        n = C.shape[axis]
        U = vel[d]
        if bc[d] == 0:   # periodic: append face 0 as face n
            U = np.concatenate([U, np.take(U, [0], axis=axis)], axis=axis)
        nf = n + 1
        # face f between cells f-1 and f; cell m sits at padded index m + 3
        L = [_take(P, axis, s, nf) for s in range(0, 5)]            # cells f-3 .. f+1
        R = [_take(P, axis, s, nf) for s in range(5, 0, -1)]        # cells f+2 .. f-2
        Cf = np.where(U >= 0, _weno(*L, eps), _weno(*R, eps))
        F = U * Cf
        hi = [slice(None)] * 3
        lo = [slice(None)] * 3
        hi[axis] = slice(1, None)
        lo[axis] = slice(0, -1)
        out += (F[tuple(hi)] - F[tuple(lo)]) / h
    return out


def _shift(P, axis, m, g, shape):
    sl = [slice(g, g + s) for s in shape]
    sl[axis] = slice(g + m, g + m + shape[axis])
    return P[tuple(sl)]


def lap_mu(C, h, bc, psi):
    P = _pad(C, bc, 1)
    mu = psi[0] + psi[1] * P + psi[2] * P ** 2 + psi[3] * P ** 3
    out = np.zeros_like(C)
    for axis in range(3):
        out += (_shift(mu, axis, 1, 1, C.shape) - 2 * _shift(mu, axis, 0, 1, C.shape)
                + _shift(mu, axis, -1, 1, C.shape)) / h ** 2
    return out


def biharm(C, h, Cn, kappa, bc):
    P = _pad(C, bc, 2)
    out = np.zeros_like(C)
    for axis in range(3):
        s = lambda m: _shift(P, axis, m, 2, C.shape)
        out += s(-2) - 4 * s(-1) + 6 * s(0) - 4 * s(1) + s(2)
    return kappa * Cn ** 2 / h ** 4 * out


def d4_matrix(n, bc):
    """Dense (1,-4,6,-4,1) operator: circulant when periodic, the square of
    the Neumann second difference when no-flux."""
    if bc == 0:
        col = np.zeros(n)
        for m, c in zip(range(-2, 3), (1, -4, 6, -4, 1)):
            col[m % n] += c
        return np.array([[col[(i - j) % n] for j in range(n)] for i in range(n)])
    D2 = np.zeros((n, n))
    for i in range(n):
        D2[i, i] = -2.0
        if i > 0:
            D2[i, i - 1] = 1.0
        if i < n - 1:
            D2[i, i + 1] = 1.0
    D2[0, 0] += 1.0
    D2[n - 1, n - 1] += 1.0
    return D2 @ D2


GAMMA = (8 / 15, 5 / 12, 3 / 4)
RHO = (0.0, -17 / 60, -5 / 12)


def step(C, u, v, w, h, Cn, Pe, dt, nsteps=1, bc=(0, 0, 0), kappa=4.0,
         psi=(0.0, 0.5, -1.5, 1.0), eps=1e-6):
    C = np.array(C, dtype=np.float64)
    nz, ny, nx = C.shape
    Eold = np.zeros_like(C)
    for _ in range(nsteps):
        for k in range(3):
            alpha = GAMMA[k] + RHO[k]
            E = -advection(C, (u, v, w), h, bc, eps) + lap_mu(C, h, bc, psi) / Pe
            B = biharm(C, h, Cn, kappa, bc)
            rhs = dt * (GAMMA[k] * E + RHO[k] * Eold) - alpha * dt * B / Pe
            r = alpha * dt * kappa * Cn ** 2 / (2 * Pe * h ** 4)
            Mx = np.eye(nx) + r * d4_matrix(nx, bc[0])
            My = np.eye(ny) + r * d4_matrix(ny, bc[1])
            Mz = np.eye(nz) + r * d4_matrix(nz, bc[2])
            M = np.kron(Mz, np.kron(My, Mx))
            C = C + np.linalg.solve(M, rhs.ravel()).reshape(C.shape)
            Eold = E
    return C
