"""Plain FP64 oracle of the split-density pressure step (sec. 3.2: eq-poi,
eq-split, eq-newpoi, eq-u) on the uniform staggered mesh of the CH path.

TEST INFRASTRUCTURE.  Only the test-suite, the smoke check and the
CPU-baseline leg of the benchmark import it; it shares no code with the GPU
library.  numpy's FFT and dense linear solve serve as library steps.

Mesh: cells [nz][ny][nx] of width h (x fastest), P and C at cell centres,
u on x faces, v on y faces (face i is the low face of cell i), w on z faces:
nz faces when z is periodic, nz + 1 between walls (zero on both walls).
x and y are periodic.

Readings where the paper is silent (listed in the design notes):
  - rho = rho2 + (rho1 - rho2) min(max(C, 0), 1): linear in C, with C
    clipped to the two pure phases so rho stays in [rho2, rho1];
  - rho on a face is the mean of the two cells it separates;
  - gradients on faces (P_i - P_{i-1}) / h, divergence at cells
    (F_{i+1} - F_i) / h, no flux through walls (dP/dz = 0 there);
  - the constant-coefficient Poisson problem lap P = rhs is solved with the
    7-point Laplacian of those operators; P has zero mean (rhs has zero mean
    as the divergence of face fluxes; its mean is removed first).
"""
import numpy as np


def density(C, rho1, rho2):
    """rho from C, linear between the pure phases (C clipped to [0, 1])."""
    return rho2 + (rho1 - rho2) * np.clip(C, 0.0, 1.0)


def face_mean(a, axis, walls):
    """Mean of the two cells on each face along `axis` (face i between cells
    i-1 and i); between walls the wall faces (0 and n) carry a copy of the
    adjacent cell (they see no flux)."""
    if not walls:
        return 0.5 * (a + np.roll(a, 1, axis=axis))
    lo = np.take(a, [0], axis=axis)
    hi = np.take(a, [a.shape[axis] - 1], axis=axis)
    inner = 0.5 * (np.take(a, range(1, a.shape[axis]), axis=axis)
                   + np.take(a, range(0, a.shape[axis] - 1), axis=axis))
    return np.concatenate([lo, inner, hi], axis=axis)


def grad(P, axis, h, walls):
    """(P_i - P_{i-1}) / h on the faces along `axis`; zero on wall faces."""
    if not walls:
        return (P - np.roll(P, 1, axis=axis)) / h
    n = P.shape[axis]
    inner = (np.take(P, range(1, n), axis=axis) - np.take(P, range(0, n - 1), axis=axis)) / h
    zero = np.zeros_like(np.take(P, [0], axis=axis))
    return np.concatenate([zero, inner, zero], axis=axis)


def div(Fx, Fy, Fz, h, zwalls):
    """(F_{i+1} - F_i) / h summed over the three directions, at the cells."""
    d = (np.roll(Fx, -1, axis=2) - Fx) / h + (np.roll(Fy, -1, axis=1) - Fy) / h
    if zwalls:
        return d + (Fz[1:] - Fz[:-1]) / h
    return d + (np.roll(Fz, -1, axis=0) - Fz) / h


def poisson(rhs, h, zwalls):
    """Zero-mean P with lap P = rhs - mean(rhs) (7-point Laplacian, periodic
    x and y, z periodic or between walls with dP/dz = 0).  FFT in x and y
    (z too when periodic); between walls, one dense solve along z per (ky, kx)
    mode, the singular mode taken as the minimum-norm (zero-mean) solution."""
    nz, ny, nx = rhs.shape
    r = rhs - rhs.mean()
    lx = -(4.0 / h ** 2) * np.sin(np.pi * np.arange(nx) / nx) ** 2
    ly = -(4.0 / h ** 2) * np.sin(np.pi * np.arange(ny) / ny) ** 2
    lxy = ly[:, None] + lx[None, :]
    if not zwalls:
        lz = -(4.0 / h ** 2) * np.sin(np.pi * np.arange(nz) / nz) ** 2
        F = np.fft.fftn(r)
        lam = lz[:, None, None] + lxy[None, :, :]
        lam[0, 0, 0] = 1.0
        Ph = F / lam
        Ph[0, 0, 0] = 0.0
        return np.real(np.fft.ifftn(Ph))
    F = np.fft.fft2(r, axes=(1, 2))                 # [nz][ny][nx] complex
    T = np.zeros((nz, nz))
    for k in range(nz):
        T[k, k] = -2.0 / h ** 2
        if k > 0:
            T[k, k - 1] = 1.0 / h ** 2
        if k < nz - 1:
            T[k, k + 1] = 1.0 / h ** 2
    T[0, 0] = T[-1, -1] = -1.0 / h ** 2            # dP/dz = 0 on both walls
    Ph = np.empty_like(F)
    for j in range(ny):
        for i in range(nx):
            A = T + lxy[j, i] * np.eye(nz)
            if j == 0 and i == 0:
                Ph[:, j, i] = np.linalg.lstsq(A, F[:, j, i], rcond=None)[0]
            else:
                Ph[:, j, i] = np.linalg.solve(A, F[:, j, i])
    P = np.real(np.fft.ifft2(Ph, axes=(1, 2)))
    return P - P.mean()


def laplacian(P, h, zwalls):
    """The 7-point Laplacian as div(grad P) of the operators above."""
    return div(grad(P, 2, h, False), grad(P, 1, h, False), grad(P, 0, h, zwalls), h, zwalls)


def pressure_step(C, u, v, w, P, Pold, h, dt, rho1, rho2, zwalls):
    """One split-density pressure step.  Inputs: C (cells), the provisional
    velocity u*, v*, w* (faces), P = P^l and Pold = P^{l-1} (cells).
    Returns u, v, w at l+1, P^{l+1}, and P^l (the next step's Pold):
      Phat = 2 P^l - P^{l-1};
      lap P^{l+1} = div[(1 - rho2/rho) grad Phat] + (rho2/dt) div u*   (eq-newpoi)
      u^{l+1} = u* - dt [grad P^{l+1} / rho2 + (1/rho - 1/rho2) grad Phat]  (eq-u)
    with rho on the faces."""
    rho = density(C, rho1, rho2)
    Phat = 2.0 * P - Pold
    walls = (False, False, zwalls)
    rf = [face_mean(rho, 2, False), face_mean(rho, 1, False), face_mean(rho, 0, zwalls)]
    gh = [grad(Phat, 2, h, False), grad(Phat, 1, h, False), grad(Phat, 0, h, zwalls)]
    flux = [(1.0 - rho2 / r) * g for r, g in zip(rf, gh)]
    rhs = div(*flux, h, zwalls) + (rho2 / dt) * div(u, v, w, h, zwalls)
    Pn = poisson(rhs, h, zwalls)
    gn = [grad(Pn, 2, h, False), grad(Pn, 1, h, False), grad(Pn, 0, h, zwalls)]
    out = [vel - dt * (g / rho2 + (1.0 / r - 1.0 / rho2) * gp)
           for vel, g, r, gp in zip((u, v, w), gn, rf, gh)]
    if zwalls:
        out[2][0] = 0.0
        out[2][-1] = 0.0
    return out[0], out[1], out[2], Pn, P.copy()
