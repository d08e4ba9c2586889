"""FFT-free definition of the discrete DBFFT problem (oracle; test
infrastructure only).

On a periodic grid of n points of the unit cell, the derivative of the
trigonometric interpolant of grid values is a circulant matrix D with
entries D_ij = S'(x_i - x_j), S the periodic sinc interpolant
(Trefethen, Spectral Methods in MATLAB, ch. 3):
    S'(0) = 0,
    S'(k h) = pi (-1)^k cot(pi k / n)   (even n, Nyquist mode symmetrized),
    S'(k h) = pi (-1)^k csc(pi k / n)   (odd n).
On even grids this interpolant drops the derivative of the Nyquist mode,
which is the even-grid reading used by the Fourier route (Sec. 2.1).

The linear DBFFT problem (Sec. 2.2 / 2.3) is the stationarity of the average
energy 1/2 <eps:C:eps> - sbar_S . e over periodic u and e, with
eps = E_U + e + sym(D u).  Assembling its Hessian densely and solving with
a pseudo-inverse (the null space is the constant and Nyquist-only modes of
each displacement component) gives the discrete solution with no FFT and
no iteration.  Feasible up to a few thousand unknowns.
"""
from __future__ import annotations

import numpy as np

from .spectral import mandel_basis, MANDEL_PAIRS


def diff_matrix(n, length=1.0):
    """Periodic spectral differentiation matrix on [0, L) with n points."""
    D = np.zeros((n, n))
    for i in range(n):
        for j in range(n):
            k = i - j
            if k % n == 0:
                continue
            if n % 2 == 0:
                D[i, j] = np.pi * (-1.0) ** k / np.tan(np.pi * k / n)
            else:
                D[i, j] = np.pi * (-1.0) ** k / np.sin(np.pi * k / n)
    return D / float(length)


def partial_matrices(shape, lengths=None):
    """Dense d/dx_a acting on C-ordered flattened grid functions of a cell
    of side lengths L1, L2, L3 (default 1, 1, 1)."""
    n1, n2, n3 = shape
    L1, L2, L3 = (1.0, 1.0, 1.0) if lengths is None else lengths
    I1, I2, I3 = np.eye(n1), np.eye(n2), np.eye(n3)
    return [np.kron(np.kron(diff_matrix(n1, L1), I2), I3),
            np.kron(np.kron(I1, diff_matrix(n2, L2)), I3),
            np.kron(np.kron(I1, I2), diff_matrix(n3, L3))]


def strain_map(shape, lengths=None):
    """Dense map u (3N, component-major) -> Mandel strains (6, N) as a
    (6N, 3N) matrix: eps_ij = (D_j u_i + D_i u_j)/2."""
    N = int(np.prod(shape))
    D = partial_matrices(shape, lengths)
    B = np.zeros((6 * N, 3 * N))
    Bm = mandel_basis()
    for a, (i, j) in enumerate(MANDEL_PAIRS):
        # eps : B_a = sum_kl B_a,kl (D_l u_k + D_k u_l)/2 = sum_kl B_a,kl D_l u_k
        for k in range(3):
            for l in range(3):
                c = Bm[a, k, l]
                if c != 0.0:
                    B[a * N:(a + 1) * N, k * N:(k + 1) * N] += c * D[l]
    return B


def assemble(shape, C_mandel, stress_mask=None, lengths=None):
    """Dense Hessian of the average energy in the unknowns (u (3N), e (|S|)).
    C_mandel: (N, 6, 6) per-voxel Mandel stiffness (C-order voxels).
    Returns (K, Bu, S) with Bu the strain map and S the Mandel indices."""
    N = int(np.prod(shape))
    if stress_mask is None:
        stress_mask = np.zeros((3, 3), dtype=bool)
    S = [a for a, (i, j) in enumerate(MANDEL_PAIRS) if stress_mask[i, j]]
    Bu = strain_map(shape, lengths)
    # block-diagonal per-voxel stiffness acting on Mandel fields (6, N)
    Cb = np.zeros((6 * N, 6 * N))
    for a in range(6):
        for b in range(6):
            Cb[a * N:(a + 1) * N, b * N:(b + 1) * N] = np.diag(C_mandel[:, a, b])
    # macro strain e_s adds the constant Mandel vector unit_s at every voxel
    Be = np.zeros((6 * N, len(S)))
    for c, a in enumerate(S):
        Be[a * N:(a + 1) * N, c] = 1.0
    Bfull = np.concatenate([Bu, Be], axis=1)
    K = Bfull.T @ Cb @ Bfull / N
    return K, Bfull, Cb, S


def solve(shape, C_mandel, load, stress_mask=None, lengths=None):
    """Direct solve of the linear problem.  Returns (u (3, n1, n2, n3),
    e (|S|), <sigma> (3x3))."""
    N = int(np.prod(shape))
    if stress_mask is None:
        stress_mask = np.zeros((3, 3), dtype=bool)
    mask = np.asarray(stress_mask, dtype=bool)
    K, Bfull, Cb, S = assemble(shape, C_mandel, mask, lengths)
    Bm = mandel_basis()
    load = np.asarray(load, dtype=np.float64)
    E_U = load * (~mask)
    sbar = np.array([np.sum(Bm[a] * load) for a in S])
    eU = np.array([np.sum(Bm[a] * E_U) for a in range(6)])
    eps0 = np.repeat(eU, N)
    # gradient of 1/2 <(eps0 + B x):C:(eps0 + B x)> - sbar.e  is  K x + B^T C eps0/N - [0; sbar]
    rhs = -(Bfull.T @ (Cb @ eps0)) / N
    rhs[3 * N:] += sbar
    x = np.linalg.lstsq(K, rhs, rcond=1e-12)[0]
    eps = eps0 + Bfull @ x
    sig = Cb @ eps
    sig_avg_m = sig.reshape(6, N).mean(axis=1)
    sig_avg = np.einsum("a,aij->ij", sig_avg_m, Bm)
    u = x[:3 * N].reshape((3,) + tuple(shape))
    return u, x[3 * N:], sig_avg
