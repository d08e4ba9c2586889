"""Fourier-space building blocks of DBFFT (oracle; test infrastructure only).

Conventions (readings of the paper where it leaves a choice open):
  * cell of side lengths L_a (default 1); voxel-centre sampling (Sec. 2.1);
  * xi_a = 2 pi m_a / L_a with m_a the signed DFT frequency of index k_a; on even
    grids the Nyquist index k_a = n_a/2 gets xi_a = 0 (Sec. 2.1 leaves even
    grids open and mentions neglecting the Nyquist frequencies);
  * the unknown is the normalized Fourier coefficient a = F[u]/N, so that
    u(x) = sum_k a(k) exp(i xi.x); stress coefficients are s = F[sigma]/N,
    whose k = 0 value is the volume average <sigma>;
  * only the R2C half spectrum k3 = 0..n3//2 is stored (Sec. 2.2: the
    duplicated terms of the real transform are removed); the real inner
    product counts the k3 = 0 plane (and the k3 = n3/2 plane on even n3)
    once and every other plane twice.
"""
from __future__ import annotations

import numpy as np


def axis_xi(n, length=1.0):
    """Frequencies xi = 2 pi m / L of one axis of n points over a length L,
    in DFT index order (Sec. 2.1, frequency vector; Nyquist zeroed on even
    n)."""
    k = np.arange(n)
    m = np.where(k < (n + 1) // 2, k, k - n).astype(np.float64)
    if n % 2 == 0:
        m[n // 2] = 0.0
    return 2.0 * np.pi * m / float(length)


def half_shape(shape):
    n1, n2, n3 = shape
    return (n1, n2, n3 // 2 + 1)


def xi_half(shape, lengths=None):
    """Frequency vector field on the half spectrum, shape (3, n1, n2, n3//2+1),
    for a cell of side lengths L1, L2, L3 (default 1, 1, 1)."""
    n1, n2, n3 = shape
    L1, L2, L3 = (1.0, 1.0, 1.0) if lengths is None else lengths
    h = half_shape(shape)
    x1 = axis_xi(n1, L1)[:, None, None]
    x2 = axis_xi(n2, L2)[None, :, None]
    x3 = axis_xi(n3, L3)[: n3 // 2 + 1][None, None, :]
    xi = np.zeros((3,) + h)
    xi[0] = np.broadcast_to(x1, h)
    xi[1] = np.broadcast_to(x2, h)
    xi[2] = np.broadcast_to(x3, h)
    return xi


def null_set(shape):
    """Boolean mask of half-spectrum frequencies whose xi is the zero vector:
    the mean plus, on even grids, the Nyquist-only points.  The operators
    s-hat, g-hat and d-hat vanish there (Sec. 2.2); those unknowns are fixed
    to zero."""
    xi = xi_half(shape)
    return np.all(xi == 0.0, axis=0)


def half_weights(shape):
    """Multiplicity of each k3 plane in the full spectrum (1 or 2)."""
    n3 = shape[2]
    w = np.full(n3 // 2 + 1, 2.0)
    w[0] = 1.0
    if n3 % 2 == 0:
        w[-1] = 1.0
    return w


# ---------------------------------------------------------------------------
# The oracle's own discrete Fourier transform: the defining sums
#   X(k) = sum_j x(j) exp(-2 pi i j k / n)
# evaluated axis by axis as products with dense n x n matrices (no fast
# algorithm).  Angles are formed from the integer j k mod n, so every entry
# is the FP64 cos / sin of 2 pi m / n for an exact integer m.
# ---------------------------------------------------------------------------

def dft_matrix(n, sign=-1):
    """W[j, k] = exp(sign 2 pi i j k / n).  The angle is taken from
    min(m, n - m) with m = j k mod n and the sine's sign restored, so that
    W[j, n - k] = conj W[j, k] holds exactly: the transform of a real field
    is then exactly Hermitian, X(-k) = conj X(k)."""
    k = np.arange(n)
    m = np.outer(k, k) % n
    mr = np.minimum(m, n - m)
    ang = 2.0 * np.pi * mr / n
    sgn = np.where(m > n - m, -1.0, 1.0)
    return np.cos(ang) + sign * 1j * sgn * np.sin(ang)


def _along(W, x, axis):
    """sum_j W[k, j] x[..., j, ...] along `axis` (W symmetric here)."""
    x = np.moveaxis(x, axis, 0)
    lead = x.shape[0]
    y = W @ x.reshape(lead, -1)
    return np.moveaxis(y.reshape((W.shape[0],) + x.shape[1:]), 0, axis)


def dft_r2c(field, shape):
    """Unnormalized forward DFT of a real field over its last three axes,
    k3 = 0..n3//2 kept (the other half is the complex conjugate)."""
    n1, n2, n3 = shape
    h3 = n3 // 2 + 1
    W3 = dft_matrix(n3)[:, :h3]
    f = np.asarray(field, dtype=np.float64)
    out = (f @ W3.real) + 1j * (f @ W3.imag)
    out = _along(dft_matrix(n2), out, -2)
    return _along(dft_matrix(n1), out, -3)


def dft_c2r(coeffs, shape):
    """Unnormalized inverse DFT back to a real field: the sum over the full
    spectrum of the half spectrum extended by X(-k) = conj X(k).  On the
    self-conjugate planes k3 = 0 and k3 = n3/2 (even n3) only the real part
    of the k3 sum counts, as for any real synthesis."""
    n1, n2, n3 = shape
    h3 = n3 // 2 + 1
    c = _along(dft_matrix(n1, +1), np.asarray(coeffs, dtype=complex), -3)
    c = _along(dft_matrix(n2, +1), c, -2)
    mult = np.full(h3, 2.0)
    mult[0] = 1.0
    if n3 % 2 == 0:
        mult[-1] = 1.0
    E = dft_matrix(n3, +1)[:h3, :] * mult[:, None]
    return c.real @ E.real - c.imag @ E.imag


def fourier(field, shape):
    """Normalized forward transform F[f]/N over the last three axes."""
    N = float(np.prod(shape))
    return dft_r2c(field, shape) / N


def real_field(coeffs, shape):
    """Synthesis u(x) = sum_k a(k) exp(i xi.x) (unnormalized inverse DFT)."""
    return dft_c2r(coeffs, shape)


def sym_grad(a, xi):
    """Fourier symmetric gradient (Sec. 2.2, eq. symgrad):
    eps_ij = (1/2)(i xi_j a_i + i xi_i a_j).  a: (3, ...) -> (3, 3, ...)."""
    g = 1j * a[:, None] * xi[None, :]          # g_ij = i xi_j a_i
    return 0.5 * (g + np.swapaxes(g, 0, 1))


def full_grad(a, xi):
    """Fourier displacement gradient for finite strains (Sec. 2.4):
    H_ij = i xi_j a_i (the printed operator omits the imaginary unit that
    the derivative rule eq. 1Ddif requires)."""
    return 1j * a[:, None] * xi[None, :]


def div(s, xi):
    """Fourier divergence (Sec. 2.2, eq. diver): (d:s)_i = i xi_j s_ij."""
    return 1j * np.einsum("ij...,j...->i...", s, xi)


def inner(u, v, w):
    """Real inner product of two half-spectrum fields (any leading axes),
    equal to Re sum over the full spectrum of conj(u).v."""
    return float(np.sum(w * (u.real * v.real + u.imag * v.imag)))


def valid_coefficients(real_vector_field, shape):
    """Coefficients of a real field with the null-set entries cleared (the
    admissible unknowns of the scheme)."""
    a = fourier(real_vector_field, shape)
    a[..., null_set(shape)] = 0.0
    return a


# Mandel basis of symmetric 3x3 tensors: orthonormal w.r.t. A:B.
MANDEL_PAIRS = ((0, 0), (1, 1), (2, 2), (1, 2), (0, 2), (0, 1))


def mandel_basis():
    B = np.zeros((6, 3, 3))
    r = 1.0 / np.sqrt(2.0)
    for a, (i, j) in enumerate(MANDEL_PAIRS):
        if i == j:
            B[a, i, i] = 1.0
        else:
            B[a, i, j] = r
            B[a, j, i] = r
    return B


def full_basis():
    """Orthonormal basis e_i (x) e_J of all 3x3 tensors (finite strains)."""
    B = np.zeros((9, 3, 3))
    for a in range(9):
        B[a, a // 3, a % 3] = 1.0
    return B
