"""Error estimates of a computed state (Sec. 3; oracle, test infrastructure
only, imported by nothing in the product).

  * equilibrium residual (eq. chedckeq): ||div sigma||_L2 / ||<sigma>||, the
    L2 norm of a field being the root mean square over the voxels of its
    Frobenius (or Euclidean) norm; at finite strains the first
    Piola-Kirchhoff stress and the divergence in the reference
    configuration (Sec. 3.3);
  * compatibility residual (eq. chedckcomp): the largest absolute value of
    any component of curl curl eps at any voxel, divided by ||<eps>||, with
    (curl curl eps)_ij = e_ikl e_jmn d_k d_m eps_ln; at finite strains
    (Sec. 3.3) max |curl_0 F| / ||<F> - I||, the curl of F taken row by row,
    (curl_0 F)_ij = e_jkl d_k F_il;
  * loading residuals (eq. chedckimp), one over the strain-prescribed and
    one over the stress-prescribed components of a mixed load.

Derivatives are spectral: multiplication of the normalized Fourier
coefficients by i xi, with the frequencies of Sec. 2.1 (xi = 2 pi m / L for
cell side lengths L, default 1; the Nyquist index of an even axis gets
xi = 0).  Fields are full tensors of shape (3, 3) + grid.
"""
from __future__ import annotations

import numpy as np

from . import spectral as sp


def levi_civita():
    e = np.zeros((3, 3, 3))
    for i, j, k in ((0, 1, 2), (1, 2, 0), (2, 0, 1)):
        e[i, j, k] = 1.0
        e[i, k, j] = -1.0
    return e


def spectral_derivative(f, shape, axes, lengths=None):
    """d_{a1} d_{a2} ... f of a real field over its last three axes."""
    c = sp.fourier(f, shape)
    xi = sp.xi_half(shape, lengths)
    for a in axes:
        c = 1j * xi[a] * c
    return sp.real_field(c, shape)


def divergence(s, shape, lengths=None):
    """(div s)_i = d_j s_ij of a tensor field (3, 3) + grid."""
    return np.stack([sum(spectral_derivative(s[i, j], shape, (j,), lengths) for j in range(3)) for i in range(3)])


def incompatibility(eps, shape, lengths=None):
    """curl curl eps (symmetric) of a small-strain field."""
    e = levi_civita()
    second = {}
    for k in range(3):
        for m in range(k, 3):
            for l in range(3):
                for n in range(3):
                    second[(k, m, l, n)] = spectral_derivative(eps[l, n], shape, (k, m), lengths)
    out = np.zeros((3, 3) + tuple(shape))
    for i in range(3):
        for j in range(3):
            for k in range(3):
                for l in range(3):
                    for m in range(3):
                        for n in range(3):
                            c = e[i, k, l] * e[j, m, n]
                            if c != 0.0:
                                out[i, j] += c * second[(min(k, m), max(k, m), l, n)]
    return out


def row_curl(F, shape, lengths=None):
    """(curl_0 F)_ij = e_jkl d_k F_il, the curl of every row of F."""
    e = levi_civita()
    out = np.zeros((3, 3) + tuple(shape))
    for i in range(3):
        for j in range(3):
            for k in range(3):
                for l in range(3):
                    if e[j, k, l] != 0.0:
                        out[i, j] += e[j, k, l] * spectral_derivative(F[i, l], shape, (k,), lengths)
    return out


def _mean(t):
    return t.reshape(3, 3, -1).mean(axis=2)


def _ratio(num, den):
    if den == 0.0:
        return 0.0 if num == 0.0 else np.inf
    return num / den


def equilibrium_residual(sig, shape, lengths=None):
    """Eq. chedckeq (P and the reference divergence at finite strains)."""
    d = divergence(sig, shape, lengths)
    l2 = np.sqrt(np.mean(np.sum(d * d, axis=0)))
    return _ratio(float(l2), float(np.linalg.norm(_mean(sig))))


def compatibility_residual(field, shape, finite=False, lengths=None):
    """Eq. chedckcomp; `field` is eps, or at finite strains the displacement
    gradient H = F - I (curl_0 F = curl_0 H, <F> - I = <H>)."""
    inc = row_curl(field, shape, lengths) if finite else incompatibility(field, shape, lengths)
    return _ratio(float(np.max(np.abs(inc))), float(np.linalg.norm(_mean(field))))


def loading_residuals(mean_strain, mean_stress, load, stress_mask, finite=False):
    """Eq. chedckimp on a mixed load: (strain part, stress part).

    Strain part: ||<eps>_E - epsbar_E|| / ||epsbar_E|| over the components E
    whose mask entry is 0 (at finite strains <F> = I + <H> against the
    prescribed F, relative to ||Fbar_E - I_E||).  Stress part:
    ||<sigma>_S - sigmabar_S|| / ||<sigma>|| over the stress-prescribed set S
    (the denominator the solver's loading test uses, which stays finite
    when the prescribed stress is zero).  An empty set gives 0."""
    load = np.asarray(load, dtype=np.float64).reshape(3, 3)
    S = np.asarray(stress_mask, dtype=bool).reshape(3, 3)
    E = ~S
    ms = np.asarray(mean_strain, dtype=np.float64).reshape(3, 3)
    if finite:
        ms = ms + np.eye(3)
        ref = load - np.eye(3)
    else:
        ref = load
    strain_part = _ratio(float(np.linalg.norm((ms - load)[E])), float(np.linalg.norm(ref[E]))) if E.any() else 0.0
    sig = np.asarray(mean_stress, dtype=np.float64).reshape(3, 3)
    stress_part = _ratio(float(np.linalg.norm((sig - load)[S])), float(np.linalg.norm(sig))) if S.any() else 0.0
    return strain_part, stress_part
