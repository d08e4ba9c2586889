"""Constitutive laws used by the oracle (test infrastructure only).

The paper derives DBFFT for any local law (Sec. 2.2 linear elasticity,
Sec. 2.4 general P(F, L, alpha) with consistent tangent K = dP/dF).  The
workloads here use:
  * isotropic linear elasticity (Sec. 3.1 material: E, nu per phase);
  * cubic elasticity rotated per grain, with a rate-dependent J2 flow rule
    integrated by backward Euler (a stand-in for the paper's crystal
    plasticity of Sec. 3.4, whose parameters live in a cited work);
  * the Saint Venant-Kirchhoff hyperelastic law of Sec. 3.3 (matrix and
    compliant pores, E and nu per phase);
  * compressible neo-Hookean hyperelasticity (a second finite-strain law).
The J2 and neo-Hookean laws are not in the paper: their parity is pinned by
closed forms and finite differences in tests/, not by the paper.
"""
from __future__ import annotations

import numpy as np

from .spectral import mandel_basis

I3 = np.eye(3)


def lame(E, nu):
    """(lambda, mu) from Young's modulus and Poisson's ratio."""
    E = np.asarray(E, dtype=np.float64)
    lam = E * nu / ((1.0 + nu) * (1.0 - 2.0 * nu))
    mu = E / (2.0 * (1.0 + nu))
    return lam, mu


def isotropic_tensor(lam, mu):
    """C_ijkl = lam d_ij d_kl + mu (d_ik d_jl + d_il d_jk) (scalars)."""
    d = I3
    return (lam * np.einsum("ij,kl->ijkl", d, d)
            + mu * (np.einsum("ik,jl->ijkl", d, d) + np.einsum("il,jk->ijkl", d, d)))


def cubic_tensor(c11, c12, c44):
    """Cubic stiffness in the crystal frame: C_iiii = c11, C_iijj = c12
    (i != j), C_ijij = C_ijji = c44 (i != j)."""
    C = np.zeros((3, 3, 3, 3))
    for i in range(3):
        for j in range(3):
            if i == j:
                C[i, i, i, i] = c11
            else:
                C[i, i, j, j] = c12
                C[i, j, i, j] = c44
                C[i, j, j, i] = c44
    return C


def rotate_tensor4(C, R):
    """C'_ijkl = R_ia R_jb R_kc R_ld C_abcd; R maps crystal to sample axes.
    R may carry leading batch axes (..., 3, 3)."""
    return np.einsum("...ia,...jb,...kc,...ld,abcd->...ijkl", R, R, R, R, C)


def tensor4_to_mandel(C):
    """6x6 matrix M_ab = B_a : C : B_b in the orthonormal Mandel basis.
    Leading batch axes allowed on C (..., 3, 3, 3, 3)."""
    B = mandel_basis()
    return np.einsum("aij,...ijkl,bkl->...ab", B, C, B)


def mandel_to_tensor4(M):
    B = mandel_basis()
    return np.einsum("aij,...ab,bkl->...ijkl", B, M, B)


def sym_to_mandel(t):
    """Mandel 6-vector of symmetric tensors with layout (3, 3, ...)."""
    B = mandel_basis()
    return np.einsum("aij,ij...->a...", B, t)


def mandel_to_sym(v):
    B = mandel_basis()
    return np.einsum("aij,a...->ij...", B, v)


# ---------------------------------------------------------------------------
# Rate-dependent J2 (von Mises) viscoplasticity, small strains.
#   sigma = C : (eps - eps_p),   d eps_p/dt = edot0 (s_eq/s0)^m n,
#   n = (3/2) dev(sigma)/s_eq,   no threshold, no hardening.
# Backward Euler over one increment dt with unknowns (sigma, y = ln dp):
#   R1 = S sigma - (eps - eps_p_n) + exp(y) n(sigma) = 0      (S = C^-1)
#   R2 = m ln(s_eq/s0) - y + ln(edot0 dt)             = 0
# ---------------------------------------------------------------------------

_ONE = np.array([1.0, 1.0, 1.0, 0.0, 0.0, 0.0])
_PDEV = np.eye(6) - np.outer(_ONE, _ONE) / 3.0


def _seq_and_n(sig):
    """Equivalent stress and flow direction of Mandel stresses (nv, 6)."""
    s = sig @ _PDEV.T
    seq = np.sqrt(1.5 * np.sum(s * s, axis=1))
    with np.errstate(invalid="ignore", divide="ignore"):
        n = 1.5 * s / seq[:, None]
    return seq, n


def j2vp_return_map(eps, eps_p_n, C, s0, m, edot0, dt, elastic_cutoff=1e-12):
    """Backward-Euler update of the J2 viscoplastic law, voxel by voxel.

    eps, eps_p_n : (nv, 6) Mandel strains at t_{n+1} and plastic strain at t_n
    C            : (nv, 6, 6) Mandel elastic stiffness
    s0           : flow stress, a scalar or one value per voxel (nv,)
    Returns sigma (nv, 6), dp (nv,), eps_p (nv, 6) and the consistent tangent
    (nv, 6, 6): [S + dp dn/dsigma + dp (m/s_eq) n n^T]^-1 with
    dn/dsigma = (3/(2 s_eq)) (P_dev - (2/3) n n^T).

    Voxels whose elastic predictor has s_eq <= elastic_cutoff * s0 are
    returned elastic (dp = 0, tangent C).
    """
    eps = np.asarray(eps, dtype=np.float64)
    nv = eps.shape[0]
    s0v = np.broadcast_to(np.asarray(s0, dtype=np.float64), (nv,))
    S = np.linalg.inv(C)
    sig_tr = np.einsum("vab,vb->va", C, eps - eps_p_n)
    seq_tr, n_tr = _seq_and_n(sig_tr)
    logc = np.log(edot0 * dt)

    sig = sig_tr.copy()
    dp = np.zeros(nv)
    tangent = C.copy()
    act = seq_tr > elastic_cutoff * s0v
    if not np.any(act):
        return sig, dp, eps_p_n.copy(), tangent
    s0 = s0v[act]

    # Scalar starting value: s_eq ~ s_eq_tr - h dp with h = n_tr : C : n_tr,
    # dp = edot0 dt (s_eq/s0)^m, solved in y = ln dp by bracketed Newton.
    h = np.einsum("va,vab,vb->v", n_tr, C, n_tr)
    st, hh = seq_tr[act], h[act]
    lo = np.minimum(np.log(0.5 * st / hh), logc + m * np.log(0.5 * st / s0))
    hi = np.log(st / hh)
    y = 0.5 * (lo + hi)
    for _ in range(200):
        g = st - hh * np.exp(y) - s0 * np.exp((y - logc) / m)
        dg = -hh * np.exp(y) - (s0 / m) * np.exp((y - logc) / m)
        lo = np.where(g > 0, y, lo)
        hi = np.where(g > 0, hi, y)
        yn = y - g / dg
        out = (yn <= lo) | (yn >= hi)
        yn = np.where(out, 0.5 * (lo + hi), yn)
        done = np.abs(yn - y) <= 1e-14 * np.maximum(1.0, np.abs(y))
        y = yn
        if np.all(done):
            break

    # Full 7-unknown Newton from (sigma_tr - exp(y) C n_tr, y).
    Ca, Sa = C[act], S[act]
    e_el = (eps - eps_p_n)[act]
    sg = sig_tr[act] - np.exp(y)[:, None] * np.einsum("vab,vb->va", Ca, n_tr[act])
    for it in range(100):
        seq, n = _seq_and_n(sg)
        ey = np.exp(y)
        R1 = np.einsum("vab,vb->va", Sa, sg) - e_el + ey[:, None] * n
        R2 = m * np.log(seq / s0) - y + logc
        dn = (1.5 / seq)[:, None, None] * (_PDEV[None] - (2.0 / 3.0) * np.einsum("va,vb->vab", n, n))
        J = np.zeros((sg.shape[0], 7, 7))
        J[:, :6, :6] = Sa + ey[:, None, None] * dn
        J[:, :6, 6] = ey[:, None] * n
        J[:, 6, :6] = (m / seq)[:, None] * n
        J[:, 6, 6] = -1.0
        R = np.concatenate([R1, R2[:, None]], axis=1)
        d = np.linalg.solve(J, -R[..., None])[..., 0]
        sg = sg + d[:, :6]
        y = y + d[:, 6]
        if np.all(np.abs(d[:, :6]) <= 1e-11 * s0[:, None]) and np.max(np.abs(d[:, 6])) <= 1e-11:
            break
    seq, n = _seq_and_n(sg)
    dpa = np.exp(y)
    dn = (1.5 / seq)[:, None, None] * (_PDEV[None] - (2.0 / 3.0) * np.einsum("va,vb->vab", n, n))
    A = Sa + dpa[:, None, None] * dn + (dpa * m / seq)[:, None, None] * np.einsum("va,vb->vab", n, n)
    sig[act] = sg
    dp[act] = dpa
    tangent[act] = np.linalg.inv(A)
    eps_p = eps_p_n.copy()
    eps_p[act] = eps_p_n[act] + dpa[:, None] * n
    return sig, dp, eps_p, tangent


# ---------------------------------------------------------------------------
# Compressible neo-Hookean:  W = mu/2 (I1 - 3) - mu ln J + lam/2 (ln J)^2
#   P = mu (F - F^-T) + lam ln J F^-T
#   K_iJkL = mu d_ik d_JL + (mu - lam ln J) Finv_Li Finv_Jk + lam Finv_Ji Finv_Lk
# ---------------------------------------------------------------------------

def neohooke_stress(F, mu, lam):
    """First Piola-Kirchhoff stress; F (..., 3, 3), mu/lam broadcastable."""
    Finv = np.linalg.inv(F)
    J = np.linalg.det(F)
    FinvT = np.swapaxes(Finv, -1, -2)
    mu = np.asarray(mu)[..., None, None]
    lam = np.asarray(lam)[..., None, None]
    return mu * (F - FinvT) + lam * np.log(J)[..., None, None] * FinvT


def neohooke_tangent(F, mu, lam):
    """dP/dF as a (..., 3, 3, 3, 3) array indexed [i, J, k, L]."""
    Finv = np.linalg.inv(F)
    lnJ = np.log(np.linalg.det(F))
    mu = np.asarray(mu, dtype=np.float64)
    lam = np.asarray(lam, dtype=np.float64)
    d = I3
    t1 = np.einsum("ik,JL->iJkL", d, d)
    t2 = np.einsum("...Li,...Jk->...iJkL", Finv, Finv)
    t3 = np.einsum("...Ji,...Lk->...iJkL", Finv, Finv)
    c2 = (mu - lam * lnJ)
    return (mu[..., None, None, None, None] * t1
            + c2[..., None, None, None, None] * t2
            + lam[..., None, None, None, None] * t3)


# ---------------------------------------------------------------------------
# Saint Venant-Kirchhoff (Sec. 3.3):  S = lam tr(E) I + 2 mu E with the
# Green-Lagrange strain E = (F^T F - I)/2, and P = F S.
#   dP = dF S + F dS,  dS = lam tr(dE) I + 2 mu dE,  dE = sym(F^T dF)
#   K_iJkL = d_ik S_LJ + lam F_iJ F_kL + mu (F_iL F_kJ + (F F^T)_ik d_JL)
# ---------------------------------------------------------------------------

def svk_second_pk(F, mu, lam):
    """Second Piola-Kirchhoff stress S of F (..., 3, 3)."""
    E = 0.5 * (np.swapaxes(F, -1, -2) @ F - I3)
    trE = np.trace(E, axis1=-2, axis2=-1)
    mu = np.asarray(mu)[..., None, None]
    lam = np.asarray(lam)[..., None, None]
    return lam * trE[..., None, None] * I3 + 2.0 * mu * E


def svk_stress(F, mu, lam):
    """First Piola-Kirchhoff stress P = F S."""
    return F @ svk_second_pk(F, mu, lam)


def svk_tangent(F, mu, lam):
    """dP/dF as a (..., 3, 3, 3, 3) array indexed [i, J, k, L]."""
    S = svk_second_pk(F, mu, lam)
    mu = np.asarray(mu, dtype=np.float64)[..., None, None, None, None]
    lam = np.asarray(lam, dtype=np.float64)[..., None, None, None, None]
    FFt = F @ np.swapaxes(F, -1, -2)
    t1 = np.einsum("ik,...LJ->...iJkL", I3, S)
    t2 = np.einsum("...iJ,...kL->...iJkL", F, F)
    t3 = np.einsum("...iL,...kJ->...iJkL", F, F)
    t4 = np.einsum("...ik,JL->...iJkL", FFt, I3)
    return t1 + lam * t2 + mu * (t3 + t4)
