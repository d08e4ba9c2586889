"""Pins of the oracle's material laws, Newton scheme (Sec. 2.4) and adjoint
gradient against closed forms, special cases and finite differences."""
import numpy as np
import pytest

from oracle import spectral as sp, solver as so, materials as mt
from paper_1905_12725_amd import microstructure as ms


S0, M, EDOT0 = 100.0, 20.0, 1e-3


def test_j2_isotropic_matches_scalar_radial_return():
    """With isotropic elasticity the return map reduces to the scalar
    equation s_eq = s_eq_tr - 3 mu dp, dp = edot0 dt (s_eq/s0)^m, solved here
    by plain bisection; sigma = sigma_tr - 2 mu dp n_tr."""
    rng = np.random.default_rng(11)
    lam, mu = mt.lame(200000.0, 0.3)
    C = mt.tensor4_to_mandel(mt.isotropic_tensor(lam, mu))
    nv = 50
    eps = rng.standard_normal((nv, 6)) * 1.5e-3
    epn = rng.standard_normal((nv, 6)) * 1e-4
    epn[:, :3] -= epn[:, :3].mean(axis=1, keepdims=True)
    dt = 0.5
    sig, dp, ep, tan = mt.j2vp_return_map(eps, epn, np.broadcast_to(C, (nv, 6, 6)), S0, M, EDOT0, dt)
    one = np.array([1, 1, 1, 0, 0, 0.0])
    for v in range(nv):
        st = C @ (eps[v] - epn[v])
        s = st - one * st[:3].sum() / 3
        seq = np.sqrt(1.5 * s @ s)
        lo, hi = 0.0, seq / (3 * mu)
        for _ in range(300):
            mid = 0.5 * (lo + hi)
            g = seq - 3 * mu * mid - S0 * (mid / (EDOT0 * dt)) ** (1 / M)
            lo, hi = (mid, hi) if g > 0 else (lo, mid)
        d = 0.5 * (lo + hi)
        expect = st - 2 * mu * d * 1.5 * s / seq
        assert np.isclose(dp[v], d, rtol=1e-10)
        assert np.allclose(sig[v], expect, rtol=1e-10, atol=1e-9)


def test_j2_tangent_finite_difference():
    rng = np.random.default_rng(12)
    R = ms.random_rotations(4, 3)
    C = mt.tensor4_to_mandel(mt.rotate_tensor4(mt.cubic_tensor(168000.0, 121000.0, 75000.0), R))
    eps = rng.standard_normal((4, 6)) * 2e-3
    epn = np.zeros((4, 6))
    sig, dp, ep, tan = mt.j2vp_return_map(eps, epn, C, S0, M, EDOT0, 0.5)
    assert np.all(dp > 0)
    h = 1e-8
    for b in range(6):
        ep_ = eps.copy(); ep_[:, b] += h
        em_ = eps.copy(); em_[:, b] -= h
        sp_, *_ = mt.j2vp_return_map(ep_, epn, C, S0, M, EDOT0, 0.5)
        sm_, *_ = mt.j2vp_return_map(em_, epn, C, S0, M, EDOT0, 0.5)
        fd = (sp_ - sm_) / (2 * h)
        assert np.allclose(tan[:, :, b], fd, rtol=1e-5, atol=1e-5 * np.abs(tan).max())
    assert np.allclose(tan, np.swapaxes(tan, 1, 2), atol=1e-8 * np.abs(tan).max())


def test_j2_elastic_limit():
    C = mt.tensor4_to_mandel(mt.isotropic_tensor(*mt.lame(1000.0, 0.3)))
    eps = np.zeros((2, 6))
    eps[1, 0] = 1e-9
    sig, dp, ep, tan = mt.j2vp_return_map(eps, np.zeros((2, 6)), np.stack([C, C]), S0, M, EDOT0, 0.5)
    assert dp[0] == 0.0
    assert np.allclose(tan[0], C)
    assert dp[1] < 1e-60


def test_neohooke_reference_tangent_is_isotropic_elasticity():
    mu, lam = 1.3, 2.1
    K = mt.neohooke_tangent(np.eye(3), np.float64(mu), np.float64(lam))
    assert np.allclose(K, mt.isotropic_tensor(lam, mu), atol=1e-14)
    assert np.allclose(mt.neohooke_stress(np.eye(3), mu, lam), 0.0, atol=1e-15)


def test_neohooke_tangent_finite_difference_and_objectivity():
    rng = np.random.default_rng(13)
    F = np.eye(3) + 0.2 * rng.standard_normal((3, 3))
    mu, lam = 1.0, 7.0 / 3.0
    K = mt.neohooke_tangent(F, np.float64(mu), np.float64(lam))
    h = 1e-7
    for k in range(3):
        for L in range(3):
            Fp = F.copy(); Fp[k, L] += h
            Fm = F.copy(); Fm[k, L] -= h
            fd = (mt.neohooke_stress(Fp, mu, lam) - mt.neohooke_stress(Fm, mu, lam)) / (2 * h)
            assert np.allclose(K[:, :, k, L], fd, atol=1e-7)
    assert np.allclose(K, np.transpose(K, (2, 3, 0, 1)), atol=1e-13)
    Q = ms.random_rotations(1, 5)[0]
    assert np.allclose(mt.neohooke_stress(Q @ F, mu, lam), Q @ mt.neohooke_stress(F, mu, lam), atol=1e-13)


def _finite_laminate(mus, lams, fractions, normal, Fbar):
    """Two-phase finite-strain laminate: F_p = Fbar + a_p (x) n, traction
    continuity P_0 n = P_1 n, f_0 a_0 + f_1 a_1 = 0; Newton in a_0."""
    n = np.zeros(3); n[normal] = 1.0
    f0, f1 = fractions
    a0 = np.zeros(3)
    for _ in range(50):
        a1 = -f0 * a0 / f1
        F0 = Fbar + np.outer(a0, n)
        F1 = Fbar + np.outer(a1, n)
        P0 = mt.neohooke_stress(F0, mus[0], lams[0])
        P1 = mt.neohooke_stress(F1, mus[1], lams[1])
        g = P0 @ n - P1 @ n
        K0 = mt.neohooke_tangent(F0, np.float64(mus[0]), np.float64(lams[0]))
        K1 = mt.neohooke_tangent(F1, np.float64(mus[1]), np.float64(lams[1]))
        A0 = np.einsum("iJkL,J,L->ik", K0, n, n)
        A1 = np.einsum("iJkL,J,L->ik", K1, n, n)
        d = np.linalg.solve(A0 + A1 * f0 / f1, -g)
        a0 = a0 + d
        if np.max(np.abs(d)) < 1e-15:
            break
    a1 = -f0 * a0 / f1
    P0 = mt.neohooke_stress(Fbar + np.outer(a0, n), mus[0], lams[0])
    P1 = mt.neohooke_stress(Fbar + np.outer(a1, n), mus[1], lams[1])
    return f0 * P0 + f1 * P1


def test_newton_finite_strain_laminate():
    shape = (8, 4, 4)
    phase = ms.laminate(shape, 0, [4, 4])
    mus = np.array([1.0, 10.0])
    lams = (3.0 - 2.0 / 3.0) * mus
    law = so.NeoHookeLaw(mus[phase], lams[phase])
    Fbar = np.array([[1.08, 0.05, 0.0], [0.02, 0.97, 0.01], [0.0, -0.03, 1.02]])
    loads = [(np.eye(3) + (k + 1) / 3 * (Fbar - np.eye(3))) - np.eye(3) for k in range(3)]
    a, e, st, info = so.newton(shape, law, loads, None, kin=so.FINITE, tol=1e-12, tol_load=1e-12,
                               newton_tol=1e-12)
    assert info.converged
    expect = _finite_laminate(mus, lams, [0.5, 0.5], 0, Fbar)
    assert np.allclose(info.sigma_bar[-1], expect, rtol=0, atol=1e-10 * np.abs(expect).max())


def test_newton_finite_homogeneous_closed_form():
    shape = (4, 4, 4)
    law = so.NeoHookeLaw(np.full(shape, 1.0), np.full(shape, 7.0 / 3.0))
    Fbar = np.diag([1.1, 1.0, 1.0])
    a, e, st, info = so.newton(shape, law, [Fbar - np.eye(3)], None, kin=so.FINITE)
    assert info.pcg_iters[0] == 0
    assert np.allclose(info.sigma_bar[-1], mt.neohooke_stress(Fbar, 1.0, 7.0 / 3.0), atol=1e-14)


def test_newton_finite_stress_control_homogeneous():
    """Uniaxial nominal stress on a homogeneous cell: DBFFT equals the 0-D
    solution of P(F)_S = 0 (solved here by a dense 3-unknown Newton)."""
    shape = (4, 4, 4)
    mu, lam = 1.0, 7.0 / 3.0
    law = so.NeoHookeLaw(np.full(shape, mu), np.full(shape, lam))
    # upper triangle of F prescribed (no free rigid rotation), diagonal and
    # lower triangle of P prescribed
    mask = np.array([[0, 0, 0], [1, 1, 0], [1, 1, 1]], dtype=bool)
    L = np.zeros((3, 3)); L[0, 0] = 0.1
    a, e, st, info = so.newton(shape, law, [L], mask, kin=so.FINITE, tol=1e-12, tol_load=1e-12,
                               newton_tol=1e-13)
    assert info.converged
    # 0-D: F = diag(1.1, s, s) by symmetry, P22(s) = 0
    s = 1.0
    for _ in range(60):
        F = np.diag([1.1, s, s])
        P = mt.neohooke_stress(F, mu, lam)[1, 1]
        h = 1e-7
        dP = (mt.neohooke_stress(np.diag([1.1, s + h, s + h]), mu, lam)[1, 1]
              - mt.neohooke_stress(np.diag([1.1, s - h, s - h]), mu, lam)[1, 1]) / (2 * h)
        s -= P / dP
    expect = mt.neohooke_stress(np.diag([1.1, s, s]), mu, lam)
    assert np.allclose(info.sigma_bar[-1], expect, atol=1e-11)
    assert np.isclose(info.eps_bar[-1][1, 1], s - 1.0, atol=1e-11)


def test_newton_j2_single_grain_matches_0d_driver():
    """A homogeneous single crystal under uniaxial strain rate with the other
    stresses zero: DBFFT's Newton equals a 0-D Newton on the five free strain
    components using the return map directly."""
    shape = (4, 4, 4)
    R = ms.random_rotations(1, 21)
    C = mt.tensor4_to_mandel(mt.rotate_tensor4(mt.cubic_tensor(168000.0, 121000.0, 75000.0), R))[0]
    Cf = np.broadcast_to(C, shape + (6, 6))
    dt = 0.5
    law = so.J2Law(Cf, S0, M, EDOT0, dt)
    mask = np.ones((3, 3), bool)
    mask[0, 0] = False
    nincr = 6
    loads = []
    for k in range(1, nincr + 1):
        L = np.zeros((3, 3)); L[0, 0] = 1e-3 * dt * k
        loads.append(L)
    a, e, st, info = so.newton(shape, law, loads, mask, tol=1e-12, tol_load=1e-12, newton_tol=1e-12)
    assert info.converged
    # 0-D driver: Mandel strain (e11 fixed, 5 free), stresses 1..5 zero.
    epn = np.zeros((1, 6))
    free = [1, 2, 3, 4, 5]
    ev = np.zeros(6)
    for k in range(1, nincr + 1):
        ev[0] = 1e-3 * dt * k
        for _ in range(60):
            sig, dp, ep, tan = mt.j2vp_return_map(ev[None], epn, C[None], S0, M, EDOT0, dt)
            res = sig[0][free]
            d = np.linalg.solve(tan[0][np.ix_(free, free)], -res)
            ev[free] += d
            if np.max(np.abs(d)) < 1e-15:
                break
        sig, dp, ep, tan = mt.j2vp_return_map(ev[None], epn, C[None], S0, M, EDOT0, dt)
        epn = ep
        s33 = mt.mandel_to_sym(sig[0])
        assert np.allclose(info.sigma_bar[k - 1], s33, rtol=0, atol=1e-8)


def test_adjoint_homogeneous_closed_form():
    """dC1111/dE(x) = (lam1 + 2 mu1)/N everywhere for a homogeneous cell."""
    shape = (4, 4, 4)
    N = 64
    nu = 0.3
    E = np.full(shape, 2.0)
    tan = so.IsoTangent(*mt.lame(E, nu))
    dtan = so.IsoTangent(*mt.lame(np.ones(shape), nu))
    G = np.zeros((3, 3)); G[0, 0] = 1.0
    J, g, fwd, adj = so.adjoint_gradient(shape, tan, dtan, G, None, G, np.zeros((3, 3)))
    lam1, mu1 = mt.lame(1.0, nu)
    assert np.isclose(J, 2.0 * (lam1 + 2 * mu1), rtol=1e-13)
    assert np.allclose(g, (lam1 + 2 * mu1) / N, rtol=1e-12)


@pytest.mark.parametrize("objective", ["c1111", "compliance", "mixed"])
def test_adjoint_finite_differences(objective):
    shape = (6, 6, 6)
    rng = np.random.default_rng(14)
    E = np.exp(0.8 * rng.standard_normal(shape))
    nu = 0.3
    G = np.zeros((3, 3)); H = np.zeros((3, 3))
    mask = np.zeros((3, 3), bool)
    load = np.zeros((3, 3))
    if objective == "c1111":
        load[0, 0] = 1.0; G[0, 0] = 1.0
    elif objective == "compliance":
        mask[:] = True; load[0, 0] = 1.0; H[0, 0] = 1.0
    else:
        mask[:] = True; mask[0, 0] = False
        load[0, 0] = 1.0; load[1, 2] = load[2, 1] = 0.3
        G[0, 0] = 1.0; G[1, 1] = 0.4; H[1, 2] = H[2, 1] = 0.7; H[0, 0] = 0.2

    def J_of(Ef):
        tan = so.IsoTangent(*mt.lame(Ef, nu))
        r = so.solve_linear(shape, tan, load, mask, tol=1e-13, tol_load=1e-13)
        return float(np.sum(G * r.sigma_bar) + np.sum(H * r.eps_bar))

    tan = so.IsoTangent(*mt.lame(E, nu))
    dtan = so.IsoTangent(*mt.lame(np.ones(shape), nu))
    J, g, fwd, adj = so.adjoint_gradient(shape, tan, dtan, load, mask, G, H, tol=1e-13)
    assert np.isclose(J, J_of(E), rtol=1e-11)
    for idx in [(0, 0, 0), (2, 3, 1), (5, 1, 4)]:
        h = 1e-4 * E[idx]
        Ep = E.copy(); Ep[idx] += h
        Em = E.copy(); Em[idx] -= h
        fd = (J_of(Ep) - J_of(Em)) / (2 * h)
        assert np.isclose(g[idx], fd, rtol=1e-6, atol=1e-9 * abs(J))


# --------------------------------------------------------------------------
# Saint Venant-Kirchhoff (Sec. 3.3)
# --------------------------------------------------------------------------

def test_svk_reference_tangent_is_isotropic_elasticity():
    mu, lam = 1.3, 2.1
    K = mt.svk_tangent(np.eye(3), np.float64(mu), np.float64(lam))
    assert np.allclose(K, mt.isotropic_tensor(lam, mu), atol=1e-14)
    assert np.allclose(mt.svk_stress(np.eye(3), mu, lam), 0.0, atol=1e-15)


def test_svk_uniaxial_stretch_closed_form():
    """F = diag(a, 1, 1): E11 = (a^2 - 1)/2, S11 = (lam + 2 mu) E11,
    S22 = S33 = lam E11, P = F S (worked by hand)."""
    mu, lam, a = 26.9, 40.4, 2.0
    e11 = 0.5 * (a * a - 1.0)
    expect = np.diag([a * (lam + 2 * mu) * e11, lam * e11, lam * e11])
    assert np.allclose(mt.svk_stress(np.diag([a, 1.0, 1.0]), mu, lam), expect, rtol=1e-15, atol=0)


def test_svk_tangent_finite_difference_symmetry_and_objectivity():
    rng = np.random.default_rng(17)
    F = np.eye(3) + 0.3 * rng.standard_normal((3, 3))
    mu, lam = 1.0, 1.5
    K = mt.svk_tangent(F, np.float64(mu), np.float64(lam))
    h = 1e-6
    for k in range(3):
        for L in range(3):
            Fp = F.copy(); Fp[k, L] += h
            Fm = F.copy(); Fm[k, L] -= h
            fd = (mt.svk_stress(Fp, mu, lam) - mt.svk_stress(Fm, mu, lam)) / (2 * h)
            assert np.allclose(K[:, :, k, L], fd, atol=1e-8)
    # hyperelastic: major symmetry of dP/dF
    assert np.allclose(K, np.transpose(K, (2, 3, 0, 1)), atol=1e-13)
    Q = ms.random_rotations(1, 8)[0]
    assert np.allclose(mt.svk_stress(Q @ F, mu, lam), Q @ mt.svk_stress(F, mu, lam), atol=1e-13)


def _finite_laminate_law(stress, tangent, mus, lams, fractions, normal, Fbar):
    """Two-phase finite-strain laminate for any law: F_p = Fbar + a_p (x) n,
    traction continuity P_0 n = P_1 n, f_0 a_0 + f_1 a_1 = 0; Newton in a_0."""
    n = np.zeros(3); n[normal] = 1.0
    f0, f1 = fractions
    a0 = np.zeros(3)
    for _ in range(50):
        a1 = -f0 * a0 / f1
        F0 = Fbar + np.outer(a0, n)
        F1 = Fbar + np.outer(a1, n)
        g = stress(F0, mus[0], lams[0]) @ n - stress(F1, mus[1], lams[1]) @ n
        A0 = np.einsum("iJkL,J,L->ik", tangent(F0, np.float64(mus[0]), np.float64(lams[0])), n, n)
        A1 = np.einsum("iJkL,J,L->ik", tangent(F1, np.float64(mus[1]), np.float64(lams[1])), n, n)
        d = np.linalg.solve(A0 + A1 * f0 / f1, -g)
        a0 = a0 + d
        if np.max(np.abs(d)) < 1e-15:
            break
    a1 = -f0 * a0 / f1
    return f0 * stress(Fbar + np.outer(a0, n), mus[0], lams[0]) + f1 * stress(Fbar + np.outer(a1, n), mus[1], lams[1])


def test_newton_svk_laminate():
    shape = (8, 4, 4)
    phase = ms.laminate(shape, 0, [4, 4])
    lam0, mu0 = mt.lame(np.array([70.0, 0.7]), 0.3)
    law = so.SVKLaw(mu0[phase], lam0[phase])
    Fbar = np.array([[1.2, 0.05, 0.0], [0.02, 0.97, 0.01], [0.0, -0.03, 1.02]])
    loads = [(np.eye(3) + (k + 1) / 4 * (Fbar - np.eye(3))) - np.eye(3) for k in range(4)]
    a, e, st, info = so.newton(shape, law, loads, None, kin=so.FINITE, tol=1e-12, tol_load=1e-12,
                               newton_tol=1e-12)
    assert info.converged
    expect = _finite_laminate_law(mt.svk_stress, mt.svk_tangent, mu0, lam0, [0.5, 0.5], 0, Fbar)
    assert np.allclose(info.sigma_bar[-1], expect, rtol=0, atol=1e-10 * np.abs(expect).max())


def test_newton_svk_homogeneous_closed_form():
    shape = (4, 5, 3)
    lam, mu = mt.lame(70.0, 0.3)
    law = so.SVKLaw(np.full(shape, mu), np.full(shape, lam))
    Fbar = np.diag([1.4, 1.0, 1.0])
    a, e, st, info = so.newton(shape, law, [Fbar - np.eye(3)], None, kin=so.FINITE)
    assert info.pcg_iters[0] == 0
    e11 = 0.5 * (1.4 ** 2 - 1.0)
    expect = np.diag([1.4 * (lam + 2 * mu) * e11, lam * e11, lam * e11])
    assert np.allclose(info.sigma_bar[-1], expect, rtol=1e-14, atol=0)


# --------------------------------------------------------------------------
# Hyperelastic adjoint (finite strains)
# --------------------------------------------------------------------------

def _hyper_law(kind, mu, lam):
    return (so.SVKLaw if kind == "svk" else so.NeoHookeLaw)(mu, lam)


@pytest.mark.parametrize("kind", ["svk", "neohooke"])
def test_hyperelastic_adjoint_homogeneous_closed_form(kind):
    """A homogeneous cell deforms uniformly, so the adjoint field has no
    fluctuation and dJ/dtheta(x) = G:P / N at every voxel."""
    shape = (4, 4, 4)
    mu = np.full(shape, 1.3)
    lam = np.full(shape, 2.0)
    Fm = np.array([[1.2, 0.1, 0.0], [0.0, 0.95, 0.05], [0.02, 0.0, 1.05]])
    G = np.zeros((3, 3)); G[0, 0] = 1.0; G[0, 1] = 0.5
    J, g, info = so.adjoint_gradient_hyperelastic(shape, _hyper_law(kind, mu, lam), [Fm - np.eye(3)], None,
                                                  G, np.zeros((3, 3)))
    if kind == "svk":
        P = mt.svk_stress(Fm, np.float64(1.3), np.float64(2.0))
    else:
        P = mt.neohooke_stress(Fm, np.float64(1.3), np.float64(2.0))
    assert np.isclose(J, float(np.sum(G * P)), rtol=1e-12)
    assert np.allclose(g, np.sum(G * P) / 64, rtol=1e-10, atol=0)


@pytest.mark.parametrize("kind,control", [("svk", "strain"), ("neohooke", "strain"), ("svk", "mixed"),
                                          ("neohooke", "mixed")])
def test_hyperelastic_adjoint_finite_differences(kind, control):
    """Gradient with respect to a per-voxel factor on both moduli against
    central differences of full Newton solves."""
    shape = (5, 4, 4)
    rng = np.random.default_rng(21 if kind == "svk" else 22)
    mu = np.exp(0.7 * rng.standard_normal(shape))
    lam = 1.5 * mu
    G = np.zeros((3, 3)); H = np.zeros((3, 3)); mask = None
    if control == "strain":
        loads = [np.diag([0.15, 0.0, -0.05]) * (k + 1) / 2 for k in range(2)]
        loads = [L + np.array([[0, 0.05, 0], [0, 0, 0], [0, 0, 0]]) * (k + 1) / 2 for k, L in enumerate(loads)]
        G[0, 0] = 1.0; G[0, 1] = 0.3; G[2, 2] = -0.4
    else:
        mask = np.array([[0, 0, 0], [1, 1, 0], [1, 1, 1]], dtype=bool)
        loads = [np.diag([0.2 * (k + 1) / 2, 0.0, 0.0]) for k in range(2)]
        G[0, 0] = 1.0; G[1, 2] = 0.5; H[1, 1] = 0.7; H[2, 0] = -0.3

    def J_of(th):
        law = _hyper_law(kind, mu * th, lam * th)
        _, _, _, inf = so.newton(shape, law, loads, mask, kin=so.FINITE, tol=1e-13, tol_load=1e-13,
                                 newton_tol=1e-13)
        assert inf.converged
        return float(np.sum(G * inf.sigma_bar[-1]) + np.sum(H * (inf.eps_bar[-1] + np.eye(3))))

    J, g, info = so.adjoint_gradient_hyperelastic(shape, _hyper_law(kind, mu, lam), loads, mask, G, H,
                                                  tol=1e-13, newton_tol=1e-13)
    assert info.converged
    assert np.isclose(J, J_of(np.ones(shape)), rtol=1e-11)
    for idx in [(0, 0, 0), (3, 2, 1)]:
        h = 1e-4
        tp = np.ones(shape); tp[idx] += h
        tm = np.ones(shape); tm[idx] -= h
        fd = (J_of(tp) - J_of(tm)) / (2 * h)
        assert np.isclose(g[idx], fd, rtol=1e-6, atol=1e-9 * abs(J)), (idx, g[idx], fd)


# --------------------------------------------------------------------------
# J2 adjoint through the load path
# --------------------------------------------------------------------------

def _j2_case(control, shape=(4, 4, 3), ngrain=3, ninc=5):
    grain, _ = ms.voronoi_grains(shape, ngrain, 41)
    R = ms.random_rotations(ngrain, 42)
    C = mt.tensor4_to_mandel(mt.rotate_tensor4(mt.cubic_tensor(168000.0, 121000.0, 75000.0), R))[grain]
    dt = 0.5
    G = np.zeros((3, 3)); H = np.zeros((3, 3))
    if control == "mixed":
        mask = np.ones((3, 3), bool); mask[0, 0] = False
        final = np.zeros((3, 3)); final[0, 0] = 1e-3 * dt * ninc
        G[0, 0] = 1.0; H[1, 1] = 3e4; H[0, 1] = H[1, 0] = -2e4
    else:
        mask = None
        final = np.zeros((3, 3)); final[0, 0] = 1e-3 * dt * ninc; final[1, 2] = final[2, 1] = 4e-4 * dt * ninc
        G[0, 0] = 1.0; G[1, 2] = G[2, 1] = 0.5; G[2, 2] = -0.3
    loads = [final * (k + 1) / ninc for k in range(ninc)]
    return C, dt, mask, loads, G, H


def _j2_J(shape, C, s0, dt, loads, mask, G, H):
    law = so.J2Law(C, s0, M, EDOT0, dt)
    _, _, _, inf = so.newton(shape, law, loads, mask, tol=1e-13, tol_load=1e-13, newton_tol=1e-13)
    assert inf.converged
    return float(np.sum(G * inf.sigma_bar[-1]) + np.sum(H * inf.eps_bar[-1]))


@pytest.mark.parametrize("control", ["mixed", "strain"])
def test_j2_path_adjoint_finite_differences(control):
    """Gradient with respect to a per-voxel factor on s0 against central
    differences of the whole incremental Newton solve (the response depends
    on the path: plastic strain carries over between increments)."""
    shape = (4, 4, 3)
    C, dt, mask, loads, G, H = _j2_case(control, shape)
    J, g, info = so.adjoint_gradient_j2(shape, so.J2Law(C, S0, M, EDOT0, dt), loads, mask, G, H, tol=1e-13,
                                        newton_tol=1e-13)
    assert info.converged
    assert np.isclose(J, _j2_J(shape, C, S0, dt, loads, mask, G, H), rtol=1e-11)
    h = 1e-4
    for idx in [(0, 0, 0), (2, 1, 2), (3, 3, 1)]:
        tp = np.full(shape, S0); tp[idx] *= 1 + h
        tm = np.full(shape, S0); tm[idx] *= 1 - h
        fd = (_j2_J(shape, C, tp, dt, loads, mask, G, H) - _j2_J(shape, C, tm, dt, loads, mask, G, H)) / (2 * h)
        assert np.isclose(g[idx], fd, rtol=1e-5, atol=1e-7 * abs(J)), (idx, g[idx], fd)


def test_j2_path_adjoint_sum_is_uniform_scaling():
    """Summed over the voxels the gradient is the derivative with respect to
    one factor on s0 everywhere."""
    shape = (4, 4, 3)
    C, dt, mask, loads, G, H = _j2_case("mixed", shape)
    J, g, _ = so.adjoint_gradient_j2(shape, so.J2Law(C, S0, M, EDOT0, dt), loads, mask, G, H, tol=1e-13,
                                     newton_tol=1e-13)
    h = 1e-4
    fd = (_j2_J(shape, C, S0 * (1 + h), dt, loads, mask, G, H) -
          _j2_J(shape, C, S0 * (1 - h), dt, loads, mask, G, H)) / (2 * h)
    assert np.isclose(np.sum(g), fd, rtol=1e-6)


def test_j2_path_adjoint_single_increment_single_crystal():
    """One grain, one increment: the cell deforms uniformly, so the gradient
    is uniform and equals the 0-D material point's derivative over N."""
    shape = (3, 3, 3)
    R = ms.random_rotations(1, 43)
    C1 = mt.tensor4_to_mandel(mt.rotate_tensor4(mt.cubic_tensor(168000.0, 121000.0, 75000.0), R))[0]
    C = np.broadcast_to(C1, shape + (6, 6))
    dt = 2.0
    ev = np.array([2e-3, -5e-4, 3e-4, 1e-3, 0.0, 7e-4])
    E = mt.mandel_to_sym(ev)
    G = np.array([[1.0, 0.2, 0.0], [0.2, 0.0, 0.0], [0.0, 0.0, 0.5]])
    J, g, _ = so.adjoint_gradient_j2(shape, so.J2Law(C, S0, M, EDOT0, dt), [E], None, G, np.zeros((3, 3)))

    def point(s0):
        sig, _, _, _ = mt.j2vp_return_map(ev[None], np.zeros((1, 6)), C1[None], s0, M, EDOT0, dt)
        return float(np.sum(G * mt.mandel_to_sym(sig[0])))

    h = 1e-5
    d = (point(S0 * (1 + h)) - point(S0 * (1 - h))) / (2 * h)
    assert np.isclose(J, point(S0), rtol=1e-12)
    assert np.allclose(g, d / 27, rtol=1e-7)
