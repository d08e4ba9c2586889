"""Pins of the oracle's error estimates of Sec. 3 (eqs. chedckeq,
chedckcomp, chedckimp and their finite-strain forms of Sec. 3.3) against
closed forms of trigonometric fields, the FFT-free differentiation matrices,
vanishing on compatible and equilibrated fields, and the operator route."""
import numpy as np

from oracle import dense, post, solver as so, materials as mt
from paper_1905_12725_amd import microstructure as ms

TWO_PI = 2.0 * np.pi


def coords(shape):
    return np.meshgrid(*[np.arange(n) / n for n in shape], indexing="ij")


def test_incompatibility_of_a_normal_strain_wave():
    """eps_11 = c0 + a cos(2 pi x2): the only incompatibility is
    eta_33 = d2 d2 eps_11 = -(2 pi)^2 a cos(2 pi x2)."""
    shape = (6, 8, 5)
    x = coords(shape)
    c0, a = 2e-3, 3e-4
    eps = np.zeros((3, 3) + shape)
    eps[0, 0] = c0 + a * np.cos(TWO_PI * x[1])
    inc = post.incompatibility(eps, shape)
    expect = np.zeros_like(inc)
    expect[2, 2] = -TWO_PI ** 2 * a * np.cos(TWO_PI * x[1])
    assert np.max(np.abs(inc - expect)) < 1e-12 * TWO_PI ** 2 * a
    assert np.isclose(post.compatibility_residual(eps, shape), TWO_PI ** 2 * a / c0, rtol=1e-12)


def test_incompatibility_of_a_shear_strain_wave():
    """eps_23 = eps_32 = a sin(2 pi x1): eta_23 = eta_32 = +(2 pi)^2 a sin(2 pi x1)
    (the sign fixes the orientation of both Levi-Civita contractions)."""
    shape = (8, 5, 6)
    x = coords(shape)
    a = 1e-3
    eps = np.zeros((3, 3) + shape)
    eps[1, 2] = eps[2, 1] = a * np.sin(TWO_PI * x[0])
    eps[0, 0] = 1e-3
    inc = post.incompatibility(eps, shape)
    expect = np.zeros_like(inc)
    expect[1, 2] = expect[2, 1] = TWO_PI ** 2 * a * np.sin(TWO_PI * x[0])
    assert np.max(np.abs(inc - expect)) < 1e-12 * TWO_PI ** 2 * a


def test_incompatibility_matches_differentiation_matrices():
    """A random symmetric field: the spectral route equals the dense
    Trefethen differentiation matrices (no FFT involved), odd and even axes."""
    shape = (4, 5, 6)
    rng = np.random.default_rng(11)
    t = rng.standard_normal((3, 3) + shape)
    eps = 0.5 * (t + np.swapaxes(t, 0, 1))
    D = dense.partial_matrices(shape)
    e = post.levi_civita()

    def d2(f, k, m):
        return (D[k] @ (D[m] @ f.reshape(-1))).reshape(shape)

    ref = np.zeros((3, 3) + shape)
    for i in range(3):
        for j in range(3):
            for k in range(3):
                for l in range(3):
                    for m in range(3):
                        for n in range(3):
                            c = e[i, k, l] * e[j, m, n]
                            if c:
                                ref[i, j] += c * d2(eps[l, n], k, m)
    inc = post.incompatibility(eps, shape)
    assert np.max(np.abs(inc - ref)) < 1e-10 * np.max(np.abs(ref))


def test_compatible_fields_have_no_incompatibility():
    """sym grad u and grad u of a random displacement (dense matrices)."""
    shape = (5, 6, 4)
    rng = np.random.default_rng(12)
    u = rng.standard_normal((3,) + shape)
    D = dense.partial_matrices(shape)
    G = np.stack([np.stack([(D[j] @ u[i].reshape(-1)).reshape(shape) for j in range(3)]) for i in range(3)])
    G[0, 0] += 1e-2  # a uniform part keeps the denominator away from zero
    eps = 0.5 * (G + np.swapaxes(G, 0, 1))
    scale = np.max(np.abs(G)) * (TWO_PI * 3) ** 2
    assert np.max(np.abs(post.incompatibility(eps, shape))) < 1e-11 * scale
    assert np.max(np.abs(post.row_curl(G, shape))) < 1e-11 * np.max(np.abs(G)) * TWO_PI * 3


def test_row_curl_of_a_wave():
    """H_11 = a cos(2 pi x2): (curl_0 H)_13 = -d2 H_11 = 2 pi a sin(2 pi x2)."""
    shape = (5, 8, 6)
    x = coords(shape)
    a = 0.05
    H = np.zeros((3, 3) + shape)
    H[0, 0] = a * np.cos(TWO_PI * x[1])
    H[1, 1] = 0.1
    c = post.row_curl(H, shape)
    expect = np.zeros_like(c)
    expect[0, 2] = TWO_PI * a * np.sin(TWO_PI * x[1])
    assert np.max(np.abs(c - expect)) < 1e-12 * TWO_PI * a
    assert np.isclose(post.compatibility_residual(H, shape, finite=True), TWO_PI * a / 0.1, rtol=1e-12)


def test_equilibrium_residual_of_a_shear_wave():
    """sigma_12 = sigma_21 = s + a sin(2 pi x1): div sigma = (0, 2 pi a cos(2 pi x1), 0),
    whose root mean square is 2 pi a / sqrt 2."""
    shape = (7, 4, 6)
    x = coords(shape)
    s, a = 3.0, 0.2
    sig = np.zeros((3, 3) + shape)
    sig[0, 1] = sig[1, 0] = s + a * np.sin(TWO_PI * x[0])
    sig[2, 2] = 1.0
    d = post.divergence(sig, shape)
    assert np.max(np.abs(d[0])) < 1e-12 and np.max(np.abs(d[2])) < 1e-12
    assert np.max(np.abs(d[1] - TWO_PI * a * np.cos(TWO_PI * x[0]))) < 1e-12
    expect = TWO_PI * a / np.sqrt(2.0) / np.sqrt(2 * s * s + 1.0)
    assert np.isclose(post.equilibrium_residual(sig, shape), expect, rtol=1e-12)


def test_equilibrium_residual_matches_the_operator_route():
    """The stress of a PCG iterate stopped early: the real-space divergence
    route equals the Fourier residual of the solver (Parseval)."""
    n = (8, 6, 7)
    phase = ms.centred_sphere(n, 0.25)
    lam, mu = mt.lame(np.asarray([1.0, 20.0])[phase], 0.3)
    tan = so.IsoTangent(lam, mu)
    L = np.zeros((3, 3)); L[0, 0] = 1e-3; L[1, 2] = L[2, 1] = 4e-4
    res = so.solve_linear(n, tan, L, tol=1e-3)
    eq_true, _ = so.true_residual(res.space, tan, res, L)
    sig = tan.stress(res.strain_field())
    eq = post.equilibrium_residual(sig, n)
    assert 1e-6 < eq < 1e-2
    assert np.isclose(eq, eq_true, rtol=1e-10)


def test_dbfft_solution_is_compatible_and_meets_its_load():
    """Mixed control: the solved strain is compatible, its average meets the
    prescribed strain components and the stress average the prescribed ones."""
    n = (6, 8, 5)
    phase = ms.centred_sphere(n, 0.25)
    lam, mu = mt.lame(np.asarray([1.0, 8.0])[phase], 0.3)
    tan = so.IsoTangent(lam, mu)
    mask = np.ones((3, 3), bool); mask[0, 0] = False
    L = np.zeros((3, 3)); L[0, 0] = 1e-3; L[1, 1] = 0.02
    res = so.solve_linear(n, tan, L, mask, tol=1e-12, tol_load=1e-12)
    eps = res.strain_field()
    sig = tan.stress(eps)
    assert post.compatibility_residual(eps, n) < 1e-10
    assert post.equilibrium_residual(sig, n) < 1e-11
    e_part, s_part = post.loading_residuals(eps.reshape(3, 3, -1).mean(axis=2), sig.reshape(3, 3, -1).mean(axis=2),
                                            L, mask)
    assert e_part < 1e-13 and s_part < 1e-11
    # a wrong prescribed stress is seen
    L2 = L.copy(); L2[1, 1] = 0.03
    _, bad = post.loading_residuals(eps.reshape(3, 3, -1).mean(axis=2), sig.reshape(3, 3, -1).mean(axis=2), L2, mask)
    assert bad > 0.1


def test_loading_residuals_finite_strain_reference():
    """At finite strains the strain part compares I + <H> with Fbar,
    relative to Fbar - I on the prescribed components."""
    Fbar = np.diag([1.2, 1.0, 1.0])
    H = np.diag([0.2 + 2e-4, 0.0, 0.0])
    e_part, s_part = post.loading_residuals(H, np.zeros((3, 3)), Fbar, np.zeros((3, 3), bool), finite=True)
    assert np.isclose(e_part, 2e-4 / 0.2, rtol=1e-9)
    assert s_part == 0.0
