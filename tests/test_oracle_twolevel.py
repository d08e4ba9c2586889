"""Pins of the oracle's two-level preconditioner (exact operator block on the
coarse Fourier set, M(xi) of Sec. 2.5 eqs. pred2/pred3 elsewhere): its
coarse basis is orthonormal, it reduces to M(xi) for a homogeneous cell, it
is the exact inverse when the coarse set is the whole spectrum (one PCG
iteration), and it is symmetric positive definite."""
import numpy as np
import pytest

from oracle import spectral as sp, solver as so, materials as mt
from paper_1905_12725_amd import microstructure as ms


def random_vector(space, seed):
    rng = np.random.default_rng(seed)
    a = sp.fourier(rng.standard_normal((3,) + space.shape), space.shape)
    a[:, space.Z] = 0.0
    return (a, rng.standard_normal(len(space.S)))


def two_phase(n, seed, contrast=20.0):
    rng = np.random.default_rng(seed)
    phase = (rng.random(n) < 0.35).astype(np.uint8)
    lam, mu = mt.lame(np.where(phase == 1, contrast, 1.0), 0.3)
    return so.IsoTangent(lam, mu)


def test_coarse_basis_is_orthonormal():
    space = so.Space((6, 5, 8))
    M = so.TwoLevelPreconditioner(space, two_phase(space.shape, 1), 1)
    for j in range(M.m):
        e = np.zeros(M.m)
        e[j] = 1.0
        b = M.basis(j)
        assert np.allclose(M.coords(b), e, atol=1e-14)
        assert abs(space.dot((b, np.zeros(0)), (b, np.zeros(0))) - 1.0) < 1e-14


def test_homogeneous_cell_gives_the_single_level_preconditioner():
    n = (8, 8, 8)
    lam, mu = mt.lame(np.full(n, 3.0), 0.25)
    tan = so.IsoTangent(lam, mu)
    space = so.Space(n, stress_mask=np.diag([False, True, True]))
    M2 = so.TwoLevelPreconditioner(space, tan, 2)
    M0 = space.preconditioner(tan.mean())
    r = random_vector(space, 3)
    a2, e2 = M2(r)
    a0, e0 = M0(r)
    assert np.allclose(a2, a0, rtol=0, atol=1e-13 * np.abs(a0).max())
    assert np.allclose(e2, e0)


def test_whole_spectrum_coarse_set_is_exact():
    """On 4^3 with kc = 2 every nonzero frequency is coarse, so M is K^-1 on
    the field unknowns and PCG under strain control stops after one step."""
    n = (4, 4, 4)
    tan = two_phase(n, 7, 50.0)
    L = np.array([[1e-3, 2e-4, 0], [2e-4, -3e-4, 1e-4], [0, 1e-4, 5e-4]])
    r = so.solve_linear(n, tan, L, tol=1e-12, tol_load=1e-12, coarse_kc=2)
    assert r.info.converged and r.info.iterations == 1
    ref = so.solve_linear(n, tan, L, tol=1e-13, tol_load=1e-13)
    assert np.allclose(r.sigma_bar, ref.sigma_bar, rtol=0, atol=1e-11 * np.abs(ref.sigma_bar).max())


def test_two_level_is_symmetric_positive_definite():
    n = (8, 6, 8)
    space = so.Space(n, stress_mask=np.diag([False, True, False]))
    M = so.TwoLevelPreconditioner(space, two_phase(n, 5), 1)
    u, v = random_vector(space, 11), random_vector(space, 12)
    Mu, Mv = M(u), M(v)
    assert abs(space.dot(u, Mv) - space.dot(Mu, v)) < 1e-12 * abs(space.dot(u, Mv))
    for seed in range(3):
        w = random_vector(space, 20 + seed)
        assert space.dot(w, M(w)) > 0.0


@pytest.mark.parametrize("kc", [1, 2])
def test_two_level_solution_matches(kc):
    n = (12, 12, 12)
    phase = ms.centred_sphere(n, 0.2)
    lam, mu = mt.lame(np.where(phase == 1, 100.0, 1.0), 0.3)
    tan = so.IsoTangent(lam, mu)
    L = np.zeros((3, 3)); L[0, 0] = 1e-3
    r2 = so.solve_linear(n, tan, L, tol=1e-11, tol_load=1e-11, coarse_kc=kc)
    r0 = so.solve_linear(n, tan, L, tol=1e-11, tol_load=1e-11)
    assert r2.info.converged
    assert np.allclose(r2.sigma_bar, r0.sigma_bar, rtol=0, atol=1e-9 * np.abs(r0.sigma_bar).max())
