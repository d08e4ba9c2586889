"""Pins of the oracle's block PCG (several loads of one cell in one block
Krylov space; Sec. 3 CG with the Sec. 2.5 preconditioner, directions taken
in blocks): one load reproduces the single-vector PCG, every load of a block
solve equals the FFT-free dense direct solve, dependent loads give
proportional solutions, and the block iteration count is bounded by the
single-vector counts."""
import numpy as np
import pytest

from oracle import dense, spectral as sp, solver as so, materials as mt
from paper_1905_12725_amd import microstructure as ms


def iso_phase_tangent(phase, E, nu):
    lam, mu = mt.lame(np.asarray(E)[phase], nu)
    return so.IsoTangent(lam, mu)


def mandel_loads(scale=1e-3):
    out = []
    for i, j in [(0, 0), (1, 1), (2, 2), (1, 2), (0, 2), (0, 1)]:
        L = np.zeros((3, 3))
        L[i, j] = L[j, i] = scale
        out.append(L)
    return out


def test_single_load_block_is_pcg():
    """With one load the block iteration is the PCG iteration (the direction
    is only rescaled): same iteration count, same solution."""
    n = (8, 8, 8)
    rng = np.random.default_rng(3)
    phase = (rng.random(n) < 0.3).astype(np.uint8)
    tan = iso_phase_tangent(phase, [1.0, 20.0], 0.3)
    L = np.array([[1e-3, 2e-4, 0], [2e-4, -3e-4, 1e-4], [0, 1e-4, 5e-4]])
    ref = so.solve_linear(n, tan, L, tol=1e-10, tol_load=1e-10)
    (res,), info = so.solve_linear_block(n, tan, [L], tol=1e-10, tol_load=1e-10)
    assert info.converged and info.iterations == ref.info.iterations
    assert info.applies == info.iterations
    assert np.allclose(res.a, ref.a, rtol=0, atol=1e-10 * np.abs(ref.a).max())
    assert np.allclose(res.sigma_bar, ref.sigma_bar, rtol=0, atol=1e-12 * np.abs(ref.sigma_bar).max())


@pytest.mark.parametrize("mask_comps", [[], [(1, 1), (2, 2)], [(0, 1)]])
def test_block_matches_dense_direct_solve(mask_comps):
    """Every load of a block solve against the dense assembled solve on 6^3
    at tol 1e-11 (on 4^3 the six loads span the 193 unknowns within ~32
    block iterations, and driven to tol 1e-13 there the finite-precision
    block recurrence loses conjugacy, as block CG does once its Krylov
    space is exhausted)."""
    n = (6, 6, 6)
    rng = np.random.default_rng(11)
    phase = (rng.random(n) < 0.4).astype(np.uint8)
    E, nu = [1.0, 8.0], 0.3
    tan = iso_phase_tangent(phase, E, nu)
    mask = np.zeros((3, 3), bool)
    for (i, j) in mask_comps:
        mask[i, j] = mask[j, i] = True
    loads = [L * (1.0 - mask) + 2e-3 * mask * (k + 1) for k, L in enumerate(mandel_loads())]
    res, info = so.solve_linear_block(n, tan, loads, mask, tol=1e-11, tol_load=1e-11)
    assert info.converged
    Cm = np.stack([mt.tensor4_to_mandel(mt.isotropic_tensor(*mt.lame(E[p], nu))) for p in phase.reshape(-1)])
    for L, r in zip(loads, res):
        u_d, e_d, sig_d = dense.solve(n, Cm, L, mask)
        assert np.allclose(r.sigma_bar, sig_d, rtol=0, atol=1e-10 * np.abs(sig_d).max())
        u_f = sp.real_field(r.a, n)
        u_d = u_d - u_d.mean(axis=(1, 2, 3), keepdims=True)
        assert np.allclose(u_f, u_d, atol=1e-8 * np.abs(u_d).max())


def test_dependent_loads_drop_a_direction():
    """Loads L, 2 L and L' span two directions: the first block has width 2
    and the solutions of L and 2 L are proportional."""
    n = (8, 8, 8)
    rng = np.random.default_rng(5)
    phase = (rng.random(n) < 0.3).astype(np.uint8)
    tan = iso_phase_tangent(phase, [1.0, 10.0], 0.3)
    L1 = mandel_loads()[0]
    L2 = mandel_loads()[5]
    res, info = so.solve_linear_block(n, tan, [L1, 2.0 * L1, L2], tol=1e-11, tol_load=1e-11)
    assert info.converged
    assert info.applies <= 2 * info.iterations
    assert np.allclose(res[1].a, 2.0 * res[0].a, rtol=0, atol=1e-10 * np.abs(res[1].a).max())
    ref = so.solve_linear(n, tan, L2, tol=1e-12, tol_load=1e-12)
    assert np.allclose(res[2].sigma_bar, ref.sigma_bar, rtol=0, atol=1e-10 * np.abs(ref.sigma_bar).max())


def test_block_iterations_bounded_by_single():
    """Each column's error is minimized over a space that contains its own
    Krylov space, so the block needs no more iterations than the slowest
    single-vector solve (one more allowed for the residual-based stop)."""
    n = (12, 12, 12)
    phase, _, _ = ms.random_spheres(n, 2, 1.0, 2.0, 0.3)
    tan = iso_phase_tangent(phase, [1.0, 100.0], 0.3)
    loads = mandel_loads()
    res, info = so.solve_linear_block(n, tan, loads, tol=1e-8, tol_load=1e-10)
    single = [so.solve_linear(n, tan, L, tol=1e-8, tol_load=1e-10).info.iterations for L in loads]
    assert info.converged
    assert info.iterations <= max(single) + 1, (info.iterations, single)
    assert max(info.col_iterations) == info.iterations
