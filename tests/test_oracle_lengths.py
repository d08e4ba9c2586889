"""Pins of the cell side lengths L_i of Sec. 2.1 (frequencies 2 pi m_i / L_i)
in the oracle: the periodic medium of a cell repeated along an axis, the
FFT-free dense solve with the same lengths, and a common scale."""
import numpy as np

from oracle import dense, solver as so, materials as mt, spectral as sp


def iso(phase, E, nu=0.3):
    lam, mu = mt.lame(np.asarray(E)[phase], nu)
    return so.IsoTangent(lam, mu)


LOAD = np.array([[1e-3, 2e-4, -1e-4], [2e-4, -3e-4, 4e-4], [-1e-4, 4e-4, 5e-4]])


def test_axis_frequencies_scale_with_length():
    assert np.allclose(sp.axis_xi(6, 2.5), sp.axis_xi(6) / 2.5)
    assert np.allclose(sp.xi_half((4, 6, 8), (2.0, 0.5, 4.0))[1], sp.xi_half((4, 6, 8))[1] / 0.5)


def test_repeated_cell_is_the_same_medium():
    """A 6^3 cell and the same cell twice along x (12 x 6 x 6 over 2 x 1 x 1)
    describe one periodic medium: the same homogenized stress, and the
    solution of the long cell is the original one repeated.  On the unit
    cube the long grid would describe voxels half as long, another medium."""
    rng = np.random.default_rng(31)
    phase = (rng.random((6, 6, 6)) < 0.4).astype(np.uint8)
    E = [1.0, 6.0]
    r1 = so.solve_linear((6, 6, 6), iso(phase, E), LOAD, tol=1e-12, tol_load=1e-12)
    twice = np.concatenate([phase, phase], axis=0)
    r2 = so.solve_linear((12, 6, 6), iso(twice, E), LOAD, tol=1e-12, tol_load=1e-12, lengths=(2.0, 1.0, 1.0))
    assert np.allclose(r2.sigma_bar, r1.sigma_bar, rtol=0, atol=1e-10 * np.abs(r1.sigma_bar).max())
    e1, e2 = r1.strain_field(), r2.strain_field()
    assert np.allclose(e2, np.concatenate([e1, e1], axis=2), atol=1e-10 * np.abs(e1).max())
    unit = so.solve_linear((12, 6, 6), iso(twice, E), LOAD, tol=1e-12, tol_load=1e-12)
    assert not np.allclose(unit.sigma_bar, r1.sigma_bar, atol=1e-6 * np.abs(r1.sigma_bar).max())


def test_dense_solve_with_lengths():
    """FFT + PCG against the direct dense solve (differentiation matrices
    on [0, L_i)), mixed control, odd and even axes of unequal lengths."""
    shape, L = (5, 4, 6), (0.7, 1.9, 1.3)
    rng = np.random.default_rng(32)
    phase = (rng.random(shape) < 0.4).astype(np.uint8)
    E, nu = [1.0, 8.0], 0.3
    mask = np.zeros((3, 3), bool)
    mask[1, 1] = mask[0, 2] = mask[2, 0] = True
    r = so.solve_linear(shape, iso(phase, E, nu), LOAD, mask, tol=1e-13, tol_load=1e-13, lengths=L)
    Cm = np.stack([mt.tensor4_to_mandel(mt.isotropic_tensor(*mt.lame(E[p], nu))) for p in phase.reshape(-1)])
    u_d, _, sig_d = dense.solve(shape, Cm, LOAD, mask, lengths=L)
    assert np.allclose(r.sigma_bar, sig_d, rtol=0, atol=1e-11 * np.abs(sig_d).max())
    u_f = sp.real_field(r.a, shape)
    u_d = u_d - u_d.mean(axis=(1, 2, 3), keepdims=True)
    assert np.allclose(u_f, u_d, atol=1e-10 * np.abs(u_d).max())
    # the unit cube is another problem here
    u1, _, sig1 = dense.solve(shape, Cm, LOAD, mask)
    assert not np.allclose(sig1, sig_d, atol=1e-6 * np.abs(sig_d).max())


def test_common_scale_changes_nothing_but_the_displacement():
    """Lengths s L, the same number of iterations: the same strains and
    stresses; the fluctuation displacement scales with s and the
    equilibrium residual (a divergence: one over a length) with 1 / s.  For
    s = 2 every frequency scales exactly, so the iterates do too."""
    shape, L, s = (6, 5, 4), (1.0, 1.5, 0.8), 2.0
    rng = np.random.default_rng(33)
    phase = (rng.random(shape) < 0.5).astype(np.uint8)
    kw = dict(tol=0.0, tol_load=0.0, max_iter=15)
    a = so.solve_linear(shape, iso(phase, [1.0, 4.0]), LOAD, lengths=L, **kw)
    b = so.solve_linear(shape, iso(phase, [1.0, 4.0]), LOAD, lengths=tuple(s * v for v in L), **kw)
    assert a.info.iterations == b.info.iterations == 15
    assert np.array_equal(b.sigma_bar, a.sigma_bar)
    assert np.array_equal(b.a, s * a.a)
    assert b.info.eq_res == a.info.eq_res / s
