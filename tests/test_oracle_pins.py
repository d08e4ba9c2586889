"""Pins of the oracle's elastic tensors, their rotation, the neo-Hookean
stress against its energy, and the residual norms of Sec. 3 (eq. chedckeq).

Each expectation below is written out by hand from the definition (a
matrix typed entry by entry, a closed form, an energy differentiated
numerically, a real-space divergence built from dense differentiation
matrices), never by calling the function under test a second time.  Each
pin is paired with a planted slip that must fail it."""
import numpy as np
import pytest

from oracle import dense, materials as mt, solver as so, spectral as sp
from paper_1905_12725_amd import microstructure as ms

C11, C12, C44 = 168000.0, 121000.0, 75000.0


def _mandel_cubic_by_hand(c11, c12, c44):
    """Cubic stiffness in the orthonormal Mandel basis (11 22 33 sqrt2*23
    sqrt2*13 sqrt2*12): c11 on the normal diagonal, c12 between normal
    components, 2 c44 on the shear diagonal, nothing else."""
    M = np.zeros((6, 6))
    for i in range(3):
        for j in range(3):
            M[i, j] = c11 if i == j else c12
    for i in range(3, 6):
        M[i, i] = 2.0 * c44
    return M


def _rot(axis, angle):
    """Right-handed rotation by `angle` about coordinate axis `axis`."""
    c, s = np.cos(angle), np.sin(angle)
    R = np.eye(3)
    i, j = [(1, 2), (2, 0), (0, 1)][axis]
    R[i, i], R[i, j], R[j, i], R[j, j] = c, -s, s, c
    return R


def test_cubic_tensor_mandel_matrix_by_hand():
    C = mt.cubic_tensor(C11, C12, C44)
    assert np.allclose(mt.tensor4_to_mandel(C), _mandel_cubic_by_hand(C11, C12, C44), rtol=1e-15, atol=1e-9)
    # minor and major symmetries
    assert np.array_equal(C, np.transpose(C, (1, 0, 2, 3)))
    assert np.array_equal(C, np.transpose(C, (0, 1, 3, 2)))
    assert np.array_equal(C, np.transpose(C, (2, 3, 0, 1)))
    # planted slip: a tensor with c44 only on C_ijij (no minor symmetry)
    # gives c44 instead of 2 c44 on the Mandel shear diagonal
    bad = C.copy()
    for i in range(3):
        for j in range(3):
            if i != j:
                bad[i, j, j, i] = 0.0
    assert not np.allclose(mt.tensor4_to_mandel(bad), _mandel_cubic_by_hand(C11, C12, C44), atol=1.0)


def test_cubic_tensor_strain_energy_of_simple_states():
    """sigma = C : eps for a pure normal strain and a pure engineering shear
    strain, computed with plain tensor algebra of the definition."""
    C = mt.cubic_tensor(C11, C12, C44)
    eps = np.zeros((3, 3)); eps[0, 0] = 1.0
    sig = np.einsum("ijkl,kl->ij", C, eps)
    assert np.allclose(sig, np.diag([C11, C12, C12]), atol=0)
    g = np.zeros((3, 3)); g[0, 1] = g[1, 0] = 0.5       # engineering shear strain 1
    sig = np.einsum("ijkl,kl->ij", C, g)
    expect = np.zeros((3, 3)); expect[0, 1] = expect[1, 0] = C44   # tau = c44 * gamma
    assert np.allclose(sig, expect, atol=0)


def test_rotation_leaves_isotropic_tensor_unchanged():
    lam, mu = mt.lame(210.0, 0.3)
    Ciso = mt.isotropic_tensor(lam, mu)
    for R in ms.random_rotations(5, 41):
        assert np.allclose(mt.rotate_tensor4(Ciso, R), Ciso, atol=1e-12 * mu)


def test_rotation_cube_symmetry():
    """A quarter turn about any cube axis maps the cubic crystal onto itself."""
    C = mt.cubic_tensor(C11, C12, C44)
    for axis in range(3):
        Cr = mt.rotate_tensor4(C, _rot(axis, np.pi / 2))
        assert np.allclose(Cr, C, atol=1e-10 * C11)
    # an eighth turn does not (c11 - c12 != 2 c44 here)
    assert not np.allclose(mt.rotate_tensor4(C, _rot(2, np.pi / 4)), C, atol=1.0)


def test_rotation_45_degrees_closed_form():
    """45 degrees about e3: in the rotated frame C'1111 = (c11+c12)/2 + c44,
    C'1122 = (c11+c12)/2 - c44, C'1212 = (c11-c12)/2; the e3 column keeps
    c11 and c12 (standard transformation of a cubic crystal to the <110>
    axes)."""
    Cr = mt.rotate_tensor4(mt.cubic_tensor(C11, C12, C44), _rot(2, np.pi / 4))
    tol = 1e-10 * C11
    assert abs(Cr[0, 0, 0, 0] - ((C11 + C12) / 2 + C44)) < tol
    assert abs(Cr[1, 1, 1, 1] - ((C11 + C12) / 2 + C44)) < tol
    assert abs(Cr[0, 0, 1, 1] - ((C11 + C12) / 2 - C44)) < tol
    assert abs(Cr[0, 1, 0, 1] - (C11 - C12) / 2) < tol
    assert abs(Cr[2, 2, 2, 2] - C11) < tol
    assert abs(Cr[0, 0, 2, 2] - C12) < tol
    assert abs(Cr[1, 2, 1, 2] - C44) < tol
    # no coupling between normal strains and the 12 shear in this frame
    assert abs(Cr[0, 0, 0, 1]) < tol


def test_rotation_maps_crystal_axes_to_sample_axes():
    """A tensor stiff along crystal axis e1 only, C = e1 e1 e1 e1, turned by
    a quarter turn about e3 that takes e1 to e2, is stiff along sample axis
    e2 only: R acts crystal -> sample, C'_ijkl = R_ia R_jb R_kc R_ld C_abcd."""
    C = np.zeros((3, 3, 3, 3)); C[0, 0, 0, 0] = 1.0
    R = _rot(2, np.pi / 2)
    assert np.allclose(R @ np.array([1.0, 0, 0]), [0, 1.0, 0])
    Cr = mt.rotate_tensor4(C, R)
    expect = np.zeros((3, 3, 3, 3)); expect[1, 1, 1, 1] = 1.0
    assert np.allclose(Cr, expect, atol=1e-15)
    # general R: stiffness along the image v = R e1 of the crystal axis
    R = ms.random_rotations(1, 43)[0]
    v = R[:, 0]
    assert np.allclose(mt.rotate_tensor4(C, R), np.einsum("i,j,k,l->ijkl", v, v, v, v), atol=1e-14)
    # planted slip: the transpose maps sample -> crystal and fails
    assert not np.allclose(mt.rotate_tensor4(C, R.T), np.einsum("i,j,k,l->ijkl", v, v, v, v), atol=1e-3)


def test_rotated_mandel_is_orthogonal_similarity():
    """Rotating a fourth-order tensor is a similarity by an orthogonal 6x6
    matrix in the Mandel basis: eigenvalues (c11+2c12, c11-c12 twice,
    2c44 three times for cubic) are kept."""
    C = mt.cubic_tensor(C11, C12, C44)
    ev = np.sort([C11 + 2 * C12, C11 - C12, C11 - C12, 2 * C44, 2 * C44, 2 * C44])
    for R in ms.random_rotations(4, 44):
        M = mt.tensor4_to_mandel(mt.rotate_tensor4(C, R))
        assert np.allclose(M, M.T, atol=1e-9)
        assert np.allclose(np.sort(np.linalg.eigvalsh(M)), ev, rtol=1e-12)


def _neo_energy(F, mu, lam):
    """W = mu/2 (I1 - 3) - mu ln J + lam/2 (ln J)^2, I1 = tr(F^T F)."""
    J = np.linalg.det(F)
    I1 = np.sum(F * F)
    return 0.5 * mu * (I1 - 3.0) - mu * np.log(J) + 0.5 * lam * np.log(J) ** 2


def test_neohooke_stress_is_energy_derivative():
    """P_iJ = dW/dF_iJ by central differences of the energy written above."""
    rng = np.random.default_rng(45)
    mu, lam = 1.3, 3.9 - 2.0 * 1.3 / 3.0
    h = 1e-6
    for _ in range(4):
        F = np.eye(3) + 0.25 * rng.standard_normal((3, 3))
        if np.linalg.det(F) < 0.2:
            continue
        P = mt.neohooke_stress(F, mu, lam)
        fd = np.zeros((3, 3))
        for i in range(3):
            for J in range(3):
                Fp = F.copy(); Fp[i, J] += h
                Fm = F.copy(); Fm[i, J] -= h
                fd[i, J] = (_neo_energy(Fp, mu, lam) - _neo_energy(Fm, mu, lam)) / (2 * h)
        assert np.allclose(P, fd, rtol=1e-7, atol=1e-8)
        # planted slip: the transpose of P is not the derivative
        assert not np.allclose(P.T, fd, atol=1e-4)


def test_neohooke_uniaxial_closed_form():
    """F = diag(a, 1, 1): J = a, F^-T = diag(1/a, 1, 1), so
    P11 = mu (a - 1/a) + lam ln(a)/a and P22 = P33 = lam ln(a)."""
    mu, lam = 1.0, 7.0 / 3.0
    for a in (0.8, 1.1, 1.5):
        P = mt.neohooke_stress(np.diag([a, 1.0, 1.0]), mu, lam)
        expect = np.diag([mu * (a - 1 / a) + lam * np.log(a) / a, lam * np.log(a), lam * np.log(a)])
        assert np.allclose(P, expect, rtol=1e-14, atol=1e-15)


def test_svk_stress_is_energy_derivative():
    """Saint Venant-Kirchhoff: W = lam/2 tr(E)^2 + mu E:E, P = dW/dF."""
    rng = np.random.default_rng(46)
    mu, lam = 26.9, 40.4
    F = np.eye(3) + 0.2 * rng.standard_normal((3, 3))

    def W(F):
        E = 0.5 * (F.T @ F - np.eye(3))
        return 0.5 * lam * np.trace(E) ** 2 + mu * np.sum(E * E)

    h = 1e-6
    fd = np.zeros((3, 3))
    for i in range(3):
        for J in range(3):
            Fp = F.copy(); Fp[i, J] += h
            Fm = F.copy(); Fm[i, J] -= h
            fd[i, J] = (W(Fp) - W(Fm)) / (2 * h)
    assert np.allclose(mt.svk_stress(F, mu, lam), fd, rtol=1e-7, atol=1e-6)


def _div_rms_dense(sig, shape):
    """RMS over voxels of (div sigma)_i = sum_j d_j sigma_ij, built with the
    dense spectral differentiation matrices (no FFT)."""
    D = dense.partial_matrices(shape)
    N = int(np.prod(shape))
    f = sig.reshape(3, 3, N)
    d = np.zeros((3, N))
    for i in range(3):
        for j in range(3):
            d[i] += D[j] @ f[i, j]
    return np.sqrt(np.sum(d * d) / N)


@pytest.mark.parametrize("shape", [(4, 6, 5), (5, 4, 4), (6, 6, 6)])
def test_residual_norm_is_rms_divergence(shape):
    """Sec. 3 eq. chedckeq: the oracle's equilibrium residual equals
    ||div sigma||_L2 (RMS over the unit cell) / ||<sigma>||_F for an
    arbitrary, non-equilibrated symmetric stress field."""
    rng = np.random.default_rng(47)
    s = rng.standard_normal((3, 3) + shape)
    sig = 0.5 * (s + np.swapaxes(s, 0, 1)) + 3.0 * np.eye(3)[:, :, None, None, None]
    space = so.Space(shape)
    r, dc = space.divergence_residual(sig)
    eq, ld = so.residual_norms(space, (r, np.zeros(0)), dc)
    mean = sig.mean(axis=(2, 3, 4))
    assert np.allclose(dc, mean, atol=1e-13)
    expect = _div_rms_dense(sig, shape) / np.linalg.norm(mean)
    assert abs(eq - expect) <= 1e-12 * expect
    assert ld == 0.0
    # the loading residual is |r_e| / ||<sigma>||_F
    re = rng.standard_normal(2)
    _, ld = so.residual_norms(space, (r, re), dc)
    assert abs(ld - np.linalg.norm(re) / np.linalg.norm(mean)) <= 1e-15 * ld
    # planted slip: counting every half-spectrum plane once misses the
    # conjugate halves and fails
    w1 = np.ones_like(space.w)
    bad = np.sqrt(sp.inner(r, r, w1)) / np.linalg.norm(mean)
    assert abs(bad - expect) > 1e-3 * expect
