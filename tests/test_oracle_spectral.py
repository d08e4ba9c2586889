"""Pins of the oracle's Fourier operators against definitions that use no FFT.

* The oracle's own DFT (dense per-axis sums) equals a brute-force triple
  sum on tiny grids, the library FFT on the workload sizes, keeps
  Parseval's identity and maps a delta to a constant.
* The spectral differentiation matrix is checked against closed-form
  derivatives of trigonometric polynomials.
* The FFT-based operator K (Sec. 2.2 eq. lineqf, sign-flipped; Sec. 2.3 for
  the macro block) is checked against the dense assembly from those
  matrices, on even, odd and non-cubic grids.
* Structural claims of Sec. 2.2/2.3: K is symmetric (Hermitian) for the real
  inner product, positive definite off the null set, and its null space has
  dimension 3 |Z|.
"""
import numpy as np
import pytest

from oracle import dense, spectral as sp, solver as so, materials as mt


def _brute_dft(f):
    """X(k) = sum_x f(x) exp(-2 pi i k.x / n), one term at a time."""
    n1, n2, n3 = f.shape
    X = np.zeros((n1, n2, n3 // 2 + 1), dtype=complex)
    for k1 in range(n1):
        for k2 in range(n2):
            for k3 in range(n3 // 2 + 1):
                acc = 0j
                for x1 in range(n1):
                    for x2 in range(n2):
                        for x3 in range(n3):
                            ph = -2 * np.pi * (k1 * x1 / n1 + k2 * x2 / n2 + k3 * x3 / n3)
                            acc += f[x1, x2, x3] * complex(np.cos(ph), np.sin(ph))
                X[k1, k2, k3] = acc
    return X


@pytest.mark.parametrize("shape", [(3, 4, 5), (4, 2, 6), (5, 3, 3)])
def test_own_dft_brute_force(shape):
    rng = np.random.default_rng(3)
    f = rng.standard_normal(shape)
    X = sp.dft_r2c(f, shape)
    assert np.allclose(X, _brute_dft(f), rtol=0, atol=1e-13 * np.abs(X).max())
    # planted slip: the wrong sign of the exponent fails
    assert not np.allclose(np.conj(X), _brute_dft(f), atol=1e-6)


@pytest.mark.parametrize("shape", [(16, 16, 16), (7, 9, 15), (12, 10, 8), (32, 6, 63)])
def test_own_dft_library_parseval_delta(shape):
    rng = np.random.default_rng(4)
    f = rng.standard_normal((2,) + shape)
    X = sp.dft_r2c(f, shape)
    lib = np.fft.rfftn(f, axes=(-3, -2, -1))
    assert np.allclose(X, lib, rtol=0, atol=1e-13 * np.abs(lib).max())
    # inverse of forward is N times the identity
    assert np.allclose(sp.dft_c2r(X, shape), np.prod(shape) * f, rtol=0, atol=1e-11 * np.prod(shape))
    # Parseval on the half spectrum with the plane weights
    N = float(np.prod(shape))
    w = sp.half_weights(shape)
    assert np.isclose(sp.inner(X, X, w) / N, np.sum(f * f), rtol=1e-12)
    # a delta at the origin transforms to a constant
    d = np.zeros(shape); d[0, 0, 0] = 1.0
    assert np.allclose(sp.dft_r2c(d, shape), 1.0, atol=1e-15)
    # the k3 = 0 plane of a real field is Hermitian (the twiddles are
    # exactly conjugate; only the order of the library's sums differs)
    n1, n2, _ = shape
    i1 = (-np.arange(n1)) % n1
    i2 = (-np.arange(n2)) % n2
    P = X[:, :, :, 0]
    assert np.allclose(P[:, i1][:, :, i2], np.conj(P), rtol=0, atol=1e-15 * np.abs(P).max())


@pytest.mark.parametrize("n", [4, 5, 6, 7, 8, 9, 16])
def test_diff_matrix_closed_form(n):
    D = dense.diff_matrix(n)
    x = (np.arange(n) + 0.5) / n
    for m in range(0, (n + 1) // 2):
        if n % 2 == 0 and m == n // 2:
            continue
        f = np.sin(2 * np.pi * m * x + 0.3)
        df = 2 * np.pi * m * np.cos(2 * np.pi * m * x + 0.3)
        assert np.allclose(D @ f, df, atol=1e-12 * max(1, m) * n)
    assert np.allclose(D @ np.ones(n), 0.0, atol=1e-12)
    if n % 2 == 0:
        # the Nyquist mode has no derivative on even grids
        assert np.allclose(D @ (-1.0) ** np.arange(n), 0.0, atol=1e-11)
    assert np.allclose(D, -D.T)


def test_axis_xi_values():
    assert np.allclose(sp.axis_xi(4) / (2 * np.pi), [0, 1, 0, -1])
    assert np.allclose(sp.axis_xi(5) / (2 * np.pi), [0, 1, 2, -2, -1])
    assert np.allclose(sp.axis_xi(6) / (2 * np.pi), [0, 1, 2, 0, -2, -1])


@pytest.mark.parametrize("n", [(4, 4, 4), (6, 4, 8), (5, 5, 5), (3, 5, 4)])
def test_null_set_size(n):
    Z = sp.null_set(n)
    # 2^(#even axes) points: every k_a in {0, n_a/2}; all of them lie on the
    # stored k3 planes.
    n_even = sum(1 for v in n if v % 2 == 0)
    assert Z.sum() == 2 ** n_even


def _random_aniso_mandel(rng, nv, scale=1.0):
    A = rng.standard_normal((nv, 6, 6))
    return scale * (np.einsum("vab,vcb->vac", A, A) + 6.0 * np.eye(6))


def _real_apply(shape, C_mandel, u, kin_mask=None):
    """Real-space K u = -div(C : sym grad u) via the oracle's Fourier route."""
    space = so.Space(shape, so.SMALL)
    tan = so.GeneralTangent(mt.mandel_to_tensor4(C_mandel.reshape(tuple(shape) + (6, 6))))
    a = sp.fourier(u, shape)
    a[:, space.Z] = 0.0
    (ka, _), _ = space.apply((a, np.zeros(0)), tan)
    return sp.real_field(ka, shape)


@pytest.mark.parametrize("shape", [(4, 4, 4), (6, 4, 8), (5, 5, 5), (5, 4, 6)])
def test_operator_equals_dense_definition(shape):
    rng = np.random.default_rng(1)
    N = int(np.prod(shape))
    C = _random_aniso_mandel(rng, N)
    u = rng.standard_normal((3,) + shape)
    f_fft = _real_apply(shape, C, u)
    K, Bfull, Cb, S = dense.assemble(shape, C)
    # the dense Hessian is of the *average* energy: K_dense = B^T C B / N,
    # and the real-space operator is its gradient per voxel: N * K_dense u
    f_dense = (K @ u.reshape(-1)) * N
    assert np.allclose(f_fft.reshape(-1), f_dense, rtol=0, atol=1e-10 * np.abs(f_dense).max())


def test_operator_sign_matters():
    """A planted sign flip of the divergence would fail the dense pin."""
    shape = (4, 4, 4)
    rng = np.random.default_rng(2)
    N = int(np.prod(shape))
    C = _random_aniso_mandel(rng, N)
    u = rng.standard_normal((3,) + shape)
    f_fft = _real_apply(shape, C, u)
    K, *_ = dense.assemble(shape, C)
    f_dense = (K @ u.reshape(-1)) * N
    assert not np.allclose(-f_fft.reshape(-1), f_dense, atol=1e-6)


def _valid_vector(space, rng):
    u = rng.standard_normal((3,) + space.shape)
    a = sp.fourier(u, space.shape)
    a[:, space.Z] = 0.0
    return (a, rng.standard_normal(len(space.S)))


@pytest.mark.parametrize("kin", [so.SMALL, so.FINITE])
@pytest.mark.parametrize("shape", [(4, 6, 8), (5, 4, 3)])
def test_operator_symmetric(kin, shape):
    rng = np.random.default_rng(3)
    mask = np.zeros((3, 3), bool)
    mask[1, 1] = mask[2, 2] = True
    mask[0, 1] = mask[1, 0] = True
    space = so.Space(shape, kin, mask)
    N = int(np.prod(shape))
    if kin == so.SMALL:
        C4 = mt.mandel_to_tensor4(_random_aniso_mandel(rng, N).reshape(shape + (6, 6)))
    else:
        A = rng.standard_normal((N, 9, 9))
        K9 = np.einsum("vab,vcb->vac", A, A) + 9 * np.eye(9)
        C4 = K9.reshape(shape + (3, 3, 3, 3))
    tan = so.GeneralTangent(C4)
    u, v = _valid_vector(space, rng), _valid_vector(space, rng)
    Ku, _ = space.apply(u, tan)
    Kv, _ = space.apply(v, tan)
    lhs, rhs = space.dot(v, Ku), space.dot(Kv, u)
    assert abs(lhs - rhs) <= 1e-12 * max(abs(lhs), 1.0)
    assert space.dot(u, Ku) > 0


def test_positive_definite_and_null_space_dimension():
    shape = (4, 4, 4)
    rng = np.random.default_rng(4)
    N = int(np.prod(shape))
    C = _random_aniso_mandel(rng, N)
    K, *_ = dense.assemble(shape, C)
    ev = np.linalg.eigvalsh(0.5 * (K + K.T))
    tol = 1e-10 * ev.max()
    Z = sp.null_set(shape)
    n_zero = int(np.sum(np.abs(ev) < tol))
    assert n_zero == 3 * 8  # |Z| = 8 on an all-even grid (full spectrum)
    assert np.all(ev > -tol)


def test_sym_grad_and_div_adjoint():
    """d = -s^H on symmetric tensors (the reason the printed operator is
    negative semi-definite)."""
    shape = (4, 6, 8)
    rng = np.random.default_rng(5)
    xi = sp.xi_half(shape)
    w = sp.half_weights(shape)
    a = rng.standard_normal((3,) + xi.shape[1:]) + 1j * rng.standard_normal((3,) + xi.shape[1:])
    t = rng.standard_normal((3, 3) + xi.shape[1:]) + 1j * rng.standard_normal((3, 3) + xi.shape[1:])
    t = 0.5 * (t + np.swapaxes(t, 0, 1))
    lhs = sp.inner(sp.sym_grad(a, xi), t, w)
    rhs = sp.inner(a, -sp.div(t, xi), w)
    assert abs(lhs - rhs) < 1e-10 * abs(lhs)


def test_compatibility_of_dbfft_strain():
    """Sec. 3 eq. chedckcomp: curl curl eps vanishes for any DBFFT strain field
    (computed here with the dense differentiation matrices)."""
    shape = (6, 6, 6)
    rng = np.random.default_rng(6)
    space = so.Space(shape)
    a, e = _valid_vector(space, rng)
    eps = space.field_of(a, e, np.zeros((3, 3)))
    D = [dense.partial_matrices(shape)[i] for i in range(3)]
    def d(f, j):
        return (D[j] @ f.reshape(-1)).reshape(shape)
    perm = np.zeros((3, 3, 3))
    perm[0, 1, 2] = perm[1, 2, 0] = perm[2, 0, 1] = 1
    perm[0, 2, 1] = perm[2, 1, 0] = perm[1, 0, 2] = -1
    inc = np.zeros((3, 3) + shape)
    for i in range(3):
        for j in range(3):
            acc = np.zeros(shape)
            for k in range(3):
                for l in range(3):
                    for m in range(3):
                        for nn in range(3):
                            c = perm[i, k, l] * perm[j, m, nn]
                            if c != 0:
                                acc += c * d(d(eps[l, nn], k), m)
            inc[i, j] = acc
    assert np.max(np.abs(inc)) < 1e-9 * np.max(np.abs(eps)) * (2 * np.pi * 3) ** 2
