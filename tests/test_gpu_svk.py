"""Saint Venant-Kirchhoff finite-strain cells (the hyperelastic law of
Sec. 3.3) through the C ABI against the oracle's Newton-DBFFT.

Bars as for the other finite-strain law: FP64 Newton solved to 1e-12 /
1e-11 within 1e-9 relative on the nominal stress and 1e-8 on the
solution coefficients; FP32-mixed (FP64 Newton residuals) within 1e-7;
the operator at a deformed state within 1e-8 (FP64; the two states agree
to the Newton tolerance) and 1e-5 (FP32).
"""
import numpy as np
import pytest

from paper_1905_12725_amd import microstructure as ms
from oracle import spectral as sp, solver as so, materials as mt

pytestmark = pytest.mark.gpu


def rel(a, b):
    return float(np.max(np.abs(np.asarray(a) - np.asarray(b))) / max(np.max(np.abs(np.asarray(b))), 1e-300))


def svk_params(E, nu=0.3):
    out = []
    for e in E:
        out += [e, nu]
    return out


def oracle_svk_law(phase, E, nu=0.3):
    lam, mu = mt.lame(np.asarray(E, dtype=np.float64)[phase], nu)
    return so.SVKLaw(mu, lam)


@pytest.mark.parametrize("n,prec", [((8, 8, 8), "fp64"), ((9, 10, 7), "fp64"), ((12, 10, 10), "fp32_mixed")])
def test_svk_porous_strain_control_parity(gpu, n, prec):
    """Compliant sphere (100 times softer, the paper's pore model) in an SVK
    matrix, uniaxial stretch F11 = 1.3 with the other directions fixed, in
    three increments."""
    import torch
    from paper_1905_12725_amd.api import Cell
    print(f"case svk strain control n={n} {prec}", flush=True)
    phase = ms.centred_sphere(n, 0.2)
    E = [70.0, 0.7]
    Fbar = np.diag([1.3, 1.0, 1.0])
    ninc = 3
    loads = [np.diag([0.3 * (k + 1) / ninc, 0.0, 0.0]) for k in range(ninc)]
    a, e, st, info = so.newton(n, oracle_svk_law(phase, E), loads, None, kin=so.FINITE, tol=1e-12,
                               tol_load=1e-12, newton_tol=1e-11)
    assert info.converged
    with Cell(n, "svk", torch.from_numpy(phase), svk_params(E), kinematics="finite", precision=prec) as cell:
        if prec == "fp64":
            gi = cell.solve(Fbar, None, n_increments=ninc, tol=1e-12, tol_load=1e-12, newton_tol=1e-11)
        else:
            gi = cell.solve(Fbar, None, n_increments=ninc, tol=1e-6, tol_load=1e-6, newton_tol=1e-10)
        ag, _ = cell.solution()
    assert gi["status"] == 0
    if prec == "fp64":
        assert rel(gi["sigma_bar"], info.sigma_bar[-1]) < 1e-9
        assert rel(ag.cpu().numpy(), a) < 1e-8
    else:
        assert rel(gi["sigma_bar"], info.sigma_bar[-1]) < 1e-7
    assert np.allclose(gi["eps_bar"], Fbar, atol=1e-14)


def test_svk_mixed_control_parity(gpu):
    """F11 prescribed with the upper triangle of F (no free rigid rotation),
    nominal stress zero on the diagonal and the lower triangle."""
    import torch
    from paper_1905_12725_amd.api import Cell
    n = (8, 6, 8)
    print("case svk mixed control", flush=True)
    rng = np.random.default_rng(43)
    phase = (rng.random(n) < 0.3).astype(np.uint8)
    E = [70.0, 7.0]
    mask = np.array([[0, 0, 0], [1, 1, 0], [1, 1, 1]], dtype=bool)
    load = np.zeros((3, 3))
    load[0, 0] = 1.2
    ninc = 2
    loads = []
    for k in range(ninc):
        L = np.zeros((3, 3))
        L[0, 0] = 0.2 * (k + 1) / ninc
        loads.append(L)
    a, e, st, info = so.newton(n, oracle_svk_law(phase, E), loads, mask, kin=so.FINITE, tol=1e-12,
                               tol_load=1e-12, newton_tol=1e-11)
    assert info.converged
    with Cell(n, "svk", torch.from_numpy(phase), svk_params(E), kinematics="finite") as cell:
        gi = cell.solve(load, mask, n_increments=ninc, tol=1e-12, tol_load=1e-12, newton_tol=1e-11)
    assert gi["status"] == 0
    assert rel(gi["sigma_bar"], info.sigma_bar[-1]) < 1e-9
    assert rel(gi["eps_bar"], info.eps_bar[-1] + np.eye(3)) < 1e-9


@pytest.mark.parametrize("prec", ["fp64", "fp32_mixed"])
@pytest.mark.parametrize("n", [(16, 16, 16), (12, 10, 8)])
def test_svk_operator_at_deformed_state(gpu, n, prec):
    """After one stretched increment the context holds F and S per voxel;
    its operator (the SVK tangent inside the z pass) applied to a random
    displacement against the oracle's tangent at the oracle's solution."""
    import torch
    from paper_1905_12725_amd.api import Cell
    print(f"case svk operator n={n} {prec}", flush=True)
    phase = ms.centred_sphere(n, 0.2)
    E = [70.0, 7.0]
    Fbar = np.diag([1.25, 1.0, 0.95])
    a, e, st, info = so.newton(n, oracle_svk_law(phase, E), [Fbar - np.eye(3)], None, kin=so.FINITE,
                               tol=1e-12, tol_load=1e-12, newton_tol=1e-12)
    space = so.Space(n, kin=so.FINITE)
    H = space.field_of(a, np.zeros(0), Fbar - np.eye(3))
    F = np.moveaxis(H, (0, 1), (-2, -1)) + np.eye(3)
    lam, mu = mt.lame(np.asarray(E)[phase], 0.3)
    tan = so.GeneralTangent(mt.svk_tangent(F, mu, lam))
    rng = np.random.default_rng(7)
    u = rng.standard_normal((3,) + n)
    with Cell(n, "svk", torch.from_numpy(phase), svk_params(E), kinematics="finite", precision=prec) as cell:
        cell.solve(Fbar, None, n_increments=1, tol=1e-12, tol_load=1e-12, newton_tol=1e-12)
        f = cell.apply(torch.from_numpy(u).cuda()).cpu().numpy()
    au = sp.fourier(u, n)
    au[:, space.Z] = 0
    (ka, _), _ = space.apply((au, np.zeros(0)), tan)
    # the two states agree to the Newton tolerance, not to rounding
    assert rel(f, sp.real_field(ka, n)) < (1e-8 if prec == "fp64" else 1e-5)


@pytest.mark.parametrize("prec", ["fp64", "fp32_mixed"])
def test_svk_batch_parity(gpu, prec):
    """SVK cells of uneven sizes in one batch against one-cell solves."""
    import torch
    from paper_1905_12725_amd.api import Batch, Cell
    sizes = [(12, 12, 12), (16, 16, 16), (10, 12, 14)]
    print(f"case svk batch {prec}", flush=True)
    E = [70.0, 0.7]
    phases = [ms.centred_sphere(n, 0.2) for n in sizes]
    Fbar = np.diag([1.2, 1.0, 1.0])
    tol = dict(tol=1e-10, tol_load=1e-10, newton_tol=1e-10) if prec == "fp64" else \
        dict(tol=1e-6, tol_load=1e-6, newton_tol=1e-9)
    cells = [Cell(n, "svk", torch.from_numpy(ph), svk_params(E), kinematics="finite", precision=prec)
             for n, ph in zip(sizes, phases)]
    with Batch(cells) as b:
        infos = b.solve([Fbar] * len(cells), None, n_increments=2, **tol)
    for c, info, n, ph in zip(cells, infos, sizes, phases):
        assert info["status"] == 0
        one = c.solve(Fbar, None, n_increments=2, **tol)
        assert rel(info["sigma_bar"], one["sigma_bar"]) < (1e-9 if prec == "fp64" else 1e-6)
        c.close()
