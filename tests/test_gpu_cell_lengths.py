"""Cell side lengths L_i (Sec. 2.1, frequencies 2 pi m_i / L_i) on the HIP
path: the operator and solves against the oracle with the same lengths,
a cell repeated along an axis against the original cell (the same periodic
medium), Newton with lengths, batches, and the argument checks of
dbfft_set_lengths.  Bars as in test_gpu_parity.py."""
import numpy as np
import pytest

from paper_1905_12725_amd import microstructure as ms
from oracle import spectral as sp, solver as so, materials as mt

pytestmark = pytest.mark.gpu

LOAD = np.array([[1e-3, 2e-4, -1e-4], [2e-4, -3e-4, 4e-4], [-1e-4, 4e-4, 5e-4]])


def rel(a, b):
    return float(np.max(np.abs(a - b)) / max(np.max(np.abs(b)), 1e-300))


def iso(phase, E, nu=0.3):
    lam, mu = mt.lame(np.asarray(E)[phase], nu)
    return so.IsoTangent(lam, mu)


@pytest.mark.parametrize("prec", ["fp64", "fp32_mixed"])
@pytest.mark.parametrize("kin", ["small", "finite"])
@pytest.mark.parametrize("n,L", [((8, 6, 10), (1.5, 0.7, 2.0)), ((5, 8, 9), (0.3, 3.0, 1.0)),
                                 ((16, 4, 32), (2.0, 0.5, 4.0))])
def test_real_apply_with_lengths(gpu, n, L, kin, prec):
    import torch
    from paper_1905_12725_amd.api import Cell
    print(f"case real_apply lengths {kin} {prec} n={n} L={L}", flush=True)
    rng = np.random.default_rng(400 + sum(n))
    phase = (rng.random(n) < 0.35).astype(np.uint8)
    u = rng.standard_normal((3,) + n)
    if kin == "small":
        tan, okin = iso(phase, [1.0, 7.0]), so.SMALL
        cell = Cell(n, "iso_phase", torch.from_numpy(phase), [1.0, 0.3, 7.0, 0.3], precision=prec, lengths=L)
    else:
        mus = np.array([1.0, 10.0])
        lams = 3.0 * mus - 2.0 * mus / 3.0
        F = np.broadcast_to(np.eye(3), n + (3, 3))
        tan, okin = so.GeneralTangent(mt.neohooke_tangent(F, mus[phase], lams[phase])), so.FINITE
        cell = Cell(n, "neohooke", torch.from_numpy(phase), [1.0, 3.0, 10.0, 30.0], kinematics="finite",
                    precision=prec, lengths=L)
    with cell:
        f = cell.apply(torch.from_numpy(u).cuda()).cpu().numpy()
    space = so.Space(n, okin, None, L)
    a = sp.fourier(u, n)
    a[:, space.Z] = 0
    (ka, _), _ = space.apply((a, np.zeros(0)), tan)
    ref = sp.real_field(ka, n)
    assert rel(f, ref) < (1e-12 if prec == "fp64" else 1e-5)


@pytest.mark.parametrize("fused", [1, 0])
def test_repeated_cell_solve(gpu, fused):
    """12 x 6 x 8 over 2 x 1 x 1, the 6 x 6 x 8 unit cell twice along x: the
    oracle's solve with the same lengths and the unit cell's own solve."""
    import torch
    from paper_1905_12725_amd.api import Cell
    print(f"case repeated cell fused={fused}", flush=True)
    rng = np.random.default_rng(410)
    phase = (rng.random((6, 6, 8)) < 0.4).astype(np.uint8)
    twice = np.concatenate([phase, phase], axis=0)
    E = [1.0, 6.0]
    params = [1.0, 0.3, 6.0, 0.3]
    mask = np.zeros((3, 3), bool); mask[1, 1] = mask[2, 2] = True
    load = LOAD.copy(); load[1, 1] = 0.0; load[2, 2] = 0.01
    ref = so.solve_linear((12, 6, 8), iso(twice, E), load, mask, tol=1e-12, tol_load=1e-12, lengths=(2.0, 1.0, 1.0))
    with Cell((12, 6, 8), "iso_phase", torch.from_numpy(twice), params, lengths=(2.0, 1.0, 1.0)) as cell:
        info = cell.solve(load, mask, tol=1e-12, tol_load=1e-12, fused_cg=fused)
    with Cell((6, 6, 8), "iso_phase", torch.from_numpy(phase), params) as one:
        info1 = one.solve(load, mask, tol=1e-12, tol_load=1e-12, fused_cg=fused)
    assert abs(info["pcg_iters"] - ref.info.iterations) <= 2
    assert rel(info["sigma_bar"], ref.sigma_bar) < 1e-9
    assert rel(info["eps_bar"], ref.eps_bar) < 1e-9
    assert rel(info["sigma_bar"], info1["sigma_bar"]) < 1e-9


def test_repeated_cell_full_size(gpu):
    """The 64^3 random-sphere cell against it twice along y on 64 x 128 x 64
    over 1 x 2 x 1 (the fused iteration at full size): the same homogenized
    stress; the same grid as a unit cube is another medium."""
    import torch
    from paper_1905_12725_amd.api import Cell
    print("case repeated cell 64 x 128 x 64", flush=True)
    n = (64, 64, 64)
    phase, _, _ = ms.random_spheres(n, 2, 3.0, 5.0, 0.30)
    twice = np.concatenate([phase, phase], axis=1)
    params = [1.0, 0.3, 100.0, 0.3]
    L = np.zeros((3, 3)); L[0, 1] = L[1, 0] = 1e-3
    with Cell(n, "iso_phase", torch.from_numpy(phase), params) as one:
        a = one.solve(L, tol=1e-10, tol_load=1e-10)
    with Cell((64, 128, 64), "iso_phase", torch.from_numpy(twice), params, lengths=(1.0, 2.0, 1.0)) as cell:
        b = cell.solve(L, tol=1e-10, tol_load=1e-10)
        cell.set_lengths((1.0, 1.0, 1.0))
        c = cell.solve(L, tol=1e-10, tol_load=1e-10)
    assert rel(b["sigma_bar"], a["sigma_bar"]) < 1e-8
    assert rel(c["sigma_bar"], a["sigma_bar"]) > 1e-3


def test_newton_with_lengths(gpu):
    """Neo-Hookean stretch on 8 x 6 x 10 over (1.5, 0.7, 2.0) against the
    oracle's Newton with the same lengths."""
    import torch
    from paper_1905_12725_amd.api import Cell
    print("case newton lengths", flush=True)
    n, Lc = (8, 6, 10), (1.5, 0.7, 2.0)
    rng = np.random.default_rng(420)
    phase = (rng.random(n) < 0.3).astype(np.uint8)
    mus = np.array([1.0, 10.0])
    lams = 3.0 * mus - 2.0 * mus / 3.0
    Fbar = np.diag([1.1, 1.0, 1.0])
    loads = [(Fbar - np.eye(3)) * (k + 1) / 2 for k in range(2)]
    a, e, st, info = so.newton(n, so.NeoHookeLaw(mus[phase], lams[phase]), loads, None, kin=so.FINITE,
                               tol=1e-12, tol_load=1e-12, newton_tol=1e-11, lengths=Lc)
    assert info.converged
    with Cell(n, "neohooke", torch.from_numpy(phase), [1.0, 3.0, 10.0, 30.0], kinematics="finite",
              lengths=Lc) as cell:
        out = cell.solve(Fbar, None, n_increments=2, tol=1e-12, tol_load=1e-12, newton_tol=1e-11)
    assert rel(out["sigma_bar"], np.asarray(info.sigma_bar[-1])) < 1e-9


@pytest.mark.parametrize("prec", ["fp64", "fp32_mixed"])
def test_batch_with_lengths(gpu, prec):
    """Cells of one batch with their own lengths: the batched solve against
    each cell solved alone."""
    import torch
    from paper_1905_12725_amd.api import Batch, Cell
    print(f"case batch lengths {prec}", flush=True)
    shapes = [((12, 6, 8), (2.0, 1.0, 1.0)), ((8, 8, 8), (1.0, 0.5, 1.5)), ((6, 10, 6), (0.8, 1.2, 1.0))]
    rng = np.random.default_rng(430)
    params = [1.0, 0.3, 5.0, 0.3]
    phases = [(rng.random(n) < 0.4).astype(np.uint8) for n, _ in shapes]
    singles = []
    for (n, Lc), ph in zip(shapes, phases):
        with Cell(n, "iso_phase", torch.from_numpy(ph), params, precision=prec, lengths=Lc) as c:
            singles.append(c.solve(LOAD, tol=1e-10, tol_load=1e-10)["sigma_bar"])
    cells = [Cell(n, "iso_phase", torch.from_numpy(ph), params, precision=prec, lengths=Lc)
             for (n, Lc), ph in zip(shapes, phases)]
    with Batch(cells) as b:
        infos = b.solve(LOAD, tol=1e-10, tol_load=1e-10)
    for c in cells:
        c.close()
    for info, s in zip(infos, singles):
        assert rel(info["sigma_bar"], s) < (1e-9 if prec == "fp64" else 1e-6)


def test_set_lengths_checks_and_drops_the_solution(gpu):
    import torch
    from paper_1905_12725_amd import _native as nat
    from paper_1905_12725_amd.api import Cell
    print("case set_lengths checks", flush=True)
    n = (8, 8, 8)
    with Cell(n, "iso_phase", torch.from_numpy(np.zeros(n, np.uint8)), [1.0, 0.3]) as cell:
        for bad in ((0.0, 1.0, 1.0), (1.0, -2.0, 1.0), (1.0, 1.0, float("nan")), (1.0, float("inf"), 1.0)):
            with pytest.raises(nat.DbfftError) as ex:
                cell.set_lengths(bad)
            assert ex.value.status == nat.DBFFT_EINVAL
        cell.solve(LOAD)
        cell.homogenize()
        cell.set_lengths((2.0, 2.0, 2.0))
        with pytest.raises(nat.DbfftError):
            cell.homogenize()
        out = cell.solve(LOAD)
        assert np.allclose(out["sigma_bar"], cell.homogenize()["sigma_bar"])
