"""dbfft_solve_many: several loads of one cell as independent PCG solves on
concurrent streams.  Every load's result must equal, bit for bit, the
result of dbfft_solve on that load (the same kernels in the same order);
the context's own solution stays as it was; failures come back per load."""
import numpy as np
import pytest

from paper_1905_12725_amd import microstructure as ms

pytestmark = pytest.mark.gpu

ENOTCONV, EINVAL, EUNSUPPORTED = 4, 1, 6


def mandel_loads(scale=1e-3):
    out = []
    for (i, j) in ((0, 0), (1, 1), (2, 2), (1, 2), (0, 2), (0, 1)):
        L = np.zeros((3, 3))
        L[i, j] = L[j, i] = scale
        out.append(L)
    return out


@pytest.mark.parametrize("prec", ["fp64", "fp32_mixed"])
@pytest.mark.parametrize("nstreams", [1, 2, 3])
def test_many_equals_one_by_one(gpu, prec, nstreams):
    import torch
    from paper_1905_12725_amd.api import Cell
    print(f"case solve_many {prec} nstreams={nstreams}", flush=True)
    n = (16, 16, 16)
    phase, _, _ = ms.random_spheres(n, 2, 2.0, 3.0, 0.3)
    loads = mandel_loads()
    with Cell(n, "iso_phase", torch.from_numpy(phase), [1.0, 0.3, 20.0, 0.3], precision=prec) as cell:
        ref = [cell.solve(L, tol=1e-10, tol_load=1e-10) for L in loads]
        got = cell.solve_many(loads, nstreams=nstreams, tol=1e-10, tol_load=1e-10)
    for r, g in zip(ref, got):
        assert g["status"] == 0
        assert g["pcg_iters"] == r["pcg_iters"]
        assert g["refine_steps"] == r["refine_steps"]
        assert np.array_equal(g["sigma_bar"], r["sigma_bar"])
        assert np.array_equal(g["eps_bar"], r["eps_bar"])


def test_many_mixed_control_with_lengths_keeps_the_solution(gpu):
    """Uniaxial stress on a cell of unequal side lengths; the context's own
    last solution is the same before and after."""
    import torch
    from paper_1905_12725_amd.api import Cell
    print("case solve_many mixed lengths", flush=True)
    n = (12, 16, 10)
    rng = np.random.default_rng(500)
    phase = (rng.random(n) < 0.4).astype(np.uint8)
    mask = np.ones((3, 3), bool); mask[0, 0] = False
    loads = [np.diag([1e-3 * (k + 1), 0.0, 0.0]) for k in range(4)]
    with Cell(n, "iso_phase", torch.from_numpy(phase), [1.0, 0.3, 5.0, 0.3], lengths=(1.2, 1.6, 1.0)) as cell:
        ref = [cell.solve(L, mask, tol=1e-11, tol_load=1e-11) for L in loads]
        before = cell.homogenize(strain=True)
        got = cell.solve_many(loads, mask, nstreams=2, tol=1e-11, tol_load=1e-11)
        after = cell.homogenize(strain=True)
    for r, g in zip(ref, got):
        assert np.array_equal(g["sigma_bar"], r["sigma_bar"])
        assert g["pcg_iters"] == r["pcg_iters"]
    assert np.array_equal(before["sigma_bar"], after["sigma_bar"])
    assert torch.equal(before["strain"], after["strain"])


def test_many_reports_failures_per_load(gpu):
    import torch
    from paper_1905_12725_amd import _native as nat
    from paper_1905_12725_amd.api import Cell
    print("case solve_many failures", flush=True)
    n = (8, 8, 8)
    phase = ms.centred_sphere(n, 0.2)
    with Cell(n, "iso_phase", torch.from_numpy(phase), [1.0, 0.3, 10.0, 0.3]) as cell:
        loads = mandel_loads()[:3]
        loads[1] = np.zeros((3, 3))  # b = 0: converged before the first iteration
        got = cell.solve_many(loads, nstreams=2, raise_on_fail=False, max_iter=3, tol=1e-12, tol_load=1e-12)
        assert [g["status"] for g in got] == [ENOTCONV, 0, ENOTCONV]
        assert got[0]["pcg_iters"] == 3 and got[1]["pcg_iters"] == 0
        with pytest.raises(nat.DbfftError) as ex:
            cell.solve_many(loads, nstreams=2, max_iter=3, tol=1e-12, tol_load=1e-12)
        assert ex.value.status == ENOTCONV and "load 0" in str(ex.value)
        for bad in (0, 9):
            with pytest.raises(nat.DbfftError) as ex:
                cell.solve_many(loads, nstreams=bad)
            assert ex.value.status == EINVAL
    with Cell(n, "neohooke", torch.from_numpy(phase), [1.0, 3.0, 10.0, 30.0], kinematics="finite") as cell:
        with pytest.raises(nat.DbfftError) as ex:
            cell.solve_many([np.eye(3)], nstreams=2)
        assert ex.value.status == EUNSUPPORTED


def test_many_follows_a_change_of_lengths(gpu):
    """Helper contexts made for one set of cell lengths take the new ones
    when the cell's lengths change between two calls (Sec. 2.1: the
    frequencies scale with 1/L), and more streams than loads are fine."""
    import torch
    from paper_1905_12725_amd.api import Cell
    print("case solve_many lengths change", flush=True)
    n = (12, 10, 16)
    rng = np.random.default_rng(501)
    phase = (rng.random(n) < 0.35).astype(np.uint8)
    loads = mandel_loads()[:3]
    with Cell(n, "iso_phase", torch.from_numpy(phase), [1.0, 0.3, 8.0, 0.3]) as cell:
        first = cell.solve_many(loads, nstreams=3, tol=1e-11, tol_load=1e-11)
        cell.set_lengths((2.0, 1.0, 0.5))
        got = cell.solve_many(loads, nstreams=4, tol=1e-11, tol_load=1e-11)
        ref = [cell.solve(L, tol=1e-11, tol_load=1e-11) for L in loads]
    for f, g, r in zip(first, got, ref):
        assert g["status"] == 0
        assert np.array_equal(g["sigma_bar"], r["sigma_bar"])
        assert g["pcg_iters"] == r["pcg_iters"]
        # strain control: stretching the axes by different factors changes
        # the microstructure's shape, so the response differs from the unit cell's
        assert not np.array_equal(g["sigma_bar"], f["sigma_bar"])
