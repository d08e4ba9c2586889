"""Batched solves (several cells of uneven grid sizes in one launch per
pass) against the CPU oracle and against one-cell solves of the same cells.

Bars: FP64 solves at tol 1e-12 within 1e-10 relative of the oracle (as
the one-cell solves); FP32-mixed linear solves (FP64 refinement) within
1e-6; graph replay and eager launches bit-identical; PCG iteration counts
of a batched cell within +-2 of its one-cell solve.
"""
import numpy as np
import pytest

from paper_1905_12725_amd import microstructure as ms
from oracle import solver as so, materials as mt

pytestmark = pytest.mark.gpu


def rel(a, b):
    return float(np.max(np.abs(np.asarray(a) - np.asarray(b))) / max(np.max(np.abs(np.asarray(b))), 1e-300))


def iso_params(E, nu):
    out = []
    for e in E:
        out += [e, nu]
    return out


LIN_SIZES = [(8, 8, 8), (12, 10, 8), (10, 12, 6), (16, 16, 16), (6, 10, 12)]


def lin_cells(prec, sizes, E=(1.0, 20.0)):
    import torch
    from paper_1905_12725_amd.api import Cell
    cells, phases = [], []
    for i, n in enumerate(sizes):
        rng = np.random.default_rng(500 + i)
        phase = (rng.random(n) < 0.2 + 0.1 * (i % 3)).astype(np.uint8)
        phases.append(phase)
        cells.append(Cell(n, "iso_phase", torch.from_numpy(phase), iso_params(E, 0.3), precision=prec))
    return cells, phases


def lin_loads(ncell):
    loads, masks = [], []
    for i in range(ncell):
        L = np.zeros((3, 3))
        m = np.zeros((3, 3), bool)
        if i % 2 == 0:
            L[0, 0] = 0.01 * (1 + i)
            L[0, 1] = L[1, 0] = 0.003
        else:
            # uniaxial stress: e11 prescribed, every other stress component zero
            m[:] = True
            m[0, 0] = False
            L[0, 0] = 0.02
        loads.append(L)
        masks.append(m)
    return loads, masks


@pytest.mark.parametrize("prec", ["fp64", "fp32_mixed"])
def test_batch_linear_parity(gpu, prec):
    from paper_1905_12725_amd.api import Batch
    print(f"case batch linear {prec} sizes={LIN_SIZES}", flush=True)
    E = (1.0, 20.0)
    cells, phases = lin_cells(prec, LIN_SIZES, E)
    loads, masks = lin_loads(len(cells))
    tol = 1e-12 if prec == "fp64" else 1e-11
    with Batch(cells) as b:
        infos = b.solve(loads, masks, tol=tol, tol_load=tol)
        tiles = b.tiles()
        sols = [c.solution()[0].cpu().numpy() for c in cells]
        homs = [c.homogenize() for c in cells]
    assert tiles.shape == (len(cells), 3)
    assert np.all((tiles[:, :2] >= 1) & (tiles[:, :2] <= 32)) and np.all(tiles[:, 2] >= 1)
    bar = 1e-10 if prec == "fp64" else 1e-6
    for i, (n, c) in enumerate(zip(LIN_SIZES, cells)):
        lam, mu = mt.lame(np.asarray(E)[phases[i]], 0.3)
        ref = so.solve_linear(n, so.IsoTangent(lam, mu), loads[i], masks[i], tol=1e-12, tol_load=1e-12)
        assert infos[i]["status"] == 0
        assert rel(infos[i]["sigma_bar"], ref.sigma_bar) < bar, i
        assert rel(homs[i]["eps_bar"], ref.eps_bar) < bar, i
        if prec == "fp64":
            assert rel(sols[i], ref.a) < 1e-9, i
        # one-cell solve of the same cell
        one = c.solve(loads[i], masks[i], tol=tol, tol_load=tol)
        assert rel(infos[i]["sigma_bar"], one["sigma_bar"]) < bar, i
        if prec == "fp64":
            assert abs(infos[i]["pcg_iters"] - one["pcg_iters"]) <= 2, i
    for c in cells:
        c.close()


def test_batch_graph_matches_eager(gpu):
    from paper_1905_12725_amd.api import Batch
    print("case batch graph vs eager", flush=True)
    cells, _ = lin_cells("fp64", LIN_SIZES)
    loads, masks = lin_loads(len(cells))
    out = []
    for use_graph in (True, False):
        with Batch(cells, use_graph=use_graph) as b:
            infos = b.solve(loads, masks, tol=1e-10, tol_load=1e-10, check_every=5)
            sols = [c.solution()[0].cpu().numpy() for c in cells]
        out.append((infos, sols))
    for i in range(len(cells)):
        assert out[0][0][i]["pcg_iters"] == out[1][0][i]["pcg_iters"]
        assert np.array_equal(out[0][0][i]["sigma_bar"], out[1][0][i]["sigma_bar"])
        assert np.array_equal(out[0][1][i], out[1][1][i])
    for c in cells:
        c.close()


def test_batch_repeated_solves_and_trivial_cell(gpu):
    """A homogeneous cell converges at once (zero fluctuation) while the
    others iterate; a second solve with another load reuses the graph."""
    import torch
    from paper_1905_12725_amd.api import Cell, Batch
    print("case batch trivial cell + repeat", flush=True)
    n0 = (8, 8, 8)
    homog = Cell(n0, "iso_phase", torch.zeros(n0, dtype=torch.uint8), iso_params([3.0, 3.0], 0.25))
    cells, phases = lin_cells("fp64", [(12, 10, 8), (10, 12, 6)])
    allc = [homog] + cells
    with Batch(allc) as b:
        for scale in (1.0, -0.5):
            loads = [scale * np.diag([0.01, 0.0, 0.0])] * 3
            infos = b.solve(loads, None, tol=1e-12, tol_load=1e-12)
            lam, mu = mt.lame(3.0, 0.25)
            exact = lam * 0.01 * scale * np.eye(3)
            exact[0, 0] += 2 * mu * 0.01 * scale
            assert infos[0]["pcg_iters"] <= 1
            assert rel(infos[0]["sigma_bar"], exact) < 1e-13
            for i, n in enumerate([(12, 10, 8), (10, 12, 6)]):
                lm, m = mt.lame(np.asarray([1.0, 20.0])[phases[i]], 0.3)
                ref = so.solve_linear(n, so.IsoTangent(lm, m), loads[0], tol=1e-12, tol_load=1e-12)
                assert rel(infos[i + 1]["sigma_bar"], ref.sigma_bar) < 1e-10
    for c in allc:
        c.close()


def neo_params(mus):
    out = []
    for m in mus:
        out += [m, 3.0 * m]
    return out


@pytest.mark.parametrize("prec", ["fp64", "fp32_mixed"])
def test_batch_neohooke_parity(gpu, prec):
    import torch
    from paper_1905_12725_amd.api import Cell, Batch
    sizes = [(8, 8, 8), (10, 10, 10), (12, 12, 12)]
    print(f"case batch neohooke {prec} sizes={sizes}", flush=True)
    mus = np.array([1.0, 10.0])
    lams = 3.0 * mus - 2.0 * mus / 3.0
    ninc = 2
    Fbar = np.diag([1.1, 1.0, 1.0])
    cells, phases = [], []
    for i, n in enumerate(sizes):
        phase = ms.centred_sphere(n, 0.15 + 0.05 * i)
        phases.append(phase)
        cells.append(Cell(n, "neohooke", torch.from_numpy(phase), neo_params(mus), kinematics="finite",
                          precision=prec))
    opts = dict(tol=1e-12, tol_load=1e-12, newton_tol=1e-11) if prec == "fp64" else \
        dict(tol=1e-6, tol_load=1e-6, newton_tol=1e-10)
    with Batch(cells) as b:
        infos = b.solve([Fbar] * len(cells), None, n_increments=ninc, **opts)
        sols = [c.solution()[0].cpu().numpy() for c in cells]
    for i, n in enumerate(sizes):
        loads = [np.diag([0.1 * (k + 1) / ninc, 0.0, 0.0]) for k in range(ninc)]
        a, e, st, info = so.newton(n, so.NeoHookeLaw(mus[phases[i]], lams[phases[i]]), loads, None, kin=so.FINITE,
                                   tol=1e-12, tol_load=1e-12, newton_tol=1e-11)
        assert infos[i]["status"] == 0 and infos[i]["increments"] == ninc
        bar = 1e-9 if prec == "fp64" else 1e-7
        print(f"  cell {i}: newton {infos[i]['newton_iters']} pcg {infos[i]['pcg_iters']} "
              f"rel {rel(infos[i]['sigma_bar'], info.sigma_bar[-1]):.2e}", flush=True)
        assert rel(infos[i]["sigma_bar"], info.sigma_bar[-1]) < bar, i
        assert rel(sols[i], a) < (1e-8 if prec == "fp64" else 1e-6), i
        assert np.allclose(infos[i]["eps_bar"], Fbar, atol=1e-14)
    for c in cells:
        c.close()


def test_batch_j2_mixed_vs_single(gpu):
    import torch
    from paper_1905_12725_amd.api import Cell, Batch
    C11, C12, C44, S0, M, EDOT0 = 168000.0, 121000.0, 75000.0, 100.0, 20.0, 1e-3
    sizes = [(8, 8, 6), (10, 8, 6)]
    print(f"case batch j2 mixed sizes={sizes}", flush=True)
    mask = np.ones((3, 3), bool)
    mask[0, 0] = False
    final = np.zeros((3, 3))
    final[0, 0] = 2e-3
    dt, ninc = 0.5, 4
    cells, ones = [], []
    for i, n in enumerate(sizes):
        grain, _ = ms.voronoi_grains(n, 5, 60 + i)
        R = ms.random_rotations(5, 61 + i)
        p = [C11, C12, C44, S0, M, EDOT0] + list(np.asarray(R).reshape(-1))
        cells.append(Cell(n, "j2vp_cubic", torch.from_numpy(grain), p))
        with Cell(n, "j2vp_cubic", torch.from_numpy(grain), p) as one:
            ones.append(one.solve(final, mask, n_increments=ninc, dt=dt, tol=1e-12, tol_load=1e-12,
                                  newton_tol=1e-11))
    with Batch(cells) as b:
        infos = b.solve([final] * 2, [mask] * 2, n_increments=ninc, dt=dt, tol=1e-12, tol_load=1e-12,
                        newton_tol=1e-11)
    for i in range(2):
        assert infos[i]["status"] == 0 and infos[i]["increments"] == ninc
        assert infos[i]["newton_iters"] == ones[i]["newton_iters"]
        assert rel(infos[i]["sigma_bar"], ones[i]["sigma_bar"]) < 1e-9
    for c in cells:
        c.close()


def test_batch_smooth_sizes_fp32_vs_fp64_single(gpu):
    """Grid sizes of the uneven-batch workload (2-3-5 smooth, 32..60) with
    radices 3 and 5: the batched FP32-mixed linear solve agrees with
    one-cell FP64 solves of the same cells."""
    import torch
    from paper_1905_12725_amd.api import Cell, Batch
    sizes = [(32, 32, 32), (36, 36, 36), (50, 50, 50), (60, 60, 60), (40, 40, 40)]
    print(f"case batch smooth sizes {sizes}", flush=True)
    E = [1.0, 10.0]
    cells, refs = [], []
    load = np.diag([0.01, 0.0, 0.0])
    for i, n in enumerate(sizes):
        phase = ms.centred_sphere(n, 0.2)
        with Cell(n, "iso_phase", torch.from_numpy(phase), iso_params(E, 0.3)) as one:
            refs.append(one.solve(load, tol=1e-10, tol_load=1e-10)["sigma_bar"])
        cells.append(Cell(n, "iso_phase", torch.from_numpy(phase), iso_params(E, 0.3), precision="fp32_mixed"))
    with Batch(cells) as b:
        infos = b.solve([load] * len(cells), None, tol=1e-10, tol_load=1e-10)
        print("tiles", b.tiles().tolist(), flush=True)
    for i in range(len(sizes)):
        assert infos[i]["status"] == 0
        assert infos[i]["eq_res"] < 1e-10
        assert rel(infos[i]["sigma_bar"], refs[i]) < 1e-8, i
    for c in cells:
        c.close()


def test_batch_rejects_mixed_classes(gpu):
    import torch
    from paper_1905_12725_amd.api import Cell, Batch
    from paper_1905_12725_amd._native import DbfftError
    n = (8, 8, 8)
    ph = torch.zeros(n, dtype=torch.uint8)
    a = Cell(n, "iso_phase", ph, iso_params([1.0, 1.0], 0.3))
    b = Cell(n, "iso_phase", ph, iso_params([1.0, 1.0], 0.3), precision="fp32_mixed")
    with pytest.raises(DbfftError) as ei:
        Batch([a, b])
    assert ei.value.status == 1
    a.close()
    b.close()


def test_batch_neohooke_smooth_sizes_fp32_vs_fp64_single(gpu):
    """Uneven-batch workload shape (neo-Hookean sphere composites, 2-3-5
    smooth sizes): the batched FP32-mixed Newton against one-cell FP64
    solves of the same cells.  Both form their Newton residuals with the
    same real z transforms and two-step x/y transforms, so this checks the
    batched PCG passes and the precision, not those shared kernels; the
    oracle pins the lengths on thin cells in test_gpu_lengths.py."""
    import torch
    from paper_1905_12725_amd.api import Cell, Batch
    sizes = [32, 36, 40, 48, 50]
    print(f"case batch neohooke smooth sizes {sizes}", flush=True)
    params = [1.0, 3.0, 10.0, 30.0]
    Fbar = np.diag([1.1, 1.0, 1.0])
    opts = dict(tol=1e-6, tol_load=1e-6, newton_tol=1e-8)
    cells, refs = [], []
    for s in sizes:
        n = (s, s, s)
        phase = ms.centred_sphere(n, 0.2)
        with Cell(n, "neohooke", torch.from_numpy(phase), params, kinematics="finite") as one:
            refs.append(one.solve(Fbar, None, n_increments=2, **opts)["sigma_bar"])
        cells.append(Cell(n, "neohooke", torch.from_numpy(phase), params, kinematics="finite",
                          precision="fp32_mixed"))
    with Batch(cells) as b:
        infos = b.solve([Fbar] * len(cells), None, n_increments=2, **opts)
    for i, s in enumerate(sizes):
        print(f"  {s}^3: newton {infos[i]['newton_iters']} pcg {infos[i]['pcg_iters']} "
              f"rel {rel(infos[i]['sigma_bar'], refs[i]):.2e}", flush=True)
        assert infos[i]["status"] == 0
        assert rel(infos[i]["sigma_bar"], refs[i]) < 1e-6, s
    for c in cells:
        c.close()


@pytest.mark.parametrize("n,prec", [((128, 128, 128), "fp64"), ((96, 96, 96), "fp64"), ((96, 96, 96), "fp32_mixed")])
def test_batch_of_large_cells_solves_cell_by_cell(gpu, n, prec):
    """Two small-strain cells of at least 96^3 voxels (128^3: the fused
    single-cell iteration; 96^3: the two-step single-cell passes): the batch
    solves them with the single-cell passes (on two streams at once), so
    each result equals the cell's own solve bit for bit."""
    import torch
    from paper_1905_12725_amd.api import Batch, Cell
    print(f"case batch of two {n} cells {prec}", flush=True)
    phase, _, _ = ms.random_spheres(n, 2, 6.0 * n[0] / 128, 10.0 * n[0] / 128, 0.3)
    params = [1.0, 0.3, 100.0, 0.3]
    loads = [np.diag([1e-3, 0.0, 0.0]), np.array([[0.0, 1e-3, 0.0], [1e-3, 0.0, 0.0], [0.0, 0.0, 0.0]])]
    cells = [Cell(n, "iso_phase", torch.from_numpy(phase), params, precision=prec) for _ in loads]
    with Batch(cells) as b:
        infos = b.solve(loads, None, tol=1e-8)
        sols = [c.solution()[0].cpu().numpy() for c in cells]
    for c, L, info, a in zip(cells, loads, infos, sols):
        one = c.solve(L, tol=1e-8)
        assert info["pcg_iters"] == one["pcg_iters"]
        assert np.array_equal(a, c.solution()[0].cpu().numpy())
        c.close()


def test_cell_by_cell_lanes_statuses_and_repeated_context(gpu):
    """The cell-by-cell path runs two cells at a time on streams of the
    batch: five 96^3 cells (three microstructures, one context listed twice,
    so all its solves stay in one lane) give the one-by-one results bit for
    bit, in the listed order for the repeated context; an iteration cap
    comes back per cell."""
    import torch
    from paper_1905_12725_amd.api import Batch, Cell
    print("case batch cell-by-cell lanes", flush=True)
    n = (96, 96, 96)
    params = [1.0, 0.3, 30.0, 0.3]
    phases = [ms.random_spheres(n, s, 4.5, 7.5, 0.3)[0] for s in (2, 3, 4)]
    cells = [Cell(n, "iso_phase", torch.from_numpy(p), params) for p in phases]
    order = [0, 1, 2, 0, 1]
    loads = [np.diag([1e-3 * (k + 1), 0.0, 0.0]) for k in range(len(order))]
    with Batch([cells[i] for i in order]) as b:
        infos = b.solve(loads, None, tol=1e-9)
        last = {i: cells[i].solution()[0].cpu().numpy() for i in range(3)}
        capped = b.solve(loads, None, raise_on_fail=False, max_iter=3, tol=1e-12, tol_load=1e-12)
    for k, (i, L) in enumerate(zip(order, loads)):
        one = cells[i].solve(L, tol=1e-9)
        assert infos[k]["status"] == 0 and infos[k]["pcg_iters"] == one["pcg_iters"], k
        assert np.array_equal(infos[k]["sigma_bar"], one["sigma_bar"]), k
    # each context's last solve in the batch is the last entry that lists it
    for i in range(3):
        k = max(j for j, o in enumerate(order) if o == i)
        cells[i].solve(loads[k], tol=1e-9)
        assert np.array_equal(last[i], cells[i].solution()[0].cpu().numpy()), i
    assert [c["status"] for c in capped] == [4] * len(order)
    assert all(c["pcg_iters"] == 3 for c in capped)
    for c in cells:
        c.close()
