"""Parity of the HIP path (through the C ABI) with the CPU oracle.

FP64 bar: operator applications within 1e-12 relative (max-norm over the
field); solutions solved to tol 1e-12 on both sides within 1e-10 relative;
PCG iteration counts at tol 1e-8 within +-2.
"""
import numpy as np
import pytest

from paper_1905_12725_amd import microstructure as ms
from oracle import spectral as sp, solver as so, materials as mt

pytestmark = pytest.mark.gpu


def iso_params(E, nu):
    out = []
    for e in E:
        out += [e, nu]
    return out


def oracle_iso(phase, E, nu):
    lam, mu = mt.lame(np.asarray(E)[phase], nu)
    return so.IsoTangent(lam, mu)


def rel(a, b):
    return float(np.max(np.abs(a - b)) / max(np.max(np.abs(b)), 1e-300))


@pytest.mark.parametrize("n", [(8, 8, 8), (16, 12, 10), (6, 10, 4), (32, 32, 32), (20, 18, 30),
                               (64, 16, 128), (128, 8, 16), (16, 256, 32), (8, 16, 256)])
def test_real_apply_iso_phase(gpu, n):
    import torch
    from paper_1905_12725_amd.api import Cell
    print(f"case real_apply iso_phase n={n}", flush=True)
    rng = np.random.default_rng(100)
    phase = (rng.random(n) < 0.35).astype(np.uint8)
    E = [1.0, 7.0]
    u = rng.standard_normal((3,) + n)
    with Cell(n, "iso_phase", torch.from_numpy(phase), iso_params(E, 0.3)) as cell:
        f = cell.apply(torch.from_numpy(u).cuda()).cpu().numpy()
    space = so.Space(n)
    a = sp.fourier(u, n)
    a[:, space.Z] = 0
    (ka, _), _ = space.apply((a, np.zeros(0)), oracle_iso(phase, E, 0.3))
    ref = sp.real_field(ka, n)
    assert rel(f, ref) < 1e-12


@pytest.mark.parametrize("kin", ["small", "finite"])
@pytest.mark.parametrize("n", [(8, 8, 8), (12, 12, 8), (8, 12, 8), (10, 10, 10), (8, 8, 12), (12, 10, 6),
                               (16, 16, 16)])
def test_real_apply_fp32(gpu, n, kin):
    """FP32 operator of the mixed-precision contexts: small strains with
    two isotropic phases, finite strains with the neo-Hookean tangent at
    F = I (the state of a fresh context).  Bar 1e-5 relative."""
    import torch
    from paper_1905_12725_amd.api import Cell
    print(f"case real_apply fp32 {kin} n={n}", flush=True)
    rng = np.random.default_rng(103)
    phase = (rng.random(n) < 0.35).astype(np.uint8)
    u = rng.standard_normal((3,) + n)
    if kin == "small":
        E = [1.0, 7.0]
        cell = Cell(n, "iso_phase", torch.from_numpy(phase), iso_params(E, 0.3), precision="fp32_mixed")
        tan, space = oracle_iso(phase, E, 0.3), so.Space(n)
    else:
        mus = np.array([1.0, 10.0])
        lams = 3.0 * mus - 2.0 * mus / 3.0
        cell = Cell(n, "neohooke", torch.from_numpy(phase), [1.0, 3.0, 10.0, 30.0], kinematics="finite",
                    precision="fp32_mixed")
        F = np.broadcast_to(np.eye(3), n + (3, 3))
        tan, space = so.GeneralTangent(mt.neohooke_tangent(F, mus[phase], lams[phase])), so.Space(n, kin=so.FINITE)
    with cell:
        f = cell.apply(torch.from_numpy(u).cuda()).cpu().numpy()
    a = sp.fourier(u, n)
    a[:, space.Z] = 0
    (ka, _), _ = space.apply((a, np.zeros(0)), tan)
    ref = sp.real_field(ka, n)
    assert rel(f, ref) < 1e-5


@pytest.mark.parametrize("n", [(8, 8, 8), (12, 10, 16), (32, 64, 64)])
def test_real_apply_aniso_grain(gpu, n):
    import torch
    from paper_1905_12725_amd.api import Cell
    print(f"case real_apply aniso n={n}", flush=True)
    rng = np.random.default_rng(101)
    ng = 5
    grain = rng.integers(0, ng, size=n).astype(np.int32)
    A = rng.standard_normal((ng, 6, 6))
    Cm = np.einsum("gab,gcb->gac", A, A) + 6 * np.eye(6)
    u = rng.standard_normal((3,) + n)
    with Cell(n, "aniso_grain", torch.from_numpy(grain), Cm.reshape(-1)) as cell:
        f = cell.apply(torch.from_numpy(u).cuda()).cpu().numpy()
    space = so.Space(n)
    a = sp.fourier(u, n)
    a[:, space.Z] = 0
    C4 = mt.mandel_to_tensor4(Cm[grain])
    (ka, _), _ = space.apply((a, np.zeros(0)), so.GeneralTangent(C4))
    ref = sp.real_field(ka, n)
    assert rel(f, ref) < 1e-12


@pytest.mark.parametrize("n", [(12, 10, 8), (16, 32, 64), (32, 16, 128)])
def test_fourier_apply_with_macro(gpu, n):
    import torch
    from paper_1905_12725_amd.api import Cell
    print(f"case fourier_apply n={n}", flush=True)
    rng = np.random.default_rng(102)
    phase = (rng.random(n) < 0.5).astype(np.uint8)
    E = [2.0, 5.0]
    space = so.Space(n)
    a = sp.fourier(rng.standard_normal((3,) + n), n)
    a[:, space.Z] = 0
    e = rng.standard_normal((3, 3)) * 0.1
    e = 0.5 * (e + e.T)
    with Cell(n, "iso_phase", torch.from_numpy(phase), iso_params(E, 0.25)) as cell:
        f, sig = cell.apply_fourier(torch.from_numpy(a).cuda(), e)
        f = f.cpu().numpy()
    eps = space.field_of(a, np.zeros(0), e)
    tan = oracle_iso(phase, E, 0.25)
    r, dc = space.divergence_residual(tan.stress(eps))
    assert rel(f, -r) < 1e-12
    assert rel(sig, dc) < 1e-12


def test_config1_sphere_solve_parity(gpu):
    """16^3 centred sphere at 20 %, contrast 10, uniaxial strain 1e-3."""
    import torch
    from paper_1905_12725_amd.api import Cell
    n = (16, 16, 16)
    print("case config1 solve", flush=True)
    phase = ms.centred_sphere(n, 0.2)
    E = [1.0, 10.0]
    load = np.zeros((3, 3)); load[0, 0] = 1e-3
    tan = oracle_iso(phase, E, 0.3)
    ref8 = so.solve_linear(n, tan, load)
    ref12 = so.solve_linear(n, tan, load, tol=1e-12, tol_load=1e-12)
    with Cell(n, "iso_phase", torch.from_numpy(phase), iso_params(E, 0.3)) as cell:
        i8 = cell.solve(load)
        i12 = cell.solve(load, tol=1e-12, tol_load=1e-12)
        h = cell.homogenize(strain=True)
        a, _ = cell.solution()
        a = a.cpu().numpy()
        strain = h["strain"].cpu().numpy()
    assert abs(i8["pcg_iters"] - ref8.info.iterations) <= 2
    assert i8["eq_res"] < 1.01e-8
    assert rel(h["sigma_bar"], ref12.sigma_bar) < 1e-10
    assert rel(a, ref12.a) < 1e-10
    eps_ref = ref12.strain_field()
    E6 = np.stack([strain[0], strain[1], strain[2], strain[3], strain[4], strain[5]])
    R6 = np.stack([eps_ref[0, 0], eps_ref[1, 1], eps_ref[2, 2], eps_ref[1, 2], eps_ref[0, 2], eps_ref[0, 1]])
    assert rel(E6, R6) < 1e-10


def test_mixed_control_parity(gpu):
    import torch
    from paper_1905_12725_amd.api import Cell
    n = (16, 12, 10)
    print("case mixed control", flush=True)
    rng = np.random.default_rng(103)
    phase = (rng.random(n) < 0.3).astype(np.uint8)
    E = [1.0, 20.0]
    mask = np.ones((3, 3), bool)
    mask[0, 0] = False
    mask[0, 1] = mask[1, 0] = False
    load = np.zeros((3, 3))
    load[0, 0] = 1e-3
    load[0, 1] = load[1, 0] = 2e-4
    load[2, 2] = 5e-3  # prescribed stress
    tan = oracle_iso(phase, E, 0.3)
    ref = so.solve_linear(n, tan, load, mask, tol=1e-12, tol_load=1e-12)
    ref8 = so.solve_linear(n, tan, load, mask)
    with Cell(n, "iso_phase", torch.from_numpy(phase), iso_params(E, 0.3)) as cell:
        i12 = cell.solve(load, mask, tol=1e-12, tol_load=1e-12)
        h = cell.homogenize()
        i8 = cell.solve(load, mask)
    assert rel(h["sigma_bar"], ref.sigma_bar) < 1e-10
    assert rel(h["eps_bar"], ref.eps_bar) < 1e-10
    assert abs(i8["pcg_iters"] - ref8.info.iterations) <= 2
    assert abs(h["sigma_bar"][2, 2] - 5e-3) < 1e-12 * 5e-3 * 10


def test_fp32_mixed_solve_accuracy(gpu):
    import torch
    from paper_1905_12725_amd.api import Cell
    n = (32, 32, 32)
    print("case fp32 mixed", flush=True)
    phase, _, _ = ms.random_spheres(n, 2, 2.0, 4.0, 0.3)
    E = [1.0, 100.0]
    load = np.zeros((3, 3)); load[0, 1] = load[1, 0] = 1e-3
    ref = so.solve_linear(n, oracle_iso(phase, E, 0.3), load, tol=1e-12, tol_load=1e-12)
    with Cell(n, "iso_phase", torch.from_numpy(phase), iso_params(E, 0.3), precision="fp32_mixed") as cell:
        info = cell.solve(load)
        sig = cell.homogenize()["sigma_bar"]
    assert info["eq_res"] < 1e-8
    assert rel(sig, ref.sigma_bar) < 1e-6


@pytest.mark.parametrize("fused", [1, 0])
@pytest.mark.parametrize("mixed_control", [False, True])
def test_fp32_mixed_residual_replacement(gpu, mixed_control, fused):
    """FP32 PCG with FP64 residual replacement keeps its direction across
    replacements (inner_tol 1e-2): <sigma> within 1e-6 of the oracle, the
    final FP64 residual below tol, and the iteration count within 10 % of
    the FP64 solve's (restarted refinement needed about a third more at this
    contrast).  inner_tol 1e-4 (replacements far apart, so the FP32
    recursion drifts and segments restart) must still converge as well."""
    import torch
    from paper_1905_12725_amd.api import Cell
    n = (32, 32, 32)
    print(f"case fp32 residual replacement mixed_control={mixed_control} fused={fused}", flush=True)
    phase, _, _ = ms.random_spheres(n, 3, 2.0, 5.0, 0.3)
    E = [1.0, 100.0]
    load = np.zeros((3, 3)); load[0, 0] = 1e-3; load[0, 1] = load[1, 0] = 5e-4
    mask = np.zeros((3, 3), bool)
    if mixed_control:
        mask[1, 1] = mask[2, 2] = True
        load[1, 1] = load[2, 2] = 0.0
    ref = so.solve_linear(n, oracle_iso(phase, E, 0.3), load, mask, tol=1e-12, tol_load=1e-12)
    ph = torch.from_numpy(phase)
    with Cell(n, "iso_phase", ph, iso_params(E, 0.3)) as c64:
        it64 = c64.solve(load, mask, tol=1e-9, tol_load=1e-9, fused_cg=fused)["pcg_iters"]
    with Cell(n, "iso_phase", ph, iso_params(E, 0.3), precision="fp32_mixed") as cell:
        for inner in (1e-2, 1e-4):
            info = cell.solve(load, mask, tol=1e-9, tol_load=1e-9, inner_tol=inner, fused_cg=fused)
            sig = cell.homogenize()["sigma_bar"]
            print(f"  inner_tol {inner:g}: {info['pcg_iters']} iterations ({it64} FP64), "
                  f"{info['refine_steps']} segments, rel {rel(sig, ref.sigma_bar):.2e}", flush=True)
            assert info["status"] == 0
            assert info["eq_res"] < 1e-9 and info["load_res"] < 1e-9
            assert rel(sig, ref.sigma_bar) < 1e-6
            if inner == 1e-2:
                assert info["pcg_iters"] <= 1.1 * it64 + 2, (info["pcg_iters"], it64)


def test_laminate_closed_form_gpu(gpu):
    import torch
    from paper_1905_12725_amd.api import Cell
    from tests.test_oracle_solver import laminate_closed_form
    n = (8, 4, 6)
    print("case laminate", flush=True)
    phase = ms.laminate(n, 0, [2, 4, 2])
    E, nu = [1.0, 25.0], 0.3
    L = np.array([[1e-3, 3e-4, -2e-4], [3e-4, 5e-4, 1e-4], [-2e-4, 1e-4, -7e-4]])
    with Cell(n, "iso_phase", torch.from_numpy(phase), iso_params(E, nu)) as cell:
        cell.solve(L, tol=1e-13, tol_load=1e-13)
        sig = cell.homogenize()["sigma_bar"]
    f1 = float(phase.mean())
    C = [mt.isotropic_tensor(*mt.lame(e, nu)) for e in E]
    expect = laminate_closed_form(C, [1 - f1, f1], 0, L)
    assert rel(sig, expect) < 1e-11


def test_homogeneous_zero_iterations_gpu(gpu):
    import torch
    from paper_1905_12725_amd.api import Cell
    n = (8, 8, 8)
    with Cell(n, "iso_phase", torch.zeros(n, dtype=torch.uint8), [2.0, 0.25]) as cell:
        info = cell.solve(np.diag([1e-3, 0, 0]))
    assert info["pcg_iters"] == 0
    lam, mu = mt.lame(2.0, 0.25)
    assert np.isclose(info["sigma_bar"][0, 0], (lam + 2 * mu) * 1e-3, rtol=1e-14)


def test_deterministic_reductions(gpu):
    import torch
    from paper_1905_12725_amd.api import Cell
    n = (24, 24, 24)
    phase = ms.centred_sphere(n, 0.2)
    outs = []
    for _ in range(2):
        with Cell(n, "iso_phase", torch.from_numpy(phase), [1.0, 0.3, 10.0, 0.3]) as cell:
            cell.solve(np.diag([1e-3, 0, 0]))
            a, _ = cell.solution()
            outs.append(a.cpu().numpy())
    assert np.array_equal(outs[0], outs[1])


@pytest.mark.parametrize("n,prec", [((64, 64, 64), "fp64"), ((32, 64, 128), "fp32_mixed")])
def test_solve_parity_power_of_two(gpu, n, prec):
    """Register-resident kernels inside a full solve, against the oracle."""
    import torch
    from paper_1905_12725_amd.api import Cell
    print(f"case solve {n} {prec}", flush=True)
    phase, _, _ = ms.random_spheres(n, 7, 3.0, 6.0, 0.25)
    E = [1.0, 30.0]
    load = np.zeros((3, 3)); load[1, 2] = load[2, 1] = 1e-3; load[0, 0] = 5e-4
    mask = np.zeros((3, 3), bool); mask[2, 2] = True
    ref = so.solve_linear(n, oracle_iso(phase, E, 0.3), load, mask, tol=1e-11, tol_load=1e-11)
    with Cell(n, "iso_phase", torch.from_numpy(phase), iso_params(E, 0.3), precision=prec) as cell:
        info = cell.solve(load, mask, tol=1e-11, tol_load=1e-11)
        sig = cell.homogenize()["sigma_bar"]
    assert rel(sig, ref.sigma_bar) < (1e-9 if prec == "fp64" else 1e-6)


@pytest.mark.parametrize("prec", ["fp64", "fp32_mixed"])
@pytest.mark.parametrize("n", [(32, 16, 24), (16, 32, 32), (64, 64, 8), (32, 24, 16), (16, 14, 12)])
def test_fused_cg_matches_separate_kernels(gpu, n, prec):
    """The fused CG iteration (residual update in the divergence pass,
    alpha in the first block of the y pass, Hermitian planes in-block)
    against the separate vector kernels (alpha in the first block of the x
    pass) and against the oracle, mixed control (uniaxial stress).  n2 = 24
    and 14 take the two-step and the LDS-engine y passes."""
    import torch
    from paper_1905_12725_amd.api import Cell
    print(f"case fused vs separate n={n} {prec}", flush=True)
    rng = np.random.default_rng(77)
    phase = (rng.random(n) < 0.3).astype(np.uint8)
    E = [1.0, 25.0]
    mask = np.ones((3, 3), bool)
    mask[0, 0] = False
    load = np.zeros((3, 3))
    load[0, 0] = 0.01
    tol = 1e-12 if prec == "fp64" else 1e-10
    out = {}
    with Cell(n, "iso_phase", torch.from_numpy(phase), iso_params(E, 0.3), precision=prec) as cell:
        for fused in (1, 0):
            info = cell.solve(load, mask, tol=tol, tol_load=tol, fused_cg=fused)
            a, e = cell.solution()
            out[fused] = (info, a.cpu().numpy())
    ref = so.solve_linear(n, oracle_iso(phase, E, 0.3), load, mask, tol=1e-12, tol_load=1e-12)
    bar = 1e-10 if prec == "fp64" else 1e-6
    for fused in (1, 0):
        assert out[fused][0]["status"] == 0
        assert rel(out[fused][0]["sigma_bar"], ref.sigma_bar) < bar
    assert rel(out[1][0]["sigma_bar"], out[0][0]["sigma_bar"]) < bar
    assert rel(out[1][1], out[0][1]) < (1e-9 if prec == "fp64" else 1e-5)
    if prec == "fp64":
        assert abs(out[1][0]["pcg_iters"] - out[0][0]["pcg_iters"]) <= 2


@pytest.mark.parametrize("prec", ["fp64", "fp32_mixed"])
@pytest.mark.parametrize("n", [(32, 32, 32), (24, 20, 30)])
def test_chunk_graph_matches_eager(gpu, n, prec):
    """Single-cell solves whose later chunks of iterations replay a captured
    HIP graph (default) against every chunk launched eagerly: the same
    launches, so bit-identical solutions and equal iteration counts; two
    solves in a row with different loads reuse or recapture the graph."""
    import torch
    from paper_1905_12725_amd.api import Cell
    print(f"case chunk graph vs eager n={n} {prec}", flush=True)
    phase, _, _ = ms.random_spheres(n, 11, 2.0, 5.0, 0.25)
    E = [1.0, 50.0]
    mask = np.zeros((3, 3), bool)
    mask[2, 2] = True
    loads = [np.diag([1e-3, 0.0, 0.0]), np.array([[0, 2e-3, 0], [2e-3, 0, 0], [0, 0, 1e-2]])]
    out = {}
    with Cell(n, "iso_phase", torch.from_numpy(phase), iso_params(E, 0.3), precision=prec) as cell:
        for graph in (1, 0):
            res = []
            for L in loads:
                info = cell.solve(L, mask, tol=1e-10, tol_load=1e-10, graph=graph, check_every=4)
                res.append((info["pcg_iters"], info["refine_steps"], cell.solution()[0].cpu().numpy()))
            out[graph] = res
    for (i1, r1, a1), (i0, r0, a0) in zip(out[1], out[0]):
        assert i1 == i0 and r1 == r0
        assert np.array_equal(a1, a0)
        assert i1 > 8


def test_concurrent_contexts_match_sequential(gpu):
    """Two contexts on two streams solving from two host threads at once give
    bit-for-bit the results of one context solving the same cases in turn
    (no state is shared between contexts; reductions have a fixed order)."""
    import threading
    import torch
    from paper_1905_12725_amd.api import Cell
    n = (64, 64, 64)
    print("case concurrent contexts 64^3", flush=True)
    phase, _, _ = ms.random_spheres(n, 2, 3.0, 5.0, 0.30)
    params = [1.0, 0.3, 100.0, 0.3]
    loads = []
    for (i, j) in ((0, 0), (1, 1), (1, 2), (0, 1)):
        L = np.zeros((3, 3)); L[i, j] = L[j, i] = 1e-3
        loads.append(L)
    with Cell(n, "iso_phase", torch.from_numpy(phase), params) as one:
        seq = [one.solve(L, tol=1e-10)["sigma_bar"] for L in loads]
    streams = [torch.cuda.Stream() for _ in range(2)]
    cells = [Cell(n, "iso_phase", torch.from_numpy(phase), params, stream=s) for s in streams]
    got = [None] * len(loads)
    errs = []

    def work(j):
        try:
            for k in range(j, len(loads), 2):
                got[k] = cells[j].solve(loads[k], tol=1e-10)["sigma_bar"]
        except Exception as e:  # reported below
            errs.append(e)

    th = [threading.Thread(target=work, args=(j,)) for j in range(2)]
    for t in th:
        t.start()
    for t in th:
        t.join()
    for c in cells:
        c.close()
    assert not errs, errs
    for a, b in zip(seq, got):
        assert np.array_equal(a, b)
