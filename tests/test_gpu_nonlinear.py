"""Parity of the HIP Newton path (Sec. 2.4) and of the adjoint gradient with
the CPU oracle; full-size workloads checked through properties."""
import numpy as np
import pytest

from paper_1905_12725_amd import microstructure as ms
from oracle import spectral as sp, solver as so, materials as mt

pytestmark = pytest.mark.gpu

C11, C12, C44 = 168000.0, 121000.0, 75000.0
S0, M, EDOT0 = 100.0, 20.0, 1e-3


def rel(a, b):
    return float(np.max(np.abs(a - b)) / max(np.max(np.abs(b)), 1e-300))


def j2_params(R):
    return [C11, C12, C44, S0, M, EDOT0] + list(np.asarray(R).reshape(-1))


def oracle_j2_law(grain, R, dt):
    C = mt.tensor4_to_mandel(mt.rotate_tensor4(mt.cubic_tensor(C11, C12, C44), R))
    return so.J2Law(C[grain], S0, M, EDOT0, dt)


@pytest.mark.parametrize("ninc", [4])
@pytest.mark.parametrize("n", [(8, 8, 6), (4, 4, 32), (3, 4, 64)])
def test_j2_mixed_control_parity(gpu, ninc, n):
    """n3 = 32 and 64 take the staged FP64 z pass (four waves per line
    group), n3 = 6 the LDS engine."""
    import torch
    from paper_1905_12725_amd.api import Cell
    print(f"case j2 mixed n={n} ninc={ninc}", flush=True)
    grain, _ = ms.voronoi_grains(n, 6, 31)
    R = ms.random_rotations(6, 32)
    dt = 0.5
    mask = np.ones((3, 3), bool)
    mask[0, 0] = False
    final = np.zeros((3, 3))
    final[0, 0] = 1e-3 * dt * ninc
    loads = [final * (k + 1) / ninc for k in range(ninc)]
    law = oracle_j2_law(grain, R, dt)
    a, e, st, info = so.newton(n, law, loads, mask, tol=1e-12, tol_load=1e-12, newton_tol=1e-11)
    assert info.converged
    with Cell(n, "j2vp_cubic", torch.from_numpy(grain), j2_params(R)) as cell:
        gi = cell.solve(final, mask, n_increments=ninc, dt=dt, tol=1e-12, tol_load=1e-12, newton_tol=1e-11)
        h = cell.homogenize(strain=True)
        ag, _ = cell.solution()
    assert gi["increments"] == ninc
    assert rel(gi["sigma_bar"], info.sigma_bar[-1]) < 1e-9
    assert rel(gi["eps_bar"], info.eps_bar[-1]) < 1e-9
    assert rel(ag.cpu().numpy(), a) < 1e-8
    # stress-controlled components vanish
    s = gi["sigma_bar"]
    assert max(abs(s[1, 1]), abs(s[2, 2]), abs(s[0, 1]), abs(s[1, 2]), abs(s[0, 2])) < 1e-8 * abs(s[0, 0])


def test_j2_full_size_steady_state(gpu):
    """64^3, 200 grains, 40 increments of 0.5 s at 1e-3/s to 2 %: without
    hardening the macroscopic axial stress approaches s0 (edot/edot0)^(1/m)
    = 100 MPa once the whole cell flows; lateral stresses stay zero."""
    import torch
    from paper_1905_12725_amd.api import Cell
    n = (64, 64, 64)
    print("case j2 full size 64^3 x 40 increments", flush=True)
    grain, _ = ms.voronoi_grains(n, 200, 3)
    R = ms.random_rotations(200, 3)
    mask = np.ones((3, 3), bool)
    mask[0, 0] = False
    final = np.zeros((3, 3))
    final[0, 0] = 0.02
    with Cell(n, "j2vp_cubic", torch.from_numpy(grain), j2_params(R)) as cell:
        info = cell.solve(final, mask, n_increments=40, dt=0.5)
    print("j2 64^3:", info["pcg_iters"], info["newton_iters"], info["sigma_bar"][0, 0], flush=True)
    assert info["increments"] == 40
    s = info["sigma_bar"]
    assert abs(s[0, 0] / 100.0 - 1.0) < 0.03
    assert max(abs(s[1, 1]), abs(s[2, 2])) < 1e-6 * abs(s[0, 0])
    assert info["eq_res"] < 1e-7


def neo_params(mus):
    out = []
    for m in mus:
        out += [m, 3.0 * m]  # kappa = 3 mu
    return out


def oracle_neo_law(phase, mus):
    mus = np.asarray(mus, dtype=float)
    lams = 3.0 * mus - 2.0 * mus / 3.0
    return so.NeoHookeLaw(mus[phase], lams[phase])


def test_neohooke_strain_control_parity(gpu):
    import torch
    from paper_1905_12725_amd.api import Cell
    n = (8, 8, 8)
    print("case neohooke strain control", flush=True)
    phase = ms.centred_sphere(n, 0.2)
    mus = [1.0, 10.0]
    Fbar = np.diag([1.1, 1.0, 1.0])
    ninc = 3
    loads = [np.diag([0.1 * (k + 1) / ninc, 0.0, 0.0]) for k in range(ninc)]
    a, e, st, info = so.newton(n, oracle_neo_law(phase, mus), loads, None, kin=so.FINITE, tol=1e-12,
                               tol_load=1e-12, newton_tol=1e-11)
    with Cell(n, "neohooke", torch.from_numpy(phase), neo_params(mus), kinematics="finite") as cell:
        gi = cell.solve(Fbar, None, n_increments=ninc, tol=1e-12, tol_load=1e-12, newton_tol=1e-11)
        ag, _ = cell.solution()
    assert rel(gi["sigma_bar"], info.sigma_bar[-1]) < 1e-9
    assert rel(ag.cpu().numpy(), a) < 1e-8
    assert np.allclose(gi["eps_bar"], Fbar, atol=1e-14)


@pytest.mark.parametrize("n", [(12, 10, 10), (8, 12, 8)])
def test_neohooke_fp32_mixed_radix_parity(gpu, n):
    """FP32 inner PCG on grids with radix-3/5 transforms: the residual stays
    on Hermitian pairs of the self-conjugate planes, so the FP32 PCG reaches
    its tolerance and Newton (FP64 residuals) the oracle's solution."""
    import torch
    from paper_1905_12725_amd.api import Cell
    print(f"case neohooke fp32 n={n}", flush=True)
    phase = ms.centred_sphere(n, 0.2)
    mus = [1.0, 10.0]
    ninc = 2
    loads = [np.diag([0.1 * (k + 1) / ninc, 0.0, 0.0]) for k in range(ninc)]
    a, e, st, info = so.newton(n, oracle_neo_law(phase, mus), loads, None, kin=so.FINITE, tol=1e-12,
                               tol_load=1e-12, newton_tol=1e-11)
    with Cell(n, "neohooke", torch.from_numpy(phase), neo_params(mus), kinematics="finite",
              precision="fp32_mixed") as cell:
        gi = cell.solve(np.diag([1.1, 1.0, 1.0]), None, n_increments=ninc, tol=1e-6, tol_load=1e-6,
                        newton_tol=1e-10)
    assert gi["status"] == 0
    assert gi["pcg_iters"] < 60 * gi["newton_iters"]
    assert rel(gi["sigma_bar"], info.sigma_bar[-1]) < 1e-7


def test_neohooke_mixed_control_parity(gpu):
    import torch
    from paper_1905_12725_amd.api import Cell
    n = (8, 6, 8)
    print("case neohooke mixed control", flush=True)
    rng = np.random.default_rng(41)
    phase = (rng.random(n) < 0.3).astype(np.uint8)
    mus = [1.0, 5.0]
    # F11 and the upper triangle of F prescribed (no rigid rotation left
    # free), nominal stress zero on the diagonal and the lower triangle
    mask = np.array([[0, 0, 0], [1, 1, 0], [1, 1, 1]], dtype=bool)
    load = np.zeros((3, 3))
    load[0, 0] = 1.08
    ninc = 2
    loads = []
    for k in range(ninc):
        L = np.zeros((3, 3))
        L[0, 0] = 0.08 * (k + 1) / ninc
        loads.append(L)
    a, e, st, info = so.newton(n, oracle_neo_law(phase, mus), loads, mask, kin=so.FINITE, tol=1e-12,
                               tol_load=1e-12, newton_tol=1e-11)
    assert info.converged
    with Cell(n, "neohooke", torch.from_numpy(phase), neo_params(mus), kinematics="finite") as cell:
        gi = cell.solve(load, mask, n_increments=ninc, tol=1e-12, tol_load=1e-12, newton_tol=1e-11)
    assert rel(gi["sigma_bar"], info.sigma_bar[-1]) < 1e-9
    oracle_F = info.eps_bar[-1] + np.eye(3)
    assert rel(gi["eps_bar"], oracle_F) < 1e-9


@pytest.mark.parametrize("objective", ["c1111", "compliance"])
def test_adjoint_parity_and_fd(gpu, objective):
    import torch
    from paper_1905_12725_amd.api import Cell
    n = (8, 8, 8)
    print(f"case adjoint {objective}", flush=True)
    E = ms.lognormal_modulus(n, 5, corr_len=2.0, sigma_log=0.7)
    nu = 0.3
    G = np.zeros((3, 3)); H = np.zeros((3, 3)); mask = np.zeros((3, 3), bool); load = np.zeros((3, 3))
    if objective == "c1111":
        load[0, 0] = 1.0; G[0, 0] = 1.0
    else:
        mask[:] = True; load[0, 0] = 1.0; H[0, 0] = 1.0
    tan = so.IsoTangent(*mt.lame(E, nu))
    dtan = so.IsoTangent(*mt.lame(np.ones(n), nu))
    J, g, fwd, adj = so.adjoint_gradient(n, tan, dtan, load, mask, G, H, tol=1e-12)
    with Cell(n, "iso_field", torch.from_numpy(E), [nu]) as cell:
        cell.solve(load, mask, tol=1e-12, tol_load=1e-12)
        gg, Jg = cell.adjoint(G, H)
        gg = gg.cpu().numpy()
    assert abs(Jg - J) < 1e-10 * abs(J)
    assert rel(gg, g) < 1e-8

    def J_of(Ef):
        with Cell(n, "iso_field", torch.from_numpy(Ef), [nu]) as c2:
            info = c2.solve(load, mask, tol=1e-12, tol_load=1e-12)
        return float(np.sum(G * info["sigma_bar"]) + np.sum(H * info["eps_bar"]))

    rng = np.random.default_rng(55)
    for _ in range(3):
        idx = tuple(int(rng.integers(0, v)) for v in n)
        h = 1e-4 * E[idx]
        Ep = E.copy(); Ep[idx] += h
        Em = E.copy(); Em[idx] -= h
        fd = (J_of(Ep) - J_of(Em)) / (2 * h)
        assert abs(gg[idx] - fd) <= 1e-5 * abs(fd) + 1e-10 * abs(J)


def test_autograd_function(gpu):
    import torch
    from paper_1905_12725_amd.api import homogenized_response, Cell
    n = (8, 8, 8)
    E = torch.from_numpy(ms.lognormal_modulus(n, 6, corr_len=2.0, sigma_log=0.5)).cuda().requires_grad_(True)
    load = np.zeros((3, 3)); load[0, 0] = 1.0
    G = np.zeros((3, 3)); G[0, 0] = 1.0
    J = homogenized_response(E, load, None, G=G, tol=1e-12)
    J.backward()
    with Cell(n, "iso_field", E.detach(), [0.3]) as cell:
        cell.solve(load, tol=1e-12, tol_load=1e-12)
        g, Jc = cell.adjoint(G)
    assert abs(J.item() - Jc) < 1e-12 * abs(Jc)
    assert torch.allclose(E.grad, g, rtol=1e-10, atol=0)
