"""Adjoint gradient of hyperelastic finite-strain cells (neo-Hookean and
Saint Venant-Kirchhoff) through the C ABI.

J = G:<P> + H:<F> at the end of the load path; the gradient is taken with
respect to a per-voxel factor theta(x) on the law's moduli, at theta = 1.

  * small odd and even grids, strain and mixed control: gradient and J
    against the oracle's adjoint (both Newton solves to 1e-12, adjoint
    solves to 1e-12): within 1e-7 of the gradient's max norm;
  * FP32-mixed cells against the FP64 cell: within 1e-6;
  * a 32^3 porous SVK cell against central differences of GPU Newton solves
    in which one voxel is given a phase of its own with moduli (1 +- h):
    within 1e-4 relative.
"""
import numpy as np
import pytest

from paper_1905_12725_amd import microstructure as ms
from oracle import solver as so, materials as mt

pytestmark = pytest.mark.gpu


def params(kind, mods):
    out = []
    for m in mods:
        out += [m, 0.3] if kind == "svk" else [m, 3.0 * m]
    return out


def oracle_law(kind, phase, mods):
    mods = np.asarray(mods, dtype=np.float64)
    if kind == "svk":
        lam, mu = mt.lame(mods[phase], 0.3)
        return so.SVKLaw(mu, lam)
    mu = mods[phase]
    return so.NeoHookeLaw(mu, 3.0 * mu - 2.0 * mu / 3.0)


def case(control):
    """Macro load (F on controlled components), mask, objective weights."""
    G = np.zeros((3, 3)); H = np.zeros((3, 3))
    if control == "strain":
        mask = None
        F = np.array([[1.2, 0.05, 0.0], [0.0, 1.0, 0.0], [0.0, 0.0, 0.97]])
        G[0, 0] = 1.0; G[0, 1] = 0.3; G[2, 2] = -0.4; G[1, 0] = 0.2
    else:
        mask = np.array([[0, 0, 0], [1, 1, 0], [1, 1, 1]], dtype=bool)
        F = np.zeros((3, 3)); F[0, 0] = 1.2
        G[0, 0] = 1.0; G[0, 2] = 0.5; H[1, 1] = 0.7; H[2, 0] = -0.3
    return F, mask, G, H


@pytest.mark.parametrize("kind", ["svk", "neohooke"])
@pytest.mark.parametrize("n,control", [((8, 6, 8), "strain"), ((9, 10, 7), "mixed"), ((8, 8, 8), "mixed")])
def test_hyper_adjoint_matches_oracle(gpu, kind, n, control):
    import torch
    from paper_1905_12725_amd.api import Cell
    print(f"case hyper adjoint {kind} n={n} {control}", flush=True)
    rng = np.random.default_rng(31)
    phase = (rng.random(n) < 0.3).astype(np.uint8)
    mods = [7.0, 0.7] if kind == "svk" else [1.0, 0.1]
    F, mask, G, H = case(control)
    ninc = 2
    U = np.eye(3) if mask is None else np.where(mask, 0.0, np.eye(3))
    loads = [(F - U) * (k + 1) / ninc for k in range(ninc)]
    Jo, go, info = so.adjoint_gradient_hyperelastic(n, oracle_law(kind, phase, mods), loads, mask, G, H,
                                                    tol=1e-12, newton_tol=1e-12)
    assert info.converged
    with Cell(n, kind, torch.from_numpy(phase), params(kind, mods), kinematics="finite") as cell:
        gi = cell.solve(F, mask, n_increments=ninc, tol=1e-12, tol_load=1e-12, newton_tol=1e-12)
        assert gi["status"] == 0
        g, J = cell.adjoint(G, H)
        g = g.cpu().numpy()
    assert abs(J - Jo) < 1e-9 * abs(Jo)
    assert np.max(np.abs(g - go)) < 1e-7 * np.max(np.abs(go))


@pytest.mark.parametrize("kind", ["svk", "neohooke"])
def test_hyper_adjoint_fp32_mixed_matches_fp64(gpu, kind):
    import torch
    from paper_1905_12725_amd.api import Cell
    n = (16, 12, 10)
    print(f"case hyper adjoint fp32-mixed {kind}", flush=True)
    phase = ms.centred_sphere(n, 0.25)
    mods = [7.0, 0.7] if kind == "svk" else [1.0, 0.1]
    F, mask, G, H = case("mixed")
    out = {}
    for prec in ("fp64", "fp32_mixed"):
        with Cell(n, kind, torch.from_numpy(phase), params(kind, mods), kinematics="finite", precision=prec) as cell:
            gi = cell.solve(F, mask, n_increments=2, tol=1e-10, tol_load=1e-10, newton_tol=1e-11)
            assert gi["status"] == 0
            g, J = cell.adjoint(G, H)
            out[prec] = (g.cpu().numpy(), J)
    g64, J64 = out["fp64"]
    g32, J32 = out["fp32_mixed"]
    assert abs(J32 - J64) < 1e-8 * abs(J64)
    assert np.max(np.abs(g32 - g64)) < 1e-6 * np.max(np.abs(g64))


def test_hyper_adjoint_32_porous_svk_vs_finite_differences(gpu):
    import torch
    from paper_1905_12725_amd.api import Cell
    n = (32, 32, 32)
    print("case hyper adjoint 32^3 porous svk finite differences", flush=True)
    phase, _, _ = ms.random_spheres(n, 4, 3.0, 5.0, 0.2)
    phase = phase.astype(np.uint8)
    mods = [70.0, 0.7]
    F, mask, G, H = case("mixed")
    opts = dict(tol=1e-12, tol_load=1e-12, newton_tol=1e-12)
    with Cell(n, "svk", torch.from_numpy(phase), params("svk", mods), kinematics="finite") as cell:
        gi = cell.solve(F, mask, n_increments=2, **opts)
        assert gi["status"] == 0
        g, J = cell.adjoint(G, H)
        g = g.cpu().numpy()
    rng = np.random.default_rng(77)
    worst = 0.0
    h = 1e-3
    for _ in range(6):
        idx = tuple(int(rng.integers(0, v)) for v in n)
        vals = []
        for s in (1.0, -1.0):
            ph = phase.copy()
            ph[idx] = 2
            m3 = mods + [mods[phase[idx]] * (1.0 + s * h)]
            with Cell(n, "svk", torch.from_numpy(ph), params("svk", m3), kinematics="finite") as c2:
                i2 = c2.solve(F, mask, n_increments=2, **opts)
                assert i2["status"] == 0
            vals.append(float(np.sum(G * i2["sigma_bar"]) + np.sum(H * i2["eps_bar"])))
        fd = (vals[0] - vals[1]) / (2 * h)
        worst = max(worst, abs(g[idx] - fd) / abs(fd))
    print(f"hyper adjoint 32^3: J = {J:.6e}, worst FD rel error {worst:.2e}", flush=True)
    assert worst < 1e-4
