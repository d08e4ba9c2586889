#!/usr/bin/env python3
"""Benchmark of the DBFFT hot path on one MI355X.

Workload: 128^3 voxel periodic cell, seeded random non-overlapping spheres
(radius 6-10 voxels, 30 % volume fraction, seed 2), stiffness contrast 100
(E = 1 / 100, nu = 0.3), six independent macroscopic strain load cases
(1e-3 times the Mandel basis tensors) giving the effective stiffness.
One step = the six preconditioned-CG solves to the paper's equilibrium
tolerance 1e-8 (right-hand sides, mean stiffness, all CG iterations and
the final residual check), inputs resident in HBM.

Prints one JSON line.  `value` is operator applications per second over
the timed steps in FP64 (every CG iteration applies the operator once).
Also reported: voxel-DOFs per second, per-kernel durations from HIP events
the launches record at each kernel's start and end over the timed region,
the roofline of the dominant kernel, the FP32-mixed (FP32 transforms and
pointwise work, FP64 dots and outer corrections) solve time against FP64
at equal homogenized-stress accuracy, and the CPU oracle timed on a
bounded sample of the same workload.  A second workload (32 neo-Hookean
cells of uneven grid sizes, 10 load increments) compares the batched
FP32-mixed solve with sequential FP64 solves; a third sweeps the phase
contrast of a sphere inclusion at 63^3 and 64^3 (iterations per case); a
fourth stretches a porous Saint Venant-Kirchhoff cell to twice its length
(63^3, 5 increments) under both preconditioner-refresh policies; a fifth
solves the six load cases as one batch against one after the other; the
64^3 J2 polycrystal (40 increments) and the 96^3 adjoint gradient are
timed last.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0

# HBM bytes per launch of the 128^3 kernels (FP64, and FP32 for the
# FP32-mixed inner iteration) measured with rocprofv3 (FETCH_SIZE x 2.000 +
# WRITE_SIZE x 1.000; the factors make a 1 GiB device copy read and write
# 1 GiB).  They hold for the kernel sources whose
# SHA-256 is recorded here and are reported as null once those change.
TRAFFIC_SOURCES = ("paper_1905_12725_amd/csrc/fft_fast.hip", "paper_1905_12725_amd/csrc/fft_common.h",
                   "paper_1905_12725_amd/csrc/pcg_core.h", "paper_1905_12725_amd/csrc/pcg.hip")
TRAFFIC_SHA256 = "8f2028f5d67fb94f288b6723d40ac1b30fd4ef582ec77f93066a0f5e428116f1"
TRAFFIC_128 = {
    "fp64": {"x_inverse_grad": 153575322, "y_inverse": 207308617, "y_forward": 207308617,
             "z_fused_tangent": 213127961, "x_forward_div": 227591867, "cg_beta": 34815,
             "cg_direction": 255661787},
    "fp32_mixed": {"x_inverse_grad": 76856972, "y_inverse": 102418812, "y_forward": 102418812,
                   "z_fused_tangent": 108695284, "x_forward_div": 123940035, "cg_beta": 34815,
                   "cg_direction": 127875436},
}


def measured_traffic(n, kind, precision="fp64"):
    import hashlib
    h = hashlib.sha256()
    for f in TRAFFIC_SOURCES:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    if h.hexdigest() != TRAFFIC_SHA256 or tuple(n) != (128, 128, 128):
        return None
    return TRAFFIC_128[precision].get(kind)


METRIC = "DBFFT operator applies/s (Gvoxel-DOF/s, %HBM) + solve time FP32-mixed vs FP64"


def mandel_loads(scale=1e-3):
    loads = []
    pairs = ((0, 0), (1, 1), (2, 2), (1, 2), (0, 2), (0, 1))
    for (i, j) in pairs:
        L = np.zeros((3, 3))
        if i == j:
            L[i, i] = scale
        else:
            L[i, j] = L[j, i] = scale / np.sqrt(2.0)
        loads.append(L)
    return loads


def kernel_bytes(n, kind, wbytes, fused=True):
    """Algorithmic HBM bytes of one launch of each kernel kind (small strain,
    phase-map material): complex half-spectrum fields of nh = n1 n2 (n3/2+1)
    entries, 2*wbytes each.  Fused CG iteration: the divergence pass also
    reads and writes r (no q vector, alpha and the Hermitian projection of
    r on the self-conjugate planes done there too), the direction kernel
    reads r, p, x and writes p, x; otherwise the update kernel reads r, q and writes r, and the
    direction kernel is the same as in the fused iteration."""
    n1, n2, n3 = n
    nh = n1 * n2 * (n3 // 2 + 1)
    c = 2 * wbytes
    N = n1 * n2 * n3
    b = {
        "x_inverse_grad": (3 + 6) * nh * c,
        "y_inverse": 12 * nh * c,
        "z_fused_tangent": 12 * nh * c + N * 1,
        "y_forward": 12 * nh * c,
        "cg_alpha": 0,
        "cg_beta": 0,
    }
    if fused:
        b.update({"x_forward_div": (6 + 3 + 3) * nh * c, "cg_direction": (9 + 6) * nh * c, "cg_update": 0})
    else:
        b.update({"x_forward_div": (6 + 3) * nh * c, "cg_update": 3 * 3 * nh * c,
                  "cg_direction": (9 + 6) * nh * c})
    return b[kind]


def run_cases(cell, loads, **opts):
    cols, iters, refine = [], 0, 0
    for L in loads:
        info = cell.solve(L, **opts)
        iters += info["pcg_iters"]
        refine += info["refine_steps"]
        cols.append(info["sigma_bar"].copy())
    return cols, iters, refine


def ceff(cols):
    """Effective stiffness in the Mandel basis from the six responses."""
    r2 = np.sqrt(2.0)
    M = np.zeros((6, 6))
    pairs = ((0, 0), (1, 1), (2, 2), (1, 2), (0, 2), (0, 1))
    for b, s in enumerate(cols):
        for a, (i, j) in enumerate(pairs):
            M[a, b] = s[i, j] * (1.0 if i == j else r2)
    return M / 1e-3


def cpu_worker(case, n, seconds):
    """One oracle process of the CPU baseline: builds load case `case` of
    the bench cell, reports "ready", waits for "go" on stdin, then runs CG
    iterations for about `seconds` (sized by the time of the right-hand
    side's operator application) and prints its iterations, wall and CPU
    time as JSON."""
    import psutil
    from paper_1905_12725_amd import microstructure as ms
    from oracle import materials as omt, solver as oso
    phase, _, _ = ms.random_spheres(n, 2, 6.0, 10.0, 0.30)
    lam, mu = omt.lame(np.asarray([1.0, 100.0])[phase], 0.3)
    tan = oso.IsoTangent(lam, mu)
    space = oso.Space(n)
    L = mandel_loads()[case]
    t0 = time.perf_counter()
    (ka, _), dc0 = space.apply(space.zeros(), tan, L)
    t_apply = time.perf_counter() - t0
    b = (-ka, np.zeros(0))
    M = space.preconditioner(tan.mean())
    k = max(1, int(round(seconds / max(t_apply, 1e-3))))
    print("ready", flush=True)
    sys.stdin.readline()
    proc = psutil.Process()
    c0 = proc.cpu_times()
    w0 = time.perf_counter()
    _, _, info = oso.pcg(space, tan, M, b, dc0, tol=0.0, tol_load=0.0, max_iter=k)
    wall = time.perf_counter() - w0
    c1 = proc.cpu_times()
    print(json.dumps({"iters": info.iterations, "wall": wall,
                      "cpu": (c1.user - c0.user) + (c1.system - c0.system)}), flush=True)


def cpu_baseline(n, seconds):
    """The oracle (NumPy, FP64) doing CG iterations of the bench workload on
    the host's cores: one process per load case (six, or fewer when the
    host has fewer cores), the host's cores split evenly between them as
    BLAS threads.  The processes build their problems, start together, and
    the rate is their summed iterations over the wall time from the start
    to the last one's end."""
    import subprocess
    ncpu = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else (os.cpu_count() or 1)
    nproc = max(1, min(6, ncpu))
    threads = max(1, ncpu // nproc)
    env = dict(os.environ)
    for v in ("OMP_NUM_THREADS", "OPENBLAS_NUM_THREADS", "MKL_NUM_THREADS"):
        env[v] = str(threads)
    env["HIP_VISIBLE_DEVICES"] = ""  # the oracle processes never touch the GPU
    procs = [subprocess.Popen([sys.executable, os.path.abspath(__file__), "--cpu-worker", str(j),
                               "--n", str(n[0]), "--cpu-seconds", str(seconds)],
                              stdin=subprocess.PIPE, stdout=subprocess.PIPE, text=True, env=env)
             for j in range(nproc)]
    try:
        for pr in procs:
            line = pr.stdout.readline()
            if line.strip() != "ready":
                raise RuntimeError(f"oracle worker did not start: {line!r}")
        w0 = time.perf_counter()
        for pr in procs:
            pr.stdin.write("go\n")
            pr.stdin.flush()
        res = [json.loads(pr.stdout.readline()) for pr in procs]
        wall = time.perf_counter() - w0
    finally:
        for pr in procs:
            try:
                pr.stdin.close()
            except OSError:
                pass
            pr.wait(timeout=600)
    iters = sum(r["iters"] for r in res)
    cpu = sum(r["cpu"] for r in res)
    return {
        "value": iters / wall,
        "unit": "applies/s",
        "cores": max(1, int(round(cpu / wall))),
        "kind": "oracle",
        "sample": f"{iters} CG iterations (one operator application each) of the same {n[0]}^3 cell, "
                  f"{nproc} oracle processes (one load case each, {threads} BLAS thread{'s' if threads > 1 else ''} each) started "
                  f"together, {wall:.1f} s wall, {cpu:.1f} s CPU; setup not counted",
        "host_cpu_count": ncpu,
        "processes": nproc,
    }


def batched_leg(log, ncell=32, ninc=10, seed=4, only_batched=False):
    """Uneven batch: `ncell` cubic cells with sizes drawn from the even
    2-3-5-smooth sizes in [32, 96], each a neo-Hookean two-phase sphere
    composite (centred sphere at 20 %, mu 1 / 10, kappa = 3 mu), stretched to
    F11 = 1.1 in `ninc` increments under strain control.  Times four legs:
    the cells solved one after the other and as one batch (one launch per
    pass over all cells, graph-replayed PCG chunks, autotuned tiles), each
    in plain FP64 and in FP32-mixed, so that the gain of batching and the
    gain of precision are reported apart; all at PCG tol 1e-6 and Newton
    tol 1e-7, errors against a batched FP64 solve at 1e-10.  `only_batched` runs the batched
    FP32-mixed solve alone (no reference, no sequential leg), for profiling."""
    import torch
    from paper_1905_12725_amd import microstructure as ms
    from paper_1905_12725_amd.api import Cell, Batch

    sizes = ms.smooth_batch_sizes(ncell, seed)
    params = [1.0, 3.0, 10.0, 30.0]
    phases = [ms.centred_sphere((s, s, s), 0.2) for s in sizes]
    Fbar = np.diag([1.1, 1.0, 1.0])
    opts = dict(tol=1e-6, tol_load=1e-6, newton_tol=1e-7)

    def make(prec):
        return [Cell((s, s, s), "neohooke", torch.from_numpy(ph), params, kinematics="finite", precision=prec)
                for s, ph in zip(sizes, phases)]

    def timed(fn):
        torch.cuda.synchronize()
        t = time.perf_counter()
        out = fn()
        torch.cuda.synchronize()
        return time.perf_counter() - t, out

    if only_batched:
        c32 = make("fp32_mixed")
        with Batch(c32) as b32:
            tb, ib = timed(lambda: b32.solve([Fbar] * ncell, None, n_increments=ninc, **opts))
        for c in c32:
            c.close()
        log(f"[bench] batch workload: batched FP32-mixed {tb:.3f} s")
        return {"sizes": sizes, "batched_fp32_mixed": {"time_s": tb,
                                                       "pcg_iters": int(sum(i["pcg_iters"] for i in ib)),
                                                       "newton_iters": int(sum(i["newton_iters"] for i in ib))}}

    c64 = make("fp64")
    with Batch(c64) as b:
        _, ref = timed(lambda: b.solve([Fbar] * ncell, None, n_increments=ninc, tol=1e-10, tol_load=1e-10,
                                       newton_tol=1e-10))
    ref = [i["sigma_bar"] for i in ref]

    def err(infos):
        return max(float(np.max(np.abs(i["sigma_bar"] - r)) / np.max(np.abs(r))) for i, r in zip(infos, ref))

    t64, i64 = timed(lambda: [c.solve(Fbar, None, n_increments=ninc, **opts) for c in c64])
    log(f"[bench] batch workload: sequential FP64 {t64:.3f} s")
    with Batch(c64) as b:
        tb64, ib64 = timed(lambda: b.solve([Fbar] * ncell, None, n_increments=ninc, **opts))
    log(f"[bench] batch workload: batched FP64 {tb64:.3f} s")
    for c in c64:
        c.close()
    c32 = make("fp32_mixed")
    t32, i32 = timed(lambda: [c.solve(Fbar, None, n_increments=ninc, **opts) for c in c32])
    log(f"[bench] batch workload: sequential FP32-mixed {t32:.3f} s")
    b32 = Batch(c32)
    tb, ib = timed(lambda: b32.solve([Fbar] * ncell, None, n_increments=ninc, **opts))
    log(f"[bench] batch workload: batched FP32-mixed {tb:.3f} s")
    b32.close()
    for c in c32:
        c.close()

    def leg(t, infos):
        return {"time_s": t, "sigma_rel_err": err(infos), "pcg_iters": int(sum(i["pcg_iters"] for i in infos)),
                "newton_iters": int(sum(i["newton_iters"] for i in infos))}
    return {
        "workload": f"{ncell} neo-Hookean sphere composites, cubic grids from the 2-3-5-smooth even sizes in "
                    f"[32, 96] (seed {seed}), F11 = 1.1 in {ninc} increments, strain control",
        "sizes": sizes,
        "voxels": int(sum(s ** 3 for s in sizes)),
        "sequential_fp64": leg(t64, i64),
        "batched_fp64": leg(tb64, ib64),
        "sequential_fp32_mixed": leg(t32, i32),
        "batched_fp32_mixed": leg(tb, ib),
        "speedup_batching_fp64": t64 / tb64,
        "speedup_batching_fp32_mixed": t32 / tb,
        "speedup_precision_sequential": t64 / t32,
        "speedup_precision_batched": tb64 / tb,
        "speedup_batched_fp32_mixed_vs_sequential_fp64": t64 / tb,
        "target_sigma_rel_err": 1e-6,
    }


def j2_polycrystal_leg(log, n=(64, 64, 64)):
    """The 64^3 polycrystal: 200 seeded Voronoi grains with uniformly random
    orientations, cubic elasticity C11 = 168, C12 = 121, C44 = 75 GPa, rate-
    dependent J2 (sigma0 = 100 MPa, m = 20, edot0 = 1e-3/s); uniaxial strain
    rate 1e-3/s to 2 % in 40 increments of 0.5 s, the other macroscopic
    stresses zero; Newton + PCG, FP64 (parity is tested at small sizes)."""
    import torch
    from paper_1905_12725_amd import microstructure as ms
    from paper_1905_12725_amd.api import Cell

    grain, _ = ms.voronoi_grains(n, 200, 3)
    R = ms.random_rotations(200, 3)
    params = [168e3, 121e3, 75e3, 100.0, 20.0, 1e-3] + list(np.asarray(R).reshape(-1))
    mask = np.ones((3, 3), bool)
    mask[0, 0] = False
    final = np.zeros((3, 3))
    final[0, 0] = 0.02
    with Cell(n, "j2vp_cubic", torch.from_numpy(grain), params) as cell:
        torch.cuda.synchronize()
        t = time.perf_counter()
        info = cell.solve(final, mask, n_increments=40, dt=0.5)
        torch.cuda.synchronize()
        el = time.perf_counter() - t
    log(f"[bench] J2 polycrystal 64^3: {el:.2f} s, {info['pcg_iters']} PCG, {info['newton_iters']} Newton, "
        f"sigma11 {info['sigma_bar'][0, 0]:.2f} MPa")
    out = {"workload": "64^3, 200 Voronoi grains (seed 3), cubic elasticity (MPa), J2 s0 = 100 MPa, m = 20, "
                       "edot0 = 1e-3/s; eps11 to 2 % at 1e-3/s in 40 increments, other stresses zero; FP64",
           "solve_s": el, "pcg_iters": int(info["pcg_iters"]), "newton_iters": int(info["newton_iters"]),
           "sigma11_MPa": float(info["sigma_bar"][0, 0]), "status": int(info["status"])}
    # adjoint through the 40 increments: d sigma11 / d s0-factor(x); summed
    # over the voxels it equals the derivative for one factor everywhere
    G = np.zeros((3, 3)); G[0, 0] = 1.0
    opts = dict(tol=1e-10, tol_load=1e-10, newton_tol=1e-9)
    with Cell(n, "j2vp_cubic", torch.from_numpy(grain), params) as cell:
        torch.cuda.synchronize()
        t = time.perf_counter()
        ia = cell.solve(final, mask, n_increments=40, dt=0.5, checkpoint=1, **opts)
        torch.cuda.synchronize()
        t_fwd = time.perf_counter() - t
        t = time.perf_counter()
        g, J = cell.adjoint(G, np.zeros((3, 3)))
        torch.cuda.synchronize()
        t_adj = time.perf_counter() - t
        gsum = float(g.sum())
    h = 1e-3
    vals = []
    for sgn in (1.0, -1.0):
        p2 = list(params)
        p2[3] = 100.0 * (1.0 + sgn * h)
        with Cell(n, "j2vp_cubic", torch.from_numpy(grain), p2) as c2:
            vals.append(float(c2.solve(final, mask, n_increments=40, dt=0.5, **opts)["sigma_bar"][0, 0]))
    fd = (vals[0] - vals[1]) / (2 * h)
    log(f"[bench] J2 adjoint 64^3 x 40 increments: forward with checkpoints {t_fwd:.2f} s, adjoint {t_adj:.2f} s, "
        f"sum of gradient {gsum:.6f} vs uniform-factor FD {fd:.6f}")
    out["adjoint"] = {"objective": "sigma11 after the last increment; gradient w.r.t. a per-voxel factor on s0",
                      "tol": 1e-10, "forward_with_checkpoints_s": t_fwd, "adjoint_s": t_adj,
                      "pcg_iters_forward": int(ia["pcg_iters"]), "J": J, "gradient_sum": gsum,
                      "uniform_factor_fd": fd, "sum_rule_rel_err": abs(gsum - fd) / abs(fd)}
    return out


def adjoint_leg(log, n=(96, 96, 96), nfd=5):
    """The 96^3 log-normal modulus field (correlation length 8 voxels,
    sigma_log 1, nu 0.3): C1111 by a strain-controlled solve and its
    gradient with respect to every voxel modulus by the adjoint solve, FP64
    and FP32-mixed (tol 1e-10), with a central finite-difference check of
    the FP64 gradient on `nfd` random voxels (the GPU tests use 50)."""
    import torch
    from paper_1905_12725_amd import microstructure as ms
    from paper_1905_12725_amd.api import Cell

    E = ms.lognormal_modulus(n, 5, corr_len=8.0, sigma_log=1.0)
    load = np.zeros((3, 3)); load[0, 0] = 1.0
    G = np.zeros((3, 3)); G[0, 0] = 1.0
    out = {"workload": f"{n[0]}^3 log-normal E (seed 5, corr 8, sigma_log 1), nu 0.3; C1111 and dC1111/dE(x)"}
    grads = {}
    for prec in ("fp64", "fp32_mixed"):
        with Cell(n, "iso_field", torch.from_numpy(E), [0.3], precision=prec) as cell:
            cell.solve(load, tol=1e-10, tol_load=1e-10)  # warm
            torch.cuda.synchronize()
            t = time.perf_counter()
            info = cell.solve(load, tol=1e-10, tol_load=1e-10)
            torch.cuda.synchronize()
            t_fwd = time.perf_counter() - t
            t = time.perf_counter()
            g, J = cell.adjoint(G)
            torch.cuda.synchronize()
            t_adj = time.perf_counter() - t
            grads[prec] = g.cpu().numpy()
        out[prec] = {"C1111": J, "forward_s": t_fwd, "adjoint_s": t_adj, "pcg_iters_forward": int(info["pcg_iters"])}
        log(f"[bench] adjoint 96^3 {prec}: forward {t_fwd:.3f} s, adjoint {t_adj:.3f} s, C1111 {J:.6f}")
    g64 = grads["fp64"]
    out["fp32_mixed_vs_fp64_grad_rel"] = float(np.max(np.abs(grads["fp32_mixed"] - g64)) / np.max(np.abs(g64)))
    rng = np.random.default_rng(55)
    worst = 0.0
    for _ in range(nfd):
        idx = tuple(int(rng.integers(0, v)) for v in n)
        h = 1e-2 * E[idx]
        vals = []
        for s in (1.0, -1.0):
            Ef = E.copy()
            Ef[idx] += s * h
            with Cell(n, "iso_field", torch.from_numpy(Ef), [0.3]) as c2:
                vals.append(float(c2.solve(load, tol=1e-12, tol_load=1e-12)["sigma_bar"][0, 0]))
        fd = (vals[0] - vals[1]) / (2 * h)
        worst = max(worst, abs(g64[idx] - fd) / abs(fd))
    out["fd_voxels"] = nfd
    out["fd_max_rel_err"] = worst
    log(f"[bench] adjoint 96^3: FD check on {nfd} voxels, max rel err {worst:.2e}")
    return out


def multi_rhs_leg(log, sizes=((64, 64, 64), (96, 96, 96), (128, 128, 128))):
    """The six Mandel load cases of the headline workload solved together:
    six contexts on the same microstructure in one batch (one launch per
    pass for all six right-hand sides), and (FP64) block PCG with the six
    loads in one block Krylov space, against the six solves one after the
    other, FP64 and FP32-mixed, PCG tol 1e-8.  Timed after one warm run of
    each."""
    import torch
    from paper_1905_12725_amd import microstructure as ms
    from paper_1905_12725_amd.api import Cell, Batch

    out = {"workload": "random spheres (radius 6-10 voxels scaled with n/128, 30 %, seed 2), contrast 100, "
                       "six Mandel strain load cases, PCG tol 1e-8"}
    loads = mandel_loads()
    params = [1.0, 0.3, 100.0, 0.3]
    for n in sizes:
        phase, _, _ = ms.random_spheres(n, 2, 6.0 * n[0] / 128, 10.0 * n[0] / 128, 0.30)
        for prec in ("fp64", "fp32_mixed"):
            cell = Cell(n, "iso_phase", torch.from_numpy(phase), params, precision=prec)
            run_cases(cell, loads[:2], tol=1e-8)
            torch.cuda.synchronize()
            t = time.perf_counter()
            _, it_seq, _ = run_cases(cell, loads, tol=1e-8)
            torch.cuda.synchronize()
            t_seq = time.perf_counter() - t
            cell.close()
            cells = [Cell(n, "iso_phase", torch.from_numpy(phase), params, precision=prec) for _ in loads]
            with Batch(cells) as b:
                b.solve(loads, None, tol=1e-8)
                torch.cuda.synchronize()
                t = time.perf_counter()
                infos = b.solve(loads, None, tol=1e-8)
                torch.cuda.synchronize()
                t_b = time.perf_counter() - t
            for c in cells:
                c.close()
            key = f"{n[0]}x{n[1]}x{n[2]}_{prec}"
            out[key] = {"sequential_s": t_seq, "batched_s": t_b, "speedup": t_seq / t_b,
                        "pcg_iters_sequential": int(it_seq),
                        "pcg_iters_batched": int(sum(i["pcg_iters"] for i in infos))}
            log(f"[bench] six cases {key}: sequential {t_seq * 1e3:.1f} ms, one batch {t_b * 1e3:.1f} ms")
            if prec == "fp64":
                # block PCG: the six loads in one block Krylov space
                cell = Cell(n, "iso_phase", torch.from_numpy(phase), params, precision=prec)
                cell.solve_block(loads, tol=1e-8)
                torch.cuda.synchronize()
                t = time.perf_counter()
                binfos, applies = cell.solve_block(loads, tol=1e-8)
                torch.cuda.synchronize()
                t_blk = time.perf_counter() - t
                cell.close()
                out[key]["block_pcg_s"] = t_blk
                out[key]["block_pcg_iters"] = int(max(i["pcg_iters"] for i in binfos))
                out[key]["block_pcg_applies"] = int(applies)
                out[key]["block_pcg_speedup"] = t_seq / t_blk
                log(f"[bench] six cases {key}: block PCG {t_blk * 1e3:.1f} ms, "
                    f"{out[key]['block_pcg_iters']} block iterations, {applies} applies (sequential {it_seq})")
            if n[0] >= 128:
                # the six cases as independent solves on two streams
                # (dbfft_solve_many): do they fill each other's gaps?
                t_c = concurrent_cases(n, phase, params, prec, loads, nstream=2)
                out[key]["two_streams_s"] = t_c
                out[key]["two_streams_speedup"] = t_seq / t_c
                log(f"[bench] six cases {key}: two streams {t_c * 1e3:.1f} ms")
    return out


def concurrent_cases(n, phase, params, prec, loads, nstream):
    """Wall time of the load cases as independent solves on `nstream`
    concurrent streams (dbfft_solve_many: one helper context, stream and host
    thread per stream), helpers created and warmed first."""
    import torch
    from paper_1905_12725_amd.api import Cell
    with Cell(n, "iso_phase", torch.from_numpy(phase), params, precision=prec) as cell:
        cell.solve_many(loads, nstreams=nstream, tol=1e-8)
        torch.cuda.synchronize()
        t = time.perf_counter()
        cell.solve_many(loads, nstreams=nstream, tol=1e-8)
        torch.cuda.synchronize()
        return time.perf_counter() - t


def svk_porous_leg(log, n=(63, 63, 63), seed=6, ninc=5):
    """Sec. 3.3 workload: Saint Venant-Kirchhoff matrix (E = 70, nu = 0.3)
    with 5 random non-overlapping spherical pores at 20 % porosity (equal
    radii, seeded), the pores modelled as SVK inclusions 100 times softer;
    uniaxial elongation F = diag(2, 1, 1) (the other directions held) in 5
    increments, Newton tolerance 1e-6, PCG 1e-8 / 1e-10, FP64.  Both
    preconditioner policies: the mean tangent refreshed at every increment,
    and the initial tangent only (the paper's choice).  Per-increment
    counts come from solves to the first k increments (k = 1..5), which
    repeat the same increments."""
    import torch
    from paper_1905_12725_amd import microstructure as ms
    from paper_1905_12725_amd.api import Cell

    r = n[0] * (0.2 * 3.0 / (4.0 * np.pi * 5.0)) ** (1.0 / 3.0)
    phase, _, radii = ms.random_spheres(n, seed, r, r, 0.2)
    Fbar = np.diag([2.0, 1.0, 1.0])
    out = {"workload": f"{n[0]}^3 SVK matrix E = 70, nu = 0.3, {len(radii)} spherical pores (radius {r:.2f} "
                       f"voxels, seed {seed}) 100x softer, porosity {float(phase.mean()):.4f}; F = diag(2, 1, 1) "
                       f"in {ninc} increments; Newton tol 1e-6, PCG tol 1e-8 / 1e-10, FP64"}
    for name, refresh in (("refresh_every_increment", 0), ("initial_tangent", 1)):
        cum_pcg, cum_newton, times = [], [], []
        with Cell(n, "svk", torch.from_numpy(phase), [70.0, 0.3, 0.7, 0.3], kinematics="finite") as cell:
            for k in range(1, ninc + 1):
                Fk = np.eye(3) + (Fbar - np.eye(3)) * k / ninc
                torch.cuda.synchronize()
                t = time.perf_counter()
                info = cell.solve(Fk, None, n_increments=k, tol=1e-8, tol_load=1e-10, newton_tol=1e-6,
                                  refresh=refresh)
                times.append(time.perf_counter() - t)
                cum_pcg.append(int(info["pcg_iters"]))
                cum_newton.append(int(info["newton_iters"]))
        res = {"pcg_iters_per_increment": [cum_pcg[0]] + [b - a for a, b in zip(cum_pcg, cum_pcg[1:])],
               "newton_iters_per_increment": [cum_newton[0]] + [b - a for a, b in zip(cum_newton, cum_newton[1:])],
               "pcg_iters_total": cum_pcg[-1], "newton_iters_total": cum_newton[-1], "solve_s": times[-1],
               "P11_final": float(info["sigma_bar"][0, 0])}
        out[name] = res
        log(f"[bench] SVK porous {name}: PCG per increment {res['pcg_iters_per_increment']}, "
            f"Newton {res['newton_iters_per_increment']}, {times[-1]:.2f} s")
    return out


def contrast_sweep(log, grids=((63, 63, 63), (64, 64, 64))):
    """Iterations against phase contrast (Sec. 3.1 strain control, Sec. 3.2
    stress control): centred sphere inclusion at 20 %, matrix E = 70,
    inclusion E = k * 70 for k = 1e-5 ... 1e4, nu = 0.3; uniaxial strain
    1e-3, or uniaxial stress with the other five components zero; FP64 PCG
    to 1e-8 equilibrium and 1e-10 loading residual, at most 1e4 iterations.
    The odd 63^3 grid is the paper's; 64^3 is its power-of-two neighbour.
    Under strain control the two-level preconditioner (coarse_kc 1 and 2,
    through the block solver with one load) is swept beside M(xi)."""
    import torch
    from paper_1905_12725_amd import microstructure as ms
    from paper_1905_12725_amd.api import Cell

    ks = [10.0 ** e for e in range(-5, 5)]
    out = {"workload": "centred sphere inclusion at 20 %, E_m = 70, E_i = k E_m, nu = 0.3, FP64, "
                       "tol 1e-8 (equilibrium) / 1e-10 (loading)", "k": ks}
    for n in grids:
        phase = ms.centred_sphere(n, 0.2)
        for control in ("strain", "stress"):
            load = np.zeros((3, 3))
            mask = np.zeros((3, 3), bool)
            if control == "strain":
                load[0, 0] = 1e-3
            else:
                load[0, 0] = 0.07
                mask[:] = True
            iters, times = [], []
            for k in ks:
                with Cell(n, "iso_phase", torch.from_numpy(phase), [70.0, 0.3, 70.0 * k, 0.3]) as cell:
                    torch.cuda.synchronize()
                    t = time.perf_counter()
                    info = cell.solve(load, mask, tol=1e-8, tol_load=1e-10, max_iter=10000)
                    times.append(time.perf_counter() - t)
                iters.append(int(info["pcg_iters"]))
            key = f"{n[0]}x{n[1]}x{n[2]}_{control}"
            out[key] = {"pcg_iters": iters, "solve_s": times}
            log(f"[bench] contrast sweep {key}: iterations {iters}")
            if control == "strain":
                # the two-level preconditioner (exact operator block on the
                # coarse frequencies |m_a| <= kc) against M(xi) alone
                for kc in (1, 2):
                    its2 = []
                    for k in ks:
                        with Cell(n, "iso_phase", torch.from_numpy(phase), [70.0, 0.3, 70.0 * k, 0.3]) as cell:
                            (inf,), _ = cell.solve_block([load], mask, tol=1e-8, tol_load=1e-10, max_iter=10000,
                                                         coarse_kc=kc, raise_on_fail=False)
                        its2.append(int(inf["pcg_iters"]))
                    out[key][f"pcg_iters_two_level_kc{kc}"] = its2
                    log(f"[bench] contrast sweep {key}: two-level kc={kc} iterations {its2}")
    return out


# PCG tolerances tried, loosest first (about four per decade)
TOL_SWEEP = (1.0, 0.5, 0.3, 0.2, 0.1, 0.05, 0.03, 0.02, 0.01, 5e-3, 3e-3, 2e-3, 1e-3, 5e-4, 3e-4, 2e-4, 1e-4,
             5e-5, 3e-5, 2e-5, 1e-5, 5e-6, 3e-6, 2e-6, 1e-6, 1e-7, 1e-8)


def bracket_equal_accuracy(cell, mixed, loads, err, fo, log, target=1e-6, repeats=3):
    """Each precision timed at the loosest PCG tolerance whose effective
    stiffness meets `target` (max relative error against the tight FP64
    reference).  Tolerances are tried loosest first; the first that meets
    the target is timed `repeats` times (median), and the tolerance tried
    just before it (which missed) is reported beside it, so the chosen
    tolerance is bracketed.  FP32-mixed also sweeps the inner FP32 solve's
    relative tolerance and keeps the fastest setting."""
    import torch

    def run(c, tol, **kw):
        torch.cuda.synchronize()
        t = time.perf_counter()
        cols, it, rf = run_cases(c, loads, tol=tol, **fo, **kw)
        torch.cuda.synchronize()
        return time.perf_counter() - t, cols, it, rf

    def sweep(name, c, **kw):
        prev = None
        for tol in TOL_SWEEP:
            dt, cols, it, rf = run(c, tol, **kw)
            e = err(cols)
            log(f"[bench] {name} {kw} tol={tol:g}: {dt:.3f} s, {it} iters, Ceff rel err {e:.2e}")
            if e <= target:
                times = sorted([dt] + [run(c, tol, **kw)[0] for _ in range(repeats - 1)])
                return {"tol": tol, "time_s": times[len(times) // 2], "pcg_iters": it, "refine_steps": rf,
                        "ceff_rel_err": e, "bracketed": prev is not None,
                        "missed_at_looser_tol": prev, **{k: v for k, v in kw.items()}}
            prev = {"tol": tol, "ceff_rel_err": e, "pcg_iters": it}
        return None

    res = {"fp64": sweep("fp64", cell)}
    best = None
    variants = []
    for inner in (1e-1, 1e-2, 1e-3, 1e-4):
        r = sweep("fp32_mixed", mixed, inner_tol=inner)
        variants.append(r)
        if r is not None and (best is None or r["time_s"] < best["time_s"]):
            best = r
    res["fp32_mixed"] = best
    res["fp32_mixed_by_inner_tol"] = variants
    if res["fp64"] and best:
        res["speedup_fp32_mixed_vs_fp64"] = res["fp64"]["time_s"] / best["time_s"]
        # the same tolerances with the six cases as independent solves on two
        # concurrent streams (dbfft_solve_many; results identical to the
        # one-by-one solves)
        conc = {}
        for name, c, r, kw in (("fp64", cell, res["fp64"], {}),
                               ("fp32_mixed", mixed, best, {"inner_tol": best["inner_tol"]})):
            c.solve_many(loads, nstreams=2, tol=r["tol"], **fo, **kw)
            times = []
            for _ in range(repeats):
                torch.cuda.synchronize()
                t = time.perf_counter()
                infos = c.solve_many(loads, nstreams=2, tol=r["tol"], **fo, **kw)
                torch.cuda.synchronize()
                times.append(time.perf_counter() - t)
            conc[name] = {"tol": r["tol"], "time_s": sorted(times)[len(times) // 2],
                          "ceff_rel_err": err([i["sigma_bar"] for i in infos]),
                          "pcg_iters": int(sum(i["pcg_iters"] for i in infos))}
            log(f"[bench] {name} two streams tol={r['tol']:g}: {conc[name]['time_s']:.3f} s")
        conc["speedup_fp32_mixed_vs_fp64"] = conc["fp64"]["time_s"] / conc["fp32_mixed"]["time_s"]
        conc["speedup_fp32_mixed_two_streams_vs_fp64_one"] = res["fp64"]["time_s"] / conc["fp32_mixed"]["time_s"]
        res["two_streams"] = conc
    res["target_ceff_rel_err"] = target
    return res


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--n", type=int, default=128)
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-mixed", action="store_true")
    ap.add_argument("--no-batch", action="store_true")
    ap.add_argument("--no-sweep", action="store_true", help="skip the phase-contrast sweep")
    ap.add_argument("--no-svk", action="store_true", help="skip the porous SVK finite-strain workload")
    ap.add_argument("--no-multi", action="store_true", help="skip the six-cases-in-one-batch comparison")
    ap.add_argument("--no-configs", action="store_true", help="skip the J2 polycrystal and adjoint workloads")
    ap.add_argument("--batch-only", action="store_true",
                    help="only the batched FP32-mixed solve of the uneven neo-Hookean batch (for profiling)")
    ap.add_argument("--unfused", action="store_true", help="separate CG vector kernels (fused_cg = 0)")
    ap.add_argument("--precision", choices=("fp64", "fp32_mixed"), default="fp64",
                    help="precision of the timed leg (fp32_mixed: to profile the FP32 kernels; "
                         "the FP32-mixed comparison leg needs fp64 here and is skipped otherwise)")
    ap.add_argument("--cpu-worker", type=int, default=None, help=argparse.SUPPRESS)
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only copy a 1 GiB FP64 tensor three times (reference kernel for HBM byte counters)")
    args = ap.parse_args()
    if args.cpu_worker is not None:
        cpu_worker(args.cpu_worker, (args.n,) * 3, args.cpu_seconds)
        return
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py runs on one GPU: the DBFFT hot path here is a single-GPU build "
              "(no multi-GPU sharding); use --gpus 1", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_1905_12725_amd import microstructure as ms
    from paper_1905_12725_amd.api import Cell

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(2)
    if args.batch_only:
        print(json.dumps({"batched": batched_leg(lambda m: print(m, file=sys.stderr, flush=True),
                                                 only_batched=True)}), flush=True)
        return
    if args.copy_calibration:
        nbytes = 1 << 30
        a = torch.ones(nbytes // 8, dtype=torch.float64, device="cuda")
        b = torch.empty_like(a)
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"copy_calibration_bytes_read": nbytes, "copy_calibration_bytes_written": nbytes,
                          "launches": 3}), flush=True)
        return
    n = (args.n,) * 3
    phase, _, _ = ms.random_spheres(n, 2, 6.0, 10.0, 0.30)
    E, nu = [1.0, 100.0], 0.3
    params = [E[0], nu, E[1], nu]
    loads = mandel_loads()
    N = int(np.prod(n))
    log = lambda *a: print(*a, file=sys.stderr, flush=True)  # noqa: E731
    log(f"[bench] {n} spheres vf={phase.mean():.4f}, contrast 100, 6 load cases")

    cell = Cell(n, "iso_phase", torch.from_numpy(phase), params, precision=args.precision)
    fo = {"fused_cg": 0 if args.unfused else 1}
    wb = 8 if args.precision == "fp64" else 4
    for _ in range(args.warmup):
        run_cases(cell, loads, tol=1e-8, **fo)
    log("[bench] warmup done")

    cell.kernel_timing(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    total_iters = 0
    cols64 = None
    for s in range(args.steps):
        cols64, it, _ = run_cases(cell, loads, tol=1e-8, **fo)
        total_iters += it
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    ktime = cell.kernel_timing(False)
    log(f"[bench] timed {args.steps} steps: {elapsed:.3f} s, {total_iters} applies")

    applies_per_s = total_iters / elapsed
    per_kernel = {}
    fused = ktime.get("cg_update", (0.0, 0))[1] == 0
    for k, (ms_tot, cnt) in ktime.items():
        if cnt > 0:
            avg = ms_tot / cnt * 1e-3
            b = kernel_bytes(n, k, wb, fused)
            per_kernel[k] = {"avg_us": avg * 1e6, "launches": cnt, "total_ms": ms_tot,
                             "bytes_per_launch": b, "GBps": (b / avg / 1e9) if b else None}
    dom = max((k for k in per_kernel if per_kernel[k]["bytes_per_launch"] > 0),
              key=lambda k: per_kernel[k]["total_ms"])
    dk = per_kernel[dom]
    apply_kinds = ("x_inverse_grad", "y_inverse", "z_fused_tangent", "y_forward", "x_forward_div")
    apply_us = sum(per_kernel[k]["avg_us"] for k in apply_kinds if k in per_kernel)
    apply_bytes = sum(kernel_bytes(n, k, wb, fused) for k in apply_kinds)
    iter_kinds = apply_kinds + ("cg_alpha", "cg_update", "cg_beta", "cg_direction")
    iter_us = sum(per_kernel[k]["avg_us"] for k in iter_kinds if k in per_kernel)
    iter_bytes = sum(kernel_bytes(n, k, wb, fused) for k in iter_kinds)

    out = {
        "metric": METRIC,
        "value": applies_per_s,
        "unit": "applies/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": elapsed / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if args.precision == "fp64" else "f32+f64",
        "data": "synthetic",
        "config": {
            "workload": f"{n[0]}^3 two-phase random spheres (radius 6-10 voxels, 30 % volume fraction, seed 2), "
                        "stiffness contrast 100, nu 0.3, six Mandel strain load cases, PCG tol 1e-8, "
                        + ("FP64" if args.precision == "fp64" else "FP32-mixed"),
            "grid": list(n),
            "volume_fraction": float(phase.mean()),
            "load_cases": 6,
            "pcg_iterations_per_step": total_iters // args.steps,
        },
        "gvoxel_dof_per_s": 3.0 * N * applies_per_s / 1e9,
        "hbm_model": {
            "apply_bytes": apply_bytes,
            "apply_us_kernels": apply_us,
            "apply_frac_of_peak": apply_bytes / (apply_us * 1e-6) / 1e9 / HBM_PEAK_GBS,
            "iteration_bytes": iter_bytes,
            "iteration_us_kernels": iter_us,
            "iteration_frac_of_peak": iter_bytes / (iter_us * 1e-6) / 1e9 / HBM_PEAK_GBS,
            "iteration_us_wall": 1e6 / applies_per_s,
            "whole_job_frac_of_peak": iter_bytes * applies_per_s / 1e9 / HBM_PEAK_GBS,
        },
        "kernels": per_kernel,
        "roofline": {
            "bound": "hbm",
            "kernel": dom,
            "achieved": dk["GBps"],
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": dk["GBps"] / HBM_PEAK_GBS,
            "traffic": measured_traffic(n, dom, args.precision),
        },
    }

    # tight FP64 reference for accuracy, then FP32-mixed vs FP64 at equal accuracy
    if not args.no_mixed and args.precision == "fp64":
        ref_cols, _, _ = run_cases(cell, loads, tol=1e-10, tol_load=1e-10, **fo)
        Cref = ceff(ref_cols)

        def err(cols):
            return float(np.max(np.abs(ceff(cols) - Cref)) / np.max(np.abs(Cref)))

        mixed = Cell(n, "iso_phase", torch.from_numpy(phase), params, precision="fp32_mixed")
        run_cases(mixed, loads, tol=1e-8, **fo)  # warm
        # per-kernel HIP-event times of the FP32 inner iterations (tol 1e-8 solves)
        mixed.kernel_timing(True)
        run_cases(mixed, loads, tol=1e-8, **fo)
        kt32 = mixed.kernel_timing(False)
        out["fp32_mixed_kernels_us"] = {k: ms_tot / cnt * 1e3 for k, (ms_tot, cnt) in kt32.items() if cnt > 0}
        res = bracket_equal_accuracy(cell, mixed, loads, err, fo, log)
        mixed.close()
        out["equal_accuracy_1e-6"] = res
        out["ceff_rel_err_fp64_tol1e-8"] = err(cols64)
    cell.close()

    if not args.no_batch:
        out["batched"] = batched_leg(log)
    if not args.no_sweep:
        out["contrast_sweep"] = contrast_sweep(log)
    if not args.no_svk:
        out["svk_porous"] = svk_porous_leg(log)
    if not args.no_multi:
        out["multi_rhs"] = multi_rhs_leg(log)
    if not args.no_configs:
        out["j2_polycrystal"] = j2_polycrystal_leg(log)
        out["adjoint"] = adjoint_leg(log)

    if not args.no_cpu_baseline:
        log("[bench] CPU oracle baseline ...")
        out["cpu_baseline"] = cpu_baseline(n, args.cpu_seconds)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
