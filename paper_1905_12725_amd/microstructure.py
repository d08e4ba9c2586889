"""Seeded synthetic microstructures and load descriptions.

These generators produce the *inputs* of a homogenization problem (phase
maps, grain maps, orientations, modulus fields, grid sizes).  They contain
none of the DBFFT arithmetic: no frequencies, no gradients, no constitutive
update.  Both the HIP path and the CPU oracle consume the arrays they return,
so the two sides see identical bytes.

Workload shapes follow the paper's numerical examples (Sec. 3: a centred
spherical inclusion at 20 % volume fraction, random spherical pores/
inclusions, a Voronoi polycrystal with random orientations) scaled to the
grids used here, plus a log-normal random modulus field.

Conventions fixed here (not in the paper):
  * voxel (i, j, k) has its centre at ((i + 0.5)/n1, (j + 0.5)/n2, (k + 0.5)/n3)
    on the unit cell; a voxel belongs to a sphere when the periodic minimum-
    image distance of its centre to the sphere centre is <= r;
  * Voronoi ties go to the lowest seed index;
  * every random draw uses numpy.random.default_rng(seed) (PCG64).
"""
from __future__ import annotations

import numpy as np

__all__ = [
    "voxel_centres",
    "centred_sphere",
    "random_spheres",
    "voronoi_grains",
    "random_rotations",
    "lognormal_modulus",
    "smooth_batch_sizes",
    "laminate",
]


def voxel_centres(n):
    """Coordinates of voxel centres on the unit cell, each of shape n."""
    n1, n2, n3 = n
    x = (np.arange(n1) + 0.5) / n1
    y = (np.arange(n2) + 0.5) / n2
    z = (np.arange(n3) + 0.5) / n3
    return np.meshgrid(x, y, z, indexing="ij")


def _periodic_dist2(n, centre):
    """Squared periodic minimum-image distance (in voxel units) of every voxel
    centre to `centre` (voxel units, float triple)."""
    d2 = np.zeros(tuple(n))
    for ax in range(3):
        shape = [1, 1, 1]
        shape[ax] = n[ax]
        c = np.arange(n[ax]) + 0.5 - centre[ax]
        c = c - n[ax] * np.round(c / n[ax])
        d2 = d2 + (c ** 2).reshape(shape)
    return d2


def _mark_sphere(phase, centre, r):
    """Set phase = 1 on voxels whose centre lies within periodic distance r
    of `centre` (voxel units), visiting only the sphere's bounding box."""
    n = phase.shape
    idx, d2 = [], []
    for ax in range(3):
        lo = int(np.floor(centre[ax] - r - 0.5)) - 1
        hi = int(np.ceil(centre[ax] + r - 0.5)) + 1
        k = np.arange(lo, hi + 1)
        k = np.unique(np.mod(k, n[ax]))
        dd = k + 0.5 - centre[ax]
        dd = dd - n[ax] * np.round(dd / n[ax])
        idx.append(k)
        d2.append(dd * dd)
    D = d2[0][:, None, None] + d2[1][None, :, None] + d2[2][None, None, :]
    sub = np.ix_(idx[0], idx[1], idx[2])
    old = phase[sub]
    inside = D <= r * r
    phase[sub] = np.where(inside, np.uint8(1), old)
    return int(np.count_nonzero(inside & (old == 0)))


def centred_sphere(n, volume_fraction=0.2):
    """uint8 phase map: 1 inside a sphere centred in the cell, 0 elsewhere.

    The radius (in voxels of the first axis) gives the requested volume
    fraction in the continuum: r = n1 * (3 vf / (4 pi))^(1/3).  The voxel
    fraction differs slightly (e.g. 840/4096 = 20.51 % at 16^3)."""
    n = tuple(int(v) for v in n)
    r = n[0] * (3.0 * volume_fraction / (4.0 * np.pi)) ** (1.0 / 3.0)
    centre = (n[0] / 2.0, n[1] / 2.0, n[2] / 2.0)
    return (_periodic_dist2(n, centre) <= r * r).astype(np.uint8)


def random_spheres(n, seed, rmin, rmax, volume_fraction, max_tries=200000):
    """uint8 phase map of seeded, non-overlapping periodic spheres.

    Radii are U[rmin, rmax] voxels, centres U[0, n)^3.  A candidate is accepted
    when its periodic centre distance to every accepted sphere is >= r_i + r_j.
    Placement stops once the voxel fraction reaches `volume_fraction`.
    Returns (phase, centres, radii)."""
    n = tuple(int(v) for v in n)
    rng = np.random.default_rng(seed)
    phase = np.zeros(n, dtype=np.uint8)
    centres = np.zeros((0, 3))
    radii = np.zeros(0)
    nn = np.array(n, dtype=float)
    nvox = float(np.prod(n))
    filled = 0
    tries = 0
    while filled / nvox < volume_fraction:
        tries += 1
        if tries > max_tries:
            raise RuntimeError("random_spheres: could not reach the volume fraction")
        r = rng.uniform(rmin, rmax)
        c = rng.uniform(0.0, 1.0, size=3) * nn
        if len(radii):
            d = c[None, :] - centres
            d = d - nn * np.round(d / nn)
            if np.any(np.sqrt(np.sum(d * d, axis=1)) < r + radii):
                continue
        centres = np.vstack([centres, c[None, :]])
        radii = np.append(radii, r)
        filled += _mark_sphere(phase, c, r)
    return phase, centres, radii


def voronoi_grains(n, ngrains, seed):
    """int32 grain map of a periodic Voronoi tessellation with `ngrains` seeds
    drawn U[0, n)^3 (voxel units).  Ties go to the lowest seed index."""
    n = tuple(int(v) for v in n)
    rng = np.random.default_rng(seed)
    seeds = rng.uniform(0.0, 1.0, size=(ngrains, 3)) * np.array(n, dtype=float)
    best = np.full(n, np.inf)
    grain = np.zeros(n, dtype=np.int32)
    for g in range(ngrains):
        d2 = _periodic_dist2(n, seeds[g])
        closer = d2 < best
        best = np.where(closer, d2, best)
        grain = np.where(closer, np.int32(g), grain)
    return grain, seeds


def random_rotations(count, seed):
    """(count, 3, 3) rotation matrices, uniform on SO(3), from normalized
    4-D Gaussian quaternions."""
    rng = np.random.default_rng(seed)
    q = rng.standard_normal(size=(count, 4))
    q /= np.linalg.norm(q, axis=1, keepdims=True)
    w, x, y, z = q[:, 0], q[:, 1], q[:, 2], q[:, 3]
    R = np.empty((count, 3, 3))
    R[:, 0, 0] = 1 - 2 * (y * y + z * z)
    R[:, 0, 1] = 2 * (x * y - z * w)
    R[:, 0, 2] = 2 * (x * z + y * w)
    R[:, 1, 0] = 2 * (x * y + z * w)
    R[:, 1, 1] = 1 - 2 * (x * x + z * z)
    R[:, 1, 2] = 2 * (y * z - x * w)
    R[:, 2, 0] = 2 * (x * z - y * w)
    R[:, 2, 1] = 2 * (y * z + x * w)
    R[:, 2, 2] = 1 - 2 * (x * x + y * y)
    return R


def lognormal_modulus(n, seed, corr_len=8.0, sigma_log=1.0):
    """Per-voxel Young's modulus E = exp(sigma_log * g), g a standardized
    Gaussian random field with squared-exponential spectrum of correlation
    length `corr_len` voxels: g = IFFT[sqrt(S(k)) FFT[w]], w white N(0,1),
    S(k) = exp(-|k|^2 l^2 / 2) with |k| = 2 pi m / n in voxel units."""
    n = tuple(int(v) for v in n)
    rng = np.random.default_rng(seed)
    w = rng.standard_normal(size=n)
    k2 = np.zeros(n)
    for ax in range(3):
        shape = [1, 1, 1]
        shape[ax] = n[ax]
        m = np.fft.fftfreq(n[ax]) * 2.0 * np.pi  # 2 pi m / n
        k2 = k2 + (m ** 2).reshape(shape)
    spec = np.sqrt(np.exp(-k2 * corr_len ** 2 / 2.0))
    g = np.real(np.fft.ifftn(spec * np.fft.fftn(w)))
    g = (g - g.mean()) / g.std()
    return np.exp(sigma_log * g)


SMOOTH_EVEN_SIZES = (32, 36, 40, 48, 50, 54, 60, 64, 72, 80, 90, 96)


def smooth_batch_sizes(count, seed, sizes=SMOOTH_EVEN_SIZES):
    """`count` cubic grid sizes drawn uniformly from the even 2*3*5-smooth
    sizes in [32, 96]."""
    rng = np.random.default_rng(seed)
    return [int(sizes[i]) for i in rng.integers(0, len(sizes), size=count)]


def laminate(n, axis, thicknesses):
    """uint8 phase map of a periodic laminate whose layers are normal to
    `axis`; `thicknesses` lists consecutive layer thicknesses in voxels, the
    layer index modulo 2 gives the phase (starting with phase 0)."""
    n = tuple(int(v) for v in n)
    if sum(thicknesses) != n[axis]:
        raise ValueError("layer thicknesses must add up to the grid size")
    line = np.concatenate([np.full(t, i % 2, dtype=np.uint8)
                           for i, t in enumerate(thicknesses)])
    shape = [1, 1, 1]
    shape[axis] = n[axis]
    return np.broadcast_to(line.reshape(shape), n).copy()
