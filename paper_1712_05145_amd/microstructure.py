"""Seeded synthetic microstructures (inputs only; none of the solver arithmetic).

Every generator returns a phase-id voxel array (uint16, C-order, grid axis d
carries x_{d+1}, cell [-1/2, 1/2)^3 sampled at voxel centres) and a per-phase
table of isotropic Lame pairs (lambda, mu).  Randomness comes from
``numpy.random.default_rng(seed)`` only.  Both the GPU path and the CPU
oracle consume these arrays unchanged.

Shapes follow the paper's kind of example (Sec. 4: a coated inclusion in a
matrix) and the benchmark workloads: one centred sphere, random spheres,
a Voronoi polycrystal, aligned fibres, laminates.
"""
import math

import numpy as np

__all__ = [
    "lame_from_young", "midpoint_reference", "voxel_centres",
    "centred_sphere", "random_spheres", "overlapping_spheres", "voronoi_polycrystal",
    "hex_fibres", "laminate", "coated_sphere", "random_phases", "serving_requests",
]


def lame_from_young(young, nu):
    """3-D isotropic Lame parameters from Young's modulus and Poisson's ratio."""
    young = np.asarray(young, dtype=np.float64)
    nu = np.asarray(nu, dtype=np.float64)
    lam = young * nu / ((1.0 + nu) * (1.0 - 2.0 * nu))
    mu = young / (2.0 * (1.0 + nu))
    return np.stack([lam, mu], axis=-1)


def midpoint_reference(lame):
    """Reference Lame pair: midpoint of the phase min/max of lambda and of mu."""
    lame = np.asarray(lame, dtype=np.float64).reshape(-1, 2)
    lam0 = 0.5 * (lame[:, 0].min() + lame[:, 0].max())
    mu0 = 0.5 * (lame[:, 1].min() + lame[:, 1].max())
    return float(lam0), float(mu0)


def voxel_centres(n):
    return -0.5 + (np.arange(n) + 0.5) / n


def _min_image(d):
    return d - np.round(d)


def centred_sphere(n, volume_fraction=0.2, young=(1.0, 10.0), nu=(0.3, 0.3)):
    """One sphere at the origin; phase 1 = inclusion."""
    if np.isscalar(n):
        n = (n, n, n)
    r = (3.0 * volume_fraction / (4.0 * math.pi)) ** (1.0 / 3.0)
    y = [voxel_centres(m) for m in n]
    d2 = y[0][:, None, None] ** 2 + y[1][None, :, None] ** 2 + y[2][None, None, :] ** 2
    phase = (d2 < r * r).astype(np.uint16)
    return phase, lame_from_young(young, nu)


def _paint_sphere(phase, centre, radius, value):
    n = phase.shape
    idx = []
    for d in range(3):
        lo = math.floor((centre[d] - radius + 0.5) * n[d] - 0.5)
        hi = math.ceil((centre[d] + radius + 0.5) * n[d] - 0.5)
        js = np.arange(lo, hi + 1)
        idx.append(js)
    y = [(-0.5 + (js + 0.5) / n[d]) for d, js in enumerate(idx)]
    d2 = (_min_image(y[0] - centre[0])[:, None, None] ** 2
          + _min_image(y[1] - centre[1])[None, :, None] ** 2
          + _min_image(y[2] - centre[2])[None, None, :] ** 2)
    inside = d2 < radius * radius
    ii = np.ix_(idx[0] % n[0], idx[1] % n[1], idx[2] % n[2])
    block = phase[ii]
    block[inside] = value
    phase[ii] = block


def random_spheres(n, count=20, rmin=0.05, rmax=0.12, seed=2, young=(1.0, 100.0), nu=(0.3, 0.3),
                   max_tries=100000):
    """Random sequential addition of non-overlapping spheres (periodic minimum image)."""
    if np.isscalar(n):
        n = (n, n, n)
    rng = np.random.default_rng(seed)
    centres, radii = [], []
    tries = 0
    while len(centres) < count:
        tries += 1
        if tries > max_tries:
            raise RuntimeError("random sequential addition did not place all spheres")
        r = rng.uniform(rmin, rmax)
        c = rng.uniform(-0.5, 0.5, size=3)
        ok = True
        for c2, r2 in zip(centres, radii):
            if np.linalg.norm(_min_image(c - c2)) < r + r2:
                ok = False
                break
        if ok:
            centres.append(c)
            radii.append(r)
    phase = np.zeros(n, dtype=np.uint16)
    for c, r in zip(centres, radii):
        _paint_sphere(phase, c, r, 1)
    return phase, lame_from_young(young, nu)


def overlapping_spheres(n, target_fraction, contrast, seed, rmin=0.05, rmax=0.12, nu=0.3):
    """Spheres added (overlap allowed) until the voxel fraction reaches the target."""
    if np.isscalar(n):
        n = (n, n, n)
    rng = np.random.default_rng(seed)
    phase = np.zeros(n, dtype=np.uint16)
    while phase.mean() < target_fraction:
        _paint_sphere(phase, rng.uniform(-0.5, 0.5, size=3), rng.uniform(rmin, rmax), 1)
    return phase, lame_from_young((1.0, contrast), (nu, nu))


def voronoi_polycrystal(n, grains=200, seed=3, lame_range=(1.0, 50.0)):
    """Periodic Voronoi tessellation; grain Lame pairs log-uniform in lame_range."""
    from scipy.spatial import cKDTree
    if np.isscalar(n):
        n = (n, n, n)
    rng = np.random.default_rng(seed)
    seeds = rng.uniform(-0.5, 0.5, size=(grains, 3))
    lo, hi = math.log(lame_range[0]), math.log(lame_range[1])
    lam = np.exp(rng.uniform(lo, hi, size=grains))
    mu = np.exp(rng.uniform(lo, hi, size=grains))
    tree = cKDTree(seeds + 0.5, boxsize=1.0)
    phase = np.empty(n, dtype=np.uint16)
    y1 = voxel_centres(n[1]) + 0.5
    y2 = voxel_centres(n[2]) + 0.5
    g1, g2 = np.meshgrid(y1, y2, indexing="ij")
    plane = np.stack([np.zeros_like(g1), g1, g2], axis=-1).reshape(-1, 3)
    y0 = voxel_centres(n[0]) + 0.5
    for i0 in range(n[0]):
        plane[:, 0] = y0[i0]
        _, idx = tree.query(plane, k=1)
        phase[i0] = idx.reshape(n[1], n[2]).astype(np.uint16)
    return phase, np.stack([lam, mu], axis=-1)


def hex_fibres(n, radius=0.04, rows=10, cols=7, jitter=0.015, seed=5,
               young=(1.0, 1000.0), nu=(0.35, 0.25)):
    """Fibres parallel to x3 on a staggered lattice, jittered with rejection."""
    if np.isscalar(n):
        n = (n, n, n)
    rng = np.random.default_rng(seed)
    min_gap = 2 * radius + 2.0 / max(n)
    centres = []
    for r in range(rows):
        for c in range(cols):
            base = np.array([-0.5 + (r + 0.5) * (1.0 / rows),
                             -0.5 + (c + 0.5) / cols + (0.5 / cols if r % 2 else 0.0)])
            for _ in range(1000):
                cand = base + rng.uniform(-jitter, jitter, size=2)
                if all(np.linalg.norm(_min_image(cand - o)) >= min_gap for o in centres):
                    centres.append(cand)
                    break
            else:
                centres.append(base)
    y0 = voxel_centres(n[0])
    y1 = voxel_centres(n[1])
    plane = np.zeros((n[0], n[1]), dtype=np.uint16)
    for c in centres:
        d2 = _min_image(y0 - c[0])[:, None] ** 2 + _min_image(y1 - c[1])[None, :] ** 2
        plane[d2 < radius * radius] = 1
    phase = np.repeat(plane[:, :, None], n[2], axis=2).astype(np.uint16)
    return phase, lame_from_young(young, nu)


def laminate(n, layer_ids, axis=2):
    """Phase array constant in the planes normal to ``axis``; layer_ids[j] is the
    phase of slice j along that axis (len(layer_ids) == n[axis])."""
    if np.isscalar(n):
        n = (n, n, n)
    ids = np.asarray(layer_ids, dtype=np.uint16)
    shp = [1, 1, 1]
    shp[axis] = n[axis]
    return np.broadcast_to(ids.reshape(shp), n).copy()


def coated_sphere(n, r1=0.25, r2=0.4):
    """Hashin-type coated inclusion: 0 core (|y| < r1), 1 coating, 2 matrix."""
    if np.isscalar(n):
        n = (n, n, n)
    y = [voxel_centres(m) for m in n]
    d = np.sqrt(y[0][:, None, None] ** 2 + y[1][None, :, None] ** 2 + y[2][None, None, :] ** 2)
    phase = np.full(n, 2, dtype=np.uint16)
    phase[d < r2] = 1
    phase[d < r1] = 0
    return phase


def plane_stress_lame(lame):
    """(lambda, mu) rows -> plane-stress in-plane moduli (2 lam mu / (lam + 2 mu), mu)."""
    lame = np.asarray(lame, dtype=np.float64)
    lam, mu = lame[:, 0], lame[:, 1]
    return np.stack([2.0 * lam * mu / (lam + 2.0 * mu), mu], axis=1)


def hashin_2d(n, r1=0.25, r2=0.4, young=(100.0, 1000.0, 453.685), nu=0.3):
    """Hashin's coated circular inclusion of Sec. 4 on a (1, n, n) grid: the
    plane is (x2, x3), every field is invariant along x1.  Phases: 0 core
    (radius r1), 1 coating (radius r2), 2 matrix; plane-stress moduli.  The
    default moduli are the paper's, with the matrix modulus that makes the
    coated inclusion neutral."""
    y = voxel_centres(n)
    d = np.sqrt(y[:, None] ** 2 + y[None, :] ** 2)
    plane = np.full((n, n), 2, dtype=np.uint16)
    plane[d < r2] = 1
    plane[d < r1] = 0
    lame = plane_stress_lame(lame_from_young(np.asarray(young, float), [nu] * len(young)))
    return plane[None, :, :], lame


def hashin_2d_contrast(n, contrast, r1=0.25, r2=0.4, nu=0.3):
    """The same geometry with core E = 1, coating E = contrast and the neutral
    matrix modulus for that pair (2-D neutral-coating condition, plane stress)."""
    e1, e2 = 1.0, float(contrast)
    k1, k2 = e1 / (2 * (1 - nu)), e2 / (2 * (1 - nu))
    mu2 = e2 / (2 * (1 + nu))
    f = (r1 / r2) ** 2
    k3 = k2 + f / (1.0 / (k1 - k2) + (1 - f) / (k2 + mu2)) if e1 != e2 else k1
    return hashin_2d(n, r1, r2, young=(e1, e2, 2 * k3 * (1 - nu)), nu=nu)


def random_phases(n, nphases, seed):
    """Independent random phase per voxel (worst case for the constitutive law)."""
    if np.isscalar(n):
        n = (n, n, n)
    rng = np.random.default_rng(seed)
    return rng.integers(0, nphases, size=n).astype(np.uint16)


def serving_requests(count=512, rate=40.0, sizes=(32, 48, 64, 96, 128), seed=4):
    """Request stream: Poisson arrivals, grid size, inclusion fraction and contrast."""
    rng = np.random.default_rng(seed)
    arrivals = np.cumsum(rng.exponential(1.0 / rate, size=count))
    out = []
    for i in range(count):
        out.append({
            "id": i,
            "arrival": float(arrivals[i]),
            "n": int(rng.choice(sizes)),
            "fraction": float(rng.uniform(0.1, 0.4)),
            "contrast": float(rng.uniform(5.0, 500.0)),
            "seed": int(rng.integers(0, 2 ** 31 - 1)),
        })
    return out
