"""Seeded geometry and initial-field generators.

Every generator is deterministic for a given seed (``numpy.random.default_rng``,
PCG64). The workloads stand in for the paper's benchmark geometries, which are
not available: the empty channel of Sect. 5.1 is reproduced exactly, while the
real fixed-bed reactor and foam of Sect. 1 and Sect. 5.1 are replaced by a
relaxed random sphere pack and a thresholded smoothed-noise foam of the same
kind of structure.
"""

from __future__ import annotations

import math

import numpy as np


# --------------------------------------------------------------------------
# masks
# --------------------------------------------------------------------------

def channel_mask(nx: int = 500, ny: int = 100, nz: int = 100) -> np.ndarray:
    """Empty square channel along x with one-voxel walls on the y and z faces.

    Sect. 5.1 describes a 500x100x100 channel with about 4.8e6 fluid nodes;
    walls occupying the outermost y and z layers of the box give
    500 * 98 * 98 = 4,802,000 fluid nodes.
    """
    m = np.zeros((nx, ny, nz), dtype=np.uint8)
    m[:, 0, :] = 1
    m[:, ny - 1, :] = 1
    m[:, :, 0] = 1
    m[:, :, nz - 1] = 1
    return m


def _stamp_sphere(mask, c, r, periodic, owner=None, label=0):
    """Mark voxels v with |v - c| <= r (minimum image on periodic axes)."""
    shape = mask.shape
    idx = []
    off = []
    for a in range(3):
        lo = int(math.floor(c[a] - r))
        hi = int(math.ceil(c[a] + r))
        v = np.arange(lo, hi + 1)
        d = v - c[a]
        if periodic[a]:
            v = np.mod(v, shape[a])
        else:
            keep = (v >= 0) & (v < shape[a])
            v = v[keep]
            d = d[keep]
        idx.append(v)
        off.append(d)
    if any(len(v) == 0 for v in idx):
        return 0
    d2 = (off[0][:, None, None] ** 2 + off[1][None, :, None] ** 2
          + off[2][None, None, :] ** 2)
    inside = d2 <= r * r
    ix, iy, iz = np.ix_(idx[0], idx[1], idx[2])
    sub = mask[ix, iy, iz]
    new = inside & (sub == 0)
    sub[inside] = 1
    mask[ix, iy, iz] = sub
    if owner is not None:
        o = owner[ix, iy, iz]
        o[new] = label
        owner[ix, iy, iz] = o
    return int(new.sum())


def _min_image(d, shape, periodic):
    d = d.copy()
    for a in range(3):
        if periodic[a]:
            d[..., a] -= shape[a] * np.round(d[..., a] / shape[a])
    return d


def rsa_spheres(shape=(32, 32, 32), radius=3.0, solid_fraction=0.20,
                periodic=(True, False, False), seed=0,
                max_tries=1_000_000) -> np.ndarray:
    """Random sequential addition of non-overlapping spheres.

    Centres are drawn uniformly in the box; a candidate is rejected if its
    centre lies closer than ``2*radius`` to an accepted one (minimum image on
    periodic axes). Spheres are added until the solid voxel fraction reaches
    ``solid_fraction``. Spheres are cut by the box on non-periodic axes.
    """
    rng = np.random.default_rng(seed)
    shape = tuple(int(s) for s in shape)
    mask = np.zeros(shape, dtype=np.uint8)
    total = float(np.prod(shape))
    centres = np.zeros((0, 3))
    solid = 0
    tries = 0
    while solid / total < solid_fraction:
        tries += 1
        if tries > max_tries:
            raise RuntimeError("rsa_spheres: could not reach the solid fraction")
        c = rng.random(3) * np.array(shape, dtype=np.float64)
        if len(centres):
            d = _min_image(centres - c, shape, periodic)
            if np.min(np.einsum("ij,ij->i", d, d)) < (2 * radius) ** 2:
                continue
        centres = np.vstack([centres, c])
        solid += _stamp_sphere(mask, c, radius, periodic)
    return mask


def relaxed_spheres(shape=(512, 128, 128), radius=8.0, porosity=0.40, seed=0,
                    tol=0.005, max_sweeps=50_000) -> np.ndarray:
    """Dense random pack of equal, non-overlapping spheres.

    Random sequential addition jams near a solid fraction of 0.38, so dense
    packs are made by collective rearrangement: ``n`` centres are drawn
    uniformly in a fully periodic box and overlapping pairs are pushed apart
    symmetrically along their centre line (Jacobi sweeps) until no two centres
    are closer than ``2*radius``. Voxels within ``radius`` of a centre
    (minimum image on all axes) are solid. Spheres are disjoint, so the solid
    fraction is trimmed to the target by dropping whole spheres.
    """
    from scipy.spatial import cKDTree

    rng = np.random.default_rng(seed)
    shape = tuple(int(s) for s in shape)
    L = np.array(shape, dtype=np.float64)
    vol = float(np.prod(shape))
    target_solid = 1.0 - porosity
    n = int(round(target_solid * vol / (4.0 / 3.0 * math.pi * radius ** 3) * 1.01)) + 1
    p = rng.random((n, 3)) * L
    d0 = 2.0 * radius
    for _ in range(max_sweeps):
        pairs = cKDTree(p, boxsize=L).query_pairs(d0, output_type="ndarray")
        if len(pairs) == 0:
            break
        i, j = pairs[:, 0], pairs[:, 1]
        d = p[j] - p[i]
        d -= L * np.round(d / L)
        dist = np.maximum(np.sqrt(np.einsum("ij,ij->i", d, d)), 1e-9)
        push = (d0 * (1.0 + 1e-3) - dist) * 0.5
        v = d * (push / dist)[:, None]
        disp = np.zeros_like(p)
        np.add.at(disp, i, -v)
        np.add.at(disp, j, v)
        p = np.mod(p + disp, L)
    else:
        raise RuntimeError("relaxed_spheres: overlap removal did not converge")
    mask = np.zeros(shape, dtype=np.uint8)
    counts = np.array([_stamp_sphere(mask, c, radius, (True, True, True)) for c in p])
    # drop spheres from the end (placement order is random) towards the target
    solid = counts.sum()
    k = n
    while k > 0 and solid / vol > target_solid + 0.5 * tol:
        k -= 1
        solid -= counts[k]
    if abs(solid / vol - target_solid) > tol:
        raise RuntimeError("relaxed_spheres: porosity %.4f outside tolerance"
                           % (1.0 - solid / vol))
    if k < n:
        mask[:] = 0
        for c in p[:k]:
            _stamp_sphere(mask, c, radius, (True, True, True))
    return mask


def foam(shape=(384, 384, 384), sigma=4.0, porosity=0.85, seed=0) -> np.ndarray:
    """Foam-like medium: smoothed Gaussian noise, thresholded.

    White noise is smoothed with a periodic Gaussian filter of width ``sigma``
    voxels; the top ``1 - porosity`` quantile becomes solid.
    """
    from scipy.ndimage import gaussian_filter

    rng = np.random.default_rng(seed)
    g = gaussian_filter(rng.standard_normal(tuple(shape)), sigma=sigma, mode="wrap")
    thr = np.quantile(g, porosity)
    return (g > thr).astype(np.uint8)


# --------------------------------------------------------------------------
# fields
# --------------------------------------------------------------------------

def init_fields(shape, seed=0, rho_amp=1e-3, u_amp=1e-2):
    """Seeded initial density and velocity fields on the full voxel box.

    Returns ``(rho, u)`` with ``rho`` of shape ``shape`` and ``u`` of shape
    ``(3,) + shape``, both float64: rho = 1 + rho_amp * N(0,1) and
    u = u_amp * N(0,1) per component.
    """
    rng = np.random.default_rng(seed)
    shape = tuple(int(s) for s in shape)
    rho = 1.0 + rho_amp * rng.standard_normal(shape)
    u = u_amp * rng.standard_normal((3,) + shape)
    return rho, u


def pbb_fraction(mask: np.ndarray, seed=0) -> np.ndarray:
    """Seeded partial-bounce-back solid fraction per voxel.

    Fluid voxels that touch a solid voxel (26-neighbourhood, periodic wrap)
    get a value drawn from U[0, 1); all other voxels get 0.
    """
    from scipy.ndimage import binary_dilation

    rng = np.random.default_rng(seed)
    solid = mask != 0
    near = binary_dilation(np.pad(solid, 1, mode="wrap"),
                           structure=np.ones((3, 3, 3), bool))[1:-1, 1:-1, 1:-1]
    ns = rng.random(mask.shape)
    ns[~near | solid] = 0.0
    return ns


# --------------------------------------------------------------------------
# named workloads
# --------------------------------------------------------------------------

WORKLOADS = {
    # the paper's empty channel (Sect. 5.1), LS with B=1 (Sect. 5.6)
    "channel-500x100x100": dict(
        shape=(500, 100, 100), periodic=(True, False, False), tau=0.8,
        force=(1e-6, 0.0, 0.0), order="lex", block=1, steps=1000),
    # 32^3 spheres of radius 3 at porosity 0.8: the parity case
    "spheres-32": dict(
        shape=(32, 32, 32), periodic=(True, False, False), tau=0.8,
        force=(1e-6, 0.0, 0.0), order="lex", block=0, steps=100),
    # fixed-bed stand-in: radius-8 sphere pack at porosity 0.40
    "spherepack-512x128x128": dict(
        shape=(512, 128, 128), periodic=(True, False, False), tau=0.6,
        force=(1e-6, 0.0, 0.0), order="lex", block=64, steps=1000),
    # foam stand-in: smoothed noise at porosity 0.85
    "foam-384": dict(
        shape=(384, 384, 384), periodic=(True, False, False), tau=0.7,
        force=(1e-6, 0.0, 0.0), order="lex", block=0, steps=500),
    # the same foam at 512^3 (114 M fluid nodes): its PDF grids hold more
    # than 2^31 - 1 elements, so the time step addresses them with 64-bit
    # offsets
    "foam-512": dict(
        shape=(512, 512, 512), periodic=(True, False, False), tau=0.7,
        force=(1e-6, 0.0, 0.0), order="lex", block=0, steps=500),
    # the same foam at 768^3 (385 M fluid nodes, a 59 GB FP64 grid)
    "foam-768": dict(
        shape=(768, 768, 768), periodic=(True, False, False), tau=0.7,
        force=(1e-6, 0.0, 0.0), order="lex", block=0, steps=500),
    # the same foam at 1024^3 (about 913 M fluid nodes, a 139 GB FP64 grid):
    # one GPU's memory nearly full
    "foam-1024": dict(
        shape=(1024, 1024, 1024), periodic=(True, False, False), tau=0.7,
        force=(1e-6, 0.0, 0.0), order="lex", block=0, steps=500),
    # adjoint workload: radius-8 sphere pack at porosity 0.5
    "spherepack-128": dict(
        shape=(128, 128, 128), periodic=(True, False, False), tau=0.8,
        force=(1e-6, 0.0, 0.0), order="lex", block=0, steps=200),
}


def workload(name: str, seed: int = 0):
    """Return ``(mask, params)`` for a named workload."""
    p = dict(WORKLOADS[name])
    shape = p["shape"]
    if name.startswith("channel"):
        mask = channel_mask(*shape)
    elif name == "spheres-32":
        mask = rsa_spheres(shape, 3.0, 0.20, p["periodic"], seed)
    elif name == "spherepack-512x128x128":
        mask = relaxed_spheres(shape, 8.0, 0.40, seed)
    elif name == "spherepack-128":
        mask = relaxed_spheres(shape, 8.0, 0.50, seed)
    elif name in ("foam-384", "foam-512", "foam-768", "foam-1024"):
        mask = foam(shape, 4.0, 0.85, seed)
    else:
        raise KeyError(name)
    return mask, p
