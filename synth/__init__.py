"""Seeded synthetic inputs for snakuscule evolution: volumes, seeds, direction tables, parameters.

This module is the only code that both the HIP path and the FP64 oracle consume. It generates
*inputs* (raw voxel volumes, seed centres, contour ids, the sampling direction table and the
parameter record) and holds none of the method's arithmetic: no weight function, no energy, no
gradient, no random rotation, no Philox. Everything here is deterministic given its seed.

Conventions shared by every consumer:
  * volumes are numpy arrays indexed ``[z][y][x]`` (x fastest), dtype uint8 / uint16 / float32;
  * physical coordinates have their origin at the centre of voxel (0, 0, 0); the physical
    position of voxel (i, j, k) is (i*hx, j*hy, k*hz) with spacing ``h = (hx, hy, hz)``;
  * 2D images are volumes with nz == 1 and dim == 2 (their z coordinate is 0).
"""
from __future__ import annotations

import dataclasses
import math
from dataclasses import dataclass, field

import numpy as np

__all__ = [
    "Params", "Workload", "icosphere", "circle_directions", "render_ellipsoids", "blurred_ball",
    "tiny_config", "slab_params", "slab_config", "plane_config", "subvolume_batch", "served_tiles",
    "CONFIG_SEED_BASE",
]

CONFIG_SEED_BASE = 0x1804063040000000


@dataclass
class Params:
    """Parameter record of one evolution run (field-for-field the C ABI's ``snk_params``).

    dim          2 or 3
    spacing      physical step per voxel along (x, y, z)
    sigma_pre    low-pass sigma of the pre-pass, physical units (0 disables it)
    i_offset, i_scale   I = (raw - i_offset) * i_scale before smoothing
    dR           outer ramp width Delta R (the inner ramp width follows from it)
    eps0         step-size constant, eps_n = eps0 / sqrt(n)
    r_min, r_max bounds on the radius R (the library raises r_min to the geometric minimum)
    r_init       initial radius R0 of every seed (unless per-seed radii are given)
    n_dirs       D, directions in the table
    n_rays       M, rays per contour-iteration (even: antithetic pairs)
    n_radial     L, radial points per ray
    seed         64-bit Philox key
    conv_tol, conv_window   freeze after conv_window consecutive steps moving less than conv_tol
    e0           energy threshold of the final selection
    flags        bit 0: no random rotation of the direction table (test mode)
    """

    dim: int = 3
    spacing: tuple = (1.0, 1.0, 1.0)
    sigma_pre: float = 1.0
    i_offset: float = 0.0
    i_scale: float = 1.0
    dR: float = 1.0
    eps0: float = 8.0
    r_min: float = 0.0
    r_max: float = 30.0
    r_init: float = 6.93
    n_dirs: int = 162
    n_rays: int = 32
    n_radial: int = 16
    seed: int = CONFIG_SEED_BASE + 1
    conv_tol: float = 1e-3
    conv_window: int = 10
    e0: float = -0.05
    flags: int = 0

    def replace(self, **kw) -> "Params":
        return dataclasses.replace(self, **kw)


@dataclass
class Workload:
    """One synthetic problem: raw volume + seeds + direction table + parameters."""

    name: str
    raw: np.ndarray                 # [z][y][x] uint8/uint16/float32
    params: Params
    dirs: np.ndarray                # (D, dim) float64 unit vectors
    seeds: np.ndarray               # (n, 3) float64 physical centres (z = 0 in 2D)
    ids: np.ndarray                 # (n,) uint32
    n_iter: int
    truth: dict = field(default_factory=dict)   # ground-truth centres / semi-axes

    @property
    def shape_xyz(self):
        nz, ny, nx = self.raw.shape
        return nx, ny, nz


# ----------------------------------------------------------------------------------------------
# direction tables
# ----------------------------------------------------------------------------------------------

def icosphere(subdiv: int) -> np.ndarray:
    """Vertices of a geodesic icosphere with ``10 * 4**subdiv + 2`` unit vectors (float64).

    Built by repeated 4-way subdivision of the icosahedron's faces, projecting new edge
    midpoints onto the sphere. Vertex order is deterministic: the 12 icosahedron vertices,
    then midpoints in order of first creation.
    """
    t = (1.0 + 5.0 ** 0.5) / 2.0
    verts = [(-1, t, 0), (1, t, 0), (-1, -t, 0), (1, -t, 0), (0, -1, t), (0, 1, t), (0, -1, -t),
             (0, 1, -t), (t, 0, -1), (t, 0, 1), (-t, 0, -1), (-t, 0, 1)]
    verts = [np.array(v, dtype=np.float64) / np.linalg.norm(v) for v in verts]
    faces = [(0, 11, 5), (0, 5, 1), (0, 1, 7), (0, 7, 10), (0, 10, 11), (1, 5, 9), (5, 11, 4),
             (11, 10, 2), (10, 7, 6), (7, 1, 8), (3, 9, 4), (3, 4, 2), (3, 2, 6), (3, 6, 8),
             (3, 8, 9), (4, 9, 5), (2, 4, 11), (6, 2, 10), (8, 6, 7), (9, 8, 1)]
    for _ in range(subdiv):
        cache = {}

        def mid(a, b):
            key = (a, b) if a < b else (b, a)
            if key not in cache:
                m = verts[a] + verts[b]
                verts.append(m / np.linalg.norm(m))
                cache[key] = len(verts) - 1
            return cache[key]

        new_faces = []
        for a, b, c in faces:
            ab, bc, ca = mid(a, b), mid(b, c), mid(c, a)
            new_faces += [(a, ab, ca), (b, bc, ab), (c, ca, bc), (ab, bc, ca)]
        faces = new_faces
    return np.stack(verts).astype(np.float64)


def circle_directions(n: int) -> np.ndarray:
    """``n`` equally spaced unit vectors in the plane, angle 2*pi*k/n (float64, shape (n, 2))."""
    ang = 2.0 * np.pi * np.arange(n, dtype=np.float64) / n
    return np.stack([np.cos(ang), np.sin(ang)], axis=1)


def directions_for(dim: int, n_dirs: int) -> np.ndarray:
    if dim == 2:
        return circle_directions(n_dirs)
    for s in range(6):
        if 10 * 4 ** s + 2 == n_dirs:
            return icosphere(s)
    raise ValueError(f"no icosphere with {n_dirs} vertices")


# ----------------------------------------------------------------------------------------------
# random geometry helpers (input generation only)
# ----------------------------------------------------------------------------------------------

def _random_rotation(rng: np.random.Generator) -> np.ndarray:
    """Uniform random rotation matrix (QR of a Gaussian matrix with sign fix)."""
    q, r = np.linalg.qr(rng.normal(size=(3, 3)))
    q = q * np.sign(np.diag(r))
    if np.linalg.det(q) < 0:
        q[:, 0] = -q[:, 0]
    return q


def render_ellipsoids(shape_zyx, spacing, centers, axes, rots, ss: int = 2) -> np.ndarray:
    """Fractional coverage (0..1, float32) of ellipsoids, supersampled ``ss`` per axis.

    centers: (n, 3) physical (x, y, z); axes: (n, 3) physical semi-axes; rots: (n, 3, 3) with the
    ellipsoid's principal axes as columns. Overlaps take the maximum coverage. A 2D image
    (shape (1, ny, nx)) renders ellipses using the first two components only.
    """
    nz, ny, nx = shape_zyx
    h = np.asarray(spacing, dtype=np.float64)
    out = np.zeros(shape_zyx, dtype=np.float32)
    off = (np.arange(ss) + 0.5) / ss - 0.5
    planar = nz == 1
    for c, ax, rm in zip(centers, axes, rots):
        ext = float(np.max(ax)) + 1.0
        lo = np.floor((c - ext) / h).astype(int)
        hi = np.ceil((c + ext) / h).astype(int)
        lo = np.maximum(lo, 0)
        hi = np.minimum(hi, np.array([nx - 1, ny - 1, nz - 1]))
        if planar:
            lo[2] = hi[2] = 0
        if np.any(hi < lo):
            continue
        xs = (np.arange(lo[0], hi[0] + 1)[:, None] + off[None, :]).ravel() * h[0]
        ys = (np.arange(lo[1], hi[1] + 1)[:, None] + off[None, :]).ravel() * h[1]
        if planar:
            zs = np.zeros(1)
            ssz = 1
        else:
            zs = (np.arange(lo[2], hi[2] + 1)[:, None] + off[None, :]).ravel() * h[2]
            ssz = ss
        Z, Y, X = np.meshgrid(zs - c[2], ys - c[1], xs - c[0], indexing="ij")
        P = np.stack([X, Y, Z], axis=-1)
        if planar:
            loc = P[..., :2] @ rm[:2, :2]
            inside = ((loc / ax[:2]) ** 2).sum(-1) <= 1.0
        else:
            loc = P @ rm
            inside = ((loc / ax) ** 2).sum(-1) <= 1.0
        bz, by, bx = inside.shape
        cov = inside.reshape(bz // ssz, ssz, by // ss, ss, bx // ss, ss).mean(axis=(1, 3, 5))
        sl = (slice(lo[2], hi[2] + 1), slice(lo[1], hi[1] + 1), slice(lo[0], hi[0] + 1))
        np.maximum(out[sl], cov.astype(np.float32), out=out[sl])
    return out


def _blur(cov: np.ndarray, sigma_vox: float) -> np.ndarray:
    from scipy.ndimage import gaussian_filter
    sig = (0.0 if cov.shape[0] == 1 else sigma_vox, sigma_vox, sigma_vox)
    return gaussian_filter(cov.astype(np.float32), sigma=sig, mode="nearest", truncate=4.0)


def _pack(rng, n_target, lo, hi, rad_fn, overlap=0.0, max_tries=200000, planar=False):
    """Random sequential addition of bounding spheres; returns centres and radii."""
    cs, rs = [], []
    tries = 0
    while len(cs) < n_target and tries < max_tries:
        tries += 1
        r = rad_fn()
        c = rng.uniform(lo + r, hi - r)
        if planar:
            c[2] = 0.0
        if cs:
            d = np.linalg.norm(np.asarray(cs) - c, axis=1)
            if np.any(d < (1.0 - overlap) * (np.asarray(rs) + r)):
                continue
        cs.append(c)
        rs.append(r)
    return np.asarray(cs), np.asarray(rs)


def _quantise(x: np.ndarray, dtype) -> np.ndarray:
    info = np.iinfo(dtype)
    return np.clip(np.rint(x), info.min, info.max).astype(dtype)


# ----------------------------------------------------------------------------------------------
# analytic test volume
# ----------------------------------------------------------------------------------------------

def blurred_ball(r, r0: float, sigma: float, dim: int = 3):
    """Indicator of a ball (disk) of radius r0 convolved with an isotropic Gaussian of width sigma,
    as a function of the distance r from its centre. sigma == 0 gives the plain indicator.

    3D: the closed form of the Gaussian-blurred sphere indicator. 2D: numerical (radial
    Hankel-free) evaluation by 1D quadrature of the Rician integral.
    """
    r = np.asarray(r, dtype=np.float64)
    if sigma == 0.0:
        return (r < r0).astype(np.float64)
    from scipy.special import erf
    if dim == 3:
        s2 = sigma * math.sqrt(2.0)
        rr = np.maximum(r, 1e-12)
        term = 0.5 * (erf((r0 - rr) / s2) + erf((r0 + rr) / s2))
        term -= sigma / (rr * math.sqrt(2.0 * math.pi)) * (
            np.exp(-(rr - r0) ** 2 / (2 * sigma ** 2)) - np.exp(-(rr + r0) ** 2 / (2 * sigma ** 2)))
        return term
    from scipy.special import i0e
    t = np.linspace(0.0, r0, 2001)
    w = np.full_like(t, t[1] - t[0])
    w[0] *= 0.5
    w[-1] *= 0.5
    out = np.empty(r.shape)
    for idx, rv in np.ndenumerate(r):
        g = (t / sigma ** 2) * np.exp(-((t - rv) ** 2) / (2 * sigma ** 2)) * i0e(t * rv / sigma ** 2)
        out[idx] = float((g * w).sum())
    return out


# ----------------------------------------------------------------------------------------------
# workload configurations
# ----------------------------------------------------------------------------------------------

def tiny_config(seed: int = CONFIG_SEED_BASE + 1) -> Workload:
    """64^3 uint8, 8 bright ellipsoids (semi-axes 4..7, random orientation), PSF sigma 1,
    background 20 / blob 180, Gaussian noise sd 8; seeds jittered +-1 voxel; D 162, M 32, L 16,
    100 iterations."""
    rng = np.random.default_rng(seed)
    shape = (64, 64, 64)
    axes = rng.uniform(4.0, 7.0, size=(8, 3))
    cs = []
    for ax in axes:
        r = float(ax.max())
        while True:
            c = rng.uniform(10.0, 54.0, size=3)
            if all(np.linalg.norm(c - c2) > r + float(a2.max()) for c2, a2 in zip(cs, axes)):
                cs.append(c)
                break
    centers = np.asarray(cs)
    rots = np.stack([_random_rotation(rng) for _ in range(8)])
    cov = render_ellipsoids(shape, (1, 1, 1), centers, axes, rots)
    blurred = _blur(cov, 1.0)
    val = 20.0 + 160.0 * blurred + rng.normal(0.0, 8.0, size=shape)
    raw = _quantise(val, np.uint8)
    r0 = 2.0 ** (1.0 / 3.0) * 5.5
    p = Params(dim=3, spacing=(1.0, 1.0, 1.0), sigma_pre=1.0, i_offset=20.0, i_scale=1.0 / 160.0,
               dR=1.0, eps0=8.0, r_min=0.0, r_max=3.0 * r0, r_init=r0, n_dirs=162, n_rays=32, n_radial=16,
               seed=seed, conv_tol=1e-3, conv_window=10, e0=-0.05)
    seeds = centers + rng.uniform(-1.0, 1.0, size=centers.shape)
    return Workload("tiny-64^3-u8-8blobs", raw, p, icosphere(2), seeds,
                    np.arange(len(seeds), dtype=np.uint32), 100,
                    {"centers": centers, "axes": axes, "rots": rots, "r0": r0})


def slab_params(seed: int, n_dirs: int = 642, n_rays: int = 64) -> Params:
    """Method parameters of the nuclei workloads (slab, batched subvolumes, served tiles): h = (1, 1, 2),
    contrast-normalised counts (background 100, peak 900), dR 0.75, R0 = 2^(1/3) * 6.5, r_max 3 R0."""
    r0 = 2.0 ** (1.0 / 3.0) * 6.5
    return Params(dim=3, spacing=(1.0, 1.0, 2.0), sigma_pre=1.0, i_offset=100.0, i_scale=1.0 / 900.0,
                  dR=0.75, eps0=8.0, r_min=0.0, r_max=3.0 * r0, r_init=r0, n_dirs=n_dirs, n_rays=n_rays,
                  n_radial=16, seed=seed, conv_tol=1e-3, conv_window=10, e0=-0.05)


def slab_config(seed: int = CONFIG_SEED_BASE + 2, n_target: int = 2000, shape_xyz=(512, 512, 128),
                n_iter: int = 500) -> Workload:
    """512x512x128 uint16 slab, h = (1, 1, 2), ~2,000 ellipsoid nuclei (physical semi-axes 3..10,
    random orientation), PSF sigma 1.2 voxels, Poisson counts with rate
    (100 + 900*blurred) * (1 - 0.3 x/(nx-1)); D 642, M 64, L 16, 500 iterations."""
    rng = np.random.default_rng(seed)
    nx, ny, nz = shape_xyz
    h = np.array([1.0, 1.0, 2.0])
    ext = np.array([nx - 1, ny - 1, nz - 1]) * h
    axes_pool = []

    def rad():
        ax = rng.uniform(3.0, 10.0, size=3)
        axes_pool.append(ax)
        return float(ax.max())

    centers, radii = _pack(rng, n_target, np.zeros(3), ext, rad, overlap=0.10)
    # the axes drawn for accepted objects: regenerate deterministically sized to the radius
    n = len(centers)
    axes = rng.uniform(3.0, 10.0, size=(n, 3))
    axes = axes * (radii / axes.max(axis=1))[:, None]
    rots = np.stack([_random_rotation(rng) for _ in range(n)])
    cov = render_ellipsoids((nz, ny, nx), h, centers, axes, rots)
    blurred = _blur(cov, 1.2)
    x = np.arange(nx, dtype=np.float32) / max(nx - 1, 1)
    lam = (100.0 + 900.0 * blurred) * (1.0 - 0.3 * x)[None, None, :]
    raw = _quantise(rng.poisson(lam).astype(np.float64), np.uint16)
    r0 = 2.0 ** (1.0 / 3.0) * 6.5
    p = slab_params(seed)
    seeds = centers + rng.uniform(-1.0, 1.0, size=centers.shape) * h
    seeds = np.clip(seeds, 0.0, ext)
    return Workload("slab-512x512x128-u16-%dnuclei" % n, raw, p, icosphere(3), seeds,
                    np.arange(n, dtype=np.uint32), n_iter,
                    {"centers": centers, "axes": axes, "rots": rots, "r0": r0})


def plane_config(seed: int = CONFIG_SEED_BASE + 3, n_target: int = 40000, size: int = 8192,
                 n_iter: int = 300) -> Workload:
    """2D image size x size uint8, touching disk / ellipse cells (semi-axes 4..12), PSF sigma 1,
    20 + 160*blurred + N(0, 10^2); 64 directions, M 16, L 16, 300 iterations."""
    rng = np.random.default_rng(seed)
    ext = np.array([size - 1.0, size - 1.0, 0.0])
    cs, ax_list = [], []
    # cell grid for overlap queries
    cell = 26.0
    grid = {}

    def near(c, r):
        gx, gy = int(c[0] // cell), int(c[1] // cell)
        for dx in (-1, 0, 1):
            for dy in (-1, 0, 1):
                for j in grid.get((gx + dx, gy + dy), ()):
                    if np.hypot(*(cs[j][:2] - c[:2])) < r + ax_list[j].max() - 1e-9:
                        return True
        return False

    tries = 0
    while len(cs) < n_target and tries < 40 * n_target:
        tries += 1
        a = rng.uniform(4.0, 12.0)
        b = a if rng.random() < 0.5 else a * rng.uniform(0.67, 1.0)
        r = max(a, b)
        if cs and rng.random() < 0.5:
            j = int(rng.integers(len(cs)))
            ang = rng.uniform(0, 2 * np.pi)
            c = cs[j] + (ax_list[j].max() + r) * np.array([np.cos(ang), np.sin(ang), 0.0])
        else:
            c = np.array([rng.uniform(r, ext[0] - r), rng.uniform(r, ext[1] - r), 0.0])
        if c[0] < r or c[1] < r or c[0] > ext[0] - r or c[1] > ext[1] - r or near(c, r):
            continue
        grid.setdefault((int(c[0] // cell), int(c[1] // cell)), []).append(len(cs))
        cs.append(c)
        ax_list.append(np.array([a, b, 1.0]))
    centers = np.asarray(cs)
    axes = np.asarray(ax_list)
    n = len(centers)
    th = rng.uniform(0, 2 * np.pi, size=n)
    rots = np.zeros((n, 3, 3))
    rots[:, 0, 0] = np.cos(th); rots[:, 0, 1] = -np.sin(th)
    rots[:, 1, 0] = np.sin(th); rots[:, 1, 1] = np.cos(th)
    rots[:, 2, 2] = 1.0
    cov = render_ellipsoids((1, size, size), (1, 1, 1), centers, axes, rots)
    blurred = _blur(cov, 1.0)
    val = 20.0 + 160.0 * blurred + rng.normal(0.0, 10.0, size=blurred.shape)
    raw = _quantise(val, np.uint8)
    r0 = 2.0 ** 0.5 * 8.0
    p = Params(dim=2, spacing=(1.0, 1.0, 1.0), sigma_pre=1.0, i_offset=20.0, i_scale=1.0 / 160.0,
               dR=1.0, eps0=8.0, r_min=0.0, r_max=3.0 * r0, r_init=r0, n_dirs=64, n_rays=16, n_radial=16,
               seed=seed, conv_tol=1e-3, conv_window=10, e0=-0.08)
    seeds = centers + np.concatenate([rng.uniform(-1, 1, size=(n, 2)), np.zeros((n, 1))], axis=1)
    return Workload("plane-%d^2-u8-%dcells" % (size, n), raw, p, circle_directions(64), seeds,
                    np.arange(n, dtype=np.uint32), n_iter,
                    {"centers": centers, "axes": axes, "rots": rots, "r0": r0})


def subvolume_batch(seed: int = CONFIG_SEED_BASE + 4, n_vol: int = 256, edge_lo: int = 32,
                    edge_hi: int = 160, n_iter: int = 200):
    """Batch of cubic uint16 subvolumes of uneven size with uneven nucleus counts (as the slab)."""
    rng = np.random.default_rng(seed)
    out = []
    for v in range(n_vol):
        e = int(rng.integers(edge_lo, edge_hi + 1))
        vol_phys = e ** 3 * 2.0
        cap = int(0.30 * vol_phys / ((4.0 / 3.0) * np.pi * 6.5 ** 3))
        n = int(min(rng.integers(10, 801), max(cap, 1)))
        wl = slab_config(seed=int(rng.integers(1 << 62)), n_target=n, shape_xyz=(e, e, e), n_iter=n_iter)
        if rng.random() < 0.5:
            wl.params = wl.params.replace(n_dirs=162, n_rays=32)
            wl.dirs = icosphere(2)
        wl.name = "sub%03d-%d^3-%d" % (v, e, len(wl.seeds))
        out.append(wl)
    return out


def served_tiles(seed: int = CONFIG_SEED_BASE + 5, n_tiles: int = 24, edge_lo: int = 64, edge_hi: int = 256,
                 halo: int = 16, max_edge: int = 288, n_iter: int = 200):
    """Pool of tile-segmentation requests: cubic uint16 tiles (core edge U{edge_lo..edge_hi} plus a
    halo, capped at max_edge), nucleus density U[20, 400] per 128^3 block, smooth multiplicative gain
    0.7-1.0 and Poisson counts, spacing (1, 1, 2); seeds are the true centres in the tile core.
    D 162, M 32, L 16."""
    rng = np.random.default_rng(seed)
    out = []
    for t in range(n_tiles):
        core = int(rng.integers(edge_lo, edge_hi + 1))
        e = min(core + 2 * halo, max_edge)
        density = rng.uniform(20.0, 400.0)
        n_target = max(1, int(density * (e ** 3) / 128.0 ** 3))
        wl = slab_config(seed=int(rng.integers(1 << 62)), n_target=n_target, shape_xyz=(e, e, e), n_iter=n_iter)
        # smooth gain field 0.7..1.0 along a random direction
        g = rng.normal(size=3)
        g /= np.linalg.norm(g)
        zz, yy, xx = np.meshgrid(*(np.linspace(0.0, 1.0, e),) * 3, indexing="ij")
        ramp = (g[0] * xx + g[1] * yy + g[2] * zz)
        ramp = (ramp - ramp.min()) / max(ramp.max() - ramp.min(), 1e-9)
        gain = (0.7 + 0.3 * ramp).astype(np.float32)
        wl.raw = np.clip(np.rint(wl.raw.astype(np.float32) * gain), 0, 65535).astype(np.uint16)
        h = np.asarray(wl.params.spacing)
        lo, hi = halo * h, (e - 1 - halo) * h
        core_mask = np.all((wl.truth["centers"] >= lo) & (wl.truth["centers"] <= hi), axis=1)
        wl.seeds = wl.truth["centers"][core_mask].copy()
        wl.ids = np.arange(len(wl.seeds), dtype=np.uint32)
        wl.params = wl.params.replace(n_dirs=162, n_rays=32)
        wl.dirs = icosphere(2)
        wl.name = "tile%02d-%d^3-%d" % (t, e, len(wl.seeds))
        out.append(wl)
    return out
