"""Large synthetic volumes generated box by box with torch (on the GPU when one is given).

Input generation only, like the rest of ``synth``: object lists, rendered coverage, a Gaussian
PSF, an intensity gain and Poisson counts. None of the method's arithmetic lives here.

Every voxel's value is a function of its global position alone, computed with elementwise torch
operations in a fixed order: the coverage of a voxel is the maximum over objects of the fraction
of its 2x2x2 sub-samples inside the object; the PSF is a separable Gaussian summed tap by tap in a
fixed order, with clamp-to-edge only at the faces of the whole volume; the Poisson count is drawn
from a counter-based generator keyed by the voxel's global index. So any box of the volume,
generated on its own, is bit for bit the same as the corresponding cut of the whole volume
generated on the same device -- tiles are reproducible without ever holding the whole volume.

The counter-based uniforms are SplitMix64 outputs (Steele, Lea and Flood, "Fast splittable
pseudorandom number generators", OOPSLA 2014): the 64-bit finaliser applied to key + counter *
0x9E3779B97F4A7C15. Poisson counts use Hoermann's transformed rejection with squeeze, PTRS
("The transformed rejection method for generating Poisson random variables", Insurance:
Mathematics and Economics 12, 1993), valid for means of 10 and more; each attempt takes two
uniforms at counters (index * 64 + attempt) * 2 + {0, 1}.
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np

__all__ = ["ObjectList", "LargeVolume", "render_coverage", "blur_box", "counter_bits", "counter_uniform", "counter_poisson",
           "pack_block", "random_rotations", "fast_subvolume_batch",
           "subvolume_workloads", "served_volume", "tile_workload"]

_M64 = (1 << 64) - 1
_CACHE = {}


def _s64(v: int) -> int:
    """A 64-bit unsigned constant as the int64 with the same bits."""
    v &= _M64
    return v - (1 << 64) if v >= (1 << 63) else v


_GAMMA = _s64(0x9E3779B97F4A7C15)
_C1 = _s64(0xBF58476D1CE4E5B9)
_C2 = _s64(0x94D049BB133111EB)


def _lsr(x, s: int):
    """Logical right shift of an int64 tensor (torch's >> is arithmetic)."""
    return (x >> s) & ((1 << (64 - s)) - 1)


def counter_bits(key: int, counter):
    """SplitMix64 output (int64 tensor holding the 64 bits) for int64 counters: the finaliser of
    key + counter * gamma."""
    z = counter * _GAMMA + _s64(key)
    z = (z ^ _lsr(z, 30)) * _C1
    z = (z ^ _lsr(z, 27)) * _C2
    return z ^ _lsr(z, 31)


def counter_uniform(key: int, counter):
    """Uniforms in (0, 1) (float64 tensor) for int64 counters: the top 53 bits of counter_bits,
    centred in their interval."""
    return (_lsr(counter_bits(key, counter), 11).double() + 0.5) * (2.0 ** -53)


def counter_poisson(lam, index, key: int, max_attempts: int = 64):
    """Poisson counts (int64 tensor) with means lam (float64 tensor, all >= 10) for voxels with
    global indices `index` (int64 tensor of the same shape): PTRS, attempt a of voxel i taking the
    uniforms at counters (i * 64 + a) * 2 and (i * 64 + a) * 2 + 1."""
    import torch
    lam = lam.reshape(-1)
    index = index.reshape(-1)
    if lam.numel() and float(lam.min()) < 10.0:
        raise ValueError("counter_poisson: PTRS needs means >= 10")
    out = torch.empty_like(index)
    todo = torch.arange(index.numel(), device=index.device)
    for attempt in range(max_attempts):
        if todo.numel() == 0:
            break
        lt = lam[todo]
        base = (index[todo] * 64 + attempt) * 2
        slam = torch.sqrt(lt)
        loglam = torch.log(lt)
        b = 0.931 + 2.53 * slam
        a = -0.059 + 0.02483 * b
        inv_alpha = 1.1239 + 1.1328 / (b - 3.4)
        vr = 0.9277 - 3.6224 / (b - 2.0)
        u = counter_uniform(key, base) - 0.5
        v = counter_uniform(key, base + 1)
        us = 0.5 - torch.abs(u)
        k = torch.floor((2.0 * a / us + b) * u + lt + 0.43)
        quick = (us >= 0.07) & (v <= vr)
        reject = (k < 0) | ((us < 0.013) & (v > us))
        kk = torch.clamp(k, min=0.0)
        lhs = torch.log(v) + torch.log(inv_alpha) - torch.log(a / (us * us) + b)
        rhs = -lt + kk * loglam - torch.lgamma(kk + 1.0)
        acc = quick | (~reject & (lhs <= rhs))
        out[todo[acc]] = k[acc].long()
        todo = todo[~acc]
    if todo.numel():
        raise RuntimeError("counter_poisson: attempts exhausted")
    return out


def random_rotations(rng: np.random.Generator, n: int) -> np.ndarray:
    """n uniform random rotation matrices (QR of Gaussian matrices with the sign fix), (n, 3, 3)."""
    q, r = np.linalg.qr(rng.normal(size=(n, 3, 3)))
    q = q * np.sign(np.diagonal(r, axis1=1, axis2=2))[:, None, :]
    neg = np.linalg.det(q) < 0
    q[neg, :, 0] = -q[neg, :, 0]
    return q


def pack_block(rng: np.random.Generator, n_target: int, lo, hi, overlap: float = 0.10,
               axes_range=(3.0, 10.0), tries: int = 3, inset: bool = False):
    """Random sequential addition of n_target ellipsoids with centres uniform in [lo, hi)
    (physical): candidates are drawn in one batch (tries * n_target), each with semi-axes
    U[axes_range] and a bounding radius equal to its largest semi-axis, and accepted in order when
    no accepted one overlaps its bounding sphere by more than `overlap`. inset: each candidate's
    centre is drawn at least its bounding radius from the faces of [lo, hi] instead. Returns centres
    (n, 3), semi-axes (n, 3) and rotations (n, 3, 3)."""
    lo = np.asarray(lo, np.float64)
    hi = np.asarray(hi, np.float64)
    m = max(1, tries * n_target)
    cen = lo + rng.random((m, 3)) * (hi - lo)
    axes = rng.uniform(axes_range[0], axes_range[1], size=(m, 3))
    rad = axes.max(axis=1)
    rots = random_rotations(rng, m)
    if inset:
        span = (hi - lo)[None, :] - 2.0 * rad[:, None]
        fits = np.all(span >= 0.0, axis=1)
        cen = np.where(fits[:, None], lo + rad[:, None] + (cen - lo) / np.maximum(hi - lo, 1e-300) * np.maximum(span, 0.0),
                       cen)
        cen, axes, rad, rots = cen[fits], axes[fits], rad[fits], rots[fits]
        m = len(cen)
    from scipy.spatial import cKDTree
    pairs = cKDTree(cen).query_pairs(r=2.0 * float(axes_range[1]) * (1.0 - overlap), output_type="ndarray")
    if len(pairs):
        d = np.linalg.norm(cen[pairs[:, 0]] - cen[pairs[:, 1]], axis=1)
        pairs = pairs[d < (1.0 - overlap) * (rad[pairs[:, 0]] + rad[pairs[:, 1]])]
    first = np.minimum(pairs[:, 0], pairs[:, 1]) if len(pairs) else np.zeros(0, np.int64)
    later = np.maximum(pairs[:, 0], pairs[:, 1]) if len(pairs) else np.zeros(0, np.int64)
    order = np.argsort(later, kind="stable")
    first, later = first[order], later[order]
    bounds = np.searchsorted(later, np.arange(m + 1))
    keep = np.zeros(m, bool)
    count = 0
    for i in range(m):
        if count >= n_target:
            break
        if not np.any(keep[first[bounds[i]:bounds[i + 1]]]):
            keep[i] = True
            count += 1
    return cen[keep], axes[keep], rots[keep]


def render_coverage(lo, shape, h, centers, axes, rots, device, ss: int = 2, chunk: int = 0):
    """Fractional coverage (float32 tensor [z][y][x] of `shape` = (nx, ny, nz)) of the box whose
    first voxel is `lo` (global voxel indices x, y, z), by ellipsoids (physical centres, semi-axes,
    rotations with the principal axes as columns), each voxel sampled at ss^3 sub-positions.
    Overlaps take the maximum coverage."""
    import torch
    nx, ny, nz = (int(v) for v in shape)
    cov = torch.zeros(nz * ny * nx, dtype=torch.float32, device=device)
    n = len(centers)
    if n == 0:
        return cov.view(nz, ny, nx)
    h = np.asarray(h, np.float64)
    lo = np.asarray(lo, np.int64)
    ext = axes.max(axis=1) + 1.0
    vlo = np.floor((centers - ext[:, None]) / h).astype(np.int64)
    vhi = np.ceil((centers + ext[:, None]) / h).astype(np.int64)
    box_hi = lo + np.array([nx, ny, nz]) - 1
    vlo = np.maximum(vlo, lo)
    vhi = np.minimum(vhi, box_hi)
    live = np.all(vhi >= vlo, axis=1)
    if not np.any(live):
        return cov.view(nz, ny, nx)
    centers, axes, rots, vlo, vhi = centers[live], axes[live], rots[live], vlo[live], vhi[live]
    B = (vhi - vlo + 1).max(axis=0)                     # padded box (x, y, z) voxels
    per = int(B.prod()) * ss ** 3
    if chunk <= 0:
        chunk = max(1, (64 << 20) // per) if torch.device(device).type != "cpu" else max(1, (4 << 20) // per)
    off = torch.tensor((np.arange(ss) + 0.5) / ss - 0.5, dtype=torch.float32, device=device)
    hx, hy, hz = (float(v) for v in h)
    for s in range(0, len(centers), chunk):
        e = min(s + chunk, len(centers))
        K = e - s
        t = lambda a, dt=torch.float32: torch.as_tensor(np.ascontiguousarray(a), dtype=dt, device=device)
        c = t(centers[s:e])
        ax = t(axes[s:e])
        R = t(rots[s:e])
        v0 = t(vlo[s:e], torch.int64)
        v1 = t(vhi[s:e], torch.int64)
        # voxel indices per axis (K, B_a) and the sub-sample positions (K, B_a * ss), physical
        ix = v0[:, 0:1] + torch.arange(int(B[0]), device=device)[None, :]
        iy = v0[:, 1:2] + torch.arange(int(B[1]), device=device)[None, :]
        iz = v0[:, 2:3] + torch.arange(int(B[2]), device=device)[None, :]
        px = ((ix.float()[:, :, None] + off[None, None, :]) * hx).reshape(K, -1) - c[:, 0:1]
        py = ((iy.float()[:, :, None] + off[None, None, :]) * hy).reshape(K, -1) - c[:, 1:2]
        pz = ((iz.float()[:, :, None] + off[None, None, :]) * hz).reshape(K, -1) - c[:, 2:3]
        dx = px[:, None, None, :]
        dy = py[:, None, :, None]
        dz = pz[:, :, None, None]
        q = None
        for j in range(3):
            r0 = R[:, 0, j].view(K, 1, 1, 1)
            r1 = R[:, 1, j].view(K, 1, 1, 1)
            r2 = R[:, 2, j].view(K, 1, 1, 1)
            lj = dx * r0 + dy * r1 + dz * r2
            lj = lj / ax[:, j].view(K, 1, 1, 1)
            q = lj * lj if q is None else q + lj * lj
        inside = (q <= 1.0).view(K, int(B[2]), ss, int(B[1]), ss, int(B[0]), ss)
        frac = inside.sum(dim=(2, 4, 6), dtype=torch.int32).float() * (1.0 / ss ** 3)  # (K, Bz, By, Bx)
        valid = ((ix <= v1[:, 0:1])[:, None, None, :] & (iy <= v1[:, 1:2])[:, None, :, None]
                 & (iz <= v1[:, 2:3])[:, :, None, None])
        lin = (((iz - int(lo[2]))[:, :, None, None] * ny + (iy - int(lo[1]))[:, None, :, None]) * nx
               + (ix - int(lo[0]))[:, None, None, :])
        cov.scatter_reduce_(0, lin[valid], frac[valid], reduce="amax")
    return cov.view(nz, ny, nx)


def gaussian_taps(sigma: float, truncate: float = 4.0) -> np.ndarray:
    """Normalised Gaussian taps of radius int(truncate * sigma + 0.5) (float64)."""
    r = int(truncate * sigma + 0.5)
    x = np.arange(-r, r + 1, dtype=np.float64)
    w = np.exp(-0.5 * x * x / (sigma * sigma))
    return w / w.sum()


def blur_box(cov, cov_lo, out_lo, out_shape, full_shape, sigma: float):
    """Separable Gaussian (sigma in voxels on every axis, taps gaussian_taps(sigma)) of a coverage box
    `cov` ([z][y][x], first voxel cov_lo), evaluated on the box out_lo + out_shape; positions beyond
    the whole volume (full_shape) take its face values (clamp-to-edge). `cov` must hold every voxel
    within the tap radius of the output box (clamped to the volume). Axes x, then y, then z; taps
    summed in order."""
    import torch
    w = gaussian_taps(sigma)
    r = (len(w) - 1) // 2
    x = cov
    for axis, dim in ((0, 2), (1, 1), (2, 0)):
        n_full = int(full_shape[axis])
        pos = torch.arange(int(out_lo[axis]), int(out_lo[axis]) + int(out_shape[axis]), device=cov.device)
        acc = None
        for k in range(-r, r + 1):
            src = torch.clamp(pos + k, 0, n_full - 1) - int(cov_lo[axis])
            term = x.index_select(dim, src) * float(w[k + r])
            acc = term if acc is None else acc + term
        x = acc
    return x


@dataclass
class ObjectList:
    centers: np.ndarray   # (n, 3) physical
    axes: np.ndarray      # (n, 3) physical semi-axes
    rots: np.ndarray      # (n, 3, 3) principal axes as columns
    block_of: np.ndarray  # (n,) block index of each object
    block_start: np.ndarray  # (n_blocks + 1,) objects of block b: block_start[b] .. block_start[b + 1]


class LargeVolume:
    """A uint16 volume of (nx, ny, nz) voxels, spacing h, built from ellipsoid nuclei packed block by
    block (block**3 voxels per block, each with a density U[dens_lo, dens_hi] nuclei per block^3
    voxels, drawn from its own seed), a Gaussian PSF (psf_sigma voxels), a smooth multiplicative
    gain between gain_lo and 1 and Poisson counts with mean (background + peak * blurred) * gain.
    Generated box by box: ``box(lo, hi)`` renders any box on its own."""

    def __init__(self, seed: int, shape_xyz=(2048, 2048, 512), spacing=(1.0, 1.0, 2.0), block: int = 128,
                 density=(20.0, 400.0), psf_sigma: float = 1.2, background: float = 100.0, peak: float = 900.0,
                 gain_lo: float = 0.7):
        self.seed = int(seed)
        self.shape = tuple(int(v) for v in shape_xyz)
        self.h = np.asarray(spacing, np.float64)
        self.block = int(block)
        self.density = density
        self.psf_sigma = float(psf_sigma)
        self.background = float(background)
        self.peak = float(peak)
        self.gain_lo = float(gain_lo)
        self.nb = tuple((n + self.block - 1) // self.block for n in self.shape)
        self._objects = None

    # -- objects ---------------------------------------------------------------------------------
    def objects(self) -> ObjectList:
        """The global object list (built once, block by block, each block from its own seed)."""
        if self._objects is not None:
            return self._objects
        cs, ax, rs, bo, starts = [], [], [], [], [0]
        nbx, nby, nbz = self.nb
        for b in range(nbx * nby * nbz):
            bx, by, bz = b % nbx, (b // nbx) % nby, b // (nbx * nby)
            rng = np.random.default_rng([self.seed, b])
            vlo = np.array([bx, by, bz]) * self.block
            vhi = np.minimum(vlo + self.block, self.shape)
            frac = float(np.prod(vhi - vlo)) / self.block ** 3
            n = int(round(rng.uniform(*self.density) * frac))
            lo = vlo * self.h
            hi = np.minimum(vhi * self.h, (np.asarray(self.shape) - 1) * self.h)
            c, a, r = pack_block(rng, n, lo, hi)
            cs.append(c)
            ax.append(a)
            rs.append(r)
            bo.append(np.full(len(c), b, np.int64))
            starts.append(starts[-1] + len(c))
        self._objects = ObjectList(np.concatenate(cs), np.concatenate(ax), np.concatenate(rs),
                                   np.concatenate(bo), np.asarray(starts, np.int64))
        return self._objects

    def objects_near(self, lo, hi, margin: float):
        """Indices (ascending) of objects whose bounding sphere comes within `margin` (physical) of the
        voxel box [lo, hi) (global voxel indices)."""
        ol = self.objects()
        if getattr(self, "_tree", None) is None:
            from scipy.spatial import cKDTree
            self._tree = cKDTree(ol.centers)
            self._rmax = float(ol.axes.max()) if len(ol.axes) else 0.0
        plo = np.asarray(lo, np.float64) * self.h - margin
        phi = (np.asarray(hi, np.float64) - 1) * self.h + margin
        mid = 0.5 * (plo + phi)
        reach = 0.5 * float(np.linalg.norm(phi - plo)) + self._rmax
        idx = np.sort(np.asarray(self._tree.query_ball_point(mid, reach), np.int64))
        if len(idx) == 0:
            return idx
        rad = ol.axes[idx].max(axis=1)
        c = ol.centers[idx]
        near = np.all((c + rad[:, None] >= plo) & (c - rad[:, None] <= phi), axis=1)
        return idx[near]

    def centers_in(self, lo, hi):
        """Indices of objects whose true centre lies in the voxel box [lo, hi - 1] (physical bounds)."""
        idx = self.objects_near(lo, hi, 0.0)
        c = self.objects().centers[idx]
        plo = np.asarray(lo, np.float64) * self.h
        phi = (np.asarray(hi, np.float64) - 1) * self.h
        return idx[np.all((c >= plo) & (c <= phi), axis=1)]

    # -- voxels ----------------------------------------------------------------------------------
    def gain(self, ix, iy, iz):
        """Smooth multiplicative gain in [gain_lo, 1] at global voxel indices (broadcast tensors)."""
        import torch
        nx, ny, nz = self.shape
        fx = ix.float() / float(nx)
        fy = iy.float() / float(ny)
        fz = iz.float() / float(nz)
        s = torch.sin(6.283185307179586 * (0.7 * fx + 0.3 * fy) + 1.3)
        c = torch.cos(6.283185307179586 * (0.45 * fy - 0.2 * fz) + 0.4)
        return self.gain_lo + (1.0 - self.gain_lo) * (0.5 + 0.5 * s * c)

    def box(self, lo, hi, device="cpu"):
        """The uint16 voxels [z][y][x] of the global box [lo, hi) (voxel indices x, y, z), as a torch
        tensor on `device`."""
        import torch
        lo = np.asarray(lo, np.int64)
        hi = np.asarray(hi, np.int64)
        full = np.asarray(self.shape, np.int64)
        if np.any(lo < 0) or np.any(hi > full) or np.any(hi <= lo):
            raise ValueError(f"box {lo}..{hi} outside the volume {full}")
        r = (len(gaussian_taps(self.psf_sigma)) - 1) // 2
        elo = np.maximum(lo - r, 0)
        ehi = np.minimum(hi + r, full)
        ol = self.objects()
        near = self.objects_near(elo, ehi, 1.0)
        cov = render_coverage(elo, ehi - elo, self.h, ol.centers[near], ol.axes[near], ol.rots[near], device)
        blurred = blur_box(cov, elo, lo, hi - lo, full, self.psf_sigma)
        ix = torch.arange(int(lo[0]), int(hi[0]), device=device).view(1, 1, -1)
        iy = torch.arange(int(lo[1]), int(hi[1]), device=device).view(1, -1, 1)
        iz = torch.arange(int(lo[2]), int(hi[2]), device=device).view(-1, 1, 1)
        lam = (self.background + self.peak * blurred) * self.gain(ix, iy, iz)
        gidx = (iz * int(full[1]) + iy) * int(full[0]) + ix
        gidx = gidx.expand_as(lam)
        k = counter_poisson(lam.double(), gidx.reshape(-1), self.seed ^ 0x5EED)
        return torch.clamp(k, 0, 65535).to(torch.int32).to(torch.uint16).view(lam.shape)

    def whole(self, device, slab: int = 64):
        """The whole volume [z][y][x] uint16 on `device`, generated in z-slabs of `slab` planes."""
        import torch
        nx, ny, nz = self.shape
        out = torch.empty((nz, ny, nx), dtype=torch.uint16, device=device)
        for z0 in range(0, nz, slab):
            z1 = min(z0 + slab, nz)
            out[z0:z1] = self.box((0, 0, z0), (nx, ny, z1), device)
        return out

    # -- requests --------------------------------------------------------------------------------
    def tile(self, rng: np.random.Generator, edge_lo: int = 64, edge_hi: int = 256, halo: int = 16):
        """A random tile request: a cubic core of edge U{edge_lo..edge_hi} voxels placed uniformly in
        the volume, grown by `halo` voxels per side and clamped at the faces. Returns (lo, hi) of the
        tile, (core_lo, core_hi) and the indices of the objects whose centres lie in the core."""
        full = np.asarray(self.shape, np.int64)
        e = int(rng.integers(edge_lo, edge_hi + 1))
        e_ax = np.minimum(e, full)
        core_lo = np.array([int(rng.integers(0, f - ea + 1)) for f, ea in zip(full, e_ax)], np.int64)
        core_hi = core_lo + e_ax
        lo = np.maximum(core_lo - halo, 0)
        hi = np.minimum(core_hi + halo, full)
        return lo, hi, core_lo, core_hi, self.centers_in(core_lo, core_hi)


def fast_subvolume_batch(seed: int, n_vol: int = 256, edge_lo: int = 32, edge_hi: int = 160, device="cpu"):
    """The batched workload's recipe rendered with torch: cubic uint16 subvolumes of edge
    U{edge_lo..edge_hi}, h = (1, 1, 2), 10..800 nuclei capped at 30% fill, packed by pack_block, PSF
    1.2 voxels, Poisson counts with mean (100 + 900 * blurred) * (1 - 0.3 x / (nx - 1)), D 642 or 162
    (half each). Yields (edge, raw tensor on device, centres, semi-axes, rotations, use_162)."""
    import torch
    rng = np.random.default_rng(seed)
    h = np.array([1.0, 1.0, 2.0])
    for v in range(n_vol):
        e = int(rng.integers(edge_lo, edge_hi + 1))
        vol_phys = e ** 3 * 2.0
        cap = int(0.30 * vol_phys / ((4.0 / 3.0) * np.pi * 6.5 ** 3))
        n = int(min(rng.integers(10, 801), max(cap, 1)))
        vseed = int(rng.integers(1 << 62))
        small = bool(rng.random() < 0.5)
        vr = np.random.default_rng(vseed)
        ext = (e - 1) * h
        c, a, r = pack_block(vr, n, np.zeros(3), ext, inset=True)   # every nucleus inside the volume
        shape = np.array([e, e, e])
        cov = render_coverage((0, 0, 0), shape, h, c, a, r, device)
        blurred = blur_box(cov, (0, 0, 0), (0, 0, 0), shape, shape, 1.2)
        ix = torch.arange(e, device=device).view(1, 1, -1)
        lam = (100.0 + 900.0 * blurred) * (1.0 - 0.3 * ix.float() / float(max(e - 1, 1)))
        iy = torch.arange(e, device=device).view(1, -1, 1)
        iz = torch.arange(e, device=device).view(-1, 1, 1)
        gidx = ((iz * e + iy) * e + ix).expand_as(lam)
        k = counter_poisson(lam.double(), gidx.reshape(-1), vseed)
        raw = torch.clamp(k, 0, 65535).to(torch.int32).to(torch.uint16).view(e, e, e)
        yield e, raw, c, a, r, small


def subvolume_workloads(seed: int, n_vol: int = 256, edge_lo: int = 32, edge_hi: int = 160, n_iter: int = 200,
                        device="cpu"):
    """The batched workload as synth.Workload records whose ``raw`` is a torch uint16 tensor on
    `device` (fast_subvolume_batch volumes; seeds = true centres + U[-1, 1] per axis in voxel units,
    clipped to the volume; D 162 with M 32 or D 642 with M 64)."""
    import synth
    out = []
    for v, (e, raw, c, a, r, small) in enumerate(fast_subvolume_batch(seed, n_vol, edge_lo, edge_hi, device)):
        vseed = seed * 1000003 + v
        rng = np.random.default_rng(vseed)
        h = np.array([1.0, 1.0, 2.0])
        ext = (e - 1) * h
        seeds = np.clip(c + rng.uniform(-1.0, 1.0, size=c.shape) * h, 0.0, ext)
        p = synth.slab_params(vseed & ((1 << 63) - 1), n_dirs=162 if small else 642, n_rays=32 if small else 64)
        wl = synth.Workload("sub%03d-%d^3-%d" % (v, e, len(seeds)), raw, p, synth.icosphere(2 if small else 3),
                            seeds, np.arange(len(seeds), dtype=np.uint32), n_iter,
                            {"centers": c, "axes": a, "rots": r})
        out.append(wl)
    return out


def served_volume(seed: int, shape_xyz=(2048, 2048, 512)) -> LargeVolume:
    """The served workload's volume: 2048 x 2048 x 512 uint16, h = (1, 1, 2), about 215,000 nuclei at
    20-400 per 128^3 block, PSF 1.2 voxels, gain 0.7-1, Poisson counts (background 100, peak 900)."""
    return LargeVolume(seed, shape_xyz=shape_xyz)


def tile_workload(vol: LargeVolume, lo, hi, idx, raw, n_iter: int = 200, seed: int = 0):
    """A tile request as a synth.Workload: `raw` is the tile's voxels [lo, hi) (any array or tensor),
    seeds are the true centres of objects `idx` in tile coordinates, ids their global object indices;
    D 162, M 32, L 16."""
    import synth
    h = vol.h
    c = vol.objects().centers[idx] - np.asarray(lo, np.float64) * h
    p = synth.slab_params(seed, n_dirs=162, n_rays=32)
    if "ico2" not in _CACHE:
        _CACHE["ico2"] = synth.icosphere(2)
    return synth.Workload("tile-%dx%dx%d-%d" % tuple(list(np.asarray(hi) - np.asarray(lo)) + [len(idx)]), raw, p,
                          _CACHE["ico2"], c, np.asarray(idx, np.uint32), n_iter, {})
