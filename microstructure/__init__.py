"""Seeded synthetic microstructures and material tables.

This module only draws random numbers and labels voxels; it holds none of
the homogenization arithmetic.  Both the FP64 CPU oracle and the GPU path
consume what it produces, so parity never depends on two random number
generators agreeing.

Conventions
-----------
* A grid has shape ``(nz, ny, nx)``; arrays are C-ordered with x fastest.
* A phase map is ``uint8`` with one label per voxel.
* Voxel ``(i, j, k)`` (x, y, z indices) has its centre at ``(i+1/2, j+1/2, k+1/2)``
  in voxel units; distances use the periodic minimum image.
* Randomness comes from SplitMix64 (Steele, Lea & Flood, "Fast splittable
  pseudorandom number generators", OOPSLA 2014), implemented from its
  published definition below.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

__all__ = [
    "SplitMix64",
    "sphere_inclusion",
    "boolean_spheres",
    "sphere_array",
    "voronoi_cells",
    "laminate",
    "eight_cube",
    "BatchSample",
    "batch_samples",
    "MaterialTable",
]

_MASK64 = (1 << 64) - 1


class SplitMix64:
    """SplitMix64: a 64-bit counter advanced by the golden-ratio increment,
    then mixed by two xor-shift-multiply rounds and a final xor-shift."""

    GAMMA = 0x9E3779B97F4A7C15

    def __init__(self, seed: int):
        self.state = seed & _MASK64

    def next_u64(self) -> int:
        self.state = (self.state + self.GAMMA) & _MASK64
        z = self.state
        z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & _MASK64
        z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & _MASK64
        return z ^ (z >> 31)

    def uniform(self) -> float:
        """Uniform double in [0, 1) from the top 53 bits."""
        return (self.next_u64() >> 11) * (1.0 / (1 << 53))

    def uniform_array(self, n: int) -> np.ndarray:
        """The next ``n`` uniforms, computed for all counters at once (the k-th
        draw mixes state + k * GAMMA, so the sequence equals n calls of
        ``uniform``)."""
        if n <= 0:
            return np.zeros(0)
        k = np.arange(1, n + 1, dtype=np.uint64)
        with np.errstate(over="ignore"):
            z = np.uint64(self.state) + k * np.uint64(self.GAMMA)
            z = (z ^ (z >> np.uint64(30))) * np.uint64(0xBF58476D1CE4E5B9)
            z = (z ^ (z >> np.uint64(27))) * np.uint64(0x94D049BB133111EB)
            z = z ^ (z >> np.uint64(31))
        self.state = (self.state + n * self.GAMMA) & _MASK64
        return (z >> np.uint64(11)).astype(np.float64) * (1.0 / (1 << 53))

    def poisson_fast(self, mean: float) -> int:
        """Same count and same draws consumed as ``poisson`` (count + 1
        uniforms), drawn in blocks."""
        start = self.state
        t, used = 0.0, 0
        block = int(mean + 6.0 * math.sqrt(mean) + 16)
        while True:
            u = self.uniform_array(block)
            c = t + np.cumsum(-np.log1p(-u))
            over = np.nonzero(c > mean)[0]
            if over.size:
                k = used + int(over[0])  # draws before the one that crossed
                self.state = (start + (k + 1) * self.GAMMA) & _MASK64
                return k
            t = float(c[-1])
            used += block

    def poisson(self, mean: float) -> int:
        """Poisson count by summing unit-rate exponential gaps until they
        exceed ``mean`` (exact for any mean; O(mean) draws)."""
        t, k = 0.0, 0
        while True:
            u = self.uniform()
            t += -math.log1p(-u)  # -log(1-u), u in [0,1) keeps the log finite
            if t > mean:
                return k
            k += 1

    def randint(self, n: int) -> int:
        """Uniform integer in [0, n)."""
        return int(self.uniform() * n)


@dataclass
class MaterialTable:
    """Per-phase Young's moduli and Poisson's ratios (index = phase label)."""

    E: np.ndarray
    nu: np.ndarray

    def __post_init__(self):
        self.E = np.asarray(self.E, dtype=np.float64).reshape(-1)
        self.nu = np.asarray(self.nu, dtype=np.float64).reshape(-1)
        assert self.E.shape == self.nu.shape

    @property
    def n_phases(self) -> int:
        return int(self.E.shape[0])


def _axis_offsets(n: int, c: float) -> np.ndarray:
    """Periodic minimum-image offsets from coordinate ``c`` to voxel centres."""
    d = (np.arange(n, dtype=np.float64) + 0.5) - c
    d -= n * np.round(d / n)
    return d


def sphere_inclusion(shape, center, radius) -> np.ndarray:
    """Label 1 inside one (periodic) sphere, 0 elsewhere.  A voxel is inside
    when its centre lies within ``radius`` of ``center`` (given in voxel units,
    ``center`` as (x, y, z))."""
    nz, ny, nx = shape
    dx = _axis_offsets(nx, center[0])
    dy = _axis_offsets(ny, center[1])
    dz = _axis_offsets(nz, center[2])
    r2 = dz[:, None, None] ** 2 + dy[None, :, None] ** 2 + dx[None, None, :] ** 2
    return (r2 <= radius * radius).astype(np.uint8)


def _stamp_equal_spheres(shape, centers, r, chunk=256):
    """Union of periodic spheres of one radius, all spheres of a chunk at once;
    the same voxel test (and float64 operation order) as ``_stamp_spheres``."""
    nz, ny, nx = shape
    out = np.zeros(shape, dtype=np.uint8)
    R = int(math.ceil(r)) + 2
    o = np.arange(-R, R + 1)
    r2 = r * r
    for a in range(0, len(centers), chunk):
        c = np.asarray(centers[a:a + chunk], dtype=np.float64)
        # per axis (z, y, x): candidate indices around the centre and offsets
        idx, off = [], []
        for col, n in ((2, nz), (1, ny), (0, nx)):
            cand = np.floor(c[:, col])[:, None].astype(np.int64) + o[None, :]
            off.append(cand + 0.5 - c[:, col][:, None])
            idx.append(np.mod(cand, n))
        dz2 = off[0][:, :, None, None] ** 2
        dy2 = off[1][:, None, :, None] ** 2
        dx2 = off[2][:, None, None, :] ** 2
        inside = (dz2 + dy2 + dx2) <= r2
        s_, i, j, k = np.nonzero(inside)
        out[idx[0][s_, i], idx[1][s_, j], idx[2][s_, k]] = 1
    return out


def _stamp_spheres(shape, centers, radii) -> np.ndarray:
    """Union of periodic spheres, stamped through each sphere's bounding box."""
    nz, ny, nx = shape
    out = np.zeros(shape, dtype=np.uint8)
    for (cx, cy, cz), r in zip(centers, radii):
        r2 = r * r
        idx = []
        off = []
        for n, c in ((nz, cz), (ny, cy), (nx, cx)):
            lo = int(math.floor(c - r - 0.5)) - 1
            hi = int(math.ceil(c + r - 0.5)) + 1
            cand = np.arange(lo, hi + 1)
            d = cand + 0.5 - c
            keep = np.abs(d) <= r + 1e-12
            cand, d = cand[keep], d[keep]
            if cand.size > n:  # sphere wider than the box: use all voxels
                d = _axis_offsets(n, c)
                cand = np.arange(n)
            idx.append(np.mod(cand, n))
            off.append(d)
        dz2 = off[0][:, None, None] ** 2
        dy2 = off[1][None, :, None] ** 2
        dx2 = off[2][None, None, :] ** 2
        inside = (dz2 + dy2 + dx2) <= r2
        sub = out[np.ix_(idx[0], idx[1], idx[2])]
        out[np.ix_(idx[0], idx[1], idx[2])] = np.maximum(sub, inside.astype(np.uint8))
    return out


@dataclass
class BooleanInfo:
    n_spheres: int
    centers: np.ndarray
    radius: float
    volume_fraction: float


def boolean_spheres(shape, radius: float, target_fraction: float, seed: int):
    """Boolean model of Poisson-placed overlapping spheres (periodized), the
    random medium of the paper's convergence study (§6.1).  The intensity
    theta is chosen so that 1 - exp(-theta * V_sphere) equals the requested
    volume fraction; the sphere count is Poisson with mean theta * volume.

    Returns (phase_map, BooleanInfo) with label 1 = spheres, 0 = matrix."""
    nz, ny, nx = shape
    rng = SplitMix64(seed)
    v_sphere = 4.0 * math.pi * radius ** 3 / 3.0
    theta = -math.log(1.0 - target_fraction) / v_sphere
    count = rng.poisson_fast(theta * nx * ny * nz)
    centers = rng.uniform_array(3 * count).reshape(count, 3) * np.array([nx, ny, nz], dtype=np.float64)
    if 2 * int(math.ceil(radius)) + 5 <= min(shape):
        phase = _stamp_equal_spheres(shape, centers, radius)
    else:
        phase = _stamp_spheres(shape, centers, [radius] * count)
    return phase, BooleanInfo(count, centers, radius, float(phase.mean()))


def sphere_array(L: int, volume_fraction: float) -> np.ndarray:
    """One centred sphere per periodic cell (§5.3, periodic array of spheres),
    radius from the requested volume fraction of the continuum cell."""
    r = (3.0 * volume_fraction / (4.0 * math.pi)) ** (1.0 / 3.0) * L
    return sphere_inclusion((L, L, L), (L / 2, L / 2, L / 2), r)


def voronoi_cells(shape, n_seeds: int, n_phases: int, seed: int):
    """Periodic Poisson-Voronoi tessellation: each voxel takes the label of the
    cell whose seed is nearest to its centre (ties: lowest seed index); each
    cell draws its phase uniformly among ``n_phases``.  Brute force over seeds,
    plane by plane, in FP64; meant for grids up to a few million voxels."""
    nz, ny, nx = shape
    rng = SplitMix64(seed)
    seeds = np.empty((n_seeds, 3))
    for s in range(n_seeds):
        seeds[s, 0] = rng.uniform() * nx
        seeds[s, 1] = rng.uniform() * ny
        seeds[s, 2] = rng.uniform() * nz
    cell_phase = np.array([rng.randint(n_phases) for _ in range(n_seeds)], dtype=np.uint8)
    out = np.empty(shape, dtype=np.uint8)
    ys = np.arange(ny) + 0.5
    xs = np.arange(nx) + 0.5
    for z in range(nz):
        best = np.full((ny, nx), np.inf)
        label = np.zeros((ny, nx), dtype=np.int64)
        dz = (z + 0.5) - seeds[:, 2]
        dz -= nz * np.round(dz / nz)
        for s in range(n_seeds):
            dy = ys - seeds[s, 1]
            dy -= ny * np.round(dy / ny)
            dx = xs - seeds[s, 0]
            dx -= nx * np.round(dx / nx)
            d2 = dz[s] * dz[s] + dy[:, None] ** 2 + dx[None, :] ** 2
            better = d2 < best
            best = np.where(better, d2, best)
            label = np.where(better, s, label)
        out[z] = cell_phase[label]
    return out, seeds, cell_phase


def voronoi_cells_fast(shape, n_seeds: int, n_phases: int, seed: int, workers: int = -1):
    """The tessellation of ``voronoi_cells`` (same seeds, same phases) labelled
    with a periodic k-d tree (scipy.spatial.cKDTree, boxsize = the cell) plane
    by plane: for grids of 10^9 voxels.  Exact ties between seeds (probability
    zero for continuous seed positions) may resolve to another index than the
    brute-force version's lowest one."""
    from scipy.spatial import cKDTree

    nz, ny, nx = shape
    rng = SplitMix64(seed)
    seeds = rng.uniform_array(3 * n_seeds).reshape(n_seeds, 3) * np.array([nx, ny, nz], dtype=np.float64)
    cell_phase = np.array([rng.randint(n_phases) for _ in range(n_seeds)], dtype=np.uint8)
    box = np.array([nx, ny, nz], dtype=np.float64)
    tree = cKDTree(np.mod(seeds, box), boxsize=box)
    out = np.empty(shape, dtype=np.uint8)
    xs = np.arange(nx) + 0.5
    ys = np.arange(ny) + 0.5
    gx, gy = np.meshgrid(xs, ys)
    pts = np.empty((ny * nx, 3))
    pts[:, 0] = gx.reshape(-1)
    pts[:, 1] = gy.reshape(-1)
    for z in range(nz):
        pts[:, 2] = z + 0.5
        _, lab = tree.query(pts, k=1, workers=workers)
        out[z] = cell_phase[lab].reshape(ny, nx)
    return out, seeds, cell_phase


def voronoi_cells_torch(shape, n_seeds: int, n_phases: int, seed: int, device="cuda", rows=16, progress=None):
    """``voronoi_cells`` evaluated with torch on ``device``: the same float64
    minimum-image squares dz^2, dy^2, dx^2 (precomputed per axis) summed in the
    same order, argmin keeping the first of equal distances (the lowest seed
    index).  ``rows`` y-rows are labelled per step; ``progress(z)`` (optional)
    is called after each plane.  Returns a uint8 tensor on ``device`` and the
    seeds and phases."""
    import torch

    nz, ny, nx = shape
    rng = SplitMix64(seed)
    seeds = np.empty((n_seeds, 3))
    for s in range(n_seeds):
        seeds[s, 0] = rng.uniform() * nx
        seeds[s, 1] = rng.uniform() * ny
        seeds[s, 2] = rng.uniform() * nz
    cell_phase = np.array([rng.randint(n_phases) for _ in range(n_seeds)], dtype=np.uint8)
    sd = torch.from_numpy(seeds).to(device)
    cp = torch.from_numpy(cell_phase).to(device)

    def sq(n, col):
        d = (torch.arange(n, device=device, dtype=torch.float64) + 0.5)[:, None] - sd[None, :, col]
        d = d - n * torch.round(d / n)
        return d * d

    dx2, dy2, dz2 = sq(nx, 0), sq(ny, 1), sq(nz, 2)  # (n, seeds)
    out = torch.empty((nz, ny, nx), dtype=torch.uint8, device=device)
    for z in range(nz):
        for a in range(0, ny, rows):
            zy = dz2[z][None, :] + dy2[a:a + rows]            # (rows, seeds)
            d2 = zy[:, None, :] + dx2[None, :, :]               # (rows, nx, seeds)
            out[z, a:a + rows] = cp[torch.argmin(d2, dim=2)]
        if progress is not None:
            progress(z)
    return out, seeds, cell_phase


def laminate(shape, layer_labels_along_x) -> np.ndarray:
    """Phase depends on the x index only: ``layer_labels_along_x[i]`` for every
    voxel with x index i."""
    nz, ny, nx = shape
    lab = np.asarray(layer_labels_along_x, dtype=np.uint8)
    assert lab.shape == (nx,)
    return np.broadcast_to(lab[None, None, :], shape).copy()


def eight_cube(L: int) -> np.ndarray:
    """The periodic cell cut into 8 cubes, the centred one being the inclusion
    (§5.2): label 1 on [L/4, 3L/4)^3, 0 elsewhere (L divisible by 4)."""
    assert L % 4 == 0
    out = np.zeros((L, L, L), dtype=np.uint8)
    a, b = L // 4, 3 * L // 4
    out[a:b, a:b, a:b] = 1
    return out


@dataclass
class BatchSample:
    L: int
    radius: float
    volume_fraction: float
    contrast: float
    nu: float
    load: int  # index of the unit macroscopic strain (Voigt order 11,22,33,23,13,12)
    seed: int
    phase: np.ndarray = field(repr=False, default=None)

    @property
    def materials(self) -> MaterialTable:
        return MaterialTable(E=[1.0, self.contrast], nu=[self.nu, self.nu])

    @property
    def macro_strain(self) -> np.ndarray:
        e = np.zeros(6)
        e[self.load] = 1.0
        return e


def batch_samples(n: int, seed: int, sizes=(32, 48, 64, 96), with_phase=True):
    """Seeded sphere-Boolean samples for batched solves: grid edge uniform over
    ``sizes``; volume fraction U[0.05, 0.4]; log10 contrast U[-2, 3]; one
    Poisson ratio U[0.2, 0.4] shared by both phases; sphere radius U[3, 8]
    voxels; one unit macroscopic strain drawn uniformly among the six."""
    rng = SplitMix64(seed)
    out = []
    for i in range(n):
        L = sizes[rng.randint(len(sizes))]
        f = 0.05 + 0.35 * rng.uniform()
        chi = 10.0 ** (-2.0 + 5.0 * rng.uniform())
        nu = 0.2 + 0.2 * rng.uniform()
        r = 3.0 + 5.0 * rng.uniform()
        load = rng.randint(6)
        s_seed = rng.next_u64()
        smp = BatchSample(L, r, f, chi, nu, load, s_seed)
        if with_phase:
            smp.phase, _ = boolean_spheres((L, L, L), r, f, s_seed)
        out.append(smp)
    return out
