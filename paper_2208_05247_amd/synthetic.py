"""Seeded synthetic inputs: gas profiles, cumulus cloud fields, surface albedo.

This module only *builds inputs*; it holds none of the tracer's arithmetic.
Both the HIP path and the CPU oracle consume the FP32 arrays it returns.

The fields follow the paper's inputs (sec. 2.3: total extinction k_ext,
cloud extinction k_ext,cloud, single-scattering albedo omega0, asymmetry g)
and its scales (sec. 2.1: cloud base/top around 1300/2000 m, cover 0.3-0.7,
albedo 0.22; sec. 2.2: 50 m horizontal, 20 m vertical spacing).  The paper's
own LES fields are not available; Gaussian cloud blobs stand in for them.

Recipe (all randomness from ``numpy.random.default_rng(seed)``):
  gas        k_gas(z) = k0 * exp(-z / 8000 m) at cell centres, ssa_gas fixed,
             Rayleigh phase function (g = 0 where there is no cloud).
  clouds     n blobs; centre x, y ~ U[0, L), z ~ U[z_lo, z_hi]; sigma ~
             U[150, 400] m (isotropic); contribution A * exp(-r^2 / 2 sigma^2)
             with periodic minimum-image distance r, cut to 0 beyond r >
             2 sigma; k_cld is the sum of the contributions, zeroed outside
             the [cloud_base, cloud_top] layer when those are given.
  mixing     k_ext = k_gas + k_cld;  ssa = (k_gas ssa_gas + k_cld ssa_cld) /
             k_ext;  g = g_cld where k_cld > 0 else 0.
"""
from __future__ import annotations

import dataclasses
from typing import Optional

import numpy as np


@dataclasses.dataclass(frozen=True)
class Grid:
    nx: int
    ny: int
    nz: int
    dx: float
    dy: float
    dz: float

    @property
    def shape3(self):
        return (self.nz, self.ny, self.nx)

    @property
    def shape2(self):
        return (self.ny, self.nx)

    @property
    def ncol(self):
        return self.nx * self.ny

    @property
    def ncell(self):
        return self.nx * self.ny * self.nz


@dataclasses.dataclass
class Fields:
    """FP32 optical properties [nz][ny][nx] plus surface albedo [ny][nx]."""

    grid: Grid
    k_ext: np.ndarray
    k_ext_cloud: np.ndarray
    ssa: np.ndarray
    g: np.ndarray
    albedo: np.ndarray

    def arrays(self):
        return (self.k_ext, self.k_ext_cloud, self.ssa, self.g)


def z_centres(grid: Grid) -> np.ndarray:
    return (np.arange(grid.nz, dtype=np.float64) + 0.5) * grid.dz


def gas_profile(grid: Grid, k0: float = 1e-5, scale_height: float = 8000.0) -> np.ndarray:
    """Gas extinction per level, k0 * exp(-z / H) at cell centres (m^-1)."""
    return k0 * np.exp(-z_centres(grid) / scale_height)


def gas_profile_column_tau(grid: Grid, tau: float, scale_height: float = 8000.0) -> np.ndarray:
    """exp(-z/H)-shaped gas profile scaled to a given column optical depth."""
    shape = np.exp(-z_centres(grid) / scale_height)
    return shape * (tau / (shape.sum() * grid.dz))


def cloud_blobs(grid: Grid, rng: np.random.Generator, n_blobs: int,
                amplitude, sigma_range=(150.0, 400.0), z_range=(800.0, 2000.0),
                layer: Optional[tuple] = None, centre_margin: bool = False) -> np.ndarray:
    """Sum of truncated Gaussian blobs (FP64 [nz][ny][nx], m^-1).

    amplitude: a float (every blob) or a callable rng -> float.
    centre_margin: keep centres at least sigma inside the z range.
    """
    nx, ny, nz = grid.nx, grid.ny, grid.nz
    Lx, Ly = nx * grid.dx, ny * grid.dy
    k = np.zeros(grid.shape3, dtype=np.float64)
    xc_cells = (np.arange(nx) + 0.5) * grid.dx
    yc_cells = (np.arange(ny) + 0.5) * grid.dy
    zc_cells = z_centres(grid)
    for _ in range(n_blobs):
        cx = rng.uniform(0.0, Lx)
        cy = rng.uniform(0.0, Ly)
        sig = rng.uniform(*sigma_range)
        lo, hi = z_range
        if centre_margin:
            lo, hi = lo + sig, max(lo + sig, hi - sig)
        cz = rng.uniform(lo, hi)
        amp = amplitude(rng) if callable(amplitude) else float(amplitude)
        cut = 2.0 * sig
        # periodic minimum-image offsets in x and y
        ddx = (xc_cells - cx + 0.5 * Lx) % Lx - 0.5 * Lx
        ddy = (yc_cells - cy + 0.5 * Ly) % Ly - 0.5 * Ly
        ddz = zc_cells - cz
        ix = np.nonzero(np.abs(ddx) <= cut)[0]
        iy = np.nonzero(np.abs(ddy) <= cut)[0]
        iz = np.nonzero(np.abs(ddz) <= cut)[0]
        if ix.size == 0 or iy.size == 0 or iz.size == 0:
            continue
        r2 = (ddz[iz, None, None] ** 2 + ddy[None, iy, None] ** 2
              + ddx[None, None, ix] ** 2)
        contrib = amp * np.exp(-r2 / (2.0 * sig * sig))
        contrib[r2 > cut * cut] = 0.0
        k[np.ix_(iz, iy, ix)] += contrib
    if layer is not None:
        base, top = layer
        outside = (zc_cells < base) | (zc_cells > top)
        k[outside, :, :] = 0.0
    return k


def mix(grid: Grid, k_gas_z: np.ndarray, ssa_gas, k_cld: np.ndarray,
        ssa_cld: float, g_cld: float, albedo) -> Fields:
    """Combine a gas profile and a cloud field into the four FP32 inputs."""
    kg = np.broadcast_to(np.asarray(k_gas_z, dtype=np.float64)[:, None, None], grid.shape3)
    sg = np.broadcast_to(np.asarray(ssa_gas, dtype=np.float64).reshape(-1, 1, 1)
                         if np.ndim(ssa_gas) else np.float64(ssa_gas), grid.shape3)
    k_ext64 = kg + k_cld
    with np.errstate(invalid="ignore", divide="ignore"):
        ssa64 = np.where(k_ext64 > 0.0, (kg * sg + k_cld * ssa_cld) / k_ext64, 0.0)
    k_ext = k_ext64.astype(np.float32)
    k_cld32 = k_cld.astype(np.float32)
    ssa = np.clip(ssa64, 0.0, 1.0).astype(np.float32)
    g = np.where(k_cld32 > 0.0, np.float32(g_cld), np.float32(0.0)).astype(np.float32)
    if np.ndim(albedo) == 0:
        alb = np.full(grid.shape2, albedo, dtype=np.float32)
    else:
        alb = np.ascontiguousarray(albedo, dtype=np.float32)
    return Fields(grid, np.ascontiguousarray(k_ext), np.ascontiguousarray(k_cld32),
                  np.ascontiguousarray(ssa), np.ascontiguousarray(g), alb)


# ---------------------------------------------------------------------------
# Named workloads
# ---------------------------------------------------------------------------

@dataclasses.dataclass
class Workload:
    name: str
    fields: Fields
    sza: float
    azimuth: float
    photons: int
    seed: int
    brick: tuple


def small_cumulus(seed: int = 1) -> Workload:
    """32x32x64 cells of 100x100x50 m, 4 blobs (peak 0.05 m^-1, ssa 0.999,
    g 0.85) over exp(-z/8 km) gas (1e-5 m^-1, ssa 0.9), albedo 0.2, sun at
    30 deg zenith / 0 deg azimuth, 2^20 photons, bricks 4x4x4."""
    grid = Grid(32, 32, 64, 100.0, 100.0, 50.0)
    rng = np.random.default_rng(seed)
    kc = cloud_blobs(grid, rng, 4, 0.05, z_range=(800.0, 2000.0))
    f = mix(grid, gas_profile(grid), 0.9, kc, 0.999, 0.85, 0.2)
    return Workload("cumulus_32x32x64", f, 30.0, 0.0, 1 << 20, 1, (4, 4, 4))


def les_cumulus(seed: int = 1, nx: int = 256, ny: int = 256, nz: int = 128,
                dx: float = 50.0, dz: float = 25.0, n_blobs: int = 200,
                photons: int = 1 << 26, sza: float = 45.0, brick=(8, 8, 8),
                albedo=0.2) -> Workload:
    """LES-shaped cumulus: 256x256x128 cells of 50x50x25 m, 200 blobs with
    log-normal amplitude (median 0.02 m^-1, sigma_ln 0.5), cloud layer
    700-2500 m, ssa 0.9995, g 0.86, sun at 45 deg zenith, 2^26 photons,
    bricks 8x8x8."""
    grid = Grid(nx, ny, nz, dx, dx, dz)
    rng = np.random.default_rng(seed)
    amp = lambda r: float(0.02 * np.exp(0.5 * r.standard_normal()))
    kc = cloud_blobs(grid, rng, n_blobs, amp, z_range=(700.0, 2500.0),
                     layer=(700.0, 2500.0), centre_margin=True)
    f = mix(grid, gas_profile(grid), 0.9, kc, 0.9995, 0.86, albedo)
    return Workload(f"les_cumulus_{nx}x{ny}x{nz}", f, sza, 0.0, photons, 1, tuple(brick))


def uniform_fields(grid: Grid, k_ext_z, k_cld_z=None, ssa_z=0.0, g_z=0.0, albedo=0.0) -> Fields:
    """Horizontally uniform fields from per-level values (scalars broadcast)."""
    def lev(v):
        return np.broadcast_to(np.asarray(v, dtype=np.float64).reshape(-1), (grid.nz,)).copy()
    ke = lev(k_ext_z)
    kc = lev(0.0 if k_cld_z is None else k_cld_z)
    ss = lev(ssa_z)
    gg = lev(g_z)
    shp = grid.shape3
    f = Fields(grid,
               np.ascontiguousarray(np.broadcast_to(ke.astype(np.float32)[:, None, None], shp)),
               np.ascontiguousarray(np.broadcast_to(kc.astype(np.float32)[:, None, None], shp)),
               np.ascontiguousarray(np.broadcast_to(ss.astype(np.float32)[:, None, None], shp)),
               np.ascontiguousarray(np.broadcast_to(gg.astype(np.float32)[:, None, None], shp)),
               np.full(grid.shape2, albedo, dtype=np.float32) if np.ndim(albedo) == 0
               else np.ascontiguousarray(albedo, dtype=np.float32))
    return f


def random_fields(grid: Grid, seed: int, k_max: float = 0.02, cloud_frac: float = 0.5,
                  albedo_range=(0.0, 1.0)) -> Fields:
    """Cell-wise random fields for small brute-force and edge-case tests."""
    rng = np.random.default_rng(seed)
    ke = rng.uniform(0.0, k_max, grid.shape3)
    kc = ke * rng.uniform(0.0, 1.0, grid.shape3) * (rng.uniform(0, 1, grid.shape3) < cloud_frac)
    ss = rng.uniform(0.0, 1.0, grid.shape3)
    gg = rng.uniform(-0.9, 0.95, grid.shape3)
    alb = rng.uniform(*albedo_range, grid.shape2)
    ke32 = ke.astype(np.float32)
    kc32 = np.minimum(kc.astype(np.float32), ke32)
    return Fields(grid, ke32, kc32, ss.astype(np.float32), gg.astype(np.float32),
                  alb.astype(np.float32))


# ---------------------------------------------------------------------------
# Several g-points: factored medium (per-g-point gas profiles, shared clouds)
# ---------------------------------------------------------------------------

@dataclasses.dataclass
class BatchedMedium:
    """FP32 factored medium: k_gas, ssa_gas [ngp][nz]; k_cloud, ssa_cloud,
    g_cloud [nz][ny][nx]; albedo [ny][nx]; flux weights [ngp]."""

    grid: Grid
    k_gas: np.ndarray
    ssa_gas: np.ndarray
    k_cloud: np.ndarray
    ssa_cloud: np.ndarray
    g_cloud: np.ndarray
    albedo: np.ndarray
    weights: np.ndarray

    @property
    def n_gpoints(self) -> int:
        return int(self.k_gas.shape[0])

    def fields_of(self, n: int) -> Fields:
        """Full FP32 optical properties of g-point n (k_ext = k_gas + k_cloud,
        omega0 k_ext = ssa_gas k_gas + ssa_cloud k_cloud)."""
        kg = self.k_gas[n].astype(np.float64)[:, None, None]
        og = self.ssa_gas[n].astype(np.float64)[:, None, None]
        kc = self.k_cloud.astype(np.float64)
        oc = self.ssa_cloud.astype(np.float64)
        ke = kg + kc
        with np.errstate(invalid="ignore", divide="ignore"):
            om = np.where(ke > 0.0, (kg * og + kc * oc) / ke, 0.0)
        ke32 = ke.astype(np.float32)
        return Fields(self.grid, np.ascontiguousarray(ke32),
                      np.ascontiguousarray(np.minimum(self.k_cloud, ke32)),
                      np.ascontiguousarray(np.clip(om, 0.0, 1.0).astype(np.float32)),
                      np.ascontiguousarray(self.g_cloud), self.albedo)


@dataclasses.dataclass
class BatchedWorkload:
    name: str
    medium: BatchedMedium
    sza: float
    azimuth: float
    photons: np.ndarray  # per g-point
    seed: int
    brick: tuple


def gpoint_set(grid: Grid, n_gp: int, rng: np.random.Generator, tau_range=(1e-3, 50.0),
               ssa_range=(0.2, 1.0)):
    """Synthetic shortwave g-points: gas column optical depth log-uniform in
    tau_range with an exp(-z/8 km) profile, gas ssa uniform in ssa_range,
    TOA flux weights Dirichlet(1)."""
    tau = np.exp(rng.uniform(np.log(tau_range[0]), np.log(tau_range[1]), n_gp))
    ssa = rng.uniform(*ssa_range, n_gp)
    w = rng.dirichlet(np.ones(n_gp))
    kg = np.stack([gas_profile_column_tau(grid, t) for t in tau]).astype(np.float32)
    og = np.repeat(ssa[:, None], grid.nz, axis=1).astype(np.float32)
    return kg, og, w


def clear_sky_columns(medium: "BatchedMedium", n_above: int = 32, top: float = 60000.0,
                      scale_height: float = 8000.0):
    """Clear-sky columns of the g-points from the top of the atmosphere to
    the surface, the input of the two-stream calculation of the flux at the
    top of the domain: n_above equal layers between the domain top H and
    `top` continue each g-point's gas profile as k(z) = k_top exp(-(z - z_top)
    / scale_height) (k_top, z_top: the domain's top level and its centre)
    with that level's single-scattering albedo; below them the domain's own
    gas levels.  Returns FP64 (tau, ssa, g) [ngp][n_above + nz] with layer 0
    at the top of the atmosphere (g = 0: Rayleigh gas); the top of the domain
    is level n_above."""
    grid = medium.grid
    H = grid.nz * grid.dz
    z_top = H - 0.5 * grid.dz
    edges = np.linspace(top, H, n_above + 1)            # downward
    kg = medium.k_gas.astype(np.float64)
    og = medium.ssa_gas.astype(np.float64)
    k_top = kg[:, -1:]
    # exact layer integrals of k_top exp(-(z - z_top)/Hs) between the edges
    up = np.exp(-(edges[:-1] - z_top) / scale_height)
    lo = np.exp(-(edges[1:] - z_top) / scale_height)
    tau_above = k_top * scale_height * (lo - up)[None, :]
    tau_dom = (kg * grid.dz)[:, ::-1]                   # top level first
    tau = np.concatenate([tau_above, tau_dom], axis=1)
    ssa = np.concatenate([np.repeat(og[:, -1:], n_above, axis=1), og[:, ::-1]], axis=1)
    return np.ascontiguousarray(tau), np.ascontiguousarray(ssa), np.zeros_like(tau)


def batched_cumulus(seed: int = 1, nx: int = 512, ny: int = 512, nz: int = 96, dx: float = 50.0,
                    dz: float = 32.0, n_gp: int = 112, photons: int = 1 << 28, n_blobs=None,
                    sza: float = 45.0, brick=(8, 8, 8), albedo=0.2) -> BatchedWorkload:
    """Batched g-points over an LES-shaped cumulus field: 512x512x96 cells
    of 50x50x32 m, 112 g-points, photon counts Multinomial(photons,
    weights) so every photon carries the same energy."""
    grid = Grid(nx, ny, nz, dx, dx, dz)
    rng = np.random.default_rng(seed)
    if n_blobs is None:  # the LES case's density: 200 blobs per 12.8 x 12.8 km
        n_blobs = max(1, int(round(200 * (nx * dx) * (ny * dx) / 12800.0 ** 2)))
    amp = lambda r: float(0.02 * np.exp(0.5 * r.standard_normal()))
    kc = cloud_blobs(grid, rng, n_blobs, amp, z_range=(700.0, 2500.0), layer=(700.0, 2500.0),
                     centre_margin=True).astype(np.float32)
    oc = np.where(kc > 0, np.float32(0.9995), np.float32(0.0)).astype(np.float32)
    gc = np.where(kc > 0, np.float32(0.86), np.float32(0.0)).astype(np.float32)
    kg, og, w = gpoint_set(grid, n_gp, rng)
    counts = rng.multinomial(photons, w).astype(np.uint64)
    alb = np.full(grid.shape2, albedo, dtype=np.float32) if np.ndim(albedo) == 0 else \
        np.ascontiguousarray(albedo, dtype=np.float32)
    med = BatchedMedium(grid, kg, og, kc, oc, gc, alb, w)
    return BatchedWorkload(f"batched_cumulus_{nx}x{ny}x{nz}_{n_gp}g", med, sza, 0.0, counts, seed,
                           tuple(brick))
