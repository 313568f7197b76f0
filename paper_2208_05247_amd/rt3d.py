"""Python binding of the rt3d C ABI (include/rt3d.h): argument marshalling
only.  Every step of the tracer runs in the HIP library ``librt3d.so``;
PyTorch supplies device memory and the stream.  There is no CPU fallback:
if the library is missing or no HIP device is present, calls raise.

uint64 tallies are held in torch.int64 tensors (same bits); use
:func:`as_uint64` to view them as numpy uint64 on the host.
"""
from __future__ import annotations

import ctypes
import dataclasses
import os
from typing import Optional, Sequence

import numpy as np
import torch

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "librt3d.so")

OK, EINVAL, EDOMAIN, EDEVICE, ETOOBIG = 0, 1, 2, 3, 4
NOALLOC_SCRATCH_BYTES = 32 << 20  # RT3D_NOALLOC_SCRATCH_BYTES
FLAG_ACCUMULATE, FLAG_VALIDATE, FLAG_TIME, FLAG_NO_MERGE, FLAG_SOBOL_ENTRY = 0x1, 0x2, 0x4, 0x8, 0x10
FLAG_WAVE_AGGREGATE = 0x20
FLAG_CELL_MASK = 0x40
LEDGER = ("incoming", "toa", "atm_dir", "atm_dif", "sfc", "rr_gain", "rr_loss", "lost")
STATS = ("photons", "collisions", "null", "scat_gas", "scat_cloud", "surface", "escape",
         "rr_kill", "rr_survive", "crossings", "absorbed", "capped")
TALLY3 = ("abs_dir", "abs_dif")
TALLY2 = ("sfc_dir", "sfc_dif", "sfc_abs", "toa_up")
EXPORTS = ("rt3d_abi_version", "rt3d_status_string", "rt3d_last_device_error",
           "rt3d_default_options", "rt3d_workspace_size", "rt3d_majorant_build",
           "rt3d_trace", "rt3d_last_trace_ms", "rt3d_finalize", "rt3d_philox4x32_10",
           "rt3d_workspace_size_batched", "rt3d_trace_batched", "rt3d_sobol_entry", "rt3d_two_stream",
           "rt3d_phase_sample", "rt3d_turn", "rt3d_trace_noalloc", "rt3d_schedule_slots")
MAX_GPOINTS = 256


class Rt3dError(RuntimeError):
    def __init__(self, status: int, what: str, detail: str = ""):
        self.status = status
        super().__init__(f"{what}: status {status} ({_status_text(status)}) {detail}".rstrip())


class Grid(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("nz", ctypes.c_int32),
                ("dx", ctypes.c_float), ("dy", ctypes.c_float), ("dz", ctypes.c_float)]


class OpticalProps(ctypes.Structure):
    _fields_ = [("k_ext", ctypes.c_void_p), ("k_ext_cloud", ctypes.c_void_p),
                ("ssa", ctypes.c_void_p), ("g", ctypes.c_void_p)]


class TalliesStruct(ctypes.Structure):
    _fields_ = [(n, ctypes.c_void_p) for n in TALLY3 + TALLY2 + ("ledger", "stats")]


class Options(ctypes.Structure):
    _fields_ = [("brick_x", ctypes.c_int32), ("brick_y", ctypes.c_int32), ("brick_z", ctypes.c_int32),
                ("diffuse_fraction", ctypes.c_float), ("rr_threshold", ctypes.c_float),
                ("flags", ctypes.c_uint32), ("max_iters", ctypes.c_uint32),
                ("photon_offset", ctypes.c_uint64), ("grid_blocks", ctypes.c_int32),
                ("block_threads", ctypes.c_int32), ("lds_majorant", ctypes.c_int32),
                ("max_walk", ctypes.c_int32), ("pool_photons", ctypes.c_int32),
                ("refill_lanes", ctypes.c_int32), ("tile_x", ctypes.c_int32), ("tile_y", ctypes.c_int32)]


class BatchedMedium(ctypes.Structure):
    _fields_ = [("k_gas", ctypes.c_void_p), ("ssa_gas", ctypes.c_void_p), ("k_cloud", ctypes.c_void_p),
                ("ssa_cloud", ctypes.c_void_p), ("g_cloud", ctypes.c_void_p),
                ("diffuse_fraction", ctypes.c_void_p)]


_lib = None


def load(path: str = LIB_PATH):
    """Load librt3d.so (no GPU needed to load it)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"{path} is missing: build it with __graft_entry__.build() "
                           "(the tracer has no CPU fallback)")
    lib = ctypes.CDLL(path)
    P, Z = ctypes.c_void_p, ctypes.c_size_t
    lib.rt3d_abi_version.restype = ctypes.c_int
    lib.rt3d_status_string.argtypes = [ctypes.c_int]
    lib.rt3d_status_string.restype = ctypes.c_char_p
    lib.rt3d_last_device_error.restype = ctypes.c_char_p
    lib.rt3d_default_options.argtypes = [ctypes.POINTER(Options)]
    lib.rt3d_workspace_size.argtypes = [ctypes.POINTER(Grid), ctypes.POINTER(Options)]
    lib.rt3d_workspace_size.restype = Z
    lib.rt3d_majorant_build.argtypes = [ctypes.POINTER(Grid), P, ctypes.c_int32, ctypes.c_int32,
                                        ctypes.c_int32, P, P]
    lib.rt3d_trace.argtypes = [ctypes.POINTER(Grid), ctypes.POINTER(OpticalProps), P, ctypes.c_double,
                               ctypes.c_double, ctypes.c_uint64, ctypes.c_uint64, ctypes.POINTER(Options),
                               ctypes.POINTER(TalliesStruct), P, Z, P]
    lib.rt3d_trace_noalloc.argtypes = [ctypes.POINTER(Grid), ctypes.POINTER(OpticalProps), P, ctypes.c_double,
                                       ctypes.c_double, ctypes.c_uint64, ctypes.c_uint64, ctypes.POINTER(Options),
                                       ctypes.POINTER(TalliesStruct), P]
    lib.rt3d_last_trace_ms.argtypes = [ctypes.POINTER(ctypes.c_float)]
    lib.rt3d_workspace_size_batched.argtypes = [ctypes.POINTER(Grid), ctypes.c_int32, ctypes.POINTER(Options)]
    lib.rt3d_workspace_size_batched.restype = Z
    lib.rt3d_trace_batched.argtypes = [ctypes.POINTER(Grid), ctypes.c_int32, ctypes.POINTER(BatchedMedium), P, P,
                                       ctypes.c_double, ctypes.c_double, ctypes.c_uint64, ctypes.POINTER(Options),
                                       ctypes.POINTER(TalliesStruct), P, Z, P]
    lib.rt3d_finalize.argtypes = [ctypes.POINTER(Grid), ctypes.POINTER(TalliesStruct), ctypes.c_uint64, P,
                                  ctypes.c_double, P, P, P, P, P, P, P]
    lib.rt3d_philox4x32_10.argtypes = [P, ctypes.c_uint64, P, ctypes.c_uint32, P]
    lib.rt3d_sobol_entry.argtypes = [ctypes.c_uint64, ctypes.c_uint32, ctypes.c_uint64, ctypes.c_uint64, P, P]
    lib.rt3d_two_stream.argtypes = [ctypes.c_int32, ctypes.c_int32, P, P, P, P, ctypes.c_double, P, P, P, P,
                                    ctypes.c_int32, P, P, P]
    lib.rt3d_phase_sample.argtypes = [ctypes.c_int32, P, P, P, ctypes.c_uint32, P]
    lib.rt3d_turn.argtypes = [P, P, P, P, ctypes.c_uint32, P]
    lib.rt3d_schedule_slots.argtypes = [ctypes.POINTER(Grid), ctypes.c_int32, P, P, ctypes.POINTER(Options),
                                        ctypes.c_uint64, ctypes.c_uint64, P, P, P]
    for name in ("rt3d_majorant_build", "rt3d_trace", "rt3d_trace_noalloc", "rt3d_last_trace_ms", "rt3d_finalize",
                 "rt3d_philox4x32_10", "rt3d_trace_batched", "rt3d_sobol_entry", "rt3d_two_stream",
                 "rt3d_phase_sample", "rt3d_turn", "rt3d_trace_noalloc", "rt3d_schedule_slots"):
        getattr(lib, name).restype = ctypes.c_int
    if lib.rt3d_abi_version() != 3:
        raise RuntimeError("librt3d.so ABI version mismatch")
    _lib = lib
    return lib


def _status_text(status: int) -> str:
    try:
        return load().rt3d_status_string(status).decode()
    except Exception:  # noqa: BLE001 - only used to format an error
        return "?"


def _check(status: int, what: str):
    if status != OK:
        detail = load().rt3d_last_device_error().decode() if status in (EDEVICE, ETOOBIG) else ""
        raise Rt3dError(status, what, detail)


def _require_device(t: torch.Tensor, name: str, dtype=None):
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise ValueError(f"{name} must be a HIP device tensor")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if dtype is not None and t.dtype != dtype:
        raise ValueError(f"{name} must have dtype {dtype}")


def _stream(stream) -> ctypes.c_void_p:
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def grid_struct(grid) -> Grid:
    return Grid(int(grid.nx), int(grid.ny), int(grid.nz), float(grid.dx), float(grid.dy), float(grid.dz))


@dataclasses.dataclass
class DeviceFields:
    """FP32 device copies of the optical properties and surface albedo."""
    grid: object
    k_ext: torch.Tensor
    k_ext_cloud: torch.Tensor
    ssa: torch.Tensor
    g: torch.Tensor
    albedo: torch.Tensor

    @classmethod
    def from_host(cls, fields, device="cuda") -> "DeviceFields":
        def up(a):
            return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).to(device)
        return cls(fields.grid, up(fields.k_ext), up(fields.k_ext_cloud), up(fields.ssa), up(fields.g),
                   up(fields.albedo))


def options(brick=(8, 8, 8), diffuse_fraction=0.0, rr_threshold=0.5, flags=0, max_iters=0,
            photon_offset=0, grid_blocks=0, block_threads=0, lds_majorant=0, max_walk=0,
            pool_photons=0, refill_lanes=0, tile=(0, 0)) -> Options:
    o = Options()
    load().rt3d_default_options(ctypes.byref(o))
    o.brick_x, o.brick_y, o.brick_z = (int(b) for b in brick)
    o.diffuse_fraction = float(diffuse_fraction)
    o.rr_threshold = float(rr_threshold)
    o.flags = int(flags)
    o.max_iters = int(max_iters)
    o.photon_offset = int(photon_offset)
    o.grid_blocks = int(grid_blocks)
    o.block_threads = int(block_threads)
    o.lds_majorant = int(lds_majorant)
    o.max_walk = int(max_walk)
    o.pool_photons = int(pool_photons)
    o.refill_lanes = int(refill_lanes)
    o.tile_x, o.tile_y = (int(t) for t in tile)
    return o


def schedule_slots(grid, photons, col_offsets, opt: Options, first_slot: int = 0, n: int | None = None):
    """Host evaluation of the photon schedule (rt3d_schedule_slots): for work
    queue slots first_slot .. first_slot+n-1 the g-point, photon id and entry
    column each slot is traced as.  No device work."""
    counts = np.ascontiguousarray(photons, dtype=np.uint64)
    offs = np.ascontiguousarray(col_offsets, dtype=np.uint64)
    if counts.ndim != 1 or offs.shape != counts.shape or not 1 <= counts.size <= MAX_GPOINTS:
        raise ValueError("photons and col_offsets must be 1-D of equal length 1..256")
    if n is None:
        n = int(counts.sum()) - int(first_slot)
    gp = np.empty(n, np.int32)
    ids = np.empty(n, np.uint64)
    cols = np.empty(n, np.uint32)
    _check(load().rt3d_schedule_slots(ctypes.byref(grid_struct(grid)), counts.size, counts.ctypes.data,
                                      offs.ctypes.data, ctypes.byref(opt), int(first_slot), int(n),
                                      gp.ctypes.data, ids.ctypes.data, cols.ctypes.data), "rt3d_schedule_slots")
    return gp, ids, cols


def workspace_size(grid, opt: Options) -> int:
    n = load().rt3d_workspace_size(ctypes.byref(grid_struct(grid)), ctypes.byref(opt))
    if n == 0:
        raise Rt3dError(EINVAL, "rt3d_workspace_size")
    return int(n)


def alloc_tallies(grid, device="cuda") -> dict:
    t = {n: torch.empty(grid.shape3, dtype=torch.int64, device=device) for n in TALLY3}
    t.update({n: torch.empty(grid.shape2, dtype=torch.int64, device=device) for n in TALLY2})
    t["ledger"] = torch.empty(len(LEDGER), dtype=torch.int64, device=device)
    t["stats"] = torch.empty(len(STATS), dtype=torch.int64, device=device)
    return t


def alloc_workspace(nbytes: int, device="cuda") -> torch.Tensor:
    ws = torch.empty(nbytes + 256, dtype=torch.uint8, device=device)
    off = (-ws.data_ptr()) % 256
    return ws[off:off + nbytes]


def tallies_struct(t: dict) -> TalliesStruct:
    for n in TALLY3 + TALLY2 + ("ledger", "stats"):
        _require_device(t[n], n, torch.int64)
    return TalliesStruct(*[t[n].data_ptr() for n in TALLY3 + TALLY2 + ("ledger", "stats")])


def trace(df: DeviceFields, sza: float, azimuth: float, photons: int, seed: int, *,
          brick=(8, 8, 8), diffuse_fraction: float = 0.0, rr_threshold: float = 0.5,
          photon_offset: int = 0, accumulate: bool = False, validate: bool = False, timed: bool = False,
          max_iters: int = 0, grid_blocks: int = 0, lds_majorant: int = 0, max_walk: int = 0,
          pool_photons: int = 0, refill_lanes: int = 0, merge: bool = True, sobol_entry: bool = False,
          tile=(0, 0), wave_aggregate: bool = False, out: Optional[dict] = None,
          workspace: Optional[torch.Tensor] = None, stream=None) -> dict:
    """rt3d_trace: raw uint64 tallies (int64 tensors) of `photons` photons."""
    lib = load()
    grid = df.grid
    for n in ("k_ext", "k_ext_cloud", "ssa", "g", "albedo"):
        _require_device(getattr(df, n), n, torch.float32)
    flags = (FLAG_ACCUMULATE if accumulate else 0) | (FLAG_VALIDATE if validate else 0) | \
            (FLAG_TIME if timed else 0) | (0 if merge else FLAG_NO_MERGE) | (FLAG_SOBOL_ENTRY if sobol_entry else 0) | \
        (FLAG_WAVE_AGGREGATE if wave_aggregate else 0)
    opt = options(brick, diffuse_fraction, rr_threshold, flags, max_iters, photon_offset, grid_blocks,
                  lds_majorant=lds_majorant, max_walk=max_walk, pool_photons=pool_photons,
                  refill_lanes=refill_lanes, tile=tile)
    gs = grid_struct(grid)
    nws = workspace_size(grid, opt)
    if workspace is None:
        workspace = alloc_workspace(nws, df.k_ext.device)
    if out is None:
        out = alloc_tallies(grid, df.k_ext.device)
    props = OpticalProps(df.k_ext.data_ptr(), df.k_ext_cloud.data_ptr(), df.ssa.data_ptr(), df.g.data_ptr())
    ts = tallies_struct(out)
    st = lib.rt3d_trace(ctypes.byref(gs), ctypes.byref(props), ctypes.c_void_p(df.albedo.data_ptr()),
                        float(sza), float(azimuth), int(photons), int(seed), ctypes.byref(opt),
                        ctypes.byref(ts), ctypes.c_void_p(workspace.data_ptr()),
                        workspace.numel() * workspace.element_size(), _stream(stream))
    _check(st, "rt3d_trace")
    out["photons"] = int(photons)
    return out


def trace_noalloc(df: DeviceFields, sza: float, azimuth: float, photons: int, seed: int, out: dict, *,
                  brick=(8, 8, 8), diffuse_fraction: float = 0.0, rr_threshold: float = 0.5,
                  photon_offset: int = 0, accumulate: bool = False, validate: bool = False, max_iters: int = 0,
                  grid_blocks: int = 0, lds_majorant: int = 0, max_walk: int = 0, pool_photons: int = 0,
                  refill_lanes: int = 0, merge: bool = True, sobol_entry: bool = False, tile=(0, 0),
                  wave_aggregate: bool = False, stream=None) -> dict:
    """rt3d_trace_noalloc: rt3d_trace with the library's static scratch as
    workspace; `out` (tallies from alloc_tallies) must be given."""
    lib = load()
    for n in ("k_ext", "k_ext_cloud", "ssa", "g", "albedo"):
        _require_device(getattr(df, n), n, torch.float32)
    flags = (FLAG_ACCUMULATE if accumulate else 0) | (FLAG_VALIDATE if validate else 0) | \
            (0 if merge else FLAG_NO_MERGE) | (FLAG_SOBOL_ENTRY if sobol_entry else 0) | \
        (FLAG_WAVE_AGGREGATE if wave_aggregate else 0)
    opt = options(brick, diffuse_fraction, rr_threshold, flags, max_iters, photon_offset, grid_blocks,
                  lds_majorant=lds_majorant, max_walk=max_walk, pool_photons=pool_photons,
                  refill_lanes=refill_lanes, tile=tile)
    gs = grid_struct(df.grid)
    props = OpticalProps(df.k_ext.data_ptr(), df.k_ext_cloud.data_ptr(), df.ssa.data_ptr(), df.g.data_ptr())
    ts = tallies_struct(out)
    st = lib.rt3d_trace_noalloc(ctypes.byref(gs), ctypes.byref(props), ctypes.c_void_p(df.albedo.data_ptr()),
                                float(sza), float(azimuth), int(photons), int(seed), ctypes.byref(opt),
                                ctypes.byref(ts), _stream(stream))
    _check(st, "rt3d_trace_noalloc")
    out["photons"] = int(photons)
    return out


@dataclasses.dataclass
class DeviceBatchedMedium:
    """Factored medium of several g-points on the device: per-g-point gas
    profiles [ngp][nz] and one shared cloud field [nz][ny][nx]."""
    grid: object
    k_gas: torch.Tensor
    ssa_gas: torch.Tensor
    k_cloud: torch.Tensor
    ssa_cloud: torch.Tensor
    g_cloud: torch.Tensor
    albedo: torch.Tensor

    @property
    def n_gpoints(self) -> int:
        return int(self.k_gas.shape[0])

    @classmethod
    def from_host(cls, medium, device="cuda") -> "DeviceBatchedMedium":
        def up(a):
            return torch.from_numpy(np.array(a, dtype=np.float32, copy=True)).to(device)
        return cls(medium.grid, up(medium.k_gas), up(medium.ssa_gas), up(medium.k_cloud), up(medium.ssa_cloud),
                   up(medium.g_cloud), up(medium.albedo))


def workspace_size_batched(grid, n_gpoints: int, opt: Options) -> int:
    n = load().rt3d_workspace_size_batched(ctypes.byref(grid_struct(grid)), int(n_gpoints), ctypes.byref(opt))
    if n == 0:
        raise Rt3dError(EINVAL, "rt3d_workspace_size_batched")
    return int(n)


def trace_batched(dm: DeviceBatchedMedium, sza: float, azimuth: float, photons: Sequence[int], seed: int, *,
                  brick=(8, 8, 8), diffuse_fraction: float = 0.0, rr_threshold: float = 0.5,
                  accumulate: bool = False, validate: bool = False, timed: bool = False, max_iters: int = 0,
                  grid_blocks: int = 0, max_walk: int = 0, pool_photons: int = 0, refill_lanes: int = 0,
                  merge: bool = True, tile=(0, 0), wave_aggregate: bool = False, cell_mask: bool = False,
                  sobol_entry: bool = False, gpoint_diffuse: Optional[torch.Tensor] = None,
                  out: Optional[dict] = None, workspace: Optional[torch.Tensor] = None, stream=None) -> dict:
    """rt3d_trace_batched: broadband raw tallies of all g-points in one launch.
    gpoint_diffuse: FP32 device [ngp] diffuse fraction per g-point (e.g.
    two_stream()'s "tod_diffuse_fraction"), else diffuse_fraction for all."""
    lib = load()
    grid = dm.grid
    for n in ("k_gas", "ssa_gas", "k_cloud", "ssa_cloud", "g_cloud", "albedo"):
        _require_device(getattr(dm, n), n, torch.float32)
    ngp = dm.n_gpoints
    if len(photons) != ngp:
        raise ValueError("one photon count per g-point")
    if gpoint_diffuse is not None:
        _require_device(gpoint_diffuse, "gpoint_diffuse", torch.float32)
        if gpoint_diffuse.numel() != ngp:
            raise ValueError("gpoint_diffuse needs one value per g-point")
    flags = (FLAG_ACCUMULATE if accumulate else 0) | (FLAG_VALIDATE if validate else 0) | \
            (FLAG_TIME if timed else 0) | (0 if merge else FLAG_NO_MERGE) | (FLAG_SOBOL_ENTRY if sobol_entry else 0) | \
        (FLAG_WAVE_AGGREGATE if wave_aggregate else 0) | (FLAG_CELL_MASK if cell_mask else 0)
    opt = options(brick, diffuse_fraction, rr_threshold, flags, max_iters, 0, grid_blocks, max_walk=max_walk,
                  pool_photons=pool_photons, refill_lanes=refill_lanes, tile=tile)
    gs = grid_struct(grid)
    nws = workspace_size_batched(grid, ngp, opt)
    if workspace is None:
        workspace = alloc_workspace(nws, dm.k_cloud.device)
    if out is None:
        out = alloc_tallies(grid, dm.k_cloud.device)
    med = BatchedMedium(dm.k_gas.data_ptr(), dm.ssa_gas.data_ptr(), dm.k_cloud.data_ptr(),
                        dm.ssa_cloud.data_ptr(), dm.g_cloud.data_ptr(),
                        gpoint_diffuse.data_ptr() if gpoint_diffuse is not None else None)
    counts = np.ascontiguousarray(np.asarray(photons, dtype=np.uint64))
    ts = tallies_struct(out)
    st = lib.rt3d_trace_batched(ctypes.byref(gs), ngp, ctypes.byref(med), counts.ctypes.data_as(ctypes.c_void_p),
                                ctypes.c_void_p(dm.albedo.data_ptr()), float(sza), float(azimuth), int(seed),
                                ctypes.byref(opt), ctypes.byref(ts), ctypes.c_void_p(workspace.data_ptr()),
                                workspace.numel() * workspace.element_size(), _stream(stream))
    _check(st, "rt3d_trace_batched")
    out["photons"] = int(counts.sum())
    return out


def last_trace_ms() -> float:
    ms = ctypes.c_float()
    _check(load().rt3d_last_trace_ms(ctypes.byref(ms)), "rt3d_last_trace_ms")
    return float(ms.value)


def majorant_build(grid, k_ext: torch.Tensor, brick, stream=None) -> torch.Tensor:
    _require_device(k_ext, "k_ext", torch.float32)
    bx, by, bz = brick
    out = torch.empty((grid.nz // bz if grid.nz % bz == 0 else 1, grid.ny // by if grid.ny % by == 0 else 1,
                       grid.nx // bx if grid.nx % bx == 0 else 1), dtype=torch.float32, device=k_ext.device)
    _check(load().rt3d_majorant_build(ctypes.byref(grid_struct(grid)), ctypes.c_void_p(k_ext.data_ptr()),
                                      bx, by, bz, ctypes.c_void_p(out.data_ptr()), _stream(stream)),
           "rt3d_majorant_build")
    return out


def finalize(grid, raw: dict, photons: int, layer_scale: Optional[torch.Tensor] = None,
             flux_scale: float = 1.0, stream=None) -> dict:
    """rt3d_finalize: FP32 normalised tallies (fractions of the TOD flux,
    optionally scaled per layer / by flux_scale)."""
    dev = raw["abs_dir"].device
    out = {n: torch.empty(grid.shape3, dtype=torch.float32, device=dev) for n in TALLY3}
    out.update({n: torch.empty(grid.shape2, dtype=torch.float32, device=dev) for n in TALLY2})
    if layer_scale is not None:
        _require_device(layer_scale, "layer_scale", torch.float64)
        if layer_scale.numel() != grid.nz:
            raise ValueError("layer_scale must have nz entries")
    ts = tallies_struct(raw)
    ls = ctypes.c_void_p(layer_scale.data_ptr()) if layer_scale is not None else ctypes.c_void_p(0)
    _check(load().rt3d_finalize(ctypes.byref(grid_struct(grid)), ctypes.byref(ts), int(photons), ls,
                                float(flux_scale), *[ctypes.c_void_p(out[n].data_ptr())
                                                     for n in TALLY3 + TALLY2], _stream(stream)),
           "rt3d_finalize")
    return out


def philox4x32_10(ctr: torch.Tensor, seed: int, stream=None) -> torch.Tensor:
    """Philox4x32-10 of each row of ctr ([n,4] int32 device tensor holding
    uint32 bits)."""
    _require_device(ctr, "ctr", torch.int32)
    if ctr.dim() != 2 or ctr.shape[1] != 4:
        raise ValueError("ctr must be [n, 4]")
    out = torch.empty_like(ctr)
    _check(load().rt3d_philox4x32_10(ctypes.c_void_p(ctr.data_ptr()), int(seed), ctypes.c_void_p(out.data_ptr()),
                                     int(ctr.shape[0]), _stream(stream)), "rt3d_philox4x32_10")
    return out


def sobol_entry(first_pass: int, n: int, column: int, seed: int, device="cuda", stream=None) -> torch.Tensor:
    """rt3d_sobol_entry: scrambled entry coordinates [n, 2] (int32 device
    tensor holding the uint32 fractions of the column width)."""
    out = torch.empty((n, 2), dtype=torch.int32, device=device)
    _check(load().rt3d_sobol_entry(int(first_pass), int(n), int(column), int(seed),
                                   ctypes.c_void_p(out.data_ptr()), _stream(stream)), "rt3d_sobol_entry")
    return out


def phase_sample(kind: str, xi: torch.Tensor, g: Optional[torch.Tensor] = None, stream=None) -> torch.Tensor:
    """rt3d_phase_sample: the tracer's cos(scattering angle) for each xi
    (FP32 device tensor); kind "hg" (needs g, same shape) or "rayleigh"."""
    _require_device(xi, "xi", torch.float32)
    k = {"hg": 0, "rayleigh": 1}[kind]
    if k == 0:
        _require_device(g, "g", torch.float32)
        if g.shape != xi.shape:
            raise ValueError("g and xi must have the same shape")
    out = torch.empty_like(xi)
    gp = ctypes.c_void_p(g.data_ptr()) if g is not None else ctypes.c_void_p(0)
    _check(load().rt3d_phase_sample(k, gp, ctypes.c_void_p(xi.data_ptr()), ctypes.c_void_p(out.data_ptr()),
                                    xi.numel(), _stream(stream)), "rt3d_phase_sample")
    return out


def turn(d: torch.Tensor, mu: torch.Tensor, t: torch.Tensor, stream=None) -> torch.Tensor:
    """rt3d_turn: directions d [n, 3] turned by polar cosine mu [n] and
    azimuth 2 pi t [n] (FP32 device tensors)."""
    for name, a in (("d", d), ("mu", mu), ("t", t)):
        _require_device(a, name, torch.float32)
    n = mu.numel()
    if d.shape != (n, 3) or t.numel() != n:
        raise ValueError("d must be [n, 3], mu and t [n]")
    out = torch.empty_like(d)
    _check(load().rt3d_turn(ctypes.c_void_p(d.data_ptr()), ctypes.c_void_p(mu.data_ptr()),
                            ctypes.c_void_p(t.data_ptr()), ctypes.c_void_p(out.data_ptr()), n, _stream(stream)),
           "rt3d_turn")
    return out


def two_stream(tau: torch.Tensor, ssa: torch.Tensor, g: torch.Tensor, albedo: torch.Tensor, mu0: float,
               tod_level: int, flux_toa: Optional[torch.Tensor] = None, stream=None) -> dict:
    """rt3d_two_stream over columns [n_cols, nlay] (FP64 device tensors,
    layer 0 at the top of the atmosphere): level fluxes "dir", "dn_dif", "up"
    [n_cols, nlay+1] and, at level tod_level, "tod_flux" (FP64) and
    "tod_diffuse_fraction" (FP32)."""
    for name, t in (("tau", tau), ("ssa", ssa), ("g", g), ("albedo", albedo)):
        _require_device(t, name, torch.float64)
    if tau.dim() != 2 or ssa.shape != tau.shape or g.shape != tau.shape or albedo.numel() != tau.shape[0]:
        raise ValueError("tau, ssa, g must be [n_cols, nlay] and albedo [n_cols]")
    if flux_toa is not None:
        _require_device(flux_toa, "flux_toa", torch.float64)
        if flux_toa.numel() != tau.shape[0]:
            raise ValueError("flux_toa must have n_cols entries")
    nc, nl = int(tau.shape[0]), int(tau.shape[1])
    dev = tau.device
    out = {k: torch.empty((nc, nl + 1), dtype=torch.float64, device=dev) for k in ("dir", "dn_dif", "up")}
    out["tod_flux"] = torch.empty(nc, dtype=torch.float64, device=dev)
    out["tod_diffuse_fraction"] = torch.empty(nc, dtype=torch.float32, device=dev)
    ptr = lambda t: ctypes.c_void_p(t.data_ptr()) if t is not None else ctypes.c_void_p(0)
    _check(load().rt3d_two_stream(nc, nl, ptr(tau), ptr(ssa), ptr(g), ptr(albedo), float(mu0), ptr(flux_toa),
                                  ptr(out["dir"]), ptr(out["dn_dif"]), ptr(out["up"]), int(tod_level),
                                  ptr(out["tod_flux"]), ptr(out["tod_diffuse_fraction"]), _stream(stream)),
           "rt3d_two_stream")
    return out


def as_uint64(t: torch.Tensor) -> np.ndarray:
    return t.detach().cpu().numpy().view(np.uint64)


def to_host(raw: dict) -> dict:
    out = {k: as_uint64(v) for k, v in raw.items() if isinstance(v, torch.Tensor)}
    out["photons"] = raw.get("photons")
    return out


def events(raw_host: dict) -> int:
    """Photon events = tentative collisions + surface interactions."""
    s = raw_host["stats"]
    return int(s[STATS.index("collisions")]) + int(s[STATS.index("surface")])
