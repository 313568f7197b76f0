"""FP64 CPU oracle of the Monte Carlo solar photon tracer (sec. 2.3 of
Veerman, van Stratum and van Heerwaarden, GRL 2022).

TEST INFRASTRUCTURE ONLY: imported by the test suite, the smoke check and
the CPU-baseline leg of the benchmark, never by the product path.  It shares
no code with the HIP implementation.  The C library ``liboracle.so`` is
built from ``rt3d_oracle.c`` by :func:`build` (gcc, FP64, pthreads).

Parity status of each function (what pins it, see ``tests/``):
  philox4x32_10 / philox4x64_10  4x64 variant: numpy's Philox known-answer;
                                  4x32: uniformity / serial-correlation tests
                                  and bit-equality with the GPU generator
  hg_cos / rayleigh_cos          Legendre moments, chi^2 against the pdfs
  majorant                       brute-force max per block (numpy)
  trace                          Beer-Lambert closed forms, vacuum/absorber
                                  Lambertian closed forms (2 E_3), Milne
                                  integral equation for isotropic slabs, an
                                  analog brute-force Monte Carlo on tiny
                                  grids, exact ledger, invariances
  direct_transmittance            closed form for horizontally uniform layers
  finalize                        exact rational scaling, checked by hand
  sobol_points                    radical inverse by digit division; Pascal
                                  matrix mod 2 (Lucas); (0, m, 2)-net property
  owen_scramble / sobol_entry     nestedness, uniformity over seeds, nets kept,
                                  N^-1 convergence on smooth integrals and on
                                  slanted-sun surface irradiance; the traced
                                  entry points predicted photon by photon;
                                  the scramble-seed counter is pinned only by
                                  bit-equality with the GPU generator
  two_stream (module)             the boundary-value problem solved by exact
                                  matrix-exponential propagation; pinned by the
                                  adding method with closed-form layers (a
                                  different algorithm), pure absorber and
                                  conservation closed forms, thin-layer
                                  backscatter by quadrature, exact Monte Carlo
                                  transport within 6 %
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from typing import Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "rt3d_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lib = None

W_ONE = 2 ** 31
ORACLE_ABI = 2
LEDGER = ("incoming", "toa", "atm_dir", "atm_dif", "sfc", "rr_gain", "rr_loss", "lost")
STATS = ("photons", "collisions", "null", "scat_gas", "scat_cloud", "surface", "escape",
         "rr_kill", "rr_survive", "crossings", "absorbed", "capped")


def build(force: bool = True) -> str:
    """Compile liboracle.so with gcc (FP64, no fast-math)."""
    if force or not os.path.exists(_LIB):
        cmd = ["gcc", "-O2", "-std=c11", "-Wall", "-fPIC", "-shared", "-pthread",
               _SRC, "-o", _LIB + ".tmp", "-lm"]
        subprocess.check_call(cmd)
        os.replace(_LIB + ".tmp", _LIB)
    return _LIB


class _Problem(ctypes.Structure):
    _fields_ = [
        ("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("nz", ctypes.c_int32),
        ("bx", ctypes.c_int32), ("by", ctypes.c_int32), ("bz", ctypes.c_int32),
        ("dx", ctypes.c_double), ("dy", ctypes.c_double), ("dz", ctypes.c_double),
        ("k_ext", ctypes.c_void_p), ("k_ext_cloud", ctypes.c_void_p),
        ("ssa", ctypes.c_void_p), ("g", ctypes.c_void_p), ("albedo", ctypes.c_void_p),
        ("sza_deg", ctypes.c_double), ("azimuth_deg", ctypes.c_double),
        ("photons", ctypes.c_uint64), ("seed", ctypes.c_uint64),
        ("photon_offset", ctypes.c_uint64),
        ("diffuse_fraction", ctypes.c_double), ("rr_threshold", ctypes.c_double),
        ("max_iters", ctypes.c_uint32), ("nthreads", ctypes.c_int32),
        ("sobol_entry", ctypes.c_int32),
    ]


class _Tallies(ctypes.Structure):
    _fields_ = [(n, ctypes.c_void_p) for n in
                ("abs_dir", "abs_dif", "sfc_dir", "sfc_dif", "sfc_abs", "toa_up", "ledger", "stats")]


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build(force=True)
        lib = ctypes.CDLL(_LIB)
        if lib.oracle_abi() != ORACLE_ABI:
            raise RuntimeError(f"{_LIB} is out of date: rebuild it with oracle.build()")
        P = ctypes.c_void_p
        lib.oracle_philox4x32_10_n.argtypes = [P, ctypes.c_uint64, P, ctypes.c_uint64]
        lib.oracle_philox4x64_10.argtypes = [P, P, P]
        lib.oracle_hg_cos_n.argtypes = [ctypes.c_double, P, P, ctypes.c_uint64]
        lib.oracle_rayleigh_cos_n.argtypes = [P, P, ctypes.c_uint64]
        lib.oracle_turn.argtypes = [P, ctypes.c_double, ctypes.c_double, P]
        lib.oracle_majorant.argtypes = [ctypes.c_int32] * 6 + [P, P]
        lib.oracle_majorant.restype = ctypes.c_int
        lib.oracle_trace.argtypes = [ctypes.POINTER(_Problem), ctypes.POINTER(_Tallies)]
        lib.oracle_trace.restype = ctypes.c_int
        lib.oracle_direct_transmittance.argtypes = (
            [ctypes.c_int32] * 3 + [ctypes.c_double] * 3 + [P, ctypes.c_double, ctypes.c_double]
            + [ctypes.c_int32] * 3)
        lib.oracle_direct_transmittance.restype = ctypes.c_double
        lib.oracle_sobol_points_n.argtypes = [P, ctypes.c_uint32, P, P]
        lib.oracle_owen_scramble_n.argtypes = [P, ctypes.c_uint32, ctypes.c_uint32, P]
        lib.oracle_sobol_entry.argtypes = [ctypes.c_uint64, ctypes.c_uint32, ctypes.c_uint64, ctypes.c_uint64, P]
        _lib = lib
    return _lib


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


# ---------------------------------------------------------------------------
# Random numbers and samplers
# ---------------------------------------------------------------------------

def philox4x32_10(ctr: np.ndarray, seed: int) -> np.ndarray:
    """Philox4x32-10 of each row of ctr ([n,4] uint32), key = seed halves."""
    c = np.ascontiguousarray(ctr, dtype=np.uint32).reshape(-1, 4)
    out = np.empty_like(c)
    _load().oracle_philox4x32_10_n(_ptr(c), ctypes.c_uint64(seed), _ptr(out), c.shape[0])
    return out


def philox4x64_10(ctr, key) -> np.ndarray:
    c = np.ascontiguousarray(ctr, dtype=np.uint64).reshape(4)
    k = np.ascontiguousarray(key, dtype=np.uint64).reshape(2)
    out = np.empty(4, dtype=np.uint64)
    _load().oracle_philox4x64_10(_ptr(c), _ptr(k), _ptr(out))
    return out


def hg_cos(g: float, xi: np.ndarray) -> np.ndarray:
    x = np.ascontiguousarray(xi, dtype=np.float64)
    out = np.empty_like(x)
    _load().oracle_hg_cos_n(float(g), _ptr(x), _ptr(out), x.size)
    return out


def rayleigh_cos(xi: np.ndarray) -> np.ndarray:
    x = np.ascontiguousarray(xi, dtype=np.float64)
    out = np.empty_like(x)
    _load().oracle_rayleigh_cos_n(_ptr(x), _ptr(out), x.size)
    return out


def turn(d, mu: float, phi: float) -> np.ndarray:
    dd = np.ascontiguousarray(d, dtype=np.float64)
    out = np.empty(3, dtype=np.float64)
    _load().oracle_turn(_ptr(dd), float(mu), float(phi), _ptr(out))
    return out


# ---------------------------------------------------------------------------
# Acceleration grid and tracing
# ---------------------------------------------------------------------------

def majorant(k_ext: np.ndarray, brick) -> np.ndarray:
    k = np.ascontiguousarray(k_ext, dtype=np.float32)
    nz, ny, nx = k.shape
    bx, by, bz = brick
    out = np.empty((nz // bz, ny // by, nx // bx), dtype=np.float32)
    rc = _load().oracle_majorant(nx, ny, nz, bx, by, bz, _ptr(k), _ptr(out))
    if rc != 0:
        raise ValueError("oracle_majorant: bad arguments")
    return out


def sobol_points(i) -> tuple:
    """Unscrambled 2D Sobol points (32-bit fractions) of indices i."""
    i = np.ascontiguousarray(i, dtype=np.uint32)
    a = np.empty_like(i)
    b = np.empty_like(i)
    _load().oracle_sobol_points_n(_ptr(i), i.size, _ptr(a), _ptr(b))
    return a, b


def owen_scramble(v, seed: int) -> np.ndarray:
    """Nested uniform scramble of 32-bit fractions v under a 32-bit seed."""
    v = np.ascontiguousarray(v, dtype=np.uint32)
    out = np.empty_like(v)
    _load().oracle_owen_scramble_n(_ptr(v), v.size, int(seed) & 0xffffffff, _ptr(out))
    return out


def sobol_entry(first: int, n: int, column: int, seed: int) -> np.ndarray:
    """Scrambled entry coordinates [n][2] (uint32 fractions of the column
    width) of passes first .. first+n-1 of a column, as the tracer uses them."""
    out = np.empty((n, 2), dtype=np.uint32)
    _load().oracle_sobol_entry(int(first), int(n), int(column), int(seed), _ptr(out))
    return out


def trace(fields, sza: float, azimuth: float, photons: int, seed: int,
          brick=(4, 4, 4), diffuse_fraction: float = 0.0, rr_threshold: float = 0.5,
          photon_offset: int = 0, max_iters: int = 1 << 24,
          nthreads: Optional[int] = None, sobol_entry: bool = False) -> dict:
    """Trace `photons` photons through `fields` (a synthetic.Fields); returns
    raw uint64 tallies, ledger and stats as numpy arrays (same units and
    meaning as the GPU library's raw tallies)."""
    grid = fields.grid
    arrs = [np.ascontiguousarray(a, dtype=np.float32) for a in fields.arrays()]
    alb = np.ascontiguousarray(fields.albedo, dtype=np.float32)
    if nthreads is None:
        nthreads = min(16, os.cpu_count() or 1)
    p = _Problem(grid.nx, grid.ny, grid.nz, brick[0], brick[1], brick[2],
                 grid.dx, grid.dy, grid.dz,
                 arrs[0].ctypes.data, arrs[1].ctypes.data, arrs[2].ctypes.data,
                 arrs[3].ctypes.data, alb.ctypes.data,
                 float(sza), float(azimuth), int(photons), int(seed), int(photon_offset),
                 float(diffuse_fraction), float(rr_threshold), int(max_iters), int(nthreads),
                 1 if sobol_entry else 0)
    out = {
        "abs_dir": np.zeros(grid.shape3, dtype=np.uint64),
        "abs_dif": np.zeros(grid.shape3, dtype=np.uint64),
        "sfc_dir": np.zeros(grid.shape2, dtype=np.uint64),
        "sfc_dif": np.zeros(grid.shape2, dtype=np.uint64),
        "sfc_abs": np.zeros(grid.shape2, dtype=np.uint64),
        "toa_up": np.zeros(grid.shape2, dtype=np.uint64),
        "ledger": np.zeros(len(LEDGER), dtype=np.uint64),
        "stats": np.zeros(len(STATS), dtype=np.uint64),
    }
    t = _Tallies(*[out[n].ctypes.data for n in
                   ("abs_dir", "abs_dif", "sfc_dir", "sfc_dif", "sfc_abs", "toa_up", "ledger", "stats")])
    rc = _load().oracle_trace(ctypes.byref(p), ctypes.byref(t))
    if rc != 0:
        raise ValueError(f"oracle_trace failed with code {rc}")
    out["photons"] = int(photons)
    return out


def direct_transmittance(fields, sza: float, azimuth: float, columns, n: int = 16) -> np.ndarray:
    """Expected direct surface irradiance (fraction of TOD flux) of the given
    surface columns [(i, j), ...] by deterministic line integrals."""
    grid = fields.grid
    k = np.ascontiguousarray(fields.k_ext, dtype=np.float32)
    lib = _load()
    return np.array([lib.oracle_direct_transmittance(grid.nx, grid.ny, grid.nz, grid.dx, grid.dy,
                                                     grid.dz, _ptr(k), float(sza), float(azimuth),
                                                     int(i), int(j), int(n))
                     for (i, j) in columns])


def finalize(raw: dict, grid, photons: int, layer_scale=None, flux_scale: float = 1.0) -> dict:
    """Normalise raw tallies: divide by (photons / ncol) * 2^31 (fractions of
    the TOD downward flux per column area), then scale 3D outputs per layer
    and 2D outputs by flux_scale.  FP64."""
    per_col = photons / grid.ncol
    norm = 1.0 / (per_col * W_ONE)
    out = {}
    ls = np.ones(grid.nz) if layer_scale is None else np.asarray(layer_scale, dtype=np.float64)
    for n in ("abs_dir", "abs_dif"):
        out[n] = raw[n].astype(np.float64) * norm * ls[:, None, None]
    for n in ("sfc_dir", "sfc_dif", "sfc_abs", "toa_up"):
        out[n] = raw[n].astype(np.float64) * norm * flux_scale
    return out
