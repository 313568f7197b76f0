"""Binding of librt3d_probe.so (include/rt3d_probe.h): the memory-system
measurement the benchmark sets the tracer against.  Argument marshalling
only; the library is separate from the tracer's librt3d.so."""
from __future__ import annotations

import ctypes
import os

import torch

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "librt3d_probe.so")
EXPORTS = ("rt3d_probe_gathers", "rt3d_probe_lanes")
MAX_CHAINS = 4
LINE_PAIR = 0x1
_lib = None


def load(path: str = LIB_PATH):
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"{path} is missing: build it with __graft_entry__.build()")
    lib = ctypes.CDLL(path)
    P = ctypes.c_void_p
    u32, u64 = ctypes.c_uint32, ctypes.c_uint64
    lib.rt3d_probe_gathers.argtypes = [P, u64, P, u64, u32, u32, u32, u32, u32, u64, P, u64, P]
    lib.rt3d_probe_gathers.restype = ctypes.c_int
    lib.rt3d_probe_lanes.argtypes = [u32]
    lib.rt3d_probe_lanes.restype = u64
    _lib = lib
    return lib


def lanes(grid_blocks: int = 0) -> int:
    return int(load().rt3d_probe_lanes(int(grid_blocks)))


def gathers(records: torch.Tensor, tally: torch.Tensor, events: int, chains: int = 1, atomics_per_16: int = 0,
            line_pair: bool = False, grid_blocks: int = 0, seed: int = 1, stream=None) -> torch.Tensor:
    """rt3d_probe_gathers over caller-owned device tensors: `records` with a
    multiple of 16 bytes per record (e.g. float32 [n, 4]), `tally` int64 [m]
    (used as uint64).  Returns the per-lane sink (FP32 device)."""
    if not (isinstance(tally, torch.Tensor) and tally.is_cuda and tally.dtype == torch.int64
            and tally.is_contiguous()):
        raise ValueError("tally must be a contiguous int64 device tensor")
    if not records.is_cuda or not records.is_contiguous() or records.numel() * records.element_size() < 16:
        raise ValueError("records must be a contiguous device tensor of 16-byte records")
    n_rec = records.numel() * records.element_size() // 16
    n = lanes(grid_blocks)
    if n == 0:
        raise RuntimeError("rt3d_probe_lanes: no HIP device")
    sink = torch.empty(n, dtype=torch.float32, device=records.device)
    s = stream if stream is not None else torch.cuda.current_stream()
    st = load().rt3d_probe_gathers(ctypes.c_void_p(records.data_ptr()), n_rec, ctypes.c_void_p(tally.data_ptr()),
                                   tally.numel(), int(events), int(chains), int(atomics_per_16),
                                   LINE_PAIR if line_pair else 0, int(grid_blocks), int(seed),
                                   ctypes.c_void_p(sink.data_ptr()), n, ctypes.c_void_p(s.cuda_stream))
    if st != 0:
        raise RuntimeError(f"rt3d_probe_gathers: status {st}")
    return sink
