"""CPU-side checks of the HIP library boundary: the shared library loads,
exports every entry point include/rt3d.h declares, and its host-only entry
points (options, workspace size, argument checks) behave as documented.
No compute call is made here."""
import ctypes
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "rt3d.h")
PKG = os.path.join(ROOT, "paper_2208_05247_amd")
# every public header and the library that implements it
HEADER_LIBS = {"rt3d.h": "librt3d.so", "rt3d_denoise.h": "librt3d.so", "rt3d_probe.h": "librt3d_probe.so"}


def declared_functions(header=HEADER):
    src = open(header).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(rt3d_[a-z0-9_]+)\s*\(", src)))


@pytest.fixture(scope="module")
def lib():
    from paper_2208_05247_amd import rt3d
    if not os.path.exists(rt3d.LIB_PATH):
        pytest.fail("librt3d.so is not built (run __graft_entry__.build())")
    return rt3d.load()


def test_exports_match_header(lib):
    from paper_2208_05247_amd import rt3d
    decl = declared_functions()
    assert decl, "no declarations found"
    out = subprocess.check_output(["nm", "-D", "--defined-only", rt3d.LIB_PATH], text=True)
    exported = set(re.findall(r"\bT (rt3d_[a-z0-9_]+)", out))
    missing = [f for f in decl if f not in exported]
    assert not missing, missing
    for f in decl:
        assert hasattr(lib, f)
    assert set(rt3d.EXPORTS) <= set(decl)


@pytest.mark.parametrize("header", sorted(HEADER_LIBS))
def test_every_header_is_exported_by_its_library(header):
    """Each public header's functions are defined by its library, and the
    measurement probe is not part of the tracer library."""
    inc = os.path.join(ROOT, "include")
    assert sorted(os.listdir(inc)) == sorted(HEADER_LIBS)
    so = os.path.join(PKG, HEADER_LIBS[header])
    if not os.path.exists(so):
        pytest.fail(f"{so} is not built (run __graft_entry__.build())")
    decl = declared_functions(os.path.join(inc, header))
    assert decl
    out = subprocess.check_output(["nm", "-D", "--defined-only", so], text=True)
    exported = set(re.findall(r"\bT (rt3d_[a-z0-9_]+)", out))
    assert not [f for f in decl if f not in exported]
    tracer = set(re.findall(r"\bT (rt3d_[a-z0-9_]+)",
                            subprocess.check_output(["nm", "-D", "--defined-only",
                                                     os.path.join(PKG, "librt3d.so")], text=True)))
    assert not [f for f in tracer if "probe" in f]


def test_abi_and_strings(lib):
    assert lib.rt3d_abi_version() == 3
    for s in range(4):
        assert lib.rt3d_status_string(s)
    assert lib.rt3d_status_string(99) == b"unknown status"


def test_default_options(lib):
    from paper_2208_05247_amd import rt3d
    o = rt3d.Options()
    lib.rt3d_default_options(ctypes.byref(o))
    assert abs(o.rr_threshold - 0.5) < 1e-7
    assert o.diffuse_fraction == 0.0 and o.flags == 0 and o.max_iters == 1 << 24
    assert o.photon_offset == 0 and o.grid_blocks == 0


def test_workspace_size_host_only(lib):
    from paper_2208_05247_amd import rt3d
    from paper_2208_05247_amd.synthetic import Grid
    g = Grid(256, 256, 128, 50.0, 50.0, 25.0)
    o = rt3d.options(brick=(8, 8, 8))
    n = rt3d.workspace_size(g, o)
    # control block, schedule tables (pass and remainder prefix sums, column
    # offsets), majorants, packed cells
    assert n == 256 + 256 + 32 * 32 * 16 * 4 + 256 * 256 * 128 * 16
    nb = rt3d.workspace_size_batched(g, 112, o)
    meta = (8 * (3 * 112 + 2) + 255) // 256 * 256
    # + gas tables, per-level cloud maxima, cloud-cell mask (512 bits per brick)
    assert nb == (256 + meta + 112 * 32 * 32 * 16 * 4 + 256 * 256 * 128 * 16 + 112 * 128 * 8 + 128 * 32 * 32 * 4
                  + 32 * 32 * 16 * 64)
    assert lib.rt3d_workspace_size_batched(ctypes.byref(rt3d.grid_struct(g)), 0, ctypes.byref(o)) == 0
    assert lib.rt3d_workspace_size_batched(ctypes.byref(rt3d.grid_struct(g)), 257, ctypes.byref(o)) == 0
    bad = rt3d.options(brick=(3, 8, 8))
    with pytest.raises(rt3d.Rt3dError):
        rt3d.workspace_size(g, bad)
    assert lib.rt3d_workspace_size(None, None) == 0
    z = rt3d.Grid(0, 4, 4, 1.0, 1.0, 1.0)
    assert lib.rt3d_workspace_size(ctypes.byref(z), None) == 0


def test_einval_before_any_launch(lib):
    """Argument errors are reported from host checks (null pointers, bad
    sizes); nothing reaches the device."""
    from paper_2208_05247_amd import rt3d
    g = rt3d.Grid(8, 8, 8, 10.0, 10.0, 10.0)
    props = rt3d.OpticalProps(0, 0, 0, 0)
    t = rt3d.TalliesStruct(*([0] * 8))
    o = rt3d.options(brick=(4, 4, 4))
    st = lib.rt3d_trace(ctypes.byref(g), ctypes.byref(props), None, 30.0, 0.0, 100, 1,
                        ctypes.byref(o), ctypes.byref(t), None, 0, None)
    assert st == rt3d.EINVAL
    st = lib.rt3d_trace(None, None, None, 30.0, 0.0, 100, 1, None, None, None, 0, None)
    assert st == rt3d.EINVAL
    assert lib.rt3d_majorant_build(ctypes.byref(g), None, 4, 4, 4, None, None) == rt3d.EINVAL
    assert lib.rt3d_finalize(None, None, 1, None, 1.0, None, None, None, None, None, None, None) == rt3d.EINVAL
    assert lib.rt3d_philox4x32_10(None, 1, None, 4, None) == rt3d.EINVAL
    ms = ctypes.c_float()
    assert lib.rt3d_last_trace_ms(ctypes.byref(ms)) == rt3d.EINVAL
    assert lib.rt3d_sobol_entry(0, 4, 0, 1, None, None) == rt3d.EINVAL
    ts = lib.rt3d_two_stream
    assert ts(0, 5, None, None, None, None, 0.5, None, None, None, None, 0, None, None, None) == rt3d.EINVAL
    fake = ctypes.c_void_p(256)  # never dereferenced: the host checks reject first
    args = [fake] * 4
    assert ts(2, 5, *args, 0.0, None, fake, fake, fake, 0, None, None, None) == rt3d.EINVAL   # mu0 = 0
    assert ts(2, 5, *args, 1.5, None, fake, fake, fake, 0, None, None, None) == rt3d.EINVAL   # mu0 > 1
    assert ts(2, 5, *args, 0.5, None, fake, fake, fake, 6, None, None, None) == rt3d.EINVAL   # level > nlay
    assert ts(2, 5, *args, 0.5, None, None, fake, fake, 0, None, None, None) == rt3d.EINVAL   # no output


def test_probe_argument_checks():
    """The memory probe's host checks reject bad arguments before any launch."""
    from paper_2208_05247_amd import probe
    lib = probe.load()
    fake = ctypes.c_void_p(256)  # never dereferenced: the host checks reject first
    ap = lib.rt3d_probe_gathers
    assert ap(None, 16, fake, 16, 8, 1, 11, 0, 4, 1, fake, 4096, None) == 1            # no records
    assert ap(fake, 0, fake, 16, 8, 1, 11, 0, 4, 1, fake, 4096, None) == 1             # empty
    assert ap(fake, 1 << 32, fake, 16, 8, 1, 11, 0, 4, 1, fake, 4096, None) == 1       # too many records
    assert ap(fake, 16, fake, 16, 8, 1, 17, 0, 4, 1, fake, 4096, None) == 1            # > 16 of 16
    assert ap(ctypes.c_void_p(264), 16, fake, 16, 8, 1, 11, 0, 4, 1, fake, 4096, None) == 1  # misaligned
    assert ap(fake, 16, fake, 16, 8, 1, 11, 0, 4, 1, fake, 4095, None) == 1            # short sink
    assert ap(fake, 16, fake, 16, 8, 0, 11, 0, 4, 1, fake, 4096, None) == 1            # no chain
    assert ap(fake, 16, fake, 16, 8, 5, 11, 0, 4, 1, fake, 4096, None) == 1            # too many chains
    assert ap(fake, 16, fake, 16, 8, 1, 11, 2, 4, 1, fake, 4096, None) == 1            # unknown flag
    assert ap(ctypes.c_void_p(272), 16, fake, 16, 8, 1, 11, 1, 4, 1, fake, 4096, None) == 1  # pair: 128-B align
    assert ap(fake, 12, fake, 16, 8, 1, 11, 1, 4, 1, fake, 4096, None) == 1            # pair: n % 8
    assert lib.rt3d_probe_lanes(5) == 5 * 1024


def test_small_photon_pools_rejected(lib):
    """A refill hands out up to 64 photon ids from one grab of the work
    queue, so pools of 1..63 ids would hand out ids of the next grab (photons
    traced twice): they are rejected on the host, before any launch."""
    from paper_2208_05247_amd import rt3d
    g = rt3d.Grid(8, 8, 8, 10.0, 10.0, 10.0)
    fake = ctypes.c_void_p(256)  # never dereferenced: the host checks reject first
    props = rt3d.OpticalProps(256, 256, 256, 256)
    t = rt3d.TalliesStruct(*([256] * 8))
    med = rt3d.BatchedMedium(256, 256, 256, 256, 256, None)
    counts = (ctypes.c_uint64 * 2)(100, 50)
    for pool in (1, 32, 63, -1):
        o = rt3d.options(brick=(4, 4, 4), pool_photons=pool)
        ws = rt3d.workspace_size(g, o)
        assert lib.rt3d_trace(ctypes.byref(g), ctypes.byref(props), fake, 30.0, 0.0, 100, 1, ctypes.byref(o),
                              ctypes.byref(t), fake, ws, None) == rt3d.EINVAL, pool
        wsb = rt3d.workspace_size_batched(g, 2, o)
        assert lib.rt3d_trace_batched(ctypes.byref(g), 2, ctypes.byref(med), counts, fake, 30.0, 0.0, 1,
                                      ctypes.byref(o), ctypes.byref(t), fake, wsb, None) == rt3d.EINVAL, pool


def test_product_path_has_no_fallback():
    """The binding imports nothing from the oracle and refuses to run
    without the HIP library."""
    src = open(os.path.join(ROOT, "paper_2208_05247_amd", "rt3d.py")).read()
    assert "oracle" not in src.replace("no CPU fallback", "")
    from paper_2208_05247_amd import rt3d
    with pytest.raises(RuntimeError):
        saved = rt3d._lib
        rt3d._lib = None
        try:
            rt3d.load(os.path.join(ROOT, "does_not_exist.so"))
        finally:
            rt3d._lib = saved


def test_denoiser_wgrad_workspace_checks(lib):
    """The deterministic weight gradient's workspace size is a host
    computation (0 for bad shapes) and a too small or missing workspace is
    rejected before any launch."""
    from paper_2208_05247_amd import denoise as dn
    dn.load()
    good = dn._Conv(8, 8, 32, 32, 16, 64, 3, 0, 0)
    n = lib.rt3d_dn_wgrad_workspace_size(ctypes.byref(good))
    # per-chunk partials of 64 x 27 x 48 weights, then 64 bias partials per block
    assert n >= 64 * 27 * 48 * 4 and n % 4 == 0
    for bad in (dn._Conv(8, 8, 32, 8, 0, 64, 3, 0, 0), dn._Conv(8, 8, 32, 32, 0, 40, 3, 0, 0),
                dn._Conv(8, 8, 32, 32, 0, 64, 2, 0, 0), dn._Conv(8, 8, 32, 32, 0, 64, 3, 1, 0)):
        assert lib.rt3d_dn_wgrad_workspace_size(ctypes.byref(bad)) == 0
    fake = ctypes.c_void_p(256)  # never dereferenced: the host checks reject first
    f = lib.rt3d_dn_conv3d_wgrad_ws
    assert f(ctypes.byref(good), fake, fake, fake, fake, None, fake, n - 1, None) == 1
    assert f(ctypes.byref(good), fake, fake, fake, fake, None, None, n, None) == 1
    assert f(ctypes.byref(good), fake, None, fake, fake, None, fake, n, None) == 1   # c2 > 0 needs x2


def test_fused_head_argument_checks(lib):
    """The fused convolution + head entry point rejects unsupported shapes and
    missing pointers on the host, before any launch."""
    from paper_2208_05247_amd import denoise as dn
    dn.load()
    fake = ctypes.c_void_p(256)  # never dereferenced: the host checks reject first
    f = lib.rt3d_dn_conv3d_fwd_head
    good = dn._Conv(8, 8, 32, 32, 16, 32, 3, 0, 0)
    assert f(ctypes.byref(good), fake, fake, fake, None, 1, None, None, 2, fake, None) == rt3d_einval()  # no head
    assert f(ctypes.byref(good), fake, fake, fake, None, 1, fake, None, 2, None, None) == rt3d_einval()  # no output
    assert f(ctypes.byref(good), fake, None, fake, None, 1, fake, None, 2, fake, None) == rt3d_einval()  # c2 needs x2
    for hcols in (0, 33):
        assert f(ctypes.byref(good), fake, fake, fake, None, 1, fake, None, hcols, fake, None) == rt3d_einval()
    for bad in (dn._Conv(8, 8, 32, 32, 16, 64, 3, 0, 0),   # 64 outputs
                dn._Conv(8, 8, 32, 32, 16, 32, 1, 0, 0),   # 1x1x1
                dn._Conv(8, 8, 32, 4, 0, 32, 3, 0, 0),     # 4-channel first layer
                dn._Conv(7, 8, 32, 32, 16, 32, 3, 1, 0)):  # odd grid with upsampling
        assert f(ctypes.byref(bad), fake, fake, fake, None, 1, fake, None, 2, fake, None) == rt3d_einval()


def rt3d_einval():
    from paper_2208_05247_amd import rt3d
    return rt3d.EINVAL


def test_pool_argument_checks(lib):
    """The forward pooling takes 8-channel groups of 16-byte aligned tensors;
    anything else is rejected on the host, before any launch."""
    from paper_2208_05247_amd import denoise as dn
    dn.load()
    fake = ctypes.c_void_p(256)  # never dereferenced: the host checks reject first
    f = lib.rt3d_dn_pool2
    assert f(fake, fake, 4, 4, 4, 12, 0, None) == rt3d_einval()                   # C not a multiple of 8
    assert f(ctypes.c_void_p(264), fake, 4, 4, 4, 16, 0, None) == rt3d_einval()   # misaligned input
    assert f(fake, ctypes.c_void_p(258), 4, 4, 4, 16, 0, None) == rt3d_einval()   # misaligned output
    assert f(fake, fake, 3, 4, 4, 16, 0, None) == rt3d_einval()                   # odd grid
    assert f(None, fake, 4, 4, 4, 16, 0, None) == rt3d_einval()
