"""Learned heating-rate denoiser: binding of include/rt3d_denoise.h and the
encoder-decoder built from its kernels.

Network (4 resolution levels, 32 base channels, BF16 weights and
activations, FP32 accumulation on the matrix cores):

  x0 [hdir/s, hdif/s, ln(1+20 k_ext dz), ln(1+200 k_abs dz)], padded to 16
     channels for training, 4 for inference (packed first layer)
  e0 = relu(conv3 x0 -> 32)           level 0
  e1 = relu(conv3 pool(e0) -> 64)     level 1
  e2 = relu(conv3 pool(e1) -> 128)    level 2
  b  = relu(conv3 pool(e2) -> 256)    level 3
  d2 = relu(conv3 [up(b), e2] -> 128)
  d1 = relu(conv3 [up(d2), e1] -> 64)
  d0 = relu(conv3 [up(d1), e0] -> 32)
  out = conv1 d0 -> 32 (FP32; channels 0, 1 used)
  prediction = out[:, :2] + (hdir/s, hdif/s)      (residual correction)

s is the mean of the noisy heating over the field (known at inference).
Every step runs in the HIP kernels; PyTorch only allocates memory.
"""
from __future__ import annotations

import ctypes
import dataclasses
import math
from typing import Dict, List, Optional

import numpy as np
import torch

from . import rt3d

CPAD = 16          # input feature channels (4 used)
HEAD = 32          # head output channels (2 used)
NOUT = 2
LEVELS = 4


class _Direct(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("nz", ctypes.c_int32),
                ("dx", ctypes.c_float), ("dy", ctypes.c_float), ("dz", ctypes.c_float),
                ("sun_x", ctypes.c_float), ("sun_y", ctypes.c_float), ("sun_z", ctypes.c_float),
                ("direct_fraction", ctypes.c_float)]


class _Conv(ctypes.Structure):
    _fields_ = [("D", ctypes.c_int32), ("H", ctypes.c_int32), ("W", ctypes.c_int32),
                ("c1", ctypes.c_int32), ("c2", ctypes.c_int32), ("cout", ctypes.c_int32),
                ("ksize", ctypes.c_int32), ("up1", ctypes.c_int32), ("yf_cols", ctypes.c_int32)]


_lib = None


def load():
    global _lib
    if _lib is not None:
        return _lib
    lib = rt3d.load()
    P, I, U = ctypes.c_void_p, ctypes.c_int32, ctypes.c_uint64
    sig = {
        "rt3d_dn_conv3d_fwd": [ctypes.POINTER(_Conv), P, P, P, P, I, P, P, I, P, P],
        "rt3d_dn_conv3d_fwd_head": [ctypes.POINTER(_Conv), P, P, P, P, I, P, P, I, P, P],
        "rt3d_dn_conv3d_fwd_pool": [ctypes.POINTER(_Conv), P, P, P, I, P, P, P],
        "rt3d_dn_flip_weights": [P, P, I, I, I, P],
        "rt3d_dn_conv3d_wgrad": [ctypes.POINTER(_Conv), P, P, P, P, P, P],
        "rt3d_dn_conv3d_wgrad_ws": [ctypes.POINTER(_Conv), P, P, P, P, P, P, ctypes.c_size_t, P],
        "rt3d_dn_relu_bwd": [P, P, P, U, P],
        "rt3d_dn_add": [P, P, P, U, P],
        "rt3d_dn_pool2": [P, P, I, I, I, I, I, P],
        "rt3d_dn_up2": [P, P, I, I, I, I, I, P],
        "rt3d_dn_mse": [P, I, P, P, I, U, P, P, P, P],
        "rt3d_dn_adam": [P, P, P, P, P, U, ctypes.c_float, ctypes.c_float, ctypes.c_float, ctypes.c_float, I, P],
        "rt3d_dn_to_bf16": [P, P, U, P],
        "rt3d_dn_features": [P, P, P, P, ctypes.c_float, ctypes.c_float, U, I, P, P, P, P],
        "rt3d_dn_direct_feature": [ctypes.POINTER(_Direct), P, P, P, P, P, P],
        "rt3d_dn_unfeature": [P, ctypes.c_float, U, P, P, P],
        "rt3d_dn_field_scale": [P, P, U, P, P],
        "rt3d_dn_residual_unfeature": [P, I, P, P, ctypes.c_float, U, P, P, P],
    }
    for name, args in sig.items():
        f = getattr(lib, name)
        f.argtypes = args
        f.restype = ctypes.c_int
    lib.rt3d_dn_last_error.restype = ctypes.c_char_p
    lib.rt3d_dn_wgrad_workspace_size.argtypes = [ctypes.POINTER(_Conv)]
    lib.rt3d_dn_wgrad_workspace_size.restype = ctypes.c_size_t
    _lib = lib
    return lib


EXPORTS = ("rt3d_dn_last_error", "rt3d_dn_conv3d_fwd", "rt3d_dn_conv3d_fwd_head", "rt3d_dn_flip_weights", "rt3d_dn_conv3d_wgrad",
           "rt3d_dn_conv3d_wgrad_ws", "rt3d_dn_wgrad_workspace_size",
           "rt3d_dn_relu_bwd", "rt3d_dn_add", "rt3d_dn_pool2", "rt3d_dn_up2", "rt3d_dn_mse", "rt3d_dn_adam",
           "rt3d_dn_to_bf16", "rt3d_dn_features", "rt3d_dn_unfeature")


def _p(t: Optional[torch.Tensor]):
    return ctypes.c_void_p(0 if t is None else t.data_ptr())


def _s():
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _check(st, what):
    if st != 0:
        detail = load().rt3d_dn_last_error().decode() if st == rt3d.EDEVICE else ""
        raise rt3d.Rt3dError(st, what, detail)


def bf16_empty(*shape, device="cuda"):
    """BF16 storage as torch.bfloat16 (the kernels read the raw bits)."""
    return torch.empty(*shape, dtype=torch.bfloat16, device=device)


# ---------------------------------------------------------------------------
# Kernel wrappers
# ---------------------------------------------------------------------------

def conv_fwd(x1, x2, w, bias, relu, cout, ksize, y1=None, y2=None, o1=None, yf=None, up1=False, yf_cols=0):
    """One convolution; with up1, x1 is at half resolution and read
    nearest-upsampled (the output grid is twice x1's); yf (FP32) keeps the
    first yf_cols channels (0: all)."""
    D, H, W, c1 = x1.shape
    if up1:
        D, H, W = 2 * D, 2 * H, 2 * W
    c2 = 0 if x2 is None else x2.shape[3]
    if x2 is not None and tuple(x2.shape[:3]) != (D, H, W):
        raise ValueError("x2 must be on the output grid")
    o1 = cout if o1 is None else o1
    if yf is not None and yf.shape[-1] != (yf_cols or cout):
        raise ValueError("yf must have yf_cols channels")
    c = _Conv(D, H, W, c1, c2, cout, ksize, 1 if up1 else 0, int(yf_cols))
    _check(load().rt3d_dn_conv3d_fwd(ctypes.byref(c), _p(x1), _p(x2), _p(w), _p(bias), int(relu), _p(y1), _p(y2),
                                     int(o1), _p(yf), _s()), "rt3d_dn_conv3d_fwd")


def conv_fwd_head(x1, x2, w, bias, relu, hw, hb, out, up1=False):
    """A 3x3x3 convolution to 32 channels followed by the 1x1x1 head hw
    [32][32] in one launch; out (FP32 [D][H][W][hcols]) receives the head's
    first hcols channels, the 32-channel activation is not stored."""
    D, H, W, c1 = x1.shape
    if up1:
        D, H, W = 2 * D, 2 * H, 2 * W
    c2 = 0 if x2 is None else x2.shape[3]
    if x2 is not None and tuple(x2.shape[:3]) != (D, H, W):
        raise ValueError("x2 must be on the output grid")
    if tuple(out.shape[:3]) != (D, H, W) or tuple(hw.shape[:1]) != (32,) or hw.numel() != 32 * 32:
        raise ValueError("out must be on the output grid and hw [32][32]")
    c = _Conv(D, H, W, c1, c2, 32, 3, 1 if up1 else 0, 0)
    _check(load().rt3d_dn_conv3d_fwd_head(ctypes.byref(c), _p(x1), _p(x2), _p(w), _p(bias), int(relu), _p(hw),
                                          _p(hb), int(out.shape[-1]), _p(out), _s()), "rt3d_dn_conv3d_fwd_head")


def conv_fwd_pool(x1, w, bias, relu, y, ypool):
    """The packed first layer and the 2x2x2 average pooling of its output in
    one launch: y [D][H][W][32] and ypool [D/2][H/2][W/2][32].  Four inputs:
    x1 BF16 [D][H][W][4], w [32][27][4], bitwise conv_fwd followed by pool2;
    five inputs (the direct-beam feature): x1 [D][H][W][8] (channels 5-7
    zero), w the 16-channel weights [32][27][16]."""
    D, H, W, cx = x1.shape
    if cx not in (4, 8) or tuple(y.shape) != (D, H, W, 32) or tuple(ypool.shape) != (D // 2, H // 2, W // 2, 32):
        raise ValueError("conv_fwd_pool: x1 [D][H][W][4 or 8], y [D][H][W][32], ypool [D/2][H/2][W/2][32]")
    c = _Conv(D, H, W, 4 if cx == 4 else 5, 0, 32, 3, 0, 0)
    _check(load().rt3d_dn_conv3d_fwd_pool(ctypes.byref(c), _p(x1), _p(w), _p(bias), int(relu), _p(y), _p(ypool),
                                          _s()), "rt3d_dn_conv3d_fwd_pool")


def flip(w, cout, cin, ksize, out):
    _check(load().rt3d_dn_flip_weights(_p(w), _p(out), cout, cin, ksize, _s()), "rt3d_dn_flip_weights")


def wgrad_workspace_size(x1, x2, cout, ksize) -> int:
    D, H, W, c1 = x1.shape
    c2 = 0 if x2 is None else x2.shape[3]
    return int(load().rt3d_dn_wgrad_workspace_size(ctypes.byref(_Conv(D, H, W, c1, c2, cout, ksize))))


def conv_wgrad(x1, x2, dz, cout, ksize, dw, db, workspace=None):
    """Weight (and bias) gradient, added to dw (db).  With a workspace
    (uint8 device tensor of at least wgrad_workspace_size bytes) the sums run
    in a fixed order and the result is bitwise reproducible; without one,
    FP32 atomics."""
    D, H, W, c1 = x1.shape
    c2 = 0 if x2 is None else x2.shape[3]
    c = _Conv(D, H, W, c1, c2, cout, ksize)
    if workspace is None:
        _check(load().rt3d_dn_conv3d_wgrad(ctypes.byref(c), _p(x1), _p(x2), _p(dz), _p(dw), _p(db), _s()),
               "rt3d_dn_conv3d_wgrad")
    else:
        _check(load().rt3d_dn_conv3d_wgrad_ws(ctypes.byref(c), _p(x1), _p(x2), _p(dz), _p(dw), _p(db),
                                              _p(workspace), workspace.numel() * workspace.element_size(), _s()),
               "rt3d_dn_conv3d_wgrad_ws")


def relu_bwd(dy, y, out):
    _check(load().rt3d_dn_relu_bwd(_p(dy), _p(y), _p(out), dy.numel(), _s()), "rt3d_dn_relu_bwd")


def add(a, b, out):
    _check(load().rt3d_dn_add(_p(a), _p(b), _p(out), a.numel(), _s()), "rt3d_dn_add")


def pool2(x, backward=False, out=None):
    if not backward:
        D, H, W, C = x.shape
        out = bf16_empty(D // 2, H // 2, W // 2, C) if out is None else out
    else:
        D, H, W, C = out.shape
    _check(load().rt3d_dn_pool2(_p(x), _p(out), D, H, W, C, int(backward), _s()), "rt3d_dn_pool2")
    return out


def up2(x, backward=False, out=None):
    if not backward:
        D, H, W, C = x.shape
        out = bf16_empty(2 * D, 2 * H, 2 * W, C) if out is None else out
    else:
        D, H, W, C = out.shape
    _check(load().rt3d_dn_up2(_p(x), _p(out), D, H, W, C, int(backward), _s()), "rt3d_dn_up2")
    return out


# ---------------------------------------------------------------------------
# Network
# ---------------------------------------------------------------------------

@dataclasses.dataclass
class Layer:
    name: str
    c1: int
    c2: int
    cout: int
    ksize: int
    relu: bool


def architecture(base: int = 32) -> List[Layer]:
    c0, c1, c2, c3 = base, 2 * base, 4 * base, 8 * base
    return [Layer("e0", CPAD, 0, c0, 3, True), Layer("e1", c0, 0, c1, 3, True),
            Layer("e2", c1, 0, c2, 3, True), Layer("b", c2, 0, c3, 3, True),
            Layer("d2", c3, c2, c2, 3, True), Layer("d1", c2, c1, c1, 3, True),
            Layer("d0", c1, c0, c0, 3, True), Layer("head", c0, 0, HEAD, 1, False)]


class Denoiser:
    """Parameters (FP32 masters, BF16 copies, gradients, Adam moments) and the
    forward / backward passes over one field."""

    def __init__(self, base: int = 32, seed: int = 0, device="cuda", n_in: int = 4):
        if n_in not in (4, 5):
            raise ValueError("n_in: 4 inputs, or 5 with the direct-beam feature")
        self.n_in = n_in
        self.layers = architecture(base)
        self.device = device
        g = torch.Generator().manual_seed(seed)
        self.p, self.pb, self.g, self.m1, self.m2 = {}, {}, {}, {}, {}
        self.bias, self.gbias, self.mb1, self.mb2 = {}, {}, {}, {}
        for L in self.layers:
            taps = L.ksize ** 3
            fan_in = taps * (L.c1 + L.c2)
            std = math.sqrt(2.0 / fan_in) if L.name != "head" else 1e-3
            w = torch.randn(L.cout, taps, L.c1 + L.c2, generator=g, dtype=torch.float32) * std
            if L.name == "e0":
                w[:, :, n_in:] = 0.0  # padding channels carry nothing
            if L.name == "head":
                w[NOUT:] = 0.0
            self.p[L.name] = w.to(device).contiguous()
            self.pb[L.name] = self.p[L.name].to(torch.bfloat16)
            self.g[L.name] = torch.zeros_like(self.p[L.name])
            self.m1[L.name] = torch.zeros_like(self.p[L.name])
            self.m2[L.name] = torch.zeros_like(self.p[L.name])
            self.bias[L.name] = torch.zeros(L.cout, dtype=torch.float32, device=device)
            self.gbias[L.name] = torch.zeros_like(self.bias[L.name])
            self.mb1[L.name] = torch.zeros_like(self.bias[L.name])
            self.mb2[L.name] = torch.zeros_like(self.bias[L.name])
        self.step_count = 0
        self.wg_ws = None

    def n_params(self) -> int:
        return sum(v.numel() for v in self.p.values()) + sum(v.numel() for v in self.bias.values())

    def state(self) -> Dict[str, torch.Tensor]:
        return {**{f"w_{k}": v for k, v in self.p.items()}, **{f"b_{k}": v for k, v in self.bias.items()}}

    def load_state(self, st: Dict[str, torch.Tensor]):
        for k in self.p:
            self.p[k].copy_(st[f"w_{k}"])
            self.pb[k].copy_(self.p[k].to(torch.bfloat16))
            self.bias[k].copy_(st[f"b_{k}"])

    # -- forward ------------------------------------------------------------
    def _conv(self, name, x1, x2=None, yf=None, up1=False, yf_cols=0):
        L = next(l for l in self.layers if l.name == name)
        D, H, W, _ = x1.shape
        if up1:
            D, H, W = 2 * D, 2 * H, 2 * W
        y = None if yf is not None else bf16_empty(D, H, W, L.cout)
        conv_fwd(x1, x2, self.pb[name], self.bias[name], L.relu, L.cout, L.ksize, y1=y, yf=yf, up1=up1,
                 yf_cols=yf_cols)
        return y

    def forward(self, feat: torch.Tensor, keep: bool = False) -> torch.Tensor:
        """feat: BF16 [D][H][W][16], or for inference [D][H][W][4] (and
        [D][H][W][8] with the direct-beam input; the first layer then runs
        packed: three x-taps per MFMA K-chunk); returns the
        FP32 head output [D][H][W][32] with keep (training) or its NOUT used
        channels [D][H][W][2]."""
        D, H, W, cf = feat.shape
        if D % 8 or H % 8 or W % 8:
            raise ValueError("grid dimensions must be multiples of 8 (three pooling levels)")
        if cf in (4, 8) and keep:
            raise ValueError("training needs the 16-channel features")
        if cf == 8 and self.n_in != 5:
            raise ValueError("8-channel features carry the direct-beam input (n_in 5)")
        a = {"x0": feat}
        if cf in (4, 8):
            # the packed first layer and its pooling in one launch (4 inputs,
            # or 5 with the direct-beam feature in 8 channels)
            L = self.layers[0]
            a["e0"] = bf16_empty(D, H, W, L.cout)
            a["p0"] = bf16_empty(D // 2, H // 2, W // 2, L.cout)
            w0 = self.pb["e0"][:, :, :4].contiguous() if cf == 4 else self.pb["e0"]
            conv_fwd_pool(feat, w0, self.bias["e0"], L.relu, a["e0"], a["p0"])
        else:
            a["e0"] = self._conv("e0", feat)
            a["p0"] = pool2(a["e0"])
        a["e1"] = self._conv("e1", a["p0"])
        a["p1"] = pool2(a["e1"])
        a["e2"] = self._conv("e2", a["p1"])
        a["p2"] = pool2(a["e2"])
        a["b"] = self._conv("b", a["p2"])
        if keep:
            # the weight gradients read the upsampled inputs: materialise them
            a["u2"] = up2(a["b"])
            a["d2"] = self._conv("d2", a["u2"], a["e2"])
            a["u1"] = up2(a["d2"])
            a["d1"] = self._conv("d1", a["u1"], a["e1"])
            a["u0"] = up2(a["d1"])
            a["d0"] = self._conv("d0", a["u0"], a["e0"])
        else:
            # inference: the convolutions read the coarser level upsampled
            a["d2"] = self._conv("d2", a["b"], a["e2"], up1=True)
            a["d1"] = self._conv("d1", a["d2"], a["e1"], up1=True)
            # the last convolution and the head in one launch (the 32-channel
            # activation is never stored); only the NOUT used channels
            out = torch.empty(D, H, W, NOUT, dtype=torch.float32, device=feat.device)
            L = next(l for l in self.layers if l.name == "d0")
            conv_fwd_head(a["d1"], a["e0"], self.pb["d0"], self.bias["d0"], L.relu, self.pb["head"],
                          self.bias["head"], out, up1=True)
            return out
        # training needs every head channel (its gradient)
        out = torch.empty(D, H, W, HEAD, dtype=torch.float32, device=feat.device)
        self._conv("head", a["d0"], yf=out, yf_cols=HEAD)
        if keep:
            self.acts = a
        return out

    # -- backward -----------------------------------------------------------
    def _data_grad(self, name, dz, out1, out2=None):
        L = next(l for l in self.layers if l.name == name)
        cin = L.c1 + L.c2
        wt = bf16_empty(cin, L.ksize ** 3, L.cout)
        flip(self.pb[name], L.cout, cin, L.ksize, wt)
        conv_fwd(dz, None, wt, None, False, cin, L.ksize, y1=out1, y2=out2, o1=L.c1)

    def _wgrad(self, name, x1, x2, dz):
        """Deterministic weight gradient (fixed-order sums in a workspace that
        grows to the largest layer's need)."""
        L = next(l for l in self.layers if l.name == name)
        need = wgrad_workspace_size(x1, x2, L.cout, L.ksize)
        if self.wg_ws is None or self.wg_ws.numel() < need:
            self.wg_ws = torch.empty(need, dtype=torch.uint8, device=x1.device)
        conv_wgrad(x1, x2, dz, L.cout, L.ksize, self.g[name], self.gbias[name], workspace=self.wg_ws)

    def backward(self, dout: torch.Tensor):
        """dout: BF16 [D][H][W][32] gradient at the head output.  Fills the
        FP32 gradients (cleared first)."""
        a = self.acts
        for k in self.g:
            self.g[k].zero_()
            self.gbias[k].zero_()
        like = lambda t: torch.empty_like(t)
        self._wgrad("head", a["d0"], None, dout)
        dd0 = like(a["d0"])
        self._data_grad("head", dout, dd0)
        relu_bwd(dd0, a["d0"], dd0)
        self._wgrad("d0", a["u0"], a["e0"], dd0)
        du0, de0 = like(a["u0"]), like(a["e0"])
        self._data_grad("d0", dd0, du0, de0)
        dd1 = up2(du0, backward=True, out=like(a["d1"]))
        relu_bwd(dd1, a["d1"], dd1)
        self._wgrad("d1", a["u1"], a["e1"], dd1)
        du1, de1 = like(a["u1"]), like(a["e1"])
        self._data_grad("d1", dd1, du1, de1)
        dd2 = up2(du1, backward=True, out=like(a["d2"]))
        relu_bwd(dd2, a["d2"], dd2)
        self._wgrad("d2", a["u2"], a["e2"], dd2)
        du2, de2 = like(a["u2"]), like(a["e2"])
        self._data_grad("d2", dd2, du2, de2)
        db_ = up2(du2, backward=True, out=like(a["b"]))
        relu_bwd(db_, a["b"], db_)
        self._wgrad("b", a["p2"], None, db_)
        dp2 = like(a["p2"])
        self._data_grad("b", db_, dp2)
        t = pool2(dp2, backward=True, out=like(a["e2"]))
        add(de2, t, de2)
        relu_bwd(de2, a["e2"], de2)
        self._wgrad("e2", a["p1"], None, de2)
        dp1 = like(a["p1"])
        self._data_grad("e2", de2, dp1)
        t = pool2(dp1, backward=True, out=like(a["e1"]))
        add(de1, t, de1)
        relu_bwd(de1, a["e1"], de1)
        self._wgrad("e1", a["p0"], None, de1)
        dp0 = like(a["p0"])
        self._data_grad("e1", de1, dp0)
        t = pool2(dp0, backward=True, out=like(a["e0"]))
        add(de0, t, de0)
        relu_bwd(de0, a["e0"], de0)
        self._wgrad("e0", a["x0"], None, de0)
        del self.acts

    def adam(self, lr: float, b1=0.9, b2=0.999, eps=1e-8):
        self.step_count += 1
        lib = load()
        for k in self.p:
            _check(lib.rt3d_dn_adam(_p(self.p[k]), _p(self.g[k]), _p(self.m1[k]), _p(self.m2[k]), _p(self.pb[k]),
                                    self.p[k].numel(), lr, b1, b2, eps, self.step_count, _s()), "rt3d_dn_adam")
            _check(lib.rt3d_dn_adam(_p(self.bias[k]), _p(self.gbias[k]), _p(self.mb1[k]), _p(self.mb2[k]), None,
                                    self.bias[k].numel(), lr, b1, b2, eps, self.step_count, _s()), "rt3d_dn_adam")


# ---------------------------------------------------------------------------
# Data transform, loss, training step and inference
# ---------------------------------------------------------------------------

def features(hdir: torch.Tensor, hdif: torch.Tensor, k_ext: torch.Tensor, k_abs: torch.Tensor, dz: float,
             scale: float, cpad: int = CPAD, direct: Optional[torch.Tensor] = None):
    """BF16 features [D][H][W][cpad] (4 used, 5 with the direct-beam feature;
    cpad 16 for training, 4 for the packed first layer of inference) and
    FP32 residual base [D][H][W][2]."""
    D, H, W = hdir.shape
    feat = bf16_empty(D, H, W, cpad)
    base = torch.empty(D, H, W, NOUT, dtype=torch.float32, device=hdir.device)
    _check(load().rt3d_dn_features(_p(hdir), _p(hdif), _p(k_ext), _p(k_abs), float(dz), float(scale), hdir.numel(),
                                   cpad, _p(direct), _p(feat), _p(base), _s()), "rt3d_dn_features")
    return feat, base


def direct_feature(k_ext: torch.Tensor, k_abs: torch.Tensor, grid, sza: float, azimuth: float,
                   direct_fraction: float, layer_scale: torch.Tensor) -> torch.Tensor:
    """rt3d_dn_direct_feature: deterministic direct-beam heating of a gray
    medium (FP32 [nz][ny][nx]), the fifth network input."""
    th, ph = math.radians(sza), math.radians(azimuth)
    d = _Direct(int(grid.nx), int(grid.ny), int(grid.nz), float(grid.dx), float(grid.dy), float(grid.dz),
                -math.sin(th) * math.sin(ph), -math.sin(th) * math.cos(ph), -math.cos(th), float(direct_fraction))
    if layer_scale.dtype != torch.float64 or layer_scale.numel() != grid.nz:
        raise ValueError("layer_scale: FP64 [nz]")
    out = torch.empty_like(k_ext)
    work = torch.empty(2, grid.ny, grid.nx, dtype=torch.float32, device=k_ext.device)
    _check(load().rt3d_dn_direct_feature(ctypes.byref(d), _p(k_ext), _p(k_abs), _p(layer_scale), _p(out), _p(work),
                                         _s()), "rt3d_dn_direct_feature")
    return out


SCALE_WORK = 2049  # RT3D_DN_SCALE_WORK


def field_scale(hdir: torch.Tensor, hdif: torch.Tensor) -> float:
    """(mean hdir + mean hdif) / 2 (1 if not positive), reduced on the device
    in FP64 in a fixed order (rt3d_dn_field_scale); returned to the host."""
    if hdir.dtype != torch.float32 or hdif.dtype != torch.float32 or hdir.shape != hdif.shape:
        raise ValueError("field_scale: two FP32 fields of one shape")
    work = torch.empty(SCALE_WORK, dtype=torch.float64, device=hdir.device)
    _check(load().rt3d_dn_field_scale(_p(hdir.contiguous()), _p(hdif.contiguous()), hdir.numel(), _p(work), _s()),
           "rt3d_dn_field_scale")
    return float(work[0].item())


def mse(out: torch.Tensor, base: torch.Tensor, target: Optional[torch.Tensor], want_grad: bool):
    nvox = base.shape[0] * base.shape[1] * base.shape[2]
    pred = torch.empty_like(base)
    dout = bf16_empty(*out.shape) if want_grad else None
    loss = torch.zeros(1, dtype=torch.float64, device=out.device) if target is not None else None
    _check(load().rt3d_dn_mse(_p(out), out.shape[-1], _p(base), _p(target), NOUT, nvox, _p(pred), _p(dout),
                              _p(loss), _s()),
           "rt3d_dn_mse")
    return pred, dout, (None if loss is None else loss / (nvox * NOUT))


def train_step(net: Denoiser, feat, base, target, lr: float) -> torch.Tensor:
    out = net.forward(feat, keep=True)
    _, dout, loss = mse(out, base, target, want_grad=True)
    net.backward(dout)
    net.adam(lr)
    return loss


def denoise(net: Denoiser, hdir: torch.Tensor, hdif: torch.Tensor, k_ext: torch.Tensor, k_abs: torch.Tensor,
            dz: float, direct: Optional[dict] = None):
    """Inference: denoised (hdir, hdif), same units as the inputs.  A network
    with the direct-beam input needs direct = the keyword arguments of
    direct_feature beyond k_ext, k_abs (grid, sza, azimuth, direct_fraction,
    layer_scale); the feature is computed here."""
    s = field_scale(hdir, hdif)
    D, H, W = hdir.shape
    dfield = None
    if net.n_in == 5:
        if direct is None:
            raise ValueError("this network takes the direct-beam feature: pass direct=")
        dfield = direct_feature(k_ext, k_abs, **direct)
    cpad = 4 if dfield is None else 8  # packed first layer: 4 inputs, or 5 in 8 channels
    feat = bf16_empty(D, H, W, cpad)
    # the residual base is not stored: the output pass forms it again
    _check(load().rt3d_dn_features(_p(hdir), _p(hdif), _p(k_ext), _p(k_abs), float(dz), float(s), hdir.numel(), cpad,
                                   _p(dfield), _p(feat), None, _s()), "rt3d_dn_features")
    out = net.forward(feat)
    od, of = torch.empty_like(hdir), torch.empty_like(hdif)
    _check(load().rt3d_dn_residual_unfeature(_p(out), out.shape[-1], _p(hdir), _p(hdif), float(s), hdir.numel(),
                                             _p(od), _p(of), _s()), "rt3d_dn_residual_unfeature")
    return od, of
