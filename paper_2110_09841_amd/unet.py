"""Learned CGLS warm start: a 3-level 3D U-Net on two CGLS iterates.

Architecture (16/32/64 channels, 3x3x3 convolutions, ReLU, 2x2x2 average
pooling, nearest upsampling followed by a convolution, skip concatenation,
1x1x1 head with a residual on the second iterate):

  in(x1, x2) -> c1a 16 -> c1b 16 (skip 1) -> pool -> c2a 32 -> c2b 32 (skip 2)
  -> pool -> c3a 64 -> c3b 64 -> up -> u2 32 | skip 2 -> d2a 32 -> d2b 32
  -> up -> u1 16 | skip 1 -> d1a 16 -> d1b 16 -> head: x0 = x2 + (w.h + b)/s

Every layer runs in the HIP kernels of libcvp.so (BF16 MFMA convolutions with
FP32 accumulation, FP32 master weights, Adam); this module only allocates the
tensors and sequences the calls.  Concatenation is free: the up-convolution
and the skip tensor write the two channel halves of one buffer.
"""
import ctypes
import math

import numpy as np
import torch

from . import _lib

IN_CH = 16          # the two iterates are packed into 16 channels (rest zero)
INPUT_SCALE = 100.0  # attenuation ~0.01/mm -> activations ~1


class NNTensor(ctypes.Structure):
    _fields_ = [("data", ctypes.c_void_p), ("d", ctypes.c_int32), ("h", ctypes.c_int32),
                ("w", ctypes.c_int32), ("channels", ctypes.c_int32), ("stride", ctypes.c_int32)]


_SIGS = {
    "cvp_nn_conv3d": [ctypes.POINTER(NNTensor), ctypes.c_void_p, ctypes.c_void_p, ctypes.POINTER(NNTensor),
                      ctypes.c_int32, ctypes.c_int32, ctypes.c_void_p],
    "cvp_nn_wgrad_workspace": [ctypes.POINTER(NNTensor), ctypes.POINTER(NNTensor), ctypes.POINTER(ctypes.c_int64)],
    "cvp_nn_conv3d_wgrad": [ctypes.POINTER(NNTensor), ctypes.POINTER(NNTensor), ctypes.c_void_p, ctypes.c_void_p,
                            ctypes.c_int64, ctypes.c_void_p],
    "cvp_nn_channel_sum": [ctypes.POINTER(NNTensor), ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64, ctypes.c_void_p],
    "cvp_nn_relu_mask": [ctypes.POINTER(NNTensor), ctypes.POINTER(NNTensor), ctypes.c_void_p],
    "cvp_nn_avgpool2": [ctypes.POINTER(NNTensor), ctypes.POINTER(NNTensor), ctypes.c_void_p],
    "cvp_nn_avgpool2_bwd": [ctypes.POINTER(NNTensor), ctypes.POINTER(NNTensor), ctypes.c_void_p],
    "cvp_nn_upsample2": [ctypes.POINTER(NNTensor), ctypes.POINTER(NNTensor), ctypes.c_void_p],
    "cvp_nn_upsample2_bwd": [ctypes.POINTER(NNTensor), ctypes.POINTER(NNTensor), ctypes.c_void_p],
    "cvp_nn_add": [ctypes.POINTER(NNTensor), ctypes.POINTER(NNTensor), ctypes.POINTER(NNTensor), ctypes.c_void_p],
    "cvp_nn_transpose_weights": [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int32, ctypes.c_int32, ctypes.c_void_p],
    "cvp_nn_pack_input": [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_float, ctypes.POINTER(NNTensor), ctypes.c_void_p],
    "cvp_nn_head": [ctypes.POINTER(NNTensor), ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_float,
                    ctypes.c_void_p, ctypes.c_void_p],
    "cvp_nn_head_bwd": [ctypes.POINTER(NNTensor), ctypes.c_void_p, ctypes.c_void_p, ctypes.c_float,
                        ctypes.POINTER(NNTensor), ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64, ctypes.c_void_p],
    "cvp_nn_mse": [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                   ctypes.c_int64, ctypes.c_void_p],
    "cvp_nn_adam": [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64, ctypes.c_float,
                    ctypes.c_float, ctypes.c_float, ctypes.c_float, ctypes.c_int32, ctypes.c_void_p, ctypes.c_void_p],
}


def lib():
    L = _lib.lib()
    if not getattr(L, "_nn_ready", False):
        for name, args in _SIGS.items():
            f = getattr(L, name)
            f.argtypes = args
            f.restype = ctypes.c_int
        L._nn_ready = True
    return L


def _p(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else ctypes.c_void_p(0)


def _s():
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def desc(t, c0=0, c=None):
    """Descriptor of a channels-last BF16 tensor (D, H, W, C), optionally the
    channel slice [c0, c0 + c)."""
    D, H, W, C = t.shape
    c = C - c0 if c is None else c
    return NNTensor(t.data_ptr() + 2 * c0, D, H, W, c, C)


def _check(st):
    if st != 0:
        raise _lib.CVPError(st, "nn kernel call failed")


def act(shape, ch, device):
    return torch.empty(tuple(shape) + (ch,), dtype=torch.bfloat16, device=device)


class Conv:
    """3x3x3 convolution parameters: FP32 master weights [27][Co][Ci], bias,
    BF16 copies (forward and transposed for backward-data), Adam state."""

    def __init__(self, ci, co, rng, device):
        self.ci, self.co = ci, co
        bound = math.sqrt(6.0 / (27 * ci))          # He-uniform for ReLU
        w = rng.uniform(-bound, bound, size=(27, co, ci)).astype(np.float32)
        self.w = torch.from_numpy(w).to(device)
        self.b = torch.zeros(co, dtype=torch.float32, device=device)
        self.wb = self.w.to(torch.bfloat16)
        self.wt = torch.empty((27, ci, co), dtype=torch.bfloat16, device=device)
        self.gw = torch.zeros_like(self.w)
        self.gb = torch.zeros_like(self.b)
        self.m = [torch.zeros_like(self.w), torch.zeros_like(self.b)]
        self.v = [torch.zeros_like(self.w), torch.zeros_like(self.b)]
        self.refresh()

    def refresh(self):
        _check(lib().cvp_nn_transpose_weights(_p(self.wb), _p(self.wt), self.co, self.ci, _s()))


LAYERS = [("c1a", IN_CH, 16, 1), ("c1b", 16, 16, 1), ("c2a", 16, 32, 2), ("c2b", 32, 32, 2), ("c3a", 32, 64, 4),
          ("c3b", 64, 64, 4), ("u2", 64, 32, 2), ("d2a", 64, 32, 2), ("d2b", 32, 32, 2), ("u1", 32, 16, 1),
          ("d1a", 32, 16, 1), ("d1b", 16, 16, 1)]   # name, Cin, Cout, resolution divisor


def forward_flops(shape, algorithmic=False):
    """Multiply-add count x 2 of one forward pass (the 3x3x3 convolutions):
    as executed (the two input channels padded to IN_CH) or algorithmic
    (two input channels)."""
    n = shape[0] * shape[1] * shape[2]
    return sum(2 * 27 * (2 if (algorithmic and name == "c1a") else ci) * co * n // (s ** 3)
               for name, ci, co, s in LAYERS)


def forward_bound_seconds(shape, peak_flops=2.5e15, peak_bytes=8e12):
    """Lower bound of one forward pass: per convolution the larger of its
    algorithmic MFMA time (BF16 peak) and its HBM time (BF16 input and output
    activations once, weights), summed over the layers."""
    n = shape[0] * shape[1] * shape[2]
    t = 0.0
    for name, ci, co, s in LAYERS:
        v = n // (s ** 3)
        cin = 2 if name == "c1a" else ci
        fl = 2 * 27 * cin * co * v
        by = 2 * v * (cin + co) + 2 * 27 * ci * co
        t += max(fl / peak_flops, by / peak_bytes)
    return t


class UNet:
    def __init__(self, shape, seed=0, device="cuda"):
        D, H, W = shape
        assert D % 4 == 0 and H % 4 == 0 and W % 4 == 0
        self.shape = tuple(shape)
        self.device = device
        rng = np.random.default_rng(seed)
        self.convs = {n: Conv(ci, co, rng, device) for n, ci, co, _ in LAYERS}
        self.hw = torch.from_numpy(rng.uniform(-0.25, 0.25, size=16).astype(np.float32)).to(device)
        self.hb = torch.zeros(1, dtype=torch.float32, device=device)
        self.ghead = torch.zeros(17, dtype=torch.float32, device=device)
        self.mh = torch.zeros(17, dtype=torch.float32, device=device)
        self.vh = torch.zeros(17, dtype=torch.float32, device=device)
        s1 = self.shape
        s2 = tuple(v // 2 for v in s1)
        s3 = tuple(v // 4 for v in s1)
        A = lambda s, c: act(s, c, device)
        self.a = {
            "in": A(s1, IN_CH), "c1a": A(s1, 16), "cat1": A(s1, 32), "p1": A(s2, 16),
            "c2a": A(s2, 32), "cat2": A(s2, 64), "p2": A(s3, 32), "c3a": A(s3, 64), "c3b": A(s3, 64),
            "up2": A(s2, 64), "d2a": A(s2, 32), "d2b": A(s2, 32), "up1": A(s1, 32), "d1a": A(s1, 16),
            "d1b": A(s1, 16),
        }
        # gradient buffers of the same shapes
        self.g = {k: torch.empty_like(v) for k, v in self.a.items()}
        self.gx0 = torch.empty(self.shape, dtype=torch.float32, device=device)
        self.x0 = torch.empty(self.shape, dtype=torch.float32, device=device)
        worst = 0
        L = lib()
        for xi, gi in (("in", "c1a"), ("cat1", "d1a")):
            n = ctypes.c_int64()
            L.cvp_nn_wgrad_workspace(ctypes.byref(desc(self.a[xi])), ctypes.byref(desc(self.a[gi])), ctypes.byref(n))
            worst = max(worst, n.value)
        n = ctypes.c_int64()
        L.cvp_nn_wgrad_workspace(ctypes.byref(desc(self.a["p2"])), ctypes.byref(desc(self.a["c3a"])), ctypes.byref(n))
        worst = max(worst, n.value, 64 * 64 * 27 * 64)
        self.work = torch.empty(worst + 4096, dtype=torch.float32, device=device)
        self.work64 = torch.empty(1024, dtype=torch.float64, device=device)
        self.loss = torch.zeros(1, dtype=torch.float64, device=device)
        self.step_count = 0

    # --------------------------------------------------------------- forward
    def _conv(self, name, x, out, relu=True):
        c = self.convs[name]
        _check(lib().cvp_nn_conv3d(ctypes.byref(x), _p(c.wb), _p(c.b), ctypes.byref(out), int(relu), 0, _s()))

    def forward(self, x1, x2):
        """x0 = x2 + U-Net(x1, x2); x1, x2 FP32 volumes (D, H, W).  Returns the
        network's own output buffer, which the next forward overwrites."""
        a, L = self.a, lib()
        self.x2 = x2
        _check(L.cvp_nn_pack_input(_p(x1), _p(x2), ctypes.c_float(INPUT_SCALE), ctypes.byref(desc(a["in"])), _s()))
        self._conv("c1a", desc(a["in"]), desc(a["c1a"]))
        self._conv("c1b", desc(a["c1a"]), desc(a["cat1"], 16, 16))            # skip 1
        _check(L.cvp_nn_avgpool2(ctypes.byref(desc(a["cat1"], 16, 16)), ctypes.byref(desc(a["p1"])), _s()))
        self._conv("c2a", desc(a["p1"]), desc(a["c2a"]))
        self._conv("c2b", desc(a["c2a"]), desc(a["cat2"], 32, 32))            # skip 2
        _check(L.cvp_nn_avgpool2(ctypes.byref(desc(a["cat2"], 32, 32)), ctypes.byref(desc(a["p2"])), _s()))
        self._conv("c3a", desc(a["p2"]), desc(a["c3a"]))
        self._conv("c3b", desc(a["c3a"]), desc(a["c3b"]))
        _check(L.cvp_nn_upsample2(ctypes.byref(desc(a["c3b"])), ctypes.byref(desc(a["up2"])), _s()))
        self._conv("u2", desc(a["up2"]), desc(a["cat2"], 0, 32))
        self._conv("d2a", desc(a["cat2"]), desc(a["d2a"]))
        self._conv("d2b", desc(a["d2a"]), desc(a["d2b"]))
        _check(L.cvp_nn_upsample2(ctypes.byref(desc(a["d2b"])), ctypes.byref(desc(a["up1"])), _s()))
        self._conv("u1", desc(a["up1"]), desc(a["cat1"], 0, 16))
        self._conv("d1a", desc(a["cat1"]), desc(a["d1a"]))
        self._conv("d1b", desc(a["d1a"]), desc(a["d1b"]))
        _check(L.cvp_nn_head(ctypes.byref(desc(a["d1b"])), _p(self.hw), _p(self.hb), _p(x2),
                             ctypes.c_float(INPUT_SCALE), _p(self.x0), _s()))
        return self.x0

    # -------------------------------------------------------------- backward
    def _conv_bwd(self, name, x_desc, y_desc, gy_desc, gx_desc):
        """Given dL/dy (post-ReLU, in gy), fill the parameter gradients and,
        if gx_desc is not None, dL/dx."""
        c, L = self.convs[name], lib()
        _check(L.cvp_nn_relu_mask(ctypes.byref(gy_desc), ctypes.byref(y_desc), _s()))
        _check(L.cvp_nn_conv3d_wgrad(ctypes.byref(x_desc), ctypes.byref(gy_desc), _p(c.gw), _p(self.work),
                                     self.work.numel(), _s()))
        _check(L.cvp_nn_channel_sum(ctypes.byref(gy_desc), _p(c.gb), _p(self.work), self.work.numel(), _s()))
        if gx_desc is not None:
            _check(L.cvp_nn_conv3d(ctypes.byref(gy_desc), _p(c.wt), None, ctypes.byref(gx_desc), 0, 1, _s()))

    def backward(self, gx0):
        """Back-propagate dL/dx0 (FP32 volume) to all parameters."""
        a, g, L = self.a, self.g, lib()
        _check(L.cvp_nn_head_bwd(ctypes.byref(desc(a["d1b"])), _p(self.hw), _p(gx0), ctypes.c_float(INPUT_SCALE),
                                 ctypes.byref(desc(g["d1b"])), _p(self.ghead), _p(self.work), self.work.numel(), _s()))
        self._conv_bwd("d1b", desc(a["d1a"]), desc(a["d1b"]), desc(g["d1b"]), desc(g["d1a"]))
        self._conv_bwd("d1a", desc(a["cat1"]), desc(a["d1a"]), desc(g["d1a"]), desc(g["cat1"]))
        # cat1 = [u1 out | skip 1]
        self._conv_bwd("u1", desc(a["up1"]), desc(a["cat1"], 0, 16), desc(g["cat1"], 0, 16), desc(g["up1"]))
        _check(L.cvp_nn_upsample2_bwd(ctypes.byref(desc(g["up1"])), ctypes.byref(desc(g["d2b"])), _s()))
        self._conv_bwd("d2b", desc(a["d2a"]), desc(a["d2b"]), desc(g["d2b"]), desc(g["d2a"]))
        self._conv_bwd("d2a", desc(a["cat2"]), desc(a["d2a"]), desc(g["d2a"]), desc(g["cat2"]))
        self._conv_bwd("u2", desc(a["up2"]), desc(a["cat2"], 0, 32), desc(g["cat2"], 0, 32), desc(g["up2"]))
        _check(L.cvp_nn_upsample2_bwd(ctypes.byref(desc(g["up2"])), ctypes.byref(desc(g["c3b"])), _s()))
        self._conv_bwd("c3b", desc(a["c3a"]), desc(a["c3b"]), desc(g["c3b"]), desc(g["c3a"]))
        self._conv_bwd("c3a", desc(a["p2"]), desc(a["c3a"]), desc(g["c3a"]), desc(g["p2"]))
        # skip 2 receives the concat slice plus the pooled path
        _check(L.cvp_nn_avgpool2_bwd(ctypes.byref(desc(g["p2"])), ctypes.byref(desc(g["up2"], 0, 32)), _s()))
        _check(L.cvp_nn_add(ctypes.byref(desc(g["cat2"], 32, 32)), ctypes.byref(desc(g["up2"], 0, 32)),
                            ctypes.byref(desc(g["cat2"], 32, 32)), _s()))
        self._conv_bwd("c2b", desc(a["c2a"]), desc(a["cat2"], 32, 32), desc(g["cat2"], 32, 32), desc(g["c2a"]))
        self._conv_bwd("c2a", desc(a["p1"]), desc(a["c2a"]), desc(g["c2a"]), desc(g["p1"]))
        _check(L.cvp_nn_avgpool2_bwd(ctypes.byref(desc(g["p1"])), ctypes.byref(desc(g["up1"], 0, 16)), _s()))
        _check(L.cvp_nn_add(ctypes.byref(desc(g["cat1"], 16, 16)), ctypes.byref(desc(g["up1"], 0, 16)),
                            ctypes.byref(desc(g["cat1"], 16, 16)), _s()))
        self._conv_bwd("c1b", desc(a["c1a"]), desc(a["cat1"], 16, 16), desc(g["cat1"], 16, 16), desc(g["c1a"]))
        self._conv_bwd("c1a", desc(a["in"]), desc(a["c1a"]), desc(g["c1a"]), None)

    def mse(self, x0, target):
        """loss = mean (x0 - target)^2 (device FP64); fills self.gx0."""
        _check(lib().cvp_nn_mse(_p(x0), _p(target), x0.numel(), _p(self.gx0), _p(self.loss), _p(self.work64),
                                self.work64.numel(), _s()))
        return self.loss

    def adam(self, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
        self.step_count += 1
        L = lib()
        for c in self.convs.values():
            _check(L.cvp_nn_adam(_p(c.w), _p(c.gw), _p(c.m[0]), _p(c.v[0]), c.w.numel(), lr, b1, b2, eps,
                                 self.step_count, _p(c.wb), _s()))
            _check(L.cvp_nn_adam(_p(c.b), _p(c.gb), _p(c.m[1]), _p(c.v[1]), c.b.numel(), lr, b1, b2, eps,
                                 self.step_count, None, _s()))
            c.refresh()
        hp = torch.cat([self.hw, self.hb])
        _check(L.cvp_nn_adam(_p(hp), _p(self.ghead), _p(self.mh), _p(self.vh), 17, lr, b1, b2, eps,
                             self.step_count, None, _s()))
        self.hw.copy_(hp[:16])
        self.hb.copy_(hp[16:])

    def train_step(self, x1, x2, target, lr=1e-3):
        x0 = self.forward(x1, x2)
        loss = self.mse(x0, target)
        self.backward(self.gx0)
        self.adam(lr)
        return loss

    def state(self):
        """Parameters as a dict of CPU tensors (checkpoint)."""
        out = {n + ".w": c.w.cpu() for n, c in self.convs.items()}
        out.update({n + ".b": c.b.cpu() for n, c in self.convs.items()})
        out["head.w"], out["head.b"] = self.hw.cpu(), self.hb.cpu()
        return out
