"""U-Net kernels (BF16 MFMA convolutions, FP32 accumulation) against the
FP64 layer reference (oracle/unet.py) on the same BF16-rounded inputs, and a
short training run that must lower the loss."""
import ctypes

import numpy as np
import pytest
import torch

from oracle import unet as OU
from paper_2110_09841_amd import unet
from paper_2110_09841_amd.unet import _check, _p, _s, desc, lib

from gpu_util import needs_gpu, say

pytestmark = [pytest.mark.gpu, needs_gpu]

BF16_ULP = 2.0 ** -8


def rnd(shape, seed, scale=1.0):
    g = torch.Generator().manual_seed(seed)
    return (scale * torch.randn(shape, generator=g)).to(torch.bfloat16)


def f64(t):
    return t.detach().cpu().double().numpy()


def ref_conv(x_bf, w_bf, b=None):
    """x (D,H,W,Ci) bf16, w (27,Co,Ci) bf16 -> (D,H,W,Co) float64"""
    return torch.from_numpy(OU.conv3d(f64(x_bf), f64(w_bf), None if b is None else f64(b)))


def close_bf16(got, ref, what, k=2.0):
    got = got.double()
    err = (got - ref).abs()
    tol = k * BF16_ULP * ref.abs() + 1e-6 * ref.abs().max()
    bad = int((err > tol).sum())
    say("%s: max abs err %.3e (max |ref| %.3e), %d out of tolerance" % (what, float(err.max()), float(ref.abs().max()), bad))
    assert bad == 0


@pytest.mark.parametrize("ci,co,shape", [(16, 16, (8, 10, 70)), (16, 32, (6, 7, 20)), (32, 64, (4, 6, 12)),
                                         (64, 32, (5, 4, 9)), (32, 16, (6, 6, 66))])
def test_conv3d_forward_backward_data_and_weight(ci, co, shape):
    D, H, W = shape
    x = rnd((D, H, W, ci), 1)
    w = rnd((27, co, ci), 2, 0.1)
    b = torch.randn(co, generator=torch.Generator().manual_seed(3)).float()
    L = lib()
    xd, wd, bd = x.cuda(), w.cuda(), b.cuda()
    y = torch.empty((D, H, W, co), dtype=torch.bfloat16, device="cuda")
    say("conv fwd", ci, co, shape)
    _check(L.cvp_nn_conv3d(ctypes.byref(desc(xd)), _p(wd), _p(bd), ctypes.byref(desc(y)), 0, 0, _s()))
    close_bf16(y.cpu(), ref_conv(x, w, b), "conv forward")
    yr = torch.empty_like(y)
    _check(L.cvp_nn_conv3d(ctypes.byref(desc(xd)), _p(wd), _p(bd), ctypes.byref(desc(yr)), 1, 0, _s()))
    close_bf16(yr.cpu(), torch.clamp(ref_conv(x, w, b), min=0), "conv forward relu")
    # backward-data: dX = conv(dY, mirrored transposed W)
    gy = rnd((D, H, W, co), 4)
    wt = torch.empty((27, ci, co), dtype=torch.bfloat16, device="cuda")
    _check(L.cvp_nn_transpose_weights(_p(wd), _p(wt), co, ci, _s()))
    gx = torch.empty((D, H, W, ci), dtype=torch.bfloat16, device="cuda")
    _check(L.cvp_nn_conv3d(ctypes.byref(desc(gy.cuda())), _p(wt), None, ctypes.byref(desc(gx)), 0, 1, _s()))
    gx_ref = torch.from_numpy(OU.conv3d_grad_input(f64(gy), f64(w)))
    close_bf16(gx.cpu(), gx_ref, "conv backward-data")
    # backward-weight (FP32 out)
    n = ctypes.c_int64()
    _check(L.cvp_nn_wgrad_workspace(ctypes.byref(desc(xd)), ctypes.byref(desc(gy.cuda())), ctypes.byref(n)))
    work = torch.empty(n.value, dtype=torch.float32, device="cuda")
    gw = torch.empty((27, co, ci), dtype=torch.float32, device="cuda")
    gyd = gy.cuda()
    _check(L.cvp_nn_conv3d_wgrad(ctypes.byref(desc(xd)), ctypes.byref(desc(gyd)), _p(gw), _p(work), n.value, _s()))
    gw_ref = torch.from_numpy(OU.conv3d_grad_weight(f64(x), f64(gy)))
    err = (gw.cpu().double() - gw_ref).abs().max() / gw_ref.abs().max()
    say("conv backward-weight rel err %.3e" % float(err))
    assert err < 1e-5
    # bias gradient
    gb = torch.empty(co, dtype=torch.float32, device="cuda")
    _check(L.cvp_nn_channel_sum(ctypes.byref(desc(gyd)), _p(gb), _p(work), n.value, _s()))
    assert np.allclose(f64(gb), OU.bias_grad(f64(gy)), rtol=1e-5, atol=1e-4)


def _crop(a, z, y, x):
    """3x3x3 neighbourhood of voxel (z, y, x) of a (D, H, W, C) array, zero
    outside the volume (the convolution's padding)."""
    D, H, W, C = a.shape
    out = np.zeros((3, 3, 3, C))
    for dz in range(3):
        for dy in range(3):
            for dx in range(3):
                zz, yy, xx = z + dz - 1, y + dy - 1, x + dx - 1
                if 0 <= zz < D and 0 <= yy < H and 0 <= xx < W:
                    out[dz, dy, dx] = a[zz, yy, xx]
    return out


# (Cin, Cout, volume edge) of the network's convolutions at the warm-start
# workload's 128^3 volume: c1a/c1b/d1b, u1/d1a, c2a, c2b/d2b, u2/d2a, c3a, c3b
NET_CONVS = [(16, 16, 128), (32, 16, 128), (16, 32, 64), (32, 32, 64), (64, 32, 64), (32, 64, 32), (64, 64, 32)]


@pytest.mark.parametrize("ci,co,edge", NET_CONVS)
def test_conv3d_at_network_shapes(ci, co, edge):
    """Each convolution shape the U-Net runs on 128^3 volumes, at its real
    size: forward and backward-data on 1500 sampled voxels (the oracle's
    convolution of each voxel's 3x3x3 neighbourhood), backward-weight (a sum
    over every voxel) in full."""
    shape = (edge, edge, edge)
    x = rnd(shape + (ci,), 11, 0.5)
    w = rnd((27, co, ci), 12, 0.1)
    b = torch.randn(co, generator=torch.Generator().manual_seed(13)).float()
    gy = rnd(shape + (co,), 14)
    L = lib()
    xd, wd, bd, gyd = x.cuda(), w.cuda(), b.cuda(), gy.cuda()
    say("network conv", ci, co, shape)
    y = torch.empty(shape + (co,), dtype=torch.bfloat16, device="cuda")
    _check(L.cvp_nn_conv3d(ctypes.byref(desc(xd)), _p(wd), _p(bd), ctypes.byref(desc(y)), 1, 0, _s()))
    wt = torch.empty((27, ci, co), dtype=torch.bfloat16, device="cuda")
    _check(L.cvp_nn_transpose_weights(_p(wd), _p(wt), co, ci, _s()))
    gx = torch.empty(shape + (ci,), dtype=torch.bfloat16, device="cuda")
    _check(L.cvp_nn_conv3d(ctypes.byref(desc(gyd)), _p(wt), None, ctypes.byref(desc(gx)), 0, 1, _s()))
    n = ctypes.c_int64()
    _check(L.cvp_nn_wgrad_workspace(ctypes.byref(desc(xd)), ctypes.byref(desc(gyd)), ctypes.byref(n)))
    work = torch.empty(n.value, dtype=torch.float32, device="cuda")
    gw = torch.empty((27, co, ci), dtype=torch.float32, device="cuda")
    _check(L.cvp_nn_conv3d_wgrad(ctypes.byref(desc(xd)), ctypes.byref(desc(gyd)), _p(gw), _p(work), n.value, _s()))
    torch.cuda.synchronize()
    xh, wh, bh, gyh = f64(x), f64(w), f64(b), f64(gy)
    yg, gxg = y.cpu().double(), gx.cpu().double()
    rng = np.random.default_rng(ci * 1000 + co + edge)
    pts = rng.integers(0, edge, size=(1500, 3))
    pts[:8] = [[0, 0, 0], [edge - 1] * 3, [0, edge - 1, 0], [edge - 1, 0, edge - 1],
               [0, 5, edge - 1], [edge // 2] * 3, [1, 1, 1], [edge - 2, edge - 2, edge - 2]]
    ref_y = np.stack([OU.conv3d(_crop(xh, *p), wh, bh, relu=True)[1, 1, 1] for p in pts])
    ref_gx = np.stack([OU.conv3d_grad_input(_crop(gyh, *p), wh)[1, 1, 1] for p in pts])
    got_y = torch.stack([yg[tuple(p)] for p in pts])
    got_gx = torch.stack([gxg[tuple(p)] for p in pts])
    close_bf16(got_y, torch.from_numpy(ref_y), "forward (relu) %dx%d @%d^3 sampled" % (ci, co, edge))
    close_bf16(got_gx, torch.from_numpy(ref_gx), "backward-data %dx%d @%d^3 sampled" % (ci, co, edge))
    gw_ref = OU.conv3d_grad_weight(xh, gyh)
    err = float(np.abs(gw.cpu().double().numpy() - gw_ref).max() / np.abs(gw_ref).max())
    say("backward-weight %dx%d @%d^3 rel err %.3e" % (ci, co, edge, err))
    assert err < 1e-5


def test_channel_slices_pool_upsample_add_head():
    L = lib()
    D, H, W = 8, 6, 10
    big = rnd((D, H, W, 32), 5).cuda()
    sl = desc(big, 16, 16)                         # channels 16..31
    pooled = torch.empty((D // 2, H // 2, W // 2, 16), dtype=torch.bfloat16, device="cuda")
    _check(L.cvp_nn_avgpool2(ctypes.byref(sl), ctypes.byref(desc(pooled)), _s()))
    ref = torch.from_numpy(OU.avgpool2(f64(big[..., 16:])))
    close_bf16(pooled.cpu(), ref, "avgpool")
    up = torch.empty((D, H, W, 16), dtype=torch.bfloat16, device="cuda")
    _check(L.cvp_nn_upsample2(ctypes.byref(desc(pooled)), ctypes.byref(desc(up)), _s()))
    refu = torch.from_numpy(OU.upsample2(f64(pooled)))
    assert torch.equal(up.cpu().double(), refu)
    gin = torch.empty((D, H, W, 16), dtype=torch.bfloat16, device="cuda")
    _check(L.cvp_nn_avgpool2_bwd(ctypes.byref(desc(pooled)), ctypes.byref(desc(gin)), _s()))
    close_bf16(gin.cpu(), torch.from_numpy(OU.avgpool2_grad(f64(pooled))), "avgpool backward")
    gsm = torch.empty_like(pooled)
    _check(L.cvp_nn_upsample2_bwd(ctypes.byref(desc(up)), ctypes.byref(desc(gsm)), _s()))
    close_bf16(gsm.cpu(), torch.from_numpy(OU.upsample2_grad(f64(up))), "upsample backward")
    s = torch.empty_like(up)
    _check(L.cvp_nn_add(ctypes.byref(desc(up)), ctypes.byref(desc(gin)), ctypes.byref(desc(s)), _s()))
    close_bf16(s.cpu(), up.cpu().double() + gin.cpu().double(), "add")
    # head and its backward
    h = rnd((D, H, W, 16), 6).cuda()
    w = torch.randn(16, generator=torch.Generator().manual_seed(7)).float().cuda()
    b = torch.tensor([0.3], device="cuda")
    x2 = torch.rand((D, H, W), device="cuda")
    x0 = torch.empty_like(x2)
    sc = unet.INPUT_SCALE
    _check(L.cvp_nn_head(ctypes.byref(desc(h)), _p(w), _p(b), _p(x2), ctypes.c_float(sc), _p(x0), _s()))
    ref0 = OU.head(f64(h), f64(w), 0.3, f64(x2), sc)
    assert np.allclose(f64(x0), ref0, rtol=1e-5, atol=1e-6)
    g = torch.rand((D, H, W), device="cuda")
    dh = torch.empty_like(h)
    dwb = torch.empty(17, device="cuda")
    work = torch.empty(4096, device="cuda")
    _check(L.cvp_nn_head_bwd(ctypes.byref(desc(h)), _p(w), _p(g), ctypes.c_float(sc), ctypes.byref(desc(dh)), _p(dwb),
                             _p(work), 4096, _s()))
    rdh, rdw, rdb = OU.head_grad(f64(h), f64(w), f64(g), sc)
    close_bf16(dh.cpu(), torch.from_numpy(rdh), "head backward dh")
    assert np.allclose(f64(dwb[:16]), rdw, rtol=1e-4)
    assert abs(float(dwb[16]) - rdb) < 1e-4 * abs(rdb)


def test_mse_and_adam():
    L = lib()
    a = torch.rand(1000, device="cuda")
    b = torch.rand(1000, device="cuda")
    g = torch.empty_like(a)
    loss = torch.zeros(1, dtype=torch.float64, device="cuda")
    work = torch.empty(1024, dtype=torch.float64, device="cuda")
    _check(L.cvp_nn_mse(_p(a), _p(b), 1000, _p(g), _p(loss), _p(work), 1024, _s()))
    ref, rgrad = OU.mse(f64(a), f64(b))
    assert abs(float(loss) - ref) < 1e-7 * ref   # FP32 differences, FP64 sum
    assert np.allclose(f64(g), rgrad, rtol=1e-6, atol=1e-9)
    p = torch.rand(50, device="cuda")
    p0 = p.cpu().double().clone()
    gr = torch.randn(50, device="cuda")
    m = torch.zeros(50, device="cuda")
    v = torch.zeros(50, device="cuda")
    pm, pv, pp = np.zeros(50), np.zeros(50), p0.numpy().copy()
    for step in range(1, 4):
        _check(L.cvp_nn_adam(_p(p), _p(gr), _p(m), _p(v), 50, 1e-2, 0.9, 0.999, 1e-8, step, None, _s()))
        pp, pm, pv = OU.adam_step(pp, f64(gr), pm, pv, step, 1e-2)
    assert np.allclose(p.cpu().double().numpy(), pp, rtol=1e-5, atol=1e-6)


def test_unet_training_lowers_loss():
    torch.manual_seed(0)
    shape = (16, 16, 16)
    net = unet.UNet(shape, seed=1)
    rng = np.random.default_rng(2)
    x2 = torch.from_numpy(rng.uniform(0, 0.02, size=shape).astype(np.float32)).cuda()
    x1 = 0.5 * x2
    target = x2 + 0.005 * torch.sin(torch.arange(16, device="cuda").float())[None, None, :]
    losses = []
    for it in range(40):
        losses.append(float(net.train_step(x1, x2, target, lr=3e-3)))
    say("unet loss %.3e -> %.3e" % (losses[0], losses[-1]))
    assert losses[-1] < 0.5 * losses[0]
