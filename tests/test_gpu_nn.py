"""Denoiser kernels against the FP64 oracle (oracle/unet.py), through the C
ABI.  Operands are bfloat16 values, so the oracle sees exactly what the
kernels see; the tolerances are the FP32-accumulation bound
K * 2^-24 * sum|terms| plus half a bfloat16 ulp (2^-9 relative, taken as
2^-8) where a result is stored in bfloat16."""
import numpy as np
import pytest
import torch

from oracle import unet as U
from paper_2111_11687_amd import binding as B

pytestmark = pytest.mark.gpu
F64 = torch.float64
U24 = 2.0 ** -24


def _bf(shape, gen, scale=1.0, positive=False):
    x = torch.randn(*shape, generator=gen, dtype=torch.float32) * scale
    if positive:
        x = x.abs()
    return x.to(torch.bfloat16)


def _f64(t):
    return t.detach().cpu().to(F64)


def _up_crop(x, d, h, w):
    return U.upsample2(x)[:, :d, :h, :w]


def _conv_ref(x, w, b=None):
    return U.conv3x3(x, w, b)


def _check_bf16_result(got, ref, absref, k):
    tol = 2.0 ** -8 * ref.abs() + k * U24 * absref + 1e-30
    bad = (got - ref).abs() > tol
    assert not bool(bad.any()), "%d of %d outside; worst %.3g vs tol %.3g" % (
        int(bad.sum()), bad.numel(), float((got - ref).abs().max()), float(tol.max()))


def test_mfma_operand_layout(engine):
    g = torch.Generator().manual_seed(1)
    a = _bf((16, 32), g)
    b = _bf((32, 16), g)
    d = torch.empty(16, 16, dtype=torch.float32, device=engine.device)
    B.nmd_debug_mfma(engine.ctx, a.to(engine.device), b.to(engine.device), d)
    engine.sync()
    ref = _f64(a) @ _f64(b)
    absref = _f64(a).abs() @ _f64(b).abs()
    assert torch.all((_f64(d) - ref).abs() <= 32 * U24 * absref + 1e-30)


# (c0, up0, c1, c_out): the forward layers of the network and the forward
# convolutions the backward-data pass runs
FWD_SHAPES = [(8, 0, 0, 16), (16, 0, 0, 16), (16, 0, 0, 32), (32, 0, 0, 32), (32, 0, 0, 64),
              (64, 0, 0, 64), (64, 1, 32, 32), (32, 1, 16, 16), (16, 0, 0, 48), (32, 0, 0, 96),
              (64, 0, 0, 32), (32, 0, 0, 16)]


@pytest.mark.parametrize("c0,up0,c1,cout", FWD_SHAPES)
def test_conv_forward(engine, c0, up0, c1, cout):
    n, d, h, w = 2, 5, 11, 21  # 2 x 2 x 3 tiles per volume, ragged in every dimension
    g = torch.Generator().manual_seed(100 + c0 + c1 + cout + up0)
    dev = engine.device
    dims0 = ((d + 1) // 2, (h + 1) // 2, (w + 1) // 2) if up0 else (d, h, w)
    x0 = _bf((n,) + dims0 + (c0,), g)
    x1 = _bf((n, d, h, w, c1), g) if c1 else None
    cin = c0 + c1
    wt = _bf((cout, 27, cin), g, scale=(2.0 / (27 * cin)) ** 0.5)
    bias = torch.randn(cout, generator=g) * 0.1
    mask = _bf((n, d, h, w, cout), g)
    y = torch.empty(n, d, h, w, cout, dtype=torch.bfloat16, device=dev)
    src = B._src(x0.to(dev), c0, bool(up0), None if x1 is None else x1.to(dev), c1)
    B.nmd_conv3d_fwd(engine.ctx, (n, d, h, w), src, wt.to(dev), bias.to(dev), cout, True,
                     mask.to(dev), y)
    engine.sync()
    xin = _f64(x0)
    if up0:
        xin = _up_crop(xin, d, h, w)
    if c1:
        xin = torch.cat([xin, _f64(x1)], -1)
    pre = _conv_ref(xin, _f64(wt), bias.to(F64))
    ref = torch.relu(pre) * (_f64(mask) > 0)
    absref = _conv_ref(xin.abs(), _f64(wt).abs()) + bias.abs().to(F64)
    _check_bf16_result(_f64(y), ref, absref, 27 * cin)


def test_conv_forward_without_bias_relu_mask(engine):
    n, d, h, w = 1, 7, 9, 33
    g = torch.Generator().manual_seed(7)
    dev = engine.device
    x = _bf((n, d, h, w, 32), g)
    wt = _bf((32, 27, 32), g, scale=0.05)
    y = torch.empty(n, d, h, w, 32, dtype=torch.bfloat16, device=dev)
    B.nmd_conv3d_fwd(engine.ctx, (n, d, h, w), B._src(x.to(dev)), wt.to(dev), None, 32, False,
                     None, y)
    engine.sync()
    ref = _conv_ref(_f64(x), _f64(wt))
    _check_bf16_result(_f64(y), ref, _conv_ref(_f64(x).abs(), _f64(wt).abs()), 27 * 32)


# (layer c_in, layer c_out, masked): backward-data shapes of the network
BWD_DATA_SHAPES = [(16, 16, True), (48, 16, False), (32, 32, True), (96, 32, False),
                   (64, 64, True), (32, 64, False), (16, 32, False)]


@pytest.mark.parametrize("cin,cout,masked", BWD_DATA_SHAPES)
def test_conv_backward_data(engine, cin, cout, masked):
    n, d, h, w = 1, 6, 10, 19
    g = torch.Generator().manual_seed(200 + cin + cout)
    dev = engine.device
    theta = torch.randn(cout, 27, cin, generator=g) * (2.0 / (27 * cin)) ** 0.5
    wb = torch.empty(cout, 27, cin, dtype=torch.bfloat16, device=dev)
    wt = torch.empty(cin, 27, cout, dtype=torch.bfloat16, device=dev)
    B.nmd_nn_cast_weight(engine.ctx, theta.to(dev), cout, cin, wb, wt)
    dy = _bf((n, d, h, w, cout), g, scale=1e-3)
    mask = _bf((n, d, h, w, cin), g) if masked else None
    dx = torch.empty(n, d, h, w, cin, dtype=torch.bfloat16, device=dev)
    B.nmd_conv3d_bwd_data(engine.ctx, (n, d, h, w), dy.to(dev), cout, wt, cin,
                          None if mask is None else mask.to(dev), dx)
    engine.sync()
    w64 = U.bf16(theta.to(F64))
    assert torch.equal(_f64(wb), w64)
    assert torch.equal(_f64(wt), w64.flip(1).permute(2, 1, 0))
    xin = torch.zeros(n, d, h, w, cin, dtype=F64, requires_grad=True)
    (U.conv3x3(xin, w64) * _f64(dy)).sum().backward()
    ref = xin.grad
    if masked:
        ref = ref * (_f64(mask) > 0)
    absref = U.conv3x3(_f64(dy).abs(), w64.abs().flip(1).permute(2, 1, 0).contiguous())
    _check_bf16_result(_f64(dx), ref, absref, 27 * cout)


# (c0, up0, c1, c_out): backward-weight shapes of the network
WGRAD_SHAPES = [(8, 0, 0, 16), (16, 0, 0, 16), (16, 0, 0, 32), (32, 0, 0, 32), (32, 0, 0, 64),
                (64, 0, 0, 64), (64, 1, 32, 32), (32, 1, 16, 16)]


@pytest.mark.parametrize("c0,up0,c1,cout", WGRAD_SHAPES)
def test_conv_backward_weight(engine, c0, up0, c1, cout):
    n, d, h, w = 2, 5, 9, 21
    g = torch.Generator().manual_seed(300 + c0 + c1 + cout + up0)
    dev = engine.device
    dims0 = ((d + 1) // 2, (h + 1) // 2, (w + 1) // 2) if up0 else (d, h, w)
    x0 = _bf((n,) + dims0 + (c0,), g)
    x1 = _bf((n, d, h, w, c1), g) if c1 else None
    cin = c0 + c1
    dy = _bf((n, d, h, w, cout), g, scale=1e-2)
    dw = torch.empty(cout, 27, cin, dtype=torch.float32, device=dev)
    db = torch.empty(cout, dtype=torch.float32, device=dev)
    src = B._src(x0.to(dev), c0, bool(up0), None if x1 is None else x1.to(dev), c1)
    B.nmd_conv3d_bwd_weight(engine.ctx, (n, d, h, w), src, dy.to(dev), cout, dw, db)
    engine.sync()
    xin = _f64(x0)
    if up0:
        xin = _up_crop(xin, d, h, w)
    if c1:
        xin = torch.cat([xin, _f64(x1)], -1)
    wv = torch.zeros(cout, 27, cin, dtype=F64, requires_grad=True)
    bv = torch.zeros(cout, dtype=F64, requires_grad=True)
    (U.conv3x3(xin, wv, bv) * _f64(dy)).sum().backward()
    wa = torch.zeros(cout, 27, cin, dtype=F64, requires_grad=True)
    (U.conv3x3(xin.abs(), wa) * _f64(dy).abs()).sum().backward()
    nvox = n * d * h * w
    k = nvox / 32 + nvox / 128 + 64  # K steps per workgroup + partials
    assert torch.all((_f64(dw) - wv.grad).abs() <= k * U24 * wa.grad + 1e-30)
    assert torch.all((_f64(db) - bv.grad).abs() <= k * U24 * _f64(dy).abs().sum((0, 1, 2, 3)) + 1e-30)


def test_pool_and_combine(engine):
    g = torch.Generator().manual_seed(11)
    dev = engine.device
    n, d, h, w, c = 1, 6, 10, 14, 32
    x = _bf((n, d, h, w, c), g)
    y = torch.empty(n, d // 2, h // 2, w // 2, c, dtype=torch.bfloat16, device=dev)
    B.nmd_nn_pool2(engine.ctx, (n, d, h, w), c, x.to(dev), y)
    # combine at the coarse level: mask * (a[:, 64:96] + up-sample backward of b)
    dc = (1, d // 2, h // 2, w // 2)
    m = _bf(dc + (c,), g)
    a = _bf(dc + (96,), g)
    bfine = _bf((n, d, h, w, 48), g)
    o1 = torch.empty(dc + (c,), dtype=torch.bfloat16, device=dev)
    B.nmd_nn_combine(engine.ctx, dc, c, m.to(dev), a.to(dev), 96, 64, 1, bfine.to(dev), 48, 16,
                     o1)
    # combine at the fine level: a[:, 32:48] + pool backward of the coarse y
    o2 = torch.empty(n, d, h, w, 16, dtype=torch.bfloat16, device=dev)
    ycoarse = _bf(dc + (16,), g)
    B.nmd_nn_combine(engine.ctx, (n, d, h, w), 16, None, bfine.to(dev), 48, 32, 2,
                     ycoarse.to(dev), 16, 0, o2)
    engine.sync()
    ref = U.avg_pool2(_f64(x))
    assert torch.all((_f64(y) - ref).abs() <= 2.0 ** -8 * ref.abs() + 8 * U24 * U.avg_pool2(_f64(x).abs()))
    bsum = _f64(bfine)[..., 16:48].reshape(1, d // 2, 2, h // 2, 2, w // 2, 2, 32).sum((2, 4, 6))
    r1 = (_f64(a)[..., 64:96] + bsum) * (_f64(m) > 0)
    assert torch.all((_f64(o1) - r1).abs() <= 2.0 ** -8 * r1.abs() + 9 * U24 * (
        _f64(a)[..., 64:96].abs() + _f64(bfine)[..., 16:48].abs().reshape(
            1, d // 2, 2, h // 2, 2, w // 2, 2, 32).sum((2, 4, 6))))
    r2 = _f64(bfine)[..., 32:48] + U.upsample2(_f64(ycoarse)) / 8
    assert torch.all((_f64(o2) - r2).abs() <= 2.0 ** -8 * r2.abs() + 2 * U24 * (
        _f64(bfine)[..., 32:48].abs() + U.upsample2(_f64(ycoarse)).abs() / 8))


@pytest.mark.parametrize("floor", [0.0, 0.3])
def test_head_loss(engine, floor):
    g = torch.Generator().manual_seed(12)
    dev = engine.device
    nvox = 5000
    feat = _bf((nvox, 16), g)
    x0 = _bf((nvox, 8), g, positive=True)
    tgt = torch.rand(nvox, generator=g)
    hw = torch.randn(16, generator=g) * 0.2
    hb = torch.randn(1, generator=g) * 0.1
    feat_d, x0_d, tgt_d, hw_d, hb_d = (t.to(dev) for t in (feat, x0, tgt, hw, hb))
    dfeat = torch.empty(nvox, 16, dtype=torch.bfloat16, device=dev)
    grad = torch.empty(18, dtype=torch.float32, device=dev)
    B.nmd_nn_head_loss(engine.ctx, nvox, feat_d, x0_d, tgt_d, hw_d, hb_d, dfeat, grad, floor)
    engine.sync()
    f = _f64(feat)
    t64 = tgt.to(F64)
    pred = _f64(x0)[:, 0] + f @ hw.to(F64) + hb.to(F64)
    e = pred - t64
    wv = 1.0 / torch.clamp(t64, min=floor) if floor > 0 else torch.ones_like(t64)
    gv = 2 * wv * e / nvox
    gf = (gv[:, None] * hw.to(F64)) * (f > 0)
    # FP32 error of the residual e (and one rounding of the weight), carried
    # into g = 2 w e / nvox and g * w_head
    sc = _f64(x0)[:, 0].abs() + f.abs() @ hw.abs().to(F64) + hb.abs().to(F64) + t64.abs()
    de = (24 * U24 * sc + 4 * U24 * e.abs()) * wv
    tol = 2.0 ** -8 * gf.abs() + (2.0 / nvox) * de[:, None] * hw.abs().to(F64)
    assert torch.all((_f64(dfeat) - gf).abs() <= tol)
    gr = _f64(grad)
    gabs = ((gv.abs() + 2 * de / nvox)[:, None] * f.abs()).sum(0)
    assert torch.all((gr[:16] - (gv[:, None] * f).sum(0)).abs() <= 1e-4 * gabs)
    assert abs(gr[16].item() - gv.sum().item()) <= 1e-4 * (gv.abs() + 2 * de / nvox).sum().item()
    lref = (wv * e * e).sum().item()
    assert abs(gr[17].item() - lref) <= 1e-5 * lref
    assert abs(U.mse(pred[None], tgt[None], floor).item() - lref / nvox) <= 1e-12 * lref


def test_adam_step(engine):
    g = torch.Generator().manual_seed(13)
    dev = engine.device
    co, ci = 16, 32
    n = co * 27 * ci
    th = torch.randn(n, generator=g)
    m = torch.randn(n, generator=g) * 1e-3
    v = torch.rand(n, generator=g) * 1e-6
    gr = torch.randn(n, generator=g) * 1e-3
    dth, dm, dv = th.to(dev), m.to(dev), v.to(dev)
    wb = torch.empty(n, dtype=torch.bfloat16, device=dev)
    wt = torch.empty(n, dtype=torch.bfloat16, device=dev)
    B.nmd_nn_adam(engine.ctx, dth, dm, dv, gr.to(dev), 3, 1e-3, w_bf16=wb, w_t_bf16=wt,
                  c_out=co, c_in=ci)
    engine.sync()
    # the kernel receives its hyperparameters as FP32: give the oracle the
    # same values (1 - 0.9f differs from 0.1 by 2.4e-7 relative)
    f32 = lambda x: float(np.float32(x))  # noqa: E731
    rt, rm, rv = U.adam_step(th, m, v, gr, 3, lr=f32(1e-3), beta1=f32(0.9), beta2=f32(0.999),
                             eps=f32(1e-8))
    # FP32 moments: a few roundings of the terms 0.9 m + 0.1 g (0.999 v + 0.001 g^2)
    m64, g64, v64 = m.to(F64), gr.to(F64), v.to(F64)
    assert torch.all((_f64(dm) - rm).abs() <= 4 * U24 * (0.9 * m64.abs() + 0.1 * g64.abs()))
    assert torch.all((_f64(dv) - rv).abs() <= 4 * U24 * (0.999 * v64 + 0.001 * g64 * g64))
    # an update of about lr = 1e-3 computed to ~1e-6 relative, then rounded into theta
    np.testing.assert_allclose(_f64(dth).numpy(), rt.numpy(), rtol=3e-7, atol=1e-8)
    # the working copies are the bf16 of the new masters
    assert torch.equal(wb.cpu(), dth.cpu().to(torch.bfloat16))
    assert torch.equal(wt.cpu().view(ci, 27, co), dth.cpu().to(torch.bfloat16).view(co, 27, ci).flip(1).permute(2, 1, 0))


def test_unet_loss_and_gradients_match_oracle(engine):
    """Whole network, one loss-and-gradient pass on an 8 x 16 x 28 box.

    Both sides round to bfloat16 at the same storage points, so they differ
    only where FP32 and FP64 accumulation land on different sides of a
    bfloat16 rounding boundary (or of a ReLU).  Those flips compound through
    the layers: the oracle itself, with its convolutions accumulated in FP32
    instead of FP64, moves its gradients by up to 1.4% (relative norm) on this
    box.  The bound is three times that."""
    from paper_2111_11687_amd import denoiser as DN
    dev = engine.device
    g = torch.Generator().manual_seed(14)
    d, h, w = 8, 16, 28
    net = DN.UNet(engine, seed=5)
    st = U.init_params(width=16, seed=6)
    for k in st:  # non-zero head and biases so every path carries gradient
        if k.endswith(".b") or k.startswith("head"):
            st[k] = torch.randn(st[k].shape, generator=g) * 0.1
    net.load_state(st)
    ws = DN.Workspace(engine, (d, h, w))
    x3 = torch.rand(1, d, h, w, 3, generator=g) * 2
    x8 = torch.zeros(d, h, w, 8)
    x8[..., :3] = x3[0]
    ws.x0.copy_(x8.to(torch.bfloat16).to(dev))
    tgt = torch.rand(d, h, w, generator=g) * 2
    ws.target.copy_(tgt.to(dev))
    net.loss_and_grad(ws)
    engine.sync()
    loss_ref, g_ref = U.loss_and_grads(st, x3.to(F64), tgt[None].to(F64), bf16_storage=True)
    assert abs(ws.loss_value(net) - loss_ref) <= 1e-3 * loss_ref
    for name, ci, co, _ in DN.layer_table():
        gw = _f64(net.p[name + ".dw"])
        if name == "enc0a":
            assert torch.all(gw[:, :, 3:] == 0)
            gw = gw[:, :, :3]
        for key, got in ((name + ".w", gw), (name + ".b", _f64(net.p[name + ".db"]))):
            ref = g_ref[key]
            rel = ((got - ref).norm() / ref.norm()).item()
            assert rel < 0.04, (key, rel)
    hg = _f64(net.hgrad)
    assert ((hg[:16] - g_ref["head.w"]).norm() / g_ref["head.w"].norm()).item() < 1e-3
    assert abs(hg[16].item() - g_ref["head.b"].item()) <= 1e-3 * abs(g_ref["head.b"].item())


def test_organ_mean_of_a_map_equals_eq2(engine):
    """The organ mean of the engine's own dose-rate map is Eq. 2."""
    from paper_2111_11687_amd import phantoms as P
    prob = P.patient_phantom(shape=(40, 32, 32), voxel_mm=(16.0, 16.0, 24.0), seed=31)
    engine.set_problem(50, prob)
    engine.run(50, 200_000, 3)
    rate, _ = engine.dose(50)
    org, _, _ = engine.organs(50)
    got = B.nmd_organ_mean_map(engine.ctx, 50, rate, prob.n_organs)
    np.testing.assert_allclose(got, org, rtol=1e-12, atol=0)


def _gather_concat(up, skip, z, y, x):
    """Input voxels (z, y, x) (integer arrays, zero outside) of the
    concatenation [nearest-up-sample(up) | skip] as FP64 [..., C]."""
    D, H, W = skip.shape[:3]
    ok = (z >= 0) & (z < D) & (y >= 0) & (y < H) & (x >= 0) & (x < W)
    zc, yc, xc = np.clip(z, 0, D - 1), np.clip(y, 0, H - 1), np.clip(x, 0, W - 1)
    v = np.concatenate([up[zc // 2, yc // 2, xc // 2], skip[zc, yc, xc]], -1).astype(np.float64)
    return v * ok[..., None]


def test_decoder_convolution_at_the_full_box_size(engine):
    """dec0a at 160 x 128 x 128 (input: up-sampled 32-channel level-1
    features | 16-channel skip): forward outputs and weight-gradient entries
    sampled and computed one by one from their definitions in FP64."""
    dev = engine.device
    g = torch.Generator().manual_seed(21)
    d, h, w = 160, 128, 128
    up = _bf((1, d // 2, h // 2, w // 2, 32), g)
    skip = _bf((1, d, h, w, 16), g)
    wt = _bf((16, 27, 48), g, scale=(2.0 / (27 * 48)) ** 0.5)
    bias = torch.randn(16, generator=g) * 0.1
    dy = _bf((1, d, h, w, 16), g, scale=1e-3)
    up_d, skip_d, wt_d, b_d, dy_d = (t.to(dev) for t in (up, skip, wt, bias, dy))
    y = torch.empty(1, d, h, w, 16, dtype=torch.bfloat16, device=dev)
    dw = torch.empty(16, 27, 48, dtype=torch.float32, device=dev)
    src = B._src(up_d, 32, True, skip_d, 16)
    B.nmd_conv3d_fwd(engine.ctx, (1, d, h, w), src, wt_d, b_d, 16, True, None, y)
    B.nmd_conv3d_bwd_weight(engine.ctx, (1, d, h, w), src, dy_d, 16, dw, None)
    engine.sync()
    upn = up[0].float().numpy()
    skn = skip[0].float().numpy()
    w64 = wt.float().numpy().astype(np.float64)
    rng = np.random.default_rng(0)
    ns = 3000
    # include the faces and corners of the box
    pts = np.stack([rng.integers(0, s, ns) for s in (d, h, w)], 1)
    pts[:8] = [[a, b, c] for a in (0, d - 1) for b in (0, h - 1) for c in (0, w - 1)]
    co = rng.integers(0, 16, ns)
    taps = np.array([(kz - 1, ky - 1, kx - 1) for kz in range(3) for ky in range(3) for kx in range(3)])
    nb = pts[:, None, :] + taps[None]  # [ns, 27, 3]
    xin = _gather_concat(upn, skn, nb[..., 0], nb[..., 1], nb[..., 2])  # [ns, 27, 48]
    pre = (xin * w64[co]).sum((1, 2)) + bias.double().numpy()[co]
    absr = (np.abs(xin) * np.abs(w64[co])).sum((1, 2)) + np.abs(bias.double().numpy()[co])
    ref = np.maximum(pre, 0)
    got = y[0].cpu().float().numpy()[pts[:, 0], pts[:, 1], pts[:, 2], co].astype(np.float64)
    assert np.all(np.abs(got - ref) <= 2.0 ** -8 * np.abs(ref) + 27 * 48 * U24 * absr)
    # weight-gradient entries: sum over all voxels of dy[v, o] * x[v + offset(t), i]
    dyn = dy[0].float().numpy()
    zz, yy, xx = np.meshgrid(np.arange(d), np.arange(h), np.arange(w), indexing="ij")
    dwn = dw.cpu().double().numpy()
    for _ in range(24):
        o, t, i = int(rng.integers(16)), int(rng.integers(27)), int(rng.integers(48))
        oz, oy, ox = taps[t]
        z2, y2, x2 = zz + oz, yy + oy, xx + ox
        ok = (z2 >= 0) & (z2 < d) & (y2 >= 0) & (y2 < h) & (x2 >= 0) & (x2 < w)
        z2, y2, x2 = np.clip(z2, 0, d - 1), np.clip(y2, 0, h - 1), np.clip(x2, 0, w - 1)
        xi = (upn[z2 // 2, y2 // 2, x2 // 2, i] if i < 32 else skn[z2, y2, x2, i - 32]) * ok
        terms = dyn[..., o].astype(np.float64) * xi.astype(np.float64)
        k = d * h * w / 2048 + 2100  # K steps per workgroup + partials, bounded
        assert abs(dwn[o, t, i] - terms.sum()) <= k * U24 * np.abs(terms).sum(), (o, t, i)
