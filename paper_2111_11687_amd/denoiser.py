"""3D U-Net denoiser of Monte Carlo dose maps, run through the C ABI of
include/nmdose_nn.h.

Not part of the paper: the learned stage added on top of its Monte Carlo.
The network maps (low-history dose, density, activity) on a box of a
phantom to the high-history dose on that box:

    level 0  conv 3->w, conv w->w                      (skip s0)
    level 1  pool, conv w->2w, conv 2w->2w             (skip s1)
    level 2  pool, conv 2w->4w, conv 4w->4w
    level 1  up-sample, concat s1, conv 6w->2w, conv 2w->2w
    level 0  up-sample, concat s0, conv 3w->w, conv w->w
    head     1x1x1 conv w->1 added to the input dose channel

with 3x3x3 convolutions (padding 1) followed by ReLU, 2x2x2 average pooling
and x2 nearest-neighbour up-sampling; w = 16.  The input dose and activity
are divided by their mean over body voxels of the box and density by
1.85 g/cm^3; the prediction is multiplied back by the dose scale.

This module owns the device tensors (through PyTorch) and sequences the
kernels; every arithmetic step runs in the HIP library.  The network input is
stored with 8 channels (3 used, 5 zero), the smallest channel count of the
convolution kernels.
"""
from __future__ import annotations

import math

import numpy as np

from . import binding as B

IN_CH = 8  # stored input channels: dose, density, activity, 5 x zero
REAL_IN = 3

# name, input channels, output channels, level; widths as multiples of w
_ARCH = (
    ("enc0a", None, 1, 0), ("enc0b", 1, 1, 0),
    ("enc1a", 1, 2, 1), ("enc1b", 2, 2, 1),
    ("mid_a", 2, 4, 2), ("mid_b", 4, 4, 2),
    ("dec1a", 6, 2, 1), ("dec1b", 2, 2, 1),
    ("dec0a", 3, 1, 0), ("dec0b", 1, 1, 0),
)


def layer_table(width=16):
    """(name, stored input channels, output channels, level)."""
    return [(n, IN_CH if ci is None else ci * width, co * width, lev) for n, ci, co, lev in _ARCH]


def conv_flops(shape, width=16):
    """Multiply-add FLOPs (2 per MAC) of the forward convolutions on a
    (d, h, w) box, counting the 3 real input channels of the first layer."""
    d, h, w = shape
    vox = [d * h * w, (d // 2) * (h // 2) * (w // 2), (d // 4) * (h // 4) * (w // 4)]
    tot = 0
    for name, ci, co, lev in layer_table(width):
        ci_real = REAL_IN if name == "enc0a" else ci
        tot += 2 * 27 * ci_real * co * vox[lev]
    return tot


class UNet:
    """Parameters (FP32 masters, Adam moments, BF16 working and flipped
    copies) on the device of `eng`."""

    def __init__(self, eng, width=16, seed=0):
        if width != 16:
            raise ValueError("the head kernel is built for 16 channels")
        self.eng = eng
        self.ctx = eng.ctx
        t = eng.torch
        self.t = t
        dev = eng.device
        self.width = width
        self.layers = layer_table(width)
        self.p = {}
        g = t.Generator().manual_seed(seed)
        for name, ci, co, _ in self.layers:
            ci_real = REAL_IN if name == "enc0a" else ci
            w = t.zeros(co, 27, ci, dtype=t.float32)
            w[:, :, :ci_real] = t.randn(co, 27, ci_real, generator=g, dtype=t.float64).float() \
                * math.sqrt(2.0 / (27 * ci_real))
            self._add(name + ".w", w.to(dev))
            self._add(name + ".b", t.zeros(co, dtype=t.float32, device=dev))
            self.p[name + ".wb"] = t.empty(co, 27, ci, dtype=t.bfloat16, device=dev)
            self.p[name + ".wt"] = t.empty(ci, 27, co, dtype=t.bfloat16, device=dev)
            self.p[name + ".dw"] = t.zeros(co, 27, ci, dtype=t.float32, device=dev)
            self.p[name + ".db"] = t.zeros(co, dtype=t.float32, device=dev)
        self._add("head.w", t.zeros(width, dtype=t.float32, device=dev))
        self._add("head.b", t.zeros(1, dtype=t.float32, device=dev))
        self.hgrad = t.zeros(18, dtype=t.float32, device=dev)
        self.step = 0
        self.refresh()

    def _add(self, key, theta):
        self.p[key] = theta.contiguous()
        self.p[key + ".m"] = self.t.zeros_like(theta)
        self.p[key + ".v"] = self.t.zeros_like(theta)

    def refresh(self):
        """Rebuild the BF16 copies from the FP32 masters."""
        for name, ci, co, _ in self.layers:
            B.nmd_nn_cast_weight(self.ctx, self.p[name + ".w"], co, ci, self.p[name + ".wb"],
                                 self.p[name + ".wt"])

    # parameters in the layout [c_out][27][c_in] with the 3 real input channels
    def state(self):
        out = {}
        for name, ci, co, _ in self.layers:
            w = self.p[name + ".w"].detach().cpu()
            out[name + ".w"] = w[:, :, :REAL_IN].clone() if name == "enc0a" else w.clone()
            out[name + ".b"] = self.p[name + ".b"].detach().cpu().clone()
        out["head.w"] = self.p["head.w"].detach().cpu().clone()
        out["head.b"] = self.p["head.b"].detach().cpu().clone()
        return out

    def load_state(self, state):
        t = self.t
        for key, val in state.items():
            dst = self.p[key]
            val = t.as_tensor(val, dtype=t.float32)
            if key == "enc0a.w":
                full = t.zeros(dst.shape, dtype=t.float32)
                full[:, :, :val.shape[2]] = val
                val = full
            dst.copy_(val.reshape(dst.shape).to(dst.device))
        self.refresh()

    def save(self, path, bias=None):
        """Parameters (and, if given, the per-organ bias table of the
        fallback) as an uncompressed .npz of plain arrays."""
        st = {k: v.numpy() for k, v in self.state().items()}
        if bias is not None:
            st["organ_bias"] = np.asarray(bias, dtype=np.float64)
        np.savez(path, step=self.step, **st)

    def load(self, path):
        """Loads parameters saved by save(); returns the organ bias table or
        None."""
        with np.load(path, allow_pickle=False) as z:
            self.load_state({k: z[k] for k in z.files if k not in ("step", "organ_bias")})
            self.step = int(z["step"])
            return np.array(z["organ_bias"]) if "organ_bias" in z.files else None

    # ------------------------------------------------------------------ run
    def forward(self, ws, events=None):
        """Network body on the prepared input ws.x0; leaves the last
        features in ws.a['d0b'].  If `events` is a dict, a pair of timing
        events recorded on the current stream around each convolution is
        appended to events[layer name]."""
        c, p, a = self.ctx, self.p, ws.a
        L0, L1, L2 = ws.dims

        def conv(name, dims, src, out):
            co = int(p[name + ".b"].numel())
            ev = None
            if events is not None:
                t = self.t
                ev = (t.cuda.Event(enable_timing=True), t.cuda.Event(enable_timing=True))
                ev[0].record(t.cuda.current_stream())
            B.nmd_conv3d_fwd(c, dims, src, p[name + ".wb"], p[name + ".b"], co, True, None, out)
            if ev is not None:
                ev[1].record(self.t.cuda.current_stream())
                events.setdefault(name, []).append(ev)

        conv("enc0a", L0, B._src(ws.x0), a["e0a"])
        conv("enc0b", L0, B._src(a["e0a"]), a["e0b"])
        B.nmd_nn_pool2(c, L0, 16, a["e0b"], a["p0"])
        conv("enc1a", L1, B._src(a["p0"]), a["e1a"])
        conv("enc1b", L1, B._src(a["e1a"]), a["e1b"])
        B.nmd_nn_pool2(c, L1, 32, a["e1b"], a["p1"])
        conv("mid_a", L2, B._src(a["p1"]), a["ma"])
        conv("mid_b", L2, B._src(a["ma"]), a["mb"])
        conv("dec1a", L1, B._src(a["mb"], 64, True, a["e1b"], 32), a["d1a"])
        conv("dec1b", L1, B._src(a["d1a"]), a["d1b"])
        conv("dec0a", L0, B._src(a["d1b"], 32, True, a["e0b"], 16), a["d0a"])
        conv("dec0b", L0, B._src(a["d0a"]), a["d0b"])

    def backward(self, ws):
        """Gradients of every parameter from the head's dfeat (ws.g['d0b'])."""
        c, p, a, g = self.ctx, self.p, ws.a, ws.g
        L0, L1, L2 = ws.dims

        def wgrad(name, dims, src, dy):
            co = int(p[name + ".b"].numel())
            B.nmd_conv3d_bwd_weight(c, dims, src, dy, co, p[name + ".dw"], p[name + ".db"])

        def dgrad(name, dims, dy, mask, dx):
            ci, co = p[name + ".wt"].shape[0], p[name + ".b"].numel()
            B.nmd_conv3d_bwd_data(c, dims, dy, int(co), p[name + ".wt"], int(ci), mask, dx)

        wgrad("dec0b", L0, B._src(a["d0a"]), g["d0b"])
        dgrad("dec0b", L0, g["d0b"], a["d0a"], g["d0a"])
        wgrad("dec0a", L0, B._src(a["d1b"], 32, True, a["e0b"], 16), g["d0a"])
        dgrad("dec0a", L0, g["d0a"], None, g["c0"])
        B.nmd_nn_combine(c, L1, 32, a["d1b"], None, 0, 0, 1, g["c0"], 48, 0, g["d1b"])
        wgrad("dec1b", L1, B._src(a["d1a"]), g["d1b"])
        dgrad("dec1b", L1, g["d1b"], a["d1a"], g["d1a"])
        wgrad("dec1a", L1, B._src(a["mb"], 64, True, a["e1b"], 32), g["d1a"])
        dgrad("dec1a", L1, g["d1a"], None, g["c1"])
        B.nmd_nn_combine(c, L2, 64, a["mb"], None, 0, 0, 1, g["c1"], 96, 0, g["mb"])
        wgrad("mid_b", L2, B._src(a["ma"]), g["mb"])
        dgrad("mid_b", L2, g["mb"], a["ma"], g["ma"])
        wgrad("mid_a", L2, B._src(a["p1"]), g["ma"])
        dgrad("mid_a", L2, g["ma"], None, g["p1"])
        B.nmd_nn_combine(c, L1, 32, a["e1b"], g["c1"], 96, 64, 2, g["p1"], 32, 0, g["e1b"])
        wgrad("enc1b", L1, B._src(a["e1a"]), g["e1b"])
        dgrad("enc1b", L1, g["e1b"], a["e1a"], g["e1a"])
        wgrad("enc1a", L1, B._src(a["p0"]), g["e1a"])
        dgrad("enc1a", L1, g["e1a"], None, g["p0"])
        B.nmd_nn_combine(c, L0, 16, a["e0b"], g["c0"], 48, 32, 2, g["p0"], 16, 0, g["e0b"])
        wgrad("enc0b", L0, B._src(a["e0a"]), g["e0b"])
        dgrad("enc0b", L0, g["e0b"], a["e0a"], g["e0a"])
        wgrad("enc0a", L0, B._src(ws.x0), g["e0a"])

    def loss_and_grad(self, ws, events=None, weight_floor=0.0):
        """Forward, loss and backward; the loss stays on the device
        (ws.loss_value(), which synchronises, reads it).  weight_floor > 0
        weights each voxel's squared error by 1/max(target, weight_floor)."""
        self.forward(ws, events)
        B.nmd_nn_head_loss(self.ctx, ws.nvox, ws.a["d0b"], ws.x0, ws.target, self.p["head.w"],
                           self.p["head.b"], ws.g["d0b"], self.hgrad, weight_floor)
        self.backward(ws)

    def adam(self, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8):
        self.step += 1
        c, p, k = self.ctx, self.p, self.step
        for name, ci, co, _ in self.layers:
            B.nmd_nn_adam(c, p[name + ".w"], p[name + ".w.m"], p[name + ".w.v"], p[name + ".dw"],
                          k, lr, beta1, beta2, eps, p[name + ".wb"], p[name + ".wt"], co, ci)
            B.nmd_nn_adam(c, p[name + ".b"], p[name + ".b.m"], p[name + ".b.v"], p[name + ".db"],
                          k, lr, beta1, beta2, eps)
        B.nmd_nn_adam(c, p["head.w"], p["head.w.m"], p["head.w.v"], self.hgrad[:16], k, lr,
                      beta1, beta2, eps)
        B.nmd_nn_adam(c, p["head.b"], p["head.b.m"], p["head.b.v"], self.hgrad[16:17], k, lr,
                      beta1, beta2, eps)

    def train_step(self, ws, lr=1e-3, events=None, weight_floor=0.0):
        self.loss_and_grad(ws, events, weight_floor)
        self.adam(lr)

    def predict(self, ws, out, events=None):
        """Denoised dose (FP64, the units of the input dose) of ws's box,
        written into the full map `out`."""
        self.forward(ws, events)
        B.nmd_nn_head_infer(self.ctx, ws.map_shape, ws.box, ws.a["d0b"], ws.x0, self.p["head.w"],
                            self.p["head.b"], ws.scale, out)


class Workspace:
    """Activations and gradients for one box of d x h x w voxels (each
    divisible by 4) of a map of `map_shape`."""

    def __init__(self, eng, shape, width=16, train=True):
        d, h, w = shape
        if d % 4 or h % 4 or w % 4:
            raise ValueError("box dimensions must be divisible by 4")
        t = eng.torch
        dev = eng.device
        self.t = t
        self.shape = tuple(shape)
        self.dims = ((1, d, h, w), (1, d // 2, h // 2, w // 2), (1, d // 4, h // 4, w // 4))
        self.nvox = d * h * w
        bf = t.bfloat16

        def buf(level, ch):
            _, dd, hh, ww = self.dims[level]
            return t.empty(dd, hh, ww, ch, dtype=bf, device=dev)

        W = width
        self.x0 = buf(0, IN_CH)
        self.target = t.empty(d, h, w, dtype=t.float32, device=dev)
        self.scale = t.ones(2, dtype=t.float64, device=dev)
        self.a = {"e0a": buf(0, W), "e0b": buf(0, W), "p0": buf(1, W), "e1a": buf(1, 2 * W),
                  "e1b": buf(1, 2 * W), "p1": buf(2, 2 * W), "ma": buf(2, 4 * W),
                  "mb": buf(2, 4 * W), "d1a": buf(1, 2 * W), "d1b": buf(1, 2 * W),
                  "d0a": buf(0, W), "d0b": buf(0, W)}
        self.g = {}
        if train:
            self.g = {"d0b": buf(0, W), "d0a": buf(0, W), "c0": buf(0, 3 * W),
                      "d1b": buf(1, 2 * W), "d1a": buf(1, 2 * W), "c1": buf(1, 6 * W),
                      "mb": buf(2, 4 * W), "ma": buf(2, 4 * W), "p1": buf(2, 2 * W),
                      "e1b": buf(1, 2 * W), "e1a": buf(1, 2 * W), "p0": buf(1, W),
                      "e0b": buf(0, W), "e0a": buf(0, W)}
        self.map_shape = None
        self.box = None

    def prepare(self, eng, map_shape, box, dose_lo, density, activity, label, dose_hi=None):
        """Network input (and target, if dose_hi is given) for `box` =
        (z0, y0, x0, d, h, w) of maps of `map_shape` (device tensors)."""
        if tuple(box[3:]) != self.shape:
            raise ValueError("box size differs from the workspace")
        self.map_shape = tuple(map_shape)
        self.box = tuple(int(b) for b in box)
        B.nmd_nn_prepare(eng.ctx, map_shape, box, dose_lo, dose_hi, density, activity, label,
                         self.x0, self.target if dose_hi is not None else None, self.scale)

    def loss_value(self, net):
        """Mean-squared error of the last loss_and_grad (synchronises)."""
        return float(net.hgrad[17].item()) / self.nvox
