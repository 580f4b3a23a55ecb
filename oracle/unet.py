"""CPU oracle for the learned denoiser -- TEST INFRASTRUCTURE ONLY.

The denoiser is not part of the paper: it is the learned stage added on top
of the Monte Carlo of Section 2 (a 3D U-Net that maps a low-history dose map
plus density and activity to the high-history dose map).  This module writes
out, in plain PyTorch CPU FP64, what that network computes:

* a 3x3x3 cross-correlation with zero padding 1 and a per-channel bias;
* ReLU; a 2x2x2 average pool; a x2 nearest-neighbour up-sample; channel
  concatenation; a 1x1x1 head added to the input dose channel (residual);
* the mean-squared-error loss and its gradients (torch autograd, FP64);
* one Adam step (Kingma and Ba 2015, Algorithm 1, with bias correction).

Tensors are channels-last, ``[N][D][H][W][C]`` (C fastest).  A conv weight is
``[C_out][27][C_in]`` with tap ``t = (kz*3 + ky)*3 + kx`` and offset
``(kz-1, ky-1, kx-1)``.

Mixed precision is part of the definition: with ``bf16=True`` the oracle
rounds to bfloat16 (round to nearest, ties to even) at exactly the points
where the network stores a tensor in BF16 -- the input, every activation,
every pooled tensor, the working copy of every weight, and, in the backward
pass, every stored gradient -- and computes everything else exactly in FP64.

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this module.  It shares no code with the HIP library.
"""
from __future__ import annotations

import math

import torch
import torch.nn.functional as F

F64 = torch.float64

# name, input channels (as multiples of the base width; 0 = network input),
# output channels (multiples of the base width), level
ARCH = (
    ("enc0a", "in", 1, 0), ("enc0b", 1, 1, 0),
    ("enc1a", 1, 2, 1), ("enc1b", 2, 2, 1),
    ("mid_a", 2, 4, 2), ("mid_b", 4, 4, 2),
    ("dec1a", 6, 2, 1), ("dec1b", 2, 2, 1),
    ("dec0a", 3, 1, 0), ("dec0b", 1, 1, 0),
)
IN_CHANNELS = 3  # normalised low-history dose, density, activity


def layer_shapes(width: int = 16):
    """(name, C_in, C_out) for the ten 3x3x3 convolutions."""
    out = []
    for name, cin, cout, _ in ARCH:
        out.append((name, IN_CHANNELS if cin == "in" else cin * width, cout * width))
    return out


# ---------------------------------------------------------------- rounding
def bf16(x: torch.Tensor) -> torch.Tensor:
    """Round to the nearest bfloat16, ties to even, returned as FP64."""
    return x.to(torch.float32).to(torch.bfloat16).to(F64)


class _RoundGrad(torch.autograd.Function):
    """Identity forward; rounds the incoming gradient to bfloat16.  Marks a
    point where the backward pass stores a gradient in BF16."""

    @staticmethod
    def forward(ctx, x):
        return x.view_as(x)

    @staticmethod
    def backward(ctx, g):
        return bf16(g)


class _Round(torch.autograd.Function):
    """Rounds to bfloat16 forward; passes the gradient through unchanged."""

    @staticmethod
    def forward(ctx, x):
        return bf16(x)

    @staticmethod
    def backward(ctx, g):
        return g


# ---------------------------------------------------------------- layers
def conv3x3(x: torch.Tensor, w: torch.Tensor, b: torch.Tensor | None = None) -> torch.Tensor:
    """y[n,z,y,x,o] = b[o] + sum_{kz,ky,kx,i} x[n,z+kz-1,y+ky-1,x+kx-1,i] w[o,t,i],
    zero outside the volume."""
    co, taps, ci = w.shape
    assert taps == 27 and x.shape[-1] == ci
    wk = w.reshape(co, 3, 3, 3, ci).permute(0, 4, 1, 2, 3)
    y = F.conv3d(x.permute(0, 4, 1, 2, 3), wk, b, padding=1)
    return y.permute(0, 2, 3, 4, 1)


def avg_pool2(x: torch.Tensor) -> torch.Tensor:
    """Mean over non-overlapping 2x2x2 blocks (every dimension even)."""
    n, d, h, w, c = x.shape
    assert d % 2 == 0 and h % 2 == 0 and w % 2 == 0
    return x.reshape(n, d // 2, 2, h // 2, 2, w // 2, 2, c).mean(dim=(2, 4, 6))


def upsample2(x: torch.Tensor) -> torch.Tensor:
    """Nearest-neighbour x2: out[z,y,x] = in[z//2, y//2, x//2]."""
    return x.repeat_interleave(2, 1).repeat_interleave(2, 2).repeat_interleave(2, 3)


# ---------------------------------------------------------------- network
def init_params(width: int = 16, seed: int = 0, dtype=torch.float32):
    """He-normal conv weights, zero biases, zero head: the untrained network
    returns its input dose channel unchanged."""
    g = torch.Generator().manual_seed(seed)
    p = {}
    for name, ci, co in layer_shapes(width):
        std = math.sqrt(2.0 / (27 * ci))
        p[name + ".w"] = (torch.randn(co, 27, ci, generator=g, dtype=F64) * std).to(dtype)
        p[name + ".b"] = torch.zeros(co, dtype=dtype)
    p["head.w"] = torch.zeros(width, dtype=dtype)
    p["head.b"] = torch.zeros(1, dtype=dtype)
    return p


def forward(params, x0: torch.Tensor, bf16_storage: bool = True, keep=None):
    """U-Net forward.  ``x0`` is ``[N][D][H][W][3]`` (D, H, W divisible by 4).
    Returns the prediction ``[N][D][H][W]`` (the input dose channel plus the
    head) and, if ``keep`` is a dict, stores every intermediate in it."""
    rnd = _Round.apply if bf16_storage else (lambda t: t)
    rg = _RoundGrad.apply if bf16_storage else (lambda t: t)

    def w_of(name):
        w = params[name + ".w"].to(F64)
        return bf16(w) if bf16_storage else w

    def conv_relu(name, x):
        pre = rg(conv3x3(x, w_of(name), params[name + ".b"].to(F64)))
        y = rnd(torch.relu(pre))
        if keep is not None:
            keep[name] = y
        return y

    x = rnd(x0.to(F64))
    e0 = conv_relu("enc0b", conv_relu("enc0a", x))
    p0 = rg(rnd(avg_pool2(e0)))
    e1 = conv_relu("enc1b", conv_relu("enc1a", p0))
    p1 = rg(rnd(avg_pool2(e1)))
    m = conv_relu("mid_b", conv_relu("mid_a", p1))
    c1 = rg(torch.cat([upsample2(m), e1], dim=-1))
    d1 = conv_relu("dec1b", conv_relu("dec1a", c1))
    c0 = rg(torch.cat([upsample2(d1), e0], dim=-1))
    d0 = conv_relu("dec0b", conv_relu("dec0a", c0))
    head = (d0 * params["head.w"].to(F64)).sum(-1) + params["head.b"].to(F64)
    pred = x[..., 0] + head
    if keep is not None:
        keep.update(x=x, p0=p0, p1=p1, c1=c1, c0=c0, head=head)
    return pred


def mse(pred: torch.Tensor, target: torch.Tensor, weight_floor: float = 0.0) -> torch.Tensor:
    """Mean of w (pred - target)^2 with w = 1/max(target, weight_floor) when
    weight_floor > 0 (inverse-variance weighting for noise whose variance
    grows with the dose), else w = 1."""
    t = target.to(F64)
    w = 1.0 / torch.clamp(t, min=weight_floor) if weight_floor > 0 else torch.ones_like(t)
    return (w * (pred - t) ** 2).mean()


def loss_and_grads(params, x0, target, bf16_storage: bool = True, weight_floor: float = 0.0):
    """Loss and d(loss)/d(param) for every parameter (FP64)."""
    leaves = {k: v.detach().to(F64).clone().requires_grad_(True) for k, v in params.items()}
    loss = mse(forward(leaves, x0, bf16_storage), target, weight_floor)
    loss.backward()
    return loss.item(), {k: v.grad for k, v in leaves.items()}


def adam_step(theta, m, v, g, step, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam update (bias-corrected), FP64.  ``step`` counts from 1."""
    theta, m, v, g = (t.to(F64) for t in (theta, m, v, g))
    m = beta1 * m + (1 - beta1) * g
    v = beta2 * v + (1 - beta2) * g * g
    mhat = m / (1 - beta1 ** step)
    vhat = v / (1 - beta2 ** step)
    return theta - lr * mhat / (torch.sqrt(vhat) + eps), m, v


# ---------------------------------------------------------------- inputs
def normalise(dose_lo, density, activity, label):
    """Network input and scale: dose and activity divided by their mean over
    body voxels (label > 0), density divided by 1.85 g/cm3.  Arrays are
    ``[D][H][W]``; returns (x0 ``[1][D][H][W][3]``, dose scale)."""
    body = torch.as_tensor(label) > 0
    d = torch.as_tensor(dose_lo, dtype=F64)
    a = torch.as_tensor(activity, dtype=F64)
    s_d = d[body].mean()
    s_a = a[body].mean()
    x = torch.stack([d / s_d, torch.as_tensor(density, dtype=F64) / 1.85, a / s_a], dim=-1)
    return x[None], s_d.item()
