"""Pins of the denoiser oracle (oracle/unet.py) against definitions that do
not go through it: the bit-level definition of round-to-nearest-even, a
brute-force convolution, adjoint identities of pooling and up-sampling,
closed forms of Adam, and central finite differences of the whole network."""
import itertools

import numpy as np
import pytest
import torch

from oracle import unet as U

F64 = torch.float64


def _bf16_bits_reference(x):
    """Round float32 to bfloat16 by its bit pattern: add 0x7FFF plus the
    lowest kept bit, then truncate the low 16 bits (finite inputs)."""
    u = np.asarray(x, dtype=np.float32).view(np.uint32).astype(np.uint64)
    lsb = (u >> 16) & 1
    r = ((u + 0x7FFF + lsb) >> 16) << 16
    return r.astype(np.uint32).view(np.float32).astype(np.float64)


def test_bf16_round_to_nearest_even():
    ties = [1 + 2.0 ** -8, 1 + 3 * 2.0 ** -8, -(1 + 2.0 ** -8), 2.0 ** -126 * (1 + 2.0 ** -8),
            3.0 * 2 ** 100 * (1 + 2.0 ** -8), 0.0, -0.0, 1.0, 65504.0]
    rng = np.random.default_rng(1)
    vals = np.concatenate([np.array(ties, dtype=np.float32),
                           (rng.standard_normal(4000) * 10.0 ** rng.uniform(-30, 30, 4000)).astype(np.float32)])
    got = U.bf16(torch.from_numpy(vals)).numpy()
    np.testing.assert_array_equal(got, _bf16_bits_reference(vals))
    # the two ties: 1 + 2^-8 goes down to 1, 1 + 3*2^-8 goes up to 1 + 2^-6
    assert got[0] == 1.0 and got[1] == 1 + 2.0 ** -6


def test_conv3x3_matches_brute_force():
    rng = np.random.default_rng(2)
    n, d, h, w, ci, co = 2, 3, 4, 5, 3, 2
    x = rng.standard_normal((n, d, h, w, ci))
    wt = rng.standard_normal((co, 27, ci))
    b = rng.standard_normal(co)
    got = U.conv3x3(torch.from_numpy(x), torch.from_numpy(wt), torch.from_numpy(b)).numpy()
    ref = np.zeros((n, d, h, w, co))
    for nn, z, y, xx, o in itertools.product(range(n), range(d), range(h), range(w), range(co)):
        acc = b[o]
        for kz, ky, kx in itertools.product(range(3), repeat=3):
            zz, yy, x2 = z + kz - 1, y + ky - 1, xx + kx - 1
            if 0 <= zz < d and 0 <= yy < h and 0 <= x2 < w:
                acc += float(np.dot(x[nn, zz, yy, x2], wt[o, (kz * 3 + ky) * 3 + kx]))
        ref[nn, z, y, xx, o] = acc
    np.testing.assert_allclose(got, ref, rtol=1e-13, atol=1e-13)


def test_conv_backward_data_is_flipped_transposed_conv():
    """<conv(x), g> = <x, conv'(g)> with w'[i,t,o] = w[o,26-t,i]: the zero
    padded correlation's adjoint."""
    rng = np.random.default_rng(3)
    x = torch.from_numpy(rng.standard_normal((1, 4, 5, 6, 3)))
    g = torch.from_numpy(rng.standard_normal((1, 4, 5, 6, 2)))
    w = torch.from_numpy(rng.standard_normal((2, 27, 3)))
    wt = w.flip(1).permute(2, 1, 0).contiguous()
    lhs = (U.conv3x3(x, w) * g).sum().item()
    rhs = (x * U.conv3x3(g, wt)).sum().item()
    assert abs(lhs - rhs) <= 1e-12 * abs(lhs)


def test_pool_and_upsample_are_adjoint():
    rng = np.random.default_rng(4)
    x = torch.from_numpy(rng.standard_normal((2, 4, 6, 8, 3)))
    y = torch.from_numpy(rng.standard_normal((2, 2, 3, 4, 3)))
    lhs = (U.avg_pool2(x) * y).sum().item()
    rhs = (x * U.upsample2(y)).sum().item() / 8
    assert abs(lhs - rhs) <= 1e-13 * max(1.0, abs(lhs))
    assert torch.equal(U.avg_pool2(U.upsample2(y)), y)
    assert torch.equal(U.upsample2(y)[:, 1::2, 0::2, 1::2], y)


def test_adam_first_step_and_constant_gradient_closed_forms():
    rng = np.random.default_rng(5)
    theta = torch.from_numpy(rng.standard_normal(500))
    g = torch.from_numpy(rng.standard_normal(500) * 10.0 ** rng.uniform(-6, 2, 500))
    m = torch.zeros(500, dtype=F64)
    v = torch.zeros(500, dtype=F64)
    lr, eps = 1e-3, 1e-8
    expect = -lr * g / (g.abs() + eps)
    th = theta
    for step in range(1, 6):
        # bias correction makes m-hat = g and v-hat = g^2 exactly for a constant g
        new, m, v = U.adam_step(th, m, v, g, step, lr=lr, eps=eps)
        np.testing.assert_allclose((new - th).numpy(), expect.numpy(), rtol=1e-9, atol=1e-15)
        th = new


def test_untrained_network_returns_its_input_dose():
    rng = np.random.default_rng(6)
    x0 = torch.from_numpy(np.abs(rng.standard_normal((1, 8, 12, 16, 3))))
    p = U.init_params(width=4, seed=1)
    pred = U.forward(p, x0)
    assert torch.equal(pred, U.bf16(x0)[..., 0])


@pytest.mark.parametrize("bf16_storage", [False])
def test_unet_gradients_match_finite_differences(bf16_storage):
    rng = np.random.default_rng(7)
    x0 = torch.from_numpy(np.abs(rng.standard_normal((1, 8, 8, 8, 3))))
    tgt = torch.from_numpy(np.abs(rng.standard_normal((1, 8, 8, 8))))
    p = U.init_params(width=4, seed=2, dtype=F64)
    for k in p:  # non-zero head and biases so that every path carries gradient
        if k.endswith(".b") or k.startswith("head"):
            p[k] = torch.from_numpy(rng.standard_normal(p[k].shape) * 0.3)
    loss, grads = U.loss_and_grads(p, x0, tgt, bf16_storage=bf16_storage)
    h = 1e-6
    pick = np.random.default_rng(8)
    for k, t in p.items():
        flat = t.reshape(-1)
        for idx in pick.choice(flat.numel(), size=min(3, flat.numel()), replace=False):
            plus = {kk: vv.clone() for kk, vv in p.items()}
            minus = {kk: vv.clone() for kk, vv in p.items()}
            plus[k].reshape(-1)[idx] += h
            minus[k].reshape(-1)[idx] -= h
            fd = (U.mse(U.forward(plus, x0, False), tgt) - U.mse(U.forward(minus, x0, False), tgt)).item() / (2 * h)
            an = grads[k].reshape(-1)[idx].item()
            assert abs(fd - an) <= 1e-6 * max(abs(an), 1e-4), (k, idx, fd, an)


def test_bf16_storage_changes_gradients_at_the_bf16_scale():
    rng = np.random.default_rng(9)
    x0 = torch.from_numpy(np.abs(rng.standard_normal((1, 8, 8, 12, 3))))
    tgt = torch.from_numpy(np.abs(rng.standard_normal((1, 8, 8, 12))))
    p = U.init_params(width=4, seed=3)
    p["head.w"] = torch.full((4,), 0.5)
    _, g_exact = U.loss_and_grads(p, x0, tgt, bf16_storage=False)
    _, g_bf = U.loss_and_grads(p, x0, tgt, bf16_storage=True)
    for k in g_exact:
        a, b = g_exact[k], g_bf[k]
        if a.abs().sum() == 0:
            continue
        rel = ((a - b).norm() / a.norm()).item()
        # a few 2^-9 relative roundings per stored tensor; the bottleneck of
        # an 8x8x12 input has 12 voxels, so its sums average little of it out
        assert 0 < rel < 0.15, (k, rel)


def test_normalise_sets_body_means_to_one():
    rng = np.random.default_rng(10)
    lab = rng.integers(0, 3, (6, 7, 8)).astype(np.uint8)
    dose = rng.uniform(0, 5, (6, 7, 8))
    act = rng.uniform(0, 2, (6, 7, 8)).astype(np.float32)
    rho = np.full((6, 7, 8), 1.85, np.float32)
    x, s = U.normalise(dose, rho, act, lab)
    body = torch.from_numpy(lab > 0)
    assert abs(x[0, ..., 0][body].mean().item() - 1) < 1e-13
    assert abs(x[0, ..., 2][body].mean().item() - 1) < 1e-13
    assert torch.allclose(x[0, ..., 1], torch.full((6, 7, 8), float(np.float32(1.85)) / 1.85, dtype=F64))
    assert abs(s - dose[lab > 0].mean()) < 1e-13 * s


def test_weighted_loss_reduces_to_the_plain_one():
    """w = 1/max(t, floor): a floor above every target gives mse/floor; a
    floor below every target gives the mean of (p - t)^2 / t."""
    rng = np.random.default_rng(11)
    p = torch.from_numpy(rng.uniform(0, 2, 1000))
    t = torch.from_numpy(rng.uniform(0.5, 1.5, 1000))
    assert abs(U.mse(p, t, 2.0).item() - U.mse(p, t).item() / 2.0) <= 1e-15
    assert abs(U.mse(p, t, 0.1).item() - (((p - t) ** 2) / t).mean().item()) <= 1e-15
