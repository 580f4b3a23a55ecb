"""Pins of the ingestion oracle (oracle/ingest.py), CPU only.

Trilinear resampling is pinned by identities (same grid; an exactly
representable shift), by its exactness on linear fields, and by
scipy.ndimage.map_coordinates (order 1) inside the source volume; the HU
conversion by its nodes, segment midpoints, thresholds and level bounds."""
import numpy as np
import pytest
from scipy import ndimage

from oracle import ingest as I

F32 = np.float32


def grid(n, spacing, origin=(0.0, 0.0, 0.0)):
    return dict(n=tuple(n), spacing=tuple(spacing), origin=tuple(origin))


def test_same_grid_is_identity():
    rng = np.random.default_rng(1)
    g = grid((7, 5, 4), (0.5, 2.0, 1.0))
    v = rng.normal(size=(4, 5, 7)).astype(F32)
    out = I.resample_linear(v, g, g, fill=-7.0)
    assert np.array_equal(out, v.astype(np.float64))


def test_half_voxel_shift_averages_neighbours():
    # destination centres midway between source centres along x (exact in f32)
    rng = np.random.default_rng(2)
    src = grid((8, 3, 3), (1.0, 1.0, 1.0))
    dst = grid((7, 3, 3), (1.0, 1.0, 1.0), origin=(0.5, 0.0, 0.0))
    v = rng.normal(size=(3, 3, 8)).astype(F32)
    out = I.resample_linear(v, src, dst, fill=0.0)
    want = 0.5 * (v[:, :, :-1].astype(np.float64) + v[:, :, 1:])
    assert np.allclose(out, want, rtol=0, atol=1e-12)


def test_linear_field_is_reproduced():
    a, b, c, d = 3.0, 0.25, -0.5, 0.125
    src = grid((20, 18, 16), (1.25, 1.5, 2.0), origin=(-3.0, 1.0, 0.5))
    dst = grid((11, 9, 7), (2.1, 2.7, 4.1), origin=(-1.1, 3.3, 2.9))

    def f(g):
        c3 = [np.float64(g["origin"][k]) + (np.arange(g["n"][k]) + 0.5) * g["spacing"][k] for k in range(3)]
        X, Y, Z = c3
        return (a + b * X[None, None, :] + c * Y[None, :, None] + d * Z[:, None, None])

    v = f(src).astype(np.float64)
    out = I.resample_linear(v.astype(F32), src, dst, fill=np.nan)
    want = f(dst)
    # every destination centre lies inside the hull of the source centres
    assert not np.isnan(out).any()
    assert np.allclose(out, want, rtol=0, atol=2e-5)


@pytest.mark.parametrize("seed", [3, 4, 5])
def test_matches_scipy_map_coordinates(seed):
    rng = np.random.default_rng(seed)
    n = tuple(int(x) for x in rng.integers(4, 12, size=3))
    src = grid(n, tuple(rng.uniform(0.5, 3.0, size=3)), tuple(rng.uniform(-5, 5, size=3)))
    ext = [src["n"][k] * src["spacing"][k] for k in range(3)]
    nd = tuple(int(x) for x in rng.integers(3, 10, size=3))
    sp = tuple(ext[k] / nd[k] * rng.uniform(0.5, 0.9) for k in range(3))
    org = tuple(src["origin"][k] + rng.uniform(0.0, 0.1) * ext[k] for k in range(3))
    dst = grid(nd, sp, org)
    v = rng.normal(size=(n[2], n[1], n[0])).astype(F32)
    out = I.resample_linear(v, src, dst, fill=np.nan)
    coords = []
    for k in range(3):
        u = (dst["origin"][k] + (np.arange(nd[k]) + 0.5) * dst["spacing"][k] - src["origin"][k]) / src["spacing"][k] - 0.5
        coords.append(u)
    Z, Y, X = np.meshgrid(coords[2], coords[1], coords[0], indexing="ij")
    ref = ndimage.map_coordinates(v.astype(np.float64), [Z, Y, X], order=1, mode="nearest")
    inside = ~np.isnan(out)
    assert inside.mean() > 0.5
    assert np.allclose(out[inside], ref[inside], rtol=0, atol=1e-5)


def test_outside_is_fill_and_border_is_clamped():
    src = grid((4, 4, 4), (1.0, 1.0, 1.0))  # spans [0, 4) mm on each axis
    v = np.arange(64, dtype=F32).reshape(4, 4, 4)
    # x centres -0.25 (outside), 0.25 (half-voxel border: clamped), 0.75
    dst = grid((3, 1, 1), (0.5, 1.0, 1.0), origin=(-0.5, 1.0, 1.0))
    out = I.resample_linear(v, src, dst, fill=-99.0)
    assert out[0, 0, 0] == -99.0
    assert out[0, 0, 1] == v[1, 1, 0]
    assert np.isclose(out[0, 0, 2], 0.75 * v[1, 1, 0] + 0.25 * v[1, 1, 1])
    # x centres 3.75 (border: clamped) and 4.25 (outside)
    dst2 = grid((2, 1, 1), (0.5, 1.0, 1.0), origin=(3.5, 1.0, 1.0))
    out2 = I.resample_linear(v, src, dst2, fill=-99.0)
    assert out2[0, 0, 0] == v[1, 1, 3] and out2[0, 0, 1] == -99.0


TABLE = dict(hu=[-1000.0, -740.0, 0.0, 1100.0, 3000.0],
             density=[0.0012, 0.26, 1.0, 1.85, 2.9],
             threshold=[-950.0, -200.0, 300.0],
             density_min=[0.0, 0.05, 0.8, 1.1],
             density_width=[0.05 / 8, 0.75 / 32, 0.4 / 64, 1.8 / 64],
             levels=[8, 32, 64, 64])


def test_hu_nodes_midpoints_and_clamping():
    xs = np.array(TABLE["hu"], dtype=F32)
    ys = np.array(TABLE["density"], dtype=F32)
    # every node but the last is the start of its segment: exact
    assert np.array_equal(I.hu_to_density(xs[:-1], TABLE), ys[:-1])
    assert np.isclose(I.hu_to_density(xs[-1:], TABLE)[0], ys[-1], rtol=1e-6)
    mid = 0.5 * (xs[:-1] + xs[1:])
    assert np.allclose(I.hu_to_density(mid, TABLE), 0.5 * (ys[:-1] + ys[1:]), rtol=1e-6)
    d = I.hu_to_density(np.array([-5000.0, 9000.0, -np.inf, np.inf, np.nan], dtype=F32), TABLE)
    assert np.allclose(d, [ys[0], ys[-1], ys[0], ys[-1], ys[0]], rtol=1e-6)


def test_materials_follow_thresholds():
    h = np.array([-2000, -951, -950, -201, -200, 299, 300, 5000, np.nan], dtype=F32)
    _, m = I.ct_to_phantom(h, TABLE)
    assert m.tolist() == [0, 0, 1, 1, 2, 2, 3, 3, 0]


def test_density_levels():
    rng = np.random.default_rng(7)
    h = rng.uniform(-1100, 3200, size=20000).astype(F32)
    d, m = I.ct_to_phantom(h, TABLE)
    exact = I.hu_to_density(h, TABLE)
    for mm in range(4):
        sel = m == mm
        lo, w, L = TABLE["density_min"][mm], TABLE["density_width"][mm], TABLE["levels"][mm]
        inrange = sel & (exact >= lo) & (exact < lo + L * w)
        assert np.all(np.abs(d[inrange] - exact[inrange]) <= 0.5 * w * (1 + 1e-5))
        levels = np.unique(d[sel])
        assert len(levels) <= L
        k = np.round((levels - lo) / w - 0.5)
        assert np.allclose(lo + (k + 0.5) * w, levels, rtol=1e-6)
