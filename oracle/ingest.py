"""CPU oracle for CT/PET ingestion -- TEST INFRASTRUCTURE ONLY.

Section 2.1 builds the phantom from the patient's images: the CT is converted
to mass density and one of four materials through an HU-to-density curve, and
the PET intensity (Bq/mL) becomes the decay density through a linear
conversion.  Section 2.2 resamples the CT onto the PET grid, so dose is
scored on the PET grid.  This module writes out what the ingestion computes:

* ``resample_linear``: trilinear interpolation of a scalar volume in
  physical coordinates onto another grid, with a fill value where the
  destination voxel centre lies outside the source volume;
* ``ct_to_phantom``: HU to density by a piecewise-linear curve, material by
  HU thresholds, and the density rounded to one of a few levels per
  material (the engine holds at most 256 distinct (material, density)
  pairs, so a CT's continuous densities are quantised).

The paper does not give its curve (it cites Schneider et al. 2000); the
curve, thresholds and levels are caller-supplied tables.

Every decision that picks an integer (inside or outside, the cell of the
interpolation, the curve segment, the material, the density level) is taken
in float32 with each operation rounded on its own, as the kernels do.  The
interpolated values are then formed in float64 from those float32 weights
and samples, so a kernel's float32 sums differ from them by rounding only.

A grid is ``dict(n=(nx, ny, nz), spacing=(sx, sy, sz), origin=(ox, oy, oz))``
in mm, ``origin`` being the outer corner of voxel (0, 0, 0); volumes are C
order ``[nz][ny][nx]``.

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this module.  It shares no code with the HIP library.
"""
from __future__ import annotations

import numpy as np

F32 = np.float32


def _axis_coords(a, src, dst):
    """Source index u of every destination voxel centre along axis a
    (0 = x, 1 = y, 2 = z), in float32: u = (o_d + (i + 1/2) s_d - o_s) / s_s - 1/2."""
    n_d = dst["n"][a]
    i = np.arange(n_d, dtype=F32)
    p = F32(dst["origin"][a]) + (i + F32(0.5)) * F32(dst["spacing"][a])
    return (p - F32(src["origin"][a])) / F32(src["spacing"][a]) - F32(0.5)


def _axis_cell(u, n):
    """Inside flag, lower index and weight of the upper neighbour."""
    inside = (u >= F32(-0.5)) & (u <= F32(n) - F32(0.5))
    uc = np.clip(u, F32(0.0), F32(n - 1))
    i0 = np.floor(uc).astype(np.int64)
    i0 = np.clip(i0, 0, max(n - 2, 0))
    t = (uc - i0.astype(F32)).astype(F32) if n > 1 else np.zeros_like(uc)
    i1 = np.minimum(i0 + 1, n - 1)
    return inside, i0, i1, t


def resample_linear(src: np.ndarray, src_grid: dict, dst_grid: dict, fill: float) -> np.ndarray:
    """Trilinear resampling of ``src`` (float32 [nz][ny][nx] on ``src_grid``)
    onto ``dst_grid``.  Inside the source volume (its voxel centres' hull
    widened by half a voxel) the value is the trilinear interpolation of the
    eight surrounding voxel centres, with constant extrapolation over the
    half-voxel border; outside it is ``fill``.  Returns float64."""
    nx, ny, nz = src_grid["n"]
    assert src.shape == (nz, ny, nx)
    cells = [_axis_cell(_axis_coords(a, src_grid, dst_grid), src_grid["n"][a]) for a in range(3)]
    (ix, x0, x1, tx), (iy, y0, y1, ty), (iz, z0, z1, tz) = cells
    v = src.astype(np.float64)
    Z0, Y0, X0 = np.ix_(z0, y0, x0)
    Z1, Y1, X1 = np.ix_(z1, y1, x1)
    wx = tx.astype(np.float64)[None, None, :]
    wy = ty.astype(np.float64)[None, :, None]
    wz = tz.astype(np.float64)[:, None, None]
    out = ((1 - wz) * ((1 - wy) * ((1 - wx) * v[Z0, Y0, X0] + wx * v[Z0, Y0, X1]) +
                       wy * ((1 - wx) * v[Z0, Y1, X0] + wx * v[Z0, Y1, X1])) +
           wz * ((1 - wy) * ((1 - wx) * v[Z1, Y0, X0] + wx * v[Z1, Y0, X1]) +
                 wy * ((1 - wx) * v[Z1, Y1, X0] + wx * v[Z1, Y1, X1])))
    inside = iz[:, None, None] & iy[None, :, None] & ix[None, None, :]
    return np.where(inside, out, float(fill))


def hu_to_density(hu: np.ndarray, table: dict) -> np.ndarray:
    """The piecewise-linear curve: ``table["hu"]`` and ``table["density"]``
    are its nodes (HU increasing; constant beyond the end nodes).  Float32,
    segment j = the last node at or below the HU; a NaN HU counts as the
    lowest HU."""
    h = np.asarray(hu, dtype=F32)
    h = np.where(np.isnan(h), F32(-np.inf), h)
    xs = np.asarray(table["hu"], dtype=F32)
    ys = np.asarray(table["density"], dtype=F32)
    K = len(xs)
    j = np.clip(np.searchsorted(xs, h, side="right") - 1, 0, K - 2)
    f = (h - xs[j]) / (xs[j + 1] - xs[j])
    f = np.clip(f, F32(0.0), F32(1.0)).astype(F32)
    return (ys[j] + f * (ys[j + 1] - ys[j])).astype(F32)


def ct_to_phantom(hu: np.ndarray, table: dict):
    """HU (float32, any shape) to (density float32, material uint8).

    ``table``: the curve of ``hu_to_density``; ``threshold`` -- increasing HU
    values, material m for threshold[m-1] <= HU < threshold[m]; and per
    material ``density_min``, ``density_width``, ``levels`` -- density level k
    covers [min + k w, min + (k+1) w) and stands for its centre
    min + (k + 1/2) w, with k clamped to [0, levels - 1].  A NaN HU counts as
    the lowest HU."""
    h = np.asarray(hu, dtype=F32)
    h = np.where(np.isnan(h), F32(-np.inf), h)
    rho = hu_to_density(h, table)
    thr = np.asarray(table["threshold"], dtype=F32)
    mat = np.zeros(h.shape, dtype=np.uint8)
    for t in thr:
        mat += (h >= t).astype(np.uint8)
    dmin = np.asarray(table["density_min"], dtype=F32)[mat]
    w = np.asarray(table["density_width"], dtype=F32)[mat]
    lv = np.asarray(table["levels"], dtype=np.int64)[mat]
    k = np.floor((rho - dmin) / w)
    k = np.clip(k, 0, lv - 1).astype(np.int64)
    dens = (dmin + (k.astype(F32) + F32(0.5)) * w).astype(F32)
    return dens, mat
