// CT ingestion (Section 2.1 and 2.2): trilinear resampling onto the dose
// grid and HU to density and material.  The kernels stream their output
// once (one thread per output voxel, x fastest, so writes coalesce and the
// source gathers of neighbouring threads share cache lines).
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include "../../include/nmdose_ingest.h"
#include "nmd_internal.hpp"

namespace nmd {
namespace {

// Per-axis mapping of destination voxels to source cells, in float32 with
// every operation rounded on its own.
struct Axis {
  float o_d, s_d, o_s, s_s;
  int32_t n_s;
};

struct ResampleArgs {
  const float *src;
  float *dst;
  Axis ax[3];
  int32_t nd[3];
  float fill;
};

struct Cell {
  int32_t i0, i1;
  float t;
  bool inside;
};

__device__ __forceinline__ Cell axis_cell(const Axis &a, int32_t i) {
#pragma clang fp contract(off)
  Cell c;
  const float p = a.o_d + ((float)i + 0.5f) * a.s_d;
  const float u = (p - a.o_s) / a.s_s - 0.5f;
  c.inside = u >= -0.5f && u <= (float)a.n_s - 0.5f;
  const float uc = fminf(fmaxf(u, 0.0f), (float)(a.n_s - 1));
  int32_t i0 = (int32_t)floorf(uc);
  i0 = min(i0, max(a.n_s - 2, 0));
  c.i0 = i0;
  c.i1 = min(i0 + 1, a.n_s - 1);
  c.t = a.n_s > 1 ? uc - (float)i0 : 0.0f;
  return c;
}

// Value of destination voxel (x, y, z) of a resampling.
__device__ __forceinline__ float resample_at(const ResampleArgs &a, int32_t x, int32_t y,
                                             int32_t z) {
  // no fused multiply-add, so that the fused ingestion reproduces the
  // resampled values bit for bit
#pragma clang fp contract(off)
  const uint64_t sx = a.ax[0].n_s, sxy = sx * (uint64_t)a.ax[1].n_s;
  const Cell cx = axis_cell(a.ax[0], x), cy = axis_cell(a.ax[1], y), cz = axis_cell(a.ax[2], z);
  if (!(cx.inside && cy.inside && cz.inside)) return a.fill;
  const float *p0 = a.src + cz.i0 * sxy, *p1 = a.src + cz.i1 * sxy;
  const uint64_t r0 = cy.i0 * sx, r1 = cy.i1 * sx;
  const float v000 = p0[r0 + cx.i0], v001 = p0[r0 + cx.i1];
  const float v010 = p0[r1 + cx.i0], v011 = p0[r1 + cx.i1];
  const float v100 = p1[r0 + cx.i0], v101 = p1[r0 + cx.i1];
  const float v110 = p1[r1 + cx.i0], v111 = p1[r1 + cx.i1];
  // weights (1 - t, t): a grid node (t = 0 or 1) returns its value exactly
  const float ux = 1.0f - cx.t, uy = 1.0f - cy.t, uz = 1.0f - cz.t;
  const float a00 = ux * v000 + cx.t * v001, a01 = ux * v010 + cx.t * v011;
  const float a10 = ux * v100 + cx.t * v101, a11 = ux * v110 + cx.t * v111;
  const float b0 = uy * a00 + cy.t * a01, b1 = uy * a10 + cy.t * a11;
  return uz * b0 + cz.t * b1;
}

// HU to (density, material) of one voxel.
__device__ __forceinline__ void ct_convert(float h, const nmd_ct_table &t, float &density,
                                           uint8_t &material) {
#pragma clang fp contract(off)
  if (h != h) h = -INFINITY;  // NaN counts as the lowest HU
  int32_t j = 0;
  while (j < t.n_nodes - 2 && h >= t.hu[j + 1]) ++j;
  float f = (h - t.hu[j]) / (t.hu[j + 1] - t.hu[j]);
  f = fminf(fmaxf(f, 0.0f), 1.0f);
  const float rho = t.density[j] + f * (t.density[j + 1] - t.density[j]);
  int32_t m = 0;
  for (int32_t k = 0; k < t.n_materials - 1; ++k) m += h >= t.hu_threshold[k] ? 1 : 0;
  float kf = floorf((rho - t.density_min[m]) / t.density_width[m]);
  kf = fminf(fmaxf(kf, 0.0f), (float)(t.levels[m] - 1));
  density = t.density_min[m] + (kf + 0.5f) * t.density_width[m];
  material = (uint8_t)m;
}

// Launch grid (ceil(nx / 256), ny, nz): one thread per destination voxel,
// its coordinates straight from the block and thread indices.
__global__ __launch_bounds__(256) void resample_kernel(ResampleArgs a) {
  const int32_t x = blockIdx.x * 256 + threadIdx.x, y = blockIdx.y, z = blockIdx.z;
  if (x >= a.nd[0]) return;
  a.dst[((uint64_t)z * a.nd[1] + y) * a.nd[0] + x] = resample_at(a, x, y, z);
}

__global__ __launch_bounds__(256) void ct_kernel(const float *hu, int64_t n, nmd_ct_table t,
                                                 float *density, uint8_t *material) {
  for (int64_t v = blockIdx.x * 256ll + threadIdx.x; v < n; v += (int64_t)gridDim.x * 256) {
    float d;
    uint8_t m;
    ct_convert(hu[v], t, d, m);
    density[v] = d;
    material[v] = m;
  }
}

// Launch grid as resample_kernel.
__global__ __launch_bounds__(256) void ingest_kernel(ResampleArgs a, nmd_ct_table t,
                                                     float *density, uint8_t *material) {
  const int32_t x = blockIdx.x * 256 + threadIdx.x, y = blockIdx.y, z = blockIdx.z;
  if (x >= a.nd[0]) return;
  const uint64_t v = ((uint64_t)z * a.nd[1] + y) * a.nd[0] + x;
  float d;
  uint8_t m;
  ct_convert(resample_at(a, x, y, z), t, d, m);
  density[v] = d;
  material[v] = m;
}

dim3 voxel_grid(const nmd_grid *g) {
  return dim3((unsigned)((g->n[0] + 255) / 256), (unsigned)g->n[1], (unsigned)g->n[2]);
}

unsigned grid_blocks(uint64_t work) {
  uint64_t b = (work + 255) / 256;
  if (b > 16384) b = 16384;
  return b ? (unsigned)b : 1u;
}

bool grid_ok(const nmd_grid *g) {
  if (!g) return false;
  for (int a = 0; a < 3; ++a) {
    if (g->n[a] < 1 || g->n[a] > 4096) return false;
    if (!(g->spacing_mm[a] > 0.0f) || !isfinite(g->spacing_mm[a])) return false;
    if (!isfinite(g->origin_mm[a])) return false;
  }
  return true;
}

ResampleArgs resample_args(const float *src, const nmd_grid *sg, const nmd_grid *dg, float fill,
                           float *dst) {
  ResampleArgs a;
  a.src = src;
  a.dst = dst;
  a.fill = fill;
  for (int k = 0; k < 3; ++k) {
    a.ax[k] = Axis{dg->origin_mm[k], dg->spacing_mm[k], sg->origin_mm[k], sg->spacing_mm[k],
                   sg->n[k]};
    a.nd[k] = dg->n[k];
  }
  return a;
}

bool overlap(const void *a, uint64_t na, const void *b, uint64_t nb) {
  const uintptr_t a0 = (uintptr_t)a, a1 = a0 + na, b0 = (uintptr_t)b, b1 = b0 + nb;
  return a0 < b1 && b0 < a1;
}

nmd_status check_table(nmd_ctx *c, const nmd_ct_table *t) {
  if (!t || t->n_nodes < 2 || t->n_nodes > NMD_CT_MAX_NODES || t->n_materials < 1 ||
      t->n_materials > NMD_CT_MAX_MATERIALS)
    return ctx_fail(c, NMD_E_INVALID, "bad table sizes");
  for (int k = 0; k < t->n_nodes; ++k) {
    if (!isfinite(t->hu[k]) || !(t->density[k] > 0.0f) || !isfinite(t->density[k]))
      return ctx_fail(c, NMD_E_INVALID, "curve node %d is not finite or its density is not > 0", k);
    if (k && !(t->hu[k] > t->hu[k - 1]))
      return ctx_fail(c, NMD_E_INVALID, "curve HU values must increase");
  }
  int total = 0;
  for (int m = 0; m < t->n_materials; ++m) {
    if (m && (!isfinite(t->hu_threshold[m - 1]) ||
              (m > 1 && !(t->hu_threshold[m - 1] > t->hu_threshold[m - 2]))))
      return ctx_fail(c, NMD_E_INVALID, "material thresholds must be finite and increase");
    if (!isfinite(t->density_min[m]) || !(t->density_width[m] > 0.0f) ||
        !isfinite(t->density_width[m]) || t->levels[m] < 1)
      return ctx_fail(c, NMD_E_INVALID, "bad density levels of material %d", m);
    if (!(t->density_min[m] + 0.5f * t->density_width[m] > 0.0f))
      return ctx_fail(c, NMD_E_INVALID, "material %d has a density level centre <= 0", m);
    total += t->levels[m];
    if (total > 256) return ctx_fail(c, NMD_E_INVALID, "more than 256 density levels in all");
  }
  return NMD_OK;
}

}  // namespace
}  // namespace nmd

using namespace nmd;

extern "C" {

nmd_status nmd_resample_linear(nmd_ctx *c, const float *src, const nmd_grid *sg,
                               const nmd_grid *dg, float fill, float *dst) {
  nmd_status s = ctx_enter(c);
  if (s) return s;
  if (!grid_ok(sg) || !grid_ok(dg)) return ctx_fail(c, NMD_E_INVALID, "bad source or destination grid");
  if (!src || !dst) return ctx_fail(c, NMD_E_INVALID, "source and destination are required");
  const uint64_t ns = (uint64_t)sg->n[0] * sg->n[1] * sg->n[2];
  const uint64_t nd = (uint64_t)dg->n[0] * dg->n[1] * dg->n[2];
  if (overlap(src, ns * 4, dst, nd * 4))
    return ctx_fail(c, NMD_E_INVALID, "source and destination overlap");
  hipLaunchKernelGGL(resample_kernel, voxel_grid(dg), dim3(256), 0, ctx_stream(c),
                     resample_args(src, sg, dg, fill, dst));
  return ctx_hip(c, hipGetLastError(), "resample_kernel");
}

nmd_status nmd_ct_ingest(nmd_ctx *c, const float *ct, const nmd_grid *cg, const nmd_grid *dg,
                         const nmd_ct_table *t, float *density, uint8_t *material) {
  nmd_status s = ctx_enter(c);
  if (s) return s;
  if (!grid_ok(cg) || !grid_ok(dg)) return ctx_fail(c, NMD_E_INVALID, "bad CT or dose grid");
  if (!ct || !density || !material)
    return ctx_fail(c, NMD_E_INVALID, "CT, density and material are required");
  if ((s = check_table(c, t))) return s;
  const uint64_t ns = (uint64_t)cg->n[0] * cg->n[1] * cg->n[2];
  const uint64_t nd = (uint64_t)dg->n[0] * dg->n[1] * dg->n[2];
  if (overlap(ct, ns * 4, density, nd * 4) || overlap(ct, ns * 4, material, nd) ||
      overlap(density, nd * 4, material, nd))
    return ctx_fail(c, NMD_E_INVALID, "CT, density and material overlap");
  hipLaunchKernelGGL(ingest_kernel, voxel_grid(dg), dim3(256), 0, ctx_stream(c),
                     resample_args(ct, cg, dg, -1000.0f, nullptr), *t, density, material);
  return ctx_hip(c, hipGetLastError(), "ingest_kernel");
}

nmd_status nmd_ct_to_phantom(nmd_ctx *c, const float *hu, int64_t n, const nmd_ct_table *t,
                             float *density, uint8_t *material) {
  nmd_status s = ctx_enter(c);
  if (s) return s;
  if (!hu || !density || !material || n < 1)
    return ctx_fail(c, NMD_E_INVALID, "hu, density, material and n >= 1 are required");
  if ((s = check_table(c, t))) return s;
  // each element is read and written by one thread, so density may be hu
  // itself; any other overlap would race
  const uint64_t nb = (uint64_t)n * 4;
  if ((hu != density && overlap(hu, nb, density, nb)) || overlap(hu, nb, material, (uint64_t)n) ||
      overlap(density, nb, material, (uint64_t)n))
    return ctx_fail(c, NMD_E_INVALID, "hu, density and material overlap");
  hipLaunchKernelGGL(ct_kernel, dim3(grid_blocks((uint64_t)n)), dim3(256), 0, ctx_stream(c), hu,
                     n, *t, density, material);
  return ctx_hip(c, hipGetLastError(), "ct_kernel");
}

}  // extern "C"
