/*
 * nmdose_ingest.h -- C ABI of the CT ingestion of the dosimetry engine.
 *
 * Section 2.1 builds the phantom from the patient's CT: each voxel's HU
 * value gives its mass density through an HU-to-density curve and one of
 * four materials (water, dry air, compact bone, lung).  Section 2.2
 * resamples the CT onto the PET grid, which is the grid the dose is scored
 * on; the PET values (Bq/mL) on that grid are the activity map of
 * nmd_set_activity, whose sum times the voxel volume is A(t_s) of Eq. 1.
 * The paper cites its curve (Schneider et al. 2000) without giving it, so the
 * curve, the material thresholds and the density levels are the caller's.
 *
 * Conventions (in addition to those of nmdose.h)
 *   A grid has n = (nx, ny, nz) voxels of spacing_mm (x, y, z); origin_mm is
 *   the outer corner of voxel (0, 0, 0), so voxel (i, j, k) is centred at
 *   origin + ((i, j, k) + 1/2) * spacing.  Volumes are C order [nz][ny][nx]
 *   (x fastest), float32, on the device.
 *   Every decision that picks an integer (inside or outside, interpolation
 *   cell, curve segment, material, density level) is taken in float32 with
 *   each operation rounded on its own (no fused multiply-add).
 *   Calls are asynchronous on the context stream and return a status; all
 *   array pointers are device pointers, struct pointers are host pointers.
 */
#ifndef NMDOSE_INGEST_H
#define NMDOSE_INGEST_H

#include <stdint.h>

#include "nmdose.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef struct {
  int32_t n[3];         /* nx, ny, nz: 1 .. 4096 each */
  float spacing_mm[3];  /* > 0 */
  float origin_mm[3];   /* finite */
} nmd_grid;

/* CT onto the dose grid (Section 2.2): dst (float [nz][ny][nx] of dst_grid)
 * = trilinear interpolation of src (float [nz][ny][nx] of src_grid) at each
 * destination voxel centre.  Along each axis the centre's source index is
 * u = (o_dst + (i + 1/2) s_dst - o_src) / s_src - 1/2; a centre with
 * u < -1/2 or u > n_src - 1/2 on any axis lies outside the source volume and
 * gets `fill` (for a CT, -1000 HU: air); inside, u is clamped to
 * [0, n_src - 1] (constant extrapolation over the half-voxel border) and the
 * eight neighbouring source voxels are weighted by their distances.  src and
 * dst must not overlap.  NMD_E_INVALID for bad grids or pointers. */
nmd_status nmd_resample_linear(nmd_ctx *ctx, const float *src, const nmd_grid *src_grid,
                               const nmd_grid *dst_grid, float fill, float *dst);

#define NMD_CT_MAX_NODES 32
#define NMD_CT_MAX_MATERIALS 8

/* HU-to-density curve, material thresholds and density levels. */
typedef struct {
  int32_t n_nodes;                             /* 2 .. NMD_CT_MAX_NODES */
  float hu[NMD_CT_MAX_NODES];                  /* strictly increasing */
  float density[NMD_CT_MAX_NODES];             /* g/cm^3, > 0 */
  int32_t n_materials;                         /* 1 .. NMD_CT_MAX_MATERIALS */
  float hu_threshold[NMD_CT_MAX_MATERIALS - 1]; /* strictly increasing, n_materials - 1 */
  float density_min[NMD_CT_MAX_MATERIALS];     /* per material */
  float density_width[NMD_CT_MAX_MATERIALS];   /* > 0 */
  int32_t levels[NMD_CT_MAX_MATERIALS];        /* >= 1; sum <= 256 */
} nmd_ct_table;

/* HU to the density and material grids of nmd_set_phantom (Section 2.1).
 * For each of the n voxels of hu (float; NaN counts as the lowest HU):
 *   density curve: rho = d_j + f (d_{j+1} - d_j), f = (h - h_j) / (h_{j+1} - h_j)
 *     clamped to [0, 1], j = the last node at or below h, clamped to
 *     [0, n_nodes - 2] (the curve is constant beyond its end nodes);
 *   material m = the number of thresholds t with h >= t;
 *   density level k = floor((rho - density_min[m]) / density_width[m])
 *     clamped to [0, levels[m] - 1], and the stored density is the level
 *     centre density_min[m] + (k + 1/2) density_width[m].
 * The levels keep the distinct (material, density) pairs of the phantom
 * within the engine's 256 (sum of levels <= 256).  Outputs: density float[n],
 * material uint8[n].  density may be hu itself (converted in place); any
 * other overlap of the three arrays is NMD_E_INVALID, as are a bad table
 * (including a level centre <= 0) and missing pointers. */
nmd_status nmd_ct_to_phantom(nmd_ctx *ctx, const float *hu, int64_t n, const nmd_ct_table *table,
                             float *density, uint8_t *material);

/* Both steps in one pass: the CT ct_hu (float [nz][ny][nx] of ct_grid) is
 * resampled onto dose_grid as by nmd_resample_linear with fill = -1000 HU,
 * and each resampled value converted as by nmd_ct_to_phantom; only density
 * (float) and material (uint8) are written, [nz][ny][nx] of dose_grid.  The
 * results equal those of the two calls bit for bit; the resampled HU volume
 * never goes to memory. */
nmd_status nmd_ct_ingest(nmd_ctx *ctx, const float *ct_hu, const nmd_grid *ct_grid,
                         const nmd_grid *dose_grid, const nmd_ct_table *table, float *density,
                         uint8_t *material);

#ifdef __cplusplus
}
#endif

#endif
