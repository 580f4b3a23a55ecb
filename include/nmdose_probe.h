/*
 * nmdose_probe.h -- measured hardware ceilings and per-unit instruction
 * probes for the roofline of the transport kernel.
 *
 * The transport of Section 2.1 (Woodcock steps, Compton/photoelectric/
 * Rayleigh events, a history-by-history tally) is bound by instruction issue,
 * gathers and FP64 atomics rather than by a dense contraction.  These entry
 * points measure what the device delivers on each of those paths, so that a
 * roofline fraction can be stated against measured ceilings as well as the
 * nominal ones, and they run one unit of the transport's work per lane on a
 * non-divergent wave, so that hardware counters (SQ_INSTS_VALU per dispatch)
 * give the VALU instructions of each unit.
 *
 * Every call allocates its own device buffers (released before it returns),
 * orders its work on the context stream and synchronises it.  Errors are
 * returned as nmd_status with a message in nmd_last_error.
 */
#ifndef NMDOSE_PROBE_H
#define NMDOSE_PROBE_H

#include <stdint.h>

#include "nmdose.h"

#ifdef __cplusplus
extern "C" {
#endif

/* Ceiling kinds and the unit of the rate they return. */
enum {
  NMD_CEIL_COPY = 0,       /* device copy of `bytes` (float4): bytes read + written per s */
  NMD_CEIL_ATOMIC_F64 = 1, /* FP64 atomic adds at scattered addresses of a `bytes`
                              table (the tally's access pattern): atomics per s */
  NMD_CEIL_GATHER_U16 = 2, /* 2-byte loads at scattered addresses of a `bytes` array
                              (the voxel-record gather of a Woodcock step): loads per s */
  NMD_CEIL_VALU_FMA = 3,   /* FP32 FMA chains: lane-operations per s            */
  NMD_CEIL_MUL64 = 4,      /* 32x32->64-bit multiplies (Philox rounds): lane-ops per s */
  NMD_CEIL_MFMA_BF16 = 5   /* v_mfma_f32_16x16x32_bf16 chains: FLOP per s        */
};

/* Run ceiling `kind` `repeats` times (1..1000) after one untimed launch and
 * return the mean rate (*rate, unit above) and launch time (*ms, may be
 * NULL).  bytes: the buffer size of the copy, atomic and gather kinds, a
 * power of two in [1 MiB, 8 GiB]; ignored by the others. */
nmd_status nmd_probe_ceiling(nmd_ctx *ctx, int32_t kind, uint64_t bytes, uint32_t repeats,
                             double *rate, double *ms);

/* Units of the transport's work (probe kernels unit_kernel<kind>). */
enum {
  NMD_UNIT_LOOP = 0,      /* the probe loop alone (a 32-bit LCG word per iteration) */
  NMD_UNIT_PHILOX = 1,    /* one Philox4x32-10 block                                  */
  NMD_UNIT_UNIFORM = 2,   /* one uniform from a 32-bit word                           */
  NMD_UNIT_STEP = 3,      /* one Woodcock step: flight, inside test, voxel index, record
                             gather, event choice (two uniforms)                       */
  NMD_UNIT_COMPTON = 4,   /* one Klein-Nishina attempt, azimuth, rotation and energy
                             factors (four uniforms)                                   */
  NMD_UNIT_RAYLEIGH = 5,  /* Thomson angle and rotation (two uniforms)                */
  NMD_UNIT_HISTORY = 6,   /* alias decay voxel, position and direction (six uniforms
                             for one Marsaglia attempt; a decay makes 4/pi of them)    */
  NMD_UNIT_MERGED = 7,    /* one merged deposit flushed to the FP64 (S, S2) tally      */
  NMD_UNIT_N = 8
};

/* Launch unit_kernel<kind> with `blocks` workgroups of 256 lanes, each lane
 * doing `iters` units (iters 1..2^20, blocks 1..65536); *ms (may be NULL)
 * receives the launch time.  The unit's VALU instruction count per wave is
 * (SQ_INSTS_VALU of the dispatch - that of NMD_UNIT_LOOP) / (waves * iters),
 * less its uniforms' share. */
nmd_status nmd_probe_unit(nmd_ctx *ctx, int32_t kind, uint32_t iters, uint32_t blocks,
                          double *ms);

/* LDS lane patterns: the byte offset of lane L (lx = L mod 16, g = L / 16)
 * of one 16-byte LDS access, as the convolutions' fragment reads and halo
 * stores make them. */
enum {
  NMD_LDS_CONTIGUOUS = 0,     /* 16 L                                      */
  NMD_LDS_HALO48 = 1,         /* 48 lx + 48 (g / 2) + 16 (g mod 2): a 16-channel
                                 halo read at a 48-byte voxel pitch           */
  NMD_LDS_P48_SAME = 2,       /* 48 lx (the four lane groups read alike)    */
  NMD_LDS_P48_FAR = 3,        /* 48 lx + 768 g                              */
  NMD_LDS_P80_G16 = 4,        /* 80 lx + 16 g                               */
  NMD_LDS_P48_LANE = 5,       /* 48 L                                       */
  NMD_LDS_GROUP_MAJOR = 6,    /* 16 lx + 256 g                              */
  NMD_LDS_P64_G16 = 7,        /* 64 lx + 16 g                               */
  NMD_LDS_HALO32 = 8,         /* 32 lx + 32 (g / 2) + 16 (g mod 2): the same read
                                 at a 32-byte pitch                          */
  NMD_LDS_P48_G16 = 9,        /* 48 lx + 16 g                               */
  NMD_LDS_STORE48 = 10,       /* 48 (L / 2) + 16 (L mod 2): a 16-channel halo
                                 store at a 48-byte pitch                    */
  NMD_LDS_P96_G16 = 11,       /* 96 lx + 16 g                               */
  NMD_LDS_N = 12
};

/* Launch `blocks` workgroups (1..65536) of four waves whose lanes each make
 * `iters` (1..2^16) 16-byte LDS accesses at the offsets of `pattern` (plus a
 * multiple of 4 KiB that varies with the iteration), reads when `write` is 0
 * and writes otherwise; *ms (may be NULL) receives the launch time.  Bank
 * conflicts per access are SQ_LDS_BANK_CONFLICT / SQ_INSTS_LDS of the
 * dispatch. */
nmd_status nmd_probe_lds(nmd_ctx *ctx, int32_t pattern, int32_t write, uint32_t iters,
                         uint32_t blocks, double *ms);

#ifdef __cplusplus
}
#endif
#endif /* NMDOSE_PROBE_H */
