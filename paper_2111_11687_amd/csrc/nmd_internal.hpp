// Internal interface between the host engine (nmd_api.hip) and the device
// kernels (nmd_kernels.hip).  Not part of the public ABI.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/nmdose.h"

namespace nmd {

constexpr int kMaxPhantoms = 64;
constexpr int kMaxPalette = 256;        // u8 voxel records
constexpr int kNGrid = 256;             // energy nodes, 1 keV .. 511 keV
constexpr int kDepCap = 64;             // distinct deposit voxels kept per history
constexpr int kRegDep = 3;              // of which held in registers
constexpr int kLdsDep = 9;              // the next ones in LDS (the rest in global memory)
constexpr int kBlock = 256;             // transport workgroup size (4 waves)
constexpr int kWavesPerBlock = kBlock / 64;
constexpr int kMaxOrganSlots = 256;     // labels 0..255
constexpr int kRecN = 10;               // per-history debug record width
constexpr int kStatN = 16;
// lanes that wait before their phase runs (unless they outnumber the
// flights): interactions, and history ends (the costlier pass)
constexpr uint32_t kPhaseMinInt = 24, kPhaseMinEnd = 40;
constexpr int kFlySteps = 2;              // Woodcock steps per flight pass and photon
constexpr int kOrgCache = 3;              // organ score slots per history, in registers
constexpr uint32_t kMaxPhotonSteps = 1u << 20;  // termination bound per photon
constexpr int kETab = 256;                // nodes of the electron range and inverse-range tables
constexpr int kMaxMaterials = 8;
constexpr float kInnerRho = 0.01f;        // g/cm^3: voxels at least this dense lie in the inner box
constexpr int kPosN = 4096;               // energy intervals of the positron spectrum's CDF
constexpr double kF18T0 = 0.6335;         // MeV, 18F beta+ endpoint kinetic energy
constexpr int kMaxLines = 8;              // gamma lines of an emitter
constexpr float kPosFloor = 0.001f;       // MeV: a positron stops when its range above this runs out
constexpr double kPosTop = 0.64;          // MeV: top of the positron range tables (endpoint 0.6335)

// Workgroups of the transport kernel the compiler must fit on one CU (it
// caps registers accordingly); a build-time tuning knob.
#ifndef NMD_TRANSPORT_MIN_BLOCKS
#define NMD_TRANSPORT_MIN_BLOCKS 3
#endif

// Model constants.
constexpr double kMeC2 = 0.51099895;            // MeV
constexpr double kNA = 6.02214076e23;
constexpr double kRe = 2.8179403262e-13;        // cm
constexpr double kJPerMeV = 1.602176634e-13;
constexpr double kERef = 0.030;                 // MeV, cross-section anchor
constexpr double kZRef = 7.4;
constexpr double kEGridMin = 1.0e-3;            // MeV
constexpr double kEGridRatio = 511.0;
// The wide grid of a phantom whose emitter has a line above 511 keV: the same
// 256 nodes from 1 keV to 1 MeV, in that phantom's own tables (the pair and
// lower lines keep the grid above).  Same first node, so only the spacing
// differs: (kNGrid - 1) / log2(1000).
constexpr double kEGridRatioW = 1000.0;
constexpr float kInvDl2W = (float)(255.0 / 9.965784284662087);
constexpr double kLineMax = 1.0;  // MeV, the emitter lines the wide grid holds
constexpr float kE0 = 0.511f;                   // annihilation photon energy
constexpr float kKappa = 1.0f + 1.0f / 16384.0f;  // majorant inflation

// Static per-phantom descriptor (device array indexed by phantom id).
struct PhantomDesc {
  const uint16_t *rec;       // per voxel: palette index | organ label << 8
  const uint4 *alias;        // {prob bits, voxel, alias voxel, 0}; voxels as x | y<<10 | z<<20
  double2 *tally;            // (S, S2) per voxel
  double2 *organ;            // (O, O2) per label slot
  double *ledger;            // [6]
  unsigned long long *stats; // [kStatN]
  const float *ln2_major;    // [kNGrid] log2 of majorant nodes, cm^-1
  const double *organ_w;     // [n_org+1] c / (V[cm^3] 1e-3 N_o), J/MeV per kg*(g/cm^3)
  unsigned long long *n_done;  // decays run since the last reset (next history id)
  int32_t nx, ny, nz, n_org;
  float fnx, fny, fnz;
  float dx, dy, dz, inv_dx, inv_dy, inv_dz;
  uint32_t n_alias;
  uint32_t pid;
  // Compton electrons above e_cut (MeV; 0 = every electron deposited on the
  // spot) walk straight ahead through the grid: per material slot s the
  // CSDA range above the cutoff R_s(T) (g/cm^2) on the nodes
  // T_i = e_cut + i / e_inv_dt, and its inverse T_s(R) on R_j = j / inv_dr_s
  // Woodcock majorants by region (region tracking): inside the inner box
  // (the bounding box of every voxel at least kInnerRho dense; voxel units
  // [b0, b1), and in cm) the phantom's majorant, elsewhere in the grid (only
  // thinner voxels) out_ratio times it, the smallest ratio that bounds those
  // voxels at every energy.  out_ratio is 0 under global tracking, and when
  // the box is the whole grid.
  float b0[3], b1[3];
  float bcm0[3], bcm1[3];
  float out_ratio, inv_out_ratio;
  const float *e_tab;    // [kMaxMaterials][2][kETab]: R_s(T_i), then T_s(R_j)
  const float *e_inv_dr; // [kMaxMaterials]
  const uint8_t *e_slot; // [kMaxPalette]: palette index -> material slot
  float e_cut;
  float e_inv_dt;
  // 18F positrons (p_on): the kinetic-energy CDF on T_i = kF18T0 i / kPosN
  // and its guide table (p_guide[k] = the last i with p_cdf[i] <= k / kPosN);
  // range tables as e_tab from kPosFloor on the nodes kPosFloor + i /
  // p_inv_dt; the Rayleigh scale of the pair's tilt (rad, 0: back to back)
  int32_t p_on;
  float p_inv_dt;
  float noncol_sigma;
  const double *p_cdf;     // [kPosN + 1]
  const int32_t *p_guide;  // [kPosN]
  const float *p_tab;    // [kMaxMaterials][2][kETab]
  const float *p_inv_dr; // [kMaxMaterials]
  const uint8_t *p_slot; // [kMaxPalette]: palette index -> material slot
  // gamma + beta emitter (em_on): line i of energy em_e[i] (MeV) when the
  // decay's uniform u < em_cum[i] (cumulative yields, in FP64 as summed on
  // the host), no photon above em_cum[em_n - 1]; em_beta (MeV) left in the
  // decay voxel
  int32_t em_on, em_n;
  double em_cum[kMaxLines];
  float em_e[kMaxLines];
  float em_beta;
  // 1: ln2_major holds the wide grid's majorant nodes followed by its
  // Klein-Nishina nodes, and energies use the wide grid's spacing
  int32_t wide;
};

// Per-run fields of one phantom of a launch.
struct RunSlot {
  unsigned long long n_hist;  // histories in this run
  unsigned long long chunk0;  // first work-queue chunk of this phantom
  int32_t id;                 // index into the descriptor array
  int32_t pad;
};

// Phantom ids of one run (for the counter update after it).
struct RunIds {
  int32_t n;
  int32_t id[kMaxPhantoms];
};

struct RunParams {
  const PhantomDesc *desc;   // device [kMaxPhantoms]
  int32_t n_ph;
  uint32_t chunk;
  unsigned long long total_chunks;
  unsigned long long *queue; // [0] claim counter, [1] abort flag
  unsigned long long abort_after;
  uint32_t seed_lo, seed_hi;
  uint32_t nph;              // photons per decay
  uint32_t mask;
  uint32_t max_real;
  float cutoff;
  uint32_t source_kind;
  float po[3], pd[3];
  const float4 *palette;     // [n_pal] (cC, cPE, cR, rho)
  int32_t n_pal;
  const float *ln2_kn;       // [kNGrid] log2(N_A sigma_KN(E_i))
  float l2emin, inv_dl2;     // grid coordinate t = (log2 E - l2emin) * inv_dl2
  uint32_t *dep_v;           // overflow deposit lists [kDepCap][n_lanes]: voxel
  double *dep_e;             //   energy
  uint32_t *dep_r;           //   voxel record
  int32_t n_slots;           // largest n_org + 1 of the launch's phantoms
  // unused: with this slot the fields after it sit 8 bytes further into the
  // argument block, and the compiler then fits the transport kernel in 167
  // VGPRs without spills (without it, 36 bytes of scratch per lane and 0.8 %
  // slower, measured)
  uint32_t spare;
  uint32_t n_lanes;
  double *hist_rec;          // debug [n_hist][kRecN] or nullptr
  RunSlot slot[kMaxPhantoms];
};

// regions: the instantiation with region majorants, needed when a phantom of
// the run has a nonzero out_ratio
hipError_t launch_transport(const RunParams &p, int grid, bool debug, bool electrons,
                            bool regions, hipStream_t s);
int transport_occupancy_blocks_per_cu(bool debug, bool electrons, bool regions, int n_slots);
size_t transport_dyn_lds_bytes(int n_slots);
hipError_t launch_finalize(const uint16_t *rec, const float4 *palette, const double2 *tally,
                           uint64_t nvox, const unsigned long long *n_decays,
                           double voxel_kg_per_rho,
                           double a_ts, double *rate, double *rel, hipStream_t s);
hipError_t launch_organ_reduce(const uint16_t *rec, const float4 *palette,
                               const double2 *tally, uint64_t nvox, int n_org,
                               const unsigned long long *n_decays,
                               double voxel_kg_per_rho, double a_ts,
                               double *acc /* [(n_org+1)*2] */, hipStream_t s);
hipError_t launch_debug_sample(int kind, float e_mev, uint64_t n, uint32_t seed_lo,
                               uint32_t seed_hi, double *out, hipStream_t s);
hipError_t launch_debug_source(const uint4 *alias, uint32_t n_alias, uint32_t pid, uint64_t n,
                               uint32_t seed_lo, uint32_t seed_hi, uint32_t nx, uint32_t ny,
                               uint32_t *out, hipStream_t s);
hipError_t launch_debug_xs(const float4 *palette, const uint8_t *used, int n_pal,
                           const float *ln2_kn, const float *ln2_major, uint64_t n,
                           const float *energies, float *out, float l2emin, float inv_dl2,
                           hipStream_t s);
hipError_t launch_zero_bytes(void *p, uint64_t nbytes, hipStream_t s);
hipError_t launch_advance(const PhantomDesc *desc, const RunIds &ids, unsigned long long n,
                          hipStream_t s);
hipError_t launch_set_u64(unsigned long long *p, unsigned long long v, hipStream_t s);
// dst[i] += src[i], i < n
hipError_t launch_add_f64(double *dst, const double *src, uint64_t n, hipStream_t s);
// run counters: dst[i] += src[i], except the largest-list slot, which takes the max
hipError_t launch_add_stats(unsigned long long *dst, const unsigned long long *src,
                            hipStream_t s);
hipError_t launch_map_organ_reduce(const uint16_t *rec, uint64_t nvox, int n_org,
                                   const double *map, double *acc /* [n_org+1] */,
                                   hipStream_t s);

// Services of the context used by the denoiser entry points (nmd_nn.hip).
nmd_status ctx_enter(nmd_ctx *c);  // validates the context and makes its device current
nmd_status ctx_fail(nmd_ctx *c, nmd_status s, const char *fmt, ...);
nmd_status ctx_hip(nmd_ctx *c, hipError_t e, const char *what);  // NMD_OK on hipSuccess
hipStream_t ctx_stream(const nmd_ctx *c);
// A context-owned device workspace of at least `bytes`, reused across calls
// (stream-ordered: only work on the context stream may use it).
nmd_status ctx_scratch(nmd_ctx *c, size_t bytes, void **p);

}  // namespace nmd
