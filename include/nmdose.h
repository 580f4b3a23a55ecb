/*
 * nmdose.h -- C ABI of the MI355X voxel Monte Carlo dosimetry engine.
 *
 * The engine computes the internal-dosimetry quantities of ARCHER-NM
 * (Peng et al., arXiv 2111.11687):
 *   - decays sampled from a PET activity map through a probability density
 *     proportional to the activity concentration (Section 2.1);
 *   - two back-to-back 0.511 MeV annihilation photons per decay with an
 *     isotropic direction drawn by Marsaglia's method (Section 2.1);
 *   - photon transport with Compton scattering (free-electron Klein-Nishina),
 *     the photoelectric effect and a Thomson-shaped Rayleigh term, a 10 keV
 *     photon cutoff, and local deposit of electron energy (Section 2.1);
 *   - a voxel dose tally with history-by-history uncertainty (Section 2.1);
 *   - the dose-rate map of Eq. 1 and the organ mean (Eq. 2) and organ
 *     uncertainty (Eq. 3) of Section 2.4.
 *
 * Conventions
 *   Arrays are C order [nz][ny][nx] with x fastest.  Voxel sizes are given in
 *   mm; internally lengths are cm and energies MeV.  Density is g/cm^3,
 *   activity concentration Bq/mL, dose rate Gy/s.
 *   Pointers documented as "device" must be device memory of the context's
 *   device (for example a torch tensor's data_ptr()); "host" pointers are
 *   ordinary CPU memory.  Input pointers stay owned by the caller and are
 *   only read during the call.  The library copies what it keeps into its
 *   own allocations, released by nmd_destroy (or when a phantom is
 *   re-registered).  Outputs are written into caller buffers.
 *   All device work is ordered on the context stream.  nmd_run_histories and
 *   nmd_get_dose are asynchronous with respect to the host; nmd_set_phantom,
 *   nmd_set_activity, nmd_get_organ_dose and the nmd_get_ledger /
 *   nmd_get_run_stats readers synchronise the stream.
 *   Every call returns a status and never aborts; the message of the last
 *   failure is available from nmd_last_error.  After NMD_E_HIP the context
 *   must be destroyed.  A context is used by one host thread at a time.
 */
#ifndef NMDOSE_H
#define NMDOSE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct nmd_ctx nmd_ctx;
typedef int32_t nmd_status;

enum {
  NMD_OK = 0,
  NMD_E_INVALID = -1,     /* bad argument value                          */
  NMD_E_SHAPE = -2,       /* dimensions out of range or inconsistent      */
  NMD_E_STATE = -3,       /* call out of order (e.g. run before activity) */
  NMD_E_OOM = -4,         /* device allocation failed                     */
  NMD_E_HIP = -5,         /* HIP runtime error; the context is unusable   */
  NMD_E_ABORTED = -6,     /* run stopped by the abort hook                */
  NMD_E_UNSUPPORTED = -7  /* input outside what the library handles       */
};

/* One material: effective atomic number and electron fraction Z/A.  The
 * photoelectric cross section scales as Z^4/E^3 per atom and the Rayleigh
 * term as Z^2/E^2; Compton is Klein-Nishina per electron. */
typedef struct {
  double z_eff;
  double z_over_a;
} nmd_material;

/* Run options (nmd_run_opts_default fills the defaults). */
typedef struct {
  uint32_t photons_per_decay;  /* 2 (annihilation pair) or 1 (point photon source) */
  uint32_t process_mask;       /* bit0 Compton, bit1 photoelectric, bit2 Rayleigh; 7 = all */
  uint32_t max_real_events;    /* per photon; 0 = unlimited; after the limit the photon
                                  is dropped and its energy booked as "discarded"      */
  float photon_cutoff_mev;     /* 0.010 (Section 2.1)                                   */
  uint32_t source_kind;        /* 0 activity map; 1 pencil beam (one photon, fixed
                                  origin and direction, no source draws)               */
  float pencil_origin_cm[3];   /* inside the grid                                      */
  float pencil_dir[3];         /* normalised by the library                            */
  uint32_t chunk;              /* histories per work-queue claim; 0 = tuned default    */
  uint32_t grid_blocks;        /* persistent workgroups; 0 = fill the device           */
  uint32_t abort_after_chunks; /* failure hook: stop after this many claims; 0 = off   */
  double *history_records;     /* device [n_decays][10] or NULL: per-history debug
                                  record (edep, escaped, n_compton, n_pe, n_rayleigh,
                                  n_steps, sum of deposit voxel indices, n distinct
                                  deposit voxels, uniforms drawn, discarded energy)    */
} nmd_run_opts;

/* Ledger slots (MeV) and run-stats slots.  NMD_STAT_LIST_MERGES counts the
 * histories that deposited in more organs than the per-history organ slots
 * hold (three), whose organ scores were merged from the deposit list.
 * NMD_STAT_OVERFLOWS counts deposits of histories whose list of distinct
 * deposit voxels (64) was full: each is scored on its own, so every mean
 * (Eq. 1, Eq. 2) stays exact but the history's square for that voxel and
 * organ is split, which biases the uncertainties low; a nonzero count marks
 * them as approximate.  NMD_STAT_GATHERS counts the voxel records the flight
 * steps read: at least one per step inside the grid, plus the records read
 * ahead for a second step that a real collision or an escape then made
 * unnecessary.  With positrons on (nmd_set_positron), NMD_LEDGER_EMITTED
 * holds the photons' energy plus the positrons' kinetic energy, and
 * NMD_LEDGER_DEP_POSITRON what the positrons lost in the grid.  With an
 * emitter (nmd_set_emitter), NMD_LEDGER_EMITTED holds the emitted photons'
 * energy plus the beta energy, and NMD_LEDGER_DEP_BETA the beta energy. */
enum { NMD_LEDGER_EMITTED = 0, NMD_LEDGER_DEP_COMPTON, NMD_LEDGER_DEP_PE, NMD_LEDGER_DEP_CUTOFF,
       NMD_LEDGER_ESCAPED, NMD_LEDGER_DISCARDED, NMD_LEDGER_DEP_POSITRON, NMD_LEDGER_DEP_BETA,
       NMD_LEDGER_N };
enum { NMD_STAT_HISTORIES = 0, NMD_STAT_PHOTONS, NMD_STAT_STEPS, NMD_STAT_NULLS,
       NMD_STAT_COMPTON, NMD_STAT_PE, NMD_STAT_RAYLEIGH, NMD_STAT_DEPOSITS, NMD_STAT_MERGED,
       NMD_STAT_MAX_MERGED, NMD_STAT_ESCAPES, NMD_STAT_OVERFLOWS, NMD_STAT_CLAIMS,
       NMD_STAT_RNG_BLOCKS, NMD_STAT_LIST_MERGES, NMD_STAT_GATHERS, NMD_STAT_N };

/* ---- context ------------------------------------------------------------ */

/* Create a context on HIP device `device`, ordering work on `hip_stream`
 * (a hipStream_t; NULL = the default stream).  *out receives the context. */
nmd_status nmd_create(nmd_ctx **out, int device, void *hip_stream);
/* Release every library allocation of the context.  NULL is accepted. */
void nmd_destroy(nmd_ctx *ctx);
/* Message of the last failed call on ctx (static text if ctx is NULL). */
const char *nmd_last_error(const nmd_ctx *ctx);
/* Change the stream later calls are ordered on. */
nmd_status nmd_set_stream(nmd_ctx *ctx, void *hip_stream);
/* Fill *opts with the defaults: 2 photons, all processes, 10 keV cutoff,
 * activity source, tuned chunk and grid. */
void nmd_run_opts_default(nmd_run_opts *opts);

/* ---- problem set-up ----------------------------------------------------- */

/* Register (or replace) phantom `phantom_id` (0..63): the CT-derived
 * density and material grid of Section 2.1 plus an optional organ label map
 * (Section 2.3).  density: device float[nvox], finite and > 0;
 * material: device uint8[nvox], < n_materials; organ_label: device
 * uint8[nvox] or NULL, 0 = no organ, 1..n_organs; materials: host
 * [n_materials], n_materials <= 8.  nx, ny <= 1024 and nz <= 4096
 * (NMD_E_UNSUPPORTED beyond).
 * Re-registering an id drops its activity and tallies.  Distinct
 * (material, density) pairs over all phantoms of a context are limited to
 * 256 (NMD_E_UNSUPPORTED beyond).  Synchronises the stream. */
nmd_status nmd_set_phantom(nmd_ctx *ctx, int32_t phantom_id, int32_t nx, int32_t ny, int32_t nz,
                           float dx_mm, float dy_mm, float dz_mm, const float *density,
                           const uint8_t *material, const uint8_t *organ_label,
                           int32_t n_organs, const nmd_material *materials, int32_t n_materials);

/* Set the activity map of a phantom: the decay probability of a voxel is
 * proportional to its activity concentration (the linear conversion of
 * Section 2.1).  activity_bq_ml: device float[nvox], finite, >= 0, not all
 * zero.  total_activity_bq is A(t_s) of Eq. 1; <= 0 means sum(A_v * V_v)
 * with V_v in mL.  Resets the phantom's tallies.  Synchronises the stream. */
nmd_status nmd_set_activity(nmd_ctx *ctx, int32_t phantom_id, const float *activity_bq_ml,
                            double total_activity_bq);

/* Electron transport above a cutoff (Section 2.1 follows electrons down to
 * a 200 keV cutoff).  With cutoff_mev > 0, every Compton electron whose
 * kinetic energy T exceeds it is walked from the interaction point in a
 * straight line along its recoil momentum (E d_in - E' d_out) through the
 * voxel grid, slowing down continuously: in each voxel it loses what the
 * voxel's mass path rho * s takes off its range above the cutoff, the range
 * being the integral of 1/S over [cutoff, T] with S the Bethe collision
 * stopping power (ICRU Report 37 form, Moller term, no density effect, no
 * radiative loss) of the voxel's material; where the range runs out it
 * leaves all it still has, and energy it carries out of the grid is booked
 * as escaped.  Electrons at or below the cutoff, and photoelectrons, are
 * deposited on the spot.  cutoff_mev: 0 (electrons deposited on the spot,
 * the default) or [0.001, 0.3] MeV; mean_excitation_ev: host
 * double[n_materials], the mean excitation energy I of each material of
 * nmd_set_phantom, in (1, 10^4) eV.  The library tabulates each material's
 * range and inverse range on 256 nodes, up to 345 keV (above the Compton
 * electrons of 511 keV photons): with an emitter line above 0.511 MeV on
 * the phantom the call returns NMD_E_UNSUPPORTED.  Resets the phantom's
 * tallies; re-registering the phantom drops the model; checkpoints do not
 * record it.  Synchronises the stream. */
nmd_status nmd_set_electrons(nmd_ctx *ctx, int32_t phantom_id, double cutoff_mev,
                             const double *mean_excitation_ev);

/* Positron physics of 18F (the emitter of Section 2.1; the paper leaves its
 * positron out).  With on = 1 every decay of the activity source emits a
 * positron before its photon pair:
 *   - its kinetic energy from the allowed beta+ spectrum of 18F (Fermi
 *     theory: p W (W0 - W)^2 F(W) in units of the electron's rest energy,
 *     endpoint 633.5 keV, F the non-relativistic Fermi function of a
 *     positron repelled by the 18O nucleus), tabulated by the library;
 *   - an isotropic direction, along which it slows down continuously on a
 *     straight line as the electrons of nmd_set_electrons do (Bethe stopping
 *     power of its material, mean excitation energies mean_excitation_ev),
 *     down to 1 keV; its losses are booked as NMD_LEDGER_DEP_POSITRON and
 *     its kinetic energy as emitted;
 *   - the photon pair is born where it stops; one that leaves the grid
 *     takes the pair with it (both photons escape);
 *   - the second photon leaves back to back with the first, tilted by an
 *     angle whose size is Rayleigh distributed with FWHM noncol_fwhm_deg
 *     (in [0, 5] degrees; 0 keeps the pair exactly back to back) about an
 *     isotropic azimuth.
 * Per decay the draws are: the decay voxel and position, the pair's
 * direction, then one uniform for the kinetic energy, the positron's
 * direction and two uniforms for the tilt.  Pencil-beam runs emit no
 * positron.  on = 0 turns it off (mean_excitation_ev may then be NULL).
 * Not together with nmd_set_emitter (NMD_E_STATE).
 * Independent of nmd_set_electrons: the positron tables run from 1 keV to
 * 640 keV.  Resets the phantom's tallies; re-registering the phantom drops
 * it; checkpoints do not record it; graphs captured before the call refuse
 * to launch.  Errors: NMD_E_STATE (phantom not registered), NMD_E_INVALID
 * (arguments).  Synchronises the stream. */
nmd_status nmd_set_positron(nmd_ctx *ctx, int32_t phantom_id, int32_t on, double noncol_fwhm_deg,
                            const double *mean_excitation_ev);

/* Gamma + beta emitters in place of the annihilation pair (the other
 * radionuclides Section 4 names, 177Lu and 131I).  With n_lines > 0 or
 * beta_mean_mev > 0, every decay of the activity source emits at most one
 * photon: line i, of energy energy_mev[i] in (0.001, 1] MeV, with
 * probability yield[i] per decay
 * (yields >= 0, summing to at most 1), in an isotropic direction; and it
 * leaves beta_mean_mev, the mean beta kinetic energy, in the decay voxel
 * (booked as NMD_LEDGER_DEP_BETA).  Per decay the draws are: the decay
 * voxel and position, one uniform for the line (cumulative yields in line
 * order; none above their sum), then the photon's direction.  n_lines (at
 * most 8) = 0 with beta_mean_mev = 0 returns to the pair source.  Not
 * together with nmd_set_positron (NMD_E_STATE).  Pencil-beam runs are
 * unchanged.  Resets the phantom's tallies; re-registering the phantom drops
 * it; checkpoints do not record it; graphs captured before the call refuse
 * to launch.  A line above 0.511 MeV puts the phantom's cross sections on
 * a wider grid (256 nodes from 1 keV to 1 MeV, in place of 1 to 511 keV)
 * and excludes Compton electron transport (NMD_E_UNSUPPORTED: its range
 * tables end at 345 keV).  energy_mev, yield: host double[n_lines].
 * Errors: NMD_E_STATE, NMD_E_INVALID, NMD_E_UNSUPPORTED.  Synchronises the
 * stream. */
nmd_status nmd_set_emitter(nmd_ctx *ctx, int32_t phantom_id, int32_t n_lines,
                           const double *energy_mev, const double *yield, double beta_mean_mev);

/* Woodcock tracking modes (the free flight of Section 2.1 samples collision
 * points against a majorant of the attenuation, with null collisions making
 * up the difference).
 *   NMD_TRACK_GLOBAL  -- one majorant for the whole phantom (the default).
 *   NMD_TRACK_REGIONS -- a majorant by region, not in the paper: the
 *     phantom's inside the inner box, the bounding box of every voxel at
 *     least 0.01 g/cm^3 dense, and a smaller one in the thinner voxels
 *     around it (air), the least multiple of the first that bounds them at
 *     every energy node.  Free flight is memoryless, so a step's optical
 *     depth is spent region by region along the ray; both modes sample the
 *     same model, with fewer null collisions here where the phantom sits in
 *     air.  Each mode draws its own random numbers, so runs of the two modes
 *     differ history by history and agree in distribution; the oracle's
 *     region mode replays this one.
 * The mode selects a separate instantiation of the transport kernel; a
 * batched run that holds a phantom in region mode runs them all in it
 * (phantoms in global mode, and phantoms whose box is the whole grid, see
 * one region there and draw as under NMD_TRACK_GLOBAL).  The tallies are
 * kept; graphs captured before the change refuse to launch (NMD_E_STATE);
 * re-registering the phantom returns it to NMD_TRACK_GLOBAL; checkpoints do
 * not record the mode.  Errors: NMD_E_STATE (phantom not registered),
 * NMD_E_INVALID (mode).  Synchronises the stream. */
enum { NMD_TRACK_GLOBAL = 0, NMD_TRACK_REGIONS = 1 };
nmd_status nmd_set_tracking(nmd_ctx *ctx, int32_t phantom_id, int32_t mode);

/* ---- transport ----------------------------------------------------------- */

/* Simulate n_decays histories of phantom `phantom_id`, or of every phantom
 * with an activity map when phantom_id is -1 (one persistent launch over a
 * shared work queue), adding to the phantom's tallies.  Histories are
 * numbered from the number already run since the last reset, and history h
 * of phantom p draws its random numbers from Philox4x32-10 with key = seed
 * and counter = (block, h, p), so repeated calls continue one stream and the
 * result does not depend on the launch shape.  opts NULL = defaults.
 * Asynchronous, except with the abort hook armed (abort_after_chunks > 0):
 * then the run scores into scratch tallies, synchronises, and adds them to
 * the phantom's only if the hook did not fire; NMD_E_ABORTED leaves the
 * tallies, organ sums, ledger, counters and history count as before the
 * call. */
nmd_status nmd_run_histories(nmd_ctx *ctx, int32_t phantom_id, uint64_t n_decays, uint64_t seed,
                             const nmd_run_opts *opts);

/* Work-queue chunk (histories per claim) and workgroup count of the last
 * nmd_run_histories launch.  With opts->chunk == 0 the chunk is tuned: the
 * first run of a phantom set with at least 2^22 decays per phantom times a
 * slice of itself with each candidate chunk and keeps the fastest (cached
 * per context, and in the file named by NMD_TUNE_CACHE if set). */
nmd_status nmd_get_last_launch(nmd_ctx *ctx, uint32_t *chunk, uint32_t *grid_blocks);

/* ---- captured runs --------------------------------------------------------- */

/* A HIP graph of one run of n_decays histories of phantom_id (-1 = all
 * with activity) followed by the organ reduction of each labelled phantom
 * and, if dose_rate_gy_s is given (single phantom), the Eq. 1 maps into
 * the device buffers dose_rate_gy_s and rel_uncertainty (may be NULL).
 * Each launch continues the phantoms' history streams exactly as
 * nmd_run_histories would, so k launches equal one run of k * n_decays.
 * The graph owns its own work-queue and deposit-list scratch.  It becomes
 * invalid (NMD_E_STATE at launch) once any of its phantoms is registered
 * again or gets a new activity map.  History records and the abort hook
 * are not available in graphs. */
typedef struct nmd_graph nmd_graph;
nmd_status nmd_graph_create(nmd_ctx *ctx, int32_t phantom_id, uint64_t n_decays, uint64_t seed,
                            const nmd_run_opts *opts, double *dose_rate_gy_s,
                            double *rel_uncertainty, nmd_graph **out);
/* Enqueue one replay on the context stream (asynchronous). */
nmd_status nmd_graph_launch(nmd_graph *graph);
/* Release the graph (waits for the context stream).  NULL is accepted. */
void nmd_graph_destroy(nmd_graph *graph);

/* Zero the tallies, ledger, statistics and history counter of a phantom
 * (-1 = all). */
nmd_status nmd_reset_tallies(nmd_ctx *ctx, int32_t phantom_id);

/* ---- results ------------------------------------------------------------- */

/* Dose-rate map of Eq. 1: (S_v / N) * c / m_v * A(t_s), with S_v the
 * deposited energy of voxel v, N the decays run since the last reset,
 * c = 1.602176634e-13 J/MeV and m_v the voxel mass; and the relative
 * history-by-history standard error s_v / D_v (0 where nothing was
 * deposited).  dose_rate_gy_s: device double[nvox]; rel_uncertainty:
 * device double[nvox] or NULL.  Asynchronous. */
nmd_status nmd_get_dose(nmd_ctx *ctx, int32_t phantom_id, double *dose_rate_gy_s,
                        double *rel_uncertainty);

/* Organ statistics for labels 1..n_organs (host arrays of n_organs, any may
 * be NULL): Eq. 2 mean voxel dose rate, Eq. 3 root-mean-square voxel
 * relative uncertainty, and the relative standard error of the organ mean
 * from per-history organ scores.  Synchronises the stream. */
nmd_status nmd_get_organ_dose(nmd_ctx *ctx, int32_t phantom_id, int32_t n_organs,
                              double *dose_rate_gy_s, double *eps_eq3, double *rel_sigma_mean);

/* Organ statistics from the last organ reduction enqueued for the phantom
 * (by nmd_get_organ_dose or by a graph launch), without reducing again;
 * same outputs as nmd_get_organ_dose.  Synchronises the stream. */
nmd_status nmd_read_organ_dose(nmd_ctx *ctx, int32_t phantom_id, int32_t n_organs,
                               double *dose_rate_gy_s, double *eps_eq3, double *rel_sigma_mean);

/* Organ dose rate from the per-history organ scores (A * O_o / N), which
 * equals Eq. 2 up to rounding; host double[n_organs].  Synchronises. */
nmd_status nmd_get_organ_score(nmd_ctx *ctx, int32_t phantom_id, int32_t n_organs,
                               double *dose_rate_gy_s);

/* Energy ledger of a phantom (host double[NMD_LEDGER_N], MeV) and run
 * counters (host uint64_t[NMD_STAT_N]).  Synchronise the stream. */
nmd_status nmd_get_ledger(nmd_ctx *ctx, int32_t phantom_id, double *ledger);
nmd_status nmd_get_run_stats(nmd_ctx *ctx, int32_t phantom_id, uint64_t *stats);

/* Raw accumulated sums: S_v (MeV) and S2_v (MeV^2) into device
 * double[nvox] buffers (either may be NULL), and the number of decays N.
 * Asynchronous. */
nmd_status nmd_get_tallies(nmd_ctx *ctx, int32_t phantom_id, double *sum_dev, double *sum2_dev,
                           uint64_t *n_decays);

/* Replace the sums S_v, S2_v (device or host double[nvox] each) and the
 * decay count N of a phantom, e.g. to resume from values read with
 * nmd_get_tallies.  The per-history organ scores, ledger and counters are
 * zeroed, so they no longer cover all N histories: until the next reset,
 * nmd_get_organ_score, and nmd_get_organ_dose / nmd_read_organ_dose with a
 * rel_sigma_mean output, return NMD_E_STATE (Eq. 1-3 from the voxel sums
 * stay available).  nmd_save / nmd_load carry the whole state instead.
 * Synchronises the stream. */
nmd_status nmd_set_tallies(nmd_ctx *ctx, int32_t phantom_id, const double *sum,
                           const double *sum2, uint64_t n_decays);

/* Checkpoint of a phantom's Monte Carlo state: the voxel sums S_v, S2_v of
 * the history-by-history method (Section 2.1), the per-history organ sums
 * behind the organ-mean uncertainty, the energy ledger, the run counters and
 * the history count N, which is also the next history id, so a run after
 * nmd_load into the same phantom id (the id is part of every history's
 * random stream) with the same seed continues the same streams, and runs
 * split by a save/load equal one run of their total.  nmd_save writes the
 * host file `path` (through a temporary file renamed on success).
 * nmd_load requires the phantom to be registered with the same geometry
 * (dimensions, voxel size, records) and activity map as when saved
 * (NMD_E_STATE otherwise; NMD_E_INVALID for an unreadable, truncated or
 * corrupted file, detected by a 64-bit checksum), and leaves the phantom
 * unchanged on any error.  A(t_s) of Eq. 1 is the one currently set.
 * Both synchronise the stream. */
nmd_status nmd_save(nmd_ctx *ctx, int32_t phantom_id, const char *path);
nmd_status nmd_load(nmd_ctx *ctx, int32_t phantom_id, const char *path);

/* ---- test hooks ----------------------------------------------------------- */

/* Draw n samples with the device samplers the transport kernel uses; sample
 * i uses the random stream of history i of phantom 0.  kind: 0 raw Philox
 * words (4 per sample), 1 uniform, 2 Marsaglia direction (3), 3 Klein-Nishina
 * (eps = E'/E, cos theta) at e_mev, 5 Thomson cos theta.  out: device
 * double[n * width].  Asynchronous. */
nmd_status nmd_debug_sample(nmd_ctx *ctx, int32_t kind, double e_mev, uint64_t n, uint64_t seed,
                            double *out);

/* Draw n decay voxels of phantom `phantom_id` with its alias table; sample
 * i uses the stream of history i.  out: device uint32[n].  Asynchronous. */
nmd_status nmd_debug_sample_source(nmd_ctx *ctx, int32_t phantom_id, uint64_t n, uint64_t seed,
                                   uint32_t *out);

/* Evaluate, in the transport kernel's FP32 arithmetic, the majorant of
 * phantom `phantom_id` and the largest attenuation coefficient over its
 * (material, density) pairs at n energies.  energies: device float[n];
 * out: device float[2n] (majorant, max mu).  Asynchronous. */
nmd_status nmd_debug_xs(nmd_ctx *ctx, int32_t phantom_id, uint64_t n, const float *energies,
                        float *out);

#ifdef __cplusplus
}
#endif
#endif /* NMDOSE_H */
