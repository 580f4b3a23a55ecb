/*
 * nmd_oracle.c -- TEST INFRASTRUCTURE ONLY.
 *
 * A plain, slow, FP64 CPU Monte Carlo of the internal-dosimetry method of
 * ARCHER-NM (Peng et al., arXiv 2111.11687): decays sampled from a PET
 * activity map, two back-to-back 0.511 MeV annihilation photons per decay
 * with an isotropic direction (Marsaglia), photoelectric and Compton
 * transport with a 10 keV photon cutoff and local deposit of the rest,
 * a voxel dose tally with history-by-history uncertainty, dose rate by
 * Eq. 1 and organ statistics by Eq. 2 and Eq. 3 (Sections 2.1 and 2.4).
 *
 * Only the test suite, the smoke check and the CPU-baseline leg of the
 * benchmark may load this file.  The product (the HIP library) never does,
 * and the two share no code.
 *
 * Where the paper is silent the model follows the readings listed in the
 * design notes: free-electron Klein-Nishina Compton, a Thomson-shaped
 * Rayleigh term, Z^4/E^3 photoelectric and Z^2/E^2 Rayleigh cross sections
 * anchored at 30 keV, tables on a 256-point 1-511 keV log grid evaluated by
 * log-log interpolation, secondary electrons deposited on the spot, vacuum
 * outside the grid.
 *
 * Three tracking modes:
 *   ORC_TRACK_EXACT    -- voxel-by-voxel ray traversal (Amanatides and Woo
 *                         1987), one optical depth per flight.  Independent
 *                         of the GPU's tracking; used for statistical parity.
 *   ORC_TRACK_WOODCOCK -- delta tracking against a majorant, consuming
 *                         uniforms in the documented per-history order so a
 *                         history can be replayed draw for draw.
 *   ORC_TRACK_REGIONS  -- the same delta tracking with a majorant by region:
 *                         the phantom's inside the bounding box of its dense
 *                         voxels, a smaller one in the thin voxels around it.
 *                         Not in the paper: a variant of its Woodcock step
 *                         that samples the same model with fewer null
 *                         collisions.
 * Two Klein-Nishina samplers: Kahn's rejection (1954) and the
 * Butcher-Messel composition-rejection.  Two random-number families, both
 * written here from their published definitions: Philox4x32-10 (Salmon et
 * al., SC'11), the device's family, which the Woodcock replay consumes in
 * the device's order; and xoshiro256** (Blackman and Vigna 2018) seeded per
 * history through SplitMix64, a family the device does not use, which the
 * exact-traversal mode draws from by default.
 *
 * Parity status: every primitive here is pinned by the CPU tests against
 * closed forms, numerical integration, published generator outputs or
 * invariants; the whole-pipeline dose of a heterogeneous phantom has no
 * closed form and is cross-checked between the two tracking modes.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* ------------------------------------------------------------------ */
/* Physical constants (CODATA 2018) and model parameters               */
/* ------------------------------------------------------------------ */
#define ORC_PI 3.14159265358979323846
#define ORC_RE_CM 2.8179403262e-13        /* classical electron radius  */
#define ORC_MEC2_MEV 0.51099895           /* electron rest energy       */
#define ORC_NA 6.02214076e23              /* Avogadro                   */
#define ORC_J_PER_MEV 1.602176634e-13
#define ORC_E0_MEV 0.511                  /* annihilation photon (2.1)  */
#define ORC_NGRID 256                     /* energy nodes               */
#define ORC_EGRID_MIN 1.0e-3              /* 1 keV                      */
#define ORC_EGRID_RATIO 511.0             /* top node = 511 keV         */
#define ORC_EGRID_RATIO_W 1000.0          /* the wide grid: top 1 MeV, for
                                             emitter lines above 511 keV */
#define ORC_LINE_MAX_MEV 1.0              /* emitter lines up to its top */
#define ORC_EREF 0.030                    /* anchor energy              */
#define ORC_ZREF 7.4                      /* anchor Z                   */
#define ORC_KAPPA (1.0 + 1.0 / 16384.0)   /* majorant inflation         */

/* 18F positrons (the emitter of Section 2.1): the beta+ endpoint kinetic
 * energy (MeV) and the charge of the daughter nucleus (18O). */
#define ORC_F18_T0 0.6335
#define ORC_F18_ZD 8.0
#define ORC_ALPHA (1.0 / 137.035999084) /* fine-structure constant */
#define ORC_POS_FLOOR 0.001 /* MeV: a positron's walk ends when its range above this runs out */
#define ORC_POS_CDF_N 4096  /* intervals of the tabulated spectrum CDF */

#define ORC_LEDGER_N 8
#define ORC_MAX_LINES 8
#define ORC_STATS_N 12
#define ORC_HREC_N 10

enum { ORC_TRACK_EXACT = 0, ORC_TRACK_WOODCOCK = 1, ORC_TRACK_REGIONS = 2 };
enum { ORC_KN_KAHN = 0, ORC_KN_BUTCHER = 1 };
enum { ORC_SRC_ACTIVITY = 0, ORC_SRC_PENCIL = 1 };
enum { ORC_EV_NULL = 0, ORC_EV_COMPTON = 1, ORC_EV_PE = 2, ORC_EV_RAYLEIGH = 3 };
/* ledger slots */
enum { L_EMIT = 0, L_DEP_C = 1, L_DEP_PE = 2, L_DEP_CUT = 3, L_ESC = 4, L_DISC = 5, L_DEP_POS = 6,
       L_DEP_BETA = 7 };
/* stats slots */
enum {
  S_HIST = 0, S_PHOTONS = 1, S_STEPS = 2, S_NULL = 3, S_COMPTON = 4, S_PE = 5,
  S_RAYLEIGH = 6, S_DEPOSITS = 7, S_MERGED = 8, S_MAXMERGED = 9, S_ESCAPES = 10,
  S_UNIFORMS = 11
};

/* ------------------------------------------------------------------ */
/* Klein-Nishina total cross section per electron (closed form)        */
/* ------------------------------------------------------------------ */
double orc_sigma_kn(double e_mev)
{
  const double k = e_mev / ORC_MEC2_MEV;
  const double a = 1.0 + 2.0 * k;
  /* ln(1 + 2k) through log1p: log(a) of the rounded a loses about
   * eps / (2k) relative, which the cancellation in the bracket below
   * (a difference of order k^2) turns into a 5e-9 error at 1 keV */
  const double l = log1p(2.0 * k);
  const double t1 = (1.0 + k) / (k * k) * (2.0 * (1.0 + k) / a - l / k);
  const double t2 = l / (2.0 * k);
  const double t3 = (1.0 + 3.0 * k) / (a * a);
  return 2.0 * ORC_PI * ORC_RE_CM * ORC_RE_CM * (t1 + t2 - t3);
}

/* Energy of node i of the grid from 1 keV to 1 keV * ratio: 1 keV *
 * ratio^(i/255), in MeV.  The pair's grid has ratio 511; a run whose emitter
 * has a line above 511 keV uses the wide grid, ratio 1000. */
static double grid_energy_r(int i, double ratio)
{
  return ORC_EGRID_MIN * pow(ratio, (double)i / (double)(ORC_NGRID - 1));
}
double orc_grid_energy(int i) { return grid_energy_r(i, ORC_EGRID_RATIO); }

/* Mass attenuation of one process at node energy e (cm^2/g).
 * process: 1 Compton, 2 photoelectric, 3 Rayleigh. */
double orc_mass_atten_closed(int process, double z, double z_over_a, double e)
{
  const double sref = orc_sigma_kn(ORC_EREF);
  const double ne = ORC_NA * z_over_a; /* electrons per gram */
  if (process == ORC_EV_COMPTON)
    return ne * orc_sigma_kn(e);
  if (process == ORC_EV_PE) {
    const double a_pe = sref / (ORC_ZREF * ORC_ZREF * ORC_ZREF);
    const double r = ORC_EREF / e;
    return ne * a_pe * z * z * z * r * r * r;
  }
  if (process == ORC_EV_RAYLEIGH) {
    const double a_r = 0.1 * sref / ORC_ZREF;
    const double r = ORC_EREF / e;
    return ne * a_r * z * r * r;
  }
  return 0.0;
}

/* Log-log interpolation on the grid of a table of ln-values. */
static void grid_locate(double ratio, double e, int *i_out, double *f_out)
{
  const double dl = log(ratio) / (double)(ORC_NGRID - 1);
  double t = (log(e) - log(ORC_EGRID_MIN)) / dl;
  int i = (int)floor(t);
  if (i < 0) i = 0;
  if (i > ORC_NGRID - 2) i = ORC_NGRID - 2;
  *i_out = i;
  *f_out = t - (double)i;
}

static double loglog(const double *lntab, int i, double f)
{
  return exp(lntab[i] + f * (lntab[i + 1] - lntab[i]));
}

/* ------------------------------------------------------------------ */
/* Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11)                    */
/* ------------------------------------------------------------------ */
void orc_philox4x32_10(const uint32_t ctr_in[4], const uint32_t key_in[2], uint32_t out[4])
{
  uint32_t c0 = ctr_in[0], c1 = ctr_in[1], c2 = ctr_in[2], c3 = ctr_in[3];
  uint32_t k0 = key_in[0], k1 = key_in[1];
  for (int r = 0; r < 10; ++r) {
    const uint64_t p0 = (uint64_t)0xD2511F53u * (uint64_t)c0;
    const uint64_t p1 = (uint64_t)0xCD9E8D57u * (uint64_t)c2;
    const uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
    const uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
    const uint32_t n0 = hi1 ^ c1 ^ k0;
    const uint32_t n2 = hi0 ^ c3 ^ k1;
    c0 = n0; c1 = lo1; c2 = n2; c3 = lo0;
    k0 += 0x9E3779B9u;
    k1 += 0xBB67AE85u;
  }
  out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

/* SplitMix64 (Steele, Lea and Flood, OOPSLA 2014): a Weyl sequence with
 * increment 0x9E3779B97F4A7C15 passed through a variant-13 mix. */
uint64_t orc_splitmix64(uint64_t *x)
{
  uint64_t z = (*x += 0x9E3779B97F4A7C15ull);
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

static uint64_t rotl64(uint64_t x, int k) { return (x << k) | (x >> (64 - k)); }

/* xoshiro256** (Blackman and Vigna 2018): output rotl(5 s1, 7) * 9, then the
 * xorshift-rotate state update. */
uint64_t orc_xoshiro256ss(uint64_t s[4])
{
  const uint64_t out = rotl64(s[1] * 5u, 7) * 9u;
  const uint64_t t = s[1] << 17;
  s[2] ^= s[0];
  s[3] ^= s[1];
  s[1] ^= s[2];
  s[0] ^= s[3];
  s[2] ^= t;
  s[3] = rotl64(s[3], 45);
  return out;
}

enum { ORC_RNG_PHILOX = 0, ORC_RNG_XOSHIRO = 1 };

/* Per-history stream.  Philox: counter = (block, hid_lo, hid_hi,
 * phantom_id), key = (seed_lo, seed_hi), words consumed in order x0..x3.
 * xoshiro256**: state from SplitMix64 over the seed, the history id and the
 * phantom id; each 64-bit output gives two words, high half first. */
typedef struct {
  uint32_t key[2];
  uint32_t hid_lo, hid_hi, pid;
  uint32_t block;
  uint32_t buf[4];
  int pos;             /* next word in buf; 4 = empty */
  int wide;            /* 0: 23-bit uniforms (one word); 1: 53-bit (two) */
  int rng;             /* ORC_RNG_* */
  uint64_t xs[4];      /* xoshiro256** state */
  uint64_t n_uniform;  /* uniforms handed out */
} orc_stream;

static void stream_init(orc_stream *s, uint64_t seed, uint64_t hid, uint32_t pid, int wide,
                        int rng)
{
  s->key[0] = (uint32_t)seed;
  s->key[1] = (uint32_t)(seed >> 32);
  s->hid_lo = (uint32_t)hid;
  s->hid_hi = (uint32_t)(hid >> 32);
  s->pid = pid;
  s->block = 0;
  s->pos = 4;
  s->wide = wide;
  s->rng = rng;
  s->n_uniform = 0;
  if (rng == ORC_RNG_XOSHIRO) {
    uint64_t x = seed;
    x = orc_splitmix64(&x) ^ hid;
    x = orc_splitmix64(&x) ^ (uint64_t)pid;
    for (int i = 0; i < 4; ++i) s->xs[i] = orc_splitmix64(&x);
  }
}

static uint32_t stream_word(orc_stream *s)
{
  if (s->pos == 4) {
    if (s->rng == ORC_RNG_XOSHIRO) {
      const uint64_t a = orc_xoshiro256ss(s->xs), b = orc_xoshiro256ss(s->xs);
      s->buf[0] = (uint32_t)(a >> 32);
      s->buf[1] = (uint32_t)a;
      s->buf[2] = (uint32_t)(b >> 32);
      s->buf[3] = (uint32_t)b;
    } else {
      uint32_t ctr[4] = { s->block, s->hid_lo, s->hid_hi, s->pid };
      orc_philox4x32_10(ctr, s->key, s->buf);
    }
    s->block++;
    s->pos = 0;
  }
  return s->buf[s->pos++];
}

/* Uniform on the open interval (0,1). */
static double stream_uniform(orc_stream *s)
{
  s->n_uniform++;
  if (!s->wide) {
    /* 23 bits plus one half: exactly representable in FP32 as well */
    const uint32_t x = stream_word(s);
    return ((double)(x >> 9) + 0.5) * (1.0 / 8388608.0);
  }
  const uint64_t hi = stream_word(s), lo = stream_word(s);
  const uint64_t x = (hi << 32) | lo;
  return ((double)(x >> 11) + 0.5) * (1.0 / 9007199254740992.0);
}

/* ------------------------------------------------------------------ */
/* Samplers                                                            */
/* ------------------------------------------------------------------ */

/* Isotropic unit vector, Marsaglia (1972): (v1, v2) uniform in the unit
 * disc; d = (2 v1 sqrt(1-s), 2 v2 sqrt(1-s), 1 - 2 s), s = v1^2 + v2^2. */
static void sample_marsaglia(orc_stream *st, double d[3])
{
  double v1, v2, s;
  do {
    v1 = 2.0 * stream_uniform(st) - 1.0;
    v2 = 2.0 * stream_uniform(st) - 1.0;
    s = v1 * v1 + v2 * v2;
  } while (s >= 1.0 || s == 0.0);
  const double q = 2.0 * sqrt(1.0 - s);
  d[0] = v1 * q;
  d[1] = v2 * q;
  d[2] = 1.0 - 2.0 * s;
}

/* Klein-Nishina, Kahn (1954) rejection.  Returns eps = E'/E and cos(theta).
 * With k = E / m c^2 and eta = E / E':
 *   branch A (prob (1+2k)/(9+2k)): eta = 1 + 2 k r2, accept r3 <= 4 (1/eta - 1/eta^2)
 *   branch B: eta = (1+2k)/(1+2k r2), accept r3 <= (cos^2 + 1/eta)/2,
 *             cos = 1 - (eta - 1)/k. */
static double sample_kn_kahn(orc_stream *st, double k, double *cost)
{
  for (;;) {
    const double r1 = stream_uniform(st);
    const double r2 = stream_uniform(st);
    const double r3 = stream_uniform(st);
    double eta;
    if (r1 <= (1.0 + 2.0 * k) / (9.0 + 2.0 * k)) {
      eta = 1.0 + 2.0 * k * r2;
      if (r3 > 4.0 * (1.0 / eta - 1.0 / (eta * eta)))
        continue;
    } else {
      eta = (1.0 + 2.0 * k) / (1.0 + 2.0 * k * r2);
      const double c = 1.0 - (eta - 1.0) / k;
      if (r3 > 0.5 * (c * c + 1.0 / eta))
        continue;
    }
    *cost = 1.0 - (eta - 1.0) / k;
    return 1.0 / eta;
  }
}

/* Klein-Nishina, Butcher-Messel composition-rejection.  The density of
 * eps on [eps0, 1] is proportional to (1/eps + eps) * g(eps) with
 * g = 1 - eps sin^2 / (1 + eps^2) in [0, 1]; 1/eps and eps are each sampled
 * exactly, chosen with weights ln(1/eps0) and (1 - eps0^2)/2. */
static double sample_kn_butcher(orc_stream *st, double k, double *cost)
{
  const double eps0 = 1.0 / (1.0 + 2.0 * k);
  const double a1 = log(1.0 + 2.0 * k);
  const double a2 = 0.5 * (1.0 - eps0 * eps0);
  for (;;) {
    const double r1 = stream_uniform(st);
    const double r2 = stream_uniform(st);
    const double r3 = stream_uniform(st);
    double eps;
    if (r1 * (a1 + a2) < a1)
      eps = exp(-a1 * r2);
    else
      eps = sqrt(eps0 * eps0 + (1.0 - eps0 * eps0) * r2);
    const double t = (1.0 - eps) / (k * eps);
    const double sin2 = t * (2.0 - t);
    const double g = 1.0 - eps * sin2 / (1.0 + eps * eps);
    if (r3 < g) {
      *cost = 1.0 - t;
      return eps;
    }
  }
}

/* Thomson angle: density (3/8)(1 + c^2) on [-1, 1]; CDF (c^3 + 3c + 4)/8.
 * Invert by Cardano: the cubic c^3 + 3c + (4 - 8u) = 0 has one real root. */
static double sample_thomson(double u)
{
  const double a = 4.0 * u - 2.0;
  const double r = sqrt(a * a + 1.0);
  return cbrt(a + r) + cbrt(a - r);
}

/* Rotate unit vector d by polar cos(theta) and azimuth 2 pi u:
 * d' = cos d + sin (cos(phi) b1 + sin(phi) b2), with (b1, b2, d) the
 * orthonormal basis of Duff et al. (JCGT 2017), which stays well conditioned
 * for every d including the poles. */
static void rotate_dir(double d[3], double cost, double uphi)
{
  double sint2 = 1.0 - cost * cost;
  const double sint = sint2 > 0.0 ? sqrt(sint2) : 0.0;
  const double cphi = cos(2.0 * ORC_PI * uphi), sphi = sin(2.0 * ORC_PI * uphi);
  const double x = d[0], y = d[1], z = d[2];
  const double sg = z >= 0.0 ? 1.0 : -1.0;
  const double a = -1.0 / (sg + z);
  const double b = x * y * a;
  const double b1[3] = { 1.0 + sg * x * x * a, sg * b, -sg * x };
  const double b2[3] = { b, sg + y * y * a, -y };
  double n3[3];
  for (int i = 0; i < 3; ++i) n3[i] = cost * d[i] + sint * (cphi * b1[i] + sphi * b2[i]);
  const double n = 1.0 / sqrt(n3[0] * n3[0] + n3[1] * n3[1] + n3[2] * n3[2]);
  d[0] = n3[0] * n;
  d[1] = n3[1] * n;
  d[2] = n3[2] * n;
}

/* ------------------------------------------------------------------ */
/* Problem description                                                 */
/* ------------------------------------------------------------------ */
typedef struct {
  int32_t nx, ny, nz;
  double dx, dy, dz;              /* cm */
  const double *density;          /* [nvox] g/cm^3 */
  const uint8_t *material;        /* [nvox] */
  const uint8_t *label;           /* [nvox] or NULL; 0 = none */
  int32_t n_organs;               /* labels 1..n_organs */
  const double *z_eff;            /* [n_mat] */
  const double *z_over_a;         /* [n_mat] */
  int32_t n_mat;
  const double *activity;         /* [nvox] >= 0, used for ORC_SRC_ACTIVITY */
} orc_phantom;

typedef struct {
  uint64_t n_hist;
  uint64_t first_hist;
  uint64_t seed;
  uint32_t pid;
  int32_t photons_per_decay;      /* 1 or 2 */
  uint32_t process_mask;          /* bit0 C, bit1 PE, bit2 R */
  int32_t max_real_events;        /* 0 = unlimited */
  double cutoff_mev;
  int32_t tracking;               /* ORC_TRACK_* */
  int32_t kn_method;              /* ORC_KN_* */
  int32_t wide_uniforms;          /* 0: 23-bit, 1: 53-bit */
  int32_t source_kind;            /* ORC_SRC_* */
  double pencil_origin[3];        /* cm */
  double pencil_dir[3];
  int32_t n_threads;              /* 0 = OpenMP default */
  double *hist_out;               /* [n_hist][ORC_HREC_N] or NULL */
  double electron_cutoff_mev;     /* 0: electrons deposit on the spot; > 0: Compton
                                     electrons above it walk straight ahead (CSDA) */
  const double *mean_excitation_ev; /* [n_mat], eV; needed when the cutoff is > 0 */
  int32_t rng;                    /* ORC_RNG_PHILOX or ORC_RNG_XOSHIRO */
  int32_t positron;               /* 0: the photon pair starts at the decay point, exactly
                                     back to back; 1: 18F positron range and non-collinearity
                                     (needs mean_excitation_ev) */
  double noncol_fwhm_rad;         /* FWHM of the pair's deviation from back to back */
  /* A gamma + beta emitter in place of the annihilation pair (n_lines > 0 or
   * beta_mean_mev > 0; activity source only): a decay emits at most one
   * photon, line i with probability line_yield[i] (the yields sum to at most
   * 1), isotropic, of energy line_mev[i] (<= 1 MeV; a line above 0.511 MeV
   * puts the run on the wide grid and excludes the electron option), and leaves
   * beta_mean_mev in its voxel. */
  int32_t n_lines;
  const double *line_mev;
  const double *line_yield;
  double beta_mean_mev;
} orc_opts;

/* Accumulators.  S, S2: [nvox]; O, O2: [n_organs + 1]; all caller-owned
 * and accumulated into (the caller zeroes them before the first run). */
typedef struct {
  double *S, *S2, *O, *O2;
  double ledger[ORC_LEDGER_N];
  uint64_t stats[ORC_STATS_N];
} orc_tally;

/* Cross-section tables built from the closed forms. */
typedef struct {
  double ln_mu_rho[8][3][ORC_NGRID];  /* ln of mass attenuation per process */
  double ln_major[ORC_NGRID];         /* ln of majorant (cm^-1)             */
  /* Woodcock majorant by region: inside the box [box_lo, box_hi) (cm), the
   * bounding box of every voxel at least ORC_INNER_RHO dense, the phantom's;
   * elsewhere in the grid (thinner voxels only) out_ratio times it, the
   * smallest multiple that bounds those voxels at every energy node.
   * has_out is 0 when the box is the whole grid. */
  double out_ratio;
  double box_lo[3], box_hi[3];
  int has_out;
  double grid_ratio; /* ORC_EGRID_RATIO, or ORC_EGRID_RATIO_W */
} orc_tables;

#define ORC_INNER_RHO 0.01f /* g/cm^3, compared in single precision as stored */

static void build_tables(const orc_phantom *ph, orc_tables *t, double ratio)
{
  t->grid_ratio = ratio;
  for (int m = 0; m < ph->n_mat; ++m)
    for (int p = 0; p < 3; ++p)
      for (int i = 0; i < ORC_NGRID; ++i)
        t->ln_mu_rho[m][p][i] = log(orc_mass_atten_closed(p + 1, ph->z_eff[m], ph->z_over_a[m],
                                                          grid_energy_r(i, ratio)));
  /* majorant: mu is linear in density, so the maximum over all voxels of
   * a material is reached at that material's largest density. */
  double rho_max[8];
  for (int m = 0; m < 8; ++m) rho_max[m] = 0.0;
  const int64_t nvox = (int64_t)ph->nx * ph->ny * ph->nz;
  for (int64_t v = 0; v < nvox; ++v)
    if (ph->density[v] > rho_max[ph->material[v]]) rho_max[ph->material[v]] = ph->density[v];
  for (int i = 0; i < ORC_NGRID; ++i) {
    double mx = 0.0;
    for (int m = 0; m < ph->n_mat; ++m) {
      if (rho_max[m] <= 0.0) continue;
      double s = 0.0;
      for (int p = 0; p < 3; ++p) s += exp(t->ln_mu_rho[m][p][i]);
      s *= rho_max[m];
      if (s > mx) mx = s;
    }
    t->ln_major[i] = log(mx);
  }
  /* the box of the dense voxels, and the largest density per material
   * outside it */
  int64_t lo[3] = { ph->nx, ph->ny, ph->nz }, hi[3] = { 0, 0, 0 };
  const int32_t n[3] = { ph->nx, ph->ny, ph->nz };
  for (int64_t v = 0; v < nvox; ++v) {
    if (!((float)ph->density[v] >= ORC_INNER_RHO)) continue;
    const int64_t c[3] = { v % n[0], (v / n[0]) % n[1], v / ((int64_t)n[0] * n[1]) };
    for (int a = 0; a < 3; ++a) {
      if (c[a] < lo[a]) lo[a] = c[a];
      if (c[a] + 1 > hi[a]) hi[a] = c[a] + 1;
    }
  }
  if (hi[0] == 0)
    for (int a = 0; a < 3; ++a) {
      lo[a] = 0;
      hi[a] = n[a];
    }
  const double h[3] = { ph->dx, ph->dy, ph->dz };
  for (int a = 0; a < 3; ++a) {
    t->box_lo[a] = (double)lo[a] * h[a];
    t->box_hi[a] = (double)hi[a] * h[a];
  }
  double rho_out[8];
  for (int m = 0; m < 8; ++m) rho_out[m] = 0.0;
  t->has_out = 0;
  for (int64_t v = 0; v < nvox; ++v) {
    const int64_t c[3] = { v % n[0], (v / n[0]) % n[1], v / ((int64_t)n[0] * n[1]) };
    int inside = 1;
    for (int a = 0; a < 3; ++a) inside = inside && c[a] >= lo[a] && c[a] < hi[a];
    if (inside) continue;
    t->has_out = 1;
    if (ph->density[v] > rho_out[ph->material[v]]) rho_out[ph->material[v]] = ph->density[v];
  }
  /* the ratio, widened by 2^-16 as the device widens its single-precision
   * product */
  t->out_ratio = 0.0;
  for (int i = 0; t->has_out && i < ORC_NGRID; ++i) {
    double mx = 0.0;
    for (int m = 0; m < ph->n_mat; ++m) {
      if (rho_out[m] <= 0.0) continue;
      double s = 0.0;
      for (int p = 0; p < 3; ++p) s += exp(t->ln_mu_rho[m][p][i]);
      s *= rho_out[m];
      if (s > mx) mx = s;
    }
    const double r = mx / exp(t->ln_major[i]);
    if (r > t->out_ratio) t->out_ratio = r;
  }
  t->out_ratio *= 1.0 + 1.0 / 65536.0;
}

/* Mass attenuation of all materials and processes at energy e. */
static void eval_mu_rho(const orc_tables *t, int n_mat, double e, double out[8][3])
{
  int i;
  double f;
  grid_locate(t->grid_ratio, e, &i, &f);
  for (int m = 0; m < n_mat; ++m)
    for (int p = 0; p < 3; ++p) out[m][p] = loglog(t->ln_mu_rho[m][p], i, f);
}

static double eval_major(const orc_tables *t, double e)
{
  int i;
  double f;
  grid_locate(t->grid_ratio, e, &i, &f);
  return ORC_KAPPA * loglog(t->ln_major, i, f);
}


static int in_box(const orc_tables *t, const double r[3])
{
  for (int a = 0; a < 3; ++a)
    if (!(r[a] >= t->box_lo[a] && r[a] < t->box_hi[a])) return 0;
  return 1;
}

/* Path length of a Woodcock step whose optical depth against the current
 * region's majorant is s * maj[*out]: the depth is spent region by region
 * along the ray from r (inside the box: the phantom's majorant; outside it:
 * the outer one).  The box is convex, so the ray crosses it along one
 * interval [tn, tf] of its parameter, found once from r: a ray inside
 * leaves at tf for good; a ray outside enters at tn (if at all) and leaves
 * at tf.  *out ends as the region of the step's end point.  Without an
 * outer region a ray leaving the box leaves the grid: the length is
 * infinite. */
static double region_walk(const orc_tables *t, const double r[3], const double d[3], double s,
                          const double maj[2], int *out)
{
  double tau = s * maj[*out];
  double tn = -INFINITY, tf = INFINITY;
  for (int a = 0; a < 3; ++a) {
    if (d[a] != 0.0) {
      const double t1 = (t->box_lo[a] - r[a]) / d[a], t2 = (t->box_hi[a] - r[a]) / d[a];
      const double a1 = t1 < t2 ? t1 : t2, a2 = t1 < t2 ? t2 : t1;
      if (a1 > tn) tn = a1;
      if (a2 < tf) tf = a2;
    } else if (!(r[a] >= t->box_lo[a] && r[a] < t->box_hi[a])) {
      tf = -INFINITY;
    }
  }
  double t0 = 0.0; /* where the inside stretch starts */
  if (*out) {
    /* a ray that misses the box, or only touches it, stays outside */
    if (!(tn < tf) || !(tf > 0.0) || tau <= maj[1] * (tn > 0.0 ? tn : 0.0))
      return tau / maj[1];
    t0 = tn > 0.0 ? tn : 0.0;
    tau -= maj[1] * t0;
    *out = 0;
  }
  const double tx = tf > t0 ? tf : t0; /* where the ray leaves the box */
  if (tau <= maj[0] * (tx - t0)) return t0 + tau / maj[0];
  tau -= maj[0] * (tx - t0);
  *out = 1;
  if (!t->has_out) return INFINITY;
  return tx + tau / maj[1];
}

/* ------------------------------------------------------------------ */
/* Per-history scoring                                                 */
/* ------------------------------------------------------------------ */
typedef struct {
  int64_t v;
  double e;
} dep_t;

typedef struct {
  dep_t *d;
  int n, cap;
} dep_list;

static void dep_push(dep_list *l, int64_t v, double e)
{
  if (l->n == l->cap) {
    l->cap = l->cap ? 2 * l->cap : 64;
    l->d = (dep_t *)realloc(l->d, sizeof(dep_t) * (size_t)l->cap);
  }
  l->d[l->n].v = v;
  l->d[l->n].e = e;
  l->n++;
}

typedef struct {
  const orc_phantom *ph;
  const orc_tables *tab;
  const orc_opts *op;
  double vol;           /* voxel volume, cm^3 */
  const int64_t *n_org; /* voxels per organ label */
  const double *cdf;    /* source CDF over voxels */
  int64_t nvox;
  const double *pos_cdf; /* positron spectrum CDF on ORC_POS_CDF_N + 1 nodes, or NULL */
} orc_ctx;

/* One photon in the exact-traversal mode.  Returns via the deposit list
 * and the per-thread ledger/stats. */
typedef struct {
  double ledger[ORC_LEDGER_N];
  uint64_t stats[ORC_STATS_N];
  double rec[ORC_HREC_N];
} orc_local;

static void add_dep(dep_list *l, orc_local *loc, int64_t v, double e, int slot)
{
  dep_push(l, v, e);
  loc->ledger[slot] += e;
  loc->stats[S_DEPOSITS]++;
  loc->rec[0] += e;
}

/* Choose the event at a collision.  t is u * mu_total (exact mode) or
 * u * majorant (Woodcock); anything above the real total is a null. */
static int choose_event(double t, double muc, double mupe, double mur)
{
  if (t < muc) return ORC_EV_COMPTON;
  if (t < muc + mupe) return ORC_EV_PE;
  if (t < muc + mupe + mur) return ORC_EV_RAYLEIGH;
  return ORC_EV_NULL;
}

/* ------------------------------------------------------------------ */
/* Electrons above the electron cutoff (Section 2.1 tracks them down   */
/* to 200 keV): continuous slowing down along a straight line          */
/* ------------------------------------------------------------------ */
#define ORC_HALF_K 0.1535375 /* 2 pi r_e^2 m_e c^2 N_A, MeV cm^2 / mol */

/* Bethe collision stopping power for electrons in MeV cm^2/g (the ICRU
 * Report 37 form with the Moller term F-), no density-effect term. */
double orc_stopping_power(double t, double z_over_a, double i_ev)
{
  const double tau = t / ORC_MEC2_MEV;
  const double g = tau + 1.0;
  const double b2 = 1.0 - 1.0 / (g * g);
  const double fm = 1.0 - b2 + (tau * tau / 8.0 - (2.0 * tau + 1.0) * log(2.0)) / (g * g);
  const double ir = i_ev * 1e-6 / ORC_MEC2_MEV;
  return ORC_HALF_K * z_over_a / b2 * (log(tau * tau * (tau + 2.0) / (2.0 * ir * ir)) + fm);
}

/* Mass path (g/cm^2) over which an electron slows from t_hi to t_lo: the
 * integral of dT / S(T), by 8-point Gauss-Legendre on 16 equal panels. */
double orc_csda_range(double t_lo, double t_hi, double z_over_a, double i_ev)
{
  static const double x[4] = { 0.1834346424956498, 0.5255324099163290, 0.7966664774136267,
                               0.9602898564975363 };
  static const double w[4] = { 0.3626837833783620, 0.3137066458778873, 0.2223810344533745,
                               0.1012285362903763 };
  if (!(t_hi > t_lo)) return 0.0;
  const int panels = 16;
  const double h = (t_hi - t_lo) / panels;
  double acc = 0.0;
  for (int p = 0; p < panels; ++p) {
    const double c = t_lo + (p + 0.5) * h;
    for (int q = 0; q < 4; ++q)
      acc += w[q] * (1.0 / orc_stopping_power(c - 0.5 * h * x[q], z_over_a, i_ev) +
                     1.0 / orc_stopping_power(c + 0.5 * h * x[q], z_over_a, i_ev));
  }
  return 0.5 * h * acc;
}

/* Kinetic energy after a mass path p from t, for p short of the range down
 * to t_floor: the root T1 of csda_range(T1, t) = p by Newton's method
 * (d/dT1 csda_range(T1, t) = -1 / S(T1)), kept inside [t_floor, t]. */
double orc_energy_after(double t, double p, double t_floor, double z_over_a, double i_ev)
{
  if (p <= 0.0) return t;
  double t1 = t - p * orc_stopping_power(t, z_over_a, i_ev);
  if (t1 < t_floor) t1 = t_floor;
  for (int it = 0; it < 60; ++it) {
    const double f = orc_csda_range(t1, t, z_over_a, i_ev) - p;
    double nt = t1 + f * orc_stopping_power(t1, z_over_a, i_ev);
    if (nt < t_floor) nt = t_floor;
    if (nt > t) nt = t;
    const double dt = fabs(nt - t1);
    t1 = nt;
    if (dt <= 1e-15 * t) break;
  }
  return t1;
}

/* Walk one electron of kinetic energy t0 > cutoff from r (inside voxel
 * (iv0, iv1, iv2)) along the unit direction de, voxel by voxel.  In each
 * voxel it loses what its mass path rho * s takes off the range; in the
 * voxel where the range above the cutoff runs out it leaves all it still
 * has.  Calls dep(v, e) per voxel; returns the energy carried out of the
 * grid.  end (may be NULL) receives the point where the range runs out
 * (positrons annihilate there); a walk that leaves the grid sets it to the
 * exit point. */
typedef void (*orc_dep_fn)(void *user, int64_t v, double e);

static double electron_walk(const orc_phantom *ph, const double *i_ev, double cutoff,
                            const double r[3], const int64_t iv_in[3], const double de[3],
                            double t0, orc_dep_fn dep, void *user, double *end)
{
  const int32_t n[3] = { ph->nx, ph->ny, ph->nz };
  const double h[3] = { ph->dx, ph->dy, ph->dz };
  int64_t iv[3] = { iv_in[0], iv_in[1], iv_in[2] };
  double tnext[3], tstep[3];
  int stp[3];
  for (int a = 0; a < 3; ++a) {
    if (de[a] > 0.0) {
      stp[a] = 1;
      tnext[a] = ((double)(iv[a] + 1) * h[a] - r[a]) / de[a];
      tstep[a] = h[a] / de[a];
    } else if (de[a] < 0.0) {
      stp[a] = -1;
      tnext[a] = ((double)iv[a] * h[a] - r[a]) / de[a];
      tstep[a] = -h[a] / de[a];
    } else {
      stp[a] = 0;
      tnext[a] = INFINITY;
      tstep[a] = INFINITY;
    }
    if (tnext[a] < 0.0) tnext[a] = 0.0;
  }
  double t = t0, s_cur = 0.0;
  for (;;) {
    const int64_t v = iv[0] + (int64_t)n[0] * (iv[1] + (int64_t)n[1] * iv[2]);
    const int m = ph->material[v];
    const double rho = ph->density[v];
    const double za = ph->z_over_a[m], ie = i_ev[m];
    int ax = 0;
    if (tnext[1] < tnext[ax]) ax = 1;
    if (tnext[2] < tnext[ax]) ax = 2;
    const double seg = tnext[ax] - s_cur;
    const double rng = orc_csda_range(cutoff, t, za, ie);
    if (rho * seg >= rng) {
      dep(user, v, t);
      if (end)
        for (int a = 0; a < 3; ++a) end[a] = r[a] + (s_cur + rng / rho) * de[a];
      return 0.0;
    }
    const double t1 = orc_energy_after(t, rho * seg, cutoff, za, ie);
    dep(user, v, t - t1);
    t = t1;
    s_cur = tnext[ax];
    iv[ax] += stp[ax];
    tnext[ax] += tstep[ax];
    if (iv[ax] < 0 || iv[ax] >= n[ax]) {
      if (end)
        for (int a = 0; a < 3; ++a) end[a] = r[a] + s_cur * de[a];
      return t;
    }
  }
}

/* Handle a real event at voxel v.  Returns 1 when the photon ends. */
typedef struct {
  dep_list *l;
  orc_local *loc;
  int slot; /* ledger slot of the deposits */
} walk_sink;

static void walk_deposit(void *user, int64_t v, double e)
{
  walk_sink *w = (walk_sink *)user;
  add_dep(w->l, w->loc, v, e, w->slot);
}

/* The Compton electron of energy te at position r in voxel v: deposited on
 * the spot, or, above the electron cutoff, walked along its recoil
 * momentum E d_in - E' d_out. */
static void compton_electron(const orc_ctx *cx, int64_t v, const double r[3], const double d_in[3],
                             const double d_out[3], double e, double e1, dep_list *l,
                             orc_local *loc)
{
  const orc_phantom *ph = cx->ph;
  const double te = e - e1;
  double p[3], pn = 0.0;
  for (int a = 0; a < 3; ++a) {
    p[a] = e * d_in[a] - e1 * d_out[a];
    pn += p[a] * p[a];
  }
  pn = sqrt(pn);
  if (!(pn > 0.0)) {
    add_dep(l, loc, v, te, L_DEP_C);
    return;
  }
  for (int a = 0; a < 3; ++a) p[a] /= pn;
  const int64_t iv[3] = { v % ph->nx, (v / ph->nx) % ph->ny, v / ((int64_t)ph->nx * ph->ny) };
  walk_sink sink = { l, loc, L_DEP_C };
  const double esc = electron_walk(ph, cx->op->mean_excitation_ev, cx->op->electron_cutoff_mev,
                                   r, iv, p, te, walk_deposit, &sink, NULL);
  if (esc > 0.0) {
    loc->ledger[L_ESC] += esc;
    loc->rec[1] += esc;
  }
}

static int do_event(const orc_ctx *cx, orc_stream *st, int ev, int64_t v, const double r[3],
                    double *E, double d[3], dep_list *l, orc_local *loc, int *n_real)
{
  const orc_opts *op = cx->op;
  (*n_real)++;
  if (ev == ORC_EV_COMPTON) {
    loc->stats[S_COMPTON]++;
    loc->rec[2] += 1.0;
    const double k = *E / ORC_MEC2_MEV;
    double cost;
    const double eps = op->kn_method == ORC_KN_KAHN ? sample_kn_kahn(st, k, &cost)
                                                    : sample_kn_butcher(st, k, &cost);
    const double uphi = stream_uniform(st);
    const double e1 = eps * *E;
    if (op->electron_cutoff_mev > 0.0 && *E - e1 > op->electron_cutoff_mev) {
      const double d_in[3] = { d[0], d[1], d[2] };
      rotate_dir(d, cost, uphi);
      compton_electron(cx, v, r, d_in, d, *E, e1, l, loc);
    } else {
      add_dep(l, loc, v, *E - e1, L_DEP_C);
      rotate_dir(d, cost, uphi);
    }
    *E = e1;
    if (*E < op->cutoff_mev) {
      add_dep(l, loc, v, *E, L_DEP_CUT);
      return 1;
    }
  } else if (ev == ORC_EV_PE) {
    loc->stats[S_PE]++;
    loc->rec[3] += 1.0;
    add_dep(l, loc, v, *E, L_DEP_PE);
    return 1;
  } else {
    loc->stats[S_RAYLEIGH]++;
    loc->rec[4] += 1.0;
    const double cost = sample_thomson(stream_uniform(st));
    const double uphi = stream_uniform(st);
    rotate_dir(d, cost, uphi);
  }
  if (op->max_real_events > 0 && *n_real >= op->max_real_events) {
    loc->ledger[L_DISC] += *E;
    loc->rec[9] += *E;
    return 1;
  }
  return 0;
}

static int masked(const orc_opts *op, int ev)
{
  return ev != ORC_EV_NULL && !(op->process_mask & (1u << (ev - 1)));
}

static void photon_woodcock(const orc_ctx *cx, orc_stream *st, double r[3], double d[3],
                            double e0, dep_list *l, orc_local *loc)
{
  const orc_phantom *ph = cx->ph;
  const int regions = cx->op->tracking == ORC_TRACK_REGIONS;
  double E = e0;
  double mur[8][3];
  double maj[2] = { 0.0, 0.0 }; /* inside the box, outside it */
  double e_cached = -1.0;
  int n_real = 0;
  int out = regions && !in_box(cx->tab, r); /* in the outer region */
  for (;;) {
    if (E != e_cached) {
      eval_mu_rho(cx->tab, ph->n_mat, E, mur);
      maj[0] = eval_major(cx->tab, E);
      maj[1] = cx->tab->has_out ? cx->tab->out_ratio * maj[0] : 0.0;
      e_cached = E;
    }
    loc->stats[S_STEPS]++;
    loc->rec[5] += 1.0;
    double s = -log(stream_uniform(st)) / maj[out];
    if (regions) {
      const double q[3] = { r[0] + s * d[0], r[1] + s * d[1], r[2] + s * d[2] };
      if (out || !in_box(cx->tab, q)) s = region_walk(cx->tab, r, d, s, maj, &out);
    }
    const int gone = isinf(s); /* left the box with nothing outside it */
    if (!gone) {
      r[0] += s * d[0];
      r[1] += s * d[1];
      r[2] += s * d[2];
    }
    const double fx = floor(r[0] / ph->dx), fy = floor(r[1] / ph->dy), fz = floor(r[2] / ph->dz);
    if (gone || fx < 0.0 || fy < 0.0 || fz < 0.0 || fx >= ph->nx || fy >= ph->ny ||
        fz >= ph->nz) {
      loc->ledger[L_ESC] += E;
      loc->rec[1] += E;
      loc->stats[S_ESCAPES]++;
      return;
    }
    const int64_t v = (int64_t)fx + (int64_t)ph->nx * ((int64_t)fy + (int64_t)ph->ny * (int64_t)fz);
    const int m = ph->material[v];
    const double rho = ph->density[v];
    const double t = stream_uniform(st) * maj[out];
    int ev = choose_event(t, rho * mur[m][0], rho * mur[m][1], rho * mur[m][2]);
    if (masked(cx->op, ev)) ev = ORC_EV_NULL;
    if (ev == ORC_EV_NULL) {
      loc->stats[S_NULL]++;
      continue;
    }
    if (do_event(cx, st, ev, v, r, &E, d, l, loc, &n_real)) return;
  }
}

static void photon_exact(const orc_ctx *cx, orc_stream *st, double r[3], int64_t iv[3], double d[3],
                         double e0, dep_list *l, orc_local *loc)
{
  const orc_phantom *ph = cx->ph;
  const int32_t n[3] = { ph->nx, ph->ny, ph->nz };
  const double h[3] = { ph->dx, ph->dy, ph->dz };
  double E = e0;
  double mur[8][3];
  double e_cached = -1.0;
  int n_real = 0;
  for (;;) {
    if (E != e_cached) {
      eval_mu_rho(cx->tab, ph->n_mat, E, mur);
      e_cached = E;
    }
    loc->stats[S_STEPS]++;
    loc->rec[5] += 1.0;
    double tau = -log(stream_uniform(st));
    /* Amanatides-Woo traversal from r inside voxel iv. */
    double tmax[3], tdel[3];
    int stp[3];
    for (int a = 0; a < 3; ++a) {
      if (d[a] > 0.0) {
        stp[a] = 1;
        tmax[a] = ((double)(iv[a] + 1) * h[a] - r[a]) / d[a];
        tdel[a] = h[a] / d[a];
      } else if (d[a] < 0.0) {
        stp[a] = -1;
        tmax[a] = ((double)iv[a] * h[a] - r[a]) / d[a];
        tdel[a] = -h[a] / d[a];
      } else {
        stp[a] = 0;
        tmax[a] = INFINITY;
        tdel[a] = INFINITY;
      }
      if (tmax[a] < 0.0) tmax[a] = 0.0;
    }
    double tcur = 0.0;
    int escaped = 0;
    int64_t v;
    double mu_c = 0, mu_pe = 0, mu_r = 0, mu_t = 0;
    for (;;) {
      v = iv[0] + (int64_t)n[0] * (iv[1] + (int64_t)n[1] * iv[2]);
      const int m = ph->material[v];
      const double rho = ph->density[v];
      mu_c = rho * mur[m][0];
      mu_pe = rho * mur[m][1];
      mu_r = rho * mur[m][2];
      mu_t = mu_c + mu_pe + mu_r;
      int ax = 0;
      if (tmax[1] < tmax[ax]) ax = 1;
      if (tmax[2] < tmax[ax]) ax = 2;
      const double seg = tmax[ax] - tcur;
      if (mu_t * seg > tau) {
        tcur += tau / mu_t;
        break;
      }
      tau -= mu_t * seg;
      tcur = tmax[ax];
      iv[ax] += stp[ax];
      tmax[ax] += tdel[ax];
      if (iv[ax] < 0 || iv[ax] >= n[ax]) {
        escaped = 1;
        break;
      }
    }
    if (escaped) {
      loc->ledger[L_ESC] += E;
      loc->rec[1] += E;
      loc->stats[S_ESCAPES]++;
      return;
    }
    for (int a = 0; a < 3; ++a) r[a] += tcur * d[a];
    int ev = choose_event(stream_uniform(st) * mu_t, mu_c, mu_pe, mu_r);
    if (ev == ORC_EV_NULL) /* u * mu_t rounded up to mu_t: take the last process present */
      ev = mu_r > 0.0 ? ORC_EV_RAYLEIGH : (mu_pe > 0.0 ? ORC_EV_PE : ORC_EV_COMPTON);
    if (masked(cx->op, ev)) {
      /* a masked process leaves the photon untouched */
      loc->stats[S_NULL]++;
      continue;
    }
    if (do_event(cx, st, ev, v, r, &E, d, l, loc, &n_real)) return;
  }
}

/* Source voxel by inversion of the cumulative activity (binary search). */
static int64_t source_voxel(const orc_ctx *cx, double u)
{
  const double target = u * cx->cdf[cx->nvox - 1];
  int64_t lo = 0, hi = cx->nvox - 1;
  while (lo < hi) {
    const int64_t mid = lo + (hi - lo) / 2;
    if (cx->cdf[mid] > target)
      hi = mid;
    else
      lo = mid + 1;
  }
  return lo;
}

/* Decay point (Section 2.1: decays follow the activity; uniform within the
 * voxel): the voxel by CDF inversion, then three position uniforms.  The
 * Woodcock replay mode takes the same two draws the device alias sampler
 * takes (a raw word for the index and a uniform for the accept test); it
 * inverts the CDF with the raw word. */
static void sample_decay(const orc_ctx *cx, orc_stream *st, int64_t iv0[3], double r0[3])
{
  const orc_phantom *ph = cx->ph;
  int64_t v;
  if (cx->op->tracking != ORC_TRACK_EXACT) {
    const uint32_t x = stream_word(st);
    st->n_uniform++;
    (void)stream_uniform(st);
    v = source_voxel(cx, ((double)x + 0.5) / 4294967296.0);
  } else {
    v = source_voxel(cx, stream_uniform(st));
  }
  iv0[0] = v % ph->nx;
  iv0[1] = (v / ph->nx) % ph->ny;
  iv0[2] = v / ((int64_t)ph->nx * ph->ny);
  r0[0] = ((double)iv0[0] + stream_uniform(st)) * ph->dx;
  r0[1] = ((double)iv0[1] + stream_uniform(st)) * ph->dy;
  r0[2] = ((double)iv0[2] + stream_uniform(st)) * ph->dz;
}

/* ------------------------------------------------------------------ */
/* 18F positrons: kinetic energy, range and the pair's non-collinearity */
/* ------------------------------------------------------------------ */

/* Allowed beta+ spectrum (Fermi theory of beta decay), unnormalised:
 * dN/dT = p W (W0 - W)^2 F(W), with W = 1 + T / m_e c^2 the positron's total
 * energy, p = sqrt(W^2 - 1) its momentum (units of m_e c^2 and m_e c), W0 the
 * total energy at the endpoint, and F the non-relativistic Fermi function
 * 2 pi eta / (1 - exp(-2 pi eta)) with eta = -Z_d alpha W / p: the positron
 * is repelled by the daughter nucleus's charge Z_d. */
double orc_beta_plus_shape(double t)
{
  if (!(t > 0.0) || !(t < ORC_F18_T0)) return 0.0;
  const double w = 1.0 + t / ORC_MEC2_MEV, w0 = 1.0 + ORC_F18_T0 / ORC_MEC2_MEV;
  const double p = sqrt(w * w - 1.0);
  const double x = -2.0 * ORC_PI * ORC_F18_ZD * ORC_ALPHA * w / p; /* 2 pi eta < 0 */
  const double f = x / -expm1(-x);
  return p * w * (w0 - w) * (w0 - w) * f;
}

/* The spectrum's CDF on the nodes T_i = T0 i / ORC_POS_CDF_N, each interval
 * integrated by 4-point Gauss-Legendre, normalised to 1 at T0. */
static void build_positron_cdf(double *cdf)
{
  static const double x[2] = { 0.3399810435848563, 0.8611363115940526 };
  static const double w[2] = { 0.6521451548625461, 0.3478548451374538 };
  const double h = ORC_F18_T0 / ORC_POS_CDF_N;
  cdf[0] = 0.0;
  for (int i = 0; i < ORC_POS_CDF_N; ++i) {
    const double c = (i + 0.5) * h;
    double acc = 0.0;
    for (int q = 0; q < 2; ++q)
      acc += w[q] * (orc_beta_plus_shape(c - 0.5 * h * x[q]) +
                     orc_beta_plus_shape(c + 0.5 * h * x[q]));
    cdf[i + 1] = cdf[i] + 0.5 * h * acc;
  }
  const double tot = cdf[ORC_POS_CDF_N];
  for (int i = 1; i <= ORC_POS_CDF_N; ++i) cdf[i] /= tot;
}

/* Kinetic energy of the positron for the uniform u: the CDF inverted on
 * its nodes, linearly within an interval. */
static double positron_energy(const double *cdf, double u)
{
  int lo = 0, hi = ORC_POS_CDF_N;
  while (hi - lo > 1) {
    const int mid = (lo + hi) / 2;
    if (cdf[mid] <= u) lo = mid;
    else hi = mid;
  }
  const double h = ORC_F18_T0 / ORC_POS_CDF_N;
  const double span = cdf[lo + 1] - cdf[lo];
  const double f = span > 0.0 ? (u - cdf[lo]) / span : 0.0;
  return (lo + f) * h;
}

/* Polar angle of the pair's deviation from back to back: the deviation is
 * an isotropic two-dimensional Gaussian of the given FWHM, so its size is
 * Rayleigh distributed, sigma sqrt(-2 ln u). */
static double noncollinear_angle(double fwhm, double u)
{
  const double sigma = fwhm / (2.0 * sqrt(2.0 * log(2.0)));
  return sigma * sqrt(-2.0 * log(u));
}

/* The positron of a decay at r0 (voxel iv0): its kinetic energy (one
 * uniform), its direction (Marsaglia) and the two uniforms of the pair's
 * deviation from back to back (*u_dev), then its straight CSDA walk down to
 * ORC_POS_FLOOR, each voxel's loss booked as a positron deposit.  Moves
 * r0 / iv0 to the annihilation point.  Returns 1 when the positron leaves
 * the grid (then the pair is born outside it and escapes). */
static int positron_start(const orc_ctx *cx, orc_stream *st, double r0[3], int64_t iv0[3],
                          double u_dev[2], dep_list *l, orc_local *loc)
{
  const orc_phantom *ph = cx->ph;
  const double t = positron_energy(cx->pos_cdf, stream_uniform(st));
  double dp[3];
  sample_marsaglia(st, dp);
  u_dev[0] = stream_uniform(st);
  u_dev[1] = stream_uniform(st);
  loc->ledger[L_EMIT] += t;
  const int64_t v0 = iv0[0] + (int64_t)ph->nx * (iv0[1] + (int64_t)ph->ny * iv0[2]);
  if (!(t > ORC_POS_FLOOR)) { /* too slow to move: it stops where it was born */
    add_dep(l, loc, v0, t, L_DEP_POS);
    return 0;
  }
  walk_sink sink = { l, loc, L_DEP_POS };
  double end[3];
  const double esc = electron_walk(ph, cx->op->mean_excitation_ev, ORC_POS_FLOOR, r0, iv0, dp, t,
                                   walk_deposit, &sink, end);
  if (esc > 0.0) {
    loc->ledger[L_ESC] += esc;
    loc->rec[1] += esc;
    return 1;
  }
  const double h[3] = { ph->dx, ph->dy, ph->dz };
  const int32_t n[3] = { ph->nx, ph->ny, ph->nz };
  for (int a = 0; a < 3; ++a) {
    r0[a] = end[a];
    int64_t i = (int64_t)floor(end[a] / h[a]);
    iv0[a] = i < 0 ? 0 : (i >= n[a] ? n[a] - 1 : i);
  }
  return 0;
}

static void run_history(const orc_ctx *cx, uint64_t hid, dep_list *l, orc_local *loc,
                        const orc_tally *tal)
{
  const orc_phantom *ph = cx->ph;
  const orc_opts *op = cx->op;
  orc_stream st;
  stream_init(&st, op->seed, hid, op->pid, op->wide_uniforms, op->rng);
  memset(loc->rec, 0, sizeof(loc->rec));
  l->n = 0;

  double r0[3], d0[3];
  int64_t iv0[3];
  int nph = op->photons_per_decay;
  if (op->source_kind == ORC_SRC_PENCIL) {
    nph = 1;
    for (int a = 0; a < 3; ++a) {
      r0[a] = op->pencil_origin[a];
      d0[a] = op->pencil_dir[a];
    }
    iv0[0] = (int64_t)floor(r0[0] / ph->dx);
    iv0[1] = (int64_t)floor(r0[1] / ph->dy);
    iv0[2] = (int64_t)floor(r0[2] / ph->dz);
  } else if (op->n_lines > 0 || op->beta_mean_mev > 0.0) {
    /* a gamma + beta emitter: the decay point, one uniform for the line
     * (or none), the beta energy left in the decay voxel, then the photon */
    sample_decay(cx, &st, iv0, r0);
    const double u = stream_uniform(&st);
    int line = -1;
    double c = 0.0;
    for (int i = 0; i < op->n_lines; ++i) {
      c += op->line_yield[i];
      if (u < c) {
        line = i;
        break;
      }
    }
    if (op->beta_mean_mev > 0.0) {
      const int64_t v0 = iv0[0] + (int64_t)ph->nx * (iv0[1] + (int64_t)ph->ny * iv0[2]);
      loc->ledger[L_EMIT] += op->beta_mean_mev;
      add_dep(l, loc, v0, op->beta_mean_mev, L_DEP_BETA);
    }
    if (line >= 0) {
      const double e0 = op->line_mev[line];
      sample_marsaglia(&st, d0);
      loc->ledger[L_EMIT] += e0;
      loc->stats[S_PHOTONS]++;
      if (op->tracking != ORC_TRACK_EXACT)
        photon_woodcock(cx, &st, r0, d0, e0, l, loc);
      else
        photon_exact(cx, &st, r0, iv0, d0, e0, l, loc);
    }
    nph = 0;
  } else {
    sample_decay(cx, &st, iv0, r0);
    sample_marsaglia(&st, d0);
  }
  /* the positron's walk; the pair is born where it ends */
  const int positron = op->positron && op->source_kind != ORC_SRC_PENCIL;
  double u_dev[2] = { 0.5, 0.5 };
  const int pair_outside = positron && positron_start(cx, &st, r0, iv0, u_dev, l, loc);
  for (int p = 0; p < nph; ++p) {
    double r[3] = { r0[0], r0[1], r0[2] };
    double d[3] = { d0[0], d0[1], d0[2] };
    int64_t iv[3] = { iv0[0], iv0[1], iv0[2] };
    loc->ledger[L_EMIT] += ORC_E0_MEV;
    loc->stats[S_PHOTONS]++;
    if (pair_outside) { /* born outside the grid: escapes, draws nothing */
      loc->ledger[L_ESC] += ORC_E0_MEV;
      loc->rec[1] += ORC_E0_MEV;
      loc->stats[S_ESCAPES]++;
      continue;
    }
    if (p == 1) {
      d[0] = -d0[0];
      d[1] = -d0[1];
      d[2] = -d0[2];
      if (positron) /* non-collinearity, from the uniforms drawn with the positron */
        rotate_dir(d, cos(noncollinear_angle(op->noncol_fwhm_rad, u_dev[0])), u_dev[1]);
    }
    if (op->tracking != ORC_TRACK_EXACT)
      photon_woodcock(cx, &st, r, d, ORC_E0_MEV, l, loc);
    else
      photon_exact(cx, &st, r, iv, d, ORC_E0_MEV, l, loc);
  }
  loc->stats[S_HIST]++;
  loc->stats[S_UNIFORMS] += st.n_uniform;
  loc->rec[8] = (double)st.n_uniform;

  /* Merge this history's deposits by voxel (history-by-history scoring). */
  int nm = 0;
  for (int i = 0; i < l->n; ++i) {
    int j;
    for (j = 0; j < nm; ++j)
      if (l->d[j].v == l->d[i].v) break;
    if (j < nm) {
      l->d[j].e += l->d[i].e;
    } else {
      l->d[nm] = l->d[i];
      nm++;
    }
  }
  loc->stats[S_MERGED] += (uint64_t)nm;
  if ((uint64_t)nm > loc->stats[S_MAXMERGED]) loc->stats[S_MAXMERGED] = (uint64_t)nm;
  loc->rec[7] = (double)nm;
  for (int i = 0; i < nm; ++i) {
    const int64_t v = l->d[i].v;
    const double e = l->d[i].e;
    loc->rec[6] += (double)v;
#pragma omp atomic
    tal->S[v] += e;
#pragma omp atomic
    tal->S2[v] += e * e;
  }
  /* Per-history organ score q_o = sum_{v in o} e_v c / (m_v N_o). */
  if (ph->label && tal->O) {
    for (int i = 0; i < nm; ++i) {
      const int o = ph->label[l->d[i].v];
      if (o == 0 || l->d[i].e < 0.0) continue;
      double q = 0.0;
      for (int j = i; j < nm; ++j) {
        if (ph->label[l->d[j].v] != o || l->d[j].e < 0.0) continue;
        const double m_kg = ph->density[l->d[j].v] * cx->vol * 1.0e-3;
        q += l->d[j].e * ORC_J_PER_MEV / (m_kg * (double)cx->n_org[o]);
        if (j > i) l->d[j].e = -1.0; /* consumed */
      }
#pragma omp atomic
      tal->O[o] += q;
#pragma omp atomic
      tal->O2[o] += q * q;
    }
  }
}

/* Run n_hist histories, accumulating into tal.  Returns 0 on success,
 * a negative value on invalid input. */
int orc_run(const orc_phantom *ph, const orc_opts *op, orc_tally *tal)
{
  if (!ph || !op || !tal || ph->nx < 1 || ph->ny < 1 || ph->nz < 1 || ph->n_mat < 1 ||
      ph->n_mat > 8)
    return -1;
  if (op->photons_per_decay < 1 || op->photons_per_decay > 2) return -1;
  if (op->tracking < ORC_TRACK_EXACT || op->tracking > ORC_TRACK_REGIONS) return -1;
  if (op->electron_cutoff_mev > 0.0 || op->positron) {
    if (!op->mean_excitation_ev) return -1;
    for (int m = 0; m < ph->n_mat; ++m)
      if (!(op->mean_excitation_ev[m] > 0.0)) return -1;
  }
  if (op->positron && !(op->noncol_fwhm_rad >= 0.0 && op->noncol_fwhm_rad < 0.1)) return -1;
  if (op->n_lines > 0 || op->beta_mean_mev > 0.0) {
    if (op->positron || op->source_kind != ORC_SRC_ACTIVITY || op->n_lines > ORC_MAX_LINES ||
        op->n_lines < 0 || !(op->beta_mean_mev >= 0.0) || (op->n_lines && (!op->line_mev ||
        !op->line_yield)))
      return -1;
    double ysum = 0.0;
    for (int i = 0; i < op->n_lines; ++i) {
      if (!(op->line_mev[i] > 0.001 && op->line_mev[i] <= ORC_LINE_MAX_MEV) ||
          !(op->line_yield[i] >= 0.0))
        return -1;
      /* the electron range tables end above the Compton electrons of 511 keV */
      if (op->line_mev[i] > ORC_E0_MEV && op->electron_cutoff_mev > 0.0) return -1;
      ysum += op->line_yield[i];
    }
    if (ysum > 1.0 + 1e-12) return -1;
  }
  const int64_t nvox = (int64_t)ph->nx * ph->ny * ph->nz;
  for (int64_t v = 0; v < nvox; ++v) {
    if (ph->material[v] >= ph->n_mat || !(ph->density[v] > 0.0) || isinf(ph->density[v]))
      return -2;
    if (ph->label && ph->label[v] > ph->n_organs) return -2;
  }

  /* an emitter line above 511 keV takes the wide grid */
  int wide = 0;
  for (int i = 0; i < op->n_lines; ++i) wide = wide || op->line_mev[i] > ORC_E0_MEV;
  orc_tables *tab = (orc_tables *)malloc(sizeof(orc_tables));
  build_tables(ph, tab, wide ? ORC_EGRID_RATIO_W : ORC_EGRID_RATIO);

  orc_ctx cx;
  cx.ph = ph;
  cx.tab = tab;
  cx.op = op;
  cx.vol = ph->dx * ph->dy * ph->dz;
  cx.nvox = nvox;
  int64_t *n_org = (int64_t *)calloc((size_t)ph->n_organs + 1, sizeof(int64_t));
  if (ph->label)
    for (int64_t v = 0; v < nvox; ++v)
      if (ph->label[v] <= ph->n_organs) n_org[ph->label[v]]++;
  cx.n_org = n_org;
  double *cdf = NULL;
  if (op->source_kind == ORC_SRC_ACTIVITY) {
    cdf = (double *)malloc(sizeof(double) * (size_t)nvox);
    double acc = 0.0;
    for (int64_t v = 0; v < nvox; ++v) {
      const double a = ph->activity[v];
      if (!(a >= 0.0) || isinf(a)) {
        free(cdf);
        free(n_org);
        free(tab);
        return -3;
      }
      acc += a;
      cdf[v] = acc;
    }
    if (!(acc > 0.0)) {
      free(cdf);
      free(n_org);
      free(tab);
      return -3;
    }
  }
  cx.cdf = cdf;
  double pos_cdf[ORC_POS_CDF_N + 1];
  cx.pos_cdf = NULL;
  if (op->positron) {
    build_positron_cdf(pos_cdf);
    cx.pos_cdf = pos_cdf;
  }

  double ledger[ORC_LEDGER_N] = { 0 };
  uint64_t stats[ORC_STATS_N] = { 0 };
#ifdef _OPENMP
  const int nthr = op->n_threads > 0 ? op->n_threads : omp_get_max_threads();
#pragma omp parallel num_threads(nthr)
#endif
  {
    dep_list l = { NULL, 0, 0 };
    orc_local loc;
    memset(&loc, 0, sizeof(loc));
    int64_t h;
#ifdef _OPENMP
#pragma omp for schedule(dynamic, 256)
#endif
    for (h = 0; h < (int64_t)op->n_hist; ++h) {
      run_history(&cx, op->first_hist + (uint64_t)h, &l, &loc, tal);
      if (op->hist_out)
        memcpy(op->hist_out + (size_t)h * ORC_HREC_N, loc.rec, sizeof(loc.rec));
    }
#ifdef _OPENMP
#pragma omp critical
#endif
    {
      for (int i = 0; i < ORC_LEDGER_N; ++i) ledger[i] += loc.ledger[i];
      for (int i = 0; i < ORC_STATS_N; ++i) {
        if (i == S_MAXMERGED) {
          if (loc.stats[i] > stats[i]) stats[i] = loc.stats[i];
        } else {
          stats[i] += loc.stats[i];
        }
      }
    }
    free(l.d);
  }
  for (int i = 0; i < ORC_LEDGER_N; ++i) tal->ledger[i] += ledger[i];
  for (int i = 0; i < ORC_STATS_N; ++i) {
    if (i == S_MAXMERGED) {
      if (stats[i] > tal->stats[i]) tal->stats[i] = stats[i];
    } else {
      tal->stats[i] += stats[i];
    }
  }
  free(cdf);
  free(n_org);
  free(tab);
  return 0;
}

/* ------------------------------------------------------------------ */
/* Outputs: Eq. 1 per voxel, Eq. 2 and Eq. 3 per organ                 */
/* ------------------------------------------------------------------ */

/* Dose per decay D_v = (S_v / N) c / m_v; history-by-history standard
 * error s_v = (c / m_v) sqrt((S2_v/N - (S_v/N)^2) / (N - 1)); relative
 * uncertainty eps_v = s_v / D_v (0 where nothing was deposited); dose rate
 * by Eq. 1: D_v * A(t_s). */
void orc_finalize(const double *S, const double *S2, const double *density, int64_t nvox,
                  double voxel_cm3, double n_decays, double a_ts_bq, double *dose_rate,
                  double *rel_unc)
{
  for (int64_t v = 0; v < nvox; ++v) {
    const double c_m = ORC_J_PER_MEV / (density[v] * voxel_cm3 * 1.0e-3);
    const double mean = S[v] / n_decays;
    const double d = mean * c_m;
    dose_rate[v] = d * a_ts_bq;
    if (rel_unc) {
      if (S[v] > 0.0 && n_decays > 1.0) {
        double var = (S2[v] / n_decays - mean * mean) / (n_decays - 1.0);
        if (var < 0.0) var = 0.0;
        rel_unc[v] = sqrt(var) * c_m / d;
      } else {
        rel_unc[v] = 0.0;
      }
    }
  }
}

/* Eq. 2 (mean of voxel dose rates over the organ) and Eq. 3 (root mean
 * square of voxel relative uncertainties over the organ), for labels
 * 1..n_organs.  Organs with no voxel get 0. */
void orc_organ_stats(const double *dose_rate, const double *rel_unc, const uint8_t *label,
                     int64_t nvox, int32_t n_organs, double *organ_rate, double *organ_eps)
{
  double *sum = (double *)calloc((size_t)n_organs + 1, sizeof(double));
  double *sum2 = (double *)calloc((size_t)n_organs + 1, sizeof(double));
  int64_t *cnt = (int64_t *)calloc((size_t)n_organs + 1, sizeof(int64_t));
  for (int64_t v = 0; v < nvox; ++v) {
    const int o = label[v];
    if (o < 1 || o > n_organs) continue;
    sum[o] += dose_rate[v];
    sum2[o] += rel_unc[v] * rel_unc[v];
    cnt[o]++;
  }
  for (int o = 1; o <= n_organs; ++o) {
    organ_rate[o - 1] = cnt[o] ? sum[o] / (double)cnt[o] : 0.0;
    organ_eps[o - 1] = cnt[o] ? sqrt(sum2[o] / (double)cnt[o]) : 0.0;
  }
  free(sum);
  free(sum2);
  free(cnt);
}

/* ------------------------------------------------------------------ */
/* Sampler access for the tests                                        */
/* ------------------------------------------------------------------ */

/* kind 0: raw Philox words; 1: uniforms; 2: Marsaglia directions (3 per
 * sample); 3: Kahn KN (eps, cos); 4: Butcher-Messel KN (eps, cos);
 * 5: Thomson cos; 6: 18F positron kinetic energy (MeV); 7: the pair's
 * deviation angle from back to back (rad) for a FWHM of e_mev rad.
 * Sample i uses the stream of history i. */
int orc_sample(int kind, double e_mev, uint64_t n, uint64_t seed, int wide, int rng,
               double *out)
{
  const double k = e_mev / ORC_MEC2_MEV;
  double pos_cdf[ORC_POS_CDF_N + 1];
  if (kind == 6) build_positron_cdf(pos_cdf);
  for (uint64_t i = 0; i < n; ++i) {
    orc_stream st;
    stream_init(&st, seed, i, 0, wide, rng);
    switch (kind) {
    case 0:
      for (int j = 0; j < 4; ++j) out[4 * i + j] = (double)stream_word(&st);
      break;
    case 1:
      out[i] = stream_uniform(&st);
      break;
    case 2:
      sample_marsaglia(&st, out + 3 * i);
      break;
    case 3:
      out[2 * i] = sample_kn_kahn(&st, k, out + 2 * i + 1);
      break;
    case 4:
      out[2 * i] = sample_kn_butcher(&st, k, out + 2 * i + 1);
      break;
    case 5:
      out[i] = sample_thomson(stream_uniform(&st));
      break;
    case 6:
      out[i] = positron_energy(pos_cdf, stream_uniform(&st));
      break;
    case 7:
      out[i] = noncollinear_angle(e_mev, stream_uniform(&st));
      break;
    default:
      return -1;
    }
  }
  return 0;
}

/* Decay points of a phantom's activity map, as the transport draws them:
 * out[4 i] = voxel index, out[4 i + 1 .. 3] = position (cm).  Sample i uses
 * the stream of history i; tracking selects the draw order (exact: one
 * uniform for the voxel; Woodcock: the device's raw word and accept
 * uniform).  Returns 0, or a negative value on invalid input. */
int orc_sample_source(const orc_phantom *ph, uint64_t n, uint64_t seed, int tracking, int wide,
                      int rng, double *out)
{
  const int64_t nvox = (int64_t)ph->nx * ph->ny * ph->nz;
  double *cdf = (double *)malloc(sizeof(double) * (size_t)nvox);
  double acc = 0.0;
  for (int64_t v = 0; v < nvox; ++v) {
    const double a = ph->activity[v];
    if (!(a >= 0.0) || isinf(a)) {
      free(cdf);
      return -3;
    }
    acc += a;
    cdf[v] = acc;
  }
  if (!(acc > 0.0)) {
    free(cdf);
    return -3;
  }
  orc_opts op;
  memset(&op, 0, sizeof op);
  op.tracking = tracking;
  orc_ctx cx;
  memset(&cx, 0, sizeof cx);
  cx.ph = ph;
  cx.op = &op;
  cx.cdf = cdf;
  cx.nvox = nvox;
  for (uint64_t i = 0; i < n; ++i) {
    orc_stream st;
    stream_init(&st, seed, i, 0, wide, rng);
    int64_t iv[3];
    double r[3];
    sample_decay(&cx, &st, iv, r);
    out[4 * i] = (double)(iv[0] + (int64_t)ph->nx * (iv[1] + (int64_t)ph->ny * iv[2]));
    out[4 * i + 1] = r[0];
    out[4 * i + 2] = r[1];
    out[4 * i + 3] = r[2];
  }
  free(cdf);
  return 0;
}

double orc_thomson_inverse(double u) { return sample_thomson(u); }

/* Table-interpolated mass attenuation (cm^2/g) of one process, as the
 * transport sees it. */
double orc_mass_atten_interp(int process, double z, double z_over_a, double e)
{
  double lt[ORC_NGRID];
  for (int i = 0; i < ORC_NGRID; ++i)
    lt[i] = log(orc_mass_atten_closed(process, z, z_over_a, orc_grid_energy(i)));
  int i;
  double f;
  grid_locate(ORC_EGRID_RATIO, e, &i, &f);
  return loglog(lt, i, f);
}

/* Majorant (cm^-1) of a phantom at energy e. */
double orc_majorant(const orc_phantom *ph, double e)
{
  orc_tables *tab = (orc_tables *)malloc(sizeof(orc_tables));
  build_tables(ph, tab, ORC_EGRID_RATIO);
  const double m = eval_major(tab, e);
  free(tab);
  return m;
}

void orc_rotate(double *d, double cost, double uphi) { rotate_dir(d, cost, uphi); }

/* One electron walk for the tests: r (cm) inside the grid, de a unit
 * direction.  Writes up to cap deposits (voxel, MeV) and the escaped
 * energy; returns the number of deposits (which may exceed cap). */
typedef struct {
  int64_t *v;
  double *e;
  int n, cap;
} walk_out;

static void walk_collect(void *user, int64_t v, double e)
{
  walk_out *o = (walk_out *)user;
  if (o->n < o->cap) {
    o->v[o->n] = v;
    o->e[o->n] = e;
  }
  o->n++;
}

int orc_electron_walk(const orc_phantom *ph, const double *i_ev, double cutoff, const double *r,
                      const double *de, double t0, int64_t *v_out, double *e_out, int cap,
                      double *escaped)
{
  const int32_t n[3] = { ph->nx, ph->ny, ph->nz };
  const double h[3] = { ph->dx, ph->dy, ph->dz };
  int64_t iv[3];
  for (int a = 0; a < 3; ++a) {
    int64_t i = (int64_t)floor(r[a] / h[a]);
    iv[a] = i < 0 ? 0 : (i >= n[a] ? n[a] - 1 : i);
  }
  walk_out o = { v_out, e_out, 0, cap };
  *escaped = 0.0;
  if (t0 <= cutoff) {
    walk_collect(&o, iv[0] + (int64_t)n[0] * (iv[1] + (int64_t)n[1] * iv[2]), t0);
    return o.n;
  }
  *escaped = electron_walk(ph, i_ev, cutoff, r, iv, de, t0, walk_collect, &o, NULL);
  return o.n;
}

