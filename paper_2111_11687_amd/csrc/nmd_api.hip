// Host engine and C ABI of the dosimetry library (see include/nmdose.h).
//
// The context owns: a (material, density) palette shared by its phantoms,
// the Klein-Nishina table, per-phantom voxel records, organ labels, alias
// tables, majorant tables and FP64 tallies, and the work-queue and
// deposit-list scratch of the transport kernel.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <unordered_map>
#include <vector>

#include "../../include/nmdose.h"
#include "nmd_internal.hpp"

using namespace nmd;

namespace {

struct DevBuf {
  void *p = nullptr;
  size_t n = 0;
  ~DevBuf() { release(); }
  void release() {
    if (p) (void)hipFree(p);
    p = nullptr;
    n = 0;
  }
  DevBuf() = default;
  DevBuf(const DevBuf &) = delete;
  DevBuf &operator=(const DevBuf &) = delete;
  DevBuf(DevBuf &&o) noexcept : p(o.p), n(o.n) {
    o.p = nullptr;
    o.n = 0;
  }
  DevBuf &operator=(DevBuf &&o) noexcept {
    if (this != &o) {
      release();
      p = o.p;
      n = o.n;
      o.p = nullptr;
      o.n = 0;
    }
    return *this;
  }
  template <class T>
  T *as() const {
    return static_cast<T *>(p);
  }
};

struct Phantom {
  int32_t nx = 0, ny = 0, nz = 0, n_org = 0;
  double dx = 0, dy = 0, dz = 0;  // cm
  uint64_t nvox = 0;
  DevBuf rec, alias, tally, organ, ledger, stats, major, organ_w;  // rec: u16 per voxel
  DevBuf major_w;  // the wide grid's majorant nodes, then its Klein-Nishina nodes
  DevBuf n_done_dev, organ_acc;      // device history counter; organ reduction output
  uint64_t gen = 0;                  // changes whenever the device buffers change
  std::vector<int64_t> organ_count;  // voxels per label 0..n_org
  std::vector<uint8_t> used;         // palette entries present
  uint32_t n_alias = 0;
  bool has_activity = false;
  bool has_label = false;
  double a_ts = 0.0;
  uint64_t n_done = 0;
  uint64_t organ_from = 0;  // histories run before the organ sums O, O2 started
  std::vector<int> pal_mat;  // palette index -> index into this phantom's materials (-1: unused)
  int n_mat = 0;
  std::vector<double> mat_zoa;  // Z/A of each material
  DevBuf e_tab, e_inv_dr, e_slot;  // electron range tables (nmd_set_electrons)
  DevBuf p_cdf, p_guide, p_tab, p_inv_dr, p_slot;  // positron tables (nmd_set_positron)
  int32_t p_on = 0;
  float p_inv_dt = 0.0f, noncol_sigma = 0.0f;
  int32_t em_n = 0;  // gamma + beta emitter (nmd_set_emitter): lines, or 0
  bool em_on = false;
  double em_cum[kMaxLines] = {};
  float em_e[kMaxLines] = {}, em_beta = 0.0f;
  int32_t box0[3] = {0, 0, 0}, box1[3] = {0, 0, 0};  // inner box, voxel indices [box0, box1)
  double out_ratio = 0.0;  // outer majorant / inner majorant (0: no outer region)
  double out_ratio_w = 0.0;  // the same on the wide grid
  bool wide = false;  // an emitter line above 511 keV: the wide grid's tables
  int32_t tracking = NMD_TRACK_GLOBAL;  // NMD_TRACK_* (nmd_set_tracking)
  float e_cut = 0.0f, e_inv_dt = 0.0f;
  uint64_t geom_hash = 0;   // FNV-1a of the voxel records, for checkpoints
  uint64_t act_hash = 0;    // FNV-1a of the alias table, for checkpoints
  double vkg() const { return dx * dy * dz * 1.0e-3; }  // kg per (g/cm^3)
};

struct PalEntry {
  double z, zoa;
  float rho;
  float4 c;  // (cC, cPE, cR, rho)
};

}  // namespace

struct nmd_ctx {
  int device = 0;
  hipStream_t stream = nullptr;
  std::string err;
  std::vector<PalEntry> pal;
  DevBuf d_pal, d_kn, d_queue, d_desc, d_dep_v, d_dep_e, d_dep_r;
  uint32_t dep_lanes = 0;
  std::string arch;                        // device name, for the tuner cache
  std::map<std::string, uint32_t> tuned;   // work-queue chunk per phantom set
  uint32_t last_chunk = 0, last_grid = 0;
  hipStream_t capture = nullptr;           // stream used to capture graphs
  uint64_t next_gen = 1;
  int cu_count = 0;
  float l2emin = 0, inv_dl2 = 0;
  std::map<int, Phantom> ph;
  DevBuf nn_scratch;  // workspace of the denoiser's backward-weight partials
  bool poisoned = false;
  double *noalloc_scratch = nullptr;  // this device's `scratch` (nmd_organ_mean_map_noalloc)
};

namespace {

nmd_status fail(nmd_ctx *c, nmd_status s, const char *fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  if (c) {
    c->err = buf;
    if (s == NMD_E_HIP) c->poisoned = true;
  }
  return s;
}

#define HIP_TRY(ctx, expr)                                                                \
  do {                                                                                    \
    hipError_t e_ = (expr);                                                               \
    if (e_ != hipSuccess)                                                                 \
      return fail(ctx, e_ == hipErrorOutOfMemory ? NMD_E_OOM : NMD_E_HIP, "%s: %s", #expr, \
                  hipGetErrorString(e_));                                                 \
  } while (0)

nmd_status dev_alloc(nmd_ctx *c, DevBuf &b, size_t bytes) {
  DevBuf nb;
  if (bytes) {
    hipError_t e = hipMalloc(&nb.p, bytes);
    if (e != hipSuccess) {
      (void)hipGetLastError();
      return fail(c, NMD_E_OOM, "hipMalloc(%zu bytes): %s", bytes, hipGetErrorString(e));
    }
    nb.n = bytes;
  }
  b = std::move(nb);
  return NMD_OK;
}

// ---- model (host side of the device tables) --------------------------------
double sigma_kn(double e) {
  const double k = e / kMeC2;
  const double a = 1.0 + 2.0 * k;
  const double l = std::log(a);
  return 2.0 * M_PI * kRe * kRe *
         ((1.0 + k) / (k * k) * (2.0 * (1.0 + k) / a - l / k) + l / (2.0 * k) -
          (1.0 + 3.0 * k) / (a * a));
}
double grid_e(int i) { return kEGridMin * std::pow(kEGridRatio, (double)i / (kNGrid - 1)); }
double grid_e_w(int i) { return kEGridMin * std::pow(kEGridRatioW, (double)i / (kNGrid - 1)); }

// Coefficients of one (material, density) pair, FP64: mu_C = cC * N_A
// sigma_KN(E), mu_PE = cPE / E^3, mu_R = cR / E^2 (cm^-1).
void pal_coeffs(double z, double zoa, double rho, double &cc, double &cpe, double &cr) {
  const double sref = sigma_kn(kERef);
  const double a_pe = sref / (kZRef * kZRef * kZRef);
  const double a_r = 0.1 * sref / kZRef;
  cc = rho * zoa;
  cpe = rho * kNA * zoa * a_pe * z * z * z * kERef * kERef * kERef;
  cr = rho * kNA * zoa * a_r * z * kERef * kERef;
}

// ---- electron ranges (host) ------------------------------------------------
// Collision stopping power of electrons (Bethe, ICRU Report 37 form with the
// Moller term, no density effect), MeV cm^2/g, for kinetic energy t (MeV),
// electron fraction zoa and mean excitation energy i_ev.
double electron_stopping(double t, double zoa, double i_ev) {
  const double k = 2.0 * M_PI * kRe * kRe * kMeC2 * kNA;  // MeV cm^2 / mol
  const double tau = t / kMeC2;
  const double g2 = (tau + 1.0) * (tau + 1.0);
  const double beta2 = tau * (tau + 2.0) / g2;
  const double fminus = 1.0 - beta2 + (tau * tau / 8.0 - (2.0 * tau + 1.0) * M_LN2) / g2;
  const double i_rel = i_ev * 1e-6 / kMeC2;
  return k * zoa / beta2 * (std::log(tau * tau * (tau + 2.0) / (2.0 * i_rel * i_rel)) + fminus);
}

constexpr double kETabTop = 0.345;  // MeV, above the largest Compton electron of 0.511 MeV

// Range above the cutoff, R(T) = integral_cut^T dT' / S(T') (g/cm^2), on the
// kETab nodes T_i = cut + i dt up to top, and its inverse T(R) on
// R_j = j dr, for one material; the integral by 3-point Gauss-Legendre on 16
// sub-intervals of every node interval.
void electron_tables(double cut, double top, double zoa, double i_ev, float *r_tab,
                     float *t_tab, float *inv_dr) {
  const int sub = 16, nf = (kETab - 1) * sub;
  const double dt = (top - cut) / (kETab - 1), h = dt / sub;
  const double xg[3] = {-std::sqrt(0.6), 0.0, std::sqrt(0.6)}, wg[3] = {5.0 / 9, 8.0 / 9, 5.0 / 9};
  std::vector<double> rf(nf + 1, 0.0);
  for (int k = 0; k < nf; ++k) {
    const double c = cut + (k + 0.5) * h;
    double acc = 0.0;
    for (int q = 0; q < 3; ++q) acc += wg[q] / electron_stopping(c + 0.5 * h * xg[q], zoa, i_ev);
    rf[k + 1] = rf[k] + 0.5 * h * acc;
  }
  for (int i = 0; i < kETab; ++i) r_tab[i] = (float)rf[i * sub];
  const double rmax = rf[nf], dr = rmax / (kETab - 1);
  int k = 0;
  for (int j = 0; j < kETab; ++j) {
    const double r = std::min(j * dr, rmax);
    while (k < nf - 1 && rf[k + 1] < r) ++k;
    const double f = (r - rf[k]) / (rf[k + 1] - rf[k]);
    t_tab[j] = (float)(cut + (k + std::min(std::max(f, 0.0), 1.0)) * h);
  }
  *inv_dr = (float)(1.0 / dr);
}

// ---- 18F positrons (host) ---------------------------------------------------
constexpr double kF18DaughterZ = 8.0;    // 18O
constexpr double kAlpha = 1.0 / 137.035999084;

// Allowed beta+ spectrum dN/dT (unnormalised): p W (W0 - W)^2 F with W the
// total energy over m_e c^2, p the momentum over m_e c and F the
// non-relativistic Fermi function 2 pi eta / (1 - exp(-2 pi eta)),
// eta = -Z alpha W / p for a positron and a daughter of charge Z.
double beta_plus_density(double t) {
  if (!(t > 0.0) || !(t < kF18T0)) return 0.0;
  const double w = 1.0 + t / kMeC2, w0 = 1.0 + kF18T0 / kMeC2;
  const double p = std::sqrt(w * w - 1.0);
  const double y = 2.0 * M_PI * kF18DaughterZ * kAlpha * w / p;  // -2 pi eta > 0
  return p * w * (w0 - w) * (w0 - w) * (y / std::expm1(y));
}

// The spectrum's CDF on T_i = T0 i / kPosN (3-point Gauss-Legendre on 8
// sub-intervals of each interval), normalised to 1 at T0, and its guide
// table: guide[k] = the last i with cdf[i] <= k / kPosN (Chen and Asau), so
// that a uniform u finds its interval from guide[floor(u kPosN)] in a step
// or two.
void positron_cdf(double *cdf, int32_t *guide) {
  const int sub = 8;
  const double h = kF18T0 / kPosN, hs = h / sub;
  const double xg[3] = {-std::sqrt(0.6), 0.0, std::sqrt(0.6)}, wg[3] = {5.0 / 9, 8.0 / 9, 5.0 / 9};
  cdf[0] = 0.0;
  for (int i = 0; i < kPosN; ++i) {
    double acc = 0.0;
    for (int k = 0; k < sub; ++k) {
      const double c = i * h + (k + 0.5) * hs;
      for (int q = 0; q < 3; ++q) acc += wg[q] * beta_plus_density(c + 0.5 * hs * xg[q]);
    }
    cdf[i + 1] = cdf[i] + 0.5 * hs * acc;
  }
  for (int i = 1; i <= kPosN; ++i) cdf[i] /= cdf[kPosN];
  int i = 0;
  for (int k = 0; k < kPosN; ++k) {
    const double u = (double)k / kPosN;
    while (i < kPosN - 1 && cdf[i + 1] <= u) ++i;
    guide[k] = i;
  }
}

float round_up_f32(double x) {
  float f = (float)x;
  if ((double)f < x) f = std::nextafter(f, INFINITY);
  return f;
}

// Voxel coordinates packed as x | y << 10 | z << 20 (grid limits 1024 x 1024 x 4096).
uint32_t pack_xyz(const Phantom &p, uint32_t v) {
  const uint32_t nx = (uint32_t)p.nx, nxy = nx * (uint32_t)p.ny;
  const uint32_t z = v / nxy, r = v - z * nxy, y = r / nx, x = r - y * nx;
  return x | (y << 10) | (z << 20);
}

nmd_status sync(nmd_ctx *c) {
  HIP_TRY(c, hipStreamSynchronize(c->stream));
  return NMD_OK;
}

nmd_status check_ctx(nmd_ctx *c) {
  if (!c) return NMD_E_INVALID;
  if (c->poisoned) return fail(c, NMD_E_HIP, "context unusable after an earlier HIP error");
  HIP_TRY(c, hipSetDevice(c->device));
  return NMD_OK;
}

Phantom *find(nmd_ctx *c, int32_t id) {
  auto it = c->ph.find(id);
  return it == c->ph.end() ? nullptr : &it->second;
}

PhantomDesc make_desc(int32_t id, const Phantom &p) {
  PhantomDesc d = {};
  d.rec = p.rec.as<uint16_t>();
  d.alias = p.alias.as<uint4>();
  d.tally = p.tally.as<double2>();
  d.organ = p.organ.as<double2>();
  d.ledger = p.ledger.as<double>();
  d.stats = p.stats.as<unsigned long long>();
  d.ln2_major = p.wide ? p.major_w.as<float>() : p.major.as<float>();
  d.wide = p.wide ? 1 : 0;
  d.organ_w = p.organ_w.as<double>();
  d.n_done = p.n_done_dev.as<unsigned long long>();
  d.nx = p.nx;
  d.ny = p.ny;
  d.nz = p.nz;
  d.n_org = p.n_org;
  d.fnx = (float)p.nx;
  d.fny = (float)p.ny;
  d.fnz = (float)p.nz;
  d.dx = (float)p.dx;
  d.dy = (float)p.dy;
  d.dz = (float)p.dz;
  d.inv_dx = (float)(1.0 / p.dx);
  d.inv_dy = (float)(1.0 / p.dy);
  d.inv_dz = (float)(1.0 / p.dz);
  d.n_alias = p.n_alias;
  d.pid = (uint32_t)id;
  // region tracking: the inner box and the outer majorant ratio; under
  // global tracking (or without an outer region) the box is the whole grid
  // and the ratio 0, which the region-tracking kernel reads as one region
  const bool regions = p.tracking == NMD_TRACK_REGIONS && p.out_ratio > 0.0;
  const double h[3] = {p.dx, p.dy, p.dz};
  const int32_t n[3] = {p.nx, p.ny, p.nz};
  for (int a = 0; a < 3; ++a) {
    const int32_t lo = regions ? p.box0[a] : 0, hi = regions ? p.box1[a] : n[a];
    d.b0[a] = (float)lo;
    d.b1[a] = (float)hi;
    d.bcm0[a] = (float)(lo * h[a]);
    d.bcm1[a] = (float)(hi * h[a]);
  }
  const double orat = p.wide ? p.out_ratio_w : p.out_ratio;
  d.out_ratio = regions ? (float)orat : 0.0f;
  d.inv_out_ratio = regions ? (float)(1.0 / orat) : 0.0f;
  d.e_tab = p.e_tab.as<float>();
  d.e_inv_dr = p.e_inv_dr.as<float>();
  d.e_slot = p.e_slot.as<uint8_t>();
  d.e_cut = p.e_cut;
  d.e_inv_dt = p.e_inv_dt;
  d.p_on = p.p_on;
  d.p_inv_dt = p.p_inv_dt;
  d.noncol_sigma = p.noncol_sigma;
  d.p_cdf = p.p_cdf.as<double>();
  d.p_guide = p.p_guide.as<int32_t>();
  d.p_tab = p.p_tab.as<float>();
  d.p_inv_dr = p.p_inv_dr.as<float>();
  d.p_slot = p.p_slot.as<uint8_t>();
  d.em_on = p.em_on ? 1 : 0;
  d.em_n = p.em_n;
  for (int i = 0; i < kMaxLines; ++i) {
    d.em_cum[i] = p.em_cum[i];
    d.em_e[i] = p.em_e[i];
  }
  d.em_beta = p.em_beta;
  return d;
}

nmd_status upload_desc(nmd_ctx *c, int32_t id, Phantom &p) {
  const PhantomDesc d = make_desc(id, p);
  HIP_TRY(c, hipMemcpyAsync(c->d_desc.as<PhantomDesc>() + id, &d, sizeof d, hipMemcpyHostToDevice,
                            c->stream));
  return sync(c);
}

// 64-bit FNV-1a over a byte range, continuing from h.
uint64_t fnv1a(const void *data, size_t n, uint64_t h = 0xcbf29ce484222325ull) {
  const unsigned char *b = static_cast<const unsigned char *>(data);
  for (size_t i = 0; i < n; ++i) {
    h ^= b[i];
    h *= 0x100000001b3ull;
  }
  return h;
}

nmd_status zero_tallies(nmd_ctx *c, Phantom &p) {
  HIP_TRY(c, launch_zero_bytes(p.tally.p, p.tally.n, c->stream));
  HIP_TRY(c, launch_zero_bytes(p.organ.p, p.organ.n, c->stream));
  HIP_TRY(c, launch_zero_bytes(p.ledger.p, p.ledger.n, c->stream));
  HIP_TRY(c, launch_zero_bytes(p.stats.p, p.stats.n, c->stream));
  HIP_TRY(c, launch_set_u64(p.n_done_dev.as<unsigned long long>(), 0ull, c->stream));
  p.n_done = 0;
  p.organ_from = 0;
  return NMD_OK;
}

template <class T>
nmd_status to_host(nmd_ctx *c, std::vector<T> &h, const T *src, uint64_t n) {
  h.resize(n);
  HIP_TRY(c, hipMemcpyAsync(h.data(), src, n * sizeof(T), hipMemcpyDefault, c->stream));
  return sync(c);
}


// ---- runs ------------------------------------------------------------------
constexpr uint32_t kTuneChunks[] = {128, 256, 512, 1024, 2048, 4096};
constexpr uint64_t kTuneMinPerPhantom = 1ull << 22;

struct RunPlan {
  RunParams rp;
  RunIds ids;
  int grid = 0;
  bool debug = false;
  bool electrons = false;   // some phantom of the run walks its Compton electrons
  bool regions = false;     // some phantom of the run has region majorants
  bool auto_chunk = false;  // caller asked for the tuned chunk
  bool tuned = false;       // a tuned chunk was known
  uint32_t abort_after = 0;
  std::string key;          // tuner key: device and phantom shapes
};

std::string tune_key(nmd_ctx *c, const std::vector<int32_t> &ids) {
  std::string k = c->arch;
  char buf[64];
  for (int32_t i : ids) {
    const Phantom &p = c->ph[i];
    snprintf(buf, sizeof buf, "|%dx%dx%d", p.nx, p.ny, p.nz);
    k += buf;
  }
  return k;
}

void load_tune_cache(nmd_ctx *c) {
  const char *path = std::getenv("NMD_TUNE_CACHE");
  if (!path) return;
  FILE *f = std::fopen(path, "r");
  if (!f) return;
  char key[4096];
  unsigned ch;
  while (std::fscanf(f, "%4095s %u", key, &ch) == 2) c->tuned[key] = ch;
  std::fclose(f);
}

void save_tune_cache(nmd_ctx *c) {
  const char *path = std::getenv("NMD_TUNE_CACHE");
  if (!path) return;
  FILE *f = std::fopen(path, "w");
  if (!f) return;
  for (auto &kv : c->tuned) std::fprintf(f, "%s %u\n", kv.first.c_str(), kv.second);
  std::fclose(f);
}

// Split the run's histories into chunks of `chunk` for the work queue.
void set_chunk(RunPlan &pl, uint64_t n, uint32_t chunk) {
  pl.rp.chunk = chunk;
  uint64_t total = 0;
  for (int i = 0; i < pl.rp.n_ph; ++i) {
    pl.rp.slot[i].n_hist = n;
    pl.rp.slot[i].chunk0 = total;
    total += (n + chunk - 1) / chunk;
  }
  pl.rp.total_chunks = total;
}

nmd_status plan_run(nmd_ctx *c, int32_t id, uint64_t n, uint64_t seed, const nmd_run_opts *opts_in,
                    RunPlan &pl) {
  nmd_run_opts o;
  if (opts_in)
    o = *opts_in;
  else
    nmd_run_opts_default(&o);
  if (o.photons_per_decay < 1 || o.photons_per_decay > 2)
    return fail(c, NMD_E_INVALID, "photons_per_decay must be 1 or 2");
  if (o.process_mask > 7) return fail(c, NMD_E_INVALID, "process_mask must be <= 7");
  if (!(o.photon_cutoff_mev >= 0.001f && o.photon_cutoff_mev <= 0.511f))
    return fail(c, NMD_E_INVALID, "photon cutoff must lie in [0.001, 0.511] MeV");
  if (o.source_kind > 1) return fail(c, NMD_E_INVALID, "source_kind must be 0 or 1");
  float pd[3] = {o.pencil_dir[0], o.pencil_dir[1], o.pencil_dir[2]};
  if (o.source_kind == 1) {
    const double nn =
        std::sqrt((double)pd[0] * pd[0] + (double)pd[1] * pd[1] + (double)pd[2] * pd[2]);
    if (!(nn > 0) || !std::isfinite(nn)) return fail(c, NMD_E_INVALID, "pencil_dir must be nonzero");
    for (int a = 0; a < 3; ++a) pd[a] = (float)(pd[a] / nn);
  }
  std::vector<int32_t> ids;
  if (id == -1) {
    for (auto &kv : c->ph)
      if (kv.second.has_activity || o.source_kind == 1) ids.push_back(kv.first);
    if (ids.empty()) return fail(c, NMD_E_STATE, "no phantom has an activity map");
    if (o.history_records) return fail(c, NMD_E_INVALID, "history_records needs a single phantom");
    // largest first: the work queue hands out a phantom's chunks in this
    // order, so the launch ends on the cheapest histories.  A history's cost
    // grows with the path a photon takes to leave the grid; the grid's
    // diagonal stands for it.  Results do not depend on the order (each
    // history's stream is keyed by seed, phantom and history).
    auto diag = [&](int32_t i) {
      const Phantom &p = c->ph[i];
      const double a = p.nx * p.dx, b = p.ny * p.dy, d = p.nz * p.dz;
      return a * a + b * b + d * d;
    };
    std::stable_sort(ids.begin(), ids.end(),
                     [&](int32_t x, int32_t y) { return diag(x) > diag(y); });
  } else {
    Phantom *p = find(c, id);
    if (!p) return fail(c, NMD_E_STATE, "phantom %d is not registered", id);
    if (o.source_kind == 0 && !p->has_activity)
      return fail(c, NMD_E_STATE, "phantom %d has no activity map", id);
    ids.push_back(id);
  }
  if (o.source_kind == 1) {
    for (int32_t i : ids) {
      const Phantom &p = c->ph[i];
      const double L[3] = {p.nx * p.dx, p.ny * p.dy, p.nz * p.dz};
      for (int a = 0; a < 3; ++a)
        if (!(o.pencil_origin_cm[a] >= 0.0f && o.pencil_origin_cm[a] < L[a]))
          return fail(c, NMD_E_INVALID, "pencil origin must lie inside the grid");
    }
  }
  int n_slots = 1;
  for (int32_t i : ids) n_slots = std::max(n_slots, c->ph[i].n_org + 1);
  pl.debug = o.history_records != nullptr;
  pl.electrons = false;
  for (int32_t i : ids)
    pl.electrons = pl.electrons || c->ph[i].e_cut > 0.0f || c->ph[i].p_on || c->ph[i].em_on;
  pl.regions = false;
  for (int32_t i : ids)
    pl.regions = pl.regions ||
                 (c->ph[i].tracking == NMD_TRACK_REGIONS && c->ph[i].out_ratio > 0.0);
  const int per_cu =
      transport_occupancy_blocks_per_cu(pl.debug, pl.electrons, pl.regions, n_slots);
  uint32_t grid = o.grid_blocks ? o.grid_blocks : (uint32_t)(c->cu_count * per_cu);
  grid = std::max<uint32_t>(1, std::min<uint32_t>(grid, 8192));
  pl.grid = (int)grid;
  const uint32_t lanes = grid * kBlock;
  if (lanes > c->dep_lanes) {
    nmd_status s;
    if ((s = dev_alloc(c, c->d_dep_v, (size_t)lanes * kDepCap * sizeof(uint32_t))) ||
        (s = dev_alloc(c, c->d_dep_e, (size_t)lanes * kDepCap * sizeof(double))) ||
        (s = dev_alloc(c, c->d_dep_r, (size_t)lanes * kDepCap * sizeof(uint32_t)))) {
      c->dep_lanes = 0;
      return s;
    }
    c->dep_lanes = lanes;
  }
  pl.key = tune_key(c, ids);
  if (pl.regions) pl.key += "|regions";
  pl.auto_chunk = o.chunk == 0;
  uint32_t chunk = o.chunk;
  if (chunk == 0) {
    auto it = c->tuned.find(pl.key);
    pl.tuned = it != c->tuned.end();
    if (pl.tuned) {
      chunk = it->second;
    } else {
      // enough claims per wave to balance, few enough to keep the queue cold
      const uint64_t waves = (uint64_t)grid * kWavesPerBlock;
      uint64_t ch = n * ids.size() / (waves * 16);
      chunk = (uint32_t)std::max<uint64_t>(64, std::min<uint64_t>(ch, 4096));
    }
  }
  RunParams &rp = pl.rp;
  rp = RunParams{};
  rp.desc = c->d_desc.as<PhantomDesc>();
  rp.n_ph = (int32_t)ids.size();
  pl.ids.n = (int32_t)ids.size();
  for (size_t i = 0; i < ids.size(); ++i) {
    rp.slot[i].id = ids[i];
    pl.ids.id[i] = ids[i];
  }
  set_chunk(pl, n, chunk);
  pl.abort_after = o.abort_after_chunks;
  rp.abort_after = o.abort_after_chunks;
  rp.seed_lo = (uint32_t)seed;
  rp.seed_hi = (uint32_t)(seed >> 32);
  rp.nph = o.source_kind == 1 ? 1u : o.photons_per_decay;
  rp.mask = o.process_mask;
  rp.max_real = o.max_real_events;
  rp.cutoff = o.photon_cutoff_mev;
  rp.source_kind = o.source_kind;
  for (int a = 0; a < 3; ++a) {
    rp.po[a] = o.pencil_origin_cm[a];
    rp.pd[a] = pd[a];
  }
  rp.palette = c->d_pal.as<float4>();
  rp.n_pal = (int32_t)c->pal.size();
  rp.ln2_kn = c->d_kn.as<float>();
  rp.l2emin = c->l2emin;
  rp.inv_dl2 = c->inv_dl2;
  rp.n_slots = n_slots;
  rp.n_lanes = lanes;
  rp.hist_rec = o.history_records;
  return NMD_OK;
}

// Enqueue one run: clear the queue, transport, advance the history
// counters.  Host mirrors of the counters advance at enqueue time.
nmd_status enqueue_run(nmd_ctx *c, RunPlan &pl, unsigned long long *queue, uint32_t *dep_v,
                       double *dep_e, uint32_t *dep_r, hipStream_t st, bool advance = true) {
  pl.rp.queue = queue;
  pl.rp.dep_v = dep_v;
  pl.rp.dep_e = dep_e;
  pl.rp.dep_r = dep_r;
  HIP_TRY(c, launch_zero_bytes(queue, 2 * sizeof(unsigned long long), st));
  HIP_TRY(c, launch_transport(pl.rp, pl.grid, pl.debug, pl.electrons, pl.regions, st));
  if (!advance) return NMD_OK;
  uint64_t n = pl.rp.n_ph ? pl.rp.slot[0].n_hist : 0;
  HIP_TRY(c, launch_advance(pl.rp.desc, pl.ids, n, st));
  for (int i = 0; i < pl.ids.n; ++i) c->ph[pl.ids.id[i]].n_done += n;
  return NMD_OK;
}

// Scoring buffers of one phantom for a run that may be stopped by the abort
// hook: the run scores into these, and they are added to the phantom's own
// only once it has finished, so a stopped run leaves no trace.
struct RunScratch {
  DevBuf tally, organ, ledger, stats;
};

// A run with the abort hook armed: transport into zeroed scratch scoring
// buffers (through a copy of the descriptor table that points at them),
// then, if the hook did not fire, add them to the phantoms' tallies and
// advance the history counters.  On NMD_E_ABORTED the phantoms are as
// before the call.
nmd_status run_abortable(nmd_ctx *c, RunPlan &pl) {
  nmd_status s;
  std::vector<RunScratch> scr(pl.ids.n);
  DevBuf desc;
  if ((s = dev_alloc(c, desc, c->d_desc.n))) return s;
  HIP_TRY(c, hipMemcpyAsync(desc.p, c->d_desc.p, c->d_desc.n, hipMemcpyDeviceToDevice,
                            c->stream));
  for (int i = 0; i < pl.ids.n; ++i) {
    const int32_t id = pl.ids.id[i];
    Phantom &p = c->ph[id];
    RunScratch &r = scr[i];
    if ((s = dev_alloc(c, r.tally, p.tally.n)) || (s = dev_alloc(c, r.organ, p.organ.n)) ||
        (s = dev_alloc(c, r.ledger, p.ledger.n)) || (s = dev_alloc(c, r.stats, p.stats.n)))
      return s;
    for (DevBuf *b : {&r.tally, &r.organ, &r.ledger, &r.stats})
      HIP_TRY(c, launch_zero_bytes(b->p, b->n, c->stream));
    PhantomDesc d = make_desc(id, p);
    d.tally = r.tally.as<double2>();
    d.organ = r.organ.as<double2>();
    d.ledger = r.ledger.as<double>();
    d.stats = r.stats.as<unsigned long long>();
    HIP_TRY(c, hipMemcpyAsync(desc.as<PhantomDesc>() + id, &d, sizeof d, hipMemcpyHostToDevice,
                              c->stream));
  }
  pl.rp.desc = desc.as<PhantomDesc>();
  if ((s = enqueue_run(c, pl, c->d_queue.as<unsigned long long>(), c->d_dep_v.as<uint32_t>(),
                       c->d_dep_e.as<double>(), c->d_dep_r.as<uint32_t>(), c->stream, false)))
    return s;
  pl.rp.desc = c->d_desc.as<PhantomDesc>();
  unsigned long long q[2] = {0, 0};
  HIP_TRY(c, hipMemcpyAsync(q, c->d_queue.p, sizeof q, hipMemcpyDeviceToHost, c->stream));
  if ((s = sync(c))) return s;
  if (q[1]) return fail(c, NMD_E_ABORTED, "run stopped by the abort hook; tallies unchanged");
  for (int i = 0; i < pl.ids.n; ++i) {
    Phantom &p = c->ph[pl.ids.id[i]];
    RunScratch &r = scr[i];
    HIP_TRY(c, launch_add_f64(p.tally.as<double>(), r.tally.as<double>(), p.nvox * 2, c->stream));
    HIP_TRY(c, launch_add_f64(p.organ.as<double>(), r.organ.as<double>(),
                              (uint64_t)(p.n_org + 1) * 2, c->stream));
    HIP_TRY(c, launch_add_f64(p.ledger.as<double>(), r.ledger.as<double>(), NMD_LEDGER_N,
                              c->stream));
    HIP_TRY(c, launch_add_stats(p.stats.as<unsigned long long>(),
                                r.stats.as<unsigned long long>(), c->stream));
  }
  const uint64_t n = pl.rp.n_ph ? pl.rp.slot[0].n_hist : 0;
  HIP_TRY(c, launch_advance(pl.rp.desc, pl.ids, n, c->stream));
  for (int i = 0; i < pl.ids.n; ++i) c->ph[pl.ids.id[i]].n_done += n;
  return sync(c);
}

nmd_status enqueue_organ_reduce(nmd_ctx *c, Phantom &p, hipStream_t st) {
  HIP_TRY(c, launch_zero_bytes(p.organ_acc.p, p.organ_acc.n, st));
  HIP_TRY(c, launch_organ_reduce(p.rec.as<uint16_t>(), c->d_pal.as<float4>(),
                                 p.tally.as<double2>(), p.nvox, p.n_org,
                                 p.n_done_dev.as<unsigned long long>(), p.vkg(), p.a_ts,
                                 p.organ_acc.as<double>(), st));
  return NMD_OK;
}

}  // namespace

struct nmd_graph {
  nmd_ctx *c = nullptr;
  hipGraph_t g = nullptr;
  hipGraphExec_t ge = nullptr;
  RunIds ids = {};
  uint64_t n = 0;
  std::vector<uint64_t> gen;  // phantom generations when captured
  DevBuf queue, dep_v, dep_e, dep_r;
};

namespace {
}  // namespace

// ---- allocation-free organ means ---------------------------------------------
// Device scratch of nmd_organ_mean_map_noalloc: one FP64 partial sum per organ
// label, 2 KiB on every device the library runs on, held until the process
// ends.  Host code never passes `scratch` itself (its host-side name is not a
// device address): the device address comes from hipGetSymbolAddress, taken
// once per device with that device current, when the first context on it is
// created.
namespace {
constexpr int kNoallocSlots = kMaxOrganSlots;
__device__ __align__(256) double scratch[kNoallocSlots];
std::mutex g_scratch_mu;
std::map<int, double *> g_scratch_ptr;  // device -> address of `scratch` there

nmd_status bind_noalloc_scratch(nmd_ctx *c) {
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  auto it = g_scratch_ptr.find(c->device);
  if (it == g_scratch_ptr.end()) {
    void *ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !ptr) {
      (void)hipGetLastError();
      return fail(c, NMD_E_HIP, "hipGetSymbolAddress(scratch): %s", hipGetErrorString(e));
    }
    it = g_scratch_ptr.emplace(c->device, static_cast<double *>(ptr)).first;
  }
  c->noalloc_scratch = it->second;
  return NMD_OK;
}
}  // namespace

// ============================================================================
// C ABI
// ============================================================================
extern "C" {

void nmd_run_opts_default(nmd_run_opts *o) {
  if (!o) return;
  std::memset(o, 0, sizeof *o);
  o->photons_per_decay = 2;
  o->process_mask = 7;
  o->max_real_events = 0;
  o->photon_cutoff_mev = 0.010f;
  o->source_kind = 0;
  o->pencil_dir[0] = 1.0f;
}

nmd_status nmd_create(nmd_ctx **out, int device, void *stream) {
  if (!out) return NMD_E_INVALID;
  *out = nullptr;
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || device < 0 || device >= ndev) {
    (void)hipGetLastError();
    return NMD_E_INVALID;
  }
  nmd_ctx *c = new nmd_ctx();
  c->device = device;
  c->stream = (hipStream_t)stream;
  if (hipSetDevice(device) != hipSuccess) {
    delete c;
    return NMD_E_HIP;
  }
  hipDeviceProp_t prop;
  if (hipGetDeviceProperties(&prop, device) != hipSuccess) {
    delete c;
    return NMD_E_HIP;
  }
  c->cu_count = prop.multiProcessorCount;
  if (bind_noalloc_scratch(c) != NMD_OK) {
    delete c;
    return NMD_E_HIP;
  }
  c->arch = prop.gcnArchName;
  for (char &ch : c->arch)
    if (ch == ' ' || ch == '|') ch = '_';
  load_tune_cache(c);
  c->l2emin = (float)std::log2(kEGridMin);
  c->inv_dl2 = (float)((kNGrid - 1) / std::log2(kEGridRatio));
  std::vector<float> kn(kNGrid);
  for (int i = 0; i < kNGrid; ++i) kn[i] = (float)std::log2(kNA * sigma_kn(grid_e(i)));
  nmd_status s;
  if ((s = dev_alloc(c, c->d_kn, kNGrid * sizeof(float))) ||
      (s = dev_alloc(c, c->d_pal, kMaxPalette * sizeof(float4))) ||
      (s = dev_alloc(c, c->d_queue, 2 * sizeof(unsigned long long))) ||
      (s = dev_alloc(c, c->d_desc, kMaxPhantoms * sizeof(PhantomDesc)))) {
    delete c;
    return s;
  }
  if (hipMemcpy(c->d_kn.p, kn.data(), kNGrid * sizeof(float), hipMemcpyHostToDevice) !=
      hipSuccess) {
    delete c;
    return NMD_E_HIP;
  }
  *out = c;
  return NMD_OK;
}

void nmd_destroy(nmd_ctx *c) {
  if (!c) return;
  (void)hipSetDevice(c->device);
  if (c->stream) (void)hipStreamSynchronize(c->stream);
  else (void)hipDeviceSynchronize();
  if (c->capture) (void)hipStreamDestroy(c->capture);
  delete c;
}

const char *nmd_last_error(const nmd_ctx *c) {
  if (!c) return "no context";
  return c->err.c_str();
}

nmd_status nmd_set_stream(nmd_ctx *c, void *stream) {
  nmd_status s = check_ctx(c);
  if (s) return s;
  c->stream = (hipStream_t)stream;
  return NMD_OK;
}

nmd_status nmd_set_phantom(nmd_ctx *c, int32_t id, int32_t nx, int32_t ny, int32_t nz, float dx_mm,
                           float dy_mm, float dz_mm, const float *density, const uint8_t *material,
                           const uint8_t *label, int32_t n_organs, const nmd_material *mats,
                           int32_t n_mat) {
  nmd_status s = check_ctx(c);
  if (s) return s;
  if (id < 0 || id >= kMaxPhantoms) return fail(c, NMD_E_INVALID, "phantom id %d out of 0..63", id);
  if (nx < 1 || ny < 1 || nz < 1)
    return fail(c, NMD_E_SHAPE, "dimensions must be >= 1 (%d, %d, %d)", nx, ny, nz);
  const uint64_t nvox = (uint64_t)nx * ny * nz;
  if (nvox >= (1ull << 31)) return fail(c, NMD_E_SHAPE, "nx*ny*nz must be < 2^31");
  if (nx > 1024 || ny > 1024 || nz > 4096)
    return fail(c, NMD_E_UNSUPPORTED, "grids are limited to 1024 x 1024 x 4096 voxels");
  if (!(dx_mm > 0 && dy_mm > 0 && dz_mm > 0) || !std::isfinite(dx_mm) || !std::isfinite(dy_mm) ||
      !std::isfinite(dz_mm))
    return fail(c, NMD_E_INVALID, "voxel sizes must be finite and > 0");
  if (!density || !material) return fail(c, NMD_E_INVALID, "density and material are required");
  if (!mats || n_mat < 1 || n_mat > 8) return fail(c, NMD_E_INVALID, "n_materials must be 1..8");
  if (n_organs < 0 || n_organs > 255) return fail(c, NMD_E_INVALID, "n_organs must be 0..255");
  for (int m = 0; m < n_mat; ++m)
    if (!(mats[m].z_eff > 0 && mats[m].z_eff < 200 && mats[m].z_over_a > 0 &&
          mats[m].z_over_a <= 1.0))
      return fail(c, NMD_E_INVALID, "material %d: need 0 < z_eff < 200 and 0 < Z/A <= 1", m);

  std::vector<float> h_rho;
  std::vector<uint8_t> h_mat, h_lab;
  if ((s = to_host(c, h_rho, density, nvox)) || (s = to_host(c, h_mat, material, nvox))) return s;
  if (label && (s = to_host(c, h_lab, label, nvox))) return s;

  // palette (strong guarantee: work on a copy)
  std::vector<PalEntry> pal = c->pal;
  std::unordered_map<uint64_t, int> key_to_q;
  std::vector<int> mat_pal_base(n_mat);
  std::vector<uint16_t> rec(nvox);
  std::vector<uint8_t> used(kMaxPalette, 0);
  std::vector<int> pal_mat(kMaxPalette, -1);
  uint64_t last_key = ~0ull;
  int last_q = 0;
  for (uint64_t v = 0; v < nvox; ++v) {
    const float r = h_rho[v];
    const uint8_t m = h_mat[v];
    if (!(r >= 1e-6f) || !std::isfinite(r))
      return fail(c, NMD_E_INVALID, "density[%llu] = %g is not finite and >= 1e-6",
                  (unsigned long long)v, (double)r);
    if (m >= n_mat)
      return fail(c, NMD_E_INVALID, "material[%llu] = %d >= n_materials", (unsigned long long)v, m);
    uint32_t rb;
    std::memcpy(&rb, &r, 4);
    const uint64_t key = ((uint64_t)m << 32) | rb;
    if (key != last_key) {
      auto it = key_to_q.find(key);
      if (it == key_to_q.end()) {
        int q = -1;
        for (size_t i = 0; i < pal.size(); ++i)
          if (pal[i].z == mats[m].z_eff && pal[i].zoa == mats[m].z_over_a && pal[i].rho == r) {
            q = (int)i;
            break;
          }
        if (q < 0) {
          if (pal.size() >= (size_t)kMaxPalette)
            return fail(c, NMD_E_UNSUPPORTED,
                        "more than %d distinct (material, density) pairs in this context",
                        kMaxPalette);
          PalEntry e;
          e.z = mats[m].z_eff;
          e.zoa = mats[m].z_over_a;
          e.rho = r;
          double cc, cpe, cr;
          pal_coeffs(e.z, e.zoa, (double)r, cc, cpe, cr);
          e.c = make_float4((float)cc, (float)cpe, (float)cr, r);
          q = (int)pal.size();
          pal.push_back(e);
        }
        it = key_to_q.emplace(key, q).first;
      }
      last_key = key;
      last_q = it->second;
    }
    rec[v] = (uint16_t)(last_q | (label ? (uint32_t)h_lab[v] << 8 : 0u));
    used[last_q] = 1;
    pal_mat[last_q] = m;
  }
  std::vector<int64_t> count(n_organs + 1, 0);
  if (label) {
    for (uint64_t v = 0; v < nvox; ++v) {
      if (h_lab[v] > n_organs)
        return fail(c, NMD_E_INVALID, "organ_label[%llu] = %d > n_organs", (unsigned long long)v,
                    h_lab[v]);
      count[h_lab[v]]++;
    }
  }

  Phantom p;
  p.nx = nx;
  p.ny = ny;
  p.nz = nz;
  p.n_org = n_organs;
  p.dx = dx_mm / 10.0;
  p.dy = dy_mm / 10.0;
  p.dz = dz_mm / 10.0;
  p.nvox = nvox;
  p.organ_count = count;
  p.used = used;
  p.pal_mat = pal_mat;
  p.n_mat = n_mat;
  for (int m = 0; m < n_mat; ++m) p.mat_zoa.push_back(mats[m].z_over_a);
  {
    const int32_t hd[3] = {nx, ny, nz};
    uint64_t h = fnv1a(hd, sizeof hd);
    h = fnv1a(rec.data(), rec.size() * sizeof(uint16_t), h);
    for (int q = 0; q < kMaxPalette; ++q)
      if (used[q]) h = fnv1a(&pal[q].c, sizeof(float4), h);
    p.geom_hash = h;
  }

  // majorant nodes: max over this phantom's pairs of the total attenuation,
  // on the pair's grid (maj) and on the wide grid (maj_w, followed by the
  // wide grid's Klein-Nishina nodes)
  std::vector<float> maj(kNGrid), maj_w(2 * kNGrid);
  for (int i = 0; i < 2 * kNGrid; ++i) {
    const bool w = i >= kNGrid;
    const double e = w ? grid_e_w(i - kNGrid) : grid_e(i);
    const double s_na = kNA * sigma_kn(e);
    double mx = 0.0;
    for (size_t q = 0; q < pal.size(); ++q) {
      if (!used[q]) continue;
      double cc, cpe, cr;
      pal_coeffs(pal[q].z, pal[q].zoa, (double)pal[q].rho, cc, cpe, cr);
      const double mu = cc * s_na + cpe / (e * e * e) + cr / (e * e);
      mx = std::max(mx, mu);
    }
    (w ? maj_w[i - kNGrid] : maj[i]) = round_up_f32(std::log2(mx));
    if (w) maj_w[i] = (float)std::log2(s_na);
  }
  // the inner box: the bounding box of the voxels at least kInnerRho dense;
  // the (material, density) pairs outside it set the outer majorant
  int32_t b0[3] = {nx, ny, nz}, b1[3] = {0, 0, 0};
  for (int32_t k = 0, v = 0; k < nz; ++k)
    for (int32_t j = 0; j < ny; ++j)
      for (int32_t i = 0; i < nx; ++i, ++v)
        if (h_rho[v] >= kInnerRho) {
          b0[0] = std::min(b0[0], i);
          b0[1] = std::min(b0[1], j);
          b0[2] = std::min(b0[2], k);
          b1[0] = std::max(b1[0], i + 1);
          b1[1] = std::max(b1[1], j + 1);
          b1[2] = std::max(b1[2], k + 1);
        }
  if (b1[0] == 0) {  // nothing that dense: one region, the whole grid
    b0[0] = b0[1] = b0[2] = 0;
    b1[0] = nx;
    b1[1] = ny;
    b1[2] = nz;
  }
  std::vector<uint8_t> used_out(kMaxPalette, 0);
  bool any_out = false;
  for (int32_t k = 0, v = 0; k < nz; ++k)
    for (int32_t j = 0; j < ny; ++j)
      for (int32_t i = 0; i < nx; ++i, ++v)
        if (i < b0[0] || i >= b1[0] || j < b0[1] || j >= b1[1] || k < b0[2] || k >= b1[2]) {
          used_out[rec[v] & 0xFFu] = 1;
          any_out = true;
        }
  // the outer majorant is out_ratio times the inner one: the largest ratio,
  // over the energy nodes, of the outer voxels' attenuation to the inner
  // majorant node (log-log interpolation keeps the bound between nodes),
  // widened by 2^-16 for the FP32 product
  double ratio = 0.0, ratio_w = 0.0;
  for (int i = 0; any_out && i < 2 * kNGrid; ++i) {
    const bool w = i >= kNGrid;
    const double e = w ? grid_e_w(i - kNGrid) : grid_e(i);
    const double s_na = kNA * sigma_kn(e);
    double mx = 0.0;
    for (size_t q = 0; q < pal.size(); ++q) {
      if (!used_out[q]) continue;
      double cc, cpe, cr;
      pal_coeffs(pal[q].z, pal[q].zoa, (double)pal[q].rho, cc, cpe, cr);
      mx = std::max(mx, cc * s_na + cpe / (e * e * e) + cr / (e * e));
    }
    if (w)
      ratio_w = std::max(ratio_w, mx / std::exp2((double)maj_w[i - kNGrid]));
    else
      ratio = std::max(ratio, mx / std::exp2((double)maj[i]));
  }
  p.out_ratio = any_out ? ratio * (1.0 + 1.0 / 65536.0) : 0.0;
  p.out_ratio_w = any_out ? ratio_w * (1.0 + 1.0 / 65536.0) : 0.0;
  for (int a = 0; a < 3; ++a) {
    p.box0[a] = b0[a];
    p.box1[a] = b1[a];
  }
  std::vector<double> ow(n_organs + 1, 0.0);
  for (int o = 0; o <= n_organs; ++o)
    ow[o] = count[o] > 0 ? kJPerMeV / (p.vkg() * (double)count[o]) : 0.0;

  p.has_label = label != nullptr;
  if ((s = dev_alloc(c, p.rec, nvox * sizeof(uint16_t))) || (s = dev_alloc(c, p.tally, nvox * sizeof(double2))) ||
      (s = dev_alloc(c, p.organ, (n_organs + 1) * sizeof(double2))) ||
      (s = dev_alloc(c, p.ledger, 8 * sizeof(double))) ||
      (s = dev_alloc(c, p.stats, 16 * sizeof(unsigned long long))) ||
      (s = dev_alloc(c, p.major, kNGrid * sizeof(float))) ||
      (s = dev_alloc(c, p.major_w, 2 * kNGrid * sizeof(float))) ||
      (s = dev_alloc(c, p.organ_w, (n_organs + 1) * sizeof(double))) ||
      (s = dev_alloc(c, p.n_done_dev, 2 * sizeof(unsigned long long))) ||
      (s = dev_alloc(c, p.organ_acc, (n_organs + 1) * 2 * sizeof(double))))
    return s;
  p.gen = c->next_gen++;
  HIP_TRY(c, hipMemcpyAsync(p.rec.p, rec.data(), nvox * sizeof(uint16_t), hipMemcpyHostToDevice,
                            c->stream));
  HIP_TRY(c, hipMemcpyAsync(p.major.p, maj.data(), kNGrid * sizeof(float), hipMemcpyHostToDevice,
                            c->stream));
  HIP_TRY(c, hipMemcpyAsync(p.major_w.p, maj_w.data(), 2 * kNGrid * sizeof(float),
                            hipMemcpyHostToDevice, c->stream));

  HIP_TRY(c, hipMemcpyAsync(p.organ_w.p, ow.data(), ow.size() * sizeof(double),
                            hipMemcpyHostToDevice, c->stream));
  std::vector<float4> pal_dev(pal.size());
  for (size_t i = 0; i < pal.size(); ++i) pal_dev[i] = pal[i].c;
  HIP_TRY(c, hipMemcpyAsync(c->d_pal.p, pal_dev.data(), pal_dev.size() * sizeof(float4),
                            hipMemcpyHostToDevice, c->stream));
  if ((s = zero_tallies(c, p))) return s;
  if ((s = sync(c))) return s;
  c->pal = pal;
  c->ph[id] = std::move(p);
  return upload_desc(c, id, c->ph[id]);
}

nmd_status nmd_set_activity(nmd_ctx *c, int32_t id, const float *act, double total_bq) {
  nmd_status s = check_ctx(c);
  if (s) return s;
  Phantom *p = find(c, id);
  if (!p) return fail(c, NMD_E_STATE, "phantom %d is not registered", id);
  if (!act) return fail(c, NMD_E_INVALID, "activity is required");
  std::vector<float> a;
  if ((s = to_host(c, a, act, p->nvox))) return s;
  double sum = 0.0;
  std::vector<uint32_t> nz;
  for (uint64_t v = 0; v < p->nvox; ++v) {
    const float x = a[v];
    if (!(x >= 0.0f) || !std::isfinite(x))
      return fail(c, NMD_E_INVALID, "activity[%llu] = %g is not finite and >= 0",
                  (unsigned long long)v, (double)x);
    if (x > 0.0f) {
      nz.push_back((uint32_t)v);
      sum += x;
    }
  }
  if (!(sum > 0.0)) return fail(c, NMD_E_INVALID, "activity map is all zero");
  // Vose's alias table over the voxels with activity, in FP64.
  const size_t n = nz.size();
  std::vector<double> q(n);
  for (size_t i = 0; i < n; ++i) q[i] = (double)a[nz[i]] * (double)n / sum;
  std::vector<uint32_t> small, large;
  small.reserve(n);
  large.reserve(n);
  for (size_t i = 0; i < n; ++i) (q[i] < 1.0 ? small : large).push_back((uint32_t)i);
  std::vector<double> prob(n, 1.0);
  std::vector<uint32_t> alias(n);
  for (size_t i = 0; i < n; ++i) alias[i] = (uint32_t)i;
  while (!small.empty() && !large.empty()) {
    const uint32_t l = small.back();
    small.pop_back();
    const uint32_t g = large.back();
    prob[l] = q[l];
    alias[l] = g;
    q[g] = (q[g] + q[l]) - 1.0;
    if (q[g] < 1.0) {
      large.pop_back();
      small.push_back(g);
    }
  }
  // leftovers are 1 up to rounding
  std::vector<uint4> tab(n);
  for (size_t i = 0; i < n; ++i) {
    float pr = (float)prob[i];
    uint32_t pb;
    std::memcpy(&pb, &pr, 4);
    tab[i] = make_uint4(pb, pack_xyz(*p, nz[i]), pack_xyz(*p, nz[alias[i]]), 0u);
  }
  DevBuf d;
  if ((s = dev_alloc(c, d, n * sizeof(uint4)))) return s;
  HIP_TRY(c, hipMemcpyAsync(d.p, tab.data(), n * sizeof(uint4), hipMemcpyHostToDevice, c->stream));
  if ((s = sync(c))) return s;
  p->alias = std::move(d);
  p->act_hash = fnv1a(tab.data(), tab.size() * sizeof(uint4));
  p->gen = c->next_gen++;
  p->n_alias = (uint32_t)n;
  p->has_activity = true;
  p->a_ts = total_bq > 0.0 ? total_bq : sum * (p->dx * p->dy * p->dz);
  if ((s = zero_tallies(c, *p))) return s;
  return upload_desc(c, id, *p);
}

nmd_status nmd_set_electrons(nmd_ctx *c, int32_t id, double cutoff_mev,
                             const double *mean_excitation_ev) {
  nmd_status s = check_ctx(c);
  if (s) return s;
  Phantom *p = find(c, id);
  if (!p) return fail(c, NMD_E_STATE, "phantom %d is not registered", id);
  if (cutoff_mev == 0.0) {
    p->e_tab.release();
    p->e_inv_dr.release();
    p->e_slot.release();
    p->e_cut = 0.0f;
    p->e_inv_dt = 0.0f;
  } else {
    if (!(cutoff_mev >= 0.001 && cutoff_mev <= 0.3))
      return fail(c, NMD_E_INVALID, "electron cutoff must be 0 or lie in [0.001, 0.3] MeV");
    if (p->wide)
      return fail(c, NMD_E_UNSUPPORTED, "the emitter has a line above 0.511 MeV: the electron "
                  "range tables end below its Compton electrons");
    if (!mean_excitation_ev)
      return fail(c, NMD_E_INVALID, "mean excitation energies are required");
    for (int m = 0; m < p->n_mat; ++m)
      if (!(mean_excitation_ev[m] > 1.0 && mean_excitation_ev[m] < 1.0e4))
        return fail(c, NMD_E_INVALID, "mean excitation energy of material %d must lie in "
                    "(1, 10^4) eV", m);
    const float cut = (float)cutoff_mev;
    std::vector<float> tab((size_t)kMaxMaterials * 2 * kETab, 0.0f), inv_dr(kMaxMaterials, 0.0f);
    for (int m = 0; m < p->n_mat; ++m)
      electron_tables((double)cut, kETabTop, p->mat_zoa[m], mean_excitation_ev[m],
                      &tab[(size_t)m * 2 * kETab], &tab[(size_t)m * 2 * kETab + kETab], &inv_dr[m]);
    std::vector<uint8_t> slot(kMaxPalette, 0);
    for (int q = 0; q < kMaxPalette; ++q) slot[q] = (uint8_t)std::max(p->pal_mat[q], 0);
    DevBuf dt, dr, ds;
    if ((s = dev_alloc(c, dt, tab.size() * sizeof(float))) ||
        (s = dev_alloc(c, dr, inv_dr.size() * sizeof(float))) ||
        (s = dev_alloc(c, ds, slot.size())))
      return s;
    HIP_TRY(c, hipMemcpyAsync(dt.p, tab.data(), dt.n, hipMemcpyHostToDevice, c->stream));
    HIP_TRY(c, hipMemcpyAsync(dr.p, inv_dr.data(), dr.n, hipMemcpyHostToDevice, c->stream));
    HIP_TRY(c, hipMemcpyAsync(ds.p, slot.data(), ds.n, hipMemcpyHostToDevice, c->stream));
    if ((s = sync(c))) return s;
    p->e_tab = std::move(dt);
    p->e_inv_dr = std::move(dr);
    p->e_slot = std::move(ds);
    p->e_cut = cut;
    p->e_inv_dt = (float)((kETab - 1) / (kETabTop - (double)cut));
  }
  p->gen = c->next_gen++;
  if (p->has_activity && (s = zero_tallies(c, *p))) return s;
  return upload_desc(c, id, *p);
}

nmd_status nmd_set_positron(nmd_ctx *c, int32_t id, int32_t on, double noncol_fwhm_deg,
                            const double *mean_excitation_ev) {
  nmd_status s = check_ctx(c);
  if (s) return s;
  Phantom *p = find(c, id);
  if (!p) return fail(c, NMD_E_STATE, "phantom %d is not registered", id);
  if (on != 0 && on != 1) return fail(c, NMD_E_INVALID, "on must be 0 or 1");
  if (on && p->em_on)
    return fail(c, NMD_E_STATE, "phantom %d has an emitter in place of the positron's pair", id);
  if (!on) {
    p->p_cdf.release();
    p->p_guide.release();
    p->p_tab.release();
    p->p_inv_dr.release();
    p->p_slot.release();
    p->p_on = 0;
    p->p_inv_dt = 0.0f;
    p->noncol_sigma = 0.0f;
  } else {
    if (!(noncol_fwhm_deg >= 0.0 && noncol_fwhm_deg <= 5.0))
      return fail(c, NMD_E_INVALID, "non-collinearity FWHM must lie in [0, 5] degrees");
    if (!mean_excitation_ev)
      return fail(c, NMD_E_INVALID, "mean excitation energies are required");
    for (int m = 0; m < p->n_mat; ++m)
      if (!(mean_excitation_ev[m] > 1.0 && mean_excitation_ev[m] < 1.0e4))
        return fail(c, NMD_E_INVALID, "mean excitation energy of material %d must lie in "
                    "(1, 10^4) eV", m);
    std::vector<float> tab((size_t)kMaxMaterials * 2 * kETab, 0.0f), inv_dr(kMaxMaterials, 0.0f);
    for (int m = 0; m < p->n_mat; ++m)
      electron_tables((double)kPosFloor, kPosTop, p->mat_zoa[m], mean_excitation_ev[m],
                      &tab[(size_t)m * 2 * kETab], &tab[(size_t)m * 2 * kETab + kETab], &inv_dr[m]);
    std::vector<double> cdf(kPosN + 1);
    std::vector<int32_t> guide(kPosN);
    positron_cdf(cdf.data(), guide.data());
    std::vector<uint8_t> slot(kMaxPalette, 0);
    for (int q = 0; q < kMaxPalette; ++q) slot[q] = (uint8_t)std::max(p->pal_mat[q], 0);
    DevBuf dc, dg, dt, dr, ds;
    if ((s = dev_alloc(c, dc, cdf.size() * sizeof(double))) ||
        (s = dev_alloc(c, dg, guide.size() * sizeof(int32_t))) ||
        (s = dev_alloc(c, dt, tab.size() * sizeof(float))) ||
        (s = dev_alloc(c, dr, inv_dr.size() * sizeof(float))) ||
        (s = dev_alloc(c, ds, slot.size())))
      return s;
    HIP_TRY(c, hipMemcpyAsync(dc.p, cdf.data(), dc.n, hipMemcpyHostToDevice, c->stream));
    HIP_TRY(c, hipMemcpyAsync(dg.p, guide.data(), dg.n, hipMemcpyHostToDevice, c->stream));
    HIP_TRY(c, hipMemcpyAsync(dt.p, tab.data(), dt.n, hipMemcpyHostToDevice, c->stream));
    HIP_TRY(c, hipMemcpyAsync(dr.p, inv_dr.data(), dr.n, hipMemcpyHostToDevice, c->stream));
    HIP_TRY(c, hipMemcpyAsync(ds.p, slot.data(), ds.n, hipMemcpyHostToDevice, c->stream));
    if ((s = sync(c))) return s;
    p->p_cdf = std::move(dc);
    p->p_guide = std::move(dg);
    p->p_tab = std::move(dt);
    p->p_inv_dr = std::move(dr);
    p->p_slot = std::move(ds);
    p->p_on = 1;
    p->p_inv_dt = (float)((kETab - 1) / (kPosTop - (double)kPosFloor));
    // Rayleigh scale sigma = FWHM / (2 sqrt(2 ln 2)) of the tilt's size
    p->noncol_sigma = (float)(noncol_fwhm_deg * M_PI / 180.0 / (2.0 * std::sqrt(2.0 * M_LN2)));
  }
  p->gen = c->next_gen++;
  if (p->has_activity && (s = zero_tallies(c, *p))) return s;
  return upload_desc(c, id, *p);
}

nmd_status nmd_set_emitter(nmd_ctx *c, int32_t id, int32_t n_lines, const double *energy_mev,
                           const double *yield, double beta_mean_mev) {
  nmd_status s = check_ctx(c);
  if (s) return s;
  Phantom *p = find(c, id);
  if (!p) return fail(c, NMD_E_STATE, "phantom %d is not registered", id);
  if (n_lines < 0 || n_lines > kMaxLines)
    return fail(c, NMD_E_INVALID, "an emitter has 0 to %d lines", kMaxLines);
  if (!(beta_mean_mev >= 0.0 && beta_mean_mev < 10.0))
    return fail(c, NMD_E_INVALID, "mean beta energy must lie in [0, 10) MeV");
  if (n_lines && (!energy_mev || !yield))
    return fail(c, NMD_E_INVALID, "line energies and yields are required");
  double cum = 0.0;
  for (int i = 0; i < n_lines; ++i) {
    if (!(energy_mev[i] > 0.001 && energy_mev[i] <= kLineMax))
      return fail(c, NMD_E_INVALID, "line %d: energy must lie in (0.001, %g] MeV", i, kLineMax);
    // the electron range tables end above the Compton electrons of 511 keV
    if (energy_mev[i] > 0.511 && p->e_cut > 0.0f)
      return fail(c, NMD_E_UNSUPPORTED, "line %d above 0.511 MeV with Compton electrons on", i);
    if (!(yield[i] >= 0.0)) return fail(c, NMD_E_INVALID, "line %d: negative yield", i);
    cum += yield[i];
  }
  if (cum > 1.0 + 1e-12) return fail(c, NMD_E_INVALID, "the yields sum to more than 1");
  const bool on = n_lines > 0 || beta_mean_mev > 0.0;
  if (on && p->p_on)
    return fail(c, NMD_E_STATE, "phantom %d emits positrons: turn them off first", id);
  p->em_on = on;
  p->em_n = on ? n_lines : 0;
  cum = 0.0;
  for (int i = 0; i < kMaxLines; ++i) {
    if (i < p->em_n) cum += yield[i];  // summed in line order, as the decay's test reads it
    p->em_cum[i] = i < p->em_n ? cum : 0.0;
    p->em_e[i] = i < p->em_n ? (float)energy_mev[i] : 0.0f;
  }
  p->em_beta = on ? (float)beta_mean_mev : 0.0f;
  p->wide = false;
  for (int i = 0; i < p->em_n; ++i) p->wide = p->wide || energy_mev[i] > 0.511;
  p->gen = c->next_gen++;
  if (p->has_activity && (s = zero_tallies(c, *p))) return s;
  return upload_desc(c, id, *p);
}

nmd_status nmd_set_tracking(nmd_ctx *c, int32_t id, int32_t mode) {
  nmd_status s = check_ctx(c);
  if (s) return s;
  Phantom *p = find(c, id);
  if (!p) return fail(c, NMD_E_STATE, "phantom %d is not registered", id);
  if (mode != NMD_TRACK_GLOBAL && mode != NMD_TRACK_REGIONS)
    return fail(c, NMD_E_INVALID, "tracking mode must be NMD_TRACK_GLOBAL or NMD_TRACK_REGIONS");
  p->tracking = mode;
  // the same model either way, so the tallies stay; graphs captured with
  // the other kernel no longer match
  p->gen = c->next_gen++;
  return upload_desc(c, id, *p);
}

nmd_status nmd_reset_tallies(nmd_ctx *c, int32_t id) {
  nmd_status s = check_ctx(c);
  if (s) return s;
  if (id == -1) {
    for (auto &kv : c->ph)
      if ((s = zero_tallies(c, kv.second))) return s;
    return NMD_OK;
  }
  Phantom *p = find(c, id);
  if (!p) return fail(c, NMD_E_STATE, "phantom %d is not registered", id);
  return zero_tallies(c, *p);
}

nmd_status nmd_run_histories(nmd_ctx *c, int32_t id, uint64_t n, uint64_t seed,
                             const nmd_run_opts *opts_in) {
  nmd_status s = check_ctx(c);
  if (s) return s;
  RunPlan plan;
  if ((s = plan_run(c, id, n, seed, opts_in, plan))) return s;
  if (n == 0) return NMD_OK;
  if (plan.abort_after) {
    s = run_abortable(c, plan);
    c->last_chunk = plan.rp.chunk;
    c->last_grid = (uint32_t)plan.grid;
    return s;
  }
  const bool tune = plan.auto_chunk && !plan.tuned && n >= kTuneMinPerPhantom;
  if (!tune) {
    if ((s = enqueue_run(c, plan, c->d_queue.as<unsigned long long>(), c->d_dep_v.as<uint32_t>(),
                         c->d_dep_e.as<double>(), c->d_dep_r.as<uint32_t>(), c->stream)))
      return s;
  } else {
    // Tune the work-queue chunk on this run itself: a slice of it with each
    // candidate, timed, then the rest with the fastest.  Histories continue
    // across the slices, so the result is that of one launch.
    const uint64_t slice = n / 16;
    float best_ms = 0.0f;
    uint32_t best = kTuneChunks[0];
    hipEvent_t e0, e1;
    HIP_TRY(c, hipEventCreate(&e0));
    HIP_TRY(c, hipEventCreate(&e1));
    uint64_t done = 0;
    for (uint32_t ch : kTuneChunks) {
      set_chunk(plan, slice, ch);
      HIP_TRY(c, hipEventRecord(e0, c->stream));
      if ((s = enqueue_run(c, plan, c->d_queue.as<unsigned long long>(), c->d_dep_v.as<uint32_t>(),
                           c->d_dep_e.as<double>(), c->d_dep_r.as<uint32_t>(), c->stream)))
        return s;
      HIP_TRY(c, hipEventRecord(e1, c->stream));
      HIP_TRY(c, hipEventSynchronize(e1));
      float ms = 0.0f;
      HIP_TRY(c, hipEventElapsedTime(&ms, e0, e1));
      if (best_ms == 0.0f || ms < best_ms) {
        best_ms = ms;
        best = ch;
      }
      done += slice;
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    c->tuned[plan.key] = best;
    save_tune_cache(c);
    set_chunk(plan, n - done, best);
    if ((s = enqueue_run(c, plan, c->d_queue.as<unsigned long long>(), c->d_dep_v.as<uint32_t>(),
                         c->d_dep_e.as<double>(), c->d_dep_r.as<uint32_t>(), c->stream)))
      return s;
  }
  c->last_chunk = plan.rp.chunk;
  c->last_grid = (uint32_t)plan.grid;
  return NMD_OK;
}

nmd_status nmd_get_dose(nmd_ctx *c, int32_t id, double *rate, double *rel) {
  nmd_status s = check_ctx(c);
  if (s) return s;
  Phantom *p = find(c, id);
  if (!p) return fail(c, NMD_E_STATE, "phantom %d is not registered", id);
  if (!p->has_activity || p->n_done == 0)
    return fail(c, NMD_E_STATE, "phantom %d has no histories yet", id);
  if (!rate) return fail(c, NMD_E_INVALID, "dose_rate buffer is required");
  HIP_TRY(c, launch_finalize(p->rec.as<uint16_t>(), c->d_pal.as<float4>(), p->tally.as<double2>(),
                             p->nvox, p->n_done_dev.as<unsigned long long>(), p->vkg(), p->a_ts,
                             rate, rel, c->stream));
  return NMD_OK;
}

nmd_status nmd_read_organ_dose(nmd_ctx *c, int32_t id, int32_t n_organs, double *rate,
                               double *eps3, double *sig_mean) {
  nmd_status s = check_ctx(c);
  if (s) return s;
  Phantom *p = find(c, id);
  if (!p) return fail(c, NMD_E_STATE, "phantom %d is not registered", id);
  if (!p->has_label) return fail(c, NMD_E_STATE, "phantom %d has no organ labels", id);
  if (!p->has_activity || p->n_done == 0)
    return fail(c, NMD_E_STATE, "phantom %d has no histories yet", id);
  if (n_organs < 0 || n_organs > p->n_org)
    return fail(c, NMD_E_INVALID, "n_organs %d exceeds the phantom's %d", n_organs, p->n_org);
  if (sig_mean && p->organ_from != 0)
    return fail(c, NMD_E_STATE,
                "phantom %d: the per-history organ sums cover %llu of %llu histories (sums "
                "restored by nmd_set_tallies); restore with nmd_load for the organ sigma",
                id, (unsigned long long)(p->n_done - p->organ_from),
                (unsigned long long)p->n_done);
  const double n = (double)p->n_done;
  std::vector<double> acc((p->n_org + 1) * 2);
  std::vector<double2> org(p->n_org + 1);
  HIP_TRY(c, hipMemcpyAsync(acc.data(), p->organ_acc.p, acc.size() * sizeof(double),
                            hipMemcpyDeviceToHost, c->stream));
  HIP_TRY(c, hipMemcpyAsync(org.data(), p->organ.p, org.size() * sizeof(double2),
                            hipMemcpyDeviceToHost, c->stream));
  if ((s = sync(c))) return s;
  for (int o = 1; o <= n_organs; ++o) {
    const double cnt = (double)p->organ_count[o];
    if (rate) rate[o - 1] = cnt > 0 ? acc[2 * o] / cnt : 0.0;
    if (eps3) eps3[o - 1] = cnt > 0 ? std::sqrt(acc[2 * o + 1] / cnt) : 0.0;
    if (sig_mean) {
      const double m = org[o].x / n;
      double var = n > 1 ? (org[o].y / n - m * m) / (n - 1.0) : 0.0;
      if (var < 0) var = 0;
      sig_mean[o - 1] = m > 0 ? std::sqrt(var) / m : 0.0;
    }
  }
  return NMD_OK;
}

nmd_status nmd_get_organ_dose(nmd_ctx *c, int32_t id, int32_t n_organs, double *rate,
                              double *eps3, double *sig_mean) {
  nmd_status s = check_ctx(c);
  if (s) return s;
  Phantom *p = find(c, id);
  if (!p) return fail(c, NMD_E_STATE, "phantom %d is not registered", id);
  if (!p->has_label) return fail(c, NMD_E_STATE, "phantom %d has no organ labels", id);
  if (!p->has_activity || p->n_done == 0)
    return fail(c, NMD_E_STATE, "phantom %d has no histories yet", id);
  if ((s = enqueue_organ_reduce(c, *p, c->stream))) return s;
  return nmd_read_organ_dose(c, id, n_organs, rate, eps3, sig_mean);
}

nmd_status nmd_organ_mean_map(nmd_ctx *c, int32_t id, const double *map, int32_t n_organs,
                              double *out) {
  nmd_status s = check_ctx(c);
  if (s) return s;
  Phantom *p = find(c, id);
  if (!p) return fail(c, NMD_E_STATE, "phantom %d is not registered", id);
  if (!p->has_label) return fail(c, NMD_E_STATE, "phantom %d has no organ labels", id);
  if (!map || !out || n_organs < 0 || n_organs > p->n_org)
    return fail(c, NMD_E_INVALID, "bad map, output or n_organs");
  DevBuf acc;
  if ((s = dev_alloc(c, acc, (p->n_org + 1) * sizeof(double)))) return s;
  HIP_TRY(c, launch_zero_bytes(acc.p, acc.n, c->stream));
  HIP_TRY(c, launch_map_organ_reduce(p->rec.as<uint16_t>(), p->nvox, p->n_org, map,
                                     acc.as<double>(), c->stream));
  std::vector<double> h(p->n_org + 1);
  HIP_TRY(c, hipMemcpyAsync(h.data(), acc.p, acc.n, hipMemcpyDeviceToHost, c->stream));
  if ((s = sync(c))) return s;
  for (int o = 1; o <= n_organs; ++o) {
    const double cnt = (double)p->organ_count[o];
    out[o - 1] = cnt > 0 ? h[o] / cnt : 0.0;
  }
  return NMD_OK;
}

nmd_status nmd_organ_mean_map_noalloc(nmd_ctx *c, int32_t id, const double *map,
                                      int32_t n_organs, double *out) {
  nmd_status s = check_ctx(c);
  if (s) return s;
  Phantom *p = find(c, id);
  if (!p) return fail(c, NMD_E_STATE, "phantom %d is not registered", id);
  if (!p->has_label) return fail(c, NMD_E_STATE, "phantom %d has no organ labels", id);
  if (!map || !out || n_organs < 0 || n_organs > p->n_org)
    return fail(c, NMD_E_INVALID, "bad map, output or n_organs");
  const int slots = p->n_org + 1;
  if (slots > kNoallocSlots)
    return fail(c, NMD_E_UNSUPPORTED, "%d organ labels exceed the %d-slot device scratch",
                slots, kNoallocSlots);
  if (!c->noalloc_scratch) return fail(c, NMD_E_STATE, "no device scratch on this device");
  double *acc = c->noalloc_scratch;
  // the previous call's sums are still there: clear this call's slots (a
  // fill kernel, so the call has no memset node if a caller captures it)
  HIP_TRY(c, launch_zero_bytes(acc, (uint64_t)slots * sizeof(double), c->stream));
  HIP_TRY(c, launch_map_organ_reduce(p->rec.as<uint16_t>(), p->nvox, p->n_org, map, acc,
                                     c->stream));
  double h[kNoallocSlots];
  HIP_TRY(c, hipMemcpyAsync(h, acc, (size_t)slots * sizeof(double), hipMemcpyDeviceToHost,
                            c->stream));
  if ((s = sync(c))) return s;
  for (int o = 1; o <= n_organs; ++o) {
    const double cnt = (double)p->organ_count[o];
    out[o - 1] = cnt > 0 ? h[o] / cnt : 0.0;
  }
  return NMD_OK;
}

nmd_status nmd_get_organ_score(nmd_ctx *c, int32_t id, int32_t n_organs, double *rate) {
  nmd_status s = check_ctx(c);
  if (s) return s;
  Phantom *p = find(c, id);
  if (!p) return fail(c, NMD_E_STATE, "phantom %d is not registered", id);
  if (!p->has_label) return fail(c, NMD_E_STATE, "phantom %d has no organ labels", id);
  if (n_organs < 0 || n_organs > p->n_org || !rate)
    return fail(c, NMD_E_INVALID, "bad n_organs or output");
  if (p->n_done == 0) return fail(c, NMD_E_STATE, "phantom %d has no histories yet", id);
  if (p->organ_from != 0)
    return fail(c, NMD_E_STATE,
                "phantom %d: the per-history organ sums do not cover the histories restored "
                "by nmd_set_tallies", id);
  std::vector<double2> org(p->n_org + 1);
  HIP_TRY(c, hipMemcpyAsync(org.data(), p->organ.p, org.size() * sizeof(double2),
                            hipMemcpyDeviceToHost, c->stream));
  if ((s = sync(c))) return s;
  for (int o = 1; o <= n_organs; ++o) rate[o - 1] = p->a_ts * org[o].x / (double)p->n_done;
  return NMD_OK;
}

nmd_status nmd_get_ledger(nmd_ctx *c, int32_t id, double *ledger) {
  nmd_status s = check_ctx(c);
  if (s) return s;
  Phantom *p = find(c, id);
  if (!p) return fail(c, NMD_E_STATE, "phantom %d is not registered", id);
  if (!ledger) return fail(c, NMD_E_INVALID, "ledger output is required");
  double l[8];
  unsigned long long st[16];
  HIP_TRY(c, hipMemcpyAsync(l, p->ledger.p, sizeof l, hipMemcpyDeviceToHost, c->stream));
  HIP_TRY(c, hipMemcpyAsync(st, p->stats.p, sizeof st, hipMemcpyDeviceToHost, c->stream));
  if ((s = sync(c))) return s;
  // the photons' energy, and the positrons' kinetic energy counted on the
  // device; an emitter's photons and beta energy are all counted there
  ledger[0] = (p->em_on ? 0.0 : (double)st[NMD_STAT_PHOTONS] * (double)kE0) + l[0];
  for (int i = 1; i < NMD_LEDGER_N; ++i) ledger[i] = l[i];
  return NMD_OK;
}

nmd_status nmd_get_run_stats(nmd_ctx *c, int32_t id, uint64_t *stats) {
  nmd_status s = check_ctx(c);
  if (s) return s;
  Phantom *p = find(c, id);
  if (!p) return fail(c, NMD_E_STATE, "phantom %d is not registered", id);
  if (!stats) return fail(c, NMD_E_INVALID, "stats output is required");
  unsigned long long st[16];
  HIP_TRY(c, hipMemcpyAsync(st, p->stats.p, sizeof st, hipMemcpyDeviceToHost, c->stream));
  if ((s = sync(c))) return s;
  for (int i = 0; i < NMD_STAT_N; ++i) stats[i] = st[i];
  return NMD_OK;
}

nmd_status nmd_get_tallies(nmd_ctx *c, int32_t id, double *sum, double *sum2, uint64_t *n) {
  nmd_status s = check_ctx(c);
  if (s) return s;
  Phantom *p = find(c, id);
  if (!p) return fail(c, NMD_E_STATE, "phantom %d is not registered", id);
  if (n) *n = p->n_done;
  if (sum)
    HIP_TRY(c, hipMemcpy2DAsync(sum, sizeof(double), p->tally.p, sizeof(double2), sizeof(double),
                                p->nvox, hipMemcpyDeviceToDevice, c->stream));
  if (sum2)
    HIP_TRY(c, hipMemcpy2DAsync(sum2, sizeof(double), p->tally.as<char>() + sizeof(double),
                                sizeof(double2), sizeof(double), p->nvox,
                                hipMemcpyDeviceToDevice, c->stream));
  return NMD_OK;
}

nmd_status nmd_set_tallies(nmd_ctx *c, int32_t id, const double *sum, const double *sum2,
                           uint64_t n) {
  nmd_status s = check_ctx(c);
  if (s) return s;
  Phantom *p = find(c, id);
  if (!p) return fail(c, NMD_E_STATE, "phantom %d is not registered", id);
  if (!p->has_activity) return fail(c, NMD_E_STATE, "phantom %d has no activity map", id);
  if (!sum || !sum2) return fail(c, NMD_E_INVALID, "both sums are required");
  if ((s = zero_tallies(c, *p))) return s;
  HIP_TRY(c, hipMemcpy2DAsync(p->tally.p, sizeof(double2), sum, sizeof(double), sizeof(double),
                              p->nvox, hipMemcpyDefault, c->stream));
  HIP_TRY(c, hipMemcpy2DAsync(p->tally.as<char>() + sizeof(double), sizeof(double2), sum2,
                              sizeof(double), sizeof(double), p->nvox, hipMemcpyDefault,
                              c->stream));
  HIP_TRY(c, launch_set_u64(p->n_done_dev.as<unsigned long long>(), n, c->stream));
  p->n_done = n;
  p->organ_from = n;
  return sync(c);
}

// ---- checkpoints ------------------------------------------------------------
// File layout (little-endian): a header, then the (S, S2) pairs of every
// voxel, the (O, O2) pairs of labels 0..n_org, the ledger and the run
// counters, then a 64-bit FNV-1a of everything before it.
namespace {
struct CkptHeader {
  char magic[8];            // "NMDCKPT1"
  uint32_t version, n_org;  // 1
  int32_t nx, ny, nz, pad;
  uint64_t nvox, n_done, organ_from;
  uint64_t geom_hash, act_hash;
  double dx, dy, dz;
};
constexpr size_t kLedgerSlots = 8, kStatSlots = 16;
}  // namespace

nmd_status nmd_save(nmd_ctx *c, int32_t id, const char *path) {
  nmd_status s = check_ctx(c);
  if (s) return s;
  Phantom *p = find(c, id);
  if (!p) return fail(c, NMD_E_STATE, "phantom %d is not registered", id);
  if (!p->has_activity) return fail(c, NMD_E_STATE, "phantom %d has no activity map", id);
  if (!path) return fail(c, NMD_E_INVALID, "path is required");
  CkptHeader h = {};
  std::memcpy(h.magic, "NMDCKPT1", 8);
  h.version = 1;
  h.n_org = (uint32_t)p->n_org;
  h.nx = p->nx;
  h.ny = p->ny;
  h.nz = p->nz;
  h.nvox = p->nvox;
  h.n_done = p->n_done;
  h.organ_from = p->organ_from;
  h.geom_hash = p->geom_hash;
  h.act_hash = p->act_hash;
  h.dx = p->dx;
  h.dy = p->dy;
  h.dz = p->dz;
  std::vector<double> tal, org, led;
  std::vector<unsigned long long> st;
  if ((s = to_host(c, tal, p->tally.as<double>(), p->nvox * 2)) ||
      (s = to_host(c, org, p->organ.as<double>(), (uint64_t)(p->n_org + 1) * 2)) ||
      (s = to_host(c, led, p->ledger.as<double>(), kLedgerSlots)) ||
      (s = to_host(c, st, p->stats.as<unsigned long long>(), kStatSlots)))
    return s;
  uint64_t sum = fnv1a(&h, sizeof h);
  sum = fnv1a(tal.data(), tal.size() * 8, sum);
  sum = fnv1a(org.data(), org.size() * 8, sum);
  sum = fnv1a(led.data(), led.size() * 8, sum);
  sum = fnv1a(st.data(), st.size() * 8, sum);
  const std::string tmp = std::string(path) + ".tmp";
  FILE *f = std::fopen(tmp.c_str(), "wb");
  if (!f) return fail(c, NMD_E_INVALID, "cannot open %s for writing", tmp.c_str());
  bool ok = std::fwrite(&h, sizeof h, 1, f) == 1 &&
            std::fwrite(tal.data(), 8, tal.size(), f) == tal.size() &&
            std::fwrite(org.data(), 8, org.size(), f) == org.size() &&
            std::fwrite(led.data(), 8, led.size(), f) == led.size() &&
            std::fwrite(st.data(), 8, st.size(), f) == st.size() &&
            std::fwrite(&sum, 8, 1, f) == 1;
  ok = (std::fclose(f) == 0) && ok;
  if (!ok || std::rename(tmp.c_str(), path) != 0) {
    std::remove(tmp.c_str());
    return fail(c, NMD_E_INVALID, "writing %s failed", path);
  }
  return NMD_OK;
}

nmd_status nmd_load(nmd_ctx *c, int32_t id, const char *path) {
  nmd_status s = check_ctx(c);
  if (s) return s;
  Phantom *p = find(c, id);
  if (!p) return fail(c, NMD_E_STATE, "phantom %d is not registered", id);
  if (!p->has_activity) return fail(c, NMD_E_STATE, "phantom %d has no activity map", id);
  if (!path) return fail(c, NMD_E_INVALID, "path is required");
  FILE *f = std::fopen(path, "rb");
  if (!f) return fail(c, NMD_E_INVALID, "cannot open %s", path);
  CkptHeader h;
  std::vector<double> tal, org, led(kLedgerSlots);
  std::vector<unsigned long long> st(kStatSlots);
  uint64_t sum = 0;
  bool ok = std::fread(&h, sizeof h, 1, f) == 1 && std::memcmp(h.magic, "NMDCKPT1", 8) == 0 &&
            h.version == 1 && h.nvox == p->nvox && h.n_org == (uint32_t)p->n_org;
  if (ok) {
    tal.resize(h.nvox * 2);
    org.resize((size_t)(h.n_org + 1) * 2);
    ok = std::fread(tal.data(), 8, tal.size(), f) == tal.size() &&
         std::fread(org.data(), 8, org.size(), f) == org.size() &&
         std::fread(led.data(), 8, led.size(), f) == led.size() &&
         std::fread(st.data(), 8, st.size(), f) == st.size() && std::fread(&sum, 8, 1, f) == 1;
  }
  std::fclose(f);
  if (!ok) return fail(c, NMD_E_INVALID, "%s is not a checkpoint of this phantom's shape", path);
  uint64_t chk = fnv1a(&h, sizeof h);
  chk = fnv1a(tal.data(), tal.size() * 8, chk);
  chk = fnv1a(org.data(), org.size() * 8, chk);
  chk = fnv1a(led.data(), led.size() * 8, chk);
  chk = fnv1a(st.data(), st.size() * 8, chk);
  if (chk != sum) return fail(c, NMD_E_INVALID, "%s: checksum mismatch", path);
  if (h.nx != p->nx || h.ny != p->ny || h.nz != p->nz || h.dx != p->dx || h.dy != p->dy ||
      h.dz != p->dz || h.geom_hash != p->geom_hash)
    return fail(c, NMD_E_STATE, "%s was saved from a different phantom geometry", path);
  if (h.act_hash != p->act_hash)
    return fail(c, NMD_E_STATE, "%s was saved with a different activity map", path);
  if (h.organ_from > h.n_done) return fail(c, NMD_E_INVALID, "%s: inconsistent counters", path);
  HIP_TRY(c, hipMemcpyAsync(p->tally.p, tal.data(), tal.size() * 8, hipMemcpyHostToDevice,
                            c->stream));
  HIP_TRY(c, hipMemcpyAsync(p->organ.p, org.data(), org.size() * 8, hipMemcpyHostToDevice,
                            c->stream));
  HIP_TRY(c, hipMemcpyAsync(p->ledger.p, led.data(), led.size() * 8, hipMemcpyHostToDevice,
                            c->stream));
  HIP_TRY(c, hipMemcpyAsync(p->stats.p, st.data(), st.size() * 8, hipMemcpyHostToDevice,
                            c->stream));
  HIP_TRY(c, launch_set_u64(p->n_done_dev.as<unsigned long long>(), h.n_done, c->stream));
  if ((s = sync(c))) return s;
  p->n_done = h.n_done;
  p->organ_from = h.organ_from;
  return NMD_OK;
}

nmd_status nmd_get_last_launch(nmd_ctx *c, uint32_t *chunk, uint32_t *grid_blocks) {
  nmd_status s = check_ctx(c);
  if (s) return s;
  if (chunk) *chunk = c->last_chunk;
  if (grid_blocks) *grid_blocks = c->last_grid;
  return NMD_OK;
}

nmd_status nmd_graph_create(nmd_ctx *c, int32_t id, uint64_t n, uint64_t seed,
                            const nmd_run_opts *opts, double *dose_rate, double *rel_unc,
                            nmd_graph **out) {
  nmd_status s = check_ctx(c);
  if (s) return s;
  if (!out) return fail(c, NMD_E_INVALID, "out is required");
  *out = nullptr;
  if (n == 0) return fail(c, NMD_E_INVALID, "n_decays must be > 0");
  if (opts && (opts->history_records || opts->abort_after_chunks))
    return fail(c, NMD_E_INVALID, "history records and the abort hook are not captured");
  if (dose_rate && id == -1) return fail(c, NMD_E_INVALID, "dose maps need a single phantom");
  RunPlan plan;
  if ((s = plan_run(c, id, n, seed, opts, plan))) return s;
  nmd_graph *g = new nmd_graph();
  g->c = c;
  g->ids = plan.ids;
  g->n = n;
  const size_t lanes = (size_t)plan.rp.n_lanes;
  if ((s = dev_alloc(c, g->queue, 2 * sizeof(unsigned long long))) ||
      (s = dev_alloc(c, g->dep_v, lanes * kDepCap * sizeof(uint32_t))) ||
      (s = dev_alloc(c, g->dep_e, lanes * kDepCap * sizeof(double))) ||
      (s = dev_alloc(c, g->dep_r, lanes * kDepCap * sizeof(uint32_t)))) {
    delete g;
    return s;
  }
  if (!c->capture && hipStreamCreateWithFlags(&c->capture, hipStreamNonBlocking) != hipSuccess) {
    delete g;
    return fail(c, NMD_E_HIP, "cannot create the capture stream");
  }
  // the host counters must not move during capture: restore them after
  std::vector<uint64_t> done(plan.ids.n);
  for (int i = 0; i < plan.ids.n; ++i) done[i] = c->ph[plan.ids.id[i]].n_done;
  hipError_t e = hipStreamBeginCapture(c->capture, hipStreamCaptureModeThreadLocal);
  if (e == hipSuccess) {
    s = enqueue_run(c, plan, g->queue.as<unsigned long long>(), g->dep_v.as<uint32_t>(),
                    g->dep_e.as<double>(), g->dep_r.as<uint32_t>(), c->capture);
    if (!s && dose_rate) {
      Phantom &p = c->ph[id];
      e = launch_finalize(p.rec.as<uint16_t>(), c->d_pal.as<float4>(), p.tally.as<double2>(),
                          p.nvox, p.n_done_dev.as<unsigned long long>(), p.vkg(), p.a_ts,
                          dose_rate, rel_unc, c->capture);
    }
    for (int i = 0; !s && e == hipSuccess && i < plan.ids.n; ++i) {
      Phantom &p = c->ph[plan.ids.id[i]];
      if (p.has_label) s = enqueue_organ_reduce(c, p, c->capture);
    }
    hipGraph_t graph = nullptr;
    const hipError_t e2 = hipStreamEndCapture(c->capture, &graph);
    if (e == hipSuccess) e = e2;
    g->g = graph;
  }
  for (int i = 0; i < plan.ids.n; ++i) c->ph[plan.ids.id[i]].n_done = done[i];
  if (!s && e == hipSuccess) e = hipGraphInstantiate(&g->ge, g->g, nullptr, nullptr, 0);
  if (s || e != hipSuccess) {
    if (g->ge) (void)hipGraphExecDestroy(g->ge);
    if (g->g) (void)hipGraphDestroy(g->g);
    delete g;
    if (s) return s;
    return fail(c, NMD_E_HIP, "graph capture failed: %s", hipGetErrorString(e));
  }
  for (int i = 0; i < plan.ids.n; ++i) g->gen.push_back(c->ph[plan.ids.id[i]].gen);
  *out = g;
  return NMD_OK;
}

nmd_status nmd_graph_launch(nmd_graph *g) {
  if (!g) return NMD_E_INVALID;
  nmd_ctx *c = g->c;
  nmd_status s = check_ctx(c);
  if (s) return s;
  for (int i = 0; i < g->ids.n; ++i) {
    Phantom *p = find(c, g->ids.id[i]);
    if (!p || p->gen != g->gen[i])
      return fail(c, NMD_E_STATE, "phantom %d changed since the graph was captured",
                  g->ids.id[i]);
  }
  HIP_TRY(c, hipGraphLaunch(g->ge, c->stream));
  for (int i = 0; i < g->ids.n; ++i) c->ph[g->ids.id[i]].n_done += g->n;
  return NMD_OK;
}

void nmd_graph_destroy(nmd_graph *g) {
  if (!g) return;
  (void)hipSetDevice(g->c->device);
  if (g->c->stream) (void)hipStreamSynchronize(g->c->stream);
  if (g->ge) (void)hipGraphExecDestroy(g->ge);
  if (g->g) (void)hipGraphDestroy(g->g);
  delete g;
}

nmd_status nmd_debug_sample(nmd_ctx *c, int32_t kind, double e_mev, uint64_t n, uint64_t seed,
                            double *out) {
  nmd_status s = check_ctx(c);
  if (s) return s;
  if (!(kind == 0 || kind == 1 || kind == 2 || kind == 3 || kind == 5))
    return fail(c, NMD_E_INVALID, "unknown sample kind %d", kind);
  if (kind == 3 && !(e_mev >= 0.001 && e_mev <= 0.511))
    return fail(c, NMD_E_INVALID, "energy must lie in [0.001, 0.511] MeV");
  if (!out && n) return fail(c, NMD_E_INVALID, "output is required");
  HIP_TRY(c, launch_debug_sample(kind, (float)e_mev, n, (uint32_t)seed, (uint32_t)(seed >> 32),
                                 out, c->stream));
  return NMD_OK;
}

nmd_status nmd_debug_sample_source(nmd_ctx *c, int32_t id, uint64_t n, uint64_t seed,
                                   uint32_t *out) {
  nmd_status s = check_ctx(c);
  if (s) return s;
  Phantom *p = find(c, id);
  if (!p || !p->has_activity) return fail(c, NMD_E_STATE, "phantom %d has no activity map", id);
  if (!out && n) return fail(c, NMD_E_INVALID, "output is required");
  HIP_TRY(c, launch_debug_source(p->alias.as<uint4>(), p->n_alias, (uint32_t)id, n, (uint32_t)seed,
                                 (uint32_t)(seed >> 32), (uint32_t)p->nx, (uint32_t)p->ny, out,
                                 c->stream));
  return NMD_OK;
}

nmd_status nmd_debug_xs(nmd_ctx *c, int32_t id, uint64_t n, const float *energies, float *out) {
  nmd_status s = check_ctx(c);
  if (s) return s;
  Phantom *p = find(c, id);
  if (!p) return fail(c, NMD_E_STATE, "phantom %d is not registered", id);
  if ((!energies || !out) && n) return fail(c, NMD_E_INVALID, "buffers are required");
  DevBuf used;
  if ((s = dev_alloc(c, used, kMaxPalette))) return s;
  HIP_TRY(c, hipMemcpyAsync(used.p, p->used.data(), kMaxPalette, hipMemcpyHostToDevice, c->stream));
  HIP_TRY(c, launch_debug_xs(c->d_pal.as<float4>(), used.as<uint8_t>(), (int)c->pal.size(),
                             c->d_kn.as<float>(), p->major.as<float>(), n, energies, out,
                             c->l2emin, c->inv_dl2, c->stream));
  return sync(c);  // `used` is freed on return
}

}  // extern "C"

// ---- services of the context for the denoiser entry points ------------------
namespace nmd {

nmd_status ctx_enter(nmd_ctx *c) { return check_ctx(c); }

nmd_status ctx_fail(nmd_ctx *c, nmd_status s, const char *fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  return fail(c, s, "%s", buf);
}

nmd_status ctx_hip(nmd_ctx *c, hipError_t e, const char *what) {
  if (e == hipSuccess) return NMD_OK;
  return fail(c, e == hipErrorOutOfMemory ? NMD_E_OOM : NMD_E_HIP, "%s: %s", what,
              hipGetErrorString(e));
}

hipStream_t ctx_stream(const nmd_ctx *c) { return c->stream; }

nmd_status ctx_scratch(nmd_ctx *c, size_t bytes, void **p) {
  if (c->nn_scratch.n < bytes) {
    // the old buffer may still be read by queued work: drain first
    nmd_status s = sync(c);
    if (s) return s;
    if ((s = dev_alloc(c, c->nn_scratch, bytes))) return s;
  }
  *p = c->nn_scratch.p;
  return NMD_OK;
}

}  // namespace nmd
