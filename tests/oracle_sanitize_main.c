/* Driver for the memory and undefined-behaviour check of the oracle: the
 * oracle's source is compiled into this file's translation unit with
 * AddressSanitizer and UndefinedBehaviorSanitizer (tests/test_oracle_sanitizers.py),
 * and every transport mode, source, option and sampler runs on a small
 * heterogeneous phantom.  Any sanitizer report aborts; the driver itself
 * checks return codes and that each ledger closes. */
#include "../oracle/nmd_oracle.c"

#include <stdio.h>

#define NX 12
#define NY 10
#define NZ 8
#define NV (NX * NY * NZ)

static int check(const char *what, int rc, const orc_tally *t)
{
  if (rc != 0) {
    fprintf(stderr, "%s: rc %d\n", what, rc);
    return 1;
  }
  double dep = 0.0;
  for (int i = 1; i < ORC_LEDGER_N; ++i)
    if (i != L_ESC && i != L_DISC) dep += t->ledger[i];
  const double bal = (dep + t->ledger[L_ESC] + t->ledger[L_DISC]) / t->ledger[L_EMIT] - 1.0;
  if (!(fabs(bal) < 1e-9)) {
    fprintf(stderr, "%s: ledger balance %g\n", what, bal);
    return 1;
  }
  return 0;
}

int main(void)
{
  static double rho[NV], act[NV], S[NV], S2[NV], hist[64 * ORC_HREC_N];
  static uint8_t mat[NV], lab[NV];
  double O[4] = { 0 }, O2[4] = { 0 };
  for (int z = 0; z < NZ; ++z)
    for (int y = 0; y < NY; ++y)
      for (int x = 0; x < NX; ++x) {
        const int v = x + NX * (y + NY * z);
        const int body = x > 1 && x < NX - 2 && y > 1 && y < NY - 2;
        mat[v] = body ? (x < 5 ? 1 : (x > 8 ? 2 : 0)) : 3;
        rho[v] = body ? (x < 5 ? 0.26 : (x > 8 ? 1.85 : 1.0)) : 0.0012;
        lab[v] = body ? (uint8_t)(1 + (x > 6) + (z > 3)) : 0;
        act[v] = body ? 1.0 + (double)((x * 7 + y * 3 + z) % 5) : 0.0;
      }
  const double zeff[4] = { 7.4, 7.5, 12.3, 7.6 }, zoa[4] = { 0.5551, 0.550, 0.515, 0.499 };
  const double iev[4] = { 75.0, 75.3, 91.9, 85.7 };
  orc_phantom ph = { NX, NY, NZ, 0.5, 0.5, 0.6, rho, mat, lab, 3, zeff, zoa, 4, act };
  const double lines[2] = { 0.113, 0.208 }, yields[2] = { 0.06, 0.10 };
  int fails = 0;
  for (int mode = 0; mode < 9; ++mode) {
    orc_opts op;
    memset(&op, 0, sizeof op);
    op.n_hist = 3000;
    op.seed = 11 + mode;
    op.photons_per_decay = 2;
    op.process_mask = 7;
    op.cutoff_mev = 0.010;
    op.tracking = mode % 3;
    op.kn_method = mode % 2;
    op.wide_uniforms = op.tracking == ORC_TRACK_EXACT;
    op.rng = op.tracking == ORC_TRACK_EXACT ? ORC_RNG_XOSHIRO : ORC_RNG_PHILOX;
    op.n_threads = 2;
    op.mean_excitation_ev = iev;
    if (mode == 3) op.electron_cutoff_mev = 0.2;
    if (mode == 4) {
      op.positron = 1;
      op.noncol_fwhm_rad = 0.0087;
    }
    if (mode == 5) {
      op.n_lines = 2;
      op.line_mev = lines;
      op.line_yield = yields;
      op.beta_mean_mev = 0.134;
    }
    if (mode == 6) {
      op.cutoff_mev = 0.15;
      op.max_real_events = 1;
      op.process_mask = 1;
      op.hist_out = hist;
      op.n_hist = 64;
    }
    if (mode == 7) {
      op.source_kind = ORC_SRC_PENCIL;
      op.pencil_origin[0] = 0.01;
      op.pencil_origin[1] = 2.5;
      op.pencil_origin[2] = 2.4;
      op.pencil_dir[0] = 1.0;
      op.electron_cutoff_mev = 0.2;
    }
    if (mode == 8) {
      op.positron = 1;
      op.electron_cutoff_mev = 0.2;
      op.photons_per_decay = 1;
    }
    memset(S, 0, sizeof S);
    memset(S2, 0, sizeof S2);
    orc_tally t;
    memset(&t, 0, sizeof t);
    t.S = S;
    t.S2 = S2;
    t.O = O;
    t.O2 = O2;
    char name[32];
    snprintf(name, sizeof name, "mode %d", mode);
    fails += check(name, orc_run(&ph, &op, &t), &t);
  }
  /* samplers and the test entry points */
  double out[4 * 200];
  for (int kind = 0; kind <= 7; ++kind)
    if (orc_sample(kind, kind == 7 ? 0.0087 : 0.3, 200, 5, kind & 1, kind & 1, out) != 0) {
      fprintf(stderr, "sample kind %d\n", kind);
      ++fails;
    }
  if (orc_sample_source(&ph, 200, 7, ORC_TRACK_WOODCOCK, 0, ORC_RNG_PHILOX, out) != 0) ++fails;
  int64_t wv[64];
  double we[64], esc = 0.0;
  const double r[3] = { 3.1, 2.6, 2.2 }, de[3] = { 0.6, 0.8, 0.0 };
  if (orc_electron_walk(&ph, iev, 0.2, r, de, 0.34, wv, we, 64, &esc) <= 0) ++fails;
  if (fails) return 1;
  printf("oracle sanitizer run: ok\n");
  return 0;
}
