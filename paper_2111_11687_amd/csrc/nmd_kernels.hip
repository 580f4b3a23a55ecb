// Device kernels of the dosimetry engine (gfx950, wave64).
//
//   transport_kernel  persistent Woodcock photon transport with a work queue,
//                     lane regeneration and history-by-history scoring
//   finalize_kernel   dose-rate and relative-uncertainty maps (Eq. 1)
//   organ_kernel      segmented per-organ reduction (Eq. 2, Eq. 3)
//   debug kernels     sampler dumps and cross-section probes for the tests
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "nmd_device.hpp"
#include "nmd_internal.hpp"

namespace nmd {

__device__ __forceinline__ uint32_t lane_id() {
  return __builtin_amdgcn_mbcnt_hi(~0u, __builtin_amdgcn_mbcnt_lo(~0u, 0u));
}
// Number of set bits of `mask` below this lane.
__device__ __forceinline__ uint32_t rank_in(unsigned long long mask) {
  return __builtin_amdgcn_mbcnt_hi((uint32_t)(mask >> 32),
                                   __builtin_amdgcn_mbcnt_lo((uint32_t)mask, 0u));
}
__device__ __forceinline__ unsigned long long uniform_u64(unsigned long long x) {
  const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)x);
  const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(x >> 32));
  return ((unsigned long long)hi << 32) | lo;
}
__device__ __forceinline__ double wave_sum(double x) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) x += __shfl_xor(x, o, 64);
  return x;
}
__device__ __forceinline__ unsigned long long wave_sum_u64(unsigned long long x) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) x += __shfl_xor(x, o, 64);
  return x;
}

// Address-space views.  Descriptor reads go through the constant space:
// they become scalar loads, which are neither repeated after every store
// (the compiler cannot otherwise rule out that a tally atomic hits the
// descriptor table) nor ordered behind the vector-memory counter; the table
// is not written while a launch runs.  Tallies, deposit lists, records and
// the queue go through the global space, so they compile to global_*
// instructions; flat_* ones would also count against the LDS counter and
// make every LDS wait wait for them.
typedef const __attribute__((address_space(4))) PhantomDesc CDesc;
template <class T>
__device__ __forceinline__ __attribute__((address_space(1))) T *G(T *p) {
  return (__attribute__((address_space(1))) T *)p;
}
template <class T>
__device__ __forceinline__ void gadd(T *p, T v) {
  __hip_atomic_fetch_add(G(p), v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ unsigned long long wave_max_u64(unsigned long long x) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    const unsigned long long y = __shfl_xor(x, o, 64);
    x = y > x ? y : x;
  }
  return x;
}

// ---------------------------------------------------------------------------
// Transport
// ---------------------------------------------------------------------------

// Per-wave accumulators in LDS, flushed to the phantom's globals when the
// wave changes phantom or exits.  Ledger slots follow NMD_LEDGER_* (slot 0,
// emitted, holds the positrons' kinetic energy; the host adds the photons'
// from their count); counters follow NMD_STAT_*.
struct WaveAcc {
  double ledger[NMD_LEDGER_N];
  unsigned long long stat[kStatN];
  float ep0[5];  // energy_params at the emission energy, for the wave's phantom
};

// Per-wave part of the dynamic LDS: organ score accumulators, majorant table
// of the wave's current phantom and its organ weights.  Each wave's region
// is a whole number of 16-byte units, so the double2 accumulators stay
// 16-byte aligned.
struct WaveLds {
  double2 *org;  // [n_slots]
  float *maj;    // [kNGrid]
  double *w;     // [n_slots]
};

__host__ __device__ inline size_t wave_lds_units(int n_slots) {  // 16-byte units
  return (size_t)n_slots + (size_t)kNGrid / 4 + ((size_t)n_slots + 1) / 2;
}

__device__ __forceinline__ WaveLds wave_lds(double2 *dyn, uint32_t wave, int n_slots) {
  double2 *base = dyn + wave_lds_units(n_slots) * wave;
  WaveLds w;
  w.org = base;
  w.maj = reinterpret_cast<float *>(base + n_slots);
  w.w = reinterpret_cast<double *>(base + n_slots + kNGrid / 4);
  return w;
}

size_t transport_dyn_lds_bytes(int n_slots) {
  return (size_t)kWavesPerBlock * wave_lds_units(n_slots) * sizeof(double2);
}

// Make this wave's LDS writes visible to its other lanes.
__device__ __forceinline__ void wave_lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "workgroup");
  __builtin_amdgcn_wave_barrier();
}

template <bool kDebug, bool kElectrons, bool kRegions>
__global__ __launch_bounds__(kBlock, kElectrons ? 2 : NMD_TRANSPORT_MIN_BLOCKS) void transport_kernel(RunParams P) {
  __shared__ float4 s_pal[kMaxPalette];
  __shared__ double s_irho[kMaxPalette];  // 1 / density, for the organ scores
  __shared__ float s_kn[kNGrid];
  __shared__ WaveAcc s_acc[kWavesPerBlock];
  __shared__ float s_start[kWavesPerBlock][6][64];  // decay point and first direction
  // list positions kRegDep .. kRegDep + kLdsDep - 1 of each lane's deposit
  // list (lane fastest, so a wave's accesses to one position are
  // conflict-free); positions beyond them are in global memory
  __shared__ uint32_t s_lv[kWavesPerBlock][kLdsDep][64];  // voxel
  __shared__ uint16_t s_lr[kWavesPerBlock][kLdsDep][64];  // voxel record
  __shared__ double s_le[kWavesPerBlock][kLdsDep][64];    // energy
  extern __shared__ double2 s_dyn[];

  const uint32_t tid = threadIdx.x;
  const uint32_t wave = tid >> 6;
  const uint32_t lane = lane_id();
  const uint32_t gl = blockIdx.x * kBlock + tid;  // lane slot in the overflow lists
  const uint32_t L = P.n_lanes;
  WaveAcc &wa = s_acc[wave];
  const WaveLds wl = wave_lds(s_dyn, wave, P.n_slots);
  float(&sst)[6][64] = s_start[wave];
  uint32_t(&lv)[kLdsDep][64] = s_lv[wave];
  uint16_t(&lr)[kLdsDep][64] = s_lr[wave];
  double(&le)[kLdsDep][64] = s_le[wave];
  constexpr uint32_t kTier = kRegDep + kLdsDep;  // first list position in global memory
  // the global positions go four at a time: a group never passes kDepCap,
  // so no bit index of a 64-bit position mask reaches 64
  static_assert(kDepCap <= 64 && (kDepCap - kTier) % 4 == 0, "deposit list tiers");
  // a history with more organs than slots has more deposit voxels than list
  // registers; three slots and the overflow bit fit the 32-bit id word
  static_assert(kOrgCache >= kRegDep && kOrgCache <= 3, "organ slots");
  static_assert(kStatN == NMD_STAT_N && kStatN <= 16, "run counters");
  // a pass's steps draw at most two words each, all buffered by reserve4
  static_assert(kFlySteps >= 1 && kFlySteps <= 2, "steps per flight pass");

  for (int i = tid; i < P.n_pal; i += kBlock) {
    const float4 q = P.palette[i];
    s_pal[i] = q;
    s_irho[i] = 1.0 / (double)q.w;
  }
  for (int i = tid; i < kNGrid; i += kBlock) s_kn[i] = P.ln2_kn[i];
  if (lane < NMD_LEDGER_N) wa.ledger[lane] = 0.0;
  if (lane < kStatN) wa.stat[lane] = 0ull;
  __syncthreads();

  Stream<kDebug> st;
  st.set_key(P.seed_lo, P.seed_hi);
  st.pid = 0u;

  // lane state: which phase the lane waits for
  constexpr uint32_t kIdle = 0, kFlight = 1, kInteract = 2, kPhotonEnd = 3;
  // bit of psteps set while the photon is outside the inner box (region
  // tracking)
  constexpr uint32_t kOuter = 0x80000000u;
  static_assert(kMaxPhotonSteps < kOuter, "step counter and region bit");
  uint32_t state = kIdle;
  uint32_t ev_v = 0, ev_r = 0;  // pending interaction: voxel and its record
  int ev_t = 0;                 // 1 Compton, 2 photoelectric, 3 Rayleigh
  float px = 0, py = 0, pz = 0, ux = 0, uy = 0, uz = 0, E = 0;
  uint32_t photon = 0, n_real = 0, cnt = 0, psteps = 0;
  // per-history counts, kept per lane for the debug records; otherwise each
  // pass adds its steps and events (ballot popcounts) to the wave's LDS
  // counters, from lane 0 while the whole wave runs in step
  uint32_t h_steps = 0, h_nulls = 0, h_cr = 0, h_pe_esc = 0;
  EnergyParams ep = {};
  // first kRegDep distinct deposit voxels of the history, in registers
  uint32_t rv[kRegDep], rr[kRegDep];
  double re[kRegDep];
#pragma unroll
  for (int i = 0; i < kRegDep; ++i) {
    rv[i] = 0u;
    rr[i] = 0u;
    re[i] = 0.0;
  }
  // the history's organ scores q_o so far: up to kOrgCache organs, their
  // ids packed eight bits each in oc_id; bit 31 is set once the history
  // touches more organs, whose scores are then merged from the deposit list
  uint32_t oc_id = 0u;
  double oc_s[kOrgCache];
#pragma unroll
  for (int k = 0; k < kOrgCache; ++k) oc_s[k] = 0.0;
  unsigned long long run_rel = 0;
  double h_esc = 0, h_disc = 0;  // debug records only

  // wave-uniform state
  int wp = -1;
  unsigned long long cur_next = 0, cur_end = 0, pend_next = 0, pend_end = 0;
  int pend_p = -1;
  bool qdone = false;
  CDesc *D = (CDesc *)P.desc;
  unsigned long long hid0 = 0;

  auto flush_wave = [&]() {
    if (wp < 0) return;
    CDesc *d = D;
    if (lane < NMD_LEDGER_N) {
      const double x = wa.ledger[lane];
      if (x != 0.0) gadd(&d->ledger[lane], x);
      wa.ledger[lane] = 0.0;
    }
    if (lane < kStatN) {
      const unsigned long long x = wa.stat[lane];
      if (lane == 9)
        __hip_atomic_fetch_max(G(&d->stats[9]), x, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      else if (x)
        gadd(&d->stats[lane], x);
      wa.stat[lane] = 0ull;
    }
    const int n_slots = d->n_org + 1;
    for (int i = lane; i < n_slots; i += 64) {
      const double2 o = wl.org[i];
      if (o.x != 0.0 || o.y != 0.0) {
        gadd(&d->organ[i].x, o.x);
        gadd(&d->organ[i].y, o.y);
      }
    }
  };

  // Energy factors at e on the wave's phantom's grid: the pair's (its
  // Klein-Nishina nodes in LDS) or, for an emitter with a line above 511 keV
  // (electron instantiation only), the wide grid, whose Klein-Nishina nodes
  // follow its majorant nodes in global memory.  D is wave-uniform.
  auto ep_at = [&](float e) -> EnergyParams {
    if (kElectrons && D->wide)
      return energy_params(e, D->ln2_major + kNGrid, wl.maj, P.l2emin, kInvDl2W);
    return energy_params(e, s_kn, wl.maj, P.l2emin, P.inv_dl2);
  };

  // load the wave's per-phantom LDS tables
  auto enter_phantom = [&]() {
    for (int i = lane; i < kNGrid; i += 64) wl.maj[i] = G(D->ln2_major)[i];
    for (int i = lane; i <= D->n_org; i += 64) {
      wl.w[i] = G(D->organ_w)[i];
      wl.org[i] = make_double2(0.0, 0.0);
    }
    wave_lds_sync();
    // every photon starts at the emission energy: its factors, once
    const EnergyParams e0 = ep_at(kE0);
    if (lane == 0) {
      wa.ep0[0] = e0.sig;
      wa.ep0[1] = e0.gpe;
      wa.ep0[2] = e0.gr;
      wa.ep0[3] = e0.mu_hat;
      wa.ep0[4] = e0.inv_mu_ln2;
    }
    wave_lds_sync();
  };

  auto start_photon = [&]() {
    const float sgn = photon == 0 ? 1.0f : -1.0f;
    px = sst[0][lane];
    py = sst[1][lane];
    pz = sst[2][lane];
    ux = sgn * sst[3][lane];
    uy = sgn * sst[4][lane];
    uz = sgn * sst[5][lane];
    E = kE0;
    n_real = 0;
    psteps = 0;
    ep.sig = wa.ep0[0];
    ep.gpe = wa.ep0[1];
    ep.gr = wa.ep0[2];
    ep.mu_hat = wa.ep0[3];
    ep.inv_mu_ln2 = wa.ep0[4];
    if (kRegions) {
      const float fx = px * D->inv_dx, fy = py * D->inv_dy, fz = pz * D->inv_dz;
      if (D->out_ratio > 0.0f &&
          !(fx >= D->b0[0] && fx < D->b1[0] && fy >= D->b0[1] && fy < D->b1[1] &&
            fz >= D->b0[2] && fz < D->b1[2])) {
        // a decay outside the inner box: its photons start in the outer region
        psteps = kOuter;
        ep.mu_hat *= D->out_ratio;
        ep.inv_mu_ln2 *= D->inv_out_ratio;
      }
    }
  };

  // Region tracking.  One Woodcock step of path length s, drawn with the
  // current region's majorant, that leaves the inner box or starts outside
  // it.  The majorant is piecewise constant along the ray -- the phantom's
  // inside the box, out_ratio times that outside it -- so the step's optical
  // depth is spent region by region (free flight is memoryless).  Returns
  // the path length to the step's end point and sets the region bit and
  // ep.mu_hat / ep.inv_mu_ln2 to the end point's region.  Without an outer
  // region a ray leaving the box leaves the grid.
  //
  // Distances to the box faces multiply by reciprocals (fast_rcp) rather
  // than dividing: a wave whose lanes diverge runs both walks below, and the
  // rounded divisions cost 3% of the whole run.
  //
  // From inside (photons on their way out of the body), the ray leaves at
  // the box's exit distance tf and the rest of the step stretches by
  // 1 / out_ratio.
  auto box_exit = [&](float s) -> float {
    CDesc *d = D;
    const float p[3] = {px, py, pz}, u[3] = {ux, uy, uz};
    float tf = 3.0e38f;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      const float b = u[a] > 0.0f ? d->bcm1[a] : d->bcm0[a];
      const float ta = u[a] != 0.0f ? (b - p[a]) * fast_rcp(u[a]) : 3.0e38f;
      tf = fminf(tf, fmaxf(ta, 0.0f));
    }
    psteps |= kOuter;
    ep.mu_hat *= d->out_ratio;
    ep.inv_mu_ln2 *= d->inv_out_ratio;
    return d->out_ratio > 0.0f ? tf + (s - tf) * d->inv_out_ratio : 3.0e38f;
  };
  // From outside (photons that started or interacted in the thin outer
  // region): the ray crosses the convex box along one interval [tn, tf] of
  // its parameter, if at all, found once from the start point.
  auto region_step = [&](float s) -> float {
    CDesc *d = D;
    const float p[3] = {px, py, pz}, u[3] = {ux, uy, uz};
    const float mu_out = ep.mu_hat, mu_in = ep.mu_hat * d->inv_out_ratio;
    float tau = s * mu_out;
    float tn = -3.0e38f, tf = 3.0e38f;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      if (u[a] != 0.0f) {
        const float iu = fast_rcp(u[a]);
        const float t1 = (d->bcm0[a] - p[a]) * iu, t2 = (d->bcm1[a] - p[a]) * iu;
        tn = fmaxf(tn, fminf(t1, t2));
        tf = fminf(tf, fmaxf(t1, t2));
      } else if (!(p[a] >= d->bcm0[a] && p[a] < d->bcm1[a])) {
        tf = -3.0e38f;
      }
    }
    const float te = fmaxf(tn, 0.0f);
    // a ray that misses the box, or only touches it, stays outside
    if (!(tn < tf) || !(tf > 0.0f) || tau <= mu_out * te) return s;
    tau -= mu_out * te;
    const float tx = fmaxf(tf, te);  // where the ray leaves the box again
    if (tau <= mu_in * (tx - te)) {
      psteps &= ~kOuter;
      ep.mu_hat = mu_in;
      ep.inv_mu_ln2 *= d->out_ratio;
      return te + tau * fast_rcp(mu_in);
    }
    tau -= mu_in * (tx - te);
    return tx + tau * fast_rcp(mu_out);
  };

  // Score the history's merged deposits: voxel sums S, S2 and the
  // per-history organ scores q_o = sum_{v in o} e_v c / (m_v N_o).
  auto flush_list = [&](bool final_flush) {
    CDesc *d = D;
    double edep = 0.0, sumv = 0.0;
#pragma unroll
    for (int i = 0; i < kRegDep; ++i) {
      if ((uint32_t)i < cnt) {
        gadd(&d->tally[rv[i]].x, re[i]);
        gadd(&d->tally[rv[i]].y, re[i] * re[i]);
        if (kDebug) {
          edep += re[i];
          sumv += (double)rv[i];
        }
      }
    }
#pragma unroll
    for (int j = 0; j < kLdsDep; ++j) {
      if ((uint32_t)(kRegDep + j) < cnt) {
        const uint32_t v = lv[j][lane];
        const double e = le[j][lane];
        gadd(&d->tally[v].x, e);
        gadd(&d->tally[v].y, e * e);
        if (kDebug) {
          edep += e;
          sumv += (double)v;
        }
      }
    }
    // global positions, four per round trip
    for (uint32_t p = kTier; p < cnt; p += 4) {
      uint32_t gv[4];
      double ge[4];
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        const bool in = p + k < cnt;
        const uint32_t idx = (in ? p + k : p) * L + gl;
        gv[k] = G(P.dep_v)[idx];
        ge[k] = G(P.dep_e)[idx];
      }
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        if (p + k < cnt) {
          gadd(&d->tally[gv[k]].x, ge[k]);
          gadd(&d->tally[gv[k]].y, ge[k] * ge[k]);
          if (kDebug) {
            edep += ge[k];
            sumv += (double)gv[k];
          }
        }
      }
    }
    if (d->n_org > 0) {
      if (!(oc_id >> 31)) {
#pragma unroll
        for (int k = 0; k < kOrgCache; ++k) {
          const uint32_t ok = (oc_id >> (8 * k)) & 0xFFu;
          if (ok) {
            atomicAdd(&wl.org[ok].x, oc_s[k]);
            atomicAdd(&wl.org[ok].y, oc_s[k] * oc_s[k]);
          }
        }
      } else {
        // more organs than slots, so more voxels than list registers: merge
        // the organ scores over the whole list, whose registers turn into
        // (organ, score) pairs first
        atomicAdd(&wa.stat[14], 1ull);
#pragma unroll
        for (int i = 0; i < kRegDep; ++i) {
          const uint32_t oi = rr[i] >> 8;
          re[i] = oi ? re[i] * wl.w[oi] * s_irho[rr[i] & 0xFFu] : 0.0;
          rr[i] = oi;
        }
        // one scan of the list per distinct organ, each summing that
        // organ's scores in list order
        unsigned long long rem = 0ull;  // bit p: position p still to merge
#pragma unroll
        for (int i = 0; i < kRegDep; ++i) rem |= rr[i] ? 1ull << i : 0ull;
#pragma unroll
        for (int j = 0; j < kLdsDep; ++j)
          if ((uint32_t)(kRegDep + j) < cnt && (lr[j][lane] >> 8)) rem |= 1ull << (kRegDep + j);
        for (uint32_t p = kTier; p < cnt; p += 4) {
          uint32_t gr[4];
#pragma unroll
          for (int k = 0; k < 4; ++k) gr[k] = G(P.dep_r)[(p + k < cnt ? p + k : p) * L + gl];
#pragma unroll
          for (int k = 0; k < 4; ++k)
            if (p + k < cnt && (gr[k] >> 8)) rem |= 1ull << (p + k);
        }
        while (rem) {
          uint32_t o = 0u;  // the organ of the first position left
          double s = 0.0;
#pragma unroll
          for (int i = 0; i < kRegDep; ++i) {
            if ((rem >> i) & 1ull) {
              o = o ? o : rr[i];
              if (rr[i] == o) {
                s += re[i];
                rem &= ~(1ull << i);
              }
            }
          }
#pragma unroll
          for (int j = 0; j < kLdsDep; ++j) {
            if ((rem >> (kRegDep + j)) & 1ull) {
              const uint32_t r = lr[j][lane];
              o = o ? o : r >> 8;
              if ((r >> 8) == o) {
                s += le[j][lane] * wl.w[o] * s_irho[r & 0xFFu];
                rem &= ~(1ull << (kRegDep + j));
              }
            }
          }
          for (uint32_t p = kTier; p < cnt; p += 4) {
            if (((rem >> p) & 0xFull) == 0ull) continue;
            uint32_t gr[4];
            double ge[4];
#pragma unroll
            for (int k = 0; k < 4; ++k) {
              const uint32_t idx = (p + k < cnt ? p + k : p) * L + gl;
              gr[k] = G(P.dep_r)[idx];
              ge[k] = G(P.dep_e)[idx];
            }
#pragma unroll
            for (int k = 0; k < 4; ++k) {
              if ((rem >> (p + k)) & 1ull) {
                o = o ? o : gr[k] >> 8;
                if ((gr[k] >> 8) == o) {
                  s += ge[k] * wl.w[o] * s_irho[gr[k] & 0xFFu];
                  rem &= ~(1ull << (p + k));
                }
              }
            }
          }
          atomicAdd(&wl.org[o].x, s);
          atomicAdd(&wl.org[o].y, s * s);
        }
      }
    }
    oc_id = 0u;
#pragma unroll
    for (int k = 0; k < kOrgCache; ++k) oc_s[k] = 0.0;
    atomicAdd(&wa.stat[8], (unsigned long long)cnt);
    atomicMax(&wa.stat[9], (unsigned long long)cnt);
    if (kDebug && final_flush) {
      double *r = P.hist_rec + run_rel * kRecN;
      r[0] = edep;
      r[1] = h_esc;
      r[2] = h_cr & 0xFFFFu;
      r[3] = h_pe_esc & 0xFFFFu;
      r[4] = h_cr >> 16;
      r[5] = h_steps;
      r[6] = sumv;
      r[7] = cnt;
      r[8] = st.n_drawn;
      r[9] = h_disc;
    }
    cnt = 0;
  };

  // Add energy e to voxel v (record r16) in the history's deposit list,
  // merged by voxel.  The registers hold the kRegDep most recent distinct
  // voxels (a shift register, so no entry is addressed by a run-time
  // index); the oldest one moves on to the next list position, which is in
  // LDS for the next kLdsDep positions and in global memory after them.
  // Add the score e c / (m_v N_o) of a deposit in organ o to the history's
  // organ slots: q_o sums these over the history's deposits in o.
  auto organ_add = [&](uint32_t r16, double e) {
    const uint32_t o = r16 >> 8;
    if (o == 0u || (oc_id >> 31)) return;
    const double sc = e * wl.w[o] * s_irho[r16 & 0xFFu];
    bool hit = false;
#pragma unroll
    for (int k = 0; k < kOrgCache; ++k) {
      const bool m = ((oc_id >> (8 * k)) & 0xFFu) == o;
      oc_s[k] += m ? sc : 0.0;
      hit = hit || m;
    }
    if (hit) return;
    bool put = false;
#pragma unroll
    for (int k = 0; k < kOrgCache; ++k) {
      const bool f = !put && ((oc_id >> (8 * k)) & 0xFFu) == 0u;
      oc_s[k] = f ? sc : oc_s[k];
      oc_id |= f ? o << (8 * k) : 0u;
      put = put || f;
    }
    if (!put) oc_id |= 0x80000000u;
  };

  auto deposit = [&](uint32_t v, uint32_t r16, double e) {
    organ_add(r16, e);
    bool found = false;
#pragma unroll
    for (int i = 0; i < kRegDep; ++i) {
      const bool m = (uint32_t)i < cnt && rv[i] == v;
      re[i] += m ? e : 0.0;
      found = found || m;
    }
    if (found) return;
    if (cnt > (uint32_t)kRegDep) {
      int hit = -1;
#pragma unroll
      for (int j = 0; j < kLdsDep; ++j)
        if ((uint32_t)(kRegDep + j) < cnt && lv[j][lane] == v) hit = j;
      if (hit >= 0) {
        le[hit][lane] += e;
        return;
      }
      // global positions, four per round trip
      for (uint32_t p = kTier; p < cnt; p += 4) {
        uint32_t gv[4];
#pragma unroll
        for (int k = 0; k < 4; ++k) gv[k] = G(P.dep_v)[(p + k < cnt ? p + k : p) * L + gl];
        int ghit = -1;
#pragma unroll
        for (int k = 3; k >= 0; --k)
          if (p + k < cnt && gv[k] == v) ghit = k;
        if (ghit >= 0) {
          G(P.dep_e)[(p + ghit) * L + gl] += e;
          return;
        }
      }
    }
    if (cnt == (uint32_t)kDepCap) {
      // list full (not reached on the phantoms here; counted): score this
      // deposit on its own, which splits the history's square for voxel v.
      // A history past its organ slots merges its organ scores from the
      // list, which will not hold this deposit: its organ score goes on its
      // own too (the organ mean stays exact, its square is split likewise).
      atomicAdd(&wa.stat[11], 1ull);
      gadd(&D->tally[v].x, e);
      gadd(&D->tally[v].y, e * e);
      const uint32_t o = r16 >> 8;
      if ((oc_id >> 31) && o != 0u) {
        const double q = e * wl.w[o] * s_irho[r16 & 0xFFu];
        atomicAdd(&wl.org[o].x, q);
        atomicAdd(&wl.org[o].y, q * q);
      }
      return;
    }
    if (cnt >= kTier) {
      const uint32_t idx = cnt * L + gl;
      G(P.dep_v)[idx] = rv[kRegDep - 1];
      G(P.dep_e)[idx] = re[kRegDep - 1];
      G(P.dep_r)[idx] = rr[kRegDep - 1];
    } else if (cnt >= (uint32_t)kRegDep) {
      const uint32_t j = cnt - kRegDep;
      lv[j][lane] = rv[kRegDep - 1];
      le[j][lane] = re[kRegDep - 1];
      lr[j][lane] = (uint16_t)rr[kRegDep - 1];
    }
#pragma unroll
    for (int i = kRegDep - 1; i > 0; --i) {
      rv[i] = rv[i - 1];
      re[i] = re[i - 1];
      rr[i] = rr[i - 1];
    }
    rv[0] = v;
    re[0] = e;
    rr[0] = r16;
    ++cnt;
  };

  // Walk a Compton electron of kinetic energy t0 (MeV, exact in FP64) from
  // the photon's event point along (qx, qy, qz), its recoil momentum E d_in
  // - E' d_out, in a straight line voxel by voxel (continuous slowing down;
  // Section 2.1 follows electrons down to its electron cutoff).  In each
  // voxel it loses what the voxel's mass path takes off its range above the
  // cutoff; where that range runs out it leaves all it still has.  Each loss
  // goes to the history's deposit list; returns the energy carried out of
  // the grid.  With is_pos, the particle is the decay's positron, walked from
  // the decay point with the positron tables down to kPosFloor; (ex, ey, ez)
  // then receives the point where its range runs out.
  auto electron_walk = [&](float qx, float qy, float qz, double t0, bool is_pos, float &ex,
                           float &ey, float &ez) -> double {
    CDesc *d = D;
    const float qq = qx * qx + qy * qy + qz * qz;
    ex = px;
    ey = py;
    ez = pz;
    if (!(qq > 0.0f)) {  // no recoil direction: the energy stays at the event
      atomicAdd(&wa.stat[7], 1ull);
      deposit(ev_v, ev_r, t0);
      return 0.0;
    }
    const float qn = __builtin_amdgcn_rsqf(qq);
    qx *= qn;
    qy *= qn;
    qz *= qn;
    const float h[3] = {d->dx, d->dy, d->dz};
    const float pos[3] = {px, py, pz};
    const float qv[3] = {qx, qy, qz};
    const int32_t n[3] = {d->nx, d->ny, d->nz};
    // the event voxel, as the flight step found it (a decay point may round
    // onto the grid's upper face: kept in its voxel)
    int iv[3] = {(int)(px * d->inv_dx), (int)(py * d->inv_dy), (int)(pz * d->inv_dz)};
#pragma unroll
    for (int a = 0; a < 3; ++a) iv[a] = iv[a] < 0 ? 0 : (iv[a] >= n[a] ? n[a] - 1 : iv[a]);
    float tn[3], td[3];
    int sp[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      if (qv[a] > 0.0f) {
        sp[a] = 1;
        tn[a] = ((float)(iv[a] + 1) * h[a] - pos[a]) * fast_rcp(qv[a]);
        td[a] = h[a] * fast_rcp(qv[a]);
      } else if (qv[a] < 0.0f) {
        sp[a] = -1;
        tn[a] = ((float)iv[a] * h[a] - pos[a]) * fast_rcp(qv[a]);
        td[a] = -h[a] * fast_rcp(qv[a]);
      } else {
        sp[a] = 0;
        tn[a] = __builtin_inff();
        td[a] = __builtin_inff();
      }
      tn[a] = fmaxf(tn[a], 0.0f);
    }
    const float cut = is_pos ? kPosFloor : d->e_cut;
    const float inv_dt = is_pos ? d->p_inv_dt : d->e_inv_dt;
    const float *tabs = is_pos ? d->p_tab : d->e_tab;
    const float *inv_drs = is_pos ? d->p_inv_dr : d->e_inv_dr;
    const uint8_t *slots = is_pos ? d->p_slot : d->e_slot;
    double t = t0;
    float tf = (float)t0;
    float s_cur = 0.0f;
    for (;;) {
      const uint32_t v =
          (uint32_t)iv[0] + (uint32_t)n[0] * ((uint32_t)iv[1] + (uint32_t)n[1] * (uint32_t)iv[2]);
      const uint32_t r16 = G(d->rec)[v];
      const uint32_t pq = r16 & 0xFFu;
      const float rho = s_pal[pq].w;
      const uint32_t slot = G(slots)[pq];
      const float *tab = tabs + slot * (2 * kETab);
      int ax = 0;  // ties go to the lower axis
      if (tn[1] < tn[ax]) ax = 1;
      if (tn[2] < tn[ax]) ax = 2;
      const float tnext = ax == 0 ? tn[0] : (ax == 1 ? tn[1] : tn[2]);
      const float mass = rho * (tnext - s_cur);
      // range above the cutoff in this voxel's material
      const float u = (tf - cut) * inv_dt;
      int i = (int)u;
      i = i < 0 ? 0 : (i > kETab - 2 ? kETab - 2 : i);
      const float r0 = G(tab)[i], r1 = G(tab)[i + 1];
      const float range = r0 + (u - (float)i) * (r1 - r0);
      const bool stop = mass >= range;
      // energy after the voxel (the cutoff's share stays with the last one)
      float t1 = 0.0f;
      if (!stop) {
        const float w = (range - mass) * G(inv_drs)[slot];
        int j = (int)w;
        j = j < 0 ? 0 : (j > kETab - 2 ? kETab - 2 : j);
        const float e0 = G(tab)[kETab + j], e1 = G(tab)[kETab + j + 1];
        t1 = fminf(fmaxf(e0 + (w - (float)j) * (e1 - e0), cut), tf);
      }
      atomicAdd(&wa.stat[7], 1ull);
      deposit(v, r16, t - (double)t1);  // one call site: one inlined copy
      if (stop) {
        const float dist = s_cur + fmaxf(range, 0.0f) / rho;
        ex = pos[0] + dist * qx;
        ey = pos[1] + dist * qy;
        ez = pos[2] + dist * qz;
        return 0.0;
      }
      t = (double)t1;
      tf = t1;
      s_cur = tnext;
      int k = -1;
#pragma unroll
      for (int a = 0; a < 3; ++a) {
        if (a == ax) {
          iv[a] += sp[a];
          tn[a] += td[a];
          k = iv[a] < 0 || iv[a] >= n[a] ? a : k;
        }
      }
      if (k >= 0) return t;
    }
  };

  // Start history rel of the wave's chunk in this lane: its decay point and
  // photon direction (or a pending positron), and its first photon.
  auto start_history = [&](unsigned long long rel) {
    run_rel = rel;
    st.start(hid0 + rel);
    float o0, o1, o2, d0, d1, d2;
    if (P.source_kind == 1) {
      o0 = P.po[0];
      o1 = P.po[1];
      o2 = P.po[2];
      d0 = P.pd[0];
      d1 = P.pd[1];
      d2 = P.pd[2];
    } else {
      // alias-table decay voxel: raw word for the column, uniform for the
      // accept test, then a uniform position inside the voxel
      const uint32_t x = st.word();
      const uint32_t j = __umulhi(x, D->n_alias);
      const float ua = st.uniform();
      typedef unsigned int u32x4v __attribute__((ext_vector_type(4)));
      const u32x4v av = G(reinterpret_cast<const u32x4v *>(D->alias))[j];
      const uint4 a = make_uint4(av.x, av.y, av.z, av.w);
      const uint32_t c = ua < __uint_as_float(a.x) ? a.y : a.z;  // x | y << 10 | z << 20
      const uint32_t ix = c & 1023u, iy = (c >> 10) & 1023u, iz = c >> 20;
      o0 = ((float)ix + st.uniform()) * D->dx;
      o1 = ((float)iy + st.uniform()) * D->dy;
      o2 = ((float)iz + st.uniform()) * D->dz;
      if (kElectrons && D->em_on) {
        // a gamma + beta emitter: one uniform picks the line (or none), the
        // beta energy stays in the decay voxel, then the photon's direction
        const double ul = (double)st.uniform();
        int line = -1;
        for (int i = 0; i < D->em_n; ++i)
          if (line < 0 && ul < D->em_cum[i]) line = i;
        sst[0][lane] = o0;
        sst[1][lane] = o1;
        sst[2][lane] = o2;
        cnt = 0;
        h_steps = h_nulls = h_cr = h_pe_esc = 0;
        if (kDebug) h_esc = h_disc = 0.0;
        if (D->em_beta > 0.0f) {
          const uint32_t v0 = ix + (uint32_t)D->nx * (iy + (uint32_t)D->ny * iz);
          atomicAdd(&wa.ledger[0], (double)D->em_beta);
          atomicAdd(&wa.ledger[NMD_LEDGER_DEP_BETA], (double)D->em_beta);
          atomicAdd(&wa.stat[7], 1ull);
          deposit(v0, (uint32_t)G(D->rec)[v0], (double)D->em_beta);
        }
        if (line < 0) {  // no photon: the history ends here
          photon = P.nph;
          state = kPhotonEnd;
          return;
        }
        marsaglia(st, d0, d1, d2);
        // one photon: start_photon takes the last photon of a pair, which it
        // negates
        const float sg = P.nph > 1 ? -1.0f : 1.0f;
        sst[3][lane] = sg * d0;
        sst[4][lane] = sg * d1;
        sst[5][lane] = sg * d2;
        photon = P.nph - 1;
        start_photon();
        E = D->em_e[line];
        atomicAdd(&wa.ledger[0], (double)E);
        ep = ep_at(E);
        if (kRegions && (psteps & kOuter)) {
          ep.mu_hat *= D->out_ratio;
          ep.inv_mu_ln2 *= D->inv_out_ratio;
        }
        state = kFlight;
        return;
      }
      marsaglia(st, d0, d1, d2);
    }
    sst[0][lane] = o0;
    sst[1][lane] = o1;
    sst[2][lane] = o2;
    sst[3][lane] = d0;
    sst[4][lane] = d1;
    sst[5][lane] = d2;
    photon = 0;
    cnt = 0;
    h_steps = h_nulls = h_cr = h_pe_esc = 0;
    if (kDebug) h_esc = h_disc = 0.0;
    if (kElectrons && D->p_on && P.source_kind != 1) {
      // the positron: kinetic energy by inverting the spectrum's CDF
      // (piecewise linear on kPosN intervals; the guide table gives the
      // interval's neighbourhood), then its direction; its walk, and the
      // pair's birth where it ends, wait for an interaction pass (event 4),
      // as the walks of Compton electrons do
      const float u = st.uniform();
      const double ud = (double)u;
      int k = (int)(u * (float)kPosN);
      k = k > kPosN - 1 ? kPosN - 1 : k;
      int i = G(D->p_guide)[k];
      const double *cdf = D->p_cdf;
      while (i < kPosN - 1 && G(cdf)[i + 1] <= ud) ++i;
      const double c0 = G(cdf)[i], c1 = G(cdf)[i + 1];
      const double f = c1 > c0 ? (ud - c0) / (c1 - c0) : 0.0;
      E = (float)(((double)i + f) * (kF18T0 / kPosN));  // the positron's kinetic energy
      marsaglia(st, ux, uy, uz);
      px = o0;
      py = o1;
      pz = o2;
      ev_t = 4;
      state = kInteract;
      return;
    }
    start_photon();
    state = kFlight;
  };

  // Claim histories for the idle lanes from the wave's chunk, claiming new
  // chunks (or switching phantom once the wave has drained) as needed.
  auto refill = [&]() {
    for (;;) {
      const unsigned long long need = __ballot(state == kIdle);
      if (need == 0) break;
      const bool any_busy = need != __ballot(1);
      if (pend_p >= 0 && !any_busy) {
        // switch phantom once every lane of the wave has finished
        flush_wave();
        wp = pend_p;
        D = (CDesc *)(P.desc + P.slot[wp].id);
        st.pid = D->pid;
        hid0 = *G(D->n_done);  // histories already run on this phantom
        cur_next = pend_next;
        cur_end = pend_end;
        pend_p = -1;
        enter_phantom();
      }
      if (cur_next < cur_end) {
        const unsigned long long avail = cur_end - cur_next;
        const uint32_t nneed = __popcll(need);
        const uint32_t r = rank_in(need);
        if (state == kIdle && r < avail) start_history(cur_next + r);
        cur_next += nneed < avail ? nneed : avail;
        continue;
      }
      if (pend_p >= 0 || qdone) break;
      unsigned long long c = 0;
      if (lane == (uint32_t)(__ffsll((long long)__ballot(1)) - 1)) {
        c = __hip_atomic_fetch_add(G(&P.queue[0]), 1ull, __ATOMIC_RELAXED,
                                   __HIP_MEMORY_SCOPE_AGENT);
        if (P.abort_after && c >= P.abort_after) {
          __hip_atomic_exchange(G(&P.queue[1]), 1ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
          c = P.total_chunks;
        }
      }
      c = uniform_u64(c);
      if (c >= P.total_chunks) {
        qdone = true;
        break;
      }
      int p = 0;
      while (p + 1 < P.n_ph && c >= P.slot[p + 1].chunk0) ++p;
      p = __builtin_amdgcn_readfirstlane(p);
      const unsigned long long first = (c - P.slot[p].chunk0) * (unsigned long long)P.chunk;
      unsigned long long last = first + P.chunk;
      last = last < P.slot[p].n_hist ? last : P.slot[p].n_hist;
      if (lane == 0) gadd(&P.desc[P.slot[p].id].stats[12], 1ull);
      if (p == wp) {
        cur_next = first;
        cur_end = last;
      } else {
        pend_p = p;
        pend_next = first;
        pend_end = last;
      }
    }
  };

  // Each pass runs one phase for the lanes in that phase's state: free
  // flights by default, interactions or history turnover once enough lanes
  // wait for them (or no lane can fly).  Gathering lanes by phase keeps the
  // wave's lanes busy on the same code; every lane still consumes its own
  // random stream in order, so results do not depend on the schedule.
  for (;;) {
    const uint32_t n_fly = __popcll(__ballot(state == kFlight));
    const uint32_t n_int = __popcll(__ballot(state == kInteract));
    const uint32_t n_end = __popcll(__ballot(state == kPhotonEnd));
    // a waiting phase runs once it has its threshold of lanes or outnumbers
    // the flights
    const bool go_int = n_int && (n_int >= kPhaseMinInt || n_int >= n_fly);
    const bool go_end = n_end && (n_end >= kPhaseMinEnd || n_end >= n_fly);
    if (go_int && (!go_end || n_int >= n_end)) {
      // ---- interactions at the collision points found by the flights
      uint32_t ek = 0u;  // the event this lane completed: 1 Compton, 2 photoelectric, 3 Rayleigh
      if (state == kInteract) {
        // the draws of one Klein-Nishina attempt and the azimuth (or the
        // Rayleigh pair): generated here for all interacting lanes at once
        if (ev_t != 2) st.reserve4();
        // a rejected Klein-Nishina attempt leaves the lane waiting for the
        // next interaction pass, so no lane holds the wave through retries
        float eps = 1.0f, cost = 1.0f;
        if (ev_t != 1 || klein_nishina_try(st, E * (float)(1.0 / kMeC2), eps, cost)) {
          if (!kElectrons || ev_t != 4) ++n_real;
          ek = (uint32_t)ev_t;
          bool pdone = false;
          double dep = -1.0;  // energy left in voxel ev_v by this event
          // a walk of this event (one call site, so one inlined copy): 1 the
          // Compton electron, 2 the decay's positron; its direction and energy
          uint32_t walk = 0u;
          float wq0 = 0.0f, wq1 = 0.0f, wq2 = 0.0f;
          double wt = 0.0;
          if (ev_t == 1) {
            if (kDebug) ++h_cr;
            const float uphi = st.uniform();
            const float e1 = eps * E;
            dep = (double)E - (double)e1;  // exact in FP64
            bool walked = false;
            if constexpr (kElectrons) {
              if (D->e_cut > 0.0f && dep > (double)D->e_cut) {
                // the electron is tracked from the event point
                const float dx0 = ux, dy0 = uy, dz0 = uz;
                rotate(ux, uy, uz, cost, uphi);
                wq0 = E * dx0 - e1 * ux;
                wq1 = E * dy0 - e1 * uy;
                wq2 = E * dz0 - e1 * uz;
                wt = dep;
                walk = 1u;
                walked = true;
              }
            }
            if (!walked) {
              atomicAdd(&wa.ledger[1], dep);
              rotate(ux, uy, uz, cost, uphi);
            }
            E = e1;
            if (E < P.cutoff) {
              // the cutoff energy stays in the same voxel: T + E' = E (or
              // E' alone when the electron has walked off with T)
              atomicAdd(&wa.ledger[3], (double)E);
              if (!walked) atomicAdd(&wa.stat[7], 1ull);
              dep = walked ? (double)E : dep + (double)E;
              pdone = true;
            } else {
              ep = ep_at(E);
              if (kRegions && (psteps & kOuter)) {  // a Compton event outside the inner box
                ep.mu_hat *= D->out_ratio;
                ep.inv_mu_ln2 *= D->inv_out_ratio;
              }
              if (walked) dep = -1.0;  // nothing left at the event point
            }
          } else if (ev_t == 2) {
            if (kDebug) ++h_pe_esc;
            dep = (double)E;
            atomicAdd(&wa.ledger[2], dep);
            pdone = true;
          } else if (kElectrons && ev_t == 4) {
            // the decay's positron, from the decay point (px, py, pz) along
            // (ux, uy, uz) with kinetic energy E
            wq0 = ux;
            wq1 = uy;
            wq2 = uz;
            wt = (double)E;
            walk = 2u;
          } else {
            if (kDebug) h_cr += 0x10000u;
            const float ct = thomson(st.uniform());
            const float uphi = st.uniform();
            rotate(ux, uy, uz, ct, uphi);
          }
          if constexpr (kElectrons) {
            if (walk) {
              float ex, ey, ez;
              const double out = electron_walk(wq0, wq1, wq2, wt, walk == 2u, ex, ey, ez);
              atomicAdd(&wa.ledger[walk == 2u ? NMD_LEDGER_DEP_POSITRON : 1], wt - out);
              if (out > 0.0) {
                atomicAdd(&wa.ledger[4], out);
                if (kDebug) h_esc += out;
              }
              if (walk == 2u) {
                atomicAdd(&wa.ledger[0], wt);  // the positron's kinetic energy, emitted
                // the pair's tilt: two uniforms drawn with the positron (in
                // the buffer this pass reserved)
                const float u1 = st.uniform(), u2 = st.uniform();
                if (out > 0.0) {
                  // the positron left the grid: the pair is born outside it
                  // and escapes, drawing nothing more
                  atomicAdd(&wa.ledger[4], (double)P.nph * (double)kE0);
                  if (kDebug) {
                    h_esc += (double)P.nph * (double)kE0;
                    h_pe_esc += P.nph << 16;
                  } else {
                    atomicAdd(&wa.stat[10], (unsigned long long)P.nph);
                  }
                  photon = P.nph - 1;
                  pdone = true;
                } else {
                  // the pair is born where the positron stops: the first
                  // photon along the decay's direction d, the second along
                  // -d tilted by a Rayleigh-distributed angle
                  sst[0][lane] = ex;
                  sst[1][lane] = ey;
                  sst[2][lane] = ez;
                  photon = 0;
                  start_photon();
                  float wx = -ux, wy = -uy, wz = -uz;
                  if (D->noncol_sigma > 0.0f) {
                    const float th =
                        D->noncol_sigma * __builtin_sqrtf(-2.0f * __logf(u1));
                    float sth, cth;
                    sincosf(th, &sth, &cth);
                    rotate_sc(wx, wy, wz, cth, sth, u2);
                  }
                  // start_photon takes the second photon's direction negated
                  sst[3][lane] = -wx;
                  sst[4][lane] = -wy;
                  sst[5][lane] = -wz;
                }
              }
            }
          }
          if (dep >= 0.0) {
            atomicAdd(&wa.stat[7], 1ull);
            deposit(ev_v, ev_r, dep);
          }
          if (!pdone && P.max_real && n_real >= P.max_real) {
            atomicAdd(&wa.ledger[5], (double)E);
            if (kDebug) h_disc += E;
            pdone = true;
          }
          state = pdone ? kPhotonEnd : kFlight;
          if (pdone && photon + 1 < P.nph) {
            // the next photon of the pair leaves at once: it draws nothing
            ++photon;
            start_photon();
            state = kFlight;
          }
        }
      }
      if (!kDebug) {
        const uint32_t c1 = __popcll(__ballot(ek == 1u));
        const uint32_t c2 = __popcll(__ballot(ek == 2u));
        const uint32_t c3 = __popcll(__ballot(ek == 3u));
        if (lane == 0) {
          atomicAdd(&wa.stat[4], (unsigned long long)c1);
          atomicAdd(&wa.stat[5], (unsigned long long)c2);
          atomicAdd(&wa.stat[6], (unsigned long long)c3);
        }
      }
      continue;
    }
    if (go_end) {
      // ---- history ends: score the history.  A photon that ends with a
      // photon of its pair still to go starts that one where it ends (in the
      // flight or interaction pass), so lanes wait here only for the history
      // end; the branch for a next photon stays as the general case.
      if (state == kPhotonEnd) {
        if (photon + 1 < P.nph) {
          ++photon;
          start_photon();
          state = kFlight;
        } else {
          atomicAdd(&wa.stat[0], 1ull);
          // an emitter's decay has one photon or none (photon == P.nph)
          atomicAdd(&wa.stat[1], (unsigned long long)((kElectrons && D->em_on)
                                                          ? (photon < P.nph ? 1u : 0u)
                                                          : P.nph));
          if (kDebug) {
            atomicAdd(&wa.stat[2], (unsigned long long)h_steps);
            atomicAdd(&wa.stat[3], (unsigned long long)h_nulls);
            atomicAdd(&wa.stat[4], (unsigned long long)(h_cr & 0xFFFFu));
            atomicAdd(&wa.stat[5], (unsigned long long)(h_pe_esc & 0xFFFFu));
            atomicAdd(&wa.stat[6], (unsigned long long)(h_cr >> 16));
            atomicAdd(&wa.stat[10], (unsigned long long)(h_pe_esc >> 16));
          }
          atomicAdd(&wa.stat[13], (unsigned long long)st.blk);
          flush_list(true);
          state = kIdle;
        }
      }
      refill();
      continue;
    }
    if (n_fly) {
      // ---- Woodcock steps: a flying photon takes up to kFlySteps steps per
      // pass, the next one only after a null collision, so the pass's fixed
      // costs (phase choice, generator refill) are shared by more steps
      uint32_t ns = 0u, nn = 0u, ne = 0u;  // this lane's steps, null collisions, escapes
      uint32_t ng = 0u;                    // and the voxel records it read
      if (state == kFlight) {
        st.reserve4();  // two steps' draws, refilled for all flying lanes at once
        // A step's length does not depend on the voxel it ends in, so the
        // end points of all the pass's steps are known before any voxel
        // record is read: the records are gathered together, and a step's
        // outcome is used only after null collisions on the steps before
        // it.  Arithmetic and draws are those of taking the steps one by one.
        // (Under region tracking a step's majorant depends on the region the
        // previous step ended in: there the steps go one by one.)
        const uint32_t w_len[2] = {st.b0, st.b2};  // each step's length word
        float qx[kFlySteps], qy[kFlySteps], qz[kFlySteps];
        bool qin[kFlySteps];
        uint32_t qv[kFlySteps], qr[kFlySteps];
        if (!kRegions) {
          float cx = px, cy = py, cz = pz;
#pragma unroll
          for (int k = 0; k < kFlySteps; ++k) {
            const float s = -fast_log2(Stream<kDebug>::to_uniform(w_len[k])) * ep.inv_mu_ln2;
            cx += s * ux;
            cy += s * uy;
            cz += s * uz;
            qx[k] = cx;
            qy[k] = cy;
            qz[k] = cz;
            const float fx = cx * D->inv_dx, fy = cy * D->inv_dy, fz = cz * D->inv_dz;
            // written so that a NaN coordinate counts as outside
            qin[k] = fx >= 0.0f && fx < D->fnx && fy >= 0.0f && fy < D->fny && fz >= 0.0f &&
                     fz < D->fnz;
            qv[k] = qin[k] ? (uint32_t)fx + (uint32_t)D->nx *
                                                ((uint32_t)fy + (uint32_t)D->ny * (uint32_t)fz)
                           : 0u;
          }
#pragma unroll
          for (int k = 0; k < kFlySteps; ++k) {
            qr[k] = qin[k] ? (uint32_t)G(D->rec)[qv[k]] : 0u;
            ng += qin[k] ? 1u : 0u;
          }
        }
#pragma unroll
        for (int k = 0; k < kFlySteps; ++k) {
          if (state != kFlight) break;
          if (kDebug) ++h_steps;
          ++ns;
          if (kRegions) {
            float s = -fast_log2(st.take_uniform()) * ep.inv_mu_ln2;
            float fx = (px + s * ux) * D->inv_dx, fy = (py + s * uy) * D->inv_dy,
                  fz = (pz + s * uz) * D->inv_dz;
            // inside the inner box (which lies in the grid), written so that
            // a NaN coordinate counts as outside; a step that leaves the box
            // or starts outside it takes the region walk
            bool in = true;
            if (!(fx >= D->b0[0] && fx < D->b1[0] && fy >= D->b0[1] && fy < D->b1[1] &&
                  fz >= D->b0[2] && fz < D->b1[2]) ||
                (psteps & kOuter)) {
              s = (psteps & kOuter) ? region_step(s) : box_exit(s);
              fx = (px + s * ux) * D->inv_dx;
              fy = (py + s * uy) * D->inv_dy;
              fz = (pz + s * uz) * D->inv_dz;
              in = fx >= 0.0f && fx < D->fnx && fy >= 0.0f && fy < D->fny && fz >= 0.0f &&
                   fz < D->fnz;
            }
            px += s * ux;
            py += s * uy;
            pz += s * uz;
            qin[k] = in;
            qv[k] = in ? (uint32_t)fx + (uint32_t)D->nx *
                                            ((uint32_t)fy + (uint32_t)D->ny * (uint32_t)fz)
                       : 0u;
            qr[k] = in ? (uint32_t)G(D->rec)[qv[k]] : 0u;
            ng += in ? 1u : 0u;
          } else {
            (void)st.take();  // the step's length word, used above
            px = qx[k];
            py = qy[k];
            pz = qz[k];
          }
          if (!qin[k]) {
            atomicAdd(&wa.ledger[4], (double)E);
            if (kDebug) h_pe_esc += 0x10000u;
            ++ne;
            if (kDebug) h_esc += E;
            state = kPhotonEnd;
          } else if ((++psteps & ~kOuter) > kMaxPhotonSteps) {
            // unreachable for valid input; bounds the loop for any input
            atomicAdd(&wa.ledger[5], (double)E);
            if (kDebug) h_disc += E;
            state = kPhotonEnd;
          } else {
            const uint32_t v = qv[k];
            const uint32_t r16 = qr[k];
            const float4 pal = s_pal[r16 & 0xFFu];
            const float mc = pal.x * ep.sig;
            const float mpe = pal.y * ep.gpe;
            const float mr = pal.z * ep.gr;
            const float t = st.take_uniform() * ep.mu_hat;
            int ev = t < mc ? 1 : (t < mc + mpe ? 2 : (t < mc + mpe + mr ? 3 : 0));
            if (ev && !((P.mask >> (ev - 1)) & 1u)) ev = 0;
            if (ev == 0) {
              if (kDebug) ++h_nulls;
              ++nn;
            } else {
              ev_t = ev;
              ev_v = v;
              ev_r = r16;
              state = kInteract;
            }
          }
        }
      }
      if (state == kPhotonEnd && photon + 1 < P.nph) {
        // the next photon of the pair leaves at once: it draws nothing
        ++photon;
        start_photon();
        state = kFlight;
      }
      // per-lane counts are at most 2: count them by their binary digits
      const uint32_t c_g = __popcll(__ballot(ng & 1u)) + 2u * __popcll(__ballot(ng & 2u));
      if (lane == 0) atomicAdd(&wa.stat[15], (unsigned long long)c_g);
      if (!kDebug) {
        const uint32_t c_s = __popcll(__ballot(ns & 1u)) + 2u * __popcll(__ballot(ns & 2u));
        const uint32_t c_n = __popcll(__ballot(nn & 1u)) + 2u * __popcll(__ballot(nn & 2u));
        const uint32_t c_e = __popcll(__ballot(ne != 0u));
        if (lane == 0) {
          atomicAdd(&wa.stat[2], (unsigned long long)c_s);
          atomicAdd(&wa.stat[3], (unsigned long long)c_n);
          atomicAdd(&wa.stat[10], (unsigned long long)c_e);
        }
      }
      continue;
    }
    // no lane is flying or waiting: the wave is idle
    refill();
    if (__ballot(state != kIdle) == 0) {
      if (pend_p >= 0) continue;
      break;
    }
  }
  flush_wave();
}

typedef void (*TransportFn)(RunParams);

static TransportFn transport_fn(bool debug, bool electrons, bool regions) {
  static const TransportFn fn[8] = {
      transport_kernel<false, false, false>, transport_kernel<false, false, true>,
      transport_kernel<false, true, false>,  transport_kernel<false, true, true>,
      transport_kernel<true, false, false>,  transport_kernel<true, false, true>,
      transport_kernel<true, true, false>,   transport_kernel<true, true, true>};
  return fn[(debug ? 4 : 0) + (electrons ? 2 : 0) + (regions ? 1 : 0)];
}

int transport_occupancy_blocks_per_cu(bool debug, bool electrons, bool regions, int n_slots) {
  int nb = 0;
  const hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(
      &nb, transport_fn(debug, electrons, regions), kBlock, transport_dyn_lds_bytes(n_slots));
  return e == hipSuccess && nb > 0 ? nb : 1;
}

hipError_t launch_transport(const RunParams &p, int grid, bool debug, bool electrons,
                            bool regions, hipStream_t s) {
  hipLaunchKernelGGL(transport_fn(debug, electrons, regions), dim3(grid), dim3(kBlock),
                     transport_dyn_lds_bytes(p.n_slots), s, p);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Finalize: Eq. 1 per voxel
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void finalize_kernel(const uint16_t *__restrict__ rec,
                                                       const float4 *__restrict__ palette,
                                                       const double2 *__restrict__ tally,
                                                       uint64_t nvox,
                                                       const unsigned long long *__restrict__ n_done,
                                                       double vkg,
                                                       double a_ts, double *__restrict__ rate,
                                                       double *__restrict__ rel) {
  const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
  const double n = (double)*n_done;
  for (uint64_t v = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; v < nvox; v += stride) {
    const double2 t = tally[v];
    const double rho = (double)palette[rec[v] & 0xFFu].w;
    const double cm = kJPerMeV / (rho * vkg);
    const double mean = t.x / n;
    rate[v] = mean * cm * a_ts;
    if (rel) {
      double r = 0.0;
      if (t.x > 0.0 && n > 1.0) {
        double var = (t.y / n - mean * mean) / (n - 1.0);
        var = var > 0.0 ? var : 0.0;
        r = sqrt(var) / mean;
      }
      rel[v] = r;
    }
  }
}

hipError_t launch_finalize(const uint16_t *rec, const float4 *palette, const double2 *tally,
                           uint64_t nvox, const unsigned long long *n_decays, double vkg,
                           double a_ts, double *rate,
                           double *rel, hipStream_t s) {
  uint64_t blocks = (nvox + 255) / 256;
  if (blocks > 8192) blocks = 8192;
  if (blocks == 0) blocks = 1;
  hipLaunchKernelGGL(finalize_kernel, dim3((uint32_t)blocks), dim3(256), 0, s, rec, palette,
                     tally, nvox, n_decays, vkg, a_ts, rate, rel);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Segmented organ reduction (Eq. 2, Eq. 3), fused with the per-voxel dose
// rate and relative uncertainty of Eq. 1 so the maps need not exist.  Lanes
// of a wave that share a label (neighbouring voxels mostly do) are summed
// with shuffles, then one LDS atomic per (wave, label) and one global atomic
// per (block, label).
// ---------------------------------------------------------------------------
__device__ __forceinline__ void voxel_rate(const double2 t, double rho, double n, double vkg,
                                           double a_ts, double &rate, double &rel) {
  const double cm = kJPerMeV / (rho * vkg);
  const double mean = t.x / n;
  rate = mean * cm * a_ts;
  rel = 0.0;
  if (t.x > 0.0 && n > 1.0) {
    double var = (t.y / n - mean * mean) / (n - 1.0);
    var = var > 0.0 ? var : 0.0;
    rel = sqrt(var) / mean;
  }
}

__global__ __launch_bounds__(256) void organ_kernel(const uint16_t *__restrict__ rec,
                                                    const float4 *__restrict__ palette,
                                                    const double2 *__restrict__ tally,
                                                    uint64_t nvox, int n_org,
                                                    const unsigned long long *__restrict__ n_done,
                                                    double vkg, double a_ts,
                                                    double *__restrict__ out) {
  __shared__ double2 s_acc[kMaxOrganSlots];
  for (int i = threadIdx.x; i < kMaxOrganSlots; i += 256) s_acc[i] = make_double2(0.0, 0.0);
  __syncthreads();
  const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
  const double n = (double)*n_done;
  const uint64_t nround = (nvox + stride - 1) / stride;
  uint64_t v = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const uint32_t lane = lane_id();
  for (uint64_t it = 0; it < nround; ++it, v += stride) {
    uint32_t o = 0;
    double a = 0.0, b = 0.0;
    if (v < nvox) {
      const uint32_t r16 = rec[v];
      o = r16 >> 8;
      if (o != 0 && (int)o <= n_org) {
        double r, e;
        voxel_rate(tally[v], (double)palette[r16 & 0xFFu].w, n, vkg, a_ts, r, e);
        a = r;
        b = e * e;
      }
    }
    bool pending = o != 0 && (int)o <= n_org;
    for (;;) {
      const unsigned long long m = __ballot(pending);
      if (m == 0) break;
      const int lead = __ffsll((long long)m) - 1;
      const uint32_t lo = __shfl(o, lead, 64);
      const bool mine = pending && o == lo;
      const double sa = wave_sum(mine ? a : 0.0);
      const double sb = wave_sum(mine ? b : 0.0);
      if ((int)lane == lead) {
        atomicAdd(&s_acc[lo].x, sa);
        atomicAdd(&s_acc[lo].y, sb);
      }
      pending = pending && !mine;
    }
  }
  __syncthreads();
  for (int i = threadIdx.x; i <= n_org; i += 256) {
    const double2 t = s_acc[i];
    if (t.x != 0.0 || t.y != 0.0) {
      atomicAdd(&out[2 * i], t.x);
      atomicAdd(&out[2 * i + 1], t.y);
    }
  }
}

hipError_t launch_organ_reduce(const uint16_t *rec, const float4 *palette,
                               const double2 *tally, uint64_t nvox, int n_org,
                               const unsigned long long *n_decays,
                               double vkg, double a_ts, double *acc, hipStream_t s) {
  uint64_t blocks = (nvox + 255) / 256;
  if (blocks > 4096) blocks = 4096;
  if (blocks == 0) blocks = 1;
  hipLaunchKernelGGL(organ_kernel, dim3((uint32_t)blocks), dim3(256), 0, s, rec, palette,
                     tally, nvox, n_org, n_decays, vkg, a_ts, acc);
  return hipGetLastError();
}

// Organ sums of a caller-supplied map (for example a denoised dose-rate map),
// with the same wave-level segmentation by label.
__global__ __launch_bounds__(256) void map_organ_kernel(const uint16_t *__restrict__ rec,
                                                        uint64_t nvox, int n_org,
                                                        const double *__restrict__ map,
                                                        double *__restrict__ out) {
  __shared__ double s_acc[kMaxOrganSlots];
  for (int i = threadIdx.x; i < kMaxOrganSlots; i += 256) s_acc[i] = 0.0;
  __syncthreads();
  const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
  const uint64_t nround = (nvox + stride - 1) / stride;
  uint64_t v = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const uint32_t lane = lane_id();
  for (uint64_t it = 0; it < nround; ++it, v += stride) {
    uint32_t o = 0;
    double a = 0.0;
    if (v < nvox) {
      o = (uint32_t)rec[v] >> 8;
      if (o != 0 && (int)o <= n_org) a = map[v];
    }
    bool pending = o != 0 && (int)o <= n_org;
    for (;;) {
      const unsigned long long m = __ballot(pending);
      if (m == 0) break;
      const int lead = __ffsll((long long)m) - 1;
      const uint32_t lo = __shfl(o, lead, 64);
      const bool mine = pending && o == lo;
      const double sa = wave_sum(mine ? a : 0.0);
      if ((int)lane == lead) atomicAdd(&s_acc[lo], sa);
      pending = pending && !mine;
    }
  }
  __syncthreads();
  for (int i = threadIdx.x; i <= n_org; i += 256)
    if (s_acc[i] != 0.0) atomicAdd(&out[i], s_acc[i]);
}

hipError_t launch_map_organ_reduce(const uint16_t *rec, uint64_t nvox, int n_org,
                                   const double *map, double *acc, hipStream_t s) {
  uint64_t blocks = (nvox + 255) / 256;
  if (blocks > 4096) blocks = 4096;
  if (blocks == 0) blocks = 1;
  hipLaunchKernelGGL(map_organ_kernel, dim3((uint32_t)blocks), dim3(256), 0, s, rec, nvox,
                     n_org, map, acc);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Test hooks
// ---------------------------------------------------------------------------
__global__ void debug_sample_kernel(int kind, float e_mev, uint64_t n, uint32_t s0, uint32_t s1,
                                    double *out) {
  const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  Stream<false> st;
  st.init(s0, s1, i, 0);
  switch (kind) {
    case 0:
      for (int j = 0; j < 4; ++j) out[4 * i + j] = (double)st.word();
      break;
    case 1:
      out[i] = (double)st.uniform();
      break;
    case 2: {
      float x, y, z;
      marsaglia(st, x, y, z);
      out[3 * i] = x;
      out[3 * i + 1] = y;
      out[3 * i + 2] = z;
      break;
    }
    case 3: {
      float c;
      const float eps = klein_nishina(st, e_mev * (float)(1.0 / kMeC2), c);
      out[2 * i] = eps;
      out[2 * i + 1] = c;
      break;
    }
    case 5:
      out[i] = (double)thomson(st.uniform());
      break;
    default:
      break;
  }
}

hipError_t launch_debug_sample(int kind, float e_mev, uint64_t n, uint32_t s0, uint32_t s1,
                               double *out, hipStream_t s) {
  const uint64_t blocks = (n + 255) / 256;
  if (blocks == 0) return hipSuccess;
  hipLaunchKernelGGL(debug_sample_kernel, dim3((uint32_t)blocks), dim3(256), 0, s, kind, e_mev, n,
                     s0, s1, out);
  return hipGetLastError();
}

__global__ void debug_source_kernel(const uint4 *alias, uint32_t n_alias, uint32_t pid, uint64_t n,
                                    uint32_t s0, uint32_t s1, uint32_t nx, uint32_t ny,
                                    uint32_t *out) {
  const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  Stream<false> st;
  st.init(s0, s1, i, pid);
  const uint32_t x = st.word();
  const uint32_t j = __umulhi(x, n_alias);
  const float ua = st.uniform();
  const uint4 a = alias[j];
  const uint32_t c = ua < __uint_as_float(a.x) ? a.y : a.z;
  out[i] = (c & 1023u) + nx * (((c >> 10) & 1023u) + ny * (c >> 20));
}

hipError_t launch_debug_source(const uint4 *alias, uint32_t n_alias, uint32_t pid, uint64_t n,
                               uint32_t s0, uint32_t s1, uint32_t nx, uint32_t ny, uint32_t *out,
                               hipStream_t s) {
  const uint64_t blocks = (n + 255) / 256;
  if (blocks == 0) return hipSuccess;
  hipLaunchKernelGGL(debug_source_kernel, dim3((uint32_t)blocks), dim3(256), 0, s, alias, n_alias,
                     pid, n, s0, s1, nx, ny, out);
  return hipGetLastError();
}

__global__ void debug_xs_kernel(const float4 *palette, const uint8_t *used, int n_pal,
                                const float *ln2_kn, const float *ln2_maj, uint64_t n,
                                const float *energies, float *out, float l2emin, float inv_dl2) {
  const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const EnergyParams ep = energy_params(energies[i], ln2_kn, ln2_maj, l2emin, inv_dl2);
  float mx = 0.0f;
  for (int q = 0; q < n_pal; ++q) {
    if (!used[q]) continue;
    const float4 p = palette[q];
    const float mc = p.x * ep.sig, mpe = p.y * ep.gpe, mr = p.z * ep.gr;
    const float mt = mc + mpe + mr;
    mx = mt > mx ? mt : mx;
  }
  out[2 * i] = ep.mu_hat;
  out[2 * i + 1] = mx;
}

hipError_t launch_debug_xs(const float4 *palette, const uint8_t *used, int n_pal,
                           const float *ln2_kn, const float *ln2_major, uint64_t n,
                           const float *energies, float *out, float l2emin, float inv_dl2,
                           hipStream_t s) {
  const uint64_t blocks = (n + 255) / 256;
  if (blocks == 0) return hipSuccess;
  hipLaunchKernelGGL(debug_xs_kernel, dim3((uint32_t)blocks), dim3(256), 0, s, palette, used,
                     n_pal, ln2_kn, ln2_major, n, energies, out, l2emin, inv_dl2);
  return hipGetLastError();
}

// After a run: advance the history counters of the phantoms it covered.
__global__ void advance_kernel(const PhantomDesc *desc, RunIds ids, unsigned long long n) {
  const int i = threadIdx.x;
  if (i < ids.n) *desc[ids.id[i]].n_done += n;
}

hipError_t launch_advance(const PhantomDesc *desc, const RunIds &ids, unsigned long long n,
                          hipStream_t s) {
  hipLaunchKernelGGL(advance_kernel, dim3(1), dim3(kMaxPhantoms), 0, s, desc, ids, n);
  return hipGetLastError();
}

__global__ void fill_u64_kernel(unsigned long long *p, unsigned long long v) { *p = v; }

__global__ void add_f64_kernel(double *__restrict__ dst, const double *__restrict__ src,
                               uint64_t n) {
  const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride)
    dst[i] += src[i];
}

hipError_t launch_add_f64(double *dst, const double *src, uint64_t n, hipStream_t s) {
  if (n == 0) return hipSuccess;
  uint64_t blocks = (n + 255) / 256;
  if (blocks > 8192) blocks = 8192;
  hipLaunchKernelGGL(add_f64_kernel, dim3((uint32_t)blocks), dim3(256), 0, s, dst, src, n);
  return hipGetLastError();
}

__global__ void add_stats_kernel(unsigned long long *dst, const unsigned long long *src) {
  const int i = threadIdx.x;
  if (i >= kStatN) return;
  if (i == NMD_STAT_MAX_MERGED)
    dst[i] = src[i] > dst[i] ? src[i] : dst[i];
  else
    dst[i] += src[i];
}

hipError_t launch_add_stats(unsigned long long *dst, const unsigned long long *src,
                            hipStream_t s) {
  hipLaunchKernelGGL(add_stats_kernel, dim3(1), dim3(64), 0, s, dst, src);
  return hipGetLastError();
}

hipError_t launch_set_u64(unsigned long long *p, unsigned long long v, hipStream_t s) {
  hipLaunchKernelGGL(fill_u64_kernel, dim3(1), dim3(1), 0, s, p, v);
  return hipGetLastError();
}

__global__ void zero_kernel(uint32_t *p, uint64_t n) {
  const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) p[i] = 0u;
}

hipError_t launch_zero_bytes(void *p, uint64_t nbytes, hipStream_t s) {
  const uint64_t n = nbytes / 4;  // callers pass multiples of 4 bytes
  if (n == 0) return hipSuccess;
  uint64_t blocks = (n + 255) / 256;
  if (blocks > 8192) blocks = 8192;
  hipLaunchKernelGGL(zero_kernel, dim3((uint32_t)blocks), dim3(256), 0, s, (uint32_t *)p, n);
  return hipGetLastError();
}

}  // namespace nmd
