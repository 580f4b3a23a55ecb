// Device-side building blocks of the transport kernel: the counter-based
// random stream, the samplers and the direction rotation, all in FP32.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "nmd_internal.hpp"

namespace nmd {

__device__ __forceinline__ float fast_log2(float x) { return __builtin_amdgcn_logf(x); }
__device__ __forceinline__ float fast_exp2(float x) { return __builtin_amdgcn_exp2f(x); }
// v_rcp_f32 and v_sqrt_f32: about an ulp from the rounded results, one
// instruction each where IEEE-rounded division and square root take about a
// dozen.  The samplers below and the transport use them on normal operands;
// their outputs then differ from the rounded ones in the last bits only.
__device__ __forceinline__ float fast_rcp(float x) { return __builtin_amdgcn_rcpf(x); }
__device__ __forceinline__ float fast_sqrt(float x) { return __builtin_amdgcn_sqrtf(x); }

// Philox4x32-10 (Salmon, Moraes, Dror and Shaw, SC'11): ten rounds of two
// 32x32->64 multiplies (one v_mad_u64_u32 each) with a Weyl-sequence key
// schedule.
// kUnroll: straight-line rounds (used where all lanes refill together)
// or a compact loop (the rarer refills inside the physics).
template <bool kUnroll = false>
__device__ __forceinline__ void philox4x32_10(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3,
                                              uint32_t k0, uint32_t k1, uint32_t &o0,
                                              uint32_t &o1, uint32_t &o2, uint32_t &o3) {
  auto round = [&]() {
    const uint64_t p0 = (uint64_t)0xD2511F53u * c0;
    const uint64_t p1 = (uint64_t)0xCD9E8D57u * c2;
    const uint32_t n0 = (uint32_t)(p1 >> 32) ^ c1 ^ k0;
    const uint32_t n2 = (uint32_t)(p0 >> 32) ^ c3 ^ k1;
    c1 = (uint32_t)p1;
    c3 = (uint32_t)p0;
    c0 = n0;
    c2 = n2;
    k0 += 0x9E3779B9u;
    k1 += 0xBB67AE85u;
  };
  if constexpr (kUnroll) {
#pragma unroll
    for (int r = 0; r < 10; ++r) round();
  } else {
#pragma unroll 1
    for (int r = 0; r < 10; ++r) round();
  }
  o0 = c0;
  o1 = c1;
  o2 = c2;
  o3 = c3;
}

// Random stream of one history: counter (block, hid_lo, hid_hi, phantom),
// key (seed_lo, seed_hi); the words of each block are handed out in order.
// Up to eight words are buffered in b0..b7 and consumed from b0 with a shift,
// so no word is ever selected by a run-time index (which would put the
// buffer in scratch memory).  Blocks are generated ahead of use where a
// phase knows its draws -- two at the start of a history, one before the
// two draws of a flight step or the first draws of an interaction -- so
// that all lanes of the phase refill together instead of one call site at a
// time.  Generating ahead never changes which word a draw returns.
template <bool kCount>
struct Stream {
  uint32_t k0, k1, h0, h1, pid, blk;
  uint32_t b0, b1, b2, b3, b4, b5, b6, b7;
  uint32_t pos;      // words buffered
  uint32_t n_drawn;  // uniforms handed out (debug records only)

  // The key and the phantom are the same for every lane of a wave: set them
  // where the wave runs in step, so that they stay in scalar registers.
  __device__ __forceinline__ void set_key(uint32_t seed_lo, uint32_t seed_hi) {
    k0 = seed_lo;
    k1 = seed_hi;
  }
  // Start the stream of history hid: its first two blocks.
  __device__ __forceinline__ void start(unsigned long long hid) {
    h0 = (uint32_t)hid;
    h1 = (uint32_t)(hid >> 32);
    philox4x32_10<true>(0u, h0, h1, pid, k0, k1, b0, b1, b2, b3);
    philox4x32_10<true>(1u, h0, h1, pid, k0, k1, b4, b5, b6, b7);
    blk = 2;
    pos = 8;
    n_drawn = 0;
  }
  __device__ __forceinline__ void init(uint32_t seed_lo, uint32_t seed_hi, unsigned long long hid,
                                       uint32_t p) {
    set_key(seed_lo, seed_hi);
    pid = p;
    start(hid);
  }
  // Append the next block after the pos buffered words (pos <= 4).
  __device__ __forceinline__ void append() {
    uint32_t n0, n1, n2, n3;
    philox4x32_10<true>(blk, h0, h1, pid, k0, k1, n0, n1, n2, n3);
    ++blk;
    const uint32_t q = pos;
    b0 = q == 0 ? n0 : b0;
    b1 = q == 0 ? n1 : (q == 1 ? n0 : b1);
    b2 = q == 0 ? n2 : (q == 1 ? n1 : (q == 2 ? n0 : b2));
    b3 = q == 0 ? n3 : (q == 1 ? n2 : (q == 2 ? n1 : (q == 3 ? n0 : b3)));
    b4 = q == 1 ? n3 : (q == 2 ? n2 : (q == 3 ? n1 : (q == 4 ? n0 : b4)));
    b5 = q == 2 ? n3 : (q == 3 ? n2 : (q == 4 ? n1 : b5));
    b6 = q == 3 ? n3 : (q == 4 ? n2 : b6);
    b7 = q == 4 ? n3 : b7;
    pos = q + 4;
  }
  // Make sure at least two (four) words are buffered.
  __device__ __forceinline__ void reserve2() {
    if (pos < 2) append();
  }
  __device__ __forceinline__ void reserve4() {
    if (pos < 4) append();
  }
  // Next word; the caller guarantees one is buffered.
  __device__ __forceinline__ uint32_t take() {
    const uint32_t x = b0;
    b0 = b1;
    b1 = b2;
    b2 = b3;
    b3 = b4;
    b4 = b5;
    b5 = b6;
    b6 = b7;
    --pos;
    if (kCount) ++n_drawn;
    return x;
  }
  __device__ __forceinline__ uint32_t word() {
    if (pos == 0) {
      philox4x32_10(blk, h0, h1, pid, k0, k1, b0, b1, b2, b3);
      ++blk;
      pos = 4;
    }
    return take();
  }
  static __device__ __forceinline__ float to_uniform(uint32_t x) {
    // ((x >> 9) + 1/2) * 2^-23: exactly representable, strictly inside (0, 1)
    return ((float)(x >> 9) + 0.5f) * (1.0f / 8388608.0f);
  }
  __device__ __forceinline__ float uniform() { return to_uniform(word()); }
  __device__ __forceinline__ float take_uniform() { return to_uniform(take()); }
};

// Isotropic direction, Marsaglia (1972).
template <class S>
__device__ __forceinline__ void marsaglia(S &st, float &dx, float &dy, float &dz) {
  float v1, v2, s;
  do {
    v1 = 2.0f * st.uniform() - 1.0f;
    v2 = 2.0f * st.uniform() - 1.0f;
    s = v1 * v1 + v2 * v2;
  } while (s >= 1.0f);
  const float q = 2.0f * fast_sqrt(1.0f - s);
  dx = v1 * q;
  dy = v2 * q;
  dz = 1.0f - 2.0f * s;
}

// Klein-Nishina energy ratio eps = E'/E and cos(theta) by the Butcher-Messel
// composition-rejection: the eps density (1/eps + eps) g(eps) on [eps0, 1]
// is split into the exactly sampled 1/eps and eps parts, weighted by
// ln(1/eps0) and (1 - eps0^2)/2, and thinned by g = 1 - eps sin^2/(1+eps^2).
// One attempt draws three uniforms and returns whether it is accepted,
// with eps and cos(theta) of the attempt.
template <class S>
__device__ __forceinline__ bool klein_nishina_try(S &st, float k, float &eps, float &cost) {
  const float a = 1.0f + 2.0f * k;
  const float eps0 = fast_rcp(a);
  const float e02 = eps0 * eps0;
  const float a1 = fast_log2(a) * 0.69314718055994531f;  // ln(1 + 2k)
  const float a2 = 0.5f * (1.0f - e02);
  const float inv_k = fast_rcp(k);
  const float r1 = st.uniform();
  const float r2 = st.uniform();
  const float r3 = st.uniform();
  if (r1 * (a1 + a2) < a1)
    eps = fast_exp2(-a1 * r2 * 1.4426950408889634f);
  else
    eps = fast_sqrt(e02 + (1.0f - e02) * r2);
  const float t = (1.0f - eps) * inv_k * fast_rcp(eps);
  const float sin2 = t * (2.0f - t);
  const float g = 1.0f - eps * sin2 * fast_rcp(1.0f + eps * eps);
  cost = 1.0f - t;
  return r3 < g;
}
template <class S>
__device__ __forceinline__ float klein_nishina(S &st, float k, float &cost) {
  float eps;
  while (!klein_nishina_try(st, k, eps, cost)) {
  }
  return eps;
}

// Thomson polar angle: invert the CDF (c^3 + 3c + 4)/8 with Cardano's root
// c = w - 1/w, w = cbrt(a + sqrt(a^2 + 1)), a = 4u - 2; the odd symmetry in
// a keeps the cancellation away.
__device__ __forceinline__ float thomson(float u) {
  const float a = 4.0f * u - 2.0f;
  const float aa = fabsf(a);
  const float w = cbrtf(aa + __builtin_sqrtf(aa * aa + 1.0f));
  return copysignf(w - 1.0f / w, a);
}

// Rotate (ux,uy,uz) by the polar angle theta (its cosine and sine given) and
// the azimuth 2 pi uphi about the orthonormal basis of Duff et al. (JCGT
// 2017): no pole special case and no loss of precision near the z axis in
// FP32.
__device__ __forceinline__ void rotate_sc(float &ux, float &uy, float &uz, float cost, float sint,
                                          float uphi) {
  const float cphi = __builtin_amdgcn_cosf(uphi);  // argument in revolutions
  const float sphi = __builtin_amdgcn_sinf(uphi);
  const float sg = uz >= 0.0f ? 1.0f : -1.0f;
  const float a = -fast_rcp(sg + uz);
  const float b = ux * uy * a;
  const float sc = sint * cphi, ss = sint * sphi;
  const float nu = cost * ux + sc * (1.0f + sg * ux * ux * a) + ss * b;
  const float nv = cost * uy + sc * (sg * b) + ss * (sg + uy * uy * a);
  const float nw = cost * uz - sc * (sg * ux) - ss * uy;
  const float n = __builtin_amdgcn_rsqf(nu * nu + nv * nv + nw * nw);
  ux = nu * n;
  uy = nv * n;
  uz = nw * n;
}

// The same with sin(theta) = sqrt(1 - cos^2(theta)), for angles that are not
// small (small ones lose their digits there and pass the sine instead).
__device__ __forceinline__ void rotate(float &ux, float &uy, float &uz, float cost, float uphi) {
  rotate_sc(ux, uy, uz, cost, fast_sqrt(fmaxf(0.0f, 1.0f - cost * cost)), uphi);
}

// Energy-dependent factors: mu_C = cC * sig, mu_PE = cPE * gpe, mu_R = cR * gr
// and the majorant.  sig and the majorant are log-log interpolated on the
// 256-node grid; the photoelectric and Rayleigh power laws are exact.
struct EnergyParams {
  float sig, gpe, gr, mu_hat, inv_mu_ln2;
};

__device__ __forceinline__ EnergyParams energy_params(float E, const float *ln2_kn,
                                                      const float *ln2_maj,
                                                      float l2emin, float inv_dl2) {
  EnergyParams p;
  const float t = (fast_log2(E) - l2emin) * inv_dl2;
  int i = (int)floorf(t);
  i = i < 0 ? 0 : (i > kNGrid - 2 ? kNGrid - 2 : i);
  const float f = t - (float)i;
  const float k0 = ln2_kn[i], k1 = ln2_kn[i + 1];
  const float m0 = ln2_maj[i], m1 = ln2_maj[i + 1];
  p.sig = fast_exp2(k0 + f * (k1 - k0));
  p.mu_hat = kKappa * fast_exp2(m0 + f * (m1 - m0));
  p.inv_mu_ln2 = 0.69314718055994531f * fast_rcp(p.mu_hat);
  const float ie = fast_rcp(E);
  p.gr = ie * ie;
  p.gpe = p.gr * ie;
  return p;
}

}  // namespace nmd
