// Measured ceilings of the hardware paths the transport kernel leans on, and
// per-unit instruction probes that build the kernel's VALU work model.
//
//   ceiling_*  HBM stream copy, random FP64 atomics, random 2-byte gathers,
//              an FP32 FMA loop, a 32x32->64-bit multiply loop and a BF16
//              matrix-core loop; each timed with HIP events on the context
//              stream.
//   unit_kernel<K>  one unit of the transport's work (a Philox block, a
//              uniform, a Woodcock step, a Compton or Rayleigh event, a
//              history start, a merged-deposit flush) per lane and loop
//              iteration, with every lane active: SQ_INSTS_VALU of these
//              dispatches, less the empty loop, gives the VALU instructions
//              of one unit on a non-divergent wave.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <vector>

#include "../../include/nmdose_probe.h"
#include "nmd_device.hpp"
#include "nmd_internal.hpp"

namespace nmd {
namespace {

__device__ __forceinline__ uint32_t mix32(uint32_t x) {
  // integer hash (lowbias32 constants), for scattered addresses
  x ^= x >> 16;
  x *= 0x7feb352du;
  x ^= x >> 15;
  x *= 0x846ca68bu;
  x ^= x >> 16;
  return x;
}

// ---- ceilings --------------------------------------------------------------

__global__ __launch_bounds__(256) void ceil_copy_kernel(const float4 *__restrict__ a,
                                                        float4 *__restrict__ b, uint64_t n) {
  const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride)
    b[i] = a[i];
}

constexpr int kOpsPerLane = 64;

__global__ __launch_bounds__(256) void ceil_atomic_kernel(double *t, uint32_t mask,
                                                          uint32_t salt) {
  const uint32_t g = blockIdx.x * blockDim.x + threadIdx.x;
  uint32_t h = mix32(g ^ salt);
#pragma unroll 8
  for (int k = 0; k < kOpsPerLane; ++k) {
    h = mix32(h + (uint32_t)k);
    __hip_atomic_fetch_add((__attribute__((address_space(1))) double *)(t + (h & mask)), 1.0,
                           __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
}

__global__ __launch_bounds__(256) void ceil_gather_kernel(const uint16_t *__restrict__ r,
                                                          uint32_t n, uint32_t salt,
                                                          uint32_t *__restrict__ out) {
  const uint32_t g = blockIdx.x * blockDim.x + threadIdx.x;
  uint32_t h = mix32(g ^ salt), acc = 0;
#pragma unroll 8
  for (int k = 0; k < kOpsPerLane; ++k) {
    h = mix32(h + (uint32_t)k);
    acc += r[__umulhi(h, n)];
  }
  if (acc == 0xFFFFFFFFu) out[0] = acc;  // keeps the loads; never true
}

constexpr int kAluIters = 4096;

__global__ __launch_bounds__(256) void ceil_fma_kernel(float seed, float *out) {
  float a[8];
#pragma unroll
  for (int j = 0; j < 8; ++j) a[j] = seed + (float)(threadIdx.x + j);
  for (int i = 0; i < kAluIters; ++i) {
#pragma unroll
    for (int j = 0; j < 8; ++j) a[j] = __builtin_fmaf(a[j], 0.999f, 0.001f);
  }
  float s = 0.0f;
#pragma unroll
  for (int j = 0; j < 8; ++j) s += a[j];
  if (s == -1.0f) out[0] = s;  // keeps the loop; never true for these inputs
}

__global__ __launch_bounds__(256) void ceil_mul64_kernel(uint32_t seed, uint32_t *out) {
  uint32_t a[8];
#pragma unroll
  for (int j = 0; j < 8; ++j) a[j] = seed + threadIdx.x * 8 + j;
  for (int i = 0; i < kAluIters; ++i) {
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      const uint64_t p = (uint64_t)0xD2511F53u * a[j];
      a[j] = (uint32_t)(p >> 32) ^ (uint32_t)p;
    }
  }
  uint32_t s = 0;
#pragma unroll
  for (int j = 0; j < 8; ++j) s ^= a[j];
  if (s == 0x12345678u) out[0] = s;
}

typedef float f32x4_t __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8_t __attribute__((ext_vector_type(8)));
typedef uint32_t u32x4_t __attribute__((ext_vector_type(4)));

__global__ __launch_bounds__(256) void ceil_mfma_kernel(uint32_t seed, float *out) {
  const u32x4_t a = {seed, seed ^ threadIdx.x, seed + 1u, seed + threadIdx.x};
  const u32x4_t b = {seed ^ 0x3c003c00u, seed, seed + 7u, threadIdx.x};
  f32x4_t c[4] = {};
  for (int i = 0; i < kAluIters / 4; ++i) {
#pragma unroll
    for (int j = 0; j < 4; ++j)
      c[j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16x8_t, a),
                                                     __builtin_bit_cast(bf16x8_t, b), c[j], 0, 0,
                                                     0);
  }
  float s = 0.0f;
#pragma unroll
  for (int j = 0; j < 4; ++j) s += c[j][0] + c[j][1] + c[j][2] + c[j][3];
  if (s == -1.0f) out[0] = s;
}

// ---- per-unit probes ---------------------------------------------------------

constexpr int kUnitGridN = 64;  // side of the probe's voxel grid (64^3 u16 records)

struct UnitArgs {
  const uint16_t *rec;  // [64^3], palette index | organ << 8
  const float4 *pal;    // [4]
  const float *ln2_kn;  // [kNGrid]
  const float *ln2_maj; // [kNGrid]
  const uint4 *alias;   // [kUnitGridN^3]
  double *tally;        // [64^3] pairs
  float l2emin, inv_dl2;
  uint32_t k0, k1;
  uint32_t iters;
  uint32_t *out;
};

// Uniforms of a probe: the LCG word of the iteration xor a constant of the
// draw (one VALU xor each, folded into the unit's count), converted the way
// the transport converts its Philox words.
struct ProbeDraws {
  uint32_t x, k;
  __device__ __forceinline__ float uniform() {
    k += 0x9e3779b9u;
    return Stream<false>::to_uniform(x ^ k);
  }
};

template <int K>
__global__ __launch_bounds__(256) void unit_kernel(UnitArgs A) {
  __shared__ float4 s_pal[4];
  __shared__ float s_kn[kNGrid], s_maj[kNGrid];
  for (int i = threadIdx.x; i < kNGrid; i += 256) {
    s_kn[i] = A.ln2_kn[i];
    s_maj[i] = A.ln2_maj[i];
  }
  if (threadIdx.x < 4) s_pal[threadIdx.x] = A.pal[threadIdx.x];
  __syncthreads();
  const uint32_t g = blockIdx.x * blockDim.x + threadIdx.x;
  // an LCG word per iteration feeds every probe; the empty loop (K = 0)
  // measures it and the loop control
  uint32_t x = mix32(g + 1u);
  uint32_t acc = 0u;
  float fx = 0.5f + (float)(g & 31u), fy = 0.5f + (float)((g >> 5) & 31u), fz = 7.5f;
  float ux = 0.48f, uy = 0.6f, uz = 0.64f, E = 0.3f;
  double dacc = 0.0;
  const EnergyParams ep0 = energy_params(0.511f, s_kn, s_maj, A.l2emin, A.inv_dl2);
  for (uint32_t it = 0; it < A.iters; ++it) {
    x = x * 1664525u + 1013904223u;
    ProbeDraws dr{x, 0u};
    if constexpr (K == 0) {
      acc ^= x;
    } else if constexpr (K == 1) {  // one Philox4x32-10 block
      uint32_t o0, o1, o2, o3;
      philox4x32_10<true>(it, x, g, 0u, A.k0, A.k1, o0, o1, o2, o3);
      acc ^= o0 ^ o1 ^ o2 ^ o3;
    } else if constexpr (K == 2) {  // one uniform from a word
      acc ^= __float_as_uint(Stream<false>::to_uniform(x));
    } else if constexpr (K == 3) {  // one Woodcock step (two uniforms)
      const float u1 = dr.uniform();
      const float u2 = dr.uniform();
      const float s = -fast_log2(u1) * ep0.inv_mu_ln2;
      fx += s * ux;
      fy += s * uy;
      fz += s * uz;
      // voxel units: the probe grid has 1 cm voxels
      const bool in = fx >= 0.0f && fx < 64.0f && fy >= 0.0f && fy < 64.0f && fz >= 0.0f &&
                      fz < 64.0f;
      // keep the walk inside the grid without a branch
      fx = in ? fx : 0.5f;
      fy = in ? fy : 0.5f;
      fz = in ? fz : 0.5f;
      const uint32_t v = (uint32_t)fx + 64u * ((uint32_t)fy + 64u * (uint32_t)fz);
      const uint32_t r16 = A.rec[v];
      const float4 p = s_pal[r16 & 3u];
      const float mc = p.x * ep0.sig, mpe = p.y * ep0.gpe, mr = p.z * ep0.gr;
      const float t = u2 * ep0.mu_hat;
      const int ev = t < mc ? 1 : (t < mc + mpe ? 2 : (t < mc + mpe + mr ? 3 : 0));
      acc += (uint32_t)ev + v;
    } else if constexpr (K == 4) {  // one Compton event (four uniforms)
      float eps, cost;
      const bool ok = klein_nishina_try(dr, E * (float)(1.0 / kMeC2), eps, cost);
      const float uphi = dr.uniform();
      const float e1 = eps * E;
      dacc += (double)E - (double)e1;
      rotate(ux, uy, uz, cost, uphi);
      const float en = ok ? fmaxf(e1, 0.02f) : E;
      const EnergyParams ep = energy_params(en, s_kn, s_maj, A.l2emin, A.inv_dl2);
      E = en < 0.05f ? 0.3f : en;
      acc ^= __float_as_uint(ep.mu_hat) ^ __float_as_uint(ep.sig) ^ __float_as_uint(ep.gpe) ^
             __float_as_uint(ep.gr) ^ __float_as_uint(ep.inv_mu_ln2);
    } else if constexpr (K == 5) {  // one Rayleigh event (two uniforms)
      const float ct = thomson(dr.uniform());
      rotate(ux, uy, uz, ct, dr.uniform());
      acc ^= __float_as_uint(ux);
    } else if constexpr (K == 6) {  // one history start (six uniforms)
      const uint32_t j = __umulhi(x, (uint32_t)(kUnitGridN * kUnitGridN * kUnitGridN));
      const float ua = dr.uniform();
      const uint4 a = A.alias[j];
      const uint32_t c = ua < __uint_as_float(a.x) ? a.y : a.z;
      const uint32_t ix = c & 1023u, iy = (c >> 10) & 1023u, iz = c >> 20;
      const float o0 = ((float)ix + dr.uniform()) * 0.2f;
      const float o1 = ((float)iy + dr.uniform()) * 0.2f;
      const float o2 = ((float)iz + dr.uniform()) * 0.3f;
      // one Marsaglia attempt (a decay makes 4/pi of them on average)
      const float v1 = 2.0f * dr.uniform() - 1.0f;
      const float v2 = 2.0f * dr.uniform() - 1.0f;
      const float s2 = v1 * v1 + v2 * v2;
      const float q = 2.0f * __builtin_sqrtf(fmaxf(1.0f - s2, 0.0f));
      const float d0 = v1 * q, d1 = v2 * q, d2 = 1.0f - 2.0f * s2;
      acc ^= __float_as_uint(o0 + o1 + o2) ^ __float_as_uint(d0 * d1 * d2) ^ (uint32_t)(s2 < 1.0f);
    } else if constexpr (K == 7) {  // one merged deposit flushed to the tally (one uniform)
      const uint32_t v = __umulhi(mix32(x), 64u * 64u * 64u);
      const double e = (double)dr.uniform();
      __hip_atomic_fetch_add((__attribute__((address_space(1))) double *)(A.tally + 2 * v), e,
                             __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      __hip_atomic_fetch_add((__attribute__((address_space(1))) double *)(A.tally + 2 * v + 1),
                             e * e, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
  }
  acc ^= __float_as_uint(fx + fy + fz + ux + uy + uz + E) ^ (uint32_t)(dacc > 1e300);
  if (acc == 0x5bd1e995u) A.out[0] = acc;  // keeps the work; practically never true
}

// LDS lane patterns (NMD_LDS_*): byte offset of lane L's 16-byte access.
constexpr int kLdsQuads = 2048;  // 32 KiB of 16-byte quads
__host__ __device__ inline uint32_t lds_offset(int p, int L) {
  const int lx = L & 15, g = L >> 4;
  switch (p) {
    case NMD_LDS_CONTIGUOUS: return 16 * L;
    case NMD_LDS_HALO48: return 48 * lx + 48 * (g >> 1) + 16 * (g & 1);
    case NMD_LDS_P48_SAME: return 48 * lx;
    case NMD_LDS_P48_FAR: return 48 * lx + 768 * g;
    case NMD_LDS_P80_G16: return 80 * lx + 16 * g;
    case NMD_LDS_P48_LANE: return 48 * L;
    case NMD_LDS_GROUP_MAJOR: return 16 * lx + 256 * g;
    case NMD_LDS_P64_G16: return 64 * lx + 16 * g;
    case NMD_LDS_HALO32: return 32 * lx + 32 * (g >> 1) + 16 * (g & 1);
    case NMD_LDS_P48_G16: return 48 * lx + 16 * g;
    case NMD_LDS_STORE48: return 48 * (L >> 1) + 16 * (L & 1);
    case NMD_LDS_P96_G16: return 96 * lx + 16 * g;
  }
  return 0;
}

// Each iteration adds (it mod 4) x 4 KiB: the same banks, a fresh address,
// so that no access can be folded into another.
__global__ __launch_bounds__(256) void lds_read_kernel(int p, uint32_t iters, uint32_t *out) {
  __shared__ u32x4_t s[kLdsQuads];
  for (int i = threadIdx.x; i < kLdsQuads; i += 256) s[i] = u32x4_t{(uint32_t)i, 1u, 2u, 3u};
  __syncthreads();
  const uint32_t q = lds_offset(p, threadIdx.x & 63) / 16;
  u32x4_t acc = {0u, 0u, 0u, 0u};
  for (uint32_t it = 0; it < iters; ++it) {
    acc += s[q + ((it & 3u) << 8)];
    __asm__ volatile("" ::: "memory");
  }
  out[threadIdx.x & 63] = acc.x ^ acc.y ^ acc.z ^ acc.w;
}

__global__ __launch_bounds__(256) void lds_write_kernel(int p, uint32_t iters, uint32_t *out) {
  __shared__ u32x4_t s[kLdsQuads];
  const uint32_t q = lds_offset(p, threadIdx.x & 63) / 16;
  u32x4_t v = {threadIdx.x, 1u, 2u, 3u};
  for (uint32_t it = 0; it < iters; ++it) {
    v.x += 1u;
    s[q + ((it & 3u) << 8)] = v;
    __asm__ volatile("" ::: "memory");
  }
  __syncthreads();
  out[threadIdx.x & 63] = s[threadIdx.x].x;
}

}  // namespace
}  // namespace nmd

using namespace nmd;

namespace {

struct Timer {
  hipEvent_t a = nullptr, b = nullptr;
  ~Timer() {
    if (a) (void)hipEventDestroy(a);
    if (b) (void)hipEventDestroy(b);
  }
};

// Device buffer released on scope exit.
struct Buf {
  void *p = nullptr;
  ~Buf() {
    if (p) (void)hipFree(p);
  }
};

nmd_status alloc(nmd_ctx *c, Buf &b, size_t n) {
  hipError_t e = hipMalloc(&b.p, n);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    return ctx_fail(c, NMD_E_OOM, "probe buffer of %zu bytes: %s", n, hipGetErrorString(e));
  }
  return NMD_OK;
}

}  // namespace

extern "C" {

nmd_status nmd_probe_ceiling(nmd_ctx *c, int32_t kind, uint64_t bytes, uint32_t repeats,
                             double *rate, double *ms) {
  nmd_status s = ctx_enter(c);
  if (s) return s;
  if (!rate) return ctx_fail(c, NMD_E_INVALID, "rate output is required");
  if (repeats == 0 || repeats > 1000) return ctx_fail(c, NMD_E_INVALID, "repeats must be 1..1000");
  const bool sized = kind == NMD_CEIL_COPY || kind == NMD_CEIL_ATOMIC_F64 ||
                     kind == NMD_CEIL_GATHER_U16;
  if (kind < 0 || kind > NMD_CEIL_MFMA_BF16) return ctx_fail(c, NMD_E_INVALID, "unknown ceiling");
  if (sized && (bytes < (1u << 20) || bytes > (8ull << 30) || (bytes & (bytes - 1))))
    return ctx_fail(c, NMD_E_INVALID, "bytes must be a power of two in [1 MiB, 8 GiB]");
  hipStream_t st = ctx_stream(c);
  Buf buf, buf2, sink;
  if ((s = alloc(c, sink, 256))) return s;
  if (sized && (s = alloc(c, buf, bytes))) return s;
  if (kind == NMD_CEIL_COPY && (s = alloc(c, buf2, bytes))) return s;
  if (sized) {
    if ((s = ctx_hip(c, launch_zero_bytes(buf.p, bytes, st), "zero"))) return s;
  }
  const int grid = 8192;
  auto launch = [&](uint32_t salt) {
    switch (kind) {
      case NMD_CEIL_COPY:
        hipLaunchKernelGGL(ceil_copy_kernel, dim3(grid), dim3(256), 0, st,
                           (const float4 *)buf.p, (float4 *)buf2.p, bytes / 16);
        break;
      case NMD_CEIL_ATOMIC_F64:
        hipLaunchKernelGGL(ceil_atomic_kernel, dim3(grid), dim3(256), 0, st, (double *)buf.p,
                           (uint32_t)(bytes / 8 - 1), salt);
        break;
      case NMD_CEIL_GATHER_U16:
        hipLaunchKernelGGL(ceil_gather_kernel, dim3(grid), dim3(256), 0, st,
                           (const uint16_t *)buf.p, (uint32_t)(bytes / 2), salt,
                           (uint32_t *)sink.p);
        break;
      case NMD_CEIL_VALU_FMA:
        hipLaunchKernelGGL(ceil_fma_kernel, dim3(grid), dim3(256), 0, st, 1.0f + salt,
                           (float *)sink.p);
        break;
      case NMD_CEIL_MUL64:
        hipLaunchKernelGGL(ceil_mul64_kernel, dim3(grid), dim3(256), 0, st, salt,
                           (uint32_t *)sink.p);
        break;
      default:
        hipLaunchKernelGGL(ceil_mfma_kernel, dim3(grid), dim3(256), 0, st, salt,
                           (float *)sink.p);
        break;
    }
  };
  launch(0u);  // warm-up
  Timer t;
  if ((s = ctx_hip(c, hipEventCreate(&t.a), "hipEventCreate"))) return s;
  if ((s = ctx_hip(c, hipEventCreate(&t.b), "hipEventCreate"))) return s;
  if ((s = ctx_hip(c, hipEventRecord(t.a, st), "hipEventRecord"))) return s;
  for (uint32_t r = 0; r < repeats; ++r) launch(r + 1u);
  if ((s = ctx_hip(c, hipEventRecord(t.b, st), "hipEventRecord"))) return s;
  if ((s = ctx_hip(c, hipEventSynchronize(t.b), "hipEventSynchronize"))) return s;
  if ((s = ctx_hip(c, hipGetLastError(), "probe launch"))) return s;
  float el = 0.0f;
  if ((s = ctx_hip(c, hipEventElapsedTime(&el, t.a, t.b), "hipEventElapsedTime"))) return s;
  const double sec = (double)el * 1e-3 / repeats;
  const double lanes = (double)grid * 256.0;
  double work = 0.0;
  switch (kind) {
    case NMD_CEIL_COPY: work = 2.0 * (double)bytes; break;          // bytes read + written
    case NMD_CEIL_ATOMIC_F64:
    case NMD_CEIL_GATHER_U16: work = lanes * kOpsPerLane; break;    // operations
    case NMD_CEIL_VALU_FMA:
    case NMD_CEIL_MUL64: work = lanes * kAluIters * 8.0; break;     // lane-operations
    default: work = (double)grid * 4.0 * (kAluIters / 4) * 4 * 2.0 * 16 * 16 * 32; break;  // FLOP
  }
  *rate = work / sec;
  if (ms) *ms = sec * 1e3;
  return NMD_OK;
}

nmd_status nmd_probe_unit(nmd_ctx *c, int32_t kind, uint32_t iters, uint32_t blocks,
                          double *ms) {
  nmd_status s = ctx_enter(c);
  if (s) return s;
  if (kind < 0 || kind >= NMD_UNIT_N) return ctx_fail(c, NMD_E_INVALID, "unknown unit");
  if (iters == 0 || iters > (1u << 20) || blocks == 0 || blocks > 65536)
    return ctx_fail(c, NMD_E_INVALID, "iters in 1..2^20 and blocks in 1..65536 required");
  hipStream_t st = ctx_stream(c);
  const size_t nv = (size_t)kUnitGridN * kUnitGridN * kUnitGridN;
  Buf rec, pal, kn, maj, alias, tally, sink;
  if ((s = alloc(c, rec, nv * 2)) || (s = alloc(c, pal, 4 * sizeof(float4))) ||
      (s = alloc(c, kn, kNGrid * 4)) || (s = alloc(c, maj, kNGrid * 4)) ||
      (s = alloc(c, alias, nv * sizeof(uint4))) || (s = alloc(c, tally, nv * 16)) ||
      (s = alloc(c, sink, 256)))
    return s;
  // soft tissue everywhere: palette 0; tables of a plausible shape
  std::vector<uint16_t> hr(nv, 0);
  for (size_t i = 0; i < nv; ++i) hr[i] = (uint16_t)((i * 2654435761u >> 30) & 3u);
  const float4 hp[4] = {{0.055f, 1e-7f, 1e-8f, 1.0f}, {0.014f, 3e-8f, 3e-9f, 0.26f},
                        {0.1f, 8e-7f, 4e-8f, 1.85f}, {6e-5f, 1e-10f, 1e-11f, 0.0012f}};
  std::vector<float> hk(kNGrid), hm(kNGrid);
  for (int i = 0; i < kNGrid; ++i) {
    hk[i] = -0.02f * (float)i;
    hm[i] = -2.5f - 0.02f * (float)i;
  }
  std::vector<uint4> ha(nv);
  for (size_t i = 0; i < nv; ++i) {
    const uint32_t v = (uint32_t)i;
    ha[i] = make_uint4(__builtin_bit_cast(uint32_t, 0.5f),
                       (v % 64u) | ((v / 64u % 64u) << 10) | ((v / 4096u) << 20),
                       ((v + 7u) % 64u) | ((v / 64u % 64u) << 10) | ((v / 4096u) << 20), 0u);
  }
  if ((s = ctx_hip(c, hipMemcpyAsync(rec.p, hr.data(), nv * 2, hipMemcpyHostToDevice, st), "copy")) ||
      (s = ctx_hip(c, hipMemcpyAsync(pal.p, hp, sizeof hp, hipMemcpyHostToDevice, st), "copy")) ||
      (s = ctx_hip(c, hipMemcpyAsync(kn.p, hk.data(), kNGrid * 4, hipMemcpyHostToDevice, st), "copy")) ||
      (s = ctx_hip(c, hipMemcpyAsync(maj.p, hm.data(), kNGrid * 4, hipMemcpyHostToDevice, st), "copy")) ||
      (s = ctx_hip(c, hipMemcpyAsync(alias.p, ha.data(), nv * sizeof(uint4), hipMemcpyHostToDevice, st), "copy")) ||
      (s = ctx_hip(c, launch_zero_bytes(tally.p, nv * 16, st), "zero")))
    return s;
  UnitArgs A;
  A.rec = (const uint16_t *)rec.p;
  A.pal = (const float4 *)pal.p;
  A.ln2_kn = (const float *)kn.p;
  A.ln2_maj = (const float *)maj.p;
  A.alias = (const uint4 *)alias.p;
  A.tally = (double *)tally.p;
  // the transport's energy grid: 1 keV .. 511 keV in 255 log steps
  A.l2emin = -9.965784f;
  A.inv_dl2 = 255.0f / 8.997179f;
  A.k0 = 0x12345678u;
  A.k1 = 0x9abcdef0u;
  A.iters = iters;
  A.out = (uint32_t *)sink.p;
  typedef void (*Fn)(UnitArgs);
  static const Fn fns[NMD_UNIT_N] = {unit_kernel<0>, unit_kernel<1>, unit_kernel<2>,
                                     unit_kernel<3>, unit_kernel<4>, unit_kernel<5>,
                                     unit_kernel<6>, unit_kernel<7>};
  Timer t;
  if ((s = ctx_hip(c, hipEventCreate(&t.a), "hipEventCreate"))) return s;
  if ((s = ctx_hip(c, hipEventCreate(&t.b), "hipEventCreate"))) return s;
  if ((s = ctx_hip(c, hipEventRecord(t.a, st), "hipEventRecord"))) return s;
  hipLaunchKernelGGL(fns[kind], dim3(blocks), dim3(256), 0, st, A);
  if ((s = ctx_hip(c, hipGetLastError(), "unit_kernel"))) return s;
  if ((s = ctx_hip(c, hipEventRecord(t.b, st), "hipEventRecord"))) return s;
  if ((s = ctx_hip(c, hipEventSynchronize(t.b), "hipEventSynchronize"))) return s;
  float el = 0.0f;
  if ((s = ctx_hip(c, hipEventElapsedTime(&el, t.a, t.b), "hipEventElapsedTime"))) return s;
  if (ms) *ms = el;
  return NMD_OK;
}

nmd_status nmd_probe_lds(nmd_ctx *c, int32_t pattern, int32_t write, uint32_t iters,
                         uint32_t blocks, double *ms) {
  nmd_status s = ctx_enter(c);
  if (s) return s;
  if (pattern < 0 || pattern >= NMD_LDS_N) return ctx_fail(c, NMD_E_INVALID, "unknown LDS pattern");
  if (iters == 0 || iters > (1u << 16) || blocks == 0 || blocks > 65536)
    return ctx_fail(c, NMD_E_INVALID, "iters in 1..2^16 and blocks in 1..65536 required");
  // every lane's quads (the pattern's offset plus up to 3 x 4 KiB) stay in
  // the 32 KiB array
  for (int L = 0; L < 64; ++L)
    if (lds_offset(pattern, L) % 16 || lds_offset(pattern, L) / 16 + (3u << 8) >= (uint32_t)kLdsQuads)
      return ctx_fail(c, NMD_E_INVALID, "LDS pattern %d out of range", pattern);
  hipStream_t st = ctx_stream(c);
  Buf sink;
  if ((s = alloc(c, sink, 256))) return s;
  Timer t;
  if ((s = ctx_hip(c, hipEventCreate(&t.a), "hipEventCreate"))) return s;
  if ((s = ctx_hip(c, hipEventCreate(&t.b), "hipEventCreate"))) return s;
  if ((s = ctx_hip(c, hipEventRecord(t.a, st), "hipEventRecord"))) return s;
  if (write)
    hipLaunchKernelGGL(lds_write_kernel, dim3(blocks), dim3(256), 0, st, pattern, iters,
                       (uint32_t *)sink.p);
  else
    hipLaunchKernelGGL(lds_read_kernel, dim3(blocks), dim3(256), 0, st, pattern, iters,
                       (uint32_t *)sink.p);
  if ((s = ctx_hip(c, hipGetLastError(), "lds probe"))) return s;
  if ((s = ctx_hip(c, hipEventRecord(t.b, st), "hipEventRecord"))) return s;
  if ((s = ctx_hip(c, hipEventSynchronize(t.b), "hipEventSynchronize"))) return s;
  float el = 0.0f;
  if ((s = ctx_hip(c, hipEventElapsedTime(&el, t.a, t.b), "hipEventElapsedTime"))) return s;
  if (ms) *ms = el;
  return NMD_OK;
}

}  // extern "C"
