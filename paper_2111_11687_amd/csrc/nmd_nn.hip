// Kernels and entry points of the learned denoiser (include/nmdose_nn.h).
//
// The convolutions are implicit GEMMs on the gfx950 matrix cores
// (v_mfma_f32_16x16x32_bf16: a 16x32 BF16 tile times a 32x16 BF16 tile into
// 16x16 FP32).  Operand layout of that instruction, per lane l of the wave:
//   A: row l%16, K elements 8*(l/16) .. 8*(l/16)+7
//   B: column l%16, the same K elements
//   D: column l%16, rows 4*(l/16) .. 4*(l/16)+3
//
//   conv_kernel     forward and backward-data: rows = 16 voxels along x,
//                   columns = 16 output channels, K = (tap, input channel).
//                   A comes from a bf16 halo tile staged in LDS (channels
//                   innermost), B straight from the weight array (L1/L2).
//   wgrad_kernel    backward-weight: rows = output channels, columns =
//                   (tap, input channel), K = voxels.  Both operands need 8
//                   voxels per lane, so the tiles are staged channel-major
//                   and the x shift of a tap is an in-register funnel shift.
//   the rest        pooling, backward combination, input preparation,
//                   head and loss, Adam: HBM-bound element-wise kernels.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <algorithm>
#include <cmath>
#include <cstdio>

#include "../../include/nmdose.h"
#include "../../include/nmdose_nn.h"
#include "nmd_internal.hpp"

using namespace nmd;

namespace {

typedef __bf16 bf16x8_t __attribute__((ext_vector_type(8)));
typedef float f32x4_t __attribute__((ext_vector_type(4)));
typedef unsigned int u32x4_t __attribute__((ext_vector_type(4)));

__device__ __forceinline__ float bf2f(uint32_t h) { return __uint_as_float(h << 16); }

// Round to nearest even (NaN stays a quiet NaN).
__device__ __forceinline__ uint32_t f2bf(float f) {
  uint32_t u = __float_as_uint(f);
  if ((u & 0x7fffffffu) > 0x7f800000u) return (u >> 16) | 0x40u;
  u += 0x7fffu + ((u >> 16) & 1u);
  return u >> 16;
}

__device__ __forceinline__ f32x4_t mfma_bf16(u32x4_t a, u32x4_t b, f32x4_t c) {
  return __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16x8_t, a),
                                                 __builtin_bit_cast(bf16x8_t, b), c, 0, 0, 0);
}

// Element j (0..7) of 8 packed bfloat16 values, as float.
__device__ __forceinline__ float unpack(const u32x4_t &v, int j) {
  const uint32_t w = (j >> 1) == 0 ? v.x : (j >> 1) == 1 ? v.y : (j >> 1) == 2 ? v.z : v.w;
  return __uint_as_float((j & 1) ? (w & 0xffff0000u) : (w << 16));
}

__device__ __forceinline__ uint32_t pack2(float lo, float hi) {
  return f2bf(lo) | (f2bf(hi) << 16);
}

struct Src {
  const uint16_t *x0;
  const uint16_t *x1;
  int32_t c0, up0, c1;
};

// ---------------------------------------------------------------------------
// Forward / backward-data convolution
// ---------------------------------------------------------------------------
// Output tile: 16 x 8 voxels in x and y, TZ planes in z (2, or 4 for the
// kernel with one column block of 16-channel chunks), one voxel of halo.
constexpr int TX = 16, TY = 8;
constexpr int HX = TX + 2, HY = TY + 2;
template <int TZ>
constexpr int halo_vox() { return HX * HY * (TZ + 2); }  // 720 or 1080 voxels
__host__ __device__ constexpr int conv_tz_of(int cc, int ncb) { return ncb == 1 && cc == 16 ? 4 : 2; }
template <int CC, int NCB>
constexpr int conv_tz() { return conv_tz_of(CC, NCB); }

// LDS voxel pitch (elements).  On gfx950 the LDS has 64 four-byte banks,
// and a ds_read_b128 serves 16 lanes per cycle: lanes 0-7 with 24-31, 8-15
// with 16-23 (and the same in the upper half-wave), so the fragment reads
// of lane groups g and g + 1 (the next 8 channels, or the next tap) meet in
// one cycle; a ds_write_b128 serves 16 consecutive lanes (bank-conflict
// counters over probe patterns).  Unpadded 16-channel voxels (32 bytes) put
// the two groups on the even and odd 16-byte bank quads, and their halo
// stores are contiguous; 32-channel voxels take a 96-byte pitch, for the
// same split of the reads.
__host__ __device__ constexpr int halo_pitch(int cc) { return cc == 32 ? 48 : cc; }

struct ConvArgs {
  Src src;
  const uint16_t *w;     // [cout][27][cin]
  const float *bias;     // [cout] or null
  const uint16_t *mask;  // [vox][cout] or null
  uint16_t *y;           // [vox][cout]
  int32_t d, h, w_, cin, cout, relu;
  int32_t tiles_x, tiles_y, tiles_z, n_tiles;  // per volume
};

// Tile index with the workgroups of one XCD (dispatched round robin over the
// 8 XCDs) taking a contiguous range of tiles, so that neighbouring halos
// meet in the same L2.
__device__ __forceinline__ int xcd_tile(int b, int n) {
  if ((n & 7) != 0) return b;
  return (b & 7) * (n >> 3) + (b >> 3);
}

template <int CC, int TZ>
__device__ __forceinline__ void stage_halo(uint16_t *s, const Src &src, int cbase, int nb, int D,
                                           int H, int W, int z0, int y0, int x0) {
  constexpr int NC8 = CC / 8;
  constexpr int P = halo_pitch(CC);
  const bool first = cbase < src.c0;
  const uint16_t *base = first ? src.x0 : src.x1;
  const int cs = first ? src.c0 : src.c1;
  const int coff = first ? cbase : cbase - src.c0;
  const bool up = first && src.up0;
  const int Ds = up ? (D + 1) >> 1 : D, Hs = up ? (H + 1) >> 1 : H, Ws = up ? (W + 1) >> 1 : W;
  for (int u = threadIdx.x; u < halo_vox<TZ>() * NC8; u += 256) {
    const int hv = u / NC8, c8 = u - hv * NC8;
    const int hz = hv / (HY * HX), r = hv - hz * (HY * HX), hy = r / HX, hx = r - hy * HX;
    int z = z0 - 1 + hz, y = y0 - 1 + hy, x = x0 - 1 + hx;
    u32x4_t val = {0u, 0u, 0u, 0u};
    if (z >= 0 && z < D && y >= 0 && y < H && x >= 0 && x < W) {
      if (up) {
        z >>= 1;
        y >>= 1;
        x >>= 1;
      }
      const size_t vox = (((size_t)nb * Ds + z) * Hs + y) * Ws + x;
      val = *reinterpret_cast<const u32x4_t *>(base + vox * cs + coff + c8 * 8);
    }
    *reinterpret_cast<u32x4_t *>(s + hv * P + c8 * 8) = val;
  }
}

// The same staging split in two: this thread's share of the halo chunk into
// registers (its global loads can then be in flight while the workgroup
// computes on the chunk before), and from registers into LDS.
template <int CC, int TZ>
constexpr int halo_regs() { return (halo_vox<TZ>() * (CC / 8) + 255) / 256; }

template <int CC, int TZ>
__device__ __forceinline__ void load_halo(u32x4_t (&rg)[(halo_regs<CC, TZ>())], const Src &src, int cbase,
                                          int nb, int D, int H, int W, int z0, int y0, int x0) {
  constexpr int NC8 = CC / 8;
  const bool first = cbase < src.c0;
  const uint16_t *base = first ? src.x0 : src.x1;
  const int cs = first ? src.c0 : src.c1;
  const int coff = first ? cbase : cbase - src.c0;
  const bool up = first && src.up0;
  const int Ds = up ? (D + 1) >> 1 : D, Hs = up ? (H + 1) >> 1 : H, Ws = up ? (W + 1) >> 1 : W;
#pragma unroll
  for (int i = 0; i < halo_regs<CC, TZ>(); ++i) {
    const int u = threadIdx.x + 256 * i;
    const int hv = u / NC8, c8 = u - hv * NC8;
    const int hz = hv / (HY * HX), r = hv - hz * (HY * HX), hy = r / HX, hx = r - hy * HX;
    int z = z0 - 1 + hz, y = y0 - 1 + hy, x = x0 - 1 + hx;
    u32x4_t val = {0u, 0u, 0u, 0u};
    if (u < halo_vox<TZ>() * NC8 && z >= 0 && z < D && y >= 0 && y < H && x >= 0 && x < W) {
      if (up) {
        z >>= 1;
        y >>= 1;
        x >>= 1;
      }
      const size_t vox = (((size_t)nb * Ds + z) * Hs + y) * Ws + x;
      val = *reinterpret_cast<const u32x4_t *>(base + vox * cs + coff + c8 * 8);
    }
    rg[i] = val;
  }
}

template <int CC, int TZ>
__device__ __forceinline__ void store_halo(uint16_t *s, const u32x4_t (&rg)[(halo_regs<CC, TZ>())]) {
  constexpr int NC8 = CC / 8;
  constexpr int P = halo_pitch(CC);
#pragma unroll
  for (int i = 0; i < halo_regs<CC, TZ>(); ++i) {
    const int u = threadIdx.x + 256 * i;
    if (u < halo_vox<TZ>() * NC8) {
      const int hv = u / NC8, c8 = u - hv * NC8;
      *reinterpret_cast<u32x4_t *>(s + hv * P + c8 * 8) = rg[i];
    }
  }
}

template <int CC, int NCB>
// one column block of 16-channel chunks: a 4-plane tile (34.6 KB of halo;
// three workgroups per CU, by registers); with 32-channel chunks the
// 2-plane halo's 69 KB of LDS allows two
__global__ __launch_bounds__(256, NCB == 1 ? (CC == 16 ? 3 : (CC == 32 ? 2 : 1)) : 1) void conv_kernel(
    ConvArgs a) {
  constexpr int NC8 = CC / 8;
  constexpr int P = halo_pitch(CC);
  constexpr int NP = 27 * NC8;          // (tap, 8-channel group) pairs per chunk
  constexpr int NS = (NP + 3) / 4;      // K steps of 32
  constexpr int TZ = conv_tz<CC, NCB>();
  constexpr int RW = TZ * TY / 4;       // output rows (z, y) per wave: 4 or 8
  __shared__ __align__(16) uint16_t s_x[halo_vox<TZ>() * P];
  // the row-shared K loop: one column block, or several of 16-channel chunks
  constexpr bool kRowShared = CC >= 16 && (NCB == 1 || CC == 16);
  static_assert(RW == 4 || kRowShared, "wide rows only in the row-shared loop");

  const int nb = blockIdx.y;
  const int t = xcd_tile(blockIdx.x, a.n_tiles);
  const int tx = t % a.tiles_x, r0 = t / a.tiles_x, ty = r0 % a.tiles_y, tz = r0 / a.tiles_y;
  const int x0 = tx * TX, y0 = ty * TY, z0 = tz * TZ;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int lx = lane & 15, g = lane >> 4;

  int rowoff[4];
#pragma unroll
  for (int rb = 0; rb < 4; ++rb) {
    const int r = wave * 4 + rb;
    rowoff[rb] = (((r / TY) * HY + (r % TY)) * HX + lx) * P;
  }
  f32x4_t acc[RW][NCB];
#pragma unroll
  for (int rb = 0; rb < RW; ++rb)
#pragma unroll
    for (int cb = 0; cb < NCB; ++cb) acc[rb][cb] = f32x4_t{0.f, 0.f, 0.f, 0.f};

  const int nchunks = a.cin / CC;
  // the row-shared path holds the next chunk's halo in registers while it
  // computes on this one
  constexpr bool kPrefetch = NCB == 1 && CC >= 16;
  u32x4_t pre[kPrefetch ? halo_regs<CC, TZ>() : 1];
  if constexpr (kPrefetch) load_halo<CC, TZ>(pre, a.src, 0, nb, a.d, a.h, a.w_, z0, y0, x0);
  for (int ch = 0; ch < nchunks; ++ch) {
    if (ch) __syncthreads();
    if constexpr (kPrefetch) {
      store_halo<CC, TZ>(s_x, pre);
      if (ch + 1 < nchunks)
        load_halo<CC, TZ>(pre, a.src, (ch + 1) * CC, nb, a.d, a.h, a.w_, z0, y0, x0);
    } else {
      stage_halo<CC, TZ>(s_x, a.src, ch * CC, nb, a.d, a.h, a.w_, z0, y0, x0);
    }
    __syncthreads();
    const uint16_t *wrow = a.w + (size_t)lx * 27 * a.cin + ch * CC;
    const size_t wcb = (size_t)16 * 27 * a.cin;  // one column block of weights
    // fragments of K step s: A from the LDS halo, B from the weight array
    auto load_step = [&](int s, u32x4_t (&av)[4], u32x4_t (&b)[NCB]) {
      const int p = 4 * s + g;
      const bool valid = p < NP;
      const int pp = valid ? p : 0;
      const int tap = pp / NC8, c8 = pp - tap * NC8;
      const int kz = tap / 9, ky = (tap / 3) % 3, kx = tap % 3;
      const int aoff = ((kz * HY + ky) * HX + kx) * P + c8 * 8;
      const int woff = tap * a.cin + c8 * 8;
#pragma unroll
      for (int cb = 0; cb < NCB; ++cb) {
        b[cb] = *reinterpret_cast<const u32x4_t *>(wrow + cb * wcb + woff);
        if (!valid) b[cb] = u32x4_t{0u, 0u, 0u, 0u};
      }
#pragma unroll
      for (int rb = 0; rb < 4; ++rb)
        av[rb] = *reinterpret_cast<const u32x4_t *>(s_x + rowoff[rb] + aoff);
    };
    if constexpr (kRowShared) {
      // K runs over (kz, kx, c8) with the three ky taps inside: the wave's
      // RW rows (one z, RW consecutive y) and 3 ky shifts touch RW + 2 halo
      // rows, so RW + 2 A fragments and 3 NCB B fragments feed 3 RW NCB
      // MFMAs (24 for a whole plane and one column block, 36 for four rows
      // and three).  With one column block no A fragment would otherwise
      // serve two MFMAs.
      constexpr int NQ = 9 * NC8;          // (kz, kx, 8-channel group) triples
      constexpr int NSQ = (NQ + 3) / 4;    // K steps of 32
      const int r0w = wave * RW;           // the wave's first row
      const int zr = r0w / TY, yb = r0w % TY;
#pragma unroll 1
      for (int sq = 0; sq < NSQ; ++sq) {
        const int q = 4 * sq + g;
        const bool valid = q < NQ;
        const int qq = valid ? q : 0;
        const int kzx = qq / NC8, c8 = qq - kzx * NC8;
        const int kz = kzx / 3, kx = kzx - 3 * kz;
        u32x4_t av[RW + 2], b[3][NCB];
#pragma unroll
        for (int ky = 0; ky < 3; ++ky) {
          const int tap = (kz * 3 + ky) * 3 + kx;
#pragma unroll
          for (int cb = 0; cb < NCB; ++cb) {
            b[ky][cb] = *reinterpret_cast<const u32x4_t *>(wrow + cb * wcb + tap * a.cin + c8 * 8);
            if (!valid) b[ky][cb] = u32x4_t{0u, 0u, 0u, 0u};
          }
        }
        const int abase = (((zr + kz) * HY + yb) * HX + lx + kx) * P + c8 * 8;
#pragma unroll
        for (int j = 0; j < RW + 2; ++j)
          av[j] = *reinterpret_cast<const u32x4_t *>(s_x + abase + j * HX * P);
#pragma unroll
        for (int ky = 0; ky < 3; ++ky)
#pragma unroll
          for (int rb = 0; rb < RW; ++rb)
#pragma unroll
            for (int cb = 0; cb < NCB; ++cb)
              acc[rb][cb] = mfma_bf16(av[rb + ky], b[ky][cb], acc[rb][cb]);
      }
      continue;
    }
    // software pipeline: step s + 1's fragments load during step s's MFMAs
    u32x4_t av[4], b[NCB], avn[4], bn[NCB];
    load_step(0, av, b);
    __builtin_amdgcn_sched_group_barrier(0x100, 4, 0);    // step 0: DS reads
    __builtin_amdgcn_sched_group_barrier(0x020, NCB, 0);  // step 0: VMEM reads
#pragma unroll
    for (int s = 0; s < NS; ++s) {
      if (s + 1 < NS) load_step(s + 1, avn, bn);
#pragma unroll
      for (int rb = 0; rb < 4; ++rb)
#pragma unroll
        for (int cb = 0; cb < NCB; ++cb) acc[rb][cb] = mfma_bf16(av[rb], b[cb], acc[rb][cb]);
      // keep that order: the next step's LDS and global reads go out before
      // this step's MFMAs, so their latency hides behind them
      if (s + 1 < NS) {
        __builtin_amdgcn_sched_group_barrier(0x100, 4, 0);    // DS reads
        __builtin_amdgcn_sched_group_barrier(0x020, NCB, 0);  // VMEM reads
      }
      __builtin_amdgcn_sched_group_barrier(0x008, 4 * NCB, 0);  // MFMA
      if (s + 1 < NS) {
#pragma unroll
        for (int rb = 0; rb < 4; ++rb) av[rb] = avn[rb];
#pragma unroll
        for (int cb = 0; cb < NCB; ++cb) b[cb] = bn[cb];
      }
    }
  }

  // epilogue: bias, ReLU, mask, round to bf16
#pragma unroll
  for (int rb = 0; rb < RW; ++rb) {
    const int r = wave * RW + rb;
    const int z = z0 + r / TY, y = y0 + r % TY;
    if (z >= a.d || y >= a.h) continue;
    const size_t rowvox = (((size_t)nb * a.d + z) * a.h + y) * a.w_;
#pragma unroll
    for (int cb = 0; cb < NCB; ++cb) {
      const int co = cb * 16 + lx;
      const float bv = a.bias ? a.bias[co] : 0.f;
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int x = x0 + 4 * g + i;
        if (x >= a.w_) continue;
        const size_t e = (rowvox + x) * a.cout + co;
        float v = acc[rb][cb][i] + bv;
        if (a.relu) v = fmaxf(v, 0.f);
        if (a.mask && !(bf2f(a.mask[e]) > 0.f)) v = 0.f;
        a.y[e] = (uint16_t)f2bf(v);
      }
    }
  }
}

// ---------------------------------------------------------------------------
// Backward-weight convolution
// ---------------------------------------------------------------------------
constexpr int WTX = 16, WTY = 4, WTZ = 2;                  // voxel tile (128)
constexpr int WHX = WTX + 2, WHY = WTY + 2, WHZ = WTZ + 2;  // halo
constexpr int WHV = WHX * WHY * WHZ;                       // 432
constexpr int WXP = 24;                                    // halo row pitch
// Channel pitches of 2 mod 4 sixteen-byte quads: lane groups g and g + 1,
// which a ds_read_b128 serves in one cycle (lanes 0-7 with 24-31, 8-15
// with 16-23), then fall on the even and the odd bank quads.
constexpr int WCP = WHZ * WHY * WXP + 16;                  // halo channel pitch (592)
constexpr int WDP = WTX * WTY * WTZ + 16;                  // dy channel pitch (144)
static_assert((WCP / 8) % 4 == 2 && (WDP / 8) % 4 == 2, "conflict-free channel pitches");

struct WgradArgs {
  Src src;
  const uint16_t *dy;  // [vox][cout]
  float *part;         // [n_vg][cout][27*cin]
  int32_t n, d, h, w_, cin, cout;
  int32_t tiles_x, tiles_y, tiles_z, n_tiles;  // n_tiles over all volumes
  int32_t n_vg, ncg;                           // voxel groups; column groups per chunk
};

// Element pair j of two packed bf16 vectors as one dword: (lo[j], hi[j]).
__device__ __forceinline__ uint32_t pair_of(const u32x4_t &lo, const u32x4_t &hi, int j) {
  const uint32_t wl = (j >> 1) == 0 ? lo.x : (j >> 1) == 1 ? lo.y : (j >> 1) == 2 ? lo.z : lo.w;
  const uint32_t wh = (j >> 1) == 0 ? hi.x : (j >> 1) == 1 ? hi.y : (j >> 1) == 2 ? hi.z : hi.w;
  return (j & 1) ? ((wl >> 16) | (wh & 0xffff0000u)) : ((wl & 0xffffu) | (wh << 16));
}

template <int CC, int NCBO, int NBW>
__global__ __launch_bounds__(256) void wgrad_kernel(WgradArgs a) {
  constexpr int NB = (27 * CC + 15) / 16;  // column blocks per chunk
  constexpr int NC8 = CC / 8;
  constexpr int COUT = NCBO * 16;
  // staging items: two x-neighbouring voxels x 8 channels, voxel pairs fastest
  constexpr int XPAIRS = WHV / 2;                     // 216 (halo rows are 18 voxels)
  constexpr int NXI = XPAIRS * NC8;
  constexpr int NXL = (NXI + 255) / 256;
  constexpr int DPAIRS = WTX * WTY * WTZ / 2;         // 64
  constexpr int NDI = DPAIRS * (COUT / 8);
  constexpr int NDL = (NDI + 255) / 256;
  // channel CC of s_x stays zero: padding columns of the last column block
  // read it, so their B fragments are zero without a per-lane mask
  __shared__ __align__(16) uint16_t s_x[(CC + 1) * WCP];
  __shared__ __align__(16) uint16_t s_dp[COUT * WDP];

  const int vg = blockIdx.x;
  const int chunk = blockIdx.y / a.ncg, cg = blockIdx.y - chunk * a.ncg;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int lx = lane & 15, g = lane >> 4;
  const int cbase = chunk * CC;
  const int tpv = a.tiles_x * a.tiles_y * a.tiles_z;

  const bool first = cbase < a.src.c0;
  const uint16_t *xbase = first ? a.src.x0 : a.src.x1;
  const int xcs = first ? a.src.c0 : a.src.c1;
  const int xcoff = first ? cbase : cbase - a.src.c0;
  const bool up = first && a.src.up0;
  const int Ds = up ? (a.d + 1) >> 1 : a.d, Hs = up ? (a.h + 1) >> 1 : a.h,
            Ws = up ? (a.w_ + 1) >> 1 : a.w_;

  f32x4_t acc[NCBO][NBW];
#pragma unroll
  for (int i = 0; i < NCBO; ++i)
#pragma unroll
    for (int j = 0; j < NBW; ++j) acc[i][j] = f32x4_t{0.f, 0.f, 0.f, 0.f};

  for (int i = threadIdx.x; i < WCP; i += 256) s_x[CC * WCP + i] = 0;

  // this lane's column of each of the wave's column blocks: LDS offset of
  // (channel, tap row), and the byte selector of v_perm_b32 that shifts the
  // 10 loaded elements by the tap's x offset (0, 1 or 2 elements)
  int coloff[NBW];
  uint32_t colsel[NBW];
#pragma unroll
  for (int j = 0; j < NBW; ++j) {
    const int nbk = (cg * 4 + wave) * NBW + j;
    const int q = nbk * 16 + lx;
    const int tap = q / CC, ci = q - tap * CC;
    const bool ok = nbk < NB && tap < 27;
    const int tp = ok ? tap : 0;
    coloff[j] = (ok ? ci : CC) * WCP + ((tp / 9) * WHY + (tp / 3) % 3) * WXP;
    colsel[j] = 0x03020100u + (uint32_t)(tp % 3) * 0x02020202u;
  }

  // registers holding the next tile while the current one is computed
  u32x4_t px[NXL][2], pd[NDL][2];
  auto load = [&](int t) {
    const int nb = t / tpv, tl = t - nb * tpv;
    const int tx = tl % a.tiles_x, r0 = tl / a.tiles_x, ty = r0 % a.tiles_y, tz = r0 / a.tiles_y;
    const int x0 = tx * WTX, y0 = ty * WTY, z0 = tz * WTZ;
#pragma unroll
    for (int i = 0; i < NXL; ++i) {
      const int u = threadIdx.x + 256 * i;
      px[i][0] = px[i][1] = u32x4_t{0u, 0u, 0u, 0u};
      if (u < NXI) {
        const int c8 = u / XPAIRS, pr = u - c8 * XPAIRS;
        const int hx = 2 * (pr % (WHX / 2)), hy = (pr / (WHX / 2)) % WHY,
                  hz = pr / ((WHX / 2) * WHY);
        int z = z0 - 1 + hz, y = y0 - 1 + hy;
        if (z >= 0 && z < a.d && y >= 0 && y < a.h) {
          if (up) {
            z >>= 1;
            y >>= 1;
          }
#pragma unroll
          for (int e = 0; e < 2; ++e) {
            int x = x0 - 1 + hx + e;
            if (x >= 0 && x < a.w_) {
              if (up) x >>= 1;
              const size_t vox = (((size_t)nb * Ds + z) * Hs + y) * Ws + x;
              px[i][e] = *reinterpret_cast<const u32x4_t *>(xbase + vox * xcs + xcoff + c8 * 8);
            }
          }
        }
      }
    }
#pragma unroll
    for (int i = 0; i < NDL; ++i) {
      const int u = threadIdx.x + 256 * i;
      pd[i][0] = pd[i][1] = u32x4_t{0u, 0u, 0u, 0u};
      if (u < NDI) {
        const int c8 = u / DPAIRS, pr = u - c8 * DPAIRS;
        const int xx = 2 * (pr % (WTX / 2)), yy = (pr / (WTX / 2)) % WTY, zz = pr / ((WTX / 2) * WTY);
        const int y = y0 + yy, z = z0 + zz;
        if (y < a.h && z < a.d) {
#pragma unroll
          for (int e = 0; e < 2; ++e) {
            const int x = x0 + xx + e;
            if (x < a.w_)
              pd[i][e] = *reinterpret_cast<const u32x4_t *>(
                  a.dy + ((((size_t)nb * a.d + z) * a.h + y) * a.w_ + x) * COUT + c8 * 8);
          }
        }
      }
    }
  };
  auto store = [&]() {
#pragma unroll
    for (int i = 0; i < NXL; ++i) {
      const int u = threadIdx.x + 256 * i;
      if (u < NXI) {
        const int c8 = u / XPAIRS, pr = u - c8 * XPAIRS;
        const int hx = 2 * (pr % (WHX / 2)), hy = (pr / (WHX / 2)) % WHY,
                  hz = pr / ((WHX / 2) * WHY);
        const int o = (hz * WHY + hy) * WXP + hx;
#pragma unroll
        for (int j = 0; j < 8; ++j)
          *reinterpret_cast<uint32_t *>(s_x + (c8 * 8 + j) * WCP + o) = pair_of(px[i][0], px[i][1], j);
      }
    }
#pragma unroll
    for (int i = 0; i < NDL; ++i) {
      const int u = threadIdx.x + 256 * i;
      if (u < NDI) {
        const int c8 = u / DPAIRS, pr = u - c8 * DPAIRS;
#pragma unroll
        for (int j = 0; j < 8; ++j)
          *reinterpret_cast<uint32_t *>(s_dp + (c8 * 8 + j) * WDP + 2 * pr) =
              pair_of(pd[i][0], pd[i][1], j);
      }
    }
  };

  // a contiguous run of tiles (x fastest): neighbouring halos meet in L2
  const int t_begin = (int)(((int64_t)a.n_tiles * vg) / a.n_vg);
  const int t_end = (int)(((int64_t)a.n_tiles * (vg + 1)) / a.n_vg);
  if (t_begin < t_end) load(t_begin);
  for (int t = t_begin; t < t_end; ++t) {
    __syncthreads();  // the previous tile's reads of LDS are done
    store();
    __syncthreads();
    if (t + 1 < t_end) load(t + 1);  // in flight during the MFMAs
    // 4 K steps of 32 voxels; group g takes 8 voxels of tile row 2s + g/2
#pragma unroll
    for (int s = 0; s < 4; ++s) {
      const int row = 2 * s + (g >> 1), xo = 8 * (g & 1);
      const int rz = row / WTY, ry = row % WTY;
      u32x4_t av[NCBO];
#pragma unroll
      for (int i = 0; i < NCBO; ++i)
        av[i] = *reinterpret_cast<const u32x4_t *>(s_dp + (i * 16 + lx) * WDP + row * WTX + xo);
      const int rowo = (rz * WHY + ry) * WXP + xo;
#pragma unroll
      for (int j = 0; j < NBW; ++j) {
        const uint16_t *pb = s_x + coloff[j] + rowo;
        const u32x4_t lo = *reinterpret_cast<const u32x4_t *>(pb);
        const uint32_t hi = *reinterpret_cast<const uint32_t *>(pb + 8);
        // word k of the shifted fragment: bytes sel of the pair (d[k+1]:d[k])
        const u32x4_t bv = {__builtin_amdgcn_perm(lo.y, lo.x, colsel[j]),
                            __builtin_amdgcn_perm(lo.z, lo.y, colsel[j]),
                            __builtin_amdgcn_perm(lo.w, lo.z, colsel[j]),
                            __builtin_amdgcn_perm(hi, lo.w, colsel[j])};
#pragma unroll
        for (int i = 0; i < NCBO; ++i) acc[i][j] = mfma_bf16(av[i], bv, acc[i][j]);
      }
    }
  }

  // partial of this voxel group
  const size_t ke = (size_t)27 * a.cin;
  float *out = a.part + (size_t)vg * COUT * ke;
#pragma unroll
  for (int j = 0; j < NBW; ++j) {
    const int nbk = (cg * 4 + wave) * NBW + j;
    const int q = nbk * 16 + lx;
    const int tap = q / CC, ci = q - tap * CC;
    if (nbk >= NB || tap >= 27) continue;
    const size_t k = (size_t)tap * a.cin + cbase + ci;
#pragma unroll
    for (int i = 0; i < NCBO; ++i)
#pragma unroll
      for (int e = 0; e < 4; ++e) out[(size_t)(i * 16 + 4 * g + e) * ke + k] = acc[i][j][e];
  }
}

// out[e] = sum over p of part[p*n + e].  A block takes 64 consecutive
// elements; its 4 waves each sum every 4th partial in order (one coalesced
// 256-byte row per load), then the 4 wave sums are added in a fixed order:
// the result does not depend on the launch.
__global__ __launch_bounds__(256) void sum_parts_kernel(const float *__restrict__ part,
                                                        int64_t n, int n_part,
                                                        float *__restrict__ out) {
  __shared__ float s[4][64];
  const int el = threadIdx.x & 63, ln = threadIdx.x >> 6;
  for (int64_t e0 = (int64_t)blockIdx.x * 64; e0 < n; e0 += (int64_t)gridDim.x * 64) {
    const int64_t e = e0 + el;
    float acc = 0.f;
    if (e < n) {
#pragma unroll 8
      for (int p = ln; p < n_part; p += 4) acc += part[(size_t)p * n + e];
    }
    s[ln][el] = acc;
    __syncthreads();
    if (ln == 0 && e < n) out[e] = (s[0][el] + s[1][el]) + (s[2][el] + s[3][el]);
    __syncthreads();
  }
}

// Per-block channel sums of a [nvox][c] bf16 tensor (the bias gradient).
__global__ __launch_bounds__(256) void chan_sum_kernel(const uint16_t *__restrict__ x,
                                                       uint64_t nvox, int c,
                                                       float *__restrict__ part) {
  __shared__ float s[256][9];
  const int c8n = c / 8;
  const int per = 256 / c8n;  // voxels per block iteration
  const int c8 = threadIdx.x % c8n, vo = threadIdx.x / c8n;
  float acc[8] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
  if (vo < per) {
    for (uint64_t v = (uint64_t)blockIdx.x * per + vo; v < nvox; v += (uint64_t)gridDim.x * per) {
      const u32x4_t q = *reinterpret_cast<const u32x4_t *>(x + v * c + c8 * 8);
#pragma unroll
      for (int j = 0; j < 8; ++j) acc[j] += unpack(q, j);
    }
  }
#pragma unroll
  for (int j = 0; j < 8; ++j) s[threadIdx.x][j] = vo < per ? acc[j] : 0.f;
  __syncthreads();
  if (threadIdx.x < c) {
    const int cc8 = threadIdx.x / 8, j = threadIdx.x % 8;
    float t = 0.f;
    for (int i = cc8; i < 256; i += c8n) t += s[i][j];
    part[(size_t)blockIdx.x * c + threadIdx.x] = t;
  }
}

// ---------------------------------------------------------------------------
// Element-wise stages
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void pool_kernel(const uint16_t *__restrict__ x,
                                                   uint16_t *__restrict__ y, int n, int D, int H,
                                                   int W, int c) {
  const int Dc = D / 2, Hc = H / 2, Wc = W / 2, c8n = c / 8;
  const uint64_t total = (uint64_t)n * Dc * Hc * Wc * c8n;
  for (uint64_t u = (uint64_t)blockIdx.x * 256 + threadIdx.x; u < total;
       u += (uint64_t)gridDim.x * 256) {
    const int c8 = (int)(u % c8n);
    uint64_t v = u / c8n;
    const int xc = (int)(v % Wc);
    v /= Wc;
    const int yc = (int)(v % Hc);
    v /= Hc;
    const int zc = (int)(v % Dc);
    const int nb = (int)(v / Dc);
    float s[8] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int k = 0; k < 8; ++k) {
      const size_t fv = (((size_t)nb * D + 2 * zc + (k >> 2)) * H + 2 * yc + ((k >> 1) & 1)) * W +
                        2 * xc + (k & 1);
      const u32x4_t q = *reinterpret_cast<const u32x4_t *>(x + fv * c + c8 * 8);
#pragma unroll
      for (int j = 0; j < 8; ++j) s[j] += unpack(q, j);
    }
    const u32x4_t o = {pack2(s[0] * 0.125f, s[1] * 0.125f), pack2(s[2] * 0.125f, s[3] * 0.125f),
                       pack2(s[4] * 0.125f, s[5] * 0.125f), pack2(s[6] * 0.125f, s[7] * 0.125f)};
    *reinterpret_cast<u32x4_t *>(y + (u / c8n) * c + c8 * 8) = o;
  }
}

__global__ __launch_bounds__(256) void combine_kernel(int n, int D, int H, int W, int c,
                                                      const uint16_t *__restrict__ mask,
                                                      const uint16_t *__restrict__ a, int sa,
                                                      int oa, int mode,
                                                      const uint16_t *__restrict__ b, int sb,
                                                      int ob, uint16_t *__restrict__ out) {
  const int c8n = c / 8;
  const uint64_t total = (uint64_t)n * D * H * W * c8n;
  for (uint64_t u = (uint64_t)blockIdx.x * 256 + threadIdx.x; u < total;
       u += (uint64_t)gridDim.x * 256) {
    const int c8 = (int)(u % c8n);
    const uint64_t v = u / c8n;
    float s[8] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
    if (a) {
      const u32x4_t q = *reinterpret_cast<const u32x4_t *>(a + v * sa + oa + c8 * 8);
#pragma unroll
      for (int j = 0; j < 8; ++j) s[j] = unpack(q, j);
    }
    if (mode != 0) {
      uint64_t r = v;
      const int x = (int)(r % W);
      r /= W;
      const int y = (int)(r % H);
      r /= H;
      const int z = (int)(r % D);
      const int nb = (int)(r / D);
      if (mode == 1) {
        const int D2 = 2 * D, H2 = 2 * H, W2 = 2 * W;
        float t[8] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int k = 0; k < 8; ++k) {
          const size_t fv = (((size_t)nb * D2 + 2 * z + (k >> 2)) * H2 + 2 * y + ((k >> 1) & 1)) *
                                W2 + 2 * x + (k & 1);
          const u32x4_t q = *reinterpret_cast<const u32x4_t *>(b + fv * sb + ob + c8 * 8);
#pragma unroll
          for (int j = 0; j < 8; ++j) t[j] += unpack(q, j);
        }
#pragma unroll
        for (int j = 0; j < 8; ++j) s[j] += t[j];
      } else {
        const size_t cv = (((size_t)nb * (D / 2) + z / 2) * (H / 2) + y / 2) * (W / 2) + x / 2;
        const u32x4_t q = *reinterpret_cast<const u32x4_t *>(b + cv * sb + ob + c8 * 8);
#pragma unroll
        for (int j = 0; j < 8; ++j) s[j] += unpack(q, j) * 0.125f;
      }
    }
    if (mask) {
      const u32x4_t q = *reinterpret_cast<const u32x4_t *>(mask + v * c + c8 * 8);
#pragma unroll
      for (int j = 0; j < 8; ++j)
        if (!(unpack(q, j) > 0.f)) s[j] = 0.f;
    }
    const u32x4_t o = {pack2(s[0], s[1]), pack2(s[2], s[3]), pack2(s[4], s[5]),
                       pack2(s[6], s[7])};
    *reinterpret_cast<u32x4_t *>(out + v * c + c8 * 8) = o;
  }
}

struct Box {
  int32_t z0, y0, x0, d, h, w;
};

// Body sums over a box: per block (dose, activity, count).
__global__ __launch_bounds__(256) void body_stats_kernel(int ny, int nx, Box bx,
                                                         const double *__restrict__ dose,
                                                         const float *__restrict__ act,
                                                         const uint8_t *__restrict__ label,
                                                         double *__restrict__ part) {
  __shared__ double s[3][256];
  const uint64_t total = (uint64_t)bx.d * bx.h * bx.w;
  double sd = 0.0, sa = 0.0, sc = 0.0;
  for (uint64_t u = (uint64_t)blockIdx.x * 256 + threadIdx.x; u < total;
       u += (uint64_t)gridDim.x * 256) {
    const int x = (int)(u % bx.w), y = (int)((u / bx.w) % bx.h), z = (int)(u / ((uint64_t)bx.w * bx.h));
    const size_t v = ((size_t)(bx.z0 + z) * ny + (bx.y0 + y)) * nx + (bx.x0 + x);
    if (label[v] > 0) {
      sd += dose[v];
      sa += (double)act[v];
      sc += 1.0;
    }
  }
  s[0][threadIdx.x] = sd;
  s[1][threadIdx.x] = sa;
  s[2][threadIdx.x] = sc;
  __syncthreads();
  for (int k = 128; k > 0; k >>= 1) {
    if ((int)threadIdx.x < k)
      for (int q = 0; q < 3; ++q) s[q][threadIdx.x] += s[q][threadIdx.x + k];
    __syncthreads();
  }
  if (threadIdx.x < 3) part[blockIdx.x * 3 + threadIdx.x] = s[threadIdx.x][0];
}

__global__ __launch_bounds__(256) void body_scale_kernel(const double *__restrict__ part,
                                                         int n_part,
                                                         double *__restrict__ scale) {
  __shared__ double s[3][256];
  double a[3] = {0.0, 0.0, 0.0};
  for (int p = threadIdx.x; p < n_part; p += 256)
    for (int q = 0; q < 3; ++q) a[q] += part[3 * p + q];
  for (int q = 0; q < 3; ++q) s[q][threadIdx.x] = a[q];
  __syncthreads();
  for (int k = 128; k > 0; k >>= 1) {
    if ((int)threadIdx.x < k)
      for (int q = 0; q < 3; ++q) s[q][threadIdx.x] += s[q][threadIdx.x + k];
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    const double sd = s[0][0], sa = s[1][0], sc = s[2][0];
    const double md = sc > 0 ? sd / sc : 0.0, ma = sc > 0 ? sa / sc : 0.0;
    scale[0] = md > 0 ? md : 1.0;
    scale[1] = ma > 0 ? ma : 1.0;
  }
}

__global__ __launch_bounds__(256) void prepare_kernel(int ny, int nx, Box bx,
                                                      const double *__restrict__ dose_lo,
                                                      const double *__restrict__ dose_hi,
                                                      const float *__restrict__ rho,
                                                      const float *__restrict__ act,
                                                      const double *__restrict__ scale,
                                                      uint16_t *__restrict__ x0,
                                                      float *__restrict__ target) {
  const uint64_t total = (uint64_t)bx.d * bx.h * bx.w;
  const double sd = scale[0], sa = scale[1];
  for (uint64_t u = (uint64_t)blockIdx.x * 256 + threadIdx.x; u < total;
       u += (uint64_t)gridDim.x * 256) {
    const int x = (int)(u % bx.w), y = (int)((u / bx.w) % bx.h), z = (int)(u / ((uint64_t)bx.w * bx.h));
    const size_t v = ((size_t)(bx.z0 + z) * ny + (bx.y0 + y)) * nx + (bx.x0 + x);
    const float f0 = (float)(dose_lo[v] / sd);
    const float f1 = (float)((double)rho[v] / 1.85);
    const float f2 = (float)((double)act[v] / sa);
    const u32x4_t o = {pack2(f0, f1), f2bf(f2), 0u, 0u};
    *reinterpret_cast<u32x4_t *>(x0 + u * 8) = o;
    if (target) target[u] = (float)(dose_hi[v] / sd);
  }
}

// Head, loss and head backward; per block partials [18].
__global__ __launch_bounds__(256) void head_loss_kernel(uint64_t nvox,
                                                        const uint16_t *__restrict__ feat,
                                                        const uint16_t *__restrict__ x0,
                                                        const float *__restrict__ tgt,
                                                        const float *__restrict__ hw,
                                                        const float *__restrict__ hb,
                                                        float wfloor,
                                                        uint16_t *__restrict__ dfeat,
                                                        float *__restrict__ part) {
  __shared__ float s[18][256];
  float w[16];
#pragma unroll
  for (int i = 0; i < 16; ++i) w[i] = hw[i];
  const float b = hb[0];
  const float gscale = 2.0f / (float)nvox;
  float acc[18];
#pragma unroll
  for (int i = 0; i < 18; ++i) acc[i] = 0.f;
  for (uint64_t v = (uint64_t)blockIdx.x * 256 + threadIdx.x; v < nvox;
       v += (uint64_t)gridDim.x * 256) {
    const u32x4_t q0 = *reinterpret_cast<const u32x4_t *>(feat + v * 16);
    const u32x4_t q1 = *reinterpret_cast<const u32x4_t *>(feat + v * 16 + 8);
    float f[16];
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      f[j] = unpack(q0, j);
      f[j + 8] = unpack(q1, j);
    }
    float hsum = 0.f;
#pragma unroll
    for (int i = 0; i < 16; ++i) hsum = fmaf(w[i], f[i], hsum);
    const float pred = bf2f(x0[v * 8]) + (hsum + b);
    const float t = tgt[v];
    const float e = pred - t;
    const float wv = wfloor > 0.f ? 1.0f / fmaxf(t, wfloor) : 1.0f;
    const float gv = gscale * (wv * e);
    float gf[16];
#pragma unroll
    for (int i = 0; i < 16; ++i) {
      gf[i] = f[i] > 0.f ? gv * w[i] : 0.f;
      acc[i] = fmaf(gv, f[i], acc[i]);
    }
    acc[16] += gv;
    acc[17] = fmaf(wv * e, e, acc[17]);
    const u32x4_t o0 = {pack2(gf[0], gf[1]), pack2(gf[2], gf[3]), pack2(gf[4], gf[5]),
                        pack2(gf[6], gf[7])};
    const u32x4_t o1 = {pack2(gf[8], gf[9]), pack2(gf[10], gf[11]), pack2(gf[12], gf[13]),
                        pack2(gf[14], gf[15])};
    *reinterpret_cast<u32x4_t *>(dfeat + v * 16) = o0;
    *reinterpret_cast<u32x4_t *>(dfeat + v * 16 + 8) = o1;
  }
#pragma unroll
  for (int i = 0; i < 18; ++i) s[i][threadIdx.x] = acc[i];
  __syncthreads();
  for (int k = 128; k > 0; k >>= 1) {
    if ((int)threadIdx.x < k)
      for (int i = 0; i < 18; ++i) s[i][threadIdx.x] += s[i][threadIdx.x + k];
    __syncthreads();
  }
  if (threadIdx.x < 18) part[blockIdx.x * 18 + threadIdx.x] = s[threadIdx.x][0];
}

__global__ __launch_bounds__(256) void head_infer_kernel(int ny, int nx, Box bx,
                                                         const uint16_t *__restrict__ feat,
                                                         const uint16_t *__restrict__ x0,
                                                         const float *__restrict__ hw,
                                                         const float *__restrict__ hb,
                                                         const double *__restrict__ scale,
                                                         double *__restrict__ out) {
  float w[16];
#pragma unroll
  for (int i = 0; i < 16; ++i) w[i] = hw[i];
  const float b = hb[0];
  const double sd = scale[0];
  const uint64_t total = (uint64_t)bx.d * bx.h * bx.w;
  for (uint64_t u = (uint64_t)blockIdx.x * 256 + threadIdx.x; u < total;
       u += (uint64_t)gridDim.x * 256) {
    const u32x4_t q0 = *reinterpret_cast<const u32x4_t *>(feat + u * 16);
    const u32x4_t q1 = *reinterpret_cast<const u32x4_t *>(feat + u * 16 + 8);
    float hsum = 0.f;
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      hsum = fmaf(w[j], unpack(q0, j), hsum);
      hsum = fmaf(w[j + 8], unpack(q1, j), hsum);
    }
    const float pred = bf2f(x0[u * 8]) + (hsum + b);
    const int x = (int)(u % bx.w), y = (int)((u / bx.w) % bx.h), z = (int)(u / ((uint64_t)bx.w * bx.h));
    const size_t v = ((size_t)(bx.z0 + z) * ny + (bx.y0 + y)) * nx + (bx.x0 + x);
    out[v] = (double)fmaxf(pred, 0.f) * sd;
  }
}

__device__ __forceinline__ size_t flipped_index(size_t e, int cout, int cin) {
  const int ci = (int)(e % cin);
  const size_t r = e / cin;
  const int t = (int)(r % 27), co = (int)(r / 27);
  return ((size_t)ci * 27 + (26 - t)) * cout + co;
}

__global__ __launch_bounds__(256) void adam_kernel(float *__restrict__ th, float *__restrict__ m,
                                                   float *__restrict__ v,
                                                   const float *__restrict__ g, int64_t n,
                                                   float lr, float b1, float b2, float eps,
                                                   float c1, float c2, uint16_t *__restrict__ wb,
                                                   uint16_t *__restrict__ wt, int cout,
                                                   int cin) {
  for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < n;
       e += (int64_t)gridDim.x * 256) {
    const float gv = g[e];
    const float mv = b1 * m[e] + (1.f - b1) * gv;
    const float vv = b2 * v[e] + (1.f - b2) * gv * gv;
    const float t = th[e] - lr * (mv * c1) / (sqrtf(vv * c2) + eps);
    m[e] = mv;
    v[e] = vv;
    th[e] = t;
    const uint16_t q = (uint16_t)f2bf(t);
    if (wb) wb[e] = q;
    if (wt) wt[flipped_index((size_t)e, cout, cin)] = q;
  }
}

__global__ __launch_bounds__(256) void cast_weight_kernel(const float *__restrict__ th, int64_t n,
                                                          uint16_t *__restrict__ wb,
                                                          uint16_t *__restrict__ wt, int cout,
                                                          int cin) {
  for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < n;
       e += (int64_t)gridDim.x * 256) {
    const uint16_t q = (uint16_t)f2bf(th[e]);
    if (wb) wb[e] = q;
    if (wt) wt[flipped_index((size_t)e, cout, cin)] = q;
  }
}

__global__ void debug_mfma_kernel(const uint16_t *__restrict__ a, const uint16_t *__restrict__ b,
                                  float *__restrict__ d) {
  const int l = threadIdx.x, r = l & 15, g = l >> 4;
  uint32_t av[4], bv[4];
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    av[k] = (uint32_t)a[r * 32 + 8 * g + 2 * k] | ((uint32_t)a[r * 32 + 8 * g + 2 * k + 1] << 16);
    bv[k] = (uint32_t)b[(8 * g + 2 * k) * 16 + r] | ((uint32_t)b[(8 * g + 2 * k + 1) * 16 + r] << 16);
  }
  f32x4_t c = {0.f, 0.f, 0.f, 0.f};
  c = mfma_bf16(u32x4_t{av[0], av[1], av[2], av[3]}, u32x4_t{bv[0], bv[1], bv[2], bv[3]}, c);
#pragma unroll
  for (int i = 0; i < 4; ++i) d[(4 * g + i) * 16 + r] = c[i];
}

// ---------------------------------------------------------------------------
// Host side
// ---------------------------------------------------------------------------
bool aligned16(const void *p) { return ((uintptr_t)p & 15u) == 0; }

unsigned grid_for(uint64_t work, unsigned cap = 8192) {
  uint64_t b = (work + 255) / 256;
  if (b > cap) b = cap;
  return b ? (unsigned)b : 1u;
}

nmd_status check_src(nmd_ctx *c, const nmd_nn_src *x, int cc, int *cin) {
  if (!x || !x->x0 || x->c0 <= 0 || x->c0 % 8 || x->c1 < 0 || x->c1 % 8 ||
      (x->c1 > 0 && !x->x1) || !aligned16(x->x0) || (x->x1 && !aligned16(x->x1)))
    return ctx_fail(c, NMD_E_INVALID, "convolution input: bad pointers or channel counts");
  if (cc && x->c0 % cc)
    return ctx_fail(c, NMD_E_UNSUPPORTED, "first input part of %d channels is not a whole "
                    "number of %d-channel chunks", x->c0, cc);
  *cin = x->c0 + x->c1;
  return NMD_OK;
}

nmd_status check_dims(nmd_ctx *c, int n, int d, int h, int w) {
  if (n < 1 || d < 1 || h < 1 || w < 1 || (uint64_t)n * d * h * w >= (1ull << 31))
    return ctx_fail(c, NMD_E_SHAPE, "bad volume %d x %d x %d x %d", n, d, h, w);
  return NMD_OK;
}

int chunk_of(int cin) { return cin == 8 ? 8 : (cin % 32 == 0 ? 32 : 16); }

template <int CC, int NCB>
hipError_t launch_conv_t(const ConvArgs &a, int n, hipStream_t s) {
  hipLaunchKernelGGL((conv_kernel<CC, NCB>), dim3((unsigned)a.n_tiles, (unsigned)n), dim3(256), 0,
                     s, a);
  return hipGetLastError();
}

nmd_status run_conv(nmd_ctx *c, int n, int d, int h, int w, const Src &src, int cin,
                    const uint16_t *wt, const float *bias, int cout, int relu,
                    const uint16_t *mask, uint16_t *y) {
  ConvArgs a;
  a.src = src;
  a.w = wt;
  a.bias = bias;
  a.mask = mask;
  a.y = y;
  a.d = d;
  a.h = h;
  a.w_ = w;
  a.cin = cin;
  a.cout = cout;
  a.relu = relu;
  a.tiles_x = (w + TX - 1) / TX;
  a.tiles_y = (h + TY - 1) / TY;
  const int cc = chunk_of(cin);
  const int ncb = cout / 16;
  const int tz = conv_tz_of(cc, ncb);  // the launched kernel's tile depth
  a.tiles_z = (d + tz - 1) / tz;
  a.n_tiles = a.tiles_x * a.tiles_y * a.tiles_z;
  hipStream_t s = ctx_stream(c);
  hipError_t e = hipErrorInvalidValue;
  if (cc == 8 && ncb == 1) e = launch_conv_t<8, 1>(a, n, s);
  else if (cc == 16 && ncb == 1) e = launch_conv_t<16, 1>(a, n, s);
  else if (cc == 16 && ncb == 2) e = launch_conv_t<16, 2>(a, n, s);
  else if (cc == 16 && ncb == 3) e = launch_conv_t<16, 3>(a, n, s);
  else if (cc == 32 && ncb == 1) e = launch_conv_t<32, 1>(a, n, s);
  else if (cc == 32 && ncb == 2) e = launch_conv_t<32, 2>(a, n, s);
  else if (cc == 32 && ncb == 4) e = launch_conv_t<32, 4>(a, n, s);
  else if (cc == 32 && ncb == 6) e = launch_conv_t<32, 6>(a, n, s);
  else
    return ctx_fail(c, NMD_E_UNSUPPORTED, "no convolution kernel for %d -> %d channels", cin, cout);
  return ctx_hip(c, e, "conv_kernel");
}

bool conv_shape_ok(int cin, int cout) {
  const int cc = chunk_of(cin);
  const int ncb = cout / 16;
  if (cout % 16 || cin % cc) return false;
  if (cin > 96 || cin < 8) return false;
  switch (cc) {
    case 8: return ncb == 1;
    case 16: return ncb >= 1 && ncb <= 3;
    default: return ncb == 1 || ncb == 2 || ncb == 4 || ncb == 6;
  }
}

}  // namespace

extern "C" {

nmd_status nmd_conv3d_fwd(nmd_ctx *c, int32_t n, int32_t d, int32_t h, int32_t w,
                          const nmd_nn_src *x, const uint16_t *weight, const float *bias,
                          int32_t c_out, int32_t relu, const uint16_t *mask, uint16_t *y) {
  nmd_status s = ctx_enter(c);
  if (s || (s = check_dims(c, n, d, h, w))) return s;
  int cin = 0;
  if ((s = check_src(c, x, 0, &cin))) return s;
  if (!conv_shape_ok(cin, c_out) || x->c0 % chunk_of(cin))
    return ctx_fail(c, NMD_E_UNSUPPORTED, "no convolution kernel for %d (+%d) -> %d channels",
                    x->c0, x->c1, c_out);
  if (!weight || !y || !aligned16(weight) || !aligned16(y) || (mask && !aligned16(mask)))
    return ctx_fail(c, NMD_E_INVALID, "weight and output must be 16-byte aligned device memory");
  const Src src{x->x0, x->x1, x->c0, x->up0 ? 1 : 0, x->c1};
  return run_conv(c, n, d, h, w, src, cin, weight, bias, c_out, relu ? 1 : 0, mask, y);
}

nmd_status nmd_conv3d_bwd_data(nmd_ctx *c, int32_t n, int32_t d, int32_t h, int32_t w,
                               const uint16_t *dy, int32_t c_out, const uint16_t *weight_t,
                               int32_t c_in, const uint16_t *mask, uint16_t *dx) {
  nmd_status s = ctx_enter(c);
  if (s || (s = check_dims(c, n, d, h, w))) return s;
  if (!dy || !weight_t || !dx || !aligned16(dy) || !aligned16(weight_t) || !aligned16(dx) ||
      (mask && !aligned16(mask)))
    return ctx_fail(c, NMD_E_INVALID, "bad pointers");
  // the adjoint is a forward convolution c_out -> c_in with the flipped weight
  if (!conv_shape_ok(c_out, c_in))
    return ctx_fail(c, NMD_E_UNSUPPORTED, "no backward-data kernel for %d <- %d channels", c_in,
                    c_out);
  const Src src{dy, nullptr, c_out, 0, 0};
  return run_conv(c, n, d, h, w, src, c_out, weight_t, nullptr, c_in, 0, mask, dx);
}

nmd_status nmd_conv3d_bwd_weight(nmd_ctx *c, int32_t n, int32_t d, int32_t h, int32_t w,
                                 const nmd_nn_src *x, const uint16_t *dy, int32_t c_out,
                                 float *dw, float *db) {
  nmd_status s = ctx_enter(c);
  if (s || (s = check_dims(c, n, d, h, w))) return s;
  int cin = 0;
  if ((s = check_src(c, x, 0, &cin))) return s;
  const int cc = chunk_of(cin);
  if (cin % cc || x->c0 % cc || cin > 96)
    return ctx_fail(c, NMD_E_UNSUPPORTED, "no backward-weight kernel for %d (+%d) input channels",
                    x->c0, x->c1);
  const int ncbo = c_out / 16;
  int nbw = 0;
  if (c_out % 16 == 0) {
    if (cc == 8 && ncbo == 1) nbw = 4;
    else if (cc == 16 && (ncbo == 1 || ncbo == 2)) nbw = 7;
    else if (cc == 32 && ncbo == 2) nbw = 14;
    else if (cc == 32 && ncbo == 4) nbw = 7;
  }
  if (!nbw)
    return ctx_fail(c, NMD_E_UNSUPPORTED, "no backward-weight kernel for %d -> %d channels", cin,
                    c_out);
  if (!dy || !dw || !aligned16(dy))
    return ctx_fail(c, NMD_E_INVALID, "bad pointers");
  WgradArgs a;
  a.src = Src{x->x0, x->x1, x->c0, x->up0 ? 1 : 0, x->c1};
  a.dy = dy;
  a.n = n;
  a.d = d;
  a.h = h;
  a.w_ = w;
  a.cin = cin;
  a.cout = c_out;
  a.tiles_x = (w + WTX - 1) / WTX;
  a.tiles_y = (h + WTY - 1) / WTY;
  a.tiles_z = (d + WTZ - 1) / WTZ;
  a.n_tiles = n * a.tiles_x * a.tiles_y * a.tiles_z;
  const int nb = (27 * cc + 15) / 16;
  a.ncg = (nb + 4 * nbw - 1) / (4 * nbw);
  const int nch = cin / cc;
  const int64_t ne = (int64_t)c_out * 27 * cin;
  // voxel groups: about 2048 workgroups, at least 2 tiles each, partials <= 64 MB
  int64_t nvg = 2048 / (nch * a.ncg);
  nvg = std::min<int64_t>(nvg, std::max<int64_t>(1, a.n_tiles / 2));
  nvg = std::min<int64_t>(nvg, std::max<int64_t>(1, (64ll << 20) / (ne * 4)));
  nvg = std::max<int64_t>(nvg, 1);
  a.n_vg = (int32_t)nvg;
  const uint64_t nvox = (uint64_t)n * d * h * w;
  const unsigned bgrid = db ? grid_for(nvox, 512) : 0;
  const size_t part_bytes = (size_t)nvg * ne * sizeof(float);
  const size_t bpart_bytes = (size_t)bgrid * c_out * sizeof(float);
  void *ws = nullptr;
  if ((s = ctx_scratch(c, part_bytes + bpart_bytes + 256, &ws))) return s;
  a.part = static_cast<float *>(ws);
  float *bpart = reinterpret_cast<float *>(static_cast<char *>(ws) + ((part_bytes + 255) & ~size_t(255)));
  hipStream_t st = ctx_stream(c);
  const dim3 grid((unsigned)nvg, (unsigned)(nch * a.ncg));
  if (cc == 8) hipLaunchKernelGGL((wgrad_kernel<8, 1, 4>), grid, dim3(256), 0, st, a);
  else if (cc == 16 && ncbo == 1) hipLaunchKernelGGL((wgrad_kernel<16, 1, 7>), grid, dim3(256), 0, st, a);
  else if (cc == 16) hipLaunchKernelGGL((wgrad_kernel<16, 2, 7>), grid, dim3(256), 0, st, a);
  else if (ncbo == 2) hipLaunchKernelGGL((wgrad_kernel<32, 2, 14>), grid, dim3(256), 0, st, a);
  else hipLaunchKernelGGL((wgrad_kernel<32, 4, 7>), grid, dim3(256), 0, st, a);
  if ((s = ctx_hip(c, hipGetLastError(), "wgrad_kernel"))) return s;
  hipLaunchKernelGGL(sum_parts_kernel, dim3((unsigned)std::min<int64_t>((ne + 63) / 64, 4096)),
                     dim3(256), 0, st, a.part, ne, (int)nvg, dw);
  if ((s = ctx_hip(c, hipGetLastError(), "sum_parts_kernel"))) return s;
  if (db) {
    hipLaunchKernelGGL(chan_sum_kernel, dim3(bgrid), dim3(256), 0, st, dy, nvox, c_out, bpart);
    if ((s = ctx_hip(c, hipGetLastError(), "chan_sum_kernel"))) return s;
    hipLaunchKernelGGL(sum_parts_kernel, dim3(1), dim3(256), 0, st, bpart, (int64_t)c_out,
                       (int)bgrid, db);
    if ((s = ctx_hip(c, hipGetLastError(), "sum_parts_kernel"))) return s;
  }
  return NMD_OK;
}

nmd_status nmd_nn_pool2(nmd_ctx *c, int32_t n, int32_t d, int32_t h, int32_t w, int32_t ch,
                        const uint16_t *x, uint16_t *y) {
  nmd_status s = ctx_enter(c);
  if (s || (s = check_dims(c, n, d, h, w))) return s;
  if (d % 2 || h % 2 || w % 2) return ctx_fail(c, NMD_E_SHAPE, "pooling needs even dimensions");
  if (ch <= 0 || ch % 8 || !x || !y || !aligned16(x) || !aligned16(y))
    return ctx_fail(c, NMD_E_INVALID, "bad channels or pointers");
  const uint64_t work = (uint64_t)n * (d / 2) * (h / 2) * (w / 2) * (ch / 8);
  hipLaunchKernelGGL(pool_kernel, dim3(grid_for(work)), dim3(256), 0, ctx_stream(c), x, y, n, d,
                     h, w, ch);
  return ctx_hip(c, hipGetLastError(), "pool_kernel");
}

nmd_status nmd_nn_combine(nmd_ctx *c, int32_t n, int32_t d, int32_t h, int32_t w, int32_t ch,
                          const uint16_t *mask, const uint16_t *a, int32_t a_stride,
                          int32_t a_off, int32_t b_mode, const uint16_t *b, int32_t b_stride,
                          int32_t b_off, uint16_t *out) {
  nmd_status s = ctx_enter(c);
  if (s || (s = check_dims(c, n, d, h, w))) return s;
  if (ch <= 0 || ch % 8 || !out || !aligned16(out) || (mask && !aligned16(mask)))
    return ctx_fail(c, NMD_E_INVALID, "bad channels, mask or output");
  if (a && (!aligned16(a) || a_stride % 8 || a_off % 8 || a_off < 0 || a_off + ch > a_stride))
    return ctx_fail(c, NMD_E_INVALID, "bad first term");
  if (b_mode < 0 || b_mode > 2 || (b_mode && (!b || !aligned16(b) || b_stride % 8 || b_off % 8 ||
                                             b_off < 0 || b_off + ch > b_stride)))
    return ctx_fail(c, NMD_E_INVALID, "bad second term");
  if (b_mode == 2 && (d % 2 || h % 2 || w % 2))
    return ctx_fail(c, NMD_E_SHAPE, "pool backward needs even dimensions");
  const uint64_t work = (uint64_t)n * d * h * w * (ch / 8);
  hipLaunchKernelGGL(combine_kernel, dim3(grid_for(work)), dim3(256), 0, ctx_stream(c), n, d, h,
                     w, ch, mask, a, a_stride, a_off, b_mode, b_mode ? b : nullptr, b_stride,
                     b_off, out);
  return ctx_hip(c, hipGetLastError(), "combine_kernel");
}

static nmd_status check_box(nmd_ctx *c, int nz, int ny, int nx, const int32_t *box, Box *bx) {
  if (!box) return ctx_fail(c, NMD_E_INVALID, "box is required");
  *bx = Box{box[0], box[1], box[2], box[3], box[4], box[5]};
  if (nz < 1 || ny < 1 || nx < 1 || bx->d < 1 || bx->h < 1 || bx->w < 1 || bx->z0 < 0 ||
      bx->y0 < 0 || bx->x0 < 0 || bx->z0 + bx->d > nz || bx->y0 + bx->h > ny ||
      bx->x0 + bx->w > nx)
    return ctx_fail(c, NMD_E_SHAPE, "box outside the %d x %d x %d map", nz, ny, nx);
  return NMD_OK;
}

nmd_status nmd_nn_prepare(nmd_ctx *c, int32_t nz, int32_t ny, int32_t nx, const int32_t *box,
                          const double *dose_lo, const double *dose_hi, const float *density,
                          const float *activity, const uint8_t *label, uint16_t *x0,
                          float *target, double *scale) {
  nmd_status s = ctx_enter(c);
  if (s) return s;
  Box bx;
  if ((s = check_box(c, nz, ny, nx, box, &bx))) return s;
  if (!dose_lo || !density || !activity || !label || !x0 || !scale || !aligned16(x0) ||
      (target && !dose_hi))
    return ctx_fail(c, NMD_E_INVALID, "bad pointers");
  const uint64_t work = (uint64_t)bx.d * bx.h * bx.w;
  const unsigned nb = grid_for(work, 1024);
  void *ws = nullptr;
  if ((s = ctx_scratch(c, (size_t)nb * 3 * sizeof(double), &ws))) return s;
  double *part = static_cast<double *>(ws);
  hipStream_t st = ctx_stream(c);
  hipLaunchKernelGGL(body_stats_kernel, dim3(nb), dim3(256), 0, st, ny, nx, bx, dose_lo,
                     activity, label, part);
  if ((s = ctx_hip(c, hipGetLastError(), "body_stats_kernel"))) return s;
  hipLaunchKernelGGL(body_scale_kernel, dim3(1), dim3(256), 0, st, part, (int)nb, scale);
  if ((s = ctx_hip(c, hipGetLastError(), "body_scale_kernel"))) return s;
  hipLaunchKernelGGL(prepare_kernel, dim3(grid_for(work)), dim3(256), 0, st, ny, nx, bx, dose_lo,
                     dose_hi, density, activity, scale, x0, target);
  return ctx_hip(c, hipGetLastError(), "prepare_kernel");
}

nmd_status nmd_nn_head_loss(nmd_ctx *c, int64_t nvox, const uint16_t *feat, const uint16_t *x0,
                            const float *target, const float *head_w, const float *head_b,
                            float weight_floor, uint16_t *dfeat, float *grad) {
  nmd_status s = ctx_enter(c);
  if (s) return s;
  if (nvox < 1 || nvox >= (1ll << 31) || !feat || !x0 || !target || !head_w || !head_b ||
      !dfeat || !grad || !aligned16(feat) || !aligned16(dfeat) || !aligned16(x0))
    return ctx_fail(c, NMD_E_INVALID, "bad size or pointers");
  const unsigned nb = grid_for((uint64_t)nvox, 1024);
  void *ws = nullptr;
  if ((s = ctx_scratch(c, (size_t)nb * 18 * sizeof(float), &ws))) return s;
  float *part = static_cast<float *>(ws);
  hipStream_t st = ctx_stream(c);
  if (!(weight_floor >= 0.f)) return ctx_fail(c, NMD_E_INVALID, "weight_floor must be >= 0");
  hipLaunchKernelGGL(head_loss_kernel, dim3(nb), dim3(256), 0, st, (uint64_t)nvox, feat, x0,
                     target, head_w, head_b, weight_floor, dfeat, part);
  if ((s = ctx_hip(c, hipGetLastError(), "head_loss_kernel"))) return s;
  hipLaunchKernelGGL(sum_parts_kernel, dim3(1), dim3(256), 0, st, part, (int64_t)18, (int)nb,
                     grad);
  return ctx_hip(c, hipGetLastError(), "sum_parts_kernel");
}

nmd_status nmd_nn_head_infer(nmd_ctx *c, int32_t nz, int32_t ny, int32_t nx, const int32_t *box,
                             const uint16_t *feat, const uint16_t *x0, const float *head_w,
                             const float *head_b, const double *scale, double *out) {
  nmd_status s = ctx_enter(c);
  if (s) return s;
  Box bx;
  if ((s = check_box(c, nz, ny, nx, box, &bx))) return s;
  if (!feat || !x0 || !head_w || !head_b || !scale || !out || !aligned16(feat) || !aligned16(x0))
    return ctx_fail(c, NMD_E_INVALID, "bad pointers");
  const uint64_t work = (uint64_t)bx.d * bx.h * bx.w;
  hipLaunchKernelGGL(head_infer_kernel, dim3(grid_for(work)), dim3(256), 0, ctx_stream(c), ny, nx,
                     bx, feat, x0, head_w, head_b, scale, out);
  return ctx_hip(c, hipGetLastError(), "head_infer_kernel");
}

nmd_status nmd_nn_adam(nmd_ctx *c, float *theta, float *m, float *v, const float *grad,
                       int64_t n, int32_t step, float lr, float beta1, float beta2, float eps,
                       uint16_t *w_bf16, uint16_t *w_t_bf16, int32_t c_out, int32_t c_in) {
  nmd_status s = ctx_enter(c);
  if (s) return s;
  if (n < 1 || !theta || !m || !v || !grad || step < 1 || !(lr > 0) || !(beta1 >= 0) ||
      !(beta1 < 1) || !(beta2 >= 0) || !(beta2 < 1) || !(eps > 0))
    return ctx_fail(c, NMD_E_INVALID, "bad Adam arguments");
  if ((w_bf16 || w_t_bf16) && (c_out < 1 || c_in < 1 || (int64_t)c_out * 27 * c_in != n))
    return ctx_fail(c, NMD_E_SHAPE, "weight copies need n = c_out*27*c_in");
  const float c1 = (float)(1.0 / (1.0 - std::pow((double)beta1, (double)step)));
  const float c2 = (float)(1.0 / (1.0 - std::pow((double)beta2, (double)step)));
  hipLaunchKernelGGL(adam_kernel, dim3(grid_for((uint64_t)n, 2048)), dim3(256), 0, ctx_stream(c),
                     theta, m, v, grad, n, lr, beta1, beta2, eps, c1, c2, w_bf16, w_t_bf16,
                     c_out, c_in);
  return ctx_hip(c, hipGetLastError(), "adam_kernel");
}

nmd_status nmd_nn_cast_weight(nmd_ctx *c, const float *theta, int32_t c_out, int32_t c_in,
                              uint16_t *w_bf16, uint16_t *w_t_bf16) {
  nmd_status s = ctx_enter(c);
  if (s) return s;
  if (!theta || c_out < 1 || c_in < 1) return ctx_fail(c, NMD_E_INVALID, "bad arguments");
  const int64_t n = (int64_t)c_out * 27 * c_in;
  hipLaunchKernelGGL(cast_weight_kernel, dim3(grid_for((uint64_t)n, 2048)), dim3(256), 0,
                     ctx_stream(c), theta, n, w_bf16, w_t_bf16, c_out, c_in);
  return ctx_hip(c, hipGetLastError(), "cast_weight_kernel");
}

nmd_status nmd_debug_mfma(nmd_ctx *c, const uint16_t *a, const uint16_t *b, float *d) {
  nmd_status s = ctx_enter(c);
  if (s) return s;
  if (!a || !b || !d) return ctx_fail(c, NMD_E_INVALID, "bad pointers");
  hipLaunchKernelGGL(debug_mfma_kernel, dim3(1), dim3(64), 0, ctx_stream(c), a, b, d);
  return ctx_hip(c, hipGetLastError(), "debug_mfma_kernel");
}

}  // extern "C"
