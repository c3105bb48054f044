// Phase 3 for many right-hand sides: per frequency k the products become
// complex matrix products,
//   forward  Y_k[b][r] = sum_c X_k[b][c] Fhat_k[r][c]          (B x Nd)
//   adjoint  Y_k[b][c] = sum_r X_k[b][r] conj(Fhat_k[r][c])    (B x Nm)
// computed on the matrix cores (MFMA) with float32 accumulation, from FP32,
// FP16 or BF16 storage of the spectrum.
//
// Forward: complex numbers are stored interleaved, so a row of X_k or Fhat_k
// is a real row of length 2*ld.  With X' = raw(X) and the two real variants
// of the spectrum rows Fr' = (re, -im, re, -im, ..) and Fi' = (im, re, ..),
// Re Y = X' Fr'^T and Im Y = X' Fi'^T: two real products over K' = 2 Nm.
// A workgroup owns BM = 16, 32 or 64 right-hand sides (TB tiles of 16) x 64
// rows of one frequency; X' is staged through LDS in chunks of 64 reals and
// shared by the 4 waves, each wave streams its own 16 spectrum rows from HBM.
// The right-hand-side tile follows the batch (a batch of 2 does not pay for
// 64): the tile rows past nrhs are clamped copies, computed and not stored.
//
// Adjoint: the reduction runs over sensors r; each wave owns 16 columns c and
// BM right-hand sides (TB MFMA tiles).  Re Y = xr fr + xi fi and
// Im Y = xi fr - xr fi, four real MFMAs per step.  X_k is small and shared
// by every workgroup of the frequency, so it is read through the caches.
//
// MFMA lane layouts (checked on gfx950): 16x16x4 f32 -- A[i][k] in lane
// i + 16 k, B[k][j] in lane j + 16 k, D[4 g + v][j] in lane j + 16 g,
// register v.  16x16x32 f16/bf16 -- lane i + 16 g holds k = 8 g .. 8 g + 7.
#include "ftm_device.h"
#include "ftm_kernels.h"

namespace ftm {

typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef _Float16 f16x8 __attribute__((ext_vector_type(8)));

constexpr int GEMM_THREADS = 256;
constexpr int GEMM_WAVES = GEMM_THREADS / 64;
constexpr int FWD_BN = 64;   // spectrum rows per workgroup (forward)
constexpr int ADJ_BN = 64;   // columns per workgroup (adjoint)
constexpr int KC = 64;       // reals of K' per LDS chunk (forward)
constexpr int LDS_PAD = 4;   // floats of padding per LDS row (bank spread)

template <class S>
struct MfmaOf;  // the 16x16x32 half-precision MFMA for a 16-bit storage format
template <>
struct MfmaOf<s_bf16> {
  static constexpr int dt = DT_BF16;
  using vec = bf16x8;
  static __device__ __forceinline__ f32x4 mma(vec a, vec b, f32x4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
  }
};
template <>
struct MfmaOf<s_f16> {
  static constexpr int dt = DT_F16;
  using vec = f16x8;
  static __device__ __forceinline__ f32x4 mma(vec a, vec b, f32x4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x32_f16(a, b, c, 0, 0, 0);
  }
};


// ---------------------------------------------------------------------------
// FP32 products on the BF16 matrix cores.  An FP32 value splits exactly into
// three BF16 terms x = x1 + x2 + x3: x1 keeps the top 8 significant bits
// (the upper half of the word), x2 the next 8 of the residual, x3 the rest
// (at most 8 bits); both subtractions are exact.  A product x y is the sum of
// the eight terms xi yj other than x3 y3, which is below 2^-28 |x y|.  Every
// term is exact in float32 and the MFMA accumulates in float32, so the result
// has FP32 accuracy.  The eight 16x16x32 BF16 instructions take 128 cycles
// where the 16x16x4 FP32 instructions doing the same multiply-adds take 256,
// and the split costs four vector operations per value.
// ---------------------------------------------------------------------------
struct Split3 {
  uint32_t h[3];  // BF16 bits of x1, x2, x3 (in the low half)
};
__device__ __forceinline__ Split3 split3(float x) {
  const uint32_t u = __float_as_uint(x);
  const float r1 = x - __uint_as_float(u & 0xffff0000u);
  const uint32_t v = __float_as_uint(r1);
  const float r2 = r1 - __uint_as_float(v & 0xffff0000u);
  return {{u >> 16, v >> 16, __float_as_uint(r2) >> 16}};
}
// pack two BF16 terms into one 32-bit word (lower k first)
__device__ __forceinline__ uint32_t pack2(uint32_t lo, uint32_t hi) { return lo | (hi << 16); }

// acc += sum of A_i B_j over all terms but A_3 B_3, smallest first
__device__ __forceinline__ f32x4 mma_split(const bf16x8 (&a)[3], const bf16x8 (&b)[3], f32x4 acc) {
  acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[2], b[1], acc, 0, 0, 0);
  acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[1], b[2], acc, 0, 0, 0);
  acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[2], b[0], acc, 0, 0, 0);
  acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[1], b[1], acc, 0, 0, 0);
  acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[0], b[2], acc, 0, 0, 0);
  acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[1], b[0], acc, 0, 0, 0);
  acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[0], b[1], acc, 0, 0, 0);
  return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[0], b[0], acc, 0, 0, 0);
}

// ---------------------------------------------------------------------------
// forward, FP32 storage: MFMA 16x16x4 f32
// ---------------------------------------------------------------------------
// NW waves per workgroup, 16 spectrum rows each.  Fewer waves per workgroup
// give more, smaller workgroups: with K = Nt + 1 frequencies the workgroup
// count is rarely a multiple of the CU count, and the CUs that take one
// workgroup more set the kernel's time.
#ifndef FTM_GEMM_FWD_NW
#define FTM_GEMM_FWD_NW 4
#endif
constexpr int GEMM_FWD_NW = FTM_GEMM_FWD_NW;


template <int NW, int TB, bool SKIP>
__global__ __launch_bounds__(64 * NW) void gemm_fwd_f32_kernel(GemvArgs a, int nbb, int nrb) {
  constexpr int TH = 64 * NW, BM = 16 * TB;
  __shared__ float xs[BM][KC + LDS_PAD];
  const int wg = xcd_order(blockIdx.x, gridDim.x);  // grids stay below 2^31 workgroups
  const int per_k = nbb * nrb;
  const int k = wg / per_k;
  const int rem = wg - k * per_k;
  const int bb = rem / nrb, rb = rem - bb * nrb;
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6, g = lane >> 4, l16 = lane & 15;
  const int b0 = bb * BM, r0 = (rb * NW + w) * 16;
  // waves whose 16 rows all lie past Nd only stage X' for the others (their
  // products would be discarded): no spectrum loads, no matrix-core work.
  // Only with SKIP (at least half the waves idle): the branch costs this
  // kernel registers, and with them a wave per SIMD
  const bool rows_live = !SKIP || __builtin_amdgcn_readfirstlane(r0) < a.Nd;
  const int kr = 2 * a.ld;  // reals per row

  const float* __restrict__ X = reinterpret_cast<const float*>(a.x) + 2 * k * a.x_k_stride;
  const int64_t xrow = 2 * a.x_rhs_stride;
  const float* __restrict__ Fk = reinterpret_cast<const float*>(a.F) + 2 * k * a.f_k_stride;
  const int r_me = min(r0 + l16, a.Nd - 1);  // clamped rows: computed, never stored
  const float* __restrict__ frow = Fk + (int64_t)r_me * kr;

  f32x4 re[TB], im[TB];
#pragma unroll
  for (int t = 0; t < TB; ++t) re[t] = im[t] = (f32x4){0.f, 0.f, 0.f, 0.f};

  // cooperative X' staging: BM rows x 64 reals = 16 BM float4; float4 e goes
  // to row e / 16, reals 4 (e mod 16) .. +3, so 16 threads read one row's 256 B
  constexpr int NST = (16 * BM + TH - 1) / TH;
  const float* __restrict__ xsrc[NST];
  int st_row[NST], st_col[NST];
#pragma unroll
  for (int q = 0; q < NST; ++q) {
    const int e = threadIdx.x + TH * q;
    st_row[q] = e >> 4;
    st_col[q] = (e & 15) * 4;
    xsrc[q] = X + min(b0 + min(st_row[q], BM - 1), a.nrhs - 1) * xrow;
  }

  for (int kc = 0; kc < kr; kc += KC) {
    // stage X'[b0..b0+BM)[kc..kc+64) (zero past the row end)
#pragma unroll
    for (int q = 0; q < NST; ++q) {
      if (16 * BM % TH != 0 && st_row[q] >= BM) continue;
      const int col = kc + st_col[q];
      float4 v = make_float4(0.f, 0.f, 0.f, 0.f);
      if (col < kr) v = *reinterpret_cast<const float4*>(xsrc[q] + col);
      *reinterpret_cast<float4*>(&xs[st_row[q]][st_col[q]]) = v;
    }
    // this wave's spectrum rows, the same 64 reals, in MFMA order (no
    // prefetch of the next chunk: its registers would cost two waves per SIMD,
    // which measured slower)
    uint4 fv[4];
#pragma unroll
    for (int s = 0; s < 4; ++s) {
      const int col = kc + 16 * s + 4 * g;
      fv[s] = rows_live && col < kr ? load_stream(frow + col) : make_uint4(0u, 0u, 0u, 0u);
    }
    __syncthreads();
    if (rows_live) {
#pragma unroll
      for (int s = 0; s < 4; ++s) {
        const float f0 = __uint_as_float(fv[s].x), f1 = __uint_as_float(fv[s].y);
        const float f2 = __uint_as_float(fv[s].z), f3 = __uint_as_float(fv[s].w);
        const float br[4] = {f0, -f1, f2, -f3};  // (re, -im, ..)
        const float bi[4] = {f1, f0, f3, f2};    // (im, re, ..)
#pragma unroll
        for (int t = 0; t < TB; ++t) {
          const float4 xa = *reinterpret_cast<const float4*>(&xs[16 * t + l16][16 * s + 4 * g]);
          const float av[4] = {xa.x, xa.y, xa.z, xa.w};
#pragma unroll
          for (int v = 0; v < 4; ++v) {
            re[t] = __builtin_amdgcn_mfma_f32_16x16x4f32(av[v], br[v], re[t], 0, 0, 0);
            im[t] = __builtin_amdgcn_mfma_f32_16x16x4f32(av[v], bi[v], im[t], 0, 0, 0);
          }
        }
      }
    }
    __syncthreads();
  }

  // D[i = b][j = r]: lane l16 + 16 g holds rows 4 g + v of column l16
  const int r = r0 + l16;
  if (r >= a.Nd) return;
  float* Y = reinterpret_cast<float*>(a.y) + 2 * k * a.y_k_stride;
  // FP32 values of the product, rounded into the next phase's format
  with_round<float>(then_round(DT_F32, a.r_next), [&](auto rnd) {
#pragma unroll
    for (int t = 0; t < TB; ++t)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int b = b0 + 16 * t + 4 * g + v;
        if (b < a.nrhs)
          *reinterpret_cast<float2*>(Y + 2 * (b * a.y_rhs_stride + r)) = make_float2(rnd(re[t][v]), rnd(im[t][v]));
      }
  });
}

// ---------------------------------------------------------------------------
// forward, FP16/BF16 storage: MFMA 16x16x32 (K' = 32 reals per instruction).
// The input arrives in 16 bits in the product's format.  The product is
// bound by its loads.  Each wave reads its 16 spectrum rows whole (16 lanes
// per row, 256 contiguous bytes each) into its own LDS slab and takes the
// MFMA operands from there: loads in the MFMA lane layout touch 64 bytes of
// 16 rows per instruction and stream 25% slower (measured with a read-only
// kernel: 4.9 vs 6.4 TB/s).
// ---------------------------------------------------------------------------
constexpr int KCH = 128;  // reals of K' per LDS chunk (half-precision forward)

template <class S, int TB>
__global__ __launch_bounds__(GEMM_THREADS) void gemm_fwd_h_kernel(GemvArgs a, int nbb, int nrb) {
  using M = MfmaOf<S>;
  constexpr int BM = 16 * TB;
  __shared__ __align__(16) uint16_t xs[BM][KCH + 8];             // X' chunk, 16-byte aligned rows
  __shared__ __align__(16) uint16_t fsh[GEMM_WAVES][16][KCH + 8];  // each wave's spectrum rows
  const int wg = xcd_order(blockIdx.x, gridDim.x);  // grids stay below 2^31 workgroups
  const int per_k = nbb * nrb;
  const int k = wg / per_k;
  const int rem = wg - k * per_k;
  const int bb = rem / nrb, rb = rem - bb * nrb;
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6, g = lane >> 4, l16 = lane & 15;
  const int b0 = bb * BM, r0 = rb * FWD_BN + w * 16;
  const int kr = 2 * a.ld;

  const uint16_t* __restrict__ X = reinterpret_cast<const uint16_t*>(a.x) + 2 * k * a.x_k_stride;
  const int64_t xrow = 2 * a.x_rhs_stride;
  const uint16_t* __restrict__ Fk = reinterpret_cast<const uint16_t*>(a.F) + 2 * k * a.f_k_stride;
  // load i of a chunk: row 4 i + lane / 16 of the wave's 16, reals 8 (lane mod 16) .. +7
  constexpr int NF = 16 * KCH / (64 * 8);  // 16-byte loads per lane and chunk
  const int f_row = lane >> 4, f_col = (lane & 15) * 8;
  const uint16_t* __restrict__ frow[NF];
#pragma unroll
  for (int i = 0; i < NF; ++i) frow[i] = Fk + (int64_t)min(r0 + 4 * i + f_row, a.Nd - 1) * kr + f_col;

  f32x4 re[TB], im[TB];
#pragma unroll
  for (int t = 0; t < TB; ++t) re[t] = im[t] = (f32x4){0.f, 0.f, 0.f, 0.f};

  // X' staging: 16-byte piece e (of 16 per row) goes to row e / 16, reals
  // 8 (e mod 16) .. +7, so 16 threads read one row's 256 B.  Chunk kc + KCH
  // is loaded into registers while the matrix cores work on chunk kc.
  int st_row[TB], st_col[TB];
  const uint16_t* __restrict__ xsrc[TB];
#pragma unroll
  for (int q = 0; q < TB; ++q) {
    const int e = threadIdx.x + GEMM_THREADS * q;
    st_row[q] = e >> 4;
    st_col[q] = (e & 15) * 8;
    xsrc[q] = X + min(b0 + st_row[q], a.nrhs - 1) * xrow;
  }
  constexpr int NS = KCH / 32;  // 32-real MFMA steps per chunk
  uint4 xv[TB], fn[NF];
  auto load_chunk = [&](int kc) {
#pragma unroll
    for (int q = 0; q < TB; ++q) {
      const int col = kc + st_col[q];
      xv[q] = col < kr ? *reinterpret_cast<const uint4*>(xsrc[q] + col) : make_uint4(0u, 0u, 0u, 0u);
    }
#pragma unroll
    for (int i = 0; i < NF; ++i)
      fn[i] = kc + f_col < kr ? load_stream(frow[i] + kc) : make_uint4(0u, 0u, 0u, 0u);
  };
  load_chunk(0);
  for (int kc = 0; kc < kr; kc += KCH) {
#pragma unroll
    for (int q = 0; q < TB; ++q) *reinterpret_cast<uint4*>(&xs[st_row[q]][st_col[q]]) = xv[q];
#pragma unroll
    for (int i = 0; i < NF; ++i) *reinterpret_cast<uint4*>(&fsh[w][4 * i + f_row][f_col]) = fn[i];
    __syncthreads();
    if (kc + KCH < kr) load_chunk(kc + KCH);
#pragma unroll
    for (int s = 0; s < NS; ++s) {
      // each 32-bit word is (re | im << 16): Fr' flips the sign of im, Fi' swaps
      const uint4 fv = *reinterpret_cast<const uint4*>(&fsh[w][l16][32 * s + 8 * g]);
      const uint32_t u[4] = {fv.x, fv.y, fv.z, fv.w};
      uint4 ur, ui;
      uint32_t* pr = reinterpret_cast<uint32_t*>(&ur);
      uint32_t* pi = reinterpret_cast<uint32_t*>(&ui);
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        pr[q] = u[q] ^ 0x80000000u;
        pi[q] = (u[q] >> 16) | (u[q] << 16);
      }
      typename M::vec br = *reinterpret_cast<const typename M::vec*>(&ur);
      typename M::vec bi = *reinterpret_cast<const typename M::vec*>(&ui);
#pragma unroll
      for (int t = 0; t < TB; ++t) {
        const typename M::vec xa = *reinterpret_cast<const typename M::vec*>(&xs[16 * t + l16][32 * s + 8 * g]);
        re[t] = M::mma(xa, br, re[t]);
        im[t] = M::mma(xa, bi, im[t]);
      }
    }
    __syncthreads();
  }

  const int r = r0 + l16;
  if (r >= a.Nd) return;
  float* Y = reinterpret_cast<float*>(a.y) + 2 * k * a.y_k_stride;
  // rounded into the product's format (that of S), then the next phase's
  with_round<float>(then_round(M::dt, a.r_next), [&](auto rnd) {
    const RoundInto<M::dt> rs;
#pragma unroll
    for (int t = 0; t < TB; ++t)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int b = b0 + 16 * t + 4 * g + v;
        if (b < a.nrhs)
          *reinterpret_cast<float2*>(Y + 2 * (b * a.y_rhs_stride + r)) = make_float2(rnd(rs(re[t][v])), rnd(rs(im[t][v])));
      }
  });
}

// ---------------------------------------------------------------------------
// forward, FP32 storage on the BF16 matrix cores (three-term split): the
// tiling of the half-precision forward kernel; X' is staged in LDS as its
// three BF16 terms, the spectrum values are split in registers.
// ---------------------------------------------------------------------------
template <int TB, bool SKIP>
__global__ __launch_bounds__(GEMM_THREADS) void gemm_fwd_x3_kernel(GemvArgs a, int nbb, int nrb) {
  constexpr int BM = 16 * TB;
  __shared__ __align__(16) uint16_t xs[3][BM][KC + 8];  // X' terms, 64 reals per chunk
  const int wg = xcd_order(blockIdx.x, gridDim.x);  // grids stay below 2^31 workgroups
  const int per_k = nbb * nrb;
  const int k = wg / per_k;
  const int rem = wg - k * per_k;
  const int bb = rem / nrb, rb = rem - bb * nrb;
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6, g = lane >> 4, l16 = lane & 15;
  const int b0 = bb * BM, r0 = rb * FWD_BN + w * 16;
  // waves whose 16 rows all lie past Nd only stage X' for the others (their
  // products would be discarded): no spectrum loads, no matrix-core work.
  // Only with SKIP (at least half the waves idle): the branch costs this
  // kernel registers, and with them a wave per SIMD
  const bool rows_live = !SKIP || __builtin_amdgcn_readfirstlane(r0) < a.Nd;
  const int kr = 2 * a.ld;

  const float* __restrict__ X = reinterpret_cast<const float*>(a.x) + 2 * k * a.x_k_stride;
  const int64_t xrow = 2 * a.x_rhs_stride;
  const float* __restrict__ Fk = reinterpret_cast<const float*>(a.F) + 2 * k * a.f_k_stride;
  const int r_me = min(r0 + l16, a.Nd - 1);  // clamped rows: computed, never stored
  const float* __restrict__ frow = Fk + (int64_t)r_me * kr;

  f32x4 re[TB], im[TB];
#pragma unroll
  for (int t = 0; t < TB; ++t) re[t] = im[t] = (f32x4){0.f, 0.f, 0.f, 0.f};

  // X' staging as in the half-precision kernel (16 threads read one row's
  // 256 B); chunk kc + KC is loaded while the matrix cores work on chunk kc
  int st_row[TB], st_col[TB];
  const float* __restrict__ xsrc[TB];
#pragma unroll
  for (int q = 0; q < TB; ++q) {
    const int e = threadIdx.x + GEMM_THREADS * q;
    st_row[q] = e >> 4;
    st_col[q] = (e & 15) * 4;
    xsrc[q] = X + min(b0 + st_row[q], a.nrhs - 1) * xrow;
  }
  float4 xv[TB];
  uint4 fn[4];  // lane (l16, g): reals kc + 32 s + 8 g .. + 7 of its row, s = 0, 1
  auto load_chunk = [&](int kc) {
#pragma unroll
    for (int q = 0; q < TB; ++q) {
      const int col = kc + st_col[q];
      xv[q] = col < kr ? *reinterpret_cast<const float4*>(xsrc[q] + col) : make_float4(0.f, 0.f, 0.f, 0.f);
    }
#pragma unroll
    for (int h = 0; h < 4; ++h) {
      const int col = kc + 32 * (h >> 1) + 8 * g + 4 * (h & 1);
      fn[h] = rows_live && col < kr ? load_stream(frow + col) : make_uint4(0u, 0u, 0u, 0u);
    }
  };
  load_chunk(0);
  for (int kc = 0; kc < kr; kc += KC) {
#pragma unroll
    for (int q = 0; q < TB; ++q) {
      const float xq[4] = {xv[q].x, xv[q].y, xv[q].z, xv[q].w};
      Split3 sp[4];
#pragma unroll
      for (int e = 0; e < 4; ++e) sp[e] = split3(xq[e]);
#pragma unroll
      for (int p = 0; p < 3; ++p)
        *reinterpret_cast<uint2*>(&xs[p][st_row[q]][st_col[q]]) =
            make_uint2(pack2(sp[0].h[p], sp[1].h[p]), pack2(sp[2].h[p], sp[3].h[p]));
    }
    uint4 fv[4] = {fn[0], fn[1], fn[2], fn[3]};
    __syncthreads();
    if (kc + KC < kr) load_chunk(kc + KC);
    if (rows_live) {
#pragma unroll
      for (int s = 0; s < 2; ++s) {
        // the 8 reals of this lane: (re, im) pairs; Fr' = (re, -im), Fi' = (im, re)
        const uint32_t u[8] = {fv[2 * s].x, fv[2 * s].y, fv[2 * s].z, fv[2 * s].w,
                               fv[2 * s + 1].x, fv[2 * s + 1].y, fv[2 * s + 1].z, fv[2 * s + 1].w};
        bf16x8 br[3], bi[3];
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const Split3 sre = split3(__uint_as_float(u[2 * q])), sim = split3(__uint_as_float(u[2 * q + 1]));
#pragma unroll
          for (int p = 0; p < 3; ++p) {
            reinterpret_cast<uint32_t*>(&br[p])[q] = pack2(sre.h[p], sim.h[p] ^ 0x8000u);
            reinterpret_cast<uint32_t*>(&bi[p])[q] = pack2(sim.h[p], sre.h[p]);
          }
        }
#pragma unroll
        for (int t = 0; t < TB; ++t) {
          bf16x8 xa[3];
#pragma unroll
          for (int p = 0; p < 3; ++p) xa[p] = *reinterpret_cast<const bf16x8*>(&xs[p][16 * t + l16][32 * s + 8 * g]);
          re[t] = mma_split(xa, br, re[t]);
          im[t] = mma_split(xa, bi, im[t]);
        }
      }
    }
    __syncthreads();
  }

  const int r = r0 + l16;
  if (r >= a.Nd) return;
  float* Y = reinterpret_cast<float*>(a.y) + 2 * k * a.y_k_stride;
  // FP32 values of the product, rounded into the next phase's format
  with_round<float>(then_round(DT_F32, a.r_next), [&](auto rnd) {
#pragma unroll
    for (int t = 0; t < TB; ++t)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int b = b0 + 16 * t + 4 * g + v;
        if (b < a.nrhs)
          *reinterpret_cast<float2*>(Y + 2 * (b * a.y_rhs_stride + r)) = make_float2(rnd(re[t][v]), rnd(im[t][v]));
      }
  });
}

// ---------------------------------------------------------------------------
// adjoint: the reduction runs over sensors r in chunks of RC = 32.  Per chunk
// the workgroup stages its spectrum tile Fhat_k[r0..r0+32)[c0..c0+64) and the
// matching X_k[b0..b0+64)[r0..r0+32) through LDS with coalesced 16-byte rows;
// the MFMA operands are then read from LDS.  Sensors past Nd are zero.
// ---------------------------------------------------------------------------
constexpr int RC = 32;

// FP32 storage: MFMA 16x16x4 f32, 8 k-steps of 4 sensors per chunk.
template <int TB>
__global__ __launch_bounds__(GEMM_THREADS) void gemm_adj_f32_kernel(GemvArgs a, int nbb, int ncb) {
  constexpr int BM = 16 * TB, NX = BM * RC / GEMM_THREADS;  // data-tile loads per thread
  __shared__ cplx<float> fs[RC][ADJ_BN + 2];
  __shared__ cplx<float> xs[BM][RC + 1];
  const int wg = xcd_order(blockIdx.x, gridDim.x);  // grids stay below 2^31 workgroups
  const int per_k = nbb * ncb;
  const int k = wg / per_k;
  const int rem = wg - k * per_k;
  const int bb = rem / ncb, cb = rem - bb * ncb;
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6, g = lane >> 4, l16 = lane & 15;
  const int b0 = bb * BM, c0 = cb * ADJ_BN;

  const cplx<float>* __restrict__ X = reinterpret_cast<const cplx<float>*>(a.x) + k * a.x_k_stride;
  const cplx<float>* __restrict__ Fk = reinterpret_cast<const cplx<float>*>(a.F) + k * a.f_k_stride;

  f32x4 re[TB], im[TB];
#pragma unroll
  for (int t = 0; t < TB; ++t) re[t] = im[t] = (f32x4){0.f, 0.f, 0.f, 0.f};

  // Sensor chunk r0 + RC is loaded into registers while the matrix cores work
  // on chunk r0: the spectrum tile (32 rows x 64 columns, two complex per
  // 16-byte load) and the data tile (BM right-hand sides x 32 sensors).
  float4 fv[4];
  cplx<float> xv[NX];
  auto load_chunk = [&](int r0) {
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int idx = tid + GEMM_THREADS * q;
      const int row = idx >> 5, col = (idx & 31) * 2;
      const int r = r0 + row, c = c0 + col;
      fv[q] = (r < a.Nd && c < a.ld) ? __builtin_bit_cast(float4, load_stream(Fk + (int64_t)r * a.ld + c))
                                      : make_float4(0.f, 0.f, 0.f, 0.f);
    }
#pragma unroll
    for (int q = 0; q < NX; ++q) {
      const int idx = tid + GEMM_THREADS * q;
      const int bl = idx >> 5, rr = idx & 31;
      const int b = min(b0 + bl, a.nrhs - 1), r = r0 + rr;
      xv[q] = r < a.Nd ? X[(int64_t)b * a.x_rhs_stride + r] : cplx<float>{0.f, 0.f};
    }
  };
  load_chunk(0);
  for (int r0 = 0; r0 < a.Nd; r0 += RC) {
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int idx = tid + GEMM_THREADS * q;
      const int row = idx >> 5, col = (idx & 31) * 2;
      fs[row][col] = {fv[q].x, fv[q].y};
      fs[row][col + 1] = {fv[q].z, fv[q].w};
    }
#pragma unroll
    for (int q = 0; q < NX; ++q) {
      const int idx = tid + GEMM_THREADS * q;
      xs[idx >> 5][idx & 31] = xv[q];
    }
    __syncthreads();
    if (r0 + RC < a.Nd) load_chunk(r0 + RC);
#pragma unroll
    for (int s = 0; s < RC / 4; ++s) {
      const cplx<float> f = fs[4 * s + g][w * 16 + l16];
#pragma unroll
      for (int t = 0; t < TB; ++t) {
        const cplx<float> x = xs[16 * t + l16][4 * s + g];
        re[t] = __builtin_amdgcn_mfma_f32_16x16x4f32(x.x, f.x, re[t], 0, 0, 0);
        re[t] = __builtin_amdgcn_mfma_f32_16x16x4f32(x.y, f.y, re[t], 0, 0, 0);
        im[t] = __builtin_amdgcn_mfma_f32_16x16x4f32(x.y, f.x, im[t], 0, 0, 0);
        im[t] = __builtin_amdgcn_mfma_f32_16x16x4f32(-x.x, f.y, im[t], 0, 0, 0);
      }
    }
    __syncthreads();
  }

  const int c = c0 + w * 16 + l16;
  if (c >= a.Nm) return;
  float* Y = reinterpret_cast<float*>(a.y) + 2 * k * a.y_k_stride;
  // FP32 values of the product, rounded into the next phase's format
  with_round<float>(then_round(DT_F32, a.r_next), [&](auto rnd) {
#pragma unroll
    for (int t = 0; t < TB; ++t)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int b = b0 + 16 * t + 4 * g + v;
        if (b < a.nrhs)
          *reinterpret_cast<float2*>(Y + 2 * (b * a.y_rhs_stride + c)) = make_float2(rnd(re[t][v]), rnd(im[t][v]));
      }
  });
}

// FP16/BF16 storage: MFMA 16x16x32, one k-step of 32 sensors per chunk.  The
// data arrive in 16 bits in the product's format; each thread loads 4 sensors
// of one right-hand side per 16-byte load.  (Tiles of 128 columns, which halve
// the data tile's reads from L2, need more registers and measured slower.)
template <class S, int TB>
__global__ __launch_bounds__(GEMM_THREADS) void gemm_adj_h_kernel(GemvArgs a, int nbb, int ncb) {
  using M = MfmaOf<S>;
  constexpr int BM = 16 * TB, NXE = BM * RC / 4;             // 16-byte pieces of the data tile
  constexpr int NX = (NXE + GEMM_THREADS - 1) / GEMM_THREADS;  // per thread
  __shared__ __align__(16) uint32_t fs[RC][ADJ_BN + 4];        // (re | im << 16) per complex
  __shared__ __align__(16) uint16_t xr16[BM][RC + 8];
  __shared__ __align__(16) uint16_t xi16[BM][RC + 8];
  const int wg = xcd_order(blockIdx.x, gridDim.x);  // grids stay below 2^31 workgroups
  const int per_k = nbb * ncb;
  const int k = wg / per_k;
  const int rem = wg - k * per_k;
  const int bb = rem / ncb, cb = rem - bb * ncb;
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6, g = lane >> 4, l16 = lane & 15;
  const int b0 = bb * BM, c0 = cb * ADJ_BN;

  const uint32_t* __restrict__ X = reinterpret_cast<const uint32_t*>(a.x) + k * a.x_k_stride;  // (re | im << 16)
  const uint32_t* __restrict__ Fk = reinterpret_cast<const uint32_t*>(a.F) + k * a.f_k_stride;

  f32x4 re[TB], im[TB];
#pragma unroll
  for (int t = 0; t < TB; ++t) re[t] = im[t] = (f32x4){0.f, 0.f, 0.f, 0.f};

  // Sensor chunk r0 + RC is loaded into registers while the matrix cores work
  // on chunk r0: the spectrum tile (32 rows x 64 columns, four complex per
  // 16-byte load) and the data tile (BM right-hand sides x 32 sensors).
  uint4 fv[2], xv[NX];
  auto load_chunk = [&](int r0) {
#pragma unroll
    for (int q = 0; q < 2; ++q) {
      const int idx = tid + GEMM_THREADS * q;
      const int row = idx >> 4, col = (idx & 15) * 4;
      const int r = r0 + row, c = c0 + col;
      fv[q] = (r < a.Nd && c < a.ld) ? load_stream(Fk + (int64_t)r * a.ld + c) : make_uint4(0u, 0u, 0u, 0u);
    }
#pragma unroll
    for (int q = 0; q < NX; ++q) {
      const int idx = tid + GEMM_THREADS * q;
      if (NXE % GEMM_THREADS != 0 && idx >= NXE) break;
      const int bl = idx >> 3, rr = (idx & 7) * 4;
      const int b = min(b0 + bl, a.nrhs - 1), r = r0 + rr;
      // 4 sensors r .. r + 3 (the row's length is a multiple of 8); those past Nd are zero
      uint4 v = r < a.Nd ? *reinterpret_cast<const uint4*>(X + (int64_t)b * a.x_rhs_stride + r)
                         : make_uint4(0u, 0u, 0u, 0u);
      if (r + 3 >= a.Nd) {
        v.y = r + 1 < a.Nd ? v.y : 0u;
        v.z = r + 2 < a.Nd ? v.z : 0u;
        v.w = r + 3 < a.Nd ? v.w : 0u;
      }
      xv[q] = v;
    }
  };
  load_chunk(0);
  for (int r0 = 0; r0 < a.Nd; r0 += RC) {
#pragma unroll
    for (int q = 0; q < 2; ++q) {
      const int idx = tid + GEMM_THREADS * q;
      const int row = idx >> 4, col = (idx & 15) * 4;
      *reinterpret_cast<uint4*>(&fs[row][col]) = fv[q];  // 16-byte aligned: rows of 68 words
    }
#pragma unroll
    for (int q = 0; q < NX; ++q) {
      const int idx = tid + GEMM_THREADS * q;
      if (NXE % GEMM_THREADS != 0 && idx >= NXE) break;
      const int bl = idx >> 3, rr = (idx & 7) * 4;
      const uint4 v = xv[q];  // (re | im << 16) of 4 sensors: split into the two planes
      *reinterpret_cast<uint2*>(&xr16[bl][rr]) =
          make_uint2((v.x & 0xffffu) | (v.y << 16), (v.z & 0xffffu) | (v.w << 16));
      *reinterpret_cast<uint2*>(&xi16[bl][rr]) =
          make_uint2((v.x >> 16) | (v.y & 0xffff0000u), (v.z >> 16) | (v.w & 0xffff0000u));
    }
    __syncthreads();
    if (r0 + RC < a.Nd) load_chunk(r0 + RC);
    // B operands: fr and fi of sensors 8 g .. 8 g + 7 at this lane's column
    uint4 ufr, ufi;
    uint32_t* pr = reinterpret_cast<uint32_t*>(&ufr);
    uint32_t* pi = reinterpret_cast<uint32_t*>(&ufi);
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const uint32_t w0 = fs[8 * g + 2 * q][w * 16 + l16], w1 = fs[8 * g + 2 * q + 1][w * 16 + l16];
      pr[q] = (w0 & 0xffffu) | (w1 << 16);
      pi[q] = (w0 >> 16) | (w1 & 0xffff0000u);
    }
    const typename M::vec fr = __builtin_bit_cast(typename M::vec, ufr);
    const typename M::vec fi = __builtin_bit_cast(typename M::vec, ufi);
#pragma unroll
    for (int t = 0; t < TB; ++t) {
      const uint4 uxr = *reinterpret_cast<const uint4*>(&xr16[16 * t + l16][8 * g]);
      const uint4 uxi = *reinterpret_cast<const uint4*>(&xi16[16 * t + l16][8 * g]);
      const uint4 uxn = make_uint4(uxr.x ^ 0x80008000u, uxr.y ^ 0x80008000u, uxr.z ^ 0x80008000u,
                                   uxr.w ^ 0x80008000u);
      const typename M::vec vxr = __builtin_bit_cast(typename M::vec, uxr);
      const typename M::vec vxi = __builtin_bit_cast(typename M::vec, uxi);
      const typename M::vec vxn = __builtin_bit_cast(typename M::vec, uxn);
      re[t] = M::mma(vxr, fr, re[t]);
      re[t] = M::mma(vxi, fi, re[t]);
      im[t] = M::mma(vxi, fr, im[t]);
      im[t] = M::mma(vxn, fi, im[t]);
    }
    __syncthreads();
  }

  const int c = c0 + w * 16 + l16;
  if (c >= a.Nm) return;
  float* Y = reinterpret_cast<float*>(a.y) + 2 * k * a.y_k_stride;
  // rounded into the product's format (that of S), then the next phase's
  with_round<float>(then_round(M::dt, a.r_next), [&](auto rnd) {
    const RoundInto<M::dt> rs;
#pragma unroll
    for (int t = 0; t < TB; ++t)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int b = b0 + 16 * t + 4 * g + v;
        if (b < a.nrhs)
          *reinterpret_cast<float2*>(Y + 2 * (b * a.y_rhs_stride + c)) = make_float2(rnd(rs(re[t][v])), rnd(rs(im[t][v])));
      }
  });
}

// FP32 storage on the BF16 matrix cores (three-term split).  The spectrum
// tile (32 sensors x 64 columns) is staged in LDS transposed, as separate
// planes of the real and imaginary BF16 terms with the sensors contiguous, so
// that a B operand (8 sensors of one column) is one 16-byte LDS read; each
// thread loads 8 sensors of one column (lanes along the columns, coalesced).
// The data tile (BM right-hand sides x 32 sensors) is staged the same way.
// Re Y = xr fr + xi fi and Im Y = xi fr + xr (-fi).
template <int TB>
__global__ __launch_bounds__(GEMM_THREADS) void gemm_adj_x3_kernel(GemvArgs a, int nbb, int ncb) {
  constexpr int BM = 16 * TB, RP = RC + 8;  // LDS row pitch in 16-bit elements (16-byte aligned rows)
  constexpr int NXT = BM * (RC / 8);        // data-tile tasks: 8 sensors of one right-hand side
  __shared__ __align__(16) uint16_t fre[3][ADJ_BN][RP];
  __shared__ __align__(16) uint16_t fim[3][ADJ_BN][RP];
  __shared__ __align__(16) uint16_t xre[3][BM][RP];
  __shared__ __align__(16) uint16_t xim[3][BM][RP];
  const int wg = xcd_order(blockIdx.x, gridDim.x);  // grids stay below 2^31 workgroups
  const int per_k = nbb * ncb;
  const int k = wg / per_k;
  const int rem = wg - k * per_k;
  const int bb = rem / ncb, cb = rem - bb * ncb;
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6, g = lane >> 4, l16 = lane & 15;
  const int b0 = bb * BM, c0 = cb * ADJ_BN;

  const cplx<float>* __restrict__ X = reinterpret_cast<const cplx<float>*>(a.x) + k * a.x_k_stride;
  const cplx<float>* __restrict__ Fk = reinterpret_cast<const cplx<float>*>(a.F) + k * a.f_k_stride;

  f32x4 re[TB], im[TB];
#pragma unroll
  for (int t = 0; t < TB; ++t) re[t] = im[t] = (f32x4){0.f, 0.f, 0.f, 0.f};

  // spectrum: thread (column tid mod 64, sensors 8 (tid / 64) ..+7); data:
  // task e = tid + 256 q is (right-hand side e / 4, sensors 8 (e mod 4) ..+7).
  // Sensor chunk r0 + RC is loaded while the matrix cores work on chunk r0.
  const int fc = tid & 63, fr0 = (tid >> 6) * 8;
  constexpr int NQ = (NXT + GEMM_THREADS - 1) / GEMM_THREADS;
  cplx<float> fv[8], xv[NQ][8];
  auto load_chunk = [&](int r0) {
    const int c = c0 + fc;
#pragma unroll
    for (int i = 0; i < 8; ++i) {
      const int r = r0 + fr0 + i;
      fv[i] = (r < a.Nd && c < a.ld) ? Fk[(int64_t)r * a.ld + c] : cplx<float>{0.f, 0.f};
    }
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
      const int e = tid + GEMM_THREADS * q;
      const int b = min(b0 + e / 4, a.nrhs - 1), rs = r0 + 8 * (e & 3);
#pragma unroll
      for (int i = 0; i < 8; ++i)
        xv[q][i] = (NXT % GEMM_THREADS == 0 || e < NXT) && rs + i < a.Nd ? X[(int64_t)b * a.x_rhs_stride + rs + i]
                                                                         : cplx<float>{0.f, 0.f};
    }
  };
  // the three terms of 8 values as three 16-byte rows of LDS
  auto put8 = [](uint16_t* d0, uint16_t* d1, uint16_t* d2, const float (&v)[8]) {
    uint32_t wv[3][4];
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const Split3 lo = split3(v[2 * i]), hi = split3(v[2 * i + 1]);
#pragma unroll
      for (int p = 0; p < 3; ++p) wv[p][i] = pack2(lo.h[p], hi.h[p]);
    }
    *reinterpret_cast<uint4*>(d0) = make_uint4(wv[0][0], wv[0][1], wv[0][2], wv[0][3]);
    *reinterpret_cast<uint4*>(d1) = make_uint4(wv[1][0], wv[1][1], wv[1][2], wv[1][3]);
    *reinterpret_cast<uint4*>(d2) = make_uint4(wv[2][0], wv[2][1], wv[2][2], wv[2][3]);
  };
  load_chunk(0);
  for (int r0 = 0; r0 < a.Nd; r0 += RC) {
    {
      float vr[8], vi[8];
#pragma unroll
      for (int i = 0; i < 8; ++i) {
        vr[i] = fv[i].x;
        vi[i] = fv[i].y;
      }
      put8(&fre[0][fc][fr0], &fre[1][fc][fr0], &fre[2][fc][fr0], vr);
      put8(&fim[0][fc][fr0], &fim[1][fc][fr0], &fim[2][fc][fr0], vi);
    }
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
      const int e = tid + GEMM_THREADS * q;
      if (NXT % GEMM_THREADS != 0 && e >= NXT) continue;
      const int bl = e / 4, rs = 8 * (e & 3);
      float vr[8], vi[8];
#pragma unroll
      for (int i = 0; i < 8; ++i) {
        vr[i] = xv[q][i].x;
        vi[i] = xv[q][i].y;
      }
      put8(&xre[0][bl][rs], &xre[1][bl][rs], &xre[2][bl][rs], vr);
      put8(&xim[0][bl][rs], &xim[1][bl][rs], &xim[2][bl][rs], vi);
    }
    __syncthreads();
    if (r0 + RC < a.Nd) load_chunk(r0 + RC);
    // B operands: the terms of fr, fi and -fi of sensors 8 g .. 8 g + 7 at
    // this lane's column
    bf16x8 fr[3], fi[3], fn[3];
#pragma unroll
    for (int p = 0; p < 3; ++p) {
      const uint4 ur = *reinterpret_cast<const uint4*>(&fre[p][w * 16 + l16][8 * g]);
      const uint4 ui = *reinterpret_cast<const uint4*>(&fim[p][w * 16 + l16][8 * g]);
      fr[p] = __builtin_bit_cast(bf16x8, ur);
      fi[p] = __builtin_bit_cast(bf16x8, ui);
      fn[p] = __builtin_bit_cast(bf16x8, make_uint4(ui.x ^ 0x80008000u, ui.y ^ 0x80008000u, ui.z ^ 0x80008000u,
                                                    ui.w ^ 0x80008000u));
    }
#pragma unroll
    for (int t = 0; t < TB; ++t) {
      bf16x8 vxr[3], vxi[3];
#pragma unroll
      for (int p = 0; p < 3; ++p) {
        vxr[p] = __builtin_bit_cast(bf16x8, *reinterpret_cast<const uint4*>(&xre[p][16 * t + l16][8 * g]));
        vxi[p] = __builtin_bit_cast(bf16x8, *reinterpret_cast<const uint4*>(&xim[p][16 * t + l16][8 * g]));
      }
      re[t] = mma_split(vxr, fr, re[t]);
      re[t] = mma_split(vxi, fi, re[t]);
      im[t] = mma_split(vxi, fr, im[t]);
      im[t] = mma_split(vxr, fn, im[t]);
    }
    __syncthreads();
  }

  const int c = c0 + w * 16 + l16;
  if (c >= a.Nm) return;
  float* Y = reinterpret_cast<float*>(a.y) + 2 * k * a.y_k_stride;
  // FP32 values of the product, rounded into the next phase's format
  with_round<float>(then_round(DT_F32, a.r_next), [&](auto rnd) {
#pragma unroll
    for (int t = 0; t < TB; ++t)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int b = b0 + 16 * t + 4 * g + v;
        if (b < a.nrhs)
          *reinterpret_cast<float2*>(Y + 2 * (b * a.y_rhs_stride + c)) = make_float2(rnd(re[t][v]), rnd(im[t][v]));
      }
  });
}

// ---------------------------------------------------------------------------
// float64 accumulation: MFMA 16x16x4 f64, from float64 storage (an all-FP64
// product) or FP32 storage (FP32 values, products exact in float64; the
// +a64 configurations).  The transformed vectors are float64 or float32 as the
// neighbouring phases store them (TX in, TY out).  Same tilings as the FP32
// kernels; a 16-byte load carries RPL = 16 / sizeof(TF) reals of the spectrum.
// Lane layout of 16x16x4 f64 (checked on gfx950): A[i][k] in lane i + 16 k and
// B[k][j] in lane j + 16 k as for 16x16x4 f32, but D[4 v + g][j] in lane
// j + 16 g, element v (f32: D[4 g + v][j]).
// ---------------------------------------------------------------------------
typedef double f64x4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ void store_c64(double* y, double re, double im, int, int) {
  *reinterpret_cast<double2*>(y) = make_double2(re, im);
}
__device__ __forceinline__ void store_c64(float* y, double re, double im, int r_gemv, int r_next) {
  const int r2 = then_round(r_gemv, r_next);
  *reinterpret_cast<float2*>(y) = make_float2((float)round_to(round_to(re, r_gemv), r2),
                                              (float)round_to(round_to(im, r_gemv), r2));
}

template <class TF, class TX, class TY, int TB>
__global__ __launch_bounds__(GEMM_THREADS) void gemm_fwd_a64_kernel(GemvArgs a, int nbb, int nrb) {
  constexpr int BM = 16 * TB, RPL = 16 / sizeof(TF), KC64 = 16 * RPL;  // reals per chunk
  __shared__ double xs[BM][KC64 + 2];
  const int wg = xcd_order(blockIdx.x, gridDim.x);  // grids stay below 2^31 workgroups
  const int per_k = nbb * nrb;
  const int k = wg / per_k;
  const int rem = wg - k * per_k;
  const int bb = rem / nrb, rb = rem - bb * nrb;
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6, g = lane >> 4, l16 = lane & 15;
  const int b0 = bb * BM, r0 = rb * FWD_BN + w * 16;
  // waves whose 16 rows all lie past Nd only stage X' for the others (their
  // products would be discarded): no spectrum loads, no matrix-core work
  const bool rows_live = __builtin_amdgcn_readfirstlane(r0) < a.Nd;
  const int kr = 2 * a.ld;

  const TX* __restrict__ X = reinterpret_cast<const TX*>(a.x) + 2 * k * a.x_k_stride;
  const int64_t xrow = 2 * a.x_rhs_stride;
  const TF* __restrict__ Fk = reinterpret_cast<const TF*>(a.F) + 2 * k * a.f_k_stride;
  const int r_me = min(r0 + l16, a.Nd - 1);  // clamped rows: computed, never stored
  const TF* __restrict__ frow = Fk + (int64_t)r_me * kr;

  f64x4 re[TB], im[TB];
#pragma unroll
  for (int t = 0; t < TB; ++t) re[t] = im[t] = (f64x4){0.0, 0.0, 0.0, 0.0};

  // X' staging, two reals per thread and step: BM rows x KC64 reals.  Chunk
  // kc + KC64 (spectrum and X') is loaded into registers while the matrix
  // cores work on chunk kc.
  constexpr int NPAIR = BM * KC64 / 2, NST = (NPAIR + GEMM_THREADS - 1) / GEMM_THREADS;
  double2 xv[NST];
  uint4 fn[4];
  auto load_chunk = [&](int kc) {
#pragma unroll
    for (int q = 0; q < NST; ++q) {
      const int e = threadIdx.x + GEMM_THREADS * q;
      if (NPAIR % GEMM_THREADS != 0 && e >= NPAIR) continue;
      const int row = e / (KC64 / 2), col = 2 * (e % (KC64 / 2));
      const TX* src = X + min(b0 + row, a.nrhs - 1) * xrow + kc + col;
      xv[q] = make_double2(0.0, 0.0);
      if (kc + col < kr) {
        if constexpr (sizeof(TX) == 8) {
          xv[q] = *reinterpret_cast<const double2*>(src);
        } else {
          const float2 f = *reinterpret_cast<const float2*>(src);
          xv[q] = make_double2((double)f.x, (double)f.y);
        }
      }
    }
    // this wave's spectrum rows: lane (l16, g) holds reals kc + RPL (4 s + g) ..
#pragma unroll
    for (int s = 0; s < 4; ++s) {
      const int col = kc + RPL * (4 * s + g);
      fn[s] = rows_live && col < kr ? load_stream(frow + col) : make_uint4(0u, 0u, 0u, 0u);
    }
  };
  load_chunk(0);
  for (int kc = 0; kc < kr; kc += KC64) {
#pragma unroll
    for (int q = 0; q < NST; ++q) {
      const int e = threadIdx.x + GEMM_THREADS * q;
      if (NPAIR % GEMM_THREADS != 0 && e >= NPAIR) continue;
      const int row = e / (KC64 / 2), col = 2 * (e % (KC64 / 2));
      xs[row][col] = xv[q].x;
      xs[row][col + 1] = xv[q].y;
    }
    uint4 fv[4];
#pragma unroll
    for (int s = 0; s < 4; ++s) fv[s] = fn[s];
    __syncthreads();
    if (kc + KC64 < kr) load_chunk(kc + KC64);
    if (rows_live) {
#pragma unroll
      for (int s = 0; s < 4; ++s) {
        double f[RPL];
        if constexpr (RPL == 2) {
          const double2 d = __builtin_bit_cast(double2, fv[s]);
          f[0] = d.x;
          f[1] = d.y;
        } else {
          f[0] = (double)__uint_as_float(fv[s].x);
          f[1] = (double)__uint_as_float(fv[s].y);
          f[2] = (double)__uint_as_float(fv[s].z);
          f[3] = (double)__uint_as_float(fv[s].w);
        }
#pragma unroll
        for (int v = 0; v < RPL; ++v) {
          // (re, -im, ..) and (im, re, ..) of the complex pair this real belongs to
          const double br = (v & 1) ? -f[v] : f[v];
          const double bi = (v & 1) ? f[v - 1] : f[v + 1];
#pragma unroll
          for (int t = 0; t < TB; ++t) {
            const double xa = xs[16 * t + l16][RPL * (4 * s + g) + v];
            re[t] = __builtin_amdgcn_mfma_f64_16x16x4f64(xa, br, re[t], 0, 0, 0);
            im[t] = __builtin_amdgcn_mfma_f64_16x16x4f64(xa, bi, im[t], 0, 0, 0);
          }
        }
      }
    }
    __syncthreads();
  }

  const int r = r0 + l16;
  if (r >= a.Nd) return;
  TY* Y = reinterpret_cast<TY*>(a.y) + 2 * k * a.y_k_stride;
#pragma unroll
  for (int t = 0; t < TB; ++t)
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int b = b0 + 16 * t + 4 * v + g;  // D[4 v + g][j] of 16x16x4 f64
      if (b < a.nrhs) store_c64(Y + 2 * (b * a.y_rhs_stride + r), re[t][v], im[t][v], a.r_gemv, a.r_next);
    }
}

// adjoint with float64 accumulation: chunks of RC64 = 16 sensors through LDS
constexpr int RC64 = 16;

template <class TF, class TX, class TY, int TB>
__global__ __launch_bounds__(GEMM_THREADS) void gemm_adj_a64_kernel(GemvArgs a, int nbb, int ncb) {
  constexpr int BM = 16 * TB;
  __shared__ cplx<double> fs[RC64][ADJ_BN + 1];
  __shared__ cplx<double> xs[BM][RC64 + 1];
  const int wg = xcd_order(blockIdx.x, gridDim.x);  // grids stay below 2^31 workgroups
  const int per_k = nbb * ncb;
  const int k = wg / per_k;
  const int rem = wg - k * per_k;
  const int bb = rem / ncb, cb = rem - bb * ncb;
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6, g = lane >> 4, l16 = lane & 15;
  const int b0 = bb * BM, c0 = cb * ADJ_BN;

  const cplx<TX>* __restrict__ X = reinterpret_cast<const cplx<TX>*>(a.x) + k * a.x_k_stride;
  const cplx<TF>* __restrict__ Fk = reinterpret_cast<const cplx<TF>*>(a.F) + k * a.f_k_stride;

  f64x4 re[TB], im[TB];
#pragma unroll
  for (int t = 0; t < TB; ++t) re[t] = im[t] = (f64x4){0.0, 0.0, 0.0, 0.0};

  // Sensor chunk r0 + RC64 is loaded into registers while the matrix cores
  // work on chunk r0: the spectrum tile RC64 x 64 (one complex per thread and
  // step, coalesced rows) and the data tile BM x RC64 (sensors past Nd are zero).
  constexpr int NF = RC64 * ADJ_BN / GEMM_THREADS, NX = (BM * RC64 + GEMM_THREADS - 1) / GEMM_THREADS;
  cplx<TF> fn[NF];
  cplx<TX> xn[NX];
  auto load_chunk = [&](int r0) {
#pragma unroll
    for (int q = 0; q < NF; ++q) {
      const int idx = tid + GEMM_THREADS * q;
      const int row = idx / ADJ_BN, col = idx % ADJ_BN;
      const int r = r0 + row, c = c0 + col;
      fn[q] = (r < a.Nd && c < a.ld) ? Fk[(int64_t)r * a.ld + c] : cplx<TF>{(TF)0, (TF)0};
    }
#pragma unroll
    for (int q = 0; q < NX; ++q) {
      const int idx = tid + GEMM_THREADS * q;
      if ((BM * RC64) % GEMM_THREADS != 0 && idx >= BM * RC64) continue;
      const int bl = idx / RC64, rr = idx % RC64;
      const int b = min(b0 + bl, a.nrhs - 1), r = r0 + rr;
      xn[q] = r < a.Nd ? X[(int64_t)b * a.x_rhs_stride + r] : cplx<TX>{(TX)0, (TX)0};
    }
  };
  load_chunk(0);
  for (int r0 = 0; r0 < a.Nd; r0 += RC64) {
#pragma unroll
    for (int q = 0; q < NF; ++q) {
      const int idx = tid + GEMM_THREADS * q;
      fs[idx / ADJ_BN][idx % ADJ_BN] = {(double)fn[q].x, (double)fn[q].y};
    }
#pragma unroll
    for (int q = 0; q < NX; ++q) {
      const int idx = tid + GEMM_THREADS * q;
      if ((BM * RC64) % GEMM_THREADS != 0 && idx >= BM * RC64) continue;
      xs[idx / RC64][idx % RC64] = {(double)xn[q].x, (double)xn[q].y};
    }
    __syncthreads();
    if (r0 + RC64 < a.Nd) load_chunk(r0 + RC64);
#pragma unroll
    for (int s = 0; s < RC64 / 4; ++s) {
      const cplx<double> f = fs[4 * s + g][w * 16 + l16];
#pragma unroll
      for (int t = 0; t < TB; ++t) {
        const cplx<double> x = xs[16 * t + l16][4 * s + g];
        re[t] = __builtin_amdgcn_mfma_f64_16x16x4f64(x.x, f.x, re[t], 0, 0, 0);
        re[t] = __builtin_amdgcn_mfma_f64_16x16x4f64(x.y, f.y, re[t], 0, 0, 0);
        im[t] = __builtin_amdgcn_mfma_f64_16x16x4f64(x.y, f.x, im[t], 0, 0, 0);
        im[t] = __builtin_amdgcn_mfma_f64_16x16x4f64(-x.x, f.y, im[t], 0, 0, 0);
      }
    }
    __syncthreads();
  }

  const int c = c0 + w * 16 + l16;
  if (c >= a.Nm) return;
  TY* Y = reinterpret_cast<TY*>(a.y) + 2 * k * a.y_k_stride;
#pragma unroll
  for (int t = 0; t < TB; ++t)
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int b = b0 + 16 * t + 4 * v + g;  // D[4 v + g][j] of 16x16x4 f64
      if (b < a.nrhs) store_c64(Y + 2 * (b * a.y_rhs_stride + c), re[t][v], im[t][v], a.r_gemv, a.r_next);
    }
}

// ---- host launchers -----------------------------------------------------------

// Right-hand sides per tile: the asked one (16, 32 or 64), else the
// smallest of them that holds the batch, capped at 64.
static int rhs_tile(const GemvArgs& a) {
  if (a.rhs_tile == 16 || a.rhs_tile == 32 || a.rhs_tile == 64) return a.rhs_tile;
  return a.nrhs <= 16 ? 16 : (a.nrhs <= 32 ? 32 : 64);
}

template <int TB>
static hipError_t gemm_fwd_go(int fdt, const GemvArgs& a, hipStream_t st) {
  const int nbb = (a.nrhs + 16 * TB - 1) / (16 * TB);
  // FP32 storage: the split-term BF16 kernel by default only at 64-RHS tiles,
  // where the product is compute bound (measured faster there, slower on
  // memory-bound smaller tiles)
  const bool split = a.gemm_kind == 2 || (a.gemm_kind == 0 && TB == 4);
  if (fdt == DT_F32 && !split) {
    const int nrb = (a.Nd + 16 * GEMM_FWD_NW - 1) / (16 * GEMM_FWD_NW);
    const int64_t nwg = (int64_t)a.K * nbb * nrb;
    if (nwg <= 0) return hipSuccess;
    if (nwg >= ((int64_t)1 << 31)) return hipErrorInvalidConfiguration;
    if (a.Nd <= 8 * GEMM_FWD_NW)
      hipLaunchKernelGGL((gemm_fwd_f32_kernel<GEMM_FWD_NW, TB, true>), dim3((unsigned)nwg), dim3(64 * GEMM_FWD_NW), 0,
                         st, a, nbb, nrb);
    else
      hipLaunchKernelGGL((gemm_fwd_f32_kernel<GEMM_FWD_NW, TB, false>), dim3((unsigned)nwg), dim3(64 * GEMM_FWD_NW), 0,
                         st, a, nbb, nrb);
    return hipGetLastError();
  }
  const int nrb = (a.Nd + FWD_BN - 1) / FWD_BN;
  const int64_t nwg = (int64_t)a.K * nbb * nrb;
  if (nwg <= 0) return hipSuccess;
  if (nwg >= ((int64_t)1 << 31)) return hipErrorInvalidConfiguration;
  const dim3 grid((unsigned)nwg), block(GEMM_THREADS);
  switch (fdt) {
    case DT_F32:
      if (a.Nd <= FWD_BN / 2) hipLaunchKernelGGL((gemm_fwd_x3_kernel<TB, true>), grid, block, 0, st, a, nbb, nrb);
      else hipLaunchKernelGGL((gemm_fwd_x3_kernel<TB, false>), grid, block, 0, st, a, nbb, nrb);
      break;
    case DT_F16:
      if (!a.x16) return hipErrorInvalidValue;  // the input of a 16-bit product is stored in 16 bits
      hipLaunchKernelGGL((gemm_fwd_h_kernel<s_f16, TB>), grid, block, 0, st, a, nbb, nrb);
      break;
    case DT_BF16:
      if (!a.x16) return hipErrorInvalidValue;
      hipLaunchKernelGGL((gemm_fwd_h_kernel<s_bf16, TB>), grid, block, 0, st, a, nbb, nrb);
      break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

template <int TB>
static hipError_t gemm_adj_go(int fdt, const GemvArgs& a, hipStream_t st) {
  const int nbb = (a.nrhs + 16 * TB - 1) / (16 * TB), ncb = (a.Nm + ADJ_BN - 1) / ADJ_BN;
  const int64_t nwg = (int64_t)a.K * nbb * ncb;
  if (nwg <= 0) return hipSuccess;
  if (nwg >= ((int64_t)1 << 31)) return hipErrorInvalidConfiguration;
  const dim3 grid((unsigned)nwg), block(GEMM_THREADS);
  switch (fdt) {
    case DT_F32:  // the split-term kernel by default at 64-RHS tiles with more than one sensor chunk
      if (a.gemm_kind == 2 || (a.gemm_kind == 0 && TB == 4 && a.Nd > RC))
        hipLaunchKernelGGL((gemm_adj_x3_kernel<TB>), grid, block, 0, st, a, nbb, ncb);
      else hipLaunchKernelGGL((gemm_adj_f32_kernel<TB>), grid, block, 0, st, a, nbb, ncb);
      break;
    case DT_F16:
      if (!a.x16) return hipErrorInvalidValue;  // the input of a 16-bit product is stored in 16 bits
      hipLaunchKernelGGL((gemm_adj_h_kernel<s_f16, TB>), grid, block, 0, st, a, nbb, ncb);
      break;
    case DT_BF16:
      if (!a.x16) return hipErrorInvalidValue;
      hipLaunchKernelGGL((gemm_adj_h_kernel<s_bf16, TB>), grid, block, 0, st, a, nbb, ncb);
      break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

template <class TF, class TX, class TY, int TB>
static hipError_t gemm_a64_go(bool adjoint, const GemvArgs& a, hipStream_t st) {
  const int nbb = (a.nrhs + 16 * TB - 1) / (16 * TB);
  const int nb2 = adjoint ? (a.Nm + ADJ_BN - 1) / ADJ_BN : (a.Nd + FWD_BN - 1) / FWD_BN;
  const int64_t nwg = (int64_t)a.K * nbb * nb2;
  if (nwg <= 0) return hipSuccess;
  if (nwg >= ((int64_t)1 << 31)) return hipErrorInvalidConfiguration;
  const dim3 grid((unsigned)nwg), block(GEMM_THREADS);
  if (adjoint) hipLaunchKernelGGL((gemm_adj_a64_kernel<TF, TX, TY, TB>), grid, block, 0, st, a, nbb, nb2);
  else hipLaunchKernelGGL((gemm_fwd_a64_kernel<TF, TX, TY, TB>), grid, block, 0, st, a, nbb, nb2);
  return hipGetLastError();
}

template <class TF>
static hipError_t gemm_a64_types(bool adjoint, bool in64, bool out64, const GemvArgs& a, int tb, hipStream_t st) {
#define FTM_A64(TX, TY)                                                          \
  switch (tb) {                                                                  \
    case 16: return gemm_a64_go<TF, TX, TY, 1>(adjoint, a, st);                  \
    case 32: return gemm_a64_go<TF, TX, TY, 2>(adjoint, a, st);                  \
    default: return gemm_a64_go<TF, TX, TY, 4>(adjoint, a, st);                  \
  }
  if (in64 && out64) { FTM_A64(double, double) }
  if (in64) { FTM_A64(double, float) }
  if (out64) { FTM_A64(float, double) }
  FTM_A64(float, float)
#undef FTM_A64
}

hipError_t launch_gemm_a64(bool adjoint, int fdt, bool in64, bool out64, const GemvArgs& a, hipStream_t st) {
  const int tb = rhs_tile(a);
  if (fdt == DT_F64) return gemm_a64_types<double>(adjoint, in64, out64, a, tb, st);
  if (fdt == DT_F32) return gemm_a64_types<float>(adjoint, in64, out64, a, tb, st);
  return hipErrorInvalidValue;
}

hipError_t launch_gemm_fwd(int fdt, const GemvArgs& a, hipStream_t st) {
  switch (rhs_tile(a)) {
    case 16: return gemm_fwd_go<1>(fdt, a, st);
    case 32: return gemm_fwd_go<2>(fdt, a, st);
    default: return gemm_fwd_go<4>(fdt, a, st);
  }
}

hipError_t launch_gemm_adj(int fdt, const GemvArgs& a, hipStream_t st) {
  switch (rhs_tile(a)) {
    case 16: return gemm_adj_go<1>(fdt, a, st);
    case 32: return gemm_adj_go<2>(fdt, a, st);
    default: return gemm_adj_go<4>(fdt, a, st);
  }
}

}  // namespace ftm
