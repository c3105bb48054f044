// Phase 3 of the matvec: the per-frequency complex matrix-vector products
// d_k = Fhat_k m_k (forward) and m_k = Fhat_k^H d_k (adjoint), k = 0 .. Nt,
// for gfx950.  Both stream the whole stored spectrum once and are bound by
// HBM bandwidth (0.5 flop per byte in float64).
//
// Spectrum layout: Fhat[k][r][c] with the column index padded to ld (a
// multiple of 8, zero filled), complex interleaved, in the storage format of
// the phase.  Every lane reads 16 bytes per load (1 complex float64, 2 complex
// float32, 4 complex float16/bfloat16), consecutive lanes consecutive columns.
//
// Forward (short and wide Fhat_k, Nd << Nm): a workgroup owns R consecutive
// rows of one frequency and sweeps all columns; every lane keeps R running
// sums and reuses each input value for R rows (a half-precision product reads
// its input in the same 16-bit format, 4 values per 16-byte load, which
// halves the input's share of the reads).  Per-lane sums are reduced
// with cross-lane shuffles and then across the 4 waves through LDS, in a fixed
// order (deterministic, no atomics).
//
// Adjoint: a workgroup owns a tile of 64 column chunks of one frequency; the
// 4 waves split the rows, each lane accumulates its own columns, and the 4
// partial sums meet in LDS.  One output element per lane, no shuffles.  This
// is the column-tiled, 2D-workgroup scheme for short and wide (conjugate)
// transposed products of Section 3.1.1.
#include "ftm_device.h"
#include "ftm_kernels.h"

namespace ftm {

constexpr int GEMV_THREADS = 256;
constexpr int GEMV_WAVES = GEMV_THREADS / 64;
#ifndef FTM_FWD_ROWS
#define FTM_FWD_ROWS 4
#endif
#ifndef FTM_ADJ_UNROLL
#define FTM_ADJ_UNROLL 5
#endif
#ifndef FTM_ADJ_RW
#define FTM_ADJ_RW 4
#endif
#ifndef FTM_ADJ_CPT
#define FTM_ADJ_CPT 1
#endif
constexpr int FWD_ROWS = FTM_FWD_ROWS;

// V consecutive complex input values, widened to TA.
template <class TI, class TA, int V>
__device__ __forceinline__ void load_in(const cplx<TI>* __restrict__ p, cplx<TA>* out) {
  if constexpr (sizeof(TI) == 8) {
#pragma unroll
    for (int v = 0; v < V; ++v) {
      const double2 d = *reinterpret_cast<const double2*>(p + v);
      out[v] = {(TA)d.x, (TA)d.y};
    }
  } else if constexpr (V == 1) {
    const float2 f = *reinterpret_cast<const float2*>(p);
    out[0] = {(TA)f.x, (TA)f.y};
  } else {
#pragma unroll
    for (int v = 0; v < V; v += 2) {
      const float4 f = *reinterpret_cast<const float4*>(p + v);
      out[v] = {(TA)f.x, (TA)f.y};
      out[v + 1] = {(TA)f.z, (TA)f.w};
    }
  }
}

// acc += f * x
template <class T>
__device__ __forceinline__ void cmac(cplx<T>& acc, cplx<T> f, cplx<T> x) {
  acc.x = fma(f.x, x.x, acc.x);
  acc.x = fma(-f.y, x.y, acc.x);
  acc.y = fma(f.x, x.y, acc.y);
  acc.y = fma(f.y, x.x, acc.y);
}
// acc += conj(f) * x
template <class T>
__device__ __forceinline__ void cmac_conj(cplx<T>& acc, cplx<T> f, cplx<T> x) {
  acc.x = fma(f.x, x.x, acc.x);
  acc.x = fma(f.y, x.y, acc.x);
  acc.y = fma(f.x, x.y, acc.y);
  acc.y = fma(-f.y, x.x, acc.y);
}

// The adjoint writes a transformed parameter vector as large as a sizeable
// fraction of the stream it reads; non-temporal stores interfere less with
// that read stream (measured: 1.30 -> 1.24 ms at Nt=1000, Nd=100, Nm=5000).
template <bool NT, class TA, class TO>
__device__ __forceinline__ void store_out(cplx<TO>* p, cplx<TA> v, int r_gemv, int r_next) {
  v = round_to(round_to(v, r_gemv), r_next);
  if constexpr (NT) {
    typedef TO v2 __attribute__((ext_vector_type(2)));
    const v2 w = {(TO)v.x, (TO)v.y};
    __builtin_nontemporal_store(w, reinterpret_cast<v2*>(p));  // one 16/8-byte store
  } else {
    *p = {(TO)v.x, (TO)v.y};
  }
}

template <class S, class TA, class TI, class TO, int R>
__global__ __launch_bounds__(GEMV_THREADS) void gemv_fwd_kernel(GemvArgs a, int nrb) {
  constexpr int V = S::V;
  using elem = typename S::elem;
  const int64_t wg = xcd_order(blockIdx.x, gridDim.x);
  const int64_t per_rhs = (int64_t)a.K * nrb;
  const int64_t b = wg / per_rhs;
  const int64_t rem = wg - b * per_rhs;
  const int64_t k = rem / nrb;
  const int r0 = (int)(rem - k * nrb) * R;
  const int nr = min(R, a.Nd - r0);

  const elem* __restrict__ Fk = reinterpret_cast<const elem*>(a.F) + k * a.f_k_stride + (int64_t)r0 * a.ld;
  const cplx<TI>* __restrict__ xk = reinterpret_cast<const cplx<TI>*>(a.x) + k * a.x_k_stride + b * a.x_rhs_stride;

  cplx<TA> acc[R];
#pragma unroll
  for (int r = 0; r < R; ++r) acc[r] = {(TA)0, (TA)0};

  const int ncv = a.ld / V;
  for (int cv = threadIdx.x; cv < ncv; cv += GEMV_THREADS) {
    uint4 fr[R];
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const int rr = r < nr ? r : nr - 1;  // tail block: re-read the last row (cache hit)
      fr[r] = load_stream(Fk + (int64_t)rr * a.ld + (int64_t)cv * V);
    }
    cplx<TA> xv[V];
    if constexpr (std::is_same<TI, h16>::value)  // V = 4 values in the spectrum's 16-bit format
      Chunk<S, TA>::decode(*reinterpret_cast<const uint4*>(xk + (int64_t)cv * V), xv);
    else
      load_in<TI, TA, V>(xk + (int64_t)cv * V, xv);
#pragma unroll
    for (int r = 0; r < R; ++r) {
      cplx<TA> f[V];
      Chunk<S, TA>::decode(fr[r], f);
#pragma unroll
      for (int v = 0; v < V; ++v) cmac(acc[r], f[v], xv[v]);
    }
  }

  __shared__ cplx<TA> red[GEMV_WAVES][R];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
#pragma unroll
  for (int r = 0; r < R; ++r) {
    TA x = acc[r].x, y = acc[r].y;
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
      x += __shfl_xor(x, off, 64);
      y += __shfl_xor(y, off, 64);
    }
    if (lane == 0) red[w][r] = {x, y};
  }
  __syncthreads();
  if ((int)threadIdx.x < nr) {
    const int r = threadIdx.x;
    cplx<TA> s = red[0][r];
#pragma unroll
    for (int q = 1; q < GEMV_WAVES; ++q) s = cadd(s, red[q][r]);
    cplx<TO>* y = reinterpret_cast<cplx<TO>*>(a.y) + k * a.y_k_stride + b * a.y_rhs_stride + r0 + r;
    store_out<false>(y, s, a.r_gemv, a.r_next);
  }
}

// RW waves split the rows of one column group (partial sums meet in LDS);
// the 4 / RW column groups of a workgroup each cover 64 * CPT column chunks.
template <class S, class TA, class TI, class TO, int RW, int CPT>
__global__ __launch_bounds__(GEMV_THREADS) void gemv_adj_kernel(GemvArgs a, int nct) {
  constexpr int V = S::V;
  constexpr int CG = GEMV_WAVES / RW;
  using elem = typename S::elem;
  const int64_t wg = xcd_order(blockIdx.x, gridDim.x);
  const int64_t per_rhs = (int64_t)a.K * nct;
  const int64_t b = wg / per_rhs;
  const int64_t rem = wg - b * per_rhs;
  const int64_t k = rem / nct;
  const int ct = (int)(rem - k * nct);
  const int lane = threadIdx.x & 63;
  const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int rg = w % RW, cg = w / RW;
  const int ncv = a.ld / V;
  const int cv0 = (ct * CG + cg) * 64 * CPT + lane;

  const elem* __restrict__ Fk = reinterpret_cast<const elem*>(a.F) + k * a.f_k_stride;
  const cplx<TI>* __restrict__ xk = reinterpret_cast<const cplx<TI>*>(a.x) + k * a.x_k_stride + b * a.x_rhs_stride;

  cplx<TA> acc[CPT][V];
#pragma unroll
  for (int i = 0; i < CPT; ++i)
#pragma unroll
    for (int v = 0; v < V; ++v) acc[i][v] = {(TA)0, (TA)0};

  // columns past the end re-read the last chunk (cache hit) and are not stored
  int cvs[CPT];
#pragma unroll
  for (int i = 0; i < CPT; ++i) cvs[i] = min(cv0 + 64 * i, ncv - 1);
#pragma unroll FTM_ADJ_UNROLL
  for (int r = rg; r < a.Nd; r += RW) {
    uint4 u[CPT];
#pragma unroll
    for (int i = 0; i < CPT; ++i) u[i] = load_stream(Fk + (int64_t)r * a.ld + (int64_t)cvs[i] * V);
    const cplx<TI> xr = xk[r];
    const cplx<TA> x = {(TA)xr.x, (TA)xr.y};
#pragma unroll
    for (int i = 0; i < CPT; ++i) {
      cplx<TA> f[V];
      Chunk<S, TA>::decode(u[i], f);
#pragma unroll
      for (int v = 0; v < V; ++v) cmac_conj(acc[i][v], f[v], x);
    }
  }

  if constexpr (RW > 1) {
    __shared__ cplx<TA> red[RW - 1][CG][64][CPT * V];
    if (rg > 0) {
#pragma unroll
      for (int i = 0; i < CPT; ++i)
#pragma unroll
        for (int v = 0; v < V; ++v) red[rg - 1][cg][lane][i * V + v] = acc[i][v];
    }
    __syncthreads();
    if (rg > 0) return;
#pragma unroll
    for (int q = 0; q < RW - 1; ++q)
#pragma unroll
      for (int i = 0; i < CPT; ++i)
#pragma unroll
        for (int v = 0; v < V; ++v) acc[i][v] = cadd(acc[i][v], red[q][cg][lane][i * V + v]);
  }
  cplx<TO>* y = reinterpret_cast<cplx<TO>*>(a.y) + k * a.y_k_stride + b * a.y_rhs_stride;
#pragma unroll
  for (int i = 0; i < CPT; ++i) {
    const int cv = cv0 + 64 * i;
    if (cv >= ncv) continue;
#pragma unroll
    for (int v = 0; v < V; ++v) {
      const int c = cv * V + v;
      if (c < a.Nm) store_out<true>(y + c, acc[i][v], a.r_gemv, a.r_next);
    }
  }
}

// ---- host launchers -----------------------------------------------------------

// Tile-shape variants (chosen per operator by the autotuner):
//   forward  0: 4 rows per workgroup (default), 1: 2 rows, 2: 8 rows, 3: 16 rows
//   adjoint  0: 4 waves split the rows (default), 1: 2 waves split the rows
//            (2 column groups), 2: 4 waves split the rows, 2 chunks per lane,
//            3: 4 waves split the rows, 4 chunks per lane
template <class S, class TA, class TI, class TO, int R>
static hipError_t fwd_go_r(const GemvArgs& a, hipStream_t st) {
  const int nrb = (a.Nd + R - 1) / R;
  const int64_t nwg = (int64_t)a.nrhs * a.K * nrb;
  if (nwg <= 0) return hipSuccess;
  hipLaunchKernelGGL((gemv_fwd_kernel<S, TA, TI, TO, R>), dim3((unsigned)nwg), dim3(GEMV_THREADS), 0, st, a, nrb);
  return hipGetLastError();
}

template <class S, class TA, class TI, class TO>
static hipError_t fwd_go(const GemvArgs& a, hipStream_t st) {
  switch (a.variant) {
    case 1: return fwd_go_r<S, TA, TI, TO, 2>(a, st);
    case 2: return fwd_go_r<S, TA, TI, TO, 8>(a, st);
    case 3: return fwd_go_r<S, TA, TI, TO, 16>(a, st);
    default: return fwd_go_r<S, TA, TI, TO, FWD_ROWS>(a, st);
  }
}

template <class S, class TA, class TI, class TO, int RW, int CPT>
static hipError_t adj_go_l(const GemvArgs& a, hipStream_t st) {
  const int ncv = a.ld / S::V;
  const int per_wg = (GEMV_WAVES / RW) * 64 * CPT;
  const int nct = (ncv + per_wg - 1) / per_wg;
  const int64_t nwg = (int64_t)a.nrhs * a.K * nct;
  if (nwg <= 0) return hipSuccess;
  hipLaunchKernelGGL((gemv_adj_kernel<S, TA, TI, TO, RW, CPT>), dim3((unsigned)nwg), dim3(GEMV_THREADS), 0, st, a,
                     nct);
  return hipGetLastError();
}

template <class S, class TA, class TI, class TO>
static hipError_t adj_go(const GemvArgs& a, hipStream_t st) {
  switch (a.variant) {
    case 1: return adj_go_l<S, TA, TI, TO, 2, 1>(a, st);
    case 2: return adj_go_l<S, TA, TI, TO, 4, 2>(a, st);
    case 3: return adj_go_l<S, TA, TI, TO, 4, 4>(a, st);
    default: return adj_go_l<S, TA, TI, TO, FTM_ADJ_RW, FTM_ADJ_CPT>(a, st);
  }
}

// Supported (storage, accumulation, input, output) combinations: see the
// intermediate storage rule in the host runtime.
template <bool ADJ>
static hipError_t gemv_dispatch(int fdt, bool acc64, bool in64, bool out64, const GemvArgs& a,
                                hipStream_t st) {
#define FTM_GO(S, TA, TI, TO) return ADJ ? adj_go<S, TA, TI, TO>(a, st) : fwd_go<S, TA, TI, TO>(a, st)
  switch (fdt) {
    case DT_F64:
      if (!acc64) break;
      if (in64 && out64) FTM_GO(s_f64, double, double, double);
      if (in64 && !out64) FTM_GO(s_f64, double, double, float);
      if (!in64 && out64) FTM_GO(s_f64, double, float, double);
      FTM_GO(s_f64, double, float, float);
    case DT_F32:
      if (in64 || out64) break;
      if (acc64) FTM_GO(s_f32, double, float, float);
      FTM_GO(s_f32, float, float, float);
    case DT_F16:
      if (in64 || out64 || acc64) break;
      if constexpr (!ADJ) {
        if (a.x16) return fwd_go<s_f16, float, h16, float>(a, st);
      }
      if (a.x16) break;
      FTM_GO(s_f16, float, float, float);
    case DT_BF16:
      if (in64 || out64 || acc64) break;
      if constexpr (!ADJ) {
        if (a.x16) return fwd_go<s_bf16, float, h16, float>(a, st);
      }
      if (a.x16) break;
      FTM_GO(s_bf16, float, float, float);
    default: break;
  }
#undef FTM_GO
  return hipErrorInvalidValue;
}

hipError_t launch_gemv_fwd(int fdt, bool acc64, bool in64, bool out64, const GemvArgs& a, hipStream_t st) {
  return gemv_dispatch<false>(fdt, acc64, in64, out64, a, st);
}
hipError_t launch_gemv_adj(int fdt, bool acc64, bool in64, bool out64, const GemvArgs& a, hipStream_t st) {
  return gemv_dispatch<true>(fdt, acc64, in64, out64, a, st);
}

// ---- spectrum format conversion (setup and inspection only) -------------------

__global__ void store_spectrum_kernel(const cplx<double>* __restrict__ src, int dt, void* dst, int64_t n) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    const cplx<double> v = round_to(src[i], dt);
    switch (dt) {
      case DT_F64: reinterpret_cast<cplx<double>*>(dst)[i] = v; break;
      case DT_F32: reinterpret_cast<cplx<float>*>(dst)[i] = {(float)v.x, (float)v.y}; break;
      case DT_F16:
        reinterpret_cast<h2*>(dst)[i] = {__half_as_ushort(__float2half_rn((float)v.x)),
                                         __half_as_ushort(__float2half_rn((float)v.y))};
        break;
      default: {  // bfloat16: v is exactly representable, keep the high half of the float
        const uint32_t ux = __float_as_uint((float)v.x), uy = __float_as_uint((float)v.y);
        reinterpret_cast<h2*>(dst)[i] = {(uint16_t)(ux >> 16), (uint16_t)(uy >> 16)};
      }
    }
  }
}

__global__ void widen_spectrum_kernel(const void* src, int dt, cplx<double>* __restrict__ dst, int64_t rows,
                                      int64_t ncol, int64_t ld) {
  const int64_t n = rows * ncol;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    const int64_t row = i / ncol, j = row * ld + (i - row * ncol);
    cplx<double> v;
    switch (dt) {
      case DT_F64: v = reinterpret_cast<const cplx<double>*>(src)[j]; break;
      case DT_F32: {
        const cplx<float> f = reinterpret_cast<const cplx<float>*>(src)[j];
        v = {(double)f.x, (double)f.y};
        break;
      }
      case DT_F16: {
        const h2 h = reinterpret_cast<const h2*>(src)[j];
        v = {(double)half_bits_to_float(h.x), (double)half_bits_to_float(h.y)};
        break;
      }
      default: {
        const h2 h = reinterpret_cast<const h2*>(src)[j];
        v = {(double)bf16_bits_to_float(h.x), (double)bf16_bits_to_float(h.y)};
      }
    }
    dst[i] = v;
  }
}

static dim3 grid_for(int64_t n) {
  int64_t g = (n + 255) / 256;
  if (g > 65536) g = 65536;
  if (g < 1) g = 1;
  return dim3((unsigned)g);
}

// The kernels' rounding of values into storage format dt (from float64, or
// from float32 after a round-to-nearest-even into float32 when from_f32).
__global__ void round_values_kernel(int dt, int from_f32, const double* __restrict__ x, double* __restrict__ y,
                                    int64_t n) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    y[i] = from_f32 ? (double)round_to((float)x[i], dt) : round_to(x[i], dt);
}

hipError_t launch_round_values(int dt, bool from_f32, const double* x, double* y, int64_t n, hipStream_t st) {
  hipLaunchKernelGGL(round_values_kernel, grid_for(n), dim3(256), 0, st, dt, from_f32 ? 1 : 0, x, y, n);
  return hipGetLastError();
}

// Per-workgroup partial sums of (y - r)^2 and r^2 over n values, in a fixed
// order (deterministic): partial[2 b], partial[2 b + 1] for workgroup b.
__global__ void sumsq_diff_kernel(const double* __restrict__ y, const double* __restrict__ r, int64_t n,
                                  double* __restrict__ partial) {
  __shared__ double sd[256], sr[256];
  double a = 0.0, c = 0.0;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    const double d = y[i] - r[i];
    a += d * d;
    c += r[i] * r[i];
  }
  sd[threadIdx.x] = a;
  sr[threadIdx.x] = c;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) {
      sd[threadIdx.x] += sd[threadIdx.x + w];
      sr[threadIdx.x] += sr[threadIdx.x + w];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    partial[2 * blockIdx.x] = sd[0];
    partial[2 * blockIdx.x + 1] = sr[0];
  }
}

hipError_t launch_sumsq_diff(const double* y, const double* r, int64_t n, double* partial, int nblocks,
                             hipStream_t st) {
  hipLaunchKernelGGL(sumsq_diff_kernel, dim3(nblocks), dim3(256), 0, st, y, r, n, partial);
  return hipGetLastError();
}

hipError_t launch_store_spectrum(const void* src, int dt, void* dst, int64_t n, hipStream_t st) {
  hipLaunchKernelGGL(store_spectrum_kernel, grid_for(n), dim3(256), 0, st,
                     reinterpret_cast<const cplx<double>*>(src), dt, dst, n);
  return hipGetLastError();
}

hipError_t launch_widen_spectrum(const void* src, int dt, void* dst, int64_t rows, int64_t ncol, int64_t ld,
                                 hipStream_t st) {
  hipLaunchKernelGGL(widen_spectrum_kernel, grid_for(rows * ncol), dim3(256), 0, st, src, dt,
                     reinterpret_cast<cplx<double>*>(dst), rows, ncol, ld);
  return hipGetLastError();
}

}  // namespace ftm
