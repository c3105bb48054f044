// Host-side launch interface of the HIP kernels (internal to the library).
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

namespace ftm {

constexpr int MAX_STAGES = 16;
// Longest transform (complex points): L = 2 Nt, or the next 7-smooth even
// length, must not exceed it.
#ifndef FTM_FFT_POINTS
#define FTM_FFT_POINTS 4096
#endif
constexpr int FFT_POINTS = FTM_FFT_POINTS;
// FFT kernel choices (for the autotuner): 0 the default (the fixed-plan
// kernels where the length has them, with the larger tile unless it gives
// fewer than 4 tiles per CU), 1 and 2 the fixed-plan kernels' larger and
// smaller column tiles, 3 the runtime-plan kernels.
constexpr int FFT_SHAPES = 4;
// Storage of a transformed vector between phases: float32, float64, or 16
// bits in the product's FP16/BF16 format (the input of a half-precision
// product on the matrix cores, where every stored value is exact in that
// format).
enum : int { ST_F32 = 0, ST_F64 = 1, ST_16 = 2 };
constexpr int FFT_SHAPE_GENERIC = 3;
// Whether length N has fixed-plan kernels.
bool fft_has_fixed(int N);

// Unsigned 32-bit division by an invariant divisor d via multiply-high
// (Granlund and Montgomery, PLDI 1994, Fig. 4.1): with l = ceil(log2 d) and
// m = floor(2^32 (2^l - d) / d) + 1, n / d = (t + ((n - t) >> min(l,1))) >> max(l-1,0)
// where t = mulhi(n, m), exact for every 32-bit n.
struct FastDiv {
  uint32_t m, s1, s2;
};
inline FastDiv make_fastdiv(uint32_t d) {
  uint32_t l = 0;
  while ((1ull << l) < d) ++l;
  FastDiv f;
  f.m = (uint32_t)(((1ull << 32) * ((1ull << l) - d)) / d + 1);
  f.s1 = l < 1 ? l : 1;
  f.s2 = l > 1 ? l - 1 : 0;
  return f;
}
__device__ __forceinline__ uint32_t fast_div(uint32_t n, FastDiv f) {
  const uint32_t t = __umulhi(n, f.m);
  return (t + ((n - t) >> f.s1)) >> f.s2;
}

// Mixed-radix plan of a length-N complex FFT: N = rad[0] * rad[1] * ...
// (at least two passes; a radix of 1 is a copy).  div_ns[s] divides by
// Ns = rad[0] * .. * rad[s-1].  Pass s reads its twiddles
// exp(-2 pi i q jm / (Ns rad[s])) (jm < Ns, q < rad[s]) from the twiddle
// table at toff[s] + jm * rad[s] + q; twiddle_entries() is the table length.
struct FftPlan {
  int N;
  int nst;
  int rad[MAX_STAGES];
  int toff[MAX_STAGES];
  FastDiv div_ns[MAX_STAGES];
  int twiddle_entries() const { return nst ? toff[nst - 1] + N : 0; }
};

// Phases 1+2 (or the setup transform of F): real series x[b][t][s] (t < Nt,
// s < S; addressing below), zero padded to N = plan.N, transformed, bins k = 0 .. N/2 written to
// out[k * out_k_stride + b * out_rhs_stride + (s / ncol) * ld_row + s % ncol].
// With xptr set (device array of nrhs pointers) right-hand side b is read from
// xptr[b] instead of x + b * x_rhs_stride.  Columns S .. pad_to-1 of every
// output row are written as zeros (pad_to <= S: none).
struct RfftArgs {
  const double* x;
  const double* const* xptr;
  int64_t pad_to;
  int64_t x_rhs_stride, x_row_stride;
  // series s of a right-hand side starts at x + (s / ncol) * x_sr +
  // (s mod ncol) * x_sc (x_sc = 1 with ncol >= S: consecutive columns)
  int64_t x_sr, x_sc;
  int64_t S;
  int Nt, nrhs;
  void* out;
  int64_t out_k_stride, out_rhs_stride, ncol, ld_row;
  int r_pad, r_fft, r_next;  // storage formats applied: input, then output
};

// Phases 4+5: half spectra in[k][b][s] (k = 0 .. N/2) -> real series
// y[b][t][s] for t < Nt, scaled by 1/N.
struct IrfftArgs {
  const void* in;
  int64_t in_k_stride, in_rhs_stride;
  int64_t S;
  int Nt, nrhs;
  double* y;
  double* const* yptr;  // optional per-right-hand-side output pointers
  int64_t y_rhs_stride, y_row_stride;
  int r_ifft, r_unpad;  // formats of the outputs (the input arrives rounded into r_ifft by the product)
};

// Phase 3: per-frequency product with the stored spectrum F[k][r][c]
// (row stride ld complex elements, k stride f_k_stride).  Forward reads
// x[k][b][c] and writes y[k][b][r]; adjoint reads x[k][b][r] and writes
// y[k][b][c].
struct GemvArgs {
  const void* F;
  int64_t f_k_stride;
  int ld, Nd, Nm, K, nrhs;
  const void* x;
  int64_t x_k_stride, x_rhs_stride;
  void* y;
  int64_t y_k_stride, y_rhs_stride;
  int r_gemv, r_next;
  int variant;   // kernel variant (tile shape), 0 = default; see ftm_gemv.hip
  int rhs_tile;  // right-hand sides per GEMM tile: 16, 32 or 64 (0: by nrhs)
  int gemm_kind; // FP32-storage GEMM: 1 FP32 MFMA, 2 BF16 MFMA on split terms, 0 default
  int x16;       // half-precision GEMM or forward GEMV: x stored in 16 bits (ST_16) in the product's format
};

// Number of tile-shape variants of the matrix-vector kernels.
constexpr int GEMV_VARIANTS = 4;

// The plans (and twiddle tables, in the transform's compute type) a transform
// can run: `fixed` for the fixed-plan kernels (descending radices for the
// forward transform, ascending for the inverse one, so that their paired
// passes take the smallest radix) and `generic` for the runtime-plan kernels.
struct FftPlans {
  const FftPlan* fixed;
  const void* fixed_tw;
  const FftPlan* generic;
  const void* generic_tw;
};
// shape: the kernel choice (0 = default; FFT_SHAPES above).
hipError_t launch_rfft(bool tc64, int out_st, const RfftArgs& a, const FftPlans& pl, int shape, hipStream_t st);
hipError_t launch_irfft(int in_st, bool tc64, const IrfftArgs& a, const FftPlans& pl, int shape, hipStream_t st);
hipError_t launch_gemv_fwd(int fdt, bool acc64, bool in64, bool out64, const GemvArgs& a,
                           hipStream_t st);
hipError_t launch_gemv_adj(int fdt, bool acc64, bool in64, bool out64, const GemvArgs& a,
                           hipStream_t st);
// Phase 3 for many right-hand sides on the matrix cores (FP32/FP16/BF16
// storage, float32 accumulation; float32 transformed vectors).
hipError_t launch_gemm_fwd(int fdt, const GemvArgs& a, hipStream_t st);
hipError_t launch_gemm_adj(int fdt, const GemvArgs& a, hipStream_t st);
// Phase 3 for many right-hand sides with float64 accumulation on the matrix
// cores (FP64 or FP32 storage; float64 or float32 transformed vectors in/out).
hipError_t launch_gemm_a64(bool adjoint, int fdt, bool in64, bool out64, const GemvArgs& a, hipStream_t st);
// Round n float64 values into storage format dt as the kernels do (from
// float32 after rounding to it, when from_f32).
hipError_t launch_round_values(int dt, bool from_f32, const double* x, double* y, int64_t n, hipStream_t st);
// Partial sums of (y - r)^2 and r^2 per workgroup (256 threads, nblocks
// workgroups): partial[2 b], partial[2 b + 1].
hipError_t launch_sumsq_diff(const double* y, const double* r, int64_t n, double* partial, int nblocks,
                             hipStream_t st);
// Round a float64 complex spectrum to storage format dt (n complex numbers).
hipError_t launch_store_spectrum(const void* src, int dt, void* dst, int64_t n, hipStream_t st);
// Widen rows x ncol complex numbers of storage format dt (row stride ld) to a
// dense float64 complex array.
hipError_t launch_widen_spectrum(const void* src, int dt, void* dst, int64_t rows, int64_t ncol,
                                 int64_t ld, hipStream_t st);

}  // namespace ftm
