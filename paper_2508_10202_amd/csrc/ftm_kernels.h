// Host-side launch interface of the HIP kernels (internal to the library).
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

namespace ftm {

constexpr int MAX_STAGES = 16;
// Largest number of complex points one FFT workgroup holds in LDS: P series
// of length N with P * N <= FFT_POINTS (64 KiB of float64 complex).
constexpr int FFT_POINTS = 4096;
constexpr int FFT_THREADS = 256;

// Mixed-radix plan of a length-N complex FFT: N = rad[0] * rad[1] * ...
struct FftPlan {
  int N;
  int nst;
  int rad[MAX_STAGES];
};

// Phases 1+2 (or the setup transform of F): real series x[b][t][s] (t < Nt,
// s < S), zero padded to N = plan.N, transformed, bins k = 0 .. N/2 written to
// out[k * out_k_stride + b * out_rhs_stride + (s / ncol) * ld_row + s % ncol].
struct RfftArgs {
  const double* x;
  int64_t x_rhs_stride, x_row_stride;
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
  int64_t y_rhs_stride, y_row_stride;
  int r_ifft, r_unpad;
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
};

hipError_t launch_rfft(bool tc64, bool out64, const RfftArgs& a, const FftPlan& plan,
                       const void* tw, hipStream_t st);
hipError_t launch_irfft(bool in64, bool tc64, const IrfftArgs& a, const FftPlan& plan,
                        const void* tw, hipStream_t st);
hipError_t launch_gemv_fwd(int fdt, bool acc64, bool in64, bool out64, const GemvArgs& a,
                           hipStream_t st);
hipError_t launch_gemv_adj(int fdt, bool acc64, bool in64, bool out64, const GemvArgs& a,
                           hipStream_t st);
// Round a float64 complex spectrum to storage format dt (n complex numbers).
hipError_t launch_store_spectrum(const void* src, int dt, void* dst, int64_t n, hipStream_t st);
// Widen rows x ncol complex numbers of storage format dt (row stride ld) to a
// dense float64 complex array.
hipError_t launch_widen_spectrum(const void* src, int dt, void* dst, int64_t rows, int64_t ncol,
                                 int64_t ld, hipStream_t st);

}  // namespace ftm
