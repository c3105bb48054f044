// Batched real FFTs over time with the zero padding (phases 1+2) and the
// unpadding (phases 4+5) fused in, for gfx950: the kernels for any plan
// (runtime radices), and the dispatch that sends the lengths compiled in
// ftm_fft_fixed.hip to their fixed-plan kernels.
//
// Each workgroup holds P complex series of length N = L in LDS and runs a
// mixed-radix (2, 3, 4, 5, 7, 8, 16) self-sorting Stockham FFT on them: every
// pass reads R points at stride N/R, applies the twiddles, does an R-point
// DFT in registers and writes the results back in sorted order (the
// formulation of Govindaraju et al., SC'08).  Two real series share one
// complex transform (real part / imaginary part) and are separated with the
// conjugate symmetry of real spectra afterwards, so P complex series carry 2P
// of the caller's real series.  Twiddles come from per-pass tables computed on
// the host in long double.
#include "ftm_device.h"
#include "ftm_dft.h"
#include "ftm_kernels.h"

namespace ftm {

// ---- LDS layout ------------------------------------------------------------------
// Complex element i of the workgroup's LDS arrays lives at slot lds_ix(i).  The
// early Stockham passes write with strides of R and of R * Ns elements, which
// hit the same LDS banks from many lanes; the remap spreads them.
//   0: identity   1: one pad element per 8   2: one pad element per 16
//   3: XOR of the 16-element slot with the row index (no extra space)
#ifndef FTM_LDS_SWIZZLE
#define FTM_LDS_SWIZZLE 3
#endif
__device__ __forceinline__ int lds_ix(int i) {
#if FTM_LDS_SWIZZLE == 1
  return i + (i >> 3);
#elif FTM_LDS_SWIZZLE == 2
  return i + (i >> 4);
#elif FTM_LDS_SWIZZLE == 3
  return i ^ ((i >> 4) & 15);
#else
  return i;
#endif
}
// LDS elements needed for n logical elements
__host__ __device__ constexpr int lds_size(int n) {
#if FTM_LDS_SWIZZLE == 1
  return n + (n >> 3) + 1;
#elif FTM_LDS_SWIZZLE == 2
  return n + (n >> 4) + 1;
#elif FTM_LDS_SWIZZLE == 3
  return (n + 15) / 16 * 16;
#else
  return n;
#endif
}

#ifndef FTM_FFT_NOHOIST
#define FTM_FFT_NOHOIST 1
#endif

// Twiddle of a stage table entry: base[idx] with a 32-bit byte offset from a
// uniform base (no 64-bit address arithmetic per load).
template <class T>
__device__ __forceinline__ cplx<T> tw_at(const cplx<T>* __restrict__ base, uint32_t idx) {
  return *reinterpret_cast<const cplx<T>*>(reinterpret_cast<const char*>(base) +
                                           (size_t)(idx * (uint32_t)sizeof(cplx<T>)));
}

// One Stockham pass of radix R over P series of length N held in LDS.
// Ns is the product of the radices of the earlier passes.  2^lt threads work
// on each series: thread tid takes series tid >> lt and the butterflies
// j = (tid mod 2^lt) + i 2^lt < N/R.  The stage's twiddles
// exp(-2 pi i q jm / (Ns R)) sit at tws[jm R + q], jm = j mod Ns.  All reads
// of the pass complete (barrier) before any write, so the pass works in place.
template <int R, int TH, int PTS, class T>
__device__ __forceinline__ void fft_pass(cplx<T>* lds, int N, int lt, int Ns, FastDiv dns,
                                         const cplx<T>* __restrict__ tws) {
  constexpr int MAXB = (PTS / TH + R - 1) / R;  // butterflies per thread
  const int nb = N / R;
  const int tps = 1 << lt;
  int tid = threadIdx.x;
#if FTM_FFT_NOHOIST
  // keep the per-pass LDS addresses from being hoisted out of the pass loop
  // for every radix at once (that would cost occupancy for little gain)
  asm volatile("" : "+v"(tid));
#endif
  const int base = (tid >> lt) * N, jj = tid & (tps - 1);
  cplx<T> v[MAXB][R];
  int jms[MAXB];
#pragma unroll
  for (int i = 0; i < MAXB; ++i) {
    const int j = jj + i * tps;
    if (j < nb) {
      const int jm = j - (int)fast_div(j, dns) * Ns;
      jms[i] = jm;
      const int src = base + j;
      v[i][0] = lds[lds_ix(src)];
#pragma unroll
      for (int q = 1; q < R; ++q) v[i][q] = cmul(lds[lds_ix(src + q * nb)], tw_at(tws, (uint32_t)(jm * R + q)));
    }
  }
  __syncthreads();
#pragma unroll
  for (int i = 0; i < MAXB; ++i) {
    const int j = jj + i * tps;
    if (j < nb) {
      dft<R>(v[i]);
      const int jm = jms[i];
      const int dst = base + (j - jm) * R + jm;
#pragma unroll
      for (int q = 0; q < R; ++q) lds[lds_ix(dst + q * Ns)] = v[i][q];
    }
  }
  __syncthreads();
}

// Forward (unnormalised, exp(-2 pi i kt/N)) FFT of P series in LDS.  RX says
// which of the costly radices the plan has (bit 0: 7, bit 1: 16); kernels for
// plans without them do not carry their register cost.
template <class T, int RX, int TH, int PTS>
__device__ void fft_lds(cplx<T>* lds, const FftPlan& plan, int P, const cplx<T>* __restrict__ tw) {
  const int lt = (31 - __clz(TH)) - (31 - __clz(P));  // log2(TH / P)
  int Ns = 1;
  for (int s = 0; s < plan.nst; ++s) {
    const int R = plan.rad[s];
    const cplx<T>* tws = tw + plan.toff[s];
    switch (R) {
      case 2: fft_pass<2, TH, PTS>(lds, plan.N, lt, Ns, plan.div_ns[s], tws); break;
      case 3: fft_pass<3, TH, PTS>(lds, plan.N, lt, Ns, plan.div_ns[s], tws); break;
      case 4: fft_pass<4, TH, PTS>(lds, plan.N, lt, Ns, plan.div_ns[s], tws); break;
      case 5: fft_pass<5, TH, PTS>(lds, plan.N, lt, Ns, plan.div_ns[s], tws); break;
      case 7:
        if constexpr ((RX & 1) != 0) fft_pass<7, TH, PTS>(lds, plan.N, lt, Ns, plan.div_ns[s], tws);
        break;
      case 16:
        if constexpr ((RX & 2) != 0) fft_pass<16, TH, PTS>(lds, plan.N, lt, Ns, plan.div_ns[s], tws);
        break;
      default: fft_pass<8, TH, PTS>(lds, plan.N, lt, Ns, plan.div_ns[s], tws); break;
    }
    Ns *= R;
  }
}

// ---- phases 1+2: pad (+round) + real FFT -------------------------------------

// Loads per thread issued together before any is consumed (memory-level
// parallelism for the strided time-series reads).
constexpr int FFT_LOAD_BATCH = 4;

// Every thread keeps one column (series) of its pair block for the loads and
// the stores, so its addresses advance by a fixed stride: thread tid owns
// column tid mod 2P and rows (or bins) tid / 2P, tid / 2P + TH / 2P, ...

template <class TC, class TO, int RX, bool HALF, int TH, int PTS>
__global__ __launch_bounds__(TH) void rfft_pad_kernel(RfftArgs a, FftPlan plan,
                                                               const cplx<TC>* __restrict__ tw,
                                                               int P, int64_t npb) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  cplx<TC>* lds = reinterpret_cast<cplx<TC>*>(smem_raw);
  const int64_t wg = xcd_order(blockIdx.x, gridDim.x);
  const int64_t b = wg / npb, pb = wg - b * npb;
  const int N = plan.N, Nt = a.Nt, two_p = 2 * P;
  const int64_t s0 = pb * two_p;
  const int lg = 31 - __clz(two_p);  // P is a power of two, 2P <= TH
  const int tid = threadIdx.x;
  const int j = tid & (two_p - 1), r0 = tid >> lg, rstep = TH >> lg;
  const int64_t s = s0 + j;
  const bool live = s < a.S;

  // zero padding t = Nt .. N-1 (phase 1)
  for (int p = 0; p < P; ++p)
    for (int t = Nt + tid; t < N; t += TH) lds[lds_ix(p * N + t)] = {(TC)0, (TC)0};
  // load, rounded to the pad and FFT formats; series 2p -> real, 2p+1 -> imaginary
  {
    const double* xb = a.xptr ? a.xptr[b] : a.x + b * a.x_rhs_stride;
    int64_t off = 0;
    if (live) {
      const int64_t rr = a.ncol >= a.S ? 0 : s / a.ncol;
      off = rr * a.x_sr + (s - rr * a.ncol) * a.x_sc;
    }
    const double* xs = xb + off;
    const int64_t xstep = (int64_t)rstep * a.x_row_stride;
    TC* comp = reinterpret_cast<TC*>(lds) + (j & 1);
    const int zb = (j >> 1) * N;
    const int r_fft2 = then_round(a.r_pad, a.r_fft);
    for (int t = r0; t < Nt; t += FFT_LOAD_BATCH * rstep) {
      const double* q = xs + (int64_t)t * a.x_row_stride;
      double v[FFT_LOAD_BATCH];
#pragma unroll
      for (int u = 0; u < FFT_LOAD_BATCH; ++u) v[u] = (live && t + u * rstep < Nt) ? q[u * xstep] : 0.0;
#pragma unroll
      for (int u = 0; u < FFT_LOAD_BATCH; ++u)
        if (t + u * rstep < Nt)
          comp[2 * lds_ix(zb + t + u * rstep)] = (TC)round_as<HALF>(round_as<HALF>(v[u], a.r_pad), r_fft2);
    }
  }
  __syncthreads();

  fft_lds<TC, RX, TH, PTS>(lds, plan, P, tw);

  // separate the two real spectra: X = (Z_k + conj Z_{N-k}) / 2,
  // Y = (Z_k - conj Z_{N-k}) / 2i; keep bins 0 .. N/2
  const int K = N / 2 + 1;
  if (live) {
    // one output row per right-hand side, or (the setup transform) the
    // columns s of row s / ncol of a [Nd][ld_row] block per bin
    const int64_t row = a.ncol >= a.S ? 0 : s / a.ncol;
    cplx<TO>* o = reinterpret_cast<cplx<TO>*>(a.out) + b * a.out_rhs_stride + row * a.ld_row + (s - row * a.ncol) +
                  r0 * a.out_k_stride;
    const int64_t ostep = (int64_t)rstep * a.out_k_stride;
    const int zb = (j >> 1) * N;
    const bool odd = j & 1;
    const int r_next2 = then_round(a.r_fft, a.r_next);
    for (int k = r0; k < K; k += rstep, o += ostep) {
      const cplx<TC> zk = lds[lds_ix(zb + k)], zr = lds[lds_ix(zb + (k == 0 ? 0 : N - k))];
      cplx<TC> X;
      if (!odd) X = {(TC)0.5 * (zk.x + zr.x), (TC)0.5 * (zk.y - zr.y)};
      else X = {(TC)0.5 * (zk.y + zr.y), (TC)0.5 * (zr.x - zk.x)};
      X = round_as<HALF>(round_as<HALF>(X, a.r_fft), r_next2);
      *o = to_store<TO>(X, a.r_next);  // one 16/8/4-byte store (16-bit: exact in format r_next)
    }
  }
  // the last pair block of a right-hand side also clears the padding columns
  // (the products read them, multiplied by the spectrum's zero padding)
  if (pb == npb - 1 && a.pad_to > a.S) {
    const int npad = (int)(a.pad_to - a.S);
    cplx<TO>* outb = reinterpret_cast<cplx<TO>*>(a.out);
    for (int i = tid; i < K * npad; i += TH) {
      const int k = i / npad;
      outb[k * a.out_k_stride + b * a.out_rhs_stride + a.S + (i - k * npad)] = cplx<TO>{};
    }
  }
}

// ---- phases 4+5: inverse real FFT + scale + unpad ---------------------------

template <class TI, class TC, int RX, bool HALF, int TH, int PTS>
__global__ __launch_bounds__(TH) void irfft_unpad_kernel(IrfftArgs a, FftPlan plan,
                                                                  const cplx<TC>* __restrict__ tw,
                                                                  int P, int64_t npb) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  cplx<TC>* lds = reinterpret_cast<cplx<TC>*>(smem_raw);
  const int64_t wg = xcd_order(blockIdx.x, gridDim.x);
  const int64_t b = wg / npb, pb = wg - b * npb;
  const int N = plan.N, Nt = a.Nt, two_p = 2 * P, hN = N / 2;
  const int64_t s0 = pb * two_p;
  const int lgp = 31 - __clz(P), lg = lgp + 1;  // P is a power of two, 2P <= TH
  const int tid = threadIdx.x;

  // Z = A + iB over the full length from the two half spectra (Hermitian
  // extension; the imaginary parts of bins 0 and N/2 are dropped, as a real
  // inverse transform does).  LDS receives conj(Z): the inverse transform is
  // conj(FFT(conj Z)).  Thread tid reads pair tid mod P at bins tid / P + n TH / P.
  {
    const int K = hN + 1;
    const int p = tid & (P - 1), k0 = tid >> lgp, kstep = TH >> lgp;
    const int64_t s = s0 + 2 * p;
    const bool liveA = s < a.S, liveB = s + 1 < a.S;
    const cplx<TI>* in = reinterpret_cast<const cplx<TI>*>(a.in) + b * a.in_rhs_stride + (liveA ? s : 0);
    const int64_t istep = (int64_t)kstep * a.in_k_stride;
    const int pb_n = p * N;
    for (int k = k0; k < K; k += FFT_LOAD_BATCH * kstep) {
      const cplx<TI>* q = in + (int64_t)k * a.in_k_stride;
      cplx<TC> A[FFT_LOAD_BATCH], B[FFT_LOAD_BATCH];
#pragma unroll
      for (int u = 0; u < FFT_LOAD_BATCH; ++u) {
        A[u] = {(TC)0, (TC)0};
        B[u] = {(TC)0, (TC)0};
        if (k + u * kstep < K) {
          if (liveA) {
            const cplx<TI> v = q[u * istep];
            A[u] = {(TC)v.x, (TC)v.y};
          }
          if (liveB) {
            const cplx<TI> v = q[u * istep + 1];
            B[u] = {(TC)v.x, (TC)v.y};
          }
        }
      }
#pragma unroll
      for (int u = 0; u < FFT_LOAD_BATCH; ++u) {
        const int kk = k + u * kstep;
        if (kk >= K) continue;
        cplx<TC> Au = A[u], Bu = B[u];  // already in the IFFT format: the product's epilogue rounded them
        if (kk == 0 || kk == hN) {
          Au.y = (TC)0;
          Bu.y = (TC)0;
        }
        lds[lds_ix(pb_n + kk)] = {Au.x - Bu.y, -(Au.y + Bu.x)};
        if (kk > 0 && kk < hN) lds[lds_ix(pb_n + N - kk)] = {Au.x + Bu.y, Au.y - Bu.x};
      }
    }
  }
  __syncthreads();

  fft_lds<TC, RX, TH, PTS>(lds, plan, P, tw);

  const int j = tid & (two_p - 1), t0 = tid >> lg, tstep = TH >> lg;
  const int64_t s = s0 + j;
  if (s >= a.S) return;
  const TC inv_n = (TC)(1.0 / (double)N);
  double* y = (a.yptr ? a.yptr[b] : a.y + b * a.y_rhs_stride) + s + (int64_t)t0 * a.y_row_stride;
  const int64_t ystep = (int64_t)tstep * a.y_row_stride;
  const int zb = (j >> 1) * N;
  const bool odd = j & 1;
  const int r_unpad2 = then_round(a.r_ifft, a.r_unpad);
  for (int t = t0; t < Nt; t += tstep, y += ystep) {
    const cplx<TC> z = lds[lds_ix(zb + t)];  // conj of N * (a_t + i b_t)
    TC v = (odd ? -z.y : z.x) * inv_n;
    v = round_as<HALF>(v, a.r_ifft);
    *y = round_as<HALF>((double)v, r_unpad2);
  }
}

// ---- host launchers -----------------------------------------------------------

// Complex series per workgroup: as many length-N series as fit in PTS points,
// but no more pairs than there are series.
static int pairs_per_wg(int N, int64_t S, int pts, int threads) {
  // a power of two (index arithmetic by shifts), no more than fit or are
  // needed, and at most one column per thread (2P <= threads)
  const int64_t need = (S + 1) / 2;
  int P = 1;
  while (2 * P * N <= pts && 2 * P <= need && 4 * P <= threads) P *= 2;
  return P;
}

static bool is_half(int dt) { return dt == DT_F16 || dt == DT_BF16; }

// radix set of a plan for the kernel instantiation: bit 0 radix 7, bit 1 radix 16
static int plan_rx(const FftPlan& plan) {
  int rx = 0;
  for (int i = 0; i < plan.nst; ++i) {
    if (plan.rad[i] == 7) rx |= 1;
    if (plan.rad[i] == 16) rx |= 2;
  }
  return rx;
}

// Workgroup shapes.  float64: 512 threads over at most 2048 points (one
// butterfly per thread for radices >= 4, 32 KiB of LDS) up to N = 2048, else
// over 4096 points.  float32 takes more pairs per workgroup for the same LDS,
// so that a workgroup reads and writes longer runs of adjacent columns.
#ifndef FTM_FFT_TH
#define FTM_FFT_TH 512
#endif
#ifndef FTM_FFT_SMALL_PTS
#define FTM_FFT_SMALL_PTS 2048
#endif
#ifndef FTM_FFT_F32_TH
#define FTM_FFT_F32_TH 512
#endif
#ifndef FTM_FFT_F32_SMALL_PTS
#define FTM_FFT_F32_SMALL_PTS 2048
#endif
#ifndef FTM_FFT_F32_PTS
#define FTM_FFT_F32_PTS 4096
#endif
static_assert(FTM_FFT_F32_PTS >= FFT_POINTS, "the float32 shape must hold the longest transform");

template <class TC, class TO, int PTS, int TH>
static hipError_t rfft_go_shape(const RfftArgs& a, const FftPlan& plan, const void* tw, hipStream_t st) {
  const int P = pairs_per_wg(plan.N, a.S, PTS, TH);
  const int64_t npb = (a.S + 2 * P - 1) / (2 * P);
  const int64_t nwg = npb * a.nrhs;
  if (nwg <= 0) return hipSuccess;
  const size_t lds = (size_t)lds_size(P * plan.N) * sizeof(cplx<TC>);
  const cplx<TC>* t = reinterpret_cast<const cplx<TC>*>(tw);
  const bool half = is_half(a.r_pad) || is_half(a.r_fft) || is_half(a.r_next);
  const dim3 g((unsigned)nwg), blk(TH);
  switch (plan_rx(plan) * 2 + (half ? 1 : 0)) {
#define FTM_RFFT_CASE(RX, H) \
  case RX * 2 + H: hipLaunchKernelGGL((rfft_pad_kernel<TC, TO, RX, H, TH, PTS>), g, blk, lds, st, a, plan, t, P, npb); break;
    FTM_RFFT_CASE(0, 0) FTM_RFFT_CASE(0, 1) FTM_RFFT_CASE(1, 0) FTM_RFFT_CASE(1, 1)
    FTM_RFFT_CASE(2, 0) FTM_RFFT_CASE(2, 1) FTM_RFFT_CASE(3, 0) FTM_RFFT_CASE(3, 1)
#undef FTM_RFFT_CASE
  }
  return hipGetLastError();
}

template <class TC, class TO>
static hipError_t rfft_go(const RfftArgs& a, const FftPlan& plan, const void* tw, hipStream_t st) {
  if constexpr (sizeof(TC) == 4) {
    if (plan.N <= FTM_FFT_F32_SMALL_PTS)
      return rfft_go_shape<TC, TO, FTM_FFT_F32_SMALL_PTS, FTM_FFT_F32_TH>(a, plan, tw, st);
    return rfft_go_shape<TC, TO, FTM_FFT_F32_PTS, FTM_FFT_F32_TH>(a, plan, tw, st);
  } else {
    if (plan.N <= FTM_FFT_SMALL_PTS) return rfft_go_shape<TC, TO, FTM_FFT_SMALL_PTS, FTM_FFT_TH>(a, plan, tw, st);
    return rfft_go_shape<TC, TO, FFT_POINTS, FTM_FFT_TH>(a, plan, tw, st);
  }
}

// Lengths with fixed-plan kernels (ftm_fft_fixed.hip, compiled once per
// length; the build compiles exactly this list).
#define FTM_FIXED_LENGTHS(X) X(128) X(256) X(400) X(512) X(1024) X(2000)
#define FTM_DECLARE_FIXED(n)                                                                                  \
  bool launch_rfft_fixed_##n(bool tc64, int out_st, const RfftArgs& a, const FftPlan& plan, const void* tw,  \
                             int shape, hipStream_t st, hipError_t* err);                                   \
  bool launch_irfft_fixed_##n(int in_st, bool tc64, const IrfftArgs& a, const FftPlan& plan, const void* tw, \
                              int shape, hipStream_t st, hipError_t* err);
FTM_FIXED_LENGTHS(FTM_DECLARE_FIXED)
#undef FTM_DECLARE_FIXED

bool fft_has_fixed(int N) {
#define FTM_IS_FIXED(n) if (N == n) return true;
  FTM_FIXED_LENGTHS(FTM_IS_FIXED)
#undef FTM_IS_FIXED
  return false;
}

hipError_t launch_rfft(bool tc64, int out_st, const RfftArgs& a, const FftPlans& pl, int shape, hipStream_t st) {
  if (shape != FFT_SHAPE_GENERIC) {
    hipError_t e = hipSuccess;
    const FftPlan& fp = *pl.fixed;
#define FTM_TRY_FIXED(n) \
  if (fp.N == n && launch_rfft_fixed_##n(tc64, out_st, a, fp, pl.fixed_tw, shape, st, &e)) return e;
    FTM_FIXED_LENGTHS(FTM_TRY_FIXED)
#undef FTM_TRY_FIXED
  }
  const FftPlan& gp = *pl.generic;
  const void* tw = pl.generic_tw;
  if (tc64) {
    if (out_st == ST_F64) return rfft_go<double, double>(a, gp, tw, st);
    if (out_st == ST_16) return rfft_go<double, h16>(a, gp, tw, st);
    return rfft_go<double, float>(a, gp, tw, st);
  }
  if (out_st == ST_16) return rfft_go<float, h16>(a, gp, tw, st);
  return rfft_go<float, float>(a, gp, tw, st);
}

template <class TI, class TC, int PTS, int TH>
static hipError_t irfft_go_shape(const IrfftArgs& a, const FftPlan& plan, const void* tw, hipStream_t st) {
  const int P = pairs_per_wg(plan.N, a.S, PTS, TH);
  const int64_t npb = (a.S + 2 * P - 1) / (2 * P);
  const int64_t nwg = npb * a.nrhs;
  if (nwg <= 0) return hipSuccess;
  const size_t lds = (size_t)lds_size(P * plan.N) * sizeof(cplx<TC>);
  const cplx<TC>* t = reinterpret_cast<const cplx<TC>*>(tw);
  const bool half = is_half(a.r_ifft) || is_half(a.r_unpad);
  const dim3 g((unsigned)nwg), blk(TH);
  switch (plan_rx(plan) * 2 + (half ? 1 : 0)) {
#define FTM_IRFFT_CASE(RX, H) \
  case RX * 2 + H: hipLaunchKernelGGL((irfft_unpad_kernel<TI, TC, RX, H, TH, PTS>), g, blk, lds, st, a, plan, t, P, npb); break;
    FTM_IRFFT_CASE(0, 0) FTM_IRFFT_CASE(0, 1) FTM_IRFFT_CASE(1, 0) FTM_IRFFT_CASE(1, 1)
    FTM_IRFFT_CASE(2, 0) FTM_IRFFT_CASE(2, 1) FTM_IRFFT_CASE(3, 0) FTM_IRFFT_CASE(3, 1)
#undef FTM_IRFFT_CASE
  }
  return hipGetLastError();
}

template <class TI, class TC>
static hipError_t irfft_go(const IrfftArgs& a, const FftPlan& plan, const void* tw, hipStream_t st) {
  if constexpr (sizeof(TC) == 4) {
    // the inverse transform gains from the wider shape (longer output rows
    // per workgroup) once there are enough workgroups to fill the chip
    const int64_t wide_wgs = (a.S + 2 * pairs_per_wg(plan.N, a.S, FTM_FFT_F32_PTS, FTM_FFT_F32_TH) - 1) /
                             (2 * pairs_per_wg(plan.N, a.S, FTM_FFT_F32_PTS, FTM_FFT_F32_TH)) * a.nrhs;
    if (plan.N <= FTM_FFT_F32_SMALL_PTS && wide_wgs < 1024)
      return irfft_go_shape<TI, TC, FTM_FFT_F32_SMALL_PTS, FTM_FFT_F32_TH>(a, plan, tw, st);
    return irfft_go_shape<TI, TC, FTM_FFT_F32_PTS, FTM_FFT_F32_TH>(a, plan, tw, st);
  } else {
    if (plan.N <= FTM_FFT_SMALL_PTS) return irfft_go_shape<TI, TC, FTM_FFT_SMALL_PTS, FTM_FFT_TH>(a, plan, tw, st);
    return irfft_go_shape<TI, TC, FFT_POINTS, FTM_FFT_TH>(a, plan, tw, st);
  }
}

hipError_t launch_irfft(int in_st, bool tc64, const IrfftArgs& a, const FftPlans& pl, int shape, hipStream_t st) {
  if (shape != FFT_SHAPE_GENERIC) {
    hipError_t e = hipSuccess;
    const FftPlan& fp = *pl.fixed;
#define FTM_TRY_FIXED(n) \
  if (fp.N == n && launch_irfft_fixed_##n(in_st, tc64, a, fp, pl.fixed_tw, shape, st, &e)) return e;
    FTM_FIXED_LENGTHS(FTM_TRY_FIXED)
#undef FTM_TRY_FIXED
  }
  const FftPlan& gp = *pl.generic;
  const void* tw = pl.generic_tw;
  if (in_st == ST_16) return hipErrorInvalidValue;  // not a storage the inverse transform reads
  if (tc64) return in_st == ST_F64 ? irfft_go<double, double>(a, gp, tw, st) : irfft_go<float, double>(a, gp, tw, st);
  return irfft_go<float, float>(a, gp, tw, st);
}

}  // namespace ftm
