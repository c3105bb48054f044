// Batched real FFTs over time (phases 1+2 and 4+5) for transform lengths
// whose plan is fixed at compile time, for gfx950.  This file is compiled once
// per length N (FTM_FIXED_N); ftm_fft.hip dispatches to it when the operator's
// plan is the one compiled here and runs the runtime-plan kernels otherwise.
//
// Two real series (adjacent columns) share one complex transform of length N,
// one as the real part and one as the imaginary part, and are separated with
// the conjugate symmetry of real spectra.  Each transform is a self-sorting
// mixed-radix Stockham FFT (Govindaraju et al., SC'08) run by T threads:
// every pass reads R points at stride N/R, applies the twiddles, does an
// R-point DFT in registers and writes the R results in sorted order.  With
// the plan fixed, every stride, butterfly count and twiddle offset is a
// constant.  The passes exchange data through the transform's own LDS slab;
// when a transform fits in one wave (T <= 64) the exchanges rely on the
// wave's in-order LDS accesses and need no workgroup barrier.
//
// A workgroup owns a tile of C adjacent columns (C/2 transforms).  It loads
// the tile's rows t < Nt with coalesced row segments into the transforms'
// slabs, and writes the tile's output rows the same way from the slabs, so
// every global access moves whole C-column row segments; in between, each
// transform runs its passes on its own slab.  The forward transform's first
// pass never reads the zero padding (inputs that can only be padding are
// zero constants), and its last pass pairs the butterflies j and N/R - j in
// one thread, so that the bins k and N - k that the separation combines meet
// in registers.  The inverse transform mirrors it: its first pass pairs
// butterflies so that each stored bin fills both its own slot and its
// mirror's (the Hermitian extension).  The forward plan lists its radices in
// descending order and the inverse plan in ascending order, so the paired
// passes take the smallest radix.  Twiddles come from the operator's per-pass
// tables (long double on the host, rounded once).
#include <algorithm>
#include <type_traits>

#include "ftm_device.h"
#include "ftm_dft.h"
#include "ftm_kernels.h"

#ifndef FTM_FIXED_N
#error "compile with -DFTM_FIXED_N=<transform length>"
#endif

namespace ftm {
namespace {

// LDS slot of complex element i of a slab: one unused slot after every 16
// elements spreads the strided accesses of the passes over the banks (lanes
// j writing j R + q, R = 16, meet 17 j + q, distinct banks), and for strides
// that are multiples of 16 the slots of a butterfly's R points are one base
// plus constants, which the LDS instructions take as immediate offsets.
__device__ __forceinline__ int lds_ix(int i) { return i + (i >> 4); }
constexpr int lds_size(int n) { return (n + (n >> 4) + 1 + 15) / 16 * 16; }
// Slot of element base + q STRIDE: for STRIDE a multiple of 16, the base's
// slot plus a constant (the compiler does not find this by itself).
template <int STRIDE>
__device__ __forceinline__ int lds_at(int base, int q) {
  if constexpr (STRIDE % 16 == 0) return lds_ix(base) + q * (STRIDE + STRIDE / 16);
  else return lds_ix(base + q * STRIDE);
}
// Slot of element base + q (q < R) for a base that is a multiple of R: for R
// dividing 16 the run stays inside one group of 16.
template <int R>
__device__ __forceinline__ int lds_run(int base, int q) {
  if constexpr (16 % R == 0) return lds_ix(base) + q;
  else return lds_ix(base + q);
}

// A plan fixed at compile time: passes of radix Rs... (product N).  Pass s
// runs after Ns(s) = rad[0] * .. * rad[s-1] points are combined and reads its
// twiddles exp(-2 pi i q jm / (Ns R)) at toff(s) + jm R + q of the operator's
// table for this plan.
template <int... Rs>
struct CPlan {
  static constexpr int nst = sizeof...(Rs);
  static constexpr int rad[nst] = {Rs...};
  static constexpr int N = (Rs * ...);
  static constexpr int ns(int s) {
    int p = 1;
    for (int i = 0; i < s; ++i) p *= rad[i];
    return p;
  }
  static constexpr int toff(int s) {
    int o = 0;
    for (int i = 0; i < s; ++i) o += ns(i + 1);
    return o;
  }
};

// Order the LDS accesses of the threads of one transform: a wave-level fence
// when the transform lives in one wave (its LDS accesses complete in issue
// order), a workgroup barrier otherwise.
template <int T>
__device__ __forceinline__ void tsync() {
  if constexpr (T <= 64) {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  } else {
    __syncthreads();
  }
}

// Twiddles of pass S for this thread's butterflies, held in registers.  For
// lengths of 1024 and more they are loaded one pass ahead (the first
// twiddled pass's during the tile load), so that no pass waits for its
// twiddles' global loads: there the slabs limit a workgroup to 4 waves per
// SIMD, which leaves the registers free (64-right-hand-side transforms at
// length 1024: 3-8% faster).  Shorter transforms run more waves, which the
// extra registers would cost, and load each pass's twiddles just before it.
template <class P>
constexpr bool tw_ahead() { return P::N >= 1024; }

// Forward transforms with half-precision rounding turn the launch's uniform
// formats into compile-time constants where they round (the bin separation,
// and the tile load when the pad phase is float64): one branch per thread
// instead of a format switch per value (64-right-hand-side forward
// transforms at length 1024 with BF16 rounding 15-18% faster).  Only for
// lengths of 1024 and more: shorter transforms would lose occupancy to the
// extra code paths' registers.  The inverse transforms, less bound by their
// vector instructions, gained nothing from it and keep the switch.
template <class P, bool HALF>
constexpr bool fixed_formats() { return HALF && P::N >= 1024; }

// with_round for kernels without half formats (every format DT_F32 or
// DT_F64): float64 values take one branch between the two instantiations;
// float values are never changed by such a rounding, so one instantiation
// without rounding serves every format.  The forward transform uses it where
// it rounds (measured on float64 transforms at length 1024 with 64
// right-hand sides: 9-11% faster than a select per value).
template <class T, class Fn>
__device__ __forceinline__ void with_round_nohalf(int dt, Fn&& f) {
  if constexpr (std::is_same<T, double>::value) {
    if (dt == DT_F32) {
      f(RoundInto<DT_F32>{});
      return;
    }
  }
  f(RoundInto<DT_F64>{});
}
// Without half formats, a rounding into `first` followed by one into
// `second` equals a single rounding into the coarser of the two.
__device__ __forceinline__ int coarser_nohalf(int first, int second) {
  return first == DT_F32 || second == DT_F32 ? DT_F32 : DT_F64;
}

// get(i, j, q): twiddle q of butterfly j = lane + i T of pass S.
template <class P, int S, int T, class TC, bool AHEAD = tw_ahead<P>()>
struct TwMid {  // registers, filled by load()
  static constexpr int R = P::rad[S], NS = P::ns(S), nb = P::N / R, MB = (nb + T - 1) / T;
  cplx<TC> w[MB][R];  // w[i][0] unused
  __device__ __forceinline__ void load(const cplx<TC>* __restrict__ tw, int lane) {
    const cplx<TC>* tws = tw + P::toff(S);
#pragma unroll
    for (int i = 0; i < MB; ++i) {
      const int j = lane + i * T;
      if (nb % T == 0 || j < nb) {
        const int jm = NS == nb ? j : j % NS;
#pragma unroll
        for (int q = 1; q < R; ++q) w[i][q] = tws[jm * R + q];
      }
    }
  }
  __device__ __forceinline__ cplx<TC> get(int i, int, int q) const { return w[i][q]; }
};
template <class P, int S, int T, class TC>
struct TwMid<P, S, T, TC, false> {  // loaded where the pass uses them
  static constexpr int R = P::rad[S], NS = P::ns(S), nb = P::N / R;
  const cplx<TC>* tws;
  __device__ __forceinline__ void load(const cplx<TC>* __restrict__ tw, int) { tws = tw + P::toff(S); }
  __device__ __forceinline__ cplx<TC> get(int, int j, int q) const { return tws[(NS == nb ? j : j % NS) * R + q]; }
};

// A middle pass S of plan P: butterfly j = lane + i T < N/R reads points
// j + q N/R, twiddles them, and writes its DFT to (j - jm) R + jm + q Ns with
// jm = j mod Ns.  All reads precede all writes (the pass works in place).
template <class P, int S, int T, class TC>
__device__ __forceinline__ void mid_pass(cplx<TC>* lds, int lane, const TwMid<P, S, T, TC>& tw) {
  constexpr int R = P::rad[S], NS = P::ns(S), nb = P::N / R, MB = (nb + T - 1) / T;
  cplx<TC> v[MB][R];
#pragma unroll
  for (int i = 0; i < MB; ++i) {
    const int j = lane + i * T;
    if (nb % T == 0 || j < nb) {
      v[i][0] = lds[lds_ix(j)];
#pragma unroll
      for (int q = 1; q < R; ++q) v[i][q] = cmul(lds[lds_at<nb>(j, q)], tw.get(i, j, q));
    }
  }
  tsync<T>();
#pragma unroll
  for (int i = 0; i < MB; ++i) {
    const int j = lane + i * T;
    if (nb % T == 0 || j < nb) {
      dft<R>(v[i]);
      const int jm = j % NS, dst = (j - jm) * R + jm;
#pragma unroll
      for (int q = 0; q < R; ++q) lds[lds_at<NS>(dst, q)] = v[i][q];
    }
  }
  tsync<T>();
}


// Paired passes (a pass with nb = N/R butterflies whose outputs or inputs are
// needed in conjugate pairs) run in units u < (nb + 1) / 2: unit 0 holds
// butterfly 0 (whose output q pairs with its own output (R - q) mod R) and,
// for even nb, butterfly nb/2 (output q pairs with its own output R-1-q);
// unit u > 0 holds butterflies u and nb - u (output q of each pairs with
// output R-1-q of the other).  With nb/2 units for even nb, a pass fits T
// threads exactly when the other passes do.
template <int nb>
__device__ __forceinline__ int partner_butterfly(int u) { return u == 0 ? nb / 2 : nb - u; }
template <int nb>
__device__ __forceinline__ bool has_second(int u) { return u != 0 || nb % 2 == 0; }

// ---- phases 1+2: pad (+round) + real FFT -------------------------------------

// First pass from the slab, where the tile load left rows t < Nt.  As
// L >= 2 Nt, only q < (R + 1) / 2 can reach such a row: the other inputs are
// zero constants.  In place: all reads precede all writes.
template <class P, int T, class TC>
__device__ __forceinline__ void rfft_first(cplx<TC>* lds, int Nt, int lane) {
  constexpr int R = P::rad[0], nb = P::N / R, MB = (nb + T - 1) / T, QL = (R + 1) / 2;
  static_assert(QL * nb >= P::N / 2, "inputs below N/2 reach a pruned slot");
  cplx<TC> v[MB][R];
#pragma unroll
  for (int i = 0; i < MB; ++i) {
    const int j = lane + i * T;
#pragma unroll
    for (int q = 0; q < R; ++q) {
      v[i][q] = {(TC)0, (TC)0};
      if (q < QL && (nb % T == 0 || j < nb) && j + q * nb < Nt) v[i][q] = lds[lds_at<nb>(j, q)];
    }
  }
  tsync<T>();
#pragma unroll
  for (int i = 0; i < MB; ++i) {
    const int j = lane + i * T;
    if (nb % T == 0 || j < nb) {
      dft<R>(v[i]);
#pragma unroll
      for (int q = 0; q < R; ++q) lds[lds_run<R>(j * R, q)] = v[i][q];
    }
  }
  tsync<T>();
}

// Bin k of both real series from Z_k and Z_{N-k}, rounded to the FFT format
// and then to r_next (the next phase's, or DT_F64 when that is the same): X = (Z_k + conj Z_{N-k}) / 2 goes to the
// slot of element k, Y = (Z_k - conj Z_{N-k}) / 2i to that of N/2 + 1 + k.
template <class TC, class RF, class RN>
__device__ __forceinline__ void sep_bin(cplx<TC>* lds, int slot_x, int slot_y, cplx<TC> zk, cplx<TC> zr, RF r_fft,
                                        RN r_next) {
  cplx<TC> X = {(TC)0.5 * (zk.x + zr.x), (TC)0.5 * (zk.y - zr.y)};
  cplx<TC> Y = {(TC)0.5 * (zk.y + zr.y), (TC)0.5 * (zr.x - zk.x)};
  lds[slot_x] = r_next(r_fft(X));
  lds[slot_y] = r_next(r_fft(Y));
}

// Last pass (Ns = nb, so jm = j) in paired units; the separated bins
// k <= N/2 of both series replace the transform in its slab.  All reads
// precede all writes.
// Twiddles of the forward transform's last pass in paired units: get1 / get2
// give twiddle q of butterflies j1 and j2 of unit lane + i T.
template <class P, int T, class TC, bool AHEAD = tw_ahead<P>()>
struct TwLast {
  static constexpr int S = P::nst - 1, R = P::rad[S], nb = P::N / R, nu = (nb + 1) / 2, MU = (nu + T - 1) / T;
  cplx<TC> w1[MU][R], w2[MU][R];  // [.][0] unused
  __device__ __forceinline__ cplx<TC> get1(int i, int, int q) const { return w1[i][q]; }
  __device__ __forceinline__ cplx<TC> get2(int i, int, int q) const { return w2[i][q]; }
  __device__ __forceinline__ void load(const cplx<TC>* __restrict__ tw, int lane) {
    const cplx<TC>* tws = tw + P::toff(S);
#pragma unroll
    for (int i = 0; i < MU; ++i) {
      const int u = lane + i * T;
      if (nu % T != 0 && u >= nu) continue;
      const int j1 = u, j2 = partner_butterfly<nb>(u);
#pragma unroll
      for (int q = 1; q < R; ++q) w1[i][q] = tws[j1 * R + q];
      if (has_second<nb>(u)) {
#pragma unroll
        for (int q = 1; q < R; ++q) w2[i][q] = tws[j2 * R + q];
      }
    }
  }
};
template <class P, int T, class TC>
struct TwLast<P, T, TC, false> {
  static constexpr int S = P::nst - 1, R = P::rad[S];
  const cplx<TC>* tws;
  __device__ __forceinline__ void load(const cplx<TC>* __restrict__ tw, int) { tws = tw + P::toff(S); }
  __device__ __forceinline__ cplx<TC> get1(int, int j1, int q) const { return tws[j1 * R + q]; }
  __device__ __forceinline__ cplx<TC> get2(int, int j2, int q) const { return tws[j2 * R + q]; }
};

// r_fft and r_next are rounding function objects (formats fixed at compile
// time for kernels with half-precision rounding).
template <class P, int T, class TC, class RF, class RN>
__device__ __forceinline__ void rfft_last(cplx<TC>* lds, int lane, const TwLast<P, T, TC>& tw, RF r_fft,
                                          RN r_next) {
  constexpr int S = P::nst - 1, R = P::rad[S], N = P::N, nb = N / R, nu = (nb + 1) / 2, hN = N / 2;
  constexpr int MU = (nu + T - 1) / T;
  cplx<TC> v1[MU][R], v2[MU][R];
#pragma unroll
  for (int i = 0; i < MU; ++i) {
    const int u = lane + i * T;
    if (nu % T != 0 && u >= nu) continue;
    const int j1 = u, j2 = partner_butterfly<nb>(u);
    v1[i][0] = lds[lds_ix(j1)];
#pragma unroll
    for (int q = 1; q < R; ++q) v1[i][q] = cmul(lds[lds_at<nb>(j1, q)], tw.get1(i, j1, q));
    if (has_second<nb>(u)) {
      v2[i][0] = lds[lds_ix(j2)];
#pragma unroll
      for (int q = 1; q < R; ++q) v2[i][q] = cmul(lds[lds_at<nb>(j2, q)], tw.get2(i, j2, q));
    }
  }
  tsync<T>();
#pragma unroll
  for (int i = 0; i < MU; ++i) {
    const int u = lane + i * T;
    if (nu % T != 0 && u >= nu) continue;
    const int j1 = u, j2 = partner_butterfly<nb>(u);
    dft<R>(v1[i]);
    if (has_second<nb>(u)) dft<R>(v2[i]);
    if (u == 0) {
#pragma unroll
      for (int q = 0; q < R; ++q)
        if (q * nb <= hN)
          sep_bin(lds, lds_at<nb>(0, q), lds_at<nb>(hN + 1, q), v1[i][q], v1[i][(R - q) % R], r_fft, r_next);
      if constexpr (nb % 2 == 0) {
#pragma unroll
        for (int q = 0; q < R; ++q)
          if (j2 + q * nb <= hN)
            sep_bin(lds, lds_at<nb>(j2, q), lds_at<nb>(hN + 1 + j2, q), v2[i][q], v2[i][R - 1 - q], r_fft,
                          r_next);
      }
    } else {
#pragma unroll
      for (int q = 0; q < R; ++q) {
        if (j1 + q * nb <= hN)
          sep_bin(lds, lds_at<nb>(j1, q), lds_at<nb>(hN + 1 + j1, q), v1[i][q], v2[i][R - 1 - q], r_fft,
                        r_next);
        if (j2 + q * nb <= hN)
          sep_bin(lds, lds_at<nb>(j2, q), lds_at<nb>(hN + 1 + j2, q), v2[i][q], v1[i][R - 1 - q], r_fft,
                        r_next);
      }
    }
  }
}

// Passes S .. nst-1 of the forward transform; w holds pass S's twiddles and
// pass S + 1's are loaded before pass S runs.
template <class P, int S, int T, class TC>
using RfftTw = typename std::conditional<S == P::nst - 1, TwLast<P, T, TC>, TwMid<P, S, T, TC>>::type;

template <class P, int S, int T, bool HALF, class TC>
__device__ __forceinline__ void rfft_passes(cplx<TC>* lds, int lane, const cplx<TC>* __restrict__ tw,
                                            const RfftTw<P, S, T, TC>& w, int r_fft, int r_next) {
  if constexpr (S == P::nst - 1) {
    if constexpr (fixed_formats<P, HALF>()) {
      with_round<TC>(r_fft, [&](auto rf) {
        with_round<TC>(r_next, [&](auto rn) { rfft_last<P, T>(lds, lane, w, rf, rn); });
      });
    } else if constexpr (HALF) {
      rfft_last<P, T>(lds, lane, w, RoundAnyFormat{r_fft}, RoundAnyFormat{r_next});
    } else {
      with_round_nohalf<TC>(coarser_nohalf(r_fft, r_next),
                            [&](auto r) { rfft_last<P, T>(lds, lane, w, r, RoundInto<DT_F64>{}); });
    }
  } else {
    RfftTw<P, S + 1, T, TC> wn;
    if constexpr (tw_ahead<P>()) wn.load(tw, lane);
    mid_pass<P, S, T>(lds, lane, w);
    if constexpr (!tw_ahead<P>()) wn.load(tw, lane);
    rfft_passes<P, S + 1, T, HALF>(lds, lane, tw, wn, r_fft, r_next);
  }
}

// Slab of transform `slot`: N + 2 complex values (the separated bins of both
// series need N + 2), rounded up to 16, plus 2, so that consecutive slabs
// start 4 (float) or 8 (float64) banks apart: the lanes of a tile load or
// store walk across the slabs of one row and then meet distinct banks.
template <int N>
constexpr int slab_size() { return lds_size(N + 2) + 2; }

// A tile of C columns (C/2 transforms of T threads) per workgroup.
template <class P, class TC, class TO, bool HALF, int T, int C>
__global__ __launch_bounds__(C / 2 * T) void rfft_fixed_kernel(RfftArgs a, const cplx<TC>* __restrict__ tw,
                                                               int64_t ntile) {
  constexpr int N = P::N, WG = C / 2 * T, SL = slab_size<N>(), ROWS = WG / C;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  cplx<TC>* slabs = reinterpret_cast<cplx<TC>*>(smem_raw);
  static_assert(P::nst >= 2, "a fixed plan has at least two passes");
  const int64_t wg = xcd_order(blockIdx.x, gridDim.x);
  const int64_t b = wg / ntile, s0 = (wg - b * ntile) * C;
  const int tid = threadIdx.x, Nt = a.Nt;
  RfftTw<P, 1, T, TC> w1;  // the first twiddled pass's, in flight during the tile load
  if constexpr (tw_ahead<P>()) w1.load(tw, tid % T);

  // tile load: thread tid takes column c = tid mod C of rows tid / C + n ROWS
  // (row-contiguous input), or, when time is the contiguous axis (a setup
  // layout with series along memory), column tid / (WG / C) of rows
  // tid mod (WG / C) + n WG / C; both series of a transform share its slab
  // (real and imaginary parts)
  {
    constexpr int TPC = WG / C;  // threads per column in the time-contiguous mapping
    const bool tmajor = a.x_row_stride == 1 && a.S > 1;
    const int c = tmajor ? tid / TPC : tid % C;
    const int t_first = tmajor ? tid % TPC : tid / C, t_step = tmajor ? TPC : ROWS;
    const int64_t s = s0 + c;
    const bool live = s < a.S;
    const double* xb = a.xptr ? a.xptr[b] : a.x + b * a.x_rhs_stride;
    int64_t off = 0;
    if (live) {
      const int64_t rr = a.ncol >= a.S ? 0 : s / a.ncol;
      off = rr * a.x_sr + (s - rr * a.ncol) * a.x_sc;
    }
    const double* xs = xb + off;
    TC* comp = reinterpret_cast<TC*>(slabs + (c / 2) * SL) + (c & 1);
    constexpr int U = 16;  // loads in flight per thread (a whole tile for most shapes)
    // whole tiles of contiguous columns on 16-byte aligned rows: columns 2j
    // and 2j + 1 are the real and imaginary parts of transform j, so one
    // 16-byte load fills a slot of its slab (float32 transforms: 64-vector
    // transforms 21-24% faster; float64 ones measured 2% slower with it)
    constexpr bool can_pair = std::is_same<TC, float>::value;
    const bool paired = can_pair && !tmajor && a.x_sc == 1 && a.ncol >= a.S && s0 + C <= a.S &&
                        (a.x_row_stride & 1) == 0 && (reinterpret_cast<uintptr_t>(xb + s0) & 15) == 0;
    auto load_tile = [&](auto r_pad, auto r_fft) {
      if (can_pair && paired) {
        constexpr int PR = WG / (C / 2), UP = U / 2;  // rows per pass, loads in flight
        const int j = tid % (C / 2);
        const double* xp = xb + s0 + 2 * j;
        cplx<TC>* slab = slabs + j * SL;
        for (int t0 = tid / (C / 2); t0 < Nt; t0 += UP * PR) {
          double2 v[UP];
#pragma unroll
          for (int u = 0; u < UP; ++u) {
            const int t = t0 + u * PR;
            v[u] = t < Nt ? *reinterpret_cast<const double2*>(xp + (int64_t)t * a.x_row_stride) : make_double2(0.0, 0.0);
          }
#pragma unroll
          for (int u = 0; u < UP; ++u) {
            const int t = t0 + u * PR;
            if (t < Nt) slab[lds_ix(t)] = {(TC)r_fft(r_pad(v[u].x)), (TC)r_fft(r_pad(v[u].y))};
          }
        }
        return;
      }
      for (int t0 = t_first; t0 < Nt; t0 += U * t_step) {
        double v[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
          const int t = t0 + u * t_step;
          v[u] = (live && t < Nt) ? xs[(int64_t)t * a.x_row_stride] : 0.0;
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
          const int t = t0 + u * t_step;
          if (t < Nt) comp[2 * lds_ix(t)] = (TC)r_fft(r_pad(v[u]));
        }
      }
    };
    const int r_fft2 = then_round(a.r_pad, a.r_fft);
    if constexpr (fixed_formats<P, HALF>()) {
      // a float64 pad phase (the input's own format) with the transform's
      // rounding fixed; other pad formats keep the switch (their fixed
      // instantiations measured slower: 0.48 -> 0.68 ms with FP32 padding)
      if (a.r_pad == DT_F64)
        with_round<double>(r_fft2, [&](auto rf) { load_tile(RoundInto<DT_F64>{}, rf); });
      else
        load_tile(RoundAnyFormat{a.r_pad}, RoundAnyFormat{r_fft2});
    } else if constexpr (HALF) {
      load_tile(RoundAnyFormat{a.r_pad}, RoundAnyFormat{r_fft2});
    } else {
      // the pad and transform roundings collapse into one (a float32
      // transform's cast alone gives it)
      with_round_nohalf<TC>(coarser_nohalf(a.r_pad, a.r_fft), [&](auto r) { load_tile(RoundInto<DT_F64>{}, r); });
    }
  }
  __syncthreads();
  {
    const int slot = tid / T, lane = tid % T;
    cplx<TC>* lds = slabs + slot * SL;
    rfft_first<P, T>(lds, Nt, lane);
    if constexpr (!tw_ahead<P>()) w1.load(tw, lane);
    // without a half format, float32 storage holds values rounded into
    // float32 (or coarser): the store's cast applies the separation's rounding
    constexpr bool store_rounds = !HALF && std::is_same<TO, float>::value;
    rfft_passes<P, 1, T, HALF>(lds, lane, tw, w1, store_rounds ? (int)DT_F64 : a.r_fft,
                               store_rounds ? (int)DT_F64 : then_round(a.r_fft, a.r_next));
  }
  __syncthreads();
  // tile store: bins k <= N/2 of column c; columns S .. pad_to-1 of the last
  // tile are the padding the products read (times the spectrum's zero
  // padding) and are written as zeros
  {
    if constexpr (!std::is_same<TO, double>::value) {
      // float32 or 16-bit output, a whole tile of live columns on rows
      // aligned to a pair: one 16- or 8-byte store writes bin k of columns 2j
      // and 2j + 1
      cplx<TO>* ob = reinterpret_cast<cplx<TO>*>(a.out) + b * a.out_rhs_stride + s0;
      constexpr uintptr_t PB = 2 * sizeof(cplx<TO>);  // bytes of a pair
      if (s0 + C <= a.S && a.ncol >= a.S && (a.out_k_stride & 1) == 0 &&
          (reinterpret_cast<uintptr_t>(ob) & (PB - 1)) == 0) {
        constexpr int PR = WG / (C / 2);  // rows per pass
        const int j = tid % (C / 2);
        const cplx<TC>* slab = slabs + j * SL;
        for (int k = tid / (C / 2); k <= N / 2; k += PR) {
          const cplx<TC> z0 = slab[lds_ix(k)], z1 = slab[lds_ix(N / 2 + 1 + k)];
          cplx<TO>* o = ob + 2 * j + (int64_t)k * a.out_k_stride;
          if constexpr (std::is_same<TO, float>::value) {
            *reinterpret_cast<float4*>(o) = make_float4((float)z0.x, (float)z0.y, (float)z1.x, (float)z1.y);
          } else {  // 16 bits, exact in format r_next
            const cplx<h16> h0 = to_store<h16>(z0, a.r_next), h1 = to_store<h16>(z1, a.r_next);
            *reinterpret_cast<uint2*>(o) = make_uint2(h0.x.b | ((uint32_t)h0.y.b << 16),
                                                      h1.x.b | ((uint32_t)h1.y.b << 16));
          }
        }
        return;
      }
    }
    const int c = tid % C;
    const int64_t s = s0 + c;
    if (s >= a.S && s >= a.pad_to) return;
    const cplx<TC>* slab = slabs + (c / 2) * SL;
    const int off = (c & 1) ? N / 2 + 1 : 0;
    cplx<TO>* o;
    if (s < a.S) {
      // one output row per right-hand side, or (the setup transform) row
      // s / ncol of a [Nd][ld_row] block per bin
      const int64_t row = a.ncol >= a.S ? 0 : s / a.ncol;
      o = reinterpret_cast<cplx<TO>*>(a.out) + b * a.out_rhs_stride + row * a.ld_row + (s - row * a.ncol);
    } else {
      o = reinterpret_cast<cplx<TO>*>(a.out) + b * a.out_rhs_stride + s;
    }
    const bool pad = s >= a.S;
    for (int k = tid / C; k <= N / 2; k += ROWS) {
      cplx<TC> z = {(TC)0, (TC)0};
      if (!pad) z = slab[lds_ix(off + k)];
      o[(int64_t)k * a.out_k_stride] = to_store<TO>(z, a.r_next);  // 16-bit: exact in format r_next
    }
  }
}

// ---- phases 4+5: inverse real FFT + scale + unpad ---------------------------

// conj of the Hermitian extension Z = A + iB at a stored bin k (direct) and at
// bin N - k (mirror): the inverse transform is conj(FFT(conj Z)) / N.
template <class TC>
__device__ __forceinline__ cplx<TC> conj_z_direct(cplx<TC> A, cplx<TC> B) { return {A.x - B.y, -(A.y + B.x)}; }
template <class TC>
__device__ __forceinline__ cplx<TC> conj_z_mirror(cplx<TC> A, cplx<TC> B) { return {A.x + B.y, A.y - B.x}; }

// First pass (Ns = 1, no twiddles) in paired units, from the bins the tile
// load left in the slab (series s at slot k, series s + 1 at slot
// N/2 + 1 + k): each stored bin fills its own input slot and its mirror's.
// All reads precede all writes.
template <class P, int T, class TC>
__device__ __forceinline__ void irfft_first(cplx<TC>* lds, int lane) {
  constexpr int R = P::rad[0], N = P::N, nb = N / R, nu = (nb + 1) / 2, hN = N / 2;
  constexpr int MU = (nu + T - 1) / T;
  cplx<TC> v1[MU][R], v2[MU][R];
#pragma unroll
  for (int i = 0; i < MU; ++i) {
    const int u = lane + i * T;
    if (nu % T != 0 && u >= nu) continue;
    const int j1 = u, j2 = partner_butterfly<nb>(u);
#pragma unroll
    for (int q = 0; q < R; ++q) {
      v1[i][q] = {(TC)0, (TC)0};
      v2[i][q] = {(TC)0, (TC)0};
    }
    if (u == 0) {
      // butterfly 0: input q*nb, mirror (R - q)*nb
#pragma unroll
      for (int q = 0; q < R; ++q) {
        const int k = q * nb;
        if (k <= hN) {
          const cplx<TC> A = lds[lds_at<nb>(0, q)], B = lds[lds_at<nb>(hN + 1, q)];
          v1[i][q] = conj_z_direct(A, B);
          if (q != 0) v1[i][(R - q) % R] = conj_z_mirror(A, B);
        }
      }
      // butterfly nb/2: input nb/2 + q*nb, mirror nb/2 + (R-1-q)*nb
      if constexpr (nb % 2 == 0) {
#pragma unroll
        for (int q = 0; q < R; ++q) {
          const int k = j2 + q * nb;
          if (k <= hN) {
            const cplx<TC> A = lds[lds_at<nb>(j2, q)], B = lds[lds_at<nb>(hN + 1 + j2, q)];
            v2[i][q] = conj_z_direct(A, B);
            if (R - 1 - q != q) v2[i][R - 1 - q] = conj_z_mirror(A, B);
          }
        }
      }
    } else {
      // butterflies u and nb - u: the mirror of input q of one is input
      // R-1-q of the other
#pragma unroll
      for (int q = 0; q < R; ++q) {
        const int k = j1 + q * nb;
        if (k <= hN) {
          const cplx<TC> A = lds[lds_at<nb>(j1, q)], B = lds[lds_at<nb>(hN + 1 + j1, q)];
          v1[i][q] = conj_z_direct(A, B);
          v2[i][R - 1 - q] = conj_z_mirror(A, B);
        }
      }
#pragma unroll
      for (int q = 0; q < R; ++q) {
        const int k = j2 + q * nb;
        if (k <= hN) {
          const cplx<TC> A = lds[lds_at<nb>(j2, q)], B = lds[lds_at<nb>(hN + 1 + j2, q)];
          v2[i][q] = conj_z_direct(A, B);
          v1[i][R - 1 - q] = conj_z_mirror(A, B);
        }
      }
    }
  }
  tsync<T>();
#pragma unroll
  for (int i = 0; i < MU; ++i) {
    const int u = lane + i * T;
    if (nu % T != 0 && u >= nu) continue;
    const int j1 = u, j2 = partner_butterfly<nb>(u);
    dft<R>(v1[i]);
#pragma unroll
    for (int q = 0; q < R; ++q) lds[lds_run<R>(j1 * R, q)] = v1[i][q];
    if (has_second<nb>(u)) {
      dft<R>(v2[i]);
#pragma unroll
      for (int q = 0; q < R; ++q) lds[lds_run<R>(j2 * R, q)] = v2[i][q];
    }
  }
  tsync<T>();
}

// Last pass (jm = j): time steps t < Nt of both series, scaled by 1/N and
// rounded by round_out (into the IFFT format, then the unpad format),
// replace the transform in its slab (series s as the real part, s + 1 as the
// imaginary part of slot t).  All reads precede all writes.
template <class P, int T, class TC, class RO>
__device__ __forceinline__ void irfft_last(cplx<TC>* lds, int Nt, int lane, const TwMid<P, P::nst - 1, T, TC>& tw,
                                           RO round_out) {
  constexpr int S = P::nst - 1, R = P::rad[S], N = P::N, nb = N / R, MB = (nb + T - 1) / T;
  const TC inv_n = (TC)(1.0 / (double)N);
  cplx<TC> v[MB][R];
#pragma unroll
  for (int i = 0; i < MB; ++i) {
    const int j = lane + i * T;
    if ((nb % T != 0 && j >= nb) || j >= Nt) continue;
    v[i][0] = lds[lds_ix(j)];
#pragma unroll
    for (int q = 1; q < R; ++q) v[i][q] = cmul(lds[lds_at<nb>(j, q)], tw.get(i, j, q));  // jm = j
  }
  tsync<T>();
#pragma unroll
  for (int i = 0; i < MB; ++i) {
    const int j = lane + i * T;
    if ((nb % T != 0 && j >= nb) || j >= Nt) continue;
    dft<R>(v[i]);
#pragma unroll
    for (int q = 0; q < R; ++q) {
      const int t = j + q * nb;
      if (t < Nt)  // W_t = N conj(y_t), y = a + i b
        lds[lds_at<nb>(j, q)] = {round_out(v[i][q].x * inv_n), round_out(-v[i][q].y * inv_n)};
    }
  }
}

// Passes S .. nst-1 of the inverse transform, with the twiddles of each pass
// loaded one pass ahead as in the forward transform.
template <class P, int S, int T, bool HALF, class TC>
__device__ __forceinline__ void irfft_passes(cplx<TC>* lds, int Nt, int lane, const cplx<TC>* __restrict__ tw,
                                             const TwMid<P, S, T, TC>& w, int r_ifft, int r_unpad) {
  if constexpr (S == P::nst - 1) {
    if constexpr (HALF) {
      irfft_last<P, T>(lds, Nt, lane, w, [=](TC x) {
        return (TC)round_as<true>((double)round_as<true>(x, r_ifft), r_unpad);
      });
    } else {
      // without a half format the two roundings collapse into one, a select
      // per value (an instantiation per format measured slower for float64
      // transforms of float64 input)
      irfft_last<P, T>(lds, Nt, lane, w, RoundNoHalf{coarser_nohalf(r_ifft, r_unpad)});
    }
  } else {
    TwMid<P, S + 1, T, TC> wn;
    if constexpr (tw_ahead<P>()) wn.load(tw, lane);
    mid_pass<P, S, T>(lds, lane, w);
    if constexpr (!tw_ahead<P>()) wn.load(tw, lane);
    irfft_passes<P, S + 1, T, HALF>(lds, Nt, lane, tw, wn, r_ifft, r_unpad);
  }
}

template <class P, class TI, class TC, bool HALF, int T, int C>
__global__ __launch_bounds__(C / 2 * T) void irfft_fixed_kernel(IrfftArgs a, const cplx<TC>* __restrict__ tw,
                                                                int64_t ntile) {
  constexpr int N = P::N, hN = N / 2, WG = C / 2 * T, SL = slab_size<N>(), ROWS = WG / C;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  cplx<TC>* slabs = reinterpret_cast<cplx<TC>*>(smem_raw);
  const int64_t wg = xcd_order(blockIdx.x, gridDim.x);
  const int64_t b = wg / ntile, s0 = (wg - b * ntile) * C;
  const int tid = threadIdx.x, Nt = a.Nt;
  static_assert(P::nst >= 2, "a fixed plan has at least two passes");
  TwMid<P, 1, T, TC> w1;  // the first twiddled pass's, in flight during the tile load
  if constexpr (tw_ahead<P>()) w1.load(tw, tid % T);

  // tile load of bins k <= N/2, which the product's epilogue already rounded
  // into the IFFT format (its next phase's); the imaginary parts of bins 0
  // and N/2 are dropped, as a real inverse transform does
  bool loaded = false;
  constexpr int U = 16;
  if constexpr (std::is_same<TI, float>::value) {
    // float32 input, a whole tile on 16-byte aligned rows: one 16-byte load
    // gives bin k of columns 2j and 2j + 1
    const cplx<float>* ib = reinterpret_cast<const cplx<float>*>(a.in) + b * a.in_rhs_stride + s0;
    if (s0 + C <= a.S && (a.in_k_stride & 1) == 0 && (reinterpret_cast<uintptr_t>(ib) & 15) == 0) {
      constexpr int PR = WG / (C / 2), UP = U / 2;  // rows per pass, loads in flight
      const int j = tid % (C / 2);
      cplx<TC>* slab = slabs + j * SL;
      const cplx<float>* ip = ib + 2 * j;
      for (int k0 = tid / (C / 2); k0 <= hN; k0 += UP * PR) {
        float4 v[UP];
#pragma unroll
        for (int u = 0; u < UP; ++u) {
          const int k = k0 + u * PR;
          v[u] = k <= hN ? *reinterpret_cast<const float4*>(ip + (int64_t)k * a.in_k_stride)
                         : make_float4(0.f, 0.f, 0.f, 0.f);
        }
#pragma unroll
        for (int u = 0; u < UP; ++u) {
          const int k = k0 + u * PR;
          if (k > hN) continue;
          cplx<TC> z0 = {(TC)v[u].x, (TC)v[u].y}, z1 = {(TC)v[u].z, (TC)v[u].w};
          if (k == 0 || k == hN) z0.y = z1.y = (TC)0;
          slab[lds_ix(k)] = z0;
          slab[lds_ix(hN + 1 + k)] = z1;
        }
      }
      loaded = true;
    }
  }
  if (!loaded) {
    const int c = tid % C;
    const bool live = s0 + c < a.S;
    const cplx<TI>* in = reinterpret_cast<const cplx<TI>*>(a.in) + b * a.in_rhs_stride + (live ? s0 + c : 0);
    cplx<TC>* slab = slabs + (c / 2) * SL;
    const int off = (c & 1) ? hN + 1 : 0;
    for (int k0 = tid / C; k0 <= hN; k0 += U * ROWS) {
      cplx<TI> v[U];
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int k = k0 + u * ROWS;
        v[u] = (live && k <= hN) ? in[(int64_t)k * a.in_k_stride] : cplx<TI>{};
      }
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int k = k0 + u * ROWS;
        if (k > hN) continue;
        cplx<TC> z = {(TC)v[u].x, (TC)v[u].y};
        if (k == 0 || k == hN) z.y = (TC)0;
        slab[lds_ix(off + k)] = z;
      }
    }
  }
  __syncthreads();
  {
    const int slot = tid / T, lane = tid % T;
    cplx<TC>* lds = slabs + slot * SL;
    irfft_first<P, T>(lds, lane);
    if constexpr (!tw_ahead<P>()) w1.load(tw, lane);
    irfft_passes<P, 1, T, HALF>(lds, Nt, lane, tw, w1, a.r_ifft, then_round(a.r_ifft, a.r_unpad));
  }
  __syncthreads();
  // tile store: rows t < Nt of column c
  {
    double* yb = a.yptr ? a.yptr[b] : a.y + b * a.y_rhs_stride;
    // whole tiles on 16-byte aligned rows: one 16-byte store writes a slot of
    // slab j, time step t of columns 2j and 2j + 1
    if (s0 + C <= a.S && (a.y_row_stride & 1) == 0 && (reinterpret_cast<uintptr_t>(yb + s0) & 15) == 0) {
      constexpr int PR = WG / (C / 2);  // rows per pass
      const int j = tid % (C / 2);
      const cplx<TC>* slab = slabs + j * SL;
      double* yp = yb + s0 + 2 * j;
      for (int t = tid / (C / 2); t < Nt; t += PR) {
        const cplx<TC> z = slab[lds_ix(t)];
        *reinterpret_cast<double2*>(yp + (int64_t)t * a.y_row_stride) = make_double2((double)z.x, (double)z.y);
      }
      return;
    }
    const int c = tid % C;
    const int64_t s = s0 + c;
    if (s >= a.S) return;
    const TC* src = reinterpret_cast<const TC*>(slabs + (c / 2) * SL) + (c & 1);
    double* y = yb + s;
    for (int t = tid / C; t < Nt; t += ROWS) y[(int64_t)t * a.y_row_stride] = (double)src[2 * lds_ix(t)];
  }
}

// ---- the plans and workgroup shapes compiled for this length -------------------

// Forward plans list the radices in descending order, inverse plans in
// ascending order; float32 transforms take radices up to 16, float64 ones up
// to 8 (a radix-16 float64 pass needs about 130 registers per thread).
#if FTM_FIXED_N == 2000
using PlanF32 = CPlan<16, 5, 5, 5>;
using PlanI32 = CPlan<5, 5, 5, 16>;
using PlanF64 = CPlan<5, 5, 5, 4, 4>;
using PlanI64 = CPlan<4, 4, 5, 5, 5>;
#elif FTM_FIXED_N == 1024
using PlanF32 = CPlan<16, 8, 8>;
using PlanI32 = CPlan<8, 8, 16>;
using PlanF64 = CPlan<8, 8, 4, 4>;
using PlanI64 = CPlan<4, 4, 8, 8>;
#elif FTM_FIXED_N == 512
using PlanF32 = CPlan<8, 8, 8>;
using PlanI32 = CPlan<8, 8, 8>;
using PlanF64 = CPlan<8, 8, 8>;
using PlanI64 = CPlan<8, 8, 8>;
#elif FTM_FIXED_N == 400
using PlanF32 = CPlan<16, 5, 5>;
using PlanI32 = CPlan<5, 5, 16>;
using PlanF64 = CPlan<5, 5, 4, 4>;
using PlanI64 = CPlan<4, 4, 5, 5>;
#elif FTM_FIXED_N == 256
using PlanF32 = CPlan<16, 16>;
using PlanI32 = CPlan<16, 16>;
using PlanF64 = CPlan<8, 8, 4>;
using PlanI64 = CPlan<4, 8, 8>;
#elif FTM_FIXED_N == 128
using PlanF32 = CPlan<16, 8>;
using PlanI32 = CPlan<8, 16>;
using PlanF64 = CPlan<8, 4, 4>;
using PlanI64 = CPlan<4, 4, 8>;
#else
#error "no fixed plan for this FTM_FIXED_N"
#endif
template <class TC>
using PlanF = typename std::conditional<sizeof(TC) == 8, PlanF64, PlanF32>::type;
template <class TC>
using PlanI = typename std::conditional<sizeof(TC) == 8, PlanI64, PlanI32>::type;
static_assert(PlanF32::N == FTM_FIXED_N && PlanI32::N == FTM_FIXED_N && PlanF64::N == FTM_FIXED_N &&
                  PlanI64::N == FTM_FIXED_N, "plan length");

// Threads per transform T (a power of two) and columns per tile C.  T gives
// each thread 128 bytes of its transform's slab (8 float64 or 16 float32
// points).  C makes a row segment of the float64 input 128 bytes for float32
// transforms (C = 16) and 64 bytes for float64 ones (C = 8, whose slabs are
// twice as large), within the 1024 threads and the LDS of one workgroup.
// Shape 2 halves C (more, smaller workgroups).
constexpr int pow2_ceil(int x) {
  int p = 1;
  while (p < x) p *= 2;
  return p;
}
template <class TC>
constexpr int threads_per_transform() {
  const int t = pow2_ceil(FTM_FIXED_N * (int)sizeof(cplx<TC>) / 128);
  return t < 16 ? 16 : (t > 256 ? 256 : t);
}
template <class TC>
constexpr int tile_columns(int shape) {
  int c = sizeof(TC) == 8 ? 8 : 16;
  while (c / 2 * threads_per_transform<TC>() > 1024) c /= 2;
  return shape == 2 ? c / 2 : c;
}
template <class P>
bool same_plan(const FftPlan& plan) {
  if (plan.N != P::N || plan.nst != P::nst) return false;
  for (int s = 0; s < P::nst; ++s)
    if (plan.rad[s] != P::rad[s] || plan.toff[s] != P::toff(s)) return false;
  return true;
}

bool is_half(int dt) { return dt == DT_F16 || dt == DT_BF16; }

// Whether the smaller tile is the default: when the larger tile gives fewer
// than 4 tiles per CU (256 CUs), or when its slabs take more than half of a
// CU's 160 KB of LDS, so that one workgroup, which synchronises at every
// pass, would run alone on each CU (length 2000: 64-right-hand-side inverse
// transforms 3.3 -> 2.6 ms in float32).
template <class TC>
bool small_tile(int64_t S, int nrhs) {
  constexpr int C = tile_columns<TC>(1);
  constexpr size_t lds = (size_t)(C / 2) * slab_size<FTM_FIXED_N>() * sizeof(cplx<TC>);
  return lds > 80 * 1024 || (S + C - 1) / C * nrhs < 4 * 256;
}
bool small_tile(int64_t S, int nrhs, bool tc64) {
  return tc64 ? small_tile<double>(S, nrhs) : small_tile<float>(S, nrhs);
}

template <class TC, class TO, int SH>
hipError_t rfft_go(const RfftArgs& a, const void* tw, hipStream_t st) {
  constexpr int T = threads_per_transform<TC>(), C = tile_columns<TC>(SH), WG = C / 2 * T;
  // the tiles cover the padding columns S .. pad_to-1 too (written as zeros)
  const int64_t ntile = (std::max(a.S, a.pad_to) + C - 1) / C;
  const int64_t nwg = ntile * a.nrhs;
  if (nwg <= 0) return hipSuccess;
  if (nwg >= ((int64_t)1 << 31)) return hipErrorInvalidConfiguration;
  const size_t lds = (size_t)(C / 2) * slab_size<FTM_FIXED_N>() * sizeof(cplx<TC>);
  const cplx<TC>* t = reinterpret_cast<const cplx<TC>*>(tw);
  if (is_half(a.r_pad) || is_half(a.r_fft) || is_half(a.r_next))
    hipLaunchKernelGGL((rfft_fixed_kernel<PlanF<TC>, TC, TO, true, T, C>), dim3((unsigned)nwg), dim3(WG), lds, st, a, t,
                       ntile);
  else
    hipLaunchKernelGGL((rfft_fixed_kernel<PlanF<TC>, TC, TO, false, T, C>), dim3((unsigned)nwg), dim3(WG), lds, st, a,
                       t, ntile);
  return hipGetLastError();
}

template <class TI, class TC, int SH>
hipError_t irfft_go(const IrfftArgs& a, const void* tw, hipStream_t st) {
  constexpr int T = threads_per_transform<TC>(), C = tile_columns<TC>(SH), WG = C / 2 * T;
  const int64_t ntile = (a.S + C - 1) / C;
  const int64_t nwg = ntile * a.nrhs;
  if (nwg <= 0) return hipSuccess;
  if (nwg >= ((int64_t)1 << 31)) return hipErrorInvalidConfiguration;
  const size_t lds = (size_t)(C / 2) * slab_size<FTM_FIXED_N>() * sizeof(cplx<TC>);
  const cplx<TC>* t = reinterpret_cast<const cplx<TC>*>(tw);
  if (is_half(a.r_ifft) || is_half(a.r_unpad))
    hipLaunchKernelGGL((irfft_fixed_kernel<PlanI<TC>, TI, TC, true, T, C>), dim3((unsigned)nwg), dim3(WG), lds, st, a,
                       t, ntile);
  else
    hipLaunchKernelGGL((irfft_fixed_kernel<PlanI<TC>, TI, TC, false, T, C>), dim3((unsigned)nwg), dim3(WG), lds, st, a,
                       t, ntile);
  return hipGetLastError();
}

}  // namespace

#define FTM_CAT2(a, b) a##b
#define FTM_CAT(a, b) FTM_CAT2(a, b)

// Forward transform with the plan compiled here; false (nothing launched) when
// the operator's plan differs.  shape: 1 the larger tile, 2 the smaller, 0
// the larger unless it gives fewer than 4 tiles per CU (the smaller tile then
// spreads the transform over more workgroups; measured faster at such sizes).
bool FTM_CAT(launch_rfft_fixed_, FTM_FIXED_N)(bool tc64, int out_st, const RfftArgs& a, const FftPlan& plan,
                                                const void* tw, int shape, hipStream_t st, hipError_t* err) {
  if (!(tc64 ? same_plan<PlanF64>(plan) : same_plan<PlanF32>(plan))) return false;
  const bool alt = shape == 2 || (shape == 0 && small_tile(a.S, a.nrhs, tc64));
#define FTM_RGO(TC, TO) *err = alt ? rfft_go<TC, TO, 2>(a, tw, st) : rfft_go<TC, TO, 1>(a, tw, st)
  if (tc64) {
    if (out_st == ST_F64) FTM_RGO(double, double);
    else if (out_st == ST_16) FTM_RGO(double, h16);
    else FTM_RGO(double, float);
  } else {
    if (out_st == ST_16) FTM_RGO(float, h16);
    else FTM_RGO(float, float);
  }
#undef FTM_RGO
  return true;
}

bool FTM_CAT(launch_irfft_fixed_, FTM_FIXED_N)(int in_st, bool tc64, const IrfftArgs& a, const FftPlan& plan,
                                                 const void* tw, int shape, hipStream_t st, hipError_t* err) {
  if (!(tc64 ? same_plan<PlanI64>(plan) : same_plan<PlanI32>(plan))) return false;
  const bool alt = shape == 2 || (shape == 0 && small_tile(a.S, a.nrhs, tc64));
#define FTM_IGO(TI, TC) *err = alt ? irfft_go<TI, TC, 2>(a, tw, st) : irfft_go<TI, TC, 1>(a, tw, st)
  if (in_st == ST_16) return false;  // not a storage the inverse transform reads
  if (tc64) {
    if (in_st == ST_F64) FTM_IGO(double, double);
    else FTM_IGO(float, double);
  } else {
    FTM_IGO(float, float);
  }
#undef FTM_IGO
  return true;
}

}  // namespace ftm
