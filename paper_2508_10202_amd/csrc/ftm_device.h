// Device-side helpers shared by the FFT and GEMV kernels: complex arithmetic,
// the storage formats of each precision, round-to-nearest-even into a format,
// and the XCD-aware workgroup order used by every streaming kernel.
#pragma once

#include <hip/hip_fp16.h>
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <type_traits>

#ifndef FTM_STREAM_NT
#define FTM_STREAM_NT 1
#endif

namespace ftm {

enum : int { DT_F64 = 0, DT_F32 = 1, DT_F16 = 2, DT_BF16 = 3 };

template <class T>
struct alignas(2 * sizeof(T)) cplx {
  T x, y;
};

template <class T>
__device__ __forceinline__ cplx<T> cadd(cplx<T> a, cplx<T> b) { return {a.x + b.x, a.y + b.y}; }
template <class T>
__device__ __forceinline__ cplx<T> csub(cplx<T> a, cplx<T> b) { return {a.x - b.x, a.y - b.y}; }
template <class T>
__device__ __forceinline__ cplx<T> cmul(cplx<T> a, cplx<T> b) {
  return {a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x};
}
// -i * a  (multiplication by the forward-transform quarter turn)
template <class T>
__device__ __forceinline__ cplx<T> mul_mi(cplx<T> a) { return {a.y, -a.x}; }
template <class T>
__device__ __forceinline__ cplx<T> cscale(cplx<T> a, T s) { return {a.x * s, a.y * s}; }

// ---------------------------------------------------------------------------
// Round-to-nearest-even into the storage formats, branch free.
//   float -> FP16: the hardware conversion (round to nearest even, subnormal
//   results kept, overflow to infinity) and back.
//   float -> BF16: the hardware conversion (v_cvt_pk_bf16_f32: round to
//   nearest even, subnormal results kept, overflow to infinity, NaN stays
//   NaN) and back (BF16 is the top half of a float).
//   double -> FP16/BF16: round to odd into float first (truncate, then set the
//   last bit if anything was dropped), then to nearest even: with float's 24
//   bits at least two more than the target's, the two steps give the direct
//   rounding (Boldo and Melquiond, IEEE TC 2008).
__device__ __forceinline__ float round_f16(float x) { return __half2float(__float2half_rn(x)); }
__device__ __forceinline__ float round_bf16(float x) { return (float)(__bf16)x; }
__device__ __forceinline__ float to_float_odd(double x) {
  const float f = (float)x;
  const double df = (double)f;
  uint32_t u = __float_as_uint(f);
  if (df != x && x == x) {
    u -= fabs(df) > fabs(x) ? 1u : 0u;  // rounded away from zero: step back to the truncation
    u |= 1u;                            // sticky: something was dropped
  }
  return __uint_as_float(u);
}

// Value of x after storage in format dt (a value of the same C type).  dt is
// uniform across a launch, so the switch is a scalar branch and only one
// format's rounding runs.
__device__ __forceinline__ double round_to(double x, int dt) {
  switch (dt) {
    case DT_F32: return (double)(float)x;
    case DT_F16: return (double)round_f16(to_float_odd(x));
    case DT_BF16: return (double)round_bf16(to_float_odd(x));
    default: return x;
  }
}
__device__ __forceinline__ float round_to(float x, int dt) {
  switch (dt) {
    case DT_F16: return round_f16(x);
    case DT_BF16: return round_bf16(x);
    default: return x;
  }
}
template <class T>
__device__ __forceinline__ cplx<T> round_to(cplx<T> a, int dt) {
  return {round_to(a.x, dt), round_to(a.y, dt)};
}

// round_to for kernels that know at compile time whether any format they apply
// is a half format (HALF); without one the rounding is a select (float64
// values into float32) or nothing (float32 values), with no branches.
template <bool HALF>
__device__ __forceinline__ double round_as(double x, int dt) {
  if constexpr (HALF) return round_to(x, dt);
  else return dt == DT_F32 ? (double)(float)x : x;
}
template <bool HALF>
__device__ __forceinline__ float round_as(float x, int dt) {
  if constexpr (HALF) return round_to(x, dt);
  else return x;
}
template <bool HALF, class T>
__device__ __forceinline__ cplx<T> round_as(cplx<T> a, int dt) {
  return {round_as<HALF>(a.x, dt), round_as<HALF>(a.y, dt)};
}

// Rounding into a format fixed at compile time: RoundInto<DT>{}(x) equals
// round_to(x, DT) (DT_F64 rounds nothing; DT_F32 nothing for float values).
template <int DT>
struct RoundInto {
  __device__ __forceinline__ float operator()(float x) const { return round_to(x, DT); }
  __device__ __forceinline__ double operator()(double x) const { return round_to(x, DT); }
  template <class T>
  __device__ __forceinline__ cplx<T> operator()(cplx<T> a) const {
    return {(*this)(a.x), (*this)(a.y)};
  }
};
// round_as<false> as a function object (no half format: a select at most).
struct RoundNoHalf {
  int dt;
  __device__ __forceinline__ float operator()(float x) const { return round_as<false>(x, dt); }
  __device__ __forceinline__ double operator()(double x) const { return round_as<false>(x, dt); }
  template <class T>
  __device__ __forceinline__ cplx<T> operator()(cplx<T> a) const {
    return {(*this)(a.x), (*this)(a.y)};
  }
};
// round_as<true> as a function object (a format switch per value).
struct RoundAnyFormat {
  int dt;
  __device__ __forceinline__ float operator()(float x) const { return round_to(x, dt); }
  __device__ __forceinline__ double operator()(double x) const { return round_to(x, dt); }
  template <class T>
  __device__ __forceinline__ cplx<T> operator()(cplx<T> a) const {
    return {(*this)(a.x), (*this)(a.y)};
  }
};
// with_round<T>(dt, f) calls f(RoundInto<dt>{}) for values of type T, with
// the uniform format dt turned into a compile-time constant by one branch,
// so that the caller's loop holds no per-value format switch.  For float
// values DT_F32 and DT_F64 share one instantiation (no rounding).
template <class T, class Fn>
__device__ __forceinline__ void with_round(int dt, Fn&& f) {
  switch (dt) {
    case DT_F16: f(RoundInto<DT_F16>{}); break;
    case DT_BF16: f(RoundInto<DT_BF16>{}); break;
    case DT_F32:
      if constexpr (std::is_same<T, double>::value) {
        f(RoundInto<DT_F32>{});
        break;
      }
      [[fallthrough]];
    default: f(RoundInto<DT_F64>{}); break;
  }
}

// Format of a second rounding that follows one into `first`: rounding into
// the same format again cannot change the value, so it becomes DT_F64, which
// round_to and round_as treat as no rounding (a uniform value: the rounding
// is skipped by a scalar branch).
__device__ __forceinline__ int then_round(int first, int second) { return second == first ? DT_F64 : second; }

// ---------------------------------------------------------------------------
// 16-bit storage of a transformed vector between two phases, in FP16 or BF16
// (the format is a launch argument).  Only values exact in that format are
// stored, so the conversion is exact.
struct h16 {
  uint16_t b;
};
__device__ __forceinline__ h16 to_h16(float v, int dt) {
  return {dt == DT_BF16 ? (uint16_t)(__float_as_uint(v) >> 16) : __half_as_ushort(__float2half_rn(v))};
}
__device__ __forceinline__ h16 to_h16(double v, int dt) { return to_h16((float)v, dt); }
// a complex value of type T stored as cplx<TS> (TS = h16: in format dt)
template <class TS, class T>
__device__ __forceinline__ cplx<TS> to_store(cplx<T> v, int dt) {
  if constexpr (std::is_same<TS, h16>::value) return {to_h16(v.x, dt), to_h16(v.y, dt)};
  else return {(TS)v.x, (TS)v.y};
}

// ---------------------------------------------------------------------------
// Storage formats of the spectrum.  Each tag names the element stored per
// complex number and how many complex numbers one 16-byte load carries.
struct s_f64 {
  using elem = cplx<double>;
  static constexpr int V = 1;
};
struct s_f32 {
  using elem = cplx<float>;
  static constexpr int V = 2;
};
struct h2 {
  uint16_t x, y;
};
struct s_f16 {
  using elem = h2;
  static constexpr int V = 4;
};
struct s_bf16 {
  using elem = h2;
  static constexpr int V = 4;
};

__device__ __forceinline__ float half_bits_to_float(uint16_t b) {
  return __half2float(__ushort_as_half(b));
}
__device__ __forceinline__ float bf16_bits_to_float(uint16_t b) {
  return __uint_as_float(((uint32_t)b) << 16);
}

// Decode the V complex numbers of one 16-byte chunk into accumulation type TA.
template <class S, class TA>
struct Chunk;

template <class TA>
struct Chunk<s_f64, TA> {
  static __device__ __forceinline__ void decode(const uint4& u, cplx<TA>* out) {
    const double2 d = *reinterpret_cast<const double2*>(&u);
    out[0] = {(TA)d.x, (TA)d.y};
  }
};
template <class TA>
struct Chunk<s_f32, TA> {
  static __device__ __forceinline__ void decode(const uint4& u, cplx<TA>* out) {
    out[0] = {(TA)__uint_as_float(u.x), (TA)__uint_as_float(u.y)};
    out[1] = {(TA)__uint_as_float(u.z), (TA)__uint_as_float(u.w)};
  }
};
template <class TA>
struct Chunk<s_f16, TA> {
  static __device__ __forceinline__ void decode(const uint4& u, cplx<TA>* out) {
    const uint32_t w[4] = {u.x, u.y, u.z, u.w};
#pragma unroll
    for (int i = 0; i < 4; ++i)
      out[i] = {(TA)half_bits_to_float(w[i] & 0xffffu), (TA)half_bits_to_float(w[i] >> 16)};
  }
};
template <class TA>
struct Chunk<s_bf16, TA> {
  static __device__ __forceinline__ void decode(const uint4& u, cplx<TA>* out) {
    const uint32_t w[4] = {u.x, u.y, u.z, u.w};
#pragma unroll
    for (int i = 0; i < 4; ++i)
      out[i] = {(TA)__uint_as_float(w[i] << 16), (TA)__uint_as_float(w[i] & 0xffff0000u)};
  }
};

// ---------------------------------------------------------------------------
// 16-byte load of data that is read exactly once (the stored spectrum): a
// non-temporal load keeps it from displacing reused data in the caches and
// streams measurably faster than a plain load on gfx950.
typedef unsigned ftm_v4u __attribute__((ext_vector_type(4)));
__device__ __forceinline__ uint4 load_stream(const void* p) {
#if FTM_STREAM_NT
  const ftm_v4u t = __builtin_nontemporal_load(reinterpret_cast<const ftm_v4u*>(p));
  return make_uint4(t.x, t.y, t.z, t.w);
#else
  return *reinterpret_cast<const uint4*>(p);
#endif
}

// ---------------------------------------------------------------------------
// Workgroups are handed to the 8 XCDs round robin (workgroup i runs on XCD
// i mod 8).  Re-number them so that each XCD works through one contiguous
// range of logical workgroup ids: neighbouring tiles, which share input
// vectors, then meet in the same XCD's L2.
constexpr int NUM_XCD = 8;
__device__ __forceinline__ int xcd_order(int i, int n) {
  const int xcd = i % NUM_XCD, local = i / NUM_XCD;
  const int base = n / NUM_XCD, rem = n % NUM_XCD;
  return xcd < rem ? xcd * (base + 1) + local : rem * (base + 1) + (xcd - rem) * base + local;
}

}  // namespace ftm
