// R-point DFTs (forward sign exp(-2 pi i jk / R)) on complex values held in
// registers, for the Stockham passes of the FFT kernels.
#pragma once

#include "ftm_device.h"

namespace ftm {

// ---- R-point DFTs, forward sign exp(-2 pi i jk / R) --------------------------

template <class T>
__device__ __forceinline__ void dft2(cplx<T>* a) {
  const cplx<T> t = a[1];
  a[1] = csub(a[0], t);
  a[0] = cadd(a[0], t);
}

template <class T>
__device__ __forceinline__ void dft3(cplx<T>* a) {
  const T s3 = (T)0.8660254037844386467637232;  // sin(pi/3)
  const cplx<T> t = cadd(a[1], a[2]);
  const cplx<T> d = cscale(csub(a[1], a[2]), s3);
  const cplx<T> m = {a[0].x - (T)0.5 * t.x, a[0].y - (T)0.5 * t.y};
  a[0] = cadd(a[0], t);
  a[1] = cadd(m, mul_mi(d));
  a[2] = csub(m, mul_mi(d));
}

template <class T>
__device__ __forceinline__ void dft4(cplx<T>* a) {
  const cplx<T> t0 = cadd(a[0], a[2]), t1 = csub(a[0], a[2]);
  const cplx<T> t2 = cadd(a[1], a[3]), t3 = mul_mi(csub(a[1], a[3]));
  a[0] = cadd(t0, t2);
  a[2] = csub(t0, t2);
  a[1] = cadd(t1, t3);
  a[3] = csub(t1, t3);
}

template <class T>
__device__ __forceinline__ void dft5(cplx<T>* a) {
  const T c1 = (T)0.3090169943749474241022934, c2 = (T)-0.8090169943749474241022934;
  const T s1 = (T)0.9510565162951535721164393, s2 = (T)0.5877852522924731291687059;
  const cplx<T> t1 = cadd(a[1], a[4]), t2 = cadd(a[2], a[3]);
  const cplx<T> d1 = csub(a[1], a[4]), d2 = csub(a[2], a[3]);
  const cplx<T> b1 = {a[0].x + c1 * t1.x + c2 * t2.x, a[0].y + c1 * t1.y + c2 * t2.y};
  const cplx<T> b2 = {a[0].x + c2 * t1.x + c1 * t2.x, a[0].y + c2 * t1.y + c1 * t2.y};
  const cplx<T> e1 = {s1 * d1.x + s2 * d2.x, s1 * d1.y + s2 * d2.y};
  const cplx<T> e2 = {s2 * d1.x - s1 * d2.x, s2 * d1.y - s1 * d2.y};
  a[0] = cadd(a[0], cadd(t1, t2));
  a[1] = cadd(b1, mul_mi(e1));
  a[4] = csub(b1, mul_mi(e1));
  a[2] = cadd(b2, mul_mi(e2));
  a[3] = csub(b2, mul_mi(e2));
}

template <class T>
__device__ __forceinline__ void dft7(cplx<T>* a) {
  const T C1 = (T)0.6234898018587335305250049, C2 = (T)-0.2225209339563144042889026,
          C3 = (T)-0.9009688679024191262361023;
  const T S1 = (T)0.7818314824680298087084445, S2 = (T)0.9749279121818236070181317,
          S3 = (T)0.4338837391175581204757683;
  const cplx<T> t1 = cadd(a[1], a[6]), t2 = cadd(a[2], a[5]), t3 = cadd(a[3], a[4]);
  const cplx<T> d1 = csub(a[1], a[6]), d2 = csub(a[2], a[5]), d3 = csub(a[3], a[4]);
  const cplx<T> x0 = a[0];
  // cos(2 pi jk/7) and sin(2 pi jk/7) for j = 1..3 at k = 1, 2, 3
  const cplx<T> b1 = {x0.x + C1 * t1.x + C2 * t2.x + C3 * t3.x, x0.y + C1 * t1.y + C2 * t2.y + C3 * t3.y};
  const cplx<T> b2 = {x0.x + C2 * t1.x + C3 * t2.x + C1 * t3.x, x0.y + C2 * t1.y + C3 * t2.y + C1 * t3.y};
  const cplx<T> b3 = {x0.x + C3 * t1.x + C1 * t2.x + C2 * t3.x, x0.y + C3 * t1.y + C1 * t2.y + C2 * t3.y};
  const cplx<T> e1 = {S1 * d1.x + S2 * d2.x + S3 * d3.x, S1 * d1.y + S2 * d2.y + S3 * d3.y};
  const cplx<T> e2 = {S2 * d1.x - S3 * d2.x - S1 * d3.x, S2 * d1.y - S3 * d2.y - S1 * d3.y};
  const cplx<T> e3 = {S3 * d1.x - S1 * d2.x + S2 * d3.x, S3 * d1.y - S1 * d2.y + S2 * d3.y};
  a[0] = cadd(x0, cadd(t1, cadd(t2, t3)));
  a[1] = cadd(b1, mul_mi(e1));
  a[6] = csub(b1, mul_mi(e1));
  a[2] = cadd(b2, mul_mi(e2));
  a[5] = csub(b2, mul_mi(e2));
  a[3] = cadd(b3, mul_mi(e3));
  a[4] = csub(b3, mul_mi(e3));
}

template <class T>
__device__ __forceinline__ void dft8(cplx<T>* a) {
  const T h = (T)0.7071067811865475244008444;  // sqrt(1/2)
  cplx<T> e[4] = {a[0], a[2], a[4], a[6]};
  cplx<T> o[4] = {a[1], a[3], a[5], a[7]};
  dft4(e);
  dft4(o);
  // o[k] *= exp(-2 pi i k / 8)
  o[1] = {h * (o[1].x + o[1].y), h * (o[1].y - o[1].x)};
  o[2] = mul_mi(o[2]);
  o[3] = {h * (o[3].y - o[3].x), -h * (o[3].x + o[3].y)};
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    a[k] = cadd(e[k], o[k]);
    a[k + 4] = csub(e[k], o[k]);
  }
}

// 16 = 4 x 4: length-4 DFTs over n1 (n = 4 n1 + n2), the twiddles
// exp(-2 pi i n2 k1 / 16), then length-4 DFTs over n2 giving bin k1 + 4 k2.
template <class T>
__device__ __forceinline__ void dft16(cplx<T>* a) {
  const T c1 = (T)0.9238795325112867561281832;  // cos(pi/8)
  const T s1 = (T)0.3826834323650897717284600;  // sin(pi/8)
  const T h = (T)0.7071067811865475244008444;   // sqrt(1/2)
  cplx<T> y[4][4];
#pragma unroll
  for (int n2 = 0; n2 < 4; ++n2) {
    cplx<T> c[4] = {a[n2], a[4 + n2], a[8 + n2], a[12 + n2]};
    dft4(c);
#pragma unroll
    for (int k1 = 0; k1 < 4; ++k1) y[k1][n2] = c[k1];
  }
  // y[k1][n2] *= exp(-2 pi i n2 k1 / 16) for the exponents 1, 2, 3, 4, 6, 9
  y[1][1] = {c1 * y[1][1].x + s1 * y[1][1].y, c1 * y[1][1].y - s1 * y[1][1].x};
  y[2][1] = {h * (y[2][1].x + y[2][1].y), h * (y[2][1].y - y[2][1].x)};
  y[3][1] = {s1 * y[3][1].x + c1 * y[3][1].y, s1 * y[3][1].y - c1 * y[3][1].x};
  y[1][2] = {h * (y[1][2].x + y[1][2].y), h * (y[1][2].y - y[1][2].x)};
  y[2][2] = mul_mi(y[2][2]);
  y[3][2] = {h * (y[3][2].y - y[3][2].x), -h * (y[3][2].x + y[3][2].y)};
  y[1][3] = {s1 * y[1][3].x + c1 * y[1][3].y, s1 * y[1][3].y - c1 * y[1][3].x};
  y[2][3] = {h * (y[2][3].y - y[2][3].x), -h * (y[2][3].x + y[2][3].y)};
  y[3][3] = {-c1 * y[3][3].x - s1 * y[3][3].y, s1 * y[3][3].x - c1 * y[3][3].y};
#pragma unroll
  for (int k1 = 0; k1 < 4; ++k1) {
    dft4(y[k1]);
#pragma unroll
    for (int k2 = 0; k2 < 4; ++k2) a[k1 + 4 * k2] = y[k1][k2];
  }
}

template <int R, class T>
__device__ __forceinline__ void dft(cplx<T>* a) {
  if constexpr (R == 1) return;
  else if constexpr (R == 2) dft2(a);
  else if constexpr (R == 3) dft3(a);
  else if constexpr (R == 4) dft4(a);
  else if constexpr (R == 5) dft5(a);
  else if constexpr (R == 7) dft7(a);
  else if constexpr (R == 16) dft16(a);
  else dft8(a);
}

}  // namespace ftm
