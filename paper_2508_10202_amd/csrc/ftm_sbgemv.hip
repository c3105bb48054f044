// Strided-batched matrix-vector products y_b = alpha op(A_b) x_b + beta y_b
// (BLAS semantics: A_b is m x n column-major with leading dimension lda,
// op = N, T or C), for real and complex single and double precision -- the
// standalone form of the phase-3 product, tuned for short-wide matrices
// (m <= n), the case Section 3.1.1 optimises.
//
// op = T / C: y_j = sum_i op(A[i + j lda]) x_i is a dot product of the
// contiguous column j with x.  A group of G lanes (G a power of two, the
// smallest that covers a column in one 16-byte load per lane, at most 64)
// owns one column at a time; the columns of a workgroup's tile are dealt to
// the groups, loads are 16 bytes wide, and the group reduces by lane
// shuffles.  Workgroups tile the columns of every matrix of the batch, so the
// grid is batch * ceil(n / 64) workgroups however short the columns are.
//
// op = N: y_i = sum_j A[i + j lda] x_j.  A workgroup owns a tile of rows of
// one matrix; its lanes cover the tile's rows (V rows per 16-byte load), its
// waves split the columns, and the partial sums meet in LDS in a fixed order.
#include "ftm.h"
#include "ftm_device.h"
#include "ftm_kernels.h"
#include "ftm_sbgemv.h"

namespace ftm {

namespace {

// element algebra: real or complex, conjugation a no-op for real types
template <class T>
struct El;
template <>
struct El<float> {
  using acc = float;
  static __device__ __forceinline__ acc zero() { return 0.f; }
  static __device__ __forceinline__ acc mac(acc s, float a, float x, bool) { return fmaf(a, x, s); }
  static __device__ __forceinline__ acc add(acc a, acc b) { return a + b; }
  static __device__ __forceinline__ acc mul(acc a, acc b) { return a * b; }
  static __device__ __forceinline__ acc shfl_xor(acc v, int m) { return __shfl_xor(v, m); }
};
template <>
struct El<double> {
  using acc = double;
  static __device__ __forceinline__ acc zero() { return 0.0; }
  static __device__ __forceinline__ acc mac(acc s, double a, double x, bool) { return fma(a, x, s); }
  static __device__ __forceinline__ acc add(acc a, acc b) { return a + b; }
  static __device__ __forceinline__ acc mul(acc a, acc b) { return a * b; }
  static __device__ __forceinline__ acc shfl_xor(acc v, int m) { return __shfl_xor(v, m); }
};
template <class R>
struct El<cplx<R>> {
  using acc = cplx<R>;
  static __device__ __forceinline__ acc zero() { return {(R)0, (R)0}; }
  // s + op(a) x, op = conjugation when cj
  static __device__ __forceinline__ acc mac(acc s, cplx<R> a, cplx<R> x, bool cj) {
    const R ai = cj ? -a.y : a.y;
    return {s.x + a.x * x.x - ai * x.y, s.y + a.x * x.y + ai * x.x};
  }
  static __device__ __forceinline__ acc add(acc a, acc b) { return {a.x + b.x, a.y + b.y}; }
  static __device__ __forceinline__ acc mul(acc a, acc b) { return {a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x}; }
  static __device__ __forceinline__ acc shfl_xor(acc v, int m) { return {__shfl_xor(v.x, m), __shfl_xor(v.y, m)}; }
};

template <class T>
__device__ __forceinline__ bool is_zero(T v) {
  return v == (T)0;
}
template <class R>
__device__ __forceinline__ bool is_zero(cplx<R> v) {
  return v.x == (R)0 && v.y == (R)0;
}

// y = alpha s + beta y; y is not read when beta is zero (BLAS semantics)
template <class T>
__device__ __forceinline__ void finish(T* y, typename El<T>::acc s, T alpha, T beta) {
  typename El<T>::acc r = El<T>::mul(alpha, s);
  if (!is_zero(beta)) r = El<T>::add(r, El<T>::mul(beta, *y));
  *y = r;
}

// V consecutive elements, loaded as one access of V * sizeof(T) <= 16 bytes
template <class T, int V>
struct alignas(sizeof(T) * V) Vec {
  T e[V];
};

constexpr int SB_THREADS = 256;  // transposed kernels
constexpr int SB_TILE = 64;      // columns per workgroup (transposed kernels)

// ---- op = T / C ---------------------------------------------------------------
// V elements per 16-byte load (1 when lda or a pointer does not allow it), G
// lanes per column.
template <class T, int V, int G, bool CJ, int CPG = 4>
__global__ __launch_bounds__(SB_THREADS) void sbgemv_t_kernel(int m, int n, T alpha, const T* __restrict__ A,
                                                               int64_t lda, int64_t sa, const T* __restrict__ x,
                                                               int64_t sx, T beta, T* __restrict__ y, int64_t sy,
                                                               int ntile) {
  using E = El<T>;
  const int64_t wg = xcd_order(blockIdx.x, gridDim.x);
  const int64_t b = wg / ntile;
  const int tile = (int)(wg - b * ntile);
  const int g = threadIdx.x / G, li = threadIdx.x % G;  // column group, lane in group
  constexpr int NG = SB_THREADS / G;
  const T* __restrict__ Ab = A + b * sa;
  const T* __restrict__ xb = x + b * sx;
  const int nchunk = (m + V - 1) / V;
  const int cend = min(n, (tile + 1) * SB_TILE);
  // CPG columns per group at a time, so that each lane has CPG loads in flight
  for (int c0 = tile * SB_TILE + g; c0 < cend; c0 += NG * CPG) {
    typename E::acc s[CPG];
    const T* __restrict__ col[CPG];
#pragma unroll
    for (int u = 0; u < CPG; ++u) {
      s[u] = E::zero();
      col[u] = Ab + (int64_t)min(c0 + u * NG, cend - 1) * lda;  // clamped columns are not stored
    }
    for (int q = li; q < nchunk; q += G) {
      const int i0 = q * V;
      if (V > 1 && i0 + V <= m) {
        const Vec<T, V> xv = *reinterpret_cast<const Vec<T, V>*>(xb + i0);
        Vec<T, V> a[CPG];
#pragma unroll
        for (int u = 0; u < CPG; ++u) a[u] = *reinterpret_cast<const Vec<T, V>*>(col[u] + i0);
#pragma unroll
        for (int u = 0; u < CPG; ++u)
#pragma unroll
          for (int v = 0; v < V; ++v) s[u] = E::mac(s[u], a[u].e[v], xv.e[v], CJ);
      } else {
        for (int v = 0; v < V && i0 + v < m; ++v) {
          const T xi = xb[i0 + v];
#pragma unroll
          for (int u = 0; u < CPG; ++u) s[u] = E::mac(s[u], col[u][i0 + v], xi, CJ);
        }
      }
    }
#pragma unroll
    for (int u = 0; u < CPG; ++u) {
#pragma unroll
      for (int d = G / 2; d > 0; d >>= 1) s[u] = E::add(s[u], E::shfl_xor(s[u], d));
      const int c = c0 + u * NG;
      if (li == 0 && c < cend) finish(y + b * sy + c, s[u], alpha, beta);
    }
  }
}

// ---- op = N ---------------------------------------------------------------------
constexpr int SBN_WAVES = 16;
template <class T, int V>
__global__ __launch_bounds__(64 * SBN_WAVES) void sbgemv_n_kernel(int m, int n, T alpha, const T* __restrict__ A,
                                                                   int64_t lda, int64_t sa, const T* __restrict__ x,
                                                                   int64_t sx, T beta, T* __restrict__ y, int64_t sy,
                                                                   int nrt) {
  using E = El<T>;
  using acc = typename E::acc;
  const int64_t wg = xcd_order(blockIdx.x, gridDim.x);
  const int64_t b = wg / nrt;
  const int rt = (int)(wg - b * nrt);
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int i0 = (rt * 64 + lane) * V;  // this lane's first row
  const T* __restrict__ Ab = A + b * sa;
  const T* __restrict__ xb = x + b * sx;
  acc s[V];
#pragma unroll
  for (int v = 0; v < V; ++v) s[v] = E::zero();
  if (i0 < m) {
    const bool full = i0 + V <= m;
#pragma unroll 8
    for (int j = w; j < n; j += SBN_WAVES) {
      const T xj = xb[j];
      const T* __restrict__ cj = Ab + (int64_t)j * lda + i0;
      if (V > 1 && full) {
        const Vec<T, V> a = *reinterpret_cast<const Vec<T, V>*>(cj);
#pragma unroll
        for (int v = 0; v < V; ++v) s[v] = E::mac(s[v], a.e[v], xj, false);
      } else {
        for (int v = 0; v < V && i0 + v < m; ++v) s[v] = E::mac(s[v], cj[v], xj, false);
      }
    }
  }
  __shared__ acc red[SBN_WAVES - 1][64 * V];
  if (w > 0) {
#pragma unroll
    for (int v = 0; v < V; ++v) red[w - 1][lane * V + v] = s[v];
  }
  __syncthreads();
  if (w > 0 || i0 >= m) return;
#pragma unroll
  for (int q = 0; q < SBN_WAVES - 1; ++q)
#pragma unroll
    for (int v = 0; v < V; ++v) s[v] = E::add(s[v], red[q][lane * V + v]);
  for (int v = 0; v < V && i0 + v < m; ++v) finish(y + b * sy + i0 + v, s[v], alpha, beta);
}

// ---- launchers --------------------------------------------------------------------

template <class T, int V, int G, bool CJ>
hipError_t go_t(int m, int n, T alpha, const T* A, int64_t lda, int64_t sa, const T* x, int64_t sx, T beta, T* y,
                int64_t sy, int64_t batch, hipStream_t st) {
  const int ntile = (n + SB_TILE - 1) / SB_TILE;
  const int64_t nwg = batch * ntile;
  hipLaunchKernelGGL((sbgemv_t_kernel<T, V, G, CJ>), dim3((unsigned)nwg), dim3(SB_THREADS), 0, st, m, n, alpha, A,
                     lda, sa, x, sx, beta, y, sy, ntile);
  return hipGetLastError();
}

// lanes per column: the smallest power of two covering ceil(m / V) loads, at most 64
template <class T, int V, bool CJ>
hipError_t pick_g(int m, int n, T alpha, const T* A, int64_t lda, int64_t sa, const T* x, int64_t sx, T beta, T* y,
                  int64_t sy, int64_t batch, hipStream_t st) {
  const int chunks = (m + V - 1) / V;
  if (chunks <= 8) return go_t<T, V, 8, CJ>(m, n, alpha, A, lda, sa, x, sx, beta, y, sy, batch, st);
  if (chunks <= 16) return go_t<T, V, 16, CJ>(m, n, alpha, A, lda, sa, x, sx, beta, y, sy, batch, st);
  if (chunks <= 32) return go_t<T, V, 32, CJ>(m, n, alpha, A, lda, sa, x, sx, beta, y, sy, batch, st);
  return go_t<T, V, 64, CJ>(m, n, alpha, A, lda, sa, x, sx, beta, y, sy, batch, st);
}

template <class T, int V>
hipError_t go_n(int m, int n, T alpha, const T* A, int64_t lda, int64_t sa, const T* x, int64_t sx, T beta, T* y,
                int64_t sy, int64_t batch, hipStream_t st) {
  const int nrt = (m + 64 * V - 1) / (64 * V);
  const int64_t nwg = batch * nrt;
  hipLaunchKernelGGL((sbgemv_n_kernel<T, V>), dim3((unsigned)nwg), dim3(64 * SBN_WAVES), 0, st, m, n, alpha, A, lda,
                     sa, x, sx, beta, y, sy, nrt);
  return hipGetLastError();
}

template <class T>
hipError_t dispatch(int op, int m, int n, const void* alpha, const void* A, int64_t lda, int64_t sa, const void* x,
                    int64_t sx, const void* beta, void* y, int64_t sy, int64_t batch, hipStream_t st) {
  constexpr int V = 16 / (int)sizeof(T);
  const T al = *reinterpret_cast<const T*>(alpha), be = *reinterpret_cast<const T*>(beta);
  const T* a = reinterpret_cast<const T*>(A);
  const T* xv = reinterpret_cast<const T*>(x);
  T* yv = reinterpret_cast<T*>(y);
  // 16-byte loads need every column start (and, for op = T / C, x) aligned
  auto aligned = [](const void* p) { return (reinterpret_cast<uintptr_t>(p) & 15) == 0; };
  const bool vec = V > 1 && lda % V == 0 && sa % V == 0 && aligned(A) &&
                   (op == FTM_OP_N || (sx % V == 0 && aligned(x)));
  if (op == FTM_OP_N) {
    // narrower loads when the row tiles of 64 V rows would leave the chip
    // with fewer than 2 workgroups per CU (short matrices, small batches)
    auto wgs = [&](int v) { return batch * ((m + 64 * v - 1) / (64 * v)); };
    if (vec && (V == 1 || wgs(V) >= 512)) return go_n<T, V>(m, n, al, a, lda, sa, xv, sx, be, yv, sy, batch, st);
    if constexpr (V == 4) {
      if (vec && wgs(2) >= 512) return go_n<T, 2>(m, n, al, a, lda, sa, xv, sx, be, yv, sy, batch, st);
    }
    return go_n<T, 1>(m, n, al, a, lda, sa, xv, sx, be, yv, sy, batch, st);
  }
  const bool cj = op == FTM_OP_C;
  if (vec) {
    return cj ? pick_g<T, V, true>(m, n, al, a, lda, sa, xv, sx, be, yv, sy, batch, st)
              : pick_g<T, V, false>(m, n, al, a, lda, sa, xv, sx, be, yv, sy, batch, st);
  }
  return cj ? pick_g<T, 1, true>(m, n, al, a, lda, sa, xv, sx, be, yv, sy, batch, st)
            : pick_g<T, 1, false>(m, n, al, a, lda, sa, xv, sx, be, yv, sy, batch, st);
}

}  // namespace

hipError_t launch_sbgemv(int type, int op, int m, int n, const void* alpha, const void* A, int64_t lda, int64_t sa,
                         const void* x, int64_t sx, const void* beta, void* y, int64_t sy, int64_t batch,
                         hipStream_t st) {
  switch (type) {
    case FTM_TYPE_S: return dispatch<float>(op, m, n, alpha, A, lda, sa, x, sx, beta, y, sy, batch, st);
    case FTM_TYPE_D: return dispatch<double>(op, m, n, alpha, A, lda, sa, x, sx, beta, y, sy, batch, st);
    case FTM_TYPE_C: return dispatch<cplx<float>>(op, m, n, alpha, A, lda, sa, x, sx, beta, y, sy, batch, st);
    case FTM_TYPE_Z: return dispatch<cplx<double>>(op, m, n, alpha, A, lda, sa, x, sx, beta, y, sy, batch, st);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace ftm
