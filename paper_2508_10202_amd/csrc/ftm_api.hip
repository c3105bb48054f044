// Host runtime behind the C ABI of include/ftm.h: operator setup (the one-time
// float64 transform of the first block column, Section 2.4 and Section 3.2.1
// "Initial state"), per-phase precision dispatch (Section 3.2), workspace and
// the stream-ordered three-kernel chain of a matvec.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>
#include <cstdio>
#include <algorithm>
#include <cstring>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "ftm.h"
#include "ftm_device.h"
#include "ftm_kernels.h"
#include "ftm_sbgemv.h"
#include "ftm_runtime.h"

using namespace ftm;
using ftm_rt::DevBuf;
using ftm_rt::DeviceGuard;
using ftm_rt::fail;
using ftm_rt::fail_hip;

namespace ftm_rt {

static thread_local std::string g_last_error;

ftm_status fail(ftm_status s, const std::string& msg) {
  g_last_error = msg;
  return s;
}

ftm_status fail_hip(const char* what, hipError_t e) {
  return fail(FTM_ERR_HIP, std::string(what) + ": " + hipGetErrorString(e));
}

Workspace carve_workspace(const ftm_operator_s* op, void* base, int64_t nrhs, bool adjoint, const ftm_precision& p) {
  int em, ed;
  ftm_operator_s::workspace_elems(p, adjoint, &em, &ed);
  Workspace w;
  char* b = reinterpret_cast<char*>(base);
  w.mhat = b;
  w.dhat = b + ftm_operator_s::round256((size_t)op->K * nrhs * op->ldm * em);
  return w;
}

}  // namespace ftm_rt

ftm_rt::Exec ftm_operator_s::exec(bool adjoint, int64_t nrhs, bool allow_profile) const {
  std::lock_guard<std::mutex> lk(mu);
  ftm_rt::Exec e;
  e.p = adjoint ? adj : fwd;
  e.gemv_variant = variant[adjoint ? 1 : 0][e.p.gemv];
  e.fft_shape_in = fft_shape[adjoint ? 1 : 0][0][e.p.fft == ftm::DT_F64 ? 1 : 0];
  e.fft_shape_out = fft_shape[adjoint ? 1 : 0][1][e.p.ifft == ftm::DT_F64 ? 1 : 0];
  e.gemm_tile = gemm_tile[adjoint ? 1 : 0][e.p.gemv];
  e.gemm_kind = gemm_kind[adjoint ? 1 : 0];
  // many right-hand sides: one pass of the spectrum through the matrix cores
  // (float64 accumulation on the float64 ones, float32 on the others)
  const bool gemm_ok = nrhs >= 2;
  e.use_gemm = gemm_ok && (rhs_mode == FTM_RHS_GEMM ||
                           (rhs_mode == FTM_RHS_AUTO && nrhs >= gemm_min_rhs[adjoint ? 1 : 0][e.p.gemv]));
  e.profile = allow_profile && profiling;
  return e;
}

namespace {

size_t dtype_bytes(int dt) {  // bytes of one complex number in storage format dt
  switch (dt) {
    case DT_F64: return 16;
    case DT_F32: return 8;
    default: return 4;
  }
}

bool valid_dtype(int32_t v) { return v >= DT_F64 && v <= DT_BF16; }

ftm_status check_precision(const ftm_precision& p) {
  if (!valid_dtype(p.pad) || !valid_dtype(p.fft) || !valid_dtype(p.gemv) || !valid_dtype(p.ifft) ||
      !valid_dtype(p.unpad))
    return fail(FTM_ERR_INVALID, "precision: every phase must be FTM_F64, FTM_F32, FTM_F16 or FTM_BF16");
  if (p.accum != DT_F64 && p.accum != DT_F32)
    return fail(FTM_ERR_INVALID, "precision: accum must be FTM_F64 or FTM_F32");
  if (p.gemv == DT_F64 && p.accum != DT_F64)
    return fail(FTM_ERR_INVALID, "precision: an FP64 product accumulates in FP64");
  if ((p.gemv == DT_F16 || p.gemv == DT_BF16) && p.accum != DT_F32)
    return fail(FTM_ERR_INVALID, "precision: FP16/BF16 products accumulate in FP32");
  return FTM_OK;
}

const ftm_precision kAllF64 = {DT_F64, DT_F64, DT_F64, DT_F64, DT_F64, DT_F64};

// Radices of length-N plans: the factor 2^e2 in as few passes as radices up
// to 2^maxbits allow, its bits spread evenly over them, then the factors 5, 3
// and 7; in
// descending order for the forward transform (its paired last pass takes the
// smallest radix) and ascending for the inverse one (paired first pass).  At
// least two passes: a lone power of two is split, and N = 2 runs 2 and 1.
void fill_plan(int N, const std::vector<int>& rad, FftPlan* plan) {
  plan->N = N;
  plan->nst = (int)rad.size();
  int Ns = 1;
  for (int i = 0; i < plan->nst; ++i) {
    plan->rad[i] = rad[i];
    plan->toff[i] = Ns == 1 && i == 0 ? 0 : plan->toff[i - 1] + Ns;  // pass i-1 took Ns = Ns_{i-1} * rad[i-1] entries
    plan->div_ns[i] = make_fastdiv((uint32_t)Ns);
    Ns *= rad[i];
  }
}

bool make_plans(int N, int maxbits, FftPlan* fwd, FftPlan* inv) {
  int n = N, e2 = 0;
  std::vector<int> rad;
  while (n % 2 == 0) { n /= 2; ++e2; }
  const int np = (e2 + maxbits - 1) / maxbits;
  for (int i = 0; i < np; ++i) {
    const int bits = (e2 + (np - i) - 1) / (np - i);  // ceil of the remaining bits over the remaining passes
    rad.push_back(1 << bits);
    e2 -= bits;
  }
  for (int r : {5, 3, 7})
    while (n % r == 0) { n /= r; rad.push_back(r); }
  if (n != 1 || rad.empty()) return false;
  if (rad.size() == 1) {
    const int r = rad[0];
    if (r == 2) rad = {2, 1};
    else if (r == 4) rad = {2, 2};
    else if (r == 8) rad = {4, 2};
    else if (r == 16) rad = {4, 4};
    else return false;
  }
  if ((int)rad.size() > MAX_STAGES) return false;
  std::sort(rad.begin(), rad.end(), [](int a, int b) { return a > b; });
  fill_plan(N, rad, fwd);
  std::reverse(rad.begin(), rad.end());
  fill_plan(N, rad, inv);
  return true;
}

}  // namespace

namespace {

ftm_status dev_alloc(DevBuf* b, size_t n) {
  b->n = 0;
  hipError_t e = hipMalloc(&b->p, n ? n : 1);
  if (e != hipSuccess) {
    b->p = nullptr;
    (void)hipGetLastError();
    return fail(FTM_ERR_OOM, "hipMalloc of " + std::to_string(n) + " bytes failed: " + hipGetErrorString(e));
  }
  b->n = n;
  return FTM_OK;
}

void dev_free(DevBuf* b) {
  if (b->p) (void)hipFree(b->p);
  b->p = nullptr;
  b->n = 0;
}

void release(ftm_operator op) {
  for (auto& r : op->recs)
    for (hipEvent_t e : r.ev) op->event_pool.push_back(e);
  op->recs.clear();
  for (hipEvent_t e : op->event_pool) (void)hipEventDestroy(e);
  op->event_pool.clear();
  dev_free(&op->tw64f);
  dev_free(&op->tw64i);
  dev_free(&op->tw32f);
  dev_free(&op->tw32i);
  for (auto& s : op->spec) dev_free(&s);
  dev_free(&op->mhat);
  dev_free(&op->dhat);
}

// Per-pass twiddle tables of a plan (see FftPlan): exp(-2 pi i q jm / (Ns R))
// evaluated in long double and rounded once to T.
template <class T>
std::vector<T> twiddle_table(const FftPlan& pl) {
  std::vector<T> t(2 * (size_t)pl.twiddle_entries());
  const long double two_pi = 6.283185307179586476925286766559005768L;
  int Ns = 1;
  for (int s = 0; s < pl.nst; ++s) {
    const int R = pl.rad[s];
    for (int jm = 0; jm < Ns; ++jm)
      for (int q = 0; q < R; ++q) {
        const long double ang = two_pi * (long double)(q * jm) / (long double)(Ns * R);
        const size_t e = (size_t)pl.toff[s] + (size_t)jm * R + q;
        t[2 * e] = (T)cosl(ang);
        t[2 * e + 1] = (T)-sinl(ang);
      }
    Ns *= R;
  }
  return t;
}

// Twiddle tables of the plans in their compute types.
ftm_status upload_twiddles(ftm_operator op, hipStream_t st) {
  const std::vector<double> t64f = twiddle_table<double>(op->plan_f64), t64i = twiddle_table<double>(op->plan_i64);
  const std::vector<float> t32f = twiddle_table<float>(op->plan_f32), t32i = twiddle_table<float>(op->plan_i32);
  ftm_status s;
  if ((s = dev_alloc(&op->tw64f, t64f.size() * sizeof(double))) != FTM_OK) return s;
  if ((s = dev_alloc(&op->tw64i, t64i.size() * sizeof(double))) != FTM_OK) return s;
  if ((s = dev_alloc(&op->tw32f, t32f.size() * sizeof(float))) != FTM_OK) return s;
  if ((s = dev_alloc(&op->tw32i, t32i.size() * sizeof(float))) != FTM_OK) return s;
  FTM_HIP(hipMemcpyAsync(op->tw64f.p, t64f.data(), op->tw64f.n, hipMemcpyHostToDevice, st));
  FTM_HIP(hipMemcpyAsync(op->tw64i.p, t64i.data(), op->tw64i.n, hipMemcpyHostToDevice, st));
  FTM_HIP(hipMemcpyAsync(op->tw32f.p, t32f.data(), op->tw32f.n, hipMemcpyHostToDevice, st));
  FTM_HIP(hipMemcpyAsync(op->tw32i.p, t32i.data(), op->tw32i.n, hipMemcpyHostToDevice, st));
  // the host vectors die at return: make the copies complete first
  FTM_HIP(hipStreamSynchronize(st));
  return FTM_OK;
}

// Make sure the spectrum copies the two configurations (and `mask`) need
// exist, creating them from the float64 spectrum.
ftm_status ensure_spectra(ftm_operator op, uint32_t mask, hipStream_t st) {
  const int64_t n = op->K * op->Nd * op->ldm;
  for (int dt = DT_F32; dt <= DT_BF16; ++dt) {
    if (!(mask & (1u << dt)) || op->spec[dt].p) continue;
    if (!op->spec[DT_F64].p)
      return fail(FTM_ERR_UNSUPPORTED, "spectrum in format " + std::to_string(dt) +
                                           " was not kept at setup and the FP64 spectrum is gone");
    ftm_status s = dev_alloc(&op->spec[dt], (size_t)n * dtype_bytes(dt));
    if (s != FTM_OK) return s;
    FTM_HIP(launch_store_spectrum(op->spec[DT_F64].p, dt, op->spec[dt].p, n, st));
  }
  return FTM_OK;
}

// Events of one profiled call (none when not profiling), taken from the
// operator's pool under its lock and filed in its record once recorded.
struct Profiler {
  ftm_operator op;
  hipStream_t st;
  bool on;
  ftm_operator_s::Rec rec{};
  Profiler(ftm_operator o, hipStream_t s, int dir, bool enabled) : op(o), st(s), on(enabled) {
    rec.dir = dir;
    if (!on) return;
    std::lock_guard<std::mutex> lk(op->mu);
    for (auto& e : rec.ev) {
      if (!op->event_pool.empty()) {
        e = op->event_pool.back();
        op->event_pool.pop_back();
      } else if (hipEventCreate(&e) != hipSuccess) {
        e = nullptr;
      }
    }
  }
  void mark(int i) {
    if (on && rec.ev[i]) (void)hipEventRecord(rec.ev[i], st);
  }
  ~Profiler() {
    if (!on) return;
    std::lock_guard<std::mutex> lk(op->mu);
    op->recs.push_back(rec);
  }
};

uint32_t needed_mask(const ftm_precision& f, const ftm_precision& a) { return (1u << f.gemv) | (1u << a.gemv); }

}  // namespace

// One direction of the matvec: x (float64, [nrhs][Nt][Sx]) -> y (float64,
// [nrhs][Nt][Sy]).  adjoint selects Fhat^H in phase 3.
ftm_status ftm_rt::run_matvec(ftm_operator op, bool adjoint, const Exec& ex, const MatvecIO& io, int64_t nrhs,
                              const Workspace& ws, hipStream_t st) {
  const ftm_precision& p = ex.p;
  const void* F = op->spec[p.gemv].p;
  if (!F) return fail(FTM_ERR_STATE, "spectrum for the configured phase-3 precision is missing");

  // Intermediates between phases are stored in float64 only when both
  // neighbouring phases are float64; otherwise the producing kernel applies
  // both phases' roundings and stores float32, which holds every such value
  // exactly (FP16 and BF16 values are float32 values).  The input of a
  // half-precision product is stored in 16 bits in the product's format, in
  // which the producer's last rounding left it: the product reads half the
  // bytes (one-vector forward product at Nt=1000, Nd=100, Nm=5000: 358 ->
  // 322 us; the one-vector adjoint reads one input value per spectrum row and
  // keeps float32).  The product's output stays float32 (measured: the
  // inverse transform reading 16-bit rows, 64 bytes per tile row, loses more
  // than the product saves).
  const bool x_hat64 = p.fft == DT_F64 && p.gemv == DT_F64;
  const bool y_hat64 = p.gemv == DT_F64 && p.ifft == DT_F64;
  const bool st16 = (p.gemv == DT_F16 || p.gemv == DT_BF16) && p.accum != DT_F64 && (ex.use_gemm || !adjoint);
  const int x_st = st16 ? ST_16 : (x_hat64 ? ST_F64 : ST_F32);
  const int y_st = y_hat64 ? ST_F64 : ST_F32;
  const int64_t Sx = adjoint ? op->Nd : op->Nm, Sy = adjoint ? op->Nm : op->Nd;
  const int ldx = adjoint ? op->ldd : op->ldm, ldy = adjoint ? op->ldm : op->ldd;
  void* xhat = adjoint ? ws.dhat : ws.mhat;
  void* yhat = adjoint ? ws.mhat : ws.dhat;

  RfftArgs ra{};
  ra.x = io.x;
  ra.xptr = io.xptr;
  ra.pad_to = ldx;
  ra.x_rhs_stride = op->Nt * Sx;
  ra.x_row_stride = Sx;
  ra.x_sr = 0;
  ra.x_sc = 1;
  ra.S = Sx;
  ra.Nt = (int)op->Nt;
  ra.nrhs = (int)nrhs;
  ra.out = xhat;
  ra.out_k_stride = nrhs * ldx;
  ra.out_rhs_stride = ldx;
  ra.ncol = Sx;
  ra.ld_row = ldx;
  ra.r_pad = p.pad;
  ra.r_fft = p.fft;
  ra.r_next = p.gemv;
  Profiler prof(op, st, adjoint ? 1 : 0, ex.profile);
  prof.mark(0);
  FTM_HIP(launch_rfft(p.fft == DT_F64, x_st, ra, op->fft_in(p.fft == DT_F64), ex.fft_shape_in, st));

  GemvArgs ga{};
  ga.F = F;
  ga.f_k_stride = op->Nd * op->ldm;
  ga.ld = op->ldm;
  ga.Nd = (int)op->Nd;
  ga.Nm = (int)op->Nm;
  ga.K = (int)op->K;
  ga.nrhs = (int)nrhs;
  ga.x = xhat;
  ga.x_k_stride = nrhs * ldx;
  ga.x_rhs_stride = ldx;
  ga.y = yhat;
  ga.y_k_stride = nrhs * ldy;
  ga.y_rhs_stride = ldy;
  ga.r_gemv = p.gemv;
  ga.r_next = p.ifft;
  ga.variant = ex.gemv_variant;
  ga.rhs_tile = ex.gemm_tile;
  ga.gemm_kind = ex.gemm_kind;
  ga.x16 = st16 ? 1 : 0;
  const bool acc64 = p.accum == DT_F64;
  prof.mark(1);
  if (ex.use_gemm) {
    if (acc64) FTM_HIP(launch_gemm_a64(adjoint, p.gemv, x_hat64, y_hat64, ga, st));
    else if (adjoint) FTM_HIP(launch_gemm_adj(p.gemv, ga, st));
    else FTM_HIP(launch_gemm_fwd(p.gemv, ga, st));
  } else if (adjoint) {
    FTM_HIP(launch_gemv_adj(p.gemv, acc64, x_hat64, y_hat64, ga, st));
  } else {
    FTM_HIP(launch_gemv_fwd(p.gemv, acc64, x_hat64, y_hat64, ga, st));
  }

  IrfftArgs ia{};
  ia.in = yhat;
  ia.in_k_stride = nrhs * ldy;
  ia.in_rhs_stride = ldy;
  ia.S = Sy;
  ia.Nt = (int)op->Nt;
  ia.nrhs = (int)nrhs;
  ia.y = io.y;
  ia.yptr = io.yptr;
  ia.y_rhs_stride = op->Nt * Sy;
  ia.y_row_stride = Sy;
  ia.r_ifft = p.ifft;
  ia.r_unpad = p.unpad;
  prof.mark(2);
  FTM_HIP(launch_irfft(y_st, p.ifft == DT_F64, ia, op->fft_out(p.ifft == DT_F64), ex.fft_shape_out, st));
  prof.mark(3);
  return FTM_OK;
}

extern "C" {

ftm_status ftm_sbgemv(int32_t type, int32_t op, int64_t m, int64_t n, const void* alpha, const void* A, int64_t lda,
                      int64_t stride_a, const void* x, int64_t stride_x, const void* beta, void* y, int64_t stride_y,
                      int64_t batch, void* stream) {
  try {
    if (type < FTM_TYPE_S || type > FTM_TYPE_Z) return fail(FTM_ERR_INVALID, "type must be FTM_TYPE_S/D/C/Z");
    if (op < FTM_OP_N || op > FTM_OP_C) return fail(FTM_ERR_INVALID, "op must be FTM_OP_N/T/C");
    if (m < 0 || n < 0 || batch < 0) return fail(FTM_ERR_INVALID, "m, n and batch must be >= 0");
    if (m == 0 || n == 0 || batch == 0) return FTM_OK;
    if (!alpha || !beta || !A || !x || !y) return fail(FTM_ERR_INVALID, "NULL argument");
    if (m >= ((int64_t)1 << 31) || n >= ((int64_t)1 << 31)) return fail(FTM_ERR_INVALID, "m and n must be < 2^31");
    if (lda < m) return fail(FTM_ERR_INVALID, "lda must be >= m");
    const int64_t nx = op == FTM_OP_N ? n : m, ny = op == FTM_OP_N ? m : n;
    const int64_t a_span = lda * (n - 1) + m;
    if (batch > 1 && (stride_a < a_span || stride_x < nx || stride_y < ny))
      return fail(FTM_ERR_INVALID, "strides must separate the batch's matrices and vectors");
    // workgroups per matrix: op N tiles at least 64 rows, op T / C 64 columns
    const int64_t per = op == FTM_OP_N ? (m + 63) / 64 : (n + 63) / 64;
    if (batch > ((int64_t)1 << 31) / per) return fail(FTM_ERR_INVALID, "too many workgroups (batch too large)");
    FTM_HIP(launch_sbgemv(type, op, (int)m, (int)n, alpha, A, lda, stride_a, x, stride_x, beta, y, stride_y, batch,
                          reinterpret_cast<hipStream_t>(stream)));
    return FTM_OK;
  } catch (...) {
    return fail(FTM_ERR_INVALID, "internal error");
  }
}

const char* ftm_status_string(ftm_status s) {
  switch (s) {
    case FTM_OK: return "ok";
    case FTM_ERR_INVALID: return "invalid argument";
    case FTM_ERR_UNSUPPORTED: return "unsupported";
    case FTM_ERR_OOM: return "out of device memory";
    case FTM_ERR_BUDGET: return "over memory budget";
    case FTM_ERR_HIP: return "HIP error";
    case FTM_ERR_STATE: return "invalid state";
  }
  return "unknown status";
}

const char* ftm_last_error(void) { return ftm_rt::g_last_error.c_str(); }

ftm_status ftm_setup_operator(ftm_operator* out, const double* F, int64_t Nt, int64_t Nd, int64_t Nm,
                              const ftm_precision* fwd, const ftm_precision* adj, uint32_t spectra,
                              int64_t max_rhs, void* stream) {
  return ftm_setup_operator_strided(out, F, Nt, Nd, Nm, Nd * Nm, Nm, 1, fwd, adj, spectra, max_rhs, stream);
}

ftm_status ftm_setup_operator_strided(ftm_operator* out, const double* F, int64_t Nt, int64_t Nd, int64_t Nm,
                                      int64_t stride_t, int64_t stride_r, int64_t stride_c,
                                      const ftm_precision* fwd, const ftm_precision* adj, uint32_t spectra,
                                      int64_t max_rhs, void* stream) {
  try {
    if (!out) return fail(FTM_ERR_INVALID, "out is NULL");
    *out = nullptr;
    if (!F) return fail(FTM_ERR_INVALID, "F is NULL");
    if (Nt < 1 || Nd < 1 || Nm < 1 || max_rhs < 1)
      return fail(FTM_ERR_INVALID, "Nt, Nd, Nm and max_rhs must be >= 1");
    {
      // the strides must address every (t, r, c) at a distinct element: in
      // increasing stride order, each stride at least the span of the smaller ones
      int64_t st[3] = {stride_t, stride_r, stride_c}, ex[3] = {Nt, Nd, Nm};
      for (int i = 0; i < 3; ++i)
        if (ex[i] > 1 && st[i] < 1) return fail(FTM_ERR_INVALID, "strides of dimensions longer than 1 must be >= 1");
      int ord[3] = {0, 1, 2};
      std::sort(ord, ord + 3, [&](int a, int b) { return st[a] < st[b]; });
      int64_t span = 1;
      for (int i = 0; i < 3; ++i) {
        if (ex[ord[i]] == 1) continue;
        if (st[ord[i]] < span) return fail(FTM_ERR_INVALID, "strides make elements of F overlap");
        span = st[ord[i]] * ex[ord[i]];
      }
    }
    // pad length: 2 Nt when it factors into 2, 3, 5 and 7 (the paper's
    // choice), else the next even length that does -- circular and linear
    // convolution agree on the first Nt outputs for any L >= 2 Nt - 1
    int64_t L = 2 * Nt;
    auto smooth = [](int64_t v) {
      for (int64_t r : {2, 3, 5, 7})
        while (v % r == 0) v /= r;
      return v == 1;
    };
    while (L <= FFT_POINTS && !smooth(L)) L += 2;
    if (L > FFT_POINTS)
      return fail(FTM_ERR_UNSUPPORTED, "no transform length of at most " + std::to_string(FFT_POINTS) +
                                           " covers Nt = " + std::to_string(Nt));
    if (Nd > (1 << 24) || Nm > (1 << 24) || Nd * Nm > ((int64_t)1 << 34) || max_rhs > (1 << 20))
      return fail(FTM_ERR_UNSUPPORTED, "size too large");
    if (spectra >> 4) return fail(FTM_ERR_INVALID, "spectra mask has bits beyond FTM_BF16");
    const ftm_precision pf = fwd ? *fwd : kAllF64, pa = adj ? *adj : kAllF64;
    ftm_status s;
    if ((s = check_precision(pf)) != FTM_OK || (s = check_precision(pa)) != FTM_OK) return s;

    FftPlan plan_f64{}, plan_i64{}, plan_f32{}, plan_i32{};
    if (!make_plans((int)L, 3, &plan_f64, &plan_i64) || !make_plans((int)L, 4, &plan_f32, &plan_i32))
      return fail(FTM_ERR_UNSUPPORTED, "no FFT plan for L = " + std::to_string(L));

    ftm_operator op = new ftm_operator_s();
    op->Nt = Nt;
    op->Nd = Nd;
    op->Nm = Nm;
    op->L = L;
    op->K = L / 2 + 1;
    op->ldm = (int)((Nm + 7) / 8 * 8);
    op->ldd = (int)((Nd + 7) / 8 * 8);
    op->max_rhs = max_rhs;
    op->plan_f64 = plan_f64;
    op->plan_i64 = plan_i64;
    op->plan_f32 = plan_f32;
    op->plan_i32 = plan_i32;
    op->fwd = pf;
    op->adj = pa;
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    auto bail = [&](ftm_status e) {
      (void)hipStreamSynchronize(st);
      release(op);
      delete op;
      return e;
    };
    if (hipGetDevice(&op->device) != hipSuccess) return bail(fail(FTM_ERR_HIP, "hipGetDevice failed"));
    if ((s = upload_twiddles(op, st)) != FTM_OK) return bail(s);

    // Fhat in float64: transform every (r, c) series of F along time.
    const int64_t nspec = op->K * Nd * op->ldm;
    if ((s = dev_alloc(&op->spec[DT_F64], (size_t)nspec * 16)) != FTM_OK) return bail(s);
    hipError_t e = hipMemsetAsync(op->spec[DT_F64].p, 0, op->spec[DT_F64].n, st);
    if (e != hipSuccess) return bail(fail_hip("hipMemsetAsync", e));
    RfftArgs ra{};
    ra.x = F;
    ra.x_rhs_stride = 0;
    ra.x_row_stride = stride_t;
    ra.x_sr = stride_r;
    ra.x_sc = stride_c;
    ra.S = Nd * Nm;
    ra.Nt = (int)Nt;
    ra.nrhs = 1;
    ra.out = op->spec[DT_F64].p;
    ra.out_k_stride = Nd * op->ldm;
    ra.out_rhs_stride = 0;
    ra.ncol = Nm;
    ra.ld_row = op->ldm;
    ra.r_pad = ra.r_fft = ra.r_next = DT_F64;
    ra.pad_to = 0;  // the spectrum's padding is cleared above
    e = launch_rfft(true, ST_F64, ra, op->fft_in(true), 0, st);
    if (e != hipSuccess) return bail(fail_hip("setup transform", e));

    const uint32_t keep = needed_mask(pf, pa) | spectra;
    if ((s = ensure_spectra(op, keep, st)) != FTM_OK) return bail(s);

    const size_t ws_m = (size_t)op->K * max_rhs * op->ldm * 16, ws_d = (size_t)op->K * max_rhs * op->ldd * 16;
    if ((s = dev_alloc(&op->mhat, ws_m)) != FTM_OK) return bail(s);
    if ((s = dev_alloc(&op->dhat, ws_d)) != FTM_OK) return bail(s);
    // padding columns of the workspaces are read (times zero) and must stay finite
    if ((e = hipMemsetAsync(op->mhat.p, 0, ws_m, st)) != hipSuccess) return bail(fail_hip("hipMemsetAsync", e));
    if ((e = hipMemsetAsync(op->dhat.p, 0, ws_d, st)) != hipSuccess) return bail(fail_hip("hipMemsetAsync", e));

    if (!(keep & (1u << DT_F64))) {
      // the copies were made on this stream; wait before freeing their source
      if ((e = hipStreamSynchronize(st)) != hipSuccess) return bail(fail_hip("hipStreamSynchronize", e));
      dev_free(&op->spec[DT_F64]);
    }
    *out = op;
    return FTM_OK;
  } catch (const std::bad_alloc&) {
    return fail(FTM_ERR_OOM, "host allocation failed");
  } catch (...) {
    return fail(FTM_ERR_INVALID, "unexpected exception in ftm_setup_operator");
  }
}

ftm_status ftm_set_precision(ftm_operator op, const ftm_precision* fwd, const ftm_precision* adj) {
  if (!op) return fail(FTM_ERR_INVALID, "operator is NULL");
  std::lock_guard<std::mutex> lk(op->mu);
  const ftm_precision pf = fwd ? *fwd : op->fwd, pa = adj ? *adj : op->adj;
  ftm_status s;
  if ((s = check_precision(pf)) != FTM_OK || (s = check_precision(pa)) != FTM_OK) return s;
  if (!op->spec[pf.gemv].p || !op->spec[pa.gemv].p)
    return fail(FTM_ERR_UNSUPPORTED, "the spectrum copy this configuration needs was not kept at setup");
  op->fwd = pf;
  op->adj = pa;
  return FTM_OK;
}

static bool overlaps(const void* a, size_t na, const void* b, size_t nb) {
  const char* pa = reinterpret_cast<const char*>(a);
  const char* pb = reinterpret_cast<const char*>(b);
  return pa < pb + nb && pb < pa + na;
}

// Validate the arguments of one matvec call (not the workspace).
static ftm_status check_call(ftm_operator op, bool adjoint, const double* x, double* y, int64_t nrhs,
                             int64_t max_rhs) {
  if (!op) return fail(FTM_ERR_INVALID, "operator is NULL");
  if (!x || !y) return fail(FTM_ERR_INVALID, "input or output is NULL");
  if (nrhs < 1 || nrhs > max_rhs)
    return fail(FTM_ERR_INVALID, "nrhs must be in [1, " + std::to_string(max_rhs) + "]");
  const int64_t nx = nrhs * op->Nt * (adjoint ? op->Nd : op->Nm);
  const int64_t ny = nrhs * op->Nt * (adjoint ? op->Nm : op->Nd);
  if (overlaps(x, (size_t)nx * 8, y, (size_t)ny * 8)) return fail(FTM_ERR_INVALID, "input and output overlap");
  return FTM_OK;
}

static ftm_status matvec_common(ftm_operator op, bool adjoint, const double* x, double* y, int64_t nrhs,
                                void* stream) {
  try {
    ftm_status s = check_call(op, adjoint, x, y, nrhs, op ? op->max_rhs : 0);
    if (s != FTM_OK) return s;
    DeviceGuard g(op->device);
    ftm_rt::MatvecIO io;
    io.x = x;
    io.y = y;
    ftm_rt::Workspace ws;
    ws.mhat = op->mhat.p;
    ws.dhat = op->dhat.p;
    return ftm_rt::run_matvec(op, adjoint, op->exec(adjoint, nrhs, true), io, nrhs, ws,
                              reinterpret_cast<hipStream_t>(stream));
  } catch (...) {
    return fail(FTM_ERR_INVALID, "unexpected exception in matvec");
  }
}

// Largest nrhs of a call that brings its own workspace.
static constexpr int64_t kMaxCallRhs = 1 << 20;

ftm_status ftm_workspace_size(ftm_operator op, int32_t adjoint, int64_t nrhs, size_t* bytes) {
  if (!op || !bytes) return fail(FTM_ERR_INVALID, "operator or bytes is NULL");
  if (nrhs < 1 || nrhs > kMaxCallRhs) return fail(FTM_ERR_INVALID, "nrhs must be in [1, 2^20]");
  const ftm_rt::Exec ex = op->exec(adjoint != 0, nrhs, false);
  *bytes = op->workspace_bytes(nrhs, adjoint != 0, ex.p);
  return FTM_OK;
}

// Workspace of one data-space Hessian action on nrhs vectors: the float64
// parameter-space intermediate F^T x ([nrhs][Nt][Nm]), then room for the
// larger of the two directions' transform workspaces.
static size_t hessian_bytes(const ftm_operator_s* op, int64_t nrhs, const ftm_rt::Exec& ef,
                            const ftm_rt::Exec& ea) {
  const size_t mid = ftm_operator_s::round256((size_t)nrhs * op->Nt * op->Nm * 8);
  const size_t wf = op->workspace_bytes(nrhs, false, ef.p), wa = op->workspace_bytes(nrhs, true, ea.p);
  return mid + (wf > wa ? wf : wa);
}

ftm_status ftm_hessian_workspace_size(ftm_operator op, int64_t nrhs, size_t* bytes) {
  if (!op || !bytes) return fail(FTM_ERR_INVALID, "operator or bytes is NULL");
  if (nrhs < 1 || nrhs > kMaxCallRhs) return fail(FTM_ERR_INVALID, "nrhs must be in [1, 2^20]");
  *bytes = hessian_bytes(op, nrhs, op->exec(false, nrhs, false), op->exec(true, nrhs, false));
  return FTM_OK;
}

ftm_status ftm_hessian_apply(ftm_operator op, const double* x, double* y, int64_t nrhs, void* workspace,
                             size_t workspace_bytes, void* stream) {
  try {
    if (!op) return fail(FTM_ERR_INVALID, "operator is NULL");
    if (!x || !y || !workspace) return fail(FTM_ERR_INVALID, "input, output or workspace is NULL");
    if (nrhs < 1 || nrhs > kMaxCallRhs) return fail(FTM_ERR_INVALID, "nrhs must be in [1, 2^20]");
    if (reinterpret_cast<uintptr_t>(workspace) % 256 != 0)
      return fail(FTM_ERR_INVALID, "workspace must be 256-byte aligned");
    const size_t nb = (size_t)nrhs * op->Nt * op->Nd * 8;
    if (overlaps(x, nb, y, nb)) return fail(FTM_ERR_INVALID, "input and output overlap");
    // both directions' configurations are copied now: the pair runs as one call
    const ftm_rt::Exec ea = op->exec(true, nrhs, true), ef = op->exec(false, nrhs, true);
    const size_t need = hessian_bytes(op, nrhs, ef, ea);
    if (workspace_bytes < need)
      return fail(FTM_ERR_INVALID, "workspace of " + std::to_string(workspace_bytes) + " bytes, the call needs " +
                                       std::to_string(need));
    if (overlaps(workspace, need, x, nb) || overlaps(workspace, need, y, nb))
      return fail(FTM_ERR_INVALID, "workspace overlaps the input or the output");
    DeviceGuard g(op->device);
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    char* base = reinterpret_cast<char*>(workspace);
    double* mid = reinterpret_cast<double*>(base);
    void* tws = base + ftm_operator_s::round256((size_t)nrhs * op->Nt * op->Nm * 8);
    ftm_rt::MatvecIO io;
    io.x = x;
    io.y = mid;
    ftm_status s = ftm_rt::run_matvec(op, true, ea, io, nrhs, ftm_rt::carve_workspace(op, tws, nrhs, true, ea.p), st);
    if (s != FTM_OK) return s;
    io.x = mid;
    io.y = y;
    return ftm_rt::run_matvec(op, false, ef, io, nrhs, ftm_rt::carve_workspace(op, tws, nrhs, false, ef.p), st);
  } catch (...) {
    return fail(FTM_ERR_INVALID, "unexpected exception in ftm_hessian_apply");
  }
}

ftm_status ftm_apply(ftm_operator op, int32_t adjoint, const double* x, double* y, int64_t nrhs, void* workspace,
                     size_t workspace_bytes, void* stream) {
  try {
    ftm_status s = check_call(op, adjoint != 0, x, y, nrhs, kMaxCallRhs);
    if (s != FTM_OK) return s;
    if (!workspace) return fail(FTM_ERR_INVALID, "workspace is NULL");
    if (reinterpret_cast<uintptr_t>(workspace) % 256 != 0)
      return fail(FTM_ERR_INVALID, "workspace must be 256-byte aligned");
    const bool adj = adjoint != 0;
    const ftm_rt::Exec ex = op->exec(adj, nrhs, true);
    const size_t need = op->workspace_bytes(nrhs, adj, ex.p);
    if (workspace_bytes < need)
      return fail(FTM_ERR_INVALID, "workspace of " + std::to_string(workspace_bytes) + " bytes, the call needs " +
                                       std::to_string(need));
    const int64_t nx = nrhs * op->Nt * (adj ? op->Nd : op->Nm), ny = nrhs * op->Nt * (adj ? op->Nm : op->Nd);
    if (overlaps(workspace, need, x, (size_t)nx * 8) || overlaps(workspace, need, y, (size_t)ny * 8))
      return fail(FTM_ERR_INVALID, "workspace overlaps the input or the output");
    DeviceGuard g(op->device);
    ftm_rt::MatvecIO io;
    io.x = x;
    io.y = y;
    const ftm_rt::Workspace ws = ftm_rt::carve_workspace(op, workspace, nrhs, adj, ex.p);
    return ftm_rt::run_matvec(op, adj, ex, io, nrhs, ws, reinterpret_cast<hipStream_t>(stream));
  } catch (...) {
    return fail(FTM_ERR_INVALID, "unexpected exception in ftm_apply");
  }
}

// ---- the library's static scratch workspace ------------------------------------
// FTM_SCRATCH_BYTES of device memory per GPU, held from the first
// ftm_apply_scratch call on that GPU until the process ends.  In host code the
// array's name is only a stand-in: kernels receive the device address that
// hipGetSymbolAddress returns for the current device, kept per device.
static __device__ __align__(256) unsigned char scratch[FTM_SCRATCH_BYTES];

namespace {
constexpr int kMaxScratchDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxScratchDevices] = {};

// Device address of the current device's scratch array (device dev current).
ftm_status scratch_address(int dev, void** out) {
  if (dev < 0 || dev >= kMaxScratchDevices) return fail(FTM_ERR_UNSUPPORTED, "device index beyond 63");
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p) return fail_hip("hipGetSymbolAddress(scratch)", e != hipSuccess ? e : hipErrorUnknown);
    g_scratch_ptr[dev] = p;
  }
  *out = g_scratch_ptr[dev];
  return FTM_OK;
}
}  // namespace

ftm_status ftm_apply_scratch(ftm_operator op, int32_t adjoint, const double* x, double* y, int64_t nrhs,
                             void* stream) {
  try {
    ftm_status s = check_call(op, adjoint != 0, x, y, nrhs, kMaxCallRhs);
    if (s != FTM_OK) return s;
    const bool adj = adjoint != 0;
    const ftm_rt::Exec ex = op->exec(adj, nrhs, false);  // no profiling events: nothing is created
    const size_t need = op->workspace_bytes(nrhs, adj, ex.p);
    if (need > (size_t)FTM_SCRATCH_BYTES)
      return fail(FTM_ERR_UNSUPPORTED, "the call needs " + std::to_string(need) + " bytes of workspace, the static "
                                       "scratch holds " + std::to_string((size_t)FTM_SCRATCH_BYTES));
    DeviceGuard g(op->device);
    void* base = nullptr;
    if ((s = scratch_address(op->device, &base)) != FTM_OK) return s;
    ftm_rt::MatvecIO io;
    io.x = x;
    io.y = y;
    const ftm_rt::Workspace ws = ftm_rt::carve_workspace(op, base, nrhs, adj, ex.p);
    return ftm_rt::run_matvec(op, adj, ex, io, nrhs, ws, reinterpret_cast<hipStream_t>(stream));
  } catch (...) {
    return fail(FTM_ERR_INVALID, "unexpected exception in ftm_apply_scratch");
  }
}

ftm_status ftm_matvec(ftm_operator op, const double* m, double* d, int64_t nrhs, void* stream) {
  return matvec_common(op, false, m, d, nrhs, stream);
}

ftm_status ftm_rmatvec(ftm_operator op, const double* d, double* m, int64_t nrhs, void* stream) {
  return matvec_common(op, true, d, m, nrhs, stream);
}

ftm_status ftm_round(int32_t dtype, int32_t from_f32, const double* x, double* y, int64_t n, void* stream) {
  if (!valid_dtype(dtype)) return fail(FTM_ERR_INVALID, "dtype must be an ftm_dtype");
  if (n < 0) return fail(FTM_ERR_INVALID, "n must be >= 0");
  if (n == 0) return FTM_OK;
  if (!x || !y) return fail(FTM_ERR_INVALID, "x or y is NULL");
  FTM_HIP(launch_round_values(dtype, from_f32 != 0, x, y, n, reinterpret_cast<hipStream_t>(stream)));
  return FTM_OK;
}

ftm_status ftm_get_spectrum(ftm_operator op, int32_t which, int64_t k0, int64_t nk, double* out, void* stream) {
  if (!op || !out) return fail(FTM_ERR_INVALID, "operator or out is NULL");
  if (!valid_dtype(which)) return fail(FTM_ERR_INVALID, "which must be an ftm_dtype");
  if (k0 < 0 || nk < 1 || k0 + nk > op->K) return fail(FTM_ERR_INVALID, "bins out of range");
  if (!op->spec[which].p) return fail(FTM_ERR_UNSUPPORTED, "no spectrum stored in that format");
  DeviceGuard g(op->device);
  const char* src = reinterpret_cast<const char*>(op->spec[which].p) +
                    (size_t)k0 * op->Nd * op->ldm * dtype_bytes(which);
  FTM_HIP(launch_widen_spectrum(src, which, out, nk * op->Nd, op->Nm, op->ldm,
                                reinterpret_cast<hipStream_t>(stream)));
  return FTM_OK;
}

ftm_status ftm_operator_info(ftm_operator op, int64_t* Nt, int64_t* Nd, int64_t* Nm, int64_t* L,
                             size_t* device_bytes) {
  if (!op) return fail(FTM_ERR_INVALID, "operator is NULL");
  if (Nt) *Nt = op->Nt;
  if (Nd) *Nd = op->Nd;
  if (Nm) *Nm = op->Nm;
  if (L) *L = op->L;
  if (device_bytes) *device_bytes = op->bytes();
  return FTM_OK;
}

ftm_status ftm_set_rhs_mode(ftm_operator op, int32_t mode) {
  if (!op) return fail(FTM_ERR_INVALID, "operator is NULL");
  if (mode < FTM_RHS_AUTO || mode > FTM_RHS_GEMM) return fail(FTM_ERR_INVALID, "unknown rhs mode");
  std::lock_guard<std::mutex> lk(op->mu);
  op->rhs_mode = mode;
  return FTM_OK;
}

ftm_status ftm_set_gemm_crossover(ftm_operator op, int64_t min_rhs) {
  if (!op) return fail(FTM_ERR_INVALID, "operator is NULL");
  if (min_rhs < 2) return fail(FTM_ERR_INVALID, "the crossover is at least 2 right-hand sides");
  std::lock_guard<std::mutex> lk(op->mu);
  for (auto& d : op->gemm_min_rhs)
    for (auto& v : d) v = min_rhs;
  return FTM_OK;
}

ftm_status ftm_profile_enable(ftm_operator op, int32_t enable) {
  if (!op) return fail(FTM_ERR_INVALID, "operator is NULL");
  std::lock_guard<std::mutex> lk(op->mu);
  op->profiling = enable != 0;
  return FTM_OK;
}

ftm_status ftm_profile_read(ftm_operator op, double* ms, int64_t* counts, int32_t reset) {
  if (!op) return fail(FTM_ERR_INVALID, "operator is NULL");
  double acc[6] = {0, 0, 0, 0, 0, 0};
  int64_t cnt[2] = {0, 0};
  DeviceGuard g(op->device);
  std::lock_guard<std::mutex> lk(op->mu);
  for (const auto& r : op->recs) {
    bool ok = true;
    for (hipEvent_t e : r.ev) ok = ok && e != nullptr;
    if (!ok) continue;
    FTM_HIP(hipEventSynchronize(r.ev[3]));
    for (int i = 0; i < 3; ++i) {
      float t = 0.f;
      FTM_HIP(hipEventElapsedTime(&t, r.ev[i], r.ev[i + 1]));
      acc[r.dir * 3 + i] += t;
    }
    cnt[r.dir] += 1;
  }
  if (ms)
    for (int i = 0; i < 6; ++i) ms[i] = acc[i];
  if (counts) {
    counts[0] = cnt[0];
    counts[1] = cnt[1];
  }
  if (reset) {
    for (auto& r : op->recs)
      for (hipEvent_t e : r.ev)
        if (e) op->event_pool.push_back(e);
    op->recs.clear();
  }
  return FTM_OK;
}

ftm_status ftm_autotune(ftm_operator op, int32_t reps, void* stream) {
  if (!op) return fail(FTM_ERR_INVALID, "operator is NULL");
  if (reps < 1 || reps > 1000) return fail(FTM_ERR_INVALID, "reps must be in [1, 1000]");
  DeviceGuard g(op->device);
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  const size_t nx = (size_t)op->Nt * (size_t)(op->Nm > op->Nd ? op->Nm : op->Nd);
  DevBuf x, y;
  ftm_status s;
  if ((s = dev_alloc(&x, nx * 8)) != FTM_OK) return s;
  if ((s = dev_alloc(&y, nx * 8)) != FTM_OK) {
    dev_free(&x);
    return s;
  }
  hipEvent_t e0 = nullptr, e1 = nullptr;
  auto done = [&](ftm_status r) {
    (void)hipStreamSynchronize(st);
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    dev_free(&x);
    dev_free(&y);
    return r;
  };
  // any finite pattern does: the kernels' speed does not depend on the values
  if (hipMemsetAsync(x.p, 0x3f, x.n, st) != hipSuccess) return done(fail(FTM_ERR_HIP, "hipMemsetAsync"));
  if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess)
    return done(fail(FTM_ERR_HIP, "hipEventCreate"));
  ftm_rt::Workspace ws;
  ws.mhat = op->mhat.p;
  ws.dhat = op->dhat.p;
  ftm_rt::MatvecIO io;
  io.x = reinterpret_cast<const double*>(x.p);
  io.y = reinterpret_cast<double*>(y.p);
  // time one configuration: one warm call, then reps timed calls
  auto time_exec = [&](bool adj, const ftm_rt::Exec& ex, double* ms) -> ftm_status {
    ftm_status r = ftm_rt::run_matvec(op, adj, ex, io, 1, ws, st);
    if (r != FTM_OK) return r;
    (void)hipEventRecord(e0, st);
    for (int i = 0; i < reps; ++i) ftm_rt::run_matvec(op, adj, ex, io, 1, ws, st);
    (void)hipEventRecord(e1, st);
    if (hipEventSynchronize(e1) != hipSuccess) return fail(FTM_ERR_HIP, "hipEventSynchronize");
    float t = 0.f;
    (void)hipEventElapsedTime(&t, e0, e1);
    *ms = t / reps;
    return FTM_OK;
  };
  // coordinate search per direction: the product's tile, then the input and
  // the output transform's kernel, each with the others at their best so far
  ftm_rt::Exec best[2];
  double best_t[2] = {0.0, 0.0};
  const bool fixed = fft_has_fixed((int)op->L);
  for (int dir = 0; dir < 2; ++dir) {
    ftm_rt::Exec ex = op->exec(dir == 1, 1, false);
    ex.use_gemm = false;
    double bt = 1e300;
    ftm_rt::Exec b = ex;
    for (int v = 0; v < GEMV_VARIANTS; ++v) {
      ex.gemv_variant = v;
      double t;
      if ((s = time_exec(dir == 1, ex, &t)) != FTM_OK) return done(s);
      if (t < bt) { bt = t; b = ex; }
    }
    ex = b;
    for (int side = 0; side < 2; ++side) {
      for (int sh = fixed ? 1 : FFT_SHAPE_GENERIC; sh < FFT_SHAPES; ++sh) {
        (side == 0 ? ex.fft_shape_in : ex.fft_shape_out) = sh;
        double t;
        if ((s = time_exec(dir == 1, ex, &t)) != FTM_OK) return done(s);
        if (t < bt) { bt = t; b = ex; }
      }
      ex = b;
    }
    best[dir] = b;
    best_t[dir] = bt;
  }
  // The FP32-storage GEMM's instructions (float32 accumulation only): the
  // faster of the FP32 MFMA and the split-term BF16 MFMA at 64 right-hand
  // sides.  Then the GEMV <-> GEMM crossover per direction: the smallest
  // batch of 2 .. 32 right-hand sides for which the matrix-core product (at
  // its default tile) is no slower than one matrix-vector product per vector
  // (33: never up to 32).
  constexpr int kMaxProbe = 32, kKindProbe = 64;
  int64_t cross[2] = {2, 2};
  {
    DevBuf xb, yb, wb;
    const size_t nbig = (size_t)kKindProbe * nx * 8;
    size_t wbytes = 0;
    for (int dir = 0; dir < 2; ++dir) {
      const size_t w = op->workspace_bytes(kKindProbe, dir == 1, best[dir].p);
      wbytes = w > wbytes ? w : wbytes;
    }
    if ((s = dev_alloc(&xb, nbig)) != FTM_OK) return done(s);
    if ((s = dev_alloc(&yb, nbig)) != FTM_OK || (s = dev_alloc(&wb, wbytes)) != FTM_OK) {
      dev_free(&xb);
      dev_free(&yb);
      return done(s);
    }
    auto release_probe = [&](ftm_status r) {
      (void)hipStreamSynchronize(st);
      dev_free(&xb);
      dev_free(&yb);
      dev_free(&wb);
      return done(r);
    };
    if (hipMemsetAsync(xb.p, 0x3f, xb.n, st) != hipSuccess) return release_probe(fail(FTM_ERR_HIP, "hipMemsetAsync"));
    ftm_rt::MatvecIO pio;
    pio.x = reinterpret_cast<const double*>(xb.p);
    pio.y = reinterpret_cast<double*>(yb.p);
    auto time_batch = [&](int dir, const ftm_rt::Exec& ex, int n, double* ms) -> ftm_status {
      const ftm_rt::Workspace pws = ftm_rt::carve_workspace(op, wb.p, n, dir == 1, ex.p);
      ftm_status r = ftm_rt::run_matvec(op, dir == 1, ex, pio, n, pws, st);
      if (r != FTM_OK) return r;
      (void)hipEventRecord(e0, st);
      for (int i = 0; i < reps; ++i) ftm_rt::run_matvec(op, dir == 1, ex, pio, n, pws, st);
      (void)hipEventRecord(e1, st);
      if (hipEventSynchronize(e1) != hipSuccess) return fail(FTM_ERR_HIP, "hipEventSynchronize");
      float t = 0.f;
      (void)hipEventElapsedTime(&t, e0, e1);
      *ms = t;
      return FTM_OK;
    };
    for (int dir = 0; dir < 2; ++dir) {
      if (best[dir].p.gemv != DT_F32 || best[dir].p.accum == DT_F64) continue;
      double tk[2] = {0.0, 0.0};
      for (int kind = 1; kind <= 2; ++kind) {
        ftm_rt::Exec ex = best[dir];
        ex.use_gemm = true;
        ex.gemm_tile = 0;
        ex.gemm_kind = kind;
        ftm_status r = time_batch(dir, ex, kKindProbe, &tk[kind - 1]);
        if (r != FTM_OK) return release_probe(r);
      }
      best[dir].gemm_kind = tk[1] < tk[0] ? 2 : 1;
    }
    for (int dir = 0; dir < 2; ++dir) {
      cross[dir] = kMaxProbe + 1;
      for (int n = 2; n <= kMaxProbe; n *= 2) {
        double t_gemm = 0.0, t_gemv = 0.0;
        for (int g = 0; g < 2; ++g) {
          ftm_rt::Exec ex = best[dir];
          ex.use_gemm = g == 0;
          ex.gemm_tile = 0;
          ftm_status r = time_batch(dir, ex, n, g == 0 ? &t_gemm : &t_gemv);
          if (r != FTM_OK) return release_probe(r);
        }
        if (t_gemm <= t_gemv) {
          cross[dir] = n;
          break;
        }
      }
    }
    (void)hipStreamSynchronize(st);
    dev_free(&xb);
    dev_free(&yb);
    dev_free(&wb);
  }
  {
    // keep the winners for the formats they were timed with
    std::lock_guard<std::mutex> lk(op->mu);
    for (int dir = 0; dir < 2; ++dir) {
      const ftm_precision& p = best[dir].p;
      op->variant[dir][p.gemv] = best[dir].gemv_variant;
      op->fft_shape[dir][0][p.fft == DT_F64 ? 1 : 0] = best[dir].fft_shape_in;
      op->fft_shape[dir][1][p.ifft == DT_F64 ? 1 : 0] = best[dir].fft_shape_out;
      op->gemm_min_rhs[dir][p.gemv] = cross[dir];
      op->gemm_kind[dir] = best[dir].gemm_kind;
      op->tuned_ms[dir] = best_t[dir];
    }
  }
  return done(FTM_OK);
}

// Error model of a configuration, shaped after eq. (error) with unit
// constants: the largest unit roundoff among its phases divided by 64 is a
// floor below which no measured error of the configuration is expected.
static double unit_roundoff(int dt) {
  switch (dt) {
    case DT_F32: return std::ldexp(1.0, -24);
    case DT_F16: return std::ldexp(1.0, -11);
    case DT_BF16: return std::ldexp(1.0, -8);
    default: return std::ldexp(1.0, -53);
  }
}

ftm_status ftm_select_precision(ftm_operator op, int32_t adjoint, double tolerance, const double* probe, int32_t reps,
                                ftm_precision* chosen, double* rel_err, double* ms, void* stream) {
  if (!op || !probe) return fail(FTM_ERR_INVALID, "operator or probe is NULL");
  if (!(tolerance > 0.0)) return fail(FTM_ERR_INVALID, "tolerance must be > 0");
  if (reps < 1 || reps > 1000) return fail(FTM_ERR_INVALID, "reps must be in [1, 1000]");
  if (!op->spec[DT_F64].p)
    return fail(FTM_ERR_UNSUPPORTED, "the float64 spectrum (the error reference) was not kept at setup");
  const bool adj = adjoint != 0;
  DeviceGuard g(op->device);
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  const int64_t ny = op->Nt * (adj ? op->Nm : op->Nd);
  const ftm_precision kRef = {DT_F64, DT_F64, DT_F64, DT_F64, DT_F64, DT_F64};
  size_t wmax = 0;
  std::vector<ftm_precision> cand;
  for (int code = 0; code < 1024; ++code) {
    ftm_precision p;
    int32_t* f[5] = {&p.pad, &p.fft, &p.gemv, &p.ifft, &p.unpad};
    double umax = 0.0;
    for (int i = 0, c = code; i < 5; ++i, c >>= 2) {
      *f[i] = c & 3;
      umax = std::max(umax, unit_roundoff(c & 3));
    }
    if (!op->spec[p.gemv].p) continue;            // its spectrum copy was not kept
    if (code != 0 && umax / 64 > tolerance) continue;  // coarser than the tolerance allows
    for (int acc = 0; acc < 2; ++acc) {
      p.accum = acc == 0 ? (p.gemv == DT_F64 ? DT_F64 : DT_F32) : DT_F64;
      if (acc == 1 && p.gemv != DT_F32) continue;  // float64 accumulation of FP32 storage only
      cand.push_back(p);
      wmax = std::max(wmax, op->workspace_bytes(1, adj, p));
    }
  }
  DevBuf yref, y, ws, part;
  constexpr int kBlocks = 256;
  ftm_status s;
  auto done = [&](ftm_status r) {
    (void)hipStreamSynchronize(st);
    dev_free(&yref);
    dev_free(&y);
    dev_free(&ws);
    dev_free(&part);
    return r;
  };
  if ((s = dev_alloc(&yref, ny * 8)) != FTM_OK || (s = dev_alloc(&y, ny * 8)) != FTM_OK ||
      (s = dev_alloc(&ws, wmax)) != FTM_OK || (s = dev_alloc(&part, 2 * kBlocks * 8)) != FTM_OK)
    return done(s);
  ftm_rt::Exec base = op->exec(adj, 1, false);
  base.use_gemm = false;
  ftm_rt::MatvecIO io;
  io.x = probe;
  auto run = [&](const ftm_precision& p, double* out) -> ftm_status {
    ftm_rt::Exec ex = base;
    ex.p = p;
    io.y = out;
    return ftm_rt::run_matvec(op, adj, ex, io, 1, ftm_rt::carve_workspace(op, ws.p, 1, adj, p), st);
  };
  if ((s = run(kRef, reinterpret_cast<double*>(yref.p))) != FTM_OK) return done(s);
  std::vector<double> host(2 * kBlocks);
  hipEvent_t e0 = nullptr, e1 = nullptr;
  if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
    if (e0) (void)hipEventDestroy(e0);
    return done(fail(FTM_ERR_HIP, "hipEventCreate"));
  }
  auto done_ev = [&](ftm_status r) {
    (void)hipStreamSynchronize(st);
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    return done(r);
  };
  ftm_precision best = kRef;
  double best_ms = 1e300, best_err = 0.0;
  for (const ftm_precision& p : cand) {
    // error against the float64 result on the probe
    if ((s = run(p, reinterpret_cast<double*>(y.p))) != FTM_OK) return done_ev(s);
    if (launch_sumsq_diff(reinterpret_cast<const double*>(y.p), reinterpret_cast<const double*>(yref.p), ny,
                          reinterpret_cast<double*>(part.p), kBlocks, st) != hipSuccess)
      return done_ev(fail(FTM_ERR_HIP, "error reduction launch"));
    if (hipMemcpyAsync(host.data(), part.p, part.n, hipMemcpyDeviceToHost, st) != hipSuccess ||
        hipStreamSynchronize(st) != hipSuccess)
      return done_ev(fail(FTM_ERR_HIP, "error reduction copy"));
    double num = 0.0, den = 0.0;
    for (int b = 0; b < kBlocks; ++b) {
      num += host[2 * b];
      den += host[2 * b + 1];
    }
    const double err = den > 0.0 ? std::sqrt(num / den) : std::sqrt(num);
    if (!(err <= tolerance)) continue;
    // time the configurations within the tolerance
    (void)hipEventRecord(e0, st);
    for (int i = 0; i < reps; ++i)
      if ((s = run(p, reinterpret_cast<double*>(y.p))) != FTM_OK) return done_ev(s);
    (void)hipEventRecord(e1, st);
    if (hipEventSynchronize(e1) != hipSuccess) return done_ev(fail(FTM_ERR_HIP, "hipEventSynchronize"));
    float t = 0.f;
    (void)hipEventElapsedTime(&t, e0, e1);
    const double tm = (double)t / reps;
    if (tm < best_ms || (tm == best_ms && err < best_err)) {
      best_ms = tm;
      best_err = err;
      best = p;
    }
  }
  {
    std::lock_guard<std::mutex> lk(op->mu);
    (adj ? op->adj : op->fwd) = best;
  }
  if (chosen) *chosen = best;
  if (rel_err) *rel_err = best_err;
  if (ms) *ms = best_ms;
  return done_ev(FTM_OK);
}

ftm_status ftm_get_tuning(ftm_operator op, ftm_tuning* out) {
  if (!op || !out) return fail(FTM_ERR_INVALID, "operator or out is NULL");
  std::lock_guard<std::mutex> lk(op->mu);
  for (int dir = 0; dir < 2; ++dir) {
    const ftm_precision& p = dir ? op->adj : op->fwd;
    out->gemv_variant[dir] = op->variant[dir][p.gemv];
    out->fft_shape[dir][0] = op->fft_shape[dir][0][p.fft == DT_F64 ? 1 : 0];
    out->fft_shape[dir][1] = op->fft_shape[dir][1][p.ifft == DT_F64 ? 1 : 0];
    out->gemm_tile[dir] = op->gemm_tile[dir][p.gemv];
    out->gemm_kind[dir] = op->gemm_kind[dir];
    out->gemm_min_rhs[dir] = op->gemm_min_rhs[dir][p.gemv];
    out->ms[dir] = op->tuned_ms[dir];
  }
  return FTM_OK;
}

ftm_status ftm_set_tuning(ftm_operator op, const ftm_tuning* t) {
  if (!op || !t) return fail(FTM_ERR_INVALID, "operator or tuning is NULL");
  for (int dir = 0; dir < 2; ++dir) {
    if (t->gemv_variant[dir] < 0 || t->gemv_variant[dir] >= GEMV_VARIANTS)
      return fail(FTM_ERR_INVALID, "gemv_variant out of range");
    for (int side = 0; side < 2; ++side)
      if (t->fft_shape[dir][side] < 0 || t->fft_shape[dir][side] >= FFT_SHAPES)
        return fail(FTM_ERR_INVALID, "fft_shape out of range");
    const int gt = t->gemm_tile[dir];
    if (gt != 0 && gt != 16 && gt != 32 && gt != 64) return fail(FTM_ERR_INVALID, "gemm_tile must be 0, 16, 32 or 64");
    if (t->gemm_kind[dir] < 0 || t->gemm_kind[dir] > 2) return fail(FTM_ERR_INVALID, "gemm_kind must be 0, 1 or 2");
    if (t->gemm_min_rhs[dir] < 2) return fail(FTM_ERR_INVALID, "gemm_min_rhs must be >= 2");
  }
  std::lock_guard<std::mutex> lk(op->mu);
  for (int dir = 0; dir < 2; ++dir) {
    const ftm_precision& p = dir ? op->adj : op->fwd;
    op->variant[dir][p.gemv] = t->gemv_variant[dir];
    op->fft_shape[dir][0][p.fft == DT_F64 ? 1 : 0] = t->fft_shape[dir][0];
    op->fft_shape[dir][1][p.ifft == DT_F64 ? 1 : 0] = t->fft_shape[dir][1];
    op->gemm_tile[dir][p.gemv] = t->gemm_tile[dir];
    op->gemm_kind[dir] = t->gemm_kind[dir];
    op->gemm_min_rhs[dir][p.gemv] = t->gemm_min_rhs[dir];
  }
  return FTM_OK;
}

struct ftm_graph_s {
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  int device = 0;
};

ftm_status ftm_graph_create(ftm_graph* out, ftm_operator op, int32_t adjoint, const double* x, double* y,
                            int64_t nrhs) {
  if (!out) return fail(FTM_ERR_INVALID, "out is NULL");
  *out = nullptr;
  if (!op || !x || !y) return fail(FTM_ERR_INVALID, "NULL argument");
  if (nrhs < 1 || nrhs > op->max_rhs) return fail(FTM_ERR_INVALID, "nrhs must be in [1, max_rhs]");
  DeviceGuard g(op->device);
  hipStream_t cs = nullptr;
  FTM_HIP(hipStreamCreateWithFlags(&cs, hipStreamNonBlocking));
  ftm_graph gr = new ftm_graph_s();
  gr->device = op->device;
  ftm_rt::MatvecIO io;
  io.x = x;
  io.y = y;
  ftm_rt::Workspace ws;
  ws.mhat = op->mhat.p;
  ws.dhat = op->dhat.p;
  ftm_status s = FTM_OK;
  hipError_t e = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
  if (e == hipSuccess) {
    // no event records inside the graph
    s = ftm_rt::run_matvec(op, adjoint != 0, op->exec(adjoint != 0, nrhs, false), io, nrhs, ws, cs);
    hipError_t e2 = hipStreamEndCapture(cs, &gr->graph);
    if (s == FTM_OK && e2 != hipSuccess) e = e2;
  }
  if (e == hipSuccess && s == FTM_OK) e = hipGraphInstantiate(&gr->exec, gr->graph, nullptr, nullptr, 0);
  (void)hipStreamDestroy(cs);
  if (e != hipSuccess || s != FTM_OK) {
    if (gr->exec) (void)hipGraphExecDestroy(gr->exec);
    if (gr->graph) (void)hipGraphDestroy(gr->graph);
    delete gr;
    return s != FTM_OK ? s : fail_hip("graph capture", e);
  }
  *out = gr;
  return FTM_OK;
}

ftm_status ftm_graph_launch(ftm_graph g, void* stream) {
  if (!g) return fail(FTM_ERR_INVALID, "graph is NULL");
  DeviceGuard dg(g->device);
  FTM_HIP(hipGraphLaunch(g->exec, reinterpret_cast<hipStream_t>(stream)));
  return FTM_OK;
}

ftm_status ftm_graph_destroy(ftm_graph g) {
  if (!g) return FTM_OK;
  DeviceGuard dg(g->device);
  if (g->exec) (void)hipGraphExecDestroy(g->exec);
  if (g->graph) (void)hipGraphDestroy(g->graph);
  delete g;
  return FTM_OK;
}

ftm_status ftm_destroy_operator(ftm_operator op) {
  if (!op) return FTM_OK;
  DeviceGuard g(op->device);
  release(op);
  delete op;
  return FTM_OK;
}

}  // extern "C"
