// Host runtime internals shared by the C ABI (ftm_api.hip) and the serving
// scheduler (ftm_server.hip): the operator object, error reporting and the
// stream-ordered kernel chain of one matvec.
#pragma once

#include <hip/hip_runtime.h>

#include <mutex>
#include <string>
#include <vector>

#include "ftm.h"
#include "ftm_kernels.h"

namespace ftm_rt {

struct DevBuf {
  void* p = nullptr;
  size_t n = 0;
};

// Device workspace of one matvec: the transformed input and output vectors,
// [K][nrhs][ld] complex each, in the intermediate storage formats of the
// direction's precision configuration.
struct Workspace {
  void* mhat = nullptr;
  void* dhat = nullptr;
};

// Inputs and outputs of one matvec: contiguous [nrhs][Nt][n] arrays, or
// device arrays of nrhs pointers (one [Nt][n] block each) when xptr/yptr are
// set.
struct MatvecIO {
  const double* x = nullptr;
  double* y = nullptr;
  const double* const* xptr = nullptr;
  double* const* yptr = nullptr;
};

// Everything a matvec reads from the operator's mutable configuration, copied
// under the operator's lock when the call is made: a concurrent
// ftm_set_precision / ftm_set_tuning cannot change a call that is being
// enqueued, and its workspace is sized for the configuration it runs.
struct Exec {
  ftm_precision p{};
  int gemv_variant = 0;
  int fft_shape_in = 0, fft_shape_out = 0;  // kernels of the two transforms (0 = default)
  int gemm_tile = 0;                         // right-hand sides per GEMM tile (0 = default)
  int gemm_kind = 0;                         // FP32-storage GEMM instructions (0 = default)
  bool use_gemm = false;
  bool profile = false;  // record HIP events around the kernels
};

}  // namespace ftm_rt

struct ftm_operator_s {
  int64_t Nt = 0, Nd = 0, Nm = 0, L = 0, K = 0;
  int ldm = 0, ldd = 0;  // padded column counts of spectra and workspaces
  int device = 0;
  int64_t max_rhs = 1;
  // length-L plans of the forward (radices in descending order) and inverse
  // (ascending) transforms, with radices up to 8 for float64 compute and up to
  // 16 for float32 (the same radix sets as the fixed-plan kernels), and their
  // per-pass twiddle tables in the compute types.  The runtime-plan kernels
  // run the forward plans.
  ftm::FftPlan plan_f64{}, plan_i64{}, plan_f32{}, plan_i32{};
  ftm_rt::DevBuf tw64f, tw64i, tw32f, tw32i;
  ftm::FftPlans fft_in(bool f64) const {
    return f64 ? ftm::FftPlans{&plan_f64, tw64f.p, &plan_f64, tw64f.p}
               : ftm::FftPlans{&plan_f32, tw32f.p, &plan_f32, tw32f.p};
  }
  ftm::FftPlans fft_out(bool f64) const {
    return f64 ? ftm::FftPlans{&plan_i64, tw64i.p, &plan_f64, tw64f.p}
               : ftm::FftPlans{&plan_i32, tw32i.p, &plan_f32, tw32f.p};
  }
  ftm_rt::DevBuf spec[4];     // Fhat[K][Nd][ldm] per storage format
  ftm_rt::DevBuf mhat, dhat;  // the operator's own workspace, sized for max_rhs

  // Mutable configuration and instrumentation; every access holds mu.
  mutable std::mutex mu;
  ftm_precision fwd{}, adj{};
  int rhs_mode = FTM_RHS_AUTO;
  int64_t gemm_min_rhs[2][4] = {{2, 2, 2, 2}, {2, 2, 2, 2}};  // [direction][storage format] crossover
  int variant[2][4] = {{0, 0, 0, 0}, {0, 0, 0, 0}};          // [direction][storage format] tile variant
  int gemm_tile[2][4] = {{0, 0, 0, 0}, {0, 0, 0, 0}};        // [direction][storage format] GEMM tile
  int gemm_kind[2] = {0, 0};                                  // [direction] FP32-storage GEMM instructions
  int fft_shape[2][2][2] = {};  // [direction][input / output transform][float64 compute] transform kernel
  double tuned_ms[2] = {0.0, 0.0};
  bool profiling = false;
  struct Rec {
    int dir;
    hipEvent_t ev[4];
  };
  std::vector<Rec> recs;
  std::vector<hipEvent_t> event_pool;

  size_t bytes() const {
    size_t b = tw64f.n + tw64i.n + tw32f.n + tw32i.n + mhat.n + dhat.n;
    for (const auto& s : spec) b += s.n;
    return b;
  }
  static size_t round256(size_t n) { return (n + 255) / 256 * 256; }
  // bytes per complex entry of m-hat and d-hat in one direction of
  // configuration p: float64 (16) where both neighbouring phases are float64,
  // else float32 (8)
  static void workspace_elems(const ftm_precision& p, bool adjoint, int* em, int* ed) {
    const int ex = (p.fft == 0 && p.gemv == 0) ? 16 : 8;   // transformed input
    const int ey = (p.gemv == 0 && p.ifft == 0) ? 16 : 8;  // transformed output
    *em = adjoint ? ey : ex;
    *ed = adjoint ? ex : ey;
  }
  // workspace bytes of one matvec of nrhs right-hand sides in one direction at
  // configuration p (a multiple of 256: m-hat, then d-hat at a 256-byte offset)
  size_t workspace_bytes(int64_t nrhs, bool adjoint, const ftm_precision& p) const {
    int em, ed;
    workspace_elems(p, adjoint, &em, &ed);
    return round256((size_t)K * nrhs * ldm * em) + round256((size_t)K * nrhs * ldd * ed);
  }
  // the copy of the direction's configuration a call runs with (locks mu)
  ftm_rt::Exec exec(bool adjoint, int64_t nrhs, bool allow_profile) const;
};

namespace ftm_rt {

ftm_status fail(ftm_status s, const std::string& msg);
ftm_status fail_hip(const char* what, hipError_t e);

#define FTM_HIP(expr)                                         \
  do {                                                        \
    hipError_t e_ = (expr);                                   \
    if (e_ != hipSuccess) return ftm_rt::fail_hip(#expr, e_); \
  } while (0)

class DeviceGuard {
 public:
  explicit DeviceGuard(int dev) {
    if (hipGetDevice(&old_) == hipSuccess && old_ != dev) {
      if (hipSetDevice(dev) == hipSuccess) switched_ = true;
    }
  }
  ~DeviceGuard() {
    if (switched_) (void)hipSetDevice(old_);
  }

 private:
  int old_ = 0;
  bool switched_ = false;
};

// Split a workspace block of op->workspace_bytes(nrhs, adjoint, p) bytes.
Workspace carve_workspace(const ftm_operator_s* op, void* base, int64_t nrhs, bool adjoint, const ftm_precision& p);

// Enqueue one matvec (phases 1-5) on st with the configuration ex.  No
// argument checks: callers validate.
ftm_status run_matvec(ftm_operator op, bool adjoint, const Exec& ex, const MatvecIO& io, int64_t nrhs,
                      const Workspace& ws, hipStream_t st);

}  // namespace ftm_rt
