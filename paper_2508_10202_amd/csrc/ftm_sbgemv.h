// Launcher of the standalone strided-batched matrix-vector product (BLAS
// column-major semantics; see ftm_sbgemv in ftm.h).  Arguments are validated
// by the caller.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace ftm {

hipError_t launch_sbgemv(int type, int op, int m, int n, const void* alpha, const void* A, int64_t lda, int64_t sa,
                         const void* x, int64_t sx, const void* beta, void* y, int64_t sy, int64_t batch,
                         hipStream_t st);

}  // namespace ftm
