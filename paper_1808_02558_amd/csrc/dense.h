// Dense FP64 building blocks used by the QTT construction (dense.hip).
#pragma once

#include "common.h"

namespace qtp {

struct Workspace {
  void* ptr = nullptr;
  size_t bytes = 0;
};

// C = alpha op(A) op(B) + beta C (row-major).  With ws, tall-K products are
// split over K into ws and reduced in a fixed order.
void gemm(hipStream_t s, int transA, int transB, int M, int N, int K,
          double alpha, const double* A, int64_t lda, const double* B,
          int64_t ldb, double beta, double* C, int64_t ldc, Workspace* ws);

// Eigen-decomposition of the symmetric n x n matrix A (destroyed), n even,
// 2 <= n <= 256: wsorted[n] eigenvalues in decreasing order and Vsorted
// (n x n row-major) with the matching eigenvectors as columns.  V and w are
// scratch of n*n and n doubles.
void sym_eig(hipStream_t s, int n, double* A, double* V, double* w,
             double* wsorted, double* Vsorted);

// out[i] = sum_{j < i} in[j]
void exclusive_scan(hipStream_t s, const int* in, int* out, int64_t n,
                    DevBuf& tmp);

// Stable ascending sort of (keys, vals) by the low key_bits bits of keys.
void radix_sort_pairs(hipStream_t s, uint64_t* keys, int32_t* vals, int64_t n,
                      int key_bits, DevBuf& tmp_keys, DevBuf& tmp_vals,
                      DevBuf& tmp_hist, DevBuf& tmp_scan);

}  // namespace qtp
