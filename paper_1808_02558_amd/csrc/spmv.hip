// Sparse product with the Newton matrix in 3x3 block-CSR form.
//
// The Schur complement S_k = N + blockdiag(H_i) has the block pattern of
// N = D^T M^-1 D: block (i, j) is non-zero iff contacts i and j share a body
// (Sec. 3.3, sparsity of N).  Each block row is one contact slot.
//
// Layout of the work: GROUP lanes of a wavefront own one block row and stream
// its values as one flat, contiguous run of doubles (9 per block), so the
// dominant value stream is read with fully coalesced loads; each value
// gathers one entry of x through the block's column index.  The three row
// sums are reduced across the group with lane shuffles.
#include "ops.h"

namespace qtp {
namespace {

constexpr int kGroup = 16;   // lanes per block row
constexpr int kBlock = 256;  // threads per workgroup

__global__ __launch_bounds__(kBlock) void bsr3_spmv_kernel(
    int nslots, const int32_t* __restrict__ rp, const int32_t* __restrict__ col,
    const double* __restrict__ val, const double* __restrict__ x,
    double* __restrict__ y) {
  const int lane = threadIdx.x & (kGroup - 1);
  const int64_t row = ((int64_t)blockIdx.x * kBlock + threadIdx.x) / kGroup;
  double a0 = 0.0, a1 = 0.0, a2 = 0.0;
  if (row < nslots) {
    const int64_t e0 = (int64_t)rp[row] * 9;
    const int64_t e1 = (int64_t)rp[row + 1] * 9;
    for (int64_t e = e0 + lane; e < e1; e += kGroup) {
      const int64_t b = e / 9;
      const int w = (int)(e - b * 9);
      const int r = w / 3;
      const int c = w - 3 * r;
      const double p = val[e] * x[3 * (int64_t)col[b] + c];
      a0 += (r == 0) ? p : 0.0;
      a1 += (r == 1) ? p : 0.0;
      a2 += (r == 2) ? p : 0.0;
    }
  }
#pragma unroll
  for (int o = kGroup / 2; o > 0; o >>= 1) {
    a0 += __shfl_xor(a0, o, kGroup);
    a1 += __shfl_xor(a1, o, kGroup);
    a2 += __shfl_xor(a2, o, kGroup);
  }
  if (row < nslots && lane < 3) {
    const double v = lane == 0 ? a0 : (lane == 1 ? a1 : a2);
    y[3 * row + lane] = v;
  }
}

__global__ void identity_tail_kernel(int64_t first, int64_t n,
                                     const double* __restrict__ x,
                                     double* __restrict__ y) {
  const int64_t i = first + (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) y[i] = x[i];
}

}  // namespace

void bsr_spmv(hipStream_t s, int nslots, int64_t n, const int32_t* rp,
              const int32_t* col, const double* val, const double* x, double* y) {
  if (nslots > 0) {
    const int64_t threads = (int64_t)nslots * kGroup;
    bsr3_spmv_kernel<<<div_up(threads, kBlock), kBlock, 0, s>>>(nslots, rp, col,
                                                                val, x, y);
    QTP_CHECK_LAUNCH();
  }
  const int64_t first = 3 * (int64_t)nslots;
  if (first < n) {
    identity_tail_kernel<<<div_up(n - first, 256), 256, 0, s>>>(first, n, x, y);
    QTP_CHECK_LAUNCH();
  }
}

}  // namespace qtp
