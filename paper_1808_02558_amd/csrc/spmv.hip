// Sparse product with the Newton matrix in 3x3 block-CSR form.
//
// The Schur complement S_k = N + blockdiag(H_i) has the block pattern of
// N = D^T M^-1 D: block (i, j) is non-zero iff contacts i and j share a body
// (Sec. 3.3, sparsity of N).  Each block row is one contact slot.
//
// Layout of the work: a group of G lanes owns one block row.  Lane 3j + r
// (j < G/3) takes row r of blocks j, j + G/3, j + 2G/3, ... of that block
// row, so one pass of the group reads G/3 consecutive blocks (a contiguous
// run of 9 G/3 doubles) and each lane needs no index arithmetic beyond a
// multiply.  The three lanes of a block read the same three entries of x.
// The partial sums of the lanes with equal r are added with lane shuffles.
// The identity rows past the last slot (at most two) are copied by the first
// lanes of the grid.
//
// Workgroups are dealt to the 8 XCDs round-robin by workgroup id, and each
// XCD has its own L2.  The id is remapped so that each XCD takes one
// contiguous eighth of the block rows: Morton order keeps the entries of x
// that a range of rows gathers inside a narrow range, so they stay in that
// XCD's L2 instead of being fetched by every XCD.
#include <algorithm>

#include "ops.h"

namespace qtp {
namespace {

constexpr int kBlock = 256;  // threads per workgroup
constexpr int kXcds = 8;

// Bijection from the hardware workgroup id to a logical block such that the
// workgroups of XCD k (ids = k mod 8) cover one contiguous range of blocks.
__device__ inline int64_t xcd_block(int64_t w, int64_t nblk) {
  const int64_t q = nblk / kXcds, rem = nblk % kXcds;
  const int64_t k = w % kXcds, idx = w / kXcds;
  return k * q + (k < rem ? k : rem) + idx;
}

template <int G>
__global__ __launch_bounds__(kBlock) void bsr3_spmv_kernel(
    int nslots, int64_t n, const int32_t* __restrict__ rp,
    const int32_t* __restrict__ col, const double* __restrict__ val,
    const double* __restrict__ x, double* __restrict__ y) {
  constexpr int J = G / 3;  // blocks per pass of the group
  const int lane = threadIdx.x & (G - 1);
  const int j = lane / 3;
  const int r = lane - 3 * j;
  const int64_t gid = xcd_block(blockIdx.x, gridDim.x) * kBlock + threadIdx.x;
  const int64_t row = gid / G;
  double acc = 0.0;
  if (row < nslots && j < J) {
    const int b1 = rp[row + 1];
    int b = rp[row] + j;
    // two blocks per trip so that both blocks' loads are in flight together
    for (; b + J < b1; b += 2 * J) {
      const double* v0 = val + (int64_t)b * 9 + 3 * r;
      const double* v1 = v0 + 9 * J;
      const int c0 = col[b], c1 = col[b + J];
      const double a0 = v0[0], a1 = v0[1], a2 = v0[2];
      const double e0 = v1[0], e1 = v1[1], e2 = v1[2];
      const double* x0 = x + 3 * (int64_t)c0;
      const double* x1 = x + 3 * (int64_t)c1;
      acc += a0 * x0[0] + a1 * x0[1] + a2 * x0[2];
      acc += e0 * x1[0] + e1 * x1[1] + e2 * x1[2];
    }
    if (b < b1) {
      const double* v = val + (int64_t)b * 9 + 3 * r;
      const double* xc = x + 3 * (int64_t)col[b];
      acc += v[0] * xc[0] + v[1] * xc[1] + v[2] * xc[2];
    }
  }
  // lanes r, r + 3, ..., r + 3 (J - 1) of the group hold the parts of row r
  const int src = lane < 3 * J ? r : lane;
  double tot = acc;
#pragma unroll
  for (int q = 1; q < J; ++q) {
    const double t = __shfl(acc, src + 3 * q, G);
    tot += t;
  }
  if (row < nslots && lane < 3) y[3 * row + lane] = tot;
  const int64_t first = 3 * (int64_t)nslots;
  if (gid < n - first) y[first + gid] = x[first + gid];
}

}  // namespace

void bsr_spmv(hipStream_t s, int nslots, int64_t n, const int32_t* rp,
              const int32_t* col, const double* val, const double* x, double* y) {
  constexpr int G = 16;
  const int64_t tail = n - 3 * (int64_t)nslots;
  QTP_REQUIRE(nslots >= 0 && tail >= 0, -1, "bsr_spmv: slots exceed the vector length");
  const int64_t threads = std::max<int64_t>((int64_t)nslots * G, tail);
  if (threads == 0) return;
  bsr3_spmv_kernel<G><<<div_up(threads, kBlock), kBlock, 0, s>>>(nslots, n, rp, col,
                                                                val, x, y);
  QTP_CHECK_LAUNCH();
}

}  // namespace qtp
