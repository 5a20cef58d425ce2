// QTT matrix-vector product y = A x (Sec. 3.2, "Fast arithmetic and TT direct
// solvers": contract one tensor dimension at a time with the k-th core).
//
// x is viewed as a tensor [2]^d with the most significant bit first (Sec. 3.1
// index convention).  After step k the intermediate is
//   Z_k[I][i_k][beta][J],  I = (i_1..i_{k-1}), J = (j_{k+1}..j_d),
//   Z_k[I][i_k][beta][J] = sum_{alpha, j_k} G_k(alpha, i_k, j_k, beta)
//                                          Z_{k-1}[I][alpha][j_k][J],
// stored row-major, so step k is a batched product of the (2 r_k) x (2 r_{k-1})
// matrix W_k[(i,beta)][(alpha,j)] with 2^{k-1} blocks of 2^{d-k} columns.
//
// One thread owns one column (I, J) of a step and a tile of TB outputs; the
// core entries it multiplies are the same for every thread of the launch,
// so they are read through the scalar cache, while the column entries are
// read with coalesced vector loads (consecutive threads, consecutive J).
#include <hip/hip_bf16.h>

#include "ops.h"

namespace qtp {
namespace {

constexpr int kThreads = 256;
constexpr int kTile = 16;

template <class T> struct CoreLoad;
template <> struct CoreLoad<double> {
  using acc = double;
  __device__ static double get(const double* p, int64_t i) { return p[i]; }
};
template <> struct CoreLoad<float> {
  using acc = float;
  __device__ static float get(const float* p, int64_t i) { return p[i]; }
};
struct bf16_t { uint16_t bits; };
template <> struct CoreLoad<bf16_t> {
  using acc = float;
  __device__ static float get(const bf16_t* p, int64_t i) {
    return __uint_as_float(((uint32_t)p[i].bits) << 16);
  }
};

// One contraction step.  in: [P][ra][2][J], out: [P][2][rb][J], P*J = ncols.
template <class CT, class IT, class OT>
__global__ __launch_bounds__(kThreads) void qtt_step_kernel(
    const CT* __restrict__ core, int ra, int rb, int log2J, int64_t ncols,
    int ntile, const IT* __restrict__ in, OT* __restrict__ out) {
  using AT = typename CoreLoad<CT>::acc;
  const int64_t c = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  if (c >= ncols) return;
  const int64_t J = (int64_t)1 << log2J;
  const int64_t p = c >> log2J;
  const int64_t jj = c & (J - 1);
  const int i = blockIdx.y / ntile;
  const int b0 = (blockIdx.y % ntile) * kTile;
  const int nb = min(kTile, rb - b0);
  AT acc[kTile];
#pragma unroll
  for (int t = 0; t < kTile; ++t) acc[t] = AT(0);
  const IT* src = in + (p * ra * 2) * J + jj;
  for (int a = 0; a < ra; ++a) {
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      const AT xv = (AT)src[(int64_t)(2 * a + j) * J];
      const int64_t cbase = ((int64_t)(a * 2 + i) * 2 + j) * rb + b0;
#pragma unroll
      for (int t = 0; t < kTile; ++t)
        if (t < nb) acc[t] += CoreLoad<CT>::get(core, cbase + t) * xv;
    }
  }
  OT* dst = out + ((p * 2 + i) * rb + b0) * J + jj;
#pragma unroll
  for (int t = 0; t < kTile; ++t)
    if (t < nb) dst[(int64_t)t * J] = (OT)acc[t];
}

template <class CT, class IT, class OT>
void launch_step(hipStream_t s, const CT* core, int ra, int rb, int d, int k,
                 const IT* in, OT* out) {
  // k is 1-based; J = 2^{d-k}; columns = 2^{k-1} * 2^{d-k} = 2^{d-1}
  const int log2J = d - k;
  const int64_t ncols = (int64_t)1 << (d - 1);
  const int ntile = div_up(rb, kTile);
  dim3 grid(div_up(ncols, kThreads), 2 * ntile);
  qtt_step_kernel<CT, IT, OT><<<grid, kThreads, 0, s>>>(core, ra, rb, log2J,
                                                        ncols, ntile, in, out);
  QTP_CHECK_LAUNCH();
}

template <class CT, class IT>
void apply_impl(hipStream_t s, int d, const int32_t* ranks, const CT* cores,
                const double* x, double* y, void* work) {
  const std::vector<int64_t> off = core_offsets(d, ranks);
  const int64_t N = (int64_t)1 << d;
  int64_t maxr = 1;
  for (int k = 0; k <= d; ++k) maxr = ranks[k] > maxr ? ranks[k] : maxr;
  IT* buf[2] = {static_cast<IT*>(work), static_cast<IT*>(work) + N * maxr};
  if (d == 1) {
    launch_step<CT, double, double>(s, cores, 1, 1, d, 1, x, y);
    return;
  }
  launch_step<CT, double, IT>(s, cores + off[0], ranks[0], ranks[1], d, 1, x,
                              buf[0]);
  int cur = 0;
  for (int k = 2; k < d; ++k) {
    launch_step<CT, IT, IT>(s, cores + off[k - 1], ranks[k - 1], ranks[k], d, k,
                            buf[cur], buf[cur ^ 1]);
    cur ^= 1;
  }
  launch_step<CT, IT, double>(s, cores + off[d - 1], ranks[d - 1], ranks[d], d,
                              d, buf[cur], y);
}

}  // namespace

std::vector<int64_t> core_offsets(int d, const int32_t* ranks) {
  std::vector<int64_t> off(d + 1, 0);
  for (int k = 0; k < d; ++k)
    off[k + 1] = off[k] + (int64_t)ranks[k] * 4 * ranks[k + 1];
  return off;
}

size_t qtt_apply_workspace(int d, const int32_t* ranks, int prec) {
  int64_t maxr = 1;
  for (int k = 0; k <= d; ++k) maxr = ranks[k] > maxr ? ranks[k] : maxr;
  const size_t es = prec == 0 ? sizeof(double) : sizeof(float);
  return 2 * ((size_t)1 << d) * (size_t)maxr * es;
}

void qtt_apply(hipStream_t s, int d, const int32_t* ranks, const void* cores,
               int prec, const double* x, double* y, void* work) {
  if (prec == 0)
    apply_impl<double, double>(s, d, ranks, static_cast<const double*>(cores), x,
                               y, work);
  else if (prec == 1)
    apply_impl<float, float>(s, d, ranks, static_cast<const float*>(cores), x, y,
                             work);
  else
    apply_impl<bf16_t, float>(s, d, ranks, static_cast<const bf16_t*>(cores), x,
                              y, work);
}

}  // namespace qtp
