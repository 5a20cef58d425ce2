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

// ---------------------------------------------------------------------------
// Level-fused contraction.  One workgroup owns a prefix I (the row bits
// already produced) and a tile of T consecutive trailing indices J'' and
// applies m consecutive cores with the intermediates in LDS:
//   load   Z[I][alpha][jj (m bits)][J'']        (T contiguous values per run)
//   m x    [ii][alpha][j jr][t] -> [ii i][beta][jr][t]
//   store  Z[I ii (m bits)][beta][J'']
// so an intermediate crosses HBM only between passes.  Each thread forms
// kBT consecutive beta of one output column, reusing every loaded value kBT
// times.
// ---------------------------------------------------------------------------
constexpr int kMaxFuse = 10;
constexpr int kBT = 4;

struct FusePlan {
  int m;                   // levels in this pass
  int ra[kMaxFuse + 1];    // ranks r_{k0-1} .. r_{k0+m-1}
  int64_t coff[kMaxFuse];  // core offsets of levels k0 .. k0+m-1
};

template <class CT, class IT, class OT, class AT>
__global__ __launch_bounds__(kThreads) void qtt_fused_kernel(
    const CT* __restrict__ cores, FusePlan P, int log2T, int log2J, int ntilesJ,
    const IT* __restrict__ in, OT* __restrict__ out) {
  extern __shared__ unsigned char smem_raw[];
  AT* buf0 = reinterpret_cast<AT*>(smem_raw);
  const int m = P.m;
  const int T = 1 << log2T;
  const int64_t Jtot = (int64_t)1 << log2J;
  const int64_t I = blockIdx.x / ntilesJ;
  const int64_t J0 = (int64_t)(blockIdx.x % ntilesJ) << log2T;
  int maxr = 1;
  for (int l = 0; l <= m; ++l) maxr = max(maxr, P.ra[l]);
  AT* buf1 = buf0 + ((int64_t)maxr << (m + log2T));
  // load
  {
    const int rin = P.ra[0];
    const int total = rin << (m + log2T);
    for (int e = threadIdx.x; e < total; e += kThreads) {
      const int t = e & (T - 1);
      const int jj = (e >> log2T) & ((1 << m) - 1);
      const int a = e >> (log2T + m);
      const int64_t gi = (((I * rin + a) << m) + jj) * Jtot + J0 + t;
      buf0[e] = (AT)in[gi];
    }
  }
  __syncthreads();
  AT* cur = buf0;
  AT* nxt = buf1;
  for (int l = 0; l < m; ++l) {
    const int ra = P.ra[l], rb = P.ra[l + 1];
    const CT* G = cores + P.coff[l];
    const int lr = m - l - 1;          // bits of jr
    const int inner = lr + log2T;      // bits of (jr, t)
    const int nbq = (rb + kBT - 1) / kBT;
    const int total = (2 << l) * nbq << inner;  // (ii', beta quad, jr, t)
    for (int e = threadIdx.x; e < total; e += kThreads) {
      const int low = e & ((1 << inner) - 1);  // (jr, t)
      const int bq = (e >> inner) % nbq;
      const int iip = (e >> inner) / nbq;
      const int i = iip & 1;
      const int ii = iip >> 1;
      const int b0 = bq * kBT;
      AT acc[kBT];
#pragma unroll
      for (int q = 0; q < kBT; ++q) acc[q] = AT(0);
      const AT* src = cur + ((int64_t)ii * ra << (lr + 1 + log2T)) + low;
      for (int a = 0; a < ra; ++a) {
#pragma unroll
        for (int j = 0; j < 2; ++j) {
          const AT xv = src[((a << 1) + j) << inner];
          const int64_t cb = (((int64_t)a * 2 + i) * 2 + j) * rb + b0;
#pragma unroll
          for (int q = 0; q < kBT; ++q)
            if (b0 + q < rb) acc[q] += CoreLoad<CT>::get(G, cb + q) * xv;
        }
      }
      AT* dst = nxt + (((int64_t)iip * rb + b0) << inner) + low;
#pragma unroll
      for (int q = 0; q < kBT; ++q)
        if (b0 + q < rb) dst[(int64_t)q << inner] = acc[q];
    }
    __syncthreads();
    AT* tmp = cur;
    cur = nxt;
    nxt = tmp;
  }
  // store: cur is [ii (m bits)][beta][t]
  {
    const int rout = P.ra[m];
    const int total = rout << (m + log2T);
    for (int e = threadIdx.x; e < total; e += kThreads) {
      const int t = e & (T - 1);
      const int b = (e >> log2T) % rout;
      const int ii = (e >> log2T) / rout;
      const int64_t gi = (((I << m) + ii) * rout + b) * Jtot + J0 + t;
      out[gi] = (OT)cur[e];
    }
  }
}

template <class CT, class IT, class OT, class AT>
void launch_fused(hipStream_t s, const CT* cores, const FusePlan& P, int d, int k0,
                  int log2T, const IT* in, OT* out, size_t lds) {
  const int log2J = d - (k0 + P.m - 1);
  const int ntilesJ = 1 << (log2J - log2T);
  const int64_t nblk = ((int64_t)1 << (k0 - 1)) * ntilesJ;
  qtt_fused_kernel<CT, IT, OT, AT><<<(unsigned)nblk, kThreads, lds, s>>>(
      cores, P, log2T, log2J, ntilesJ, in, out);
  QTP_CHECK_LAUNCH();
}

// Greedy pass plan: the longest run of levels whose slab fits the LDS budget.
template <class CT, class IT>
void apply_fused(hipStream_t s, int d, const int32_t* ranks, const CT* cores,
                 const double* x, double* y, void* work) {
  using AT = IT;
  const std::vector<int64_t> off = core_offsets(d, ranks);
  const int64_t N = (int64_t)1 << d;
  int64_t maxr = 1;
  for (int k = 0; k <= d; ++k) maxr = ranks[k] > maxr ? ranks[k] : maxr;
  const size_t budget = 32768 / sizeof(AT);  // elements per LDS buffer
  IT* buf[2] = {static_cast<IT*>(work), static_cast<IT*>(work) + N * maxr};
  int k0 = 1, cur = 0;
  bool first = true;
  while (k0 <= d) {
    int m = std::min(kMaxFuse, d - k0 + 1), log2T = 0;
    for (; m >= 1; --m) {
      const int log2J = d - (k0 + m - 1);
      log2T = std::min(4, log2J);
      int rm = 1;
      for (int l = 0; l <= m; ++l) rm = std::max<int>(rm, ranks[k0 - 1 + l]);
      // enough workgroups to fill the 256 CUs (unless no shorter pass helps)
      const int64_t nblk = ((int64_t)1 << (k0 - 1)) << (log2J - log2T);
      if (((size_t)rm << (m + log2T)) <= budget && (nblk >= 1024 || m == 1)) break;
    }
    QTP_REQUIRE(m >= 1, -1, "QTT rank too large for the fused apply");
    FusePlan P{};
    P.m = m;
    int rm = 1;
    for (int l = 0; l <= m; ++l) {
      P.ra[l] = ranks[k0 - 1 + l];
      rm = std::max(rm, P.ra[l]);
    }
    for (int l = 0; l < m; ++l) P.coff[l] = off[k0 - 1 + l];
    const size_t lds = 2 * sizeof(AT) * ((size_t)rm << (m + log2T));
    const bool last = k0 + m - 1 == d;
    if (first && last)
      launch_fused<CT, double, double, AT>(s, cores, P, d, k0, log2T, x, y, lds);
    else if (first)
      launch_fused<CT, double, IT, AT>(s, cores, P, d, k0, log2T, x, buf[cur], lds);
    else if (last)
      launch_fused<CT, IT, double, AT>(s, cores, P, d, k0, log2T, buf[cur ^ 1], y, lds);
    else
      launch_fused<CT, IT, IT, AT>(s, cores, P, d, k0, log2T, buf[cur ^ 1], buf[cur], lds);
    first = false;
    cur ^= 1;
    k0 += m;
  }
}

template <class CT, class IT>
void apply_levels(hipStream_t s, int d, const int32_t* ranks, const CT* cores,
                  const double* x, double* y, void* work);

template <class CT, class IT>
void apply_impl(hipStream_t s, int d, const int32_t* ranks, const CT* cores,
                const double* x, double* y, void* work) {
  int64_t rmax = 1;
  for (int k = 0; k <= d; ++k) rmax = ranks[k] > rmax ? ranks[k] : rmax;
  if (rmax <= 64) {
    apply_fused<CT, IT>(s, d, ranks, cores, x, y, work);
    return;
  }
  apply_levels<CT, IT>(s, d, ranks, cores, x, y, work);
}

template <class CT, class IT>
void apply_levels(hipStream_t s, int d, const int32_t* ranks, const CT* cores,
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
