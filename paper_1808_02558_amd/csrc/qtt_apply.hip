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

#include <algorithm>

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

// ---------------------------------------------------------------------------
// Register-resident fusion for small ranks.  One thread owns one column pair
// (I, J'') of a pass over M levels and keeps its whole fibre
// Z[I][alpha][jj (M bits)][J''] (alpha < R) in registers: each level replaces
// the leading remaining column bit j by the row bit i at the same position,
// so no data moves between threads and no barrier is needed.  The core
// entries are the same for every thread and are read through the scalar
// cache; the fibres are read and written with loads and stores that are
// coalesced over consecutive J''.
// ---------------------------------------------------------------------------
template <int R, int M, class CT, class IT, class OT, class AT>
__global__ __launch_bounds__(kThreads) void qtt_reg_kernel(
    const CT* __restrict__ cores, FusePlan P, int log2J, int64_t nthreads,
    const IT* __restrict__ in, OT* __restrict__ out) {
  // With fewer than 16 trailing indices the fibres of one workgroup form one
  // contiguous run of the input (and of the output): it is staged through
  // LDS with coalesced loads and stores instead of strided per-thread ones.
  extern __shared__ unsigned char qtt_reg_smem[];
  AT* stage = reinterpret_cast<AT*>(qtt_reg_smem);
  const bool staged = log2J < 4;
  const int64_t tid0 = (int64_t)blockIdx.x * kThreads;
  const int64_t tid = tid0 + threadIdx.x;
  const int cnt = (int)min<int64_t>(kThreads, nthreads - tid0);
  const bool live = threadIdx.x < cnt;
  const int64_t Jtot = (int64_t)1 << log2J;
  const int64_t I = tid >> log2J;
  const int64_t J = tid & (Jtot - 1);
  const int64_t Il = (int64_t)threadIdx.x >> log2J;  // prefix within the block
  constexpr int F = 1 << M;
  AT v[R][F];
  const int r0 = P.ra[0];
  if (staged) {
    const int64_t n_in = (int64_t)cnt * r0 * F;
    const IT* src = in + tid0 * r0 * F;
    for (int64_t e = threadIdx.x; e < n_in; e += kThreads) stage[e] = (AT)src[e];
    __syncthreads();
    if (live) {
#pragma unroll
      for (int a = 0; a < R; ++a) {
        if (a < r0) {
#pragma unroll
          for (int p = 0; p < F; ++p)
            v[a][p] = stage[(((Il * r0 + a) << M) + p) * Jtot + J];
        }
      }
    }
    __syncthreads();
  } else if (live) {
#pragma unroll
    for (int a = 0; a < R; ++a) {
      if (a < r0) {
#pragma unroll
        for (int p = 0; p < F; ++p)
          v[a][p] = (AT)in[(((I * r0 + a) << M) + p) * Jtot + J];
      }
    }
  }
#pragma unroll
  for (int l = 0; l < M; ++l) {
    const int ra = P.ra[l], rb = P.ra[l + 1];
    const CT* G = cores + P.coff[l];
    const int sh = M - 1 - l;  // position of this level's bit in the fibre
#pragma unroll
    for (int g = 0; g < F / 2; ++g) {
      const int p0 = ((g >> sh) << (sh + 1)) | (g & ((1 << sh) - 1));
      const int p1 = p0 | (1 << sh);
      AT t0[R], t1[R];
#pragma unroll
      for (int b = 0; b < R; ++b) {
        t0[b] = AT(0);
        t1[b] = AT(0);
      }
#pragma unroll
      for (int a = 0; a < R; ++a) {
        if (a < ra) {
          const AT x0 = v[a][p0], x1 = v[a][p1];
          const int64_t c00 = (int64_t)(a * 4) * rb;  // (a, i = 0, j = 0)
#pragma unroll
          for (int b = 0; b < R; ++b) {
            if (b < rb) {
              t0[b] += CoreLoad<CT>::get(G, c00 + b) * x0 +
                       CoreLoad<CT>::get(G, c00 + rb + b) * x1;
              t1[b] += CoreLoad<CT>::get(G, c00 + 2 * rb + b) * x0 +
                       CoreLoad<CT>::get(G, c00 + 3 * rb + b) * x1;
            }
          }
        }
      }
#pragma unroll
      for (int b = 0; b < R; ++b) {
        if (b < rb) {
          v[b][p0] = t0[b];
          v[b][p1] = t1[b];
        }
      }
    }
  }
  const int rm = P.ra[M];
  if (staged) {
    if (live) {
#pragma unroll
      for (int b = 0; b < R; ++b) {
        if (b < rm) {
#pragma unroll
          for (int p = 0; p < F; ++p)
            stage[(((Il << M) + p) * rm + b) * Jtot + J] = v[b][p];
        }
      }
    }
    __syncthreads();
    const int64_t n_out = (int64_t)cnt * rm * F;
    OT* dst = out + tid0 * rm * F;
    for (int64_t e = threadIdx.x; e < n_out; e += kThreads) dst[e] = (OT)stage[e];
  } else if (live) {
#pragma unroll
    for (int b = 0; b < R; ++b) {
      if (b < rm) {
#pragma unroll
        for (int p = 0; p < F; ++p)
          out[(((I << M) + p) * rm + b) * Jtot + J] = (OT)v[b][p];
      }
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

template <int R, int M, class CT, class IT, class OT, class AT>
void launch_reg(hipStream_t s, const CT* cores, const FusePlan& P, int d, int k0,
                const IT* in, OT* out) {
  const int log2J = d - (k0 + M - 1);
  const int64_t nthreads = (int64_t)1 << (d - M);  // 2^{k0-1} prefixes x 2^{log2J}
  const size_t lds = log2J < 4 ? sizeof(AT) * kThreads * R * (1 << M) : 0;
  qtt_reg_kernel<R, M, CT, IT, OT, AT><<<div_up(nthreads, kThreads), kThreads, lds, s>>>(
      cores, P, log2J, nthreads, in, out);
  QTP_CHECK_LAUNCH();
}

// Register pass over M levels whose ranks are all <= R (R * 2^M values per
// thread; FP64 keeps R <= 16).
template <class CT, class IT, class OT, class AT>
bool try_reg_pass(hipStream_t s, const CT* cores, const FusePlan& P, int d, int k0,
                  int R, const IT* in, OT* out) {
  const int M = P.m;
  const bool wide = sizeof(AT) == 8;
#define QTP_REG(RR, MM)                                                       \
  if (R <= RR && M == MM) {                                                   \
    launch_reg<RR, MM, CT, IT, OT, AT>(s, cores, P, d, k0, in, out);          \
    return true;                                                              \
  }
  if (wide) {
    QTP_REG(4, 3)
    QTP_REG(4, 2)
    QTP_REG(8, 2)
    QTP_REG(4, 1)
    QTP_REG(8, 1)
    QTP_REG(16, 1)
  } else {
    QTP_REG(4, 4)
    QTP_REG(4, 3)
    QTP_REG(8, 3)
    QTP_REG(4, 2)
    QTP_REG(8, 2)
    QTP_REG(16, 2)
    QTP_REG(4, 1)
    QTP_REG(8, 1)
    QTP_REG(16, 1)
    if (sizeof(CT) != 2) {
      QTP_REG(32, 1)
    }
  }
#undef QTP_REG
  return false;
}

// Levels a register pass can take from level k0 (1-based) on: the largest M
// whose window of ranks fits the register budget while the pass still has
// at least 2^17 threads (512 workgroups), or 0 when no register pass fits;
// the LDS-fused pass then takes over.
int reg_levels(int d, const int32_t* ranks, int k0, bool wide, bool bf16, int* R_out) {
  const int cap_threads = d > 17 ? d - 17 : 0;  // M <= d - 17 keeps 2^17 threads
  for (int M = std::min(4, d - k0 + 1); M >= 1; --M) {
    if (M > 1 && M > cap_threads) continue;
    int rm = 1;
    for (int l = 0; l <= M; ++l) rm = std::max<int>(rm, ranks[k0 - 1 + l]);
    int R = 4;
    while (R < rm) R <<= 1;
    // register budget: R * 2^M values plus 2R accumulators (FP64 one step
    // narrower so that no variant needs more than ~160 VGPRs)
    const int maxR = wide ? (M == 4 ? 0 : M == 3 ? 4 : M == 2 ? 8 : 16)
                          : (M == 4 ? 4 : M == 3 ? 8 : M == 2 ? 16 : (bf16 ? 16 : 32));
    if (R <= maxR) {
      *R_out = R;
      return M;
    }
  }
  return 0;
}

// Greedy pass plan: register passes while the ranks are small, otherwise the
// longest run of levels whose slab fits the LDS budget.
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
    int R = 0;
    const int mr = reg_levels(d, ranks, k0, sizeof(AT) == 8, sizeof(CT) == 2, &R);
    if (mr > 0) {
      FusePlan P{};
      P.m = mr;
      for (int l = 0; l <= mr; ++l) P.ra[l] = ranks[k0 - 1 + l];
      for (int l = 0; l < mr; ++l) P.coff[l] = off[k0 - 1 + l];
      const bool last = k0 + mr - 1 == d;
      bool ok;
      if (first && last)
        ok = try_reg_pass<CT, double, double, AT>(s, cores, P, d, k0, R, x, y);
      else if (first)
        ok = try_reg_pass<CT, double, IT, AT>(s, cores, P, d, k0, R, x, buf[cur]);
      else if (last)
        ok = try_reg_pass<CT, IT, double, AT>(s, cores, P, d, k0, R, buf[cur ^ 1], y);
      else
        ok = try_reg_pass<CT, IT, IT, AT>(s, cores, P, d, k0, R, buf[cur ^ 1], buf[cur]);
      QTP_REQUIRE(ok, -1, "QTT apply: no register kernel for this pass");
      first = false;
      cur ^= 1;
      k0 += mr;
      continue;
    }
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
