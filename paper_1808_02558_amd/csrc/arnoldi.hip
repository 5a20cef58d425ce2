// Arnoldi steps of right-preconditioned flexible GMRES (Saad 1993) with
// classical Gram-Schmidt applied twice, arranged so that one step is six
// launches with the block-Jacobi preconditioner (eight with the QTT inverse)
// and the host never waits inside a restart cycle except to read a residual
// estimate that lags one step behind the queued work.
//
// Step j (basis V_0..V_j orthonormal, w = V_{j+1} the raw product):
//   next : V_j = (w_j - sum_l h2_l V_l) / h_{j,j-1}, the second Gram-Schmidt
//          correction of step j-1 deferred to here, fused with the block-Jacobi
//          part of the preconditioner (z = L^-T L^-1 V_j, or t = L^-1 V_j when
//          the QTT inverse sits between the two factors);
//   (spmv w = S z_j by the caller)
//   dots : per-block partials of h1 = V^T w, summed by a one-workgroup pass;
//   orth : w -= V h1, partials of h2 = V^T w and of |w|^2 in one pass; the
//          one-workgroup pass after it sums them, forms the Hessenberg column
//          h_j = h1 + h2 with h_{j+1,j}^2 = |w|^2 - |h2|^2 (the norm of
//          w - V h2 by Pythagoras, V being orthonormal), applies the Givens
//          rotations and stores the residual estimate |g_{j+1}| into a
//          host-visible status ring.
// Every reduction is deterministic: per-block partials in a fixed layout and
// a fixed-order sum in the second pass; no floating-point atomics.  (A
// last-block-done scheme would save the second launch, but the device-scope
// fences it needs flush and invalidate the L2 of every XCD and cost far more
// than a launch.)
#include <algorithm>

#include "ops.h"

namespace qtp {
namespace {

constexpr int kThreads = 256;
constexpr int kNextThreads = 192;  // 64 slots of 3 unknowns per workgroup
constexpr int kFinThreads = 1024;  // threads of the one-workgroup sum

// out[l] = sum_b partial[l * nblk + b] for l < nout, in a fixed order; one
// wavefront per output, reading its row of partials coalesced.
__device__ void sum_partials(int nblk, int nout, const double* __restrict__ partial,
                             double* out) {
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  for (int l = wave; l < nout; l += kFinThreads / 64) {
    double acc = 0.0;
    const double* row = partial + (int64_t)l * nblk;
    for (int b = lane; b < nblk; b += 64) acc += row[b];
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) acc += __shfl_xor(acc, o, 64);
    if (lane == 0) out[l] = acc;
  }
}

__global__ __launch_bounds__(kNextThreads) void next_kernel(
    int nprev, const double* __restrict__ V, int64_t n, int nslots,
    double* __restrict__ d, double inv0, double beta, const double* src, double* vj,
    const double* __restrict__ Linv, int full, double* __restrict__ zout) {
  __shared__ double hs[kArnMaxRestart];
  __shared__ double vs[kNextThreads];
  if (threadIdx.x < nprev) hs[threadIdx.x] = d[kArnH2 + threadIdx.x];
  if (nprev == 0 && blockIdx.x == 0 && threadIdx.x < kArnMaxRestart + 1)
    d[kArnG + threadIdx.x] = threadIdx.x == 0 ? beta : 0.0;
  __syncthreads();
  const double inv = nprev > 0 ? d[kArnInv] : inv0;
  const int64_t i = (int64_t)blockIdx.x * kNextThreads + threadIdx.x;
  double v = 0.0;
  if (i < n) {
    double w = src[i];
    for (int l = 0; l < nprev; ++l) w -= hs[l] * V[(int64_t)l * n + i];
    v = w * inv;
    vj[i] = v;
  }
  vs[threadIdx.x] = v;
  __syncthreads();
  if (i >= n) return;
  const int64_t s = i / 3;
  if (s >= nslots) {
    zout[i] = v;  // identity rows past the last slot
    return;
  }
  const int ls = threadIdx.x / 3;
  const int r = threadIdx.x - 3 * ls;
  const double* m = Linv + s * 6;
  const double x0 = vs[3 * ls], x1 = vs[3 * ls + 1], x2 = vs[3 * ls + 2];
  const double t0 = m[0] * x0;
  const double t1 = m[1] * x0 + m[2] * x1;
  const double t2 = m[3] * x0 + m[4] * x1 + m[5] * x2;
  double z;
  if (full) {
    z = r == 0 ? m[0] * t0 + m[1] * t1 + m[3] * t2
               : (r == 1 ? m[2] * t1 + m[4] * t2 : m[5] * t2);
  } else {
    z = r == 0 ? t0 : (r == 1 ? t1 : t2);
  }
  zout[i] = z;
}

// h1 = V^T w over nvec <= NV vectors.
template <int NV>
__global__ __launch_bounds__(kThreads) void dots_kernel(
    int nvec, const double* __restrict__ V, const double* __restrict__ w, int64_t n,
    double* __restrict__ partial) {
  __shared__ double red[NV][kThreads / 64];
  double acc[NV];
#pragma unroll
  for (int l = 0; l < NV; ++l) acc[l] = 0.0;
  const int64_t stride = (int64_t)gridDim.x * kThreads;
  for (int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x; i < n; i += stride) {
    double v[NV];
#pragma unroll
    for (int l = 0; l < NV; ++l) v[l] = l < nvec ? V[(int64_t)l * n + i] : 0.0;
    const double wi = w[i];
#pragma unroll
    for (int l = 0; l < NV; ++l) acc[l] += v[l] * wi;
  }
  const int wave = threadIdx.x >> 6;
#pragma unroll
  for (int l = 0; l < NV; ++l) {
    double s = acc[l];
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o, 64);
    if ((threadIdx.x & 63) == 0) red[l][wave] = s;
  }
  __syncthreads();
  if (threadIdx.x < nvec) {
    double s = 0.0;
    for (int q = 0; q < kThreads / 64; ++q) s += red[threadIdx.x][q];
    partial[(int64_t)threadIdx.x * gridDim.x + blockIdx.x] = s;
  }
}

__global__ __launch_bounds__(kFinThreads) void dots_finish_kernel(
    int nblk, int nvec, const double* __restrict__ partial, double* __restrict__ d) {
  sum_partials(nblk, nvec, partial, d + kArnH1);
}

// w -= V h1; partials of h2 = V^T w and of |w|^2 (the latter last).
template <int NV>
__global__ __launch_bounds__(kThreads) void orth_kernel(
    int nvec, const double* __restrict__ V, double* __restrict__ w, int64_t n,
    double* __restrict__ partial, const double* __restrict__ d) {
  __shared__ double hs[NV];
  __shared__ double red[NV + 1][kThreads / 64];
  if (threadIdx.x < NV) hs[threadIdx.x] = threadIdx.x < nvec ? d[kArnH1 + threadIdx.x] : 0.0;
  __syncthreads();
  double acc[NV + 1];
#pragma unroll
  for (int l = 0; l <= NV; ++l) acc[l] = 0.0;
  const int64_t stride = (int64_t)gridDim.x * kThreads;
  for (int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x; i < n; i += stride) {
    double v[NV];
#pragma unroll
    for (int l = 0; l < NV; ++l) v[l] = l < nvec ? V[(int64_t)l * n + i] : 0.0;
    double wi = w[i];
#pragma unroll
    for (int l = 0; l < NV; ++l) wi -= hs[l] * v[l];
    w[i] = wi;
#pragma unroll
    for (int l = 0; l < NV; ++l) acc[l] += v[l] * wi;
    acc[NV] += wi * wi;
  }
  const int wave = threadIdx.x >> 6;
#pragma unroll
  for (int l = 0; l <= NV; ++l) {
    double s = acc[l];
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o, 64);
    if ((threadIdx.x & 63) == 0) red[l][wave] = s;
  }
  __syncthreads();
  if (threadIdx.x <= nvec) {
    const int l = threadIdx.x < nvec ? threadIdx.x : NV;  // the norm goes last
    double s = 0.0;
    for (int q = 0; q < kThreads / 64; ++q) s += red[l][q];
    partial[(int64_t)threadIdx.x * gridDim.x + blockIdx.x] = s;
  }
}

// Sums the orth partials, then the Hessenberg column j = nvec - 1, its Givens
// rotation and the residual estimate (one thread).
__global__ __launch_bounds__(kFinThreads) void orth_finish_kernel(
    int nblk, int nvec, const double* __restrict__ partial, double* __restrict__ d,
    double* __restrict__ status, int64_t tag) {
  __shared__ double fin[kArnMaxRestart + 1];
  __shared__ double H[kArnMaxRestart + 1], cs[kArnMaxRestart], sn[kArnMaxRestart];
  const int j = nvec - 1;
  sum_partials(nblk, nvec + 1, partial, fin);
  if (threadIdx.x < j) {
    cs[threadIdx.x] = d[kArnCs + threadIdx.x];
    sn[threadIdx.x] = d[kArnSn + threadIdx.x];
  }
  __syncthreads();
  if (threadIdx.x <= j) {
    d[kArnH2 + threadIdx.x] = fin[threadIdx.x];
    H[threadIdx.x] = d[kArnH1 + threadIdx.x] + fin[threadIdx.x];
  }
  __syncthreads();
  if (threadIdx.x != 0) return;
  double* Hd = d + kArnH + (int64_t)j * kArnLd;
  double* g = d + kArnG;
  double h2sq = 0.0;
  for (int i = 0; i <= j; ++i) h2sq += fin[i] * fin[i];
  const double hn2 = fin[nvec] - h2sq;
  const double hn = hn2 > 0.0 ? sqrt(hn2) : (hn2 == hn2 ? 0.0 : hn2);
  H[j + 1] = hn;
  d[kArnInv] = hn > 0.0 ? 1.0 / hn : 0.0;
  for (int i = 0; i < j; ++i) {
    const double t = cs[i] * H[i] + sn[i] * H[i + 1];
    H[i + 1] = -sn[i] * H[i] + cs[i] * H[i + 1];
    H[i] = t;
  }
  const double den = hypot(H[j], H[j + 1]);
  const double c = den > 0.0 ? H[j] / den : 1.0;
  const double s = den > 0.0 ? H[j + 1] / den : 0.0;
  d[kArnCs + j] = c;
  d[kArnSn + j] = s;
  H[j] = den;
  H[j + 1] = 0.0;
  for (int i = 0; i <= j + 1; ++i) Hd[i] = H[i];
  const double gj = g[j];
  g[j + 1] = -s * gj;
  g[j] = c * gj;
  // one word, so no ordering against other stores is needed: a breakdown
  // (hn = 0) ends the cycle like convergence does
  const double res = hn == 0.0 ? 0.0 : fabs(s * gj);
  __hip_atomic_store(status + (tag & (kArnRing - 1)), res, __ATOMIC_RELAXED,
                     __HIP_MEMORY_SCOPE_SYSTEM);
}

// y = H(0:jend, 0:jend)^-1 g(0:jend) by back substitution (H staged in LDS).
__global__ __launch_bounds__(kFinThreads) void solve_kernel(int jend, double* __restrict__ d) {
  __shared__ double H[kArnMaxRestart][kArnMaxRestart];
  __shared__ double y[kArnMaxRestart];
  for (int e = threadIdx.x; e < jend * jend; e += kFinThreads) {
    const int k = e / jend, i = e - k * jend;  // column k, row i
    H[k][i] = d[kArnH + (int64_t)k * kArnLd + i];
  }
  if (threadIdx.x < jend) y[threadIdx.x] = d[kArnG + threadIdx.x];
  __syncthreads();
  if (threadIdx.x != 0) return;
  for (int i = jend - 1; i >= 0; --i) {
    double t = y[i];
    for (int k = i + 1; k < jend; ++k) t -= H[k][i] * y[k];
    y[i] = t / H[i][i];
  }
  for (int i = 0; i < jend; ++i) d[kArnY + i] = y[i];
}

// Workgroups of the Arnoldi reductions: at most 512 (two per CU), which
// measured faster than 1024 (more partial sums to add) and than 256.
int reduce_grid(int64_t n) {
  int64_t b = (n + kThreads - 1) / kThreads;
  return (int)std::max<int64_t>(1, std::min<int64_t>(b, 512));
}

}  // namespace

size_t arnoldi_partial_doubles(int64_t n) {
  return (size_t)reduce_grid(n) * (kArnMaxRestart + 1);  // [output][block]
}

void arnoldi_next(hipStream_t s, const Arnoldi& a, int nprev, const double* V,
                  int64_t n, int nslots, double inv0, double beta, const double* src,
                  double* vj, const double* Linv, int full, double* zout) {
  QTP_REQUIRE(nprev >= 0 && nprev <= kArnMaxRestart, -1, "arnoldi_next: nprev");
  QTP_REQUIRE(3 * (int64_t)nslots <= n, -1, "arnoldi_next: slots exceed n");
  if (n == 0) return;
  next_kernel<<<div_up(n, kNextThreads), kNextThreads, 0, s>>>(
      nprev, V, n, nslots, a.d, inv0, beta, src, vj, Linv, full, zout);
  QTP_CHECK_LAUNCH();
}

void arnoldi_dots(hipStream_t s, const Arnoldi& a, int nvec, const double* V,
                  int64_t n, const double* w) {
  QTP_REQUIRE(nvec >= 1 && nvec <= kArnMaxRestart, -1, "arnoldi_dots: nvec");
  const int nb = reduce_grid(n);
  if (nvec <= 8)
    dots_kernel<8><<<nb, kThreads, 0, s>>>(nvec, V, w, n, a.partial);
  else if (nvec <= 16)
    dots_kernel<16><<<nb, kThreads, 0, s>>>(nvec, V, w, n, a.partial);
  else
    dots_kernel<32><<<nb, kThreads, 0, s>>>(nvec, V, w, n, a.partial);
  QTP_CHECK_LAUNCH();
  dots_finish_kernel<<<1, kFinThreads, 0, s>>>(nb, nvec, a.partial, a.d);
  QTP_CHECK_LAUNCH();
}

void arnoldi_orth(hipStream_t s, const Arnoldi& a, int nvec, const double* V,
                  int64_t n, double* w, int64_t tag) {
  QTP_REQUIRE(nvec >= 1 && nvec <= kArnMaxRestart, -1, "arnoldi_orth: nvec");
  const int nb = reduce_grid(n);
  if (nvec <= 8)
    orth_kernel<8><<<nb, kThreads, 0, s>>>(nvec, V, w, n, a.partial, a.d);
  else if (nvec <= 16)
    orth_kernel<16><<<nb, kThreads, 0, s>>>(nvec, V, w, n, a.partial, a.d);
  else
    orth_kernel<32><<<nb, kThreads, 0, s>>>(nvec, V, w, n, a.partial, a.d);
  QTP_CHECK_LAUNCH();
  orth_finish_kernel<<<1, kFinThreads, 0, s>>>(nb, nvec, a.partial, a.d, a.status, tag);
  QTP_CHECK_LAUNCH();
}

void arnoldi_solve(hipStream_t s, const Arnoldi& a, int jend) {
  QTP_REQUIRE(jend >= 1 && jend <= kArnMaxRestart, -1, "arnoldi_solve: jend");
  solve_kernel<<<1, kFinThreads, 0, s>>>(jend, a.d);
  QTP_CHECK_LAUNCH();
}

}  // namespace qtp
