// Vector kernels of the Krylov solve and the block-Jacobi scaling.
//
// Reductions are deterministic: every block writes one partial sum per
// output in a fixed order, and a second single-block pass adds the partials
// in index order.  No floating-point atomics.
#include <algorithm>

#include "ops.h"

namespace qtp {
namespace {

constexpr int kThreads = 256;
constexpr int kMaxBlocks = 1024;
constexpr int kMaxVec = 64;  // most vectors a multi-dot handles per pass

__device__ inline double block_sum(double v, double* sh) {
  // wavefront reduction, then across the 4 wavefronts of the block
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  const int w = threadIdx.x >> 6;
  __syncthreads();
  if ((threadIdx.x & 63) == 0) sh[w] = v;
  __syncthreads();
  double s = 0.0;
  if (threadIdx.x == 0) {
    for (int i = 0; i < kThreads / 64; ++i) s += sh[i];
  }
  return s;  // valid in thread 0
}

// One pass over up to NV basis vectors V_l (register blocked: each V_l[i] is
// loaded once and kept in a register for both of its uses).
//   MODE 0: partial dots V_l . w
//   MODE 1: w -= sum_l h_l V_l, then partial dots V_l . w (new w)
//   MODE 2: w -= sum_l h_l V_l, then the partial of |w|^2
//   MODE 3: w -= sum_l h_l V_l only
// Partials go to partial[blk * pstride + poff + l].
template <int NV, int MODE>
__global__ __launch_bounds__(kThreads) void cgs_kernel(
    int nvec, const double* __restrict__ V, int64_t ldv,
    const double* __restrict__ h, double* __restrict__ w, int64_t n,
    double* __restrict__ partial, int pstride, int poff) {
  constexpr int NACC = MODE == 0 || MODE == 1 ? NV : 1;
  __shared__ double hs[NV];
  __shared__ double red[NACC][kThreads / 64];
  if (MODE != 0) {
    if (threadIdx.x < NV) hs[threadIdx.x] = threadIdx.x < nvec ? h[threadIdx.x] : 0.0;
    __syncthreads();
  }
  double acc[NACC];
#pragma unroll
  for (int l = 0; l < NACC; ++l) acc[l] = 0.0;
  const int64_t stride = (int64_t)gridDim.x * kThreads;
  for (int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x; i < n; i += stride) {
    double v[NV];
#pragma unroll
    for (int l = 0; l < NV; ++l) v[l] = l < nvec ? V[(int64_t)l * ldv + i] : 0.0;
    double wi = w[i];
    if (MODE != 0) {
#pragma unroll
      for (int l = 0; l < NV; ++l) wi -= hs[l] * v[l];
      w[i] = wi;
    }
    if (MODE == 0 || MODE == 1) {
#pragma unroll
      for (int l = 0; l < NV; ++l) acc[l] += v[l] * wi;
    } else if (MODE == 2) {
      acc[0] += wi * wi;
    }
  }
  if (MODE == 3) return;
  const int nout = MODE == 2 ? 1 : nvec;
  const int wave = threadIdx.x >> 6;
#pragma unroll
  for (int l = 0; l < NACC; ++l) {
    double s = acc[l];
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o, 64);
    if ((threadIdx.x & 63) == 0) red[l][wave] = s;
  }
  __syncthreads();
  if (threadIdx.x < nout) {
    double s = 0.0;
    for (int q = 0; q < kThreads / 64; ++q) s += red[threadIdx.x][q];
    partial[(int64_t)blockIdx.x * pstride + poff + threadIdx.x] = s;
  }
}

template <int MODE>
void launch_cgs(hipStream_t s, int nb, int nvec, const double* V, int64_t ldv,
                const double* h, double* w, int64_t n, double* partial, int pstride,
                int poff) {
  if (nvec <= 8)
    cgs_kernel<8, MODE><<<nb, kThreads, 0, s>>>(nvec, V, ldv, h, w, n, partial,
                                                pstride, poff);
  else if (nvec <= 16)
    cgs_kernel<16, MODE><<<nb, kThreads, 0, s>>>(nvec, V, ldv, h, w, n, partial,
                                                 pstride, poff);
  else
    cgs_kernel<32, MODE><<<nb, kThreads, 0, s>>>(nvec, V, ldv, h, w, n, partial,
                                                 pstride, poff);
  QTP_CHECK_LAUNCH();
}

// out[l] = sum_b partial[b * nvec + l] in a fixed order; one wavefront per
// output l (grid = nvec, 64 threads).
__global__ void finish_kernel(int nblk, int nvec, const double* __restrict__ partial,
                              double* __restrict__ out) {
  const int l = blockIdx.x;
  double acc = 0.0;
  for (int b = threadIdx.x; b < nblk; b += 64) acc += partial[(int64_t)b * nvec + l];
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) acc += __shfl_xor(acc, o, 64);
  if (threadIdx.x == 0) out[l] = acc;
}

void finish(hipStream_t s, int nblk, int nvec, const double* partial, double* out) {
  finish_kernel<<<nvec, 64, 0, s>>>(nblk, nvec, partial, out);
  QTP_CHECK_LAUNCH();
}

__global__ void scale_kernel(const double* __restrict__ a, int inv,
                             const double* __restrict__ x, double* __restrict__ y,
                             int64_t n) {
  const double s = inv ? 1.0 / a[0] : a[0];
  for (int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * kThreads)
    y[i] = s * x[i];
}

__global__ void multi_axpy_kernel(int nvec, const double* __restrict__ X,
                                  int64_t ldx, const double* __restrict__ c,
                                  double* __restrict__ y, int64_t n) {
  __shared__ double cs[kMaxVec];
  if (threadIdx.x < nvec) cs[threadIdx.x] = c[threadIdx.x];
  __syncthreads();
  for (int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * kThreads) {
    double v = y[i];
    for (int l = 0; l < nvec; ++l) v += cs[l] * X[(int64_t)l * ldx + i];
    y[i] = v;
  }
}

__global__ void sub_kernel(const double* __restrict__ x, const double* __restrict__ y,
                           double* __restrict__ z, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * kThreads)
    z[i] = x[i] - y[i];
}

__global__ void add_kernel(const double* __restrict__ x, double* __restrict__ y,
                           int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * kThreads)
    y[i] += x[i];
}

__global__ void nonfinite_kernel(const double* __restrict__ x, int64_t n,
                                 int* __restrict__ out) {
  for (int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * kThreads)
    if (!isfinite(x[i])) out[0] = 1;  // benign race: every writer stores 1
}

// ---- block Jacobi -----------------------------------------------------------

// L^-1 (lower triangle, row-major) of chol(A + shift I) for the symmetric
// 3x3 A given by its lower triangle; false when a pivot is not positive.
__device__ bool chol_inv3(double a00, double a10, double a11, double a20, double a21,
                          double a22, double shift, double out[6]) {
  a00 += shift;
  a11 += shift;
  a22 += shift;
  if (!(a00 > 0.0)) return false;
  const double l00 = sqrt(a00);
  const double l10 = a10 / l00;
  const double l20 = a20 / l00;
  const double d1 = a11 - l10 * l10;
  if (!(d1 > 0.0)) return false;
  const double l11 = sqrt(d1);
  const double l21 = (a21 - l20 * l10) / l11;
  const double d2 = a22 - l20 * l20 - l21 * l21;
  if (!(d2 > 0.0)) return false;
  const double l22 = sqrt(d2);
  const double m00 = 1.0 / l00;
  const double m11 = 1.0 / l11;
  const double m22 = 1.0 / l22;
  const double m10 = -l10 * m00 / l11;
  const double m21 = -l21 * m11 / l22;
  const double m20 = -(l20 * m00 + l21 * m10) / l22;
  out[0] = m00; out[1] = m10; out[2] = m11;
  out[3] = m20; out[4] = m21; out[5] = m22;
  return isfinite(m00) && isfinite(m10) && isfinite(m11) && isfinite(m20) &&
         isfinite(m21) && isfinite(m22);
}

// Block-Jacobi factors.  A diagonal block of S is positive definite, but late
// in the PDIP a barrier term lambda/(-f) g g^T can exceed the rest by 1e16
// and rounding then breaks the Cholesky; the preconditioner only needs an
// SPD approximation, so the block is shifted by 1e-14, 1e-12, ... times its
// largest diagonal entry until the factorisation succeeds.
__global__ void bj_factor_kernel(int nslots, const int32_t* __restrict__ rp,
                                 const int32_t* __restrict__ col,
                                 const double* __restrict__ val,
                                 double* __restrict__ Linv, int* __restrict__ bad) {
  const int s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= nslots) return;
  int b = -1;
  for (int q = rp[s]; q < rp[s + 1]; ++q)
    if (col[q] == s) { b = q; break; }
  double out[6] = {1, 0, 1, 0, 0, 1};
  if (b < 0) {
    bad[0] = 1;
  } else {
    const double* A = val + (int64_t)b * 9;
    const double a00 = A[0], a10 = A[3], a11 = A[4], a20 = A[6], a21 = A[7],
                 a22 = A[8];
    const double dmax = fmax(fabs(a00), fmax(fabs(a11), fabs(a22)));
    bool ok = chol_inv3(a00, a10, a11, a20, a21, a22, 0.0, out);
    for (double rel = 1e-14; !ok && rel <= 1e-6; rel *= 100.0)
      ok = chol_inv3(a00, a10, a11, a20, a21, a22, rel * dmax, out);
    if (!ok) {
      bad[0] = 1;
      for (int q = 0; q < 6; ++q) out[q] = (q == 0 || q == 2 || q == 5) ? 1.0 : 0.0;
    }
  }
  for (int q = 0; q < 6; ++q) Linv[(int64_t)s * 6 + q] = out[q];
}

__global__ void bj_apply_kernel(int nslots, int64_t n, const double* __restrict__ Linv,
                                int trans, const double* __restrict__ x,
                                double* __restrict__ y) {
  const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (s < nslots) {
    const double* m = Linv + s * 6;
    const double x0 = x[3 * s], x1 = x[3 * s + 1], x2 = x[3 * s + 2];
    double y0, y1, y2;
    if (!trans) {
      y0 = m[0] * x0;
      y1 = m[1] * x0 + m[2] * x1;
      y2 = m[3] * x0 + m[4] * x1 + m[5] * x2;
    } else {
      y0 = m[0] * x0 + m[1] * x1 + m[3] * x2;
      y1 = m[2] * x1 + m[4] * x2;
      y2 = m[5] * x2;
    }
    y[3 * s] = y0;
    y[3 * s + 1] = y1;
    y[3 * s + 2] = y2;
  } else {
    const int64_t u = 3 * (int64_t)nslots + (s - nslots);
    if (u < n) y[u] = x[u];
  }
}

// vout_b = L_s^-1 A_b L_c^-T for every block b = (s, c)
__global__ void bj_scale_matrix_kernel(int nslots, const int32_t* __restrict__ rp,
                                       const int32_t* __restrict__ col,
                                       const double* __restrict__ val,
                                       const double* __restrict__ Linv,
                                       double* __restrict__ vout) {
  const int s = blockIdx.x;
  double Ls[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
  const double* m = Linv + (int64_t)s * 6;
  Ls[0] = m[0]; Ls[3] = m[1]; Ls[4] = m[2]; Ls[6] = m[3]; Ls[7] = m[4]; Ls[8] = m[5];
  for (int q = rp[s] + threadIdx.x; q < rp[s + 1]; q += blockDim.x) {
    const int c = col[q];
    const double* mc = Linv + (int64_t)c * 6;
    double Lc[9] = {mc[0], 0, 0, mc[1], mc[2], 0, mc[3], mc[4], mc[5]};
    const double* A = val + (int64_t)q * 9;
    double T[9];
    for (int r = 0; r < 3; ++r)
      for (int cc = 0; cc < 3; ++cc) {
        double acc = 0.0;
        for (int t = 0; t < 3; ++t) acc += Ls[3 * r + t] * A[3 * t + cc];
        T[3 * r + cc] = acc;
      }
    double* O = vout + (int64_t)q * 9;
    for (int r = 0; r < 3; ++r)
      for (int cc = 0; cc < 3; ++cc) {
        double acc = 0.0;
        for (int t = 0; t < 3; ++t) acc += T[3 * r + t] * Lc[3 * cc + t];
        O[3 * r + cc] = acc;
      }
  }
}

int grid_for(int64_t n) {
  int64_t b = (n + kThreads - 1) / kThreads;
  if (b > kMaxBlocks) b = kMaxBlocks;
  if (b < 1) b = 1;
  return (int)b;
}

}  // namespace

int reduce_blocks(int64_t n) { return grid_for(n); }

void multi_dot(hipStream_t s, int nvec, const double* V, int64_t ldv,
               const double* w, int64_t n, double* partial, double* out) {
  QTP_REQUIRE(nvec >= 1 && nvec <= kMaxVec, -1, "multi_dot: nvec out of range");
  const int nb = grid_for(n);
  for (int c0 = 0; c0 < nvec; c0 += 32)
    launch_cgs<0>(s, nb, std::min(32, nvec - c0), V + (int64_t)c0 * ldv, ldv,
                  nullptr, const_cast<double*>(w), n, partial, nvec, c0);
  finish(s, nb, nvec, partial, out);
}

void cgs_update_dot(hipStream_t s, int nvec, const double* V, int64_t ldv,
                    const double* h, double* w, int64_t n, double* partial,
                    double* out) {
  QTP_REQUIRE(nvec >= 1 && nvec <= kMaxVec, -1, "cgs_update_dot: nvec out of range");
  const int nb = grid_for(n);
  if (nvec <= 32) {
    launch_cgs<1>(s, nb, nvec, V, ldv, h, w, n, partial, nvec, 0);
    finish(s, nb, nvec, partial, out);
    return;
  }
  for (int c0 = 0; c0 < nvec; c0 += 32)
    launch_cgs<3>(s, nb, std::min(32, nvec - c0), V + (int64_t)c0 * ldv, ldv,
                  h + c0, w, n, partial, 0, 0);
  multi_dot(s, nvec, V, ldv, w, n, partial, out);
}

void cgs_update_norm2(hipStream_t s, int nvec, const double* V, int64_t ldv,
                      const double* h, double* w, int64_t n, double* partial,
                      double* out) {
  QTP_REQUIRE(nvec >= 1 && nvec <= kMaxVec, -1, "cgs_update_norm2: nvec out of range");
  const int nb = grid_for(n);
  int c0 = 0;
  for (; nvec - c0 > 32; c0 += 32)
    launch_cgs<3>(s, nb, 32, V + (int64_t)c0 * ldv, ldv, h + c0, w, n, partial, 0, 0);
  launch_cgs<2>(s, nb, nvec - c0, V + (int64_t)c0 * ldv, ldv, h + c0, w, n, partial,
                1, 0);
  finish(s, nb, 1, partial, out);
}

void dot(hipStream_t s, const double* x, const double* y, int64_t n,
         double* partial, double* out) {
  multi_dot(s, 1, x, n, y, n, partial, out);
}

void scale_dev(hipStream_t s, const double* a_dev, int inv, const double* x,
               double* y, int64_t n) {
  scale_kernel<<<grid_for(n), kThreads, 0, s>>>(a_dev, inv, x, y, n);
  QTP_CHECK_LAUNCH();
}

void multi_axpy(hipStream_t s, int nvec, const double* X, int64_t ldx,
                const double* c, double* y, int64_t n) {
  QTP_REQUIRE(nvec >= 1 && nvec <= kMaxVec, -1, "multi_axpy: nvec out of range");
  multi_axpy_kernel<<<grid_for(n), kThreads, 0, s>>>(nvec, X, ldx, c, y, n);
  QTP_CHECK_LAUNCH();
}

void sub(hipStream_t s, const double* x, const double* y, double* z, int64_t n) {
  sub_kernel<<<grid_for(n), kThreads, 0, s>>>(x, y, z, n);
  QTP_CHECK_LAUNCH();
}

void add_inplace(hipStream_t s, const double* x, double* y, int64_t n) {
  add_kernel<<<grid_for(n), kThreads, 0, s>>>(x, y, n);
  QTP_CHECK_LAUNCH();
}

void any_nonfinite(hipStream_t s, const double* x, int64_t n, int* out) {
  nonfinite_kernel<<<grid_for(n), kThreads, 0, s>>>(x, n, out);
  QTP_CHECK_LAUNCH();
}

void bj_factor(hipStream_t s, int nslots, const int32_t* rp, const int32_t* col,
               const double* val, double* Linv, int* bad) {
  if (nslots <= 0) return;
  bj_factor_kernel<<<div_up(nslots, 256), 256, 0, s>>>(nslots, rp, col, val,
                                                       Linv, bad);
  QTP_CHECK_LAUNCH();
}

void bj_apply(hipStream_t s, int nslots, int64_t n, const double* Linv, int trans,
              const double* x, double* y) {
  const int64_t tail = n - 3 * (int64_t)nslots;
  const int64_t threads = (int64_t)nslots + tail;
  bj_apply_kernel<<<div_up(threads, 256), 256, 0, s>>>(nslots, n, Linv, trans, x,
                                                       y);
  QTP_CHECK_LAUNCH();
}

void bj_scale_matrix(hipStream_t s, int nslots, const int32_t* rp,
                     const int32_t* col, const double* val, const double* Linv,
                     double* vout) {
  if (nslots <= 0) return;
  bj_scale_matrix_kernel<<<nslots, 64, 0, s>>>(nslots, rp, col, val, Linv, vout);
  QTP_CHECK_LAUNCH();
}

}  // namespace qtp
