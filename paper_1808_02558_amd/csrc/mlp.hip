// Learned warm start of the PDIP: per-contact features and a 3 x 128 FP32
// MLP (11 -> 128 -> 128 -> 128 -> 3, tanh hidden layers) with its own
// forward, backward and Adam kernels.
//
// The paper starts each PDIP from zero tangential impulses and a preset
// normal impulse because warm starts drift off the central path (Sec. 3.3,
// "Re-using information across timesteps").  Here the network predicts each
// contact's impulse from local features; the PDIP starts from that point,
// strictly inside the cone, with multipliers on the central path of t0, and
// falls back to the cold start when it does not converge.
//
// Features (scaled units): Phi/(h g h), D_i^T v/(g h) (3), n (3),
// r_a/r_bar, r_b/r_bar (0 for a wall), contacts of a, contacts of b (0 for a
// wall).  Output p: gamma_n = exp(p0), gamma_t = 0.9 mu gamma_n (p1, p2) /
// max(1, |(p1, p2)|).  Loss: mean over rows and outputs of (p - y)^2.
#include <cmath>

#include "dense.h"
#include "mlp.h"
#include "timestep.h"

namespace qtp {
namespace {

constexpr int kT = 256;

// ---- features ---------------------------------------------------------------
__global__ void features_kernel(int nc, int M, double h, double vbar, double rbar,
                                const int32_t* __restrict__ a,
                                const int32_t* __restrict__ b,
                                const double* __restrict__ phi,
                                const double* __restrict__ frame,
                                const double* __restrict__ rad,
                                const double* __restrict__ v,
                                const double* __restrict__ w,
                                const int32_t* __restrict__ bptr,
                                float* __restrict__ X) {
  const int i = blockIdx.x * kT + threadIdx.x;
  if (i >= nc) return;
  const bool wall = b[i] >= M;
  const int B = wall ? a[i] : b[i];
  const int A = wall ? -1 : a[i];
  const double* f = frame + 9 * (int64_t)i;
  double rel[3] = {0.0, 0.0, 0.0};
  for (int role = 0; role < 2; ++role) {
    const int body = role == 0 ? B : A;
    if (body < 0) continue;
    const double sgn = role == 1 ? -1.0 : 1.0;
    const double rr = rad[body];
    for (int c = 0; c < 3; ++c) {
      const double d0 = f[3 * c], d1 = f[3 * c + 1], d2 = f[3 * c + 2];
      const double x0 = f[1] * d2 - f[2] * d1;
      const double x1 = f[2] * d0 - f[0] * d2;
      const double x2 = f[0] * d1 - f[1] * d0;
      rel[c] += sgn * (d0 * v[3 * body] + d1 * v[3 * body + 1] + d2 * v[3 * body + 2]) -
                rr * (x0 * w[3 * body] + x1 * w[3 * body + 1] + x2 * w[3 * body + 2]);
    }
  }
  float* o = X + 11 * (int64_t)i;
  o[0] = (float)(phi[i] / h / vbar);
  for (int c = 0; c < 3; ++c) o[1 + c] = (float)(rel[c] / vbar);
  for (int c = 0; c < 3; ++c) o[4 + c] = (float)f[c];
  o[7] = (float)(rad[a[i]] / rbar);
  o[8] = wall ? 0.f : (float)(rad[b[i]] / rbar);
  o[9] = (float)(bptr[a[i] + 1] - bptr[a[i]]);
  o[10] = wall ? 0.f : (float)(bptr[b[i] + 1] - bptr[b[i]]);
}

// ---- FP32 GEMM with fused epilogue -----------------------------------------
// C[M x N] = epi(op(A) op(B)); EPI 0: plain, 1: + bias, 2: tanh(. + bias),
// 3: . * (1 - H^2) with H [M x N] (the tanh derivative).  Split-K partials
// (EPI 0 only) are reduced in a fixed order.
constexpr int TM = 64, TN = 64, TK = 16;

template <int EPI>
__global__ __launch_bounds__(256) void sgemm_kernel(
    int transA, int transB, int M, int N, int K, int kchunk,
    const float* __restrict__ A, int lda, const float* __restrict__ B, int ldb,
    float* __restrict__ C, int ldc, const float* __restrict__ bias,
    const float* __restrict__ H, int partial_mode) {
  __shared__ float As[TK][TM + 1];
  __shared__ float Bs[TK][TN + 1];
  const int tx = threadIdx.x & 15, ty = threadIdx.x >> 4;
  const int m0 = blockIdx.x * TM, n0 = blockIdx.y * TN;
  const int kbeg = blockIdx.z * kchunk;
  const int kend = min(K, kbeg + kchunk);
  float acc[4][4] = {};
  for (int k0 = kbeg; k0 < kend; k0 += TK) {
    for (int e = threadIdx.x; e < TM * TK; e += 256) {
      int mm, kk;
      if (!transA) { mm = e / TK; kk = e % TK; } else { kk = e / TM; mm = e % TM; }
      const int gm = m0 + mm, gk = k0 + kk;
      float v = 0.f;
      if (gm < M && gk < kend)
        v = transA ? A[(int64_t)gk * lda + gm] : A[(int64_t)gm * lda + gk];
      As[kk][mm] = v;
    }
    for (int e = threadIdx.x; e < TK * TN; e += 256) {
      int kk, nn;
      if (!transB) { kk = e / TN; nn = e % TN; } else { nn = e / TK; kk = e % TK; }
      const int gn = n0 + nn, gk = k0 + kk;
      float v = 0.f;
      if (gn < N && gk < kend)
        v = transB ? B[(int64_t)gn * ldb + gk] : B[(int64_t)gk * ldb + gn];
      Bs[kk][nn] = v;
    }
    __syncthreads();
#pragma unroll
    for (int kk = 0; kk < TK; ++kk) {
      float a[4], bb[4];
#pragma unroll
      for (int i = 0; i < 4; ++i) a[i] = As[kk][ty + 16 * i];
#pragma unroll
      for (int j = 0; j < 4; ++j) bb[j] = Bs[kk][tx + 16 * j];
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) acc[i][j] += a[i] * bb[j];
    }
    __syncthreads();
  }
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const int gm = m0 + ty + 16 * i;
    if (gm >= M) continue;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int gn = n0 + tx + 16 * j;
      if (gn >= N) continue;
      float v = acc[i][j];
      if (partial_mode) {
        C[((int64_t)blockIdx.z * M + gm) * N + gn] = v;
        continue;
      }
      if (EPI == 1 || EPI == 2) v += bias[gn];
      if (EPI == 2) v = tanhf(v);
      if (EPI == 3) {
        const float hh = H[(int64_t)gm * ldc + gn];
        v *= 1.f - hh * hh;
      }
      C[(int64_t)gm * ldc + gn] = v;
    }
  }
}

__global__ void sreduce_kernel(int M, int N, int nsplit, const float* __restrict__ part,
                               float* __restrict__ C, int ldc) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (int64_t)M * N) return;
  float s = 0.f;
  for (int z = 0; z < nsplit; ++z) s += part[(int64_t)z * M * N + e];
  C[(e / N) * ldc + e % N] = s;
}

// column sums of G [M x N] into out[N] (fixed order over rows)
__global__ void colsum_kernel(int M, int N, const float* __restrict__ G,
                              float* __restrict__ out) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= N) return;
  float s = 0.f;
  for (int r = 0; r < M; ++r) s += G[(int64_t)r * N + c];
  out[c] = s;
}

// G = 2 (P - Y) / (3 B); per-block partial sums of (P - Y)^2
__global__ void loss_grad_kernel(int B, const float* __restrict__ P,
                                 const float* __restrict__ Y, float* __restrict__ G,
                                 double* __restrict__ part) {
  __shared__ double sh[kT];
  double acc = 0.0;
  for (int e = blockIdx.x * kT + threadIdx.x; e < 3 * B; e += gridDim.x * kT) {
    const float d = P[e] - Y[e];
    G[e] = 2.f * d / (3.f * (float)B);
    acc += (double)d * d;
  }
  sh[threadIdx.x] = acc;
  __syncthreads();
  for (int o = kT / 2; o > 0; o >>= 1) {
    if (threadIdx.x < o) sh[threadIdx.x] += sh[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[blockIdx.x] = sh[0];
}

__global__ void normalise_kernel(int64_t n, const float* __restrict__ X,
                                 const float* __restrict__ mean,
                                 const float* __restrict__ istd, float* __restrict__ Xn) {
  const int64_t e = (int64_t)blockIdx.x * kT + threadIdx.x;
  if (e >= n * 11) return;
  const int k = (int)(e % 11);
  Xn[e] = (X[e] - mean[k]) * istd[k];
}

// per-block partial sums of x and x^2 per feature
__global__ void moments_kernel(int64_t n, const float* __restrict__ X,
                               double* __restrict__ part) {
  __shared__ double s1[11][kT / 64], s2[11][kT / 64];
  double a[11], q[11];
  for (int k = 0; k < 11; ++k) a[k] = q[k] = 0.0;
  for (int64_t r = (int64_t)blockIdx.x * kT + threadIdx.x; r < n; r += (int64_t)gridDim.x * kT)
    for (int k = 0; k < 11; ++k) {
      const double x = X[r * 11 + k];
      a[k] += x;
      q[k] += x * x;
    }
  const int wv = threadIdx.x >> 6;
  for (int k = 0; k < 11; ++k) {
    double u = a[k], v = q[k];
    for (int o = 32; o > 0; o >>= 1) {
      u += __shfl_xor(u, o, 64);
      v += __shfl_xor(v, o, 64);
    }
    if ((threadIdx.x & 63) == 0) {
      s1[k][wv] = u;
      s2[k][wv] = v;
    }
  }
  __syncthreads();
  if (threadIdx.x < 11) {
    double u = 0.0, v = 0.0;
    for (int i = 0; i < kT / 64; ++i) {
      u += s1[threadIdx.x][i];
      v += s2[threadIdx.x][i];
    }
    part[blockIdx.x * 22 + threadIdx.x] = u;
    part[blockIdx.x * 22 + 11 + threadIdx.x] = v;
  }
}

__global__ void adam_kernel(int64_t n, float* __restrict__ p, const float* __restrict__ g,
                            float* __restrict__ m, float* __restrict__ v, float lr,
                            float b1, float b2, float eps, float c1, float c2) {
  const int64_t i = (int64_t)blockIdx.x * kT + threadIdx.x;
  if (i >= n) return;
  const float gi = g[i];
  const float mi = b1 * m[i] + (1.f - b1) * gi;
  const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
  m[i] = mi;
  v[i] = vi;
  p[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
}

// predicted impulses into the PDIP start (scaled units), multipliers on the
// central path of t0
__global__ void warm_start_kernel(int nc, double mu, double t0, double floor_n,
                                  const int32_t* __restrict__ slot,
                                  const float* __restrict__ P,
                                  double* __restrict__ gamma, double* __restrict__ lam) {
  const int i = blockIdx.x * kT + threadIdx.x;
  if (i >= nc) return;
  const float* p = P + 3 * (int64_t)i;
  double gn = fmax(exp(fmin(fmax((double)p[0], -30.0), 30.0)), floor_n);
  double q1 = p[1], q2 = p[2];
  const double nq = fmax(1.0, sqrt(q1 * q1 + q2 * q2));
  const double g1 = 0.9 * mu * gn * q1 / nq, g2 = 0.9 * mu * gn * q2 / nq;
  const int64_t u = 3 * (int64_t)slot[i];
  gamma[u] = gn;
  gamma[u + 1] = g1;
  gamma[u + 2] = g2;
  const double f1 = (g1 * g1 + g2 * g2) / (2.0 * mu * gn) - 0.5 * mu * gn;
  lam[i] = 1.0 / (t0 * (-f1));
  lam[nc + i] = 1.0 / (t0 * gn);
}

// training targets of the solved impulses (scaled units): log gamma_n and the
// friction ratio gamma_t / (mu gamma_n) projected into the unit disc
__global__ void targets_kernel(int nc, double mu, const int32_t* __restrict__ slot,
                               const double* __restrict__ gamma, float* __restrict__ Y) {
  const int i = blockIdx.x * kT + threadIdx.x;
  if (i >= nc) return;
  const int64_t u = 3 * (int64_t)slot[i];
  const double gn = gamma[u];
  const double q1 = gamma[u + 1] / (mu * gn), q2 = gamma[u + 2] / (mu * gn);
  const double nq = fmax(1.0, sqrt(q1 * q1 + q2 * q2));
  Y[3 * (int64_t)i] = (float)log(fmax(gn, 1e-6));
  Y[3 * (int64_t)i + 1] = (float)(q1 / nq);
  Y[3 * (int64_t)i + 2] = (float)(q2 / nq);
}

void sgemm(hipStream_t s, int transA, int transB, int M, int N, int K, const float* A,
           int lda, const float* B, int ldb, float* C, int ldc, int epi,
           const float* bias, const float* H, DevBuf* ws) {
  const dim3 tiles(div_up(M, TM), div_up(N, TN), 1);
  const int ntiles = (int)(tiles.x * tiles.y);
  if (epi == 0 && ws && ntiles < 64 && K > 1024) {
    int nsplit = std::min(div_up(K, 256), 256 / ntiles + 1);
    const int kchunk = div_up(div_up(K, nsplit), TK) * TK;
    nsplit = div_up(K, kchunk);
    ws->ensure(sizeof(float) * (size_t)nsplit * M * N);
    sgemm_kernel<0><<<dim3(tiles.x, tiles.y, nsplit), 256, 0, s>>>(
        transA, transB, M, N, K, kchunk, A, lda, B, ldb, ws->as<float>(), N, nullptr,
        nullptr, 1);
    QTP_CHECK_LAUNCH();
    sreduce_kernel<<<div_up((int64_t)M * N, 256), 256, 0, s>>>(M, N, nsplit,
                                                              ws->as<float>(), C, ldc);
    QTP_CHECK_LAUNCH();
    return;
  }
  const int kchunk = div_up(std::max(K, 1), TK) * TK;
  switch (epi) {
    case 0:
      sgemm_kernel<0><<<tiles, 256, 0, s>>>(transA, transB, M, N, K, kchunk, A, lda, B,
                                            ldb, C, ldc, bias, H, 0);
      break;
    case 1:
      sgemm_kernel<1><<<tiles, 256, 0, s>>>(transA, transB, M, N, K, kchunk, A, lda, B,
                                            ldb, C, ldc, bias, H, 0);
      break;
    case 2:
      sgemm_kernel<2><<<tiles, 256, 0, s>>>(transA, transB, M, N, K, kchunk, A, lda, B,
                                            ldb, C, ldc, bias, H, 0);
      break;
    default:
      sgemm_kernel<3><<<tiles, 256, 0, s>>>(transA, transB, M, N, K, kchunk, A, lda, B,
                                            ldb, C, ldc, bias, H, 0);
  }
  QTP_CHECK_LAUNCH();
}

constexpr int kL[5] = {11, 128, 128, 128, 3};

}  // namespace

int64_t mlp_param_count() {
  int64_t t = 0;
  for (int l = 0; l < 4; ++l) t += (int64_t)kL[l] * kL[l + 1] + kL[l + 1];
  return t;
}

// offsets of W_l and b_l in the flat parameter vector
static void offsets(int64_t* W, int64_t* bo) {
  int64_t o = 0;
  for (int l = 0; l < 4; ++l) {
    W[l] = o;
    o += (int64_t)kL[l] * kL[l + 1];
    bo[l] = o;
    o += kL[l + 1];
  }
}

void mlp_features(Ctx& c, float* X) {
  QTP_REQUIRE(c.ct.valid && c.qp.valid && !c.qp.stale, QTP_E_STATE,
              "detect and assemble before computing features");
  Scene& sc = c.scene;
  const int nc = c.ct.nc;
  if (nc == 0) return;
  // mean radius (fixed-order host sum of block partials)
  std::vector<double> r(sc.M);
  QTP_HIP(hipMemcpyAsync(r.data(), sc.radius.get(), sizeof(double) * sc.M,
                         hipMemcpyDeviceToHost, c.stream));
  QTP_HIP(hipStreamSynchronize(c.stream));
  double rs = 0.0;
  for (double x : r) rs += x;
  const double rbar = rs / sc.M;
  features_kernel<<<div_up(nc, kT), kT, 0, c.stream>>>(
      nc, sc.M, sc.h, c.qp.vbar, rbar, c.ct.a.as<int32_t>(), c.ct.b.as<int32_t>(),
      c.ct.phi.as<double>(), c.ct.frame.as<double>(), sc.radius.as<double>(),
      sc.v.as<double>(), sc.w.as<double>(), c.qp.body_ptr.as<int32_t>(), X);
  QTP_CHECK_LAUNCH();
  QTP_HIP(hipStreamSynchronize(c.stream));
}

void mlp_set_params(Ctx& c, const float* params) {
  Mlp& m = c.mlp;
  const int64_t np = mlp_param_count();
  m.params.ensure(sizeof(float) * np);
  m.grads.ensure(sizeof(float) * np);
  m.m1.ensure(sizeof(float) * np);
  m.m2.ensure(sizeof(float) * np);
  QTP_HIP(hipMemcpyAsync(m.params.get(), params, sizeof(float) * np,
                         hipMemcpyDeviceToDevice, c.stream));
  QTP_HIP(hipMemsetAsync(m.m1.get(), 0, sizeof(float) * np, c.stream));
  QTP_HIP(hipMemsetAsync(m.m2.get(), 0, sizeof(float) * np, c.stream));
  m.adam_t = 0;
  m.have_params = true;
  if (!m.have_norm) {
    std::vector<float> mean(11, 0.f), istd(11, 1.f);
    m.mean.ensure(sizeof(float) * 11);
    m.istd.ensure(sizeof(float) * 11);
    QTP_HIP(hipMemcpyAsync(m.mean.get(), mean.data(), sizeof(float) * 11,
                           hipMemcpyHostToDevice, c.stream));
    QTP_HIP(hipMemcpyAsync(m.istd.get(), istd.data(), sizeof(float) * 11,
                           hipMemcpyHostToDevice, c.stream));
  }
  QTP_HIP(hipStreamSynchronize(c.stream));
}

void mlp_fit_normalisation(Ctx& c, const float* X, int64_t n) {
  QTP_REQUIRE(n >= 2, QTP_E_ARG, "need at least two rows");
  const int nb = (int)std::min<int64_t>(256, div_up(n, kT));
  c.mlp.part.ensure(sizeof(double) * 22 * nb);
  moments_kernel<<<nb, kT, 0, c.stream>>>(n, X, c.mlp.part.as<double>());
  QTP_CHECK_LAUNCH();
  std::vector<double> h(22 * nb);
  QTP_HIP(hipMemcpyAsync(h.data(), c.mlp.part.get(), sizeof(double) * 22 * nb,
                         hipMemcpyDeviceToHost, c.stream));
  QTP_HIP(hipStreamSynchronize(c.stream));
  std::vector<float> mean(11), istd(11);
  for (int k = 0; k < 11; ++k) {
    double s1 = 0.0, s2 = 0.0;
    for (int b = 0; b < nb; ++b) {
      s1 += h[22 * b + k];
      s2 += h[22 * b + 11 + k];
    }
    const double mu = s1 / n;
    const double var = std::max(s2 / n - mu * mu, 0.0);
    mean[k] = (float)mu;
    istd[k] = (float)(var > 1e-12 ? 1.0 / std::sqrt(var) : 1.0);
  }
  c.mlp.mean.ensure(sizeof(float) * 11);
  c.mlp.istd.ensure(sizeof(float) * 11);
  QTP_HIP(hipMemcpyAsync(c.mlp.mean.get(), mean.data(), sizeof(float) * 11,
                         hipMemcpyHostToDevice, c.stream));
  QTP_HIP(hipMemcpyAsync(c.mlp.istd.get(), istd.data(), sizeof(float) * 11,
                         hipMemcpyHostToDevice, c.stream));
  QTP_HIP(hipStreamSynchronize(c.stream));
  c.mlp.have_norm = true;
}

void mlp_get_normalisation(Ctx& c, float* mean_host, float* istd_host) {
  QTP_REQUIRE(c.mlp.have_norm, QTP_E_STATE, "no normalisation fitted");
  QTP_HIP(hipMemcpyAsync(mean_host, c.mlp.mean.get(), sizeof(float) * 11,
                         hipMemcpyDeviceToHost, c.stream));
  QTP_HIP(hipMemcpyAsync(istd_host, c.mlp.istd.get(), sizeof(float) * 11,
                         hipMemcpyDeviceToHost, c.stream));
  QTP_HIP(hipStreamSynchronize(c.stream));
}

// forward pass on B rows; keeps the activations for a backward pass
void mlp_forward(Ctx& c, const float* X, int B, float* P) {
  Mlp& m = c.mlp;
  QTP_REQUIRE(m.have_params, QTP_E_STATE, "MLP parameters not set");
  const hipStream_t s = c.stream;
  int64_t Wo[4], bo[4];
  offsets(Wo, bo);
  const float* prm = m.params.as<float>();
  m.xn.ensure(sizeof(float) * 11 * (size_t)B);
  for (int l = 0; l < 3; ++l) m.h[l].ensure(sizeof(float) * 128 * (size_t)B);
  normalise_kernel<<<div_up((int64_t)B * 11, kT), kT, 0, s>>>(
      B, X, m.mean.as<float>(), m.istd.as<float>(), m.xn.as<float>());
  QTP_CHECK_LAUNCH();
  const float* in = m.xn.as<float>();
  for (int l = 0; l < 4; ++l) {
    float* out = l < 3 ? m.h[l].as<float>() : P;
    sgemm(s, 0, 0, B, kL[l + 1], kL[l], in, kL[l], prm + Wo[l], kL[l + 1], out,
          kL[l + 1], l < 3 ? 2 : 1, prm + bo[l], nullptr, nullptr);
    in = out;
  }
}

double mlp_loss_grad(Ctx& c, const float* X, const float* Y, int B) {
  Mlp& m = c.mlp;
  const hipStream_t s = c.stream;
  m.p.ensure(sizeof(float) * 3 * (size_t)B);
  mlp_forward(c, X, B, m.p.as<float>());
  int64_t Wo[4], bo[4];
  offsets(Wo, bo);
  const float* prm = m.params.as<float>();
  float* grd = m.grads.as<float>();
  m.g[0].ensure(sizeof(float) * 128 * (size_t)B);
  m.g[1].ensure(sizeof(float) * 128 * (size_t)B);
  m.g3.ensure(sizeof(float) * 3 * (size_t)B);
  const int nb = std::min(256, div_up((int64_t)3 * B, kT));
  m.part.ensure(sizeof(double) * std::max(nb, 22 * 256));
  loss_grad_kernel<<<nb, kT, 0, s>>>(B, m.p.as<float>(), Y, m.g3.as<float>(),
                                     m.part.as<double>());
  QTP_CHECK_LAUNCH();
  std::vector<double> h(nb);
  QTP_HIP(hipMemcpyAsync(h.data(), m.part.get(), sizeof(double) * nb,
                         hipMemcpyDeviceToHost, s));
  // backward through the 4 layers; G holds dLoss/d(pre-activation output)
  const float* G = m.g3.as<float>();
  int gi = 0;
  for (int l = 3; l >= 0; --l) {
    const float* hin = l == 0 ? m.xn.as<float>() : m.h[l - 1].as<float>();
    // dW_l = h_in^T G, db_l = column sums of G
    sgemm(s, 1, 0, kL[l], kL[l + 1], B, hin, kL[l], G, kL[l + 1], grd + Wo[l],
          kL[l + 1], 0, nullptr, nullptr, &m.ws);
    colsum_kernel<<<1, 256, 0, s>>>(B, kL[l + 1], G, grd + bo[l]);
    QTP_CHECK_LAUNCH();
    if (l > 0) {
      float* Gn = m.g[gi].as<float>();
      // G_{l-1} = (G W_l^T) * (1 - h_{l-1}^2)
      sgemm(s, 0, 1, B, kL[l], kL[l + 1], G, kL[l + 1], prm + Wo[l], kL[l + 1], Gn,
            kL[l], 3, nullptr, m.h[l - 1].as<float>(), nullptr);
      G = Gn;
      gi ^= 1;
    }
  }
  QTP_HIP(hipStreamSynchronize(s));
  double sse = 0.0;
  for (double v : h) sse += v;
  return sse / (3.0 * B);
}

double mlp_train_step(Ctx& c, const float* X, const float* Y, int B, double lr) {
  const double loss = mlp_loss_grad(c, X, Y, B);
  Mlp& m = c.mlp;
  const int64_t np = mlp_param_count();
  m.adam_t += 1;
  const double b1 = 0.9, b2 = 0.999;
  const float c1 = (float)(1.0 - std::pow(b1, m.adam_t));
  const float c2 = (float)(1.0 - std::pow(b2, m.adam_t));
  adam_kernel<<<div_up(np, kT), kT, 0, c.stream>>>(
      np, m.params.as<float>(), m.grads.as<float>(), m.m1.as<float>(), m.m2.as<float>(),
      (float)lr, (float)b1, (float)b2, 1e-8f, c1, c2);
  QTP_CHECK_LAUNCH();
  QTP_HIP(hipStreamSynchronize(c.stream));
  return loss;
}

void mlp_targets(Ctx& c, float* Y) {
  QTP_REQUIRE(c.pd.have_gamma, QTP_E_STATE, "solve the PDIP before computing targets");
  const int nc = c.ct.nc;
  if (nc == 0) return;
  targets_kernel<<<div_up(nc, kT), kT, 0, c.stream>>>(
      nc, c.scene.mu, c.ct.slot.as<int32_t>(), c.pd.gamma.as<double>(), Y);
  QTP_CHECK_LAUNCH();
  QTP_HIP(hipStreamSynchronize(c.stream));
}

// features -> prediction -> PDIP start (gamma, lambda) on the padded layout
void mlp_warm_start(Ctx& c, double t0, double* gamma, double* lam) {
  const int nc = c.ct.nc;
  Mlp& m = c.mlp;
  m.feat.ensure(sizeof(float) * 11 * (size_t)std::max(nc, 1));
  m.p.ensure(sizeof(float) * 3 * (size_t)std::max(nc, 1));
  mlp_features(c, m.feat.as<float>());
  mlp_forward(c, m.feat.as<float>(), nc, m.p.as<float>());
  warm_start_kernel<<<div_up(nc, kT), kT, 0, c.stream>>>(
      nc, c.scene.mu, t0, c.cfg.warm_floor, c.ct.slot.as<int32_t>(), m.p.as<float>(),
      gamma, lam);
  QTP_CHECK_LAUNCH();
}

}  // namespace qtp
