// The Newton-step solve S x = rhs (Sec. 3.3, "TT Newton system solver"): the
// approximate QTT inverse used directly with iterative refinement, or as the
// right preconditioner of a flexible GMRES (Saad 1993) with classical
// Gram-Schmidt applied twice.  All vectors stay on the device; only the
// (m+1) x m Hessenberg matrix and its Givens rotations live on the host.
#include <hip/hip_bf16.h>

#include <cmath>

#include "context.h"

namespace qtp {
namespace {

constexpr int kThreads = 256;

__global__ void axpby_kernel(double a, const double* __restrict__ x, double b,
                             double* __restrict__ y, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * kThreads)
    y[i] = a * x[i] + (b == 0.0 ? 0.0 : b * y[i]);
}

__global__ void cast_f32_kernel(const double* __restrict__ x, float* __restrict__ y,
                                int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  if (i < n) y[i] = (float)x[i];
}

__global__ void cast_bf16_kernel(const double* __restrict__ x,
                                 uint16_t* __restrict__ y, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  if (i < n) {
    // round to nearest even from the FP32 value
    const float f = (float)x[i];
    uint32_t u = __float_as_uint(f);
    const uint32_t lsb = (u >> 16) & 1u;
    u += 0x7fffu + lsb;
    y[i] = (uint16_t)(u >> 16);
  }
}

void axpby(hipStream_t s, double a, const double* x, double b, double* y,
           int64_t n) {
  int64_t nb = (n + kThreads - 1) / kThreads;
  if (nb > 1024) nb = 1024;
  axpby_kernel<<<(int)nb, kThreads, 0, s>>>(a, x, b, y, n);
  QTP_CHECK_LAUNCH();
}

double read_scalar(Ctx& c, const double* dev) {
  double h = 0.0;
  QTP_HIP(hipMemcpyAsync(&h, dev, sizeof(double), hipMemcpyDeviceToHost, c.stream));
  QTP_HIP(hipStreamSynchronize(c.stream));
  return h;
}

double norm2(Ctx& c, const double* x) {
  double* sc = c.scal.as<double>();
  dot(c.stream, x, x, c.n, c.partial.as<double>(), sc);
  return std::sqrt(read_scalar(c, sc));
}

void ensure_krylov(Ctx& c, int m) {
  const int64_t n = c.n;
  c.V.ensure(sizeof(double) * (size_t)(m + 1) * n);
  c.Z.ensure(sizeof(double) * (size_t)m * n);
  c.w.ensure(sizeof(double) * n);
  c.r.ensure(sizeof(double) * n);
  c.t1.ensure(sizeof(double) * n);
  c.t2.ensure(sizeof(double) * n);
  c.partial.ensure(sizeof(double) * (size_t)reduce_blocks(n) * 64);
  c.scal.ensure(sizeof(double) * 256);
  c.flag.ensure(sizeof(int) * 16);
}

void spmv(Ctx& c, const double* x, double* y) {
  TimedLaunch tl(c, "bsr_spmv");
  bsr_spmv(c.stream, c.nslots, c.n, c.rp.as<int32_t>(), c.col.as<int32_t>(),
           c.val.as<double>(), x, y);
}

// r = rhs - S x ; returns |r|
double residual(Ctx& c, const double* rhs, const double* x, double* r) {
  spmv(c, x, r);
  sub(c.stream, rhs, r, r, c.n);
  return norm2(c, r);
}

int fgmres(Ctx& c, const double* rhs, double* x, qtp_solve_stats* st) {
  const int64_t n = c.n;
  const int m = c.cfg.fgmres_restart;
  ensure_krylov(c, m);
  double* V = c.V.as<double>();
  double* Z = c.Z.as<double>();
  double* r = c.r.as<double>();
  double* sc = c.scal.as<double>();
  double* part = c.partial.as<double>();
  const double tol = c.cfg.solve_tol;

  const double bnorm = norm2(c, rhs);
  QTP_HIP(hipMemsetAsync(x, 0, sizeof(double) * n, c.stream));
  if (!(std::isfinite(bnorm))) throw Error(QTP_E_NUMERIC, "rhs is not finite");
  if (bnorm == 0.0) {
    st->iterations = 0;
    st->rel_residual = 0.0;
    return QTP_OK;
  }
  QTP_HIP(hipMemcpyAsync(r, rhs, sizeof(double) * n, hipMemcpyDeviceToDevice,
                         c.stream));
  double beta = bnorm;
  int it = 0;
  std::vector<double> H((size_t)(m + 1) * m), cs(m), sn(m), g(m + 1), y(m);
  std::vector<double> hbuf(130);
  bool done = false;
  while (!done && it < c.cfg.fgmres_maxit) {
    if (beta <= tol * bnorm) break;
    axpby(c.stream, 1.0 / beta, r, 0.0, V, n);
    std::fill(g.begin(), g.end(), 0.0);
    g[0] = beta;
    int jend = 0;
    for (int j = 0; j < m; ++j) {
      double* vj = V + (int64_t)j * n;
      double* zj = Z + (int64_t)j * n;
      double* w = V + (int64_t)(j + 1) * n;
      precond_apply(c, vj, zj);
      spmv(c, zj, w);
      {
        TimedLaunch tl(c, "cgs2");
        multi_dot(c.stream, j + 1, V, n, w, n, part, sc);
        cgs_update_dot(c.stream, j + 1, V, n, sc, w, n, part, sc + 64);
        cgs_update_norm2(c.stream, j + 1, V, n, sc + 64, w, n, part, sc + 128);
      }
      QTP_HIP(hipMemcpyAsync(hbuf.data(), sc, sizeof(double) * 129,
                             hipMemcpyDeviceToHost, c.stream));
      QTP_HIP(hipStreamSynchronize(c.stream));
      double* Hj = &H[(size_t)j * (m + 1)];  // column j, length m+1
      for (int i = 0; i <= j; ++i) Hj[i] = hbuf[i] + hbuf[64 + i];
      const double hn = std::sqrt(hbuf[128]);
      Hj[j + 1] = hn;
      if (!std::isfinite(hn)) throw Error(QTP_E_NUMERIC, "FGMRES breakdown (NaN)");
      if (hn > 0.0) axpby(c.stream, 1.0 / hn, w, 0.0, w, n);
      for (int i = 0; i < j; ++i) {
        const double t = cs[i] * Hj[i] + sn[i] * Hj[i + 1];
        Hj[i + 1] = -sn[i] * Hj[i] + cs[i] * Hj[i + 1];
        Hj[i] = t;
      }
      const double den = std::hypot(Hj[j], Hj[j + 1]);
      cs[j] = Hj[j] / den;
      sn[j] = Hj[j + 1] / den;
      Hj[j] = den;
      Hj[j + 1] = 0.0;
      g[j + 1] = -sn[j] * g[j];
      g[j] = cs[j] * g[j];
      ++it;
      jend = j + 1;
      if (std::fabs(g[j + 1]) <= tol * bnorm || it >= c.cfg.fgmres_maxit || hn == 0.0)
        break;
    }
    // back substitution H y = g, then x += Z y
    for (int i = jend - 1; i >= 0; --i) {
      double t = g[i];
      for (int k = i + 1; k < jend; ++k) t -= H[(size_t)k * (m + 1) + i] * y[k];
      y[i] = t / H[(size_t)i * (m + 1) + i];
    }
    QTP_HIP(hipMemcpyAsync(sc + 192, y.data(), sizeof(double) * jend,
                           hipMemcpyHostToDevice, c.stream));
    multi_axpy(c.stream, jend, Z, n, sc + 192, x, n);
    beta = residual(c, rhs, x, r);
    if (beta <= tol * bnorm) done = true;
  }
  st->iterations = it;
  st->rel_residual = beta / bnorm;
  return beta <= tol * bnorm ? QTP_OK : QTP_NOT_CONVERGED;
}

// x = P rhs, then x += P (rhs - S x) until the residual meets the tolerance
int refine(Ctx& c, const double* rhs, double* x, qtp_solve_stats* st) {
  ensure_krylov(c, 1);
  double* r = c.r.as<double>();
  double* z = c.w.as<double>();
  const double bnorm = norm2(c, rhs);
  if (bnorm == 0.0) {
    QTP_HIP(hipMemsetAsync(x, 0, sizeof(double) * c.n, c.stream));
    st->iterations = 0;
    st->rel_residual = 0.0;
    return QTP_OK;
  }
  precond_apply(c, rhs, x);
  double rn = residual(c, rhs, x, r);
  int it = 0;
  while (rn > c.cfg.solve_tol * bnorm && it < c.cfg.fgmres_maxit) {
    precond_apply(c, r, z);
    add_inplace(c.stream, z, x, c.n);
    rn = residual(c, rhs, x, r);
    ++it;
    if (!std::isfinite(rn)) throw Error(QTP_E_NUMERIC, "refinement diverged");
  }
  st->iterations = it;
  st->rel_residual = rn / bnorm;
  return rn <= c.cfg.solve_tol * bnorm ? QTP_OK : QTP_NOT_CONVERGED;
}

}  // namespace

void ensure_lp_cores(Ctx& c, Qtt& q) {
  const int prec = c.cfg.precision;
  if (prec == 0 || q.lp_prec == prec) return;
  const int64_t tot = q.total();
  if (prec == 1) {
    q.cores_lp.ensure(sizeof(float) * tot);
    cast_f32_kernel<<<div_up(tot, kThreads), kThreads, 0, c.stream>>>(
        q.cores.as<double>(), q.cores_lp.as<float>(), tot);
  } else {
    q.cores_lp.ensure(sizeof(uint16_t) * tot);
    cast_bf16_kernel<<<div_up(tot, kThreads), kThreads, 0, c.stream>>>(
        q.cores.as<double>(), q.cores_lp.as<uint16_t>(), tot);
  }
  QTP_CHECK_LAUNCH();
  q.lp_prec = prec;
}

void precond_factor(Ctx& c) {
  QTP_REQUIRE(c.have_matrix, QTP_E_STATE, "no Newton matrix loaded");
  ensure_krylov(c, 1);
  c.Linv.ensure(sizeof(double) * 6 * (size_t)(c.nslots > 0 ? c.nslots : 1));
  int* bad = c.flag.as<int>();
  QTP_HIP(hipMemsetAsync(bad, 0, sizeof(int), c.stream));
  bj_factor(c.stream, c.nslots, c.rp.as<int32_t>(), c.col.as<int32_t>(),
            c.val.as<double>(), c.Linv.as<double>(), bad);
  int hbad = 0;
  QTP_HIP(hipMemcpyAsync(&hbad, bad, sizeof(int), hipMemcpyDeviceToHost, c.stream));
  QTP_HIP(hipStreamSynchronize(c.stream));
  QTP_REQUIRE(hbad == 0, QTP_E_NUMERIC,
              "block-Jacobi: a diagonal block is not positive definite");
}

void precond_apply(Ctx& c, const double* v, double* z) {
  QTP_REQUIRE(c.have_precond, QTP_E_STATE, "preconditioner not built");
  double* t1 = c.t1.as<double>();
  double* t2 = c.t2.as<double>();
  bj_apply(c.stream, c.nslots, c.n, c.Linv.as<double>(), 0, v, t1);
  if (c.have_inverse && c.use_qtt) {
    Qtt& X = c.X;
    const void* cores = X.cores.get();
    if (c.cfg.precision != 0) {
      ensure_lp_cores(c, X);
      cores = X.cores_lp.get();
    }
    c.qtt_work.ensure(qtt_apply_workspace(X.d, X.ranks.data(), c.cfg.precision));
    TimedLaunch tl(c, "qtt_apply");
    qtt_apply(c.stream, X.d, X.ranks.data(), cores, c.cfg.precision, t1, t2,
              c.qtt_work.get());
    bj_apply(c.stream, c.nslots, c.n, c.Linv.as<double>(), 1, t2, z);
  } else {
    bj_apply(c.stream, c.nslots, c.n, c.Linv.as<double>(), 1, t1, z);
  }
}

int newton_solve(Ctx& c, const double* rhs, double* x, qtp_solve_stats* st) {
  QTP_REQUIRE(c.have_matrix, QTP_E_STATE, "no Newton matrix loaded");
  QTP_REQUIRE(c.have_precond, QTP_E_STATE, "preconditioner not built");
  hipEvent_t e0, e1;
  QTP_HIP(hipEventCreate(&e0));
  QTP_HIP(hipEventCreate(&e1));
  QTP_HIP(hipEventRecord(e0, c.stream));
  int rc = c.cfg.solve_mode == 0 ? refine(c, rhs, x, st) : fgmres(c, rhs, x, st);
  QTP_HIP(hipEventRecord(e1, c.stream));
  QTP_HIP(hipEventSynchronize(e1));
  float ms = 0.f;
  QTP_HIP(hipEventElapsedTime(&ms, e0, e1));
  st->ms = ms;
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  return rc;
}

}  // namespace qtp
