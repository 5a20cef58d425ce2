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

Arnoldi arnoldi_state(Ctx& c) {
  if (c.arn_status.empty()) {
    c.arn_status.alloc(sizeof(double) * kArnRing);
    double* h = c.arn_status.host<double>();
    for (int i = 0; i < kArnRing; ++i) h[i] = kArnEmpty;
  }
  c.arn_d.ensure(sizeof(double) * kArnDoubles);
  c.arn_partial.ensure(sizeof(double) * arnoldi_partial_doubles(c.n));
  Arnoldi a;
  a.d = c.arn_d.as<double>();
  a.partial = c.arn_partial.as<double>();
  a.status = c.arn_status.dev<double>();
  return a;
}

// Waits until the device has stored status entry `tag`, returns it and empties
// the slot again (the device is at most one step ahead, far less than the
// ring).  Polls the stream now and then so that a failed or finished stream
// cannot leave the host spinning.
double wait_status(Ctx& c, int64_t tag) {
  double* e = c.arn_status.host<double>() + (tag & (kArnRing - 1));
  int64_t spins = 0;
  double v;
  while ((v = *reinterpret_cast<volatile double*>(e)) == kArnEmpty) {
    if ((++spins & 1023) == 0) {
      const hipError_t q = hipStreamQuery(c.stream);
      if (q == hipSuccess) {
        v = *reinterpret_cast<volatile double*>(e);
        if (v != kArnEmpty) break;
        throw Error(QTP_E_HIP, "FGMRES: residual estimate missing after the stream drained");
      }
      if (q != hipErrorNotReady) QTP_HIP(q);
    }
    __builtin_ia32_pause();
  }
  *reinterpret_cast<volatile double*>(e) = kArnEmpty;
  return v;
}

// Right-preconditioned FGMRES(m).  Within a restart cycle the host queues step
// j and only then reads the residual estimate of step j - 1, so the device
// always has the next step queued; a step queued after convergence is
// discarded (it touches only column j of the Hessenberg and entries >= j of
// g).  Each cycle ends with the true residual rhs - S x.
int fgmres(Ctx& c, const double* rhs, double* x, qtp_solve_stats* st) {
  const int64_t n = c.n;
  const int m = c.cfg.fgmres_restart;
  ensure_krylov(c, m);
  const Arnoldi a = arnoldi_state(c);
  double* V = c.V.as<double>();
  double* Z = c.Z.as<double>();
  double* r = c.r.as<double>();
  double* t1 = c.t1.as<double>();
  double* t2 = c.t2.as<double>();
  const double tol = c.cfg.solve_tol;
  const bool qtt = c.have_inverse && c.use_qtt;
  const double* Linv = c.Linv.as<double>();

  const double bnorm = norm2(c, rhs);  // synchronises: no step is in flight
  {
    double* ring = c.arn_status.host<double>();
    for (int i = 0; i < kArnRing; ++i) ring[i] = kArnEmpty;
  }
  QTP_HIP(hipMemsetAsync(x, 0, sizeof(double) * n, c.stream));
  if (!(std::isfinite(bnorm))) throw Error(QTP_E_NUMERIC, "rhs is not finite");
  if (bnorm == 0.0) {
    st->iterations = 0;
    st->rel_residual = 0.0;
    return QTP_OK;
  }
  const void* qcores = nullptr;
  if (qtt) {
    qcores = c.X.cores.get();
    if (c.cfg.precision != 0) {
      ensure_lp_cores(c, c.X);
      qcores = c.X.cores_lp.get();
    }
    c.qtt_work.ensure(qtt_apply_workspace(c.X.d, c.X.ranks.data(), c.cfg.precision));
  }
  double beta = bnorm;
  const double* res_src = rhs;  // x = 0: the first residual is rhs itself
  int it = 0;
  std::vector<int64_t> tags(m);
  while (it < c.cfg.fgmres_maxit && beta > tol * bnorm) {
    const int jmax = std::min(m, c.cfg.fgmres_maxit - it);
    int jend = jmax;
    for (int j = 0; j < jmax; ++j) {
      double* vj = V + (int64_t)j * n;
      double* zj = Z + (int64_t)j * n;
      double* w = V + (int64_t)(j + 1) * n;
      {
        TimedLaunch tl(c, "arnoldi_next");
        arnoldi_next(c.stream, a, j == 0 ? 0 : j, V, n, c.nslots, 1.0 / beta, beta,
                     j == 0 ? res_src : vj, vj, Linv, qtt ? 0 : 1, qtt ? t1 : zj);
      }
      if (qtt) {
        {
          TimedLaunch tl(c, "qtt_apply");
          qtt_apply(c.stream, c.X.d, c.X.ranks.data(), qcores, c.cfg.precision, t1, t2,
                    c.qtt_work.get());
        }
        bj_apply(c.stream, c.nslots, n, Linv, 1, t2, zj);
      }
      spmv(c, zj, w);
      {
        TimedLaunch tl(c, "arnoldi_dots");
        arnoldi_dots(c.stream, a, j + 1, V, n, w);
      }
      tags[j] = ++c.arn_tag;
      {
        TimedLaunch tl(c, "arnoldi_orth");
        arnoldi_orth(c.stream, a, j + 1, V, n, w, tags[j]);
      }
      if (j >= 1) {
        const double res = wait_status(c, tags[j - 1]);
        if (!std::isfinite(res)) throw Error(QTP_E_NUMERIC, "FGMRES breakdown (NaN)");
        if (res <= tol * bnorm) {
          // converged or broke down; step j is discarded, but its status
          // slot is emptied once it lands so the ring stays consistent
          (void)wait_status(c, tags[j]);
          jend = j;
          break;
        }
      }
    }
    if (jend == jmax) {
      const double res = wait_status(c, tags[jmax - 1]);
      if (!std::isfinite(res)) throw Error(QTP_E_NUMERIC, "FGMRES breakdown (NaN)");
    }
    it += jend;
    arnoldi_solve(c.stream, a, jend);
    multi_axpy(c.stream, jend, Z, n, a.d + kArnY, x, n);
    beta = residual(c, rhs, x, r);
    res_src = r;
    if (!std::isfinite(beta)) throw Error(QTP_E_NUMERIC, "FGMRES: residual not finite");
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
  hipEvent_t e0 = c.take_event(), e1 = c.take_event();
  QTP_HIP(hipEventRecord(e0, c.stream));
  int rc = c.cfg.solve_mode == 0 ? refine(c, rhs, x, st) : fgmres(c, rhs, x, st);
  QTP_HIP(hipEventRecord(e1, c.stream));
  QTP_HIP(hipEventSynchronize(e1));
  float ms = 0.f;
  QTP_HIP(hipEventElapsedTime(&ms, e0, e1));
  st->ms = ms;
  c.event_pool.push_back(e0);
  c.event_pool.push_back(e1);
  return rc;
}

}  // namespace qtp
