// Primal-dual interior point on the conic QP of one time step (Sec. 2.4,
// "Primal-Dual Interior Point methods", "The PDIP step", "Application to the
// CCP"; Sec. 3.3 "PDIP iteration").  The paper leaves the t rule and the line
// search open; they are those of the textbook primal-dual method (Boyd &
// Vandenberghe, Convex Optimization, Sec. 11.7).
//
// Per contact i (scaled units, slot s_i):
//   f_i     = (g_1^2 + g_2^2) / (2 mu g_n) - mu g_n / 2   (cone, convex form:
//             the paper's quadratic divided by mu g_n > 0, same feasible set)
//   f_Nc+i  = -g_n
//   eta = -f^T lambda,  t = mu_pd m / eta,  m = 2 Nc
//   r_dual  = N g + r + Df^T lambda,  r_cent = -lambda f - 1/t
//   S = N + blockdiag(H_i),  H_i = l_i hess f_i + l_i/(-f_i) grad f_i grad f_i^T
//                                  + l_{Nc+i}/g_n e_n e_n^T
//   rhs = -(N g + r) + (1/t) (grad f_i / f_i + e_n / g_n)
//   Delta lambda from the second block row; step 0.99 min(1, -l/Dl), halved
//   until strictly feasible, then until |r_t| decreases by (1 - 0.01 s).
// Reductions are deterministic: per-block partials summed on the host in
// block order.
#include <algorithm>
#include <chrono>
#include <cmath>

#include "timestep.h"

namespace qtp {
namespace {

constexpr int kT = 256;
constexpr int kMaxBlk = 512;

struct ContactState {
  double gn, g1, g2, f1, f2, l1, l2;
  double gr[3];  // grad f_i of the cone constraint
};

__device__ inline void eval(double mu, double gn, double g1, double g2, double l1,
                            double l2, ContactState& cs) {
  cs.gn = gn; cs.g1 = g1; cs.g2 = g2; cs.l1 = l1; cs.l2 = l2;
  const double t2 = g1 * g1 + g2 * g2;
  cs.f1 = t2 / (2.0 * mu * gn) - 0.5 * mu * gn;
  cs.f2 = -gn;
  cs.gr[0] = -t2 / (2.0 * mu * gn * gn) - 0.5 * mu;
  cs.gr[1] = g1 / (mu * gn);
  cs.gr[2] = g2 / (mu * gn);
}

__device__ inline double block_reduce_sum(double v, double* sh) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  __syncthreads();
  if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = v;
  __syncthreads();
  double s = 0.0;
  for (int i = 0; i < kT / 64; ++i) s += sh[i];
  return s;
}

__device__ inline double block_reduce_max(double v, double* sh) {
  for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, 64));
  __syncthreads();
  if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = v;
  __syncthreads();
  double s = sh[0];
  for (int i = 1; i < kT / 64; ++i) s = fmax(s, sh[i]);
  return s;
}

__device__ inline double block_reduce_min(double v, double* sh) {
  for (int o = 32; o > 0; o >>= 1) v = fmin(v, __shfl_xor(v, o, 64));
  __syncthreads();
  if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = v;
  __syncthreads();
  double s = sh[0];
  for (int i = 1; i < kT / 64; ++i) s = fmin(s, sh[i]);
  return s;
}

__global__ void init_kernel(int nc, double mu, const int32_t* __restrict__ slot,
                            double* __restrict__ gamma, double* __restrict__ lam) {
  const int i = blockIdx.x * kT + threadIdx.x;
  if (i >= nc) return;
  const int64_t u = 3 * (int64_t)slot[i];
  gamma[u] = 1.0;
  gamma[u + 1] = 0.0;
  gamma[u + 2] = 0.0;
  ContactState cs;
  eval(mu, 1.0, 0.0, 0.0, 0.0, 0.0, cs);
  lam[i] = 1.0 / (-cs.f1);        // t0 = 1
  lam[nc + i] = 1.0 / (-cs.f2);
}

// Start from the previous step (Sec. 3.3, re-using information across time
// steps): a contact that kept its slot starts from its previous normal
// impulse (at least floor_n) and, with keep_t, its previous friction impulse
// pulled inside 0.9 of the cone (the paper zeroes it); other contacts take
// the cold start.  Multipliers on the central path of t0 for the re-used
// contacts, of t = 1 for the others.
__global__ void prev_start_kernel(int nc, double mu, double t0, double floor_n,
                                  int keep_t, const int32_t* __restrict__ slot,
                                  const int32_t* __restrict__ old_slot,
                                  const double* __restrict__ gprev,
                                  double* __restrict__ gamma, double* __restrict__ lam) {
  const int i = blockIdx.x * kT + threadIdx.x;
  if (i >= nc) return;
  const int64_t u = 3 * (int64_t)slot[i];
  double gn = 1.0, g1 = 0.0, g2 = 0.0, tc = 1.0;
  if (old_slot[i] >= 0) {
    gn = fmax(gprev[u], floor_n);
    if (keep_t) {
      g1 = gprev[u + 1];
      g2 = gprev[u + 2];
      const double gt = sqrt(g1 * g1 + g2 * g2), cap = 0.9 * mu * gn;
      if (gt > cap) {
        g1 *= cap / gt;
        g2 *= cap / gt;
      }
    }
    tc = t0;
  }
  gamma[u] = gn;
  gamma[u + 1] = g1;
  gamma[u + 2] = g2;
  ContactState cs;
  eval(mu, gn, g1, g2, 0.0, 0.0, cs);
  lam[i] = 1.0 / (tc * (-cs.f1));
  lam[nc + i] = 1.0 / (tc * (-cs.f2));
}

// partial: -f^T lambda
__global__ void gap_kernel(int nc, double mu, const int32_t* __restrict__ slot,
                           const double* __restrict__ gamma,
                           const double* __restrict__ lam, double* __restrict__ part) {
  __shared__ double sh[kT / 64];
  double acc = 0.0;
  for (int i = blockIdx.x * kT + threadIdx.x; i < nc; i += gridDim.x * kT) {
    const int64_t u = 3 * (int64_t)slot[i];
    ContactState cs;
    eval(mu, gamma[u], gamma[u + 1], gamma[u + 2], lam[i], lam[nc + i], cs);
    acc += -cs.f1 * cs.l1 - cs.f2 * cs.l2;
  }
  const double s = block_reduce_sum(acc, sh);
  if (threadIdx.x == 0) part[blockIdx.x] = s;
}

// residuals at (gamma + s dgamma, lambda + s dlambda) with u + s w:
// partial [3 per block]: sum r_dual^2, sum r_cent^2, max |r_dual|
__global__ void resid_kernel(int nc, double mu, double t, double step,
                             const int32_t* __restrict__ slot,
                             const double* __restrict__ gamma,
                             const double* __restrict__ dgamma,
                             const double* __restrict__ lam,
                             const double* __restrict__ dlam,
                             const double* __restrict__ u,
                             const double* __restrict__ w,
                             double* __restrict__ part) {
  __shared__ double sh[kT / 64];
  double rd2 = 0.0, rc2 = 0.0, rdm = 0.0;
  for (int i = blockIdx.x * kT + threadIdx.x; i < nc; i += gridDim.x * kT) {
    const int64_t q = 3 * (int64_t)slot[i];
    ContactState cs;
    eval(mu, gamma[q] + step * dgamma[q], gamma[q + 1] + step * dgamma[q + 1],
         gamma[q + 2] + step * dgamma[q + 2], lam[i] + step * dlam[i],
         lam[nc + i] + step * dlam[nc + i], cs);
    for (int c = 0; c < 3; ++c) {
      double r = u[q + c] + step * w[q + c] + cs.l1 * cs.gr[c];
      if (c == 0) r -= cs.l2;
      rd2 += r * r;
      rdm = fmax(rdm, fabs(r));
    }
    const double c1 = -cs.l1 * cs.f1 - 1.0 / t;
    const double c2 = -cs.l2 * cs.f2 - 1.0 / t;
    rc2 += c1 * c1 + c2 * c2;
  }
  const double a = block_reduce_sum(rd2, sh);
  const double b = block_reduce_sum(rc2, sh);
  const double m = block_reduce_max(rdm, sh);
  if (threadIdx.x == 0) {
    part[3 * blockIdx.x] = a;
    part[3 * blockIdx.x + 1] = b;
    part[3 * blockIdx.x + 2] = m;
  }
}

// S diagonal blocks = N's + H_i, and the Schur right-hand side
__global__ void newton_setup_kernel(int nc, double mu, double t,
                                    const int32_t* __restrict__ slot,
                                    const int32_t* __restrict__ diagpos,
                                    const double* __restrict__ gamma,
                                    const double* __restrict__ lam,
                                    const double* __restrict__ u,
                                    const double* __restrict__ valN,
                                    double* __restrict__ valS,
                                    double* __restrict__ rhs) {
  const int i = blockIdx.x * kT + threadIdx.x;
  if (i >= nc) return;
  const int s = slot[i];
  const int64_t q = 3 * (int64_t)s;
  ContactState cs;
  eval(mu, gamma[q], gamma[q + 1], gamma[q + 2], lam[i], lam[nc + i], cs);
  const double gn = cs.gn, g1 = cs.g1, g2 = cs.g2, t2 = g1 * g1 + g2 * g2;
  double hf[9];
  hf[0] = t2 / (mu * gn * gn * gn);
  hf[1] = hf[3] = -g1 / (mu * gn * gn);
  hf[2] = hf[6] = -g2 / (mu * gn * gn);
  hf[4] = hf[8] = 1.0 / (mu * gn);
  hf[5] = hf[7] = 0.0;
  const double coef = cs.l1 / (-cs.f1);
  const int64_t p = 9 * (int64_t)diagpos[s];
  for (int r = 0; r < 3; ++r)
    for (int c2 = 0; c2 < 3; ++c2) {
      double h = cs.l1 * hf[3 * r + c2] + coef * cs.gr[r] * cs.gr[c2];
      if (r == 0 && c2 == 0) h += cs.l2 / gn;
      valS[p + 3 * r + c2] = valN[p + 3 * r + c2] + h;
    }
  const double it = 1.0 / t;
  rhs[q] = -u[q] + it * (cs.gr[0] / cs.f1 + 1.0 / gn);
  rhs[q + 1] = -u[q + 1] + it * (cs.gr[1] / cs.f1);
  rhs[q + 2] = -u[q + 2] + it * (cs.gr[2] / cs.f1);
}

// Delta lambda and the partial min of -lambda / Delta lambda over Dl < 0
__global__ void dlam_kernel(int nc, double mu, double t,
                            const int32_t* __restrict__ slot,
                            const double* __restrict__ gamma,
                            const double* __restrict__ dgamma,
                            const double* __restrict__ lam,
                            double* __restrict__ dlam, double* __restrict__ part) {
  __shared__ double sh[kT / 64];
  double mn = INFINITY;
  for (int i = blockIdx.x * kT + threadIdx.x; i < nc; i += gridDim.x * kT) {
    const int64_t q = 3 * (int64_t)slot[i];
    ContactState cs;
    eval(mu, gamma[q], gamma[q + 1], gamma[q + 2], lam[i], lam[nc + i], cs);
    const double jd1 = cs.gr[0] * dgamma[q] + cs.gr[1] * dgamma[q + 1] +
                       cs.gr[2] * dgamma[q + 2];
    const double jd2 = -dgamma[q];
    const double rc1 = -cs.l1 * cs.f1 - 1.0 / t;
    const double rc2 = -cs.l2 * cs.f2 - 1.0 / t;
    const double d1 = (rc1 - cs.l1 * jd1) / cs.f1;
    const double d2 = (rc2 - cs.l2 * jd2) / cs.f2;
    dlam[i] = d1;
    dlam[nc + i] = d2;
    if (d1 < 0.0) mn = fmin(mn, -cs.l1 / d1);
    if (d2 < 0.0) mn = fmin(mn, -cs.l2 / d2);
  }
  const double m = block_reduce_min(mn, sh);
  if (threadIdx.x == 0) part[blockIdx.x] = m;
}

// partial count of constraints with f >= 0 at gamma + s dgamma
__global__ void infeasible_kernel(int nc, double mu, double step,
                                  const int32_t* __restrict__ slot,
                                  const double* __restrict__ gamma,
                                  const double* __restrict__ dgamma,
                                  double* __restrict__ part) {
  __shared__ double sh[kT / 64];
  double cnt = 0.0;
  for (int i = blockIdx.x * kT + threadIdx.x; i < nc; i += gridDim.x * kT) {
    const int64_t q = 3 * (int64_t)slot[i];
    ContactState cs;
    eval(mu, gamma[q] + step * dgamma[q], gamma[q + 1] + step * dgamma[q + 1],
         gamma[q + 2] + step * dgamma[q + 2], 0.0, 0.0, cs);
    // f1 is evaluated only where g_n > 0 (otherwise f2 >= 0 already fails)
    if (cs.f2 >= 0.0 || !(cs.f1 < 0.0)) cnt += 1.0;
  }
  const double s = block_reduce_sum(cnt, sh);
  if (threadIdx.x == 0) part[blockIdx.x] = s;
}

__global__ void update_kernel(int nc, double step, const int32_t* __restrict__ slot,
                              double* __restrict__ gamma,
                              const double* __restrict__ dgamma,
                              double* __restrict__ lam, const double* __restrict__ dlam) {
  const int i = blockIdx.x * kT + threadIdx.x;
  if (i >= nc) return;
  const int64_t q = 3 * (int64_t)slot[i];
  for (int c = 0; c < 3; ++c) gamma[q + c] += step * dgamma[q + c];
  lam[i] += step * dlam[i];
  lam[nc + i] += step * dlam[nc + i];
}

__global__ void add_vec_kernel(int64_t n, const double* __restrict__ a,
                               double* __restrict__ y) {
  const int64_t i = (int64_t)blockIdx.x * kT + threadIdx.x;
  if (i < n) y[i] += a[i];
}

int nblocks(int nc) { return std::max(1, std::min(kMaxBlk, div_up(nc, kT))); }

std::vector<double> read_part(Ctx& c, int count) {
  std::vector<double> h(count);
  QTP_HIP(hipMemcpyAsync(h.data(), c.pd.part.get(), sizeof(double) * count,
                         hipMemcpyDeviceToHost, c.stream));
  QTP_HIP(hipStreamSynchronize(c.stream));
  return h;
}

double now_ms() {
  using namespace std::chrono;
  return duration<double, std::milli>(steady_clock::now().time_since_epoch()).count();
}

}  // namespace

// start: 0 cold (Sec. 3.3), 1 previous step's impulses, 2 learned
static int pdip_run(Ctx& c, qtp_step_stats* st, int start) {
  QTP_REQUIRE(c.qp.valid && !c.qp.stale, QTP_E_STATE, "assemble before the PDIP solve");
  const hipStream_t s = c.stream;
  Scene& sc = c.scene;
  Qp& qp = c.qp;
  Pdip& pd = c.pd;
  const int nc = c.ct.nc;
  const int d = sc.log2n;
  const int64_t n = (int64_t)1 << d;
  const double mu = sc.mu;
  const double mu_pd = 10.0, alpha = 0.01, beta = 0.5;
  const int max_backtrack = 80;
  // Newton matrix S on the QP pattern (values start as N)
  c.log2n = d;
  c.n = n;
  c.nslots = (int)(n / 3);
  c.nnzb = qp.nnzb;
  c.rp.ensure(sizeof(int32_t) * (c.nslots + 1));
  c.col.ensure(sizeof(int32_t) * qp.nnzb);
  c.val.ensure(sizeof(double) * 9 * qp.nnzb);
  QTP_HIP(hipMemcpyAsync(c.rp.get(), qp.rp.get(), sizeof(int32_t) * (c.nslots + 1),
                         hipMemcpyDeviceToDevice, s));
  QTP_HIP(hipMemcpyAsync(c.col.get(), qp.col.get(), sizeof(int32_t) * qp.nnzb,
                         hipMemcpyDeviceToDevice, s));
  QTP_HIP(hipMemcpyAsync(c.val.get(), qp.valN.get(), sizeof(double) * 9 * qp.nnzb,
                         hipMemcpyDeviceToDevice, s));
  c.have_matrix = true;
  c.have_precond = false;
  c.pat.valid = false;
  // iterate
  const int ncap = std::max(nc, 1);
  pd.gamma.ensure(sizeof(double) * n);
  pd.dgamma.ensure(sizeof(double) * n);
  pd.u.ensure(sizeof(double) * n);
  pd.wv.ensure(sizeof(double) * n);
  pd.rhs.ensure(sizeof(double) * n);
  pd.lam.ensure(sizeof(double) * 2 * ncap);
  pd.dlam.ensure(sizeof(double) * 2 * ncap);
  pd.part.ensure(sizeof(double) * 3 * kMaxBlk);
  QTP_HIP(hipMemsetAsync(pd.gamma.get(), 0, sizeof(double) * n, s));
  QTP_HIP(hipMemsetAsync(pd.dgamma.get(), 0, sizeof(double) * n, s));
  QTP_HIP(hipMemsetAsync(pd.wv.get(), 0, sizeof(double) * n, s));
  QTP_HIP(hipMemsetAsync(pd.rhs.get(), 0, sizeof(double) * n, s));
  QTP_HIP(hipMemsetAsync(pd.dlam.get(), 0, sizeof(double) * 2 * ncap, s));
  const int32_t* slot = c.ct.slot.as<int32_t>();
  double* gamma = pd.gamma.as<double>();
  double* dgamma = pd.dgamma.as<double>();
  double* lam = pd.lam.as<double>();
  double* dlam = pd.dlam.as<double>();
  double* u = pd.u.as<double>();
  double* wv = pd.wv.as<double>();
  double* part = pd.part.as<double>();
  const int nb = nblocks(nc);
  st->n_contacts = nc;
  st->pdip_iterations = 0;
  st->converged = 0;
  st->fgmres_iterations = 0;
  st->max_fgmres = 0;
  st->ms_precond = 0.0;
  st->ms_solve = 0.0;
  st->qtt_used = 0;
  st->qtt_trial_iterations = 0;
  st->plain_trial_iterations = 0;
  c.auto_qtt = false;
  pd.log.clear();
  std::vector<double> solve_ms;
  const double t_begin = now_ms();
  if (nc == 0) {
    pd.have_gamma = true;
    st->converged = 1;
    st->gap = 0.0;
    st->dual_inf = 0.0;
    st->ms_pdip = 0.0;
    return QTP_OK;
  }
  if (start == 2) {
    mlp_warm_start(c, c.cfg.warm_t0, gamma, lam);
  } else if (start == 1) {
    prev_start_kernel<<<div_up(nc, kT), kT, 0, s>>>(
        nc, mu, c.cfg.warm_t0, c.cfg.warm_floor, c.cfg.warm_start == 3 ? 1 : 0, slot,
        c.ct.old_slot.as<int32_t>(), pd.gamma_prev.as<double>(), gamma, lam);
    QTP_CHECK_LAUNCH();
  } else {
    init_kernel<<<div_up(nc, kT), kT, 0, s>>>(nc, mu, slot, gamma, lam);
    QTP_CHECK_LAUNCH();
  }
  const double m = 2.0 * nc;
  int it = 0;
  double gap = 0.0, rdinf = 0.0;
  int rc = QTP_NOT_CONVERGED;
  for (;;) {
    gap_kernel<<<nb, kT, 0, s>>>(nc, mu, slot, gamma, lam, part);
    QTP_CHECK_LAUNCH();
    gap = 0.0;
    for (double v : read_part(c, nb)) gap += v;
    // mu m / eta, capped at the t whose central point meets the gap tolerance
    const double t = std::min(mu_pd * m / gap, mu_pd / c.cfg.pdip_gap_tol);
    // u = N gamma + r
    bsr_spmv(s, c.nslots, n, qp.rp.as<int32_t>(), qp.col.as<int32_t>(),
             qp.valN.as<double>(), gamma, u);
    add_vec_kernel<<<div_up(n, kT), kT, 0, s>>>(n, qp.r.as<double>(), u);
    QTP_CHECK_LAUNCH();
    resid_kernel<<<nb, kT, 0, s>>>(nc, mu, t, 0.0, slot, gamma, dgamma, lam, dlam, u,
                                   wv, part);
    QTP_CHECK_LAUNCH();
    double rd2 = 0.0, rc2 = 0.0;
    rdinf = 0.0;
    {
      const auto h = read_part(c, 3 * nb);
      for (int b = 0; b < nb; ++b) {
        rd2 += h[3 * b];
        rc2 += h[3 * b + 1];
        rdinf = std::max(rdinf, h[3 * b + 2]);
      }
    }
    if (!std::isfinite(gap) || !std::isfinite(rd2))
      throw Error(QTP_E_NUMERIC, "PDIP: non-finite iterate");
    if (gap / m <= c.cfg.pdip_gap_tol && rdinf <= c.cfg.pdip_dual_tol) {
      rc = QTP_OK;
      break;
    }
    if (it >= (start != 0 ? std::min(c.cfg.warm_maxit, c.cfg.pdip_maxit)
                          : c.cfg.pdip_maxit))
      break;
    // Newton system
    newton_setup_kernel<<<div_up(nc, kT), kT, 0, s>>>(
        nc, mu, t, slot, qp.diagpos.as<int32_t>(), gamma, lam, u,
        qp.valN.as<double>(), c.val.as<double>(), pd.rhs.as<double>());
    QTP_CHECK_LAUNCH();
    const double pre0 = st->ms_precond;
    double t0 = now_ms();
    precond_factor(c);
    c.have_precond = true;
    st->ms_precond += now_ms() - t0;
    const int mode = c.cfg.qtt_mode;
    qtp_solve_stats ss{};
    int src;
    double sms;
    const bool trial = mode == 2 && it == 0 && c.auto_skip == 0;
    if (mode == 2 && it == 0 && !trial) --c.auto_skip;
    if (trial) {
      // auto: solve the first Newton step with X = I and with the QTT inverse,
      // keep the faster for the rest of the time step
      c.use_qtt = false;
      t0 = now_ms();
      src = newton_solve(c, pd.rhs.as<double>(), dgamma, &ss);
      const double ms_i = now_ms() - t0;
      if (src != QTP_OK) throw Error(QTP_E_NUMERIC, "Newton-step solve did not converge");
      st->plain_trial_iterations = ss.iterations;
      t0 = now_ms();
      build_inverse(c, c.have_inverse ? 1 : 0);
      c.use_qtt = true;
      const double ms_b = now_ms() - t0;
      st->ms_precond += ms_b;
      pd.dtrial.ensure(sizeof(double) * n);
      qtp_solve_stats s2{};
      t0 = now_ms();
      // the QTT trial may use twice the block-Jacobi trial's iterations (plus
      // 10): beyond that it has lost, so stop paying for it
      int src2;
      {
        struct Restore {
          int& v;
          int old;
          ~Restore() { v = old; }
        } restore{c.cfg.fgmres_maxit, c.cfg.fgmres_maxit};
        c.cfg.fgmres_maxit = std::min(c.cfg.fgmres_maxit, 2 * ss.iterations + 10);
        src2 = newton_solve(c, pd.rhs.as<double>(), pd.dtrial.as<double>(), &s2);
      }
      const double ms_x = now_ms() - t0;
      st->qtt_trial_iterations = s2.iterations;
      st->ms_solve += ms_i + ms_x;
      st->fgmres_iterations += ss.iterations + s2.iterations;
      c.auto_qtt = src2 == QTP_OK && ms_b + ms_x < ms_i;
      c.use_qtt = c.auto_qtt;
      // a lost trial is repeated after 1, 3, 7, ... skipped time steps (at
      // most 63), a won one at the next step
      if (c.auto_qtt) {
        c.auto_losses = 0;
      } else {
        c.auto_losses = std::min(c.auto_losses + 1, 6);
        c.auto_skip = (1 << c.auto_losses) - 1;
      }
      if (c.auto_qtt) {
        QTP_HIP(hipMemcpyAsync(dgamma, pd.dtrial.get(), sizeof(double) * n,
                               hipMemcpyDeviceToDevice, s));
        ss = s2;
        sms = ms_x;
        st->qtt_used += 1;
      } else {
        sms = ms_i;
      }
    } else {
      const bool q = mode == 1 || (mode == 2 && c.auto_qtt);
      if (q) {
        t0 = now_ms();
        build_inverse(c, (it > 0 || c.have_inverse) ? 1 : 0);
        st->ms_precond += now_ms() - t0;
        st->qtt_used += 1;
      }
      c.use_qtt = q;
      t0 = now_ms();
      src = newton_solve(c, pd.rhs.as<double>(), dgamma, &ss);
      sms = now_ms() - t0;
      st->ms_solve += sms;
      st->fgmres_iterations += ss.iterations;
      if (src != QTP_OK) throw Error(QTP_E_NUMERIC, "Newton-step solve did not converge");
    }
    solve_ms.push_back(sms);
    st->max_fgmres = std::max(st->max_fgmres, ss.iterations);
    pd.log.push_back(qtp_newton_record{it, ss.iterations, c.use_qtt ? 1 : 0, sms,
                                       st->ms_precond - pre0, ss.rel_residual});
    // Delta lambda and the step bound
    dlam_kernel<<<nb, kT, 0, s>>>(nc, mu, t, slot, gamma, dgamma, lam, dlam, part);
    QTP_CHECK_LAUNCH();
    double smax = 1.0;
    for (double v : read_part(c, nb)) smax = std::min(smax, v);
    double step = 0.99 * smax;
    int nbt = 0;
    for (;;) {
      infeasible_kernel<<<nb, kT, 0, s>>>(nc, mu, step, slot, gamma, dgamma, part);
      QTP_CHECK_LAUNCH();
      double bad = 0.0;
      for (double v : read_part(c, nb)) bad += v;
      if (bad == 0.0) break;
      step *= beta;
      if (++nbt > max_backtrack)
        throw Error(QTP_E_NUMERIC, "line search: no strictly feasible step");
    }
    const double norm0 = std::sqrt(rd2 + rc2);
    bsr_spmv(s, c.nslots, n, qp.rp.as<int32_t>(), qp.col.as<int32_t>(),
             qp.valN.as<double>(), dgamma, wv);
    for (;;) {
      resid_kernel<<<nb, kT, 0, s>>>(nc, mu, t, step, slot, gamma, dgamma, lam, dlam,
                                     u, wv, part);
      QTP_CHECK_LAUNCH();
      double a2 = 0.0, b2 = 0.0;
      const auto h = read_part(c, 3 * nb);
      for (int b = 0; b < nb; ++b) {
        a2 += h[3 * b];
        b2 += h[3 * b + 1];
      }
      if (std::sqrt(a2 + b2) <= (1.0 - alpha * step) * norm0) break;
      step *= beta;
      if (++nbt > max_backtrack) break;
    }
    update_kernel<<<div_up(nc, kT), kT, 0, s>>>(nc, step, slot, gamma, dgamma, lam, dlam);
    QTP_CHECK_LAUNCH();
    ++it;
  }
  QTP_HIP(hipStreamSynchronize(s));
  pd.have_gamma = true;
  st->pdip_iterations = it;
  st->converged = rc == QTP_OK;
  st->gap = gap / m;
  st->dual_inf = rdinf;
  st->ms_pdip = now_ms() - t_begin;
  if (!solve_ms.empty()) {
    std::sort(solve_ms.begin(), solve_ms.end());
    st->newton_solve_ms_median = solve_ms[solve_ms.size() / 2];
  } else {
    st->newton_solve_ms_median = 0.0;
  }
  return rc;
}

}  // namespace qtp

namespace qtp {
namespace {
__global__ void gather_impulses_kernel(int nc, double gbar,
                                       const int32_t* __restrict__ slot,
                                       const double* __restrict__ gamma,
                                       double* __restrict__ out) {
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i >= nc) return;
  const int64_t q = 3 * (int64_t)slot[i];
  for (int c = 0; c < 3; ++c) out[3 * (int64_t)i + c] = gbar * gamma[q + c];
}
}  // namespace

// The learned start when configured and trained, with the cold start of
// Sec. 3.3 as the fallback when that run fails or does not converge.
int pdip_solve(Ctx& c, qtp_step_stats* st) {
  st->warm_started = 0;
  st->warm_fallback = 0;
  st->warm_iterations = 0;
  st->persistent_contacts = c.ct.n_persistent;
  st->slots_rebuilt = c.ct.rebuilt ? 1 : 0;
  Pdip& pd = c.pd;
  int start = 0;
  if (c.cfg.warm_start == 2 && c.mlp.have_params && c.ct.nc > 0) start = 2;
  if ((c.cfg.warm_start == 1 || c.cfg.warm_start == 3) && pd.have_prev &&
      c.ct.n_persistent > 0 &&
      pd.prev_n == (int64_t)1 << c.scene.log2n)
    start = 1;
  // after k consecutive failed warm starts the next 2^k - 1 steps start cold
  // (k <= 6): a start that has stopped helping is not paid for every step
  if (start != 0 && pd.warm_skip > 0) {
    --pd.warm_skip;
    start = 0;
  }
  int rc = QTP_NOT_CONVERGED;
  if (start != 0) {
    st->warm_started = start;
    try {
      rc = pdip_run(c, st, start);
    } catch (const Error& e) {
      if (e.status != QTP_E_NUMERIC) throw;
    }
    if (rc == QTP_OK) {
      pd.warm_losses = 0;
    } else {
      pd.warm_losses = std::min(pd.warm_losses + 1, 6);
      pd.warm_skip = (1 << pd.warm_losses) - 1;
      const int wit = st->pdip_iterations;
      const double wpre = st->ms_precond, wsol = st->ms_solve, wpd = st->ms_pdip;
      const int wfg = st->fgmres_iterations;
      rc = pdip_run(c, st, 0);
      st->warm_fallback = 1;
      st->warm_iterations = wit;
      st->ms_precond += wpre;
      st->ms_solve += wsol;
      st->ms_pdip += wpd;  // the failed warm run is part of the cost
      st->fgmres_iterations += wfg;
    }
  } else {
    rc = pdip_run(c, st, 0);
  }
  // keep the solution on the slot layout for a start from it next step
  if (rc == QTP_OK && c.ct.nc > 0) {
    const int64_t n = (int64_t)1 << c.scene.log2n;
    pd.gamma_prev.ensure(sizeof(double) * n);
    QTP_HIP(hipMemcpyAsync(pd.gamma_prev.get(), pd.gamma.get(), sizeof(double) * n,
                           hipMemcpyDeviceToDevice, c.stream));
    pd.have_prev = true;
    pd.prev_n = n;
  } else {
    pd.have_prev = false;
  }
  return rc;
}

void gather_impulses(Ctx& c, double* out) {
  QTP_REQUIRE(c.pd.have_gamma, QTP_E_STATE, "no PDIP solution");
  const int nc = c.ct.nc;
  if (nc == 0) return;
  gather_impulses_kernel<<<div_up(nc, 256), 256, 0, c.stream>>>(
      nc, c.qp.gbar, c.ct.slot.as<int32_t>(), c.pd.gamma.as<double>(), out);
  QTP_CHECK_LAUNCH();
  QTP_HIP(hipStreamSynchronize(c.stream));
}

}  // namespace qtp
