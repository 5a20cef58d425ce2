// C-ABI of the qtp library: argument checks, context management, and the
// translation of internal errors into qtp_status codes.  Nothing here
// computes; every step runs in the kernels of the other files.
#include <chrono>
#include <cmath>
#include <cstring>

#include "context.h"

using qtp::Ctx;
using qtp::Error;

struct qtp_ctx_s {
  Ctx c;
};

namespace {

thread_local std::string g_create_error;

template <class F>
qtp_status guarded(qtp_ctx ctx, F&& f) {
  if (!ctx) return QTP_E_ARG;
  try {
    ctx->c.err.clear();
    return (qtp_status)f(ctx->c);
  } catch (const Error& e) {
    ctx->c.err = e.what();
    return (qtp_status)e.status;
  } catch (const std::bad_alloc&) {
    ctx->c.err = "host allocation failed";
    return QTP_E_OOM;
  } catch (const std::exception& e) {
    ctx->c.err = e.what();
    return QTP_E_HIP;
  }
}

bool valid_d(int d) { return d >= 2 && d <= 30; }

}  // namespace

int64_t qtp::Qtt::total() const {
  int64_t t = 0;
  for (int k = 0; k < d; ++k) t += (int64_t)ranks[k] * 4 * ranks[k + 1];
  return t;
}

qtp::KTimer& qtp::Ctx::timer(const char* name) {
  for (auto& kv : timers)
    if (kv.first == name) return kv.second;
  timers.emplace_back(name, KTimer{});
  return timers.back().second;
}

void qtp::Ctx::flush_timers() {
  for (auto& kv : timers) {
    for (auto& e : kv.second.pending) {
      QTP_HIP(hipEventSynchronize(e.second));
      float ms = 0.f;
      QTP_HIP(hipEventElapsedTime(&ms, e.first, e.second));
      kv.second.ms += ms;
      kv.second.count += 1;
      event_pool.push_back(e.first);
      event_pool.push_back(e.second);
    }
    kv.second.pending.clear();
  }
}

void qtp::Ctx::check_cfg() {
  QTP_REQUIRE(cfg.precision >= 0 && cfg.precision <= 2, QTP_E_ARG, "bad precision");
  QTP_REQUIRE(cfg.qtt_rmax >= 1 && cfg.qtt_rmax <= 64, QTP_E_ARG, "qtt_rmax out of [1,64]");
  QTP_REQUIRE(cfg.qtt_rmax_s >= 1 && cfg.qtt_rmax_s <= 64, QTP_E_ARG, "qtt_rmax_s out of [1,64]");
  QTP_REQUIRE(cfg.qtt_eps > 0.0 && cfg.qtt_eps < 1.0, QTP_E_ARG, "qtt_eps out of (0,1)");
  QTP_REQUIRE(cfg.fgmres_restart >= 1 && cfg.fgmres_restart <= qtp::kArnMaxRestart,
              QTP_E_ARG, "fgmres_restart out of [1,32]");
  QTP_REQUIRE(cfg.fgmres_maxit >= 1, QTP_E_ARG, "fgmres_maxit < 1");
  QTP_REQUIRE(cfg.solve_tol > 0.0, QTP_E_ARG, "solve_tol <= 0");
  QTP_REQUIRE(cfg.solve_mode == 0 || cfg.solve_mode == 1, QTP_E_ARG, "bad solve_mode");
  QTP_REQUIRE(cfg.ns_iters >= 0 && cfg.ns_iters_hot >= 0, QTP_E_ARG, "ns_iters < 0");
  QTP_REQUIRE(cfg.qtt_mode >= 0 && cfg.qtt_mode <= 2, QTP_E_ARG, "qtt_mode out of [0,2]");
  QTP_REQUIRE(cfg.warm_start >= 0 && cfg.warm_start <= 3, QTP_E_ARG,
              "warm_start must be 0, 1, 2 or 3");
  QTP_REQUIRE(cfg.slot_mode == 0 || cfg.slot_mode == 1, QTP_E_ARG,
              "slot_mode must be 0 or 1");
  QTP_REQUIRE(cfg.warm_maxit >= 1, QTP_E_ARG, "warm_maxit must be >= 1");
  QTP_REQUIRE(cfg.warm_floor >= 0.0 && std::isfinite(cfg.warm_floor), QTP_E_ARG,
              "warm_floor must be finite and >= 0");
}

extern "C" {

void qtp_config_default(qtp_config* cfg) {
  if (!cfg) return;
  std::memset(cfg, 0, sizeof(*cfg));
  cfg->precision = QTP_PREC_F64;
  cfg->qtt_eps = 1e-2;
  cfg->qtt_rmax = 32;
  cfg->qtt_rmax_s = 16;
  cfg->ns_iters = 8;
  cfg->ns_iters_hot = 2;
  cfg->solve_mode = 1;
  cfg->solve_tol = 1e-8;
  cfg->fgmres_restart = 30;
  cfg->fgmres_maxit = 1000;
  cfg->pdip_gap_tol = 1e-8;
  cfg->pdip_dual_tol = 1e-4;
  cfg->pdip_maxit = 100;
  cfg->warm_start = 0;
  cfg->seed = 0;
  cfg->warm_t0 = 100.0;
  cfg->warm_floor = 0.0;
  cfg->slot_mode = 0;
  cfg->warm_maxit = 100;
  cfg->qtt_mode = 2;
}

qtp_status qtp_create(const qtp_config* cfg, void* hip_stream, qtp_ctx* out) {
  if (!out) return QTP_E_ARG;
  *out = nullptr;
  qtp_ctx h = nullptr;
  try {
    h = new qtp_ctx_s();
  } catch (...) {
    return QTP_E_OOM;
  }
  if (cfg) h->c.cfg = *cfg;
  else qtp_config_default(&h->c.cfg);
  h->c.stream = static_cast<hipStream_t>(hip_stream);
  qtp_status st = guarded(h, [](Ctx& c) {
    c.check_cfg();
    return QTP_OK;
  });
  if (st != QTP_OK) {
    g_create_error = h->c.err;
    delete h;
    return st;
  }
  *out = h;
  return QTP_OK;
}

void qtp_destroy(qtp_ctx ctx) {
  if (!ctx) return;
  if (ctx->c.stream) (void)hipStreamSynchronize(ctx->c.stream);
  else (void)hipDeviceSynchronize();
  try {
    ctx->c.flush_timers();
  } catch (...) {
  }
  delete ctx;
}

const char* qtp_last_error(qtp_ctx ctx) {
  if (!ctx) return g_create_error.c_str();
  return ctx->c.err.c_str();
}

qtp_status qtp_set_config(qtp_ctx ctx, const qtp_config* cfg) {
  if (!cfg) return QTP_E_ARG;
  return guarded(ctx, [&](Ctx& c) {
    qtp_config old = c.cfg;
    c.cfg = *cfg;
    try {
      c.check_cfg();
    } catch (...) {
      c.cfg = old;
      throw;
    }
    c.X.lp_prec = 0;  // reduced-precision copies follow the new precision
    // a new configuration starts the trial and warm-start back-offs afresh
    c.auto_losses = c.auto_skip = 0;
    c.pd.warm_losses = c.pd.warm_skip = 0;
    return QTP_OK;
  });
}

qtp_status qtp_bsr_spmv(qtp_ctx ctx, int log2n, const int32_t* row_ptr,
                        const int32_t* col, const double* val, const double* x,
                        double* y) {
  return guarded(ctx, [&](Ctx& c) {
    QTP_REQUIRE(valid_d(log2n), QTP_E_ARG, "log2n out of [2,30]");
    QTP_REQUIRE(row_ptr && col && val && x && y, QTP_E_ARG, "null pointer");
    QTP_REQUIRE(x != y, QTP_E_ARG, "x and y alias");
    const int64_t n = (int64_t)1 << log2n;
    qtp::bsr_spmv(c.stream, (int)(n / 3), n, row_ptr, col, val, x, y);
    QTP_HIP(hipStreamSynchronize(c.stream));
    return QTP_OK;
  });
}

qtp_status qtp_qtt_apply(qtp_ctx ctx, int d, const int32_t* ranks,
                         const void* cores, int precision, const double* x,
                         double* y) {
  return guarded(ctx, [&](Ctx& c) {
    QTP_REQUIRE(d >= 1 && d <= 30, QTP_E_ARG, "d out of [1,30]");
    QTP_REQUIRE(ranks && cores && x && y, QTP_E_ARG, "null pointer");
    QTP_REQUIRE(x != y, QTP_E_ARG, "x and y alias");
    QTP_REQUIRE(precision >= 0 && precision <= 2, QTP_E_ARG, "bad precision");
    QTP_REQUIRE(ranks[0] == 1 && ranks[d] == 1, QTP_E_ARG, "r_0 and r_d must be 1");
    for (int k = 0; k <= d; ++k)
      QTP_REQUIRE(ranks[k] >= 1 && ranks[k] <= 256, QTP_E_ARG, "rank out of [1,256]");
    c.qtt_work.ensure(qtp::qtt_apply_workspace(d, ranks, precision));
    qtp::qtt_apply(c.stream, d, ranks, cores, precision, x, y, c.qtt_work.get());
    QTP_HIP(hipStreamSynchronize(c.stream));
    return QTP_OK;
  });
}

qtp_status qtp_set_newton_matrix(qtp_ctx ctx, int log2n, const int32_t* row_ptr,
                                 const int32_t* col, const double* val) {
  return guarded(ctx, [&](Ctx& c) {
    QTP_REQUIRE(valid_d(log2n), QTP_E_ARG, "log2n out of [2,30]");
    QTP_REQUIRE(row_ptr && col && val, QTP_E_ARG, "null pointer");
    const int64_t n = (int64_t)1 << log2n;
    const int ns = (int)(n / 3);
    int32_t h_nnzb = 0;
    QTP_HIP(hipMemcpyAsync(&h_nnzb, row_ptr + ns, sizeof(int32_t),
                           hipMemcpyDeviceToHost, c.stream));
    QTP_HIP(hipStreamSynchronize(c.stream));
    QTP_REQUIRE(h_nnzb >= ns, QTP_E_ARG, "row_ptr[S] smaller than the slot count");
    c.log2n = log2n;
    c.n = n;
    c.nslots = ns;
    c.nnzb = h_nnzb;
    c.rp.ensure(sizeof(int32_t) * (ns + 1));
    c.col.ensure(sizeof(int32_t) * (size_t)h_nnzb);
    c.val.ensure(sizeof(double) * 9 * (size_t)h_nnzb);
    QTP_HIP(hipMemcpyAsync(c.rp.get(), row_ptr, sizeof(int32_t) * (ns + 1),
                           hipMemcpyDeviceToDevice, c.stream));
    QTP_HIP(hipMemcpyAsync(c.col.get(), col, sizeof(int32_t) * (size_t)h_nnzb,
                           hipMemcpyDeviceToDevice, c.stream));
    QTP_HIP(hipMemcpyAsync(c.val.get(), val, sizeof(double) * 9 * (size_t)h_nnzb,
                           hipMemcpyDeviceToDevice, c.stream));
    QTP_HIP(hipStreamSynchronize(c.stream));
    c.have_matrix = true;
    c.have_precond = false;
    c.pat.valid = false;
    return QTP_OK;
  });
}

qtp_status qtp_precond_build(qtp_ctx ctx, int hot) {
  return guarded(ctx, [&](Ctx& c) {
    hipEvent_t e0, e1;
    QTP_HIP(hipEventCreate(&e0));
    QTP_HIP(hipEventCreate(&e1));
    QTP_HIP(hipEventRecord(e0, c.stream));
    qtp::precond_factor(c);
    c.have_precond = true;
    qtp::build_inverse(c, hot);
    c.use_qtt = true;
    QTP_HIP(hipEventRecord(e1, c.stream));
    QTP_HIP(hipEventSynchronize(e1));
    float ms = 0.f;
    QTP_HIP(hipEventElapsedTime(&ms, e0, e1));
    c.build_ms = ms;
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    return QTP_OK;
  });
}

qtp_status qtp_get_precond_stats(qtp_ctx ctx, qtp_precond_stats* out) {
  return guarded(ctx, [&](Ctx& c) {
    QTP_REQUIRE(out, QTP_E_ARG, "null pointer");
    QTP_REQUIRE(c.have_inverse, QTP_E_STATE, "no preconditioner built");
    out->ns_iterations = c.ns_done;
    out->probe_residual = c.probe_residual;
    int ms = 0, mx = 0;
    for (int r : c.A.ranks) ms = r > ms ? r : ms;
    for (int r : c.X.ranks) mx = r > mx ? r : mx;
    out->max_rank_s = ms;
    out->max_rank_x = mx;
    out->ms = c.build_ms;
    return QTP_OK;
  });
}

qtp_status qtp_precond_load_qtt(qtp_ctx ctx, int d, const int32_t* ranks,
                                const double* cores) {
  return guarded(ctx, [&](Ctx& c) {
    QTP_REQUIRE(c.have_matrix, QTP_E_STATE, "no Newton matrix loaded");
    QTP_REQUIRE(d == c.log2n, QTP_E_ARG, "QTT size does not match the matrix");
    QTP_REQUIRE(ranks && cores, QTP_E_ARG, "null pointer");
    QTP_REQUIRE(ranks[0] == 1 && ranks[d] == 1, QTP_E_ARG, "r_0 and r_d must be 1");
    for (int k = 0; k <= d; ++k)
      QTP_REQUIRE(ranks[k] >= 1 && ranks[k] <= 256, QTP_E_ARG, "rank out of [1,256]");
    qtp::precond_factor(c);
    c.have_precond = true;
    c.X.d = d;
    c.X.ranks.assign(ranks, ranks + d + 1);
    const int64_t tot = c.X.total();
    c.X.cores.ensure(sizeof(double) * tot);
    QTP_HIP(hipMemcpyAsync(c.X.cores.get(), cores, sizeof(double) * tot,
                           hipMemcpyDeviceToDevice, c.stream));
    c.X.lp_prec = 0;
    c.have_inverse = true;
    c.use_qtt = true;
    QTP_HIP(hipStreamSynchronize(c.stream));
    return QTP_OK;
  });
}

qtp_status qtp_newton_solve(qtp_ctx ctx, const double* rhs, double* x,
                            qtp_solve_stats* stats) {
  return guarded(ctx, [&](Ctx& c) {
    QTP_REQUIRE(rhs && x, QTP_E_ARG, "null pointer");
    QTP_REQUIRE(rhs != x, QTP_E_ARG, "rhs and x alias");
    qtp_solve_stats local{};
    qtp_solve_stats* st = stats ? stats : &local;
    return qtp::newton_solve(c, rhs, x, st);
  });
}

qtp_status qtp_precond_apply(qtp_ctx ctx, const double* v, double* z) {
  return guarded(ctx, [&](Ctx& c) {
    QTP_REQUIRE(v && z && v != z, QTP_E_ARG, "bad vector pointers");
    qtp::precond_apply(c, v, z);
    QTP_HIP(hipStreamSynchronize(c.stream));
    return QTP_OK;
  });
}

qtp_status qtp_set_bodies(qtp_ctx ctx, int M, const double* x, const double* v,
                          const double* w, const double* radius,
                          const double* mass) {
  return guarded(ctx, [&](Ctx& c) {
    QTP_REQUIRE(M >= 1 && M < (1 << 30), QTP_E_ARG, "M out of range");
    QTP_REQUIRE(x && v && w && radius && mass, QTP_E_ARG, "null pointer");
    qtp::Scene& sc = c.scene;
    sc.M = M;
    const size_t b3 = sizeof(double) * 3 * (size_t)M, b1 = sizeof(double) * M;
    sc.x.ensure(b3);
    sc.v.ensure(b3);
    sc.w.ensure(b3);
    sc.radius.ensure(b1);
    sc.mass.ensure(b1);
    QTP_HIP(hipMemcpyAsync(sc.x.get(), x, b3, hipMemcpyDeviceToDevice, c.stream));
    QTP_HIP(hipMemcpyAsync(sc.v.get(), v, b3, hipMemcpyDeviceToDevice, c.stream));
    QTP_HIP(hipMemcpyAsync(sc.w.get(), w, b3, hipMemcpyDeviceToDevice, c.stream));
    QTP_HIP(hipMemcpyAsync(sc.radius.get(), radius, b1, hipMemcpyDeviceToDevice, c.stream));
    QTP_HIP(hipMemcpyAsync(sc.mass.get(), mass, b1, hipMemcpyDeviceToDevice, c.stream));
    QTP_HIP(hipStreamSynchronize(c.stream));
    c.ct.valid = false;
    c.qp.valid = false;
    return QTP_OK;
  });
}

qtp_status qtp_set_walls(qtp_ctx ctx, int nw, const double* planes_host) {
  return guarded(ctx, [&](Ctx& c) {
    QTP_REQUIRE(nw >= 0 && nw <= 1024, QTP_E_ARG, "nw out of [0,1024]");
    QTP_REQUIRE(nw == 0 || planes_host, QTP_E_ARG, "null planes");
    c.scene.nw = nw;
    c.scene.planes.ensure(sizeof(double) * 4 * (size_t)(nw > 0 ? nw : 1));
    if (nw > 0)
      QTP_HIP(hipMemcpyAsync(c.scene.planes.get(), planes_host, sizeof(double) * 4 * nw,
                             hipMemcpyHostToDevice, c.stream));
    QTP_HIP(hipStreamSynchronize(c.stream));
    c.ct.valid = false;
    return QTP_OK;
  });
}

qtp_status qtp_set_params(qtp_ctx ctx, double mu, double h, double delta,
                          const double* gravity_host, int log2n) {
  return guarded(ctx, [&](Ctx& c) {
    QTP_REQUIRE(mu > 0.0 && h > 0.0 && delta >= 0.0, QTP_E_ARG, "mu, h > 0, delta >= 0");
    QTP_REQUIRE(gravity_host, QTP_E_ARG, "null gravity");
    QTP_REQUIRE(valid_d(log2n) && log2n <= 26, QTP_E_ARG, "log2n out of [2,26]");
    qtp::Scene& sc = c.scene;
    sc.mu = mu;
    sc.h = h;
    sc.delta = delta;
    for (int k = 0; k < 3; ++k) sc.g[k] = gravity_host[k];
    sc.log2n = log2n;
    sc.have_params = true;
    c.ct.valid = false;
    return QTP_OK;
  });
}

qtp_status qtp_detect(qtp_ctx ctx, int* n_contacts) {
  return guarded(ctx, [&](Ctx& c) {
    QTP_REQUIRE(c.scene.have_params && c.scene.M > 0, QTP_E_STATE,
                "set bodies and params first");
    const int nc = qtp::detect_contacts(c);
    if (n_contacts) *n_contacts = nc;
    return QTP_OK;
  });
}

qtp_status qtp_get_contacts(qtp_ctx ctx, int32_t* a, int32_t* b, double* phi,
                            double* frame, uint64_t* key, int32_t* slot) {
  return guarded(ctx, [&](Ctx& c) {
    QTP_REQUIRE(c.ct.valid, QTP_E_STATE, "no contacts detected");
    const int nc = c.ct.nc;
    auto cp = [&](void* dst, const qtp::DevBuf& src, size_t es) {
      if (dst && nc > 0)
        QTP_HIP(hipMemcpyAsync(dst, src.get(), es * nc, hipMemcpyDeviceToDevice, c.stream));
    };
    cp(a, c.ct.a, sizeof(int32_t));
    cp(b, c.ct.b, sizeof(int32_t));
    cp(phi, c.ct.phi, sizeof(double));
    cp(frame, c.ct.frame, 9 * sizeof(double));
    cp(key, c.ct.key, sizeof(uint64_t));
    cp(slot, c.ct.slot, sizeof(int32_t));
    QTP_HIP(hipStreamSynchronize(c.stream));
    return QTP_OK;
  });
}

qtp_status qtp_assemble(qtp_ctx ctx) {
  return guarded(ctx, [&](Ctx& c) {
    qtp::assemble_qp(c);
    return QTP_OK;
  });
}

qtp_status qtp_get_qp(qtp_ctx ctx, int32_t* row_ptr, int32_t* col, double* valN,
                      double* r, int64_t* nnzb) {
  return guarded(ctx, [&](Ctx& c) {
    QTP_REQUIRE(c.qp.valid, QTP_E_STATE, "no assembled QP");
    const int64_t n = (int64_t)1 << c.scene.log2n;
    const int ns = (int)(n / 3);
    if (nnzb) *nnzb = c.qp.nnzb;
    if (row_ptr)
      QTP_HIP(hipMemcpyAsync(row_ptr, c.qp.rp.get(), sizeof(int32_t) * (ns + 1),
                             hipMemcpyDeviceToDevice, c.stream));
    if (col)
      QTP_HIP(hipMemcpyAsync(col, c.qp.col.get(), sizeof(int32_t) * c.qp.nnzb,
                             hipMemcpyDeviceToDevice, c.stream));
    if (valN)
      QTP_HIP(hipMemcpyAsync(valN, c.qp.valN.get(), sizeof(double) * 9 * c.qp.nnzb,
                             hipMemcpyDeviceToDevice, c.stream));
    if (r)
      QTP_HIP(hipMemcpyAsync(r, c.qp.r.get(), sizeof(double) * n,
                             hipMemcpyDeviceToDevice, c.stream));
    QTP_HIP(hipStreamSynchronize(c.stream));
    return QTP_OK;
  });
}

qtp_status qtp_pdip_solve(qtp_ctx ctx, qtp_step_stats* stats) {
  return guarded(ctx, [&](Ctx& c) {
    qtp_step_stats local{};
    qtp_step_stats* st = stats ? stats : &local;
    return qtp::pdip_solve(c, st);
  });
}

qtp_status qtp_get_impulses(qtp_ctx ctx, double* gamma) {
  return guarded(ctx, [&](Ctx& c) {
    QTP_REQUIRE(gamma, QTP_E_ARG, "null pointer");
    qtp::gather_impulses(c, gamma);
    return QTP_OK;
  });
}

qtp_status qtp_integrate(qtp_ctx ctx) {
  return guarded(ctx, [&](Ctx& c) {
    qtp::integrate(c);
    return QTP_OK;
  });
}

qtp_status qtp_get_state(qtp_ctx ctx, double* x, double* v, double* w) {
  return guarded(ctx, [&](Ctx& c) {
    QTP_REQUIRE(c.scene.M > 0, QTP_E_STATE, "no bodies");
    const size_t b3 = sizeof(double) * 3 * (size_t)c.scene.M;
    if (x) QTP_HIP(hipMemcpyAsync(x, c.scene.x.get(), b3, hipMemcpyDeviceToDevice, c.stream));
    if (v) QTP_HIP(hipMemcpyAsync(v, c.scene.v.get(), b3, hipMemcpyDeviceToDevice, c.stream));
    if (w) QTP_HIP(hipMemcpyAsync(w, c.scene.w.get(), b3, hipMemcpyDeviceToDevice, c.stream));
    QTP_HIP(hipStreamSynchronize(c.stream));
    return QTP_OK;
  });
}

qtp_status qtp_step(qtp_ctx ctx, qtp_step_stats* stats) {
  return guarded(ctx, [&](Ctx& c) {
    QTP_REQUIRE(c.scene.have_params && c.scene.M > 0, QTP_E_STATE,
                "set bodies and params first");
    qtp_step_stats local{};
    qtp_step_stats* st = stats ? stats : &local;
    using clk = std::chrono::steady_clock;
    auto ms = [](clk::time_point a, clk::time_point b) {
      return std::chrono::duration<double, std::milli>(b - a).count();
    };
    const auto t0 = clk::now();
    qtp::detect_contacts(c);
    const auto t1 = clk::now();
    qtp::assemble_qp(c);
    const auto t2 = clk::now();
    const int rc = qtp::pdip_solve(c, st);
    const auto t3 = clk::now();
    qtp::integrate(c);
    const auto t4 = clk::now();
    st->ms_detect = ms(t0, t1);
    st->ms_assemble = ms(t1, t2);
    st->ms_pdip = ms(t2, t3);
    st->ms_integrate = ms(t3, t4);
    st->ms_total = ms(t0, t4);
    return rc;
  });
}

int64_t qtp_mlp_param_count(void) { return qtp::mlp_param_count(); }

qtp_status qtp_mlp_features(qtp_ctx ctx, float* X) {
  return guarded(ctx, [&](Ctx& c) {
    QTP_REQUIRE(X, QTP_E_ARG, "null pointer");
    qtp::mlp_features(c, X);
    return QTP_OK;
  });
}

qtp_status qtp_mlp_targets(qtp_ctx ctx, float* Y) {
  return guarded(ctx, [&](Ctx& c) {
    QTP_REQUIRE(Y, QTP_E_ARG, "null pointer");
    qtp::mlp_targets(c, Y);
    return QTP_OK;
  });
}

qtp_status qtp_mlp_set_params(qtp_ctx ctx, const float* params) {
  return guarded(ctx, [&](Ctx& c) {
    QTP_REQUIRE(params, QTP_E_ARG, "null pointer");
    qtp::mlp_set_params(c, params);
    return QTP_OK;
  });
}

qtp_status qtp_mlp_get_params(qtp_ctx ctx, float* params) {
  return guarded(ctx, [&](Ctx& c) {
    QTP_REQUIRE(params, QTP_E_ARG, "null pointer");
    QTP_REQUIRE(c.mlp.have_params, QTP_E_STATE, "MLP parameters not set");
    QTP_HIP(hipMemcpyAsync(params, c.mlp.params.get(),
                           sizeof(float) * qtp::mlp_param_count(),
                           hipMemcpyDeviceToDevice, c.stream));
    QTP_HIP(hipStreamSynchronize(c.stream));
    return QTP_OK;
  });
}

qtp_status qtp_mlp_fit_normalization(qtp_ctx ctx, const float* X, int64_t n) {
  return guarded(ctx, [&](Ctx& c) {
    QTP_REQUIRE(X, QTP_E_ARG, "null pointer");
    qtp::mlp_fit_normalisation(c, X, n);
    return QTP_OK;
  });
}

qtp_status qtp_mlp_get_normalization(qtp_ctx ctx, float* mean_host, float* istd_host) {
  return guarded(ctx, [&](Ctx& c) {
    QTP_REQUIRE(mean_host && istd_host, QTP_E_ARG, "null pointer");
    qtp::mlp_get_normalisation(c, mean_host, istd_host);
    return QTP_OK;
  });
}

qtp_status qtp_mlp_forward(qtp_ctx ctx, const float* X, int B, float* P) {
  return guarded(ctx, [&](Ctx& c) {
    QTP_REQUIRE(X && P && B >= 1, QTP_E_ARG, "bad arguments");
    qtp::mlp_forward(c, X, B, P);
    QTP_HIP(hipStreamSynchronize(c.stream));
    return QTP_OK;
  });
}

qtp_status qtp_mlp_loss_grad(qtp_ctx ctx, const float* X, const float* Y, int B,
                             float* grads, double* loss_host) {
  return guarded(ctx, [&](Ctx& c) {
    QTP_REQUIRE(X && Y && B >= 1, QTP_E_ARG, "bad arguments");
    const double loss = qtp::mlp_loss_grad(c, X, Y, B);
    if (loss_host) *loss_host = loss;
    if (grads) {
      QTP_HIP(hipMemcpyAsync(grads, c.mlp.grads.get(),
                             sizeof(float) * qtp::mlp_param_count(),
                             hipMemcpyDeviceToDevice, c.stream));
      QTP_HIP(hipStreamSynchronize(c.stream));
    }
    return QTP_OK;
  });
}

qtp_status qtp_mlp_train_step(qtp_ctx ctx, const float* X, const float* Y, int B,
                              double lr, double* loss_host) {
  return guarded(ctx, [&](Ctx& c) {
    QTP_REQUIRE(X && Y && B >= 1 && lr > 0.0, QTP_E_ARG, "bad arguments");
    const double loss = qtp::mlp_train_step(c, X, Y, B, lr);
    if (loss_host) *loss_host = loss;
    return QTP_OK;
  });
}

qtp_status qtp_profile(qtp_ctx ctx, int enable) {
  return guarded(ctx, [&](Ctx& c) {
    c.flush_timers();
    c.timers.clear();
    c.profile = enable != 0;
    return QTP_OK;
  });
}

qtp_status qtp_get_kernel_time(qtp_ctx ctx, const char* name, double* ms_total,
                               int64_t* launches) {
  return guarded(ctx, [&](Ctx& c) {
    QTP_REQUIRE(name && ms_total && launches, QTP_E_ARG, "null pointer");
    c.flush_timers();
    *ms_total = 0.0;
    *launches = 0;
    for (auto& kv : c.timers)
      if (kv.first == name) {
        *ms_total = kv.second.ms;
        *launches = kv.second.count;
      }
    return QTP_OK;
  });
}

int qtp_get_newton_log(qtp_ctx ctx, qtp_newton_record* records_host, int capacity) {
  if (!ctx || capacity < 0 || (capacity > 0 && !records_host)) return QTP_E_ARG;
  const auto& log = ctx->c.pd.log;
  const int n = (int)log.size();
  for (int i = 0; i < n && i < capacity; ++i) records_host[i] = log[i];
  return n;
}

int qtp_get_qtt_ranks(qtp_ctx ctx, int which, int32_t* ranks_host) {
  if (!ctx || !ranks_host || (which != 0 && which != 1)) return QTP_E_ARG;
  const qtp::Qtt& q = which == 0 ? ctx->c.A : ctx->c.X;
  if (q.d == 0) return QTP_E_STATE;
  for (int k = 0; k <= q.d; ++k) ranks_host[k] = q.ranks[k];
  return q.d;
}

qtp_status qtp_get_qtt_cores(qtp_ctx ctx, int which, double* cores,
                             int64_t capacity) {
  return guarded(ctx, [&](Ctx& c) {
    QTP_REQUIRE(cores && (which == 0 || which == 1), QTP_E_ARG, "bad arguments");
    const qtp::Qtt& q = which == 0 ? c.A : c.X;
    QTP_REQUIRE(q.d > 0, QTP_E_STATE, "no QTT of that kind");
    QTP_REQUIRE(capacity >= q.total(), QTP_E_ARG, "capacity too small");
    QTP_HIP(hipMemcpyAsync(cores, q.cores.get(), sizeof(double) * q.total(),
                           hipMemcpyDeviceToDevice, c.stream));
    QTP_HIP(hipStreamSynchronize(c.stream));
    return QTP_OK;
  });
}

}  // extern "C"
