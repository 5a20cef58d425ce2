// Learned warm start: state and entry points (mlp.hip).
#pragma once

#include "common.h"

namespace qtp {

struct Ctx;

struct Mlp {
  bool have_params = false, have_norm = false;
  int64_t adam_t = 0;
  DevBuf params, grads, m1, m2;   // flat FP32: W1 b1 W2 b2 W3 b3 W4 b4
  DevBuf mean, istd;              // feature normalisation [11]
  DevBuf xn, h[3], g[2], g3, p;   // activations and back-propagated terms
  DevBuf part, feat, ws;
};

int64_t mlp_param_count();
void mlp_features(Ctx& c, float* X);
void mlp_targets(Ctx& c, float* Y);
void mlp_set_params(Ctx& c, const float* params);
void mlp_fit_normalisation(Ctx& c, const float* X, int64_t n);
void mlp_get_normalisation(Ctx& c, float* mean_host, float* istd_host);
void mlp_forward(Ctx& c, const float* X, int B, float* P);
double mlp_loss_grad(Ctx& c, const float* X, const float* Y, int B);
double mlp_train_step(Ctx& c, const float* X, const float* Y, int B, double lr);
void mlp_warm_start(Ctx& c, double t0, double* gamma, double* lam);

}  // namespace qtp
