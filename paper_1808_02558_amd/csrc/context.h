// The library context: configuration, stream, persistent device state and
// workspaces.  One context per stream; calls on one context are serialised
// by the caller.
#pragma once

#include "../../include/qtp.h"
#include "common.h"
#include "ops.h"

namespace qtp {

// A QTT matrix held by the context: FP64 master cores plus optional
// reduced-precision copies used by the apply.
struct Qtt {
  int d = 0;
  std::vector<int32_t> ranks;   // d + 1
  DevBuf cores;                 // FP64, concatenated
  DevBuf cores_lp;              // FP32 or BF16 copy (precision != 0)
  int lp_prec = 0;              // precision of cores_lp (0 = none)
  int64_t total() const;
};

struct Ctx {
  qtp_config cfg{};
  hipStream_t stream = nullptr;
  std::string err;

  // Newton matrix (BSR3)
  int log2n = 0;
  int64_t n = 0;
  int nslots = 0;
  int64_t nnzb = 0;
  DevBuf rp, col, val;
  bool have_matrix = false;

  // preconditioner
  DevBuf Linv;        // [nslots][6]
  DevBuf sval;        // scaled values L^-1 S L^-T (BSR3)
  Qtt A;              // compressed scaled matrix
  Qtt X;              // approximate inverse
  bool have_precond = false;
  bool have_inverse = false;

  // workspaces
  DevBuf qtt_work;
  DevBuf V, Z, w, r, t1, t2;  // Krylov vectors
  DevBuf partial, scal;       // reductions
  DevBuf flag;                // int flags

  void check_cfg();
};

// Solver entry points (solver.hip)
int newton_solve(Ctx& c, const double* rhs, double* x, qtp_solve_stats* st);
void precond_apply(Ctx& c, const double* v, double* z);
void precond_factor(Ctx& c);          // block-Jacobi factors of the matrix
void ensure_lp_cores(Ctx& c, Qtt& q);  // reduced-precision copy of q
// QTT construction (qtt_build.hip)
void build_inverse(Ctx& c, int hot);

}  // namespace qtp
