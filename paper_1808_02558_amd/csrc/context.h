// The library context: configuration, stream, persistent device state and
// workspaces.  One context per stream; calls on one context are serialised
// by the caller.
#pragma once

#include "../../include/qtp.h"
#include "common.h"
#include "mlp.h"
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

// z-order (interleaved row/column bits) structure of the scaled matrix: the
// sorted entries and, per tree level k, the non-zero blocks (rows of the
// level-k unfolding) with the map from the finer level to them.
struct Pattern {
  bool valid = false;
  int d = 0;
  int64_t nent = 0, nval = 0;
  DevBuf keys, perm;
  std::vector<int64_t> nrows;   // rows of W_k, k = 1..d
  std::vector<DevBuf> seg;      // seg[k]: finer item -> row of W_k
  std::vector<DevBuf> rowkey;   // rowkey[k]: z prefix of each row of W_k
};

// Bodies, walls and step parameters of one time step (library copies).
struct Scene {
  int M = 0, nw = 0;
  DevBuf x, v, w, radius, mass, planes;
  double mu = 0.5, h = 1e-3, delta = 0.0;
  double g[3] = {0.0, 0.0, -9.81};
  int log2n = 0;
  bool have_params = false;
};

// The ordered active set: a, b (b >= M: wall b - M), gap, frame rows
// (n, t1, t2), Morton key and slot of each contact.
struct Contacts {
  int nc = 0;
  int npairs = 0;
  bool valid = false;
  DevBuf a, b, key, phi, frame, slot, bounds;
  DevBuf cell_key, cell_idx, cell_start, cell_stop;
  // slot re-use across time steps: the previous step's pairs (a << 32 | b,
  // sorted) with their slots, and per current contact its old slot or -1
  DevBuf prev_pair, prev_slot, old_slot;
  DevBuf taken, free_pos, free_list, new_rank, new_val, scan_tmp;
  int prev_n = -1;           // contacts of the previous step (-1: none)
  int prev_nslots = 0;
  int n_persistent = 0;      // contacts of this step that kept their slot
  bool rebuilt = false;      // this step fell back to the fresh map
};

// The QP of Sec. 2.3 in scaled units on the slot layout: N (BSR3, with
// identity dummy blocks), r (padded), and the body -> contact incidence.
struct Qp {
  bool valid = false;
  bool stale = false;  // positions moved since assembly
  double mbar = 0.0, vbar = 0.0, gbar = 0.0;  // mass, velocity, impulse scales
  int64_t nnzb = 0;
  DevBuf rp, col, valN, r, diagpos, inv_slot;
  DevBuf body_ptr, body_ent;  // incidence: (contact << 1) | (role A)
};

// PDIP iterate and work vectors.
struct Pdip {
  DevBuf gamma, dgamma, u, wv, rhs;   // padded [n]
  DevBuf dtrial;                       // second Newton step of the auto trial
  DevBuf lam, dlam;                    // [2 nc]: cone part then gamma_n part
  DevBuf part;                         // reduction partials
  bool have_gamma = false;
  std::vector<qtp_newton_record> log; // one record per Newton step
  DevBuf gamma_prev;                   // last converged solution (slot layout)
  bool have_prev = false;
  int warm_losses = 0;                 // consecutive failed warm starts
  int warm_skip = 0;                   // steps left that start cold
  int64_t prev_n = 0;
};

// Optional event timing of selected kernels on the context's stream.
struct KTimer {
  std::vector<std::pair<hipEvent_t, hipEvent_t>> pending;
  double ms = 0.0;
  int64_t count = 0;
};

struct BuildCache;
void destroy_build_cache(BuildCache* bc);

struct Ctx {
  ~Ctx() {
    destroy_build_cache(bcache);
    for (hipEvent_t e : event_pool) (void)hipEventDestroy(e);
  }
  BuildCache* bcache = nullptr;  // persistent scratch of the QTT construction
  qtp_config cfg{};
  bool profile = false;
  std::vector<std::pair<std::string, KTimer>> timers;
  std::vector<hipEvent_t> event_pool;  // recycled timing events
  KTimer& timer(const char* name);
  void flush_timers();
  hipEvent_t take_event() {
    if (event_pool.empty()) {
      hipEvent_t e;
      QTP_HIP(hipEventCreate(&e));
      return e;
    }
    hipEvent_t e = event_pool.back();
    event_pool.pop_back();
    return e;
  }
  hipStream_t stream = nullptr;
  std::string err;

  Scene scene;
  Contacts ct;
  Qp qp;
  Pdip pd;
  Mlp mlp;
  // temporaries of detection and assembly
  DevBuf tmp1, cnt, offs, cnt2, offs2, ua, ub, pk, perm, perm2;
  DevBuf sk, sv, sh, ss;  // sort and scan scratch

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
  bool use_qtt = true;          // apply X (else the block-Jacobi part only)
  bool auto_qtt = false;        // auto mode's choice for the current time step
  int auto_losses = 0;          // consecutive trials the QTT inverse lost
  int auto_skip = 0;            // time steps left before the next trial
  Pattern pat;
  int ns_done = 0;              // Newton-Schulz iterations of the last build
  double probe_residual = 0.0;  // rms of z - S~ X z over the probes
  double build_ms = 0.0;

  // workspaces
  DevBuf qtt_work;
  DevBuf V, Z, w, r, t1, t2;  // Krylov vectors
  DevBuf partial, scal;       // reductions
  DevBuf flag;                // int flags
  DevBuf arn_d, arn_partial;           // Arnoldi solve state
  HostBuf arn_status;                  // residual estimates for the host
  int64_t arn_tag = 0;                 // last status tag issued

  void check_cfg();
};

// Records events around a launch when the context profiles.
struct TimedLaunch {
  Ctx& c;
  KTimer* t = nullptr;
  hipEvent_t a = nullptr, b = nullptr;
  TimedLaunch(Ctx& ctx, const char* name) : c(ctx) {
    if (!c.profile) return;
    t = &c.timer(name);
    a = c.take_event();
    b = c.take_event();
    QTP_HIP(hipEventRecord(a, c.stream));
  }
  ~TimedLaunch() {
    if (!t) return;
    (void)hipEventRecord(b, c.stream);
    t->pending.emplace_back(a, b);
  }
};

// Solver entry points (solver.hip)
int newton_solve(Ctx& c, const double* rhs, double* x, qtp_solve_stats* st);
void precond_apply(Ctx& c, const double* v, double* z);
void precond_factor(Ctx& c);          // block-Jacobi factors of the matrix
void ensure_lp_cores(Ctx& c, Qtt& q);  // reduced-precision copy of q
// QTT construction (qtt_build.hip)
void build_inverse(Ctx& c, int hot);
// Time step (contacts.hip, assembly.hip, pdip.hip)
int detect_contacts(Ctx& c);
void assemble_qp(Ctx& c);
int pdip_solve(Ctx& c, qtp_step_stats* st);
void integrate(Ctx& c);
void gather_impulses(Ctx& c, double* out);

}  // namespace qtp
