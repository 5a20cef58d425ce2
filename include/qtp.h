/* qtp -- QTT-accelerated primal-dual interior-point Newton-step solver for
 * frictional rigid-body contact, for one AMD MI355X (gfx950).
 *
 * C ABI.  All array arguments are DEVICE pointers unless a comment says
 * "host".  The caller owns every pointer it passes; the library reads inputs
 * during the call (or copies them into the context) and writes outputs into
 * caller buffers.  Every launch goes on the stream given to qtp_create, and
 * every call returns after its work is enqueued AND completed on that stream
 * unless noted.  No call throws or aborts: errors are returned as a negative
 * qtp_status and the message is available from qtp_last_error(ctx).
 *
 * Method: Corona, Gorsich, Jayakumar, Veerapaneni, "Tensor Train accelerated
 * solvers for nonsmooth rigid body dynamics" (arXiv 1808.02558).  Each entry
 * point names the passage that defines its operation.
 *
 * Layouts shared by several calls
 * -------------------------------
 * Unknowns.  A padded problem has n = 2^d unknowns.  Contact slot s in
 * [0, S), S = floor(n/3), owns unknowns 3s + {0: normal, 1: t1, 2: t2}
 * (Sec. 3.3: the contact hierarchy embedded in a uniform tree whose unused
 * leaves are dummy unknowns with an identity block).  Unknowns 3S..n-1 are
 * always dummies.
 *
 * BSR3 matrix.  A symmetric matrix on that layout stored as 3x3 blocks in
 * block-compressed-row form over slots: row_ptr[S+1] (int32), col[nnzb]
 * (int32 slot index, increasing within a block row), val[nnzb*9] (double,
 * each block row-major).  A dummy slot's block row is one identity block.
 * The dummy unknowns 3S..n-1 act as the identity and are not stored.
 *
 * QTT matrix (Sec. 3.2).  Ranks r_0..r_d (host int32 array of d+1 entries,
 * r_0 = r_d = 1).  Core k (k = 1..d) is an array [r_{k-1}][2][2][r_k]
 * indexed (alpha, i_k, j_k, beta), row-major; the cores are concatenated in
 * order k = 1..d.  A(i, j) = G_1(i_1, j_1) ... G_d(i_d, j_d) with i_1 the
 * most significant bit of the row index (Sec. 3.1 index convention).
 */
#ifndef QTP_H
#define QTP_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct qtp_ctx_s* qtp_ctx;

typedef enum {
  QTP_OK = 0,
  QTP_NOT_CONVERGED = 1, /* result written, but an iteration cap was hit */
  QTP_E_ARG = -1,        /* invalid argument; nothing was launched */
  QTP_E_OOM = -2,
  QTP_E_HIP = -3,        /* a HIP runtime error; see qtp_last_error */
  QTP_E_CAPACITY = -4,   /* contacts do not fit in floor(2^d/3) slots */
  QTP_E_NUMERIC = -5,    /* NaN/Inf or a non-positive pivot */
  QTP_E_STATE = -6       /* call order violated (e.g. solve before setup) */
} qtp_status;

typedef enum {
  QTP_PREC_F64 = 0,  /* FP64 cores and intermediates */
  QTP_PREC_F32 = 1,  /* FP32 cores and intermediates */
  QTP_PREC_BF16 = 2  /* BF16 cores, FP32 accumulation and intermediates */
} qtp_precision;

typedef struct {
  int precision;        /* qtp_precision of the QTT preconditioner apply */
  double qtt_eps;       /* relative TT truncation tolerance (Algorithm 1) */
  int qtt_rmax;         /* rank cap of the approximate inverse X */
  int qtt_rmax_s;       /* rank cap of the compressed scaled matrix */
  int ns_iters;         /* Newton-Schulz iterations for a cold inverse */
  int ns_iters_hot;     /* Newton-Schulz iterations for a hot-started inverse */
  int solve_mode;       /* 0: X * rhs + iterative refinement, 1: FGMRES */
  double solve_tol;     /* relative residual of the Newton-step solve */
  int fgmres_restart;   /* FGMRES restart length m, 1..32 */
  int fgmres_maxit;     /* total FGMRES (or refinement) iteration cap */
  double pdip_gap_tol;  /* PDIP stop: gap / m */
  double pdip_dual_tol; /* PDIP stop: |r_dual|_inf in scaled units */
  int pdip_maxit;
  int warm_start;       /* 0 cold (gamma = (1, 0, 0));
                           1 Sec. 3.3 re-use: contacts that kept their slot
                             (slot_mode 1) start from their previous normal
                             impulse with zero friction, new ones cold;
                           2 learned (MLP);
                           3 as 1, keeping the previous friction impulse too;
                           1-3 fall back to cold after warm_maxit iterations;
                           after k consecutive fallbacks the next 2^k - 1
                           solves (k <= 6) start cold */
  uint64_t seed;
  double warm_t0;       /* central-path parameter of the learned start */
  int qtt_mode;         /* PDIP preconditioner: 0 block-Jacobi only (X = I),
                           1 QTT inverse on every Newton step,
                           2 auto: the first Newton step of a time step is
                             solved with both, the faster is kept (the QTT
                             solve stops at twice the block-Jacobi
                             iterations plus 10, a loss); after a lost trial
                             the next 2^k - 1 time steps (k consecutive
                             losses, k <= 6) skip the trial and use
                             block-Jacobi */
  double warm_floor;    /* learned and previous-step starts: lower bound on
                           the starting normal impulse in scaled units (keeps
                           the start away from the cone's boundary) */
  int slot_mode;        /* 0: fresh slot map every step (Morton rank order);
                           1: contacts present in the previous step keep their
                             slot, new ones take the next free slot at or
                             after their fresh one, rebuilt when none is left
                             (Sec. 3.3, re-use across time steps) */
  int warm_maxit;       /* PDIP iterations allowed to a warm start before the
                           cold start takes over */
} qtp_config;

/* Fills a config with the defaults: FP64, eps 1e-2, rmax 32, rmax_s 16,
 * FGMRES(30) to 1e-8, PDIP gap 1e-8 and dual 1e-4, 100 PDIP iterations. */
void qtp_config_default(qtp_config* cfg);

/* Creates a context bound to `hip_stream` (a hipStream_t; NULL = default
 * stream) on the current device.  cfg may be NULL (defaults). */
qtp_status qtp_create(const qtp_config* cfg, void* hip_stream, qtp_ctx* out);
void qtp_destroy(qtp_ctx ctx);
const char* qtp_last_error(qtp_ctx ctx);
/* Updates the configuration of an existing context (host struct); the auto
 * mode's trial and the warm-start back-offs restart from zero. */
qtp_status qtp_set_config(qtp_ctx ctx, const qtp_config* cfg);

/* ---------------------------------------------------------------------------
 * Building blocks of the Newton-step solve (Sec. 3.2-3.3).
 * ------------------------------------------------------------------------- */

/* y = A x for a BSR3 matrix on n = 2^d unknowns (d = log2n): the sparse
 * product with the Schur complement S_k, whose block pattern is that of
 * N = D^T M^-1 D (Sec. 3.3, sparsity of N).  x, y: [n] double, must not
 * alias.  Returns QTP_E_ARG for d outside [2, 30] or null pointers. */
qtp_status qtp_bsr_spmv(qtp_ctx ctx, int log2n, const int32_t* row_ptr,
                        const int32_t* col, const double* val, const double* x,
                        double* y);

/* y = A x for a QTT matrix (Sec. 3.2: the TT matrix-vector product contracts
 * one dimension at a time, O(r^2 N log N)).  ranks: host [d+1].  cores:
 * device, element type by `precision` (double / float / bf16 as uint16).
 * x, y: [2^d] double, may not alias.  Intermediates use the context's
 * workspace.  Ranks must be in [1, 256]. */
qtp_status qtp_qtt_apply(qtp_ctx ctx, int d, const int32_t* ranks,
                         const void* cores, int precision, const double* x,
                         double* y);

/* ---------------------------------------------------------------------------
 * The Newton-step solve on a loaded matrix (Sec. 3.3, "TT Newton system
 * solver": the approximate TT inverse used as a direct solver with iterative
 * refinement, or as the preconditioner of a Krylov method).
 * ------------------------------------------------------------------------- */

/* Copies a BSR3 Newton matrix S into the context (device to device).
 * nnzb = row_ptr[S] is read back from the device. */
qtp_status qtp_set_newton_matrix(qtp_ctx ctx, int log2n, const int32_t* row_ptr,
                                 const int32_t* col, const double* val);

/* Builds the preconditioner for the loaded matrix: the block-Jacobi factors
 * L = blockdiag(chol S_ss), the QTT compression of L^-1 S L^-T (a right-to-
 * left block-sparse Algorithm 1) and its approximate inverse X (Newton-
 * Schulz with TT rounding).  hot != 0 starts Newton-Schulz from the previous
 * X (the inverse update of Sec. 3.2-3.3); otherwise from a scaled identity.
 * Preconditioner P = L^-T X L^-1.  Must follow qtp_set_newton_matrix. */
qtp_status qtp_precond_build(qtp_ctx ctx, int hot);

/* Same as qtp_precond_build but loads a given FP64 QTT inverse X instead of
 * computing one (the block-Jacobi factors are still computed from S). */
qtp_status qtp_precond_load_qtt(qtp_ctx ctx, int d, const int32_t* ranks,
                                const double* cores);

typedef struct {
  int iterations;        /* FGMRES iterations or refinement steps */
  double rel_residual;   /* |b - S x| / |b| recomputed at the end */
  double ms;             /* wall time of the solve on the stream */
} qtp_solve_stats;

/* Solves S x = rhs to the configured relative residual.  rhs, x: [2^d]
 * double (may not alias).  Returns QTP_NOT_CONVERGED (with x and stats
 * written) when the iteration cap is reached. */
qtp_status qtp_newton_solve(qtp_ctx ctx, const double* rhs, double* x,
                            qtp_solve_stats* stats);

/* Applies the current preconditioner: z = L^-T X L^-1 v. */
qtp_status qtp_precond_apply(qtp_ctx ctx, const double* v, double* z);

typedef struct {
  int ns_iterations;      /* Newton-Schulz iterations run by the last build */
  double probe_residual;  /* max over the two probes of rms(z - S~ X z) */
  int max_rank_s;         /* largest rank of the compressed S~ */
  int max_rank_x;         /* largest rank of X */
  double ms;              /* wall time of the last build */
} qtp_precond_stats;

/* Statistics of the last qtp_precond_build on this context. */
qtp_status qtp_get_precond_stats(qtp_ctx ctx, qtp_precond_stats* out);

/* ---------------------------------------------------------------------------
 * One time step of frictional contact dynamics (Sec. 2.1-2.4, 3.3).
 * ------------------------------------------------------------------------- */

/* Copies M spheres into the context (Sec. 2.1): x, v, w [M][3] double (centre,
 * velocity, angular velocity), radius [M], mass [M] (device pointers). */
qtp_status qtp_set_bodies(qtp_ctx ctx, int M, const double* x, const double* v,
                          const double* w, const double* radius,
                          const double* mass);

/* Static container planes [nw][4]: unit normal n into the domain and offset o
 * (inside: n.x - o >= 0).  Host pointer.  Walls have infinite mass. */
qtp_status qtp_set_walls(qtp_ctx ctx, int nw, const double* planes_host);

/* Friction coefficient mu (Sec. 2.2), step h, active-set threshold delta
 * (A(q, delta) = {Phi <= delta}), gravity [3] (host), padded size 2^log2n. */
qtp_status qtp_set_params(qtp_ctx ctx, double mu, double h, double delta,
                          const double* gravity_host, int log2n);

/* Contact detection (Sec. 2.2) and ordering (Sec. 3.3).  Writes the number of
 * contacts.  QTP_E_CAPACITY when they exceed floor(2^log2n / 3) slots. */
qtp_status qtp_detect(qtp_ctx ctx, int* n_contacts);

/* Copies the ordered contacts out (device buffers of nc entries): a, b
 * (int32; b >= M means wall b - M), phi [nc], frame [nc][9] (rows n, t1, t2),
 * key [nc] (uint64 Morton key), slot [nc] (int32).  Any pointer may be NULL. */
qtp_status qtp_get_contacts(qtp_ctx ctx, int32_t* a, int32_t* b, double* phi,
                            double* frame, uint64_t* key, int32_t* slot);

/* Assembles N = D^T M^-1 D and r = b + D^T M^-1 k (Sec. 2.3) in scaled units
 * (N * m_bar, r / (g h)) on the slot layout.  Follows qtp_detect. */
qtp_status qtp_assemble(qtp_ctx ctx);

/* Copies the assembled QP out: BSR3 pattern (row_ptr [S+1], col [nnzb]),
 * values of N [nnzb*9] and r [2^d]; returns nnzb through *nnzb (host). Any
 * array pointer may be NULL to query nnzb only. */
qtp_status qtp_get_qp(qtp_ctx ctx, int32_t* row_ptr, int32_t* col, double* valN,
                      double* r, int64_t* nnzb);

typedef struct {
  int n_contacts;
  int pdip_iterations;
  int converged;
  int fgmres_iterations;   /* total over the Newton steps */
  int max_fgmres;          /* largest count of one Newton step */
  double gap;              /* final eta / m */
  double dual_inf;         /* final |r_dual|_inf, scaled units */
  double ms_detect, ms_assemble, ms_precond, ms_solve, ms_pdip, ms_integrate;
  double ms_total;
  double newton_solve_ms_median;
  int qtt_used;            /* Newton steps solved with the QTT inverse */
  int qtt_trial_iterations;   /* auto mode: FGMRES its of the QTT trial */
  int plain_trial_iterations; /* auto mode: FGMRES its of the X = I trial */
  int warm_started;        /* start used: 0 cold, 1 previous step, 2 learned */
  int warm_fallback;       /* 1 when it failed and the cold start ran */
  int warm_iterations;     /* PDIP iterations spent in the failed warm run */
  int persistent_contacts; /* slot_mode 1: contacts that kept their slot */
  int slots_rebuilt;       /* slot_mode 1: 1 when the map fell back to fresh */
} qtp_step_stats;

/* PDIP on the assembled QP (Sec. 2.4 with the Schur-complement Newton system
 * of Sec. 3.3; each Newton step solved by qtp_newton_solve's method with the
 * QTT preconditioner built on the first step and hot-started afterwards).
 * Start: gamma = (1, 0, 0) per contact in scaled units (Sec. 3.3).  Returns
 * QTP_NOT_CONVERGED when pdip_maxit is reached. */
qtp_status qtp_pdip_solve(qtp_ctx ctx, qtp_step_stats* stats);

/* One Newton step of the last PDIP solve: its PDIP iteration, the FGMRES
 * iterations and wall milliseconds of the kept solve (the preconditioner
 * already built), the milliseconds spent building preconditioners for it,
 * whether the QTT inverse was applied, and the final relative residual. */
typedef struct {
  int pdip_iteration;
  int fgmres_iterations;
  int used_qtt;
  double solve_ms;
  double precond_ms;
  double rel_residual;
} qtp_newton_record;

/* Copies up to `capacity` records of the last PDIP solve into host memory
 * and returns how many the solve made (which may exceed capacity), or a
 * negative status. */
int qtp_get_newton_log(qtp_ctx ctx, qtp_newton_record* records_host, int capacity);

/* Impulses of the last PDIP solve in the contact frame, physical units
 * (N s): [nc][3] double. */
qtp_status qtp_get_impulses(qtp_ctx ctx, double* gamma);

/* Semi-implicit update (Sec. 2.2): v += M^-1 (h f + D gamma), x += h v. */
qtp_status qtp_integrate(qtp_ctx ctx);

/* Copies the body state out: x, v, w [M][3] (any may be NULL). */
qtp_status qtp_get_state(qtp_ctx ctx, double* x, double* v, double* w);

/* detect + assemble + PDIP + integrate. */
qtp_status qtp_step(qtp_ctx ctx, qtp_step_stats* stats);

/* ---------------------------------------------------------------------------
 * Learned warm start (an MLP 11 -> 128 -> 128 -> 128 -> 3, FP32, tanh).
 * The paper starts the PDIP cold (Sec. 3.3, "Re-using information across
 * timesteps"); with warm_start = 2 the start is the network's prediction,
 * strictly inside the cone, with multipliers on the central path of warm_t0,
 * and the cold start runs when that PDIP does not converge.
 * Parameters are one flat FP32 vector W1 b1 W2 b2 W3 b3 W4 b4 with W_l
 * stored [fan_in][fan_out] row-major (x W + b).
 * ------------------------------------------------------------------------- */

/* Number of FP32 parameters (host). */
int64_t qtp_mlp_param_count(void);

/* Per-contact features of the current contacts [nc][11] FP32 (device);
 * follows qtp_detect and qtp_assemble. */
qtp_status qtp_mlp_features(qtp_ctx ctx, float* X);

/* Training targets [nc][3] FP32 (device) of the last PDIP solve's impulses in
 * scaled units: log(gamma_n) and gamma_t / (mu gamma_n) projected into the
 * unit disc, the inverse of the warm start's output map.  Valid after
 * qtp_pdip_solve (or qtp_step, which leaves the contacts of its solve). */
qtp_status qtp_mlp_targets(qtp_ctx ctx, float* Y);

/* Sets / gets the parameters (device, qtp_mlp_param_count floats); setting
 * resets the Adam moments. */
qtp_status qtp_mlp_set_params(qtp_ctx ctx, const float* params);
qtp_status qtp_mlp_get_params(qtp_ctx ctx, float* params);

/* Fits the feature z-scoring to n rows of X [n][11] (device); the mean and
 * inverse deviation can be read back (host [11] each). */
qtp_status qtp_mlp_fit_normalization(qtp_ctx ctx, const float* X, int64_t n);
qtp_status qtp_mlp_get_normalization(qtp_ctx ctx, float* mean_host,
                                     float* istd_host);

/* P [B][3] = network(normalised X [B][11]) (device). */
qtp_status qtp_mlp_forward(qtp_ctx ctx, const float* X, int B, float* P);

/* Loss (mean squared error over rows and outputs) and its gradient with
 * respect to every parameter (device, qtp_mlp_param_count floats). */
qtp_status qtp_mlp_loss_grad(qtp_ctx ctx, const float* X, const float* Y, int B,
                             float* grads, double* loss_host);

/* One Adam step (Kingma & Ba; beta 0.9 / 0.999, eps 1e-8) on a batch. */
qtp_status qtp_mlp_train_step(qtp_ctx ctx, const float* X, const float* Y,
                              int B, double lr, double* loss_host);

/* ---------------------------------------------------------------------------
 * Measurement hooks.
 * ------------------------------------------------------------------------- */

/* Enables (1) or disables (0) event timing of the Newton-step kernels on the
 * context's stream and clears the accumulated times.  Timed groups:
 * "bsr_spmv" (one sparse product), "qtt_apply" (one QTT product, all
 * levels), "cgs2" (one Arnoldi orthogonalisation). */
qtp_status qtp_profile(qtp_ctx ctx, int enable);

/* Total milliseconds and launch count of a timed group since qtp_profile. */
qtp_status qtp_get_kernel_time(qtp_ctx ctx, const char* name, double* ms_total,
                               int64_t* launches);

/* Ranks of the current compressed matrix (which = 0) or inverse (which = 1):
 * writes up to d+1 ints into ranks_host and returns d, or a negative status. */
int qtp_get_qtt_ranks(qtp_ctx ctx, int which, int32_t* ranks_host);

/* Copies the FP64 cores of the compressed matrix (which = 0) or inverse
 * (which = 1) into a device buffer of at least `capacity` doubles. */
qtp_status qtp_get_qtt_cores(qtp_ctx ctx, int which, double* cores,
                             int64_t capacity);

#ifdef __cplusplus
}
#endif

#endif /* QTP_H */
