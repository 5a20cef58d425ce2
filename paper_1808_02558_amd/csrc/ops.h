// Internal launchers of the qtp kernels (host side).  Every launcher enqueues
// on the given stream and returns without synchronising.
#pragma once

#include "common.h"

namespace qtp {

// ---- BSR3 sparse product (spmv.hip) ----------------------------------------
// y = A x; A has nslots block rows of 3x3 blocks, n >= 3*nslots unknowns,
// unknowns 3*nslots..n-1 are identity rows.
void bsr_spmv(hipStream_t s, int nslots, int64_t n, const int32_t* rp,
              const int32_t* col, const double* val, const double* x, double* y);

// ---- QTT matrix-vector product (qtt_apply.hip) -------------------------------
// Offsets (in elements) of each core in the concatenated core array.
std::vector<int64_t> core_offsets(int d, const int32_t* ranks);
// Bytes of workspace that qtt_apply needs for these ranks and precision.
size_t qtt_apply_workspace(int d, const int32_t* ranks, int prec);
void qtt_apply(hipStream_t s, int d, const int32_t* ranks, const void* cores,
               int prec, const double* x, double* y, void* work);

// ---- vector kernels (blas1.hip) ---------------------------------------------
// Number of per-block partial sums a reduction over n elements produces.
int reduce_blocks(int64_t n);
// out[l] = V_l . w for l < nvec (V rows of length n with leading dim ldv).
// partial: reduce_blocks(n) * nvec doubles of scratch.
void multi_dot(hipStream_t s, int nvec, const double* V, int64_t ldv,
               const double* w, int64_t n, double* partial, double* out);
// w -= sum_l h[l] V_l ; then out[l] = V_l . w (new w) for l < nvec.
void cgs_update_dot(hipStream_t s, int nvec, const double* V, int64_t ldv,
                    const double* h, double* w, int64_t n, double* partial,
                    double* out);
// w -= sum_l h[l] V_l ; then out[0] = w . w.
void cgs_update_norm2(hipStream_t s, int nvec, const double* V, int64_t ldv,
                      const double* h, double* w, int64_t n, double* partial,
                      double* out);
// out[0] = x . y
void dot(hipStream_t s, const double* x, const double* y, int64_t n,
         double* partial, double* out);
// y = a * x   (a read from device memory a_dev[0], inverted when inv != 0)
void scale_dev(hipStream_t s, const double* a_dev, int inv, const double* x,
               double* y, int64_t n);
// y += sum_l c[l] X_l   (c on device)
void multi_axpy(hipStream_t s, int nvec, const double* X, int64_t ldx,
                const double* c, double* y, int64_t n);
// z = x - y
void sub(hipStream_t s, const double* x, const double* y, double* z, int64_t n);
// y += x
void add_inplace(hipStream_t s, const double* x, double* y, int64_t n);
// Non-finite check: out[0] = 1 if any entry of x is NaN/Inf else 0.
void any_nonfinite(hipStream_t s, const double* x, int64_t n, int* out);

// ---- Arnoldi steps of FGMRES (arnoldi.hip) ------------------------------------
constexpr int kArnMaxRestart = 32;  // longest restart cycle
constexpr int kArnLd = 64;          // leading dimension of the Hessenberg columns
constexpr int kArnRing = 64;        // entries of the host status ring (power of 2)
// Offsets (in doubles) of the device solve state Arnoldi::d.
enum : int {
  kArnH1 = 0,      // first Gram-Schmidt coefficients of the current step
  kArnH2 = 64,     // second (re-orthogonalisation) coefficients
  kArnInv = 128,   // 1 / h_{j+1,j} of the last step (0 on breakdown)
  kArnG = 192,     // rotated right-hand side beta e_1
  kArnCs = 256,    // Givens cosines
  kArnSn = 320,    // Givens sines
  kArnY = 384,     // least-squares solution of the cycle
  kArnH = 448,     // Hessenberg, column j at kArnH + j * kArnLd
  kArnDoubles = kArnH + kArnLd * kArnMaxRestart
};
// The host-visible status ring holds one double per Arnoldi step: the
// least-squares residual |g_{j+1}| (0 on a breakdown, NaN when the step went
// non-finite), written by the device with a single system-scope store into a
// slot the host has set to -1 (empty).
constexpr double kArnEmpty = -1.0;
struct Arnoldi {
  double* d = nullptr;          // kArnDoubles doubles (device)
  double* partial = nullptr;    // arnoldi_partial_doubles(n) doubles (device)
  double* status = nullptr;     // kArnRing entries, device view of pinned memory
};
size_t arnoldi_partial_doubles(int64_t n);
// V_j = (src - sum_{l<nprev} h2_l V_l) * inv, inv = d[kArnInv] when nprev > 0
// else inv0 (nprev == 0 also sets g = beta e_1); then zout = L^-T L^-1 V_j
// (full = 1) or L^-1 V_j (full = 0).  src may alias vj.
void arnoldi_next(hipStream_t s, const Arnoldi& a, int nprev, const double* V,
                  int64_t n, int nslots, double inv0, double beta, const double* src,
                  double* vj, const double* Linv, int full, double* zout);
// h1 = V_{0..nvec-1}^T w
void arnoldi_dots(hipStream_t s, const Arnoldi& a, int nvec, const double* V,
                  int64_t n, const double* w);
// w -= V h1; h2 = V^T w; Hessenberg column nvec - 1, Givens rotation and the
// status entry tag mod kArnRing.
void arnoldi_orth(hipStream_t s, const Arnoldi& a, int nvec, const double* V,
                  int64_t n, double* w, int64_t tag);
// d[kArnY..] = least-squares solution of the first jend columns
void arnoldi_solve(hipStream_t s, const Arnoldi& a, int jend);

// ---- block-Jacobi scaling (blas1.hip) ---------------------------------------
// Linv[s][6] = lower triangle (row-major: l00 l10 l11 l20 l21 l22) of the
// inverse of chol(A_ss), the diagonal 3x3 block of block row s.
// bad[0] is set to 1 when a pivot is not positive.
void bj_factor(hipStream_t s, int nslots, const int32_t* rp, const int32_t* col,
               const double* val, double* Linv, int* bad);
// y = L^-1 x (trans = 0) or y = L^-T x (trans = 1); identity beyond 3*nslots.
void bj_apply(hipStream_t s, int nslots, int64_t n, const double* Linv,
              int trans, const double* x, double* y);
// Scaled matrix: vout = L^-1 A L^-T blockwise (same BSR3 pattern).
void bj_scale_matrix(hipStream_t s, int nslots, const int32_t* rp,
                     const int32_t* col, const double* val, const double* Linv,
                     double* vout);

}  // namespace qtp
