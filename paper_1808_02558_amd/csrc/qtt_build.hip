// QTT compression of the scaled Newton matrix and its approximate inverse.
//
// Compression (Sec. 3.1 Algorithm 1, Sec. 3.2 matrix tensorisation).  The
// block-Jacobi scaled matrix S~ = L^-1 S L^-T is tensorised with modes
// b_k = 2 i_k + j_k, i.e. its entries are ordered by the interleaved bits
// z = (i_1 j_1 i_2 j_2 ... i_d j_d) of (row, column).  Algorithm 1 is run from
// the last mode to the first, directly on the non-zeros: at core k the
// unfolding has one row per non-zero block of size 2^{d-k+1} (a distinct
// prefix of z) and 4 r_k columns (the child b_k and the rank index of the
// already compressed right part), so only non-zero blocks are ever stored.
// Each step forms the Gram matrix W^T W, takes its leading eigenvectors
// (= right singular vectors of W) as the core, and carries W V to the
// parent blocks.  Truncation per bond: the discarded squared singular values
// sum to at most (eps |S~|_F)^2 / (d - 1), with a rank cap.
//
// Inverse (Sec. 3.2 inverse updates, Sec. 3.3 hot start).  Newton-Schulz
// X <- X (2 I - Y), Y = S~_TT X, with every product rounded (TT rounding:
// Gram matrices of the right interfaces, then a left-to-right truncated
// eigen-decomposition sweep).  Started from a scaled identity or from the
// previous X.  Progress is judged on two fixed probe vectors with the exact
// S~ (sparse product) and the best iterate is kept.
#include <algorithm>
#include <cmath>

#include "context.h"
#include "dense.h"

namespace qtp {
namespace {

constexpr int kT = 256;

__device__ inline uint64_t spread_bits(uint64_t v) {
  // spread the low 32 bits of v to even bit positions
  v &= 0xffffffffull;
  v = (v | (v << 16)) & 0x0000ffff0000ffffull;
  v = (v | (v << 8)) & 0x00ff00ff00ff00ffull;
  v = (v | (v << 4)) & 0x0f0f0f0f0f0f0f0full;
  v = (v | (v << 2)) & 0x3333333333333333ull;
  v = (v | (v << 1)) & 0x5555555555555555ull;
  return v;
}

__device__ inline uint64_t zkey(uint64_t row, uint64_t col) {
  return (spread_bits(row) << 1) | spread_bits(col);
}

__global__ void block_rows_kernel(int nslots, const int32_t* __restrict__ rp,
                                  int32_t* __restrict__ brow) {
  const int s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= nslots) return;
  for (int q = rp[s]; q < rp[s + 1]; ++q) brow[q] = s;
}

__global__ void entry_keys_kernel(int64_t nnzb, int nslots, int64_t n,
                                  const int32_t* __restrict__ brow,
                                  const int32_t* __restrict__ col,
                                  uint64_t* __restrict__ keys,
                                  int32_t* __restrict__ perm) {
  const int64_t e = (int64_t)blockIdx.x * kT + threadIdx.x;
  const int64_t nval = 9 * nnzb;
  const int64_t ntail = n - 3 * (int64_t)nslots;
  if (e < nval) {
    const int64_t q = e / 9;
    const int w = (int)(e - 9 * q);
    const uint64_t row = 3 * (uint64_t)brow[q] + w / 3;
    const uint64_t cl = 3 * (uint64_t)col[q] + w % 3;
    keys[e] = zkey(row, cl);
    perm[e] = (int32_t)e;
  } else if (e < nval + ntail) {
    const uint64_t u = 3 * (uint64_t)nslots + (e - nval);
    keys[e] = zkey(u, u);
    perm[e] = (int32_t)e;  // >= nval: identity entry
  }
}

// flag[i] = 1 when key[i] >> shift differs from key[i-1] >> shift
__global__ void head_flags_kernel(const uint64_t* __restrict__ keys, int64_t n,
                                  int shift, int* __restrict__ flag) {
  const int64_t i = (int64_t)blockIdx.x * kT + threadIdx.x;
  if (i >= n) return;
  flag[i] = (i == 0 || (keys[i] >> shift) != (keys[i - 1] >> shift)) ? 1 : 0;
}

// seg[i] = index of i's segment; heads write their shifted key to ukey
__global__ void seg_ids_kernel(const uint64_t* __restrict__ keys, int64_t n,
                               int shift, const int* __restrict__ flag,
                               const int* __restrict__ excl, int32_t* __restrict__ seg,
                               uint64_t* __restrict__ ukey) {
  const int64_t i = (int64_t)blockIdx.x * kT + threadIdx.x;
  if (i >= n) return;
  const int id = excl[i] + flag[i] - 1;
  seg[i] = id;
  if (flag[i]) ukey[id] = keys[i] >> shift;
}

// Leaf level: W_d[leaf][z & 3] = value, and the squared norm partials.
__global__ void fill_leaves_kernel(int64_t nent, int64_t nval,
                                   const uint64_t* __restrict__ keys,
                                   const int32_t* __restrict__ perm,
                                   const int32_t* __restrict__ leaf,
                                   const double* __restrict__ sval,
                                   double* __restrict__ W) {
  const int64_t i = (int64_t)blockIdx.x * kT + threadIdx.x;
  if (i >= nent) return;
  const int32_t p = perm[i];
  const double v = p < nval ? sval[p] : 1.0;
  W[(int64_t)leaf[i] * 4 + (keys[i] & 3)] = v;
}

__global__ void sumsq_kernel(const double* __restrict__ x, int64_t n,
                             double* __restrict__ partial) {
  __shared__ double sh[kT / 64];
  double acc = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * kT + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * kT)
    acc += x[i] * x[i];
  for (int o = 32; o > 0; o >>= 1) acc += __shfl_xor(acc, o, 64);
  if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = acc;
  __syncthreads();
  if (threadIdx.x == 0) {
    double s = 0.0;
    for (int i = 0; i < kT / 64; ++i) s += sh[i];
    partial[blockIdx.x] = s;
  }
}

// Parent rows: W_{k-1}[parent[q]][b(q) r + a] = P[q][a]
__global__ void scatter_parent_kernel(int64_t nrows, int r,
                                      const int32_t* __restrict__ parent,
                                      const uint64_t* __restrict__ rowkey,
                                      const double* __restrict__ P,
                                      double* __restrict__ Wp) {
  const int64_t e = (int64_t)blockIdx.x * kT + threadIdx.x;
  if (e >= nrows * r) return;
  const int64_t q = e / r;
  const int a = (int)(e - q * r);
  const int b = (int)(rowkey[q] & 3);
  Wp[(int64_t)parent[q] * 4 * r + b * r + a] = P[e];
}

// core[a][c] = V[c][a] for a < r, c < ncol (V is ncol x ncol row-major)
__global__ void take_columns_T_kernel(int ncol, int r, const double* __restrict__ V,
                                      double* __restrict__ core) {
  const int e = blockIdx.x * kT + threadIdx.x;
  if (e >= r * ncol) return;
  const int a = e / ncol, c = e % ncol;
  core[e] = V[(int64_t)c * ncol + a];
}

// out[i][j] = V[i][j] for j < r (first r columns of an n x n matrix)
__global__ void take_columns_kernel(int n, int r, const double* __restrict__ V,
                                    double* __restrict__ out) {
  const int e = blockIdx.x * kT + threadIdx.x;
  if (e >= n * r) return;
  const int i = e / r, j = e % r;
  out[e] = V[(int64_t)i * n + j];
}

// C_k = A_k (x) B_k contracted over the inner mode:
// C[(a,b)][i][j][(a',b')] = sum_l A[a][i][l][a'] B[b][l][j][b']
__global__ void tt_matmul_core_kernel(int ra, int ra2, int rb, int rb2,
                                      const double* __restrict__ A,
                                      const double* __restrict__ B,
                                      double* __restrict__ C) {
  const int64_t R2 = (int64_t)ra2 * rb2;
  const int64_t total = (int64_t)ra * rb * 4 * R2;
  const int64_t e = (int64_t)blockIdx.x * kT + threadIdx.x;
  if (e >= total) return;
  const int64_t right = e % R2;
  const int ij = (int)((e / R2) % 4);
  const int64_t left = e / (R2 * 4);
  const int a = (int)(left / rb), b = (int)(left % rb);
  const int a2 = (int)(right / rb2), b2 = (int)(right % rb2);
  const int i = ij >> 1, j = ij & 1;
  double s = 0.0;
#pragma unroll
  for (int l = 0; l < 2; ++l)
    s += A[(((int64_t)a * 2 + i) * 2 + l) * ra2 + a2] *
         B[(((int64_t)b * 2 + l) * 2 + j) * rb2 + b2];
  C[e] = s;
}

// C = alpha A + beta B in TT form: first cores side by side, last cores
// stacked, middle cores block-diagonal (ranks add).
__global__ void tt_add_core_kernel(int ra, int ra2, int rb, int rb2, int first,
                                   int last, double alpha, double beta,
                                   const double* __restrict__ A,
                                   const double* __restrict__ B,
                                   double* __restrict__ C) {
  const int rc = first ? 1 : ra + rb;
  const int rc2 = last ? 1 : ra2 + rb2;
  const int64_t total = (int64_t)rc * 4 * rc2;
  const int64_t e = (int64_t)blockIdx.x * kT + threadIdx.x;
  if (e >= total) return;
  const int c2 = (int)(e % rc2);
  const int m = (int)((e / rc2) % 4);
  const int c = (int)(e / ((int64_t)rc2 * 4));
  double v;
  if (first && last) {
    v = alpha * A[m] + beta * B[m];
  } else if (first) {
    v = c2 < ra2 ? alpha * A[(int64_t)m * ra2 + c2]
                 : beta * B[(int64_t)m * rb2 + (c2 - ra2)];
  } else if (last) {
    v = c < ra ? A[(int64_t)c * 4 + m] : B[(int64_t)(c - ra) * 4 + m];
  } else if (c < ra && c2 < ra2) {
    v = A[((int64_t)c * 4 + m) * ra2 + c2];
  } else if (c >= ra && c2 >= ra2) {
    v = B[((int64_t)(c - ra) * 4 + m) * rb2 + (c2 - ra2)];
  } else {
    v = 0.0;
  }
  C[e] = v;
}

__global__ void fill_identity_core_kernel(double* __restrict__ core, double a) {
  const int e = threadIdx.x;
  if (e < 4) core[e] = (e == 0 || e == 3) ? a : 0.0;
}

__global__ void probe_kernel(int64_t n, double* __restrict__ z1,
                             double* __restrict__ z2) {
  const int64_t i = (int64_t)blockIdx.x * kT + threadIdx.x;
  if (i >= n) return;
  z1[i] = 1.0;
  z2[i] = (__popcll((unsigned long long)i) & 1) ? -1.0 : 1.0;
}

// out[0] = max_s sum_j |A_sj| over rows (Gershgorin bound); one block.
// Per-block maximum Gershgorin row sum of the scaled matrix (dummy rows of
// the identity contribute 1); the host takes the maximum of the partials.
__global__ void gershgorin_kernel(int nslots, const int32_t* __restrict__ rp,
                                  const double* __restrict__ val,
                                  double* __restrict__ part) {
  __shared__ double sh[kT];
  double m = 1.0;
  for (int s = blockIdx.x * kT + threadIdx.x; s < nslots; s += gridDim.x * kT) {
    double r0 = 0.0, r1 = 0.0, r2 = 0.0;
    for (int q = rp[s]; q < rp[s + 1]; ++q) {
      const double* b = val + (int64_t)q * 9;
      r0 += fabs(b[0]) + fabs(b[1]) + fabs(b[2]);
      r1 += fabs(b[3]) + fabs(b[4]) + fabs(b[5]);
      r2 += fabs(b[6]) + fabs(b[7]) + fabs(b[8]);
    }
    m = fmax(m, fmax(r0, fmax(r1, r2)));
  }
  sh[threadIdx.x] = m;
  __syncthreads();
  for (int o = kT / 2; o > 0; o >>= 1) {
    if (threadIdx.x < o) sh[threadIdx.x] = fmax(sh[threadIdx.x], sh[threadIdx.x + o]);
    __syncthreads();
  }
  if (threadIdx.x == 0) part[blockIdx.x] = sh[0];
}

int trunc_rank(const std::vector<double>& ev, double delta2, int cap) {
  const int n = (int)ev.size();
  std::vector<double> tail(n + 1, 0.0);
  for (int i = n - 1; i >= 0; --i) tail[i] = tail[i + 1] + std::max(ev[i], 0.0);
  int r = n;
  for (int l = 1; l <= n; ++l)
    if (tail[l] <= delta2) { r = l; break; }
  r = std::max(r, 1);
  return std::min(r, cap);
}

// Host-side handle to a QTT on the device (FP64 cores).
struct DQtt {
  int d = 0;
  std::vector<int32_t> r;     // d + 1
  std::vector<int64_t> off;   // d + 1
  DevBuf buf;
  double* core(int k) const { return buf.as<double>() + off[k]; }  // 0-based
  void alloc(int d_, const std::vector<int32_t>& ranks) {
    d = d_;
    r = ranks;
    off.assign(d + 1, 0);
    for (int k = 0; k < d; ++k) off[k + 1] = off[k] + (int64_t)r[k] * 4 * r[k + 1];
    buf.ensure(sizeof(double) * (size_t)std::max<int64_t>(off[d], 1));
  }
};

void copy_into(hipStream_t s, const DQtt& src, Qtt& dst) {
  dst.d = src.d;
  dst.ranks = src.r;
  const int64_t tot = src.off[src.d];
  dst.cores.ensure(sizeof(double) * tot);
  QTP_HIP(hipMemcpyAsync(dst.cores.get(), src.buf.get(), sizeof(double) * tot,
                         hipMemcpyDeviceToDevice, s));
  dst.lp_prec = 0;
}

void load_from(hipStream_t s, const Qtt& src, DQtt& dst) {
  dst.alloc(src.d, src.ranks);
  QTP_HIP(hipMemcpyAsync(dst.buf.get(), src.cores.get(),
                         sizeof(double) * dst.off[dst.d], hipMemcpyDeviceToDevice, s));
}

// Scratch shared by the construction steps.  It lives as long as the
// context, so the buffers only grow: no allocation (and no hipFree, which
// synchronises the device) in steady state.
struct Scratch {
  DevBuf gram, evA, evV, evw, evws, evVs, gemm_ws, t1, t2, t3, partial;
  DevBuf z1, z2, y1, y2;
  // rounding
  DevBuf Wb, Wn, Bb, T2, Mm;
  std::vector<DevBuf> zc;
  // compression
  DevBuf W, Pm, Wp;
  std::vector<DevBuf> cores;
  // pattern
  DevBuf brow, tk, tv, th, ts, flag, excl, g;
  // Newton-Schulz iterates
  DQtt A, X, AX, Y, XY, T, Xn, bestX;
  Workspace ws() { return Workspace{gemm_ws.get(), gemm_ws.bytes()}; }
};

__global__ void set_value_kernel(double* __restrict__ p, double v) {
  if (threadIdx.x == 0) p[0] = v;
}

void set_value(hipStream_t s, double* p, double v) {
  set_value_kernel<<<1, 64, 0, s>>>(p, v);
  QTP_CHECK_LAUNCH();
}

double host_sum(hipStream_t s, const double* partial, int n) {
  std::vector<double> h(n);
  QTP_HIP(hipMemcpyAsync(h.data(), partial, sizeof(double) * n,
                         hipMemcpyDeviceToHost, s));
  QTP_HIP(hipStreamSynchronize(s));
  double t = 0.0;
  for (double v : h) t += v;
  return t;
}

// Eigen-decomposition of the symmetric c x c matrix at `M` (destroyed);
// returns the eigenvalues (host, decreasing) and leaves the sorted
// eigenvectors (columns) in sc.evVs.
std::vector<double> eig_host(hipStream_t s, int c, double* M, Scratch& sc) {
  sc.evV.ensure(sizeof(double) * c * c);
  sc.evw.ensure(sizeof(double) * c);
  sc.evws.ensure(sizeof(double) * c);
  sc.evVs.ensure(sizeof(double) * c * c);
  sym_eig(s, c, M, sc.evV.as<double>(), sc.evw.as<double>(), sc.evws.as<double>(),
          sc.evVs.as<double>());
  std::vector<double> ev(c);
  QTP_HIP(hipMemcpyAsync(ev.data(), sc.evws.get(), sizeof(double) * c,
                         hipMemcpyDeviceToHost, s));
  QTP_HIP(hipStreamSynchronize(s));
  return ev;
}

// TT rounding of Y into Z with per-bond tolerance eps |Y| / sqrt(d-1) and
// rank cap rmax.  Returns |Y|_F.
double tt_round(hipStream_t s, const DQtt& Y, double eps, int rmax, DQtt& Z,
                Scratch& sc) {
  const int d = Y.d;
  const auto& R = Y.r;
  // right Gram matrices G_k (bond k between cores k and k+1, 1-based k),
  // G_d = [1]; G_{k-1} = sum_b Y_k[:,b,:] G_k Y_k[:,b,:]^T
  std::vector<int64_t> goff(d + 1, 0);
  for (int k = 0; k < d; ++k) goff[k + 1] = goff[k] + (int64_t)R[k] * R[k];
  sc.gram.ensure(sizeof(double) * (size_t)(goff[d] + 1));
  double* G = sc.gram.as<double>();
  auto Gk = [&](int k) { return G + goff[k]; };  // R[k] x R[k]
  set_value(s, Gk(d), 1.0);
  int64_t maxT = 1;
  for (int k = 1; k <= d; ++k) maxT = std::max<int64_t>(maxT, (int64_t)R[k - 1] * 4 * R[k]);
  sc.t1.ensure(sizeof(double) * maxT);
  Workspace ws = sc.ws();
  for (int k = d; k >= 1; --k) {
    const double* Yk = Y.core(k - 1);
    double* T = sc.t1.as<double>();
    // T[(a,b)][c] = sum_e Y_k[(a,b)][e] G_k[e][c]
    gemm(s, 0, 0, 4 * R[k - 1], R[k], R[k], 1.0, Yk, R[k], Gk(k), R[k], 0.0, T,
         R[k], &ws);
    // G_{k-1}[a][a'] = sum_{(b,c)} T[a][(b,c)] Y_k[a'][(b,c)]
    gemm(s, 0, 1, R[k - 1], R[k - 1], 4 * R[k], 1.0, T, 4 * R[k], Yk, 4 * R[k],
         0.0, Gk(k - 1), R[k - 1], &ws);
  }
  double nrm2 = 0.0;
  QTP_HIP(hipMemcpyAsync(&nrm2, Gk(0), sizeof(double), hipMemcpyDeviceToHost, s));
  QTP_HIP(hipStreamSynchronize(s));
  const double nrm = std::sqrt(std::max(nrm2, 0.0));
  const double delta2 = eps * eps * nrm2 / std::max(d - 1, 1);
  // left-to-right truncation
  std::vector<int32_t> rz(d + 1, 1);
  if ((int)sc.zc.size() < d) sc.zc.resize(d);
  std::vector<DevBuf>& zc = sc.zc;
  int64_t maxW = 1;
  for (int k = 0; k <= d; ++k) maxW = std::max<int64_t>(maxW, (int64_t)R[k] * 256);
  DevBuf &Wb = sc.Wb, &Wn = sc.Wn, &Bb = sc.Bb, &T2 = sc.T2, &Mm = sc.Mm;
  Wb.ensure(sizeof(double) * maxW);
  Wn.ensure(sizeof(double) * maxW);
  set_value(s, Wb.as<double>(), 1.0);
  int rp = 1;  // current left rank r'_{k-1}
  for (int k = 1; k <= d; ++k) {
    const double* Yk = Y.core(k - 1);
    // B = W Y_k : (rp x R_{k-1}) (R_{k-1} x 4 R_k)
    Bb.ensure(sizeof(double) * (size_t)rp * 4 * R[k]);
    gemm(s, 0, 0, rp, 4 * R[k], R[k - 1], 1.0, Wb.as<double>(), R[k - 1], Yk,
         4 * R[k], 0.0, Bb.as<double>(), 4 * R[k], &ws);
    if (k == d) {
      zc[k - 1].ensure(sizeof(double) * rp * 4);
      QTP_HIP(hipMemcpyAsync(zc[k - 1].get(), Bb.get(), sizeof(double) * rp * 4,
                             hipMemcpyDeviceToDevice, s));
      rz[k - 1] = rp;
      break;
    }
    const int c = 4 * rp;
    // M = B G_k B^T with B viewed as c x R_k
    T2.ensure(sizeof(double) * (size_t)c * R[k]);
    gemm(s, 0, 0, c, R[k], R[k], 1.0, Bb.as<double>(), R[k], Gk(k), R[k], 0.0,
         T2.as<double>(), R[k], &ws);
    Mm.ensure(sizeof(double) * (size_t)c * c);
    gemm(s, 0, 1, c, c, R[k], 1.0, T2.as<double>(), R[k], Bb.as<double>(), R[k],
         0.0, Mm.as<double>(), c, &ws);
    std::vector<double> ev = eig_host(s, c, Mm.as<double>(), sc);
    const int rk = trunc_rank(ev, delta2, std::min(rmax, std::min(c, (int)R[k])));
    // core_k[(a,b)][beta] = U[(a,b)][beta], beta < rk
    zc[k - 1].ensure(sizeof(double) * (size_t)c * rk);
    take_columns_kernel<<<div_up((int64_t)c * rk, kT), kT, 0, s>>>(
        c, rk, sc.evVs.as<double>(), zc[k - 1].as<double>());
    QTP_CHECK_LAUNCH();
    // W = U_r^T B : (rk x c)(c x R_k)
    gemm(s, 1, 0, rk, R[k], c, 1.0, zc[k - 1].as<double>(), rk, Bb.as<double>(),
         R[k], 0.0, Wn.as<double>(), R[k], &ws);
    Wb.swap(Wn);
    rz[k - 1] = rp;
    rz[k] = rk;
    rp = rk;
  }
  rz[0] = 1;
  rz[d] = 1;
  Z.alloc(d, rz);
  for (int k = 0; k < d; ++k)
    QTP_HIP(hipMemcpyAsync(Z.core(k), zc[k].get(),
                           sizeof(double) * (size_t)rz[k] * 4 * rz[k + 1],
                           hipMemcpyDeviceToDevice, s));
  return nrm;
}

void tt_matmul(hipStream_t s, const DQtt& A, const DQtt& B, DQtt& C) {
  std::vector<int32_t> rc(A.d + 1);
  for (int k = 0; k <= A.d; ++k) rc[k] = A.r[k] * B.r[k];
  C.alloc(A.d, rc);
  for (int k = 0; k < A.d; ++k) {
    const int64_t tot = (int64_t)rc[k] * 4 * rc[k + 1];
    tt_matmul_core_kernel<<<div_up(tot, kT), kT, 0, s>>>(
        A.r[k], A.r[k + 1], B.r[k], B.r[k + 1], A.core(k), B.core(k), C.core(k));
    QTP_CHECK_LAUNCH();
  }
}

void tt_axpby(hipStream_t s, double alpha, const DQtt& A, double beta,
              const DQtt& B, DQtt& C) {
  const int d = A.d;
  std::vector<int32_t> rc(d + 1);
  rc[0] = rc[d] = 1;
  for (int k = 1; k < d; ++k) rc[k] = A.r[k] + B.r[k];
  C.alloc(d, rc);
  for (int k = 0; k < d; ++k) {
    const int64_t tot = (int64_t)rc[k] * 4 * rc[k + 1];
    tt_add_core_kernel<<<div_up(tot, kT), kT, 0, s>>>(
        A.r[k], A.r[k + 1], B.r[k], B.r[k + 1], k == 0, k == d - 1, alpha, beta,
        A.core(k), B.core(k), C.core(k));
    QTP_CHECK_LAUNCH();
  }
}

void scaled_identity(hipStream_t s, int d, double a, DQtt& X) {
  X.alloc(d, std::vector<int32_t>(d + 1, 1));
  for (int k = 0; k < d; ++k) {
    fill_identity_core_kernel<<<1, 64, 0, s>>>(X.core(k), k == 0 ? a : 1.0);
    QTP_CHECK_LAUNCH();
  }
}

struct Builder {
  Ctx& c;
  Scratch sc;
  explicit Builder(Ctx& ctx) : c(ctx) {
    sc.gemm_ws.ensure(sizeof(double) * ((size_t)8 << 20));  // split-K partials
  }

  // ---- pattern (z-order) of the scaled matrix ----------------------------
  void build_pattern() {
    auto& P = c.pat;
    const hipStream_t s = c.stream;
    const int d = c.log2n;
    const int64_t nval = 9 * c.nnzb;
    const int64_t ntail = c.n - 3 * (int64_t)c.nslots;
    const int64_t nent = nval + ntail;
    QTP_REQUIRE(nent < (int64_t)INT32_MAX, QTP_E_CAPACITY, "too many non-zeros");
    P.d = d;
    P.nent = nent;
    P.nval = nval;
    P.keys.ensure(sizeof(uint64_t) * nent);
    P.perm.ensure(sizeof(int32_t) * nent);
    DevBuf& brow = sc.brow;
    brow.ensure(sizeof(int32_t) * (size_t)std::max<int64_t>(c.nnzb, 1));
    block_rows_kernel<<<div_up(c.nslots, kT), kT, 0, s>>>(c.nslots, c.rp.as<int32_t>(),
                                                         brow.as<int32_t>());
    QTP_CHECK_LAUNCH();
    entry_keys_kernel<<<div_up(nent, kT), kT, 0, s>>>(
        c.nnzb, c.nslots, c.n, brow.as<int32_t>(), c.col.as<int32_t>(),
        P.keys.as<uint64_t>(), P.perm.as<int32_t>());
    QTP_CHECK_LAUNCH();
    DevBuf &tk = sc.tk, &tv = sc.tv, &th = sc.th, &ts = sc.ts;
    radix_sort_pairs(s, P.keys.as<uint64_t>(), P.perm.as<int32_t>(), nent, 2 * d,
                     tk, tv, th, ts);
    // level structure: rows of W_k are distinct prefixes z >> 2(d-k+1)
    P.nrows.assign(d + 1, 0);
    P.seg.resize(d + 1);
    P.rowkey.resize(d + 1);
    DevBuf &flag = sc.flag, &excl = sc.excl;
    // leaves (k = d): segments of z >> 2 over the sorted entries
    int64_t cur_n = nent;
    const uint64_t* cur_keys = P.keys.as<uint64_t>();
    for (int k = d; k >= 1; --k) {
      flag.ensure(sizeof(int) * cur_n);
      excl.ensure(sizeof(int) * cur_n);
      head_flags_kernel<<<div_up(cur_n, kT), kT, 0, s>>>(cur_keys, cur_n, 2,
                                                          flag.as<int>());
      QTP_CHECK_LAUNCH();
      exclusive_scan(s, flag.as<int>(), excl.as<int>(), cur_n, ts);
      int last_ex = 0, last_f = 0;
      QTP_HIP(hipMemcpyAsync(&last_ex, excl.as<int>() + cur_n - 1, sizeof(int),
                             hipMemcpyDeviceToHost, s));
      QTP_HIP(hipMemcpyAsync(&last_f, flag.as<int>() + cur_n - 1, sizeof(int),
                             hipMemcpyDeviceToHost, s));
      QTP_HIP(hipStreamSynchronize(s));
      const int64_t nrows = (int64_t)last_ex + last_f;
      P.nrows[k] = nrows;
      P.seg[k].ensure(sizeof(int32_t) * cur_n);
      P.rowkey[k].ensure(sizeof(uint64_t) * nrows);
      seg_ids_kernel<<<div_up(cur_n, kT), kT, 0, s>>>(
          cur_keys, cur_n, 2, flag.as<int>(), excl.as<int>(), P.seg[k].as<int32_t>(),
          P.rowkey[k].as<uint64_t>());
      QTP_CHECK_LAUNCH();
      // P.seg[k] maps the items of the finer level (entries for k = d, rows
      // of W_{k+1} otherwise) to rows of W_k
      cur_keys = P.rowkey[k].as<uint64_t>();
      cur_n = nrows;
    }
    QTP_HIP(hipStreamSynchronize(s));
    QTP_REQUIRE(P.nrows[1] == 1, QTP_E_STATE, "pattern: root level must be one block");
    P.valid = true;
  }

  // ---- compression of the scaled matrix (values in c.sval) ----------------
  void compress(double eps, int rmax, DQtt& A) {
    auto& P = c.pat;
    const hipStream_t s = c.stream;
    const int d = c.log2n;
    Workspace ws = sc.ws();
    // leaves
    DevBuf &W = sc.W, &Pm = sc.Pm, &Wp = sc.Wp;
    W.ensure(sizeof(double) * 4 * P.nrows[d]);
    QTP_HIP(hipMemsetAsync(W.get(), 0, sizeof(double) * 4 * P.nrows[d], s));
    fill_leaves_kernel<<<div_up(P.nent, kT), kT, 0, s>>>(
        P.nent, P.nval, P.keys.as<uint64_t>(), P.perm.as<int32_t>(),
        P.seg[d].as<int32_t>(), c.sval.as<double>(), W.as<double>());
    QTP_CHECK_LAUNCH();
    sc.partial.ensure(sizeof(double) * 1024);
    const int nb = (int)std::min<int64_t>(1024, div_up(4 * P.nrows[d], kT));
    sumsq_kernel<<<nb, kT, 0, s>>>(W.as<double>(), 4 * P.nrows[d],
                                   sc.partial.as<double>());
    QTP_CHECK_LAUNCH();
    const double nrm2 = host_sum(s, sc.partial.as<double>(), nb);
    const double delta2 = eps * eps * nrm2 / std::max(d - 1, 1);
    std::vector<int32_t> r(d + 1, 1);
    if ((int)sc.cores.size() < d) sc.cores.resize(d);
    std::vector<DevBuf>& cores = sc.cores;
    int rk = 1;  // r_k of the current level's right part
    for (int k = d; k >= 2; --k) {
      const int cols = 4 * rk;
      const int64_t nrows = P.nrows[k];
      sc.gram.ensure(sizeof(double) * cols * cols);
      gemm(s, 1, 0, cols, cols, (int)nrows, 1.0, W.as<double>(), cols,
           W.as<double>(), cols, 0.0, sc.gram.as<double>(), cols, &ws);
      std::vector<double> ev = eig_host(s, cols, sc.gram.as<double>(), sc);
      const int cap = (int)std::min<int64_t>(std::min<int64_t>(rmax, cols), nrows);
      const int rn = trunc_rank(ev, delta2, cap);
      // core_k[a][(b, beta)] = V[(b, beta)][a]
      cores[k - 1].ensure(sizeof(double) * (size_t)rn * cols);
      take_columns_T_kernel<<<div_up((int64_t)rn * cols, kT), kT, 0, s>>>(
          cols, rn, sc.evVs.as<double>(), cores[k - 1].as<double>());
      QTP_CHECK_LAUNCH();
      // projected rows: Pm = W V_r  (nrows x rn), V_r = first rn columns
      sc.t3.ensure(sizeof(double) * (size_t)cols * rn);
      take_columns_kernel<<<div_up((int64_t)cols * rn, kT), kT, 0, s>>>(
          cols, rn, sc.evVs.as<double>(), sc.t3.as<double>());
      QTP_CHECK_LAUNCH();
      Pm.ensure(sizeof(double) * (size_t)nrows * rn);
      gemm(s, 0, 0, (int)nrows, rn, cols, 1.0, W.as<double>(), cols,
           sc.t3.as<double>(), rn, 0.0, Pm.as<double>(), rn, nullptr);
      // parents
      const int64_t np = P.nrows[k - 1];
      Wp.ensure(sizeof(double) * (size_t)np * 4 * rn);
      QTP_HIP(hipMemsetAsync(Wp.get(), 0, sizeof(double) * (size_t)np * 4 * rn, s));
      scatter_parent_kernel<<<div_up(nrows * rn, kT), kT, 0, s>>>(
          nrows, rn, P.seg[k - 1].as<int32_t>(), P.rowkey[k].as<uint64_t>(),
          Pm.as<double>(), Wp.as<double>());
      QTP_CHECK_LAUNCH();
      W.swap(Wp);
      r[k - 1] = rn;
      rk = rn;
    }
    // core_1 = W_1 (1 x 4 r_1)
    cores[0].ensure(sizeof(double) * 4 * rk);
    QTP_HIP(hipMemcpyAsync(cores[0].get(), W.get(), sizeof(double) * 4 * rk,
                           hipMemcpyDeviceToDevice, s));
    A.alloc(d, r);
    for (int k = 0; k < d; ++k)
      QTP_HIP(hipMemcpyAsync(A.core(k), cores[k].get(),
                             sizeof(double) * (size_t)r[k] * 4 * r[k + 1],
                             hipMemcpyDeviceToDevice, s));
  }

  // probe residual max_z |z - S~ X z| / |z| with the exact scaled matrix
  double probe(const DQtt& X) {
    const hipStream_t s = c.stream;
    const int64_t n = c.n;
    sc.z1.ensure(sizeof(double) * n);
    sc.z2.ensure(sizeof(double) * n);
    sc.y1.ensure(sizeof(double) * n);
    sc.y2.ensure(sizeof(double) * n);
    probe_kernel<<<div_up(n, kT), kT, 0, s>>>(n, sc.z1.as<double>(), sc.z2.as<double>());
    QTP_CHECK_LAUNCH();
    c.qtt_work.ensure(qtt_apply_workspace(X.d, X.r.data(), 0));
    double worst = 0.0;
    for (int t = 0; t < 2; ++t) {
      double* z = (t == 0 ? sc.z1 : sc.z2).as<double>();
      qtt_apply(s, X.d, X.r.data(), X.buf.get(), 0, z, sc.y1.as<double>(),
                c.qtt_work.get());
      bsr_spmv(s, c.nslots, n, c.rp.as<int32_t>(), c.col.as<int32_t>(),
               c.sval.as<double>(), sc.y1.as<double>(), sc.y2.as<double>());
      sub(s, z, sc.y2.as<double>(), sc.y2.as<double>(), n);
      sc.partial.ensure(sizeof(double) * 1024);
      const int nb = (int)std::min<int64_t>(1024, div_up(n, kT));
      sumsq_kernel<<<nb, kT, 0, s>>>(sc.y2.as<double>(), n, sc.partial.as<double>());
      QTP_CHECK_LAUNCH();
      const double rr = host_sum(s, sc.partial.as<double>(), nb);
      worst = std::max(worst, std::sqrt(rr / (double)n));
    }
    return worst;
  }
};

}  // namespace

struct BuildCache {
  Builder b;
  explicit BuildCache(Ctx& c) : b(c) {}
};

void destroy_build_cache(BuildCache* bc) { delete bc; }

void build_inverse(Ctx& c, int hot) {
  QTP_REQUIRE(c.have_matrix, QTP_E_STATE, "no Newton matrix loaded");
  const hipStream_t s = c.stream;
  // scaled matrix S~ = L^-1 S L^-T
  c.sval.ensure(sizeof(double) * 9 * (size_t)c.nnzb);
  bj_scale_matrix(s, c.nslots, c.rp.as<int32_t>(), c.col.as<int32_t>(),
                  c.val.as<double>(), c.Linv.as<double>(), c.sval.as<double>());
  if (!c.bcache) c.bcache = new BuildCache(c);
  Builder& b = c.bcache->b;
  Scratch& sc = b.sc;
  if (!c.pat.valid || c.pat.d != c.log2n) b.build_pattern();
  DQtt& A = sc.A;
  b.compress(c.cfg.qtt_eps, c.cfg.qtt_rmax_s, A);
  copy_into(s, A, c.A);
  // Newton-Schulz on S~_TT with probe monitoring on the exact S~
  const int d = c.log2n;
  DQtt& X = sc.X;
  int iters = c.cfg.ns_iters;
  if (hot && c.have_inverse && c.X.d == d) {
    load_from(s, c.X, X);
    iters = c.cfg.ns_iters_hot;
  } else {
    const int nb = std::max(1, std::min(1024, div_up(c.nslots, kT)));
    sc.partial.ensure(sizeof(double) * 1024);
    gershgorin_kernel<<<nb, kT, 0, s>>>(c.nslots, c.rp.as<int32_t>(), c.sval.as<double>(),
                                        sc.partial.as<double>());
    QTP_CHECK_LAUNCH();
    std::vector<double> hp(nb);
    QTP_HIP(hipMemcpyAsync(hp.data(), sc.partial.get(), sizeof(double) * nb,
                           hipMemcpyDeviceToHost, s));
    QTP_HIP(hipStreamSynchronize(s));
    const double lam = *std::max_element(hp.begin(), hp.end());
    scaled_identity(s, d, 1.0 / lam, X);
  }
  double best = b.probe(X);
  DQtt& bestX = sc.bestX;
  bestX.alloc(d, X.r);
  QTP_HIP(hipMemcpyAsync(bestX.buf.get(), X.buf.get(), sizeof(double) * X.off[d],
                         hipMemcpyDeviceToDevice, s));
  c.ns_done = 0;
  for (int it = 0; it < iters; ++it) {
    DQtt &AX = sc.AX, &Y = sc.Y, &XY = sc.XY, &T = sc.T, &Xn = sc.Xn;
    tt_matmul(s, A, X, AX);
    tt_round(s, AX, c.cfg.qtt_eps, c.cfg.qtt_rmax_s, Y, sc);
    tt_matmul(s, X, Y, XY);
    tt_axpby(s, 2.0, X, -1.0, XY, T);
    tt_round(s, T, c.cfg.qtt_eps, c.cfg.qtt_rmax, Xn, sc);
    const double pr = b.probe(Xn);
    X.buf.swap(Xn.buf);
    std::swap(X.r, Xn.r);
    std::swap(X.off, Xn.off);
    ++c.ns_done;
    if (!(pr < best)) break;  // no progress on the exact matrix: keep the best
    best = pr;
    bestX.alloc(d, X.r);
    QTP_HIP(hipMemcpyAsync(bestX.buf.get(), X.buf.get(), sizeof(double) * X.off[d],
                           hipMemcpyDeviceToDevice, s));
  }
  copy_into(s, bestX, c.X);
  QTP_HIP(hipStreamSynchronize(s));
  c.probe_residual = best;
  c.have_inverse = true;
}

}  // namespace qtp
