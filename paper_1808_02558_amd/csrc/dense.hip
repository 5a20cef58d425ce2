// Dense building blocks of the QTT construction: an FP64 GEMM (with split-K
// for the tall-skinny Gram products), a symmetric Jacobi eigensolver for the
// small matrices whose eigenvectors become TT cores, an exclusive scan and a
// stable LSD radix sort of 64-bit keys.
#include "dense.h"

namespace qtp {
namespace {

// ---------------------------------------------------------------------------
// GEMM: C[M x N] = alpha * op(A) op(B) + beta * C, row-major, FP64.
// 64 x 64 output tile per 256-thread block, 4 x 4 outputs per thread,
// K staged through LDS in slices of 16.  Split-K: blockIdx.z takes a K range
// and writes its partial to Cpart[z][M][N] (beta ignored), reduced in order
// afterwards.
// ---------------------------------------------------------------------------
constexpr int TM = 64, TN = 64, TK = 16;

__global__ __launch_bounds__(256) void gemm_kernel(
    int transA, int transB, int M, int N, int K, int kchunk, double alpha,
    const double* __restrict__ A, int64_t lda, const double* __restrict__ B,
    int64_t ldb, double beta, double* __restrict__ C, int64_t ldc,
    int partial_mode) {
  __shared__ double As[TK][TM + 1];
  __shared__ double Bs[TK][TN + 1];
  const int tx = threadIdx.x & 15, ty = threadIdx.x >> 4;
  const int m0 = blockIdx.x * TM, n0 = blockIdx.y * TN;
  const int kbeg = blockIdx.z * kchunk;
  const int kend = min(K, kbeg + kchunk);
  double acc[4][4] = {};
  for (int k0 = kbeg; k0 < kend; k0 += TK) {
    // load A tile: TM x TK elements, 256 threads -> 4 each
    for (int e = threadIdx.x; e < TM * TK; e += 256) {
      int mm, kk;
      if (!transA) { mm = e / TK; kk = e % TK; } else { kk = e / TM; mm = e % TM; }
      const int gm = m0 + mm, gk = k0 + kk;
      double v = 0.0;
      if (gm < M && gk < kend)
        v = transA ? A[(int64_t)gk * lda + gm] : A[(int64_t)gm * lda + gk];
      As[kk][mm] = v;
    }
    for (int e = threadIdx.x; e < TK * TN; e += 256) {
      int kk, nn;
      if (!transB) { kk = e / TN; nn = e % TN; } else { nn = e / TK; kk = e % TK; }
      const int gn = n0 + nn, gk = k0 + kk;
      double v = 0.0;
      if (gn < N && gk < kend)
        v = transB ? B[(int64_t)gn * ldb + gk] : B[(int64_t)gk * ldb + gn];
      Bs[kk][nn] = v;
    }
    __syncthreads();
#pragma unroll
    for (int kk = 0; kk < TK; ++kk) {
      double a[4], b[4];
#pragma unroll
      for (int i = 0; i < 4; ++i) a[i] = As[kk][ty + 16 * i];
#pragma unroll
      for (int j = 0; j < 4; ++j) b[j] = Bs[kk][tx + 16 * j];
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) acc[i][j] += a[i] * b[j];
    }
    __syncthreads();
  }
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const int gm = m0 + ty + 16 * i;
    if (gm >= M) continue;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int gn = n0 + tx + 16 * j;
      if (gn >= N) continue;
      if (partial_mode) {
        C[((int64_t)blockIdx.z * M + gm) * N + gn] = acc[i][j];
      } else {
        double* c = C + (int64_t)gm * ldc + gn;
        *c = alpha * acc[i][j] + (beta == 0.0 ? 0.0 : beta * *c);
      }
    }
  }
}

__global__ void splitk_reduce_kernel(int M, int N, int nsplit, double alpha,
                                     const double* __restrict__ part, double beta,
                                     double* __restrict__ C, int64_t ldc) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (int64_t)M * N) return;
  double s = 0.0;
  for (int z = 0; z < nsplit; ++z) s += part[(int64_t)z * M * N + e];
  const int64_t m = e / N, n = e % N;
  double* c = C + m * ldc + n;
  *c = alpha * s + (beta == 0.0 ? 0.0 : beta * *c);
}

// ---------------------------------------------------------------------------
// Symmetric eigensolver: cyclic Jacobi with the round-robin parallel
// ordering (n/2 disjoint rotations per round, n-1 rounds per sweep).  One
// workgroup; A (n x n) and V (n x n) in global memory (L2 resident for the
// sizes used, n <= 256).  Each thread updates whole 2x2 quads of A in place,
// so no double buffer is needed.
// ---------------------------------------------------------------------------
constexpr int kEigThreads = 1024;

__device__ inline int rr_partner(int pos, int round, int n) {
  // position -> player in the round-robin schedule; player 0 fixed
  if (pos == 0) return 0;
  return 1 + (pos - 1 + round) % (n - 1);
}

// NMAX > 0: A (n <= NMAX) is copied into LDS, and V too when V_LDS; the
// rotations then run out of LDS.  NMAX == 0: both stay in global memory.
template <int NMAX, bool V_LDS>
__global__ __launch_bounds__(kEigThreads) void jacobi_eig_kernel(
    int n, double* __restrict__ Ag, double* __restrict__ Vg, double* __restrict__ w,
    int max_sweeps, double tol) {
  __shared__ int pp[128], qq[128];
  __shared__ double cs[128], sn[128];
  __shared__ double red[kEigThreads / 64];
  __shared__ int stop;
  __shared__ double Al[NMAX > 0 ? NMAX * NMAX : 1];
  __shared__ double Vl[V_LDS ? NMAX * NMAX : 1];
  double* A = NMAX > 0 ? Al : Ag;
  double* V = V_LDS ? Vl : Vg;
  const int tid = threadIdx.x;
  const int half = n / 2;
  if (NMAX > 0)
    for (int e = tid; e < n * n; e += kEigThreads) Al[e] = Ag[e];
  for (int e = tid; e < n * n; e += kEigThreads)
    V[e] = (e / n == e % n) ? 1.0 : 0.0;
  __syncthreads();
  for (int sweep = 0; sweep < max_sweeps; ++sweep) {
    // convergence test: off-diagonal vs total Frobenius norm
    double off = 0.0, tot = 0.0;
    for (int e = tid; e < n * n; e += kEigThreads) {
      const double a = A[e];
      tot += a * a;
      if (e / n != e % n) off += a * a;
    }
    for (int o = 32; o > 0; o >>= 1) {
      off += __shfl_xor(off, o, 64);
      tot += __shfl_xor(tot, o, 64);
    }
    if ((tid & 63) == 0) red[tid >> 6] = off;
    __syncthreads();
    if (tid == 0) {
      double s = 0.0;
      for (int i = 0; i < kEigThreads / 64; ++i) s += red[i];
      red[0] = s;
    }
    __syncthreads();
    const double offs = red[0];
    __syncthreads();
    if ((tid & 63) == 0) red[tid >> 6] = tot;
    __syncthreads();
    if (tid == 0) {
      double s = 0.0;
      for (int i = 0; i < kEigThreads / 64; ++i) s += red[i];
      stop = (offs <= tol * tol * s) ? 1 : 0;
    }
    __syncthreads();
    if (stop) break;
    for (int round = 0; round < n - 1; ++round) {
      // pairs: (pos k, pos n-1-k)
      if (tid < half) {
        int p = rr_partner(tid, round, n);
        int q = rr_partner(n - 1 - tid, round, n);
        if (p > q) { const int t = p; p = q; q = t; }
        const double app = A[p * n + p], aqq = A[q * n + q], apq = A[p * n + q];
        double c = 1.0, s = 0.0;
        if (apq != 0.0 && fabs(apq) > 1e-300) {
          const double theta = (aqq - app) / (2.0 * apq);
          const double t = (theta >= 0.0 ? 1.0 : -1.0) /
                           (fabs(theta) + sqrt(theta * theta + 1.0));
          c = 1.0 / sqrt(t * t + 1.0);
          s = t * c;
        }
        pp[tid] = p; qq[tid] = q; cs[tid] = c; sn[tid] = s;
      }
      __syncthreads();
      // A <- J^T A J over all quads {p_i, q_i} x {p_j, q_j}
      for (int e = tid; e < half * half; e += kEigThreads) {
        const int bi = e / half, bj = e % half;
        const int pi = pp[bi], qi = qq[bi], pj = pp[bj], qj = qq[bj];
        const double ci = cs[bi], si = sn[bi], cj = cs[bj], sj = sn[bj];
        const double a00 = A[pi * n + pj], a01 = A[pi * n + qj];
        const double a10 = A[qi * n + pj], a11 = A[qi * n + qj];
        // rows: R_i^T B with R = [[c, s], [-s, c]]
        const double b00 = ci * a00 - si * a10, b01 = ci * a01 - si * a11;
        const double b10 = si * a00 + ci * a10, b11 = si * a01 + ci * a11;
        // columns: (.) R_j
        A[pi * n + pj] = cj * b00 - sj * b01;
        A[pi * n + qj] = sj * b00 + cj * b01;
        A[qi * n + pj] = cj * b10 - sj * b11;
        A[qi * n + qj] = sj * b10 + cj * b11;
      }
      // V <- V J
      for (int e = tid; e < n * half; e += kEigThreads) {
        const int r = e / half, b = e % half;
        const int p = pp[b], q = qq[b];
        const double c = cs[b], s = sn[b];
        const double vp = V[r * n + p], vq = V[r * n + q];
        V[r * n + p] = c * vp - s * vq;
        V[r * n + q] = s * vp + c * vq;
      }
      __syncthreads();
    }
  }
  for (int i = tid; i < n; i += kEigThreads) w[i] = A[i * n + i];
  if (V_LDS)
    for (int e = tid; e < n * n; e += kEigThreads) Vg[e] = Vl[e];
}

// order[i] = index of the i-th largest eigenvalue (ties by index)
__global__ void eig_sort_kernel(int n, const double* __restrict__ w,
                                const double* __restrict__ V,
                                double* __restrict__ wsorted,
                                double* __restrict__ Vsorted) {
  for (int i = threadIdx.x; i < n; i += blockDim.x) {
    int rank = 0;
    const double wi = w[i];
    for (int j = 0; j < n; ++j) {
      const double wj = w[j];
      rank += (wj > wi) || (wj == wi && j < i);
    }
    wsorted[rank] = wi;
    for (int r = 0; r < n; ++r) Vsorted[r * n + rank] = V[r * n + i];
  }
}

// ---------------------------------------------------------------------------
// Exclusive scan of int32 (three passes: block sums, scan of sums, apply).
// ---------------------------------------------------------------------------
constexpr int kScanT = 256;
constexpr int kScanItems = 8;
constexpr int kScanTile = kScanT * kScanItems;

__device__ int block_exclusive_scan(int v, int* sh, int* total) {
  const int tid = threadIdx.x;
  sh[tid] = v;
  __syncthreads();
  for (int o = 1; o < kScanT; o <<= 1) {
    const int t = tid >= o ? sh[tid - o] : 0;
    __syncthreads();
    sh[tid] += t;
    __syncthreads();
  }
  const int incl = sh[tid];
  *total = sh[kScanT - 1];
  __syncthreads();
  return incl - v;
}

__global__ void scan_tile_sums(const int* __restrict__ in, int64_t n,
                               int* __restrict__ sums) {
  __shared__ int sh[kScanT];
  const int64_t base = (int64_t)blockIdx.x * kScanTile + threadIdx.x * kScanItems;
  int s = 0;
  for (int i = 0; i < kScanItems; ++i)
    if (base + i < n) s += in[base + i];
  int tot;
  block_exclusive_scan(s, sh, &tot);
  if (threadIdx.x == 0) sums[blockIdx.x] = tot;
}

__global__ void scan_apply(const int* __restrict__ in, int64_t n,
                           const int* __restrict__ offs, int* __restrict__ out) {
  __shared__ int sh[kScanT];
  const int64_t base = (int64_t)blockIdx.x * kScanTile + threadIdx.x * kScanItems;
  int v[kScanItems];
  int s = 0;
  for (int i = 0; i < kScanItems; ++i) {
    v[i] = base + i < n ? in[base + i] : 0;
    s += v[i];
  }
  int tot;
  int ex = block_exclusive_scan(s, sh, &tot) + offs[blockIdx.x];
  for (int i = 0; i < kScanItems; ++i) {
    if (base + i < n) out[base + i] = ex;
    ex += v[i];
  }
}

// ---------------------------------------------------------------------------
// Stable LSD radix sort, 4-bit digits, one element per thread per tile.
// ---------------------------------------------------------------------------
constexpr int kSortT = 256;
constexpr int kBins = 16;

__global__ void radix_hist(const uint64_t* __restrict__ keys, int64_t n, int shift,
                           int ntiles, int* __restrict__ hist) {
  __shared__ int h[kBins];
  if (threadIdx.x < kBins) h[threadIdx.x] = 0;
  __syncthreads();
  const int64_t i = (int64_t)blockIdx.x * kSortT + threadIdx.x;
  if (i < n) atomicAdd(&h[(keys[i] >> shift) & (kBins - 1)], 1);
  __syncthreads();
  if (threadIdx.x < kBins) hist[(int64_t)threadIdx.x * ntiles + blockIdx.x] = h[threadIdx.x];
}

__global__ void radix_scatter(const uint64_t* __restrict__ kin,
                              const int32_t* __restrict__ vin, int64_t n, int shift,
                              int ntiles, const int* __restrict__ offs,
                              uint64_t* __restrict__ kout, int32_t* __restrict__ vout) {
  __shared__ unsigned char dig[kSortT];
  const int64_t i = (int64_t)blockIdx.x * kSortT + threadIdx.x;
  const bool ok = i < n;
  uint64_t k = 0;
  int dg = kBins;  // sentinel for out-of-range
  if (ok) {
    k = kin[i];
    dg = (int)((k >> shift) & (kBins - 1));
  }
  dig[threadIdx.x] = (unsigned char)dg;
  __syncthreads();
  if (!ok) return;
  int rank = 0;
  for (int t = 0; t < (int)threadIdx.x; ++t) rank += dig[t] == dg;
  const int64_t pos = (int64_t)offs[(int64_t)dg * ntiles + blockIdx.x] + rank;
  kout[pos] = k;
  vout[pos] = vin[i];
}

}  // namespace

void gemm(hipStream_t s, int transA, int transB, int M, int N, int K,
          double alpha, const double* A, int64_t lda, const double* B,
          int64_t ldb, double beta, double* C, int64_t ldc, Workspace* ws) {
  if (M <= 0 || N <= 0) return;
  if (K <= 0) {
    // C = beta C
    gemm_kernel<<<dim3(div_up(M, TM), div_up(N, TN), 1), 256, 0, s>>>(
        transA, transB, M, N, 0, 1, alpha, A, lda, B, ldb, beta, C, ldc, 0);
    QTP_CHECK_LAUNCH();
    return;
  }
  const int tiles = div_up(M, TM) * div_up(N, TN);
  int nsplit = 1;
  if (ws && tiles < 256 && K > 4 * TK * 16) {
    nsplit = (int)std::min<int64_t>(div_up(K, 256), 512 / tiles + 1);
    nsplit = std::max(1, std::min(nsplit, 1024));
    const size_t need = sizeof(double) * (size_t)nsplit * M * N;
    if (need > ws->bytes) nsplit = std::max<int64_t>(1, ws->bytes / (sizeof(double) * (size_t)M * N));
  }
  const int kchunk = div_up(div_up(K, nsplit), TK) * TK;
  nsplit = div_up(K, kchunk);
  if (nsplit == 1) {
    gemm_kernel<<<dim3(div_up(M, TM), div_up(N, TN), 1), 256, 0, s>>>(
        transA, transB, M, N, K, kchunk, alpha, A, lda, B, ldb, beta, C, ldc, 0);
    QTP_CHECK_LAUNCH();
    return;
  }
  double* part = static_cast<double*>(ws->ptr);
  gemm_kernel<<<dim3(div_up(M, TM), div_up(N, TN), nsplit), 256, 0, s>>>(
      transA, transB, M, N, K, kchunk, 1.0, A, lda, B, ldb, 0.0, part, N, 1);
  QTP_CHECK_LAUNCH();
  splitk_reduce_kernel<<<div_up((int64_t)M * N, 256), 256, 0, s>>>(
      M, N, nsplit, alpha, part, beta, C, ldc);
  QTP_CHECK_LAUNCH();
}

void sym_eig(hipStream_t s, int n, double* A, double* V, double* w,
             double* wsorted, double* Vsorted) {
  QTP_REQUIRE(n >= 2 && n <= 256 && n % 2 == 0, -1, "sym_eig: n must be even in [2,256]");
  if (n <= 64)
    jacobi_eig_kernel<64, true><<<1, kEigThreads, 0, s>>>(n, A, V, w, 30, 1e-15);
  else if (n <= 128)
    jacobi_eig_kernel<128, false><<<1, kEigThreads, 0, s>>>(n, A, V, w, 30, 1e-15);
  else
    jacobi_eig_kernel<0, false><<<1, kEigThreads, 0, s>>>(n, A, V, w, 30, 1e-15);
  QTP_CHECK_LAUNCH();
  eig_sort_kernel<<<1, 256, 0, s>>>(n, w, V, wsorted, Vsorted);
  QTP_CHECK_LAUNCH();
}

void exclusive_scan(hipStream_t s, const int* in, int* out, int64_t n,
                    DevBuf& tmp) {
  if (n <= 0) return;
  // tile counts of every level of the recursion, all scratch in one buffer
  std::vector<int64_t> lev;
  for (int64_t m = n; m > 1 || lev.empty();) {
    const int64_t nt = (m + kScanTile - 1) / kScanTile;
    lev.push_back(nt);
    if (nt == 1) break;
    m = nt;
  }
  size_t total = 0;
  for (int64_t nt : lev) total += 2 * (size_t)nt;
  tmp.ensure(sizeof(int) * (total + 2));
  std::vector<int*> sums(lev.size()), offs(lev.size());
  {
    int* p = tmp.as<int>();
    for (size_t l = 0; l < lev.size(); ++l) {
      sums[l] = p;
      offs[l] = p + lev[l];
      p += 2 * lev[l];
    }
  }
  // up: tile sums of each level
  const int* cur = in;
  int64_t cur_n = n;
  for (size_t l = 0; l < lev.size(); ++l) {
    scan_tile_sums<<<(int)lev[l], kScanT, 0, s>>>(cur, cur_n, sums[l]);
    QTP_CHECK_LAUNCH();
    cur = sums[l];
    cur_n = lev[l];
  }
  // down: the top level has one tile, offset 0
  QTP_HIP(hipMemsetAsync(offs.back(), 0, sizeof(int), s));
  for (size_t l = lev.size() - 1; l-- > 0;) {
    scan_apply<<<(int)lev[l + 1], kScanT, 0, s>>>(sums[l], lev[l], offs[l + 1], offs[l]);
    QTP_CHECK_LAUNCH();
  }
  scan_apply<<<(int)lev[0], kScanT, 0, s>>>(in, n, offs[0], out);
  QTP_CHECK_LAUNCH();
}

void radix_sort_pairs(hipStream_t s, uint64_t* keys, int32_t* vals, int64_t n,
                      int key_bits, DevBuf& tmp_keys, DevBuf& tmp_vals,
                      DevBuf& tmp_hist, DevBuf& tmp_scan) {
  if (n <= 1) return;
  const int ntiles = div_up(n, kSortT);
  tmp_keys.ensure(sizeof(uint64_t) * n);
  tmp_vals.ensure(sizeof(int32_t) * n);
  tmp_hist.ensure(sizeof(int) * 2 * (size_t)kBins * ntiles);
  int* hist = tmp_hist.as<int>();
  int* offs = hist + (size_t)kBins * ntiles;
  uint64_t* ka = keys;
  int32_t* va = vals;
  uint64_t* kb = tmp_keys.as<uint64_t>();
  int32_t* vb = tmp_vals.as<int32_t>();
  int passes = 0;
  for (int shift = 0; shift < key_bits; shift += 4) {
    radix_hist<<<ntiles, kSortT, 0, s>>>(ka, n, shift, ntiles, hist);
    QTP_CHECK_LAUNCH();
    exclusive_scan(s, hist, offs, (int64_t)kBins * ntiles, tmp_scan);
    radix_scatter<<<ntiles, kSortT, 0, s>>>(ka, va, n, shift, ntiles, offs, kb, vb);
    QTP_CHECK_LAUNCH();
    std::swap(ka, kb);
    std::swap(va, vb);
    ++passes;
  }
  if (passes & 1) {
    QTP_HIP(hipMemcpyAsync(keys, ka, sizeof(uint64_t) * n, hipMemcpyDeviceToDevice, s));
    QTP_HIP(hipMemcpyAsync(vals, va, sizeof(int32_t) * n, hipMemcpyDeviceToDevice, s));
  }
}

}  // namespace qtp
