// Assembly of the QP data of Sec. 2.3 on the slot layout:
//   N = D^T M^-1 D,  r = b + D^T M^-1 k,  b_i = [Phi_i / h, 0, 0],
//   k = M v + h f  (so D^T M^-1 k = D^T (v + h M^-1 f)),
// in scaled units (N * m_bar, r / (g h)).  D_i maps the impulses of contact
// i (along n, t1, t2) to the forces and torques on its bodies (Sec. 2.2):
// the body the normal points to (sphere b of a pair, the sphere of a wall
// contact) gets [c ; -r (n x c)], the other sphere [-c ; -r (n x c)].
// Spheres: M = diag(m I_3, (2/5) m r^2 I_3); walls are static.
//
// Block (i, j) of N is non-zero iff contacts i and j share a body (Sec. 3.3):
// the block row of slot s_i lists the contacts incident to i's bodies, merged
// in slot order (the incidence is sorted by body, then slot), each block
// summing the shared bodies' terms.  Slots follow the contact order unless
// persistent slots are kept across time steps.
#include <cmath>

#include "dense.h"
#include "timestep.h"

namespace qtp {
namespace {

constexpr int kT = 256;

// incidence entries: key = (body << sbits) | slot, value = (contact << 1) |
// is_role_A
__global__ void incidence_kernel(int nc, int M, int sbits, const int32_t* __restrict__ a,
                                 const int32_t* __restrict__ b,
                                 const int32_t* __restrict__ slot,
                                 const int32_t* __restrict__ offs,
                                 uint64_t* __restrict__ key, int32_t* __restrict__ val) {
  const int i = blockIdx.x * kT + threadIdx.x;
  if (i >= nc) return;
  const bool wall = b[i] >= M;
  int w = offs[i];
  const int bodyB = wall ? a[i] : b[i];
  const uint64_t sl = (uint64_t)slot[i];
  key[w] = ((uint64_t)bodyB << sbits) | sl;
  val[w] = i << 1;
  if (!wall) {
    key[w + 1] = ((uint64_t)a[i] << sbits) | sl;
    val[w + 1] = (i << 1) | 1;
  }
}

__global__ void entries_per_contact_kernel(int nc, int M, const int32_t* __restrict__ b,
                                           int* __restrict__ cnt) {
  const int i = blockIdx.x * kT + threadIdx.x;
  if (i < nc) cnt[i] = b[i] >= M ? 1 : 2;
}

__global__ void body_ptr_kernel(int nent, int M, int sbits, const uint64_t* __restrict__ key,
                                int32_t* __restrict__ ptr) {
  // ptr[body] = first entry of body; ptr[M] = nent (bodies without entries
  // get the start of the next body with entries, filled by a backward pass)
  const int e = blockIdx.x * kT + threadIdx.x;
  if (e >= nent) return;
  const int bk = (int)(key[e] >> sbits);
  if (e == 0 || (int)(key[e - 1] >> sbits) != bk) {
    const int prev = e == 0 ? -1 : (int)(key[e - 1] >> sbits);
    for (int q = prev + 1; q <= bk; ++q) ptr[q] = e;
  }
  if (e == nent - 1)
    for (int q = bk + 1; q <= M; ++q) ptr[q] = nent;
}

__global__ void inv_slot_kernel(int nc, const int32_t* __restrict__ slot,
                                int32_t* __restrict__ inv) {
  const int i = blockIdx.x * kT + threadIdx.x;
  if (i < nc) inv[slot[i]] = i;
}

__device__ inline int body_B(int i, int M, const int32_t* a, const int32_t* b) {
  return b[i] >= M ? a[i] : b[i];
}
__device__ inline int body_A(int i, int M, const int32_t* a, const int32_t* b) {
  return b[i] >= M ? -1 : a[i];
}

__global__ void row_counts_kernel(int nslots, int M, const int32_t* __restrict__ inv,
                                  const int32_t* __restrict__ a,
                                  const int32_t* __restrict__ b,
                                  const int32_t* __restrict__ bptr,
                                  int* __restrict__ cnt) {
  const int s = blockIdx.x * kT + threadIdx.x;
  if (s >= nslots) return;
  const int i = inv[s];
  if (i < 0) {
    cnt[s] = 1;
    return;
  }
  const int B = body_B(i, M, a, b), A = body_A(i, M, a, b);
  int n = bptr[B + 1] - bptr[B];
  if (A >= 0) n += bptr[A + 1] - bptr[A] - 1;
  cnt[s] = n;
}

// 6x3 block of D for contact j and body role (A or B)
__device__ inline void d_block(const double* __restrict__ frame, int j, bool roleA,
                               double rad, double Dm[6][3]) {
  const double* f = frame + 9 * (int64_t)j;
  const double n0 = f[0], n1 = f[1], n2 = f[2];
  for (int c = 0; c < 3; ++c) {
    const double d0 = f[3 * c], d1 = f[3 * c + 1], d2 = f[3 * c + 2];
    const double sgn = roleA ? -1.0 : 1.0;
    Dm[0][c] = sgn * d0;
    Dm[1][c] = sgn * d1;
    Dm[2][c] = sgn * d2;
    // n x c
    const double x0 = n1 * d2 - n2 * d1;
    const double x1 = n2 * d0 - n0 * d2;
    const double x2 = n0 * d1 - n1 * d0;
    Dm[3][c] = -rad * x0;
    Dm[4][c] = -rad * x1;
    Dm[5][c] = -rad * x2;
  }
}

__device__ inline void add_block(double out[9], const double Di[6][3],
                                 const double Dj[6][3], double im, double ii) {
  for (int c = 0; c < 3; ++c)
    for (int c2 = 0; c2 < 3; ++c2) {
      double acc = 0.0;
      for (int k = 0; k < 3; ++k) acc += Di[k][c] * im * Dj[k][c2];
      for (int k = 3; k < 6; ++k) acc += Di[k][c] * ii * Dj[k][c2];
      out[3 * c + c2] += acc;
    }
}

__global__ void fill_rows_kernel(int nslots, int M, double mbar,
                                 const int32_t* __restrict__ inv,
                                 const int32_t* __restrict__ a,
                                 const int32_t* __restrict__ b,
                                 const int32_t* __restrict__ slot,
                                 const double* __restrict__ frame,
                                 const double* __restrict__ rad,
                                 const double* __restrict__ mass,
                                 const int32_t* __restrict__ bptr,
                                 const int32_t* __restrict__ bent,
                                 const int32_t* __restrict__ rp,
                                 int32_t* __restrict__ col, double* __restrict__ val,
                                 int32_t* __restrict__ diagpos) {
  const int s = blockIdx.x * kT + threadIdx.x;
  if (s >= nslots) return;
  int w = rp[s];
  const int i = inv[s];
  if (i < 0) {
    col[w] = s;
    for (int q = 0; q < 9; ++q) val[9 * (int64_t)w + q] = (q % 4 == 0) ? 1.0 : 0.0;
    diagpos[s] = w;
    return;
  }
  const int B = body_B(i, M, a, b), A = body_A(i, M, a, b);
  double DiB[6][3], DiA[6][3];
  d_block(frame, i, false, rad[B], DiB);
  if (A >= 0) d_block(frame, i, true, rad[A], DiA);
  const double imB = 1.0 / mass[B], iiB = 1.0 / (0.4 * mass[B] * rad[B] * rad[B]);
  double imA = 0.0, iiA = 0.0;
  if (A >= 0) {
    imA = 1.0 / mass[A];
    iiA = 1.0 / (0.4 * mass[A] * rad[A] * rad[A]);
  }
  int pB = bptr[B], eB = bptr[B + 1];
  int pA = A >= 0 ? bptr[A] : 0, eA = A >= 0 ? bptr[A + 1] : 0;
  while (pB < eB || pA < eA) {
    const int sB = pB < eB ? slot[bent[pB] >> 1] : INT32_MAX;
    const int sA = pA < eA ? slot[bent[pA] >> 1] : INT32_MAX;
    const int sj = sB < sA ? sB : sA;
    const int j = sB == sj ? (bent[pB] >> 1) : (bent[pA] >> 1);
    const int jB = sB == sj ? j : -1;
    const int jA = sA == sj ? j : -1;
    double blk[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
    double Dj[6][3];
    if (jB == j) {  // shares body B of contact i
      const bool roleA = bent[pB] & 1;
      d_block(frame, j, roleA, rad[B], Dj);
      add_block(blk, DiB, Dj, imB, iiB);
      ++pB;
    }
    if (jA == j) {  // shares body A of contact i
      const bool roleA = bent[pA] & 1;
      d_block(frame, j, roleA, rad[A], Dj);
      add_block(blk, DiA, Dj, imA, iiA);
      ++pA;
    }
    col[w] = slot[j];
    for (int q = 0; q < 9; ++q) val[9 * (int64_t)w + q] = mbar * blk[q];
    if (j == i) diagpos[s] = w;
    ++w;
  }
}

// r_i = (b_i + D_i^T v_free) / vbar on the padded layout
__global__ void rhs_kernel(int nc, int M, double h, double vbar, double3 g,
                           const int32_t* __restrict__ a, const int32_t* __restrict__ b,
                           const int32_t* __restrict__ slot,
                           const double* __restrict__ phi,
                           const double* __restrict__ frame,
                           const double* __restrict__ rad,
                           const double* __restrict__ v, const double* __restrict__ w,
                           double* __restrict__ r) {
  const int i = blockIdx.x * kT + threadIdx.x;
  if (i >= nc) return;
  const int B = body_B(i, M, a, b), A = body_A(i, M, a, b);
  double acc[3] = {phi[i] / h, 0.0, 0.0};
  double Dm[6][3];
  for (int role = 0; role < 2; ++role) {
    const int body = role == 0 ? B : A;
    if (body < 0) continue;
    d_block(frame, i, role == 1, rad[body], Dm);
    const double vf[6] = {v[3 * body] + h * g.x, v[3 * body + 1] + h * g.y,
                          v[3 * body + 2] + h * g.z, w[3 * body], w[3 * body + 1],
                          w[3 * body + 2]};
    for (int c = 0; c < 3; ++c) {
      double s = 0.0;
      for (int k = 0; k < 6; ++k) s += Dm[k][c] * vf[k];
      acc[c] += s;
    }
  }
  const int64_t u = 3 * (int64_t)slot[i];
  for (int c = 0; c < 3; ++c) r[u + c] = acc[c] / vbar;
}

__global__ void mass_sum_kernel(int M, const double* __restrict__ m,
                                double* __restrict__ part) {
  __shared__ double sh[kT];
  double acc = 0.0;
  for (int i = blockIdx.x * kT + threadIdx.x; i < M; i += gridDim.x * kT) acc += m[i];
  sh[threadIdx.x] = acc;
  __syncthreads();
  for (int o = kT / 2; o > 0; o >>= 1) {
    if (threadIdx.x < o) sh[threadIdx.x] += sh[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[blockIdx.x] = sh[0];
}

// v <- v_free + M^-1 D gamma (physical units), x <- x + h v
__global__ void integrate_kernel(int M, double h, double gbar, double3 g,
                                 const int32_t* __restrict__ bptr,
                                 const int32_t* __restrict__ bent,
                                 const int32_t* __restrict__ slot,
                                 const double* __restrict__ frame,
                                 const double* __restrict__ rad,
                                 const double* __restrict__ mass,
                                 const double* __restrict__ gamma,
                                 double* __restrict__ x, double* __restrict__ v,
                                 double* __restrict__ w) {
  const int q = blockIdx.x * kT + threadIdx.x;
  if (q >= M) return;
  double F[6] = {0, 0, 0, 0, 0, 0};
  double Dm[6][3];
  for (int e = bptr[q]; e < bptr[q + 1]; ++e) {
    const int j = bent[e] >> 1;
    const bool roleA = bent[e] & 1;
    d_block(frame, j, roleA, rad[q], Dm);
    const int64_t u = 3 * (int64_t)slot[j];
    const double g0 = gamma[u] * gbar, g1 = gamma[u + 1] * gbar, g2 = gamma[u + 2] * gbar;
    for (int k = 0; k < 6; ++k) F[k] += (Dm[k][0] * g0 + Dm[k][1] * g1) + Dm[k][2] * g2;
  }
  const double im = 1.0 / mass[q];
  const double ii = 1.0 / (0.4 * mass[q] * rad[q] * rad[q]);
  const double gg[3] = {g.x, g.y, g.z};
  for (int k = 0; k < 3; ++k) {
    const double vn = (v[3 * q + k] + h * gg[k]) + im * F[k];
    v[3 * q + k] = vn;
    x[3 * q + k] += h * vn;
    w[3 * q + k] += ii * F[3 + k];
  }
}

}  // namespace

void assemble_qp(Ctx& c) {
  QTP_REQUIRE(c.ct.valid, QTP_E_STATE, "detect before assemble");
  Scene& sc = c.scene;
  Contacts& ct = c.ct;
  Qp& qp = c.qp;
  const hipStream_t s = c.stream;
  const int M = sc.M, nc = ct.nc;
  const int d = sc.log2n;
  const int64_t n = (int64_t)1 << d;
  const int nslots = (int)(n / 3);
  // scales: m_bar = mean mass, v_bar = |g| h, gamma_bar = m_bar v_bar
  const int nb = std::min(256, div_up(M, kT));
  c.tmp1.ensure(sizeof(double) * nb);
  mass_sum_kernel<<<nb, kT, 0, s>>>(M, sc.mass.as<double>(), c.tmp1.as<double>());
  QTP_CHECK_LAUNCH();
  std::vector<double> part(nb);
  QTP_HIP(hipMemcpyAsync(part.data(), c.tmp1.get(), sizeof(double) * nb,
                         hipMemcpyDeviceToHost, s));
  QTP_HIP(hipStreamSynchronize(s));
  double msum = 0.0;
  for (double p : part) msum += p;
  qp.mbar = msum / M;
  qp.vbar = std::sqrt(sc.g[0] * sc.g[0] + sc.g[1] * sc.g[1] + sc.g[2] * sc.g[2]) * sc.h;
  QTP_REQUIRE(qp.vbar > 0.0, QTP_E_ARG, "gravity and h must be non-zero");
  qp.gbar = qp.mbar * qp.vbar;
  // body -> contact incidence, sorted by body then contact
  const int ncap = std::max(nc, 1);
  c.cnt.ensure(sizeof(int) * (ncap + 1));
  c.offs.ensure(sizeof(int) * (ncap + 1));
  int nent = 0;
  if (nc > 0) {
    entries_per_contact_kernel<<<div_up(nc, kT), kT, 0, s>>>(nc, M, ct.b.as<int32_t>(),
                                                            c.cnt.as<int>());
    QTP_CHECK_LAUNCH();
    QTP_HIP(hipMemsetAsync(c.cnt.as<int>() + nc, 0, sizeof(int), s));
    exclusive_scan(s, c.cnt.as<int>(), c.offs.as<int>(), nc + 1, c.ss);
    QTP_HIP(hipMemcpyAsync(&nent, c.offs.as<int>() + nc, sizeof(int),
                           hipMemcpyDeviceToHost, s));
    QTP_HIP(hipStreamSynchronize(s));
  }
  const int necap = std::max(nent, 1);
  c.pk.ensure(sizeof(uint64_t) * necap);
  qp.body_ent.ensure(sizeof(int32_t) * necap);
  qp.body_ptr.ensure(sizeof(int32_t) * (M + 1));
  if (nent > 0) {
    int sbits = 1;
    while (((int64_t)1 << sbits) < nslots) ++sbits;
    incidence_kernel<<<div_up(nc, kT), kT, 0, s>>>(nc, M, sbits, ct.a.as<int32_t>(),
                                                  ct.b.as<int32_t>(), ct.slot.as<int32_t>(),
                                                  c.offs.as<int32_t>(), c.pk.as<uint64_t>(),
                                                  qp.body_ent.as<int32_t>());
    QTP_CHECK_LAUNCH();
    int bits = 1;
    while (((int64_t)1 << bits) < M) ++bits;
    radix_sort_pairs(s, c.pk.as<uint64_t>(), qp.body_ent.as<int32_t>(), nent,
                     bits + sbits, c.sk, c.sv, c.sh, c.ss);
    body_ptr_kernel<<<div_up(nent, kT), kT, 0, s>>>(nent, M, sbits, c.pk.as<uint64_t>(),
                                                   qp.body_ptr.as<int32_t>());
    QTP_CHECK_LAUNCH();
  } else {
    QTP_HIP(hipMemsetAsync(qp.body_ptr.get(), 0, sizeof(int32_t) * (M + 1), s));
  }
  // slot -> contact
  qp.inv_slot.ensure(sizeof(int32_t) * nslots);
  QTP_HIP(hipMemsetAsync(qp.inv_slot.get(), 0xff, sizeof(int32_t) * nslots, s));
  if (nc > 0) {
    inv_slot_kernel<<<div_up(nc, kT), kT, 0, s>>>(nc, ct.slot.as<int32_t>(),
                                                 qp.inv_slot.as<int32_t>());
    QTP_CHECK_LAUNCH();
  }
  // block-row counts and pattern
  c.cnt2.ensure(sizeof(int) * (nslots + 1));
  qp.rp.ensure(sizeof(int32_t) * (nslots + 1));
  row_counts_kernel<<<div_up(nslots, kT), kT, 0, s>>>(
      nslots, M, qp.inv_slot.as<int32_t>(), ct.a.as<int32_t>(), ct.b.as<int32_t>(),
      qp.body_ptr.as<int32_t>(), c.cnt2.as<int>());
  QTP_CHECK_LAUNCH();
  QTP_HIP(hipMemsetAsync(c.cnt2.as<int>() + nslots, 0, sizeof(int), s));
  exclusive_scan(s, c.cnt2.as<int>(), qp.rp.as<int>(), nslots + 1, c.ss);
  int nnzb = 0;
  QTP_HIP(hipMemcpyAsync(&nnzb, qp.rp.as<int32_t>() + nslots, sizeof(int),
                         hipMemcpyDeviceToHost, s));
  QTP_HIP(hipStreamSynchronize(s));
  qp.nnzb = nnzb;
  qp.col.ensure(sizeof(int32_t) * nnzb);
  qp.valN.ensure(sizeof(double) * 9 * (size_t)nnzb);
  qp.diagpos.ensure(sizeof(int32_t) * nslots);
  fill_rows_kernel<<<div_up(nslots, kT), kT, 0, s>>>(
      nslots, M, qp.mbar, qp.inv_slot.as<int32_t>(), ct.a.as<int32_t>(),
      ct.b.as<int32_t>(), ct.slot.as<int32_t>(), ct.frame.as<double>(),
      sc.radius.as<double>(), sc.mass.as<double>(), qp.body_ptr.as<int32_t>(),
      qp.body_ent.as<int32_t>(), qp.rp.as<int32_t>(), qp.col.as<int32_t>(),
      qp.valN.as<double>(), qp.diagpos.as<int32_t>());
  QTP_CHECK_LAUNCH();
  qp.r.ensure(sizeof(double) * n);
  QTP_HIP(hipMemsetAsync(qp.r.get(), 0, sizeof(double) * n, s));
  if (nc > 0) {
    rhs_kernel<<<div_up(nc, kT), kT, 0, s>>>(
        nc, M, sc.h, qp.vbar, make_double3(sc.g[0], sc.g[1], sc.g[2]),
        ct.a.as<int32_t>(), ct.b.as<int32_t>(), ct.slot.as<int32_t>(),
        ct.phi.as<double>(), ct.frame.as<double>(), sc.radius.as<double>(),
        sc.v.as<double>(), sc.w.as<double>(), qp.r.as<double>());
    QTP_CHECK_LAUNCH();
  }
  QTP_HIP(hipStreamSynchronize(s));
  qp.valid = true;
  qp.stale = false;
}

void integrate(Ctx& c) {
  QTP_REQUIRE(c.qp.valid && !c.qp.stale && c.pd.have_gamma, QTP_E_STATE,
              "solve before integrate");
  Scene& sc = c.scene;
  integrate_kernel<<<div_up(sc.M, kT), kT, 0, c.stream>>>(
      sc.M, sc.h, c.qp.gbar, make_double3(sc.g[0], sc.g[1], sc.g[2]),
      c.qp.body_ptr.as<int32_t>(), c.qp.body_ent.as<int32_t>(),
      c.ct.slot.as<int32_t>(), c.ct.frame.as<double>(), sc.radius.as<double>(),
      sc.mass.as<double>(), c.pd.gamma.as<double>(), sc.x.as<double>(),
      sc.v.as<double>(), sc.w.as<double>());
  QTP_CHECK_LAUNCH();
  QTP_HIP(hipStreamSynchronize(c.stream));
  c.ct.valid = false;  // positions moved: contacts must be detected again
  c.qp.stale = true;  // the QP stays readable but belongs to the old positions
}

}  // namespace qtp
