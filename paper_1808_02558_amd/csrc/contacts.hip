// Contact detection, frames, Morton ordering and the slot map (Sec. 2.2:
// gap function, contact frame and the active set A(q, delta) = {Phi <= delta};
// Sec. 3.3: contacts ordered by a spatial octree hierarchy and embedded in a
// uniform tree of 2^d leaves whose unused leaves are dummies).
//
// Compiled without floating-point contraction: the active-set predicate, the
// gaps, frames and Morton keys are evaluated in a fixed operation order so
// that the contact list, its order and its keys are reproducible bit for bit
// by an independent CPU implementation.
//
//  * sphere pair (a < b): active iff |x_b - x_a|^2 <= (r_a + r_b + delta)^2,
//    n = (x_b - x_a) / |x_b - x_a|, Phi = |x_b - x_a| - r_a - r_b,
//    key point (x_a + x_b) / 2;
//  * sphere a and wall w (body M + w): Phi = n_w . x_a - o_w - r_a <= delta,
//    n = n_w, key point x_a - r_a n_w;
//  * t1 = normalise(n x e_k), k = argmin |n_k| (lowest k on ties), t2 = n x t1;
//  * key: 21-bit-per-axis Morton code of the key point over the bounding box
//    of the spheres, x most significant; order by (key, a, b).
#include <algorithm>
#include <climits>
#include <cmath>

#include "dense.h"
#include "timestep.h"

namespace qtp {
namespace {

constexpr int kT = 256;

__device__ inline bool pair_active(const double* __restrict__ x,
                                   const double* __restrict__ rad, double delta,
                                   int a, int b) {
  const double dx = x[3 * b] - x[3 * a];
  const double dy = x[3 * b + 1] - x[3 * a + 1];
  const double dz = x[3 * b + 2] - x[3 * a + 2];
  const double d2 = (dx * dx + dy * dy) + dz * dz;
  const double s = (rad[a] + rad[b]) + delta;
  return d2 <= s * s;
}

__device__ inline double wall_phi(const double* __restrict__ x,
                                  const double* __restrict__ rad,
                                  const double* __restrict__ pl, int a) {
  return (((pl[0] * x[3 * a] + pl[1] * x[3 * a + 1]) + pl[2] * x[3 * a + 2]) -
          pl[3]) - rad[a];
}

// per-block min/max of (x - r) and (x + r) per axis and max radius
__global__ void bounds_kernel(int M, const double* __restrict__ x,
                              const double* __restrict__ rad,
                              double* __restrict__ part) {
  __shared__ double sh[7][kT];
  double v[7] = {INFINITY, INFINITY, INFINITY, -INFINITY, -INFINITY, -INFINITY,
                 -INFINITY};
  for (int i = blockIdx.x * kT + threadIdx.x; i < M; i += gridDim.x * kT) {
    for (int k = 0; k < 3; ++k) {
      v[k] = fmin(v[k], x[3 * i + k] - rad[i]);
      v[3 + k] = fmax(v[3 + k], x[3 * i + k] + rad[i]);
    }
    v[6] = fmax(v[6], rad[i]);
  }
  for (int k = 0; k < 7; ++k) sh[k][threadIdx.x] = v[k];
  __syncthreads();
  for (int o = kT / 2; o > 0; o >>= 1) {
    if (threadIdx.x < o)
      for (int k = 0; k < 7; ++k) {
        const double a = sh[k][threadIdx.x], b = sh[k][threadIdx.x + o];
        sh[k][threadIdx.x] = k < 3 ? fmin(a, b) : fmax(a, b);
      }
    __syncthreads();
  }
  if (threadIdx.x == 0)
    for (int k = 0; k < 7; ++k) part[blockIdx.x * 7 + k] = sh[k][0];
}

__global__ void cell_ids_kernel(int M, const double* __restrict__ x, double3 org,
                                double cell, int3 dims, uint64_t* __restrict__ key,
                                int32_t* __restrict__ idx) {
  const int i = blockIdx.x * kT + threadIdx.x;
  if (i >= M) return;
  const int cx = (int)floor((x[3 * i] - org.x) / cell);
  const int cy = (int)floor((x[3 * i + 1] - org.y) / cell);
  const int cz = (int)floor((x[3 * i + 2] - org.z) / cell);
  key[i] = ((uint64_t)(cx + 1) * dims.y + (cy + 1)) * dims.z + (cz + 1);
  idx[i] = i;
}

__global__ void cell_range_kernel(int M, const uint64_t* __restrict__ key,
                                  int32_t* __restrict__ start,
                                  int32_t* __restrict__ stop) {
  const int i = blockIdx.x * kT + threadIdx.x;
  if (i >= M) return;
  const uint64_t k = key[i];
  if (i == 0 || key[i - 1] != k) start[k] = i;
  if (i == M - 1 || key[i + 1] != k) stop[k] = i + 1;
}

// MODE 0: count active pairs (a < b) per sphere a; MODE 1: write them.
template <int MODE>
__global__ void pairs_kernel(int M, const double* __restrict__ x,
                             const double* __restrict__ rad, double delta,
                             double3 org, double cell, int3 dims,
                             const int32_t* __restrict__ start,
                             const int32_t* __restrict__ stop,
                             const int32_t* __restrict__ sorted_idx,
                             int32_t* __restrict__ count,
                             const int32_t* __restrict__ offs,
                             int32_t* __restrict__ pa, int32_t* __restrict__ pb) {
  const int i = blockIdx.x * kT + threadIdx.x;
  if (i >= M) return;
  const int cx = (int)floor((x[3 * i] - org.x) / cell) + 1;
  const int cy = (int)floor((x[3 * i + 1] - org.y) / cell) + 1;
  const int cz = (int)floor((x[3 * i + 2] - org.z) / cell) + 1;
  int n = 0;
  int w = MODE == 1 ? offs[i] : 0;
  for (int ox = -1; ox <= 1; ++ox)
    for (int oy = -1; oy <= 1; ++oy)
      for (int oz = -1; oz <= 1; ++oz) {
        const int64_t c = ((int64_t)(cx + ox) * dims.y + (cy + oy)) * dims.z + (cz + oz);
        const int s0 = start[c], s1 = stop[c];
        for (int t = s0; t < s1; ++t) {
          const int j = sorted_idx[t];
          if (j <= i) continue;
          if (pair_active(x, rad, delta, i, j)) {
            if (MODE == 0) {
              ++n;
            } else {
              pa[w] = i;
              pb[w] = j;
              ++w;
            }
          }
        }
      }
  if (MODE == 0) count[i] = n;
}

template <int MODE>
__global__ void walls_kernel(int M, int nw, const double* __restrict__ x,
                             const double* __restrict__ rad,
                             const double* __restrict__ planes, double delta,
                             int32_t* __restrict__ count,
                             const int32_t* __restrict__ offs, int base,
                             int32_t* __restrict__ pa, int32_t* __restrict__ pb) {
  const int i = blockIdx.x * kT + threadIdx.x;
  if (i >= M) return;
  int n = 0;
  int w = MODE == 1 ? base + offs[i] : 0;
  for (int k = 0; k < nw; ++k)
    if (wall_phi(x, rad, planes + 4 * k, i) <= delta) {
      if (MODE == 0) {
        ++n;
      } else {
        pa[w] = i;
        pb[w] = M + k;
        ++w;
      }
    }
  if (MODE == 0) count[i] = n;
}

__device__ inline uint64_t spread3(uint64_t v) {
  v &= 0x1fffffull;
  v = (v | (v << 32)) & 0x1f00000000ffffull;
  v = (v | (v << 16)) & 0x1f0000ff0000ffull;
  v = (v | (v << 8)) & 0x100f00f00f00f00full;
  v = (v | (v << 4)) & 0x10c30c30c30c30c3ull;
  v = (v | (v << 2)) & 0x1249249249249249ull;
  return v;
}

__device__ inline uint64_t quantise(double p, double lo, double hi) {
  double q = floor(((p - lo) / (hi - lo)) * 2097152.0);
  if (q < 0.0) q = 0.0;
  if (q > 2097151.0) q = 2097151.0;
  return (uint64_t)q;
}

// Morton key of each contact's key point; sort keys for the (key, a, b) order
__global__ void contact_keys_kernel(int nc, int M, const int32_t* __restrict__ pa,
                                    const int32_t* __restrict__ pb,
                                    const double* __restrict__ x,
                                    const double* __restrict__ rad,
                                    const double* __restrict__ planes,
                                    const double* __restrict__ bounds,
                                    uint64_t* __restrict__ key) {
  const int i = blockIdx.x * kT + threadIdx.x;
  if (i >= nc) return;
  const int a = pa[i], b = pb[i];
  double p[3];
  if (b < M) {
    for (int k = 0; k < 3; ++k) p[k] = (x[3 * a + k] + x[3 * b + k]) * 0.5;
  } else {
    const double* pl = planes + 4 * (b - M);
    for (int k = 0; k < 3; ++k) p[k] = x[3 * a + k] - rad[a] * pl[k];
  }
  const uint64_t qx = quantise(p[0], bounds[0], bounds[3]);
  const uint64_t qy = quantise(p[1], bounds[1], bounds[4]);
  const uint64_t qz = quantise(p[2], bounds[2], bounds[5]);
  key[i] = (spread3(qx) << 2) | (spread3(qy) << 1) | spread3(qz);
}

__global__ void gather_int_kernel(int n, const int32_t* __restrict__ perm,
                                  const int32_t* __restrict__ in,
                                  int32_t* __restrict__ out) {
  const int i = blockIdx.x * kT + threadIdx.x;
  if (i < n) out[i] = in[perm[i]];
}

__global__ void gather_key_kernel(int n, const int32_t* __restrict__ perm,
                                  const uint64_t* __restrict__ in,
                                  uint64_t* __restrict__ out) {
  const int i = blockIdx.x * kT + threadIdx.x;
  if (i < n) out[i] = in[perm[i]];
}

__global__ void iota_kernel(int n, int32_t* __restrict__ v) {
  const int i = blockIdx.x * kT + threadIdx.x;
  if (i < n) v[i] = i;
}

__global__ void widen_kernel(int n, const int32_t* __restrict__ in,
                             uint64_t* __restrict__ out) {
  const int i = blockIdx.x * kT + threadIdx.x;
  if (i < n) out[i] = (uint64_t)(uint32_t)in[i];
}

// gaps and frames in the final order; slot of each contact
__global__ void frames_kernel(int nc, int M, int nslots,
                              const int32_t* __restrict__ pa,
                              const int32_t* __restrict__ pb,
                              const double* __restrict__ x,
                              const double* __restrict__ rad,
                              const double* __restrict__ planes,
                              double* __restrict__ phi, double* __restrict__ frame,
                              int32_t* __restrict__ slot, int* __restrict__ bad) {
  const int i = blockIdx.x * kT + threadIdx.x;
  if (i >= nc) return;
  const int a = pa[i], b = pb[i];
  double n0, n1, n2, ph;
  if (b < M) {
    const double dx = x[3 * b] - x[3 * a];
    const double dy = x[3 * b + 1] - x[3 * a + 1];
    const double dz = x[3 * b + 2] - x[3 * a + 2];
    const double d2 = (dx * dx + dy * dy) + dz * dz;
    const double dist = sqrt(d2);
    if (!(dist > 0.0)) bad[0] = 1;
    n0 = dx / dist;
    n1 = dy / dist;
    n2 = dz / dist;
    ph = (dist - rad[a]) - rad[b];
  } else {
    const double* pl = planes + 4 * (b - M);
    n0 = pl[0];
    n1 = pl[1];
    n2 = pl[2];
    ph = wall_phi(x, rad, pl, a);
  }
  const double a0 = fabs(n0), a1 = fabs(n1), a2 = fabs(n2);
  double c0, c1, c2;
  if (a0 <= a1 && a0 <= a2) {
    c0 = 0.0; c1 = n2; c2 = -n1;
  } else if (a1 <= a2) {
    c0 = -n2; c1 = 0.0; c2 = n0;
  } else {
    c0 = n1; c1 = -n0; c2 = 0.0;
  }
  const double cn = sqrt((c0 * c0 + c1 * c1) + c2 * c2);
  const double t0 = c0 / cn, t1 = c1 / cn, t2 = c2 / cn;
  const double s0 = n1 * t2 - n2 * t1;
  const double s1 = n2 * t0 - n0 * t2;
  const double s2 = n0 * t1 - n1 * t0;
  double* f = frame + 9 * (int64_t)i;
  f[0] = n0; f[1] = n1; f[2] = n2;
  f[3] = t0; f[4] = t1; f[5] = t2;
  f[6] = s0; f[7] = s1; f[8] = s2;
  phi[i] = ph;
  slot[i] = (int32_t)(((int64_t)i * nslots) / nc);
}

// ---- slot re-use across time steps (Sec. 3.3) --------------------------------

__global__ void pair_keys_kernel(int nc, const int32_t* __restrict__ a,
                                 const int32_t* __restrict__ b, uint64_t* __restrict__ out) {
  const int i = blockIdx.x * kT + threadIdx.x;
  if (i < nc) out[i] = ((uint64_t)(uint32_t)a[i] << 32) | (uint32_t)b[i];
}

// old[i] = slot of the same pair in the previous step or -1; marks taken
// slots and flags the new contacts
__global__ void lookup_kernel(int nc, const int32_t* __restrict__ a,
                              const int32_t* __restrict__ b,
                              const uint64_t* __restrict__ prev,
                              const int32_t* __restrict__ prev_slot, int np,
                              int32_t* __restrict__ old, int* __restrict__ taken,
                              int* __restrict__ isnew) {
  const int i = blockIdx.x * kT + threadIdx.x;
  if (i >= nc) return;
  const uint64_t key = ((uint64_t)(uint32_t)a[i] << 32) | (uint32_t)b[i];
  int lo = 0, hi = np;
  while (lo < hi) {
    const int mid = (lo + hi) >> 1;
    if (prev[mid] < key) lo = mid + 1; else hi = mid;
  }
  if (lo < np && prev[lo] == key) {
    const int s = prev_slot[lo];
    old[i] = s;
    taken[s] = 1;
    isnew[i] = 0;
  } else {
    old[i] = -1;
    isnew[i] = 1;
  }
}

// taken -> free flags in place (entry nslots is the scan's terminator)
__global__ void flip_kernel(int nslots, int* __restrict__ f) {
  const int s = blockIdx.x * kT + threadIdx.x;
  if (s < nslots) f[s] = 1 - f[s];
  else if (s == nslots) f[s] = 0;
}

__global__ void free_list_kernel(int nslots, const int* __restrict__ flag,
                                 const int* __restrict__ pos, int32_t* __restrict__ list) {
  const int s = blockIdx.x * kT + threadIdx.x;
  if (s < nslots && flag[s]) list[pos[s]] = s;
}

// val[k] = (index in the free list of the first free slot at or after the
// fresh slot of the k-th new contact) - k
__global__ void new_val_kernel(int nc, int nslots, const int32_t* __restrict__ old,
                               const int* __restrict__ rank,
                               const int32_t* __restrict__ list, int nfree,
                               int* __restrict__ val) {
  const int i = blockIdx.x * kT + threadIdx.x;
  if (i >= nc || old[i] >= 0) return;
  const int64_t tau = ((int64_t)i * nslots) / nc;
  int lo = 0, hi = nfree;
  while (lo < hi) {
    const int mid = (lo + hi) >> 1;
    if (list[mid] < tau) lo = mid + 1; else hi = mid;
  }
  val[rank[i]] = lo - rank[i];
}

// inclusive max-scan in blocks of kScanItems; block maxima to bmax
constexpr int kScanItems = 4 * kT;
__global__ void max_scan_block_kernel(int n, int* __restrict__ v, int* __restrict__ bmax) {
  __shared__ int sh[kT];
  const int base = blockIdx.x * kScanItems + threadIdx.x * 4;
  int loc[4];
  int run = INT_MIN;
  for (int q = 0; q < 4; ++q) {
    const int e = base + q;
    run = max(run, e < n ? v[e] : INT_MIN);
    loc[q] = run;
  }
  sh[threadIdx.x] = run;
  __syncthreads();
  for (int o = 1; o < kT; o <<= 1) {
    const int t = threadIdx.x >= o ? sh[threadIdx.x - o] : INT_MIN;
    __syncthreads();
    sh[threadIdx.x] = max(sh[threadIdx.x], t);
    __syncthreads();
  }
  const int before = threadIdx.x > 0 ? sh[threadIdx.x - 1] : INT_MIN;
  for (int q = 0; q < 4; ++q) {
    const int e = base + q;
    if (e < n) v[e] = max(loc[q], before);
  }
  if (threadIdx.x == kT - 1) bmax[blockIdx.x] = sh[kT - 1];
}

// exclusive max over the block maxima, in order (one thread: few blocks)
__global__ void max_scan_carry_kernel(int nb, int* __restrict__ bmax) {
  if (threadIdx.x != 0) return;
  int run = INT_MIN;
  for (int k = 0; k < nb; ++k) {
    const int t = bmax[k];
    bmax[k] = run;
    run = max(run, t);
  }
}

__global__ void max_scan_add_kernel(int n, int* __restrict__ v, const int* __restrict__ carry) {
  const int e = blockIdx.x * kT + threadIdx.x;
  if (e < n) v[e] = max(v[e], carry[e / kScanItems]);
}

__global__ void assign_kernel(int nc, const int32_t* __restrict__ old,
                              const int* __restrict__ rank, const int* __restrict__ mx,
                              const int32_t* __restrict__ list, int nfree,
                              int32_t* __restrict__ slot, int* __restrict__ overflow) {
  const int i = blockIdx.x * kT + threadIdx.x;
  if (i >= nc) return;
  if (old[i] >= 0) {
    slot[i] = old[i];
    return;
  }
  const int k = rank[i];
  const int64_t j = (int64_t)k + mx[k];
  if (j >= nfree) overflow[0] = 1;  // benign race: every writer stores 1
  else slot[i] = list[j];
}

// Persistent slots from the previous step's map; leaves ct.slot (the fresh
// map) untouched when a new contact finds no free slot.
void persistent_slots(Ctx& c, int nc, int nslots) {
  Contacts& ct = c.ct;
  const hipStream_t s = c.stream;
  ct.old_slot.ensure(sizeof(int32_t) * nc);
  ct.taken.ensure(sizeof(int) * (nslots + 1));
  ct.free_pos.ensure(sizeof(int) * (nslots + 1));
  ct.free_list.ensure(sizeof(int32_t) * std::max(nslots, 1));
  ct.new_rank.ensure(sizeof(int) * (nc + 1));
  ct.new_val.ensure(sizeof(int) * (nc + 1));
  c.cnt.ensure(sizeof(int) * (nc + 1));
  QTP_HIP(hipMemsetAsync(ct.taken.get(), 0, sizeof(int) * (nslots + 1), s));
  QTP_HIP(hipMemsetAsync(c.cnt.as<int>() + nc, 0, sizeof(int), s));
  lookup_kernel<<<div_up(nc, kT), kT, 0, s>>>(
      nc, ct.a.as<int32_t>(), ct.b.as<int32_t>(), ct.prev_pair.as<uint64_t>(),
      ct.prev_slot.as<int32_t>(), ct.prev_n, ct.old_slot.as<int32_t>(),
      ct.taken.as<int>(), c.cnt.as<int>());
  QTP_CHECK_LAUNCH();
  flip_kernel<<<div_up(nslots + 1, kT), kT, 0, s>>>(nslots, ct.taken.as<int>());
  QTP_CHECK_LAUNCH();
  exclusive_scan(s, ct.taken.as<int>(), ct.free_pos.as<int>(), nslots + 1, c.ss);
  exclusive_scan(s, c.cnt.as<int>(), ct.new_rank.as<int>(), nc + 1, c.ss);
  int hv[2] = {0, 0};
  QTP_HIP(hipMemcpyAsync(&hv[0], ct.free_pos.as<int>() + nslots, sizeof(int),
                         hipMemcpyDeviceToHost, s));
  QTP_HIP(hipMemcpyAsync(&hv[1], ct.new_rank.as<int>() + nc, sizeof(int),
                         hipMemcpyDeviceToHost, s));
  QTP_HIP(hipStreamSynchronize(s));
  const int nfree = hv[0], K = hv[1];
  free_list_kernel<<<div_up(nslots, kT), kT, 0, s>>>(
      nslots, ct.taken.as<int>(), ct.free_pos.as<int>(), ct.free_list.as<int32_t>());
  QTP_CHECK_LAUNCH();
  if (K > 0) {
    new_val_kernel<<<div_up(nc, kT), kT, 0, s>>>(
        nc, nslots, ct.old_slot.as<int32_t>(), ct.new_rank.as<int>(),
        ct.free_list.as<int32_t>(), nfree, ct.new_val.as<int>());
    QTP_CHECK_LAUNCH();
    const int nb = div_up(K, kScanItems);
    ct.scan_tmp.ensure(sizeof(int) * nb);
    max_scan_block_kernel<<<nb, kT, 0, s>>>(K, ct.new_val.as<int>(), ct.scan_tmp.as<int>());
    QTP_CHECK_LAUNCH();
    if (nb > 1) {
      max_scan_carry_kernel<<<1, 64, 0, s>>>(nb, ct.scan_tmp.as<int>());
      QTP_CHECK_LAUNCH();
      max_scan_add_kernel<<<div_up(K, kT), kT, 0, s>>>(K, ct.new_val.as<int>(),
                                                      ct.scan_tmp.as<int>());
      QTP_CHECK_LAUNCH();
    }
  }
  int* ovf = c.flag.as<int>() + 1;
  QTP_HIP(hipMemsetAsync(ovf, 0, sizeof(int), s));
  // the assignment goes to new_rank's storage only after it is read: use the
  // free-position buffer (nslots + 1 >= nc ints) as the output
  int32_t* out = reinterpret_cast<int32_t*>(ct.free_pos.get());
  assign_kernel<<<div_up(nc, kT), kT, 0, s>>>(
      nc, ct.old_slot.as<int32_t>(), ct.new_rank.as<int>(), ct.new_val.as<int>(),
      ct.free_list.as<int32_t>(), nfree, out, ovf);
  QTP_CHECK_LAUNCH();
  int hovf = 0;
  QTP_HIP(hipMemcpyAsync(&hovf, ovf, sizeof(int), hipMemcpyDeviceToHost, s));
  QTP_HIP(hipStreamSynchronize(s));
  if (hovf) {
    ct.rebuilt = true;
    ct.n_persistent = 0;
    return;
  }
  QTP_HIP(hipMemcpyAsync(ct.slot.get(), out, sizeof(int32_t) * nc,
                         hipMemcpyDeviceToDevice, s));
  ct.n_persistent = nc - K;
}

// The pairs of this step sorted, with their slots, for the next step.
void save_slot_map(Ctx& c, int nc, int nslots, int key_bits) {
  Contacts& ct = c.ct;
  const hipStream_t s = c.stream;
  ct.prev_pair.ensure(sizeof(uint64_t) * std::max(nc, 1));
  ct.prev_slot.ensure(sizeof(int32_t) * std::max(nc, 1));
  if (nc > 0) {
    pair_keys_kernel<<<div_up(nc, kT), kT, 0, s>>>(nc, ct.a.as<int32_t>(),
                                                  ct.b.as<int32_t>(),
                                                  ct.prev_pair.as<uint64_t>());
    QTP_CHECK_LAUNCH();
    QTP_HIP(hipMemcpyAsync(ct.prev_slot.get(), ct.slot.get(), sizeof(int32_t) * nc,
                           hipMemcpyDeviceToDevice, s));
    radix_sort_pairs(s, ct.prev_pair.as<uint64_t>(), ct.prev_slot.as<int32_t>(), nc,
                     key_bits, c.sk, c.sv, c.sh, c.ss);
  }
  ct.prev_n = nc;
  ct.prev_nslots = nslots;
}

}  // namespace

int detect_contacts(Ctx& c) {
  Scene& sc = c.scene;
  Contacts& ct = c.ct;
  const hipStream_t s = c.stream;
  const int M = sc.M;
  QTP_REQUIRE(M >= 1, QTP_E_STATE, "no bodies set");
  c.pd.have_gamma = false;  // impulses belong to the previous contact set
  // bounding box and the largest radius
  const int nb = std::min(256, div_up(M, kT));
  c.tmp1.ensure(sizeof(double) * 7 * nb);
  bounds_kernel<<<nb, kT, 0, s>>>(M, sc.x.as<double>(), sc.radius.as<double>(),
                                 c.tmp1.as<double>());
  QTP_CHECK_LAUNCH();
  std::vector<double> part(7 * nb);
  QTP_HIP(hipMemcpyAsync(part.data(), c.tmp1.get(), sizeof(double) * 7 * nb,
                         hipMemcpyDeviceToHost, s));
  QTP_HIP(hipStreamSynchronize(s));
  double bnd[7] = {INFINITY, INFINITY, INFINITY, -INFINITY, -INFINITY, -INFINITY,
                   -INFINITY};
  for (int b = 0; b < nb; ++b)
    for (int k = 0; k < 7; ++k)
      bnd[k] = k < 3 ? std::min(bnd[k], part[7 * b + k]) : std::max(bnd[k], part[7 * b + k]);
  QTP_REQUIRE(std::isfinite(bnd[0]) && std::isfinite(bnd[3]) && std::isfinite(bnd[6]),
              QTP_E_NUMERIC, "non-finite body positions or radii");
  ct.bounds.ensure(sizeof(double) * 8);
  QTP_HIP(hipMemcpyAsync(ct.bounds.get(), bnd, sizeof(double) * 7,
                         hipMemcpyHostToDevice, s));
  // uniform cell grid with edge 2 max(r) + delta (origin: min of x - r)
  // slightly enlarged so that rounding never moves an active pair two cells apart
  const double cell = (2.0 * bnd[6] + sc.delta) * (1.0 + 1e-9);
  const double3 org = make_double3(bnd[0], bnd[1], bnd[2]);
  int3 dims;
  dims.x = (int)std::floor((bnd[3] - bnd[0]) / cell) + 3;
  dims.y = (int)std::floor((bnd[4] - bnd[1]) / cell) + 3;
  dims.z = (int)std::floor((bnd[5] - bnd[2]) / cell) + 3;
  const int64_t ncell = (int64_t)dims.x * dims.y * dims.z;
  QTP_REQUIRE(ncell < ((int64_t)1 << 31), QTP_E_CAPACITY, "cell grid too large");
  ct.cell_key.ensure(sizeof(uint64_t) * M);
  ct.cell_idx.ensure(sizeof(int32_t) * M);
  cell_ids_kernel<<<div_up(M, kT), kT, 0, s>>>(M, sc.x.as<double>(), org, cell, dims,
                                              ct.cell_key.as<uint64_t>(),
                                              ct.cell_idx.as<int32_t>());
  QTP_CHECK_LAUNCH();
  int key_bits = 1;
  while (((int64_t)1 << key_bits) < ncell) ++key_bits;
  radix_sort_pairs(s, ct.cell_key.as<uint64_t>(), ct.cell_idx.as<int32_t>(), M,
                   key_bits, c.sk, c.sv, c.sh, c.ss);
  ct.cell_start.ensure(sizeof(int32_t) * ncell);
  ct.cell_stop.ensure(sizeof(int32_t) * ncell);
  QTP_HIP(hipMemsetAsync(ct.cell_start.get(), 0, sizeof(int32_t) * ncell, s));
  QTP_HIP(hipMemsetAsync(ct.cell_stop.get(), 0, sizeof(int32_t) * ncell, s));
  cell_range_kernel<<<div_up(M, kT), kT, 0, s>>>(M, ct.cell_key.as<uint64_t>(),
                                                ct.cell_start.as<int32_t>(),
                                                ct.cell_stop.as<int32_t>());
  QTP_CHECK_LAUNCH();
  // count, scan, write: sphere pairs then walls
  c.cnt.ensure(sizeof(int32_t) * (M + 1));
  c.offs.ensure(sizeof(int32_t) * (M + 1));
  pairs_kernel<0><<<div_up(M, kT), kT, 0, s>>>(
      M, sc.x.as<double>(), sc.radius.as<double>(), sc.delta, org, cell, dims,
      ct.cell_start.as<int32_t>(), ct.cell_stop.as<int32_t>(),
      ct.cell_idx.as<int32_t>(), c.cnt.as<int32_t>(), nullptr, nullptr, nullptr);
  QTP_CHECK_LAUNCH();
  QTP_HIP(hipMemsetAsync(c.cnt.as<int32_t>() + M, 0, sizeof(int32_t), s));
  exclusive_scan(s, c.cnt.as<int>(), c.offs.as<int>(), M + 1, c.ss);
  int npair = 0;
  QTP_HIP(hipMemcpyAsync(&npair, c.offs.as<int32_t>() + M, sizeof(int), hipMemcpyDeviceToHost, s));
  QTP_HIP(hipStreamSynchronize(s));
  c.cnt2.ensure(sizeof(int32_t) * (M + 1));
  c.offs2.ensure(sizeof(int32_t) * (M + 1));
  walls_kernel<0><<<div_up(M, kT), kT, 0, s>>>(M, sc.nw, sc.x.as<double>(),
                                              sc.radius.as<double>(), sc.planes.as<double>(),
                                              sc.delta, c.cnt2.as<int32_t>(), nullptr, 0,
                                              nullptr, nullptr);
  QTP_CHECK_LAUNCH();
  QTP_HIP(hipMemsetAsync(c.cnt2.as<int32_t>() + M, 0, sizeof(int32_t), s));
  exclusive_scan(s, c.cnt2.as<int>(), c.offs2.as<int>(), M + 1, c.ss);
  int nwc = 0;
  QTP_HIP(hipMemcpyAsync(&nwc, c.offs2.as<int32_t>() + M, sizeof(int), hipMemcpyDeviceToHost, s));
  QTP_HIP(hipStreamSynchronize(s));
  const int nc = npair + nwc;
  const int nslots = (int)(((int64_t)1 << sc.log2n) / 3);
  ct.nc = nc;
  if (nc > nslots)
    throw Error(QTP_E_CAPACITY, "contacts exceed the slots of 2^d: raise log2n");
  const int ncap = std::max(nc, 1);
  c.ua.ensure(sizeof(int32_t) * ncap);
  c.ub.ensure(sizeof(int32_t) * ncap);
  if (npair > 0) {
    pairs_kernel<1><<<div_up(M, kT), kT, 0, s>>>(
        M, sc.x.as<double>(), sc.radius.as<double>(), sc.delta, org, cell, dims,
        ct.cell_start.as<int32_t>(), ct.cell_stop.as<int32_t>(),
        ct.cell_idx.as<int32_t>(), nullptr, c.offs.as<int32_t>(), c.ua.as<int32_t>(),
        c.ub.as<int32_t>());
    QTP_CHECK_LAUNCH();
  }
  if (nwc > 0) {
    walls_kernel<1><<<div_up(M, kT), kT, 0, s>>>(
        M, sc.nw, sc.x.as<double>(), sc.radius.as<double>(), sc.planes.as<double>(),
        sc.delta, nullptr, c.offs2.as<int32_t>(), npair, c.ua.as<int32_t>(),
        c.ub.as<int32_t>());
    QTP_CHECK_LAUNCH();
  }
  ct.a.ensure(sizeof(int32_t) * ncap);
  ct.b.ensure(sizeof(int32_t) * ncap);
  ct.key.ensure(sizeof(uint64_t) * ncap);
  ct.phi.ensure(sizeof(double) * ncap);
  ct.frame.ensure(sizeof(double) * 9 * ncap);
  ct.slot.ensure(sizeof(int32_t) * ncap);
  if (nc > 0) {
    // order by (key, a, b): stable sorts by b, then a, then key
    c.pk.ensure(sizeof(uint64_t) * nc);
    c.perm.ensure(sizeof(int32_t) * nc);
    c.perm2.ensure(sizeof(int32_t) * nc);
    iota_kernel<<<div_up(nc, kT), kT, 0, s>>>(nc, c.perm.as<int32_t>());
    QTP_CHECK_LAUNCH();
    int bbits = 1;
    while (((int64_t)1 << bbits) < (int64_t)M + sc.nw) ++bbits;
    for (int pass = 0; pass < 3; ++pass) {
      if (pass == 0) {
        gather_int_kernel<<<div_up(nc, kT), kT, 0, s>>>(nc, c.perm.as<int32_t>(),
                                                       c.ub.as<int32_t>(), c.perm2.as<int32_t>());
        QTP_CHECK_LAUNCH();
        widen_kernel<<<div_up(nc, kT), kT, 0, s>>>(nc, c.perm2.as<int32_t>(),
                                                  c.pk.as<uint64_t>());
      } else if (pass == 1) {
        gather_int_kernel<<<div_up(nc, kT), kT, 0, s>>>(nc, c.perm.as<int32_t>(),
                                                       c.ua.as<int32_t>(), c.perm2.as<int32_t>());
        QTP_CHECK_LAUNCH();
        widen_kernel<<<div_up(nc, kT), kT, 0, s>>>(nc, c.perm2.as<int32_t>(),
                                                  c.pk.as<uint64_t>());
      } else {
        // Morton keys of the contacts in their original order, then gathered
        contact_keys_kernel<<<div_up(nc, kT), kT, 0, s>>>(
            nc, M, c.ua.as<int32_t>(), c.ub.as<int32_t>(), sc.x.as<double>(),
            sc.radius.as<double>(), sc.planes.as<double>(), ct.bounds.as<double>(),
            ct.key.as<uint64_t>());
        QTP_CHECK_LAUNCH();
        gather_key_kernel<<<div_up(nc, kT), kT, 0, s>>>(nc, c.perm.as<int32_t>(),
                                                       ct.key.as<uint64_t>(), c.pk.as<uint64_t>());
      }
      QTP_CHECK_LAUNCH();
      radix_sort_pairs(s, c.pk.as<uint64_t>(), c.perm.as<int32_t>(), nc,
                       pass == 2 ? 63 : bbits, c.sk, c.sv, c.sh, c.ss);
    }
    // final order: perm; the sorted keys are in c.pk
    gather_int_kernel<<<div_up(nc, kT), kT, 0, s>>>(nc, c.perm.as<int32_t>(),
                                                   c.ua.as<int32_t>(), ct.a.as<int32_t>());
    QTP_CHECK_LAUNCH();
    gather_int_kernel<<<div_up(nc, kT), kT, 0, s>>>(nc, c.perm.as<int32_t>(),
                                                   c.ub.as<int32_t>(), ct.b.as<int32_t>());
    QTP_CHECK_LAUNCH();
    QTP_HIP(hipMemcpyAsync(ct.key.get(), c.pk.get(), sizeof(uint64_t) * nc,
                           hipMemcpyDeviceToDevice, s));
    c.flag.ensure(sizeof(int) * 16);
    QTP_HIP(hipMemsetAsync(c.flag.get(), 0, sizeof(int), s));
    frames_kernel<<<div_up(nc, kT), kT, 0, s>>>(
        nc, M, nslots, ct.a.as<int32_t>(), ct.b.as<int32_t>(), sc.x.as<double>(),
        sc.radius.as<double>(), sc.planes.as<double>(), ct.phi.as<double>(),
        ct.frame.as<double>(), ct.slot.as<int32_t>(), c.flag.as<int>());
    QTP_CHECK_LAUNCH();
    int bad = 0;
    QTP_HIP(hipMemcpyAsync(&bad, c.flag.get(), sizeof(int), hipMemcpyDeviceToHost, s));
    QTP_HIP(hipStreamSynchronize(s));
    QTP_REQUIRE(bad == 0, QTP_E_NUMERIC, "coincident sphere centres");
  }
  ct.rebuilt = false;
  ct.n_persistent = 0;
  if (c.cfg.slot_mode == 1) {
    if (nc > 0 && ct.prev_n > 0 && ct.prev_nslots == nslots) persistent_slots(c, nc, nslots);
    int bbits = 1;
    while (((int64_t)1 << bbits) < (int64_t)M + sc.nw) ++bbits;
    save_slot_map(c, nc, nslots, 32 + bbits);
  } else {
    ct.prev_n = -1;
  }
  QTP_HIP(hipStreamSynchronize(s));
  ct.valid = true;
  return nc;
}

}  // namespace qtp
