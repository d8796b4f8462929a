// Observables of a density state (Sec. III and IV of the paper):
//   sigma   = (1/V) sum |Phi_P - phibar_P|                      (Eq. for sigma(t))
//   Y_2^P   = sqrt(sum y^2 Phi_P / (nx phibar_P sum_rows y^2)),  y = row + 1/2 - ny/2 (Eq. width)
//   sigma_D = (1/V) sum |Phi_P^a - Phi_P^b|                     (Eq. for sigma_Delta)
//   particles: connected clusters of sites with Phi_P >= threshold, nearest-
//   neighbour connectivity on the periodic grid, each labelled by its lowest
//   site index; per particle the polymer content N = sum Phi_P, the
//   Phi_P-weighted centroid and the gyration tensor of Eq. gyration_tensor,
//   evaluated as the weighted covariance (the double sum over site pairs
//   equals it), from minimum-image offsets to the particle's label site;
//   R and c_rel from its eigenvalues (Eqs. asph, rel_asph).
//   nucleation events (Sec. IV, nucleation stage): a particle none of whose
//   sites was a particle site at the previous tracking sample is new.
// Phi_P = Phi_A + Phi_B is formed in the storage precision; sums in FP64.
#pragma once
#include <hip/hip_runtime.h>

#include "kernels.hpp"

namespace epdlb {
namespace obs {

__device__ __forceinline__ double wave_sum_d(double v) {
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// Writes the block's sums of a and b to part[2 * blockIdx.x + {0, 1}].
__device__ __forceinline__ void block_pair(double a, double b, double* part) {
  __shared__ double red[2][16];
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6, nw = (blockDim.x + 63) >> 6;
  a = wave_sum_d(a);
  b = wave_sum_d(b);
  if (lane == 0) {
    red[0][wid] = a;
    red[1][wid] = b;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    double sa = 0.0, sb = 0.0;
    for (int w = 0; w < nw; ++w) {
      sa += red[0][w];
      sb += red[1][w];
    }
    part[2 * blockIdx.x] = sa;
    part[2 * blockIdx.x + 1] = sb;
  }
}

// Labels (site index on the particles, -1 elsewhere), the block partial sums
// of |Phi_P - phibar_P| and y^2 Phi_P, and cleared per-site accumulators
// (ov, the overlap flags of tracking, may be null).
template <typename T>
__global__ void __launch_bounds__(256) k_obs_init(const T* __restrict__ phi, long n, int nx, int ny, double thr,
                                                  double phibar, int* __restrict__ label, double* __restrict__ part,
                                                  int* __restrict__ area, int* __restrict__ wrap,
                                                  double* __restrict__ sums, int* __restrict__ count,
                                                  int* __restrict__ ov) {
  const long i = long(blockIdx.x) * blockDim.x + threadIdx.x;
  double s = 0.0, m = 0.0;
  if (i == 0) *count = 0;
  if (i < n) {
    area[i] = 0;
    wrap[i] = 0;
    if (ov) ov[i] = 0;
#pragma unroll
    for (int k = 0; k < 6; ++k) sums[6 * i + k] = 0.0;
    const T pP = phi[i] + phi[n + i];
    const double p = double(pP);
    label[i] = p >= thr ? int(i) : -1;
    s = fabs(p - phibar);
    const double y = double(i / nx) + 0.5 - 0.5 * double(ny);
    m = y * y * p;
  }
  block_pair(s, m, part);
}

// Root of x: follow the parent links (labels only decrease; roots point to themselves).
// Parent reads go to L2 (agent scope), so links made by other CUs are seen.
__device__ __forceinline__ int find_root(const int* L, int x) {
  int p = __hip_atomic_load(L + x, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  while (p != x) {
    x = p;
    p = __hip_atomic_load(L + x, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
  return x;
}

// Joins the trees of a and b: the larger root is linked below the smaller one
// with atomicMin; when the larger node was no longer a root, its former
// parent is joined in the next round, so no link is lost.  Every failed round
// lowers max(a, b) (the atomic returns a parent below b), so the loop ends
// within n rounds.
__device__ __forceinline__ void unite(int* L, int a, int b) {
  while (true) {
    a = find_root(L, a);
    b = find_root(L, b);
    if (a == b) return;
    if (a > b) {
      const int t = a;
      a = b;
      b = t;
    }
    const int old = atomicMin(&L[b], a);
    if (old == b) return;
    b = old;
  }
}

// Each particle site joins its right and lower neighbours (periodic) when they
// are particle sites: every nearest-neighbour edge is visited once.
__global__ void __launch_bounds__(256) k_ccl_merge(int* L, long n, int nx, int ny) {
  const long i = long(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= n || L[i] < 0) return;
  const int x = int(i % nx), y = int(i / nx);
  const int r = y * nx + ((x + 1) & (nx - 1));
  const int d = ((y + 1) & (ny - 1)) * nx + x;
  if (L[r] >= 0) unite(L, int(i), r);
  if (L[d] >= 0) unite(L, int(i), d);
}

__global__ void __launch_bounds__(256) k_ccl_compress(int* L, long n) {
  const long i = long(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= n || L[i] < 0) return;
  L[i] = find_root(L, int(i));
}

// Per-particle sums, indexed by the label site: area, and of w = Phi_P: w,
// w dx, w dy, w dx^2, w dx dy, w dy^2 with (dx, dy) the minimum-image offset
// to the label site; wrap flag when an offset reaches half the box.  Runs of
// lanes with the same label are summed in the wave first (segmented scan), so
// each run issues one set of atomics.
template <typename T>
__global__ void __launch_bounds__(256) k_particle_accum(const T* __restrict__ phi, const int* __restrict__ L, long n,
                                                        int nx, int ny, int* __restrict__ area,
                                                        double* __restrict__ sums, int* __restrict__ wrap) {
  const long i = long(blockIdx.x) * blockDim.x + threadIdx.x;
  const int lane = threadIdx.x & 63;
  int key = -1;
  double v[6] = {0, 0, 0, 0, 0, 0};
  int cnt = 0, wr = 0;
  if (i < n) {
    key = L[i];
    if (key >= 0) {
      const T pP = phi[i] + phi[n + i];
      const double w = double(pP);
      const int x = int(i % nx), y = int(i / nx);
      const int rx = key % nx, ry = key / nx;
      const int dx = ((x - rx + nx + nx / 2) & (nx - 1)) - nx / 2;
      const int dy = ((y - ry + ny + ny / 2) & (ny - 1)) - ny / 2;
      v[0] = w;
      v[1] = w * dx;
      v[2] = w * dy;
      v[3] = w * dx * dx;
      v[4] = w * dx * dy;
      v[5] = w * dy * dy;
      cnt = 1;
      wr = (dx == -nx / 2 || dy == -ny / 2) ? 1 : 0;
    }
  }
  // start lane of this lane's run of equal keys
  const int prev = __shfl_up(key, 1, 64);
  int start = (lane == 0 || prev != key) ? lane : 0;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const int s2 = __shfl_up(start, o, 64);
    if (lane >= o) start = max(start, s2);
  }
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    double u[6];
#pragma unroll
    for (int k = 0; k < 6; ++k) u[k] = __shfl_up(v[k], o, 64);
    const int c2 = __shfl_up(cnt, o, 64);
    const int w2 = __shfl_up(wr, o, 64);
    if (lane - o >= start) {
#pragma unroll
      for (int k = 0; k < 6; ++k) v[k] += u[k];
      cnt += c2;
      wr |= w2;
    }
  }
  const int next = __shfl_down(key, 1, 64);
  const bool tail = lane == 63 || next != key;
  if (key >= 0 && tail) {
    atomicAdd(&area[key], cnt);
#pragma unroll
    for (int k = 0; k < 6; ++k) atomicAdd(&sums[6L * key + k], v[k]);
    if (wr) atomicOr(&wrap[key], 1);
  }
}

// Tracking: flags the particles (by label) that cover a site which was a
// particle site at the previous sample.  Every writer stores the same value.
__global__ void __launch_bounds__(256) k_overlap(const int* __restrict__ L, const unsigned char* __restrict__ prev,
                                                 int* __restrict__ ov, long n) {
  const long i = long(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i < n && prev[i]) {
    const int key = L[i];
    if (key >= 0) ov[key] = 1;
  }
}

// Tracking: the particle sites of this sample, for the next one.
__global__ void __launch_bounds__(256) k_store_prev(const int* __restrict__ L, unsigned char* __restrict__ prev,
                                                    long n) {
  const long i = long(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i < n) prev[i] = L[i] >= 0 ? 1 : 0;
}

// One entry per particle (label sites), in arrival order; the host sorts.
struct Particle {
  int label, area, wraps, born;
  double content, cx, cy, gxx, gxy, gyy, R, c_rel;
};

__global__ void __launch_bounds__(256) k_particle_list(const int* __restrict__ L, const int* __restrict__ area,
                                                       const double* __restrict__ sums, const int* __restrict__ wrap,
                                                       const int* __restrict__ ov, long n, int nx, int ny, int* count,
                                                       Particle* out, int cap) {
  const long i = long(blockIdx.x) * blockDim.x + threadIdx.x;
  const bool root = i < n && L[i] == int(i);
  // one counter update per wave
  const unsigned long long mask = __ballot(root);
  if (!mask) return;
  const int lane = threadIdx.x & 63;
  const int leader = __ffsll(mask) - 1;
  int base = 0;
  if (lane == leader) base = atomicAdd(count, __popcll(mask));
  base = __shfl(base, leader, 64);
  if (!root) return;
  const int k = base + __popcll(mask & ((1ull << lane) - 1));
  if (k >= cap) return;
  const double* s = sums + 6L * i;
  const double N = s[0];
  const double mx = s[1] / N, my = s[2] / N;
  const double gxx = s[3] / N - mx * mx, gxy = s[4] / N - mx * my, gyy = s[5] / N - my * my;
  const double tr = gxx + gyy;
  const double half = sqrt(0.25 * (gxx - gyy) * (gxx - gyy) + gxy * gxy);
  const double c = 2.0 * half;  // lambda_+ - lambda_-
  const double R = sqrt(fmax(tr, 0.0));
  Particle p;
  p.label = int(i);
  p.area = area[i];
  p.wraps = wrap[i];
  p.born = ov ? (ov[i] == 0 ? 1 : 0) : 0;
  p.content = N;
  const int rx = int(i % nx), ry = int(i / nx);
  double cx = fmod(double(rx) + mx, double(nx));
  double cy = fmod(double(ry) + my, double(ny));
  p.cx = cx < 0 ? cx + nx : cx;
  p.cy = cy < 0 ? cy + ny : cy;
  p.gxx = gxx;
  p.gxy = gxy;
  p.gyy = gyy;
  p.R = R;
  p.c_rel = tr > 0.0 ? c * c / (tr * tr) : 0.0;
  out[k] = p;
}

// Block partial sums of |Phi_P^a - Phi_P^b| (second value 0).
template <typename T>
__global__ void __launch_bounds__(256) k_sigma_delta(const T* __restrict__ pa, const T* __restrict__ pb, long n,
                                                     double* __restrict__ part) {
  const long i = long(blockIdx.x) * blockDim.x + threadIdx.x;
  double s = 0.0;
  if (i < n) {
    const T a = pa[i] + pa[n + i];
    const T b = pb[i] + pb[n + i];
    s = fabs(double(a) - double(b));
  }
  block_pair(s, 0.0, part);
}

// The first members of nblocks (<= 4096) partial pairs, added in block order
// by one thread (the order a host loop over the pairs takes): out[0].
__global__ void __launch_bounds__(256) k_sum_pairs_in_order(const double* __restrict__ part, int nblocks,
                                                            double* __restrict__ out) {
  __shared__ double s[4096];
  for (int k = threadIdx.x; k < nblocks; k += blockDim.x) s[k] = part[2 * k];
  __syncthreads();
  if (threadIdx.x == 0) {
    double sum = 0.0;
    for (int k = 0; k < nblocks; ++k) sum += s[k];
    out[0] = sum;
  }
}

}  // namespace obs
}  // namespace epdlb
