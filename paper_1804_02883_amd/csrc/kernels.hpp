// HIP kernels of the hybrid LB/EPD step (gfx950).
//
// Layout everywhere: structure-of-arrays planes, row-major [y][x] with x
// contiguous, nx x ny sites per plane, plane stride `plane` elements.
// T is the storage/arithmetic type (float or double); all grid-wide sums are
// accumulated in double and finished by the last block to arrive, in a fixed
// order, so results are deterministic.
#pragma once
#include "fft.hpp"

namespace epdlb {

// Device scalars shared between kernels (double).
enum Scal : int {
  kMeanA = 0, kMeanB = 1, kMeanS = 2,  // site means of the current omega planes
  kQS = 3, kGaugeS = 4,                 // Q_S and the constant it was computed with
  kQPf = 5, kQPb = 6,                   // Q_P from the forward and backward chains
  kNumScal = 8
};

// ---------------------------------------------------------------------------
// Deterministic grid reduction: per-block sums -> partials -> last block.
// ---------------------------------------------------------------------------
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// Reduces NV per-thread values over the block; thread 0 gets the sums.
template <int NV>
__device__ __forceinline__ void block_sum(double (&v)[NV], double* red /*[16*NV]*/) {
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  const int nw = (blockDim.x + 63) >> 6;
#pragma unroll
  for (int i = 0; i < NV; ++i) v[i] = wave_sum(v[i]);
  __syncthreads();
  if (lane == 0)
#pragma unroll
    for (int i = 0; i < NV; ++i) red[wid * NV + i] = v[i];
  __syncthreads();
  if (threadIdx.x == 0) {
#pragma unroll
    for (int i = 0; i < NV; ++i) {
      double s = 0.0;
      for (int w = 0; w < nw; ++w) s += red[w * NV + i];
      v[i] = s;
    }
  }
}

// Writes this block's NV sums to partials[slot*NV..], then, in the last block
// to finish, sums all nslots partials in slot order into out[0..NV-1] and
// resets the counter.  Returns true in the last block (all threads).
template <int NV>
__device__ bool grid_sum(double (&v)[NV], double* red, double* partials, int slot, int nslots,
                         unsigned* counter, double* out) {
  block_sum<NV>(v, red);
  __shared__ int is_last;
  if (threadIdx.x == 0) {
#pragma unroll
    for (int i = 0; i < NV; ++i) partials[slot * NV + i] = v[i];
    __threadfence();
    const unsigned prev = atomicAdd(counter, 1u);
    is_last = (prev == unsigned(nslots - 1));
  }
  __syncthreads();
  if (!is_last) return false;
  __threadfence();
  double acc[NV];
#pragma unroll
  for (int i = 0; i < NV; ++i) acc[i] = 0.0;
  for (int s = threadIdx.x; s < nslots; s += blockDim.x)
#pragma unroll
    for (int i = 0; i < NV; ++i) acc[i] += __hip_atomic_load(&partials[s * NV + i], __ATOMIC_RELAXED,
                                                             __HIP_MEMORY_SCOPE_AGENT);
  block_sum<NV>(acc, red);
  if (threadIdx.x == 0) {
#pragma unroll
    for (int i = 0; i < NV; ++i) out[i] = acc[i];
    *counter = 0u;
  }
  return true;
}

// ---------------------------------------------------------------------------
// Chain propagators: one contour step = row pass (K_x) + column pass (K_y).
// Both chains (forward = 0, backward = 1) run in the same launch.
// ---------------------------------------------------------------------------
template <typename T> struct PropArgs {
  const T* wA;
  const T* wB;
  const double* scal;     // kMeanA, kMeanB: gauge constants
  T* q[2];                // chain planes q_1..q_N at q[c] + (j-1)*plane
  T* tmp;                 // 2 planes: row-pass output per chain
  const T* mult_x;        // exp(-R_G^2 kx^2 ds)/nx in FFT order
  const T* mult_y;        // exp(-R_G^2 ky^2 ds)/ny
  const T2<T>* tw_x;      // exp(-2 pi i e/nx)
  const T2<T>* tw_y;
  int nx, ny;
  long plane;
  int j;                  // contour step: computes q_{j+1} from q_j
  int nsteps;             // N
  T a[2];                 // A-fraction of the segment each chain uses this step
  double* partials;       // last step: Q partial sums
  unsigned* counter;
  double* qout;           // last step: scal + kQPf (2 values)
  double dA;
  int nf;                 // transforms per block
};

template <typename T>
__device__ __forceinline__ T boltz(T wa, T wb, T a, T ca, T cb) {
  const T x = a * (wa - ca) + (T(1) - a) * (wb - cb);
  return exp(T(-0.5) * x);
}

template <typename T, int L>
__global__ void __launch_bounds__(256) k_prop_row(PropArgs<T> P) {
  using S = Split<L>;
  constexpr int N1 = S::N1, N2 = S::N2;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  T* lre = reinterpret_cast<T*>(smem_raw);
  RowMap<L> map;
  T* lim = lre + RowMap<L>::size(P.nf);
  const int f = threadIdx.x / N1, lane = threadIdx.x % N1;
  const int c = blockIdx.y;
  const int rp = blockIdx.x * P.nf + f;
  const bool active = rp < P.ny / 2;
  const long r0 = long(2 * rp) * P.nx, r1 = r0 + P.nx;
  const T a = P.a[c];
  const T ca = T(P.scal[kMeanA]), cb = T(P.scal[kMeanB]);
  const bool pureA = (a == T(1)), pureB = (a == T(0));
  const T* qin = P.q[c] + long(P.j - 1) * P.plane;
  T re[N2], im[N2];
#pragma unroll
  for (int n2 = 0; n2 < N2; ++n2) {
    T va = T(0), vb = T(0);
    if (active) {
      const int x = lane + N1 * n2;
      T ea, eb;
      if (pureA) {
        ea = exp(T(-0.5) * (P.wA[r0 + x] - ca));
        eb = exp(T(-0.5) * (P.wA[r1 + x] - ca));
      } else if (pureB) {
        ea = exp(T(-0.5) * (P.wB[r0 + x] - cb));
        eb = exp(T(-0.5) * (P.wB[r1 + x] - cb));
      } else {
        ea = boltz(P.wA[r0 + x], P.wB[r0 + x], a, ca, cb);
        eb = boltz(P.wA[r1 + x], P.wB[r1 + x], a, ca, cb);
      }
      if (P.j == 0) {
        va = ea;
        vb = eb;
      } else {
        va = ea * qin[r0 + x];
        vb = eb * qin[r1 + x];
      }
    }
    re[n2] = va;
    im[n2] = vb;
  }
  fft_forward<T, L>(re, im, f, lane, map, P.tw_x, lre, lim);
#pragma unroll
  for (int m = 0; m < S::M; ++m)
#pragma unroll
    for (int k1 = 0; k1 < N1; ++k1) {
      const T g = P.mult_x[freq_index<L>(lane, m, k1)];
      re[m * N1 + k1] *= g;
      im[m * N1 + k1] *= g;
    }
  fft_inverse<T, L>(re, im, f, lane, map, P.tw_x, lre, lim);
  if (active) {
    T* out = P.tmp + c * P.plane;
#pragma unroll
    for (int n2 = 0; n2 < N2; ++n2) {
      const int x = lane + N1 * n2;
      out[r0 + x] = re[n2];
      out[r1 + x] = im[n2];
    }
  }
}

template <typename T, int L, int NF>
__global__ void __launch_bounds__(256) k_prop_col(PropArgs<T> P) {
  using S = Split<L>;
  constexpr int N1 = S::N1, N2 = S::N2;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  __shared__ double red[16 * 1];
  T* lre = reinterpret_cast<T*>(smem_raw);
  ColMap<L, NF> map;
  T* lim = lre + ColMap<L, NF>::size();
  const int f = threadIdx.x % NF, lane = threadIdx.x / NF;
  const int c = blockIdx.y;
  const int cp = blockIdx.x * NF + f;
  const bool active = cp < P.nx / 2;
  const int x0 = 2 * cp;
  const T2<T>* in = reinterpret_cast<const T2<T>*>(P.tmp + c * P.plane);
  T re[N2], im[N2];
#pragma unroll
  for (int n2 = 0; n2 < N2; ++n2) {
    const int y = lane + N1 * n2;
    T2<T> v;
    v.x = T(0);
    v.y = T(0);
    if (active) v = in[(long(y) * P.nx + x0) >> 1];
    re[n2] = v.x;
    im[n2] = v.y;
  }
  fft_forward<T, L>(re, im, f, lane, map, P.tw_y, lre, lim);
#pragma unroll
  for (int m = 0; m < S::M; ++m)
#pragma unroll
    for (int k1 = 0; k1 < N1; ++k1) {
      const T g = P.mult_y[freq_index<L>(lane, m, k1)];
      re[m * N1 + k1] *= g;
      im[m * N1 + k1] *= g;
    }
  fft_inverse<T, L>(re, im, f, lane, map, P.tw_y, lre, lim);
  const T a = P.a[c];
  const T ca = T(P.scal[kMeanA]), cb = T(P.scal[kMeanB]);
  T2<T>* out = reinterpret_cast<T2<T>*>(P.q[c] + long(P.j) * P.plane);
  double qsum = 0.0;
  if (active) {
    const T2<T>* wa2 = reinterpret_cast<const T2<T>*>(P.wA);
    const T2<T>* wb2 = reinterpret_cast<const T2<T>*>(P.wB);
#pragma unroll
    for (int n2 = 0; n2 < N2; ++n2) {
      const int y = lane + N1 * n2;
      const long i2 = (long(y) * P.nx + x0) >> 1;
      T ea, eb;
      if (a == T(1)) {
        const T2<T> w = wa2[i2];
        ea = exp(T(-0.5) * (w.x - ca));
        eb = exp(T(-0.5) * (w.y - ca));
      } else if (a == T(0)) {
        const T2<T> w = wb2[i2];
        ea = exp(T(-0.5) * (w.x - cb));
        eb = exp(T(-0.5) * (w.y - cb));
      } else {
        const T2<T> u = wa2[i2], w = wb2[i2];
        ea = boltz(u.x, w.x, a, ca, cb);
        eb = boltz(u.y, w.y, a, ca, cb);
      }
      T2<T> o;
      o.x = re[n2] * ea;
      o.y = im[n2] * eb;
      out[i2] = o;
      qsum += double(o.x) + double(o.y);
    }
  }
  if (P.j == P.nsteps - 1) {
    // Q_P = dA * sum_r q_N(r) for this chain (block-uniform branch)
    double v[1] = {qsum};
    const int nslots = gridDim.x;
    double res[1];
    if (grid_sum<1>(v, red, P.partials + c * nslots, blockIdx.x, nslots, P.counter + c, res) &&
        threadIdx.x == 0)
      P.qout[c] = res[0] * P.dA;
  }
}

// ---------------------------------------------------------------------------
// Densities (contour integrals, solvent) and S = sum_I Phi_I/D_I - S~.
// ---------------------------------------------------------------------------
template <typename T> struct DensArgs {
  const T* q[2];
  const T* wS;
  const T* stilde;
  T* phi;        // 3 planes
  T* S;
  const double* scal;
  const T* wnA;  // node weights, N+1 each
  const T* wnB;
  long n;        // sites
  int N;
  double V, phiP, phiSbar, invDA, invDB, invDS;
};

template <typename T>
__global__ void __launch_bounds__(256) k_density(DensArgs<T> P) {
  const long i = long(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= P.n) return;
  const int N = P.N;
  T sA = T(0), sB = T(0);
  // node 0: q_0 = 1, node N: q'_0 = 1
  {
    const T prod = P.q[1][long(N - 1) * P.n + i];
    sA += P.wnA[0] * prod;
    sB += P.wnB[0] * prod;
  }
  for (int j = 1; j < N; ++j) {
    const T prod = P.q[0][long(j - 1) * P.n + i] * P.q[1][long(N - j - 1) * P.n + i];
    sA += P.wnA[j] * prod;
    sB += P.wnB[j] * prod;
  }
  {
    const T prod = P.q[0][long(N - 1) * P.n + i];
    sA += P.wnA[N] * prod;
    sB += P.wnB[N] * prod;
  }
  const T cP = T(P.V * P.phiP / P.scal[kQPf]);
  const T cS = T(P.V * P.phiSbar / P.scal[kQS]);
  const T pA = cP * sA, pB = cP * sB;
  const T pS = cS * exp(-(P.wS[i] - T(P.scal[kGaugeS])));
  P.phi[i] = pA;
  P.phi[P.n + i] = pB;
  P.phi[2 * P.n + i] = pS;
  if (P.S) P.S[i] = pA * T(P.invDA) + pB * T(P.invDB) + pS * T(P.invDS) - P.stilde[i];
}

// ---------------------------------------------------------------------------
// Site means of omega and Q_S (used at seeding and after host uploads).
// ---------------------------------------------------------------------------
template <typename T> struct StatArgs {
  const T* w;   // 3 planes
  long n;
  double* scal;
  double* partials;
  unsigned* counter;
  double dA;
};

template <typename T>
__global__ void __launch_bounds__(256) k_field_stats(StatArgs<T> P) {
  __shared__ double red[16 * 4];
  const double cS = P.scal[kMeanS];
  double v[4] = {0.0, 0.0, 0.0, 0.0};
  for (long i = long(blockIdx.x) * blockDim.x + threadIdx.x; i < P.n; i += long(gridDim.x) * blockDim.x) {
    v[0] += double(P.w[i]);
    v[1] += double(P.w[P.n + i]);
    const T ws = P.w[2 * P.n + i];
    v[2] += double(ws);
    v[3] += double(exp(-(ws - T(cS))));
  }
  double res[4];
  if (grid_sum<4>(v, red, P.partials, blockIdx.x, gridDim.x, P.counter, res) && threadIdx.x == 0) {
    P.scal[kMeanA] = res[0] / double(P.n);
    P.scal[kMeanB] = res[1] / double(P.n);
    P.scal[kMeanS] = res[2] / double(P.n);
    P.scal[kQS] = res[3] * P.dA;
    P.scal[kGaugeS] = cS;
  }
}

// ---------------------------------------------------------------------------
// Advection (donor cell) + chemical potential + EPD field update, fused.
// Tile TX x TY outputs; inputs staged with a 2-site halo in LDS.
// ---------------------------------------------------------------------------
constexpr int kTX = 32, kTY = 8;
constexpr int kHX = kTX + 4, kHY = kTY + 4;   // input region (halo 2)
constexpr int kMX = kTX + 2, kMY = kTY + 2;   // mu region (halo 1)

template <typename T> struct UpdArgs {
  const T* phi;    // 3 planes Phi^n
  const T* w;      // 3 planes omega^n
  const T* u;      // 2 planes u^{n-1} (lattice units)
  T* wout;         // 3 planes omega^{n+1}
  T* stilde;       // sum_I Phi~_I / D_I
  double* scal;
  double* partials;
  unsigned* counter;
  int nx, ny;
  long n;
  T chi[3][3];
  T kappa;
  T coef[3];       // D_I dt / dx^2
  T invD[3];
  int advect;      // 0: no flow coupling
  double dA;
};

template <typename T>
__global__ void __launch_bounds__(256) k_advect_update(UpdArgs<T> P) {
  __shared__ T sIn[8][kHY][kHX];   // phi[3], w[3], ux, uy
  __shared__ T sMu[3][kMY][kMX];
  __shared__ T sWt[3][kMY][kMX];
  __shared__ double red[16 * 4];
  const int tx0 = blockIdx.x * kTX, ty0 = blockIdx.y * kTY;
  const int tid = threadIdx.x;
  for (int e = tid; e < kHX * kHY; e += blockDim.x) {
    const int lx = e % kHX, ly = e / kHX;
    const int gx = (tx0 + lx - 2 + P.nx) & (P.nx - 1);
    const int gy = (ty0 + ly - 2 + P.ny) & (P.ny - 1);
    const long gi = long(gy) * P.nx + gx;
#pragma unroll
    for (int I = 0; I < 3; ++I) {
      sIn[I][ly][lx] = P.phi[I * P.n + gi];
      sIn[3 + I][ly][lx] = P.w[I * P.n + gi];
    }
    if (P.advect) {
      sIn[6][ly][lx] = P.u[gi];
      sIn[7][ly][lx] = P.u[P.n + gi];
    } else {
      sIn[6][ly][lx] = T(0);
      sIn[7][ly][lx] = T(0);
    }
  }
  __syncthreads();
  // advected fields and mu~ on the halo-1 region
  for (int e = tid; e < kMX * kMY; e += blockDim.x) {
    const int mx = e % kMX, my = e / kMX;
    const int lx = mx + 1, ly = my + 1;  // position in sIn
    const T uxc = sIn[6][ly][lx], uyc = sIn[7][ly][lx];
    // face velocities
    const T uxe = T(0.5) * (uxc + sIn[6][ly][lx + 1]);
    const T uxw = T(0.5) * (sIn[6][ly][lx - 1] + uxc);
    const T uyn = T(0.5) * (uyc + sIn[7][ly + 1][lx]);
    const T uys = T(0.5) * (sIn[7][ly - 1][lx] + uyc);
    T pt[3], wt[3];
#pragma unroll
    for (int I = 0; I < 3; ++I) {
      const T c = sIn[I][ly][lx];
      const T Je = uxe >= T(0) ? uxe * c : uxe * sIn[I][ly][lx + 1];
      const T Jw = uxw >= T(0) ? uxw * sIn[I][ly][lx - 1] : uxw * c;
      const T Jn = uyn >= T(0) ? uyn * c : uyn * sIn[I][ly + 1][lx];
      const T Js = uys >= T(0) ? uys * sIn[I][ly - 1][lx] : uys * c;
      pt[I] = c - (Je - Jw) - (Jn - Js);
      const T w = sIn[3 + I][ly][lx];
      const T upx = uxc > T(0) ? uxc : T(0), umx = uxc < T(0) ? uxc : T(0);
      const T upy = uyc > T(0) ? uyc : T(0), umy = uyc < T(0) ? uyc : T(0);
      wt[I] = w - (upx * (w - sIn[3 + I][ly][lx - 1]) + umx * (sIn[3 + I][ly][lx + 1] - w)) -
              (upy * (w - sIn[3 + I][ly - 1][lx]) + umy * (sIn[3 + I][ly + 1][lx] - w));
    }
    const T tot = pt[0] + pt[1] + pt[2];
#pragma unroll
    for (int I = 0; I < 3; ++I) {
      T acc = T(0);
#pragma unroll
      for (int J = 0; J < 3; ++J)
        if (J != I) acc += P.chi[I][J] * pt[J];
      sMu[I][my][mx] = acc - wt[I] + P.kappa * (tot - T(1));
      sWt[I][my][mx] = wt[I];
    }
    if (mx >= 1 && mx <= kTX && my >= 1 && my <= kTY) {
      const long gi = long(ty0 + my - 1) * P.nx + (tx0 + mx - 1);
      P.stilde[gi] = pt[0] * P.invD[0] + pt[1] * P.invD[1] + pt[2] * P.invD[2];
    }
  }
  __syncthreads();
  double v[4] = {0.0, 0.0, 0.0, 0.0};
  const T cS = T(P.scal[kMeanS]);
  {
    const int ox = tid % kTX, oy = tid / kTX;  // 256 threads = 32 x 8 outputs
    const int mx = ox + 1, my = oy + 1;
    const long gi = long(ty0 + oy) * P.nx + (tx0 + ox);
#pragma unroll
    for (int I = 0; I < 3; ++I) {
      const T lap = sMu[I][my][mx + 1] + sMu[I][my][mx - 1] + sMu[I][my + 1][mx] +
                    sMu[I][my - 1][mx] - T(4) * sMu[I][my][mx];
      const T wn = sWt[I][my][mx] - P.coef[I] * lap;
      P.wout[I * P.n + gi] = wn;
      v[I] = double(wn);
      if (I == 2) v[3] = double(exp(-(wn - cS)));
    }
  }
  const int slot = blockIdx.y * gridDim.x + blockIdx.x;
  const int nslots = gridDim.x * gridDim.y;
  double res[4];
  if (grid_sum<4>(v, red, P.partials, slot, nslots, P.counter, res) && threadIdx.x == 0) {
    P.scal[kGaugeS] = double(cS);
    P.scal[kMeanA] = res[0] / double(P.n);
    P.scal[kMeanB] = res[1] / double(P.n);
    P.scal[kMeanS] = res[2] / double(P.n);
    P.scal[kQS] = res[3] * P.dA;
  }
}

// ---------------------------------------------------------------------------
// Force reconstruction in k-space: row FFT of S, column FFT x multiplier x
// inverse, row inverse giving f_x + i f_y; external force; lattice units.
// ---------------------------------------------------------------------------
template <typename T> struct ForceArgs {
  const T* S;
  T2<T>* spec;          // nx*ny complex work plane
  T* F;                 // 2 planes (lattice units)
  const T2<T>* tw_x;
  const T2<T>* tw_y;
  int nx, ny;
  long n;
  double kx0, ky0;      // 2 pi/(nx dx), 2 pi/(ny dx)
  double pref;          // (kT/v)/dt / (nx ny)
  double conv;          // dt^2/dx (physical -> lattice), 0 if uncoupled
  double gext;          // external force amplitude in lattice units
  int nf;
};

template <typename T, int L>
__global__ void __launch_bounds__(256) k_force_row_fwd(ForceArgs<T> P) {
  using S = Split<L>;
  constexpr int N1 = S::N1, N2 = S::N2;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  T* lre = reinterpret_cast<T*>(smem_raw);
  RowMap<L> map;
  T* lim = lre + RowMap<L>::size(P.nf);
  const int f = threadIdx.x / N1, lane = threadIdx.x % N1;
  const int y = blockIdx.x * P.nf + f;
  const bool active = y < P.ny;
  T re[N2], im[N2];
#pragma unroll
  for (int n2 = 0; n2 < N2; ++n2) {
    re[n2] = active ? P.S[long(y) * P.nx + lane + N1 * n2] : T(0);
    im[n2] = T(0);
  }
  fft_forward<T, L>(re, im, f, lane, map, P.tw_x, lre, lim);
  if (active) {
#pragma unroll
    for (int m = 0; m < S::M; ++m)
#pragma unroll
      for (int k1 = 0; k1 < N1; ++k1) {
        T2<T> o;
        o.x = re[m * N1 + k1];
        o.y = im[m * N1 + k1];
        P.spec[long(y) * P.nx + freq_index<L>(lane, m, k1)] = o;
      }
  }
}

template <typename T, int L, int NF>
__global__ void __launch_bounds__(256) k_force_col(ForceArgs<T> P) {
  using S = Split<L>;
  constexpr int N1 = S::N1, N2 = S::N2;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  T* lre = reinterpret_cast<T*>(smem_raw);
  ColMap<L, NF> map;
  T* lim = lre + ColMap<L, NF>::size();
  const int f = threadIdx.x % NF, lane = threadIdx.x / NF;
  const int kxi = blockIdx.x * NF + f;   // column = x wavenumber index
  const bool active = kxi < P.nx;
  T re[N2], im[N2];
#pragma unroll
  for (int n2 = 0; n2 < N2; ++n2) {
    T2<T> v;
    v.x = T(0);
    v.y = T(0);
    if (active) v = P.spec[long(lane + N1 * n2) * P.nx + kxi];
    re[n2] = v.x;
    im[n2] = v.y;
  }
  fft_forward<T, L>(re, im, f, lane, map, P.tw_y, lre, lim);
  const int mx = kxi < P.nx / 2 ? kxi : kxi - P.nx;
  const double kx = P.kx0 * mx;
  const bool nyq_x = (kxi == P.nx / 2);
#pragma unroll
  for (int m = 0; m < S::M; ++m)
#pragma unroll
    for (int k1 = 0; k1 < N1; ++k1) {
      const int kyi = freq_index<L>(lane, m, k1);
      const int my = kyi < P.ny / 2 ? kyi : kyi - P.ny;
      const double ky = P.ky0 * my;
      const double k2 = kx * kx + ky * ky;
      const double inv = k2 > 0.0 ? P.pref / k2 : 0.0;
      const T al = nyq_x ? T(0) : T(inv * kx);
      const T be = (kyi == P.ny / 2) ? T(0) : T(inv * ky);
      const T sr = re[m * N1 + k1], si = im[m * N1 + k1];
      // G = i al S + i (i be S) = (i al - be) S
      re[m * N1 + k1] = -al * si - be * sr;
      im[m * N1 + k1] = al * sr - be * si;
    }
  fft_inverse<T, L>(re, im, f, lane, map, P.tw_y, lre, lim);
  if (active) {
#pragma unroll
    for (int n2 = 0; n2 < N2; ++n2) {
      T2<T> o;
      o.x = re[n2];
      o.y = im[n2];
      P.spec[long(lane + N1 * n2) * P.nx + kxi] = o;
    }
  }
}

template <typename T, int L>
__global__ void __launch_bounds__(256) k_force_row_inv(ForceArgs<T> P) {
  using S = Split<L>;
  constexpr int N1 = S::N1, N2 = S::N2;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  T* lre = reinterpret_cast<T*>(smem_raw);
  RowMap<L> map;
  T* lim = lre + RowMap<L>::size(P.nf);
  const int f = threadIdx.x / N1, lane = threadIdx.x % N1;
  const int y = blockIdx.x * P.nf + f;
  const bool active = y < P.ny;
  T re[N2], im[N2];
#pragma unroll
  for (int m = 0; m < S::M; ++m)
#pragma unroll
    for (int k1 = 0; k1 < N1; ++k1) {
      T2<T> v;
      v.x = T(0);
      v.y = T(0);
      if (active) v = P.spec[long(y) * P.nx + freq_index<L>(lane, m, k1)];
      re[m * N1 + k1] = v.x;
      im[m * N1 + k1] = v.y;
    }
  fft_inverse<T, L>(re, im, f, lane, map, P.tw_x, lre, lim);
  if (active) {
    const T conv = T(P.conv);
    const T fext = T(y < P.ny / 2 ? -P.gext : P.gext);
#pragma unroll
    for (int n2 = 0; n2 < N2; ++n2) {
      const long i = long(y) * P.nx + lane + N1 * n2;
      P.F[i] = re[n2] * conv + fext;
      P.F[P.n + i] = im[n2] * conv;
    }
  }
}

// ---------------------------------------------------------------------------
// D2Q9 lattice Boltzmann: pull stream + BGK collision with second-order force.
// ---------------------------------------------------------------------------
template <typename T> struct LbArgs {
  const T* fin;    // 9 planes f* (previous post-collision)
  T* fout;         // 9 planes
  const T* F;      // 2 planes
  T* rho;
  T* u;            // 2 planes
  int nx, ny;
  long n;
  T omega;         // 1/tau
  T fpre;          // 1 - 1/(2 tau)
};

template <typename T>
__global__ void __launch_bounds__(256) k_lb(LbArgs<T> P) {
  const long i = long(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= P.n) return;
  const int x = int(i & (P.nx - 1));
  const int y = int(i / P.nx);
  const int xm = (x - 1) & (P.nx - 1), xp = (x + 1) & (P.nx - 1);
  const long ym = long((y - 1) & (P.ny - 1)) * P.nx, yp = long((y + 1) & (P.ny - 1)) * P.nx;
  const long yc = long(y) * P.nx;
  // pull: f_i(x) = f*_i(x - c_i); c = (0,0),(1,0),(0,1),(-1,0),(0,-1),(1,1),(-1,1),(-1,-1),(1,-1)
  T f[9];
  f[0] = P.fin[0 * P.n + yc + x];
  f[1] = P.fin[1 * P.n + yc + xm];
  f[2] = P.fin[2 * P.n + ym + x];
  f[3] = P.fin[3 * P.n + yc + xp];
  f[4] = P.fin[4 * P.n + yp + x];
  f[5] = P.fin[5 * P.n + ym + xm];
  f[6] = P.fin[6 * P.n + ym + xp];
  f[7] = P.fin[7 * P.n + yp + xp];
  f[8] = P.fin[8 * P.n + yp + xm];
  const T Fx = P.F[i], Fy = P.F[P.n + i];
  const T rho = f[0] + f[1] + f[2] + f[3] + f[4] + f[5] + f[6] + f[7] + f[8];
  const T jx = f[1] - f[3] + f[5] - f[6] - f[7] + f[8];
  const T jy = f[2] - f[4] + f[5] + f[6] - f[7] - f[8];
  const T ir = T(1) / rho;
  const T ux = (jx + T(0.5) * Fx) * ir;
  const T uy = (jy + T(0.5) * Fy) * ir;
  const T usq = ux * ux + uy * uy;
  constexpr int cx[9] = {0, 1, 0, -1, 0, 1, -1, -1, 1};
  constexpr int cy[9] = {0, 0, 1, 0, -1, 1, 1, -1, -1};
#pragma unroll
  for (int k = 0; k < 9; ++k) {
    const T w = k == 0 ? T(4.0 / 9.0) : (k < 5 ? T(1.0 / 9.0) : T(1.0 / 36.0));
    const T cu = T(cx[k]) * ux + T(cy[k]) * uy;
    const T feq = w * rho * (T(1) + T(3) * cu + T(4.5) * cu * cu - T(1.5) * usq);
    const T cF = T(cx[k]) * Fx + T(cy[k]) * Fy;
    const T cmuF = (T(cx[k]) - ux) * Fx + (T(cy[k]) - uy) * Fy;
    const T src = w * (T(3) * cmuF + T(9) * cu * cF);
    P.fout[k * P.n + i] = f[k] - (f[k] - feq) * P.omega + P.fpre * src;
  }
  P.rho[i] = rho;
  P.u[i] = ux;
  P.u[P.n + i] = uy;
}

}  // namespace epdlb
