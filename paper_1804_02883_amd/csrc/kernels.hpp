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
  kGext = 7,                            // reverse-Poiseuille force amplitude, lattice units
  // surrogate mode (maxima of non-negative values, updated atomically)
  kNnResid = 8,                         // max |sum Phi - 1| of surrogate steps since the last check
  kResidEx = 9,                         // max |sum Phi - 1| of the last exact step
  kNnErrLast = 10,                      // max |Phi_NN - Phi_exact| (A, B) at the last exact step
  kNnErr = 11,                          // the same, maximum over all exact steps
  kNnErrUse = 12,                       // the same, over exact steps that ended surrogate steps
  kNumScal = 13
};

// ---------------------------------------------------------------------------
// XCD-aware tile order.  Workgroups are handed to the 8 XCDs of an MI355X
// round-robin by linear id, and each XCD has its own L2.  Remapping so that
// XCD k processes the k-th contiguous range of logical tiles keeps
// neighbouring tiles (which share cache lines and halos) in one L2.
// ---------------------------------------------------------------------------
constexpr int kNumXcd = 8;

// Replicas of one grid shape share a launch: replica z's planes, tables and
// scalars sit `rs` bytes after replica z-1's (blockIdx.z = z).
template <class X>
__device__ __forceinline__ X* sh(X* p, long off) {
  return (X*)((const char*)p + off);
}
__device__ __forceinline__ int xcd_tile(int linear, int total) {
  if (total % kNumXcd) return linear;
  return (linear % kNumXcd) * (total / kNumXcd) + linear / kNumXcd;
}

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

// Writes this block's NV sums to partials[slot*NV + i].  A later kernel
// (or a later stage of the consumer) adds the partials in slot order, so the
// grid-wide sums are deterministic and need no device-scope fences here.
template <int NV>
__device__ __forceinline__ void block_partial(double (&v)[NV], double* red, double* partials, int slot) {
  block_sum<NV>(v, red);
  if (threadIdx.x == 0)
#pragma unroll
    for (int i = 0; i < NV; ++i) partials[slot * NV + i] = v[i];
}

// Sums nslots partials of NV values each, in slot order, over one block.
// Each thread loads four of its slots at a time before adding them in order,
// so the loads of a batch are in flight together.
template <int NV>
__device__ __forceinline__ void sum_partials(const double* partials, int nslots, double (&acc)[NV],
                                             double* red) {
#pragma unroll
  for (int i = 0; i < NV; ++i) acc[i] = 0.0;
  const int step = blockDim.x;
  for (int s0 = threadIdx.x; s0 < nslots; s0 += 4 * step) {
    double v[4][NV];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const int s = s0 + k * step;
#pragma unroll
      for (int i = 0; i < NV; ++i) v[k][i] = s < nslots ? partials[s * NV + i] : 0.0;
    }
#pragma unroll
    for (int k = 0; k < 4; ++k)
      if (s0 + k * step < nslots)
#pragma unroll
        for (int i = 0; i < NV; ++i) acc[i] += v[k][i];
  }
  block_sum<NV>(acc, red);
}

// Finishes the field statistics: partials of (sum w_A, sum w_B, sum w_S,
// sum exp(-(w_S - gauge))) -> means, Q_S and the gauge it used.  One block.
__global__ void __launch_bounds__(256) k_finish_stats(const double* partials, int nslots, double* scal,
                                                      long n, double dA, long rs) {
  __shared__ double red[16 * 4];
  partials = sh(partials, long(blockIdx.z) * rs);
  scal = sh(scal, long(blockIdx.z) * rs);
  double acc[4];
  sum_partials<4>(partials, nslots, acc, red);
  if (threadIdx.x == 0) {
    scal[kGaugeS] = scal[kMeanS];  // the constant the exponentials were taken with
    scal[kMeanA] = acc[0] / double(n);
    scal[kMeanB] = acc[1] / double(n);
    scal[kMeanS] = acc[2] / double(n);
    scal[kQS] = acc[3] * dA;
  }
}

// ---------------------------------------------------------------------------
// Chain propagators.  K = K_x K_y = K_y K_x, so each contour step applies its
// two one-dimensional convolutions in alternating order: even steps x then y,
// odd steps y then x.  The last convolution of step a and the first one of
// step a+1 then share an orientation and run in ONE kernel with q_{a+1}
// stored in between: N + 1 launches for N contour steps, both chains per
// launch (blockIdx.y = chain; 0 forward, 1 backward).
// ---------------------------------------------------------------------------
template <typename T> struct PropArgs {
  const T* wA;
  const T* wB;
  const T* EA;            // exp(-(w_A - c_A)/2), written once per propagation
  const T* EB;            // exp(-(w_B - c_B)/2)
  const double* scal;     // kMeanA, kMeanB: gauge constants
  T* q[2];                // q_1..q_N of chain c at q[c] + (j-1)*plane
  T* tmp;                 // 2 planes (per chain): data between the two convolutions of a step
  const T* mult_x;        // exp(-R_G^2 kx^2 ds)/nx in FFT order
  const T* mult_y;        // exp(-R_G^2 ky^2 ds)/ny
  const T2<T>* tw_x;      // exp(-2 pi i e/nx)
  const T2<T>* tw_y;
  int nx, ny;
  long plane;
  int a;                  // contour step finished by the first convolution
  int first;              // input is E(step 0) (q_0 = 1) instead of tmp
  int mid;                // after convolution 1: x E(step a), store q_{a+1}
  int second;             // then x E(step a+1), convolution 2, store tmp
  int last;               // with mid: partial sums of q_N for Q_P
  T frac[2][2];           // A fraction of the segment used by chain c at step a (+0/+1)
  double* partials;       // last: per-block sums of q_N, chain c at [c*gridDim.x]
  int nf;                 // transforms per block (row kernels)
  int nrep;               // replicas in the launch (gridDim.z)
  long rs;                // replica stride in bytes
  __device__ void shift(long o) {
    wA = sh(wA, o), wB = sh(wB, o), EA = sh(EA, o), EB = sh(EB, o), scal = sh(scal, o);
    q[0] = sh(q[0], o), q[1] = sh(q[1], o), tmp = sh(tmp, o), mult_x = sh(mult_x, o);
    mult_y = sh(mult_y, o), tw_x = sh(tw_x, o), tw_y = sh(tw_y, o);
    partials = sh(partials, o);
  }
};


template <typename T>
__device__ __forceinline__ T boltz(T wa, T wb, T a, T ca, T cb) {
  const T x = a * (wa - ca) + (T(1) - a) * (wb - cb);
  return exp(T(-0.5) * x);
}

// Half-step Boltzmann factor exp(-(w_seg - c_seg)/2) of a segment with A
// fraction `fr` at flat index i: a plane load for pure A or B segments, the
// mixed junction segment from the potentials.
template <typename T>
__device__ __forceinline__ T efactor(const PropArgs<T>& P, T fr, T ca, T cb, long i) {
  if (fr == T(1)) return P.EA[i];
  if (fr == T(0)) return P.EB[i];
  return boltz(P.wA[i], P.wB[i], fr, ca, cb);
}
template <typename T>
__device__ __forceinline__ T2<T> efactor2(const PropArgs<T>& P, T fr, T ca, T cb, long i2) {
  if (fr == T(1)) return reinterpret_cast<const T2<T>*>(P.EA)[i2];
  if (fr == T(0)) return reinterpret_cast<const T2<T>*>(P.EB)[i2];
  const T2<T> u = reinterpret_cast<const T2<T>*>(P.wA)[i2];
  const T2<T> w = reinterpret_cast<const T2<T>*>(P.wB)[i2];
  T2<T> e;
  e.x = boltz(u.x, w.x, fr, ca, cb);
  e.y = boltz(u.y, w.y, fr, ca, cb);
  return e;
}


// Convolution with the real, even multiplier g in the lane layout.
template <typename T, int L, int R, class V>
__device__ __forceinline__ void convolve(T* re, T* im, int j, const V& lds, const Twiddles<T, L, R>& twf,
                                         const Twiddles<T, L, R>& twi, const T* g) {
  fft_forward(re, im, j, lds, twf);
#pragma unroll
  for (int m = 0; m < R; ++m) {
    re[m] *= g[m];
    im[m] *= g[m];
  }
  fft_inverse(re, im, j, lds, twi);
}

// x-oriented kernel: rows 2rp and 2rp+1 of one chain packed as one complex
// row (the multiplier is real and even, so the two real rows stay apart).
template <typename T, int L, int R>
__global__ void __launch_bounds__(512) k_prop_row(PropArgs<T> P) {
  constexpr int TL = L / R;
  using V = LdsView<T, L, R, true, 1>;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  __shared__ double red[16 * 1];
  const int f = threadIdx.x / TL, j = threadIdx.x % TL;
  V lds{reinterpret_cast<T2<T>*>(smem_raw), f};
  P.shift(long(blockIdx.z) * P.rs);
  const int c = blockIdx.y;
  const int rp = blockIdx.x * P.nf + f;
  const bool active = rp < P.ny / 2;
  const long r0 = long(2 * rp) * P.nx, r1 = r0 + P.nx;
  const T ca = T(P.scal[kMeanA]), cb = T(P.scal[kMeanB]);
  const T fr0 = c == 0 ? P.frac[0][0] : P.frac[1][0], fr1 = c == 0 ? P.frac[0][1] : P.frac[1][1];
  Twiddles<T, L, R> twf, twi;
  load_fwd_twiddles(twf, j, P.tw_x);
  load_inv_twiddles(twi, j, P.tw_x);
  T g[R];
#pragma unroll
  for (int m = 0; m < R; ++m) g[m] = P.mult_x[j + TL * m];
  T* tmp = P.tmp + c * P.plane;
  // half-step factors of step a (loaded early: they overlap the first convolution)
  T ea[R], eb[R];
  if (P.first) {
    // the first pass takes its factors from the potentials and leaves the
    // factor planes of the later passes: A's from the forward chain's blocks,
    // B's from the backward chain's (the same values a separate pass gave)
    T* Ep = const_cast<T*>(c == 0 ? P.EA : P.EB);
    const T pure = c == 0 ? T(1) : T(0);
#pragma unroll
    for (int m = 0; m < R; ++m) {
      const int x = j + TL * m;
      ea[m] = eb[m] = T(0);
      if (active) {
        const T wa0 = P.wA[r0 + x], wb0 = P.wB[r0 + x], wa1 = P.wA[r1 + x], wb1 = P.wB[r1 + x];
        const T p0 = boltz(wa0, wb0, pure, ca, cb), p1 = boltz(wa1, wb1, pure, ca, cb);
        Ep[r0 + x] = p0;
        Ep[r1 + x] = p1;
        ea[m] = fr0 == pure ? p0 : boltz(wa0, wb0, fr0, ca, cb);
        eb[m] = fr0 == pure ? p1 : boltz(wa1, wb1, fr0, ca, cb);
      }
    }
  } else {
#pragma unroll
    for (int m = 0; m < R; ++m) {
      const int x = j + TL * m;
      ea[m] = active && P.mid ? efactor(P, fr0, ca, cb, r0 + x) : T(0);
      eb[m] = active && P.mid ? efactor(P, fr0, ca, cb, r1 + x) : T(0);
    }
  }
  T re[R], im[R];
#pragma unroll
  for (int m = 0; m < R; ++m) {
    const int x = j + TL * m;
    if (P.first) {
      re[m] = ea[m];
      im[m] = eb[m];
    } else {
      re[m] = active ? tmp[r0 + x] : T(0);
      im[m] = active ? tmp[r1 + x] : T(0);
    }
  }
  convolve(re, im, j, lds, twf, twi, g);
  double qsum = 0.0;
  if (P.mid) {
    T* qo = (c == 0 ? P.q[0] : P.q[1]) + long(P.a) * P.plane;
#pragma unroll
    for (int m = 0; m < R; ++m) {
      const int x = j + TL * m;
      re[m] *= ea[m];
      im[m] *= eb[m];
      if (active) {
        qo[r0 + x] = re[m];
        qo[r1 + x] = im[m];
      }
      qsum += double(re[m]) + double(im[m]);
    }
    if (P.second) {
      if (fr1 != fr0) {
#pragma unroll
        for (int m = 0; m < R; ++m) {
          const int x = j + TL * m;
          ea[m] = active ? efactor(P, fr1, ca, cb, r0 + x) : T(0);
          eb[m] = active ? efactor(P, fr1, ca, cb, r1 + x) : T(0);
        }
      }
#pragma unroll
      for (int m = 0; m < R; ++m) {
        re[m] *= ea[m];
        im[m] *= eb[m];
      }
      convolve(re, im, j, lds, twf, twi, g);
    }
  }
  if ((!P.mid || P.second) && active) {
#pragma unroll
    for (int m = 0; m < R; ++m) {
      const int x = j + TL * m;
      tmp[r0 + x] = re[m];
      tmp[r1 + x] = im[m];
    }
  }
  if (P.last) {
    double v[1] = {qsum};
    block_partial<1>(v, red, P.partials + c * gridDim.x, blockIdx.x);
  }
}

// y-oriented kernel: columns 2cp and 2cp+1 packed as one complex column; NF
// transforms per block interleaved lane by lane so that each global access
// of a wavefront covers NF consecutive column pairs.
template <typename T, int L, int R, int NF>
__global__ void __launch_bounds__(512) k_prop_col(PropArgs<T> P) {
  constexpr int TL = L / R;
  using V = LdsView<T, L, R, false, NF>;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  __shared__ double red[16 * 1];
  const int f = threadIdx.x % NF, j = threadIdx.x / NF;
  V lds{reinterpret_cast<T2<T>*>(smem_raw), f};
  P.shift(long(blockIdx.z) * P.rs);
  const int lt = xcd_tile(blockIdx.y * gridDim.x + blockIdx.x, gridDim.x * gridDim.y);
  const int c = lt / gridDim.x, tile = lt % gridDim.x;
  const int cp = tile * NF + f;
  const bool active = cp < P.nx / 2;
  const int x0 = 2 * cp;
  const T ca = T(P.scal[kMeanA]), cb = T(P.scal[kMeanB]);
  const T fr0 = c == 0 ? P.frac[0][0] : P.frac[1][0], fr1 = c == 0 ? P.frac[0][1] : P.frac[1][1];
  Twiddles<T, L, R> twf, twi;
  load_fwd_twiddles(twf, j, P.tw_y);
  load_inv_twiddles(twi, j, P.tw_y);
  T g[R];
#pragma unroll
  for (int m = 0; m < R; ++m) g[m] = P.mult_y[j + TL * m];
  T2<T>* tmp2 = reinterpret_cast<T2<T>*>(P.tmp + c * P.plane);
  T2<T> e[R];
#pragma unroll
  for (int m = 0; m < R; ++m) {
    const long i2 = (long(j + TL * m) * P.nx + x0) >> 1;
    e[m].x = T(0);
    e[m].y = T(0);
    if (active && (P.first || P.mid)) e[m] = efactor2(P, fr0, ca, cb, i2);
  }
  T re[R], im[R];
#pragma unroll
  for (int m = 0; m < R; ++m) {
    const long i2 = (long(j + TL * m) * P.nx + x0) >> 1;
    if (P.first) {
      re[m] = e[m].x;
      im[m] = e[m].y;
    } else {
      T2<T> v;
      v.x = T(0);
      v.y = T(0);
      if (active) v = tmp2[i2];
      re[m] = v.x;
      im[m] = v.y;
    }
  }
  convolve(re, im, j, lds, twf, twi, g);
  double qsum = 0.0;
  if (P.mid) {
    T2<T>* qo = reinterpret_cast<T2<T>*>((c == 0 ? P.q[0] : P.q[1]) + long(P.a) * P.plane);
#pragma unroll
    for (int m = 0; m < R; ++m) {
      const long i2 = (long(j + TL * m) * P.nx + x0) >> 1;
      re[m] *= e[m].x;
      im[m] *= e[m].y;
      T2<T> o;
      o.x = re[m];
      o.y = im[m];
      if (active) qo[i2] = o;
      qsum += double(o.x) + double(o.y);
    }
    if (P.second) {
      if (fr1 != fr0) {
#pragma unroll
        for (int m = 0; m < R; ++m) {
          const long i2 = (long(j + TL * m) * P.nx + x0) >> 1;
          if (active) e[m] = efactor2(P, fr1, ca, cb, i2);
        }
      }
#pragma unroll
      for (int m = 0; m < R; ++m) {
        re[m] *= e[m].x;
        im[m] *= e[m].y;
      }
      convolve(re, im, j, lds, twf, twi, g);
    }
  }
  if ((!P.mid || P.second) && active) {
#pragma unroll
    for (int m = 0; m < R; ++m) {
      const long i2 = (long(j + TL * m) * P.nx + x0) >> 1;
      T2<T> o;
      o.x = re[m];
      o.y = im[m];
      tmp2[i2] = o;
    }
  }
  if (P.last) {
    double v[1] = {qsum};
    block_partial<1>(v, red, P.partials + c * gridDim.x, tile);
  }
}

// ---------------------------------------------------------------------------
// Densities (contour integrals, solvent) and S = sum_I Phi_I/D_I - S~.
// ---------------------------------------------------------------------------
template <typename T> struct DensArgs {
  const double* qpart;  // per-block sums of q_N from the last column pass, 2 chains
  int nqpart;           // blocks per chain
  double dA;
  double* scal_out;     // scal: receives Q_P (both chains)
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
  int nrep;
  long rs;
  __device__ void shift(long o) {
    qpart = sh(qpart, o), scal_out = sh(scal_out, o), q[0] = sh(q[0], o), q[1] = sh(q[1], o);
    wS = sh(wS, o), stilde = sh(stilde, o), phi = sh(phi, o), scal = sh(scal, o);
    wnA = sh(wnA, o), wnB = sh(wnB, o);
    if (S) S = sh(S, o);
  }
};

template <typename T>
__global__ void __launch_bounds__(256) k_density(DensArgs<T> P) {
  __shared__ double red[16 * 2];
  __shared__ double qp_s;
  P.shift(long(blockIdx.z) * P.rs);
  {
    // Q_P from the column-pass partials, in fixed order (same in every block)
    double acc[2];
    double tmp[2] = {0.0, 0.0};
    for (int s = threadIdx.x; s < P.nqpart; s += blockDim.x) {
      tmp[0] += P.qpart[s];
      tmp[1] += P.qpart[P.nqpart + s];
    }
    acc[0] = tmp[0];
    acc[1] = tmp[1];
    block_sum<2>(acc, red);
    if (threadIdx.x == 0) {
      qp_s = acc[0] * P.dA;
      if (blockIdx.x == 0) {
        P.scal_out[kQPf] = acc[0] * P.dA;
        P.scal_out[kQPb] = acc[1] * P.dA;
      }
    }
    __syncthreads();
  }
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
  const T cP = T(P.V * P.phiP / qp_s);
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
  int nrep;
  long rs;
  __device__ void shift(long o) { w = sh(w, o), scal = sh(scal, o), partials = sh(partials, o); }
};

template <typename T>
__global__ void __launch_bounds__(256) k_field_stats(StatArgs<T> P) {
  __shared__ double red[16 * 4];
  P.shift(long(blockIdx.z) * P.rs);
  const double cS = P.scal[kMeanS];
  double v[4] = {0.0, 0.0, 0.0, 0.0};
  for (long i = long(blockIdx.x) * blockDim.x + threadIdx.x; i < P.n; i += long(gridDim.x) * blockDim.x) {
    v[0] += double(P.w[i]);
    v[1] += double(P.w[P.n + i]);
    const T ws = P.w[2 * P.n + i];
    v[2] += double(ws);
    v[3] += double(exp(-(ws - T(cS))));
  }
  block_partial<4>(v, red, P.partials, blockIdx.x);
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
  const double* scal;
  double* partials;
  int nx, ny;
  long n;
  T chi[3][3];
  T kappa;
  T coef[3];       // D_I dt / dx^2
  T invD[3];
  int advect;      // 0: no flow coupling
  int nrep;
  long rs;
  __device__ void shift(long o) {
    phi = sh(phi, o), w = sh(w, o), u = sh(u, o), wout = sh(wout, o), stilde = sh(stilde, o);
    scal = sh(scal, o), partials = sh(partials, o);
  }
};

// One Euler-forward convection step at LDS position (lx, ly) of a tile holding
// phi[3], omega[3], ux, uy: donor-cell flux form for Phi (face velocity the
// mean of the two cell velocities, upwind cell by its sign), upwind form for
// the auxiliary convection of omega (App. C, first comment).
template <typename T>
__device__ __forceinline__ void advect_site(const T (&sIn)[8][kHY][kHX], int lx, int ly, T (&pt)[3], T (&wt)[3]) {
  const T uxc = sIn[6][ly][lx], uyc = sIn[7][ly][lx];
  // face velocities
  const T uxe = T(0.5) * (uxc + sIn[6][ly][lx + 1]);
  const T uxw = T(0.5) * (sIn[6][ly][lx - 1] + uxc);
  const T uyn = T(0.5) * (uyc + sIn[7][ly + 1][lx]);
  const T uys = T(0.5) * (sIn[7][ly - 1][lx] + uyc);
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
}

// Loads the tile at (tx0, ty0) with a halo of 2 into sIn (velocities zero
// when the flow does not advect).  Launched with kTX * kTY threads; every
// thread issues all its loads before the first LDS write, so the block waits
// for one memory round trip instead of one per pass.
template <typename T>
__device__ __forceinline__ void load_advect_tile(const UpdArgs<T>& P, int tx0, int ty0, T (&sIn)[8][kHY][kHX]) {
  constexpr int kThr = kTX * kTY, kIt = (kHX * kHY + kThr - 1) / kThr;
  T v[kIt][8];
  long gi[kIt];
#pragma unroll
  for (int it = 0; it < kIt; ++it) {
    const int e = threadIdx.x + it * kThr;
    if (e < kHX * kHY) {
      const int lx = e % kHX, ly = e / kHX;
      const int gx = (tx0 + lx - 2 + P.nx) & (P.nx - 1);
      const int gy = (ty0 + ly - 2 + P.ny) & (P.ny - 1);
      gi[it] = long(gy) * P.nx + gx;
#pragma unroll
      for (int I = 0; I < 3; ++I) {
        v[it][I] = P.phi[I * P.n + gi[it]];
        v[it][3 + I] = P.w[I * P.n + gi[it]];
      }
      v[it][6] = P.advect ? P.u[gi[it]] : T(0);
      v[it][7] = P.advect ? P.u[P.n + gi[it]] : T(0);
    }
  }
#pragma unroll
  for (int it = 0; it < kIt; ++it) {
    const int e = threadIdx.x + it * kThr;
    if (e < kHX * kHY) {
      const int lx = e % kHX, ly = e / kHX;
#pragma unroll
      for (int k = 0; k < 8; ++k) sIn[k][ly][lx] = v[it][k];
    }
  }
}

template <typename T>
__global__ void __launch_bounds__(256) k_advect_update(UpdArgs<T> P) {
  __shared__ T sIn[8][kHY][kHX];   // phi[3], w[3], ux, uy
  __shared__ T sMu[3][kMY][kMX];
  __shared__ T sWt[3][kMY][kMX];
  __shared__ double red[16 * 4];
  P.shift(long(blockIdx.z) * P.rs);
  const int lt = xcd_tile(blockIdx.y * gridDim.x + blockIdx.x, gridDim.x * gridDim.y);
  const int tx0 = (lt % gridDim.x) * kTX, ty0 = (lt / gridDim.x) * kTY;
  const int tid = threadIdx.x;
  load_advect_tile(P, tx0, ty0, sIn);
  __syncthreads();
  // advected fields and mu~ on the halo-1 region, 34 x 10 sites: the first
  // pass gives each 32-lane half of a wave one row of 32 sites, so that every
  // LDS access of the stencil is 32 consecutive words of one row (no bank
  // conflicts); the second covers rows 8-9 and then columns 32-33
  static_assert(kTX == 32 && kTY == 8 && kMX == 34 && kMY == 10, "halo-1 pass mapping");
  for (int pass = 0; pass < 2; ++pass) {
    int mx, my;
    if (pass == 0) {
      mx = tid & 31, my = tid >> 5;
    } else if (tid < 64) {
      mx = tid & 31, my = 8 + (tid >> 5);
    } else if (tid < 84) {
      mx = 32 + ((tid - 64) & 1), my = (tid - 64) >> 1;
    } else {
      break;
    }
    T pt[3], wt[3];
    advect_site(sIn, mx + 1, my + 1, pt, wt);  // position in sIn
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
  block_partial<4>(v, red, P.partials, lt);
}

// The convection step alone: Phi~ -> phit and the auxiliary-convected omega
// -> wt (3 planes each), for the Phi -> omega inversion that follows it.
template <typename T>
__global__ void __launch_bounds__(256) k_advect_only(UpdArgs<T> P, T* __restrict__ phit, T* __restrict__ wt) {
  __shared__ T sIn[8][kHY][kHX];
  const int lt = xcd_tile(blockIdx.y * gridDim.x + blockIdx.x, gridDim.x * gridDim.y);
  const int tx0 = (lt % gridDim.x) * kTX, ty0 = (lt / gridDim.x) * kTY;
  load_advect_tile(P, tx0, ty0, sIn);
  __syncthreads();
  const int ox = threadIdx.x % kTX, oy = threadIdx.x / kTX;  // 256 threads = 32 x 8 sites
  T pt[3], w[3];
  advect_site(sIn, ox + 2, oy + 2, pt, w);
  const long gi = long(ty0 + oy) * P.nx + (tx0 + ox);
#pragma unroll
  for (int I = 0; I < 3; ++I) {
    phit[I * P.n + gi] = pt[I];
    wt[I * P.n + gi] = w[I];
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
  const double* scal;   // kGext: external force amplitude in lattice units
  int nf;
  int nrep;
  long rs;
  __device__ void shift(long o) {
    S = sh(S, o), spec = sh(spec, o), F = sh(F, o), tw_x = sh(tw_x, o), tw_y = sh(tw_y, o);
    scal = sh(scal, o);
  }
};

template <typename T, int L, int R>
__global__ void __launch_bounds__(512) k_force_row_fwd(ForceArgs<T> P) {
  constexpr int TL = L / R;
  using V = LdsView<T, L, R, true, 1>;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  const int f = threadIdx.x / TL, j = threadIdx.x % TL;
  V lds{reinterpret_cast<T2<T>*>(smem_raw), f};
  P.shift(long(blockIdx.z) * P.rs);
  const int y = blockIdx.x * P.nf + f;
  const bool active = y < P.ny;
  Twiddles<T, L, R> twf;
  load_fwd_twiddles(twf, j, P.tw_x);
  T re[R], im[R];
#pragma unroll
  for (int m = 0; m < R; ++m) {
    re[m] = active ? P.S[long(y) * P.nx + j + TL * m] : T(0);
    im[m] = T(0);
  }
  fft_forward(re, im, j, lds, twf);
  if (active) {
#pragma unroll
    for (int m = 0; m < R; ++m) {
      T2<T> o;
      o.x = re[m];
      o.y = im[m];
      P.spec[long(y) * P.nx + j + TL * m] = o;
    }
  }
}

template <typename T, int L, int R, int NF>
__global__ void __launch_bounds__(512) k_force_col(ForceArgs<T> P) {
  constexpr int TL = L / R;
  using V = LdsView<T, L, R, false, NF>;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  const int f = threadIdx.x % NF, j = threadIdx.x / NF;
  V lds{reinterpret_cast<T2<T>*>(smem_raw), f};
  P.shift(long(blockIdx.z) * P.rs);
  const int kxi = xcd_tile(blockIdx.x, gridDim.x) * NF + f;   // column = x wavenumber index
  const bool active = kxi < P.nx;
  Twiddles<T, L, R> twf, twi;
  load_fwd_twiddles(twf, j, P.tw_y);
  load_inv_twiddles(twi, j, P.tw_y);
  T re[R], im[R];
#pragma unroll
  for (int m = 0; m < R; ++m) {
    T2<T> v;
    v.x = T(0);
    v.y = T(0);
    if (active) v = P.spec[long(j + TL * m) * P.nx + kxi];
    re[m] = v.x;
    im[m] = v.y;
  }
  fft_forward(re, im, j, lds, twf);
  const int mx = kxi < P.nx / 2 ? kxi : kxi - P.nx;
  const double kx = P.kx0 * mx;
  const bool nyq_x = (kxi == P.nx / 2);
#pragma unroll
  for (int m = 0; m < R; ++m) {
    const int kyi = j + TL * m;
    const int my = kyi < P.ny / 2 ? kyi : kyi - P.ny;
    const double ky = P.ky0 * my;
    const double k2 = kx * kx + ky * ky;
    const double inv = k2 > 0.0 ? P.pref / k2 : 0.0;
    const T al = nyq_x ? T(0) : T(inv * kx);
    const T be = (kyi == P.ny / 2) ? T(0) : T(inv * ky);
    const T sr = re[m], si = im[m];
    // G = i al S + i (i be S) = (i al - be) S: real part f_x, imaginary part f_y
    re[m] = -al * si - be * sr;
    im[m] = al * sr - be * si;
  }
  fft_inverse(re, im, j, lds, twi);
  if (active) {
#pragma unroll
    for (int m = 0; m < R; ++m) {
      T2<T> o;
      o.x = re[m];
      o.y = im[m];
      P.spec[long(j + TL * m) * P.nx + kxi] = o;
    }
  }
}

template <typename T, int L, int R>
__global__ void __launch_bounds__(512) k_force_row_inv(ForceArgs<T> P) {
  constexpr int TL = L / R;
  using V = LdsView<T, L, R, true, 1>;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  const int f = threadIdx.x / TL, j = threadIdx.x % TL;
  V lds{reinterpret_cast<T2<T>*>(smem_raw), f};
  P.shift(long(blockIdx.z) * P.rs);
  const int y = blockIdx.x * P.nf + f;
  const bool active = y < P.ny;
  Twiddles<T, L, R> twi;
  load_inv_twiddles(twi, j, P.tw_x);
  T re[R], im[R];
#pragma unroll
  for (int m = 0; m < R; ++m) {
    T2<T> v;
    v.x = T(0);
    v.y = T(0);
    if (active) v = P.spec[long(y) * P.nx + j + TL * m];
    re[m] = v.x;
    im[m] = v.y;
  }
  fft_inverse(re, im, j, lds, twi);
  if (active) {
    const T conv = T(P.conv);
    const double g = P.scal[kGext];
    const T fext = T(y < P.ny / 2 ? -g : g);
#pragma unroll
    for (int m = 0; m < R; ++m) {
      const long i = long(y) * P.nx + j + TL * m;
      P.F[i] = re[m] * conv + fext;
      P.F[P.n + i] = im[m] * conv;
    }
  }
}

// ---------------------------------------------------------------------------
// D2Q9 lattice Boltzmann: pull stream + BGK collision with second-order force.
// Populations are stored as deviations g_i = f_i - w_i from the rest state
// (rho = 1, u = 0) so that FP32 keeps the small momentum of slow flows.
// ---------------------------------------------------------------------------
template <typename T> struct LbArgs {
  const T* fin;    // 9 planes g* = f* - w (previous post-collision)
  T* fout;         // 9 planes
  const T* F;      // 2 planes
  T* rho;
  T* u;            // 2 planes
  int nx, ny;
  long n;
  T omega;         // BGK: 1/tau
  T fpre;          // BGK: 1 - 1/(2 tau)
  T gs, gb, gg;    // multi-relaxation: shear, bulk and non-hydrodynamic factors
  T umax2;         // flow-speed guard: |u|^2 above this sets guard[kGuardMach]
  unsigned* guard; // kNumGuard flags of the replica, set (never cleared) by the kernel
  int nrep;
  long rs;
  __device__ void shift(long o) {
    fin = sh(fin, o), fout = sh(fout, o), F = sh(F, o), rho = sh(rho, o), u = sh(u, o);
    guard = sh(guard, o);
  }
};

// Stability flags of one replica, raised by the LB kernel and reported by the
// host at the next synchronisation: the flow speed above the guard, a
// negative post-collision population, a density or velocity that is not finite.
enum Guard : int { kGuardMach = 0, kGuardNegative = 1, kGuardNonFinite = 2, kNumGuard = 3 };

// Flags of one lane over the sites it updates; raised in memory by lb_raise.
struct LbFlags {
  bool nonfinite = false, fast = false, neg = false;
};
template <typename T>
__device__ __forceinline__ void lb_check(LbFlags& fl, T rho, T usq, T umax2, T fmin) {
  const bool nf = !isfinite(rho) || !isfinite(usq);
  fl.nonfinite |= nf;
  fl.fast |= !nf && usq > umax2;
  fl.neg |= !nf && fmin < T(0);
}
// Lanes that found a condition store its flag (a rare path; all store 1).
__device__ __forceinline__ void lb_raise(unsigned* guard, const LbFlags& fl) {
  if (fl.nonfinite) guard[kGuardNonFinite] = 1u;
  if (fl.fast) guard[kGuardMach] = 1u;
  if (fl.neg) guard[kGuardNegative] = 1u;
}

// MRT = false: BGK collision with relaxation time tau and the second-order
// force term.  MRT = true: the multi-relaxation collision in moment space
// (moments of the deviations g = f - w, so rho - 1 and the stress minus its
// rest value keep full precision):
//   u = (j + F/2)/rho,  Pi_eq = rho/3 I + rho u u,  N = Pi - Pi_eq,
//   Pi* = Pi_eq + gs (N - tr(N)/2 I) + gb tr(N)/2 I
//         + (1 + gs)/2 [u F + F u - (u.F) I] + (1 + gb)/2 (u.F) I,
//   f*_i = H_i(rho, j + F, Pi*) + gg (f_i - H_i(rho, j, Pi)),
// H_i(rho, j, Pi) = w_i [rho + 3 j.c_i + 4.5 (Pi - rho/3 I):(c_i c_i - I/3)],
// the populations that carry exactly (rho, j, Pi).
// Pull streaming of one site: g_k(x) = g*_k(x - c_k) from the previous buffer;
// c = (0,0),(1,0),(0,1),(-1,0),(0,-1),(1,1),(-1,1),(-1,-1),(1,-1).
template <typename T>
__device__ __forceinline__ void lb_pull(const LbArgs<T>& P, int x, int y, T (&g)[9]) {
  const int xm = (x - 1) & (P.nx - 1), xp = (x + 1) & (P.nx - 1);
  const long ym = long((y - 1) & (P.ny - 1)) * P.nx, yp = long((y + 1) & (P.ny - 1)) * P.nx;
  const long yc = long(y) * P.nx;
  g[0] = P.fin[0 * P.n + yc + x];
  g[1] = P.fin[1 * P.n + yc + xm];
  g[2] = P.fin[2 * P.n + ym + x];
  g[3] = P.fin[3 * P.n + yc + xp];
  g[4] = P.fin[4 * P.n + yp + x];
  g[5] = P.fin[5 * P.n + ym + xm];
  g[6] = P.fin[6 * P.n + ym + xp];
  g[7] = P.fin[7 * P.n + yp + xp];
  g[8] = P.fin[8 * P.n + yp + xm];
}

// Collision of the pulled populations g of site i with the force (Fx, Fy);
// stores f*, rho, u and records the guard's conditions in fl.
template <typename T, bool MRT>
__device__ __forceinline__ void lb_collide(const LbArgs<T>& P, long i, const T (&g)[9], T Fx, T Fy, LbFlags& fl) {
  // sum_i w_i = 1 and sum_i w_i c_i = 0, so the deviations carry rho - 1 and the momentum
  const T drho = ((g[0] + g[1]) + (g[2] + g[3])) + ((g[4] + g[5]) + (g[6] + g[7])) + g[8];
  const T rho = T(1) + drho;
  const T jx = (g[1] - g[3]) + (g[5] - g[6]) + (g[8] - g[7]);
  const T jy = (g[2] - g[4]) + (g[5] + g[6]) - (g[7] + g[8]);
  const T ir = T(1) / rho;
  const T ux = (jx + T(0.5) * Fx) * ir;
  const T uy = (jy + T(0.5) * Fy) * ir;
  const T usq = ux * ux + uy * uy;
  constexpr int cx[9] = {0, 1, 0, -1, 0, 1, -1, -1, 1};
  constexpr int cy[9] = {0, 0, 1, 0, -1, 1, 1, -1, -1};
  if constexpr (MRT) {
    // second moments of g: sum_i w_i c_i c_i = I/3, so Pi - rho/3 I = Sg - drho/3 I
    const T sxx = (g[1] + g[3]) + ((g[5] + g[6]) + (g[7] + g[8]));
    const T syy = (g[2] + g[4]) + ((g[5] + g[6]) + (g[7] + g[8]));
    const T sxy = (g[5] - g[6]) + (g[7] - g[8]);
    const T third = T(1.0 / 3.0);
    // A = Pi - rho/3 I (pre-collision), B = Pi* - rho/3 I (post-collision)
    const T axx = sxx - third * drho, ayy = syy - third * drho, axy = sxy;
    const T nxx = axx - rho * ux * ux, nyy = ayy - rho * uy * uy, nxy = axy - rho * ux * uy;
    const T htr = T(0.5) * (nxx + nyy);
    const T uF = ux * Fx + uy * Fy;
    const T cs_ = T(0.5) * (T(1) + P.gs), cb_ = T(0.5) * (T(1) + P.gb);
    const T bxx = rho * ux * ux + P.gs * (nxx - htr) + P.gb * htr + cs_ * (T(2) * ux * Fx - uF) + cb_ * uF;
    const T byy = rho * uy * uy + P.gs * (nyy - htr) + P.gb * htr + cs_ * (T(2) * uy * Fy - uF) + cb_ * uF;
    const T bxy = rho * ux * uy + P.gs * nxy + cs_ * (ux * Fy + uy * Fx);
    const T jxs = jx + Fx, jys = jy + Fy;
    // The moving populations from the expansion; the rest population is their
    // complement to rho - 1, its exact value: the rounded weights would
    // otherwise leave the stress term a trace of about eps |rho u u| per step,
    // a systematic drift of the mass.
    T o[9];
#pragma unroll
    for (int k = 1; k < 9; ++k) {
      const T w = k < 5 ? T(1.0 / 9.0) : T(1.0 / 36.0);
      const T qx = T(cx[k] * cx[k]) - third, qy = T(cy[k] * cy[k]) - third, qxy = T(2 * cx[k] * cy[k]);
      const T hpost = w * (drho + T(3) * (T(cx[k]) * jxs + T(cy[k]) * jys) +
                           T(4.5) * (bxx * qx + byy * qy + bxy * qxy));
      const T hpre = w * (drho + T(3) * (T(cx[k]) * jx + T(cy[k]) * jy) +
                          T(4.5) * (axx * qx + ayy * qy + axy * qxy));
      o[k] = hpost + P.gg * (g[k] - hpre);
    }
    o[0] = drho - (((o[1] + o[2]) + (o[3] + o[4])) + ((o[5] + o[6]) + (o[7] + o[8])));
    T fmin = o[0] + T(4.0 / 9.0);
#pragma unroll
    for (int k = 0; k < 9; ++k) {
      P.fout[k * P.n + i] = o[k];
      fmin = min(fmin, o[k] + (k == 0 ? T(4.0 / 9.0) : (k < 5 ? T(1.0 / 9.0) : T(1.0 / 36.0))));
    }
    lb_check(fl, rho, usq, P.umax2, fmin);
    P.rho[i] = rho;
    P.u[i] = ux;
    P.u[P.n + i] = uy;
    return;
  }
  T fmin = T(1);
#pragma unroll
  for (int k = 0; k < 9; ++k) {
    const T w = k == 0 ? T(4.0 / 9.0) : (k < 5 ? T(1.0 / 9.0) : T(1.0 / 36.0));
    const T cu = T(cx[k]) * ux + T(cy[k]) * uy;
    // f^eq - w = w (rho - 1) + w rho (3 c.u + 4.5 (c.u)^2 - 1.5 u^2)
    const T geq = w * drho + w * rho * (T(3) * cu + T(4.5) * cu * cu - T(1.5) * usq);
    const T cF = T(cx[k]) * Fx + T(cy[k]) * Fy;
    const T cmuF = (T(cx[k]) - ux) * Fx + (T(cy[k]) - uy) * Fy;
    const T src = w * (T(3) * cmuF + T(9) * cu * cF);
    const T o = g[k] - (g[k] - geq) * P.omega + P.fpre * src;
    P.fout[k * P.n + i] = o;
    fmin = min(fmin, o + w);
  }
  lb_check(fl, rho, usq, P.umax2, fmin);
  P.rho[i] = rho;
  P.u[i] = ux;
  P.u[P.n + i] = uy;
}

template <typename T, bool MRT>
__global__ void __launch_bounds__(256) k_lb(LbArgs<T> P) {
  P.shift(long(blockIdx.z) * P.rs);
  const long i = long(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= P.n) return;
  const int x = int(i & (P.nx - 1)), y = int(i / P.nx);
  T g[9];
  lb_pull(P, x, y, g);
  LbFlags fl;
  lb_collide<T, MRT>(P, i, g, P.F[i], P.F[P.n + i], fl);
  lb_raise(P.guard, fl);
}

// The row-inverse force pass fused with the LB step of the same rows: the
// x-inverse FFT of the force spectrum gives (f_x, f_y) of nf rows per block,
// stored as the lattice force F (as k_force_row_inv does) and handed to the LB
// step of those sites in registers (as k_lb does with F from memory).  The
// populations the LB pulls (neighbouring rows of the previous buffer, which
// no block of this launch writes) are loaded before the transform, so their
// latency overlaps it.
template <typename T, int L, int R, bool MRT>
__global__ void __launch_bounds__(512) k_force_inv_lb(ForceArgs<T> P, LbArgs<T> B) {
  constexpr int TL = L / R;
  using V = LdsView<T, L, R, true, 1>;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  const int f = threadIdx.x / TL, j = threadIdx.x % TL;
  V lds{reinterpret_cast<T2<T>*>(smem_raw), f};
  P.shift(long(blockIdx.z) * P.rs);
  B.shift(long(blockIdx.z) * B.rs);
  const int y = blockIdx.x * P.nf + f;
  const bool active = y < P.ny;
  Twiddles<T, L, R> twi;
  load_inv_twiddles(twi, j, P.tw_x);
  T re[R], im[R];
#pragma unroll
  for (int m = 0; m < R; ++m) {
    T2<T> v;
    v.x = T(0);
    v.y = T(0);
    if (active) v = P.spec[long(y) * P.nx + j + TL * m];
    re[m] = v.x;
    im[m] = v.y;
  }
  T g[R][9];
  if (active) {
#pragma unroll
    for (int m = 0; m < R; ++m) lb_pull(B, j + TL * m, y, g[m]);
  }
  fft_inverse(re, im, j, lds, twi);
  if (!active) return;
  const T conv = T(P.conv);
  const double ge = P.scal[kGext];
  const T fext = T(y < P.ny / 2 ? -ge : ge);
  LbFlags fl;
#pragma unroll
  for (int m = 0; m < R; ++m) {
    const long i = long(y) * P.nx + j + TL * m;
    const T Fx = re[m] * conv + fext, Fy = im[m] * conv;
    P.F[i] = Fx;
    P.F[P.n + i] = Fy;
    lb_collide<T, MRT>(B, i, g[m], Fx, Fy, fl);
  }
  lb_raise(B.guard, fl);
}

}  // namespace epdlb
