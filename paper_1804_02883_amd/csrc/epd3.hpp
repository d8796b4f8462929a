// Chain propagators and densities on a three-dimensional periodic grid
// (Sec. II: the split step, the density integrals and Eq. phi_s, with the
// heat kernel exp(-R_G^2 |k|^2 ds) of three dimensions).
//
// One contour step q -> E K (E q), E = exp(-(w_j - c_j)/2), runs as
//   FFT along x of E q (the factor applied as the lines load) -> FFT along y
//   -> FFT along z, heat multiplier, inverse FFT along z -> inverse FFT along
//   y -> inverse FFT along x, storing q' = E Re / n.
// The FFT kernel transforms whole lines in LDS with the radix-2 Stockham
// formulation (natural order in and out, a ping-pong pair of buffers per
// line): every line is read and written once per pass.  Lines along x are
// contiguous; lines along y and z are strided, and a block's lines are
// neighbours in x, so each load instruction of a wave covers consecutive
// addresses.  Sums (gauge, Q_P, Q_S) are FP64 block partials in fixed slots,
// added in slot order.
#pragma once
#include <hip/hip_runtime.h>

namespace epdlb {
namespace epd3 {

constexpr int kThreads = 256;
constexpr int kRedBlocks = 256;
constexpr int kMaxLen = 512;

template <typename T> struct Cx {
  T re, im;
};

__device__ __forceinline__ void sin_cos_pi(double x, double* s, double* c) { sincospi(x, s, c); }
__device__ __forceinline__ void sin_cos_pi(float x, float* s, float* c) { sincospif(x, s, c); }

// c = exp(-(a (wA - cA) + (1 - a)(wB - cB)) / 2), the gauge from the field sums.
template <typename T>
__device__ __forceinline__ T half_step_factor(T wa, T wb, T a, const double* sums, double inv_n) {
  const T cA = T(sums[0] * inv_n), cB = T(sums[2] * inv_n);
  return exp(-(a * (wa - cA) + (T(1) - a) * (wb - cB)) * T(0.5));
}

struct LineArgs {
  int L;         // line length (power of two, <= kMaxLen)
  long st;       // element stride along the line
  long count;    // number of lines
  long g;        // base(l) = (l / g) * gs + (l % g) * gi
  long gs, gi;
  int mode;      // -1 forward, +1 inverse, 2 forward, heat multiplier, inverse
  int lb;        // lines per block; > 0: lines interleaved across lanes (strided passes)
  int nx, ny, nz;
  double heat;   // R_G^2 ds (2 pi / dx)^2: |k|^2 R_G^2 ds = heat (mx^2/nx^2 + my^2/ny^2 + mz^2/nz^2)
  // x passes only: fuse = 1 loads E q (q == nullptr: E) instead of C; fuse = 2
  // stores q' = E Re(.) / n instead of C (E from wA, wB, a and the field sums)
  int fuse;
  const void* wA;
  const void* wB;
  const void* q;
  void* qn;
  const double* sums;
  double inv_n;
  double a;
};

// Stockham transform of the lines held in LDS (natural order in and out):
// one radix-2 stage when log2 L is odd, then radix-4 stages; src and dst
// alternate, *out receives the buffer that holds the result.  dir -1 or +1.
// tw[m] = (cos, sin)(pi m / (L/2)), m < L: the stage of sub-length Ns takes
// the angle dir pi r k / (2 Ns) (radix 4, r < 4) from entry r k L / (4 Ns),
// and dir pi k / Ns (radix 2) from entry k L / (2 Ns).
template <typename T>
__device__ __forceinline__ void stockham(Cx<T>* buf0, Cx<T>* buf1, const Cx<T>* tw, int L, int t, int TL,
                                         bool active, int dir, Cx<T>** out) {
  Cx<T>* src = buf0;
  Cx<T>* dst = buf1;
  int Ns = 1;
  if (L > 1 && (__builtin_ctz(unsigned(L)) & 1)) {
    if (active) {
      for (int j = t; j < L / 2; j += TL) {
        const int k = j % Ns;
        const Cx<T> w = tw[k * (L / (2 * Ns))];
        const T c = w.re, s = dir > 0 ? w.im : -w.im;
        const Cx<T> u = src[j];
        const Cx<T> v0 = src[j + L / 2];
        const T vr = v0.re * c - v0.im * s, vi = v0.re * s + v0.im * c;
        const int d = (j / Ns) * Ns * 2 + k;
        dst[d].re = u.re + vr;
        dst[d].im = u.im + vi;
        dst[d + Ns].re = u.re - vr;
        dst[d + Ns].im = u.im - vi;
      }
    }
    __syncthreads();
    Cx<T>* tmp = src;
    src = dst;
    dst = tmp;
    Ns = 2;
  }
  for (; Ns < L; Ns *= 4) {
    if (active) {
      for (int j = t; j < L / 4; j += TL) {
        const int k = j % Ns;
        const int step = k * (L / (4 * Ns));
        T vr[4], vi[4];
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const Cx<T> a = src[j + r * (L / 4)];
          const Cx<T> w = tw[r * step];
          const T c = w.re, s = dir > 0 ? w.im : -w.im;
          vr[r] = a.re * c - a.im * s;
          vi[r] = a.re * s + a.im * c;
        }
        // 4-point DFT with i^dir: (dir i) v = (-dir vi, dir vr)
        const T dr = T(dir);
        const T s02r = vr[0] + vr[2], s02i = vi[0] + vi[2], d02r = vr[0] - vr[2], d02i = vi[0] - vi[2];
        const T s13r = vr[1] + vr[3], s13i = vi[1] + vi[3], d13r = vr[1] - vr[3], d13i = vi[1] - vi[3];
        const int d = (j / Ns) * Ns * 4 + k;
        dst[d].re = s02r + s13r;
        dst[d].im = s02i + s13i;
        dst[d + Ns].re = d02r - dr * d13i;
        dst[d + Ns].im = d02i + dr * d13r;
        dst[d + 2 * Ns].re = s02r - s13r;
        dst[d + 2 * Ns].im = s02i - s13i;
        dst[d + 3 * Ns].re = d02r + dr * d13i;
        dst[d + 3 * Ns].im = d02i - dr * d13r;
      }
    }
    __syncthreads();
    Cx<T>* tmp = src;
    src = dst;
    dst = tmp;
  }
  *out = src;
}

// Transform every line of C in place.  Contiguous lines (A.lb == 0): TL =
// max(L/2, 1) consecutive threads per line, kThreads / TL lines per block.
// Strided lines (A.lb > 0): A.lb lines per block, interleaved across lanes
// (lane % lb picks the line), so that the lanes of one load instruction read
// neighbouring lines' elements: consecutive addresses.  Dynamic LDS
// lines * (2 L + 2) complex values (the 2 pad the lines across banks), then
// the L twiddles.
template <typename T>
__global__ void __launch_bounds__(kThreads) k_p3_fft(Cx<T>* __restrict__ C, LineArgs A) {
  extern __shared__ __align__(16) unsigned char lds_raw[];
  const int L = A.L;
  const int lines = A.lb > 0 ? A.lb : kThreads / (L > 1 ? L / 2 : 1);
  const int TL = kThreads / lines;
  const int sub = A.lb > 0 ? int(threadIdx.x) % lines : int(threadIdx.x) / TL;
  const int t = A.lb > 0 ? int(threadIdx.x) / lines : int(threadIdx.x) % TL;
  const long l = long(blockIdx.x) * lines + sub;
  const bool active = l < A.count;
  Cx<T>* base_lds = reinterpret_cast<Cx<T>*>(lds_raw);
  Cx<T>* b0 = base_lds + long(sub) * (2 * L + 2);
  Cx<T>* b1 = b0 + L;
  Cx<T>* tw = base_lds + long(lines) * (2 * L + 2);
  for (int m = threadIdx.x; m < L; m += kThreads) {
    T sv, cv;
    sin_cos_pi(L > 1 ? T(2 * m) / T(L) : T(0), &sv, &cv);
    tw[m].re = cv;
    tw[m].im = sv;
  }
  const long base = active ? (l / A.g) * A.gs + (l % A.g) * A.gi : 0;
  const T* wA = static_cast<const T*>(A.wA);
  const T* wB = static_cast<const T*>(A.wB);
  if (active) {
    if (A.fuse == 1) {
      const T* q = static_cast<const T*>(A.q);
      for (int e = t; e < L; e += TL) {
        const long i = base + e * A.st;
        const T f = half_step_factor(wA[i], wB[i], T(A.a), A.sums, A.inv_n);
        b0[e].re = q ? f * q[i] : f;
        b0[e].im = T(0);
      }
    } else {
      for (int e = t; e < L; e += TL) b0[e] = C[base + e * A.st];
    }
  }
  __syncthreads();
  Cx<T>* res;
  stockham(b0, b1, tw, L, t, TL, active, A.mode == 1 ? 1 : -1, &res);
  if (A.mode == 2) {
    // heat multiplier at (mx, my, mz); this pass runs along z
    if (active) {
      const int x = int(base % A.nx), y = int(base / A.nx);
      const int mx = x < (A.nx + 1) / 2 ? x : x - A.nx, my = y < (A.ny + 1) / 2 ? y : y - A.ny;
      const double kxy = double(mx) * mx / (double(A.nx) * A.nx) + double(my) * my / (double(A.ny) * A.ny);
      const T fxy = T(exp(-A.heat * kxy));  // the factor separates: exp(-h kxy) exp(-h kz)
      const T hz = T(A.heat / (double(L) * L));
      for (int e = t; e < L; e += TL) {
        const int mz = e < (L + 1) / 2 ? e : e - L;
        const T f = fxy * exp(-hz * T(mz * mz));
        res[e].re *= f;
        res[e].im *= f;
      }
    }
    __syncthreads();
    Cx<T>* other = res == b0 ? b1 : b0;
    stockham(res, other, tw, L, t, TL, active, 1, &res);
  }
  if (active) {
    if (A.fuse == 2) {
      T* qn = static_cast<T*>(A.qn);
      for (int e = t; e < L; e += TL) {
        const long i = base + e * A.st;
        qn[i] = half_step_factor(wA[i], wB[i], T(A.a), A.sums, A.inv_n) * res[e].re * T(A.inv_n);
      }
    } else {
      for (int e = t; e < L; e += TL) C[base + e * A.st] = res[e];
    }
  }
}

// part[block] = sum over the block's grid-stride elements of a (exp_shift:
// of exp(-(a - sums[0] inv_n)) instead), FP64, fixed-order block reduction.
template <typename T>
__global__ void __launch_bounds__(kThreads) k_p3_sum(const T* __restrict__ a, long n, int expo,
                                                     const double* __restrict__ sums, double inv_n,
                                                     double* __restrict__ part) {
  __shared__ double red[kThreads];
  const double c = expo ? sums[0] * inv_n : 0.0;
  double acc = 0.0;
  for (long i = long(blockIdx.x) * blockDim.x + threadIdx.x; i < n; i += long(gridDim.x) * blockDim.x)
    acc += expo ? double(exp(-(a[i] - T(c)))) : double(a[i]);
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int s = kThreads / 2; s > 0; s /= 2) {
    if (int(threadIdx.x) < s) red[threadIdx.x] += red[threadIdx.x + s];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[blockIdx.x] = red[0];
}

// out[0] = sum of part[0..nb) in slot order.  One block.
__global__ void __launch_bounds__(kThreads) k_p3_finish(const double* __restrict__ part, int nb,
                                                        double* __restrict__ out) {
  __shared__ double red[kThreads];
  double acc = 0.0;
  for (int b = threadIdx.x; b < nb; b += blockDim.x) acc += part[b];
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int s = kThreads / 2; s > 0; s /= 2) {
    if (int(threadIdx.x) < s) red[threadIdx.x] += red[threadIdx.x + s];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[0] = red[0];
}

template <typename T>
__global__ void __launch_bounds__(kThreads) k_p3_fill(T* __restrict__ a, T v, long n) {
  for (long i = long(blockIdx.x) * blockDim.x + threadIdx.x; i < n; i += long(gridDim.x) * blockDim.x) a[i] = v;
}

struct DensArgs {
  int N;
  long n;
  double V_over_dV;   // V / dV = number of sites
  double phiP;
  const double* wAn;  // node weights, N + 1 each
  const double* wBn;
  const double* sums; // [0] sum wA, [2] sum wB, [4] sum wS, [6] sum q_N, [8] sum exp(-(wS - cS))
  double inv_n;
};

// Phi_A = (V phibar_P / Q_P) sum_j wA_j q_j qb_{N-j}, Phi_B likewise, Phi_S =
// V (1 - phibar_P) exp(-(wS - cS)) / Q_S, with Q = dV * sum (dV cancels).
template <typename T>
__global__ void __launch_bounds__(kThreads) k_p3_density(const T* __restrict__ q, const T* __restrict__ qb,
                                                         const T* __restrict__ wS, T* __restrict__ phi,
                                                         DensArgs D) {
  const double sP = D.V_over_dV * D.phiP / D.sums[6];
  const double sS = D.V_over_dV * (1.0 - D.phiP) / D.sums[8];
  const T cS = T(D.sums[4] * D.inv_n);
  for (long i = long(blockIdx.x) * blockDim.x + threadIdx.x; i < D.n; i += long(gridDim.x) * blockDim.x) {
    T sa = T(0), sb = T(0);
    for (int j = 0; j <= D.N; ++j) {
      const T pr = q[long(j) * D.n + i] * qb[long(D.N - j) * D.n + i];
      sa += T(D.wAn[j]) * pr;
      sb += T(D.wBn[j]) * pr;
    }
    phi[i] = T(sP) * sa;
    phi[D.n + i] = T(sP) * sb;
    phi[2 * D.n + i] = T(sS) * exp(-(wS[i] - cS));
  }
}

}  // namespace epd3
}  // namespace epdlb
