// Register + LDS FFT building blocks for gfx950 (64-wide wavefronts).
//
// A length-L transform is split L = N1 x N2 (N1 <= N2, powers of two).  A
// group of N1 lanes owns one transform:
//   time layout  lane n1 holds v[n2] = x[n1 + N1*n2],            n2 = 0..N2-1
//   freq layout  lane t  holds r[m*N1 + k1] = X[(t + N1*m) + N2*k1],
//                m = 0..N2/N1-1, k1 = 0..N1-1
// The forward transform is an N2-point DFT in registers, a twiddle by
// W_L^{n1*k2}, one LDS exchange, and N1-point DFTs in registers.  The inverse
// runs the same steps backwards, so a pointwise multiplier can be applied in
// the (permuted) frequency layout with no reordering.  Global loads in the
// time layout are contiguous across the N1 lanes of a group.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace epdlb {

template <typename T> struct vec2;
template <> struct vec2<float> { using type = float2; };
template <> struct vec2<double> { using type = double2; };
template <typename T> using T2 = typename vec2<T>::type;

// ---------------------------------------------------------------------------
// Compile-time twiddles exp(-2 pi i e / 64), e = 0..63, from Taylor series on
// the first octant plus exact symmetries (no runtime trig in the inner DFTs).
// ---------------------------------------------------------------------------
constexpr double kTwoPi = 6.283185307179586476925286766559;

constexpr double taylor_sin(double x) {
  double term = x, sum = x;
  for (int n = 1; n < 16; ++n) {
    term *= -x * x / double((2 * n) * (2 * n + 1));
    sum += term;
  }
  return sum;
}
constexpr double taylor_cos(double x) {
  double term = 1.0, sum = 1.0;
  for (int n = 1; n < 16; ++n) {
    term *= -x * x / double((2 * n - 1) * (2 * n));
    sum += term;
  }
  return sum;
}
// cos of 2 pi e / 64 for integer e, reduced to an angle <= pi/4.
constexpr double cos64(int e) {
  e &= 63;
  if (e > 32) e = 64 - e;            // cos(2 pi - a) = cos(a)
  if (e > 16) return -cos64(32 - e); // cos(pi - a) = -cos(a)
  if (e > 8) return taylor_sin(kTwoPi * double(16 - e) / 64.0);  // cos(pi/2 - a) = sin(a)
  return taylor_cos(kTwoPi * double(e) / 64.0);
}
constexpr double sin64(int e) { return cos64(e - 16); }  // sin(a) = cos(a - pi/2)

struct TwTable {
  double c[64];
  double s[64];
  constexpr TwTable() : c(), s() {
    for (int e = 0; e < 64; ++e) {
      c[e] = cos64(e);
      s[e] = sin64(e);
    }
  }
};
static constexpr TwTable kTw{};

constexpr int brev(int k, int bits) {
  int r = 0;
  for (int b = 0; b < bits; ++b) r |= ((k >> b) & 1) << (bits - 1 - b);
  return r;
}
constexpr int ilog2(int n) { return n <= 1 ? 0 : 1 + ilog2(n / 2); }

// In-register DFT of size R (power of two, R <= 64), natural order in and out.
// SIGN = -1: X[k] = sum x[n] e^{-2 pi i nk/R};  SIGN = +1: conjugate kernel.
// Radix-2 decimation in frequency; the bit reversal is a register renaming.
template <typename T, int R, int SIGN>
__device__ __forceinline__ void dft(T* re, T* im) {
  static_assert(R >= 1 && R <= 64 && (R & (R - 1)) == 0, "DFT size");
  if constexpr (R > 1) {
#pragma unroll
    for (int h = R / 2; h >= 1; h >>= 1) {
#pragma unroll
      for (int b = 0; b < R; b += 2 * h) {
#pragma unroll
        for (int k = 0; k < h; ++k) {
          const int i = b + k, j = i + h;
          const T xr = re[i] - re[j];
          const T xi = im[i] - im[j];
          re[i] = re[i] + re[j];
          im[i] = im[i] + im[j];
          const int e = k * (64 / (2 * h));  // W_{2h}^k in units of 2 pi / 64
          if (e == 0) {
            re[j] = xr;
            im[j] = xi;
          } else if (e == 16) {  // multiply by SIGN * i
            re[j] = SIGN > 0 ? -xi : xi;
            im[j] = SIGN > 0 ? xr : -xr;
          } else {
            const T c = T(kTw.c[e]);
            const T s = SIGN > 0 ? T(kTw.s[e]) : T(-kTw.s[e]);
            re[j] = xr * c - xi * s;
            im[j] = xr * s + xi * c;
          }
        }
      }
    }
    T tr[R], ti[R];
#pragma unroll
    for (int k = 0; k < R; ++k) {
      tr[k] = re[brev(k, ilog2(R))];
      ti[k] = im[brev(k, ilog2(R))];
    }
#pragma unroll
    for (int k = 0; k < R; ++k) {
      re[k] = tr[k];
      im[k] = ti[k];
    }
  }
}

// Split of a transform length into N1 lanes x N2 registers.
template <int L> struct Split {
  static constexpr int N1 = L <= 32 ? 4 : L <= 128 ? 8 : L <= 512 ? 16 : 32;
  static constexpr int N2 = L / N1;
  static constexpr int M = N2 / N1;
  static_assert(N1 * N2 == L && N2 % N1 == 0, "split");
};

// LDS addressing for one exchange buffer: element (transform f, k2, n1) of
// the real or imaginary component.
//  * RowMap (lanes of one transform contiguous; nf transforms per block, only
//    the per-transform base depends on nf): f*FS + k2*(N1+1) + n1;
//  * ColMap (NF transforms interleaved, NF a compile-time constant so every
//    LDS access is a base register plus an immediate offset):
//    f + NF*n1 + (NF*N1 + 16)*k2, which puts lanes with different n1 inside
//    one wavefront into different bank groups.
template <int L> struct RowMap {
  using S = Split<L>;
  static constexpr int N1 = S::N1, N2 = S::N2;
  static constexpr int FS = N2 * (N1 + 1) + 1;
  __host__ __device__ static constexpr int size(int nf) { return FS * nf; }
  __device__ __forceinline__ int idx(int f, int k2, int n1) const {
    return f * FS + k2 * (N1 + 1) + n1;
  }
};
template <int L, int NF> struct ColMap {
  using S = Split<L>;
  static constexpr int N1 = S::N1, N2 = S::N2;
  static constexpr int K2S = NF * N1 + 16;
  __host__ __device__ static constexpr int size() { return K2S * N2; }
  __device__ __forceinline__ int idx(int f, int k2, int n1) const {
    return f + NF * n1 + K2S * k2;
  }
};

// Forward transform: time layout in (re/im[N2]) -> freq layout out.
// `tw` holds W_L^e = exp(-2 pi i e/L), e = 0..L-1.  All lanes of the block
// must call this (it contains block barriers).
template <typename T, int L, class Map>
__device__ __forceinline__ void fft_forward(T* re, T* im, int f, int lane, const Map& map,
                                            const T2<T>* __restrict__ tw, T* lre, T* lim) {
  using S = Split<L>;
  constexpr int N1 = S::N1, N2 = S::N2, M = S::M;
  dft<T, N2, -1>(re, im);
#pragma unroll
  for (int k2 = 1; k2 < N2; ++k2) {
    const T2<T> w = tw[lane * k2];
    const T r = re[k2] * w.x - im[k2] * w.y;
    im[k2] = re[k2] * w.y + im[k2] * w.x;
    re[k2] = r;
  }
  __syncthreads();
#pragma unroll
  for (int k2 = 0; k2 < N2; ++k2) {
    lre[map.idx(f, k2, lane)] = re[k2];
    lim[map.idx(f, k2, lane)] = im[k2];
  }
  __syncthreads();
#pragma unroll
  for (int m = 0; m < M; ++m) {
#pragma unroll
    for (int n1 = 0; n1 < N1; ++n1) {
      re[m * N1 + n1] = lre[map.idx(f, lane + N1 * m, n1)];
      im[m * N1 + n1] = lim[map.idx(f, lane + N1 * m, n1)];
    }
  }
#pragma unroll
  for (int m = 0; m < M; ++m) dft<T, N1, -1>(re + m * N1, im + m * N1);
}

// Inverse transform (unnormalised): freq layout in -> time layout out.
template <typename T, int L, class Map>
__device__ __forceinline__ void fft_inverse(T* re, T* im, int f, int lane, const Map& map,
                                            const T2<T>* __restrict__ tw, T* lre, T* lim) {
  using S = Split<L>;
  constexpr int N1 = S::N1, N2 = S::N2, M = S::M;
#pragma unroll
  for (int m = 0; m < M; ++m) dft<T, N1, +1>(re + m * N1, im + m * N1);
  __syncthreads();
#pragma unroll
  for (int m = 0; m < M; ++m) {
#pragma unroll
    for (int n1 = 0; n1 < N1; ++n1) {
      lre[map.idx(f, lane + N1 * m, n1)] = re[m * N1 + n1];
      lim[map.idx(f, lane + N1 * m, n1)] = im[m * N1 + n1];
    }
  }
  __syncthreads();
#pragma unroll
  for (int k2 = 0; k2 < N2; ++k2) {
    re[k2] = lre[map.idx(f, k2, lane)];
    im[k2] = lim[map.idx(f, k2, lane)];
  }
#pragma unroll
  for (int k2 = 1; k2 < N2; ++k2) {
    const T2<T> w = tw[lane * k2];  // multiply by the conjugate twiddle
    const T r = re[k2] * w.x + im[k2] * w.y;
    im[k2] = im[k2] * w.x - re[k2] * w.y;
    re[k2] = r;
  }
  dft<T, N2, +1>(re, im);
}

// Frequency index held in register slot (m, k1) by lane t.
template <int L>
__device__ __forceinline__ int freq_index(int t, int m, int k1) {
  using S = Split<L>;
  return (t + S::N1 * m) + S::N2 * k1;
}

}  // namespace epdlb
