// Register + LDS Stockham FFT for gfx950 (64-wide wavefronts).
//
// One length-L transform is owned by T = L/R lanes; lane j holds the R
// elements j + T*m (m = 0..R-1) in registers, in BOTH the time and the
// frequency domain, so global loads and stores are contiguous across lanes
// and a pointwise multiplier is applied without any reordering.
//
// The forward transform is a Stockham auto-sort FFT (decimation in time) with
// radices [R0, R, ..., R] (R0 = L / R^(S-1)); the inverse runs radices
// [R, ..., R, R0] with conjugate twiddles.  Each pass is a radix-r DFT in
// registers; consecutive passes exchange data through LDS.  The first pass of
// each direction reads registers and the last one leaves its outputs in
// registers, so a forward+inverse pair costs 2(S-1) LDS round trips.
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
constexpr int ipow(int b, int e) { return e == 0 ? 1 : b * ipow(b, e - 1); }

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

// Pass structure of a length-L transform with R values per lane.
template <int L, int R> struct Plan {
  static constexpr int passes() {
    int s = 1, p = R;
    while (p < L) {
      p *= R;
      ++s;
    }
    return s;
  }
  static constexpr int S = passes();              // number of radix passes
  static constexpr int R0 = L / ipow(R, S - 1);   // the one small radix
  static constexpr int T = L / R;                 // lanes per transform
  static constexpr int LP = L + L / 64;           // LDS length per transform (slack kept)
  static_assert(R0 >= 2 && R0 <= R && R0 * ipow(R, S - 1) == L, "plan");
  // LDS position of element i: a permutation inside each aligned group of 16
  // elements (128 bytes, one pass over the 32 banks), i xor (5 g mod 16) with
  // g = i / 16.  The strided writes of the early passes (stride r elements
  // across lanes) and the contiguous reads then fall into distinct 8-byte bank
  // pairs within each 16-lane group, where an additive pad of one element per
  // 64 left them 2- to 4-way conflicted.
  __device__ static __forceinline__ int skew(int i) { return i ^ ((5 * (i >> 4)) & 15); }
  // Interleaved views (NF transforms side by side, NF = 4 or 8): a lane's
  // bank pair is f + NF * (position mod 16/NF), so only the low bits of the
  // position matter, and within a group of 16 lanes the same-f lanes hold
  // consecutive butterflies.  Their reads are consecutive positions, their
  // writes r apart for r = 4 or 8 (pairs 2r apart in a pass after a radix-2
  // one).  Xoring bits 2 and 3 into bits 0 and 1 keeps four consecutive
  // positions distinct mod 4 and makes four positions at those strides
  // distinct mod 4 as well, where the group xor above left them 2-way
  // conflicted.
  __device__ static __forceinline__ int skew_il(int i) { return i ^ (((i >> 2) ^ (i >> 3)) & 3); }
};

// LDS view of one transform: complex element i (real and imaginary part
// side by side, one 64-/128-bit access each).
//  * CONTIG:      transform f occupies [f*LP, (f+1)*LP)
//  * interleaved: transforms are the fastest index (f + NF*skew_il(i)), so that
//                 lanes of one wavefront holding different transforms hit
//                 consecutive banks
template <typename T, int L, int R, bool CONTIG, int NF>
struct LdsView {
  T2<T>* buf;
  int f;
  __device__ __forceinline__ int at(int i) const {
    if constexpr (CONTIG) return f * Plan<L, R>::LP + Plan<L, R>::skew(i);
    else return f + NF * Plan<L, R>::skew_il(i);
  }
  // complex elements needed for nf transforms
  __host__ __device__ static constexpr int size_elems(int nf) {
    return CONTIG ? Plan<L, R>::LP * nf : NF * Plan<L, R>::LP;
  }
};

// One Stockham pass of radix r over sub-transforms of length Ns.
// Input element of butterfly jj, leg q: in[jj + q*L/r].  Output element:
// out[(jj/Ns)*Ns*r + jj%Ns + q*Ns].  FROM_REG / TO_REG: the pass reads /
// leaves its data in the lane's registers (natural layout j + T*m).
template <typename T, int L, int R, int r, int Ns, int SIGN, bool FROM_REG, bool TO_REG, class V>
__device__ __forceinline__ void stockham_pass(T* re, T* im, int j, const V& lds, const T2<T>* w1s,
                                              const T2<T>* whs) {
  constexpr int TL = L / R;
  constexpr int SUB = R / r;
  T vr[R], vi[R];
#pragma unroll
  for (int s = 0; s < SUB; ++s) {
    const int jj = j + TL * s;
#pragma unroll
    for (int q = 0; q < r; ++q) {
      if constexpr (FROM_REG) {
        vr[s * r + q] = re[s + q * SUB];
        vi[s * r + q] = im[s + q * SUB];
      } else {
        const T2<T> v = lds.buf[lds.at(jj + q * (L / r))];
        vr[s * r + q] = v.x;
        vi[s * r + q] = v.y;
      }
    }
    if constexpr (Ns > 1) {
      // twiddles W^(k q), k = jj mod Ns, for q = 1..r-1: W^k and W^(k r/2)
      // come preloaded (q >= r/2 restarts from the latter to bound the
      // recurrence); complex products in between
      const T2<T> w1 = w1s[s];
      const T2<T> wh = whs[s];
      const T w1y = SIGN > 0 ? -w1.y : w1.y;
      const T why = SIGN > 0 ? -wh.y : wh.y;
      T cr = T(1), ci = T(0);
#pragma unroll
      for (int q = 1; q < r; ++q) {
        if (q == r / 2) {
          cr = wh.x;
          ci = why;
        } else {
          const T t = cr * w1.x - ci * w1y;
          ci = cr * w1y + ci * w1.x;
          cr = t;
        }
        const T x = vr[s * r + q] * cr - vi[s * r + q] * ci;
        vi[s * r + q] = vr[s * r + q] * ci + vi[s * r + q] * cr;
        vr[s * r + q] = x;
      }
    }
    dft<T, r, SIGN>(vr + s * r, vi + s * r);
  }
  if constexpr (TO_REG) {
    // last pass: Ns = L/r, so jj < Ns and the outputs are jj + q*Ns = j + T*(s + q*SUB)
#pragma unroll
    for (int s = 0; s < SUB; ++s)
#pragma unroll
      for (int q = 0; q < r; ++q) {
        re[s + q * SUB] = vr[s * r + q];
        im[s + q * SUB] = vi[s * r + q];
      }
  } else {
    __syncthreads();  // previous readers of the buffer are done
#pragma unroll
    for (int s = 0; s < SUB; ++s) {
      const int jj = j + TL * s;
      const int base = (jj / Ns) * Ns * r + (jj & (Ns - 1));
#pragma unroll
      for (int q = 0; q < r; ++q) {
        T2<T> v;
        v.x = vr[s * r + q];
        v.y = vi[s * r + q];
        lds.buf[lds.at(base + q * Ns)] = v;
      }
    }
    __syncthreads();
  }
}

// Radix and sub-transform length of pass P in each direction.
template <int L, int R, int P, bool FWD> struct PassInfo {
  using PL = Plan<L, R>;
  static constexpr int r = FWD ? (P == 0 ? PL::R0 : R) : (P == PL::S - 1 ? PL::R0 : R);
  static constexpr int Ns = P == 0 ? 1 : PassInfo<L, R, P - 1, FWD>::Ns * PassInfo<L, R, P - 1, FWD>::r;
};
template <int L, int R, bool FWD> struct PassInfo<L, R, -1, FWD> {
  static constexpr int r = 1, Ns = 1;
};

// Twiddles of every pass, loaded once per kernel so that no pass waits on a
// table load: w1[P][s] = W_L^(k e), wh[P][s] = W_L^(k (r/2) e), with
// k = (j + T s) mod Ns and e = L/(Ns r).
template <typename T, int L, int R> struct Twiddles {
  static constexpr int S = Plan<L, R>::S;
  T2<T> w1[S][R], wh[S][R];
};
template <typename T, int L, int R, int P, bool FWD>
__device__ __forceinline__ void load_twiddles(Twiddles<T, L, R>& t, int j, const T2<T>* __restrict__ tw) {
  using PI = PassInfo<L, R, P, FWD>;
  constexpr int r = PI::r, Ns = PI::Ns, TL = L / R;
  if constexpr (Ns > 1) {
#pragma unroll
    for (int s = 0; s < R / r; ++s) {
      const int k = (j + TL * s) & (Ns - 1);
      t.w1[P][s] = tw[k * (L / (Ns * r))];
      t.wh[P][s] = tw[k * (r / 2) * (L / (Ns * r))];
    }
  }
  if constexpr (P + 1 < Plan<L, R>::S) load_twiddles<T, L, R, P + 1, FWD>(t, j, tw);
}

template <typename T, int L, int R, int P, bool FWD, class V>
__device__ __forceinline__ void run_passes(T* re, T* im, int j, const V& lds, const Twiddles<T, L, R>& t) {
  using PI = PassInfo<L, R, P, FWD>;
  constexpr int S = Plan<L, R>::S;
  stockham_pass<T, L, R, PI::r, PI::Ns, FWD ? -1 : +1, P == 0, P == S - 1>(re, im, j, lds, t.w1[P], t.wh[P]);
  if constexpr (P + 1 < S) run_passes<T, L, R, P + 1, FWD>(re, im, j, lds, t);
}

// Twiddle sets for a forward and an inverse transform (load both before the
// data arrives; `tw` holds W_L^e = exp(-2 pi i e/L)).
template <typename T, int L, int R>
__device__ __forceinline__ void load_fwd_twiddles(Twiddles<T, L, R>& t, int j, const T2<T>* tw) {
  load_twiddles<T, L, R, 0, true>(t, j, tw);
}
template <typename T, int L, int R>
__device__ __forceinline__ void load_inv_twiddles(Twiddles<T, L, R>& t, int j, const T2<T>* tw) {
  load_twiddles<T, L, R, 0, false>(t, j, tw);
}

// x (time, lane layout j + T*m) -> X (frequency, same layout), radices
// [R0, R, ..., R].  Every lane of the block must call it.
template <typename T, int L, int R, class V>
__device__ __forceinline__ void fft_forward(T* re, T* im, int j, const V& lds, const Twiddles<T, L, R>& t) {
  run_passes<T, L, R, 0, true>(re, im, j, lds, t);
}
// Inverse (unnormalised), radices [R, ..., R, R0].
template <typename T, int L, int R, class V>
__device__ __forceinline__ void fft_inverse(T* re, T* im, int j, const V& lds, const Twiddles<T, L, R>& t) {
  run_passes<T, L, R, 0, false>(re, im, j, lds, t);
}

}  // namespace epdlb
