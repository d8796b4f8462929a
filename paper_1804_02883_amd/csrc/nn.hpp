// Density surrogate: a 4-layer dilated 3x3 convolutional network mapping the
// EPD potentials to the copolymer densities (inference and training kernels,
// BF16 MFMA with FP32 accumulation, gfx950).
//
// Network (periodic grid, channels last):
//   x   = (w_A - <w_A>, w_B - <w_B>, w_S - <w_S>, f_A, 1/N)          5 channels
//   z_l = b_l + sum_t sum_ci a_{l-1}[r + d_l t][ci] W_l[t][ci][co],  d_l = 1, 2, 4, 8
//   a_l = SiLU(z_l) (l = 1..3),  o = z_4 (2 channels),  Phi_hat = softplus(o)
// Inference rescales Phi_hat to the exact species means and takes Phi_S from
// its closed form, so the compressibility constraint on the means holds
// exactly as for the chain propagators (Sec. II, Eqs. for Phi_P and Phi_S).
//
// Tensor storage (bf16, per sample): channel-blocked rows,
//   [y][x / 32][chunk][x % 32][8 channels],  chunk = position / 8,
// so that the 32 consecutive sites an MFMA operand covers read (and the
// epilogue writes) 512 contiguous bytes per 16-byte chunk.  Positions:
//   16-channel tensors (x, output gradient): channel c at position c.
//   64-channel tensors (activations, pre-activations, their gradients): the
//   logical channel c sits at position s(c) chosen so that every lane of the
//   32x32 MFMA epilogue owns 32 contiguous positions (see c_of_s64).
//
// MFMA operands (v_mfma_f32_32x32x16_bf16): A = weights (rows = output
// channels), B = activations (columns = 32 consecutive x sites).  For k-step
// ks, lane l of either operand carries storage input channels
// (CI/2)*(l/32) + 8*ks + [0, 8), so each lane loads CI/2 contiguous channels
// of one site per tap and the packed weight fragments follow the same
// pairing.  Output lane l, register i: site l%32, output row
// 8*(i/4) + 4*(l/32) + i%4.
#pragma once
#include <hip/hip_runtime.h>

#include "kernels.hpp"

namespace epdlb {
namespace nn {

typedef __attribute__((__vector_size__(8 * sizeof(__bf16)))) __bf16 bf16x8;
typedef __attribute__((__vector_size__(16 * sizeof(float)))) float f32x16;
typedef __attribute__((__vector_size__(4 * sizeof(unsigned)))) unsigned u32x4;

constexpr int kLayers = 4;
constexpr int kHid = 64;  // hidden channels
constexpr int kXC = 16;   // stored channels of x and of dL/do
constexpr int kTW = 32;   // tile width (x sites) of the conv kernels
constexpr int kSB = 1;    // site rows per wave in the conv kernels
constexpr int kConvThreads = 512;
constexpr int kConvTH = (kConvThreads / 64) * kSB;  // tile height: 8 rows

// Logical FP32 parameters: for l = 0..3, W_l [9][cin][cout] then b_l [cout].
constexpr int kNnParams = 9 * 5 * 64 + 64 + 2 * (9 * 64 * 64 + 64) + 9 * 64 * 2 + 2;  // 77954
// Packed forward fragments of the four layers (bf16 elements).
constexpr long kFwdFragElems = 9L * 1 * 2 * 512 + 2 * (9L * 4 * 2 * 512) + 9L * 4 * 1 * 512;
// Inference projection of the last hidden layer onto the output taps:
// p[2t + c](r) = sum_ci a3[r][ci] W4[t][ci][c], 18 rows of one 32-row block.
constexpr int kProjRows = 18;
constexpr long kProjFragElems = 4L * 64 * 8;

// logical channel counts and dilations per layer
__host__ __device__ constexpr int cin_of(int l) { return l == 0 ? 5 : kHid; }
__host__ __device__ constexpr int cout_of(int l) { return l == 3 ? 2 : kHid; }
__host__ __device__ constexpr int dil_of(int l) { return 1 << l; }

// Logical channel held at storage position s of a 64-channel tensor.
__host__ __device__ inline int c_of_s64(int s) {
  const int h = s >> 5, b = (s >> 4) & 1, i = s & 15;
  return 32 * b + 8 * (i >> 2) + 4 * h + (i & 3);
}

// v_rcp_f32 (about 1 ulp) instead of an IEEE division: far below the BF16
// rounding of the stored activations
__device__ __forceinline__ float sigm(float z) { return __builtin_amdgcn_rcpf(1.0f + __expf(-z)); }
__device__ __forceinline__ float silu(float z) { return z * sigm(z); }
__device__ __forceinline__ float silu_grad(float z) {
  const float s = sigm(z);
  return s * (1.0f + z * (1.0f - s));
}
// softplus(z) = log(1 + e^z), evaluated without overflow
__device__ __forceinline__ float softplus(float z) { return fmaxf(z, 0.0f) + log1pf(__expf(-fabsf(z))); }

__device__ __forceinline__ bf16x8 as_bf16x8(u32x4 v) { return __builtin_bit_cast(bf16x8, v); }

// Element offset of 16-byte chunk c of site (x, y) in a C-channel tensor.
template <int C>
__device__ __forceinline__ long blk_off(int x, int y, int nx, int c) {
  return ((long(y) * (nx >> 5) + (x >> 5)) * (C / 8) + c) * 256 + (x & 31) * 8;
}

__device__ __forceinline__ double nn_wave_sum(double v) {
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}
__device__ __forceinline__ double nn_wave_max(double v) {
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) v = fmax(v, __shfl_xor(v, o, 64));
  return v;
}

// Block reduction of NV values: sums for the first NS, maxima for the rest.
// Thread 0 receives the results.
template <int NV, int NS>
__device__ __forceinline__ void nn_block_reduce(double (&v)[NV], double* red /*[16*NV]*/) {
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  const int nw = (blockDim.x + 63) >> 6;
#pragma unroll
  for (int i = 0; i < NV; ++i) v[i] = i < NS ? nn_wave_sum(v[i]) : nn_wave_max(v[i]);
  __syncthreads();
  if (lane == 0)
#pragma unroll
    for (int i = 0; i < NV; ++i) red[wid * NV + i] = v[i];
  __syncthreads();
  if (threadIdx.x == 0)
#pragma unroll
    for (int i = 0; i < NV; ++i) {
      double s = red[i];
      for (int w = 1; w < nw; ++w) s = i < NS ? s + red[w * NV + i] : fmax(s, red[w * NV + i]);
      v[i] = s;
    }
}

// ---------------------------------------------------------------------------
// Convolution main loop: acc[sb][nb] += sum over 9 taps and CI channels.
// `w` points to this layer's packed fragments in LDS:
// [tap][ks][nb][lane] of 8 bf16 each.  x: this lane's site column; y0: the
// wave's first row.  nx, ny are powers of two (periodic wrap by masking).
// ---------------------------------------------------------------------------
// The activations of tap t+1 are loaded while tap t's MFMAs run.
template <int CI, int SB>
__device__ __forceinline__ void load_tap(const __bf16* __restrict__ in, int nx, int ny, int d, int x, int y0,
                                         int t, int g, u32x4 (&v)[SB][CI / 16]) {
  constexpr int KS = CI / 16;
  const int ty = t / 3 - 1, tx = t % 3 - 1;
  const int xs = (x + d * tx) & (nx - 1);
#pragma unroll
  for (int sb = 0; sb < SB; ++sb) {
    const int ys = (y0 + sb + d * ty) & (ny - 1);
#pragma unroll
    for (int ks = 0; ks < KS; ++ks)
      v[sb][ks] = *reinterpret_cast<const u32x4*>(in + blk_off<CI>(xs, ys, nx, KS * g + ks));
  }
}

template <int CI, int NB, int SB = kSB>
__device__ __forceinline__ void conv_mma(const __bf16* __restrict__ in, const bf16x8* w, int nx, int ny, int d,
                                         int x, int y0, f32x16 (&acc)[SB][NB]) {
  constexpr int KS = CI / 16;
  const int lane = threadIdx.x & 63;
  const int g = lane >> 5;
#pragma unroll
  for (int sb = 0; sb < SB; ++sb)
#pragma unroll
    for (int nb = 0; nb < NB; ++nb)
#pragma unroll
      for (int i = 0; i < 16; ++i) acc[sb][nb][i] = 0.0f;
  if constexpr (KS == 1) {
    // few MFMAs per tap: issue every tap's loads first
    u32x4 all[9][SB][1];
#pragma unroll
    for (int t = 0; t < 9; ++t) load_tap<CI, SB>(in, nx, ny, d, x, y0, t, g, all[t]);
#pragma unroll
    for (int t = 0; t < 9; ++t)
#pragma unroll
      for (int nb = 0; nb < NB; ++nb) {
        const bf16x8 a = w[(t * NB + nb) * 64 + lane];
#pragma unroll
        for (int sb = 0; sb < SB; ++sb)
          acc[sb][nb] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, as_bf16x8(all[t][sb][0]), acc[sb][nb], 0, 0, 0);
      }
    return;
  }
  u32x4 cur[SB][KS], nxt[SB][KS];
  load_tap<CI, SB>(in, nx, ny, d, x, y0, 0, g, cur);
#pragma unroll 1
  for (int t = 0; t < 9; ++t) {
    if (t < 8) load_tap<CI, SB>(in, nx, ny, d, x, y0, t + 1, g, nxt);
#pragma unroll
    for (int ks = 0; ks < KS; ++ks)
#pragma unroll
      for (int nb = 0; nb < NB; ++nb) {
        const bf16x8 a = w[((t * KS + ks) * NB + nb) * 64 + lane];
#pragma unroll
        for (int sb = 0; sb < SB; ++sb)
          acc[sb][nb] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, as_bf16x8(cur[sb][ks]), acc[sb][nb], 0, 0, 0);
      }
#pragma unroll
    for (int sb = 0; sb < SB; ++sb)
#pragma unroll
      for (int ks = 0; ks < KS; ++ks) cur[sb][ks] = nxt[sb][ks];
  }
}

// Copies `bytes` (multiple of 16) of packed fragments into LDS.
__device__ __forceinline__ void stage_weights(const __bf16* __restrict__ src, bf16x8* dst, int bytes) {
  const u32x4* s = reinterpret_cast<const u32x4*>(src);
  u32x4* d = reinterpret_cast<u32x4*>(dst);
  for (int i = threadIdx.x; i < bytes / 16; i += blockDim.x) d[i] = s[i];
}

// Tiles of the conv kernels: kTW x kConvTH sites; tile index = sample-major.
struct TileInfo {
  int z, x0, y0;
};
__device__ __forceinline__ TileInfo tile_of(int tile, int nx, int tiles_per_sample, int th = kConvTH) {
  TileInfo ti;
  ti.z = tile / tiles_per_sample;
  const int r = tile - ti.z * tiles_per_sample;
  const int tx = nx / kTW;
  ti.x0 = (r % tx) * kTW;
  ti.y0 = (r / tx) * th;
  return ti;
}

// ---------------------------------------------------------------------------
// Hidden-layer convolutions (64 output channels).
//   EPI_FWD:       out = SiLU(z), z = conv + bias      (inference)
//   EPI_FWD_TRAIN: also stores z
//   EPI_BWD:       out = conv * SiLU'(zin)   (backward-data: conv of the
//                  gradient with flipped taps and transposed weights)
// ---------------------------------------------------------------------------
enum { EPI_FWD = 0, EPI_FWD_TRAIN = 1, EPI_BWD = 2, EPI_FWD_PROJ = 3 };

struct ConvArgs {
  const __bf16* in;     // [sample][site][CI]
  long in_bs;           // elements per sample of `in`
  const int* slots;     // if set, sample z reads in + slots[z] * in_bs
  const __bf16* wfrag;  // packed fragments (global)
  const float* bias;    // logical bias (EPI_FWD*)
  __bf16* out;          // [sample][site][64]
  __bf16* zout;         // EPI_FWD_TRAIN
  const __bf16* zin;    // EPI_BWD: pre-activation of the layer below
  long bs;              // elements per sample of out / zout / zin
  const __bf16* pfrag;  // EPI_FWD_PROJ: projection fragments [4 k-steps][64 lanes][8]
  float* proj;          // EPI_FWD_PROJ: 18 FP32 planes of `plane` sites
  long plane;
  int nx, ny, d;
  int tiles_per_sample, ntiles;
};

// Bias + SiLU (forward) or SiLU'(z) (backward-data) and the stores of one
// wave's kSB x 32 sites x 64 channels.  ACC_BIAS: the accumulators started
// at the bias.
template <int EPI, int SB = kSB, bool ACC_BIAS = false>
__device__ __forceinline__ void epilogue_hidden(const ConvArgs& P, f32x16 (&acc)[SB][2], int z, int x, int y0,
                                                const float* bias_s, const bf16x8* pw = nullptr) {
  const int lane = threadIdx.x & 63;
  const int h = lane >> 5;
  if constexpr (EPI == EPI_FWD_PROJ) {
    // the activations this lane holds (positions 32h..32h+31 of its site)
    // are exactly its B operand for k-steps 0..3 of the next contraction
#pragma unroll
    for (int sb = 0; sb < SB; ++sb) {
      f32x16 pr;
#pragma unroll
      for (int i = 0; i < 16; ++i) pr[i] = 0.0f;
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        bf16x8 b;
#pragma unroll
        for (int j = 0; j < 8; ++j) {
          const int s = 8 * q + j, nb = s >> 4, i = s & 15;
          b[j] = __bf16(silu(ACC_BIAS ? acc[sb][nb][i] : acc[sb][nb][i] + bias_s[32 * nb + 8 * (i >> 2) + 4 * h + (i & 3)]));
        }
        pr = __builtin_amdgcn_mfma_f32_32x32x16_bf16(pw[q * 64 + lane], b, pr, 0, 0, 0);
      }
      const long site = long(y0 + sb) * P.nx + x;
#pragma unroll
      for (int i = 0; i < 16; ++i) {
        const int m = 8 * (i >> 2) + 4 * h + (i & 3);
        if (m < kProjRows) P.proj[long(m) * P.plane + site] = pr[i];
      }
    }
    return;
  }
  {
#pragma unroll
    for (int sb = 0; sb < SB; ++sb) {
      // this lane's 32 positions are chunks 4h .. 4h+3 of its site
      const long base = long(z) * P.bs + blk_off<kHid>(x, y0 + sb, P.nx, 4 * h);
      float v[32];
      if (EPI == EPI_BWD) {
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const bf16x8 zz = as_bf16x8(*reinterpret_cast<const u32x4*>(P.zin + base + q * 256));
#pragma unroll
          for (int j = 0; j < 8; ++j) {
            const int s = 8 * q + j;  // position within this lane's 32
            v[s] = acc[sb][s >> 4][s & 15] * silu_grad(float(zz[j]));
          }
        }
      } else {
#pragma unroll
        for (int s = 0; s < 32; ++s) {
          const int nb = s >> 4, i = s & 15;
          v[s] = ACC_BIAS ? acc[sb][nb][i] : acc[sb][nb][i] + bias_s[32 * nb + 8 * (i >> 2) + 4 * h + (i & 3)];
        }
        if (EPI == EPI_FWD_TRAIN) {
#pragma unroll
          for (int q = 0; q < 4; ++q) {
            bf16x8 o;
#pragma unroll
            for (int j = 0; j < 8; ++j) o[j] = __bf16(v[8 * q + j]);
            *reinterpret_cast<u32x4*>(P.zout + base + q * 256) = __builtin_bit_cast(u32x4, o);
          }
        }
#pragma unroll
        for (int s = 0; s < 32; ++s) v[s] = silu(v[s]);
      }
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        bf16x8 o;
#pragma unroll
        for (int j = 0; j < 8; ++j) o[j] = __bf16(v[8 * q + j]);
        *reinterpret_cast<u32x4*>(P.out + base + q * 256) = __builtin_bit_cast(u32x4, o);
      }
    }
  }
}

template <int CI, int EPI, int SB = kSB, int NW = kConvThreads / 64>
__global__ void __launch_bounds__(NW * 64) k_conv_hidden(ConvArgs P) {
  extern __shared__ __attribute__((aligned(16))) unsigned char nn_lds[];
  constexpr int KS = CI / 16, NB = 2;
  bf16x8* w = reinterpret_cast<bf16x8*>(nn_lds);
  __shared__ float bias_s[kHid];
  __shared__ bf16x8 pw_s[EPI == EPI_FWD_PROJ ? 4 * 64 : 1];
  stage_weights(P.wfrag, w, 9 * KS * NB * 64 * 16);
  if constexpr (EPI == EPI_FWD_PROJ) stage_weights(P.pfrag, pw_s, 4 * 64 * 16);
  if (EPI != EPI_BWD && threadIdx.x < kHid) bias_s[threadIdx.x] = P.bias[threadIdx.x];
  __syncthreads();
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6, h = lane >> 5;
  const int blk = xcd_tile(blockIdx.x, gridDim.x);
  for (int tile = blk; tile < P.ntiles; tile += gridDim.x) {
    const TileInfo ti = tile_of(tile, P.nx, P.tiles_per_sample, NW * SB);
    const __bf16* in = P.in + long(P.slots ? P.slots[ti.z] : ti.z) * P.in_bs;
    const int x = ti.x0 + (lane & 31);
    const int y0 = ti.y0 + wid * SB;
    f32x16 acc[SB][NB];
    conv_mma<CI, NB, SB>(in, w, P.nx, P.ny, P.d, x, y0, acc);
    epilogue_hidden<EPI, SB>(P, acc, ti.z, x, y0, bias_s, pw_s);
  }
}

// ---------------------------------------------------------------------------
// 64-channel hidden convolutions on row tiles (all epilogue kinds).
// One workgroup of kConv64Threads per CU (4 waves per SIMD) keeps the layer's
// packed weights in LDS; each wave walks 32-site row tiles of one contiguous
// band of the tile range (one band per XCD, so the halo rows a band re-reads
// stay in that XCD's L2).
// The tensor offset of (x, y, chunk) separates into a row term, uniform over
// the wave, and a per-lane column term, so the activations come in through
// buffer loads with the row term as the scalar offset and the chunk step as
// the immediate: no per-tap address arithmetic.  The next tap's activations
// are issued before the current tap's weight fragments and MFMAs (scheduling
// fences keep that order; the other waves of the SIMD cover the LDS latency);
// forward kinds start the accumulators at the bias.
// ---------------------------------------------------------------------------
constexpr unsigned kBufWord3 = 0x00020000u;  // raw buffer, 32-bit elements
constexpr int kConv64Threads = 1024;

__device__ __forceinline__ void load_tap_buf(__amdgpu_buffer_rsrc_t r, int row_off, int col_off, u32x4 (&b)[4]) {
#pragma unroll
  for (int ks = 0; ks < 4; ++ks)
    b[ks] = __builtin_bit_cast(u32x4, __builtin_amdgcn_raw_buffer_load_b128(r, col_off + ks * 512, row_off, 0));
}
__device__ __forceinline__ void load_frags(const bf16x8* w, int t, bf16x8 (&a)[8]) {
  const int lane = threadIdx.x & 63;
#pragma unroll
  for (int j = 0; j < 8; ++j) a[j] = w[(t * 8 + j) * 64 + lane];
}
__device__ __forceinline__ void mma_tap(const bf16x8 (&a)[8], const u32x4 (&b)[4], f32x16 (&acc)[1][2]) {
#pragma unroll
  for (int ks = 0; ks < 4; ++ks)
#pragma unroll
    for (int nb = 0; nb < 2; ++nb)
      acc[0][nb] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a[ks * 2 + nb], as_bf16x8(b[ks]), acc[0][nb], 0, 0, 0);
}

template <int EPI>
__global__ void __launch_bounds__(kConv64Threads) __attribute__((amdgpu_waves_per_eu(4, 4))) k_conv64(ConvArgs P) {
  constexpr int NW = kConv64Threads / 64;
  extern __shared__ __attribute__((aligned(16))) unsigned char nn_lds[];
  bf16x8* w = reinterpret_cast<bf16x8*>(nn_lds);
  __shared__ __attribute__((aligned(16))) float bias_s[kHid];
  __shared__ bf16x8 pw_s[EPI == EPI_FWD_PROJ ? 4 * 64 : 1];
  stage_weights(P.wfrag, w, 9 * 4 * 2 * 64 * 16);
  if constexpr (EPI == EPI_FWD_PROJ) stage_weights(P.pfrag, pw_s, 4 * 64 * 16);
  if (EPI != EPI_BWD && threadIdx.x < kHid) bias_s[threadIdx.x] = P.bias[threadIdx.x];
  __syncthreads();
  const int lane = threadIdx.x & 63, g = lane >> 5;
  const int wid = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int nx = P.nx, ny = P.ny, d = P.d;
  const int rpr = nx >> 5, lg = __builtin_ctz(rpr);  // row tiles per grid row
  const int row_bytes = rpr * 4096;                  // 32 sites x 64 channels x 2 bytes per row tile
  // tiles [start, start + band) for this workgroup's XCD
  int start = 0, band = P.ntiles, loc = blockIdx.x, per = gridDim.x;
  if ((gridDim.x % kNumXcd) == 0 && (P.ntiles % kNumXcd) == 0) {
    band = P.ntiles / kNumXcd;
    start = (blockIdx.x % kNumXcd) * band;
    loc = blockIdx.x / kNumXcd;
    per = gridDim.x / kNumXcd;
  }
  for (int m = loc * NW + wid; m < band; m += per * NW) {
    const int rt = start + m;
    const int z = rt / P.tiles_per_sample;
    const int r = rt - z * P.tiles_per_sample;
    const int y = r >> lg;
    const int x = ((r & (rpr - 1)) << 5) + (lane & 31);
    const __bf16* in = P.in + long(P.slots ? P.slots[z] : z) * P.in_bs;
    const __amdgpu_buffer_rsrc_t rs =
        __builtin_amdgcn_make_buffer_rsrc(const_cast<__bf16*>(in), 0, int(P.in_bs * 2), kBufWord3);
    int ro[3], co[3];
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      ro[k] = ((y + (k - 1) * d) & (ny - 1)) * row_bytes;
      const int xs = (x + (k - 1) * d) & (nx - 1);
      co[k] = (xs >> 5) * 4096 + (xs & 31) * 16 + g * 2048;  // lane group g holds chunks 4g .. 4g+3
    }
    f32x16 acc[1][2];
#pragma unroll
    for (int nb = 0; nb < 2; ++nb)
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        // output rows of register group q: 32 nb + 8 q + 4 g + [0, 4)
        float4 bv = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
        if (EPI != EPI_BWD) bv = *reinterpret_cast<const float4*>(&bias_s[32 * nb + 8 * q + 4 * g]);
        acc[0][nb][4 * q + 0] = bv.x;
        acc[0][nb][4 * q + 1] = bv.y;
        acc[0][nb][4 * q + 2] = bv.z;
        acc[0][nb][4 * q + 3] = bv.w;
      }
    u32x4 b0[4], b1[4];
    load_tap_buf(rs, ro[0], co[0], b0);
#pragma unroll
    for (int t = 0; t < 9; ++t) {
      if (t < 8) {
        const int tn = t + 1;  // taps in (ty, tx) row-major order
        if (t & 1) load_tap_buf(rs, ro[tn / 3], co[tn % 3], b0);
        else load_tap_buf(rs, ro[tn / 3], co[tn % 3], b1);
      }
      __builtin_amdgcn_sched_barrier(0);
      bf16x8 a[8];
      load_frags(w, t, a);
      if (t & 1) mma_tap(a, b1, acc);
      else mma_tap(a, b0, acc);
      __builtin_amdgcn_sched_barrier(0);
    }
    epilogue_hidden<EPI, 1, EPI != EPI_BWD>(P, acc, z, x, y, bias_s, pw_s);
  }
}

// ---------------------------------------------------------------------------
// First layer for inference, reading the potentials directly: the B operand
// of lane group 0 is (w_A - <w_A>, w_B - <w_B>, w_S - <w_S>, f_A, 1/N, 0, 0, 0)
// in BF16 (the same values k_nn_input stores), group 1 carries the zero
// channels 8..15.
// ---------------------------------------------------------------------------
template <typename T>
struct InArgs {
  ConvArgs c;        // out, bs, nx, ny, d = 1, tiles, wfrag (16-channel layer), bias
  const T* w;        // 3 planes
  const double* mean;
  long plane;
  float fA, invN;
};

// Row tiles in XCD bands as in k_conv64 (c.ntiles counts 32-site rows).  A
// wave converts the 3 x 34 sites its row tile reads (halo included) once into
// B operands in its own LDS slots; each tap then reads its operand with one
// 16-byte LDS load (lane group 1 reads the zero slot).
constexpr int kInStage = 3 * 34 + 1;  // B operands per wave: 3 rows x 34 sites, then zero

template <typename T>
__global__ void __launch_bounds__(kConvThreads) __attribute__((amdgpu_waves_per_eu(4, 4))) k_conv_in(InArgs<T> P) {
  constexpr int NW = kConvThreads / 64;
  extern __shared__ __attribute__((aligned(16))) unsigned char nn_lds[];
  bf16x8* w = reinterpret_cast<bf16x8*>(nn_lds);
  __shared__ __attribute__((aligned(16))) float bias_s[kHid];
  __shared__ bf16x8 stage_s[NW * kInStage];
  stage_weights(P.c.wfrag, w, 9 * 2 * 64 * 16);
  if (threadIdx.x < kHid) bias_s[threadIdx.x] = P.c.bias[threadIdx.x];
  const int lane = threadIdx.x & 63, g = lane >> 5;
  const int wid = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  bf16x8* st = stage_s + wid * kInStage;
  if (lane == 0) {
    bf16x8 zero;
#pragma unroll
    for (int j = 0; j < 8; ++j) zero[j] = __bf16(0.0f);
    st[kInStage - 1] = zero;
  }
  __syncthreads();
  const int nx = P.c.nx, ny = P.c.ny;
  const int rpr = nx >> 5, lg = __builtin_ctz(rpr);
  const double dA = P.mean[0], dB = P.mean[1], dS = P.mean[2];
  const __bf16 bfA = __bf16(P.fA), binvN = __bf16(P.invN);
  int start = 0, band = P.c.ntiles, loc = blockIdx.x, per = gridDim.x;
  if ((gridDim.x % kNumXcd) == 0 && (P.c.ntiles % kNumXcd) == 0) {
    band = P.c.ntiles / kNumXcd;
    start = (blockIdx.x % kNumXcd) * band;
    loc = blockIdx.x / kNumXcd;
    per = gridDim.x / kNumXcd;
  }
  for (int m = loc * NW + wid; m < band; m += per * NW) {
    const int r = start + m;  // one sample
    const int y = r >> lg;
    const int x0 = (r & (rpr - 1)) << 5;
    // the previous tile's reads of this wave's slots come before the rewrite
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    // stage: slot e = row * 34 + col holds site (x0 - 1 + col, y - 1 + row)
#pragma unroll
    for (int k = 0; k < 2; ++k) {
      const int e = lane + 64 * k;
      if (e < 3 * 34) {
        const int row = e / 34, col = e - row * 34;
        const long i = long((y - 1 + row) & (ny - 1)) * nx + ((x0 - 1 + col) & (nx - 1));
        bf16x8 b;
        b[0] = __bf16(float(double(P.w[i]) - dA));
        b[1] = __bf16(float(double(P.w[P.plane + i]) - dB));
        b[2] = __bf16(float(double(P.w[2 * P.plane + i]) - dS));
        b[3] = bfA;
        b[4] = binvN;
        b[5] = b[6] = b[7] = __bf16(0.0f);
        st[e] = b;
      }
    }
    f32x16 acc[1][2];
#pragma unroll
    for (int nb = 0; nb < 2; ++nb)
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const float4 bv = *reinterpret_cast<const float4*>(&bias_s[32 * nb + 8 * q + 4 * g]);
        acc[0][nb][4 * q + 0] = bv.x;
        acc[0][nb][4 * q + 1] = bv.y;
        acc[0][nb][4 * q + 2] = bv.z;
        acc[0][nb][4 * q + 3] = bv.w;
      }
    // the slots written above by other lanes of this wave are visible here
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    const int xl = lane & 31;
#pragma unroll
    for (int t = 0; t < 9; ++t) {
      const bf16x8 b = st[g ? kInStage - 1 : (t / 3) * 34 + xl + (t % 3)];
#pragma unroll
      for (int nb = 0; nb < 2; ++nb)
        acc[0][nb] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(w[(t * 2 + nb) * 64 + lane], b, acc[0][nb], 0, 0, 0);
    }
    epilogue_hidden<EPI_FWD, 1, true>(P.c, acc, 0, x0 + xl, y, bias_s);
  }
}

// ---------------------------------------------------------------------------
// Output of the inference path: o_c(r) = b_c + sum_t p[2t + c](r + 8 (ty, tx)),
// Phi_hat = softplus(o) into two planes of T, per-workgroup sums in
// partials[2*block + c].
// ---------------------------------------------------------------------------
template <typename T>
__global__ void __launch_bounds__(256) k_nn_out_stencil(const float* __restrict__ proj, const float* __restrict__ bias,
                                                        T* __restrict__ phi, double* __restrict__ partials, int nx,
                                                        int ny, int d) {
  __shared__ double red[16 * 2];
  const long n = long(nx) * ny;
  const long i = long(blockIdx.x) * blockDim.x + threadIdx.x;
  double r[2] = {0.0, 0.0};
  if (i < n) {
    const int x = int(i % nx), y = int(i / nx);
    float o0 = bias[0], o1 = bias[1];
#pragma unroll
    for (int t = 0; t < 9; ++t) {
      const long j = long((y + d * (t / 3 - 1)) & (ny - 1)) * nx + ((x + d * (t % 3 - 1)) & (nx - 1));
      o0 += proj[long(2 * t) * n + j];
      o1 += proj[long(2 * t + 1) * n + j];
    }
    const float p0 = softplus(o0), p1 = softplus(o1);
    phi[i] = T(p0);
    phi[n + i] = T(p1);
    r[0] = p0;
    r[1] = p1;
  }
  nn_block_reduce<2, 2>(r, red);
  if (threadIdx.x == 0) {
    partials[2 * blockIdx.x] = r[0];
    partials[2 * blockIdx.x + 1] = r[1];
  }
}

// Projection fragments: lane l, k-step q, element j: row m = l % 32 (tap m / 2,
// output m % 2), stored input position 32 (l / 32) + 8 q + j.
__global__ void __launch_bounds__(256) k_pack_proj(const float* __restrict__ W4, __bf16* __restrict__ frag) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= int(kProjFragElems)) return;
  const int j = e & 7, lane = (e >> 3) & 63, q = e >> 9;
  const int m = lane & 31, s = 32 * (lane >> 5) + 8 * q + j;
  const int ci = c_of_s64(s);
  float v = 0.0f;
  if (m < kProjRows) v = W4[(long(m >> 1) * kHid + ci) * 2 + (m & 1)];
  frag[e] = __bf16(v);
}

// ---------------------------------------------------------------------------
// Output layer (64 -> 2, one 32-row MFMA block of which rows 0, 1 are used).
//   EPO_INFER: writes softplus(o) to two planes of T; per-workgroup sums of
//              them go to partials[2*block + c].
//   EPO_TRAIN: loss against targets, dL/do into the 16-channel gradient
//              tensor; per-workgroup (sum of squared scaled residuals, max
//              abs error) in partials[2*block + {0, 1}].
// ---------------------------------------------------------------------------
enum { EPO_INFER = 0, EPO_TRAIN = 1 };

template <typename T>
struct OutArgs {
  const __bf16* in;
  long in_bs;
  const __bf16* wfrag;
  const float* bias;
  T* phi;             // EPO_INFER: 2 planes of `plane` elements
  long plane;
  const float* tgt;   // EPO_TRAIN: per slot 2 planes of float
  long tgt_bs;
  const int* slots;   // EPO_TRAIN: dataset slot of sample z
  __bf16* gout;       // EPO_TRAIN: [sample][site][16]
  float inv_phiP;     // 1 / phibar_P
  float gscale;       // 2 / (M phibar_P), M = scaled residuals in the loss
  double* partials;
  int nx, ny, d;
  int tiles_per_sample, ntiles;
};

template <typename T, int EPO>
__global__ void __launch_bounds__(kConvThreads) k_conv_out(OutArgs<T> P) {
  extern __shared__ __attribute__((aligned(16))) unsigned char nn_lds[];
  constexpr int CI = kHid, KS = CI / 16, NB = 1;
  bf16x8* w = reinterpret_cast<bf16x8*>(nn_lds);
  stage_weights(P.wfrag, w, 9 * KS * NB * 64 * 16);
  __syncthreads();
  const float b0 = P.bias[0], b1 = P.bias[1];
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  double r[2] = {0.0, 0.0};  // INFER: sums of Phi_hat_A, B; TRAIN: sum r^2, max |err|
  const int blk = xcd_tile(blockIdx.x, gridDim.x);
  for (int tile = blk; tile < P.ntiles; tile += gridDim.x) {
    const TileInfo ti = tile_of(tile, P.nx, P.tiles_per_sample);
    const __bf16* in = P.in + long(ti.z) * P.in_bs;
    const int x = ti.x0 + (lane & 31);
    const int y0 = ti.y0 + wid * kSB;
    f32x16 acc[kSB][NB];
    conv_mma<CI, NB>(in, w, P.nx, P.ny, P.d, x, y0, acc);
    if (lane < 32) {
#pragma unroll
      for (int sb = 0; sb < kSB; ++sb) {
        const long site = long(y0 + sb) * P.nx + x;
        const float o0 = acc[sb][0][0] + b0, o1 = acc[sb][0][1] + b1;
        const float p0 = softplus(o0), p1 = softplus(o1);
        if (EPO == EPO_INFER) {
          P.phi[long(ti.z) * 2 * P.plane + site] = T(p0);
          P.phi[long(ti.z) * 2 * P.plane + P.plane + site] = T(p1);
          r[0] += double(p0);
          r[1] += double(p1);
        } else {
          const float* tg = P.tgt + long(P.slots[ti.z]) * P.tgt_bs;
          const float e0 = p0 - tg[site], e1 = p1 - tg[P.plane + site];
          const float r0 = e0 * P.inv_phiP, r1 = e1 * P.inv_phiP;
          r[0] += double(r0) * r0 + double(r1) * r1;
          r[1] = fmax(r[1], fmax(fabs(double(e0)), fabs(double(e1))));
          bf16x8 gv, zero;
#pragma unroll
          for (int j = 0; j < 8; ++j) gv[j] = zero[j] = __bf16(0.0f);
          gv[0] = __bf16(P.gscale * r0 * sigm(o0));
          gv[1] = __bf16(P.gscale * r1 * sigm(o1));
          __bf16* gp = P.gout + long(ti.z) * P.plane * kXC;
          *reinterpret_cast<u32x4*>(gp + blk_off<kXC>(x, y0 + sb, P.nx, 0)) = __builtin_bit_cast(u32x4, gv);
          *reinterpret_cast<u32x4*>(gp + blk_off<kXC>(x, y0 + sb, P.nx, 1)) = __builtin_bit_cast(u32x4, zero);
        }
      }
    }
  }
  __shared__ double red[16 * 2];
  if (EPO == EPO_INFER)
    nn_block_reduce<2, 2>(r, red);
  else
    nn_block_reduce<2, 1>(r, red);
  if (threadIdx.x == 0) {
    P.partials[2 * blockIdx.x] = r[0];
    P.partials[2 * blockIdx.x + 1] = r[1];
  }
}

// ---------------------------------------------------------------------------
// Weight gradients: dW[t][ci][co] = sum over sites r of a[r + d t][ci] g[r][co]
// (and db[co] = sum_r g[r][co]).  One workgroup = 9 waves, wave t owns tap t;
// a tile of kTW x TH sites of g and its halo of a are staged in LDS (row
// stride C + 8 bf16: the two lane halves of a fragment read sites 8 apart,
// which then fall 32 banks apart).  MFMA with the site index as the
// contraction: A = a (rows = ci), B = g (columns = co).  Each workgroup
// accumulates its tiles in registers and writes one partial; a second kernel
// adds the partials in workgroup order (deterministic).
// ---------------------------------------------------------------------------
struct WgradArgs {
  const __bf16* a;  // [sample][site][CI]
  long a_bs;
  const int* slots;  // if set, sample z of `a` is slot slots[z]
  const __bf16* g;   // [sample][site][CO]
  long g_bs;
  float* part;   // [block][9][CI][CO]
  float* partb;  // [block][CO]
  int nx, ny, d;
  int tiles_per_sample, ntiles;
};

template <int C>
__device__ __forceinline__ void stage_tile(const __bf16* __restrict__ src, __bf16* dst, int nx, int ny, int gx0,
                                           int gy0, int hw, int hh) {
  constexpr int RS = C + 8;
  constexpr int CH = C / 8;  // 16-byte chunks per site
  const int sites = hw * hh;
  const int total = sites * CH;
  for (int e = threadIdx.x; e < total; e += blockDim.x) {
    const int ch = e / sites, s = e - ch * sites;  // consecutive threads: consecutive sites
    const int hx = s % hw, hy = s / hw;
    const int gx = (gx0 + hx) & (nx - 1), gy = (gy0 + hy) & (ny - 1);
    const u32x4 v = *reinterpret_cast<const u32x4*>(src + blk_off<C>(gx, gy, nx, ch));
    *reinterpret_cast<u32x4*>(dst + long(s) * RS + 8 * ch) = v;
  }
}

template <int CI, int CO, int TH>
__global__ void __launch_bounds__(576) k_conv_wgrad(WgradArgs P) {
  extern __shared__ __attribute__((aligned(16))) unsigned char nn_lds[];
  constexpr int RA = CI + 8, RG = CO + 8;
  constexpr int MB = CI > 32 ? CI / 32 : 1;
  constexpr int NB = CO > 32 ? CO / 32 : 1;
  const int d = P.d;
  const int hw = kTW + 2 * d, hh = TH + 2 * d;
  __bf16* la = reinterpret_cast<__bf16*>(nn_lds);
  __bf16* lg = la + long(hw) * hh * RA;
  const int lane = threadIdx.x & 63, t = threadIdx.x >> 6, gsel = lane >> 5;
  const int ty = t / 3 - 1, tx = t % 3 - 1;
  f32x16 acc[MB][NB], accb[NB];
#pragma unroll
  for (int mb = 0; mb < MB; ++mb)
#pragma unroll
    for (int nb = 0; nb < NB; ++nb)
#pragma unroll
      for (int i = 0; i < 16; ++i) acc[mb][nb][i] = 0.0f;
#pragma unroll
  for (int nb = 0; nb < NB; ++nb)
#pragma unroll
    for (int i = 0; i < 16; ++i) accb[nb][i] = 0.0f;
  bf16x8 ones;
#pragma unroll
  for (int j = 0; j < 8; ++j) ones[j] = __bf16(1.0f);
  const int txs = P.nx / kTW;
  for (int tile = blockIdx.x; tile < P.ntiles; tile += gridDim.x) {
    const int z = tile / P.tiles_per_sample;
    const int rr = tile - z * P.tiles_per_sample;
    const int x0 = (rr % txs) * kTW, y0 = (rr / txs) * TH;
    const __bf16* a = P.a + long(P.slots ? P.slots[z] : z) * P.a_bs;
    const __bf16* g = P.g + long(z) * P.g_bs;
    __syncthreads();  // previous tile's reads are done
    stage_tile<CI>(a, la, P.nx, P.ny, x0 - d, y0 - d, hw, hh);
    stage_tile<CO>(g, lg, P.nx, P.ny, x0, y0, kTW, TH);
    __syncthreads();
#pragma unroll 1
    for (int ks = 0; ks < TH * kTW / 16; ++ks) {
      const int yy = ks >> 1, xb = (ks & 1) * 16 + 8 * gsel;
      bf16x8 A[MB], B[NB];
#pragma unroll
      for (int mb = 0; mb < MB; ++mb) {
        const int ci = 32 * mb + (lane & 31);
        const __bf16* src = la + (long(yy + d + d * ty) * hw + (xb + d + d * tx)) * RA + ci;
#pragma unroll
        for (int j = 0; j < 8; ++j) A[mb][j] = ci < CI ? src[j * RA] : __bf16(0.0f);
      }
#pragma unroll
      for (int nb = 0; nb < NB; ++nb) {
        const int co = 32 * nb + (lane & 31);
        const __bf16* src = lg + (long(yy) * kTW + xb) * RG + co;
#pragma unroll
        for (int j = 0; j < 8; ++j) B[nb][j] = co < CO ? src[j * RG] : __bf16(0.0f);
      }
#pragma unroll
      for (int mb = 0; mb < MB; ++mb)
#pragma unroll
        for (int nb = 0; nb < NB; ++nb)
          acc[mb][nb] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(A[mb], B[nb], acc[mb][nb], 0, 0, 0);
      if (t == 4)
#pragma unroll
        for (int nb = 0; nb < NB; ++nb)
          accb[nb] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ones, B[nb], accb[nb], 0, 0, 0);
    }
  }
  float* part = P.part + (long(blockIdx.x) * 9 + t) * CI * CO;
#pragma unroll
  for (int mb = 0; mb < MB; ++mb)
#pragma unroll
    for (int nb = 0; nb < NB; ++nb)
#pragma unroll
      for (int i = 0; i < 16; ++i) {
        const int ci = 32 * mb + 8 * (i >> 2) + 4 * (lane >> 5) + (i & 3);
        const int co = 32 * nb + (lane & 31);
        if (ci < CI && co < CO) part[ci * CO + co] = acc[mb][nb][i];
      }
  if (t == 4 && lane < 32)
#pragma unroll
    for (int nb = 0; nb < NB; ++nb) {
      const int co = 32 * nb + lane;
      if (co < CO) P.partb[long(blockIdx.x) * CO + co] = accb[nb][0];
    }
}

// Sums the weight-gradient partials in block order and maps storage channel
// positions back to logical (ci, co).  grad: this layer's logical W
// [9][cil][col] followed by its bias [col].
struct WredArgs {
  const float* part;
  const float* partb;
  int nblocks;
  int CIs, COs;        // stored channel counts of a and g
  int in64, out64;     // 1 if the tensor uses the 64-channel storage order
  int cil, col;        // logical channel counts
  float* grad;
};

__device__ __forceinline__ int s_of_c64(int c) {
  const int b = c >> 5, r = c & 31;
  const int i = 4 * (r >> 3) + (r & 3), h = (r >> 2) & 1;
  return 32 * h + 16 * b + i;
}

__global__ void __launch_bounds__(256) k_wgrad_reduce(WredArgs P) {
  const int nw = 9 * P.cil * P.col;
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e < nw) {
    const int co = e % P.col, ci = (e / P.col) % P.cil, t = e / (P.col * P.cil);
    const int si = P.in64 ? s_of_c64(ci) : ci, so = P.out64 ? s_of_c64(co) : co;
    const long stride = long(9) * P.CIs * P.COs;
    const float* p = P.part + (long(t) * P.CIs + si) * P.COs + so;
    float s = 0.0f;
    for (int b = 0; b < P.nblocks; ++b) s += p[b * stride];
    P.grad[e] = s;
  } else if (e < nw + P.col) {
    const int co = e - nw;
    const int so = P.out64 ? s_of_c64(co) : co;
    float s = 0.0f;
    for (int b = 0; b < P.nblocks; ++b) s += P.partb[long(b) * P.COs + so];
    P.grad[e] = s;
  }
}

// ---------------------------------------------------------------------------
// Packing FP32 logical weights W[t][ci][co] into MFMA A fragments.
//   forward:  rows = co, k = stored input channel of a_{l-1}
//   backward: rows = ci, k = stored channel of g_l, tap 8 - t
// ---------------------------------------------------------------------------
struct PackArgs {
  const float* W;  // logical [9][cil][col]
  int cil, col;
  int CIs, NB;     // stored input channels of the operator, output blocks
  int in64;        // operator input uses the 64-channel storage order
  int bwd;
  __bf16* frag;    // [9][CIs/16][NB][64][8]
};

__global__ void __launch_bounds__(256) k_pack(PackArgs P) {
  const int KS = P.CIs / 16;
  const long total = long(9) * KS * P.NB * 64 * 8;
  const long e = long(blockIdx.x) * blockDim.x + threadIdx.x;
  if (e >= total) return;
  const int j = int(e & 7), lane = int((e >> 3) & 63);
  long rest = e >> 9;
  const int nb = int(rest % P.NB);
  rest /= P.NB;
  const int ks = int(rest % KS), t = int(rest / KS);
  const int s_in = (P.CIs / 2) * (lane >> 5) + 8 * ks + j;
  const int c_in = P.in64 ? c_of_s64(s_in) : s_in;
  const int r = 32 * nb + (lane & 31);
  float v = 0.0f;
  if (!P.bwd) {
    if (c_in < P.cil && r < P.col) v = P.W[(long(t) * P.cil + c_in) * P.col + r];
  } else {
    if (c_in < P.col && r < P.cil) v = P.W[(long(8 - t) * P.cil + r) * P.col + c_in];
  }
  P.frag[e] = __bf16(v);
}

// Mini-batch slot list passed by value (kernel arguments are copied at
// launch), written to device memory in stream order.
constexpr int kMaxBatch = 64;
struct SlotList {
  int n;
  int s[kMaxBatch];
};
__global__ void k_set_slots(SlotList L, int* dst) {
  if (threadIdx.x < L.n) dst[threadIdx.x] = L.s[threadIdx.x];
}

// Adam (Kingma & Ba 2015) on FP32 master weights; c1 = lr / (1 - b1^t),
// c2 = 1 / (1 - b2^t) are the bias corrections of step t.
__global__ void __launch_bounds__(256) k_adam(float* w, const float* g, float* m, float* v, int n, float b1,
                                             float b2, float c1, float c2, float eps) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n) return;
  const float gg = g[e];
  const float mm = b1 * m[e] + (1.0f - b1) * gg;
  const float vv = b2 * v[e] + (1.0f - b2) * gg * gg;
  m[e] = mm;
  v[e] = vv;
  w[e] -= c1 * mm / (sqrtf(vv * c2) + eps);
}

// ---------------------------------------------------------------------------
// Network input from the potentials: x[site] = (w_I - <w_I>, f_A, 1/N, 0...).
// Optionally copies Phi_A, Phi_B to float target planes (training pairs).
// ---------------------------------------------------------------------------
template <typename T>
__global__ void __launch_bounds__(256) k_nn_input(const T* __restrict__ w, const double* __restrict__ mean,
                                                  long n, int nx, float fA, float invN, __bf16* __restrict__ x,
                                                  const T* __restrict__ phi, float* __restrict__ tgt) {
  const long i = long(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int sx = int(i % nx), sy = int(i / nx);
  bf16x8 v0, v1;
  v0[0] = __bf16(float(double(w[i]) - mean[0]));
  v0[1] = __bf16(float(double(w[n + i]) - mean[1]));
  v0[2] = __bf16(float(double(w[2 * n + i]) - mean[2]));
  v0[3] = __bf16(fA);
  v0[4] = __bf16(invN);
#pragma unroll
  for (int j = 5; j < 8; ++j) v0[j] = __bf16(0.0f);
#pragma unroll
  for (int j = 0; j < 8; ++j) v1[j] = __bf16(0.0f);
  *reinterpret_cast<u32x4*>(x + blk_off<kXC>(sx, sy, nx, 0)) = __builtin_bit_cast(u32x4, v0);
  *reinterpret_cast<u32x4*>(x + blk_off<kXC>(sx, sy, nx, 1)) = __builtin_bit_cast(u32x4, v1);
  if (tgt) {
    tgt[i] = float(phi[i]);
    tgt[n + i] = float(phi[n + i]);
  }
}


// Maximum of non-negative doubles: their bit patterns order like the values
// (a NaN orders above every finite value and so stays visible).
// Most workgroups find the running maximum already larger and skip the atomic.
__device__ __forceinline__ void atomic_max_nonneg(double* p, double v) {
  unsigned long long* q = reinterpret_cast<unsigned long long*>(p);
  const unsigned long long bits = static_cast<unsigned long long>(__double_as_longlong(v));
  if (__hip_atomic_load(q, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) >= bits) return;
  atomicMax(q, bits);
}

// ---------------------------------------------------------------------------
// Surrogate densities from the output planes (after k_conv_out<EPO_INFER>):
//   Phi_A = Phi_hat_A f_A phibar_P n / sum Phi_hat_A   (same for B)
//   Phi_S = V phibar_S exp(-(w_S - c_S)) / Q_S          (closed form)
//   S     = sum_I Phi_I / D_I - S~ [- corr]
// mode 0 (surrogate step): the densities become the state; the residual
//   max |sum Phi - 1| goes to scal[kNnResid].
// mode 1 (exact step, the state holds the exact densities): S is still
//   formed from the surrogate (the force differences one estimator at both
//   ends); corr = sum_{A,B} (Phi_NN - Phi_exact)/D_I is kept for the next
//   step, whose S~ was advected from exact densities; the surrogate's error
//   and the exact residual go to scal.
// use_corr: the previous step was exact.
// ---------------------------------------------------------------------------
template <typename T>
struct NormArgs {
  const T* src;  // Phi_hat A, B (may alias phi in mode 0)
  T* phi;        // state densities, 3 planes
  const double* part;
  int nslots;
  const T* wS;
  const T* stilde;
  T* S;
  T* corr;
  double* scal;
  long n;
  double sumA, sumB;  // exact site sums of Phi_A and Phi_B
  double V, phiSbar, invDA, invDB, invDS;
  int mode, use_corr;
};

template <typename T>
__global__ void __launch_bounds__(256) k_nn_norm(NormArgs<T> P) {
  __shared__ double red[16 * 3];
  __shared__ double scale_s[2];
  const long n = P.n;
  const long i = long(blockIdx.x) * blockDim.x + threadIdx.x;
  const bool in = i < n;
  // this site's inputs are issued first, so their latency overlaps that of
  // the partial sums below
  T hA = T(0), hB = T(0), wS = T(0), st = T(0), cr = T(0), eA = T(0), eB = T(0), eS = T(0);
  if (in) {
    hA = P.src[i];
    hB = P.src[n + i];
    wS = P.wS[i];
    st = P.stilde[i];
    if (P.use_corr) cr = P.corr[i];
    if (P.mode != 0) {
      eA = P.phi[i];
      eB = P.phi[n + i];
      eS = P.phi[2 * n + i];
    }
  }
  {
    // four slots per thread in flight at a time, added in slot order
    double acc[2] = {0.0, 0.0};
    const int step = blockDim.x;
    for (int s0 = threadIdx.x; s0 < P.nslots; s0 += 4 * step) {
      double v[4][2];
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        const int s = s0 + k * step;
        v[k][0] = s < P.nslots ? P.part[2 * s] : 0.0;
        v[k][1] = s < P.nslots ? P.part[2 * s + 1] : 0.0;
      }
#pragma unroll
      for (int k = 0; k < 4; ++k)
        if (s0 + k * step < P.nslots) {
          acc[0] += v[k][0];
          acc[1] += v[k][1];
        }
    }
    nn_block_reduce<2, 2>(acc, red);
    if (threadIdx.x == 0) {
      scale_s[0] = P.sumA / acc[0];
      scale_s[1] = P.sumB / acc[1];
    }
    __syncthreads();
  }
  double m[3] = {0.0, 0.0, 0.0};  // surrogate residual, surrogate error, exact residual
  if (in) {
    const T pA = T(scale_s[0]) * hA, pB = T(scale_s[1]) * hB;
    const T cS = T(P.V * P.phiSbar / P.scal[kQS]);
    const T pS = cS * exp(-(wS - T(P.scal[kGaugeS])));
    T Sv = pA * T(P.invDA) + pB * T(P.invDB) + pS * T(P.invDS) - st;
    if (P.use_corr) Sv -= cr;
    if (P.mode == 0) {
      P.phi[i] = pA;
      P.phi[n + i] = pB;
      P.phi[2 * n + i] = pS;
      m[0] = fabs(double(pA) + double(pB) + double(pS) - 1.0);
    } else {
      P.corr[i] = (pA - eA) * T(P.invDA) + (pB - eB) * T(P.invDB);
      m[1] = fmax(fabs(double(pA) - double(eA)), fabs(double(pB) - double(eB)));
      m[2] = fabs(double(eA) + double(eB) + double(eS) - 1.0);
    }
    P.S[i] = Sv;
  }
  nn_block_reduce<3, 0>(m, red);
  if (threadIdx.x == 0) {
    if (P.mode == 0) {
      atomic_max_nonneg(P.scal + kNnResid, m[0]);
    } else {
      atomic_max_nonneg(P.scal + kNnErrLast, m[1]);
      atomic_max_nonneg(P.scal + kNnErr, m[1]);
      if (!P.use_corr) atomic_max_nonneg(P.scal + kNnErrUse, m[1]);  // surrogate steps came before
      atomic_max_nonneg(P.scal + kResidEx, m[2]);
    }
  }
}

// k_nn_norm fused with the row-forward FFT of the force source (the first
// pass of the force reconstruction, as k_force_row_fwd): each workgroup takes
// nf rows of the grid, normalises its sites as k_nn_norm does (the scale from
// the output kernel's partials, added in the same fixed order in every
// workgroup), keeps S in registers and transforms it along x into the
// force spectrum.
template <typename T, int L, int R>
__global__ void __launch_bounds__(512) k_norm_force_row(ForceArgs<T> F, NormArgs<T> P) {
  constexpr int TL = L / R;
  using V = LdsView<T, L, R, true, 1>;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  __shared__ double red[16 * 3];
  __shared__ double scale_s[2];
  const int f = threadIdx.x / TL, j = threadIdx.x % TL;
  V lds{reinterpret_cast<T2<T>*>(smem_raw), f};
  const int y = blockIdx.x * F.nf + f;
  const bool in = y < F.ny;
  const long n = P.n;
  Twiddles<T, L, R> twf;
  load_fwd_twiddles(twf, j, F.tw_x);
  T hA[R], hB[R], wS[R], st[R], cr[R], eA[R], eB[R], eS[R];
#pragma unroll
  for (int m = 0; m < R; ++m) {
    hA[m] = hB[m] = wS[m] = st[m] = cr[m] = eA[m] = eB[m] = eS[m] = T(0);
    if (in) {
      const long i = long(y) * F.nx + j + TL * m;
      hA[m] = P.src[i];
      hB[m] = P.src[n + i];
      wS[m] = P.wS[i];
      st[m] = P.stilde[i];
      if (P.use_corr) cr[m] = P.corr[i];
      if (P.mode != 0) {
        eA[m] = P.phi[i];
        eB[m] = P.phi[n + i];
        eS[m] = P.phi[2 * n + i];
      }
    }
  }
  {
    double acc[2] = {0.0, 0.0};
    const int step = blockDim.x;
    for (int s0 = threadIdx.x; s0 < P.nslots; s0 += 4 * step) {
      double v[4][2];
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        const int s = s0 + k * step;
        v[k][0] = s < P.nslots ? P.part[2 * s] : 0.0;
        v[k][1] = s < P.nslots ? P.part[2 * s + 1] : 0.0;
      }
#pragma unroll
      for (int k = 0; k < 4; ++k)
        if (s0 + k * step < P.nslots) {
          acc[0] += v[k][0];
          acc[1] += v[k][1];
        }
    }
    nn_block_reduce<2, 2>(acc, red);
    if (threadIdx.x == 0) {
      scale_s[0] = P.sumA / acc[0];
      scale_s[1] = P.sumB / acc[1];
    }
    __syncthreads();
  }
  const T cS = T(P.V * P.phiSbar / P.scal[kQS]);
  const T gS = T(P.scal[kGaugeS]);
  double mx[3] = {0.0, 0.0, 0.0};  // surrogate residual, surrogate error, exact residual
  T re[R], im[R];
#pragma unroll
  for (int m = 0; m < R; ++m) {
    const T pA = T(scale_s[0]) * hA[m], pB = T(scale_s[1]) * hB[m];
    const T pS = cS * exp(-(wS[m] - gS));
    T Sv = pA * T(P.invDA) + pB * T(P.invDB) + pS * T(P.invDS) - st[m];
    if (P.use_corr) Sv -= cr[m];
    re[m] = in ? Sv : T(0);
    im[m] = T(0);
    if (in) {
      const long i = long(y) * F.nx + j + TL * m;
      if (P.mode == 0) {
        P.phi[i] = pA;
        P.phi[n + i] = pB;
        P.phi[2 * n + i] = pS;
        mx[0] = fmax(mx[0], fabs(double(pA) + double(pB) + double(pS) - 1.0));
      } else {
        P.corr[i] = (pA - eA[m]) * T(P.invDA) + (pB - eB[m]) * T(P.invDB);
        mx[1] = fmax(mx[1], fmax(fabs(double(pA) - double(eA[m])), fabs(double(pB) - double(eB[m]))));
        mx[2] = fmax(mx[2], fabs(double(eA[m]) + double(eB[m]) + double(eS[m]) - 1.0));
      }
      P.S[i] = Sv;
    }
  }
  nn_block_reduce<3, 0>(mx, red);
  if (threadIdx.x == 0) {
    if (P.mode == 0) {
      atomic_max_nonneg(P.scal + kNnResid, mx[0]);
    } else {
      atomic_max_nonneg(P.scal + kNnErrLast, mx[1]);
      atomic_max_nonneg(P.scal + kNnErr, mx[1]);
      if (!P.use_corr) atomic_max_nonneg(P.scal + kNnErrUse, mx[1]);  // surrogate steps came before
      atomic_max_nonneg(P.scal + kResidEx, mx[2]);
    }
  }
  fft_forward(re, im, j, lds, twf);
  if (in) {
#pragma unroll
    for (int m = 0; m < R; ++m) {
      T2<T> o;
      o.x = re[m];
      o.y = im[m];
      F.spec[long(y) * F.nx + j + TL * m] = o;
    }
  }
}

// Clears scal slots (bit i of mask: slot kNnResid + i).  One thread.
__global__ void k_nn_reset(double* scal, int mask) {
  if (threadIdx.x == 0)
    for (int i = 0; i < 5; ++i)
      if (mask & (1 << i)) scal[kNnResid + i] = 0.0;
}

}  // namespace nn
}  // namespace epdlb
