// Ceilings of one 64 -> 64 channel 3x3 convolution layer of the surrogate on
// a 512 x 512 grid, launched as the layer kernel is (256 workgroups of 1,024
// threads, 4,096 waves, each wave two 32-site row tiles):
//   mfma        the layer's matrix work alone: per tile 9 taps x 4 k-steps x
//               2 output blocks of v_mfma_f32_32x32x16_bf16 on register
//               operands (72 per tile, 19.3 GFLOP per launch)
//   store       the layer's activation stores alone: per tile and lane four
//               16-byte stores in the channel-blocked layout (33.5 MB)
//   mfma_store  both, each tile's stores after its MFMAs, as the layer does
//   mfma_long   16 times the matrix work per wave (the sustained MFMA rate)
// Each is timed with HIP events over `reps` back-to-back launches after a
// warm-up; prints one JSON line.  Build: hipcc -O3 --offload-arch=gfx950 (see
// paper_1804_02883_amd/build.py); run: paper_1804_02883_amd/probes/conv_floor.
#include <hip/hip_runtime.h>

#include <cstdio>

#define CK(x)                                                                              \
  do {                                                                                     \
    hipError_t e_ = (x);                                                                   \
    if (e_ != hipSuccess) {                                                                \
      std::fprintf(stderr, "HIP error %s at line %d\n", hipGetErrorString(e_), __LINE__); \
      return 1;                                                                            \
    }                                                                                      \
  } while (0)

typedef __attribute__((__vector_size__(8 * sizeof(__bf16)))) __bf16 bf16x8;
typedef __attribute__((__vector_size__(16 * sizeof(float)))) float f32x16;
typedef __attribute__((__vector_size__(4 * sizeof(unsigned)))) unsigned u32x4;

constexpr int kThreads = 1024;
constexpr int kBlocks = 256;
constexpr int kWaves = kBlocks * kThreads / 64;  // 4,096
constexpr int kTiles = 512 * 512 / 32;           // 8,192 row tiles of 32 sites
constexpr int kTilesPerWave = kTiles / kWaves;   // 2
constexpr int kTileBytes = 32 * 64 * 2;          // 32 sites x 64 channels, BF16
constexpr int kMfmaPerTile = 9 * 4 * 2;

template <bool MFMA, bool STORE, int REPEAT>
__global__ void __launch_bounds__(kThreads) k_floor(unsigned char* __restrict__ out, float* __restrict__ sink) {
  const int lane = threadIdx.x & 63;
  const int wave = blockIdx.x * (kThreads / 64) + (threadIdx.x >> 6);
  float keep = 0.0f;
  for (int k = 0; k < kTilesPerWave; ++k) {
    const int tile = wave * kTilesPerWave + k;
    // operands that depend on the tile, so that no tile's products can be
    // shared with another's
    bf16x8 a, b;
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      a[j] = __bf16(float((lane * 8 + j + tile) & 15) * 0.0625f);
      b[j] = __bf16(float((lane + j * 3 + tile) & 7) * 0.125f);
    }
    f32x16 acc[2];
#pragma unroll
    for (int i = 0; i < 16; ++i) acc[0][i] = acc[1][i] = 0.0f;
    if constexpr (MFMA) {
      for (int rep = 0; rep < REPEAT; ++rep) {
#pragma unroll
        for (int t = 0; t < kMfmaPerTile / 2; ++t) {
          acc[0] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, acc[0], 0, 0, 0);
          acc[1] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(b, a, acc[1], 0, 0, 0);
        }
      }
    }
    if constexpr (STORE) {
      // lane l: site l % 32, channel chunks 4 (l / 32) .. 4 (l / 32) + 3
      unsigned char* base = out + long(tile) * kTileBytes + (lane & 31) * 16 + (lane >> 5) * 2048;
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        bf16x8 o;
#pragma unroll
        for (int j = 0; j < 8; ++j) o[j] = __bf16(acc[q >> 1][8 * (q & 1) + j] + float(tile));
        *reinterpret_cast<u32x4*>(base + q * 512) = __builtin_bit_cast(u32x4, o);
      }
    } else {
#pragma unroll
      for (int i = 0; i < 16; ++i) keep += acc[0][i] + acc[1][i];
    }
  }
  if constexpr (!STORE) sink[wave * 64 + lane] = keep;
}

template <bool MFMA, bool STORE, int REPEAT>
static int time_kernel(const char* name, unsigned char* out, float* sink, int reps, bool comma) {
  hipEvent_t e0, e1;
  CK(hipEventCreate(&e0));
  CK(hipEventCreate(&e1));
  for (int i = 0; i < 3; ++i) k_floor<MFMA, STORE, REPEAT><<<kBlocks, kThreads>>>(out, sink);
  CK(hipGetLastError());
  CK(hipDeviceSynchronize());
  CK(hipEventRecord(e0, 0));
  for (int i = 0; i < reps; ++i) k_floor<MFMA, STORE, REPEAT><<<kBlocks, kThreads>>>(out, sink);
  CK(hipEventRecord(e1, 0));
  CK(hipEventSynchronize(e1));
  float ms = 0.0f;
  CK(hipEventElapsedTime(&ms, e0, e1));
  const double us = 1e3 * double(ms) / reps;
  const double flop = MFMA ? double(REPEAT) * kTiles * kMfmaPerTile * 32.0 * 32.0 * 16.0 * 2.0 : 0.0;
  const double bytes = STORE ? double(kTiles) * kTileBytes : 0.0;
  std::printf("%s\"%s\": {\"us\": %.3f, \"tflops\": %.1f, \"store_gbs\": %.1f}", comma ? ", " : "", name, us,
              flop / us * 1e-6, bytes / us * 1e-3);
  CK(hipEventDestroy(e0));
  CK(hipEventDestroy(e1));
  return 0;
}

int main() {
  unsigned char* out = nullptr;
  float* sink = nullptr;
  CK(hipMalloc(&out, size_t(kTiles) * kTileBytes));
  CK(hipMalloc(&sink, size_t(kWaves) * 64 * sizeof(float)));
  const int reps = 50;
  std::printf("{\"grid\": \"512x512, 64 channels\", \"launches\": %d, ", reps);
  if (time_kernel<true, false, 1>("mfma", out, sink, reps, false)) return 1;
  if (time_kernel<false, true, 1>("store", out, sink, reps, true)) return 1;
  if (time_kernel<true, true, 1>("mfma_store", out, sink, reps, true)) return 1;
  if (time_kernel<true, false, 16>("mfma_long", out, sink, 10, true)) return 1;
  std::printf("}\n");
  CK(hipFree(out));
  CK(hipFree(sink));
  return 0;
}
