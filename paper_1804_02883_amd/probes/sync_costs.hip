// Costs of the global synchronisation choices on one GPU, measured for the
// design of the step (kernel boundaries between the passes of a step, graph
// replay of a step): host submission and GPU time per dependent kernel as
// stream launches and as graph nodes, and the cost of a device-wide barrier
// inside one cooperative kernel (an atomic arrival counter with a generation
// flag, and cooperative groups' grid.sync), each checked for stale reads.
// Prints one JSON line.  Build: hipcc -O3 --offload-arch=gfx950 (see
// paper_1804_02883_amd/build.py); run: paper_1804_02883_amd/probes/sync_costs.
#include <hip/hip_cooperative_groups.h>
#include <hip/hip_runtime.h>

#include <chrono>
#include <cstdio>

#define CK(x)                                                                              \
  do {                                                                                     \
    hipError_t e_ = (x);                                                                   \
    if (e_ != hipSuccess) {                                                                \
      std::fprintf(stderr, "HIP error %s at line %d\n", hipGetErrorString(e_), __LINE__); \
      return 1;                                                                            \
    }                                                                                      \
  } while (0)

__global__ void k_empty(int* p) {
  if (threadIdx.x == 0 && blockIdx.x == 0 && p[0] == 12345) p[1] = 0;
}

// Arrival counter + generation flag; every wait is bounded (err set on timeout).
__device__ inline void counter_barrier(unsigned* count, unsigned* gen, unsigned nb, int* err) {
  __syncthreads();
  if (threadIdx.x == 0) {
    const unsigned g = __hip_atomic_load(gen, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    const unsigned a = __hip_atomic_fetch_add(count, 1u, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT);
    if (a == nb - 1) {
      __hip_atomic_store(count, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      __hip_atomic_fetch_add(gen, 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
    } else {
      long spins = 0;
      while (__hip_atomic_load(gen, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT) == g) {
        if (++spins > 4000000) {
          atomicExch(err, 1);
          break;
        }
        __builtin_amdgcn_s_sleep(1);
      }
    }
  }
  __syncthreads();
}

// nphase phases: each block writes `per` floats of its own region, then after
// the barrier reads the last float another block wrote (stale reads counted).
__global__ void k_counter_phases(unsigned* count, unsigned* gen, int* err, int* bad, float* buf, int per,
                                 int nphase) {
  const unsigned nb = gridDim.x;
  for (int ph = 0; ph < nphase; ++ph) {
    float* mine = buf + size_t(blockIdx.x) * per;
    for (int i = threadIdx.x; i < per; i += blockDim.x) mine[i] = float(ph * 4096 + blockIdx.x);
    counter_barrier(count, gen, nb, err);
    const unsigned other = (blockIdx.x + 37) % nb;
    if (threadIdx.x == 0 && buf[size_t(other) * per + (per - 1)] != float(ph * 4096 + other)) atomicAdd(bad, 1);
    counter_barrier(count, gen, nb, err);
  }
}

__global__ void k_grid_sync_phases(int* bad, float* buf, int per, int nphase) {
  auto grid = cooperative_groups::this_grid();
  const unsigned nb = gridDim.x;
  for (int ph = 0; ph < nphase; ++ph) {
    float* mine = buf + size_t(blockIdx.x) * per;
    for (int i = threadIdx.x; i < per; i += blockDim.x) mine[i] = float(ph * 4096 + blockIdx.x);
    grid.sync();
    const unsigned other = (blockIdx.x + 37) % nb;
    if (threadIdx.x == 0 && buf[size_t(other) * per + (per - 1)] != float(ph * 4096 + other)) atomicAdd(bad, 1);
    grid.sync();
  }
}

int main() {
  int* dp;
  CK(hipMalloc(&dp, 64));
  CK(hipMemset(dp, 0, 64));
  hipStream_t s;
  CK(hipStreamCreateWithFlags(&s, hipStreamNonBlocking));
  hipEvent_t e0, e1;
  CK(hipEventCreate(&e0));
  CK(hipEventCreate(&e1));
  using clk = std::chrono::steady_clock;
  auto us = [](clk::duration d) { return std::chrono::duration<double, std::micro>(d).count(); };
  // dependent stream launches
  for (int w = 0; w < 100; ++w) hipLaunchKernelGGL(k_empty, dim3(256), dim3(256), 0, s, dp);
  CK(hipStreamSynchronize(s));
  const int M = 4000;
  auto t0 = clk::now();
  CK(hipEventRecord(e0, s));
  for (int i = 0; i < M; ++i) hipLaunchKernelGGL(k_empty, dim3(256), dim3(256), 0, s, dp);
  CK(hipEventRecord(e1, s));
  auto t1 = clk::now();
  CK(hipStreamSynchronize(s));
  float ms = 0.f;
  CK(hipEventElapsedTime(&ms, e0, e1));
  const double stream_host = us(t1 - t0) / M, stream_gpu = ms * 1e3 / M;
  // graph of G dependent nodes, replayed R times
  const int G = 100, R = 40;
  hipGraph_t g;
  hipGraphExec_t ge;
  CK(hipStreamBeginCapture(s, hipStreamCaptureModeRelaxed));
  for (int i = 0; i < G; ++i) hipLaunchKernelGGL(k_empty, dim3(256), dim3(256), 0, s, dp);
  CK(hipStreamEndCapture(s, &g));
  CK(hipGraphInstantiate(&ge, g, nullptr, nullptr, 0));
  CK(hipGraphLaunch(ge, s));
  CK(hipStreamSynchronize(s));
  t0 = clk::now();
  CK(hipEventRecord(e0, s));
  for (int r = 0; r < R; ++r) CK(hipGraphLaunch(ge, s));
  CK(hipEventRecord(e1, s));
  t1 = clk::now();
  CK(hipStreamSynchronize(s));
  CK(hipEventElapsedTime(&ms, e0, e1));
  const double graph_host = us(t1 - t0) / (G * R), graph_gpu = ms * 1e3 / (G * R);
  // device-wide barriers, one 256-thread block per compute unit
  int dev = 0;
  CK(hipGetDevice(&dev));
  hipDeviceProp_t prop;
  CK(hipGetDeviceProperties(&prop, dev));
  const int nb = prop.multiProcessorCount;
  unsigned* cnt;
  int *err, *bad;
  CK(hipMalloc(&cnt, 256));
  CK(hipMalloc(&err, 64));
  CK(hipMalloc(&bad, 64));
  const int per_max = 1 << 16;
  float* buf;
  CK(hipMalloc(&buf, size_t(nb) * per_max * sizeof(float)));
  std::printf("{\"device\": \"%s\", \"cus\": %d, \"stream_launch_host_us\": %.3f, \"stream_launch_gpu_us\": %.3f, "
              "\"graph_node_host_us\": %.3f, \"graph_node_gpu_us\": %.3f, \"barriers\": [",
              prop.gcnArchName, nb, stream_host, stream_gpu, graph_host, graph_gpu);
  bool first = true;
  for (int per : {64, 65536}) {
    for (int mode = 0; mode < 2; ++mode) {
      const int nph = 200;
      CK(hipMemset(cnt, 0, 256));
      CK(hipMemset(err, 0, 64));
      CK(hipMemset(bad, 0, 64));
      unsigned* gen = cnt + 16;
      void* args_c[] = {&cnt, &gen, &err, &bad, &buf, (void*)&per, (void*)&nph};
      void* args_g[] = {&bad, &buf, (void*)&per, (void*)&nph};
      CK(hipStreamSynchronize(s));
      CK(hipEventRecord(e0, s));
      if (mode == 0)
        CK(hipLaunchCooperativeKernel((void*)k_counter_phases, dim3(nb), dim3(256), args_c, 0, s));
      else
        CK(hipLaunchCooperativeKernel((void*)k_grid_sync_phases, dim3(nb), dim3(256), args_g, 0, s));
      CK(hipEventRecord(e1, s));
      CK(hipStreamSynchronize(s));
      CK(hipEventElapsedTime(&ms, e0, e1));
      int herr = 0, hbad = 0;
      CK(hipMemcpy(&herr, err, 4, hipMemcpyDeviceToHost));
      CK(hipMemcpy(&hbad, bad, 4, hipMemcpyDeviceToHost));
      std::printf("%s{\"kind\": \"%s\", \"floats_per_block\": %d, \"us_per_barrier\": %.2f, \"timeouts\": %d, "
                  "\"stale_reads\": %d}",
                  first ? "" : ", ", mode == 0 ? "counter" : "grid_sync", per, ms * 1e3 / (2 * nph), herr, hbad);
      first = false;
    }
  }
  std::printf("]}\n");
  return 0;
}
