// Vector kernels of the Phi -> omega inversion (App. C, comments 2 and 3):
// nonlinear Fletcher-Reeves conjugate gradients on the functional
//   G(omega) = (V phibar_P / N) ln Q_P + V phibar_S ln Q_S + dA sum_I sum_r omega_I Phi~_I,
// whose gradient is dA (Phi~ - Phi[omega]).  The descent direction is
// s = Phi[omega] - Phi~; directions d = s + beta d with beta the ratio of
// successive |s|^2; each line search takes the secant root of d . s from a
// trial point.  The density evaluations are the ordinary stages; these
// kernels do the vector updates and the dot products, all over the three
// planes of a field set (m = 3 nx ny elements).  Dot products accumulate in
// FP64: block partials in fixed slots, summed in slot order by k_cg_finish,
// so the sums do not depend on scheduling.  Optional diagonal preconditioning
// builds the directions from z = s / m, m = (N Phi_A, N Phi_B, Phi_S) the
// local response at the current iterate, with the factor (s.z)_new / (s.z)_old.
#pragma once
#include <hip/hip_runtime.h>

#include "kernels.hpp"

namespace epdlb {
namespace cg {

constexpr int kBlocks = 1024;   // fixed grid of the vector kernels (grid-stride)
constexpr int kThreads = 256;

// s = phi - target and, with z, z = s / m (planes A, B: m = N phi; S: m = phi);
// part[block] = sum s^2, part[kBlocks + block] = sum s.z (s^2 without z).
template <typename T>
__global__ void __launch_bounds__(kThreads) k_cg_resid(const T* __restrict__ phi, const T* __restrict__ target,
                                                       T* __restrict__ s, T* __restrict__ z, long m, long n,
                                                       T Nc, double* __restrict__ part) {
  __shared__ double red[16 * 2];
  double acc[2] = {0.0, 0.0};
  for (long i = long(blockIdx.x) * blockDim.x + threadIdx.x; i < m; i += long(gridDim.x) * blockDim.x) {
    const T ph = phi[i];
    const T v = ph - target[i];
    s[i] = v;
    acc[0] += double(v) * double(v);
    if (z) {
      const T mv = (i < 2 * n ? Nc : T(1)) * ph;
      const T zv = mv > T(0) ? v / mv : v;  // a density rounded to zero keeps s
      z[i] = zv;
      acc[1] += double(v) * double(zv);
    }
  }
  if (!z) acc[1] = acc[0];
  block_sum<2>(acc, red);
  if (threadIdx.x == 0) {
    part[blockIdx.x] = acc[0];
    part[kBlocks + blockIdx.x] = acc[1];
  }
}

// New direction and trial point: d = z (first) or z + beta d (z = s without
// preconditioning); xt = x + alpha_t d; part[block] = sum d . s.
template <typename T>
__global__ void __launch_bounds__(kThreads) k_cg_trial(const T* __restrict__ s, const T* __restrict__ z,
                                                       T* __restrict__ d, const T* __restrict__ x,
                                                       T* __restrict__ xt, T beta, int first, T alpha_t, long m,
                                                       double* __restrict__ part) {
  __shared__ double red[16];
  double acc[1] = {0.0};
  for (long i = long(blockIdx.x) * blockDim.x + threadIdx.x; i < m; i += long(gridDim.x) * blockDim.x) {
    const T sv = s[i];
    const T zv = z[i];
    const T dv = first ? zv : zv + beta * d[i];
    d[i] = dv;
    xt[i] = x[i] + alpha_t * dv;
    acc[0] += double(dv) * double(sv);
  }
  block_sum<1>(acc, red);
  if (threadIdx.x == 0) part[blockIdx.x] = acc[0];
}

// part[block] = sum d . (phi - target): the directional derivative at the trial point.
template <typename T>
__global__ void __launch_bounds__(kThreads) k_cg_dirdot(const T* __restrict__ d, const T* __restrict__ phi,
                                                        const T* __restrict__ target, long m,
                                                        double* __restrict__ part) {
  __shared__ double red[16];
  double acc[1] = {0.0};
  for (long i = long(blockIdx.x) * blockDim.x + threadIdx.x; i < m; i += long(gridDim.x) * blockDim.x)
    acc[0] += double(d[i]) * double(phi[i] - target[i]);
  block_sum<1>(acc, red);
  if (threadIdx.x == 0) part[blockIdx.x] = acc[0];
}

// x += alpha d.
template <typename T>
__global__ void __launch_bounds__(kThreads) k_cg_axpy(T* __restrict__ x, const T* __restrict__ d, T alpha, long m) {
  for (long i = long(blockIdx.x) * blockDim.x + threadIdx.x; i < m; i += long(gridDim.x) * blockDim.x)
    x[i] += alpha * d[i];
}

// out[q] = sum over b of part[q * nblk + b], q < nq, in slot order per thread
// then a fixed block reduction.  One block.
__global__ void __launch_bounds__(kThreads) k_cg_finish(const double* __restrict__ part, int nblk, int nq,
                                                        double* __restrict__ out) {
  __shared__ double red[16 * 2];
  double acc[2] = {0.0, 0.0};
  for (int b = threadIdx.x; b < nblk; b += blockDim.x) {
    acc[0] += part[b];
    if (nq > 1) acc[1] += part[nblk + b];
  }
  block_sum<2>(acc, red);
  if (threadIdx.x == 0) {
    out[0] = acc[0];
    out[1] = nq > 1 ? acc[1] : 0.0;
  }
}

}  // namespace cg
}  // namespace epdlb
