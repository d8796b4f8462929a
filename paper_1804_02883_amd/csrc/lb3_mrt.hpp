// The paper's multi-relaxation collision (Sec. II, Eq. force_col) for the
// three-dimensional D3Q19 fluid, with the trace split of three dimensions:
// in moment space, with A = Pi - rho/3 I the stress of the deviations,
//   u = (j + F/2)/rho,  N = A - rho u u,  t = tr(N)/3,
//   B = rho u u + gs (N - t I) + gb t I
//       + (1 + gs)/2 [u F + F u - (2/3)(u.F) I] + (1 + gb)/3 (u.F) I,
//   g*_i = H_i(rho, j + F, B) + gg (g_i - H_i(rho, j, A)),
// H_i(rho, j, Q) = w_i [(rho - 1) + 3 j.c_i + 4.5 Q:(c_i c_i - I/3)], the
// deviations that carry exactly (rho, j, Q); the rest population is the
// complement of the moving ones to rho - 1, its exact value.  Streaming,
// layout and launch shape are those of k_lb3.
#pragma once
#include "lb3.hpp"

namespace epdlb {
namespace lb3 {

template <typename T> struct Lb3MrtArgs {
  Lb3Args<T> b;
  T gs, gb, gg;  // shear, bulk and non-hydrodynamic factors
};

// Q:(c_k c_k - I/3) for a symmetric Q (k is a constant after unrolling).
template <typename T>
__device__ __forceinline__ T qdot(int k, T qxx, T qyy, T qzz, T qxy, T qxz, T qyz) {
  const T third = T(1.0 / 3.0);
  const int a = kCx[k], b = kCy[k], c = kCz[k];
  return qxx * (T(a * a) - third) + qyy * (T(b * b) - third) + qzz * (T(c * c) - third) +
         T(2 * a * b) * qxy + T(2 * a * c) * qxz + T(2 * b * c) * qyz;
}

template <typename T, bool MOM>
__global__ void __launch_bounds__(kThreads) k_lb3_mrt(Lb3MrtArgs<T> M) {
  const Lb3Args<T>& P = M.b;
  const int nx = P.nx, ny = P.ny, nz = P.nz;
  const int y = __builtin_amdgcn_readfirstlane(int(blockIdx.x) * kRows + int(threadIdx.x) / kWave);
  const int z = blockIdx.y;
  if (y >= ny) return;
  const int lane = threadIdx.x % kWave;
  const int yr[3] = {y == 0 ? ny - 1 : y - 1, y, y + 1 == ny ? 0 : y + 1};
  const int zr[3] = {z == 0 ? nz - 1 : z - 1, z, z + 1 == nz ? 0 : z + 1};
  const T* src[kQ];
#pragma unroll
  for (int k = 0; k < kQ; ++k)
    src[k] = P.fin + long(k) * P.n + (long(zr[1 - kCz[k]]) * ny + yr[1 - kCy[k]]) * nx;
  const long row = (long(z) * ny + y) * nx;
  const T third = T(1.0 / 3.0);
  for (int x = lane; x < nx; x += kWave) {
    const int xs[3] = {x == 0 ? nx - 1 : x - 1, x, x + 1 == nx ? 0 : x + 1};
    T g[kQ];
#pragma unroll
    for (int k = 0; k < kQ; ++k) g[k] = src[k][xs[1 - kCx[k]]];
    const long i = row + x;
    const T Fx = P.F[i], Fy = P.F[P.n + i], Fz = P.F[2 * P.n + i];
    // moments of the deviations: sum w = 1, sum w c = 0, sum w c c = I/3
    T drho = T(0), jx = T(0), jy = T(0), jz = T(0);
    T sxx = T(0), syy = T(0), szz = T(0), sxy = T(0), sxz = T(0), syz = T(0);
#pragma unroll
    for (int k = 0; k < kQ; ++k) {
      const T v = g[k];
      drho += v;
      if (kCx[k] != 0) { jx = kCx[k] > 0 ? jx + v : jx - v; sxx += v; }
      if (kCy[k] != 0) { jy = kCy[k] > 0 ? jy + v : jy - v; syy += v; }
      if (kCz[k] != 0) { jz = kCz[k] > 0 ? jz + v : jz - v; szz += v; }
      if (kCx[k] * kCy[k] != 0) sxy = kCx[k] * kCy[k] > 0 ? sxy + v : sxy - v;
      if (kCx[k] * kCz[k] != 0) sxz = kCx[k] * kCz[k] > 0 ? sxz + v : sxz - v;
      if (kCy[k] * kCz[k] != 0) syz = kCy[k] * kCz[k] > 0 ? syz + v : syz - v;
    }
    const T rho = T(1) + drho;
    const T ir = T(1) / rho;
    const T ux = (jx + T(0.5) * Fx) * ir, uy = (jy + T(0.5) * Fy) * ir, uz = (jz + T(0.5) * Fz) * ir;
    // A = Pi - rho/3 I (pre-collision); N its non-equilibrium part
    const T axx = sxx - third * drho, ayy = syy - third * drho, azz = szz - third * drho;
    const T nxx = axx - rho * ux * ux, nyy = ayy - rho * uy * uy, nzz = azz - rho * uz * uz;
    const T nxy = sxy - rho * ux * uy, nxz = sxz - rho * ux * uz, nyz = syz - rho * uy * uz;
    const T t = third * (nxx + nyy + nzz);
    const T uF = ux * Fx + uy * Fy + uz * Fz;
    const T cs_ = T(0.5) * (T(1) + M.gs), cb_ = third * (T(1) + M.gb);
    const T dtr = M.gb * t + cb_ * uF - cs_ * T(2.0 / 3.0) * uF;  // isotropic part of B - rho u u - gs N
    const T bxx = rho * ux * ux + M.gs * (nxx - t) + dtr + cs_ * T(2) * ux * Fx;
    const T byy = rho * uy * uy + M.gs * (nyy - t) + dtr + cs_ * T(2) * uy * Fy;
    const T bzz = rho * uz * uz + M.gs * (nzz - t) + dtr + cs_ * T(2) * uz * Fz;
    const T bxy = rho * ux * uy + M.gs * nxy + cs_ * (ux * Fy + uy * Fx);
    const T bxz = rho * ux * uz + M.gs * nxz + cs_ * (ux * Fz + uz * Fx);
    const T byz = rho * uy * uz + M.gs * nyz + cs_ * (uy * Fz + uz * Fy);
    const T jxs = jx + Fx, jys = jy + Fy, jzs = jz + Fz;
    // each moving population is stored as soon as it is formed; only their sum stays
    T moving = T(0);
#pragma unroll
    for (int k = 1; k < kQ; ++k) {
      const T w = weight<T>(k);
      const T hpost = w * (drho + T(3) * cdot(k, jxs, jys, jzs) + T(4.5) * qdot(k, bxx, byy, bzz, bxy, bxz, byz));
      const T hpre = w * (drho + T(3) * cdot(k, jx, jy, jz) + T(4.5) * qdot(k, axx, ayy, azz, sxy, sxz, syz));
      const T o = hpost + M.gg * (g[k] - hpre);
      P.fout[long(k) * P.n + i] = o;
      moving += o;
    }
    P.fout[i] = drho - moving;
    if (MOM) {
      P.rho[i] = rho;
      P.u[i] = ux;
      P.u[P.n + i] = uy;
      P.u[2 * P.n + i] = uz;
    }
  }
}

}  // namespace lb3
}  // namespace epdlb
