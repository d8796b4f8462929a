// Three-dimensional lattice Boltzmann fluid: D3Q19, the scheme the paper
// names for three dimensions (end of Sec. II), with the collision and body
// force of the two-dimensional fluid (Sec. II, Eq. LB_prop and Eq. force_col
// at gamma_s = gamma_b = 0): pull streaming, BGK relaxation with time tau
// towards the second-order equilibrium, the second-order force term
//   (1 - 1/(2 tau)) w_i [3 (c_i - u).F + 9 (c_i.u)(c_i.F)],
// and u = (sum f_i c_i + F/2) / rho.
//
// Layout: 19 planes of nx*ny*nz values, [i][z][y][x], x contiguous, holding
// the deviations g_i = f_i - w_i from the rest state (FP32 keeps the small
// momentum of slow flows).  Force and velocity: 3 planes (x, y, z).
//
// The step moves 19 values in and 19 out per site plus the force: it is a
// streaming kernel bound by HBM.  Each value is read by exactly one site (the
// one its velocity points to), so the only reuse is the cache line that two
// neighbouring x-chunks share when a population moves along x.  One wave
// walks a whole row in chunks of 64 sites, so that shared line, and the
// periodic wrap in x, stay with one compute unit; the rows of a wave's
// sources are wave-uniform, so every load is a scalar base plus a lane offset.
#pragma once
#include <hip/hip_runtime.h>

namespace epdlb {
namespace lb3 {

constexpr int kQ = 19;
constexpr int kWave = 64;
constexpr int kRows = 4;  // rows (y) per block: one wave each
constexpr int kThreads = kWave * kRows;

// c_i: rest, +x, -x, +y, -y, +z, -z, then the face diagonals
// (1,1,0) (-1,-1,0) (1,-1,0) (-1,1,0) (1,0,1) (-1,0,-1) (1,0,-1) (-1,0,1)
// (0,1,1) (0,-1,-1) (0,1,-1) (0,-1,1); weights 1/3, 1/18 (axes), 1/36 (diagonals).
constexpr int kCx[kQ] = {0, 1, -1, 0, 0, 0, 0, 1, -1, 1, -1, 1, -1, 1, -1, 0, 0, 0, 0};
constexpr int kCy[kQ] = {0, 0, 0, 1, -1, 0, 0, 1, -1, -1, 1, 0, 0, 0, 0, 1, -1, 1, -1};
constexpr int kCz[kQ] = {0, 0, 0, 0, 0, 1, -1, 0, 0, 0, 0, 1, -1, -1, 1, 1, -1, -1, 1};

template <typename T> __device__ __forceinline__ T weight(int k) {
  return k == 0 ? T(1.0 / 3.0) : (k < 7 ? T(1.0 / 18.0) : T(1.0 / 36.0));
}

template <typename T> __device__ __forceinline__ T signed_term(int c, T v) { return c > 0 ? v : -v; }

// c_k . a with the zero components left out (k is a constant after unrolling).
template <typename T> __device__ __forceinline__ T cdot(int k, T ax, T ay, T az) {
  const int a = kCx[k], b = kCy[k], c = kCz[k];
  if (a != 0 && b != 0) return signed_term(a, ax) + signed_term(b, ay);
  if (a != 0 && c != 0) return signed_term(a, ax) + signed_term(c, az);
  if (b != 0 && c != 0) return signed_term(b, ay) + signed_term(c, az);
  if (a != 0) return signed_term(a, ax);
  if (b != 0) return signed_term(b, ay);
  if (c != 0) return signed_term(c, az);
  return T(0);
}

template <typename T> struct Lb3Args {
  const T* fin;  // 19 planes g* (post-collision of the previous step)
  T* fout;       // 19 planes
  const T* F;    // 3 planes
  T* rho;        // written when the kernel stores the moments
  T* u;          // 3 planes
  int nx, ny, nz;
  long n;        // nx ny nz
  T omega;       // 1/tau
  T fpre;        // 1 - 1/(2 tau)
};

// One step at every site.  Grid (ceil(ny / kRows), nz), block kThreads.
template <typename T, bool MOM>
__global__ void __launch_bounds__(kThreads) k_lb3(Lb3Args<T> P) {
  const int nx = P.nx, ny = P.ny, nz = P.nz;
  const int y = __builtin_amdgcn_readfirstlane(int(blockIdx.x) * kRows + int(threadIdx.x) / kWave);
  const int z = blockIdx.y;
  if (y >= ny) return;
  const int lane = threadIdx.x % kWave;
  // source rows: index 1 - c (c = +1 reads the previous row, -1 the next)
  const int yr[3] = {y == 0 ? ny - 1 : y - 1, y, y + 1 == ny ? 0 : y + 1};
  const int zr[3] = {z == 0 ? nz - 1 : z - 1, z, z + 1 == nz ? 0 : z + 1};
  const T* src[kQ];
#pragma unroll
  for (int k = 0; k < kQ; ++k)
    src[k] = P.fin + long(k) * P.n + (long(zr[1 - kCz[k]]) * ny + yr[1 - kCy[k]]) * nx;
  const long row = (long(z) * ny + y) * nx;
  for (int x = lane; x < nx; x += kWave) {
    const int xs[3] = {x == 0 ? nx - 1 : x - 1, x, x + 1 == nx ? 0 : x + 1};
    T g[kQ];
#pragma unroll
    for (int k = 0; k < kQ; ++k) g[k] = src[k][xs[1 - kCx[k]]];
    const long i = row + x;
    const T Fx = P.F[i], Fy = P.F[P.n + i], Fz = P.F[2 * P.n + i];
    // sum_i w_i = 1 and sum_i w_i c_i = 0: the deviations carry rho - 1 and the momentum
    T drho = T(0), jx = T(0), jy = T(0), jz = T(0);
#pragma unroll
    for (int k = 0; k < kQ; ++k) {
      drho += g[k];
      if (kCx[k] != 0) jx = kCx[k] > 0 ? jx + g[k] : jx - g[k];
      if (kCy[k] != 0) jy = kCy[k] > 0 ? jy + g[k] : jy - g[k];
      if (kCz[k] != 0) jz = kCz[k] > 0 ? jz + g[k] : jz - g[k];
    }
    const T rho = T(1) + drho;
    const T ir = T(1) / rho;
    const T ux = (jx + T(0.5) * Fx) * ir, uy = (jy + T(0.5) * Fy) * ir, uz = (jz + T(0.5) * Fz) * ir;
    const T usq = ux * ux + uy * uy + uz * uz;
    const T uF = ux * Fx + uy * Fy + uz * Fz;
#pragma unroll
    for (int k = 0; k < kQ; ++k) {
      const T w = weight<T>(k);
      const T cu = cdot(k, ux, uy, uz);
      const T cF = cdot(k, Fx, Fy, Fz);
      // f^eq - w = w (rho - 1) + w rho (3 c.u + 4.5 (c.u)^2 - 1.5 u^2)
      const T geq = w * drho + w * rho * (T(3) * cu + T(4.5) * cu * cu - T(1.5) * usq);
      const T s = w * (T(3) * (cF - uF) + T(9) * cu * cF);
      P.fout[long(k) * P.n + i] = g[k] - (g[k] - geq) * P.omega + P.fpre * s;
    }
    if (MOM) {
      P.rho[i] = rho;
      P.u[i] = ux;
      P.u[P.n + i] = uy;
      P.u[2 * P.n + i] = uz;
    }
  }
}

// g = f^eq(rho, u) - w from the moments in P.rho and P.u (grid as k_lb3).
template <typename T>
__global__ void __launch_bounds__(kThreads) k_lb3_equilibrium(Lb3Args<T> P) {
  const int y = __builtin_amdgcn_readfirstlane(int(blockIdx.x) * kRows + int(threadIdx.x) / kWave);
  const int z = blockIdx.y;
  if (y >= P.ny) return;
  const long row = (long(z) * P.ny + y) * P.nx;
  for (int x = threadIdx.x % kWave; x < P.nx; x += kWave) {
    const long i = row + x;
    const T rho = P.rho[i];
    const T ux = P.u[i], uy = P.u[P.n + i], uz = P.u[2 * P.n + i];
    const T usq = ux * ux + uy * uy + uz * uz;
#pragma unroll
    for (int k = 0; k < kQ; ++k) {
      const T w = weight<T>(k);
      const T cu = cdot(k, ux, uy, uz);
      P.fout[long(k) * P.n + i] = w * (rho - T(1)) + w * rho * (T(3) * cu + T(4.5) * cu * cu - T(1.5) * usq);
    }
  }
}

}  // namespace lb3
}  // namespace epdlb
