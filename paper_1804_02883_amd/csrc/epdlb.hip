// Host runtime and C ABI of libepdlb.so (see include/epdlb.h).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "epdlb.h"
#include "kernels.hpp"

using namespace epdlb;

namespace {

thread_local std::string g_err;

int fail(int code, const std::string& msg) {
  g_err = msg;
  return code;
}

#define HIPCHK(expr)                                                                       \
  do {                                                                                     \
    hipError_t e_ = (expr);                                                                \
    if (e_ != hipSuccess)                                                                  \
      return fail(EPDLB_EHIP, std::string(#expr) + ": " + hipGetErrorString(e_));         \
  } while (0)

#define CHK(expr)          \
  do {                     \
    int r_ = (expr);       \
    if (r_ != EPDLB_OK) return r_; \
  } while (0)

bool is_pow2(int v) { return v > 0 && (v & (v - 1)) == 0; }

// ---------------------------------------------------------------------------
// SplitMix64 (Steele, Lea, Flood 2014) in counter mode + Box-Muller.
// ---------------------------------------------------------------------------
uint64_t splitmix_draw(uint64_t seed, uint64_t k) {
  uint64_t z = seed + (k + 1) * 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}
double unit_open0(uint64_t bits) { return (double((bits >> 11)) + 1.0) * 0x1.0p-53; }

// ---------------------------------------------------------------------------
// Device arena layout (all offsets 256-byte aligned).
// ---------------------------------------------------------------------------
struct Layout {
  size_t omega[2], phi, stilde, S, q[2], tmp, spec, F, fstar[2], rho, u;
  size_t mult_x, mult_y, tw_x, tw_y, wnA, wnB, scal, partials, counters;
  size_t total;
  size_t n_partials;
};

size_t align256(size_t v) { return (v + 255) & ~size_t(255); }

Layout make_layout(const epdlb_params& p) {
  const size_t es = p.precision == 0 ? 8 : 4;
  const size_t n = size_t(p.nx) * p.ny;
  const size_t plane = n * es;
  const int N = p.n_contour;
  Layout L{};
  size_t off = 0;
  auto take = [&](size_t bytes) {
    size_t o = off;
    off = align256(off + bytes);
    return o;
  };
  L.omega[0] = take(3 * plane);
  L.omega[1] = take(3 * plane);
  L.phi = take(3 * plane);
  L.stilde = take(plane);
  L.S = take(plane);
  L.q[0] = take(size_t(N) * plane);
  L.q[1] = take(size_t(N) * plane);
  L.tmp = take(2 * plane);
  L.spec = take(2 * plane);
  L.F = take(2 * plane);
  L.fstar[0] = take(9 * plane);
  L.fstar[1] = take(9 * plane);
  L.rho = take(plane);
  L.u = take(2 * plane);
  L.mult_x = take(size_t(p.nx) * es);
  L.mult_y = take(size_t(p.ny) * es);
  L.tw_x = take(size_t(p.nx) * 2 * es);
  L.tw_y = take(size_t(p.ny) * 2 * es);
  L.wnA = take(size_t(N + 1) * es);
  L.wnB = take(size_t(N + 1) * es);
  L.scal = take(kNumScal * sizeof(double));
  L.n_partials = 4 * (n / 64 + 4096);
  L.partials = take(L.n_partials * sizeof(double));
  L.counters = take(16 * sizeof(unsigned));
  L.total = off;
  return L;
}

}  // namespace

// ---------------------------------------------------------------------------
// Context
// ---------------------------------------------------------------------------
struct epdlb_ctx {
  epdlb_params p{};
  int device = 0;
  hipStream_t stream = nullptr;
  bool own_stream = false;
  unsigned char* base = nullptr;
  bool own_mem = false;
  Layout L{};
  int cur = 0;    // current omega buffer
  int fcur = 0;   // current f* buffer
  bool seeded = false;
  int64_t nstep = 0;
  std::vector<double> seg_a;   // A fraction per segment
  int nf_row = 1, nf_col = 1, nf_frow = 1, nf_fcol = 1;
  // per-launch event profiler (epdlb_profile_start / epdlb_profile_read)
  bool prof_on = false;
  int prof_used = 0;
  std::vector<hipEvent_t> prof_ev;  // 2 per launch
  std::vector<int> prof_kind;
  template <typename T> T* ptr(size_t off) const { return reinterpret_cast<T*>(base + off); }
};

namespace {

enum Kind { K_STATS, K_ADVECT, K_PROP_ROW, K_PROP_COL, K_DENSITY, K_FROW_FWD, K_FCOL, K_FROW_INV, K_LB,
            K_NUM };
const char* const kKindName[K_NUM] = {"field_stats", "advect_update", "prop_row", "prop_col", "density",
                                      "force_row_fwd", "force_col", "force_row_inv", "lb"};

// Event pair around one launch while the profiler has room; never blocks.
struct ProfScope {
  epdlb_ctx* c;
  int kind;
  bool rec;
  ProfScope(epdlb_ctx* ctx, int k) : c(ctx), kind(k) {
    rec = c->prof_on && size_t(2 * c->prof_used + 1) < c->prof_ev.size();
    if (rec) (void)hipEventRecord(c->prof_ev[2 * c->prof_used], c->stream);
  }
  ~ProfScope() {
    if (!rec) return;
    (void)hipEventRecord(c->prof_ev[2 * c->prof_used + 1], c->stream);
    c->prof_kind[c->prof_used] = kind;
    ++c->prof_used;
  }
};

int validate(const epdlb_params* p) {
  if (!p) return fail(EPDLB_EINVAL, "params is NULL");
  if (p->abi_version != EPDLB_ABI_VERSION) return fail(EPDLB_EINVAL, "abi_version mismatch");
  if (!is_pow2(p->nx) || p->nx < 32 || p->nx > 1024)
    return fail(EPDLB_EINVAL, "nx must be a power of two in [32, 1024]");
  if (!is_pow2(p->ny) || p->ny < 16 || p->ny > 1024)
    return fail(EPDLB_EINVAL, "ny must be a power of two in [16, 1024]");
  if (p->n_contour < 2 || p->n_contour > 256) return fail(EPDLB_EINVAL, "n_contour must be in [2, 256]");
  if (!(p->f_A > 0.0 && p->f_A < 1.0)) return fail(EPDLB_EINVAL, "f_A must be in (0, 1)");
  if (!(p->phi_P > 0.0 && p->phi_P < 1.0)) return fail(EPDLB_EINVAL, "phi_P must be in (0, 1)");
  if (!(p->D_S > 0 && p->D_A > 0 && p->D_B > 0)) return fail(EPDLB_EINVAL, "diffusion constants must be > 0");
  if (!(p->R_G > 0 && p->dx > 0 && p->dt > 0)) return fail(EPDLB_EINVAL, "R_G, dx, dt must be > 0");
  if (!(p->lb_tau > 0.5)) return fail(EPDLB_EINVAL, "lb_tau must be > 1/2");
  if (p->precision != 0 && p->precision != 1) return fail(EPDLB_EINVAL, "precision must be 0 or 1");
  if (p->g_units != 0 && p->g_units != 1) return fail(EPDLB_EINVAL, "g_units must be 0 or 1");
  if (!std::isfinite(p->g) || !std::isfinite(p->kT_over_v) || !std::isfinite(p->kappa_H) ||
      !std::isfinite(p->chi_AB) || !std::isfinite(p->chi_AS) || !std::isfinite(p->chi_BS))
    return fail(EPDLB_EINVAL, "non-finite parameter");
  return EPDLB_OK;
}

double g_lattice(const epdlb_params& p) { return p.g_units ? p.g : p.g * p.dt * p.dt / p.dx; }

template <int L> int split_n1() { return Split<L>::N1; }
int n1_of(int L) {
  switch (L) {
    case 16: return split_n1<16>();
    case 32: return split_n1<32>();
    case 64: return split_n1<64>();
    case 128: return split_n1<128>();
    case 256: return split_n1<256>();
    case 512: return split_n1<512>();
    case 1024: return split_n1<1024>();
  }
  return 0;
}

int clampi(int v, int lo, int hi) { return v < lo ? lo : (v > hi ? hi : v); }

// ---------------------------------------------------------------------------
// Launch helpers (one instantiation per transform length).
// ---------------------------------------------------------------------------
template <typename K>
hipError_t prep_lds(K kernel, size_t bytes) {
  if (bytes <= 65536) return hipSuccess;
  return hipFuncSetAttribute(reinterpret_cast<const void*>(kernel),
                             hipFuncAttributeMaxDynamicSharedMemorySize, int(bytes));
}

template <typename T, int L>
hipError_t launch_prop_row(const PropArgs<T>& a, hipStream_t s) {
  const size_t lds = 2 * size_t(RowMap<L>::size(a.nf)) * sizeof(T);
  hipError_t e = prep_lds(k_prop_row<T, L>, lds);
  if (e != hipSuccess) return e;
  const int tiles = (a.ny / 2 + a.nf - 1) / a.nf;
  hipLaunchKernelGGL((k_prop_row<T, L>), dim3(tiles, 2), dim3(a.nf * Split<L>::N1), lds, s, a);
  return hipGetLastError();
}
template <typename T, int L, int W>
hipError_t launch_prop_col_w(const PropArgs<T>& a, hipStream_t s) {
  constexpr int NF = W * 64 / Split<L>::N1;
  const size_t lds = 2 * size_t(ColMap<L, NF>::size()) * sizeof(T);
  hipError_t e = prep_lds(k_prop_col<T, L, NF>, lds);
  if (e != hipSuccess) return e;
  const int tiles = (a.nx / 2 + NF - 1) / NF;
  hipLaunchKernelGGL((k_prop_col<T, L, NF>), dim3(tiles, 2), dim3(NF * Split<L>::N1), lds, s, a);
  return hipGetLastError();
}
template <typename T, int L>
hipError_t launch_prop_col(const PropArgs<T>& a, hipStream_t s) {
  switch (a.nf) {
    case 1: return launch_prop_col_w<T, L, 1>(a, s);
    case 2: return launch_prop_col_w<T, L, 2>(a, s);
    case 4: return launch_prop_col_w<T, L, 4>(a, s);
  }
  return hipErrorInvalidValue;
}
template <typename T, int L>
hipError_t launch_force_row_fwd(const ForceArgs<T>& a, hipStream_t s) {
  const size_t lds = 2 * size_t(RowMap<L>::size(a.nf)) * sizeof(T);
  hipError_t e = prep_lds(k_force_row_fwd<T, L>, lds);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL((k_force_row_fwd<T, L>), dim3((a.ny + a.nf - 1) / a.nf),
                     dim3(a.nf * Split<L>::N1), lds, s, a);
  return hipGetLastError();
}
template <typename T, int L, int W>
hipError_t launch_force_col_w(const ForceArgs<T>& a, hipStream_t s) {
  constexpr int NF = W * 64 / Split<L>::N1;
  const size_t lds = 2 * size_t(ColMap<L, NF>::size()) * sizeof(T);
  hipError_t e = prep_lds(k_force_col<T, L, NF>, lds);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL((k_force_col<T, L, NF>), dim3((a.nx + NF - 1) / NF), dim3(NF * Split<L>::N1), lds,
                     s, a);
  return hipGetLastError();
}
template <typename T, int L>
hipError_t launch_force_col(const ForceArgs<T>& a, hipStream_t s) {
  switch (a.nf) {
    case 1: return launch_force_col_w<T, L, 1>(a, s);
    case 2: return launch_force_col_w<T, L, 2>(a, s);
    case 4: return launch_force_col_w<T, L, 4>(a, s);
  }
  return hipErrorInvalidValue;
}
template <typename T, int L>
hipError_t launch_force_row_inv(const ForceArgs<T>& a, hipStream_t s) {
  const size_t lds = 2 * size_t(RowMap<L>::size(a.nf)) * sizeof(T);
  hipError_t e = prep_lds(k_force_row_inv<T, L>, lds);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL((k_force_row_inv<T, L>), dim3((a.ny + a.nf - 1) / a.nf),
                     dim3(a.nf * Split<L>::N1), lds, s, a);
  return hipGetLastError();
}

#define EPDLB_SWITCH_L(L, FN, T, ...)                 \
  switch (L) {                                        \
    case 16: return FN<T, 16>(__VA_ARGS__);           \
    case 32: return FN<T, 32>(__VA_ARGS__);           \
    case 64: return FN<T, 64>(__VA_ARGS__);           \
    case 128: return FN<T, 128>(__VA_ARGS__);         \
    case 256: return FN<T, 256>(__VA_ARGS__);         \
    case 512: return FN<T, 512>(__VA_ARGS__);         \
    case 1024: return FN<T, 1024>(__VA_ARGS__);       \
  }                                                   \
  return hipErrorInvalidValue;

template <typename T> hipError_t prop_row(int L, const PropArgs<T>& a, hipStream_t s) {
  EPDLB_SWITCH_L(L, launch_prop_row, T, a, s)
}
template <typename T> hipError_t prop_col(int L, const PropArgs<T>& a, hipStream_t s) {
  EPDLB_SWITCH_L(L, launch_prop_col, T, a, s)
}
template <typename T> hipError_t force_row_fwd(int L, const ForceArgs<T>& a, hipStream_t s) {
  EPDLB_SWITCH_L(L, launch_force_row_fwd, T, a, s)
}
template <typename T> hipError_t force_col(int L, const ForceArgs<T>& a, hipStream_t s) {
  EPDLB_SWITCH_L(L, launch_force_col, T, a, s)
}
template <typename T> hipError_t force_row_inv(int L, const ForceArgs<T>& a, hipStream_t s) {
  EPDLB_SWITCH_L(L, launch_force_row_inv, T, a, s)
}

// ---------------------------------------------------------------------------
// Stages
// ---------------------------------------------------------------------------
template <typename T>
int stage_stats(epdlb_ctx* c) {
  const long n = long(c->p.nx) * c->p.ny;
  StatArgs<T> a;
  a.w = c->ptr<T>(c->L.omega[c->cur]);
  a.n = n;
  a.scal = c->ptr<double>(c->L.scal);
  a.partials = c->ptr<double>(c->L.partials);
  a.counter = c->ptr<unsigned>(c->L.counters) + 0;
  a.dA = c->p.dx * c->p.dx;
  const int blocks = int(std::min<long>(1024, (n + 255) / 256));
  ProfScope ps(c, K_STATS);
  hipLaunchKernelGGL((k_field_stats<T>), dim3(blocks), dim3(256), 0, c->stream, a);
  HIPCHK(hipGetLastError());
  return EPDLB_OK;
}

template <typename T>
int stage_advect_update(epdlb_ctx* c) {
  const epdlb_params& p = c->p;
  UpdArgs<T> a;
  const long n = long(p.nx) * p.ny;
  a.phi = c->ptr<T>(c->L.phi);
  a.w = c->ptr<T>(c->L.omega[c->cur]);
  a.u = c->ptr<T>(c->L.u);
  a.wout = c->ptr<T>(c->L.omega[1 - c->cur]);
  a.stilde = c->ptr<T>(c->L.stilde);
  a.scal = c->ptr<double>(c->L.scal);
  a.partials = c->ptr<double>(c->L.partials);
  a.counter = c->ptr<unsigned>(c->L.counters) + 0;
  a.nx = p.nx;
  a.ny = p.ny;
  a.n = n;
  const double chi[3][3] = {{0, p.chi_AB, p.chi_AS}, {p.chi_AB, 0, p.chi_BS}, {p.chi_AS, p.chi_BS, 0}};
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) a.chi[i][j] = T(chi[i][j]);
  a.kappa = T(p.kappa_H);
  const double D[3] = {p.D_A, p.D_B, p.D_S};
  for (int i = 0; i < 3; ++i) {
    a.coef[i] = T(D[i] * p.dt / (p.dx * p.dx));
    a.invD[i] = T(1.0 / D[i]);
  }
  a.advect = p.couple_lb ? 1 : 0;
  a.dA = p.dx * p.dx;
  {
    ProfScope ps(c, K_ADVECT);
    hipLaunchKernelGGL((k_advect_update<T>), dim3(p.nx / kTX, p.ny / kTY), dim3(kTX * kTY), 0, c->stream, a);
  }
  HIPCHK(hipGetLastError());
  c->cur = 1 - c->cur;
  return EPDLB_OK;
}

template <typename T>
int stage_densities(epdlb_ctx* c, bool with_S) {
  const epdlb_params& p = c->p;
  const int N = p.n_contour;
  const long n = long(p.nx) * p.ny;
  PropArgs<T> a;
  a.wA = c->ptr<T>(c->L.omega[c->cur]);
  a.wB = a.wA + n;
  a.scal = c->ptr<double>(c->L.scal);
  a.q[0] = c->ptr<T>(c->L.q[0]);
  a.q[1] = c->ptr<T>(c->L.q[1]);
  a.tmp = c->ptr<T>(c->L.tmp);
  a.mult_x = c->ptr<T>(c->L.mult_x);
  a.mult_y = c->ptr<T>(c->L.mult_y);
  a.tw_x = c->ptr<T2<T>>(c->L.tw_x);
  a.tw_y = c->ptr<T2<T>>(c->L.tw_y);
  a.nx = p.nx;
  a.ny = p.ny;
  a.plane = n;
  a.nsteps = N;
  a.partials = c->ptr<double>(c->L.partials);
  a.counter = c->ptr<unsigned>(c->L.counters) + 1;
  a.qout = c->ptr<double>(c->L.scal) + kQPf;
  a.dA = p.dx * p.dx;
  for (int j = 0; j < N; ++j) {
    a.j = j;
    a.a[0] = T(c->seg_a[j]);
    a.a[1] = T(c->seg_a[N - 1 - j]);
    a.nf = c->nf_row;
    {
      ProfScope ps(c, K_PROP_ROW);
      HIPCHK(prop_row<T>(p.nx, a, c->stream));
    }
    a.nf = c->nf_col;
    {
      ProfScope ps(c, K_PROP_COL);
      HIPCHK(prop_col<T>(p.ny, a, c->stream));
    }
  }
  DensArgs<T> d;
  d.q[0] = a.q[0];
  d.q[1] = a.q[1];
  d.wS = a.wA + 2 * n;
  d.stilde = c->ptr<T>(c->L.stilde);
  d.phi = c->ptr<T>(c->L.phi);
  d.S = with_S ? c->ptr<T>(c->L.S) : nullptr;
  d.scal = a.scal;
  d.wnA = c->ptr<T>(c->L.wnA);
  d.wnB = c->ptr<T>(c->L.wnB);
  d.n = n;
  d.N = N;
  d.V = double(n) * p.dx * p.dx;
  d.phiP = p.phi_P;
  d.phiSbar = 1.0 - p.phi_P;
  d.invDA = 1.0 / p.D_A;
  d.invDB = 1.0 / p.D_B;
  d.invDS = 1.0 / p.D_S;
  {
    ProfScope ps(c, K_DENSITY);
    hipLaunchKernelGGL((k_density<T>), dim3((n + 255) / 256), dim3(256), 0, c->stream, d);
  }
  HIPCHK(hipGetLastError());
  return EPDLB_OK;
}

template <typename T>
int stage_force(epdlb_ctx* c) {
  const epdlb_params& p = c->p;
  ForceArgs<T> a;
  a.S = c->ptr<T>(c->L.S);
  a.spec = c->ptr<T2<T>>(c->L.spec);
  a.F = c->ptr<T>(c->L.F);
  a.tw_x = c->ptr<T2<T>>(c->L.tw_x);
  a.tw_y = c->ptr<T2<T>>(c->L.tw_y);
  a.nx = p.nx;
  a.ny = p.ny;
  a.n = long(p.nx) * p.ny;
  a.kx0 = 2.0 * M_PI / (p.nx * p.dx);
  a.ky0 = 2.0 * M_PI / (p.ny * p.dx);
  a.pref = p.kT_over_v / p.dt / (double(p.nx) * p.ny);
  a.conv = p.couple_lb ? p.dt * p.dt / p.dx : 0.0;
  a.gext = g_lattice(p);
  a.nf = c->nf_frow;
  {
    ProfScope ps(c, K_FROW_FWD);
    HIPCHK(force_row_fwd<T>(p.nx, a, c->stream));
  }
  a.nf = c->nf_fcol;
  {
    ProfScope ps(c, K_FCOL);
    HIPCHK(force_col<T>(p.ny, a, c->stream));
  }
  a.nf = c->nf_frow;
  {
    ProfScope ps(c, K_FROW_INV);
    HIPCHK(force_row_inv<T>(p.nx, a, c->stream));
  }
  return EPDLB_OK;
}

template <typename T>
int stage_lb(epdlb_ctx* c) {
  const epdlb_params& p = c->p;
  LbArgs<T> a;
  const long n = long(p.nx) * p.ny;
  a.fin = c->ptr<T>(c->L.fstar[c->fcur]);
  a.fout = c->ptr<T>(c->L.fstar[1 - c->fcur]);
  a.F = c->ptr<T>(c->L.F);
  a.rho = c->ptr<T>(c->L.rho);
  a.u = c->ptr<T>(c->L.u);
  a.nx = p.nx;
  a.ny = p.ny;
  a.n = n;
  a.omega = T(1.0 / p.lb_tau);
  a.fpre = T(1.0 - 0.5 / p.lb_tau);
  {
    ProfScope ps(c, K_LB);
    hipLaunchKernelGGL((k_lb<T>), dim3((n + 255) / 256), dim3(256), 0, c->stream, a);
  }
  HIPCHK(hipGetLastError());
  c->fcur = 1 - c->fcur;
  return EPDLB_OK;
}

template <typename T>
int run_stage_t(epdlb_ctx* c, int stage) {
  switch (stage) {
    case EPDLB_STAGE_ADVECT_UPDATE: return stage_advect_update<T>(c);
    case EPDLB_STAGE_DENSITIES: return stage_densities<T>(c, true);
    case EPDLB_STAGE_FORCE: return stage_force<T>(c);
    case EPDLB_STAGE_LB: return stage_lb<T>(c);
  }
  return fail(EPDLB_EINVAL, "unknown stage");
}

int run_stage(epdlb_ctx* c, int stage) {
  return c->p.precision == 0 ? run_stage_t<double>(c, stage) : run_stage_t<float>(c, stage);
}

// ---------------------------------------------------------------------------
// Host <-> device copies with conversion
// ---------------------------------------------------------------------------
template <typename T>
int upload_t(epdlb_ctx* c, size_t off, const double* src, size_t count) {
  std::vector<T> tmp(count);
  for (size_t i = 0; i < count; ++i) tmp[i] = T(src[i]);
  HIPCHK(hipMemcpyAsync(c->base + off, tmp.data(), count * sizeof(T), hipMemcpyHostToDevice, c->stream));
  HIPCHK(hipStreamSynchronize(c->stream));
  return EPDLB_OK;
}
int upload(epdlb_ctx* c, size_t off, const double* src, size_t count) {
  return c->p.precision == 0 ? upload_t<double>(c, off, src, count) : upload_t<float>(c, off, src, count);
}
template <typename T>
int download_t(epdlb_ctx* c, size_t off, double* dst, size_t count) {
  std::vector<T> tmp(count);
  HIPCHK(hipMemcpyAsync(tmp.data(), c->base + off, count * sizeof(T), hipMemcpyDeviceToHost, c->stream));
  HIPCHK(hipStreamSynchronize(c->stream));
  for (size_t i = 0; i < count; ++i) dst[i] = double(tmp[i]);
  return EPDLB_OK;
}
int download(epdlb_ctx* c, size_t off, double* dst, size_t count) {
  return c->p.precision == 0 ? download_t<double>(c, off, dst, count) : download_t<float>(c, off, dst, count);
}
size_t elem(const epdlb_ctx* c) { return c->p.precision == 0 ? 8 : 4; }

// Constant tables: twiddles, heat-kernel multipliers, node weights.
int upload_tables(epdlb_ctx* c) {
  const epdlb_params& p = c->p;
  const int N = p.n_contour;
  const double ds = 1.0 / N;
  auto mult = [&](int L, std::vector<double>& out) {
    out.resize(L);
    for (int k = 0; k < L; ++k) {
      const int m = k < L / 2 ? k : k - L;
      const double kk = 2.0 * M_PI * m / (L * p.dx);
      out[k] = std::exp(-p.R_G * p.R_G * kk * kk * ds) / L;
    }
  };
  auto tw = [&](int L, std::vector<double>& out) {
    out.resize(2 * L);
    for (int e = 0; e < L; ++e) {
      const double ang = 2.0 * M_PI * double(e) / double(L);
      out[2 * e] = std::cos(ang);
      out[2 * e + 1] = -std::sin(ang);
    }
  };
  std::vector<double> v;
  mult(p.nx, v);
  CHK(upload(c, c->L.mult_x, v.data(), v.size()));
  mult(p.ny, v);
  CHK(upload(c, c->L.mult_y, v.data(), v.size()));
  tw(p.nx, v);
  CHK(upload(c, c->L.tw_x, v.data(), v.size()));
  tw(p.ny, v);
  CHK(upload(c, c->L.tw_y, v.data(), v.size()));
  // segment A fractions and node weights (trapezoid over each segment)
  c->seg_a.assign(N, 0.0);
  for (int j = 0; j < N; ++j) {
    double a = p.f_A * N - j;
    c->seg_a[j] = a < 0 ? 0.0 : (a > 1 ? 1.0 : a);
  }
  std::vector<double> wA(N + 1, 0.0), wB(N + 1, 0.0);
  for (int j = 0; j < N; ++j) {
    wA[j] += 0.5 * ds * c->seg_a[j];
    wA[j + 1] += 0.5 * ds * c->seg_a[j];
    wB[j] += 0.5 * ds * (1.0 - c->seg_a[j]);
    wB[j + 1] += 0.5 * ds * (1.0 - c->seg_a[j]);
  }
  CHK(upload(c, c->L.wnA, wA.data(), wA.size()));
  CHK(upload(c, c->L.wnB, wB.data(), wB.size()));
  HIPCHK(hipMemsetAsync(c->base + c->L.scal, 0, kNumScal * sizeof(double), c->stream));
  HIPCHK(hipMemsetAsync(c->base + c->L.counters, 0, 16 * sizeof(unsigned), c->stream));
  HIPCHK(hipStreamSynchronize(c->stream));
  return EPDLB_OK;
}

int compute_stats(epdlb_ctx* c) {
  // twice: the first pass fixes the means, the second evaluates Q_S with them
  for (int k = 0; k < 2; ++k) CHK(c->p.precision == 0 ? stage_stats<double>(c) : stage_stats<float>(c));
  return EPDLB_OK;
}

// LB at f^eq(rho = 1, u_init); u_init the analytic reverse-Poiseuille profile.
int init_lb(epdlb_ctx* c) {
  const epdlb_params& p = c->p;
  const size_t n = size_t(p.nx) * p.ny;
  std::vector<double> ux(p.ny, 0.0);
  if (p.init_flow) {
    const double F0 = g_lattice(p);
    const double nu = (p.lb_tau - 0.5) / 3.0;
    const double Ly = p.ny;
    for (int y = 0; y < p.ny; ++y) {
      const double Y = y + 0.5 - Ly / 2;
      ux[y] = -(F0 / (2 * nu)) * Y * (std::fabs(Y) - Ly / 2);
    }
  }
  static const int cx[9] = {0, 1, 0, -1, 0, 1, -1, -1, 1};
  static const double w[9] = {4.0 / 9, 1.0 / 9, 1.0 / 9, 1.0 / 9, 1.0 / 9,
                              1.0 / 36, 1.0 / 36, 1.0 / 36, 1.0 / 36};
  std::vector<double> f(9 * n), u(2 * n, 0.0), rho(n, 1.0);
  for (int y = 0; y < p.ny; ++y)
    for (int x = 0; x < p.nx; ++x) {
      const size_t i = size_t(y) * p.nx + x;
      const double vx = ux[y];
      u[i] = vx;
      for (int k = 0; k < 9; ++k) {
        const double cu = cx[k] * vx;
        f[k * n + i] = w[k] * (1.0 + 3.0 * cu + 4.5 * cu * cu - 1.5 * vx * vx);
      }
    }
  c->fcur = 0;
  CHK(upload(c, c->L.fstar[0], f.data(), f.size()));
  CHK(upload(c, c->L.u, u.data(), u.size()));
  CHK(upload(c, c->L.rho, rho.data(), rho.size()));
  return EPDLB_OK;
}

int check_finite(epdlb_ctx* c) {
  double s[kNumScal];
  HIPCHK(hipMemcpyAsync(s, c->base + c->L.scal, sizeof(s), hipMemcpyDeviceToHost, c->stream));
  HIPCHK(hipStreamSynchronize(c->stream));
  for (int i = 0; i < kNumScal; ++i)
    if (!std::isfinite(s[i])) return fail(EPDLB_ENONFINITE, "non-finite partition function or field mean");
  return EPDLB_OK;
}

}  // namespace

// ---------------------------------------------------------------------------
// C ABI
// ---------------------------------------------------------------------------
extern "C" {

int epdlb_params_default(epdlb_params* p) {
  if (!p) return fail(EPDLB_EINVAL, "params is NULL");
  std::memset(p, 0, sizeof(*p));
  p->abi_version = EPDLB_ABI_VERSION;
  p->nx = 32;
  p->ny = 32;
  p->n_contour = 16;
  p->f_A = 0.5;
  p->phi_P = 0.1;
  p->chi_AB = 1.5 / 16;
  p->chi_AS = 1.5 / 16;
  p->chi_BS = 0.0;
  p->kappa_H = 20.0 / 16;
  p->D_S = 1.0;
  p->D_A = 1.0 / 16;
  p->D_B = 1.0 / 16;
  p->R_G = 1.0;
  p->dx = 1.0 / 3.0;
  p->dt = 0.002;
  p->kT_over_v = 1.0;
  p->lb_tau = 1.0;
  p->g = 1e-5;
  p->g_units = 0;
  p->precision = 0;
  p->init_flow = 1;
  p->couple_lb = 1;
  return EPDLB_OK;
}

int epdlb_validate(const epdlb_params* p) { return validate(p); }

int epdlb_workspace_bytes(const epdlb_params* p, size_t* bytes) {
  CHK(validate(p));
  if (!bytes) return fail(EPDLB_EINVAL, "bytes is NULL");
  *bytes = make_layout(*p).total;
  return EPDLB_OK;
}

int epdlb_noise_fill(uint64_t seed, double sigma, int32_t nx, int32_t ny, double* out) {
  if (!out || nx <= 0 || ny <= 0) return fail(EPDLB_EINVAL, "bad noise arguments");
  const size_t count = size_t(3) * nx * ny;
  for (size_t e = 0; e < count; ++e) {
    const size_t pair = e / 2;
    const double u1 = unit_open0(splitmix_draw(seed, 2 * pair));
    const double u2 = unit_open0(splitmix_draw(seed, 2 * pair + 1));
    const double r = std::sqrt(-2.0 * std::log(u1));
    const double ang = 2.0 * M_PI * u2;
    out[e] = sigma * ((e & 1) ? r * std::sin(ang) : r * std::cos(ang));
  }
  return EPDLB_OK;
}

int epdlb_create(const epdlb_params* p, int device, void* stream, void* workspace,
                 size_t workspace_bytes, epdlb_ctx** out) {
  CHK(validate(p));
  if (!out) return fail(EPDLB_EINVAL, "out is NULL");
  *out = nullptr;
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || ndev <= device || device < 0)
    return fail(EPDLB_ENODEV, "no HIP device with that index");
  HIPCHK(hipSetDevice(device));
  hipDeviceProp_t prop;
  HIPCHK(hipGetDeviceProperties(&prop, device));
  if (std::strncmp(prop.gcnArchName, "gfx950", 6) != 0)
    return fail(EPDLB_ENODEV, std::string("library built for gfx950, device is ") + prop.gcnArchName);
  epdlb_ctx* c = new (std::nothrow) epdlb_ctx();
  if (!c) return fail(EPDLB_ENOMEM, "host allocation failed");
  c->p = *p;
  c->device = device;
  c->L = make_layout(*p);
  if (stream) {
    c->stream = reinterpret_cast<hipStream_t>(stream);
  } else {
    if (hipStreamCreateWithFlags(&c->stream, hipStreamNonBlocking) != hipSuccess) {
      delete c;
      return fail(EPDLB_EHIP, "hipStreamCreate failed");
    }
    c->own_stream = true;
  }
  if (workspace) {
    if (workspace_bytes < c->L.total || (reinterpret_cast<uintptr_t>(workspace) & 255)) {
      epdlb_destroy(c);
      return fail(EPDLB_ENOMEM, "workspace too small or not 256-byte aligned");
    }
    c->base = static_cast<unsigned char*>(workspace);
  } else {
    void* m = nullptr;
    if (hipMalloc(&m, c->L.total) != hipSuccess) {
      epdlb_destroy(c);
      return fail(EPDLB_ENOMEM, "hipMalloc of the state arena failed");
    }
    c->base = static_cast<unsigned char*>(m);
    c->own_mem = true;
  }
  // launch shapes.  Row passes: nf transforms of n1x lanes per block; column
  // passes: nf = wavefronts per block.  Prefer enough blocks to cover the CUs.
  const int n1x = n1_of(p->nx), n1y = n1_of(p->ny);
  auto pick_row = [&](int transforms, int chains) {
    int nf = 256 / n1x;
    while (nf * n1x > 64 && chains * ((transforms + nf - 1) / nf) < 512) nf /= 2;
    return clampi(nf, 1, transforms);
  };
  auto pick_col = [&](int transforms, int chains) {
    int w = 4;
    while (w > 1 && chains * ((transforms + w * 64 / n1y - 1) / (w * 64 / n1y)) < 512) w /= 2;
    return w;
  };
  c->nf_row = pick_row(p->ny / 2, 2);
  c->nf_col = pick_col(p->nx / 2, 2);
  c->nf_frow = pick_row(p->ny, 1);
  c->nf_fcol = pick_col(p->nx, 1);
  int r = upload_tables(c);
  if (r != EPDLB_OK) {
    epdlb_destroy(c);
    return r;
  }
  *out = c;
  return EPDLB_OK;
}

int epdlb_set_fields(epdlb_ctx* c, const double* omega) {
  if (!c || !omega) return fail(EPDLB_EINVAL, "NULL argument");
  HIPCHK(hipSetDevice(c->device));
  const size_t n = size_t(c->p.nx) * c->p.ny;
  c->cur = 0;
  CHK(upload(c, c->L.omega[0], omega, 3 * n));
  HIPCHK(hipMemsetAsync(c->base + c->L.scal, 0, kNumScal * sizeof(double), c->stream));
  CHK(compute_stats(c));
  CHK(c->p.precision == 0 ? stage_densities<double>(c, false) : stage_densities<float>(c, false));
  CHK(init_lb(c));
  HIPCHK(hipStreamSynchronize(c->stream));
  c->seeded = true;
  c->nstep = 0;
  return check_finite(c);
}

int epdlb_seed(epdlb_ctx* c, uint64_t seed, double sigma) {
  if (!c) return fail(EPDLB_EINVAL, "ctx is NULL");
  std::vector<double> w(size_t(3) * c->p.nx * c->p.ny);
  CHK(epdlb_noise_fill(seed, sigma, c->p.nx, c->p.ny, w.data()));
  return epdlb_set_fields(c, w.data());
}

int epdlb_set_state(epdlb_ctx* c, const double* omega, const double* phi, const double* fstar,
                    const double* u) {
  if (!c || !omega || !phi || !fstar || !u) return fail(EPDLB_EINVAL, "NULL argument");
  HIPCHK(hipSetDevice(c->device));
  const size_t n = size_t(c->p.nx) * c->p.ny;
  c->cur = 0;
  c->fcur = 0;
  CHK(upload(c, c->L.omega[0], omega, 3 * n));
  CHK(upload(c, c->L.phi, phi, 3 * n));
  CHK(upload(c, c->L.fstar[0], fstar, 9 * n));
  CHK(upload(c, c->L.u, u, 2 * n));
  HIPCHK(hipMemsetAsync(c->base + c->L.scal, 0, kNumScal * sizeof(double), c->stream));
  CHK(compute_stats(c));
  HIPCHK(hipStreamSynchronize(c->stream));
  c->seeded = true;
  c->nstep = 0;
  return EPDLB_OK;
}

int epdlb_step(epdlb_ctx* c, int64_t n) {
  if (!c) return fail(EPDLB_EINVAL, "ctx is NULL");
  if (!c->seeded) return fail(EPDLB_ESTATE, "step before seed/set_fields/set_state");
  if (n < 0) return fail(EPDLB_EINVAL, "negative step count");
  HIPCHK(hipSetDevice(c->device));
  for (int64_t s = 0; s < n; ++s) {
    for (int st = EPDLB_STAGE_ADVECT_UPDATE; st <= EPDLB_STAGE_LB; ++st) CHK(run_stage(c, st));
    ++c->nstep;
  }
  return EPDLB_OK;
}

int epdlb_run_stage(epdlb_ctx* c, int32_t stage) {
  if (!c) return fail(EPDLB_EINVAL, "ctx is NULL");
  if (!c->seeded) return fail(EPDLB_ESTATE, "stage before seed/set_fields/set_state");
  HIPCHK(hipSetDevice(c->device));
  return run_stage(c, stage);
}

int epdlb_sync(epdlb_ctx* c) {
  if (!c) return fail(EPDLB_EINVAL, "ctx is NULL");
  HIPCHK(hipStreamSynchronize(c->stream));
  return check_finite(c);
}

int epdlb_read_densities(epdlb_ctx* c, double* a, double* b, double* s) {
  if (!c || !a || !b || !s) return fail(EPDLB_EINVAL, "NULL argument");
  const size_t n = size_t(c->p.nx) * c->p.ny, pl = n * elem(c);
  CHK(download(c, c->L.phi, a, n));
  CHK(download(c, c->L.phi + pl, b, n));
  return download(c, c->L.phi + 2 * pl, s, n);
}

int epdlb_read_fields(epdlb_ctx* c, double* a, double* b, double* s) {
  if (!c || !a || !b || !s) return fail(EPDLB_EINVAL, "NULL argument");
  const size_t n = size_t(c->p.nx) * c->p.ny, pl = n * elem(c);
  const size_t o = c->L.omega[c->cur];
  CHK(download(c, o, a, n));
  CHK(download(c, o + pl, b, n));
  return download(c, o + 2 * pl, s, n);
}

int epdlb_read_velocity(epdlb_ctx* c, double* rho, double* ux, double* uy) {
  if (!c || !rho || !ux || !uy) return fail(EPDLB_EINVAL, "NULL argument");
  const size_t n = size_t(c->p.nx) * c->p.ny, pl = n * elem(c);
  CHK(download(c, c->L.rho, rho, n));
  CHK(download(c, c->L.u, ux, n));
  return download(c, c->L.u + pl, uy, n);
}

int epdlb_read_populations(epdlb_ctx* c, double* f) {
  if (!c || !f) return fail(EPDLB_EINVAL, "NULL argument");
  return download(c, c->L.fstar[c->fcur], f, 9 * size_t(c->p.nx) * c->p.ny);
}

static int aux_loc(epdlb_ctx* c, int which, size_t* off, size_t* planes) {
  switch (which) {
    case EPDLB_AUX_STILDE: *off = c->L.stilde; *planes = 1; return EPDLB_OK;
    case EPDLB_AUX_S: *off = c->L.S; *planes = 1; return EPDLB_OK;
    case EPDLB_AUX_FORCE: *off = c->L.F; *planes = 2; return EPDLB_OK;
  }
  return fail(EPDLB_EINVAL, "unknown aux plane");
}

int epdlb_read_aux(epdlb_ctx* c, int32_t which, double* out) {
  if (!c || !out) return fail(EPDLB_EINVAL, "NULL argument");
  size_t off, planes;
  CHK(aux_loc(c, which, &off, &planes));
  return download(c, off, out, planes * size_t(c->p.nx) * c->p.ny);
}

int epdlb_write_aux(epdlb_ctx* c, int32_t which, const double* in) {
  if (!c || !in) return fail(EPDLB_EINVAL, "NULL argument");
  size_t off, planes;
  CHK(aux_loc(c, which, &off, &planes));
  return upload(c, off, in, planes * size_t(c->p.nx) * c->p.ny);
}

int epdlb_read_diag(epdlb_ctx* c, epdlb_diag* d) {
  if (!c || !d) return fail(EPDLB_EINVAL, "NULL argument");
  double s[kNumScal];
  HIPCHK(hipMemcpyAsync(s, c->base + c->L.scal, sizeof(s), hipMemcpyDeviceToHost, c->stream));
  HIPCHK(hipStreamSynchronize(c->stream));
  d->step = c->nstep;
  d->Q_P = s[kQPf];
  d->Q_P_bwd = s[kQPb];
  d->Q_S = s[kQS];
  d->gauge_S = s[kGaugeS];
  d->mean_omega[0] = s[kMeanA];
  d->mean_omega[1] = s[kMeanB];
  d->mean_omega[2] = s[kMeanS];
  return EPDLB_OK;
}

int epdlb_profile_start(epdlb_ctx* c, int32_t max_launches) {
  if (!c || max_launches < 1) return fail(EPDLB_EINVAL, "bad profile arguments");
  HIPCHK(hipSetDevice(c->device));
  const size_t need = 2 * size_t(max_launches);
  while (c->prof_ev.size() < need) {
    hipEvent_t e;
    HIPCHK(hipEventCreate(&e));
    c->prof_ev.push_back(e);
  }
  c->prof_kind.assign(max_launches, 0);
  c->prof_used = 0;
  c->prof_on = true;
  return EPDLB_OK;
}

int epdlb_profile_read(epdlb_ctx* c, epdlb_kernel_stat* out, int32_t cap, int32_t* n_out) {
  if (!c || !out || !n_out || cap < 1) return fail(EPDLB_EINVAL, "bad profile arguments");
  HIPCHK(hipStreamSynchronize(c->stream));
  double tot[K_NUM] = {0}, mn[K_NUM], mx[K_NUM] = {0};
  int64_t cnt[K_NUM] = {0};
  for (int k = 0; k < K_NUM; ++k) mn[k] = 1e300;
  for (int i = 0; i < c->prof_used; ++i) {
    float ms = 0.f;
    HIPCHK(hipEventElapsedTime(&ms, c->prof_ev[2 * i], c->prof_ev[2 * i + 1]));
    const int k = c->prof_kind[i];
    tot[k] += ms;
    cnt[k] += 1;
    mn[k] = std::min(mn[k], double(ms));
    mx[k] = std::max(mx[k], double(ms));
  }
  int n = 0;
  for (int k = 0; k < K_NUM && n < cap; ++k) {
    if (!cnt[k]) continue;
    std::memset(&out[n], 0, sizeof(out[n]));
    std::snprintf(out[n].name, sizeof(out[n].name), "%s", kKindName[k]);
    out[n].launches = cnt[k];
    out[n].total_ms = tot[k];
    out[n].min_ms = mn[k];
    out[n].max_ms = mx[k];
    ++n;
  }
  *n_out = n;
  c->prof_on = false;
  c->prof_used = 0;
  return EPDLB_OK;
}

void epdlb_destroy(epdlb_ctx* c) {
  if (!c) return;
  for (hipEvent_t e : c->prof_ev) (void)hipEventDestroy(e);
  if (c->stream) (void)hipStreamSynchronize(c->stream);
  if (c->own_mem && c->base) (void)hipFree(c->base);
  if (c->own_stream && c->stream) (void)hipStreamDestroy(c->stream);
  delete c;
}

const char* epdlb_last_error(void) { return g_err.c_str(); }

}  // extern "C"
