// Host runtime and C ABI of libepdlb.so (see include/epdlb.h).
#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <new>
#include <string>
#include <tuple>
#include <vector>

#include "epdlb.h"
#include "kernels.hpp"
#include "nn.hpp"
#include "obs.hpp"
#include "cg.hpp"
#include "lb3.hpp"
#include "lb3_mrt.hpp"
#include "epd3.hpp"

using namespace epdlb;

// Scratch of the allocation-free entry point (epdlb_sigma_delta_noalloc):
// block partial sums of up to kNoAllocMaxSites sites, 2 doubles per 256
// sites, then one double for their total (64 KiB + 256 B).  Each device holds
// its own copy until the process ends; host code reaches it only through the
// address hipGetSymbolAddress gives for the current device (noalloc_scratch
// below), never through this name.
constexpr long kNoAllocMaxSites = 1024L * 1024L;
constexpr int kNoAllocMaxBlocks = int(kNoAllocMaxSites / 256);
static __device__ __align__(256) double scratch[2 * kNoAllocMaxBlocks + 32];

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
  size_t omega[2], phi, stilde, S, q[2], tmp, spec, F, fstar[2], rho, u, boltz;
  size_t mult_x, mult_y, tw_x, tw_y, wnA, wnB, scal, partials, counters;
  // surrogate mode only (density_mode 1)
  size_t nn_act[2], nn_w, nn_frag, nn_phin, nn_corr, nn_proj;
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
  L.boltz = take(2 * plane);
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
  if (p.density_mode == 1) {
    L.nn_act[0] = take(n * nn::kHid * 2);
    L.nn_act[1] = take(n * nn::kHid * 2);
    L.nn_w = take(size_t(nn::kNnParams) * sizeof(float));
    L.nn_frag = take(size_t(nn::kFwdFragElems + nn::kProjFragElems) * 2);
    L.nn_proj = take(size_t(nn::kProjRows) * n * sizeof(float));
    L.nn_phin = take(2 * plane);
    L.nn_corr = take(plane);
  }
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
  int nrep = 1;                // replicas of this grid shape sharing every launch
  size_t rstride = 0;          // bytes from one replica's arena to the next
  std::vector<epdlb_params> rp;  // per-replica parameters (g, f_A may differ)
  size_t roff(int r) const { return size_t(r) * rstride; }
  // FFT launch shapes: R values per lane, nf transforms per block
  struct Shape {
    int R, nf;
  };
  Shape sh_row{8, 1}, sh_col{8, 4}, sh_frow{8, 1}, sh_fcol{8, 4};
  // per-launch event profiler (epdlb_profile_start / epdlb_profile_read)
  bool prof_on = false;
  int prof_used = 0;
  std::vector<hipEvent_t> prof_ev;  // 2 per launch
  std::vector<int> prof_kind;
  // captured multi-kernel steps, keyed by (steps, omega parity, f* parity)
  struct GraphEntry {
    int steps, cur, fcur, kind;
    hipGraphExec_t exec;
  };
  std::vector<GraphEntry> graphs;
  hipStream_t cap_stream = nullptr;
  bool use_graph = true;
  // Surrogate steps are single steps whose kind the host picks per step; on
  // MI355X (ROCm 7) their ~12 launches go out faster as stream launches than
  // as a one-step graph (measured 0.110-0.114 against 0.115-0.120 ms per step
  // at 512^2), so graphs are opt-in there (EPDLB_SUR_GRAPH=1).
  bool sur_graph = false;
  // surrogate mode
  bool nn_ready = false;      // weights loaded
  bool last_exact = true;     // previous step (or the seed) had exact densities
  bool force_exact = false;   // residual test asks for an exact step
  int64_t n_exact = 0, n_triggered = 0;
  double resid_nn_max = 0.0;
  bool validated = false;     // the last measured surrogate error is within err_tol
  double* snap = nullptr;     // pinned: device maxima at the last check point
  hipEvent_t snap_ev = nullptr;
  bool snap_pending = false;
  int64_t snap_exact = 0;     // exact steps taken when the snapshot was queued
  // observables scratch, allocated at the first epdlb_observables call
  unsigned char* obs = nullptr;
  // per replica: the scratch holds the particle sites of a previous tracking sample
  std::vector<unsigned char> track_valid;
  // Phi -> omega inversion: device scratch (6 field sets, partials, results)
  // and a pinned pair of doubles for the host's decisions; allocated at
  // create (cg_invert = 1) or at the first epdlb_invert_densities call
  unsigned char* cg = nullptr;
  double* cg_host = nullptr;
  epdlb_cg_info cg_last{};
  int64_t cg_totals[4] = {0, 0, 0, 0};  // inversions, iterations, evaluations, unconverged
  // offsets are taken modulo 2^64 so that buffers outside the arena (the
  // inversion's scratch) can stand in for arena buffers in a stage
  template <typename T> T* ptr(size_t off) const {
    return reinterpret_cast<T*>(reinterpret_cast<uintptr_t>(base) + off);
  }
  size_t off_of(const void* q) const { return size_t(reinterpret_cast<uintptr_t>(q) - reinterpret_cast<uintptr_t>(base)); }
};

namespace {

int nn_after_seed(epdlb_ctx* c);

enum Kind { K_STATS, K_ADVECT, K_FINISH, K_PROP_ROW, K_PROP_COL, K_DENSITY, K_FROW_FWD, K_FCOL,
            K_FROW_INV, K_LB, K_NN_CONV0, K_NN_CONV, K_NN_OUT, K_NN_NORM, K_NN_RESET, K_ADVECT_ONLY, K_CG,
            K_FINV_LB, K_NORM_FROW, K_NUM };
const char* const kKindName[K_NUM] = {"field_stats", "advect_update", "finish_stats",
                                      "prop_row",    "prop_col",      "density",       "force_row_fwd",
                                      "force_col",   "force_row_inv", "lb",            "nn_conv0",
                                      "nn_conv",     "nn_out",        "nn_norm",       "nn_reset",
                                      "advect_only", "cg_vector",     "force_inv_lb",  "nn_norm_force_row"};

// Profiling: while the profiler has room, the next kernel launch records a
// start/stop event pair at the kernel's own start and end (AMD's extended
// launch), so the times are kernel durations even when the host is slower
// than the GPU.  Recording never blocks.
thread_local hipEvent_t tl_ev_start = nullptr;
thread_local hipEvent_t tl_ev_stop = nullptr;

template <typename F, typename... Args>
void launch_k(F kernel, dim3 grid, dim3 block, size_t lds, hipStream_t s, Args... args) {
  if (tl_ev_start) {
    hipExtLaunchKernelGGL(kernel, grid, block, uint32_t(lds), s, tl_ev_start, tl_ev_stop, 0u, args...);
    tl_ev_start = tl_ev_stop = nullptr;  // one launch per armed pair
  } else {
    hipLaunchKernelGGL(kernel, grid, block, lds, s, args...);
  }
}

struct ProfScope {
  epdlb_ctx* c;
  int kind;
  bool rec;
  ProfScope(epdlb_ctx* ctx, int k) : c(ctx), kind(k) {
    rec = c->prof_on && size_t(2 * c->prof_used + 1) < c->prof_ev.size();
    if (rec) {
      tl_ev_start = c->prof_ev[2 * c->prof_used];
      tl_ev_stop = c->prof_ev[2 * c->prof_used + 1];
    }
  }
  ~ProfScope() {
    if (!rec) return;
    if (tl_ev_start) {  // armed but not consumed: nothing recorded
      tl_ev_start = tl_ev_stop = nullptr;
      return;
    }
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
  if (p->lb_mrt != 0 && p->lb_mrt != 1) return fail(EPDLB_EINVAL, "lb_mrt must be 0 or 1");
  if (p->lb_mrt == 1 && !(std::fabs(p->lb_gamma_s) < 1.0 && std::fabs(p->lb_gamma_b) < 1.0 &&
                          std::fabs(p->lb_gamma_g) < 1.0))
    return fail(EPDLB_EINVAL, "lb_gamma_s, lb_gamma_b, lb_gamma_g must lie in (-1, 1)");
  if (p->precision != 0 && p->precision != 1) return fail(EPDLB_EINVAL, "precision must be 0 or 1");
  if (p->g_units != 0 && p->g_units != 1) return fail(EPDLB_EINVAL, "g_units must be 0 or 1");
  if (!std::isfinite(p->g) || !std::isfinite(p->kT_over_v) || !std::isfinite(p->kappa_H) ||
      !std::isfinite(p->chi_AB) || !std::isfinite(p->chi_AS) || !std::isfinite(p->chi_BS))
    return fail(EPDLB_EINVAL, "non-finite parameter");
  if (p->density_mode != 0 && p->density_mode != 1) return fail(EPDLB_EINVAL, "density_mode must be 0 or 1");
  if (p->density_mode == 1 &&
      (p->fallback_every < 1 || p->check_every < 1 || !(p->resid_tol > 0.0) || !std::isfinite(p->resid_tol) ||
       !(p->err_tol >= 0.0) || !std::isfinite(p->err_tol)))
    return fail(EPDLB_EINVAL,
                "surrogate mode needs fallback_every >= 1, check_every >= 1, resid_tol > 0, err_tol >= 0");
  if (p->cg_invert != 0 && p->cg_invert != 1) return fail(EPDLB_EINVAL, "cg_invert must be 0 or 1");
  if (p->cg_precond != 0 && p->cg_precond != 1) return fail(EPDLB_EINVAL, "cg_precond must be 0 or 1");
  if (p->cg_invert == 1) {
    if (p->density_mode != 0) return fail(EPDLB_EINVAL, "cg_invert needs exact densities (density_mode 0)");
    if (p->cg_max_iter < 0 || p->cg_max_iter > 1000000) return fail(EPDLB_EINVAL, "cg_max_iter must be in [0, 1e6]");
    if (!(p->cg_tol > 0.0) || !std::isfinite(p->cg_tol)) return fail(EPDLB_EINVAL, "cg_tol must be > 0");
    if (p->precision == 1 && p->cg_tol < 1e-6)
      return fail(EPDLB_EINVAL, "cg_tol below 1e-6 needs FP64 fields (precision 0)");
  }
  if (!(p->mach_max >= 0.0) || !std::isfinite(p->mach_max)) return fail(EPDLB_EINVAL, "mach_max must be >= 0");
  return EPDLB_OK;
}

// Segment A fractions a_j = clip(f_A N - j, 0, 1) of a parameter set.
std::vector<double> segment_fractions(const epdlb_params& p) {
  const int N = p.n_contour;
  std::vector<double> a(N);
  for (int j = 0; j < N; ++j) {
    const double v = p.f_A * N - j;
    a[j] = v < 0 ? 0.0 : (v > 1 ? 1.0 : v);
  }
  return a;
}

double g_lattice(const epdlb_params& p) { return p.g_units ? p.g : p.g * p.dt * p.dt / p.dx; }

// Lattice kinematic shear viscosity of the configured collision (rho = 1).
double lb_nu(const epdlb_params& p) {
  return p.lb_mrt ? (1.0 / 6.0) * (1.0 + p.lb_gamma_s) / (1.0 - p.lb_gamma_s) : (p.lb_tau - 0.5) / 3.0;
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

template <typename T, int L, int R>
constexpr bool fft_ok() {
  return (R == 8 || ((R == 16 || R == 4 || R == 2) && sizeof(T) == 4)) && L >= R;
}
constexpr int kMaxColThreads = 512;

template <typename T, int L, int R>
hipError_t launch_prop_row_r(const PropArgs<T>& a, hipStream_t s) {
  if constexpr (fft_ok<T, L, R>()) {
    using V = LdsView<T, L, R, true, 1>;
    const size_t lds = 2 * size_t(V::size_elems(a.nf)) * sizeof(T);
    hipError_t e = prep_lds(k_prop_row<T, L, R>, lds);
    if (e != hipSuccess) return e;
    const int tiles = (a.ny / 2 + a.nf - 1) / a.nf;
    launch_k((k_prop_row<T, L, R>), dim3(tiles, 2, a.nrep), dim3(a.nf * (L / R)), lds, s, a);
    return hipGetLastError();
  }
  return hipErrorInvalidValue;
}
template <typename T, int L>
hipError_t launch_prop_row(const PropArgs<T>& a, int R, hipStream_t s) {
  switch (R) {
    case 16: return launch_prop_row_r<T, L, 16>(a, s);
    case 4: return launch_prop_row_r<T, L, 4>(a, s);
    case 2: return launch_prop_row_r<T, L, 2>(a, s);
  }
  return launch_prop_row_r<T, L, 8>(a, s);
}

template <typename T, int L, int R, int NF>
hipError_t launch_prop_col_rn(const PropArgs<T>& a, hipStream_t s) {
  if constexpr (fft_ok<T, L, R>() && NF * (L / R) <= kMaxColThreads && (sizeof(T) == 4 || NF == 4)) {
    using V = LdsView<T, L, R, false, NF>;
    const size_t lds = 2 * size_t(V::size_elems(NF)) * sizeof(T);
    hipError_t e = prep_lds(k_prop_col<T, L, R, NF>, lds);
    if (e != hipSuccess) return e;
    const int tiles = (a.nx / 2 + NF - 1) / NF;
    launch_k((k_prop_col<T, L, R, NF>), dim3(tiles, 2, a.nrep), dim3(NF * (L / R)), lds, s, a);
    return hipGetLastError();
  }
  return hipErrorInvalidValue;
}
template <typename T, int L, int R>
hipError_t launch_prop_col_r(const PropArgs<T>& a, hipStream_t s) {
  switch (a.nf) {
    case 4: return launch_prop_col_rn<T, L, R, 4>(a, s);
    case 8: return launch_prop_col_rn<T, L, R, 8>(a, s);
    case 16: return launch_prop_col_rn<T, L, R, 16>(a, s);
  }
  return hipErrorInvalidValue;
}
template <typename T, int L>
hipError_t launch_prop_col(const PropArgs<T>& a, int R, hipStream_t s) {
  switch (R) {
    case 16: return launch_prop_col_r<T, L, 16>(a, s);
    case 4: return launch_prop_col_r<T, L, 4>(a, s);
    case 2: return launch_prop_col_r<T, L, 2>(a, s);
  }
  return launch_prop_col_r<T, L, 8>(a, s);
}

template <typename T, int L, int R>
hipError_t launch_force_row_fwd_r(const ForceArgs<T>& a, hipStream_t s) {
  if constexpr (fft_ok<T, L, R>()) {
    using V = LdsView<T, L, R, true, 1>;
    const size_t lds = 2 * size_t(V::size_elems(a.nf)) * sizeof(T);
    hipError_t e = prep_lds(k_force_row_fwd<T, L, R>, lds);
    if (e != hipSuccess) return e;
    launch_k((k_force_row_fwd<T, L, R>), dim3((a.ny + a.nf - 1) / a.nf, 1, a.nrep), dim3(a.nf * (L / R)),
                       lds, s, a);
    return hipGetLastError();
  }
  return hipErrorInvalidValue;
}
template <typename T, int L>
hipError_t launch_force_row_fwd(const ForceArgs<T>& a, int R, hipStream_t s) {
  switch (R) {
    case 16: return launch_force_row_fwd_r<T, L, 16>(a, s);
    case 4: return launch_force_row_fwd_r<T, L, 4>(a, s);
    case 2: return launch_force_row_fwd_r<T, L, 2>(a, s);
  }
  return launch_force_row_fwd_r<T, L, 8>(a, s);
}
template <typename T, int L, int R>
hipError_t launch_force_row_inv_r(const ForceArgs<T>& a, hipStream_t s) {
  if constexpr (fft_ok<T, L, R>()) {
    using V = LdsView<T, L, R, true, 1>;
    const size_t lds = 2 * size_t(V::size_elems(a.nf)) * sizeof(T);
    hipError_t e = prep_lds(k_force_row_inv<T, L, R>, lds);
    if (e != hipSuccess) return e;
    launch_k((k_force_row_inv<T, L, R>), dim3((a.ny + a.nf - 1) / a.nf, 1, a.nrep), dim3(a.nf * (L / R)),
                       lds, s, a);
    return hipGetLastError();
  }
  return hipErrorInvalidValue;
}
template <typename T, int L>
hipError_t launch_force_row_inv(const ForceArgs<T>& a, int R, hipStream_t s) {
  switch (R) {
    case 16: return launch_force_row_inv_r<T, L, 16>(a, s);
    case 4: return launch_force_row_inv_r<T, L, 4>(a, s);
    case 2: return launch_force_row_inv_r<T, L, 2>(a, s);
  }
  return launch_force_row_inv_r<T, L, 8>(a, s);
}
template <typename T, int L, int R, int NF>
hipError_t launch_force_col_rn(const ForceArgs<T>& a, hipStream_t s) {
  if constexpr (fft_ok<T, L, R>() && NF * (L / R) <= kMaxColThreads && (sizeof(T) == 4 || NF == 4)) {
    using V = LdsView<T, L, R, false, NF>;
    const size_t lds = 2 * size_t(V::size_elems(NF)) * sizeof(T);
    hipError_t e = prep_lds(k_force_col<T, L, R, NF>, lds);
    if (e != hipSuccess) return e;
    launch_k((k_force_col<T, L, R, NF>), dim3((a.nx + NF - 1) / NF, 1, a.nrep), dim3(NF * (L / R)), lds, s,
                       a);
    return hipGetLastError();
  }
  return hipErrorInvalidValue;
}
template <typename T, int L, int R>
hipError_t launch_force_col_r(const ForceArgs<T>& a, hipStream_t s) {
  switch (a.nf) {
    case 4: return launch_force_col_rn<T, L, R, 4>(a, s);
    case 8: return launch_force_col_rn<T, L, R, 8>(a, s);
    case 16: return launch_force_col_rn<T, L, R, 16>(a, s);
  }
  return hipErrorInvalidValue;
}
template <typename T, int L>
hipError_t launch_force_col(const ForceArgs<T>& a, int R, hipStream_t s) {
  switch (R) {
    case 16: return launch_force_col_r<T, L, 16>(a, s);
    case 4: return launch_force_col_r<T, L, 4>(a, s);
    case 2: return launch_force_col_r<T, L, 2>(a, s);
  }
  return launch_force_col_r<T, L, 8>(a, s);
}

// Row-inverse force pass fused with the LB step (R = 4 or 8; other shapes run
// the two kernels separately).
template <typename T, int L, int R, bool MRT>
hipError_t launch_force_inv_lb_r(const ForceArgs<T>& a, const LbArgs<T>& b, hipStream_t s) {
  if constexpr (fft_ok<T, L, R>()) {
    using V = LdsView<T, L, R, true, 1>;
    const size_t lds = 2 * size_t(V::size_elems(a.nf)) * sizeof(T);
    hipError_t e = prep_lds(k_force_inv_lb<T, L, R, MRT>, lds);
    if (e != hipSuccess) return e;
    launch_k((k_force_inv_lb<T, L, R, MRT>), dim3((a.ny + a.nf - 1) / a.nf, 1, a.nrep), dim3(a.nf * (L / R)),
             lds, s, a, b);
    return hipGetLastError();
  }
  return hipErrorInvalidValue;
}
template <typename T, int L>
hipError_t launch_force_inv_lb(const ForceArgs<T>& a, const LbArgs<T>& b, int R, bool mrt, hipStream_t s) {
  switch (R) {
    case 4: return mrt ? launch_force_inv_lb_r<T, L, 4, true>(a, b, s) : launch_force_inv_lb_r<T, L, 4, false>(a, b, s);
    case 8: return mrt ? launch_force_inv_lb_r<T, L, 8, true>(a, b, s) : launch_force_inv_lb_r<T, L, 8, false>(a, b, s);
  }
  return hipErrorInvalidValue;
}
bool force_inv_lb_shape(int R) { return R == 4 || R == 8; }

// The surrogate's normalisation fused with the row-forward force pass (R = 4 or 8).
template <typename T, int L, int R>
hipError_t launch_norm_force_row_r(const ForceArgs<T>& a, const nn::NormArgs<T>& q, hipStream_t s) {
  if constexpr (fft_ok<T, L, R>()) {
    using V = LdsView<T, L, R, true, 1>;
    const size_t lds = 2 * size_t(V::size_elems(a.nf)) * sizeof(T);
    hipError_t e = prep_lds(nn::k_norm_force_row<T, L, R>, lds);
    if (e != hipSuccess) return e;
    launch_k((nn::k_norm_force_row<T, L, R>), dim3((a.ny + a.nf - 1) / a.nf, 1, 1), dim3(a.nf * (L / R)), lds, s,
             a, q);
    return hipGetLastError();
  }
  return hipErrorInvalidValue;
}
template <typename T, int L>
hipError_t launch_norm_force_row(const ForceArgs<T>& a, const nn::NormArgs<T>& q, int R, hipStream_t s) {
  switch (R) {
    case 4: return launch_norm_force_row_r<T, L, 4>(a, q, s);
    case 8: return launch_norm_force_row_r<T, L, 8>(a, q, s);
  }
  return hipErrorInvalidValue;
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

template <typename T> hipError_t prop_row(int L, int R, const PropArgs<T>& a, hipStream_t s) {
  EPDLB_SWITCH_L(L, launch_prop_row, T, a, R, s)
}
template <typename T> hipError_t prop_col(int L, int R, const PropArgs<T>& a, hipStream_t s) {
  EPDLB_SWITCH_L(L, launch_prop_col, T, a, R, s)
}
template <typename T> hipError_t force_row_fwd(int L, int R, const ForceArgs<T>& a, hipStream_t s) {
  EPDLB_SWITCH_L(L, launch_force_row_fwd, T, a, R, s)
}
template <typename T> hipError_t force_col(int L, int R, const ForceArgs<T>& a, hipStream_t s) {
  EPDLB_SWITCH_L(L, launch_force_col, T, a, R, s)
}
template <typename T> hipError_t force_row_inv(int L, int R, const ForceArgs<T>& a, hipStream_t s) {
  EPDLB_SWITCH_L(L, launch_force_row_inv, T, a, R, s)
}
template <typename T>
hipError_t force_inv_lb(int L, int R, const ForceArgs<T>& a, const LbArgs<T>& b, bool mrt, hipStream_t s) {
  EPDLB_SWITCH_L(L, launch_force_inv_lb, T, a, b, R, mrt, s)
}
template <typename T>
hipError_t norm_force_row(int L, int R, const ForceArgs<T>& a, const nn::NormArgs<T>& q, hipStream_t s) {
  EPDLB_SWITCH_L(L, launch_norm_force_row, T, a, q, R, s)
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
  a.nrep = c->nrep;
  a.rs = long(c->rstride);
  const int blocks = int(std::min<long>(1024, (n + 255) / 256));
  ProfScope ps(c, K_STATS);
  launch_k((k_field_stats<T>), dim3(blocks, 1, c->nrep), dim3(256), 0, c->stream, a);
  HIPCHK(hipGetLastError());
  launch_k(k_finish_stats, dim3(1, 1, c->nrep), dim3(256), 0, c->stream, a.partials, blocks, a.scal, n,
           c->p.dx * c->p.dx, long(c->rstride));
  HIPCHK(hipGetLastError());
  return EPDLB_OK;
}

template <typename T>
UpdArgs<T> make_upd_args(epdlb_ctx* c, bool flow) {
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
  a.advect = flow && p.couple_lb ? 1 : 0;
  a.nrep = c->nrep;
  a.rs = long(c->rstride);
  return a;
}

// flow = false: mu and the omega update at the stored fields without
// convection (used after the Phi -> omega inversion, which convects first).
template <typename T>
int stage_advect_update(epdlb_ctx* c, bool flow = true) {
  const epdlb_params& p = c->p;
  const long n = long(p.nx) * p.ny;
  UpdArgs<T> a = make_upd_args<T>(c, flow);
  {
    ProfScope ps(c, K_ADVECT);
    launch_k((k_advect_update<T>), dim3(p.nx / kTX, p.ny / kTY, c->nrep), dim3(kTX * kTY), 0, c->stream, a);
  }
  HIPCHK(hipGetLastError());
  {
    ProfScope ps(c, K_FINISH);
    launch_k(k_finish_stats, dim3(1, 1, c->nrep), dim3(256), 0, c->stream, a.partials,
             (p.nx / kTX) * (p.ny / kTY), c->ptr<double>(c->L.scal), n, p.dx * p.dx, long(c->rstride));
  }
  HIPCHK(hipGetLastError());
  c->cur = 1 - c->cur;
  return EPDLB_OK;
}

template <typename T>
PropArgs<T> make_prop_args(epdlb_ctx* c) {
  const epdlb_params& p = c->p;
  const long n = long(p.nx) * p.ny;
  PropArgs<T> a;
  a.wA = c->ptr<T>(c->L.omega[c->cur]);
  a.wB = a.wA + n;
  a.EA = c->ptr<T>(c->L.boltz);
  a.EB = a.EA + n;
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
  a.partials = c->ptr<double>(c->L.partials);
  a.a = 0;
  a.first = a.mid = a.second = a.last = 0;
  a.frac[0][0] = a.frac[0][1] = a.frac[1][0] = a.frac[1][1] = T(1);
  a.nf = 1;
  a.nrep = c->nrep;
  a.rs = long(c->rstride);
  return a;
}

template <typename T>
int stage_densities(epdlb_ctx* c, bool with_S) {
  const epdlb_params& p = c->p;
  const int N = p.n_contour;
  const long n = long(p.nx) * p.ny;
  PropArgs<T> a = make_prop_args<T>(c);
  auto launch = [&](bool row) -> int {
    if (row) {
      a.nf = c->sh_row.nf;
      ProfScope ps(c, K_PROP_ROW);
      HIPCHK(prop_row<T>(p.nx, c->sh_row.R, a, c->stream));
    } else {
      a.nf = c->sh_col.nf;
      ProfScope ps(c, K_PROP_COL);
      HIPCHK(prop_col<T>(p.ny, c->sh_col.R, a, c->stream));
    }
    return EPDLB_OK;
  };
  // step 0 starts with its x convolution of E(step 0); that first pass also
  // writes the half-step factor planes the later passes read
  // segment A fractions (uniform over the replicas of a launch)
  const std::vector<double> segA = segment_fractions(p);
  auto seg = [&](int chain, int step) { return T(segA[chain == 0 ? step : N - 1 - step]); };
  a.a = 0;
  a.first = 1;
  a.mid = a.second = a.last = 0;
  for (int ch = 0; ch < 2; ++ch) a.frac[ch][0] = a.frac[ch][1] = seg(ch, 0);
  CHK(launch(true));
  // boundary a -> a+1: last convolution of step a and first of step a+1
  // (y-oriented after an even step, x-oriented after an odd one)
  a.first = 0;
  a.mid = 1;
  for (int s = 0; s < N; ++s) {
    a.a = s;
    a.second = s + 1 < N;
    a.last = s + 1 == N;
    for (int ch = 0; ch < 2; ++ch) {
      a.frac[ch][0] = seg(ch, s);
      a.frac[ch][1] = s + 1 < N ? seg(ch, s + 1) : seg(ch, s);
    }
    CHK(launch(s % 2 == 1));
  }
  DensArgs<T> d;
  d.qpart = a.partials;
  // partial slots of the final propagator launch (x-oriented if N-1 is odd)
  d.nqpart = ((N - 1) % 2 == 1) ? (p.ny / 2 + c->sh_row.nf - 1) / c->sh_row.nf
                                : (p.nx / 2 + c->sh_col.nf - 1) / c->sh_col.nf;
  d.dA = p.dx * p.dx;
  d.scal_out = c->ptr<double>(c->L.scal);
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
  d.nrep = c->nrep;
  d.rs = long(c->rstride);
  {
    ProfScope ps(c, K_DENSITY);
    launch_k((k_density<T>), dim3((n + 255) / 256, 1, c->nrep), dim3(256), 0, c->stream, d);
  }
  HIPCHK(hipGetLastError());
  return EPDLB_OK;
}

template <typename T>
ForceArgs<T> make_force_args(epdlb_ctx* c) {
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
  a.scal = c->ptr<double>(c->L.scal);
  a.nf = 1;
  a.nrep = c->nrep;
  a.rs = long(c->rstride);
  return a;
}

template <typename T>
int stage_force(epdlb_ctx* c) {
  const epdlb_params& p = c->p;
  ForceArgs<T> a = make_force_args<T>(c);
  a.nf = c->sh_frow.nf;
  {
    ProfScope ps(c, K_FROW_FWD);
    HIPCHK(force_row_fwd<T>(p.nx, c->sh_frow.R, a, c->stream));
  }
  a.nf = c->sh_fcol.nf;
  {
    ProfScope ps(c, K_FCOL);
    HIPCHK(force_col<T>(p.ny, c->sh_fcol.R, a, c->stream));
  }
  a.nf = c->sh_frow.nf;
  {
    ProfScope ps(c, K_FROW_INV);
    HIPCHK(force_row_inv<T>(p.nx, c->sh_frow.R, a, c->stream));
  }
  return EPDLB_OK;
}

template <typename T>
LbArgs<T> make_lb_args(epdlb_ctx* c) {
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
  a.gs = T(p.lb_gamma_s);
  a.gb = T(p.lb_gamma_b);
  a.gg = T(p.lb_gamma_g);
  // |u| > mach_max c_s, c_s^2 = 1/3 in lattice units; 0 disables the speed test
  a.umax2 = p.mach_max > 0.0 ? T(p.mach_max * p.mach_max / 3.0) : T(INFINITY);
  a.guard = c->ptr<unsigned>(c->L.counters);
  a.nrep = c->nrep;
  a.rs = long(c->rstride);
  return a;
}

template <typename T>
int stage_lb(epdlb_ctx* c) {
  const epdlb_params& p = c->p;
  const long n = long(p.nx) * p.ny;
  const LbArgs<T> a = make_lb_args<T>(c);
  {
    ProfScope ps(c, K_LB);
    if (p.lb_mrt)
      launch_k((k_lb<T, true>), dim3((n + 255) / 256, 1, c->nrep), dim3(256), 0, c->stream, a);
    else
      launch_k((k_lb<T, false>), dim3((n + 255) / 256, 1, c->nrep), dim3(256), 0, c->stream, a);
  }
  HIPCHK(hipGetLastError());
  c->fcur = 1 - c->fcur;
  return EPDLB_OK;
}

// Force and LB of one step: the row-inverse force pass and the LB step share a
// launch when the row shape allows it; otherwise the two stages as above.
// norm (surrogate steps, may be NULL): the network's normalisation, launched
// together with the first force pass (its shape is then a fusable one).
template <typename T>
int stage_force_lb(epdlb_ctx* c, const nn::NormArgs<T>* norm = nullptr) {
  const epdlb_params& p = c->p;
  if (!force_inv_lb_shape(c->sh_frow.R)) {
    CHK(stage_force<T>(c));
    return stage_lb<T>(c);
  }
  ForceArgs<T> a = make_force_args<T>(c);
  a.nf = c->sh_frow.nf;
  if (norm) {
    ProfScope ps(c, K_NORM_FROW);
    HIPCHK(norm_force_row<T>(p.nx, c->sh_frow.R, a, *norm, c->stream));
  } else {
    ProfScope ps(c, K_FROW_FWD);
    HIPCHK(force_row_fwd<T>(p.nx, c->sh_frow.R, a, c->stream));
  }
  a.nf = c->sh_fcol.nf;
  {
    ProfScope ps(c, K_FCOL);
    HIPCHK(force_col<T>(p.ny, c->sh_fcol.R, a, c->stream));
  }
  a.nf = c->sh_frow.nf;
  const LbArgs<T> b = make_lb_args<T>(c);
  {
    ProfScope ps(c, K_FINV_LB);
    HIPCHK(force_inv_lb<T>(p.nx, c->sh_frow.R, a, b, p.lb_mrt != 0, c->stream));
  }
  c->fcur = 1 - c->fcur;
  return EPDLB_OK;
}

int run_force_lb(epdlb_ctx* c) {
  return c->p.precision == 0 ? stage_force_lb<double>(c) : stage_force_lb<float>(c);
}

// ---------------------------------------------------------------------------
// Phi -> omega inversion (App. C, comments 1-3): the scratch holds the target
// composition Phi~, the iterate x, the direction d, the descent direction s,
// the trial point xt and the evaluated densities, 3 planes each.
// ---------------------------------------------------------------------------
struct CgLayout {
  size_t set[7];  // target, x, d, s, xt, phi, z (preconditioned direction source)
  size_t part, out, total;
};
enum { CG_TARGET, CG_X, CG_D, CG_S, CG_XT, CG_PHI, CG_Z, CG_NSETS };

CgLayout cg_layout(const epdlb_params& p) {
  const size_t es = p.precision == 0 ? 8 : 4;
  const size_t set = 3 * size_t(p.nx) * p.ny * es;
  CgLayout L{};
  size_t off = 0;
  for (int i = 0; i < CG_NSETS; ++i) {
    L.set[i] = off;
    off = align256(off + set);
  }
  L.part = off;
  off = align256(off + 2 * cg::kBlocks * sizeof(double));
  L.out = off;
  off = align256(off + 2 * sizeof(double));
  L.total = off;
  return L;
}

int ensure_cg(epdlb_ctx* c) {
  if (c->cg) return EPDLB_OK;
  void* m = nullptr;
  if (hipMalloc(&m, cg_layout(c->p).total) != hipSuccess) return fail(EPDLB_ENOMEM, "inversion scratch allocation failed");
  void* h = nullptr;
  if (hipHostMalloc(&h, 2 * sizeof(double), hipHostMallocDefault) != hipSuccess) {
    (void)hipFree(m);
    return fail(EPDLB_ENOMEM, "pinned host allocation failed");
  }
  c->cg = static_cast<unsigned char*>(m);
  c->cg_host = static_cast<double*>(h);
  return EPDLB_OK;
}

template <typename T> T* cg_set(epdlb_ctx* c, int which) {
  return reinterpret_cast<T*>(c->cg + cg_layout(c->p).set[which]);
}

// Densities of the field set at `w` into `phi` through the ordinary stages
// (field statistics, propagators, density integrals), the arena's omega and
// Phi buffers standing in for them during the call.
template <typename T>
int cg_eval(epdlb_ctx* c, const T* w, T* phi) {
  const size_t w0 = c->L.omega[c->cur], p0 = c->L.phi;
  c->L.omega[c->cur] = c->off_of(w);
  c->L.phi = c->off_of(phi);
  int r = stage_stats<T>(c);
  if (r == EPDLB_OK) r = stage_densities<T>(c, false);
  c->L.omega[c->cur] = w0;
  c->L.phi = p0;
  return r;
}

// Sums the partials of nq quantities and brings them to the host (synchronises).
int cg_reduce(epdlb_ctx* c, int nq, double* out) {
  const CgLayout L = cg_layout(c->p);
  double* part = reinterpret_cast<double*>(c->cg + L.part);
  double* dev = reinterpret_cast<double*>(c->cg + L.out);
  {
    ProfScope ps(c, K_CG);
    launch_k(cg::k_cg_finish, dim3(1), dim3(cg::kThreads), 0, c->stream, (const double*)part, cg::kBlocks, nq, dev);
  }
  HIPCHK(hipGetLastError());
  HIPCHK(hipMemcpyAsync(c->cg_host, dev, 2 * sizeof(double), hipMemcpyDeviceToHost, c->stream));
  HIPCHK(hipStreamSynchronize(c->stream));
  out[0] = c->cg_host[0];
  out[1] = c->cg_host[1];
  return EPDLB_OK;
}

// Fletcher-Reeves iteration from x towards Phi[x] = target (both in the
// scratch); x holds the result.  info gets the counts and residuals.
template <typename T>
int cg_invert(epdlb_ctx* c, double tol, int max_iter, epdlb_cg_info* info) {
  const long n = long(c->p.nx) * c->p.ny, m = 3 * n;
  const CgLayout L = cg_layout(c->p);
  T* tgt = cg_set<T>(c, CG_TARGET);
  T* x = cg_set<T>(c, CG_X);
  T* d = cg_set<T>(c, CG_D);
  T* s = cg_set<T>(c, CG_S);
  T* xt = cg_set<T>(c, CG_XT);
  T* phi = cg_set<T>(c, CG_PHI);
  T* z = c->p.cg_precond ? cg_set<T>(c, CG_Z) : nullptr;
  double* part = reinterpret_cast<double*>(c->cg + L.part);
  const dim3 grid(cg::kBlocks), blk(cg::kThreads);
  *info = epdlb_cg_info{};
  double r2 = 0.0, sz = 0.0, sums[2];
  // descent direction s = Phi[x] - target (and z = s / m), |s|^2 and s.z
  auto resid = [&](double* out2) -> int {
    CHK(cg_eval<T>(c, x, phi));
    ++info->evals;
    {
      ProfScope ps(c, K_CG);
      launch_k((cg::k_cg_resid<T>), grid, blk, 0, c->stream, (const T*)phi, (const T*)tgt, s, z, m, n,
               T(c->p.n_contour), part);
    }
    HIPCHK(hipGetLastError());
    return cg_reduce(c, 2, out2);
  };
  // d = z (first) or z + beta d, trial point x + alpha_t d; returns d.s and d.s(trial)
  auto trial = [&](double beta, int first, double alpha_t) -> int {
    {
      ProfScope ps(c, K_CG);
      launch_k((cg::k_cg_trial<T>), grid, blk, 0, c->stream, (const T*)s, (const T*)(z ? z : s), d, (const T*)x,
               xt, T(beta), first, T(alpha_t), m, part);
    }
    HIPCHK(hipGetLastError());
    CHK(cg_eval<T>(c, xt, phi));
    ++info->evals;
    {
      ProfScope ps(c, K_CG);
      launch_k((cg::k_cg_dirdot<T>), grid, blk, 0, c->stream, (const T*)d, (const T*)phi, (const T*)tgt, m,
               part + cg::kBlocks);
    }
    HIPCHK(hipGetLastError());
    return cg_reduce(c, 2, sums);
  };
  {
    double v[2];
    CHK(resid(v));
    r2 = v[0];
    sz = v[1];
  }
  info->resid0 = info->resid = std::sqrt(r2 / double(n));
  info->converged = info->resid < tol;
  double beta = 0.0, alpha_t = 1.0;
  int first = 1;
  for (int it = 1; it <= max_iter && !info->converged; ++it) {
    CHK(trial(beta, first, alpha_t));
    if (!(sums[0] > 0.0) && !first) {
      // not a descent direction: restart along s
      ++info->restarts;
      first = 1;
      CHK(trial(0.0, 1, alpha_t));
    }
    const double delta0 = sums[0], curv = sums[0] - sums[1];
    const double alpha = curv > 0.0 ? alpha_t * delta0 / curv : alpha_t;
    {
      ProfScope ps(c, K_CG);
      launch_k((cg::k_cg_axpy<T>), grid, blk, 0, c->stream, x, (const T*)d, T(alpha), m);
    }
    HIPCHK(hipGetLastError());
    double v[2];
    CHK(resid(v));
    info->iters = it;
    info->resid = std::sqrt(v[0] / double(n));
    info->converged = info->resid < tol;
    if (!std::isfinite(info->resid)) break;  // a state that blew up: stop, unconverged
    beta = v[1] / sz;
    r2 = v[0];
    sz = v[1];
    alpha_t = alpha;
    first = 0;
  }
  ++c->cg_totals[0];
  c->cg_totals[1] += info->iters;
  c->cg_totals[2] += info->evals;
  if (!info->converged) ++c->cg_totals[3];
  c->cg_last = *info;
  return EPDLB_OK;
}

// Convection, inversion of the convected composition from the auxiliary-
// convected omega, then mu and the omega update at (Phi~, omega~).
template <typename T>
int stage_advect_cg(epdlb_ctx* c) {
  const epdlb_params& p = c->p;
  CHK(ensure_cg(c));
  {
    const UpdArgs<T> a = make_upd_args<T>(c, true);
    ProfScope ps(c, K_ADVECT_ONLY);
    launch_k((k_advect_only<T>), dim3(p.nx / kTX, p.ny / kTY), dim3(kTX * kTY), 0, c->stream, a,
             cg_set<T>(c, CG_TARGET), cg_set<T>(c, CG_X));
  }
  HIPCHK(hipGetLastError());
  epdlb_cg_info info;
  CHK(cg_invert<T>(c, p.cg_tol, p.cg_max_iter, &info));
  const int cur0 = c->cur;
  const size_t w0 = c->L.omega[cur0], p0 = c->L.phi;
  c->L.omega[cur0] = c->off_of(cg_set<T>(c, CG_X));
  c->L.phi = c->off_of(cg_set<T>(c, CG_TARGET));
  const int r = stage_advect_update<T>(c, false);
  c->L.omega[cur0] = w0;
  c->L.phi = p0;
  return r;
}

template <typename T>
int run_stage_t(epdlb_ctx* c, int stage) {
  switch (stage) {
    case EPDLB_STAGE_ADVECT_UPDATE: return c->p.cg_invert ? stage_advect_cg<T>(c) : stage_advect_update<T>(c);
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
// Autotuner for the FFT pass launch shapes (values per lane R, transforms per
// block nf).  A candidate is timed as a captured graph of `reps` back-to-back
// launches; the passes write scratch planes only (row output, chain plane 2,
// Q partials, force spectrum and force planes), so the state is unchanged.
// ---------------------------------------------------------------------------
enum Family { F_PROP_ROW, F_PROP_COL, F_FORCE_ROW, F_FORCE_COL, F_NUM };
const char* const kFamilyName[F_NUM] = {"prop_row", "prop_col", "force_row", "force_col"};

epdlb_ctx::Shape& family_shape(epdlb_ctx* c, int f) {
  switch (f) {
    case F_PROP_ROW: return c->sh_row;
    case F_PROP_COL: return c->sh_col;
    case F_FORCE_ROW: return c->sh_frow;
    default: return c->sh_fcol;
  }
}

template <typename T>
hipError_t launch_family(epdlb_ctx* c, int fam, int R, int nf, hipStream_t s) {
  const epdlb_params& p = c->p;
  if (fam == F_PROP_ROW || fam == F_PROP_COL) {
    PropArgs<T> a = make_prop_args<T>(c);
    a.a = 0;  // fused boundary kernel: writes q_1 and the scratch plane
    a.mid = a.second = 1;
    a.nf = nf;
    return fam == F_PROP_ROW ? prop_row<T>(p.nx, R, a, s) : prop_col<T>(p.ny, R, a, s);
  }
  ForceArgs<T> a = make_force_args<T>(c);
  a.nf = nf;
  if (fam == F_FORCE_ROW) {
    // the row passes of the force together with the LB step, as the step runs
    // them: fused with the row inverse where the shape allows, else after it
    // (the LB part writes u, rho, the guard words and the other population
    // buffer: epdlb_autotune keeps the first three)
    hipError_t e = force_row_fwd<T>(p.nx, R, a, s);
    if (e != hipSuccess) return e;
    const LbArgs<T> b = make_lb_args<T>(c);
    if (force_inv_lb_shape(R)) return force_inv_lb<T>(p.nx, R, a, b, p.lb_mrt != 0, s);
    e = force_row_inv<T>(p.nx, R, a, s);
    if (e != hipSuccess) return e;
    const long n = long(p.nx) * p.ny;
    if (p.lb_mrt)
      launch_k((k_lb<T, true>), dim3((n + 255) / 256, 1, c->nrep), dim3(256), 0, s, b);
    else
      launch_k((k_lb<T, false>), dim3((n + 255) / 256, 1, c->nrep), dim3(256), 0, s, b);
    return hipGetLastError();
  }
  return force_col<T>(p.ny, R, a, s);
}

// Average microseconds per launch of one candidate, or a negative value if the
// candidate cannot be launched.
double time_candidate(epdlb_ctx* c, int fam, int R, int nf, int reps) {
  auto launch = [&](hipStream_t s) {
    return c->p.precision == 0 ? launch_family<double>(c, fam, R, nf, s)
                               : launch_family<float>(c, fam, R, nf, s);
  };
  if (launch(c->stream) != hipSuccess) {
    (void)hipGetLastError();
    return -1.0;
  }
  if (hipStreamSynchronize(c->stream) != hipSuccess) return -1.0;
  if (!c->cap_stream && hipStreamCreateWithFlags(&c->cap_stream, hipStreamNonBlocking) != hipSuccess)
    return -1.0;
  if (hipStreamBeginCapture(c->cap_stream, hipStreamCaptureModeRelaxed) != hipSuccess) return -1.0;
  bool ok = true;
  for (int i = 0; i < reps && ok; ++i) ok = launch(c->cap_stream) == hipSuccess;
  hipGraph_t g = nullptr;
  if (hipStreamEndCapture(c->cap_stream, &g) != hipSuccess || !ok || !g) {
    if (g) (void)hipGraphDestroy(g);
    return -1.0;
  }
  hipGraphExec_t ge = nullptr;
  hipError_t e = hipGraphInstantiate(&ge, g, nullptr, nullptr, 0);
  (void)hipGraphDestroy(g);
  if (e != hipSuccess) return -1.0;
  hipEvent_t e0, e1;
  (void)hipEventCreate(&e0);
  (void)hipEventCreate(&e1);
  double best = 1e30;
  (void)hipGraphLaunch(ge, c->stream);  // warm
  for (int t = 0; t < 3; ++t) {
    (void)hipEventRecord(e0, c->stream);
    (void)hipGraphLaunch(ge, c->stream);
    (void)hipEventRecord(e1, c->stream);
    (void)hipEventSynchronize(e1);
    float ms = 0.f;
    (void)hipEventElapsedTime(&ms, e0, e1);
    best = std::min(best, 1e3 * double(ms) / reps);
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  (void)hipGraphExecDestroy(ge);
  return best;
}

void drop_graphs(epdlb_ctx* c) {
  for (auto& g : c->graphs) (void)hipGraphExecDestroy(g.exec);
  c->graphs.clear();
}

std::string tune_key(const epdlb_ctx* c, int fam) {
  char buf[128];
  std::snprintf(buf, sizeof(buf), "gfx950 %d %d %d %d x%d %s", c->p.nx, c->p.ny, c->p.n_contour,
                c->p.precision, c->nrep, kFamilyName[fam]);
  return buf;
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
// FP64 scalars of replica r: zero, except the external-force amplitude.
int reset_scal(epdlb_ctx* c, int r) {
  double sc[kNumScal] = {0};
  sc[kGext] = g_lattice(c->rp[r]);
  const unsigned guard[16] = {0};
  HIPCHK(hipMemcpyAsync(c->base + c->roff(r) + c->L.scal, sc, sizeof(sc), hipMemcpyHostToDevice, c->stream));
  HIPCHK(hipMemcpyAsync(c->base + c->roff(r) + c->L.counters, guard, sizeof(guard), hipMemcpyHostToDevice,
                        c->stream));
  HIPCHK(hipStreamSynchronize(c->stream));
  return EPDLB_OK;
}

// Constant tables of every replica: twiddles, heat-kernel multipliers,
// contour node weights; scalars.
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
  std::vector<double> mx, my, tx, ty;
  mult(p.nx, mx);
  mult(p.ny, my);
  tw(p.nx, tx);
  tw(p.ny, ty);
  for (int r = 0; r < c->nrep; ++r) {
    const size_t o = c->roff(r);
    CHK(upload(c, o + c->L.mult_x, mx.data(), mx.size()));
    CHK(upload(c, o + c->L.mult_y, my.data(), my.size()));
    CHK(upload(c, o + c->L.tw_x, tx.data(), tx.size()));
    CHK(upload(c, o + c->L.tw_y, ty.data(), ty.size()));
    // node weights: trapezoid over each segment, split by its A fraction
    const std::vector<double> a = segment_fractions(c->rp[r]);
    std::vector<double> wA(N + 1, 0.0), wB(N + 1, 0.0);
    for (int j = 0; j < N; ++j) {
      wA[j] += 0.5 * ds * a[j];
      wA[j + 1] += 0.5 * ds * a[j];
      wB[j] += 0.5 * ds * (1.0 - a[j]);
      wB[j + 1] += 0.5 * ds * (1.0 - a[j]);
    }
    CHK(upload(c, o + c->L.wnA, wA.data(), wA.size()));
    CHK(upload(c, o + c->L.wnB, wB.data(), wB.size()));
    CHK(reset_scal(c, r));
  }
  return EPDLB_OK;
}

int compute_stats(epdlb_ctx* c) {
  // twice: the first pass fixes the means, the second evaluates Q_S with them
  for (int k = 0; k < 2; ++k) CHK(c->p.precision == 0 ? stage_stats<double>(c) : stage_stats<float>(c));
  return EPDLB_OK;
}

// Populations live on the device as deviations from the rest weights w_i.
const double kW9[9] = {4.0 / 9, 1.0 / 9, 1.0 / 9, 1.0 / 9, 1.0 / 9, 1.0 / 36, 1.0 / 36, 1.0 / 36, 1.0 / 36};

int upload_populations(epdlb_ctx* c, size_t off, const double* f) {
  const size_t n = size_t(c->p.nx) * c->p.ny;
  std::vector<double> g(9 * n);
  for (int k = 0; k < 9; ++k)
    for (size_t i = 0; i < n; ++i) g[k * n + i] = f[k * n + i] - kW9[k];
  return upload(c, off, g.data(), g.size());
}

// LB of replica r at f^eq(rho = 1, u_init); u_init the analytic
// reverse-Poiseuille profile, into the current population buffer.
int init_lb(epdlb_ctx* c, int r) {
  const epdlb_params& p = c->rp[r];
  const size_t n = size_t(p.nx) * p.ny;
  std::vector<double> ux(p.ny, 0.0);
  if (p.init_flow) {
    const double F0 = g_lattice(p);
    const double nu = lb_nu(p);
    const double Ly = p.ny;
    for (int y = 0; y < p.ny; ++y) {
      const double Y = y + 0.5 - Ly / 2;
      ux[y] = -(F0 / (2 * nu)) * Y * (std::fabs(Y) - Ly / 2);
    }
  }
  static const int cx[9] = {0, 1, 0, -1, 0, 1, -1, -1, 1};
  std::vector<double> f(9 * n), u(2 * n, 0.0), rho(n, 1.0);
  for (int y = 0; y < p.ny; ++y)
    for (int x = 0; x < p.nx; ++x) {
      const size_t i = size_t(y) * p.nx + x;
      const double vx = ux[y];
      u[i] = vx;
      for (int k = 0; k < 9; ++k) {
        const double cu = cx[k] * vx;
        f[k * n + i] = kW9[k] * (1.0 + 3.0 * cu + 4.5 * cu * cu - 1.5 * vx * vx);
      }
    }
  const size_t o = c->roff(r);
  CHK(upload_populations(c, o + c->L.fstar[c->fcur], f.data()));
  CHK(upload(c, o + c->L.u, u.data(), u.size()));
  CHK(upload(c, o + c->L.rho, rho.data(), rho.size()));
  return EPDLB_OK;
}

// New potentials for the replicas whose entry of `omega` is non-null: Phi =
// Phi[omega] (recomputed for the whole group) and their LB restarted.
int set_fields_group(epdlb_ctx* c, const double* const* omega) {
  HIPCHK(hipSetDevice(c->device));
  const size_t n = size_t(c->p.nx) * c->p.ny;
  if (c->track_valid.size() != size_t(c->nrep)) c->track_valid.assign(size_t(c->nrep), 0);
  for (int r = 0; r < c->nrep; ++r) {
    if (!omega[r]) continue;
    CHK(upload(c, c->roff(r) + c->L.omega[c->cur], omega[r], 3 * n));
    CHK(reset_scal(c, r));
    c->track_valid[size_t(r)] = 0;  // a new run for tracking
  }
  CHK(compute_stats(c));
  CHK(c->p.precision == 0 ? stage_densities<double>(c, false) : stage_densities<float>(c, false));
  for (int r = 0; r < c->nrep; ++r)
    if (omega[r]) CHK(init_lb(c, r));
  HIPCHK(hipStreamSynchronize(c->stream));
  c->seeded = true;
  if (c->p.density_mode == 1) CHK(nn_after_seed(c));
  return EPDLB_OK;
}

int run_sur_step(epdlb_ctx* c, int kind);

// Capture `steps` hybrid steps from the current buffer parity into a graph.
// kind 0: exact densities; 1..4: surrogate-mode steps (see run_sur_step).
int get_graph(epdlb_ctx* c, int steps, int kind, hipGraphExec_t* out) {
  for (auto& g : c->graphs)
    if (g.steps == steps && g.cur == c->cur && g.fcur == c->fcur && g.kind == kind) {
      *out = g.exec;
      return EPDLB_OK;
    }
  if (!c->cap_stream) HIPCHK(hipStreamCreateWithFlags(&c->cap_stream, hipStreamNonBlocking));
  const int cur0 = c->cur, fcur0 = c->fcur;
  const bool prof0 = c->prof_on;
  hipStream_t user = c->stream;
  c->stream = c->cap_stream;
  c->prof_on = false;
  HIPCHK(hipStreamBeginCapture(c->cap_stream, hipStreamCaptureModeRelaxed));
  int r = EPDLB_OK;
  for (int s = 0; s < steps && r == EPDLB_OK; ++s) {
    if (kind == 0) {
      for (int st = EPDLB_STAGE_ADVECT_UPDATE; st <= EPDLB_STAGE_DENSITIES && r == EPDLB_OK; ++st) r = run_stage(c, st);
      if (r == EPDLB_OK) r = run_force_lb(c);
    } else {
      r = run_sur_step(c, kind);
    }
  }
  hipGraph_t graph = nullptr;
  hipError_t e = hipStreamEndCapture(c->cap_stream, &graph);
  c->stream = user;
  c->prof_on = prof0;
  c->cur = cur0;
  c->fcur = fcur0;
  if (r != EPDLB_OK) {
    if (graph) (void)hipGraphDestroy(graph);
    return r;
  }
  HIPCHK(e);
  hipGraphExec_t exec = nullptr;
  e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
  (void)hipGraphDestroy(graph);
  HIPCHK(e);
  c->graphs.push_back({steps, cur0, fcur0, kind, exec});
  *out = exec;
  return EPDLB_OK;
}

// Default launch shapes (R = 8 values per lane).  Row passes: nf transforms of
// L/R lanes per block (<= 256 lanes); column passes: NF transforms
// interleaved, NF*L/R <= 512 lanes, NF = 8 where it fits.
void default_shapes(epdlb_ctx* c) {
  const epdlb_params* p = &c->p;
  auto row_nf = [&](int L, int transforms) {
    const int tl = L / 8;
    return clampi(256 / tl, 1, transforms);
  };
  auto col_nf = [&](int L) { return (L / 8) * 8 <= 512 ? 8 : 4; };
  c->sh_row = {8, row_nf(p->nx, p->ny / 2)};
  c->sh_col = {8, p->precision == 0 ? 4 : col_nf(p->ny)};
  c->sh_frow = {8, row_nf(p->nx, p->ny)};
  c->sh_fcol = {8, p->precision == 0 ? 4 : col_nf(p->ny)};
}

int check_finite(epdlb_ctx* c) {
  for (int r = 0; r < c->nrep; ++r) {
    double s[kNumScal];
    unsigned g[kNumGuard];
    HIPCHK(hipMemcpyAsync(s, c->base + c->roff(r) + c->L.scal, sizeof(s), hipMemcpyDeviceToHost, c->stream));
    HIPCHK(hipMemcpyAsync(g, c->base + c->roff(r) + c->L.counters, sizeof(g), hipMemcpyDeviceToHost, c->stream));
    HIPCHK(hipStreamSynchronize(c->stream));
    const std::string who = c->nrep > 1 ? " (replica " + std::to_string(r) + " of its group)" : "";
    for (int i = 0; i < kNumScal; ++i)
      if (!std::isfinite(s[i])) return fail(EPDLB_ENONFINITE, "non-finite partition function or field mean" + who);
    if (g[kGuardNonFinite]) return fail(EPDLB_ENONFINITE, "non-finite LB density or velocity" + who);
    if (g[kGuardMach]) return fail(EPDLB_EUNSTABLE, "LB flow speed above mach_max times the speed of sound" + who);
    if (g[kGuardNegative]) return fail(EPDLB_EUNSTABLE, "negative LB population" + who);
  }
  return EPDLB_OK;
}

}  // namespace

#include "nn_host.hpp"

// ---------------------------------------------------------------------------
// Batched replicas: replicas of one grid shape form a group that shares every
// launch (blockIdx.z = replica); groups are independent branches of one
// captured graph per step pair, forked from and joined to the batch stream.
// ---------------------------------------------------------------------------
struct epdlb_batch {
  int device = 0;
  hipStream_t stream = nullptr;
  bool own_stream = false;
  std::vector<epdlb_ctx*> groups;
  std::vector<std::pair<int, int>> where;  // replica -> (group, index in group)
  struct G {
    int steps;
    hipGraphExec_t exec;
  };
  std::vector<G> graphs;
  hipStream_t cap = nullptr;
  std::vector<hipStream_t> fork;
  hipEvent_t ev_fork = nullptr;
  std::vector<hipEvent_t> ev_join;
  int64_t nstep = 0;
  bool seeded = false;
  bool prof = false;  // profiling: stream launches, group after group
};

namespace {

bool same_model(const epdlb_params& a, const epdlb_params& b) {
  return a.n_contour == b.n_contour && a.phi_P == b.phi_P && a.chi_AB == b.chi_AB && a.chi_AS == b.chi_AS &&
         a.chi_BS == b.chi_BS && a.kappa_H == b.kappa_H && a.D_S == b.D_S && a.D_A == b.D_A &&
         a.D_B == b.D_B && a.R_G == b.R_G && a.dx == b.dx && a.dt == b.dt && a.kT_over_v == b.kT_over_v &&
         a.lb_tau == b.lb_tau && a.g_units == b.g_units && a.precision == b.precision &&
         a.init_flow == b.init_flow && a.couple_lb == b.couple_lb && a.lb_mrt == b.lb_mrt &&
         a.lb_gamma_s == b.lb_gamma_s && a.lb_gamma_b == b.lb_gamma_b && a.lb_gamma_g == b.lb_gamma_g &&
         a.mach_max == b.mach_max;
}

// A group context over `rp` (same grid shape), arena allocated here.
int make_group(const std::vector<epdlb_params>& rp, int device, epdlb_ctx** out) {
  epdlb_ctx* c = new (std::nothrow) epdlb_ctx();
  if (!c) return fail(EPDLB_ENOMEM, "host allocation failed");
  c->p = rp[0];
  c->rp = rp;
  c->nrep = int(rp.size());
  c->device = device;
  if (const char* env = std::getenv("EPDLB_GRAPH")) c->use_graph = std::atoi(env) != 0;
  if (const char* env = std::getenv("EPDLB_SUR_GRAPH")) c->sur_graph = std::atoi(env) != 0;
  c->L = make_layout(c->p);
  c->rstride = c->L.total;
  if (hipStreamCreateWithFlags(&c->stream, hipStreamNonBlocking) != hipSuccess) {
    delete c;
    return fail(EPDLB_EHIP, "hipStreamCreate failed");
  }
  c->own_stream = true;
  void* m = nullptr;
  if (hipMalloc(&m, c->rstride * c->nrep) != hipSuccess) {
    epdlb_destroy(c);
    return fail(EPDLB_ENOMEM, "hipMalloc of a replica group arena failed");
  }
  c->base = static_cast<unsigned char*>(m);
  c->own_mem = true;
  default_shapes(c);
  const int r = upload_tables(c);
  if (r != EPDLB_OK) {
    epdlb_destroy(c);
    return r;
  }
  *out = c;
  return EPDLB_OK;
}

void drop_batch_graphs(epdlb_batch* b) {
  for (auto& g : b->graphs) (void)hipGraphExecDestroy(g.exec);
  b->graphs.clear();
}

// One graph of `steps` steps of every group, groups as parallel branches.
int batch_graph(epdlb_batch* b, int steps, hipGraphExec_t* out) {
  for (auto& g : b->graphs)
    if (g.steps == steps) {
      *out = g.exec;
      return EPDLB_OK;
    }
  const size_t G = b->groups.size();
  if (!b->cap) {
    HIPCHK(hipStreamCreateWithFlags(&b->cap, hipStreamNonBlocking));
    HIPCHK(hipEventCreateWithFlags(&b->ev_fork, hipEventDisableTiming));
    b->fork.resize(G);
    b->ev_join.resize(G);
    for (size_t i = 0; i < G; ++i) {
      HIPCHK(hipStreamCreateWithFlags(&b->fork[i], hipStreamNonBlocking));
      HIPCHK(hipEventCreateWithFlags(&b->ev_join[i], hipEventDisableTiming));
    }
  }
  std::vector<int> cur0(G), fcur0(G);
  std::vector<hipStream_t> own(G);
  for (size_t i = 0; i < G; ++i) {
    cur0[i] = b->groups[i]->cur;
    fcur0[i] = b->groups[i]->fcur;
    own[i] = b->groups[i]->stream;
    b->groups[i]->stream = b->fork[i];
    b->groups[i]->prof_on = false;
  }
  HIPCHK(hipStreamBeginCapture(b->cap, hipStreamCaptureModeRelaxed));
  int r = EPDLB_OK;
  if (hipEventRecord(b->ev_fork, b->cap) != hipSuccess) r = fail(EPDLB_EHIP, "fork event");
  for (size_t i = 0; i < G && r == EPDLB_OK; ++i) {
    epdlb_ctx* c = b->groups[i];
    if (hipStreamWaitEvent(b->fork[i], b->ev_fork, 0) != hipSuccess) r = fail(EPDLB_EHIP, "fork wait");
    for (int st = 0; st < steps && r == EPDLB_OK; ++st) {
      for (int k = EPDLB_STAGE_ADVECT_UPDATE; k <= EPDLB_STAGE_DENSITIES && r == EPDLB_OK; ++k) r = run_stage(c, k);
      if (r == EPDLB_OK) r = run_force_lb(c);
    }
    if (r == EPDLB_OK && hipEventRecord(b->ev_join[i], b->fork[i]) != hipSuccess) r = fail(EPDLB_EHIP, "join");
    if (r == EPDLB_OK && hipStreamWaitEvent(b->cap, b->ev_join[i], 0) != hipSuccess)
      r = fail(EPDLB_EHIP, "join wait");
  }
  hipGraph_t graph = nullptr;
  const hipError_t e = hipStreamEndCapture(b->cap, &graph);
  for (size_t i = 0; i < G; ++i) {
    b->groups[i]->stream = own[i];
    b->groups[i]->cur = cur0[i];
    b->groups[i]->fcur = fcur0[i];
  }
  if (r != EPDLB_OK) {
    if (graph) (void)hipGraphDestroy(graph);
    return r;
  }
  HIPCHK(e);
  hipGraphExec_t exec = nullptr;
  const hipError_t e2 = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
  (void)hipGraphDestroy(graph);
  HIPCHK(e2);
  b->graphs.push_back({steps, exec});
  *out = exec;
  return EPDLB_OK;
}

int batch_replica(epdlb_batch* b, int32_t r, epdlb_ctx** c, int* idx) {
  if (!b || r < 0 || size_t(r) >= b->where.size()) return fail(EPDLB_EINVAL, "bad batch or replica index");
  *c = b->groups[b->where[r].first];
  *idx = b->where[r].second;
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
  p->density_mode = 0;
  p->fallback_every = 50;
  p->check_every = 10;
  p->resid_tol = 1e-3;
  p->err_tol = 1e-3;
  p->lb_mrt = 0;
  p->lb_gamma_s = p->lb_gamma_b = p->lb_gamma_g = 0.0;
  p->cg_invert = 0;
  p->cg_max_iter = 1000;
  p->cg_tol = 1e-8;
  p->cg_precond = 0;
  p->mach_max = 0.5;
  return EPDLB_OK;
}

int epdlb_validate(const epdlb_params* p) { return validate(p); }

int epdlb_mrt_gammas(double eta, double eta_B, double rho, double dx, double dt, int32_t dim,
                     double* gamma_s, double* gamma_b) {
  if (!gamma_s || !gamma_b) return fail(EPDLB_EINVAL, "NULL output");
  if (dim != 2 && dim != 3) return fail(EPDLB_EINVAL, "dim must be 2 or 3");
  const double v[5] = {eta, eta_B, rho, dx, dt};
  for (double x : v)
    if (!(x > 0.0) || !std::isfinite(x)) return fail(EPDLB_EINVAL, "eta, eta_B, rho, dx, dt must be finite and > 0");
  // eta = (dt rho cs2 / 2) (1 + g)/(1 - g)  <=>  g = (a - 1)/(a + 1), a = 2 eta/(dt rho cs2)
  const double cs2 = dx * dx / (3.0 * dt * dt);
  const double a = 2.0 * eta / (dt * rho * cs2);
  const double b = double(dim) * eta_B / (dt * rho * cs2);
  *gamma_s = (a - 1.0) / (a + 1.0);
  *gamma_b = (b - 1.0) / (b + 1.0);
  return EPDLB_OK;
}

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
  device_cus();
  epdlb_ctx* c = new (std::nothrow) epdlb_ctx();
  if (!c) return fail(EPDLB_ENOMEM, "host allocation failed");
  c->p = *p;
  c->rp.assign(1, *p);
  c->nrep = 1;
  c->device = device;
  if (const char* env = std::getenv("EPDLB_GRAPH")) c->use_graph = std::atoi(env) != 0;
  if (const char* env = std::getenv("EPDLB_SUR_GRAPH")) c->sur_graph = std::atoi(env) != 0;
  c->L = make_layout(*p);
  c->rstride = c->L.total;
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
  default_shapes(c);
  if (p->cg_invert == 1 && ensure_cg(c) != EPDLB_OK) {
    epdlb_destroy(c);
    return fail(EPDLB_ENOMEM, "inversion scratch allocation failed");
  }
  if (p->density_mode == 1) {
    if (hipHostMalloc(reinterpret_cast<void**>(&c->snap), 3 * sizeof(double), hipHostMallocDefault) != hipSuccess ||
        hipEventCreateWithFlags(&c->snap_ev, hipEventDisableTiming) != hipSuccess) {
      epdlb_destroy(c);
      return fail(EPDLB_ENOMEM, "pinned host buffer or event for the residual test failed");
    }
  }
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
  c->cur = 0;
  c->fcur = 0;
  CHK(set_fields_group(c, &omega));
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
  CHK(upload_populations(c, c->L.fstar[0], fstar));
  CHK(upload(c, c->L.u, u, 2 * n));
  CHK(reset_scal(c, 0));
  CHK(compute_stats(c));
  HIPCHK(hipStreamSynchronize(c->stream));
  c->seeded = true;
  c->nstep = 0;
  if (c->p.density_mode == 1) CHK(nn_after_seed(c));
  return EPDLB_OK;
}

int epdlb_get_state(epdlb_ctx* c, double* omega, double* phi, double* fstar, double* u) {
  if (!c || !omega || !phi || !fstar || !u) return fail(EPDLB_EINVAL, "NULL argument");
  if (!c->seeded) return fail(EPDLB_ESTATE, "no state before seed/set_fields/set_state");
  const size_t n = size_t(c->p.nx) * c->p.ny;
  CHK(download(c, c->L.omega[c->cur], omega, 3 * n));
  CHK(download(c, c->L.phi, phi, 3 * n));
  CHK(epdlb_read_populations(c, fstar));
  CHK(download(c, c->L.u, u, 2 * n));
  return EPDLB_OK;
}

int epdlb_device_views(epdlb_ctx* c, epdlb_dev_views* v) {
  if (!c || !v) return fail(EPDLB_EINVAL, "NULL argument");
  v->precision = c->p.precision;
  v->plane = int64_t(c->p.nx) * c->p.ny;
  v->omega = c->base + c->L.omega[c->cur];
  v->phi = c->base + c->L.phi;
  v->rho = c->base + c->L.rho;
  v->u = c->base + c->L.u;
  return EPDLB_OK;
}

int epdlb_step(epdlb_ctx* c, int64_t n) {
  if (!c) return fail(EPDLB_EINVAL, "ctx is NULL");
  if (!c->seeded) return fail(EPDLB_ESTATE, "step before seed/set_fields/set_state");
  if (n < 0) return fail(EPDLB_EINVAL, "negative step count");
  HIPCHK(hipSetDevice(c->device));
  if (c->p.density_mode == 1) {
    if (!c->nn_ready) return fail(EPDLB_ESTATE, "surrogate mode: weights not loaded (epdlb_surrogate_set_weights)");
    for (int64_t s = 0; s < n; ++s) {
      const bool exact = c->force_exact || c->nstep % c->p.fallback_every == 0 ||
                         (c->p.err_tol > 0.0 && !c->validated);
      const int kind = (exact ? 3 : 1) + (c->last_exact ? 1 : 0);
      if (c->use_graph && c->sur_graph && !c->prof_on) {
        hipGraphExec_t g;
        CHK(get_graph(c, 1, kind, &g));
        HIPCHK(hipGraphLaunch(g, c->stream));
        c->cur = 1 - c->cur;
        c->fcur = 1 - c->fcur;
      } else {
        CHK(run_sur_step(c, kind));
      }
      if (exact) {
        ++c->n_exact;
        c->force_exact = false;
      }
      c->last_exact = exact;
      ++c->nstep;
      if (c->nstep % c->p.check_every == 0) CHK(nn_check(c));
    }
    return EPDLB_OK;
  }
  // the inversion decides its iteration count on the host: no graphs
  if (c->use_graph && !c->prof_on && !c->p.cg_invert) {
    // replay captured two-step graphs (buffer parity returns to its start),
    // then a one-step graph for an odd remainder
    while (n > 0) {
      const int k = n >= 2 ? 2 : 1;
      hipGraphExec_t g;
      CHK(get_graph(c, k, 0, &g));
      HIPCHK(hipGraphLaunch(g, c->stream));
      if (k == 1) {
        c->cur = 1 - c->cur;
        c->fcur = 1 - c->fcur;
      }
      c->nstep += k;
      n -= k;
    }
    return EPDLB_OK;
  }
  for (int64_t s = 0; s < n; ++s) {
    for (int st = EPDLB_STAGE_ADVECT_UPDATE; st <= EPDLB_STAGE_DENSITIES; ++st) CHK(run_stage(c, st));
    CHK(run_force_lb(c));
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
  const size_t n = size_t(c->p.nx) * c->p.ny;
  CHK(download(c, c->L.fstar[c->fcur], f, 9 * n));
  for (int k = 0; k < 9; ++k)
    for (size_t i = 0; i < n; ++i) f[k * n + i] += kW9[k];
  return EPDLB_OK;
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

}  // extern "C"

// ---------------------------------------------------------------------------
// Observables (Sec. III, IV)
// ---------------------------------------------------------------------------
namespace {

// Scratch layout: labels, areas, wrap flags, counter (int32), per-site sums
// (6 doubles), particle list (n/2 + 1 entries), block partials.
struct ObsLayout {
  size_t labels, area, wrap, count, sums, list, part, ov, prev, total;
  int cap, nblocks;
};
ObsLayout obs_layout(long n, int nrep) {
  auto up = [](size_t v) { return (v + 255) & ~size_t(255); };
  ObsLayout o{};
  o.nblocks = int((n + 255) / 256);
  o.cap = int(n / 2 + 1);
  size_t off = 0;
  o.labels = off; off = up(off + 4 * size_t(n));
  o.area = off; off = up(off + 4 * size_t(n));
  o.wrap = off; off = up(off + 4 * size_t(n));
  o.count = off; off = up(off + 4);
  o.sums = off; off = up(off + 48 * size_t(n));
  o.list = off; off = up(off + sizeof(obs::Particle) * size_t(o.cap));
  o.part = off; off = up(off + 16 * size_t(o.nblocks));
  o.ov = off; off = up(off + 4 * size_t(n));
  o.prev = off; off = up(off + size_t(n) * size_t(nrep));
  o.total = off;
  return o;
}

// Observables of replica r of the context.  track: also mark each particle
// new (born) unless it covers a particle site of the replica's previous
// tracking sample, then keep this sample's particle sites.  all (may be
// null) receives every particle in label order.
template <typename T>
int observables_t(epdlb_ctx* c, int r, double thr, epdlb_obs* out, epdlb_particle* particles, int max_particles,
                  int32_t* labels, bool track = false, std::vector<obs::Particle>* all = nullptr) {
  const epdlb_params& p = c->rp[size_t(r)];
  const long n = long(p.nx) * p.ny;
  const ObsLayout o = obs_layout(n, c->nrep);
  if (c->track_valid.size() != size_t(c->nrep)) c->track_valid.assign(size_t(c->nrep), 0);
  if (!c->obs) {
    void* m = nullptr;
    if (hipMalloc(&m, o.total) != hipSuccess) return fail(EPDLB_ENOMEM, "observables scratch allocation failed");
    c->obs = static_cast<unsigned char*>(m);
  }
  unsigned char* b = c->obs;
  int* L = reinterpret_cast<int*>(b + o.labels);
  int* area = reinterpret_cast<int*>(b + o.area);
  int* wrap = reinterpret_cast<int*>(b + o.wrap);
  int* count = reinterpret_cast<int*>(b + o.count);
  double* sums = reinterpret_cast<double*>(b + o.sums);
  obs::Particle* list = reinterpret_cast<obs::Particle*>(b + o.list);
  double* part = reinterpret_cast<double*>(b + o.part);
  int* ov = track ? reinterpret_cast<int*>(b + o.ov) : nullptr;
  unsigned char* prev = b + o.prev + size_t(r) * size_t(n);
  const T* phi = c->ptr<T>(c->roff(r) + c->L.phi);
  hipStream_t s = c->stream;
  const dim3 grid(unsigned(o.nblocks)), blk(256);
  hipLaunchKernelGGL(obs::k_obs_init<T>, grid, blk, 0, s, phi, n, p.nx, p.ny, thr, p.phi_P, L, part, area, wrap, sums,
                     count, ov);
  hipLaunchKernelGGL(obs::k_ccl_merge, grid, blk, 0, s, L, n, p.nx, p.ny);
  hipLaunchKernelGGL(obs::k_ccl_compress, grid, blk, 0, s, L, n);
  if (track && c->track_valid[size_t(r)])
    hipLaunchKernelGGL(obs::k_overlap, grid, blk, 0, s, (const int*)L, (const unsigned char*)prev, ov, n);
  hipLaunchKernelGGL(obs::k_particle_accum<T>, grid, blk, 0, s, phi, (const int*)L, n, p.nx, p.ny, area, sums, wrap);
  hipLaunchKernelGGL(obs::k_particle_list, grid, blk, 0, s, (const int*)L, (const int*)area, (const double*)sums,
                     (const int*)wrap, (const int*)ov, n, p.nx, p.ny, count, list, o.cap);
  if (track) hipLaunchKernelGGL(obs::k_store_prev, grid, blk, 0, s, (const int*)L, prev, n);
  HIPCHK(hipGetLastError());
  std::vector<double> hp(2 * size_t(o.nblocks));
  int cnt = 0;
  HIPCHK(hipMemcpyAsync(hp.data(), part, hp.size() * sizeof(double), hipMemcpyDeviceToHost, s));
  HIPCHK(hipMemcpyAsync(&cnt, count, 4, hipMemcpyDeviceToHost, s));
  if (labels) HIPCHK(hipMemcpyAsync(labels, L, 4 * size_t(n), hipMemcpyDeviceToHost, s));
  HIPCHK(hipStreamSynchronize(s));
  if (cnt < 0 || cnt > o.cap) return fail(EPDLB_EHIP, "particle count out of range");
  std::vector<obs::Particle> hl(static_cast<size_t>(cnt));
  if (cnt) {
    HIPCHK(hipMemcpyAsync(hl.data(), list, sizeof(obs::Particle) * size_t(cnt), hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
  }
  std::sort(hl.begin(), hl.end(), [](const obs::Particle& x, const obs::Particle& y) { return x.label < y.label; });
  // block partials in block order: deterministic sums
  double ssum = 0.0, msum = 0.0;
  for (int k = 0; k < o.nblocks; ++k) {
    ssum += hp[2 * size_t(k)];
    msum += hp[2 * size_t(k) + 1];
  }
  const double ny = p.ny;
  const double y2sum = (ny * ny * ny - ny) / 12.0;  // sum over rows of (row + 1/2 - ny/2)^2
  out->sigma = ssum / double(n);
  out->y2p = std::sqrt(msum / (double(p.nx) * p.phi_P * y2sum));
  out->n_particles = cnt;
  int nw = 0;
  for (const auto& q : hl) nw += q.wraps ? 1 : 0;
  out->n_wrapping = nw;
  const int m = std::min(cnt, max_particles);
  for (int k = 0; k < m; ++k) {
    const obs::Particle& q = hl[size_t(k)];
    epdlb_particle& r = particles[k];
    r.label = q.label;
    r.area = q.area;
    r.wraps = q.wraps;
    r.born = q.born;
    r.content = q.content;
    r.cx = q.cx;
    r.cy = q.cy;
    r.gxx = q.gxx;
    r.gxy = q.gxy;
    r.gyy = q.gyy;
    r.R = q.R;
    r.c_rel = q.c_rel;
  }
  if (track) c->track_valid[size_t(r)] = 1;
  if (all) *all = std::move(hl);
  return EPDLB_OK;
}

// Observables of replica r with tracking; the new particles go to events.
int track_replica(epdlb_ctx* c, int r, double threshold, epdlb_obs* out, epdlb_particle* events, int max_events,
                  int32_t* n_events) {
  if (!out || !n_events) return fail(EPDLB_EINVAL, "NULL argument");
  if (max_events < 0 || (max_events > 0 && !events)) return fail(EPDLB_EINVAL, "bad event array");
  if (!std::isfinite(threshold)) return fail(EPDLB_EINVAL, "non-finite threshold");
  HIPCHK(hipSetDevice(c->device));
  std::vector<obs::Particle> all;
  CHK(c->p.precision == 0 ? observables_t<double>(c, r, threshold, out, nullptr, 0, nullptr, true, &all)
                          : observables_t<float>(c, r, threshold, out, nullptr, 0, nullptr, true, &all));
  int k = 0;
  for (const obs::Particle& q : all) {
    if (!q.born) continue;
    if (k < max_events) {
      epdlb_particle& e = events[k];
      e.label = q.label;
      e.area = q.area;
      e.wraps = q.wraps;
      e.born = 1;
      e.content = q.content;
      e.cx = q.cx;
      e.cy = q.cy;
      e.gxx = q.gxx;
      e.gxy = q.gxy;
      e.gyy = q.gyy;
      e.R = q.R;
      e.c_rel = q.c_rel;
    }
    ++k;
  }
  *n_events = k;
  return EPDLB_OK;
}

// sigma_Delta of the current densities of two contexts: per-block partial
// sums into part (device, 2 doubles per 256 sites), copied to hp (host, same
// size) and added there in block order.
template <typename T>
int sigma_delta_core(epdlb_ctx* a, epdlb_ctx* b, double* part, double* hp, double* out) {
  const long n = long(a->p.nx) * a->p.ny;
  const int nblocks = int((n + 255) / 256);
  HIPCHK(hipStreamSynchronize(b->stream));
  hipLaunchKernelGGL(obs::k_sigma_delta<T>, dim3(unsigned(nblocks)), dim3(256), 0, a->stream,
                     (const T*)a->ptr<T>(a->L.phi), (const T*)b->ptr<T>(b->L.phi), n, part);
  hipError_t e = hipGetLastError();
  if (e == hipSuccess) e = hipMemcpyAsync(hp, part, 2 * size_t(nblocks) * sizeof(double), hipMemcpyDeviceToHost,
                                          a->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(a->stream);
  if (e != hipSuccess) return fail(EPDLB_EHIP, std::string("sigma_delta: ") + hipGetErrorString(e));
  double sum = 0.0;
  for (int k = 0; k < nblocks; ++k) sum += hp[2 * size_t(k)];
  *out = sum / double(n);
  return EPDLB_OK;
}

template <typename T>
int sigma_delta_t(epdlb_ctx* a, epdlb_ctx* b, double* out) {
  const long n = long(a->p.nx) * a->p.ny;
  const int nblocks = int((n + 255) / 256);
  void* m = nullptr;
  if (hipMalloc(&m, 16 * size_t(nblocks)) != hipSuccess) return fail(EPDLB_ENOMEM, "sigma_delta scratch allocation failed");
  std::vector<double> hp(2 * size_t(nblocks));
  const int r = sigma_delta_core<T>(a, b, static_cast<double*>(m), hp.data(), out);
  (void)hipFree(m);
  return r;
}

}  // namespace

extern "C" {

int epdlb_observables(epdlb_ctx* c, double threshold, epdlb_obs* out, epdlb_particle* particles,
                      int32_t max_particles, int32_t* labels) {
  if (!c || !out) return fail(EPDLB_EINVAL, "NULL argument");
  if (max_particles < 0 || (max_particles > 0 && !particles)) return fail(EPDLB_EINVAL, "bad particle array");
  if (!std::isfinite(threshold)) return fail(EPDLB_EINVAL, "non-finite threshold");
  if (!c->seeded) return fail(EPDLB_ESTATE, "no state before seed/set_fields/set_state");
  HIPCHK(hipSetDevice(c->device));
  return c->p.precision == 0 ? observables_t<double>(c, 0, threshold, out, particles, max_particles, labels)
                             : observables_t<float>(c, 0, threshold, out, particles, max_particles, labels);
}

int epdlb_track_particles(epdlb_ctx* c, double threshold, epdlb_obs* out, epdlb_particle* events,
                          int32_t max_events, int32_t* n_events) {
  if (!c) return fail(EPDLB_EINVAL, "NULL argument");
  if (!c->seeded) return fail(EPDLB_ESTATE, "no state before seed/set_fields/set_state");
  return track_replica(c, 0, threshold, out, events, max_events, n_events);
}

int epdlb_track_reset(epdlb_ctx* c) {
  if (!c) return fail(EPDLB_EINVAL, "ctx is NULL");
  c->track_valid.assign(size_t(c->nrep), 0);
  return EPDLB_OK;
}

int epdlb_batch_observables(epdlb_batch* b, int32_t replica, double threshold, epdlb_obs* out,
                            epdlb_particle* particles, int32_t max_particles, int32_t* labels) {
  epdlb_ctx* c;
  int i;
  CHK(batch_replica(b, replica, &c, &i));
  if (!out) return fail(EPDLB_EINVAL, "NULL argument");
  if (max_particles < 0 || (max_particles > 0 && !particles)) return fail(EPDLB_EINVAL, "bad particle array");
  if (!std::isfinite(threshold)) return fail(EPDLB_EINVAL, "non-finite threshold");
  if (!c->seeded) return fail(EPDLB_ESTATE, "no state before seed/set_fields");
  HIPCHK(hipSetDevice(c->device));
  HIPCHK(hipStreamSynchronize(b->stream));
  return c->p.precision == 0 ? observables_t<double>(c, i, threshold, out, particles, max_particles, labels)
                             : observables_t<float>(c, i, threshold, out, particles, max_particles, labels);
}

int epdlb_batch_track_particles(epdlb_batch* b, int32_t replica, double threshold, epdlb_obs* out,
                                epdlb_particle* events, int32_t max_events, int32_t* n_events) {
  epdlb_ctx* c;
  int i;
  CHK(batch_replica(b, replica, &c, &i));
  if (!c->seeded) return fail(EPDLB_ESTATE, "no state before seed/set_fields");
  HIPCHK(hipSetDevice(c->device));
  HIPCHK(hipStreamSynchronize(b->stream));
  return track_replica(c, i, threshold, out, events, max_events, n_events);
}

int epdlb_batch_track_reset(epdlb_batch* b, int32_t replica) {
  epdlb_ctx* c;
  int i;
  CHK(batch_replica(b, replica, &c, &i));
  if (c->track_valid.size() != size_t(c->nrep)) c->track_valid.assign(size_t(c->nrep), 0);
  c->track_valid[size_t(i)] = 0;
  return EPDLB_OK;
}

int epdlb_sigma_delta(epdlb_ctx* a, epdlb_ctx* b, double* out) {
  if (!a || !b || !out) return fail(EPDLB_EINVAL, "NULL argument");
  if (a->device != b->device || a->p.nx != b->p.nx || a->p.ny != b->p.ny || a->p.precision != b->p.precision)
    return fail(EPDLB_EINVAL, "sigma_delta needs two contexts on one device with the same grid and precision");
  if (!a->seeded || !b->seeded) return fail(EPDLB_ESTATE, "no state before seed/set_fields/set_state");
  HIPCHK(hipSetDevice(a->device));
  return a->p.precision == 0 ? sigma_delta_t<double>(a, b, out) : sigma_delta_t<float>(a, b, out);
}

}  // extern "C"

namespace {

constexpr int kNoAllocMaxDevices = 64;
std::mutex g_noalloc_mu;
void* g_noalloc_ptr[kNoAllocMaxDevices] = {nullptr};

// Device address of `scratch` on the current device `dev`, looked up once per
// device with that device current.
int noalloc_scratch(int dev, double** out) {
  if (dev < 0 || dev >= kNoAllocMaxDevices) return fail(EPDLB_EINVAL, "device index above the no-allocation table");
  std::lock_guard<std::mutex> lock(g_noalloc_mu);
  if (!g_noalloc_ptr[dev]) {
    void* ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !ptr)
      return fail(EPDLB_EHIP, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
    g_noalloc_ptr[dev] = ptr;
  }
  *out = static_cast<double*>(g_noalloc_ptr[dev]);
  return EPDLB_OK;
}

}  // namespace

extern "C" {

int epdlb_sigma_delta_noalloc(epdlb_ctx* a, epdlb_ctx* b, double* out) {
  if (!a || !b || !out) return fail(EPDLB_EINVAL, "NULL argument");
  if (a->device != b->device || a->p.nx != b->p.nx || a->p.ny != b->p.ny || a->p.precision != b->p.precision)
    return fail(EPDLB_EINVAL, "sigma_delta needs two contexts on one device with the same grid and precision");
  if (!a->seeded || !b->seeded) return fail(EPDLB_ESTATE, "no state before seed/set_fields/set_state");
  const long n = long(a->p.nx) * a->p.ny;
  if (n > kNoAllocMaxSites)
    return fail(EPDLB_EINVAL, "grid above the no-allocation limit of " + std::to_string(kNoAllocMaxSites) + " sites");
  HIPCHK(hipSetDevice(a->device));
  double* part = nullptr;
  CHK(noalloc_scratch(a->device, &part));
  double* total = part + 2 * kNoAllocMaxBlocks;
  const int nblocks = int((n + 255) / 256);
  HIPCHK(hipStreamSynchronize(b->stream));
  if (a->p.precision == 0)
    hipLaunchKernelGGL(obs::k_sigma_delta<double>, dim3(unsigned(nblocks)), dim3(256), 0, a->stream,
                       (const double*)a->ptr<double>(a->L.phi), (const double*)b->ptr<double>(b->L.phi), n, part);
  else
    hipLaunchKernelGGL(obs::k_sigma_delta<float>, dim3(unsigned(nblocks)), dim3(256), 0, a->stream,
                       (const float*)a->ptr<float>(a->L.phi), (const float*)b->ptr<float>(b->L.phi), n, part);
  HIPCHK(hipGetLastError());
  // the same block-order total as the host loop of epdlb_sigma_delta
  hipLaunchKernelGGL(obs::k_sum_pairs_in_order, dim3(1), dim3(256), 0, a->stream, (const double*)part, nblocks,
                     total);
  HIPCHK(hipGetLastError());
  double sum = 0.0;
  HIPCHK(hipMemcpyAsync(&sum, total, sizeof(double), hipMemcpyDeviceToHost, a->stream));
  HIPCHK(hipStreamSynchronize(a->stream));
  *out = sum / double(n);
  return EPDLB_OK;
}

int epdlb_invert_densities(epdlb_ctx* c, const double* phi_target, int32_t max_iter, double tol,
                           epdlb_cg_info* info) {
  if (!c || !phi_target) return fail(EPDLB_EINVAL, "ctx or phi_target is NULL");
  if (!c->seeded) return fail(EPDLB_ESTATE, "inversion before seed/set_fields/set_state");
  if (c->nrep != 1) return fail(EPDLB_EINVAL, "inversion of a batch replica group is not supported");
  if (c->p.density_mode != 0) return fail(EPDLB_EINVAL, "inversion needs exact densities (density_mode 0)");
  if (max_iter < 0 || max_iter > 1000000 || !(tol > 0.0) || !std::isfinite(tol))
    return fail(EPDLB_EINVAL, "max_iter must be in [0, 1e6] and tol > 0");
  HIPCHK(hipSetDevice(c->device));
  CHK(ensure_cg(c));
  const size_t n = size_t(c->p.nx) * c->p.ny;
  for (size_t i = 0; i < 3 * n; ++i)
    if (!std::isfinite(phi_target[i]) || !(phi_target[i] > 0.0))
      return fail(EPDLB_EINVAL, "phi_target must be finite and positive");
  auto run = [&](auto tag) -> int {
    using T = decltype(tag);
    T* tgt = cg_set<T>(c, CG_TARGET);
    T* x = cg_set<T>(c, CG_X);
    T* w = c->ptr<T>(c->L.omega[c->cur]);
    std::vector<T> tmp(3 * n);
    for (size_t i = 0; i < 3 * n; ++i) tmp[i] = T(phi_target[i]);
    HIPCHK(hipMemcpyAsync(tgt, tmp.data(), 3 * n * sizeof(T), hipMemcpyHostToDevice, c->stream));
    HIPCHK(hipMemcpyAsync(x, w, 3 * n * sizeof(T), hipMemcpyDeviceToDevice, c->stream));
    epdlb_cg_info r;
    CHK(cg_invert<T>(c, tol, max_iter, &r));
    HIPCHK(hipMemcpyAsync(w, x, 3 * n * sizeof(T), hipMemcpyDeviceToDevice, c->stream));
    CHK(stage_stats<T>(c));
    CHK(stage_densities<T>(c, false));
    HIPCHK(hipStreamSynchronize(c->stream));
    if (info) *info = r;
    return EPDLB_OK;
  };
  return c->p.precision == 0 ? run(double()) : run(float());
}

int epdlb_cg_stats(epdlb_ctx* c, epdlb_cg_info* last, int64_t* totals) {
  if (!c) return fail(EPDLB_EINVAL, "ctx is NULL");
  if (last) *last = c->cg_last;
  if (totals)
    for (int i = 0; i < 4; ++i) totals[i] = c->cg_totals[i];
  return EPDLB_OK;
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
  d->n_exact = c->n_exact;
  d->n_triggered = c->n_triggered;
  d->nn_err_last = s[kNnErrLast];
  d->nn_err_max = s[kNnErr];
  d->resid_nn_max = std::max(c->resid_nn_max, s[kNnResid]);
  d->resid_exact = s[kResidEx];
  d->nn_err_in_use = s[kNnErrUse];
  return EPDLB_OK;
}

int epdlb_autotune(epdlb_ctx* c, int32_t reps, const char* cache_path) {
  if (!c || reps < 1) return fail(EPDLB_EINVAL, "bad autotune arguments");
  HIPCHK(hipSetDevice(c->device));
  HIPCHK(hipStreamSynchronize(c->stream));
  // cached results
  std::vector<std::string> cache_lines;
  if (cache_path) {
    if (FILE* fp = std::fopen(cache_path, "r")) {
      char line[256];
      while (std::fgets(line, sizeof(line), fp)) cache_lines.emplace_back(line);
      std::fclose(fp);
    }
  }
  const bool fp32 = c->p.precision == 1;
  // the force-row candidates run the LB step: keep u, rho and the guard words
  // of every replica and put them back afterwards
  const size_t plane = size_t(c->p.nx) * c->p.ny * elem(c);
  const size_t keep_bytes = 3 * plane + 16 * sizeof(unsigned);
  unsigned char* keep = nullptr;
  HIPCHK(hipMalloc(&keep, keep_bytes * size_t(c->nrep)));
  auto copy_state = [&](bool save) -> int {
    for (int r = 0; r < c->nrep; ++r) {
      unsigned char* k = keep + keep_bytes * size_t(r);
      unsigned char* o = c->base + c->roff(r);
      const std::pair<size_t, size_t> parts[3] = {{c->L.u, 2 * plane}, {c->L.rho, plane},
                                                  {c->L.counters, 16 * sizeof(unsigned)}};
      size_t at = 0;
      for (const auto& pt : parts) {
        HIPCHK(hipMemcpyAsync(save ? k + at : o + pt.first, save ? o + pt.first : k + at, pt.second,
                              hipMemcpyDeviceToDevice, c->stream));
        at += pt.second;
      }
    }
    HIPCHK(hipStreamSynchronize(c->stream));
    return EPDLB_OK;
  };
  if (int e = copy_state(true)) {
    (void)hipFree(keep);
    return e;
  }
  const char* verbose_env = std::getenv("EPDLB_TUNE_VERBOSE");
  const bool verbose = verbose_env && std::atoi(verbose_env) != 0;
  for (int fam = 0; fam < F_NUM; ++fam) {
    const std::string key = tune_key(c, fam);
    bool found = false;
    for (auto& l : cache_lines) {
      if (l.compare(0, key.size(), key) == 0 && l.size() > key.size() && l[key.size()] == ' ') {
        int R = 0, nf = 0;
        double us = 0;
        if (std::sscanf(l.c_str() + key.size(), "%d %d %lf", &R, &nf, &us) == 3 &&
            time_candidate(c, fam, R, nf, 1) >= 0.0) {
          family_shape(c, fam) = {R, nf};
          found = true;
        }
      }
    }
    if (found) continue;
    const bool row = (fam == F_PROP_ROW || fam == F_FORCE_ROW);
    const int L = row ? c->p.nx : c->p.ny;
    const int transforms = fam == F_PROP_ROW ? c->p.ny / 2 : c->p.ny;
    double best = 1e30;
    epdlb_ctx::Shape best_sh = family_shape(c, fam);
    const int Rs[4] = {2, 4, 8, 16};
    for (int R : Rs) {
      if (R != 8 && !fp32) continue;
      if (row) {
        for (int nf = 1; nf * (L / R) <= 512 && nf <= transforms; nf *= 2) {
          const double us = time_candidate(c, fam, R, nf, reps);
          if (verbose) std::fprintf(stderr, "[tune] %s R=%d nf=%d: %.3f us\n", kFamilyName[fam], R, nf, us);
          if (us > 0 && us < best) best = us, best_sh = {R, nf};
        }
      } else {
        const int nfs[3] = {4, 8, 16};
        for (int nf : nfs) {
          const double us = time_candidate(c, fam, R, nf, reps);
          if (verbose) std::fprintf(stderr, "[tune] %s R=%d nf=%d: %.3f us\n", kFamilyName[fam], R, nf, us);
          if (us > 0 && us < best) best = us, best_sh = {R, nf};
        }
      }
    }
    family_shape(c, fam) = best_sh;
    if (cache_path && best < 1e29) {
      if (FILE* fp = std::fopen(cache_path, "a")) {
        std::fprintf(fp, "%s %d %d %.3f\n", key.c_str(), best_sh.R, best_sh.nf, best);
        std::fclose(fp);
      }
    }
  }
  drop_graphs(c);
  const hipError_t se = hipStreamSynchronize(c->stream);
  const int e = se == hipSuccess ? copy_state(false)
                                 : fail(EPDLB_EHIP, std::string("autotune: ") + hipGetErrorString(se));
  (void)hipFree(keep);
  return e;
}

int epdlb_get_shapes(epdlb_ctx* c, epdlb_shape* out, int32_t cap, int32_t* n_out) {
  if (!c || !out || !n_out || cap < F_NUM) return fail(EPDLB_EINVAL, "bad shape arguments");
  for (int f = 0; f < F_NUM; ++f) {
    std::memset(&out[f], 0, sizeof(out[f]));
    std::snprintf(out[f].family, sizeof(out[f].family), "%s", kFamilyName[f]);
    out[f].R = family_shape(c, f).R;
    out[f].nf = family_shape(c, f).nf;
  }
  *n_out = F_NUM;
  return EPDLB_OK;
}

int epdlb_set_shape(epdlb_ctx* c, const char* family, int32_t R, int32_t nf) {
  if (!c || !family) return fail(EPDLB_EINVAL, "NULL argument");
  for (int f = 0; f < F_NUM; ++f)
    if (std::strcmp(family, kFamilyName[f]) == 0) {
      HIPCHK(hipSetDevice(c->device));
      if (time_candidate(c, f, R, nf, 1) < 0.0) return fail(EPDLB_EINVAL, "shape cannot be launched");
      family_shape(c, f) = {R, nf};
      drop_graphs(c);
      return EPDLB_OK;
    }
  return fail(EPDLB_EINVAL, "unknown pass family");
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
  drop_graphs(c);
  if (c->cap_stream) (void)hipStreamDestroy(c->cap_stream);
  for (hipEvent_t e : c->prof_ev) (void)hipEventDestroy(e);
  if (c->stream) (void)hipStreamSynchronize(c->stream);
  if (c->own_mem && c->base) (void)hipFree(c->base);
  if (c->obs) (void)hipFree(c->obs);
  if (c->cg) (void)hipFree(c->cg);
  if (c->cg_host) (void)hipHostFree(c->cg_host);
  if (c->snap) (void)hipHostFree(c->snap);
  if (c->snap_ev) (void)hipEventDestroy(c->snap_ev);
  if (c->own_stream && c->stream) (void)hipStreamDestroy(c->stream);
  delete c;
}

int epdlb_batch_create(const epdlb_params* params, int32_t n_replicas, int device, void* stream,
                       epdlb_batch** out) {
  if (!params || n_replicas < 1 || !out) return fail(EPDLB_EINVAL, "bad batch arguments");
  *out = nullptr;
  for (int r = 0; r < n_replicas; ++r) {
    CHK(validate(&params[r]));
    if (params[r].cg_invert) return fail(EPDLB_EINVAL, "cg_invert is not supported in a batch");
    if (!same_model(params[0], params[r]))
      return fail(EPDLB_EINVAL, "replicas may differ only in nx, ny, g and f_A");
    if (params[r].density_mode != 0) return fail(EPDLB_EINVAL, "batched replicas run the exact densities only");
  }
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || ndev <= device || device < 0)
    return fail(EPDLB_ENODEV, "no HIP device with that index");
  HIPCHK(hipSetDevice(device));
  hipDeviceProp_t prop;
  HIPCHK(hipGetDeviceProperties(&prop, device));
  if (std::strncmp(prop.gcnArchName, "gfx950", 6) != 0)
    return fail(EPDLB_ENODEV, std::string("library built for gfx950, device is ") + prop.gcnArchName);
  epdlb_batch* b = new (std::nothrow) epdlb_batch();
  if (!b) return fail(EPDLB_ENOMEM, "host allocation failed");
  b->device = device;
  if (stream) {
    b->stream = reinterpret_cast<hipStream_t>(stream);
  } else {
    if (hipStreamCreateWithFlags(&b->stream, hipStreamNonBlocking) != hipSuccess) {
      delete b;
      return fail(EPDLB_EHIP, "hipStreamCreate failed");
    }
    b->own_stream = true;
  }
  // group by grid shape and A fraction (which fixes every launch's segment
  // fractions), keeping first-appearance order
  std::vector<std::tuple<int, int, double>> shapes;
  std::vector<std::vector<int>> members;
  b->where.resize(n_replicas);
  for (int r = 0; r < n_replicas; ++r) {
    const std::tuple<int, int, double> sh{params[r].nx, params[r].ny, params[r].f_A};
    size_t g = 0;
    while (g < shapes.size() && shapes[g] != sh) ++g;
    if (g == shapes.size()) {
      shapes.push_back(sh);
      members.emplace_back();
    }
    b->where[r] = {int(g), int(members[g].size())};
    members[g].push_back(r);
  }
  for (size_t g = 0; g < shapes.size(); ++g) {
    std::vector<epdlb_params> rp;
    for (int r : members[g]) rp.push_back(params[r]);
    epdlb_ctx* c = nullptr;
    const int rc = make_group(rp, device, &c);
    if (rc != EPDLB_OK) {
      epdlb_batch_destroy(b);
      return rc;
    }
    b->groups.push_back(c);
  }
  *out = b;
  return EPDLB_OK;
}

int epdlb_batch_seed(epdlb_batch* b, const uint64_t* seeds, double sigma) {
  if (!b || !seeds) return fail(EPDLB_EINVAL, "NULL argument");
  for (size_t g = 0; g < b->groups.size(); ++g) {
    epdlb_ctx* c = b->groups[g];
    const size_t n3 = size_t(3) * c->p.nx * c->p.ny;
    std::vector<std::vector<double>> w(c->nrep, std::vector<double>(n3));
    std::vector<const double*> ptrs(c->nrep);
    for (size_t r = 0; r < b->where.size(); ++r)
      if (b->where[r].first == int(g)) {
        const int i = b->where[r].second;
        CHK(epdlb_noise_fill(seeds[r], sigma, c->p.nx, c->p.ny, w[i].data()));
        ptrs[i] = w[i].data();
      }
    c->cur = 0;
    c->fcur = 0;
    CHK(set_fields_group(c, ptrs.data()));
    c->nstep = 0;
    CHK(check_finite(c));
  }
  b->nstep = 0;
  b->seeded = true;
  return EPDLB_OK;
}

int epdlb_batch_set_fields(epdlb_batch* b, int32_t replica, const double* omega) {
  epdlb_ctx* c;
  int i;
  CHK(batch_replica(b, replica, &c, &i));
  if (!omega || !b->seeded) return fail(EPDLB_ESTATE, "seed the batch before replacing one replica");
  std::vector<const double*> ptrs(c->nrep, nullptr);
  ptrs[i] = omega;
  CHK(set_fields_group(c, ptrs.data()));
  return check_finite(c);
}

int epdlb_batch_step(epdlb_batch* b, int64_t n) {
  if (!b) return fail(EPDLB_EINVAL, "batch is NULL");
  if (!b->seeded) return fail(EPDLB_ESTATE, "step before seed");
  if (n < 0) return fail(EPDLB_EINVAL, "negative step count");
  HIPCHK(hipSetDevice(b->device));
  if (b->prof) {
    // profiled steps: each group's launches on the batch stream, in order
    for (int64_t s = 0; s < n; ++s) {
      for (auto* c : b->groups) {
        hipStream_t own = c->stream;
        c->stream = b->stream;
        int r = EPDLB_OK;
        for (int k = EPDLB_STAGE_ADVECT_UPDATE; k <= EPDLB_STAGE_DENSITIES && r == EPDLB_OK; ++k) r = run_stage(c, k);
        if (r == EPDLB_OK) r = run_force_lb(c);
        c->stream = own;
        CHK(r);
        ++c->nstep;
      }
      ++b->nstep;
    }
    drop_batch_graphs(b);  // parities may have changed
    return EPDLB_OK;
  }
  // the graphs' branches start after work already queued on the batch stream
  while (n > 0) {
    const int k = n >= 2 ? 2 : 1;
    hipGraphExec_t g;
    CHK(batch_graph(b, k, &g));
    HIPCHK(hipGraphLaunch(g, b->stream));
    if (k == 1) {
      for (auto* c : b->groups) {
        c->cur = 1 - c->cur;
        c->fcur = 1 - c->fcur;
      }
      drop_batch_graphs(b);  // parities changed: recapture from the new state
    }
    for (auto* c : b->groups) c->nstep += k;
    b->nstep += k;
    n -= k;
  }
  return EPDLB_OK;
}

int epdlb_batch_sync(epdlb_batch* b) {
  if (!b) return fail(EPDLB_EINVAL, "batch is NULL");
  HIPCHK(hipStreamSynchronize(b->stream));
  for (auto* c : b->groups) CHK(check_finite(c));
  return EPDLB_OK;
}

int epdlb_batch_read_densities(epdlb_batch* b, int32_t replica, double* pa, double* pb, double* ps) {
  epdlb_ctx* c;
  int i;
  CHK(batch_replica(b, replica, &c, &i));
  if (!pa || !pb || !ps) return fail(EPDLB_EINVAL, "NULL argument");
  HIPCHK(hipStreamSynchronize(b->stream));
  const size_t n = size_t(c->p.nx) * c->p.ny, pl = n * elem(c), o = c->roff(i) + c->L.phi;
  CHK(download(c, o, pa, n));
  CHK(download(c, o + pl, pb, n));
  return download(c, o + 2 * pl, ps, n);
}

int epdlb_batch_read_fields(epdlb_batch* b, int32_t replica, double* wa, double* wb, double* ws) {
  epdlb_ctx* c;
  int i;
  CHK(batch_replica(b, replica, &c, &i));
  if (!wa || !wb || !ws) return fail(EPDLB_EINVAL, "NULL argument");
  HIPCHK(hipStreamSynchronize(b->stream));
  const size_t n = size_t(c->p.nx) * c->p.ny, pl = n * elem(c), o = c->roff(i) + c->L.omega[c->cur];
  CHK(download(c, o, wa, n));
  CHK(download(c, o + pl, wb, n));
  return download(c, o + 2 * pl, ws, n);
}

int epdlb_batch_read_velocity(epdlb_batch* b, int32_t replica, double* rho, double* ux, double* uy) {
  epdlb_ctx* c;
  int i;
  CHK(batch_replica(b, replica, &c, &i));
  if (!rho || !ux || !uy) return fail(EPDLB_EINVAL, "NULL argument");
  HIPCHK(hipStreamSynchronize(b->stream));
  const size_t n = size_t(c->p.nx) * c->p.ny, pl = n * elem(c), o = c->roff(i);
  CHK(download(c, o + c->L.rho, rho, n));
  CHK(download(c, o + c->L.u, ux, n));
  return download(c, o + c->L.u + pl, uy, n);
}

int epdlb_batch_read_diag(epdlb_batch* b, int32_t replica, epdlb_diag* d) {
  epdlb_ctx* c;
  int i;
  CHK(batch_replica(b, replica, &c, &i));
  if (!d) return fail(EPDLB_EINVAL, "NULL argument");
  HIPCHK(hipStreamSynchronize(b->stream));
  double s[kNumScal];
  HIPCHK(hipMemcpyAsync(s, c->base + c->roff(i) + c->L.scal, sizeof(s), hipMemcpyDeviceToHost, c->stream));
  HIPCHK(hipStreamSynchronize(c->stream));
  *d = epdlb_diag{};
  d->step = b->nstep;
  d->Q_P = s[kQPf];
  d->Q_P_bwd = s[kQPb];
  d->Q_S = s[kQS];
  d->gauge_S = s[kGaugeS];
  d->mean_omega[0] = s[kMeanA];
  d->mean_omega[1] = s[kMeanB];
  d->mean_omega[2] = s[kMeanS];
  return EPDLB_OK;
}

int epdlb_batch_autotune(epdlb_batch* b, int32_t reps, const char* cache_path) {
  if (!b) return fail(EPDLB_EINVAL, "batch is NULL");
  HIPCHK(hipStreamSynchronize(b->stream));
  for (auto* c : b->groups) CHK(epdlb_autotune(c, reps, cache_path));
  drop_batch_graphs(b);
  return EPDLB_OK;
}

int epdlb_batch_profile_start(epdlb_batch* b, int32_t max_launches) {
  if (!b) return fail(EPDLB_EINVAL, "batch is NULL");
  for (auto* c : b->groups) CHK(epdlb_profile_start(c, max_launches));
  b->prof = true;
  return EPDLB_OK;
}

int epdlb_batch_profile_read(epdlb_batch* b, epdlb_kernel_stat* out, int32_t cap, int32_t* n_out) {
  if (!b || !out || !n_out || cap < 1) return fail(EPDLB_EINVAL, "bad profile arguments");
  HIPCHK(hipStreamSynchronize(b->stream));
  std::vector<epdlb_kernel_stat> all;
  for (auto* c : b->groups) {
    epdlb_kernel_stat tmp[32];
    int32_t n = 0;
    CHK(epdlb_profile_read(c, tmp, 32, &n));
    for (int i = 0; i < n; ++i) {
      bool merged = false;
      for (auto& a : all)
        if (std::strcmp(a.name, tmp[i].name) == 0) {
          a.launches += tmp[i].launches;
          a.total_ms += tmp[i].total_ms;
          a.min_ms = std::min(a.min_ms, tmp[i].min_ms);
          a.max_ms = std::max(a.max_ms, tmp[i].max_ms);
          merged = true;
        }
      if (!merged) all.push_back(tmp[i]);
    }
  }
  int n = 0;
  for (auto& a : all)
    if (n < cap) out[n++] = a;
  *n_out = n;
  b->prof = false;
  return EPDLB_OK;
}

int epdlb_batch_info(epdlb_batch* b, int32_t* n_groups, int64_t* sites) {
  if (!b || !n_groups || !sites) return fail(EPDLB_EINVAL, "NULL argument");
  *n_groups = int32_t(b->groups.size());
  int64_t s = 0;
  for (auto* c : b->groups) s += int64_t(c->nrep) * c->p.nx * c->p.ny;
  *sites = s;
  return EPDLB_OK;
}

void epdlb_batch_destroy(epdlb_batch* b) {
  if (!b) return;
  if (b->stream) (void)hipStreamSynchronize(b->stream);
  drop_batch_graphs(b);
  for (auto* c : b->groups) epdlb_destroy(c);
  for (auto s : b->fork) (void)hipStreamDestroy(s);
  for (auto e : b->ev_join) (void)hipEventDestroy(e);
  if (b->ev_fork) (void)hipEventDestroy(b->ev_fork);
  if (b->cap) (void)hipStreamDestroy(b->cap);
  if (b->own_stream && b->stream) (void)hipStreamDestroy(b->stream);
  delete b;
}

const char* epdlb_last_error(void) { return g_err.c_str(); }

}  // extern "C"

// ---------------------------------------------------------------------------
// Density surrogate
// ---------------------------------------------------------------------------
int epdlb_surrogate_set_weights(epdlb_ctx* c, const float* w, int64_t count) {
  if (!c || !w) return fail(EPDLB_EINVAL, "NULL argument");
  if (c->p.density_mode != 1) return fail(EPDLB_ESTATE, "context was not created with density_mode = 1");
  if (count != nn::kNnParams) return fail(EPDLB_EINVAL, "expected EPDLB_NN_PARAMS weights");
  for (int64_t i = 0; i < count; ++i)
    if (!std::isfinite(w[i])) return fail(EPDLB_EINVAL, "non-finite weight");
  HIPCHK(hipSetDevice(c->device));
  float* dw = c->ptr<float>(c->L.nn_w);
  HIPCHK(hipMemcpyAsync(dw, w, sizeof(float) * count, hipMemcpyHostToDevice, c->stream));
  HIPCHK(nn_pack(dw, c->ptr<__bf16>(c->L.nn_frag), nullptr, c->stream));
  hipLaunchKernelGGL(nn::k_pack_proj, dim3(unsigned((nn::kProjFragElems + 255) / 256)), dim3(256), 0, c->stream,
                     (const float*)(dw + nn_offsets().W[3]), c->ptr<__bf16>(c->L.nn_frag) + nn::kFwdFragElems);
  HIPCHK(hipGetLastError());
  HIPCHK(hipStreamSynchronize(c->stream));
  c->nn_ready = true;
  if (c->seeded) CHK(nn_after_seed(c));
  return EPDLB_OK;
}

int epdlb_nn_create(int32_t nx, int32_t ny, int32_t capacity, int32_t max_batch, int device, void* stream,
                    epdlb_nn** out) {
  if (!out) return fail(EPDLB_EINVAL, "out is NULL");
  *out = nullptr;
  if (!is_pow2(nx) || nx < 32 || nx > 1024 || !is_pow2(ny) || ny < 16 || ny > 1024)
    return fail(EPDLB_EINVAL, "nx, ny must be powers of two, 32 <= nx <= 1024, 16 <= ny <= 1024");
  if (capacity < 1 || max_batch < 1 || max_batch > capacity || max_batch > nn::kMaxBatch)
    return fail(EPDLB_EINVAL, "bad capacity or batch (1 <= max_batch <= min(capacity, 64))");
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || ndev <= device || device < 0)
    return fail(EPDLB_ENODEV, "no HIP device with that index");
  HIPCHK(hipSetDevice(device));
  hipDeviceProp_t prop;
  HIPCHK(hipGetDeviceProperties(&prop, device));
  if (std::strncmp(prop.gcnArchName, "gfx950", 6) != 0)
    return fail(EPDLB_ENODEV, std::string("library built for gfx950, device is ") + prop.gcnArchName);
  device_cus();
  epdlb_nn* t = new (std::nothrow) epdlb_nn();
  if (!t) return fail(EPDLB_ENOMEM, "host allocation failed");
  t->device = device;
  t->nx = nx;
  t->ny = ny;
  t->n = long(nx) * ny;
  t->capacity = capacity;
  t->max_batch = max_batch;
  const size_t n = size_t(t->n);
  const FragOffsets fo = frag_offsets();
  size_t off = 0;
  std::vector<size_t> offs;
  auto take = [&](size_t bytes) {
    offs.push_back(off);
    off = align256(off + bytes);
  };
  const size_t P = nn::kNnParams;
  for (int i = 0; i < 4; ++i) take(P * sizeof(float));        // w g m v
  take(fo.ftotal * 2);                                        // ffrag
  take(fo.btotal * 2);                                        // bfrag
  take(size_t(capacity) * n * nn::kXC * 2);                   // x
  take(size_t(capacity) * 2 * n * sizeof(float));             // tgt
  for (int i = 0; i < 6; ++i) take(size_t(max_batch) * n * nn::kHid * 2);  // act, z
  take(size_t(max_batch) * n * nn::kXC * 2);                  // g4
  for (int i = 0; i < 2; ++i) take(size_t(max_batch) * n * nn::kHid * 2);  // gb
  take(2 * n * sizeof(float));                                // pred
  take(size_t(max_batch) * sizeof(int));                      // slots
  take(2 * kConvMaxBlocks * sizeof(double));                  // lpart
  take(size_t(kWgradMaxBlocks) * 9 * 64 * 64 * sizeof(float));  // wpart
  take(size_t(kWgradMaxBlocks) * 64 * sizeof(float));         // wpartb
  take((5 * n + 3) * sizeof(double));                         // stage
  if (hipMalloc(&t->mem, off) != hipSuccess) {
    delete t;
    return fail(EPDLB_ENOMEM, "hipMalloc of the trainer arena failed");
  }
  unsigned char* b = static_cast<unsigned char*>(t->mem);
  int k = 0;
  t->w = reinterpret_cast<float*>(b + offs[k++]);
  t->g = reinterpret_cast<float*>(b + offs[k++]);
  t->m = reinterpret_cast<float*>(b + offs[k++]);
  t->v = reinterpret_cast<float*>(b + offs[k++]);
  t->ffrag = reinterpret_cast<__bf16*>(b + offs[k++]);
  t->bfrag = reinterpret_cast<__bf16*>(b + offs[k++]);
  t->x = reinterpret_cast<__bf16*>(b + offs[k++]);
  t->tgt = reinterpret_cast<float*>(b + offs[k++]);
  for (int i = 0; i < 3; ++i) {
    t->act[i] = reinterpret_cast<__bf16*>(b + offs[k++]);
    t->zz[i] = reinterpret_cast<__bf16*>(b + offs[k++]);
  }
  t->g4 = reinterpret_cast<__bf16*>(b + offs[k++]);
  t->gb[0] = reinterpret_cast<__bf16*>(b + offs[k++]);
  t->gb[1] = reinterpret_cast<__bf16*>(b + offs[k++]);
  t->pred = reinterpret_cast<float*>(b + offs[k++]);
  t->slots = reinterpret_cast<int*>(b + offs[k++]);
  t->lpart = reinterpret_cast<double*>(b + offs[k++]);
  t->wpart = reinterpret_cast<float*>(b + offs[k++]);
  t->wpartb = reinterpret_cast<float*>(b + offs[k++]);
  t->stage = reinterpret_cast<double*>(b + offs[k++]);
  if (stream) {
    t->stream = reinterpret_cast<hipStream_t>(stream);
  } else {
    if (hipStreamCreateWithFlags(&t->stream, hipStreamNonBlocking) != hipSuccess) {
      epdlb_nn_destroy(t);
      return fail(EPDLB_EHIP, "hipStreamCreate failed");
    }
    t->own_stream = true;
  }
  // zero weights and moments until set_weights
  if (hipMemsetAsync(t->w, 0, 4 * align256(P * sizeof(float)), t->stream) != hipSuccess ||
      nn_pack(t->w, t->ffrag, t->bfrag, t->stream) != hipSuccess || hipStreamSynchronize(t->stream) != hipSuccess) {
    epdlb_nn_destroy(t);
    return fail(EPDLB_EHIP, "clearing the trainer weights failed");
  }
  t->packed_bwd = true;
  *out = t;
  return EPDLB_OK;
}

int epdlb_nn_set_weights(epdlb_nn* t, const float* w, int64_t count) {
  if (!t || !w) return fail(EPDLB_EINVAL, "NULL argument");
  if (count != nn::kNnParams) return fail(EPDLB_EINVAL, "expected EPDLB_NN_PARAMS weights");
  for (int64_t i = 0; i < count; ++i)
    if (!std::isfinite(w[i])) return fail(EPDLB_EINVAL, "non-finite weight");
  HIPCHK(hipSetDevice(t->device));
  HIPCHK(hipMemcpyAsync(t->w, w, sizeof(float) * count, hipMemcpyHostToDevice, t->stream));
  const size_t pb = align256(size_t(nn::kNnParams) * sizeof(float));
  HIPCHK(hipMemsetAsync(t->m, 0, 2 * pb, t->stream));  // m and v are adjacent
  HIPCHK(nn_pack(t->w, t->ffrag, t->bfrag, t->stream));
  HIPCHK(hipStreamSynchronize(t->stream));
  t->adam_t = 0;
  t->packed_bwd = true;
  return EPDLB_OK;
}

int epdlb_nn_get_weights(epdlb_nn* t, float* w, int64_t count) {
  if (!t || !w) return fail(EPDLB_EINVAL, "NULL argument");
  if (count != nn::kNnParams) return fail(EPDLB_EINVAL, "expected EPDLB_NN_PARAMS weights");
  HIPCHK(hipSetDevice(t->device));
  HIPCHK(hipMemcpyAsync(w, t->w, sizeof(float) * count, hipMemcpyDeviceToHost, t->stream));
  HIPCHK(hipStreamSynchronize(t->stream));
  return EPDLB_OK;
}

int epdlb_nn_set_pair(epdlb_nn* t, int32_t slot, const double* omega, const double* phi, double f_A,
                      int32_t n_contour) {
  if (!t || !omega || !phi) return fail(EPDLB_EINVAL, "NULL argument");
  if (slot < 0 || slot >= t->capacity) return fail(EPDLB_EINVAL, "slot index out of range");
  if (!(f_A > 0.0 && f_A < 1.0) || n_contour < 1) return fail(EPDLB_EINVAL, "bad f_A or n_contour");
  HIPCHK(hipSetDevice(t->device));
  const size_t n = size_t(t->n);
  std::vector<double> h(5 * n + 3);
  std::memcpy(h.data(), omega, 3 * n * sizeof(double));
  std::memcpy(h.data() + 3 * n, phi, 2 * n * sizeof(double));
  for (int I = 0; I < 3; ++I) {
    double sum = 0.0;
    for (size_t i = 0; i < n; ++i) sum += omega[I * n + i];
    h[5 * n + I] = sum / double(n);
  }
  HIPCHK(hipMemcpyAsync(t->stage, h.data(), h.size() * sizeof(double), hipMemcpyHostToDevice, t->stream));
  hipLaunchKernelGGL(nn::k_nn_input<double>, dim3(unsigned((n + 255) / 256)), dim3(256), 0, t->stream,
                     (const double*)t->stage, (const double*)(t->stage + 5 * n), long(n), t->nx, float(f_A),
                     float(1.0 / n_contour), t->x + size_t(slot) * n * nn::kXC, (const double*)(t->stage + 3 * n),
                     t->tgt + size_t(slot) * 2 * n);
  HIPCHK(hipGetLastError());
  HIPCHK(hipStreamSynchronize(t->stream));
  return EPDLB_OK;
}

int epdlb_nn_capture(epdlb_nn* t, int32_t slot, epdlb_ctx* c) {
  if (!t || !c) return fail(EPDLB_EINVAL, "NULL argument");
  if (slot < 0 || slot >= t->capacity) return fail(EPDLB_EINVAL, "slot index out of range");
  if (c->p.nx != t->nx || c->p.ny != t->ny || c->device != t->device)
    return fail(EPDLB_EINVAL, "simulation grid or device differs from the trainer's");
  if (c->p.density_mode != 0) return fail(EPDLB_EINVAL, "pairs come from a simulation with exact densities");
  if (!c->seeded) return fail(EPDLB_ESTATE, "simulation not seeded");
  HIPCHK(hipSetDevice(t->device));
  HIPCHK(hipStreamSynchronize(c->stream));
  const long n = t->n;
  const float fA = float(c->p.f_A), invN = float(1.0 / c->p.n_contour);
  const double* mean = c->ptr<double>(c->L.scal) + kMeanA;
  __bf16* x = t->x + size_t(slot) * n * nn::kXC;
  float* tg = t->tgt + size_t(slot) * 2 * n;
  if (c->p.precision == 0)
    hipLaunchKernelGGL(nn::k_nn_input<double>, dim3(unsigned((n + 255) / 256)), dim3(256), 0, t->stream,
                       (const double*)c->ptr<double>(c->L.omega[c->cur]), mean, n, t->nx, fA, invN, x,
                       (const double*)c->ptr<double>(c->L.phi), tg);
  else
    hipLaunchKernelGGL(nn::k_nn_input<float>, dim3(unsigned((n + 255) / 256)), dim3(256), 0, t->stream,
                       (const float*)c->ptr<float>(c->L.omega[c->cur]), mean, n, t->nx, fA, invN, x,
                       (const float*)c->ptr<float>(c->L.phi), tg);
  HIPCHK(hipGetLastError());
  HIPCHK(hipStreamSynchronize(t->stream));
  return EPDLB_OK;
}

static int nn_read_loss(epdlb_nn* t, int count, double* loss, double* max_err) {
  std::vector<double> h(2 * size_t(t->last_nblocks));
  HIPCHK(hipMemcpyAsync(h.data(), t->lpart, h.size() * sizeof(double), hipMemcpyDeviceToHost, t->stream));
  HIPCHK(hipStreamSynchronize(t->stream));
  double s = 0.0, mx = 0.0;
  for (int b = 0; b < t->last_nblocks; ++b) {
    s += h[2 * b];
    mx = std::max(mx, h[2 * b + 1]);
  }
  if (loss) *loss = s / (double(count) * double(t->n) * 2.0);
  if (max_err) *max_err = mx;
  return EPDLB_OK;
}

int epdlb_nn_evaluate(epdlb_nn* t, const int32_t* slots, int32_t count, double phi_scale, double* loss,
                      double* max_err, float* grad) {
  if (!t) return fail(EPDLB_EINVAL, "NULL argument");
  if (!(phi_scale > 0.0)) return fail(EPDLB_EINVAL, "phi_scale must be > 0");
  HIPCHK(hipSetDevice(t->device));
  CHK(nn_upload_slots(t, slots, count));
  CHK(nn_forward_train(t, count, phi_scale));
  if (grad) {
    CHK(nn_backward(t, count));
    HIPCHK(hipMemcpyAsync(grad, t->g, sizeof(float) * nn::kNnParams, hipMemcpyDeviceToHost, t->stream));
  }
  return nn_read_loss(t, count, loss, max_err);
}

int epdlb_nn_train_step(epdlb_nn* t, const int32_t* slots, int32_t count, double phi_scale, double lr) {
  if (!t) return fail(EPDLB_EINVAL, "NULL argument");
  if (!(phi_scale > 0.0) || !(lr > 0.0)) return fail(EPDLB_EINVAL, "phi_scale and lr must be > 0");
  HIPCHK(hipSetDevice(t->device));
  CHK(nn_upload_slots(t, slots, count));
  t->last_count = count;
  CHK(nn_forward_train(t, count, phi_scale));
  CHK(nn_backward(t, count));
  ++t->adam_t;
  const double b1 = 0.9, b2 = 0.999;
  const float c1 = float(lr / (1.0 - std::pow(b1, t->adam_t)));
  const float c2 = float(1.0 / (1.0 - std::pow(b2, t->adam_t)));
  hipLaunchKernelGGL(nn::k_adam, dim3((nn::kNnParams + 255) / 256), dim3(256), 0, t->stream, t->w,
                     (const float*)t->g, t->m, t->v, int(nn::kNnParams), float(b1), float(b2), c1, c2, 1e-8f);
  HIPCHK(hipGetLastError());
  HIPCHK(nn_pack(t->w, t->ffrag, t->bfrag, t->stream));
  return EPDLB_OK;
}

int epdlb_nn_last_loss(epdlb_nn* t, double* loss, double* max_err) {
  if (!t) return fail(EPDLB_EINVAL, "NULL argument");
  if (t->last_count < 1) return fail(EPDLB_ESTATE, "no training step yet");
  HIPCHK(hipSetDevice(t->device));
  return nn_read_loss(t, t->last_count, loss, max_err);
}

int epdlb_nn_predict(epdlb_nn* t, int32_t slot, double* phi_hat) {
  if (!t || !phi_hat) return fail(EPDLB_EINVAL, "NULL argument");
  if (slot < 0 || slot >= t->capacity) return fail(EPDLB_EINVAL, "slot index out of range");
  HIPCHK(hipSetDevice(t->device));
  CHK(nn_upload_slots(t, &slot, 1));
  const NnOffsets o = nn_offsets();
  const FragOffsets fo = frag_offsets();
  const long n = t->n;
  const int tps = (t->nx / nn::kTW) * (t->ny / nn::kConvTH);
  nn::ConvArgs a{};
  a.nx = t->nx;
  a.ny = t->ny;
  a.tiles_per_sample = a.ntiles = tps;
  a.bs = n * nn::kHid;
  for (int l = 0; l < 3; ++l) {
    a.in = l == 0 ? t->x : t->act[l - 1];
    a.in_bs = n * (l == 0 ? nn::kXC : nn::kHid);
    a.slots = l == 0 ? t->slots : nullptr;
    a.wfrag = t->ffrag + fo.f[l];
    a.bias = t->w + o.b[l];
    a.out = t->act[l];
    a.d = nn::dil_of(l);
    const hipError_t e = l == 0 ? conv_hidden<nn::kXC, nn::EPI_FWD>(a, t->stream)
                                : conv_hidden<nn::kHid, nn::EPI_FWD>(a, t->stream);
    HIPCHK(e);
  }
  nn::OutArgs<float> q{};
  q.in = t->act[2];
  q.in_bs = n * nn::kHid;
  q.wfrag = t->ffrag + fo.f[3];
  q.bias = t->w + o.b[3];
  q.phi = t->pred;
  q.plane = n;
  q.partials = t->lpart;
  q.nx = t->nx;
  q.ny = t->ny;
  q.d = nn::dil_of(3);
  q.tiles_per_sample = q.ntiles = tps;
  int nb = 0;
  HIPCHK((conv_out<float, nn::EPO_INFER>(q, t->stream, &nb)));
  std::vector<float> h(2 * size_t(n));
  HIPCHK(hipMemcpyAsync(h.data(), t->pred, h.size() * sizeof(float), hipMemcpyDeviceToHost, t->stream));
  HIPCHK(hipStreamSynchronize(t->stream));
  for (size_t i = 0; i < h.size(); ++i) phi_hat[i] = h[i];
  return EPDLB_OK;
}

void epdlb_nn_destroy(epdlb_nn* t) {
  if (!t) return;
  if (t->stream) (void)hipStreamSynchronize(t->stream);
  if (t->mem) (void)hipFree(t->mem);
  if (t->own_stream && t->stream) (void)hipStreamDestroy(t->stream);
  delete t;
}

// ---------------------------------------------------------------------------
// Three-dimensional fluid: D3Q19 populations, force and moments of one box.
// ---------------------------------------------------------------------------
struct epdlb_lb3 {
  int device = 0;
  int nx = 0, ny = 0, nz = 0;
  long n = 0;
  int precision = 0;
  double tau = 1.0;
  void* mem = nullptr;
  void* f[2] = {nullptr, nullptr};
  void* F = nullptr;
  void* rho = nullptr;
  void* u = nullptr;
  int cur = 0;  // f[cur] holds the post-collision populations of the last step
  bool have_moments = false;
  int mrt = 0;  // 0: BGK at tau; 1: multi-relaxation with the factors below
  double gs = 0.0, gb = 0.0, gg = 0.0;
  hipStream_t stream = nullptr;
  bool own_stream = false;
  std::vector<hipEvent_t> ev;  // start/stop pairs of epdlb_lb3_profile
  size_t es() const { return precision ? sizeof(float) : sizeof(double); }
};

namespace {

double lb3_weight(int k) { return k == 0 ? 1.0 / 3.0 : (k < 7 ? 1.0 / 18.0 : 1.0 / 36.0); }

template <typename T> lb3::Lb3Args<T> lb3_args(epdlb_lb3* c, int from) {
  lb3::Lb3Args<T> a;
  a.fin = static_cast<const T*>(c->f[from]);
  a.fout = static_cast<T*>(c->f[from ^ 1]);
  a.F = static_cast<const T*>(c->F);
  a.rho = static_cast<T*>(c->rho);
  a.u = static_cast<T*>(c->u);
  a.nx = c->nx;
  a.ny = c->ny;
  a.nz = c->nz;
  a.n = c->n;
  a.omega = T(1.0 / c->tau);
  a.fpre = T(1.0 - 0.5 / c->tau);
  return a;
}

dim3 lb3_grid(const epdlb_lb3* c) { return dim3((c->ny + lb3::kRows - 1) / lb3::kRows, c->nz); }

// One step from f[cur] into f[cur ^ 1]; the moments are stored when mom.
template <typename T> int lb3_launch(epdlb_lb3* c, bool mom) {
  const auto a = lb3_args<T>(c, c->cur);
  if (c->mrt) {
    lb3::Lb3MrtArgs<T> m;
    m.b = a;
    m.gs = T(c->gs);
    m.gb = T(c->gb);
    m.gg = T(c->gg);
    if (mom)
      launch_k((lb3::k_lb3_mrt<T, true>), lb3_grid(c), dim3(lb3::kThreads), 0, c->stream, m);
    else
      launch_k((lb3::k_lb3_mrt<T, false>), lb3_grid(c), dim3(lb3::kThreads), 0, c->stream, m);
    HIPCHK(hipGetLastError());
    c->cur ^= 1;
    return EPDLB_OK;
  }
  if (mom)
    launch_k((lb3::k_lb3<T, true>), lb3_grid(c), dim3(lb3::kThreads), 0, c->stream, a);
  else
    launch_k((lb3::k_lb3<T, false>), lb3_grid(c), dim3(lb3::kThreads), 0, c->stream, a);
  HIPCHK(hipGetLastError());
  c->cur ^= 1;
  return EPDLB_OK;
}

int lb3_steps(epdlb_lb3* c, int64_t n, hipEvent_t* ev) {
  for (int64_t s = 0; s < n; ++s) {
    if (ev) {
      tl_ev_start = ev[2 * s];
      tl_ev_stop = ev[2 * s + 1];
    }
    const bool mom = s + 1 == n;
    CHK(c->precision ? lb3_launch<float>(c, mom) : lb3_launch<double>(c, mom));
  }
  if (n > 0) c->have_moments = true;
  return EPDLB_OK;
}

// Host FP64 values -> device planes in the context's precision.
int lb3_upload(epdlb_lb3* c, void* dst, const double* src, size_t count, const double* minus_w) {
  if (c->precision) {
    std::vector<float> h(count);
    for (size_t i = 0; i < count; ++i) h[i] = float(minus_w ? src[i] - minus_w[i / size_t(c->n)] : src[i]);
    HIPCHK(hipMemcpyAsync(dst, h.data(), count * sizeof(float), hipMemcpyHostToDevice, c->stream));
    HIPCHK(hipStreamSynchronize(c->stream));
  } else {
    std::vector<double> h(count);
    for (size_t i = 0; i < count; ++i) h[i] = minus_w ? src[i] - minus_w[i / size_t(c->n)] : src[i];
    HIPCHK(hipMemcpyAsync(dst, h.data(), count * sizeof(double), hipMemcpyHostToDevice, c->stream));
    HIPCHK(hipStreamSynchronize(c->stream));
  }
  return EPDLB_OK;
}

int lb3_download(epdlb_lb3* c, double* dst, const void* src, size_t count, const double* plus_w) {
  if (c->precision) {
    std::vector<float> h(count);
    HIPCHK(hipMemcpyAsync(h.data(), src, count * sizeof(float), hipMemcpyDeviceToHost, c->stream));
    HIPCHK(hipStreamSynchronize(c->stream));
    for (size_t i = 0; i < count; ++i) dst[i] = plus_w ? plus_w[i / size_t(c->n)] + double(h[i]) : double(h[i]);
  } else {
    std::vector<double> h(count);
    HIPCHK(hipMemcpyAsync(h.data(), src, count * sizeof(double), hipMemcpyDeviceToHost, c->stream));
    HIPCHK(hipStreamSynchronize(c->stream));
    for (size_t i = 0; i < count; ++i) dst[i] = plus_w ? plus_w[i / size_t(c->n)] + h[i] : h[i];
  }
  return EPDLB_OK;
}

bool all_finite(const double* v, size_t count) {
  for (size_t i = 0; i < count; ++i)
    if (!std::isfinite(v[i])) return false;
  return true;
}

}  // namespace

int epdlb_lb3_create(int32_t nx, int32_t ny, int32_t nz, double tau, int32_t precision, int device, void* stream,
                     epdlb_lb3** out) {
  if (!out) return fail(EPDLB_EINVAL, "out is NULL");
  *out = nullptr;
  if (nx < 1 || ny < 1 || nz < 1 || nx > 4096 || ny > 4096 || nz > 4096)
    return fail(EPDLB_EINVAL, "nx, ny, nz must lie in [1, 4096]");
  if (!(tau > 0.5) || !std::isfinite(tau)) return fail(EPDLB_EINVAL, "tau must be a finite value > 1/2");
  if (precision != 0 && precision != 1) return fail(EPDLB_EINVAL, "precision must be 0 or 1");
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || ndev <= device || device < 0)
    return fail(EPDLB_ENODEV, "no HIP device with that index");
  HIPCHK(hipSetDevice(device));
  hipDeviceProp_t prop;
  HIPCHK(hipGetDeviceProperties(&prop, device));
  if (std::strncmp(prop.gcnArchName, "gfx950", 6) != 0)
    return fail(EPDLB_ENODEV, std::string("library built for gfx950, device is ") + prop.gcnArchName);
  epdlb_lb3* c = new (std::nothrow) epdlb_lb3();
  if (!c) return fail(EPDLB_ENOMEM, "host allocation failed");
  c->device = device;
  c->nx = nx;
  c->ny = ny;
  c->nz = nz;
  c->n = long(nx) * ny * nz;
  c->precision = precision;
  c->tau = tau;
  const size_t plane = align256(size_t(c->n) * c->es());
  const size_t fbytes = lb3::kQ * plane;
  const size_t total = 2 * fbytes + 3 * plane + plane + 3 * plane;
  if (hipMalloc(&c->mem, total) != hipSuccess) {
    delete c;
    return fail(EPDLB_ENOMEM, "hipMalloc of the populations failed");
  }
  unsigned char* b = static_cast<unsigned char*>(c->mem);
  c->f[0] = b;
  c->f[1] = b + fbytes;
  c->F = b + 2 * fbytes;
  c->rho = b + 2 * fbytes + 3 * plane;
  c->u = b + 2 * fbytes + 4 * plane;
  if (stream) {
    c->stream = reinterpret_cast<hipStream_t>(stream);
  } else {
    if (hipStreamCreateWithFlags(&c->stream, hipStreamNonBlocking) != hipSuccess) {
      epdlb_lb3_destroy(c);
      return fail(EPDLB_EHIP, "hipStreamCreate failed");
    }
    c->own_stream = true;
  }
  // rest state (g = 0: rho = 1, u = 0) and no force
  if (hipMemsetAsync(c->mem, 0, total, c->stream) != hipSuccess || hipStreamSynchronize(c->stream) != hipSuccess) {
    epdlb_lb3_destroy(c);
    return fail(EPDLB_EHIP, "clearing the populations failed");
  }
  *out = c;
  return EPDLB_OK;
}

int epdlb_lb3_set_populations(epdlb_lb3* c, const double* f) {
  if (!c || !f) return fail(EPDLB_EINVAL, "NULL argument");
  const size_t count = size_t(lb3::kQ) * size_t(c->n);
  if (!all_finite(f, count)) return fail(EPDLB_EINVAL, "non-finite population");
  HIPCHK(hipSetDevice(c->device));
  double w[lb3::kQ];
  for (int k = 0; k < lb3::kQ; ++k) w[k] = lb3_weight(k);
  CHK(lb3_upload(c, c->f[c->cur], f, count, w));
  c->have_moments = false;
  return EPDLB_OK;
}

int epdlb_lb3_set_equilibrium(epdlb_lb3* c, const double* rho, const double* u) {
  if (!c) return fail(EPDLB_EINVAL, "NULL context");
  const size_t n = size_t(c->n);
  if ((rho && !all_finite(rho, n)) || (u && !all_finite(u, 3 * n))) return fail(EPDLB_EINVAL, "non-finite moment");
  if (rho)
    for (size_t i = 0; i < n; ++i)
      if (!(rho[i] > 0.0)) return fail(EPDLB_EINVAL, "density must be > 0");
  HIPCHK(hipSetDevice(c->device));
  std::vector<double> ones;
  if (!rho) ones.assign(n, 1.0);
  CHK(lb3_upload(c, c->rho, rho ? rho : ones.data(), n, nullptr));
  if (u) {
    CHK(lb3_upload(c, c->u, u, 3 * n, nullptr));
  } else {
    HIPCHK(hipMemsetAsync(c->u, 0, 3 * n * c->es(), c->stream));
  }
  // the arguments of a step from f[cur ^ 1] write f[cur], the state
  if (c->precision)
    launch_k((lb3::k_lb3_equilibrium<float>), lb3_grid(c), dim3(lb3::kThreads), 0, c->stream, lb3_args<float>(c, c->cur ^ 1));
  else
    launch_k((lb3::k_lb3_equilibrium<double>), lb3_grid(c), dim3(lb3::kThreads), 0, c->stream, lb3_args<double>(c, c->cur ^ 1));
  HIPCHK(hipGetLastError());
  HIPCHK(hipStreamSynchronize(c->stream));
  c->have_moments = false;
  return EPDLB_OK;
}

int epdlb_lb3_set_force(epdlb_lb3* c, const double* F) {
  if (!c) return fail(EPDLB_EINVAL, "NULL context");
  HIPCHK(hipSetDevice(c->device));
  const size_t count = 3 * size_t(c->n);
  if (!F) {
    HIPCHK(hipMemsetAsync(c->F, 0, count * c->es(), c->stream));
    HIPCHK(hipStreamSynchronize(c->stream));
    return EPDLB_OK;
  }
  if (!all_finite(F, count)) return fail(EPDLB_EINVAL, "non-finite force");
  return lb3_upload(c, c->F, F, count, nullptr);
}

int epdlb_lb3_set_collision(epdlb_lb3* c, int32_t mrt, double gamma_s, double gamma_b, double gamma_g) {
  if (!c) return fail(EPDLB_EINVAL, "NULL context");
  if (mrt != 0 && mrt != 1) return fail(EPDLB_EINVAL, "mrt must be 0 or 1");
  if (mrt) {
    for (double g : {gamma_s, gamma_b, gamma_g})
      if (!(g > -1.0 && g < 1.0)) return fail(EPDLB_EINVAL, "gamma_s, gamma_b, gamma_g must lie in (-1, 1)");
    c->gs = gamma_s;
    c->gb = gamma_b;
    c->gg = gamma_g;
  }
  c->mrt = mrt;
  return EPDLB_OK;
}

int epdlb_lb3_step(epdlb_lb3* c, int64_t n) {
  if (!c) return fail(EPDLB_EINVAL, "NULL context");
  if (n < 0) return fail(EPDLB_EINVAL, "negative step count");
  HIPCHK(hipSetDevice(c->device));
  return lb3_steps(c, n, nullptr);
}

int epdlb_lb3_profile(epdlb_lb3* c, int32_t n, double* ms) {
  if (!c || !ms) return fail(EPDLB_EINVAL, "NULL argument");
  if (n < 1 || n > 4096) return fail(EPDLB_EINVAL, "n must lie in [1, 4096]");
  HIPCHK(hipSetDevice(c->device));
  while (c->ev.size() < size_t(2 * n)) {
    hipEvent_t e;
    HIPCHK(hipEventCreate(&e));
    c->ev.push_back(e);
  }
  const int r = lb3_steps(c, n, c->ev.data());
  tl_ev_start = tl_ev_stop = nullptr;
  CHK(r);
  HIPCHK(hipStreamSynchronize(c->stream));
  for (int s = 0; s < n; ++s) {
    float t = 0.f;
    HIPCHK(hipEventElapsedTime(&t, c->ev[2 * s], c->ev[2 * s + 1]));
    ms[s] = t;
  }
  return EPDLB_OK;
}

int epdlb_lb3_sync(epdlb_lb3* c) {
  if (!c) return fail(EPDLB_EINVAL, "NULL context");
  HIPCHK(hipSetDevice(c->device));
  HIPCHK(hipStreamSynchronize(c->stream));
  return EPDLB_OK;
}

int epdlb_lb3_read_populations(epdlb_lb3* c, double* f) {
  if (!c || !f) return fail(EPDLB_EINVAL, "NULL argument");
  HIPCHK(hipSetDevice(c->device));
  double w[lb3::kQ];
  for (int k = 0; k < lb3::kQ; ++k) w[k] = lb3_weight(k);
  return lb3_download(c, f, c->f[c->cur], size_t(lb3::kQ) * size_t(c->n), w);
}

int epdlb_lb3_read_velocity(epdlb_lb3* c, double* rho, double* u) {
  if (!c || !rho || !u) return fail(EPDLB_EINVAL, "NULL argument");
  if (!c->have_moments) return fail(EPDLB_ESTATE, "no step since the populations were set");
  HIPCHK(hipSetDevice(c->device));
  CHK(lb3_download(c, rho, c->rho, size_t(c->n), nullptr));
  return lb3_download(c, u, c->u, 3 * size_t(c->n), nullptr);
}

void epdlb_lb3_destroy(epdlb_lb3* c) {
  if (!c) return;
  if (c->stream) (void)hipStreamSynchronize(c->stream);
  for (hipEvent_t e : c->ev) (void)hipEventDestroy(e);
  if (c->mem) (void)hipFree(c->mem);
  if (c->own_stream && c->stream) (void)hipStreamDestroy(c->stream);
  delete c;
}

// ---------------------------------------------------------------------------
// Chain propagators and densities on a three-dimensional grid.
// ---------------------------------------------------------------------------
struct epdlb_epd3 {
  int device = 0;
  int nx = 0, ny = 0, nz = 0;
  long n = 0;
  int N = 0;
  double f_A = 0.5, phi_P = 0.1, R_G = 1.0, dx = 1.0;
  int precision = 0;
  void* mem = nullptr;
  void* w = nullptr;    // 3 planes
  void* phi = nullptr;  // 3 planes
  void* q = nullptr;    // N + 1 planes
  void* qb = nullptr;   // N + 1 planes
  void* C = nullptr;    // n complex
  double* part = nullptr;
  double* sums = nullptr;  // 16
  double* nodes = nullptr; // wA_j, wB_j: 2 (N + 1)
  std::vector<double> seg;  // A-content of each contour segment
  std::vector<hipEvent_t> ev;  // start/stop pairs of the timed FFT launches (epdlb_epd3_profile)
  size_t ev_used = 0;          // pairs armed in the current evaluation; 0 when not profiling
  bool profiling = false;
  hipStream_t stream = nullptr;
  bool own_stream = false;
  size_t es() const { return precision ? sizeof(float) : sizeof(double); }
};

namespace {

bool pow2_upto(int v, int m) { return v >= 1 && v <= m && (v & (v - 1)) == 0; }

template <typename T>
int p3_fft(epdlb_epd3* c, int axis, int mode, int fuse = 0, const T* q = nullptr, T* qn = nullptr, T a = T(0)) {
  epd3::LineArgs A;
  const long n = c->n;
  A.fuse = fuse;
  A.wA = c->w;
  A.wB = static_cast<const T*>(c->w) + n;
  A.q = q;
  A.qn = qn;
  A.sums = c->sums;
  A.inv_n = 1.0 / double(n);
  A.a = double(a);
  A.nx = c->nx;
  A.ny = c->ny;
  A.nz = c->nz;
  A.mode = mode;
  A.heat = c->R_G * c->R_G / c->N * (2.0 * M_PI / c->dx) * (2.0 * M_PI / c->dx);
  if (axis == 0) {
    A.L = c->nx; A.st = 1; A.count = long(c->ny) * c->nz; A.g = 1; A.gs = c->nx; A.gi = 0;
  } else if (axis == 1) {
    A.L = c->ny; A.st = c->nx; A.count = long(c->nx) * c->nz; A.g = c->nx; A.gs = long(c->nx) * c->ny; A.gi = 1;
  } else {
    A.L = c->nz; A.st = long(c->nx) * c->ny; A.count = long(c->nx) * c->ny; A.g = 1; A.gs = 1; A.gi = 0;
  }
  if (A.L == 1 && mode != 2 && fuse == 0) return EPDLB_OK;  // a transform of length 1 is the identity
  // strided lines (y, z): up to 16 neighbouring lines per block, interleaved
  // across lanes, with the LDS held to 96 KB; contiguous lines (x): half a
  // line's length of threads per line
  A.lb = 0;
  if (axis > 0) {
    long lb = 16;
    while (lb > 1 && (size_t(lb) * (2 * A.L + 2) + A.L) * sizeof(epd3::Cx<T>) > 98304) lb /= 2;
    A.lb = int(lb);
  }
  const long lines = A.lb > 0 ? A.lb : epd3::kThreads / (A.L > 1 ? A.L / 2 : 1);
  const size_t lds = (size_t(lines) * (2 * A.L + 2) + A.L) * sizeof(epd3::Cx<T>);
  const long blocks = (A.count + lines - 1) / lines;
  HIPCHK(prep_lds(epd3::k_p3_fft<T>, lds));
  if (c->profiling && 2 * c->ev_used + 1 < c->ev.size()) {
    tl_ev_start = c->ev[2 * c->ev_used];
    tl_ev_stop = c->ev[2 * c->ev_used + 1];
    ++c->ev_used;
  }
  launch_k((epd3::k_p3_fft<T>), dim3(unsigned(blocks)), dim3(epd3::kThreads), lds, c->stream,
           static_cast<epd3::Cx<T>*>(c->C), A);
  HIPCHK(hipGetLastError());
  return EPDLB_OK;
}

template <typename T> int p3_sum(epdlb_epd3* c, const T* a, int expo, const double* shift_sum, double* out) {
  launch_k((epd3::k_p3_sum<T>), dim3(epd3::kRedBlocks), dim3(epd3::kThreads), 0, c->stream, a, c->n, expo,
           shift_sum, 1.0 / double(c->n), c->part);
  HIPCHK(hipGetLastError());
  launch_k(epd3::k_p3_finish, dim3(1), dim3(epd3::kThreads), 0, c->stream, static_cast<const double*>(c->part),
           epd3::kRedBlocks, out);
  HIPCHK(hipGetLastError());
  return EPDLB_OK;
}

template <typename T> int p3_densities(epdlb_epd3* c) {
  const long n = c->n;
  const T* w = static_cast<const T*>(c->w);
  const T *wA = w, *wB = w + n, *wS = w + 2 * n;
  const double inv_n = 1.0 / double(n);
  const dim3 eg(unsigned(std::min<long>((n + epd3::kThreads - 1) / epd3::kThreads, 4096)));
  CHK(p3_sum<T>(c, wA, 0, nullptr, c->sums + 0));
  CHK(p3_sum<T>(c, wB, 0, nullptr, c->sums + 2));
  CHK(p3_sum<T>(c, wS, 0, nullptr, c->sums + 4));
  for (int chain = 0; chain < 2; ++chain) {
    T* q = static_cast<T*>(chain ? c->qb : c->q);
    launch_k((epd3::k_p3_fill<T>), eg, dim3(epd3::kThreads), 0, c->stream, q, T(1), n);
    HIPCHK(hipGetLastError());
    for (int j = 0; j < c->N; ++j) {
      const int seg = chain ? c->N - 1 - j : j;
      const T a = T(c->seg[seg]);
      // the half-step factors ride on the x passes: E q as the lines load, E Re / n as they store
      CHK(p3_fft<T>(c, 0, -1, 1, static_cast<const T*>(q + long(j) * n), nullptr, a));
      CHK(p3_fft<T>(c, 1, -1));
      CHK(p3_fft<T>(c, 2, 2));
      CHK(p3_fft<T>(c, 1, 1));
      CHK(p3_fft<T>(c, 0, 1, 2, nullptr, q + long(j + 1) * n, a));
    }
  }
  CHK(p3_sum<T>(c, static_cast<const T*>(c->q) + long(c->N) * n, 0, nullptr, c->sums + 6));
  CHK(p3_sum<T>(c, wS, 1, c->sums + 4, c->sums + 8));
  epd3::DensArgs D;
  D.N = c->N;
  D.n = n;
  D.V_over_dV = double(n);
  D.phiP = c->phi_P;
  D.wAn = c->nodes;
  D.wBn = c->nodes + (c->N + 1);
  D.sums = c->sums;
  D.inv_n = inv_n;
  launch_k((epd3::k_p3_density<T>), eg, dim3(epd3::kThreads), 0, c->stream, static_cast<const T*>(c->q),
           static_cast<const T*>(c->qb), wS, static_cast<T*>(c->phi), D);
  HIPCHK(hipGetLastError());
  return EPDLB_OK;
}

}  // namespace

int epdlb_epd3_create(int32_t nx, int32_t ny, int32_t nz, int32_t n_contour, double f_A, double phi_P, double R_G,
                      double dx, int32_t precision, int device, void* stream, epdlb_epd3** out) {
  if (!out) return fail(EPDLB_EINVAL, "out is NULL");
  *out = nullptr;
  if (!pow2_upto(nx, epd3::kMaxLen) || !pow2_upto(ny, epd3::kMaxLen) || !pow2_upto(nz, epd3::kMaxLen))
    return fail(EPDLB_EINVAL, "nx, ny, nz must be powers of two in [1, 512]");
  if (n_contour < 2 || n_contour > 256) return fail(EPDLB_EINVAL, "n_contour must be in [2, 256]");
  if (!(f_A > 0.0 && f_A < 1.0) || !(phi_P > 0.0 && phi_P < 1.0))
    return fail(EPDLB_EINVAL, "f_A and phi_P must lie in (0, 1)");
  if (!(R_G > 0.0) || !(dx > 0.0) || !std::isfinite(R_G) || !std::isfinite(dx))
    return fail(EPDLB_EINVAL, "R_G and dx must be finite and > 0");
  if (precision != 0 && precision != 1) return fail(EPDLB_EINVAL, "precision must be 0 or 1");
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || ndev <= device || device < 0)
    return fail(EPDLB_ENODEV, "no HIP device with that index");
  HIPCHK(hipSetDevice(device));
  hipDeviceProp_t prop;
  HIPCHK(hipGetDeviceProperties(&prop, device));
  if (std::strncmp(prop.gcnArchName, "gfx950", 6) != 0)
    return fail(EPDLB_ENODEV, std::string("library built for gfx950, device is ") + prop.gcnArchName);
  epdlb_epd3* c = new (std::nothrow) epdlb_epd3();
  if (!c) return fail(EPDLB_ENOMEM, "host allocation failed");
  c->device = device;
  c->nx = nx;
  c->ny = ny;
  c->nz = nz;
  c->n = long(nx) * ny * nz;
  c->N = n_contour;
  c->f_A = f_A;
  c->phi_P = phi_P;
  c->R_G = R_G;
  c->dx = dx;
  c->precision = precision;
  // contour tables: A-content of each segment and trapezoid node weights over the A and B parts
  const int N = n_contour;
  const double ds = 1.0 / N;
  c->seg.resize(N);
  for (int j = 0; j < N; ++j) c->seg[j] = std::min(1.0, std::max(0.0, f_A * N - j));
  std::vector<double> nodes(2 * size_t(N + 1), 0.0);
  for (int j = 0; j <= N; ++j) {
    if (j >= 1) {
      nodes[j] += 0.5 * ds * c->seg[j - 1];
      nodes[N + 1 + j] += 0.5 * ds * (1.0 - c->seg[j - 1]);
    }
    if (j <= N - 1) {
      nodes[j] += 0.5 * ds * c->seg[j];
      nodes[N + 1 + j] += 0.5 * ds * (1.0 - c->seg[j]);
    }
  }
  const size_t plane = align256(size_t(c->n) * c->es());
  const size_t cbytes = align256(size_t(c->n) * 2 * c->es());
  const size_t total = 3 * plane + 3 * plane + 2 * size_t(N + 1) * plane + cbytes +
                       align256(epd3::kRedBlocks * sizeof(double)) + align256(16 * sizeof(double)) +
                       align256(nodes.size() * sizeof(double));
  if (hipMalloc(&c->mem, total) != hipSuccess) {
    delete c;
    return fail(EPDLB_ENOMEM, "hipMalloc of the propagator planes failed");
  }
  unsigned char* b = static_cast<unsigned char*>(c->mem);
  c->w = b;
  b += 3 * plane;
  c->phi = b;
  b += 3 * plane;
  c->q = b;
  b += size_t(N + 1) * plane;
  c->qb = b;
  b += size_t(N + 1) * plane;
  c->C = b;
  b += cbytes;
  c->part = reinterpret_cast<double*>(b);
  b += align256(epd3::kRedBlocks * sizeof(double));
  c->sums = reinterpret_cast<double*>(b);
  b += align256(16 * sizeof(double));
  c->nodes = reinterpret_cast<double*>(b);
  if (stream) {
    c->stream = reinterpret_cast<hipStream_t>(stream);
  } else {
    if (hipStreamCreateWithFlags(&c->stream, hipStreamNonBlocking) != hipSuccess) {
      epdlb_epd3_destroy(c);
      return fail(EPDLB_EHIP, "hipStreamCreate failed");
    }
    c->own_stream = true;
  }
  if (hipMemcpyAsync(c->nodes, nodes.data(), nodes.size() * sizeof(double), hipMemcpyHostToDevice, c->stream) !=
          hipSuccess ||
      hipStreamSynchronize(c->stream) != hipSuccess) {
    epdlb_epd3_destroy(c);
    return fail(EPDLB_EHIP, "uploading the contour weights failed");
  }
  *out = c;
  return EPDLB_OK;
}

int epdlb_epd3_densities(epdlb_epd3* c, const double* omega, double* phi, double* Q_P, double* Q_S) {
  if (!c || !omega || !phi) return fail(EPDLB_EINVAL, "NULL argument");
  const size_t n = size_t(c->n);
  if (!all_finite(omega, 3 * n)) return fail(EPDLB_EINVAL, "non-finite potential");
  HIPCHK(hipSetDevice(c->device));
  if (c->precision) {
    std::vector<float> h(3 * n);
    for (size_t i = 0; i < 3 * n; ++i) h[i] = float(omega[i]);
    HIPCHK(hipMemcpyAsync(c->w, h.data(), h.size() * sizeof(float), hipMemcpyHostToDevice, c->stream));
    HIPCHK(hipStreamSynchronize(c->stream));
    CHK(p3_densities<float>(c));
    HIPCHK(hipMemcpyAsync(h.data(), c->phi, h.size() * sizeof(float), hipMemcpyDeviceToHost, c->stream));
    HIPCHK(hipStreamSynchronize(c->stream));
    for (size_t i = 0; i < 3 * n; ++i) phi[i] = h[i];
  } else {
    HIPCHK(hipMemcpyAsync(c->w, omega, 3 * n * sizeof(double), hipMemcpyHostToDevice, c->stream));
    CHK(p3_densities<double>(c));
    HIPCHK(hipMemcpyAsync(phi, c->phi, 3 * n * sizeof(double), hipMemcpyDeviceToHost, c->stream));
    HIPCHK(hipStreamSynchronize(c->stream));
  }
  double s[16];
  HIPCHK(hipMemcpyAsync(s, c->sums, sizeof(s), hipMemcpyDeviceToHost, c->stream));
  HIPCHK(hipStreamSynchronize(c->stream));
  const double dV = c->dx * c->dx * c->dx;
  if (Q_P) *Q_P = dV * s[6];
  if (Q_S) *Q_S = dV * s[8];
  if (!std::isfinite(s[6]) || !std::isfinite(s[8]) || !(s[6] > 0.0))
    return fail(EPDLB_ENONFINITE, "a partition function is not finite and positive");
  return EPDLB_OK;
}

int epdlb_epd3_time(epdlb_epd3* c, int32_t reps, double* ms) {
  if (!c || !ms) return fail(EPDLB_EINVAL, "NULL argument");
  if (reps < 1 || reps > 1000) return fail(EPDLB_EINVAL, "reps must lie in [1, 1000]");
  HIPCHK(hipSetDevice(c->device));
  hipEvent_t e0, e1;
  HIPCHK(hipEventCreate(&e0));
  if (hipEventCreate(&e1) != hipSuccess) {
    (void)hipEventDestroy(e0);
    return fail(EPDLB_EHIP, "hipEventCreate failed");
  }
  int r = hipEventRecord(e0, c->stream) == hipSuccess ? EPDLB_OK : EPDLB_EHIP;
  for (int k = 0; k < reps && r == EPDLB_OK; ++k) r = c->precision ? p3_densities<float>(c) : p3_densities<double>(c);
  float t = 0.f;
  if (r == EPDLB_OK && (hipEventRecord(e1, c->stream) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
                        hipEventElapsedTime(&t, e0, e1) != hipSuccess))
    r = fail(EPDLB_EHIP, "timing events failed");
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  CHK(r);
  *ms = double(t) / reps;
  return EPDLB_OK;
}

int epdlb_epd3_profile(epdlb_epd3* c, double* fft_ms, int32_t* fft_launches) {
  if (!c || !fft_ms || !fft_launches) return fail(EPDLB_EINVAL, "NULL argument");
  HIPCHK(hipSetDevice(c->device));
  const size_t need = 2 * size_t(10 * c->N + 2);
  while (c->ev.size() < need) {
    hipEvent_t e;
    HIPCHK(hipEventCreate(&e));
    c->ev.push_back(e);
  }
  c->profiling = true;
  c->ev_used = 0;
  const int r = c->precision ? p3_densities<float>(c) : p3_densities<double>(c);
  c->profiling = false;
  tl_ev_start = tl_ev_stop = nullptr;
  CHK(r);
  HIPCHK(hipStreamSynchronize(c->stream));
  double total = 0.0;
  for (size_t k = 0; k < c->ev_used; ++k) {
    float t = 0.f;
    HIPCHK(hipEventElapsedTime(&t, c->ev[2 * k], c->ev[2 * k + 1]));
    total += t;
  }
  *fft_ms = total;
  *fft_launches = int32_t(c->ev_used);
  return EPDLB_OK;
}

void epdlb_epd3_destroy(epdlb_epd3* c) {
  if (!c) return;
  if (c->stream) (void)hipStreamSynchronize(c->stream);
  for (hipEvent_t e : c->ev) (void)hipEventDestroy(e);
  if (c->mem) (void)hipFree(c->mem);
  if (c->own_stream && c->stream) (void)hipStreamDestroy(c->stream);
  delete c;
}
