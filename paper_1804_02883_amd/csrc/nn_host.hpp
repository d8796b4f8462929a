// Host side of the density surrogate: parameter layout, fragment packing,
// launchers, the surrogate stage of a simulation step, and the trainer
// object (epdlb_nn).  Included once by epdlb.hip after its internal helpers
// (error handling, launch_k/ProfScope, stages), whose translation unit it is
// part of.
#pragma once
#include "nn.hpp"

namespace {

struct NnOffsets {
  int W[4], b[4], total;
};
NnOffsets nn_offsets() {
  NnOffsets o{};
  int off = 0;
  for (int l = 0; l < nn::kLayers; ++l) {
    o.W[l] = off;
    off += 9 * nn::cin_of(l) * nn::cout_of(l);
    o.b[l] = off;
    off += nn::cout_of(l);
  }
  o.total = off;
  return o;
}

// Forward operator of layer l: stored input channels, 32-row output blocks.
int fwd_cis(int l) { return l == 0 ? nn::kXC : nn::kHid; }
int fwd_nb(int l) { return l == 3 ? 1 : 2; }
// Backward-data operator of layer l (1..3): input = gradient of z_l.
int bwd_cis(int l) { return l == 3 ? nn::kXC : nn::kHid; }
size_t frag_elems(int cis, int nb) { return size_t(9) * (cis / 16) * nb * 512; }

struct FragOffsets {
  size_t f[4], b[4], ftotal, btotal;
};
FragOffsets frag_offsets() {
  FragOffsets o{};
  size_t off = 0;
  for (int l = 0; l < 4; ++l) {
    o.f[l] = off;
    off += frag_elems(fwd_cis(l), fwd_nb(l));
  }
  o.ftotal = off;
  off = 0;
  o.b[0] = 0;
  for (int l = 1; l < 4; ++l) {
    o.b[l] = off;
    off += frag_elems(bwd_cis(l), 2);
  }
  o.btotal = off;
  return o;
}

hipError_t nn_pack(const float* w, __bf16* ffrag, __bf16* bfrag, hipStream_t s) {
  const NnOffsets o = nn_offsets();
  const FragOffsets fo = frag_offsets();
  for (int l = 0; l < 4; ++l) {
    nn::PackArgs a{w + o.W[l], nn::cin_of(l), nn::cout_of(l), fwd_cis(l), fwd_nb(l), l > 0 ? 1 : 0, 0,
                   ffrag + fo.f[l]};
    const size_t total = frag_elems(a.CIs, a.NB);
    hipLaunchKernelGGL(nn::k_pack, dim3(unsigned((total + 255) / 256)), dim3(256), 0, s, a);
  }
  if (bfrag)
    for (int l = 1; l < 4; ++l) {
      nn::PackArgs a{w + o.W[l], nn::cin_of(l), nn::cout_of(l), bwd_cis(l), 2, l < 3 ? 1 : 0, 1,
                     bfrag + fo.b[l]};
      const size_t total = frag_elems(a.CIs, a.NB);
      hipLaunchKernelGGL(nn::k_pack, dim3(unsigned((total + 255) / 256)), dim3(256), 0, s, a);
    }
  return hipGetLastError();
}

// Two workgroups of the 64-channel convolutions fit one CU (72 KB of LDS
// weights each); larger grids loop over tiles.
constexpr int kConvMaxBlocks = 512;
constexpr int kWgradMaxBlocks = 256;

// Compute units of the current device, cached per device (the first call
// happens at create time, outside any stream capture).
int device_cus() {
  static int cache[64] = {0};
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return 256;
  if (!cache[dev]) {
    int n = 0;
    if (hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || n <= 0) n = 256;
    cache[dev] = n;
  }
  return cache[dev];
}

// `a` carries tiles of kTW x kConvTH sites (ntiles over all samples); the
// 64-channel kernel re-tiles into 32-site rows, one workgroup per CU.
template <int CI, int EPI>
hipError_t conv_hidden(const nn::ConvArgs& a, hipStream_t s) {
  const size_t lds = size_t(9) * (CI / 16) * 2 * 64 * 16;
  if constexpr (CI == nn::kHid) {
    nn::ConvArgs b = a;
    const int nsamples = a.ntiles / a.tiles_per_sample;
    b.tiles_per_sample = (a.nx / nn::kTW) * a.ny;
    b.ntiles = b.tiles_per_sample * nsamples;
    constexpr int nw = nn::kConv64Threads / 64;
    const int grid = std::min(device_cus(), (b.ntiles + nw - 1) / nw);
    auto k = nn::k_conv64<EPI>;
    hipError_t e = prep_lds(k, lds);
    if (e != hipSuccess) return e;
    launch_k(k, dim3(grid), dim3(nn::kConv64Threads), lds, s, b);
  } else {
    auto k = nn::k_conv_hidden<CI, EPI>;
    hipError_t e = prep_lds(k, lds);
    if (e != hipSuccess) return e;
    launch_k(k, dim3(std::min(a.ntiles, kConvMaxBlocks)), dim3(nn::kConvThreads), lds, s, a);
  }
  return hipGetLastError();
}

template <typename T, int EPO>
hipError_t conv_out(const nn::OutArgs<T>& a, hipStream_t s, int* nblocks) {
  const size_t lds = size_t(9) * 4 * 1 * 64 * 16;
  *nblocks = std::min(a.ntiles, kConvMaxBlocks);
  launch_k(nn::k_conv_out<T, EPO>, dim3(*nblocks), dim3(nn::kConvThreads), lds, s, a);
  return hipGetLastError();
}

template <int CI, int CO, int TH>
hipError_t conv_wgrad(nn::WgradArgs a, int nsamples, hipStream_t s, int* nblocks) {
  a.tiles_per_sample = (a.nx / nn::kTW) * (a.ny / TH);
  a.ntiles = a.tiles_per_sample * nsamples;
  const int d = a.d;
  const size_t lds = size_t(nn::kTW + 2 * d) * (TH + 2 * d) * (CI + 8) * 2 + size_t(TH) * nn::kTW * (CO + 8) * 2;
  auto k = nn::k_conv_wgrad<CI, CO, TH>;
  hipError_t e = prep_lds(k, lds);
  if (e != hipSuccess) return e;
  *nblocks = std::min(a.ntiles, kWgradMaxBlocks);
  launch_k(k, dim3(*nblocks), dim3(576), lds, s, a);
  return hipGetLastError();
}

hipError_t wgrad_reduce(const float* part, const float* partb, int nblocks, int l, float* grad, hipStream_t s) {
  nn::WredArgs a;
  a.part = part;
  a.partb = partb;
  a.nblocks = nblocks;
  a.CIs = fwd_cis(l);
  a.COs = l == 3 ? nn::kXC : nn::kHid;
  a.in64 = l > 0 ? 1 : 0;
  a.out64 = l < 3 ? 1 : 0;
  a.cil = nn::cin_of(l);
  a.col = nn::cout_of(l);
  a.grad = grad;
  const int total = 9 * a.cil * a.col + a.col;
  hipLaunchKernelGGL(nn::k_wgrad_reduce, dim3((total + 255) / 256), dim3(256), 0, s, a);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Surrogate stage of a simulation step (density_mode 1): potentials ->
// network -> renormalised densities and the force source S.
//   mode 0: surrogate step; mode 1: after the exact densities (see k_nn_norm)
// ---------------------------------------------------------------------------
// defer (may be NULL): when the force's row shape can take it, the
// normalisation is not launched here but handed back (*defer filled, returns
// with *deferred = true) for stage_force_lb to fuse with its first pass.
template <typename T>
int stage_nn(epdlb_ctx* c, int mode, int use_corr, nn::NormArgs<T>* defer = nullptr, bool* deferred = nullptr) {
  const epdlb_params& p = c->p;
  const long n = long(p.nx) * p.ny;
  const NnOffsets o = nn_offsets();
  const FragOffsets fo = frag_offsets();
  T* w = c->ptr<T>(c->L.omega[c->cur]);
  T* phi = c->ptr<T>(c->L.phi);
  double* scal = c->ptr<double>(c->L.scal);
  __bf16* act0 = c->ptr<__bf16>(c->L.nn_act[0]);
  __bf16* act1 = c->ptr<__bf16>(c->L.nn_act[1]);
  const float* wts = c->ptr<float>(c->L.nn_w);
  const __bf16* ff = c->ptr<__bf16>(c->L.nn_frag);
  const int tps = (p.nx / nn::kTW) * (p.ny / nn::kConvTH);
  nn::ConvArgs a{};
  a.nx = p.nx;
  a.ny = p.ny;
  a.tiles_per_sample = a.ntiles = tps;
  a.bs = n * nn::kHid;
  {
    // first layer straight from the potentials
    nn::InArgs<T> ia{};
    ia.c = a;
    ia.c.wfrag = ff + fo.f[0];
    ia.c.bias = wts + o.b[0];
    ia.c.out = act0;
    ia.c.d = 1;
    ia.w = w;
    ia.mean = scal + kMeanA;
    ia.plane = n;
    ia.fA = float(p.f_A);
    ia.invN = float(1.0 / p.n_contour);
    // 32-site row tiles; two workgroups per CU
    ia.c.tiles_per_sample = ia.c.ntiles = (p.nx / nn::kTW) * p.ny;
    constexpr int nw = nn::kConvThreads / 64;
    const int grid = std::min(2 * device_cus(), (ia.c.ntiles + nw - 1) / nw);
    ProfScope ps(c, K_NN_CONV0);
    launch_k(nn::k_conv_in<T>, dim3(grid), dim3(nn::kConvThreads), size_t(9) * 2 * 64 * 16, c->stream, ia);
  }
  HIPCHK(hipGetLastError());
  // second hidden layer, then the third with the output taps' projection
  // fused into its epilogue (its activations are never stored)
  a.in = act0;
  a.in_bs = n * nn::kHid;
  a.wfrag = ff + fo.f[1];
  a.bias = wts + o.b[1];
  a.out = act1;
  a.d = nn::dil_of(1);
  {
    ProfScope ps(c, K_NN_CONV);
    HIPCHK((conv_hidden<nn::kHid, nn::EPI_FWD>(a, c->stream)));
  }
  float* proj = c->ptr<float>(c->L.nn_proj);
  a.in = act1;
  a.wfrag = ff + fo.f[2];
  a.bias = wts + o.b[2];
  a.out = nullptr;
  a.d = nn::dil_of(2);
  a.pfrag = ff + nn::kFwdFragElems;
  a.proj = proj;
  a.plane = n;
  {
    ProfScope ps(c, K_NN_CONV);
    HIPCHK((conv_hidden<nn::kHid, nn::EPI_FWD_PROJ>(a, c->stream)));
  }
  T* dst = mode == 0 ? phi : c->ptr<T>(c->L.nn_phin);
  const int nslots = int((n + 255) / 256);
  double* partials = c->ptr<double>(c->L.partials);
  {
    ProfScope ps(c, K_NN_OUT);
    launch_k(nn::k_nn_out_stencil<T>, dim3(unsigned(nslots)), dim3(256), 0, c->stream, (const float*)proj,
             wts + o.b[3], dst, partials, p.nx, p.ny, nn::dil_of(3));
  }
  HIPCHK(hipGetLastError());
  nn::NormArgs<T> r{};
  r.src = dst;
  r.phi = phi;
  r.part = partials;
  r.nslots = nslots;
  r.wS = w + 2 * n;
  r.stilde = c->ptr<T>(c->L.stilde);
  r.S = c->ptr<T>(c->L.S);
  r.corr = c->ptr<T>(c->L.nn_corr);
  r.scal = scal;
  r.n = n;
  r.sumA = p.f_A * p.phi_P * double(n);
  r.sumB = (1.0 - p.f_A) * p.phi_P * double(n);
  r.V = double(n) * p.dx * p.dx;
  r.phiSbar = 1.0 - p.phi_P;
  r.invDA = 1.0 / p.D_A;
  r.invDB = 1.0 / p.D_B;
  r.invDS = 1.0 / p.D_S;
  r.mode = mode;
  r.use_corr = use_corr;
  if (deferred) *deferred = false;
  if (defer && deferred && force_inv_lb_shape(c->sh_frow.R)) {
    *defer = r;
    *deferred = true;
    return EPDLB_OK;
  }
  {
    ProfScope ps(c, K_NN_NORM);
    launch_k(nn::k_nn_norm<T>, dim3(unsigned((n + 255) / 256)), dim3(256), 0, c->stream, r);
  }
  HIPCHK(hipGetLastError());
  return EPDLB_OK;
}

int stage_nn_any(epdlb_ctx* c, int mode, int use_corr) {
  return c->p.precision == 0 ? stage_nn<double>(c, mode, use_corr) : stage_nn<float>(c, mode, use_corr);
}

// One hybrid step in surrogate mode.  kind: 1/2 surrogate step (use_corr
// 0/1), 3/4 exact step (use_corr 0/1).
template <typename T>
int run_sur_step_t(epdlb_ctx* c, int kind) {
  const bool exact = kind >= 3;
  const int uc = (kind == 2 || kind == 4) ? 1 : 0;
  CHK(stage_advect_update<T>(c));
  if (exact) {
    {
      ProfScope ps(c, K_NN_RESET);
      // last-exact-step slots: kResidEx, kNnErrLast
      launch_k(nn::k_nn_reset, dim3(1), dim3(64), 0, c->stream, c->ptr<double>(c->L.scal),
               (1 << (kResidEx - kNnResid)) | (1 << (kNnErrLast - kNnResid)));
    }
    HIPCHK(hipGetLastError());
    CHK(stage_densities<T>(c, false));
  }
  nn::NormArgs<T> norm{};
  bool deferred = false;
  CHK(stage_nn<T>(c, exact ? 1 : 0, uc, &norm, &deferred));
  return stage_force_lb<T>(c, deferred ? &norm : nullptr);
}

int run_sur_step(epdlb_ctx* c, int kind) {
  return c->p.precision == 0 ? run_sur_step_t<double>(c, kind) : run_sur_step_t<float>(c, kind);
}

// Residual test (host side, one check interval behind the device): the
// device maxima are copied to pinned memory at every check point and read at
// the next one, so the stream never waits for the host.
int nn_check(epdlb_ctx* c) {
  if (c->snap_pending) {
    HIPCHK(hipEventSynchronize(c->snap_ev));
    const double r_nn = c->snap[0], r_ex = c->snap[1], err_last = c->snap[2];
    c->resid_nn_max = std::max(c->resid_nn_max, r_nn);
    // the surrogate is trusted while the last exact step measured its error within err_tol
    if (c->p.err_tol > 0.0) c->validated = err_last <= c->p.err_tol;
    // an exact step since the snapshot has already re-anchored the densities
    if (r_nn - r_ex > c->p.resid_tol && c->n_exact == c->snap_exact) {
      c->force_exact = true;
      ++c->n_triggered;
    }
    c->snap_pending = false;
  }
  double* scal = c->ptr<double>(c->L.scal);
  HIPCHK(hipMemcpyAsync(c->snap, scal + kNnResid, 3 * sizeof(double), hipMemcpyDeviceToHost, c->stream));
  HIPCHK(hipEventRecord(c->snap_ev, c->stream));
  launch_k(nn::k_nn_reset, dim3(1), dim3(64), 0, c->stream, scal, 1);
  HIPCHK(hipGetLastError());
  c->snap_pending = true;
  c->snap_exact = c->n_exact;
  return EPDLB_OK;
}

// Exact densities are the state right after seeding: evaluate the network
// once so that the first step's force differences surrogate densities.
int nn_after_seed(epdlb_ctx* c) {
  c->last_exact = true;
  c->force_exact = false;
  c->validated = false;
  c->n_exact = 0;
  c->n_triggered = 0;
  c->resid_nn_max = 0.0;
  c->snap_pending = false;
  launch_k(nn::k_nn_reset, dim3(1), dim3(64), 0, c->stream, c->ptr<double>(c->L.scal), 31);
  HIPCHK(hipGetLastError());
  if (!c->nn_ready) return EPDLB_OK;
  CHK(stage_nn_any(c, 1, 0));
  // the seed's comparison follows no surrogate step: not an in-use error
  launch_k(nn::k_nn_reset, dim3(1), dim3(64), 0, c->stream, c->ptr<double>(c->L.scal),
           1 << (kNnErrUse - kNnResid));
  HIPCHK(hipGetLastError());
  HIPCHK(hipStreamSynchronize(c->stream));
  return EPDLB_OK;
}

}  // namespace

// ---------------------------------------------------------------------------
// Trainer: dataset of (potentials -> densities) pairs on the device, forward
// and backward passes over mini-batches, Adam on FP32 master weights.
// ---------------------------------------------------------------------------
struct epdlb_nn {
  int device = 0;
  hipStream_t stream = nullptr;
  bool own_stream = false;
  int nx = 0, ny = 0;
  long n = 0;
  int capacity = 0, max_batch = 0;
  void* mem = nullptr;
  float *w = nullptr, *g = nullptr, *m = nullptr, *v = nullptr;
  __bf16 *ffrag = nullptr, *bfrag = nullptr;
  __bf16* x = nullptr;    // dataset inputs [slot][site][16]
  float* tgt = nullptr;   // dataset targets [slot][2][site]
  __bf16 *act[3] = {}, *zz[3] = {}, *g4 = nullptr, *gb[2] = {};
  float* pred = nullptr;  // [2][site]
  int* slots = nullptr;
  double* lpart = nullptr;
  float *wpart = nullptr, *wpartb = nullptr;
  double* stage = nullptr;  // 5 planes + 3 means for host uploads
  int adam_t = 0;
  int last_nblocks = 0;
  int last_count = 0;
  bool packed_bwd = false;
};

namespace {

int nn_forward_train(epdlb_nn* t, int count, double phi_scale) {
  const NnOffsets o = nn_offsets();
  const FragOffsets fo = frag_offsets();
  const long n = t->n;
  const int tps = (t->nx / nn::kTW) * (t->ny / nn::kConvTH);
  nn::ConvArgs a{};
  a.nx = t->nx;
  a.ny = t->ny;
  a.tiles_per_sample = tps;
  a.ntiles = tps * count;
  a.bs = n * nn::kHid;
  for (int l = 0; l < 3; ++l) {
    a.in = l == 0 ? t->x : t->act[l - 1];
    a.in_bs = n * (l == 0 ? nn::kXC : nn::kHid);
    a.slots = l == 0 ? t->slots : nullptr;
    a.wfrag = t->ffrag + fo.f[l];
    a.bias = t->w + o.b[l];
    a.out = t->act[l];
    a.zout = t->zz[l];
    a.d = nn::dil_of(l);
    hipError_t e = l == 0 ? conv_hidden<nn::kXC, nn::EPI_FWD_TRAIN>(a, t->stream)
                          : conv_hidden<nn::kHid, nn::EPI_FWD_TRAIN>(a, t->stream);
    HIPCHK(e);
  }
  nn::OutArgs<float> q{};
  q.in = t->act[2];
  q.in_bs = n * nn::kHid;
  q.wfrag = t->ffrag + fo.f[3];
  q.bias = t->w + o.b[3];
  q.plane = n;
  q.tgt = t->tgt;
  q.tgt_bs = 2 * n;
  q.slots = t->slots;
  q.gout = t->g4;
  q.inv_phiP = float(1.0 / phi_scale);
  const double M = double(count) * double(n) * 2.0;
  q.gscale = float(2.0 / (M * phi_scale));
  q.partials = t->lpart;
  q.nx = t->nx;
  q.ny = t->ny;
  q.d = nn::dil_of(3);
  q.tiles_per_sample = tps;
  q.ntiles = tps * count;
  HIPCHK((conv_out<float, nn::EPO_TRAIN>(q, t->stream, &t->last_nblocks)));
  return EPDLB_OK;
}

int nn_backward(epdlb_nn* t, int count) {
  const NnOffsets o = nn_offsets();
  const FragOffsets fo = frag_offsets();
  const long n = t->n;
  const int tps = (t->nx / nn::kTW) * (t->ny / nn::kConvTH);
  if (!t->packed_bwd) {
    HIPCHK(nn_pack(t->w, t->ffrag, t->bfrag, t->stream));
    t->packed_bwd = true;
  }
  nn::ConvArgs a{};
  a.nx = t->nx;
  a.ny = t->ny;
  a.tiles_per_sample = tps;
  a.ntiles = tps * count;
  a.bs = n * nn::kHid;
  nn::WgradArgs wa{};
  wa.nx = t->nx;
  wa.ny = t->ny;
  wa.part = t->wpart;
  wa.partb = t->wpartb;
  int nb = 0;
  // layer 3: dL/dz_2 = conv^T(g4) * SiLU'(z_2); dW_3 from (a_2, g4)
  a.in = t->g4;
  a.in_bs = n * nn::kXC;
  a.wfrag = t->bfrag + fo.b[3];
  a.zin = t->zz[2];
  a.out = t->gb[0];
  a.d = nn::dil_of(3);
  HIPCHK((conv_hidden<nn::kXC, nn::EPI_BWD>(a, t->stream)));
  wa.a = t->act[2];
  wa.a_bs = n * nn::kHid;
  wa.slots = nullptr;
  wa.g = t->g4;
  wa.g_bs = n * nn::kXC;
  wa.d = nn::dil_of(3);
  HIPCHK((conv_wgrad<nn::kHid, nn::kXC, 4>(wa, count, t->stream, &nb)));
  HIPCHK(wgrad_reduce(t->wpart, t->wpartb, nb, 3, t->g + o.W[3], t->stream));
  // layers 2 and 1
  __bf16* gin = t->gb[0];
  __bf16* gout = t->gb[1];
  for (int l = 2; l >= 1; --l) {
    a.in = gin;
    a.in_bs = n * nn::kHid;
    a.wfrag = t->bfrag + fo.b[l];
    a.zin = t->zz[l - 1];
    a.out = gout;
    a.d = nn::dil_of(l);
    HIPCHK((conv_hidden<nn::kHid, nn::EPI_BWD>(a, t->stream)));
    wa.a = t->act[l - 1];
    wa.a_bs = n * nn::kHid;
    wa.g = gin;
    wa.g_bs = n * nn::kHid;
    wa.d = nn::dil_of(l);
    HIPCHK((conv_wgrad<nn::kHid, nn::kHid, 8>(wa, count, t->stream, &nb)));
    HIPCHK(wgrad_reduce(t->wpart, t->wpartb, nb, l, t->g + o.W[l], t->stream));
    std::swap(gin, gout);
  }
  // layer 0: dW_0 from (x, dL/dz_0)
  wa.a = t->x;
  wa.a_bs = n * nn::kXC;
  wa.slots = t->slots;
  wa.g = gin;
  wa.g_bs = n * nn::kHid;
  wa.d = 1;
  HIPCHK((conv_wgrad<nn::kXC, nn::kHid, 8>(wa, count, t->stream, &nb)));
  HIPCHK(wgrad_reduce(t->wpart, t->wpartb, nb, 0, t->g + o.W[0], t->stream));
  return EPDLB_OK;
}

int nn_upload_slots(epdlb_nn* t, const int32_t* slots, int count) {
  if (!slots || count < 1 || count > t->max_batch) return fail(EPDLB_EINVAL, "slot list size out of range");
  nn::SlotList L{};
  L.n = count;
  for (int i = 0; i < count; ++i) {
    if (slots[i] < 0 || slots[i] >= t->capacity) return fail(EPDLB_EINVAL, "slot index out of range");
    L.s[i] = slots[i];
  }
  hipLaunchKernelGGL(nn::k_set_slots, dim3(1), dim3(nn::kMaxBatch), 0, t->stream, L, t->slots);
  HIPCHK(hipGetLastError());
  return EPDLB_OK;
}

}  // namespace
