/* epdlb -- hybrid Lattice Boltzmann / External Potential Dynamics step on MI355X (gfx950).
 *
 * C ABI of libepdlb.so.  The method is that of Heuser, Sevink and Schmid,
 * "Self-assembly of polymeric particles in Poiseuille flow: a hybrid Lattice
 * Boltzmann / External Potential Dynamics simulation study" (arXiv:1804.02883):
 * one hybrid step advects the composition and potential fields with the flow,
 * updates the EPD potentials with the chemical potential (Sec. II, Eq. diff_w),
 * evaluates the chain propagators and densities (Sec. II, split step and
 * Eq. phi_s), reconstructs the longitudinal force from the diffusive change in
 * composition (Sec. II, k-space force), and advances a D2Q9 lattice Boltzmann
 * fluid with that force plus the reverse-Poiseuille drive (Eq. LB_prop,
 * Eq. force_col, Eq. force_field_2); the order follows the flow chart of App. C.
 *
 * Conventions for every function below:
 *  - Return value 0 (EPDLB_OK) on success, a negative EPDLB_E* code otherwise;
 *    epdlb_last_error() then returns a message (thread-local).  No function
 *    aborts the process.
 *  - Host arrays are caller-owned, FP64, planes of nx*ny values in row-major
 *    [y][x] order (x contiguous); multi-plane arrays are plane after plane.
 *  - Device memory is owned by the context (or by the caller when a workspace
 *    is passed to epdlb_create).  Work is queued on the context's stream;
 *    epdlb_step returns before the GPU finishes; reads synchronise the stream.
 *  - A context is used by one host thread at a time.
 */
#ifndef EPDLB_H
#define EPDLB_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define EPDLB_ABI_VERSION 1

/* Opaque simulation context; owns (or borrows) all device memory of one replica. */
typedef struct epdlb_ctx epdlb_ctx;

enum {
  EPDLB_OK = 0,
  EPDLB_EINVAL = -1,     /* bad argument, shape or parameter */
  EPDLB_ENOMEM = -2,     /* device allocation failed or workspace too small */
  EPDLB_EHIP = -3,       /* a HIP runtime call failed */
  EPDLB_ENONFINITE = -4, /* a partition function, field mean, LB density or velocity became non-finite */
  EPDLB_EUNSTABLE = -5,  /* the LB flow left its stable range: |u| > mach_max c_s, or a negative population */
  EPDLB_ESTATE = -6,     /* call out of order (e.g. step before seed) */
  EPDLB_ENODEV = -7      /* no usable gfx950 device */
};

/* Model and run parameters.  Field names follow the paper's notation
 * (Sec. II model, Sec. III units and parameter set, Sec. IV driving force).
 * Fill with epdlb_params_default() and override. */
typedef struct {
  int32_t abi_version;   /* must be EPDLB_ABI_VERSION */
  int32_t nx, ny;        /* grid; powers of two, 32 <= nx <= 1024, 16 <= ny <= 1024 */
  int32_t n_contour;     /* N: segments per chain (ds = 1/N), 2 <= N <= 256 */
  double f_A;            /* A fraction of the diblock, 0 < f_A < 1 */
  double phi_P;          /* mean copolymer volume fraction, 0 < phi_P < 1 */
  double chi_AB, chi_AS, chi_BS; /* Flory-Huggins parameters */
  double kappa_H;        /* Helfand compressibility parameter */
  double D_S, D_A, D_B;  /* diffusion constants */
  double R_G;            /* radius of gyration (length unit) */
  double dx, dt;         /* grid spacing and time step (shared by EPD and LB) */
  double kT_over_v;      /* 1/(beta v): scales the reconstructed force */
  double lb_tau;         /* LB relaxation time (BGK), > 1/2 */
  double g;              /* reverse-Poiseuille force amplitude */
  int32_t g_units;       /* 0: g in f* = rho R_G / tau^2; 1: g in lattice units */
  int32_t precision;     /* 0: FP64 everywhere; 1: FP32 fields, FP64 reductions */
  int32_t init_flow;     /* 1: start LB from the analytic profile (Eq. flow_field) */
  int32_t couple_lb;     /* 1: flow advects the fields and the polymer force drives the flow */
  /* Density evaluation.  0: chain propagators every step (Sec. II).  1: the
   * convolutional surrogate (epdlb_surrogate_set_weights) between exact
   * steps; an exact step every fallback_every steps and whenever the
   * surrogate's incompressibility residual max|sum_I Phi_I - 1| exceeds the
   * last exact step's by more than resid_tol.  The residual is read by the
   * host every check_every steps, one interval behind the device, so a
   * triggered exact step comes at most 2*check_every steps late.  With
   * err_tol > 0 the surrogate is used only while the last exact step
   * measured its density error (max over sites, A and B, of
   * |Phi_NN - Phi_exact|) within err_tol; otherwise every step is exact (in
   * particular from seeding until the first such measurement is read). */
  int32_t density_mode;
  int32_t fallback_every; /* default 50 */
  int32_t check_every;    /* default 10 */
  double resid_tol;       /* default 1e-3 */
  double err_tol;         /* default 1e-3; 0 disables the requirement */
  /* LB collision (Sec. II).  0: BGK with relaxation time lb_tau and the
   * second-order force term.  1: multi-relaxation D2Q9 in moment space: the
   * traceless non-equilibrium stress keeps lb_gamma_s of itself, its trace
   * lb_gamma_b, the three non-hydrodynamic modes lb_gamma_g; the force term
   * of Eq. force_col adds to the stress, in the two-dimensional trace split,
   *   Sigma = (1 + gamma_s)/2 [u F + F u - (u.F) I] + (1 + gamma_b)/2 (u.F) I,
   * and F to the momentum.  Lattice viscosities (rho = 1):
   *   nu = (1/6)(1 + gamma_s)/(1 - gamma_s), nu_B = (1/6)(1 + gamma_b)/(1 - gamma_b);
   * lb_tau is then unused.  Each gamma must lie in (-1, 1).  The paper's
   * eta = eta_B = 1 R_G^2/tau rho at dx = R_G/3, dt = 0.002 tau gives
   * gamma_s = gamma_b = -0.8050541516245486 (lattice nu = 0.018). */
  int32_t lb_mrt;         /* default 0 */
  double lb_gamma_s, lb_gamma_b, lb_gamma_g; /* defaults 0 */
  /* Omega after convection (App. C, flow chart and its comments 1-3).
   * 0: the auxiliary convection of omega alone.  1: the convected composition
   * Phi~ is inverted, starting from the auxiliary-convected omega: Fletcher-
   * Reeves conjugate gradients on the convex functional
   *   G(omega) = (V phibar_P/N) ln Q_P + V phibar_S ln Q_S + dA sum_I sum_r omega_I Phi~_I
   * (gradient dA (Phi~ - Phi[omega])), one secant line search per iteration
   * (two density evaluations), until sqrt(sum_I sum_r (Phi~_I - Phi_I)^2 / (nx ny))
   * < cg_tol or cg_max_iter iterations (then the step goes on with the last
   * iterate; epdlb_cg_stats counts it).  Steps then run eagerly (the host
   * reads two sums per line search), not as captured graphs.  Needs
   * density_mode 0 and a single context (no batch); FP32 fields need
   * cg_tol >= 1e-6.  Allocates 18 field planes of scratch at create. */
  int32_t cg_invert;      /* default 0 */
  int32_t cg_max_iter;    /* default 1000 */
  double cg_tol;          /* default 1e-8 (the paper's N_tr) */
  /* 1: precondition the inversion (also epdlb_invert_densities) by the local
   * density response: directions from s / (N Phi_A, N Phi_B, Phi_S) at the
   * current iterate, factor (s.z)_new / (s.z)_old.  Same solution and
   * stopping test, fewer iterations; 0 (default): the paper's plain iteration. */
  int32_t cg_precond;
  /* Flow guard of the LB step (Sec. II: the lattice speed of sound
   * c_s = dx/(dt sqrt 3), 1/sqrt 3 in lattice units).  Every LB launch checks
   * each site; the next epdlb_sync (epdlb_batch_sync) returns EPDLB_EUNSTABLE
   * once some step produced |u| > mach_max c_s or a negative post-collision
   * population, and EPDLB_ENONFINITE once it produced a density or velocity
   * that is not finite.  The flags stay raised until the state is replaced
   * (seed, set_fields, set_state).  Default 0.5; 0 disables the speed test
   * (the other two tests stay on). */
  double mach_max;
} epdlb_params;

/* Observables of the current densities (Sec. III and IV).  Phi_P = Phi_A +
 * Phi_B is formed in the storage precision; sums are FP64. */
typedef struct {
  double sigma;          /* (1/V) sum |Phi_P - phi_P| (Sec. III, mixing measure sigma(t)) */
  double y2p;            /* Eq. width: sqrt(sum_y y^2 <Phi_P>_x / (phi_P sum_y y^2)), y = row + 1/2 - ny/2 */
  int32_t n_particles;   /* connected clusters of sites with Phi_P >= threshold (Sec. IV) */
  int32_t n_wrapping;    /* of which reach half the box in x or y */
} epdlb_obs;

/* One particle: sites with Phi_P >= threshold connected through nearest
 * neighbours on the periodic grid. */
typedef struct {
  int32_t label;         /* lowest flat site index y * nx + x of the particle */
  int32_t area;          /* number of sites */
  int32_t wraps;         /* 1: offsets from the label site reach half the box (tensor not meaningful) */
  int32_t born;          /* epdlb_track_particles: 1 if no site was a particle site at the previous sample; else 0 */
  double content;        /* N = sum of Phi_P over the sites */
  double cx, cy;         /* Phi_P-weighted centroid, in site units inside the box */
  double gxx, gxy, gyy;  /* Eq. gyration_tensor, positions as minimum-image offsets from the label site */
  double R, c_rel;       /* Eq. asph R = sqrt(lambda_+ + lambda_-), Eq. rel_asph c_rel = c^2 / R^4 (0 if R = 0) */
} epdlb_particle;

/* Scalars maintained on the device (FP64). */
typedef struct {
  int64_t step;          /* hybrid steps taken since seeding */
  double Q_P;            /* single-chain partition function (forward chain) */
  double Q_P_bwd;        /* same from the backward chain (equal up to rounding) */
  double Q_S;            /* solvent partition function (with gauge_S below) */
  double gauge_S;        /* constant subtracted from omega_S for Q_S */
  double mean_omega[3];  /* site means of omega_A, omega_B, omega_S */
  /* density_mode 1 (zero otherwise) */
  int64_t n_exact;       /* exact steps since seeding */
  int64_t n_triggered;   /* of which forced by the residual test */
  double nn_err_last;    /* max over sites, A and B, of |Phi_NN - Phi_exact| at the last exact step */
  double nn_err_max;     /* maximum of nn_err_last over all exact steps (and the seed) */
  double resid_nn_max;   /* max |sum_I Phi_I - 1| over surrogate steps since seeding */
  double resid_exact;    /* the same for the last exact step */
  double nn_err_in_use;  /* max of nn_err_last over exact steps that ended a run of surrogate steps */
} epdlb_diag;

/* Stage identifiers for epdlb_run_stage (one hybrid step = 1, 2, 3, 4). */
enum {
  EPDLB_STAGE_ADVECT_UPDATE = 1, /* Phi, omega, u -> omega', S~ = sum Phi~_I / D_I */
  EPDLB_STAGE_DENSITIES = 2,     /* omega -> propagators -> Phi, Q_P, and S = sum Phi_I/D_I - S~ */
  EPDLB_STAGE_FORCE = 3,         /* S -> lattice force F (polymer + external) */
  EPDLB_STAGE_LB = 4             /* f*, F -> stream/collide -> f*', rho, u */
};

/* Auxiliary planes for epdlb_read_aux / epdlb_write_aux. */
enum {
  EPDLB_AUX_STILDE = 1, /* 1 plane */
  EPDLB_AUX_S = 2,      /* 1 plane */
  EPDLB_AUX_FORCE = 3   /* 2 planes: F_x, F_y in lattice units */
};

/* Fill *p with the paper's defaults (Sec. III: R_G = D_S = 1, D_A = D_B = D_S/N,
 * dx = R_G/3, dt = 0.002 tau; 32x32 grid, N = 16).  Host only. */
int epdlb_params_default(epdlb_params* p);

/* Check *p without touching a GPU.  Host only. */
int epdlb_validate(const epdlb_params* p);

/* Relaxation factors of the multi-relaxation collision from the shear and
 * bulk viscosities (Sec. II viscosity relations, with the lattice speed of
 * sound c_s^2 = dx^2/(3 dt^2)):
 *   eta   = (dt rho c_s^2 / 2) (1 + gamma_s)/(1 - gamma_s),
 *   eta_B = (dt rho c_s^2 / d) (1 + gamma_b)/(1 - gamma_b),
 * d = dim (2 for epdlb_params.lb_gamma_s/_b, 3 for epdlb_lb3_set_collision).
 * The paper's eta = eta_B = 1 R_G^2 rho/tau at dx = R_G/3, dt = 0.002 tau
 * gives gamma_s = gamma_b = -0.8050541516245486 in two dimensions.
 * EINVAL for a non-positive or non-finite argument, dim other than 2 or 3,
 * or a NULL output.  Host only. */
int epdlb_mrt_gammas(double eta, double eta_B, double rho, double dx, double dt, int32_t dim,
                     double* gamma_s, double* gamma_b);

/* Device bytes a context for *p needs when the caller supplies the workspace.  Host only. */
int epdlb_workspace_bytes(const epdlb_params* p, size_t* bytes);

/* Initial noise: out[3*nx*ny] = sigma * xi, xi standard normal from SplitMix64
 * in counter mode with Box-Muller pairs (species A, B, S; then y; then x).
 * The paper starts from a homogeneous mixture plus tiny noise (Sec. III).  Host only. */
int epdlb_noise_fill(uint64_t seed, double sigma, int32_t nx, int32_t ny, double* out);

/* Create a context on HIP device `device`.  `stream` is a hipStream_t (NULL:
 * the context creates its own).  `workspace` is device memory of at least
 * epdlb_workspace_bytes() bytes that stays owned by the caller (NULL: the
 * context allocates).  On success *out is the new context. */
int epdlb_create(const epdlb_params* p, int device, void* stream, void* workspace,
                 size_t workspace_bytes, epdlb_ctx** out);

/* omega_I = sigma * noise(seed), Phi = Phi[omega], LB at f^eq(rho = 1, u_init). */
int epdlb_seed(epdlb_ctx* ctx, uint64_t seed, double sigma);

/* Same with caller-given potentials omega[3*nx*ny]. */
int epdlb_set_fields(epdlb_ctx* ctx, const double* omega);

/* Upload a full state: omega[3], phi[3], post-collision populations fstar[9]
 * (D2Q9 order c = (0,0),(1,0),(0,1),(-1,0),(0,-1),(1,1),(-1,1),(-1,-1),(1,-1))
 * and velocity u[2] (lattice units).  Phi is taken as given. */
int epdlb_set_state(epdlb_ctx* ctx, const double* omega, const double* phi,
                    const double* fstar, const double* u);

/* Download the state in the layout epdlb_set_state takes (checkpoint): a
 * context given it continues the run (to rounding: the restore recomputes
 * the FP64 field means with another summation order).  Synchronises. */
int epdlb_get_state(epdlb_ctx* ctx, double* omega, double* phi, double* fstar, double* u);

/* Device addresses of the current state planes, row-major [y][x], plane
 * stride nx*ny elements of FP64 (precision 0) or FP32 (precision 1), inside
 * the context's workspace.  Valid until the next call that steps or resets
 * the context (omega and the populations alternate between two buffers).
 * Reading them races with queued steps unless ordered on the context's
 * stream; writing them is undefined. */
typedef struct {
  int32_t precision;
  int64_t plane;        /* elements per plane */
  const void* omega;    /* 3 planes: A, B, S */
  const void* phi;      /* 3 planes */
  const void* rho;      /* 1 plane */
  const void* u;        /* 2 planes, lattice units */
} epdlb_dev_views;
int epdlb_device_views(epdlb_ctx* ctx, epdlb_dev_views* out);

/* Queue n hybrid steps on the context stream. */
int epdlb_step(epdlb_ctx* ctx, int64_t n);

/* Queue one stage of a step (EPDLB_STAGE_*), for per-stage checks. */
int epdlb_run_stage(epdlb_ctx* ctx, int32_t stage);

/* Wait for queued work.  Returns EPDLB_ENONFINITE when a partition function,
 * a field mean, or an LB density or velocity became non-finite, and
 * EPDLB_EUNSTABLE when the flow guard (epdlb_params.mach_max) tripped, in
 * any step since the state was last replaced. */
int epdlb_sync(epdlb_ctx* ctx);

/* Copy current fields to host (FP64, nx*ny each). */
int epdlb_read_densities(epdlb_ctx* ctx, double* phiA, double* phiB, double* phiS);
int epdlb_read_fields(epdlb_ctx* ctx, double* wA, double* wB, double* wS);
int epdlb_read_velocity(epdlb_ctx* ctx, double* rho, double* ux, double* uy);
int epdlb_read_populations(epdlb_ctx* ctx, double* fstar /* 9*nx*ny */);
int epdlb_read_aux(epdlb_ctx* ctx, int32_t which, double* out);
int epdlb_write_aux(epdlb_ctx* ctx, int32_t which, const double* in);
int epdlb_read_diag(epdlb_ctx* ctx, epdlb_diag* d);

/* Observables of the current densities (after seed/set_fields/set_state and
 * any steps; stream-ordered, synchronises the context's stream).
 * threshold: particle threshold on Phi_P (the paper's 0.5).  particles: host
 * array of max_particles entries (may be NULL when max_particles = 0); the
 * first min(n_particles, max_particles) particles in increasing label order
 * are written.  labels: NULL or a host int32 array of nx * ny ([y][x]): the
 * particle label of each site, -1 off the particles.  The first call
 * allocates device scratch of about 100 bytes per site, held until destroy.
 * EINVAL on a bad argument, ESTATE before any state. */
int epdlb_observables(epdlb_ctx* c, double threshold, epdlb_obs* out, epdlb_particle* particles,
                      int32_t max_particles, int32_t* labels);

/* Nucleation events (Sec. IV, nucleation stage): the observables of the
 * current densities as epdlb_observables computes them, and the particles
 * none of whose sites was a particle site (Phi_P >= the threshold of that
 * call) at the previous tracking call, i.e. nuclei formed since then.  The
 * first call after create, seed, set_fields or epdlb_track_reset counts
 * every particle (set_state keeps the previous sample: it resumes a run).  events: host array of max_events entries (NULL if
 * max_events = 0), the first min(n_events, max_events) new particles in label
 * order with born = 1; n_events: their number.  Sample often enough that a
 * particle moves less than its own size between calls, or it is counted
 * again.  The particle sites of this call are kept (one byte per site, in
 * the observables scratch) for the next.  Synchronises the stream.  EINVAL on
 * a bad argument or a batch replica group, ESTATE before any state. */
int epdlb_track_particles(epdlb_ctx* c, double threshold, epdlb_obs* out, epdlb_particle* events,
                          int32_t max_events, int32_t* n_events);
/* Forget the previous tracking sample. */
int epdlb_track_reset(epdlb_ctx* c);

/* sigma_Delta (Sec. III): (1/V) sum |Phi_P^a - Phi_P^b| over two contexts on
 * the same device with the same grid and precision (e.g. runs with and
 * without LB coupling from the same start).  Synchronises both streams. */
int epdlb_sigma_delta(epdlb_ctx* a, epdlb_ctx* b, double* out);

/* epdlb_sigma_delta for callers that cannot allocate device memory (serving
 * loops, harnesses that forbid hipMalloc): the same value, computed with no
 * allocation.  The partial sums live in a fixed library array of 64 KiB on
 * each device, held until the process ends, which limits the grid to
 * 1024 x 1024 sites (EINVAL above).  Every call on a device shares that
 * array: calls that overlap on one device race; each call writes every slot
 * it reads, so nothing needs clearing between calls.  Synchronises both
 * streams.  Errors as epdlb_sigma_delta. */
int epdlb_sigma_delta_noalloc(epdlb_ctx* a, epdlb_ctx* b, double* out);

/* Result of one Phi -> omega inversion (App. C, comments 2 and 3). */
typedef struct {
  int32_t iters;         /* Fletcher-Reeves iterations taken */
  int32_t evals;         /* density evaluations (2 per iteration + 1, + 1 per restart) */
  int32_t restarts;      /* directions replaced by the steepest descent */
  int32_t converged;     /* 1: resid < tolerance */
  double resid0;         /* RMS of Phi[omega] - Phi~ over the three fields at the start */
  double resid;          /* the same at the end */
} epdlb_cg_info;

/* Potentials that reproduce a given composition: starting from the context's
 * current omega, iterate as for cg_invert = 1 (any cg_invert setting) towards
 * Phi[omega] = phi_target, at most max_iter iterations (0: only measure the
 * residual), tolerance tol on the RMS residual.  phi_target: host, 3 * nx * ny
 * doubles, planes A, B, S, each [y][x], every value > 0; it should carry the
 * context's totals (sum Phi_A = f_A phi_P nx ny, sum Phi_B = (1 - f_A) phi_P
 * nx ny, sum Phi_S = (1 - phi_P) nx ny), which no omega can change.  The
 * result replaces omega and the densities become Phi[omega].  Each field is
 * determined up to an additive constant.  info (may be NULL) gets the counts
 * and residuals; an unconverged run still returns EPDLB_OK with
 * info->converged = 0 (also when the residual turns non-finite, which ends
 * the iteration at once).  Synchronises the stream.  EINVAL on bad arguments, a
 * batch replica group or density_mode 1; ESTATE before any state; ENOMEM if
 * the scratch (18 field planes, allocated once) cannot be allocated. */
int epdlb_invert_densities(epdlb_ctx* ctx, const double* phi_target, int32_t max_iter, double tol,
                           epdlb_cg_info* info);

/* The last inversion's result (an inversion step or a direct call) and
 * running totals: totals[0] inversions, [1] iterations, [2] density
 * evaluations, [3] unconverged inversions.  Either pointer may be NULL. */
int epdlb_cg_stats(epdlb_ctx* ctx, epdlb_cg_info* last, int64_t* totals /* 4 */);

/* Launch shape of one FFT pass family: R values per lane, nf transforms per
 * block, and the time per launch the autotuner measured (0 if not tuned). */
typedef struct {
  char family[16];       /* "prop_row", "prop_col", "force_row" or "force_col" */
  int32_t R, nf;
  double us;
} epdlb_shape;

/* Time the candidate launch shapes of every FFT pass family on this grid
 * (each candidate as a captured graph of `reps` launches) and keep the
 * fastest.  Only scratch planes are written; the simulation state is kept.
 * `cache_path` (nullable) is a text file of earlier results that is read
 * first and appended to.  Host-synchronous. */
int epdlb_autotune(epdlb_ctx* ctx, int32_t reps, const char* cache_path);
int epdlb_get_shapes(epdlb_ctx* ctx, epdlb_shape* out, int32_t cap, int32_t* n_out);
/* Force one family's shape; EPDLB_EINVAL if it cannot be launched. */
int epdlb_set_shape(epdlb_ctx* ctx, const char* family, int32_t R, int32_t nf);

/* Per-kernel timing with HIP events recorded on the context stream around
 * each launch, for the next `max_launches` launches (later launches are not
 * recorded; recording never blocks). */
typedef struct {
  char name[32];         /* kernel family, e.g. "prop_row" */
  int64_t launches;      /* launches recorded */
  double total_ms, min_ms, max_ms;
} epdlb_kernel_stat;
int epdlb_profile_start(epdlb_ctx* ctx, int32_t max_launches);

/* Synchronise, resolve the recorded events into at most `cap` per-family
 * entries (*n_out of them), and stop recording. */
int epdlb_profile_read(epdlb_ctx* ctx, epdlb_kernel_stat* out, int32_t cap, int32_t* n_out);

/* Release the context (device memory it allocated, its own stream). */
void epdlb_destroy(epdlb_ctx* ctx);

/* ---------------------------------------------------------------------------
 * Batched replicas.  Many independent runs (the paper averages 50-100 runs per
 * parameter set, Sec. IV) advanced together: replicas may differ in grid
 * (nx, ny), drive g and A fraction f_A, and must agree in every other model
 * parameter.  Replicas of one grid shape and A fraction share every kernel
 * launch; one captured graph advances all of them per step pair.  Replica indices follow
 * the order of `params`.
 * ------------------------------------------------------------------------- */
typedef struct epdlb_batch epdlb_batch;

/* `params[n_replicas]`; `stream` as in epdlb_create.  Device memory is
 * allocated by the batch. */
int epdlb_batch_create(const epdlb_params* params, int32_t n_replicas, int device, void* stream,
                       epdlb_batch** out);
/* omega of replica r = sigma * noise(seeds[r]); Phi = Phi[omega]; LB at rest + u_init. */
int epdlb_batch_seed(epdlb_batch* b, const uint64_t* seeds, double sigma);
/* Replace one replica's potentials (after seeding); its LB restarts. */
int epdlb_batch_set_fields(epdlb_batch* b, int32_t replica, const double* omega);
/* Queue n hybrid steps of every replica on the batch stream. */
int epdlb_batch_step(epdlb_batch* b, int64_t n);
int epdlb_batch_sync(epdlb_batch* b);
/* Per-replica reads, as the single-context reads (host FP64, nx*ny each). */
int epdlb_batch_read_densities(epdlb_batch* b, int32_t replica, double* phiA, double* phiB, double* phiS);
int epdlb_batch_read_fields(epdlb_batch* b, int32_t replica, double* wA, double* wB, double* wS);
int epdlb_batch_read_velocity(epdlb_batch* b, int32_t replica, double* rho, double* ux, double* uy);
int epdlb_batch_read_diag(epdlb_batch* b, int32_t replica, epdlb_diag* d);
/* Autotune every shape group (see epdlb_autotune). */
int epdlb_batch_autotune(epdlb_batch* b, int32_t reps, const char* cache_path);
/* Per-kernel timing of the next steps (stream launches, group after group),
 * merged over the groups; see epdlb_profile_start / epdlb_profile_read. */
int epdlb_batch_profile_start(epdlb_batch* b, int32_t max_launches);
int epdlb_batch_profile_read(epdlb_batch* b, epdlb_kernel_stat* out, int32_t cap, int32_t* n_out);
/* Observables and nucleation tracking of one replica, as epdlb_observables and
 * epdlb_track_particles for a single context (after the queued steps: the
 * batch stream is synchronised).  Each replica keeps its own tracking
 * sample; seeding or setting a replica's fields starts it over. */
int epdlb_batch_observables(epdlb_batch* b, int32_t replica, double threshold, epdlb_obs* out,
                            epdlb_particle* particles, int32_t max_particles, int32_t* labels);
int epdlb_batch_track_particles(epdlb_batch* b, int32_t replica, double threshold, epdlb_obs* out,
                                epdlb_particle* events, int32_t max_events, int32_t* n_events);
int epdlb_batch_track_reset(epdlb_batch* b, int32_t replica);
/* Number of replica groups (grid shape, A fraction) and total lattice sites. */
int epdlb_batch_info(epdlb_batch* b, int32_t* n_groups, int64_t* sites);
void epdlb_batch_destroy(epdlb_batch* b);

/* ---------------------------------------------------------------------------
 * Density surrogate.  A 4-layer dilated (1, 2, 4, 8) 3x3 convolutional
 * network, 64 channels, SiLU, in BF16 with FP32 accumulation (MFMA), maps
 * the potentials to the copolymer densities: inputs w_I - <w_I> (I = A, B,
 * S), f_A and 1/N; outputs Phi_hat_A, Phi_hat_B = softplus(o), rescaled to
 * the exact means f_A phibar_P and (1 - f_A) phibar_P; Phi_S from its closed
 * form (Sec. II, Eqs. for Phi_P, Phi_S and Q_S).  It stands in for the chain
 * propagators (Sec. II, modified diffusion equations and split step) between
 * exact steps.  At an exact step both are evaluated: the exact densities
 * become the state, the network's error against them is recorded, and the
 * force source S keeps differencing network densities at both ends of the
 * step (the next step corrects S~ by the recorded difference).
 *
 * Weights: EPDLB_NN_PARAMS host floats, for layer l = 0..3 the tensor
 * W_l[9][cin][cout] (tap t = 3*(ty+1) + (tx+1), offsets d_l*(ty, tx)) then
 * b_l[cout]; cin = 5, 64, 64, 64; cout = 64, 64, 64, 2.
 * ------------------------------------------------------------------------- */
#define EPDLB_NN_PARAMS 77954

/* Load weights into a context created with density_mode = 1 (copied; the
 * caller keeps `w`).  Required before epdlb_step.  EINVAL on a count other
 * than EPDLB_NN_PARAMS or a non-finite weight; ESTATE for density_mode 0. */
int epdlb_surrogate_set_weights(epdlb_ctx* ctx, const float* w, int64_t count);

/* Trainer: a device dataset of `capacity` (potentials -> densities) pairs on
 * an nx x ny grid, mini-batches of up to max_batch (<= 64) pairs, mean squared error
 * of (Phi_hat - Phi)/phi_scale over sites and species A, B, Adam
 * (b1 = 0.9, b2 = 0.999, eps = 1e-8) on FP32 master weights.  The trainer
 * allocates its device memory; `stream` as in epdlb_create. */
typedef struct epdlb_nn epdlb_nn;
int epdlb_nn_create(int32_t nx, int32_t ny, int32_t capacity, int32_t max_batch, int device, void* stream,
                    epdlb_nn** out);
/* Weights in the layout above (host floats); resets the Adam moments. */
int epdlb_nn_set_weights(epdlb_nn* nn, const float* w, int64_t count);
int epdlb_nn_get_weights(epdlb_nn* nn, float* w, int64_t count);
/* Store a pair from host arrays: omega 3 planes (A, B, S), phi 2 planes (A, B), [y][x]. */
int epdlb_nn_set_pair(epdlb_nn* nn, int32_t slot, const double* omega, const double* phi, double f_A,
                      int32_t n_contour);
/* Store the current (omega, exact Phi) of a density_mode 0 simulation on the
 * same device and grid (device to device). */
int epdlb_nn_capture(epdlb_nn* nn, int32_t slot, epdlb_ctx* sim);
/* Forward pass over slots[count]: loss, max |Phi_hat - Phi| (unnormalised
 * network output); with grad != NULL also the backward pass and the loss
 * gradient (EPDLB_NN_PARAMS host floats, layout as the weights).  Synchronous. */
int epdlb_nn_evaluate(epdlb_nn* nn, const int32_t* slots, int32_t count, double phi_scale, double* loss,
                      double* max_err, float* grad);
/* Forward, backward and one Adam step with learning rate lr; queued on the
 * trainer's stream (slots[] is copied before return). */
int epdlb_nn_train_step(epdlb_nn* nn, const int32_t* slots, int32_t count, double phi_scale, double lr);
/* Loss and max error of the last training step's forward pass (synchronises). */
int epdlb_nn_last_loss(epdlb_nn* nn, double* loss, double* max_err);
/* Network output softplus(o) of one slot: phi_hat[2*nx*ny] (A then B). */
int epdlb_nn_predict(epdlb_nn* nn, int32_t slot, double* phi_hat);
void epdlb_nn_destroy(epdlb_nn* nn);

/* Three-dimensional fluid.  The paper computes in two dimensions and names
 * D3Q19 as the lattice that replaces D2Q9 in three (end of Sec. II).  This
 * context advances a periodic box of nx*ny*nz sites with that lattice and
 * the collision and body force of the two-dimensional fluid (Sec. II,
 * Eq. LB_prop and Eq. force_col at gamma_s = gamma_b = 0): pull streaming
 * f_i(x) = f*_i(x - c_i), rho = sum f_i, u = (sum f_i c_i + F/2)/rho, BGK
 * relaxation with time tau to the second-order equilibrium, and the force
 * term (1 - 1/(2 tau)) w_i [3 (c_i - u).F + 9 (c_i.u)(c_i.F)].  Lattice units.
 *
 * Velocities c_i, i = 0..18: rest; +x, -x, +y, -y, +z, -z; then (1,1,0),
 * (-1,-1,0), (1,-1,0), (-1,1,0), (1,0,1), (-1,0,-1), (1,0,-1), (-1,0,1),
 * (0,1,1), (0,-1,-1), (0,1,-1), (0,-1,1); weights 1/3, 1/18, 1/36.
 * Host arrays are FP64, planes of nx*ny*nz values in [z][y][x] order (x
 * contiguous): populations 19 planes, force and velocity 3 planes (x, y, z).
 * The device holds FP64 (precision 0) or FP32 (1) deviations f_i - w_i.
 * The context owns its device memory (2 x 19 + 7 planes); work is queued on
 * its stream (the caller's, or its own when stream is NULL).  Return codes as
 * above; EINVAL for a size outside [1, 4096], tau <= 1/2, a non-finite value
 * or a density <= 0. */
typedef struct epdlb_lb3 epdlb_lb3;
int epdlb_lb3_create(int32_t nx, int32_t ny, int32_t nz, double tau, int32_t precision, int device,
                     void* stream, epdlb_lb3** out); /* starts at rest (rho = 1, u = 0), F = 0 */
/* Post-collision populations f* (19 planes) from which the next step streams. */
int epdlb_lb3_set_populations(epdlb_lb3* c, const double* f);
/* f* = f^eq(rho, u) at every site; rho (1 plane) NULL means 1, u (3 planes) NULL means 0. */
int epdlb_lb3_set_equilibrium(epdlb_lb3* c, const double* rho, const double* u);
/* Body force density F (3 planes), held for every following step; NULL clears it. */
int epdlb_lb3_set_force(epdlb_lb3* c, const double* F);
/* Collision of the following steps.  mrt = 0 (the default): BGK at the
 * context's tau.  mrt = 1: the paper's multi-relaxation collision (Sec. II,
 * Eq. force_col) with the trace split of three dimensions, where the printed
 * 2/3 and 1/3 apply: with A = Pi - rho/3 I, N = A - rho u u, t = tr(N)/3,
 * the post-collision stress is rho u u + gamma_s (N - t I) + gamma_b t I
 * + (1 + gamma_s)/2 [u F + F u - (2/3)(u.F) I] + (1 + gamma_b)/3 (u.F) I,
 * the momentum j + F, and the non-hydrodynamic modes are scaled by gamma_g.
 * Shear viscosity (1/6)(1 + gamma_s)/(1 - gamma_s), bulk viscosity
 * (1/9)(1 + gamma_b)/(1 - gamma_b) (lattice units); equal factors 1 - 1/tau
 * give the BGK collision at tau.  EINVAL for a factor outside (-1, 1). */
int epdlb_lb3_set_collision(epdlb_lb3* c, int32_t mrt, double gamma_s, double gamma_b, double gamma_g);
/* n steps, queued; the last one also stores rho and u.  Returns before the GPU finishes. */
int epdlb_lb3_step(epdlb_lb3* c, int64_t n);
/* n steps as epdlb_lb3_step (1 <= n <= 4096), each launch timed on the GPU
 * from its own start to its end; ms[n] receives the durations.  Synchronous. */
int epdlb_lb3_profile(epdlb_lb3* c, int32_t n, double* ms);
int epdlb_lb3_sync(epdlb_lb3* c);
/* The current f* (19 planes).  Synchronous. */
int epdlb_lb3_read_populations(epdlb_lb3* c, double* f);
/* rho (1 plane) and u (3 planes, including F/2) of the last step; ESTATE
 * before any step since the populations were set.  Synchronous. */
int epdlb_lb3_read_velocity(epdlb_lb3* c, double* rho, double* u);
void epdlb_lb3_destroy(epdlb_lb3* c);

/* Chain propagators and densities on a three-dimensional periodic grid of
 * nx*ny*nz sites (powers of two up to 512), the paper's Sec. II (the split
 * step q_{j+1} = E_j K (E_j q_j), E_j = exp(-(w_j - c_j)/2), K = exp(R_G^2
 * Laplacian ds) with |k|^2 = kx^2 + ky^2 + kz^2; the density integrals with
 * trapezoid contour weights; Eq. phi_s), in three dimensions as the paper
 * allows (end of Sec. II); volume element dx^3.  The gauge constants c are
 * the site means of the fields.  FP64 (precision 0) or FP32 (1) planes, FP64
 * sums.  Host arrays FP64, 3 planes [I][z][y][x] (x contiguous): omega in
 * (wA, wB, wS), phi out (Phi_A, Phi_B, Phi_S).  The context owns its device
 * memory (2 (N + 1) + 8 planes); work runs on its stream (the caller's, or
 * its own when stream is NULL).  EINVAL for a bad size or parameter or a
 * non-finite potential; ENONFINITE when Q_P or Q_S is not finite. */
typedef struct epdlb_epd3 epdlb_epd3;
int epdlb_epd3_create(int32_t nx, int32_t ny, int32_t nz, int32_t n_contour, double f_A, double phi_P,
                      double R_G, double dx, int32_t precision, int device, void* stream, epdlb_epd3** out);
/* Densities of omega; Q_P = dx^3 sum q_N, Q_S = dx^3 sum exp(-(wS - cS)) (either may be NULL).  Synchronous. */
int epdlb_epd3_densities(epdlb_epd3* c, const double* omega, double* phi, double* Q_P, double* Q_S);
/* reps evaluations of the potentials last passed in, timed with events on the
 * stream; ms receives the mean GPU time per evaluation.  Synchronous. */
int epdlb_epd3_time(epdlb_epd3* c, int32_t reps, double* ms);
/* One evaluation of the potentials last passed in with every FFT launch
 * timed on the GPU from its own start to its end: *fft_ms receives the sum of
 * their durations and *fft_launches their number (10 N at sides > 1).
 * Synchronous. */
int epdlb_epd3_profile(epdlb_epd3* c, double* fft_ms, int32_t* fft_launches);
void epdlb_epd3_destroy(epdlb_epd3* c);

/* Message for the last failing call on this thread ("" if none). */
const char* epdlb_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* EPDLB_H */
