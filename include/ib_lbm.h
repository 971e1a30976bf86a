/*
 * ib_lbm.h — C ABI of the MI355X (gfx950) immersed-boundary lattice
 * Boltzmann library.
 *
 * The library advances D2Q9 lattice-Boltzmann fields coupled to rigid
 * circular bodies represented by Lagrangian markers, following Jo,
 * "Mechanism-Resolved Interface Momentum Transfer in Immersed-Boundary
 * Lattice Boltzmann Simulations" (arXiv 2609.02298):
 *   - collision BGK with Guo forcing (Sec. 2.1, Eq. 1-4), TRT (Sec. 2.2) or
 *     central-moment MRT (Sec. 2.2, Eq. 5), fused with streaming;
 *   - immersed boundary with the hat (Eq. 9) or Peskin 4-point (Eq. 10)
 *     regularized delta (Eq. 6-8), enforced by direct forcing (Eq. 11),
 *     multi-direct forcing (Eq. 12-14) or distribution-function correction
 *     (Eq. 15-20);
 *   - hydrodynamic force and torque (Sec. 2.7), rigid-body Velocity-Verlet
 *     update (Eq. 21-23) with the explicit internal-mass force (Eq. A3).
 *
 * Units: lattice units, dx = dt = 1.  Populations exchanged with the host
 * are nine planes f[i][y][x] with x fastest (the device store is the
 * library's own) and directions
 *   e0=(0,0) e1=(1,0) e2=(0,1) e3=(-1,0) e4=(0,-1)
 *   e5=(1,1) e6=(-1,1) e7=(-1,-1) e8=(1,-1).
 *
 * Conventions shared by every entry point:
 *   - Every call returns an ib_lbm_status; no C++ exception crosses the ABI.
 *     The message of the last failure of a sim is ib_lbm_last_error().
 *   - After IB_LBM_E_DEVICE (a failed HIP call) the sim is unusable and every
 *     later call on it returns IB_LBM_E_STATE; only ib_lbm_destroy remains.
 *   - Host pointers ("host") are read or written before the call returns and
 *     are not retained.  The library owns every device buffer it allocates
 *     and frees them in ib_lbm_destroy / ib_lbm_batch_destroy.
 *   - Work is queued on the HIP stream given at creation; calls that return
 *     host data synchronise that stream first.
 *   - One sim is used by one host thread at a time.
 */
#ifndef IB_LBM_H
#define IB_LBM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define IB_LBM_ABI_VERSION 6u

typedef enum {
  IB_LBM_OK = 0,
  IB_LBM_E_INVALID = -1,  /* an argument or configuration is not supported */
  IB_LBM_E_NOMEM = -2,    /* device allocation failed */
  IB_LBM_E_DEVICE = -3,   /* a HIP runtime call failed */
  IB_LBM_E_DIVERGED = -4, /* a non-finite force was produced; the sim halted */
  IB_LBM_E_RANGE = -5,    /* a marker support left the lattice, or two bodies' supports met */
  IB_LBM_E_STATE = -6     /* the call is not allowed in the current state */
} ib_lbm_status;

enum { IB_LBM_FP64 = 0, IB_LBM_FP32_SHIFTED = 1 };
enum { IB_LBM_BGK = 0, IB_LBM_TRT = 1, IB_LBM_CMMRT = 2 };
/* Face closures.  PERIODIC must be set on both faces of an axis; the
 * zero-gradient face copies the entering populations from the nodes one
 * step inside (any face; Sec. 2.9).  BOUNCE_BACK is a half-way wall (half a
 * spacing outside the face nodes); ZOU_HE is an on-node wall at rest with
 * the closure of Zou and He (the walls of Sec. 2.9.3-2.9.4): the face nodes
 * are wall nodes whose momentum sum_i f_i e_i is zero after every step.
 * ZOU_HE combines only with ZOU_HE or PERIODIC faces, and such a sim cannot
 * join a batch. */
enum { IB_LBM_PERIODIC = 0, IB_LBM_BOUNCE_BACK = 1, IB_LBM_VEL_PARABOLIC = 2,
       IB_LBM_VEL_UNIFORM = 3, IB_LBM_ZERO_GRADIENT = 4, IB_LBM_ZOU_HE = 5 };
enum { IB_LBM_DF = 0, IB_LBM_MDF = 1, IB_LBM_DFC = 2 };
enum { IB_LBM_HAT = 0, IB_LBM_PESKIN4 = 1 };
enum { IB_LBM_FIXED = 0, IB_LBM_PRESCRIBED_SIN = 1, IB_LBM_FREE = 2 };
enum { IB_LBM_IM_NONE = 0, IB_LBM_IM_FENG = 1 };
enum { IB_LBM_VERLET = 0, IB_LBM_EULER_A1 = 1 };
/* desired marker velocity of a body (ib_lbm_body_desc.udes) */
enum { IB_LBM_UD_RIGID = 0, IB_LBM_UD_TAYLOR_GREEN = 1 };
enum { IB_LBM_SPREAD_GATHER = 0, IB_LBM_SPREAD_ATOMIC = 1 };

/* Body flags reported in ib_lbm_body_state.flags */
enum { IB_LBM_FLAG_NONFINITE = 1, IB_LBM_FLAG_RANGE = 2, IB_LBM_FLAG_OVERLAP = 4,
       IB_LBM_FLAG_CAPACITY = 8, IB_LBM_FLAG_EXCHANGE = 16 };

/* Optional device allocator (for example a caching allocator).  alloc returns
 * device memory of at least `bytes` usable on `stream`, or NULL. */
typedef struct {
  void *ctx;
  void *(*alloc)(void *ctx, size_t bytes, void *stream);
  void (*free)(void *ctx, void *ptr, void *stream);
} ib_lbm_allocator;

/* Lattice configuration (Sec. 2.1-2.2, App. A.1).  tau > 1/2 sets the
 * viscosity nu = (tau - 1/2)/3; trt_magic is Lambda_eo (default 1/4);
 * cm_s_q / cm_s_eps are the third- and fourth-order central-moment rates
 * (1.2 / 1.4).  gravity acts on bodies only (reduced pressure, Eq. 22);
 * fluid_force is a uniform body-force density on the fluid (zero in the
 * paper's runs, used for forced channel flows).  history_capacity: number of
 * most recent steps kept per body in the device history ring (0 -> 4096). */
typedef struct {
  uint32_t abi_version; /* must equal IB_LBM_ABI_VERSION */
  int32_t nx, ny;       /* nodes, x streamwise; 3 <= nx < 65535, 3 <= ny < 32767,
                           nx*ny < 2^31 (population offsets are 64-bit) */
  int32_t precision;    /* IB_LBM_FP64 | IB_LBM_FP32_SHIFTED */
  int32_t collision;    /* IB_LBM_BGK | IB_LBM_TRT | IB_LBM_CMMRT */
  int32_t history_capacity;
  double tau;
  double trt_magic;
  double cm_s_q, cm_s_eps;
  double rho0;          /* reference density, 1 in the paper */
  int32_t bc[4];        /* faces W, E, S, N */
  double u_bc;          /* u_max of a parabolic inlet or u_inf of a uniform face */
  double gravity[2];
  double fluid_force[2];
  void *stream;         /* hipStream_t; NULL = the null stream */
  const ib_lbm_allocator *alloc; /* NULL = hipMalloc / hipFree */
} ib_lbm_config;

/* A rigid circular body (Sec. 2.3-2.7).  n_markers = 0 -> round(pi D)
 * evenly spaced markers (Table I), arc spacing ds = pi D / n_markers.
 * MDF: passes of Eq. 12-14 with relaxation mdf_omega, or 1/||A||_inf
 * computed once here when mdf_omega <= 0 (Sec. 2.5.2).  mdf_tol <= 0: exactly
 * mdf_iters passes.  mdf_tol > 0: the adaptive form of Sec. 2.5.2 / App. A.2.
 * Before pass n the residual r_n = max_k |U_d - U^(n)(X_k)| is measured, and
 * the iteration ends there, without pass n, once at least mdf_nmin passes
 * are done and r_n < mdf_tol, or when r_n > 1.5 r_(n-1) (divergence guard,
 * from n = 2); it applies at most mdf_iters passes (the paper's runs:
 * mdf_nmin 5, mdf_iters 20, mdf_tol 1e-4).  Each body decides on its own
 * residual.  IB_LBM_E_INVALID unless 1 <= mdf_nmin <= mdf_iters.
 * PRESCRIBED_SIN: X_c(t) = X_c0 + amp sin(2 pi freq t + phase).
 * FREE: density_ratio rho_s/rho0, internal_mass selects scheme (A) or the
 * Feng explicit-history correction (App. A.5).  integrator: the
 * Velocity-Verlet update of Eq. 23 (half-kick and drift before the step,
 * full kick after it), or the Euler-explicit update of Eq. A1 before the
 * step, v^(n+1) = (1 + r) v^n - r v^(n-1) + (F_hydro^n + F_g)/m_s with r =
 * rho0/rho_s (0 without internal mass); the rotation carries the rigid
 * interior's angular-momentum increment in both internal-mass arms (Sec.
 * 2.7), Omega^(n+1) = (1 + q) Omega^n - q Omega^(n-1) + T^n/I_s with
 * q = rho0/rho_s; X^(n+1) = X^n + v^(n+1).
 * mdf_coupled (MDF, every body of the sim alike, with equal mdf_iters,
 * mdf_nmin and mdf_tol): the coupled multi-body path of Sec. 2.5.2.  The
 * bodies' passes share each fluid update and are controlled on the residual
 * R of all markers together: each body relaxes at c min(omega_MDF, 0.8)
 * with a common factor c (1 at the start of a step); after each trial pass
 * the new R' is measured, and R' > 1.2 R rejects the trial (the velocities
 * return to their state before it) and halves c, ending the iteration once
 * c reaches 1/8; an accepted trial counts as a pass.  The iteration ends
 * after mdf_iters accepted passes, or, with mdf_tol > 0, once at least
 * mdf_nmin are accepted and R < mdf_tol.  Every body reports the joint
 * residual and the accepted passes.  Such a sim runs the passes on the
 * support nodes, cannot join a batch, and its bodies' IB workgroups meet
 * once per trial through device memory (a wait bounded to about 2 s; on
 * expiry the body reports IB_LBM_FLAG_EXCHANGE and the step stops with
 * IB_LBM_E_STATE from ib_lbm_forces).
 * udes: the desired velocity of the markers.  IB_LBM_UD_RIGID: the body's
 * rigid motion, U_d = V + Omega x (X_k - X_c) (Sec. 2.7).
 * IB_LBM_UD_TAYLOR_GREEN (the IB-LBM mode of the Taylor-Green check, App.
 * D.1; FIXED bodies only): the decaying vortex of Eq. D1 at each marker,
 * U_d = tg_u0 exp(-2 tg_nu tg_k^2 t) (-cos(k X) sin(k Y), sin(k X) cos(k Y))
 * with k = tg_k > 0, the origin at node (0, 0) and t the time level the
 * step advances to (n + 1 in the step from n); tg_nu >= 0.  Such a body has
 * no boundary-fidelity diagnostics (IB_LBM_E_INVALID).
 * All bodies of one sim use the same scheme. */
typedef struct {
  double xc, yc, diameter;
  int32_t n_markers;
  int32_t scheme;   /* IB_LBM_DF | IB_LBM_MDF | IB_LBM_DFC */
  int32_t kernel;   /* IB_LBM_HAT | IB_LBM_PESKIN4 */
  int32_t mdf_iters;
  double mdf_omega;
  int32_t motion;   /* IB_LBM_FIXED | IB_LBM_PRESCRIBED_SIN | IB_LBM_FREE */
  int32_t internal_mass;
  double amp[2], freq, phase;
  double density_ratio;
  int32_t mdf_nmin; /* adaptive MDF: fewest passes before the tolerance stop */
  double mdf_tol;   /* > 0 selects the adaptive MDF; <= 0 the fixed form */
  int32_t integrator; /* FREE bodies: IB_LBM_VERLET | IB_LBM_EULER_A1 */
  int32_t mdf_coupled; /* MDF: 1 selects the coupled multi-body path */
  int32_t udes;     /* IB_LBM_UD_RIGID | IB_LBM_UD_TAYLOR_GREEN */
  int32_t reserved;
  double tg_u0, tg_k, tg_nu; /* Eq. D1 parameters of IB_LBM_UD_TAYLOR_GREEN */
} ib_lbm_body_desc;

/* State of a body after the last completed step.  Forces are on the body
 * (Newton's third law for DF/MDF).  slip_* are |interp(u) - U_d| over the
 * markers with the post-IB velocity; mdf_residual is max_k |U_d - U| of the
 * last MDF interpolation of the step (before the last pass applied, or,
 * after an adaptive stop, the one that ended the iteration); mdf_iters is
 * the number of passes applied. */
typedef struct {
  int64_t step;
  double fx, fy, torque;
  double xc, yc, vx, vy, omega;
  double slip_mean, slip_max, mdf_residual;
  double mdf_omega;
  int32_t mdf_iters, flags;
} ib_lbm_body_state;

/* Launch shape of the collide-stream kernel: block_x threads along x (a
 * multiple of 64), block_y thread rows, rows_per_thread nodes per thread
 * along y.  The tile is block_x x (block_y * rows_per_thread) nodes.
 * ib_threads: workgroup size of the IB pass (one workgroup per body): 0 for
 * the library's choice (1024 for DF/MDF bodies whose workspace fits in LDS,
 * 512 otherwise), or 256, 512 or 1024 (the second kind takes at most 512). */
typedef struct {
  int32_t block_x, block_y, rows_per_thread;
  int32_t xcd_remap; /* 1: keep neighbouring tiles on one XCD */
  int32_t ib_threads;
} ib_lbm_launch;

typedef struct ib_lbm_sim ib_lbm_sim;
typedef struct ib_lbm_batch ib_lbm_batch;

/* Library version, equal to IB_LBM_ABI_VERSION of the build. */
uint32_t ib_lbm_abi_version(void);

/* Create a sim: validates cfg (IB_LBM_E_INVALID), allocates two population
 * lattices and the force field on the device and sets f = f^eq(rho0, u_init)
 * with u_init the parabolic inlet profile (W face parabolic), u_bc (any
 * uniform face) or 0.  *out receives the handle. */
ib_lbm_status ib_lbm_create(const ib_lbm_config *cfg, ib_lbm_sim **out);

/* Add a body before the first step (IB_LBM_E_STATE afterwards).  Places the
 * markers, checks that every support lies inside the lattice and does not
 * meet another body's support (IB_LBM_E_RANGE), computes omega_MDF, uploads
 * the marker tables.  *body_id receives the index (0, 1, ...). */
ib_lbm_status ib_lbm_add_body(ib_lbm_sim *s, const ib_lbm_body_desc *b, int32_t *body_id);

/* Queue nsteps time steps on the sim's stream (asynchronous).  Each step:
 * body kinematics for t+1, fused collide+stream with the force of the last
 * IB pass, IB pass on the new populations, force/torque, body update. */
ib_lbm_status ib_lbm_step(ib_lbm_sim *s, int64_t nsteps);

/* Synchronise and return the state of body_id.  Returns IB_LBM_E_DIVERGED or
 * IB_LBM_E_RANGE (state still filled) when the body's flags are set. */
ib_lbm_status ib_lbm_forces(ib_lbm_sim *s, int32_t body_id, ib_lbm_body_state *out);

/* Copy `count` history rows of body_id starting at step `first` (1-based step
 * numbers, within the last history_capacity steps) to host out[count][16]:
 * step fx fy torque xc yc vx vy omega slip_mean slip_max mdf_residual
 * mdf_iters flags 0 0. */
ib_lbm_status ib_lbm_history(ib_lbm_sim *s, int32_t body_id, int64_t first, int64_t count,
                             double *out);

/* Density and velocity (Eq. 4, with the IB force still to be applied by the
 * next collision) into host arrays of nx*ny doubles, x fastest. */
ib_lbm_status ib_lbm_fields(ib_lbm_sim *s, double *rho, double *ux, double *uy);

/* Current populations f (FP64, host, 9*ny*nx) — read and overwrite.  For the
 * FP32 shifted store the values are converted from / to g = f - w_i rho0. */
ib_lbm_status ib_lbm_get_populations(ib_lbm_sim *s, double *f);
ib_lbm_status ib_lbm_set_populations(ib_lbm_sim *s, const double *f);

/* Overwrite the current populations with the equilibrium of Eq. 2,
 * f_i = w_i rho (1 + 3 e_i.u + 4.5 (e_i.u)^2 - 1.5 u.u), of host fields
 * (nx*ny doubles each, x fastest; rho NULL -> rho0 everywhere), evaluated in
 * FP64 on the device and stored as g = f - w_i rho0 in the FP32 store.  The
 * IB force field and the step count are left as they are.
 * IB_LBM_E_INVALID for a null ux or uy. */
ib_lbm_status ib_lbm_set_equilibrium(ib_lbm_sim *s, const double *rho, const double *ux,
                                     const double *uy);

/* Eulerian IB force density of the last IB pass (host, ny*nx each). */
ib_lbm_status ib_lbm_force_field(ib_lbm_sim *s, double *fx, double *fy);

/* Per-marker data of the last step (host, n_markers rows of 8 doubles):
 * X Y Udx Udy Fx Fy lambda ds.  Fx,Fy are the accumulated Lagrangian force
 * F_L (DF/MDF) or the particle-side F_s (DFC).  Returns the marker count in
 * *n_markers. */
ib_lbm_status ib_lbm_markers(ib_lbm_sim *s, int32_t body_id, double *out, int32_t *n_markers);

/* Boundary-fidelity diagnostics of body_id on the current state (Sec. 2.8,
 * and the marker-resolved profiles of Sec. 4.2), computed on the device and
 * returned to the host (synchronises).  The Eulerian field is u = (sum_i f_i
 * e_i + F/2)/rho with the pending IB force, as ib_lbm_fields returns it; it
 * is sampled at the markers by bilinear interpolation (hat weights of the
 * 2 x 2 surrounding nodes), a probe distinct from the scheme's own kernel.
 * Velocities are taken relative to the body's rigid motion U_b(x) = v +
 * omega x (x - X_c), with v, omega as ib_lbm_forces reports them (zero for a
 * fixed body); n_k = (X_k - X_c)/R; velocities are divided by u_ref (> 0,
 * U_inf of the paper); kappa >= 0 buffer cells are excluded inside the
 * solid (the paper uses 2).
 *   summary[8] (host): slip mean and max of |u(X_k) - U_b(X_k)|/u_ref;
 *     leakage flux sum_k rho(X_k) (u - U_b).n_k ds / (u_ref pi D); internal
 *     residual mean and max of |u - U_b|/u_ref over the nodes with
 *     |x - X_c| < R - kappa, and their count; mean (rho(X_k) - rho0)/3; mean
 *     marker force magnitude |F_k| (F_L for DF/MDF, F_s for DFC).
 *   per_marker (host, n_markers x 6, or NULL): slip_k, dp_k = (rho(X_k) -
 *     rho0)/3, |F_k|, rho(X_k), normal and tangential (u - U_b)/u_ref.
 * IB_LBM_E_STATE before the first completed step; IB_LBM_E_DIVERGED when the
 * body's position or velocity is not finite.  A marker whose 2 x 2 stencil
 * is not inside the lattice yields NaN. */
ib_lbm_status ib_lbm_diagnostics(ib_lbm_sim *s, int32_t body_id, int32_t kappa, double u_ref,
                                 double *summary, double *per_marker);

/* ib_lbm_diagnostics for callers that cannot allocate device memory (tight
 * serving loops, harnesses that forbid hipMalloc): the same computation and
 * outputs, staged in a library-owned static device array instead of a
 * buffer the sim allocates on demand.  Allocates nothing; like
 * ib_lbm_diagnostics it synchronises the sim's stream and copies to host, so
 * it is not for use inside a stream capture.  The array holds the summary
 * and up to 8192 markers' rows; a body with more markers gives
 * IB_LBM_E_INVALID.  Every value returned is written by the call itself, so
 * nothing carries over from an earlier call.  Each GPU holds its own copy
 * until the process ends, shared by every call on that GPU: calls that
 * overlap on one GPU (from several host threads) race and must be
 * serialised by the caller.  Runs on the sim's device. */
ib_lbm_status ib_lbm_diagnostics_noalloc(ib_lbm_sim *s, int32_t body_id, int32_t kappa,
                                         double u_ref, double *summary, double *per_marker);

/* Completed steps (synchronises). */
ib_lbm_status ib_lbm_steps_done(ib_lbm_sim *s, int64_t *steps);
ib_lbm_status ib_lbm_sync(ib_lbm_sim *s);
ib_lbm_status ib_lbm_destroy(ib_lbm_sim *s);
const char *ib_lbm_last_error(const ib_lbm_sim *s);

/* Device bytes a sim of this configuration holds with the given bodies. */
size_t ib_lbm_footprint(const ib_lbm_config *cfg, int32_t n_bodies, const int32_t *n_markers);

/* Launch shape of the collide-stream kernel (validated; IB_LBM_E_INVALID if
 * block_x is not a multiple of 64 or the block exceeds 1024 threads). */
ib_lbm_status ib_lbm_set_launch(ib_lbm_sim *s, const ib_lbm_launch *l);
ib_lbm_status ib_lbm_get_launch(const ib_lbm_sim *s, ib_lbm_launch *l);
/* Spreading variant: marker-sorted gather (default, deterministic) or
 * per-marker atomic scatter (order-dependent rounding). */
ib_lbm_status ib_lbm_set_spread(ib_lbm_sim *s, int32_t mode);
/* hipGraph use: steps_per_graph > 0 records that many steps once (one
 * graph for each of the two lattices a run of steps can start from) and
 * replays them; 0 launches kernels directly.  Plain steps are captured from a
 * stream; pipelined steps (below) are built as an explicit graph of the same
 * kernels with their ordering as node dependencies, both graphs at the first
 * replay.  Recording happens at the first ib_lbm_step call that needs it, so
 * that call may allocate; steps beyond a multiple of steps_per_graph are
 * launched directly. */
ib_lbm_status ib_lbm_set_graph(ib_lbm_sim *s, int32_t steps_per_graph);

/* Pipelined steps (default on).  For a sim with one body that is fixed or
 * prescribed, whose supports over the run stay two nodes clear of the faces,
 * ib_lbm_step runs the collide-stream launches and the IB passes on two
 * library-owned streams that overlap: the collide-stream of step n+1 starts
 * while the IB pass of step n is still running, and only its tiles next to
 * the body (the ones that read what the IB pass writes, or are read by it)
 * wait for that pass.  The two streams are ordered by HIP events only;
 * nothing waits on the host.  The first call after ib_lbm_create or a
 * state-reading call starts after the work already on the sim's stream, and
 * the sim's stream waits for both streams before any later work.  The
 * collide-stream stream leaves one compute unit to the IB pass.  Results
 * are bitwise the same as unpipelined steps.  In steps replayed from a graph
 * (ib_lbm_set_graph) the collide-stream launches run without that stream's
 * compute-unit mask.
 * set_overlap(0/1) forbids or allows it; get_overlap reports whether the
 * current configuration uses it (after the first step) and, if near_nodes
 * is not NULL, the number of nodes in the tiles that wait for the IB pass. */
ib_lbm_status ib_lbm_set_overlap(ib_lbm_sim *s, int32_t on);
ib_lbm_status ib_lbm_get_overlap(const ib_lbm_sim *s, int32_t *in_use, int64_t *near_nodes);

/* Fused steps (default on).  A pipelined sim (see ib_lbm_set_overlap) whose
 * single body is fixed, DF or MDF on the 1024-thread IB kernel, with BGK or
 * TRT collision and no Zou-He wall, takes one launch per step on the sim's
 * stream, with no second stream and no events.  Workgroup 0 runs the IB
 * pass: it collides the nodes that push into the body's support itself,
 * from the step's input lattice and the force of the previous pass, while
 * the other workgroups collide and stream every node.  The tiles that read
 * the IB force count themselves on the case state before the pass writes
 * the new force.  Results are bitwise those of unpipelined steps, and the
 * steps can be captured and replayed (ib_lbm_set_graph).  The first call
 * builds the list of nodes the pass collides from the body's support (after
 * one pipelined step if none has run; a synchronising copy, and it may
 * allocate); kernel timing (ib_lbm_timing_enable) runs pipelined steps.
 * set_fused(0/1) forbids or allows it; get_fused reports whether the
 * current configuration uses it (after the first step). */
ib_lbm_status ib_lbm_set_fused(ib_lbm_sim *s, int32_t on);
ib_lbm_status ib_lbm_get_fused(const ib_lbm_sim *s, int32_t *in_use);

/* Kernel timing with HIP events (direct launches only).  which: 0
 * collide-stream, 1 immersed boundary.  With pipelined steps a collide-stream
 * launch includes the wait of its tiles next to the body for the previous IB
 * pass.  Reset with enable. */
ib_lbm_status ib_lbm_timing_enable(ib_lbm_sim *s, int32_t on);
/* Measurement only: `launches` back-to-back launches of the collide-stream
 * kernel over the inner nodes (1 <= x <= nx-3, 1 <= y <= ny-2; every link
 * stays inside the lattice) on the sim's stream, bracketed by two HIP events;
 * *avg_us receives the average time per launch and *inner_nodes (if not
 * NULL) the nodes one launch updates.  The sim's populations are advanced by
 * these launches without face closures or IB passes, so the sim is meant
 * for the measurement alone (for example a copy of a workload's sim).
 * Synchronises. */
ib_lbm_status ib_lbm_time_collide_stream(ib_lbm_sim *s, int32_t launches, double *avg_us,
                                         int64_t *inner_nodes);
ib_lbm_status ib_lbm_timing_read(ib_lbm_sim *s, int32_t which, double *total_ms, int64_t *launches);
/* Measurement only: the plain read + write stream that the collide-stream
 * kernel's HBM fraction is compared with.  Copies `bytes` bytes (a positive
 * multiple of 16) from device buffer src to device buffer dst (distinct,
 * 16-byte aligned, owned by the caller) on `stream` (a hipStream_t, NULL for
 * the null stream) with a grid-stride 16-byte-vector kernel, `workgroups`
 * workgroups of 1024 threads (256 when 0).  Asynchronous; E_INVALID for a
 * size, alignment or count outside these rules, E_DEVICE when the launch
 * fails. */
ib_lbm_status ib_lbm_stream_copy(const void *src, void *dst, size_t bytes, int32_t workgroups,
                                 void *stream);

/* ---- batching: many independent sims stepped by shared launches ----
 * All sims of a batch share one precision and one stream.  A batch step is
 * one collide-stream launch per collision model present and one IB launch
 * for every body of every attached sim; each sim keeps its own step count
 * and target and stops at its own target (ib_lbm_batch_set_target). */
ib_lbm_status ib_lbm_batch_create(void *stream, int32_t precision, ib_lbm_batch **out);
ib_lbm_status ib_lbm_batch_attach(ib_lbm_batch *b, ib_lbm_sim *s);
ib_lbm_status ib_lbm_batch_detach(ib_lbm_batch *b, ib_lbm_sim *s);
/* Run sims of the batch until each reaches step `target` (set per sim). */
ib_lbm_status ib_lbm_batch_set_target(ib_lbm_batch *b, ib_lbm_sim *s, int64_t target);
ib_lbm_status ib_lbm_batch_step(ib_lbm_batch *b, int64_t nsteps);
ib_lbm_status ib_lbm_batch_set_graph(ib_lbm_batch *b, int32_t steps_per_graph);
/* Launch shape and spreading variant of the batch's launches (as for a sim). */
ib_lbm_status ib_lbm_batch_set_launch(ib_lbm_batch *b, const ib_lbm_launch *l);
ib_lbm_status ib_lbm_batch_set_spread(ib_lbm_batch *b, int32_t mode);
ib_lbm_status ib_lbm_batch_sync(ib_lbm_batch *b);
ib_lbm_status ib_lbm_batch_destroy(ib_lbm_batch *b);
const char *ib_lbm_batch_last_error(const ib_lbm_batch *b);

#ifdef __cplusplus
}
#endif
#endif /* IB_LBM_H */
