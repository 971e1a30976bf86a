/*
 * Plain single-threaded FP64 reference ("oracle") of the IB-LBM time step of
 * Jo, "Mechanism-Resolved Interface Momentum Transfer in Immersed-Boundary
 * Lattice Boltzmann Simulations" (arXiv 2609.02298).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may link, load or
 * call this code: only the test suite, the smoke check and the CPU-baseline
 * leg of the benchmark use it.  It shares no source with the HIP library.
 *
 * Lattice units throughout (dx = dt = h = 1).  Populations are stored as
 * nine planes f[i][y][x], x fastest.  Direction order:
 *   e0=(0,0) e1=(1,0) e2=(0,1) e3=(-1,0) e4=(0,-1)
 *   e5=(1,1) e6=(-1,1) e7=(-1,-1) e8=(1,-1)
 */
#ifndef IBLBM_ORACLE_H
#define IBLBM_ORACLE_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum { OR_BGK = 0, OR_TRT = 1, OR_CMMRT = 2 };
enum { OR_PERIODIC = 0, OR_BOUNCE_BACK = 1, OR_VEL_PARABOLIC = 2, OR_VEL_UNIFORM = 3,
       OR_ZERO_GRADIENT = 4, OR_ZOU_HE = 5 };
enum { OR_DF = 0, OR_MDF = 1, OR_DFC = 2 };
enum { OR_HAT = 0, OR_PESKIN4 = 1 };
enum { OR_FIXED = 0, OR_PRESCRIBED_SIN = 1, OR_FREE = 2 };
enum { OR_IM_NONE = 0, OR_IM_FENG = 1 };
enum { OR_VERLET = 0, OR_EULER_A1 = 1 };
enum { OR_UD_RIGID = 0, OR_UD_TAYLOR_GREEN = 1 };

typedef struct {
  int32_t nx, ny;
  int32_t collision;
  int32_t pad0;
  double tau;
  double trt_magic;        /* Lambda_eo */
  double cm_s_q, cm_s_eps; /* third- and fourth-order central-moment rates */
  double rho0;
  int32_t bc[4];           /* faces W, E, S, N */
  double u_bc;             /* u_max (parabolic) or u_inf (uniform) */
  double gravity[2];       /* acts on bodies only (reduced pressure) */
  double fluid_force[2];   /* uniform body force density on the fluid */
} or_config;

typedef struct {
  double xc, yc, diameter;
  int32_t n_markers;
  int32_t scheme;
  int32_t kernel;
  int32_t mdf_iters;
  double mdf_omega;        /* <= 0: 1/||A||_inf computed at add_body */
  int32_t motion;
  int32_t internal_mass;
  double amp[2], freq, phase;
  double density_ratio;
  int32_t mdf_nmin;        /* adaptive MDF: fewest passes before the tolerance stop */
  int32_t pad1;
  double mdf_tol;          /* > 0: adaptive MDF (Sec. 2.5.2, App. A.2); <= 0: mdf_iters passes */
  int32_t integrator;      /* free bodies: OR_VERLET (Eq. 23) or OR_EULER_A1 (Eq. A1) */
  int32_t mdf_coupled;     /* MDF: the bodies of the sim iterate jointly with the
                              coupled-path controls of Sec. 2.5.2 (same value on every body) */
  int32_t udes;            /* desired marker velocity: OR_UD_RIGID (the body's rigid
                              motion, Sec. 2.7) or OR_UD_TAYLOR_GREEN (Eq. D1, fixed
                              markers of the IB-LBM Taylor-Green mode, App. D.1) */
  int32_t pad2;
  double tg_u0, tg_k, tg_nu;  /* Eq. D1: amplitude u0, wavenumber k, viscosity nu */
} or_body_desc;

typedef struct or_sim or_sim;

or_sim *or_create(const or_config *cfg);
void or_destroy(or_sim *s);
/* returns body id >= 0, or -1 invalid, -5 support outside the domain */
int or_add_body(or_sim *s, const or_body_desc *b);
/* returns 0, or -5 when a marker support left the domain (sim halted) */
int or_step(or_sim *s, int64_t nsteps);
int64_t or_steps_done(const or_sim *s);

void or_get_populations(const or_sim *s, double *f);
void or_set_populations(or_sim *s, const double *f);
void or_get_force(const or_sim *s, double *fx, double *fy);
void or_fields(const or_sim *s, double *rho, double *ux, double *uy);
/* out[16]: step fx fy torque xc yc vx vy omega slip_mean slip_max mdf_residual
 *          mdf_iters ... (rest zero) */
int or_body_state(const or_sim *s, int b, double *out);
/* per marker 8 values: X Y Udx Udy Fx Fy lambda ds */
int or_markers(const or_sim *s, int b, double *out);
double or_body_omega(const or_sim *s, int b);
/* Euler-explicit rigid-body step of Eq. (A1); st as for the Verlet kicks
 * with st[10] = Omega^(n-1). */
void or_body_euler(double ms, double mf, double Is, int internal_mass, const double *g, double *st);
/* MDF residual r_n of each interpolation of the last step (out holds
 * mdf_iters doubles); returns their number. */
int or_mdf_residuals(const or_sim *s, int b, double *out);
/* Boundary-fidelity diagnostics of body b on the current field (Sec. 2.8,
 * Sec. 4.2): sum[8] and, when pm is not NULL, 6 values per marker. */
int or_diagnostics(const or_sim *s, int b, int kappa, double u_ref, double *sum, double *pm);

/* unit-level pieces used by the pins */
double or_phi(int kernel, double r);
void or_equilibrium(double rho, double ux, double uy, double *feq);
void or_collide_node(const or_config *cfg, const double *fin, double Fx, double Fy, double *fout);
double or_interp(int kernel, int nx, const double *field, double X, double Y);
void or_spread(int kernel, int nx, double *field, double F, double X, double Y, double ds);
int or_dense_A(int kernel, double xc, double yc, double diameter, int nb, double *A);
int or_dfc_lambda(int kernel, double xc, double yc, double diameter, int nb, double *lambda);
/* free-body update pieces (Eq. 23, A3) */
/* st[12]: x y vx vy vpx vpy om Fhx Fhy T dFIMx dFIMy */
void or_body_half_kick(double ms, double mf, double Is, int internal_mass,
                       const double *gvec, double *st);
void or_body_full_kick(double ms, double mf, double Is, const double *gvec, double *st);

#ifdef __cplusplus
}
#endif
#endif
