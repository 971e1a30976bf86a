/*
 * Plain single-threaded FP64 reference ("oracle") of the IB-LBM time step of
 * Jo, arXiv 2609.02298.  TEST INFRASTRUCTURE ONLY: nothing in the product
 * path may link, load or call it; the tests, the smoke check and the CPU
 * baseline of the benchmark are its only users.  It shares no code with the
 * HIP library and is built with -O2 -ffp-contract=off (no fast-math).
 *
 * Everything here is written the slow, obvious way: dense loops over the
 * whole lattice, a 9x9 matrix and Gaussian elimination for the central-moment
 * collision, brute force where a formula allows it.  Each function names the
 * passage of the paper it follows.  Where the paper leaves a detail open the
 * function states the reading taken (the same readings are listed with the
 * design notes of the repository).
 *
 * Parity status: every function below is pinned by a CPU test against a
 * property that the paper or the mathematics fixes (moments, conservation,
 * closed forms, printed worked values, brute force).  None is "parity
 * unpinned".
 */
#include "iblbm_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>

/* D2Q9 lattice (Sec. 2.1, Eq. 1-2): e_0 rest, e_1..4 axial, e_5..8 diagonal. */
static const int EX[9] = {0, 1, 0, -1, 0, 1, -1, -1, 1};
static const int EY[9] = {0, 0, 1, 0, -1, 1, 1, -1, -1};
static const int OPP[9] = {0, 3, 4, 1, 2, 7, 8, 5, 6};
static const double W[9] = {4.0 / 9.0,  1.0 / 9.0,  1.0 / 9.0,  1.0 / 9.0, 1.0 / 9.0,
                            1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0};

#define OR_MAX_BODIES 8

typedef struct {
  or_body_desc d;
  int nb;
  double ds;        /* marker spacing pi*D/N_b (Table I) */
  double radius;
  double omega_mdf; /* MDF relaxation */
  double *X, *Y;    /* marker positions */
  double *Udx, *Udy;
  double *Fx, *Fy;  /* DF/MDF: F_L^total per marker; DFC: F_s per marker */
  double *lambda;   /* DFC */
  double *mdfU;     /* scratch */
  double *mdf_r;    /* MDF residual of each interpolation of the last step */
  int mdf_nr;       /* number of interpolations of the last step */
  /* rigid-body state */
  double xc0, yc0;
  double xc, yc, vx, vy, vpx, vpy, om;
  double vhx, vhy, omh;
  double omp;       /* Omega^(n-1) (Euler-explicit update) */
  double fhx, fhy, torque;
  double dimx, dimy;
  double ms, mf, Is;
  double slip_mean, slip_max, mdf_res;
  int mdf_iters_done;
} or_body;

struct or_sim {
  or_config c;
  int n;        /* nx*ny */
  double *f;    /* post-stream (post-IBM for DFC) populations, 9*n */
  double *fc;   /* post-collision scratch, 9*n */
  double *Fx, *Fy; /* Eulerian IB force density from the last IBM (DF/MDF) */
  double *tmpa, *tmpb, *tmpc; /* scratch fields */
  int nbody;
  or_body body[OR_MAX_BODIES];
  int64_t step;
  int halted;
};

/* ------------------------------------------------------------------ */
/* Equilibrium, Eq. (2): f_i^eq = w_i rho [1 + e.u/cs^2 + (e.u)^2/(2cs^4) - u.u/(2cs^2)],
 * cs^2 = 1/3. */
void or_equilibrium(double rho, double ux, double uy, double *feq) {
  const double cs2 = 1.0 / 3.0;
  double uu = ux * ux + uy * uy;
  for (int i = 0; i < 9; i++) {
    double eu = EX[i] * ux + EY[i] * uy;
    feq[i] = W[i] * rho * (1.0 + eu / cs2 + (eu * eu) / (2.0 * cs2 * cs2) - uu / (2.0 * cs2));
  }
}

/* Guo source without its relaxation prefactor (Eq. 3):
 * S_i = w_i [ (e_i - u)/cs^2 + (e_i.u) e_i / cs^4 ] . F */
static void guo_source(double ux, double uy, double Fx, double Fy, double *S) {
  const double cs2 = 1.0 / 3.0;
  for (int i = 0; i < 9; i++) {
    double eu = EX[i] * ux + EY[i] * uy;
    double ax = (EX[i] - ux) / cs2 + eu * EX[i] / (cs2 * cs2);
    double ay = (EY[i] - uy) / cs2 + eu * EY[i] / (cs2 * cs2);
    S[i] = W[i] * (ax * Fx + ay * Fy);
  }
}

/* Moments with the half-force velocity, Eq. (4). */
static void moments(const double *f, double Fx, double Fy, double *rho, double *ux, double *uy) {
  double r = 0, jx = 0, jy = 0;
  for (int i = 0; i < 9; i++) {
    r += f[i];
    jx += f[i] * EX[i];
    jy += f[i] * EY[i];
  }
  *rho = r;
  *ux = (jx + 0.5 * Fx) / r;
  *uy = (jy + 0.5 * Fy) / r;
}

/* b^e for e = 0, 1, 2 by repeated multiplication (each product rounded
 * once, as a correctly rounded pow would). */
static double ipow(double b, int e) {
  double r = 1.0;
  for (int k = 0; k < e; k++) r *= b;
  return r;
}

/* Solve A x = b (n x n, row-major) by Gaussian elimination with partial
 * pivoting.  A and b are overwritten. */
static void gauss_solve(int n, double *A, double *b, double *x) {
  for (int col = 0; col < n; col++) {
    int piv = col;
    for (int r = col + 1; r < n; r++)
      if (fabs(A[r * n + col]) > fabs(A[piv * n + col])) piv = r;
    if (piv != col) {
      for (int c = 0; c < n; c++) {
        double t = A[col * n + c];
        A[col * n + c] = A[piv * n + c];
        A[piv * n + c] = t;
      }
      double t = b[col];
      b[col] = b[piv];
      b[piv] = t;
    }
    for (int r = col + 1; r < n; r++) {
      double m = A[r * n + col] / A[col * n + col];
      for (int c = col; c < n; c++) A[r * n + c] -= m * A[col * n + c];
      b[r] -= m * b[col];
    }
  }
  for (int r = n - 1; r >= 0; r--) {
    double s = b[r];
    for (int c = r + 1; c < n; c++) s -= A[r * n + c] * x[c];
    x[r] = s / A[r * n + r];
  }
}

/* Collision at one node with body force (Fx,Fy).
 *  BGK + Guo: Eq. (1)-(3).
 *  TRT (Sec. 2.2): even rate s_e = 1/tau sets the viscosity (reading: the
 *    usual choice, and the one for which Lambda_e = Lambda_o is BGK);
 *    Lambda_e = 1/s_e - 1/2, Lambda_o = Lambda_eo / Lambda_e,
 *    s_o = 1/(Lambda_o + 1/2).  The symmetric / antisymmetric source parts
 *    relax with (1 - s_e/2) and (1 - s_o/2).
 *  CM-MRT (Eq. 5): k = T(u) f with rows (e_x-u_x)^p (e_y-u_y)^q in the order
 *    00,10,01,20,02,11,21,12,22; Lambda = diag(0,0,0,w,w,w,s_q,s_q,s_eps),
 *    w = 1/tau.  Reading (the paper defers k^eq and R to its ref. [38]):
 *    k^eq = (rho,0,0,rho/3,rho/3,0,0,0,rho/9), the central moments of the
 *    Maxwellian, and R = (0,Fx,Fy,0,0,0,Fy/3,Fx/3,0), the central moments of
 *    the continuous forcing term.  f = T(u)^-1 k^* by Gaussian elimination. */
void or_collide_node(const or_config *cfg, const double *fin, double Fx, double Fy, double *fout) {
  double rho, ux, uy;
  moments(fin, Fx, Fy, &rho, &ux, &uy);
  double feq[9], S[9];
  or_equilibrium(rho, ux, uy, feq);
  guo_source(ux, uy, Fx, Fy, S);
  if (cfg->collision == OR_BGK) {
    double tau = cfg->tau;
    for (int i = 0; i < 9; i++)
      fout[i] = fin[i] - (fin[i] - feq[i]) / tau + (1.0 - 1.0 / (2.0 * tau)) * S[i];
  } else if (cfg->collision == OR_TRT) {
    double se = 1.0 / cfg->tau;
    double lam_e = 1.0 / se - 0.5;
    double lam_o = cfg->trt_magic / lam_e;
    double so = 1.0 / (lam_o + 0.5);
    for (int i = 0; i < 9; i++) {
      int j = OPP[i];
      double fp = 0.5 * (fin[i] + fin[j]), fm = 0.5 * (fin[i] - fin[j]);
      double ep = 0.5 * (feq[i] + feq[j]), em = 0.5 * (feq[i] - feq[j]);
      double sp = 0.5 * (S[i] + S[j]), sm = 0.5 * (S[i] - S[j]);
      fout[i] = fin[i] - se * (fp - ep) - so * (fm - em) + (1.0 - 0.5 * se) * sp +
                (1.0 - 0.5 * so) * sm;
    }
  } else {
    static const int P[9] = {0, 1, 0, 2, 0, 1, 2, 1, 2};
    static const int Q[9] = {0, 0, 1, 0, 2, 1, 1, 2, 2};
    double T[81], k[9];
    for (int m = 0; m < 9; m++) {
      k[m] = 0.0;
      for (int i = 0; i < 9; i++) {
        T[m * 9 + i] = ipow(EX[i] - ux, P[m]) * ipow(EY[i] - uy, Q[m]);
        k[m] += T[m * 9 + i] * fin[i];
      }
    }
    double w = 1.0 / cfg->tau;
    double lam[9] = {0, 0, 0, w, w, w, cfg->cm_s_q, cfg->cm_s_q, cfg->cm_s_eps};
    double keq[9] = {rho, 0, 0, rho / 3.0, rho / 3.0, 0, 0, 0, rho / 9.0};
    double R[9] = {0, Fx, Fy, 0, 0, 0, Fy / 3.0, Fx / 3.0, 0};
    double ks[9];
    for (int m = 0; m < 9; m++)
      ks[m] = (1.0 - lam[m]) * k[m] + lam[m] * keq[m] + (1.0 - 0.5 * lam[m]) * R[m];
    gauss_solve(9, T, ks, fout);
  }
}

/* ------------------------------------------------------------------ */
/* Regularized delta kernels, Eq. (9) hat and Eq. (10) Peskin 4-point. */
double or_phi(int kernel, double r) {
  double a = fabs(r);
  if (kernel == OR_HAT) return a < 1.0 ? 1.0 - a : 0.0;
  if (a <= 1.0) return 0.125 * (3.0 - 2.0 * a + sqrt(1.0 + 4.0 * a - 4.0 * a * a));
  if (a <= 2.0) return 0.125 * (5.0 - 2.0 * a - sqrt(-7.0 + 12.0 * a - 4.0 * a * a));
  return 0.0;
}

/* Support of a marker at coordinate X along one axis (Sec. 2.4): the hat
 * touches floor(X), floor(X)+1; P4 floor(X)-1 .. floor(X)+2. */
static int support_lo(int kernel, double X) { return (int)floor(X) - (kernel == OR_HAT ? 0 : 1); }
static int support_n(int kernel) { return kernel == OR_HAT ? 2 : 4; }

/* D_h(x - X) h^2 with h = 1, Eq. (6). */
static double delta2(int kernel, double x, double y, double X, double Y) {
  return or_phi(kernel, x - X) * or_phi(kernel, y - Y);
}

/* ------------------------------------------------------------------ */
static void place_markers(or_body *b) {
  /* Markers evenly spaced on the circle (Table I), starting angle 0
   * (reading: the paper does not state it). */
  for (int k = 0; k < b->nb; k++) {
    double th = 2.0 * M_PI * (double)k / (double)b->nb;
    b->X[k] = b->xc + b->radius * cos(th);
    b->Y[k] = b->yc + b->radius * sin(th);
  }
}

static int supports_inside(const or_sim *s, const or_body *b) {
  int ns = support_n(b->d.kernel);
  for (int k = 0; k < b->nb; k++) {
    int x0 = support_lo(b->d.kernel, b->X[k]), y0 = support_lo(b->d.kernel, b->Y[k]);
    if (x0 < 0 || y0 < 0 || x0 + ns - 1 > s->c.nx - 1 || y0 + ns - 1 > s->c.ny - 1) return 0;
  }
  return 1;
}

/* Row sum of the interpolation-spreading matrix of one marker set:
 * Wsum(l) = sum_x D_h(x - X_l) sum_m D_h(x - X_m), via a dense field. */
static void wsum_dense(int nx, int ny, int kernel, int nb, const double *X, const double *Y,
                       double *field, double *wsum) {
  for (int i = 0; i < nx * ny; i++) field[i] = 0.0;
  int ns = support_n(kernel);
  for (int m = 0; m < nb; m++) {
    int x0 = support_lo(kernel, X[m]), y0 = support_lo(kernel, Y[m]);
    for (int jy = 0; jy < ns; jy++)
      for (int jx = 0; jx < ns; jx++) {
        int x = x0 + jx, y = y0 + jy;
        if (x < 0 || y < 0 || x >= nx || y >= ny) continue;
        field[y * nx + x] += delta2(kernel, x, y, X[m], Y[m]);
      }
  }
  for (int l = 0; l < nb; l++) {
    int x0 = support_lo(kernel, X[l]), y0 = support_lo(kernel, Y[l]);
    double s = 0.0;
    for (int jy = 0; jy < ns; jy++)
      for (int jx = 0; jx < ns; jx++) {
        int x = x0 + jx, y = y0 + jy;
        if (x < 0 || y < 0 || x >= nx || y >= ny) continue;
        s += field[y * nx + x] * delta2(kernel, x, y, X[l], Y[l]);
      }
    wsum[l] = s;
  }
}

/* Dense A_lm = sum_x D_h(x-X_l) D_h(x-X_m) ds h^2 (Sec. 2.5.2), built by brute
 * force over every node of a box that holds all supports. */
int or_dense_A(int kernel, double xc, double yc, double diameter, int nb, double *A) {
  double R = 0.5 * diameter, ds = M_PI * diameter / nb;
  double *X = malloc(sizeof(double) * nb), *Y = malloc(sizeof(double) * nb);
  for (int k = 0; k < nb; k++) {
    double th = 2.0 * M_PI * (double)k / (double)nb;
    X[k] = xc + R * cos(th);
    Y[k] = yc + R * sin(th);
  }
  int xlo = (int)floor(xc - R) - 4, xhi = (int)ceil(xc + R) + 4;
  int ylo = (int)floor(yc - R) - 4, yhi = (int)ceil(yc + R) + 4;
  for (int l = 0; l < nb; l++)
    for (int m = 0; m < nb; m++) {
      double s = 0.0;
      for (int y = ylo; y <= yhi; y++)
        for (int x = xlo; x <= xhi; x++)
          s += delta2(kernel, x, y, X[l], Y[l]) * delta2(kernel, x, y, X[m], Y[m]);
      A[l * nb + m] = s * ds;
    }
  free(X);
  free(Y);
  return 0;
}

/* DFC correction scale, Eq. (17), for one circle with rho_f = 1, by brute
 * force over a box holding all supports. */
int or_dfc_lambda(int kernel, double xc, double yc, double diameter, int nb, double *lambda) {
  double R = 0.5 * diameter, ds = M_PI * diameter / nb;
  double *X = malloc(sizeof(double) * nb), *Y = malloc(sizeof(double) * nb);
  for (int k = 0; k < nb; k++) {
    double th = 2.0 * M_PI * (double)k / (double)nb;
    X[k] = xc + R * cos(th);
    Y[k] = yc + R * sin(th);
  }
  int xlo = (int)floor(xc - R) - 4, xhi = (int)ceil(xc + R) + 4;
  int ylo = (int)floor(yc - R) - 4, yhi = (int)ceil(yc + R) + 4;
  for (int k = 0; k < nb; k++) {
    double wsum = 0.0;
    for (int y = ylo; y <= yhi; y++)
      for (int x = xlo; x <= xhi; x++) {
        double dk = delta2(kernel, x, y, X[k], Y[k]);
        if (dk == 0.0) continue;
        double wt = 0.0;
        for (int m = 0; m < nb; m++) wt += delta2(kernel, x, y, X[m], Y[m]);
        wsum += wt * dk;
      }
    lambda[k] = 1.0 / (2.0 * 1.0 * ds * wsum);
  }
  free(X);
  free(Y);
  return 0;
}

/* ------------------------------------------------------------------ */
or_sim *or_create(const or_config *cfg) {
  if (cfg->nx < 3 || cfg->ny < 3 || !(cfg->tau > 0.5)) return NULL;
  or_sim *s = calloc(1, sizeof(or_sim));
  s->c = *cfg;
  s->n = cfg->nx * cfg->ny;
  s->f = calloc((size_t)9 * s->n, sizeof(double));
  s->fc = calloc((size_t)9 * s->n, sizeof(double));
  s->Fx = calloc(s->n, sizeof(double));
  s->Fy = calloc(s->n, sizeof(double));
  s->tmpa = calloc(s->n, sizeof(double));
  s->tmpb = calloc(s->n, sizeof(double));
  s->tmpc = calloc(s->n, sizeof(double));
  /* Initial state (reading; the paper does not give one): equilibrium at
   * rho0 with the inlet / far-field velocity everywhere, else at rest. */
  int nx = cfg->nx, ny = cfg->ny;
  for (int y = 0; y < ny; y++)
    for (int x = 0; x < nx; x++) {
      double ux = 0.0;
      if (cfg->bc[0] == OR_VEL_PARABOLIC)
        ux = 4.0 * cfg->u_bc * (y + 0.5) * (ny - 0.5 - y) / ((double)ny * ny);
      else if (cfg->bc[0] == OR_VEL_UNIFORM || cfg->bc[1] == OR_VEL_UNIFORM ||
               cfg->bc[2] == OR_VEL_UNIFORM || cfg->bc[3] == OR_VEL_UNIFORM)
        ux = cfg->u_bc;
      double feq[9];
      or_equilibrium(cfg->rho0, ux, 0.0, feq);
      for (int i = 0; i < 9; i++) s->f[(size_t)i * s->n + y * nx + x] = feq[i];
    }
  return s;
}

void or_destroy(or_sim *s) {
  if (!s) return;
  for (int b = 0; b < s->nbody; b++) {
    or_body *B = &s->body[b];
    free(B->X); free(B->Y); free(B->Udx); free(B->Udy);
    free(B->Fx); free(B->Fy); free(B->lambda); free(B->mdfU); free(B->mdf_r);
  }
  free(s->f); free(s->fc); free(s->Fx); free(s->Fy);
  free(s->tmpa); free(s->tmpb); free(s->tmpc);
  free(s);
}

int or_add_body(or_sim *s, const or_body_desc *d) {
  if (s->nbody >= OR_MAX_BODIES || d->diameter <= 0) return -1;
  if (s->nbody > 0 && s->body[0].d.scheme != d->scheme) return -1;
  /* the coupled MDF path is a property of the sim: every body agrees, with
   * the same bounds and tolerance */
  if (s->nbody > 0 && d->scheme == OR_MDF &&
      (s->body[0].d.mdf_coupled != d->mdf_coupled ||
       (d->mdf_coupled && (s->body[0].d.mdf_iters != d->mdf_iters ||
                           s->body[0].d.mdf_nmin != d->mdf_nmin ||
                           s->body[0].d.mdf_tol != d->mdf_tol))))
    return -1;
  if (d->scheme == OR_MDF && (d->mdf_iters < 1 || d->mdf_iters > 1000 || (d->mdf_tol > 0.0 && (d->mdf_nmin < 1 || d->mdf_nmin > d->mdf_iters))))
    return -1;
  /* Taylor-Green markers stay where they are placed */
  if (d->udes == OR_UD_TAYLOR_GREEN && (d->motion != OR_FIXED || !(d->tg_k > 0.0) || !(d->tg_nu >= 0.0)))
    return -1;
  if (d->udes != OR_UD_RIGID && d->udes != OR_UD_TAYLOR_GREEN) return -1;
  or_body *b = &s->body[s->nbody];
  memset(b, 0, sizeof(*b));
  b->d = *d;
  b->nb = d->n_markers > 0 ? d->n_markers : (int)lround(M_PI * d->diameter);
  b->radius = 0.5 * d->diameter;
  b->ds = M_PI * d->diameter / b->nb;
  size_t nb = b->nb;
  b->X = calloc(nb, 8); b->Y = calloc(nb, 8); b->Udx = calloc(nb, 8); b->Udy = calloc(nb, 8);
  b->Fx = calloc(nb, 8); b->Fy = calloc(nb, 8); b->lambda = calloc(nb, 8);
  b->mdfU = calloc(2 * nb, 8);
  /* residuals of one step: at most one per pass, plus the first and one per
   * rejected trial of the coupled path (at most three) */
  b->mdf_r = calloc((d->mdf_iters > 0 ? (size_t)d->mdf_iters : 1) + 4, 8);
  b->xc0 = b->xc = d->xc;
  b->yc0 = b->yc = d->yc;
  double rs = d->density_ratio * s->c.rho0, area = M_PI * b->radius * b->radius;
  b->ms = rs * area;
  b->mf = s->c.rho0 * area;
  b->Is = 0.5 * b->ms * b->radius * b->radius;
  place_markers(b);
  if (!supports_inside(s, b)) return -5;
  /* omega_MDF = 1/||A||_inf with ||A||_inf = ds * max_l Wsum(l), once at
   * initialisation (Sec. 2.5.2). */
  b->omega_mdf = d->mdf_omega;
  if (d->scheme == OR_MDF && !(d->mdf_omega > 0.0)) {
    double *ws = malloc(sizeof(double) * nb);
    wsum_dense(s->c.nx, s->c.ny, d->kernel, b->nb, b->X, b->Y, s->tmpa, ws);
    double mx = 0.0;
    for (int l = 0; l < b->nb; l++) mx = ws[l] > mx ? ws[l] : mx;
    b->omega_mdf = 1.0 / (b->ds * mx);
    free(ws);
  }
  return s->nbody++;
}

double or_body_omega(const or_sim *s, int b) { return s->body[b].omega_mdf; }
int or_mdf_residuals(const or_sim *s, int b, double *out) {
  const or_body *B = &s->body[b];
  for (int i = 0; i < B->mdf_nr; i++) out[i] = B->mdf_r[i];
  return B->mdf_nr;
}
int64_t or_steps_done(const or_sim *s) { return s->step; }

/* ------------------------------------------------------------------ */
/* Rigid-body Velocity-Verlet (Eq. 23) with the explicitly lagged
 * internal-mass force of Eq. (A3); torque-only rotation (Sec. 2.7). */
void or_body_half_kick(double ms, double mf, double Is, int internal_mass, const double *g,
                       double *st) {
  /* st: 0 x 1 y 2 vx 3 vy 4 vpx 5 vpy 6 om 7 Fhx 8 Fhy 9 T 10 dFIMx 11 dFIMy.
   * Net gravity F_g = (m_s - m_f) g (Eq. 22); Delta F_IM^n = m_f (v^n - v^(n-1))
   * (Eq. A3, scheme B-2) or 0 (scheme A), held for both half-kicks. */
  double Fgx = (ms - mf) * g[0], Fgy = (ms - mf) * g[1];
  st[10] = internal_mass == OR_IM_FENG ? mf * (st[2] - st[4]) : 0.0;
  st[11] = internal_mass == OR_IM_FENG ? mf * (st[3] - st[5]) : 0.0;
  st[4] = st[2];
  st[5] = st[3];
  st[2] += (st[7] + Fgx + st[10]) / (2.0 * ms);
  st[3] += (st[8] + Fgy + st[11]) / (2.0 * ms);
  st[0] += st[2];
  st[1] += st[3];
  st[6] += st[9] / (2.0 * Is);
}

/* Second half-kick with the new hydrodynamic force and torque in st[7..9]. */
void or_body_full_kick(double ms, double mf, double Is, const double *g, double *st) {
  double Fgx = (ms - mf) * g[0], Fgy = (ms - mf) * g[1];
  st[2] += (st[7] + Fgx + st[10]) / (2.0 * ms);
  st[3] += (st[8] + Fgy + st[11]) / (2.0 * ms);
  st[6] += st[9] / (2.0 * Is);
}

/* Euler-explicit update of Eq. (A1), the integrator of the paper's
 * wake-interaction cross-check: v^(n+1) = (1 + r) v^n - r v^(n-1) +
 * (F_hydro^n + F_g)/m_s with r = m_f/m_s (= rho_f/rho_s) for the Feng form
 * and r = 0 without it.  The rotation carries the internal angular-momentum
 * increment in both arms (Sec. 2.7: the ablation of Sec. 5.2 holds the
 * rotational update fixed and toggles only the translational correction):
 * Omega^(n+1) = (1 + q) Omega^n - q Omega^(n-1) + T^n/I_s with q = I_f/I_s
 * = m_f/m_s (reading: the increment is that of the rigid interior,
 * I_f (Omega^n - Omega^(n-1))); X^(n+1) = X^n + v^(n+1) (reading).
 * st: 0 x 1 y 2 vx 3 vy 4 vpx 5 vpy 6 om 7 Fhx 8 Fhy 9 T 10 Omega^(n-1);
 * on return 2,3,6 hold the new velocities, 4,5,10 the old. */
void or_body_euler(double ms, double mf, double Is, int internal_mass, const double *g, double *st) {
  const double r = internal_mass == OR_IM_FENG ? mf / ms : 0.0;
  const double Fgx = (ms - mf) * g[0], Fgy = (ms - mf) * g[1];
  const double vx = (1.0 + r) * st[2] - r * st[4] + (st[7] + Fgx) / ms;
  const double vy = (1.0 + r) * st[3] - r * st[5] + (st[8] + Fgy) / ms;
  const double q = mf / ms;
  const double om = (1.0 + q) * st[6] - q * st[10] + st[9] / Is;
  st[4] = st[2];
  st[5] = st[3];
  st[10] = st[6];
  st[2] = vx;
  st[3] = vy;
  st[6] = om;
  st[0] += vx;
  st[1] += vy;
}

static void body_pre(or_sim *s, or_body *b, int64_t n) {
  double t1 = (double)(n + 1);
  if (b->d.motion == OR_FIXED) {
    b->vhx = b->vhy = b->omh = 0.0;
  } else if (b->d.motion == OR_PRESCRIBED_SIN) {
    /* X_c(t) = X_c0 + amp sin(2 pi f t + phase), U = dX_c/dt at t_{n+1} */
    double ph = 2.0 * M_PI * b->d.freq * t1 + b->d.phase;
    b->xc = b->xc0 + b->d.amp[0] * sin(ph);
    b->yc = b->yc0 + b->d.amp[1] * sin(ph);
    b->vhx = b->d.amp[0] * 2.0 * M_PI * b->d.freq * cos(ph);
    b->vhy = b->d.amp[1] * 2.0 * M_PI * b->d.freq * cos(ph);
    b->vx = b->vhx;
    b->vy = b->vhy;
    b->omh = 0.0;
  } else if (b->d.integrator == OR_EULER_A1) {
    double st[12] = {b->xc, b->yc, b->vx, b->vy, b->vpx, b->vpy, b->om,
                     b->fhx, b->fhy, b->torque, b->omp, 0};
    or_body_euler(b->ms, b->mf, b->Is, b->d.internal_mass, s->c.gravity, st);
    b->xc = st[0]; b->yc = st[1];
    b->vx = b->vhx = st[2]; b->vy = b->vhy = st[3]; b->om = b->omh = st[6];
    b->vpx = st[4]; b->vpy = st[5]; b->omp = st[10];
    b->dimx = b->dimy = 0.0;
  } else {
    double st[12] = {b->xc, b->yc, b->vx, b->vy, b->vpx, b->vpy, b->om,
                     b->fhx, b->fhy, b->torque, 0, 0};
    or_body_half_kick(b->ms, b->mf, b->Is, b->d.internal_mass, s->c.gravity, st);
    b->xc = st[0]; b->yc = st[1]; b->vhx = st[2]; b->vhy = st[3];
    b->vpx = st[4]; b->vpy = st[5]; b->omh = st[6];
    b->dimx = st[10]; b->dimy = st[11];
  }
  place_markers(b);
  /* Rigid-body marker velocity U_d = v + Omega x (X_k - X_c) (Sec. 2.7).
   * Reading: under Velocity-Verlet v and Omega are the last full-step
   * values v^n, Omega^n, still in b->vx, b->vy, b->om here; the half-step
   * values only advance the position.  Otherwise the velocity just set. */
  const int verlet = b->d.motion == OR_FREE && b->d.integrator != OR_EULER_A1;
  const double ux = verlet ? b->vx : b->vhx, uy = verlet ? b->vy : b->vhy;
  const double uo = verlet ? b->om : b->omh;
  for (int k = 0; k < b->nb; k++) {
    double rx = b->X[k] - b->xc, ry = b->Y[k] - b->yc;
    b->Udx[k] = ux - uo * ry;
    b->Udy[k] = uy + uo * rx;
  }
  if (b->d.udes == OR_UD_TAYLOR_GREEN) {
    /* IB-LBM mode of the Taylor-Green check (App. D.1): the desired velocity
     * of each (fixed) marker is the decaying vortex of Eq. D1 at the marker,
     * with the origin at node (0, 0).  Reading: it is evaluated at t_(n+1),
     * the time level the step advances to, as the prescribed kinematics
     * above are. */
    const double k = b->d.tg_k, t = t1;
    const double amp = b->d.tg_u0 * exp(-2.0 * b->d.tg_nu * k * k * t);
    for (int m = 0; m < b->nb; m++) {
      b->Udx[m] = -amp * cos(k * b->X[m]) * sin(k * b->Y[m]);
      b->Udy[m] = amp * sin(k * b->X[m]) * cos(k * b->Y[m]);
    }
  }
}

static void body_post(or_sim *s, or_body *b) {
  if (b->d.motion != OR_FREE || b->d.integrator == OR_EULER_A1) return;
  double st[12] = {b->xc, b->yc, b->vhx, b->vhy, b->vpx, b->vpy, b->omh,
                   b->fhx, b->fhy, b->torque, b->dimx, b->dimy};
  or_body_full_kick(b->ms, b->mf, b->Is, s->c.gravity, st);
  b->vx = st[2]; b->vy = st[3]; b->om = st[6];
}

/* ------------------------------------------------------------------ */
/* Collide every node, Eq. (1)-(5).  The force is the IB force of the last
 * IBM pass (zero for DFC, Sec. 2.5.3) plus the uniform fluid force. */
static void collide_all(or_sim *s) {
  int n = s->n;
  for (int p = 0; p < n; p++) {
    double fin[9], fout[9];
    for (int i = 0; i < 9; i++) fin[i] = s->f[(size_t)i * n + p];
    double Fx = s->Fx[p] + s->c.fluid_force[0], Fy = s->Fy[p] + s->c.fluid_force[1];
    or_collide_node(&s->c, fin, Fx, Fy, fout);
    for (int i = 0; i < 9; i++) s->fc[(size_t)i * n + p] = fout[i];
  }
}

/* Wall velocity of a velocity face for a link leaving node row y along e_i:
 * the parabola is evaluated at the link mid-point (reading). */
static void face_velocity(const or_sim *s, int face, int y, int i, double *uwx, double *uwy) {
  int ny = s->c.ny;
  *uwy = 0.0;
  if (s->c.bc[face] == OR_VEL_PARABOLIC) {
    double ym = y + 0.5 * EY[i];
    *uwx = 4.0 * s->c.u_bc * (ym + 0.5) * (ny - 0.5 - ym) / ((double)ny * ny);
  } else {
    *uwx = s->c.u_bc;
  }
}

/* Streaming f_i(x + e_i) <- f_i^post(x) (Eq. 1) with the boundary faces.
 * Readings (the paper names its faces but not their closures, except the
 * Zou-He walls of the sedimentation runs):
 *   wall: half-way bounce-back, f_opp(i)(x) <- f_i^post(x);
 *   velocity face: f_opp(i)(x) <- f_i^post(x) - 6 w_i rho0 (e_i . u_w);
 *   a link leaving through a wall and a velocity face is treated as wall;
 *   zero-gradient face: after streaming, the populations entering through
 *   the face at its node line are copied from the adjacent interior line;
 *   periodic: wrap-around. */
static void stream_all(or_sim *s) {
  int nx = s->c.nx, ny = s->c.ny, n = s->n;
  const int *bc = s->c.bc;
  for (int y = 0; y < ny; y++)
    for (int x = 0; x < nx; x++)
      for (int i = 0; i < 9; i++) {
        double p = s->fc[(size_t)i * n + y * nx + x];
        int xd = x + EX[i], yd = y + EY[i];
        int cross[4] = {xd < 0, xd > nx - 1, yd < 0, yd > ny - 1};
        if (cross[0] && bc[0] == OR_PERIODIC) { xd += nx; cross[0] = 0; }
        if (cross[1] && bc[1] == OR_PERIODIC) { xd -= nx; cross[1] = 0; }
        if (cross[2] && bc[2] == OR_PERIODIC) { yd += ny; cross[2] = 0; }
        if (cross[3] && bc[3] == OR_PERIODIC) { yd -= ny; cross[3] = 0; }
        if (!cross[0] && !cross[1] && !cross[2] && !cross[3]) {
          s->f[(size_t)i * n + yd * nx + xd] = p;
          continue;
        }
        int wall = 0, vel = -1;
        for (int fce = 0; fce < 4; fce++) {
          if (!cross[fce]) continue;
          if (bc[fce] == OR_BOUNCE_BACK) wall = 1;
          if ((bc[fce] == OR_VEL_PARABOLIC || bc[fce] == OR_VEL_UNIFORM) && vel < 0) vel = fce;
        }
        if (wall) {
          s->f[(size_t)OPP[i] * n + y * nx + x] = p;
        } else if (vel >= 0) {
          double uwx, uwy;
          face_velocity(s, vel, y, i, &uwx, &uwy);
          s->f[(size_t)OPP[i] * n + y * nx + x] =
              p - 6.0 * W[i] * s->c.rho0 * (EX[i] * uwx + EY[i] * uwy);
        }
        /* a link leaving only through zero-gradient faces is dropped; the
         * copy below fills the entering populations */
      }
  /* zero-gradient copies, faces in the order W, E, S, N */
  for (int fce = 0; fce < 4; fce++) {
    if (bc[fce] != OR_ZERO_GRADIENT) continue;
    for (int i = 0; i < 9; i++) {
      int enters = (fce == 0 && EX[i] > 0) || (fce == 1 && EX[i] < 0) ||
                   (fce == 2 && EY[i] > 0) || (fce == 3 && EY[i] < 0);
      if (!enters) continue;
      if (fce < 2) {
        int xb = fce == 0 ? 0 : nx - 1, xi = fce == 0 ? 1 : nx - 2;
        for (int y = 0; y < ny; y++)
          s->f[(size_t)i * n + y * nx + xb] = s->f[(size_t)i * n + y * nx + xi];
      } else {
        int yb = fce == 2 ? 0 : ny - 1, yi = fce == 2 ? 1 : ny - 2;
        for (int x = 0; x < nx; x++)
          s->f[(size_t)i * n + yb * nx + x] = s->f[(size_t)i * n + yi * nx + x];
      }
    }
  }
}

/* No-slip walls with the on-node velocity closure of Zou and He at zero wall
 * velocity (the walls of Sec. 2.9.3-2.9.4).  The wall nodes are the face
 * nodes themselves; after streaming, the populations that would have come
 * from outside are rebuilt from the known ones so that the node has zero
 * momentum: the normal one by bounce-back of its opposite, the two diagonal
 * ones by bounce-back corrected with half the tangential imbalance of the
 * known axial pair (for the south wall f2 = f4, f5 = f7 - (f1 - f3)/2,
 * f6 = f8 + (f1 - f3)/2; the other walls by symmetry).  A corner of two such
 * walls has five unknowns: the three pointing into the fluid are bounce-back
 * of their opposites and the two buried diagonals share what the density of
 * the diagonal inner node leaves (reading: the paper does not give the
 * corner rule; this is the usual one).  Links that leave through these faces
 * were dropped by the streaming. */
static void zou_he_walls(or_sim *s) {
  int nx = s->c.nx, ny = s->c.ny, n = s->n;
  const int *bc = s->c.bc;
  double *f = s->f;
#define F(i, x, y) f[(size_t)(i) * n + (size_t)(y) * nx + (x)]
  for (int y = 0; y < ny; y++)
    for (int x = 0; x < nx; x++) {
      int w = x == 0 && bc[0] == OR_ZOU_HE, e = x == nx - 1 && bc[1] == OR_ZOU_HE;
      int so = y == 0 && bc[2] == OR_ZOU_HE, no = y == ny - 1 && bc[3] == OR_ZOU_HE;
      if ((w || e) && (so || no)) {
        /* corner: i_in are the axial and diagonal populations pointing into
         * the fluid, a and b the buried diagonals */
        int sx = w ? 1 : -1, sy = so ? 1 : -1;
        int ix = sx > 0 ? 1 : 3, iy = sy > 0 ? 2 : 4;
        int id = -1, ia = -1, ib = -1;
        for (int i = 5; i < 9; i++) {
          if (EX[i] == sx && EY[i] == sy) id = i;
          else if (EX[i] == -sx && EY[i] == sy) ia = i;
          else if (EX[i] == sx && EY[i] == -sy) ib = i;
        }
        F(ix, x, y) = F(OPP[ix], x, y);
        F(iy, x, y) = F(OPP[iy], x, y);
        F(id, x, y) = F(OPP[id], x, y);
        double rc = 0.0;
        for (int i = 0; i < 9; i++) rc += F(i, x + sx, y + sy);
        double known = 0.0;
        for (int i = 0; i < 9; i++)
          if (i != ia && i != ib) known += F(i, x, y);
        F(ia, x, y) = F(ib, x, y) = 0.5 * (rc - known);
      } else if (so || no) {
        int in = so ? 2 : 4;               /* normal population into the fluid */
        int d1 = so ? 5 : 8, d2 = so ? 6 : 7; /* diagonals into the fluid, +x and -x */
        double t = 0.5 * (F(1, x, y) - F(3, x, y));
        F(in, x, y) = F(OPP[in], x, y);
        F(d1, x, y) = F(OPP[d1], x, y) - t;
        F(d2, x, y) = F(OPP[d2], x, y) + t;
      } else if (w || e) {
        int in = w ? 1 : 3;
        int d1 = w ? 5 : 6, d2 = w ? 8 : 7;   /* diagonals into the fluid, +y and -y */
        double t = 0.5 * (F(2, x, y) - F(4, x, y));
        F(in, x, y) = F(OPP[in], x, y);
        F(d1, x, y) = F(OPP[d1], x, y) - t;
        F(d2, x, y) = F(OPP[d2], x, y) + t;
      }
    }
#undef F
}

/* ------------------------------------------------------------------ */
/* Interpolation of a scalar field to (X,Y), Eq. (7). */
static double interp_nx(int nx, int kernel, const double *field, double X, double Y) {
  int ns = support_n(kernel);
  int x0 = support_lo(kernel, X), y0 = support_lo(kernel, Y);
  double acc = 0.0;
  for (int jy = 0; jy < ns; jy++)
    for (int jx = 0; jx < ns; jx++) {
      int x = x0 + jx, y = y0 + jy;
      acc += field[y * nx + x] * delta2(kernel, x, y, X, Y);
    }
  return acc;
}

/* Spreading of a marker quantity into a field, Eq. (8): field += F D_h ds. */
static void spread_nx(int nx, int kernel, double *field, double F, double X, double Y,
                      double ds) {
  int ns = support_n(kernel);
  int x0 = support_lo(kernel, X), y0 = support_lo(kernel, Y);
  for (int jy = 0; jy < ns; jy++)
    for (int jx = 0; jx < ns; jx++) {
      int x = x0 + jx, y = y0 + jy;
      field[y * nx + x] += F * delta2(kernel, x, y, X, Y) * ds;
    }
}

static double interp(const or_sim *s, int kernel, const double *field, double X, double Y) {
  return interp_nx(s->c.nx, kernel, field, X, Y);
}
static void spread_add(const or_sim *s, int kernel, double *field, double F, double X, double Y,
                       double ds) {
  spread_nx(s->c.nx, kernel, field, F, X, Y, ds);
}

/* Exported for the pins: stencil interpolation / spreading on an nx-wide
 * field (the caller keeps the support inside the field). */
double or_interp(int kernel, int nx, const double *field, double X, double Y) {
  return interp_nx(nx, kernel, field, X, Y);
}
void or_spread(int kernel, int nx, double *field, double F, double X, double Y, double ds) {
  spread_nx(nx, kernel, field, F, X, Y, ds);
}

/* Fluid density and force-free velocity u* of the post-stream field. */
static void post_stream_moments(const or_sim *s, double *rho, double *ux, double *uy) {
  int n = s->n;
  for (int p = 0; p < n; p++) {
    double r = 0, jx = 0, jy = 0;
    for (int i = 0; i < 9; i++) {
      double v = s->f[(size_t)i * n + p];
      r += v;
      jx += v * EX[i];
      jy += v * EY[i];
    }
    rho[p] = r;
    ux[p] = jx / r;
    uy[p] = jy / r;
  }
}

/* Direct forcing, Eq. (11) with interpolation Eq. (7) and spreading Eq. (8). */
static void ibm_df(or_sim *s) {
  int n = s->n;
  double *rho = s->tmpa, *ux = s->tmpb, *uy = s->tmpc;
  post_stream_moments(s, rho, ux, uy);
  for (int p = 0; p < n; p++) s->Fx[p] = s->Fy[p] = 0.0;
  for (int b = 0; b < s->nbody; b++) {
    or_body *B = &s->body[b];
    for (int k = 0; k < B->nb; k++) {
      double rX = interp(s, B->d.kernel, rho, B->X[k], B->Y[k]);
      double Ux = interp(s, B->d.kernel, ux, B->X[k], B->Y[k]);
      double Uy = interp(s, B->d.kernel, uy, B->X[k], B->Y[k]);
      B->Fx[k] = 2.0 * rX * (B->Udx[k] - Ux);
      B->Fy[k] = 2.0 * rX * (B->Udy[k] - Uy);
    }
    B->mdf_iters_done = 1;
    B->mdf_res = 0.0;
  }
  for (int b = 0; b < s->nbody; b++) {
    or_body *B = &s->body[b];
    for (int k = 0; k < B->nb; k++) {
      spread_add(s, B->d.kernel, s->Fx, B->Fx[k], B->X[k], B->Y[k], B->ds);
      spread_add(s, B->d.kernel, s->Fy, B->Fy[k], B->X[k], B->Y[k], B->ds);
    }
  }
}

/* Multi-direct forcing, Eq. (12)-(14).  Pass n interpolates U^(n) from the
 * node velocities u^(n-1), forms F^(n) = 2 rho(X_k) (U_d - U^(n)) and adds
 * omega/(2 rho) spread(F^(n)) to the node velocities; F_total = sum_n omega
 * F^(n), and the Eulerian force is the spread of F_total.  rho(X_k) is
 * interpolated once per step.  The bodies iterate one after the other: no
 * node lies in the supports of two bodies (the library refuses such bodies),
 * so a body's passes change only its own nodes and the order of the bodies
 * does not matter.
 *
 * Fixed form (mdf_tol <= 0): mdf_iters passes.  Adaptive form (mdf_tol > 0,
 * Sec. 2.5.2 and App. A.2): the residual r_n = max_k |U_d - U^(n)(X_k)| is
 * measured before pass n is applied, and the iteration ends there, without
 * pass n, once at least mdf_nmin passes are done and r_n < mdf_tol, or when
 * r_n > 1.5 r_{n-1} (divergence guard); it applies at most mdf_iters passes.
 * Reading: the guard holds from the second interpolation on, also before
 * mdf_nmin passes are done.  The reported residual is that of the last
 * interpolation, the count that of the passes applied. */
static void ibm_mdf(or_sim *s) {
  int n = s->n;
  double *rho = s->tmpa, *ux = s->tmpb, *uy = s->tmpc;
  post_stream_moments(s, rho, ux, uy);
  double *sx = calloc(n, sizeof(double)), *sy = calloc(n, sizeof(double));
  for (int b = 0; b < s->nbody; b++) {
    or_body *B = &s->body[b];
    double *ex = B->mdfU, *ey = B->mdfU + B->nb;
    double *rX = calloc(B->nb, sizeof(double));
    for (int k = 0; k < B->nb; k++) {
      B->Fx[k] = B->Fy[k] = 0.0;
      rX[k] = interp(s, B->d.kernel, rho, B->X[k], B->Y[k]);
    }
    const int adaptive = B->d.mdf_tol > 0.0;
    double rprev = 0.0;
    B->mdf_iters_done = 0;
    B->mdf_nr = 0;
    for (int it = 1; it <= B->d.mdf_iters; it++) {
      double res = 0.0;
      for (int k = 0; k < B->nb; k++) {
        ex[k] = B->Udx[k] - interp(s, B->d.kernel, ux, B->X[k], B->Y[k]);
        ey[k] = B->Udy[k] - interp(s, B->d.kernel, uy, B->X[k], B->Y[k]);
        double r = sqrt(ex[k] * ex[k] + ey[k] * ey[k]);
        res = r > res ? r : res;
      }
      B->mdf_res = res;
      B->mdf_r[B->mdf_nr++] = res;
      if (adaptive && ((it > B->d.mdf_nmin && res < B->d.mdf_tol) || (it > 1 && res > 1.5 * rprev)))
        break;
      rprev = res;
      for (int p = 0; p < n; p++) sx[p] = sy[p] = 0.0;
      for (int k = 0; k < B->nb; k++) {
        double Fnx = 2.0 * rX[k] * ex[k], Fny = 2.0 * rX[k] * ey[k];
        B->Fx[k] += B->omega_mdf * Fnx;
        B->Fy[k] += B->omega_mdf * Fny;
        spread_add(s, B->d.kernel, sx, B->omega_mdf * Fnx, B->X[k], B->Y[k], B->ds);
        spread_add(s, B->d.kernel, sy, B->omega_mdf * Fny, B->X[k], B->Y[k], B->ds);
      }
      for (int p = 0; p < n; p++) {
        ux[p] += sx[p] / (2.0 * rho[p]);
        uy[p] += sy[p] / (2.0 * rho[p]);
      }
      B->mdf_iters_done = it;
    }
    free(rX);
  }
  for (int p = 0; p < n; p++) s->Fx[p] = s->Fy[p] = 0.0;
  for (int b = 0; b < s->nbody; b++) {
    or_body *B = &s->body[b];
    for (int k = 0; k < B->nb; k++) {
      spread_add(s, B->d.kernel, s->Fx, B->Fx[k], B->X[k], B->Y[k], B->ds);
      spread_add(s, B->d.kernel, s->Fy, B->Fy[k], B->X[k], B->Y[k], B->ds);
    }
  }
  free(sx);
  free(sy);
}

/* Largest |U_d - U(X_k)| over every marker of every body, with U
 * interpolated from the node velocities (ux, uy); the per-marker errors go
 * to each body's mdfU (x then y). */
static double joint_residual(or_sim *s, const double *ux, const double *uy) {
  double res = 0.0;
  for (int b = 0; b < s->nbody; b++) {
    or_body *B = &s->body[b];
    double *ex = B->mdfU, *ey = B->mdfU + B->nb;
    for (int k = 0; k < B->nb; k++) {
      ex[k] = B->Udx[k] - interp(s, B->d.kernel, ux, B->X[k], B->Y[k]);
      ey[k] = B->Udy[k] - interp(s, B->d.kernel, uy, B->X[k], B->Y[k]);
      double r = sqrt(ex[k] * ex[k] + ey[k] * ey[k]);
      res = r > res ? r : res;
    }
  }
  return res;
}

static void record_residual(or_sim *s, double r) {
  for (int b = 0; b < s->nbody; b++) {
    or_body *B = &s->body[b];
    if (B->mdf_nr < B->d.mdf_iters + 4) B->mdf_r[B->mdf_nr++] = r;
  }
}

/* Coupled multi-body MDF (Sec. 2.5.2, the two-particle path): the bodies'
 * forces share the fluid update of every pass, and the iteration is
 * controlled on the residual of all markers together.  Reading of the
 * paper's controls, in its order:
 *   - each body's initial relaxation is omega_0 = min(omega_MDF, 0.8), and
 *     a common factor c (1 at the start of every step) scales them;
 *   - a pass is a trial: F^(n) = 2 rho(X_k)(U_d - U) from the current
 *     interpolation, u += c omega_0/(2 rho) spread(F^(n)) for every body,
 *     then the joint residual R' of the new velocities;
 *   - if R' > 1.2 R (R: the residual before the trial) the trial is
 *     rejected: the velocities return to their state before it and c is
 *     halved; the iteration ends once c reaches 0.125, else the same F^(n)
 *     is tried again with the halved factor;
 *   - an accepted trial adds c omega_0 F^(n) to F_total and counts as a
 *     pass; the iteration ends once at least mdf_nmin passes are accepted
 *     and R < mdf_tol (when mdf_tol > 0), or after mdf_iters accepted passes.
 * The single-body guard r_n > 1.5 r_(n-1) is not used on this path.  Every
 * body reports the joint residual and the number of accepted passes. */
static void ibm_mdf_coupled(or_sim *s) {
  int n = s->n;
  double *rho = s->tmpa, *ux = s->tmpb, *uy = s->tmpc;
  post_stream_moments(s, rho, ux, uy);
  double *sx = calloc(n, sizeof(double)), *sy = calloc(n, sizeof(double));
  double *pux = malloc(sizeof(double) * n), *puy = malloc(sizeof(double) * n);
  double *rX[OR_MAX_BODIES], *Fn[OR_MAX_BODIES], om0[OR_MAX_BODIES];
  for (int b = 0; b < s->nbody; b++) {
    or_body *B = &s->body[b];
    rX[b] = calloc(B->nb, sizeof(double));
    Fn[b] = calloc(2 * (size_t)B->nb, sizeof(double));
    for (int k = 0; k < B->nb; k++) {
      B->Fx[k] = B->Fy[k] = 0.0;
      rX[b][k] = interp(s, B->d.kernel, rho, B->X[k], B->Y[k]);
    }
    om0[b] = B->omega_mdf < 0.8 ? B->omega_mdf : 0.8;
    B->mdf_nr = 0;
  }
  const or_body_desc *d0 = &s->body[0].d;
  const int nmax = d0->mdf_iters, nmin = d0->mdf_tol > 0.0 ? d0->mdf_nmin : d0->mdf_iters;
  double c = 1.0;
  double R = joint_residual(s, ux, uy);
  record_residual(s, R);
  int accepted = 0;
  for (;;) {
    if (accepted >= nmax || (d0->mdf_tol > 0.0 && accepted >= nmin && R < d0->mdf_tol)) break;
    for (int b = 0; b < s->nbody; b++) {
      or_body *B = &s->body[b];
      const double *ex = B->mdfU, *ey = B->mdfU + B->nb;
      for (int k = 0; k < B->nb; k++) {
        Fn[b][k] = 2.0 * rX[b][k] * ex[k];
        Fn[b][B->nb + k] = 2.0 * rX[b][k] * ey[k];
      }
    }
    memcpy(pux, ux, sizeof(double) * n);
    memcpy(puy, uy, sizeof(double) * n);
    int stop = 0;
    for (;;) {
      for (int p = 0; p < n; p++) sx[p] = sy[p] = 0.0;
      for (int b = 0; b < s->nbody; b++) {
        or_body *B = &s->body[b];
        const double w = c * om0[b];
        for (int k = 0; k < B->nb; k++) {
          spread_add(s, B->d.kernel, sx, w * Fn[b][k], B->X[k], B->Y[k], B->ds);
          spread_add(s, B->d.kernel, sy, w * Fn[b][B->nb + k], B->X[k], B->Y[k], B->ds);
        }
      }
      for (int p = 0; p < n; p++) {
        ux[p] = pux[p] + sx[p] / (2.0 * rho[p]);
        uy[p] = puy[p] + sy[p] / (2.0 * rho[p]);
      }
      const double Rt = joint_residual(s, ux, uy);
      record_residual(s, Rt);
      if (!(Rt > 1.2 * R)) {
        for (int b = 0; b < s->nbody; b++) {
          or_body *B = &s->body[b];
          const double w = c * om0[b];
          for (int k = 0; k < B->nb; k++) {
            B->Fx[k] += w * Fn[b][k];
            B->Fy[k] += w * Fn[b][B->nb + k];
          }
        }
        accepted++;
        R = Rt;
        break;
      }
      /* reject: back to the velocities before the trial */
      memcpy(ux, pux, sizeof(double) * n);
      memcpy(uy, puy, sizeof(double) * n);
      c *= 0.5;
      if (c <= 0.125) {
        stop = 1;
        break;
      }
    }
    if (stop) {
      (void)joint_residual(s, ux, uy); /* per-marker errors of the kept state */
      break;
    }
  }
  for (int b = 0; b < s->nbody; b++) {
    or_body *B = &s->body[b];
    B->mdf_res = R;
    B->mdf_iters_done = accepted;
    free(rX[b]);
    free(Fn[b]);
  }
  for (int p = 0; p < n; p++) s->Fx[p] = s->Fy[p] = 0.0;
  for (int b = 0; b < s->nbody; b++) {
    or_body *B = &s->body[b];
    for (int k = 0; k < B->nb; k++) {
      spread_add(s, B->d.kernel, s->Fx, B->Fx[k], B->X[k], B->Y[k], B->ds);
      spread_add(s, B->d.kernel, s->Fy, B->Fy[k], B->X[k], B->Y[k], B->ds);
    }
  }
  free(sx);
  free(sy);
  free(pux);
  free(puy);
}

/* Distribution-function correction, Eq. (15)-(20).  All markers of all
 * bodies interpolate the uncorrected post-stream field first (one Jacobi
 * pass); W_total sums D_h over every marker of every body; rho_f = rho0. */
static void ibm_dfc(or_sim *s) {
  int n = s->n, nx = s->c.nx;
  double rf = s->c.rho0;
  for (int p = 0; p < n; p++) s->Fx[p] = s->Fy[p] = 0.0;
  double *Wt = s->tmpa;
  for (int p = 0; p < n; p++) Wt[p] = 0.0;
  for (int b = 0; b < s->nbody; b++) {
    or_body *B = &s->body[b];
    for (int k = 0; k < B->nb; k++) spread_add(s, B->d.kernel, Wt, 1.0, B->X[k], B->Y[k], 1.0);
  }
  double **df = calloc(s->nbody, sizeof(double *));
  for (int b = 0; b < s->nbody; b++) {
    or_body *B = &s->body[b];
    df[b] = calloc((size_t)9 * B->nb, sizeof(double));
    for (int k = 0; k < B->nb; k++) {
      double wsum = interp(s, B->d.kernel, Wt, B->X[k], B->Y[k]);
      B->lambda[k] = 1.0 / (2.0 * rf * B->ds * wsum);
      double fs[9];
      for (int i = 0; i < 9; i++) fs[i] = interp(s, B->d.kernel, s->f + (size_t)i * n, B->X[k], B->Y[k]);
      double Fsx = 0.0, Fsy = 0.0;
      for (int i = 0; i < 9; i++) {
        const double cs2 = 1.0 / 3.0;
        double fbar = fs[OPP[i]] + 2.0 * W[i] * rf * (EX[i] * B->Udx[k] + EY[i] * B->Udy[k]) / cs2;
        double d = B->lambda[k] * (fbar - fs[i]);
        df[b][(size_t)9 * k + i] = d;
        Fsx += EX[i] * d;
        Fsy += EY[i] * d;
      }
      B->Fx[k] = -B->ds * Fsx;
      B->Fy[k] = -B->ds * Fsy;
    }
    B->mdf_iters_done = 0;
    B->mdf_res = 0.0;
  }
  for (int b = 0; b < s->nbody; b++) {
    or_body *B = &s->body[b];
    for (int k = 0; k < B->nb; k++)
      for (int i = 0; i < 9; i++)
        spread_add(s, B->d.kernel, s->f + (size_t)i * n, df[b][(size_t)9 * k + i], B->X[k], B->Y[k],
                   B->ds);
    free(df[b]);
  }
  free(df);
  (void)nx;
}

/* Hydrodynamic force and torque (Sec. 2.7): DF/MDF by Newton's third law
 * from the Eulerian force spread by the body's own markers,
 * F_hydro = -sum_x f(x) h^2 and T = -sum_k (X_k - X_c) x F_L ds; DFC from the
 * particle-side marker forces F_hydro = sum_k F_s, T = sum_k (X_k-X_c) x F_s. */
static void body_forces(or_sim *s) {
  int n = s->n;
  for (int b = 0; b < s->nbody; b++) {
    or_body *B = &s->body[b];
    double fx = 0, fy = 0, tq = 0;
    if (B->d.scheme == OR_DFC) {
      for (int k = 0; k < B->nb; k++) {
        fx += B->Fx[k];
        fy += B->Fy[k];
        tq += (B->X[k] - B->xc) * B->Fy[k] - (B->Y[k] - B->yc) * B->Fx[k];
      }
    } else {
      double *ex = calloc(n, sizeof(double)), *ey = calloc(n, sizeof(double));
      for (int k = 0; k < B->nb; k++) {
        spread_add(s, B->d.kernel, ex, B->Fx[k], B->X[k], B->Y[k], B->ds);
        spread_add(s, B->d.kernel, ey, B->Fy[k], B->X[k], B->Y[k], B->ds);
        tq -= ((B->X[k] - B->xc) * B->Fy[k] - (B->Y[k] - B->yc) * B->Fx[k]) * B->ds;
      }
      for (int p = 0; p < n; p++) {
        fx -= ex[p];
        fy -= ey[p];
      }
      free(ex);
      free(ey);
    }
    B->fhx = fx;
    B->fhy = fy;
    B->torque = tq;
  }
}

/* Post-IB velocity (u* + f/2rho for DF/MDF, moments of the corrected
 * populations for DFC) and marker slip |interp(u) - U_d| (Sec. 2.8). */
static void body_slip(or_sim *s) {
  double *rho = s->tmpa, *ux = s->tmpb, *uy = s->tmpc;
  or_fields(s, rho, ux, uy);
  for (int b = 0; b < s->nbody; b++) {
    or_body *B = &s->body[b];
    double sm = 0, mx = 0;
    for (int k = 0; k < B->nb; k++) {
      double Ux = interp(s, B->d.kernel, ux, B->X[k], B->Y[k]);
      double Uy = interp(s, B->d.kernel, uy, B->X[k], B->Y[k]);
      double e = sqrt((Ux - B->Udx[k]) * (Ux - B->Udx[k]) + (Uy - B->Udy[k]) * (Uy - B->Udy[k]));
      sm += e;
      mx = e > mx ? e : mx;
    }
    B->slip_mean = sm / B->nb;
    B->slip_max = mx;
  }
}

int or_step(or_sim *s, int64_t nsteps) {
  if (s->halted) return -5;
  for (int64_t t = 0; t < nsteps; t++) {
    for (int b = 0; b < s->nbody; b++) body_pre(s, &s->body[b], s->step);
    for (int b = 0; b < s->nbody; b++)
      if (!supports_inside(s, &s->body[b])) {
        s->halted = 1;
        return -5;
      }
    collide_all(s);
    stream_all(s);
    zou_he_walls(s);
    if (s->nbody > 0) {
      int scheme = s->body[0].d.scheme;
      if (scheme == OR_DF) ibm_df(s);
      else if (scheme == OR_MDF && s->body[0].d.mdf_coupled) ibm_mdf_coupled(s);
      else if (scheme == OR_MDF) ibm_mdf(s);
      else ibm_dfc(s);
      body_forces(s);
      body_slip(s);
      for (int b = 0; b < s->nbody; b++) body_post(s, &s->body[b]);
    }
    s->step++;
  }
  return 0;
}

/* ------------------------------------------------------------------ */
void or_get_populations(const or_sim *s, double *f) { memcpy(f, s->f, sizeof(double) * 9 * s->n); }
void or_set_populations(or_sim *s, const double *f) { memcpy(s->f, f, sizeof(double) * 9 * s->n); }
void or_get_force(const or_sim *s, double *fx, double *fy) {
  memcpy(fx, s->Fx, sizeof(double) * s->n);
  memcpy(fy, s->Fy, sizeof(double) * s->n);
}

/* Density and velocity of the current state, Eq. (4), with the IB force
 * still to be applied by the next collision plus the uniform fluid force. */
void or_fields(const or_sim *s, double *rho, double *ux, double *uy) {
  int n = s->n;
  for (int p = 0; p < n; p++) {
    double fin[9];
    for (int i = 0; i < 9; i++) fin[i] = s->f[(size_t)i * n + p];
    moments(fin, s->Fx[p] + s->c.fluid_force[0], s->Fy[p] + s->c.fluid_force[1], &rho[p], &ux[p],
            &uy[p]);
  }
}

/* Boundary-fidelity diagnostics (Sec. 2.8) and the marker profiles of
 * Sec. 4.2, on the current Eulerian field u = (sum_i f_i e_i + F/2)/rho.
 * Readings: the field is sampled at the markers by bilinear interpolation
 * (the hat kernel, Eq. 9), a probe distinct from the scheme's own kernel;
 * velocities are taken relative to the body's rigid motion U_b(x) = v +
 * Omega x (x - X_c) with the velocities reported for the body after the
 * step (zero for a fixed body); n_k = (X_k - X_c)/R.
 *   sum[0..1] slip mean / max: |u(X_k) - U_b(X_k)| / u_ref
 *   sum[2]    leakage flux sum_k rho(X_k) (u - U_b).n_k ds / (u_ref pi D)
 *   sum[3..5] internal residual: mean / max of |u - U_b| / u_ref over the
 *             nodes with |x - X_c| < R - kappa, and their count
 *   sum[6]    mean pressure deviation (rho(X_k) - rho0) c_s^2
 *   sum[7]    mean marker force magnitude |F_k| (F_L of DF/MDF, F_s of DFC)
 *   pm[6k..]  slip_k, dp_k, |F_k|, rho(X_k), normal and tangential
 *             relative velocity / u_ref */
int or_diagnostics(const or_sim *s, int b, int kappa, double u_ref, double *sum, double *pm) {
  if (b < 0 || b >= s->nbody || kappa < 0 || !(u_ref > 0)) return -1;
  const or_body *B = &s->body[b];
  const int n = s->n, nx = s->c.nx, ny = s->c.ny;
  double *rho = malloc(sizeof(double) * n), *ux = malloc(sizeof(double) * n),
         *uy = malloc(sizeof(double) * n);
  or_fields(s, rho, ux, uy);
  const double xc = B->xc, yc = B->yc, R = B->radius;
  const double vx = B->d.motion == OR_FREE ? B->vx : B->vhx;
  const double vy = B->d.motion == OR_FREE ? B->vy : B->vhy;
  const double om = B->d.motion == OR_FREE ? B->om : B->omh;
  const double cs2 = 1.0 / 3.0;
  double slip_sum = 0, slip_max = 0, flux = 0, dp_sum = 0, f_sum = 0;
  for (int k = 0; k < B->nb; k++) {
    const double X = B->X[k], Y = B->Y[k];
    const double rk = interp(s, OR_HAT, rho, X, Y);
    const double dx = interp(s, OR_HAT, ux, X, Y) - (vx - om * (Y - yc));
    const double dy = interp(s, OR_HAT, uy, X, Y) - (vy + om * (X - xc));
    const double nxk = (X - xc) / R, nyk = (Y - yc) / R;
    const double slip = sqrt(dx * dx + dy * dy) / u_ref;
    const double dp = (rk - s->c.rho0) * cs2;
    const double fm = sqrt(B->Fx[k] * B->Fx[k] + B->Fy[k] * B->Fy[k]);
    slip_sum += slip;
    slip_max = slip > slip_max ? slip : slip_max;
    flux += rk * (dx * nxk + dy * nyk) * B->ds;
    dp_sum += dp;
    f_sum += fm;
    if (pm) {
      double *o = pm + 6 * k;
      o[0] = slip;
      o[1] = dp;
      o[2] = fm;
      o[3] = rk;
      o[4] = (dx * nxk + dy * nyk) / u_ref;
      o[5] = (-dx * nyk + dy * nxk) / u_ref;
    }
  }
  double in_sum = 0, in_max = 0;
  long in_n = 0;
  const double Ri = R - kappa;
  for (int y = 0; y < ny && Ri > 0; y++)
    for (int x = 0; x < nx; x++) {
      const double rx = x - xc, ry = y - yc;
      if (rx * rx + ry * ry >= Ri * Ri) continue;
      const int p = y * nx + x;
      const double dx = ux[p] - (vx - om * ry), dy = uy[p] - (vy + om * rx);
      const double m = sqrt(dx * dx + dy * dy) / u_ref;
      in_sum += m;
      in_max = m > in_max ? m : in_max;
      in_n++;
    }
  sum[0] = slip_sum / B->nb;
  sum[1] = slip_max;
  sum[2] = flux / (u_ref * M_PI * B->d.diameter);
  sum[3] = in_n ? in_sum / in_n : 0.0;
  sum[4] = in_max;
  sum[5] = (double)in_n;
  sum[6] = dp_sum / B->nb;
  sum[7] = f_sum / B->nb;
  free(rho); free(ux); free(uy);
  return 0;
}

int or_body_state(const or_sim *s, int b, double *out) {
  if (b < 0 || b >= s->nbody) return -1;
  const or_body *B = &s->body[b];
  memset(out, 0, sizeof(double) * 16);
  out[0] = (double)s->step;
  out[1] = B->fhx;
  out[2] = B->fhy;
  out[3] = B->torque;
  out[4] = B->xc;
  out[5] = B->yc;
  out[6] = B->d.motion == OR_FREE ? B->vx : B->vhx;
  out[7] = B->d.motion == OR_FREE ? B->vy : B->vhy;
  out[8] = B->d.motion == OR_FREE ? B->om : B->omh;
  out[9] = B->slip_mean;
  out[10] = B->slip_max;
  out[11] = B->mdf_res;
  out[12] = B->mdf_iters_done;
  out[13] = B->omega_mdf;
  return 0;
}

int or_markers(const or_sim *s, int b, double *out) {
  if (b < 0 || b >= s->nbody) return -1;
  const or_body *B = &s->body[b];
  for (int k = 0; k < B->nb; k++) {
    double *o = out + 8 * k;
    o[0] = B->X[k];
    o[1] = B->Y[k];
    o[2] = B->Udx[k];
    o[3] = B->Udy[k];
    o[4] = B->Fx[k];
    o[5] = B->Fy[k];
    o[6] = B->lambda[k];
    o[7] = B->ds;
  }
  return B->nb;
}
