// Immersed-boundary pass for gfx950: one workgroup per body.
//
// Per step and body the workgroup
//   1. advances the body kinematics to t+1 (fixed, prescribed sine, or the
//      half-kick and drift of the Velocity-Verlet update, Eq. 23 / A3);
//   2. places the markers and their 1D delta weights (Eq. 6, 9, 10);
//   3. builds the support set of the body: per lattice row the union of the
//      marker stencils on the left and right arc, counted and prefix-summed
//      into a compact node list (rows x at most two x-intervals);
//   4. runs the enforcement scheme on that node list:
//        DF  (Eq. 11) / MDF (Eq. 12-14): interpolate rho and u* to the
//            markers, N Richardson passes with spreading back into the node
//            list, then spread F_total into the Eulerian force field;
//        DFC (Eq. 15-20): correction scale lambda_k (Eq. 17, cached for fixed
//            bodies), interpolate the nine populations, bounce-back target,
//            correction, spread the correction into the populations;
//   5. reduces force, torque, slip and MDF residual in FP64 with a fixed
//      order (wave shuffles, then LDS), and finishes the body update.
// Spreading is a gather: each support node sums over the markers of an
// angular window around it, in marker order, so results are reproducible
// run to run.  An atomic-scatter variant is kept for comparison.
// The node and marker arrays live in LDS when they fit, else in a global
// workspace of the body (the same code reaches both through flat pointers).
#include "ib_lbm_internal.h"

namespace iblbm {

__constant__ int c_exi[9] = {0, 1, 0, -1, 0, 1, -1, -1, 1};
__constant__ int c_eyi[9] = {0, 0, 1, 0, -1, 1, 1, -1, -1};
__constant__ int c_oppi[9] = {0, 3, 4, 1, 2, 7, 8, 5, 6};
__constant__ double c_w[9] = {4.0 / 9.0,  1.0 / 9.0,  1.0 / 9.0,  1.0 / 9.0, 1.0 / 9.0,
                              1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0};

// Regularized delta kernels: hat (Eq. 9) and Peskin 4-point (Eq. 10).
__device__ __forceinline__ double delta1(int kernel, double r) {
  const double a = fabs(r);
  if (kernel == kHat) return a < 1.0 ? 1.0 - a : 0.0;
  if (a <= 1.0) return 0.125 * (3.0 - 2.0 * a + sqrt(1.0 + 4.0 * a - 4.0 * a * a));
  if (a <= 2.0) return 0.125 * (5.0 - 2.0 * a - sqrt(-7.0 + 12.0 * a - 4.0 * a * a));
  return 0.0;
}

// ---- fixed-order block reductions (wave64 shuffles, then LDS) ----
__device__ __forceinline__ double wave_sum(double v) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o, 64);
  return v;
}
__device__ __forceinline__ double wave_max(double v) {
  for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_down(v, o, 64));
  return v;
}
// Reduces four values at once: three sums and one max; result valid in all threads.
__device__ void block_reduce4(double &a, double &b, double &c, double &m, double *red) {
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6, nw = (blockDim.x + 63) >> 6;
  a = wave_sum(a); b = wave_sum(b); c = wave_sum(c); m = wave_max(m);
  __syncthreads();
  if (lane == 0) { red[4 * wv] = a; red[4 * wv + 1] = b; red[4 * wv + 2] = c; red[4 * wv + 3] = m; }
  __syncthreads();
  double sa = 0, sb = 0, sc = 0, sm = -1e300;
  for (int w = 0; w < nw; w++) {
    sa += red[4 * w]; sb += red[4 * w + 1]; sc += red[4 * w + 2]; sm = fmax(sm, red[4 * w + 3]);
  }
  a = sa; b = sb; c = sc; m = sm;
  __syncthreads();
}

// Exclusive prefix sum of cnt[0..n) into off[0..n], off[n] = total.  Serial
// per wave chunk, then across waves; n is at most a few thousand.
__device__ void block_scan(const int *cnt, int *off, int n, int *sh) {
  const int nth = blockDim.x;
  const int per = (n + nth - 1) / nth;
  const int b0 = min(n, threadIdx.x * per), b1 = min(n, b0 + per);
  int s = 0;
  for (int i = b0; i < b1; i++) s += cnt[i];
  // inclusive scan of per-thread sums through LDS (Hillis-Steele)
  sh[threadIdx.x] = s;
  __syncthreads();
  for (int o = 1; o < nth; o <<= 1) {
    const int v = threadIdx.x >= o ? sh[threadIdx.x - o] : 0;
    __syncthreads();
    sh[threadIdx.x] += v;
    __syncthreads();
  }
  int run = sh[threadIdx.x] - s;
  for (int i = b0; i < b1; i++) { off[i] = run; run += cnt[i]; }
  if (threadIdx.x == nth - 1) off[n] = sh[nth - 1];
  __syncthreads();
}

struct WsLayout {
  // doubles
  double *X, *Y, *Udx, *Udy, *wx, *wy, *Fx, *Fy, *Ftx, *Fty, *rhoX, *lam, *dlt;
  double *nrho, *nux, *nuy, *nW, *accx, *accy;
  // ints
  int *ix0, *iy0, *nidx, *rmin, *rmax, *lmin, *lmax, *ra1, *rl1, *ra2, *cnt, *off, *nxy, *nkc;
};

__device__ __forceinline__ WsLayout carve(double *base, int nb, int ns, int mr, int mn) {
  WsLayout L;
  double *p = base;
  L.X = p; p += nb; L.Y = p; p += nb; L.Udx = p; p += nb; L.Udy = p; p += nb;
  L.wx = p; p += nb * ns; L.wy = p; p += nb * ns;
  L.Fx = p; p += nb; L.Fy = p; p += nb; L.Ftx = p; p += nb; L.Fty = p; p += nb;
  L.rhoX = p; p += nb; L.lam = p; p += nb; L.dlt = p; p += 9 * nb;
  L.nrho = p; p += mn; L.nux = p; p += mn; L.nuy = p; p += mn; L.nW = p; p += mn;
  L.accx = p; p += mn; L.accy = p; p += mn;
  int *q = (int *)p;
  L.ix0 = q; q += nb; L.iy0 = q; q += nb; L.nidx = q; q += nb * ns * ns;
  L.lmin = q; q += mr; L.lmax = q; q += mr; L.rmin = q; q += mr; L.rmax = q; q += mr;
  L.ra1 = q; q += mr; L.rl1 = q; q += mr; L.ra2 = q; q += mr; L.cnt = q; q += mr;
  L.off = q; q += mr + 1; L.nxy = q; q += mn; L.nkc = q; q += mn;
  return L;
}

// Gather over the angular marker window of node (x,y): sum_k v_k D_h for two
// marker arrays at once.
__device__ __forceinline__ void gather2(const WsLayout &L, int nb, int ns, int win, int kc, int x,
                                        int y, const double *va, const double *vb, double &oa,
                                        double &ob) {
  double a = 0.0, b = 0.0;
  const bool all = 2 * win + 1 >= nb;
  const int k0 = all ? 0 : kc - win, k1 = all ? nb - 1 : kc + win;
  for (int kk = k0; kk <= k1; kk++) {
    int k = kk;
    if (k < 0) k += nb; else if (k >= nb) k -= nb;
    const int jx = x - L.ix0[k], jy = y - L.iy0[k];
    if ((unsigned)jx < (unsigned)ns && (unsigned)jy < (unsigned)ns) {
      const double w = L.wx[k * ns + jx] * L.wy[k * ns + jy];
      a += va[k] * w;
      b += vb[k] * w;
    }
  }
  oa = a;
  ob = b;
}

// Interpolation of a node array to marker k (Eq. 7).
__device__ __forceinline__ double interp1(const WsLayout &L, int ns, int k, const double *nv) {
  double acc = 0.0;
  for (int jy = 0; jy < ns; jy++) {
    double row = 0.0;
    for (int jx = 0; jx < ns; jx++) row += nv[L.nidx[(k * ns + jy) * ns + jx]] * L.wx[k * ns + jx];
    acc += row * L.wy[k * ns + jy];
  }
  return acc;
}

template <typename T>
__device__ void body_step(const CaseDesc &c, const BodyDesc &B, int64_t step, double *dyn,
                          int lds_doubles, int spread_mode, double *red, int *ish, double *bsh) {
  const int tid = threadIdx.x, nth = blockDim.x;
  BodyState *bs = B.state;
  const int nb = B.nb, ns = B.ns, s = ns / 2;
  const bool shift = sizeof(T) == 4;
  const double rho0 = c.rho0;
  const int nx = c.nx, ny = c.ny;
  const int64_t plane = c.plane;

  // ---- 1. kinematics for t_{n+1}
  if (tid == 0) {
    double xc = bs->xc, yc = bs->yc, vhx = 0, vhy = 0, omh = 0;
    if (B.motion == kPrescribedSin) {
      const double t1 = (double)(step + 1);
      const double ph = 2.0 * M_PI * B.freq * t1 + B.phase;
      const double sn = sin(ph), cn = cos(ph);
      xc = B.xc0 + B.amp[0] * sn;
      yc = B.yc0 + B.amp[1] * sn;
      vhx = B.amp[0] * 2.0 * M_PI * B.freq * cn;
      vhy = B.amp[1] * 2.0 * M_PI * B.freq * cn;
      bs->vx = vhx;
      bs->vy = vhy;
    } else if (B.motion == kFree) {
      // Eq. (23) first half-kick and drift with the lagged internal-mass
      // force of Eq. (A3) and the net gravity of Eq. (22).
      const double fgx = (B.ms - B.mf) * c.grav_x;
      const double fgy = (B.ms - B.mf) * c.grav_y;
      const double dimx = B.internal_mass == kImFeng ? B.mf * (bs->vx - bs->vpx) : 0.0;
      const double dimy = B.internal_mass == kImFeng ? B.mf * (bs->vy - bs->vpy) : 0.0;
      bs->vpx = bs->vx;
      bs->vpy = bs->vy;
      bs->dimx = dimx;
      bs->dimy = dimy;
      vhx = bs->vx + (bs->fhx + fgx + dimx) / (2.0 * B.ms);
      vhy = bs->vy + (bs->fhy + fgy + dimy) / (2.0 * B.ms);
      xc += vhx;
      yc += vhy;
      omh = bs->om + bs->torque / (2.0 * B.Is);
    }
    bs->xc = xc; bs->yc = yc;
    bs->vhx = vhx; bs->vhy = vhy; bs->omh = omh;
    bsh[0] = xc; bsh[1] = yc; bsh[2] = vhx; bsh[3] = vhy; bsh[4] = omh;
    ish[0] = 0;  // error flags
  }
  const bool in_lds = lds_doubles >= B.ws_doubles;
  double *base = in_lds ? dyn : B.ws;
  const WsLayout L = carve(base, nb, ns, B.max_rows, B.max_nodes);
  // row tables start empty
  for (int r = tid; r < B.max_rows; r += nth) {
    L.lmin[r] = 1 << 30; L.lmax[r] = -1; L.rmin[r] = 1 << 30; L.rmax[r] = -1;
  }
  __syncthreads();
  const double xc = bsh[0], yc = bsh[1], vhx = bsh[2], vhy = bsh[3], omh = bsh[4];
  const int ylo = (int)floor(yc - B.radius) - ns;

  // ---- 2. markers, weights, row intervals
  for (int k = tid; k < nb; k += nth) {
    const double X = xc + B.radius * B.cos_t[k];
    const double Y = yc + B.radius * B.sin_t[k];
    L.X[k] = X;
    L.Y[k] = Y;
    L.Udx[k] = vhx - omh * (Y - yc);
    L.Udy[k] = vhy + omh * (X - xc);
    const int ix0 = (int)floor(X) - (s - 1), iy0 = (int)floor(Y) - (s - 1);
    L.ix0[k] = ix0;
    L.iy0[k] = iy0;
    if (ix0 < 0 || iy0 < 0 || ix0 + ns - 1 > nx - 1 || iy0 + ns - 1 > ny - 1) atomicOr(&ish[0], kFlagRange);
    for (int j = 0; j < ns; j++) {
      L.wx[k * ns + j] = delta1(B.kernel, (double)(ix0 + j) - X);
      L.wy[k * ns + j] = delta1(B.kernel, (double)(iy0 + j) - Y);
    }
    const bool left = X < xc;
    for (int j = 0; j < ns; j++) {
      const int r = iy0 + j - ylo;
      if (r < 0 || r >= B.max_rows) { atomicOr(&ish[0], kFlagCapacity); continue; }
      if (left) { atomicMin(&L.lmin[r], ix0); atomicMax(&L.lmax[r], ix0 + ns - 1); }
      else { atomicMin(&L.rmin[r], ix0); atomicMax(&L.rmax[r], ix0 + ns - 1); }
    }
  }
  __syncthreads();
  if (ish[0]) {
    if (tid == 0) { bs->flags |= ish[0]; bs->box_valid = 0; }
    return;
  }
  // ---- 3. row intervals -> compact node list
  for (int r = tid; r < B.max_rows; r += nth) {
    const bool lv = L.lmax[r] >= 0, rv = L.rmax[r] >= 0;
    int a1 = 0, l1 = 0, a2 = 0, l2 = 0;
    if (lv && rv && L.rmin[r] <= L.lmax[r] + 1) {
      a1 = min(L.lmin[r], L.rmin[r]);
      l1 = max(L.lmax[r], L.rmax[r]) - a1 + 1;
    } else {
      if (lv) { a1 = L.lmin[r]; l1 = L.lmax[r] - a1 + 1; }
      if (rv) {
        if (lv) { a2 = L.rmin[r]; l2 = L.rmax[r] - a2 + 1; }
        else { a1 = L.rmin[r]; l1 = L.rmax[r] - a1 + 1; }
      }
    }
    L.ra1[r] = a1; L.rl1[r] = l1; L.ra2[r] = a2; L.cnt[r] = l1 + l2;
  }
  __syncthreads();
  block_scan(L.cnt, L.off, B.max_rows, ish + 16);
  const int S = L.off[B.max_rows];
  if (S > B.max_nodes) {
    if (tid == 0) { bs->flags |= kFlagCapacity; bs->box_valid = 0; }
    return;
  }
  const T *fpop = (const T *)c.f[c.state->cur ^ 1];
  T *fpop_w = (T *)c.f[c.state->cur ^ 1];
  // nodes: coordinates, angular window centre, moments
  const double inv_dth = 1.0 / B.dtheta;
  for (int j = tid; j < S; j += nth) {
    int lo = 0, hi = B.max_rows - 1;
    while (lo < hi) {
      const int mid = (lo + hi + 1) >> 1;
      if (L.off[mid] <= j) lo = mid; else hi = mid - 1;
    }
    const int r = lo, loc = j - L.off[r];
    const int x = loc < L.rl1[r] ? L.ra1[r] + loc : L.ra2[r] + (loc - L.rl1[r]);
    const int y = ylo + r;
    L.nxy[j] = x | (y << 16);
    const float th = atan2f((float)(y - yc), (float)(x - xc));
    int kc = (int)rintf(th * (float)inv_dth);
    kc %= nb;
    if (kc < 0) kc += nb;
    L.nkc[j] = kc;
    if (B.scheme != kDFC) {
      const int64_t p = (int64_t)y * nx + x;
      double sm = 0, jx = 0, jy = 0;
      for (int i = 0; i < 9; i++) {
        const double v = (double)fpop[i * plane + p] + (shift ? c_w[i] * rho0 : 0.0);
        sm += v;
        jx += v * c_exi[i];
        jy += v * c_eyi[i];
      }
      L.nrho[j] = sm;
      L.nux[j] = jx / sm;
      L.nuy[j] = jy / sm;
    }
    L.accx[j] = 0.0;
    L.accy[j] = 0.0;
  }
  // marker -> node indices
  for (int k = tid; k < nb; k += nth) {
    for (int jy = 0; jy < ns; jy++) {
      const int r = L.iy0[k] + jy - ylo;
      for (int jx = 0; jx < ns; jx++) {
        const int x = L.ix0[k] + jx;
        const int loc = (x >= L.ra1[r] && x < L.ra1[r] + L.rl1[r]) ? x - L.ra1[r]
                                                                  : L.rl1[r] + x - L.ra2[r];
        L.nidx[(k * ns + jy) * ns + jx] = L.off[r] + loc;
      }
    }
  }
  __syncthreads();

  const double ds = B.ds;
  double fsum_x = 0, fsum_y = 0, tq = 0, resmax = 0;
  if (B.scheme != kDFC) {
    // ---- 4a. DF (one pass, omega 1) / MDF (N passes, omega_MDF)
    const int N = B.scheme == kDF ? 1 : B.mdf_iters;
    const double om = B.scheme == kDF ? 1.0 : B.omega_mdf;
    for (int k = tid; k < nb; k += nth) {
      L.rhoX[k] = interp1(L, ns, k, L.nrho);
      L.Ftx[k] = 0.0;
      L.Fty[k] = 0.0;
    }
    for (int n = 1; n <= N; n++) {
      __syncthreads();
      for (int k = tid; k < nb; k += nth) {
        const double Ux = interp1(L, ns, k, L.nux), Uy = interp1(L, ns, k, L.nuy);
        const double ex = L.Udx[k] - Ux, ey = L.Udy[k] - Uy;
        const double Fx = 2.0 * L.rhoX[k] * ex, Fy = 2.0 * L.rhoX[k] * ey;
        L.Fx[k] = om * Fx;
        L.Fy[k] = om * Fy;
        L.Ftx[k] += om * Fx;
        L.Fty[k] += om * Fy;
        if (n == N) resmax = fmax(resmax, sqrt(ex * ex + ey * ey));
      }
      __syncthreads();
      if (spread_mode == 0) {
        for (int j = tid; j < S; j += nth) {
          const int x = L.nxy[j] & 0xffff, y = L.nxy[j] >> 16;
          double sx, sy;
          gather2(L, nb, ns, B.window, L.nkc[j], x, y, L.Fx, L.Fy, sx, sy);
          const double h = 1.0 / (2.0 * L.nrho[j]);
          L.nux[j] += sx * ds * h;
          L.nuy[j] += sy * ds * h;
        }
      } else {
        for (int k = tid; k < nb; k += nth)
          for (int q = 0; q < ns * ns; q++) {
            const double w = L.wx[k * ns + (q % ns)] * L.wy[k * ns + (q / ns)];
            atomicAdd(&L.accx[L.nidx[k * ns * ns + q]], L.Fx[k] * w);
            atomicAdd(&L.accy[L.nidx[k * ns * ns + q]], L.Fy[k] * w);
          }
        __syncthreads();
        for (int j = tid; j < S; j += nth) {
          const double h = 1.0 / (2.0 * L.nrho[j]);
          L.nux[j] += L.accx[j] * ds * h;
          L.nuy[j] += L.accy[j] * ds * h;
          L.accx[j] = 0.0;
          L.accy[j] = 0.0;
        }
      }
    }
    __syncthreads();
    // Eulerian force f(x) = sum_k F_total D_h ds (Eq. 8) into the force field
    T *frc = (T *)c.force;
    if (spread_mode == 0) {
      for (int j = tid; j < S; j += nth) {
        const int x = L.nxy[j] & 0xffff, y = L.nxy[j] >> 16;
        double fx, fy;
        gather2(L, nb, ns, B.window, L.nkc[j], x, y, L.Ftx, L.Fty, fx, fy);
        const int64_t p = (int64_t)y * nx + x;
        frc[p] = (T)(fx * ds);
        frc[plane + p] = (T)(fy * ds);
      }
    } else {
      for (int k = tid; k < nb; k += nth)
        for (int q = 0; q < ns * ns; q++) {
          const double w = L.wx[k * ns + (q % ns)] * L.wy[k * ns + (q / ns)];
          atomicAdd(&L.accx[L.nidx[k * ns * ns + q]], L.Ftx[k] * w);
          atomicAdd(&L.accy[L.nidx[k * ns * ns + q]], L.Fty[k] * w);
        }
      __syncthreads();
      for (int j = tid; j < S; j += nth) {
        const int x = L.nxy[j] & 0xffff, y = L.nxy[j] >> 16;
        const int64_t p = (int64_t)y * nx + x;
        frc[p] = (T)(L.accx[j] * ds);
        frc[plane + p] = (T)(L.accy[j] * ds);
        L.accx[j] = 0.0;
        L.accy[j] = 0.0;
      }
    }
    // force on the body: -sum_k F_total ds sum_x D_h (Newton's third law),
    // torque -sum_k r_k x F_total ds (Sec. 2.7)
    for (int k = tid; k < nb; k += nth) {
      double wsx = 0, wsy = 0;
      for (int j = 0; j < ns; j++) { wsx += L.wx[k * ns + j]; wsy += L.wy[k * ns + j]; }
      const double wsum = wsx * wsy;
      fsum_x -= L.Ftx[k] * ds * wsum;
      fsum_y -= L.Fty[k] * ds * wsum;
      tq -= ((L.X[k] - xc) * L.Fty[k] - (L.Y[k] - yc) * L.Ftx[k]) * ds;
    }
  } else {
    // ---- 4b. DFC
    if (!bs->lambda_valid) {
      for (int j = tid; j < S; j += nth) {
        const int x = L.nxy[j] & 0xffff, y = L.nxy[j] >> 16;
        double wt = 0.0;
        const bool all = 2 * B.window + 1 >= nb;
        const int kc = L.nkc[j];
        const int k0 = all ? 0 : kc - B.window, k1 = all ? nb - 1 : kc + B.window;
        for (int kk = k0; kk <= k1; kk++) {
          int k = kk;
          if (k < 0) k += nb; else if (k >= nb) k -= nb;
          const int jx = x - L.ix0[k], jy = y - L.iy0[k];
          if ((unsigned)jx < (unsigned)ns && (unsigned)jy < (unsigned)ns)
            wt += L.wx[k * ns + jx] * L.wy[k * ns + jy];
        }
        L.nW[j] = wt;
      }
      __syncthreads();
      for (int k = tid; k < nb; k += nth) {
        const double wsum = interp1(L, ns, k, L.nW);
        L.lam[k] = 1.0 / (2.0 * rho0 * ds * wsum);
        B.lambda_cache[k] = L.lam[k];
      }
    } else {
      for (int k = tid; k < nb; k += nth) L.lam[k] = B.lambda_cache[k];
    }
    __syncthreads();
    // Eq. (15)-(18), (20): interpolate the stored populations; the bounce-back
    // target minus f* only involves f*_opp - f*_i, the same in f and in g.
    for (int k = tid; k < nb; k += nth) {
      double gi[9];
      for (int i = 0; i < 9; i++) gi[i] = 0.0;
      for (int jy = 0; jy < ns; jy++) {
        const int y = L.iy0[k] + jy;
        for (int jx = 0; jx < ns; jx++) {
          const int x = L.ix0[k] + jx;
          const double w = L.wx[k * ns + jx] * L.wy[k * ns + jy];
          const int64_t p = (int64_t)y * nx + x;
          for (int i = 0; i < 9; i++) gi[i] += (double)fpop[i * plane + p] * w;
        }
      }
      const double lam = L.lam[k];
      double fsx = 0, fsy = 0;
      for (int i = 0; i < 9; i++) {
        const double eud = c_exi[i] * L.Udx[k] + c_eyi[i] * L.Udy[k];
        const double d = lam * (gi[c_oppi[i]] - gi[i] + 6.0 * c_w[i] * rho0 * eud);
        L.dlt[9 * k + i] = d;
        fsx += c_exi[i] * d;
        fsy += c_eyi[i] * d;
      }
      L.Ftx[k] = -ds * fsx;
      L.Fty[k] = -ds * fsy;
    }
    __syncthreads();
    // Eq. (19): f_i(x) <- f*_i(x) + sum_k delta f_i D_h ds, then the
    // post-correction velocity for the slip diagnostic.
    if (spread_mode == 0) {
      for (int j = tid; j < S; j += nth) {
        const int x = L.nxy[j] & 0xffff, y = L.nxy[j] >> 16;
        const int kc = L.nkc[j];
        double corr[9];
        for (int i = 0; i < 9; i++) corr[i] = 0.0;
        const bool all = 2 * B.window + 1 >= nb;
        const int k0 = all ? 0 : kc - B.window, k1 = all ? nb - 1 : kc + B.window;
        for (int kk = k0; kk <= k1; kk++) {
          int k = kk;
          if (k < 0) k += nb; else if (k >= nb) k -= nb;
          const int jx = x - L.ix0[k], jy = y - L.iy0[k];
          if ((unsigned)jx < (unsigned)ns && (unsigned)jy < (unsigned)ns) {
            const double w = L.wx[k * ns + jx] * L.wy[k * ns + jy];
            for (int i = 0; i < 9; i++) corr[i] += L.dlt[9 * k + i] * w;
          }
        }
        const int64_t p = (int64_t)y * nx + x;
        double sm = 0, jxs = 0, jys = 0;
        for (int i = 0; i < 9; i++) {
          const T nv = (T)((double)fpop[i * plane + p] + corr[i] * ds);
          fpop_w[i * plane + p] = nv;
          const double v = (double)nv + (shift ? c_w[i] * rho0 : 0.0);
          sm += v;
          jxs += v * c_exi[i];
          jys += v * c_eyi[i];
        }
        L.nux[j] = jxs / sm;
        L.nuy[j] = jys / sm;
      }
    } else {
      // atomic scatter of the nine corrections, two components at a time
      for (int i0 = 0; i0 < 9; i0 += 2) {
        for (int k = tid; k < nb; k += nth)
          for (int q = 0; q < ns * ns; q++) {
            const double w = L.wx[k * ns + (q % ns)] * L.wy[k * ns + (q / ns)];
            atomicAdd(&L.accx[L.nidx[k * ns * ns + q]], L.dlt[9 * k + i0] * w);
            if (i0 + 1 < 9) atomicAdd(&L.accy[L.nidx[k * ns * ns + q]], L.dlt[9 * k + i0 + 1] * w);
          }
        __syncthreads();
        for (int j = tid; j < S; j += nth) {
          const int x = L.nxy[j] & 0xffff, y = L.nxy[j] >> 16;
          const int64_t p = (int64_t)y * nx + x;
          fpop_w[i0 * plane + p] = (T)((double)fpop[i0 * plane + p] + L.accx[j] * ds);
          if (i0 + 1 < 9)
            fpop_w[(i0 + 1) * plane + p] = (T)((double)fpop[(i0 + 1) * plane + p] + L.accy[j] * ds);
          L.accx[j] = 0.0;
          L.accy[j] = 0.0;
        }
        __syncthreads();
      }
      for (int j = tid; j < S; j += nth) {
        const int x = L.nxy[j] & 0xffff, y = L.nxy[j] >> 16;
        const int64_t p = (int64_t)y * nx + x;
        double sm = 0, jxs = 0, jys = 0;
        for (int i = 0; i < 9; i++) {
          const double v = (double)fpop[i * plane + p] + (shift ? c_w[i] * rho0 : 0.0);
          sm += v;
          jxs += v * c_exi[i];
          jys += v * c_eyi[i];
        }
        L.nux[j] = jxs / sm;
        L.nuy[j] = jys / sm;
      }
    }
    for (int k = tid; k < nb; k += nth) {
      fsum_x += L.Ftx[k];
      fsum_y += L.Fty[k];
      tq += (L.X[k] - xc) * L.Fty[k] - (L.Y[k] - yc) * L.Ftx[k];
    }
  }
  __syncthreads();
  // ---- 5. slip with the post-IB velocity, reductions, body update
  double slip_sum = 0, slip_max = 0;
  for (int k = tid; k < nb; k += nth) {
    const double Ux = interp1(L, ns, k, L.nux), Uy = interp1(L, ns, k, L.nuy);
    const double e = sqrt((Ux - L.Udx[k]) * (Ux - L.Udx[k]) + (Uy - L.Udy[k]) * (Uy - L.Udy[k]));
    slip_sum += e;
    slip_max = fmax(slip_max, e);
    double *mo = B.markers_out + 8 * k;
    mo[0] = L.X[k]; mo[1] = L.Y[k]; mo[2] = L.Udx[k]; mo[3] = L.Udy[k];
    mo[4] = L.Ftx[k]; mo[5] = L.Fty[k]; mo[6] = B.scheme == kDFC ? L.lam[k] : 0.0; mo[7] = ds;
  }
  double a = fsum_x, b = fsum_y, cq = tq, m = fmax(resmax, 0.0);
  block_reduce4(a, b, cq, m, red);
  double s1 = slip_sum, s2 = 0, s3 = 0, s4 = slip_max;
  block_reduce4(s1, s2, s3, s4, red);
  if (tid == 0) {
    int flags = 0;
    if (!isfinite(a) || !isfinite(b) || !isfinite(cq) || !isfinite(s1)) flags |= kFlagNonfinite;
    bs->fhx = a;
    bs->fhy = b;
    bs->torque = cq;
    bs->slip_mean = s1 / nb;
    bs->slip_max = s4;
    bs->mdf_res = B.scheme == kMDF ? m : 0.0;
    bs->mdf_iters_done = B.scheme == kDFC ? 0 : (B.scheme == kDF ? 1 : B.mdf_iters);
    if (B.scheme == kDFC) {
      bs->box_valid = 0;
      if (B.motion == kFixed) bs->lambda_valid = 1;
    } else {
      bs->box[0] = max(0, (int)floor(xc - B.radius) - ns);
      bs->box[1] = max(0, (int)floor(yc - B.radius) - ns);
      bs->box[2] = min(nx - 1, (int)floor(xc + B.radius) + ns + 1);
      bs->box[3] = min(ny - 1, (int)floor(yc + B.radius) + ns + 1);
      bs->box_valid = 1;
    }
    if (B.motion == kFree) {
      const double fgx = (B.ms - B.mf) * c.grav_x, fgy = (B.ms - B.mf) * c.grav_y;
      bs->vx = vhx + (a + fgx + bs->dimx) / (2.0 * B.ms);
      bs->vy = vhy + (b + fgy + bs->dimy) / (2.0 * B.ms);
      bs->om = omh + cq / (2.0 * B.Is);
      if (!isfinite(bs->vx) || !isfinite(bs->vy) || fabs(bs->vx) > 0.5 || fabs(bs->vy) > 0.5)
        flags |= kFlagNonfinite;
    } else if (B.motion == kFixed) {
      bs->vx = 0.0; bs->vy = 0.0; bs->om = 0.0;
    }
    bs->flags |= flags;
    const int64_t row = step % B.hist_cap;
    double *h = B.history + row * kHistCols;
    h[0] = (double)(step + 1); h[1] = a; h[2] = b; h[3] = cq;
    h[4] = xc; h[5] = yc; h[6] = bs->vx; h[7] = bs->vy; h[8] = B.motion == kFree ? bs->om : omh;
    h[9] = bs->slip_mean; h[10] = s4; h[11] = bs->mdf_res;
    h[12] = bs->mdf_iters_done; h[13] = bs->flags; h[14] = 0; h[15] = 0;
  }
}

template <typename T>
__global__ __launch_bounds__(kIbmThreads) void ibm_kernel(const CaseDesc *__restrict__ cases,
                                                          const IbmSlot *__restrict__ slots,
                                                          int lds_doubles, int spread_mode) {
  extern __shared__ double dyn[];
  __shared__ double red[4 * (kIbmThreads / 64)];
  __shared__ int ish[16 + kIbmThreads];
  __shared__ double bsh[16];
  const IbmSlot sl = slots[blockIdx.x];
  const CaseDesc &c = cases[sl.cas];
  CaseState *cs = c.state;
  const int64_t step = cs->step;
  const bool active = step < cs->target && !(cs->flags & kCaseHalted);
  if (!active) return;
  if (sl.body >= 0) {
    body_step<T>(c, c.bodies[sl.body], step, dyn, lds_doubles, spread_mode, red, ish, bsh);
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    __threadfence();
    const int prev = atomicAdd(&cs->done, 1);
    if (prev == sl.slots_in_case - 1) {
      __threadfence();
      // A body that failed this step (support outside the lattice, work
      // space too small, non-finite force) stops the case without completing
      // the step; bodies whose supports could meet within the next step stop
      // it after completing this one.
      int bflags = 0;
      for (int b = 0; b < c.nbodies; b++)
        bflags |= __hip_atomic_load(&c.bodies[b].state->flags, __ATOMIC_RELAXED,
                                    __HIP_MEMORY_SCOPE_AGENT);
      bool meet = false;
      for (int a = 0; a < c.nbodies && !bflags; a++)
        for (int b = a + 1; b < c.nbodies; b++) {
          const BodyDesc &A = c.bodies[a], &Bb = c.bodies[b];
          const double dx = __hip_atomic_load(&A.state->xc, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) -
                            __hip_atomic_load(&Bb.state->xc, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
          const double dy = __hip_atomic_load(&A.state->yc, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) -
                            __hip_atomic_load(&Bb.state->yc, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
          const double lim = A.radius + Bb.radius + A.ns + Bb.ns + 4.0;
          if (dx * dx + dy * dy <= lim * lim) {
            meet = true;
            A.state->flags |= kFlagOverlap;
          }
        }
      cs->done = 0;
      if (bflags) {
        cs->flags |= kCaseHalted;
      } else {
        cs->cur ^= 1;
        cs->step = step + 1;
        if (meet) cs->flags |= kCaseHalted;
      }
      __threadfence();
    }
  }
}

constexpr int kIbmDynLds = 128 * 1024;
int ibm_max_lds_bytes() { return kIbmDynLds; }

hipError_t launch_ibm(int precision, const CaseDesc *cases, const IbmSlot *slots, int nslots,
                      int lds_bytes, int spread_mode, hipStream_t stream) {
  if (nslots <= 0) return hipSuccess;
  static bool configured = false;
  if (!configured) {
    // allow the large dynamic LDS workspace (gfx950 has 160 KB per CU)
    (void)hipFuncSetAttribute((const void *)ibm_kernel<double>,
                              hipFuncAttributeMaxDynamicSharedMemorySize, kIbmDynLds);
    (void)hipFuncSetAttribute((const void *)ibm_kernel<float>,
                              hipFuncAttributeMaxDynamicSharedMemorySize, kIbmDynLds);
    configured = true;
  }
  const int lds_doubles = lds_bytes / 8;
  if (precision == kPrecFP64)
    hipLaunchKernelGGL(ibm_kernel<double>, dim3(nslots), dim3(kIbmThreads), lds_bytes, stream,
                       cases, slots, lds_doubles, spread_mode);
  else
    hipLaunchKernelGGL(ibm_kernel<float>, dim3(nslots), dim3(kIbmThreads), lds_bytes, stream,
                       cases, slots, lds_doubles, spread_mode);
  return hipGetLastError();
}

}  // namespace iblbm
