// Fused D2Q9 collide + stream for gfx950.
//
// One thread owns one node per row it visits: it reads the node's nine
// post-stream populations (coalesced: nine planes, x fastest), collides them
// with BGK + Guo forcing (Eq. 1-4), TRT (Sec. 2.2) or the central-moment
// operator (Eq. 5), and pushes the nine results to the neighbours of the
// other lattice ("two-lattice push"), applying the face closures on the fly.
// The kernel is HBM-bound: 9 reads + 9 writes per node, 144 B (FP64) or
// 72 B (FP32 shifted) of algorithmic traffic per node update.  Nothing here
// is a dense contraction, so there is no MFMA.
//
// The FP32 path stores and collides the shifted populations
// g_i = f_i - w_i rho0 with FP32 arithmetic; bounce-back and the velocity
// closure are linear in g because w_opp(i) = w_i.
#include "ib_lbm_internal.h"

namespace iblbm {

__constant__ int c_ex[9] = {0, 1, 0, -1, 0, 1, -1, -1, 1};
__constant__ int c_ey[9] = {0, 0, 1, 0, -1, 1, 1, -1, -1};

#define EXI(i) ((i) == 1 || (i) == 5 || (i) == 8 ? 1 : ((i) == 3 || (i) == 6 || (i) == 7 ? -1 : 0))
#define EYI(i) ((i) == 2 || (i) == 5 || (i) == 6 ? 1 : ((i) == 4 || (i) == 7 || (i) == 8 ? -1 : 0))
#define OPPI(i) ((i) == 0 ? 0 : ((i) <= 4 ? (((i) + 1) & 3) + 1 : (((i) - 3) & 3) + 5))

template <typename R>
__device__ __forceinline__ R wgt(int i) {
  return i == 0 ? R(4) / R(9) : (i <= 4 ? R(1) / R(9) : R(1) / R(36));
}

// ---------------------------------------------------------------- collision
// f holds the stored values (f, or g = f - w rho0 when SHIFT).  sum_f is
// sum_i f_i, so the equilibrium in either form is w_i (sum_f + rho P_i(u)).
// Everything is computed in place to keep the register footprint small.
template <typename R>
__device__ __forceinline__ R eq_term(int i, R sum, R rho, R ux, R uy, R uu) {
  const R eu = R(EXI(i)) * ux + R(EYI(i)) * uy;
  return wgt<R>(i) * (sum + rho * (R(3) * eu + R(4.5) * eu * eu - R(1.5) * uu));
}
template <typename R>
__device__ __forceinline__ R guo_term(int i, R ux, R uy, R Fx, R Fy, R uF) {
  const R eu = R(EXI(i)) * ux + R(EYI(i)) * uy;
  const R eF = R(EXI(i)) * Fx + R(EYI(i)) * Fy;
  return wgt<R>(i) * (R(3) * (eF - uF) + R(9) * eu * eF);
}

template <typename R, bool SHIFT, int COL>
__device__ __forceinline__ void collide(R (&f)[9], R Fx, R Fy, const CaseDesc &c) {
  const R sum = ((f[0] + f[1]) + (f[2] + f[3])) + ((f[4] + f[5]) + (f[6] + f[7])) + f[8];
  const R rho = SHIFT ? R(c.rho0) + sum : sum;
  const R jx = (f[1] - f[3]) + (f[5] - f[6]) + (f[8] - f[7]);
  const R jy = (f[2] - f[4]) + (f[5] + f[6]) - (f[7] + f[8]);
  const R inv_rho = R(1) / rho;
  const R ux = (jx + R(0.5) * Fx) * inv_rho;
  const R uy = (jy + R(0.5) * Fy) * inv_rho;

  if constexpr (COL == kBGK) {
    const R uu = ux * ux + uy * uy;
    const R uF = ux * Fx + uy * Fy;
    const R om = R(c.omega);
    const R pf = R(1) - R(0.5) * om;
#pragma unroll
    for (int i = 0; i < 9; i++)
      f[i] = f[i] - om * (f[i] - eq_term<R>(i, sum, rho, ux, uy, uu)) +
             pf * guo_term<R>(i, ux, uy, Fx, Fy, uF);
  } else if constexpr (COL == kTRT) {
    const R uu = ux * ux + uy * uy;
    const R uF = ux * Fx + uy * Fy;
    const R se = R(c.s_e), so = R(c.s_o);
    const R pe = R(1) - R(0.5) * se, po = R(1) - R(0.5) * so;
    f[0] = f[0] - se * (f[0] - eq_term<R>(0, sum, rho, ux, uy, uu)) +
           pe * guo_term<R>(0, ux, uy, Fx, Fy, uF);
#pragma unroll
    for (int i = 1; i <= 8; i++) {
      const int j = OPPI(i);
      if (j < i) continue;
      const R ei = eq_term<R>(i, sum, rho, ux, uy, uu), ej = eq_term<R>(j, sum, rho, ux, uy, uu);
      const R si = guo_term<R>(i, ux, uy, Fx, Fy, uF), sj = guo_term<R>(j, ux, uy, Fx, Fy, uF);
      const R fp = R(0.5) * (f[i] + f[j]), fm = R(0.5) * (f[i] - f[j]);
      const R even = -se * (fp - R(0.5) * (ei + ej)) + pe * R(0.5) * (si + sj);
      const R odd = -so * (fm - R(0.5) * (ei - ej)) + po * R(0.5) * (si - sj);
      f[i] = f[i] + even + odd;
      f[j] = f[j] + even - odd;
    }
  } else {
    // Central moments k_pq = sum_i f_i (e_x - u_x)^p (e_y - u_y)^q.  D2Q9 is
    // the tensor product of {-1,0,1} x {-1,0,1}, so the transform factorises
    // into a 3-point transform along x for each row e_y, then along y.  The
    // grid [ey+1][ex+1] of populations is row -1: 7 4 8, row 0: 3 0 1,
    // row +1: 6 2 5; all transforms run in place on these nine values.
    R a00 = f[7], a01 = f[4], a02 = f[8];
    R a10 = f[3], a11 = f[0], a12 = f[1];
    R a20 = f[6], a21 = f[2], a22 = f[5];
    const R ux2 = ux * ux, uy2 = uy * uy;
    // forward along x: (v-1, v0, v1) -> (k0, k1, k2)
#define IBL_FWD(u, u2, m, z, p)                                  \
    {                                                            \
      const R s0 = (m) + (z) + (p), s1 = (p) - (m), s2 = (p) + (m); \
      (m) = s0;                                                  \
      (z) = s1 - (u) * s0;                                       \
      (p) = s2 - R(2) * (u) * s1 + (u2) * s0;                    \
    }
    IBL_FWD(ux, ux2, a00, a01, a02);
    IBL_FWD(ux, ux2, a10, a11, a12);
    IBL_FWD(ux, ux2, a20, a21, a22);
    // forward along y for p = 0, 1, 2 (columns): k[p][q] lands in a[q][p]
    IBL_FWD(uy, uy2, a00, a10, a20);
    IBL_FWD(uy, uy2, a01, a11, a21);
    IBL_FWD(uy, uy2, a02, a12, a22);
#undef IBL_FWD
    // now a[q][p] = k_pq.  Relaxation, Eq. (5): Lambda =
    // diag(0,0,0,w,w,w,s_q,s_q,s_eps); equilibrium central moments
    // (rho,0,0,rho/3,rho/3,0,0,0,rho/9); forcing central moments
    // (0,Fx,Fy,0,0,0,Fy/3,Fx/3,0).  The shifted form subtracts the central
    // moments of rho0 w_i, which factorise as c_p(ux) c_q(uy) with
    // c = (1, -u, 1/3 + u^2).
    const R om = R(c.omega), sq = R(c.s_q), seps = R(c.s_eps);
    const R r0 = SHIFT ? R(c.rho0) : R(0);
    const R third = R(1) / R(3);
    const R E20 = sum * third - r0 * ux2;
    const R E02 = sum * third - r0 * uy2;
    const R E11 = -r0 * ux * uy;
    const R E21 = r0 * uy * (third + ux2);
    const R E12 = r0 * ux * (third + uy2);
    const R E22 = sum * (R(1) / R(9)) - r0 * (third * (ux2 + uy2) + ux2 * uy2);
    const R pq = (R(1) - R(0.5) * sq) * third;
    a01 += Fx;                                       // k10
    a10 += Fy;                                       // k01
    a02 = a02 - om * (a02 - E20);                    // k20
    a20 = a20 - om * (a20 - E02);                    // k02
    a11 = a11 - om * (a11 - E11);                    // k11
    a12 = a12 - sq * (a12 - E21) + pq * Fy;          // k21
    a21 = a21 - sq * (a21 - E12) + pq * Fx;          // k12
    a22 = a22 - seps * (a22 - E22);                  // k22
    // back: central -> raw moments, then the 3-point values at -1, 0, 1
#define IBL_BWD(u, u2, m, z, p)                                  \
    {                                                            \
      const R M0 = (m);                                          \
      const R M1 = (z) + (u) * M0;                               \
      const R M2 = (p) + R(2) * (u) * (z) + (u2) * M0;           \
      (z) = M0 - M2;                                             \
      (p) = R(0.5) * (M2 + M1);                                  \
      (m) = R(0.5) * (M2 - M1);                                  \
    }
    IBL_BWD(uy, uy2, a00, a10, a20);
    IBL_BWD(uy, uy2, a01, a11, a21);
    IBL_BWD(uy, uy2, a02, a12, a22);
    IBL_BWD(ux, ux2, a00, a01, a02);
    IBL_BWD(ux, ux2, a10, a11, a12);
    IBL_BWD(ux, ux2, a20, a21, a22);
#undef IBL_BWD
    f[7] = a00; f[4] = a01; f[8] = a02;
    f[3] = a10; f[0] = a11; f[1] = a12;
    f[6] = a20; f[2] = a21; f[5] = a22;
  }
}

// ------------------------------------------------------------ streaming
__device__ __forceinline__ bool is_vel(int b) { return b == kVelParabolic || b == kVelUniform; }

// Push population i of node (x,y) with value v, applying the face closures:
//   periodic faces wrap; a link leaving through a zero-gradient face is
//   dropped, and the populations entering a zero-gradient face are copies of
//   those one node inside (column 1 for W, nx-2 for E, row 1 for S, ny-2 for
//   N), written as duplicate stores of the pushes that land there (every
//   such push comes from a face node); a corner of two zero-gradient faces
//   takes its diagonal population from the diagonal inner node, which is
//   what copying the columns and then the rows gives.  A link leaving
//   through a wall returns as opp(i) at the node (half-way bounce-back);
//   through a velocity face it returns as opp(i) - 6 w_i rho0 (e_i . u_w),
//   u_w evaluated at the link mid-point.  A link leaving through a wall and
//   a velocity face is a wall link; among velocity faces the first of W, E,
//   S, N is used.  A link leaving through a Zou-He face is dropped (it is
//   neither a wall nor a velocity face here); zou_he_kernel rebuilds what
//   the wall node is missing.  GZG: zero-gradient faces other than the east
//   one are present (the general copy rules); otherwise only the east face
//   can be zero-gradient, the usual outflow, which keeps the common case's
//   code short.
template <typename T, bool GZG>
__device__ void push_one(const CaseDesc &c, T *dst, int x, int y, int i, T v) {
  const int nx = c.nx, ny = c.ny;
  const uint32_t plane = (uint32_t)c.plane;
  int xd = x + c_ex[i], yd = y + c_ey[i];
  bool cw = xd < 0, ce = xd >= nx, cs = yd < 0, cn = yd >= ny;
  if (cw && c.bc[kFaceW] == kPeriodic) { xd += nx; cw = false; }
  if (ce && c.bc[kFaceE] == kPeriodic) { xd -= nx; ce = false; }
  if (cs && c.bc[kFaceS] == kPeriodic) { yd += ny; cs = false; }
  if (cn && c.bc[kFaceN] == kPeriodic) { yd -= ny; cn = false; }
  int j = i, xs = xd, ys = yd;
  if (cw || ce || cs || cn) {
    if (GZG) {
      if ((cw && c.bc[kFaceW] == kZeroGradient) || (ce && c.bc[kFaceE] == kZeroGradient) ||
          (cs && c.bc[kFaceS] == kZeroGradient) || (cn && c.bc[kFaceN] == kZeroGradient))
        return;
    } else {
      if (ce && c.bc[kFaceE] == kZeroGradient) return;
    }
    j = OPPI(i);
    xs = x;
    ys = y;
    const bool wall = (cw && c.bc[kFaceW] == kBounceBack) || (ce && c.bc[kFaceE] == kBounceBack) ||
                      (cs && c.bc[kFaceS] == kBounceBack) || (cn && c.bc[kFaceN] == kBounceBack);
    if (!wall) {
      int vf = -1;
      if (cw && is_vel(c.bc[kFaceW])) vf = kFaceW;
      else if (ce && is_vel(c.bc[kFaceE])) vf = kFaceE;
      else if (cs && is_vel(c.bc[kFaceS])) vf = kFaceS;
      else if (cn && is_vel(c.bc[kFaceN])) vf = kFaceN;
      if (vf < 0) return;
      T uw;
      if (c.bc[vf] == kVelParabolic) {
        const T ym = T(y) + T(0.5) * T(c_ey[i]);
        uw = T(4) * T(c.u_bc) * (ym + T(0.5)) * (T(ny) - T(0.5) - ym) * T(c.inv_ny2);
      } else {
        uw = T(c.u_bc);
      }
      v = v - T(6) * wgt<T>(i) * T(c.rho0) * (T(c_ex[i]) * uw);
    }
  }
  if (!GZG) {
    dst[(uint32_t)j * plane + (uint32_t)ys * nx + xs] = v;
    if (c.bc[kFaceE] == kZeroGradient && xs == nx - 2 && (j == 3 || j == 6 || j == 7))
      dst[(uint32_t)j * plane + (uint32_t)ys * nx + (nx - 1)] = v;
    return;
  }
  T *d = dst + (uint32_t)j * plane;
  d[(uint32_t)ys * nx + xs] = v;
  // the column (W / E) and row (S / N) this value is copied to, and their
  // corner when both apply
  int xc = -1, yc = -1;
  if (c.bc[kFaceW] == kZeroGradient && xs == 1 && c_ex[j] > 0) xc = 0;
  if (c.bc[kFaceE] == kZeroGradient && xs == nx - 2 && c_ex[j] < 0) xc = nx - 1;
  if (c.bc[kFaceS] == kZeroGradient && ys == 1 && c_ey[j] > 0) yc = 0;
  if (c.bc[kFaceN] == kZeroGradient && ys == ny - 2 && c_ey[j] < 0) yc = ny - 1;
  if (xc >= 0) d[(uint32_t)ys * nx + xc] = v;
  if (yc >= 0) {
    d[(uint32_t)yc * nx + xs] = v;
    if (xc >= 0) d[(uint32_t)yc * nx + xc] = v;
  }
}

// All nine pushes of a face node.
template <typename T, bool GZG>
__device__ __forceinline__ void push_boundary9(const CaseDesc *c, T *dst, int x, int y, T f0, T f1,
                                            T f2, T f3, T f4, T f5, T f6, T f7, T f8) {
  push_one<T, GZG>(*c, dst, x, y, 0, f0);
  push_one<T, GZG>(*c, dst, x, y, 1, f1);
  push_one<T, GZG>(*c, dst, x, y, 2, f2);
  push_one<T, GZG>(*c, dst, x, y, 3, f3);
  push_one<T, GZG>(*c, dst, x, y, 4, f4);
  push_one<T, GZG>(*c, dst, x, y, 5, f5);
  push_one<T, GZG>(*c, dst, x, y, 6, f6);
  push_one<T, GZG>(*c, dst, x, y, 7, f7);
  push_one<T, GZG>(*c, dst, x, y, 8, f8);
}

// The node's IB force if it lies in the force box (consumed: cleared once
// read), plus the uniform fluid force.
template <typename T>
__device__ __forceinline__ void node_force(T *frc, uint32_t plane, uint32_t p, int x, int y,
                                           bool in_box, int fb0, int fy0, int fb1, int fy1,
                                           T &Fx, T &Fy) {
  if (in_box && x >= fb0 && x <= fb1 && y >= fy0 && y <= fy1) {
    const T a = frc[p], b = frc[plane + p];
    if (a != T(0) || b != T(0)) {
      Fx += a;
      Fy += b;
      frc[p] = T(0);
      frc[plane + p] = T(0);
    }
  }
}

// Collide and stream the inner nodes (1 <= x <= nx-3, 1 <= y <= ny-2) of
// tile (tx, ty) of case c from f[cur] into f[cur^1]: every link stays inside
// the lattice, so every push is a plain store.  The other nodes (the face
// nodes) are left to collide_stream_face_kernel, which keeps the face rules
// out of this kernel and its register footprint small.  `force` allows the
// IB force of the case's force box to be read (and cleared once applied).
template <typename T, int COL>
__device__ __forceinline__ void collide_stream_tile(const CaseDesc *cp, int tx, int ty, int cur,
                                                    int rpt, bool force) {
  const CaseDesc &c = *cp;
  const CaseState *cs = c.state;
  const T *__restrict__ src = (const T *)c.f[cur];
  T *__restrict__ dst = (T *)c.f[cur ^ 1];
  T *__restrict__ frc = (T *)c.force;
  const int TX = blockDim.x, TY = blockDim.y * rpt;
  const int nx = c.nx, ny = c.ny;
  const uint32_t plane = (uint32_t)c.plane;
  const int x = tx * TX + threadIdx.x;
  const int ybase = ty * TY;
  const int xt0 = tx * TX, xt1 = xt0 + TX - 1, yt1 = ybase + TY - 1;
  // IB force only inside the union of the bodies' force boxes
  int fb0 = 0, fy0 = 0, fb1 = -1, fy1 = -1;
  bool tile_force = false;
  if (force && cs->fbox_valid) {
    fb0 = cs->fbox[0]; fy0 = cs->fbox[1]; fb1 = cs->fbox[2]; fy1 = cs->fbox[3];
    tile_force = !(fb1 < xt0 || fb0 > xt1 || fy1 < ybase || fy0 > yt1);
  }
  const T ffx = T(c.fluid_fx), ffy = T(c.fluid_fy);
  if (x < 1 || x > nx - 3) return;
  for (int r = 0; r < rpt; r++) {
    const int y = ybase + threadIdx.y + r * blockDim.y;
    if (y < 1 || y > ny - 2) continue;
    const uint32_t p = (uint32_t)y * nx + x;
    T f[9];
#pragma unroll
    for (int i = 0; i < 9; i++) f[i] = src[(uint32_t)i * plane + p];
    T Fx = ffx, Fy = ffy;
    node_force<T>(frc, plane, p, x, y, tile_force, fb0, fy0, fb1, fy1, Fx, Fy);
    collide<T, sizeof(T) == 4, COL>(f, Fx, Fy, c);
#pragma unroll
    for (int i = 0; i < 9; i++) dst[(uint32_t)i * plane + p + EXI(i) + EYI(i) * nx] = f[i];
  }
}

// The hold-rectangle tiles of a pipelined step (a few dozen workgroups on
// the step's critical path, so latency rather than bandwidth): every row's
// populations and IB force are loaded before any is used, and before the
// case's halt flag is known.  The force is read at every node: outside the
// force box it is zero (each step's collide-stream consumes the box of the
// previous IB pass), so the result is that of collide_stream_tile.
template <typename T, int COL, int RPT>
__device__ __forceinline__ void collide_stream_tile_near(const CaseDesc *cp, int tx, int ty, int cur) {
  const CaseDesc &c = *cp;
  const CaseState *cs = c.state;
  const T *__restrict__ src = (const T *)c.f[cur];
  T *__restrict__ dst = (T *)c.f[cur ^ 1];
  T *__restrict__ frc = (T *)c.force;
  const int TX = blockDim.x, TY = blockDim.y * RPT;
  const int nx = c.nx, ny = c.ny;
  const uint32_t plane = (uint32_t)c.plane;
  const int x = tx * TX + threadIdx.x;
  const int ybase = ty * TY;
  if (x < 1 || x > nx - 3) return;
  T f[RPT][9], fa[RPT], fb[RPT];
  bool ok[RPT];
#pragma unroll
  for (int r = 0; r < RPT; r++) {
    const int y = ybase + threadIdx.y + r * blockDim.y;
    ok[r] = y >= 1 && y <= ny - 2;
    const uint32_t p = (uint32_t)(ok[r] ? y : 1) * nx + x;
#pragma unroll
    for (int i = 0; i < 9; i++) f[r][i] = src[(uint32_t)i * plane + p];
    fa[r] = frc[p];
    fb[r] = frc[plane + p];
  }
  if (__hip_atomic_load(&cs->flags, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) & kCaseHalted) return;
  const T ffx = T(c.fluid_fx), ffy = T(c.fluid_fy);
#pragma unroll
  for (int r = 0; r < RPT; r++) {
    if (!ok[r]) continue;
    const int y = ybase + threadIdx.y + r * blockDim.y;
    const uint32_t p = (uint32_t)y * nx + x;
    T Fx = ffx, Fy = ffy;
    if (fa[r] != T(0) || fb[r] != T(0)) {
      Fx += fa[r];
      Fy += fb[r];
      frc[p] = T(0);
      frc[plane + p] = T(0);
    }
    collide<T, sizeof(T) == 4, COL>(f[r], Fx, Fy, c);
#pragma unroll
    for (int i = 0; i < 9; i++) dst[(uint32_t)i * plane + p + EXI(i) + EYI(i) * nx] = f[r][i];
  }
}

// Every inner node of every case (batches flatten (case, tile) through
// tile_prefix).
template <typename T, int COL>
__global__ __launch_bounds__(1024) void collide_stream_kernel(const CaseDesc *__restrict__ cases,
                                                              const int32_t *__restrict__ tile_prefix,
                                                              int ncases, int ntiles, int rpt,
                                                              int xcd_remap) {
  const int nb = gridDim.x;
  int t = blockIdx.x;
  if (xcd_remap) t = (blockIdx.x & 7) * (nb >> 3) + (blockIdx.x >> 3);
  if (t >= ntiles) return;
  int ci = 0;
  if (ncases > 1) {
    int lo = 0, hi = ncases - 1;
    while (lo < hi) {
      const int mid = (lo + hi + 1) >> 1;
      if (tile_prefix[mid] <= t) lo = mid; else hi = mid - 1;
    }
    ci = lo;
  }
  const CaseDesc *cp = cases + ci;
  const CaseState *cs = cp->state;
  if (cs->step >= cs->target || (cs->flags & kCaseHalted)) return;
  const int local = t - tile_prefix[ci];
  collide_stream_tile<T, COL>(cp, local % cp->tiles_x, local / cp->tiles_x, cs->cur, rpt, true);
}

// The face nodes of every case, kFaceBlock per workgroup (face_prefix[i] is
// the first workgroup of case i, so the case is uniform in a workgroup), with
// the face closures.  cur < 0: each case's current lattice from its state;
// otherwise the lattice given (a pipelined step, whose case state the IB pass
// may be updating).
template <typename T, int COL, bool GZG>
__global__ __launch_bounds__(kFaceBlock) void collide_stream_face_kernel(const CaseDesc *__restrict__ cases,
                                                                  const int32_t *__restrict__ face_prefix,
                                                                  int ncases, int nblocks, int cur_arg,
                                                                  int force) {
  const int blk = blockIdx.x;
  if (blk >= nblocks) return;
  int ci = 0;
  if (ncases > 1) {
    int lo = 0, hi = ncases - 1;
    while (lo < hi) {
      const int mid = (lo + hi + 1) >> 1;
      if (face_prefix[mid] <= blk) lo = mid; else hi = mid - 1;
    }
    ci = lo;
  }
  const CaseDesc *cp = cases + ci;
  const CaseDesc &c = *cp;
  const CaseState *cs = c.state;
  const int m = (blk - face_prefix[ci]) * kFaceBlock + (int)threadIdx.x;
  if (m >= face_nodes(c.nx, c.ny)) return;
  const int nx = c.nx, ny = c.ny;
  int x, y;
  if (m < nx) {
    x = m; y = 0;
  } else if (m < 2 * nx) {
    x = m - nx; y = ny - 1;
  } else {
    const int q = m - 2 * nx, col = q / (ny - 2);
    x = col == 0 ? 0 : (col == 1 ? nx - 2 : nx - 1);
    y = 1 + q % (ny - 2);
  }
  const uint32_t plane = (uint32_t)c.plane;
  const uint32_t p = (uint32_t)y * nx + x;
  // The populations are loaded before the case state is known (a latency
  // chain on a small launch): from the given lattice, or from both lattices
  // when the state names it.
  T f[9];
  int cur = cur_arg;
  if (cur >= 0) {
    const T *__restrict__ src = (const T *)c.f[cur];
#pragma unroll
    for (int i = 0; i < 9; i++) f[i] = src[(uint32_t)i * plane + p];
    if (__hip_atomic_load(&cs->flags, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) & kCaseHalted) return;
  } else {
    const T *__restrict__ s0 = (const T *)c.f[0];
    const T *__restrict__ s1 = (const T *)c.f[1];
    T g[9];
#pragma unroll
    for (int i = 0; i < 9; i++) {
      f[i] = s0[(uint32_t)i * plane + p];
      g[i] = s1[(uint32_t)i * plane + p];
    }
    if (cs->step >= cs->target || (cs->flags & kCaseHalted)) return;
    cur = cs->cur;
    if (cur) {
#pragma unroll
      for (int i = 0; i < 9; i++) f[i] = g[i];
    }
  }
  T *__restrict__ dst = (T *)c.f[cur ^ 1];
  T *__restrict__ frc = (T *)c.force;
  T Fx = T(c.fluid_fx), Fy = T(c.fluid_fy);
  const bool box = force && cs->fbox_valid;
  node_force<T>(frc, plane, p, x, y, box, box ? cs->fbox[0] : 0, box ? cs->fbox[1] : 0,
                box ? cs->fbox[2] : -1, box ? cs->fbox[3] : -1, Fx, Fy);
  collide<T, sizeof(T) == 4, COL>(f, Fx, Fy, c);
  push_boundary9<T, GZG>(cp, dst, x, y, f[0], f[1], f[2], f[3], f[4], f[5], f[6], f[7], f[8]);
}

// No-slip walls with the on-node closure of Zou and He at zero wall
// velocity, applied to the wall nodes after the step's streaming is
// complete (the pushes of inner and face nodes have all landed).  The
// populations that would have come from outside are rebuilt so that the
// node has no momentum: the normal one as its opposite, the two diagonals
// as their opposites corrected by half the tangential imbalance of the
// axial pair.  A corner of two such walls bounces the three populations
// pointing into the fluid and shares between the two buried diagonals what
// the density of the diagonal inner node leaves.  The relations pair
// populations of equal weight, so they hold unchanged for the shifted FP32
// store (g = f - w rho0).  Links leaving through these faces were dropped
// by push_one.  One thread per perimeter node: rows 0 and ny-1, then
// columns 0 and nx-1 between them.
template <typename T>
__global__ __launch_bounds__(256) void zou_he_kernel(const CaseDesc *__restrict__ cp, int cur_arg) {
  const CaseDesc &c = *cp;
  const CaseState *cs = c.state;
  const int nx = c.nx, ny = c.ny;
  const int m = blockIdx.x * blockDim.x + (int)threadIdx.x;
  if (m >= 2 * nx + 2 * (ny - 2)) return;
  int x, y;
  if (m < 2 * nx) {
    x = m % nx;
    y = m < nx ? 0 : ny - 1;
  } else {
    const int q = m - 2 * nx;
    x = q < ny - 2 ? 0 : nx - 1;
    y = 1 + q % (ny - 2);
  }
  const bool w = x == 0 && c.bc[kFaceW] == kZouHe, e = x == nx - 1 && c.bc[kFaceE] == kZouHe;
  const bool so = y == 0 && c.bc[kFaceS] == kZouHe, no = y == ny - 1 && c.bc[kFaceN] == kZouHe;
  if (!(w || e || so || no)) return;
  int cur = cur_arg;
  if (cur < 0) {
    if (cs->step >= cs->target || (cs->flags & kCaseHalted)) return;
    cur = cs->cur;
  } else if (__hip_atomic_load(&cs->flags, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) & kCaseHalted) {
    return;
  }
  T *__restrict__ f = (T *)c.f[cur ^ 1];
  const uint32_t plane = (uint32_t)c.plane;
  const uint32_t p = (uint32_t)y * nx + x;
  T v[9];
#pragma unroll
  for (int i = 0; i < 9; i++) v[i] = f[i * plane + p];
  if ((w || e) && (so || no)) {
    const int sx = w ? 1 : -1, sy = so ? 1 : -1;
    const int ix = sx > 0 ? 1 : 3, iy = sy > 0 ? 2 : 4;
    // diagonal into the fluid, and the two buried ones
    const int id = sx > 0 ? (sy > 0 ? 5 : 8) : (sy > 0 ? 6 : 7);
    const int ia = sx > 0 ? (sy > 0 ? 6 : 7) : (sy > 0 ? 5 : 8);  // (-sx, sy)
    const int ib = sx > 0 ? (sy > 0 ? 8 : 5) : (sy > 0 ? 7 : 6);  // (sx, -sy)
    v[ix] = v[OPPI(ix)];
    v[iy] = v[OPPI(iy)];
    v[id] = v[OPPI(id)];
    const uint32_t pc = (uint32_t)(y + sy) * nx + (x + sx);
    double rc = 0.0, known = 0.0;
#pragma unroll
    for (int i = 0; i < 9; i++) {
      rc += (double)f[i * plane + pc];
      if (i != ia && i != ib) known += (double)v[i];
    }
    const T b = T(0.5 * (rc - known));
    f[ix * plane + p] = v[ix];
    f[iy * plane + p] = v[iy];
    f[id * plane + p] = v[id];
    f[ia * plane + p] = b;
    f[ib * plane + p] = b;
  } else if (so || no) {
    const int in = so ? 2 : 4, d1 = so ? 5 : 8, d2 = so ? 6 : 7;
    const T t = T(0.5) * (v[1] - v[3]);
    f[in * plane + p] = v[OPPI(in)];
    f[d1 * plane + p] = v[OPPI(d1)] - t;
    f[d2 * plane + p] = v[OPPI(d2)] + t;
  } else {
    const int in = w ? 1 : 3, d1 = w ? 5 : 6, d2 = w ? 8 : 7;
    const T t = T(0.5) * (v[2] - v[4]);
    f[in * plane + p] = v[OPPI(in)];
    f[d1 * plane + p] = v[OPPI(d1)] - t;
    f[d2 * plane + p] = v[OPPI(d2)] + t;
  }
}

hipError_t launch_zou_he(int precision, const CaseDesc *c, int nx, int ny, int cur, hipStream_t stream) {
  const int n = 2 * nx + 2 * (ny - 2);
  const int blocks = (n + 255) / 256;
  if (precision == kPrecFP64)
    hipLaunchKernelGGL(zou_he_kernel<double>, dim3(blocks), dim3(256), 0, stream, c, cur);
  else
    hipLaunchKernelGGL(zou_he_kernel<float>, dim3(blocks), dim3(256), 0, stream, c, cur);
  return hipGetLastError();
}

// One part of a pipelined step of a single case (see PipeArgs): the tiles
// of the hold rectangle (NEAR), which read the IB force and are read by the
// IB pass, or all other tiles, which do neither (force = 0, passed at run
// time, which keeps this instance's register allocation that of the plain
// kernel).  The input lattice `cur` comes from the host: the IB pass of the
// previous step may still be updating the case state while the far tiles
// run.
template <typename T, int COL, bool NEAR>
__global__ __launch_bounds__(1024) void collide_stream_pipe_kernel(const CaseDesc *__restrict__ cases,
                                                                   int ntiles, int rpt, int xcd_remap,
                                                                   PipeArgs pa, int force) {
  const CaseDesc *cp = cases;
  const CaseState *cs = cp->state;
  const int nb = gridDim.x;
  int t = blockIdx.x;
  if (xcd_remap) t = (t & 7) * (nb >> 3) + (t >> 3);
  if (NEAR) {
    if (t >= pa.hntx * pa.hnty) return;
    const int tx = pa.htx0 + t % pa.hntx, ty = pa.hty0 + t / pa.hntx;
    if (rpt == 1) {
      collide_stream_tile_near<T, COL, 1>(cp, tx, ty, pa.cur);
    } else if (rpt == 2) {
      collide_stream_tile_near<T, COL, 2>(cp, tx, ty, pa.cur);
    } else {
      if (__hip_atomic_load(&cs->flags, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) & kCaseHalted) return;
      collide_stream_tile<T, COL>(cp, tx, ty, pa.cur, rpt, true);
    }
    return;
  }
  if (__hip_atomic_load(&cs->flags, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) & kCaseHalted) return;
  if (t >= ntiles) return;
  const int tx = t % cp->tiles_x, ty = t / cp->tiles_x;
  if (tx >= pa.htx0 && tx < pa.htx0 + pa.hntx && ty >= pa.hty0 && ty < pa.hty0 + pa.hnty) return;
  collide_stream_tile<T, COL>(cp, tx, ty, pa.cur, rpt, force != 0);
}

#define IBL_DISPATCH(precision, collision, LAUNCH)                                             \
  if ((precision) == kPrecFP64) {                                                              \
    if ((collision) == kBGK) LAUNCH(double, kBGK);                                             \
    else if ((collision) == kTRT) LAUNCH(double, kTRT);                                        \
    else LAUNCH(double, kCMMRT);                                                               \
  } else {                                                                                     \
    if ((collision) == kBGK) LAUNCH(float, kBGK);                                              \
    else if ((collision) == kTRT) LAUNCH(float, kTRT);                                         \
    else LAUNCH(float, kCMMRT);                                                                \
  }

hipError_t launch_collide_stream(int precision, int collision, const CaseDesc *cases,
                                 const int32_t *tile_prefix, int ncases, int ntiles,
                                 LaunchShape shape, hipStream_t stream) {
  if (ntiles <= 0) return hipSuccess;
  int grid = ntiles;
  if (shape.xcd_remap) grid = (ntiles + 7) / 8 * 8;
  dim3 block(shape.block_x, shape.block_y);
  const int rpt = shape.rows_per_thread;
  const int remap = shape.xcd_remap;
#define IBL_LAUNCH(T, C)                                                                        \
  hipLaunchKernelGGL((collide_stream_kernel<T, C>), dim3(grid), block, 0, stream, cases,        \
                     tile_prefix, ncases, ntiles, rpt, remap)
  IBL_DISPATCH(precision, collision, IBL_LAUNCH)
#undef IBL_LAUNCH
  return hipGetLastError();
}

hipError_t launch_collide_stream_faces(int precision, int collision, const CaseDesc *cases,
                                       const int32_t *face_prefix, int ncases, int nblocks, int cur,
                                       int force, int general_zg, hipStream_t stream) {
  if (nblocks <= 0) return hipSuccess;
#define IBL_LAUNCH(T, C)                                                                         \
  if (general_zg)                                                                                \
    hipLaunchKernelGGL((collide_stream_face_kernel<T, C, true>), dim3(nblocks), dim3(kFaceBlock), \
                       0, stream, cases, face_prefix, ncases, nblocks, cur, force);              \
  else                                                                                           \
    hipLaunchKernelGGL((collide_stream_face_kernel<T, C, false>), dim3(nblocks), dim3(kFaceBlock), \
                       0, stream, cases, face_prefix, ncases, nblocks, cur, force)
  IBL_DISPATCH(precision, collision, IBL_LAUNCH)
#undef IBL_LAUNCH
  return hipGetLastError();
}

hipError_t launch_collide_stream_pipe(int precision, int collision, const CaseDesc *cases, int ntiles,
                                      LaunchShape shape, const PipeArgs &pa, int near,
                                      hipStream_t stream) {
  if (ntiles <= 0) return hipSuccess;
  int grid = near ? pa.hntx * pa.hnty : ntiles;
  if (shape.xcd_remap) grid = (grid + 7) / 8 * 8;
  dim3 block(shape.block_x, shape.block_y);
  const int rpt = shape.rows_per_thread;
  const int remap = shape.xcd_remap;
#define IBL_LAUNCH(T, C)                                                                        \
  if (near)                                                                                     \
    hipLaunchKernelGGL((collide_stream_pipe_kernel<T, C, true>), dim3(grid), block, 0, stream,  \
                       cases, ntiles, rpt, remap, pa, 1);                                       \
  else                                                                                          \
    hipLaunchKernelGGL((collide_stream_pipe_kernel<T, C, false>), dim3(grid), block, 0, stream, \
                       cases, ntiles, rpt, remap, pa, 0)
  IBL_DISPATCH(precision, collision, IBL_LAUNCH)
#undef IBL_LAUNCH
  return hipGetLastError();
}
#undef IBL_DISPATCH

// ------------------------------------------------------------ utilities
// Equilibrium start state f^eq(rho0, u_init): u_init is the parabolic inlet
// profile (W face parabolic), u_bc (any uniform face) or 0.
template <typename T>
__global__ void init_eq_kernel(CaseDesc c, int buf) {
  const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= c.plane) return;
  const int y = (int)(p / c.nx);
  double ux = 0.0;
  if (c.bc[kFaceW] == kVelParabolic)
    ux = 4.0 * c.u_bc * (y + 0.5) * (c.ny - 0.5 - y) * c.inv_ny2;
  else if (c.bc[0] == kVelUniform || c.bc[1] == kVelUniform || c.bc[2] == kVelUniform ||
           c.bc[3] == kVelUniform)
    ux = c.u_bc;
  T *f = (T *)c.f[buf];
  const bool shift = sizeof(T) == 4;
  for (int i = 0; i < 9; i++) {
    const double eu = c_ex[i] * ux;
    const double w = wgt<double>(i);
    const double feq = w * c.rho0 * (1.0 + 3.0 * eu + 4.5 * eu * eu - 1.5 * ux * ux);
    f[i * c.plane + p] = (T)(shift ? feq - w * c.rho0 : feq);
  }
  T *frc = (T *)c.force;
  frc[p] = T(0);
  frc[c.plane + p] = T(0);
}

hipError_t launch_init_equilibrium(const CaseDesc &c, int buf, hipStream_t stream) {
  const int threads = 256;
  const int blocks = (int)((c.plane + threads - 1) / threads);
  if (c.precision == kPrecFP64)
    hipLaunchKernelGGL(init_eq_kernel<double>, dim3(blocks), dim3(threads), 0, stream, c, buf);
  else
    hipLaunchKernelGGL(init_eq_kernel<float>, dim3(blocks), dim3(threads), 0, stream, c, buf);
  return hipGetLastError();
}

// Density and velocity of the current state, Eq. (4), FP64 output.
template <typename T>
__global__ void fields_kernel(CaseDesc c, int buf, double *rho, double *ux, double *uy) {
  const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= c.plane) return;
  const T *f = (const T *)c.f[buf];
  const T *frc = (const T *)c.force;
  const bool shift = sizeof(T) == 4;
  double s = 0, jx = 0, jy = 0;
  for (int i = 0; i < 9; i++) {
    const double v = (double)f[i * c.plane + p] + (shift ? wgt<double>(i) * c.rho0 : 0.0);
    s += v;
    jx += v * c_ex[i];
    jy += v * c_ey[i];
  }
  const double Fx = (double)frc[p] + c.fluid_fx, Fy = (double)frc[c.plane + p] + c.fluid_fy;
  rho[p] = s;
  ux[p] = (jx + 0.5 * Fx) / s;
  uy[p] = (jy + 0.5 * Fy) / s;
}

hipError_t launch_fields(const CaseDesc &c, int buf, double *rho, double *ux, double *uy,
                         hipStream_t stream) {
  const int threads = 256;
  const int blocks = (int)((c.plane + threads - 1) / threads);
  if (c.precision == kPrecFP64)
    hipLaunchKernelGGL(fields_kernel<double>, dim3(blocks), dim3(threads), 0, stream, c, buf, rho,
                       ux, uy);
  else
    hipLaunchKernelGGL(fields_kernel<float>, dim3(blocks), dim3(threads), 0, stream, c, buf, rho,
                       ux, uy);
  return hipGetLastError();
}

template <typename T>
__global__ void export_kernel(CaseDesc c, int buf, double *out) {
  const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= c.plane) return;
  const T *f = (const T *)c.f[buf];
  const bool shift = sizeof(T) == 4;
  for (int i = 0; i < 9; i++)
    out[i * c.plane + p] = (double)f[i * c.plane + p] + (shift ? wgt<double>(i) * c.rho0 : 0.0);
}

template <typename T>
__global__ void import_kernel(CaseDesc c, int buf, const double *in) {
  const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= c.plane) return;
  T *f = (T *)c.f[buf];
  const bool shift = sizeof(T) == 4;
  for (int i = 0; i < 9; i++)
    f[i * c.plane + p] = (T)(in[i * c.plane + p] - (shift ? wgt<double>(i) * c.rho0 : 0.0));
}

template <typename T>
__global__ void force_export_kernel(CaseDesc c, double *fx, double *fy) {
  const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= c.plane) return;
  const T *frc = (const T *)c.force;
  fx[p] = (double)frc[p];
  fy[p] = (double)frc[c.plane + p];
}

hipError_t launch_export(const CaseDesc &c, int buf, double *out, hipStream_t stream) {
  const int threads = 256;
  const int blocks = (int)((c.plane + threads - 1) / threads);
  if (c.precision == kPrecFP64)
    hipLaunchKernelGGL(export_kernel<double>, dim3(blocks), dim3(threads), 0, stream, c, buf, out);
  else
    hipLaunchKernelGGL(export_kernel<float>, dim3(blocks), dim3(threads), 0, stream, c, buf, out);
  return hipGetLastError();
}

hipError_t launch_import(const CaseDesc &c, int buf, const double *in, hipStream_t stream) {
  const int threads = 256;
  const int blocks = (int)((c.plane + threads - 1) / threads);
  if (c.precision == kPrecFP64)
    hipLaunchKernelGGL(import_kernel<double>, dim3(blocks), dim3(threads), 0, stream, c, buf, in);
  else
    hipLaunchKernelGGL(import_kernel<float>, dim3(blocks), dim3(threads), 0, stream, c, buf, in);
  return hipGetLastError();
}

hipError_t launch_force_export(const CaseDesc &c, double *fx, double *fy, hipStream_t stream) {
  const int threads = 256;
  const int blocks = (int)((c.plane + threads - 1) / threads);
  if (c.precision == kPrecFP64)
    hipLaunchKernelGGL(force_export_kernel<double>, dim3(blocks), dim3(threads), 0, stream, c, fx,
                       fy);
  else
    hipLaunchKernelGGL(force_export_kernel<float>, dim3(blocks), dim3(threads), 0, stream, c, fx,
                       fy);
  return hipGetLastError();
}

}  // namespace iblbm
