// Device code of the D2Q9 collide + stream shared by every kernel that
// updates lattice nodes: the collision (BGK, TRT, central-moment MRT), the
// pushes with the face closures, and the per-tile and per-face-node bodies
// of the collide-stream kernels, which the fused step kernel runs too.
#pragma once
#include "ib_lbm_internal.h"

namespace iblbm {

static __constant__ int c_ex[9] = {0, 1, 0, -1, 0, 1, -1, -1, 1};
static __constant__ int c_ey[9] = {0, 0, 1, 0, -1, 1, 1, -1, -1};

#define EXI(i) ((i) == 1 || (i) == 5 || (i) == 8 ? 1 : ((i) == 3 || (i) == 6 || (i) == 7 ? -1 : 0))
#define EYI(i) ((i) == 2 || (i) == 5 || (i) == 6 ? 1 : ((i) == 4 || (i) == 7 || (i) == 8 ? -1 : 0))
#define OPPI(i) ((i) == 0 ? 0 : ((i) <= 4 ? (((i) + 1) & 3) + 1 : (((i) - 3) & 3) + 5))

template <typename R>
__device__ __forceinline__ R wgt(int i) {
  return i == 0 ? R(4) / R(9) : (i <= 4 ? R(1) / R(9) : R(1) / R(36));
}

// ---------------------------------------------------------------- collision
// No automatic contraction of multiply-adds here: every function below that
// does arithmetic turns it off for its body (and lbm_kernels.hip is compiled
// with -ffp-contract=off as well), and every fused multiply-add is written
// out with fmad.  Each kernel that inlines the collision (plain, pipelined,
// batched and fused steps, face nodes, the IB pass's own collision of its
// support) then performs exactly the same rounding, whichever source file
// it is compiled in, and a node's result does not depend on which launch
// updated it.
template <typename R>
__device__ __forceinline__ R fmad(R a, R b, R c) {
  if constexpr (sizeof(R) == 4) return __builtin_fmaf(a, b, c);
  else return __builtin_fma(a, b, c);
}

// f holds the stored values (f, or g = f - w rho0 when SHIFT).  sum_f is
// sum_i f_i, so the equilibrium in either form is w_i (sum_f + rho P_i(u)),
// P_i = 3 e.u + 4.5 (e.u)^2 - 1.5 u.u; m15uu = -1.5 u.u.
// Everything is computed in place to keep the register footprint small.
//
// BGK and TRT work on the four pairs (i, opposite of i) and the rest
// population.  With a = e_i.u, A = e_i.j (j = rho u, the momentum with half
// the force) and b = e_i.F for the first of a pair, the equilibrium splits
// into its even part w (sum_f + rho (4.5 a^2 - 1.5 u.u)) and its odd part
// +-3 w A, and the Guo source w [3 (e - u) + 9 (e.u) e].F into the even part
// w (9 a b - 3 u.F) and the odd part +-3 w b.  The even part of the
// non-equilibrium relaxes at s_e, the odd part at s_o (BGK: both omega), each
// source part is weighted by 1 - s/2 (Eq. 3-4 and the TRT of Sec. 2.2).
// Writing the pairs this way takes about half the arithmetic of evaluating
// nine equilibria; a node without force skips the source terms (they are
// exactly zero there).
//
// The odd part carries the equilibrium's momentum, which the collision must
// return unchanged.  3w = 1/3 or 1/12 is not a binary number: rounded to
// FP32 it is 3e-8 too large, and the collision would then add that fraction
// of s_o j to the momentum at every node and step, a systematic force that
// shifts a long FP32 run's drag by 1e-4.  In FP32 the product therefore
// carries the constant's rounding residue as a second term, so the
// momentum is returned to within rounding that does not accumulate.
template <typename R>
struct PairOut {
  R e, o;  // even and odd increments: f_i += e + o, f_opp += e - o
};

// x * c for the exact constant c = 1/n (n = 3, 12): FP64 as is, FP32 with
// the residue c - fl32(c) as a second term.
template <typename R, int N>
__device__ __forceinline__ R times_inv(R x) {
  #pragma clang fp contract(off)
  constexpr double c = 1.0 / N;
  if constexpr (sizeof(R) == 4) {
    constexpr float hi = (float)c;
    constexpr float lo = (float)(c - (double)hi);
    return fmad(x, R(hi), x * R(lo));
  } else {
    return x * R(c);
  }
}

template <typename R, int N3W>
__device__ __forceinline__ PairOut<R> pair_relax(R fi, R fj, R a, R A, R w, R sum, R rho,
                                                 R m15uu, R se, R so) {
  #pragma clang fp contract(off)
  const R ev = w * fmad(rho, fmad(R(4.5) * a, a, m15uu), sum);
  const R od = times_inv<R, N3W>(A);
  PairOut<R> r;
  r.e = se * fmad(R(-0.5), fi + fj, ev);
  r.o = so * fmad(R(-0.5), fi - fj, od);
  return r;
}

template <typename R, int N3W>
__device__ __forceinline__ void pair_source(PairOut<R> &r, R a, R b, R w, R m3uF, R pe, R po) {
  #pragma clang fp contract(off)
  r.e = fmad(pe, w * fmad(R(9) * a, b, m3uF), r.e);
  r.o = fmad(po, times_inv<R, N3W>(b), r.o);
}

// C carries the rates (omega, s_e, s_o, s_q, s_eps) and rho0: a CaseDesc or
// the by-value LeanArgs.
template <typename R, bool SHIFT, int COL, typename C>
__device__ __forceinline__ void collide(R (&f)[9], R Fx, R Fy, const C &c) {
  #pragma clang fp contract(off)
  const R sum = ((f[0] + f[1]) + (f[2] + f[3])) + ((f[4] + f[5]) + (f[6] + f[7])) + f[8];
  const R rho = SHIFT ? R(c.rho0) + sum : sum;
  const R jx = (f[1] - f[3]) + (f[5] - f[6]) + (f[8] - f[7]);
  const R jy = (f[2] - f[4]) + (f[5] + f[6]) - (f[7] + f[8]);
  const R inv_rho = R(1) / rho;
  const R jfx = fmad(R(0.5), Fx, jx), jfy = fmad(R(0.5), Fy, jy);
  const R ux = jfx * inv_rho;
  const R uy = jfy * inv_rho;

  if constexpr (COL == kBGK || COL == kTRT) {
    const R m15uu = R(-1.5) * fmad(ux, ux, uy * uy);
    const R se = COL == kBGK ? R(c.omega) : R(c.s_e);
    const R so = COL == kBGK ? R(c.omega) : R(c.s_o);
    const R w1 = R(1) / R(9), w2 = R(1) / R(36), w0 = R(4) / R(9);
    // pairs (1,3), (2,4), (5,7), (6,8): e.u = ux, uy, ux + uy, uy - ux
    const R a5 = ux + uy, a6 = uy - ux;
    PairOut<R> p1 = pair_relax<R, 3>(f[1], f[3], ux, jfx, w1, sum, rho, m15uu, se, so);
    PairOut<R> p2 = pair_relax<R, 3>(f[2], f[4], uy, jfy, w1, sum, rho, m15uu, se, so);
    PairOut<R> p5 = pair_relax<R, 12>(f[5], f[7], a5, jfx + jfy, w2, sum, rho, m15uu, se, so);
    PairOut<R> p6 = pair_relax<R, 12>(f[6], f[8], a6, jfy - jfx, w2, sum, rho, m15uu, se, so);
    R d0 = se * (w0 * fmad(rho, m15uu, sum) - f[0]);
    if (Fx != R(0) || Fy != R(0)) {
      const R m3uF = R(-3) * fmad(ux, Fx, uy * Fy);
      const R pe = fmad(R(-0.5), se, R(1)), po = fmad(R(-0.5), so, R(1));
      pair_source<R, 3>(p1, ux, Fx, w1, m3uF, pe, po);
      pair_source<R, 3>(p2, uy, Fy, w1, m3uF, pe, po);
      pair_source<R, 12>(p5, a5, Fx + Fy, w2, m3uF, pe, po);
      pair_source<R, 12>(p6, a6, Fy - Fx, w2, m3uF, pe, po);
      d0 = fmad(pe, w0 * m3uF, d0);
    }
    f[0] = f[0] + d0;
    f[1] = (f[1] + p1.e) + p1.o;
    f[3] = (f[3] + p1.e) - p1.o;
    f[2] = (f[2] + p2.e) + p2.o;
    f[4] = (f[4] + p2.e) - p2.o;
    f[5] = (f[5] + p5.e) + p5.o;
    f[7] = (f[7] + p5.e) - p5.o;
    f[6] = (f[6] + p6.e) + p6.o;
    f[8] = (f[8] + p6.e) - p6.o;
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
    // forward along x: (v-1, v0, v1) -> (k0, k1, k2):
    // k0 = s0, k1 = s1 - u s0, k2 = s2 - 2 u s1 + u^2 s0
#define IBL_FWD(u, u2, m, z, p)                                  \
    {                                                            \
      const R s0 = (m) + (z) + (p), s1 = (p) - (m), s2 = (p) + (m); \
      (m) = s0;                                                  \
      (z) = fmad(-(u), s0, s1);                                  \
      (p) = fmad((u2), s0, fmad(R(-2) * (u), s1, s2));           \
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
    const R E20 = fmad(-r0, ux2, sum * third);
    const R E02 = fmad(-r0, uy2, sum * third);
    const R E11 = -r0 * ux * uy;
    const R E21 = r0 * uy * (third + ux2);
    const R E12 = r0 * ux * (third + uy2);
    const R E22 = fmad(-r0, fmad(third, ux2 + uy2, ux2 * uy2), sum * (R(1) / R(9)));
    const R pq = fmad(R(-0.5), sq, R(1)) * third;
    a01 += Fx;                                       // k10
    a10 += Fy;                                       // k01
    a02 = fmad(-om, a02 - E20, a02);                 // k20
    a20 = fmad(-om, a20 - E02, a20);                 // k02
    a11 = fmad(-om, a11 - E11, a11);                 // k11
    a12 = fmad(pq, Fy, fmad(-sq, a12 - E21, a12));   // k21
    a21 = fmad(pq, Fx, fmad(-sq, a21 - E12, a21));   // k12
    a22 = fmad(-seps, a22 - E22, a22);               // k22
    // back: central -> raw moments, then the 3-point values at -1, 0, 1:
    // M1 = k1 + u k0, M2 = k2 + 2 u k1 + u^2 k0
#define IBL_BWD(u, u2, m, z, p)                                  \
    {                                                            \
      const R M0 = (m);                                          \
      const R M1 = fmad((u), M0, (z));                           \
      const R M2 = fmad((u2), M0, fmad(R(2) * (u), (z), (p)));   \
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
  #pragma clang fp contract(off)
  const int nx = c.nx, ny = c.ny, nseg = c.nseg;
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
  T *d = dst + j * kSeg;
  if (!GZG) {
    d[pop_node(xs, ys, nseg)] = v;
    if (c.bc[kFaceE] == kZeroGradient && xs == nx - 2 && (j == 3 || j == 6 || j == 7))
      d[pop_node(nx - 1, ys, nseg)] = v;
    return;
  }
  d[pop_node(xs, ys, nseg)] = v;
  // the column (W / E) and row (S / N) this value is copied to, and their
  // corner when both apply
  int xc = -1, yc = -1;
  if (c.bc[kFaceW] == kZeroGradient && xs == 1 && c_ex[j] > 0) xc = 0;
  if (c.bc[kFaceE] == kZeroGradient && xs == nx - 2 && c_ex[j] < 0) xc = nx - 1;
  if (c.bc[kFaceS] == kZeroGradient && ys == 1 && c_ey[j] > 0) yc = 0;
  if (c.bc[kFaceN] == kZeroGradient && ys == ny - 2 && c_ey[j] < 0) yc = ny - 1;
  if (xc >= 0) d[pop_node(xc, ys, nseg)] = v;
  if (yc >= 0) {
    d[pop_node(xs, yc, nseg)] = v;
    if (xc >= 0) d[pop_node(xc, yc, nseg)] = v;
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

// Offsets, from a node's population-0 offset, of the nodes its pushes reach
// in x: e_x = +1 from the last lane of a segment lands in the next segment,
// e_x = -1 from its first lane in the previous one.
__device__ __forceinline__ int seg_dx_plus(int x) {
  return (x & (kSeg - 1)) == kSeg - 1 ? kSegBlock - (kSeg - 1) : 1;
}
__device__ __forceinline__ int seg_dx_minus(int x) {
  return (x & (kSeg - 1)) == 0 ? (kSeg - 1) - kSegBlock : -1;
}

// The nine pushes of an inner node (every link stays inside the lattice).
// d: the destination lattice at the node's population-0 offset; rs: values
// per row (nseg kSegBlock).
template <typename T>
__device__ __forceinline__ void push_inner(T *__restrict__ d, int dxp, int dxm, int rs,
                                           const T (&f)[9]) {
#pragma unroll
  for (int i = 0; i < 9; i++)
    d[i * kSeg + (EXI(i) > 0 ? dxp : (EXI(i) < 0 ? dxm : 0)) + EYI(i) * rs] = f[i];
}

__device__ __forceinline__ int ld_agent(const int32_t *p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// A word that is the same for the whole launch and that no kernel running
// beside this one writes, loaded through the scalar data cache: after the
// first wave of a compute unit the others find it there, instead of every
// wave of the chip asking the one L2 channel that holds it.
__device__ __forceinline__ int ld_uniform(const int32_t *p) {
  return *(const __attribute__((address_space(4))) int32_t *)p;
}


// Inner nodes of one case from by-value arguments (LeanArgs).  The case's
// halt flag and force box are words of its state that every wave needs; they
// are read through the scalar data cache (one miss per compute unit), not
// as vector loads that would all meet in one L2 channel.
//
// lean_tile_index maps the launch's tile number t to the tile (tx, ty) that
// mode MODE updates (false: none); lean_tile updates it with the thread at
// (lx, ly) of a bx x by workgroup shape, as a kernel of its own or as a part
// of a fused launch.
template <int MODE>
__device__ __forceinline__ bool lean_tile_index(const LeanArgs &a, int t, int &tx, int &ty) {
  if (MODE == 1) {
    if (t >= a.hntx * a.hnty) return false;
    tx = a.htx0 + t % a.hntx;
    ty = a.hty0 + t / a.hntx;
    return true;
  }
  if (t >= a.ntiles) return false;
  tx = t % a.tiles_x;
  ty = t / a.tiles_x;
  return !(MODE == 2 && tx >= a.htx0 && tx < a.htx0 + a.hntx && ty >= a.hty0 && ty < a.hty0 + a.hnty);
}

template <typename T, int COL, int MODE>
__device__ __forceinline__ void lean_tile(const LeanArgs &a, int tx, int ty, int lx, int ly, int bx,
                                          int by) {
  #pragma clang fp contract(off)
  const T *__restrict__ src = (const T *)a.src;
  T *__restrict__ dst = (T *)a.dst;
  T *__restrict__ frc = (T *)a.force;
  const CaseState *cs = a.state;
  const int rpt = a.rpt;
  const int TX = bx, TY = by * rpt;
  const int nx = a.nx, ny = a.ny, nseg = a.nseg;
  const uint32_t plane = (uint32_t)nx * (uint32_t)ny;
  const int x = tx * TX + lx;
  if (x < 1 || x > nx - 3) return;
  const int ybase = ty * TY;
  const int dxp = seg_dx_plus(x), dxm = seg_dx_minus(x), rs = nseg * kSegBlock;
  const T ffx = T(a.fluid_fx), ffy = T(a.fluid_fy);
  // A halted case keeps its lattices as they are.  The flag is set by the IB
  // pass of an earlier launch; a pipelined far tile (MODE 2) runs beside the
  // IB pass of the previous step and may miss a halt that pass sets, and then
  // writes only the lattice that the halted case no longer reads.
  if (ld_uniform(&cs->flags) & kCaseHalted) return;
  // the force box (MODE 0): written by the IB pass of an earlier launch,
  // never by one running beside this kernel
  int fv = 0, f0 = 0, f1 = 0, f2 = 0, f3 = 0;
  if (MODE == 0) {
    fv = ld_uniform(&cs->fbox_valid);
    f0 = ld_uniform(&cs->fbox[0]);
    f1 = ld_uniform(&cs->fbox[1]);
    f2 = ld_uniform(&cs->fbox[2]);
    f3 = ld_uniform(&cs->fbox[3]);
  }
  for (int r = 0; r < rpt; r++) {
    const int y = ybase + ly + r * by;
    if (y < 1 || y > ny - 2) continue;
    const int64_t b0 = pop_node(x, y, nseg);
    T f[9];
#pragma unroll
    for (int i = 0; i < 9; i++) f[i] = src[b0 + i * kSeg];
    const uint32_t p = (uint32_t)y * nx + x;
    T Fx = ffx, Fy = ffy;
    T fa = T(0), fb = T(0);
    if (MODE == 1) {
      fa = frc[p];
      fb = frc[plane + p];
    }
    if (MODE == 1) {
      if (fa != T(0) || fb != T(0)) {
        Fx += fa;
        Fy += fb;
        frc[p] = T(0);
        frc[plane + p] = T(0);
      }
    } else if (MODE == 0) {
      node_force<T>(frc, plane, p, x, y, a.force_on && fv != 0, f0, f1, f2, f3, Fx, Fy);
    }
    collide<T, sizeof(T) == 4, COL>(f, Fx, Fy, a);
    push_inner<T>(dst + b0, dxp, dxm, rs, f);
  }
}

// The face nodes of every case, kFaceBlock per workgroup (face_prefix[i] is
// the first workgroup of case i, so the case is uniform in a workgroup), with
// the face closures.  cur < 0: each case's current lattice from its state;
// otherwise the lattice given (a sim stepped on its own, whose case state
// the IB pass of a pipelined step may be updating).
// face_node updates face node t of face workgroup blk.
template <typename T, int COL, bool GZG>
__device__ __forceinline__ void face_node(const CaseDesc *__restrict__ cases,
                                          const int32_t *__restrict__ face_prefix, int ncases,
                                          int nblocks, int blk, int t, int cur_arg, int force) {
  #pragma clang fp contract(off)
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
  const int m = (blk - face_prefix[ci]) * kFaceBlock + t;
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
  const int64_t pn = pop_node(x, y, c.nseg);
  // The populations are loaded before the case state is known (a latency
  // chain on a small launch): from the given lattice, or from both lattices
  // when the state names it.
  T f[9];
  int cur = cur_arg;
  if (cur >= 0) {
    const T *__restrict__ src = (const T *)c.f[cur] + pn;
#pragma unroll
    for (int i = 0; i < 9; i++) f[i] = src[i * kSeg];
    if (__hip_atomic_load(&cs->flags, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) & kCaseHalted) return;
  } else {
    const T *__restrict__ s0 = (const T *)c.f[0] + pn;
    const T *__restrict__ s1 = (const T *)c.f[1] + pn;
    T g[9];
#pragma unroll
    for (int i = 0; i < 9; i++) {
      f[i] = s0[i * kSeg];
      g[i] = s1[i * kSeg];
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

}  // namespace iblbm
