// Fused D2Q9 collide + stream for gfx950.
//
// One thread owns one node per row it visits: it reads the node's nine
// post-stream populations (coalesced: nine runs of 64 values of the node's
// row segment, see pop_node), collides them
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
#include "lbm_device.h"

namespace iblbm {

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
  const int nx = c.nx, ny = c.ny, nseg = c.nseg;
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
  const int dxp = seg_dx_plus(x), dxm = seg_dx_minus(x), rs = nseg * kSegBlock;
  for (int r = 0; r < rpt; r++) {
    const int y = ybase + threadIdx.y + r * blockDim.y;
    if (y < 1 || y > ny - 2) continue;
    const int64_t b0 = pop_node(x, y, nseg);
    T f[9];
#pragma unroll
    for (int i = 0; i < 9; i++) f[i] = src[b0 + i * kSeg];
    T Fx = ffx, Fy = ffy;
    node_force<T>(frc, plane, (uint32_t)y * nx + x, x, y, tile_force, fb0, fy0, fb1, fy1, Fx, Fy);
    collide<T, sizeof(T) == 4, COL>(f, Fx, Fy, c);
    push_inner<T>(dst + b0, dxp, dxm, rs, f);
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

// Inner nodes of one case, one tile per workgroup (lean_tile).
template <typename T, int COL, int MODE>
__global__ __launch_bounds__(1024) void collide_stream_lean_kernel(const LeanArgs a) {
  const int nb = gridDim.x;
  int t = blockIdx.x;
  if (a.remap) t = (t & 7) * (nb >> 3) + (t >> 3);
  int tx, ty;
  if (!lean_tile_index<MODE>(a, t, tx, ty)) return;
  lean_tile<T, COL, MODE>(a, tx, ty, threadIdx.x, threadIdx.y, blockDim.x, blockDim.y);
}

template <typename T, int COL, bool GZG>
__global__ __launch_bounds__(kFaceBlock) void collide_stream_face_kernel(const CaseDesc *__restrict__ cases,
                                                                  const int32_t *__restrict__ face_prefix,
                                                                  int ncases, int nblocks, int cur_arg,
                                                                  int force) {
  face_node<T, COL, GZG>(cases, face_prefix, ncases, nblocks, blockIdx.x, threadIdx.x, cur_arg, force);
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
  T *__restrict__ f = (T *)c.f[cur ^ 1] + pop_node(x, y, c.nseg);
  T v[9];
#pragma unroll
  for (int i = 0; i < 9; i++) v[i] = f[i * kSeg];
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
    const T *fc = (const T *)c.f[cur ^ 1] + pop_node(x + sx, y + sy, c.nseg);
    double rc = 0.0, known = 0.0;
#pragma unroll
    for (int i = 0; i < 9; i++) {
      rc += (double)fc[i * kSeg];
      if (i != ia && i != ib) known += (double)v[i];
    }
    const T b = T(0.5 * (rc - known));
    f[ix * kSeg] = v[ix];
    f[iy * kSeg] = v[iy];
    f[id * kSeg] = v[id];
    f[ia * kSeg] = b;
    f[ib * kSeg] = b;
  } else if (so || no) {
    const int in = so ? 2 : 4, d1 = so ? 5 : 8, d2 = so ? 6 : 7;
    const T t = T(0.5) * (v[1] - v[3]);
    f[in * kSeg] = v[OPPI(in)];
    f[d1 * kSeg] = v[OPPI(d1)] - t;
    f[d2 * kSeg] = v[OPPI(d2)] + t;
  } else {
    const int in = w ? 1 : 3, d1 = w ? 5 : 6, d2 = w ? 8 : 7;
    const T t = T(0.5) * (v[2] - v[4]);
    f[in * kSeg] = v[OPPI(in)];
    f[d1 * kSeg] = v[OPPI(d1)] - t;
    f[d2 * kSeg] = v[OPPI(d2)] + t;
  }
}

hipError_t launch_zou_he(int precision, const CaseDesc *c, int nx, int ny, int cur, hipStream_t stream,
                         LaunchTarget *ns) {
  const int n = 2 * nx + 2 * (ny - 2);
  const int blocks = (n + 255) / 256;
  if (precision == kPrecFP64) return issue(zou_he_kernel<double>, dim3(blocks), dim3(256), 0, stream, ns, c, cur);
  return issue(zou_he_kernel<float>, dim3(blocks), dim3(256), 0, stream, ns, c, cur);
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
                                       int force, int general_zg, hipStream_t stream, LaunchTarget *ns) {
  if (nblocks <= 0) return nothing_to_launch(stream, ns);
#define IBL_LAUNCH(T, C)                                                                         \
  return general_zg ? issue(collide_stream_face_kernel<T, C, true>, dim3(nblocks), dim3(kFaceBlock), \
                            0, stream, ns, cases, face_prefix, ncases, nblocks, cur, force)        \
                    : issue(collide_stream_face_kernel<T, C, false>, dim3(nblocks), dim3(kFaceBlock), \
                            0, stream, ns, cases, face_prefix, ncases, nblocks, cur, force)
  IBL_DISPATCH(precision, collision, IBL_LAUNCH)
#undef IBL_LAUNCH
}

hipError_t launch_collide_stream_lean(int precision, int collision, const LeanArgs &a, int mode,
                                      LaunchShape shape, hipStream_t stream, LaunchTarget *ns) {
  int grid = mode == 1 ? a.hntx * a.hnty : a.ntiles;
  if (grid <= 0) return nothing_to_launch(stream, ns);
  if (a.remap) grid = (grid + 7) / 8 * 8;
  dim3 block(shape.block_x, shape.block_y);
#define IBL_LAUNCH(T, C)                                                                              \
  return mode == 1   ? issue(collide_stream_lean_kernel<T, C, 1>, dim3(grid), block, 0, stream, ns, a) \
         : mode == 2 ? issue(collide_stream_lean_kernel<T, C, 2>, dim3(grid), block, 0, stream, ns, a) \
                     : issue(collide_stream_lean_kernel<T, C, 0>, dim3(grid), block, 0, stream, ns, a)
  IBL_DISPATCH(precision, collision, IBL_LAUNCH)
#undef IBL_LAUNCH
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
  T *f = (T *)c.f[buf] + pop_node((int)(p - (int64_t)y * c.nx), y, c.nseg);
  const bool shift = sizeof(T) == 4;
  for (int i = 0; i < 9; i++) {
    const double eu = c_ex[i] * ux;
    const double w = wgt<double>(i);
    const double feq = w * c.rho0 * (1.0 + 3.0 * eu + 4.5 * eu * eu - 1.5 * ux * ux);
    f[i * kSeg] = (T)(shift ? feq - w * c.rho0 : feq);
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
  const int y = (int)(p / c.nx), x = (int)(p - (int64_t)y * c.nx);
  const T *f = (const T *)c.f[buf] + pop_node(x, y, c.nseg);
  const T *frc = (const T *)c.force;
  const bool shift = sizeof(T) == 4;
  double s = 0, jx = 0, jy = 0;
  for (int i = 0; i < 9; i++) {
    const double v = (double)f[i * kSeg] + (shift ? wgt<double>(i) * c.rho0 : 0.0);
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
  const int y = (int)(p / c.nx), x = (int)(p - (int64_t)y * c.nx);
  const T *f = (const T *)c.f[buf] + pop_node(x, y, c.nseg);
  const bool shift = sizeof(T) == 4;
  for (int i = 0; i < 9; i++)
    out[i * c.plane + p] = (double)f[i * kSeg] + (shift ? wgt<double>(i) * c.rho0 : 0.0);
}

template <typename T>
__global__ void import_kernel(CaseDesc c, int buf, const double *in) {
  const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= c.plane) return;
  const int y = (int)(p / c.nx), x = (int)(p - (int64_t)y * c.nx);
  T *f = (T *)c.f[buf] + pop_node(x, y, c.nseg);
  const bool shift = sizeof(T) == 4;
  for (int i = 0; i < 9; i++)
    f[i * kSeg] = (T)(in[i * c.plane + p] - (shift ? wgt<double>(i) * c.rho0 : 0.0));
}

// f = f^eq(rho, u) of Eq. 2 at every node from FP64 fields (rho null:
// rho0), shifted by w_i rho0 in the FP32 store.
template <typename T>
__global__ void set_eq_kernel(CaseDesc c, int buf, const double *rho, const double *ux,
                              const double *uy) {
  const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= c.plane) return;
  const int y = (int)(p / c.nx), x = (int)(p - (int64_t)y * c.nx);
  T *f = (T *)c.f[buf] + pop_node(x, y, c.nseg);
  const bool shift = sizeof(T) == 4;
  const double r = rho ? rho[p] : c.rho0, u = ux[p], v = uy[p];
  const double uu = u * u + v * v;
  for (int i = 0; i < 9; i++) {
    const double eu = c_ex[i] * u + c_ey[i] * v;
    const double w = wgt<double>(i);
    const double feq = w * r * (1.0 + 3.0 * eu + 4.5 * eu * eu - 1.5 * uu);
    f[i * kSeg] = (T)(shift ? feq - w * c.rho0 : feq);
  }
}

hipError_t launch_set_equilibrium(const CaseDesc &c, int buf, const double *rho, const double *ux,
                                  const double *uy, hipStream_t stream) {
  const int threads = 256;
  const int blocks = (int)((c.plane + threads - 1) / threads);
  if (c.precision == kPrecFP64)
    hipLaunchKernelGGL(set_eq_kernel<double>, dim3(blocks), dim3(threads), 0, stream, c, buf, rho, ux, uy);
  else
    hipLaunchKernelGGL(set_eq_kernel<float>, dim3(blocks), dim3(threads), 0, stream, c, buf, rho, ux, uy);
  return hipGetLastError();
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
