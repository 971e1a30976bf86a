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
// Steps 2-3 depend only on the body position: for a fixed body they run
// once and are cached, later steps copy the tables in bulk.
// Spreading is a gather: each support node keeps the list of markers whose
// stencil covers it (sorted by marker index, built with the tables) and sums
// over it in that order, so results are reproducible run to run and follow
// the marker order of the plain definition.  An atomic-scatter variant is
// kept for comparison.  The workspace lives in LDS when it fits (LDS
// instantiation), else in a global buffer of the body.
#include <mutex>

#include "ib_lbm_internal.h"
#include "lbm_device.h"

namespace iblbm {

__constant__ int c_exi[9] = {0, 1, 0, -1, 0, 1, -1, -1, 1};
__constant__ int c_eyi[9] = {0, 0, 1, 0, -1, 1, 1, -1, -1};
// opposite direction, a compile-time function so that unrolled loops index
// register arrays with constants
__device__ __forceinline__ constexpr int opp_of(int i) {
  return i == 0 ? 0 : (i <= 4 ? ((i + 1) & 3) + 1 : ((i - 3) & 3) + 5);
}
__constant__ double c_w[9] = {4.0 / 9.0,  1.0 / 9.0,  1.0 / 9.0,  1.0 / 9.0, 1.0 / 9.0,
                              1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0};

constexpr int kIbmDynLds = 150 * 1024;

// Regularized delta kernels: hat (Eq. 9) and Peskin 4-point (Eq. 10).
__device__ __forceinline__ double delta1(int kernel, double r) {
  const double a = fabs(r);
  if (kernel == kHat) return a < 1.0 ? 1.0 - a : 0.0;
  if (a <= 1.0) return 0.125 * (3.0 - 2.0 * a + sqrt(1.0 + 4.0 * a - 4.0 * a * a));
  if (a <= 2.0) return 0.125 * (5.0 - 2.0 * a - sqrt(-7.0 + 12.0 * a - 4.0 * a * a));
  return 0.0;
}

// A device-memory pointer the compiler cannot place by itself (one read
// from a descriptor) makes generic (flat) accesses, and a flat access also
// counts as an LDS operation: the next LDS wait or barrier of the wave then
// waits until a flat store has reached the cache, a long round trip beside
// a chip-wide stream.  Stores on the IB pass's late path go through this
// global-address-space view instead.
template <typename T>
using gmem = __attribute__((address_space(1))) T;
template <typename T>
__device__ __forceinline__ gmem<T> *to_global(T *p) {
  return (gmem<T> *)p;
}

// ---- fixed-order block reductions (wave64 shuffles, then LDS) ----
// A double moved across lanes by a DPP pattern (both 32-bit halves).
template <int CTRL>
__device__ __forceinline__ double dpp_f64(double v) {
  const unsigned long long b = (unsigned long long)__double_as_longlong(v);
  const int lo = __builtin_amdgcn_update_dpp(0, (int)(unsigned)b, CTRL, 0xF, 0xF, false);
  const int hi = __builtin_amdgcn_update_dpp(0, (int)(unsigned)(b >> 32), CTRL, 0xF, 0xF, false);
  return __longlong_as_double((long long)(((unsigned long long)(unsigned)hi << 32) | (unsigned)lo));
}
__device__ __forceinline__ double lane_f64(double v, int lane) {
  const unsigned long long b = (unsigned long long)__double_as_longlong(v);
  const unsigned lo = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)b, lane);
  const unsigned hi = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)(b >> 32), lane);
  return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}
// Wave64 sum and maximum with every lane active: within each row of 16
// lanes a fixed tree of lane exchanges (pairs, pairs of pairs, half-row
// mirror, row mirror; each step leaves the same value in both partners, as
// IEEE addition commutes), then the four row totals in a fixed order.
__device__ __forceinline__ double wave_sum(double v) {
  v += dpp_f64<0xB1>(v);   // quad_perm [1,0,3,2]
  v += dpp_f64<0x4E>(v);   // quad_perm [2,3,0,1]
  v += dpp_f64<0x141>(v);  // row_half_mirror
  v += dpp_f64<0x140>(v);  // row_mirror
  return (lane_f64(v, 0) + lane_f64(v, 16)) + (lane_f64(v, 32) + lane_f64(v, 48));
}
__device__ __forceinline__ double wave_max(double v) {
  v = fmax(v, dpp_f64<0xB1>(v));
  v = fmax(v, dpp_f64<0x4E>(v));
  v = fmax(v, dpp_f64<0x141>(v));
  v = fmax(v, dpp_f64<0x140>(v));
  return fmax(fmax(lane_f64(v, 0), lane_f64(v, 16)), fmax(lane_f64(v, 32), lane_f64(v, 48)));
}
// Sums a, b, c, d and maxima m1, m2 over the workgroup, each in a fixed
// order: wave totals, then the wave totals (one lane of wave 0 each) by the
// same wave tree.  The results are valid in the threads of wave 0.
// Threads at or past `nlive` must hold a = b = c = d = +0 and maxima that are
// 0 or held by a live thread as well (all values are non-negative): a wave
// with no live thread writes those totals without reducing them, which is
// what its tree would give.  On the IB pass's one compute unit the FP64
// wave reductions of sixteen waves compete for four SIMDs.
__device__ __forceinline__ void block_reduce6(double &a, double &b, double &c, double &d, double &m1,
                                              double &m2, double *red, int nlive) {
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6, nw = (blockDim.x + 63) >> 6;
  if (wv * 64 < nlive) {
    a = wave_sum(a); b = wave_sum(b); c = wave_sum(c); d = wave_sum(d);
    m1 = wave_max(m1); m2 = wave_max(m2);
  } else {
    a = 0.0; b = 0.0; c = 0.0; d = 0.0; m1 = 0.0; m2 = 0.0;
  }
  // (red is used once per pass, so nothing earlier needs a barrier here)
  if (lane == 0) {
    red[6 * wv] = a; red[6 * wv + 1] = b; red[6 * wv + 2] = c; red[6 * wv + 3] = d;
    red[6 * wv + 4] = m1; red[6 * wv + 5] = m2;
  }
  __syncthreads();
  if (wv == 0) {
    const bool in = lane < nw;
    const double *r = red + 6 * min(lane, nw - 1);
    a = wave_sum(in ? r[0] : 0.0);
    b = wave_sum(in ? r[1] : 0.0);
    c = wave_sum(in ? r[2] : 0.0);
    d = wave_sum(in ? r[3] : 0.0);
    m1 = wave_max(in ? r[4] : -1e300);
    m2 = wave_max(in ? r[5] : -1e300);
  }
}

// Exclusive prefix sum of cnt[0..n) into off[0..n], off[n] = total.  Each
// thread sums a contiguous chunk, chunk sums are scanned with wave shuffles
// and one pass over the wave totals.  wsum holds at least 33 ints.
__device__ __forceinline__ void block_scan(const int *cnt, int *off, int n, int *wsum) {
  const int nth = blockDim.x, lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int per = (n + nth - 1) / nth;
  const int b0 = min(n, threadIdx.x * per), b1 = min(n, b0 + per);
  int s = 0;
  for (int i = b0; i < b1; i++) s += cnt[i];
  int inc = s;
  for (int o = 1; o < 64; o <<= 1) {
    const int v = __shfl_up(inc, o, 64);
    if (lane >= o) inc += v;
  }
  if (lane == 63) wsum[wv] = inc;
  __syncthreads();
  if (threadIdx.x == 0) {
    int run = 0;
    for (int w = 0; w < (nth + 63) / 64; w++) {
      const int t = wsum[w];
      wsum[w] = run;
      run += t;
    }
    wsum[32] = run;
  }
  __syncthreads();
  int run = wsum[wv] + inc - s;
  for (int i = b0; i < b1; i++) { off[i] = run; run += cnt[i]; }
  if (threadIdx.x == 0) off[n] = wsum[32];
  __syncthreads();
}

// Per-marker tables are stored marker-fastest (entry q of marker k at
// q * nb + k), so that the 64 lanes of a wave, which handle 64 consecutive
// markers, read consecutive LDS words and hit distinct banks.
struct WsLayout {
  int nb, mn, ns;
  double *X, *Y, *Udx, *Udy, *wx, *wy;                           // table doubles
  int *ix0, *iy0, *nrow, *ra1, *rl1, *ra2, *off, *nxy, *noff, *nent, *ell, *S;  // table ints
  double *rhoX, *Fx, *Fy, *Ftx, *Fty, *lam, *dlt;                // per-step, markers
  void *stage;                                                   // DFC populations
  double *nrho, *nux, *nuy, *nW;                                 // per-step, nodes
  double *Ux, *Uy, *Bm;  // marker-space MDF: velocities at the markers, band matrix
  int bw;                // its half-width (0: the passes run on the support nodes)
  double *Fnx, *Fny, *pux, *puy;  // coupled MDF: unrelaxed forces, node velocities before a trial
  int *lmin, *lmax, *rmin, *rmax, *cnt, *ncnt, *nfill;  // construction scratch (per-step area)
};

__device__ __forceinline__ WsLayout carve(double *base, const BodyDesc &B) {
  const int nb = B.nb, ns = B.ns, mr = B.max_rows, mn = B.max_nodes;
  WsLayout L;
  L.nb = nb;
  L.mn = mn;
  L.ns = ns;
  double *p = base;
  L.X = p; p += nb; L.Y = p; p += nb; L.Udx = p; p += nb; L.Udy = p; p += nb;
  L.wx = p; p += nb * ns; L.wy = p; p += nb * ns;
  int *q = (int *)p;
  L.nrow = q; q += nb * ns; L.nxy = q; q += mn;
  L.ell = q; q += B.scheme != kDFC ? ell_width(ns) * mn : 0; L.S = q;
  q = (int *)(base + ws_tab_hot(B.scheme, nb, ns, mn));
  L.ix0 = q; q += nb; L.iy0 = q; q += nb;
  L.ra1 = q; q += mr; L.rl1 = q; q += mr; L.ra2 = q; q += mr; L.off = q; q += mr + 1;
  L.noff = q; q += mn + 1; L.nent = q;
  double *d = base + ws_tab_total(B.scheme, nb, ns, mr, mn);
  // arrays a scheme does not use alias the start of the per-step area (never
  // null, so that every pointer provably stays in the workspace's address
  // space and the LDS instantiation uses LDS instructions)
  L.rhoX = L.Fx = L.Fy = L.lam = L.dlt = L.nrho = L.nW = L.nux = L.nuy = d;
  L.Ux = L.Uy = L.Bm = d;
  L.Fnx = L.Fny = L.pux = L.puy = d;
  L.bw = 0;
  L.stage = (void *)d;
  if (B.scheme != kDFC) {
    L.rhoX = d; d += nb; L.Fx = d; d += nb; L.Fy = d; d += nb; L.Ftx = d; d += nb; L.Fty = d; d += nb;
    L.nrho = d; d += mn;
    L.nux = d; d += mn; L.nuy = d; d += mn;
    L.bw = B.mdf_band;
    const bool mk = B.mdf_band > 0 || B.mdf_coupled;
    L.Ux = d; d += mk ? nb : 0; L.Uy = d; d += mk ? nb : 0;
    if (B.mdf_coupled) {
      L.Fnx = d; d += nb; L.Fny = d; d += nb;
      L.pux = d; d += mn; L.puy = d; d += mn;
    }
    // the band overlays the node velocities, which the marker-space passes
    // no longer need once U^(1) is interpolated
    L.Bm = L.nux;
  } else {
    L.Ftx = d; d += nb; L.Fty = d; d += nb; L.lam = d; d += nb; L.dlt = d; d += 9 * nb;
    L.stage = (void *)d;  // 9 x mn populations of the stored type
    L.nW = d;             // overlays the staging area before it is filled
  }
  int *c = (int *)(base + ws_tab_total(B.scheme, nb, ns, mr, mn) + (B.scheme == kDFC ? 12 * nb : 5 * nb));
  L.lmin = c; c += mr; L.lmax = c; c += mr; L.rmin = c; c += mr; L.rmax = c; c += mr; L.cnt = c;
  c += mr;
  L.ncnt = c; c += mn; L.nfill = c;
  return L;
}

// Support node of stencil slot q = jy * ns + jx of marker k.  A marker's
// stencil row lies in one x-interval of its support row, so its nodes are
// consecutive in the compact numbering: the table keeps each stencil row's
// first node (nrow, marker-fastest) and adds jx.
__device__ __forceinline__ int NROW(const WsLayout &L, int k, int jy) { return L.nrow[jy * L.nb + k]; }
__device__ __forceinline__ int NIDX(const WsLayout &L, int k, int q) {
  const int sh = L.ns == 4 ? 2 : 1;
  return NROW(L, k, q >> sh) + (q & (L.ns - 1));
}
__device__ __forceinline__ double &WX(const WsLayout &L, int k, int j) { return L.wx[j * L.nb + k]; }
__device__ __forceinline__ double &WY(const WsLayout &L, int k, int j) { return L.wy[j * L.nb + k]; }
__device__ __forceinline__ double &DLT(const WsLayout &L, int k, int i) { return L.dlt[i * L.nb + k]; }

// Node velocities of the DFC pass, kept in the population staging area:
// node j's (ux, uy) as two doubles in slot j of the first planes (the bits of
// each double split over two planes of floats for the FP32 store), so that
// a thread writing node j only overwrites values of node j.
__device__ __forceinline__ void put_u(float *stg, int mn, int j, double ux, double uy) {
  uint32_t *w = (uint32_t *)stg;
  const uint64_t bx = (uint64_t)__double_as_longlong(ux), by = (uint64_t)__double_as_longlong(uy);
  w[j] = (uint32_t)bx;
  w[mn + j] = (uint32_t)(bx >> 32);
  w[2 * mn + j] = (uint32_t)by;
  w[3 * mn + j] = (uint32_t)(by >> 32);
}
__device__ __forceinline__ void put_u(double *stg, int mn, int j, double ux, double uy) {
  stg[j] = ux;
  stg[mn + j] = uy;
}
__device__ __forceinline__ void get_u(const float *stg, int mn, int j, double &ux, double &uy) {
  const uint32_t *w = (const uint32_t *)stg;
  ux = __longlong_as_double((long long)(((uint64_t)w[mn + j] << 32) | w[j]));
  uy = __longlong_as_double((long long)(((uint64_t)w[3 * mn + j] << 32) | w[2 * mn + j]));
}
__device__ __forceinline__ void get_u(const double *stg, int mn, int j, double &ux, double &uy) {
  ux = stg[j];
  uy = stg[mn + j];
}

// Marker loops run LPM lanes per marker (2, or 4 in the 1024-thread kernel
// with Peskin 4-point): lanes m*LPM .. m*LPM+LPM-1 of a wave share marker
// k, lane h sums the stencil rows [h NS/LPM, (h+1) NS/LPM) and group_sum
// adds the partial sums of the group with DPP quad permutations (lanes
// 0<->1, 2<->3, then 0,1<->2,3 of every quad).  IEEE addition commutes, so
// every lane of a group holds the same total.  All lanes of a group are
// always active together (the loops over LPM nb entries step by a block
// size that is a multiple of LPM).
template <int LPM>
__device__ __forceinline__ double group_sum(double v) {
  if (LPM >= 2) v += dpp_f64<0xB1>(v);  // quad_perm [1,0,3,2]
  if (LPM >= 4) v += dpp_f64<0x4E>(v);  // quad_perm [2,3,0,1]
  return v;
}

// Partial interp2 of the packed node velocities (see group_sum).
template <int NS, int LPM, typename T>
__device__ __forceinline__ void interp_packed_u(const WsLayout &L, int k, int h, const T *stg, int mn,
                                                double &oa, double &ob) {
  constexpr int R = NS / LPM;
  double a = 0.0, b = 0.0;
#pragma unroll
  for (int r = 0; r < R; r++) {
    const int jy = h * R + r;
    double ra = 0.0, rb = 0.0;
#pragma unroll
    for (int jx = 0; jx < NS; jx++) {
      double ux, uy;
      get_u(stg, mn, NROW(L, k, jy) + jx, ux, uy);
      const double w = WX(L, k, jx);
      ra += ux * w;
      rb += uy * w;
    }
    a += ra * WY(L, k, jy);
    b += rb * WY(L, k, jy);
  }
  oa = group_sum<LPM>(a);
  ob = group_sum<LPM>(b);
}

// Spreading by gather: node j sums v_k D_h(x_j - X_k) over the markers
// covering it, in increasing marker order.
template <int NS>
__device__ __forceinline__ double node_weight(const WsLayout &L, int kq) {
  const int k = kq >> 4, q = kq & 15;
  return WX(L, k, q % NS) * WY(L, k, q / NS);
}

// Entries of the node-fastest lists: (marker << 4) | stencil slot, with
// kEllPad marking a padding slot (it repeats a real entry of the node, or
// entry 0, and takes weight 0) and kEllMore on the last slot of a node whose
// list continues in the CSR list (denser marker spacings).
constexpr int kEllPad = int(0x80000000u);
constexpr int kEllMore = 0x40000000;

// Calls f(k, w) for the markers k covering node j, in increasing marker
// order: the fixed-width slots first (one load each, at consecutive
// addresses for consecutive nodes; padding adds w = 0, which leaves every
// sum unchanged), then, rarely, the rest of the CSR list.
template <int NS, typename F>
__device__ __forceinline__ void for_node_entries(const WsLayout &L, int j, F &&f) {
  constexpr int U = NS == 4 ? 6 : 3;
  int kq[U];
#pragma unroll
  for (int u = 0; u < U; u++) kq[u] = L.ell[u * L.mn + j];
#pragma unroll
  for (int u = 0; u < U; u++) {
    const int v = kq[u] & ~(kEllPad | kEllMore);
    const double w = node_weight<NS>(L, v);
    f(v >> 4, kq[u] < 0 ? 0.0 : w);
  }
  if (kq[U - 1] & kEllMore) {
    for (int e = L.noff[j] + U; e < L.noff[j + 1]; e++) {
      const int q = L.nent[e];
      f(q >> 4, node_weight<NS>(L, q));
    }
  }
}

// The same from the CSR list alone (DFC), the weights formed on the fly.
template <int NS, typename F>
__device__ __forceinline__ void for_node_entries_csr(const WsLayout &L, int j, F &&f) {
  constexpr int U = NS == 4 ? 6 : 3;
  const int e0 = L.noff[j], e1 = L.noff[j + 1];
  int kq[U];
#pragma unroll
  for (int u = 0; u < U; u++) kq[u] = L.nent[min(e0 + u, e1 - 1)];
#pragma unroll
  for (int u = 0; u < U; u++) f(kq[u] >> 4, e0 + u < e1 ? node_weight<NS>(L, kq[u]) : 0.0);
  for (int e = e0 + U; e < e1; e++) {
    const int q = L.nent[e];
    f(q >> 4, node_weight<NS>(L, q));
  }
}

template <int NS>
__device__ __forceinline__ void gather2(const WsLayout &L, int j, const double *va,
                                        const double *vb, double &oa, double &ob) {
  double a = 0.0, b = 0.0;
  for_node_entries<NS>(L, j, [&](int k, double w) {
    a += va[k] * w;
    b += vb[k] * w;
  });
  oa = a;
  ob = b;
}

// Interpolation of node arrays to marker k (Eq. 7): rows in x weighted by
// w_x, then by w_y; lane h of the marker's group takes NS / LPM of the rows
// (see group_sum).
template <int NS, int LPM>
__device__ __forceinline__ double interp1(const WsLayout &L, int k, int h, const double *nv) {
  constexpr int R = NS / LPM;
  double acc = 0.0;
#pragma unroll
  for (int r = 0; r < R; r++) {
    const int jy = h * R + r;
    double row = 0.0;
    const int j0 = NROW(L, k, jy);
#pragma unroll
    for (int jx = 0; jx < NS; jx++) row += nv[j0 + jx] * WX(L, k, jx);
    acc += row * WY(L, k, jy);
  }
  return group_sum<LPM>(acc);
}

template <int NS, int LPM>
__device__ __forceinline__ void interp2(const WsLayout &L, int k, int h, const double *na,
                                        const double *nb_, double &oa, double &ob) {
  constexpr int R = NS / LPM;
  double a = 0.0, b = 0.0;
#pragma unroll
  for (int r = 0; r < R; r++) {
    const int jy = h * R + r;
    double ra = 0.0, rb = 0.0;
#pragma unroll
    for (int jx = 0; jx < NS; jx++) {
      const int j = NROW(L, k, jy) + jx;
      const double w = WX(L, k, jx);
      ra += na[j] * w;
      rb += nb_[j] * w;
    }
    a += ra * WY(L, k, jy);
    b += rb * WY(L, k, jy);
  }
  oa = group_sum<LPM>(a);
  ob = group_sum<LPM>(b);
}

// Steps 2-3: markers, weights and the compact support.  Returns the node
// count, or -1 with error flags in ish[0].
__device__ __forceinline__ int build_tables(const CaseDesc &c, const BodyDesc &B, const WsLayout &L, double xc,
                            double yc, double udx, double udy, double udo, int ylo, int *ish,
                            int *wsum) {
  const int tid = threadIdx.x, nth = blockDim.x;
  const int nb = B.nb, ns = B.ns, s = ns / 2, nx = c.nx, ny = c.ny;
  for (int r = tid; r < B.max_rows; r += nth) {
    L.lmin[r] = 1 << 30; L.lmax[r] = -1; L.rmin[r] = 1 << 30; L.rmax[r] = -1;
  }
  __syncthreads();
  for (int k = tid; k < nb; k += nth) {
    const double X = xc + B.radius * B.cos_t[k];
    const double Y = yc + B.radius * B.sin_t[k];
    L.X[k] = X;
    L.Y[k] = Y;
    L.Udx[k] = udx - udo * (Y - yc);
    L.Udy[k] = udy + udo * (X - xc);
    const int ix0 = (int)floor(X) - (s - 1), iy0 = (int)floor(Y) - (s - 1);
    L.ix0[k] = ix0;
    L.iy0[k] = iy0;
    if (ix0 < 0 || iy0 < 0 || ix0 + ns - 1 > nx - 1 || iy0 + ns - 1 > ny - 1) atomicOr(&ish[0], kFlagRange);
    for (int j = 0; j < ns; j++) {
      WX(L, k, j) = delta1(B.kernel, (double)(ix0 + j) - X);
      WY(L, k, j) = delta1(B.kernel, (double)(iy0 + j) - Y);
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
  if (ish[0]) return -1;
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
  block_scan(L.cnt, L.off, B.max_rows, wsum);
  const int S = L.off[B.max_rows];
  if (S > B.max_nodes) {
    if (tid == 0) ish[0] |= kFlagCapacity;
    __syncthreads();
    return -1;
  }
  for (int j = tid; j < S; j += nth) {
    int lo = 0, hi = B.max_rows - 1;
    while (lo < hi) {
      const int mid = (lo + hi + 1) >> 1;
      if (L.off[mid] <= j) lo = mid; else hi = mid - 1;
    }
    const int r = lo, loc = j - L.off[r];
    const int x = loc < L.rl1[r] ? L.ra1[r] + loc : L.ra2[r] + (loc - L.rl1[r]);
    L.nxy[j] = x | ((ylo + r) << 16);
    L.ncnt[j] = 0;
  }
  for (int k = tid; k < nb; k += nth) {
    for (int jy = 0; jy < ns; jy++) {
      const int r = L.iy0[k] + jy - ylo;
      const int x = L.ix0[k];
      const int loc = (x >= L.ra1[r] && x < L.ra1[r] + L.rl1[r]) ? x - L.ra1[r] : L.rl1[r] + x - L.ra2[r];
      L.nrow[jy * nb + k] = L.off[r] + loc;
    }
  }
  __syncthreads();
  // node -> marker lists (CSR): count, scan, fill, then sort each short list
  // by marker index so the gather order does not depend on atomic timing
  const int nq = ns * ns;
  for (int e = tid; e < nb * nq; e += nth) {
    const int q = e / nb, k = e - q * nb;  // e = q * nb + k
    atomicAdd(&L.ncnt[NIDX(L, k, q)], 1);
  }
  __syncthreads();
  block_scan(L.ncnt, L.noff, S, wsum);
  for (int j = tid; j < S; j += nth) L.nfill[j] = L.noff[j];
  __syncthreads();
  for (int e = tid; e < nb * nq; e += nth) {
    const int q = e / nb, k = e - q * nb;  // e = q * nb + k
    const int pos = atomicAdd(&L.nfill[NIDX(L, k, q)], 1);
    L.nent[pos] = (k << 4) | q;
  }
  __syncthreads();
  const int uw = ell_width(ns), mn = B.max_nodes;
  for (int j = tid; j < S; j += nth) {
    const int e0 = L.noff[j], e1 = L.noff[j + 1];
    for (int a = e0 + 1; a < e1; a++) {
      const int v = L.nent[a];
      int b = a - 1;
      while (b >= e0 && L.nent[b] > v) { L.nent[b + 1] = L.nent[b]; b--; }
      L.nent[b + 1] = v;
    }
    // the node-fastest copy of the first entries (DF/MDF)
    const int cnt = e1 - e0;
    for (int u = 0; u < (B.scheme != kDFC ? uw : 0); u++) {
      int v = u < cnt ? L.nent[e0 + u] : ((cnt > 0 ? L.nent[e1 - 1] : 0) | kEllPad);
      if (u == uw - 1 && cnt > uw) v |= kEllMore;
      L.ell[u * mn + j] = v;
    }
    if (cnt > uw) atomicOr(&ish[5], 1);
  }
  if (tid == 0) L.S[0] = S;
  __syncthreads();
  return S;
}

// Copies n doubles with the threads from `first` on (16-byte copies, four
// loads in flight per thread before the stores; workspace bases are 16-byte
// aligned).
__device__ __forceinline__ void copy_doubles(double *dst, const double *src, int n, int first = 0) {
  const int n2 = n >> 1;
  const double2 *s2 = (const double2 *)src;
  double2 *d2 = (double2 *)dst;
  const int nth = blockDim.x - first;
  int i = (int)threadIdx.x - first;
  if (i < 0) return;
  for (; i + 3 * nth < n2; i += 4 * nth) {
    const double2 a = s2[i], b = s2[i + nth], c = s2[i + 2 * nth], d = s2[i + 3 * nth];
    d2[i] = a;
    d2[i + nth] = b;
    d2[i + 2 * nth] = c;
    d2[i + 3 * nth] = d;
  }
  for (; i < n2; i += nth) d2[i] = s2[i];
  if ((n & 1) && (int)threadIdx.x == first) dst[n - 1] = src[n - 1];
}

// Largest value of r over the workgroup (every thread returns it).
__device__ __forceinline__ double block_max(double r, double *red) {
  r = wave_max(r);
  __syncthreads();
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = r;
  __syncthreads();
  double m = red[0];
  for (int w = 1; w < (int)(blockDim.x >> 6); w++) m = fmax(m, red[w]);
  return m;
}

// Coupled MDF: the workgroups of a case's bodies publish their residuals of
// one round and take the largest over the case.  Thread 0 stores its value
// in the round's slot (rounds alternate between two slots: a workgroup can
// only start round e + 2 after every workgroup has counted itself into
// round e + 1, by which time round e's slot has been read), counts itself in
// with a release, and waits with acquire loads, bounded to about 2 s, until
// every body of the case has counted itself into this round.  On expiry the
// body is flagged and the exchange returns a NaN, which ends its iteration;
// a body that failed before its passes counts itself into every round at
// once and leaves a NaN, which the exchange passes on.
constexpr int kExchangeSpins = 1 << 22;
__device__ __forceinline__ double case_exchange_max(CaseState *cs, int body, int nbc, int round,
                                                    double r, double *bsh_x, int *flag) {
  if (threadIdx.x == 0) {
    const int slot = round & 1;
    __hip_atomic_store(&cs->xr[slot][body], r, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    __hip_atomic_fetch_add(&cs->xcnt, 1, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
    const int target = (round + 1) * nbc;
    int spins = 0;
    while (__hip_atomic_load(&cs->xcnt, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT) < target &&
           spins < kExchangeSpins) {
      __builtin_amdgcn_s_sleep(8);
      spins++;
    }
    double m = r;
    if (spins >= kExchangeSpins) {
      m = __builtin_nan("");
      *flag = 1;
    } else {
      for (int b = 0; b < nbc; b++) {
        const double v = __hip_atomic_load(&cs->xr[slot][b], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        m = v != v ? v : fmax(m, v);
        if (m != m) break;
      }
    }
    *bsh_x = m;
  }
  __syncthreads();
  const double m = *bsh_x;
  __syncthreads();
  return m;
}

// Bounded wait of thread 0 until the hold-rectangle workgroups of a fused
// step have all counted themselves (they have read and cleared the IB
// force); false if they did not within the spin limit.
constexpr int kHoldSpins = 1 << 22;
__device__ __forceinline__ bool hold_wait(CaseState *cs, int nhold) {
  int spins = 0;
  while (__hip_atomic_load(&cs->hold_seen, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT) < nhold &&
         spins < kHoldSpins) {
    __builtin_amdgcn_s_sleep(4);
    spins++;
  }
  return spins < kHoldSpins;
}

// The tiles of a fused step wait here until the IB pass of the launch has
// read its kinematics and copied its cached tables from device memory
// (CaseState::gate == seq), so that those dependent loads do not queue
// behind the tiles' streaming.  A schedule, not a dependency: after the
// spin limit the workgroup goes ahead anyway.
constexpr int kGateSpins = 1 << 16;
__device__ __forceinline__ void gate_wait(const CaseState *cs, int seq) {
  if (threadIdx.x == 0) {
    int spins = 0;
    while (__hip_atomic_load(&cs->gate, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != seq &&
           spins < kGateSpins) {
      __builtin_amdgcn_s_sleep(16);
      spins++;
    }
  }
  __syncthreads();
}
__device__ __forceinline__ void gate_open(CaseState *cs, int seq) {
  __hip_atomic_store(&cs->gate, seq, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Bounded wait of thread 0 until the source workgroups of a fused step have
// all staged their pushes; false if they did not within the spin limit.
__device__ __forceinline__ bool src_wait(CaseState *cs, int nsrc) {
  int spins = 0;
  while (__hip_atomic_load(&cs->src_seen, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT) < nsrc &&
         spins < kHoldSpins) {
    __builtin_amdgcn_s_sleep(2);
    spins++;
  }
  return spins < kHoldSpins;
}

// FAST: the 1024-thread instance for DF/MDF bodies with an LDS workspace
// and gather spreading (no DFC or atomic-scatter code, so that it fits 128
// VGPRs); marker loops then run one lane per stencil row.
// SELF_COL >= 0 (fused steps, a fixed body): the post-stream populations of
// the support nodes are not read from the lattice, which the rest of the
// launch is still writing, but from B.pstage, where the launch's nsrc
// source workgroups (fused_src) have staged them; the pass writes the new
// force only after the nhold hold-rectangle workgroups have read the
// previous one.
template <typename T, bool LDS, int NS, bool FAST, int SELF_COL = -1>
__device__ __forceinline__ void body_step(const CaseDesc &c, const BodyDesc &B, int64_t step, int cur,
                                          double *dyn, int spread_mode, double *red, int *ish,
                                          double *bsh, int nhold = 0, int seq = 0, int nsrc = 0) {
  constexpr int LPM = FAST ? NS : 2;
  const int tid = threadIdx.x, nth = blockDim.x;
  BodyState *bs = B.state;
  const int nb = B.nb;
  constexpr int ns = NS;
  const bool shift = sizeof(T) == 4;
  const double rho0 = c.rho0;
  const int nx = c.nx;
  const uint32_t plane = (uint32_t)c.plane;
  // post-stream populations of this step (the IB pass runs after the
  // collide-stream into lattice cur ^ 1)
  const T *fpop = (const T *)c.f[cur ^ 1];
  T *fpop_w = (T *)c.f[cur ^ 1];

  // A fixed body of the 1024-thread instance copies the hot part of its
  // cached tables with waves 1.. while thread 0 advances the kinematics
  // (wave 0 issues no copy loads for its kinematics loads to queue behind).
  // Before the cache is first filled this copies stale words, which the
  // table build below overwrites (the barrier after the kinematics orders
  // the two).
  if (FAST && B.motion == kFixed) copy_doubles(dyn, B.tab_cache, B.ws_tab_hot, 64);

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
    } else if (B.motion == kFree && B.integrator == kEulerA1) {
      // Euler-explicit update of Eq. (A1) from the force of the last step:
      // v^(n+1) = (1 + r) v^n - r v^(n-1) + (F^n + F_g)/m_s with r = m_f/m_s
      // (0 without internal mass); the rotation with the rigid interior's
      // angular-momentum increment, I_f/I_s = m_f/m_s, in both arms (the
      // internal-mass switch acts on the translation only); the position by
      // the new velocity.
      const double r = B.internal_mass == kImFeng ? B.mf / B.ms : 0.0;
      const double q = B.mf / B.ms;
      const double fgx = (B.ms - B.mf) * c.grav_x;
      const double fgy = (B.ms - B.mf) * c.grav_y;
      vhx = (1.0 + r) * bs->vx - r * bs->vpx + (bs->fhx + fgx) / B.ms;
      vhy = (1.0 + r) * bs->vy - r * bs->vpy + (bs->fhy + fgy) / B.ms;
      omh = (1.0 + q) * bs->om - q * bs->omp + bs->torque / B.Is;
      bs->vpx = bs->vx;
      bs->vpy = bs->vy;
      bs->omp = bs->om;
      bs->dimx = 0.0;
      bs->dimy = 0.0;
      xc += vhx;
      yc += vhy;
    } else if (B.motion == kFree) {
      // Eq. (23) first half-kick and drift, with the internal-mass force of
      // Eq. (A3) held over the step and the net gravity of Eq. (22).
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
    // Rigid-body velocity the markers are driven to: the one just set, but
    // under Velocity-Verlet the last full-step v^n, Omega^n (the half-step
    // values only advance the position).  With the half-step values the
    // torque-only rotation feeds back on itself by a factor -I_f,eff/I_s per
    // step, which exceeds one near neutral buoyancy.
    const bool verlet = B.motion == kFree && B.integrator != kEulerA1;
    bsh[13] = verlet ? bs->vx : vhx;
    bsh[14] = verlet ? bs->vy : vhy;
    bsh[15] = verlet ? bs->om : omh;
    bs->xc = xc; bs->yc = yc;
    bs->vhx = vhx; bs->vhy = vhy; bs->omh = omh;
    bsh[0] = xc; bsh[1] = yc; bsh[2] = vhx; bsh[3] = vhy; bsh[4] = omh;
    // state the final update needs, kept on chip so that it is not read
    // back from device memory at the end of the pass
    bsh[5] = B.motion == kFree ? bs->dimx : 0.0;
    bsh[6] = B.motion == kFree ? bs->dimy : 0.0;
    ish[0] = 0;
    ish[1] = bs->tables_valid;
    ish[2] = bs->lambda_valid;
    ish[3] = bs->flags;
    ish[4] = bs->tables_full;
    ish[5] = 0;  // set by build_tables when a node's list outgrows its fixed-width copy
    ish[6] = 0;  // set when the coupled-MDF workgroups of the case fail to meet
  }
  if (tid == 64) {
    // what the end of the pass needs from the descriptors, staged on chip
    // beside the kinematics (the pass's stores to device memory would
    // otherwise make the serial tail load them again)
    ish[10] = B.scheme == kDFC ? 0 : 1;
    ish[11] = B.scheme == kDFC ? 0 : (B.scheme == kDF ? 1 : B.mdf_iters);
    ish[12] = B.motion;
    ish[13] = B.scheme;
    ish[14] = c.ny;
    ish[15] = B.integrator;
    bsh[7] = __longlong_as_double((long long)(B.history + (step % B.hist_cap) * kHistCols));
    bsh[17] = __longlong_as_double((long long)B.markers_out);
    bsh[8] = B.ms;
    bsh[9] = (B.ms - B.mf) * c.grav_x;
    bsh[10] = (B.ms - B.mf) * c.grav_y;
    bsh[11] = B.Is;
    bsh[12] = B.radius;
  }
  __syncthreads();
  // the centre for the tables; the later uses read the kinematics from bsh
  // again, so that no register holds them through the whole pass
  const double xc = bsh[0], yc = bsh[1];
  constexpr bool in_lds = LDS;
  double *base = LDS ? dyn : B.ws;
  const WsLayout L = carve(base, B);
  const int ylo = (int)floor(yc - B.radius) - ns;
  const bool fixed = B.motion == kFixed;

  // ---- 2-3. tables: cached for fixed bodies
  int S;
  if (fixed && ish[1]) {
    // a DF/MDF step without long node lists reads only the hot part (already
    // copied by the 1024-thread instance)
    if (in_lds && (ish[4] || !FAST)) copy_doubles(base, B.tab_cache, ish[4] ? B.ws_tab : B.ws_tab_hot);
    __syncthreads();
    S = L.S[0];
  } else {
    S = build_tables(c, B, L, xc, yc, bsh[13], bsh[14], bsh[15], ylo, ish, ish + 16);
    if (S < 0) {
      if (tid == 0) {
        const int f = ish[3] | ish[0];
        bs->flags = f;
        bs->box_valid = 0;
        ish[50] = f;
        ish[51] = 0;
        if (B.scheme == kMDF && B.mdf_coupled) {
          // the other bodies of a coupled case would wait for this one:
          // leave a NaN residual and count this body into every round
          const int body = SELF_COL >= 0 ? 0 : (int)(&B - c.bodies);
          const double nan = __builtin_nan("");
          __hip_atomic_store(&c.state->xr[0][body], nan, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
          __hip_atomic_store(&c.state->xr[1][body], nan, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
          __hip_atomic_fetch_add(&c.state->xcnt, 1 << 24, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
        }
      }
      return;
    }
    if (fixed) {
      if (in_lds) copy_doubles(B.tab_cache, base, B.ws_tab);
      if (tid == 0) {
        bs->tables_full = (B.scheme == kDFC || ish[5]) ? 1 : 0;
        bs->tables_valid = 1;
      }
    }
  }
  // fused step: kinematics and tables are in LDS, the tiles may stream.  The
  // pass's remaining loads from device memory (the staged support
  // populations) then run beside the stream: opening the gate here rather
  // than after them shortens the FP32 step by about 2 us (28.1 against 30.6
  // us on the 2000x800 cylinder; 28.7 with the gate at the kinematics
  // barrier, 28.7 after the source workgroups' count).
  if constexpr (SELF_COL >= 0)
    if (tid == 0) gate_open(c.state, seq);
  if (B.udes == kUdTaylorGreen) {
    // IB-LBM mode of the Taylor-Green check (App. D.1): the fixed markers are
    // driven to the decaying vortex of Eq. D1 at t_{n+1}, origin at node (0, 0)
    const double k = B.tg_k;
    const double amp = B.tg_u0 * exp(-2.0 * B.tg_nu * k * k * (double)(step + 1));
    for (int m = tid; m < nb; m += nth) {
      const double X = L.X[m], Y = L.Y[m];
      L.Udx[m] = -amp * cos(k * X) * sin(k * Y);
      L.Udy[m] = amp * sin(k * X) * cos(k * Y);
    }
    __syncthreads();
  }
  const double ds = B.ds;
  double fsum_x = 0, fsum_y = 0, tq = 0, resmax = 0;

  if (FAST || B.scheme != kDFC) {
    // ---- 4a. DF (one pass, omega 1) / MDF (N passes, omega_MDF)
    // moments of the post-stream populations at the support nodes; the
    // loads of UM nodes per thread are issued before any is used (one round
    // trip to device memory covers up to UM * 512 nodes)
    constexpr int UM = FAST ? 1 : (sizeof(T) == 4 ? 3 : 2);
    T *const stg = (T *)B.pstage;
    if constexpr (SELF_COL >= 0) {
      // the launch's source workgroups have staged the support's pushes
      if (tid == 0) {
        if (src_wait(c.state, nsrc)) ish[56] |= 1;
        else ish[3] |= kFlagExchange;
      }
      __syncthreads();
    }
    for (int j0 = tid; j0 < S; j0 += UM * nth) {
      T v[UM][9];
#pragma unroll
      for (int u = 0; u < UM; u++) {
        const int j = j0 + u * nth;
        if (j < S) {
          if constexpr (SELF_COL >= 0) {
#pragma unroll
            for (int i = 0; i < 9; i++) v[u][i] = stg[i * B.max_nodes + j];
          } else {
            const int x = L.nxy[j] & 0xffff, y = L.nxy[j] >> 16;
            const T *fp = fpop + pop_node(x, y, c.nseg);
#pragma unroll
            for (int i = 0; i < 9; i++) v[u][i] = fp[i * kSeg];
          }
        }
      }
#pragma unroll
      for (int u = 0; u < UM; u++) {
        const int j = j0 + u * nth;
        if (j >= S) continue;
        double sm = 0, jx = 0, jy = 0;
#pragma unroll
        for (int i = 0; i < 9; i++) {
          const double w = (double)v[u][i] + (shift ? c_w[i] * rho0 : 0.0);
          sm += w;
          jx += w * c_exi[i];
          jy += w * c_eyi[i];
        }
        L.nrho[j] = sm;
        L.nux[j] = jx / sm;
        L.nuy[j] = jy / sm;
      }
    }
    __syncthreads();
    T *frc = (T *)c.force;
    double *accx = B.acc, *accy = B.acc + B.max_nodes;
    if (B.scheme == kDF) {
      // DF, Eq. (11): one interpolation of u*, F_L = 2 rho(X) (U_d - U)
      for (int kk = tid; kk < LPM * nb; kk += nth) {
        const int k = kk / LPM, h = kk % LPM;
        const double rX = interp1<NS, LPM>(L, k, h, L.nrho);
        double Ux, Uy;
        interp2<NS, LPM>(L, k, h, L.nux, L.nuy, Ux, Uy);
        if (h == 0) {
          L.rhoX[k] = rX;
          L.Ftx[k] = 2.0 * rX * (L.Udx[k] - Ux);
          L.Fty[k] = 2.0 * rX * (L.Udy[k] - Uy);
        }
      }
    } else if (B.mdf_coupled) {
      // Coupled multi-body MDF (Sec. 2.5.2, the two-particle path), on the
      // support nodes.  Every trial pass spreads c omega_0 F^(n), omega_0 =
      // min(omega_MDF, 0.8), into the node velocities, re-interpolates them
      // and takes the residual R' of all the case's markers (the bodies'
      // workgroups exchange theirs); R' > 1.2 R rejects the trial (the node
      // velocities return to their saved state) and halves c, ending the
      // iteration once c reaches 1/8, else the trial is a pass: F_total takes
      // it and the next F^(n) comes from the new interpolation.  The
      // iteration ends after mdf_iters passes, or, with a tolerance, once at
      // least mdf_nmin passes are kept and R < tol.  Every workgroup of the
      // case takes the same decisions from the same exchanged values.
      const int N = B.mdf_iters;
      const double tol = B.mdf_tol;
      const int nmin = tol > 0.0 ? B.mdf_nmin : N;
      const double om0 = fmin(B.omega_mdf, 0.8);
      // (a fused step's descriptor is a copy in the kernel arguments: its
      // single body is body 0)
      const int body = SELF_COL >= 0 ? 0 : (int)(&B - c.bodies), nbc = c.nbodies;
      CaseState *cs = c.state;
      int round = 0;
      // pass 1's interpolation of u* and rho(X): errors, unrelaxed forces
      double rloc = 0.0;
      for (int kk = tid; kk < LPM * nb; kk += nth) {
        const int k = kk / LPM, h = kk % LPM;
        const double rX = interp1<NS, LPM>(L, k, h, L.nrho);
        double Ux, Uy;
        interp2<NS, LPM>(L, k, h, L.nux, L.nuy, Ux, Uy);
        if (h == 0) {
          const double ex = L.Udx[k] - Ux, ey = L.Udy[k] - Uy;
          L.rhoX[k] = rX;
          L.Fnx[k] = 2.0 * rX * ex;
          L.Fny[k] = 2.0 * rX * ey;
          L.Ftx[k] = 0.0;
          L.Fty[k] = 0.0;
          rloc = fmax(rloc, sqrt(ex * ex + ey * ey));
        }
      }
      double R = case_exchange_max(cs, body, nbc, round++, block_max(rloc, red), &bsh[16], &ish[6]);
      for (int j = tid; j < S; j += nth) L.nrho[j] = ds / (2.0 * L.nrho[j]);
      __syncthreads();
      double cf = 1.0;
      int kept = 0;
      bool stop = R != R;
      while (!stop && kept < N && !(tol > 0.0 && kept >= nmin && R < tol)) {
        for (int j = tid; j < S; j += nth) {
          L.pux[j] = L.nux[j];
          L.puy[j] = L.nuy[j];
        }
        for (;;) {
          const double w = cf * om0;
          for (int k = tid; k < nb; k += nth) {
            L.Fx[k] = w * L.Fnx[k];
            L.Fy[k] = w * L.Fny[k];
          }
          __syncthreads();
          for (int j = tid; j < S; j += nth) {
            double sx, sy;
            gather2<NS>(L, j, L.Fx, L.Fy, sx, sy);
            L.nux[j] = L.pux[j] + sx * L.nrho[j];
            L.nuy[j] = L.puy[j] + sy * L.nrho[j];
          }
          __syncthreads();
          rloc = 0.0;
          for (int kk = tid; kk < LPM * nb; kk += nth) {
            const int k = kk / LPM, h = kk % LPM;
            double Ux, Uy;
            interp2<NS, LPM>(L, k, h, L.nux, L.nuy, Ux, Uy);
            if (h == 0) {
              const double ex = L.Udx[k] - Ux, ey = L.Udy[k] - Uy;
              L.Ux[k] = ex;
              L.Uy[k] = ey;
              rloc = fmax(rloc, sqrt(ex * ex + ey * ey));
            }
          }
          const double Rt =
              case_exchange_max(cs, body, nbc, round++, block_max(rloc, red), &bsh[16], &ish[6]);
          if (Rt != Rt) {
            stop = true;
            break;
          }
          if (!(Rt > 1.2 * R)) {
            for (int k = tid; k < nb; k += nth) {
              L.Ftx[k] += L.Fx[k];
              L.Fty[k] += L.Fy[k];
              L.Fnx[k] = 2.0 * L.rhoX[k] * L.Ux[k];
              L.Fny[k] = 2.0 * L.rhoX[k] * L.Uy[k];
            }
            kept++;
            R = Rt;
            __syncthreads();
            break;
          }
          // rejected: back to the velocities before the trial
          for (int j = tid; j < S; j += nth) {
            L.nux[j] = L.pux[j];
            L.nuy[j] = L.puy[j];
          }
          __syncthreads();
          cf *= 0.5;
          if (cf <= 0.125) {
            stop = true;
            break;
          }
        }
      }
      resmax = R;
      if (tid == 0) ish[11] = kept;
      __syncthreads();
    } else if (FAST && L.bw > 0) {
      // MDF, Eq. (12)-(14), in marker space.  Interpolating the updated node
      // velocities of Eq. (14) gives U^(n+1) = U^(n) + omega B F^(n) with
      // B_kl = sum_x D_h(x - X_k) D_h(x - X_l) ds / (2 rho(x)), the same
      // iteration up to rounding.  B couples only markers whose stencils
      // share a node, so it is a band of half-width bw around the diagonal
      // (marker indices wrap around the circle); it is built once per step
      // and each pass is a short dot product per marker instead of an
      // interpolation and a spreading over the support nodes.  The node
      // velocities are not updated; the velocity after the passes, which the
      // slip needs, is U at the markers.
      const int N = B.mdf_iters;
      const double om = B.omega_mdf;
      const double tol = B.mdf_tol;
      const bool adapt = tol > 0.0;
      const int bw = L.bw;
      // U^(1) and rho(X) from the force-free post-stream moments
      for (int kk = tid; kk < LPM * nb; kk += nth) {
        const int k = kk / LPM, h = kk % LPM;
        const double rX = interp1<NS, LPM>(L, k, h, L.nrho);
        double Ux, Uy;
        interp2<NS, LPM>(L, k, h, L.nux, L.nuy, Ux, Uy);
        if (h == 0) {
          L.rhoX[k] = rX;
          L.Ux[k] = Ux;
          L.Uy[k] = Uy;
        }
      }
      __syncthreads();
      for (int j = tid; j < S; j += nth) L.nrho[j] = ds / (2.0 * L.nrho[j]);
      __syncthreads();
      // B: one thread per (k, l = k + d), 0 <= d <= bw, over the nodes the
      // two stencils share (stencil origins from the node coordinates),
      // rows outer and columns inner.  B is symmetric: row k keeps its
      // entries d = 0..bw, and B_(k, k-d) is read as entry d of row k - d.
      // It overlays the node velocities, read for the last time above.
      for (int t = tid; t < nb * (bw + 1); t += nth) {
        const int k = t / (bw + 1), dd = t - k * (bw + 1);
        const int l = k + dd < nb ? k + dd : k + dd - nb;
        const int xyk = L.nxy[NROW(L, k, 0)], xyl = L.nxy[NROW(L, l, 0)];
        const int dx = (xyl & 0xffff) - (xyk & 0xffff), dy = (xyl >> 16) - (xyk >> 16);
        double b = 0.0;
        if (dx > -ns && dx < ns && dy > -ns && dy < ns) {
#pragma unroll
          for (int jy = 0; jy < ns; jy++) {
            const int ly = jy - dy;
            if (ly < 0 || ly >= ns) continue;
            const int r0 = NROW(L, k, jy);
            double row = 0.0;
#pragma unroll
            for (int jx = 0; jx < ns; jx++) {
              const int lx = jx - dx;
              if (lx < 0 || lx >= ns) continue;
              row += WX(L, k, jx) * WX(L, l, lx) * L.nrho[r0 + jx];
            }
            b += WY(L, k, jy) * WY(L, l, ly) * row;
          }
        }
        L.Bm[k * (bw + 1) + dd] = b;
      }
      __syncthreads();
      double rprev = 0.0;
      for (int n = 1; n <= N; n++) {
        // F^(n) = 2 rho(X) (U_d - U^(n)), relaxed: omega F^(n)
        double rloc = 0.0;
        for (int k = tid; k < nb; k += nth) {
          const double ex = L.Udx[k] - L.Ux[k], ey = L.Udy[k] - L.Uy[k];
          const double rX = L.rhoX[k];
          const double Fx = 2.0 * rX * ex, Fy = 2.0 * rX * ey;
          L.Fx[k] = om * Fx;
          L.Fy[k] = om * Fy;
          if (!adapt) {
            L.Ftx[k] = (n == 1 ? 0.0 : L.Ftx[k]) + om * Fx;
            L.Fty[k] = (n == 1 ? 0.0 : L.Fty[k]) + om * Fy;
          }
          rloc = fmax(rloc, sqrt(ex * ex + ey * ey));
        }
        if (!adapt && n == N) resmax = rloc;
        if (adapt) {
          rloc = wave_max(rloc);
          if ((tid & 63) == 0) red[tid >> 6] = rloc;
        }
        __syncthreads();
        if (adapt) {
          double rn = red[0];
          for (int w = 1; w < (nth >> 6); w++) rn = fmax(rn, red[w]);
          resmax = rn;
          if ((n > B.mdf_nmin && rn < tol) || (n > 1 && rn > 1.5 * rprev)) break;
          rprev = rn;
          if (tid == 0) ish[11] = n;
          for (int k = tid; k < nb; k += nth) {
            L.Ftx[k] = (n == 1 ? 0.0 : L.Ftx[k]) + L.Fx[k];
            L.Fty[k] = (n == 1 ? 0.0 : L.Fty[k]) + L.Fy[k];
          }
        }
        // U^(n+1) = U^(n) + B (omega F^(n)), the band split over the lanes
        for (int kk = tid; kk < LPM * nb; kk += nth) {
          const int k = kk / LPM, h = kk % LPM;
          double sx = 0.0, sy = 0.0;
          for (int d = h - bw; d <= bw; d += LPM) {
            int l = k + d;
            l = l < 0 ? l + nb : (l >= nb ? l - nb : l);
            // B_(k,l) is entry |d| of the earlier row in circular order
            const double bkl = d >= 0 ? L.Bm[k * (bw + 1) + d] : L.Bm[l * (bw + 1) - d];
            sx += bkl * L.Fx[l];
            sy += bkl * L.Fy[l];
          }
          sx = group_sum<LPM>(sx);
          sy = group_sum<LPM>(sy);
          if (h == 0) {
            L.Ux[k] += sx;
            L.Uy[k] += sy;
          }
        }
        __syncthreads();
      }
    } else {
      // MDF, Eq. (12)-(14): N passes of interpolation, force and spreading
      // back into the node velocities with relaxation omega_MDF; rho(X) is
      // interpolated once, in the first pass; F_total accumulates omega F^(n).
      // After the first pass's interpolation nrho holds ds / (2 rho(x)), the
      // factor of every pass (each node's thread converts its own entry).
      // Adaptive form (tolerance > 0, Sec. 2.5.2 / App. A.2): the residual
      // r_n = max_k |U_d - U^(n)| is reduced over the workgroup before pass n
      // is applied; the iteration ends there, without pass n, after at least
      // nmin passes once r_n < tol, or when r_n > 1.5 r_(n-1).  F_total then
      // takes omega F^(n) only once the pass is kept.
      const int N = B.mdf_iters;
      const double om = B.omega_mdf;
      const double tol = B.mdf_tol;
      const bool adapt = tol > 0.0;
      double rprev = 0.0;
      for (int n = 1; n <= N; n++) {
        double rloc = 0.0;
        for (int kk = tid; kk < LPM * nb; kk += nth) {
          const int k = kk / LPM, h = kk % LPM;
          // the marker's own operands are loaded ahead of the node gathers
          const double udx = L.Udx[k], udy = L.Udy[k];
          const double rX = n == 1 ? interp1<NS, LPM>(L, k, h, L.nrho) : L.rhoX[k];
          const bool acc = n > 1 && !adapt;
          const double ftx = acc ? L.Ftx[k] : 0.0, fty = acc ? L.Fty[k] : 0.0;
          double Ux, Uy;
          interp2<NS, LPM>(L, k, h, L.nux, L.nuy, Ux, Uy);
          if (h == 0) {
            if (n == 1) L.rhoX[k] = rX;
            const double ex = udx - Ux, ey = udy - Uy;
            const double Fx = 2.0 * rX * ex, Fy = 2.0 * rX * ey;
            L.Fx[k] = om * Fx;
            L.Fy[k] = om * Fy;
            if (!adapt) {
              L.Ftx[k] = ftx + om * Fx;
              L.Fty[k] = fty + om * Fy;
            }
            rloc = fmax(rloc, sqrt(ex * ex + ey * ey));
          }
        }
        if (!adapt && n == N) resmax = rloc;
        if (adapt) {
          rloc = wave_max(rloc);
          if ((tid & 63) == 0) red[tid >> 6] = rloc;
        }
        __syncthreads();
        if (adapt) {
          // every thread takes the same decision from the same partials
          double rn = red[0];
          for (int w = 1; w < (nth >> 6); w++) rn = fmax(rn, red[w]);
          resmax = rn;
          if ((n > B.mdf_nmin && rn < tol) || (n > 1 && rn > 1.5 * rprev)) break;
          rprev = rn;
          if (tid == 0) ish[11] = n;
          for (int k = tid; k < nb; k += nth) {
            L.Ftx[k] = (n == 1 ? 0.0 : L.Ftx[k]) + L.Fx[k];
            L.Fty[k] = (n == 1 ? 0.0 : L.Fty[k]) + L.Fy[k];
          }
        }
        if (n == 1)
          for (int j = tid; j < S; j += nth) L.nrho[j] = ds / (2.0 * L.nrho[j]);
        if (FAST || spread_mode == 0) {
          for (int j = tid; j < S; j += nth) {
            double sx, sy;
            gather2<NS>(L, j, L.Fx, L.Fy, sx, sy);
            L.nux[j] += sx * L.nrho[j];
            L.nuy[j] += sy * L.nrho[j];
          }
        } else {
          for (int j = tid; j < S; j += nth) { accx[j] = 0.0; accy[j] = 0.0; }
          __syncthreads();
          for (int k = tid; k < nb; k += nth)
            for (int q = 0; q < ns * ns; q++) {
              const double w = WX(L, k, q % ns) * WY(L, k, q / ns);
              atomicAdd(&accx[NIDX(L, k, q)], L.Fx[k] * w);
              atomicAdd(&accy[NIDX(L, k, q)], L.Fy[k] * w);
            }
          __syncthreads();
          for (int j = tid; j < S; j += nth) {
            L.nux[j] += accx[j] * L.nrho[j];
            L.nuy[j] += accy[j] * L.nrho[j];
          }
        }
        __syncthreads();
      }
    }
    // the descriptor fields of the force write, read before the wait below
    gmem<T> *const gfrc = to_global(frc);
    gmem<T> *const fpv = to_global((T *)B.fprev);
    const int fpv_plane = B.max_nodes;
    const bool is_df = B.scheme == kDF;
    if constexpr (SELF_COL >= 0) {
      // the tiles that read the previous force have all done so
      if (tid == 0) {
        if (hold_wait(c.state, nhold)) ish[56] |= 2;
        else ish[3] |= kFlagExchange;
      }
    }
    __syncthreads();
    // Eulerian force f(x) = sum_k F_total D_h ds (Eq. 8) into the force field
    // (and, for fused steps, its copy); DF also forms the post-IB node
    // velocity u* + f/(2 rho) for the slip
    if (FAST || spread_mode == 0) {
      for (int j = tid; j < S; j += nth) {
        const int x = L.nxy[j] & 0xffff, y = L.nxy[j] >> 16;
        double fx, fy;
        gather2<NS>(L, j, L.Ftx, L.Fty, fx, fy);
        const uint32_t p = (uint32_t)y * nx + x;
        const T vx = (T)(fx * ds), vy = (T)(fy * ds);
        gfrc[p] = vx;
        gfrc[plane + p] = vy;
        if (fpv) {
          fpv[j] = vx;
          fpv[fpv_plane + j] = vy;
        }
        if (is_df) {
          const double h = 1.0 / (2.0 * L.nrho[j]);
          L.nux[j] += fx * ds * h;
          L.nuy[j] += fy * ds * h;
        }
      }
    } else {
      for (int j = tid; j < S; j += nth) { accx[j] = 0.0; accy[j] = 0.0; }
      __syncthreads();
      for (int k = tid; k < nb; k += nth)
        for (int q = 0; q < ns * ns; q++) {
          const double w = WX(L, k, q % ns) * WY(L, k, q / ns);
          atomicAdd(&accx[NIDX(L, k, q)], L.Ftx[k] * w);
          atomicAdd(&accy[NIDX(L, k, q)], L.Fty[k] * w);
        }
      __syncthreads();
      for (int j = tid; j < S; j += nth) {
        const int x = L.nxy[j] & 0xffff, y = L.nxy[j] >> 16;
        const uint32_t p = (uint32_t)y * nx + x;
        frc[p] = (T)(accx[j] * ds);
        frc[plane + p] = (T)(accy[j] * ds);
        if (B.scheme == kDF) {
          const double h = 1.0 / (2.0 * L.nrho[j]);
          L.nux[j] += accx[j] * ds * h;
          L.nuy[j] += accy[j] * ds * h;
        }
      }
    }
    // force on the body: -sum_k F_total ds sum_x D_h (Newton's third law),
    // torque -sum_k r_k x F_total ds (Sec. 2.7)
    const double xcm = bsh[0], ycm = bsh[1];
    for (int k = tid; k < nb; k += nth) {
      double wsx = 0, wsy = 0;
      for (int j = 0; j < ns; j++) { wsx += WX(L, k, j); wsy += WY(L, k, j); }
      const double wsum = wsx * wsy;
      fsum_x -= L.Ftx[k] * ds * wsum;
      fsum_y -= L.Fty[k] * ds * wsum;
      tq -= ((L.X[k] - xcm) * L.Fty[k] - (L.Y[k] - ycm) * L.Ftx[k]) * ds;
    }
  } else if constexpr (!FAST) {
    // ---- 4b. DFC
    if (!(fixed && ish[2])) {
      for (int j = tid; j < S; j += nth) {
        double wt = 0.0;
        for (int e = L.noff[j]; e < L.noff[j + 1]; e++) wt += node_weight<NS>(L, L.nent[e]);
        L.nW[j] = wt;  // W_total(x) of Eq. (17)
      }
      __syncthreads();
      for (int kk = tid; kk < LPM * nb; kk += nth) {
        const int k = kk / LPM, h = kk % LPM;
        const double wsum = interp1<NS, LPM>(L, k, h, L.nW);
        if (h == 0) {
          L.lam[k] = 1.0 / (2.0 * rho0 * ds * wsum);
          B.lambda_cache[k] = L.lam[k];
        }
      }
      if (fixed && tid == 0) bs->lambda_valid = 1;
    } else {
      for (int k = tid; k < nb; k += nth) L.lam[k] = B.lambda_cache[k];
    }
    __syncthreads();
    // Stage the support populations in LDS (rows of the support are
    // contiguous in x, so these loads coalesce), one plane per direction.
    T *stg = (T *)L.stage;
    const int mn = B.max_nodes;
    for (int j0 = tid; j0 < S; j0 += 2 * nth) {
      T v[2][9];
#pragma unroll
      for (int u = 0; u < 2; u++) {
        const int j = j0 + u * nth;
        if (j < S) {
          const int x = L.nxy[j] & 0xffff, y = L.nxy[j] >> 16;
          const T *fp = fpop + pop_node(x, y, c.nseg);
#pragma unroll
          for (int i = 0; i < 9; i++) v[u][i] = fp[i * kSeg];
        }
      }
#pragma unroll
      for (int u = 0; u < 2; u++) {
        const int j = j0 + u * nth;
        if (j < S) {
#pragma unroll
          for (int i = 0; i < 9; i++) stg[i * mn + j] = v[u][i];
        }
      }
    }
    __syncthreads();
    // Eq. (15)-(18), (20): interpolate the stored populations; the bounce-back
    // target minus f* only involves f*_opp - f*_i, the same in f and in g.
    for (int kk = tid; kk < LPM * nb; kk += nth) {
      const int k = kk / LPM, h = kk % LPM;
      double gi[9];
#pragma unroll
      for (int i = 0; i < 9; i++) gi[i] = 0.0;
#pragma unroll
      for (int r = 0; r < NS / LPM; r++) {
        const int jy = h * (NS / LPM) + r;
        double row[9];
#pragma unroll
        for (int i = 0; i < 9; i++) row[i] = 0.0;
#pragma unroll
        for (int jx = 0; jx < NS; jx++) {
          const int j = NROW(L, k, jy) + jx;
          const double w = WX(L, k, jx);
#pragma unroll
          for (int i = 0; i < 9; i++) row[i] += (double)stg[i * mn + j] * w;
        }
        const double wy = WY(L, k, jy);
#pragma unroll
        for (int i = 0; i < 9; i++) gi[i] += row[i] * wy;
      }
#pragma unroll
      for (int i = 0; i < 9; i++) gi[i] = group_sum<LPM>(gi[i]);
      if (h) continue;
      const double lam = L.lam[k];
      double fsx = 0, fsy = 0;
#pragma unroll
      for (int i = 0; i < 9; i++) {
        const double eud = c_exi[i] * L.Udx[k] + c_eyi[i] * L.Udy[k];
        const double d = lam * (gi[opp_of(i)] - gi[i] + 6.0 * c_w[i] * rho0 * eud);
        DLT(L, k, i) = d;
        fsx += c_exi[i] * d;
        fsy += c_eyi[i] * d;
      }
      L.Ftx[k] = -ds * fsx;
      L.Fty[k] = -ds * fsy;
    }
    __syncthreads();
    // Eq. (19): f_i(x) <- f*_i(x) + sum_k delta f_i D_h ds.  The corrected
    // populations also replace the staged ones (each node only touches its
    // own entries) for the slip diagnostic.
    if (spread_mode == 0) {
      for (int j = tid; j < S; j += nth) {
        const int x = L.nxy[j] & 0xffff, y = L.nxy[j] >> 16;
        double corr[9];
#pragma unroll
        for (int i = 0; i < 9; i++) corr[i] = 0.0;
        for_node_entries_csr<NS>(L, j, [&](int k, double w) {
#pragma unroll
          for (int i = 0; i < 9; i++) corr[i] += DLT(L, k, i) * w;
        });
        T *fw = fpop_w + pop_node(x, y, c.nseg);
#pragma unroll
        for (int i = 0; i < 9; i++) {
          const T nv = (T)((double)stg[i * mn + j] + corr[i] * ds);
          fw[i * kSeg] = nv;
          stg[i * mn + j] = nv;
        }
      }
    } else {
      double *accx = B.acc, *accy = B.acc + B.max_nodes;
      for (int i0 = 0; i0 < 9; i0 += 2) {
        for (int j = tid; j < S; j += nth) { accx[j] = 0.0; accy[j] = 0.0; }
        __syncthreads();
        for (int k = tid; k < nb; k += nth)
          for (int q = 0; q < ns * ns; q++) {
            const double w = WX(L, k, q % ns) * WY(L, k, q / ns);
            atomicAdd(&accx[NIDX(L, k, q)], DLT(L, k, i0) * w);
            if (i0 + 1 < 9) atomicAdd(&accy[NIDX(L, k, q)], DLT(L, k, i0 + 1) * w);
          }
        __syncthreads();
        for (int j = tid; j < S; j += nth) {
          const int x = L.nxy[j] & 0xffff, y = L.nxy[j] >> 16;
          T *fw = fpop_w + pop_node(x, y, c.nseg);
          const T na = (T)((double)stg[i0 * mn + j] + accx[j] * ds);
          fw[i0 * kSeg] = na;
          stg[i0 * mn + j] = na;
          if (i0 + 1 < 9) {
            const T nb2 = (T)((double)stg[(i0 + 1) * mn + j] + accy[j] * ds);
            fw[(i0 + 1) * kSeg] = nb2;
            stg[(i0 + 1) * mn + j] = nb2;
          }
        }
        __syncthreads();
      }
    }
    __syncthreads();
    // velocity of the corrected populations at every support node
    for (int j = tid; j < S; j += nth) {
      double sm = 0, jxs = 0, jys = 0;
#pragma unroll
      for (int i = 0; i < 9; i++) {
        const double v = (double)stg[i * mn + j] + (shift ? c_w[i] * rho0 : 0.0);
        sm += v;
        jxs += v * c_exi[i];
        jys += v * c_eyi[i];
      }
      put_u(stg, mn, j, jxs / sm, jys / sm);
    }
    for (int k = tid; k < nb; k += nth) {
      fsum_x += L.Ftx[k];
      fsum_y += L.Fty[k];
      tq += (L.X[k] - bsh[0]) * L.Fty[k] - (L.Y[k] - bsh[1]) * L.Ftx[k];
    }
  }
  __syncthreads();
  // ---- 5. slip with the post-IB velocity, reductions, body update
  // The marker-space passes leave the velocity at the markers, so no lane
  // group interpolates here, and marker k's lanes are k, k + nb, ...: the
  // slip terms then sit in the first nb threads, like the force sums, and
  // only their waves reduce.  Otherwise lane h of marker k is LPM k + h.
  const bool mspace = FAST && L.bw > 0 && ish[13] == kMDF;
  const int nlive = mspace ? nb : LPM * nb;
  double slip_sum = 0, slip_max = 0;
  for (int kk = tid; kk < LPM * nb; kk += nth) {
    const int k = mspace ? kk % nb : kk / LPM, h = mspace ? kk / nb : kk % LPM;
    double Ux, Uy;
    if (!FAST && B.scheme == kDFC) {
      interp_packed_u<NS, LPM, T>(L, k, h, (const T *)L.stage, B.max_nodes, Ux, Uy);
    } else if (mspace) {
      Ux = L.Ux[k];  // the marker-space passes end with the post-IB velocity
      Uy = L.Uy[k];
    } else {
      interp2<NS, LPM>(L, k, h, L.nux, L.nuy, Ux, Uy);
    }
    // the marker's output row (X Y Udx Udy Fx Fy lambda ds), split over
    // the lanes of its group
    gmem<double> *mo = to_global((double *)__double_as_longlong(bsh[17])) + 8 * k;
    if (h == 0) {
      const double e = sqrt((Ux - L.Udx[k]) * (Ux - L.Udx[k]) + (Uy - L.Udy[k]) * (Uy - L.Udy[k]));
      slip_sum += e;
      slip_max = fmax(slip_max, e);
    }
    if (LPM == 2) {
      if (h == 0) {
        mo[0] = L.X[k]; mo[1] = L.Y[k]; mo[2] = L.Udx[k]; mo[3] = L.Udy[k];
      } else {
        mo[4] = L.Ftx[k]; mo[5] = L.Fty[k]; mo[6] = (!FAST && B.scheme == kDFC) ? L.lam[k] : 0.0; mo[7] = ds;
      }
    } else {
      if (h == 0) {
        mo[0] = L.X[k]; mo[1] = L.Y[k];
      } else if (h == 1) {
        mo[2] = L.Udx[k]; mo[3] = L.Udy[k];
      } else if (h == 2) {
        mo[4] = L.Ftx[k]; mo[5] = L.Fty[k];
      } else {
        mo[6] = (!FAST && B.scheme == kDFC) ? L.lam[k] : 0.0; mo[7] = ds;
      }
    }
  }
  double a = fsum_x, b = fsum_y, cq = tq, m = fmax(resmax, 0.0);
  double s1 = slip_sum, s4 = slip_max;
  block_reduce6(a, b, cq, s1, m, s4, red, nlive);
  if (tid == 0) {
    // every value is formed in registers and written once (no read-back of
    // device memory on this serial tail; the descriptor values come from
    // the on-chip copy made with the kinematics)
    const int motion = ish[12], scheme = ish[13], iters = ish[11], box_valid = ish[10];
    const double xc = bsh[0], yc = bsh[1], vhx = bsh[2], vhy = bsh[3], omh = bsh[4];
    int flags = 0;
    if (!isfinite(a) || !isfinite(b) || !isfinite(cq) || !isfinite(s1)) flags |= kFlagNonfinite;
    const double slip_mean = s1 / nb;
    const double mdf_res = scheme == kMDF ? m : 0.0;
    int box[4] = {0, 0, -1, -1};
    if (box_valid) {
      const double r = bsh[12];
      box[0] = max(0, (int)floor(xc - r) - ns);
      box[1] = max(0, (int)floor(yc - r) - ns);
      box[2] = min(nx - 1, (int)floor(xc + r) + ns + 1);
      box[3] = min(ish[14] - 1, (int)floor(yc + r) + ns + 1);
    }
    double vx = vhx, vy = vhy, om = omh;
    if (motion == kFree && ish[15] == kEulerA1) {
      // the Euler-explicit velocity was set before the step; the new force
      // enters the next one
      if (!isfinite(vx) || !isfinite(vy) || fabs(vx) > 0.5 || fabs(vy) > 0.5) flags |= kFlagNonfinite;
    } else if (motion == kFree) {
      const double ms = bsh[8];
      vx = vhx + (a + bsh[9] + bsh[5]) / (2.0 * ms);
      vy = vhy + (b + bsh[10] + bsh[6]) / (2.0 * ms);
      om = omh + cq / (2.0 * bsh[11]);
      if (!isfinite(vx) || !isfinite(vy) || fabs(vx) > 0.5 || fabs(vy) > 0.5) flags |= kFlagNonfinite;
    } else if (motion == kFixed) {
      vx = 0.0; vy = 0.0; om = 0.0;
    }
    flags |= ish[3];
    if (ish[6]) flags |= kFlagExchange;
    gmem<BodyState> *const gbs = to_global(bs);
    gbs->fhx = a;
    gbs->fhy = b;
    gbs->torque = cq;
    gbs->slip_mean = slip_mean;
    gbs->slip_max = s4;
    gbs->mdf_res = mdf_res;
    gbs->mdf_iters_done = iters;
    gbs->box[0] = box[0]; gbs->box[1] = box[1]; gbs->box[2] = box[2]; gbs->box[3] = box[3];
    gbs->box_valid = box_valid;
    if (motion != kPrescribedSin) {
      gbs->vx = vx; gbs->vy = vy; gbs->om = om;
    }
    gbs->flags = flags;
    gmem<double> *const h = to_global((double *)__double_as_longlong(bsh[7]));
    h[0] = (double)(step + 1); h[1] = a; h[2] = b; h[3] = cq;
    h[4] = xc; h[5] = yc; h[6] = vx; h[7] = vy; h[8] = motion == kFree ? om : omh;
    h[9] = slip_mean; h[10] = s4; h[11] = mdf_res;
    h[12] = iters; h[13] = flags; h[14] = 0; h[15] = 0;
    // for the case-level update of a single-body case
    ish[50] = flags;
    ish[51] = box_valid;
    ish[52] = box[0]; ish[53] = box[1]; ish[54] = box[2]; ish[55] = box[3];
  }
}

// One workgroup per IB slot: kIbmThreads threads, or kIbmThreadsFast for
// the FAST instance (every body of the launch DF/MDF, in LDS, gather
// spreading; see body_step).  With replicas > 1 each slot is launched that
// many times (one workgroup per XCD for replicas = 8) and the first of them
// to start takes the slot: every copy adds one to the slot's counter
// ticket[slot], which stream order leaves at a multiple of `replicas` when
// a launch begins, and the copy that draws that multiple runs the pass; the
// others leave at once.  No per-launch argument is involved, so the launch
// can be replayed from a captured graph.  A pass that shares the chip with
// a large launch on another stream then starts on whichever XCD frees a
// compute unit first.
template <typename T, bool FAST>
__global__ __launch_bounds__(FAST ? kIbmThreadsFast : kIbmThreads) void ibm_kernel(
    const CaseDesc *__restrict__ cases, const IbmSlot *__restrict__ slots, int lds_doubles,
    int spread_mode, int replicas, uint32_t *ticket) {
  extern __shared__ double dyn[];
  __shared__ double red[6 * ((FAST ? kIbmThreadsFast : kIbmThreads) / 64)];
  // ish: [0..15] flags and switches, [16..48] scan scratch, [50..55] the
  // body's final flags, force-box flag and force box
  __shared__ int ish[56];
  __shared__ double bsh[18];
  const int slot = replicas > 1 ? (int)blockIdx.x / replicas : (int)blockIdx.x;
  // the ticket is taken by a thread of wave 1 while all threads read the
  // slot and the case state; nothing is written before the outcome is known
  if (replicas > 1 && threadIdx.x == 64) ish[49] = atomicAdd(&ticket[slot], 1u) % (uint32_t)replicas == 0u;
  const IbmSlot sl = slots[slot];
  const CaseDesc &c = cases[sl.cas];
  CaseState *cs = c.state;
  const int64_t step = cs->step;
  const int cur = cs->cur;
  const bool active = step < cs->target && !(cs->flags & kCaseHalted);
  if (replicas > 1) {
    __syncthreads();
    if (!ish[49]) return;
  }
  if (!active) return;
  if (threadIdx.x == 0) ish[50] = 0;
  if (sl.body >= 0) {
    const BodyDesc &B = c.bodies[sl.body];
    const bool lds = lds_doubles >= B.ws_doubles;
    if constexpr (FAST) {
      if (B.ns == 2) body_step<T, true, 2, true>(c, B, step, cur, dyn, spread_mode, red, ish, bsh);
      else body_step<T, true, 4, true>(c, B, step, cur, dyn, spread_mode, red, ish, bsh);
    } else if (B.ns == 2) {
      if (lds) body_step<T, true, 2, false>(c, B, step, cur, dyn, spread_mode, red, ish, bsh);
      else body_step<T, false, 2, false>(c, B, step, cur, dyn, spread_mode, red, ish, bsh);
    } else {
      if (lds) body_step<T, true, 4, false>(c, B, step, cur, dyn, spread_mode, red, ish, bsh);
      else body_step<T, false, 4, false>(c, B, step, cur, dyn, spread_mode, red, ish, bsh);
    }
  }
  __syncthreads();
  if (threadIdx.x != 0) return;
  if (sl.slots_in_case == 1) {
    // the only workgroup of its case: no other body to wait for; the body's
    // flags and force box come from the workgroup's shared memory
    if (sl.body >= 0 && ish[50]) {
      cs->flags |= kCaseHalted;
    } else {
      if (sl.body >= 0 && ish[51]) {
        cs->fbox[0] = ish[52]; cs->fbox[1] = ish[53];
        cs->fbox[2] = ish[54]; cs->fbox[3] = ish[55];
        cs->fbox_valid = 1;
      } else {
        cs->fbox_valid = 0;
      }
      cs->cur = cur ^ 1;
      cs->step = step + 1;
    }
    cs->xcnt = 0;
    return;
  }
  __threadfence();
  const int prev = atomicAdd(&cs->done, 1);
  if (prev != sl.slots_in_case - 1) return;
  __threadfence();
  // Last workgroup of its case.  A body that failed this step (support
  // outside the lattice, work space too small, non-finite force) stops the
  // case without completing the step; bodies whose supports could meet within
  // the next step stop it after completing this one.  The union of the
  // bodies' force boxes tells the next collide-stream launch where to read
  // the IB force.
  int bflags = 0, bv = 0, b0 = 1 << 30, b1 = 1 << 30, b2 = -1, b3 = -1;
  for (int b = 0; b < c.nbodies; b++) {
    BodyState *st = c.bodies[b].state;
    bflags |= __hip_atomic_load(&st->flags, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    if (__hip_atomic_load(&st->box_valid, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) {
      bv = 1;
      b0 = min(b0, __hip_atomic_load(&st->box[0], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT));
      b1 = min(b1, __hip_atomic_load(&st->box[1], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT));
      b2 = max(b2, __hip_atomic_load(&st->box[2], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT));
      b3 = max(b3, __hip_atomic_load(&st->box[3], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT));
    }
  }
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
  cs->xcnt = 0;
  if (bflags) {
    cs->flags |= kCaseHalted;
  } else {
    cs->fbox[0] = b0; cs->fbox[1] = b1; cs->fbox[2] = b2; cs->fbox[3] = b3;
    cs->fbox_valid = bv;
    cs->cur ^= 1;
    cs->step = step + 1;
    if (meet) cs->flags |= kCaseHalted;
  }
  __threadfence();
}

// ---- fused step: one launch per step for a case with a single fixed
// DF/MDF body (see FusedArgs).  The IB pass needs no post-stream lattice
// from this launch (it collides its support itself), the tiles need only
// the force of the previous pass (the hold tiles read and clear it before
// the pass writes the new one), so nothing in the launch depends on
// anything but that count, and consecutive steps are ordered by the stream
// alone.  The tiles start streaming once the pass has its kinematics and
// tables (gate_wait, when `gated`): beside a chip-wide stream those
// dependent loads take several times longer.  In FP64 the tiles bound the
// launch and start at once.

// The IB workgroup of a fused step: the pass, then the case-level update of
// a single-body case (the same as ibm_kernel's), after the hold tiles have
// all counted themselves, which also holds when the pass does not run.
template <typename T, int COL>
__device__ __forceinline__ void fused_ib(const FusedArgs &a, int nhold, double *dyn, double *red,
                                         int *ish, double *bsh) {
  const CaseDesc &c = a.cd;
  CaseState *cs = c.state;
  const int64_t step = cs->step;
  const int cur = cs->cur;
  const bool active = step < cs->target && !(cs->flags & kCaseHalted);
  if (threadIdx.x == 0) {
    ish[50] = 0;
    ish[56] = 0;
  }
  if (active) {
    const BodyDesc &B = a.bd;
    if (B.ns == 2)
      body_step<T, true, 2, true, COL>(c, B, step, cur, dyn, 0, red, ish, bsh, nhold, a.seq, a.nsrc);
    else
      body_step<T, true, 4, true, COL>(c, B, step, cur, dyn, 0, red, ish, bsh, nhold, a.seq, a.nsrc);
  }
  __syncthreads();
  if (threadIdx.x != 0) return;
  // A pass that ran through has opened the gate and seen both counts
  // complete; one that ended early or did not run opens the gate and waits
  // for the counts here, before they are reset for the next launch.
  bool met = ish[56] == 3;
  if (!met) {
    gate_open(cs, a.seq);
    met = hold_wait(cs, nhold) && src_wait(cs, a.nsrc);
  }
  __hip_atomic_store(&cs->hold_seen, 0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  __hip_atomic_store(&cs->src_seen, 0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  if (!active) return;
  if (ish[50] || !met) {
    cs->flags |= kCaseHalted;
  } else {
    if (ish[51]) {
      cs->fbox[0] = ish[52]; cs->fbox[1] = ish[53];
      cs->fbox[2] = ish[54]; cs->fbox[3] = ish[55];
      cs->fbox_valid = 1;
    } else {
      cs->fbox_valid = 0;
    }
    cs->cur = cur ^ 1;
    cs->step = step + 1;
  }
  cs->xcnt = 0;
}

// A source workgroup of a fused step: one node that pushes into the
// support per thread collides, as a tile does (the same collide function,
// the force the tiles read, kept in BodyDesc::fprev), from the step's input
// lattice, and its pushes into the support are staged population-major in
// BodyDesc::pstage; then the workgroup counts itself.
template <typename T, int COL>
__device__ __forceinline__ void fused_src(const FusedArgs &a, int w) {
  const CaseDesc &c = a.cd;
  const BodyDesc &B = a.bd;
  const int u = w * kFusedThreads + (int)threadIdx.x;
  if (u < B.n_src) {
    const SrcNode r = B.src[u];
    const T *fp = (const T *)c.f[a.cur] + r.off;
    T f[9];
#pragma unroll
    for (int i = 0; i < 9; i++) f[i] = fp[i * kSeg];
    T Fx = T(c.fluid_fx), Fy = T(c.fluid_fy);
    const int mn = B.max_nodes;
    if (r.map[0] >= 0) {
      const T *fpv = (const T *)B.fprev;
      const T fa = fpv[r.map[0]], fb = fpv[mn + r.map[0]];
      if (fa != T(0) || fb != T(0)) {
        Fx += fa;
        Fy += fb;
      }
    }
    collide<T, sizeof(T) == 4, COL>(f, Fx, Fy, c);
    T *stg = (T *)B.pstage;
#pragma unroll
    for (int i = 0; i < 9; i++)
      if (r.map[i] >= 0) stg[i * mn + r.map[i]] = f[i];
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    __threadfence();
    __hip_atomic_fetch_add(&c.state->src_seen, 1, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
  }
}

template <typename T, int COL, bool GZG>
__global__ __launch_bounds__(kFusedThreads) void step_fused_kernel(const FusedArgs a) {
  extern __shared__ double dyn[];
  __shared__ double red[6 * (kFusedThreads / 64)];
  // ish as in ibm_kernel, and [56]: the counts the pass has seen complete
  // (1: source workgroups, 2: hold tiles)
  __shared__ int ish[57];
  __shared__ double bsh[18];
  int b = blockIdx.x;
  const int nhold = a.lean.hntx * a.lean.hnty;
  const int nfw = a.nface;
  const int lx = threadIdx.x % a.bx, ly = threadIdx.x / a.bx;
  if (b == 0) {
    fused_ib<T, COL>(a, nhold, dyn, red, ish, bsh);
    return;
  }
  if (b <= a.nsrc) {
    fused_src<T, COL>(a, b - 1);
    return;
  }
  b -= a.nsrc;
  if (b <= nhold) {
    if (a.gated) gate_wait(a.lean.state, a.seq);
    int tx, ty;
    if (lean_tile_index<1>(a.lean, b - 1, tx, ty)) lean_tile<T, COL, 1>(a.lean, tx, ty, lx, ly, a.bx, a.by);
    // every read and clear of the force by this workgroup is done and
    // written back before it counts itself
    __syncthreads();
    if (threadIdx.x == 0) {
      __threadfence();
      __hip_atomic_fetch_add(&((CaseState *)a.lean.state)->hold_seen, 1, __ATOMIC_RELEASE,
                             __HIP_MEMORY_SCOPE_AGENT);
    }
    return;
  }
  int r = b - 1 - nhold;
  if (r < nfw) {
    // face nodes, one face workgroup (kFaceBlock nodes) per workgroup: the
    // face work is latency-bound, so it is spread over as many compute
    // units as the standalone face launch uses
    if (threadIdx.x >= kFaceBlock) return;
    face_node<T, COL, GZG>(a.c, a.face_prefix, 1, a.nface, r, (int)threadIdx.x, a.cur, 0);
    return;
  }
  r -= nfw;
  // the far tiles, neighbours kept on one XCD as in the other launches
  const int nfar = (int)gridDim.x - 1 - a.nsrc - nhold - nfw;
  int t = r;
  if (a.lean.remap) t = (r & 7) * (nfar >> 3) + (r >> 3);
  int tx, ty;
  if (!lean_tile_index<2>(a.lean, t, tx, ty)) return;
  if (a.gated) gate_wait(a.lean.state, a.seq);
  lean_tile<T, COL, 2>(a.lean, tx, ty, lx, ly, a.bx, a.by);
}

int fused_grid(const FusedArgs &a) {
  const int nhold = a.lean.hntx * a.lean.hnty;
  const int nfw = a.nface;
  int nfar = a.lean.ntiles;
  if (a.lean.remap) nfar = (nfar + 7) / 8 * 8;
  return 1 + a.nsrc + nhold + nfw + nfar;
}

hipError_t launch_step_fused(int precision, int collision, const FusedArgs &a, int lds_bytes,
                             hipStream_t stream, LaunchTarget *ns) {
  static bool configured = false;
  if (!configured) {
    (void)hipFuncSetAttribute((const void *)step_fused_kernel<float, kBGK, false>,
                              hipFuncAttributeMaxDynamicSharedMemorySize, kIbmDynLds);
    (void)hipFuncSetAttribute((const void *)step_fused_kernel<float, kBGK, true>,
                              hipFuncAttributeMaxDynamicSharedMemorySize, kIbmDynLds);
    (void)hipFuncSetAttribute((const void *)step_fused_kernel<float, kTRT, false>,
                              hipFuncAttributeMaxDynamicSharedMemorySize, kIbmDynLds);
    (void)hipFuncSetAttribute((const void *)step_fused_kernel<float, kTRT, true>,
                              hipFuncAttributeMaxDynamicSharedMemorySize, kIbmDynLds);
    (void)hipFuncSetAttribute((const void *)step_fused_kernel<double, kBGK, false>,
                              hipFuncAttributeMaxDynamicSharedMemorySize, kIbmDynLds);
    (void)hipFuncSetAttribute((const void *)step_fused_kernel<double, kBGK, true>,
                              hipFuncAttributeMaxDynamicSharedMemorySize, kIbmDynLds);
    (void)hipFuncSetAttribute((const void *)step_fused_kernel<double, kTRT, false>,
                              hipFuncAttributeMaxDynamicSharedMemorySize, kIbmDynLds);
    (void)hipFuncSetAttribute((const void *)step_fused_kernel<double, kTRT, true>,
                              hipFuncAttributeMaxDynamicSharedMemorySize, kIbmDynLds);
    configured = true;
  }
  if (collision != kBGK && collision != kTRT) return hipErrorInvalidValue;
  if (a.bx <= 0 || a.by <= 0 || a.bx * a.by != kFusedThreads || a.lean.hntx <= 0 || a.lean.hnty <= 0 ||
      a.nsrc <= 0)
    return hipErrorInvalidValue;
  if (lds_bytes > kIbmDynLds) return hipErrorInvalidValue;
  const dim3 grid(fused_grid(a)), block(kFusedThreads);
#define IBL_FUSED(TT, CC, GG) return issue(step_fused_kernel<TT, CC, GG>, grid, block, lds_bytes, stream, ns, a)
  if (precision == kPrecFP64) {
    if (collision == kBGK) { if (a.gzg) IBL_FUSED(double, kBGK, true); IBL_FUSED(double, kBGK, false); }
    if (a.gzg) IBL_FUSED(double, kTRT, true);
    IBL_FUSED(double, kTRT, false);
  }
  if (collision == kBGK) { if (a.gzg) IBL_FUSED(float, kBGK, true); IBL_FUSED(float, kBGK, false); }
  if (a.gzg) IBL_FUSED(float, kTRT, true);
  IBL_FUSED(float, kTRT, false);
#undef IBL_FUSED
}

// ---- boundary-fidelity diagnostics (Sec. 2.8, marker profiles of Sec. 4.2)
// Density and velocity at node (x, y) with the pending IB force (Eq. 4).
template <typename T>
__device__ __forceinline__ void node_moments(const CaseDesc &c, const T *f, const T *frc, int x, int y,
                                             double &rho, double &ux, double &uy) {
  const bool shift = sizeof(T) == 4;
  const uint32_t plane = (uint32_t)c.plane;
  const uint32_t p = (uint32_t)y * c.nx + x;
  const T *fp = f + pop_node(x, y, c.nseg);
  double s = 0, jx = 0, jy = 0;
#pragma unroll
  for (int i = 0; i < 9; i++) {
    const double v = (double)fp[i * kSeg] + (shift ? c_w[i] * c.rho0 : 0.0);
    s += v;
    jx += v * c_exi[i];
    jy += v * c_eyi[i];
  }
  const double Fx = (double)frc[p] + c.fluid_fx, Fy = (double)frc[plane + p] + c.fluid_fy;
  rho = s;
  ux = (jx + 0.5 * Fx) / s;
  uy = (jy + 0.5 * Fy) / s;
}

// One workgroup per call.  Markers: the field sampled bilinearly (the hat
// weights of the 2 x 2 nodes around X_k), relative to the rigid motion
// U_b(x) = v + om x (x - X_c); interior: nodes with |x - X_c| < R - kappa.
// Sums and maxima are reduced in a fixed order (wave trees, then the waves
// in index order); out[8] as the C entry point documents, pm[6 k ..] per
// marker.
constexpr int kDiagThreads = 256;
template <typename T>
__global__ void __launch_bounds__(kDiagThreads)
diag_kernel(CaseDesc c, int buf, const double *mk, int nb, double xc, double yc, double vx,
            double vy, double om, double radius, double diameter, double ds, int kappa,
            double u_ref, double *out, double *pm) {
  __shared__ double red[8 * (kDiagThreads / 64)];
  const int tid = threadIdx.x, nth = blockDim.x;
  const T *f = (const T *)c.f[buf];
  const T *frc = (const T *)c.force;
  const int nx = c.nx;
  double s_slip = 0, m_slip = 0, s_flux = 0, s_dp = 0, s_f = 0;
  for (int k = tid; k < nb; k += nth) {
    const double *m = mk + 8 * k;
    const double X = m[0], Y = m[1];
    // the 2 x 2 stencil must lie in the lattice (false for NaN positions);
    // a marker outside gives NaN and no loads
    if (!(X >= 0.0 && Y >= 0.0 && X < (double)(nx - 1) && Y < (double)(c.ny - 1))) {
      const double nan = __builtin_nan("");
      s_slip += nan;
      s_flux += nan;
      if (pm)
        for (int i = 0; i < 6; i++) pm[6 * k + i] = nan;
      continue;
    }
    const int x0 = (int)floor(X), y0 = (int)floor(Y);
    double rk = 0, uxk = 0, uyk = 0;
    for (int jy = 0; jy < 2; jy++)
      for (int jx = 0; jx < 2; jx++) {
        const double w = delta1(kHat, (double)(x0 + jx) - X) * delta1(kHat, (double)(y0 + jy) - Y);
        double r, u, v;
        node_moments<T>(c, f, frc, x0 + jx, y0 + jy, r, u, v);
        rk += r * w;
        uxk += u * w;
        uyk += v * w;
      }
    const double dx = uxk - (vx - om * (Y - yc)), dy = uyk - (vy + om * (X - xc));
    const double nxk = (X - xc) / radius, nyk = (Y - yc) / radius;
    const double slip = sqrt(dx * dx + dy * dy) / u_ref;
    const double dp = (rk - c.rho0) * (1.0 / 3.0);
    const double fm = sqrt(m[4] * m[4] + m[5] * m[5]);
    s_slip += slip;
    m_slip = fmax(m_slip, slip);
    s_flux += rk * (dx * nxk + dy * nyk) * ds;
    s_dp += dp;
    s_f += fm;
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
  double s_in = 0, m_in = 0, n_in = 0;
  const double ri = radius - kappa;
  if (ri > 0) {
    const int bx0 = max(0, (int)ceil(xc - ri)), bx1 = min(nx - 1, (int)floor(xc + ri));
    const int by0 = max(0, (int)ceil(yc - ri)), by1 = min(c.ny - 1, (int)floor(yc + ri));
    const int bw = bx1 - bx0 + 1, bh = by1 - by0 + 1;
    const int nq = bw > 0 && bh > 0 ? bw * bh : 0;
    for (int q = tid; q < nq; q += nth) {
      const int x = bx0 + q % bw, y = by0 + q / bw;
      const double rx = x - xc, ry = y - yc;
      if (rx * rx + ry * ry >= ri * ri) continue;
      double r, u, v;
      node_moments<T>(c, f, frc, x, y, r, u, v);
      const double dx = u - (vx - om * ry), dy = v - (vy + om * rx);
      const double mg = sqrt(dx * dx + dy * dy) / u_ref;
      s_in += mg;
      m_in = fmax(m_in, mg);
      n_in += 1.0;
    }
  }
  double v8[8] = {s_slip, m_slip, s_flux, s_in, m_in, n_in, s_dp, s_f};
  const int lane = tid & 63, wv = tid >> 6, nw = nth >> 6;
#pragma unroll
  for (int i = 0; i < 8; i++) {
    const bool mx = i == 1 || i == 4;
    v8[i] = mx ? wave_max(v8[i]) : wave_sum(v8[i]);
    if (lane == 0) red[8 * wv + i] = v8[i];
  }
  __syncthreads();
  if (tid == 0) {
    double t[8];
    for (int i = 0; i < 8; i++) {
      t[i] = red[i];
      for (int w = 1; w < nw; w++)
        t[i] = (i == 1 || i == 4) ? fmax(t[i], red[8 * w + i]) : t[i] + red[8 * w + i];
    }
    out[0] = t[0] / nb;
    out[1] = t[1];
    out[2] = t[2] / (u_ref * M_PI * diameter);
    out[3] = t[5] > 0 ? t[3] / t[5] : 0.0;
    out[4] = t[4];
    out[5] = t[5];
    out[6] = t[6] / nb;
    out[7] = t[7] / nb;
  }
}

hipError_t launch_diagnostics(const CaseDesc &c, int buf, const double *markers, int nb, double xc,
                              double yc, double vx, double vy, double om, double radius,
                              double ds, int kappa, double u_ref, double *out, double *pm,
                              hipStream_t stream) {
  if (c.precision == kPrecFP64)
    hipLaunchKernelGGL(diag_kernel<double>, dim3(1), dim3(kDiagThreads), 0, stream, c, buf, markers,
                       nb, xc, yc, vx, vy, om, radius, 2.0 * radius, ds, kappa, u_ref, out, pm);
  else
    hipLaunchKernelGGL(diag_kernel<float>, dim3(1), dim3(kDiagThreads), 0, stream, c, buf, markers,
                       nb, xc, yc, vx, vy, om, radius, 2.0 * radius, ds, kappa, u_ref, out, pm);
  return hipGetLastError();
}

// Device staging of the allocation-free diagnostics entry point: the
// summary (8 doubles) and up to kDiagScratchMarkers per-marker rows of 6.
// Each GPU holds its own copy for the life of the process; host code reaches
// it only through the address hipGetSymbolAddress returns on that device.
constexpr int kDiagScratchMarkers = 8192;
static __device__ __align__(256) double scratch[8 + 6 * kDiagScratchMarkers];

int diag_scratch_markers() { return kDiagScratchMarkers; }

hipError_t diag_scratch(double **ptr) {
  constexpr int kMaxDevices = 64;
  static std::mutex mu;
  static double *addr[kMaxDevices];
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lk(mu);
  if (!addr[dev]) {
    void *p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    addr[dev] = (double *)p;
  }
  *ptr = addr[dev];
  return hipSuccess;
}

int ibm_max_lds_bytes() { return kIbmDynLds; }

hipError_t launch_ibm(int precision, const CaseDesc *cases, const IbmSlot *slots, int nslots,
                      int lds_bytes, int spread_mode, int fast, int replicas, uint32_t *ticket,
                      int threads, hipStream_t stream, LaunchTarget *ns) {
  if (nslots <= 0) return nothing_to_launch(stream, ns);
  static bool configured = false;
  if (!configured) {
    // allow the large dynamic LDS workspace (gfx950 has 160 KB per CU)
    (void)hipFuncSetAttribute((const void *)ibm_kernel<double, false>,
                              hipFuncAttributeMaxDynamicSharedMemorySize, kIbmDynLds);
    (void)hipFuncSetAttribute((const void *)ibm_kernel<float, false>,
                              hipFuncAttributeMaxDynamicSharedMemorySize, kIbmDynLds);
    (void)hipFuncSetAttribute((const void *)ibm_kernel<double, true>,
                              hipFuncAttributeMaxDynamicSharedMemorySize, kIbmDynLds);
    (void)hipFuncSetAttribute((const void *)ibm_kernel<float, true>,
                              hipFuncAttributeMaxDynamicSharedMemorySize, kIbmDynLds);
    configured = true;
  }
  const int lds_doubles = lds_bytes / 8;
  if (replicas < 1) replicas = 1;
  const int grid = nslots * replicas;
  // the kernel's loops stride by the workgroup size and its staging needs
  // more than one wave: any of 256, 512, 1024 up to the launch bound
  const int bound = fast ? kIbmThreadsFast : kIbmThreads;
  const int nt = threads >= 256 ? (threads < bound ? threads : bound) : bound;
  if (precision == kPrecFP64)
    return fast ? issue(ibm_kernel<double, true>, dim3(grid), dim3(nt), lds_bytes, stream, ns, cases,
                        slots, lds_doubles, spread_mode, replicas, ticket)
                : issue(ibm_kernel<double, false>, dim3(grid), dim3(nt), lds_bytes, stream, ns, cases,
                        slots, lds_doubles, spread_mode, replicas, ticket);
  return fast ? issue(ibm_kernel<float, true>, dim3(grid), dim3(nt), lds_bytes, stream, ns, cases,
                      slots, lds_doubles, spread_mode, replicas, ticket)
              : issue(ibm_kernel<float, false>, dim3(grid), dim3(nt), lds_bytes, stream, ns, cases,
                      slots, lds_doubles, spread_mode, replicas, ticket);
}

}  // namespace iblbm
