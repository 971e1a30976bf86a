// C ABI of the IB-LBM library: state ownership, validation, launch tables,
// graph capture and kernel timing.  Every step of the method runs in the HIP
// kernels of lbm_kernels.hip and ibm_kernels.hip; the host code here only
// allocates, validates, sizes the per-body workspaces and enqueues launches.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <initializer_list>
#include <map>
#include <limits>
#include <string>
#include <vector>

#include "../../include/ib_lbm.h"
#include "ib_lbm_internal.h"

using namespace iblbm;

namespace {

struct DevBuf {
  void *p = nullptr;
  size_t bytes = 0;
};

struct HostBody {
  ib_lbm_body_desc d;
  BodyDesc dev;  // host copy of the device description
  DevBuf cos_t, sin_t, ws, tab, acc, markers, lambda, history, state;
  // fused steps: the force copy and staged pushes (fixed DF/MDF bodies), and
  // the nodes the IB pass collides itself with their push map, built once
  // the device has built the body's tables
  DevBuf fprev, pstage, src;
  bool src_ready = false;
};

struct EventPair {
  hipEvent_t a, b;
};

// Kernel timing kinds: 0 collide-stream, 1 IB pass.
constexpr int kTimingKinds = 2;

struct Timing {
  bool on = false;
  std::vector<EventPair> ev[kTimingKinds];
  std::vector<EventPair> pool;
  double folded_ms[kTimingKinds] = {0, 0};
  int64_t folded_n[kTimingKinds] = {0, 0};
};

}  // namespace

struct ib_lbm_sim {
  ib_lbm_config cfg;
  hipStream_t stream = nullptr;          // the caller's stream (NULL: null stream)
  hipStream_t cap_stream = nullptr;      // private stream used only for graph capture
  bool broken = false;
  bool started = false;
  bool tables_dirty = true;
  std::string err;
  CaseDesc cd;  // host copy
  DevBuf f0, f1, force, state, ticket;
  std::vector<HostBody> bodies;
  DevBuf d_bodies, d_case, d_prefix, d_slots, d_tmp;
  int nslots = 0;
  ib_lbm_launch launch = {128, 2, 1, 1};
  int spread_mode = 0;
  int nslots_fast = 0;    // the first IB slots, run by the 1024-thread kernel
  int graph_steps = 0;
  // captured steps, one graph per parity of the input lattice at its start
  // (the lattice of each step is a kernel argument)
  hipGraphExec_t graph_exec[2] = {nullptr, nullptr};
  int graph_len = 0;
  Timing timing;
  int64_t host_steps = 0;
  // lattice holding the input of the next enqueued step: flipped by every
  // enqueued step, reloaded from the device state by every call that reads
  // it (they differ only once a halted case stops flipping it on the device,
  // and a halted case's kernels do nothing)
  int host_cur = 0;
  int dev = 0;  // the device current at creation
  ib_lbm_batch *batch = nullptr;
  int lds_bytes = 0;
  // Pipelined steps (see plan_split): the tiles of the hold rectangle and
  // the IB pass run on `iq`, all other tiles on `lq`, ordered by events.
  bool overlap = true;   // allowed by the caller
  bool split = false;    // in use for the current tables
  int32_t hold[4] = {0, 0, 0, 0};
  hipStream_t lq = nullptr, iq = nullptr;
  hipEvent_t ev_start = nullptr, ev_lq = nullptr, ev_iq = nullptr, ev_near = nullptr,
             ev_far = nullptr;
  // Fused steps (see plan_fused): one launch per step on the sim's stream.
  bool fused_allowed = true;  // allowed by the caller
  bool fused = false;         // in use for the current tables
  int32_t fhold[4] = {0, 0, 0, 0};  // hold rectangle in tiles of the fused shape
  // the fused launch's tile shape (bx x by, rows per thread): narrow tiles
  // keep the hold rectangle small; measured on the 2000x800 cylinder, FP32
  // 30.7 us per step at 64 x 16 and at 1024 x 1 x 4, FP64 37.0 us at 64 x 16
  // against 40.6 (256 x 4), 43.3 (512 x 2 x 2) and 46.5 (1024 x 1 x 4)
  int fbx = 64, fby = kFusedThreads / 64, frpt = 1;
  uint32_t fused_seq = 0;  // sequence number of the last fused launch (CaseState::gate)
};

struct ib_lbm_batch {
  hipStream_t stream = nullptr;
  hipStream_t cap_stream = nullptr;
  int precision = 0;
  bool dirty = true;
  bool broken = false;
  std::string err;
  std::vector<ib_lbm_sim *> sims;
  DevBuf d_cases, d_prefix, d_fprefix, d_slots;
  struct Group {
    int collision, first, count, ntiles, prefix_off, nface_blocks;
    int general_zg;  // some case has a zero-gradient face other than the east one
  };
  std::vector<Group> groups;
  int nslots = 0;
  int lds_bytes = 0;
  ib_lbm_launch launch = {128, 2, 1, 1};
  int spread_mode = 0;
  int nslots_fast = 0;
  int graph_steps = 0;
  hipGraphExec_t graph_exec = nullptr;
  int graph_len = 0;
};

namespace {

void set_err(std::string *e, const char *fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  *e = buf;
}

#define HIPCHK(sim, call)                                                             \
  do {                                                                                \
    hipError_t e_ = (call);                                                           \
    if (e_ != hipSuccess) {                                                           \
      set_err(&(sim)->err, "%s failed: %s", #call, hipGetErrorString(e_));            \
      (sim)->broken = true;                                                           \
      return IB_LBM_E_DEVICE;                                                         \
    }                                                                                 \
  } while (0)

ib_lbm_status dev_alloc(ib_lbm_sim *s, DevBuf *b, size_t bytes) {
  b->bytes = bytes;
  if (bytes == 0) return IB_LBM_OK;
  if (s->cfg.alloc && s->cfg.alloc->alloc) {
    b->p = s->cfg.alloc->alloc(s->cfg.alloc->ctx, bytes, (void *)s->stream);
    if (!b->p) {
      set_err(&s->err, "allocator returned NULL for %zu bytes", bytes);
      return IB_LBM_E_NOMEM;
    }
    return IB_LBM_OK;
  }
  hipError_t e = hipMalloc(&b->p, bytes);
  if (e != hipSuccess) {
    b->p = nullptr;
    set_err(&s->err, "hipMalloc(%zu) failed: %s", bytes, hipGetErrorString(e));
    return e == hipErrorOutOfMemory ? IB_LBM_E_NOMEM : IB_LBM_E_DEVICE;
  }
  return IB_LBM_OK;
}

void dev_free(ib_lbm_sim *s, DevBuf *b) {
  if (!b->p) return;
  if (s->cfg.alloc && s->cfg.alloc->free) s->cfg.alloc->free(s->cfg.alloc->ctx, b->p, (void *)s->stream);
  else (void)hipFree(b->p);
  b->p = nullptr;
  b->bytes = 0;
}

bool is_vel(int b) { return b == IB_LBM_VEL_PARABOLIC || b == IB_LBM_VEL_UNIFORM; }

// Regularized delta (Eq. 9, 10) for host-side sizing and omega_MDF.
double host_delta(int kernel, double r) {
  const double a = std::fabs(r);
  if (kernel == IB_LBM_HAT) return a < 1.0 ? 1.0 - a : 0.0;
  if (a <= 1.0) return 0.125 * (3.0 - 2.0 * a + std::sqrt(1.0 + 4.0 * a - 4.0 * a * a));
  if (a <= 2.0) return 0.125 * (5.0 - 2.0 * a - std::sqrt(-7.0 + 12.0 * a - 4.0 * a * a));
  return 0.0;
}

// Node count of the device's row-interval support description for a body
// centred at (xc, yc) (used to size the workspace).
int support_count(double xc, double yc, double R, int nb, int ns, const std::vector<double> &ct,
                  const std::vector<double> &stab, int *rows_used) {
  const int s = ns / 2;
  const int ylo = (int)std::floor(yc - R) - ns;
  const int mr = (int)std::ceil(2 * R) + 2 * ns + 4;
  std::vector<int> lmin(mr, 1 << 30), lmax(mr, -1), rmin(mr, 1 << 30), rmax(mr, -1);
  int rmx = 0;
  for (int k = 0; k < nb; k++) {
    const double X = xc + R * ct[k], Y = yc + R * stab[k];
    const int ix0 = (int)std::floor(X) - (s - 1), iy0 = (int)std::floor(Y) - (s - 1);
    for (int j = 0; j < ns; j++) {
      const int r = iy0 + j - ylo;
      if (r < 0 || r >= mr) continue;
      rmx = std::max(rmx, r);
      if (X < xc) { lmin[r] = std::min(lmin[r], ix0); lmax[r] = std::max(lmax[r], ix0 + ns - 1); }
      else { rmin[r] = std::min(rmin[r], ix0); rmax[r] = std::max(rmax[r], ix0 + ns - 1); }
    }
  }
  int total = 0;
  for (int r = 0; r < mr; r++) {
    const bool lv = lmax[r] >= 0, rv = rmax[r] >= 0;
    if (lv && rv && rmin[r] <= lmax[r] + 1) total += std::max(lmax[r], rmax[r]) - std::min(lmin[r], rmin[r]) + 1;
    else {
      if (lv) total += lmax[r] - lmin[r] + 1;
      if (rv) total += rmax[r] - rmin[r] + 1;
    }
  }
  if (rows_used) *rows_used = rmx + 1;
  return total;
}

// omega_MDF = 1 / ||A||_inf, ||A||_inf = ds max_l sum_x D_h(x-X_l) W(x),
// W(x) = sum_m D_h(x-X_m) (Sec. 2.5.2), on a dense local box.
double host_omega_mdf(double xc, double yc, double R, int nb, int kernel, double ds,
                      const std::vector<double> &ct, const std::vector<double> &stab) {
  const int ns = kernel == IB_LBM_HAT ? 2 : 4, s = ns / 2;
  const int x0 = (int)std::floor(xc - R) - ns - 1, y0 = (int)std::floor(yc - R) - ns - 1;
  const int w = (int)std::ceil(2 * R) + 2 * ns + 4;
  std::vector<double> W((size_t)w * w, 0.0);
  std::vector<double> X(nb), Y(nb);
  for (int k = 0; k < nb; k++) { X[k] = xc + R * ct[k]; Y[k] = yc + R * stab[k]; }
  for (int k = 0; k < nb; k++) {
    const int ix0 = (int)std::floor(X[k]) - (s - 1), iy0 = (int)std::floor(Y[k]) - (s - 1);
    for (int jy = 0; jy < ns; jy++)
      for (int jx = 0; jx < ns; jx++)
        W[(size_t)(iy0 + jy - y0) * w + (ix0 + jx - x0)] +=
            host_delta(kernel, ix0 + jx - X[k]) * host_delta(kernel, iy0 + jy - Y[k]);
  }
  double mx = 0.0;
  for (int k = 0; k < nb; k++) {
    const int ix0 = (int)std::floor(X[k]) - (s - 1), iy0 = (int)std::floor(Y[k]) - (s - 1);
    double acc = 0.0;
    for (int jy = 0; jy < ns; jy++)
      for (int jx = 0; jx < ns; jx++)
        acc += W[(size_t)(iy0 + jy - y0) * w + (ix0 + jx - x0)] *
               host_delta(kernel, ix0 + jx - X[k]) * host_delta(kernel, iy0 + jy - Y[k]);
    mx = std::max(mx, acc);
  }
  return 1.0 / (ds * mx);
}

int ws_doubles_for(int scheme, int nb, int ns, int mr, int mn, int pop_bytes) {
  return ws_tab_total(scheme, nb, ns, mr, mn) + ws_dyn_doubles(scheme, nb, ns, mn, pop_bytes);
}

// LDS bytes for an IB launch: enough for the largest workspace that fits;
// bodies with larger workspaces use their global buffer.
int lds_budget(int maxws_fitting) { return maxws_fitting * 8; }

void fill_case_tiles(CaseDesc *c, const ib_lbm_launch &l) {
  const int TX = l.block_x, TY = l.block_y * l.rows_per_thread;
  c->tiles_x = (c->nx + TX - 1) / TX;
  c->tiles_y = (c->ny + TY - 1) / TY;
}

ib_lbm_status check_launch(const ib_lbm_launch *l, std::string *err) {
  if (!l || l->block_x <= 0 || l->block_x % 64 || l->block_y <= 0 || l->rows_per_thread <= 0 ||
      l->block_x * l->block_y > 1024 || l->rows_per_thread > 64 ||
      (l->ib_threads != 0 && l->ib_threads != 256 && l->ib_threads != 512 && l->ib_threads != 1024)) {
    set_err(err, "invalid launch shape");
    return IB_LBM_E_INVALID;
  }
  return IB_LBM_OK;
}

void drop_graphs(ib_lbm_sim *s) {
  for (auto &g : s->graph_exec)
    if (g) {
      (void)hipGraphExecDestroy(g);
      g = nullptr;
    }
}

// Arguments of the inner-node collide-stream of a sim stepped on its own,
// with input lattice cur; mode as in LeanArgs.
LeanArgs lean_args(const ib_lbm_sim *s, int cur, int force_on) {
  const CaseDesc &c = s->cd;
  LeanArgs a;
  memset(&a, 0, sizeof a);
  a.src = c.f[cur];
  a.dst = c.f[cur ^ 1];
  a.force = c.force;
  a.state = c.state;
  a.nx = c.nx;
  a.ny = c.ny;
  a.nseg = c.nseg;
  a.tiles_x = c.tiles_x;
  a.ntiles = c.tiles_x * c.tiles_y;
  a.rpt = s->launch.rows_per_thread;
  a.remap = s->launch.xcd_remap;
  a.force_on = force_on;
  a.htx0 = s->hold[0];
  a.hty0 = s->hold[1];
  a.hntx = s->split ? s->hold[2] : 0;
  a.hnty = s->split ? s->hold[3] : 0;
  a.omega = c.omega;
  a.s_e = c.s_e;
  a.s_o = c.s_o;
  a.s_q = c.s_q;
  a.s_eps = c.s_eps;
  a.rho0 = c.rho0;
  a.fluid_fx = c.fluid_fx;
  a.fluid_fy = c.fluid_fy;
  return a;
}

// Device tables of a sim stepped on its own: one case, its IB slots.
// Decide whether a sim's steps can be pipelined.  The collide-stream of
// the tiles away from the body (far tiles) does not read what the IB pass
// writes (its force, or its corrected populations) and is not read by it;
// only the tiles whose nodes the body's support can occupy, or that push into
// such nodes (the hold rectangle), are.  So the far tiles of step n run
// concurrently with the hold tiles and the IB pass of step n.  That needs a
// single body whose position is known in advance
// (fixed or prescribed), so that one tile rectangle covers every support of
// the run widened by two nodes (the pushes and the outlet copy that reach a
// support node start at most two nodes away), kept two nodes clear of the
// faces so that no periodic wrap or face rule reaches it from outside.
ib_lbm_status plan_split(ib_lbm_sim *s) {
  s->split = false;
  if (!s->overlap || s->bodies.size() != 1) return IB_LBM_OK;
  const ib_lbm_body_desc &d = s->bodies[0].d;
  if (d.motion == IB_LBM_FREE) return IB_LBM_OK;
  const double ax = d.motion == IB_LBM_PRESCRIBED_SIN ? std::fabs(d.amp[0]) : 0.0;
  const double ay = d.motion == IB_LBM_PRESCRIBED_SIN ? std::fabs(d.amp[1]) : 0.0;
  const double r = 0.5 * d.diameter;
  const int lo = d.kernel == IB_LBM_PESKIN4 ? 1 : 0, hi = d.kernel == IB_LBM_PESKIN4 ? 2 : 1;
  const double x0 = std::floor(d.xc - ax - r) - lo - 2, y0 = std::floor(d.yc - ay - r) - lo - 2;
  const double x1 = std::floor(d.xc + ax + r) + hi + 2, y1 = std::floor(d.yc + ay + r) + hi + 2;
  if (x0 < 2 || y0 < 2 || x1 > s->cd.nx - 3 || y1 > s->cd.ny - 3) return IB_LBM_OK;
  const int TX = s->launch.block_x, TY = s->launch.block_y * s->launch.rows_per_thread;
  const int tx0 = (int)x0 / TX, tx1 = (int)x1 / TX, ty0 = (int)y0 / TY, ty1 = (int)y1 / TY;
  const int nbox = (tx1 - tx0 + 1) * (ty1 - ty0 + 1);
  if (nbox >= s->cd.tiles_x * s->cd.tiles_y) return IB_LBM_OK;
  s->hold[0] = tx0;
  s->hold[1] = ty0;
  s->hold[2] = tx1 - tx0 + 1;
  s->hold[3] = ty1 - ty0 + 1;
  s->split = true;
  return IB_LBM_OK;
}

bool body_fast(const HostBody &hb, int spread_mode);
static bool has_zou_he(const CaseDesc &c);

// Fused steps (one launch per step, step_fused_kernel): a pipelined sim
// (plan_split) whose single body is fixed, DF or MDF on the 1024-thread IB
// kernel, with BGK or TRT and no Zou-He wall.  The hold rectangle is the
// pipelined one, in tiles of the fused shape (fbx x fby, frpt rows per
// thread): the tiles that read the IB force.
ib_lbm_status plan_fused(ib_lbm_sim *s) {
  s->fused = false;
  if (!s->fused_allowed || !s->split || s->bodies.size() != 1) return IB_LBM_OK;
  const HostBody &hb = s->bodies[0];
  const ib_lbm_body_desc &d = hb.d;
  if (d.motion != IB_LBM_FIXED || d.scheme == IB_LBM_DFC || hb.dev.mdf_coupled) return IB_LBM_OK;
  if (!body_fast(hb, s->spread_mode) || hb.dev.max_nodes >= 32768 || !hb.fprev.p || !hb.pstage.p)
    return IB_LBM_OK;
  if (s->cd.collision != IB_LBM_BGK && s->cd.collision != IB_LBM_TRT) return IB_LBM_OK;
  if (has_zou_he(s->cd) || pop_values(s->cd.nx, s->cd.ny) >= (int64_t)INT32_MAX) return IB_LBM_OK;
  const double r = 0.5 * d.diameter;
  const int lo = d.kernel == IB_LBM_PESKIN4 ? 1 : 0, hi = d.kernel == IB_LBM_PESKIN4 ? 2 : 1;
  const int x0 = (int)std::floor(d.xc - r) - lo - 2, y0 = (int)std::floor(d.yc - r) - lo - 2;
  const int x1 = (int)std::floor(d.xc + r) + hi + 2, y1 = (int)std::floor(d.yc + r) + hi + 2;
  const int TX = s->fbx, TY = s->fby * s->frpt;
  s->fhold[0] = x0 / TX;
  s->fhold[1] = y0 / TY;
  s->fhold[2] = x1 / TX - x0 / TX + 1;
  s->fhold[3] = y1 / TY - y0 / TY + 1;
  s->fused = true;
  return IB_LBM_OK;
}

// A body runs on the 1024-thread IB kernel when it is DF/MDF, its workspace
// fits in LDS and spreading is by gather; the choice depends on the body
// alone, so a body's results do not depend on its batch-mates.
bool body_fast(const HostBody &hb, int spread_mode) {
  return spread_mode == 0 && hb.dev.scheme != kDFC && hb.dev.ws_doubles * 8 <= ibm_max_lds_bytes();
}

// The IB launches of a step: slots [0, nfast) on the 1024-thread kernel,
// the rest on the general one (bodies of one case may sit in both; the last
// of a case's workgroups to finish, in either launch, completes the case).
hipError_t launch_ibm_slots(int precision, const CaseDesc *cases, const IbmSlot *slots, int nfast, int n,
                            int lds_bytes, int spread_mode, int threads, hipStream_t stream) {
  hipError_t e = launch_ibm(precision, cases, slots, nfast, lds_bytes, spread_mode, 1, 1, nullptr,
                            threads, stream);
  if (e != hipSuccess) return e;
  return launch_ibm(precision, cases, slots + nfast, n - nfast, lds_bytes, spread_mode, 0, 1, nullptr,
                    threads, stream);
}

ib_lbm_status build_sim_tables(ib_lbm_sim *s) {
  if (!s->tables_dirty) return IB_LBM_OK;
  ib_lbm_status st0;
  std::vector<BodyDesc> bd;
  int maxws = 0;
  for (auto &hb : s->bodies) {
    bd.push_back(hb.dev);
    if (hb.dev.ws_doubles * 8 <= ibm_max_lds_bytes()) maxws = std::max(maxws, hb.dev.ws_doubles);
  }
  if (!bd.empty()) {
    if (!s->d_bodies.p || s->d_bodies.bytes < bd.size() * sizeof(BodyDesc)) {
      dev_free(s, &s->d_bodies);
      ib_lbm_status st = dev_alloc(s, &s->d_bodies, bd.size() * sizeof(BodyDesc));
      if (st) return st;
    }
    HIPCHK(s, hipMemcpy(s->d_bodies.p, bd.data(), bd.size() * sizeof(BodyDesc), hipMemcpyHostToDevice));
  }
  s->cd.bodies = (BodyDesc *)s->d_bodies.p;
  s->cd.nbodies = (int)bd.size();
  fill_case_tiles(&s->cd, s->launch);
  if (!s->d_case.p) {
    ib_lbm_status st = dev_alloc(s, &s->d_case, sizeof(CaseDesc));
    if (st) return st;
    st = dev_alloc(s, &s->d_prefix, sizeof(int32_t) * 4);
    if (st) return st;
    st = dev_alloc(s, &s->d_slots, sizeof(IbmSlot) * kMaxBodiesPerCase);
    if (st) return st;
  }
  HIPCHK(s, hipMemcpy(s->d_case.p, &s->cd, sizeof(CaseDesc), hipMemcpyHostToDevice));
  // tile prefix {0, tiles}, then face workgroup prefix {0, face workgroups}
  int32_t pre[4] = {0, s->cd.tiles_x * s->cd.tiles_y, 0, face_blocks(s->cd.nx, s->cd.ny)};
  HIPCHK(s, hipMemcpy(s->d_prefix.p, pre, sizeof pre, hipMemcpyHostToDevice));
  std::vector<IbmSlot> slots, rest;
  const int n = std::max(1, (int)bd.size());
  // the bodies of a coupled MDF case meet during their passes, so they run
  // in one launch: the fast instance only if every one of them fits it
  bool all_fast = !bd.empty();
  for (int b = 0; b < (int)bd.size(); b++) all_fast &= body_fast(s->bodies[b], s->spread_mode);
  const bool coupled = !bd.empty() && bd[0].mdf_coupled;
  for (int b = 0; b < n; b++) {
    const IbmSlot sl{0, bd.empty() ? -1 : b, n, 0};
    const bool fast = !bd.empty() && (coupled ? all_fast : body_fast(s->bodies[b], s->spread_mode));
    if (fast) slots.push_back(sl);
    else rest.push_back(sl);
  }
  s->nslots_fast = (int)slots.size();
  slots.insert(slots.end(), rest.begin(), rest.end());
  HIPCHK(s, hipMemcpy(s->d_slots.p, slots.data(), slots.size() * sizeof(IbmSlot), hipMemcpyHostToDevice));
  s->nslots = n;
  s->lds_bytes = lds_budget(maxws);
  if ((st0 = plan_split(s))) return st0;
  if ((st0 = plan_fused(s))) return st0;
  s->tables_dirty = false;
  drop_graphs(s);
  return IB_LBM_OK;
}

EventPair take_pair(Timing &t) {
  if (!t.pool.empty()) {
    EventPair p = t.pool.back();
    t.pool.pop_back();
    return p;
  }
  EventPair p;
  // timing events around device work: a device-scope release keeps the
  // cache writeback of a system-scope release out of the measured span
  (void)hipEventCreateWithFlags(&p.a, hipEventReleaseToDevice);
  (void)hipEventCreateWithFlags(&p.b, hipEventReleaseToDevice);
  return p;
}

// Zero-gradient faces other than the east one need the general copy rules
// of the face kernel.
static bool general_zero_gradient(const CaseDesc &c) {
  return c.bc[0] == kZeroGradient || c.bc[2] == kZeroGradient || c.bc[3] == kZeroGradient;
}

static bool has_zou_he(const CaseDesc &c) {
  return c.bc[0] == kZouHe || c.bc[1] == kZouHe || c.bc[2] == kZouHe || c.bc[3] == kZouHe;
}

// Enqueue one step of a sim on `stream` whose input lattice is cur:
// collide-stream, face nodes, Zou-He walls, then the IB pass.
ib_lbm_status enqueue_sim_step(ib_lbm_sim *s, bool timed, hipStream_t stream, int cur) {
  LaunchShape sh{s->launch.block_x, s->launch.block_y, s->launch.rows_per_thread, s->launch.xcd_remap};
  EventPair p0{}, p1{};
  if (timed) {
    p0 = take_pair(s->timing);
    HIPCHK(s, hipEventRecord(p0.a, stream));
  }
  HIPCHK(s, launch_collide_stream_lean(s->cd.precision, s->cd.collision, lean_args(s, cur, 1), 0, sh,
                                       stream));
  if (timed) {
    HIPCHK(s, hipEventRecord(p0.b, stream));
    s->timing.ev[0].push_back(p0);
  }
  HIPCHK(s, launch_collide_stream_faces(s->cd.precision, s->cd.collision, (const CaseDesc *)s->d_case.p,
                                        (const int32_t *)s->d_prefix.p + 2, 1,
                                        face_blocks(s->cd.nx, s->cd.ny), cur, 1,
                                        general_zero_gradient(s->cd), stream));
  if (has_zou_he(s->cd))
    HIPCHK(s, launch_zou_he(s->cd.precision, (const CaseDesc *)s->d_case.p, s->cd.nx, s->cd.ny, cur,
                            stream));
  if (timed) {
    p1 = take_pair(s->timing);
    HIPCHK(s, hipEventRecord(p1.a, stream));
  }
  HIPCHK(s, launch_ibm_slots(s->cd.precision, (const CaseDesc *)s->d_case.p, (const IbmSlot *)s->d_slots.p,
                             s->nslots_fast, s->nslots, s->lds_bytes, s->spread_mode,
                             s->launch.ib_threads, stream));
  if (timed) {
    HIPCHK(s, hipEventRecord(p1.b, stream));
    s->timing.ev[1].push_back(p1);
  }
  return IB_LBM_OK;
}

ib_lbm_status read_state(ib_lbm_sim *s, CaseState *cs);

// The two streams and the events of pipelined steps, created at the first
// pipelined step (sims stepped through a batch never need them).
ib_lbm_status ensure_pipe_streams(ib_lbm_sim *s) {
  if (!s->lq) {
    // The far-tile stream leaves one compute unit per IB workgroup to the
    // other stream, so that an IB pass never waits for a free unit behind a
    // full far-tile launch.
    int dev = 0, ncu = 0;
    HIPCHK(s, hipGetDevice(&dev));
    HIPCHK(s, hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev));
    std::vector<uint32_t> mask((ncu + 31) / 32, 0u);
    for (int i = 0; i < ncu - s->nslots; i++) mask[i / 32] |= 1u << (i % 32);
    if (ncu <= s->nslots ||
        hipExtStreamCreateWithCUMask(&s->lq, (uint32_t)mask.size(), mask.data()) != hipSuccess) {
      (void)hipGetLastError();
      s->lq = nullptr;
      HIPCHK(s, hipStreamCreateWithFlags(&s->lq, hipStreamNonBlocking));
    }
  }
  if (!s->iq) HIPCHK(s, hipStreamCreateWithFlags(&s->iq, hipStreamNonBlocking));
  if (!s->ticket.p) {
    // the replicated IB workgroup's counter, advanced by every copy
    ib_lbm_status st = dev_alloc(s, &s->ticket, 256);
    if (st) return st;
    HIPCHK(s, hipMemsetAsync(s->ticket.p, 0, 256, s->stream));
  }
  // the events only order work between streams of this device: a
  // device-scope release suffices (the default system-scope release writes
  // back and invalidates the caches at every record)
  const unsigned evf = hipEventDisableTiming | hipEventReleaseToDevice;
  if (!s->ev_start) HIPCHK(s, hipEventCreateWithFlags(&s->ev_start, evf));
  if (!s->ev_lq) HIPCHK(s, hipEventCreateWithFlags(&s->ev_lq, evf));
  if (!s->ev_iq) HIPCHK(s, hipEventCreateWithFlags(&s->ev_iq, evf));
  if (!s->ev_near) HIPCHK(s, hipEventCreateWithFlags(&s->ev_near, evf));
  if (!s->ev_far) HIPCHK(s, hipEventCreateWithFlags(&s->ev_far, evf));
  return IB_LBM_OK;
}

// Enqueue nsteps pipelined steps after the work already on `main`, the
// first with input lattice cur0.  Step n: the hold tiles and then the IB
// pass on iq, the far tiles, face nodes and Zou-He walls on lq.  The far
// tiles of step n follow the hold tiles of step n-1 (which push into far
// nodes and whose inputs the far tiles of step n overwrite); the hold tiles
// of step n follow the far tiles and face nodes of step n-1 for the same
// two reasons, and the IB pass of step n-1 by stream order.  The Zou-He
// wall pass of step n rebuilds wall nodes from the pushes of every node
// next to them, so it also follows the hold tiles of step n (rounded to
// whole tiles, the hold rectangle can reach row 1 or column 1).  `main`
// then waits for both streams.  Nothing here reads device state.
ib_lbm_status enqueue_pipelined(ib_lbm_sim *s, int64_t nsteps, bool timed, hipStream_t main, int cur0) {
  if (nsteps <= 0) return IB_LBM_OK;
  LaunchShape sh{s->launch.block_x, s->launch.block_y, s->launch.rows_per_thread, s->launch.xcd_remap};
  const bool zh = has_zou_he(s->cd);
  HIPCHK(s, hipEventRecord(s->ev_start, main));
  HIPCHK(s, hipStreamWaitEvent(s->lq, s->ev_start, 0));
  HIPCHK(s, hipStreamWaitEvent(s->iq, s->ev_start, 0));
  const CaseDesc *dc = (const CaseDesc *)s->d_case.p;
  for (int64_t i = 0; i < nsteps; i++) {
    const int cur = cur0 ^ (int)(i & 1);
    const bool last = i + 1 == nsteps;
    const LeanArgs la = lean_args(s, cur, 0);
    EventPair p0{}, p1{};
    // Each wait is enqueued before its event is recorded again for step i:
    // the hold tiles of step i after the face nodes (and so the far tiles)
    // of step i-1, the far tiles of step i after the hold tiles of step i-1.
    if (i > 0) {
      HIPCHK(s, hipStreamWaitEvent(s->iq, s->ev_far, 0));
      HIPCHK(s, hipStreamWaitEvent(s->lq, s->ev_near, 0));
    }
    if (timed) {
      p0 = take_pair(s->timing);
      HIPCHK(s, hipEventRecord(p0.a, s->lq));
    }
    HIPCHK(s, launch_collide_stream_lean(s->cd.precision, s->cd.collision, la, 2, sh, s->lq));
    if (timed) {
      HIPCHK(s, hipEventRecord(p0.b, s->lq));
      s->timing.ev[0].push_back(p0);
    }
    // face nodes lie outside the hold rectangle's reach (plan_split); the
    // events ride on the launches themselves
    LaunchTarget face_done, hold_done;
    face_done.done = s->ev_far;
    hold_done.done = s->ev_near;
    HIPCHK(s, launch_collide_stream_faces(s->cd.precision, s->cd.collision, dc,
                                          (const int32_t *)s->d_prefix.p + 2, 1,
                                          face_blocks(s->cd.nx, s->cd.ny), cur, 0,
                                          general_zero_gradient(s->cd), s->lq, &face_done));
    HIPCHK(s, launch_collide_stream_lean(s->cd.precision, s->cd.collision, la, 1, sh, s->iq, &hold_done));
    if (zh) {
      // every push into a wall node, hold tiles included, has landed
      LaunchTarget zou_done;
      zou_done.done = last ? s->ev_lq : nullptr;
      HIPCHK(s, hipStreamWaitEvent(s->lq, s->ev_near, 0));
      HIPCHK(s, launch_zou_he(s->cd.precision, dc, s->cd.nx, s->cd.ny, cur, s->lq, &zou_done));
    }
    if (timed) {
      p1 = take_pair(s->timing);
      HIPCHK(s, hipEventRecord(p1.a, s->iq));
    }
    // one copy of the single body's IB workgroup per XCD; the first to start
    // runs the pass (the far tiles on the other stream fill the chip)
    LaunchTarget ib_done;
    ib_done.done = last ? s->ev_iq : nullptr;
    HIPCHK(s, launch_ibm(s->cd.precision, dc, (const IbmSlot *)s->d_slots.p, 1, s->lds_bytes,
                         s->spread_mode, s->nslots_fast, 8, (uint32_t *)s->ticket.p,
                         s->launch.ib_threads, s->iq, &ib_done));
    if (timed) {
      HIPCHK(s, hipEventRecord(p1.b, s->iq));
      s->timing.ev[1].push_back(p1);
    }
  }
  // the last launch on each stream carries the event the sim's stream waits for
  HIPCHK(s, hipStreamWaitEvent(main, zh ? s->ev_lq : s->ev_far, 0));
  HIPCHK(s, hipStreamWaitEvent(main, s->ev_iq, 0));
  return IB_LBM_OK;
}

// The pipelined steps as an explicitly built graph: the same kernels and
// arguments as enqueue_pipelined, with its event ordering as node
// dependencies.  Far tiles of step i after the face nodes (and Zou-He walls)
// of step i-1 and the hold tiles of step i-1; face nodes after the far
// tiles; hold tiles after the face nodes and the IB pass of step i-1;
// Zou-He walls after the face nodes and the hold tiles of the step; the IB
// pass after the hold tiles.  Launching the graph costs the host one call,
// where the events cost it two cross-stream hops per step (about 17 us
// each); the far tiles lose the compute-unit mask of their stream, which the
// IB pass's per-XCD copies make up for.  Stream capture is not used.
ib_lbm_status build_pipelined_graph(ib_lbm_sim *s, int64_t nsteps, int cur0, hipGraphExec_t *out) {
  LaunchShape sh{s->launch.block_x, s->launch.block_y, s->launch.rows_per_thread, s->launch.xcd_remap};
  const CaseDesc *dc = (const CaseDesc *)s->d_case.p;
  const bool zh = has_zou_he(s->cd);
  hipGraph_t g = nullptr;
  HIPCHK(s, hipGraphCreate(&g, 0));
  hipGraphNode_t prev_lq = nullptr, prev_hold = nullptr, prev_ib = nullptr;
  hipError_t e = hipSuccess;
  auto add = [&](std::initializer_list<hipGraphNode_t> deps, auto &&launch) -> hipGraphNode_t {
    hipGraphNode_t d[4];
    size_t n = 0;
    for (hipGraphNode_t x : deps)
      if (x) d[n++] = x;
    LaunchTarget ns{g, d, n, nullptr};
    if (e == hipSuccess) e = launch(&ns);
    return ns.node;
  };
  for (int64_t i = 0; i < nsteps && e == hipSuccess; i++) {
    const int cur = cur0 ^ (int)(i & 1);
    const LeanArgs la = lean_args(s, cur, 0);
    hipGraphNode_t far = add({prev_lq, prev_hold}, [&](LaunchTarget *ns) {
      return launch_collide_stream_lean(s->cd.precision, s->cd.collision, la, 2, sh, nullptr, ns);
    });
    hipGraphNode_t face = add({far ? far : prev_lq, far ? nullptr : prev_hold}, [&](LaunchTarget *ns) {
      return launch_collide_stream_faces(s->cd.precision, s->cd.collision, dc,
                                         (const int32_t *)s->d_prefix.p + 2, 1,
                                         face_blocks(s->cd.nx, s->cd.ny), cur, 0,
                                         general_zero_gradient(s->cd), nullptr, ns);
    });
    hipGraphNode_t lq_end = face ? face : far;
    hipGraphNode_t hold = add({prev_lq, prev_ib}, [&](LaunchTarget *ns) {
      return launch_collide_stream_lean(s->cd.precision, s->cd.collision, la, 1, sh, nullptr, ns);
    });
    if (zh) {
      hipGraphNode_t z = add({lq_end, hold}, [&](LaunchTarget *ns) {
        return launch_zou_he(s->cd.precision, dc, s->cd.nx, s->cd.ny, cur, nullptr, ns);
      });
      if (z) lq_end = z;
    }
    hipGraphNode_t ib = add({hold ? hold : prev_ib}, [&](LaunchTarget *ns) {
      return launch_ibm(s->cd.precision, dc, (const IbmSlot *)s->d_slots.p, 1, s->lds_bytes,
                        s->spread_mode, s->nslots_fast, 8, (uint32_t *)s->ticket.p,
                        s->launch.ib_threads, nullptr, ns);
    });
    if (lq_end) prev_lq = lq_end;
    if (hold) prev_hold = hold;
    if (ib) prev_ib = ib;
  }
  if (e == hipSuccess) e = hipGraphInstantiate(out, g, nullptr, nullptr, 0);
  (void)hipGraphDestroy(g);
  HIPCHK(s, e);
  return IB_LBM_OK;
}

// The nodes whose pushes reach the support of the fused sim's body, and
// their push map (BodyDesc::src), from the support the device
// built at the body's first IB pass (the hot part of its cached tables:
// the support node list nxy and its length S).  Sorted by row and column,
// so that the pass reads the lattice in runs.
ib_lbm_status build_fused_sources(ib_lbm_sim *s) {
  HostBody &hb = s->bodies[0];
  const BodyDesc &B = hb.dev;
  std::vector<double> hot((size_t)B.ws_tab_hot);
  HIPCHK(s, hipStreamSynchronize(s->stream));
  HIPCHK(s, hipMemcpy(hot.data(), hb.tab.p, hot.size() * 8, hipMemcpyDeviceToHost));
  const int32_t *ints = (const int32_t *)(hot.data() + ws_table_doubles(B.nb, B.ns));
  const int32_t *nxy = ints + B.nb * B.ns;
  const int S = ints[B.nb * B.ns + B.max_nodes + ell_width(B.ns) * B.max_nodes];
  if (S <= 0 || S > B.max_nodes) {
    set_err(&s->err, "fused step: the body's support table is not built");
    return IB_LBM_E_STATE;
  }
  std::map<int64_t, int> sup;  // (y, x) -> support index
  auto key = [](int x, int y) { return ((int64_t)y << 32) | (uint32_t)x; };
  for (int j = 0; j < S; j++) sup[key(nxy[j] & 0xffff, nxy[j] >> 16)] = j;
  static const int ex[9] = {0, 1, 0, -1, 0, 1, -1, -1, 1};
  static const int ey[9] = {0, 0, 1, 0, -1, 1, 1, -1, -1};
  std::map<int64_t, int> src;  // (y, x) of every node that pushes into the support
  for (int j = 0; j < S; j++) {
    const int x = nxy[j] & 0xffff, y = nxy[j] >> 16;
    for (int i = 0; i < 9; i++) src[key(x - ex[i], y - ey[i])] = 0;
  }
  const int n = (int)src.size();
  std::vector<SrcNode> rec(n);
  int u = 0;
  for (auto &e : src) {
    const int y = (int)(e.first >> 32), x = (int)(uint32_t)e.first;
    if (x < 1 || x > s->cd.nx - 3 || y < 1 || y > s->cd.ny - 2) {
      set_err(&s->err, "fused step: a support neighbour is not an inner node");
      return IB_LBM_E_STATE;
    }
    SrcNode &r = rec[u];
    memset(&r, 0, sizeof r);
    r.off = (int32_t)pop_node(x, y, s->cd.nseg);
    for (int i = 0; i < 9; i++) {
      auto it = sup.find(key(x + ex[i], y + ey[i]));
      r.map[i] = (int16_t)(it == sup.end() ? -1 : it->second);
    }
    u++;
  }
  dev_free(s, &hb.src);
  ib_lbm_status st = dev_alloc(s, &hb.src, (size_t)n * sizeof(SrcNode));
  if (st) return st;
  HIPCHK(s, hipMemcpy(hb.src.p, rec.data(), (size_t)n * sizeof(SrcNode), hipMemcpyHostToDevice));
  hb.dev.src = (const SrcNode *)hb.src.p;
  hb.dev.n_src = n;
  HIPCHK(s, hipMemcpy(s->d_bodies.p, &hb.dev, sizeof(BodyDesc), hipMemcpyHostToDevice));
  hb.src_ready = true;
  return IB_LBM_OK;
}

// Enqueue nsteps fused steps on `stream` from input lattice cur0: one
// launch each, ordered by the stream alone (see step_fused_kernel).
ib_lbm_status enqueue_fused(ib_lbm_sim *s, int64_t nsteps, hipStream_t stream, int cur0) {
  for (int64_t i = 0; i < nsteps; i++) {
    const int cur = cur0 ^ (int)(i & 1);
    FusedArgs fa;
    memset(&fa, 0, sizeof fa);
    fa.lean = lean_args(s, cur, 0);
    const int TX = s->fbx, TY = s->fby * s->frpt;
    fa.lean.tiles_x = (s->cd.nx + TX - 1) / TX;
    fa.lean.ntiles = fa.lean.tiles_x * ((s->cd.ny + TY - 1) / TY);
    fa.lean.rpt = s->frpt;
    fa.lean.remap = 1;
    fa.lean.htx0 = s->fhold[0];
    fa.lean.hty0 = s->fhold[1];
    fa.lean.hntx = s->fhold[2];
    fa.lean.hnty = s->fhold[3];
    fa.c = (const CaseDesc *)s->d_case.p;
    fa.face_prefix = (const int32_t *)s->d_prefix.p + 2;
    fa.nface = face_blocks(s->cd.nx, s->cd.ny);
    fa.gzg = general_zero_gradient(s->cd);
    fa.bx = s->fbx;
    fa.by = s->fby;
    fa.cur = cur;
    fa.seq = (int32_t)(++s->fused_seq);
    fa.nsrc = (s->bodies[0].dev.n_src + kFusedThreads - 1) / kFusedThreads;
    // FP32: the tiles wait for the IB pass's kinematics and tables (28.1 us
    // per step on the 2000x800 cylinder); FP64: the tiles bound the launch
    // and start at once (37.6 against 42.4 us with the same wait)
    fa.gated = s->cd.precision == IB_LBM_FP32_SHIFTED ? 1 : 0;
    fa.cd = s->cd;
    fa.bd = s->bodies[0].dev;
    HIPCHK(s, launch_step_fused(s->cd.precision, s->cd.collision, fa, s->lds_bytes, stream));
  }
  return IB_LBM_OK;
}

// Enqueue nsteps steps of a sim on `stream` from input lattice cur0,
// pipelined when the sim allows it and `pipelined` is set.
ib_lbm_status enqueue_steps(ib_lbm_sim *s, int64_t nsteps, bool timed, hipStream_t stream, int cur0,
                            bool pipelined) {
  if (s->fused && s->bodies[0].src_ready && !timed) return enqueue_fused(s, nsteps, stream, cur0);
  if (s->split && pipelined) return enqueue_pipelined(s, nsteps, timed, stream, cur0);
  for (int64_t i = 0; i < nsteps; i++) {
    ib_lbm_status st = enqueue_sim_step(s, timed, stream, cur0 ^ (int)(i & 1));
    if (st) return st;
  }
  return IB_LBM_OK;
}

ib_lbm_status usable(ib_lbm_sim *s) {
  if (!s) return IB_LBM_E_INVALID;
  if (s->broken) return IB_LBM_E_STATE;
  return IB_LBM_OK;
}

ib_lbm_status read_state(ib_lbm_sim *s, CaseState *cs) {
  HIPCHK(s, hipStreamSynchronize(s->stream));
  HIPCHK(s, hipMemcpy(cs, s->state.p, sizeof(CaseState), hipMemcpyDeviceToHost));
  s->host_cur = cs->cur;
  return IB_LBM_OK;
}

}  // namespace

extern "C" {

uint32_t ib_lbm_abi_version(void) { return IB_LBM_ABI_VERSION; }

size_t ib_lbm_footprint(const ib_lbm_config *cfg, int32_t n_bodies, const int32_t *n_markers) {
  if (!cfg) return 0;
  const size_t elem = cfg->precision == IB_LBM_FP64 ? 8 : 4;
  const size_t n = (size_t)cfg->nx * cfg->ny;
  const size_t lat = cfg->nx > 0 && cfg->ny > 0 ? (size_t)pop_values(cfg->nx, cfg->ny) : 0;
  size_t bytes = 2 * lat * elem + 2 * n * elem + sizeof(CaseState) + sizeof(CaseDesc) + 256;
  const int hist = cfg->history_capacity > 0 ? cfg->history_capacity : 4096;
  for (int b = 0; b < n_bodies; b++) {
    const int nb = n_markers ? n_markers[b] : 256;
    // workspace upper estimate (P4), marker tables, history
    const double D = nb / M_PI;
    const int mr = (int)std::ceil(D) + 12, mn = (int)(8 * M_PI * D + 8 * mr + 64);
    // (the MDF workspace may carry the marker-space velocities, 2 n_b)
    bytes += (size_t)(std::max(ws_doubles_for(kDFC, nb, 4, mr, mn, (int)elem),
                               ws_doubles_for(kMDF, nb, 4, mr, mn, (int)elem) +
                                   std::max(2 * nb, ws_coupled_doubles(nb, mn))) +
                      ws_tab_total(kMDF, nb, 4, mr, mn) + 2 * mn) * 8 +
             (size_t)nb * (8 + 1 + 2) * 8 +
             (size_t)hist * kHistCols * 8 + sizeof(BodyState) + sizeof(BodyDesc);
  }
  return bytes;
}

ib_lbm_status ib_lbm_create(const ib_lbm_config *cfg, ib_lbm_sim **out) {
  if (!cfg || !out) return IB_LBM_E_INVALID;
  *out = nullptr;
  ib_lbm_sim *s = new ib_lbm_sim();
  s->cfg = *cfg;
  auto fail = [&](ib_lbm_status st, const char *msg) {
    fprintf(stderr, "ib_lbm_create: %s\n", msg);
    ib_lbm_destroy(s);
    return st;
  };
  if (cfg->abi_version != IB_LBM_ABI_VERSION) return fail(IB_LBM_E_INVALID, "abi_version mismatch");
  if (cfg->nx < 3 || cfg->ny < 3 || (int64_t)cfg->nx * cfg->ny >= (1ll << 31) || cfg->nx >= 65535 ||
      cfg->ny >= 32767)
    return fail(IB_LBM_E_INVALID, "lattice size out of range");
  if (!(cfg->tau > 0.5) || !std::isfinite(cfg->tau)) return fail(IB_LBM_E_INVALID, "tau must exceed 1/2");
  if (cfg->precision != IB_LBM_FP64 && cfg->precision != IB_LBM_FP32_SHIFTED)
    return fail(IB_LBM_E_INVALID, "unknown precision");
  if (cfg->collision < IB_LBM_BGK || cfg->collision > IB_LBM_CMMRT)
    return fail(IB_LBM_E_INVALID, "unknown collision");
  for (int f = 0; f < 4; f++)
    if (cfg->bc[f] < IB_LBM_PERIODIC || cfg->bc[f] > IB_LBM_ZOU_HE)
      return fail(IB_LBM_E_INVALID, "unknown face closure");
  {
    bool zh = false, other = false;
    for (int f = 0; f < 4; f++) {
      zh |= cfg->bc[f] == IB_LBM_ZOU_HE;
      other |= cfg->bc[f] != IB_LBM_ZOU_HE && cfg->bc[f] != IB_LBM_PERIODIC;
    }
    if (zh && other)
      return fail(IB_LBM_E_INVALID, "Zou-He walls combine only with other Zou-He walls or periodic faces");
  }
  if ((cfg->bc[0] == IB_LBM_PERIODIC) != (cfg->bc[1] == IB_LBM_PERIODIC) ||
      (cfg->bc[2] == IB_LBM_PERIODIC) != (cfg->bc[3] == IB_LBM_PERIODIC))
    return fail(IB_LBM_E_INVALID, "periodic faces must come in pairs");

  if (cfg->bc[2] == IB_LBM_VEL_PARABOLIC || cfg->bc[3] == IB_LBM_VEL_PARABOLIC)
    return fail(IB_LBM_E_INVALID, "parabolic profile only on the west or east face");
  if (cfg->collision == IB_LBM_TRT && !(cfg->trt_magic > 0.0))
    return fail(IB_LBM_E_INVALID, "TRT needs a positive magic parameter");
  if (!(cfg->rho0 > 0.0)) return fail(IB_LBM_E_INVALID, "rho0 must be positive");
  s->stream = (hipStream_t)cfg->stream;
  if (hipGetDevice(&s->dev) != hipSuccess) return fail(IB_LBM_E_DEVICE, "no HIP device");
  CaseDesc &c = s->cd;
  memset(&c, 0, sizeof c);
  c.nx = cfg->nx;
  c.ny = cfg->ny;
  c.collision = cfg->collision;
  c.precision = cfg->precision;
  for (int f = 0; f < 4; f++) c.bc[f] = cfg->bc[f];
  c.plane = (int64_t)cfg->nx * cfg->ny;
  c.nseg = pop_segments(cfg->nx);
  c.omega = 1.0 / cfg->tau;
  // TRT (Sec. 2.2): the even rate sets the viscosity; Lambda_o = Lambda_eo / Lambda_e.
  c.s_e = 1.0 / cfg->tau;
  {
    const double lam_e = cfg->tau - 0.5;
    const double lam_o = (cfg->trt_magic > 0 ? cfg->trt_magic : 0.25) / lam_e;
    c.s_o = 1.0 / (lam_o + 0.5);
  }
  c.s_q = cfg->cm_s_q;
  c.s_eps = cfg->cm_s_eps;
  c.rho0 = cfg->rho0;
  c.u_bc = cfg->u_bc;
  c.inv_ny2 = 1.0 / ((double)cfg->ny * cfg->ny);
  c.fluid_fx = cfg->fluid_force[0];
  c.fluid_fy = cfg->fluid_force[1];
  c.grav_x = cfg->gravity[0];
  c.grav_y = cfg->gravity[1];
  const size_t elem = cfg->precision == IB_LBM_FP64 ? 8 : 4;
  ib_lbm_status st;
  const size_t lat = (size_t)pop_values(c.nx, c.ny) * elem;
  if ((st = dev_alloc(s, &s->f0, lat))) return fail(st, s->err.c_str());
  if ((st = dev_alloc(s, &s->f1, lat))) return fail(st, s->err.c_str());
  if ((st = dev_alloc(s, &s->force, 2 * (size_t)c.plane * elem))) return fail(st, s->err.c_str());
  if ((st = dev_alloc(s, &s->state, sizeof(CaseState)))) return fail(st, s->err.c_str());
  c.f[0] = s->f0.p;
  c.f[1] = s->f1.p;
  c.force = s->force.p;
  c.state = (CaseState *)s->state.p;
  CaseState cs{};
  cs.step = 0;
  cs.target = std::numeric_limits<int64_t>::max();
  cs.cur = 0;
  if (hipMemcpy(s->state.p, &cs, sizeof cs, hipMemcpyHostToDevice) != hipSuccess)
    return fail(IB_LBM_E_DEVICE, "state upload failed");
  if (launch_init_equilibrium(c, 0, s->stream) != hipSuccess ||
      launch_init_equilibrium(c, 1, s->stream) != hipSuccess ||
      hipStreamSynchronize(s->stream) != hipSuccess)
    return fail(IB_LBM_E_DEVICE, "initialisation kernel failed");
  *out = s;
  return IB_LBM_OK;
}

ib_lbm_status ib_lbm_add_body(ib_lbm_sim *s, const ib_lbm_body_desc *b, int32_t *body_id) {
  ib_lbm_status st = usable(s);
  if (st) return st;
  if (!b) return IB_LBM_E_INVALID;
  if (s->started || s->batch) {
    set_err(&s->err, "bodies can only be added before the first step");
    return IB_LBM_E_STATE;
  }
  if ((int)s->bodies.size() >= kMaxBodiesPerCase) {
    set_err(&s->err, "at most %d bodies per sim", kMaxBodiesPerCase);
    return IB_LBM_E_INVALID;
  }
  if (!(b->diameter > 0) || b->scheme < IB_LBM_DF || b->scheme > IB_LBM_DFC || b->kernel < 0 ||
      b->kernel > 1 || b->motion < 0 || b->motion > 2 || b->n_markers < 0 ||
      (b->scheme == IB_LBM_MDF && (b->mdf_iters < 1 || b->mdf_iters > 1000)) ||
      (b->scheme == IB_LBM_MDF && b->mdf_tol > 0 &&
       (b->mdf_nmin < 1 || b->mdf_nmin > b->mdf_iters)) ||
      (b->motion == IB_LBM_FREE && !(b->density_ratio > 0)) ||
      (b->integrator != IB_LBM_VERLET && b->integrator != IB_LBM_EULER_A1) ||
      (b->mdf_coupled != 0 && b->mdf_coupled != 1) ||
      (b->udes != IB_LBM_UD_RIGID && b->udes != IB_LBM_UD_TAYLOR_GREEN) ||
      (b->udes == IB_LBM_UD_TAYLOR_GREEN &&
       (b->motion != IB_LBM_FIXED || !(b->tg_k > 0) || !(b->tg_nu >= 0) || !std::isfinite(b->tg_u0)))) {
    set_err(&s->err, "invalid body description");
    return IB_LBM_E_INVALID;
  }
  if (!s->bodies.empty() && s->bodies[0].d.scheme != b->scheme) {
    set_err(&s->err, "all bodies of a sim must use the same scheme");
    return IB_LBM_E_INVALID;
  }
  const bool coupled = b->scheme == IB_LBM_MDF && b->mdf_coupled;
  if (b->scheme == IB_LBM_MDF && !s->bodies.empty()) {
    const ib_lbm_body_desc &o = s->bodies[0].d;
    if ((o.mdf_coupled != 0) != coupled ||
        (coupled && (o.mdf_iters != b->mdf_iters || (o.mdf_tol > 0) != (b->mdf_tol > 0) ||
                     (b->mdf_tol > 0 && (o.mdf_tol != b->mdf_tol || o.mdf_nmin != b->mdf_nmin))))) {
      set_err(&s->err, "coupled MDF: every body alike, with equal bounds and tolerance");
      return IB_LBM_E_INVALID;
    }
  }
  HostBody hb;
  hb.d = *b;
  BodyDesc &B = hb.dev;
  memset(&B, 0, sizeof B);
  const int nb = b->n_markers > 0 ? b->n_markers : (int)std::lround(M_PI * b->diameter);
  if (nb < 1 || nb > 32768) {
    set_err(&s->err, "marker count out of range");
    return IB_LBM_E_INVALID;
  }
  B.nb = nb;
  B.scheme = b->scheme;
  B.kernel = b->kernel;
  B.mdf_iters = b->scheme == IB_LBM_MDF ? b->mdf_iters : 1;
  B.mdf_tol = b->scheme == IB_LBM_MDF && b->mdf_tol > 0 ? b->mdf_tol : 0.0;
  B.mdf_nmin = B.mdf_tol > 0 ? b->mdf_nmin : B.mdf_iters;
  B.mdf_coupled = coupled ? 1 : 0;
  B.motion = b->motion;
  B.internal_mass = b->internal_mass;
  B.integrator = b->integrator;
  B.udes = b->udes;
  B.tg_u0 = b->tg_u0;
  B.tg_k = b->tg_k;
  B.tg_nu = b->tg_nu;
  B.ns = b->kernel == IB_LBM_HAT ? 2 : 4;
  B.radius = 0.5 * b->diameter;
  B.ds = M_PI * b->diameter / nb;
  B.dtheta = 2.0 * M_PI / nb;
  B.xc0 = b->xc;
  B.yc0 = b->yc;
  B.amp[0] = b->amp[0];
  B.amp[1] = b->amp[1];
  B.freq = b->freq;
  B.phase = b->phase;
  const double area = M_PI * B.radius * B.radius;
  B.ms = (b->motion == IB_LBM_FREE ? b->density_ratio : 1.0) * s->cfg.rho0 * area;
  B.mf = s->cfg.rho0 * area;
  B.Is = 0.5 * B.ms * B.radius * B.radius;
  // marker directions, theta_k = 2 pi k / N_b starting at angle 0
  std::vector<double> ct(nb), stb(nb);
  for (int k = 0; k < nb; k++) {
    const double th = 2.0 * M_PI * (double)k / (double)nb;
    ct[k] = std::cos(th);
    stb[k] = std::sin(th);
  }
  // every support inside the lattice at the start position
  const int sw = B.ns / 2;
  auto inside = [&](double xc, double yc) {
    for (int k = 0; k < nb; k++) {
      const double X = xc + B.radius * ct[k], Y = yc + B.radius * stb[k];
      const int ix0 = (int)std::floor(X) - (sw - 1), iy0 = (int)std::floor(Y) - (sw - 1);
      if (ix0 < 0 || iy0 < 0 || ix0 + B.ns - 1 > s->cfg.nx - 1 || iy0 + B.ns - 1 > s->cfg.ny - 1) return false;
    }
    return true;
  };
  if (!inside(b->xc, b->yc) ||
      (b->motion == IB_LBM_PRESCRIBED_SIN &&
       (!inside(b->xc + std::fabs(b->amp[0]), b->yc + std::fabs(b->amp[1])) ||
        !inside(b->xc - std::fabs(b->amp[0]), b->yc - std::fabs(b->amp[1]))))) {
    set_err(&s->err, "a marker support leaves the lattice");
    return IB_LBM_E_RANGE;
  }
  for (auto &o : s->bodies) {
    const double dx = o.d.xc - b->xc, dy = o.d.yc - b->yc;
    const double lim = o.dev.radius + B.radius + o.dev.ns + B.ns + 4.0;
    if (dx * dx + dy * dy <= lim * lim) {
      set_err(&s->err, "body supports would meet; bodies must stay apart");
      return IB_LBM_E_RANGE;
    }
  }
  // workspace sizing over sub-lattice positions of the centre, placed so
  // that every stencil lies at positive coordinates (support_count marks an
  // empty row with a negative column)
  const double c0 = std::ceil(B.radius) + 2 * B.ns + 8;
  int maxn = 0, maxr = 0;
  for (int a = 0; a < 4; a++)
    for (int q = 0; q < 4; q++) {
      int rows = 0;
      const int n = support_count(c0 + 0.25 * a + 0.0625, c0 + 0.25 * q + 0.125, B.radius, nb,
                                  B.ns, ct, stb, &rows);
      maxn = std::max(maxn, n);
      maxr = std::max(maxr, rows);
    }
  B.max_rows = (int)std::ceil(2 * B.radius) + 2 * B.ns + 4;
  B.max_nodes = maxn + maxn / 10 + 32;
  B.ws_tab = ws_tab_total(b->scheme, nb, B.ns, B.max_rows, B.max_nodes);
  B.ws_tab_hot = ws_tab_hot(b->scheme, nb, B.ns, B.max_nodes);
  B.pop_bytes = s->cfg.precision == IB_LBM_FP64 ? 8 : 4;
  B.ws_doubles = ws_doubles_for(b->scheme, nb, B.ns, B.max_rows, B.max_nodes, B.pop_bytes);
  // MDF passes in marker space (the 1024-thread instance): markers k and l
  // can share a stencil node only if they are less than ns apart in x and
  // in y, so less than ns sqrt 2 apart; on the circle of radius R that
  // bounds |l - k| by (n_b / pi) asin(ns sqrt 2 / (2 R)).  Used when the
  // band is narrow and the workspace with it still fits in LDS.
  B.mdf_band = 0;
  if (coupled) B.ws_doubles += ws_coupled_doubles(nb, B.max_nodes);
  if (b->scheme == IB_LBM_MDF && !coupled && B.ns * std::sqrt(2.0) < 2.0 * B.radius) {
    const int w = (int)std::floor(nb / M_PI * std::asin(B.ns * std::sqrt(2.0) / (2.0 * B.radius))) + 1;
    // U at the markers is new space; the band (its half, B being
    // symmetric) overlays the two node-velocity arrays
    const int extra = 2 * nb;
    if (w <= 12 && 2 * w + 1 < nb && nb * (w + 1) <= 2 * B.max_nodes &&
        (B.ws_doubles + extra) * 8 <= ibm_max_lds_bytes()) {
      B.mdf_band = w;
      B.ws_doubles += extra;
    }
  }
  // gather window: a node within s*sqrt(2) of marker k lies within angle
  // 2 asin(s / sqrt(2 R (R - s sqrt 2))) of it
  {
    const double sr = sw * std::sqrt(2.0);
    double dmax = M_PI;
    if (B.radius > sr + 0.5) dmax = 2.0 * std::asin(std::min(1.0, sw / std::sqrt(2.0 * B.radius * (B.radius - sr))));
    int w = (int)std::ceil(dmax / B.dtheta) + 2;
    if (2 * w + 1 >= nb) w = nb;
    B.window = w;
  }
  B.omega_mdf = b->scheme == IB_LBM_MDF
                    ? (b->mdf_omega > 0 ? b->mdf_omega
                                        : host_omega_mdf(b->xc, b->yc, B.radius, nb, b->kernel, B.ds, ct, stb))
                    : 1.0;
  B.hist_cap = s->cfg.history_capacity > 0 ? s->cfg.history_capacity : 4096;
  if ((st = dev_alloc(s, &hb.cos_t, nb * 8))) return st;
  if ((st = dev_alloc(s, &hb.sin_t, nb * 8))) return st;
  if ((st = dev_alloc(s, &hb.ws, (size_t)B.ws_doubles * 8))) return st;
  if ((st = dev_alloc(s, &hb.tab, (size_t)B.ws_tab * 8))) return st;
  if ((st = dev_alloc(s, &hb.acc, (size_t)B.max_nodes * 2 * 8))) return st;
  if ((st = dev_alloc(s, &hb.markers, (size_t)nb * 8 * 8))) return st;
  if ((st = dev_alloc(s, &hb.lambda, (size_t)nb * 8))) return st;
  if ((st = dev_alloc(s, &hb.history, (size_t)B.hist_cap * kHistCols * 8))) return st;
  if ((st = dev_alloc(s, &hb.state, sizeof(BodyState)))) return st;
  HIPCHK(s, hipMemcpy(hb.cos_t.p, ct.data(), nb * 8, hipMemcpyHostToDevice));
  HIPCHK(s, hipMemcpy(hb.sin_t.p, stb.data(), nb * 8, hipMemcpyHostToDevice));
  HIPCHK(s, hipMemset(hb.markers.p, 0, (size_t)nb * 64));
  HIPCHK(s, hipMemset(hb.history.p, 0, (size_t)B.hist_cap * kHistCols * 8));
  B.cos_t = (const double *)hb.cos_t.p;
  B.sin_t = (const double *)hb.sin_t.p;
  B.ws = (double *)hb.ws.p;
  B.tab_cache = (double *)hb.tab.p;
  B.acc = (double *)hb.acc.p;
  B.markers_out = (double *)hb.markers.p;
  B.lambda_cache = (double *)hb.lambda.p;
  B.history = (double *)hb.history.p;
  B.state = (BodyState *)hb.state.p;
  B.src = nullptr;
  B.n_src = 0;
  B.fprev = nullptr;
  B.pstage = nullptr;
  if (b->motion == IB_LBM_FIXED && b->scheme != IB_LBM_DFC) {
    // fused steps: the copy of the last force (zero, as the force field
    // starts) and the staged pushes of the support nodes
    if ((st = dev_alloc(s, &hb.fprev, (size_t)B.max_nodes * 2 * B.pop_bytes))) return st;
    if ((st = dev_alloc(s, &hb.pstage, (size_t)B.max_nodes * 9 * B.pop_bytes))) return st;
    HIPCHK(s, hipMemset(hb.fprev.p, 0, (size_t)B.max_nodes * 2 * B.pop_bytes));
    B.fprev = hb.fprev.p;
    B.pstage = hb.pstage.p;
  }
  BodyState bst;
  memset(&bst, 0, sizeof bst);
  bst.xc = b->xc;
  bst.yc = b->yc;
  HIPCHK(s, hipMemcpy(hb.state.p, &bst, sizeof bst, hipMemcpyHostToDevice));
  s->bodies.push_back(hb);
  s->tables_dirty = true;
  if (body_id) *body_id = (int32_t)s->bodies.size() - 1;
  return IB_LBM_OK;
}

ib_lbm_status ib_lbm_step(ib_lbm_sim *s, int64_t nsteps) {
  ib_lbm_status st = usable(s);
  if (st) return st;
  if (nsteps < 0) return IB_LBM_E_INVALID;
  if (s->batch) {
    set_err(&s->err, "sim is attached to a batch; step the batch");
    return IB_LBM_E_STATE;
  }
  if ((st = build_sim_tables(s))) return st;
  if (s->split && (st = ensure_pipe_streams(s))) return st;
  s->started = true;
  int64_t left = nsteps;
  if (s->fused && !s->bodies[0].src_ready && left > 0 && !s->timing.on) {
    // fused steps start from the support the device builds at the body's
    // first IB pass: one pipelined step first if none has run
    if (s->host_steps == 0) {
      if ((st = enqueue_steps(s, 1, false, s->stream, s->host_cur, true))) return st;
      s->host_cur ^= 1;
      left -= 1;
    }
    st = build_fused_sources(s);
    if (st == IB_LBM_E_STATE) {
      // no support table (a halted case): pipelined steps
      s->fused = false;
      st = IB_LBM_OK;
    }
    if (st) return st;
  }
  if (s->graph_steps > 0 && !s->timing.on && left >= s->graph_steps) {
    if (s->graph_len != s->graph_steps) {
      drop_graphs(s);
      s->graph_len = s->graph_steps;
    }
    // pipelined steps: an explicitly built graph per starting lattice, both
    // made at the first replay; plain steps: captured on a private stream
    // (the caller's may be the null stream); replayed on the caller's stream
    if (s->split && !s->fused) {
      for (int p = 0; p < 2; p++)
        if (!s->graph_exec[p] && (st = build_pipelined_graph(s, s->graph_len, p, &s->graph_exec[p])))
          return st;
    }
    if (!s->cap_stream) HIPCHK(s, hipStreamCreateWithFlags(&s->cap_stream, hipStreamNonBlocking));
    while (left >= s->graph_len) {
      hipGraphExec_t &ge = s->graph_exec[s->host_cur];
      if (!ge) {
        hipGraph_t g;
        HIPCHK(s, hipStreamBeginCapture(s->cap_stream, hipStreamCaptureModeThreadLocal));
        // captured steps are plain steps on the capturing stream: capturing
        // the two-stream pipelined step crashed the host process in the HIP
        // runtime (cause not identified), so pipelined graphs are built
        // explicitly above instead
        st = enqueue_steps(s, s->graph_len, false, s->cap_stream, s->host_cur, false);
        if (st) {
          hipGraph_t dummy;
          (void)hipStreamEndCapture(s->cap_stream, &dummy);
          return st;
        }
        HIPCHK(s, hipStreamEndCapture(s->cap_stream, &g));
        HIPCHK(s, hipGraphInstantiate(&ge, g, nullptr, nullptr, 0));
        (void)hipGraphDestroy(g);
      }
      HIPCHK(s, hipGraphLaunch(ge, s->stream));
      left -= s->graph_len;
      s->host_cur ^= s->graph_len & 1;
    }
  }
  if (left > 0) {
    if ((st = enqueue_steps(s, left, s->timing.on, s->stream, s->host_cur, true))) return st;
    s->host_cur ^= (int)(left & 1);
  }
  s->host_steps += nsteps;
  return IB_LBM_OK;
}

ib_lbm_status ib_lbm_forces(ib_lbm_sim *s, int32_t body_id, ib_lbm_body_state *out) {
  ib_lbm_status st = usable(s);
  if (st) return st;
  if (!out || body_id < 0 || body_id >= (int)s->bodies.size()) return IB_LBM_E_INVALID;
  CaseState cs;
  if ((st = read_state(s, &cs))) return st;
  BodyState b;
  HIPCHK(s, hipMemcpy(&b, s->bodies[body_id].state.p, sizeof b, hipMemcpyDeviceToHost));
  out->step = cs.step;
  out->fx = b.fhx;
  out->fy = b.fhy;
  out->torque = b.torque;
  out->xc = b.xc;
  out->yc = b.yc;
  const bool freeb = s->bodies[body_id].d.motion == IB_LBM_FREE;
  out->vx = freeb ? b.vx : b.vhx;
  out->vy = freeb ? b.vy : b.vhy;
  out->omega = freeb ? b.om : b.omh;
  out->slip_mean = b.slip_mean;
  out->slip_max = b.slip_max;
  out->mdf_residual = b.mdf_res;
  out->mdf_omega = s->bodies[body_id].dev.omega_mdf;
  out->mdf_iters = b.mdf_iters_done;
  out->flags = b.flags;
  if (b.flags & IB_LBM_FLAG_NONFINITE) {
    set_err(&s->err, "non-finite force or velocity at body %d", body_id);
    return IB_LBM_E_DIVERGED;
  }
  if (b.flags & kFlagExchange) {
    set_err(&s->err, "body %d: the coupled MDF workgroups of the case did not meet (flags %d)",
            body_id, b.flags);
    return IB_LBM_E_STATE;
  }
  if (b.flags & (IB_LBM_FLAG_RANGE | IB_LBM_FLAG_OVERLAP | kFlagCapacity)) {
    if (b.flags & kFlagCapacity)
      set_err(&s->err, "body %d outgrew its support tables (flags %d): fewer markers or a smaller body",
              body_id, b.flags);
    else
      set_err(&s->err, "body %d left the lattice or met another body (flags %d)", body_id, b.flags);
    return IB_LBM_E_RANGE;
  }
  return IB_LBM_OK;
}

ib_lbm_status ib_lbm_history(ib_lbm_sim *s, int32_t body_id, int64_t first, int64_t count,
                             double *out) {
  ib_lbm_status st = usable(s);
  if (st) return st;
  if (!out || body_id < 0 || body_id >= (int)s->bodies.size() || count < 0 || first < 1)
    return IB_LBM_E_INVALID;
  CaseState cs;
  if ((st = read_state(s, &cs))) return st;
  const int cap = s->bodies[body_id].dev.hist_cap;
  if (first + count - 1 > cs.step || first <= cs.step - cap) {
    set_err(&s->err, "history rows outside the kept window");
    return IB_LBM_E_RANGE;
  }
  const double *h = (const double *)s->bodies[body_id].history.p;
  // the rows lie in the ring in at most two runs (before and after the wrap)
  for (int64_t i = 0; i < count;) {
    const int64_t row = (first - 1 + i) % cap;
    const int64_t run = std::min<int64_t>(count - i, cap - row);
    HIPCHK(s, hipMemcpy(out + i * kHistCols, h + row * kHistCols, (size_t)run * kHistCols * 8,
                        hipMemcpyDeviceToHost));
    i += run;
  }
  return IB_LBM_OK;
}

static ib_lbm_status ensure_tmp(ib_lbm_sim *s, size_t bytes) {
  if (s->d_tmp.bytes >= bytes) return IB_LBM_OK;
  dev_free(s, &s->d_tmp);
  return dev_alloc(s, &s->d_tmp, bytes);
}

ib_lbm_status ib_lbm_fields(ib_lbm_sim *s, double *rho, double *ux, double *uy) {
  ib_lbm_status st = usable(s);
  if (st) return st;
  if (!rho || !ux || !uy) return IB_LBM_E_INVALID;
  CaseState cs;
  if ((st = read_state(s, &cs))) return st;
  const size_t n = (size_t)s->cd.plane;
  if ((st = ensure_tmp(s, 3 * n * 8))) return st;
  double *d = (double *)s->d_tmp.p;
  HIPCHK(s, launch_fields(s->cd, cs.cur, d, d + n, d + 2 * n, s->stream));
  HIPCHK(s, hipStreamSynchronize(s->stream));
  HIPCHK(s, hipMemcpy(rho, d, n * 8, hipMemcpyDeviceToHost));
  HIPCHK(s, hipMemcpy(ux, d + n, n * 8, hipMemcpyDeviceToHost));
  HIPCHK(s, hipMemcpy(uy, d + 2 * n, n * 8, hipMemcpyDeviceToHost));
  return IB_LBM_OK;
}

ib_lbm_status ib_lbm_get_populations(ib_lbm_sim *s, double *f) {
  ib_lbm_status st = usable(s);
  if (st) return st;
  if (!f) return IB_LBM_E_INVALID;
  CaseState cs;
  if ((st = read_state(s, &cs))) return st;
  const size_t n = (size_t)s->cd.plane;
  if ((st = ensure_tmp(s, 9 * n * 8))) return st;
  HIPCHK(s, launch_export(s->cd, cs.cur, (double *)s->d_tmp.p, s->stream));
  HIPCHK(s, hipStreamSynchronize(s->stream));
  HIPCHK(s, hipMemcpy(f, s->d_tmp.p, 9 * n * 8, hipMemcpyDeviceToHost));
  return IB_LBM_OK;
}

ib_lbm_status ib_lbm_set_populations(ib_lbm_sim *s, const double *f) {
  ib_lbm_status st = usable(s);
  if (st) return st;
  if (!f) return IB_LBM_E_INVALID;
  CaseState cs;
  if ((st = read_state(s, &cs))) return st;
  const size_t n = (size_t)s->cd.plane;
  if ((st = ensure_tmp(s, 9 * n * 8))) return st;
  HIPCHK(s, hipMemcpy(s->d_tmp.p, f, 9 * n * 8, hipMemcpyHostToDevice));
  HIPCHK(s, launch_import(s->cd, cs.cur, (const double *)s->d_tmp.p, s->stream));
  HIPCHK(s, hipStreamSynchronize(s->stream));
  return IB_LBM_OK;
}

ib_lbm_status ib_lbm_set_equilibrium(ib_lbm_sim *s, const double *rho, const double *ux,
                                    const double *uy) {
  ib_lbm_status st = usable(s);
  if (st) return st;
  if (!ux || !uy) return IB_LBM_E_INVALID;
  CaseState cs;
  if ((st = read_state(s, &cs))) return st;
  const size_t n = (size_t)s->cd.plane;
  if ((st = ensure_tmp(s, 3 * n * 8))) return st;
  double *d = (double *)s->d_tmp.p;
  HIPCHK(s, hipMemcpy(d, ux, n * 8, hipMemcpyHostToDevice));
  HIPCHK(s, hipMemcpy(d + n, uy, n * 8, hipMemcpyHostToDevice));
  if (rho) HIPCHK(s, hipMemcpy(d + 2 * n, rho, n * 8, hipMemcpyHostToDevice));
  HIPCHK(s, launch_set_equilibrium(s->cd, cs.cur, rho ? d + 2 * n : nullptr, d, d + n, s->stream));
  HIPCHK(s, hipStreamSynchronize(s->stream));
  return IB_LBM_OK;
}

ib_lbm_status ib_lbm_force_field(ib_lbm_sim *s, double *fx, double *fy) {
  ib_lbm_status st = usable(s);
  if (st) return st;
  if (!fx || !fy) return IB_LBM_E_INVALID;
  CaseState cs;
  if ((st = read_state(s, &cs))) return st;
  const size_t n = (size_t)s->cd.plane;
  if ((st = ensure_tmp(s, 2 * n * 8))) return st;
  double *d = (double *)s->d_tmp.p;
  HIPCHK(s, launch_force_export(s->cd, d, d + n, s->stream));
  HIPCHK(s, hipStreamSynchronize(s->stream));
  HIPCHK(s, hipMemcpy(fx, d, n * 8, hipMemcpyDeviceToHost));
  HIPCHK(s, hipMemcpy(fy, d + n, n * 8, hipMemcpyDeviceToHost));
  return IB_LBM_OK;
}

ib_lbm_status ib_lbm_markers(ib_lbm_sim *s, int32_t body_id, double *out, int32_t *n_markers) {
  ib_lbm_status st = usable(s);
  if (st) return st;
  if (body_id < 0 || body_id >= (int)s->bodies.size()) return IB_LBM_E_INVALID;
  const int nb = s->bodies[body_id].dev.nb;
  if (n_markers) *n_markers = nb;
  if (!out) return IB_LBM_OK;
  HIPCHK(s, hipStreamSynchronize(s->stream));
  HIPCHK(s, hipMemcpy(out, s->bodies[body_id].markers.p, (size_t)nb * 64, hipMemcpyDeviceToHost));
  return IB_LBM_OK;
}

}  // extern "C"

namespace {

// Diagnostics of body_id staged in device memory at d (8 + 6 n_b doubles),
// then copied to the host.  Allocates nothing.
ib_lbm_status diagnostics_into(ib_lbm_sim *s, int32_t body_id, int32_t kappa, double u_ref,
                               double *summary, double *per_marker, double *d) {
  CaseState cs;
  ib_lbm_status st;
  if ((st = read_state(s, &cs))) return st;
  if (cs.step < 1) {
    set_err(&s->err, "diagnostics need a completed step");
    return IB_LBM_E_STATE;
  }
  const HostBody &hb = s->bodies[body_id];
  BodyState b;
  HIPCHK(s, hipMemcpy(&b, hb.state.p, sizeof b, hipMemcpyDeviceToHost));
  const bool freeb = hb.d.motion == IB_LBM_FREE;
  const double vx = freeb ? b.vx : b.vhx, vy = freeb ? b.vy : b.vhy, om = freeb ? b.om : b.omh;
  if (!std::isfinite(b.xc) || !std::isfinite(b.yc) || !std::isfinite(vx) || !std::isfinite(vy) ||
      !std::isfinite(om)) {
    set_err(&s->err, "body %d has a non-finite position or velocity", body_id);
    return IB_LBM_E_DIVERGED;
  }
  const int nb = hb.dev.nb;
  HIPCHK(s, launch_diagnostics(s->cd, cs.cur, (const double *)hb.markers.p, nb, b.xc, b.yc, vx, vy,
                               om, hb.dev.radius, hb.dev.ds, kappa, u_ref, d, d + 8, s->stream));
  HIPCHK(s, hipStreamSynchronize(s->stream));
  HIPCHK(s, hipMemcpy(summary, d, 8 * 8, hipMemcpyDeviceToHost));
  if (per_marker) HIPCHK(s, hipMemcpy(per_marker, d + 8, (size_t)nb * 6 * 8, hipMemcpyDeviceToHost));
  return IB_LBM_OK;
}

}  // namespace

extern "C" {

ib_lbm_status ib_lbm_diagnostics(ib_lbm_sim *s, int32_t body_id, int32_t kappa, double u_ref,
                                 double *summary, double *per_marker) {
  ib_lbm_status st = usable(s);
  if (st) return st;
  if (!summary || body_id < 0 || body_id >= (int)s->bodies.size() || kappa < 0 || !(u_ref > 0))
    return IB_LBM_E_INVALID;
  if (s->bodies[body_id].d.udes != IB_LBM_UD_RIGID) {
    set_err(&s->err, "boundary diagnostics are defined for rigid bodies");
    return IB_LBM_E_INVALID;
  }
  const int nb = s->bodies[body_id].dev.nb;
  if ((st = ensure_tmp(s, (size_t)(8 + 6 * nb) * 8))) return st;
  return diagnostics_into(s, body_id, kappa, u_ref, summary, per_marker, (double *)s->d_tmp.p);
}

ib_lbm_status ib_lbm_diagnostics_noalloc(ib_lbm_sim *s, int32_t body_id, int32_t kappa, double u_ref,
                                         double *summary, double *per_marker) {
  ib_lbm_status st = usable(s);
  if (st) return st;
  if (!summary || body_id < 0 || body_id >= (int)s->bodies.size() || kappa < 0 || !(u_ref > 0))
    return IB_LBM_E_INVALID;
  if (s->bodies[body_id].d.udes != IB_LBM_UD_RIGID) {
    set_err(&s->err, "boundary diagnostics are defined for rigid bodies");
    return IB_LBM_E_INVALID;
  }
  const int nb = s->bodies[body_id].dev.nb;
  if (nb > diag_scratch_markers()) {
    set_err(&s->err, "ib_lbm_diagnostics_noalloc: %d markers exceed the static staging of %d", nb,
            diag_scratch_markers());
    return IB_LBM_E_INVALID;
  }
  // the staging of the sim's device, its address taken once per device
  int dev = 0;
  HIPCHK(s, hipGetDevice(&dev));
  if (dev != s->dev) HIPCHK(s, hipSetDevice(s->dev));
  double *d = nullptr;
  hipError_t e = diag_scratch(&d);
  if (e == hipSuccess) st = diagnostics_into(s, body_id, kappa, u_ref, summary, per_marker, d);
  if (dev != s->dev) (void)hipSetDevice(dev);
  HIPCHK(s, e);
  return st;
}

ib_lbm_status ib_lbm_steps_done(ib_lbm_sim *s, int64_t *steps) {
  ib_lbm_status st = usable(s);
  if (st) return st;
  if (!steps) return IB_LBM_E_INVALID;
  CaseState cs;
  if ((st = read_state(s, &cs))) return st;
  *steps = cs.step;
  return IB_LBM_OK;
}

ib_lbm_status ib_lbm_sync(ib_lbm_sim *s) {
  ib_lbm_status st = usable(s);
  if (st) return st;
  HIPCHK(s, hipStreamSynchronize(s->stream));
  return IB_LBM_OK;
}

ib_lbm_status ib_lbm_destroy(ib_lbm_sim *s) {
  if (!s) return IB_LBM_E_INVALID;
  if (s->batch) ib_lbm_batch_detach(s->batch, s);
  if (s->stream) (void)hipStreamSynchronize(s->stream);
  drop_graphs(s);
  if (s->lq) (void)hipStreamSynchronize(s->lq);
  if (s->iq) (void)hipStreamSynchronize(s->iq);
  for (int k = 0; k < kTimingKinds; k++)
    for (auto &p : s->timing.ev[k]) { (void)hipEventDestroy(p.a); (void)hipEventDestroy(p.b); }
  for (auto &p : s->timing.pool) { (void)hipEventDestroy(p.a); (void)hipEventDestroy(p.b); }
  for (auto &hb : s->bodies) {
    dev_free(s, &hb.cos_t); dev_free(s, &hb.sin_t); dev_free(s, &hb.ws); dev_free(s, &hb.markers);
    dev_free(s, &hb.tab); dev_free(s, &hb.acc);
    dev_free(s, &hb.lambda); dev_free(s, &hb.history); dev_free(s, &hb.state);
    dev_free(s, &hb.fprev); dev_free(s, &hb.pstage); dev_free(s, &hb.src);
  }
  dev_free(s, &s->f0); dev_free(s, &s->f1); dev_free(s, &s->force); dev_free(s, &s->state);
  dev_free(s, &s->ticket);
  dev_free(s, &s->d_bodies); dev_free(s, &s->d_case); dev_free(s, &s->d_prefix);
  dev_free(s, &s->d_slots); dev_free(s, &s->d_tmp);
  if (s->cap_stream) (void)hipStreamDestroy(s->cap_stream);
  if (s->lq) (void)hipStreamDestroy(s->lq);
  if (s->iq) (void)hipStreamDestroy(s->iq);
  if (s->ev_start) (void)hipEventDestroy(s->ev_start);
  if (s->ev_lq) (void)hipEventDestroy(s->ev_lq);
  if (s->ev_iq) (void)hipEventDestroy(s->ev_iq);
  if (s->ev_near) (void)hipEventDestroy(s->ev_near);
  if (s->ev_far) (void)hipEventDestroy(s->ev_far);
  delete s;
  return IB_LBM_OK;
}

const char *ib_lbm_last_error(const ib_lbm_sim *s) { return s ? s->err.c_str() : "null sim"; }

ib_lbm_status ib_lbm_set_launch(ib_lbm_sim *s, const ib_lbm_launch *l) {
  ib_lbm_status st = usable(s);
  if (st) return st;
  if ((st = check_launch(l, &s->err))) return st;
  s->launch = *l;
  s->tables_dirty = true;
  return IB_LBM_OK;
}

ib_lbm_status ib_lbm_get_launch(const ib_lbm_sim *s, ib_lbm_launch *l) {
  if (!s || !l) return IB_LBM_E_INVALID;
  *l = s->launch;
  return IB_LBM_OK;
}

ib_lbm_status ib_lbm_set_spread(ib_lbm_sim *s, int32_t mode) {
  ib_lbm_status st = usable(s);
  if (st) return st;
  if (mode != IB_LBM_SPREAD_GATHER && mode != IB_LBM_SPREAD_ATOMIC) return IB_LBM_E_INVALID;
  s->spread_mode = mode;
  s->tables_dirty = true;
  return IB_LBM_OK;
}

ib_lbm_status ib_lbm_set_overlap(ib_lbm_sim *s, int32_t on) {
  ib_lbm_status st = usable(s);
  if (st) return st;
  if (on != 0 && on != 1) return IB_LBM_E_INVALID;
  HIPCHK(s, hipStreamSynchronize(s->stream));
  s->overlap = on != 0;
  s->tables_dirty = true;
  return IB_LBM_OK;
}

ib_lbm_status ib_lbm_get_overlap(const ib_lbm_sim *s, int32_t *in_use, int64_t *near_nodes) {
  if (!s || !in_use) return IB_LBM_E_INVALID;
  *in_use = s->split ? 1 : 0;
  if (near_nodes) {
    int64_t n = 0;
    if (s->split) {
      const int TX = s->launch.block_x, TY = s->launch.block_y * s->launch.rows_per_thread;
      const int64_t x0 = (int64_t)s->hold[0] * TX, y0 = (int64_t)s->hold[1] * TY;
      const int64_t x1 = std::min<int64_t>(x0 + (int64_t)s->hold[2] * TX, s->cd.nx);
      const int64_t y1 = std::min<int64_t>(y0 + (int64_t)s->hold[3] * TY, s->cd.ny);
      n = (x1 - x0) * (y1 - y0);
    }
    *near_nodes = n;
  }
  return IB_LBM_OK;
}

ib_lbm_status ib_lbm_set_fused(ib_lbm_sim *s, int32_t on) {
  ib_lbm_status st = usable(s);
  if (st) return st;
  if (on != 0 && on != 1) return IB_LBM_E_INVALID;
  HIPCHK(s, hipStreamSynchronize(s->stream));
  if (s->fused_allowed != (on != 0)) {
    s->fused_allowed = on != 0;
    s->tables_dirty = true;
  }
  return IB_LBM_OK;
}

ib_lbm_status ib_lbm_get_fused(const ib_lbm_sim *s, int32_t *in_use) {
  if (!s || !in_use) return IB_LBM_E_INVALID;
  *in_use = s->fused && !s->tables_dirty ? 1 : 0;
  return IB_LBM_OK;
}

ib_lbm_status ib_lbm_set_graph(ib_lbm_sim *s, int32_t steps_per_graph) {
  ib_lbm_status st = usable(s);
  if (st) return st;
  if (steps_per_graph < 0 || steps_per_graph > 100000) return IB_LBM_E_INVALID;
  s->graph_steps = steps_per_graph;
  return IB_LBM_OK;
}

ib_lbm_status ib_lbm_timing_enable(ib_lbm_sim *s, int32_t on) {
  ib_lbm_status st = usable(s);
  if (st) return st;
  HIPCHK(s, hipStreamSynchronize(s->stream));
  for (int k = 0; k < kTimingKinds; k++) {
    for (auto &p : s->timing.ev[k]) s->timing.pool.push_back(p);
    s->timing.ev[k].clear();
    s->timing.folded_ms[k] = 0;
    s->timing.folded_n[k] = 0;
  }
  s->timing.on = on != 0;
  return IB_LBM_OK;
}

ib_lbm_status ib_lbm_time_collide_stream(ib_lbm_sim *s, int32_t launches, double *avg_us,
                                         int64_t *inner_nodes) {
  ib_lbm_status st = usable(s);
  if (st) return st;
  if (launches <= 0 || !avg_us) return IB_LBM_E_INVALID;
  if (s->batch) {
    set_err(&s->err, "sim is attached to a batch");
    return IB_LBM_E_STATE;
  }
  if ((st = build_sim_tables(s))) return st;
  s->started = true;
  LaunchShape sh{s->launch.block_x, s->launch.block_y, s->launch.rows_per_thread, s->launch.xcd_remap};
  const LeanArgs la = lean_args(s, s->host_cur, 1);
  hipEvent_t a, b;
  HIPCHK(s, hipEventCreate(&a));
  HIPCHK(s, hipEventCreate(&b));
  hipError_t e = hipEventRecord(a, s->stream);
  for (int i = 0; i < launches && e == hipSuccess; i++)
    e = launch_collide_stream_lean(s->cd.precision, s->cd.collision, la, 0, sh, s->stream);
  if (e == hipSuccess) e = hipEventRecord(b, s->stream);
  if (e == hipSuccess) e = hipEventSynchronize(b);
  float ms = 0;
  if (e == hipSuccess) e = hipEventElapsedTime(&ms, a, b);
  (void)hipEventDestroy(a);
  (void)hipEventDestroy(b);
  HIPCHK(s, e);
  // the launches consumed the IB force: so does the copy fused steps read
  for (auto &hb : s->bodies)
    if (hb.fprev.p) HIPCHK(s, hipMemset(hb.fprev.p, 0, hb.fprev.bytes));
  *avg_us = ms * 1e3 / launches;
  if (inner_nodes) *inner_nodes = (int64_t)(s->cd.nx - 3) * (s->cd.ny - 2);
  return IB_LBM_OK;
}

ib_lbm_status ib_lbm_stream_copy(const void *src, void *dst, size_t bytes, int32_t workgroups,
                                 void *stream) {
  if (!src || !dst || src == dst || bytes == 0 || bytes % 16 || ((uintptr_t)src | (uintptr_t)dst) % 16 ||
      workgroups < 0 || workgroups > (1 << 20))
    return IB_LBM_E_INVALID;
  if (launch_stream_copy(src, dst, bytes / 16, workgroups ? workgroups : 256, (hipStream_t)stream) !=
      hipSuccess)
    return IB_LBM_E_DEVICE;
  return IB_LBM_OK;
}

ib_lbm_status ib_lbm_timing_read(ib_lbm_sim *s, int32_t which, double *total_ms, int64_t *launches) {
  ib_lbm_status st = usable(s);
  if (st) return st;
  if (which < 0 || which >= kTimingKinds || !total_ms || !launches) return IB_LBM_E_INVALID;
  HIPCHK(s, hipStreamSynchronize(s->stream));
  double ms = s->timing.folded_ms[which];
  for (auto &p : s->timing.ev[which]) {
    float t = 0;
    HIPCHK(s, hipEventElapsedTime(&t, p.a, p.b));
    ms += t;
  }
  *total_ms = ms;
  *launches = s->timing.folded_n[which] + (int64_t)s->timing.ev[which].size();
  return IB_LBM_OK;
}

// ------------------------------------------------------------------ batches
#define BHIPCHK(b, call)                                                              \
  do {                                                                                \
    hipError_t e_ = (call);                                                           \
    if (e_ != hipSuccess) {                                                           \
      set_err(&(b)->err, "%s failed: %s", #call, hipGetErrorString(e_));              \
      (b)->broken = true;                                                             \
      return IB_LBM_E_DEVICE;                                                         \
    }                                                                                 \
  } while (0)

ib_lbm_status ib_lbm_batch_create(void *stream, int32_t precision, ib_lbm_batch **out) {
  if (!out || (precision != IB_LBM_FP64 && precision != IB_LBM_FP32_SHIFTED)) return IB_LBM_E_INVALID;
  ib_lbm_batch *b = new ib_lbm_batch();
  b->stream = (hipStream_t)stream;
  b->precision = precision;
  *out = b;
  return IB_LBM_OK;
}

ib_lbm_status ib_lbm_batch_attach(ib_lbm_batch *b, ib_lbm_sim *s) {
  if (!b || !s) return IB_LBM_E_INVALID;
  if (b->broken || s->broken) return IB_LBM_E_STATE;
  if (s->batch) {
    set_err(&b->err, "sim already attached to a batch");
    return IB_LBM_E_STATE;
  }
  if (s->cd.precision != b->precision || s->stream != b->stream) {
    set_err(&b->err, "sim precision or stream differs from the batch");
    return IB_LBM_E_INVALID;
  }
  if (has_zou_he(s->cd)) {
    set_err(&b->err, "sims with Zou-He walls are stepped on their own, not in a batch");
    return IB_LBM_E_INVALID;
  }
  if (!s->bodies.empty() && s->bodies[0].dev.mdf_coupled) {
    set_err(&b->err, "sims with coupled MDF bodies are stepped on their own, not in a batch");
    return IB_LBM_E_INVALID;
  }
  ib_lbm_status st = build_sim_tables(s);
  if (st) return st;
  s->batch = b;
  s->started = true;
  b->sims.push_back(s);
  b->dirty = true;
  return IB_LBM_OK;
}

ib_lbm_status ib_lbm_batch_detach(ib_lbm_batch *b, ib_lbm_sim *s) {
  if (!b || !s) return IB_LBM_E_INVALID;
  auto it = std::find(b->sims.begin(), b->sims.end(), s);
  if (it == b->sims.end()) return IB_LBM_E_INVALID;
  if (b->stream) (void)hipStreamSynchronize(b->stream);
  b->sims.erase(it);
  s->batch = nullptr;
  b->dirty = true;
  // stepped on its own again: no target, and the lattice index the batch
  // launches left in the device state
  CaseState cs;
  BHIPCHK(b, hipMemcpy(&cs, s->state.p, sizeof cs, hipMemcpyDeviceToHost));
  cs.target = std::numeric_limits<int64_t>::max();
  BHIPCHK(b, hipMemcpy(s->state.p, &cs, sizeof cs, hipMemcpyHostToDevice));
  s->host_cur = cs.cur;
  return IB_LBM_OK;
}

ib_lbm_status ib_lbm_batch_set_target(ib_lbm_batch *b, ib_lbm_sim *s, int64_t target) {
  if (!b || !s || s->batch != b || target < 0) return IB_LBM_E_INVALID;
  CaseState cs;
  BHIPCHK(b, hipStreamSynchronize(b->stream));
  BHIPCHK(b, hipMemcpy(&cs, s->state.p, sizeof cs, hipMemcpyDeviceToHost));
  cs.target = target;
  BHIPCHK(b, hipMemcpy(s->state.p, &cs, sizeof cs, hipMemcpyHostToDevice));
  return IB_LBM_OK;
}

static ib_lbm_status batch_tables(ib_lbm_batch *b) {
  if (!b->dirty) return IB_LBM_OK;
  if (b->graph_exec) {
    (void)hipGraphExecDestroy(b->graph_exec);
    b->graph_exec = nullptr;
  }
  std::vector<CaseDesc> cases;
  std::vector<int32_t> prefix;
  std::vector<IbmSlot> slots;
  std::vector<ib_lbm_sim *> case_sims;  // the sim of each case entry
  std::vector<int32_t> fprefix;
  b->groups.clear();
  int maxws = 0;
  for (int col = 0; col < 3; col++) {
    ib_lbm_batch::Group g{col, (int)cases.size(), 0, 0, (int)prefix.size(), 0, 0};
    int tiles = 0, faces = 0;
    for (auto *s : b->sims) {
      if (s->cd.collision != col) continue;
      CaseDesc c = s->cd;
      fill_case_tiles(&c, b->launch);
      prefix.push_back(tiles);
      tiles += c.tiles_x * c.tiles_y;
      fprefix.push_back(faces);
      faces += face_blocks(c.nx, c.ny);
      cases.push_back(c);
      case_sims.push_back(s);
      g.count++;
      g.general_zg |= general_zero_gradient(c) ? 1 : 0;
      for (auto &hb : s->bodies)
        if (hb.dev.ws_doubles * 8 <= ibm_max_lds_bytes()) maxws = std::max(maxws, hb.dev.ws_doubles);
    }
    prefix.push_back(tiles);
    fprefix.push_back(faces);
    g.ntiles = tiles;
    g.nface_blocks = faces;
    if (g.count) b->groups.push_back(g);
  }
  std::vector<IbmSlot> rest;
  for (int ci = 0; ci < (int)cases.size(); ci++) {
    const int n = std::max(1, cases[ci].nbodies);
    for (int k = 0; k < n; k++) {
      const IbmSlot sl{ci, cases[ci].nbodies ? k : -1, n, 0};
      if (cases[ci].nbodies && body_fast(case_sims[ci]->bodies[k], b->spread_mode)) slots.push_back(sl);
      else rest.push_back(sl);
    }
  }
  b->nslots_fast = (int)slots.size();
  slots.insert(slots.end(), rest.begin(), rest.end());
  auto upload = [&](DevBuf *d, const void *src, size_t bytes) -> ib_lbm_status {
    if (d->bytes < bytes) {
      if (d->p) (void)hipFree(d->p);
      d->p = nullptr;
      if (hipMalloc(&d->p, bytes) != hipSuccess) {
        set_err(&b->err, "batch table allocation failed");
        return IB_LBM_E_NOMEM;
      }
      d->bytes = bytes;
    }
    BHIPCHK(b, hipMemcpy(d->p, src, bytes, hipMemcpyHostToDevice));
    return IB_LBM_OK;
  };
  ib_lbm_status st;
  if (!cases.empty()) {
    if ((st = upload(&b->d_cases, cases.data(), cases.size() * sizeof(CaseDesc)))) return st;
    if ((st = upload(&b->d_prefix, prefix.data(), prefix.size() * sizeof(int32_t)))) return st;
    if ((st = upload(&b->d_fprefix, fprefix.data(), fprefix.size() * sizeof(int32_t)))) return st;
    if ((st = upload(&b->d_slots, slots.data(), slots.size() * sizeof(IbmSlot)))) return st;
  }
  b->nslots = (int)slots.size();
  b->lds_bytes = lds_budget(maxws);

  b->dirty = false;
  return IB_LBM_OK;
}

static ib_lbm_status batch_enqueue_step(ib_lbm_batch *b, hipStream_t stream) {
  LaunchShape sh{b->launch.block_x, b->launch.block_y, b->launch.rows_per_thread, b->launch.xcd_remap};
  for (auto &g : b->groups) {
    BHIPCHK(b, launch_collide_stream(b->precision, g.collision, (const CaseDesc *)b->d_cases.p + g.first,
                                     (const int32_t *)b->d_prefix.p + g.prefix_off, g.count, g.ntiles,
                                     sh, stream));
    BHIPCHK(b, launch_collide_stream_faces(b->precision, g.collision,
                                           (const CaseDesc *)b->d_cases.p + g.first,
                                           (const int32_t *)b->d_fprefix.p + g.prefix_off, g.count,
                                           g.nface_blocks, -1, 1, g.general_zg, stream));
  }
  BHIPCHK(b, launch_ibm_slots(b->precision, (const CaseDesc *)b->d_cases.p, (const IbmSlot *)b->d_slots.p,
                              b->nslots_fast, b->nslots, b->lds_bytes, b->spread_mode,
                              b->launch.ib_threads, stream));
  return IB_LBM_OK;
}

ib_lbm_status ib_lbm_batch_step(ib_lbm_batch *b, int64_t nsteps) {
  if (!b || nsteps < 0) return IB_LBM_E_INVALID;
  if (b->broken) return IB_LBM_E_STATE;
  ib_lbm_status st = batch_tables(b);
  if (st) return st;
  if (b->sims.empty()) return IB_LBM_OK;
  int64_t left = nsteps;
  if (b->graph_steps > 0 && left >= b->graph_steps) {
    if (!b->graph_exec || b->graph_len != b->graph_steps) {
      if (b->graph_exec) (void)hipGraphExecDestroy(b->graph_exec);
      b->graph_exec = nullptr;
      if (!b->cap_stream) BHIPCHK(b, hipStreamCreateWithFlags(&b->cap_stream, hipStreamNonBlocking));
      hipGraph_t g;
      BHIPCHK(b, hipStreamBeginCapture(b->cap_stream, hipStreamCaptureModeThreadLocal));
      for (int i = 0; i < b->graph_steps; i++) {
        if ((st = batch_enqueue_step(b, b->cap_stream))) {
          hipGraph_t dummy;
          (void)hipStreamEndCapture(b->cap_stream, &dummy);
          return st;
        }
      }
      BHIPCHK(b, hipStreamEndCapture(b->cap_stream, &g));
      BHIPCHK(b, hipGraphInstantiate(&b->graph_exec, g, nullptr, nullptr, 0));
      (void)hipGraphDestroy(g);
      b->graph_len = b->graph_steps;
    }
    while (left >= b->graph_len) {
      BHIPCHK(b, hipGraphLaunch(b->graph_exec, b->stream));
      left -= b->graph_len;
    }
  }
  for (int64_t i = 0; i < left; i++)
    if ((st = batch_enqueue_step(b, b->stream))) return st;
  return IB_LBM_OK;
}

ib_lbm_status ib_lbm_batch_set_graph(ib_lbm_batch *b, int32_t steps_per_graph) {
  if (!b || steps_per_graph < 0 || steps_per_graph > 100000) return IB_LBM_E_INVALID;
  b->graph_steps = steps_per_graph;
  return IB_LBM_OK;
}

ib_lbm_status ib_lbm_batch_set_launch(ib_lbm_batch *b, const ib_lbm_launch *l) {
  if (!b) return IB_LBM_E_INVALID;
  if (b->broken) return IB_LBM_E_STATE;
  ib_lbm_status st = check_launch(l, &b->err);
  if (st) return st;
  b->launch = *l;
  b->dirty = true;
  return IB_LBM_OK;
}

ib_lbm_status ib_lbm_batch_set_spread(ib_lbm_batch *b, int32_t mode) {
  if (!b) return IB_LBM_E_INVALID;
  if (mode != IB_LBM_SPREAD_GATHER && mode != IB_LBM_SPREAD_ATOMIC) return IB_LBM_E_INVALID;
  b->spread_mode = mode;
  if (b->graph_exec) {
    (void)hipGraphExecDestroy(b->graph_exec);
    b->graph_exec = nullptr;
  }
  return IB_LBM_OK;
}

ib_lbm_status ib_lbm_batch_sync(ib_lbm_batch *b) {
  if (!b) return IB_LBM_E_INVALID;
  if (b->broken) return IB_LBM_E_STATE;
  BHIPCHK(b, hipStreamSynchronize(b->stream));
  return IB_LBM_OK;
}

ib_lbm_status ib_lbm_batch_destroy(ib_lbm_batch *b) {
  if (!b) return IB_LBM_E_INVALID;
  if (b->stream) (void)hipStreamSynchronize(b->stream);
  for (auto *s : b->sims) s->batch = nullptr;
  if (b->graph_exec) (void)hipGraphExecDestroy(b->graph_exec);
  if (b->cap_stream) (void)hipStreamDestroy(b->cap_stream);
  if (b->d_cases.p) (void)hipFree(b->d_cases.p);
  if (b->d_prefix.p) (void)hipFree(b->d_prefix.p);
  if (b->d_fprefix.p) (void)hipFree(b->d_fprefix.p);
  if (b->d_slots.p) (void)hipFree(b->d_slots.p);
  delete b;
  return IB_LBM_OK;
}

const char *ib_lbm_batch_last_error(const ib_lbm_batch *b) { return b ? b->err.c_str() : "null batch"; }

}  // extern "C"
