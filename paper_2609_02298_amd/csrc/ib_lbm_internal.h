// Internal device/host data structures of the IB-LBM library (gfx950).
//
// A "case" is one lattice with its bodies.  Kernels never take per-step
// scalar arguments: every case carries its own step counter, target and
// current-buffer index in device memory, so a batch of cases of different
// sizes and step counts is advanced by the same launches, and a captured
// graph of launches stays valid while the batch composition is unchanged.
#pragma once

#include <hip/hip_runtime.h>
#include <hip/hip_ext.h>
#include <stdint.h>

#include <tuple>
#include <utility>

namespace iblbm {

enum { kPrecFP64 = 0, kPrecFP32 = 1 };
enum { kBGK = 0, kTRT = 1, kCMMRT = 2 };
enum { kVerlet = 0, kEulerA1 = 1 };
enum { kUdRigid = 0, kUdTaylorGreen = 1 };
enum { kPeriodic = 0, kBounceBack = 1, kVelParabolic = 2, kVelUniform = 3, kZeroGradient = 4,
       kZouHe = 5 };
enum { kFaceW = 0, kFaceE = 1, kFaceS = 2, kFaceN = 3 };
enum { kDF = 0, kMDF = 1, kDFC = 2 };
enum { kHat = 0, kPeskin4 = 1 };
enum { kFixed = 0, kPrescribedSin = 1, kFree = 2 };
enum { kImNone = 0, kImFeng = 1 };

// body flags (same values as the public IB_LBM_FLAG_*)
enum { kFlagNonfinite = 1, kFlagRange = 2, kFlagOverlap = 4, kFlagCapacity = 8, kFlagExchange = 16 };
// case flags
enum { kCaseHalted = 1 };

constexpr int kMaxBodiesPerCase = 8;
constexpr int kIbmThreads = 512;
constexpr int kIbmThreadsFast = 1024;
constexpr int kHistCols = 16;

// Population storage of a lattice.  Each row is cut along x into segments
// of kSeg nodes (the last one padded), and the nine populations of one
// segment are stored one after the other, kSeg values each:
//   value (i, x, y) at ((y * nseg + x / kSeg) * 9 + i) * kSeg + x % kSeg.
// A wave of 64 nodes of one row then reads and writes nine runs of 64
// values that lie together in one block of 9 kSeg values, rather than in
// nine planes far apart; on lattices larger than the Infinity Cache that
// keeps more of the HBM traffic in open DRAM pages.  Offsets are 64-bit.
constexpr int kSegLog = 6;
constexpr int kSeg = 1 << kSegLog;
constexpr int kSegBlock = 9 * kSeg;  // values of one segment
__host__ __device__ inline int pop_segments(int nx) { return (nx + kSeg - 1) >> kSegLog; }
// offset of population 0 of node (x, y); population i is kSeg * i further
__host__ __device__ inline int64_t pop_node(int x, int y, int nseg) {
  return ((int64_t)y * nseg + (x >> kSegLog)) * kSegBlock + (x & (kSeg - 1));
}
// values of one lattice
__host__ __device__ inline int64_t pop_values(int nx, int ny) {
  return (int64_t)ny * pop_segments(nx) * kSegBlock;
}

// Mutable per-case state, device resident.
struct CaseState {
  int64_t step;    // completed steps
  int64_t target;  // kernels do nothing once step >= target
  int32_t cur;     // buffer holding the current post-stream populations
  int32_t flags;   // kCaseHalted
  int32_t done;    // IB workgroups of this step that have finished
  int32_t fbox_valid;  // the union of the bodies' force boxes below is set
  int32_t fbox[4];     // x0 y0 x1 y1 of the nodes that carry IB force
  // Coupled MDF: the IB workgroups of the case exchange their residuals
  // through xr (two rounds' worth, alternating), counting arrivals in xcnt;
  // the last workgroup of a step resets xcnt.
  int32_t xcnt;
  // Fused steps: the workgroups of the tiles that read the IB force count
  // themselves here once they have read (and cleared) it; the IB pass of the
  // same launch writes the new force only after all of them, then resets it.
  int32_t hold_seen;
  // Fused steps: the IB pass sets this to the launch's sequence number once
  // its loads from device memory are done; the tiles start streaming then
  // (a schedule only: they do not depend on the pass).
  int32_t gate;
  // Fused steps: the workgroups that collide the nodes pushing into the
  // support count themselves here once their pushes are staged; the IB pass
  // takes the support's moments after all of them, then resets it.
  int32_t src_seen;
  double xr[2][kMaxBodiesPerCase];
};

// Mutable per-body state, device resident.
struct BodyState {
  double xc, yc;        // centre at the last completed step
  double vx, vy;        // velocity v^n
  double vpx, vpy;      // v^(n-1)
  double om;            // angular velocity
  double omp;           // Omega^(n-1) (Euler-explicit update)
  double vhx, vhy, omh; // half-step values used for U_d in the last step
  double fhx, fhy, torque;
  double dimx, dimy;    // internal-mass force held over the step
  double slip_mean, slip_max, mdf_res;
  int32_t mdf_iters_done;
  int32_t flags;
  int32_t box[4];       // x0 y0 x1 y1 of the nodes that carry IB force
  int32_t box_valid;
  int32_t lambda_valid; // DFC cache filled (fixed bodies)
  int32_t tables_valid; // geometry tables cached (fixed bodies)
  int32_t tables_full;  // a step needs the whole cached table, not only its hot part
};

// A node whose pushes reach the support of a fused step's body: the offset
// of its population 0 in a lattice (pop_node) and, per population i, the
// support node it is pushed to (-1: none; map[0] is the node itself, also
// the index of its force in BodyDesc::fprev).  32 bytes: two 16-byte loads.
struct alignas(16) SrcNode {
  int32_t off;
  int16_t map[9];
  int16_t pad[5];
};

// Constant per-body description plus pointers to the body's device buffers.
struct BodyDesc {
  int32_t nb, scheme, kernel, mdf_iters;
  int32_t motion, internal_mass;
  int32_t integrator;   // free bodies: kVerlet (Eq. 23) or kEulerA1 (Eq. A1)
  int32_t mdf_band;     // > 0: MDF passes in marker space with this band half-width
  int32_t mdf_coupled;  // MDF bodies of the case iterate jointly (coupled path)
  int32_t udes;         // desired velocity: kUdRigid or kUdTaylorGreen (Eq. D1)
  int32_t ns;           // support width: 2 (hat) or 4 (P4)
  int32_t window;       // half width of the angular marker window of the gather
  int32_t max_rows, max_nodes;
  int32_t ws_doubles;   // workspace size
  int32_t hist_cap;
  double radius, ds, dtheta, omega_mdf;
  double xc0, yc0, amp[2], freq, phase;
  double ms, mf, Is;
  double tg_u0, tg_k, tg_nu;  // Eq. D1 (kUdTaylorGreen)
  const double *cos_t, *sin_t;  // marker directions (n_b each)
  double *ws;           // global workspace (used when it does not fit in LDS)
  double *tab_cache;    // cached geometry tables of a fixed body (ws_tab doubles)
  double *acc;          // 2 x max_nodes scratch of the atomic-scatter variant
  int32_t ws_tab;       // doubles of the table part of the workspace
  int32_t ws_tab_hot;   // doubles of its hot part (what a DF/MDF step reads)
  int32_t pop_bytes;    // bytes of one stored population (8 FP64, 4 FP32 shifted)
  int32_t mdf_nmin;     // adaptive MDF: fewest passes before the tolerance stop
  double mdf_tol;       // > 0: adaptive MDF with this tolerance; else mdf_iters passes
  double *markers_out;  // n_b x 8: X Y Udx Udy Fx Fy lambda ds
  double *lambda_cache; // n_b
  double *history;      // hist_cap x kHistCols
  // Fused steps (fixed DF/MDF bodies): the IB pass collides the support
  // nodes and their neighbours itself.  src: one SrcNode per such node
  // (n_src of them).  fprev: the force the last pass wrote to the support
  // nodes (2 x max_nodes, the population type); pstage: the pushed
  // populations of the support nodes (population-major: 9 planes of
  // max_nodes).  Null when unused.
  const struct SrcNode *src;
  int32_t n_src;
  int32_t pad_src;
  void *fprev;
  void *pstage;
  BodyState *state;
};

// Constant per-case description (copied into a device table by a batch).
struct CaseDesc {
  int32_t nx, ny;
  int32_t collision, precision;
  int32_t bc[4];
  int32_t tiles_x, tiles_y;
  int32_t nbodies;
  int32_t nseg;         // population segments per row, pop_segments(nx)
  int64_t plane;        // nx*ny (nodes; the force field has two planes of this size)
  double omega, s_e, s_o, s_q, s_eps;  // relaxation rates
  double rho0, u_bc, inv_ny2;
  double fluid_fx, fluid_fy;
  double grav_x, grav_y;  // gravity acting on bodies (Eq. 22)
  void *f[2];           // two population lattices (segment-blocked, see pop_node)
  void *force;          // IB force density, 2 planes
  CaseState *state;
  BodyDesc *bodies;     // device array of nbodies
};

// Workspace of one body, in doubles.  The table part (marker geometry,
// compact support description, node -> marker lists) comes first so that it
// can be cached and copied in bulk; the per-step arrays follow.  Within the
// table, what a step reads comes first (the hot part, ws_tab_hot doubles),
// what only the construction, DFC and nodes with long lists read follows.
//   doubles: X Y Udx Udy (nb each), wx wy (nb*ns each)
//   ints:    nrow (nb*ns: the first support node of each stencil row), nxy
//            (mn), ell (DF/MDF only, ell_width(ns)*mn:
//            the first entries of each node's list, node-fastest), S (1)
//            [padded to even: the end of the hot part]
//            ix0 iy0 (nb each), ra1 rl1 ra2 (mr each), off (mr+1),
//            noff (mn+1), nent (nb*ns*ns) [padded to even]
//   per step, DF/MDF: rhoX Fx Fy Ftx Fty (nb each), nrho nux nuy (mn each),
//                     then Ux Uy (nb each, marker-space or coupled MDF) and,
//                     coupled MDF, Fnx Fny (nb each), pux puy (mn each)
//   per step, DFC:    Ftx Fty lam (nb each), dlt (9 nb), then the staged
//                     populations (9 mn of T), overlaid by the W_total node
//                     array while the correction scale is built and, at the
//                     end, by the node velocities of the corrected populations
// Fixed width of the node-fastest copy of the node -> marker lists: a node
// is covered by at most this many markers at unit marker spacing.
__host__ __device__ inline int ell_width(int ns) { return ns == 4 ? 6 : 3; }
__host__ __device__ inline int ws_table_doubles(int nb, int ns) { return nb * (4 + 2 * ns); }
__host__ __device__ inline int ws_hot_ints(int scheme, int nb, int ns, int mn) {
  const int n = nb * ns + mn + (scheme != 2 ? ell_width(ns) * mn : 0) + 1;
  return (n + 1) & ~1;
}
__host__ __device__ inline int ws_table_ints(int scheme, int nb, int ns, int mr, int mn) {
  const int n = 2 * nb + 4 * mr + 1 + mn + 1 + nb * ns * ns;
  return ws_hot_ints(scheme, nb, ns, mn) + ((n + 1) & ~1);
}
__host__ __device__ inline int ws_tab_hot(int scheme, int nb, int ns, int mn) {
  return ws_table_doubles(nb, ns) + ws_hot_ints(scheme, nb, ns, mn) / 2;
}
__host__ __device__ inline int ws_tab_total(int scheme, int nb, int ns, int mr, int mn) {
  return ws_table_doubles(nb, ns) + ws_table_ints(scheme, nb, ns, mr, mn) / 2;
}
__host__ __device__ inline int ws_dyn_doubles(int scheme, int nb, int ns, int mn, int pop_bytes) {
  if (scheme == 2) return nb * 12 + (9 * mn * pop_bytes + 7) / 8;
  return nb * 5 + mn * 3;
}
// the coupled MDF path adds the marker errors and unrelaxed forces (4 nb)
// and the node velocities before a trial pass (2 mn)
__host__ __device__ inline int ws_coupled_doubles(int nb, int mn) { return 4 * nb + 2 * mn; }

// One IB workgroup: the body `body` of case `cas` (body = -1: a case without
// bodies, which only advances the step counter).
struct IbmSlot {
  int32_t cas;
  int32_t body;
  int32_t slots_in_case;
  int32_t pad;
};

// Number of face nodes of an nx x ny lattice: rows y = 0 and ny-1, columns
// x = 0, nx-2 and nx-1 in between (the nodes with a link that leaves the
// lattice, and the column the zero-gradient outlet copies from).
__host__ __device__ inline int face_nodes(int nx, int ny) { return 2 * nx + 3 * (ny - 2); }
// The face launch gives every case whole workgroups of kFaceBlock nodes, so
// that a workgroup's case (and every read of its description) is uniform.
constexpr int kFaceBlock = 256;
__host__ __device__ inline int face_blocks(int nx, int ny) {
  return (face_nodes(nx, ny) + kFaceBlock - 1) / kFaceBlock;
}

struct LaunchShape {
  int32_t block_x, block_y, rows_per_thread, xcd_remap;
};

// Everything the inner-node collide-stream of one case reads, passed by
// value.  A sim stepped on its own knows on the host which lattice holds
// the step's input, so a workgroup's first memory accesses are its
// populations, with the case's halt flag (and force box) loaded beside
// them, rather than a chain of loads through the case descriptor and
// state.  mode: 0 every tile, 1 only the tiles of the hold rectangle
// (htx0, hty0, hntx x hnty tiles; they read the IB force at every node),
// 2 every tile outside it (no IB force).  force_on (mode 0): read the IB
// force inside the case's force box.
struct LeanArgs {
  const void *src;
  void *dst;
  void *force;
  const CaseState *state;
  int32_t nx, ny, nseg, tiles_x, ntiles, rpt, remap, force_on;
  int32_t htx0, hty0, hntx, hnty;
  double omega, s_e, s_o, s_q, s_eps, rho0, fluid_fx, fluid_fy;
};

// ---- kernel launchers (defined in the .hip files) ----
// A launcher launches on its stream unless given a LaunchTarget.  With a
// graph, the target takes the same kernel with the same arguments as a node
// of that explicitly built graph, after its dependencies (node is null when
// nothing is added).  Without one, the kernel is launched on the stream with
// `done` as the launch's completion event: the event is recorded by the
// kernel's own completion, with no separate marker packet behind it.
struct LaunchTarget {
  hipGraph_t graph = nullptr;
  const hipGraphNode_t *deps = nullptr;
  size_t ndeps = 0;
  hipGraphNode_t node = nullptr;
  hipEvent_t done = nullptr;
};

template <typename Tup, size_t... I>
inline void arg_pointers(Tup &t, void **p, std::index_sequence<I...>) {
  ((p[I] = (void *)&std::get<I>(t)), ...);
}

// What a launcher returns when it has no work: a direct launch's completion
// event is still recorded, so that waits on it keep their order.
inline hipError_t nothing_to_launch(hipStream_t stream, LaunchTarget *ns) {
  if (ns && !ns->graph && ns->done) return hipEventRecord(ns->done, stream);
  return hipSuccess;
}

template <typename... P, typename... A>
inline hipError_t issue(void (*kernel)(P...), dim3 grid, dim3 block, unsigned shmem,
                        hipStream_t stream, LaunchTarget *ns, A &&...args) {
  std::tuple<std::decay_t<P>...> vals(std::forward<A>(args)...);
  void *ptrs[sizeof...(P) > 0 ? sizeof...(P) : 1];
  arg_pointers(vals, ptrs, std::index_sequence_for<P...>{});
  if (!ns) return hipLaunchKernel((const void *)kernel, grid, block, ptrs, shmem, stream);
  if (!ns->graph)
    return hipExtLaunchKernel((const void *)kernel, grid, block, ptrs, shmem, stream, nullptr,
                              ns->done, 0);
  hipKernelNodeParams p{};
  p.func = (void *)kernel;
  p.gridDim = grid;
  p.blockDim = block;
  p.sharedMemBytes = shmem;
  p.kernelParams = ptrs;
  p.extra = nullptr;
  return hipGraphAddKernelNode(&ns->node, ns->graph, ns->deps, ns->ndeps, &p);
}

// Inner nodes of every case of a batch, each case's input lattice from its
// device state (batches flatten (case, tile) through tile_prefix).
hipError_t launch_collide_stream(int precision, int collision, const CaseDesc *cases,
                                 const int32_t *tile_prefix, int ncases, int ntiles,
                                 LaunchShape shape, hipStream_t stream);
// Inner nodes of one case with its arguments by value (see LeanArgs).
hipError_t launch_collide_stream_lean(int precision, int collision, const LeanArgs &a, int mode,
                                      LaunchShape shape, hipStream_t stream, LaunchTarget *ns = nullptr);
// The face nodes (rows 0 and ny-1, columns 0, nx-2, nx-1) with the face
// closures; face_prefix[i] is the first workgroup of case i (face_blocks per
// case), nblocks the total; cur < 0 takes each case's lattice from its state.
hipError_t launch_collide_stream_faces(int precision, int collision, const CaseDesc *cases,
                                       const int32_t *face_prefix, int ncases, int nblocks, int cur,
                                       int force, int general_zg, hipStream_t stream,
                                       LaunchTarget *ns = nullptr);
// IB launch over nslots slots; replicas > 1 (with a per-slot counter that
// every copy advances, see ibm_kernel) lets the first-started copy of each
// slot run it.  threads: workgroup size (0: the instance's default), capped
// at the instance's launch bound.
hipError_t launch_ibm(int precision, const CaseDesc *cases, const IbmSlot *slots, int nslots,
                      int lds_bytes, int spread_mode, int fast, int replicas, uint32_t *ticket,
                      int threads, hipStream_t stream, LaunchTarget *ns = nullptr);
// One launch per step for a case with a single fixed DF/MDF body
// (step_fused_kernel): workgroup 0 runs the IB pass; the next nsrc
// workgroups collide the nodes that push into the body's support, from the
// step's input lattice, and stage those pushes for the pass (CaseState::
// src_seen); then the tiles of the hold rectangle (lean.htx0..hnty: every node that
// carries IB force), which read and clear the force and count themselves in
// CaseState::hold_seen; then the face nodes, one face workgroup of
// kFaceBlock nodes per workgroup; then every other tile.  All workgroups have kFusedThreads
// threads; a tile is a logical bx x by workgroup (bx * by = kFusedThreads)
// with lean.rpt rows per thread.
constexpr int kFusedThreads = 1024;
struct FusedArgs {
  LeanArgs lean;
  const CaseDesc *c;
  const int32_t *face_prefix;
  int32_t nface, gzg, bx, by;
  int32_t cur;  // the step's input lattice (faces and tiles; the IB pass reads the case state)
  int32_t seq;  // the launch's sequence number (CaseState::gate)
  int32_t nsrc; // workgroups of the support's own collision (BodyDesc::n_src nodes)
  int32_t gated;  // the tiles wait for the IB pass's kinematics and tables (CaseState::gate)
  // copies of *c and of its single body descriptor, as uploaded: the IB
  // pass and the source workgroups read them from the kernel arguments
  // (scalar loads at launch) instead of following c -> bodies -> fields
  // through device memory, a chain of dependent round trips at the start
  // of the launch's critical path
  CaseDesc cd;
  BodyDesc bd;
};
int fused_grid(const FusedArgs &a);
hipError_t launch_step_fused(int precision, int collision, const FusedArgs &a, int lds_bytes,
                             hipStream_t stream, LaunchTarget *ns = nullptr);
hipError_t launch_zou_he(int precision, const CaseDesc *c, int nx, int ny, int cur, hipStream_t stream,
                         LaunchTarget *ns = nullptr);
hipError_t launch_init_equilibrium(const CaseDesc &c, int buf, hipStream_t stream);
// The reference stream of ib_lbm_stream_copy (n 16-byte vectors).
hipError_t launch_stream_copy(const void *src, void *dst, size_t n, int workgroups, hipStream_t stream);
hipError_t launch_fields(const CaseDesc &c, int buf, double *rho, double *ux, double *uy,
                         hipStream_t stream);
hipError_t launch_export(const CaseDesc &c, int buf, double *out, hipStream_t stream);
hipError_t launch_import(const CaseDesc &c, int buf, const double *in, hipStream_t stream);
hipError_t launch_set_equilibrium(const CaseDesc &c, int buf, const double *rho, const double *ux,
                                  const double *uy, hipStream_t stream);
hipError_t launch_force_export(const CaseDesc &c, double *fx, double *fy, hipStream_t stream);
hipError_t launch_diagnostics(const CaseDesc &c, int buf, const double *markers, int nb, double xc,
                              double yc, double vx, double vy, double om, double radius,
                              double ds, int kappa, double u_ref, double *out, double *pm,
                              hipStream_t stream);
int ibm_max_lds_bytes();
// Staging of the allocation-free diagnostics: its device address on the
// current device (taken once per device), and its capacity in markers.
hipError_t diag_scratch(double **ptr);
int diag_scratch_markers();

}  // namespace iblbm
