// Internal types of the NeuralFVM HIP library: padded device layout, patch
// table, physics parameters and the launchers every kernel file provides.
#pragma once

#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <functional>
#include <vector>

namespace nfvm {

// Kernel-timing events for the next main-kernel launch of the calling thread
// (set by the grid's profiler; null when not timing).  The launch records
// them itself at the kernel's start and end (hipExtLaunchKernelGGL), so
// the interval is the kernel's own run time, and clears them, so the
// finalising kernels that follow are not timed.
struct LaunchEvents {
  hipEvent_t start = nullptr, stop = nullptr;    // the main kernel
  hipEvent_t fstart = nullptr, fstop = nullptr;  // its finaliser (NFVM_LAUNCH_FIN)
};
extern thread_local LaunchEvents t_launch_ev;

#define NFVM_LAUNCH(K, G, B, SH, S, ...)                                                     \
  do {                                                                                       \
    if (::nfvm::t_launch_ev.start) {                                                         \
      hipExtLaunchKernelGGL(K, G, B, SH, S, ::nfvm::t_launch_ev.start,                       \
                            ::nfvm::t_launch_ev.stop, 0, __VA_ARGS__);                       \
      ::nfvm::t_launch_ev.start = ::nfvm::t_launch_ev.stop = nullptr;                        \
    } else {                                                                                 \
      hipLaunchKernelGGL(K, G, B, SH, S, __VA_ARGS__);                                       \
    }                                                                                        \
  } while (0)

// The same for a finalising kernel (its own pair of events).
#define NFVM_LAUNCH_FIN(K, G, B, SH, S, ...)                                                 \
  do {                                                                                       \
    if (::nfvm::t_launch_ev.fstart) {                                                        \
      hipExtLaunchKernelGGL(K, G, B, SH, S, ::nfvm::t_launch_ev.fstart,                      \
                            ::nfvm::t_launch_ev.fstop, 0, __VA_ARGS__);                      \
      ::nfvm::t_launch_ev.fstart = ::nfvm::t_launch_ev.fstop = nullptr;                      \
    } else {                                                                                 \
      hipLaunchKernelGGL(K, G, B, SH, S, __VA_ARGS__);                                       \
    }                                                                                        \
  } while (0)


// Cell type byte of the fine grid (interior and ghost cells):
//   low 7 bits: patch id (0 fluid, 1 solid block, 2..7 default wall of face
//   0..5, 8.. user patches in descriptor order); bit 7: fluid cell whose
//   omega is held at the wall value (Sec. 2.7).
constexpr int MAX_PATCHES = 128;
constexpr int PID_FLUID = 0;
constexpr int PID_SOLID = 1;
constexpr int PID_DEFWALL = 2;
constexpr int PID_USER = 8;
constexpr uint8_t FIXED_BIT = 0x80;

enum { K_WALL = 0, K_INLET = 1, K_OUTLET = 2 };

// Multigrid cell class per level: 0 inactive (all children solid),
// 1 regular (active, all faces coefficient 1), 2 irregular (read the face
// coefficient arrays).
enum { MG_INACTIVE = 0, MG_REGULAR = 1, MG_IRREGULAR = 2 };

struct bf16 {
  uint16_t v;
};

struct DevPatch {
  int kind;
  int T_dirichlet;  // wall with a fixed temperature
  double U[3];
  double T, k, omega, T_wall;  // temperatures as deviations from T_ref
  double nut;  // eddy viscosity of the inlet values (filled on the device)
};

// Padded level layout.  Cell (i, j, k), i in [-1, nx], j in [-1, ny],
// k in [-gz, nz - 1 + gz], sits at off + k*sxy + j*sx + i; rows are padded to
// a multiple of 16 elements so interior rows start aligned.
struct Geom {
  int nx, ny, nz, dim;
  int sx, sxy, gz;
  int off, total;
  double hx, hy, hz;
  // > 0: the Jacobi sweeps of this multigrid level divide by this scalar
  // (Algorithm 1's reading of eq. jacobi_pc) instead of the cell's diagonal
  double sd;
  __host__ __device__ inline int idx(int i, int j, int k) const {
    return off + k * sxy + j * sx + i;
  }
  __host__ __device__ inline long long cells() const {
    return (long long)nx * ny * nz;
  }
};

Geom make_geom(int dim, int nx, int ny, int nz, double hx, double hy, double hz);

// Column tiling of a level: 64 x 4 columns per workgroup, each thread walks
// cz consecutive z planes.  Workgroups are dealt to the 8 XCDs round robin
// (block b runs on XCD b % 8); tile_of gives each XCD one contiguous range of
// tiles (x fastest), so neighbouring tiles mostly share an L2.
struct Tiles {
  int ntx, nty, ntz, cz, total, grid;
};
Tiles make_tiles(int nx, int ny, int nz, int target_blocks);
__device__ __forceinline__ bool tile_of(const Tiles& T, int& tx, int& ty, int& tz) {
  const int per = T.grid >> 3;
  const int b = blockIdx.x;
  const int t = (b & 7) * per + (b >> 3);
  if (t >= T.total) return false;
  tx = t % T.ntx;
  ty = (t / T.ntx) % T.nty;
  tz = t / (T.ntx * T.nty);
  return true;
}

struct Phys {
  double nu, alpha_T, inv_Pr_t, inv_sigma_k, inv_sigma_w, dt;
  int komega, energy, buoyancy;
  double g[3], T_ref, beta_T;
};

// Tunable kernels: tile targets (workgroups per launch, see Tiles) chosen per
// level by the autotuner.
enum {
  TK_SMOOTH = 0,
  TK_SMOOTH_ZERO,
  TK_RESTRICT,  // on the fine level of the pair
  TK_PROLONG,   // on the fine level of the pair
  TK_START,
  TK_APPLY,
  TK_UPDATE,
  TK_SMOOTH2,   // two level-0 sweeps in one pass
  TK_LEVEL_COUNT
};
enum { TP_EXPLICIT = 0, TP_DESTROY, TP_RHS, TP_PROJECT, TP_COUNT };
constexpr int TILE_DEFAULT = 4096;

// One multigrid level on the device.
struct Level {
  int tt[TK_LEVEL_COUNT];       // tile target per tunable kernel
  Geom g;
  uint8_t* cls;                 // MG_* per padded cell
  uint8_t* full;                // 1: cell and all 26 neighbours active and inside (coarse levels)
  float* cf[3];                 // face coefficients; face between cell q-1 and q along d at idx(q)
  void* x[2];                   // iterate, ping-pong (storage type of the level)
  void* b;                      // right-hand side
  int cur;                      // which x is current
  uint16_t* code;               // level 0 only: face codes (else null)
  bool nearest = false;         // correction from the next coarser level taken
                                // as nearest (piecewise constant), not linear
  bool wide = false;            // coarse level stored in the level-0 type (mixed
                                // precision: FP32 instead of BF16)
};

// Level-0 face code of a cell: 2 bits per face (x-, x+, y-, y+, z-, z+ from
// bit 0), each the face coefficient c_f in {0, 1, 2}; inactive cells hold
// FACE_CODE_INACTIVE.
constexpr uint32_t FACE_CODE_INACTIVE = 0xFFFFu;
void launch_face_codes(const Geom& g, const uint8_t* cls, const float* cx, const float* cy,
                       const float* cz, uint16_t* code, hipStream_t s);

// Reverse mode of the explicit stage (forward Euler) at the state st (seven
// padded FP64 arrays u v w p theta k omega, theta = T - T_ref; p is not
// read and may be null): from the
// dense adjoints yb of the outputs u v w T k omega, the dense adjoints xb of
// the inputs u v w p T k omega, nu_t being the closure of k and omega.
// W (6 padded arrays), pass (2), L4S (6) and nu (1, nu_t) are scratch.
void launch_explicit_adjoint(const Geom& g, const Phys& ph, const uint8_t* type,
                             const DevPatch* pt, const double* const st[7],
                             const double* const yb[6], double* W, double* pass, double* L4S,
                             double* nu, double* const xb[7], hipStream_t s);

// Reverse mode of the destruction step over tau at the state st (five
// padded FP64 arrays u v w k omega): from the dense adjoints kb, wb of its k
// and omega, the dense adjoints xb of u v w k omega.  E (6 padded arrays)
// and M (9) are scratch.
void launch_destroy_adjoint(const Geom& g, const Phys& ph, const uint8_t* type,
                            const DevPatch* pt, const double* const st[5], double tau,
                            const double* kb, const double* wb, double* E, double* M,
                            double* const xb[5], hipStream_t s);

// out = scale (a + b) over n dense FP64 values; zeroing of a dense array on
// the cells whose omega is held (wall-adjacent fluid cells).
void launch_dense_add(size_t n, const double* a, const double* b, double* out, hipStream_t s,
                      double scale = 1.0);
void launch_zero_held(const Geom& g, const uint8_t* type, double* a, hipStream_t s);

// Device-wide reduction scratch: per-block partials and the reduced scalars.
struct RedBuf {
  double* partial;
  double* out;
  int max_blocks;  // partial holds max_blocks * RED_MAX_NV values
  // host-coherent copy of the scalars the host reads (stopping state,
  // norms, step statistics), written by the finalising kernels; may be null
  double* mirror;
};

// Scalars of the pressure iteration kept on the device.
enum {
  S_BB = 0,        // ||b||^2
  S_RR = 1,        // ||r||^2
  S_ZR = 2,        // (z, r)
  S_ZQ = 3,        // (z, q_prev)
  S_PQ = 4,        // (p, q) of the current iteration (the previous one while it is formed)
  S_ZW = 5,        // (z, A z)
  S_ALPHA = 6,     // step length of the current iteration
  S_DIV = 7,       // max face divergence
  S_MINK = 8,
  S_MINW = 9,
  S_DONE = 10,     // 1 once the iteration has met its stopping rule
  S_ITER = 11,     // preconditioner applications so far
  S_TOL2 = 12,     // tol^2
  S_MAXIT = 13,
  S_FORCED = 14,   // < 0: stop on tol
  S_BETA = 15,     // direction coefficient of the current iteration
  S_APREV = 16,    // step length of the previous iteration (its x update is deferred)
  S_COUNT = 17
};

// Most values one block of a reducing kernel stores in red.partial.
constexpr int RED_MAX_NV = 3;

// Host-side check before a reducing launch: nblocks blocks storing nv
// partials each must fit red.partial (throws the library's error otherwise;
// defined in engine.cpp).
[[noreturn]] void fail_partials(int nblocks, int nv, int max_blocks);
inline void check_partials(const RedBuf& red, int nblocks, int nv) {
  if (nv > RED_MAX_NV || nblocks > red.max_blocks) fail_partials(nblocks, nv, red.max_blocks);
}

// ---- launchers (defined in the .hip files) --------------------------------
// Reduce nblocks partials of nv values (op 0 sum, 1 max, 2 min) into
// red.out[slot0] (and red.out[slot1] when nv == 2).
void launch_finalize(int nv, int op, const RedBuf& red, int nblocks, int slot0, int slot1,
                     hipStream_t s);
// Algorithm 1's outer iteration on level 0: x += z (z the level's current
// iterate), then r = b - A x rounded into the level's right-hand side, with
// ||r||^2 through the CG update's finaliser (iteration count, stopping rule).
template <class O, class S>
void launch_plain_update(const Level& l0, O* x, const O* b, const RedBuf& red, hipStream_t s);

// The x update the last CG iteration of a solve deferred (iterations with an
// even index leave x += alpha p to the next one): to be launched once the
// solve has stopped, before anything reads x; no-op when nothing is pending.
template <class O, class S>
void launch_fcg_flush(const Level& l0, O* x, void* const* dir, const double* ctl,
                      hipStream_t s);

// Workgroups of the largest reducing launch of one pressure solve on level
// 0 (CG start, apply and update with the level's current tiles).
int fcg_max_blocks(const Level& l0);
// x[0 .. n) = v on stream s (a kernel, so that it may be captured).
void launch_fill_f64(double* x, int n, double v, hipStream_t s);

void launch_classify(const Geom& g, const uint8_t* solid_dense, const int* patch_rect,
                     int n_patches_user, DevPatch* patches, double nu, int komega,
                     uint8_t* type, hipStream_t s);
void launch_fix_omega(const Geom& g, const DevPatch* pt, uint8_t* type, hipStream_t s);
void launch_level0(const Geom& g, const uint8_t* type, const DevPatch* patches, uint8_t* cls,
                   float* cx, float* cy, float* cz, hipStream_t s);
void launch_coarsen(const Geom& fine, const uint8_t* fcls, float* const fcf[3], const Geom& crs,
                    uint8_t* ccls, float* ccf[3], hipStream_t s);
void launch_coarse_factor(const Geom& g, const uint8_t* cls, float* const cf[3], int* cmap,
                          int* ncount, double* work, int max_n, hipStream_t s);

template <class F>
void launch_set_omega_wall(const Geom& g, const Phys& ph, const DevPatch* pt, const uint8_t* type,
                           F* om, hipStream_t s);
template <class F>
void launch_pack(const Geom& g, const double* dense, F* padded, double offset, hipStream_t s);
template <class F>
void launch_unpack(const Geom& g, const F* padded, double* dense, double offset, hipStream_t s);

// Velocity in V, transported scalars (T, k, omega) in F.
template <class V, class F>
struct FieldSet {
  V *u, *v, *w;
  F *T, *k, *om;
};

// second-order explicit stage (option): nu_t from k and omega on fluid
// cells, and out = (a + c) / 2 over the box
template <class V, class F>
void launch_nut(const Geom& g, const Phys& ph, const uint8_t* type, const F* k, const F* om,
                F* nut, hipStream_t s);
template <class V, class F>
void launch_rk2_average(const Geom& g, FieldSet<V, F> a, FieldSet<V, F> c, FieldSet<V, F> out,
                        hipStream_t s);

template <class V, class F>
void launch_destroy(const Geom& g, const Phys& ph, const uint8_t* type, const DevPatch* pt,
                    const V* u, const V* v, const V* w, const F* k, const F* om, double tau,
                    F* k_out, F* om_out, F* nut_out, const RedBuf* red, int tt, hipStream_t s);
// (nut: eddy viscosity per cell, written by the destruction half step that
// precedes the explicit step)
template <class V, class F, class P>
void launch_explicit(const Geom& g, const Phys& ph, const uint8_t* type, const DevPatch* pt,
                     FieldSet<V, F> in, const P* p, const F* nut, FieldSet<V, F> out, int tt,
                     hipStream_t s);
template <class V, class O>
void launch_rhs_b(const Geom& g, const Phys& ph, const uint8_t* type, const DevPatch* pt,
                  const V* u, const V* v, const V* w, O* b, const RedBuf& red, int tt,
                  hipStream_t s);
// reads u* (u, v, w), writes the corrected velocity to (uo, vo, wo); when
// ||b|| = 0 (red.out[S_BB]) the increment phi is taken as 0 and cleared
template <class V, class P, class O>
void launch_project(const Geom& g, const Phys& ph, const uint8_t* type, const DevPatch* pt,
                    O* phi, const V* u, const V* v, const V* w, V* uo, V* vo, V* wo, P* p,
                    const RedBuf& red, int tt, hipStream_t s);

// multigrid (S: storage of the level, C: arithmetic)
// (ctl: red.out; every kernel returns at once when ctl[S_DONE] != 0)
template <class S, class C>
void launch_smooth(const Level& l, const void* xin, void* xout, double wj, bool from_zero,
                   const double* ctl, hipStream_t s);
// Reverse mode of the pressure step (dense FP64 adjoints; rhs and lam are the
// solve's padded right-hand side and solution in the outer type O).
template <class O>
void launch_adj_phibar(const Geom& g, const Phys& ph, const uint8_t* type, const DevPatch* pt,
                       const double* ub, const double* vb, const double* wb, const double* pb,
                       O* rhs, hipStream_t s);
template <class O>
void launch_adj_velocity(const Geom& g, const Phys& ph, const uint8_t* type, const DevPatch* pt,
                         const O* lam, const double* ub, const double* vb, const double* wb,
                         double* usb, double* vsb, double* wsb, hipStream_t s);
// Two sweeps in one pass on a level that takes them (sweep_pair: level 0
// with nx a multiple of 4); bitwise the result of two launch_smooth calls.
bool sweep_pair(const Level& l);
template <class S, class C>
void launch_smooth2(const Level& l, const void* xin, void* xout, double wj, const double* ctl,
                    hipStream_t s);
template <class S, class C, class SC>
void launch_resid_restrict(const Level& f, const Level& c, const double* ctl, hipStream_t s,
                           void* zc = nullptr, double wj = 0.0);
template <class S, class C, class SC>
void launch_prolong(const Level& f, const Level& c, const double* ctl, hipStream_t s);
template <class SC, class C>
void launch_coarse_solve(const Level& c, const int* cmap, const int* ncount, const double* ainv,
                         int max_n, const double* ctl, hipStream_t s);
template <class S>
void launch_fill_zero(const Level& l, void* x, const double* ctl, hipStream_t s);

void launch_mark_full(const Level& l, hipStream_t s);

// One-workgroup V-cycle over levels top .. L-1 with the iterates and
// right-hand sides held in LDS (compute precision); reads b of level top,
// writes x[0] of level top.
constexpr int BOTTOM_MAX_LEVELS = 12;
struct BottomLevel {
  Geom g;
  const uint8_t* cls;
  const float* cf0;
  const float* cf1;
  const float* cf2;
  int n;  // cells (nx * ny * nz)
  // LDS byte offsets: iterates, right-hand side, x / y / z face
  // coefficients, damping over diagonal (wj / D), class bytes
  int bx0, bx1, bb, bfx, bfy, bfz, bwd, bcl;
  float inx, inxy;  // 1 / nx and 1 / (nx ny) for division-free cell indices
};
struct Bottom {
  int nlev;  // levels top .. L-1
  int nu1, nu2;
  double wj;
  BottomLevel lv[BOTTOM_MAX_LEVELS];
  const int* cmap;  // padded indices of the coarsest active cells
  const int* ncount;
  const double* ainv;
  int max_n;
  int bcidx;       // LDS byte offset of the coarsest cells' compact indices
  int zero_bytes;  // leading LDS bytes (iterates, right-hand sides) cleared per launch
  size_t lds_bytes;
  const void* img;  // LDS bytes [zero_bytes, lds_bytes) as built by launch_bottom_image
};
template <class C>
void launch_bottom_image(const Bottom& B, void* img, hipStream_t s);
template <class SC, class C>
size_t bottom_lds_limit();
template <class SC, class C>
void launch_bottom(const Bottom& B, const void* btop, void* xtop, const double* ctl,
                   hipStream_t s);

// flexible CG on level 0 (O: outer type, S: level-0 storage).  The stopping
// rule runs on the device: launch_fcg_start sets S_DONE / S_ITER from tol,
// max_cycles and forced; every later kernel of an iteration returns at once
// when S_DONE is set, so surplus iterations enqueued by the host are no-ops.
// (fin = false: no finalising kernel; used by the autotuner)
template <class O, class S>
void launch_fcg_start(const Level& l0, const O* b, const O* x0, O* r, O* x, const RedBuf& red,
                      bool have_x0, double tol, int max_cycles, int forced, hipStream_t s,
                      bool fin = true, void* z0 = nullptr, double wj = 0.0);
template <class O, class S>
void launch_fcg_apply(const Level& l0, const O* r, void* const* dir, const RedBuf& red,
                      hipStream_t s, bool fin = true);
template <class O, class S>
void launch_fcg_update(const Level& l0, O* x, O* r, void* const* dir, const RedBuf& red,
                       hipStream_t s, bool fin = true, void* z0 = nullptr, double wj = 0.0);

// ---- batched iterations of several grids ----------------------------------------
constexpr int MAX_LEVELS = 20;

// What the batched CG iteration needs of one grid: its levels and V-cycle
// settings, the coarsest solve, and the level-0 CG vectors (outer type O).
struct MgGridDesc {
  Level* lv;  // levels 0 .. L-1; cur is advanced as the iteration is laid out
  int L, bottom_top, nu1, nu2;
  int nu1c, nu2c;  // sweeps on the levels below the finest
  double wj;
  const Bottom* bot;  // when bottom_top >= 0
  const int* cmap;
  const int* ncount;
  const double* ainv;
  int coarse_max;
  void* zero[MAX_LEVELS];  // buffer of level l's fused first sweep, or null
  RedBuf red;
  void *x, *r;
  void* dir[2];  // the two level-0 direction buffers (storage type of level 0)
};

// One flexible-CG iteration of several grids as a list of launches: per
// level, one batched launch covers the tiles of every grid (one workgroup
// per grid for the bottom solves and finalisers).  `blob` holds the argument
// structs and tile lists; each op is called with the device address the
// blob was copied to.
struct BatchOps {
  std::vector<unsigned char> blob;
  std::vector<std::function<void(const unsigned char*, hipStream_t)>> ops;
};
template <class O, class S0, class SC, class C>
void plan_fcg_iteration(MgGridDesc* grids, int n, BatchOps& out);

}  // namespace nfvm
