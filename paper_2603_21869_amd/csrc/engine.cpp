// Host engine of one grid: device buffers, multigrid hierarchy, and the
// order of kernels in a time step (Sec. 2.6: destruction over dt/2, explicit
// step, projection, destruction over dt/2) and in the pressure solve.
#include "engine.hpp"
#include "post.hpp"

#include <math.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <cmath>
#include <map>
#include <mutex>

namespace nfvm {

// ---- allocator hook ------------------------------------------------------------
static nfvm_alloc_fn g_alloc = nullptr;
static nfvm_free_fn g_free = nullptr;
static void* g_ctx = nullptr;

void set_allocator(nfvm_alloc_fn a, nfvm_free_fn f, void* ctx) {
  g_alloc = a;
  g_free = f;
  g_ctx = ctx;
}

void* dev_alloc(size_t bytes) {
  if (g_alloc) return g_alloc(bytes, g_ctx);
  void* p = nullptr;
  if (hipMalloc(&p, bytes) != hipSuccess) {
    (void)hipGetLastError();
    return nullptr;
  }
  return p;
}

void dev_free(void* p) {
  if (!p) return;
  if (g_free) {
    g_free(p, g_ctx);
    return;
  }
  (void)hipFree(p);
}

constexpr int COARSE_MAX = 512;

// ---- descriptor checks ---------------------------------------------------------
void validate_desc(const nfvm_grid_desc& d) {
  auto bad = [](const std::string& m) { throw Error{NFVM_E_INVAL, m}; };
  if (d.dim != 2 && d.dim != 3) bad("dim must be 2 or 3");
  for (int a = 0; a < d.dim; ++a)
    if (d.n[a] < 1 || !(d.h[a] > 0)) bad("cell counts and spacings must be positive");
  if (d.dim == 2 && d.n[2] != 1) bad("2D grids need n[2] == 1");
  if (d.dim == 3 && d.n[2] < 1) bad("n[2] must be positive");
  const long long padded = (long long)(d.n[0] + 18) * (d.n[1] + 2) * (d.n[2] + 2);
  if (padded >= (1LL << 31)) bad("grid too large for 32-bit cell indices");
  if (!(d.dt > 0) || !(d.nu > 0)) bad("dt and nu must be positive");
  if (d.precision < NFVM_FP64 || d.precision > NFVM_MIXED) bad("unknown precision");
  if (d.n_levels < 1 || d.n_levels > MAX_LEVELS) bad("n_levels must be in [1, 20]");
  for (int a = 0; a < d.dim; ++a)
    if (d.n[a] % (1 << (d.n_levels - 1))) bad("every axis must halve exactly n_levels-1 times");
  if (d.nu1 < 0 || d.nu2 < 0 || d.nu1 + d.nu2 < 1) bad("need at least one smoothing sweep");
  if (d.nu_coarse < 0 || d.nu_coarse > 64) bad("nu_coarse must be in 0 .. 64");
  if (d.coarse_fp32_cells < 0) bad("coarse_fp32_cells must not be negative");
  if (d.n_patches < 0 || d.n_patches > MAX_PATCHES - PID_USER) bad("too many patches");
  if (d.n_patches > 0 && !d.patches) bad("patches pointer is NULL");
  for (int q = 0; q < d.n_patches; ++q) {
    const nfvm_patch& p = d.patches[q];
    if (p.face < 0 || p.face >= 2 * d.dim) bad("patch face out of range");
    if (p.kind < NFVM_WALL || p.kind > NFVM_OUTLET) bad("unknown patch kind");
  }
  if (d.max_cycles < 0) bad("max_cycles must be >= 0");
}

static Geom level_geom(const nfvm_grid_desc& d, int l) {
  const int f = 1 << l;
  return make_geom(d.dim, d.n[0] / f, d.n[1] / f, d.dim == 3 ? d.n[2] / f : 1, d.h[0] * f,
                   d.h[1] * f, d.dim == 3 ? d.h[2] * f : d.h[2]);
}

static void sizes_of(int prec, size_t& V, size_t& F, size_t& P, size_t& O, size_t& S0,
                     size_t& SC) {
  if (prec == NFVM_FP64) { V = F = P = O = S0 = SC = 8; }
  else if (prec == NFVM_FP32) { V = F = P = O = S0 = SC = 4; }
  else { V = 8; F = 4; P = 8; O = 8; S0 = 4; SC = 2; }
}

// Blocks of the largest launch of any reducing kernel on a level-0 grid:
// make_tiles covers at most ceil(nx / 64) x ceil(ny / 4) columns (fewer for
// the four-cells-per-thread kernels) times nz planes and rounds the block
// count up to a multiple of 8, and every block, padding ones included,
// stores its partial.
static int max_blocks_of(const Geom& g) {
  const long long t = (long long)((g.nx + 63) / 64) * ((g.ny + 3) / 4) * g.nz;
  return (int)((t + 7) / 8 * 8);
}

// Tile targets (blocks per launch) the autotuner times for each kernel.
static const int TILE_CANDIDATES[] = {512, 2048, 8192, 32768, 1 << 30};
static constexpr int N_TILE_CANDIDATES = 5;

void reduction_blocks(const nfvm_grid_desc& d, int* needed, int* capacity) {
  validate_desc(d);
  const Geom g = level_geom(d, 0);
  int need = 0;
  for (int ci = 0; ci <= N_TILE_CANDIDATES; ++ci) {
    const int t = ci < N_TILE_CANDIDATES ? TILE_CANDIDATES[ci] : TILE_DEFAULT;
    // cell tiles (physics kernels, one-cell CG passes) and four-cell tiles
    need = std::max(need, make_tiles(g.nx, g.ny, g.nz, t).grid);
    if (g.nx % 4 == 0) need = std::max(need, make_tiles(g.nx / 4, g.ny, g.nz, t).grid);
  }
  *needed = need;
  *capacity = max_blocks_of(g);
}

void fail_partials(int nblocks, int nv, int max_blocks) {
  throw Error{NFVM_E_DEVICE, "reduction of " + std::to_string(nblocks) + " blocks x " +
                                 std::to_string(nv) + " values exceeds the partial buffer (" +
                                 std::to_string(max_blocks) + " blocks)"};
}

// Mixed precision: coarse levels with at least this many cells are held in
// FP32, the level-0 storage type, unless the descriptor sets another bound.
constexpr long long COARSE_FP32_CELLS = 131072;

// Whether coarse level l of a grid is stored in the level-0 type rather than
// the coarse one (only mixed precision has two).
static bool wide_level(const nfvm_grid_desc& d, int l) {
  if (d.precision != NFVM_MIXED || l == 0) return false;
  const long long lim = d.coarse_fp32_cells > 0 ? d.coarse_fp32_cells : COARSE_FP32_CELLS;
  return (long long)level_geom(d, l).cells() >= lim;
}

size_t footprint_bytes(const nfvm_grid_desc& d) {
  size_t V, F, P, O, S0, SC;
  sizes_of(d.precision, V, F, P, O, S0, SC);
  const Geom g = level_geom(d, 0);
  const size_t T = (size_t)g.total, N = (size_t)g.cells();
  size_t b = 0;
  b += 6 * T * V + 7 * T * F + T * P + T;           // fields (ping-pong), nu_t, pressure, types
  b += 3 * T * O + 2 * T * S0;                      // b, phi, r; two directions
  b += T * O;                                       // initial guess of the solve call
  b += 8 * N + (d.solid_mask ? N : 0);              // dense staging, mask
  for (int l = 0; l < d.n_levels; ++l) {
    const Geom gl = level_geom(d, l);
    b += (size_t)gl.total * (1 + 4 * d.dim + 3 * (l == 0 || wide_level(d, l) ? S0 : SC));
    b += l == 0 ? (size_t)gl.total * 2 : (size_t)gl.total;  // face codes / full flags
  }
  b += 160 * 1024;                                  // bottom solver's LDS image
  b += (size_t)max_blocks_of(g) * RED_MAX_NV * 8 + 4096;  // reduction partials
  b += (size_t)2 * COARSE_MAX * COARSE_MAX * 8 + COARSE_MAX * 4;  // dense coarse inverse
  b += MAX_PATCHES * sizeof(DevPatch) + 5 * 4 * MAX_PATCHES;
  return b;
}

// ---- autotuner cache ------------------------------------------------------------------
static std::mutex g_tune_mu;
static std::map<TuneKey, int> g_tune;

bool tune_lookup(const TuneKey& k, int* v) {
  std::lock_guard<std::mutex> lk(g_tune_mu);
  auto it = g_tune.find(k);
  if (it == g_tune.end()) return false;
  *v = it->second;
  return true;
}

bool tune_lookup_near(const TuneKey& k, int* v) {
  // the entry of the same kernel, dimension and precision whose shape has
  // the closest cell count (log scale; ties to the smaller shape)
  std::lock_guard<std::mutex> lk(g_tune_mu);
  const double want = std::log((double)k.nx * k.ny * k.nz);
  double best = 1e300;
  bool found = false;
  for (const auto& kv : g_tune) {
    const TuneKey& e = kv.first;
    if (e.kid != k.kid || e.dim != k.dim || e.prec != k.prec) continue;
    const double d = std::fabs(std::log((double)e.nx * e.ny * e.nz) - want);
    if (d < best) {
      best = d;
      *v = kv.second;
      found = true;
    }
  }
  return found;
}

void tune_store(const TuneKey& k, int v) {
  std::lock_guard<std::mutex> lk(g_tune_mu);
  g_tune[k] = v;
}

std::vector<std::pair<TuneKey, int>> tune_entries() {
  std::lock_guard<std::mutex> lk(g_tune_mu);
  return std::vector<std::pair<TuneKey, int>>(g_tune.begin(), g_tune.end());
}

// ---- kernel timing ------------------------------------------------------------------
hipEvent_t GridBase::next_event() {
  if (ev_used == ev_pool.size()) {
    hipEvent_t e;
    NFVM_CK(hipEventCreate(&e));
    ev_pool.push_back(e);
  }
  return ev_pool[ev_used++];
}

thread_local LaunchEvents t_launch_ev;

// The main kernel launched between prof_begin and prof_end records the pair
// of events at its own start and end, and its finaliser (if any) a pair of
// its own.
void GridBase::prof_begin(int kid, double bytes) {
  LaunchEvents e{};
  if (prof_mask & (1u << kid)) {
    ProfRec r{kid, next_event(), next_event(), bytes < 0 ? prof_bytes[kid] : bytes};
    e.start = r.a;
    e.stop = r.b;
    prof_pending.push_back(r);
  }
  if (prof_mask & (1u << NFVM_K_FINALIZE)) {
    ProfRec r{NFVM_K_FINALIZE, next_event(), next_event(), 0.0};
    e.fstart = r.a;
    e.fstop = r.b;
    prof_pending.push_back(r);
  }
  t_launch_ev = e;
}

void GridBase::prof_end(int) {
  // records of launches that did not happen are dropped
  for (hipEvent_t unused : {t_launch_ev.start, t_launch_ev.fstart}) {
    if (!unused) continue;
    for (size_t i = prof_pending.size(); i-- > 0;)
      if (prof_pending[i].a == unused) {
        prof_pending.erase(prof_pending.begin() + i);
        break;
      }
  }
  t_launch_ev = LaunchEvents{};
}

void GridBase::prof_collect() {
  for (const ProfRec& r : prof_pending) {
    float ms = 0;
    NFVM_CK(hipEventElapsedTime(&ms, r.a, r.b));
    prof_launches[r.kid] += 1;
    prof_seconds[r.kid] += ms * 1e-3;
    prof_bytes_sum[r.kid] += r.bytes;
  }
  prof_pending.clear();
  ev_used = 0;
}

void GridBase::prof_reset(uint32_t mask) {
  if (stream) NFVM_CK(hipStreamSynchronize(stream));
  prof_pending.clear();
  ev_used = 0;
  prof_mask = mask;
  for (int k = 0; k < NFVM_K_COUNT; ++k) {
    prof_launches[k] = 0;
    prof_seconds[k] = 0;
    prof_bytes_sum[k] = 0;
  }
}

void GridBase::prof_release() {
  for (hipEvent_t e : ev_pool) (void)hipEventDestroy(e);
  ev_pool.clear();
}

// ---- the grid ------------------------------------------------------------------
template <class V, class F, class P, class O, class S0, class SC, class C>
class GridT : public GridBase {
 public:
  Geom g{};
  Phys ph{};
  int L = 1, nu1 = 2, nu2 = 2;
  int nuc = 0;  // sweeps on the levels below the finest (0: nu1, nu2)
  int pre_of(int l) const { return l > 0 && nuc > 0 ? nuc : nu1; }
  int post_of(int l) const { return l > 0 && nuc > 0 ? nuc : nu2; }
  double wj = 0.8;
  std::vector<std::unique_ptr<DevBuf>> pool;
  uint8_t* type = nullptr;
  DevPatch* patches = nullptr;
  V* vel[3][2] = {};   // u v w
  F* sca[3][2] = {};   // T k omega
  int fcur[6] = {0, 0, 0, 0, 0, 0};
  P* p = nullptr;
  F* nut = nullptr;  // eddy viscosity of the stored k, omega (written by the first half step)
  std::vector<Level> lv;
  O *bvec = nullptr, *phi = nullptr, *r = nullptr, *x0 = nullptr;
  // the two buffers of the CG search direction (level-0 storage type), which
  // alternate between iterations
  void* dir[2] = {nullptr, nullptr};
  double* stage = nullptr;
  double* adj_scratch = nullptr;  // reverse modes of the explicit and destruction steps
  double* adj_dense = nullptr;    // reverse mode of the whole step
  double* adj_heun = nullptr;     // ... and of its Heun explicit stage
  RedBuf red{};
  int* cmap = nullptr;
  int* ncount = nullptr;
  double* work = nullptr;
  double* hs = nullptr;  // host-coherent mirror of the scalars (written by the device)
  double* tune_out = nullptr;  // scratch scalars of the autotuner's CG launches
  hipEvent_t ev_step[2][2] = {};  // start / end of the last two steps
  hipEvent_t ev0 = nullptr, ev1 = nullptr;

  // Device memory of the grid: while the grid is set up, every buffer is
  // carved from one allocation (the arena, sized by the footprint model),
  // 256-byte aligned and followed by a zeroed guard zone that no kernel
  // writes; buffers created later (options) get allocations of their own.
  static constexpr size_t GUARD = 4096;
  DevBuf arena;
  size_t arena_off = 0;
  bool arena_open = false;
  std::vector<std::pair<size_t, std::string>> guards;  // guard offset, buffer before it

  template <class T>
  T* alloc(size_t count, const char* what = "buffer") {
    const size_t bytes = count * sizeof(T);
    if (arena_open) {
      const size_t off = (arena_off + 255) & ~(size_t)255;
      if (off + bytes + GUARD > arena.bytes)
        throw Error{NFVM_E_NOMEM, std::string("grid memory model too small at ") + what};
      arena_off = off + bytes;
      guards.emplace_back(arena_off, what);
      arena_off += GUARD;
      return (T*)((unsigned char*)arena.p + off);
    }
    pool.emplace_back(new DevBuf());
    pool.back()->alloc(bytes, stream);
    return pool.back()->template as<T>();
  }

  // Names of the buffers whose guard zone holds a non-zero byte (an
  // out-of-bounds store past the buffer); empty when all are intact.
  std::string check_guards() override {
    std::string bad;
    if (!arena.p || guards.empty()) return bad;
    NFVM_CK(hipStreamSynchronize(stream));
    std::vector<unsigned char> h(GUARD);
    for (const auto& gr : guards) {
      // (on the grid's stream: a copy on the legacy stream is refused while
      // another thread, a serving lane, captures a graph)
      NFVM_CK(hipMemcpyAsync(h.data(), (unsigned char*)arena.p + gr.first, GUARD,
                             hipMemcpyDeviceToHost, stream));
      NFVM_CK(hipStreamSynchronize(stream));
      for (unsigned char c : h)
        if (c) {
          bad += (bad.empty() ? "" : ", ") + gr.second;
          break;
        }
    }
    return bad;
  }

  ~GridT() override {
    if (stream) (void)hipStreamSynchronize(stream);
    drop_graphs();
    prof_release();
    pool.clear();
    arena.release();
    if (hs) (void)hipHostFree(hs);
    for (auto& pr : ev_step)
      for (hipEvent_t e : pr)
        if (e) (void)hipEventDestroy(e);
    if (ev0) (void)hipEventDestroy(ev0);
    if (ev1) (void)hipEventDestroy(ev1);
    if (own_stream && stream) (void)hipStreamDestroy(stream);
  }

  void init(const nfvm_grid_desc& d, const nfvm_fields* init) {
    // one allocation for every buffer of the set-up (the footprint model
    // bounds them; 2 MiB more covers alignment and guard zones)
    arena.alloc(footprint_bytes(d) + ((size_t)2 << 20), stream);
    arena_open = true;
    desc = d;
    desc.patches = nullptr;
    desc.solid_mask = nullptr;
    tol = d.tol;
    max_cycles = d.max_cycles;
    g = level_geom(d, 0);
    ncells = g.cells();
    L = d.n_levels;
    nu1 = d.nu1;
    nu2 = d.nu2;
    nuc = d.nu_coarse;
    wj = d.omega_jacobi > 0 ? d.omega_jacobi : (d.dim == 3 ? 6.0 / 7.0 : 4.0 / 5.0);
    ph.nu = d.nu;
    ph.alpha_T = d.alpha_T;
    ph.inv_Pr_t = 1.0 / d.Pr_t;
    ph.inv_sigma_k = 1.0 / d.sigma_k;
    ph.inv_sigma_w = 1.0 / d.sigma_w;
    ph.dt = d.dt;
    ph.komega = (d.physics & NFVM_PHYS_KOMEGA) ? 1 : 0;
    ph.energy = (d.physics & NFVM_PHYS_ENERGY) ? 1 : 0;
    ph.buoyancy = (d.physics & NFVM_PHYS_BUOYANCY) ? 1 : 0;
    for (int a = 0; a < 3; ++a) ph.g[a] = d.gravity[a];
    ph.T_ref = d.T_ref;
    ph.beta_T = d.beta_T;

    {
      // algorithmic bytes per launch: operands read once, results written once
      const double N = (double)ncells, sv = sizeof(V), sf = sizeof(F), sp = sizeof(P),
                   so = sizeof(O), s0 = sizeof(S0);
      const double scs = wide_level(d, 1) ? sizeof(S0) : sizeof(SC);  // level 1
      const double nc = L > 1 ? (double)level_geom(d, 1).cells() : 0.0;
      // level 0 reads a 2-byte face code per cell; the restriction also
      // writes the coarse level's first sweep, the CG update the level-0 one
      // (V-cycles with nu1 + nu2 even); the CG passes read z, r and the
      // previous direction (apply), and z, the previous direction, x, r
      // (update, which writes the new direction and forms its image A p
      // from it instead of storing one)
      prof_bytes[NFVM_K_SMOOTH0] = N * (3 * s0 + 2);
      prof_bytes[NFVM_K_SMOOTH0_PAIR] = N * (3 * s0 + 2);  // (two sweeps, one pass)
      prof_bytes[NFVM_K_SMOOTH0_ZERO] = N * (2 * s0 + 2);
      prof_bytes[NFVM_K_RESTRICT0] = N * (2 * s0 + 2) + nc * (2 * scs + 1);
      prof_bytes[NFVM_K_PROLONG0] = N * (2 * s0 + 1) + nc * (scs + 1);
      prof_bytes[NFVM_K_EXPLICIT] = N * (6 * sv + 7 * sf + sp + 1);
      prof_bytes[NFVM_K_DESTROY] = N * (3 * sv + 5 * sf + 1);  // (the first half step)
      prof_bytes[NFVM_K_RHS] = N * (3 * sv + so + 1);
      prof_bytes[NFVM_K_PROJECT] = N * (6 * sv + 2 * sp + so + 1);
      prof_bytes[NFVM_K_FCG_APPLY] = N * (2 * s0 + so + 2);
      // (x is read and written every other iteration)
      prof_bytes[NFVM_K_FCG_UPDATE] = N * (5 * s0 + 3 * so + 2);
    }
    NFVM_CK(hipEventCreate(&ev0));
    NFVM_CK(hipEventCreate(&ev1));
    for (auto& pr : ev_step)
      for (hipEvent_t& e : pr) NFVM_CK(hipEventCreate(&e));
    NFVM_CK(hipHostMalloc((void**)&hs, S_COUNT * sizeof(double),
                          hipHostMallocMapped | hipHostMallocCoherent));
    memset(hs, 0, S_COUNT * sizeof(double));

    // patch table: 0 fluid (unused), 1 solid blocks, 2..7 default walls, then user patches
    std::vector<DevPatch> tab(MAX_PATCHES);
    memset(tab.data(), 0, tab.size() * sizeof(DevPatch));
    for (auto& t : tab) t.kind = K_WALL;
    // temperatures are held as deviations from T_ref on the device
    tab[PID_SOLID].T_dirichlet = isnan(d.T_solid) ? 0 : 1;
    tab[PID_SOLID].T_wall = d.T_solid - d.T_ref;
    std::vector<int> rect(5 * std::max(1, (int)d.n_patches));
    for (int qi = 0; qi < d.n_patches; ++qi) {
      const nfvm_patch& s = d.patches[qi];
      DevPatch& t = tab[PID_USER + qi];
      t.kind = s.kind;
      for (int a = 0; a < 3; ++a) t.U[a] = s.U[a];
      t.T = s.T - d.T_ref;
      t.k = s.k;
      t.omega = s.omega;
      t.T_wall = s.T_wall - d.T_ref;
      t.T_dirichlet = (s.kind == NFVM_WALL && !isnan(s.T_wall)) ? 1 : 0;
      rect[5 * qi + 0] = s.face;
      rect[5 * qi + 1] = s.lo[0];
      rect[5 * qi + 2] = s.lo[1];
      rect[5 * qi + 3] = s.hi[0];
      rect[5 * qi + 4] = s.hi[1];
    }
    patches = alloc<DevPatch>(MAX_PATCHES, "patch table");
    NFVM_CK(hipMemcpyAsync(patches, tab.data(), tab.size() * sizeof(DevPatch),
                           hipMemcpyHostToDevice, stream));
    int* rect_d = alloc<int>(rect.size(), "patch rectangles");
    NFVM_CK(hipMemcpyAsync(rect_d, rect.data(), rect.size() * sizeof(int), hipMemcpyHostToDevice,
                           stream));
    uint8_t* solid_d = nullptr;
    if (d.solid_mask) {
      solid_d = alloc<uint8_t>((size_t)ncells, "solid mask");
      NFVM_CK(hipMemcpyAsync(solid_d, d.solid_mask, (size_t)ncells, hipMemcpyHostToDevice,
                             stream));
    }
    type = alloc<uint8_t>(g.total, "cell types");
    launch_classify(g, solid_d, rect_d, d.n_patches, patches, d.nu, ph.komega, type, stream);
    if (ph.komega) launch_fix_omega(g, patches, type, stream);

    for (int f = 0; f < 3; ++f)
      for (int c = 0; c < 2; ++c) {
        vel[f][c] = alloc<V>(g.total, "velocity");
        sca[f][c] = alloc<F>(g.total, "T/k/omega");
      }
    p = alloc<P>(g.total, "pressure");
    nut = alloc<F>(g.total, "eddy viscosity");
    stage = alloc<double>((size_t)ncells, "host staging");

    // multigrid hierarchy
    lv.resize(L);
    const size_t s0 = sizeof(S0), sc = sizeof(SC);
    for (int l = 0; l < L; ++l) {
      Level& v = lv[l];
      v.g = level_geom(d, l);
      v.cls = alloc<uint8_t>(v.g.total, "level classes");
      v.full = l > 0 ? alloc<uint8_t>(v.g.total, "level full flags") : nullptr;
      for (int a = 0; a < 3; ++a) v.cf[a] = a < d.dim ? alloc<float>(v.g.total, "level face coefficients") : nullptr;
      v.wide = wide_level(d, l);
      const size_t es = l == 0 || v.wide ? s0 : sc;
      for (int c = 0; c < 2; ++c) v.x[c] = alloc<uint8_t>(v.g.total * es, "level iterate");
      v.b = alloc<uint8_t>(v.g.total * es, "level right-hand side");
      v.cur = 0;
      v.code = nullptr;
      for (int t = 0; t < TK_LEVEL_COUNT; ++t) v.tt[t] = TILE_DEFAULT;
      if (l == 0) {
        launch_level0(v.g, type, patches, v.cls, v.cf[0], v.cf[1], d.dim == 3 ? v.cf[2] : v.cf[0],
                      stream);
        v.code = alloc<uint16_t>(v.g.total, "face codes");
        launch_face_codes(v.g, v.cls, v.cf[0], v.cf[1], d.dim == 3 ? v.cf[2] : v.cf[0], v.code,
                          stream);
      } else
        launch_coarsen(lv[l - 1].g, lv[l - 1].cls, lv[l - 1].cf, v.g, v.cls, v.cf, stream);
      if (l > 0) launch_mark_full(v, stream);
    }
    cmap = alloc<int>(COARSE_MAX, "coarsest map");
    ncount = alloc<int>(1, "coarsest count");
    work = alloc<double>((size_t)2 * COARSE_MAX * COARSE_MAX, "coarsest inverse");
    launch_coarse_factor(lv[L - 1].g, lv[L - 1].cls, lv[L - 1].cf, cmap, ncount, work, COARSE_MAX,
                         stream);
    NFVM_CK(hipGetLastError());
    int nc = 0;
    NFVM_CK(hipMemcpyAsync(&nc, ncount, sizeof(int), hipMemcpyDeviceToHost, stream));
    NFVM_CK(hipStreamSynchronize(stream));
    if (nc > COARSE_MAX)
      throw Error{NFVM_E_INVAL, "coarsest level has " + std::to_string(nc) +
                                    " fluid cells; at most 512 (add levels)"};
    n_coarse = nc;

    setup_bottom();

    bvec = alloc<O>(g.total, "Poisson b");
    phi = alloc<O>(g.total, "CG x");
    r = alloc<O>(g.total, "CG r");
    dir[0] = alloc<S0>(g.total, "CG direction (even iterations)");
    dir[1] = alloc<S0>(g.total, "CG direction (odd iterations)");
    x0 = alloc<O>(g.total, "initial guess");
    red.max_blocks = max_blocks_of(g);
    red.partial = alloc<double>((size_t)red.max_blocks * RED_MAX_NV, "reduction partials");
    red.out = alloc<double>(S_COUNT, "solver scalars");
    {
      double init[S_COUNT] = {};
      init[S_FORCED] = 1e30;
      tune_out = alloc<double>(S_COUNT, "tuning scalars");
      NFVM_CK(hipMemcpyAsync(tune_out, init, sizeof init, hipMemcpyHostToDevice, stream));
      NFVM_CK(hipStreamSynchronize(stream));
    }
    NFVM_CK(hipHostGetDevicePointer((void**)&red.mirror, hs, 0));

    arena_open = false;
    for (int t = 0; t < TP_COUNT; ++t) tp[t] = TILE_DEFAULT;
    if (use_autotune) autotune();
    clear_increment();
    if (init) set_fields(init);
    NFVM_CK(hipStreamSynchronize(stream));
  }

  // The pressure increment of the last step, the initial guess of the next
  // step's solve; cleared whenever it no longer belongs to the stored fields.
  void clear_increment() {
    NFVM_CK(hipMemsetAsync(phi, 0, (size_t)g.total * sizeof(O), stream));
  }

  // ---- autotuner: for every tunable kernel and level, time a few tile
  // targets on this grid and keep the fastest (cached per shape and
  // precision for the process).
  int tp[TP_COUNT];

  template <class Fn>
  float time_it(Fn&& fn) {
    fn();  // warm
    NFVM_CK(hipEventRecord(ev0, stream));
    for (int r = 0; r < 3; ++r) fn();
    NFVM_CK(hipEventRecord(ev1, stream));
    NFVM_CK(hipEventSynchronize(ev1));
    float ms = 0;
    NFVM_CK(hipEventElapsedTime(&ms, ev0, ev1));
    return ms;
  }

  bool tune_cached_only = false;

  template <class Fn>
  int tune_one(int kid, const Geom& gg, Fn&& launch) {
    const int* cand = TILE_CANDIDATES;
    TuneKey key{kid, gg.nx, gg.ny, gg.nz, desc.dim, desc.precision};
    int cached;
    if (tune_lookup(key, &cached)) return cached;
    // served grids never tune: the choice of the tuned shape nearest in
    // size, else the default
    if (tune_cached_only) return tune_lookup_near(key, &cached) ? cached : TILE_DEFAULT;
    int best = TILE_DEFAULT;
    float bt = 1e30f;
    for (int ci = 0; ci < N_TILE_CANDIDATES; ++ci) {
      const int c = cand[ci];
      const float t = time_it([&] { launch(c); });
      if (t < bt) {
        bt = t;
        best = c;
      }
    }
    tune_store(key, best);
    return best;
  }

  void autotune() {
    NFVM_CK(hipStreamSynchronize(stream));
    // physics kernels first: phi is still zero, so the projection leaves p alone
    {
      FieldSet<V, F> in{vcur(0), vcur(1), vcur(2), scur(3), scur(4), scur(5)};
      FieldSet<V, F> out{valt(0), valt(1), valt(2), salt(3), salt(4), salt(5)};
      tp[TP_EXPLICIT] = tune_one(100 + TP_EXPLICIT, g, [&](int tt) {
        launch_explicit<V, F, P>(g, ph, type, patches, in, p, nut, out, tt, stream);
      });
      tp[TP_DESTROY] = tune_one(100 + TP_DESTROY, g, [&](int tt) {
        launch_destroy<V, F>(g, ph, type, patches, vcur(0), vcur(1), vcur(2), scur(4), scur(5),
                             0.0, salt(4), salt(5), nut, nullptr, tt, stream);
      });
      tp[TP_RHS] = tune_one(100 + TP_RHS, g, [&](int tt) {
        launch_rhs_b<V, O>(g, ph, type, patches, vcur(0), vcur(1), vcur(2), bvec, red, tt, stream);
      });
      tp[TP_PROJECT] = tune_one(100 + TP_PROJECT, g, [&](int tt) {
        launch_project<V, P, O>(g, ph, type, patches, phi, vcur(0), vcur(1), vcur(2), valt(0),
                                valt(1), valt(2), p, red, tt, stream);
      });
    }
    const int last = bottom_top >= 0 ? bottom_top : L - 1;  // levels with per-level kernels
    for (int l = 0; l < last; ++l) {
      Level& v = lv[l];
      if (l == 0) {
        v.tt[TK_SMOOTH] = tune_one(TK_SMOOTH, v.g, [&](int tt) {
          v.tt[TK_SMOOTH] = tt;
          launch_smooth<S0, C>(v, v.x[0], v.x[1], wj, false, red.out, stream);
        });
        v.tt[TK_SMOOTH_ZERO] = tune_one(TK_SMOOTH_ZERO, v.g, [&](int tt) {
          v.tt[TK_SMOOTH_ZERO] = tt;
          launch_smooth<S0, C>(v, nullptr, v.x[0], wj, true, red.out, stream);
        });
        if (sweep_pair(v))
          v.tt[TK_SMOOTH2] = tune_one(TK_SMOOTH2, v.g, [&](int tt) {
            v.tt[TK_SMOOTH2] = tt;
            launch_smooth2<S0, C>(v, v.x[0], v.x[1], wj, red.out, stream);
          });
        v.tt[TK_RESTRICT] = tune_one(TK_RESTRICT + (lv[1].wide ? 4000 : 0), v.g, [&](int tt) {
          v.tt[TK_RESTRICT] = tt;
          restrict_as(0);
        });
        v.tt[TK_PROLONG] = tune_one(TK_PROLONG + (lv[1].wide ? 4000 : 0), v.g, [&](int tt) {
          v.tt[TK_PROLONG] = tt;
          prolong_as(0);
        });
        v.tt[TK_START] = tune_one(TK_START, v.g, [&](int tt) {
          v.tt[TK_START] = tt;
          launch_fcg_start<O, S0>(v, bvec, x0, r, phi, red, false, 1.0, 1, -1, stream, false,
                                  zero0(), wj);
        });
        // the CG passes are timed with their finalising kernels (the block
        // count they sum grows with the tile count), on scratch scalars whose
        // stopping rule never fires (forced count 1e30)
        RedBuf tr = red;
        tr.out = tune_out;
        tr.mirror = nullptr;
        v.tt[TK_APPLY] = tune_one(TK_APPLY, v.g, [&](int tt) {
          v.tt[TK_APPLY] = tt;
          launch_fcg_apply<O, S0>(v, r, dir, tr, stream, true);
        });
        v.tt[TK_UPDATE] = tune_one(TK_UPDATE, v.g, [&](int tt) {
          v.tt[TK_UPDATE] = tt;
          launch_fcg_update<O, S0>(v, phi, r, dir, tr, stream, true, zero0(), wj);
        });
      } else {
        // (the tuning key tells the storage types of the level and the next)
        const int tk = 1000 + (v.wide ? 2000 : 0) + (lv[l + 1].wide ? 4000 : 0);
        v.tt[TK_SMOOTH] = tune_one(TK_SMOOTH + tk, v.g, [&](int tt) {
          v.tt[TK_SMOOTH] = tt;
          smooth_as(l, v.x[0], v.x[1], false);
        });
        v.tt[TK_SMOOTH_ZERO] = tune_one(TK_SMOOTH_ZERO + tk, v.g, [&](int tt) {
          v.tt[TK_SMOOTH_ZERO] = tt;
          smooth_as(l, nullptr, v.x[0], true);
        });
        v.tt[TK_RESTRICT] = tune_one(TK_RESTRICT + tk, v.g, [&](int tt) {
          v.tt[TK_RESTRICT] = tt;
          restrict_as(l);
        });
        v.tt[TK_PROLONG] = tune_one(TK_PROLONG + tk, v.g, [&](int tt) {
          v.tt[TK_PROLONG] = tt;
          prolong_as(l);
        });
      }
    }
    NFVM_CK(hipGetLastError());
    // leave every buffer the tuning touched as a fresh grid has it
    const size_t ob = (size_t)g.total * sizeof(O);
    for (O* bufp : {bvec, phi, r, x0}) NFVM_CK(hipMemsetAsync(bufp, 0, ob, stream));
    for (void* d : dir) NFVM_CK(hipMemsetAsync(d, 0, (size_t)g.total * sizeof(S0), stream));
    for (int l = 0; l < L; ++l) {
      const size_t es = (size_t)lv[l].g.total * elem_size(l);
      for (int c = 0; c < 2; ++c) NFVM_CK(hipMemsetAsync(lv[l].x[c], 0, es, stream));
      NFVM_CK(hipMemsetAsync(lv[l].b, 0, es, stream));
    }
    NFVM_CK(hipMemsetAsync(red.out, 0, S_COUNT * sizeof(double), stream));
    NFVM_CK(hipMemsetAsync(red.partial, 0, (size_t)red.max_blocks * RED_MAX_NV * sizeof(double),
                           stream));
    NFVM_CK(hipStreamSynchronize(stream));
  }

  // ---- fields -------------------------------------------------------------------
  V* vcur(int f) { return vel[f][fcur[f]]; }
  V* valt(int f) { return vel[f][fcur[f] ^ 1]; }
  F* scur(int f) { return sca[f - 3][fcur[f]]; }
  F* salt(int f) { return sca[f - 3][fcur[f] ^ 1]; }

  void set_fields(const nfvm_fields* in) override {
    const double* src[7] = {in->u, in->v, in->w, in->T, in->k, in->omega, in->p};
    for (int f = 0; f < 7; ++f)
      if (!src[f]) throw Error{NFVM_E_INVAL, "all seven field pointers are required"};
    const size_t bytes = (size_t)ncells * sizeof(double);
    for (int f = 0; f < 6; ++f) {
      NFVM_CK(hipMemcpyAsync(stage, src[f], bytes, hipMemcpyHostToDevice, stream));
      if (f < 3)
        launch_pack<V>(g, stage, vcur(f), 0.0, stream);
      else
        launch_pack<F>(g, stage, scur(f), f == 3 ? ph.T_ref : 0.0, stream);
      NFVM_CK(hipStreamSynchronize(stream));
    }
    NFVM_CK(hipMemcpyAsync(stage, src[6], bytes, hipMemcpyHostToDevice, stream));
    launch_pack<P>(g, stage, p, 0.0, stream);
    if (ph.komega) launch_set_omega_wall<F>(g, ph, patches, type, scur(5), stream);
    clear_increment();
    NFVM_CK(hipGetLastError());
    NFVM_CK(hipStreamSynchronize(stream));
  }

  void get_fields(nfvm_fields* out) override {
    double* dst[7] = {out->u, out->v, out->w, out->T, out->k, out->omega, out->p};
    for (int f = 0; f < 7; ++f)
      if (!dst[f]) throw Error{NFVM_E_INVAL, "all seven field pointers are required"};
    const size_t bytes = (size_t)ncells * sizeof(double);
    for (int f = 0; f < 7; ++f) {
      if (f < 3)
        launch_unpack<V>(g, vcur(f), stage, 0.0, stream);
      else if (f < 6)
        launch_unpack<F>(g, scur(f), stage, f == 3 ? ph.T_ref : 0.0, stream);
      else
        launch_unpack<P>(g, p, stage, 0.0, stream);
      NFVM_CK(hipMemcpyAsync(dst[f], stage, bytes, hipMemcpyDeviceToHost, stream));
      NFVM_CK(hipStreamSynchronize(stream));
    }
  }

  void lambda2(double* out) override {
    if (!out) throw Error{NFVM_E_INVAL, "an output array is required"};
    launch_lambda2<V>(g, ph, type, patches, vcur(0), vcur(1), vcur(2), stage, stream);
    NFVM_CK(hipGetLastError());
    NFVM_CK(hipMemcpyAsync(out, stage, (size_t)ncells * sizeof(double), hipMemcpyDeviceToHost,
                           stream));
    NFVM_CK(hipStreamSynchronize(stream));
  }

  void probe(const double* pts, int n, double* out) override {
    if (n < 0 || (n > 0 && (!pts || !out)))
      throw Error{NFVM_E_INVAL, "points and an output array are required"};
    // points and results pass through the staging buffer
    if ((long long)7 * n > ncells)
      throw Error{NFVM_E_INVAL, "at most " + std::to_string(ncells / 7) +
                                    " probe points per call on this grid"};
    if (n == 0) return;
    double* dp = stage;
    double* dout = stage + 3 * (size_t)n;
    NFVM_CK(hipMemcpyAsync(dp, pts, 3 * (size_t)n * sizeof(double), hipMemcpyHostToDevice,
                           stream));
    launch_probe<V, F>(g, type, vcur(0), vcur(1), vcur(2), scur(3), scur(4), scur(5), ph.T_ref,
                       dp, n, dout, stream);
    NFVM_CK(hipGetLastError());
    NFVM_CK(hipMemcpyAsync(out, dout, 4 * (size_t)n * sizeof(double), hipMemcpyDeviceToHost,
                           stream));
    NFVM_CK(hipStreamSynchronize(stream));
  }

  void explicit_adjoint(const nfvm_fields& st, const nfvm_fields& bar,
                        const nfvm_fields& out) override {
    const double* sp[7] = {st.u, st.v, st.w, st.p, st.T, st.k, st.omega};
    const double* yb[6] = {bar.u, bar.v, bar.w, bar.T, bar.k, bar.omega};
    double* xb[7] = {out.u, out.v, out.w, out.p, out.T, out.k, out.omega};
    for (const double* q : sp)
      if (!q) throw Error{NFVM_E_INVAL, "all seven state arrays are required"};
    for (const double* q : yb)
      if (!q) throw Error{NFVM_E_INVAL, "the six output adjoints are required"};
    for (double* q : xb)
      if (!q) throw Error{NFVM_E_INVAL, "all seven input adjoint arrays are required"};
    const size_t T = (size_t)g.total;
    // (allocated on first use: 22 padded FP64 arrays)
    if (!adj_scratch) adj_scratch = alloc<double>(22 * T, "adjoint scratch");
    double* S = adj_scratch;
    // (the Jacobian does not depend on p, which is therefore not packed)
    const double* sd[7];
    for (int f = 0; f < 7; ++f) {
      sd[f] = f == 3 ? nullptr : S + f * T;
      if (f != 3) launch_pack<double>(g, sp[f], S + f * T, f == 4 ? ph.T_ref : 0.0, stream);
    }
    launch_explicit_adjoint(g, ph, type, patches, sd, yb, S + 7 * T, S + 13 * T, S + 15 * T,
                            S + 21 * T, xb, stream);
    NFVM_CK(hipGetLastError());
    NFVM_CK(hipStreamSynchronize(stream));
  }

  void destroy_adjoint(const nfvm_fields& st, double tau, const double* kb, const double* wb,
                       const nfvm_fields& out) override {
    const double* sp[5] = {st.u, st.v, st.w, st.k, st.omega};
    double* xb[5] = {out.u, out.v, out.w, out.k, out.omega};
    for (const double* q : sp)
      if (!q) throw Error{NFVM_E_INVAL, "the state's u, v, w, k and omega are required"};
    for (double* q : xb)
      if (!q) throw Error{NFVM_E_INVAL, "the adjoints of u, v, w, k and omega are required"};
    if (!kb || !wb) throw Error{NFVM_E_INVAL, "the adjoints of k and omega are required"};
    if (!(tau >= 0.0)) throw Error{NFVM_E_INVAL, "tau must be >= 0"};
    const size_t T = (size_t)g.total;
    if (!adj_scratch) adj_scratch = alloc<double>(22 * T, "adjoint scratch");
    double* S = adj_scratch;
    const double* sd[5];
    for (int f = 0; f < 5; ++f) {
      launch_pack<double>(g, sp[f], S + f * T, 0.0, stream);
      sd[f] = S + f * T;
    }
    launch_destroy_adjoint(g, ph, type, patches, sd, tau, kb, wb, S + 5 * T, S + 11 * T, xb,
                           stream);
    NFVM_CK(hipGetLastError());
    NFVM_CK(hipStreamSynchronize(stream));
  }

  // Reverse mode of one whole step at a state: the step is run forward from
  // the state on the grid's fields (which keep its result), with the stage
  // inputs the reverse modes need kept as dense copies, then the stages'
  // reverse modes are applied in reverse order.
  void step_adjoint(const nfvm_fields& st, const nfvm_fields& bar, const nfvm_fields& out,
                    double tol_, int maxc, int forced, nfvm_step_stats* stt,
                    nfvm_status* status) override {
    const double* sp[7] = {st.u, st.v, st.w, st.p, st.T, st.k, st.omega};
    const double* bp[7] = {bar.u, bar.v, bar.w, bar.p, bar.T, bar.k, bar.omega};
    double* op[7] = {out.u, out.v, out.w, out.p, out.T, out.k, out.omega};
    for (int f = 0; f < 7; ++f)
      if (!sp[f] || !bp[f] || !op[f])
        throw Error{NFVM_E_INVAL, "all seven state, adjoint and output arrays are required"};
    const size_t N = (size_t)ncells;
    // dense scratch: s0 (7), k and omega after the first destruction (2),
    // the explicit stage's u, v, w, k, omega (5), the projected u, v, w (3),
    // the adjoint of that velocity (3), a destruction's reverse mode (5),
    // the pressure step's (3), the explicit stage's (7)
    if (!adj_dense) adj_dense = alloc<double>(35 * N, "step adjoint scratch");
    double* D = adj_dense;
    auto slot = [&](int q) { return D + (size_t)q * N; };
    // Heun's stage (U + E(E(U))) / 2: the first stage's u v w T k omega (6),
    // the second stage's input adjoints (7), the first stage's (7)
    if (rk_order == 2 && !adj_heun) adj_heun = alloc<double>(20 * N, "Heun step adjoint scratch");
    auto hslot = [&](int q) { return adj_heun + (size_t)q * N; };
    NFVM_CK(hipStreamSynchronize(stream));
    // the state as the grid's fields, omega held on wall-adjacent cells (as
    // nfvm_set_fields loads fields)
    for (int f = 0; f < 3; ++f) launch_pack<V>(g, sp[f], vcur(f), 0.0, stream);
    launch_pack<P>(g, sp[3], p, 0.0, stream);
    launch_pack<F>(g, sp[4], scur(3), ph.T_ref, stream);
    launch_pack<F>(g, sp[5], scur(4), 0.0, stream);
    launch_pack<F>(g, sp[6], scur(5), 0.0, stream);
    if (ph.komega) launch_set_omega_wall<F>(g, ph, patches, type, scur(5), stream);
    clear_increment();
    for (int f = 0; f < 3; ++f) launch_unpack<V>(g, vcur(f), slot(f), 0.0, stream);
    launch_unpack<P>(g, p, slot(3), 0.0, stream);
    launch_unpack<F>(g, scur(3), slot(4), ph.T_ref, stream);
    launch_unpack<F>(g, scur(4), slot(5), 0.0, stream);
    launch_unpack<F>(g, scur(5), slot(6), 0.0, stream);
    // forward: destruction over dt/2, explicit stage, pressure step
    const double half = 0.5 * ph.dt;
    if (ph.komega) {
      launch_destroy<V, F>(g, ph, type, patches, vcur(0), vcur(1), vcur(2), scur(4), scur(5),
                           half, salt(4), salt(5), nut, nullptr, tp[TP_DESTROY], stream);
      swap(4);
      swap(5);
    }
    launch_unpack<F>(g, scur(4), slot(7), 0.0, stream);
    launch_unpack<F>(g, scur(5), slot(8), 0.0, stream);
    {
      FieldSet<V, F> in{vcur(0), vcur(1), vcur(2), scur(3), scur(4), scur(5)};
      FieldSet<V, F> outf{valt(0), valt(1), valt(2), salt(3), salt(4), salt(5)};
      launch_explicit<V, F, P>(g, ph, type, patches, in, p, nut, outf, tp[TP_EXPLICIT], stream);
      if (rk_order == 2) {
        // the first stage kept, then the second Euler step from it (nu_t of
        // its k and omega) averaged with the start, as the step takes it
        launch_unpack<V>(g, outf.u, hslot(0), 0.0, stream);
        launch_unpack<V>(g, outf.v, hslot(1), 0.0, stream);
        launch_unpack<V>(g, outf.w, hslot(2), 0.0, stream);
        launch_unpack<F>(g, outf.T, hslot(3), ph.T_ref, stream);
        launch_unpack<F>(g, outf.k, hslot(4), 0.0, stream);
        launch_unpack<F>(g, outf.om, hslot(5), 0.0, stream);
        if (ph.komega) launch_nut<V, F>(g, ph, type, outf.k, outf.om, nut, stream);
        launch_explicit<V, F, P>(g, ph, type, patches, outf, p, nut, rk2, tp[TP_EXPLICIT],
                                 stream);
        launch_rk2_average<V, F>(g, in, rk2, outf, stream);
      }
      for (int f = 0; f < 6; ++f) swap(f);
    }
    for (int f = 0; f < 3; ++f) launch_unpack<V>(g, vcur(f), slot(9 + f), 0.0, stream);
    launch_unpack<F>(g, scur(4), slot(12), 0.0, stream);
    launch_unpack<F>(g, scur(5), slot(13), 0.0, stream);
    launch_rhs_b<V, O>(g, ph, type, patches, vcur(0), vcur(1), vcur(2), bvec, red, tp[TP_RHS],
                       stream);
    int cyc = 0;
    double rel = 0.0;
    last_diag.clear();
    nfvm_status sst = solve(false, tol_, maxc, forced, &cyc, &rel);
    if (sst == NFVM_E_DIVERGED) {
      last_diag = diagnose();
      *status = sst;
      return;
    }
    flush_x();
    launch_project<V, P, O>(g, ph, type, patches, phi, vcur(0), vcur(1), vcur(2), valt(0),
                            valt(1), valt(2), p, red, tp[TP_PROJECT], stream);
    swap(0);
    swap(1);
    swap(2);
    for (int f = 0; f < 3; ++f) launch_unpack<V>(g, vcur(f), slot(14 + f), 0.0, stream);
    if (ph.komega) {  // (completes the step on the grid's fields)
      launch_destroy<V, F>(g, ph, type, patches, vcur(0), vcur(1), vcur(2), scur(4), scur(5),
                           half, salt(4), salt(5), nullptr, nullptr, tp[TP_DESTROY], stream);
      swap(4);
      swap(5);
    }
    clear_increment();
    NFVM_CK(hipGetLastError());
    NFVM_CK(hipStreamSynchronize(stream));
    if (stt) {
      memset(&stt[0], 0, sizeof stt[0]);
      stt[0].cycles = cyc;
      stt[0].status = sst;
      stt[0].rel_residual = rel;
      stt[0].min_k = stt[0].min_omega = NAN;
    }
    // reverse: second destruction (its velocity is the projected one, also a
    // step output), pressure step, explicit stage, first destruction
    double* ub1[3] = {slot(17), slot(18), slot(19)};
    double* d5[5] = {slot(20), slot(21), slot(22), slot(23), slot(24)};
    const double* ksb = bp[5];
    const double* wsb = bp[6];
    if (ph.komega) {
      const nfvm_fields s2{slot(14), slot(15), slot(16), nullptr, nullptr, slot(12), slot(13)};
      const nfvm_fields o2{d5[0], d5[1], d5[2], nullptr, nullptr, d5[3], d5[4]};
      destroy_adjoint(s2, half, bp[5], bp[6], o2);
      for (int f = 0; f < 3; ++f) launch_dense_add(N, bp[f], d5[f], ub1[f], stream);
      ksb = d5[3];
      wsb = d5[4];
    } else {
      for (int f = 0; f < 3; ++f)
        NFVM_CK(hipMemcpyAsync(ub1[f], bp[f], N * sizeof(double), hipMemcpyDeviceToDevice,
                               stream));
    }
    double* usb[3] = {slot(25), slot(26), slot(27)};
    nfvm_status ast = NFVM_OK;
    pressure_adjoint(ub1[0], ub1[1], ub1[2], bp[3], usb[0], usb[1], usb[2], tol_, maxc, forced,
                     stt ? &stt[1] : nullptr, &ast);
    if (ast == NFVM_E_DIVERGED) {
      *status = ast;
      return;
    }
    double* xo[7];
    for (int f = 0; f < 7; ++f) xo[f] = slot(28 + f);
    {
      const nfvm_fields s1{slot(0), slot(1), slot(2), slot(3), slot(4), slot(7), slot(8)};
      const nfvm_fields b1{usb[0], usb[1], usb[2], nullptr, const_cast<double*>(bp[4]),
                           const_cast<double*>(ksb), const_cast<double*>(wsb)};
      const nfvm_fields o1{xo[0], xo[1], xo[2], xo[3], xo[4], xo[5], xo[6]};
      if (rk_order == 2) {
        // the adjoint of (U + E(E(U))) / 2 is (b + J1^T J2^T b) / 2, J2 the
        // Jacobian of the second stage at the first stage's output U1, J1 that
        // of the first at U (p passes to both stages)
        const nfvm_fields s2{hslot(0), hslot(1), hslot(2), slot(3), hslot(3), hslot(4), hslot(5)};
        const nfvm_fields z{hslot(6), hslot(7), hslot(8), hslot(9), hslot(10), hslot(11),
                            hslot(12)};
        explicit_adjoint(s2, b1, z);
        const nfvm_fields zb{z.u, z.v, z.w, nullptr, z.T, z.k, z.omega};
        const nfvm_fields y{hslot(13), hslot(14), hslot(15), hslot(16), hslot(17), hslot(18),
                            hslot(19)};
        explicit_adjoint(s1, zb, y);
        const double* b6[6] = {usb[0], usb[1], usb[2], bp[4], ksb, wsb};
        const double* y6[6] = {y.u, y.v, y.w, y.T, y.k, y.omega};
        double* x6[6] = {xo[0], xo[1], xo[2], xo[4], xo[5], xo[6]};
        for (int f = 0; f < 6; ++f) launch_dense_add(N, b6[f], y6[f], x6[f], stream, 0.5);
        launch_dense_add(N, z.p, y.p, xo[3], stream, 0.5);
      } else {
        explicit_adjoint(s1, b1, o1);
      }
    }
    launch_dense_add(N, bp[3], xo[3], op[3], stream);  // p^n also passes to p
    NFVM_CK(hipMemcpyAsync(op[4], xo[4], N * sizeof(double), hipMemcpyDeviceToDevice, stream));
    if (ph.komega) {
      const nfvm_fields s0{slot(0), slot(1), slot(2), nullptr, nullptr, slot(5), slot(6)};
      const nfvm_fields o0{d5[0], d5[1], d5[2], nullptr, nullptr, d5[3], d5[4]};
      destroy_adjoint(s0, half, xo[5], xo[6], o0);
      for (int f = 0; f < 3; ++f) launch_dense_add(N, xo[f], d5[f], op[f], stream);
      NFVM_CK(hipMemcpyAsync(op[5], d5[3], N * sizeof(double), hipMemcpyDeviceToDevice, stream));
      NFVM_CK(hipMemcpyAsync(op[6], d5[4], N * sizeof(double), hipMemcpyDeviceToDevice, stream));
      // the load holds omega on wall-adjacent cells whatever its input
      launch_zero_held(g, type, op[6], stream);
    } else {
      for (int f : {0, 1, 2, 5, 6})
        NFVM_CK(hipMemcpyAsync(op[f], xo[f], N * sizeof(double), hipMemcpyDeviceToDevice,
                               stream));
    }
    NFVM_CK(hipGetLastError());
    NFVM_CK(hipStreamSynchronize(stream));
    *status = sst != NFVM_OK ? sst : ast;
  }

  // ---- multigrid ------------------------------------------------------------------
  // Storage type of level l: the level-0 type on level 0 and on wide coarse
  // levels, the coarse type elsewhere.  fn is called with a value of it.
  template <class Fn>
  void as_level(int l, Fn&& fn) const {
    if (l == 0 || lv[l].wide)
      fn(S0{});
    else
      fn(SC{});
  }
  size_t elem_size(int l) const { return l == 0 || lv[l].wide ? sizeof(S0) : sizeof(SC); }
  // sweep on level l >= 1, residual and restriction from level l to l + 1,
  // prolongation and correction from level l + 1 to l, in the levels' types
  void smooth_as(int l, const void* xin, void* xout, bool zero) {
    as_level(l, [&](auto t) {
      launch_smooth<decltype(t), C>(lv[l], xin, xout, wj, zero, red.out, stream);
    });
  }
  void restrict_as(int l) {
    as_level(l, [&](auto f) {
      as_level(l + 1, [&](auto c) {
        launch_resid_restrict<decltype(f), C, decltype(c)>(lv[l], lv[l + 1], red.out, stream,
                                                           zero_of(l + 1), wj);
      });
    });
  }
  void prolong_as(int l) {
    as_level(l, [&](auto f) {
      as_level(l + 1, [&](auto c) {
        launch_prolong<decltype(f), C, decltype(c)>(lv[l], lv[l + 1], red.out, stream);
      });
    });
  }

  void smooth(int l, bool zero) {
    Level& v = lv[l];
    const void* xin = zero ? nullptr : v.x[v.cur];
    void* xout = zero ? v.x[0] : v.x[v.cur ^ 1];
    const int kid = zero ? NFVM_K_SMOOTH0_ZERO : NFVM_K_SMOOTH0;
    if (l == 0) {
      prof_begin(kid);
      launch_smooth<S0, C>(v, xin, xout, wj, zero, red.out, stream);
      prof_end(kid);
    } else {
      // x in, b, x out and the class byte (from zero: no x in)
      const double nc = (double)v.g.cells(), sc = elem_size(l);
      prof_begin(NFVM_K_SMOOTH_C, nc * ((zero ? 2 : 3) * sc + 1));
      smooth_as(l, xin, xout, zero);
      prof_end(NFVM_K_SMOOTH_C);
    }
    v.cur = zero ? 0 : (v.cur ^ 1);
  }

  // Algorithmic bytes of the coarse-level transfers between levels l and
  // l + 1 (the fine side: x, b and class byte read, or x read and written
  // with the class byte; the coarse side: b and the fused first sweep
  // written with the class byte, or the correction read with it).
  double restrict_bytes(int l, bool fused) const {
    const double nf = (double)lv[l].g.cells(), nc = (double)lv[l + 1].g.cells();
    const double sf = elem_size(l), sc = elem_size(l + 1);
    return nf * (2 * sf + 1) + nc * ((fused ? 2 : 1) * sc + 1);
  }
  double prolong_bytes(int l) const {
    const double nf = (double)lv[l].g.cells(), nc = (double)lv[l + 1].g.cells();
    const double sf = elem_size(l), sc = elem_size(l + 1);
    return nf * (2 * sf + 1) + nc * (sc + 1);
  }
  // the bottom solver: its top level's b read and x written, the constant
  // LDS image read; the coarsest dense solve: the inverse and its vectors
  double bottom_bytes_moved() const {
    const double nt = (double)lv[bottom_top].g.cells(), sc = elem_size(bottom_top);
    return nt * 2 * sc + (double)(bot.lds_bytes - bot.zero_bytes);
  }
  double coarse_bytes_moved() const {
    const double n = (double)n_coarse, sc = elem_size(L - 1);
    return n * n * 8 + n * (2 * sc + 4);
  }
  // CG start: b read, r and x written, the level-0 right-hand side and (fused)
  // first sweep written, the face code; with an initial guess it is read too
  double start_bytes(bool have_x0) const {
    const double N = (double)ncells, so = sizeof(O), s0 = sizeof(S0);
    return N * ((have_x0 ? 4 : 3) * so + 2 + (zero0() ? 2 : 1) * s0);
  }
  int n_coarse = 0;  // active cells of the coarsest level

  // levels bottom_top .. L-1 run in one LDS-resident workgroup
  int bottom_top = -1;
  // nearest (piecewise-constant) prolongation on every level; the bottom
  // solver's prolongation is linear, so it is not used then
  bool nearest = false;
  // explicit stage: 1 forward Euler, 2 Heun (second stage written to rk2)
  int rk_order = 1;
  // Algorithm 1 as printed: V(0,1) cycle of undamped sweeps with the scalar
  // diagonal, nearest upsampling, one coarsest sweep, plain outer iteration
  bool literal = false;
  bool use_pairs = true;  // two level-0 sweeps per pass where the level takes them
  FieldSet<V, F> rk2{};
  Bottom bot{};

  // LDS layout of the bottom solver: iterates and right-hand sides of every
  // level first (cleared per launch), then face coefficients, class bytes and
  // the compact indices of the coarsest cells.
  static size_t al16(size_t v) { return (v + 15) & ~(size_t)15; }
  static size_t faces_bytes(const Geom& g) {
    size_t f = (size_t)(g.nx + 1) * g.ny * g.nz + (size_t)g.nx * (g.ny + 1) * g.nz;
    if (g.dim == 3) f += (size_t)g.nx * g.ny * (g.nz + 1);
    return al16(f * sizeof(float));
  }
  static size_t bottom_bytes(const Geom& g) {
    return al16(3 * g.cells() * sizeof(C)) + faces_bytes(g) + al16(g.cells() * sizeof(C)) +
           al16(g.cells());
  }

  void setup_bottom() {
    bottom_top = -1;
    if (!use_bottom || nearest || literal || L < 3) return;
    // (the top level in global memory is held in either storage type; both
    // kernels get the same LDS limit)
    const size_t limit = std::min(bottom_lds_limit<SC, C>(), bottom_lds_limit<S0, C>());
    size_t bytes = al16(COARSE_MAX * sizeof(int));
    int top = L;
    for (int l = L - 1; l >= 1; --l) {
      const size_t need = bytes + bottom_bytes(lv[l].g);
      if (need > limit || L - l > BOTTOM_MAX_LEVELS) break;
      bytes = need;
      top = l;
    }
    if (top > L - 2) return;  // fewer than two levels would fit
    bottom_top = top;
    bot.nlev = L - top;
    bot.nu1 = pre_of(top);  // (every level of the bottom solver is a coarse one)
    bot.nu2 = post_of(top);
    bot.wj = wj;
    size_t off = 0;
    for (int l = top; l < L; ++l) {
      BottomLevel& b = bot.lv[l - top];
      b.g = lv[l].g;
      b.cls = lv[l].cls;
      b.cf0 = lv[l].cf[0];
      b.cf1 = lv[l].cf[1];
      b.cf2 = desc.dim == 3 ? lv[l].cf[2] : lv[l].cf[0];
      b.n = (int)lv[l].g.cells();
      b.bx0 = (int)off;
      b.bx1 = (int)(off + b.n * sizeof(C));
      b.bb = (int)(off + 2 * b.n * sizeof(C));
      off = al16(off + 3 * b.n * sizeof(C));
    }
    bot.zero_bytes = (int)off;
    for (int l = top; l < L; ++l) {
      BottomLevel& b = bot.lv[l - top];
      const Geom& g = lv[l].g;
      b.bfx = (int)off;
      b.bfy = (int)(off + (size_t)(g.nx + 1) * g.ny * g.nz * sizeof(float));
      b.bfz = (int)(b.bfy + (size_t)g.nx * (g.ny + 1) * g.nz * sizeof(float));
      off += faces_bytes(g);
      b.bwd = (int)off;
      off += al16(g.cells() * sizeof(C));
      b.bcl = (int)off;
      b.inx = 1.0f / (float)g.nx;
      b.inxy = 1.0f / ((float)g.nx * (float)g.ny);
      off += al16(g.cells());
    }
    bot.bcidx = (int)off;
    off += al16(COARSE_MAX * sizeof(int));
    bot.cmap = cmap;
    bot.ncount = ncount;
    bot.ainv = work;
    bot.max_n = COARSE_MAX;
    bot.lds_bytes = off;
    if (off - bot.zero_bytes > bot_img_bytes) {
      bot_img_bytes = off - bot.zero_bytes;
      bot_img = alloc<unsigned char>(bot_img_bytes, "bottom LDS image");
    }
    bot.img = bot_img;
    launch_bottom_image<C>(bot, bot_img, stream);
    NFVM_CK(hipGetLastError());
  }
  unsigned char* bot_img = nullptr;
  size_t bot_img_bytes = 0;

  // Level-0 buffer that the CG start / update kernels fill with the first
  // pre-smoothing sweep (from zero) of the next V-cycle, or null when level 0
  // is handled by the bottom solver or the coarsest solve.
  void* zero0() const { return fused_zero(0) ? lv[0].x[0] : nullptr; }
  // Whether level l gets its first pre-smoothing sweep from the kernel that
  // writes its right-hand side (CG start / update for level 0, the
  // restriction from level l - 1 otherwise): levels that run a regular
  // V-cycle step with pre-smoothing.  The CG update reads the V-cycle's
  // result z around every cell while it writes level 0's fused sweep; with
  // nu1 + nu2 odd the sweeps leave z in the buffer that sweep goes to, so
  // level 0 then sweeps from zero itself.
  bool fused_zero(int l) const {
    return pre_of(l) > 0 && l != bottom_top && l < L - 1 && (l > 0 || (nu1 + nu2) % 2 == 0);
  }
  void* zero_of(int l) const { return fused_zero(l) ? lv[l].x[0] : nullptr; }

  void vcycle(int l) {
    Level& v = lv[l];
    if (l == bottom_top) {
      v.cur = 0;
      prof_begin(NFVM_K_BOTTOM, bottom_bytes_moved());
      as_level(l, [&](auto t) { launch_bottom<decltype(t), C>(bot, v.b, v.x[0], red.out, stream); });
      prof_end(NFVM_K_BOTTOM);
      return;
    }
    if (l == L - 1 && literal) {
      smooth(l, true);  // Algorithm 1's coarsest level: one sweep from zero
      return;
    }
    if (l == L - 1) {
      v.cur = 0;
      prof_begin(NFVM_K_BOTTOM, coarse_bytes_moved());
      as_level(l, [&](auto t) {
        launch_coarse_solve<decltype(t), C>(v, cmap, ncount, work, COARSE_MAX, red.out, stream);
      });
      prof_end(NFVM_K_BOTTOM);
      return;
    }
    if (pre_of(l) > 0) {
      if (fused_zero(l)) {
        v.cur = 0;  // first sweep from zero done by the kernel that wrote v.b
      } else {
        smooth(l, true);
      }
      sweeps(l, pre_of(l) - 1, true);
    } else {
      v.cur = 0;
      // (no pre-smoothing: the iterate is zeroed, one store per cell)
      if (l == 0) {
        prof_begin(NFVM_K_SMOOTH0_ZERO, (double)v.g.cells() * sizeof(S0));
        launch_fill_zero<S0>(v, v.x[0], red.out, stream);
        prof_end(NFVM_K_SMOOTH0_ZERO);
      } else {
        prof_begin(NFVM_K_SMOOTH_C, (double)v.g.cells() * elem_size(l));
        as_level(l, [&](auto t) { launch_fill_zero<decltype(t)>(v, v.x[0], red.out, stream); });
        prof_end(NFVM_K_SMOOTH_C);
      }
    }
    if (l == 0) {
      prof_begin(NFVM_K_RESTRICT0);
      restrict_as(0);
      prof_end(NFVM_K_RESTRICT0);
    } else {
      prof_begin(NFVM_K_RESTRICT_C, restrict_bytes(l, zero_of(l + 1) != nullptr));
      restrict_as(l);
      prof_end(NFVM_K_RESTRICT_C);
    }
    vcycle(l + 1);
    if (l == 0) {
      prof_begin(NFVM_K_PROLONG0);
      prolong_as(0);
      prof_end(NFVM_K_PROLONG0);
    } else {
      prof_begin(NFVM_K_PROLONG_C, prolong_bytes(l));
      prolong_as(l);
      prof_end(NFVM_K_PROLONG_C);
    }
    sweeps(l, post_of(l), false);
  }

  // Two-sweep passes on level 0 in this V-cycle: before and after the coarse
  // correction.  Each pass flips the level's iterate buffer once where two
  // sweeps flip it twice, and with a fused first sweep the cycle's result must
  // end in the buffer that sweep does not write (an odd number of flips, as
  // with nu1 + nu2 even and single sweeps): pairs are dropped, the pre-
  // smoothing's last, until the number of pairs is even.
  void sweep_pairs(int& pre, int& post) const {
    pre = post = 0;
    if (!use_pairs || literal || !sweep_pair(lv[0]) || L < 2) return;
    const int m1 = pre_of(0) > 0 ? pre_of(0) - 1 : 0;  // (the first sweep is apart)
    pre = m1 / 2;
    post = post_of(0) / 2;
    if (fused_zero(0) && (pre + post) % 2 == 1) {
      if (pre > 0)
        --pre;
      else
        --post;
    }
  }
  // n sweeps on level l after its first (pre: before the coarse correction)
  void sweeps(int l, int n, bool pre) {
    if (l == 0) {
      int pp, pq;
      sweep_pairs(pp, pq);
      for (int k = pre ? pp : pq; k > 0 && n >= 2; --k, n -= 2) {
        Level& v = lv[0];
        prof_begin(NFVM_K_SMOOTH0_PAIR);
        launch_smooth2<S0, C>(v, v.x[v.cur], v.x[v.cur ^ 1], wj, red.out, stream);
        prof_end(NFVM_K_SMOOTH0_PAIR);
        v.cur ^= 1;
      }
    }
    for (; n > 0; --n) smooth(l, false);
  }

  // One preconditioned flexible-CG iteration (all kernels are no-ops once
  // the device-side stopping rule has fired).
  void fcg_iteration() {
    if (literal) {
      // Algorithm 1's outer loop: the cycle's correction added, the residual
      // formed again
      vcycle(0);
      prof_begin(NFVM_K_FCG_UPDATE, (double)ncells * (2 * sizeof(O) + sizeof(S0) + 2));
      launch_plain_update<O, S0>(lv[0], phi, bvec, red, stream);
      prof_end(NFVM_K_FCG_UPDATE);
      return;
    }
    vcycle(0);
    prof_begin(NFVM_K_FCG_APPLY);
    launch_fcg_apply<O, S0>(lv[0], r, dir, red, stream);
    prof_end(NFVM_K_FCG_APPLY);
    prof_begin(NFVM_K_FCG_UPDATE);
    launch_fcg_update<O, S0>(lv[0], phi, r, dir, red, stream, true, zero0(), wj);
    prof_end(NFVM_K_FCG_UPDATE);
  }

  int predicted = 8;  // iterations of the last solve: enqueued before the first check

  // ---- graphs: one CG iteration, and the step prefix / suffix for both field
  // parities (the ping-pong buffers alternate every step) ----
  struct PartGraph {
    hipGraphExec_t exec = nullptr;
    int post[6];
  };
  hipGraphExec_t g_iter = nullptr;
  // keyed by the buffer state (one bit per field) at the start of the part
  PartGraph g_pre[64], g_suf[64];

  template <class Fn>
  hipGraphExec_t capture(Fn&& fn) {
    hipGraph_t gr = nullptr;
    NFVM_CK(hipStreamSynchronize(stream));  // capture starts on an idle stream
    NFVM_CK(hipStreamBeginCapture(stream, hipStreamCaptureModeThreadLocal));
    try {
      fn();
    } catch (...) {
      // leave the stream out of capture mode before the error goes up
      (void)hipStreamEndCapture(stream, &gr);
      if (gr) (void)hipGraphDestroy(gr);
      throw;
    }
    NFVM_CK(hipStreamEndCapture(stream, &gr));
    hipGraphExec_t ex = nullptr;
    NFVM_CK(hipGraphInstantiate(&ex, gr, nullptr, nullptr, 0));
    NFVM_CK(hipGraphDestroy(gr));
    return ex;
  }

  void drop_graphs() {
    if (g_iter) (void)hipGraphExecDestroy(g_iter);
    g_iter = nullptr;
    for (int i = 0; i < 64; ++i) {
      if (g_pre[i].exec) (void)hipGraphExecDestroy(g_pre[i].exec);
      if (g_suf[i].exec) (void)hipGraphExecDestroy(g_suf[i].exec);
      g_pre[i].exec = g_suf[i].exec = nullptr;
    }
  }

  bool graphs_on() const { return use_graphs && prof_mask == 0; }

  void run_iteration() {
    if (!graphs_on()) {
      fcg_iteration();
      return;
    }
    if (!g_iter) g_iter = capture([&] { fcg_iteration(); });
    NFVM_CK(hipGraphLaunch(g_iter, stream));
  }

  // Flexible CG preconditioned by one V-cycle; b in bvec, result in phi.
  nfvm_status solve(bool have_x0, double tol_, int maxc, int forced, int* cycles, double* rel,
                    bool started = false) {
    if (!started) {
      prof_begin(NFVM_K_FCG_START, start_bytes(have_x0));
      launch_fcg_start<O, S0>(lv[0], bvec, x0, r, phi, red, have_x0, tol_, maxc, forced, stream,
                              true, zero0(), wj);
      prof_end(NFVM_K_FCG_START);
    }
    int ahead = forced >= 0 ? forced : std::min(predicted, maxc);
    for (int i = 0; i < ahead; ++i) run_iteration();
    NFVM_CK(hipGetLastError());
    const int limit = std::max(maxc, forced) + 2;  // the device stops at max_cycles
    for (int enq = ahead;; ++enq) {
      // the finalising kernels mirror the stopping state into hs
      NFVM_CK(hipStreamSynchronize(stream));
      prof_collect();
      if (hs[S_DONE] != 0.0) break;
      if (enq >= limit) throw Error{NFVM_E_DEVICE, "stopping state of the solve not observed"};
      run_iteration();
      NFVM_CK(hipGetLastError());
    }
    return solve_result(forced, tol_, cycles, rel);
  }

  // Post-mortem of a solve that ended with a non-finite residual: the
  // solver's scalars and every device array that holds a non-finite value
  // (count and first padded index), read back to the host.
  std::string diagnose() {
    static const char* SN[S_COUNT] = {"bb", "rr", "zr", "zq", "pq", "zw", "alpha", "div",
                                      "mink", "minw", "done", "iter", "tol2", "maxit",
                                      "forced", "beta", "aprev"};
    std::string m = "scalars:";
    double sc[S_COUNT];
    NFVM_CK(hipMemcpyAsync(sc, red.out, sizeof sc, hipMemcpyDeviceToHost, stream));
    NFVM_CK(hipStreamSynchronize(stream));
    char buf[96];
    for (int i = 0; i < S_COUNT; ++i) {
      snprintf(buf, sizeof buf, " %s=%.6g", SN[i], sc[i]);
      m += buf;
    }
    std::string bad;
    std::vector<unsigned char> h;
    auto scan = [&](const std::string& name, const void* p, size_t n, int es) {
      if (!p || !n) return;
      h.resize(n * es);
      NFVM_CK(hipMemcpyAsync(h.data(), p, n * es, hipMemcpyDeviceToHost, stream));
      NFVM_CK(hipStreamSynchronize(stream));
      size_t cnt = 0, first = 0;
      for (size_t i = 0; i < n; ++i) {
        bool fin;
        if (es == 8) {
          double v;
          memcpy(&v, &h[i * 8], 8);
          fin = isfinite(v);
        } else if (es == 4) {
          float v;
          memcpy(&v, &h[i * 4], 4);
          fin = isfinite(v);
        } else {
          uint16_t v;
          memcpy(&v, &h[i * 2], 2);
          fin = (v & 0x7F80u) != 0x7F80u;  // bf16: exponent all ones is inf or NaN
        }
        if (!fin && cnt++ == 0) first = i;
      }
      if (cnt) {
        snprintf(buf, sizeof buf, " %s[%zu non-finite, first at %zu]", name.c_str(), cnt, first);
        bad += buf;
      }
    };
    const size_t T = (size_t)g.total;
    scan("b", bvec, T, sizeof(O));
    scan("phi", phi, T, sizeof(O));
    scan("r", r, T, sizeof(O));
    scan("p (even)", dir[0], T, sizeof(S0));
    scan("p (odd)", dir[1], T, sizeof(S0));
    for (int l = 0; l < L; ++l) {
      const int es = (int)elem_size(l);
      const size_t n = (size_t)lv[l].g.total;
      scan("L" + std::to_string(l) + ".x0", lv[l].x[0], n, es);
      scan("L" + std::to_string(l) + ".x1", lv[l].x[1], n, es);
      scan("L" + std::to_string(l) + ".b", lv[l].b, n, es);
    }
    scan("pressure", p, T, sizeof(P));
    for (int f = 0; f < 3; ++f) scan("vel" + std::to_string(f), vcur(f), T, sizeof(V));
    for (int f = 3; f < 6; ++f) scan("scalar" + std::to_string(f), scur(f), T, sizeof(F));
    scan("nut", nut, T, sizeof(F));
    const std::string gb = check_guards();
    if (!gb.empty()) m += " out-of-bounds store past: " + gb + ";";
    return m + (bad.empty() ? " arrays: all finite" : " non-finite arrays:" + bad);
  }

  // Outcome of a finished solve from the mirrored scalars.
  nfvm_status solve_result(int forced, double tol_, int* cycles, double* rel) {
    const int it = (int)hs[S_ITER];
    const double bn = sqrt(hs[S_BB]), rn = sqrt(hs[S_RR]);
    *rel = bn > 0 ? rn / bn : 0.0;
    *cycles = it;
    if (forced < 0) predicted = std::max(1, it);
    if (!isfinite(rn) || !isfinite(bn)) return NFVM_E_DIVERGED;
    if (forced < 0 && bn > 0 && rn > tol_ * bn) return NFVM_E_NOTCONV;
    return NFVM_OK;
  }

  void mg_solve(const double* b_dev, double* x_dev, double tol_, int maxc, int forced,
                nfvm_step_stats* stt, nfvm_status* status) override {
    NFVM_CK(hipEventRecord(ev0, stream));
    launch_pack<O>(g, b_dev, bvec, 0.0, stream);
    launch_pack<O>(g, x_dev, x0, 0.0, stream);
    int cyc = 0;
    double rel = 0;
    last_diag.clear();
    nfvm_status st = solve(true, tol_, maxc, forced, &cyc, &rel);
    if (st == NFVM_E_DIVERGED) last_diag = diagnose();
    flush_x();
    launch_unpack<O>(g, phi, x_dev, 0.0, stream);
    NFVM_CK(hipEventRecord(ev1, stream));
    NFVM_CK(hipStreamSynchronize(stream));
    prof_collect();
    // b = 0: the solution is 0 whatever the initial guess
    if (hs[S_BB] == 0.0)
      NFVM_CK(hipMemsetAsync(x_dev, 0, (size_t)ncells * sizeof(double), stream));
    clear_increment();
    NFVM_CK(hipStreamSynchronize(stream));
    float ms = 0;
    NFVM_CK(hipEventElapsedTime(&ms, ev0, ev1));
    if (stt) {
      memset(stt, 0, sizeof *stt);
      stt->cycles = cyc;
      stt->status = st;
      stt->rel_residual = rel;
      stt->seconds = ms * 1e-3;
      stt->min_k = stt->min_omega = NAN;
    }
    *status = st;
  }

  void pressure_adjoint(const double* ub, const double* vb, const double* wb, const double* pb,
                        double* usb, double* vsb, double* wsb, double tol_, int maxc, int forced,
                        nfvm_step_stats* stt, nfvm_status* status) override {
    NFVM_CK(hipEventRecord(ev0, stream));
    // lambda = A^-1 (pbar - dt G^T ubar), then usbar = ubar + (dB/du*)^T lambda
    launch_adj_phibar<O>(g, ph, type, patches, ub, vb, wb, pb, bvec, stream);
    NFVM_CK(hipGetLastError());
    int cyc = 0;
    double rel = 0;
    last_diag.clear();
    nfvm_status st = solve(false, tol_, maxc, forced, &cyc, &rel);
    if (st == NFVM_E_DIVERGED) last_diag = diagnose();
    flush_x();
    launch_adj_velocity<O>(g, ph, type, patches, phi, ub, vb, wb, usb, vsb, wsb, stream);
    NFVM_CK(hipGetLastError());
    NFVM_CK(hipEventRecord(ev1, stream));
    NFVM_CK(hipStreamSynchronize(stream));
    prof_collect();
    clear_increment();  // (phi held lambda; it is not the step's increment)
    NFVM_CK(hipStreamSynchronize(stream));
    float ms = 0;
    NFVM_CK(hipEventElapsedTime(&ms, ev0, ev1));
    if (stt) {
      memset(stt, 0, sizeof *stt);
      stt->cycles = cyc;
      stt->status = st;
      stt->rel_residual = rel;
      stt->seconds = ms * 1e-3;
      stt->min_k = stt->min_omega = NAN;
    }
    *status = st;
  }

  void mg_solve_scratch(const double* b_dev, double* x_dev, double tol_, int maxc, int forced,
                        nfvm_step_stats* stt, nfvm_status* status, double* scratch,
                        size_t n_doubles) override {
    // scalars first (32 doubles keep the partials 256-byte aligned)
    const size_t head = 32;
    const size_t cap = n_doubles > head ? (n_doubles - head) / RED_MAX_NV : 0;
    const int need = fcg_max_blocks(lv[0]);
    if ((size_t)need > cap)
      throw Error{NFVM_E_INVAL, "the solve's reductions need " + std::to_string(need) +
                                    " workgroups of partials; the scratch holds " +
                                    std::to_string(cap)};
    RedBuf s = red;
    s.out = scratch;
    s.partial = scratch + head;
    s.max_blocks = (int)std::min<size_t>(cap, 1u << 30);
    launch_fill_f64(s.out, (int)head, 0.0, stream);
    NFVM_CK(hipGetLastError());
    const RedBuf own = red;
    const bool graphs = use_graphs;
    red = s;
    use_graphs = false;  // the captured iteration refers to the grid's own buffers
    try {
      mg_solve(b_dev, x_dev, tol_, maxc, forced, stt, status);
    } catch (...) {
      red = own;
      use_graphs = graphs;
      throw;
    }
    red = own;
    use_graphs = graphs;
  }

  void swap(int f) { fcur[f] ^= 1; }

  // destruction over dt/2, explicit step, Poisson right-hand side, CG start
  void step_prefix() {
    const double half = 0.5 * ph.dt;
    if (ph.komega) {
      prof_begin(NFVM_K_DESTROY);
      launch_destroy<V, F>(g, ph, type, patches, vcur(0), vcur(1), vcur(2), scur(4), scur(5),
                           half, salt(4), salt(5), nut, nullptr, tp[TP_DESTROY], stream);
      prof_end(NFVM_K_DESTROY);
      swap(4);
      swap(5);
    }
    FieldSet<V, F> in{vcur(0), vcur(1), vcur(2), scur(3), scur(4), scur(5)};
    FieldSet<V, F> out{valt(0), valt(1), valt(2), salt(3), salt(4), salt(5)};
    prof_begin(NFVM_K_EXPLICIT);
    launch_explicit<V, F, P>(g, ph, type, patches, in, p, nut, out, tp[TP_EXPLICIT], stream);
    if (rk_order == 2) {
      // Heun: a second Euler step from the first stage, averaged with the start
      if (ph.komega) launch_nut<V, F>(g, ph, type, out.k, out.om, nut, stream);
      launch_explicit<V, F, P>(g, ph, type, patches, out, p, nut, rk2, tp[TP_EXPLICIT], stream);
      launch_rk2_average<V, F>(g, in, rk2, out, stream);
    }
    prof_end(NFVM_K_EXPLICIT);
    for (int f = 0; f < 6; ++f) swap(f);
    prof_begin(NFVM_K_RHS);
    launch_rhs_b<V, O>(g, ph, type, patches, vcur(0), vcur(1), vcur(2), bvec, red,
                       tp[TP_RHS], stream);
    prof_end(NFVM_K_RHS);
    // initial guess: the previous step's increment (warm start), else zero
    prof_begin(NFVM_K_FCG_START, start_bytes(use_warm));
    launch_fcg_start<O, S0>(lv[0], bvec, use_warm ? phi : x0, r, phi, red, use_warm, tol,
                            max_cycles, -1, stream, true, zero0(), wj);
    prof_end(NFVM_K_FCG_START);
  }

  // the CG x update the solve's last iteration deferred (none in Algorithm
  // 1's plain iteration, which updates x every time)
  void flush_x() {
    if (!literal) launch_fcg_flush<O, S0>(lv[0], phi, dir, red.out, stream);
  }

  // projection, destruction over dt/2 (with the min k / omega reduction)
  void step_suffix() {
    const double half = 0.5 * ph.dt;
    flush_x();
    prof_begin(NFVM_K_PROJECT);
    launch_project<V, P, O>(g, ph, type, patches, phi, vcur(0), vcur(1), vcur(2), valt(0),
                            valt(1), valt(2), p, red, tp[TP_PROJECT], stream);
    prof_end(NFVM_K_PROJECT);
    swap(0);
    swap(1);
    swap(2);
    if (ph.komega) {
      prof_begin(NFVM_K_DESTROY);
      launch_destroy<V, F>(g, ph, type, patches, vcur(0), vcur(1), vcur(2), scur(4), scur(5),
                           half, salt(4), salt(5), nullptr, &red, tp[TP_DESTROY], stream);
      prof_end(NFVM_K_DESTROY);
      swap(4);
      swap(5);
    }
  }

  template <class Fn>
  void run_part(PartGraph* cache, Fn&& fn) {
    if (!graphs_on()) {
      fn();
      return;
    }
    int key = 0;
    for (int f = 0; f < 6; ++f) key |= fcur[f] << f;
    PartGraph& pg = cache[key];
    if (!pg.exec) {
      pg.exec = capture(fn);
      for (int f = 0; f < 6; ++f) pg.post[f] = fcur[f];
    } else {
      for (int f = 0; f < 6; ++f) fcur[f] = pg.post[f];
    }
    NFVM_CK(hipGraphLaunch(pg.exec, stream));
  }

  // ---- time steps (the GridBase state machine) ----
  // Steps run back to back with one host synchronisation each (the solve's
  // convergence check); the statistics of a step (face divergence, min k,
  // min omega, run time) are read at the next synchronisation, when the
  // mirror still holds them, and after the last step.
  struct Run {
    int n = 0, s = 0;  // steps asked / started
    nfvm_step_stats* stt = nullptr;
    nfvm_status worst = NFVM_OK, final_st = NFVM_OK;
    bool solving = false;
    int enq = 0;        // iterations enqueued for the running solve
    int converged = 0;  // steps whose solve met tol
    int pend = -1, pend_cyc = 0;  // step whose statistics are read at the next synchronisation
    double pend_rel = 0;
    nfvm_status pend_st = NFVM_OK;
  } run;

  void run_start_step() {
    NFVM_CK(hipEventRecord(ev_step[run.s & 1][0], stream));
    run_part(g_pre, [&] { step_prefix(); });
    NFVM_CK(hipGetLastError());
    run.solving = true;
    run.enq = 0;
  }

  void run_begin(int n, nfvm_step_stats* stt) override {
    run = Run{};
    last_diag.clear();
    run.n = n;
    run.stt = stt;
    if (n > 0) run_start_step();
  }

  int run_ahead() const override {
    if (!run.solving) return -1;
    return std::max(0, std::min(predicted, max_cycles) - run.enq);
  }

  void run_enqueued(int k) override { run.enq += k; }

  nfvm_status run_status() const override { return run.final_st; }
  int run_converged() const override { return run.converged; }

  // the previous step's statistics; false if it diverged
  bool run_collect() {
    if (run.pend < 0) return true;
    nfvm_status st = run.pend_st;
    if (!isfinite(hs[S_DIV])) st = NFVM_E_DIVERGED;
    if (run.stt) {
      float ms = 0;
      NFVM_CK(hipEventElapsedTime(&ms, ev_step[run.pend & 1][0], ev_step[run.pend & 1][1]));
      nfvm_step_stats& o = run.stt[run.pend];
      o.cycles = run.pend_cyc;
      o.status = st;
      o.rel_residual = run.pend_rel;
      o.max_face_div = hs[S_DIV];
      o.min_k = ph.komega ? hs[S_MINK] : NAN;
      o.min_omega = ph.komega ? hs[S_MINW] : NAN;
      o.seconds = ms * 1e-3;
    }
    run.pend = -1;
    if (st == NFVM_E_DIVERGED) return false;
    if (st != NFVM_OK && run.worst == NFVM_OK) run.worst = st;
    return true;
  }

  bool run_after_sync() override {
    prof_collect();
    if (!run_collect()) {
      run.final_st = NFVM_E_DIVERGED;
      run.solving = false;
      return true;
    }
    if (run.solving) {
      if (hs[S_DONE] == 0.0) {
        // the device stops at max_cycles
        if (run.enq >= max_cycles + 2)
          throw Error{NFVM_E_DEVICE, "stopping state of the solve not observed"};
        return false;
      }
      run.solving = false;
      int cyc = 0;
      double rel = 0;
      const nfvm_status st = solve_result(-1, tol, &cyc, &rel);
      if (st == NFVM_E_DIVERGED) {
        last_diag = "step " + std::to_string(run.s) + ": " + diagnose();
        if (run.stt) {
          memset(&run.stt[run.s], 0, sizeof run.stt[run.s]);
          run.stt[run.s].status = st;
          run.stt[run.s].cycles = cyc;
          run.stt[run.s].rel_residual = rel;
        }
        run.final_st = st;
        return true;
      }
      if (st == NFVM_OK) ++run.converged;
      run_part(g_suf, [&] { step_suffix(); });
      NFVM_CK(hipGetLastError());
      NFVM_CK(hipEventRecord(ev_step[run.s & 1][1], stream));
      run.pend = run.s;
      run.pend_cyc = cyc;
      run.pend_rel = rel;
      run.pend_st = st;
      if (++run.s < run.n) run_start_step();
      return false;
    }
    if (run.s >= run.n) {  // the last step's statistics are read above
      run.final_st = run.worst;
      return true;
    }
    return false;
  }

  void step(int n, nfvm_step_stats* stt, nfvm_status* status) override {
    run_begin(n, stt);
    for (;;) {
      const int ahead = run_ahead();
      if (ahead >= 0) {
        const int k = std::max(1, ahead);
        for (int i = 0; i < k; ++i) run_iteration();
        run_enqueued(k);
        NFVM_CK(hipGetLastError());
      }
      NFVM_CK(hipStreamSynchronize(stream));
      if (run_after_sync()) break;
    }
    *status = run_status();
  }

  // ---- batched iterations ----
  // grids batch together when they share precision and prolongation
  int type_id() const override { return desc.precision + (nearest ? 16 : 0) + (literal ? 32 : 0); }

  void mg_desc(MgGridDesc& d) {
    memset(&d, 0, sizeof d);
    d.lv = lv.data();
    d.L = L;
    d.bottom_top = bottom_top;
    d.nu1 = nu1;
    d.nu2 = nu2;
    d.nu1c = pre_of(1);
    d.nu2c = post_of(1);
    d.wj = wj;
    d.bot = &bot;
    d.cmap = cmap;
    d.ncount = ncount;
    d.ainv = work;
    d.coarse_max = COARSE_MAX;
    for (int l = 0; l < L; ++l) d.zero[l] = zero_of(l);
    d.red = red;
    d.x = phi;
    d.r = r;
    d.dir[0] = dir[0];
    d.dir[1] = dir[1];
  }

  std::unique_ptr<IterPlan> make_plan(const std::vector<GridBase*>& same) override {
    if (literal)
      throw Error{NFVM_E_INVAL, "grids in Algorithm 1's literal mode are stepped alone, not batched"};
    std::vector<MgGridDesc> ds(same.size());
    for (size_t i = 0; i < same.size(); ++i) {
      if (same[i]->type_id() != type_id() || same[i]->stream != stream)
        throw Error{NFVM_E_INVAL, "batched grids must share precision and stream"};
      static_cast<GridT*>(same[i])->mg_desc(ds[i]);
    }
    std::unique_ptr<IterPlan> pl(new IterPlan());
    plan_fcg_iteration<O, S0, SC, C>(ds.data(), (int)ds.size(), pl->ops);
    pl->blob.alloc(pl->ops.blob.size(), stream);
    NFVM_CK(hipMemcpyAsync(pl->blob.p, pl->ops.blob.data(), pl->ops.blob.size(),
                           hipMemcpyHostToDevice, stream));
    bool graphs = true;
    for (GridBase* g : same) graphs = graphs && g->use_graphs && g->prof_mask == 0;
    if (graphs) pl->exec = capture([&] {
      for (auto& op : pl->ops.ops) op((const unsigned char*)pl->blob.p, stream);
    });
    NFVM_CK(hipStreamSynchronize(stream));
    return pl;
  }

  void set_option(int opt, double v) override {
    if (opt == NFVM_OPT_GRAPHS) {
      NFVM_CK(hipStreamSynchronize(stream));
      drop_graphs();
      use_graphs = v != 0.0;
    } else if (opt == NFVM_OPT_PREDICT) {
      predicted = std::max(1, (int)v);
    } else if (opt == NFVM_OPT_AUTOTUNE) {
      use_autotune = v != 0.0;
      if (!use_autotune) {
        for (auto& lvl : lv)
          for (int t = 0; t < TK_LEVEL_COUNT; ++t) lvl.tt[t] = TILE_DEFAULT;
        for (int t = 0; t < TP_COUNT; ++t) tp[t] = TILE_DEFAULT;
      } else {
        autotune();
        clear_increment();
      }
      NFVM_CK(hipStreamSynchronize(stream));
      drop_graphs();
    } else if (opt == NFVM_OPT_WARM_START) {
      NFVM_CK(hipStreamSynchronize(stream));
      drop_graphs();
      use_warm = v != 0.0;
    } else if (opt == NFVM_OPT_BOTTOM) {
      NFVM_CK(hipStreamSynchronize(stream));
      drop_graphs();
      use_bottom = v != 0.0;
      setup_bottom();
    } else if (opt == NFVM_OPT_RK_ORDER) {
      if (v != 1.0 && v != 2.0) throw Error{NFVM_E_INVAL, "Runge-Kutta order must be 1 or 2"};
      NFVM_CK(hipStreamSynchronize(stream));
      drop_graphs();
      if (v == 2.0 && !rk2.om) {  // allocated last: a failed set is made again
        rk2.u = alloc<V>(g.total);
        rk2.v = alloc<V>(g.total);
        rk2.w = alloc<V>(g.total);
        rk2.T = alloc<F>(g.total);
        rk2.k = alloc<F>(g.total);
        rk2.om = alloc<F>(g.total);
        NFVM_CK(hipStreamSynchronize(stream));
      }
      rk_order = (int)v;
    } else if (opt == NFVM_OPT_SWEEP_PAIRS) {
      if (v != 0.0 && v != 1.0) throw Error{NFVM_E_INVAL, "sweep pairs must be 0 or 1"};
      NFVM_CK(hipStreamSynchronize(stream));
      drop_graphs();
      use_pairs = v != 0.0;
    } else if (opt == NFVM_OPT_LITERAL) {
      if (v != 0.0 && v != 1.0) throw Error{NFVM_E_INVAL, "literal mode must be 0 or 1"};
      NFVM_CK(hipStreamSynchronize(stream));
      drop_graphs();
      literal = v != 0.0;
      if (literal) {
        nu1 = 0;
        nu2 = 1;
        nuc = 0;
        wj = 1.0;
      } else {
        nu1 = desc.nu1;
        nu2 = desc.nu2;
        nuc = desc.nu_coarse;
        wj = desc.omega_jacobi > 0 ? desc.omega_jacobi : (desc.dim == 3 ? 6.0 / 7.0 : 4.0 / 5.0);
      }
      for (int l = 0; l < L; ++l) {
        Geom& gl = lv[l].g;
        gl.sd = literal ? 2.0 / (gl.hx * gl.hx) + 2.0 / (gl.hy * gl.hy) +
                              (desc.dim == 3 ? 2.0 / (gl.hz * gl.hz) : 0.0)
                        : 0.0;
        if (l + 1 < L) lv[l].nearest = nearest || literal;
      }
      setup_bottom();
    } else if (opt == NFVM_OPT_PROLONG) {
      if (v != 0.0 && v != 1.0)
        throw Error{NFVM_E_INVAL, "prolongation must be 0 (linear) or 1 (nearest)"};
      NFVM_CK(hipStreamSynchronize(stream));
      drop_graphs();
      nearest = v != 0.0;
      for (int l = 0; l + 1 < L; ++l) lv[l].nearest = nearest || literal;
      setup_bottom();
    } else {
      throw Error{NFVM_E_INVAL, "unknown option"};
    }
  }
};

// <velocity, scalars, pressure, outer solve, level-0 storage, coarse storage, V-cycle arithmetic>
typedef GridT<double, double, double, double, double, double, double> GridFP64;
typedef GridT<float, float, float, float, float, float, float> GridFP32;
typedef GridT<double, float, double, double, float, bf16, float> GridMixed;

std::unique_ptr<GridBase> make_grid(const nfvm_grid_desc& d, const nfvm_fields* init,
                                    hipStream_t stream, int tune_mode) {
  validate_desc(d);
  std::unique_ptr<GridBase> gb;
  if (d.precision == NFVM_FP64)
    gb.reset(new GridFP64());
  else if (d.precision == NFVM_FP32)
    gb.reset(new GridFP32());
  else
    gb.reset(new GridMixed());
  gb->use_autotune = tune_mode != 0;
  if (tune_mode == 2) {
    if (d.precision == NFVM_FP64)
      static_cast<GridFP64*>(gb.get())->tune_cached_only = true;
    else if (d.precision == NFVM_FP32)
      static_cast<GridFP32*>(gb.get())->tune_cached_only = true;
    else
      static_cast<GridMixed*>(gb.get())->tune_cached_only = true;
  }
  if (stream) {
    gb->stream = stream;
  } else {
    NFVM_CK(hipStreamCreateWithFlags(&gb->stream, hipStreamNonBlocking));
    gb->own_stream = true;
  }
  if (d.precision == NFVM_FP64)
    static_cast<GridFP64*>(gb.get())->init(d, init);
  else if (d.precision == NFVM_FP32)
    static_cast<GridFP32*>(gb.get())->init(d, init);
  else
    static_cast<GridMixed*>(gb.get())->init(d, init);
  return gb;
}

IterPlan::~IterPlan() {
  if (exec) (void)hipGraphExecDestroy(exec);
}

void IterPlan::launch(hipStream_t s) {
  if (exec) {
    NFVM_CK(hipGraphLaunch(exec, s));
    return;
  }
  for (auto& op : ops.ops) op((const unsigned char*)blob.p, s);
}

void BatchRunner::add(GridBase* g, int n_steps, nfvm_step_stats* stt) {
  if (g->stream != stream) throw Error{NFVM_E_INVAL, "grid is not on the runner's stream"};
  for (GridBase* o : gs)
    if (o == g) throw Error{NFVM_E_INVAL, "grid added twice"};
  g->run_begin(n_steps, stt);
  gs.push_back(g);
  dirty = true;
}

std::vector<GridBase*> BatchRunner::advance() {
  std::vector<GridBase*> over;
  if (gs.empty()) return over;
  if (dirty) {
    plans.clear();
    std::vector<int> types;
    for (GridBase* g : gs)
      if (std::find(types.begin(), types.end(), g->type_id()) == types.end())
        types.push_back(g->type_id());
    for (int t : types) {
      std::vector<GridBase*> same;
      for (GridBase* g : gs)
        if (g->type_id() == t) same.push_back(g);
      plans.push_back(same[0]->make_plan(same));
    }
    dirty = false;
  }
  // as many iterations as the grid closest to its stopping rule is
  // predicted to need (grids already stopped skip them on the device)
  int k = -1;
  for (GridBase* g : gs) {
    const int a = g->run_ahead();
    if (a >= 0) k = k < 0 ? a : std::min(k, a);
  }
  if (k >= 0) {
    k = std::max(1, k);
    for (int i = 0; i < k; ++i)
      for (auto& pl : plans) pl->launch(stream);
    for (GridBase* g : gs)
      if (g->run_ahead() >= 0) g->run_enqueued(k);
    NFVM_CK(hipGetLastError());
  }
  NFVM_CK(hipStreamSynchronize(stream));
  std::vector<GridBase*> keep;
  for (GridBase* g : gs) (g->run_after_sync() ? over : keep).push_back(g);
  if (!over.empty()) {
    gs.swap(keep);
    dirty = true;
  }
  return over;
}

}  // namespace nfvm
