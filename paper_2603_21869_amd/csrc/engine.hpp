// Host engine: one grid on the device and the orchestration of a time step.
#pragma once

#include <hip/hip_runtime.h>

#include <memory>
#include <string>
#include <tuple>
#include <vector>

#include "../../include/nfvm.h"
#include "nfvm_internal.hpp"

namespace nfvm {

// thrown inside the library only; converted to nfvm_status at the C ABI
struct Error {
  nfvm_status st;
  std::string msg;
};

void set_error(const std::string& m);
void* dev_alloc(size_t bytes);
void dev_free(void* p);

#define NFVM_CK(call)                                                                     \
  do {                                                                                    \
    hipError_t e_ = (call);                                                               \
    if (e_ != hipSuccess)                                                                 \
      throw ::nfvm::Error{NFVM_E_DEVICE, std::string(#call) + ": " + hipGetErrorString(e_)}; \
  } while (0)

// Owned device buffer.
struct DevBuf {
  void* p = nullptr;
  size_t bytes = 0;
  DevBuf() = default;
  DevBuf(const DevBuf&) = delete;
  DevBuf& operator=(const DevBuf&) = delete;
  ~DevBuf() { release(); }
  void release() {
    if (p) dev_free(p);
    p = nullptr;
    bytes = 0;
  }
  void alloc(size_t n, hipStream_t s) {
    release();
    bytes = n;
    p = dev_alloc(n ? n : 16);
    if (!p) throw Error{NFVM_E_NOMEM, "device allocation of " + std::to_string(n) + " bytes failed"};
    NFVM_CK(hipMemsetAsync(p, 0, n ? n : 16, s));
  }
  template <class T>
  T* as() const {
    return (T*)p;
  }
};

size_t footprint_bytes(const nfvm_grid_desc& d);
// Largest block count of a reducing level-0 launch over every tile target
// the autotuner may pick, and the block capacity of the grid's partials.
void reduction_blocks(const nfvm_grid_desc& d, int* needed, int* capacity);

// autotuner results, per kernel, level shape, dimension and precision
struct TuneKey {
  int kid, nx, ny, nz, dim, prec;
  bool operator<(const TuneKey& o) const {
    return std::tie(kid, nx, ny, nz, dim, prec) < std::tie(o.kid, o.nx, o.ny, o.nz, o.dim, o.prec);
  }
};
bool tune_lookup(const TuneKey& k, int* v);
// The cached choice of the same kernel, dimension and precision at the shape
// nearest in cell count (false: none cached yet).
bool tune_lookup_near(const TuneKey& k, int* v);
void tune_store(const TuneKey& k, int v);
std::vector<std::pair<TuneKey, int>> tune_entries();
void validate_desc(const nfvm_grid_desc& d);

// One CG iteration of several grids of one precision: the batched launches
// of plan_fcg_iteration, their arguments in device memory, replayed as one
// graph when graphs are on.
struct IterPlan {
  DevBuf blob;
  BatchOps ops;
  hipGraphExec_t exec = nullptr;
  IterPlan() = default;
  IterPlan(const IterPlan&) = delete;
  IterPlan& operator=(const IterPlan&) = delete;
  ~IterPlan();
  void launch(hipStream_t s);
};

class GridBase {
 public:
  virtual ~GridBase() = default;
  virtual void step(int n, nfvm_step_stats* st, nfvm_status* status) = 0;

  // ---- time steps as a state machine.  step() drives it for one grid; a
  // BatchRunner drives several grids on one stream, enqueuing the CG
  // iterations of all of them as batched launches.
  // Start n steps (enqueues the first step's prefix); stt: NULL or n entries.
  virtual void run_begin(int n, nfvm_step_stats* stt) = 0;
  // -1 while no pressure solve is under way, else the iterations still
  // predicted before its stopping rule fires (0: check after each one).
  virtual int run_ahead() const = 0;
  virtual void run_enqueued(int k) = 0;
  // After a synchronisation of the grid's stream: read what the device
  // mirrored, finish a converged solve (suffix, next prefix); true once all
  // steps are over or one failed.
  virtual bool run_after_sync() = 0;
  virtual nfvm_status run_status() const = 0;
  // time steps whose pressure solve met its tolerance so far
  virtual int run_converged() const = 0;
  // grids of one type_id share batched launches
  virtual int type_id() const = 0;
  virtual std::unique_ptr<IterPlan> make_plan(const std::vector<GridBase*>& same_type) = 0;

  virtual void mg_solve(const double* b_dev, double* x_dev, double tol, int max_cycles, int forced,
                        nfvm_step_stats* st, nfvm_status* status) = 0;
  // Reverse mode of the pressure step: the adjoints of u*, v*, w* (dense
  // device FP64) for those of the step's velocity and pressure.
  virtual void pressure_adjoint(const double* ub, const double* vb, const double* wb,
                                const double* pb, double* usb, double* vsb, double* wsb,
                                double tol, int max_cycles, int forced, nfvm_step_stats* st,
                                nfvm_status* status) = 0;
  // The same solve with its reduction partials and scalars in the n_doubles
  // doubles of device memory at scratch (256-byte aligned) instead of the
  // grid's own, launched without the captured graphs; allocates nothing.
  virtual void mg_solve_scratch(const double* b_dev, double* x_dev, double tol, int max_cycles,
                                int forced, nfvm_step_stats* st, nfvm_status* status,
                                double* scratch, size_t n_doubles) = 0;
  virtual void get_fields(nfvm_fields* out) = 0;
  virtual void lambda2(double* out) = 0;
  virtual void probe(const double* pts, int n, double* out) = 0;
  // device FP64 dense arrays; see nfvm_explicit_adjoint_device
  virtual void explicit_adjoint(const nfvm_fields& st, const nfvm_fields& bar,
                                const nfvm_fields& out) = 0;
  virtual void destroy_adjoint(const nfvm_fields& st, double tau, const double* kb,
                               const double* wb, const nfvm_fields& out) = 0;
  virtual void step_adjoint(const nfvm_fields& st, const nfvm_fields& bar, const nfvm_fields& out,
                            double tol, int maxc, int forced, nfvm_step_stats* stt,
                            nfvm_status* status) = 0;
  virtual void set_fields(const nfvm_fields* in) = 0;
  virtual void set_option(int opt, double v) = 0;
  // buffers whose guard zone an out-of-bounds store has written (empty: none)
  virtual std::string check_guards() = 0;
  bool use_graphs = true;
  bool use_bottom = true;
  bool use_warm = false;
  bool use_autotune = true;
  // kernel timing (nfvm_profile)
  struct ProfRec {
    int kid;
    hipEvent_t a, b;
    double bytes;  // algorithmic bytes of the launch
  };
  uint32_t prof_mask = 0;
  std::vector<hipEvent_t> ev_pool;
  size_t ev_used = 0;
  std::vector<ProfRec> prof_pending;
  long long prof_launches[NFVM_K_COUNT] = {};
  double prof_seconds[NFVM_K_COUNT] = {};
  double prof_bytes[NFVM_K_COUNT] = {};      // per launch, for the level-0 and physics kernels
  double prof_bytes_sum[NFVM_K_COUNT] = {};  // summed over the timed launches
  hipEvent_t next_event();
  // time the next kernel launched (and, with NFVM_K_FINALIZE in the mask,
  // its finaliser) as kernel kid moving `bytes` (< 0: prof_bytes[kid])
  void prof_begin(int kid, double bytes = -1.0);
  void prof_end(int kid);
  void prof_collect();  // after a stream synchronisation
  void prof_reset(uint32_t mask);
  void prof_release();

  // what the last failed solve left on the device (solver scalars, arrays
  // holding non-finite values); empty after a good one
  std::string last_diag;
  hipStream_t stream = nullptr;
  bool own_stream = false;
  long long ncells = 0;
  nfvm_grid_desc desc{};
  double tol = 1e-6;
  int max_cycles = 100;
};

// Several grids advanced together on one stream: per round, the next CG
// iterations of every grid whose pressure solve is under way as batched
// launches (one plan per precision), then one synchronisation, after which
// each grid finishes a converged solve and starts its next step.  Grids may
// join (add) at any round; a grid leaves when advance() returns it.
class BatchRunner {
 public:
  explicit BatchRunner(hipStream_t s) : stream(s) {}
  // g must run on this runner's stream
  void add(GridBase* g, int n_steps, nfvm_step_stats* stt);
  std::vector<GridBase*> advance();
  size_t size() const { return gs.size(); }

 private:
  hipStream_t stream;
  std::vector<GridBase*> gs;
  std::vector<std::unique_ptr<IterPlan>> plans;
  bool dirty = true;
};

// tune_mode: 0 default tiles, 1 autotune (cached per shape), 2 cached choices only
std::unique_ptr<GridBase> make_grid(const nfvm_grid_desc& d, const nfvm_fields* init,
                                    hipStream_t stream, int tune_mode = 1);

}  // namespace nfvm

struct nfvm_grid {
  std::unique_ptr<nfvm::GridBase> g;
};
