// C ABI entry points of libnfvm.so (declared in include/nfvm.h): argument
// checks, conversion of library errors to nfvm_status, thread-local messages.
#include <string.h>

#include <string>
#include <vector>

#include "engine.hpp"

namespace nfvm {
void set_allocator(nfvm_alloc_fn a, nfvm_free_fn f, void* ctx);
static thread_local std::string t_err;
void set_error(const std::string& m) { t_err = m; }
}  // namespace nfvm

using namespace nfvm;

template <class Fn>
static nfvm_status guard(Fn&& fn) {
  try {
    return fn();
  } catch (const Error& e) {
    set_error(e.msg);
    // a failed HIP call leaves its code as this thread's last error: clear
    // it, so that the next call's launch check does not report it again
    (void)hipGetLastError();
    return e.st;
  } catch (const std::bad_alloc&) {
    set_error("host allocation failed");
    return NFVM_E_NOMEM;
  } catch (const std::exception& e) {
    set_error(e.what());
    return NFVM_E_DEVICE;
  }
}

static nfvm_status fail(nfvm_status st, const char* msg) {
  set_error(msg);
  return st;
}

extern "C" {

nfvm_status nfvm_set_allocator(nfvm_alloc_fn alloc, nfvm_free_fn free_fn, void* ctx) {
  if ((alloc == nullptr) != (free_fn == nullptr))
    return fail(NFVM_E_INVAL, "allocator and free function must be given together");
  set_allocator(alloc, free_fn, ctx);
  return NFVM_OK;
}

nfvm_status nfvm_init_grid(const nfvm_grid_desc* desc, const nfvm_fields* init, void* stream,
                           nfvm_grid_t* out) {
  if (!desc || !out) return fail(NFVM_E_INVAL, "desc and out are required");
  *out = nullptr;
  return guard([&] {
    auto g = make_grid(*desc, init, (hipStream_t)stream);
    *out = new nfvm_grid{std::move(g)};
    return NFVM_OK;
  });
}

nfvm_status nfvm_step(nfvm_grid_t grid, int32_t n_steps, nfvm_step_stats* stats) {
  if (!grid || n_steps < 0) return fail(NFVM_E_INVAL, "bad grid or step count");
  return guard([&] {
    nfvm_status st = NFVM_OK;
    grid->g->step(n_steps, stats, &st);
    if (st == NFVM_E_DIVERGED)
      set_error("non-finite residual or field" +
                (grid->g->last_diag.empty() ? std::string() : "; " + grid->g->last_diag));
    if (st == NFVM_E_NOTCONV) set_error("pressure solve reached max_cycles");
    return st;
  });
}

// The grids' own streams wait for the work enqueued before the call; the
// batch runs on the first grid's stream, and the others wait for it after.
struct StreamJoin {
  std::vector<GridBase*> gs;
  std::vector<hipStream_t> own;
  std::vector<hipEvent_t> evs;
  hipStream_t s = nullptr;
  explicit StreamJoin(const std::vector<GridBase*>& g) : gs(g) {
    s = gs[0]->stream;
    for (GridBase* x : gs) {
      own.push_back(x->stream);
      if (x->stream == s) continue;
      hipEvent_t e = nullptr;
      NFVM_CK(hipEventCreateWithFlags(&e, hipEventDisableTiming));
      evs.push_back(e);
      NFVM_CK(hipEventRecord(e, x->stream));
      NFVM_CK(hipStreamWaitEvent(s, e, 0));
      x->stream = s;
    }
  }
  ~StreamJoin() {
    hipEvent_t e = nullptr;
    const bool ok = hipEventCreateWithFlags(&e, hipEventDisableTiming) == hipSuccess &&
                    hipEventRecord(e, s) == hipSuccess;
    for (size_t i = 0; i < gs.size(); ++i) {
      gs[i]->stream = own[i];
      if (own[i] != s && ok) (void)hipStreamWaitEvent(own[i], e, 0);
    }
    if (e) (void)hipEventDestroy(e);
    for (hipEvent_t x : evs) (void)hipEventDestroy(x);
  }
};

nfvm_status nfvm_step_batch(nfvm_grid_t* grids, int32_t n_grids, int32_t n_steps,
                            nfvm_step_stats* stats, nfvm_status* statuses) {
  if (!grids || n_grids < 1 || n_steps < 0)
    return fail(NFVM_E_INVAL, "grids, n_grids >= 1 and n_steps >= 0 are required");
  std::vector<GridBase*> gs;
  for (int i = 0; i < n_grids; ++i) {
    if (!grids[i]) return fail(NFVM_E_INVAL, "grid is NULL");
    for (GridBase* o : gs)
      if (o == grids[i]->g.get()) return fail(NFVM_E_INVAL, "a grid appears twice");
    gs.push_back(grids[i]->g.get());
  }
  return guard([&] {
    StreamJoin join(gs);
    BatchRunner br(join.s);
    for (int i = 0; i < n_grids; ++i)
      br.add(gs[i], n_steps, stats ? stats + (size_t)i * n_steps : nullptr);
    while (br.size()) br.advance();
    nfvm_status first = NFVM_OK;
    for (int i = 0; i < n_grids; ++i) {
      const nfvm_status st = gs[i]->run_status();
      if (statuses) statuses[i] = st;
      if (st != NFVM_OK && first == NFVM_OK) first = st;
    }
    if (first == NFVM_E_DIVERGED) set_error("non-finite residual or field");
    if (first == NFVM_E_NOTCONV) set_error("pressure solve reached max_cycles");
    return first;
  });
}

nfvm_status nfvm_mg_solve_device(nfvm_grid_t grid, const double* b_dev, double* x_dev, double tol,
                                 int32_t max_cycles, int32_t forced_cycles,
                                 nfvm_step_stats* stats) {
  if (!grid || !b_dev || !x_dev) return fail(NFVM_E_INVAL, "grid, b and x are required");
  return guard([&] {
    nfvm_status st = NFVM_OK;
    grid->g->mg_solve(b_dev, x_dev, tol, max_cycles, forced_cycles, stats, &st);
    if (st == NFVM_E_NOTCONV) set_error("pressure solve reached max_cycles");
    if (st == NFVM_E_DIVERGED) set_error("non-finite residual");
    return st;
  });
}

nfvm_status nfvm_mg_solve_adjoint_device(nfvm_grid_t grid, const double* xbar_dev,
                                         double* bbar_dev, double tol, int32_t max_cycles,
                                         int32_t forced_cycles, nfvm_step_stats* stats) {
  // A is symmetric: the adjoint solve is the solve with xbar on the right
  return nfvm_mg_solve_device(grid, xbar_dev, bbar_dev, tol, max_cycles, forced_cycles, stats);
}

nfvm_status nfvm_pressure_adjoint_device(nfvm_grid_t grid, const double* ubar,
                                         const double* vbar, const double* wbar,
                                         const double* pbar, double* usbar, double* vsbar,
                                         double* wsbar, double tol, int32_t max_cycles,
                                         int32_t forced_cycles, nfvm_step_stats* stats) {
  if (!grid || !ubar || !vbar || !wbar || !pbar || !usbar || !vsbar || !wsbar)
    return fail(NFVM_E_INVAL, "grid and all seven arrays are required");
  return guard([&] {
    nfvm_status st = NFVM_OK;
    grid->g->pressure_adjoint(ubar, vbar, wbar, pbar, usbar, vsbar, wsbar, tol, max_cycles,
                              forced_cycles, stats, &st);
    if (st == NFVM_E_NOTCONV) set_error("adjoint pressure solve reached max_cycles");
    if (st == NFVM_E_DIVERGED) set_error("non-finite residual");
    return st;
  });
}

nfvm_status nfvm_explicit_adjoint_device(nfvm_grid_t grid, const nfvm_fields* state,
                                         const nfvm_fields* bar, nfvm_fields* out) {
  if (!grid || !state || !bar || !out) return fail(NFVM_E_INVAL, "grid, state, bar and out are required");
  return guard([&] {
    grid->g->explicit_adjoint(*state, *bar, *out);
    return NFVM_OK;
  });
}

nfvm_status nfvm_destroy_adjoint_device(nfvm_grid_t grid, const nfvm_fields* state, double tau,
                                        const double* kbar, const double* wbar,
                                        nfvm_fields* out) {
  if (!grid || !state || !out) return fail(NFVM_E_INVAL, "grid, state and out are required");
  return guard([&] {
    grid->g->destroy_adjoint(*state, tau, kbar, wbar, *out);
    return NFVM_OK;
  });
}

nfvm_status nfvm_step_adjoint_device(nfvm_grid_t grid, const nfvm_fields* state,
                                     const nfvm_fields* bar, nfvm_fields* out, double tol,
                                     int32_t max_cycles, int32_t forced_cycles,
                                     nfvm_step_stats* stats) {
  if (!grid || !state || !bar || !out)
    return fail(NFVM_E_INVAL, "grid, state, bar and out are required");
  return guard([&] {
    nfvm_status st = NFVM_OK;
    grid->g->step_adjoint(*state, *bar, *out, tol, max_cycles, forced_cycles, stats, &st);
    if (st == NFVM_E_NOTCONV) set_error("a pressure solve reached max_cycles");
    if (st == NFVM_E_DIVERGED) set_error("non-finite residual");
    return st;
  });
}

nfvm_status nfvm_mg_solve(nfvm_grid_t grid, const double* b, double* x, double tol,
                          int32_t max_cycles, int32_t forced_cycles, nfvm_step_stats* stats) {
  if (!grid || !b || !x) return fail(NFVM_E_INVAL, "grid, b and x are required");
  return guard([&] {
    const size_t bytes = (size_t)grid->g->ncells * sizeof(double);
    DevBuf bd, xd;
    hipStream_t s = grid->g->stream;
    bd.alloc(bytes, s);
    xd.alloc(bytes, s);
    NFVM_CK(hipMemcpyAsync(bd.p, b, bytes, hipMemcpyHostToDevice, s));
    NFVM_CK(hipMemcpyAsync(xd.p, x, bytes, hipMemcpyHostToDevice, s));
    nfvm_status st = NFVM_OK;
    grid->g->mg_solve(bd.as<double>(), xd.as<double>(), tol, max_cycles, forced_cycles, stats,
                      &st);
    NFVM_CK(hipMemcpyAsync(x, xd.p, bytes, hipMemcpyDeviceToHost, s));
    NFVM_CK(hipStreamSynchronize(s));
    if (st == NFVM_E_NOTCONV) set_error("pressure solve reached max_cycles");
    if (st == NFVM_E_DIVERGED) set_error("non-finite residual");
    return st;
  });
}

nfvm_status nfvm_get_fields(nfvm_grid_t grid, nfvm_fields* out) {
  if (!grid || !out) return fail(NFVM_E_INVAL, "grid and out are required");
  return guard([&] {
    grid->g->get_fields(out);
    return NFVM_OK;
  });
}

nfvm_status nfvm_lambda2(nfvm_grid_t grid, double* lambda2) {
  if (!grid || !lambda2) return fail(NFVM_E_INVAL, "grid and lambda2 are required");
  return guard([&] {
    grid->g->lambda2(lambda2);
    return NFVM_OK;
  });
}

nfvm_status nfvm_line_probe(nfvm_grid_t grid, const double* pts, int32_t n, double* out) {
  if (!grid) return fail(NFVM_E_INVAL, "grid is required");
  return guard([&] {
    grid->g->probe(pts, n, out);
    return NFVM_OK;
  });
}

nfvm_status nfvm_set_fields(nfvm_grid_t grid, const nfvm_fields* in) {
  if (!grid || !in) return fail(NFVM_E_INVAL, "grid and fields are required");
  return guard([&] {
    grid->g->set_fields(in);
    return NFVM_OK;
  });
}

nfvm_status nfvm_grid_footprint(const nfvm_grid_desc* desc, size_t* bytes) {
  if (!desc || !bytes) return fail(NFVM_E_INVAL, "desc and bytes are required");
  return guard([&] {
    validate_desc(*desc);
    *bytes = footprint_bytes(*desc);
    return NFVM_OK;
  });
}

nfvm_status nfvm_free_grid(nfvm_grid_t grid) {
  if (!grid) return fail(NFVM_E_INVAL, "grid is NULL");
  return guard([&] {
    std::string bad;
    try {
      bad = grid->g->check_guards();
    } catch (...) {
      delete grid;
      throw;
    }
    delete grid;
    if (!bad.empty())
      throw Error{NFVM_E_DEVICE, "out-of-bounds device store past: " + bad};
    return NFVM_OK;
  });
}

nfvm_status nfvm_profile(nfvm_grid_t grid, uint32_t kernel_mask) {
  if (!grid) return fail(NFVM_E_INVAL, "grid is NULL");
  return guard([&] {
    grid->g->prof_reset(kernel_mask & ((1u << NFVM_K_COUNT) - 1));
    return NFVM_OK;
  });
}

nfvm_status nfvm_profile_read(nfvm_grid_t grid, int32_t kernel, int64_t* launches,
                              double* seconds, double* bytes_per_launch) {
  if (!grid || kernel < 0 || kernel >= NFVM_K_COUNT)
    return fail(NFVM_E_INVAL, "bad grid or kernel id");
  if (launches) *launches = grid->g->prof_launches[kernel];
  if (seconds) *seconds = grid->g->prof_seconds[kernel];
  if (bytes_per_launch) {
    const long long n = grid->g->prof_launches[kernel];
    *bytes_per_launch = n ? grid->g->prof_bytes_sum[kernel] / (double)n : grid->g->prof_bytes[kernel];
  }
  return NFVM_OK;
}

nfvm_status nfvm_reduction_blocks(const nfvm_grid_desc* desc, int32_t* needed,
                                  int32_t* capacity) {
  if (!desc || !needed || !capacity) return fail(NFVM_E_INVAL, "desc, needed and capacity are required");
  return guard([&] {
    int n = 0, c = 0;
    reduction_blocks(*desc, &n, &c);
    *needed = n;
    *capacity = c;
    return NFVM_OK;
  });
}

nfvm_status nfvm_set_option(nfvm_grid_t grid, int32_t option, double value) {
  if (!grid) return fail(NFVM_E_INVAL, "grid is NULL");
  return guard([&] {
    grid->g->set_option(option, value);
    return NFVM_OK;
  });
}

nfvm_status nfvm_tune(const nfvm_grid_desc* desc) {
  if (!desc) return fail(NFVM_E_INVAL, "desc is required");
  return guard([&] {
    auto g = make_grid(*desc, nullptr, nullptr, 1);
    NFVM_CK(hipStreamSynchronize(g->stream));
    g.reset();
    return NFVM_OK;
  });
}

nfvm_status nfvm_tuning_table(int32_t* entries, int32_t max, int32_t* count) {
  if (!count || (max > 0 && !entries)) return fail(NFVM_E_INVAL, "count and entries are required");
  auto all = tune_entries();
  int n = 0;
  for (const auto& kv : all) {
    if (n >= max) break;
    int32_t* e = entries + 7 * n;
    e[0] = kv.first.kid;
    e[1] = kv.first.nx;
    e[2] = kv.first.ny;
    e[3] = kv.first.nz;
    e[4] = kv.first.dim;
    e[5] = kv.first.prec;
    e[6] = kv.second;
    ++n;
  }
  *count = n;
  return NFVM_OK;
}

const char* nfvm_last_error(void) { return t_err.c_str(); }

}  // extern "C"
