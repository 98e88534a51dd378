// Serving loop: requests of different grid sizes are queued, admitted while
// their summed device footprint stays inside the HBM budget and a slot is
// free, and run on their own HIP streams so that admitted solves overlap on
// the device.  A slot picks up the next admissible request as soon as its
// previous one finishes (continuous admission at step boundaries); a finished
// solve releases its device memory at once and keeps its fields on the host
// until polled.
#include <math.h>
#include <string.h>

#include <chrono>
#include <condition_variable>
#include <deque>
#include <map>
#include <mutex>
#include <thread>
#include <vector>

#include "engine.hpp"

using namespace nfvm;

namespace {

enum { Q_QUEUED = 0, Q_RUNNING = 1, Q_DONE = 2 };

struct Request {
  uint64_t id = 0;
  nfvm_grid_desc desc{};
  std::vector<nfvm_patch> patches;
  std::vector<uint8_t> mask;
  std::vector<double> f[7];  // u v w p T k omega, host FP64
  int n_steps = 0;
  size_t footprint = 0;
  int state = Q_QUEUED;
  nfvm_status status = NFVM_OK;
  nfvm_step_stats last{};
  double t[4] = {-1, -1, -1, -1};  // submit, admit, first converged step, done
  std::string err;
};

double now_since(std::chrono::steady_clock::time_point t0) {
  return std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
}

}  // namespace

struct nfvm_server {
  std::mutex mu;
  std::condition_variable cv;
  std::deque<uint64_t> queue;
  std::map<uint64_t, std::unique_ptr<Request>> reqs;
  size_t budget = 0, used = 0;
  int slots = 1, running = 0;
  bool stop = false;
  uint64_t next_id = 1;
  int device = 0;
  std::chrono::steady_clock::time_point t0 = std::chrono::steady_clock::now();
  std::vector<std::thread> workers;

  // first request in arrival order whose footprint fits the free budget
  Request* take_admissible() {
    for (auto it = queue.begin(); it != queue.end(); ++it) {
      Request* r = reqs[*it].get();
      if (used + r->footprint <= budget) {
        queue.erase(it);
        return r;
      }
    }
    return nullptr;
  }

  void run(Request* r) {
    nfvm_fields init;
    init.u = r->f[0].data();
    init.v = r->f[1].data();
    init.w = r->f[2].data();
    init.p = r->f[3].data();
    init.T = r->f[4].data();
    init.k = r->f[5].data();
    init.omega = r->f[6].data();
    nfvm_grid_desc d = r->desc;
    d.patches = r->patches.empty() ? nullptr : r->patches.data();
    d.solid_mask = r->mask.empty() ? nullptr : r->mask.data();
    nfvm_status st = NFVM_OK;
    try {
      // tiles: the autotuner's cached choices, never a tuning run on the
      // request's critical path
      std::unique_ptr<GridBase> g = make_grid(d, &init, nullptr, 2);
      for (int s = 0; s < r->n_steps; ++s) {
        nfvm_step_stats ss{};
        nfvm_status one = NFVM_OK;
        g->step(1, &ss, &one);
        r->last = ss;
        if (one == NFVM_OK && r->t[2] < 0) {
          std::lock_guard<std::mutex> lk(mu);
          r->t[2] = now_since(t0);
        }
        if (one == NFVM_E_DIVERGED) {
          st = one;
          break;
        }
        if (one != NFVM_OK && st == NFVM_OK) st = one;
      }
      if (st != NFVM_E_DIVERGED) g->get_fields(&init);
    } catch (const Error& e) {
      st = e.st;
      r->err = e.msg;
    } catch (const std::exception& e) {
      st = NFVM_E_DEVICE;
      r->err = e.what();
    }
    std::lock_guard<std::mutex> lk(mu);
    r->status = st;
    r->state = Q_DONE;
    r->t[3] = now_since(t0);
    used -= r->footprint;
    --running;
    cv.notify_all();
  }

  void worker() {
    (void)hipSetDevice(device);
    for (;;) {
      Request* r = nullptr;
      {
        std::unique_lock<std::mutex> lk(mu);
        cv.wait(lk, [&] {
          if (stop) return true;
          for (uint64_t id : queue)
            if (used + reqs[id]->footprint <= budget) return true;
          return false;
        });
        if (stop) return;
        r = take_admissible();
        if (!r) continue;
        used += r->footprint;
        ++running;
        r->state = Q_RUNNING;
        r->t[1] = now_since(t0);
      }
      run(r);
    }
  }
};


static nfvm_status sfail(nfvm_status st, const std::string& m) {
  set_error(m);
  return st;
}

extern "C" {

nfvm_status nfvm_server_create(double hbm_budget_bytes, int32_t max_slots, nfvm_server_t* out) {
  if (!out || max_slots < 1) return sfail(NFVM_E_INVAL, "out and max_slots >= 1 are required");
  *out = nullptr;
  auto* s = new nfvm_server();
  (void)hipGetDevice(&s->device);
  if (hbm_budget_bytes > 0) {
    s->budget = (size_t)hbm_budget_bytes;
  } else {
    size_t fr = 0, tot = 0;
    if (hipMemGetInfo(&fr, &tot) != hipSuccess) {
      delete s;
      return sfail(NFVM_E_DEVICE, "hipMemGetInfo failed");
    }
    s->budget = (size_t)(0.9 * (double)fr);
  }
  s->slots = max_slots;
  for (int i = 0; i < max_slots; ++i) s->workers.emplace_back([s] { s->worker(); });
  *out = s;
  return NFVM_OK;
}

nfvm_status nfvm_submit(nfvm_server_t s, const nfvm_grid_desc* desc, const nfvm_fields* init,
                        int32_t n_steps, uint64_t* ticket) {
  if (!s || !desc || !init || !ticket || n_steps < 0)
    return sfail(NFVM_E_INVAL, "server, desc, init, ticket and n_steps >= 0 are required");
  const double* src[7] = {init->u, init->v, init->w, init->p, init->T, init->k, init->omega};
  for (int f = 0; f < 7; ++f)
    if (!src[f]) return sfail(NFVM_E_INVAL, "all seven init fields are required");
  std::unique_ptr<Request> r(new Request());
  try {
    validate_desc(*desc);
    r->footprint = footprint_bytes(*desc);
  } catch (const Error& e) {
    return sfail(e.st, e.msg);
  }
  if (r->footprint > s->budget)
    return sfail(NFVM_E_NOMEM, "request footprint " + std::to_string(r->footprint) +
                                   " B exceeds the server budget");
  r->desc = *desc;
  r->patches.assign(desc->patches, desc->patches + desc->n_patches);
  const size_t N = (size_t)desc->n[0] * desc->n[1] * desc->n[2];
  if (desc->solid_mask) r->mask.assign(desc->solid_mask, desc->solid_mask + N);
  for (int f = 0; f < 7; ++f) r->f[f].assign(src[f], src[f] + N);
  r->n_steps = n_steps;
  std::lock_guard<std::mutex> lk(s->mu);
  r->id = s->next_id++;
  r->t[0] = now_since(s->t0);
  *ticket = r->id;
  s->queue.push_back(r->id);
  s->reqs[r->id] = std::move(r);
  s->cv.notify_all();
  return NFVM_OK;
}

nfvm_status nfvm_poll(nfvm_server_t s, uint64_t ticket, nfvm_fields* out, nfvm_step_stats* last) {
  if (!s) return sfail(NFVM_E_INVAL, "server is NULL");
  std::unique_ptr<Request> r;
  {
    std::lock_guard<std::mutex> lk(s->mu);
    auto it = s->reqs.find(ticket);
    if (it == s->reqs.end()) return sfail(NFVM_E_NOTFOUND, "unknown ticket");
    if (it->second->state != Q_DONE) return NFVM_PENDING;
    r = std::move(it->second);
    s->reqs.erase(it);
  }
  if (out) {
    double* dst[7] = {out->u, out->v, out->w, out->p, out->T, out->k, out->omega};
    for (int f = 0; f < 7; ++f)
      if (dst[f]) memcpy(dst[f], r->f[f].data(), r->f[f].size() * sizeof(double));
  }
  if (last) *last = r->last;
  if (r->status != NFVM_OK) set_error(r->err.empty() ? "request finished with an error" : r->err);
  return r->status;
}

nfvm_status nfvm_request_times(nfvm_server_t s, uint64_t ticket, double times[4]) {
  if (!s || !times) return sfail(NFVM_E_INVAL, "server and times are required");
  std::lock_guard<std::mutex> lk(s->mu);
  auto it = s->reqs.find(ticket);
  if (it == s->reqs.end()) return sfail(NFVM_E_NOTFOUND, "unknown ticket");
  for (int i = 0; i < 4; ++i) times[i] = it->second->t[i];
  return NFVM_OK;
}

nfvm_status nfvm_server_drain(nfvm_server_t s) {
  if (!s) return sfail(NFVM_E_INVAL, "server is NULL");
  std::unique_lock<std::mutex> lk(s->mu);
  s->cv.wait(lk, [&] { return s->queue.empty() && s->running == 0; });
  return NFVM_OK;
}

nfvm_status nfvm_server_destroy(nfvm_server_t s) {
  if (!s) return sfail(NFVM_E_INVAL, "server is NULL");
  {
    std::unique_lock<std::mutex> lk(s->mu);
    s->cv.wait(lk, [&] { return s->running == 0; });
    s->stop = true;
    s->cv.notify_all();
  }
  for (auto& t : s->workers) t.join();
  delete s;
  return NFVM_OK;
}

}  // extern "C"
