// Serving loop: requests of different grid sizes are queued and admitted,
// first fit in arrival order, while their summed device footprint stays
// inside the HBM budget and fewer than max_slots grids run.  Admitted grids
// run in up to three lanes, each a host thread with its own HIP stream and a
// BatchRunner: per round, the CG iterations of all the lane's grids whose
// pressure solve is under way run as batched launches (one launch per
// multigrid kernel and level over the tiles of every grid), then one
// synchronisation.  Lanes overlap on the device, so one lane's host work
// (a synchronisation, a grid's creation or the download of its fields) does
// not leave the device idle.  A grid whose solve converged goes on to its
// next step at once; a request joins its lane at the next round after its
// admission (continuous batching); a finished request releases its device
// memory at once and keeps its fields on the host until polled.
#include <math.h>
#include <string.h>

#include <chrono>
#include <condition_variable>
#include <algorithm>
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

  // One admitted request: its grid and per-step statistics.
  struct Active {
    Request* r;
    std::unique_ptr<GridBase> g;
    std::vector<nfvm_step_stats> stats;
  };

  std::unique_ptr<GridBase> make(Request* r, hipStream_t s) {
    nfvm_fields init;
    double** dst[7] = {&init.u, &init.v, &init.w, &init.p, &init.T, &init.k, &init.omega};
    for (int f = 0; f < 7; ++f) *dst[f] = r->f[f].data();
    nfvm_grid_desc d = r->desc;
    d.patches = r->patches.empty() ? nullptr : r->patches.data();
    d.solid_mask = r->mask.empty() ? nullptr : r->mask.data();
    // tiles: the autotuner's cached choices, never a tuning run on the
    // request's critical path
    return make_grid(d, &init, s, 2);
  }

  void finish(Active& a, nfvm_status st, const std::string& err) {
    Request* r = a.r;
    for (const nfvm_step_stats& x : a.stats)  // the last step that ran
      if (x.status != NFVM_PENDING) r->last = x;
    if (a.g && st != NFVM_E_DIVERGED) {
      try {
        nfvm_fields out;
        double** dst[7] = {&out.u, &out.v, &out.w, &out.p, &out.T, &out.k, &out.omega};
        for (int f = 0; f < 7; ++f) *dst[f] = r->f[f].data();
        a.g->get_fields(&out);
      } catch (const Error& e) {
        st = e.st;
        r->err = e.msg;
      }
    }
    a.g.reset();
    std::lock_guard<std::mutex> lk(mu);
    r->status = st;
    if (!err.empty()) r->err = err;
    r->state = Q_DONE;
    r->t[3] = now_since(t0);
    used -= r->footprint;
    --running;
    cv.notify_all();
  }

  // one lane: up to cap grids advanced together on the lane's stream
  void worker(int cap) {
    (void)hipSetDevice(device);
    hipStream_t s = nullptr;
    if (hipStreamCreateWithFlags(&s, hipStreamNonBlocking) != hipSuccess) s = nullptr;
    std::vector<Active> act;
    std::unique_ptr<BatchRunner> br(new BatchRunner(s));
    for (;;) {
      std::vector<Request*> admit;
      {
        std::unique_lock<std::mutex> lk(mu);
        if (act.empty())
          cv.wait(lk, [&] {
            if (stop) return true;
            if (running >= slots) return false;
            for (uint64_t id : queue)
              if (used + reqs[id]->footprint <= budget) return true;
            return false;
          });
        if (stop && act.empty()) break;
        while ((int)(act.size() + admit.size()) < cap && running < slots) {
          Request* r = take_admissible();
          if (!r) break;
          used += r->footprint;
          ++running;
          r->state = Q_RUNNING;
          r->t[1] = now_since(t0);
          admit.push_back(r);
        }
      }
      for (Request* r : admit) {
        Active a{r, nullptr, std::vector<nfvm_step_stats>(r->n_steps)};
        for (nfvm_step_stats& x : a.stats) x.status = NFVM_PENDING;
        try {
          if (!s) throw Error{NFVM_E_DEVICE, "stream creation failed"};
          a.g = make(r, s);
          br->add(a.g.get(), r->n_steps, a.stats.data());
          act.push_back(std::move(a));
        } catch (const Error& e) {
          finish(a, e.st, e.msg);
        } catch (const std::exception& e) {
          finish(a, NFVM_E_DEVICE, e.what());
        }
      }
      if (act.empty()) continue;
      std::vector<GridBase*> over;
      try {
        over = br->advance();
      } catch (const Error& e) {
        // a device error ends every running request
        for (Active& a : act) finish(a, e.st, e.msg);
        act.clear();
        br.reset(new BatchRunner(s));
        continue;
      } catch (const std::exception& e) {
        for (Active& a : act) finish(a, NFVM_E_DEVICE, e.what());
        act.clear();
        br.reset(new BatchRunner(s));
        continue;
      }
      for (auto it = act.begin(); it != act.end();) {
        Active& a = *it;
        if (a.r->t[2] < 0 && a.g->run_converged() > 0) {
          std::lock_guard<std::mutex> lk(mu);
          a.r->t[2] = now_since(t0);
        }
        if (std::find(over.begin(), over.end(), a.g.get()) != over.end()) {
          finish(a, a.g->run_status(), "");
          it = act.erase(it);
        } else {
          ++it;
        }
      }
    }
    br.reset();
    if (s) (void)hipStreamDestroy(s);
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
  const int lanes = std::min(max_slots, 3);
  const int cap = (max_slots + lanes - 1) / lanes;
  for (int i = 0; i < lanes; ++i) s->workers.emplace_back([s, cap] { s->worker(cap); });
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
