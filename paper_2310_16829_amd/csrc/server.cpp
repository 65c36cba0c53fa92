// Request loop with continuous batching over resident specimens: worker threads (slots) take
// the first runnable queued request; a specimen runs one request at a time, in submission
// order; specimen builds are admitted by device footprint against the budget, in order.
#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <mutex>
#include <set>
#include <string>
#include <thread>
#include <vector>

#include "lma.h"
#include "planner.hpp"

namespace {

using Clock = std::chrono::steady_clock;

struct Request {
  int64_t ticket = 0;
  lma_request r{};
  lma_optics optics{};
  lma_lattice lattice{};
  std::vector<double> inner, outer;
  int64_t need = 0;                       // BUILD: footprint admitted against the budget
  Clock::time_point submitted;
};

struct Done {
  lma_status status = LMA_OK;
  std::string message;
  double latency_ms = 0.0, service_ms = 0.0;
};

struct Specimen {
  lma_plan* plan = nullptr;
  int64_t bytes = 0;                      // admitted footprint while resident or building
  bool busy = false;
};

}  // namespace

struct lma_server {
  std::mutex m;
  std::condition_variable work_cv, done_cv;
  std::deque<Request> queue;
  std::map<int64_t, Done> done;
  std::set<int64_t> active;               // tickets queued or running
  std::vector<Specimen> spec;
  std::vector<std::thread> workers;
  int64_t budget = 0, in_use = 0, next_ticket = 1;
  int running = 0;
  bool stopping = false;

  // first runnable request: its specimen is idle and has no earlier queued request; a build
  // also needs the budget and no earlier queued build
  bool pick(Request* out) {
    std::vector<char> seen(spec.size(), 0);
    bool build_seen = false;
    for (auto it = queue.begin(); it != queue.end(); ++it) {
      const int s = it->r.specimen;
      const bool first_of_specimen = !seen[s];
      seen[s] = 1;
      const bool is_build = it->r.kind == LMA_REQ_BUILD;
      if (!first_of_specimen || spec[s].busy) {
        build_seen |= is_build;
        continue;
      }
      if (is_build && !spec[s].plan) {
        if (build_seen || in_use + it->need > budget) {
          build_seen = true;
          continue;
        }
        in_use += it->need;
        spec[s].bytes = it->need;
      }
      // a build for a resident specimen is refused when it runs: no bytes are admitted for it
      spec[s].busy = true;
      *out = std::move(*it);
      queue.erase(it);
      return true;
    }
    return false;
  }

  lma_status run(Request& q, std::string* msg) {
    Specimen& sp = spec[q.r.specimen];
    const lma_request& r = q.r;
    lma_status st = LMA_OK;
    auto check = [&](lma_status s) {
      if (s != LMA_OK && st == LMA_OK) {
        st = s;
        *msg = lma_last_error();
      }
      return s == LMA_OK;
    };
    if (r.kind == LMA_REQ_BUILD) {
      if (sp.plan) {
        *msg = "specimen " + std::to_string(r.specimen) + " is already resident (release it first)";
        return LMA_ERR_STATE;
      }
      lma_detectors d{(int32_t)q.inner.size(), q.inner.data(), q.outer.data()};
      lma_plan* plan = nullptr;
      const int32_t flags = (r.flags & LMA_HOST_ONLY) ? LMA_HOST_ONLY : LMA_OWN_STREAM;
      if (check(lma_build_basis(&q.optics, &q.lattice, &d, nullptr, flags, &plan))) sp.plan = plan;
      return st;
    }
    if (r.kind == LMA_REQ_RELEASE) {
      lma_destroy(sp.plan);
      sp.plan = nullptr;
      return st;
    }
    if (!sp.plan) {
      *msg = "specimen " + std::to_string(r.specimen) + " is not resident";
      return LMA_ERR_STATE;
    }
    if (r.kind == LMA_REQ_IMAGE) {
      if (check(lma_image(sp.plan, r.potential, r.nslices, r.image, r.flags, r.weight))) check(lma_synchronize(sp.plan));
    } else if (r.kind == LMA_REQ_PLAIN) {
      if (check(lma_plain_image(sp.plan, r.potential, r.nslices, r.image, r.flags, r.weight)))
        check(lma_synchronize(sp.plan));
    } else if (r.kind == LMA_REQ_EDIT) {
      int32_t nt = 0, np = 0;
      check(lma_recompute_local(sp.plan, r.potential, r.nslices, r.bbox, r.radius, r.image, &nt, &np));
    }
    return st;
  }

  // while stopping with nothing running, queued requests that can never start (a build the
  // budget cannot admit, and everything queued behind it) fail instead of waiting forever
  void fail_stuck() {
    while (!queue.empty()) {
      Request& q = queue.front();
      Done d;
      d.status = LMA_ERR_OOM;
      d.message = "server stopped before the request could be admitted";
      done[q.ticket] = std::move(d);
      active.erase(q.ticket);
      queue.pop_front();
    }
    done_cv.notify_all();
  }

  void worker() {
    std::unique_lock<std::mutex> lk(m);
    for (;;) {
      Request q;
      work_cv.wait(lk, [&] {
        if (pick(&q)) return true;
        if (stopping && running == 0 && !queue.empty()) fail_stuck();
        return stopping && queue.empty();
      });
      if (q.ticket == 0) return;   // stopping with nothing left
      ++running;
      lk.unlock();
      const Clock::time_point start = Clock::now();
      Done d;
      try {
        d.status = run(q, &d.message);
      } catch (const std::exception& e) {
        d.status = LMA_ERR_DEVICE;
        d.message = e.what();
      }
      const Clock::time_point end = Clock::now();
      d.latency_ms = std::chrono::duration<double, std::milli>(end - q.submitted).count();
      d.service_ms = std::chrono::duration<double, std::milli>(end - start).count();
      lk.lock();
      --running;
      Specimen& sp = spec[q.r.specimen];
      sp.busy = false;
      // a release frees the specimen's bytes, and so does a build that left no plan; a refused
      // build for a resident specimen admitted none
      const bool freed = (q.r.kind == LMA_REQ_RELEASE) || (q.r.kind == LMA_REQ_BUILD && !sp.plan);
      if (freed) {
        in_use -= sp.bytes;
        sp.bytes = 0;
      }
      done[q.ticket] = std::move(d);
      active.erase(q.ticket);
      done_cv.notify_all();
      work_cv.notify_all();
    }
  }
};

namespace {

lma_status server_fail(lma_status s, const std::string& msg) {
  lma::set_last_error(msg);
  return s;
}

}  // namespace

extern "C" {

lma_status lma_server_create(int32_t slots, int32_t max_specimens, int64_t budget_bytes, lma_server** out) {
  if (!out) return server_fail(LMA_ERR_ARG, "out is null");
  *out = nullptr;
  if (slots < 1 || slots > 64) return server_fail(LMA_ERR_ARG, "slots must be in 1..64");
  if (max_specimens < 1 || max_specimens > 4096) return server_fail(LMA_ERR_ARG, "max_specimens must be in 1..4096");
  if (budget_bytes <= 0) return server_fail(LMA_ERR_ARG, "budget_bytes must be > 0");
  try {
    lma_server* s = new lma_server();
    s->budget = budget_bytes;
    s->spec.resize(max_specimens);
    for (int i = 0; i < slots; ++i) s->workers.emplace_back([s] { s->worker(); });
    *out = s;
    return LMA_OK;
  } catch (const std::exception& e) {
    return server_fail(LMA_ERR_OOM, e.what());
  }
}

lma_status lma_server_submit(lma_server* s, const lma_request* r, int64_t* ticket) {
  const Clock::time_point submitted = Clock::now();
  if (!s || !r || !ticket) return server_fail(LMA_ERR_ARG, "null argument");
  if (r->specimen < 0 || r->specimen >= (int32_t)s->spec.size()) return server_fail(LMA_ERR_ARG, "specimen out of range");
  Request q;
  q.r = *r;
  switch (r->kind) {
    case LMA_REQ_BUILD: {
      if (!r->optics || !r->lattice || !r->detectors) return server_fail(LMA_ERR_ARG, "build needs optics, lattice, detectors");
      if (r->nslices < 1) return server_fail(LMA_ERR_ARG, "nslices must be >= 1");
      const lma_detectors& d = *r->detectors;
      if (d.n < 1 || d.n > 32 || !d.inner || !d.outer) return server_fail(LMA_ERR_ARG, "bad detectors");
      q.optics = *r->optics;
      q.lattice = *r->lattice;
      q.inner.assign(d.inner, d.inner + d.n);
      q.outer.assign(d.outer, d.outer + d.n);
      lma_detectors dc{d.n, q.inner.data(), q.outer.data()};
      lma_status st = lma_footprint(&q.optics, &q.lattice, &dc, r->nslices, &q.need);
      if (st != LMA_OK) return st;
      if (q.need > s->budget) return server_fail(LMA_ERR_OOM, "the specimen's footprint exceeds the server budget");
      break;
    }
    case LMA_REQ_IMAGE:
    case LMA_REQ_PLAIN:
    case LMA_REQ_EDIT:
      if (!r->potential || !r->image || r->nslices < 1) return server_fail(LMA_ERR_ARG, "request needs potential, image, nslices");
      break;
    case LMA_REQ_RELEASE:
      break;
    default:
      return server_fail(LMA_ERR_ARG, "unknown request kind");
  }
  q.r.optics = nullptr;
  q.r.lattice = nullptr;
  q.r.detectors = nullptr;
  q.submitted = submitted;
  {
    std::lock_guard<std::mutex> lk(s->m);
    if (s->stopping) return server_fail(LMA_ERR_STATE, "server is stopping");
    q.ticket = s->next_ticket++;
    *ticket = q.ticket;
    s->active.insert(q.ticket);
    s->queue.push_back(std::move(q));
  }
  s->work_cv.notify_all();
  return LMA_OK;
}

lma_status lma_server_wait(lma_server* s, int64_t ticket, double* latency_ms, double* service_ms) {
  if (!s) return server_fail(LMA_ERR_ARG, "server is null");
  std::unique_lock<std::mutex> lk(s->m);
  if (ticket < 1 || ticket >= s->next_ticket) return server_fail(LMA_ERR_ARG, "unknown ticket");
  // a ticket neither queued, running nor done was already waited for
  s->done_cv.wait(lk, [&] { return s->done.count(ticket) || !s->active.count(ticket); });
  if (!s->done.count(ticket)) return server_fail(LMA_ERR_ARG, "ticket " + std::to_string(ticket) + " was already waited for");
  Done d = std::move(s->done[ticket]);
  s->done.erase(ticket);
  lk.unlock();
  if (latency_ms) *latency_ms = d.latency_ms;
  if (service_ms) *service_ms = d.service_ms;
  if (d.status != LMA_OK) return server_fail(d.status, d.message);
  return LMA_OK;
}

lma_status lma_server_plan(lma_server* s, int32_t specimen, lma_plan** plan) {
  if (!s || !plan) return server_fail(LMA_ERR_ARG, "null argument");
  std::lock_guard<std::mutex> lk(s->m);
  if (specimen < 0 || specimen >= (int32_t)s->spec.size()) return server_fail(LMA_ERR_ARG, "specimen out of range");
  *plan = s->spec[specimen].plan;
  return LMA_OK;
}

lma_status lma_server_in_use(lma_server* s, int64_t* bytes) {
  if (!s || !bytes) return server_fail(LMA_ERR_ARG, "null argument");
  std::lock_guard<std::mutex> lk(s->m);
  *bytes = s->in_use;
  return LMA_OK;
}

void lma_server_destroy(lma_server* s) {
  if (!s) return;
  {
    std::lock_guard<std::mutex> lk(s->m);
    s->stopping = true;
  }
  s->work_cv.notify_all();
  for (auto& t : s->workers) t.join();
  for (auto& sp : s->spec) lma_destroy(sp.plan);
  delete s;
}

}  // extern "C"
