// Serving runtime: continuous batching of contraction requests.
//
// Many independent CTM runs (each with its own resident block tensors and
// cached plans, one plan per contraction of its enlarged-corner chain) submit
// requests; a request is one chain of contractions whose step i > 0 takes the
// output of step i - 1 as its A operand.  The server
//   * admits queued requests in arrival order while its device memory pool
//     can hold their intermediates and workspaces (admission by HBM budget),
//     letting a request that fits pass one that does not, at most 16 times
//     per waiting request (bounded bypass, no starvation);
//   * every tick, merges the next step of every admitted request into ONE
//     grouped launch (yastn_contract_jobs) on its stream, so requests that
//     arrive while others run join the very next launch and their work
//     overlaps on the device (continuous batching, not a queue);
//   * retires a request when the event recorded after the tick holding its
//     last step has completed, and returns its memory to the pool.
// Steps of one request run in consecutive ticks on one stream, so stream
// order carries the chain's dependencies and no host wait is needed between
// ticks; at most `max_ahead` ticks are outstanding.  The pool is one device
// allocation made at creation: serving itself never calls hipMalloc.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <deque>
#include <map>
#include <new>
#include <string>
#include <unordered_map>
#include <vector>

#include "planner.hpp"

namespace yastn {
const char *last_error_cstr();
}

using namespace yastn;

namespace {

constexpr size_t kAlign = 256;

size_t align_up(size_t b) { return (b + kAlign - 1) / kAlign * kAlign; }

double now_ms() {
  using namespace std::chrono;
  return duration<double, std::milli>(steady_clock::now().time_since_epoch()).count();
}

// First-fit allocator over one device range [0, size).
class Pool {
 public:
  explicit Pool(size_t size) : size_(size) { free_[0] = size; }
  bool alloc(size_t bytes, size_t *off) {
    for (auto it = free_.begin(); it != free_.end(); ++it)
      if (it->second >= bytes) {
        *off = it->first;
        const size_t rest = it->second - bytes;
        const size_t at = it->first + bytes;
        free_.erase(it);
        if (rest) free_[at] = rest;
        used_ += bytes;
        peak_ = std::max(peak_, used_);
        return true;
      }
    return false;
  }
  void release(size_t off, size_t bytes) {
    used_ -= bytes;
    auto it = free_.emplace(off, bytes).first;
    auto nx = std::next(it);
    if (nx != free_.end() && it->first + it->second == nx->first) {
      it->second += nx->second;
      free_.erase(nx);
    }
    if (it != free_.begin()) {
      auto pv = std::prev(it);
      if (pv->first + pv->second == it->first) {
        pv->second += it->second;
        free_.erase(it);
      }
    }
  }
  size_t used() const { return used_; }
  size_t peak() const { return peak_; }
  size_t size() const { return size_; }

 private:
  size_t size_, used_ = 0, peak_ = 0;
  std::map<size_t, size_t> free_;  // offset -> bytes
};

struct Request {
  int64_t id = 0;
  int nsteps = 0;
  yastn_plan_t plans[YASTN_MAX_CHAIN] = {};
  const void *a0 = nullptr;
  const void *b[YASTN_MAX_CHAIN] = {};
  void *out = nullptr;
  size_t c_bytes[YASTN_MAX_CHAIN] = {}, ws_bytes[YASTN_MAX_CHAIN] = {};
  size_t footprint = 0;  // pool bytes: intermediates of steps 0..n-2 and every workspace
  // runtime
  int state = YASTN_REQ_QUEUED;
  int next_step = 0;
  int64_t last_tick = -1;
  size_t pool_off = 0;
  void *inter[YASTN_MAX_CHAIN] = {};
  void *ws[YASTN_MAX_CHAIN] = {};
  double t_submit = 0, t_admit = 0, t_done = 0;
  int bypassed = 0;  // later requests admitted while this one waited
  // pointer arrays handed to yastn_contract_jobs for the step being launched
  const void *pa[1] = {}, *pb[1] = {};
  void *pc[1] = {};
};

struct Tick {
  int64_t id;
  hipEvent_t ev;
};

}  // namespace

struct yastn_server_s {
  hipStream_t stream = nullptr;
  char *base = nullptr;
  Pool *pool = nullptr;
  int max_ahead = 2;
  int64_t next_id = 1, next_tick = 0;
  std::deque<int64_t> queue;                       // submitted, not admitted (FIFO)
  std::vector<int64_t> running;                    // admitted, not retired
  std::unordered_map<int64_t, Request> reqs;       // every request not yet forgotten
  std::deque<Tick> ticks;                          // launched, not retired (in order)
  std::vector<hipEvent_t> spare;                   // events free for reuse
  yastn_server_stats st{};
};

namespace {

yastn_status fail(yastn_status s, const std::string &m) { return set_error(s, m); }

// Retire every completed tick at the head of the tick queue (wait = block on the
// oldest one first).
yastn_status retire(yastn_server_s *s, bool wait) {
  while (!s->ticks.empty()) {
    Tick &tk = s->ticks.front();
    hipError_t e = wait ? hipEventSynchronize(tk.ev) : hipEventQuery(tk.ev);
    if (e == hipErrorNotReady) return YASTN_OK;
    if (e != hipSuccess) {
      (void)hipGetLastError();
      return fail(YASTN_ERR_HIP, std::string("server tick: ") + hipGetErrorString(e));
    }
    wait = false;
    const double t = now_ms();
    for (size_t i = 0; i < s->running.size();) {
      Request &r = s->reqs[s->running[i]];
      if (r.last_tick >= 0 && r.last_tick <= tk.id) {
        r.state = YASTN_REQ_DONE;
        r.t_done = t;
        if (r.footprint) s->pool->release(r.pool_off, r.footprint);
        s->st.completed += 1;
        s->running[i] = s->running.back();
        s->running.pop_back();
      } else {
        ++i;
      }
    }
    s->spare.push_back(tk.ev);
    s->ticks.pop_front();
  }
  return YASTN_OK;
}

// Admission in arrival order with bounded bypass: a queued request whose
// footprint does not fit now is skipped and later requests that fit are
// admitted past it, but each waiting request can be passed at most
// kMaxBypass times; once a request has been passed that often nothing is
// admitted past it any more (it is admitted next, as soon as memory frees
// up), so no request starves behind a stream of smaller ones.
constexpr int kMaxBypass = 16;

void admit_one(yastn_server_s *s, Request &r, size_t off) {
    r.pool_off = off;
    char *p = s->base + off;
    for (int i = 0; i < r.nsteps; ++i) {
      if (i + 1 < r.nsteps) {
        r.inter[i] = p;
        p += align_up(r.c_bytes[i]);
      } else {
        r.inter[i] = r.out;
      }
    }
    for (int i = 0; i < r.nsteps; ++i) {
      r.ws[i] = r.ws_bytes[i] ? p : nullptr;
      p += align_up(r.ws_bytes[i]);
    }
    r.state = YASTN_REQ_RUNNING;
    r.t_admit = now_ms();
    s->running.push_back(r.id);
    s->st.admitted += 1;
}

void admit(yastn_server_s *s) {
  size_t k = 0;
  while (k < s->queue.size()) {
    Request &r = s->reqs[s->queue[k]];
    size_t off = 0;
    if (!r.footprint || s->pool->alloc(r.footprint, &off)) {
      admit_one(s, r, off);
      // every request still waiting ahead of it has been passed once more;
      // one that reached the bound stops admission past it
      bool bound = false;
      for (size_t i = 0; i < k; ++i) bound |= ++s->reqs[s->queue[i]].bypassed >= kMaxBypass;
      if (k > 0) s->st.bypasses += 1;
      s->queue.erase(s->queue.begin() + (std::ptrdiff_t)k);
      if (bound) return;
      continue;
    }
    if (r.bypassed >= kMaxBypass) return;  // the bound: nothing passes this request
    ++k;
  }
}

}  // namespace

extern "C" {

yastn_status yastn_server_create(size_t pool_bytes, int32_t max_ahead, void *hip_stream, yastn_server_t *out) {
  if (!out) return fail(YASTN_ERR_ARG, "null server output");
  *out = nullptr;
  if (max_ahead < 1 || max_ahead > 64) return fail(YASTN_ERR_ARG, "max_ahead must be in 1..64");
  yastn_server_s *s = new (std::nothrow) yastn_server_s();
  if (!s) return fail(YASTN_ERR_NOMEM, "host allocation");
  s->stream = reinterpret_cast<hipStream_t>(hip_stream);
  s->max_ahead = max_ahead;
  if (pool_bytes) {
    void *p = nullptr;
    hipError_t e = hipMalloc(&p, align_up(pool_bytes));
    if (e != hipSuccess) {
      (void)hipGetLastError();
      delete s;
      return fail(e == hipErrorOutOfMemory ? YASTN_ERR_NOMEM : YASTN_ERR_HIP,
                  std::string("server pool: ") + hipGetErrorString(e));
    }
    s->base = static_cast<char *>(p);
  }
  s->pool = new (std::nothrow) Pool(pool_bytes ? align_up(pool_bytes) : 0);
  if (!s->pool) {
    if (s->base) (void)hipFree(s->base);
    delete s;
    return fail(YASTN_ERR_NOMEM, "host allocation");
  }
  s->st.pool_bytes = s->pool->size();
  *out = s;
  return YASTN_OK;
}

yastn_status yastn_server_submit(yastn_server_t s, const yastn_request *rq, int64_t *id) {
  if (!s || !rq || !id) return fail(YASTN_ERR_ARG, "null argument");
  if (rq->nsteps < 1 || rq->nsteps > YASTN_MAX_CHAIN) return fail(YASTN_ERR_ARG, "nsteps must be in 1..YASTN_MAX_CHAIN");
  if (!rq->plans || !rq->b || !rq->out) return fail(YASTN_ERR_ARG, "null request arrays");
  Request r;
  r.nsteps = rq->nsteps;
  r.a0 = rq->a0;
  r.out = rq->out;
  for (int i = 0; i < r.nsteps; ++i) {
    if (!rq->plans[i]) return fail(YASTN_ERR_ARG, "null plan in request");
    r.plans[i] = rq->plans[i];
    r.b[i] = rq->b[i];
    yastn_options o;
    int32_t nprob = 0;
    yastn_status e = yastn_plan_info(r.plans[i], &o, &nprob);
    if (e) return e;
    if (nprob != 1) return fail(YASTN_ERR_STATE, "request steps must be single-problem plans");
    yastn_tensor_desc c;
    int64_t c_numel = 0;
    if ((e = yastn_plan_output(r.plans[i], 0, &c, &c_numel))) return e;
    size_t ws = 0;
    if ((e = yastn_plan_workspace(r.plans[i], &ws))) return e;
    r.c_bytes[i] = size_t(c_numel) * (o.out_dtype == YASTN_DTYPE_F64 ? 8 : 4);
    r.ws_bytes[i] = ws;
    if (i + 1 < r.nsteps) r.footprint += align_up(r.c_bytes[i]);
    r.footprint += align_up(ws);
  }
  if (r.footprint > s->pool->size()) return fail(YASTN_ERR_NOMEM, "request needs more memory than the server pool");
  r.id = s->next_id++;
  r.t_submit = now_ms();
  s->queue.push_back(r.id);
  s->reqs.emplace(r.id, r);
  s->st.submitted += 1;
  s->st.queued_peak = std::max<int64_t>(s->st.queued_peak, (int64_t)s->queue.size());
  *id = r.id;
  return YASTN_OK;
}

yastn_status yastn_server_step(yastn_server_t s, int32_t *launched) {
  if (!s) return fail(YASTN_ERR_ARG, "null server");
  if (launched) *launched = 0;
  yastn_status e = retire(s, false);
  if (e) return e;
  admit(s);
  // the next step of every admitted request whose chain is not fully launched
  std::vector<yastn_job> jobs;
  std::vector<int64_t> who;
  for (int64_t rid : s->running) {
    Request &r = s->reqs[rid];
    if (r.next_step >= r.nsteps) continue;
    const int i = r.next_step;
    r.pa[0] = i == 0 ? r.a0 : r.inter[i - 1];
    r.pb[0] = r.b[i];
    r.pc[0] = r.inter[i];
    jobs.push_back(yastn_job{r.plans[i], r.pa, r.pb, r.pc, r.ws[i]});
    who.push_back(rid);
  }
  if (jobs.empty()) return YASTN_OK;
  if ((int)s->ticks.size() >= s->max_ahead && (e = retire(s, true))) return e;
  // one grouped launch per precision class (plans of one launch must agree)
  std::vector<char> done(jobs.size(), 0);
  for (size_t i = 0; i < jobs.size(); ++i) {
    if (done[i]) continue;
    yastn_options oi;
    int32_t np = 0;
    (void)yastn_plan_info(jobs[i].plan, &oi, &np);
    std::vector<yastn_job> group;
    for (size_t j = i; j < jobs.size(); ++j) {
      if (done[j]) continue;
      yastn_options oj;
      (void)yastn_plan_info(jobs[j].plan, &oj, &np);
      if (oj.precision == oi.precision && oj.in_dtype == oi.in_dtype && oj.out_dtype == oi.out_dtype) {
        group.push_back(jobs[j]);
        done[j] = 1;
      }
    }
    if ((e = yastn_contract_jobs(group.data(), (int32_t)group.size(), s->stream))) return e;
  }
  hipEvent_t ev;
  if (!s->spare.empty()) {
    ev = s->spare.back();
    s->spare.pop_back();
  } else if (hipEventCreateWithFlags(&ev, hipEventDisableTiming) != hipSuccess) {
    (void)hipGetLastError();
    return fail(YASTN_ERR_HIP, "event creation failed");
  }
  if (hipEventRecord(ev, s->stream) != hipSuccess) {
    (void)hipGetLastError();
    return fail(YASTN_ERR_HIP, "event record failed");
  }
  const int64_t tick = s->next_tick++;
  for (int64_t rid : who) {
    Request &r = s->reqs[rid];
    r.next_step += 1;
    if (r.next_step == r.nsteps) r.last_tick = tick;
  }
  s->ticks.push_back(Tick{tick, ev});
  s->st.ticks += 1;
  s->st.launched_steps += (int64_t)jobs.size();
  s->st.max_batch = std::max<int64_t>(s->st.max_batch, (int64_t)jobs.size());
  if (launched) *launched = (int32_t)jobs.size();
  return YASTN_OK;
}

yastn_status yastn_server_query(yastn_server_t s, int64_t id, int32_t *state, double *latency_ms) {
  if (!s || !state) return fail(YASTN_ERR_ARG, "null argument");
  auto it = s->reqs.find(id);
  if (it == s->reqs.end()) return fail(YASTN_ERR_ARG, "unknown request id");
  *state = it->second.state;
  if (latency_ms) *latency_ms = it->second.state == YASTN_REQ_DONE ? it->second.t_done - it->second.t_submit : -1.0;
  return YASTN_OK;
}

yastn_status yastn_server_forget(yastn_server_t s, int64_t id) {
  if (!s) return fail(YASTN_ERR_ARG, "null server");
  auto it = s->reqs.find(id);
  if (it == s->reqs.end()) return fail(YASTN_ERR_ARG, "unknown request id");
  if (it->second.state != YASTN_REQ_DONE) return fail(YASTN_ERR_STATE, "request not finished");
  s->reqs.erase(it);
  return YASTN_OK;
}

yastn_status yastn_server_drain(yastn_server_t s) {
  if (!s) return fail(YASTN_ERR_ARG, "null server");
  for (;;) {
    yastn_status e = yastn_server_step(s, nullptr);
    if (e) return e;
    if (s->queue.empty() && s->running.empty()) return YASTN_OK;
    if ((e = retire(s, true))) return e;
  }
}

yastn_status yastn_server_get_stats(yastn_server_t s, yastn_server_stats *out) {
  if (!s || !out) return fail(YASTN_ERR_ARG, "null argument");
  *out = s->st;
  out->queued = (int64_t)s->queue.size();
  out->running = (int64_t)s->running.size();
  out->pool_used = s->pool->used();
  out->pool_peak = s->pool->peak();
  return YASTN_OK;
}

void yastn_server_destroy(yastn_server_t s) {
  if (!s) return;
  if (!s->ticks.empty()) (void)hipStreamSynchronize(s->stream);
  for (auto &t : s->ticks) (void)hipEventDestroy(t.ev);
  for (hipEvent_t e : s->spare) (void)hipEventDestroy(e);
  if (s->base) (void)hipFree(s->base);
  delete s->pool;
  delete s;
}

}  // extern "C"
