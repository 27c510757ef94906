// Request server with continuous batching at GMRES-cycle granularity.
//
// Requests are grouped by (restart length, precision, cycle cap, Krylov
// iteration, size class); each group has its own batch engine, HIP stream and
// host thread.  A group's thread runs cycles back to back: between cycles it
// retires every finished problem (back substitution and output, result
// published to the ticket) and admits queued requests of its group in arrival
// order while their device footprint fits the server's budget and a slot is
// free; admitted requests run their set-up phase and join the next cycle.
// Groups therefore overlap on the device and on the host, and a short
// request does not wait for a long one's cycle: the problems of one engine
// advance in lockstep, one step per launch at the pace of the largest, so
// centres of very different sizes go to different groups.  A request's
// arithmetic does not depend on the other problems in the batch (per-problem
// kernels and reductions), so its result is the same alone and in the mix.
#include "server.h"

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <thread>
#include <tuple>

namespace fds {

namespace {

using Clock = std::chrono::steady_clock;

struct Pending {
  uint64_t ticket;
  SolveRequest req;
  size_t bytes;
  Clock::time_point submitted;
  hipEvent_t ready;   // recorded on the submitter's stream (inputs written)
};

// restart_m, precision, max_cycles, flags, size class
using Key = std::tuple<int, int, int, unsigned, int>;

// Size class of a plan's coupled rectangle: by default centres up to 512
// and above 512 nodes per side (two groups per option set: on a served
// stream with n from 64 to 2048 this gave the lowest median latency of the
// splits tried, 4.6 ms against 5.8 ms for three classes bounded at 256 and
// 1024); FDS_SERVER_CLASSES ("a,b,...", ascending) sets other bounds.
int size_class(const fds_plan* p) {
  static const std::vector<int> bounds = [] {
    std::vector<int> v;
    if (const char* e = std::getenv("FDS_SERVER_CLASSES")) {
      int prev = 0;
      for (const char* q = e; *q;) {
        char* end = nullptr;
        const long b = std::strtol(q, &end, 10);
        if (end == q || b <= prev || b > (1 << 20)) { v.clear(); break; }
        v.push_back((int)b);
        prev = (int)b;
        q = *end == ',' ? end + 1 : end;
        if (*end != ',' && *end != 0) { v.clear(); break; }
      }
    }
    if (v.empty()) v = {512};
    return v;
  }();
  const int n = std::max(p->nx, p->ny);
  int c = 0;
  while (c < (int)bounds.size() && n > bounds[c]) ++c;
  return c;
}

Key key_of(const fds_plan* p) {
  return Key{p->opt.restart_m, p->opt.precision, p->opt.max_cycles, p->opt.flags, size_class(p)};
}

double seconds_since(Clock::time_point a) { return std::chrono::duration<double>(Clock::now() - a).count(); }

}  // namespace

}  // namespace fds

struct fds_server {
  struct Group {
    fds::Key key;
    hipStream_t stream = nullptr;
    std::unique_ptr<fds::Engine> eng;   // touched by the group's thread only
    std::map<int, fds::Pending> running;
    int next_id = 0;
    double tasks_seen = 0;
    std::thread th;
  };

  size_t budget = 0;
  int max_slots = 0;
  int device = 0;
  // everything below is guarded by mu (an engine belongs to its group's thread)
  std::mutex mu;
  std::condition_variable cv;   // new requests, freed memory or slots, stop
  std::condition_variable done_cv;   // a result was published
  std::deque<fds::Pending> queue;
  std::map<uint64_t, fds_result> done;
  std::map<uint64_t, int> state;   // 0 queued, 1 running, 2 done
  uint64_t next_ticket = 1;
  bool stop = false;
  std::vector<hipEvent_t> event_pool;
  fds_server_stats stats{};
  size_t used = 0;   // footprint of the admitted requests
  int running = 0;   // admitted requests not yet published
  std::map<fds::Key, std::unique_ptr<Group>> groups;

  void group_loop(Group* g);
  bool admissible_locked(const Group* g) const;
  bool has_queued_locked(const Group* g) const;
  void publish_locked(const fds::Pending& p, const fds_result& r);
  void fail_group(Group* g, fds_status st);
  hipEvent_t take_event();
};

hipEvent_t fds_server::take_event() {
  {
    std::lock_guard<std::mutex> lk(mu);
    if (!event_pool.empty()) {
      hipEvent_t e = event_pool.back();
      event_pool.pop_back();
      return e;
    }
  }
  hipEvent_t e = nullptr;
  FDS_HIP(hipEventCreateWithFlags(&e, hipEventDisableTiming));
  return e;
}

void fds_server::publish_locked(const fds::Pending& p, const fds_result& r0) {
  fds_result r = r0;
  r.seconds = fds::seconds_since(p.submitted);
  done[p.ticket] = r;
  state[p.ticket] = 2;
  stats.completed += 1;
  // the event's wait was queued before the set-up phase, which has finished
  if (p.ready) event_pool.push_back(p.ready);
  done_cv.notify_all();
}

// Publishes a failure for every request of the group and drops its engine
// (its state is unknown after a failure).
void fds_server::fail_group(Group* g, fds_status st) {
  fds_result r{};
  r.status = st;
  std::lock_guard<std::mutex> lk(mu);
  for (auto& pr : g->running) {
    publish_locked(pr.second, r);
    used -= pr.second.bytes;
    --running;
  }
  g->running.clear();
  if (g->eng) stats.host_tasks_s += g->eng->host_task_seconds() - g->tasks_seen;
  g->tasks_seen = 0;
  g->eng.reset();
  cv.notify_all();
}

bool fds_server::has_queued_locked(const Group* g) const {
  for (const fds::Pending& p : queue)
    if (fds::key_of(p.req.plan) == g->key) return true;
  return false;
}

// Whether the group's first queued request can be admitted now: a slot is
// free and its footprint fits the budget (always, when nothing runs at all).
bool fds_server::admissible_locked(const Group* g) const {
  if (running >= max_slots) return false;
  for (const fds::Pending& p : queue)
    if (fds::key_of(p.req.plan) == g->key) return used + p.bytes <= budget || running == 0;
  return false;
}

void fds_server::group_loop(Group* g) {
  (void)hipSetDevice(device);
  using fds::Clock;
  while (true) {
    std::vector<fds::Pending> take;
    bool mid_flight = false;
    {
      std::unique_lock<std::mutex> lk(mu);
      cv.wait(lk, [&] { return stop || !g->running.empty() || admissible_locked(g); });
      if (stop && g->running.empty() && !has_queued_locked(g)) return;
      // the group's queued requests in arrival order, while slots are free
      // and the footprint fits (the first that does not fit blocks the rest,
      // so that a large request is not starved)
      mid_flight = running > 0;
      for (auto it = queue.begin(); it != queue.end() && running < max_slots;) {
        if (fds::key_of(it->req.plan) != g->key) {
          ++it;
          continue;
        }
        if (used + it->bytes > budget && running > 0) break;
        used += it->bytes;
        ++running;
        state[it->ticket] = 1;
        take.push_back(*it);
        it = queue.erase(it);
      }
    }
    double t_admit = 0, t_launch = 0, t_wait = 0, t_retire = 0;
    if (!take.empty()) {
      const auto t0 = Clock::now();
      std::vector<fds::SolveRequest> reqs;
      std::vector<int> ids;
      std::vector<hipEvent_t> evs;
      for (const fds::Pending& p : take) {
        reqs.push_back(p.req);
        ids.push_back(g->next_id++);
        evs.push_back(p.ready);
      }
      try {
        if (!g->stream) FDS_HIP(hipStreamCreateWithFlags(&g->stream, hipStreamNonBlocking));
        if (!g->eng) {
          g->eng.reset(new fds::Engine(std::get<0>(g->key), std::get<1>(g->key), std::get<2>(g->key),
                                       max_slots, g->stream, std::get<3>(g->key)));
          // the set changes at most cycle boundaries under continuous
          // batching: cycles are launched kernel by kernel
          g->eng->set_graphs(false);
        }
        g->eng->admit(reqs, ids, evs);
        for (size_t i = 0; i < ids.size(); ++i) g->running[ids[i]] = take[i];
        std::lock_guard<std::mutex> lk(mu);
        stats.admitted += ids.size();
        if (mid_flight) stats.admitted_mid_flight += ids.size();
        stats.bytes_in_use = used;
        stats.peak_bytes_in_use = std::max<uint64_t>(stats.peak_bytes_in_use, used);
      } catch (const fds::Error& e) {
        {
          fds_result r{};
          r.status = e.status;
          std::lock_guard<std::mutex> lk(mu);
          for (size_t i = 0; i < take.size(); ++i) {
            if (g->running.count(ids[i])) continue;   // failed with the group below
            publish_locked(take[i], r);
            used -= take[i].bytes;
            --running;
          }
        }
        fail_group(g, e.status);
        continue;
      }
      t_admit = fds::seconds_since(t0);
    }
    if (g->running.empty()) continue;
    std::vector<std::pair<int, fds::SolveOutcome>> retired;
    bool cycled = false;
    try {
      auto t0 = Clock::now();
      cycled = g->eng->cycle_launch();
      t_launch = fds::seconds_since(t0);
      if (cycled) {
        t0 = Clock::now();
        g->eng->cycle_finish();
        t_wait = fds::seconds_since(t0);
      }
      const std::vector<int> fin = g->eng->finished_ids();
      if (!fin.empty()) {
        t0 = Clock::now();
        retired = g->eng->retire(fin);
        t_retire = fds::seconds_since(t0);
      }
    } catch (const fds::Error& e) {
      fail_group(g, e.status);
      continue;
    }
    std::lock_guard<std::mutex> lk(mu);
    for (auto& pr : retired) {
      auto it = g->running.find(pr.first);
      if (it == g->running.end()) continue;
      publish_locked(it->second, pr.second.res);
      used -= it->second.bytes;
      --running;
      g->running.erase(it);
    }
    if (cycled) stats.cycles += 1;
    stats.bytes_in_use = used;
    stats.host_admit_s += t_admit;
    stats.host_retire_s += t_retire;
    stats.host_launch_s += t_launch;
    stats.host_wait_s += t_wait;
    const double tasks = g->eng->host_task_seconds();
    stats.host_tasks_s += tasks - g->tasks_seen;
    g->tasks_seen = tasks;
    if (!retired.empty()) cv.notify_all();   // memory and slots were freed
  }
}

namespace fds {

fds_server* server_create(size_t budget, int max_slots) {
  if (budget == 0 || max_slots < 1) throw Error(FDS_E_INVALID_ARG, "bad server limits");
  auto* s = new fds_server();
  s->budget = budget;
  s->max_slots = max_slots;
  FDS_HIP(hipGetDevice(&s->device));
  return s;
}

void server_destroy(fds_server* s) {
  if (!s) return;
  std::vector<fds_server::Group*> gs;
  {
    std::lock_guard<std::mutex> lk(s->mu);
    s->stop = true;
    for (auto& kv : s->groups) gs.push_back(kv.second.get());
  }
  s->cv.notify_all();
  // every group thread drains its queued and running requests, then exits
  for (auto* g : gs)
    if (g->th.joinable()) g->th.join();
  for (auto* g : gs) {
    g->eng.reset();
    if (g->stream) (void)hipStreamDestroy(g->stream);
  }
  s->groups.clear();
  for (hipEvent_t e : s->event_pool) (void)hipEventDestroy(e);
  for (auto& p : s->queue)
    if (p.ready) (void)hipEventDestroy(p.ready);
  delete s;
}

fds_status server_submit(fds_server* s, fds_plan* plan, const double* rhs, const double* bc,
                         double* x, double tol, hipStream_t stream, uint64_t* ticket) {
  if (!s || !plan || !rhs || !x || !ticket || !(tol >= 0.0)) throw Error(FDS_E_INVALID_ARG, "bad submit arguments");
  const size_t bytes = Engine::bytes_per_problem(plan, plan->opt.restart_m, plan->opt.precision);
  if (bytes > s->budget) throw Error(FDS_E_NOMEM, "request footprint exceeds the server budget");
  hipEvent_t ev = s->take_event();
  const hipError_t e = hipEventRecord(ev, stream);
  if (e != hipSuccess) {
    std::lock_guard<std::mutex> lk(s->mu);
    s->event_pool.push_back(ev);
    FDS_HIP(e);
  }
  std::lock_guard<std::mutex> lk(s->mu);
  if (s->stop) {
    s->event_pool.push_back(ev);
    throw Error(FDS_E_INVALID_ARG, "server is shutting down");
  }
  const uint64_t t = s->next_ticket++;
  s->queue.push_back(Pending{t, SolveRequest{plan, rhs, bc, x, tol}, bytes, Clock::now(), ev});
  s->state[t] = 0;
  s->stats.submitted += 1;
  *ticket = t;
  // the request's group, with its thread, on first use
  const Key k = key_of(plan);
  auto& slot = s->groups[k];
  if (!slot) {
    slot.reset(new fds_server::Group());
    slot->key = k;
    fds_server::Group* g = slot.get();
    g->th = std::thread([s, g] { s->group_loop(g); });
  }
  s->cv.notify_all();
  return FDS_OK;
}

fds_status server_poll(fds_server* s, uint64_t ticket, fds_result* res) {
  if (!s) throw Error(FDS_E_INVALID_ARG, "server is NULL");
  std::lock_guard<std::mutex> lk(s->mu);
  auto it = s->state.find(ticket);
  if (it == s->state.end()) throw Error(FDS_E_INVALID_ARG, "unknown ticket");
  if (it->second != 2) return FDS_PENDING;
  fds_result r = s->done[ticket];
  s->done.erase(ticket);
  s->state.erase(it);
  if (res) *res = r;
  return (fds_status)r.status;
}

fds_status server_wait_any(fds_server* s, int64_t timeout_us, uint64_t* ticket, fds_result* res) {
  if (!s || !ticket) throw Error(FDS_E_INVALID_ARG, "NULL argument");
  std::unique_lock<std::mutex> lk(s->mu);
  auto ready = [&] { return !s->done.empty(); };
  if (timeout_us < 0) {
    s->done_cv.wait(lk, ready);
  } else if (!s->done_cv.wait_for(lk, std::chrono::microseconds(timeout_us), ready)) {
    return FDS_PENDING;
  }
  auto it = s->done.begin();
  const uint64_t t = it->first;
  const fds_result r = it->second;
  s->done.erase(it);
  s->state.erase(t);
  *ticket = t;
  if (res) *res = r;
  return (fds_status)r.status;
}

void server_stats(fds_server* s, fds_server_stats* out) {
  if (!s || !out) throw Error(FDS_E_INVALID_ARG, "NULL argument");
  std::lock_guard<std::mutex> lk(s->mu);
  fds_server_stats st = s->stats;
  int q = 0, r = 0;
  for (auto& kv : s->state) {
    if (kv.second == 0) ++q;
    if (kv.second == 1) ++r;
  }
  st.queued = q;
  st.running = r;
  *out = st;
}

}  // namespace fds
