// Request server with continuous batching at GMRES-cycle granularity.
//
// A host thread owns one batch engine, on a HIP stream of its own, per
// (restart length, precision, cycle cap, Krylov iteration).  Between cycles it retires every
// finished problem (back substitution and output, result published to the
// ticket) and admits queued requests in arrival order while their device
// footprint fits the budget and a slot is free; admitted requests run their
// set-up phase and join the next cycle of the running batch.  The cycles of
// all engines are queued before the thread waits for any of them, so groups
// of different precision or restart length overlap on the device.  A
// request's arithmetic does not depend on the other problems in the batch
// (per-problem kernels and reductions), so its result is the same alone and
// in the mix.
#include "server.h"

#include <chrono>
#include <condition_variable>
#include <deque>
#include <map>
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

using Key = std::tuple<int, int, int, unsigned>;   // restart_m, precision, max_cycles, flags

Key key_of(const fds_plan* p) {
  return Key{p->opt.restart_m, p->opt.precision, p->opt.max_cycles, p->opt.flags};
}

struct Group {
  hipStream_t stream = nullptr;
  std::unique_ptr<Engine> eng;
  std::map<int, Pending> running;   // engine id -> request
  bool launched = false;
};

}  // namespace

}  // namespace fds

struct fds_server {
  size_t budget = 0;
  int max_slots = 0;
  int device = 0;
  std::mutex mu;
  std::condition_variable cv;
  std::deque<fds::Pending> queue;
  std::map<uint64_t, fds_result> done;
  std::map<uint64_t, int> state;   // 0 queued, 1 running, 2 done
  uint64_t next_ticket = 1;
  bool stop = false;
  std::thread worker;
  std::vector<hipEvent_t> event_pool;   // guarded by mu
  fds_server_stats stats{};             // guarded by mu
  // worker-thread state
  std::map<fds::Key, fds::Group> groups;
  size_t used = 0;
  int running = 0;
  int next_id = 0;
  double tasks_base = 0;   // task-list seconds of engines already destroyed

  void run();
  void admit_from_queue();
  void publish(const fds::Pending& p, const fds_result& r);
  void fail_group(fds::Group& g, fds_status st);
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

void fds_server::publish(const fds::Pending& p, const fds_result& r0) {
  fds_result r = r0;
  r.seconds = std::chrono::duration<double>(fds::Clock::now() - p.submitted).count();
  std::lock_guard<std::mutex> lk(mu);
  done[p.ticket] = r;
  state[p.ticket] = 2;
  stats.completed += 1;
  // the event's wait was queued before the set-up phase, which has finished
  if (p.ready) event_pool.push_back(p.ready);
}

void fds_server::fail_group(fds::Group& g, fds_status st) {
  fds_result r{};
  r.status = st;
  for (auto& pr : g.running) {
    publish(pr.second, r);
    used -= pr.second.bytes;
    --running;
  }
  g.running.clear();
  if (g.eng) tasks_base += g.eng->host_task_seconds();
  g.eng.reset();   // its state is unknown after a failure
  g.launched = false;
}

// Move queued requests into their engines while the footprint fits the
// budget and slots are free (arrival order; the head of the queue blocks
// the rest so that a large request is not starved).
void fds_server::admit_from_queue() {
  std::map<fds::Key, std::vector<fds::Pending>> take;
  const bool mid_flight = running > 0;   // problems admitted earlier still iterate
  {
    std::lock_guard<std::mutex> lk(mu);
    size_t u = used;
    int r = running;
    while (!queue.empty() && r < max_slots) {
      const fds::Pending& p = queue.front();
      if (u + p.bytes > budget && r > 0) break;
      u += p.bytes;
      ++r;
      state[p.ticket] = 1;
      take[fds::key_of(p.req.plan)].push_back(p);
      queue.pop_front();
    }
  }
  for (auto& kv : take) {
    fds::Group& g = groups[kv.first];
    std::vector<fds::SolveRequest> reqs;
    std::vector<int> ids;
    std::vector<hipEvent_t> evs;
    for (const fds::Pending& p : kv.second) {
      reqs.push_back(p.req);
      ids.push_back(next_id++);
      evs.push_back(p.ready);
    }
    try {
      if (!g.stream) FDS_HIP(hipStreamCreateWithFlags(&g.stream, hipStreamNonBlocking));
      if (!g.eng) {
        g.eng.reset(new fds::Engine(std::get<0>(kv.first), std::get<1>(kv.first), std::get<2>(kv.first),
                                    max_slots, g.stream, std::get<3>(kv.first)));
        // the set changes at most cycle boundaries under continuous batching,
        // so cycles are launched kernel by kernel (no graph capture while
        // the submitting threads build plans)
        g.eng->set_graphs(false);
      }
      g.eng->admit(reqs, ids, evs);
      for (size_t i = 0; i < ids.size(); ++i) {
        g.running[ids[i]] = kv.second[i];
        used += kv.second[i].bytes;
        ++running;
      }
      std::lock_guard<std::mutex> lk(mu);
      stats.admitted += ids.size();
      if (mid_flight) stats.admitted_mid_flight += ids.size();
      stats.bytes_in_use = used;
      stats.peak_bytes_in_use = std::max<uint64_t>(stats.peak_bytes_in_use, used);
    } catch (const fds::Error& e) {
      fds_result r{};
      r.status = e.status;
      for (const fds::Pending& p : kv.second) {
        bool admitted = false;
        for (auto& pr : g.running) admitted |= pr.second.ticket == p.ticket;
        if (!admitted) publish(p, r);
      }
      fail_group(g, e.status);
    }
  }
}

void fds_server::run() {
  (void)hipSetDevice(device);
  using fds::Clock;
  auto secs = [](Clock::time_point a) { return std::chrono::duration<double>(Clock::now() - a).count(); };
  while (true) {
    {
      std::unique_lock<std::mutex> lk(mu);
      cv.wait(lk, [&] { return stop || !queue.empty() || running > 0; });
      if (stop && queue.empty() && running == 0) return;
    }
    double t_admit = 0, t_launch = 0, t_wait = 0, t_retire = 0;
    auto t0 = Clock::now();
    admit_from_queue();
    t_admit = secs(t0);
    // queue one cycle of every group, then wait for each in turn
    for (auto& kv : groups) {
      fds::Group& g = kv.second;
      g.launched = false;
      if (!g.eng || g.running.empty()) continue;
      try {
        t0 = Clock::now();
        g.launched = g.eng->cycle_launch();
        t_launch += secs(t0);
      } catch (const fds::Error& e) {
        fail_group(g, e.status);
      }
    }
    uint64_t cycles = 0;
    for (auto& kv : groups) {
      fds::Group& g = kv.second;
      if (!g.eng || !g.launched) continue;
      try {
        t0 = Clock::now();
        g.eng->cycle_finish();
        t_wait += secs(t0);
        g.launched = false;
        ++cycles;
        const std::vector<int> fin = g.eng->finished_ids();
        if (fin.empty()) continue;
        t0 = Clock::now();
        auto retired = g.eng->retire(fin);
        t_retire += secs(t0);
        for (auto& pr : retired) {
          auto it = g.running.find(pr.first);
          if (it == g.running.end()) continue;
          publish(it->second, pr.second.res);
          used -= it->second.bytes;
          --running;
          g.running.erase(it);
        }
      } catch (const fds::Error& e) {
        fail_group(g, e.status);
      }
    }
    double t_tasks = 0;
    for (auto& kv : groups)
      if (kv.second.eng) t_tasks += kv.second.eng->host_task_seconds();
    std::lock_guard<std::mutex> lk(mu);
    stats.cycles += cycles;
    stats.bytes_in_use = used;
    stats.host_admit_s += t_admit;
    stats.host_retire_s += t_retire;
    stats.host_launch_s += t_launch;
    stats.host_wait_s += t_wait;
    stats.host_tasks_s = tasks_base + t_tasks;
  }
}

namespace fds {

fds_server* server_create(size_t budget, int max_slots) {
  if (budget == 0 || max_slots < 1) throw Error(FDS_E_INVALID_ARG, "bad server limits");
  auto* s = new fds_server();
  s->budget = budget;
  s->max_slots = max_slots;
  FDS_HIP(hipGetDevice(&s->device));
  s->worker = std::thread([s] { s->run(); });
  return s;
}

void server_destroy(fds_server* s) {
  if (!s) return;
  {
    std::lock_guard<std::mutex> lk(s->mu);
    s->stop = true;
  }
  s->cv.notify_all();
  if (s->worker.joinable()) s->worker.join();
  for (auto& kv : s->groups) {
    kv.second.eng.reset();
    if (kv.second.stream) (void)hipStreamDestroy(kv.second.stream);
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
  const uint64_t t = s->next_ticket++;
  s->queue.push_back(Pending{t, SolveRequest{plan, rhs, bc, x, tol}, bytes, Clock::now(), ev});
  s->state[t] = 0;
  s->stats.submitted += 1;
  *ticket = t;
  s->cv.notify_one();
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
