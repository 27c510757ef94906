// Request server with continuous batching at GMRES-cycle granularity.
//
// A host thread owns one HIP stream and one batch engine per (restart length,
// precision, cycle cap).  Between cycles it retires every finished problem
// (back substitution and output, result published to the ticket) and admits
// queued requests in arrival order while their device footprint fits the
// budget and a slot is free; admitted requests run their set-up phase and
// join the next cycle of the running batch.  A request's arithmetic does not
// depend on the other problems in the batch (per-problem kernels and
// reductions), so its result is the same alone and in the mix.
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
};

using Key = std::tuple<int, int, int>;   // restart_m, precision, max_cycles

Key key_of(const fds_plan* p) { return Key{p->opt.restart_m, p->opt.precision, p->opt.max_cycles}; }

struct Group {
  std::unique_ptr<Engine> eng;
  std::map<int, Pending> running;   // engine id -> request
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
  hipStream_t stream = nullptr;
  // worker-thread state
  std::map<fds::Key, fds::Group> groups;
  size_t used = 0;
  int running = 0;
  int next_id = 0;

  void run();
  void admit_from_queue();
  void publish(const fds::Pending& p, const fds_result& r);
};

void fds_server::publish(const fds::Pending& p, const fds_result& r0) {
  fds_result r = r0;
  r.seconds = std::chrono::duration<double>(fds::Clock::now() - p.submitted).count();
  std::lock_guard<std::mutex> lk(mu);
  done[p.ticket] = r;
  state[p.ticket] = 2;
}

// Move queued requests into their engines while the footprint fits the
// budget and slots are free (arrival order; the head of the queue blocks
// the rest so that a large request is not starved).
void fds_server::admit_from_queue() {
  std::map<fds::Key, std::vector<fds::Pending>> take;
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
    if (!g.eng)
      g.eng.reset(new fds::Engine(std::get<0>(kv.first), std::get<1>(kv.first), std::get<2>(kv.first),
                                  max_slots, stream));
    std::vector<fds::SolveRequest> reqs;
    std::vector<int> ids;
    for (const fds::Pending& p : kv.second) {
      reqs.push_back(p.req);
      ids.push_back(next_id++);
    }
    try {
      g.eng->admit(reqs, ids);
      for (size_t i = 0; i < ids.size(); ++i) {
        g.running[ids[i]] = kv.second[i];
        used += kv.second[i].bytes;
        ++running;
      }
    } catch (const fds::Error& e) {
      fds_result r{};
      r.status = e.status;
      for (const fds::Pending& p : kv.second) publish(p, r);
      g.eng.reset();   // its state is unknown after a failed set-up
      for (auto& pr : g.running) publish(pr.second, r);
      for (auto& pr : g.running) { used -= pr.second.bytes; --running; }
      g.running.clear();
    }
  }
}

void fds_server::run() {
  (void)hipSetDevice(device);
  while (true) {
    {
      std::unique_lock<std::mutex> lk(mu);
      cv.wait(lk, [&] { return stop || !queue.empty() || running > 0; });
      if (stop && queue.empty() && running == 0) return;
    }
    admit_from_queue();
    for (auto& kv : groups) {
      fds::Group& g = kv.second;
      if (!g.eng || g.running.empty()) continue;
      try {
        g.eng->step_cycle();
        const std::vector<int> fin = g.eng->finished_ids();
        if (fin.empty()) continue;
        for (auto& pr : g.eng->retire(fin)) {
          auto it = g.running.find(pr.first);
          if (it == g.running.end()) continue;
          publish(it->second, pr.second.res);
          used -= it->second.bytes;
          --running;
          g.running.erase(it);
        }
      } catch (const fds::Error& e) {
        fds_result r{};
        r.status = e.status;
        for (auto& pr : g.running) {
          publish(pr.second, r);
          used -= pr.second.bytes;
          --running;
        }
        g.running.clear();
        g.eng.reset();
      }
    }
  }
}

namespace fds {

fds_server* server_create(size_t budget, int max_slots) {
  if (budget == 0 || max_slots < 1) throw Error(FDS_E_INVALID_ARG, "bad server limits");
  auto* s = new fds_server();
  s->budget = budget;
  s->max_slots = max_slots;
  FDS_HIP(hipGetDevice(&s->device));
  FDS_HIP(hipStreamCreateWithFlags(&s->stream, hipStreamNonBlocking));
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
  s->groups.clear();
  if (s->stream) (void)hipStreamDestroy(s->stream);
  delete s;
}

fds_status server_submit(fds_server* s, fds_plan* plan, const double* rhs, const double* bc,
                         double* x, double tol, uint64_t* ticket) {
  if (!s || !plan || !rhs || !x || !ticket || !(tol >= 0.0)) throw Error(FDS_E_INVALID_ARG, "bad submit arguments");
  const size_t bytes = Engine::bytes_per_problem(plan, plan->opt.restart_m, plan->opt.precision);
  if (bytes > s->budget) throw Error(FDS_E_NOMEM, "request footprint exceeds the server budget");
  std::lock_guard<std::mutex> lk(s->mu);
  const uint64_t t = s->next_ticket++;
  s->queue.push_back(Pending{t, SolveRequest{plan, rhs, bc, x, tol}, bytes, Clock::now()});
  s->state[t] = 0;
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

}  // namespace fds
