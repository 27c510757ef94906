// Request server.  A host thread owns one HIP stream and a running batch
// engine; between GMRES cycles it retires finished requests and admits
// queued ones while their device footprint fits the budget and a slot is
// free.
#include "server.h"

#include <chrono>
#include <condition_variable>
#include <deque>
#include <map>
#include <mutex>
#include <thread>

namespace fds {

struct Pending {
  uint64_t ticket;
  SolveRequest req;
  size_t bytes;
};

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
  void run();
};

void fds_server::run() {
  (void)hipSetDevice(device);
  while (true) {
    std::vector<fds::Pending> batch;
    {
      std::unique_lock<std::mutex> lk(mu);
      cv.wait(lk, [&] { return stop || !queue.empty(); });
      if (stop && queue.empty()) return;
      size_t used = 0;
      const int m = queue.front().req.plan->opt.restart_m;
      const int prec = queue.front().req.plan->opt.precision;
      while (!queue.empty() && (int)batch.size() < max_slots) {
        const fds::Pending& p = queue.front();
        if (p.req.plan->opt.restart_m != m || p.req.plan->opt.precision != prec) break;
        if (!batch.empty() && used + p.bytes > budget) break;
        used += p.bytes;
        batch.push_back(p);
        state[p.ticket] = 1;
        queue.pop_front();
      }
    }
    std::vector<fds::SolveRequest> reqs;
    int max_cycles = 1;
    for (auto& p : batch) {
      reqs.push_back(p.req);
      max_cycles = std::max(max_cycles, p.req.plan->opt.max_cycles);
    }
    std::vector<fds::SolveOutcome> out;
    fds_status err = FDS_OK;
    try {
      fds::Engine eng(reqs, reqs[0].plan->opt.restart_m, reqs[0].plan->opt.precision, max_cycles, stream);
      out = eng.run();
    } catch (const fds::Error& e) {
      err = e.status;
    } catch (...) {
      err = FDS_E_DEVICE;
    }
    std::lock_guard<std::mutex> lk(mu);
    for (size_t i = 0; i < batch.size(); ++i) {
      fds_result r{};
      if (err != FDS_OK) r.status = err;
      else r = out[i].res;
      done[batch[i].ticket] = r;
      state[batch[i].ticket] = 2;
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
  s->queue.push_back(Pending{t, SolveRequest{plan, rhs, bc, x, tol}, bytes});
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
