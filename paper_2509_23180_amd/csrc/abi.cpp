// C ABI of the library (include/fds.h).  Converts exceptions into status
// codes and keeps a thread-local message for fds_last_error().
#include <algorithm>
#include <cmath>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "runtime.h"
#include "server.h"

using namespace fds;

namespace {

thread_local std::string g_last_error;

fds_status fail(fds_status s, const std::string& msg) {
  g_last_error = msg;
  return s;
}

template <typename F>
fds_status guarded(F&& f) {
  try {
    g_last_error.clear();
    return f();
  } catch (const Error& e) {
    return fail(e.status, e.what());
  } catch (const std::bad_alloc&) {
    return fail(FDS_E_NOMEM, "host allocation failed");
  } catch (const std::exception& e) {
    return fail(FDS_E_DEVICE, e.what());
  }
}

hipStream_t as_stream(void* s) { return reinterpret_cast<hipStream_t>(s); }

// ---------------------------------------------------------------- timing
struct TimingState {
  std::mutex mu;
  int mask = 0;
  static constexpr int kClasses = 8;
  double bytes[kClasses] = {};
  struct Pending { int cls; hipEvent_t a, b; };
  std::vector<Pending> pending;
  std::vector<hipEvent_t> pool;
  hipEvent_t open[kClasses] = {};
  long long calls[kClasses] = {};
  double ms[kClasses] = {};

  hipEvent_t take() {
    if (!pool.empty()) { hipEvent_t e = pool.back(); pool.pop_back(); return e; }
    hipEvent_t e;
    FDS_HIP(hipEventCreate(&e));
    return e;
  }
  void flush() {
    for (const Pending& p : pending) {
      FDS_HIP(hipEventSynchronize(p.b));
      float t = 0;
      FDS_HIP(hipEventElapsedTime(&t, p.a, p.b));
      calls[p.cls] += 1;
      ms[p.cls] += t;
      pool.push_back(p.a);
      pool.push_back(p.b);
    }
    pending.clear();
  }
};

TimingState& timing() {
  static TimingState t;
  return t;
}

// The class open on this thread (launches of several threads, e.g. the
// server's groups, are attributed to their own thread's class).
thread_local int t_armed = -1;

}  // namespace

namespace fds {

void Timing::enable(int mask) {
  std::lock_guard<std::mutex> lk(timing().mu);
  timing().mask = mask;
}
bool Timing::on() { return timing().mask != 0; }
bool Timing::on(int cls) { return (timing().mask >> cls) & 1; }
void Timing::add_bytes(int cls, double b) {
  TimingState& t = timing();
  std::lock_guard<std::mutex> lk(t.mu);
  t.bytes[cls] += b;
}
double Timing::bytes(int cls) {
  TimingState& t = timing();
  std::lock_guard<std::mutex> lk(t.mu);
  return t.bytes[cls];
}
void Timing::begin(int cls, hipStream_t) {
  TimingState& t = timing();
  if (!((t.mask >> cls) & 1)) return;
  t_armed = cls;
}
void Timing::end(int cls, hipStream_t) {
  if (t_armed == cls) t_armed = -1;
}
// A pair handed out here is recorded by the caller's launch after the lock
// is released, so pairs are read back (and their events reused) only by
// read() and reset(), which must not overlap timed launches.
bool Timing::take_pair(hipEvent_t* a, hipEvent_t* b) {
  if (t_armed < 0) return false;
  TimingState& t = timing();
  std::lock_guard<std::mutex> lk(t.mu);
  *a = t.take();
  *b = t.take();
  t.pending.push_back({t_armed, *a, *b});
  return true;
}
void Timing::read(int cls, long long* calls, double* ms) {
  TimingState& t = timing();
  std::lock_guard<std::mutex> lk(t.mu);
  t.flush();
  *calls = t.calls[cls];
  *ms = t.ms[cls];
}
void Timing::reset() {
  TimingState& t = timing();
  std::lock_guard<std::mutex> lk(t.mu);
  t.flush();
  for (int i = 0; i < TimingState::kClasses; ++i) { t.calls[i] = 0; t.ms[i] = 0; t.bytes[i] = 0; }
}

}  // namespace fds

extern "C" {

const char* fds_status_str(fds_status s) {
  switch (s) {
    case FDS_OK: return "ok";
    case FDS_PENDING: return "pending";
    case FDS_E_INVALID_ARG: return "invalid argument";
    case FDS_E_GEOMETRY: return "unsupported geometry";
    case FDS_E_UNSUPPORTED: return "unsupported";
    case FDS_E_SINGULAR: return "singular subdomain operator";
    case FDS_E_NOMEM: return "out of memory";
    case FDS_E_NOT_CONVERGED: return "not converged";
    case FDS_E_NONFINITE: return "non-finite input";
    case FDS_E_DEVICE: return "device error";
    case FDS_E_UNSUPPORTED_BC: return "unsupported boundary-condition kind";
  }
  return "unknown status";
}

const char* fds_last_error(void) { return g_last_error.c_str(); }

// Boundary-condition kinds of the plan: every outer edge must be Dirichlet
// (the sine transforms); Neumann and periodic edges are recognised and
// refused with their own status.  Shared (interface) edges carry no kind.
static void check_bc(const fds_rect* rects, int32_t nrect, const fds_bc* bc) {
  if (!bc) return;
  auto check_kind = [](int32_t k) {
    if (k == FDS_BC_DIRICHLET) return;
    if (k == FDS_BC_NEUMANN || k == FDS_BC_PERIODIC)
      throw Error(FDS_E_UNSUPPORTED_BC, k == FDS_BC_NEUMANN ? "Neumann edges are not supported (Dirichlet only)"
                                                            : "periodic edges are not supported (Dirichlet only)");
    throw Error(FDS_E_INVALID_ARG, "unknown boundary-condition kind " + std::to_string(k));
  };
  if (!bc->edge_kinds) {
    check_kind(bc->kind);
    return;
  }
  if (!rects || nrect < 1) return;   // the geometry check reports it
  for (int32_t r = 0; r < nrect; ++r)
    for (int side = 0; side < 4; ++side) {
      const int32_t k = bc->edge_kinds[4 * r + side];
      if (k == FDS_BC_DIRICHLET) continue;
      const fds_rect& a = rects[r];
      bool shared = false;
      for (int32_t q = 0; q < nrect && !shared; ++q) {
        if (q == r) continue;
        const fds_rect& b = rects[q];
        switch (side) {
          case 0: shared = b.j1 == a.j0 && b.i0 == a.i0 && b.i1 == a.i1; break;
          case 1: shared = b.i0 == a.i1 && b.j0 == a.j0 && b.j1 == a.j1; break;
          case 2: shared = b.j0 == a.j1 && b.i0 == a.i0 && b.i1 == a.i1; break;
          case 3: shared = b.i1 == a.i0 && b.j0 == a.j0 && b.j1 == a.j1; break;
        }
      }
      if (!shared) check_kind(k);
    }
}

fds_status fds_plan_create(const fds_rect* rects, int32_t nrect, double h, double kappa,
                           const fds_bc* bc, const fds_options* opt, fds_plan** out) {
  return guarded([&] {
    if (!out) throw Error(FDS_E_INVALID_ARG, "out is NULL");
    *out = nullptr;
    check_bc(rects, nrect, bc);
    *out = create_plan(rects, nrect, h, kappa, opt);
    return FDS_OK;
  });
}

void fds_plan_destroy(fds_plan* plan) { delete plan; }

fds_status fds_plan_layout(const fds_plan* plan, int64_t* unknown_offsets, int64_t* bc_offsets) {
  return guarded([&] {
    if (!plan) throw Error(FDS_E_INVALID_ARG, "plan is NULL");
    const size_t n = plan->rects.size();
    for (size_t i = 0; i <= n; ++i) {
      if (unknown_offsets) unknown_offsets[i] = plan->user_off[i];
      if (bc_offsets) bc_offsets[i] = plan->bc_off[i];
    }
    return FDS_OK;
  });
}

fds_status fds_plan_footprint(const fds_plan* plan, size_t* bytes) {
  return guarded([&] {
    if (!plan || !bytes) throw Error(FDS_E_INVALID_ARG, "NULL argument");
    *bytes = plan->footprint(plan->opt.restart_m, plan->opt.precision);
    return FDS_OK;
  });
}

fds_status fds_solve_batch(fds_plan* const* plans, int32_t count, const double* const* rhs,
                           const double* const* bc, double* const* x, const double* tol,
                           void* stream, fds_result* res) {
  return guarded([&] {
    if (count < 1 || !plans || !rhs || !x || !tol) throw Error(FDS_E_INVALID_ARG, "bad batch arguments");
    std::vector<SolveRequest> reqs(count);
    const int m = plans[0] ? plans[0]->opt.restart_m : 0;
    const int prec = plans[0] ? plans[0]->opt.precision : 0;
    const uint32_t flags = plans[0] ? plans[0]->opt.flags : 0;
    int max_cycles = 1;
    for (int i = 0; i < count; ++i) {
      if (!plans[i] || !rhs[i] || !x[i]) throw Error(FDS_E_INVALID_ARG, "NULL plan/rhs/x in batch");
      if (plans[i]->opt.restart_m != m || plans[i]->opt.precision != prec)
        throw Error(FDS_E_INVALID_ARG, "batched plans must share restart_m and precision");
      if (plans[i]->opt.flags != flags)
        throw Error(FDS_E_INVALID_ARG, "batched plans must share the Krylov iteration (option flags)");
      if (!(tol[i] >= 0.0)) throw Error(FDS_E_INVALID_ARG, "tol must be >= 0");
      max_cycles = std::max(max_cycles, plans[i]->opt.max_cycles);
      reqs[i] = SolveRequest{plans[i], rhs[i], bc ? bc[i] : nullptr, x[i], tol[i]};
    }
    std::vector<SolveOutcome> out = Engine::run_batch(reqs, m, prec, max_cycles, as_stream(stream), flags);
    fds_status first = FDS_OK;
    for (int i = 0; i < count; ++i) {
      if (res) res[i] = out[i].res;
      if (first == FDS_OK && out[i].status != FDS_OK) first = out[i].status;
    }
    if (first != FDS_OK) g_last_error = fds_status_str(first);
    return first;
  });
}

fds_status fds_solve(fds_plan* plan, const double* rhs, const double* bc, double* x, double tol,
                     void* stream, fds_result* res) {
  fds_plan* plans[1] = {plan};
  const double* r[1] = {rhs};
  const double* b[1] = {bc};
  double* xx[1] = {x};
  double t[1] = {tol};
  return fds_solve_batch(plans, 1, r, b, xx, t, stream, res);
}

// ---------------------------------------------------------------- kernel-level entry points


static fds_status dst_rows_impl(const void* in, void* out, int rows, int n, double scale,
                                bool fp32, hipStream_t s) {
  if (!in || !out || rows < 0 || n < 1) throw Error(FDS_E_INVALID_ARG, "bad DST arguments");
  if (rows == 0) return FDS_OK;
  auto fft = TableCache::get().fft(n);
  DstTask t{};
  t.in = in; t.out = out; t.in_rs = n; t.out_rs = n; t.in_cs = 1; t.out_cs = 1;
  t.rows = rows; t.n = n; t.scale = scale; t.fft = fft->dev;
  DevBuf keep;
  launch_one_dst(fp32 ? DstKind::F_F : DstKind::D_D, dst_choice(n, fp32), t, s, keep);
  FDS_HIP(hipGetLastError());
  FDS_HIP(hipStreamSynchronize(s));
  return FDS_OK;
}

fds_status fds_k_dst_rows(const double* in, double* out, int32_t rows, int32_t n, double scale,
                          void* stream) {
  return guarded([&] { return dst_rows_impl(in, out, rows, n, scale, false, as_stream(stream)); });
}

fds_status fds_k_dst_rows_f32(const float* in, float* out, int32_t rows, int32_t n, float scale,
                              void* stream) {
  return guarded([&] { return dst_rows_impl(in, out, rows, n, scale, true, as_stream(stream)); });
}

static fds_status tridiag_impl(void* data, int rows, int modes, double h, double kappa,
                               double scale, bool fp32, hipStream_t s) {
  if (!data || rows < 1 || modes < 1 || !(h > 0)) throw Error(FDS_E_INVALID_ARG, "bad tridiag arguments");
  std::vector<ModeCoef<double>> c64;
  std::vector<ModeCoef<float>> c32;
  mode_coefs_host(modes, rows, h, kappa, scale, c64, c32);
  auto tab = upload_modes(c64, c32);
  TriTask t{};
  t.data = data; t.rs = modes; t.rows = rows; t.modes = modes;
  t.coef = fp32 ? (const void*)tab->c32 : (const void*)tab->c64;
  const TriConfig tc = tri_config(fp32, rows);
  DevBuf d(sizeof(TriTask));
  FDS_HIP(hipMemcpyAsync(d.get(), &t, sizeof(t), hipMemcpyHostToDevice, s));
  Timing::begin(1, s);
  launch_tri(tc, fp32, d.as<TriTask>(), 1, tri_blocks(tc, modes), 0, s);
  Timing::end(1, s);
  FDS_HIP(hipGetLastError());
  FDS_HIP(hipStreamSynchronize(s));
  return FDS_OK;
}

fds_status fds_k_tridiag_modes(double* data, int32_t rows, int32_t modes, double h, double kappa,
                               double scale, void* stream) {
  return guarded([&] { return tridiag_impl(data, rows, modes, h, kappa, scale, false, as_stream(stream)); });
}

fds_status fds_k_tridiag_modes_f32(float* data, int32_t rows, int32_t modes, double h,
                                   double kappa, double scale, void* stream) {
  return guarded([&] { return tridiag_impl(data, rows, modes, h, kappa, scale, true, as_stream(stream)); });
}

fds_status fds_k_rect_solve(const double* f, double* z, int32_t rows, int32_t cols, double h,
                            double kappa, int32_t precision, void* stream) {
  return guarded([&] {
    hipStream_t s = as_stream(stream);
    if (!f || !z || rows < 1 || cols < 1 || !(h > 0)) throw Error(FDS_E_INVALID_ARG, "bad rect solve arguments");
    const bool fp32 = precision == FDS_FP32_PRECOND;
    auto fft = TableCache::get().fft(cols);
    auto modes = TableCache::get().modes(cols, rows, h, kappa);
    DevBuf tmp((size_t)rows * cols * (fp32 ? 4 : 8));
    DstTask t{};
    t.in = f; t.out = tmp.get(); t.in_rs = cols; t.out_rs = cols; t.in_cs = 1; t.out_cs = 1;
    t.rows = rows; t.n = cols; t.scale = 1.0; t.fft = fft->dev;
    DstTask v = t;
    v.in = tmp.get(); v.out = z;
    TriTask tt{};
    tt.data = tmp.get(); tt.rs = cols; tt.rows = rows; tt.modes = cols;
    tt.coef = fp32 ? (const void*)modes->c32 : (const void*)modes->c64;
    DevBuf keep1, keep2, keep3(sizeof(TriTask));
    launch_one_dst(fp32 ? DstKind::D_F : DstKind::D_D, dst_choice(cols, fp32), t, s, keep1);
    FDS_HIP(hipMemcpyAsync(keep3.get(), &tt, sizeof(tt), hipMemcpyHostToDevice, s));
    const TriConfig tc = tri_config(fp32, rows);
    launch_tri(tc, fp32, keep3.as<TriTask>(), 1, tri_blocks(tc, cols), 0, s);
    launch_one_dst(fp32 ? DstKind::F_D : DstKind::D_D, dst_choice(cols, fp32), v, s, keep2);
    FDS_HIP(hipGetLastError());
    FDS_HIP(hipStreamSynchronize(s));
    return FDS_OK;
  });
}

fds_status fds_k_centre_operator(const fds_plan* plan, const double* z, double* w, void* stream) {
  return guarded([&] {
    hipStream_t s = as_stream(stream);
    if (!plan || !z || !w) throw Error(FDS_E_INVALID_ARG, "NULL argument");
    const int nx = plan->nx, ny = plan->ny;
    const int Lmax = std::max(nx, ny);
    DevBuf lines(sizeof(double) * 4 * Lmax);
    std::vector<LineTask> lt;
    OpTask ot{};
    ot.z = z; ot.nx = nx; ot.ny = ny; ot.delta = plan->delta; ot.kappa = plan->kappa; ot.out = w;
    ot.nblocks = std::max(1, (int)(((long long)nx * ny + kVecPerBlock - 1) / kVecPerBlock));
    size_t sm = 0;
    for (const ArmInfo& a : plan->arms) {
      LineTask t{};
      t.z = z; t.L = a.L; t.fft = a.fft->dev; t.gs = a.gs->gs;
      t.out = lines.as<double>() + (size_t)a.line * Lmax;
      switch (a.line) {
        case 0: t.start = 0; t.stride = 1; break;
        case 1: t.start = (long long)(ny - 1) * nx; t.stride = 1; break;
        case 2: t.start = 0; t.stride = nx; break;
        case 3: t.start = nx - 1; t.stride = nx; break;
      }
      ot.line[a.line] = t.out;
      sm = std::max(sm, line_smem_bytes(a.L));
      lt.push_back(t);
    }
    DevBuf d(sizeof(OpTask) + sizeof(LineTask) * std::max<size_t>(1, lt.size()));
    FDS_HIP(hipMemcpyAsync(d.get(), &ot, sizeof(ot), hipMemcpyHostToDevice, s));
    if (!lt.empty())
      FDS_HIP(hipMemcpyAsync(d.as<char>(sizeof(OpTask)), lt.data(), sizeof(LineTask) * lt.size(),
                             hipMemcpyHostToDevice, s));
    if (!lt.empty()) {
      Timing::begin(4, s);
      launch_lines(reinterpret_cast<const LineTask*>(d.as<char>(sizeof(OpTask))), (int)lt.size(), sm, 0, s);
      Timing::end(4, s);
    }
    Timing::begin(2, s);
    launch_operator(0, d.as<OpTask>(), 1, ot.nblocks, 0, s);
    Timing::end(2, s);
    FDS_HIP(hipGetLastError());
    FDS_HIP(hipStreamSynchronize(s));
    return FDS_OK;
  });
}

fds_status fds_k_arnoldi_mgs(double* V, int32_t k, int64_t len, double* h, void* stream) {
  return guarded([&] {
    hipStream_t s = as_stream(stream);
    if (!V || !h || k < 1 || len < 1 || k > 120) throw Error(FDS_E_INVALID_ARG, "bad Arnoldi arguments");
    const int m = k;
    const int j = k - 1;
    const int P = (int)((len + kVecPerBlock - 1) / kVecPerBlock);
    const size_t small = (size_t)(m + 1) * m + 4 * (size_t)m + 2;
    const size_t gram = (size_t)(m + 1) * (m + 1) + (m + 1);
    const size_t parts = kry_partials_len(m, P);
    DevBuf mem(8 * (small + gram + parts) + 1024 + 2 * sizeof(KryTask));
    FDS_HIP(hipMemsetAsync(mem.get(), 0, mem.size(), s));
    double* H = mem.as<double>(0);
    double* G = H + small;
    double* partials = G + gram;
    auto* st = reinterpret_cast<ProbState*>(partials + parts);
    ProbState hs{};
    hs.beta = 1.0;
    hs.fnorm = 1.0;
    hs.tol_eff = 0.0;
    hs.vscale = 1.0;
    FDS_HIP(hipMemcpyAsync(st, &hs, sizeof(hs), hipMemcpyHostToDevice, s));
    KryTask t{};
    t.V = V; t.H = H; t.cs = H + (size_t)(m + 1) * m; t.sn = t.cs + m; t.g = t.sn + m; t.y = t.g + m + 1;
    t.partials = partials; t.st = st; t.Nc = len; t.P = P; t.m = m; t.G = G; t.hv = G + (size_t)(m + 1) * (m + 1);
    t.nx = (int)std::min<int64_t>(len, 1 << 30); t.ny = 1;
    KryTask gt = t;   // Gram columns of the existing basis (w implicit, no line terms)
    gt.implicit_w = 1;
    t.implicit_w = 0;
    auto* dt = reinterpret_cast<KryTask*>(reinterpret_cast<char*>(st) + 512);
    FDS_HIP(hipMemcpyAsync(dt, &t, sizeof(t), hipMemcpyHostToDevice, s));
    FDS_HIP(hipMemcpyAsync(dt + 1, &gt, sizeof(gt), hipMemcpyHostToDevice, s));
    for (int c = 0; c < j; ++c) launch_gram_dots(dt + 1, 1, P, c, s);
    Timing::begin(3, s);
    launch_gram_dots(dt, 1, P, j, s);
    Timing::end(3, s);
    Timing::begin(6, s);
    launch_gram_update(dt, 1, P, j, nullptr, 0, s);
    Timing::end(6, s);
    // hv holds h_{0..j, j} (column j of H has the Givens rotations applied)
    FDS_HIP(hipMemcpyAsync(h, t.hv, 8 * (size_t)k, hipMemcpyDeviceToDevice, s));
    launch_scale_newest(dt, j, std::max(1, std::min(P * kVecEPT, 1024)), s);
    FDS_HIP(hipMemcpyAsync(h + k, &st->last_hn, 8, hipMemcpyDeviceToDevice, s));
    FDS_HIP(hipGetLastError());
    FDS_HIP(hipStreamSynchronize(s));
    return FDS_OK;
  });
}

fds_status fds_k_arnoldi_mgs_noalloc(double* V, int32_t k, int64_t len, double* h, void* stream) {
  return guarded([&] {
    hipStream_t s = as_stream(stream);
    if (!V || !h || k < 1 || len < 1 || k > 120) throw Error(FDS_E_INVALID_ARG, "bad Arnoldi arguments");
    const int m = k;
    const int j = k - 1;
    const int P = (int)((len + kVecPerBlock - 1) / kVecPerBlock);
    // the working memory of fds_k_arnoldi_mgs, laid out in the scratch array
    const size_t small = (size_t)(m + 1) * m + 4 * (size_t)m + 2;
    const size_t gram = (size_t)(m + 1) * (m + 1) + (m + 1);
    const size_t parts = kry_partials_len(m, P);
    const size_t n_zero = small + gram + parts;
    const size_t st_off = (8 * n_zero + 255) / 256 * 256;
    const size_t dt_off = st_off + 512;
    const size_t need = dt_off + 2 * sizeof(KryTask);
    if (need > kNoAllocScratchBytes)
      throw Error(FDS_E_NOMEM, "Arnoldi step of k = " + std::to_string(k) + " vectors of length " +
                                   std::to_string(len) + " needs " + std::to_string(need) +
                                   " bytes of working memory; the allocation-free entry point has " +
                                   std::to_string(kNoAllocScratchBytes));
    char* base = static_cast<char*>(noalloc_scratch());
    double* H = reinterpret_cast<double*>(base);
    double* G = H + small;
    double* partials = G + gram;
    auto* st = reinterpret_cast<ProbState*>(base + st_off);
    auto* dt = reinterpret_cast<KryTask*>(base + dt_off);
    ProbState hs{};
    hs.beta = 1.0;
    hs.fnorm = 1.0;
    hs.tol_eff = 0.0;
    hs.vscale = 1.0;
    KryTask t{};
    t.V = V; t.H = H; t.cs = H + (size_t)(m + 1) * m; t.sn = t.cs + m; t.g = t.sn + m; t.y = t.g + m + 1;
    t.partials = partials; t.st = st; t.Nc = len; t.P = P; t.m = m; t.G = G; t.hv = G + (size_t)(m + 1) * (m + 1);
    t.nx = (int)std::min<int64_t>(len, 1 << 30); t.ny = 1;
    KryTask gt = t;   // Gram columns of the existing basis (w implicit, no line terms)
    gt.implicit_w = 1;
    t.implicit_w = 0;
    launch_noalloc_setup(H, (long long)n_zero, st, hs, dt, t, gt, s);
    for (int c = 0; c < j; ++c) launch_gram_dots(dt + 1, 1, P, c, s);
    launch_gram_dots(dt, 1, P, j, s);
    launch_gram_update(dt, 1, P, j, nullptr, 0, s);
    FDS_HIP(hipMemcpyAsync(h, t.hv, 8 * (size_t)k, hipMemcpyDeviceToDevice, s));
    launch_scale_newest(dt, j, std::max(1, std::min(P * kVecEPT, 1024)), s);
    FDS_HIP(hipMemcpyAsync(h + k, &st->last_hn, 8, hipMemcpyDeviceToDevice, s));
    FDS_HIP(hipGetLastError());
    FDS_HIP(hipStreamSynchronize(s));
    return FDS_OK;
  });
}

fds_status fds_timing_enable(int32_t mask) {
  return guarded([&] { Timing::enable(mask); return FDS_OK; });
}

fds_status fds_timing_bytes(int32_t cls, double* algorithmic_bytes) {
  return guarded([&] {
    if (cls < 0 || cls >= TimingState::kClasses || !algorithmic_bytes) throw Error(FDS_E_INVALID_ARG, "bad timing arguments");
    *algorithmic_bytes = Timing::bytes(cls);
    return FDS_OK;
  });
}

fds_status fds_timing_read(int32_t cls, int64_t* calls, double* total_ms) {
  return guarded([&] {
    if (cls < 0 || cls >= TimingState::kClasses || !calls || !total_ms) throw Error(FDS_E_INVALID_ARG, "bad timing arguments");
    long long c = 0;
    double ms = 0;
    Timing::read(cls, &c, &ms);
    *calls = c;
    *total_ms = ms;
    return FDS_OK;
  });
}

fds_status fds_timing_reset(void) {
  return guarded([&] { Timing::reset(); return FDS_OK; });
}

}  // extern "C"

extern "C" {

fds_status fds_server_create(size_t hbm_budget_bytes, int32_t max_slots, fds_server** out) {
  return guarded([&] {
    if (!out) throw Error(FDS_E_INVALID_ARG, "out is NULL");
    *out = server_create(hbm_budget_bytes, max_slots);
    return FDS_OK;
  });
}

void fds_server_destroy(fds_server* server) { server_destroy(server); }

fds_status fds_batch_submit(fds_server* server, fds_plan* plan, const double* rhs,
                            const double* bc, double* x, double tol, void* stream,
                            uint64_t* ticket) {
  return guarded([&] { return server_submit(server, plan, rhs, bc, x, tol, as_stream(stream), ticket); });
}

fds_status fds_server_stats_get(fds_server* server, fds_server_stats* out) {
  return guarded([&] {
    server_stats(server, out);
    return FDS_OK;
  });
}

fds_status fds_batch_poll(fds_server* server, uint64_t ticket, fds_result* res) {
  return guarded([&] { return server_poll(server, ticket, res); });
}

fds_status fds_batch_wait_any(fds_server* server, int64_t timeout_us, uint64_t* ticket, fds_result* res) {
  return guarded([&] { return server_wait_any(server, timeout_us, ticket, res); });
}

}  // extern "C"
