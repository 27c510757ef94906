// Host runtime: device buffers, shared tables, plans and the batched engine.
#pragma once

#include <map>
#include <memory>
#include <mutex>
#include <tuple>
#include <vector>

#include "fds_internal.h"
#include "kernels.h"

namespace fds {

// ---------------------------------------------------------------- device buffer
// Device memory cache (alloc.cpp): blocks are kept per device and size class
// after release and handed out again, so repeated solves allocate nothing
// from the runtime.  Cached bytes above FDS_CACHE_BYTES (default 64 GiB) are
// returned to the runtime.
void* device_cache_alloc(size_t bytes, size_t* capacity);
void device_cache_free(void* p, size_t capacity);
// Mapped, coherent host memory (flags the kernels write), cached the same way.
void* host_mapped_alloc(size_t bytes, void** device_ptr);
void host_mapped_free(void* p, size_t bytes);

class DevBuf {
 public:
  DevBuf() = default;
  explicit DevBuf(size_t bytes) { alloc(bytes); }
  ~DevBuf() { release(); }
  DevBuf(const DevBuf&) = delete;
  DevBuf& operator=(const DevBuf&) = delete;
  DevBuf(DevBuf&& o) noexcept : p_(o.p_), n_(o.n_), cap_(o.cap_) { o.p_ = nullptr; o.n_ = 0; o.cap_ = 0; }
  DevBuf& operator=(DevBuf&& o) noexcept {
    if (this != &o) {
      release();
      p_ = o.p_; n_ = o.n_; cap_ = o.cap_;
      o.p_ = nullptr; o.n_ = 0; o.cap_ = 0;
    }
    return *this;
  }
  void alloc(size_t bytes) {
    release();
    if (bytes) p_ = device_cache_alloc(bytes, &cap_);
    n_ = bytes;
  }
  // The caller guarantees that no queued work still uses the memory (every
  // release in this library follows a synchronisation of the stream that
  // used it).
  void release() {
    if (p_) device_cache_free(p_, cap_);
    p_ = nullptr;
    n_ = 0;
    cap_ = 0;
  }
  template <typename T> T* as(size_t byte_off = 0) const {
    return reinterpret_cast<T*>(static_cast<char*>(p_) + byte_off);
  }
  void* get() const { return p_; }
  size_t size() const { return n_; }

 private:
  void* p_ = nullptr;
  size_t n_ = 0;
  size_t cap_ = 0;
};

// ---------------------------------------------------------------- shared tables
struct FftTable {           // one transform length
  DevBuf mem;
  FftDesc host;             // with device pointers filled in
  const FftDesc* dev;       // device copy of `host`
  WaveDesc wave64, wave32;  // wave-parallel transform descriptors
};

struct ModeTable {          // per-mode tridiagonal coefficients, FP64 and FP32
  DevBuf mem;
  const ModeCoef<double>* c64;
  const ModeCoef<float>* c32;
};

struct GsTable {            // Schur line coefficients delta^2 (2/N) g_k
  DevBuf mem;
  const double* gs;
  // Dense line operator for n <= kDenseLineMax (else null), n x n FP64,
  // element (k, i) at k n + i: delta^2 (2/N) S diag(g) S (symmetric),
  // applied to a line of z
  const double* mfull = nullptr;
};
constexpr int kDenseLineMax = 1024;
// Dense line operators in use (n <= kDenseLineMax unless FDS_LINES=fft).
bool dense_lines(int n);

// Process-wide cache of device tables (per device), keyed by length and by
// (length, rows, h, kappa).  Transform tables live until process exit.
class TableCache {
 public:
  static TableCache& get();
  std::shared_ptr<FftTable> fft(int n);
  // unit: solve T_k y = r exactly (coefficients in the orthonormal sine
  // basis); otherwise the DST normalisation 2/(n+1) is folded in.
  std::shared_ptr<ModeTable> modes(int n, int m, double h, double kappa, bool unit = false);
  // dense: also form the n x n line operator (n <= kDenseLineMax)
  std::shared_ptr<GsTable> gs(int n, int m, double h, double kappa, bool dense = true);
  // wave-transform descriptor of the table whose device FftDesc is `dev`
  WaveDesc wave_desc(const FftDesc* dev, bool fp32);

 private:
  std::mutex mu_;
  std::map<std::pair<int, int>, std::shared_ptr<FftTable>> fft_;
  std::map<const FftDesc*, std::shared_ptr<FftTable>> by_dev_;
  // kappa-dependent tables are held by the plans that use them: the cache
  // only finds a live one again, so a stream of requests with continuous
  // kappa does not keep every table ever built (their memory returns to the
  // device-memory cache when the last plan using them is destroyed)
  std::map<std::tuple<int, int, int, double, double, bool>, std::weak_ptr<ModeTable>> modes_;
  std::map<std::tuple<int, int, int, double, double, bool>, std::weak_ptr<GsTable>> gs_;
};

// Tables of the interface Krylov iteration for an nx x ny centre (IkTask):
// eigenvalues along each axis, the orthonormal sine vectors' first-node
// values, and the corner entries of the per-mode tridiagonal inverses.
struct IkPlanTable {
  DevBuf mem;
  const double *lamx, *lamy, *qx, *qy, *t00, *t0n, *s00, *s0n;
};
std::shared_ptr<IkPlanTable> build_ik_table(int nx, int ny, double h, double kappa);
// Host copy of the Schur line coefficients delta^2 (2/N) g_k of an arm.
std::vector<double> schur_gs_host(int n, int m, double h, double kappa);
struct DiagTable {           // reciprocal of a diagonal preconditioner, centre layout
  DevBuf mem;
  const double* dinv = nullptr;
};

// Per-mode coefficients for `n` modes of an m-row tridiagonal system whose
// right-hand side is multiplied by `scale`.
void mode_coefs_host(int n, int m, double h, double kappa, double scale,
                     std::vector<ModeCoef<double>>& c64, std::vector<ModeCoef<float>>& c32);
std::shared_ptr<ModeTable> upload_modes(const std::vector<ModeCoef<double>>& c64,
                                        const std::vector<ModeCoef<float>>& c32);

// Radix schedule of a complex FFT of length N (16s, then one of 8/4/2, 3s,
// 5s, then other primes ascending).
std::vector<int> fft_radices(int N);
// True when every radix of the schedule of L has a register butterfly.
bool fixed_radices(int L);
// Algorithm for the length-(n+1) FFT behind a DST-I of length n: kind, the
// Stockham length L it runs, and the LDS entries per buffer.
struct FftShape { int kind; int L; int lds_len; };
FftShape fft_shape(int n);
// Schedule of the wave-parallel transform (fft_shape when it has register
// butterflies only, else a Rader or Bluestein schedule that has).
FftShape wave_shape(int n);
// Threads per row for the workgroup-wide transform of length n (power of
// two, 32..256).
int dst_threads_per_row(int n);
size_t dst_smem_bytes(int n, bool fp32);
bool dst_twiddles_in_lds(int n, bool fp32);
size_t line_smem_bytes(int n);
// Wave-parallel row transform: lanes per row G, register budget E (complex
// entries per lane and pass), wavefronts per workgroup, LDS bytes.  E == 0
// when the length needs a radix without a register butterfly or more
// registers than allowed.
struct WaveCfg { int E; int G; int waves; int rows_per_block; size_t smem; };
// big: one row per workgroup of 128/256/512 lanes, tables read from global memory.
WaveCfg dst_wave_config(int n, bool fp32, bool big);
// Lanes per row of the wave transform of length n, and its radix schedule
// for an inner FFT of length L (empty when L has a prime factor above 5).
int wave_lanes(int n);
std::vector<int> wave_radices(int L, int G);
// Row sine transform algorithm for length n: the wave-parallel LDS FFT
// (default where WaveCfg allows), the workgroup-wide LDS FFT, or the dense
// sine matrix on the matrix cores (n <= 1024).  FDS_DST_ALGO=wave|fft|gemm|auto
// selects it for measurements.
struct DstChoice {
  bool gemm;
  int rt;
  int ct;
  int rows_per_block;
  size_t smem;
  int wave_e;    // > 0: wave-parallel kernel with this register budget
  int threads;   // workgroup size
  int wave_big;  // wave kernel with one row per workgroup
};
DstChoice dst_choice(int n, bool fp32);
// One variant ("wave": the wave FFT where its schedule allows, a row per
// wavefront if possible, else the workgroup FFT; "wavebig": the wave FFT with
// a row per workgroup, else the workgroup FFT; "fft": the workgroup FFT;
// "gemm": the matrix-core product for n <= 512, else as "wave").
DstChoice dst_choice_variant(int n, bool fp32, const std::string& mode);
// Autotuner (tune.cpp): on the first request for (device, n, precision) every
// variant runs on a batch of synthetic rows and the fastest is kept.
DstChoice dst_tuned_choice(int n, bool fp32);
// One launch of the row transform of a single task record (copied to `keep`).
void launch_one_dst(DstKind kind, const DstChoice& ch, const DstTask& t0, hipStream_t s,
                    DevBuf& keep);

// ---------------------------------------------------------------- plan
enum RectKind { RK_CENTRE = 0, RK_N = 1, RK_S = 2, RK_E = 3, RK_W = 4 };
// centre boundary line fed by an arm: 0 S (row 0), 1 N (row ny-1), 2 W (col 0), 3 E (col nx-1)
int line_of_kind(int kind);

struct ArmInfo {
  int rect;                  // index in plan order
  int kind;
  int line;                  // centre line id
  int L;                     // line length (= arm cols)
  int rows;                  // arm rows (Thomas length, interface row first)
  std::shared_ptr<FftTable> fft;
  std::shared_ptr<ModeTable> modes;
  std::shared_ptr<GsTable> gs;
};

}  // namespace fds

struct fds_plan {
  int device = 0;
  std::vector<fds_rect> rects;
  std::vector<fds::RectDev> rd;      // per rect (user order); off relative to a problem
  std::vector<int> kind;
  fds::RectDev cdev{};               // the coupled block as one rectangle (offset 0)
  std::vector<fds::ArmInfo> arms;
  double h = 0, delta = 0, kappa = 0;
  fds_options opt{};
  int nx = 0, ny = 0;
  long long n_unknowns = 0, bc_total = 0, n_internal = 0;
  std::vector<long long> user_off, bc_off;
  std::shared_ptr<fds::FftTable> fft_c;
  std::shared_ptr<fds::ModeTable> modes_c;
  std::shared_ptr<fds::ModeTable> modes_cu;   // centre, unit scale (flexible variant)
  std::shared_ptr<fds::IkPlanTable> ik;       // interface Krylov iteration (or null)
  std::shared_ptr<fds::DiagTable> jacobi;     // FDS_JACOBI: 1/diag(L_c) (or null)
  double floor_coef = 0;
  bool interface_krylov() const { return (opt.flags & FDS_FLAG_INTERFACE_KRYLOV) != 0; }
  size_t footprint(int m, int precision) const;
};

namespace fds {

fds_plan* create_plan(const fds_rect* rects, int nrect, double h, double kappa,
                      const fds_options* opt);
// 1 / diag(L_c) of a plan (Jacobi preconditioner).
std::shared_ptr<DiagTable> build_jacobi_table(const fds_plan* p);

// ---------------------------------------------------------------- engine
struct SolveRequest {
  fds_plan* plan;
  const double* rhs;
  const double* bc;
  double* x;
  double tol;
};

struct SolveOutcome {
  fds_status status;
  fds_result res;
};

// Batched right-preconditioned GMRES(m) / FGMRES(m): every kernel of an
// Arnoldi step serves all running problems of the engine in one launch.
// Problems are admitted (set-up phase: lift, arm pre-solves, f', initial
// residual) and retired (back substitution, output, global residual) between
// cycles, which is what the request server uses for continuous batching.
class Engine {
 public:
  // capacity: most problems held at once (state pool and flag array size).
  Engine(int m, int precision, int max_cycles, int capacity, hipStream_t stream, uint32_t flags = 0);
  ~Engine();
  // Allocates the problems and runs their set-up phase (blocks until done).
  // wait_events (may be empty, else one per request, entries may be null):
  // the set-up reads the request's inputs only after the event completed.
  void admit(const std::vector<SolveRequest>& reqs, const std::vector<int>& ids,
             const std::vector<hipEvent_t>& wait_events = {});
  // One GMRES cycle of every unfinished problem; false once none is running.
  bool step_cycle();
  // The same cycle in three parts, so that the host can queue the cycles of
  // several engines (on their own streams) before waiting for any of them:
  // cycle_launch() queues the cycle (false: nothing to run), cycle_finish()
  // waits for it and returns whether a problem is still running.
  bool cycle_launch();
  bool cycle_finish();
  // Cycles of a fixed set of problems (from the second cycle on the same
  // set) are replayed from one captured HIP graph instead of being launched
  // kernel by kernel.  Off by default; FDS_GRAPH=1 turns it on.
  void set_graphs(bool on);
  int graph_replays() const;
  // Host seconds spent rebuilding task lists after the set changed.
  double host_task_seconds() const;
  // Problems that finished (converged, stalled, failed or out of cycles).
  std::vector<int> finished_ids() const;
  // Back substitution and output of the given problems; frees their memory.
  std::vector<std::pair<int, SolveOutcome>> retire(const std::vector<int>& ids);
  int free_slots() const;
  int active() const;
  static size_t bytes_per_problem(const fds_plan* p, int m, int precision);
  // Whole batch: admit all, cycle until done, retire all (request order).
  static std::vector<SolveOutcome> run_batch(const std::vector<SolveRequest>& reqs, int m,
                                             int precision, int max_cycles, hipStream_t stream,
                                             uint32_t flags = 0);

 private:
  struct Impl;
  std::unique_ptr<Impl> impl_;
};

// Process-wide timing by kernel class (see fds_timing_*).

}  // namespace fds
