// Autotuners for the row sine transform and the segmented tridiagonal solve.
//
// Which implementation of the DST-I is fastest depends on the length (the
// factorisation of n + 1 decides between mixed-radix, Rader and Bluestein
// FFTs and their LDS traffic; short rows favour the dense product on the
// matrix cores) and on the precision.  On the first request for a (device,
// n, precision) each available variant transforms a synthetic batch of rows
// (about 8 MB of data) a few times, timed with HIP events on a private
// stream, and the fastest is kept for the rest of the process.  Plans ask at
// creation time, so a solve never waits for tuning.
//
// FDS_TUNE_FILE names a table of earlier measurements on this kind of device
// ("n precision variant" per line, precision 0 FP64 / 1 FP32, variant
// wave|wavebig|fft|gemm; "tri rows precision mpb ls" for the tridiagonal
// solve): an entry found there is not measured again, and a new measurement
// is appended to the file (when it is writable).  Request
// paths that build plans as requests arrive use it so that a new length does
// not cost a device measurement.
#include <algorithm>
#include <fstream>
#include <cstdio>
#include <cstdlib>
#include <map>
#include <mutex>
#include <string>
#include <tuple>
#include <vector>

#include "runtime.h"

namespace fds {

void launch_one_dst(DstKind kind, const DstChoice& ch, const DstTask& t0, hipStream_t s,
                    DevBuf& keep) {
  const bool fp32 = kind != DstKind::D_D;
  DstTask t = t0;
  t.rpb = ch.gemm ? 1 : ch.rows_per_block;
  t.tw_lds = (ch.gemm || ch.wave_e) ? 0 : (dst_twiddles_in_lds(t.n, fp32) ? 1 : 0);
  if (ch.wave_e) {
    t.wd = TableCache::get().wave_desc(t.fft, fp32);
    t.io_f32 = dst_io_flags(kind);
  }
  t.block_begin = 0;
  keep.alloc(sizeof(DstTask));
  FDS_HIP(hipMemcpyAsync(keep.get(), &t, sizeof(t), hipMemcpyHostToDevice, s));
  const int nb = (t.rows + ch.rows_per_block - 1) / ch.rows_per_block;
  Timing::begin(0, s);
  if (ch.gemm) launch_dst_gemm(kind, ch.rt, ch.ct, keep.as<DstTask>(), 1, nb, ch.smem, 0, s);
  else if (ch.wave_e)
    launch_dst_wave(kind, ch.wave_e, ch.wave_big != 0, keep.as<DstTask>(), 1, nb, ch.threads, ch.smem, 0, s);
  else launch_dst(kind, keep.as<DstTask>(), 1, nb, ch.smem, 0, s);
  Timing::end(0, s);
}

namespace {

bool same(const DstChoice& a, const DstChoice& b) {
  return a.gemm == b.gemm && a.wave_e == b.wave_e && a.wave_big == b.wave_big && a.rt == b.rt && a.ct == b.ct &&
         a.threads == b.threads && a.rows_per_block == b.rows_per_block;
}

// Milliseconds per launch of one variant over `rows` rows of length n.
double time_variant(const DstChoice& ch, int n, bool fp32, int rows, void* in, void* out,
                    hipStream_t s) {
  DstTask t{};
  t.in = in; t.out = out; t.in_rs = n; t.out_rs = n; t.in_cs = 1; t.out_cs = 1;
  t.rows = rows; t.n = n; t.scale = 1.0; t.fft = TableCache::get().fft(n)->dev;
  const DstKind kind = fp32 ? DstKind::F_F : DstKind::D_D;
  DevBuf keep;
  launch_one_dst(kind, ch, t, s, keep);   // warm-up (code load, LDS opt-in)
  hipEvent_t a, b;
  FDS_HIP(hipEventCreate(&a));
  FDS_HIP(hipEventCreate(&b));
  const int reps = 3;
  FDS_HIP(hipEventRecord(a, s));
  for (int r = 0; r < reps; ++r) {
    DevBuf k;
    launch_one_dst(kind, ch, t, s, k);
    FDS_HIP(hipStreamSynchronize(s));   // k is released after its launch finished
  }
  FDS_HIP(hipEventRecord(b, s));
  FDS_HIP(hipEventSynchronize(b));
  float ms = 0;
  FDS_HIP(hipEventElapsedTime(&ms, a, b));
  (void)hipEventDestroy(a);
  (void)hipEventDestroy(b);
  FDS_HIP(hipGetLastError());
  return ms / reps;
}

const char* variant_name(const DstChoice& c) {
  return c.gemm ? "gemm" : c.wave_big ? "wavebig" : c.wave_e ? "wave" : "fft";
}

// The tables of FDS_TUNE_FILE, read once (under the caller's lock):
// transforms (n, fp32) -> variant, tridiagonal solves (rows, fp32) ->
// (modes per block, rows per segment; 0 0 for the unsegmented kernel).
struct TuneTables {
  std::map<std::pair<int, bool>, std::string> dst;
  std::map<std::pair<int, bool>, std::pair<int, int>> tri;
};

TuneTables& tune_tables() {
  static TuneTables t;
  static std::once_flag once;
  std::call_once(once, [] {
    if (const char* path = std::getenv("FDS_TUNE_FILE")) {
      std::ifstream in(path);
      std::string line;
      while (std::getline(in, line)) {
        char mode[32] = {0};
        int n = 0, prec = 0, mpb = 0, ls = 0;
        if (std::sscanf(line.c_str(), "tri %d %d %d %d", &n, &prec, &mpb, &ls) == 4) {
          if (n > 0 && (prec == 0 || prec == 1)) t.tri[{n, prec != 0}] = {mpb, ls};
        } else if (std::sscanf(line.c_str(), "%d %d %31s", &n, &prec, mode) == 3) {
          const std::string m = mode;
          if (n > 0 && (prec == 0 || prec == 1) && (m == "wave" || m == "wavebig" || m == "fft" || m == "gemm"))
            t.dst[{n, prec != 0}] = m;
        }
      }
    }
  });
  return t;
}

std::map<std::pair<int, bool>, std::string>& tune_table() { return tune_tables().dst; }

void tune_table_append(int n, bool fp32, const char* mode) {
  const char* path = std::getenv("FDS_TUNE_FILE");
  if (!path) return;
  if (FILE* f = std::fopen(path, "a")) {
    std::fprintf(f, "%d %d %s\n", n, fp32 ? 1 : 0, mode);
    std::fclose(f);
  }
}

void tri_table_append(int rows, bool fp32, const TriConfig& c) {
  const char* path = std::getenv("FDS_TUNE_FILE");
  if (!path) return;
  if (FILE* f = std::fopen(path, "a")) {
    std::fprintf(f, "tri %d %d %d %d\n", rows, fp32 ? 1 : 0, c.seg ? c.mpb : 0, c.seg ? c.ls : 0);
    std::fclose(f);
  }
}

// Milliseconds per launch of a tridiagonal configuration on `modes` systems
// of `rows` rows.
double time_tri(const TriConfig& c, bool fp32, int rows, int modes, void* data, const void* coef,
                hipStream_t s) {
  TriTask t{};
  t.data = data; t.rs = modes; t.js = 0; t.rows = rows; t.modes = modes; t.coef = coef;
  DevBuf task(sizeof(TriTask));
  FDS_HIP(hipMemcpyAsync(task.get(), &t, sizeof(t), hipMemcpyHostToDevice, s));
  const int nb = tri_blocks(c, modes);
  launch_tri(c, fp32, task.as<TriTask>(), 1, nb, 0, s);   // warm-up
  hipEvent_t a, b;
  FDS_HIP(hipEventCreate(&a));
  FDS_HIP(hipEventCreate(&b));
  const int reps = 4;
  FDS_HIP(hipEventRecord(a, s));
  for (int r = 0; r < reps; ++r) launch_tri(c, fp32, task.as<TriTask>(), 1, nb, 0, s);
  FDS_HIP(hipEventRecord(b, s));
  FDS_HIP(hipEventSynchronize(b));
  float ms = 0;
  FDS_HIP(hipEventElapsedTime(&ms, a, b));
  (void)hipEventDestroy(a);
  (void)hipEventDestroy(b);
  FDS_HIP(hipGetLastError());
  return ms / reps;
}

}  // namespace

DstChoice dst_tuned_choice(int n, bool fp32) {
  static std::mutex mu;
  static std::map<std::tuple<int, int, bool>, DstChoice> tuned;
  int dev = 0;
  FDS_HIP(hipGetDevice(&dev));
  std::lock_guard<std::mutex> lk(mu);
  auto key = std::make_tuple(dev, n, fp32);
  auto it = tuned.find(key);
  if (it != tuned.end()) return it->second;
  {
    auto& table = tune_table();
    auto t = table.find({n, fp32});
    if (t != table.end()) {
      const DstChoice c = dst_choice_variant(n, fp32, t->second);
      tuned[key] = c;
      return c;
    }
  }

  std::vector<DstChoice> cand;
  for (const char* mode : {"wave", "wavebig", "fft", "gemm"}) {
    const DstChoice c = dst_choice_variant(n, fp32, mode);
    bool dup = false;
    for (const DstChoice& o : cand) dup |= same(o, c);
    if (!dup) cand.push_back(c);
  }
  DstChoice best = cand[0];
  if (cand.size() > 1) {
    const size_t w = fp32 ? 4 : 8;
    // batched use: several thousand rows per launch (about 32 MB of data)
    const int rows = std::max(256, std::min(65536, (1 << 23) / std::max(n, 1)));
    hipStream_t s;
    FDS_HIP(hipStreamCreateWithFlags(&s, hipStreamNonBlocking));
    {
      DevBuf in((size_t)rows * n * w), out((size_t)rows * n * w);
      FDS_HIP(hipMemsetAsync(in.get(), 0, in.size(), s));
      double tbest = -1;
      const bool log = std::getenv("FDS_TUNE_LOG") != nullptr;
      for (size_t i = 0; i < cand.size(); ++i) {
        double ms;
        try {
          ms = time_variant(cand[i], n, fp32, rows, in.get(), out.get(), s);
        } catch (const Error&) {
          continue;   // e.g. a variant whose LDS need exceeds the CU
        }
        if (log)
          std::fprintf(stderr, "[fds tune] n=%d %s rows=%d %s: %.1f us\n", n, fp32 ? "fp32" : "fp64",
                       rows, variant_name(cand[i]), ms * 1e3);
        if (tbest < 0 || ms < tbest) {
          tbest = ms;
          best = cand[i];
        }
      }
      FDS_HIP(hipStreamSynchronize(s));
    }
    (void)hipStreamDestroy(s);
  }
  tuned[key] = best;
  if (cand.size() > 1) tune_table_append(n, fp32, variant_name(best));
  return best;
}

}  // namespace fds

namespace fds {

// Segmentation of the per-mode tridiagonal solve, measured like the
// transforms: on the first request for (device, rows, precision) every
// instantiated configuration that holds the rows solves a synthetic batch
// (about 32 MB), and the fastest is kept (and appended to FDS_TUNE_FILE).
TriConfig tri_config(bool fp32, int rows) {
  const char* seg = std::getenv("FDS_TRI_SEG");
  const char* tune = std::getenv("FDS_TRI_TUNE");
  if (seg || (tune && std::string(tune) == "0")) return tri_config_static(fp32, rows);
  static std::mutex mu;
  static std::map<std::tuple<int, int, bool>, TriConfig> tuned;
  int dev = 0;
  FDS_HIP(hipGetDevice(&dev));
  std::lock_guard<std::mutex> lk(mu);
  auto key = std::make_tuple(dev, rows, fp32);
  auto it = tuned.find(key);
  if (it != tuned.end()) return it->second;
  const std::vector<TriConfig> cand = tri_configs(rows);
  {
    const auto& table = tune_tables().tri;   // read-only once loaded
    auto t = table.find({rows, fp32});
    if (t != table.end()) {
      for (const TriConfig& c : cand)
        if ((!c.seg && t->second.first == 0) || (c.seg && c.mpb == t->second.first && c.ls == t->second.second)) {
          tuned[key] = c;
          return c;
        }
    }
  }
  TriConfig best = cand[0];
  if (cand.size() > 1) {
    const size_t w = fp32 ? 4 : 8;
    const int modes = std::max(64, std::min(65536, (1 << 22) / std::max(rows, 1)));
    hipStream_t s;
    FDS_HIP(hipStreamCreateWithFlags(&s, hipStreamNonBlocking));
    {
      DevBuf data((size_t)rows * modes * w);
      FDS_HIP(hipMemsetAsync(data.get(), 0, data.size(), s));
      auto tab = TableCache::get().modes(modes, rows, 1.0 / (std::max(rows, modes) + 1), 0.0, true);
      const void* coef = fp32 ? (const void*)tab->c32 : (const void*)tab->c64;
      double tbest = -1;
      const bool log = std::getenv("FDS_TUNE_LOG") != nullptr;
      for (const TriConfig& c : cand) {
        const double ms = time_tri(c, fp32, rows, modes, data.get(), coef, s);
        if (log)
          std::fprintf(stderr, "[fds tune] tri rows=%d %s modes=%d mpb=%d ls=%d: %.1f us\n", rows,
                       fp32 ? "fp32" : "fp64", modes, c.mpb, c.ls, ms * 1e3);
        if (tbest < 0 || ms < tbest) {
          tbest = ms;
          best = c;
        }
      }
      FDS_HIP(hipStreamSynchronize(s));
    }
    (void)hipStreamDestroy(s);
  }
  tuned[key] = best;
  if (cand.size() > 1) tri_table_append(rows, fp32, best);
  return best;
}

}  // namespace fds
