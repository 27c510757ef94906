// Device tables: FFT twiddles, per-mode tridiagonal coefficients and Schur
// line coefficients.  All values are computed on the host in FP64 (long
// double where the angle reduction benefits) and uploaded once.
#include <algorithm>
#include <cmath>
#include <tuple>
#include <mutex>
#include <map>
#include <complex>
#include <cstdlib>
#include <cstring>
#include <string>

#include "runtime.h"

namespace fds {

// Host-to-device upload of a table, ordered on a private non-blocking stream
// of the calling thread and waited for: no legacy-stream operation, so plans
// can be built while another thread captures or replays a graph.
static void upload(void* dst, const void* src, size_t bytes) {
  thread_local hipStream_t s = nullptr;
  if (!s) FDS_HIP(hipStreamCreateWithFlags(&s, hipStreamNonBlocking));
  FDS_HIP(hipMemcpyAsync(dst, src, bytes, hipMemcpyHostToDevice, s));
  FDS_HIP(hipStreamSynchronize(s));
}


std::vector<int> fft_radices(int N) {
  // radix-16 and radix-8 butterflies run in registers, so powers of two go
  // out in as few passes as possible
  std::vector<int> r;
  int n = N;
  while (n % 16 == 0) { r.push_back(16); n /= 16; }
  if (n % 8 == 0) { r.push_back(8); n /= 8; }
  if (n % 4 == 0) { r.push_back(4); n /= 4; }
  if (n % 2 == 0) { r.push_back(2); n /= 2; }
  while (n % 3 == 0) { r.push_back(3); n /= 3; }
  while (n % 5 == 0) { r.push_back(5); n /= 5; }
  for (int p = 7; n > 1; p += 2) {
    while (n % p == 0) { r.push_back(p); n /= p; }
    if ((long long)p * p > n && n > 1) { r.push_back(n); n = 1; }
  }
  if ((int)r.size() > kMaxPass) throw Error(FDS_E_UNSUPPORTED, "FFT length has too many factors");
  return r;
}

bool fixed_radices(int L) {
  for (int R : fft_radices(L))
    if (R != 2 && R != 3 && R != 4 && R != 5 && R != 8 && R != 16) return false;
  return true;
}

// Relative cost of one Stockham FFT of length L (per output, summed over
// passes): a pass costs one LDS round trip plus its butterfly arithmetic;
// other primes take direct sums.
static double stockham_cost(int L) {
  double c = 0;
  for (int R : fft_radices(L)) {
    switch (R) {
      case 2: c += 1.0; break;
      case 3: c += 1.6; break;
      case 4: c += 1.3; break;
      case 5: c += 2.0; break;
      case 8: c += 1.7; break;
      case 16: c += 2.2; break;
      default: c += 1.5 * R; break;
    }
  }
  return c * L;
}

static bool is_prime(int p) {
  if (p < 2) return false;
  for (int d = 2; (long long)d * d <= p; ++d)
    if (p % d == 0) return false;
  return true;
}

// Convolution length of Bluestein's algorithm for a length-N DFT: at least
// 2N - 1, with radices that have register butterflies.  FDS_BLUE_M selects
// the smallest 5-smooth length ("smooth", fewest points) or the smallest
// 2^a or 3 2^a ("pow2", fewest passes).
static int bluestein_len(int N) {
  static const int mode = [] {
    const char* e = std::getenv("FDS_BLUE_M");
    if (e && std::string(e) == "pow2") return 1;
    if (e && std::string(e) == "p2") return 2;
    return 0;
  }();
  int M = 2 * N - 1;
  if (mode >= 1) {
    int p = 1;
    while (p < M) p *= 2;
    int q = 3;
    while (q < M) q *= 2;
    return mode == 2 ? p : std::min(p, q);
  }
  auto smooth = [](int v) {
    for (int p : {2, 3, 5}) while (v % p == 0) v /= p;
    return v == 1;
  };
  while (!smooth(M)) ++M;
  return M;
}

FftShape fft_shape(int n) {
  const int N = n + 1;
  FftShape s{FFT_MIXED, N, N};
  double best = stockham_cost(N);
  if (N > 7 && is_prime(N)) {
    const double c = 2.0 * stockham_cost(N - 1) + 3.0 * N;
    if (c < best) { best = c; s = FftShape{FFT_RADER, N - 1, N}; }
  }
  const int M = bluestein_len(N);
  // both LDS buffers of an FP64 row (plus the line-kernel scratch) must fit
  const bool fits = (size_t)M * 3 * sizeof(double2) + sizeof(double) * (N + 1) <= 160u * 1024u;
  if (N > 8 && fits) {
    const double c = 2.0 * stockham_cost(M) + 4.0 * M;
    if (c < best) { best = c; s = FftShape{FFT_BLUESTEIN, M, M}; }
  }
  return s;
}

int dst_threads_per_row(int n) {
  // about one radix-4 butterfly per thread and pass; FDS_DST_TPR overrides
  // (32..256, power of two) for tuning measurements
  if (const char* e = std::getenv("FDS_DST_TPR")) {
    const int v = std::atoi(e);
    if (v == 32 || v == 64 || v == 128 || v == 256) return v;
  }
  const int W = fft_shape(n).lds_len;
  int G = 32;
  while (G < 256 && 2 * G <= W / 4) G *= 2;
  return G;
}

static size_t row_buffers(int n, bool fp32) {
  const int rpb = kBlock / dst_threads_per_row(n);
  return (size_t)rpb * 2 * fft_shape(n).lds_len * (fp32 ? sizeof(float2) : sizeof(double2));
}

bool dst_twiddles_in_lds(int n, bool fp32) {
  if (const char* e = std::getenv("FDS_DST_TWLDS")) return std::atoi(e) != 0;
  const size_t tw = (size_t)fft_shape(n).L * (fp32 ? sizeof(float2) : sizeof(double2));
  return row_buffers(n, fp32) + tw <= 96u * 1024u;
}

size_t dst_smem_bytes(int n, bool fp32) {
  const size_t tw = dst_twiddles_in_lds(n, fp32)
                        ? (size_t)fft_shape(n).L * (fp32 ? sizeof(float2) : sizeof(double2)) : 0;
  return row_buffers(n, fp32) + tw;
}

// Entries of the per-pass twiddle table: sum over passes of (R - 1) Ns.
static int wave_twiddle_len(const std::vector<int>& rad) {
  int ns = 1, t = 0;
  for (int R : rad) {
    t += (R - 1) * ns;
    ns *= R;
  }
  return t;
}

static int lanes_for(int L) {
  // lanes per row: as many as keep every lane of a radix-4 pass busy (one
  // wavefront per row from L = 256 on), so short batches still spread over
  // many wavefronts; FDS_DST_G overrides (16, 32, 64) for measurements
  // (read once: the cached table images follow the schedule of this choice)
  static const int forced = [] {
    const char* e = std::getenv("FDS_DST_G");
    const int v = e ? std::atoi(e) : 0;
    return (v == 16 || v == 32 || v == 64) ? v : 0;
  }();
  if (forced) return forced;
  int G = 16;
  while (G < 64 && 4 * (2 * G) <= L) G *= 2;
  return G;
}

// Register budget (complex entries per lane) of a wave schedule, or 0.
static int wave_need(int n, int L, int G, const std::vector<int>& rad) {
  if (rad.empty()) return 0;
  int need = (n + G - 1) / G;  // row elements per lane
  for (int R : rad) need = std::max(need, (L / R + G - 1) / G * R);
  return need;
}

// Lanes per row of the one-row-per-workgroup ("big") wave transform.
static int big_lanes(int L) {
  static const int forced = [] {
    const char* e = std::getenv("FDS_DST_BIGG");
    const int v = e ? std::atoi(e) : 0;
    return (v == 128 || v == 256 || v == 512) ? v : 0;
  }();
  if (forced) return forced;
  return L >= 3072 ? 512 : L >= 1024 ? 256 : 128;
}

// FFT schedule of the wave-parallel transform and the lane count its radices
// are built for.  The workgroup schedule when its radices have register
// butterflies only; otherwise Rader (N prime, N - 1 5-smooth) or Bluestein
// over the smallest 5-smooth length >= 2N - 1, whichever is wave-schedulable
// and cheaper.  When no schedule fits one wavefront per row (at most 32
// entries per lane), the same candidates are tried with a workgroup per row
// (big_lanes lanes, the FP64 row alone in LDS).  G == 0: no wave schedule.
struct WaveSched {
  FftShape shp;
  int G;
};

static WaveSched wave_sched(int n) {
  const int N = n + 1;
  const FftShape s0 = fft_shape(n);
  struct Cand { FftShape s; double cost; bool own; };
  std::vector<Cand> cand;
  if (fixed_radices(s0.L)) cand.push_back({s0, 0.0, true});
  if (N > 7 && is_prime(N) && s0.kind != FFT_RADER)
    cand.push_back({FftShape{FFT_RADER, N - 1, N}, 2.0 * stockham_cost(N - 1) + 3.0 * N, false});
  const int M = bluestein_len(N);
  if (N > 8 && !(s0.kind == FFT_BLUESTEIN && s0.L == M))
    cand.push_back({FftShape{FFT_BLUESTEIN, M, M}, 2.0 * stockham_cost(M) + 4.0 * M, false});
  for (int big = 0; big < 2; ++big) {
    int bi = -1;
    for (size_t i = 0; i < cand.size(); ++i) {
      const FftShape& s = cand[i].s;
      const int G = big ? big_lanes(s.L) : lanes_for(s.L);
      const int need = wave_need(n, s.L, G, wave_radices(s.L, G));
      if (need <= 0 || need > 32) continue;
      if (big && wave_layout<double>(s.kind, N, s.L, s.lds_len, s.L).row_bytes > 160 * 1024) continue;
      if (cand[i].own) { bi = (int)i; break; }   // the workgroup schedule is kept when it qualifies
      if (bi < 0 || cand[i].cost < cand[bi].cost) bi = (int)i;
    }
    if (bi >= 0) {
      const FftShape& s = cand[bi].s;
      return WaveSched{s, big ? big_lanes(s.L) : lanes_for(s.L)};
    }
  }
  return WaveSched{s0, 0};
}

FftShape wave_shape(int n) { return wave_sched(n).shp; }

int wave_lanes(int n) {
  const WaveSched w = wave_sched(n);
  return w.G ? w.G : lanes_for(w.shp.L);
}

std::vector<int> wave_radices(int L, int G) {
  // powers of two in passes as long as every pass keeps L/R >= G
  // butterflies, then 3s and 5s (other primes: not a wave schedule)
  const int rmax = std::max(2, L / G);
  std::vector<int> r;
  int m = L, a = 0;
  while (m % 2 == 0) { m /= 2; ++a; }
  for (int R : {16, 8, 4}) {
    const int e = R == 16 ? 4 : R == 8 ? 3 : 2;
    while (a >= e && R <= rmax) { r.push_back(R); a -= e; }
  }
  while (a > 0) { r.push_back(2); --a; }
  while (m % 3 == 0) { r.push_back(3); m /= 3; }
  while (m % 5 == 0) { r.push_back(5); m /= 5; }
  if (m != 1 || r.size() > 12) r.clear();
  return r;
}

WaveCfg dst_wave_config(int n, bool fp32, bool big) {
  WaveCfg c{0, 0, 0, 0, 0};
  const WaveSched ws = wave_sched(n);
  if (ws.G == 0) return c;
  const FftShape shp = ws.shp;
  const std::vector<int> rad = wave_radices(shp.L, ws.G);
  const int twl = wave_twiddle_len(rad);
  const WaveLayout lay = fp32 ? wave_layout<float>(shp.kind, n + 1, shp.L, shp.lds_len, twl)
                              : wave_layout<double>(shp.kind, n + 1, shp.L, shp.lds_len, twl);
  if (big) {
    // one row per workgroup; the tables stay in global memory
    const int G = big_lanes(shp.L);
    const int need = wave_need(n, shp.L, G, rad);
    if (need == 0) return c;
    for (int e : {8, 16, 32})
      if (need <= e) { c.E = e; break; }
    if (!c.E || (size_t)lay.row_bytes > 160u * 1024u) return WaveCfg{0, 0, 0, 0, 0};
    c.G = G;
    c.waves = G / 64;
    c.rows_per_block = 1;
    c.smem = (size_t)lay.row_bytes;
    return c;
  }
  if (ws.G > 64) return c;   // only the workgroup-per-row form fits
  const int G = ws.G;
  const int need = wave_need(n, shp.L, G, rad);
  if (need == 0) return c;
  for (int e : {4, 8, 16, 32, 64})
    if ((e <= 32 || fp32) && need <= e) { c.E = e; break; }
  if (!c.E) return c;
  c.G = G;
  // workgroup size with the most rows resident per CU (160 KB of LDS, at most
  // 16 wavefronts); ties go to the larger workgroup (fewer table copies)
  int best = -1;
  for (int waves : {1, 2, 4}) {
    const int rpb = waves * 64 / c.G;
    const size_t smem = (size_t)lay.rows + (size_t)rpb * lay.row_bytes;
    if (smem > 160u * 1024u) continue;
    const int blocks = std::min((int)(160u * 1024u / smem), 16 / waves);
    const int resident = blocks * rpb;
    if (resident >= best) {
      best = resident;
      c.waves = waves;
      c.rows_per_block = rpb;
      c.smem = smem;
    }
  }
  if (best <= 0) c.E = 0;
  return c;
}

DstChoice dst_choice(int n, bool fp32) {
  // FDS_DST_ALGO=wave|fft|gemm pins a variant; otherwise the autotuner's
  // measured choice (FDS_DST_TUNE=0: the static preference, wave where
  // possible).  Memoised per (setting, n, precision): task-list construction
  // asks for every transform of every problem.
  static std::mutex mu;
  static std::map<std::tuple<std::string, int, bool>, DstChoice> memo;
  const char* env = std::getenv("FDS_DST_ALGO");
  std::string mode = env ? env : "auto";
  if (mode == "auto") {
    const char* t = std::getenv("FDS_DST_TUNE");
    if (!(t && std::string(t) == "0")) return dst_tuned_choice(n, fp32);
    mode = "wave";
  }
  std::lock_guard<std::mutex> lk(mu);
  auto key = std::make_tuple(mode, n, fp32);
  auto it = memo.find(key);
  if (it != memo.end()) return it->second;
  const DstChoice c = dst_choice_variant(n, fp32, mode);
  memo[key] = c;
  return c;
}

DstChoice dst_choice_variant(int n, bool fp32, const std::string& mode) {
  DstChoice c{false, 1, 4, 0, 0, 0, kBlock};
  if (mode == "gemm" && n <= kGemmMaxN) {
    const int np = (n + 63) / 64 * 64;
    c.gemm = true;
    c.rt = np <= 256 ? 2 : 1;
    c.ct = 4;
    c.rows_per_block = c.rt * 16;
    c.smem = gemm_smem_bytes(n, fp32, c.rt);
    return c;
  }
  if (mode != "fft") {
    // "wave": a row per wavefront where possible, else a row per workgroup;
    // "wavebig": a row per workgroup
    for (int big = mode == "wavebig" ? 1 : 0; big < 2; ++big) {
      const WaveCfg w = dst_wave_config(n, fp32, big != 0);
      if (w.E) {
        c.wave_e = w.E;
        c.wave_big = big;
        c.threads = 64 * w.waves;
        c.rows_per_block = w.rows_per_block;
        c.smem = w.smem;
        return c;
      }
    }
  }
  c.rows_per_block = kBlock / dst_threads_per_row(n);
  c.smem = dst_smem_bytes(n, fp32);
  return c;
}

size_t line_smem_bytes(int n) {
  const FftShape s = fft_shape(n);
  return sizeof(double2) * ((size_t)2 * s.lds_len + s.L) + sizeof(double) * (n + 1);
}

TableCache& TableCache::get() {
  static TableCache* c = new TableCache();   // never destroyed (see alloc.cpp)
  return *c;
}

static int current_device() {
  int d = 0;
  FDS_HIP(hipGetDevice(&d));
  return d;
}

static size_t align_up(size_t x, size_t a) { return (x + a - 1) / a * a; }

using cld = std::complex<long double>;
static const long double kPi = 3.141592653589793238462643383279502884L;

// exp(-2 pi i t / N) with the integer t reduced modulo N first
static cld unit_root(long long t, long long N) {
  t %= N;
  if (t < 0) t += N;
  const long double a = 2.0L * kPi * (long double)t / (long double)N;
  return cld(cosl(a), -sinl(a));
}

// Forward DFT on the host (plan construction only), recursive mixed radix.
static std::vector<cld> host_dft(const std::vector<cld>& x) {
  const int N = (int)x.size();
  if (N == 1) return x;
  int p = 2;
  while (N % p) ++p;
  if (p == N) {
    std::vector<cld> X(N);
    for (int k = 0; k < N; ++k) {
      cld s = 0;
      for (int j = 0; j < N; ++j) s += x[j] * unit_root((long long)j * k, N);
      X[k] = s;
    }
    return X;
  }
  const int M = N / p;
  std::vector<std::vector<cld>> sub(p);
  for (int r = 0; r < p; ++r) {
    std::vector<cld> xr(M);
    for (int j = 0; j < M; ++j) xr[j] = x[j * p + r];
    sub[r] = host_dft(xr);
  }
  std::vector<cld> X(N);
  for (int k = 0; k < N; ++k) {
    cld s = 0;
    for (int r = 0; r < p; ++r) s += unit_root((long long)r * k, N) * sub[r][k % M];
    X[k] = s;
  }
  return X;
}

static int primitive_root(int p) {
  const int phi = p - 1;
  std::vector<int> fs;
  int m = phi;
  for (int d = 2; (long long)d * d <= m; ++d)
    if (m % d == 0) { fs.push_back(d); while (m % d == 0) m /= d; }
  if (m > 1) fs.push_back(m);
  auto powmod = [](long long b, long long e, long long mod) {
    long long r = 1;
    b %= mod;
    while (e) { if (e & 1) r = r * b % mod; b = b * b % mod; e >>= 1; }
    return r;
  };
  for (int g = 2; g < p; ++g) {
    bool ok = true;
    for (int q : fs) if (powmod(g, phi / q, p) == 1) { ok = false; break; }
    if (ok) return g;
  }
  throw Error(FDS_E_UNSUPPORTED, "no primitive root");
}

// Convolution kernel (DFT of the Rader sequence or of the Bluestein chirp,
// scaled by 1/L), chirp and Rader permutations of one FFT schedule.
struct ShapeTables {
  std::vector<cld> kern, chirp;
  std::vector<int> pin, pout;
};

static ShapeTables shape_tables(const FftShape& shp, int N) {
  ShapeTables st;
  const int L = shp.L;
  std::vector<cld> kern;
  if (shp.kind == FFT_RADER) {
    const int g = primitive_root(N);
    long long gp = 1, gi = 1;
    long long ginv = 1;
    for (int e = 0; e < N - 2; ++e) ginv = ginv * g % N;  // g^{N-2} = g^{-1}
    std::vector<cld> b(L);
    st.pin.resize(L);
    st.pout.resize(L);
    for (int q = 0; q < L; ++q) {
      st.pin[q] = (int)gi;
      st.pout[q] = (int)gp;
      b[q] = unit_root(gp, N);
      gi = gi * ginv % N;
      gp = gp * g % N;
    }
    kern = host_dft(b);
  } else if (shp.kind == FFT_BLUESTEIN) {
    std::vector<cld> h(L, cld(0, 0));
    st.chirp.resize(N);
    for (int j = 0; j < N; ++j) {
      // exp(-i pi j^2/N) = exp(-2 pi i (j^2 mod 2N) / (2N))
      const cld c = unit_root((long long)j * j % (2LL * N), 2LL * N);
      st.chirp[j] = c;
      h[j] = std::conj(c);
      if (j > 0) h[L - j] = std::conj(c);
    }
    kern = host_dft(h);
  }
  for (const cld& v : kern) st.kern.push_back(v / (long double)L);
  return st;
}

std::shared_ptr<FftTable> TableCache::fft(int n) {
  const int dev = current_device();
  auto key = std::make_pair(dev, n);
  {
    // the lock covers the lookups and the insertion only: building and
    // uploading a table runs unlocked, so threads that build plans do not
    // stall threads that only look tables up
    std::lock_guard<std::mutex> lk(mu_);
    auto it = fft_.find(key);
    if (it != fft_.end()) return it->second;
  }
  const int N = n + 1;
  const FftShape shp = fft_shape(n);
  const int L = shp.L;
  auto t = std::make_shared<FftTable>();
  std::vector<int> rad = fft_radices(L);
  const bool rader = shp.kind == FFT_RADER, blue = shp.kind == FFT_BLUESTEIN;
  const int nk = (rader || blue) ? L : 0;
  const int nch = blue ? N : 0;
  size_t o = align_up(sizeof(FftDesc), 256);
  auto take = [&](size_t bytes) { size_t r = o; o = align_up(o + bytes, 256); return r; };
  const size_t o_tw64 = take(sizeof(double2) * L), o_tw32 = take(sizeof(float2) * L);
  const size_t o_p64 = take(sizeof(double2) * (N + 1)), o_p32 = take(sizeof(float2) * (N + 1));
  const size_t o_pin = take(sizeof(int) * (rader ? L : 1)), o_pout = take(sizeof(int) * (rader ? L : 1));
  const size_t o_k64 = take(sizeof(double2) * std::max(nk, 1)), o_k32 = take(sizeof(float2) * std::max(nk, 1));
  const size_t o_c64 = take(sizeof(double2) * std::max(nch, 1)), o_c32 = take(sizeof(float2) * std::max(nch, 1));
  const int np = n <= kGemmMaxN ? (n + 63) / 64 * 64 : 0;
  const size_t o_s64 = take(sizeof(double) * std::max((size_t)np * np, (size_t)1));
  const size_t o_s32 = take(sizeof(float) * std::max((size_t)np * np, (size_t)1));
  // the wave-parallel transform may run another schedule (wave_shape)
  const WaveSched wsch = wave_sched(n);
  const FftShape wshp = wsch.shp;
  const int wL = wshp.L;
  const std::vector<int> wrad = wsch.G ? wave_radices(wL, wsch.G) : std::vector<int>{};
  const int twl = wave_twiddle_len(wrad);
  const WaveLayout wl64 = wave_layout<double>(wshp.kind, N, wL, wshp.lds_len, twl);
  const WaveLayout wl32 = wave_layout<float>(wshp.kind, N, wL, wshp.lds_len, twl);
  const size_t o_w64 = take((size_t)wl64.rows), o_w32 = take((size_t)wl32.rows);
  const size_t total = o;
  std::vector<unsigned char> host(total, 0);
  auto* tw64 = reinterpret_cast<double2*>(host.data() + o_tw64);
  auto* tw32 = reinterpret_cast<float2*>(host.data() + o_tw32);
  for (int t0 = 0; t0 < L; ++t0) {
    const cld w = unit_root(t0, L);
    tw64[t0] = double2{(double)w.real(), (double)w.imag()};
    tw32[t0] = float2{(float)w.real(), (float)w.imag()};
  }
  auto* p64 = reinterpret_cast<double2*>(host.data() + o_p64);
  auto* p32 = reinterpret_cast<float2*>(host.data() + o_p32);
  for (int k = 0; k <= N; ++k) {
    const long double a = kPi * (long double)k / (long double)N;
    const double c = (double)cosl(a), s = (double)sinl(a);
    p64[k] = double2{c, s};
    p32[k] = float2{(float)c, (float)s};
  }
  const ShapeTables stab = shape_tables(shp, N);
  if (rader) {
    std::memcpy(host.data() + o_pin, stab.pin.data(), sizeof(int) * L);
    std::memcpy(host.data() + o_pout, stab.pout.data(), sizeof(int) * L);
  }
  if (blue) {
    auto* c64 = reinterpret_cast<double2*>(host.data() + o_c64);
    auto* c32 = reinterpret_cast<float2*>(host.data() + o_c32);
    for (int j = 0; j < N; ++j) {
      c64[j] = double2{(double)stab.chirp[j].real(), (double)stab.chirp[j].imag()};
      c32[j] = float2{(float)stab.chirp[j].real(), (float)stab.chirp[j].imag()};
    }
  }
  if (!stab.kern.empty()) {
    auto* k64 = reinterpret_cast<double2*>(host.data() + o_k64);
    auto* k32 = reinterpret_cast<float2*>(host.data() + o_k32);
    for (int q = 0; q < L; ++q) {
      const cld v = stab.kern[q];
      k64[q] = double2{(double)v.real(), (double)v.imag()};
      k32[q] = float2{(float)v.real(), (float)v.imag()};
    }
  }
  if (np) {
    auto* s64 = reinterpret_cast<double*>(host.data() + o_s64);
    auto* s32 = reinterpret_cast<float*>(host.data() + o_s32);
    for (int j = 0; j < n; ++j)
      for (int c = 0; c < n; ++c) {
        // sin(pi (j+1)(c+1) / N) with the integer reduced modulo 2N
        const long long tt = (long long)(j + 1) * (c + 1) % (2LL * N);
        const long double v = sinl(kPi * (long double)tt / (long double)N);
        s64[(size_t)j * np + c] = (double)v;
        s32[(size_t)j * np + c] = (float)v;
      }
  }
  // table images in the LDS layout of the wave-parallel row transform
  {
    const ShapeTables wtab = (wshp.kind == shp.kind && wL == L) ? stab : shape_tables(wshp, N);
    // per-pass twiddles: pass (R, Ns) holds exp(-2 pi i r k stw / wL) at
    // (r-1) Ns + k, stw = wL / (Ns R)
    std::vector<cld> ptw;
    {
      int ns = 1;
      for (int R : wrad) {
        const int stw = wL / (ns * R);
        for (int r = 1; r < R; ++r)
          for (int k = 0; k < ns; ++k) ptw.push_back(unit_root((long long)r * k * stw, wL));
        ns *= R;
      }
    }
    std::vector<cld> post(N + 1);
    for (int k = 0; k <= N; ++k) {
      const long double a = kPi * (long double)k / (long double)N;
      post[k] = cld(cosl(a), sinl(a));
    }
    auto put_c = [](unsigned char* dst, const std::vector<cld>& v, bool f32) {
      for (size_t i = 0; i < v.size(); ++i) {
        if (f32) {
          const float2 x{(float)v[i].real(), (float)v[i].imag()};
          std::memcpy(dst + i * sizeof(x), &x, sizeof(x));
        } else {
          const double2 x{(double)v[i].real(), (double)v[i].imag()};
          std::memcpy(dst + i * sizeof(x), &x, sizeof(x));
        }
      }
    };
    auto put = [&](size_t base, const WaveLayout& w, bool f32) {
      unsigned char* img = host.data() + base;
      put_c(img + w.tw, ptw, f32);
      put_c(img + w.post, post, f32);
      if (wshp.kind != FFT_MIXED) put_c(img + w.kern, wtab.kern, f32);
      if (wshp.kind == FFT_BLUESTEIN) put_c(img + w.chirp, wtab.chirp, f32);
      if (wshp.kind == FFT_RADER) {
        std::memcpy(img + w.pin, wtab.pin.data(), sizeof(int) * wL);
        std::memcpy(img + w.pout, wtab.pout.data(), sizeof(int) * wL);
      }
    };
    put(o_w64, wl64, false);
    put(o_w32, wl32, true);
  }
  t->mem.alloc(total);
  FftDesc d{};
  for (int prec = 0; prec < 2; ++prec) {
    WaveDesc& w = prec ? t->wave32 : t->wave64;
    w = WaveDesc{};
    w.N = N;
    w.L = wL;
    w.W = wshp.lds_len;
    w.kind = wshp.kind;
    w.npass = (int)wrad.size();
    w.twlen = twl;
    w.img_chunks = (prec ? wl32.rows : wl64.rows) / 16;
    w.img = t->mem.as<uint4>(prec ? o_w32 : o_w64);
    for (size_t i = 0; i < wrad.size(); ++i) w.radices |= (unsigned long long)wrad[i] << (5 * i);
  }
  d.N = N;
  d.np = np;
  d.smat64 = np ? t->mem.as<double>(o_s64) : nullptr;
  d.smat32 = np ? t->mem.as<float>(o_s32) : nullptr;
  d.kind = shp.kind;
  d.L = L;
  d.W = shp.lds_len;
  d.npass = (int)rad.size();
  for (size_t i = 0; i < rad.size(); ++i) d.radix[i] = rad[i];
  d.tw64 = t->mem.as<double2>(o_tw64);
  d.tw32 = t->mem.as<float2>(o_tw32);
  d.post64 = t->mem.as<double2>(o_p64);
  d.post32 = t->mem.as<float2>(o_p32);
  d.perm_in = rader ? t->mem.as<int>(o_pin) : nullptr;
  d.perm_out = rader ? t->mem.as<int>(o_pout) : nullptr;
  d.kern64 = nk ? t->mem.as<double2>(o_k64) : nullptr;
  d.kern32 = nk ? t->mem.as<float2>(o_k32) : nullptr;
  d.chirp64 = blue ? t->mem.as<double2>(o_c64) : nullptr;
  d.chirp32 = blue ? t->mem.as<float2>(o_c32) : nullptr;
  std::memcpy(host.data(), &d, sizeof(d));
  upload(t->mem.get(), host.data(), total);
  t->host = d;
  t->dev = t->mem.as<FftDesc>(0);
  std::lock_guard<std::mutex> lk(mu_);
  auto it = fft_.find(key);
  if (it != fft_.end()) return it->second;   // built meanwhile by another thread
  fft_[key] = t;
  by_dev_[t->dev] = t;
  return t;
}

WaveDesc TableCache::wave_desc(const FftDesc* dev, bool fp32) {
  std::lock_guard<std::mutex> lk(mu_);
  auto it = by_dev_.find(dev);
  if (it == by_dev_.end()) throw Error(FDS_E_INVALID_ARG, "unknown transform table");
  return fp32 ? it->second->wave32 : it->second->wave64;
}

// theta_k with cosh(theta_k) = -a_k/(2 delta),
// a_k = -4 delta + 2 delta cos(k pi/N) + kappa:
//   u = -a_k/(2 delta) - 1 = 2 sin^2(k pi/(2N)) - kappa/(2 delta) (no cancellation),
//   theta = log1p(u + sqrt(u (u + 2))).
static bool mode_theta(int k, int N, double delta, double kappa, double* theta) {
  const long double pi = 3.141592653589793238462643383279502884L;
  const long double s = sinl(pi * (long double)k / (2.0L * (long double)N));
  const long double u = 2.0L * s * s - (long double)kappa / (2.0L * (long double)delta);
  if (!(u > 0.0L)) return false;
  *theta = (double)log1pl(u + sqrtl(u * (u + 2.0L)));
  return true;
}

void mode_coefs_host(int n, int m, double h, double kappa, double scale,
                     std::vector<ModeCoef<double>>& c64, std::vector<ModeCoef<float>>& c32) {
  const int N = n + 1;
  const double delta = 1.0 / (h * h);
  c64.resize(n);
  c32.resize(n);
  for (int k = 1; k <= n; ++k) {
    double th;
    if (!mode_theta(k, N, delta, kappa, &th))
      throw Error(FDS_E_UNSUPPORTED, "kappa makes a sine mode oscillatory (not diagonally dominant)");
    const double q = std::exp(-th);
    const double e1 = std::expm1(-2.0 * m * th) / std::expm1(-2.0 * th);  // (1-q^2m)/(1-q^2)
    const double beta = q * q / (1.0 + q * q * e1);
    const double sc = -(q / delta) * scale;
    const double lq = std::log2(q);
    auto fill = [&](ModeCoef<double>& c, double tiny_exp) {
      long long K = (long long)std::floor(tiny_exp / lq);
      if (K > m - 1) K = m - 1;
      if (K < 0) K = 0;
      c.q = q;
      c.qinv = std::exp(th);
      c.sc = sc;
      c.beta = beta;
      c.qK = std::exp(-(double)K * th);
      c.K = (int)K;
    };
    ModeCoef<double> a{};
    fill(a, -900.0);
    c64[k - 1] = a;
    ModeCoef<double> b{};
    fill(b, -100.0);
    c32[k - 1] = ModeCoef<float>{(float)b.q, (float)b.qinv, (float)b.sc, (float)b.beta,
                                 (float)b.qK, b.K};
  }
}

std::shared_ptr<ModeTable> upload_modes(const std::vector<ModeCoef<double>>& c64,
                                        const std::vector<ModeCoef<float>>& c32) {
  const size_t n = c64.size();
  auto t = std::make_shared<ModeTable>();
  const size_t o32 = align_up(sizeof(ModeCoef<double>) * n, 256);
  t->mem.alloc(o32 + sizeof(ModeCoef<float>) * n);
  upload(t->mem.get(), c64.data(), sizeof(ModeCoef<double>) * n);
  upload(t->mem.as<char>(o32), c32.data(), sizeof(ModeCoef<float>) * n);
  t->c64 = t->mem.as<ModeCoef<double>>(0);
  t->c32 = t->mem.as<ModeCoef<float>>(o32);
  return t;
}

std::shared_ptr<ModeTable> TableCache::modes(int n, int m, double h, double kappa, bool unit) {
  const int dev = current_device();
  auto key = std::make_tuple(dev, n, m, h, kappa, unit);
  {
    std::lock_guard<std::mutex> lk(mu_);
    auto it = modes_.find(key);
    if (it != modes_.end()) {
      if (auto live = it->second.lock()) return live;
      modes_.erase(it);
    }
  }
  std::vector<ModeCoef<double>> c64;
  std::vector<ModeCoef<float>> c32;
  mode_coefs_host(n, m, h, kappa, unit ? 1.0 : 2.0 / (n + 1), c64, c32);
  auto t = upload_modes(c64, c32);
  std::lock_guard<std::mutex> lk(mu_);
  auto it = modes_.find(key);
  if (it != modes_.end())
    if (auto live = it->second.lock()) return live;
  if (modes_.size() > 4096)   // drop the keys of tables no plan holds any more
    for (auto i = modes_.begin(); i != modes_.end();) i = i->second.expired() ? modes_.erase(i) : std::next(i);
  modes_[key] = t;
  return t;
}

// Schur line coefficients of an arm with line length n and m rows (the
// interface row first):  g_k = [T_k^{-1}]_{11} = -sinh(m theta)/(delta sinh((m+1) theta))
//                           = -(q/delta) (1 - q^{2m})/(1 - q^{2m+2}),
// stored as delta^2 (2/N) g_k.
std::vector<double> schur_gs_host(int n, int m, double h, double kappa) {
  const int N = n + 1;
  const double delta = 1.0 / (h * h);
  std::vector<double> v(n);
  for (int k = 1; k <= n; ++k) {
    double th;
    if (!mode_theta(k, N, delta, kappa, &th))
      throw Error(FDS_E_UNSUPPORTED, "kappa makes a sine mode oscillatory (not diagonally dominant)");
    const double q = std::exp(-th);
    const double g = -(q / delta) * (std::expm1(-2.0 * m * th) / std::expm1(-2.0 * (m + 1) * th));
    v[k - 1] = delta * delta * (2.0 / N) * g;
  }
  return v;
}

std::shared_ptr<GsTable> TableCache::gs(int n, int m, double h, double kappa, bool want_dense) {
  const int dev = current_device();
  auto key = std::make_tuple(dev, n, m, h, kappa, want_dense);
  {
    std::lock_guard<std::mutex> lk(mu_);
    auto it = gs_.find(key);
    if (it != gs_.end()) {
      if (auto live = it->second.lock()) return live;
      gs_.erase(it);
    }
  }
  const int N = n + 1;
  const std::vector<double> v = schur_gs_host(n, m, h, kappa);
  auto t = std::make_shared<GsTable>();
  const bool dense = want_dense && n <= kDenseLineMax;
  const size_t nn = (size_t)n * n;
  std::vector<double> host(n + (dense ? nn : 0));
  std::copy(v.begin(), v.end(), host.begin());
  if (dense) {
    // S diag(gs) S by product to sum: sin(a) sin(b) = (cos(a-b) - cos(a+b))/2,
    // so M_ik = (c(|i-k|) - c(i+k))/2 with c(t) = sum_l gs_l cos(pi l t/N)
    // (i, k, l = 1..n; angles reduced modulo 2N before the cosine).
    std::vector<long double> cs(2 * N);  // cos(pi r/N), r < 2N
    for (int r = 0; r < 2 * N; ++r) cs[r] = cosl(kPi * (long double)r / (long double)N);
    std::vector<long double> c(2 * N + 1);
    for (int tt = 0; tt <= 2 * N; ++tt) {
      long double acc = 0;
      for (int l = 1; l <= n; ++l) acc += (long double)v[l - 1] * cs[(long long)l * tt % (2LL * N)];
      c[tt] = acc;
    }
    double* mf = host.data() + n;
    for (int i = 1; i <= n; ++i)
      for (int k = 1; k <= n; ++k)
        mf[(size_t)(k - 1) * n + (i - 1)] = (double)(0.5L * (c[std::abs(i - k)] - c[i + k]));
  }
  t->mem.alloc(sizeof(double) * host.size());
  upload(t->mem.get(), host.data(), sizeof(double) * host.size());
  t->gs = t->mem.as<double>(0);
  if (dense) {
    t->mfull = t->gs + n;
  }
  std::lock_guard<std::mutex> lk(mu_);
  auto it = gs_.find(key);
  if (it != gs_.end())
    if (auto live = it->second.lock()) return live;
  if (gs_.size() > 4096)
    for (auto i = gs_.begin(); i != gs_.end();) i = i->second.expired() ? gs_.erase(i) : std::next(i);
  gs_[key] = t;
  return t;
}

// Corner entries of T^{-1} for T = tridiag(delta, a, delta) of order m with
// a = -2 delta cosh(theta) (theta from mode_theta):
//   [T^{-1}]_{11} = -sinh(m theta) / (delta sinh((m+1) theta)),
//   [T^{-1}]_{1m} = -sinh(theta)   / (delta sinh((m+1) theta)),
// in the decaying form q = e^{-theta} (no overflow for long systems).
static void corner_inverse(double theta, int m, double delta, double* t11, double* t1m) {
  const double den = -std::expm1(-2.0 * (m + 1) * theta);
  *t11 = -(std::exp(-theta) * -std::expm1(-2.0 * m * theta) / den) / delta;
  *t1m = -(std::exp(-(double)m * theta) * -std::expm1(-2.0 * theta) / den) / delta;
}

std::shared_ptr<IkPlanTable> build_ik_table(int nx, int ny, double h, double kappa) {
  const double delta = 1.0 / (h * h);
  const double pi = 3.14159265358979323846;
  std::vector<double> host(4 * (size_t)nx + 4 * (size_t)ny);
  double* lamx = host.data();
  double* qx = lamx + nx;
  double* t00 = qx + nx;
  double* t0n = t00 + nx;
  double* lamy = t0n + nx;
  double* qy = lamy + ny;
  double* s00 = qy + ny;
  double* s0n = s00 + ny;
  // double-precision closed forms (relative errors of a few units in the
  // last place); theta from cosh(theta) = 1 + u, u = 2 sin^2(k pi/(2N)) -
  // kappa/(2 delta), without cancellation
  auto axis = [&](int n, int m, double* lam, double* q, double* c11, double* c1m) {
    const int N = n + 1;
    const double sq = std::sqrt(2.0 / N);
    for (int k = 1; k <= n; ++k) {
      const double sh = std::sin(pi * k / (2.0 * N));
      lam[k - 1] = -4.0 * delta * sh * sh;   // 2 delta (cos(k pi/N) - 1)
      q[k - 1] = sq * std::sin(pi * k / N);
      const double u = 2.0 * sh * sh - kappa / (2.0 * delta);
      if (!(u > 0.0))
        throw Error(FDS_E_UNSUPPORTED, "kappa makes a sine mode oscillatory (not diagonally dominant)");
      const double th = std::log1p(u + std::sqrt(u * (u + 2.0)));
      corner_inverse(th, m, delta, &c11[k - 1], &c1m[k - 1]);
    }
  };
  axis(nx, ny, lamx, qx, t00, t0n);   // x modes: systems of ny rows
  axis(ny, nx, lamy, qy, s00, s0n);   // y modes: systems of nx columns
  auto t = std::make_shared<IkPlanTable>();
  t->mem.alloc(sizeof(double) * host.size());
  upload(t->mem.get(), host.data(), sizeof(double) * host.size());
  const double* b = t->mem.as<double>(0);
  t->lamx = b;
  t->qx = b + nx;
  t->t00 = b + 2 * (size_t)nx;
  t->t0n = b + 3 * (size_t)nx;
  t->lamy = b + 4 * (size_t)nx;
  t->qy = t->lamy + ny;
  t->s00 = t->lamy + 2 * (size_t)ny;
  t->s0n = t->lamy + 3 * (size_t)ny;
  return t;
}

bool dense_lines(int n) {
  const char* e = std::getenv("FDS_LINES");
  const bool fft = e && std::string(e) == "fft";
  return !fft && n <= kDenseLineMax;
}

}  // namespace fds

namespace fds {

// Jacobi preconditioner of Section 3.2: D = diag(L_c) = diag(A_c) minus the
// diagonal of every arm's Schur term.  On a boundary line of length n the arm
// term is delta^2 [A_a^{-1}] restricted to its interface row, Q diag(g) Q in
// the line's sine basis, whose diagonal is sum_k gs_k sin^2(pi i k/N)
// (gs_k = delta^2 (2/N) g_k); a corner node collects the terms of both lines.
std::shared_ptr<DiagTable> build_jacobi_table(const fds_plan* p) {
  const int nx = p->nx, ny = p->ny;
  std::vector<double> d((size_t)nx * ny, -4.0 * p->delta + p->kappa);
  for (const ArmInfo& a : p->arms) {
    const int n = a.L, N = n + 1;
    const std::vector<double> gs = schur_gs_host(n, a.rows, p->h, p->kappa);
    for (int i = 1; i <= n; ++i) {
      long double acc = 0;
      for (int k = 1; k <= n; ++k) {
        const long double sn = sinl(kPi * (long double)((long long)i * k % (2LL * N)) / (long double)N);
        acc += (long double)gs[k - 1] * sn * sn;
      }
      size_t at = 0;
      switch (a.line) {
        case 0: at = (size_t)(i - 1); break;
        case 1: at = (size_t)(ny - 1) * nx + (i - 1); break;
        case 2: at = (size_t)(i - 1) * nx; break;
        default: at = (size_t)(i - 1) * nx + (nx - 1); break;
      }
      d[at] -= (double)acc;
    }
  }
  for (double& v : d) v = 1.0 / v;
  auto t = std::make_shared<DiagTable>();
  t->mem.alloc(sizeof(double) * d.size());
  upload(t->mem.get(), d.data(), sizeof(double) * d.size());
  t->dinv = t->mem.as<double>(0);
  return t;
}

}  // namespace fds
