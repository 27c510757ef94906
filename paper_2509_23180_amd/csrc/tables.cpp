// Device tables: FFT twiddles, per-mode tridiagonal coefficients and Schur
// line coefficients.  All values are computed on the host in FP64 (long
// double where the angle reduction benefits) and uploaded once.
#include <cmath>
#include <cstring>

#include "runtime.h"

namespace fds {

std::vector<int> fft_radices(int N) {
  std::vector<int> r;
  int n = N;
  while (n % 4 == 0) { r.push_back(4); n /= 4; }
  while (n % 2 == 0) { r.push_back(2); n /= 2; }
  while (n % 3 == 0) { r.push_back(3); n /= 3; }
  while (n % 5 == 0) { r.push_back(5); n /= 5; }
  for (int p = 7; n > 1; p += 2) {
    while (n % p == 0) { r.push_back(p); n /= p; }
    if ((long long)p * p > n && n > 1) { r.push_back(n); n = 1; }
  }
  if ((int)r.size() > kMaxPass) throw Error(FDS_E_UNSUPPORTED, "FFT length has too many factors");
  return r;
}

int dst_threads_per_row(int n) {
  const int N = n + 1;
  if (N <= 64) return 32;
  if (N <= 160) return 64;
  if (N <= 640) return 128;
  return 256;
}

size_t dst_smem_bytes(int n, bool fp32) {
  const int G = dst_threads_per_row(n);
  const int rpb = kBlock / G;
  return (size_t)rpb * 2 * (n + 1) * (fp32 ? sizeof(float2) : sizeof(double2));
}

TableCache& TableCache::get() {
  static TableCache c;
  return c;
}

static int current_device() {
  int d = 0;
  FDS_HIP(hipGetDevice(&d));
  return d;
}

static size_t align_up(size_t x, size_t a) { return (x + a - 1) / a * a; }

std::shared_ptr<FftTable> TableCache::fft(int n) {
  const int dev = current_device();
  std::lock_guard<std::mutex> lk(mu_);
  auto key = std::make_pair(dev, n);
  auto it = fft_.find(key);
  if (it != fft_.end()) return it->second;
  const int N = n + 1;
  auto t = std::make_shared<FftTable>();
  std::vector<int> rad = fft_radices(N);
  // layout: [FftDesc][tw64 N][tw32 N][post64 N+1][post32 N+1]
  size_t o_desc = 0;
  size_t o_tw64 = align_up(sizeof(FftDesc), 256);
  size_t o_tw32 = align_up(o_tw64 + sizeof(double2) * N, 256);
  size_t o_p64 = align_up(o_tw32 + sizeof(float2) * N, 256);
  size_t o_p32 = align_up(o_p64 + sizeof(double2) * (N + 1), 256);
  size_t total = align_up(o_p32 + sizeof(float2) * (N + 1), 256);
  std::vector<unsigned char> host(total, 0);
  auto* tw64 = reinterpret_cast<double2*>(host.data() + o_tw64);
  auto* tw32 = reinterpret_cast<float2*>(host.data() + o_tw32);
  auto* p64 = reinterpret_cast<double2*>(host.data() + o_p64);
  auto* p32 = reinterpret_cast<float2*>(host.data() + o_p32);
  const long double pi = 3.141592653589793238462643383279502884L;
  for (int t0 = 0; t0 < N; ++t0) {
    const long double a = 2.0L * pi * (long double)t0 / (long double)N;
    const double c = (double)cosl(a), s = (double)-sinl(a);
    tw64[t0] = double2{c, s};
    tw32[t0] = float2{(float)c, (float)s};
  }
  for (int k = 0; k <= N; ++k) {
    const long double a = pi * (long double)k / (long double)N;
    const double c = (double)cosl(a), s = (double)sinl(a);
    p64[k] = double2{c, s};
    p32[k] = float2{(float)c, (float)s};
  }
  t->mem.alloc(total);
  FftDesc d{};
  d.N = N;
  d.npass = (int)rad.size();
  for (size_t i = 0; i < rad.size(); ++i) d.radix[i] = rad[i];
  d.tw64 = t->mem.as<double2>(o_tw64);
  d.tw32 = t->mem.as<float2>(o_tw32);
  d.post64 = t->mem.as<double2>(o_p64);
  d.post32 = t->mem.as<float2>(o_p32);
  std::memcpy(host.data() + o_desc, &d, sizeof(d));
  FDS_HIP(hipMemcpy(t->mem.get(), host.data(), total, hipMemcpyHostToDevice));
  t->host = d;
  t->dev = t->mem.as<FftDesc>(o_desc);
  fft_[key] = t;
  return t;
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
  FDS_HIP(hipMemcpy(t->mem.get(), c64.data(), sizeof(ModeCoef<double>) * n, hipMemcpyHostToDevice));
  FDS_HIP(hipMemcpy(t->mem.as<char>(o32), c32.data(), sizeof(ModeCoef<float>) * n,
                    hipMemcpyHostToDevice));
  t->c64 = t->mem.as<ModeCoef<double>>(0);
  t->c32 = t->mem.as<ModeCoef<float>>(o32);
  return t;
}

std::shared_ptr<ModeTable> TableCache::modes(int n, int m, double h, double kappa) {
  const int dev = current_device();
  std::lock_guard<std::mutex> lk(mu_);
  auto key = std::make_tuple(dev, n, m, h, kappa);
  auto it = modes_.find(key);
  if (it != modes_.end()) return it->second;
  std::vector<ModeCoef<double>> c64;
  std::vector<ModeCoef<float>> c32;
  mode_coefs_host(n, m, h, kappa, 2.0 / (n + 1), c64, c32);
  auto t = upload_modes(c64, c32);
  modes_[key] = t;
  return t;
}

// Schur line coefficients of an arm with line length n and m rows (the
// interface row first):  g_k = [T_k^{-1}]_{11} = -sinh(m theta)/(delta sinh((m+1) theta))
//                           = -(q/delta) (1 - q^{2m})/(1 - q^{2m+2}),
// stored as delta^2 (2/N) g_k.
std::shared_ptr<GsTable> TableCache::gs(int n, int m, double h, double kappa) {
  const int dev = current_device();
  std::lock_guard<std::mutex> lk(mu_);
  auto key = std::make_tuple(dev, n, m, h, kappa);
  auto it = gs_.find(key);
  if (it != gs_.end()) return it->second;
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
  auto t = std::make_shared<GsTable>();
  t->mem.alloc(sizeof(double) * n);
  FDS_HIP(hipMemcpy(t->mem.get(), v.data(), sizeof(double) * n, hipMemcpyHostToDevice));
  t->gs = t->mem.as<double>(0);
  gs_[key] = t;
  return t;
}

}  // namespace fds
