// HIP kernels of the hot path (gfx950).  Every kernel works on a list of
// task records so one launch serves all rectangles / problems of a batch.
#include "kernels.h"
#include <algorithm>
#include <cstdio>
#include <cstdlib>
#include <map>
#include <mutex>

#include "fft_device.h"

namespace fds {

// =====================================================================
// Row sine transforms (forward and inverse are the same transform).
// T: arithmetic type; TIn / TOut: storage types of input and output.
// =====================================================================
template <typename T, typename TIn, typename TOut>
__global__ void __launch_bounds__(kBlock) k_dst_rows(const DstTask* __restrict__ tasks, int ntasks,
                                                      int jidx) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  __shared__ int slot;
  const DstTask& tk = tasks[find_task(tasks, ntasks, &slot)];
  if (tk.skip && *tk.skip) return;
  const FftDesc& f = *tk.fft;
  const int N = f.N;
  const int n = tk.n;
  const int G = kBlock / tk.rpb;
  const int grp = threadIdx.x / G;
  const int g = threadIdx.x - grp * G;
  const int row = (blockIdx.x - tk.block_begin) * tk.rpb + grp;
  const bool valid = row < tk.rows;
  C2<T>* twl = reinterpret_cast<C2<T>*>(smem_raw);
  C2<T>* A = twl + (tk.tw_lds ? f.L : 0) + (size_t)grp * 2 * f.W;
  C2<T>* B = A + f.W;
  const C2<T>* tw = stage_twiddles<T>(f, twl, tk.tw_lds != 0);
  const TIn* in = static_cast<const TIn*>(tk.in) + (long long)jidx * tk.in_js +
                  (long long)(valid ? row : 0) * tk.in_rs;
  const long long ics = tk.in_cs;
  if (tk.in_scale) {
    // normalise the basis vector while reading it and write it back once
    const double sc = *tk.in_scale;
    if (valid) dst_pack<T>(A, N, g, G, [&](int j) { return T(double(in[(long long)(j - 1) * ics]) * sc); });
    __syncthreads();
    if (valid) {
      TIn* inw = const_cast<TIn*>(in);
      for (int j = 1 + g; j <= n; j += G) {
        const double v = double(in[(long long)(j - 1) * ics]) * sc;
        inw[(long long)(j - 1) * ics] = TIn(v);
      }
    }
  } else if (valid) {
    dst_pack<T>(A, N, g, G, [&](int j) { return T(in[(long long)(j - 1) * ics]); });
  }
  __syncthreads();
  const C2<T>* Cr = fft_lds<T>(A, B, f, tw, g, G);
  if (valid) {
    TOut* out = static_cast<TOut*>(tk.out) + (long long)jidx * tk.out_js + (long long)row * tk.out_rs;
    const C2<T>* post = fft_post<T>(f);
    const T scale = T(tk.scale);
    for (int k = 1 + g; k <= n; k += G) {
      const T X = scale * dst_post<T>(Cr, post, N, k);
      TOut* o = out + (long long)(k - 1) * tk.out_cs;
      if (tk.accumulate) *o = TOut(T(*o) + X);
      else *o = TOut(X);
    }
  }
}


// =====================================================================
// Sine transform of rows as a product with the dense sine matrix on the
// matrix cores: out[r][c] = scale * sum_j x[r][j] S[j][c],
// S[j][c] = sin(pi (j+1)(c+1)/(n+1)).  A block takes RT*16 rows of x into
// LDS; wave w accumulates the 16x16 tiles of columns [w*CT*16, (w+1)*CT*16)
// with v_mfma_*_16x16x4 (A lane l: A[l%16][l/16], B lane l: B[l/16][l%16]).
// =====================================================================
typedef double v4d_t __attribute__((ext_vector_type(4)));
typedef float v4f_t __attribute__((ext_vector_type(4)));

template <typename T> struct MfmaAcc;
template <> struct MfmaAcc<double> { using t = v4d_t; };
template <> struct MfmaAcc<float> { using t = v4f_t; };

__device__ __forceinline__ v4d_t mfma16x16x4(double a, double b, v4d_t c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}
__device__ __forceinline__ v4f_t mfma16x16x4(float a, float b, v4f_t c) {
  return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}
// row of register v of lane l in the 16x16 result tile
template <typename T> __device__ __forceinline__ int mfma_row(int l, int v);
template <> __device__ __forceinline__ int mfma_row<double>(int l, int v) { return 4 * v + (l >> 4); }
template <> __device__ __forceinline__ int mfma_row<float>(int l, int v) { return 4 * (l >> 4) + v; }

template <typename T> __device__ __forceinline__ const T* fft_smat(const FftDesc& f);
template <> __device__ __forceinline__ const double* fft_smat<double>(const FftDesc& f) { return f.smat64; }
template <> __device__ __forceinline__ const float* fft_smat<float>(const FftDesc& f) { return f.smat32; }

template <typename T, typename TIn, typename TOut, int RT, int CT>
__global__ void __launch_bounds__(kBlock) k_dst_gemm(const DstTask* __restrict__ tasks, int ntasks,
                                                      int jidx) {
  using Acc = typename MfmaAcc<T>::t;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  __shared__ int slot;
  const DstTask& tk = tasks[find_task(tasks, ntasks, &slot)];
  if (tk.skip && *tk.skip) return;
  const FftDesc& f = *tk.fft;
  const int n = tk.n;
  const int np = f.np;
  const int ld = np + 1;                      // padded LDS row stride
  constexpr int RB = RT * 16;
  T* xs = reinterpret_cast<T*>(smem_raw);     // RB x ld
  const int r0 = (blockIdx.x - tk.block_begin) * RB;
  const TIn* in = static_cast<const TIn*>(tk.in) + (long long)jidx * tk.in_js;
  const double sc_in = tk.in_scale ? *tk.in_scale : 1.0;
  TIn* inw = const_cast<TIn*>(in);
  for (int e = threadIdx.x; e < RB * np; e += kBlock) {
    const int r = e / np, j = e - (e / np) * np;
    const int row = r0 + r;
    T v = T(0);
    if (row < tk.rows && j < n) {
      const long long a = (long long)row * tk.in_rs + (long long)j * tk.in_cs;
      const double x = double(in[a]) * sc_in;
      if (tk.in_scale) inw[a] = TIn(x);
      v = T(x);
    }
    xs[r * ld + j] = v;
  }
  __syncthreads();
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const T* S = fft_smat<T>(f);
  const int ar = lane & 15, ak = lane >> 4;
  TOut* out = static_cast<TOut*>(tk.out) + (long long)jidx * tk.out_js;
  const T scale = T(tk.scale);
  for (int cbase = 0; cbase < np; cbase += 4 * CT * 16) {
    const int c0 = cbase + wave * CT * 16;
    if (c0 >= np) break;
    Acc acc[RT][CT];
#pragma unroll
    for (int a = 0; a < RT; ++a)
#pragma unroll
      for (int b = 0; b < CT; ++b) acc[a][b] = Acc{T(0), T(0), T(0), T(0)};
    const T* Sl = S + (long long)ak * np + c0 + ar;
    for (int k0 = 0; k0 < np; k0 += 4) {
      T bv[CT];
#pragma unroll
      for (int b = 0; b < CT; ++b) bv[b] = (c0 + b * 16 < np) ? Sl[(long long)k0 * np + b * 16] : T(0);
#pragma unroll
      for (int a = 0; a < RT; ++a) {
        const T av = xs[(a * 16 + ar) * ld + k0 + ak];
#pragma unroll
        for (int b = 0; b < CT; ++b) acc[a][b] = mfma16x16x4(av, bv[b], acc[a][b]);
      }
    }
#pragma unroll
    for (int a = 0; a < RT; ++a)
#pragma unroll
      for (int b = 0; b < CT; ++b)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int row = r0 + a * 16 + mfma_row<T>(lane, v);
          const int col = c0 + b * 16 + ar;
          if (row < tk.rows && col < n) {
            TOut* o = out + (long long)row * tk.out_rs + (long long)col * tk.out_cs;
            const T X = scale * acc[a][b][v];
            if (tk.accumulate) *o = TOut(T(*o) + X);
            else *o = TOut(X);
          }
        }
  }
}

// =====================================================================
// Per-mode tridiagonal solves, one lane per mode, in place.
//   forward:  w_i = sc r_i + q w_{i-1},   s = sum q^{i-1} w_i
//   backward: y_i = w_i - gamma q^{i-1} + q y_{i+1},  gamma = beta s
// =====================================================================
template <typename T>
__global__ void __launch_bounds__(kBlock) k_tridiag(const TriTask* __restrict__ tasks, int ntasks,
                                                     int jidx) {
  __shared__ int slot;
  const TriTask& tk = tasks[find_task(tasks, ntasks, &slot)];
  if (tk.skip && *tk.skip) return;
  const int k = (blockIdx.x - tk.block_begin) * kBlock + threadIdx.x;
  if (k >= tk.modes) return;
  const ModeCoef<T> c = static_cast<const ModeCoef<T>*>(tk.coef)[k];
  T* d = static_cast<T*>(tk.data) + (long long)jidx * tk.js + k;
  const long long rs = tk.rs;
  const int m = tk.rows;
  double* v = tk.vin ? tk.vin + (long long)jidx * tk.vjs + k : nullptr;
  const double sc = tk.vin ? *tk.vscale : 1.0;
  T w = T(0), s = T(0), p = T(1);
#pragma unroll 4
  for (int i = 0; i < m; ++i) {
    T r;
    if (v) {
      const double a = v[i * rs] * sc;
      v[i * rs] = a;
      r = T(a);
    } else {
      r = d[i * rs];
    }
    if (tk.identity) {   // no preconditioner: z^ = v^
      d[i * rs] = r;
      continue;
    }
    w = c.sc * r + c.q * w;
    d[i * rs] = w;
    s += p * w;
    p *= c.q;
  }
  if (tk.identity) return;
  const T gam = c.beta * s;
  T y = T(0);
  p = T(0);
#pragma unroll 4
  for (int i = m - 1; i >= 0; --i) {
    p = (i > c.K) ? T(0) : ((i == c.K) ? c.qK : p * c.qinv);
    y = d[i * rs] - gam * p + c.q * y;
    d[i * rs] = y;
  }
}


// Segmented variant: a block serves MPB consecutive modes and splits the rows
// into segments of LS rows held in registers, one segment per thread
// (thread t: mode t % MPB, segment t / MPB).  Both first-order recurrences
// are solved per segment with a zero carry; the carries follow in closed form
// (constant coefficient q):
//   forward  w_{i0+t} = w_loc_t + q^{t+1} c,        c = w_{i0-1}
//            sum_i q^i w_i = sum_s q^{i0}(A_s + c_s q (1-q^{2L})/(1-q^2))
//   backward y_{i0+t} = y_loc_t + q^{L-t} d,        d = y_{i0+L}
// so the data is read once and written once.
// Threads per block of a segment length: 32-row segments keep up to 64
// values per thread in registers, which needs more than the 128 VGPRs a
// 1024-thread block leaves each thread (576 threads: 8 modes x 72 segments,
// systems of up to 2304 rows, at three wavefronts per SIMD).
constexpr int kTriMaxThreadsLong = 576;
template <int LS>
constexpr int tri_max_threads() { return LS >= 32 ? kTriMaxThreadsLong : 1024; }

template <typename T, int LS, int MPB>
__global__ void __launch_bounds__(tri_max_threads<LS>()) k_tridiag_seg(const TriTask* __restrict__ tasks,
                                                                       int ntasks, int jidx) {
  constexpr int SEGMAX = 1024 / MPB;
  __shared__ int slot;
  __shared__ T sa[SEGMAX][MPB];
  __shared__ T sb[SEGMAX][MPB];
  __shared__ T sg[MPB];
  const TriTask& tk = tasks[find_task(tasks, ntasks, &slot)];
  if (tk.skip && *tk.skip) return;
  const int lane = threadIdx.x % MPB;
  const int s = threadIdx.x / MPB;
  const int m = tk.rows;
  const int S = (m + LS - 1) / LS;
  const int k = (blockIdx.x - tk.block_begin) * MPB + lane;
  const bool act = k < tk.modes && s < S;
  const int i0 = s * LS;
  const int L = act ? min(LS, m - i0) : 0;
  ModeCoef<T> c{};
  if (k < tk.modes) c = static_cast<const ModeCoef<T>*>(tk.coef)[k];
  const int rs = (int)tk.rs;
  T* d = static_cast<T*>(tk.data) + (long long)jidx * tk.js + (long long)i0 * rs + (k < tk.modes ? k : 0);
  T x[LS];
  // a full segment loads (and stores) without per-row guards, so all LS
  // loads of a thread are in flight together
  const bool full = L == LS;
  if (tk.vin) {
    double* v = tk.vin + (long long)jidx * tk.vjs + (long long)i0 * rs + (k < tk.modes ? k : 0);
    const double sc = *tk.vscale;
    double a[LS];
    if (full) {
#pragma unroll
      for (int t = 0; t < LS; ++t) a[t] = v[t * rs];
#pragma unroll
      for (int t = 0; t < LS; ++t) {
        a[t] *= sc;
        v[t * rs] = a[t];
        x[t] = T(a[t]);
      }
    } else {
#pragma unroll
      for (int t = 0; t < LS; ++t) {
        if (t < L) {
          a[t] = v[t * rs] * sc;
          v[t * rs] = a[t];
          x[t] = T(a[t]);
        } else {
          x[t] = T(0);
        }
      }
    }
  } else if (full) {
#pragma unroll
    for (int t = 0; t < LS; ++t) x[t] = d[t * rs];
  } else {
#pragma unroll
    for (int t = 0; t < LS; ++t) x[t] = (t < L) ? d[t * rs] : T(0);
  }
  if (tk.identity) {   // no preconditioner: z^ = v^
#pragma unroll
    for (int t = 0; t < LS; ++t)
      if (full || t < L) d[t * rs] = x[t];
    return;
  }
  // local forward sweep
  T w = T(0), A = T(0), p = T(1);
#pragma unroll
  for (int t = 0; t < LS; ++t) {
    if (full || t < L) {
      w = c.sc * x[t] + c.q * w;
      x[t] = w;
      A += p * w;
      p *= c.q;
    }
  }
  if (act) {
    sa[s][lane] = w;
    sb[s][lane] = A;
  }
  __syncthreads();
  // The carries run serially over the S segments of a mode.  Their LDS inputs
  // do not depend on the carry, so they are read eight segments at a time
  // (SEGMAX is a multiple of 8: the reads past S stay inside the arrays and
  // go unused); only the last segment can be shorter than LS.
  static_assert(SEGMAX % 8 == 0, "segment chunks of 8");
  const int Llast = m - (S - 1) * LS;
  if (s == 0 && k < tk.modes) {
    // forward carries, the first-row weight sum and gamma
    T qLf = T(1), Bf = T(0), q2 = c.q;
    for (int t = 0; t < LS; ++t) { Bf += q2; q2 *= c.q * c.q; qLf *= c.q; }
    T qLl = T(1), Bl = T(0);
    q2 = c.q;
    for (int t = 0; t < Llast; ++t) { Bl += q2; q2 *= c.q * c.q; qLl *= c.q; }
    T carry = T(0), qi0 = T(1), stot = T(0);
    for (int s0 = 0; s0 < S; s0 += 8) {
      T E[8], As[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        E[u] = sa[s0 + u][lane];
        As[u] = sb[s0 + u][lane];
      }
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        const int ss = s0 + u;
        if (ss < S) {
          const bool last = ss == S - 1;
          const T qL = last ? qLl : qLf, B = last ? Bl : Bf;
          stot += qi0 * (As[u] + carry * B);
          sa[ss][lane] = carry;
          sb[ss][lane] = qi0;
          carry = E[u] + qL * carry;
          qi0 *= qL;
        }
      }
    }
    sg[lane] = c.beta * stot;
  }
  __syncthreads();
  T y = T(0);
  if (act) {
    const T cin = sa[s][lane], qi0 = sb[s][lane], gam = sg[lane];
    T pc = c.q, pg = qi0;
#pragma unroll
    for (int t = 0; t < LS; ++t) {
      if (full || t < L) {
        x[t] = x[t] + pc * cin - gam * pg;
        pc *= c.q;
        pg *= c.q;
      }
    }
#pragma unroll
    for (int t = LS - 1; t >= 0; --t) {
      if (full || t < L) {
        y = x[t] + c.q * y;
        x[t] = y;
      }
    }
    sa[s][lane] = y;
  }
  __syncthreads();
  if (s == 0 && k < tk.modes) {
    T qLf = T(1), qLl = T(1);
    for (int t = 0; t < LS; ++t) qLf *= c.q;
    for (int t = 0; t < Llast; ++t) qLl *= c.q;
    T dc = T(0);
    for (int s0 = ((S - 1) / 8) * 8; s0 >= 0; s0 -= 8) {
      T D[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) D[u] = sa[s0 + u][lane];
#pragma unroll
      for (int u = 7; u >= 0; --u) {
        const int ss = s0 + u;
        if (ss < S) {
          const T qL = ss == S - 1 ? qLl : qLf;
          sb[ss][lane] = dc;
          dc = D[u] + qL * dc;
        }
      }
    }
  }
  __syncthreads();
  if (act) {
    const T din = sb[s][lane];
    T pw = c.q;
#pragma unroll
    for (int t = LS - 1; t >= 0; --t) {
      if (full || t < L) {
        x[t] += pw * din;
        pw *= c.q;
      }
    }
#pragma unroll
    for (int t = 0; t < LS; ++t)
      if (full || t < L) d[t * rs] = x[t];
  }
}


// =====================================================================
// Schur line terms: out = delta^2 (2/N) S diag(g) S z_line (FP64).
// One block per line; two sine transforms in LDS.  Used by the kernel-level
// operator entry point; the solver forms these terms with the batched row
// transforms, which spread a line over many lanes and take the autotuner's
// schedule.
// =====================================================================
__global__ void __launch_bounds__(kBlock) k_schur_lines(const LineTask* __restrict__ tasks, int jidx) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  const LineTask& tk = tasks[blockIdx.x];
  if (tk.skip && *tk.skip) return;
  const FftDesc& f = *tk.fft;
  const int N = f.N;
  const int L = tk.L;
  double2* twl = reinterpret_cast<double2*>(smem_raw);
  double2* A = twl + f.L;
  double2* B = A + f.W;
  double* mid = reinterpret_cast<double*>(B + f.W);
  const double2* tw = stage_twiddles<double>(f, twl, true);
  const int g = threadIdx.x;
  const long long st = tk.stride;
  if (tk.z_f32) {
    const float* z = static_cast<const float*>(tk.z) + (long long)jidx * tk.z_js + tk.start;
    dst_pack<double>(A, N, g, kBlock, [&](int j) { return double(z[(long long)(j - 1) * st]); });
  } else {
    const double* z = static_cast<const double*>(tk.z) + (long long)jidx * tk.z_js + tk.start;
    dst_pack<double>(A, N, g, kBlock, [&](int j) { return z[(long long)(j - 1) * st]; });
  }
  __syncthreads();
  const double2* C = fft_lds<double>(A, B, f, tw, g, kBlock);
  for (int k = 1 + g; k <= L; k += kBlock) mid[k - 1] = tk.gs[k - 1] * dst_post<double>(C, f.post64, N, k);
  __syncthreads();
  dst_pack<double>(A, N, g, kBlock, [&](int j) { return mid[j - 1]; });
  __syncthreads();
  C = fft_lds<double>(A, B, f, tw, g, kBlock);
  for (int k = 1 + g; k <= L; k += kBlock) tk.out[k - 1] = dst_post<double>(C, f.post64, N, k);
}

// Schur line terms as dense products with the precomputed line operator:
// out_i = sum_k M(k, i) v_k, v the line of z.  A block covers 64 outputs of one line; its four
// wavefronts take quarters of k and are added in a fixed order.
__global__ void __launch_bounds__(kBlock) k_lines_dense(const LineTask* __restrict__ tasks,
                                                         int ntasks, int jidx) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  __shared__ int slot;
  __shared__ double part[4][64];
  const LineTask& tk = tasks[find_task(tasks, ntasks, &slot)];
  if (tk.skip && *tk.skip) return;
  const int L = tk.L;
  double* v = reinterpret_cast<double*>(smem_raw);
  const long long base = (long long)jidx * tk.z_js + tk.start;
  for (int k = threadIdx.x; k < L; k += kBlock) {
    const long long idx = base + (long long)k * tk.stride;
    v[k] = tk.z_f32 ? double(static_cast<const float*>(tk.z)[idx]) : static_cast<const double*>(tk.z)[idx];
  }
  __syncthreads();
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int i = (blockIdx.x - tk.block_begin) * 64 + lane;
  const int q = (L + 3) / 4;
  const int k0 = min(L, wave * q), k1 = min(L, k0 + q);
  double a[8] = {0, 0, 0, 0, 0, 0, 0, 0};
  if (i < L) {
    const double* m = tk.mat + i;
    int k = k0;
    for (; k + 7 < k1; k += 8) {
#pragma unroll
      for (int u = 0; u < 8; ++u) a[u] = fma(m[(long long)(k + u) * L], v[k + u], a[u]);
    }
    for (; k < k1; ++k) a[0] = fma(m[(long long)k * L], v[k], a[0]);
  }
  part[wave][lane] = ((a[0] + a[1]) + (a[2] + a[3])) + ((a[4] + a[5]) + (a[6] + a[7]));
  __syncthreads();
  if (wave == 0 && i < L) tk.out[i] = (part[0][lane] + part[1][lane]) + (part[2][lane] + part[3][lane]);
}

// Boundary columns of z = S y (see ColTask): one wave per row.
__global__ void __launch_bounds__(kBlock) k_idst_cols(const ColTask* __restrict__ tasks, int ntasks,
                                                       int jidx) {
  __shared__ int slot;
  const ColTask& tk = tasks[find_task(tasks, ntasks, &slot)];
  if (tk.skip && *tk.skip) return;
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int r = (blockIdx.x - tk.block_begin) * (kBlock / 64) + wave;
  if (r >= tk.ny) return;
  const double2* post = tk.fft->post64;
  double odd = 0.0, even = 0.0;   // k odd / k even (k = 1..nx)
  if (tk.y32) {
    const float* y = tk.y32 + (long long)jidx * tk.y_js + (long long)r * tk.nx;
    #pragma unroll 4
    for (int k = 1 + lane; k <= tk.nx; k += 64) {
      const double v = double(y[k - 1]) * post[k].y;
      if (k & 1) odd += v;
      else even += v;
    }
  } else {
    const double* y = tk.y + (long long)r * tk.nx;
    #pragma unroll 4
    for (int k = 1 + lane; k <= tk.nx; k += 64) {
      const double v = y[k - 1] * post[k].y;
      if (k & 1) odd += v;
      else even += v;
    }
  }
  odd = wave_sum(odd);
  even = wave_sum(even);
  if (lane == 0) {
    if (tk.zw) tk.zw[r] = tk.scale * (odd + even);
    if (tk.ze) tk.ze[r] = tk.scale * (odd - even);
  }
  if (tk.bc) {
    const double* v = tk.v + (long long)jidx * tk.Nc + (long long)r * tk.nx;
    double vo = 0.0, ve = 0.0;
    #pragma unroll 4
    for (int k = 1 + lane; k <= tk.nx; k += 64) {
      const double x = v[k - 1] * post[k].y;
      if (k & 1) vo += x;
      else ve += x;
    }
    vo = wave_sum(vo);
    ve = wave_sum(ve);
    if (lane == 0) {
      double* bc = tk.bc + (long long)2 * tk.ny * jidx;
      bc[r] = tk.scale * (vo + ve);
      bc[tk.ny + r] = tk.scale * (vo - ve);
    }
  }
}

// =====================================================================
// Centre operator (5-point stencil with zero data outside the centre, minus
// the Schur line terms).  mode 0: out = L_c z.  mode 1: out = f' - L_c z,
// with block partial sums of out^2 and z^2.
// =====================================================================
template <int MODE>
__global__ void __launch_bounds__(kBlock) k_operator(const OpTask* __restrict__ tasks, int ntasks,
                                                      int jidx) {
  __shared__ int slot;
  __shared__ double red[4];
  const OpTask& tk = tasks[find_task(tasks, ntasks, &slot)];
  if (tk.skip && *tk.skip) return;
  const int b = blockIdx.x - tk.block_begin;
  const int nx = tk.nx, ny = tk.ny;
  const long long Nc = (long long)nx * ny;
  const double d = tk.delta;
  const double diag = tk.kappa - 4.0 * d;
  double* out = tk.out + (long long)jidx * tk.out_js;
  double rr = 0.0, zz = 0.0;
  const long long base = (long long)b * kVecPerBlock;
  auto body = [&](auto zp) {
    for (int e = 0; e < kVecEPT; ++e) {
      const long long idx = base + (long long)e * kBlock + threadIdx.x;
      if (idx >= Nc) break;
      const int r = (int)(idx / nx);
      const int c = (int)(idx - (long long)r * nx);
      const double zc = double(zp[idx]);
      double nb = 0.0;
      if (c > 0) nb += double(zp[idx - 1]);
      if (c < nx - 1) nb += double(zp[idx + 1]);
      if (r > 0) nb += double(zp[idx - nx]);
      if (r < ny - 1) nb += double(zp[idx + nx]);
      double w = d * nb + diag * zc;
      if (r == 0 && tk.line[0]) w -= tk.line[0][c];
      if (r == ny - 1 && tk.line[1]) w -= tk.line[1][c];
      if (c == 0 && tk.line[2]) w -= tk.line[2][r];
      if (c == nx - 1 && tk.line[3]) w -= tk.line[3][r];
      if (MODE == 0) {
        out[idx] = w;
      } else {
        const double res = tk.fp[idx] - w;
        out[idx] = res;
        rr += res * res;
        zz += zc * zc;
      }
    }
  };
  if (tk.z_f32) body(static_cast<const float*>(tk.z) + (long long)jidx * tk.z_js);
  else body(static_cast<const double*>(tk.z) + (long long)jidx * tk.z_js);
  if (MODE == 1) {
    const double s1 = block_sum(rr, red);
    const double s2 = block_sum(zz, red);
    if (threadIdx.x == 0) {
      tk.partials[b] = s1;
      tk.partials[tk.nblocks + b] = s2;
    }
  }
}

// =====================================================================
// Arnoldi step j with modified Gram-Schmidt in compact (one-reduction) form
// (Swirydowicz, Langou, Ananthan, Yang, Thomas, "Low synchronization
// Gram-Schmidt and GMRES algorithms", 2021).  MGS takes
//   h_i = <w - sum_{l<i} h_l v_l, v_i> = <w, v_i> - sum_{l<i} h_l <v_l, v_i>,
// so one pass computing the Gram column <v_i, v_j> and the projections
// <w, v_i>, a triangular recurrence and one update pass give the same
// coefficients as the i-by-i passes.
// w is either stored in V[j+1] (flexible variant: w = L_c z_j) or implicit,
// w = v_j - s with s the Schur line terms on the boundary lines (plain
// variant: L_c A_c^{-1} v = v - S A_c^{-1} v).
// =====================================================================
__device__ __forceinline__ double line_term(const KryTask& tk, long long idx) {
  // (the centre has fewer than 2^32 nodes)
  const unsigned ui = (unsigned)idx, unx = (unsigned)tk.nx;
  const int r = (int)(ui / unx);
  const int c = (int)(ui - (unsigned)r * unx);
  double s = 0.0;
  if (tk.post) {
    // sine basis of the centre: (Q s)[r][k] with the S/N blocks diagonal,
    // (N/2) gs_k z^[r][k], and the W/E terms spread along the row by
    // Q e_1 = sqrt(2/N) sin(pi k/N), Q e_nx = (-1)^(k+1) sqrt(2/N) sin(pi k/N)
    if (r == 0 && tk.gs[0]) s += tk.half_n * tk.gs[0][c] * tk.zhat[c];
    if (r == tk.ny - 1 && tk.gs[1]) s += tk.half_n * tk.gs[1][c] * tk.zhat[idx];
    if (tk.line[2] || tk.line[3]) {
      const double q = tk.qscale * tk.post[c + 1].y;
      if (tk.line[2]) s += q * tk.line[2][r];
      if (tk.line[3]) s += ((c & 1) ? -q : q) * tk.line[3][r];
    }
    return s;
  }
  if (r == 0 && tk.line[0]) s += tk.line[0][c];
  if (r == tk.ny - 1 && tk.line[1]) s += tk.line[1][c];
  if (c == 0 && tk.line[2]) s += tk.line[2][r];
  if (c == tk.nx - 1 && tk.line[3]) s += tk.line[3][r];
  return s;
}

// w^[r][k] of the flexible variant's operator Q L_c Q^T z^_j at element idx,
// in the orthonormal sine basis of the centre's x direction (coefficients of
// row r at r nx + k - 1):
//   w^[r][k] = d (z^[r-1][k] + z^[r+1][k]) + (kappa - 4 d + 2 d cos(pi k/N)) z^[r][k]
//             - [r = 0] (N/2) gsS[k-1] z^[0][k] - [r = ny-1] (N/2) gsN[k-1] z^[ny-1][k]
//             - sqrt(2/N) sin(pi k/N) sW[r] - sqrt(2/N) sin(pi k nx/N) sE[r]:
// the S/N Schur blocks are diagonal in this basis and the W/E line terms
// (physical, from the dense line operators) enter as rank-one terms per row.
__device__ __forceinline__ double spec_w(const KryTask& tk, int j, long long idx) {
  const unsigned ui = (unsigned)idx, unx = (unsigned)tk.nx;
  const int r = (int)(ui / unx);
  const int c = (int)(ui - (unsigned)r * unx);
  const float* z = tk.Z + (long long)j * tk.Nc;
  const double2 cs = tk.post[c + 1];
  const double zc = double(z[idx]);
  double nb = 0.0;
  if (r > 0) nb += double(z[idx - tk.nx]);
  if (r < tk.ny - 1) nb += double(z[idx + tk.nx]);
  const double d = tk.delta;
  double w = d * nb + (tk.kappa - 4.0 * d + 2.0 * d * cs.x) * zc;
  if (r == 0 && tk.gs[0]) w -= tk.half_n * tk.gs[0][c] * zc;
  if (r == tk.ny - 1 && tk.gs[1]) w -= tk.half_n * tk.gs[1][c] * zc;
  if (tk.line[2]) w -= tk.qscale * cs.y * tk.line[2][r];
  if (tk.line[3]) w -= tk.qscale * ((c & 1) ? -cs.y : cs.y) * tk.line[3][r];
  return w;
}

// Row sums out[d] = sum_{q < ncols} src[d * ld + q] for d < D <= blockDim.x,
// with the whole block: each row is cut into C = blockDim.x / D contiguous
// chunks whose loads are issued eight at a time, and the chunk sums are added
// in chunk order (a fixed order).  scratch holds blockDim.x doubles; out is
// in LDS and is complete when the function returns.
__device__ void reduce_rows(const double* src, long long ld, int D, int ncols, double* scratch,
                            double* out) {
  const int T = blockDim.x;
  int C = T / D;
  if (C > ncols) C = ncols;
  if (C < 1) C = 1;
  const int chunk = (ncols + C - 1) / C;
  const int e = threadIdx.x;
  double s = 0.0;
  if (e < D * C) {
    const int d = e / C, c = e - d * C;
    const int q0 = c * chunk;
    const int q1 = min(ncols, q0 + chunk);
    const double* p = src + (long long)d * ld;
    int q = q0;
    for (; q + 8 <= q1; q += 8) {
      double v[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) v[u] = ld_agent(p + q + u);
#pragma unroll
      for (int u = 0; u < 8; ++u) s += v[u];
    }
    for (; q < q1; ++q) s += ld_agent(p + q);
  }
  scratch[e] = s;
  __syncthreads();
  if (e < D) {
    double t = 0.0;
    for (int c = 0; c < C; ++c) t += scratch[e * C + c];
    out[e] = t;
  }
  __syncthreads();
}

__device__ void gram_recur(const KryTask& tk, int j, double* lds);

// Gram column and MGS coefficients of step j from the dot sums (row t of
// `src`, ncols entries at src + t ld): G[:, j] = <v_i, v_j>, a_i = <w, v_i>,
// h_i = a_i - sum_{l<i} h_l G_li.  The recurrence runs in LDS: after h_l is
// final every i > l subtracts h_l G_li in parallel.
// lds: 3 (j+1) + j (j+1)/2 doubles; scratch: blockDim.x doubles.
__device__ void gram_solve_block(const KryTask& tk, int j, double* lds, const double* src, long long ld,
                                 int ncols, double* scratch) {
  const int nd = j + 1;
  const int m1 = tk.m + 1;
  double* dots = lds;                 // 2 nd
  double* a = dots + 2 * nd;          // nd
  double* Gt = a + nd;                // column i of the strict upper triangle at i (i - 1) / 2
  reduce_rows(src, ld, 2 * nd, ncols, scratch, dots);
  gram_recur(tk, j, lds);
}

// The MGS recurrence of step j from dots[0, nd) = G[:, j] and dots[nd, 2 nd)
// = <v_i, u> in LDS (layout as in gram_solve_block); writes G[:, j], hv and
// column j of H.
__device__ void gram_recur(const KryTask& tk, int j, double* lds) {
  const int nd = j + 1;
  const int m1 = tk.m + 1;
  double* dots = lds;
  double* a = dots + 2 * nd;
  double* Gt = a + nd;
  const int ntri = nd * (nd - 1) / 2;
  for (int e = threadIdx.x; e < ntri; e += blockDim.x) {
    int i = (int)((1.0 + sqrt(1.0 + 8.0 * e)) * 0.5);
    while (i * (i - 1) / 2 > e) --i;
    while ((i + 1) * i / 2 <= e) ++i;
    const int l = e - i * (i - 1) / 2;
    Gt[e] = (i < j) ? tk.G[l + i * m1] : -1.0;
  }
  __syncthreads();
  for (int t = threadIdx.x; t < nd; t += blockDim.x) {
    tk.G[t + j * m1] = dots[t];
    a[t] = tk.implicit_w ? dots[t] - dots[nd + t] : dots[nd + t];
  }
  for (int l = threadIdx.x; l < j; l += blockDim.x) Gt[j * (j - 1) / 2 + l] = dots[l];
  __syncthreads();
  if (nd <= 64) {
    // one wavefront, lane i holding a_i: after step l, h_l is final and is
    // broadcast by a lane shuffle (no workgroup barriers); the subtractions
    // run in the same order as below
    if (threadIdx.x < 64) {
      const int i = threadIdx.x;
      double ai = i < nd ? a[i] : 0.0;
      for (int l = 0; l + 1 < nd; ++l) {
        const double hl = __shfl(ai, l, 64);
        if (i > l && i < nd) ai -= hl * Gt[i * (i - 1) / 2 + l];
      }
      if (i < nd) {
        tk.hv[i] = ai;
        tk.H[i + j * m1] = ai;
      }
    }
    return;
  }
  for (int l = 0; l < nd; ++l) {
    const double hl = a[l];
    __syncthreads();
    for (int i = l + 1 + threadIdx.x; i < nd; i += blockDim.x) a[i] -= hl * Gt[i * (i - 1) / 2 + l];
    __syncthreads();
  }
  for (int i = threadIdx.x; i < nd; i += blockDim.x) {
    tk.hv[i] = a[i];
    tk.H[i + j * m1] = a[i];
  }
}

// Block partials of <v_i, v_j> (i <= j) and of <v_i, u> with u = w when w is
// stored, u = s (the Schur line terms, zero off the boundary) otherwise; the
// problem's last block then forms the Gram column and the coefficients.
__global__ void __launch_bounds__(kBlock) k_gram_dots(const KryTask* __restrict__ tasks, int ntasks,
                                                       int j) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  __shared__ int slot;
  __shared__ int lastf;
  __shared__ double red[2 * 121][4];
  const KryTask& tk = tasks[find_task(tasks, ntasks, &slot)];
  if (tk.st->cycle_done) return;
  const int b = blockIdx.x - tk.block_begin;
  const long long Nc = tk.Nc;
  const long long base = (long long)b * kVecPerBlock;
  const bool stored = !tk.implicit_w;
  double xj[kVecEPT], uv[kVecEPT];
  const double* vj = tk.V + (long long)j * Nc;
  double* w = tk.V + (long long)(j + 1) * Nc;
  if (tk.fuse_op) {
    // flexible variant: w = Q L_c Q^T z^_j formed and stored here
#pragma unroll
    for (int e = 0; e < kVecEPT; ++e) {
      const long long idx = base + (long long)e * kBlock + threadIdx.x;
      const bool ok = idx < Nc;
      xj[e] = ok ? vj[idx] : 0.0;
      uv[e] = ok ? spec_w(tk, j, idx) : 0.0;
      if (ok) w[idx] = uv[e];
    }
  } else {
#pragma unroll
    for (int e = 0; e < kVecEPT; ++e) {
      const long long idx = base + (long long)e * kBlock + threadIdx.x;
      const bool ok = idx < Nc;
      xj[e] = ok ? vj[idx] : 0.0;
      uv[e] = !ok ? 0.0 : (stored ? w[idx] : line_term(tk, idx));
    }
  }
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  for (int i = 0; i <= j; ++i) {
    const double* vi = tk.V + (long long)i * Nc;
    double a = 0.0, c = 0.0;
#pragma unroll
    for (int e = 0; e < kVecEPT; ++e) {
      const long long idx = base + (long long)e * kBlock + threadIdx.x;
      const double v = (i == j) ? xj[e] : ((idx < Nc) ? vi[idx] : 0.0);
      a += v * xj[e];
      c += v * uv[e];
    }
    a = wave_sum_last(a);
    c = wave_sum_last(c);
    if (lane == 63) {
      red[i][wave] = a;
      red[121 + i][wave] = c;
    }
  }
  __syncthreads();
  const int nd = j + 1;
  for (int t = threadIdx.x; t < 2 * nd; t += kBlock) {
    const int row = t < nd ? t : 121 + (t - nd);
    const double s = (red[row][0] + red[row][1]) + (red[row][2] + red[row][3]);
    st_agent(tk.partials + (size_t)(kPartDots + t) * tk.P + b, s);
  }
  // Two-level fixed-order reduction: the last block of each group of
  // kGramGroup blocks sums the group's partials; the last group to finish
  // sums the group sums and solves.  One group: the partials directly.
  double* lds = reinterpret_cast<double*>(smem_raw);
  double* scratch = &red[0][0];
  const int P = tk.P;
  const double* part = tk.partials + (size_t)kPartDots * P;
  const int ng = gram_groups(P);
  if (ng == 1) {
    if (last_block_of_problem(&tk.st->ctr_dots, P, &lastf)) gram_solve_block(tk, j, lds, part, P, P, scratch);
    return;
  }
  double* gsum = tk.partials + (size_t)(2 * (tk.m + 1) + 4) * P;
  int* gctr = reinterpret_cast<int*>(gsum + (size_t)2 * (tk.m + 1) * ng);
  const int g = b / kGramGroup;
  const int gb = min(kGramGroup, P - g * kGramGroup);
  if (!last_block_of_problem(gctr + g, gb, &lastf)) return;
  reduce_rows(part + g * kGramGroup, P, 2 * nd, gb, scratch, lds);
  for (int t = threadIdx.x; t < 2 * nd; t += kBlock) st_agent(gsum + (size_t)t * ng + g, lds[t]);
  if (last_block_of_problem(&tk.st->ctr_dots, ng, &lastf)) gram_solve_block(tk, j, lds, gsum, ng, ng, scratch);
}

// h_{j+1,j} = ||w|| (nrm2 = ||w||^2, summed by the caller), Givens update of
// column j and the convergence test on |g_{j+1}| (thread 0 of one block of
// the problem).  V[j+1] is normalised by the next step's tridiagonal solve
// (ProbState::vscale).  When the problem's cycle ends, its host-visible flag
// receives `tag`.
// Column j of H and the stored rotations into LDS (every block of the pass
// does this at its start, so the finishing block does not wait for them).
__device__ __forceinline__ void mgs_finish_preload(const KryTask& tk, int j, double* col, double* cs,
                                                   double* sn) {
  const int m1 = tk.m + 1;
  for (int i = threadIdx.x; i <= j; i += blockDim.x) col[i] = tk.H[i + j * m1];
  for (int i = threadIdx.x; i < j; i += blockDim.x) {
    cs[i] = tk.cs[i];
    sn[i] = tk.sn[i];
  }
}

// (col, cs, sn filled by mgs_finish_preload and published by a barrier)
__device__ void mgs_finish_block(const KryTask& tk, int j, int* flags, int tag, double nrm2,
                                 double* col, double* cs, double* sn) {
  ProbState* st = tk.st;
  const int m1 = tk.m + 1;
  if (threadIdx.x != 0) return;
  const double hn = sqrt(nrm2);
  const bool breakdown = !(hn > 1e-14 * st->beta);
  col[j + 1] = hn;
  st->last_hn = hn;
  st->vscale = breakdown ? 1.0 : 1.0 / hn;
  for (int i = 0; i < j; ++i) {
    const double a = col[i], c2 = col[i + 1];
    col[i] = cs[i] * a + sn[i] * c2;
    col[i + 1] = -sn[i] * a + cs[i] * c2;
  }
  const double a = col[j];
  const double rho = hypot(a, hn);
  double c = 1.0, s = 0.0;
  if (rho > 0.0) {
    c = a / rho;
    s = hn / rho;
  }
  tk.cs[j] = c;
  tk.sn[j] = s;
  col[j] = rho;
  col[j + 1] = 0.0;
  for (int i = 0; i <= j + 1; ++i) tk.H[i + j * m1] = col[i];
  const double gj = tk.g[j];
  tk.g[j + 1] = -s * gj;
  tk.g[j] = c * gj;
  st->j_done = j + 1;
  st->iterations += 1;
  const double est = fabs(tk.g[j + 1]);
  if (!(est > st->tol_eff * st->fnorm) || breakdown || j + 1 == tk.m) {
    st->cycle_done = 1;
    if (flags) {
      flags[tk.flag_idx] = tag;
      __threadfence_system();
    }
  }
}

// w_new = w - sum_i h_i v_i  -> V[j+1], with block partials of ||w_new||^2;
// the problem's last block then finishes the step (mgs_finish_block).
__global__ void __launch_bounds__(kBlock) k_gram_update(const KryTask* __restrict__ tasks, int ntasks,
                                                         int j, int* flags, int tag) {
  __shared__ int slot;
  __shared__ int lastf;
  __shared__ double red[4];
  __shared__ double hs[121];
  __shared__ double col[122];
  __shared__ double cs[121], sn[121];
  __shared__ double scratch[kBlock];
  const KryTask& tk = tasks[find_task(tasks, ntasks, &slot)];
  if (tk.st->cycle_done) return;
  for (int i = threadIdx.x; i <= j; i += kBlock) hs[i] = tk.hv[i];
  mgs_finish_preload(tk, j, col, cs, sn);
  __syncthreads();
  const int b = blockIdx.x - tk.block_begin;
  const long long Nc = tk.Nc;
  const long long base = (long long)b * kVecPerBlock;
  double* w = tk.V + (long long)(j + 1) * Nc;
  const double* vj = tk.V + (long long)j * Nc;
  double acc[kVecEPT], xj[kVecEPT];
#pragma unroll
  for (int e = 0; e < kVecEPT; ++e) {
    const long long idx = base + (long long)e * kBlock + threadIdx.x;
    const bool ok = idx < Nc;
    xj[e] = ok ? vj[idx] : 0.0;
    acc[e] = !ok ? 0.0 : (tk.implicit_w ? xj[e] - line_term(tk, idx) : w[idx]);
  }
  // Loads are predicated by value (not by branch) so that all of them are in
  // flight together; two basis vectors per trip.
  int i = 0;
  for (; i + 1 < j; i += 2) {
    const double* va = tk.V + (long long)i * Nc;
    const double* vb = va + Nc;
    const double ha = hs[i], hb = hs[i + 1];
    double a[kVecEPT], c[kVecEPT];
#pragma unroll
    for (int e = 0; e < kVecEPT; ++e) {
      const long long idx = base + (long long)e * kBlock + threadIdx.x;
      const bool ok = idx < Nc;
      a[e] = ok ? va[idx] : 0.0;
      c[e] = ok ? vb[idx] : 0.0;
    }
#pragma unroll
    for (int e = 0; e < kVecEPT; ++e) {
      acc[e] -= ha * a[e];
      acc[e] -= hb * c[e];
    }
  }
  if (i < j) {
    const double* va = tk.V + (long long)i * Nc;
    const double ha = hs[i];
#pragma unroll
    for (int e = 0; e < kVecEPT; ++e) {
      const long long idx = base + (long long)e * kBlock + threadIdx.x;
      acc[e] -= ha * ((idx < Nc) ? va[idx] : 0.0);
    }
  }
#pragma unroll
  for (int e = 0; e < kVecEPT; ++e) acc[e] -= hs[j] * xj[e];
  double nrm = 0.0;
#pragma unroll
  for (int e = 0; e < kVecEPT; ++e) {
    const long long idx = base + (long long)e * kBlock + threadIdx.x;
    if (idx < Nc) {
      w[idx] = acc[e];
      nrm += acc[e] * acc[e];
    }
  }
  const double s = block_sum(nrm, red);
  if (threadIdx.x == 0) st_agent(tk.partials + (size_t)kPartNorm * tk.P + b, s);
  if (last_block_of_problem(&tk.st->ctr_upd, tk.P, &lastf)) {
    reduce_rows(tk.partials + (size_t)kPartNorm * tk.P, tk.P, 1, tk.P, scratch, red);
    mgs_finish_block(tk, j, flags, tag, red[0], col, cs, sn);
  }
}

// ---- lagged Gram columns (exact preconditioner) ----------------------
// Boundary dots of step j: block i (< kLagMaxJ) of a problem forms
// <v_i, s> with one wavefront per boundary line (s is zero elsewhere; a
// corner takes both of its lines' terms, as in line_term).  The problem's
// last block then runs the MGS recurrence with a_i = G_ij - <v_i, s>, the
// Gram column G[:, j] having been stored by the previous update pass (or set
// to e_0 at the start of the cycle).
__global__ void __launch_bounds__(kBlock) k_gram_bdots(const KryTask* __restrict__ tasks, int ntasks,
                                                        int j) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  __shared__ int lastf;
  __shared__ double wred[4];
  const int t = blockIdx.x / kLagMaxJ;
  const int i = blockIdx.x - t * kLagMaxJ;
  if (t >= ntasks) return;
  const KryTask& tk = tasks[t];
  if (tk.st->cycle_done) return;
  const int nd = j + 1;
  const int q = threadIdx.x >> 6, lane = threadIdx.x & 63;
  double acc = 0.0;
  if (tk.post) {
    // sine basis of the centre: rows 0 / ny-1 pair v^_i with the diagonal
    // S/N terms (N/2) gs_k z^; columns pair the physical boundary values of
    // v_i (bc) with the W/E line terms
    if (i <= j) {
      const double* vi = tk.V + (long long)i * tk.Nc;
      if (q < 2 && tk.gs[q]) {
        const long long row = q == 0 ? 0 : (long long)(tk.ny - 1) * tk.nx;
        #pragma unroll 4
        for (int p = lane; p < tk.nx; p += 64)
          acc += vi[row + p] * (tk.half_n * tk.gs[q][p] * tk.zhat[row + p]);
      } else if (q >= 2 && tk.line[q]) {
        const double* b = tk.bc + (long long)2 * tk.ny * i + (q == 3 ? tk.ny : 0);
        #pragma unroll 4
        for (int p = lane; p < tk.ny; p += 64) acc += b[p] * tk.line[q][p];
      }
    }
  } else if (i <= j && tk.line[q]) {
    const double* s = tk.line[q];
    const double* vi = tk.V + (long long)i * tk.Nc;
    const int len = q < 2 ? tk.nx : tk.ny;
    for (int p = lane; p < len; p += 64) {
      const long long idx = q == 0 ? (long long)p
                          : q == 1 ? (long long)(tk.ny - 1) * tk.nx + p
                          : q == 2 ? (long long)p * tk.nx
                                   : (long long)p * tk.nx + (tk.nx - 1);
      acc += vi[idx] * s[p];
    }
  }
  acc = wave_sum(acc);
  if (lane == 0) wred[q] = acc;
  __syncthreads();
  double* u = tk.partials + (size_t)(kPartDots + nd) * tk.P;   // u_i at row kPartDots + nd + i
  if (threadIdx.x == 0 && i <= j) st_agent(u + (size_t)i * tk.P, (wred[0] + wred[1]) + (wred[2] + wred[3]));
  if (!last_block_of_problem(&tk.st->ctr_dots, kLagMaxJ, &lastf)) return;
  double* lds = reinterpret_cast<double*>(smem_raw);
  const int m1 = tk.m + 1;
  for (int e = threadIdx.x; e < nd; e += kBlock) {
    lds[e] = tk.G[e + j * m1];
    lds[nd + e] = ld_agent(u + (size_t)e * tk.P);
  }
  __syncthreads();
  gram_recur(tk, j, lds);
}

// Update of step j with the next Gram column: w = v_j - s - sum h_i v_i is
// stored in V[j+1] (unnormalised, as in k_gram_update), and the same pass
// accumulates <v_i, w> (i <= j) and ||w||^2 from the values it holds in
// registers.  The last block finishes the step (mgs_finish_block) and stores
// G[i, j+1] = <v_i, w> / h_{j+1,j}, G[j+1, j+1] = ||w||^2 / h_{j+1,j}^2.
// MJ >= j + 1 basis vectors; each round a thread loads EU elements of each
// of them (vector min(i, j) for i > j, so every load is in bounds and none
// is behind a branch; those values are then cleared).  The dots use the
// two-level reduction of k_gram_dots.
template <int MJ, int EU>
__global__ void __launch_bounds__(kBlock) k_gram_update_lag(const KryTask* __restrict__ tasks, int ntasks,
                                                             int j, int* flags, int tag) {
  static_assert(kVecEPT % EU == 0, "rounds must cover the block");
  __shared__ int slot;
  __shared__ int lastf;
  __shared__ double hs[MJ];
  __shared__ double col[122];
  __shared__ double cs[121], sn[121];
  __shared__ double scratch[kBlock];
  __shared__ double dred[MJ + 1][4];
  __shared__ double gcol[MJ + 1];
  const KryTask& tk = tasks[find_task(tasks, ntasks, &slot)];
  if (tk.st->cycle_done) return;
  // hs: coefficients of v_0..v_{j-1} (zero from j on); v_j's is taken apart
  // so that it is subtracted last, as in k_gram_update
  for (int i = threadIdx.x; i < MJ; i += kBlock) hs[i] = i < j ? tk.hv[i] : 0.0;
  mgs_finish_preload(tk, j, col, cs, sn);
  const double hj = tk.hv[j];   // (hs, col, cs, sn are published after round 0's loads are issued)
  const int b = blockIdx.x - tk.block_begin;
  const long long Nc = tk.Nc;
  const long long base = (long long)b * kVecPerBlock;
  double* w = tk.V + (long long)(j + 1) * Nc;
  // the basis through global-address-space pointers: one uniform base per
  // vector and one 32-bit lane offset shared by all of its loads
  using GD = const double __attribute__((address_space(1)));
  using GB = const unsigned char __attribute__((address_space(1)));
  GD* Vg = (GD*)(tk.V);
  double d[MJ + 1];
#pragma unroll
  for (int i = 0; i <= MJ; ++i) d[i] = 0.0;
#pragma unroll 1
  for (int r = 0; r < kVecEPT / EU; ++r) {
    unsigned off[EU], boff[EU];
    bool ok[EU];
#pragma unroll
    for (int u = 0; u < EU; ++u) {
      const long long idx = base + (long long)(r * EU + u) * kBlock + threadIdx.x;
      ok[u] = idx < Nc;
      off[u] = (unsigned)(ok[u] ? idx : Nc - 1);
      boff[u] = off[u] * 8u;   // byte offset (a centre vector is below 4 GiB)
    }
    // vectors beyond j load v_j again (in bounds, cached); their
    // coefficients are zero and their dot sums are never reduced, so no
    // selects are needed
    double vv[EU][MJ], xj[EU];
    GD* vj = Vg + (long long)j * Nc;
#pragma unroll
    for (int u = 0; u < EU; ++u) xj[u] = vj[off[u]];
#pragma unroll
    for (int i = 0; i < MJ; ++i) {
      GB* vi = (GB*)(Vg + (long long)min(i, j) * Nc);
#pragma unroll
      for (int u = 0; u < EU; ++u) vv[u][i] = *(GD*)(vi + boff[u]);
    }
    if (r == 0) __syncthreads();
#pragma unroll
    for (int u = 0; u < EU; ++u) {
      const long long idx = base + (long long)(r * EU + u) * kBlock + threadIdx.x;
      double acc = xj[u] - (ok[u] ? line_term(tk, idx) : 0.0);
#pragma unroll
      for (int i = 0; i < MJ; ++i) acc -= hs[i] * vv[u][i];   // hs[i] = 0 for i >= j
      acc -= hj * xj[u];
      acc = ok[u] ? acc : 0.0;
      if (ok[u]) w[idx] = acc;
      d[MJ] += acc * acc;
#pragma unroll
      for (int i = 0; i < MJ; ++i) d[i] += vv[u][i] * acc;
    }
  }
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int nd = j + 1;
#pragma unroll
  for (int i = 0; i <= MJ; ++i) {
    if (i <= j || i == MJ) {
      const double v = wave_sum_last(d[i]);
      if (lane == 63) dred[i][wave] = v;
    }
  }
  __syncthreads();
  // rows 0..j: <v_i, w>; row nd: ||w||^2 (all reduced together)
  const int P = tk.P;
  double* part = tk.partials + (size_t)kPartDots * P;
  for (int t = threadIdx.x; t <= nd; t += kBlock) {
    const int r = t < nd ? t : MJ;
    st_agent(part + (size_t)t * P + b, (dred[r][0] + dred[r][1]) + (dred[r][2] + dred[r][3]));
  }
  const int ng = gram_groups(P);
  if (ng == 1) {
    if (!last_block_of_problem(&tk.st->ctr_upd, P, &lastf)) return;
    reduce_rows(part, P, nd + 1, P, scratch, gcol);
  } else {
    double* gsum = tk.partials + (size_t)(2 * (tk.m + 1) + 4) * P;
    int* gctr = reinterpret_cast<int*>(gsum + (size_t)2 * (tk.m + 1) * ng);
    const int g = b / kGramGroup;
    const int gb = min(kGramGroup, P - g * kGramGroup);
    if (!last_block_of_problem(gctr + g, gb, &lastf)) return;
    reduce_rows(part + g * kGramGroup, P, nd + 1, gb, scratch, gcol);
    for (int t = threadIdx.x; t <= nd; t += kBlock) st_agent(gsum + (size_t)t * ng + g, gcol[t]);
    if (!last_block_of_problem(&tk.st->ctr_upd, ng, &lastf)) return;
    reduce_rows(gsum, ng, nd + 1, ng, scratch, gcol);
  }
  const double nrm2 = gcol[nd];
  mgs_finish_block(tk, j, flags, tag, nrm2, col, cs, sn);
  if (threadIdx.x == 0) {
    // ProbState::vscale = 1 / h_{j+1,j}
    const double vs = tk.st->vscale;
    const int m1 = tk.m + 1;
    for (int t = 0; t < nd; ++t) tk.G[t + (j + 1) * m1] = gcol[t] * vs;
    tk.G[(j + 1) + (j + 1) * m1] = nrm2 * vs * vs;
  }
}

// v *= 1 / h_{j+1,j} for the kernel-level Arnoldi entry point.
__global__ void k_scale_newest(const KryTask* __restrict__ tasks, int j) {
  const KryTask& tk = tasks[0];
  const double s = tk.st->vscale;
  double* w = tk.V + (long long)(j + 1) * tk.Nc;
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < tk.Nc;
       i += (long long)gridDim.x * blockDim.x)
    w[i] *= s;
}

// Back substitution R y = g over the j_done columns.
__global__ void __launch_bounds__(kBlock) k_ls_solve(const KryTask* __restrict__ tasks, int ntasks) {
  // one workgroup per problem: the triangle of H is staged in LDS with every
  // thread (column l at l k), then one wavefront back-substitutes; lane i
  // (and i + 64) holds the running right-hand side s_i, and y_i, once
  // final, is broadcast by a lane shuffle
  extern __shared__ __align__(16) unsigned char smem_raw[];
  double* Hs = reinterpret_cast<double*>(smem_raw);
  const KryTask& tk = tasks[blockIdx.x];
  if (tk.st->finished) return;
  const int k = tk.st->j_done;
  const int m1 = tk.m + 1;
  for (int e = threadIdx.x; e < k * k; e += kBlock) {
    const int l = e / k, i = e - l * k;
    Hs[e] = i <= l ? tk.H[i + l * m1] : 0.0;
  }
  __syncthreads();
  if (threadIdx.x >= 64) return;
  const int lane = threadIdx.x;
  const int i0 = lane, i1 = lane + 64;
  double s0 = i0 < k ? tk.g[i0] : 0.0;
  double s1 = i1 < k ? tk.g[i1] : 0.0;
  for (int i = k - 1; i >= 0; --i) {
    const double d = Hs[i + i * k];
    const double si = __shfl(i < 64 ? s0 : s1, i & 63, 64);
    const double yi = (d != 0.0) ? si / d : 0.0;
    if (lane == (i & 63)) tk.y[i] = yi;
    if (i0 < i) s0 -= Hs[i0 + i * k] * yi;
    if (i1 < i) s1 -= Hs[i1 + i * k] * yi;
  }
}

// u = V y (plain variant) or u = Z y (flexible variant, sine coefficients);
// the preconditioner / inverse transform then adds it to x.
template <int FLEX>
__global__ void __launch_bounds__(kBlock) k_combine(const KryTask* __restrict__ tasks, int ntasks) {
  __shared__ int slot;
  __shared__ double ys[128];
  const KryTask& tk = tasks[find_task(tasks, ntasks, &slot)];
  if (tk.st->finished) return;
  const int k = tk.st->j_done;
  for (int i = threadIdx.x; i < k; i += kBlock) ys[i] = tk.y[i];
  __syncthreads();
  const int b = blockIdx.x - tk.block_begin;
  const long long Nc = tk.Nc;
  const long long base = (long long)b * kVecPerBlock;
#pragma unroll
  for (int e = 0; e < kVecEPT; ++e) {
    const long long idx = base + (long long)e * kBlock + threadIdx.x;
    if (idx < Nc) {
      double acc = 0.0;
      if (FLEX) {
        for (int i = 0; i < k; ++i) acc += ys[i] * double(tk.Z[(long long)i * Nc + idx]);
        tk.u[idx] = acc;
      } else {
        for (int i = 0; i < k; ++i) acc += ys[i] * tk.V[(long long)i * Nc + idx];
        tk.u[idx] = acc;
      }
    }
  }
}

// After the residual operator (mode 1 writes r into V[0] and the partials).
// Restart decision, one block per problem: beta = ||r||, the stopping tests
// (tolerance with the rounding floor, cycle cap, stagnation) and the state
// for the next cycle.  The decision is taken here, before any block scales
// V[0], because the tests read state that this kernel updates.
__global__ void __launch_bounds__(kBlock) k_restart(const KryTask* __restrict__ tasks, int ntasks,
                                                     int initial, int max_cycles) {
  __shared__ double red[4];
  const KryTask& tk = tasks[blockIdx.x];
  ProbState* st = tk.st;
  if (st->finished) return;
  if (initial) {   // the Gram reduction's group counters start at zero
    const int ng = gram_groups(tk.P);
    if (ng > 1) {
      int* gctr = reinterpret_cast<int*>(tk.partials + kry_partials_len(tk.m, tk.P) - ng);
      for (int g = threadIdx.x; g < ng; g += kBlock) gctr[g] = 0;
    }
  }
  const double r2 = sum_partials(tk.partials + (size_t)kPartRes * tk.P, tk.P, red);
  const double x2 = sum_partials(tk.partials + (size_t)(kPartRes + 1) * tk.P, tk.P, red);
  if (threadIdx.x != 0) return;
  const double beta = sqrt(r2);
  const double fnorm = initial ? beta : st->fnorm;
  bool done = false;
  int reason = FDS_STOP_NONE;
  const double rel = fnorm > 0.0 ? beta / fnorm : 0.0;
  double tol_eff = st->tol;
  if (fnorm > 0.0) tol_eff = fmax(st->tol, 2.0 * st->floor_coef * sqrt(x2) / fnorm);
  const bool finite = isfinite(beta) && isfinite(x2);
  if (!finite) {
    done = true;
    reason = FDS_STOP_NONE;
  } else if (fnorm == 0.0 || rel <= tol_eff) {
    done = true;
    reason = (fnorm == 0.0 || rel <= st->tol) ? FDS_STOP_TOL : FDS_STOP_AT_FLOOR;
  } else if (!initial && st->cycles + 1 >= max_cycles) {
    done = true;
    reason = FDS_STOP_MAX_CYCLES;
  } else if (!initial && st->cycles >= 2 && rel > 0.9 * st->prev_rel) {
    // no 10% gain over a cycle: within twice the effective tolerance this is
    // the rounding floor (the floor estimate is only an estimate), otherwise
    // the iteration has stalled
    done = true;
    reason = rel <= 2.0 * tol_eff ? FDS_STOP_AT_FLOOR : FDS_STOP_STAGNATION;
  }
  if (initial) st->fnorm = fnorm;
  else st->cycles += 1;
  st->beta = beta;
  st->xnorm = sqrt(x2);
  st->tol_eff = tol_eff;
  st->prev_rel = rel;
  if (!finite) st->nonfinite = 1;
  if (done) {
    st->finished = 1;
    st->cycle_done = 1;
    st->stop_reason = reason;
    st->rscale = 0.0;
  } else {
    st->cycle_done = 0;
    st->j_done = 0;
    st->vscale = 1.0;
    st->rscale = 1.0 / beta;
    tk.g[0] = beta;
    tk.G[0] = 1.0;   // <v_0, v_0> (the lagged Gram columns start here)
  }
}

// V[0] = r / beta for the problems that continue (after k_restart).
__global__ void __launch_bounds__(kBlock) k_restart_scale(const KryTask* __restrict__ tasks,
                                                           int ntasks) {
  __shared__ int slot;
  const KryTask& tk = tasks[find_task(tasks, ntasks, &slot)];
  const ProbState* st = tk.st;
  if (st->finished) return;
  const double inv = st->rscale;
  const long long base = (long long)(blockIdx.x - tk.block_begin) * kVecPerBlock;
#pragma unroll
  for (int e = 0; e < kVecEPT; ++e) {
    const long long idx = base + (long long)e * kBlock + threadIdx.x;
    if (idx < tk.Nc) tk.V[idx] *= inv;
  }
}

// =====================================================================
// Layout conversion with Dirichlet lift (mode 0) and gather-out (mode 1).
// =====================================================================
template <int MODE>
__global__ void __launch_bounds__(kBlock) k_lift(const LiftTask* __restrict__ tasks, int ntasks) {
  __shared__ int slot;
  const LiftTask& tk = tasks[find_task(tasks, ntasks, &slot)];
  const RectDev& rd = tk.rd;
  const long long total = (long long)rd.rows * rd.cols;
  const long long e0 = (long long)(blockIdx.x - tk.block_begin) * kBlock + threadIdx.x;
  const long long stride = (long long)tk.nblocks * kBlock;
  for (long long e = e0; e < total; e += stride) {
    const int r = (int)(e / rd.cols);
    const int c = (int)(e - (long long)r * rd.cols);
    const int i = rd.ai + rd.ar * r + rd.ac * c;
    const int j = rd.aj + rd.br * r + rd.bcc * c;
    const long long uidx = rd.user_off + (long long)(j - rd.jlo) * rd.uwidth + (i - rd.ilo);
    const long long iidx = rd.off + (long long)r * rd.ld + c;
    if (MODE == 1) {
      tk.xuser[uidx] = tk.xint[iidx];
      continue;
    }
    double v = tk.rhs[uidx];
    if (tk.bc) {
      const int ni[4] = {i + 1, i - 1, i, i};
      const int nj[4] = {j, j, j + 1, j - 1};
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int a = ni[q], bq = nj[q];
        if (a < rd.bi0 || a > rd.bi1 || bq < rd.bj0 || bq > rd.bj1) continue;  // other subdomain
        const bool on_i0 = a == rd.bi0, on_i1 = a == rd.bi1;
        const bool on_j0 = bq == rd.bj0, on_j1 = bq == rd.bj1;
        if (!(on_i0 || on_i1 || on_j0 || on_j1)) continue;  // interior unknown
        bool unknown = false;
        const bool inner_j = bq > rd.bj0 && bq < rd.bj1;
        const bool inner_i = a > rd.bi0 && a < rd.bi1;
        if (on_i0 && inner_j && (rd.iface_mask & 1)) unknown = true;
        if (on_i1 && inner_j && (rd.iface_mask & 2)) unknown = true;
        if (on_j0 && inner_i && (rd.iface_mask & 4)) unknown = true;
        if (on_j1 && inner_i && (rd.iface_mask & 8)) unknown = true;
        if (unknown) continue;
        const int bw = rd.bi1 - rd.bi0 + 1;
        v -= tk.delta * tk.bc[rd.bc_off + (long long)(bq - rd.bj0) * bw + (a - rd.bi0)];
      }
    }
    tk.out[iidx] = v;
  }
}

// Interface right-hand-side updates (see IfaceTask); one block per problem.
__global__ void k_iface(const IfaceTask* __restrict__ tasks, int ntasks) {
  const IfaceTask& tk = tasks[blockIdx.x];
  for (int a = 0; a < tk.nlines; ++a) {
    double* dst = tk.dst[a] + tk.dst_start[a];
    const double* src = tk.src[a] + tk.src_start[a];
    const long long ds = tk.dst_stride[a], ss = tk.src_stride[a];
    for (int t = threadIdx.x; t < tk.L[a]; t += blockDim.x) dst[t * ds] -= tk.delta * src[t * ss];
    __syncthreads();
  }
}

// Composite residual over the internal layout (partials of r^2 and b^2).
__global__ void __launch_bounds__(kBlock) k_residual(const ResTask* __restrict__ tasks, int ntasks) {
  __shared__ int slot;
  __shared__ double red[4];
  const ResTask& tk = tasks[find_task(tasks, ntasks, &slot)];
  const RectDev& rd = tk.rd;
  const long long total = (long long)rd.rows * rd.cols;
  const int b = blockIdx.x - tk.block_begin;
  const long long stride = (long long)tk.nblocks * kBlock;
  const double* p = tk.p + rd.off;
  double rr = 0.0, bb = 0.0;
  for (long long e = (long long)b * kBlock + threadIdx.x; e < total; e += stride) {
    const int r = (int)(e / rd.cols);
    const int c = (int)(e - (long long)r * rd.cols);
    const long long q = (long long)r * rd.ld + c;
    double nb = 0.0;
    if (r > 0) nb += p[q - rd.ld];
    else if (rd.halo_off[0] >= 0) nb += tk.p[rd.halo_off[0] + c * rd.halo_stride[0]];
    if (r < rd.rows - 1) nb += p[q + rd.ld];
    else if (rd.halo_off[1] >= 0) nb += tk.p[rd.halo_off[1] + c * rd.halo_stride[1]];
    if (c > 0) nb += p[q - 1];
    else if (rd.halo_off[2] >= 0) nb += tk.p[rd.halo_off[2] + r * rd.halo_stride[2]];
    if (c < rd.cols - 1) nb += p[q + 1];
    else if (rd.halo_off[3] >= 0) nb += tk.p[rd.halo_off[3] + r * rd.halo_stride[3]];
    const double Ap = tk.delta * nb + (tk.kappa - 4.0 * tk.delta) * p[q];
    const double bv = tk.b[rd.off + q];
    const double res = bv - Ap;
    rr += res * res;
    bb += bv * bv;
  }
  const double s1 = block_sum(rr, red);
  const double s2 = block_sum(bb, red);
  if (threadIdx.x == 0) {
    tk.partials[b] = s1;
    tk.partials[tk.pstride + b] = s2;
  }
}

// Composite residual sums of each problem, fixed order (one block per problem).
__global__ void __launch_bounds__(kBlock) k_res_sum(const ResSumTask* __restrict__ tasks) {
  __shared__ double red[4];
  const ResSumTask& tk = tasks[blockIdx.x];
  const double rr = sum_partials(tk.partials, tk.n, red);
  const double bb = sum_partials(tk.partials + tk.n, tk.n, red);
  if (threadIdx.x == 0) {
    tk.st->res_rr = rr;
    tk.st->res_bb = bb;
  }
}

// Copies, zero fills and diagonal scalings of whole vectors, batched over
// problems.
__global__ void __launch_bounds__(kBlock) k_copy(const CopyTask* __restrict__ tasks, int ntasks) {
  __shared__ int slot;
  const CopyTask& tk = tasks[find_task(tasks, ntasks, &slot)];
  if (tk.skip && *tk.skip) return;
  const long long stride = (long long)tk.nblocks * kBlock;
  const double* mul = tk.mul;
  for (long long e = (long long)(blockIdx.x - tk.block_begin) * kBlock + threadIdx.x; e < tk.count;
       e += stride)
    tk.dst[e] = tk.src ? (mul ? tk.src[e] * mul[e] : tk.src[e]) : 0.0;
}

// Number of problems whose current cycle is still running.
__global__ void k_count_active(const ProbState* __restrict__ st, int n, int* __restrict__ out) {
  __shared__ double red[4];
  double c = 0.0;
  for (int i = threadIdx.x; i < n; i += kBlock) c += st[i].cycle_done ? 0.0 : 1.0;
  const double s = block_sum(c, red);
  if (threadIdx.x == 0) *out = (int)s;
}


// =====================================================================
// Launchers
// =====================================================================
void launch_dst(DstKind kind, const DstTask* tasks, int ntasks, int nblocks, size_t smem, int jidx,
                hipStream_t s) {
  if (nblocks <= 0) return;
  static size_t g_dd = 0, g_df = 0, g_ff = 0, g_fd = 0;
  switch (kind) {
    case DstKind::D_D: ensure_smem(k_dst_rows<double, double, double>, smem, &g_dd); break;
    case DstKind::D_F: ensure_smem(k_dst_rows<float, double, float>, smem, &g_df); break;
    case DstKind::F_F: ensure_smem(k_dst_rows<float, float, float>, smem, &g_ff); break;
    case DstKind::F_D: ensure_smem(k_dst_rows<float, float, double>, smem, &g_fd); break;
  }
  switch (kind) {
    case DstKind::D_D:
      FDS_LAUNCH((k_dst_rows<double, double, double>), dim3(nblocks), dim3(kBlock), smem, s,
                         tasks, ntasks, jidx);
      break;
    case DstKind::D_F:
      FDS_LAUNCH((k_dst_rows<float, double, float>), dim3(nblocks), dim3(kBlock), smem, s,
                         tasks, ntasks, jidx);
      break;
    case DstKind::F_F:
      FDS_LAUNCH((k_dst_rows<float, float, float>), dim3(nblocks), dim3(kBlock), smem, s,
                         tasks, ntasks, jidx);
      break;
    case DstKind::F_D:
      FDS_LAUNCH((k_dst_rows<float, float, double>), dim3(nblocks), dim3(kBlock), smem, s,
                         tasks, ntasks, jidx);
      break;
  }
}

size_t gemm_smem_bytes(int n, bool fp32, int rt) {
  const int np = (n + 63) / 64 * 64;
  return (size_t)rt * 16 * (np + 1) * (fp32 ? sizeof(float) : sizeof(double));
}

void launch_dst_gemm(DstKind kind, int rt, int ct, const DstTask* tasks, int ntasks, int nblocks,
                     size_t smem, int jidx, hipStream_t s) {
  if (nblocks <= 0) return;
#define FDS_G(T, TI, TO, R, C)                                                                    \
  do {                                                                                           \
    static size_t granted = 0;                                                                   \
    ensure_smem(k_dst_gemm<T, TI, TO, R, C>, smem, &granted);                                    \
    FDS_LAUNCH((k_dst_gemm<T, TI, TO, R, C>), dim3(nblocks), dim3(kBlock), smem, s, tasks, \
                       ntasks, jidx);                                                            \
  } while (0)
#define FDS_G_CT(T, TI, TO, R)                      \
  switch (ct) {                                     \
    case 1: FDS_G(T, TI, TO, R, 1); break;          \
    case 2: FDS_G(T, TI, TO, R, 2); break;          \
    case 3: FDS_G(T, TI, TO, R, 3); break;          \
    default: FDS_G(T, TI, TO, R, 4); break;         \
  }
#define FDS_G_RT(T, TI, TO)                         \
  if (rt == 1) { FDS_G_CT(T, TI, TO, 1) } else { FDS_G_CT(T, TI, TO, 2) }
  switch (kind) {
    case DstKind::D_D: FDS_G_RT(double, double, double); break;
    case DstKind::D_F: FDS_G_RT(float, double, float); break;
    case DstKind::F_F: FDS_G_RT(float, float, float); break;
    case DstKind::F_D: FDS_G_RT(float, float, double); break;
  }
#undef FDS_G_RT
#undef FDS_G_CT
#undef FDS_G
}

void launch_tridiag(bool fp32, const TriTask* tasks, int ntasks, int nblocks, int jidx,
                    hipStream_t s) {
  if (nblocks <= 0) return;
  if (fp32)
    FDS_LAUNCH(k_tridiag<float>, dim3(nblocks), dim3(kBlock), 0, s, tasks, ntasks, jidx);
  else
    FDS_LAUNCH(k_tridiag<double>, dim3(nblocks), dim3(kBlock), 0, s, tasks, ntasks, jidx);
}

// A segmented configuration for systems of `rows` rows, if (mpb, ls) fits.
static bool tri_fit(int mpb, int ls, int rows, TriConfig* c) {
  const int S = (rows + ls - 1) / ls;
  if (S > (ls >= 32 ? kTriMaxThreadsLong : 1024) / mpb) return false;
  c->seg = true;
  c->ls = ls;
  c->mpb = mpb;
  c->threads = std::max(64, mpb * (S < 1 ? 1 : S));
  return true;
}

std::vector<TriConfig> tri_configs(int rows) {
  std::vector<TriConfig> out;
  for (int mpb : {8, 16, 32, 64})
    for (int ls : {4, 8, 16, 32}) {
      TriConfig c{false, 0, 0, 0};
      if (tri_fit(mpb, ls, rows, &c)) out.push_back(c);
    }
  if (out.empty()) out.push_back(TriConfig{false, 0, 0, 0});
  return out;
}

TriConfig tri_config_static(bool fp32, int max_rows) {
  (void)fp32;
  // register segments of 8 to 32 rows (the shortest that fits); up to 1024
  // threads per block: 16 modes x 64 segments, 32 x 32, 64 x 16, or 8 x 128
  // for the longest systems.  Fewest modes per block first: a problem's
  // modes then spread over more blocks (16 modes x 8 bytes still read whole
  // 128-byte lines per row).
  TriConfig c{false, 0, 0, 0};
  const int lsmax = 32;
  // tuning override "mpb,ls": taken when the pair is instantiated and fits
  if (const char* e = std::getenv("FDS_TRI_SEG")) {
    int mpb = 0, ls = 0;
    if (std::sscanf(e, "%d,%d", &mpb, &ls) == 2 && (mpb == 8 || mpb == 16 || mpb == 32 || mpb == 64) &&
        (ls == 4 || ls == 8 || ls == 16 || ls == 32) && tri_fit(mpb, ls, max_rows, &c))
      return c;
  }
  // (8 modes per block last: up to 128 segments, for systems of more than
  // 1024 (FP64 with 16-row segments) or 2048 rows)
  for (int mpb : {16, 32, 64, 8})
    for (int ls = 8; ls <= lsmax; ls *= 2)
      if (tri_fit(mpb, ls, max_rows, &c)) return c;
  return c;
}

int tri_blocks(const TriConfig& c, int modes) {
  return c.seg ? (modes + c.mpb - 1) / c.mpb : (modes + kBlock - 1) / kBlock;
}

void launch_tri(const TriConfig& c, bool fp32, const TriTask* tasks, int ntasks, int nblocks,
                int jidx, hipStream_t s) {
  if (nblocks <= 0) return;
  if (!c.seg) {
    launch_tridiag(fp32, tasks, ntasks, nblocks, jidx, s);
    return;
  }
  if (c.threads > (c.ls >= 32 ? kTriMaxThreadsLong : 1024))
    throw Error(FDS_E_INVALID_ARG, "tridiagonal launch wider than its kernel's bound");
  const dim3 blk(c.threads);
#define FDS_SEG(T, L, M) \
  FDS_LAUNCH((k_tridiag_seg<T, L, M>), dim3(nblocks), blk, 0, s, tasks, ntasks, jidx)
#define FDS_SEG_MPB(T, L)                      \
  switch (c.mpb) {                             \
    case 64: FDS_SEG(T, L, 64); break;         \
    case 32: FDS_SEG(T, L, 32); break;         \
    case 8: FDS_SEG(T, L, 8); break;           \
    default: FDS_SEG(T, L, 16); break;         \
  }
  if (fp32) {
    switch (c.ls) {
      case 4: FDS_SEG_MPB(float, 4); break;
      case 8: FDS_SEG_MPB(float, 8); break;
      case 16: FDS_SEG_MPB(float, 16); break;
      default: FDS_SEG_MPB(float, 32); break;
    }
  } else {
    switch (c.ls) {
      case 4: FDS_SEG_MPB(double, 4); break;
      case 8: FDS_SEG_MPB(double, 8); break;
      case 16: FDS_SEG_MPB(double, 16); break;
      default: FDS_SEG_MPB(double, 32); break;
    }
  }
#undef FDS_SEG_MPB
#undef FDS_SEG
}

void launch_lines_dense(const LineTask* tasks, int ntasks, int nblocks, int lmax, int jidx,
                        hipStream_t s) {
  if (ntasks <= 0) return;
  const size_t smem = sizeof(double) * (size_t)lmax;
  static size_t granted = 0;
  ensure_smem(k_lines_dense, smem, &granted);
  FDS_LAUNCH(k_lines_dense, dim3(nblocks), dim3(kBlock), smem, s, tasks, ntasks, jidx);
}

void launch_lines(const LineTask* tasks, int ntasks, size_t smem, int jidx, hipStream_t s) {
  if (ntasks <= 0) return;
  static size_t granted = 0;
  ensure_smem(k_schur_lines, smem, &granted);
  FDS_LAUNCH(k_schur_lines, dim3(ntasks), dim3(kBlock), smem, s, tasks, jidx);
}

void launch_operator(int mode, const OpTask* tasks, int ntasks, int nblocks, int jidx,
                     hipStream_t s) {
  if (nblocks <= 0) return;
  if (mode == 0)
    FDS_LAUNCH(k_operator<0>, dim3(nblocks), dim3(kBlock), 0, s, tasks, ntasks, jidx);
  else
    FDS_LAUNCH(k_operator<1>, dim3(nblocks), dim3(kBlock), 0, s, tasks, ntasks, jidx);
}

// LDS of the Gram step of column j: dots (2 (j+1)), coefficients (j+1) and
// the strict upper triangle of the old Gram columns (j (j+1) / 2).
static size_t gram_solve_smem(int j) {
  return sizeof(double) * (3 * (size_t)(j + 1) + (size_t)j * (j + 1) / 2);
}

// Static LDS of k_gram_dots (its per-wavefront dot table).
constexpr size_t kGramDotsStatic = sizeof(double) * 2 * 121 * 4;

// The dynamic part reaches 60000 bytes at j = 119; with the static table the
// kernel then needs more than the 64 KiB granted by default.
void launch_gram_dots(const KryTask* tasks, int ntasks, int nblocks, int j, hipStream_t s) {
  if (nblocks <= 0) return;
  const size_t smem = gram_solve_smem(j);
  static size_t granted = 0;
  ensure_smem(k_gram_dots, smem + kGramDotsStatic, &granted);
  FDS_LAUNCH(k_gram_dots, dim3(nblocks), dim3(kBlock), smem, s, tasks, ntasks, j);
}

void launch_gram_bdots(const KryTask* tasks, int ntasks, int j, hipStream_t s) {
  if (ntasks <= 0) return;
  FDS_LAUNCH(k_gram_bdots, dim3(ntasks * kLagMaxJ), dim3(kBlock), gram_solve_smem(j), s, tasks, ntasks, j);
}

void launch_gram_update_lag(const KryTask* tasks, int ntasks, int nblocks, int m, int j, int* flags,
                            int tag, hipStream_t s) {
  if (nblocks <= 0) return;
  if (m > kLagMaxJ || j >= m) throw Error(FDS_E_INVALID_ARG, "lagged Gram columns need j < m <= 32");
  // basis vectors held per round: the smallest multiple of 4 >= j + 1 from
  // 12 on (fewer redundant loads of v_j than powers of two: +1.6% on the
  // plain workload); at most 32 loads per thread and round, which keeps
  // three wavefronts per SIMD resident
#define FDS_LAG(MJ, EU)                                                                         \
  FDS_LAUNCH((k_gram_update_lag<MJ, (EU < kVecEPT ? EU : kVecEPT)>), dim3(nblocks), dim3(kBlock), 0, s, \
             tasks, ntasks, j, flags, tag)
  if (j < 4) FDS_LAG(4, 4);
  else if (j < 8) FDS_LAG(8, 2);
  else if (j < 12) FDS_LAG(12, 1);
  else if (j < 16) FDS_LAG(16, 1);
  else if (j < 20) FDS_LAG(20, 1);
  else if (j < 24) FDS_LAG(24, 1);
  else if (j < 28) FDS_LAG(28, 1);
  else FDS_LAG(32, 1);
#undef FDS_LAG
}

void launch_gram_update(const KryTask* tasks, int ntasks, int nblocks, int j, int* flags, int tag,
                        hipStream_t s) {
  if (nblocks <= 0) return;
  FDS_LAUNCH(k_gram_update, dim3(nblocks), dim3(kBlock), 0, s, tasks, ntasks, j, flags, tag);
}

void launch_scale_newest(const KryTask* tasks, int j, int nblocks, hipStream_t s) {
  FDS_LAUNCH(k_scale_newest, dim3(nblocks), dim3(kBlock), 0, s, tasks, j);
}

void launch_idst_cols(const ColTask* tasks, int ntasks, int nblocks, int jidx, hipStream_t s) {
  if (nblocks <= 0) return;
  FDS_LAUNCH(k_idst_cols, dim3(nblocks), dim3(kBlock), 0, s, tasks, ntasks, jidx);
}

void launch_ls_solve(const KryTask* tasks, int ntasks, int m, hipStream_t s) {
  if (ntasks <= 0) return;
  if (m < 1 || m > 120) throw Error(FDS_E_INVALID_ARG, "restart length out of range");
  // LDS: the k x k triangle of H, k <= m <= 120 (opt-in above 64 KiB)
  const size_t smem = sizeof(double) * (size_t)m * m;
  static size_t granted = 0;
  ensure_smem(k_ls_solve, smem, &granted);
  FDS_LAUNCH(k_ls_solve, dim3(ntasks), dim3(kBlock), smem, s, tasks, ntasks);
}

void launch_combine(bool flex, const KryTask* tasks, int ntasks, int nblocks, hipStream_t s) {
  if (nblocks <= 0) return;
  if (flex)
    FDS_LAUNCH(k_combine<1>, dim3(nblocks), dim3(kBlock), 0, s, tasks, ntasks);
  else
    FDS_LAUNCH(k_combine<0>, dim3(nblocks), dim3(kBlock), 0, s, tasks, ntasks);
}

void launch_restart(const KryTask* tasks, int ntasks, int nblocks, int initial, int max_cycles,
                    hipStream_t s) {
  if (nblocks <= 0) return;
  FDS_LAUNCH(k_restart, dim3(ntasks), dim3(kBlock), 0, s, tasks, ntasks, initial, max_cycles);
  FDS_LAUNCH(k_restart_scale, dim3(nblocks), dim3(kBlock), 0, s, tasks, ntasks);
}

void launch_restart_decide(const KryTask* tasks, int ntasks, int initial, int max_cycles, hipStream_t s) {
  if (ntasks <= 0) return;
  FDS_LAUNCH(k_restart, dim3(ntasks), dim3(kBlock), 0, s, tasks, ntasks, initial, max_cycles);
}

void launch_lift(int mode, const LiftTask* tasks, int ntasks, int nblocks, hipStream_t s) {
  if (nblocks <= 0) return;
  if (mode == 0) FDS_LAUNCH(k_lift<0>, dim3(nblocks), dim3(kBlock), 0, s, tasks, ntasks);
  else FDS_LAUNCH(k_lift<1>, dim3(nblocks), dim3(kBlock), 0, s, tasks, ntasks);
}

void launch_iface(const IfaceTask* tasks, int ntasks, hipStream_t s) {
  if (ntasks <= 0) return;
  FDS_LAUNCH(k_iface, dim3(ntasks), dim3(kBlock), 0, s, tasks, ntasks);
}

void launch_res_sum(const ResSumTask* tasks, int ntasks, hipStream_t s) {
  if (ntasks <= 0) return;
  FDS_LAUNCH(k_res_sum, dim3(ntasks), dim3(kBlock), 0, s, tasks);
}

void launch_copy(const CopyTask* tasks, int ntasks, int nblocks, hipStream_t s) {
  if (nblocks <= 0) return;
  FDS_LAUNCH(k_copy, dim3(nblocks), dim3(kBlock), 0, s, tasks, ntasks);
}

void launch_residual(const ResTask* tasks, int ntasks, int nblocks, hipStream_t s) {
  if (nblocks <= 0) return;
  FDS_LAUNCH(k_residual, dim3(nblocks), dim3(kBlock), 0, s, tasks, ntasks);
}

void launch_count_active(const ProbState* st, int n, int* out, hipStream_t s) {
  FDS_LAUNCH(k_count_active, dim3(1), dim3(kBlock), 0, s, st, n, out);
}

// ------------------------------------------------ allocation-free Arnoldi step
// Working memory of fds_k_arnoldi_mgs_noalloc: Hessenberg column, Givens
// arrays, Gram matrix, block partials and hand-off counters, the problem
// state and the two task records, in one array of fixed size that each
// device holds for the life of the process.  Host code never names the
// array: it uses the device address looked up once per device below.
static __device__ __align__(256) unsigned char scratch[kNoAllocScratchBytes];

namespace {
std::mutex g_scratch_mu;
std::map<int, void*> g_scratch_ptr;
}  // namespace

void* noalloc_scratch() {
  int dev = 0;
  FDS_HIP(hipGetDevice(&dev));
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  auto it = g_scratch_ptr.find(dev);
  if (it != g_scratch_ptr.end()) return it->second;
  void* ptr = nullptr;
  FDS_HIP(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)));
  if (!ptr) throw Error(FDS_E_DEVICE, "no device address for the scratch array");
  g_scratch_ptr[dev] = ptr;
  return ptr;
}

// Zero the first n_zero doubles (partials and counters must start at zero)
// and write the state and the task records behind them; the records arrive
// as kernel arguments, so nothing is copied from host memory.
__global__ void k_noalloc_setup(double* __restrict__ zero, long long n_zero, ProbState* st,
                                ProbState hs, KryTask* dt, KryTask t0, KryTask t1) {
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n_zero;
       i += (long long)gridDim.x * blockDim.x)
    zero[i] = 0.0;
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    *st = hs;
    dt[0] = t0;
    dt[1] = t1;
  }
}

void launch_noalloc_setup(double* zero, long long n_zero, ProbState* st, const ProbState& hs,
                          KryTask* dt, const KryTask& t0, const KryTask& t1, hipStream_t s) {
  const long long per = (long long)kBlock * 8;
  const int nb = (int)std::max(1LL, std::min(1024LL, (n_zero + per - 1) / per));
  FDS_LAUNCH(k_noalloc_setup, dim3(nb), dim3(kBlock), 0, s, zero, n_zero, st, hs, dt, t0, t1);
}

}  // namespace fds
