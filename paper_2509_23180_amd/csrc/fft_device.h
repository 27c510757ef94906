// Device-side sine transform (DST-I) built on an LDS-resident mixed-radix
// Stockham FFT.  Shared by the row-transform kernel and the Schur line kernel.
//
// DST-I of length n (paper Section 2.1: the sine eigenvectors of the
// Dirichlet line matrix; the transform is evaluated through an FFT):
//   X_k = sum_{j=1..n} x_j sin(pi j k / N),  N = n + 1,  k = 1..n.
// With z the odd extension of x to length 2N (z_0 = z_N = 0, z_j = x_j,
// z_{2N-j} = -x_j) the length-2N DFT satisfies Z_k = -2i X_k.  The real
// length-2N DFT is obtained from one complex FFT of length N of
// c_t = z_{2t} + i z_{2t+1}:  Z_k = (A + B)/2 - (i/2) W^k (A - B),
// A = C_k, B = conj(C_{N-k}), W = exp(-i pi/N).  Hence
//   X_k = -(1/4) [ Im(A + B) - (cos(pi k/N) Re(A-B) + sin(pi k/N) Im(A-B)) ].
#pragma once

#include "fds_internal.h"

namespace fds {

template <typename T> struct cx;
template <> struct cx<double> { using t = double2; };
template <> struct cx<float> { using t = float2; };
template <typename T> using C2 = typename cx<T>::t;

template <typename T> __device__ __forceinline__ const C2<T>* fft_tw(const FftDesc& f);
template <> __device__ __forceinline__ const double2* fft_tw<double>(const FftDesc& f) { return f.tw64; }
template <> __device__ __forceinline__ const float2* fft_tw<float>(const FftDesc& f) { return f.tw32; }
template <typename T> __device__ __forceinline__ const C2<T>* fft_post(const FftDesc& f);
template <> __device__ __forceinline__ const double2* fft_post<double>(const FftDesc& f) { return f.post64; }
template <> __device__ __forceinline__ const float2* fft_post<float>(const FftDesc& f) { return f.post32; }
template <typename T> __device__ __forceinline__ const C2<T>* fft_kern(const FftDesc& f);
template <> __device__ __forceinline__ const double2* fft_kern<double>(const FftDesc& f) { return f.kern64; }
template <> __device__ __forceinline__ const float2* fft_kern<float>(const FftDesc& f) { return f.kern32; }
template <typename T> __device__ __forceinline__ const C2<T>* fft_chirp(const FftDesc& f);
template <> __device__ __forceinline__ const double2* fft_chirp<double>(const FftDesc& f) { return f.chirp64; }
template <> __device__ __forceinline__ const float2* fft_chirp<float>(const FftDesc& f) { return f.chirp32; }

template <typename C> __device__ __forceinline__ C cadd(C a, C b) { return C{a.x + b.x, a.y + b.y}; }
template <typename C> __device__ __forceinline__ C csub(C a, C b) { return C{a.x - b.x, a.y - b.y}; }
template <typename C, typename T> __device__ __forceinline__ C cscale(C a, T s) { return C{a.x * s, a.y * s}; }
template <typename C> __device__ __forceinline__ C cmul(C a, C b) {
  return C{a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x};
}
// multiply by -i and +i
template <typename C> __device__ __forceinline__ C cmi(C a) { return C{a.y, -a.x}; }
template <typename C> __device__ __forceinline__ C cpi(C a) { return C{-a.y, a.x}; }

// ---------------------------------------------------------------- small DFTs
// Forward DFTs (kernel exp(-2 pi i jk/R)) of fixed small sizes.
template <typename T, typename C> __device__ __forceinline__ void dft2(C* v) {
  C a = v[0], b = v[1];
  v[0] = cadd(a, b);
  v[1] = csub(a, b);
}

template <typename T, typename C> __device__ __forceinline__ void dft3(C* v) {
  const T s = T(0.866025403784438646763723170752936183);  // sin(2 pi/3)
  C t1 = cadd(v[1], v[2]);
  C t2 = csub(v[0], cscale(t1, T(0.5)));
  C d = cscale(csub(v[1], v[2]), s);
  v[0] = cadd(v[0], t1);
  v[1] = cadd(t2, cmi(d));
  v[2] = cadd(t2, cpi(d));
}

template <typename T, typename C> __device__ __forceinline__ void dft4(C* v) {
  C a = cadd(v[0], v[2]), b = csub(v[0], v[2]);
  C c = cadd(v[1], v[3]), d = csub(v[1], v[3]);
  v[0] = cadd(a, c);
  v[2] = csub(a, c);
  v[1] = cadd(b, cmi(d));
  v[3] = cadd(b, cpi(d));
}

template <typename T, typename C> __device__ __forceinline__ void dft5(C* v) {
  const T c1 = T(0.309016994374947424102293417182819059);   // cos(2 pi/5)
  const T c2 = T(-0.809016994374947424102293417182819059);  // cos(4 pi/5)
  const T s1 = T(0.951056516295153572116439333379382143);   // sin(2 pi/5)
  const T s2 = T(0.587785252292473129168705954639072769);   // sin(4 pi/5)
  C a1 = cadd(v[1], v[4]), b1 = csub(v[1], v[4]);
  C a2 = cadd(v[2], v[3]), b2 = csub(v[2], v[3]);
  C x0 = v[0];
  C r1 = cadd(x0, cadd(cscale(a1, c1), cscale(a2, c2)));
  C r2 = cadd(x0, cadd(cscale(a1, c2), cscale(a2, c1)));
  C i1 = cadd(cscale(b1, s1), cscale(b2, s2));
  C i2 = csub(cscale(b1, s2), cscale(b2, s1));
  v[0] = cadd(x0, cadd(a1, a2));
  v[1] = cadd(r1, cmi(i1));
  v[4] = cadd(r1, cpi(i1));
  v[2] = cadd(r2, cmi(i2));
  v[3] = cadd(r2, cpi(i2));
}

// Length 8: outputs 2m from the length-4 DFT of v_r + v_{r+4}, outputs
// 2m+1 from the length-4 DFT of (v_r - v_{r+4}) w8^r, w8 = exp(-i pi/4).
template <typename T, typename C> __device__ __forceinline__ void dft8(C* v) {
  const T h = T(0.707106781186547524400844362104849039);  // 1/sqrt(2)
  C a[4], b[4];
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    a[r] = cadd(v[r], v[r + 4]);
    b[r] = csub(v[r], v[r + 4]);
  }
  b[1] = C{(b[1].x + b[1].y) * h, (b[1].y - b[1].x) * h};
  b[2] = cmi(b[2]);
  b[3] = C{(b[3].y - b[3].x) * h, -(b[3].x + b[3].y) * h};
  dft4<T>(a);
  dft4<T>(b);
#pragma unroll
  for (int m = 0; m < 4; ++m) {
    v[2 * m] = a[m];
    v[2 * m + 1] = b[m];
  }
}

// Length 16 as 4 x 4: with n = r1 + 4 r2 and k = m2 + 4 m1,
// X_k = sum_{r1} w4^{r1 m1} w16^{r1 m2} sum_{r2} w4^{r2 m2} v_{r1 + 4 r2}.
template <typename T, typename C> __device__ __forceinline__ void dft16(C* v) {
  const T c1 = T(0.923879532511286756128183189396788933);  // cos(pi/8)
  const T s1 = T(0.382683432365089771728459984030398867);  // sin(pi/8)
  const T h = T(0.707106781186547524400844362104849039);
  C y[4][4];
#pragma unroll
  for (int r1 = 0; r1 < 4; ++r1) {
#pragma unroll
    for (int r2 = 0; r2 < 4; ++r2) y[r1][r2] = v[r1 + 4 * r2];
    dft4<T>(y[r1]);
  }
  // y[r1][m2] *= w16^{r1 m2}; w16^e = (cos(pi e/8), -sin(pi e/8))
  y[1][1] = cmul(y[1][1], C{c1, -s1});
  y[1][2] = cmul(y[1][2], C{h, -h});
  y[1][3] = cmul(y[1][3], C{s1, -c1});
  y[2][1] = cmul(y[2][1], C{h, -h});
  y[2][2] = cmi(y[2][2]);
  y[2][3] = cmul(y[2][3], C{-h, -h});
  y[3][1] = cmul(y[3][1], C{s1, -c1});
  y[3][2] = cmul(y[3][2], C{-h, -h});
  y[3][3] = cmul(y[3][3], C{-c1, s1});
#pragma unroll
  for (int m2 = 0; m2 < 4; ++m2) {
    C z[4] = {y[0][m2], y[1][m2], y[2][m2], y[3][m2]};
    dft4<T>(z);
#pragma unroll
    for (int m1 = 0; m1 < 4; ++m1) v[m2 + 4 * m1] = z[m1];
  }
}

template <int R, typename T, typename C> __device__ __forceinline__ void dftR(C* v) {
  if constexpr (R == 2) dft2<T>(v);
  else if constexpr (R == 3) dft3<T>(v);
  else if constexpr (R == 4) dft4<T>(v);
  else if constexpr (R == 5) dft5<T>(v);
  else if constexpr (R == 8) dft8<T>(v);
  else dft16<T>(v);
}

// One Stockham pass of fixed radix R over a row group of G threads.
//   Ns: product of the radices already applied; stw = N/(Ns R).
template <int R, typename T>
__device__ __forceinline__ void stockham_pass(const C2<T>* __restrict__ src, C2<T>* __restrict__ dst,
                                              const C2<T>* __restrict__ tw, int N, int Ns, int g,
                                              int G) {
  using C = C2<T>;
  const int NR = N / R;
  const int stw = N / (Ns * R);
  for (int j = g; j < NR; j += G) {
    const int k = j % Ns;
    C v[R];
#pragma unroll
    for (int r = 0; r < R; ++r) v[r] = src[j + r * NR];
    if (k != 0) {
#pragma unroll
      for (int r = 1; r < R; ++r) v[r] = cmul(v[r], tw[r * k * stw]);
    }
    dftR<R, T>(v);
    const int base = (j - k) * R + k;
#pragma unroll
    for (int r = 0; r < R; ++r) dst[base + r * Ns] = v[r];
  }
}

// Generic radix (any R dividing N): every output is a length-R sum whose
// combined twiddle index is r (k stw + q N/R) mod N.
template <typename T>
__device__ __forceinline__ void generic_pass(const C2<T>* __restrict__ src, C2<T>* __restrict__ dst,
                                             const C2<T>* __restrict__ tw, int N, int Ns, int R,
                                             int g, int G) {
  using C = C2<T>;
  const int NR = N / R;
  const int stw = N / (Ns * R);
  for (int o = g; o < N; o += G) {
    const int k = o % Ns;
    const int q = (o / Ns) % R;
    const int jb = o / (Ns * R);
    const int j = jb * Ns + k;
    const int step = (k * stw + q * NR) % N;
    int idx = 0;
    C acc = C{T(0), T(0)};
    for (int r = 0; r < R; ++r) {
      const C a = src[j + r * NR];
      const C w = tw[idx];
      acc.x += a.x * w.x - a.y * w.y;
      acc.y += a.x * w.y + a.y * w.x;
      idx += step;
      if (idx >= N) idx -= N;
    }
    dst[o] = acc;
  }
}

// Stockham FFT of length L (radix schedule `radix`) in LDS buffer `a`
// (scratch `b`).  Every group of the block must run the same schedule
// (block-wide barriers).  Returns the buffer holding the result.
template <typename T>
__device__ C2<T>* stockham_lds(C2<T>* a, C2<T>* b, int L, int npass, const int* radix,
                               const C2<T>* tw, int g, int G) {
  int Ns = 1;
  C2<T>* src = a;
  C2<T>* dst = b;
  for (int p = 0; p < npass; ++p) {
    const int R = radix[p];
    switch (R) {
      case 2: stockham_pass<2, T>(src, dst, tw, L, Ns, g, G); break;
      case 3: stockham_pass<3, T>(src, dst, tw, L, Ns, g, G); break;
      case 4: stockham_pass<4, T>(src, dst, tw, L, Ns, g, G); break;
      case 5: stockham_pass<5, T>(src, dst, tw, L, Ns, g, G); break;
      case 8: stockham_pass<8, T>(src, dst, tw, L, Ns, g, G); break;
      case 16: stockham_pass<16, T>(src, dst, tw, L, Ns, g, G); break;
      default: generic_pass<T>(src, dst, tw, L, Ns, R, g, G); break;
    }
    __syncthreads();
    C2<T>* t = src;
    src = dst;
    dst = t;
    Ns *= R;
  }
  return src;
}

// Complex FFT of length f.N of the data in LDS buffer `a` (scratch `b`; both
// hold max(N, L) entries).  Returns the buffer holding the N outputs.
template <typename T>
__device__ C2<T>* fft_lds(C2<T>* a, C2<T>* b, const FftDesc& f, const C2<T>* tw, int g, int G) {
  using C = C2<T>;
  if (f.kind == FFT_MIXED) return stockham_lds<T>(a, b, f.N, f.npass, f.radix, tw, g, G);
  const int N = f.N, L = f.L;
  const C* K = fft_kern<T>(f);
  if (f.kind == FFT_RADER) {
    // X_0 = x_0 + sum_{j>0} x_j;  X_{g^m} = x_0 + (a~ * b)_m with a~_q = x_{g^{-q}}
    const C x0 = a[0];
    for (int q = g; q < L; q += G) b[q] = a[f.perm_in[q]];
    __syncthreads();
    C* r = stockham_lds<T>(b, a, L, f.npass, f.radix, tw, g, G);
    const C X0 = C{x0.x + r[0].x, x0.y + r[0].y};
    C* o = (r == a) ? b : a;
    for (int t = g; t < L; t += G) {
      const C v = cmul(r[t], K[t]);
      o[t] = C{v.x, -v.y};
    }
    __syncthreads();
    C* r2 = stockham_lds<T>(o, r, L, f.npass, f.radix, tw, g, G);
    C* fin = (r2 == a) ? b : a;
    for (int m = g; m < L; m += G) {
      const C v = r2[m];
      fin[f.perm_out[m]] = C{x0.x + v.x, x0.y - v.y};
    }
    if (g == 0) fin[0] = X0;
    __syncthreads();
    return fin;
  }
  // Bluestein: X_k = c_k sum_j (x_j c_j) conj(c_{k-j}),  c_t = exp(-i pi t^2/N)
  const C* ch = fft_chirp<T>(f);
  for (int j = g; j < L; j += G) a[j] = (j < N) ? cmul(a[j], ch[j]) : C{T(0), T(0)};
  __syncthreads();
  C* r = stockham_lds<T>(a, b, L, f.npass, f.radix, tw, g, G);
  C* o = (r == a) ? b : a;
  for (int t = g; t < L; t += G) {
    const C v = cmul(r[t], K[t]);
    o[t] = C{v.x, -v.y};
  }
  __syncthreads();
  C* r2 = stockham_lds<T>(o, r, L, f.npass, f.radix, tw, g, G);
  C* fin = (r2 == a) ? b : a;
  for (int k = g; k < N; k += G) {
    const C v = r2[k];
    fin[k] = cmul(ch[k], C{v.x, -v.y});
  }
  __syncthreads();
  return fin;
}

// Pack the odd extension of a real row into c_t = z_{2t} + i z_{2t+1}.
// `load(j)` returns x_j for 1 <= j <= n.
template <typename T, typename Load>
__device__ __forceinline__ void dst_pack(C2<T>* a, int N, int g, int G, Load load) {
  for (int t = g; t < N; t += G) {
    T v[2];
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const int j = 2 * t + h;
      T z = T(0);
      if (j > 0 && j < N) z = load(j);
      else if (j > N) z = -load(2 * N - j);
      v[h] = z;
    }
    a[t] = C2<T>{v[0], v[1]};
  }
}

// X_k from the complex FFT result C (k = 1..N-1).
template <typename T>
__device__ __forceinline__ T dst_post(const C2<T>* C, const C2<T>* post, int N, int k) {
  const C2<T> A = C[k];
  const C2<T> Bc = C[N - k];
  const C2<T> w = post[k];
  const T imsum = A.y - Bc.y;
  const T dre = A.x - Bc.x;
  const T dim = A.y + Bc.y;
  return T(-0.25) * (imsum - (w.x * dre + w.y * dim));
}

// Copy the twiddle table of the Stockham FFT into LDS (whole block).
template <typename T>
__device__ __forceinline__ const C2<T>* stage_twiddles(const FftDesc& f, C2<T>* lds, bool use) {
  const C2<T>* tw = fft_tw<T>(f);
  if (!use) return tw;
  for (int t = threadIdx.x; t < f.L; t += blockDim.x) lds[t] = tw[t];
  return lds;
}

// ---------------------------------------------------------------- cross-block hand-off
// The last block of a problem to finish a launch does the problem's serial
// work (partials are added in a fixed order, so the result does not depend
// on which block is last).  Partials that another block of the same launch
// reads are stored and loaded as agent-scope relaxed atomics, which the
// memory model keeps coherent across the XCDs' L2 caches; a device-wide fence
// would instead write back and invalidate the whole L2 in every block.  Each
// block waits for its stores to complete, then counts itself in; the last
// block resets the counter for the next launch.
__device__ __forceinline__ void st_agent(double* p, double v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ double ld_agent(const double* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

#if defined(FDS_HANDOFF_FENCED)
// Release/acquire form (build option): the block's stores are ordered before
// the counter increment by a workgroup barrier and an agent-scope release on
// the increment; the last block takes an agent-scope acquire before it reads.
// On gfx950 the release writes back the XCD's L2 and the acquire invalidates
// it, which the relaxed form below avoids.
__device__ __forceinline__ bool last_block_of_problem(int* ctr, int nblocks, int* sflag) {
  __syncthreads();
  if (threadIdx.x == 0) {
    const int old = __hip_atomic_fetch_add(ctr, 1, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT);
    const int last = (old == nblocks - 1) ? 1 : 0;
    if (last) __hip_atomic_store(ctr, 0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    *sflag = last;
  }
  __syncthreads();
  const bool last = *sflag != 0;
  if (last) __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
  return last;
}
#else
// Relaxed form (default).  Ordering without fences: (1) every partial is an
// agent-scope atomic store, which gfx950 writes through to the coherent level
// past the XCD's L2; (2) `s_waitcnt vmcnt(0)` waits until those stores have
// completed, and its "memory" clobber, like the barrier after it, keeps the
// compiler from moving any memory access across; (3) only then does thread 0
// increment the counter; (4) the last block issues its agent-scope atomic
// loads of the partials after the increment has returned, behind a barrier,
// so they cannot be hoisted above it and they bypass the non-coherent L2.
__device__ __forceinline__ bool last_block_of_problem(int* ctr, int nblocks, int* sflag) {
  asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
  __syncthreads();
  if (threadIdx.x == 0) {
    const int old = __hip_atomic_fetch_add(ctr, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    const int last = (old == nblocks - 1) ? 1 : 0;
    if (last) __hip_atomic_store(ctr, 0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    *sflag = last;
  }
  __syncthreads();
  return *sflag != 0;
}
#endif

// ---------------------------------------------------------------- reductions
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// Wavefront sum with DPP lane moves (register to register, no LDS crossbar):
// quad swaps, half-row and row mirrors, then the row broadcasts of lanes 15
// and 31.  The full sum is valid in lane 63 only.
template <int CTRL, int ROW_MASK>
__device__ __forceinline__ double dpp_add(double v) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_update_dpp(0, (int)b, CTRL, ROW_MASK, 0xf, false);
  const int hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), CTRL, ROW_MASK, 0xf, false);
  return v + __longlong_as_double(((long long)hi << 32) | (long long)(unsigned)lo);
}
__device__ __forceinline__ double wave_sum_last(double v) {
  v = dpp_add<0xB1, 0xf>(v);    // quad_perm [1,0,3,2]
  v = dpp_add<0x4E, 0xf>(v);    // quad_perm [2,3,0,1]
  v = dpp_add<0x141, 0xf>(v);   // row_half_mirror
  v = dpp_add<0x140, 0xf>(v);   // row_mirror: every lane holds its row's sum
  v = dpp_add<0x142, 0xa>(v);   // row_bcast:15 into rows 1 and 3
  v = dpp_add<0x143, 0xc>(v);   // row_bcast:31 into rows 2 and 3
  return v;
}

// Sum over a block of kBlock threads; every thread receives the same bits.
__device__ __forceinline__ double block_sum(double v, double* red) {
  v = wave_sum(v);
  const int w = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 0) red[w] = v;
  __syncthreads();
  const double r = (red[0] + red[1]) + (red[2] + red[3]);
  __syncthreads();
  return r;
}

// Fixed-order sum of P partials (identical result in every block).
__device__ __forceinline__ double sum_partials(const double* p, int P, double* red) {
  double acc = 0.0;
  for (int i = threadIdx.x; i < P; i += kBlock) acc += p[i];
  return block_sum(acc, red);
}

// Task of this block: the last record with block_begin <= blockIdx.x
// (records are sorted by block_begin).  The first wave compares 64 records
// per load round and counts with a ballot, so the search costs one dependent
// load per 64 records; the result is made wave-uniform so that the record's
// fields are read with scalar loads.
template <typename Task>
__device__ __forceinline__ int find_task(const Task* tasks, int ntasks, int* slot) {
  if (threadIdx.x < 64) {
    const int b = blockIdx.x;
    int cnt = 0;
    for (int t0 = 0; t0 < ntasks; t0 += 64) {
      const int t = t0 + (int)threadIdx.x;
      const bool le = t < ntasks && tasks[t].block_begin <= b;
      const unsigned long long m = __ballot(le);
      cnt += __popcll(m);
      if (m != ~0ull) break;
    }
    if (threadIdx.x == 0) *slot = cnt - 1;
  }
  __syncthreads();
  return __builtin_amdgcn_readfirstlane(*slot);
}

}  // namespace fds
