// Wave-parallel sine transform of rows (DST-I through the packed complex FFT
// of length N = n + 1 described in fft_device.h).
//
// A group of G lanes (G = 16, 32 or 64, so a group never straddles a
// wavefront) owns one row and one LDS buffer.  Every Stockham pass first reads
// all of its butterfly inputs into registers and only then writes its
// outputs, so a pass runs in place; lanes of one wavefront execute their LDS
// instructions in order, so the passes need no workgroup barrier.  Radix-8
// and radix-16 butterflies run in registers, which halves the LDS round trips
// of a radix-4 schedule.  The Rader permutations and the convolution kernel
// multiply are folded into the first and last passes of the inner FFTs.
// Twiddles, permutations, kernels and the post-processing table are copied to
// LDS once per workgroup, while the rows are being loaded.
#pragma once

#include "fft_device.h"

namespace fds {

// Compiler-level fence between the read phase and the write phase of a pass
// (the hardware keeps a wavefront's LDS operations in order).
__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
  __builtin_amdgcn_wave_barrier();
}

// Barrier between the phases of a pass: the wavefront's own when a row
// lives in one wavefront, the workgroup's when a row spans the workgroup.
template <bool BIG>
__device__ __forceinline__ void row_sync() {
  if constexpr (BIG) __syncthreads();
  else wave_sync();
}

// Pointer into the table image: generic (the image in LDS) or, for BIG, a
// global-address-space pointer, so that the compiler knows table reads do not
// alias the row buffer and can issue them ahead of the pass's LDS stores.
template <bool BIG, typename U>
struct TabPtr {
  using type = const U*;
};
template <typename U>
struct TabPtr<true, U> {
#if defined(__HIP_DEVICE_COMPILE__)
  using type = const U __attribute__((address_space(1)))*;
#else
  using type = const U*;   // host pass: the kernel body is never run there
#endif
};
template <bool BIG, typename U>
__device__ __forceinline__ typename TabPtr<BIG, U>::type tab_at(const unsigned char* base, int off) {
  return (typename TabPtr<BIG, U>::type)(base + off);
}

// q = j / d for 0 <= j < 2^22, d >= 1, via a float reciprocal and one fix-up.
__device__ __forceinline__ int wdiv(int j, int d, float rd) {
  int q = (int)((float)j * rd);
  if (q * d > j) --q;
  else if ((q + 1) * d <= j) ++q;
  return q;
}

// One in-place Stockham pass of radix R over a length-L FFT held by G lanes.
// `load(q)` supplies input q on the first pass, `store(t, v)` takes output t
// on the last pass; other passes read and write `buf`.  `tw` is this pass's
// twiddle table ((r-1) Ns + k); the first pass (Ns = 1) has none to apply.
// With TWE the twiddles are read together with the data (one LDS wait per
// pass) at the cost of holding them in registers.
template <int R, typename T, int E, bool TWE, bool BIG, typename TW, typename Load, typename Store>
__device__ __forceinline__ void wave_pass(C2<T>* buf, TW tw, int L, int Ns, int g, int G,
                                          bool first, bool last, Load& load, Store& store) {
  using C = C2<T>;
  constexpr int NB = E / R;
  // Launder L and g so that the pass addresses are formed here and not
  // hoisted out of the caller's pass loop for every radix at once (that
  // costs hundreds of registers).
  asm volatile("" : "+v"(L), "+v"(g));
  const int NR = L / R;
  const float rNs = 1.0f / (float)Ns;
  const bool twid = Ns > 1;
  C v[NB][R];
  C w[TWE ? NB : 1][TWE ? R : 1];
  int kk[NB];
#pragma unroll
  for (int b = 0; b < NB; ++b) {
    const int j = g + b * G;
    kk[b] = j - wdiv(j, Ns, rNs) * Ns;
    if (j < NR) {
      if (first) {
#pragma unroll
        for (int r = 0; r < R; ++r) v[b][r] = load(j + r * NR);
      } else {
#pragma unroll
        for (int r = 0; r < R; ++r) v[b][r] = buf[wpad<T>(j + r * NR)];
      }
      if constexpr (TWE) {
        if (twid) {
#pragma unroll
          for (int r = 1; r < R; ++r) w[b][r] = tw[(r - 1) * Ns + kk[b]];
        }
      }
    }
  }
  row_sync<BIG>();
#pragma unroll
  for (int b = 0; b < NB; ++b) {
    const int j = g + b * G;
    if (j < NR) {
      const int k = kk[b];
      if (twid) {
#pragma unroll
        for (int r = 1; r < R; ++r) {
          if constexpr (TWE) v[b][r] = cmul(v[b][r], w[b][r]);
          else v[b][r] = cmul(v[b][r], tw[(r - 1) * Ns + k]);
        }
      }
      dftR<R, T>(v[b]);
      const int base = (j - k) * R + k;
      if (last) {
#pragma unroll
        for (int r = 0; r < R; ++r) store(base + r * Ns, v[b][r]);
      } else {
#pragma unroll
        for (int r = 0; r < R; ++r) buf[wpad<T>(base + r * Ns)] = v[b][r];
      }
    }
  }
  row_sync<BIG>();
}

// Length-L FFT in place in `buf` with the radix schedule of `d` (all radices
// in {2, 3, 4, 5, 8, 16}; the host checks this and the register budget E).
template <typename T, int E, bool BIG, typename TW, typename Load, typename Store>
__device__ __forceinline__ void wave_fft(C2<T>* buf, TW tw, const WaveDesc& d, int g, int G, Load load,
                                         Store store) {
  constexpr bool TWE = E * sizeof(T) <= 128;
  const int L = d.L, np = d.npass;
  int Ns = 1;
  TW twp = tw;
  for (int p = 0; p < np; ++p) {
    const int R = (int)((d.radices >> (5 * p)) & 31u);
    const bool first = p == 0, last = p == np - 1;
    // (a radix above E never occurs: the host sizes E for the schedule)
    switch (R) {
      case 16:
        if constexpr (E >= 16) wave_pass<16, T, E, TWE, BIG>(buf, twp, L, Ns, g, G, first, last, load, store);
        break;
      case 8:
        if constexpr (E >= 8) wave_pass<8, T, E, TWE, BIG>(buf, twp, L, Ns, g, G, first, last, load, store);
        break;
      case 4: wave_pass<4, T, E, TWE, BIG>(buf, twp, L, Ns, g, G, first, last, load, store); break;
      case 2: wave_pass<2, T, E, TWE, BIG>(buf, twp, L, Ns, g, G, first, last, load, store); break;
      case 3: wave_pass<3, T, E, TWE, BIG>(buf, twp, L, Ns, g, G, first, last, load, store); break;
      default:
        if constexpr (E >= 5) wave_pass<5, T, E, TWE, BIG>(buf, twp, L, Ns, g, G, first, last, load, store);
        break;
    }
    twp += (R - 1) * Ns;
    Ns *= R;
  }
}

// Complex FFT of length N of the packed row in `buf` (positions 0..N-1),
// result in natural order at positions 0..N-1.
// `tabs` is the table image: in LDS, or the global image itself when BIG.
template <typename T, int E, bool BIG>
__device__ __forceinline__ void wave_row_fft(C2<T>* buf, const WaveDesc& d, const unsigned char* tabs,
                                             const WaveLayout& lay, int g, int G) {
  using C = C2<T>;
  const auto tw = tab_at<BIG, C>(tabs, lay.tw);
  const int kind = d.kind, N = d.N, L = d.L;
  if (kind == FFT_MIXED) {
    wave_fft<T, E, BIG>(buf, tw, d, g, G, [&](int q) { return buf[wpad<T>(q)]; },
                   [&](int t, C v) { buf[wpad<T>(t)] = v; });
    return;
  }
  const auto K = tab_at<BIG, C>(tabs, lay.kern);
  if (kind == FFT_RADER) {
    // X_0 = sum_j x_j; X_{g^m} = x_0 + (a~ * b)_m with a~_q = x_{g^{-q}}: one FFT
    // of a~, a product with the transformed kernel, and a second FFT of the
    // conjugate (the inverse FFT up to conjugation; K carries the 1/L).
    const auto pin = tab_at<BIG, int>(tabs, lay.pin);
    const auto pout = tab_at<BIG, int>(tabs, lay.pout);
    const C x0 = buf[wpad<T>(0)];
    wave_fft<T, E, BIG>(buf, tw, d, g, G, [&](int q) { return buf[wpad<T>(pin[q])]; },
                   [&](int t, C v) {
                     if (t == 0) buf[wpad<T>(L)] = v;  // sum of x_1..x_{N-1}, kept for X_0
                     const C u = cmul(v, K[t]);
                     buf[wpad<T>(t)] = C{u.x, -u.y};
                   });
    const C s = buf[wpad<T>(L)];
    wave_fft<T, E, BIG>(buf, tw, d, g, G, [&](int q) { return buf[wpad<T>(q)]; },
                   [&](int m, C v) { buf[wpad<T>(pout[m])] = C{x0.x + v.x, x0.y - v.y}; });
    if (g == 0) buf[wpad<T>(0)] = C{x0.x + s.x, x0.y + s.y};
    row_sync<BIG>();
    return;
  }
  // Bluestein: X_k = c_k sum_j (x_j c_j) conj(c_{k-j}), c_t = exp(-i pi t^2/N),
  // as a cyclic convolution of length L >= 2N - 1.
  const auto ch = tab_at<BIG, C>(tabs, lay.chirp);
  wave_fft<T, E, BIG>(buf, tw, d, g, G,
                 [&](int q) { return q < N ? cmul(buf[wpad<T>(q)], ch[q]) : C{T(0), T(0)}; },
                 [&](int t, C v) {
                   const C u = cmul(v, K[t]);
                   buf[wpad<T>(t)] = C{u.x, -u.y};
                 });
  wave_fft<T, E, BIG>(buf, tw, d, g, G, [&](int q) { return buf[wpad<T>(q)]; },
                 [&](int k, C v) {
                   if (k < N) buf[wpad<T>(k)] = cmul(ch[k], C{v.x, -v.y});
                 });
}

}  // namespace fds
