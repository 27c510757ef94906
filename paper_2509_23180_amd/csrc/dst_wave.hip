// Wave-parallel row sine transform kernel and its launcher.
#include "kernels.h"

#include "fft_device.h"
#include "fft_wave.h"

namespace fds {

// =====================================================================
// Wave-parallel row sine transform.  G = blockDim.x / rpb lanes per row
// (16, 32 or 64); E is the register budget of a pass (complex entries per
// lane).  The row is read once, coalesced, and scattered into the packed
// odd extension c_t = z_{2t} + i z_{2t+1} in LDS; the table image is copied
// to LDS in the same phase, and after one workgroup barrier every row group
// runs on its own.
// =====================================================================
// Row element j (1..n) of `p` as T; `f32` selects the storage type.
template <typename T>
__device__ __forceinline__ T io_load(const void* p, bool f32, long long i) {
  return f32 ? T(static_cast<const float*>(p)[i]) : T(static_cast<const double*>(p)[i]);
}
template <typename T>
__device__ __forceinline__ void io_store(void* p, bool f32, long long i, T v) {
  if (f32) static_cast<float*>(p)[i] = float(v);
  else static_cast<double*>(p)[i] = double(v);
}

//
// BIG: one row per workgroup (G = blockDim.x = 128, 256 or 512 lanes) for rows
// whose buffer and tables do not fit LDS together.  The passes are separated
// by workgroup barriers, and the tables are read from the global image (it
// stays resident in L2); LDS holds the row only.
template <typename T, int E, bool BIG>
__global__ void __launch_bounds__(BIG ? 512 : 256) k_dst_wave(const DstTask* __restrict__ tasks, int ntasks,
                                                  int jidx) {
  using C = C2<T>;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  __shared__ int slot;
  const DstTask& tk = tasks[find_task(tasks, ntasks, &slot)];
  if (tk.skip && *tk.skip) return;
  const WaveDesc& d = tk.wd;
  const int N = d.N, n = tk.n;
  const int rpb = BIG ? 1 : tk.rpb;
  const int G = (int)blockDim.x / rpb;
  const int grp = BIG ? 0 : (int)threadIdx.x / G;
  const int g = (int)threadIdx.x - grp * G;
  const int row = (blockIdx.x - tk.block_begin) * rpb + grp;
  const bool valid = row < tk.rows;
  const bool in32 = (tk.io_f32 & 1) != 0, out32 = (tk.io_f32 & 2) != 0;
  const WaveLayout lay = wave_layout<T>(d.kind, N, d.L, d.W, d.twlen);
  const unsigned char* tabs = BIG ? reinterpret_cast<const unsigned char*>(d.img) : smem_raw;
  C* buf = reinterpret_cast<C*>(smem_raw + (BIG ? 0 : lay.rows + grp * lay.row_bytes));
  T* bz = reinterpret_cast<T*>(buf);

  // ---- issue the row loads, the normalisation factor and the table image
  // together (the index is clamped so that every load is in bounds and none
  // waits behind a branch)
  const long long ioff = (long long)jidx * tk.in_js + (long long)(valid ? row : 0) * tk.in_rs;
  const long long ics = tk.in_cs;
  const double sc = tk.in_scale ? *tk.in_scale : 1.0;
  T x[E];
#pragma unroll
  for (int i = 0; i < E; ++i) {
    const int j = 1 + g + i * G;
    x[i] = io_load<T>(tk.in, in32, ioff + (long long)((j <= n ? j : 1) - 1) * ics);
  }
  if constexpr (!BIG) {
    const uint4* img = d.img;
    const int nch = d.img_chunks, last = nch - 1;
    uint4* dst = reinterpret_cast<uint4*>(smem_raw);
    const int bd = (int)blockDim.x;
    for (int c = (int)threadIdx.x; c < nch; c += 4 * bd) {
      const uint4 a0 = img[c];
      const uint4 a1 = img[min(c + bd, last)];
      const uint4 a2 = img[min(c + 2 * bd, last)];
      const uint4 a3 = img[min(c + 3 * bd, last)];
      dst[c] = a0;
      if (c + bd < nch) dst[c + bd] = a1;
      if (c + 2 * bd < nch) dst[c + 2 * bd] = a2;
      if (c + 3 * bd < nch) dst[c + 3 * bd] = a3;
    }
  }
  // ---- normalisation (the basis vector is written back once, scaled)
  if (tk.in_scale) {
    void* inw = const_cast<void*>(tk.in);
#pragma unroll
    for (int i = 0; i < E; ++i) {
      const int j = 1 + g + i * G;
      const double v = double(x[i]) * sc;
      x[i] = T(v);
      if (valid && j <= n) io_store<double>(inw, in32, ioff + (long long)(j - 1) * ics, v);
    }
  }
  // ---- scatter into the packed odd extension: z_j = x_j, z_{2N-j} = -x_j,
  // z_0 = z_N = 0; z_m is component m & 1 of c_{m >> 1}
#pragma unroll
  for (int i = 0; i < E; ++i) {
    const int j = 1 + g + i * G;
    if (j <= n) {
      bz[2 * wpad<T>(j >> 1) + (j & 1)] = x[i];
      const int m = 2 * N - j;
      bz[2 * wpad<T>(m >> 1) + (m & 1)] = -x[i];
    }
  }
  if (g == 0) {
    bz[0] = T(0);
    bz[2 * wpad<T>(N >> 1) + (N & 1)] = T(0);
  }
  __syncthreads();
  if (!valid) return;

  wave_row_fft<T, E, BIG>(buf, d, tabs, lay, g, G);

  // ---- X_k = -(1/4)[Im(A+B) - (cos(pi k/N) Re(A-B) + sin(pi k/N) Im(A-B))],
  // A = C_k, B = conj(C_{N-k}); all LDS reads first, then the stores
  const auto post = tab_at<BIG, C>(tabs, lay.post);
  const long long ooff = (long long)jidx * tk.out_js + (long long)row * tk.out_rs;
  const T scale = T(tk.scale);
  const long long ocs = tk.out_cs;
  T X[E];
#pragma unroll
  for (int i = 0; i < E; ++i) {
    const int k0 = 1 + g + i * G;
    const int k = k0 <= n ? k0 : 1;
    const C A = buf[wpad<T>(k)];
    const C Bc = buf[wpad<T>(N - k)];
    const C w = post[k];
    X[i] = scale * (T(-0.25) * ((A.y - Bc.y) - (w.x * (A.x - Bc.x) + w.y * (A.y + Bc.y))));
  }
  if (tk.accumulate) {
    T prev[E];
#pragma unroll
    for (int i = 0; i < E; ++i) {
      const int k0 = 1 + g + i * G;
      prev[i] = io_load<T>(tk.out, out32, ooff + (long long)((k0 <= n ? k0 : 1) - 1) * ocs);
    }
#pragma unroll
    for (int i = 0; i < E; ++i) X[i] += prev[i];
  }
#pragma unroll
  for (int i = 0; i < E; ++i) {
    const int k = 1 + g + i * G;
    if (k <= n) io_store<T>(tk.out, out32, ooff + (long long)(k - 1) * ocs, X[i]);
  }
}

template <typename T, int E, bool BIG>
static void launch_wave_e(const DstTask* tasks, int ntasks, int nblocks, int threads, size_t smem,
                          int jidx, hipStream_t s) {
  static size_t granted = 0;
  ensure_smem(k_dst_wave<T, E, BIG>, smem, &granted);
  FDS_LAUNCH((k_dst_wave<T, E, BIG>), dim3(nblocks), dim3(threads), smem, s, tasks, ntasks, jidx);
}

template <typename T>
static void launch_wave_t(int E, bool big, const DstTask* tasks, int ntasks, int nblocks, int threads,
                          size_t smem, int jidx, hipStream_t s) {
  if (big) {
    switch (E) {
      case 8: launch_wave_e<T, 8, true>(tasks, ntasks, nblocks, threads, smem, jidx, s); return;
      case 16: launch_wave_e<T, 16, true>(tasks, ntasks, nblocks, threads, smem, jidx, s); return;
      case 32: launch_wave_e<T, 32, true>(tasks, ntasks, nblocks, threads, smem, jidx, s); return;
      default: break;
    }
  } else {
    switch (E) {
      case 4: launch_wave_e<T, 4, false>(tasks, ntasks, nblocks, threads, smem, jidx, s); return;
      case 8: launch_wave_e<T, 8, false>(tasks, ntasks, nblocks, threads, smem, jidx, s); return;
      case 16: launch_wave_e<T, 16, false>(tasks, ntasks, nblocks, threads, smem, jidx, s); return;
      case 32: launch_wave_e<T, 32, false>(tasks, ntasks, nblocks, threads, smem, jidx, s); return;
      case 64:
        if constexpr (sizeof(T) == 4) {
          launch_wave_e<T, 64, false>(tasks, ntasks, nblocks, threads, smem, jidx, s);
          return;
        }
        break;
      default: break;
    }
  }
  throw Error(FDS_E_UNSUPPORTED, "wave transform: register budget out of range");
}

void launch_dst_wave(DstKind kind, int E, bool big, const DstTask* tasks, int ntasks, int nblocks,
                     int threads, size_t smem, int jidx, hipStream_t s) {
  if (nblocks <= 0) return;
  if (threads != 64 && threads != 128 && threads != 256 && !(big && threads == 512))
    throw Error(FDS_E_INVALID_ARG, "wave transform: bad workgroup size");
  if (kind == DstKind::D_D) launch_wave_t<double>(E, big, tasks, ntasks, nblocks, threads, smem, jidx, s);
  else launch_wave_t<float>(E, big, tasks, ntasks, nblocks, threads, smem, jidx, s);
}

}  // namespace fds
