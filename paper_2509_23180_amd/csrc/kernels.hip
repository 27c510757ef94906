// HIP kernels of the hot path (gfx950).  Every kernel works on a list of
// task records so one launch serves all rectangles / problems of a batch.
#include "kernels.h"

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
  C2<T>* A = reinterpret_cast<C2<T>*>(smem_raw) + (size_t)grp * 2 * f.W;
  C2<T>* B = A + f.W;
  const TIn* in = static_cast<const TIn*>(tk.in) + (long long)jidx * tk.in_js +
                  (long long)(valid ? row : 0) * tk.in_rs;
  const long long ics = tk.in_cs;
  if (valid) {
    dst_pack<T>(A, N, g, G, [&](int j) { return T(in[(long long)(j - 1) * ics]); });
  }
  __syncthreads();
  const C2<T>* Cr = fft_lds<T>(A, B, f, g, G);
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
  T w = T(0), s = T(0), p = T(1);
#pragma unroll 4
  for (int i = 0; i < m; ++i) {
    w = c.sc * d[i * rs] + c.q * w;
    d[i * rs] = w;
    s += p * w;
    p *= c.q;
  }
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

// =====================================================================
// Schur line terms: out = delta^2 (2/N) S diag(g) S z_line (FP64).
// One block per line; two sine transforms in LDS.
// =====================================================================
__global__ void __launch_bounds__(kBlock) k_schur_lines(const LineTask* __restrict__ tasks, int jidx) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  const LineTask& tk = tasks[blockIdx.x];
  if (tk.skip && *tk.skip) return;
  const FftDesc& f = *tk.fft;
  const int N = f.N;
  const int L = tk.L;
  double2* A = reinterpret_cast<double2*>(smem_raw);
  double2* B = A + f.W;
  double* mid = reinterpret_cast<double*>(B + f.W);
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
  const double2* C = fft_lds<double>(A, B, f, g, kBlock);
  for (int k = 1 + g; k <= L; k += kBlock) mid[k - 1] = tk.gs[k - 1] * dst_post<double>(C, f.post64, N, k);
  __syncthreads();
  dst_pack<double>(A, N, g, kBlock, [&](int j) { return mid[j - 1]; });
  __syncthreads();
  C = fft_lds<double>(A, B, f, g, kBlock);
  for (int k = 1 + g; k <= L; k += kBlock) tk.out[k - 1] = dst_post<double>(C, f.post64, N, k);
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
// Arnoldi, modified Gram-Schmidt.  Pass i (0 <= i <= j+1) of step j:
//   i > 0:   h_{i-1,j} = sum of the previous pass's partials;
//            w -= h_{i-1,j} v_{i-1}
//   i <= j:  partials of <w, v_i>;  i == j+1: partials of <w, w>
// w lives in V[j+1].
// =====================================================================
__global__ void __launch_bounds__(kBlock) k_mgs_pass(const KryTask* __restrict__ tasks, int ntasks,
                                                      int i, int j) {
  __shared__ int slot;
  __shared__ double red[4];
  const KryTask& tk = tasks[find_task(tasks, ntasks, &slot)];
  if (tk.st->cycle_done) return;
  const int b = blockIdx.x - tk.block_begin;
  const long long Nc = tk.Nc;
  const int P = tk.P;
  double* w = tk.V + (long long)(j + 1) * Nc;
  double hprev = 0.0;
  if (i > 0) {
    hprev = sum_partials(tk.partials + ((i - 1) & 1) * P, P, red);
    if (b == 0 && threadIdx.x == 0) tk.H[(i - 1) + j * (tk.m + 1)] = hprev;
  }
  const double* vprev = tk.V + (long long)(i > 0 ? i - 1 : 0) * Nc;
  const double* vi = tk.V + (long long)(i <= j ? i : 0) * Nc;
  double acc = 0.0;
  const long long base = (long long)b * kVecPerBlock;
#pragma unroll
  for (int e = 0; e < kVecEPT; ++e) {
    const long long idx = base + (long long)e * kBlock + threadIdx.x;
    if (idx < Nc) {
      double wv = w[idx];
      if (i > 0) {
        wv -= hprev * vprev[idx];
        w[idx] = wv;
      }
      acc += (i <= j) ? wv * vi[idx] : wv * wv;
    }
  }
  const double s = block_sum(acc, red);
  if (threadIdx.x == 0) tk.partials[(i & 1) * P + b] = s;
}

// Norm, normalisation of v_{j+1}, Givens update of column j and the
// convergence test on |g_{j+1}| (block 0, thread 0).
__global__ void __launch_bounds__(kBlock) k_mgs_finish(const KryTask* __restrict__ tasks, int ntasks,
                                                        int j) {
  __shared__ int slot;
  __shared__ double red[4];
  const KryTask& tk = tasks[find_task(tasks, ntasks, &slot)];
  ProbState* st = tk.st;
  if (st->cycle_done) return;
  const int b = blockIdx.x - tk.block_begin;
  const long long Nc = tk.Nc;
  const double nrm2 = sum_partials(tk.partials + ((j + 1) & 1) * tk.P, tk.P, red);
  const double hn = sqrt(nrm2);
  const bool breakdown = !(hn > 1e-14 * st->beta);
  if (!breakdown) {
    const double inv = 1.0 / hn;
    double* w = tk.V + (long long)(j + 1) * Nc;
    const long long base = (long long)b * kVecPerBlock;
#pragma unroll
    for (int e = 0; e < kVecEPT; ++e) {
      const long long idx = base + (long long)e * kBlock + threadIdx.x;
      if (idx < Nc) w[idx] *= inv;
    }
  }
  if (b == 0 && threadIdx.x == 0) {
    const int m1 = tk.m + 1;
    double* H = tk.H;
    H[(j + 1) + j * m1] = hn;
    st->last_hn = hn;
    for (int i = 0; i < j; ++i) {
      const double a = H[i + j * m1], c2 = H[(i + 1) + j * m1];
      H[i + j * m1] = tk.cs[i] * a + tk.sn[i] * c2;
      H[(i + 1) + j * m1] = -tk.sn[i] * a + tk.cs[i] * c2;
    }
    const double a = H[j + j * m1];
    const double rho = hypot(a, hn);
    double c = 1.0, s = 0.0;
    if (rho > 0.0) {
      c = a / rho;
      s = hn / rho;
    }
    tk.cs[j] = c;
    tk.sn[j] = s;
    H[j + j * m1] = rho;
    H[(j + 1) + j * m1] = 0.0;
    const double gj = tk.g[j];
    tk.g[j + 1] = -s * gj;
    tk.g[j] = c * gj;
    st->j_done = j + 1;
    st->iterations += 1;
    const double est = fabs(tk.g[j + 1]);
    if (!(est > st->tol_eff * st->fnorm) || breakdown || j + 1 == tk.m) st->cycle_done = 1;
  }
}

// Back substitution R y = g over the j_done columns (one thread per problem).
__global__ void k_ls_solve(const KryTask* __restrict__ tasks, int ntasks) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= ntasks) return;
  const KryTask& tk = tasks[t];
  if (tk.st->finished) return;
  const int k = tk.st->j_done;
  const int m1 = tk.m + 1;
  for (int i = k - 1; i >= 0; --i) {
    double s = tk.g[i];
    for (int l = i + 1; l < k; ++l) s -= tk.H[i + l * m1] * tk.y[l];
    const double d = tk.H[i + i * m1];
    tk.y[i] = (d != 0.0) ? s / d : 0.0;
  }
}

// u = V y (plain variant) or x += Z y (flexible variant).
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
        tk.x[idx] += acc;
      } else {
        for (int i = 0; i < k; ++i) acc += ys[i] * tk.V[(long long)i * Nc + idx];
        tk.u[idx] = acc;
      }
    }
  }
}

// After the residual operator (mode 1 writes r into V[0] and the partials):
// beta = ||r||, convergence / floor / stagnation tests, normalise v_0.
__global__ void __launch_bounds__(kBlock) k_restart(const KryTask* __restrict__ tasks, int ntasks,
                                                     int initial, int max_cycles) {
  __shared__ int slot;
  __shared__ double red[4];
  const KryTask& tk = tasks[find_task(tasks, ntasks, &slot)];
  ProbState* st = tk.st;
  if (st->finished) return;
  const int b = blockIdx.x - tk.block_begin;
  const double r2 = sum_partials(tk.partials + 2 * tk.P, tk.P, red);
  const double x2 = sum_partials(tk.partials + 3 * tk.P, tk.P, red);
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
    done = true;
    reason = FDS_STOP_STAGNATION;
  }
  if (!done) {
    const double inv = 1.0 / beta;
    const long long base = (long long)b * kVecPerBlock;
#pragma unroll
    for (int e = 0; e < kVecEPT; ++e) {
      const long long idx = base + (long long)e * kBlock + threadIdx.x;
      if (idx < tk.Nc) tk.V[idx] *= inv;
    }
  }
  if (b == 0 && threadIdx.x == 0) {
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
    } else {
      st->cycle_done = 0;
      st->j_done = 0;
      tk.g[0] = beta;
    }
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
    if (MODE == 1) {
      tk.xuser[uidx] = tk.xint[rd.off + e];
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
    tk.out[rd.off + e] = v;
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
    double nb = 0.0;
    if (r > 0) nb += p[e - rd.cols];
    else if (rd.halo_off[0] >= 0) nb += tk.p[rd.halo_off[0] + c * rd.halo_stride[0]];
    if (r < rd.rows - 1) nb += p[e + rd.cols];
    else if (rd.halo_off[1] >= 0) nb += tk.p[rd.halo_off[1] + c * rd.halo_stride[1]];
    if (c > 0) nb += p[e - 1];
    else if (rd.halo_off[2] >= 0) nb += tk.p[rd.halo_off[2] + r * rd.halo_stride[2]];
    if (c < rd.cols - 1) nb += p[e + 1];
    else if (rd.halo_off[3] >= 0) nb += tk.p[rd.halo_off[3] + r * rd.halo_stride[3]];
    const double Ap = tk.delta * nb + (tk.kappa - 4.0 * tk.delta) * p[e];
    const double bv = tk.b[rd.off + e];
    const double res = bv - Ap;
    rr += res * res;
    bb += bv * bv;
  }
  const double s1 = block_sum(rr, red);
  const double s2 = block_sum(bb, red);
  if (threadIdx.x == 0) {
    tk.partials[b] = s1;
    tk.partials[tk.nblocks + b] = s2;
  }
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
// Dynamic LDS above 64 KiB must be opted into per kernel (gfx950 has 160 KiB
// per CU).
template <typename K>
static void ensure_smem(K kernel, size_t smem, size_t* granted) {
  if (smem <= 65536 || smem <= *granted) return;
  if (smem > 160 * 1024) throw Error(FDS_E_UNSUPPORTED, "transform too long for LDS");
  FDS_HIP(hipFuncSetAttribute(reinterpret_cast<const void*>(kernel),
                              hipFuncAttributeMaxDynamicSharedMemorySize, (int)smem));
  *granted = smem;
}

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
      hipLaunchKernelGGL((k_dst_rows<double, double, double>), dim3(nblocks), dim3(kBlock), smem, s,
                         tasks, ntasks, jidx);
      break;
    case DstKind::D_F:
      hipLaunchKernelGGL((k_dst_rows<float, double, float>), dim3(nblocks), dim3(kBlock), smem, s,
                         tasks, ntasks, jidx);
      break;
    case DstKind::F_F:
      hipLaunchKernelGGL((k_dst_rows<float, float, float>), dim3(nblocks), dim3(kBlock), smem, s,
                         tasks, ntasks, jidx);
      break;
    case DstKind::F_D:
      hipLaunchKernelGGL((k_dst_rows<float, float, double>), dim3(nblocks), dim3(kBlock), smem, s,
                         tasks, ntasks, jidx);
      break;
  }
}

void launch_tridiag(bool fp32, const TriTask* tasks, int ntasks, int nblocks, int jidx,
                    hipStream_t s) {
  if (nblocks <= 0) return;
  if (fp32)
    hipLaunchKernelGGL(k_tridiag<float>, dim3(nblocks), dim3(kBlock), 0, s, tasks, ntasks, jidx);
  else
    hipLaunchKernelGGL(k_tridiag<double>, dim3(nblocks), dim3(kBlock), 0, s, tasks, ntasks, jidx);
}

void launch_lines(const LineTask* tasks, int ntasks, size_t smem, int jidx, hipStream_t s) {
  if (ntasks <= 0) return;
  static size_t granted = 0;
  ensure_smem(k_schur_lines, smem, &granted);
  hipLaunchKernelGGL(k_schur_lines, dim3(ntasks), dim3(kBlock), smem, s, tasks, jidx);
}

void launch_operator(int mode, const OpTask* tasks, int ntasks, int nblocks, int jidx,
                     hipStream_t s) {
  if (nblocks <= 0) return;
  if (mode == 0)
    hipLaunchKernelGGL(k_operator<0>, dim3(nblocks), dim3(kBlock), 0, s, tasks, ntasks, jidx);
  else
    hipLaunchKernelGGL(k_operator<1>, dim3(nblocks), dim3(kBlock), 0, s, tasks, ntasks, jidx);
}

void launch_mgs_pass(const KryTask* tasks, int ntasks, int nblocks, int i, int j, hipStream_t s) {
  hipLaunchKernelGGL(k_mgs_pass, dim3(nblocks), dim3(kBlock), 0, s, tasks, ntasks, i, j);
}

void launch_mgs_finish(const KryTask* tasks, int ntasks, int nblocks, int j, hipStream_t s) {
  hipLaunchKernelGGL(k_mgs_finish, dim3(nblocks), dim3(kBlock), 0, s, tasks, ntasks, j);
}

void launch_ls_solve(const KryTask* tasks, int ntasks, hipStream_t s) {
  hipLaunchKernelGGL(k_ls_solve, dim3((ntasks + 63) / 64), dim3(64), 0, s, tasks, ntasks);
}

void launch_combine(bool flex, const KryTask* tasks, int ntasks, int nblocks, hipStream_t s) {
  if (flex)
    hipLaunchKernelGGL(k_combine<1>, dim3(nblocks), dim3(kBlock), 0, s, tasks, ntasks);
  else
    hipLaunchKernelGGL(k_combine<0>, dim3(nblocks), dim3(kBlock), 0, s, tasks, ntasks);
}

void launch_restart(const KryTask* tasks, int ntasks, int nblocks, int initial, int max_cycles,
                    hipStream_t s) {
  hipLaunchKernelGGL(k_restart, dim3(nblocks), dim3(kBlock), 0, s, tasks, ntasks, initial,
                     max_cycles);
}

void launch_lift(int mode, const LiftTask* tasks, int ntasks, int nblocks, hipStream_t s) {
  if (nblocks <= 0) return;
  if (mode == 0) hipLaunchKernelGGL(k_lift<0>, dim3(nblocks), dim3(kBlock), 0, s, tasks, ntasks);
  else hipLaunchKernelGGL(k_lift<1>, dim3(nblocks), dim3(kBlock), 0, s, tasks, ntasks);
}

void launch_iface(const IfaceTask* tasks, int ntasks, hipStream_t s) {
  if (ntasks <= 0) return;
  hipLaunchKernelGGL(k_iface, dim3(ntasks), dim3(kBlock), 0, s, tasks, ntasks);
}

void launch_residual(const ResTask* tasks, int ntasks, int nblocks, hipStream_t s) {
  if (nblocks <= 0) return;
  hipLaunchKernelGGL(k_residual, dim3(nblocks), dim3(kBlock), 0, s, tasks, ntasks);
}

void launch_count_active(const ProbState* st, int n, int* out, hipStream_t s) {
  hipLaunchKernelGGL(k_count_active, dim3(1), dim3(kBlock), 0, s, st, n, out);
}

}  // namespace fds
