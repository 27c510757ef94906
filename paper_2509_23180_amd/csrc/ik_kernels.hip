// Kernels of the interface Krylov iteration (see IkTask in fds_internal.h).
//
// Right-preconditioned GMRES on L_c p_c = f'_c (paper Section 2.4) with the
// basis kept in coordinates: the unit interior residual of the cycle plus
// orthonormal sine coefficients on the lines that carry an arm.  One Arnoldi
// step is three launches: the cross-axis sums of A_c^{-1} between x lines
// and y lines (k_ik_cross, whose last block also forms the corner values),
// then two passes over the coordinates in blocks of kIkSlab: w = v_j - S
// A_c^{-1} v_j with the dot products of modified Gram-Schmidt in its
// one-reduction form (k_ik_wdots), and the update with the norm and the
// Givens step (k_ik_update).  Stored basis vectors are not normalised in
// place: rscale[i] holds the factor of vector i.  The cycle start and end
// touch the whole centre: the interior residual is split from the lines
// (k_ik_extract), sine-transformed and solved per mode by the existing
// kernels, and k_ik_start turns the results into the first basis vector and
// S A_c^{-1} of the interior residual; at the end the update's coordinates
// (k_ik_combine) become sine coefficients along x (k_ik_compose) for the
// per-mode solve and the inverse transform into x.
#include "kernels.h"

#include <algorithm>

#include "fft_device.h"

namespace fds {

namespace {

constexpr int kIkWaves = kIkThreads / 64;

// Block sum over kIkThreads threads: wavefront sums (wave_sum, every lane
// gets its wavefront's sum), then the wavefronts in order.  `red` holds kIkWaves doubles; every thread gets the result.
__device__ __forceinline__ double ik_block_sum(double v, double* red) {
  v = wave_sum(v);
  const int w = threadIdx.x >> 6;
  __syncthreads();
  if ((threadIdx.x & 63) == 0) red[w] = v;
  __syncthreads();
  double s = 0.0;
#pragma unroll
  for (int i = 0; i < kIkWaves; ++i) s += red[i];
  return s;
}

// Line and position of coordinate e >= 1 (line -1 past the end).
__device__ __forceinline__ int ik_line_of(const IkTask& tk, int e, int* pos) {
  const int c = e - 1;
#pragma unroll
  for (int a = 0; a < 4; ++a) {
    const int o = tk.off[a];
    const int L = a < 2 ? tk.nx : tk.ny;
    if (o >= 0 && c >= o && c < o + L) {
      *pos = c - o;
      return a;
    }
  }
  *pos = 0;
  return -1;
}

__device__ __forceinline__ double sgn(int k) { return (k & 1) ? -1.0 : 1.0; }

// 1/d to full double precision: the hardware reciprocal estimate refined by
// two steps of Newton's iteration r <- r + r (1 - d r) (each step squares the
// relative error).  d is a sum of the operator's eigenvalues: finite,
// nonzero and far from the denormal range.
__device__ __forceinline__ double recip(double d) {
  double r = __builtin_amdgcn_rcp(d);
  double e = fma(-d, r, 1.0);
  r = fma(r, e, r);
  e = fma(-d, r, 1.0);
  return fma(r, e, r);
}

}  // namespace

// ---------------------------------------------------------------- cycle start

// Residual r (in u) -> its values on the owned line nodes (rline, y-line
// corners owned by an x line set to zero), u = r with those nodes zeroed
// (the interior part), and block sums of the interior part's squares.
__global__ void __launch_bounds__(kBlock) k_ik_extract(const IkTask* __restrict__ tasks, int ntasks) {
  __shared__ int slot;
  __shared__ double red[4];
  const IkTask& tk = tasks[find_task(tasks, ntasks, &slot)];
  if (tk.st->finished) return;
  const int b = blockIdx.x - tk.block_begin;
  const long long base = (long long)b * kVecPerBlock;
  const int nx = tk.nx, ny = tk.ny;
  const bool hasS = tk.off[0] >= 0, hasN = tk.off[1] >= 0;
  const bool hasW = tk.off[2] >= 0, hasE = tk.off[3] >= 0;
  double r2 = 0.0;
#pragma unroll
  for (int e = 0; e < kVecEPT; ++e) {
    const long long idx = base + (long long)e * kBlock + threadIdx.x;
    if (idx >= tk.Nc) continue;
    const int y = (int)(idx / nx);
    const int x = (int)(idx - (long long)y * nx);
    const double r = tk.u[idx];
    int a = -1, p = 0;
    if (y == 0 && hasS) { a = 0; p = x; }
    else if (y == ny - 1 && hasN) { a = 1; p = x; }
    else if (x == 0 && hasW) { a = 2; p = y; }
    else if (x == nx - 1 && hasE) { a = 3; p = y; }
    if (a < 0) {
      r2 += r * r;
      continue;
    }
    tk.rline[(long long)a * tk.lmax + p] = r;
    tk.u[idx] = 0.0;
    if (a < 2) {   // a corner owned by this x line: the y line's slot is empty
      if (x == 0 && hasW) tk.rline[(long long)2 * tk.lmax + y] = 0.0;
      if (x == nx - 1 && hasE) tk.rline[(long long)3 * tk.lmax + y] = 0.0;
    }
  }
  const double s = block_sum(r2, red);
  if (threadIdx.x == 0) tk.partials[b] = s;
}

// After the interior residual's sine transform, per-mode solve, boundary
// columns and line transforms: eta = ||r_int||, dhat = S A^{-1} r_int / eta,
// v_0 = (eta, line coefficients of r) / beta and g_0 = beta.  Two phases over
// the coordinates: the raw terms go to dhat while the corner sums (the W/E
// terms at the shared corners) and ||rho||^2 are reduced; then each thread
// re-reads its own entries, moves the corner values onto the S/N lines that
// own those corners, and writes v_0.
__global__ void __launch_bounds__(kIkThreads) k_ik_start(const IkTask* __restrict__ tasks, int ntasks) {
  __shared__ double red[5 * kIkWaves];
  const IkTask& tk = tasks[blockIdx.x];
  if (tk.st->finished) return;
  const int w = threadIdx.x >> 6;
  double e2 = 0.0;
  for (int b = threadIdx.x; b < tk.P; b += kIkThreads) e2 += tk.partials[b];
  const double eta2 = ik_block_sum(e2, red);
  const double eta = sqrt(eta2);
  const double inv_eta = eta > 0.0 ? 1.0 / eta : 0.0;
  const int nco = 1 + tk.nb;
  const int nx = tk.nx, ny = tk.ny;
  const bool hasS = tk.off[0] >= 0, hasN = tk.off[1] >= 0;
  const bool fix = (tk.off[2] >= 0 || tk.off[3] >= 0) && (hasS || hasN);
  // phase 1: raw terms, corner sums W . qy, W . sigma qy, E . qy, E . sigma qy
  double p0 = 0.0, p1 = 0.0, p2 = 0.0, p3 = 0.0, rr = 0.0;
  for (int e = 1 + (int)threadIdx.x; e < nco; e += kIkThreads) {
    int i = 0;
    const int a = ik_line_of(tk, e, &i);
    double ahat;
    if (a == 0) ahat = tk.tz[i];
    else if (a == 1) ahat = tk.tz[(long long)(ny - 1) * nx + i];
    else ahat = tk.zc[(a - 2) * ny + i];
    const double sh = tk.gd[a][i] * tk.gscale[a] * ahat * inv_eta;
    tk.dhat[e - 1] = sh;
    if (a >= 2) {
      const double v = sh * tk.qy[i];
      if (a == 2) { p0 += v; p1 += sgn(i) * v; }
      else { p2 += v; p3 += sgn(i) * v; }
    }
    const double rv = tk.rho[e - 1];
    rr += rv * rv;
  }
  p0 = wave_sum(p0); p1 = wave_sum(p1); p2 = wave_sum(p2); p3 = wave_sum(p3); rr = wave_sum(rr);
  __syncthreads();
  if ((threadIdx.x & 63) == 0) {
    red[w] = p0;
    red[kIkWaves + w] = p1;
    red[2 * kIkWaves + w] = p2;
    red[3 * kIkWaves + w] = p3;
    red[4 * kIkWaves + w] = rr;
  }
  __syncthreads();
  double c[5];
#pragma unroll
  for (int k = 0; k < 5; ++k) {
    double sum = 0.0;
    for (int q = 0; q < kIkWaves; ++q) sum += red[k * kIkWaves + q];
    c[k] = sum;
  }
  const double beta = sqrt(eta2 + c[4]);
  const double ib = beta > 0.0 ? 1.0 / beta : 0.0;
  const double w0 = hasS ? 1.0 : 0.0, w1 = hasN ? 1.0 : 0.0;
  // phase 2: corner correction and v_0 (every entry was written by this thread)
  for (int e = threadIdx.x; e < nco; e += kIkThreads) {
    if (e == 0) {
      tk.Vb[0] = eta * ib;
      continue;
    }
    tk.Vb[e] = tk.rho[e - 1] * ib;
    if (!fix) continue;
    int i = 0;
    const int a = ik_line_of(tk, e, &i);
    double sh = tk.dhat[e - 1];
    if (a >= 2) {
      const int b = (a - 2) * 2;
      sh -= w0 * c[b] * tk.qy[i] + w1 * c[b + 1] * sgn(i) * tk.qy[i];
    } else {
      const double qx = tk.qx[i];   // S takes the y = 0 corners (sums 0 / 2), N the y = ny-1 ones (1 / 3)
      sh += c[a] * qx + c[2 + a] * sgn(i) * qx;
    }
    tk.dhat[e - 1] = sh;
  }
  if (threadIdx.x == 0) {
    tk.g[0] = beta;
    tk.G[0] = 1.0;
    tk.rscale[0] = 1.0;
    tk.scal[0] = eta;
    tk.scal[1] = inv_eta;
    tk.scal[2] = beta;
  }
}

// ---------------------------------------------------------------- Arnoldi step

namespace {

// Schur term of coordinate (line a, position i) of step j before the corner
// correction: gd_a[i] (N/2) ((A^{-1} b)_a)_i with b = rs V_j: the same-axis
// diagonal terms plus the cross sums over the source ranges.
__device__ __forceinline__ double ik_raw_term(const IkTask& tk, const double* vj, double rs, int a, int i) {
  const long long lm = tk.lmax;
  auto ld = [](const double* p) { return *p; };
  double ahat, cross = 0.0;
  if (a < 2) {   // x line: same axis + sums from the y lines (direction y->x)
    const double bS = tk.off[0] >= 0 ? vj[1 + tk.off[0] + i] : 0.0;
    const double bN = tk.off[1] >= 0 ? vj[1 + tk.off[1] + i] : 0.0;
    ahat = (a == 0 ? tk.t00[i] * bS + tk.t0n[i] * bN : tk.t0n[i] * bS + tk.t00[i] * bN) * rs;
    if (tk.nya) {
      const double* py = tk.xpart + 4LL * kIkXParts * lm;
      const int k0 = a == 0 ? 0 : 2;
      double c0 = 0.0, c1 = 0.0;
#pragma unroll
      for (int p = 0; p < kIkXParts; ++p) {
        c0 += ld(py + ((long long)k0 * kIkXParts + p) * lm + i);
        c1 += ld(py + ((long long)(k0 + 1) * kIkXParts + p) * lm + i);
      }
      cross = tk.qx[i] * (c0 + sgn(i) * c1);
    }
  } else {       // y line: same axis + sums from the x lines (direction x->y)
    const double bW = tk.off[2] >= 0 ? vj[1 + tk.off[2] + i] : 0.0;
    const double bE = tk.off[3] >= 0 ? vj[1 + tk.off[3] + i] : 0.0;
    ahat = (a == 2 ? tk.s00[i] * bW + tk.s0n[i] * bE : tk.s0n[i] * bW + tk.s00[i] * bE) * rs;
    if (tk.nxa) {
      const double* px = tk.xpart;
      const int k0 = a == 2 ? 0 : 2;
      double c0 = 0.0, c1 = 0.0;
#pragma unroll
      for (int p = 0; p < kIkXParts; ++p) {
        c0 += ld(px + ((long long)k0 * kIkXParts + p) * lm + i);
        c1 += ld(px + ((long long)(k0 + 1) * kIkXParts + p) * lm + i);
      }
      cross = tk.qy[i] * (c0 + sgn(i) * c1);
    }
  }
  return tk.gd[a][i] * tk.gscale[a] * (ahat + cross);
}

// Corner correction of a raw term (c: the four corner values of the W/E
// terms, zero when one axis has no line).
__device__ __forceinline__ double ik_corner(const IkTask& tk, const double* c, int a, int i, double sh) {
  if (a >= 2) {
    const int b = (a - 2) * 2;
    const double w0 = tk.off[0] >= 0 ? 1.0 : 0.0, w1 = tk.off[1] >= 0 ? 1.0 : 0.0;
    return sh - (w0 * c[b] * tk.qy[i] + w1 * c[b + 1] * sgn(i) * tk.qy[i]);
  }
  return sh + c[a] * tk.qx[i] + c[2 + a] * sgn(i) * tk.qx[i];
}

}  // namespace

// Cross-axis sums of step j.  Direction x->y (sources on the S/N lines, x
// modes k; targets on the W/E lines, y modes l):
//   acc0[l] = sum_k R_lk qx_k b^S_k,          acc1[l] = sum_k R_lk qx_k b^N_k,
//   acc2[l] = sum_k R_lk (-1)^k qx_k b^S_k,   acc3[l] = sum_k R_lk (-1)^k qx_k b^N_k,
// R_lk = 1/(lamx_k + lamy_l + kappa), b = rscale_j V_j; direction y->x the
// same with the axes (and S/N, W/E) exchanged.  A block covers kIkXTile
// targets (one per lane) and one of kIkXParts source ranges; its
// wavefronts take the range's sources in turn (source s to wavefront s mod
// 8: one parity per wavefront, so the alternating sums follow from the
// per-wavefront sums), staged in LDS.  Blocks of direction x->y also form
// their shares of the corner values of the W/E lines' terms, which move to
// the S/N lines that own those corners.
__global__ void __launch_bounds__(kIkXThreads) k_ik_cross(const IkTask* __restrict__ tasks, int ntasks, int j) {
  constexpr int kW = kIkXThreads / 64;
  __shared__ int slot;
  __shared__ double lam_s[kIkXStage], w0[kIkXStage], w1[kIkXStage];
  __shared__ double red[2][kW][64];
  const IkTask& tk = tasks[find_task(tasks, ntasks, &slot)];
  if (tk.st->cycle_done) return;
  const double rs = tk.rscale[j];
  int b = blockIdx.x - tk.block_begin;
  const bool xy = b < tk.nxa;
  if (!xy) b -= tk.nxa;
  const int tile = b / kIkXParts, part = b - tile * kIkXParts;
  const int ns = xy ? tk.nx : tk.ny;
  const int nt = xy ? tk.ny : tk.nx;
  const double* lams = xy ? tk.lamx : tk.lamy;
  const double* lamt = xy ? tk.lamy : tk.lamx;
  const double* qs = xy ? tk.qx : tk.qy;
  const int oa = tk.off[xy ? 0 : 2], ob = tk.off[xy ? 1 : 3];
  const double* vj = tk.Vb + (long long)j * tk.ldv;
  const double* v = vj + 1;
  const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int t = tile * kIkXTile + lane;
  const bool live = t < nt;
  const double lt = live ? lamt[t] : 0.0;
  // this part's sources: an even start and length (a multiple of 8)
  const int Q = ((ns + kIkXParts - 1) / kIkXParts + 7) / 8 * 8;
  const int sa = part * Q, sb = min(ns, sa + Q);
  double a0 = 0.0, a1 = 0.0;
  for (int c0 = sa; c0 < sb; c0 += kIkXStage) {
    const int n = min(sb - c0, kIkXStage);
    __syncthreads();
    for (int s = threadIdx.x; s < n; s += kIkXThreads) {
      const int g = c0 + s;
      lam_s[s] = lams[g] + tk.kappa;
      w0[s] = oa >= 0 ? qs[g] * v[oa + g] * rs : 0.0;
      w1[s] = ob >= 0 ? qs[g] * v[ob + g] * rs : 0.0;
    }
    __syncthreads();
    if (live) {
      // c0 is even: source c0 + s has the parity of s, which is wv's
      for (int s = wv; s < n; s += kW) {
        const double r = recip(lt + lam_s[s]);
        a0 += r * w0[s];
        a1 += r * w1[s];
      }
    }
  }
  red[0][wv][lane] = a0;
  red[1][wv][lane] = a1;
  __syncthreads();
  if (wv != 0) return;
  double s0 = 0.0, s1 = 0.0, s2 = 0.0, s3 = 0.0;
  if (live) {
#pragma unroll
    for (int w = 0; w < kW; ++w) {
      const double x = red[0][w][lane], y = red[1][w][lane];
      s0 += x;
      s1 += y;
      s2 += (w & 1) ? -x : x;
      s3 += (w & 1) ? -y : y;
    }
    const long long lm = tk.lmax;
    double* out = tk.xpart + (xy ? 0LL : 4LL * kIkXParts * lm);
    out[(0LL * kIkXParts + part) * lm + t] = s0;
    out[(1LL * kIkXParts + part) * lm + t] = s1;
    out[(2LL * kIkXParts + part) * lm + t] = s2;
    out[(3LL * kIkXParts + part) * lm + t] = s3;
  }
  if (!xy) return;
  // This block's share of the four corner values of the W/E lines' terms
  // (their values at y = 0 and y = ny-1: <term, qy> and <term, sigma qy>),
  // which are linear in the cross sums: over its targets l, with the
  // same-axis terms added by the blocks of the first source range.  The
  // step kernels add the shares in block order.
  double p[4] = {0.0, 0.0, 0.0, 0.0};
  if (live) {
    const int l = t;
    const double q = tk.qy[l], sq = sgn(l) * q;
    const double bW = tk.off[2] >= 0 ? v[tk.off[2] + l] * rs : 0.0;
    const double bE = tk.off[3] >= 0 ? v[tk.off[3] + l] * rs : 0.0;
    if (tk.off[2] >= 0) {
      double term = q * (s0 + sgn(l) * s1);
      if (part == 0) term += tk.s00[l] * bW + tk.s0n[l] * bE;
      term *= tk.gd[2][l] * tk.gscale[2];
      p[0] = term * q;
      p[1] = term * sq;
    }
    if (tk.off[3] >= 0) {
      double term = q * (s2 + sgn(l) * s3);
      if (part == 0) term += tk.s0n[l] * bW + tk.s00[l] * bE;
      term *= tk.gd[3][l] * tk.gscale[3];
      p[2] = term * q;
      p[3] = term * sq;
    }
  }
#pragma unroll
  for (int k = 0; k < 4; ++k) p[k] = wave_sum(p[k]);
  if (lane == 0)
    for (int k = 0; k < 4; ++k) tk.cpart[(long long)b * 4 + k] = p[k];
}

// Step j, first pass over the coordinates (kIkSlab per block): w = b_j -
// c0 dhat - S A^{-1} b_j with b_j = rscale_j V_j (stored in Wv), and the
// block's parts of <w, V_i> and <V_j, V_i> (i <= j).  The problem's last block sums the parts in block
// order, scales them to the normalised basis, stores the Gram column j and
// runs the MGS recurrence h_i = <w, v_i> - sum_{l<i} h_l <v_l, v_i> (one-
// reduction form of modified Gram-Schmidt) into hv.
__global__ void __launch_bounds__(kBlock) k_ik_wdots(const IkTask* __restrict__ tasks, int ntasks, int j) {
  constexpr int kW = kBlock / 64;
  __shared__ int slot;
  __shared__ int lastf;
  __shared__ double gred[4][kW];
  __shared__ double ws[kIkSlab], vs[kIkSlab];
  __shared__ double av[122], gv[122];
  __shared__ double cv[4];
  extern __shared__ __align__(16) double gt[];   // strict upper triangle of G, column i at i (i - 1) / 2
  const IkTask& tk = tasks[find_task(tasks, ntasks, &slot)];
  ProbState* st = tk.st;
  if (st->cycle_done) return;
  const int b = blockIdx.x - tk.block_begin;
  const int nco = 1 + tk.nb;
  const int m1 = tk.m + 1;
  const double rs = tk.rscale[j];
  const double* vj = tk.Vb + (long long)j * tk.ldv;
  const double c0 = rs * vj[0];
  // corner values: the shares of the x->y cross blocks, summed by a fixed
  // tree (thread t takes shares t/4, t/4 + 64, ... of corner t % 4; lanes of
  // one corner are then combined by shuffles, the wavefronts in order)
  {
    const int cc = threadIdx.x & 3;
    double v = 0.0;
    for (int k = threadIdx.x >> 2; k < tk.nxa; k += kBlock / 4) v += tk.cpart[(long long)k * 4 + cc];
#pragma unroll
    for (int o = 4; o < 64; o <<= 1) v += __shfl_xor(v, o, 64);
    if ((threadIdx.x & 63) < 4) gred[cc][threadIdx.x >> 6] = v;
    __syncthreads();
    if (threadIdx.x < 4) {
      double sum = 0.0;
      for (int w = 0; w < kW; ++w) sum += gred[threadIdx.x][w];
      cv[threadIdx.x] = sum;
    }
    __syncthreads();
  }
  double c[4];
  for (int k = 0; k < 4; ++k) c[k] = cv[k];
  // w and v_j of the slab (one coordinate per thread) into LDS
  {
    const int e = b * kIkSlab + (int)threadIdx.x;
    double wq = 0.0, vq = 0.0;
    if (e < nco) {
      vq = vj[e];
      if (e == 0) {
        wq = c0;
      } else {
        int i = 0;
        const int a = ik_line_of(tk, e, &i);
        const double sh = ik_corner(tk, c, a, i, ik_raw_term(tk, vj, rs, a, i));
        wq = rs * vq - c0 * tk.dhat[e - 1] - sh;
      }
      tk.Wv[e] = wq;
    }
    ws[threadIdx.x] = wq;
    vs[threadIdx.x] = vq;
  }
  __syncthreads();
  // dots: wavefront wv takes basis vectors i = wv, wv + kW, ... over the whole
  // slab (lane l: coordinates l, l + 64, ...), kIkDotChunk of them with their
  // loads in flight together; each sum ends in lane 63, which stores it
  {
    constexpr int R = kIkSlab / 64;
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    double wl[R], vl[R];
#pragma unroll
    for (int r = 0; r < R; ++r) {
      wl[r] = ws[lane + 64 * r];
      vl[r] = vs[lane + 64 * r];
    }
    const int e0 = b * kIkSlab + lane;
    for (int i0 = wv; i0 <= j; i0 += kW * kIkDotChunk) {
      double x[kIkDotChunk][R];
#pragma unroll
      for (int q = 0; q < kIkDotChunk; ++q) {
        const int i = i0 + q * kW;
#pragma unroll
        for (int r = 0; r < R; ++r) {
          const int e = e0 + 64 * r;
          x[q][r] = (i <= j && e < nco) ? tk.Vb[(long long)i * tk.ldv + e] : 0.0;
        }
      }
#pragma unroll
      for (int q = 0; q < kIkDotChunk; ++q) {
        const int i = i0 + q * kW;
        double pa = 0.0, pg = 0.0;
#pragma unroll
        for (int r = 0; r < R; ++r) {
          pa += wl[r] * x[q][r];
          pg += vl[r] * x[q][r];
        }
        pa = wave_sum_last(pa);
        pg = wave_sum_last(pg);
        if (lane == 63 && i <= j) {
          st_agent(tk.dpart + (long long)i * tk.nslab + b, pa);
          st_agent(tk.dpart + (long long)(m1 + i) * tk.nslab + b, pg);
        }
      }
    }
  }
  if (!last_block_of_problem(&st->ctr_dots, tk.nslab, &lastf)) return;
  for (int t = threadIdx.x; t < 2 * (j + 1); t += kBlock) {
    const int i = t <= j ? t : t - (j + 1);
    const int row = t <= j ? i : m1 + i;
    // all parts loaded before any is added (they arrive together)
    double part[kIkMaxSlabs];
#pragma unroll
    for (int k = 0; k < kIkMaxSlabs; ++k)
      part[k] = k < tk.nslab ? ld_agent(tk.dpart + (long long)row * tk.nslab + k) : 0.0;
    double sum = 0.0;
#pragma unroll
    for (int k = 0; k < kIkMaxSlabs; ++k) sum += part[k];
    if (t <= j) av[i] = sum * tk.rscale[i];
    else gv[i] = sum * tk.rscale[i] * rs;
  }
  // the earlier Gram columns (G_li, l < i < j) into LDS, column j from gv
  const int ntri = j * (j + 1) / 2;
  for (int e = threadIdx.x; e < ntri; e += kBlock) {
    int i = (int)((1.0 + sqrt(1.0 + 8.0 * e)) * 0.5);
    while (i * (i - 1) / 2 > e) --i;
    while ((i + 1) * i / 2 <= e) ++i;
    const int l = e - i * (i - 1) / 2;
    gt[e] = i < j ? tk.G[l + (long long)i * m1] : 0.0;
  }
  __syncthreads();
  for (int l = threadIdx.x; l < j; l += kBlock) {
    tk.G[l + (long long)j * m1] = gv[l];
    gt[j * (j - 1) / 2 + l] = gv[l];
  }
  __syncthreads();
  // h = L^{-1} a with L unit lower triangular (L_il = G_li, l < i): one
  // wavefront, rows i = lane and lane + 64 (j < 128); each step broadcasts
  // the finished h_l and updates the later rows, with the Gram entries of 16
  // steps read from LDS ahead of their use
  if (threadIdx.x < 64) {
    const int i0 = threadIdx.x, i1 = threadIdx.x + 64;
    double a0 = i0 <= j ? av[i0] : 0.0, a1 = i1 <= j ? av[i1] : 0.0;
    const int b0 = i0 * (i0 - 1) / 2, b1 = i1 * (i1 - 1) / 2;
    for (int l0 = 0; l0 < j; l0 += 16) {
      double g0[16], g1[16];
#pragma unroll
      for (int u = 0; u < 16; ++u) {
        const int l = l0 + u;
        g0[u] = (l < i0 && i0 <= j) ? gt[b0 + l] : 0.0;
        g1[u] = (l < i1 && i1 <= j) ? gt[b1 + l] : 0.0;
      }
#pragma unroll
      for (int u = 0; u < 16; ++u) {
        const int l = l0 + u;
        if (l < j) {
          const double hl = l < 64 ? __shfl(a0, l, 64) : __shfl(a1, l - 64, 64);
          a0 -= hl * g0[u];
          a1 -= hl * g1[u];
        }
      }
    }
    if (i0 <= j) tk.hv[i0] = a0;
    if (i1 <= j) tk.hv[i1] = a1;
  }
}

// Step j, second pass: V_{j+1} = w - sum_i h_i rscale_i V_i (stored
// unnormalised) with the block's part of ||V_{j+1}||^2; the problem's last
// block forms h_{j+1,j}, the normalising factor rscale_{j+1}, the Givens
// update of column j and the convergence test.
__global__ void __launch_bounds__(kBlock) k_ik_update(const IkTask* __restrict__ tasks, int ntasks, int j,
                                                       int* flags, int tag) {
  __shared__ int slot;
  __shared__ int lastf;
  __shared__ double hs[122 + kIkUpdChunk];
  __shared__ double col[122], cs[121], sn[121];
  __shared__ double red[4];
  const IkTask& tk = tasks[find_task(tasks, ntasks, &slot)];
  ProbState* st = tk.st;
  if (st->cycle_done) return;
  const int b = blockIdx.x - tk.block_begin;
  const int nco = 1 + tk.nb;
  const int m1 = tk.m + 1;
  // the step's coefficients and the earlier rotations (read by every block,
  // so the finishing block has them at hand)
  for (int i = threadIdx.x; i <= j; i += kBlock) {
    col[i] = tk.hv[i];
    hs[i] = col[i] * tk.rscale[i];
  }
  for (int i = j + 1 + (int)threadIdx.x; i < 122 + kIkUpdChunk; i += kBlock) hs[i] = 0.0;
  for (int i = threadIdx.x; i < j; i += kBlock) {
    cs[i] = tk.cs[i];
    sn[i] = tk.sn[i];
  }
  __syncthreads();
  double* vn = tk.Vb + (long long)(j + 1) * tk.ldv;
  // one coordinate per thread; the loads of kIkUpdChunk basis vectors are in
  // flight together (hs is zero past j)
  double nn = 0.0;
  {
    const int e = b * kIkSlab + (int)threadIdx.x;
    if (e < nco) {
      double x = tk.Wv[e];
      for (int i0 = 0; i0 <= j; i0 += kIkUpdChunk) {
        double xv[kIkUpdChunk];
#pragma unroll
        for (int g = 0; g < kIkUpdChunk; ++g)
          xv[g] = i0 + g <= j ? tk.Vb[(long long)(i0 + g) * tk.ldv + e] : 0.0;
#pragma unroll
        for (int g = 0; g < kIkUpdChunk; ++g) x -= hs[i0 + g] * xv[g];
      }
      vn[e] = x;
      nn = x * x;
    }
  }
  const double s = block_sum(nn, red);
  if (threadIdx.x == 0) st_agent(tk.dpart + (long long)2 * m1 * tk.nslab + b, s);
  if (!last_block_of_problem(&st->ctr_upd, tk.nslab, &lastf)) return;
  if (threadIdx.x != 0) return;
  double part[kIkMaxSlabs];
#pragma unroll
  for (int k = 0; k < kIkMaxSlabs; ++k)
    part[k] = k < tk.nslab ? ld_agent(tk.dpart + (long long)2 * m1 * tk.nslab + k) : 0.0;
  double n2 = 0.0;
#pragma unroll
  for (int k = 0; k < kIkMaxSlabs; ++k) n2 += part[k];
  const double hn = sqrt(n2);
  const bool breakdown = !(hn > 1e-14 * st->beta);
  tk.rscale[j + 1] = breakdown ? 1.0 : 1.0 / hn;
  st->last_hn = hn;
  // Givens update of column j (in LDS): the previous rotations, then a new one
  col[j + 1] = hn;
  for (int i = 0; i < j; ++i) {
    const double a = col[i], c2 = col[i + 1];
    col[i] = cs[i] * a + sn[i] * c2;
    col[i + 1] = -sn[i] * a + cs[i] * c2;
  }
  const double a = col[j];
  const double rho = hypot(a, hn);
  double c = 1.0, s1 = 0.0;
  if (rho > 0.0) {
    c = a / rho;
    s1 = hn / rho;
  }
  tk.cs[j] = c;
  tk.sn[j] = s1;
  col[j] = rho;
  col[j + 1] = 0.0;
  for (int i = 0; i <= j + 1; ++i) tk.H[i + (long long)j * m1] = col[i];
  const double gj = tk.g[j];
  tk.g[j + 1] = -s1 * gj;
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

// ---------------------------------------------------------------- cycle end

// Coordinates of the update V y (k = steps of the cycle) and the factor of
// the interior residual's sine coefficients in it (scal[4] = u_0 / eta).
__global__ void __launch_bounds__(kIkThreads) k_ik_combine(const IkTask* __restrict__ tasks, int ntasks) {
  __shared__ double ys[128];
  const IkTask& tk = tasks[blockIdx.x];
  if (tk.st->finished) return;
  const int k = tk.st->j_done;
  for (int i = threadIdx.x; i < k; i += kIkThreads) ys[i] = tk.y[i] * tk.rscale[i];
  __syncthreads();
  const int nco = 1 + tk.nb;
  for (int e = threadIdx.x; e < nco; e += kIkThreads) {
    double acc = 0.0;
    for (int i = 0; i < k; ++i) acc += ys[i] * tk.Vb[(long long)i * tk.ldv + e];
    tk.ucoef[e] = acc;
    if (e == 0) tk.scal[4] = acc * tk.scal[1];
  }
}

// Sine coefficients along x of the update: scal[4] V0 plus the S/N line
// coefficients on rows 0 / ny-1 plus the W/E lines' physical values times the
// sine vectors' first / last node values; written to tz for the per-mode
// solve and the inverse transform.
__global__ void __launch_bounds__(kBlock) k_ik_compose(const IkTask* __restrict__ tasks, int ntasks) {
  __shared__ int slot;
  const IkTask& tk = tasks[find_task(tasks, ntasks, &slot)];
  if (tk.st->finished) return;
  const int b = blockIdx.x - tk.block_begin;
  const long long base = (long long)b * kVecPerBlock;
  const int nx = tk.nx, ny = tk.ny;
  const double s0 = tk.scal[4];
  const double* us = tk.off[0] >= 0 ? tk.ucoef + 1 + tk.off[0] : nullptr;
  const double* un = tk.off[1] >= 0 ? tk.ucoef + 1 + tk.off[1] : nullptr;
  const double* pw = tk.off[2] >= 0 ? tk.uphys : nullptr;
  const double* pe = tk.off[3] >= 0 ? tk.uphys + ny : nullptr;
#pragma unroll
  for (int e = 0; e < kVecEPT; ++e) {
    const long long idx = base + (long long)e * kBlock + threadIdx.x;
    if (idx >= tk.Nc) continue;
    const int y = (int)(idx / nx);
    const int k = (int)(idx - (long long)y * nx);
    double v = s0 * tk.V0[idx];
    if (y == 0 && us) v += us[k];
    if (y == ny - 1 && un) v += un[k];
    const double qk = tk.qx[k];
    if (pw) v += qk * pw[y];
    if (pe) v += sgn(k) * qk * pe[y];
    tk.tz[idx] = v;
  }
}

// ---------------------------------------------------------------- launchers

void launch_ik_extract(const IkTask* tasks, int ntasks, int nblocks, hipStream_t s) {
  if (nblocks <= 0) return;
  FDS_LAUNCH(k_ik_extract, dim3(nblocks), dim3(kBlock), 0, s, tasks, ntasks);
}

void launch_ik_start(const IkTask* tasks, int ntasks, int max_coords, hipStream_t s) {
  if (ntasks <= 0) return;
  if (max_coords > kIkMaxCoords)
    throw Error(FDS_E_INVALID_ARG, "interface Krylov vector longer than the step kernels hold");
  FDS_LAUNCH(k_ik_start, dim3(ntasks), dim3(kIkThreads), 0, s, tasks, ntasks);
}

void launch_ik_cross(const IkTask* tasks, int ntasks, int nblocks, int j, hipStream_t s) {
  if (nblocks <= 0) return;
  FDS_LAUNCH(k_ik_cross, dim3(nblocks), dim3(kIkXThreads), 0, s, tasks, ntasks, j);
}

void launch_ik_wdots(const IkTask* tasks, int ntasks, int nblocks, int j, hipStream_t s) {
  if (nblocks <= 0) return;
  const size_t smem = sizeof(double) * std::max<size_t>(1, (size_t)j * (j + 1) / 2);
  static size_t granted = 0;
  ensure_smem(k_ik_wdots, smem + 8192, &granted);
  FDS_LAUNCH(k_ik_wdots, dim3(nblocks), dim3(kBlock), smem, s, tasks, ntasks, j);
}

void launch_ik_update(const IkTask* tasks, int ntasks, int nblocks, int j, int* flags, int tag,
                      hipStream_t s) {
  if (nblocks <= 0) return;
  FDS_LAUNCH(k_ik_update, dim3(nblocks), dim3(kBlock), 0, s, tasks, ntasks, j, flags, tag);
}

void launch_ik_combine(const IkTask* tasks, int ntasks, hipStream_t s) {
  if (ntasks <= 0) return;
  FDS_LAUNCH(k_ik_combine, dim3(ntasks), dim3(kIkThreads), 0, s, tasks, ntasks);
}

void launch_ik_compose(const IkTask* tasks, int ntasks, int nblocks, hipStream_t s) {
  if (nblocks <= 0) return;
  FDS_LAUNCH(k_ik_compose, dim3(nblocks), dim3(kBlock), 0, s, tasks, ntasks);
}

}  // namespace fds
