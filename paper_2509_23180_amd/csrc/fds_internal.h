// Internal types shared by the host runtime and the HIP kernels.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <stdexcept>
#include <string>

#include "../../include/fds.h"

namespace fds {

constexpr int kMaxPass = 24;     // radix passes of one FFT plan
constexpr int kBlock = 256;      // threads per block for most kernels
constexpr int kMaxArms = 4;
constexpr int kMaxRects = 64;     // rectangles per plan (a chain and its two end arms)
#if defined(FDS_VEC_EPT)
constexpr int kVecEPT = FDS_VEC_EPT;   // (development builds: block size A/B)
#else
constexpr int kVecEPT = 8;       // centre-vector elements per thread in reduction kernels
#endif
constexpr int kVecPerBlock = kBlock * kVecEPT;

// ---------------------------------------------------------------- errors
struct Error : std::runtime_error {
  fds_status status;
  Error(fds_status s, const std::string& m) : std::runtime_error(m), status(s) {}
};

#define FDS_HIP(call)                                                                  \
  do {                                                                                 \
    hipError_t e_ = (call);                                                            \
    if (e_ != hipSuccess)                                                              \
      throw ::fds::Error(e_ == hipErrorOutOfMemory ? FDS_E_NOMEM : FDS_E_DEVICE,       \
                         std::string(#call) + ": " + hipGetErrorString(e_));           \
  } while (0)

// ---------------------------------------------------------------- timing
// Per-class kernel timing.  Between begin(cls) and end(cls) every kernel
// launch records its own start/stop events through the dispatch packet
// (hipExtLaunchKernel), so timing adds no packets to the stream.
struct Timing {
  static void enable(int mask);
  static bool on();
  static bool on(int cls);
  static void add_bytes(int cls, double bytes);
  static double bytes(int cls);
  static void begin(int cls, hipStream_t s);
  static void end(int cls, hipStream_t s);
  // events for the next launch when a class is being timed
  static bool take_pair(hipEvent_t* start, hipEvent_t* stop);
  static void read(int cls, long long* calls, double* ms);
  static void reset();
};

// ---------------------------------------------------------------- FFT plan
// Complex FFT of length N = n + 1 used to evaluate the DST-I of length n.
//   kind 0 (mixed radix): Stockham passes over N.
//   kind 1 (Rader, N prime): the N-1 outputs k != 0 form a cyclic
//          convolution of length L = N-1 evaluated with two inner FFTs.
//   kind 2 (Bluestein): chirp-z, a cyclic convolution of power-of-two
//          length L >= 2N-1 evaluated with two inner FFTs.
// `radix`, `tw*` describe the inner (kind 1, 2) or the full (kind 0) FFT.
enum FftKind { FFT_MIXED = 0, FFT_RADER = 1, FFT_BLUESTEIN = 2 };

struct FftDesc {
  int N;
  int kind;
  int L;                  // length of the Stockham FFT actually run
  int W;                  // LDS entries per buffer: max(N, L)
  int npass;
  int radix[kMaxPass];
  const double2* tw64;    // L entries  exp(-2 pi i t / L)
  const float2* tw32;
  const double2* post64;  // N+1 entries (cos(pi k / N), sin(pi k / N))
  const float2* post32;
  const int* perm_in;     // Rader: g^{-q} mod N, q < L
  const int* perm_out;    // Rader: g^{q} mod N, q < L
  const double2* kern64;  // Rader / Bluestein: FFT_L(kernel) / L
  const float2* kern32;
  const double2* chirp64; // Bluestein: exp(-i pi t^2 / N), t < N
  const float2* chirp32;
  // dense sine matrix for the matrix-core variant (n <= kGemmMaxN), padded
  // with zeros to np x np, np a multiple of 64; NULL when not built
  int np;
  int pad1;
  const double* smat64;
  const float* smat32;
};

constexpr int kGemmMaxN = 1024;

// ---------------------------------------------------------------- wave DST
// LDS layout of the wave-parallel row transform: the workgroup's copy of the
// tables (twiddles, post-processing, convolution kernel, chirp, Rader
// permutations) followed by one padded buffer per row.  The same layout is
// used for the table image in device memory, so staging is one plain copy.
// Padded LDS index: one spare entry per 256 bytes keeps the strided accesses
// of the early passes spread over the banks.
template <typename T> __host__ __device__ __forceinline__ int wpad(int i) {
  return i + (i >> (sizeof(T) == 8 ? 4 : 5));
}

// Byte offsets of the per-workgroup tables and of the row buffers.  The
// twiddles are stored per pass: pass p (radix R, Ns = product of the earlier
// radices) holds w^{r k L/(Ns R)} at (r-1) Ns + k, k < Ns, 1 <= r < R, so
// the lanes of a pass read consecutive entries.
struct WaveLayout {
  int tw, post, kern, chirp, pin, pout, rows, row_bytes;
};

template <typename T>
__host__ __device__ __forceinline__ WaveLayout wave_layout(int kind, int N, int L, int W, int twlen) {
  const int cb = (int)sizeof(T) * 2;
  WaveLayout w;
  w.tw = 0;
  w.post = w.tw + twlen * cb;
  w.kern = w.post + (N + 1) * cb;
  w.chirp = w.kern + (kind != FFT_MIXED ? L : 0) * cb;
  w.pin = w.chirp + (kind == FFT_BLUESTEIN ? N : 0) * cb;
  w.pout = w.pin + (kind == FFT_RADER ? L : 0) * 4;
  w.rows = (w.pout + (kind == FFT_RADER ? L : 0) * 4 + 15) / 16 * 16;
  w.row_bytes = ((wpad<T>(W - 1) + 1) * cb + 15) / 16 * 16;
  return w;
}

// Everything the wave-parallel transform needs about its length, carried in
// the task record itself (no dependent load through FftDesc).
struct WaveDesc {
  int N, L, W, kind, npass, twlen;
  int img_chunks;           // 16-byte chunks of `img`
  int pad;
  const uint4* img;         // table image in the LDS layout, task precision
  unsigned long long radices;  // radix of pass p in bits [5p, 5p+5) (at most 12 passes)
};

// Per-mode coefficients of the constant-coefficient tridiagonal solve
//   delta y[i-1] + a y[i] + delta y[i+1] = s r[i],  a = -delta (q + 1/q),
// written as -(delta/q) (L U + q^2 e1 e1^T) y = s r with L = I - qZ,
// U = I - qZ^T (Sherman-Morrison correction of the first row).
template <typename T>
struct ModeCoef {
  T q;      // exp(-theta), cosh(theta) = -a/(2 delta)
  T qinv;   // 1/q
  T sc;     // -(q/delta) * s   (s = the DST normalisation 2/(n+1))
  T beta;   // q^2 / (1 + q^2 (1 - q^{2m})/(1 - q^2))
  T qK;     // q^K
  int K;    // largest exponent kept before q^K would underflow (<= m-1)
};

// ---------------------------------------------------------------- problem state
struct ProbState {
  int cycle_done;   // remaining Arnoldi steps of this cycle are skipped
  int finished;     // everything is skipped
  int j_done;       // Arnoldi steps completed in the current cycle
  int stop_reason;  // fds_stop_reason
  int iterations;
  int cycles;
  int nonfinite;
  int ctr_dots;     // blocks of the current Gram-dot launch that finished
  int ctr_upd;      // blocks of the current update launch that finished
  int ctr_aux;      // blocks of the current interface-iteration cross-sum launch that finished
  double beta;      // true residual norm at the start of the current cycle
  double fnorm;     // ||f'_c||_2
  double tol;
  double tol_eff;
  double prev_rel;
  double xnorm;
  double floor_coef;   // unit roundoff times a bound of ||L_c||_inf
  double last_hn;      // h_{j+1,j} of the latest Arnoldi step
  double vscale;       // factor that normalises the newest basis vector V[j]
  double rscale;     // restart: scale of the new V[0] (0 when the problem stopped)
  double res_rr;     // composite residual: sum of r^2 and of b^2 (after the solve)
  double res_bb;
};

// ---------------------------------------------------------------- task records
// One record per independent piece of work; blocks map to records through
// block_begin (sorted ascending).
struct DstTask {
  const void* in;
  void* out;
  long long in_rs, out_rs;    // row strides (elements)
  long long in_js, out_js;    // added once per Krylov index j
  long long in_cs, out_cs;    // element stride along a row
  int rows, n;
  int rpb;                    // rows per block
  int accumulate;             // out += result
  int tw_lds;                 // 1: stage the twiddles in LDS ahead of the row buffers
  int io_f32;                 // wave kernel: bit 0 input FP32, bit 1 output FP32
  double scale;
  const FftDesc* fft;
  const int* skip;            // skip when *skip != 0
  const double* in_scale;     // if set: input *= *in_scale, written back in place
  int block_begin;
  int pad;
  WaveDesc wd;                // wave-parallel kernel only
};

struct TriTask {
  void* data;
  long long rs, js;
  int rows, modes;
  const void* coef;           // ModeCoef<T>[modes]
  const int* skip;
  int block_begin;
  int pad;
  // Optional source: the right-hand side is read from vin (FP64, layout of
  // data, step stride vjs) times *vscale, and vin is written back scaled
  // (the Krylov basis vector is normalised in the same pass); the solution
  // goes to data.
  double* vin;
  long long vjs;
  const double* vscale;
  int identity;               // 1: no solve, data = the scaled right-hand side (P = I)
  int pad_t;
};

// Schur line term: out[k] = sum_l Sline(k,l) z_line[l] with
// Sline = delta^2 (2/N) S diag(g) S on one boundary line of the centre.
struct LineTask {
  const void* z;              // centre vector (FP64, or FP32 if z_f32)
  long long z_js;
  long long start;            // first element of the line
  long long stride;           // element stride along the line
  int L;
  int z_f32;
  int pad_l;
  int pad;
  const FftDesc* fft;
  const double* gs;           // delta^2 (2/N) g_k, k = 1..L
  double* out;                // L doubles
  const int* skip;
  const double* mat;          // dense operator (element (k, i) at k L + i), or null
  int block_begin;
  int pad2;
};

// Centre operator w = A_c z - sum_a S_ca z  (mode 0), or the residual
// r = f' - L_c z with partial sums of r^2 and z^2 (mode 1).
struct OpTask {
  const void* z;
  long long z_js;
  int z_f32;
  int nx, ny;
  int nblocks;
  double* out;
  long long out_js;
  const double* fp;
  const double* line[4];      // S (row 0), N (row ny-1), W (col 0), E (col nx-1); NULL if none
  double delta, kappa;
  double* partials;           // mode 1: [2 * nblocks]
  const int* skip;
  int block_begin;
  int pad;
};

// Krylov bookkeeping of one problem.
struct KryTask {
  double* V;                  // (m+1) x Nc
  float* Z;                   // m x Nc (flexible variant) or NULL
  double* x;                  // centre solution (Nc)
  double* u;                  // scratch centre vector (Nc)
  double* H;                  // (m+1) x m, column-major (H[i + j (m+1)])
  double* cs;
  double* sn;
  double* g;                  // m+1
  double* y;                  // m
  double* partials;           // (2(m+1) + 4) x P block partials, see kPart*
  double* G;                  // (m+1) x (m+1) Gram matrix <v_i, v_j>, column-major
  double* hv;                 // m+1 Gram-Schmidt coefficients of the current step
  ProbState* st;
  long long Nc;
  int P;                      // blocks covering Nc
  int m;
  int nx, ny;
  int implicit_w;             // 1: w = v_j - s (exact preconditioner), 0: w stored in V[j+1]
  int block_begin;
  const double* line[4];      // Schur line terms s on the centre's boundary lines (or NULL)
  int flag_idx;               // slot of this problem in the host-visible flag array
  int gram_lag;               // 1: Gram columns come from the update pass (see kLagMaxJ)
  // Plain variant in the centre's orthonormal sine basis: the Schur term of
  // w = v_j - Q s (see qs_term) takes the S/N blocks as per-mode scalings of
  // the solve's sine coefficients z^ (rows 0 and ny-1) and the W/E line
  // terms line[2] / line[3] as rank-one terms per row; line[0] / line[1] are
  // then NULL.  bc holds the physical values of every basis vector on
  // columns 0 and nx-1 (vector i at bc + 2 ny i, W then E) for <v_i, s>.
  const double* gs[2];        // delta^2 (2/N) g_k of the S / N arm, or NULL
  const double* zhat;         // z^ (ny x nx)
  const double2* post;        // (cos, sin)(pi k / N), k = 0..N
  double* bc;
  double qscale;              // sqrt(2/N)
  double half_n;              // N/2
  // Flexible variant: the dot pass forms w = Q L_c Q^T z^_j itself (see
  // spec_w; gs, line[2..3], post, qscale, half_n as above) and stores it in
  // V[j+1].
  int fuse_op;
  int pad_f;
  double delta, kappa;
};

// Lagged Gram columns (exact preconditioner, restart length <= kLagMaxJ):
// the update pass of step j also forms <v_i, v_{j+1}> from the values it
// holds, so the dot pass of step j+1 reduces to <v_i, s> over the boundary
// lines where the Schur terms s live.
constexpr int kLagMaxJ = 32;

// partial-sum slots (each P wide) inside KryTask::partials
constexpr int kPartRes = 0;   // residual r^2 (P) and x^2 (P)
constexpr int kPartNorm = 2;  // ||w||^2
constexpr int kPartDots = 3;  // 2(m+1) dot products
// Behind the 2(m+1)+4 slots: the Gram reduction's first level, 2(m+1) rows of
// ng group sums (one per kGramGroup blocks), then ng int group counters.
constexpr int kGramGroup = 16;
// (one level, ng = 1, up to 64 blocks: the partials are summed directly)
__host__ __device__ inline int gram_groups(int P) { return P <= 64 ? 1 : (P + kGramGroup - 1) / kGramGroup; }
__host__ __device__ inline size_t kry_partials_len(int m, int P) {
  const size_t ng = (size_t)gram_groups(P);
  return (size_t)(2 * (m + 1) + 4) * P + (size_t)2 * (m + 1) * ng + ng;
}

// Rectangle of a problem in the library's internal layout: rows x cols with
// the sine-transform axis (cols) contiguous.  Global node of element (r, c):
//   i = ai + ar r + ac c,  j = aj + br r + bc c.
struct RectDev {
  int rows, cols;
  long long off;              // into the internal vectors
  long long ld;               // internal row stride (cols, or the width of the
                              // merged coupled block the rectangle is part of)
  long long user_off;         // into the user unknown vector
  long long bc_off;           // into the user Dirichlet-data vector
  int ai, ar, ac, aj, br, bcc;
  int ilo, jlo, uwidth;       // user block origin (global node) and width
  int bi0, bj0, bi1, bj1;     // closed box
  int iface_mask;             // box sides whose interior nodes are unknowns:
                              // 1: i=bi0, 2: i=bi1, 4: j=bj0, 8: j=bj1
  // neighbour lines across internal sides: 0: r=-1, 1: r=rows, 2: c=-1, 3: c=cols
  long long halo_off[4];      // -1 if Dirichlet
  long long halo_stride[4];
};

// Boundary columns of z = S y for every row of the sine coefficients y:
// z[r][0] = sum_k y[r][k] sin(pi k/N), z[r][nx-1] = sum_k y[r][k] (-1)^{k+1} sin(pi k/N).
struct ColTask {
  const double* y;
  double* zw;                 // column 0 (ny values) or NULL
  double* ze;                 // column nx-1 or NULL
  const FftDesc* fft;
  int nx, ny;
  const int* skip;
  int block_begin;
  int pad;
  const float* y32;           // FP32 coefficients (used instead of y when set)
  long long y_js;             // y32 stride per Arnoldi step
  double scale;               // factor on the sums (1: z = S y)
  const double* v;            // also: basis vector v_j (step stride Nc) ...
  double* bc;                 // ... whose boundary columns go to bc + 2 ny j (W, E), or NULL
  long long Nc;
};

struct LiftTask {
  RectDev rd;
  const double* rhs;          // user unknown vector
  const double* bc;           // user Dirichlet data (NULL = zero)
  double* out;                // internal vector base
  double* xuser;              // gather-out target
  const double* xint;         // gather-out source base
  double delta, kappa;
  int block_begin;
  int nblocks;
};

// Composite residual b - A p over one rectangle (internal layout); halo
// lines read neighbouring rectangles of the same internal vector.
struct ResTask {
  RectDev rd;
  const double* p;            // internal vector base
  const double* b;
  double delta, kappa;
  double* partials;           // block sums of r^2 at [b], of b^2 at [pstride + b]
  int block_begin;
  int nblocks;
  int pstride;                // blocks of the whole problem (all rectangles)
  int pad;
};

// Sum of a problem's residual block partials into its state (one block).
struct ResSumTask {
  const double* partials;     // [2 * n]
  int n;
  int pad;
  ProbState* st;
};

// dst[0..count) = src[0..count), or 0 when src is null.
struct CopyTask {
  double* dst;
  const double* src;          // null: zero fill
  long long count;
  int block_begin;
  int nblocks;
  const double* mul;          // if set: dst = src * mul, element by element
  const int* skip;            // skip when *skip != 0
};

// Interface right-hand side updates between the centre and its arms of one
// problem, applied line after line by one block (lines of two arms share the
// centre's corner node):
//   f'_c formation:     fp[line_a] -= delta * q_a[row 0]
//   back substitution:  b_a[row 0] -= delta * x_c[line_a]
struct IfaceTask {
  double* dst[kMaxArms];
  const double* src[kMaxArms];
  long long dst_start[kMaxArms], dst_stride[kMaxArms];
  long long src_start[kMaxArms], src_stride[kMaxArms];
  int L[kMaxArms];
  int nlines;
  int pad;
  double delta;
};

// ---------------------------------------------------------------- interface Krylov
// Krylov iteration on the coupled rectangle's interface lines.  With the
// exact preconditioner the operator of right-preconditioned GMRES is
// I - S A_c^{-1}, and S (the Schur terms of the independent subdomains) only
// reads and writes the centre's boundary lines that carry an arm.  Every
// basis vector is therefore the interior part of the cycle's residual times a
// scalar plus a vector supported on those lines.  A vector is stored by its
// coordinates in an orthonormal system: [0] the coefficient of the unit
// interior residual, then for each line that carries an arm its orthonormal
// sine coefficients along the line (x lines S/N own the corner nodes they
// share with W/E lines).  Inner products of coordinates equal those of the
// centre vectors, so Gram-Schmidt and Givens run on vectors of length
// 1 + (sum of line lengths).  The operator needs (A_c^{-1} b) on the lines for
// a line-supported b: its blocks between lines of one axis are diagonal in
// the sine basis (corner entries of the per-mode tridiagonal inverses), and
// between the two axes they are sums of 1/(lambda_x + lambda_y + kappa)
// (the eigenvalues of A_c) against the sine values at the line positions.
constexpr int kIkThreads = 1024;  // threads of the per-problem kernels (start, combine)
constexpr int kIkEPT = 9;         // coordinates per thread there: 1 + lines <= 9216
constexpr int kIkMaxCoords = kIkThreads * kIkEPT;
constexpr int kIkSlab = kBlock;   // coordinates per block of the step kernels (one per thread)
constexpr int kIkMaxSlabs = (kIkMaxCoords + kIkSlab - 1) / kIkSlab;
constexpr int kIkDotChunk = 8;    // basis vectors per wavefront whose loads are in flight together
constexpr int kIkUpdChunk = 16;   // the same in the update pass
constexpr int kIkXThreads = 512;  // cross-axis sums: threads per block (8 wavefronts)
constexpr int kIkXTile = 64;      // cross-axis sums: target modes per block (one per lane)
constexpr int kIkXParts = 4;      // cross-axis sums: source ranges per target tile
constexpr int kIkXStage = 1024;   // cross-axis sums: source modes staged in LDS at a time

struct IkTask {
  ProbState* st;
  double* H;                  // Hessenberg, rotations, g, y: as in KryTask
  double* cs;
  double* sn;
  double* g;
  double* y;
  double* G;                  // Gram columns <v_l, v_i>, column-major (m+1)^2
  double* hv;                 // m+2: MGS coefficients of the current step (then its H column)
  double* Vb;                 // (m+1) x ldv coordinates
  int ldv, nb;                // row stride; sum of the present line lengths
  int m, flag_idx;
  int nx, ny;
  long long Nc;
  int P;                      // blocks of kVecPerBlock over the centre
  int present;                // bit a: line a carries an arm (0 S, 1 N, 2 W, 3 E)
  int off[4];                 // coordinate offset of line a (after the [0] entry), -1 if absent
  int nxa, nya;               // cross blocks of direction x->y and y->x (0 if unused)
  int nslab;                  // blocks of the step kernels (kIkSlab coordinates each)
  // plan tables
  const double* lamx;         // eigenvalues 2 delta (cos(k pi/(nx+1)) - 1)
  const double* lamy;
  const double* qx;           // orthonormal sine vector value at the first node
  const double* qy;
  const double* t00;          // [T_k^{-1}]_{00} and [T_k^{-1}]_{0,ny-1} of x mode k (x lines)
  const double* t0n;
  const double* s00;          // the same for y mode l (y lines)
  const double* s0n;
  const double* gd[4];        // Schur term of the arm on line a: delta^2 (2/N) g_k (line sine basis x N/2)
  double gscale[4];           // N/2 of line a (gd holds the S-matrix form's coefficients)
  double kappa;
  // per-problem work arrays
  double* u;                  // residual, then its interior part (Nc)
  double* V0;                 // sine coefficients along x of the interior residual (Nc)
  double* tz;                 // T^{-1} V0 at the cycle start, the update at the cycle end (Nc)
  double* rline;              // 4 x lmax: residual on each line's owned nodes
  double* rho;                // nb: line sine coefficients of rline
  double* zcol;               // 2 x ny: A^{-1} r_int on columns 0 and nx-1
  double* zc;                 // 2 x ny: their sine coefficients
  double* ucoef;              // 1 + nb: coordinates of the cycle's update V y
  double* uphys;              // 2 x ny: W/E lines of the update, physical values
  double* dhat;               // nb: S A^{-1} of the unit interior residual
  double* xpart;              // cross sums: [dir 2][acc 4][part kIkXParts][lmax]
  double* rscale;             // m+1: factor that normalises stored basis vector i
  double* Wv;                 // ldv: w of the current step
  double* dpart;              // (2 (m+1) + 1) x nslab block partials of the step kernels
  double* cpart;              // 4 x nxa: corner-value shares of the x->y cross blocks
  double* scal;               // [0] eta, [1] 1/eta (0 if eta = 0), [2] beta, [3] 1.0, [4] update
                              // factor of V0
  double* partials;           // >= P doubles: block sums of the interior residual
  int lmax;
  int block_begin;
};

}  // namespace fds
