// Batched GMRES engine (paper Section 2.4 and Algorithm 1).
//
// Per problem:  lift the Dirichlet data into the right-hand side; solve every
// arm A_a q_a = b_a with the fast solver; f'_c = b_c - sum_a R_ca q_a; solve
// L_c x_c = f'_c with restarted right-preconditioned GMRES(m) (plain FP64) or
// flexible GMRES(m) with an FP32 preconditioner; back-substitute the arms
// A_a p_a = b_a - R_ac x_c.  Every kernel launch serves all problems of the
// current set; problems whose cycle ended skip their work.  Problems join
// (admit: set-up phase) and leave (retire: back substitution and output) at
// cycle boundaries, so a request stream is served by continuous batching.
// Every kernel works on one problem's data with fixed-order reductions and a
// per-problem kernel configuration, so a problem's result does not depend on
// which other problems share its launches.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <cstdlib>
#include <functional>
#include <string>

#include "runtime.h"

namespace fds {

namespace {

size_t align256(size_t x) { return (x + 255) / 256 * 256; }

int div_up(long long a, long long b) { return (int)((a + b - 1) / b); }

// Task records of one launch; the device copy lives in the owning set's blob.
template <typename T>
struct TaskList {
  std::vector<T> h;
  const T* dptr = nullptr;
  int nblocks = 0;
  size_t smem = 0;
  const T* dev() const { return dptr; }
  int n() const { return (int)h.size(); }
};

template <typename T>
void add_block_task(TaskList<T>& tl, T t, int nblocks) {
  t.block_begin = tl.nblocks;
  tl.h.push_back(t);
  tl.nblocks += nblocks;
}

// All task lists of a set in one device allocation, written by one copy.
struct Blob {
  std::vector<unsigned char> host;
  DevBuf dev;
  std::vector<std::function<void(const unsigned char*)>> fix;
  template <typename T>
  void add(TaskList<T>& tl) {
    if (tl.h.empty()) return;
    const size_t off = align256(host.size());
    host.resize(off + sizeof(T) * tl.h.size());
    std::memcpy(host.data() + off, tl.h.data(), sizeof(T) * tl.h.size());
    TaskList<T>* p = &tl;
    fix.push_back([p, off](const unsigned char* base) { p->dptr = reinterpret_cast<const T*>(base + off); });
  }
  void upload(hipStream_t s) {
    if (host.empty()) return;
    dev.alloc(host.size());
    FDS_HIP(hipMemcpyAsync(dev.get(), host.data(), host.size(), hipMemcpyHostToDevice, s));
    for (auto& f : fix) f(dev.as<unsigned char>());
  }
};

// Row sine transforms of one stage, grouped by kernel configuration (wave
// FFT, workgroup FFT, or matrix-core product) so every launch runs one
// instantiation.
struct DstStage {
  DstKind kind = DstKind::D_D;
  struct Sub {
    DstChoice ch;
    TaskList<DstTask> tl;
  };
  std::vector<Sub> subs;
  explicit DstStage(DstKind k = DstKind::D_D) : kind(k) {}
  bool fp32() const { return kind != DstKind::D_D; }
  void add(DstTask t) {
    const DstChoice ch = dst_choice(t.n, fp32());
    Sub* sub = nullptr;
    for (Sub& s : subs)
      if (s.ch.gemm == ch.gemm && s.ch.rt == ch.rt && s.ch.ct == ch.ct &&
          s.ch.wave_e == ch.wave_e && s.ch.wave_big == ch.wave_big && s.ch.threads == ch.threads)
        sub = &s;
    if (!sub) {
      subs.push_back(Sub{ch, TaskList<DstTask>{}});
      sub = &subs.back();
    }
    t.rpb = ch.gemm ? 1 : ch.rows_per_block;
    t.tw_lds = (ch.gemm || ch.wave_e) ? 0 : (dst_twiddles_in_lds(t.n, fp32()) ? 1 : 0);
    if (ch.wave_e) {
      t.wd = TableCache::get().wave_desc(t.fft, fp32());
      t.io_f32 = dst_io_flags(kind);
    }
    add_block_task(sub->tl, t, div_up(t.rows, ch.rows_per_block));
    sub->tl.smem = std::max(sub->tl.smem, ch.smem);
  }
  int n() const {
    int c = 0;
    for (const Sub& s : subs) c += s.tl.n();
    return c;
  }
  void stage(Blob& b) {
    for (Sub& s : subs) b.add(s.tl);
  }
  void launch(int jidx, hipStream_t st) const {
    for (const Sub& s : subs) {
      if (s.ch.gemm)
        launch_dst_gemm(kind, s.ch.rt, s.ch.ct, s.tl.dev(), s.tl.n(), s.tl.nblocks, s.tl.smem, jidx, st);
      else if (s.ch.wave_e)
        launch_dst_wave(kind, s.ch.wave_e, s.ch.wave_big != 0, s.tl.dev(), s.tl.n(), s.tl.nblocks, s.ch.threads,
                        s.tl.smem, jidx, st);
      else
        launch_dst(kind, s.tl.dev(), s.tl.n(), s.tl.nblocks, s.tl.smem, jidx, st);
    }
  }
};

// Tridiagonal solves of one stage, grouped by the configuration each task's
// own row count selects.
struct TriStage {
  bool fp32 = false;
  struct Sub {
    TriConfig c;
    TaskList<TriTask> tl;
  };
  std::vector<Sub> subs;
  void add(TriTask t) {
    const TriConfig c = tri_config(fp32, t.rows);
    Sub* sub = nullptr;
    for (Sub& s : subs)
      if (s.c.seg == c.seg && s.c.ls == c.ls && s.c.mpb == c.mpb && s.c.threads == c.threads) sub = &s;
    if (!sub) {
      subs.push_back(Sub{c, TaskList<TriTask>{}});
      sub = &subs.back();
    }
    add_block_task(sub->tl, t, tri_blocks(c, t.modes));
  }
  int n() const {
    int c = 0;
    for (const Sub& s : subs) c += s.tl.n();
    return c;
  }
  void stage(Blob& b) {
    for (Sub& s : subs) b.add(s.tl);
  }
  void launch(hipStream_t st, int jidx = 0) const {
    for (const Sub& s : subs) launch_tri(s.c, fp32, s.tl.dev(), s.tl.n(), s.tl.nblocks, jidx, st);
  }
};

// Buffer layout of one problem, shared by allocation and footprint queries.
struct SlotLayout {
  size_t b_int, x_int, tmpd, ahat, fp, V, u, zbuf, lines, small, partials, respart, Z, tmpf, gram, zcols,
      bc, total;
  // interface Krylov iteration
  size_t V0, Vb, rline, rho, zcol, zc, ucoef, uphys, dhat, xpart, scal, rscale, Wv, dpart, cpart;
};

// Interface Krylov iteration: coordinates of the lines that carry an arm.
struct IkGeom {
  int nb = 0, ldv = 0, off[4] = {-1, -1, -1, -1};
  int nxa = 0, nya = 0;   // cross-sum blocks of the two directions
  int nslab = 1;          // blocks of the coordinate passes
};

IkGeom ik_geom(const fds_plan* p) {
  IkGeom g;
  for (const ArmInfo& a : p->arms) {
    g.off[a.line] = 0;
  }
  for (int a = 0; a < 4; ++a)
    if (g.off[a] == 0) {
      g.off[a] = g.nb;
      g.nb += a < 2 ? p->nx : p->ny;
    }
  g.ldv = (1 + g.nb + 31) / 32 * 32;
  const bool xl = g.off[0] >= 0 || g.off[1] >= 0, yl = g.off[2] >= 0 || g.off[3] >= 0;
  if (xl && yl) {
    g.nxa = div_up(p->ny, kIkXTile) * kIkXParts;   // x -> y: targets along y
    g.nya = div_up(p->nx, kIkXTile) * kIkXParts;
  }
  g.nslab = div_up(1 + g.nb, kIkSlab);
  return g;
}

int res_blocks_of(const fds_plan* p) {
  int nb = 0;
  for (const RectDev& d : p->rd) nb += std::max(1, div_up((long long)d.rows * d.cols, (long long)kBlock * 8));
  return nb;
}

SlotLayout layout_of(const fds_plan* p, int m, int precision) {
  const long long Nc = (long long)p->nx * p->ny;
  const long long Nint = p->n_internal;
  const int P = std::max(1, div_up(Nc, kVecPerBlock));
  const int Lmax = std::max(p->nx, p->ny);
  const bool flex = precision != FDS_FP64;
  SlotLayout L{};
  size_t o = 0;
  auto take = [&](size_t bytes) { size_t r = o; o += align256(bytes); return r; };
  L.b_int = take(8 * Nint);
  L.x_int = take(8 * Nint);
  L.tmpd = take(8 * Nint);
  L.ahat = take(8 * (Nint - Nc));   // sine coefficients of the arms' right-hand sides
  L.fp = take(8 * Nc);
  if (p->interface_krylov()) {
    const IkGeom g = ik_geom(p);
    L.u = take(8 * Nc);
    L.V0 = take(8 * Nc);
    L.lines = take(8 * 8 * (size_t)Lmax);   // four line terms, then four lines of scratch
    L.small = take(8 * ((size_t)(m + 1) * m + 4 * (size_t)m + 2));
    L.partials = take(8 * kry_partials_len(m, P));
    L.gram = take(8 * ((size_t)(m + 1) * (m + 1) + (m + 1)));
    L.respart = take(8 * 2 * (size_t)res_blocks_of(p));
    L.Vb = take(8 * (size_t)(m + 1) * g.ldv);
    L.rline = take(8 * 4 * (size_t)Lmax);
    L.rho = take(8 * (size_t)std::max(1, g.nb));
    L.zcol = take(8 * 2 * (size_t)p->ny);
    L.zc = take(8 * 2 * (size_t)p->ny);
    L.ucoef = take(8 * (size_t)(1 + g.nb));
    L.uphys = take(8 * 2 * (size_t)p->ny);
    L.dhat = take(8 * (size_t)std::max(1, g.nb));
    L.xpart = take(8 * 8 * kIkXParts * (size_t)Lmax);
    L.scal = take(8 * 16);
    L.rscale = take(8 * (size_t)(m + 1));
    L.Wv = take(8 * (size_t)g.ldv);
    L.dpart = take(8 * (size_t)(2 * (m + 1) + 1) * g.nslab);
    L.cpart = take(8 * 4 * (size_t)std::max(1, g.nxa));
    L.total = o;
    return L;
  }
  L.V = take(8 * (size_t)(m + 1) * Nc);
  L.u = take(8 * Nc);
  L.zbuf = flex ? 0 : take(8 * Nc);
  L.lines = take(8 * 8 * (size_t)Lmax);   // four line terms, then four lines of scratch
  L.small = take(8 * ((size_t)(m + 1) * m + 4 * (size_t)m + 2));
  L.partials = take(8 * kry_partials_len(m, P));
  L.gram = take(8 * ((size_t)(m + 1) * (m + 1) + (m + 1)));
  L.zcols = take(8 * 2 * (size_t)p->ny);
  L.bc = flex ? 0 : take(8 * 2 * (size_t)p->ny * (m + 1));
  L.respart = take(8 * 2 * (size_t)res_blocks_of(p));
  L.Z = flex ? take(4 * (size_t)m * Nc) : 0;
  L.tmpf = flex ? take(4 * Nc) : 0;
  L.total = o;
  return L;
}

}  // namespace

// One solve: its device memory and its slot in the engine's state pool.
struct Problem {
  SolveRequest req;
  fds_plan* plan = nullptr;
  int id = 0;                     // caller's id (returned by retire)
  int idx = 0;                    // index in the state pool / flag array
  DevBuf mem;
  double *b_int = nullptr, *x_int = nullptr, *tmpd = nullptr, *ahat = nullptr, *fp = nullptr, *V = nullptr,
         *u = nullptr, *zbuf = nullptr, *lines = nullptr, *H = nullptr, *cs = nullptr,
         *sn = nullptr, *g = nullptr, *y = nullptr, *partials = nullptr, *respart = nullptr,
         *G = nullptr, *hv = nullptr, *zcols = nullptr, *bc = nullptr;
  float *Z = nullptr, *tmpf = nullptr;
  // interface Krylov iteration
  double *V0 = nullptr, *Vb = nullptr, *rline = nullptr, *rho = nullptr, *zcol = nullptr, *zc = nullptr,
         *ucoef = nullptr, *uphys = nullptr, *dhat = nullptr, *xpart = nullptr, *scal = nullptr,
         *rscale = nullptr, *Wv = nullptr, *dpart = nullptr, *cpart = nullptr;
  double scal_init[16] = {0, 0, 0, 1.0};   // scal[3] = 1 (unit scale of a solve's input)
  ProbState* st = nullptr;
  long long Nc = 0, Nint = 0;
  int P = 0, Lmax = 0, res_blocks = 0;
};

namespace {

// The plain variant keeps the Gram columns from the update pass (one pass over
// the basis per step instead of two) when the restart length allows;
// FDS_GRAM_LAG=0 turns this off (measurements, A/B tests).
bool gram_lag_enabled(int m, bool flex) {
  if (flex || m > kLagMaxJ) return false;
  const char* v = std::getenv("FDS_GRAM_LAG");
  return !(v && std::string(v) == "0");
}

// Task lists of every phase for one set of problems.
struct TaskSet {
  int m = 0;
  bool flex = false;
  // arms: the forward transform of b_a is kept (ahat); the set-up needs the
  // solution's interface row only, and the back substitution changes the
  // right-hand side in the interface row only, so each takes a one-row
  // transform instead of a whole-arm one
  DstStage cyc_fwd, cyc_inv, arm_fwd, arm_inv, arm_inv0, bs_fwd0;
  TriStage it_tri, cyc_tri, arm_tri;
  TaskList<LineTask> it_lines_d, x_lines_d;  // dense line operators
  // line terms without a dense operator: S (gs * (S z_line)) by the batched
  // row transforms (forward, coefficient scaling, inverse)
  DstStage it_lnf, it_lni, x_lnf, x_lni;
  TaskList<CopyTask> it_lnm, x_lnm;
  int lmax_dense = 0;
  TaskList<ColTask> it_cols;
  // Jacobi preconditioner: z^ = Q D^-1 Q^T v^ (inverse transform, diagonal
  // scaling, forward transform; z^ = v^ is first written to Z_j in FP32)
  DstStage it_jinv{DstKind::F_D}, it_jfwd{DstKind::D_F};
  TaskList<CopyTask> it_jdiag;
  TaskList<OpTask> res_op;
  TaskList<KryTask> kry;
  TaskList<LiftTask> lift, gather;
  TaskList<IfaceTask> iface_fp, iface_bs;
  TaskList<ResTask> resid;
  TaskList<ResSumTask> res_sum;
  TaskList<CopyTask> setup_copy, fin_copy, arm_copy;
  std::vector<Problem*> probs;
  Blob blob;

  bool lag = false;   // lagged Gram columns (exact preconditioner, m <= kLagMaxJ)
  // interface Krylov iteration
  bool ik = false;
  TaskList<IkTask> ik_p, ik_x, ik_1;   // blocks over the centre / cross sums / one per problem
  TaskList<IkTask> ik_s;               // coordinate blocks of the step passes
  DstStage ik_lfwd, ik_linv;           // line transforms at the cycle start / end
  TriStage ik_tri0;                    // T^{-1} of the interior residual's coefficients
  TaskList<ColTask> ik_cols;           // its values on columns 0 and nx-1
  int ik_max_coords = 1;               // longest coordinate vector (1 + nb) of the set

  TaskSet(int m_, bool flex_, bool ik_ = false) : m(m_), flex(flex_), ik(ik_) {
    it_tri.fp32 = flex;
    lag = !ik && gram_lag_enabled(m_, flex_);
  }
  void add_problem_ik(Problem& sl);
  void ik_cycle_start(hipStream_t s) const;
  void add_problem(Problem& sl);
  void upload(hipStream_t s) {
    for (DstStage* d : {&cyc_fwd, &cyc_inv, &arm_fwd, &arm_inv, &arm_inv0, &bs_fwd0, &ik_lfwd, &ik_linv, &it_jinv,
                        &it_jfwd,
                        &it_lnf, &it_lni, &x_lnf, &x_lni})
      d->stage(blob);
    blob.add(it_jdiag);
    blob.add(it_lnm);
    blob.add(x_lnm);
    for (TriStage* t : {&it_tri, &cyc_tri, &arm_tri, &ik_tri0}) t->stage(blob);
    blob.add(ik_p);
    blob.add(ik_s);
    blob.add(ik_x);
    blob.add(ik_1);
    blob.add(ik_cols);
    blob.add(it_lines_d);
    blob.add(x_lines_d);
    blob.add(it_cols);
    blob.add(res_op);
    blob.add(kry);
    blob.add(lift);
    blob.add(gather);
    blob.add(iface_fp);
    blob.add(iface_bs);
    blob.add(resid);
    blob.add(res_sum);
    blob.add(setup_copy);
    blob.add(fin_copy);
    blob.add(arm_copy);
    blob.upload(s);
  }
  // called with the line class open: the two transforms of the transform
  // path are timed with the transform class
  void launch_x_lines(hipStream_t s) const {
    launch_lines_dense(x_lines_d.dev(), x_lines_d.n(), x_lines_d.nblocks, lmax_dense, 0, s);
    if (x_lnm.n()) launch_line_stages(x_lnf, x_lnm, x_lni, 0, s);
  }
  static void launch_line_stages(const DstStage& fwd, const TaskList<CopyTask>& mul, const DstStage& inv,
                                 int jidx, hipStream_t s) {
    Timing::end(4, s);
    Timing::begin(0, s);
    fwd.launch(jidx, s);
    Timing::end(0, s);
    Timing::begin(4, s);
    launch_copy(mul.dev(), mul.n(), mul.nblocks, s);
    Timing::end(4, s);
    Timing::begin(0, s);
    inv.launch(jidx, s);
    Timing::end(0, s);
    Timing::begin(4, s);
  }
  // S (gs * (S z)) on one line into `out`, through `tmp` (L doubles each)
  static void add_line_stages(DstStage& fwd, TaskList<CopyTask>& mul, DstStage& inv, const double* z,
                              long long stride, int L, const double* gs, double* tmp, double* out,
                              const FftDesc* fft, const int* skip) {
    DstTask f{};
    f.in = z; f.in_cs = stride; f.out = tmp; f.out_cs = 1;
    f.rows = 1; f.n = L; f.scale = 1.0; f.fft = fft; f.skip = skip;
    fwd.add(f);
    CopyTask c{tmp, tmp, L, 0, 1, gs, skip};
    add_block_task(mul, c, 1);
    DstTask v{};
    v.in = tmp; v.in_cs = 1; v.out = out; v.out_cs = 1;
    v.rows = 1; v.n = L; v.scale = 1.0; v.fft = fft; v.skip = skip;
    inv.add(v);
  }
  void iteration(int j, int* flags_dev, int tag, hipStream_t s) const;
  void end_of_cycle(int max_cycles, hipStream_t s) const;
};

void TaskSet::add_problem(Problem& sl) {
  probs.push_back(&sl);
  fds_plan* p = sl.plan;
  const RectDev& cd = p->cdev;
  const int nx = p->nx, ny = p->ny;
  const long long Nc = sl.Nc;
  const int* skip_it = &sl.st->cycle_done;
  const int* skip_fin = &sl.st->finished;
  const FftDesc* fftc = p->fft_c->dev;
  const int rpb_c = kBlock / dst_threads_per_row(nx);

  // ---- per-iteration work on the centre.  The Krylov basis of both variants
  // lives in the orthonormal sine basis of the centre (Q = sqrt(2/N) S along
  // x), so the preconditioner A_c^{-1} = Q^T T^{-1} Q reduces to the
  // tridiagonal solve per mode.  The solve reads v_j times ProbState::vscale,
  // writes v_j back normalised, and writes z^ to FP64 scratch (plain) or to
  // z^_j in FP32 (flexible, Z).  The W/E Schur lines need z on
  // the centre's columns 0 / nx-1 (row sums of z^); the plain variant also
  // keeps the physical boundary columns of v_j for <v_i, s>.
  bool west = false, east = false;
  for (const ArmInfo& a : p->arms) { west |= a.line == 2; east |= a.line == 3; }
  const double qscale = std::sqrt(2.0 / (nx + 1));
  if (ik) add_problem_ik(sl);
  if (!ik) {
    TriTask tt{};
    tt.data = flex ? (void*)sl.Z : (void*)sl.tmpd; tt.rs = nx; tt.js = flex ? Nc : 0;
    tt.rows = ny; tt.modes = nx;
    tt.coef = flex ? (const void*)p->modes_cu->c32 : (const void*)p->modes_cu->c64;
    tt.skip = skip_it;
    tt.vin = sl.V; tt.vjs = Nc; tt.vscale = &sl.st->vscale;
    const bool jacobi = p->opt.precision == FDS_JACOBI;
    tt.identity = (p->opt.precision == FDS_NO_PRECOND || jacobi) ? 1 : 0;   // z^ = v^ (P = I)
    it_tri.add(tt);
    if (jacobi) {
      DstTask a{};
      a.in = sl.Z; a.in_rs = nx; a.in_cs = 1; a.in_js = Nc;
      a.out = sl.tmpd; a.out_rs = nx; a.out_cs = 1;
      a.rows = ny; a.n = nx; a.scale = qscale; a.fft = fftc; a.skip = skip_it;
      it_jinv.add(a);
      const int nb = std::max(1, div_up(Nc, (long long)kBlock * 8));
      CopyTask c{sl.tmpd, sl.tmpd, Nc, 0, nb, p->jacobi->dinv, skip_it};
      add_block_task(it_jdiag, c, nb);
      DstTask b{};
      b.in = sl.tmpd; b.in_rs = nx; b.in_cs = 1;
      b.out = sl.Z; b.out_rs = nx; b.out_cs = 1; b.out_js = Nc;
      b.rows = ny; b.n = nx; b.scale = qscale; b.fft = fftc; b.skip = skip_it;
      it_jfwd.add(b);
    }
    if (west || east) {
      ColTask ct{};
      if (flex) { ct.y32 = sl.Z; ct.y_js = Nc; }
      else { ct.y = sl.tmpd; ct.v = sl.V; ct.bc = sl.bc; ct.Nc = Nc; }
      ct.scale = qscale;
      ct.zw = west ? sl.zcols : nullptr; ct.ze = east ? sl.zcols + ny : nullptr;
      ct.fft = fftc; ct.nx = nx; ct.ny = ny; ct.skip = skip_it;
      add_block_task(it_cols, ct, div_up(ny, kBlock / 64));
    }
  }
  // ---- end of cycle: u = V y (plain) or Z y (flexible), sine coefficients;
  // plain: u = T^{-1} u; then x_c += Q^T u.  The true residual r (in u) then
  // becomes v_0 = Q r.
  {
    if (!flex) {
      TriTask tt{};
      tt.data = ik ? sl.tmpd : sl.u; tt.rs = nx; tt.rows = ny; tt.modes = nx; tt.coef = p->modes_cu->c64;
      tt.skip = skip_fin;
      cyc_tri.add(tt);
    }
    DstTask v{};
    v.in = ik ? sl.tmpd : sl.u; v.in_rs = nx; v.in_cs = 1; v.out = sl.x_int + cd.off; v.out_rs = nx;
    v.out_cs = 1; v.accumulate = 1;
    v.rows = ny; v.n = nx; v.rpb = rpb_c; v.scale = qscale; v.fft = fftc; v.skip = skip_fin;
    v.tw_lds = dst_twiddles_in_lds(nx, false);
    cyc_inv.add(v);
    DstTask f{};
    f.in = sl.u; f.in_rs = nx; f.in_cs = 1; f.out = ik ? sl.V0 : sl.V; f.out_rs = nx; f.out_cs = 1;
    f.rows = ny; f.n = nx; f.rpb = rpb_c; f.scale = qscale; f.fft = fftc; f.skip = skip_fin;
    f.tw_lds = dst_twiddles_in_lds(nx, false);
    cyc_fwd.add(f);
  }
  // ---- Schur lines and operators
  OpTask ot{};
  ot.nx = nx; ot.ny = ny; ot.nblocks = sl.P; ot.delta = p->delta; ot.kappa = p->kappa;
  for (int q = 0; q < 4; ++q) ot.line[q] = nullptr;
  IfaceTask fi{}, bi{};
  fi.delta = bi.delta = p->delta;
  for (const ArmInfo& a : p->arms) {
    LineTask lt{};
    lt.L = a.L;
    lt.fft = a.fft->dev;
    lt.gs = a.gs->gs;
    lt.out = sl.lines + (size_t)a.line * sl.Lmax;
    switch (a.line) {
      case 0: lt.start = 0; lt.stride = 1; break;
      case 1: lt.start = (long long)(ny - 1) * nx; lt.stride = 1; break;
      case 2: lt.start = 0; lt.stride = nx; break;
      case 3: lt.start = nx - 1; lt.stride = nx; break;
    }
    ot.line[a.line] = lt.out;
    LineTask li = lt;
    li.skip = skip_it;
    // S/N blocks are diagonal in the centre's sine basis (spec_w, and
    // qs terms in the plain Arnoldi step): no line term per step; the
    // interface iteration forms its own
    const bool it_line = a.line >= 2 && !ik;
    li.z = sl.zcols + (a.line == 3 ? ny : 0); li.z_js = 0; li.z_f32 = 0;
    li.start = 0; li.stride = 1;
    LineTask lx = lt;
    lx.z = sl.x_int + cd.off; lx.z_js = 0; lx.z_f32 = 0; lx.skip = skip_fin;
    if (dense_lines(a.L) && a.gs->mfull) {
      li.mat = a.gs->mfull;
      lx.mat = a.gs->mfull;
      if (it_line) add_block_task(it_lines_d, li, div_up(a.L, 64));
      add_block_task(x_lines_d, lx, div_up(a.L, 64));
      lmax_dense = std::max(lmax_dense, a.L);
    } else {
      double* tmp = sl.lines + (size_t)(4 + a.line) * sl.Lmax;
      if (it_line)
        add_line_stages(it_lnf, it_lnm, it_lni, static_cast<const double*>(li.z), 1, a.L, a.gs->gs, tmp,
                        lt.out, a.fft->dev, skip_it);
      add_line_stages(x_lnf, x_lnm, x_lni, sl.x_int + cd.off + lt.start, lt.stride, a.L, a.gs->gs, tmp,
                      lt.out, a.fft->dev, skip_fin);
    }

    // f'_c formation and back substitution
    const RectDev& ad = p->rd[a.rect];
    const int q = fi.nlines++;
    fi.dst[q] = sl.fp; fi.dst_start[q] = lt.start; fi.dst_stride[q] = lt.stride;
    fi.src[q] = sl.x_int; fi.src_start[q] = ad.off; fi.src_stride[q] = 1; fi.L[q] = a.L;
    bi.dst[q] = sl.x_int; bi.dst_start[q] = ad.off; bi.dst_stride[q] = 1;
    bi.src[q] = sl.x_int; bi.src_start[q] = cd.off + lt.start; bi.src_stride[q] = lt.stride;
    bi.L[q] = a.L;
    bi.nlines = fi.nlines;

    // arm solves (FP64).  Set-up: b_a -> ahat (kept), copied to tmpd, per-mode
    // solves, interface row -> x_int.  Back substitution: ahat copied to
    // tmpd, its interface row replaced by the transform of the updated
    // interface row of the right-hand side, per-mode solves, tmpd -> x_int.
    const int rpb = kBlock / dst_threads_per_row(a.L);
    double* ah = sl.ahat + (ad.off - sl.Nc);
    DstTask f{};
    f.in = sl.b_int + ad.off; f.in_rs = a.L; f.in_cs = 1;
    f.out = ah; f.out_rs = a.L; f.out_cs = 1;
    f.rows = a.rows; f.n = a.L; f.rpb = rpb; f.scale = 1.0; f.fft = a.fft->dev; f.skip = nullptr;
    f.tw_lds = dst_twiddles_in_lds(a.L, false);
    arm_fwd.add(f);
    DstTask fb = f;
    fb.in = sl.x_int + ad.off; fb.out = sl.tmpd + ad.off; fb.rows = 1;
    bs_fwd0.add(fb);
    TriTask at{};
    at.data = sl.tmpd + ad.off; at.rs = a.L; at.rows = a.rows; at.modes = a.L;
    at.coef = a.modes->c64; at.skip = nullptr;
    arm_tri.add(at);
    DstTask iv = f;
    iv.in = sl.tmpd + ad.off; iv.out = sl.x_int + ad.off;
    arm_inv.add(iv);
    DstTask iv0 = iv;
    iv0.rows = 1;
    arm_inv0.add(iv0);
  }
  iface_fp.h.push_back(fi);
  iface_bs.h.push_back(bi);
  {
    OpTask r = ot;
    r.z = sl.x_int + cd.off; r.z_js = 0; r.z_f32 = 0;
    r.out = sl.u; r.out_js = 0; r.fp = sl.fp;
    r.partials = sl.partials + (size_t)kPartRes * sl.P;
    r.skip = skip_fin;
    add_block_task(res_op, r, sl.P);
  }
  if (ik) {
    // restart decision and least squares only (no stored centre basis)
    KryTask k{};
    k.x = sl.x_int + cd.off; k.u = sl.u; k.H = sl.H; k.cs = sl.cs; k.sn = sl.sn; k.g = sl.g;
    k.y = sl.y; k.partials = sl.partials; k.st = sl.st; k.Nc = Nc; k.P = sl.P; k.m = m; k.G = sl.G;
    k.hv = sl.hv; k.nx = nx; k.ny = ny; k.flag_idx = sl.idx;
    add_block_task(kry, k, sl.P);
  } else {
    KryTask k{};
    k.V = sl.V; k.Z = sl.Z; k.x = sl.x_int + cd.off; k.u = sl.u; k.H = sl.H; k.cs = sl.cs;
    k.sn = sl.sn; k.g = sl.g; k.y = sl.y; k.partials = sl.partials; k.st = sl.st; k.Nc = Nc;
    k.P = sl.P; k.m = m; k.G = sl.G; k.hv = sl.hv; k.nx = nx; k.ny = ny;
    k.flag_idx = sl.idx;
    k.gram_lag = lag ? 1 : 0;
    k.implicit_w = flex ? 0 : 1;
    for (int q = 0; q < 4; ++q) k.line[q] = (q >= 2 && !flex) ? ot.line[q] : nullptr;
    for (const ArmInfo& a : p->arms)
      if (a.line < 2) k.gs[a.line] = a.gs->gs;
    k.post = p->fft_c->host.post64;
    k.qscale = qscale;
    k.half_n = 0.5 * (nx + 1);
    if (!flex) {
      k.zhat = sl.tmpd;
      k.bc = sl.bc;
    } else {
      // the dot pass applies the operator itself (spec_w)
      k.fuse_op = 1;
      k.delta = p->delta;
      k.kappa = p->kappa;
      k.line[2] = ot.line[2];
      k.line[3] = ot.line[3];
    }
    add_block_task(kry, k, sl.P);
  }
  // ---- layout conversion and composite residual
  for (size_t r = 0; r < p->rd.size(); ++r) {
    const RectDev& d = p->rd[r];
    const long long tot = (long long)d.rows * d.cols;
    LiftTask lt{};
    lt.rd = d; lt.rhs = sl.req.rhs; lt.bc = sl.req.bc; lt.out = sl.b_int; lt.xuser = sl.req.x;
    lt.xint = sl.x_int; lt.delta = p->delta; lt.kappa = p->kappa;
    const int nb = std::max(1, div_up(tot, (long long)kBlock * 4));
    lt.nblocks = nb;
    add_block_task(lift, lt, nb);
    add_block_task(gather, lt, nb);
  }
  {
    const int total = res_blocks_of(p);
    int off = 0;
    for (size_t r = 0; r < p->rd.size(); ++r) {
      const RectDev& d = p->rd[r];
      ResTask rt{};
      rt.rd = d; rt.p = sl.x_int; rt.b = sl.b_int; rt.delta = p->delta; rt.kappa = p->kappa;
      const int nb = std::max(1, div_up((long long)d.rows * d.cols, (long long)kBlock * 8));
      rt.nblocks = nb;
      rt.partials = sl.respart + off;
      rt.pstride = total;
      off += nb;
      add_block_task(resid, rt, nb);
    }
    sl.res_blocks = off;
    res_sum.h.push_back(ResSumTask{sl.respart, total, 0, sl.st});
  }
  // set-up copies: f'_c starts as b_c and x_c at zero; the back substitution
  // starts the arms' interface rows from b_a
  const long long coff = p->cdev.off;
  auto copy = [&](TaskList<CopyTask>& tl, double* dst, const double* src, long long count) {
    if (count <= 0) return;
    const int nb = std::max(1, div_up(count, (long long)kBlock * 8));
    CopyTask c{dst, src, count, 0, nb};
    add_block_task(tl, c, nb);
  };
  copy(setup_copy, sl.fp, sl.b_int + coff, sl.Nc);
  copy(setup_copy, sl.x_int + coff, nullptr, sl.Nc);
  // (the back substitution needs b_a's interface row only: the other rows
  // enter through ahat)
  for (const ArmInfo& a : p->arms) {
    const long long o = p->rd[a.rect].off;
    copy(fin_copy, sl.x_int + o, sl.b_int + o, a.L);
  }
  copy(arm_copy, sl.tmpd + coff + sl.Nc, sl.ahat, sl.Nint - sl.Nc);
}

// Task records of the interface Krylov iteration for one problem.
void TaskSet::add_problem_ik(Problem& sl) {
  fds_plan* p = sl.plan;
  const int nx = p->nx, ny = p->ny;
  const IkGeom g = ik_geom(p);
  const int* skip_fin = &sl.st->finished;
  IkTask t{};
  t.st = sl.st; t.H = sl.H; t.cs = sl.cs; t.sn = sl.sn; t.g = sl.g; t.y = sl.y; t.G = sl.G; t.hv = sl.hv;
  t.Vb = sl.Vb; t.ldv = g.ldv; t.nb = g.nb; t.m = m; t.flag_idx = sl.idx;
  t.nx = nx; t.ny = ny; t.Nc = sl.Nc; t.P = sl.P;
  for (int a = 0; a < 4; ++a) {
    t.off[a] = g.off[a];
    t.gd[a] = nullptr;
    t.gscale[a] = 0.0;
  }
  for (const ArmInfo& a : p->arms) {
    t.gd[a.line] = a.gs->gs;
    t.gscale[a.line] = 0.5 * (a.L + 1);
    t.present |= 1 << a.line;
  }
  t.nxa = g.nxa; t.nya = g.nya; t.nslab = g.nslab;
  t.rscale = sl.rscale; t.Wv = sl.Wv; t.dpart = sl.dpart; t.cpart = sl.cpart;
  t.lamx = p->ik->lamx; t.lamy = p->ik->lamy; t.qx = p->ik->qx; t.qy = p->ik->qy;
  t.t00 = p->ik->t00; t.t0n = p->ik->t0n; t.s00 = p->ik->s00; t.s0n = p->ik->s0n;
  t.kappa = p->kappa;
  t.u = sl.u; t.V0 = sl.V0; t.tz = sl.tmpd; t.rline = sl.rline; t.rho = sl.rho; t.zcol = sl.zcol;
  t.zc = sl.zc; t.ucoef = sl.ucoef; t.uphys = sl.uphys; t.dhat = sl.dhat; t.xpart = sl.xpart;
  t.scal = sl.scal; t.partials = sl.partials + (size_t)kPartNorm * sl.P; t.lmax = sl.Lmax;
  ik_max_coords = std::max(ik_max_coords, 1 + g.nb);
  add_block_task(ik_s, t, g.nslab);
  add_block_task(ik_p, t, sl.P);
  if (g.nxa + g.nya > 0) add_block_task(ik_x, t, g.nxa + g.nya);
  add_block_task(ik_1, t, 1);
  // cycle start: T^{-1} of the interior residual's coefficients (read from
  // V0, which is written back unchanged: scale scal[3] = 1) into tz, its
  // values on columns 0 / nx-1, and the line transforms
  TriTask tt{};
  tt.data = sl.tmpd; tt.rs = nx; tt.rows = ny; tt.modes = nx; tt.coef = p->modes_cu->c64;
  tt.skip = skip_fin; tt.vin = sl.V0; tt.vjs = 0; tt.vscale = sl.scal + 3;
  ik_tri0.add(tt);
  if (g.off[2] >= 0 || g.off[3] >= 0) {
    ColTask ct{};
    ct.y = sl.tmpd; ct.zw = g.off[2] >= 0 ? sl.zcol : nullptr; ct.ze = g.off[3] >= 0 ? sl.zcol + ny : nullptr;
    ct.fft = p->fft_c->dev; ct.nx = nx; ct.ny = ny; ct.skip = skip_fin; ct.scale = std::sqrt(2.0 / (nx + 1));
    add_block_task(ik_cols, ct, div_up(ny, kBlock / 64));
  }
  // transform tables from the plan (the arms' lines have the centre's side
  // lengths): no table lookups while the set is rebuilt
  const FftDesc* fft_line[4] = {p->fft_c->dev, p->fft_c->dev, nullptr, nullptr};
  for (const ArmInfo& a : p->arms) fft_line[a.line] = a.fft->dev;
  auto line_dst = [&](DstStage& st, const double* in, double* out, int L, const FftDesc* fft) {
    DstTask d{};
    d.in = in; d.out = out; d.in_rs = L; d.out_rs = L; d.in_cs = 1; d.out_cs = 1;
    d.rows = 1; d.n = L; d.scale = std::sqrt(2.0 / (L + 1)); d.skip = skip_fin;
    d.fft = fft;
    d.tw_lds = dst_twiddles_in_lds(L, false);
    st.add(d);
  };
  for (int a = 0; a < 4; ++a) {
    if (g.off[a] < 0) continue;
    const int L = a < 2 ? nx : ny;
    line_dst(ik_lfwd, sl.rline + (size_t)a * sl.Lmax, sl.rho + g.off[a], L, fft_line[a]);
    if (a >= 2) {
      line_dst(ik_lfwd, sl.zcol + (size_t)(a - 2) * ny, sl.zc + (size_t)(a - 2) * ny, ny, fft_line[a]);
      line_dst(ik_linv, sl.ucoef + 1 + g.off[a], sl.uphys + (size_t)(a - 2) * ny, ny, fft_line[a]);
    }
  }
}

// Cycle start of the interface iteration (after the residual r is in u and
// the restart decision is taken): split r into its interior part and its
// lines, transform the interior part along x, solve per mode, read the
// solution's values on the lines, transform the lines, then v_0 and
// S A^{-1} of the unit interior residual.
void TaskSet::ik_cycle_start(hipStream_t s) const {
  Timing::begin(2, s);
  launch_ik_extract(ik_p.dev(), ik_p.n(), ik_p.nblocks, s);
  Timing::end(2, s);
  Timing::begin(0, s);
  cyc_fwd.launch(0, s);
  Timing::end(0, s);
  Timing::begin(1, s);
  ik_tri0.launch(s);
  Timing::end(1, s);
  if (ik_cols.n()) {
    Timing::begin(7, s);
    launch_idst_cols(ik_cols.dev(), ik_cols.n(), ik_cols.nblocks, 0, s);
    Timing::end(7, s);
  }
  Timing::begin(0, s);
  ik_lfwd.launch(0, s);
  Timing::end(0, s);
  Timing::begin(5, s);
  launch_ik_start(ik_1.dev(), ik_1.n(), ik_max_coords, s);
  Timing::end(5, s);
}

// One Arnoldi step j of every problem of the set whose cycle is running.
void TaskSet::iteration(int j, int* flags_dev, int tag, hipStream_t s) const {
  if (ik) {
    if (ik_x.n()) {
      Timing::begin(4, s);
      launch_ik_cross(ik_x.dev(), ik_x.n(), ik_x.nblocks, j, s);
      Timing::end(4, s);
    }
    Timing::begin(3, s);
    launch_ik_wdots(ik_s.dev(), ik_s.n(), ik_s.nblocks, j, s);
    Timing::end(3, s);
    Timing::begin(6, s);
    launch_ik_update(ik_s.dev(), ik_s.n(), ik_s.nblocks, j, flags_dev, tag, s);
    Timing::end(6, s);
    FDS_HIP(hipGetLastError());
    return;
  }
  Timing::begin(1, s);
  it_tri.launch(s, j);
  Timing::end(1, s);
  if (it_jdiag.n()) {
    Timing::begin(0, s);
    it_jinv.launch(j, s);
    launch_copy(it_jdiag.dev(), it_jdiag.n(), it_jdiag.nblocks, s);
    it_jfwd.launch(j, s);
    Timing::end(0, s);
  }
  if (it_cols.n()) {
    Timing::begin(7, s);
    launch_idst_cols(it_cols.dev(), it_cols.n(), it_cols.nblocks, j, s);
    Timing::end(7, s);
  }
  if (it_lnm.n() || it_lines_d.n()) {
    Timing::begin(4, s);
    launch_lines_dense(it_lines_d.dev(), it_lines_d.n(), it_lines_d.nblocks, lmax_dense, j, s);
    if (it_lnm.n()) launch_line_stages(it_lnf, it_lnm, it_lni, j, s);
    Timing::end(4, s);
  }
  Timing::begin(3, s);
  if (lag) launch_gram_bdots(kry.dev(), kry.n(), j, s);
  else launch_gram_dots(kry.dev(), kry.n(), kry.nblocks, j, s);
  Timing::end(3, s);
  Timing::begin(6, s);
  if (lag) launch_gram_update_lag(kry.dev(), kry.n(), kry.nblocks, m, j, flags_dev, tag, s);
  else launch_gram_update(kry.dev(), kry.n(), kry.nblocks, j, flags_dev, tag, s);
  Timing::end(6, s);
  FDS_HIP(hipGetLastError());
}

void TaskSet::end_of_cycle(int max_cycles, hipStream_t s) const {
  if (ik) {
    // x += A^{-1} (V y): coordinates of the update, its W/E lines in physical
    // values, its sine coefficients along x, the per-mode solve and the
    // inverse transform; then the true residual, the restart decision and
    // the next cycle's start
    Timing::begin(5, s);
    launch_ls_solve(kry.dev(), kry.n(), m, s);
    launch_ik_combine(ik_1.dev(), ik_1.n(), s);
    Timing::end(5, s);
    Timing::begin(0, s);
    ik_linv.launch(0, s);
    Timing::end(0, s);
    Timing::begin(2, s);
    launch_ik_compose(ik_p.dev(), ik_p.n(), ik_p.nblocks, s);
    Timing::end(2, s);
    Timing::begin(1, s);
    cyc_tri.launch(s);
    Timing::end(1, s);
    Timing::begin(0, s);
    cyc_inv.launch(0, s);
    Timing::end(0, s);
    if (x_lnm.n() || x_lines_d.n()) {
      Timing::begin(4, s);
      launch_x_lines(s);
      Timing::end(4, s);
    }
    Timing::begin(2, s);
    launch_operator(1, res_op.dev(), res_op.n(), res_op.nblocks, 0, s);
    Timing::end(2, s);
    Timing::begin(5, s);
    launch_restart_decide(kry.dev(), kry.n(), 0, max_cycles, s);
    Timing::end(5, s);
    ik_cycle_start(s);
    FDS_HIP(hipGetLastError());
    return;
  }
  Timing::begin(5, s);
  launch_ls_solve(kry.dev(), kry.n(), m, s);
  launch_combine(flex, kry.dev(), kry.n(), kry.nblocks, s);
  Timing::end(5, s);
  if (!flex) {
    Timing::begin(1, s);
    cyc_tri.launch(s);
    Timing::end(1, s);
  }
  Timing::begin(0, s);
  cyc_inv.launch(0, s);
  Timing::end(0, s);
  if (x_lnm.n() || x_lines_d.n()) {
    Timing::begin(4, s);
    launch_x_lines(s);
    Timing::end(4, s);
  }
  Timing::begin(2, s);
  launch_operator(1, res_op.dev(), res_op.n(), res_op.nblocks, 0, s);
  Timing::end(2, s);
  Timing::begin(0, s);   // v_0 = Q r (before the restart kernels scale it)
  cyc_fwd.launch(0, s);
  Timing::end(0, s);
  Timing::begin(5, s);
  launch_restart(kry.dev(), kry.n(), kry.nblocks, 0, max_cycles, s);
  Timing::end(5, s);
  FDS_HIP(hipGetLastError());
}

// Line term of one arm: the line in and out, plus the dense operator when
// the term is a dense product.
// Algorithmic bytes of `times` Schur line terms of one arm: the dense
// operator (line class: the line in and out, the matrix), or two line
// transforms (transform class: in and out each) around the coefficient
// scaling (line class: the line in and out, the coefficients).
void add_line_bytes(const ArmInfo& a, double times) {
  if (dense_lines(a.L) && a.gs->mfull) {
    Timing::add_bytes(4, times * (16.0 * a.L + 8.0 * a.L * a.L));
  } else {
    Timing::add_bytes(0, times * 32.0 * a.L);
    Timing::add_bytes(4, times * 24.0 * a.L);
  }
}

}  // namespace

struct Engine::Impl {
  int m, precision, max_cycles;
  bool flex;
  bool ik = false;                    // interface Krylov iteration
  hipStream_t s;
  int capacity = 0;
  DevBuf states;                      // state pool (capacity entries)
  std::vector<ProbState> host_states;
  int* flags_host = nullptr;          // per pool index: serial of the last cycle that ended (mapped)
  int* flags_dev = nullptr;
  std::vector<int> free_idx;
  std::vector<std::unique_ptr<Problem>> active;
  std::unique_ptr<TaskSet> cur;       // task lists of `active` (null when stale)
  int cycle_serial = 0;
  // cycle in flight (between cycle_launch and cycle_finish)
  bool in_flight = false;
  std::vector<ProbState> before;
  // captured cycle of the current task set
  // one hipGraph per GMRES cycle (FDS_GRAPH=1): off by default, since a
  // capture and instantiation cost about 0.7 ms, more than the launches of
  // the cycles a solve replays it for (measured on the plain and batching
  // workloads; the host enqueues a cycle faster than the device runs it)
  bool graphs = false;
  long long ts_gen = 0;               // bumped whenever `cur` is replaced
  long long cycles_on_gen = 0;        // cycles run with the current task set
  // cycles of an unchanged task set launched kernel by kernel before one is
  // captured (capture and instantiation cost about what a few cycles' launches do)
  int graph_after = 1;
  long long graph_gen = -1;
  hipGraphExec_t gexec = nullptr;
  hipStream_t cap_stream = nullptr;   // capture only (nothing runs on it)
  int replays = 0;
  double t_tasks = 0;                 // host seconds building task lists

  ~Impl() {
    // the device buffers go back to the cache: nothing queued may still use them
    if (s) (void)hipStreamSynchronize(s);
    if (gexec) (void)hipGraphExecDestroy(gexec);
    if (cap_stream) (void)hipStreamDestroy(cap_stream);
    if (flags_host) host_mapped_free(flags_host, sizeof(int) * capacity);
  }
  void set_cur(std::unique_ptr<TaskSet> ts) {
    cur = std::move(ts);
    ++ts_gen;
    cycles_on_gen = 0;
  }
  void launch_graph_cycle(TaskSet& ts);
  void read_states();
  TaskSet& current();
  void setup_phase(TaskSet& ts);
  std::vector<SolveOutcome> finalize_phase(TaskSet& ts);
  // Algorithmic bytes (each operand read once, each result written once) of
  // the work every problem did in the cycle that just ended, by kernel class.
  void account_cycle(const std::vector<ProbState>& before);
  void account_arms(const std::vector<Problem*>& probs, bool setup_phase);
};

void Engine::Impl::read_states() {
  FDS_HIP(hipMemcpyAsync(host_states.data(), states.get(), sizeof(ProbState) * capacity,
                         hipMemcpyDeviceToHost, s));
  FDS_HIP(hipStreamSynchronize(s));
}

TaskSet& Engine::Impl::current() {
  if (!cur) {
    const auto t0 = std::chrono::steady_clock::now();
    std::unique_ptr<TaskSet> ts(new TaskSet(m, flex, ik));
    for (auto& p : active) ts->add_problem(*p);
    ts->upload(s);
    set_cur(std::move(ts));
    t_tasks += std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  }
  return *cur;
}

// Every Arnoldi step of a cycle and the cycle's end, captured once per task
// set and replayed: the kernels of a step take their step index as a launch
// argument and find everything else through the task lists, which stay put
// while the set is unchanged.  All m steps are in the graph; a problem whose
// cycle ended early skips its blocks (its cycle_done flag), as it does in
// kernel-by-kernel mode while other problems still iterate.
void Engine::Impl::launch_graph_cycle(TaskSet& ts) {
  if (graph_gen != ts_gen) {
    if (gexec) {
      FDS_HIP(hipGraphExecDestroy(gexec));
      gexec = nullptr;
    }
    if (!cap_stream) FDS_HIP(hipStreamCreateWithFlags(&cap_stream, hipStreamNonBlocking));
    FDS_HIP(hipStreamBeginCapture(cap_stream, hipStreamCaptureModeRelaxed));
    hipGraph_t g = nullptr;
    try {
      for (int j = 0; j < m; ++j) ts.iteration(j, flags_dev, 0, cap_stream);
      ts.end_of_cycle(max_cycles, cap_stream);
    } catch (...) {
      (void)hipStreamEndCapture(cap_stream, &g);
      if (g) (void)hipGraphDestroy(g);
      throw;
    }
    FDS_HIP(hipStreamEndCapture(cap_stream, &g));
    const hipError_t e = hipGraphInstantiate(&gexec, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    FDS_HIP(e);
    graph_gen = ts_gen;
  }
  FDS_HIP(hipGraphLaunch(gexec, s));
  ++replays;
}

Engine::Engine(int m, int precision, int max_cycles, int capacity, hipStream_t stream, uint32_t flags)
    : impl_(new Impl()) {
  Impl& I = *impl_;
  if (capacity < 1) throw Error(FDS_E_INVALID_ARG, "engine capacity must be positive");
  I.ik = (flags & FDS_FLAG_INTERFACE_KRYLOV) != 0;
  if (const char* g = std::getenv("FDS_GRAPH")) I.graphs = std::string(g) != "0";
  if (const char* g = std::getenv("FDS_GRAPH_AFTER")) I.graph_after = std::max(1, std::atoi(g));
  I.m = m;
  I.precision = precision;
  I.flex = precision != FDS_FP64;   // FP32 preconditioner or none: flexible GMRES
  I.max_cycles = max_cycles;
  I.s = stream;
  I.capacity = capacity;
  I.states.alloc(sizeof(ProbState) * capacity);
  I.host_states.assign(capacity, ProbState{});
  void* fd = nullptr;
  I.flags_host = static_cast<int*>(host_mapped_alloc(sizeof(int) * capacity, &fd));
  I.flags_dev = static_cast<int*>(fd);
  std::memset(I.flags_host, 0, sizeof(int) * capacity);
  for (int i = capacity - 1; i >= 0; --i) I.free_idx.push_back(i);
}

Engine::~Engine() = default;

size_t Engine::bytes_per_problem(const fds_plan* p, int m, int precision) {
  return layout_of(p, m, precision).total + sizeof(ProbState);
}

int Engine::free_slots() const { return (int)impl_->free_idx.size(); }
int Engine::active() const { return (int)impl_->active.size(); }
void Engine::set_graphs(bool on) { impl_->graphs = on; }
double Engine::host_task_seconds() const { return impl_->t_tasks; }
int Engine::graph_replays() const { return impl_->replays; }

void Engine::admit(const std::vector<SolveRequest>& reqs, const std::vector<int>& ids,
                   const std::vector<hipEvent_t>& wait_events) {
  Impl& I = *impl_;
  if (reqs.empty()) return;
  if (I.in_flight) throw Error(FDS_E_INVALID_ARG, "admit while a cycle is in flight");
  for (hipEvent_t e : wait_events)
    if (e) FDS_HIP(hipStreamWaitEvent(I.s, e, 0));
  if ((int)reqs.size() > (int)I.free_idx.size()) throw Error(FDS_E_NOMEM, "engine has no free slot");
  const int m = I.m;
  const bool flex = I.flex;
  std::vector<Problem*> fresh;
  for (size_t r = 0; r < reqs.size(); ++r) {
    std::unique_ptr<Problem> up(new Problem());
    Problem& sl = *up;
    sl.req = reqs[r];
    sl.plan = reqs[r].plan;
    sl.id = ids.empty() ? (int)r : ids[r];
    sl.idx = I.free_idx.back();
    fds_plan* p = sl.plan;
    if (p->interface_krylov() != I.ik)
      throw Error(FDS_E_INVALID_ARG, "the plans of one engine must share the Krylov iteration");
    const SlotLayout L = layout_of(p, m, I.precision);
    sl.mem.alloc(L.total);
    I.free_idx.pop_back();
    sl.Nc = (long long)p->nx * p->ny;
    sl.Nint = p->n_internal;
    sl.P = std::max(1, div_up(sl.Nc, kVecPerBlock));
    sl.Lmax = std::max(p->nx, p->ny);
    sl.b_int = sl.mem.as<double>(L.b_int);
    sl.x_int = sl.mem.as<double>(L.x_int);
    sl.tmpd = sl.mem.as<double>(L.tmpd);
    sl.ahat = sl.mem.as<double>(L.ahat);
    sl.fp = sl.mem.as<double>(L.fp);
    sl.V = sl.mem.as<double>(L.V);
    sl.u = sl.mem.as<double>(L.u);
    sl.zbuf = flex ? nullptr : sl.mem.as<double>(L.zbuf);
    sl.lines = sl.mem.as<double>(L.lines);
    double* small = sl.mem.as<double>(L.small);
    sl.H = small;
    sl.cs = sl.H + (size_t)(m + 1) * m;
    sl.sn = sl.cs + m;
    sl.g = sl.sn + m;
    sl.y = sl.g + (m + 1);
    sl.partials = sl.mem.as<double>(L.partials);
    sl.respart = sl.mem.as<double>(L.respart);
    sl.G = sl.mem.as<double>(L.gram);
    sl.hv = sl.G + (size_t)(m + 1) * (m + 1);
    sl.zcols = sl.mem.as<double>(L.zcols);
    sl.bc = flex ? nullptr : sl.mem.as<double>(L.bc);
    sl.Z = flex ? sl.mem.as<float>(L.Z) : nullptr;
    sl.tmpf = flex ? sl.mem.as<float>(L.tmpf) : nullptr;
    if (I.ik) {
      sl.zbuf = nullptr;
      sl.bc = nullptr;
      sl.zcols = nullptr;
      sl.V = nullptr;
      sl.V0 = sl.mem.as<double>(L.V0);
      sl.Vb = sl.mem.as<double>(L.Vb);
      sl.rline = sl.mem.as<double>(L.rline);
      sl.rho = sl.mem.as<double>(L.rho);
      sl.zcol = sl.mem.as<double>(L.zcol);
      sl.zc = sl.mem.as<double>(L.zc);
      sl.ucoef = sl.mem.as<double>(L.ucoef);
      sl.uphys = sl.mem.as<double>(L.uphys);
      sl.dhat = sl.mem.as<double>(L.dhat);
      sl.xpart = sl.mem.as<double>(L.xpart);
      sl.scal = sl.mem.as<double>(L.scal);
      sl.rscale = sl.mem.as<double>(L.rscale);
      sl.Wv = sl.mem.as<double>(L.Wv);
      sl.dpart = sl.mem.as<double>(L.dpart);
      sl.cpart = sl.mem.as<double>(L.cpart);
      FDS_HIP(hipMemcpyAsync(sl.scal, sl.scal_init, sizeof(sl.scal_init), hipMemcpyHostToDevice, I.s));
    }
    sl.st = I.states.as<ProbState>() + sl.idx;
    ProbState& hs = I.host_states[sl.idx];
    hs = ProbState{};
    hs.tol = sl.req.tol;
    hs.tol_eff = sl.req.tol;
    hs.floor_coef = p->floor_coef;
    hs.vscale = 1.0;
    I.flags_host[sl.idx] = 0;
    fresh.push_back(up.get());
    I.active.push_back(std::move(up));
  }
  // initial states: one copy per run of consecutive pool indices
  std::vector<int> idx;
  for (Problem* p : fresh) idx.push_back(p->idx);
  std::sort(idx.begin(), idx.end());
  for (size_t a = 0; a < idx.size();) {
    size_t b = a + 1;
    while (b < idx.size() && idx[b] == idx[b - 1] + 1) ++b;
    FDS_HIP(hipMemcpyAsync(I.states.as<ProbState>() + idx[a], &I.host_states[idx[a]],
                           sizeof(ProbState) * (b - a), hipMemcpyHostToDevice, I.s));
    a = b;
  }
  std::unique_ptr<TaskSet> ts(new TaskSet(m, flex, I.ik));
  for (Problem* p : fresh) ts->add_problem(*p);
  ts->upload(I.s);
  I.setup_phase(*ts);
  // when the new problems are the whole set, their task lists serve the cycles
  if (fresh.size() == I.active.size()) I.set_cur(std::move(ts));
  else I.cur.reset();
}

void Engine::Impl::setup_phase(TaskSet& ts) {
  Timing::begin(5, s);
  launch_lift(0, ts.lift.dev(), ts.lift.n(), ts.lift.nblocks, s);
  Timing::end(5, s);
  if (ts.arm_fwd.n()) {
    Timing::begin(0, s);
    ts.arm_fwd.launch(0, s);
    Timing::end(0, s);
    launch_copy(ts.arm_copy.dev(), ts.arm_copy.n(), ts.arm_copy.nblocks, s);
    Timing::begin(1, s);
    ts.arm_tri.launch(s);
    Timing::end(1, s);
    Timing::begin(0, s);
    ts.arm_inv0.launch(0, s);
    Timing::end(0, s);
  }
  launch_copy(ts.setup_copy.dev(), ts.setup_copy.n(), ts.setup_copy.nblocks, s);
  launch_iface(ts.iface_fp.dev(), ts.iface_fp.n(), s);
  Timing::begin(4, s);
  ts.launch_x_lines(s);
  Timing::end(4, s);
  Timing::begin(2, s);
  launch_operator(1, ts.res_op.dev(), ts.res_op.n(), ts.res_op.nblocks, 0, s);
  Timing::end(2, s);
  if (ik) {
    launch_restart_decide(ts.kry.dev(), ts.kry.n(), 1, max_cycles, s);
    ts.ik_cycle_start(s);
  } else {
    ts.cyc_fwd.launch(0, s);   // v_0 = Q r (sine basis of the centre)
    launch_restart(ts.kry.dev(), ts.kry.n(), ts.kry.nblocks, 1, max_cycles, s);
  }
  FDS_HIP(hipGetLastError());
  read_states();
  if (Timing::on()) account_arms(ts.probs, true);
}

bool Engine::step_cycle() {
  if (!cycle_launch()) return false;
  return cycle_finish();
}

bool Engine::cycle_launch() {
  Impl& I = *impl_;
  if (I.in_flight) throw Error(FDS_E_INVALID_ARG, "a cycle is already in flight");
  bool any = false;
  for (auto& p : I.active) any |= !I.host_states[p->idx].finished;
  if (!any) return false;
  TaskSet& ts = I.current();
  I.before = I.host_states;
  // per-kernel events cannot be captured: timed cycles launch kernel by kernel
  if (I.graphs && I.cycles_on_gen >= I.graph_after && !Timing::on()) {
    I.launch_graph_cycle(ts);
  } else {
    const int tag = ++I.cycle_serial;
    for (int j = 0; j < I.m; ++j) {
      if (j >= 2) {
        // stop launching once every running problem reported the end of this
        // cycle (the finish kernel writes the tag to mapped host memory)
        bool all = true;
        const volatile int* fl = I.flags_host;
        for (auto& p : I.active)
          if (!I.before[p->idx].finished && fl[p->idx] != tag) { all = false; break; }
        if (all) break;
      }
      ts.iteration(j, I.flags_dev, tag, I.s);
    }
    ts.end_of_cycle(I.max_cycles, I.s);
  }
  ++I.cycles_on_gen;
  FDS_HIP(hipMemcpyAsync(I.host_states.data(), I.states.get(), sizeof(ProbState) * I.capacity,
                         hipMemcpyDeviceToHost, I.s));
  I.in_flight = true;
  return true;
}

bool Engine::cycle_finish() {
  Impl& I = *impl_;
  if (!I.in_flight) throw Error(FDS_E_INVALID_ARG, "no cycle in flight");
  FDS_HIP(hipStreamSynchronize(I.s));
  I.in_flight = false;
  if (Timing::on()) I.account_cycle(I.before);
  for (auto& p : I.active) if (!I.host_states[p->idx].finished) return true;
  return false;
}

std::vector<int> Engine::finished_ids() const {
  std::vector<int> out;
  for (auto& p : impl_->active)
    if (impl_->host_states[p->idx].finished) out.push_back(p->id);
  return out;
}

std::vector<std::pair<int, SolveOutcome>> Engine::retire(const std::vector<int>& ids) {
  Impl& I = *impl_;
  std::vector<std::pair<int, SolveOutcome>> res;
  if (ids.empty()) return res;
  if (I.in_flight) throw Error(FDS_E_INVALID_ARG, "retire while a cycle is in flight");
  size_t hit = 0;
  for (auto& p : I.active)
    if (std::find(ids.begin(), ids.end(), p->id) != ids.end()) ++hit;
  if (hit == 0) return res;
  std::unique_ptr<TaskSet> own;
  TaskSet* ts = nullptr;
  if (hit == I.active.size() && I.cur) {
    ts = I.cur.get();   // retiring everything: the cycle task lists cover it
  } else {
    own.reset(new TaskSet(I.m, I.flex, I.ik));
    for (auto& p : I.active)
      if (std::find(ids.begin(), ids.end(), p->id) != ids.end()) own->add_problem(*p);
    own->upload(I.s);
    ts = own.get();
  }
  std::vector<SolveOutcome> out = I.finalize_phase(*ts);
  for (size_t i = 0; i < ts->probs.size(); ++i) res.emplace_back(ts->probs[i]->id, out[i]);
  // release: the stream is idle after finalize_phase
  std::vector<std::unique_ptr<Problem>> keep;
  for (auto& p : I.active) {
    if (std::find(ids.begin(), ids.end(), p->id) != ids.end()) I.free_idx.push_back(p->idx);
    else keep.push_back(std::move(p));
  }
  I.active = std::move(keep);
  I.cur.reset();
  return res;
}

std::vector<SolveOutcome> Engine::Impl::finalize_phase(TaskSet& ts) {
  // the arms' interface rows start from b_a
  launch_copy(ts.fin_copy.dev(), ts.fin_copy.n(), ts.fin_copy.nblocks, s);
  launch_iface(ts.iface_bs.dev(), ts.iface_bs.n(), s);
  if (ts.bs_fwd0.n()) {
    launch_copy(ts.arm_copy.dev(), ts.arm_copy.n(), ts.arm_copy.nblocks, s);
    Timing::begin(0, s);
    ts.bs_fwd0.launch(0, s);
    Timing::end(0, s);
    Timing::begin(1, s);
    ts.arm_tri.launch(s);
    Timing::end(1, s);
    Timing::begin(0, s);
    ts.arm_inv.launch(0, s);
    Timing::end(0, s);
  }
  launch_lift(1, ts.gather.dev(), ts.gather.n(), ts.gather.nblocks, s);
  launch_residual(ts.resid.dev(), ts.resid.n(), ts.resid.nblocks, s);
  launch_res_sum(ts.res_sum.dev(), ts.res_sum.n(), s);
  FDS_HIP(hipGetLastError());
  read_states();
  if (Timing::on()) account_arms(ts.probs, false);
  std::vector<SolveOutcome> out(ts.probs.size());
  for (size_t i = 0; i < ts.probs.size(); ++i) {
    const Problem& sl = *ts.probs[i];
    const ProbState& st = host_states[sl.idx];
    const double rr = st.res_rr, bb = st.res_bb;
    SolveOutcome& o = out[i];
    o.res.iterations = st.iterations;
    o.res.cycles = st.cycles;
    o.res.stop_reason = st.stop_reason;
    o.res.relres_schur = st.fnorm > 0 ? st.beta / st.fnorm : 0.0;
    o.res.relres_global = bb > 0 ? std::sqrt(rr / bb) : std::sqrt(rr);
    o.res.seconds = 0;
    if (st.nonfinite) o.status = FDS_E_NONFINITE;
    else if (!st.finished) { o.status = FDS_E_NOT_CONVERGED; o.res.stop_reason = FDS_STOP_MAX_CYCLES; }
    else if (st.stop_reason == FDS_STOP_TOL || st.stop_reason == FDS_STOP_AT_FLOOR) o.status = FDS_OK;
    else o.status = FDS_E_NOT_CONVERGED;
    o.res.status = o.status;
  }
  return out;
}

void Engine::Impl::account_cycle(const std::vector<ProbState>& before) {
  const double wz = flex ? 4.0 : 8.0;     // storage of z and of the transform scratch
  for (auto& up : active) {
    const Problem& sl = *up;
    if (before[sl.idx].finished) continue;
    const double Nc = (double)sl.Nc;
    const int its = host_states[sl.idx].iterations - before[sl.idx].iterations;
    if (ik) {
      // per step: the cross sums read two source lines per axis and write
      // their sums; the dot pass reads v_0..v_j (the coordinates) and writes
      // w; the update reads w and v_0..v_j and writes v_{j+1}
      const IkGeom g = ik_geom(sl.plan);
      const double nco = 1.0 + g.nb;
      double dots = 0, upd = 0;
      for (int j = 0; j < its; ++j) {
        dots += 8.0 * (j + 2) * nco;
        upd += 8.0 * (j + 3) * nco;
      }
      Timing::add_bytes(4, its * 8.0 * (2.0 * g.nb + 4.0 * (sl.plan->nx + sl.plan->ny)));
      Timing::add_bytes(3, dots);
      Timing::add_bytes(6, upd);
      // cycle end: compose (read V0, write tz), solve (read, write), inverse
      // transform into x (read tz, read and write x), residual (read x and
      // f', write r); cycle start: extract (read r, write the interior
      // part), forward transform (read, write V0), solve (read V0, write it
      // back and tz)
      Timing::add_bytes(2, Nc * (16.0 + 24.0 + 16.0));
      Timing::add_bytes(1, Nc * (16.0 + 24.0));
      Timing::add_bytes(0, Nc * (24.0 + 16.0));
      Timing::add_bytes(7, Nc * 8.0);
      for (const ArmInfo& a : sl.plan->arms) add_line_bytes(a, 1.0);
      continue;
    }
    // per Arnoldi step (sine basis): the tridiagonal solve reads v_j, writes
    // it back normalised and writes z^ (FP64 plain, FP32 z^_j flexible); the
    // boundary columns read z^ (plain: and v_j); flexible: the dot pass also
    // applies the operator (reads z^_j, writes w).  Gram dots read
    // v_0..v_j (and w if stored), the update reads v_0..v_j (and w if
    // stored) and writes w.
    Timing::add_bytes(1, its * Nc * (8.0 + 8.0 + wz));
    if (flex) {
      Timing::add_bytes(7, its * Nc * wz);
      // the dot pass also reads z^_j (4) and writes w (8); the w it no
      // longer reads (8) is counted with the dots below
      Timing::add_bytes(3, its * Nc * 4.0);
    } else {
      Timing::add_bytes(7, its * Nc * 16.0);   // z^ and v_j row sums
    }
    // W/E line terms per step (the S/N blocks are diagonal in the sine basis)
    for (const ArmInfo& a : sl.plan->arms)
      if (a.line >= 2) add_line_bytes(a, its);
    double dots = 0, upd = 0;
    const bool lagged = gram_lag_enabled(m, flex);
    const double bnd = 2.0 * (sl.plan->nx + sl.plan->ny);   // boundary-line points
    for (int j = 0; j < its; ++j) {
      if (lagged) {
        // boundary dots read v_0..v_j and s on the lines; the update reads
        // v_0..v_j (s on the lines) and writes w
        dots += 16.0 * (j + 1) * bnd;
        upd += (8.0 * (j + 1) + 8.0) * Nc;
      } else {
        dots += (8.0 * (j + 1) + (flex ? 8.0 : 0.0)) * Nc;
        upd += (8.0 * (j + 1) + 8.0 + (flex ? 8.0 : 0.0)) * Nc;
      }
    }
    Timing::add_bytes(3, dots);
    Timing::add_bytes(6, upd);
    // end of cycle: plain variant applies A_c^{-1} to V y (transforms and
    // tridiagonal solve in FP64, accumulate into x); residual operator reads
    // x and f', writes r; line terms of x
    // inverse transform of u into x (read u, read and write x), forward
    // transform of the residual into v_0; plain: the solve on u
    Timing::add_bytes(0, Nc * (24.0 + 16.0));
    if (!flex) Timing::add_bytes(1, Nc * 16.0);
    Timing::add_bytes(2, Nc * 24.0);
    for (const ArmInfo& a : sl.plan->arms) add_line_bytes(a, 1.0);
  }
}

void Engine::Impl::account_arms(const std::vector<Problem*>& probs, bool setup_phase) {
  for (const Problem* sl : probs) {
    for (const ArmInfo& a : sl->plan->arms) {
      // one whole-arm transform and one interface-row transform per phase
      const double na = (double)a.L * a.rows;
      Timing::add_bytes(0, 16.0 * (na + a.L));
      Timing::add_bytes(1, 16.0 * na);
    }
    const double Nc = (double)sl->Nc;
    if (setup_phase) {
      Timing::add_bytes(2, Nc * 24.0);
      for (const ArmInfo& a : sl->plan->arms) add_line_bytes(a, 1.0);
    }
  }
}

std::vector<SolveOutcome> Engine::run_batch(const std::vector<SolveRequest>& reqs, int m,
                                            int precision, int max_cycles, hipStream_t stream,
                                            uint32_t flags) {
  auto t0 = std::chrono::steady_clock::now();
  Engine e(m, precision, max_cycles, (int)reqs.size(), stream, flags);
  std::vector<int> ids(reqs.size());
  for (size_t i = 0; i < reqs.size(); ++i) ids[i] = (int)i;
  e.admit(reqs, ids);
  int cyc = 0;
  while (e.step_cycle()) {
    if (++cyc > max_cycles + 2) break;
  }
  std::vector<SolveOutcome> out(reqs.size());
  for (auto& pr : e.retire(ids)) out[pr.first] = pr.second;
  const double sec = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  for (auto& o : out) o.res.seconds = sec;
  return out;
}

}  // namespace fds
