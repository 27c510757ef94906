// Plan creation: geometry validation, classification of the coupled block
// and the independent arms (paper Section 2.4, last paragraph), internal
// layout and shared tables.
#include <algorithm>
#include <cmath>
#include <string>

#include "runtime.h"

namespace fds {

int line_of_kind(int kind) {
  switch (kind) {
    case RK_S: return 0;
    case RK_N: return 1;
    case RK_W: return 2;
    case RK_E: return 3;
    default: return -1;
  }
}

static bool share_edge(const fds_rect& a, const fds_rect& b) {
  if (a.i1 == b.i0 || a.i0 == b.i1) return std::min(a.j1, b.j1) - std::max(a.j0, b.j0) > 0;
  if (a.j1 == b.j0 || a.j0 == b.j1) return std::min(a.i1, b.i1) - std::max(a.i0, b.i0) > 0;
  return false;
}

static bool interiors_overlap(const fds_rect& a, const fds_rect& b) {
  return std::min(a.i1, b.i1) > std::max(a.i0, b.i0) && std::min(a.j1, b.j1) > std::max(a.j0, b.j0);
}

fds_plan* create_plan(const fds_rect* rects, int nrect, double h, double kappa,
                      const fds_options* opt) {
  if (!rects || nrect < 1 || nrect > kMaxRects) throw Error(FDS_E_INVALID_ARG, "need 1..64 rectangles");
  if (!(h > 0.0) || !std::isfinite(h)) throw Error(FDS_E_INVALID_ARG, "h must be positive");
  if (!std::isfinite(kappa)) throw Error(FDS_E_INVALID_ARG, "kappa must be finite");
  fds_options o{30, 200, FDS_FP64, 0};
  if (opt) o = *opt;
  if (o.restart_m < 1 || o.restart_m > 120) throw Error(FDS_E_INVALID_ARG, "restart_m must be in 1..120");
  if (o.max_cycles < 1) throw Error(FDS_E_INVALID_ARG, "max_cycles must be >= 1");
  if (o.precision != FDS_FP64 && o.precision != FDS_FP32_PRECOND && o.precision != FDS_NO_PRECOND &&
      o.precision != FDS_JACOBI)
    throw Error(FDS_E_INVALID_ARG, "unknown precision");
  if (o.flags & ~(uint32_t)FDS_FLAG_INTERFACE_KRYLOV) throw Error(FDS_E_INVALID_ARG, "unknown option flags");
  if ((o.flags & FDS_FLAG_INTERFACE_KRYLOV) && o.precision != FDS_FP64)
    throw Error(FDS_E_INVALID_ARG, "the interface Krylov iteration is an FP64 method");
  for (int r = 0; r < nrect; ++r) {
    const fds_rect& a = rects[r];
    if (a.i0 < 0 || a.j0 < 0 || a.i1 - a.i0 < 2 || a.j1 - a.j0 < 2)
      throw Error(FDS_E_GEOMETRY, "rectangle " + std::to_string(r) + " has no interior node");
    if ((long long)(a.i1 - a.i0 + 1) * (a.j1 - a.j0 + 1) > (1LL << 31))
      throw Error(FDS_E_INVALID_ARG, "rectangle too large");
  }
  for (int a = 0; a < nrect; ++a)
    for (int b = a + 1; b < nrect; ++b)
      if (interiors_overlap(rects[a], rects[b])) throw Error(FDS_E_GEOMETRY, "rectangles overlap");

  std::vector<int> deg(nrect, 0);
  for (int a = 0; a < nrect; ++a)
    for (int b = 0; b < nrect; ++b)
      if (a != b && share_edge(rects[a], rects[b])) deg[a]++;
  // Coupled subdomains: every rectangle sharing edges with two or more others;
  // without one, the first of those with the most neighbours.  Several coupled
  // rectangles must form a straight chain of equal width, which is solved as
  // one coupled block (their union with the lines between them).
  std::vector<int> chain;
  for (int r = 0; r < nrect; ++r)
    if (deg[r] >= 2) chain.push_back(r);
  if (chain.empty()) chain.push_back((int)(std::max_element(deg.begin(), deg.end()) - deg.begin()));
  fds_rect M = rects[chain[0]];
  const int K = (int)chain.size();
  if (K > 1) {
    bool same_i = true, same_j = true;
    for (int r : chain) {
      same_i = same_i && rects[r].i0 == M.i0 && rects[r].i1 == M.i1;
      same_j = same_j && rects[r].j0 == M.j0 && rects[r].j1 == M.j1;
    }
    if (!same_i && !same_j)
      throw Error(FDS_E_GEOMETRY, "the coupled rectangles (those sharing edges with two or more others) "
                                  "must form a straight chain of equal width");
    const bool vert = same_i;
    std::sort(chain.begin(), chain.end(), [&](int a, int b) {
      return vert ? rects[a].j0 < rects[b].j0 : rects[a].i0 < rects[b].i0;
    });
    for (int t = 1; t < K; ++t) {
      const fds_rect& lo = rects[chain[t - 1]];
      const fds_rect& hi = rects[chain[t]];
      if (vert ? hi.j0 != lo.j1 : hi.i0 != lo.i1)
        throw Error(FDS_E_GEOMETRY, "the coupled rectangles must follow each other along the chain");
    }
    M = rects[chain[0]];
    const fds_rect& last = rects[chain[K - 1]];
    if (vert) M.j1 = last.j1;
    else M.i1 = last.i1;
  }
  std::vector<char> is_coupled(nrect, 0);
  for (int r : chain) is_coupled[r] = 1;

  auto* p = new fds_plan();
  try {
    FDS_HIP(hipGetDevice(&p->device));
    p->rects.assign(rects, rects + nrect);
    p->h = h;
    p->delta = 1.0 / (h * h);
    p->kappa = kappa;
    p->opt = o;
    p->nx = M.i1 - M.i0 - 1;
    p->ny = M.j1 - M.j0 - 1;
    if ((long long)p->nx * p->ny > (1LL << 31)) throw Error(FDS_E_INVALID_ARG, "coupled block too large");
    p->kind.assign(nrect, RK_CENTRE);
    int used_lines = 0;
    std::vector<int> arm_on_line(4, -1);
    for (int r = 0; r < nrect; ++r) {
      if (is_coupled[r]) continue;
      const fds_rect& a = rects[r];
      int kind = -1;
      if (a.j0 == M.j1 && a.i0 == M.i0 && a.i1 == M.i1) kind = RK_N;
      else if (a.j1 == M.j0 && a.i0 == M.i0 && a.i1 == M.i1) kind = RK_S;
      else if (a.i0 == M.i1 && a.j0 == M.j0 && a.j1 == M.j1) kind = RK_E;
      else if (a.i1 == M.i0 && a.j0 == M.j0 && a.j1 == M.j1) kind = RK_W;
      if (kind < 0)
        throw Error(FDS_E_GEOMETRY, "rectangle " + std::to_string(r) +
                                        " does not share a full side of the coupled rectangle");
      const int line = line_of_kind(kind);
      if (used_lines & (1 << line)) throw Error(FDS_E_GEOMETRY, "two rectangles on one side");
      used_lines |= 1 << line;
      arm_on_line[line] = r;
      for (int b = 0; b < nrect; ++b)
        if (b != r && !is_coupled[b] && share_edge(a, rects[b]))
          throw Error(FDS_E_GEOMETRY, "rectangle " + std::to_string(r) + " touches two others");
      p->kind[r] = kind;
    }

    // ---- internal layout: the coupled block first (row-major over the
    // interior of M), then the arms in user order
    const long long nx = p->nx, ny = p->ny;
    p->rd.resize(nrect);
    long long off = nx * ny, uoff = 0, boff = 0;
    std::vector<long long> ioff(nrect, 0);
    for (int r = 0; r < nrect; ++r) {
      if (is_coupled[r]) continue;
      const fds_rect& a = rects[r];
      const long long rows = (p->kind[r] == RK_N || p->kind[r] == RK_S) ? a.j1 - a.j0 : a.i1 - a.i0;
      const long long cols = (p->kind[r] == RK_N || p->kind[r] == RK_S) ? a.i1 - a.i0 - 1 : a.j1 - a.j0 - 1;
      ioff[r] = off;
      off += rows * cols;
    }
    p->n_internal = off;
    // does another rectangle share (part of) side s of a (1: i=i0, 2: i=i1, 4: j=j0, 8: j=j1)?
    auto shared_sides = [&](int r) {
      const fds_rect& a = rects[r];
      int m = 0;
      for (int b = 0; b < nrect; ++b) {
        if (b == r) continue;
        const fds_rect& q = rects[b];
        const bool jo = std::min(a.j1, q.j1) - std::max(a.j0, q.j0) > 0;
        const bool io = std::min(a.i1, q.i1) - std::max(a.i0, q.i0) > 0;
        if (q.i1 == a.i0 && jo) m |= 1;
        if (q.i0 == a.i1 && jo) m |= 2;
        if (q.j1 == a.j0 && io) m |= 4;
        if (q.j0 == a.j1 && io) m |= 8;
      }
      return m;
    };
    // position of each coupled rectangle along the chain
    std::vector<int> pos(nrect, -1);
    for (int t = 0; t < K; ++t) pos[chain[t]] = t;
    const bool vert = K > 1 && rects[chain[0]].i0 == M.i0 && rects[chain[0]].i1 == M.i1 &&
                      rects[chain[1]].j0 == rects[chain[0]].j1;
    p->user_off.resize(nrect + 1);
    p->bc_off.resize(nrect + 1);
    for (int r = 0; r < nrect; ++r) {
      const fds_rect& a = rects[r];
      RectDev d{};
      d.bi0 = a.i0; d.bj0 = a.j0; d.bi1 = a.i1; d.bj1 = a.j1;
      for (int s = 0; s < 4; ++s) { d.halo_off[s] = -1; d.halo_stride[s] = 0; }
      const int k = p->kind[r];
      switch (k) {
        case RK_CENTRE: {
          // owned nodes: the interior, plus the line shared with a chain
          // neighbour listed after this rectangle
          int ilo = a.i0 + 1, ihi = a.i1 - 1, jlo = a.j0 + 1, jhi = a.j1 - 1;
          const int t = pos[r];
          const bool own_lo = t > 0 && r < chain[t - 1];
          const bool own_hi = t < K - 1 && r < chain[t + 1];
          if (vert) { if (own_lo) jlo = a.j0; if (own_hi) jhi = a.j1; }
          else { if (own_lo) ilo = a.i0; if (own_hi) ihi = a.i1; }
          d.rows = jhi - jlo + 1; d.cols = ihi - ilo + 1;
          d.off = (long long)(jlo - M.j0 - 1) * nx + (ilo - M.i0 - 1);
          d.ld = nx;
          d.ai = ilo; d.ar = 0; d.ac = 1; d.aj = jlo; d.br = 1; d.bcc = 0;
          d.ilo = ilo; d.jlo = jlo; d.uwidth = d.cols;
          d.iface_mask = shared_sides(r);
          // neighbour lines: inside the coupled block, or an arm's interface
          // line (indexed along the side of M), or Dirichlet
          auto arm_line = [&](int line, long long along) {
            const int q = arm_on_line[line];
            return q < 0 ? -1LL : ioff[q] + along;
          };
          if (jlo - 1 > M.j0) { d.halo_off[0] = d.off - nx; d.halo_stride[0] = 1; }
          else { d.halo_off[0] = arm_line(0, ilo - M.i0 - 1); d.halo_stride[0] = 1; }
          if (jhi + 1 < M.j1) { d.halo_off[1] = d.off + (long long)d.rows * nx; d.halo_stride[1] = 1; }
          else { d.halo_off[1] = arm_line(1, ilo - M.i0 - 1); d.halo_stride[1] = 1; }
          if (ilo - 1 > M.i0) { d.halo_off[2] = d.off - 1; d.halo_stride[2] = nx; }
          else { d.halo_off[2] = arm_line(2, jlo - M.j0 - 1); d.halo_stride[2] = 1; }
          if (ihi + 1 < M.i1) { d.halo_off[3] = d.off + d.cols; d.halo_stride[3] = nx; }
          else { d.halo_off[3] = arm_line(3, jlo - M.j0 - 1); d.halo_stride[3] = 1; }
          for (int s = 0; s < 4; ++s)
            if (d.halo_off[s] < 0) d.halo_stride[s] = 0;
          break;
        }
        case RK_N:
          d.rows = a.j1 - a.j0; d.cols = a.i1 - a.i0 - 1;
          d.ai = a.i0 + 1; d.ar = 0; d.ac = 1; d.aj = a.j0; d.br = 1; d.bcc = 0;
          d.ilo = a.i0 + 1; d.jlo = a.j0; d.uwidth = d.cols; d.iface_mask = 4;
          d.halo_off[0] = (ny - 1) * nx; d.halo_stride[0] = 1;
          break;
        case RK_S:
          d.rows = a.j1 - a.j0; d.cols = a.i1 - a.i0 - 1;
          d.ai = a.i0 + 1; d.ar = 0; d.ac = 1; d.aj = a.j1; d.br = -1; d.bcc = 0;
          d.ilo = a.i0 + 1; d.jlo = a.j0 + 1; d.uwidth = d.cols; d.iface_mask = 8;
          d.halo_off[0] = 0; d.halo_stride[0] = 1;
          break;
        case RK_E:
          d.rows = a.i1 - a.i0; d.cols = a.j1 - a.j0 - 1;
          d.ai = a.i0; d.ar = 1; d.ac = 0; d.aj = a.j0 + 1; d.br = 0; d.bcc = 1;
          d.ilo = a.i0; d.jlo = a.j0 + 1; d.uwidth = d.rows; d.iface_mask = 1;
          d.halo_off[0] = nx - 1; d.halo_stride[0] = nx;
          break;
        case RK_W:
          d.rows = a.i1 - a.i0; d.cols = a.j1 - a.j0 - 1;
          d.ai = a.i1; d.ar = -1; d.ac = 0; d.aj = a.j0 + 1; d.br = 0; d.bcc = 1;
          d.ilo = a.i0 + 1; d.jlo = a.j0 + 1; d.uwidth = d.rows; d.iface_mask = 2;
          d.halo_off[0] = 0; d.halo_stride[0] = nx;
          break;
      }
      if (k != RK_CENTRE) { d.off = ioff[r]; d.ld = d.cols; }
      d.user_off = uoff;
      d.bc_off = boff;
      p->user_off[r] = uoff;
      p->bc_off[r] = boff;
      uoff += (long long)d.rows * d.cols;
      boff += (long long)(a.i1 - a.i0 + 1) * (a.j1 - a.j0 + 1);
      p->rd[r] = d;
    }
    p->user_off[nrect] = uoff;
    p->bc_off[nrect] = boff;
    p->n_unknowns = uoff;
    p->bc_total = boff;
    // the coupled block as one rectangle (offset 0 of the internal layout)
    {
      RectDev& cd = p->cdev;
      cd = RectDev{};
      cd.rows = (int)ny; cd.cols = (int)nx; cd.off = 0; cd.ld = nx;
      cd.bi0 = M.i0; cd.bj0 = M.j0; cd.bi1 = M.i1; cd.bj1 = M.j1;
      for (int s = 0; s < 4; ++s) { cd.halo_off[s] = -1; cd.halo_stride[s] = 0; }
    }

    // ---- tables; kappa > 0: singular subdomain check first
    auto check_singular = [&](long long rows, long long cols) {
      if (kappa <= 0.0) return;
      const double pi = 3.14159265358979323846;
      double best = 1e300;
      for (long long k = 1; k <= cols; ++k) {
        const double lx = p->delta * (2.0 * std::cos(k * pi / (cols + 1)) - 2.0);
        for (long long l = 1; l <= rows; ++l) {
          const double ly = p->delta * (2.0 * std::cos(l * pi / (rows + 1)) - 2.0);
          best = std::min(best, std::fabs(lx + ly + kappa));
        }
      }
      if (best <= 64.0 * 1.1102230246251565e-16 * 8.0 * p->delta)
        throw Error(FDS_E_SINGULAR, "a subdomain operator is singular for this kappa");
    };
    check_singular(p->ny, p->nx);
    for (int r = 0; r < nrect; ++r)
      if (p->kind[r] != RK_CENTRE) check_singular(p->rd[r].rows, p->rd[r].cols);

    TableCache& tc = TableCache::get();
    p->fft_c = tc.fft(p->nx);
    // settle the transform variants now (the autotuner measures on first use)
    for (int len : {p->nx, p->ny}) {
      (void)dst_choice(len, false);
      (void)dst_choice(len, true);
    }
    p->modes_c = tc.modes(p->nx, p->ny, h, kappa);
    p->modes_cu = tc.modes(p->nx, p->ny, h, kappa, true);
    if (p->opt.flags & FDS_FLAG_INTERFACE_KRYLOV) {
      // lines of the arms present (x lines S/N have nx nodes, y lines ny)
      long long lines = 0;
      for (int r = 0; r < nrect; ++r)
        if (p->kind[r] != RK_CENTRE) lines += line_of_kind(p->kind[r]) < 2 ? p->nx : p->ny;
      if (p->nx < 2 || p->ny < 2 || 1 + lines > kIkMaxCoords) p->opt.flags &= ~(uint32_t)FDS_FLAG_INTERFACE_KRYLOV;
      else p->ik = build_ik_table(p->nx, p->ny, h, kappa);
    }
    const bool dense_ops = !p->interface_krylov();   // the line operators of the other paths
    for (int r = 0; r < nrect; ++r) {
      if (p->kind[r] == RK_CENTRE) continue;
      ArmInfo ai{};
      ai.rect = r;
      ai.kind = p->kind[r];
      ai.line = line_of_kind(ai.kind);
      ai.L = p->rd[r].cols;
      ai.rows = p->rd[r].rows;
      ai.fft = tc.fft(ai.L);
      ai.modes = tc.modes(ai.L, ai.rows, h, kappa);
      ai.gs = tc.gs(ai.L, ai.rows, h, kappa, dense_ops);
      p->arms.push_back(ai);
    }
    p->floor_coef = 1.1102230246251565e-16 * (9.0 * p->delta + std::fabs(kappa));
    if (p->opt.precision == FDS_JACOBI) p->jacobi = build_jacobi_table(p);
  } catch (...) {
    delete p;
    throw;
  }
  return p;
}

}  // namespace fds

size_t fds_plan::footprint(int m, int precision) const {
  return fds::Engine::bytes_per_problem(this, m, precision);
}
