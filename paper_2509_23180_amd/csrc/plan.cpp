// Plan creation: geometry validation, classification of the coupled centre
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
  if (!rects || nrect < 1 || nrect > 1 + kMaxArms) throw Error(FDS_E_INVALID_ARG, "need 1..5 rectangles");
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
  const int c = (int)(std::max_element(deg.begin(), deg.end()) - deg.begin());
  const fds_rect C = rects[c];

  auto* p = new fds_plan();
  try {
    FDS_HIP(hipGetDevice(&p->device));
    p->rects.assign(rects, rects + nrect);
    p->centre = c;
    p->h = h;
    p->delta = 1.0 / (h * h);
    p->kappa = kappa;
    p->opt = o;
    p->nx = C.i1 - C.i0 - 1;
    p->ny = C.j1 - C.j0 - 1;
    p->kind.assign(nrect, RK_CENTRE);
    int used_lines = 0;
    for (int r = 0; r < nrect; ++r) {
      if (r == c) continue;
      const fds_rect& a = rects[r];
      int kind = -1;
      if (a.j0 == C.j1 && a.i0 == C.i0 && a.i1 == C.i1) kind = RK_N;
      else if (a.j1 == C.j0 && a.i0 == C.i0 && a.i1 == C.i1) kind = RK_S;
      else if (a.i0 == C.i1 && a.j0 == C.j0 && a.j1 == C.j1) kind = RK_E;
      else if (a.i1 == C.i0 && a.j0 == C.j0 && a.j1 == C.j1) kind = RK_W;
      if (kind < 0)
        throw Error(FDS_E_GEOMETRY, "rectangle " + std::to_string(r) +
                                        " does not share a full side of the coupled rectangle");
      const int line = line_of_kind(kind);
      if (used_lines & (1 << line)) throw Error(FDS_E_GEOMETRY, "two rectangles on one side");
      used_lines |= 1 << line;
      for (int b = 0; b < nrect; ++b)
        if (b != r && b != c && share_edge(a, rects[b]))
          throw Error(FDS_E_GEOMETRY, "several coupled subdomains are not supported");
      p->kind[r] = kind;
    }

    // ---- internal layout: centre first, then the arms in user order
    p->rd.resize(nrect);
    long long off = 0, uoff = 0, boff = 0;
    std::vector<int> order;
    order.push_back(c);
    for (int r = 0; r < nrect; ++r)
      if (r != c) order.push_back(r);
    std::vector<long long> ioff(nrect);
    for (int r : order) {
      const fds_rect& a = rects[r];
      long long rows, cols;
      if (p->kind[r] == RK_CENTRE) { rows = a.j1 - a.j0 - 1; cols = a.i1 - a.i0 - 1; }
      else if (p->kind[r] == RK_N || p->kind[r] == RK_S) { rows = a.j1 - a.j0; cols = a.i1 - a.i0 - 1; }
      else { rows = a.i1 - a.i0; cols = a.j1 - a.j0 - 1; }
      ioff[r] = off;
      off += rows * cols;
    }
    p->n_internal = off;
    p->user_off.resize(nrect + 1);
    p->bc_off.resize(nrect + 1);
    for (int r = 0; r < nrect; ++r) {
      const fds_rect& a = rects[r];
      RectDev d{};
      d.off = ioff[r];
      d.bi0 = a.i0; d.bj0 = a.j0; d.bi1 = a.i1; d.bj1 = a.j1;
      for (int s = 0; s < 4; ++s) { d.halo_off[s] = -1; d.halo_stride[s] = 0; }
      const int k = p->kind[r];
      switch (k) {
        case RK_CENTRE:
          d.rows = a.j1 - a.j0 - 1; d.cols = a.i1 - a.i0 - 1;
          d.ai = a.i0 + 1; d.ar = 0; d.ac = 1; d.aj = a.j0 + 1; d.br = 1; d.bcc = 0;
          d.ilo = a.i0 + 1; d.jlo = a.j0 + 1; d.uwidth = d.cols;
          break;
        case RK_N:
          d.rows = a.j1 - a.j0; d.cols = a.i1 - a.i0 - 1;
          d.ai = a.i0 + 1; d.ar = 0; d.ac = 1; d.aj = a.j0; d.br = 1; d.bcc = 0;
          d.ilo = a.i0 + 1; d.jlo = a.j0; d.uwidth = d.cols; d.iface_mask = 4;
          break;
        case RK_S:
          d.rows = a.j1 - a.j0; d.cols = a.i1 - a.i0 - 1;
          d.ai = a.i0 + 1; d.ar = 0; d.ac = 1; d.aj = a.j1; d.br = -1; d.bcc = 0;
          d.ilo = a.i0 + 1; d.jlo = a.j0 + 1; d.uwidth = d.cols; d.iface_mask = 8;
          break;
        case RK_E:
          d.rows = a.i1 - a.i0; d.cols = a.j1 - a.j0 - 1;
          d.ai = a.i0; d.ar = 1; d.ac = 0; d.aj = a.j0 + 1; d.br = 0; d.bcc = 1;
          d.ilo = a.i0; d.jlo = a.j0 + 1; d.uwidth = d.rows; d.iface_mask = 1;
          break;
        case RK_W:
          d.rows = a.i1 - a.i0; d.cols = a.j1 - a.j0 - 1;
          d.ai = a.i1; d.ar = -1; d.ac = 0; d.aj = a.j0 + 1; d.br = 0; d.bcc = 1;
          d.ilo = a.i0 + 1; d.jlo = a.j0 + 1; d.uwidth = d.rows; d.iface_mask = 2;
          break;
      }
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

    // halos between the centre and its arms (composite residual)
    RectDev& cd = p->rd[c];
    const long long nx = p->nx, ny = p->ny;
    for (int r = 0; r < nrect; ++r) {
      if (r == c) continue;
      RectDev& ad = p->rd[r];
      const int line = line_of_kind(p->kind[r]);
      long long start = 0, stride = 1;
      switch (line) {
        case 0: start = 0; stride = 1; cd.iface_mask |= 4; cd.halo_off[0] = ad.off; cd.halo_stride[0] = 1; break;
        case 1: start = (ny - 1) * nx; stride = 1; cd.iface_mask |= 8; cd.halo_off[1] = ad.off; cd.halo_stride[1] = 1; break;
        case 2: start = 0; stride = nx; cd.iface_mask |= 1; cd.halo_off[2] = ad.off; cd.halo_stride[2] = 1; break;
        case 3: start = nx - 1; stride = nx; cd.iface_mask |= 2; cd.halo_off[3] = ad.off; cd.halo_stride[3] = 1; break;
      }
      ad.halo_off[0] = cd.off + start;
      ad.halo_stride[0] = stride;
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
    for (int r = 0; r < nrect; ++r) check_singular(p->rd[r].rows, p->rd[r].cols);

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
        if (r != c) lines += line_of_kind(p->kind[r]) < 2 ? p->nx : p->ny;
      if (p->nx < 2 || p->ny < 2 || 1 + lines > kIkMaxCoords) p->opt.flags &= ~(uint32_t)FDS_FLAG_INTERFACE_KRYLOV;
      else p->ik = build_ik_table(p->nx, p->ny, h, kappa);
    }
    const bool dense_ops = !p->interface_krylov();   // the line operators of the other paths
    for (int r = 0; r < nrect; ++r) {
      if (r == c) continue;
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
