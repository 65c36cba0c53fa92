// Banded-GEMM layout of the probe contraction for a scan window. FP64 positions in exact
// integer lattice units; alpha rounded to FP32 once, as in the per-pixel contraction.
#include <algorithm>
#include <map>
#include <numeric>
#include <tuple>

#include "planner.hpp"

namespace lma {

namespace {

// minimum-image offset in [-Q/2, Q/2)
inline int64_t wrap_offset(int64_t d, int64_t Q) {
  const int64_t h = Q / 2;
  int64_t r = ((d + h) % Q + Q) % Q;
  return r - h;
}

inline int pos_mod(int64_t v, int64_t m) { return (int)(((v % m) + m) % m); }

}  // namespace

void build_stencil(const HostPlan& h, int max_ks, int max_rect, StencilPlan* sp) {
  *sp = StencilPlan();
  const int Px = h.lat.px, Py = h.lat.py, L = h.lat.L;
  if (4 % h.ncls_x != 0 || 4 % h.ncls_y != 0) {
    sp->why = "coefficient sets per axis do not divide 4";
    return;
  }
  if ((4 * (int64_t)h.Rfx) % Px != 0 || (4 * (int64_t)h.Rfy) % Py != 0) {
    sp->why = "4 probes are not a whole number of translates";
    return;
  }
  sp->sub_dx = (int)(4 * (int64_t)h.Rfx / Px);
  sp->sub_dy = (int)(4 * (int64_t)h.Rfy / Py);
  sp->tile_dx = 2 * sp->sub_dx;
  sp->tile_dy = 2 * sp->sub_dy;

  // unwrapped translate coordinates of every neighbour of the 16 probes of sub-block (0, 0):
  // X = (p - d - offset) / spacing, with d the minimum-image offset probe - translate, so X is
  // congruent to the translate's index modulo R_f and lies next to the probe
  struct Entry { int m; int64_t X, Y; std::complex<double> alpha; };
  std::vector<Entry> ent;
  ent.reserve((size_t)16 * L);
  int64_t Xmin = INT64_MAX, Ymin = INT64_MAX, Xmax = INT64_MIN, Ymax = INT64_MIN;
  for (int m = 0; m < 16; ++m) {
    const int a = h.wa0 + (m & 3), b = h.wb0 + (m >> 2);
    int s, shx, shy;
    h.probe_set(a, b, &s, &shx, &shy);
    const int64_t pxu = (int64_t)a * h.stepPx, pyu = (int64_t)b * h.stepPy;
    for (int j = 0; j < L; ++j) {
      const int ta = (h.set_dx[(size_t)s * L + j] + shx) % h.Rfx;
      const int tb = (h.set_dy[(size_t)s * L + j] + shy) % h.Rfy;
      const int64_t txu = ((int64_t)ta * h.stepTx + h.oxu) % h.Qx;
      const int64_t tyu = ((int64_t)tb * h.stepTy + h.oyu) % h.Qy;
      const int64_t dx = wrap_offset(pxu % h.Qx - txu, h.Qx);
      const int64_t dy = wrap_offset(pyu % h.Qy - tyu, h.Qy);
      const int64_t nx = pxu - dx - h.oxu, ny = pyu - dy - h.oyu;
      if (nx % h.stepTx != 0 || ny % h.stepTy != 0) {
        sp->why = "translate position off the lattice";
        return;
      }
      const int64_t X = nx / h.stepTx, Y = ny / h.stepTy;
      if (pos_mod(X, h.Rfx) != ta || pos_mod(Y, h.Rfy) != tb) {
        sp->why = "unwrapped translate does not match its index";
        return;
      }
      ent.push_back({m, X, Y, h.alpha[(size_t)s * L + j]});
      Xmin = std::min(Xmin, X); Xmax = std::max(Xmax, X);
      Ymin = std::min(Ymin, Y); Ymax = std::max(Ymax, Y);
    }
  }
  // K-steps: per row of the union, runs of 4 translates from the row's leftmost one
  std::map<int64_t, std::pair<int64_t, int64_t>> span;   // Y -> (xs, xe)
  for (const Entry& e : ent) {
    auto it = span.find(e.Y);
    if (it == span.end()) span[e.Y] = {e.X, e.X};
    else { it->second.first = std::min(it->second.first, e.X); it->second.second = std::max(it->second.second, e.X); }
  }
  std::vector<std::pair<int64_t, int64_t>> steps;       // (Y, x0)
  int64_t xend = Xmax;
  for (const auto& kv : span) {
    const int64_t xs = kv.second.first, xe = kv.second.second;
    for (int64_t x0 = xs; x0 <= xe; x0 += 4) {
      steps.push_back({kv.first, x0});
      xend = std::max(xend, x0 + 3);
    }
  }
  sp->nks = (int)steps.size();
  sp->W = (int)(xend - Xmin + 1) + sp->sub_dx;
  sp->H = (int)(Ymax - Ymin + 1) + sp->sub_dy;
  if (sp->nks > max_ks) {
    sp->why = "sub-block needs more K-steps than the kernel holds in registers";
    return;
  }
  if ((int64_t)sp->W * sp->H > max_rect) {
    sp->why = "translate rectangle does not fit the workgroup's LDS";
    return;
  }
  sp->ox0 = pos_mod(Xmin, h.Rfx);
  sp->oy0 = pos_mod(Ymin, h.Rfy);
  sp->tiles_x = (h.ww + 7) / 8;
  sp->tiles_y = (h.wh + 7) / 8;
  std::map<std::tuple<int, int64_t, int64_t>, std::complex<double>> at;
  for (const Entry& e : ent) {
    auto key = std::make_tuple(e.m, e.X, e.Y);
    if (at.count(key)) {
      sp->why = "a probe reaches one translate twice";
      return;
    }
    at[key] = e.alpha;
  }
  sp->ks_off.resize(sp->nks);
  sp->a.assign((size_t)sp->nks * 64, std::complex<float>(0.f, 0.f));
  size_t placed = 0;
  for (int ks = 0; ks < sp->nks; ++ks) {
    const int64_t Y = steps[ks].first, x0 = steps[ks].second;
    sp->ks_off[ks] = (int)((Y - Ymin) * sp->W + (x0 - Xmin));
    for (int l = 0; l < 64; ++l) {
      auto it = at.find(std::make_tuple(l % 16, x0 + l / 16, Y));
      if (it != at.end()) {
        sp->a[(size_t)ks * 64 + l] = std::complex<float>((float)it->second.real(), (float)it->second.imag());
        ++placed;
      }
    }
  }
  if (placed != ent.size()) {
    sp->why = "K-steps do not cover every neighbour";
    return;
  }
  sp->ok = true;
}

}  // namespace lma
