// Rectangle partition of the scan window under a residency budget (Sec. 4.2.4).
#include <algorithm>
#include <numeric>

#include "planner.hpp"

namespace lma {

void probe_translates(const HostPlan& h, int a, int b, std::vector<int32_t>* out) {
  int s, shx, shy;
  h.probe_set(h.wa0 + a, h.wb0 + b, &s, &shx, &shy);
  const int L = h.lat.L;
  for (int j = 0; j < L; ++j) {
    const int ta = (h.set_dx[(size_t)s * L + j] + shx) % h.Rfx;
    const int tb = (h.set_dy[(size_t)s * L + j] + shy) % h.Rfy;
    out->push_back(tb * h.Rfx + ta);
  }
}

namespace {

// I_{f,S,L} of the rectangle of probes [a0, a0 + w) x [b0, b0 + h), increasing
std::vector<int32_t> rect_translates(const HostPlan& h, int a0, int b0, int w, int hh, std::vector<uint8_t>* mark) {
  std::vector<int32_t> nb, out;
  nb.reserve(h.lat.L);
  for (int b = b0; b < b0 + hh; ++b)
    for (int a = a0; a < a0 + w; ++a) {
      nb.clear();
      probe_translates(h, a, b, &nb);
      for (int32_t t : nb)
        if (!(*mark)[t]) {
          (*mark)[t] = 1;
          out.push_back(t);
        }
    }
  for (int32_t t : out) (*mark)[t] = 0;
  std::sort(out.begin(), out.end());
  return out;
}

}  // namespace

bool build_partition(const HostPlan& h, int64_t max_rows, PartPlan* pp, std::string* why) {
  *pp = PartPlan();
  pp->max_rows = max_rows;
  std::vector<uint8_t> mark((size_t)h.n_translates(), 0);
  // every part of the row-major tiling by w x hh rectangles (edge ones clipped) needs at most
  // max_rows translates
  auto fits = [&](int w, int hh) {
    for (int b0 = 0; b0 < h.wh; b0 += hh)
      for (int a0 = 0; a0 < h.ww; a0 += w)
        if ((int64_t)rect_translates(h, a0, b0, std::min(w, h.ww - a0), std::min(hh, h.wh - b0), &mark).size() >
            max_rows)
          return false;
    return true;
  };
  // the widest rectangles first, then the tallest at that width. A tiling that fits at some
  // height fits at height 1 (each one-row part lies inside a part of the taller tiling), so the
  // widest usable width is the widest whose one-row tiling fits.
  int bw = 0, bh = 0;
  for (int w = h.ww; w >= 1 && bw == 0; --w)
    if (fits(w, 1)) bw = w;
  if (bw == 0) {
    *why = "the residency budget holds fewer translates than one probe needs";
    return false;
  }
  for (int hh = h.wh; hh >= 1; --hh)
    if (fits(bw, hh)) {
      bh = hh;
      break;
    }
  pp->w = bw;
  pp->h = bh;
  const int64_t NT = h.n_translates();
  std::vector<int32_t> slot_of((size_t)NT, -1);
  std::vector<int32_t> prev;
  std::vector<int32_t> free_slots;
  for (int b0 = 0; b0 < h.wh; b0 += bh)
    for (int a0 = 0; a0 < h.ww; a0 += bw) {
      PartPlan::Part p;
      p.a0 = a0;
      p.b0 = b0;
      p.w = std::min(bw, h.ww - a0);
      p.h = std::min(bh, h.wh - b0);
      p.translates = rect_translates(h, a0, b0, p.w, p.h, &mark);
      pp->slots = std::max<int64_t>(pp->slots, (int64_t)p.translates.size());
      pp->parts.push_back(std::move(p));
    }
  // resident rows: translates shared with the previous part keep their row
  for (int32_t s = (int32_t)pp->slots - 1; s >= 0; --s) free_slots.push_back(s);
  for (PartPlan::Part& p : pp->parts) {
    std::vector<int32_t> gone;
    std::set_difference(prev.begin(), prev.end(), p.translates.begin(), p.translates.end(), std::back_inserter(gone));
    for (int32_t t : gone) {
      free_slots.push_back(slot_of[t]);
      slot_of[t] = -1;
    }
    for (int32_t t : p.translates)
      if (slot_of[t] < 0) {
        slot_of[t] = free_slots.back();
        free_slots.pop_back();
        p.fresh.push_back(t);
        p.fresh_slot.push_back(slot_of[t]);
      }
    p.row_of.assign((size_t)NT, -1);
    for (int32_t t : p.translates) p.row_of[t] = slot_of[t];
    pp->multislice_calls += (int64_t)p.fresh.size();
    prev = p.translates;
  }
  return true;
}

}  // namespace lma
