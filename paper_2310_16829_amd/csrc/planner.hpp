// Host planner of an LMA simulation: everything before the first kernel launch, FP64.
#pragma once
#include <complex>
#include <cstdint>
#include <string>
#include <vector>

#include "lma.h"

namespace lma {

using cd = std::complex<double>;

constexpr int kMaxDet = 8;

struct HostPlan {
  lma_optics op{};
  lma_lattice lat{};
  int ndet = 0;
  std::vector<double> det_inner, det_outer;

  // ---- lattices (Sec. 4.2.1): positions in integer units of l/Q along each axis -------
  int Rfx = 0, Rfy = 0;          // I_f size
  int64_t Qx = 0, Qy = 0;        // units per cell
  int64_t oxu = 0, oyu = 0;      // I_offset in units
  int64_t stepPx = 0, stepPy = 0;  // probe spacing in units
  int64_t stepTx = 0, stepTy = 0;  // I_f spacing in units
  int gx = 0, gy = 0;            // gcd(P, R_f) per axis
  int ncls_x = 0, ncls_y = 0;    // coefficient sets per axis
  int nsets = 0;

  // ---- probe, propagator, detectors ------------------------------------------------------
  std::vector<cd> spec;          // normalised probe spectrum [ny][nx], sum |.|^2 = XY
  int n_aperture = 0;
  std::vector<cd> prop;          // P(k) / (XY) with the band limit [ny][nx]
  std::vector<uint32_t> detmask; // ring bits per frequency [ny][nx]
  std::vector<int32_t> comp_flat;   // D detector pixels, sorted by (mask, flat index)
  std::vector<uint32_t> comp_mask;  // [D]
  std::vector<int32_t> comp_map;    // [ny][nx] -> compacted index or -1
  std::vector<int32_t> chunk_start; // chunks of compacted pixels with one ring mask
  std::vector<int32_t> chunk_len;
  std::vector<uint32_t> chunk_mask;

  // ---- coefficient sets (Sec. 4.2.2) -----------------------------------------------------
  std::vector<int32_t> set_nbr;  // [nsets][L] translate index t = b*Rfx + a of each neighbour
  std::vector<int32_t> set_dx, set_dy;  // [nsets][L] neighbour index offset from the set's base
  std::vector<cd> alpha;         // [nsets][L]
  std::vector<double> residual;  // [nsets] relative LSQ residual

  // ---- window and resident rows ------------------------------------------------------------
  int wa0 = 0, wb0 = 0, ww = 0, wh = 0;
  std::vector<int32_t> rows;     // translate index of each resident row, increasing
  std::vector<int32_t> row_of;   // [Rfy*Rfx] -> row or -1

  int64_t n_translates() const { return (int64_t)Rfx * Rfy; }
  int64_t n_probes() const { return (int64_t)ww * wh; }
  int D() const { return (int)comp_flat.size(); }
  // probe (a, b) -> coefficient set and index shift of its neighbours
  void probe_set(int a, int b, int* set, int* sx, int* sy) const;
  // fractional position (pos / l) of translate t and of probe (a, b)
  void translate_frac(int t, double* fx, double* fy) const;
  void probe_frac(int a, int b, double* fx, double* fy) const;
};

// Validates the arguments and builds every host table. Returns LMA_OK or an error with a
// message in *err.
lma_status build_host_plan(const lma_optics* op, const lma_lattice* lat, const lma_detectors* det,
                           HostPlan* hp, std::string* err);

// Validation and sizes only (no tables): used by lma_footprint.
lma_status check_arguments(const lma_optics* op, const lma_lattice* lat, const lma_detectors* det,
                           std::string* err);

// Relativistic constants.
void electron_constants(double kv, double* lambda, double* sigma);

}  // namespace lma
