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
  std::vector<cd> uspec;         // normalised spectrum of the input wave u, sum |.|^2 = XY
  int n_aperture = 0;
  std::vector<cd> prop;          // P(k) / (XY) with the band limit [ny][nx]
  // option (ii): translate windows of wnx x wny pixels (0: none)
  int wnx = 0, wny = 0;
  std::vector<cd> wspec;         // DFT of u cropped to a window centred on it [wny][wnx]
  std::vector<cd> wprop;         // window propagator / (wnx wny), the cell's band limit [wny][wnx]
  std::vector<uint32_t> detmask; // ring bits per frequency [ny][nx]
  std::vector<int32_t> comp_flat;   // D detector pixels (flat index), sorted by (mask, kx, ky)
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

// Window tables of option (ii) (wspec, wprop) for h.lat.prop_nx x h.lat.prop_ny windows.
void build_window_tables(HostPlan& h);

}  // namespace lma

namespace lma {

// Layout of the contraction as a banded complex GEMM (the combination step of
// Fig. lma_pseudocode, eqs. lma_approximation_exit1 / exit2) for a whole scan window.
//
// Probes are taken in 4 x 4 sub-blocks (M = 16 rows of a 16x16 MFMA tile); four sub-blocks
// form an 8 x 8 super-tile handled by one workgroup. The translates the super-tile needs lie
// in a W x H rectangle of I_f (periodic). For one sub-block, the union of its probes'
// L-nearest sets is cut into K-steps of 4 translates adjacent along x within one row of the
// rectangle; A[probe][translate] holds alpha where the translate is one of that probe's
// neighbours and 0 elsewhere. The pattern is the same for every sub-block of the window up
// to a whole-translate shift when the number of coefficient sets along each axis divides 4
// (Case 1, or Case 2 with c in {2, 4}).
struct StencilPlan {
  bool ok = false;
  std::string why;             // reason when !ok
  int nks = 0;                 // K-steps per sub-block (implemented K = 4 nks)
  int W = 0, H = 0;            // translate rectangle of a super-tile
  int ox0 = 0, oy0 = 0;        // rectangle origin of super-tile (0, 0), translate index in [0, R_f)
  int tile_dx = 0, tile_dy = 0;  // rectangle shift between super-tiles (8 probes)
  int sub_dx = 0, sub_dy = 0;    // shift between sub-blocks (4 probes)
  int tiles_x = 0, tiles_y = 0;  // super-tiles covering the window
  std::vector<int32_t> ks_off;   // [nks] rectangle index (row * W + col) of each step's first translate
  std::vector<std::complex<float>> a;  // [nks][64] A fragment: lane l holds A[l % 16][4 ks + l / 16]
};

// Builds the banded-GEMM layout for the plan's window; ok = false (with a reason) when the
// window does not have the shift-invariant structure, the rectangle exceeds max_rect
// translates or the sub-block needs more than max_ks K-steps.
void build_stencil(const HostPlan& h, int max_ks, int max_rect, StencilPlan* sp);

}  // namespace lma

namespace lma {

// Partition of the scan window into rectangles P_1..P_l under a residency budget of M
// propagated translates (Sec. 4.2.4, rectangle strategy). Every rectangle but those clipped
// at the window's right and bottom edges has the same size w x h: the widest (up to the
// window width) whose row-major tiling keeps every part's translate set I_{f,P_j,L} within M
// translates, and at that width the tallest. Parts are taken row-major; translates shared by
// consecutive parts stay resident, so the number of multislice runs is
// T = sum_j |I_{f,P_j,L}| - sum_j |I_{f,P_j,L} cap I_{f,P_{j+1},L}|.
struct PartPlan {
  struct Part {
    int a0 = 0, b0 = 0, w = 0, h = 0;        // probes, relative to the window origin
    std::vector<int32_t> translates;         // I_{f,P_j,L}, increasing
    std::vector<int32_t> fresh;              // translates not resident from the previous part
    std::vector<int32_t> fresh_slot;         // resident row each of them is written to
    std::vector<int32_t> row_of;             // [Rfy*Rfx] -> resident row while this part is formed, or -1
  };
  int64_t max_rows = 0;          // M
  int w = 0, h = 0;              // rectangle size
  int64_t slots = 0;             // resident rows needed: max_j |I_{f,P_j,L}|
  int64_t multislice_calls = 0;  // T
  std::vector<Part> parts;
};

// The L-nearest translates of window probe (a, b) (window-relative), appended to out.
void probe_translates(const HostPlan& h, int a, int b, std::vector<int32_t>* out);

// Rectangle partition of the window for at most max_rows resident translates. Returns false
// (with a reason) when even one probe needs more than max_rows.
bool build_partition(const HostPlan& h, int64_t max_rows, PartPlan* pp, std::string* why);

}  // namespace lma

namespace lma {
// Sets the calling thread's lma_last_error message.
void set_last_error(const std::string& msg);
}  // namespace lma
