// Launchers of the gfx950 kernels (host-callable, implemented in kernels.hip).
#pragma once
#include <hip/hip_runtime.h>
#include <cstdint>

namespace lma {
namespace dev {

// Device tables of a plan (all device pointers). Tables read by column passes are stored
// transposed, [kx][ky].
struct Tables {
  int nx = 0, ny = 0;
  int tw = 0;                        // tile width of the wave layout (0: tile_width(nx, ny))
  int64_t Qx = 1, Qy = 1;            // lattice units per cell (wave positions are in units)
  const float2* specT = nullptr;     // probe spectrum / (XY)          [nx][ny]
  const float2* propT = nullptr;     // propagator * band limit / (XY) [nx][ny]
  const float2* twx = nullptr;       // exp(-2 pi i t / nx)            [nx]
  const float2* twy = nullptr;       // exp(-2 pi i t / ny)            [ny]
  const int32_t* compT = nullptr;    // frequency -> detector pixel or -1 [nx][ny]
  const uint32_t* maskT = nullptr;   // ring bits per frequency        [nx][ny]
  // kx columns [zc0, zc1) are zero after every column pass: the band-limited propagator
  // vanishes on all of them and they hold no detector pixel. Column passes skip the tile
  // columns inside the range; row passes write only the others, and read only the others
  // when their input comes from a column pass.
  int zc0 = 0, zc1 = 0;
  // kx columns [ic0, ic1) where the spectrum the initial waves start from (specT) vanishes for
  // every ky: the initial-wave pass skips their tile columns and the first row pass does not
  // read them
  int ic0 = 0, ic1 = 0;
  // the propagator (with its band limit) vanishes at ky positions [3 ny/8, 5 ny/8) of every
  // column: column transforms of 512 or 64 points skip forming those outputs and treat them
  // as zeros on the way back
  int prop_z34 = 0;
  // radix schedule of the transforms (0: base order; 1: its last stage first; 2: its first
  // stage last; -1: each length's own default); lengths built with one schedule ignore it
  int sched = -1;
};

struct Contraction {
  const void* basis = nullptr;       // [rows][D] float2, or 4 x bf16 (hi_re, lo_re, hi_im, lo_im)
  int split_bf16 = 0;
  int D = 0;
  const int32_t* row_of = nullptr;   // [Rfy*Rfx] -> resident row
  const int32_t* set_dx = nullptr;   // [nsets][L]
  const int32_t* set_dy = nullptr;   // [nsets][L]
  const float2* alpha = nullptr;     // [nsets][L]
  int L = 0, Rfx = 0, Rfy = 0, ncls_x = 1, ncls_y = 1, stepx = 0, stepy = 0;
  int wa0 = 0, wb0 = 0, ww = 0, wh = 0;
  const int32_t* chunk_start = nullptr;
  const int32_t* chunk_len = nullptr;
  const uint32_t* chunk_mask = nullptr;
  int nchunks = 0;
  int ndet = 0;
  double scale = 1.0;                // XY (exit spectra are stored divided by XY)
  double* img = nullptr;             // [ndet][wh][ww]
  const int32_t* probe_list = nullptr;  // optional subset of window probes (index b*ww + a)
  int n_list = 0;
  // instead of the ring sums (at most one of them):
  float* patterns = nullptr;         // 4-D STEM: [probe][D] |psi_hat|^2 / (XY)
  const int32_t* bin_of = nullptr;   // 3-D STEM: annulus of each detector pixel, or -1
  int nbins = 0;
  double* radial = nullptr;          // 3-D STEM: [nbins][probe] annulus sums of |psi_hat|^2 / (XY)
};

// The contraction of a whole window as a banded complex GEMM on MFMA (layout built on the host
// by build_stencil): one workgroup per (8 x 8-probe super-tile, detector-pixel chunk).
struct Stencil {
  const void* basis = nullptr;       // as in Contraction
  int split_bf16 = 0;
  int D = 0;
  const int32_t* row_of = nullptr;
  int Rfx = 0, Rfy = 0;
  int nks = 0;                       // K-steps per 4 x 4 sub-block
  int W = 0, H = 0;                  // translate rectangle of a super-tile
  int ox0 = 0, oy0 = 0, tile_dx = 0, tile_dy = 0, sub_dx = 0, sub_dy = 0;
  int tiles_x = 0, tiles_y = 0;      // super-tiles of the launch: tile_x0 + [0, tiles_x) x tile_y0 + [0, tiles_y)
  int tile_x0 = 0, tile_y0 = 0;
  const int32_t* ks_off = nullptr;   // [nks]
  const float2* a = nullptr;         // [nks][64] A fragments
  int ww = 0, wh = 0;
  int pa0 = 0, pa1 = 0, pb0 = 0, pb1 = 0;  // probes [pa0, pa1) x [pb0, pb1) of the window are
                                           // added to the image; the others are not formed
  const int32_t* chunk_start = nullptr;
  const int32_t* chunk_len = nullptr;
  const uint32_t* chunk_mask = nullptr;
  int nchunks = 0;
  int ndet = 0;
  double scale = 1.0;
  double* img = nullptr;             // [ndet][wh][ww]
  const float2* zeros = nullptr;     // 16 zero bytes (copies of absent rows and pixels)
  // split-BF16 basis: A fragments of the bf16 MFMA, [ceil(nks/4)][64] x 32 bytes (see
  // k_contract_bf16); null: the FP32 MFMA on converted values
  const void* abf = nullptr;
};
// largest K-step count and translate rectangle the MFMA contraction accepts
constexpr int kStencilMaxKs = 96;
constexpr int kStencilMaxRect = 1152;

bool supported(int nx, int ny);

hipError_t transmission(const float* v, float2* t, int64_t n, double sigma, hipStream_t s);
// A wave batch is stored [B][ny/TW][nx/TW][TW][TW] (TW x TW tiles, TW = tile_width) and every
// pass updates it in place. Between passes a wave is in the mixed domain (y spatial, x frequency).
int tile_width(int nx, int ny);
// forces the tile width (4, 8 or 16; anything else restores the default), a tuning knob
void set_tile_width(int tw);
// whether the passes are built for this grid with tile width tw
bool tile_width_ok(int nx, int ny, int tw);
// radix schedules the passes of this grid are built with at tile width tw (1 or 3)
int radix_schedules(int nx, int ny, int tw);
// initial waves u(. - pos_w): column IFFT of spectrum * modulation
hipError_t init_waves(const Tables& T, float2* work, const int64_t* wave_u, int B, hipStream_t s);
// row pass of slice j: row IFFT, * t_j, row FFT
// after_column: the waves come from a column pass (every slice but the first), so their
// zero kx columns (the band gap) need not be read; otherwise they come from init_waves and
// the columns of the input spectrum's gap (ic0, ic1) are not read
hipError_t row_pass(const Tables& T, float2* work, const float2* trans_j, int B, bool after_column, hipStream_t s);
// row pass of slice j over the waves of several specimens of one grid (their column passes
// share T): wave w multiplies by spec_trans[wave_spec[w]] + slice_off (each specimen's t_j)
hipError_t row_pass_specimens(const Tables& T, float2* work, const float2* const* spec_trans, const int32_t* wave_spec,
                              int64_t slice_off, int B, bool after_column, hipStream_t s);
// row pass of slice j for waves propagated on windows (Tw: the window's tables): row IFFT,
// * t_j of the cell at each wave's window (origin: its position in pixels minus half the
// window), row FFT; with last, no row FFT (the window's wave is left in real space)
hipError_t row_pass_window(const Tables& Tw, float2* work, const float2* trans_j, int cell_nx, int cell_ny,
                           const int64_t* wave_u, int64_t Qx, int64_t Qy, bool last, bool after_column, int B,
                           hipStream_t s);
// places each window's real-space wave in the cell (zero elsewhere) and row-transforms it
// on the cell's grid (T: the cell's tables, work: the cell's wave batch)
hipError_t embed_windows(const Tables& T, float2* work, const Tables& Tw, const float2* win, const int64_t* wave_u,
                         int B, hipStream_t s);
// column pass of a middle slice: column FFT, * P, column IFFT
hipError_t col_pass(const Tables& T, float2* work, int B, hipStream_t s);
// last column pass, LMA: column FFT, * P, keep the detector pixels as basis rows
hipError_t col_gather(const Tables& T, float2* work, int B, void* basis, int D, const int32_t* wave_row,
                      int split_bf16, hipStream_t s);
// last column pass, plain: column FFT, * P, ring sums of |.|^2 added to img[r][wave_out[w]]
hipError_t col_reduce(const Tables& T, float2* work, int B, const int32_t* wave_out, double* img, int ndet,
                      int64_t img_stride, double scale, hipStream_t s);
// probe-coefficient contraction and detector reduction (ring sums, or the 4-D / 3-D outputs)
hipError_t contract(const Contraction& c, hipStream_t s);
// largest annulus count of the 3-D output
constexpr int kMaxRadialBins = 512;
// out[i] = scale * |in[i]|^2 as float, n values
hipError_t intensity(const float2* in, float* out, int64_t n, double scale, hipStream_t s);
// the same contraction for a whole window on MFMA
hipError_t contract_stencil(const Stencil& c, hipStream_t s);
// out[0..n) = 0 by a kernel (no memset node when a caller captures the stream)
hipError_t fill_zero(double* out, int64_t n, hipStream_t s);
// out = (acc ? out : 0) + w * img, n doubles, device memory
hipError_t scale_out(double* out, const double* img, int64_t n, double w, int acc, hipStream_t s);

}  // namespace dev
}  // namespace lma
