// Host planner: argument validation, probe spectrum, propagator, detector pixel list,
// input-wave lattice, nearest translates and least-squares coefficients. FP64.
#include "planner.hpp"

#include <algorithm>
#include <cmath>
#include <cstring>
#include <numeric>

#include "lsq.hpp"

namespace lma {

namespace {

constexpr double kPi = 3.14159265358979323846;
constexpr double kHcEvA = 12398.4198;   // h c, eV * Angstrom
constexpr double kM0c2Ev = 510998.95;   // electron rest energy, eV
constexpr int kChunk = 256;             // detector pixels per contraction chunk

bool pow2_in(int n, int lo, int hi) { return n >= lo && n <= hi && (n & (n - 1)) == 0; }
// grid sides the slice passes are built for: powers of two, and 96, 192, 384 (3 x 2^a) and
// 640 (5 x 2^7)
bool grid_side_ok(int n) { return pow2_in(n, 16, 2048) || n == 96 || n == 192 || n == 384 || n == 640; }

// spatial frequency index in FFT order
inline int freq_index(int m, int n) { return m < (n + 1) / 2 ? m : m - n; }

int64_t lcm64(int64_t a, int64_t b) { return a / std::gcd(a, b) * b; }

// minimum-image offset in [-Q/2, Q/2)
inline int64_t min_image(int64_t d, int64_t Q) {
  int64_t h = Q / 2;
  int64_t r = ((d + h) % Q + Q) % Q;
  return r - h;
}

bool finite(double x) { return std::isfinite(x); }

}  // namespace

// Window tables of option (ii): the input wave cropped to a wnx x wny window centred on it,
// u_W(x') = u(x' - (wnx/2, wny/2)) with u = IDFT(uspec) / (XY) on the cell, is evaluated at the
// window's pixels by separable sums over the non-zero part of the spectrum, then transformed
// by the window's DFT; the window propagator keeps the cell's band limit (same pixel size).
void build_window_tables(HostPlan& h) {
  const int nx = h.op.nx, ny = h.op.ny, wx = h.lat.prop_nx, wy = h.lat.prop_ny;
  h.wnx = wx;
  h.wny = wy;
  // exp(sign 2 pi i t / n) for t < n, FP64
  auto table = [](int n, double sign) {
    std::vector<cd> t(n);
    for (int i = 0; i < n; ++i) {
      const double a = sign * 2.0 * kPi * (double)i / (double)n;
      t[i] = cd(std::cos(a), std::sin(a));
    }
    return t;
  };
  auto wrap = [](int64_t v, int64_t n) { return (size_t)(((v % n) + n) % n); };
  const std::vector<cd> ex = table(nx, 1.0), ey = table(ny, 1.0), fx = table(wx, -1.0), fy = table(wy, -1.0);
  double umax = 0.0;
  for (const cd& u : h.uspec) umax = std::max(umax, std::abs(u));
  // A[ky][x'] = sum_kx uspec[ky][kx] exp(2 pi i kx (x' - wx/2) / nx)
  std::vector<cd> A((size_t)ny * wx, cd(0.0));
  for (int my = 0; my < ny; ++my)
    for (int mx = 0; mx < nx; ++mx) {
      const cd s = h.uspec[(size_t)my * nx + mx];
      if (std::abs(s) <= 1e-18 * umax) continue;
      const int64_t kx = freq_index(mx, nx);
      for (int x = 0; x < wx; ++x) A[(size_t)my * wx + x] += s * ex[wrap(kx * (x - wx / 2), nx)];
    }
  // u_W[y'][x'] = sum_ky A[ky][x'] exp(2 pi i ky (y' - wy/2) / ny) / (XY)
  std::vector<cd> uw((size_t)wy * wx, cd(0.0));
  const double inv = 1.0 / ((double)nx * ny);
  for (int my = 0; my < ny; ++my) {
    const int64_t ky = freq_index(my, ny);
    for (int y = 0; y < wy; ++y) {
      const cd e = ey[wrap(ky * (y - wy / 2), ny)] * inv;
      for (int x = 0; x < wx; ++x) uw[(size_t)y * wx + x] += A[(size_t)my * wx + x] * e;
    }
  }
  // window DFT, rows then columns
  std::vector<cd> tmp((size_t)wy * wx, cd(0.0));
  for (int y = 0; y < wy; ++y)
    for (int q = 0; q < wx; ++q) {
      cd acc(0.0);
      for (int x = 0; x < wx; ++x) acc += uw[(size_t)y * wx + x] * fx[((size_t)q * x) % wx];
      tmp[(size_t)y * wx + q] = acc;
    }
  h.wspec.assign((size_t)wy * wx, cd(0.0));
  for (int q = 0; q < wy; ++q)
    for (int x = 0; x < wx; ++x) {
      cd acc(0.0);
      for (int y = 0; y < wy; ++y) acc += tmp[(size_t)y * wx + x] * fy[((size_t)q * y) % wy];
      h.wspec[(size_t)q * wx + x] = acc;
    }
  // propagator on the window's frequencies, the cell's band radius
  const double kbw = h.op.bandlimit * std::min(nx / (2.0 * h.op.lx), ny / (2.0 * h.op.ly));
  const double lwx = h.op.lx * wx / nx, lwy = h.op.ly * wy / ny;
  h.wprop.assign((size_t)wy * wx, cd(0.0));
  for (int my = 0; my < wy; ++my) {
    const double ky = (double)freq_index(my, wy) / lwy;
    for (int mx = 0; mx < wx; ++mx) {
      const double kx = (double)freq_index(mx, wx) / lwx;
      const double k2 = kx * kx + ky * ky;
      if (k2 < kbw * kbw) {
        const double ph = -kPi * h.op.wavelength * h.op.dz * k2;
        h.wprop[(size_t)my * wx + mx] = cd(std::cos(ph), std::sin(ph)) / ((double)wx * wy);
      }
    }
  }
}

void electron_constants(double kv, double* lambda, double* sigma) {
  double ev = kv * 1e3;
  double lam = kHcEvA / std::sqrt(ev * (2.0 * kM0c2Ev + ev));
  if (lambda) *lambda = lam;
  if (sigma) *sigma = 2.0 * kPi / (lam * ev) * (kM0c2Ev + ev) / (2.0 * kM0c2Ev + ev);
}

lma_status check_arguments(const lma_optics* op, const lma_lattice* lat, const lma_detectors* det,
                           std::string* err) {
  if (!op || !lat || !det) { *err = "null argument"; return LMA_ERR_ARG; }
  if (!grid_side_ok(op->nx) || !grid_side_ok(op->ny)) {
    *err = "nx and ny must be powers of two in [16, 2048] or one of 96, 192, 384, 640";
    return LMA_ERR_UNSUPPORTED;
  }
  if (!(op->lx > 0) || !(op->ly > 0) || !finite(op->lx) || !finite(op->ly)) { *err = "cell size must be positive"; return LMA_ERR_ARG; }
  if (!(op->wavelength > 0) || !finite(op->wavelength)) { *err = "wavelength must be positive"; return LMA_ERR_ARG; }
  if (!finite(op->sigma)) { *err = "sigma must be finite"; return LMA_ERR_ARG; }
  if (!(op->dz > 0) || !finite(op->dz)) { *err = "dz must be positive"; return LMA_ERR_ARG; }
  if (!(op->bandlimit > 0) || !(op->bandlimit <= 1.0)) { *err = "bandlimit must be in (0, 1]"; return LMA_ERR_ARG; }
  if (!(op->alpha_max > 0) || !finite(op->alpha_max)) { *err = "alpha_max must be positive"; return LMA_ERR_ARG; }
  if (!finite(op->defocus) || !finite(op->cs)) { *err = "defocus and cs must be finite"; return LMA_ERR_ARG; }
  if (lat->px < 1 || lat->py < 1 || lat->px > (1 << 20) || lat->py > (1 << 20)) { *err = "scan size out of range"; return LMA_ERR_ARG; }
  if (lat->rx < 1 || lat->ry < 1 || lat->rx > (1 << 20) || lat->ry > (1 << 20)) { *err = "input-wave lattice size out of range"; return LMA_ERR_ARG; }
  if (lat->f < 1 || lat->rx % lat->f || lat->ry % lat->f) { *err = "f must be >= 1 and divide rx and ry"; return LMA_ERR_ARG; }
  int rfx = lat->rx / lat->f, rfy = lat->ry / lat->f;
  if ((lat->px % rfx && rfx % lat->px) || (lat->py % rfy && rfy % lat->py)) {
    *err = "probe and input-wave lattices incompatible: along each axis one of P and R/f must divide the other";
    return LMA_ERR_ARG;
  }
  if ((int64_t)rfx * rfy > (int64_t)1 << 28) { *err = "too many translates"; return LMA_ERR_UNSUPPORTED; }
  if (lat->L < 1 || (int64_t)lat->L > (int64_t)rfx * rfy) { *err = "L must be in [1, |I_f|]"; return LMA_ERR_ARG; }
  if (lat->L > 2048) { *err = "L above 2048"; return LMA_ERR_UNSUPPORTED; }
  if (lat->basis_kind != LMA_BASIS_PROBE && lat->basis_kind != LMA_BASIS_GAUSSIAN &&
      lat->basis_kind != LMA_BASIS_TRIGPOLY) {
    *err = "unknown input wave kind";
    return LMA_ERR_UNSUPPORTED;
  }
  if (lat->basis_kind == LMA_BASIS_TRIGPOLY &&
      (rfx % 2 == 0 || rfy % 2 == 0 || rfx > op->nx || rfy > op->ny)) {
    *err = "the trigonometric input wave needs an odd number of translates per axis (2n + 1), at most the grid side";
    return LMA_ERR_ARG;
  }
  if (!std::isfinite(lat->basis_param) || lat->basis_param < 0.0) { *err = "basis_param must be >= 0"; return LMA_ERR_ARG; }
  if (lat->prop_nx != 0 || lat->prop_ny != 0) {
    if (!grid_side_ok(lat->prop_nx) || !grid_side_ok(lat->prop_ny) || lat->prop_nx > op->nx || lat->prop_ny > op->ny) {
      *err = "translate window sides must be grid sides (powers of two from 16, or 96, 192, 384, 640) within the grid";
      return LMA_ERR_UNSUPPORTED;
    }
  }
  if (lat->precision != LMA_GEMM_FP32 && lat->precision != LMA_GEMM_SPLIT_BF16) { *err = "unknown precision"; return LMA_ERR_ARG; }
  const int32_t* w = lat->window;
  bool whole = w[0] == 0 && w[1] == 0 && w[2] == 0 && w[3] == 0;
  if (!whole && (w[0] < 0 || w[1] < 0 || w[2] < 1 || w[3] < 1 || w[0] + w[2] > lat->px || w[1] + w[3] > lat->py)) {
    *err = "scan window outside the scan";
    return LMA_ERR_ARG;
  }
  if (lat->batch < 0 || lat->hbm_budget_bytes < 0) { *err = "batch and budget must be >= 0"; return LMA_ERR_ARG; }
  if (!finite(lat->offset_x) || !finite(lat->offset_y)) { *err = "offset must be finite"; return LMA_ERR_ARG; }
  for (int ax = 0; ax < 2; ++ax) {
    int64_t P = ax ? lat->py : lat->px, R = ax ? lat->ry : lat->rx;
    int64_t Q = 2 * lcm64(P, R);
    double off = (ax ? lat->offset_y : lat->offset_x) * (double)(Q / R);
    if (std::fabs(off - std::nearbyint(off)) > 1e-9) {
      *err = "offset must be a multiple of 1/(2 lcm(P, R)) of the cell";
      return LMA_ERR_ARG;
    }
  }
  if (det->n < 1 || det->n > kMaxDet || !det->inner || !det->outer) { *err = "1 to 8 detectors required"; return LMA_ERR_ARG; }
  for (int r = 0; r < det->n; ++r) {
    if (!(det->inner[r] >= 0) || !(det->outer[r] > det->inner[r]) || !finite(det->outer[r])) {
      *err = "detector angles must satisfy 0 <= inner < outer";
      return LMA_ERR_ARG;
    }
  }
  return LMA_OK;
}

void HostPlan::probe_set(int a, int b, int* set, int* sx, int* sy) const {
  int cx = a % ncls_x, cy = b % ncls_y;
  *set = cy * ncls_x + cx;
  *sx = (a / ncls_x) * (Rfx / gx);
  *sy = (b / ncls_y) * (Rfy / gy);
}

void HostPlan::translate_frac(int t, double* fx, double* fy) const {
  int ta = t % Rfx, tb = t / Rfx;
  *fx = (double)((ta * stepTx + oxu) % Qx) / (double)Qx;
  *fy = (double)((tb * stepTy + oyu) % Qy) / (double)Qy;
}

void HostPlan::probe_frac(int a, int b, double* fx, double* fy) const {
  *fx = (double)(a * stepPx % Qx) / (double)Qx;
  *fy = (double)(b * stepPy % Qy) / (double)Qy;
}

lma_status build_host_plan(const lma_optics* op, const lma_lattice* lat, const lma_detectors* det,
                           HostPlan* hp, std::string* err) {
  lma_status st = check_arguments(op, lat, det, err);
  if (st != LMA_OK) return st;
  HostPlan& h = *hp;
  h.op = *op;
  h.lat = *lat;
  h.ndet = det->n;
  h.det_inner.assign(det->inner, det->inner + det->n);
  h.det_outer.assign(det->outer, det->outer + det->n);
  const int nx = op->nx, ny = op->ny;
  const double XY = (double)nx * ny;
  const double lam = op->wavelength;

  // ---- probe spectrum, propagator, ring masks (eqs. probe_wave_function, aberration_function,
  //      aperture_function; Fresnel propagator of Sec. 3.2 in Fourier space) ---------------------
  h.spec.assign((size_t)nx * ny, cd(0.0));
  h.prop.assign((size_t)nx * ny, cd(0.0));
  h.detmask.assign((size_t)nx * ny, 0u);
  const double kbw = op->bandlimit * std::min(nx / (2.0 * op->lx), ny / (2.0 * op->ly));
  const double kbw2 = kbw * kbw;
  const double amax2 = op->alpha_max * op->alpha_max;
  int nap = 0;
  for (int my = 0; my < ny; ++my) {
    double ky = (double)freq_index(my, ny) / op->ly;
    for (int mx = 0; mx < nx; ++mx) {
      double kx = (double)freq_index(mx, nx) / op->lx;
      double k2 = kx * kx + ky * ky;
      double t2 = (lam * lam) * k2;
      size_t i = (size_t)my * nx + mx;
      if (t2 < amax2) {
        double chi = 0.5 * kPi * op->cs * (lam * lam * lam) * k2 * k2 - kPi * op->defocus * lam * k2;
        h.spec[i] = cd(std::cos(chi), -std::sin(chi));
        ++nap;
      }
      bool band = k2 < kbw2;
      if (band) {
        double ph = -kPi * lam * op->dz * k2;
        h.prop[i] = cd(std::cos(ph), std::sin(ph)) / XY;
        uint32_t m = 0;
        for (int r = 0; r < h.ndet; ++r) {
          double lo = h.det_inner[r], hi = h.det_outer[r];
          if (t2 >= lo * lo && t2 < hi * hi) m |= 1u << r;
        }
        h.detmask[i] = m;
      }
    }
  }
  if (nap == 0) { *err = "the aperture contains no grid frequency"; return LMA_ERR_ARG; }
  h.n_aperture = nap;
  const double norm = std::sqrt(XY / nap);
  for (auto& s : h.spec) s *= norm;

  // ---- input wave u (Sec. 4.2.3) ----------------------------------------------------------------
  if (lat->basis_kind == LMA_BASIS_GAUSSIAN) {
    // g_sigma sampled on the grid: its DFT is the continuous transform, a Gaussian
    // exp(-2 pi^2 sigma^2 |k|^2) up to a constant, as long as sigma is well above the pixel
    // and well below the cell (aliasing and wrap-around below 1e-30 for the paper's sigma)
    const double sg = lat->basis_param > 0.0 ? lat->basis_param : lam / (2.0 * op->alpha_max);
    h.uspec.assign((size_t)nx * ny, cd(0.0));
    double s2 = 0.0;
    for (int my = 0; my < ny; ++my) {
      const double ky = (double)freq_index(my, ny) / op->ly;
      for (int mx = 0; mx < nx; ++mx) {
        const double kx = (double)freq_index(mx, nx) / op->lx;
        const double g = std::exp(-2.0 * kPi * kPi * sg * sg * (kx * kx + ky * ky));
        h.uspec[(size_t)my * nx + mx] = cd(g, 0.0);
        s2 += g * g;
      }
    }
    const double un = std::sqrt(XY / s2);
    for (auto& u : h.uspec) u *= un;
  } else if (lat->basis_kind == LMA_BASIS_TRIGPOLY) {
    // u = phi_nx(2 pi x / lx) phi_ny(2 pi y / ly) with phi_n(t) = sum_{|k| <= n} e^{ikt}
    // cos(k pi / (2n + 2)) (eq. rauhut), the cell as its period and 2n + 1 translates per axis:
    // its DFT holds the weights at the grid frequencies |m| <= n and nothing else
    const int nxd = (lat->rx / lat->f - 1) / 2, nyd = (lat->ry / lat->f - 1) / 2;
    h.uspec.assign((size_t)nx * ny, cd(0.0));
    double s2 = 0.0;
    for (int my = 0; my < ny; ++my) {
      const int ky = freq_index(my, ny);
      if (std::abs(ky) > nyd) continue;
      for (int mx = 0; mx < nx; ++mx) {
        const int kx = freq_index(mx, nx);
        if (std::abs(kx) > nxd) continue;
        const double g = std::cos(kx * kPi / (2.0 * nxd + 2.0)) * std::cos(ky * kPi / (2.0 * nyd + 2.0));
        h.uspec[(size_t)my * nx + mx] = cd(g, 0.0);
        s2 += g * g;
      }
    }
    const double un = std::sqrt(XY / s2);
    for (auto& u : h.uspec) u *= un;
  } else {
    h.uspec = h.spec;
  }

  // ---- detector pixel list: sorted by (ring mask, kx, ky), cut into uniform chunks -----------
  // Within one ring mask the pixels of a kx column are consecutive, so the last column pass,
  // whose lanes hold consecutive ky of one kx, writes runs of neighbouring basis entries.
  std::vector<int32_t> pix;
  for (int x = 0; x < nx; ++x)
    for (int y = 0; y < ny; ++y)
      if (h.detmask[(size_t)y * nx + x]) pix.push_back(y * nx + x);
  if (pix.empty()) { *err = "no detector pixel lies inside the band limit"; return LMA_ERR_ARG; }
  std::stable_sort(pix.begin(), pix.end(), [&](int32_t a, int32_t b) { return h.detmask[a] < h.detmask[b]; });
  h.comp_flat = pix;
  h.comp_mask.resize(pix.size());
  h.comp_map.assign((size_t)nx * ny, -1);
  for (size_t d = 0; d < pix.size(); ++d) {
    h.comp_mask[d] = h.detmask[pix[d]];
    h.comp_map[pix[d]] = (int32_t)d;
  }
  h.chunk_start.clear(); h.chunk_len.clear(); h.chunk_mask.clear();
  for (size_t d = 0; d < pix.size();) {
    size_t e = d;
    while (e < pix.size() && h.comp_mask[e] == h.comp_mask[d] && e - d < (size_t)kChunk) ++e;
    h.chunk_start.push_back((int32_t)d);
    h.chunk_len.push_back((int32_t)(e - d));
    h.chunk_mask.push_back(h.comp_mask[d]);
    d = e;
  }

  // ---- lattices in exact integer units (Sec. 4.2.1) --------------------------------------------
  h.Rfx = lat->rx / lat->f;
  h.Rfy = lat->ry / lat->f;
  h.Qx = 2 * lcm64(lat->px, lat->rx);
  h.Qy = 2 * lcm64(lat->py, lat->ry);
  h.stepPx = h.Qx / lat->px;
  h.stepPy = h.Qy / lat->py;
  h.stepTx = (h.Qx / lat->rx) * lat->f;
  h.stepTy = (h.Qy / lat->ry) * lat->f;
  h.oxu = ((int64_t)std::llround(lat->offset_x * (double)(h.Qx / lat->rx)) % h.Qx + h.Qx) % h.Qx;
  h.oyu = ((int64_t)std::llround(lat->offset_y * (double)(h.Qy / lat->ry)) % h.Qy + h.Qy) % h.Qy;
  h.gx = std::gcd(lat->px, h.Rfx);
  h.gy = std::gcd(lat->py, h.Rfy);
  h.ncls_x = lat->px / h.gx;
  h.ncls_y = lat->py / h.gy;
  h.nsets = h.ncls_x * h.ncls_y;

  // ---- option (ii): translate windows ----------------------------------------------------------
  if (lat->prop_nx > 0) {
    // translates on pixels: every position in units times the grid size is a multiple of Q
    if ((h.stepTx * nx) % h.Qx || (h.oxu * nx) % h.Qx || (h.stepTy * ny) % h.Qy || (h.oyu * ny) % h.Qy) {
      *err = "windowed propagation needs translates on pixels";
      return LMA_ERR_ARG;
    }
    build_window_tables(h);
  }

  // squared distance in exact integers when the units are square (l_x/Q_x == l_y/Q_y exactly)
  double p1 = op->lx * (double)h.Qy, e1 = std::fma(op->lx, (double)h.Qy, -p1);
  double p2 = op->ly * (double)h.Qx, e2 = std::fma(op->ly, (double)h.Qx, -p2);
  const bool square = (p1 == p2 && e1 == e2);
  const long double ux = (long double)op->lx / (long double)h.Qx;
  const long double uy = (long double)op->ly / (long double)h.Qy;

  const int L = lat->L;
  const int64_t NT = h.n_translates();
  h.set_nbr.assign((size_t)h.nsets * L, 0);
  h.set_dx.assign((size_t)h.nsets * L, 0);
  h.set_dy.assign((size_t)h.nsets * L, 0);
  h.alpha.assign((size_t)h.nsets * L, cd(0.0));
  h.residual.assign(h.nsets, 0.0);

  // frequencies of the least-squares system: the DFT preserves the residual up to XY, so the
  // residual runs over every frequency where the probe or u is non-zero (for u = psi_0 the
  // aperture; frequencies where u is below 1e-18 of its peak and the probe vanishes add
  // nothing at FP64 precision)
  std::vector<int32_t> kidx;
  double umax = 0.0;
  for (const cd& u : h.uspec) umax = std::max(umax, std::abs(u));
  for (int i = 0; i < nx * ny; ++i)
    if (std::abs(h.spec[i]) > 0.0 || std::abs(h.uspec[i]) > 1e-18 * umax) kidx.push_back(i);
  const int m = (int)kidx.size();

  struct Key { long double d2; int64_t i2; int64_t dy, dx; int32_t t; };
  std::vector<Key> keys((size_t)NT);
  for (int sy = 0; sy < h.ncls_y; ++sy) {
    for (int sx = 0; sx < h.ncls_x; ++sx) {
      const int s = sy * h.ncls_x + sx;
      const int64_t pxu = (int64_t)sx * h.stepPx, pyu = (int64_t)sy * h.stepPy;
      for (int tb = 0; tb < h.Rfy; ++tb) {
        int64_t tyu = (tb * h.stepTy + h.oyu) % h.Qy;
        int64_t dy = min_image(pyu - tyu, h.Qy);
        for (int ta = 0; ta < h.Rfx; ++ta) {
          int64_t txu = (ta * h.stepTx + h.oxu) % h.Qx;
          int64_t dx = min_image(pxu - txu, h.Qx);
          Key& k = keys[(size_t)tb * h.Rfx + ta];
          k.i2 = dx * dx + dy * dy;
          long double fx = dx * ux, fy = dy * uy;
          k.d2 = fx * fx + fy * fy;
          k.dy = dy; k.dx = dx;
          k.t = tb * h.Rfx + ta;
        }
      }
      auto less = [square](const Key& a, const Key& b) {
        if (square) { if (a.i2 != b.i2) return a.i2 < b.i2; }
        else if (a.d2 != b.d2) return a.d2 < b.d2;
        if (a.dy != b.dy) return a.dy < b.dy;
        return a.dx < b.dx;
      };
      std::partial_sort(keys.begin(), keys.begin() + L, keys.end(), less);
      for (int j = 0; j < L; ++j) {
        h.set_nbr[(size_t)s * L + j] = keys[j].t;
        h.set_dx[(size_t)s * L + j] = keys[j].t % h.Rfx;
        h.set_dy[(size_t)s * L + j] = keys[j].t / h.Rfx;
      }
      // least squares over those frequencies (Sec. 4.2.2):
      //   min || psi_hat_p - sum_j alpha_j u_hat e^{-2 pi i k.i_j} ||
      std::vector<cd> A((size_t)m * L), b(m);
      auto phase = [&](int k, int64_t xu, int64_t yu) {
        int mx = freq_index(k % nx, nx), my = freq_index(k / nx, ny);
        int64_t ax = ((int64_t)mx * xu % h.Qx + h.Qx) % h.Qx;
        int64_t ay = ((int64_t)my * yu % h.Qy + h.Qy) % h.Qy;
        double turns = (double)ax / (double)h.Qx + (double)ay / (double)h.Qy;
        double a = -2.0 * kPi * turns;
        return cd(std::cos(a), std::sin(a));
      };
      for (int j = 0; j < L; ++j) {
        int t = h.set_nbr[(size_t)s * L + j];
        int64_t txu = ((t % h.Rfx) * h.stepTx + h.oxu) % h.Qx;
        int64_t tyu = ((t / h.Rfx) * h.stepTy + h.oyu) % h.Qy;
        for (int r = 0; r < m; ++r) A[(size_t)j * m + r] = h.uspec[kidx[r]] * phase(kidx[r], txu, tyu);
      }
      double bn2 = 0.0;
      for (int r = 0; r < m; ++r) {
        b[r] = h.spec[kidx[r]] * phase(kidx[r], pxu, pyu);
        bn2 += std::norm(b[r]);
      }
      const double rcond = 2.220446049250313e-16 * XY;
      if (lat->basis_kind == LMA_BASIS_TRIGPOLY) {
        // closed form (Sec. 2): the translates span the frequencies K_+ = {|m_x| <= n_x,
        // |m_y| <= n_y}, and on K_+ the combination is an inverse DFT of length 2n + 1 per axis,
        //   alpha_j = 1/(Rfx Rfy) sum_{k in K_+} psi_hat_p[k] / u_hat[k] e^{+2 pi i k.i_j}
        // (M^-1 = diag(1/c) W* / (2n + 1) per axis); kept at the set's L nearest translates,
        // with the relative residual of that combination over every frequency
        std::vector<int32_t> kplus;
        for (int r = 0; r < m; ++r)
          if (std::abs(h.uspec[kidx[r]]) > 0.0) kplus.push_back(r);
        const double inv = 1.0 / ((double)h.Rfx * (double)h.Rfy);
        std::vector<cd> approx(m, cd(0.0));
        for (int j = 0; j < L; ++j) {
          const int t = h.set_nbr[(size_t)s * L + j];
          const int64_t txu = ((t % h.Rfx) * h.stepTx + h.oxu) % h.Qx;
          const int64_t tyu = ((t / h.Rfx) * h.stepTy + h.oyu) % h.Qy;
          cd acc(0.0);
          for (int r : kplus) acc += b[r] / h.uspec[kidx[r]] * std::conj(phase(kidx[r], txu, tyu));
          acc *= inv;
          h.alpha[(size_t)s * L + j] = acc;
          for (int r = 0; r < m; ++r) approx[r] += acc * A[(size_t)j * m + r];
        }
        double rn2 = 0.0;
        for (int r = 0; r < m; ++r) rn2 += std::norm(b[r] - approx[r]);
        h.residual[s] = std::sqrt(rn2 / bn2);
      } else if (m < L) {
        // fewer equations than unknowns: pad with zero rows (the minimum-norm solution is unchanged)
        std::vector<cd> A2((size_t)L * L, cd(0.0)), b2(L, cd(0.0));
        for (int j = 0; j < L; ++j)
          for (int r = 0; r < m; ++r) A2[(size_t)j * L + r] = A[(size_t)j * m + r];
        for (int r = 0; r < m; ++r) b2[r] = b[r];
        LsqResult res = lsq_min_norm(std::move(A2), L, L, std::move(b2), rcond);
        for (int j = 0; j < L; ++j) h.alpha[(size_t)s * L + j] = res.x[j];
        h.residual[s] = res.residual / std::sqrt(bn2);
      } else {
        LsqResult res = lsq_min_norm(std::move(A), m, L, std::move(b), rcond);
        for (int j = 0; j < L; ++j) h.alpha[(size_t)s * L + j] = res.x[j];
        h.residual[s] = res.residual / std::sqrt(bn2);
      }
    }
  }

  // ---- window and resident rows ---------------------------------------------------------------
  const int32_t* w = lat->window;
  if (w[0] == 0 && w[1] == 0 && w[2] == 0 && w[3] == 0) {
    h.wa0 = 0; h.wb0 = 0; h.ww = lat->px; h.wh = lat->py;
  } else {
    h.wa0 = w[0]; h.wb0 = w[1]; h.ww = w[2]; h.wh = w[3];
  }
  std::vector<uint8_t> need((size_t)NT, 0);
  // probes with the same set and shift share rows; walk the distinct (set, shift) pairs
  for (int b = h.wb0; b < h.wb0 + h.wh; ++b) {
    for (int a = h.wa0; a < h.wa0 + h.ww; ++a) {
      int s, shx, shy;
      h.probe_set(a, b, &s, &shx, &shy);
      for (int j = 0; j < L; ++j) {
        int ta = (h.set_dx[(size_t)s * L + j] + shx) % h.Rfx;
        int tb = (h.set_dy[(size_t)s * L + j] + shy) % h.Rfy;
        need[(size_t)tb * h.Rfx + ta] = 1;
      }
    }
  }
  h.rows.clear();
  h.row_of.assign((size_t)NT, -1);
  for (int64_t t = 0; t < NT; ++t)
    if (need[t]) {
      h.row_of[t] = (int32_t)h.rows.size();
      h.rows.push_back((int32_t)t);
    }
  return LMA_OK;
}

}  // namespace lma
