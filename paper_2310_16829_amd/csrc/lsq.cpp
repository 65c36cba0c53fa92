// Minimum-norm complex least squares: Householder QR followed by a one-sided (Hestenes)
// Jacobi SVD of the triangular factor. FP64, host only.
#include "lsq.hpp"

#include <algorithm>
#include <cmath>

namespace lma {

LsqResult lsq_min_norm(std::vector<cd> A, int m, int n, std::vector<cd> b, double rcond) {
  LsqResult out;
  auto a = [&](int i, int j) -> cd& { return A[(size_t)j * m + i]; };
  // --- Householder QR: A = Q R, b <- Q^H b ---------------------------------------------
  std::vector<cd> v(m);
  for (int k = 0; k < n && k < m; ++k) {
    double nx2 = 0.0;
    for (int i = k; i < m; ++i) nx2 += std::norm(a(i, k));
    double nx = std::sqrt(nx2);
    if (nx == 0.0) continue;
    cd x0 = a(k, k);
    cd ph = std::abs(x0) > 0.0 ? x0 / std::abs(x0) : cd(1.0, 0.0);
    cd alpha = -ph * nx;
    double vn2 = 0.0;
    for (int i = k; i < m; ++i) {
      v[i] = a(i, k);
      if (i == k) v[i] -= alpha;
      vn2 += std::norm(v[i]);
    }
    if (vn2 == 0.0) continue;
    for (int c = k; c < n; ++c) {
      cd s = 0.0;
      for (int i = k; i < m; ++i) s += std::conj(v[i]) * a(i, c);
      s *= 2.0 / vn2;
      for (int i = k; i < m; ++i) a(i, c) -= s * v[i];
    }
    cd s = 0.0;
    for (int i = k; i < m; ++i) s += std::conj(v[i]) * b[i];
    s *= 2.0 / vn2;
    for (int i = k; i < m; ++i) b[i] -= s * v[i];
  }
  double res2 = 0.0;
  for (int i = n; i < m; ++i) res2 += std::norm(b[i]);

  // --- one-sided Jacobi SVD of R (n x n upper triangle): R V = W, columns orthogonal ----
  std::vector<cd> W((size_t)n * n, cd(0.0)), V((size_t)n * n, cd(0.0));
  for (int j = 0; j < n; ++j) {
    for (int i = 0; i <= j && i < m; ++i) W[(size_t)j * n + i] = a(i, j);
    V[(size_t)j * n + j] = 1.0;
  }
  const double tol = 1e-15;
  for (int sweep = 0; sweep < 80; ++sweep) {
    double off = 0.0;
    for (int p = 0; p < n - 1; ++p) {
      for (int q = p + 1; q < n; ++q) {
        cd* wp = &W[(size_t)p * n];
        cd* wq = &W[(size_t)q * n];
        double al = 0.0, be = 0.0;
        cd ga = 0.0;
        for (int i = 0; i < n; ++i) {
          al += std::norm(wp[i]);
          be += std::norm(wq[i]);
          ga += std::conj(wp[i]) * wq[i];
        }
        double g = std::abs(ga);
        if (g == 0.0 || g <= tol * std::sqrt(al * be)) continue;
        off = std::max(off, g / std::sqrt(al * be));
        cd e = std::conj(ga / g);           // makes the off-diagonal real and positive
        double zeta = (be - al) / (2.0 * g);
        double t = (zeta >= 0.0 ? 1.0 : -1.0) / (std::abs(zeta) + std::sqrt(1.0 + zeta * zeta));
        double c = 1.0 / std::sqrt(1.0 + t * t), s = c * t;
        cd* vp = &V[(size_t)p * n];
        cd* vq = &V[(size_t)q * n];
        for (int i = 0; i < n; ++i) {
          cd xq = wq[i] * e, xp = wp[i];
          wp[i] = c * xp - s * xq;
          wq[i] = s * xp + c * xq;
          cd yq = vq[i] * e, yp = vp[i];
          vp[i] = c * yp - s * yq;
          vq[i] = s * yp + c * yq;
        }
      }
    }
    if (off <= tol) break;
  }
  std::vector<double> sig(n);
  double smax = 0.0;
  for (int j = 0; j < n; ++j) {
    double s2 = 0.0;
    for (int i = 0; i < n; ++i) s2 += std::norm(W[(size_t)j * n + i]);
    sig[j] = std::sqrt(s2);
    smax = std::max(smax, sig[j]);
  }
  out.x.assign(n, cd(0.0));
  out.sigma_max = smax;
  out.sigma_min_kept = smax;
  double cut = rcond * smax;
  for (int j = 0; j < n; ++j) {
    cd uc = 0.0;                                  // U_j^H c with U_j = W_j / sigma_j
    for (int i = 0; i < n; ++i) uc += std::conj(W[(size_t)j * n + i]) * b[i];
    if (sig[j] > cut && sig[j] > 0.0) {
      cd coef = uc / (sig[j] * sig[j]);
      for (int i = 0; i < n; ++i) out.x[i] += V[(size_t)j * n + i] * coef;
      out.rank++;
      out.sigma_min_kept = std::min(out.sigma_min_kept, sig[j]);
    } else if (sig[j] > 0.0) {
      res2 += std::norm(uc / sig[j]);
    }
  }
  out.residual = std::sqrt(res2);
  return out;
}

}  // namespace lma
