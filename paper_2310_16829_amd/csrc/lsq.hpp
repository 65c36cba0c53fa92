// Minimum-norm complex least squares in FP64 (host).
#pragma once
#include <complex>
#include <vector>

namespace lma {

using cd = std::complex<double>;

// Solves min ||A x - b||_2 for A (m x n, column-major, m >= n) with the minimum-norm
// solution among the minimisers: Householder QR of A, then a one-sided Jacobi SVD of R,
// singular values below rcond * sigma_max dropped. Returns x (n) and the residual norm.
struct LsqResult {
  std::vector<cd> x;
  double residual = 0.0;
  double sigma_max = 0.0, sigma_min_kept = 0.0;
  int rank = 0;
};

LsqResult lsq_min_norm(std::vector<cd> A, int m, int n, std::vector<cd> b, double rcond);

}  // namespace lma
