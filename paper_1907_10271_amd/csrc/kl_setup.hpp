// Host-side KL set-up (Section 3.1, Eqs. covarianceFunction and inftyKL).
#pragma once

#include <vector>

namespace mlmc {

// Gauss-Legendre nodes (ascending) and weights on [-1, 1]
void gauss_legendre(int n, std::vector<double> &x, std::vector<double> &w);

// closed-form eigenpairs of exp(-|x - y|/omega) on [-a, a], decreasing eigenvalue
struct Exp1D {
  double a = 0.0;
  std::vector<double> lam, w, norm;
  std::vector<int> parity;  // 0 even (cos), 1 odd (sin)
  double mode(int i, double x_centred) const;
};
Exp1D exp1d_eigen(double a, double omega, int n);

// separable exponential on [0, Lx] x [0, Ly]: K largest products
struct SeparableKL {
  double Lx = 0, Ly = 0;
  Exp1D x, y;
  std::vector<double> mu;     // includes the variance
  std::vector<int> ix, iy;    // factor indices of each selected mode
};
SeparableKL separable_kl(double Lx, double Ly, double var, double wx, double wy, int K);

// Matern-3/2 by Nystrom on a tensor Gauss-Legendre grid (x fastest)
struct MaternKL {
  int n = 0, K = 0;
  double var = 0, length = 0;
  std::vector<double> px, py, wq;  // grid points and weights
  std::vector<double> mu;          // K largest eigenvalues
  std::vector<double> phi;         // [n][K] eigenfunction values at the grid
  double mu_next = 0;
  double max_residual = 0;         // max relative eigen-residual of the K pairs
};
MaternKL matern_kl(double Lx, double Ly, double var, double length, int nqx, int nqy, int K);

}  // namespace mlmc
