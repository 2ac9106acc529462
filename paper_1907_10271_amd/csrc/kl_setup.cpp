// Host-side set-up of the KL expansions of the fibre-angle field
// (Section 3.1, Eqs. covarianceFunction and inftyKL).
//
//  * Separable exponential covariance: the 1-D factors on a centred interval
//    [-a, a] have closed-form eigenpairs, lambda = 2c / (w^2 + c^2) with
//    c = 1/omega, even modes cos(w x) where c cos(wa) = w sin(wa), odd modes
//    sin(w x) where w cos(wa) = -c sin(wa).  Roots are bracketed one per
//    quarter period and found by bisection to the last bit.  2-D eigenpairs
//    are the products; the K largest are kept (ties by (i + j, i)).
//  * Isotropic Matern-3/2 covariance: Nystrom discretisation on a tensor
//    Gauss-Legendre grid, W^1/2 k W^1/2, whose top K eigenpairs come from a
//    Lanczos run with full re-orthogonalisation and a Jacobi eigen-solve of
//    the tridiagonal matrix.  Grid values are v / sqrt(w); the sign of each
//    eigenvector is fixed by a positive projection on the weights
//    h_j = ((j * 2654435761) mod 1000003) / 1000003 - 0.5.
#include "kl_setup.hpp"

#include <algorithm>
#include <cmath>
#include <numeric>
#include <stdexcept>

namespace mlmc {

void gauss_legendre(int n, std::vector<double> &x, std::vector<double> &w) {
  x.assign(n, 0.0);
  w.assign(n, 0.0);
  for (int i = 0; i < n; ++i) {
    // Newton on P_n from the Tricomi initial guess; nodes ascending
    double z = -std::cos(M_PI * (i + 0.75) / (n + 0.5));
    double dp = 0.0;
    for (int it = 0; it < 100; ++it) {
      double p0 = 1.0, p1 = z;
      for (int k = 2; k <= n; ++k) {
        double p2 = ((2.0 * k - 1.0) * z * p1 - (k - 1.0) * p0) / k;
        p0 = p1;
        p1 = p2;
      }
      dp = n * (z * p1 - p0) / (z * z - 1.0);
      double dz = p1 / dp;
      z -= dz;
      if (std::fabs(dz) < 1e-16) break;
    }
    {
      double p0 = 1.0, p1 = z;
      for (int k = 2; k <= n; ++k) {
        double p2 = ((2.0 * k - 1.0) * z * p1 - (k - 1.0) * p0) / k;
        p0 = p1;
        p1 = p2;
      }
      dp = n * (z * p1 - p0) / (z * z - 1.0);
    }
    x[i] = z;
    w[i] = 2.0 / ((1.0 - z * z) * dp * dp);
  }
}

static double bisect(double lo, double hi, double (*f)(double, double, double), double a, double c) {
  double flo = f(lo, a, c);
  for (int it = 0; it < 200; ++it) {
    double mid = 0.5 * (lo + hi);
    if (mid <= lo || mid >= hi) break;
    double fm = f(mid, a, c);
    if (fm == 0.0) return mid;
    if ((fm > 0) == (flo > 0)) { lo = mid; flo = fm; } else { hi = mid; }
  }
  return 0.5 * (lo + hi);
}

static double f_even(double w, double a, double c) { return c * std::cos(w * a) - w * std::sin(w * a); }
static double f_odd(double w, double a, double c) { return w * std::cos(w * a) + c * std::sin(w * a); }

Exp1D exp1d_eigen(double a, double omega, int n) {
  const double c = 1.0 / omega;
  Exp1D r;
  for (int k = 0; (int)r.w.size() < n; ++k) {
    double lo = k * M_PI / a, mid = (k * M_PI + 0.5 * M_PI) / a, hi = (k + 1) * M_PI / a;
    r.w.push_back(bisect(lo, mid, f_even, a, c));
    r.parity.push_back(0);
    if ((int)r.w.size() < n) {
      r.w.push_back(bisect(mid, hi, f_odd, a, c));
      r.parity.push_back(1);
    }
  }
  for (double w : r.w) r.lam.push_back(2.0 * c / (w * w + c * c));
  for (size_t i = 0; i < r.w.size(); ++i) {
    double w = r.w[i];
    double s = std::sin(2.0 * w * a) / (2.0 * w);
    r.norm.push_back(1.0 / std::sqrt(r.parity[i] == 0 ? a + s : a - s));
  }
  r.a = a;
  return r;
}

double Exp1D::mode(int i, double xc) const {
  return norm[i] * (parity[i] == 0 ? std::cos(w[i] * xc) : std::sin(w[i] * xc));
}

SeparableKL separable_kl(double Lx, double Ly, double var, double wx, double wy, int K) {
  SeparableKL s;
  int nc = K + 2;
  s.x = exp1d_eigen(0.5 * Lx, wx, nc);
  s.y = exp1d_eigen(0.5 * Ly, wy, nc);
  struct Cand { double mu; int i, j; };
  std::vector<Cand> c;
  for (int i = 0; i < nc; ++i)
    for (int j = 0; j < nc; ++j) c.push_back({var * s.x.lam[i] * s.y.lam[j], i, j});
  std::stable_sort(c.begin(), c.end(), [](const Cand &p, const Cand &q) {
    if (p.mu != q.mu) return p.mu > q.mu;
    if (p.i + p.j != q.i + q.j) return p.i + p.j < q.i + q.j;
    return p.i < q.i;
  });
  for (int k = 0; k < K; ++k) {
    s.mu.push_back(c[k].mu);
    s.ix.push_back(c[k].i);
    s.iy.push_back(c[k].j);
  }
  s.Lx = Lx;
  s.Ly = Ly;
  return s;
}

// cyclic Jacobi eigenvalue iteration for a dense symmetric matrix (row-major m x m);
// on return A holds the eigenvalues on its diagonal and V the eigenvectors (columns)
static void jacobi_eigen(std::vector<double> &A, std::vector<double> &V, int m) {
  V.assign((size_t)m * m, 0.0);
  for (int i = 0; i < m; ++i) V[(size_t)i * m + i] = 1.0;
  double norm = 0.0;
  for (double v : A) norm += v * v;
  for (int sweep = 0; sweep < 100; ++sweep) {
    double off = 0.0;
    for (int p = 0; p < m; ++p)
      for (int q = p + 1; q < m; ++q) off += A[(size_t)p * m + q] * A[(size_t)p * m + q];
    if (off <= 1e-34 * norm) break;
    for (int p = 0; p < m; ++p) {
      for (int q = p + 1; q < m; ++q) {
        double apq = A[(size_t)p * m + q];
        if (apq == 0.0) continue;
        double app = A[(size_t)p * m + p], aqq = A[(size_t)q * m + q];
        double tau = (aqq - app) / (2.0 * apq);
        double t = (tau >= 0 ? 1.0 : -1.0) / (std::fabs(tau) + std::sqrt(1.0 + tau * tau));
        double cs = 1.0 / std::sqrt(1.0 + t * t), sn = t * cs;
        for (int k = 0; k < m; ++k) {  // columns p, q
          double akp = A[(size_t)k * m + p], akq = A[(size_t)k * m + q];
          A[(size_t)k * m + p] = cs * akp - sn * akq;
          A[(size_t)k * m + q] = sn * akp + cs * akq;
        }
        for (int k = 0; k < m; ++k) {  // rows p, q
          double apk = A[(size_t)p * m + k], aqk = A[(size_t)q * m + k];
          A[(size_t)p * m + k] = cs * apk - sn * aqk;
          A[(size_t)q * m + k] = sn * apk + cs * aqk;
        }
        for (int k = 0; k < m; ++k) {
          double vkp = V[(size_t)k * m + p], vkq = V[(size_t)k * m + q];
          V[(size_t)k * m + p] = cs * vkp - sn * vkq;
          V[(size_t)k * m + q] = sn * vkp + cs * vkq;
        }
      }
    }
  }
}

static double sign_weight(long j) {
  unsigned long long v = (unsigned long long)j * 2654435761ull;
  return (double)(v % 1000003ull) / 1000003.0 - 0.5;
}

static double matern32(double r, double var, double len) {
  double z = std::sqrt(3.0) * r / len;
  return var * (1.0 + z) * std::exp(-z);
}

MaternKL matern_kl(double Lx, double Ly, double var, double length, int nqx, int nqy, int K) {
  MaternKL out;
  out.var = var;
  out.length = length;
  std::vector<double> gx, wx, gy, wy;
  gauss_legendre(nqx, gx, wx);
  gauss_legendre(nqy, gy, wy);
  const int n = nqx * nqy;
  out.px.resize(n);
  out.py.resize(n);
  out.wq.resize(n);
  for (int iy = 0; iy < nqy; ++iy)
    for (int ix = 0; ix < nqx; ++ix) {
      int j = iy * nqx + ix;
      out.px[j] = 0.5 * Lx * (gx[ix] + 1.0);
      out.py[j] = 0.5 * Ly * (gy[iy] + 1.0);
      out.wq[j] = 0.5 * Lx * wx[ix] * 0.5 * Ly * wy[iy];
    }
  std::vector<double> sw(n);
  for (int j = 0; j < n; ++j) sw[j] = std::sqrt(out.wq[j]);
  std::vector<double> S((size_t)n * n);
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < n; ++j) {
      double dx = out.px[i] - out.px[j], dy = out.py[i] - out.py[j];
      S[(size_t)i * n + j] = sw[i] * matern32(std::sqrt(dx * dx + dy * dy), var, length) * sw[j];
    }
  // Lanczos with full re-orthogonalisation
  int m = std::min(n, std::max(8 * K, 200));
  std::vector<double> Vb((size_t)(m + 1) * n, 0.0), alpha(m, 0.0), beta(m, 0.0), w(n);
  double nrm = 0.0;
  for (int j = 0; j < n; ++j) {
    Vb[j] = sign_weight(j) + 0.25;
    nrm += Vb[j] * Vb[j];
  }
  nrm = std::sqrt(nrm);
  for (int j = 0; j < n; ++j) Vb[j] /= nrm;
  int steps = m;
  for (int k = 0; k < m; ++k) {
    const double *v = &Vb[(size_t)k * n];
    for (int i = 0; i < n; ++i) {
      double s = 0.0;
      const double *row = &S[(size_t)i * n];
      for (int j = 0; j < n; ++j) s += row[j] * v[j];
      w[i] = s;
    }
    double a = 0.0;
    for (int i = 0; i < n; ++i) a += v[i] * w[i];
    alpha[k] = a;
    for (int pass = 0; pass < 2; ++pass)
      for (int l = 0; l <= k; ++l) {
        const double *u = &Vb[(size_t)l * n];
        double d = 0.0;
        for (int i = 0; i < n; ++i) d += u[i] * w[i];
        for (int i = 0; i < n; ++i) w[i] -= d * u[i];
      }
    double b = 0.0;
    for (int i = 0; i < n; ++i) b += w[i] * w[i];
    b = std::sqrt(b);
    beta[k] = b;
    if (b < 1e-300 || k == m - 1) { steps = k + 1; break; }
    double *vn = &Vb[(size_t)(k + 1) * n];
    for (int i = 0; i < n; ++i) vn[i] = w[i] / b;
  }
  std::vector<double> T((size_t)steps * steps, 0.0), U;
  for (int k = 0; k < steps; ++k) {
    T[(size_t)k * steps + k] = alpha[k];
    if (k + 1 < steps) T[(size_t)k * steps + k + 1] = T[(size_t)(k + 1) * steps + k] = beta[k];
  }
  jacobi_eigen(T, U, steps);
  std::vector<int> order(steps);
  std::iota(order.begin(), order.end(), 0);
  std::sort(order.begin(), order.end(),
            [&](int p, int q) { return T[(size_t)p * steps + p] > T[(size_t)q * steps + q]; });
  if (steps < K + 1) throw std::runtime_error("Nystrom grid too small for the requested modes");
  out.mu.resize(K);
  out.phi.assign((size_t)n * K, 0.0);
  out.max_residual = 0.0;
  for (int k = 0; k < K; ++k) {
    int c = order[k];
    std::vector<double> y(n, 0.0);
    for (int l = 0; l < steps; ++l) {
      double s = U[(size_t)l * steps + c];
      const double *u = &Vb[(size_t)l * n];
      for (int i = 0; i < n; ++i) y[i] += s * u[i];
    }
    double yn = 0.0;
    for (double v : y) yn += v * v;
    yn = std::sqrt(yn);
    for (double &v : y) v /= yn;
    // Rayleigh quotient and residual
    std::vector<double> Sy(n, 0.0);
    for (int i = 0; i < n; ++i) {
      double s = 0.0;
      const double *row = &S[(size_t)i * n];
      for (int j = 0; j < n; ++j) s += row[j] * y[j];
      Sy[i] = s;
    }
    double rq = 0.0;
    for (int i = 0; i < n; ++i) rq += y[i] * Sy[i];
    double res = 0.0;
    for (int i = 0; i < n; ++i) res += (Sy[i] - rq * y[i]) * (Sy[i] - rq * y[i]);
    out.max_residual = std::max(out.max_residual, std::sqrt(res) / std::fabs(rq));
    out.mu[k] = rq;
    double proj = 0.0;
    for (int i = 0; i < n; ++i) proj += sign_weight(i) * (y[i] / sw[i]);
    double sg = proj < 0 ? -1.0 : 1.0;
    for (int i = 0; i < n; ++i) out.phi[(size_t)i * K + k] = sg * y[i] / sw[i];
  }
  out.mu_next = T[(size_t)order[K] * steps + order[K]];
  out.n = n;
  out.K = K;
  return out;
}

}  // namespace mlmc
