"""Pins of the oracle's KL expansions (Eqs. covarianceFunction, inftyKL).

* 1-D exponential: roots satisfy their transcendental equations, the
  closed-form eigenvalues agree with an independent Nystrom solve of the
  same kernel, the eigenfunctions are orthonormal, and the eigenvalues sum
  to the operator trace ``2a``.
* 2-D separable exponential: the oracle's Nystrom machinery applied to the
  separable kernel reproduces the closed-form products (this pins the
  Nystrom code used for the Matern covariance).
* 2-D separable exponential, selection and order: the ten largest
  eigenvalues of a 2-D Nystrom solve of the full covariance operator on the
  strip (no use of the product structure in the eigensolve, Richardson
  extrapolated over two grids) equal the oracle's closed-form products in
  value and order, and its eigenvectors equal the oracle's modes.
* Matern: the oracle's kernel is the general Matern form
  ``s^2 2^(1-nu)/Gamma(nu) (sqrt(2 nu) r/l)^nu K_nu(sqrt(2 nu) r/l)`` at
  ``nu = 3/2`` (modified Bessel function from scipy); trace identity of the
  discrete operator, orthonormality in the quadrature inner product,
  Nystrom interpolation reproduces the grid values, eigen-equation
  residuals, robust sign convention, and a sample variance check of the
  synthesised field.
"""
import math

import numpy as np
import pytest
from scipy.sparse.linalg import LinearOperator, eigsh
from scipy.special import gamma, kv

import mlmc_inputs as mi
from oracle.kl import (KL, exp1d_eigen, exp1d_mode, gauss_legendre_grid, matern32,
                       nystrom_eigen, wrinkle)

C1 = mi.load_config("strip_c1")
C2 = mi.load_config("strip_c2")


def test_exp1d_roots_and_eigenvalues():
    a, om = 10.0, 2.0
    c = 1 / om
    lam, w, par = exp1d_eigen(a, om, 12)
    for wi, p in zip(w, par):
        f = c * math.cos(wi * a) - wi * math.sin(wi * a) if p == 0 else wi * math.cos(wi * a) + c * math.sin(wi * a)
        assert abs(f) < 1e-12 * max(1, wi)
    assert np.all(np.diff(lam) < 0)
    # independent: Nystrom on a fine Gauss-Legendre grid
    g, wq = np.polynomial.legendre.leggauss(1500)
    x, wq = a * g, a * wq
    Kmat = np.exp(-np.abs(x[:, None] - x[None, :]) / om)
    ev = np.sort(np.linalg.eigvalsh(np.sqrt(wq)[:, None] * Kmat * np.sqrt(wq)[None, :]))[::-1]
    np.testing.assert_allclose(lam, ev[:12], rtol=2e-4)  # Nystrom error of the kinked kernel is O(1e-4) here
    # orthonormality by quadrature
    F = np.stack([exp1d_mode(x, a, wi, p) for wi, p in zip(w, par)], axis=1)
    np.testing.assert_allclose(F.T @ (wq[:, None] * F), np.eye(12), atol=1e-12)


def test_exp1d_trace():
    a, om = 2.5, 2.0
    lam, _, _ = exp1d_eigen(a, om, 4000)
    # sum of all eigenvalues = int k(x,x) dx = 2a; the tail decays like 1/n^2
    tail = 2 * (1 / om) / (math.pi / (2 * a)) ** 2 / 4000
    assert abs(lam.sum() + tail - 2 * a) < 5e-4


def test_nystrom_2d_separable_is_kron_of_1d():
    # the 2-D Nystrom machinery on a separable kernel must reproduce the
    # products of independent 1-D Nystrom eigenpairs exactly (Kronecker identity)
    Lx, Ly, nqx, nqy = 20.0, 5.0, 40, 16
    grid, wq = gauss_legendre_grid(Lx, Ly, nqx, nqy)
    s2 = 0.01

    def kern(P, R):
        return s2 * np.exp(-np.abs(P[:, None, 0] - R[None, :, 0]) / 2.0
                           - np.abs(P[:, None, 1] - R[None, :, 1]) / 2.0)
    mu, phi, proj = nystrom_eigen(kern, grid, wq, 8)

    def one_d(L, n):
        g, w = np.polynomial.legendre.leggauss(n)
        x, w = 0.5 * L * (g + 1), 0.5 * L * w
        S = np.sqrt(w)[:, None] * np.exp(-np.abs(x[:, None] - x[None, :]) / 2.0) * np.sqrt(w)[None, :]
        e, v = np.linalg.eigh(S)
        return e, v / np.sqrt(w)[:, None]
    ex, vx = one_d(Lx, nqx)
    ey, vy = one_d(Ly, nqy)
    prods = np.sort((s2 * np.outer(ey, ex)).ravel())[::-1]
    np.testing.assert_allclose(mu[:40], prods[:40], rtol=1e-12)
    # top mode is the product of the top 1-D modes (grid order: x fastest)
    top = np.kron(vy[:, -1], vx[:, -1])
    assert abs(abs(np.sum(wq * top * phi[:, 0])) - 1.0) < 1e-12
    assert np.all(proj > 0)


def test_exp_separable_modes_orthonormal():
    kl = KL(C1)
    grid, wq = gauss_legendre_grid(C1["Lx"], C1["Ly"], 200, 60)
    F = kl.modes_at(grid)
    np.testing.assert_allclose(F.T @ (wq[:, None] * F), np.eye(kl.K), atol=1e-10)


def test_exp_separable_selection_and_gaps():
    kl = KL(C1)
    assert len(kl.mu) == 10 and np.all(np.diff(kl.mu) < 0)
    gaps = -np.diff(np.concatenate([kl.mu, [kl.mu_next]])) / kl.mu[0]
    assert gaps.min() > 1e-6        # the selected set and its order are well defined
    # variance fraction captured by 10 modes on the 20 x 5 strip
    frac = kl.mu.sum() / (kl.var * C1["Lx"] * C1["Ly"])
    assert 0.4 < frac < 0.55


def _nystrom_2d_separable(Lx, Ly, corr_x, corr_y, var, nqx, nqy, k):
    """Top-``k`` eigenpairs of the Nystrom discretisation of the 2-D operator
    with kernel ``var exp(-|dx|/corr_x - |dy|/corr_y)`` on a tensor
    Gauss-Legendre grid (x fastest).  The matrix is applied as a whole 2-D
    operator; the eigensolver sees one symmetric matrix of order nqx*nqy."""
    gx, wx = np.polynomial.legendre.leggauss(nqx)
    gy, wy = np.polynomial.legendre.leggauss(nqy)
    x, wx = 0.5 * Lx * (gx + 1.0), 0.5 * Lx * wx
    y, wy = 0.5 * Ly * (gy + 1.0), 0.5 * Ly * wy
    sx, sy = np.sqrt(wx), np.sqrt(wy)
    Ex = sx[:, None] * np.exp(-np.abs(x[:, None] - x[None, :]) / corr_x) * sx[None, :]
    Ey = sy[:, None] * np.exp(-np.abs(y[:, None] - y[None, :]) / corr_y) * sy[None, :]
    n = nqx * nqy
    op = LinearOperator((n, n), dtype=np.float64,
                        matvec=lambda v: var * (Ey @ v.reshape(nqy, nqx) @ Ex.T).ravel())
    ev, vec = eigsh(op, k=k, which="LA", tol=1e-13)
    order = np.argsort(ev)[::-1]
    X, Y = np.meshgrid(x, y)
    W = np.outer(wy, wx).ravel()
    return ev[order], vec[:, order] / np.sqrt(W)[:, None], np.stack([X.ravel(), Y.ravel()], 1), W


def test_separable_selection_matches_a_2d_nystrom_solve():
    # Eqs. covarianceFunction / inftyKL: the truncated expansion keeps the K
    # largest eigenvalues of the 2-D covariance operator, in decreasing order.
    kl = KL(C1)
    kw = dict(Lx=C1["Lx"], Ly=C1["Ly"], corr_x=C1["kl"]["corr_x"], corr_y=C1["kl"]["corr_y"], var=kl.var, k=12)
    mu_c, _, _, _ = _nystrom_2d_separable(nqx=100, nqy=25, **kw)
    mu_f, vec, pts, W = _nystrom_2d_separable(nqx=200, nqy=50, **kw)
    # the kinked kernel makes the Nystrom eigenvalues converge like h^2:
    # one Richardson step removes that term
    mu_x = (4.0 * mu_f - mu_c) / 3.0
    np.testing.assert_allclose(mu_f[:kl.K], kl.mu, rtol=3e-3)
    np.testing.assert_allclose(mu_x[:kl.K], kl.mu, rtol=1e-4)
    # the (K+1)-th eigenvalue is the first one left out
    assert abs(mu_x[kl.K] / kl.mu_next - 1.0) < 1e-4
    # same modes in the same order: quadrature inner products of +-1
    F = kl.modes_at(pts)
    inner = np.abs(np.sum(W[:, None] * F * vec[:, :kl.K], axis=0))
    assert np.all(inner > 0.9999), inner


@pytest.mark.parametrize("length", [1.5, 0.7])
def test_matern32_is_the_general_matern_form_at_nu_three_halves(length):
    nu, var = 1.5, 0.0027
    r = np.array([1e-3, 0.01, 0.1, 0.3, 0.5, 0.9, 1.5, 2.2, 3.0, 4.5, 7.0, 11.0])
    z = math.sqrt(2.0 * nu) * r / length
    general = var * 2.0 ** (1.0 - nu) / gamma(nu) * z ** nu * kv(nu, z)
    np.testing.assert_allclose(matern32(r, var, length), general, rtol=1e-13, atol=0)
    assert matern32(np.array([0.0]), var, length)[0] == var


def test_matern_nystrom_identities():
    kl = KL(C2)
    # trace of the discrete operator: sum mu = s^2 sum w = s^2 |Omega|
    assert abs(kl.all_mu.sum() - kl.var * C2["Lx"] * C2["Ly"]) < 1e-12 * kl.var * 100
    G = kl.phi_grid.T @ (kl.wq[:, None] * kl.phi_grid)
    np.testing.assert_allclose(G, np.eye(kl.K), atol=1e-12)
    # Nystrom interpolation reproduces the grid values
    np.testing.assert_allclose(kl.modes_at(kl.grid), kl.phi_grid, rtol=0, atol=1e-11)
    # eigen-equation residual  int k(x,y) phi(y) dy = mu phi(x)  at off-grid points
    pts = np.array([[1.3, 0.7], [10.1, 2.2], [17.9, 4.4]])
    lhs = kl.kernel(pts, kl.grid) @ (kl.wq[:, None] * kl.phi_grid)
    np.testing.assert_allclose(lhs, kl.modes_at(pts) * kl.mu[None, :], rtol=1e-12, atol=1e-15)
    assert kl.sign_projection.min() > 1e-3
    gaps = -np.diff(np.concatenate([kl.mu, [kl.mu_next]])) / kl.mu[0]
    assert gaps.min() > 1e-5


def test_matern_quadrature_convergence():
    cfg = dict(C2)
    cfg["kl"] = dict(C2["kl"], nystrom=[128, 32])
    fine = KL(cfg)
    base = KL(C2)
    np.testing.assert_allclose(base.mu, fine.mu, rtol=2e-3)


def test_field_sample_variance_matches_modes():
    kl = KL(C1)
    pts = np.array([[3.0, 1.0], [10.0, 2.5], [16.5, 4.0]])
    phi = kl.modes_at(pts)
    var_pred = (phi ** 2) @ kl.mu
    xi = mi.strip_xi(C1, 0, 0, 20000)
    th = (phi @ (np.sqrt(kl.mu)[:, None] * xi[:, :kl.K].T)).T
    v = th.var(axis=0)
    # sample variance of a Gaussian: sd ~ var * sqrt(2/N)
    assert np.all(np.abs(v - var_pred) < 4 * var_pred * math.sqrt(2 / 20000))


def test_wrinkle_is_sech_squared():
    x = np.linspace(0, 20, 41)
    np.testing.assert_allclose(wrinkle(x, 0.05, 9.0, 1.3), 0.05 / np.cosh((x - 9.0) / 1.3) ** 2, rtol=1e-13)
    assert np.all(wrinkle(x, 0.0, 9.0, 1.3) == 0)
