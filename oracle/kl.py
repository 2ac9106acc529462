"""Random fibre-angle fields: covariance operators and truncated KL expansions.

Section 3.1 models the misalignment angle as a Gaussian random field with a
two-point covariance (Eq. covarianceFunction: separable exponential with
variance ``s^2`` and correlation lengths ``omega_1, omega_2``) and
represents it by its Karhunen-Loeve expansion (Eq. inftyKL)
``Phi(x) = sum_n sqrt(mu_n) phi_n(x) xi_n``, truncated after ``N_KL`` terms,
with ``(mu_n, phi_n)`` the eigenpairs of the covariance operator in
decreasing order of ``mu_n``.

Two covariance families are implemented:

* ``exp_separable`` -- the paper's covariance.  Its 1-D factors on a
  centred interval ``[-a, a]`` have closed-form eigenpairs (the classical
  Ghanem-Spanos solution, the text the paper cites for KL): with
  ``c = 1/omega`` the eigenvalue is ``2c / (w^2 + c^2)``; even modes
  ``cos(w x)`` solve ``c cos(wa) - w sin(wa) = 0`` and odd modes
  ``sin(w x)`` solve ``w cos(wa) + c sin(wa) = 0``.  2-D eigenpairs are
  products; ties in ``mu`` are broken by ``(i + j, i)``.
* ``matern32`` -- an isotropic Matern covariance with smoothness 3/2,
  ``k(r) = s^2 (1 + sqrt3 r / l) exp(-sqrt3 r / l)`` (used by the waviness
  workloads in place of the paper's exponential).  No closed form exists,
  so the operator is discretised by the Nystrom method on a tensor
  Gauss-Legendre grid (independent of the FE level) and eigenvectors are
  extended to any point by Nystrom interpolation.  The sign of each
  eigenvector is fixed so that its projection on a fixed pseudo-random
  weight vector ``h_j = ((j * 2654435761) mod 1000003) / 1000003 - 0.5``
  is positive.

A localised wrinkle ``A sech^2((x - x0) / w)`` (uniform in y) can be added to
the field.
"""
from __future__ import annotations

import math

import numpy as np
from scipy.optimize import brentq


# ----------------------------------------------------------------------------
# separable exponential: closed-form 1-D eigenpairs
# ----------------------------------------------------------------------------

def exp1d_eigen(a: float, omega: float, n: int):
    """First ``n`` eigenpairs of ``exp(-|x - y| / omega)`` on ``[-a, a]``.

    Returns ``(lam, w, parity)`` sorted by decreasing ``lam``; parity 0 means
    an even mode ``cos(w x) / sqrt(a + sin(2wa)/(2w))`` and 1 an odd mode
    ``sin(w x) / sqrt(a - sin(2wa)/(2w))``.
    """
    c = 1.0 / omega
    roots = []
    k = 0
    while len(roots) < 2 * n + 2:
        lo, hi = k * math.pi / a, (k * math.pi + 0.5 * math.pi) / a
        f_even = lambda w: c * math.cos(w * a) - w * math.sin(w * a)
        roots.append((brentq(f_even, lo, hi, xtol=1e-300, rtol=4 * np.finfo(float).eps, maxiter=500), 0))
        lo2, hi2 = hi, (k + 1) * math.pi / a
        f_odd = lambda w: w * math.cos(w * a) + c * math.sin(w * a)
        roots.append((brentq(f_odd, lo2, hi2, xtol=1e-300, rtol=4 * np.finfo(float).eps, maxiter=500), 1))
        k += 1
    roots.sort(key=lambda t: t[0])
    roots = roots[:n]
    w = np.array([r[0] for r in roots])
    par = np.array([r[1] for r in roots], dtype=int)
    lam = 2.0 * c / (w * w + c * c)
    return lam, w, par


def exp1d_mode(x: np.ndarray, a: float, w: float, parity: int) -> np.ndarray:
    """Normalised 1-D eigenfunction at centred coordinates ``x`` in ``[-a, a]``."""
    if parity == 0:
        return np.cos(w * x) / math.sqrt(a + math.sin(2 * w * a) / (2 * w))
    return np.sin(w * x) / math.sqrt(a - math.sin(2 * w * a) / (2 * w))


# ----------------------------------------------------------------------------
# Matern-3/2 via Nystrom on a Gauss-Legendre grid
# ----------------------------------------------------------------------------

def matern32(r: np.ndarray, var: float, length: float) -> np.ndarray:
    z = math.sqrt(3.0) * r / length
    return var * (1.0 + z) * np.exp(-z)


def gauss_legendre_grid(Lx: float, Ly: float, nqx: int, nqy: int):
    """Tensor Gauss-Legendre points (x fastest) and weights on ``[0,Lx] x [0,Ly]``."""
    gx, wx = np.polynomial.legendre.leggauss(nqx)
    gy, wy = np.polynomial.legendre.leggauss(nqy)
    px, wxs = 0.5 * Lx * (gx + 1.0), 0.5 * Lx * wx
    py, wys = 0.5 * Ly * (gy + 1.0), 0.5 * Ly * wy
    X, Y = np.meshgrid(px, py)
    WX, WY = np.meshgrid(wxs, wys)
    return np.stack([X.ravel(), Y.ravel()], axis=1), (WX * WY).ravel()


def nystrom_eigen(kernel, grid: np.ndarray, wq: np.ndarray, K: int):
    """Top ``K`` eigenpairs of the Nystrom discretisation of a covariance operator.

    ``kernel(P, R)`` evaluates ``k`` between point sets ``P [n,2]`` and ``R [m,2]``.
    The symmetric matrix ``W^1/2 k W^1/2`` is diagonalised; grid values of
    the eigenfunctions are ``v / sqrt(w)`` (unit norm in the quadrature inner
    product) with the sign fixed by :func:`sign_weights`.  Returns
    ``(mu_all_desc, phi_grid [n, K], sign_projection [K])``.
    """
    Kmat = kernel(grid, grid)
    sw = np.sqrt(wq)
    S = sw[:, None] * Kmat * sw[None, :]
    evals, evecs = np.linalg.eigh(S)
    order = np.argsort(evals)[::-1]
    phi = evecs[:, order[:K]] / sw[:, None]
    proj = sign_weights(len(wq)) @ phi
    phi = phi * np.sign(proj)[None, :]
    return evals[order], phi, np.abs(proj)


def sign_weights(n: int) -> np.ndarray:
    j = np.arange(n, dtype=np.int64)
    return ((j * 2654435761) % 1000003).astype(np.float64) / 1000003.0 - 0.5


class KL:
    """Truncated KL expansion of the configured angle field (values in radians)."""

    def __init__(self, cfg: dict):
        kl = cfg["kl"]
        self.Lx, self.Ly = float(cfg["Lx"]), float(cfg["Ly"])
        self.kind = kl["type"]
        self.K = int(kl["n_modes"])
        s = float(kl["sigma_rad"]) if "sigma_rad" in kl else math.radians(kl["sigma_deg"])
        self.var = s * s
        if self.kind == "exp_separable":
            ax, ay = 0.5 * self.Lx, 0.5 * self.Ly
            nc = self.K + 2
            lx, wx, px = exp1d_eigen(ax, kl["corr_x"], nc)
            ly, wy, py = exp1d_eigen(ay, kl["corr_y"], nc)
            cand = [(self.var * lx[i] * ly[j], i, j) for i in range(nc) for j in range(nc)]
            cand.sort(key=lambda t: (-t[0], t[1] + t[2], t[1]))
            self.pairs = [(i, j) for _, i, j in cand[:self.K]]
            self.mu = np.array([m for m, _, _ in cand[:self.K]])
            self.mu_next = cand[self.K][0]
            self._x = (ax, wx, px)
            self._y = (ay, wy, py)
        elif self.kind == "matern32":
            self.length = float(kl["length"])
            nqx, nqy = kl["nystrom"]
            self.grid, self.wq = gauss_legendre_grid(self.Lx, self.Ly, nqx, nqy)
            mu_all, self.phi_grid, self.sign_projection = nystrom_eigen(
                self.kernel, self.grid, self.wq, self.K)
            self.all_mu = mu_all
            self.mu = mu_all[:self.K].copy()
            self.mu_next = mu_all[self.K]
        else:
            raise ValueError(f"unknown covariance {self.kind}")

    def kernel(self, P: np.ndarray, R: np.ndarray) -> np.ndarray:
        """Covariance ``k(p, r)`` between point sets (Matern-3/2, Euclidean distance)."""
        d = P[:, None, :] - R[None, :, :]
        return matern32(np.sqrt((d * d).sum(-1)), self.var, self.length)

    def modes_at(self, pts: np.ndarray) -> np.ndarray:
        """Normalised eigenfunctions ``phi_n`` at points ``[n, 2]`` -> ``[n, K]``."""
        pts = np.asarray(pts, dtype=np.float64).reshape(-1, 2)
        out = np.empty((len(pts), self.K))
        if self.kind == "exp_separable":
            ax, wx, px = self._x
            ay, wy, py = self._y
            xc = pts[:, 0] - ax
            yc = pts[:, 1] - ay
            for n, (i, j) in enumerate(self.pairs):
                out[:, n] = exp1d_mode(xc, ax, wx[i], px[i]) * exp1d_mode(yc, ay, wy[j], py[j])
            return out
        # Nystrom interpolation, in chunks to bound memory
        coef = self.phi_grid * self.wq[:, None]
        for s in range(0, len(pts), 4096):
            k = self.kernel(pts[s:s + 4096], self.grid)
            out[s:s + 4096] = (k @ coef) / self.mu[None, :]
        return out

    def field(self, pts: np.ndarray, xi_row: np.ndarray) -> np.ndarray:
        """Angle field (rad) at ``pts`` for one sample row ``[xi_1..xi_K, A, x0, w]``."""
        phi = self.modes_at(pts)
        val = phi @ (np.sqrt(self.mu) * xi_row[:self.K])
        return val + wrinkle(pts[:, 0], xi_row[self.K], xi_row[self.K + 1], xi_row[self.K + 2])


def wrinkle(x: np.ndarray, A: float, x0: float, w: float) -> np.ndarray:
    """``A sech^2((x - x0)/w)`` written with decaying exponentials only."""
    if A == 0.0:
        return np.zeros_like(x)
    e = np.exp(-2.0 * np.abs((x - x0) / w))
    return A * 4.0 * e / (1.0 + e) ** 2
