"""Laminated Reissner-Mindlin plate buckling (Section 4.1 of the paper).

* Classical laminate theory, Eq. CLTABD: ``A = sum Qbar_k (z_k - z_{k-1})``,
  ``B = 1/2 sum Qbar_k (z_k^2 - z_{k-1}^2)``, ``D = 1/3 sum Qbar_k (z_k^3 - z_{k-1}^3)``;
  plies listed bottom to top, the first at ``z = -t/2``; each ply angle is
  the pristine angle plus its sample's constant offset.
* Reissner-Mindlin plate with unknowns ``(u, v, w, theta_x, theta_y)`` per
  node (five per node, in-plane and bending coupled through ``B``);
  generalised strains ``eps = (u_x, v_y, u_y + v_x)``,
  ``kappa = (tx_x, ty_y, tx_y + ty_x)`` and transverse shear
  ``gamma = grad w - theta`` (Eq. momentequil / MomentWeakForm, shear
  stiffness ``k G t`` with ``k = 5/6``).
* Bilinear Q4 elements with selective reduced integration: membrane,
  coupling and bending terms with 2x2 Gauss points, the shear term with
  the single centre point (``"shear": "sri"``, the default).  For thick
  panels that one-point shear term leaves a checkerboard ``w`` mode with
  almost no energy, which becomes a spurious buckling mode; ``"shear":
  "mitc4"`` uses the assumed transverse shear strain of Bathe and Dvorkin's
  MITC4 element instead (``gamma_x`` sampled at the midpoints of the two
  edges along x and interpolated linearly across, ``gamma_y`` likewise
  between the midpoints of the edges along y; 2x2 Gauss points).
* ``"condensed": true`` is the decoupled model of Section 4.1: in-plane
  stress from ``A`` and moments from ``D* = D - B^T A^-1 B``, i.e. the
  element is built with ``(A, 0, D*)``; with a prescribed membrane load the
  in-plane unknowns then carry no geometric stiffness, so the buckling load
  equals that of the 3-unknown plate ``(w, theta_x, theta_y)`` with ``D*``.
* Geometric stiffness of a unit compressive edge load ``N0 = 1`` along x:
  ``K_G = int w_x w_x`` (2x2 Gauss).  The printed weak form uses
  ``sigma = diag(-1, 0)`` on the right-hand side, which would make the
  critical value negative; the load is taken as compressive so that the
  smallest positive ``lambda`` of ``K phi = lambda K_G phi`` (Eq. matrixeig)
  is the critical edge load in N/mm.
* Hard simply-supported edges: ``w = 0`` on all edges, the rotation
  tangential to each edge is zero (``theta_y`` on x = 0, a; ``theta_x`` on
  y = 0, b); in-plane rigid motions are removed by ``u = 0`` on x = 0 and
  ``v = 0`` on y = 0.

The paper's own panel (Test Problem II: 636 x 212 mm, eight 0.8 mm plies,
``"condensed": true``, ``"shear": "mitc4"``) reproduces the printed
pristine load of 278.59 kN to 0.17% at 128 x 128 when 0.8 mm is read as the
ply thickness and the load as the total edge force ``lambda L_y``; that is
pinned (tests/test_oracle_plate.py).  The 500 mm panel workload has no
printed value to pin against.
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np
import scipy.linalg as sla
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from .material import Qbar, ply_Q
from .mesh import GP_REF, Mesh, level_mesh, shape_q1

NDOF = 5


def laminate_abd(Q: np.ndarray, angles_rad, t_ply: float):
    """``(A, B, D)`` of a stack of identical plies at ``angles_rad`` (bottom first)."""
    n = len(angles_rad)
    z = -0.5 * n * t_ply + t_ply * np.arange(n + 1)
    A = np.zeros((3, 3))
    B = np.zeros((3, 3))
    D = np.zeros((3, 3))
    for k, th in enumerate(angles_rad):
        Qb = Qbar(Q, th)
        A += Qb * (z[k + 1] - z[k])
        B += Qb * (z[k + 1] ** 2 - z[k] ** 2) / 2.0
        D += Qb * (z[k + 1] ** 3 - z[k] ** 3) / 3.0
    return A, B, D


def _shear_rows(mesh: Mesh, xi: float, eta: float) -> np.ndarray:
    """Rows of ``gamma = grad w - theta`` (2 x 20) at a reference point."""
    N, dxi, deta = shape_q1(xi, eta)
    dNx, dNy = dxi / (0.5 * mesh.hx), deta / (0.5 * mesh.hy)
    Bs = np.zeros((2, 20))
    for a in range(4):
        Bs[0, 5 * a + 2] = dNx[a]
        Bs[0, 5 * a + 3] = -N[a]
        Bs[1, 5 * a + 2] = dNy[a]
        Bs[1, 5 * a + 4] = -N[a]
    return Bs


def plate_element(mesh: Mesh, A, B, D, As, shear: str = "sri"):
    """Element stiffness (20 x 20) and geometric stiffness (20 x 20) of one Q4 RM element."""
    jx, jy = 0.5 * mesh.hx, 0.5 * mesh.hy
    det = jx * jy
    Dmb = np.block([[A, B], [B, D]])
    Ke = np.zeros((20, 20))
    KG = np.zeros((20, 20))
    for xi, eta in GP_REF:
        N, dxi, deta = shape_q1(xi, eta)
        dNx, dNy = dxi / jx, deta / jy
        Bm = np.zeros((6, 20))
        for a in range(4):
            u, v, w, tx, ty = (5 * a + c for c in range(5))
            Bm[0, u] = dNx[a]
            Bm[1, v] = dNy[a]
            Bm[2, u] = dNy[a]
            Bm[2, v] = dNx[a]
            Bm[3, tx] = dNx[a]
            Bm[4, ty] = dNy[a]
            Bm[5, tx] = dNy[a]
            Bm[5, ty] = dNx[a]
        Ke += det * Bm.T @ Dmb @ Bm
        g = np.zeros(20)
        for a in range(4):
            g[5 * a + 2] = dNx[a]
        KG += det * np.outer(g, g)
    if shear == "sri":
        # transverse shear, one-point rule (weight 4)
        Bs = _shear_rows(mesh, 0.0, 0.0)
        Ke += 4.0 * det * Bs.T @ As @ Bs
    elif shear == "mitc4":
        # assumed shear strain: gamma_x tied at (0, -1), (0, 1), gamma_y at (-1, 0), (1, 0)
        gx_lo, gx_hi = _shear_rows(mesh, 0.0, -1.0)[0], _shear_rows(mesh, 0.0, 1.0)[0]
        gy_lo, gy_hi = _shear_rows(mesh, -1.0, 0.0)[1], _shear_rows(mesh, 1.0, 0.0)[1]
        for xi, eta in GP_REF:
            Bs = np.vstack([0.5 * (1 - eta) * gx_lo + 0.5 * (1 + eta) * gx_hi,
                            0.5 * (1 - xi) * gy_lo + 0.5 * (1 + xi) * gy_hi])
            Ke += det * Bs.T @ As @ Bs
    else:
        raise ValueError(f"unknown shear treatment {shear!r}")
    return Ke, KG


def plate_element_bending_only(mesh: Mesh, D, As, shear: str = "sri"):
    """3-dof element (w, theta_x, theta_y) with bending ``D`` only: the decoupled
    model of Section 4.1 (pass ``D*`` for the condensed laminate)."""
    Ke5, KG5 = plate_element(mesh, np.eye(3), np.zeros((3, 3)), D, As, shear)
    keep = [5 * a + c for a in range(4) for c in (2, 3, 4)]
    return Ke5[np.ix_(keep, keep)], KG5[np.ix_(keep, keep)]


def _assemble_uniform(mesh: Mesh, Ke, ndof):
    el = mesh.elements()
    dofs = (ndof * el[:, :, None] + np.arange(ndof)[None, None, :]).reshape(mesh.n_elem, 4 * ndof)
    nd = 4 * ndof
    rows = np.repeat(dofs, nd, axis=1).ravel()
    cols = np.tile(dofs, (1, nd)).ravel()
    vals = np.tile(Ke.ravel(), mesh.n_elem)
    n = ndof * mesh.n_nodes
    return sp.coo_matrix((vals, (rows, cols)), shape=(n, n)).tocsr()


def ss_constrained_dofs(mesh: Mesh, ndof: int = 5) -> np.ndarray:
    """Hard simply-supported constraints (see the module docstring)."""
    i, j = np.meshgrid(np.arange(mesh.nx + 1), np.arange(mesh.ny + 1))
    i, j = i.ravel(), j.ravel()
    nid = mesh.node_id(i, j)
    xedge = (i == 0) | (i == mesh.nx)
    yedge = (j == 0) | (j == mesh.ny)
    off = 2 if ndof == 5 else 0          # position of w
    c = [ndof * nid[xedge | yedge] + off,            # w
         ndof * nid[xedge] + off + 2,                # theta_y on x-edges
         ndof * nid[yedge] + off + 1]                # theta_x on y-edges
    if ndof == 5:
        c += [ndof * nid[i == 0] + 0,                # u on x = 0
              ndof * nid[j == 0] + 1]                # v on y = 0
    return np.unique(np.concatenate(c))


def condensed_bending(A, B, D):
    """``D* = D - B^T A^-1 B`` (Section 4.1, the decoupled model)."""
    return D - B.T @ np.linalg.solve(A, B)


@dataclass
class PlateSystem:
    K: sp.csr_matrix      # constrained stiffness (free dofs only)
    KG: sp.csr_matrix
    free: np.ndarray
    n_full: int


class PlateModel:
    """One level of the panel workload."""

    def __init__(self, cfg: dict, level: int):
        self.cfg = cfg
        self.level = level
        self.mesh = level_mesh(cfg, level)
        m = cfg["material"]
        self.Q = ply_Q(m["E11"], m["E22"], m["G12"], m["nu12"])
        self.t = cfg["ply_t"] * len(cfg["layup_deg"])
        self.As = cfg["shear_k"] * m["G12"] * self.t * np.eye(2)
        self.layup = np.radians(np.asarray(cfg["layup_deg"], float))

    def abd(self, offsets_rad):
        return laminate_abd(self.Q, self.layup + np.asarray(offsets_rad), self.cfg["ply_t"])

    def system(self, offsets_rad, ndof: int = 5) -> PlateSystem:
        A, B, D = self.abd(offsets_rad)
        shear = self.cfg.get("shear", "sri")
        if self.cfg.get("condensed", False):
            D, B = condensed_bending(A, B, D), np.zeros((3, 3))
        if ndof == 5:
            Ke, KGe = plate_element(self.mesh, A, B, D, self.As, shear)
        else:
            Ke, KGe = plate_element_bending_only(self.mesh, D, self.As, shear)
        K = _assemble_uniform(self.mesh, Ke, ndof)
        KG = _assemble_uniform(self.mesh, self.cfg.get("N0", 1.0) * KGe, ndof)
        con = ss_constrained_dofs(self.mesh, ndof)
        free = np.setdiff1d(np.arange(K.shape[0]), con)
        return PlateSystem(K[free][:, free].tocsr(), KG[free][:, free].tocsr(), free, K.shape[0])

    def buckling_load(self, offsets_rad, method: str = "eigsh", ndof: int = 5, k: int = 3):
        """Smallest positive ``lambda`` with ``K phi = lambda K_G phi`` (= 1 / largest
        eigenvalue ``mu`` of ``K_G phi = mu K phi``), in N/mm of edge load."""
        s = self.system(offsets_rad, ndof)
        if method == "dense":
            mu = sla.eigh(s.KG.toarray(), s.K.toarray(), eigvals_only=True)
            return 1.0 / mu.max()
        lu = spla.splu(s.K.tocsc())
        Minv = spla.LinearOperator(s.K.shape, matvec=lu.solve)
        vals = spla.eigsh(s.KG, k=k, M=s.K, Minv=Minv, which="LA", tol=1e-14,
                          return_eigenvectors=False, maxiter=20000)
        return 1.0 / np.max(vals)


def eigen_count_below(K: sp.spmatrix, KG: sp.spmatrix, sigma: float) -> int:
    """Number of eigenvalues ``lambda < sigma`` of ``K phi = lambda K_G phi``
    (Eq. matrixeig), by Sylvester's law of inertia: with ``K`` positive
    definite it equals the number of negative eigenvalues of
    ``K - sigma K_G``, read off the block-diagonal factor of a symmetric
    indefinite (Bunch-Kaufman) LDL^T factorisation of the dense matrix.  Small
    meshes only (dense, O(n^3))."""
    A = (K - sigma * KG).toarray()
    _, D, _ = sla.ldl(A, lower=True)
    n = D.shape[0]
    neg, i = 0, 0
    while i < n:
        if i + 1 < n and D[i + 1, i] != 0.0:
            neg += int(np.sum(np.linalg.eigvalsh(D[i:i + 2, i:i + 2]) < 0.0))
            i += 2
        else:
            neg += int(D[i, i] < 0.0)
            i += 1
    return neg


def navier_orthotropic(D: np.ndarray, a: float, b: float, m_max: int = 20) -> float:
    """Kirchhoff buckling load of a specially orthotropic simply-supported plate under
    uniaxial ``N_x`` (Navier solution, one half-wave across ``b``):
    ``N = pi^2/b^2 min_m [D11 (m b/a)^2 + 2 (D12 + 2 D66) + D22 (a/(m b))^2]``."""
    best = math.inf
    for m in range(1, m_max + 1):
        r = m * b / a
        best = min(best, math.pi ** 2 / b ** 2 * (D[0, 0] * r * r + 2 * (D[0, 1] + 2 * D[2, 2]) + D[1, 1] / (r * r)))
    return best
