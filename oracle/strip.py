"""Plane-stress orthotropic strip: Q1 finite elements, PCG, QoI.

Follows Section 3.1 of the paper: bilinear quadrilateral elements on a
uniformly refined mesh give a linear system ``K d = f`` (Eq.
matrixinplane) whose load comes from the prescribed end-shortening (the
Dirichlet conditions of Test I), with a misalignment-dependent rotated
stiffness at every integration point.  The workloads here use the
two-unknown plane-stress form of that model (``u, v`` per node); the
quantity of interest keeps the paper's idea of a maximum over the
integration points of the elements in a central sub-region, here of the
compressive stress along the local fibre direction.

Element stiffness ``K_e = sum_q w_q det(J) B_q^T Qbar(theta_q) B_q`` with
2x2 Gauss quadrature; ``theta_q`` is the angle field at Gauss point ``q``.
Unknowns are interleaved per node, ``(u, v)``.

Boundary conditions of the workloads: ``u = v = 0`` on ``x = 0`` and
``u = -delta`` on ``x = Lx``; other boundary dofs are free.  The system is
solved for the free dofs, ``K_ff d_f = -K_fc g_c``.

Solvers: Jacobi-preconditioned CG on ``K_ff`` from ``x_0 = 0``, stopped
when the recursively updated residual satisfies ``||r||_2 <= rtol ||b||_2``;
and a sparse direct LU solve.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from .material import Qbar, T_eps, material_from_cfg
from .mesh import GP_REF, Mesh, level_mesh, shape_q1


def strain_matrices(mesh: Mesh):
    """``B_q`` (3 x 8) and ``w_q det J`` for the four Gauss points of a rectangle."""
    Bs, wdet = [], []
    jx, jy = 0.5 * mesh.hx, 0.5 * mesh.hy          # dx/dxi, dy/deta
    for xi, eta in GP_REF:
        _, dxi, deta = shape_q1(xi, eta)
        dNx, dNy = dxi / jx, deta / jy
        B = np.zeros((3, 8))
        B[0, 0::2] = dNx
        B[1, 1::2] = dNy
        B[2, 0::2] = dNy
        B[2, 1::2] = dNx
        Bs.append(B)
        wdet.append(1.0 * 1.0 * jx * jy)
    return Bs, wdet


def element_stiffness(mesh: Mesh, Q: np.ndarray, theta4) -> np.ndarray:
    Bs, wdet = strain_matrices(mesh)
    Ke = np.zeros((8, 8))
    for q in range(4):
        Ke += wdet[q] * Bs[q].T @ Qbar(Q, theta4[q]) @ Bs[q]
    return Ke


def element_dofs(mesh: Mesh) -> np.ndarray:
    el = mesh.elements()
    d = np.empty((mesh.n_elem, 8), dtype=np.int64)
    d[:, 0::2] = 2 * el
    d[:, 1::2] = 2 * el + 1
    return d


def T_eps_batch(theta: np.ndarray) -> np.ndarray:
    """``T_eps`` for an array of angles, shape ``theta.shape + (3, 3)``."""
    c, s = np.cos(theta), np.sin(theta)
    T = np.empty(theta.shape + (3, 3))
    T[..., 0, 0], T[..., 0, 1], T[..., 0, 2] = c * c, s * s, c * s
    T[..., 1, 0], T[..., 1, 1], T[..., 1, 2] = s * s, c * c, -c * s
    T[..., 2, 0], T[..., 2, 1], T[..., 2, 2] = -2 * c * s, 2 * c * s, c * c - s * s
    return T


def element_matrices(mesh: Mesh, Q: np.ndarray, theta: np.ndarray) -> np.ndarray:
    """All element stiffness matrices ``[n_elem, 8, 8]``:
    ``K_e = sum_q w_q det J B_q^T (T_q^T Q T_q) B_q``."""
    theta = np.asarray(theta).reshape(mesh.n_elem, 4)
    Bs, wdet = strain_matrices(mesh)
    T = T_eps_batch(theta)                                   # [E, 4, 3, 3]
    Qb = np.einsum("eqji,jk,eqkl->eqil", T, Q, T)            # T^T Q T
    Ke = np.zeros((mesh.n_elem, 8, 8))
    for q in range(4):
        Ke += wdet[q] * np.einsum("ia,eij,jb->eab", Bs[q], Qb[:, q], Bs[q])
    return Ke


def assemble(mesh: Mesh, Q: np.ndarray, theta: np.ndarray) -> sp.csr_matrix:
    """Global stiffness ``K`` (CSR, unconstrained) for angles ``theta[n_elem, 4]``."""
    dofs = element_dofs(mesh)
    vals = element_matrices(mesh, Q, theta)
    rows = np.repeat(dofs, 8, axis=1).ravel()
    cols = np.tile(dofs, (1, 8)).ravel()
    n = 2 * mesh.n_nodes
    return sp.coo_matrix((vals.ravel(), (rows, cols)), shape=(n, n)).tocsr()


@dataclass
class Dirichlet:
    dofs: np.ndarray      # constrained dof ids (sorted)
    values: np.ndarray    # prescribed values, same length


def strip_bcs(mesh: Mesh, delta: float) -> Dirichlet:
    """Left edge clamped (u = v = 0), right edge ``u = -delta``."""
    j = np.arange(mesh.ny + 1)
    left = mesh.node_id(0, j)
    right = mesh.node_id(mesh.nx, j)
    dofs = np.concatenate([2 * left, 2 * left + 1, 2 * right])
    vals = np.concatenate([np.zeros(2 * len(left)), np.full(len(right), -delta)])
    o = np.argsort(dofs)
    return Dirichlet(dofs[o], vals[o])


def reduce_system(K: sp.csr_matrix, bc: Dirichlet):
    n = K.shape[0]
    free = np.setdiff1d(np.arange(n), bc.dofs)
    Kff = K[free][:, free].tocsr()
    Kfc = K[free][:, bc.dofs]
    b = -(Kfc @ bc.values)
    return free, Kff, b


@dataclass
class PCGResult:
    x: np.ndarray
    iters: int
    relres: float          # recursive ||r|| / ||b||
    true_relres: float     # ||b - A x|| / ||b||
    converged: bool


def jacobi_pcg(A: sp.csr_matrix, b: np.ndarray, rtol: float, max_iter: int = 100000) -> PCGResult:
    """Textbook preconditioned CG with ``M = diag(A)``, ``x_0 = 0``."""
    dinv = 1.0 / A.diagonal()
    x = np.zeros_like(b)
    r = b.copy()
    bnorm = np.linalg.norm(b)
    if bnorm == 0.0:
        return PCGResult(x, 0, 0.0, 0.0, True)
    z = dinv * r
    p = z.copy()
    rz = r @ z
    it = 0
    rn = bnorm
    while it < max_iter:
        if rn <= rtol * bnorm:
            break
        Ap = A @ p
        alpha = rz / (p @ Ap)
        x += alpha * p
        r -= alpha * Ap
        rn = np.linalg.norm(r)
        it += 1
        z = dinv * r
        rz_new = r @ z
        beta = rz_new / rz
        rz = rz_new
        p = z + beta * p
    tr = np.linalg.norm(b - A @ x) / bnorm
    return PCGResult(x, it, rn / bnorm, tr, rn <= rtol * bnorm)


def sample_theta(kl, mesh: Mesh, xi_row: np.ndarray) -> np.ndarray:
    """Angle field at the 2x2 Gauss points of every element, ``[n_elem, 4]``."""
    gp = mesh.gauss_points().reshape(-1, 2)
    return kl.field(gp, xi_row).reshape(mesh.n_elem, 4)


def in_region(mesh: Mesh, region) -> np.ndarray:
    """Elements whose centroid lies inside ``[x0, x1] x [y0, y1]``."""
    c = mesh.element_centroids()
    x0, x1, y0, y1 = region
    return (c[:, 0] >= x0) & (c[:, 0] <= x1) & (c[:, 1] >= y0) & (c[:, 1] <= y1)


def fibre_stress_qoi(mesh: Mesh, Q: np.ndarray, theta: np.ndarray, d: np.ndarray, region) -> float:
    """Maximum compressive stress along the local fibre direction, ``max(-sigma_11)``,
    over the Gauss points of the elements whose centroid is in ``region``.
    ``sigma_11`` is the first component of the material-axes stress
    ``Q T_eps(theta_q) B_q d_e``."""
    theta = np.asarray(theta).reshape(mesh.n_elem, 4)
    Bs, _ = strain_matrices(mesh)
    dofs = element_dofs(mesh)
    sel = np.nonzero(in_region(mesh, region))[0]
    de = d[dofs[sel]]                                        # [S, 8]
    best = -np.inf
    for q in range(4):
        eps = de @ Bs[q].T                                   # [S, 3]
        T = T_eps_batch(theta[sel, q])                       # [S, 3, 3]
        sig_mat = np.einsum("ij,sjk,sk->si", Q, T, eps)
        best = max(best, float(np.max(-sig_mat[:, 0])))
    return best


@dataclass
class StripSolve:
    q: float
    iters: int
    relres: float
    true_relres: float
    converged: bool
    d: np.ndarray
    theta: np.ndarray


class StripModel:
    """One level of the strip workload: mesh, material, KL field, BCs."""

    def __init__(self, cfg: dict, level: int, kl=None):
        from .kl import KL
        self.cfg = cfg
        self.level = level
        self.mesh = level_mesh(cfg, level)
        self.Q = material_from_cfg(cfg)
        self.kl = kl if kl is not None else KL(cfg)
        self.bc = strip_bcs(self.mesh, cfg["delta"])
        self.region = cfg["qoi_region"]
        self._modes = None

    def modes(self) -> np.ndarray:
        """Eigenfunctions at this level's Gauss points ``[n_elem * 4, K]`` (they do
        not depend on the sample, so they are evaluated once per level)."""
        if self._modes is None:
            self._modes = self.kl.modes_at(self.mesh.gauss_points().reshape(-1, 2))
        return self._modes

    def theta(self, xi_row: np.ndarray) -> np.ndarray:
        """Angle field at the Gauss points, ``[n_elem, 4]`` (Eq. inftyKL, truncated)."""
        K = self.kl.K
        val = self.modes() @ (np.sqrt(self.kl.mu) * xi_row[:K])
        gx = self.mesh.gauss_points().reshape(-1, 2)[:, 0]
        from .kl import wrinkle
        val = val + wrinkle(gx, xi_row[K], xi_row[K + 1], xi_row[K + 2])
        return val.reshape(self.mesh.n_elem, 4)

    def solve_theta(self, theta: np.ndarray, method: str = "pcg", rtol: float = None,
                    max_iter: int = None) -> StripSolve:
        rtol = self.cfg["rtol"] if rtol is None else rtol
        max_iter = self.cfg.get("max_iter", 100000) if max_iter is None else max_iter
        K = assemble(self.mesh, self.Q, theta)
        free, Kff, b = reduce_system(K, self.bc)
        if method == "pcg":
            res = jacobi_pcg(Kff, b, rtol, max_iter)
            xf, it, rr, tr, ok = res.x, res.iters, res.relres, res.true_relres, res.converged
        elif method == "direct":
            xf = spla.splu(Kff.tocsc()).solve(b)
            it, ok = 0, True
            rr = tr = np.linalg.norm(b - Kff @ xf) / np.linalg.norm(b)
        else:
            raise ValueError(method)
        d = np.zeros(K.shape[0])
        d[free] = xf
        d[self.bc.dofs] = self.bc.values
        q = fibre_stress_qoi(self.mesh, self.Q, theta, d, self.region)
        return StripSolve(q, it, rr, tr, ok, d, theta)

    def solve(self, xi_row: np.ndarray, method: str = "pcg", rtol: float = None) -> StripSolve:
        return self.solve_theta(self.theta(xi_row), method, rtol)
