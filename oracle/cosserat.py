"""Cosserat continuum model of Test Problem I (Section 3.1 of the paper).

Test infrastructure: a plain FP64 implementation used only by the tests, the
smoke check and the CPU baseline of the benchmark.

Model, as Section 3.1 states it:

* a square domain ``[0, L]^2`` of unidirectional prepreg whose fibres make
  the random angle ``Phi(x)`` with the x axis (Eq. covarianceFunction, a
  separable exponential field, expanded by Eq. inftyKL and truncated after
  ``N_KL = 50 + 50 l`` terms on level ``l``);
* plane strain with three unknowns per node, the displacements ``u, v``
  and the independent Cosserat rotation ``theta_3``;
* Cosserat strains ``eps_ij = du_i/dx_j + e_ij3 theta_3`` and curvatures
  ``kappa_j = d theta_3 / dx_j``, i.e. ``eps_11 = u_x``, ``eps_22 = v_y``,
  ``eps_12 = u_y + theta_3``, ``eps_21 = v_x - theta_3``;
* stresses ``sigma = C* eps`` and couple stresses ``m = D* kappa`` with the
  fibre-frame matrices ``C, D`` rotated by ``Phi``: ``C* = T^-1 C T`` and
  ``D* = R^-1 D R`` (Section 3.1).  Here ``T`` rotates the (non-symmetric)
  strain tensor, ``eps' = R eps R^T`` written on the four components
  ``(11, 22, 12, 21)``, and ``R`` the curvature vector; both are orthogonal,
  so ``T^-1 = T^T`` and the rotated matrices stay symmetric;
* the weak form Eq. VarCosserat discretised with bilinear elements for all
  three fields and 2x2 Gauss quadrature, giving ``K d = f``
  (Eq. matrixinplane) with ``M = 3 nnode`` unknowns (243 on the 8 x 8
  level-0 mesh);
* boundary conditions ``u = 0`` on ``x = 0``, ``u = Delta < 0`` on
  ``x = L``, ``v = 0`` on ``y = 0`` and ``y = L``; ``theta_3`` is free;
* quantity of interest, Eq. failureCriterion: the effective stress
  ``tau_e = sqrt(sigma_12^2 + (sigma_22 / R)^2)`` in fibre axes, its
  ratio ``f = tau_e / tau_y`` maximised over the Gauss points of the
  elements inside the central square ``Omega'`` (side ``L / 2``), and the
  compressive strength from the mean axial stress over ``Omega'``.

Readings where the paper is silent or garbled (the constitutive matrices
come from another paper of the authors and are not printed):

* fibre-frame ``C`` on ``(eps_11, eps_22, eps_12, eps_21)`` is
  ``[[Q11, Q12, 0, 0], [Q12, Q22, 0, 0], [0, 0, G_par, 0], [0, 0, 0, G_orth]]``:
  the reduced orthotropic stiffness from rule-of-mixtures constants of the
  given fibre and matrix moduli (``E_1 = v_f E_f + (1 - v_f) E_m``,
  ``1/E_2 = v_f/E_f + (1 - v_f)/E_m``, ``nu_12`` from the workload), a
  shear stiffness parallel to the fibres from the inverse rule of mixtures
  of the shear moduli (matrix dominated) and one orthogonal to them from
  the direct rule (fibre dominated), about five times larger, so the
  stress is not symmetric, as Section 3.1 describes;
* ``D = diag(v_f E_f d^2 / 16, (1 - v_f) E_m d^2 / 16)``: the bending
  stiffness of circular fibres of diameter ``d`` per unit area for
  rotation gradients along the fibres, and the matrix's across them;
* ``sigma_12`` in ``tau_e`` is the fibre-frame shear stress conjugate to
  ``eps_12`` (sliding along the fibres), ``R`` comes from the workload;
* the printed strength ``sigma = f* / |Omega'| int sigma_x`` scales the
  mean stress by ``f*``; since the problem is linear, the load at which
  ``tau_e`` first reaches ``tau_y`` is the applied one divided by ``f*``,
  so the strength is ``-(1 / f*) (1 / |Omega'|) int sigma_x`` (positive in
  compression, independent of ``Delta``).
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from .mesh import GP_REF, Mesh, level_mesh, shape_q1
from .strip import Dirichlet, jacobi_pcg, reduce_system

NDOF = 3


# ---------------------------------------------------------------- material
def fibre_frame_matrices(fib: dict):
    """``(C [4x4], D [2x2])`` in fibre axes from the constituent constants."""
    vf, Ef, Em, Gf, Gm, d = fib["v_f"], fib["E_f"], fib["E_m"], fib["G_f"], fib["G_m"], fib["d"]
    E1 = vf * Ef + (1.0 - vf) * Em
    E2 = 1.0 / (vf / Ef + (1.0 - vf) / Em)
    nu12 = fib["nu12"]
    nu21 = nu12 * E2 / E1
    den = 1.0 - nu12 * nu21
    g_par = 1.0 / (vf / Gf + (1.0 - vf) / Gm)
    g_orth = vf * Gf + (1.0 - vf) * Gm
    C = np.array([[E1 / den, nu12 * E2 / den, 0.0, 0.0],
                  [nu12 * E2 / den, E2 / den, 0.0, 0.0],
                  [0.0, 0.0, g_par, 0.0],
                  [0.0, 0.0, 0.0, g_orth]])
    D = np.diag([vf * Ef * d * d / 16.0, (1.0 - vf) * Em * d * d / 16.0])
    return C, D


def rotation_2(phi: float) -> np.ndarray:
    """Rows are the fibre axes ``(cos phi, sin phi)`` and ``(-sin phi, cos phi)``."""
    c, s = math.cos(phi), math.sin(phi)
    return np.array([[c, s], [-s, c]])


# component order of the strain and stress vectors
PAIRS = [(0, 0), (1, 1), (0, 1), (1, 0)]


def rotation_4(phi: float) -> np.ndarray:
    """``T`` with ``eps'_v = T eps_v`` for ``eps' = R eps R^T`` on the components ``(11, 22, 12, 21)``."""
    R = rotation_2(phi)
    T = np.empty((4, 4))
    for p, (i, j) in enumerate(PAIRS):
        for q, (a, b) in enumerate(PAIRS):
            T[p, q] = R[i, a] * R[j, b]
    return T


def rotated_matrices(C: np.ndarray, D: np.ndarray, phi: float):
    """``C* = T^-1 C T`` and ``D* = R^-1 D R`` (Section 3.1)."""
    T = rotation_4(phi)
    R = rotation_2(phi)
    return np.linalg.solve(T, C @ T), np.linalg.solve(R, D @ R)


# ---------------------------------------------------------------- element
def strain_operators(mesh: Mesh):
    """Per Gauss point: ``Be`` (4 x 12) giving ``(eps_11, eps_22, eps_12, eps_21)``,
    ``Bk`` (2 x 12) giving ``(kappa_1, kappa_2)`` from the element unknowns
    ``(u, v, theta_3)`` of its four nodes, and the weight ``w det J``."""
    jx, jy = 0.5 * mesh.hx, 0.5 * mesh.hy
    out = []
    for xi, eta in GP_REF:
        N, dxi, deta = shape_q1(xi, eta)
        dNx, dNy = dxi / jx, deta / jy
        Be = np.zeros((4, 12))
        Bk = np.zeros((2, 12))
        for a in range(4):
            u, v, t = 3 * a, 3 * a + 1, 3 * a + 2
            Be[0, u] = dNx[a]          # u_x
            Be[1, v] = dNy[a]          # v_y
            Be[2, u] = dNy[a]          # u_y + theta_3
            Be[2, t] = N[a]
            Be[3, v] = dNx[a]          # v_x - theta_3
            Be[3, t] = -N[a]
            Bk[0, t] = dNx[a]
            Bk[1, t] = dNy[a]
        out.append((Be, Bk, jx * jy))
    return out


def element_stiffness(mesh: Mesh, C: np.ndarray, D: np.ndarray, phi4) -> np.ndarray:
    """``K_e = sum_q w_q det J (Be^T C*(phi_q) Be + Bk^T D*(phi_q) Bk)``."""
    Ke = np.zeros((12, 12))
    for q, (Be, Bk, w) in enumerate(strain_operators(mesh)):
        Cs, Ds = rotated_matrices(C, D, phi4[q])
        Ke += w * (Be.T @ Cs @ Be + Bk.T @ Ds @ Bk)
    return Ke


def element_dofs(mesh: Mesh) -> np.ndarray:
    el = mesh.elements()
    return (NDOF * el[:, :, None] + np.arange(NDOF)[None, None, :]).reshape(len(el), 12)


def assemble(mesh: Mesh, C: np.ndarray, D: np.ndarray, theta: np.ndarray) -> sp.csr_matrix:
    """Global ``K`` (unknowns ``(u, v, theta_3)`` per node) for angles ``theta [n_elem, 4]``."""
    dofs = element_dofs(mesh)
    rows, cols, vals = [], [], []
    for e in range(mesh.n_elem):
        Ke = element_stiffness(mesh, C, D, theta[e])
        rows.append(np.repeat(dofs[e], 12))
        cols.append(np.tile(dofs[e], 12))
        vals.append(Ke.ravel())
    n = NDOF * mesh.n_nodes
    K = sp.coo_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))), shape=(n, n))
    return K.tocsr()


def cosserat_bcs(mesh: Mesh, delta: float) -> Dirichlet:
    """``u = 0`` on x = 0, ``u = delta`` on x = L, ``v = 0`` on y = 0 and y = L."""
    nnx = mesh.nx + 1
    dofs, vals = {}, {}
    for j in range(mesh.ny + 1):
        dofs[NDOF * (j * nnx)] = 0.0
        dofs[NDOF * (j * nnx + mesh.nx)] = delta
    for i in range(nnx):
        dofs[NDOF * i + 1] = 0.0
        dofs[NDOF * (mesh.ny * nnx + i) + 1] = 0.0
    keys = np.array(sorted(dofs))
    return Dirichlet(keys, np.array([dofs[k] for k in keys]))


# ---------------------------------------------------------------- quantity of interest
def in_region(mesh: Mesh, region) -> np.ndarray:
    """Elements whose centroid lies in ``[x0, x1] x [y0, y1]`` (with edges on the
    region's sides these are the elements contained in it)."""
    c = mesh.element_centroids()
    x0, x1, y0, y1 = region
    return (c[:, 0] >= x0) & (c[:, 0] <= x1) & (c[:, 1] >= y0) & (c[:, 1] <= y1)


def gauss_point_stresses(mesh: Mesh, C: np.ndarray, D: np.ndarray, theta: np.ndarray, d: np.ndarray):
    """Global stresses ``(s11, s22, s12, s21)`` at every Gauss point, ``[n_elem, 4, 4]``."""
    dofs = element_dofs(mesh)
    de = d[dofs]
    ops = strain_operators(mesh)
    out = np.empty((mesh.n_elem, 4, 4))
    for e in range(mesh.n_elem):
        for q, (Be, _, _) in enumerate(ops):
            Cs, _ = rotated_matrices(C, D, theta[e, q])
            out[e, q] = Cs @ (Be @ de[e])
    return out


def strength_qoi(mesh: Mesh, C: np.ndarray, D: np.ndarray, theta: np.ndarray, d: np.ndarray, region,
                 R: float, tau_y: float):
    """Eq. failureCriterion: returns ``(strength, f_star, mean_sigma_x)``."""
    sig = gauss_point_stresses(mesh, C, D, theta, d)
    sel = np.nonzero(in_region(mesh, region))[0]
    f_star = 0.0
    integral = 0.0
    area = 0.0
    w = 0.25 * mesh.hx * mesh.hy     # 2x2 Gauss weight times det J
    for e in sel:
        for q in range(4):
            loc = rotation_4(theta[e, q]) @ sig[e, q]      # fibre-frame (11, 22, 12, 21)
            tau_e = math.sqrt(loc[2] ** 2 + (loc[1] / R) ** 2)
            f_star = max(f_star, tau_e / tau_y)
            integral += w * sig[e, q, 0]
            area += w
    mean_sx = integral / area
    return -mean_sx / f_star, f_star, mean_sx


# ---------------------------------------------------------------- model
def modes_on_level(cfg: dict, level: int) -> int:
    """``N_KL`` of ``level`` (Section 3.2: ``50 + 50 l``, from the workload's ``modes_per_level``)."""
    base, step = cfg["kl"]["modes_per_level"]
    return min(int(base + step * level), int(cfg["kl"]["n_modes"]))


@dataclass
class CosseratSolve:
    q: float
    f_star: float
    mean_sigma_x: float
    iters: int
    relres: float
    true_relres: float
    converged: bool
    d: np.ndarray


class CosseratModel:
    """One level of the Cosserat workload."""

    def __init__(self, cfg: dict, level: int, kl=None):
        from .kl import KL
        self.cfg = cfg
        self.level = level
        self.mesh = level_mesh(cfg, level)
        self.C, self.D = fibre_frame_matrices(cfg["fibre"])
        self.kl = KL(cfg) if kl is None else kl
        self.n_modes = modes_on_level(cfg, level)
        self.bc = cosserat_bcs(self.mesh, cfg["delta"])
        self.region = cfg["qoi_region"]
        self._modes = None

    def modes(self) -> np.ndarray:
        if self._modes is None:
            self._modes = self.kl.modes_at(self.mesh.gauss_points().reshape(-1, 2))[:, :self.n_modes]
        return self._modes

    def theta(self, xi_row: np.ndarray) -> np.ndarray:
        """Angles at the Gauss points ``[n_elem, 4]``: Eq. inftyKL with this level's ``N_KL`` terms."""
        k = self.n_modes
        val = self.modes() @ (np.sqrt(self.kl.mu[:k]) * xi_row[:k])
        return val.reshape(self.mesh.n_elem, 4)

    def solve_theta(self, theta: np.ndarray, method: str = "pcg", rtol: float = None) -> CosseratSolve:
        rtol = self.cfg["rtol"] if rtol is None else rtol
        K = assemble(self.mesh, self.C, self.D, theta)
        free, Kff, b = reduce_system(K, self.bc)
        if method == "pcg":
            res = jacobi_pcg(Kff, b, rtol, self.cfg.get("max_iter", 100000))
            xf, it, rr, tr, ok = res.x, res.iters, res.relres, res.true_relres, res.converged
        elif method == "direct":
            xf = spla.splu(Kff.tocsc()).solve(b)
            it, ok = 0, True
            rr = tr = float(np.linalg.norm(b - Kff @ xf) / np.linalg.norm(b))
        else:
            raise ValueError(method)
        d = np.zeros(K.shape[0])
        d[free] = xf
        d[self.bc.dofs] = self.bc.values
        fib = self.cfg["fibre"]
        q, f_star, msx = strength_qoi(self.mesh, self.C, self.D, theta, d, self.region, fib["R"], fib["tau_c"])
        return CosseratSolve(q, f_star, msx, it, rr, tr, ok, d)

    def solve(self, xi_row: np.ndarray, method: str = "pcg", rtol: float = None) -> CosseratSolve:
        return self.solve_theta(self.theta(xi_row), method, rtol)
