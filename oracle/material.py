"""Orthotropic ply stiffness and its rotation by the fibre angle.

Section 3.1 (Cosserat model) rotates the constitutive matrices by the local
misalignment angle with a strain transformation matrix.  The printed form
``(T)^-1 C T`` is not symmetric; the oracle uses the energy-consistent
rotation ``Qbar = T_eps^T Q T_eps`` (the standard result for engineering
strains), where ``T_eps`` maps global strains ``(eps_x, eps_y, gamma_xy)``
to fibre axes rotated by ``+theta`` from the x axis.
Section 4.1 uses the same rotated ply tensor ``Qbar^(k)`` inside the laminate
integrals of Eq. CLTABD.
"""
from __future__ import annotations

import numpy as np


def ply_Q(E11: float, E22: float, G12: float, nu12: float) -> np.ndarray:
    """Plane-stress reduced stiffness of one orthotropic ply in its own axes."""
    nu21 = nu12 * E22 / E11
    den = 1.0 - nu12 * nu21
    return np.array([[E11 / den, nu12 * E22 / den, 0.0],
                     [nu12 * E22 / den, E22 / den, 0.0],
                     [0.0, 0.0, G12]])


def T_eps(theta: float) -> np.ndarray:
    """Engineering-strain transformation from global axes to fibre axes at angle ``theta``."""
    c, s = np.cos(theta), np.sin(theta)
    return np.array([[c * c, s * s, c * s],
                     [s * s, c * c, -c * s],
                     [-2.0 * c * s, 2.0 * c * s, c * c - s * s]])


def Qbar(Q: np.ndarray, theta: float) -> np.ndarray:
    """Global-axes stiffness of a ply whose fibres make angle ``theta`` with x."""
    T = T_eps(theta)
    return T.T @ Q @ T


def material_from_cfg(cfg: dict) -> np.ndarray:
    m = cfg["material"]
    return ply_Q(m["E11"], m["E22"], m["G12"], m["nu12"])
