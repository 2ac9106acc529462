"""Structured quadrilateral meshes and their uniform refinement.

Follows Section 2.3 (implementation of MLMC): the level hierarchy is made by
uniform refinement, the element size halving from one level to the next,
so that the number of unknowns grows by ``m = 4`` per level in 2-D.

Numbering (shared convention of the whole project, a layout choice, not
arithmetic): node ``(i, j)`` has id ``j * (nx + 1) + i``; element
``(ex, ey)`` has id ``ey * nx + ex`` and local nodes
``(ex, ey), (ex+1, ey), (ex+1, ey+1), (ex, ey+1)``; the 2x2 Gauss points of
an element are ordered ``(-,-), (+,-), (-,+), (+,+)`` in reference
coordinates ``(xi, eta)``.
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np

GAUSS_2 = (-1.0 / math.sqrt(3.0), 1.0 / math.sqrt(3.0))
# reference coordinates of the 2x2 Gauss points in the project order
GP_REF = [(GAUSS_2[0], GAUSS_2[0]), (GAUSS_2[1], GAUSS_2[0]),
          (GAUSS_2[0], GAUSS_2[1]), (GAUSS_2[1], GAUSS_2[1])]
# reference coordinates of the four element nodes (counter-clockwise)
NODE_REF = [(-1.0, -1.0), (1.0, -1.0), (1.0, 1.0), (-1.0, 1.0)]


@dataclass(frozen=True)
class Mesh:
    Lx: float
    Ly: float
    nx: int
    ny: int

    @property
    def hx(self) -> float:
        return self.Lx / self.nx

    @property
    def hy(self) -> float:
        return self.Ly / self.ny

    @property
    def n_nodes(self) -> int:
        return (self.nx + 1) * (self.ny + 1)

    @property
    def n_elem(self) -> int:
        return self.nx * self.ny

    def node_id(self, i, j):
        return j * (self.nx + 1) + i

    def node_xy(self) -> np.ndarray:
        i = np.arange(self.nx + 1)
        j = np.arange(self.ny + 1)
        X, Y = np.meshgrid(i * self.hx, j * self.hy)
        return np.stack([X.ravel(), Y.ravel()], axis=1)

    def elements(self) -> np.ndarray:
        """``[n_elem, 4]`` node ids, counter-clockwise from the lower-left node."""
        ex, ey = np.meshgrid(np.arange(self.nx), np.arange(self.ny))
        ex, ey = ex.ravel(), ey.ravel()
        n0 = self.node_id(ex, ey)
        return np.stack([n0, n0 + 1, n0 + self.nx + 2, n0 + self.nx + 1], axis=1)

    def element_origin(self) -> np.ndarray:
        ex, ey = np.meshgrid(np.arange(self.nx), np.arange(self.ny))
        return np.stack([ex.ravel() * self.hx, ey.ravel() * self.hy], axis=1)

    def element_centroids(self) -> np.ndarray:
        return self.element_origin() + 0.5 * np.array([self.hx, self.hy])

    def gauss_points(self) -> np.ndarray:
        """Physical coordinates of the 2x2 Gauss points, ``[n_elem, 4, 2]``."""
        o = self.element_origin()
        out = np.empty((self.n_elem, 4, 2))
        for q, (xi, eta) in enumerate(GP_REF):
            out[:, q, 0] = o[:, 0] + 0.5 * (1.0 + xi) * self.hx
            out[:, q, 1] = o[:, 1] + 0.5 * (1.0 + eta) * self.hy
        return out


def level_mesh(cfg: dict, level: int) -> Mesh:
    """Mesh of ``level``: the level-0 mesh refined ``level`` times (h_l = 2^-l h_0)."""
    if "Lx" in cfg:
        return Mesh(cfg["Lx"], cfg["Ly"], cfg["nx0"] << level, cfg["ny0"] << level)
    return Mesh(cfg["a"], cfg["b"], cfg["nx0"] << level, cfg["ny0"] << level)


def shape_q1(xi: float, eta: float):
    """Bilinear shape functions and their reference derivatives at (xi, eta)."""
    N = np.array([0.25 * (1 + a * xi) * (1 + b * eta) for a, b in NODE_REF])
    dxi = np.array([0.25 * a * (1 + b * eta) for a, b in NODE_REF])
    deta = np.array([0.25 * b * (1 + a * xi) for a, b in NODE_REF])
    return N, dxi, deta
