"""Pins of the oracle's plate model (Section 4.1) and of Algorithm 2 (Section 2.4)."""
import math

import numpy as np
import pytest

import mlmc_inputs as mi
from oracle.mesh import Mesh
from oracle.plate import (PlateModel, laminate_abd, navier_orthotropic, plate_element)
from oracle.sr import indicator, sr_chain, sr_pair

C4 = mi.load_config("plate_c4")


def test_abd_closed_forms():
    m = PlateModel(C4, 0)
    # a single-angle stack is homogeneous: A = Q t, B = 0, D = Q t^3 / 12
    from oracle.material import Qbar
    A, B, D = laminate_abd(m.Q, [0.3] * 8, 0.125)
    Qb = Qbar(m.Q, 0.3)
    np.testing.assert_allclose(A, Qb * 1.0, rtol=1e-13)
    assert np.abs(B).max() < 1e-12 * np.abs(A).max()
    np.testing.assert_allclose(D, Qb / 12.0, rtol=1e-12)
    # symmetric pristine layup: B = 0
    A, B, D = m.abd(np.zeros(8))
    assert np.abs(B).max() < 1e-10
    # an unsymmetric perturbation gives B != 0
    _, B2, _ = m.abd(np.radians([3, 0, 0, 0, 0, 0, 0, 0]))
    assert np.abs(B2).max() > 1.0


def test_element_symmetry_and_rigid_modes():
    mesh = Mesh(10.0, 10.0, 1, 1)
    m = PlateModel(C4, 0)
    A, B, D = m.abd(np.radians([2, -1, 3, 0, 1, -2, 0, 1]))
    Ke, KG = plate_element(mesh, A, B, D, m.As)
    np.testing.assert_allclose(Ke, Ke.T, atol=1e-9 * np.abs(Ke).max())
    xy = mesh.node_xy()[mesh.elements()[0]]
    modes = []
    for a in range(4):
        pass
    def vec(f):
        v = np.zeros(20)
        for a in range(4):
            v[5 * a:5 * a + 5] = f(*xy[a])
        return v
    rigid = [vec(lambda x, y: [1, 0, 0, 0, 0]), vec(lambda x, y: [0, 1, 0, 0, 0]),
             vec(lambda x, y: [-y, x, 0, 0, 0]), vec(lambda x, y: [0, 0, 1, 0, 0]),
             vec(lambda x, y: [0, 0, x, 1, 0]), vec(lambda x, y: [0, 0, y, 0, 1])]
    for v in rigid:
        assert np.abs(Ke @ v).max() < 1e-9 * np.abs(Ke).max()


def test_decoupling_when_B_is_zero():
    # symmetric layup: the coupled 5-dof model equals the bending-only 3-dof model
    m = PlateModel(C4, 0)
    l5 = m.buckling_load(np.zeros(8), ndof=5)
    l3 = m.buckling_load(np.zeros(8), ndof=3)
    assert abs(l5 - l3) < 1e-10 * l3


def test_dense_vs_sparse_eigensolver():
    m = PlateModel(C4, 0)
    off = mi.plate_offsets(C4, 0, 0, 2)
    for row in off:
        assert abs(m.buckling_load(row, "dense") - m.buckling_load(row, "eigsh")) < 1e-10 * m.buckling_load(row)


def test_crossply_converges_to_navier():
    cfg = dict(C4, layup_deg=[0.0, 90.0, 90.0, 0.0], ply_t=0.25)
    errs = []
    for lv in range(3):
        m = PlateModel(cfg, lv)
        _, _, D = m.abd(np.zeros(4))
        assert abs(D[0, 2]) < 1e-9 and abs(D[1, 2]) < 1e-9
        nav = navier_orthotropic(D, cfg["a"], cfg["b"])
        errs.append((m.buckling_load(np.zeros(4)) - nav) / nav)
    # FE error is positive (from above) and falls about 4x per level (rate ~ M^-1)
    assert all(e > 0 for e in errs)
    assert 3.0 < errs[0] / errs[1] < 5.5 and 3.0 < errs[1] / errs[2] < 5.5
    assert errs[2] < 5e-4


def test_pristine_monotone_under_refinement():
    lams = [PlateModel(C4, lv).buckling_load(np.zeros(8)) for lv in range(3)]
    assert lams[0] > lams[1] > lams[2]


def test_sr_far_threshold_exits_at_jmin():
    calls = []
    def lam_at(j):
        calls.append(j)
        return [1.0, 0.9, 0.88, 0.875][j]
    lam, j, _ = sr_chain(lam_at, 3, lam_star=0.1, m=4, alpha=1.0, j_min=1)
    assert j == 1 and calls == [0, 1] and lam == 0.9
    assert indicator(lam, 0.1) == 0


def test_sr_without_exit_is_plain_mlmc():
    lam_vals = [1.0, 0.9, 0.88, 0.875]
    # alpha -> 0 makes the threshold factor 1/(m^alpha - 1) infinite: no early exit
    lam, j, lams = sr_chain(lambda j: lam_vals[j], 3, lam_star=0.89, m=4, alpha=1e-12, j_min=1)
    assert j == 3 and lam == 0.875
    qf, qc, y, n = sr_pair(lambda j: lam_vals[j], 2, lam_star=0.885, m=4, alpha=1e-12)
    assert (qf, qc, y) == (indicator(0.88, 0.885), indicator(0.9, 0.885), 1)


def test_sr_close_sample_refines():
    lam_vals = [0.95, 0.90, 0.887, 0.8832]
    lam, j, _ = sr_chain(lambda j: lam_vals[j], 3, lam_star=0.885, m=4, alpha=1.0, j_min=1)
    # |0.90-0.885| = 0.015 < 0.05/3 -> refine; |0.887-0.885| < 0.013/3 -> refine; level 3 is the last
    assert j == 3 and lam == 0.8832
