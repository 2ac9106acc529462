"""Pins of the oracle's plate model (Section 4.1) and of Algorithm 2 (Section 2.4)."""
import math

import numpy as np
import pytest

import mlmc_inputs as mi
from oracle.mesh import Mesh
from oracle.plate import (PlateModel, condensed_bending, laminate_abd, navier_orthotropic, plate_element)
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


T2 = mi.load_config("plate_t2")


def _null_dim(K):
    ev = np.linalg.eigvalsh(K)
    return int(np.sum(np.abs(ev) < 1e-9 * ev.max()))


def test_mitc4_element_has_only_the_rigid_zero_modes():
    """MITC4 transverse shear (Bathe-Dvorkin): the 20x20 element of a coupled
    laminate has exactly the six rigid motions as zero-energy modes; the
    one-point shear rule has two more (hourglass modes, among them the
    checkerboard w that becomes the thick panel's spurious buckling mode)."""
    m = PlateModel(T2, 0)
    A, B, D = m.abd(np.radians([2.0, -1.0, 3.0, 0.0, -2.0, 1.0, 0.5, -3.0]))
    Km, _ = plate_element(m.mesh, A, B, D, m.As, "mitc4")
    Ks, _ = plate_element(m.mesh, A, B, D, m.As, "sri")
    assert np.abs(Km - Km.T).max() <= 1e-12 * np.abs(Km).max()
    assert _null_dim(Km) == 6 and _null_dim(Ks) == 8
    # the rigid motions: u, v translations, in-plane rotation, w = 1, and the
    # tilts w = x, theta_x = 1 and w = y, theta_y = 1
    xs = np.array([-1.0, 1.0, 1.0, -1.0]) * 0.5 * m.mesh.hx
    ys = np.array([-1.0, -1.0, 1.0, 1.0]) * 0.5 * m.mesh.hy
    rig = np.zeros((6, 20))
    for a in range(4):
        rig[0, 5 * a] = 1.0
        rig[1, 5 * a + 1] = 1.0
        rig[2, 5 * a], rig[2, 5 * a + 1] = -ys[a], xs[a]
        rig[3, 5 * a + 2] = 1.0
        rig[4, 5 * a + 2], rig[4, 5 * a + 3] = xs[a], 1.0
        rig[5, 5 * a + 2], rig[5, 5 * a + 4] = ys[a], 1.0
    assert np.abs(Km @ rig.T).max() <= 1e-9 * np.abs(Km).max()


def test_condensed_bending_is_the_schur_complement():
    """D* = D - B^T A^-1 B is the inverse of the bending block of the inverse
    laminate matrix [[A, B], [B, D]]^-1; it equals D for the pristine Winckler
    stacking, whose B vanishes."""
    m = PlateModel(T2, 0)
    A, B, D = m.abd(np.radians([2.0, -1.0, 3.0, 0.0, -2.0, 1.0, 0.5, -3.0]))
    assert np.abs(B).max() > 1.0
    inv = np.linalg.inv(np.block([[A, B], [B, D]]))
    np.testing.assert_allclose(np.linalg.inv(inv[3:, 3:]), condensed_bending(A, B, D), rtol=1e-10, atol=1e-6)
    A0, B0, D0 = m.abd(np.zeros(8))
    assert np.abs(B0).max() <= 1e-12 * np.abs(D0).max()
    np.testing.assert_allclose(condensed_bending(A0, B0, D0), D0, rtol=1e-12, atol=1e-12 * np.abs(D0).max())


def test_condensed_five_unknown_model_equals_the_three_unknown_plate():
    m = PlateModel(T2, 0)
    off = mi.plate_offsets(T2, 0, 0, 1)[0]
    l5, l3 = m.buckling_load(off, ndof=5), m.buckling_load(off, ndof=3)
    assert abs(l5 - l3) <= 1e-10 * l3


def test_panel_load_converges_to_the_printed_value():
    """Test Problem II pristine panel with 0.8 mm plies: the load converges
    from above under refinement (with MITC4; the one-point shear rule drops
    to a checkerboard mode at 64x64), and the total edge force lambda L_y is
    within 0.5% of the 278.59 kN the paper prints for its pristine panel
    (the figure caption of Section 4)."""
    lam = [PlateModel(T2, lv).buckling_load(np.zeros(8)) for lv in (0, 1)]
    assert lam[0] > lam[1] and (lam[0] - lam[1]) < 1e-2 * lam[1]
    force_kn = lam[1] * T2["b"] / 1000.0
    assert abs(force_kn - 278.59) <= 5e-3 * 278.59, force_kn
    sri = PlateModel(dict(T2, shear="sri"), 1).buckling_load(np.zeros(8))
    assert sri < 0.5 * lam[1]


@pytest.mark.parametrize("name,fixture", [("plate_c4", "lambda_crit.json"), ("plate_t2", "lambda_crit_plate_t2.json")])
def test_threshold_fixtures_match_the_workloads(name, fixture):
    """The failure thresholds in the workload definitions are the ones the
    oracle-only pilot wrote (its level-0 quantile times the ratio of the
    pristine loads on the finest and the coarsest level)."""
    import json
    import os
    with open(os.path.join(os.path.dirname(__file__), "golden", fixture)) as f:
        gold = json.load(f)
    cfg = mi.load_config(name)
    assert cfg["lambda_crit"] == gold["lambda_crit"]
    assert gold["p_target"] == cfg["p_target"]
    assert abs(gold["level0_quantile"] * gold["pristine_top"] / gold["pristine_level0"] - gold["lambda_crit"]) \
        <= 1e-12 * gold["lambda_crit"]
    assert gold["level0_mean"] - 4 * gold["level0_std"] < gold["level0_quantile"] < gold["level0_mean"]


def test_panel_load_error_rate_alpha_one():
    """The paper reports that the FE error of its panel's buckling load falls
    with order alpha ~ 1 in the number of unknowns M (Section 4, the
    convergence figure).  M grows four-fold per level, so successive
    differences of the pristine load shrink about four-fold."""
    lam = [PlateModel(T2, lv).buckling_load(np.zeros(8)) for lv in (0, 1, 2)]
    d01, d12 = lam[0] - lam[1], lam[1] - lam[2]
    assert d01 > 0 and d12 > 0
    alpha = math.log(d01 / d12) / math.log(4.0)
    assert 0.8 < alpha < 1.2, alpha


def test_eigen_count_below_matches_the_dense_spectrum():
    # Sylvester count of K - sigma K_G against a brute-force dense generalised
    # eigen-decomposition of the 16x16 panel, at shifts between and around the
    # lowest eigenvalues
    import scipy.linalg as sla
    from oracle.plate import PlateModel, eigen_count_below
    cfg = mi.load_config("plate_c4")
    off = mi.plate_offsets(cfg, 0, 3, 1)[0]
    s = PlateModel(cfg, 0).system(off)
    mu = sla.eigh(s.KG.toarray(), s.K.toarray(), eigvals_only=True)
    lam = np.sort(1.0 / mu[mu > 1e-12 * mu.max()])
    shifts = [0.5 * lam[0], lam[0] * (1 - 1e-6), lam[0] * (1 + 1e-6), 0.5 * (lam[1] + lam[2]),
              0.5 * (lam[3] + lam[4]), lam[6] * (1 + 1e-6)]
    for sig in shifts:
        assert eigen_count_below(s.K, s.KG, sig) == int(np.sum(lam < sig)), sig


def test_inertia_at_32_marks_the_lowest_buckling_load():
    # 0 negative pivots just below lambda_1, 1 between lambda_1 and lambda_2:
    # the check the GPU runs after each eigen-solve, on the oracle's side
    import scipy.sparse.linalg as spla
    from oracle.plate import PlateModel, eigen_count_below
    cfg = mi.load_config("plate_c4")
    off = mi.plate_offsets(cfg, 1, 0, 1)[0]
    s = PlateModel(cfg, 1).system(off)
    lu = spla.splu(s.K.tocsc())
    vals = spla.eigsh(s.KG, k=3, M=s.K, Minv=spla.LinearOperator(s.K.shape, matvec=lu.solve), which="LA",
                      tol=1e-14, return_eigenvectors=False)
    lam = np.sort(1.0 / vals)
    assert eigen_count_below(s.K, s.KG, lam[0] * (1 - 1e-6)) == 0
    assert eigen_count_below(s.K, s.KG, 0.5 * (lam[0] + lam[1])) == 1
    assert eigen_count_below(s.K, s.KG, lam[1] * (1 - 1e-6)) == 1
