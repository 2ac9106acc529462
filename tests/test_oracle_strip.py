"""Pins of the oracle's strip model against mathematics it must satisfy.

Each check is independent of the oracle's own formulas: tensor rotation
written out from the fibre direction vector, rigid-body modes, exactness of
bilinear elements on linear fields (patch test), the closed-form off-axis
uniaxial stress state, a dense direct solve, and the QoI region: exactly
the central half of the element columns and rows at every level, and a
displacement field whose stress peaks outside the region.
"""
import math

import numpy as np
import pytest

import mlmc_inputs as mi
from oracle.material import Qbar, T_eps, ply_Q
from oracle.mesh import Mesh, level_mesh
from oracle.strip import (Dirichlet, StripModel, assemble, element_matrices, fibre_stress_qoi,
                          jacobi_pcg, reduce_system, strip_bcs)

CFG = mi.load_config("strip_c1")
M = CFG["material"]
Q = ply_Q(M["E11"], M["E22"], M["G12"], M["nu12"])


def test_ply_Q_values():
    # plane-stress reduced stiffness written from the compliance matrix
    S = np.array([[1 / M["E11"], -M["nu12"] / M["E11"], 0],
                  [-M["nu12"] / M["E11"], 1 / M["E22"], 0],
                  [0, 0, 1 / M["G12"]]])
    np.testing.assert_allclose(Q, np.linalg.inv(S), rtol=1e-14)


@pytest.mark.parametrize("theta", [0.0, 0.3, -0.7, 1.2, math.pi / 2])
def test_T_eps_is_tensor_rotation(theta):
    rng = np.random.default_rng(1)
    ex, ey, gxy = rng.standard_normal(3)
    E = np.array([[ex, gxy / 2], [gxy / 2, ey]])
    f = np.array([math.cos(theta), math.sin(theta)])      # fibre direction
    n = np.array([-math.sin(theta), math.cos(theta)])     # transverse direction
    want = [f @ E @ f, n @ E @ n, 2 * f @ E @ n]
    np.testing.assert_allclose(T_eps(theta) @ [ex, ey, gxy], want, atol=1e-15)


def test_qbar_symmetry_and_invariants():
    th = np.linspace(-1.5, 1.5, 13)
    inv1 = [Qbar(Q, t)[0, 0] + Qbar(Q, t)[1, 1] + 2 * Qbar(Q, t)[0, 1] for t in th]
    inv2 = [Qbar(Q, t)[2, 2] - Qbar(Q, t)[0, 1] for t in th]
    np.testing.assert_allclose(inv1, inv1[0], rtol=1e-13)
    np.testing.assert_allclose(inv2, inv2[0], rtol=1e-12)
    for t in th:
        Qb = Qbar(Q, t)
        np.testing.assert_allclose(Qb, Qb.T, atol=1e-9)
        np.testing.assert_allclose(Qbar(Q, t + math.pi), Qb, rtol=1e-12, atol=1e-8)
    np.testing.assert_allclose(Qbar(Q, 0.0), Q, atol=1e-10)
    Q90 = Qbar(Q, math.pi / 2)
    np.testing.assert_allclose([Q90[0, 0], Q90[1, 1], Q90[0, 1], Q90[2, 2]],
                               [Q[1, 1], Q[0, 0], Q[0, 1], Q[2, 2]], rtol=1e-12)


def test_element_rigid_modes_and_symmetry():
    mesh = Mesh(1.0, 0.5, 1, 1)
    rng = np.random.default_rng(2)
    Ke = element_matrices(mesh, Q, rng.uniform(-0.5, 0.5, (1, 4)))[0]
    np.testing.assert_allclose(Ke, Ke.T, rtol=1e-13, atol=1e-9)
    xy = mesh.node_xy()[mesh.elements()[0]]
    tx = np.tile([1.0, 0.0], 4)
    ty = np.tile([0.0, 1.0], 4)
    rot = np.ravel(np.stack([-xy[:, 1], xy[:, 0]], axis=1))
    for v in (tx, ty, rot):
        assert np.abs(Ke @ v).max() < 1e-10 * np.abs(Ke).max()
    ev = np.linalg.eigvalsh(Ke)
    assert np.sum(ev < 1e-9 * ev.max()) == 3


def test_global_K_three_zero_modes_then_spd():
    mesh = Mesh(4.0, 1.0, 8, 2)
    rng = np.random.default_rng(3)
    K = assemble(mesh, Q, rng.uniform(-0.3, 0.3, (mesh.n_elem, 4))).toarray()
    np.testing.assert_allclose(K, K.T, rtol=0, atol=1e-9 * np.abs(K).max())
    ev = np.linalg.eigvalsh(K)
    assert np.sum(ev < 1e-10 * ev.max()) == 3
    free, Kff, _ = reduce_system(assemble(mesh, Q, rng.uniform(-0.3, 0.3, (mesh.n_elem, 4))),
                                 strip_bcs(mesh, 0.01))
    assert np.linalg.eigvalsh(Kff.toarray()).min() > 0


def test_patch_test_linear_field_exact():
    mesh = Mesh(3.0, 2.0, 6, 4)
    th = 0.37
    K = assemble(mesh, Q, np.full((mesh.n_elem, 4), th))
    xy = mesh.node_xy()
    a = np.array([1e-3, -2e-3, 0.5e-3, 0.7e-3, -1e-3, 0.2e-3])
    u = a[0] + a[1] * xy[:, 0] + a[2] * xy[:, 1]
    v = a[3] + a[4] * xy[:, 0] + a[5] * xy[:, 1]
    d_exact = np.ravel(np.stack([u, v], axis=1))
    i, j = np.meshgrid(np.arange(mesh.nx + 1), np.arange(mesh.ny + 1))
    bnd = ((i == 0) | (i == mesh.nx) | (j == 0) | (j == mesh.ny)).ravel()
    nodes = np.nonzero(bnd)[0]
    dofs = np.sort(np.concatenate([2 * nodes, 2 * nodes + 1]))
    bc = Dirichlet(dofs, d_exact[dofs])
    free, Kff, b = reduce_system(K, bc)
    xf = np.linalg.solve(Kff.toarray(), b)
    np.testing.assert_allclose(xf, d_exact[free], rtol=0, atol=1e-14)


@pytest.mark.parametrize("theta_deg", [0.0, 3.0, -7.5, 20.0])
def test_off_axis_uniaxial_closed_form(theta_deg):
    th = math.radians(theta_deg)
    delta, L = 0.01, 20.0
    mesh = Mesh(L, 5.0, 16, 4)
    K = assemble(mesh, Q, np.full((mesh.n_elem, 4), th))
    j = np.arange(mesh.ny + 1)
    left, right = mesh.node_id(0, j), mesh.node_id(mesh.nx, j)
    dofs = np.concatenate([2 * left, [1], 2 * right])
    vals = np.concatenate([np.zeros(len(left)), [0.0], np.full(len(right), -delta)])
    o = np.argsort(dofs)
    bc = Dirichlet(dofs[o], vals[o])
    free, Kff, b = reduce_system(K, bc)
    d = np.zeros(K.shape[0])
    d[free] = np.linalg.solve(Kff.toarray(), b)
    d[bc.dofs] = bc.values
    c, s = math.cos(th), math.sin(th)
    S11 = c ** 4 / M["E11"] + (1 / M["G12"] - 2 * M["nu12"] / M["E11"]) * s * s * c * c + s ** 4 / M["E22"]
    q_closed = c * c * delta / (L * S11)
    q = fibre_stress_qoi(mesh, Q, np.full((mesh.n_elem, 4), th), d, [5, 15, 1.25, 3.75])
    assert abs(q - q_closed) <= 1e-11 * q_closed
    if theta_deg == 0.0:
        assert abs(q - 67.5) < 1e-10


def test_pcg_matches_dense_solve_c1_levels():
    for level in (0, 1):
        model = StripModel(CFG, level)
        xi = mi.strip_xi(CFG, level, 0, 2)
        for row in xi:
            th = model.theta(row)
            K = assemble(model.mesh, model.Q, th)
            free, Kff, b = reduce_system(K, model.bc)
            x_dense = np.linalg.solve(Kff.toarray(), b)
            res = jacobi_pcg(Kff, b, 1e-13)
            assert res.converged and res.true_relres < 1e-12
            np.testing.assert_allclose(res.x, x_dense, rtol=0, atol=1e-10 * np.abs(x_dense).max())
            sd = model.solve_theta(th, method="direct")
            sp = model.solve_theta(th, rtol=1e-13)
            assert abs(sd.q - sp.q) <= 1e-10 * abs(sd.q)
            d = np.zeros(K.shape[0])
            d[free] = x_dense
            d[model.bc.dofs] = model.bc.values
            assert abs(fibre_stress_qoi(model.mesh, model.Q, th, d, model.region) - sd.q) <= 1e-11 * sd.q


def test_pcg_stopping_rule():
    model = StripModel(CFG, 0)
    th = model.theta(mi.strip_xi(CFG, 0, 0, 1)[0])
    free, Kff, b = reduce_system(assemble(model.mesh, model.Q, th), model.bc)
    r10 = jacobi_pcg(Kff, b, 1e-10)
    r6 = jacobi_pcg(Kff, b, 1e-6)
    assert r10.relres <= 1e-10 and r6.relres <= 1e-6
    assert r6.iters < r10.iters
    one = jacobi_pcg(Kff, b, 1e-10, max_iter=1)
    assert one.iters == 1 and not one.converged


def test_qoi_converges_under_refinement():
    # same sample on nested meshes: level differences shrink (Section 2.2, V_l -> 0)
    cfg = dict(CFG)
    row = mi.strip_xi(cfg, 0, 0, 1)[0]
    qs = [StripModel(cfg, l).solve(row, method="direct").q for l in range(4)]
    d = np.abs(np.diff(qs))
    assert d[2] < d[0]


@pytest.mark.parametrize("name", ["strip_c1", "strip_c2", "strip_c3"])
def test_qoi_region_is_the_central_half_of_elements(name):
    # Section 3.2 takes the maximum over the integration points of a central
    # sub-region; the workloads use the central half in each direction, which
    # on these meshes is exactly element columns [nx/4, 3nx/4) and rows
    # [ny/4, 3ny/4) at every level (element (i, j) has id j nx + i).
    from oracle.strip import in_region
    cfg = mi.load_config(name)
    for level in range(cfg["n_levels"]):
        mesh = level_mesh(cfg, level)
        nx, ny = mesh.nx, mesh.ny
        expect = np.array([j * nx + i for j in range(ny // 4, 3 * ny // 4) for i in range(nx // 4, 3 * nx // 4)])
        got = np.nonzero(in_region(mesh, cfg["qoi_region"]))[0]
        np.testing.assert_array_equal(got, expect)


def test_qoi_takes_the_maximum_inside_the_region_only():
    # nodal displacement u = -c x^2, v = 0 at theta = 0: the compressive
    # fibre stress grows with x, so the QoI comes from the last element
    # column inside the region, not from the loaded end x = Lx.
    mesh = level_mesh(CFG, 0)
    c = 1e-4
    xy = mesh.node_xy()
    d = np.zeros(2 * mesh.n_nodes)
    d[0::2] = -c * xy[:, 0] ** 2
    theta = np.zeros((mesh.n_elem, 4))
    q = fibre_stress_qoi(mesh, Q, theta, d, CFG["qoi_region"])
    i_last = 3 * mesh.nx // 4 - 1
    # u is linear in x inside an element (bilinear interpolant of a function
    # of x alone), so eps_xx = (u_b - u_a) / h = -c (x_a + x_b) there
    xa, xb = i_last * mesh.hx, (i_last + 1) * mesh.hx
    eps_xx = -c * (xa + xb)
    assert abs(q - (-Q[0, 0] * eps_xx)) <= 1e-12 * abs(q)
    # over the whole strip the maximum would be larger (last column at x = Lx)
    q_all = fibre_stress_qoi(mesh, Q, theta, d, [0.0, CFG["Lx"], 0.0, CFG["Ly"]])
    assert q_all > 1.3 * q
