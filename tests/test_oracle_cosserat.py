"""Pins of the Cosserat oracle of Test Problem I (Section 3.1): the printed
level-0 unknown count, rotation and symmetry properties, the element's zero
modes, a patch test, the closed-form strength of the aligned composite,
linearity of the strength in the load, direct against iterative solves, the
QoI region, and the separable KL modes with level-dependent truncation."""
import math

import numpy as np
import pytest

import mlmc_inputs as mi
from oracle import cosserat as co
from oracle.mesh import Mesh

CFG = mi.load_config("cosserat_t1")


def test_level0_has_the_printed_243_unknowns():
    # Section 3.2: h_0 = L / 8, 64 elements and M_0 = 243 unknowns (3 per node)
    m = co.CosseratModel(CFG, 0)
    assert m.mesh.n_elem == 64
    C, D = co.fibre_frame_matrices(CFG["fibre"])
    K = co.assemble(m.mesh, C, D, np.zeros((64, 4)))
    assert K.shape == (243, 243)
    assert [co.modes_on_level(CFG, l) for l in range(6)] == [50, 100, 150, 200, 250, 300]


@pytest.mark.parametrize("phi", [0.0, 0.3, -1.1, 2.5])
def test_rotation_is_the_tensor_rotation(phi):
    rng = np.random.default_rng(1)
    eps = rng.standard_normal((2, 2))                     # non-symmetric Cosserat strain
    R = co.rotation_2(phi)
    ref = R @ eps @ R.T
    vec = np.array([eps[i, j] for i, j in co.PAIRS])
    got = co.rotation_4(phi) @ vec
    assert np.allclose(got, [ref[i, j] for i, j in co.PAIRS], atol=1e-15)
    T = co.rotation_4(phi)
    assert np.allclose(T @ T.T, np.eye(4), atol=1e-15)    # orthogonal: T^-1 = T^T
    C, D = co.fibre_frame_matrices(CFG["fibre"])
    Cs, Ds = co.rotated_matrices(C, D, phi)
    assert np.allclose(Cs, Cs.T, rtol=0, atol=1e-10 * np.abs(C).max())
    assert np.allclose(Cs, T.T @ C @ T, rtol=0, atol=1e-10 * np.abs(C).max())
    assert np.allclose(Ds, R.T @ D @ R, rtol=0, atol=1e-15)
    # energy is frame invariant
    assert abs(vec @ Cs @ vec - got @ C @ got) <= 1e-12 * abs(got @ C @ got)
    if phi == 0.0:
        assert np.array_equal(T, np.eye(4))


def test_shear_parallel_to_the_fibres_is_the_soft_one():
    # Section 3.1: shear stiffness parallel to the fibres is much smaller than orthogonal to them
    C, _ = co.fibre_frame_matrices(CFG["fibre"])
    assert C[3, 3] > 4.5 * C[2, 2]
    f = CFG["fibre"]
    assert abs(C[2, 2] - 1.0 / (f["v_f"] / f["G_f"] + (1 - f["v_f"]) / f["G_m"])) < 1e-9
    assert abs(C[3, 3] - (f["v_f"] * f["G_f"] + (1 - f["v_f"]) * f["G_m"])) < 1e-9


def test_element_zero_modes_are_the_rigid_motions():
    mesh = Mesh(1.0, 0.7, 1, 1)
    C, D = co.fibre_frame_matrices(CFG["fibre"])
    Ke = co.element_stiffness(mesh, C, D, [0.2, -0.1, 0.05, 0.3])
    assert np.allclose(Ke, Ke.T, rtol=0, atol=1e-9 * np.abs(Ke).max())
    ev = np.linalg.eigvalsh(Ke)
    assert np.sum(np.abs(ev) < 1e-10 * ev.max()) == 3 and ev.min() > -1e-10 * ev.max()
    xy = np.array([[0.0, 0.0], [1.0, 0.0], [1.0, 0.7], [0.0, 0.7]])
    modes = [np.tile([1.0, 0.0, 0.0], 4), np.tile([0.0, 1.0, 0.0], 4),
             np.ravel([[-y, x, 1.0] for x, y in xy])]        # rigid rotation: u = -y, v = x, theta_3 = 1
    for mvec in modes:
        assert np.abs(Ke @ mvec).max() < 1e-10 * np.abs(Ke).max()
    # a uniform Cosserat rotation alone is not free of energy
    t = np.tile([0.0, 0.0, 1.0], 4)
    assert t @ Ke @ t > 1e-3 * ev.max()


@pytest.mark.parametrize("phi", [0.0, 0.25, -0.6])
def test_patch_test_linear_field_is_exact(phi):
    # linear u, v with the constant theta_3 that makes sigma_12 = sigma_21 (moment
    # equilibrium with no couple stress): with all boundary unknowns prescribed
    # the finite element solution is exact at every interior node
    mesh = Mesh(3.0, 2.0, 6, 4)
    C, D = co.fibre_frame_matrices(CFG["fibre"])
    Cs, _ = co.rotated_matrices(C, D, phi)
    a, b, c, d = 1e-3, -4e-4, 7e-4, 2e-4                 # u = a x + b y, v = c x + d y
    e0 = np.array([a, d, b, c])                          # strains with theta_3 = 0
    dt = np.array([0.0, 0.0, 1.0, -1.0])                 # their change per unit theta_3
    s0, s1 = Cs @ e0, Cs @ dt
    th = -(s0[2] - s0[3]) / (s1[2] - s1[3])
    xy = mesh.node_xy()
    exact = np.stack([a * xy[:, 0] + b * xy[:, 1], c * xy[:, 0] + d * xy[:, 1], np.full(len(xy), th)], 1).ravel()
    K = co.assemble(mesh, C, D, np.full((mesh.n_elem, 4), phi))
    nnx = mesh.nx + 1
    bnd = [n for n in range(mesh.n_nodes) if n % nnx in (0, mesh.nx) or n // nnx in (0, mesh.ny)]
    con = np.array(sorted(3 * n + k for n in bnd for k in range(3)))
    free = np.setdiff1d(np.arange(3 * mesh.n_nodes), con)
    Kff = K[free][:, free].toarray()
    rhs = -(K[free][:, con] @ exact[con])
    sol = np.linalg.solve(Kff, rhs)
    assert np.abs(sol - exact[free]).max() <= 1e-12 * np.abs(exact).max()


def test_aligned_composite_strength_closed_form():
    # Phi = 0 with the workload's supports: u = Delta x / L, v = 0, theta_3 = 0 is
    # the exact solution, sigma_x = C11 Delta / L, sigma_22 = C12 Delta / L and
    # sigma_12 = 0, so f* = |C12 Delta / L| / (R tau_y) and the strength is
    # C11 R tau_y / C12, whatever Delta
    m = co.CosseratModel(CFG, 1)
    s = m.solve_theta(np.zeros((m.mesh.n_elem, 4)), method="direct")
    C, _ = co.fibre_frame_matrices(CFG["fibre"])
    f = CFG["fibre"]
    assert abs(s.mean_sigma_x - C[0, 0] * CFG["delta"] / CFG["Lx"]) <= 1e-11 * abs(s.mean_sigma_x)
    assert abs(s.q - C[0, 0] * f["R"] * f["tau_c"] / C[0, 1]) <= 1e-11 * s.q
    xy = m.mesh.node_xy()
    assert np.abs(s.d[0::3] - CFG["delta"] * xy[:, 0] / CFG["Lx"]).max() <= 1e-13
    assert np.abs(s.d[1::3]).max() <= 1e-15 and np.abs(s.d[2::3]).max() <= 1e-13


def test_strength_does_not_depend_on_the_load_and_solvers_agree():
    xi = mi.strip_xi(CFG, 0, 0, 1)[0]
    m = co.CosseratModel(CFG, 0)
    a = m.solve(xi, method="direct")
    m2 = co.CosseratModel(dict(CFG, delta=3.7 * CFG["delta"]), 0, m.kl)
    b = m2.solve(xi, method="direct")
    assert abs(a.q - b.q) <= 1e-12 * a.q
    assert abs(b.mean_sigma_x - 3.7 * a.mean_sigma_x) <= 1e-12 * abs(b.mean_sigma_x)
    c = m.solve(xi, rtol=1e-13)
    assert c.converged and abs(c.q - a.q) <= 1e-9 * a.q


@pytest.mark.parametrize("level", [0, 1, 2, 3])
def test_qoi_region_is_the_central_square(level):
    # Omega': the square of side 1.25 omega_1 = L / 2 centred in the domain
    mesh = co.CosseratModel(CFG, level).mesh
    sel = co.in_region(mesh, CFG["qoi_region"]).reshape(mesh.ny, mesh.nx)
    ref = np.zeros_like(sel)
    ref[mesh.ny // 4:3 * mesh.ny // 4, mesh.nx // 4:3 * mesh.nx // 4] = True
    assert np.array_equal(sel, ref)
    assert abs(CFG["qoi_region"][1] - CFG["qoi_region"][0] - 1.25 * CFG["kl"]["corr_x"]) < 1e-12


def test_anisotropic_separable_modes_against_a_2d_nystrom_solve():
    # the 10 largest eigenvalues of Eq. covarianceFunction with omega_1 != omega_2
    # and their order, against a direct 2-D Nystrom solve on a Gauss-Legendre grid
    from oracle.kl import KL, gauss_legendre_grid
    cfg = dict(CFG, kl=dict(CFG["kl"], n_modes=10))
    kl = KL(cfg)
    s2 = CFG["kl"]["sigma_rad"] ** 2
    errs = []
    for nq in (36, 72):
        grid, w = gauss_legendre_grid(CFG["Lx"], CFG["Ly"], nq, nq)
        d = np.abs(grid[:, None, :] - grid[None, :, :])
        K = s2 * np.exp(-d[..., 0] / CFG["kl"]["corr_x"] - d[..., 1] / CFG["kl"]["corr_y"])
        sw = np.sqrt(w)
        ev = np.sort(np.linalg.eigvalsh(sw[:, None] * K * sw[None, :]))[::-1][:10]
        errs.append(np.abs(ev - kl.mu).max() / kl.mu[0])
    # the kernel's kink makes the quadrature converge slowly: the Nystrom values
    # approach the closed-form ones (error about halved per doubling) and are
    # within 1% of the largest at 72 x 72
    assert errs[1] < 0.7 * errs[0] and errs[1] < 1e-2
    assert np.allclose(kl.mu, ev, rtol=2e-2)
    # and the level truncation takes the leading modes of one expansion
    m0, m1 = co.CosseratModel(CFG, 0), co.CosseratModel(CFG, 1)
    assert m0.n_modes == 50 and m1.n_modes == 100
    assert np.all(np.diff(m0.kl.mu) <= 0)
    xi = mi.strip_xi(CFG, 1, 0, 1)[0]
    pts = m0.mesh.gauss_points().reshape(-1, 2)
    phi = m0.kl.modes_at(pts)
    assert np.allclose(m0.theta(xi).ravel(), phi[:, :50] @ (np.sqrt(m0.kl.mu[:50]) * xi[:50]), atol=1e-15)
