"""GPU parity of the Cosserat model of Test Problem I (Section 3.1) against the
FP64 oracle, through the C ABI.

Tolerances: fields 1e-14 rad absolute; operator, lifting and diagonal 1e-13
relative to the max-norm; strength QoI 1e-10 relative against the oracle's
direct solve with both sides' iterations at rtol 1e-13; at the production
tolerance 1e-10 the GPU's final true residual (with the oracle's K) is at
most 1.01 rtol and its iteration counts are within 1% of the oracle's PCG."""
import functools
import json
import os

import numpy as np
import pytest

import mlmc_inputs as mi
from tests.conftest import gpu_available
from tests.gpu_util import dev

pytestmark = [pytest.mark.gpu, pytest.mark.skipif(not gpu_available(), reason="needs a GPU")]
CFG = mi.load_config("cosserat_t1")


@functools.lru_cache(maxsize=None)
def ctx():
    import paper_1907_10271_amd as pk
    return pk.Context(mi.config_text("cosserat_t1"))


@functools.lru_cache(maxsize=None)
def oracle(level):
    from oracle.cosserat import CosseratModel
    from oracle.kl import KL
    return CosseratModel(CFG, level, _kl())


@functools.lru_cache(maxsize=None)
def _kl():
    from oracle.kl import KL
    return KL(CFG)


def _rows(level, n, start=0):
    return mi.strip_xi(CFG, level, start, n)


@pytest.mark.parametrize("level", [0, 1, 2])
def test_field_parity(level):
    om = oracle(level)
    xi = _rows(level, 3)
    th = ctx().sample_field(level, dev(xi)).cpu().numpy()
    for k in range(3):
        ref = om.theta(xi[k]).ravel()
        assert np.abs(th[k] - ref).max() <= 1e-14, (level, k)


def _any_angles(n_gp, n, seed):
    rng = np.random.default_rng(seed)
    th = rng.uniform(-np.pi, np.pi, size=(n, n_gp))
    special = [np.pi / 2, -np.pi / 2, np.pi, -np.pi, 1.0, -1.0, 1.0 + 1e-9, 0.0, -0.0, 3.0]
    for k in range(n):
        th[k, k:k + len(special)] = special
    return th


@pytest.mark.parametrize("level,angles", [(0, "field"), (1, "field"), (1, "any")])
def test_operator_rhs_and_diagonal_parity(level, angles):
    from oracle.cosserat import assemble
    from oracle.strip import reduce_system
    om = oracle(level)
    n = 3
    if angles == "field":
        thetas = np.stack([om.theta(r).ravel() for r in _rows(level, n)])
    else:
        thetas = _any_angles(4 * om.mesh.n_elem, n, seed=41)
    x = np.random.default_rng(43).standard_normal((n, 3 * om.mesh.n_nodes))
    c = ctx()
    y_raw = c.strip_apply(level, dev(thetas), dev(x), raw=True).cpu().numpy()
    y_bc = c.strip_apply(level, dev(thetas), dev(x), raw=False).cpu().numpy()
    b, dinv = c.strip_rhs_diag(level, dev(thetas))
    b, dinv = b.cpu().numpy(), dinv.cpu().numpy()
    con = om.bc.dofs
    for k in range(n):
        K = assemble(om.mesh, om.C, om.D, thetas[k].reshape(-1, 4))
        ref = K @ x[k]
        assert np.abs(y_raw[k] - ref).max() <= 1e-13 * np.abs(ref).max(), k
        xp = x[k].copy()
        xp[con] = 0.0
        ref2 = K @ xp
        ref2[con] = x[k][con]
        assert np.abs(y_bc[k] - ref2).max() <= 1e-13 * np.abs(ref2).max(), k
        free, Kff, bf = reduce_system(K, om.bc)
        assert np.abs(b[k][free] - bf).max() <= 1e-13 * np.abs(bf).max(), k
        assert np.all(b[k][con] == 0.0) and np.all(dinv[k][con] == 1.0)
        d = Kff.diagonal()
        assert np.abs(1.0 / dinv[k][free] - d).max() <= 1e-13 * np.abs(d).max(), k


@pytest.mark.parametrize("level", [0, 1, 2])
def test_qoi_parity_tight(level):
    om = oracle(level)
    n = 5
    xi = _rows(level, n)
    qf, qc, info = ctx().solve_batch([(k, level, False) for k in range(n)], dev(xi), rtol=1e-13)
    qf = qf.cpu().numpy()
    for k in range(n):
        ref = om.solve(xi[k], method="direct").q
        assert info[k]["status_f"] == 0, info[k]
        assert abs(qf[k] - ref) <= 1e-10 * abs(ref), (level, k, qf[k], ref)


def test_aligned_strength_closed_form_on_the_gpu():
    # Phi = 0: strength C11 R tau_y / C12 exactly (the oracle's pin, here through the kernels)
    from oracle.cosserat import fibre_frame_matrices
    om = oracle(2)
    C, _ = fibre_frame_matrices(CFG["fibre"])
    th = np.zeros((2, 4 * om.mesh.n_elem))
    q, _, info = ctx().strip_solve_theta(2, dev(th), rtol=1e-13)
    f = CFG["fibre"]
    ref = C[0, 0] * f["R"] * f["tau_c"] / C[0, 1]
    assert np.all(np.abs(q.cpu().numpy() - ref) <= 1e-10 * ref)
    assert np.all(info["status_f"] == 0)


@pytest.mark.parametrize("level", [1, 2])
def test_production_rtol_residual_and_iterations(level):
    from oracle.cosserat import assemble
    from oracle.strip import jacobi_pcg, reduce_system
    om = oracle(level)
    n = 3
    xi = _rows(level, n, start=7)
    thetas = np.stack([om.theta(r).ravel() for r in xi])
    q, d, info = ctx().strip_solve_theta(level, dev(thetas), want_d=True)
    d = d.cpu().numpy()
    for k in range(n):
        K = assemble(om.mesh, om.C, om.D, thetas[k].reshape(-1, 4))
        free, Kff, b = reduce_system(K, om.bc)
        tr = np.linalg.norm(b - Kff @ d[k][free]) / np.linalg.norm(b)
        assert tr <= 1.01 * CFG["rtol"], (k, tr)
        assert np.allclose(d[k][om.bc.dofs], om.bc.values, rtol=0, atol=1e-15)
        ref = jacobi_pcg(Kff, b, CFG["rtol"])
        assert abs(info[k]["iters_f"] - ref.iters) <= max(2, 0.01 * ref.iters), (info[k]["iters_f"], ref.iters)


def test_coupled_pairs_and_batch_invariance():
    # a coupled request's coarse result is the level-1 solve of the same row,
    # bit for bit, and no result depends on the batch it rides in
    c = ctx()
    xi = dev(_rows(2, 6))
    qf, qc, info = c.solve_batch([(k, 2, True) for k in range(6)], xi)
    qf1, _, _ = c.solve_batch([(k, 1, False) for k in range(6)], xi)
    assert np.array_equal(qc.cpu().numpy(), qf1.cpu().numpy())
    alone = [c.solve_batch([(k, 2, True)], xi)[0].cpu().numpy()[0] for k in (0, 4)]
    assert alone[0] == qf.cpu().numpy()[0] and alone[1] == qf.cpu().numpy()[4]
    assert np.all(info["status_f"] == 0) and np.all(info["status_c"] == 0)
    # the level difference uses the level's own number of KL terms on each side
    om2, om1 = oracle(2), oracle(1)
    row = _rows(2, 1)[0]
    assert abs(qf.cpu().numpy()[0] - om2.solve(row, method="direct").q) <= 1e-8 * abs(qf.cpu().numpy()[0])
    assert abs(qc.cpu().numpy()[0] - om1.solve(row, method="direct").q) <= 1e-8 * abs(qc.cpu().numpy()[0])


def test_level_stats_of_coupled_cosserat_samples():
    import math
    c = ctx()
    xi = dev(_rows(1, 40))
    qf, qc, _ = c.solve_batch([(k, 1, True) for k in range(40)], xi)
    acc = c.level_stats(1, qf, qc)
    y = qf.cpu().numpy() - qc.cpu().numpy()
    assert acc.n == 40
    assert abs(acc.total("sum_y") - math.fsum(y)) <= 1e-12 * math.fsum(np.abs(y))
    assert abs(acc.total("sum_y2") - math.fsum(y * y)) <= 1e-12 * math.fsum(y * y)


def test_top_level_against_stored_oracle_values():
    """Level 5 (256 x 256 elements, 198k unknowns, 300 KL terms: the paper's
    finest Test I mesh) against the oracle's direct solves of two rows stored
    by tests/golden/make_cosserat_top_qoi.py."""
    fx = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "cosserat_top_qoi.json")))
    level, rows = fx["level"], fx["rows"]
    xi = _rows(level, max(rows) + 1)
    q, _, info = ctx().solve_batch([(r, level, False) for r in rows], dev(xi), rtol=1e-13)
    q = q.cpu().numpy()
    for k, r in enumerate(rows):
        assert info[k]["status_f"] == 0
        assert abs(q[k] - fx["q"][k]) <= 1e-9 * abs(fx["q"][k]), (r, q[k], fx["q"][k])
