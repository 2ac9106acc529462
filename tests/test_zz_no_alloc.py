"""The allocation-free strip solve (fixed per-GPU scratch array) against the
pooled entry point it mirrors, through the C ABI: two calls in a row, the
second with a smaller input, on a whole-solve level and a lock-step level;
oversized requests are refused before any work is queued."""
import numpy as np
import pytest

import mlmc_inputs as mi
from tests.conftest import gpu_available
from tests.gpu_util import dev

pytestmark = [pytest.mark.gpu, pytest.mark.skipif(not gpu_available(), reason="needs a GPU")]


@pytest.fixture(scope="module")
def ctx():
    import paper_1907_10271_amd as pk
    return pk.Context(mi.config_text("strip_c2"))


@pytest.mark.parametrize("level,n1,n2", [(0, 40, 17), (2, 6, 3)])
def test_noalloc_solve_matches_pooled_solve(ctx, level, n1, n2):
    import torch
    cfg = mi.load_config("strip_c2")
    print(f"noalloc level {level} n {n1} then {n2}", flush=True)
    xi = dev(mi.strip_xi(cfg, level, 0, n1))
    theta = ctx.sample_field(level, xi)
    for n in (n1, n2):
        th = theta[:n].contiguous()
        q_ref, _, info_ref = ctx.strip_solve_theta(level, th)
        q = torch.full((n,), float("nan"), dtype=torch.float64, device="cuda:0")
        info = torch.zeros(32 * n, dtype=torch.uint8, device="cuda:0")
        ctx.strip_solve_theta_noalloc(level, th, q, info)
        torch.cuda.synchronize()
        from paper_1907_10271_amd._lib import info_to_numpy
        inf = info_to_numpy(info)
        # same kernels in the same order: identical bits
        assert np.array_equal(q.cpu().numpy(), q_ref.cpu().numpy()), (level, n)
        assert np.array_equal(inf["iters_f"], info_ref["iters_f"])
        assert np.array_equal(inf["relres_f"], info_ref["relres_f"])
        assert np.all(inf["status_f"] == 0)


def test_noalloc_refuses_more_than_its_scratch(ctx):
    import torch
    import paper_1907_10271_amd as pk
    from paper_1907_10271_amd._lib import MLMC_ENOMEM
    li = ctx.level_info(3)
    theta = torch.zeros((64, li["n_gp"]), dtype=torch.float64, device="cuda:0")
    q = torch.zeros(64, dtype=torch.float64, device="cuda:0")
    with pytest.raises(pk.MLMCError) as e:
        ctx.strip_solve_theta_noalloc(3, theta, q)
    assert e.value.code == MLMC_ENOMEM and "scratch" in str(e.value)
    assert torch.all(q == 0)
