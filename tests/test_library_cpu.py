"""Host-side checks of the C ABI (no GPU needed): the built library loads and
exports every entry point declared in include/mlmc.h, and the Python
binding's record layouts match the header."""
import ctypes as C
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    text = open(os.path.join(ROOT, "include", "mlmc.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(mlmc_[a-z_]+)\s*\(", text)))


def test_library_exports_every_declared_symbol():
    from paper_1907_10271_amd import _lib
    lib = _lib.load()
    names = declared_functions()
    assert len(names) >= 13
    missing = [n for n in names if not hasattr(lib, n)]
    assert not missing, missing
    assert set(names) == set(_lib.EXPORTS)


def test_record_layouts_match_header():
    from paper_1907_10271_amd import _lib
    assert C.sizeof(_lib.Request) == 16
    assert C.sizeof(_lib.Info) == 32
    assert C.sizeof(_lib.LevelAcc) == 3 * 8 + 9 * 8


def test_product_path_does_not_import_oracle():
    pkg = os.path.join(ROOT, "paper_1907_10271_amd")
    for dirpath, _, files in os.walk(pkg):
        for f in files:
            if f.endswith((".py", ".hip", ".cpp", ".hpp", ".h")):
                src = open(os.path.join(dirpath, f)).read()
                assert "import oracle" not in src and "from oracle" not in src, f
                assert "oracle/" not in src.replace("oracle/ ", ""), f


def test_missing_library_fails_loudly(monkeypatch, tmp_path):
    from paper_1907_10271_amd import _lib
    monkeypatch.setattr(_lib, "_lib", None)
    monkeypatch.setattr(_lib, "LIB_PATH", str(tmp_path / "nope.so"))
    with pytest.raises(RuntimeError, match="HIP library missing"):
        _lib.load()


class _NoLib:
    """Stands in for the loaded library: any call means a bad tensor got past
    the binding's checks."""

    def __getattr__(self, name):
        raise AssertionError(f"library entry point {name} reached with a bad tensor")


def _fake_context(cfg, level_info):
    from paper_1907_10271_amd import _lib
    ctx = object.__new__(_lib.Context)
    ctx.lib, ctx.h, ctx.cfg = _NoLib(), None, cfg
    ctx.n_levels = cfg["n_levels"]
    ctx.n_params = len(cfg["layup_deg"]) if cfg["kind"] == "plate" else cfg["kl"]["n_modes"] + 3
    ctx.level_info = lambda level: dict(level_info)
    return ctx


STRIP_INFO = {"n_nodes": 297, "n_dofs": 594, "n_elem": 256, "n_gp": 1024}


@pytest.mark.parametrize("bad", ["float32", "sliced", "narrow", "host", "ndim"])
def test_strip_calls_reject_bad_tensors_before_the_library(bad):
    import torch

    import mlmc_inputs as mi
    ctx = _fake_context(mi.load_config("strip_c1"), STRIP_INFO)
    k = ctx.n_params
    # a device-side check cannot pass on a CPU-only machine, so every case
    # that is well formed apart from its location fails at the device check
    xi = {"float32": torch.zeros(4, k, dtype=torch.float32),
          "sliced": torch.zeros(4, 2 * k, dtype=torch.float64)[:, ::2],
          "narrow": torch.zeros(4, k - 1, dtype=torch.float64),
          "host": torch.zeros(4, k, dtype=torch.float64),
          "ndim": torch.zeros(4 * k, dtype=torch.float64)}[bad]
    msg = {"float32": "float64", "sliced": "contiguous", "narrow": "at least",
           "host": "device tensor", "ndim": "dimensions"}[bad]
    with pytest.raises(ValueError, match=msg):
        ctx.solve_batch([(0, 1, True)], xi)
    with pytest.raises(ValueError, match=msg):
        ctx.sample_field(0, xi)


def test_strip_operator_checks_theta_and_x_shapes():
    import torch

    import mlmc_inputs as mi
    ctx = _fake_context(mi.load_config("strip_c1"), STRIP_INFO)
    x = torch.zeros(3, STRIP_INFO["n_dofs"], dtype=torch.float64)
    with pytest.raises(ValueError, match="extent 1"):
        ctx.strip_apply(0, torch.zeros(3, STRIP_INFO["n_gp"] - 1, dtype=torch.float64), x)
    with pytest.raises(ValueError, match="extent 0"):
        ctx.strip_apply(0, torch.zeros(2, STRIP_INFO["n_gp"], dtype=torch.float64), x)
    with pytest.raises(ValueError, match="extent 1"):
        ctx.strip_apply(0, torch.zeros(3, STRIP_INFO["n_gp"], dtype=torch.float64), x[:, :10].contiguous())
    with pytest.raises(ValueError, match="float64"):
        ctx.strip_rhs_diag(0, torch.zeros(3, STRIP_INFO["n_gp"], dtype=torch.float32))
    with pytest.raises(ValueError, match="extent 1"):
        ctx.strip_solve_theta(0, torch.zeros(3, 7, dtype=torch.float64))


def test_request_rows_and_levels_are_checked():
    from paper_1907_10271_amd import _lib
    with pytest.raises(ValueError, match="sample row 5"):
        _lib._check_requests([(0, 0, False), (5, 1, True)], n_rows=5, n_levels=2)
    with pytest.raises(ValueError, match="level 2"):
        _lib._check_requests([(0, 2, False)], n_rows=5, n_levels=2)
    with pytest.raises(ValueError, match="sample row -1"):
        _lib._check_requests([(-1, 0, False)], n_rows=5, n_levels=2)
    _lib._check_requests([(4, 1, True)], n_rows=5, n_levels=2)


@pytest.mark.parametrize("bad", ["float32", "plies", "sliced", "host"])
def test_plate_calls_reject_bad_tensors_before_the_library(bad):
    import torch

    import mlmc_inputs as mi
    cfg = mi.load_config("plate_c4")
    ctx = _fake_context(cfg, {"n_nodes": 289, "n_dofs": 1445, "n_elem": 256, "n_gp": 1024})
    npl = len(cfg["layup_deg"])
    off = {"float32": torch.zeros(4, npl, dtype=torch.float32),
           "plies": torch.zeros(4, npl + 1, dtype=torch.float64),
           "sliced": torch.zeros(4, 2 * npl, dtype=torch.float64)[:, :npl],
           "host": torch.zeros(4, npl, dtype=torch.float64)}[bad]
    msg = {"float32": "float64", "plies": "extent 1", "sliced": "contiguous", "host": "device tensor"}[bad]
    with pytest.raises(ValueError, match=msg):
        ctx.buckle_batch([(0, 1, True)], off)
    with pytest.raises(ValueError, match=msg):
        ctx.plate_apply(0, off, torch.zeros(4, 5 * 289, dtype=torch.float64))


def test_level_stats_checks_its_inputs():
    import torch

    import mlmc_inputs as mi
    ctx = _fake_context(mi.load_config("strip_c1"), STRIP_INFO)
    with pytest.raises(ValueError, match="float64"):
        ctx.level_stats(0, torch.zeros(8, dtype=torch.float32))
    with pytest.raises(ValueError, match="extent 0"):
        ctx.level_stats(1, torch.zeros(8, dtype=torch.float64), torch.zeros(7, dtype=torch.float64))
