"""ctypes binding of ``libmlmc.so`` (declared in include/mlmc.h).

Argument marshalling only: every numerical step runs in the HIP library.
PyTorch provides device memory (tensors passed by ``data_ptr()``) and the
current HIP stream.  The library must have been built
(``python -m paper_1907_10271_amd.build``); loading fails loudly otherwise.
"""
from __future__ import annotations

import ctypes as C
import json
import math
import os
from typing import Optional, Sequence, Union

import numpy as np

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "lib", "libmlmc.so")
# per-mesh engine and angle-storage choices written by the autotuner
TUNING_PATH = os.path.join(_PKG, "tuning", "mi355x.json")

MLMC_OK, MLMC_EINVAL, MLMC_ENOMEM, MLMC_EHIP, MLMC_ESTATE = 0, -1, -2, -3, -4
FP64, MIXED = 0, 1
S_OK, S_NOCONV, S_NAN, S_BREAKDOWN, S_SKIPPED, S_NOTLOWEST = 0, 1, 2, 3, 4, 5

EXPORTS = ["mlmc_create", "mlmc_destroy", "mlmc_last_error", "mlmc_level_info", "mlmc_num_levels",
           "mlmc_footprint", "mlmc_sample_field", "mlmc_strip_apply", "mlmc_strip_rhs_diag",
           "mlmc_strip_solve_theta", "mlmc_solve_batch", "mlmc_buckle_batch", "mlmc_level_stats",
           "mlmc_profile_enable", "mlmc_profile_read", "mlmc_plate_apply", "mlmc_reserve",
           "mlmc_strip_solve_theta_noalloc"]
# bytes of the fixed per-GPU scratch array of mlmc_strip_solve_theta_noalloc
SCRATCH_BYTES = 64 << 20


class Request(C.Structure):
    _fields_ = [("sample", C.c_int64), ("level", C.c_int32), ("coupled", C.c_int32)]


class Info(C.Structure):
    _fields_ = [("iters_f", C.c_int32), ("iters_c", C.c_int32), ("relres_f", C.c_double),
                ("relres_c", C.c_double), ("status_f", C.c_int32), ("status_c", C.c_int32)]


class LevelAcc(C.Structure):
    _fields_ = [("n", C.c_int64), ("n_plus", C.c_int64), ("n_minus", C.c_int64),
                ("sum_y", C.c_double), ("sum_y2", C.c_double), ("sum_qf", C.c_double),
                ("sum_qc", C.c_double), ("sum_cost", C.c_double), ("comp_y", C.c_double),
                ("comp_y2", C.c_double), ("comp_qf", C.c_double), ("comp_qc", C.c_double)]

    def total(self, name: str) -> float:
        comp = {"sum_y": "comp_y", "sum_y2": "comp_y2", "sum_qf": "comp_qf", "sum_qc": "comp_qc"}[name]
        return getattr(self, name) + getattr(self, comp)


INFO_DTYPE = np.dtype([("iters_f", "<i4"), ("iters_c", "<i4"), ("relres_f", "<f8"), ("relres_c", "<f8"),
                       ("status_f", "<i4"), ("status_c", "<i4")])
assert INFO_DTYPE.itemsize == C.sizeof(Info) == 32

_lib = None


class MLMCError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"mlmc error {code}: {msg}")
        self.code = code


def load() -> C.CDLL:
    """Load the HIP library (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"HIP library missing: {LIB_PATH} (run python -m paper_1907_10271_amd.build)")
    lib = C.CDLL(LIB_PATH)
    vp, i, d, sz = C.c_void_p, C.c_int, C.c_double, C.c_size_t
    lib.mlmc_create.argtypes = [C.c_char_p, sz, C.POINTER(vp)]
    lib.mlmc_destroy.argtypes = [vp]
    lib.mlmc_destroy.restype = None
    lib.mlmc_last_error.argtypes = [vp]
    lib.mlmc_last_error.restype = C.c_char_p
    lib.mlmc_level_info.argtypes = [vp, i] + [C.POINTER(C.c_int64)] * 4
    lib.mlmc_num_levels.argtypes = [vp]
    lib.mlmc_footprint.argtypes = [vp, i, i, i, C.POINTER(sz)]
    lib.mlmc_reserve.argtypes = [vp, i, i, i]
    lib.mlmc_sample_field.argtypes = [vp, i, i, vp, i, vp, i, vp]
    lib.mlmc_strip_apply.argtypes = [vp, i, i, vp, vp, vp, i, vp]
    lib.mlmc_strip_rhs_diag.argtypes = [vp, i, i, vp, vp, vp, vp]
    lib.mlmc_strip_solve_theta.argtypes = [vp, i, i, vp, vp, vp, vp, i, d, vp]
    lib.mlmc_strip_solve_theta_noalloc.argtypes = [vp, i, i, vp, vp, vp, d, vp]
    lib.mlmc_solve_batch.argtypes = [vp, i, C.POINTER(Request), vp, C.c_int64, i, vp, vp, vp, i, d, vp]
    lib.mlmc_buckle_batch.argtypes = [vp, i, C.POINTER(Request), vp, C.c_int64, vp, vp, vp, i, d, vp]
    lib.mlmc_level_stats.argtypes = [vp, i, i, vp, vp, d, d, C.POINTER(LevelAcc), vp]
    lib.mlmc_plate_apply.argtypes = [vp, i, i, vp, i, vp, vp, vp]
    lib.mlmc_profile_enable.argtypes = [vp, i]
    lib.mlmc_profile_read.argtypes = [vp, i, C.POINTER(C.c_double), C.POINTER(C.c_int64), C.POINTER(C.c_double)]
    _lib = lib
    return lib


def with_tuning(cfg: dict) -> dict:
    """The strip workload with the autotuner's per-mesh choices as
    ``level_options`` (unless it has its own, or no tuning file exists)."""
    if cfg.get("kind") != "strip" or "level_options" in cfg or not os.path.exists(TUNING_PATH):
        return cfg
    with open(TUNING_PATH) as f:
        doc = json.load(f)
    opts = {k: {"engine": v["engine"], "angles": v["angles"], "sweep_rows": int(v.get("sweep_rows", 0))}
            for k, v in doc.get("choices", {}).items()}
    return dict(cfg, level_options=opts)


def _torch():
    import torch
    return torch


def _ptr(t) -> Optional[int]:
    return None if t is None else t.data_ptr()


def _check_dev(*specs) -> None:
    """Raise ValueError unless every tensor is a contiguous FP64 tensor on a
    GPU with the given shape.  Each spec is ``(tensor, name, shape)`` or
    ``(tensor, name, shape, min_cols)``: ``None`` in ``shape`` = any extent,
    ``min_cols`` bounds the last extent from below.  The library reads these
    buffers with the row widths the shapes imply, so a mismatch must never
    reach it.  Layouts are checked for all tensors before their location."""
    torch = _torch()
    for spec in specs:
        t, name, shape = spec[:3]
        min_cols = spec[3] if len(spec) > 3 else None
        if not isinstance(t, torch.Tensor):
            raise ValueError(f"{name}: expected a torch tensor, got {type(t).__name__}")
        if t.dtype != torch.float64:
            raise ValueError(f"{name}: must be float64, got {t.dtype}")
        if not t.is_contiguous():
            raise ValueError(f"{name}: must be contiguous")
        if t.dim() != len(shape):
            raise ValueError(f"{name}: expected {len(shape)} dimensions, got shape {tuple(t.shape)}")
        for k, want in enumerate(shape):
            if want is not None and t.shape[k] != want:
                raise ValueError(f"{name}: extent {k} is {t.shape[k]}, expected {want} (shape {tuple(t.shape)})")
        if min_cols is not None and t.shape[-1] < min_cols:
            raise ValueError(f"{name}: rows of {t.shape[-1]} values, at least {min_cols} needed")
    for spec in specs:
        if not spec[0].is_cuda:
            raise ValueError(f"{spec[1]}: must be a device tensor, got device {spec[0].device}")


def _check_requests(requests: Sequence, n_rows: int, n_levels: int) -> None:
    for k, r in enumerate(requests):
        if len(r) != 3:
            raise ValueError(f"request {k}: expected (sample_row, level, coupled), got {r!r}")
        s, lvl = int(r[0]), int(r[1])
        if not 0 <= s < n_rows:
            raise ValueError(f"request {k}: sample row {s} outside [0, {n_rows})")
        if not 0 <= lvl < n_levels:
            raise ValueError(f"request {k}: level {lvl} outside [0, {n_levels})")


def _stream(stream=None) -> int:
    torch = _torch()
    s = torch.cuda.current_stream() if stream is None else stream
    return s.cuda_stream


def info_to_numpy(buf) -> np.ndarray:
    """Device ``uint8`` buffer of ``mlmc_info`` records -> numpy structured array."""
    host = buf.cpu().numpy()
    return host.view(INFO_DTYPE)


class Context:
    """Owns one ``mlmc_ctx`` (a workload definition on the current HIP device)."""

    def __init__(self, config: Union[str, dict], mem_budget_bytes: int = 0):
        self.lib = load()
        cfg = dict(config) if isinstance(config, dict) else json.loads(config)
        self.cfg = with_tuning(cfg)
        text = json.dumps(self.cfg)
        h = C.c_void_p()
        rc = self.lib.mlmc_create(text.encode(), mem_budget_bytes, C.byref(h))
        if rc != MLMC_OK:
            raise MLMCError(rc, self.lib.mlmc_last_error(None).decode())
        self.h = h
        self.n_levels = self.lib.mlmc_num_levels(self.h)
        # values per parameter row: K KL coefficients + 3 wrinkle values for a
        # strip, one offset per ply for a plate
        if self.cfg.get("kind") == "plate":
            self.n_params = len(self.cfg["layup_deg"])
        else:
            self.n_params = int(self.cfg["kl"]["n_modes"]) + 3

    def close(self):
        if getattr(self, "h", None):
            self.lib.mlmc_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _check(self, rc: int):
        if rc != MLMC_OK:
            raise MLMCError(rc, self.lib.mlmc_last_error(self.h).decode())

    # ------------------------------------------------------------ queries
    def level_info(self, level: int):
        v = [C.c_int64() for _ in range(4)]
        self._check(self.lib.mlmc_level_info(self.h, level, *[C.byref(x) for x in v]))
        return {"n_nodes": v[0].value, "n_dofs": v[1].value, "n_elem": v[2].value, "n_gp": v[3].value}

    def footprint(self, kind: int, level: int, precision: int = FP64) -> int:
        b = C.c_size_t()
        self._check(self.lib.mlmc_footprint(self.h, kind, level, precision, C.byref(b)))
        return b.value

    def reserve(self, level: int, n: int, precision: int = FP64) -> None:
        """Allocate the workspace for ``n`` requests of ``level`` now."""
        self._check(self.lib.mlmc_reserve(self.h, level, n, precision))

    # ------------------------------------------------------------ strip
    def sample_field(self, level: int, xi, dtype: int = 0, stream=None):
        torch = _torch()
        _check_dev((xi, "xi", (None, None), self.n_params))
        n = xi.shape[0]
        ngp = self.level_info(level)["n_gp"]
        out = torch.empty((n, ngp), dtype=torch.float64 if dtype == 0 else torch.int16, device=xi.device)
        self._check(self.lib.mlmc_sample_field(self.h, level, n, _ptr(xi), xi.shape[1], _ptr(out), dtype,
                                               _stream(stream)))
        return out

    def strip_apply(self, level: int, theta, x, raw: bool = False, stream=None):
        torch = _torch()
        li = self.level_info(level)
        _check_dev((x, "x", (None, li["n_dofs"])),
                   (theta, "theta", (x.shape[0] if x.dim() else None, li["n_gp"])))
        y = torch.empty_like(x)
        self._check(self.lib.mlmc_strip_apply(self.h, level, x.shape[0], _ptr(theta), _ptr(x), _ptr(y), int(raw),
                                              _stream(stream)))
        return y

    def strip_rhs_diag(self, level: int, theta, stream=None):
        torch = _torch()
        li = self.level_info(level)
        _check_dev((theta, "theta", (None, li["n_gp"])))
        n = theta.shape[0]
        nd = li["n_dofs"]
        b = torch.empty((n, nd), dtype=torch.float64, device=theta.device)
        dinv = torch.empty_like(b)
        self._check(self.lib.mlmc_strip_rhs_diag(self.h, level, n, _ptr(theta), _ptr(b), _ptr(dinv),
                                                 _stream(stream)))
        return b, dinv

    def strip_solve_theta(self, level: int, theta, precision: int = FP64, rtol: float = 0.0,
                          want_d: bool = False, stream=None):
        torch = _torch()
        _check_dev((theta, "theta", (None, self.level_info(level)["n_gp"])))
        n = theta.shape[0]
        q = torch.empty(n, dtype=torch.float64, device=theta.device)
        info = torch.zeros(n * 32, dtype=torch.uint8, device=theta.device)
        d = None
        if want_d:
            d = torch.empty((n, self.level_info(level)["n_dofs"]), dtype=torch.float64, device=theta.device)
        self._check(self.lib.mlmc_strip_solve_theta(self.h, level, n, _ptr(theta), _ptr(q), _ptr(d), _ptr(info),
                                                    precision, rtol, _stream(stream)))
        return q, d, info_to_numpy(info)

    def strip_solve_theta_noalloc(self, level: int, theta, q, info=None, rtol: float = 0.0, stream=None):
        """FP64 solves of the given fields with the library's fixed scratch
        array as workspace: the call allocates no device memory.  The caller
        passes the outputs ``q`` (float64 ``[n]``) and optionally ``info``
        (uint8 ``[n * 32]``)."""
        torch = _torch()
        _check_dev((theta, "theta", (None, self.level_info(level)["n_gp"])), (q, "q", (theta.shape[0],)))
        if info is not None:
            if info.dtype != torch.uint8 or not info.is_contiguous() or info.numel() < 32 * theta.shape[0] \
                    or not info.is_cuda:
                raise ValueError("info: must be a contiguous uint8 device tensor of at least 32 n bytes")
        self._check(self.lib.mlmc_strip_solve_theta_noalloc(self.h, level, theta.shape[0], _ptr(theta), _ptr(q),
                                                            _ptr(info), rtol, _stream(stream)))
        return q, (None if info is None else info_to_numpy(info)[:theta.shape[0]])

    def solve_batch(self, requests: Sequence, xi, precision: int = FP64, rtol: float = 0.0, stream=None):
        """``requests``: sequence of ``(sample_row, level, coupled)``."""
        torch = _torch()
        _check_dev((xi, "xi", (None, None), self.n_params))
        _check_requests(requests, xi.shape[0], self.n_levels)
        n = len(requests)
        arr = (Request * max(n, 1))()
        for k, (s, l, c) in enumerate(requests):
            arr[k].sample, arr[k].level, arr[k].coupled = int(s), int(l), int(bool(c))
        qf = torch.empty(n, dtype=torch.float64, device=xi.device)
        qc = torch.empty(n, dtype=torch.float64, device=xi.device)
        info = torch.zeros(max(n, 1) * 32, dtype=torch.uint8, device=xi.device)
        self._check(self.lib.mlmc_solve_batch(self.h, n, arr, _ptr(xi), xi.shape[0], xi.shape[1], _ptr(qf), _ptr(qc),
                                              _ptr(info), precision, rtol, _stream(stream)))
        return qf, qc, info_to_numpy(info)[:n]

    # ------------------------------------------------------------ plate
    def buckle_batch(self, requests: Sequence, offsets, precision: int = FP64, tol: float = 0.0, stream=None):
        torch = _torch()
        _check_dev((offsets, "offsets", (None, self.n_params)))
        _check_requests(requests, offsets.shape[0], self.n_levels)
        n = len(requests)
        arr = (Request * max(n, 1))()
        for k, (s, l, c) in enumerate(requests):
            arr[k].sample, arr[k].level, arr[k].coupled = int(s), int(l), int(bool(c))
        lf = torch.empty(n, dtype=torch.float64, device=offsets.device)
        lc = torch.empty(n, dtype=torch.float64, device=offsets.device)
        info = torch.zeros(max(n, 1) * 32, dtype=torch.uint8, device=offsets.device)
        self._check(self.lib.mlmc_buckle_batch(self.h, n, arr, _ptr(offsets), offsets.shape[0], _ptr(lf), _ptr(lc), _ptr(info),
                                               precision, tol, _stream(stream)))
        return lf, lc, info_to_numpy(info)[:n]

    # ------------------------------------------------------------ diagnostics
    def profile(self, on: bool = True):
        self._check(self.lib.mlmc_profile_enable(self.h, int(on)))

    def profile_read(self, kernel: int):
        ms, n, b = C.c_double(), C.c_int64(), C.c_double()
        self._check(self.lib.mlmc_profile_read(self.h, kernel, C.byref(ms), C.byref(n), C.byref(b)))
        return {"ms": ms.value, "launches": n.value, "bytes": b.value}

    def plate_apply(self, level: int, offsets, x, geometric: bool = False, stream=None):
        torch = _torch()
        _check_dev((offsets, "offsets", (None, self.n_params)),
                   (x, "x", (offsets.shape[0] if offsets.dim() else None, 5 * self.level_info(level)["n_nodes"])))
        y = torch.empty_like(x)
        self._check(self.lib.mlmc_plate_apply(self.h, level, x.shape[0], _ptr(offsets), int(geometric), _ptr(x),
                                              _ptr(y), _stream(stream)))
        return y

    # ------------------------------------------------------------ sums
    def level_stats(self, level: int, q_fine, q_coarse=None, cost_per_sample: float = 0.0,
                    lambda_star: float = math.nan, acc: Optional[LevelAcc] = None, stream=None) -> LevelAcc:
        acc = LevelAcc() if acc is None else acc
        specs = [(q_fine, "q_fine", (None,))]
        if q_coarse is not None:
            specs.append((q_coarse, "q_coarse", (q_fine.shape[0] if q_fine.dim() else None,)))
        _check_dev(*specs)
        self._check(self.lib.mlmc_level_stats(self.h, level, q_fine.shape[0], _ptr(q_fine), _ptr(q_coarse),
                                              cost_per_sample, lambda_star, C.byref(acc), _stream(stream)))
        return acc
