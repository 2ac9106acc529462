"""Seeded synthetic inputs shared by the GPU path and the CPU oracle.

This module holds the workload definitions (JSON files under ``configs/``)
and the random draws that parameterise every sample.  It contains none of
the method's arithmetic: no covariance, no KL modes, no finite elements.
Both the GPU library and the oracle receive the very same arrays, so no
random-number parity between them is needed.

Random draws follow the sampling model of the paper:

* strip samples (Test I, KL expansion of the misalignment field,
  Eq. ``inftyKL``): ``xi_n ~ N(0, 1)`` i.i.d., optionally followed by the
  three wrinkle parameters of the waviness workloads
  (amplitude ``A ~ U(0, A_max)``, centre ``x0 ~ U(x0_lo, x0_hi)``, width
  ``w ~ U(w_lo, w_hi)``);
* plate samples (Test II, Section "Model Setup"): one constant offset per
  ply, ``phi_i ~ N(0, sigma_ply^2)``, returned in radians.

Row layout of a strip sample: ``[xi_1 .. xi_K, A_rad, x0_mm, w_mm]``
(always ``K + 3`` columns; without a wrinkle ``A = 0`` and ``w = 1``).

Streams: ``SeedSequence(190710271 + config_index)`` spawns one child per
level (plus one for a pilot run).  Samples are drawn in blocks of
``BLOCK`` rows; block ``b`` of level ``l`` has its own generator seeded
from ``(child_l, b)``, so any range of sample indices can be drawn
directly (resume, sharding) and sample ``j`` of level ``l`` is always the
same row.
"""
from __future__ import annotations

import json
import math
import os
from typing import Optional

import numpy as np

BASE_SEED = 190710271
BLOCK = 256
CONFIG_DIR = os.path.join(os.path.dirname(os.path.abspath(__file__)), "configs")

CONFIG_FILES = {
    "strip_c1": "strip_c1.json",
    "strip_c2": "strip_c2.json",
    "strip_c3": "strip_c3.json",
    "plate_c4": "plate_c4.json",
    "serve_c5": "serve_c5.json",
    "plate_t2": "plate_t2.json",
    "cosserat_t1": "cosserat_t1.json",
}


def config_path(name: str) -> str:
    return os.path.join(CONFIG_DIR, CONFIG_FILES.get(name, name))


def load_config(name: str) -> dict:
    """Return the workload definition ``name`` as a dict."""
    with open(config_path(name)) as f:
        return json.load(f)


def config_text(name: str) -> str:
    with open(config_path(name)) as f:
        return f.read()


def _block_generator(config_index: int, stream: int, block: int) -> np.random.Generator:
    ss = np.random.SeedSequence(BASE_SEED + config_index, spawn_key=(stream, block))
    return np.random.Generator(np.random.PCG64(ss))


def _draw_rows(config_index: int, stream: int, start: int, n: int, ncols: int, fill) -> np.ndarray:
    out = np.empty((n, ncols), dtype=np.float64)
    if n == 0:
        return out
    b0, b1 = start // BLOCK, (start + n - 1) // BLOCK
    row = 0
    for b in range(b0, b1 + 1):
        blk = fill(_block_generator(config_index, stream, b))
        lo = max(start, b * BLOCK) - b * BLOCK
        hi = min(start + n, (b + 1) * BLOCK) - b * BLOCK
        out[row:row + hi - lo] = blk[lo:hi]
        row += hi - lo
    return out


def strip_xi(cfg: dict, level: int, start: int, n: int, stream: Optional[int] = None) -> np.ndarray:
    """Rows ``start .. start+n-1`` of the strip sample stream of ``level``.

    Returns an ``[n, K + 3]`` float64 array (see the module docstring).
    """
    k = int(cfg["kl"]["n_modes"])
    wr = cfg.get("wrinkle")
    stream = level if stream is None else stream

    def fill(g: np.random.Generator) -> np.ndarray:
        blk = np.empty((BLOCK, k + 3))
        blk[:, :k] = g.standard_normal((BLOCK, k))
        if wr:
            u = g.random((BLOCK, 3))
            blk[:, k] = math.radians(wr["A_max_deg"]) * u[:, 0]
            blk[:, k + 1] = wr["x0"][0] + (wr["x0"][1] - wr["x0"][0]) * u[:, 1]
            blk[:, k + 2] = wr["w"][0] + (wr["w"][1] - wr["w"][0]) * u[:, 2]
        else:
            blk[:, k] = 0.0
            blk[:, k + 1] = 0.0
            blk[:, k + 2] = 1.0
        return blk

    return _draw_rows(int(cfg["config_index"]), stream, start, n, k + 3, fill)


def plate_offsets(cfg: dict, level: int, start: int, n: int, stream: Optional[int] = None) -> np.ndarray:
    """Ply-angle offsets in radians, ``[n, n_plies]`` float64."""
    nply = len(cfg["layup_deg"])
    sd = math.radians(cfg["ply_sigma_deg"])
    stream = level if stream is None else stream

    def fill(g: np.random.Generator) -> np.ndarray:
        return sd * g.standard_normal((BLOCK, nply))

    return _draw_rows(int(cfg["config_index"]), stream, start, n, nply, fill)


def poisson_arrivals(rate: float, duration: float, seed: int) -> np.ndarray:
    """Arrival times (s) of a Poisson stream of ``rate`` requests/s."""
    g = np.random.Generator(np.random.PCG64(np.random.SeedSequence(BASE_SEED + 5, spawn_key=(seed,))))
    n_est = int(rate * duration * 1.2 + 50)
    t = np.cumsum(g.exponential(1.0 / rate, n_est))
    while t[-1] < duration:
        t = np.concatenate([t, t[-1] + np.cumsum(g.exponential(1.0 / rate, n_est))])
    return t[t < duration]


def request_mix(n: int, seed: int, strip_share: float, strip_weights, plate_weights) -> np.ndarray:
    """Draw ``n`` request kinds and levels: ``[n, 2]`` int64 (kind 0 strip / 1 plate, level)."""
    g = np.random.Generator(np.random.PCG64(np.random.SeedSequence(BASE_SEED + 5, spawn_key=(seed, 1))))
    kind = (g.random(n) >= strip_share).astype(np.int64)
    sw = np.asarray(strip_weights, float) / np.sum(strip_weights)
    pw = np.asarray(plate_weights, float) / np.sum(plate_weights)
    lv = np.where(kind == 0, g.choice(len(sw), n, p=sw), g.choice(len(pw), n, p=pw))
    return np.stack([kind, lv.astype(np.int64)], axis=1)
