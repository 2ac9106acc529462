"""Shared helpers of the GPU tests (contexts and oracle models are cached per module)."""
import functools

import numpy as np

import mlmc_inputs as mi


@functools.lru_cache(maxsize=None)
def context(name: str, engine: str = "auto"):
    """Context of a workload; engine "lockstep" turns the one-work-group-per-
    sample solver of the coarse strip levels off, so every level runs the
    lock-step engine; engine "one_wg" keeps small plate batches of the narrower
    bands in the one-work-group kernel (otherwise they take the wide form, with
    the same results to the bit)."""
    import paper_1907_10271_amd as pk
    if engine == "auto":
        return pk.Context(mi.config_text(name))
    if engine == "one_wg":
        return pk.Context(dict(mi.load_config(name), wide_batch_per_bw=0))
    assert engine == "lockstep"
    return pk.Context(dict(mi.load_config(name), small_solver="off"))


@functools.lru_cache(maxsize=None)
def oracle_kl(name: str):
    from oracle.kl import KL
    return KL(mi.load_config(name))


@functools.lru_cache(maxsize=None)
def oracle_strip(name: str, level: int):
    from oracle.strip import StripModel
    return StripModel(mi.load_config(name), level, oracle_kl(name))


def dev(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda:0")


def raw_batch_call(ctx, fn: str, requests, rows, n_out=None):
    """Call mlmc_solve_batch or mlmc_buckle_batch through ctypes with no
    checks of the Python binding (to reach the library's own argument
    checks); returns the status code."""
    import ctypes as C
    import torch
    from paper_1907_10271_amd import _lib
    n = len(requests)
    arr = (_lib.Request * max(n, 1))()
    for k, (s, l, c) in enumerate(requests):
        arr[k].sample, arr[k].level, arr[k].coupled = int(s), int(l), int(bool(c))
    qf = torch.zeros(max(n, 1), dtype=torch.float64, device="cuda:0")
    qc = torch.zeros_like(qf)
    info = torch.zeros(max(n, 1) * 32, dtype=torch.uint8, device="cuda:0")
    st = torch.cuda.current_stream().cuda_stream
    if fn == "solve":
        return ctx.lib.mlmc_solve_batch(ctx.h, n, arr, rows.data_ptr(), rows.shape[0], rows.shape[1], qf.data_ptr(),
                                        qc.data_ptr(), info.data_ptr(), 0, 0.0, st)
    return ctx.lib.mlmc_buckle_batch(ctx.h, n, arr, rows.data_ptr(), rows.shape[0], qf.data_ptr(), qc.data_ptr(),
                                     info.data_ptr(), 0, 0.0, st)
