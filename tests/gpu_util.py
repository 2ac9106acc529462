"""Shared helpers of the GPU tests (contexts and oracle models are cached per module)."""
import functools

import numpy as np

import mlmc_inputs as mi


@functools.lru_cache(maxsize=None)
def context(name: str, engine: str = "auto"):
    """Context of a workload; engine "lockstep" turns the one-work-group-per-
    sample solver of the coarse levels off, so every level runs the lock-step
    engine."""
    import paper_1907_10271_amd as pk
    if engine == "auto":
        return pk.Context(mi.config_text(name))
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
