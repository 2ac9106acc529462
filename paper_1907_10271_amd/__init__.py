"""MI355X-native multilevel Monte Carlo sample-solve engine.

The compute path is the HIP library ``lib/libmlmc.so`` (C ABI in
``include/mlmc.h``); :mod:`._lib` binds it with ctypes, :mod:`.driver`
runs the MLMC algorithms of the paper on top of it.  Importing the package
loads nothing; the library is loaded on first use and a missing build is a
hard error.
"""
from ._lib import (FP64, MIXED, S_BREAKDOWN, S_NAN, S_NOCONV, S_NOTLOWEST, S_OK, S_SKIPPED, Context,
                   LevelAcc, MLMCError, load)

__all__ = ["Context", "LevelAcc", "MLMCError", "load", "FP64", "MIXED", "S_OK", "S_NOCONV", "S_NAN",
           "S_BREAKDOWN", "S_SKIPPED", "S_NOTLOWEST"]
