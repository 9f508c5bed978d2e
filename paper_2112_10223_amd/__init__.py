"""MI355X (gfx950) SpKAdd: hash and sliding-hash addition of k sparse CSC matrices.

The compute path is the C ABI of libspkadd.so (include/spkadd.h).  The Python
names mirror the C entry points: spkadd_plan, spkadd_symbolic, spkadd_numeric,
spkadd_free.  The convenience wrapper spkadd() runs all of them in sequence.
"""
from .binding import (Opts, Plan, SpkaddError, make_opts, spkadd, spkadd_free, spkadd_get_stats, spkadd_numeric,
                      spkadd_plan, spkadd_symbolic, spkadd_trace, SPKADD_F32, SPKADD_F64, SPKADD_FLAG_TRACE,
                      SPKADD_FLAG_VALIDATE, SPKADD_BIN_AUTO, SPKADD_BIN_WAVE, SPKADD_BIN_WG, SPKADD_BIN_WINDOW)

__all__ = ["Opts", "Plan", "SpkaddError", "make_opts", "spkadd", "spkadd_free", "spkadd_get_stats",
           "spkadd_numeric", "spkadd_plan", "spkadd_symbolic", "spkadd_trace", "SPKADD_F32", "SPKADD_F64",
           "SPKADD_FLAG_TRACE", "SPKADD_FLAG_VALIDATE", "SPKADD_BIN_AUTO", "SPKADD_BIN_WAVE", "SPKADD_BIN_WG",
           "SPKADD_BIN_WINDOW"]
