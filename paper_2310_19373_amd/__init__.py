"""Exhaustive QUBO solving in Gray-code order on MI355X (gfx950).

The public functions load the HIP library on first use; importing the package
(or its ``inputs`` module) touches no GPU.
"""
__version__ = "0.1.0"

_API = ("solve", "solve_batched", "solve_range", "merge_topk", "solve_resumable", "logz", "LogZ", "logz_moments",
        "marginals", "logz_sample", "masks_to_bits", "QuboError", "UncertainError")


def __getattr__(name):
    if name in _API:
        from . import api

        return getattr(api, name)
    raise AttributeError(name)
