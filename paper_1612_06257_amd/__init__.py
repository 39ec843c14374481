"""Batched HighwayHash (arXiv:1612.06257) on AMD Instinct MI355X (gfx950).

The hashing runs in hand-written HIP kernels behind a C ABI (``libhh.so``,
declared in ``include/hh.h``).  ``paper_1612_06257_amd.hh`` is the thin Python
binding (argument marshalling only); ``workloads`` holds the seeded input
generators.  The binding is imported lazily so that the generators stay usable
on a machine without the built library.
"""
import importlib

__all__ = ["hh", "workloads"]


def __getattr__(name):
    if name in __all__:
        return importlib.import_module("." + name, __name__)
    raise AttributeError(name)
