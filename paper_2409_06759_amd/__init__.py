"""MI355X-native spin-orbital CCD/CCSD residual engine (HIP, gfx950).

The numerical work runs in ``libccmi.so`` (C ABI in ``include/cc.h``);
``engine`` is a thin PyTorch front end (device memory and streams only).
Importing this package does not load the shared library; the first use of
``engine`` does, and fails loudly if it has not been built.
"""
import importlib

__all__ = ["engine"]


def __getattr__(name):
    if name == "engine":
        return importlib.import_module(__name__ + ".engine")
    raise AttributeError(name)
