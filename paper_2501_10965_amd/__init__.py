"""MI355X (gfx950) DSMC + DIG hot path of arXiv:2501.10965.

The compute path is libdig.so (HIP kernels behind the C ABI of include/dig.h);
this package only marshals arguments.  Importing it does not require a GPU;
creating a simulation does, and fails loudly if libdig.so is missing.
"""
from ._lib import DigError, load  # noqa: F401

__all__ = ["DigError", "load", "DSMC"]


def __getattr__(name):
    if name == "DSMC":
        from .dsmc import DSMC
        return DSMC
    raise AttributeError(name)
