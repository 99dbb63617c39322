"""MTP evaluation on AMD MI355X: Python front end of the HIP library libmtp.

The computation (neighbour lists, moments, contractions, adjoint, grade)
runs in libmtp.so (include/mtp.h); this package marshals torch device
tensors to it.  Importing the package does not load the library; the first
Potential does.
"""
__all__ = ["Potential", "Batch"]


def __getattr__(name):
    if name in ("Potential", "Batch"):
        from . import model
        return getattr(model, name)
    raise AttributeError(name)
