"""hipphylo: phylogenetic log-likelihoods and branch-length gradients on AMD Instinct MI355X.

The compute path is the HIP library ``libhipphylo.so`` (C ABI in include/hipphylo.h);
this package is its Python binding.  Importing :class:`Instance` loads the library and
raises if it has not been built - there is no CPU fallback.
"""
from ._lib import HPError, default_scaling, load as load_library  # noqa: F401


def __getattr__(name):
    if name == "Instance":
        from .instance import Instance
        return Instance
    raise AttributeError(name)


__all__ = ["Instance", "HPError", "default_scaling", "load_library"]
