"""MI355X (gfx950) projection library for PGD-TO (arXiv 2511.13905).

The compute path is the HIP library ``libpgdto.so`` (C ABI in include/pgdto.h);
``api`` binds it for torch tensors.  ``inputs`` holds the seeded synthetic
problem generators.
"""
from . import inputs  # noqa: F401

__all__ = ["inputs", "api", "native"]


def __getattr__(name):
    # the binding needs torch and the built library; load it on first use
    # (import_module, not "from . import": that form asks this hook again)
    import importlib
    if name == "api":
        return importlib.import_module(__name__ + ".api")
    if name == "native":
        return importlib.import_module(__name__ + "._native")
    raise AttributeError(name)
