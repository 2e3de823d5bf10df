"""MI355X (gfx950) force evaluation for periodic molecular dynamics.

The binding of the C ABI (include/mdx.h) lives in ``paper_2503_20541_amd.mdx``
and is loaded on first use of any attribute of this package, so that
``python -m paper_2503_20541_amd.build`` can run before the library exists.
Using the package without a built libmdx.so raises ImportError.
"""
from __future__ import annotations

import importlib


def __getattr__(name):
    mod = importlib.import_module(".mdx", __name__)
    try:
        return getattr(mod, name)
    except AttributeError:
        raise AttributeError(f"module {__name__!r} has no attribute {name!r}") from None
