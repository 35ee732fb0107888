"""MI355X-native nonoverlapping domain decomposition for extreme learning machines.

The solver is the HIP library libelmddm.so (C ABI in include/elmddm.h);
`binding` wraps it for Python callers that keep their data in torch
device tensors, and `solver` adds a convenience layer that prepares the
inputs of one problem.
"""
from . import binding  # noqa: F401
