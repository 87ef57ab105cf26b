"""gabm: MI355X-native per-day transmission step of a differentiable
agent-based epidemic model (GradABM), as a C-ABI HIP library with a thin
Python binding.

Import ``paper_2207_09714_amd.gabm`` for the binding; it loads
``libgabm.so`` built in-tree by ``paper_2207_09714_amd/build.py`` and raises
if the library is missing.
"""

__all__ = ["gabm"]
