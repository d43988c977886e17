"""EnSF analysis step on MI355X: HIP kernels behind the C ABI of include/ensf.h.

The shared library is built in-tree by `python -m paper_2407_12168_amd.build`;
`paper_2407_12168_amd.ensf` is its Python binding.
"""
from . import ensf  # noqa: F401
