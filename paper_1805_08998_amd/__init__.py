"""MI355X hierarchical-matrix product (HIP library + ctypes binding).

The compute path lives in libhmat.so (see include/hmat.h); `hmat` is the
binding with the same entry-point names. Importing this package does not load
the library; the first call does, and fails loudly if it is not built.
"""

from . import hmat  # noqa: F401
