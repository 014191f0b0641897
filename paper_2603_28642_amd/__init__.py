"""Row-splitting ILU preconditioned least squares on AMD MI355X (gfx950).

The solver itself is the HIP library ``_lib/librsilu.so`` (C ABI in
include/rsilu.h); ``rsilu`` is its ctypes binding.
"""

from . import rsilu  # noqa: F401
