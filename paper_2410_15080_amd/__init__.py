"""MI355X-native contraction of hybrid tensor networks (h-TNs).

The compute path is libhtn.so (hand-written HIP for gfx950, C ABI in
include/htn.h); ``htn`` is its Python binding.  Importing the package does not
touch the GPU.
"""

from . import htn  # noqa: F401
