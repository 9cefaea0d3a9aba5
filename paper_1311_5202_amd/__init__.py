"""MI355X-native fast directional Burton-Miller BEM (arXiv 1311.5202).

The compute path is the HIP library libfdbem.so behind the C ABI of
include/fdbem.h; this package only marshals arguments to it.  Importing
works without the library (so it can be built); any call that needs it
raises if it is missing.
"""

from ._abi import LIB_PATH, OPS, FdaError, lib  # noqa: F401
from .fda import Batch, Net, Plan, analyze, build, near_correction, nystrom_nodes  # noqa: F401
