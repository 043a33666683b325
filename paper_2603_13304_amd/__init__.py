"""pepsnet: Block Belief Propagation on kagome PEPS for MI355X (gfx950).

The compute path is the HIP library ``libpepsnet.so`` built from ``csrc/``
(see ``include/pepsnet.h`` for the C ABI); ``binding`` marshals arguments to
it and nothing else.  There is no CPU fallback: importing the binding fails
when the library has not been built.
"""
from .binding import (BBP_BF16X3, BBP_FP32, BBP_FP64, BBP_KAGOME_INF_HEX,  # noqa: F401
                      BBP_KAGOME_OPEN, BBP_SVD_FULL, BBP_SVD_RAND, Batch, PepsNet, Server,
                      PepsnetError, describe, library_path, load_library)
