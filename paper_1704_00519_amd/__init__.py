"""MI355X (gfx950) implementation of the conservative sharp-interface method
for compressible multi-material flows (Pan, Han, Hu & Adams,
arXiv:1704.00519): a C-ABI HIP library (``libmmfv.so``, ``include/mmfv.h``)
and this thin Python binding."""
from ._lib import (MM_DEVICE, MM_HOST, MMError, Solver, Batch, load,
                   make_config, LIB_PATH, EXPORTS, batch_run_noalloc)

__all__ = ["Solver", "Batch", "MMError", "load", "make_config", "MM_HOST", "MM_DEVICE",
           "LIB_PATH", "EXPORTS", "batch_run_noalloc"]
