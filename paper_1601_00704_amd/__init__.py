"""MI355X-native generalized lattice Boltzmann (GLBM) solver for shale permeability.

The hot path — the stream-and-collide sweep, the FP64 residual and Darcy-flux
reductions, warm-start initialisation and the CNN kernels — lives in the HIP
library ``lib/libglbm.so`` (sources in ``csrc/``, C ABI in ``include/glbm.h``).
``glbm`` is its ctypes binding; importing it loads the library and fails
loudly if it has not been built (``python -m paper_1601_00704_amd.build``).
"""
