"""MI355X-native colour-gradient + near-contact-interaction lattice Boltzmann.

The compute path is the HIP C-ABI library ``liblbnci.so`` (kernels under
``csrc/``, declarations in ``include/lbnci.h``); ``lb`` is its ctypes binding.
"""
from .lb import (Lattice, Batch, Stream, LB_BATCH_LAUNCH, LB_BATCH_PERSISTENT, LB_BATCH_AUTO, Params, LBError, lattice_tables, load_library, LB_D2Q9, LB_D3Q27,
                 LB_STORE_FP32, LB_STORE_FP16_DEV, LB_STORE_BF16_DEV, LB_STORE_FP32_F32, STORAGE)

__all__ = ["Lattice", "Batch", "Stream", "LB_BATCH_LAUNCH", "LB_BATCH_PERSISTENT", "LB_BATCH_AUTO", "Params", "LBError", "lattice_tables", "load_library", "LB_D2Q9", "LB_D3Q27",
           "LB_STORE_FP32", "LB_STORE_FP16_DEV", "LB_STORE_BF16_DEV", "LB_STORE_FP32_F32", "STORAGE"]
