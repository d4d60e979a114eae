"""MI355X-native DNN chemistry update (arXiv 2508.18969, ODENet-style).

``binding.ChemDNN`` wraps the C ABI of ``libchemdnn.so`` (see
``include/chem_dnn.h``); ``build.build()`` compiles it for gfx950.
"""
from .binding import (BF16, FP8E4M3, FP16, FP32, ChemDNN, ChemDNNError, autograd_function,  # noqa: F401
                      lib, make_desc, workspace_bytes)
