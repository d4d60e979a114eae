"""MI355X-native DNN chemistry update (arXiv 2508.18969, ODENet-style).

``binding.ChemDNN`` wraps the chemistry update and ``binding.PropNet`` the
property networks of the C ABI of ``libchemdnn.so`` (see
``include/chem_dnn.h``); ``build.build()`` compiles it for gfx950.
"""
from .binding import (BF16, FP8E4M3, FP16, FP32, ChemDNN, ChemDNNError, autograd_function,  # noqa: F401
                      PropNet, lib, make_desc, make_prop_desc, prop_workspace_bytes, workspace_bytes)
