"""MI355X-native variance-reduced stochastic EM for penalised PET reconstruction.

The compute path is the HIP library ``_lib/libsvr.so`` (C ABI in
``include/svr.h``); ``binding`` marshals torch tensors and streams into it.
"""

from .binding import (  # noqa: F401
    SvrError, SystemMatrix, Recon, Server, params, geometry, lib, LIB_PATH, EXPORTED, splitmix64_orders,
    SVR_W_F32, SVR_W_F16, SVR_W_BF16,
)
