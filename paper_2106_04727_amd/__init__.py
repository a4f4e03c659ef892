"""MI355X-native parallel nearest-neighbour-chain HAC (ParChain).

The clustering runs in ``libparchain.so`` (HIP kernels for gfx950 behind the
C ABI of ``include/parchain.h``); this package only marshals arguments.
"""
from .parchain import (  # noqa: F401
    LINKAGES,
    PCError,
    Context,
    Server,
    hac,
    hac_device,
    load_library,
    workspace_bytes,
    version,
)
