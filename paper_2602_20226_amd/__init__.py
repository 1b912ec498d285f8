"""MI355X-native QTT contraction and rounding (libqtt, gfx950 HIP kernels).

The Python surface is a thin ctypes binding over the C ABI in include/qtt.h;
see paper_2602_20226_amd.qtt.  Importing the package does not load the
library; the first call does, and raises ImportError if it was not built.
"""
from . import qtt  # noqa: F401
from .qtt import (  # noqa: F401
    QttError,
    add,
    contract,
    contract_backward,
    contract_round,
    contract_zipup,
    fit,
    inner,
    inner_backward,
    load_library,
    orthogonalize,
    rank_bounds,
    round_tt,
    to_device,
    to_host,
)
