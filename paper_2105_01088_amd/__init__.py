"""MI355X library for one imaginary-time step of the SGS variational method
(Boutin & Bauer, arXiv:2105.01088).

The computation lives in the HIP library ``libsgs.so`` (C ABI in
``include/sgs.h``); this package only marshals arguments to it.  Importing the
package does not load the library; the first use of ``SGS`` does, and raises
if it has not been built (``python -m paper_2105_01088_amd.build``).
"""

from ._lib import (  # noqa: F401
    SGS,
    SGSError,
    load_library,
    default_options,
    SGS_FP64,
    SGS_FP32_FORCE,
    SGS_W_PRINTED,
    SGS_W_UNIT,
    SGS_UPD_EULER,
    SGS_UPD_EXP,
    SGS_OBS_POLY,
    SGS_OBS_RENYI2,
    SGS_OBS_VARIANCE,
    SGS_REN_AUTO,
    SGS_REN_BLOCK,
    SGS_REN_SPLIT,
    rotate_state,
    rotate_state_noalloc,
)
from .protocol import grow  # noqa: F401
