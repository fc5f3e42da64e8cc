"""MI355X-native recurrence quantification analysis (RQA).

The hot path (time-delay embedding, thresholded L1/L2/L-infinity distances,
diagonal / vertical / white-vertical line histograms) runs in hand-written HIP
kernels for gfx950 behind the C ABI of ``librqa.so`` (``include/rqa.h``); this
package only marshals arguments to it.
"""
from .rqa import (RQA, RQAResult, RQAError, Server, measures_from_hist, make_params,  # noqa: F401
                  norm_code, workspace_plan)
from ._lib import LIB_PATH, SIGNATURES  # noqa: F401
