"""MI355X-native DeGraF key-point detection, robust local optical flow tracking and dense
interpolation.

The compute path is the gfx950 HIP library ``libdegraf_flow.so`` behind the C ABI in
``include/degraf_flow.h``; this package only marshals tensors and streams into it.  Importing the
package does not load the library; the first call does, and raises if it is not built.
"""
from .api import (Batch, DetectFn, EpicOpts, TrackFn, TrackOpts, autotune, detect, detect_backward,  # noqa: F401
                  detect_count, detect_pyramids, epic, epic_async, epic_workspace_bytes, get_tuning, gm_fit, pyramid,
                  pyramid_layout, set_tuning, track, track_backward, track_batched, track_pyramids, track_run,
                  track_workspace_bytes)
