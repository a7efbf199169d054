"""MI355X-native DeGraF key-point detection and robust local optical flow tracking.

The compute path is the gfx950 HIP library ``libdegraf_flow.so`` behind the C ABI in
``include/degraf_flow.h``; this package only marshals tensors and streams into it.  Importing the
package does not load the library; the first call does, and raises if it is not built.
"""
from .api import (Batch, TrackFn, TrackOpts, autotune, get_tuning, set_tuning, detect, detect_count, pyramid, pyramid_layout, track,  # noqa: F401
                  track_backward, track_pyramids, track_run, track_workspace_bytes)
