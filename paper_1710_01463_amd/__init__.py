"""librsvd for AMD MI355X: randomized truncated SVD (RSVD) and full-SVD truncation.

The heavy lifting is in the HIP library librsvd.so (include/librsvd.h); this
package only marshals arguments and owns torch-allocated outputs.
"""
from .rsvd import (Plan, RSVDFunction, fullsvd_truncate, rsvd, rsvd_batch, rsvd_truncate,  # noqa: F401
                   rsvd_truncate_adaptive, rsvd_truncate_noalloc)

__all__ = ["rsvd_truncate", "rsvd_truncate_adaptive", "rsvd_truncate_noalloc", "fullsvd_truncate", "Plan", "RSVDFunction", "rsvd",
           "rsvd_batch"]
