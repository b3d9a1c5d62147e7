"""Split search for sparse oblique forests on AMD Instinct MI355X (gfx950).

The compute path is the HIP library libsof.so (C ABI in include/sof.h); this
package holds its sources (csrc/), the build script, the Python binding
(sof.py) and the seeded synthetic workloads (workloads.py).
"""
from .sof import (Context, DeviceFrontier, SofError, find_splits, partition, project, splits_from_numpy,
                  splits_to_numpy, to_device, version, workspace_size)

__all__ = ["Context", "DeviceFrontier", "SofError", "find_splits", "partition", "project",
           "splits_from_numpy", "splits_to_numpy", "to_device", "version", "workspace_size"]
