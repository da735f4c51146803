"""MI355X (gfx950) cutting voxel projector.

Hand-written HIP kernels behind a C ABI (include/cvp.h, libcvp.so); this
package is the thin Python binding.  Kulvait & Rose, "Cutting Voxel Projector
a New Approach to Construct 3D Cone Beam CT Operator" (2021).
"""
from .cvp import (TT, Batch, BatchedCGLS, BackProject, CGLS, Geometry, Options, Project,  # noqa: F401
                  backproject, backproject_batched, cgls, project, project_batched)
