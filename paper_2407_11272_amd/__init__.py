"""MI355X (gfx950) generalized-winding-number voxelization (arXiv 2407.11272).

The compute path is the HIP library ``libwn.so`` (C ABI in ``include/wn.h``);
this package only marshals torch tensors and streams into it.  Importing the
package does not load the library; the first call does, and raises if it has
not been built (there is no CPU fallback).
"""
from .api import (  # noqa: F401
    Grid,
    MeshJob,
    Morpher,
    wn_adam,
    wn_morph_step,
    wn_cubify,
    wn_marching_cubes,
    wn_laplacian_smooth,
    wn_sample_surface,
    wn_nn_distance,
    wn_chamfer_hausdorff,
    evaluate_occupancy,
    wn_autotune,
    wn_voxelize_batched,
    wn_workspace_size_batched,
    Workspace,
    as_mesh,
    voxelize,
    SlicedBackward,
    wn_backward,
    wn_backward_naive,
    wn_voxelize_naive,
    wn_build_strips,
    wn_build_face_pairs,
    wn_flip_duplicate,
    wn_voxelize_strips,
    wn_get_device_error,
    wn_occupancy,
    wn_occupancy_backward,
    wn_release_workspace,
    wn_sigmoid_mse,
    wn_version,
    wn_voxelize,
    wn_workspace_size,
)
from ._lib import WnError  # noqa: F401
from .serve import GpuExecutor, Server, ServeRequest, ServeResult, run_plain_fifo  # noqa: F401
from .autograd import (  # noqa: F401
    NaiveWindingNumber,
    SigmoidOccupancy,
    WindingNumber,
    naive_winding_number,
    soft_occupancy,
    winding_number,
)
