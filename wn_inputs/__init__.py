"""Seeded synthetic inputs shared by the oracle tests, the GPU tests and the benchmark.

This package builds meshes, voxel-grid descriptors, loss targets and request traces.
It holds none of the winding-number arithmetic: no solid angles, no sums over faces,
no occupancy maps. Both the FP64 oracle and the HIP path take what it produces as
plain arrays.
"""
from .meshgen import (  # noqa: F401
    Grid,
    icosphere,
    uv_ellipsoid,
    random_rotation,
    ellipsoid_union,
    delete_faces,
    jitter,
    reverse_faces,
    concat_meshes,
    cube_mesh,
    octahedron_mesh,
    ellipsoid_inside,
    grid_flat_index,
    ellipsoid_target_on_grid,
    Ellipsoid,
    random_ellipsoid,
    signed_volume,
)
from .configs import (  # noqa: F401
    config1_icosphere,
    config2_ellipsoid_union,
    config3_differentiable,
    config4_batch,
    config5_trace,
    uniform_samples,
    evaluation_samples,
    SEEDS,
)
