"""Seeded synthetic inputs for the bilinear point rasterizer.

This module only draws random numbers and assembles cameras; it contains none
of the rasterizer's arithmetic (projection, splatting, sorting, blending).
Both the CPU oracle and the HIP path consume exactly these arrays.

The paper measures on trained INPC models of the Mip-NeRF360 and Tanks and
Temples scenes (Section 4.1); neither the datasets nor trained weights exist
here, so these generators stand in for them with the same shapes: megapixel
images, millions of points per sample, a depth density proportional to 1/d
(the viewpoint-specific sampling density of Eq. 4), and opacities inside
(0, 1) as produced by the activation of Section 3.3.
"""

from .scenes import (  # noqa: F401
    Camera,
    Scene,
    BatchedScene,
    canonical_camera,
    look_at_camera,
    make_config,
    config1,
    config2,
    config3,
    config4,
    config5,
    cluster_points,
    cluster_mixture,
    sample_mixture,
    multisample_clouds,
    sh_raw,
)
