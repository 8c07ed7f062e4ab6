"""Seeded synthetic workloads shaped like the paper's industrial scenes.

The paper's own data (seven Basler template/working pairs, Sec. III) is not
available, so every image here is generated: analytic shapes rendered with
4x4 supersampling, placed at known poses, then distorted by occlusion, a
global gain and offset, clutter and noise.  This module holds no part of the
detector's arithmetic; both the oracle tests and the GPU path consume its
images.
"""
from .workloads import (  # noqa: F401
    C4,
    C4_MODELS,
    C4_SIZES,
    CONFIGS,
    BatchScene,
    c4_image,
    c4_model,
    c5_poses,
    Instance,
    Scene,
    make_model_shape,
    paste_rot90,
    render_model,
    render_posed,
    render_scene,
    scene_for_config,
)
