"""Seeded synthetic inputs for the renderer and for its CPU oracle.

This module only *draws* inputs: scene grids, MLP weights, camera poses and
intrinsics, random rays, pixel subsets.  It holds none of the rendering or
warping arithmetic (no ray generation, no sampling, no interpolation, no
compositing, no projection); both the GPU library and the oracle receive the
same bytes from here and compute everything else themselves.

Workload shapes follow the paper's evaluation setting (800x800 frames of a
dense voxel-grid model, camera orbits with small per-frame motion) with
synthetic content standing in for the trained models and datasets, which are
not available here.
"""
from .scene import (BOX_LO, BOX_HI, DENSITY_SHIFT, OCC_SIGMA, N_FEAT, HASH_RES, HASH_LOG2_SIZE, HASH_FEAT,
                    make_scene, make_mlp, make_model_grid, make_hash_tables)
from .camera import (intrinsics, look_at, orbit_pose, orbit_poses,
                     sphere_poses, relative_pose, Camera, make_camera, as_f32)
from .rays import random_rays, pixel_subset, training_pixels
from .configs import CONFIGS, get_config

__all__ = [
    "BOX_LO", "BOX_HI", "DENSITY_SHIFT", "OCC_SIGMA", "N_FEAT",
    "HASH_RES", "HASH_LOG2_SIZE", "HASH_FEAT", "make_hash_tables",
    "make_scene", "make_mlp", "make_model_grid",
    "intrinsics", "look_at", "orbit_pose", "orbit_poses", "sphere_poses",
    "relative_pose", "Camera", "make_camera", "as_f32",
    "random_rays", "pixel_subset", "training_pixels",
    "CONFIGS", "get_config",
]
