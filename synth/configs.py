"""The five workload configurations (sizes and seeds; no arithmetic).

frame64_grid32        64x64 frame, 32^3 grid, 64 samples/ray, no skipping,
                      no termination.
frame800_grid160      800x800 frame, 160^3 grid, 256 samples/ray, occupancy
                      skip, termination at transmittance 1e-4.
orbit32_frame800      the 800x800 scene on a 32-frame orbit (1 deg/frame);
                      references every 16th frame; targets warped from the
                      nearest reference, holes re-rendered.
views8_frame800_fp16  8 views of the 800x800 scene on the radius-4 sphere in
                      one launch; FP16 grid storage and BF16 MLP.
train8192_views8      one fwd+bwd step on 8192 rays drawn from 8 views of a
                      hidden scene.
"""
from dataclasses import dataclass, field


@dataclass(frozen=True)
class Config:
    name: str
    width: int
    height: int
    res: int
    n_samples: int
    use_occupancy: bool
    et_threshold: float
    scene_seed: int = 0
    mlp_seed: int = 1
    n_frames: int = 1
    ref_every: int = 0
    n_views: int = 1
    pose_seed: int = 2
    storage: str = "f32"
    compute: str = "f32"
    n_rays: int = 0
    extra: dict = field(default_factory=dict)


CONFIGS = {
    "frame64_grid32": Config("frame64_grid32", 64, 64, 32, 64, False, 0.0),
    "frame800_grid160": Config("frame800_grid160", 800, 800, 160, 256, True, 1e-4),
    "orbit32_frame800": Config("orbit32_frame800", 800, 800, 160, 256, True, 1e-4, n_frames=32, ref_every=16),
    "views8_frame800_fp16": Config("views8_frame800_fp16", 800, 800, 160, 256, True, 1e-4, n_views=8, pose_seed=2,
                   storage="f16", compute="bf16"),
    "train8192_views8": Config("train8192_views8", 800, 800, 160, 256, False, 1e-4, n_views=8, pose_seed=3,
                   n_rays=8192,
                   extra={"gt_scene_seed": 10, "gt_mlp_seed": 20, "model_grid_seed": 11,
                          "model_mlp_seed": 21, "ray_seed": 12}),
}


def get_config(name):
    return CONFIGS[name]
