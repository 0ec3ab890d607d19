"""Writes tests/golden/amb17_reference.npz: the float64 oracle's colours on
the precision-path workload, for the BF16 quality criterion.

Workload: the 160^3 scene (seed 0) with the seed-1 MLP, eight 800x800 views
on the radius-4 sphere (pose seed 2), 16,384 seeded pixels per view (seed
1700 + view).  Stored per pixel (float32):
  o64 -- the oracle at the workload's own settings (256 samples per ray,
         occupancy skipping, termination at transmittance 1e-4);
  g   -- the converged reference: 1024 samples per ray, no skipping and no
         termination.
Calls only the oracle and the input generators.  Run from the repository
root:  python tests/golden/make_amb17_reference.py
"""
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
import synth  # noqa: E402

W = H = 800
VIEWS = 8
PER_VIEW = 16384
OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "amb17_reference.npz")


def pixels():
    return np.stack([synth.pixel_subset(W, H, PER_VIEW, seed=1700 + v) for v in range(VIEWS)]).astype(np.int32)


def rays(om_cam_fn, pix):
    o = np.empty((VIEWS * PER_VIEW, 3), np.float32)
    d = np.empty((VIEWS * PER_VIEW, 3), np.float32)
    for v in range(VIEWS):
        oo, dd = oracle.generate_rays(om_cam_fn(v), pix[v].astype(np.int64))
        o[v * PER_VIEW:(v + 1) * PER_VIEW], d[v * PER_VIEW:(v + 1) * PER_VIEW] = oo, dd
    return o, d


def model_and_cams():
    dens, feats = synth.make_scene(160, seed=0)
    mlp = synth.make_mlp(1)
    om = oracle.Model(dens, feats, mlp, density_shift=synth.DENSITY_SHIFT)
    om.set_occupancy(oracle.build_occupancy(om, synth.OCC_SIGMA))
    f, cx, cy = synth.intrinsics(W, H)
    poses = synth.sphere_poses(VIEWS, seed=2)
    return om, (lambda v: oracle.camera(W, H, f, cx, cy, synth.as_f32(poses[v])))


def main():
    om, cam = model_and_cams()
    pix = pixels()
    o, d = rays(cam, pix)
    t0 = time.time()
    o64, _, _ = oracle.render_rays(om, oracle.opts(256, 1e-4, True), o, d)
    t1 = time.time()
    g, _, _ = oracle.render_rays(om, oracle.opts(1024), o, d)
    t2 = time.time()
    meta = {"views": VIEWS, "per_view": PER_VIEW, "width": W, "height": H, "scene_seed": 0, "mlp_seed": 1,
            "pose_seed": 2, "pixel_seed": "1700 + view", "o64": "256 samples, occupancy, termination 1e-4",
            "g": "1024 samples, no skipping, no termination"}
    np.savez_compressed(OUT, pix=pix, o64=o64.astype(np.float32), g=g.astype(np.float32),
                        meta=np.array(json.dumps(meta)))
    print("wrote %s (o64 %.1f s, g %.1f s, %d threads)" % (OUT, t1 - t0, t2 - t1, oracle.num_threads()))


if __name__ == "__main__":
    main()
