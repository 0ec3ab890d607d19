"""Pin for the oracle's bfloat16 one-step diagnostic, which bounds how far a
float32 kernel that rounds the same values to bfloat16 may drift from the
oracle when one rounded value lands on the adjacent bfloat16 number.

A single-sample ray through a box of constant density and constant features
has compositing weight 1 - exp(-sigma L) and an MLP input fixed by the
feature vector and the view encoding; the largest first-order colour change
of one bfloat16 step of one MLP input value is then computed independently
with torch autograd (the layer Jacobians through the active ReLUs, rounding
passed straight through) and numpy's float32 spacing scaled to bfloat16's
8-bit significand."""
import math

import numpy as np
import torch

import synth


def test_flip_effect_matches_autograd(orc):
    rng = np.random.default_rng(90)
    R = 5
    fvec = rng.normal(0, 1.2, 12).astype(np.float32)
    feats = np.broadcast_to(fvec, (R, R, R, 12)).copy()
    raw, shift = 0.7, -0.2
    dens = np.full((R, R, R), raw, np.float32)
    mlp = synth.make_mlp(91, bias_std=0.2)
    m = orc.Model(dens, feats, mlp, density_shift=shift, round_bf16=True)
    f, cx, cy = synth.intrinsics(16, 16)
    cam = orc.camera(16, 16, f, cx, cy, synth.as_f32(synth.orbit_pose(3)))
    pix = np.arange(0, 256, 7)
    _, _, acc, diag = orc.render_pixels(m, orc.opts(1), cam, pix, flip=True)
    o, d = orc.generate_rays(cam, pix)
    hit = acc > 0
    assert hit.sum() > 10

    def r(t):
        return t.to(torch.float32).to(torch.bfloat16).to(torch.float64)

    W = {k: torch.from_numpy(mlp[k].astype(np.float64)) for k in mlp}
    Wr = {k: (r(W[k]) if k.startswith("w") else W[k]) for k in W}

    def bf16_step(v):
        v32 = np.abs(v.numpy().astype(np.float32))
        return torch.from_numpy(np.where(v32 == 0, 0.0, np.spacing(v32).astype(np.float64) * 2.0 ** 16))

    for k in np.nonzero(hit)[0]:
        x = torch.from_numpy(orc.mlp_input(m, fvec[None].astype(np.float64), d[k:k + 1])[0])
        xr = r(x)
        h1 = torch.relu(Wr["w0"] @ xr + W["b0"])
        h1r = r(h1)
        h2 = torch.relu(Wr["w1"] @ h1r + W["b1"])
        h2r = r(h2)
        c = torch.sigmoid(Wr["w2"] @ h2r + W["b2"])
        # rounding passed straight through: the value is the rounded one, the
        # derivative that of the identity
        def st(t):
            return t + (r(t) - t).detach()

        def from_h2(v):
            return Wr["w2"] @ v + W["b2"]

        def from_h1(v):
            return from_h2(st(torch.relu(Wr["w1"] @ v + W["b1"])))

        def from_x(v):
            return from_h1(st(torch.relu(Wr["w0"] @ v + W["b0"])))

        J2 = torch.autograd.functional.jacobian(from_h2, h2r)
        J1 = torch.autograd.functional.jacobian(from_h1, h1r)
        J0 = torch.autograd.functional.jacobian(from_x, xr)
        g = torch.stack([(J2.abs() * bf16_step(h2r)).max(1).values, (J1.abs() * bf16_step(h1r)).max(1).values,
                         (J0.abs() * bf16_step(xr)).max(1).values]).max(0).values
        effect = float((g * c * (1 - c)).max())
        w = float(acc[k])     # one sample: its weight is the ray's opacity
        sigma = math.log1p(math.exp(float(np.float32(raw)) + float(np.float32(shift))))
        tn, tf, _ = orc.ray_box(o[k:k + 1], d[k:k + 1])
        assert abs(w - (1 - math.exp(-sigma * float(tf[0] - tn[0])))) < 1e-6
        assert effect > 0
        assert abs(diag["flip"][k] - w * effect) <= 1e-12 * w * effect + 1e-300, (diag["flip"][k], w * effect)
    # no MLP evaluated on a miss: nothing can flip
    assert np.all(diag["flip"][~hit] == 0.0)
