#!/usr/bin/env python3
"""Benchmark of the dense-grid NeRF renderer with sparse radiance warping on
one MI355X.

Timed step: one full 800x800 frame of the 160^3 scene (FP32 grid and MLP, up
to 256 samples per ray, occupancy skipping, early termination at 1e-4)
through render_frame; value = evaluated ray samples per second (samples that
pass through the MLP), inputs resident in HBM.  After the timed region the
same JSON line reports the other measured forms as sub-objects: the 32-frame
SpaRW orbit (FPS, mask fraction, PSNR against full renders), the precision
path (8 views in one call, FP16 grid + BF16 MLP, against FP32 on the same
rays), the fwd+bwd training step, and the per-stage times.  The roofline object is for the dominant kernel (the
feature-gather + MLP stage), timed with HIP events on its launch stream.
The CPU baseline is the plain oracle on a bounded, seeded pixel sample.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W]
"""
import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "ray samples/s + 800x800 FPS (full vs SpaRW); fwd+bwd samples/s; BF16 vs FP32"
MLP_FLOP_PER_SAMPLE = 2 * (12 * 128 + 128 * 128 + 128 * 3)   # 36,608 useful FLOP
PEAK_FP32_TFLOPS = 157.3
PEAK_HBM_GBS = 8000.0
# Training step, per evaluated sample, the method's own work on FP32 MFMA:
# the forward render (as above), the adjoint's forward recomputation (the
# same 36,608 useful FLOP: the view-encoding part of layer 0 is per ray), the
# MLP backward (W1^T dp1 and the feature rows of W0^T dp0) and the weight
# gradients (outer products of the three layers): 152,576 FLOP per sample.
RECOMPUTE_FLOP_PER_SAMPLE = MLP_FLOP_PER_SAMPLE                      # 36,608
BWD_FLOP_PER_SAMPLE = 2 * (128 * 128 + 12 * 128)                     # 35,840
WGRAD_FLOP_PER_SAMPLE = 2 * (128 * 39 + 128 * 128 + 3 * 128)        # 43,520
# Compositing adjoint, algorithmic bytes per live sample: weight, colour and
# distance in, density and colour gradients out (4 + 12 + 4 + 4 + 12 + 4).
BWD_COMPOSITE_BYTES_PER_SAMPLE = 40
# Warp of a W x H reference into a W x H target, algorithmic bytes per pixel:
# reference colour + z-depth read (16), z-buffer clear (8), one 64-bit
# atomic per splat (8), resolve: z-buffer read (8), winner colour + depth
# read (16), colour, depth and mask written (12 + 4 + 1), hole list (~3).
WARP_BYTES_PER_PIXEL = 76


def log(msg):
    print("[bench] " + msg, file=sys.stderr, flush=True)


def psnr(a, b):
    import torch
    mse = torch.mean((a.double() - b.double()) ** 2).item()
    return float("inf") if mse == 0 else 10.0 * math.log10(1.0 / mse)


def build_scene(res, device):
    import synth
    import paper_2404_11852_amd as cic
    dens, feats = synth.make_scene(res, seed=0)
    mlp = synth.make_mlp(1)
    model = cic.Model(dens, feats, mlp, device=device, density_shift=synth.DENSITY_SHIFT)
    model.build_occupancy(synth.OCC_SIGMA)
    return model, (dens, feats, mlp)


def camera(W, H, pose):
    import synth
    import paper_2404_11852_amd as cic
    f, cx, cy = synth.intrinsics(W, H)
    return cic.make_camera(W, H, f, cx, cy, synth.as_f32(pose))


# Counted traffic (bytes beyond L2: FETCH_SIZE x 2.000 + WRITE_SIZE x 1.000,
# calibrated on a 1 GiB copy), L2 hit rate and MFMA busy fraction, from the rocprofv3 counter
# passes summarised in profiles/counters_800x800_frame.md, per launch of:
#   fp32       the headline MLP kernel (ray order, 800x800 frame)
#   bf16_ray   the BF16 MLP over the 8-view pass (3 chunks), ray order
#   bf16_voxel the same in voxel order with LDS brick tiles
#   adjoint    the fused MLP adjoint of the 8192-ray training step
#   backward_grid  the same step's compositing adjoint and grid-gradient kernels
# each valid for the kernel sources it was counted on (sha256 prefix of the
# listed files); a changed source reports None.
COUNTED = {
    "fp32": (3.477e9 + 0.723e9, 0.812, 0.85, ("mlp.hip", "mlp_common.h", "common.h", "kernels.h"),
             "f098081d8dbefc0b"),
    "bf16_ray": (14.656e9 + 5.362e9, 0.849, 0.38, ("mlp_bf16.hip", "mlp_common.h", "common.h", "kernels.h"),
                 "d47056beed240362"),
    "bf16_voxel": (23.608e9 + 6.942e9, 0.245, 0.50, ("mlp_bf16.hip", "mlp_common.h", "common.h", "kernels.h"),
                   "d47056beed240362"),
    "adjoint": (0.624e9 + 0.162e9, 0.373, 0.68, ("backward.hip", "mlp_common.h", "common.h", "kernels.h"),
                "4466ec48d1580a7d"),
    # compositing adjoint + brick-segment gradient tiles + tile gather (one step)
    "backward_grid": (0.323e9 + 0.008e9 + 0.241e9 + 0.307e9 + 0.689e9 + 0.212e9, None, None,
                      ("backward.hip", "mlp_common.h", "common.h", "kernels.h"), "4466ec48d1580a7d"),
}
# feature bytes a sample's gather requests from the grid in the MLP kernel:
# 8 vertices x 12 channels x 4 B (the density is gathered by the march)
GATHER_BYTES_PER_SAMPLE = 8 * 12 * 4


def counted(key):
    """(bytes per launch, L2 hit, MFMA busy) as counted, or Nones once the
    kernel sources differ from the ones the counters were taken on."""
    import hashlib
    nbytes, hit, busy, files, src = COUNTED[key]
    csrc = os.path.join(os.path.dirname(os.path.abspath(__file__)), "paper_2404_11852_amd", "csrc")
    h = hashlib.sha256()
    for f in files:
        with open(os.path.join(csrc, f), "rb") as fh:
            h.update(fh.read())
    return (nbytes, hit, busy) if h.hexdigest()[:16] == src else (None, None, None)


def hbm_block(key, ms):
    """Counted traffic of one launch and its rate against the HBM peak."""
    nbytes, hit, busy = counted(key)
    if nbytes is None or ms <= 0:
        return {"traffic": None, "hbm_frac": None, "l2_hit": None, "mfma_busy": None}
    return {"traffic": nbytes, "hbm_frac": nbytes / (ms * 1e-3) / 1e9 / PEAK_HBM_GBS, "l2_hit": hit,
            "mfma_busy": busy}


def workspace_bench(model, opts, cam, W, H, steps):
    """The headline frame with the workspace bounded: the library runs the
    rays in as many passes as the bound needs (same image bits)."""
    import torch
    import paper_2404_11852_amd as cic
    from paper_2404_11852_amd import _lib
    full = _lib.workspace_bytes(_lib.OP_RENDER_FRAME, W * H, model.grid, opts)
    one = _lib.workspace_bytes(_lib.OP_RENDER_FRAME, 1, model.grid, opts)
    per_ray = (full - one) / (W * H - 1)
    out = {"one_pass_bytes": full, "bytes_per_ray": per_ray}
    ref = cic.render_frame(model, opts, cam)[0]
    for gb in (2, 1):
        lim = gb << 30
        try:
            cic.set_workspace_limit(lim)
            t, _, _ = timed_frames(model, opts, cam, steps, 1)
            img = cic.render_frame(model, opts, cam)[0]
        finally:
            cic.set_workspace_limit(None)
        rays = int((lim - one) // per_ray) + 1
        out["limit_%dGiB" % gb] = {"ms_per_frame": 1e3 * t / steps, "passes": -(-(W * H) // rays),
                                   "same_image": bool(torch.equal(img, ref))}
    return out


def stage_rooflines(stage_ms, live, rays):
    """Fractions of the frame's other stages against their bounds, from
    lower-bound algorithmic work on counts the host knows (live samples and
    rays of the frame): the march writes each live sample's slot (index 2 B,
    weight 4 B) and per ray its interval record and count (20 B) after reading
    the ray (24 B) -- its occupancy and density reads depend on the scene and
    are left out, so its figure is a floor; the compaction reads the slots
    (6 B) and writes the ray-ordered records (ray 4, index 2, weight 4 B),
    plus the ray's count and offset (8 B); the reduce reads weight and colour
    (16 B) per live sample and writes colour, depth and opacity (20 B) per
    ray; the per-ray direction term costs 6,912 FLOP per ray on the vector
    ALUs (FP32 vector peak 157.3 TFLOP/s)."""
    out = {}
    work = {"march": (6 * live + 44 * rays, "hbm"), "compact": (16 * live + 8 * rays, "hbm"),
            "reduce": (16 * live + 20 * rays, "hbm"), "embed": (6912 * rays, "valu")}
    for k, (w, bound) in work.items():
        ms = stage_ms.get(k, 0.0)
        if ms <= 0:
            continue
        if bound == "hbm":
            gbs = w / (ms * 1e-3) / 1e9
            out[k] = {"bound": "hbm", "achieved": gbs, "peak": PEAK_HBM_GBS, "unit": "GB/s",
                      "frac": gbs / PEAK_HBM_GBS, "bytes": w}
        else:
            tf = w / (ms * 1e-3) / 1e12
            out[k] = {"bound": "valu", "achieved": tf, "peak": PEAK_FP32_TFLOPS, "unit": "TFLOP/s",
                      "frac": tf / PEAK_FP32_TFLOPS, "flop": w}
    return out


def measure_peaks():
    """On-box check of the published peaks the fractions use: a 2 GiB
    device-to-device copy (read + write bytes per second) and 8192^3 float32
    and bfloat16 matrix products through torch."""
    import torch
    out = {}
    src = torch.empty(1 << 29, dtype=torch.float32, device="cuda:0").fill_(1.0)
    dst = torch.empty_like(src)
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    for _ in range(2):
        dst.copy_(src)
    a.record()
    for _ in range(5):
        dst.copy_(src)
    b.record()
    torch.cuda.synchronize()
    out["copy_GBs"] = 5 * 2 * src.numel() * 4 / (a.elapsed_time(b) * 1e-3) / 1e9
    del src, dst
    m = torch.randn(8192, 8192, device="cuda:0")
    n = torch.randn(8192, 8192, device="cuda:0")
    for _ in range(2):
        torch.mm(m, n)
    a.record()
    for _ in range(5):
        torch.mm(m, n)
    b.record()
    torch.cuda.synchronize()
    out["fp32_gemm_TFs"] = 5 * 2 * 8192 ** 3 / (a.elapsed_time(b) * 1e-3) / 1e12
    # the same product in bfloat16 (2-D, contiguous operands)
    mb, nb = m.to(torch.bfloat16).contiguous(), n.to(torch.bfloat16).contiguous()
    for _ in range(3):
        torch.mm(mb, nb)
    a.record()
    for _ in range(10):
        torch.mm(mb, nb)
    b.record()
    torch.cuda.synchronize()
    out["bf16_gemm_TFs"] = 10 * 2 * 8192 ** 3 / (a.elapsed_time(b) * 1e-3) / 1e12
    out["published"] = {"hbm_GBs": PEAK_HBM_GBS, "fp32_mfma_TFs": PEAK_FP32_TFLOPS, "bf16_mfma_TFs": 2500.0}
    return out


def timed_frames(model, opts, cam, steps, warmup):
    """Warm up, then time exactly `steps` render_frame calls."""
    import torch
    import paper_2404_11852_amd as cic
    from paper_2404_11852_amd import _lib
    for _ in range(warmup):
        cic.render_frame(model, opts, cam)
    n_eval = torch.zeros(1, dtype=torch.int64, device=model.device)
    torch.cuda.synchronize()
    _lib.timing_enable(True)
    t0 = time.perf_counter()
    for _ in range(steps):
        cic.render_frame(model, opts, cam, n_eval=n_eval)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    stages = _lib.timing_read()
    _lib.timing_enable(False)
    return t1 - t0, int(n_eval.item()), stages


def sparw_orbit(model, opts, W, H, n_frames=32, ref_every=16, max_angle_deg=0.0, full=None):
    """Orbit of n_frames, references every ref_every-th frame rendered in
    full, targets warped from the nearest reference (ties to the earlier one)
    with holes re-rendered; max_angle_deg > 0 turns on the warp-angle test.
    Returns timing and quality against full renders (passed in as `full`, or
    rendered here)."""
    import torch
    import synth
    import paper_2404_11852_amd as cic
    from paper_2404_11852_amd import _lib
    poses = [synth.orbit_pose(k) for k in range(n_frames)]
    refs = list(range(0, n_frames, ref_every))
    cams = [camera(W, H, p) for p in poses]
    sopts = cic.make_opts(opts.n_samples, opts.et_threshold, bool(opts.use_occupancy), tuple(opts.bg),
                          opts.void_acc, opts.order, warp_max_angle=max_angle_deg)

    def nearest(k):
        return min(refs, key=lambda r: (abs(k - r), r))

    def run():
        out = {}
        ref_img = {}
        nm = []
        for k in range(n_frames):
            if k in refs:
                rgb, dz, _ = cic.render_frame(model, opts, cams[k])
                ref_img[k] = (rgb, dz)
                out[k] = rgb
        for k in range(n_frames):
            if k in refs:
                continue
            r = nearest(k)
            T = synth.relative_pose(synth.as_f32(poses[r]), synth.as_f32(poses[k]))
            rgb, dz, mask, n_masked = cic.render_frame_sparw(model, sopts, cams[r], ref_img[r][0], ref_img[r][1],
                                                             cams[k], torch.from_numpy(T))
            out[k] = rgb
            nm.append(n_masked)
        return out, nm

    run()   # warm-up
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    out, nm = run()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    # per-target time, references excluded
    ref_rgbd = {r: cic.render_frame(model, opts, cams[r])[:2] for r in refs}
    torch.cuda.synchronize()
    _lib.timing_enable(True)
    tt0 = time.perf_counter()
    for k in range(n_frames):
        if k in refs:
            continue
        r = nearest(k)
        T = synth.relative_pose(synth.as_f32(poses[r]), synth.as_f32(poses[k]))
        cic.render_frame_sparw(model, sopts, cams[r], ref_rgbd[r][0], ref_rgbd[r][1], cams[k], torch.from_numpy(T))
    torch.cuda.synchronize()
    tt1 = time.perf_counter()
    st = _lib.timing_read()
    _lib.timing_enable(False)
    full_s = None
    if full is None:
        full_t0 = time.perf_counter()
        full = [cic.render_frame(model, opts, c)[0] for c in cams]
        torch.cuda.synchronize()
        full_s = time.perf_counter() - full_t0
    ps = [psnr(out[k], full[k]) for k in range(n_frames) if k not in refs]
    fr = [int(x.item()) / float(W * H) for x in nm]
    n_t = n_frames - len(refs)
    res = {
        "frames": n_frames, "references": len(refs), "window": ref_every, "max_angle_deg": max_angle_deg,
        "fps": n_frames / (t1 - t0),
        "ms_per_target": 1e3 * (tt1 - tt0) / n_t,
        "mask_fraction_mean": sum(fr) / len(fr), "mask_fraction_max": max(fr),
        "psnr_vs_full_mean_db": sum(ps) / len(ps), "psnr_vs_full_min_db": min(ps),
    }
    # per-target stage times (warp, then the hole rays through march ... reduce)
    res["stage_ms_per_target"] = {k: v[0] / n_t for k, v in st.items() if v[1]}
    warp_ms, warp_n = st["warp"]
    if warp_n:
        gbs = WARP_BYTES_PER_PIXEL * W * H / (warp_ms / warp_n * 1e-3) / 1e9
        res["warp_roofline"] = {"bound": "hbm", "achieved": gbs, "peak": PEAK_HBM_GBS, "unit": "GB/s",
                                "frac": gbs / PEAK_HBM_GBS, "ms_per_warp": warp_ms / warp_n,
                                "bytes_per_warp": WARP_BYTES_PER_PIXEL * W * H}
    if full_s is not None:
        res["fps_full_render"] = n_frames / full_s
        res["speedup_vs_full"] = full_s / (t1 - t0)
    return res, full


def sparw_sweep(model, opts, W, H, windows=(6, 16, 26), angles=(0.0, 8.0, 4.0, 2.0), n_frames=32):
    """Window / warp-angle sweep over one orbit (Sec. III-C): the first entry
    (window 16, no angle test) also carries the full-render comparison."""
    base, full = sparw_orbit(model, opts, W, H, n_frames=n_frames, ref_every=16)
    sweep = []
    for w in windows:
        for a in angles:
            if w == 16 and a == 0.0:
                r = dict(base)
            else:
                r, _ = sparw_orbit(model, opts, W, H, n_frames=n_frames, ref_every=w, max_angle_deg=a, full=full)
            r["speedup_vs_full"] = base["fps_full_render"] and r["fps"] / base["fps_full_render"]
            sweep.append({k: r[k] for k in ("window", "max_angle_deg", "fps", "ms_per_target", "mask_fraction_mean",
                                            "psnr_vs_full_mean_db", "psnr_vs_full_min_db", "speedup_vs_full")})
    base["sweep"] = sweep
    return base


def sparw_bf16(scene, occ, W, H):
    """The 32-frame SpaRW orbit (window 16) with the precision path: FP16
    grids and the BF16 MLP, in ray and in voxel order; PSNR against the same
    model's full renders."""
    import torch
    import synth
    import paper_2404_11852_amd as cic
    dens, feats, mlp = scene
    m = cic.Model(dens, feats, mlp, device="cuda:0", storage=torch.float16, density_shift=synth.DENSITY_SHIFT,
                  compute=cic.CIC_BF16)
    m.set_occupancy(occ)
    out = {}
    for name, order in (("ray", cic.CIC_ORDER_RAY), ("voxel", cic.CIC_ORDER_VOXEL)):
        r, _ = sparw_orbit(m, cic.make_opts(256, 1e-4, True, order=order), W, H, n_frames=32, ref_every=16)
        out[name] = {k: r[k] for k in ("fps", "ms_per_target", "fps_full_render", "speedup_vs_full",
                                       "mask_fraction_mean", "psnr_vs_full_mean_db", "psnr_vs_full_min_db",
                                       "stage_ms_per_target")}
    return out


def sequence_bench(model, opts, W, H, n_frames=65, window=16):
    """Off-trajectory references (Eq. 5-6) over an orbit: the two-stream
    schedule against the serial one, and the paper's lead of half a window
    against a lead that centres each reference on the window it serves.
    Reports throughput, the frame clock (intervals between consecutive frame
    completions) and PSNR against full renders."""
    import numpy as np
    import torch
    import synth
    import paper_2404_11852_amd as cic
    from paper_2404_11852_amd import _lib
    cams = [camera(W, H, synth.orbit_pose(k)) for k in range(n_frames)]
    full = [cic.render_frame(model, opts, c)[0] for c in cams]
    torch.cuda.synchronize()

    def run(overlap, lead, part=0):
        cic.render_sequence(model, opts, cams, window, lead=lead, overlap=overlap, target_cus_per_xcd=part)
        torch.cuda.synchronize()
        _lib.timing_enable(True)
        t0 = time.perf_counter()
        rgb, dz, mask, nm, refs = cic.render_sequence(model, opts, cams, window, lead=lead, overlap=overlap,
                                                      target_cus_per_xcd=part)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        clock = _lib.timing_frames()
        _lib.timing_enable(False)
        iv = np.diff(np.array(clock))     # intervals between target frames (frame 0 reported apart)
        ps = [psnr(rgb[k], full[k]) for k in range(1, n_frames)]
        fr = (nm[1:].double() / (W * H)).cpu().numpy()
        return {"overlap": overlap, "target_cus_per_xcd": part, "lead_frames": window / 2.0 if lead < 0 else lead,
                "fps": n_frames / (t1 - t0), "ms_total": 1e3 * (t1 - t0), "frame0_ms": float(clock[0]),
                "frame_interval_ms": {"p50": float(np.percentile(iv, 50)), "p95": float(np.percentile(iv, 95)),
                                      "max": float(iv.max())},
                "mask_fraction_mean": float(fr.mean()),
                "psnr_vs_full_mean_db": float(np.mean(ps)), "psnr_vs_full_min_db": float(np.min(ps))}

    res = {"frames": n_frames, "window": window, "references": 1 + (n_frames - 1 + window - 1) // window - 1,
           "runs": [run(False, -1.0), run(True, -1.0), run(True, 1.5 * window)]
           + [run(True, -1.0, t) for t in (16, 20, 24)] + [run(True, 1.5 * window, 20)]}
    return res


def variants_bench(model, opts, W, H, n_frames=32):
    """The paper's comparison variants on the same 32-frame orbit as the
    SpaRW sweep: DS-2 (half resolution + bilinear upsample) and Temp-N
    (warp from the previous output frame, full render every N frames), with
    PSNR against full renders of the same frames."""
    import numpy as np
    import torch
    import synth
    import paper_2404_11852_amd as cic
    cams = [camera(W, H, synth.orbit_pose(k)) for k in range(n_frames)]
    full = [cic.render_frame(model, opts, c)[0] for c in cams]
    torch.cuda.synchronize()
    out = {}
    for fac in (2,):
        [cic.render_frame_ds(model, opts, cams[0], fac) for _ in range(2)]
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        imgs = [cic.render_frame_ds(model, opts, c, fac) for c in cams]
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        ps = [psnr(imgs[k], full[k]) for k in range(n_frames)]
        out["ds%d" % fac] = {"fps": n_frames / (t1 - t0), "psnr_vs_full_mean_db": float(np.mean(ps)),
                             "psnr_vs_full_min_db": float(np.min(ps))}
    for win in (6, 16):
        cic.render_temporal(model, opts, cams, win)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        rgb, dz, mask, nm = cic.render_temporal(model, opts, cams, win)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        ps = [psnr(rgb[k], full[k]) for k in range(n_frames) if k % win]
        fr = [int(nm[k]) / float(W * H) for k in range(n_frames) if k % win]
        out["temp%d" % win] = {"fps": n_frames / (t1 - t0), "psnr_vs_full_mean_db": float(np.mean(ps)),
                               "psnr_vs_full_min_db": float(np.min(ps)), "mask_fraction_mean": float(np.mean(fr))}
    return out


def hash_bench(W, H, steps, dense_ms=None):
    """The multi-level encoding workload (hierarchical encodings): the same
    160^3 density grid and MLP, features from 4 levels of 3 features (32, 64,
    128, 256 cells per axis; 2^19-entry tables, the two finest levels
    hashed), 800x800 frames in ray and voxel order, with float32 tables and
    the FP32 MLP, then with float16 tables and the BF16 MLP (voxel order
    stages each segment's level boxes in LDS)."""
    import synth
    import paper_2404_11852_amd as cic
    dens, _ = synth.make_scene(160, seed=0)
    h = synth.make_hash_tables(30)
    model = cic.Model(dens, None, synth.make_mlp(1), density_shift=synth.DENSITY_SHIFT, hash_enc=h)
    model.build_occupancy(synth.OCC_SIGMA)
    cam = camera(W, H, synth.orbit_pose(0))
    import torch
    bmodel = cic.Model(dens, None, synth.make_mlp(1), storage=torch.float16, density_shift=synth.DENSITY_SHIFT,
                       hash_enc=h, compute=cic.CIC_BF16)
    bmodel.set_occupancy(model.occupancy)
    out = {"levels_cells": list(h["res"]), "log2_table": h["log2_size"],
           "hashed_levels": [int((r + 1) ** 3 > (1 << h["log2_size"])) for r in h["res"]]}
    imgs = {}
    for name, m, order in (("ray", model, cic.CIC_ORDER_RAY), ("voxel", model, cic.CIC_ORDER_VOXEL),
                           ("bf16_ray", bmodel, cic.CIC_ORDER_RAY), ("bf16_voxel", bmodel, cic.CIC_ORDER_VOXEL)):
        opts = cic.make_opts(256, et_threshold=1e-4, use_occupancy=True, order=order)
        t, n_eval, stages = timed_frames(m, opts, cam, steps, 2)
        ms = 1e3 * t / steps
        sm = {k: v[0] / max(v[1], 1) * (v[1] / steps) for k, v in stages.items() if v[1]}
        out[name] = {"ms_per_frame": ms, "samples_per_s": n_eval / t, "stage_ms": sm}
        mlp_ms = sm.get("mlp", 0.0)
        if mlp_ms > 0:
            bf = name.startswith("bf16")
            peak = 2500.0 if bf else PEAK_FP32_TFLOPS
            ach = MLP_FLOP_PER_SAMPLE * (n_eval / steps) / (mlp_ms * 1e-3) / 1e12
            out[name]["mlp_roofline"] = {"bound": "mfma", "achieved": ach, "peak": peak, "unit": "TFLOP/s",
                                         "frac": ach / peak}
        if name.startswith("bf16"):
            imgs[name] = cic.render_frame(m, opts, cam)[0]
    out["bf16_tables"] = "float16 (the multi-level tables), MLP in BF16"
    out["bf16_voxel_equals_ray_order"] = bool(torch.equal(imgs["bf16_ray"], imgs["bf16_voxel"]))
    return out


AMB17_GOLDEN = os.path.join(ROOT, "tests", "golden", "amb17_reference.npz")


def precision_bench(scene, occ, steps):
    """Eight 800x800 views on the radius-4 sphere in one render_rays call:
    FP16 grids + BF16 MLP against the FP32 path on the same rays.  Quality:
    PSNR against the float64 oracle's converged reference G (1024 samples,
    no skipping or termination) on 16,384 seeded pixels per view, from the
    stored oracle colours in tests/golden/amb17_reference.npz (written by
    make_amb17_reference.py), next to the oracle's own PSNR at the
    workload's settings; margin = PSNR(G, BF16) - (PSNR(G, oracle) - 0.1 dB).
    The two error sources are measured apart: FP16 grid with the FP32 MLP,
    FP32 grid with the BF16 MLP."""
    import numpy as np
    import torch
    import synth
    import paper_2404_11852_amd as cic
    from paper_2404_11852_amd import _lib
    dens, feats, mlp = scene
    W = H = 800
    models = {}
    for name, storage, compute in (("bf16", torch.float16, cic.CIC_BF16), ("fp32", torch.float32, cic.CIC_F32),
                                   ("f32grid_bf16mlp", torch.float32, cic.CIC_BF16),
                                   ("f16grid_f32mlp", torch.float16, cic.CIC_F32)):
        m = cic.Model(dens, feats, mlp, device="cuda:0", storage=storage, density_shift=synth.DENSITY_SHIFT,
                      compute=compute)
        m.set_occupancy(occ)
        models[name] = m
    f, cx, cy = synth.intrinsics(W, H)
    rays = [cic.generate_rays(cic.make_camera(W, H, f, cx, cy, synth.as_f32(p))) for p in synth.sphere_poses(8, 2)]
    o = torch.cat([r[0] for r in rays]).contiguous()
    d = torch.cat([r[1] for r in rays]).contiguous()
    go = cic.make_opts(256, 1e-4, True)
    gv = cic.make_opts(256, 1e-4, True, order=cic.CIC_ORDER_VOXEL)
    out = {}
    imgs = {}
    for name, model, go in (("bf16", models["bf16"], go), ("bf16_voxel", models["bf16"], gv),
                            ("fp32", models["fp32"], go)):
        cic.render_rays(model, go, o, d)
        n_eval = torch.zeros(1, dtype=torch.int64, device="cuda:0")
        torch.cuda.synchronize()
        _lib.timing_enable(True)
        t0 = time.perf_counter()
        for _ in range(steps):
            rgb, _, _ = cic.render_rays(model, go, o, d, n_eval=n_eval)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        st = _lib.timing_read()
        _lib.timing_enable(False)
        imgs[name] = rgb
        ne = int(n_eval.item()) / steps
        out[name] = {"samples_per_s": ne * steps / (t1 - t0), "ms_per_launch": 1e3 * (t1 - t0) / steps,
                     "fps_800x800_per_view": 8 * steps / (t1 - t0), "evaluated_samples": ne,
                     "stage_ms": {k: v[0] / steps for k, v in st.items() if v[1]}}
    out["speedup_bf16_vs_fp32"] = out["bf16"]["samples_per_s"] / out["fp32"]["samples_per_s"]
    out["speedup_bf16_voxel_vs_fp32"] = out["bf16_voxel"]["samples_per_s"] / out["fp32"]["samples_per_s"]
    out["bf16_voxel_equals_ray_order"] = bool(torch.equal(imgs["bf16_voxel"], imgs["bf16"]))
    out["psnr_bf16_vs_fp32_gpu_db"] = psnr(imgs["bf16"], imgs["fp32"])
    out["max_abs_bf16_vs_fp32_gpu"] = float((imgs["bf16"] - imgs["fp32"]).abs().max().item())
    for name, key in (("bf16", "bf16_ray"), ("bf16_voxel", "bf16_voxel")):
        mlp_ms = out[name]["stage_ms"].get("mlp", 0.0)
        if mlp_ms > 0:
            ach = MLP_FLOP_PER_SAMPLE * out[name]["evaluated_samples"] / (mlp_ms * 1e-3) / 1e12
            out[name + "_mlp_roofline"] = dict({"bound": "mfma", "achieved": ach, "peak": 2500.0, "unit": "TFLOP/s",
                                                "frac": ach / 2500.0}, **hbm_block(key, mlp_ms))
    if os.path.exists(AMB17_GOLDEN):
        gold = np.load(AMB17_GOLDEN)
        pix = gold["pix"]
        sel = torch.from_numpy((np.arange(pix.shape[0])[:, None] * (W * H) + pix).reshape(-1).astype(np.int64))
        g = gold["g"].astype(np.float64)
        o64 = gold["o64"].astype(np.float64)

        def p_np(a, b):
            mse = float(np.mean((a - b) ** 2))
            return float("inf") if mse == 0 else 10.0 * math.log10(1.0 / mse)

        cols = {"bf16": imgs["bf16_voxel"], "fp32": imgs["fp32"]}
        for name in ("f32grid_bf16mlp", "f16grid_f32mlp"):
            cols[name], _, _ = cic.render_rays(models[name], go, o, d)
        q = {"pixels": int(sel.numel()), "psnr_G_oracle_db": p_np(g, o64)}
        for name, img in cols.items():
            v = img[sel.cuda()].double().cpu().numpy()
            q["psnr_G_%s_db" % name] = p_np(g, v)
            q["psnr_oracle_%s_db" % name] = p_np(o64, v)
            q["max_abs_oracle_%s" % name] = float(np.abs(v - o64).max())
        q["margin_db"] = q["psnr_G_bf16_db"] - (q["psnr_G_oracle_db"] - 0.1)
        q["criterion"] = "PSNR(G, BF16) >= PSNR(G, oracle) - 0.1 dB"
        out["quality_vs_converged"] = q
    out["workload"] = "8 views x 800x800 (5.12M rays, one call), 160^3 grid, 256 samples, skip + termination"
    return out


def fwd_bwd_bench(steps):
    """One MSE training step (forward + adjoint) on 8192 rays drawn from 8
    views of a hidden scene; model grids N(0, 0.01), FP32."""
    import numpy as np
    import torch
    import synth
    import paper_2404_11852_amd as cic
    from paper_2404_11852_amd import _lib
    ex = synth.get_config("train8192_views8").extra
    W = H = 800
    f, cx, cy = synth.intrinsics(W, H)
    poses = synth.sphere_poses(8, seed=3)
    view, pix = synth.training_pixels(8, W, H, 8192, seed=ex["ray_seed"])
    o = torch.empty((8192, 3), device="cuda:0")
    d = torch.empty((8192, 3), device="cuda:0")
    for v in range(8):
        sel = torch.from_numpy(np.nonzero(view == v)[0]).cuda()
        oo, dd = cic.generate_rays(cic.make_camera(W, H, f, cx, cy, synth.as_f32(poses[v])),
                                   torch.from_numpy(pix[view == v]))
        o[sel], d[sel] = oo, dd
    gd, gf = synth.make_scene(160, seed=ex["gt_scene_seed"])
    gt_model = cic.Model(gd, gf, synth.make_mlp(ex["gt_mlp_seed"]), device="cuda:0",
                         density_shift=synth.DENSITY_SHIFT)
    go = cic.make_opts(256, 1e-4)
    target, _, _ = cic.render_rays(gt_model, go, o, d)
    md, mf = synth.make_model_grid(160, seed=ex["model_grid_seed"])
    model = cic.Model(md, mf, synth.make_mlp(ex["model_mlp_seed"]), device="cuda:0",
                      density_shift=synth.DENSITY_SHIFT)
    grads = {"density": torch.zeros_like(model.density), "features": torch.zeros_like(model.features)}
    for k, v in model.w.items():
        grads[k] = torch.zeros_like(v)

    def step(n_eval=None):
        for g in grads.values():
            g.zero_()
        rgb, _, _ = cic.render_rays(model, go, o, d, n_eval=n_eval)
        d_rgb = (2.0 / rgb.numel()) * (rgb - target)
        cic.render_backward(model, go, o, d, d_rgb, grads=grads)

    step()
    n_eval = torch.zeros(1, dtype=torch.int64, device="cuda:0")
    torch.cuda.synchronize()
    _lib.timing_enable(True)
    t0 = time.perf_counter()
    for _ in range(steps):
        step(n_eval)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    st = _lib.timing_read()
    _lib.timing_enable(False)
    ne = int(n_eval.item()) / steps
    sm = {k: v[0] / steps for k, v in st.items() if v[1]}
    out = {"samples_per_s": ne * steps / (t1 - t0), "ms_per_step": 1e3 * (t1 - t0) / steps,
           "evaluated_samples_per_step": ne, "stage_ms_per_step": sm,
           "workload": "8192 rays from 8 views, 160^3 model grids N(0,0.01), 256 samples, fwd + adjoint, FP32"}
    mfma_ms = sum(sm.get(k, 0.0) for k in ("mlp", "bwd_mlp"))
    if mfma_ms > 0:
        flop = (MLP_FLOP_PER_SAMPLE + RECOMPUTE_FLOP_PER_SAMPLE + BWD_FLOP_PER_SAMPLE + WGRAD_FLOP_PER_SAMPLE) * ne
        ach = flop / (mfma_ms * 1e-3) / 1e12
        out["mfma_roofline"] = {"bound": "mfma", "stages": "mlp (forward) + bwd_mlp (fused recompute, MLP backward, "
                                                           "weight gradients)",
                                "flop_per_sample": flop / max(ne, 1), "achieved": ach,
                                "peak": PEAK_FP32_TFLOPS, "unit": "TFLOP/s", "frac": ach / PEAK_FP32_TFLOPS,
                                "whole_step_frac": flop / (out["ms_per_step"] * 1e-3) / 1e12 / PEAK_FP32_TFLOPS}
    if sm.get("bwd_mlp", 0.0) > 0:
        out["mfma_roofline"]["adjoint_kernel"] = dict({"stage": "bwd_mlp"}, **hbm_block("adjoint", sm["bwd_mlp"]))
    if sm.get("bwd_composite", 0.0) > 0:
        # the stage: compositing adjoint, brick-segment gradient tiles, their
        # gather into the grids; algorithmic bytes counted for the first only
        gbs = BWD_COMPOSITE_BYTES_PER_SAMPLE * ne / (sm["bwd_composite"] * 1e-3) / 1e9
        out["bwd_composite_roofline"] = dict({"bound": "hbm", "stages": "compositing adjoint + grid-gradient tiles",
                                              "achieved_compositing_bytes": gbs, "peak": PEAK_HBM_GBS,
                                              "unit": "GB/s", "frac": gbs / PEAK_HBM_GBS},
                                             **hbm_block("backward_grid", sm["bwd_composite"]))
    return out


def cpu_baseline(scene, target_s=12.0):
    """The oracle, as it stands, on a seeded pixel sample of the same frame."""
    import numpy as np
    import oracle
    import synth
    dens, feats, mlp = scene
    om = oracle.Model(dens, feats, mlp, density_shift=synth.DENSITY_SHIFT)
    om.set_occupancy(oracle.build_occupancy(om, synth.OCC_SIGMA))
    f, cx, cy = synth.intrinsics(800, 800)
    oc = oracle.camera(800, 800, f, cx, cy, synth.as_f32(synth.orbit_pose(0)))
    op = oracle.opts(256, 1e-4, True)
    n = 512
    while True:
        pix = synth.pixel_subset(800, 800, n, seed=99)
        t0 = time.perf_counter()
        _, _, _, diag = oracle.render_pixels(om, op, oc, pix)
        dt = time.perf_counter() - t0
        if dt >= target_s / 4 or n >= 640000:
            break
        n = min(640000, int(n * max(2.0, (target_s / 4) / max(dt, 1e-3))))
    if dt < target_s and n < 640000:
        n = min(640000, int(n * target_s / max(dt, 1e-3)))
        pix = synth.pixel_subset(800, 800, n, seed=99)
        t0 = time.perf_counter()
        _, _, _, diag = oracle.render_pixels(om, op, oc, pix)
        dt = time.perf_counter() - t0
    ns = int(diag["n_eval"].sum())
    threads = oracle.num_threads()
    # one thread, on a sample sized for about 2 s
    n1 = max(64, min(n, int(n * 2.0 / max(dt * threads, 1e-3))))
    pix1 = synth.pixel_subset(800, 800, n1, seed=98)
    oracle.set_threads(1)
    try:
        t0 = time.perf_counter()
        _, _, _, d1 = oracle.render_pixels(om, op, oc, pix1)
        dt1 = time.perf_counter() - t0
    finally:
        oracle.set_threads(threads)
    model_name = ""
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    model_name = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return {"value": ns / dt, "unit": "samples/s", "cores": threads, "kind": "oracle",
            "sample": "%d seeded pixels of the 800x800 frame (%d evaluated samples, %.1f s)" % (n, ns, dt),
            "single_thread_value": int(d1["n_eval"].sum()) / dt1,
            "single_thread_sample": "%d seeded pixels, %.1f s" % (n1, dt1),
            "host_cpu": model_name, "host_nproc": os.cpu_count()}


def profile_run():
    """Short fixed workload for hardware-counter passes: a 1 GiB device copy
    (calibrates FETCH_SIZE / WRITE_SIZE against known bytes), then two 800x800
    frames in ray order, two in voxel order, one frame of the multi-level
    encoding model in each order (float32 tables, FP32 MLP, then float16
    tables, BF16 MLP), the 8-view precision-path launches (BF16 in ray and in
    voxel order, FP32) and one training step."""
    import torch
    import synth
    import paper_2404_11852_amd as cic
    src = torch.empty(1 << 28, dtype=torch.float32, device="cuda:0").fill_(1.0)
    dst = torch.empty_like(src)
    dst.copy_(src)
    torch.cuda.synchronize()
    del src, dst
    model, scene = build_scene(160, "cuda:0")
    cam = camera(800, 800, synth.orbit_pose(0))
    for order in (cic.CIC_ORDER_RAY, cic.CIC_ORDER_VOXEL):
        opts = cic.make_opts(256, 1e-4, True, order=order)
        for _ in range(2):
            cic.render_frame(model, opts, cam)
    torch.cuda.synchronize()
    dens, _, mlp = scene
    hmodel = cic.Model(dens, None, mlp, density_shift=synth.DENSITY_SHIFT, hash_enc=synth.make_hash_tables(30))
    hmodel.build_occupancy(synth.OCC_SIGMA)
    for order in (cic.CIC_ORDER_RAY, cic.CIC_ORDER_VOXEL):
        cic.render_frame(hmodel, cic.make_opts(256, 1e-4, True, order=order), cam)
    torch.cuda.synchronize()
    bmodel = cic.Model(dens, None, mlp, storage=torch.float16, density_shift=synth.DENSITY_SHIFT,
                       hash_enc=synth.make_hash_tables(30), compute=cic.CIC_BF16)
    bmodel.set_occupancy(model.occupancy)
    for order in (cic.CIC_ORDER_RAY, cic.CIC_ORDER_VOXEL):
        cic.render_frame(bmodel, cic.make_opts(256, 1e-4, True, order=order), cam)
    torch.cuda.synchronize()
    precision_bench(scene, model.occupancy, 1)
    fwd_bwd_bench(1)
    torch.cuda.synchronize()
    print("profile run done", flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--order", choices=["ray", "voxel"], default="ray")
    ap.add_argument("--skip-sparw", action="store_true")
    ap.add_argument("--skip-hash", action="store_true")
    ap.add_argument("--skip-cpu", action="store_true")
    ap.add_argument("--skip-precision", action="store_true")
    ap.add_argument("--skip-fwd-bwd", action="store_true")
    ap.add_argument("--profile-run", action="store_true",
                    help="run the short fixed workload used for rocprofv3 counter passes and exit")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: the library has no multi-GPU path "
              "(rays would shard by pixel tiles with the grid replicated). "
              "Run with --gpus 1.", file=sys.stderr)
        sys.exit(2)

    if args.profile_run:
        profile_run()
        return
    import torch
    import paper_2404_11852_amd as cic
    device = "cuda:0"
    W = H = 800
    log("building 160^3 scene")
    model, scene = build_scene(160, device)
    opts = cic.make_opts(256, et_threshold=1e-4, use_occupancy=True,
                         order=cic.CIC_ORDER_VOXEL if args.order == "voxel" else cic.CIC_ORDER_RAY)
    cam = camera(W, H, __import__("synth").orbit_pose(0))

    log("timing %d frames after %d warm-up" % (args.steps, args.warmup))
    dt, n_eval, stages = timed_frames(model, opts, cam, args.steps, args.warmup)
    ms_step = 1e3 * dt / args.steps
    samples_per_frame = n_eval / args.steps
    value = n_eval / dt
    mlp_ms, mlp_n = stages["mlp"]
    mlp_ms_per = mlp_ms / max(mlp_n, 1)
    achieved = MLP_FLOP_PER_SAMPLE * samples_per_frame / (mlp_ms_per * 1e-3) / 1e12
    traffic, l2_hit, mfma_busy = counted("fp32")
    stage_ms = {k: (v[0] / v[1] if v[1] else 0.0) for k, v in stages.items() if v[1]}
    log("%.3f ms/frame, %.3g samples/s, mlp %.3f ms/launch" % (ms_step, value, mlp_ms_per))

    # the other order, for the memory-centric A/B
    other = cic.make_opts(256, et_threshold=1e-4, use_occupancy=True,
                          order=cic.CIC_ORDER_RAY if args.order == "voxel" else cic.CIC_ORDER_VOXEL)
    dt2, n2, st2 = timed_frames(model, other, cam, max(5, args.steps // 2), 1)
    ab = {"order": "voxel" if args.order == "ray" else "ray", "ms_per_frame": 1e3 * dt2 / max(5, args.steps // 2),
          "stage_ms": {k: (v[0] / v[1] if v[1] else 0.0) for k, v in st2.items() if v[1]}}

    out = {
        "metric": METRIC,
        "value": value,
        "unit": "samples/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "800x800 full-frame render, 160^3 dense grid (raw density + 12 features, FP32), "
                               "up to 256 samples/ray, occupancy skip, termination at T<1e-4, "
                               "39-128-128-3 MLP (FP32 MFMA)",
                   "width": W, "height": H, "grid_res": 160, "n_samples": 256, "order": args.order},
        "fps_full_800x800": 1e3 / ms_step,
        "evaluated_samples_per_frame": samples_per_frame,
        "stage_ms_per_launch": stage_ms,
        "stage_rooflines": stage_rooflines(stage_ms, samples_per_frame, W * H),
        "order_ab": ab,
        "roofline": {"bound": "mfma", "kernel": "k_mlp_fwd_f32 (feature gather + MLP)",
                     "achieved": achieved, "peak": PEAK_FP32_TFLOPS, "unit": "TFLOP/s",
                     "frac": achieved / PEAK_FP32_TFLOPS, "traffic": traffic,
                     "flop_per_launch": MLP_FLOP_PER_SAMPLE * samples_per_frame,
                     "ms_per_launch": mlp_ms_per,
                     "hbm_frac": (traffic / (mlp_ms_per * 1e-3) / 1e9 / PEAK_HBM_GBS) if traffic else None,
                     "gather": {"requested_bytes_per_sample": GATHER_BYTES_PER_SAMPLE,
                                "effective_GBs": GATHER_BYTES_PER_SAMPLE * samples_per_frame / (mlp_ms_per * 1e-3) / 1e9,
                                "l2_hit": l2_hit},
                     "mfma_busy": mfma_busy},
    }
    log("bounded workspace")
    out["workspace"] = workspace_bench(model, opts, cam, W, H, max(5, args.steps // 2))
    if not args.skip_hash:
        log("multi-level encoding workload")
        out["hash_encoding"] = hash_bench(W, H, max(3, args.steps // 4))
    if not args.skip_sparw:
        log("SpaRW orbit")
        out["sparw"] = sparw_sweep(model, opts, W, H)
    if not args.skip_sparw:
        log("SpaRW orbit, FP16 grid + BF16 MLP")
        out["sparw_bf16"] = sparw_bf16(scene, model.occupancy, W, H)
    if not args.skip_sparw:
        log("off-trajectory references, serial vs two streams")
        out["sequence"] = sequence_bench(model, opts, W, H)
    if not args.skip_sparw:
        log("comparison variants DS-2, Temp-6, Temp-16")
        out["variants"] = variants_bench(model, opts, W, H)
    if not args.skip_precision:
        log("precision path (8 views, FP16 grid + BF16 MLP)")
        out["precision"] = precision_bench(scene, model.occupancy, max(3, args.steps // 4))
    if not args.skip_fwd_bwd:
        log("fwd+bwd training step")
        out["fwd_bwd"] = fwd_bwd_bench(max(3, args.steps // 2))
    log("on-box peak check (copy, FP32 GEMM)")
    out["peaks_measured"] = measure_peaks()
    if not args.skip_cpu:
        log("CPU baseline (oracle)")
        out["cpu_baseline"] = cpu_baseline(scene)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
