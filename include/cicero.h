/*
 * C interface of the MI355X (gfx950) renderer for grid-based NeRF with
 * sparse radiance warping (SpaRW), after arXiv 2404.11852.
 *
 * General conventions (every entry point):
 *  - All array pointers are DEVICE pointers owned by the caller; the library
 *    never allocates or frees device memory.  Scratch memory is passed in as
 *    a workspace (ws, ws_bytes); its required size comes from
 *    cic_workspace_bytes().  Contents of the workspace are undefined after a
 *    call; it may be reused by the next call on the same stream.
 *  - Calls are asynchronous on `stream` (a hipStream_t; NULL = the null
 *    stream).  No call synchronises the host; counts the GPU produces stay
 *    in device memory.
 *  - Arguments are validated on the host before anything is launched.
 *    Return value: CIC_OK (0), or a negative code: CIC_ERR_INVALID (-1) bad
 *    argument, CIC_ERR_WORKSPACE (-2) workspace too small, CIC_ERR_HIP (-3)
 *    HIP runtime error (launch failure), CIC_ERR_DEVICE (-4) the current
 *    device is not gfx950.  cic_last_error_message() describes the last
 *    failure of the calling thread.
 *  - Gradient outputs of render_backward are ACCUMULATED (+=); the caller
 *    zeroes them.
 *  - Calls that share a workspace must not overlap (same stream, or
 *    ordered by the caller).
 *  - The library keeps no HIP object (stream, event) from one call to the
 *    next: the streams it runs on are the caller's, and the events it needs
 *    live for one call.  The only exception is the benchmark timing hooks
 *    while they are enabled (cic_timing_enable).
 *
 * Data layout:
 *  - Grid: vertices on the corners of the box [box_lo, box_hi] ("align
 *    corners"), res[a] vertices per axis.  density is the raw (pre-
 *    activation) value, [res0][res1][res2] with the last index fastest;
 *    features are [res0][res1][res2][n_feat], channel fastest.  Storage is
 *    float32 or float16 (IEEE binary16) for both.
 *  - Occupancy: one byte per voxel, [(res0-1)][(res1-1)][(res2-1)],
 *    nonzero = occupied (see build_occupancy).
 *  - MLP weights: float32 row-major [out][in]; inputs are the interpolated
 *    features, the view direction and its sinusoidal encoding.
 *  - Rays: rays_o, rays_d float32 [n][3]; directions are expected to be unit
 *    length (distances are measured in units of |d|).
 *  - Frames: pixel p = j*width + i (row j, column i); rgb float32 [H*W][3].
 *  - Cameras: OpenCV axes (x right, y down, z forward); c2w is row-major
 *    3x4 [R | eye]; pixel centres at (i + 1/2, j + 1/2).
 */
#ifndef CICERO_H
#define CICERO_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef void *cic_stream_t; /* hipStream_t */

enum {
    CIC_OK = 0,
    CIC_ERR_INVALID = -1,
    CIC_ERR_WORKSPACE = -2,
    CIC_ERR_HIP = -3,
    CIC_ERR_DEVICE = -4
};

/* storage / compute types */
enum { CIC_F32 = 0, CIC_F16 = 1, CIC_BF16 = 2 };

/* sample processing order for the feature gather + MLP stage */
enum { CIC_ORDER_RAY = 0, CIC_ORDER_VOXEL = 1 };

/* operations, for cic_workspace_bytes */
enum {
    CIC_OP_RENDER_RAYS = 0,
    CIC_OP_RENDER_FRAME = 1,
    CIC_OP_WARP_FRAME = 2,
    CIC_OP_RENDER_FRAME_SPARW = 3,
    CIC_OP_RENDER_BACKWARD = 4,
    CIC_OP_RENDER_SEQUENCE = 5,     /* n_items = pixels per frame */
    CIC_OP_RENDER_FRAME_DS = 6      /* n_items = full-resolution pixels */
};

typedef struct {
    int32_t res[3];            /* vertices per axis, each in [2, 1024] */
    int32_t n_feat;            /* feature channels; must be 12 */
    int32_t storage;           /* CIC_F32 or CIC_F16 (density and features) */
    float box_lo[3];
    float box_hi[3];
    float density_shift;       /* added to the interpolated raw density before softplus */
    const void *density;       /* device, [res0][res1][res2] */
    const void *features;      /* device, [res0][res1][res2][n_feat], 4-byte aligned */
    const uint8_t *occupancy;  /* device, [(res0-1)(res1-1)(res2-1)], or NULL */
    /* Multi-level feature encoding (the hierarchical encodings of Sec. IV-A,
     * as a multiresolution hash grid).  hash_levels = 0: the features come
     * from `features`.  hash_levels = 4: `features` is unused and each
     * sample's 12 features are 3 per level, level l interpolated trilinearly
     * on a grid of hash_res[l] cells per axis over the box; vertex (x, y, z)
     * of level l reads entry (x (N+1) + y)(N+1) + z of the level's table when
     * (N+1)^3 <= 2^hash_log2_size, else entry
     * (x * 1 ^ y * 2654435761 ^ z * 805459861) mod 2^hash_log2_size (32-bit
     * unsigned arithmetic).  Density, occupancy and voxel order still use the
     * dense density grid.  Forward rendering only (render_backward rejects it). */
    int32_t hash_levels;       /* 0 or 4 */
    int32_t hash_res[4];       /* cells per axis of each level, each in [1, 4096] */
    int32_t hash_log2_size;    /* table entries per level = 2^hash_log2_size, in [8, 24] */
    const void *hash_tables;   /* device, [4][2^hash_log2_size][3], of type `storage`, 4-byte aligned */
} cic_grid;

typedef struct {
    int32_t compute;           /* CIC_F32 (FP32 MFMA) or CIC_BF16 (BF16 MFMA, FP32 accumulate) */
    int32_t in_dim;            /* n_feat + 3 + 6*pe_freqs; must be 39 */
    int32_t hidden;            /* must be 128 */
    int32_t pe_freqs;          /* must be 4 */
    const float *w0, *b0;      /* device, [hidden][in_dim], [hidden] */
    const float *w1, *b1;      /* device, [hidden][hidden], [hidden] */
    const float *w2, *b2;      /* device, [3][hidden], [3] */
} cic_mlp;

typedef struct {
    int32_t n_samples;         /* samples per ray, 1..1024 */
    float et_threshold;        /* early termination: stop once transmittance < this; 0 = off */
    int32_t use_occupancy;     /* skip voxels whose occupancy byte is 0 (needs grid.occupancy) */
    float bg[3];               /* background colour added with weight T_stop */
    float void_acc;            /* frames: z-depth is +inf where opacity < void_acc */
    int32_t order;             /* CIC_ORDER_RAY or CIC_ORDER_VOXEL */
    float warp_max_angle;      /* SpaRW: degrees; a target pixel is warped only if the rays from the two
                                  cameras to its visible reference point subtend less than this, else
                                  rendered (Sec. III-C); 0 = off */
} cic_opts;

typedef struct {
    int32_t width, height;     /* pixels, each in [1, 16384] */
    float f, cx, cy;           /* focal length and principal point in pixels */
    float c2w[12];             /* row-major 3x4 [R | eye] */
} cic_camera;

/* Bytes of workspace needed by operation `op` for `n_items` rays (render_rays,
 * render_backward) or pixels (the frame operations).  Returns 0 on invalid
 * arguments.  render_rays, render_frame and render_backward also accept a
 * smaller workspace, down to cic_workspace_bytes(op, 1, ...): they then run
 * the rays in more passes of fewer rays each (per pass about 22 B (ray
 * order) or 32 B (voxel order) per sample slot, n_samples slots per ray, and
 * a few hundred bytes per ray), with the same results for render_rays and
 * render_frame; render_backward adds each pass's weight gradients in turn,
 * so their float32 sums depend on the pass size. */
size_t cic_workspace_bytes(int op, int64_t n_items, const cic_grid *grid, const cic_opts *opts);

/* Description of the calling thread's last error ("" if none). */
const char *cic_last_error_message(void);

/* Occupancy for empty-space skipping (the paper's Indexing stage finds the
 * voxel of each sample, Sec. II-B; skipping empty voxels is the usual
 * companion of dense-grid models).  occ[v] = 1 iff any of the voxel's eight
 * vertices has softplus(raw + density_shift) > occ_sigma, evaluated as
 * (raw + density_shift) > log(expm1(occ_sigma)) in float32 (the threshold
 * is computed in float64 on the host and rounded once).  float16 grids are
 * widened to float32 first.  occ: device, (res0-1)(res1-1)(res2-1) bytes. */
int build_occupancy(const cic_grid *grid, float occ_sigma, uint8_t *occ, cic_stream_t stream);

/* One ray per pixel (Sec. II-B Indexing): origin = camera centre,
 * direction = normalize(R * ((i+1/2-cx)/f, (j+1/2-cy)/f, 1)), in float32.
 * pix: device int64 pixel indices [n], or NULL for all width*height pixels
 * (then n must equal width*height).  rays_o, rays_d: device [n][3]. */
int generate_rays(const cic_camera *cam, int64_t n, const int64_t *pix,
                  float *rays_o, float *rays_d, cic_stream_t stream);

/* Render a batch of rays: Indexing, Feature Gathering and Feature
 * Computation of Sec. II-B, accumulated along each ray with the standard
 * volume-rendering quadrature (Fig. 1 caption).  Per ray: slab interval
 * [t_near, t_far] with the box, N samples at t_k = t_near + (k+1/2) delta,
 * delta = (t_far - t_near)/N; sigma_k = softplus(trilerp(density) + shift);
 * T_0 = 1, T_{k+1} = T_k exp(-sigma_k delta); w_k = T_k (1 - exp(-sigma_k delta));
 * c_k = MLP(trilerp(features), direction); rgb = sum w_k c_k + T_stop bg;
 * depth_t = sum w_k t_k; acc = 1 - T_stop.  With early termination the
 * first sample with T_k < et_threshold and all later ones are dropped and
 * T_stop is that T_k.  Skipped (unoccupied) voxels contribute sigma = 0.
 * Missed rays give rgb = bg, depth_t = 0, acc = 0.
 * opts->order = CIC_ORDER_VOXEL evaluates the MLP stage in voxel-bucket
 * order (the memory-centric ordering of Sec. IV-A; with BF16 compute on a
 * dense grid each brick's features are staged once in on-chip memory).
 * Results equal ray order's bit for bit (each sample's colour depends only
 * on its own inputs, and the compositing reads samples in ray order).
 * rgb [n][3], depth_t [n], acc [n]: device float32.  n_eval (device int64,
 * nullable) is increased by the number of samples that went through the MLP. */
int render_rays(const cic_grid *grid, const cic_mlp *mlp, const cic_opts *opts, int64_t n_rays,
                const float *rays_o, const float *rays_d,
                float *rgb, float *depth_t, float *acc, int64_t *n_eval,
                void *ws, size_t ws_bytes, cic_stream_t stream);

/* Render every pixel of a frame: generate_rays + render_rays, then the
 * frame's z-depth depth_z = (depth_t/acc) * dot(d, camera forward) where
 * acc >= void_acc, else +inf (the depth buffer SpaRW needs, Sec. III-B).
 * rgb [H*W][3], depth_z [H*W], acc [H*W] (acc nullable). */
int render_frame(const cic_grid *grid, const cic_mlp *mlp, const cic_opts *opts, const cic_camera *cam,
                 float *rgb, float *depth_z, float *acc, int64_t *n_eval,
                 void *ws, size_t ws_bytes, cic_stream_t stream);

/* SpaRW steps 1-3 (Sec. III-B, Eq. 1-3) in float32 without FMA contraction:
 * each reference pixel with finite depth D becomes
 * P = D ((i+1/2-cx)/f, (j+1/2-cy)/f, 1) (Eq. 1), P' = R P + t with
 * ref_T_tgt = [R | t] (row-major 3x4, reference camera -> target camera,
 * Eq. 2), and lands on target pixel (floor(u), floor(v)) with
 * u = f_t X'/Z' + cx_t, v = f_t Y'/Z' + cy_t (Eq. 3) if Z' > 0 and inside the
 * image.  A reference pixel with depth +inf is a direction: it is rotated
 * only and carries depth +inf.  Each target pixel keeps the smallest depth,
 * ties to the smallest reference pixel index (64-bit packed-key atomic min).
 * max_angle_deg > 0 adds the "when to warp" test of Sec. III-C to the
 * visible (z-buffer winning) point of each target pixel: a finite point whose
 * rays from the two camera centres subtend max_angle_deg or more
 * (cos <= cos(max_angle), float32; the reference centre in target coordinates
 * is the translation of ref_T_tgt) leaves the pixel a hole, to be rendered;
 * points at infinity always pass.
 * Outputs (target size): tgt_rgb [H][W][3], tgt_depth_z [H][W] (+inf for
 * directions, 0 at holes), mask [H][W] u8 (1 = hole to re-render: nothing
 * landed, or the visible point failed the angle test), src_index [H][W]
 * int32 (nullable; reference pixel or -1).  Reference rgb/depth:
 * [Hr][Wr][3], [Hr][Wr]. */
int warp_frame(const cic_camera *ref, const cic_camera *tgt, const float ref_T_tgt[12],
               const float *ref_rgb, const float *ref_depth_z, float max_angle_deg,
               float *tgt_rgb, float *tgt_depth_z, uint8_t *mask, int32_t *src_index,
               void *ws, size_t ws_bytes, cic_stream_t stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid allocation): the same
 * warp as warp_frame, with the same arguments and results (bit for bit),
 * but without a workspace.  Its z-buffer is a device array inside the
 * library, one per GPU, of 2^21 64-bit entries (16 MiB, held until the
 * process ends), so the target frame has at most 2,097,152 pixels; larger
 * targets return CIC_ERR_INVALID before anything is launched.  The call
 * allocates nothing (no hipMalloc, no library allocation); its first call
 * on a device looks up that device's array.  Every call on one GPU uses the
 * same array: calls that overlap on one GPU (different streams, or several
 * host threads) race and give undefined results; calls ordered on one
 * stream are safe, each fills the z-buffer before using it. */
int warp_frame_noalloc(const cic_camera *ref, const cic_camera *tgt, const float ref_T_tgt[12],
                       const float *ref_rgb, const float *ref_depth_z, float max_angle_deg,
                       float *tgt_rgb, float *tgt_depth_z, uint8_t *mask, int32_t *src_index,
                       cic_stream_t stream);

/* SpaRW for one target frame (Sec. III-B, Eq. 4): warp_frame, then render the
 * pixels of the mask (void pixels, those reached only by directions, are not
 * re-rendered) with render_rays and put them in place of the warped values.
 * out_rgb [H][W][3], out_depth_z [H][W], mask [H][W]; n_masked (device
 * int64, nullable) receives the number of re-rendered pixels; n_eval as in
 * render_rays.  Requires width*height <= 2^21 for the target. */
int render_frame_sparw(const cic_grid *grid, const cic_mlp *mlp, const cic_opts *opts,
                       const cic_camera *ref, const float *ref_rgb, const float *ref_depth_z,
                       const cic_camera *tgt, const float ref_T_tgt[12],
                       float *out_rgb, float *out_depth_z, uint8_t *mask,
                       int64_t *n_masked, int64_t *n_eval,
                       void *ws, size_t ws_bytes, cic_stream_t stream);

/* Eq. 5-6 (Sec. III-C, reference frame rendering): the pose of an
 * off-trajectory reference, extrapolated from the two newest camera poses.
 * Poses are camera-to-world, row-major 3x4 [R | c], host float32.  The
 * centre continues at the velocity (c_cur - c_prev) per frame interval for
 * `steps` intervals (t_r = steps * dt); the orientation continues at the
 * angular velocity that took R_prev to R_cur: the world-frame rotation
 * R_cur R_prev^T raised to the power `steps` in axis-angle form, applied to
 * R_cur.  float64 arithmetic, rounded once.  Host only, no device work.
 * Errors: NULL pointer or non-finite value -> CIC_ERR_INVALID. */
int cic_extrapolate_pose(const float c2w_prev[12], const float c2w_cur[12], float steps, float c2w_out[12]);

/* Eq. 2's rigid transform from reference-camera to target-camera
 * coordinates for camera-to-world poses: inverse(C2W_tgt) C2W_ref =
 * [R_t^T R_r | R_t^T (c_r - c_t)], float64, rounded once (host only). */
int cic_relative_pose(const float c2w_ref[12], const float c2w_tgt[12], float ref_T_tgt[12]);

/* render_sequence flags */
enum { CIC_SEQ_OVERLAP = 1, CIC_SEQ_TEMPORAL = 2 };

/* A camera trajectory rendered with SpaRW and off-trajectory references
 * (Sec. III-C, Eq. 5-6; Fig. 7 and 8 for the pipelines).
 * Schedule: frame 0 is rendered in full and is reference R_0.  Frames
 * 1..n_frames-1 form windows of `window` consecutive targets; window w
 * starts at frame s_w = 1 + w*window and every target in it is rendered by
 * render_frame_sparw from R_w.  R_{w+1} (w + 1 < number of windows) has the
 * pose cic_extrapolate_pose(cams[s_w - 1], cams[s_w], lead), i.e. it needs
 * only the poses known when window w starts; lead < 0 selects the paper's
 * t_r = window/2 frame intervals.  References use the intrinsics of
 * cams[s_w].
 * flags & CIC_SEQ_OVERLAP: references render on `ref_stream` (a second
 * stream the caller owns, default priority, not `stream`) concurrently with
 * the previous window's targets on `stream` (Fig. 8); the reference work
 * stays ordered after everything issued to `stream` before the call, and
 * `stream` waits for all of it before any later work.  The events that
 * order the two streams are created by the call and destroyed before it
 * returns.  Without the flag everything runs on `stream`, R_{w+1} after
 * window w (Fig. 7a), and ref_stream is not used (may be NULL).  Both give
 * identical results.
 * target_cus_per_xcd > 0 (with CIC_SEQ_OVERLAP) states that the chip is
 * partitioned as the paper splits the work between two engines: `stream`
 * is restricted to that many CUs of each XCD and `ref_stream` to the rest,
 * as made by cic_stream_create_cu_masked with roles 0 and 1; the persistent
 * kernels are sized to each share.  Must be below the CUs per XCD (a
 * multiple of 4 splits every shader engine evenly); 0 means both streams
 * may use the whole chip.  Results are identical in every mode.
 * cams: host array of n_frames cameras, all of one size with width*height
 * <= 2^21.  Outputs (device, frame-major): rgb [n_frames][H*W][3],
 * depth_z [n_frames][H*W], mask [n_frames][H*W] (1 = pixel rendered; all of
 * frame 0), n_masked [n_frames] int64 (nullable; rendered pixels per frame),
 * n_eval as in render_rays.  ref_c2w (host, nullable) receives the poses of
 * R_1, R_2, ... ([n_windows - 1][12]).  Workspace:
 * cic_workspace_bytes(CIC_OP_RENDER_SEQUENCE, H*W, ...).  Calls that share
 * a device from several host threads at once are not supported.
 * flags = CIC_SEQ_TEMPORAL selects the Temp-N comparison variant of the
 * paper's evaluation instead (Sec. VI-B): frames 0, N, 2N, ... are rendered
 * in full and every other frame is warped from the previous output frame
 * (its colour and z-depth, with its own pose), holes rendered, so warping
 * errors carry from frame to frame; lead, target_cus_per_xcd and ref_c2w are
 * unused and OVERLAP may not be combined with it. */
int render_sequence(const cic_grid *grid, const cic_mlp *mlp, const cic_opts *opts,
                    const cic_camera *cams, int32_t n_frames, int32_t window, float lead, int32_t flags,
                    int32_t target_cus_per_xcd,
                    float *rgb, float *depth_z, uint8_t *mask, int64_t *n_masked,
                    float *ref_c2w, int64_t *n_eval,
                    void *ws, size_t ws_bytes, cic_stream_t stream, cic_stream_t ref_stream);

/* The two streams of render_sequence's CU-partitioned overlap (the paper's
 * split of reference and target rendering between two engines, Sec. III-C
 * and Fig. 8, on one GPU): a stream of the current device restricted to
 * target_cus_per_xcd CUs of each XCD (role 0, targets) or to the remaining
 * CUs (role 1, references), default priority.  The caller owns it and
 * releases it with cic_stream_destroy (which waits for its work to finish)
 * before the HIP runtime shuts down.  Errors: CIC_ERR_INVALID for a role
 * other than 0/1 or a count outside [1, CUs per XCD - 1], CIC_ERR_HIP if the
 * runtime refuses; *out is NULL on error. */
int cic_stream_create_cu_masked(int32_t target_cus_per_xcd, int32_t role, cic_stream_t *out);
int cic_stream_destroy(cic_stream_t stream);

/* DS-s comparison variant of the paper's evaluation (Sec. VI-B, DS-2):
 * render the frame at 1/factor resolution -- same pose, ceil(W/s) x ceil(H/s)
 * pixels, focal length f/s and principal point (cx/s, cy/s), in float32 --
 * then upsample the colour bilinearly to W x H (output pixel centre i + 1/2
 * at (i + 1/2)/s - 1/2 in low-resolution pixel index space, border clamped).
 * factor in [1, 16]; rgb [H*W][3] device float32; n_eval as in render_rays.
 * Workspace: cic_workspace_bytes(CIC_OP_RENDER_FRAME_DS, W*H, ...). */
int render_frame_ds(const cic_grid *grid, const cic_mlp *mlp, const cic_opts *opts, const cic_camera *cam,
                    int32_t factor, float *rgb, int64_t *n_eval, void *ws, size_t ws_bytes, cic_stream_t stream);

/* Adjoint of render_rays (the derivative of the same quadrature; the paper
 * itself is inference-only).  The forward is recomputed per ray, on chip,
 * inside the fused MLP adjoint kernel (no per-sample activations go to
 * memory); nothing from a previous forward call is needed.  Upstream gradients d_rgb [n][3],
 * d_depth_t [n] (nullable), d_acc [n] (nullable).  Accumulates (+=) into
 * d_density [res0][res1][res2], d_features [res0][res1][res2][12] and the
 * MLP gradients shaped like the weights (all float32, device).  float32
 * grids and CIC_F32 compute only.  The MLP gradients are the same bits on
 * every call; the grid gradients can differ in their last bits between
 * calls, because the samples of a brick are summed in the order the
 * bucketing's atomic cursors placed them. */
int render_backward(const cic_grid *grid, const cic_mlp *mlp, const cic_opts *opts, int64_t n_rays,
                    const float *rays_o, const float *rays_d,
                    const float *d_rgb, const float *d_depth_t, const float *d_acc,
                    float *d_density, float *d_features,
                    float *d_w0, float *d_b0, float *d_w1, float *d_b1, float *d_w2, float *d_b2,
                    void *ws, size_t ws_bytes, cic_stream_t stream);

/* Stage timing for benchmarks.  While enabled (per calling thread), every
 * kernel launch of the stages below is bracketed by HIP events recorded on
 * the launch stream.  cic_timing_read waits for the recorded events and
 * writes, per stage, the summed milliseconds and the number of launches
 * since the last enable; it fills at most n_stages entries of each array
 * (host pointers).  Every cic_timing_enable call destroys the events of the
 * calling thread, so after cic_timing_enable(0) the library holds no HIP
 * object for it; call that before the HIP runtime shuts down.  Stages: */
enum {
    CIC_STAGE_MARCH = 0,      /* ray march + transmittance scan */
    CIC_STAGE_COMPACT = 1,    /* count scan, compaction, voxel bucketing */
    CIC_STAGE_MLP = 2,        /* feature gather + MLP (forward) */
    CIC_STAGE_REDUCE = 3,     /* per-ray accumulation */
    CIC_STAGE_WARP = 4,       /* z-buffer splat + resolve */
    CIC_STAGE_RAYGEN = 5,     /* pixel rays */
    CIC_STAGE_BACKWARD = 6,   /* adjoint: compositing adjoint + grid-gradient tiles (feature and density) */
    CIC_STAGE_BWD_MLP = 7,    /* adjoint: recomputed forward + MLP backward + weight gradients (fused) */
    CIC_STAGE_BWD_WGRAD = 8,  /* no launches (the weight gradients are part of CIC_STAGE_BWD_MLP) */
    CIC_STAGE_EMBED = 9,      /* per-ray direction term of layer 0 */
    CIC_STAGE_COUNT = 10
};
int cic_timing_enable(int on);
int cic_timing_read(double *ms, int64_t *launches, int n_stages);

/* Frame clock of the last render_sequence call made while timing was on:
 * writes to ms (host, up to cap entries) the completion time of each frame,
 * in milliseconds after the call's first work began on its stream, and
 * returns the number of frames (or a negative error code). */
int cic_timing_frames(double *ms, int cap);

#ifdef __cplusplus
}
#endif

#endif /* CICERO_H */
