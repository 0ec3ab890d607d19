// Host-side launchers of the renderer's kernels (one translation unit per
// group of kernels; the C interface in api.hip strings them together).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "common.h"

namespace cic {

// Per-ray state written by the march: t_near, delta, T_stop, sum w_k t_k.
struct RayInfo {
    float tn, delta, t_stop, depth_t;
};

// Device buffers of one render pass (carved from the caller's workspace).
struct RenderBufs {
    int64_t n;             // rays in this pass (upper bound when n_active is set)
    int n_samples;
    const float *rays_o, *rays_d;
    const uint32_t *n_active;  // device count of active rays (nullable)
    RayInfo *info;
    uint32_t *count;       // [n] live samples per ray
    uint32_t *offsets;     // [n+1] exclusive scan of count
    uint32_t *scan_tmp;    // block sums
    uint16_t *slot_k;      // [n*N] live sample indices, per-ray fixed slots
    float *slot_w;         // [n*N] their weights
    uint32_t *rec_ray;     // [n*N] compacted: ray of each live sample
    uint16_t *rec_k;       // [n*N] its sample index
    float *rec_w;          // [n*N] its weight
    float *rec_c;          // [n*N*3] MLP colour per live sample
    float *slot_t;         // [n*N] transmittance T_k of live samples (adjoint only; nullable)
    float *rec_t;          // [n*N] compacted T_k (adjoint only; nullable)
    float *z0;             // [n][128] per-ray direction term of layer 0 (FP32 compute)
    uint32_t *enc;         // [n][16] per-ray view encoding in BF16: lane group q's 7 inputs in words 4q..4q+3
    // voxel order
    uint32_t *rec_key;     // [n*N] brick of each live sample
    uint32_t *brick_off;   // [n_bricks+1] counts, then cursors
    uint32_t *brick_tmp;   // block sums for the brick scan
    uint32_t *perm;        // [n*N] sample order for the MLP stage
    uint32_t *seg_brick;   // voxel order (nullable): [max segments] brick of each segment of the LDS-tile kernels
    int64_t n_bricks;
    uint32_t *work_ctr;    // voxel order: per-XCD segment counters of the LDS-tile MLP kernels (kXcds words)
    uint32_t *seg_off;     // voxel order: [n_bricks+1] exclusive scan of segments per brick
    int grid_cus;          // CUs the launch stream may use, a multiple of 8 (0 = the whole device): sizes the
                           // persistent kernels' grids
};

// Per-sample row of MLP vectors the adjoint's weight gradients read from LDS:
// inputs with a constant 1 in the padding slot (so the bias gradients fall
// out of the same products), both hidden activations, the first hidden
// layer's pre-activation gradient, the output-logit gradient (16 wide, 3
// used) and the second hidden layer's pre-activation gradient.
constexpr int kStX = 0, kStH1 = 40, kStH2 = 168, kStDP0 = 296, kStDL = 424, kStDP1 = 440;

// scan.hip
size_t scan_tmp_elems(int64_t n);
void launch_exclusive_scan(const uint32_t *in, uint32_t *out, uint32_t *tmp, int64_t n, hipStream_t s);

// render.hip
template <typename T>
void launch_march(const GridK &g, const OptsK &o, const RenderBufs &b, hipStream_t s);
void launch_compact(const GridK &g, const RenderBufs &b, bool voxel_keys, hipStream_t s);
void launch_brick_scatter(const RenderBufs &b, hipStream_t s);
void launch_fill_u32(uint32_t *p, uint32_t v, int64_t n, hipStream_t s);
void launch_fill_u64(uint64_t *p, uint64_t v, int64_t n, hipStream_t s);
void launch_fill_u8(uint8_t *p, uint8_t v, int64_t n, hipStream_t s);

// segments of at most kTileSeg samples per brick for the LDS-tile MLP kernels,
// and of at most kFgSeg samples for the brick-tile gradient accumulation
constexpr int kTileSeg = 2048;
__host__ __device__ inline int64_t tile_max_segments(int64_t n_bricks, int64_t ns)
{
    return n_bricks + ns / kTileSeg + 1;
}
constexpr int kFgSeg = 512;
// seg_off[k] = first segment of brick k (exclusive scan of ceil(count / seg));
// seg_off[n_bricks] = the number of segments; with `table` (seg ==
// kTileSeg), also seg_brick, the brick of every segment
void launch_brick_segments(const RenderBufs &b, int seg, bool table, hipStream_t s);

// upsample.hip
void launch_upsample_bilinear(const float *lo, int w, int h, float *out, int W, int H, int s, hipStream_t st);
// Final per-ray accumulation.  out_map (nullable) maps ray -> output slot;
// frame_cam (nullable) switches depth output to frame z-depth.
void launch_reduce(const RenderBufs &b, const OptsK &o, float *rgb, float *depth, float *acc,
                   const int32_t *out_map, const cic_camera *frame_cam, int64_t *n_eval, hipStream_t s);
void launch_generate_rays(const cic_camera &cam, int64_t n, int64_t base, const int64_t *pix, const int32_t *pix32,
                          const uint32_t *n_active, float *o, float *d, hipStream_t s);
template <typename T>
void launch_build_occupancy(const GridK &g, float thr, uint8_t *occ, hipStream_t s);

// mlp.hip
int mlp_lds_bytes(int compute);
template <typename T>
void launch_mlp_forward(const GridK &g, const cic_mlp &m, const RenderBufs &b, bool voxel, hipStream_t s);
// mlp_bf16.hip: the BF16 forward (called by launch_mlp_forward for BF16 compute)
template <typename T>
void launch_mlp_forward_bf16(const GridK &g, const cic_mlp &m, const RenderBufs &b, bool voxel, hipStream_t s);
// per-ray BF16 view encoding into b.enc (BF16 compute; rays with live samples)
void launch_ray_encode_bf16(const RenderBufs &b, hipStream_t s);
// per-ray direction term of layer 0 into b.z0 (rays with live samples)
void launch_ray_embed(const cic_mlp &m, const RenderBufs &b, hipStream_t s);

// warp.hip
void launch_warp(const cic_camera &ref, const cic_camera &tgt, const float T[12], float cmin, const float *ref_rgb,
                 const float *ref_depth, uint64_t *zbuf, float *tgt_rgb, float *tgt_depth, uint8_t *mask,
                 int32_t *src_index, int32_t *hole_idx, uint32_t *n_holes, hipStream_t s);
void launch_sparw_finish(const uint32_t *n_holes, int64_t *n_masked, hipStream_t s);

// backward.hip
struct BackwardBufs {
    const float *d_rgb, *d_depth_t, *d_acc;
    float *d_density, *d_features;
    float *d_w0, *d_b0, *d_w1, *d_b1, *d_w2, *d_b2;
    float *partials;       // weight-gradient partial sums, one per adjoint workgroup (at most kWgBlocks)
    float *rec_df;         // [n*N][12] feature gradient per live sample (ray order)
    float *rec_draw;       // [n*N] raw-density gradient per live sample
    float *seg_tiles;      // [max segments][kFgTileFloats] each segment's accumulated gradient tile
};
// 9^3 vertices x (12 feature + 1 density) gradient channels per brick tile
constexpr int kFgTileFloats = (kBrick + 1) * (kBrick + 1) * (kBrick + 1) * 13;
constexpr int kWgBlocks = 1024;
// per-block partial products: dp0^T[x|1] (128x48), dp1^T h1 (128x128),
// dl^T h2 (16x128), dp1^T ones (128x16), dl^T ones (16x16)
constexpr int kPartialFloats = 128 * 48 + 128 * 128 + 16 * 128 + 128 * 16 + 16 * 16;
void launch_backward_composite(const GridK &g, const OptsK &o, const RenderBufs &b, const BackwardBufs &bb,
                               hipStream_t s);
// recomputed forward, MLP backward and weight gradients, fused (ray order);
// also writes the samples' colours rec_c, which the compositing adjoint reads
void launch_mlp_adjoint(const GridK &g, const cic_mlp &m, const RenderBufs &b, const BackwardBufs &bb, hipStream_t s);
// brick-tile accumulation of the feature and density gradients written by the
// MLP backward and the compositing adjoint, then their addition to the grids
void launch_feature_grads_bricks(const GridK &g, const RenderBufs &b, const BackwardBufs &bb, hipStream_t s);
// most segments of kFgSeg samples a pass of ns sample slots can have
inline int64_t fg_max_segments(int64_t n_bricks, int64_t ns) { return n_bricks + ns / kFgSeg + 1; }

}  // namespace cic
