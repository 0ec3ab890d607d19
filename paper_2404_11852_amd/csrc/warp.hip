// Sparse radiance warping, steps 1-3 (Sec. III-B, Eq. 1-3), in float32 with
// the expression order fixed (no contraction), and the resolve step that
// finds the disoccluded pixels for step 4.
//
// Z-buffer: one 64-bit key per target pixel, (float bits of depth << 32) |
// reference pixel index, combined with 64-bit atomic min (in LDS per block of
// reference pixels, then once per touched target pixel in global memory).  For positive
// floats the bit pattern orders like the value, so the minimum key is the
// nearest splat and, among equal depths, the smallest reference index: the
// result is independent of execution order and needs no locks.
#include <climits>

#include "kernels.h"

namespace cic {

__device__ __forceinline__ uint32_t f32_bits(float v) { return __float_as_uint(v); }

// Reference -> target rigid transform, row-major 3x4.
struct WarpT {
    float m[12];
};

// Eq. 1-2 for reference pixel (i, j) at depth D: back-project, then move into
// target-camera coordinates.  A point at infinity moves by the rotation only
// and keeps depth +inf for the z-test.
__device__ __forceinline__ void warp_point(const cic_camera &ref, const WarpT &T, int i, int j, float D, float &Xt,
                                           float &Yt, float &Zt, float &kz)
{
    const float a = (((float)i + 0.5f) - ref.cx) / ref.f;
    const float b = (((float)j + 0.5f) - ref.cy) / ref.f;
    if (D == INFINITY) {
        Xt = (T.m[0] * a + T.m[1] * b) + T.m[2];
        Yt = (T.m[4] * a + T.m[5] * b) + T.m[6];
        Zt = (T.m[8] * a + T.m[9] * b) + T.m[10];
        kz = INFINITY;
    } else {
        const float X = D * a, Y = D * b, Z = D;
        Xt = ((T.m[0] * X + T.m[1] * Y) + T.m[2] * Z) + T.m[3];
        Yt = ((T.m[4] * X + T.m[5] * Y) + T.m[6] * Z) + T.m[7];
        Zt = ((T.m[8] * X + T.m[9] * Y) + T.m[10] * Z) + T.m[11];
        kz = Zt;
    }
}

// Angle test of Sec. III-C in target-camera coordinates (target centre at
// the origin, reference centre at the translation of T): cos of the angle the
// two rays subtend at the point must exceed cmin.
__device__ __forceinline__ bool angle_ok(float Xt, float Yt, float Zt, const WarpT &T, float cmin)
{
    const float rx = Xt - T.m[3], ry = Yt - T.m[7], rz = Zt - T.m[11];
    const float dot = (Xt * rx + Yt * ry) + Zt * rz;
    const float n1 = sqrtf((Xt * Xt + Yt * Yt) + Zt * Zt);
    const float n2 = sqrtf((rx * rx + ry * ry) + rz * rz);
    return dot / (n1 * n2) > cmin;
}

// Splat: one workgroup per 16x16 block of reference pixels.  With small
// camera motion a block's splats land in a small target window, so the
// workgroup first combines them in an LDS tile (64-bit LDS atomic min, the
// same packed key) and then issues one global atomic min per touched target
// pixel; when the window exceeds the tile it falls back to one global atomic
// per splat.  The minimum does not depend on the order, so both give the same
// z-buffer.
constexpr int kSplatBlock = 16;
constexpr int kSplatTile = 4096;   // target pixels in the LDS window (32 KB of keys)

__global__ __launch_bounds__(256) void k_warp_splat(cic_camera ref, cic_camera tgt, WarpT T, const float *ref_depth,
                                                    unsigned long long *zbuf)
{
    __shared__ unsigned long long tile[kSplatTile];
    __shared__ int box[4];   // min x, min y, max x, max y of this block's target pixels
    const int i = blockIdx.x * kSplatBlock + (int)(threadIdx.x % kSplatBlock);
    const int j = blockIdx.y * kSplatBlock + (int)(threadIdx.x / kSplatBlock);
    if (threadIdx.x == 0) {
        box[0] = INT_MAX;
        box[1] = INT_MAX;
        box[2] = INT_MIN;
        box[3] = INT_MIN;
    }
    __syncthreads();
    bool hit = false;
    int px = 0, py = 0;
    unsigned long long key = ~0ull;
    if (i < ref.width && j < ref.height) {
        const int64_t src = (int64_t)j * ref.width + i;
        const float D = ref_depth[src];
        if (D == D) {
            float Xt, Yt, Zt, kz;
            warp_point(ref, T, i, j, D, Xt, Yt, Zt, kz);
            if (Zt > 0.0f) {
                const float u = tgt.f * (Xt / Zt) + tgt.cx;
                const float v = tgt.f * (Yt / Zt) + tgt.cy;
                if (u >= 0.0f && u < (float)tgt.width && v >= 0.0f && v < (float)tgt.height) {
                    hit = true;
                    px = (int)floorf(u);
                    py = (int)floorf(v);
                    key = ((unsigned long long)f32_bits(kz) << 32) | (unsigned long long)(uint32_t)src;
                }
            }
        }
    }
    // bounding box: wavefront reductions, then one LDS atomic per wavefront
    int bx0 = hit ? px : INT_MAX, by0 = hit ? py : INT_MAX, bx1 = hit ? px : INT_MIN, by1 = hit ? py : INT_MIN;
#pragma unroll
    for (int off = kWave / 2; off > 0; off >>= 1) {
        bx0 = min(bx0, __shfl_xor(bx0, off, kWave));
        by0 = min(by0, __shfl_xor(by0, off, kWave));
        bx1 = max(bx1, __shfl_xor(bx1, off, kWave));
        by1 = max(by1, __shfl_xor(by1, off, kWave));
    }
    if (lane_id() == 0 && bx0 != INT_MAX) {
        atomicMin(&box[0], bx0);
        atomicMin(&box[1], by0);
        atomicMax(&box[2], bx1);
        atomicMax(&box[3], by1);
    }
    __syncthreads();
    const int x0 = box[0], y0 = box[1];
    if (x0 == INT_MAX) return;   // nothing landed (uniform: every thread reads the same box)
    const int tw = box[2] - x0 + 1, th = box[3] - y0 + 1;
    if ((int64_t)tw * th > kSplatTile) {
        if (hit) atomicMin(&zbuf[(int64_t)py * tgt.width + px], key);
        return;
    }
    const int n = tw * th;
    for (int e = threadIdx.x; e < n; e += blockDim.x) tile[e] = ~0ull;
    __syncthreads();
    if (hit) atomicMin(&tile[(py - y0) * tw + (px - x0)], key);
    __syncthreads();
    for (int e = threadIdx.x; e < n; e += blockDim.x) {
        const unsigned long long k = tile[e];
        if (k != ~0ull) atomicMin(&zbuf[(int64_t)(y0 + e / tw) * tgt.width + (x0 + e % tw)], k);
    }
}

// Resolve: the z-buffer winner is the visible reference point.  With the
// angle test on (cmin >= -1) a finite winner that fails it makes the pixel a
// hole, as does an empty z-buffer entry.  A block resolves kResolvePasses x
// 256 consecutive target pixels, keeps each pass's hole flags, reserves the
// block's share of the hole list with one atomic and writes its holes in
// pixel order (an LDS prefix over the passes' wavefront counts), so the list
// takes one device-wide atomic per block instead of one per wavefront.
constexpr int kResolvePasses = 8;
constexpr int kResolveWaves = 4;   // 256 threads

__global__ __launch_bounds__(256) void k_warp_resolve(int64_t np, const unsigned long long *zbuf, cic_camera ref,
                                                      WarpT T, float cmin, const float *ref_depth,
                                                      const float *ref_rgb, float *tgt_rgb, float *tgt_depth,
                                                      uint8_t *mask, int32_t *src_index, int32_t *hole_idx,
                                                      uint32_t *n_holes)
{
    __shared__ uint32_t wave_cnt[kResolvePasses * kResolveWaves];
    __shared__ uint32_t block_base;
    const int lane = lane_id(), wave = threadIdx.x / kWave;
    const int64_t p0 = (int64_t)blockIdx.x * kResolvePasses * 256;
    uint32_t holes = 0;   // bit i: the pixel of pass i is a hole
#pragma unroll
    for (int it = 0; it < kResolvePasses; ++it) {
        const int64_t p = p0 + it * 256 + threadIdx.x;
        const bool in = p < np;
        const unsigned long long key = in ? zbuf[p] : ~0ull;
        const uint32_t s = (uint32_t)(key & 0xffffffffull);
        bool hole = in && key == ~0ull;
        if (in && !hole && cmin >= -1.0f) {
            const float D = ref_depth[s];
            if (D != INFINITY) {
                float Xt, Yt, Zt, kz;
                warp_point(ref, T, (int)(s % (uint32_t)ref.width), (int)(s / (uint32_t)ref.width), D, Xt, Yt, Zt,
                           kz);
                hole = !angle_ok(Xt, Yt, Zt, T, cmin);
            }
        }
        if (in) {
            if (hole) {
                tgt_rgb[3 * p] = tgt_rgb[3 * p + 1] = tgt_rgb[3 * p + 2] = 0.f;
                tgt_depth[p] = 0.f;
                mask[p] = 1;
                if (src_index) src_index[p] = -1;
            } else {
                tgt_rgb[3 * p] = ref_rgb[3 * (int64_t)s];
                tgt_rgb[3 * p + 1] = ref_rgb[3 * (int64_t)s + 1];
                tgt_rgb[3 * p + 2] = ref_rgb[3 * (int64_t)s + 2];
                tgt_depth[p] = __uint_as_float((uint32_t)(key >> 32));
                mask[p] = 0;
                if (src_index) src_index[p] = (int32_t)s;
            }
        }
        const uint64_t hm = __ballot(hole);
        if (lane == 0) wave_cnt[it * kResolveWaves + wave] = (uint32_t)__popcll(hm);
        holes |= hole ? (1u << it) : 0u;
    }
    if (!hole_idx) return;   // uniform over the grid
    __syncthreads();
    if (threadIdx.x == 0) {
        // exclusive prefix over (pass, wave) in pixel order, then the block's reservation
        uint32_t run = 0;
        for (int i = 0; i < kResolvePasses * kResolveWaves; ++i) {
            const uint32_t c = wave_cnt[i];
            wave_cnt[i] = run;
            run += c;
        }
        block_base = run ? atomicAdd(n_holes, run) : 0u;
    }
    __syncthreads();
    const uint32_t base = block_base;
#pragma unroll
    for (int it = 0; it < kResolvePasses; ++it) {
        const bool hole = (holes >> it) & 1u;
        const uint64_t hm = __ballot(hole);
        if (hole) {
            const int64_t p = p0 + it * 256 + threadIdx.x;
            hole_idx[base + wave_cnt[it * kResolveWaves + wave] + (uint32_t)__popcll(hm & lanes_below_mask())] =
                (int32_t)p;
        }
    }
}

void launch_warp(const cic_camera &ref, const cic_camera &tgt, const float T[12], float cmin, const float *ref_rgb,
                 const float *ref_depth, uint64_t *zbuf, float *tgt_rgb, float *tgt_depth, uint8_t *mask,
                 int32_t *src_index, int32_t *hole_idx, uint32_t *n_holes, hipStream_t s)
{
    const int64_t nt = (int64_t)tgt.width * tgt.height;
    const int64_t nr = (int64_t)ref.width * ref.height;
    WarpT wt;
    for (int k = 0; k < 12; ++k) wt.m[k] = T[k];
    launch_fill_u64(zbuf, ~0ull, nt, s);
    if (n_holes) launch_fill_u32(n_holes, 0u, 1, s);
    (void)nr;
    const dim3 grid((unsigned)((ref.width + kSplatBlock - 1) / kSplatBlock),
                    (unsigned)((ref.height + kSplatBlock - 1) / kSplatBlock));
    hipLaunchKernelGGL(k_warp_splat, grid, dim3(kSplatBlock * kSplatBlock), 0, s, ref, tgt, wt, ref_depth,
                       (unsigned long long *)zbuf);
    const int64_t per_block = (int64_t)kResolvePasses * 256;
    hipLaunchKernelGGL(k_warp_resolve, dim3((unsigned)((nt + per_block - 1) / per_block)), dim3(256), 0, s, nt,
                       (const unsigned long long *)zbuf, ref, wt, cmin, ref_depth, ref_rgb, tgt_rgb, tgt_depth, mask,
                       src_index, hole_idx, n_holes);
}

__global__ void k_sparw_finish(const uint32_t *n_holes, int64_t *n_masked)
{
    if (threadIdx.x == 0 && blockIdx.x == 0) *n_masked = (int64_t)*n_holes;
}

void launch_sparw_finish(const uint32_t *n_holes, int64_t *n_masked, hipStream_t s)
{
    hipLaunchKernelGGL(k_sparw_finish, dim3(1), dim3(64), 0, s, n_holes, n_masked);
}

}  // namespace cic
