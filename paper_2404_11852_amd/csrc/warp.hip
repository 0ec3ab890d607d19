// Sparse radiance warping, steps 1-3 (Sec. III-B, Eq. 1-3), in float32 with
// the expression order fixed (no contraction), and the resolve step that
// finds the disoccluded pixels for step 4.
//
// Z-buffer: one 64-bit key per target pixel, (float bits of depth << 32) |
// reference pixel index, combined with a 64-bit atomic min.  For positive
// floats the bit pattern orders like the value, so the minimum key is the
// nearest splat and, among equal depths, the smallest reference index: the
// result is independent of execution order and needs no locks.
#include "kernels.h"

namespace cic {

__device__ __forceinline__ uint32_t f32_bits(float v) { return __float_as_uint(v); }

__global__ __launch_bounds__(256) void k_warp_splat(cic_camera ref, cic_camera tgt, float T0, float T1, float T2,
                                                    float T3, float T4, float T5, float T6, float T7, float T8,
                                                    float T9, float T10, float T11, const float *ref_depth,
                                                    unsigned long long *zbuf)
{
    const int64_t src = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t n = (int64_t)ref.width * ref.height;
    if (src >= n) return;
    const float D = ref_depth[src];
    if (D != D) return;
    const int i = (int)(src % ref.width), j = (int)(src / ref.width);
    const float a = (((float)i + 0.5f) - ref.cx) / ref.f;
    const float b = (((float)j + 0.5f) - ref.cy) / ref.f;
    float Xt, Yt, Zt, kz;
    if (D == INFINITY) {
        Xt = (T0 * a + T1 * b) + T2;
        Yt = (T4 * a + T5 * b) + T6;
        Zt = (T8 * a + T9 * b) + T10;
        kz = INFINITY;
    } else {
        const float X = D * a, Y = D * b, Z = D;
        Xt = ((T0 * X + T1 * Y) + T2 * Z) + T3;
        Yt = ((T4 * X + T5 * Y) + T6 * Z) + T7;
        Zt = ((T8 * X + T9 * Y) + T10 * Z) + T11;
        kz = Zt;
    }
    if (!(Zt > 0.0f)) return;
    const float u = tgt.f * (Xt / Zt) + tgt.cx;
    const float v = tgt.f * (Yt / Zt) + tgt.cy;
    if (!(u >= 0.0f && u < (float)tgt.width && v >= 0.0f && v < (float)tgt.height)) return;
    const int64_t p = (int64_t)floorf(v) * tgt.width + (int64_t)floorf(u);
    const unsigned long long key = ((unsigned long long)f32_bits(kz) << 32) | (unsigned long long)(uint32_t)src;
    atomicMin(&zbuf[p], key);
}

// Resolve: copy the winning reference pixel, or mark a hole and append it to
// the hole list (one atomic per wavefront).
__global__ __launch_bounds__(256) void k_warp_resolve(int64_t np, const unsigned long long *zbuf, const float *ref_rgb,
                                                      float *tgt_rgb, float *tgt_depth, uint8_t *mask,
                                                      int32_t *src_index, int32_t *hole_idx, uint32_t *n_holes)
{
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const bool in = p < np;
    const unsigned long long key = in ? zbuf[p] : 0ull;
    const bool hole = in && key == ~0ull;
    if (in) {
        if (hole) {
            tgt_rgb[3 * p] = tgt_rgb[3 * p + 1] = tgt_rgb[3 * p + 2] = 0.f;
            tgt_depth[p] = 0.f;
            mask[p] = 1;
            if (src_index) src_index[p] = -1;
        } else {
            const uint32_t s = (uint32_t)(key & 0xffffffffull);
            tgt_rgb[3 * p] = ref_rgb[3 * (int64_t)s];
            tgt_rgb[3 * p + 1] = ref_rgb[3 * (int64_t)s + 1];
            tgt_rgb[3 * p + 2] = ref_rgb[3 * (int64_t)s + 2];
            tgt_depth[p] = __uint_as_float((uint32_t)(key >> 32));
            mask[p] = 0;
            if (src_index) src_index[p] = (int32_t)s;
        }
    }
    if (hole_idx) {
        const uint64_t hm = __ballot(hole);
        if (hm) {
            uint32_t base = 0;
            const int leader = __ffsll((unsigned long long)hm) - 1;
            if (lane_id() == leader) base = atomicAdd(n_holes, (uint32_t)__popcll(hm));
            base = __shfl(base, leader, kWave);
            if (hole) hole_idx[base + (uint32_t)__popcll(hm & lanes_below_mask())] = (int32_t)p;
        }
    }
}

void launch_warp(const cic_camera &ref, const cic_camera &tgt, const float T[12], const float *ref_rgb,
                 const float *ref_depth, uint64_t *zbuf, float *tgt_rgb, float *tgt_depth, uint8_t *mask,
                 int32_t *src_index, int32_t *hole_idx, uint32_t *n_holes, hipStream_t s)
{
    const int64_t nt = (int64_t)tgt.width * tgt.height;
    const int64_t nr = (int64_t)ref.width * ref.height;
    launch_fill_u64(zbuf, ~0ull, nt, s);
    if (n_holes) launch_fill_u32(n_holes, 0u, 1, s);
    hipLaunchKernelGGL(k_warp_splat, dim3((unsigned)((nr + 255) / 256)), dim3(256), 0, s, ref, tgt, T[0], T[1], T[2],
                       T[3], T[4], T[5], T[6], T[7], T[8], T[9], T[10], T[11], ref_depth,
                       (unsigned long long *)zbuf);
    hipLaunchKernelGGL(k_warp_resolve, dim3((unsigned)((nt + 255) / 256)), dim3(256), 0, s, nt,
                       (const unsigned long long *)zbuf, ref_rgb, tgt_rgb, tgt_depth, mask, src_index, hole_idx,
                       n_holes);
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
