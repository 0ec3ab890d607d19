// Device-side building blocks shared by the renderer's kernels (gfx950,
// wave64).  Whole library is compiled with -ffp-contract=off so that the
// float32 geometry below (ray/box interval, sample positions, voxel index,
// warp projection) rounds exactly as written; arithmetic that may fuse uses
// fmaf explicitly.
#pragma once

#include <hip/hip_runtime.h>
#include <hip/hip_fp16.h>
#include <stdint.h>

#include "cicero.h"

namespace cic {

constexpr int kWave = 64;
constexpr int kBrick = 8;            // voxels per brick edge (voxel-order bucketing)
constexpr int kMaxSamples = 1024;    // samples per ray
#ifndef CIC_CHUNK_LOG2
#define CIC_CHUNK_LOG2 21
#endif
constexpr int64_t kChunkRays = (int64_t)1 << CIC_CHUNK_LOG2;  // rays per pipeline pass

// Grid description as the kernels see it (filled on the host).
struct GridK {
    int r0, r1, r2;        // vertices per axis
    float lo[3], hi[3];
    float scale[3];        // (r-1)/(hi-lo) per axis, float32 as computed on the host
    float shift;           // density shift before softplus
    const void *density;
    const void *features;
    const uint8_t *occ;    // nullptr when skipping is off
    int nb1, nb2;          // bricks along axes 1 and 2
    // multi-level encoding (hlevels = 0: dense features)
    int hlevels;
    int hN[4];             // cells per axis of each level
    int hdense[4];         // level stored densely ((N+1)^3 fits the table)
    float hscale[4][3];    // N / (hi - lo) per axis, float32 as computed on the host
    uint32_t hmask;        // table entries per level - 1
    const void *htab;      // [4][hmask+1][3]
};

struct OptsK {
    int n_samples;
    float et_threshold;
    float bg[3];
    float void_acc;
};

// --------------------------------------------------------------------------
// storage loads
// --------------------------------------------------------------------------
template <typename T> __device__ __forceinline__ float ldv(const T *p, int64_t i);
template <> __device__ __forceinline__ float ldv<float>(const float *p, int64_t i) { return p[i]; }
template <> __device__ __forceinline__ float ldv<__half>(const __half *p, int64_t i) { return __half2float(p[i]); }

// max(v, 0) and the clamp to [0, 1] on the float's bit pattern: one integer
// instruction each, where fmaxf/fminf also canonicalise NaNs first.  Equal to
// fmaxf(v, 0) and fminf(fmaxf(v, 0), 1) for every non-NaN v (a non-negative
// float orders like its bits) up to the sign of a zero result.
__device__ __forceinline__ float relu_bits(float v) { return __int_as_float(max(__float_as_int(v), 0)); }
__device__ __forceinline__ float clamp01_bits(float v)
{
    return __int_as_float(min(max(__float_as_int(v), 0), 0x3f800000));
}

// --------------------------------------------------------------------------
// float32 geometry (decides integers; written in the same expression order
// as the reference description, no contraction)
// --------------------------------------------------------------------------

// Slab test against the box: 0 <= t_near < t_far on a hit.
__device__ __forceinline__ bool ray_box(const float o[3], const float d[3], const GridK &g, float &tn, float &tf)
{
    float a = -INFINITY, b = INFINITY;
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        float inv = 1.0f / d[k];
        float t0 = (g.lo[k] - o[k]) * inv;
        float t1 = (g.hi[k] - o[k]) * inv;
        a = fmaxf(a, fminf(t0, t1));
        b = fminf(b, fmaxf(t0, t1));
    }
    a = fmaxf(a, 0.0f);
    tn = a;
    tf = b;
    return a < b;
}

// Sample k of a ray: t_k = t_near + (k + 1/2) delta, x = o + t_k d.
__device__ __forceinline__ float sample_t(float tn, float delta, int k)
{
    return tn + ((float)k + 0.5f) * delta;
}

// World position -> lower vertex index of the voxel and fraction inside it.
__device__ __forceinline__ void locate(const float x[3], const GridK &g, int i0[3], float fr[3])
{
    const int rr[3] = {g.r0, g.r1, g.r2};
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        float u = (x[k] - g.lo[k]) * g.scale[k];
        int i = (int)floorf(u);
        i = i < 0 ? 0 : i;
        i = i > rr[k] - 2 ? rr[k] - 2 : i;
        float f = u - (float)i;
        fr[k] = clamp01_bits(f);
        i0[k] = i;
    }
}

__device__ __forceinline__ int64_t cell_index(const GridK &g, const int i0[3])
{
    return ((int64_t)i0[0] * (g.r1 - 1) + i0[1]) * (int64_t)(g.r2 - 1) + i0[2];
}

__device__ __forceinline__ int64_t vertex_index(const GridK &g, int x, int y, int z)
{
    return ((int64_t)x * g.r1 + y) * (int64_t)g.r2 + z;
}

__device__ __forceinline__ uint32_t brick_of(const GridK &g, const int i0[3])
{
    return ((uint32_t)(i0[0] / kBrick) * g.nb1 + (uint32_t)(i0[1] / kBrick)) * g.nb2 + (uint32_t)(i0[2] / kBrick);
}

// Recompute the voxel of sample k of a ray (bit-identical to the march).
__device__ __forceinline__ void sample_voxel(const float o[3], const float d[3], float tn, float delta, int k,
                                             const GridK &g, int i0[3], float fr[3], float &tk)
{
    tk = sample_t(tn, delta, k);
    float x[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) x[a] = o[a] + tk * d[a];
    locate(x, g, i0, fr);
}

// Pixel ray in float32 (centre of pixel (i, j), pinhole camera).
__device__ __forceinline__ void pixel_ray(const cic_camera &c, int i, int j, float o[3], float d[3])
{
    float a = (((float)i + 0.5f) - c.cx) / c.f;
    float b = (((float)j + 0.5f) - c.cy) / c.f;
    float dx = (c.c2w[0] * a + c.c2w[1] * b) + c.c2w[2];
    float dy = (c.c2w[4] * a + c.c2w[5] * b) + c.c2w[6];
    float dz = (c.c2w[8] * a + c.c2w[9] * b) + c.c2w[10];
    float n = sqrtf((dx * dx + dy * dy) + dz * dz);
    d[0] = dx / n;
    d[1] = dy / n;
    d[2] = dz / n;
    o[0] = c.c2w[3];
    o[1] = c.c2w[7];
    o[2] = c.c2w[11];
}

// --------------------------------------------------------------------------
// float32 arithmetic
// --------------------------------------------------------------------------
__device__ __forceinline__ float lerpf(float a, float b, float t) { return fmaf(t, b - a, a); }

// Trilinear interpolation of one scalar channel (stride = channels per vertex).
template <typename T>
__device__ __forceinline__ float trilerp1(const T *v, const GridK &g, const int i0[3], const float fr[3], int stride,
                                          int ch)
{
    const int64_t sx = (int64_t)g.r1 * g.r2 * stride, sy = (int64_t)g.r2 * stride, sz = stride;
    const int64_t b = vertex_index(g, i0[0], i0[1], i0[2]) * stride + ch;
    float v000 = ldv(v, b), v001 = ldv(v, b + sz), v010 = ldv(v, b + sy), v011 = ldv(v, b + sy + sz);
    float v100 = ldv(v, b + sx), v101 = ldv(v, b + sx + sz), v110 = ldv(v, b + sx + sy),
          v111 = ldv(v, b + sx + sy + sz);
    float c00 = lerpf(v000, v001, fr[2]), c01 = lerpf(v010, v011, fr[2]);
    float c10 = lerpf(v100, v101, fr[2]), c11 = lerpf(v110, v111, fr[2]);
    float c0 = lerpf(c00, c01, fr[1]), c1 = lerpf(c10, c11, fr[1]);
    return lerpf(c0, c1, fr[0]);
}

// Cell of level l holding position x: lower vertex index (clamped to the
// level's cells) and fraction inside it (float32 locate, as the dense grid's).
__device__ __forceinline__ void hash_cell(const GridK &g, int l, const float x[3], int i0[3], float fr[3])
{
    const int N = g.hN[l];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        const float u = (x[a] - g.lo[a]) * g.hscale[l][a];
        int i = (int)floorf(u);
        i = i < 0 ? 0 : i;
        i = i > N - 1 ? N - 1 : i;
        const float f = u - (float)i;
        fr[a] = clamp01_bits(f);
        i0[a] = i;
    }
}

// Table entry of vertex (vx, vy, vz) of level l: dense index on levels whose
// (N+1)^3 vertices fit the table, spatial hash (XOR of the coordinates times
// per-axis primes, modulo the table size) on the others.
__device__ __forceinline__ uint32_t hash_entry(const GridK &g, int l, uint32_t vx, uint32_t vy, uint32_t vz)
{
    const uint32_t n1 = (uint32_t)g.hN[l] + 1u;
    return g.hdense[l] ? (vx * n1 + vy) * n1 + vz : (vx ^ (vy * 2654435761u) ^ (vz * 805459861u)) & g.hmask;
}

// Trilinear interpolation of a cell's 8 corner values v[c][f] (corner c =
// x bit 2, y bit 1, z bit 0), z then y then x (the order of trilerp1).
__device__ __forceinline__ void lerp3_corners(const float v[8][3], const float fr[3], float out[3])
{
#pragma unroll
    for (int f = 0; f < 3; ++f) {
        const float c00 = lerpf(v[0][f], v[1][f], fr[2]), c01 = lerpf(v[2][f], v[3][f], fr[2]);
        const float c10 = lerpf(v[4][f], v[5][f], fr[2]), c11 = lerpf(v[6][f], v[7][f], fr[2]);
        out[f] = lerpf(lerpf(c00, c01, fr[1]), lerpf(c10, c11, fr[1]), fr[0]);
    }
}

// Values 3e .. 3e+2 of an array (the 3 features of entry e of a level's
// table, or features 3q .. 3q+2 of vertex v of the dense grid, e = 4v + q).
// float16: the 6 bytes lie in the two aligned 32-bit words from byte
// (6e & ~3), inside the array when it is 4-byte aligned and holds a multiple
// of 2 entries: one 64-bit load instead of three 16-bit ones.
template <typename T> __device__ __forceinline__ void load_entry3(const T *tab, uint64_t e, float out[3]);
template <> __device__ __forceinline__ void load_entry3<float>(const float *tab, uint64_t e, float out[3])
{
#pragma unroll
    for (int f = 0; f < 3; ++f) out[f] = tab[e * 3 + f];
}
template <> __device__ __forceinline__ void load_entry3<__half>(const __half *tab, uint64_t e, float out[3])
{
    const uint32_t *w = (const uint32_t *)((const char *)tab + ((e * 6) & ~(uint64_t)3));
    const uint32_t a = w[0], b = w[1], sh = ((uint32_t)e & 1u) * 16u;
    const uint32_t lo = __builtin_amdgcn_alignbit(b, a, sh), hi = b >> sh;
    out[0] = __half2float(__ushort_as_half((unsigned short)(lo & 0xffffu)));
    out[1] = __half2float(__ushort_as_half((unsigned short)(lo >> 16)));
    out[2] = __half2float(__ushort_as_half((unsigned short)(hi & 0xffffu)));
}

// The 8 corners' features of cell i0 of level l, from the table.
template <typename T>
__device__ __forceinline__ void hash_corners(const GridK &g, int l, const int i0[3], float v[8][3])
{
    const T *tab = (const T *)g.htab + (size_t)l * ((size_t)g.hmask + 1) * 3;
#pragma unroll
    for (int c = 0; c < 8; ++c) {
        const uint32_t e = hash_entry(g, l, (uint32_t)(i0[0] + ((c >> 2) & 1)), (uint32_t)(i0[1] + ((c >> 1) & 1)),
                                      (uint32_t)(i0[2] + (c & 1)));
        load_entry3(tab, e, v[c]);
    }
}

// Features 3q .. 3q+2 of the dense 12-channel feature grid at cell i0.
template <typename T>
__device__ __forceinline__ void trilerp3(const T *feat, const GridK &g, const int i0[3], const float fr[3], int q,
                                         float out[3])
{
    const int64_t sx = (int64_t)g.r1 * g.r2, sy = g.r2;
    const int64_t b = vertex_index(g, i0[0], i0[1], i0[2]);
    float v[8][3];
#pragma unroll
    for (int c = 0; c < 8; ++c) {
        const int64_t vtx = b + ((c >> 2) & 1) * sx + ((c >> 1) & 1) * sy + (c & 1);
        load_entry3(feat, (uint64_t)(4 * vtx + q), v[c]);
    }
    lerp3_corners(v, fr, out);
}

// One level of the multi-level encoding at position x: 3 features,
// trilinear over the level's cell.
template <typename T>
__device__ __forceinline__ void hash_level3(const GridK &g, int l, const float x[3], float out[3])
{
    int i0[3];
    float fr[3], v[8][3];
    hash_cell(g, l, x, i0, fr);
    hash_corners<T>(g, l, i0, v);
    lerp3_corners(v, fr, out);
}

__device__ __forceinline__ float sigmoidf(float x) { return 1.0f / (1.0f + expf(-x)); }

// --------------------------------------------------------------------------
// wavefront primitives
// --------------------------------------------------------------------------
__device__ __forceinline__ int lane_id() { return (int)(threadIdx.x & (kWave - 1)); }

// Inclusive prefix sum across the 64 lanes (Hillis-Steele).
__device__ __forceinline__ float wave_incl_scan(float v)
{
    const int l = lane_id();
#pragma unroll
    for (int off = 1; off < kWave; off <<= 1) {
        float u = __shfl_up(v, off, kWave);
        if (l >= off) v += u;
    }
    return v;
}

// Sum across the wave; every lane gets the identical value.
__device__ __forceinline__ float wave_sum(float v)
{
#pragma unroll
    for (int off = kWave / 2; off > 0; off >>= 1) v += __shfl_xor(v, off, kWave);
    return v;
}

__device__ __forceinline__ uint64_t lanes_below_mask() { return (1ull << lane_id()) - 1ull; }

// Batch range of this workgroup's XCD.  Workgroups are dispatched to the 8
// XCDs round-robin, so blocks x, x+8, x+16, ... share one L2; giving each
// XCD one contiguous eighth of the (ray-ordered) samples keeps the grid
// region those rays touch in that XCD's L2.  (Only performance depends on
// the dispatch order.)
constexpr int kXcds = 8;
struct BatchRange {
    int64_t first, end, stride;
};
__device__ __forceinline__ BatchRange xcd_batches(int64_t nbatch, int waves, int wave)
{
    const int xcd = blockIdx.x % kXcds, slot = blockIdx.x / kXcds, nslots = gridDim.x / kXcds;
    const int64_t per = (nbatch + kXcds - 1) / kXcds;
    const int64_t lo = xcd * per, hi = lo + per < nbatch ? lo + per : nbatch;
    return {lo + (int64_t)slot * waves + wave, hi, (int64_t)nslots * waves};
}


}  // namespace cic
