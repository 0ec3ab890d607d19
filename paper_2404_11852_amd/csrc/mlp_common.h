// Device helpers shared by the FP32 and BF16 MLP kernels: the per-sample
// inputs of layer 0 (trilinear feature gather or multi-level encoding, and
// the view-direction encoding) and the persistent grids' size.
#pragma once
#include "kernels.h"

namespace cic {

typedef float f4_t __attribute__((ext_vector_type(4)));
typedef float f2_t __attribute__((ext_vector_type(2)));

// Input index (0..38, or -1 for padding) of chunk c for lane group q.
__host__ __device__ __forceinline__ int l0_input(int c, int q)
{
    if (c < 3) return 3 * q + c;
    if (c == 3) return q < 3 ? 12 + q : -1;
    const int jj = (c - 4) >> 1, p = 3 * q + jj;
    return ((c - 4) & 1) ? 27 + p : 15 + p;
}

__device__ __forceinline__ float pick3(int i, float a, float b, float c) { return i == 0 ? a : (i == 1 ? b : c); }

// float32 weights in LDS (in floats), pre-permuted into per-lane MFMA
// fragment order: W0 [t 8][c2 5][lane 64][2] (lane l of output tile t holds
// row 16t + l%16 at the inputs of chunks 2*c2, 2*c2+1 of lane group l/16),
// W1 [t 8][c4 8][lane 64][4] (row 16t + l%16, columns 16*c4 + 4*(l/16) + r),
// W2 [q 4][ch 3][t 8][r 4] (column 16t + 4q + r of output row ch), biases.
// PAD inserts 4 floats after every 16 lanes of a W1 block: the fragment reads
// stay conflict-free, and a read of W1 transposed (lane l taking row
// 16 c4 + 4 (l/16) + rr, column 16 ti + l%16) puts the 64 lanes on 64
// distinct banks instead of 16.
template <bool PAD>
struct F32Lds {
    static constexpr int kW1Block = PAD ? 272 : 256;
    static constexpr int kW0 = 0;
    static constexpr int kW1 = kW0 + 8 * 5 * 64 * 2;
    static constexpr int kW2 = kW1 + 64 * kW1Block;
    static constexpr int kB0 = kW2 + 4 * 3 * 8 * 4;
    static constexpr int kB1 = kB0 + 128;
    static constexpr int kB2 = kB1 + 128;
    static constexpr int kSize = kB2 + 4;
    // first float of lane `lane` of W1 block (t * 8 + c4)
    __host__ __device__ static constexpr int w1(int blk, int lane)
    {
        return kW1 + blk * kW1Block + 4 * (PAD ? lane + (lane >> 4) : lane);
    }
};
constexpr int kOffW0 = F32Lds<false>::kW0;
constexpr int kOffW1 = F32Lds<false>::kW1;
constexpr int kOffW2 = F32Lds<false>::kW2;
constexpr int kOffB0 = F32Lds<false>::kB0;
constexpr int kOffB1 = F32Lds<false>::kB1;
constexpr int kOffB2 = F32Lds<false>::kB2;
constexpr int kLdsF32 = F32Lds<false>::kSize;

template <bool PAD = false>
__device__ __forceinline__ void stage_weights_f32(const cic_mlp &m, float *lds)
{
    typedef F32Lds<PAD> L;
    const int nt = blockDim.x;
    for (int i = threadIdx.x; i < 8 * 10 * 64; i += nt) {
        const int l = i & 63, c = (i >> 6) % 10, t = i / 640;
        const int row = 16 * t + (l & 15), src = l0_input(c, l >> 4);
        lds[L::kW0 + ((t * 5 + (c >> 1)) * 64 + l) * 2 + (c & 1)] = src >= 0 ? m.w0[row * 39 + src] : 0.f;
    }
    for (int i = threadIdx.x; i < 8 * 32 * 64; i += nt) {
        const int l = i & 63, c = (i >> 6) & 31, t = i >> 11;
        const int row = 16 * t + (l & 15), col = 16 * (c >> 2) + 4 * (l >> 4) + (c & 3);
        lds[L::w1(t * 8 + (c >> 2), l) + (c & 3)] = m.w1[row * 128 + col];
    }
    for (int i = threadIdx.x; i < 384; i += nt) {
        const int q = i / 96, ch = (i / 32) % 3, t = (i / 4) % 8, r = i & 3;
        lds[L::kW2 + i] = m.w2[ch * 128 + 16 * t + 4 * q + r];
    }
    for (int i = threadIdx.x; i < 128; i += nt) {
        lds[L::kB0 + i] = m.b0[i];
        lds[L::kB1 + i] = m.b1[i];
    }
    if (threadIdx.x < 3) lds[L::kB2 + threadIdx.x] = m.b2[threadIdx.x];
}

// View-encoding inputs of lane group q (layer-0 chunks 3-9): direction
// component q (q = 3 pads with 0), then sin and cos of encoding pairs
// p = 3q..3q+2, p = 4*component + octave.
__device__ __forceinline__ void encode_group(const float d[3], int q, float x[7])
{
    x[0] = q < 3 ? pick3(q, d[0], d[1], d[2]) : 0.f;
#pragma unroll
    for (int jj = 0; jj < 3; ++jj) {
        const int p = 3 * q + jj;
        const float a = ldexpf(pick3(p >> 2, d[0], d[1], d[2]), p & 3);
        float sn, cs;
        sincosf(a, &sn, &cs);
        x[1 + 2 * jj] = sn;
        x[2 + 2 * jj] = cs;
    }
}

// The ray data a sample's gather needs: its ray, sample index, interval
// start and step, origin and direction.
struct SampleRay {
    uint32_t ray;
    int k;
    float tn, delta;
    float o[3], d[3];
};

__device__ __forceinline__ void load_sample_ray(const RenderBufs &b, uint32_t ray, int k, SampleRay &r)
{
    r.ray = ray;
    r.k = k;
    const RayInfo inf = b.info[ray];
    r.tn = inf.tn;
    r.delta = inf.delta;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        r.o[a] = b.rays_o[3 * (int64_t)ray + a];
        r.d[a] = b.rays_d[3 * (int64_t)ray + a];
    }
}

// Sample position o + t_k d in float32 (the march's sample point).
__device__ __forceinline__ void sample_position(const SampleRay &r, float xp[3])
{
    const float tk = sample_t(r.tn, r.delta, r.k);
#pragma unroll
    for (int a = 0; a < 3; ++a) xp[a] = r.o[a] + tk * r.d[a];
}

// Layer-0 inputs of one sample for this lane's group q (PE = false: only
// the three feature channels; the direction terms come from a per-ray
// table).
template <typename T, bool PE = true>
__device__ __forceinline__ void sample_inputs_from(const GridK &g, const SampleRay &r, int q, float x[10])
{
    if (g.hlevels) {
        // multi-level encoding: lane group q gathers level q
        float xp[3];
        sample_position(r, xp);
        hash_level3<T>(g, q, xp, x);
    } else {
        int i0[3];
        float fr[3], tk;
        sample_voxel(r.o, r.d, r.tn, r.delta, r.k, g, i0, fr, tk);
        const T *feat = (const T *)g.features;
        if constexpr (sizeof(T) == 2) {
            trilerp3(feat, g, i0, fr, q, x);   // float16: one 64-bit load per vertex
        } else {
#pragma unroll
            for (int c = 0; c < 3; ++c) x[c] = trilerp1(feat, g, i0, fr, 12, 3 * q + c);
        }
    }
    if (!PE) {
#pragma unroll
        for (int c = 3; c < 10; ++c) x[c] = 0.f;
        return;
    }
    encode_group(r.d, q, x + 3);
}

template <typename T, bool PE = true>
__device__ __forceinline__ void sample_inputs(const GridK &g, const RenderBufs &b, int64_t rec, int q, float x[10])
{
    SampleRay r;
    load_sample_ray(b, b.rec_ray[rec], b.rec_k[rec], r);
    sample_inputs_from<T, PE>(g, r, q, x);
}

// Output sigmoid from the hardware base-2 exponential and reciprocal:
// 1 / (1 + 2^(-x log2 e)), within about 1e-6 relative of the correctly
// rounded value for |x| < 20 (the rounding of x log2 e dominates), in 4
// instructions where the library's expf and IEEE division take about 25.
__device__ __forceinline__ float sigmoid_hw(float x)
{
    return __builtin_amdgcn_rcpf(1.0f + __builtin_amdgcn_exp2f(-1.44269504088896341f * x));
}

inline int num_cus(const RenderBufs &b)
{
    if (b.grid_cus > 0) return b.grid_cus;
    int dev = 0, n = 0;
    (void)hipGetDevice(&dev);
    (void)hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, dev);
    return n > 0 ? n : 256;
}

}  // namespace cic
