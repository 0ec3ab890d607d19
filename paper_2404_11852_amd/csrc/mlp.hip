// Feature Gathering + Feature Computation (Sec. II-B) for the compacted live
// samples: trilinear gather of the 12 feature channels, the view-direction
// encoding, and the 39 -> 128 -> 128 -> 3 MLP on MFMA.
//
// Layout.  The MLP runs transposed, H^T = W X^T, so that samples sit on the
// MFMA's N axis: with v_mfma_f32_16x16x4_f32 the result tile of one layer
// (lane l holds outputs 4*(l/16)+r of sample l%16) is directly the B operand
// of the next layer once the reduction index is permuted the same way in the
// weights.  Activations therefore never leave registers; weights are staged
// once per workgroup in LDS, pre-permuted into per-lane fragment order so
// every A-operand read is one contiguous, conflict-free ds_read_b64/b128.
// The 3-wide output layer runs on the vector ALUs with a cross-lane sum.
//
// Input permutation of layer 0 (10 chunks of 4 = 40 >= 39 inputs): lane
// group q of each sample computes features 3q..3q+2 (chunks 0-2), the
// direction component q (chunk 3; q = 3 pads with 0) and sin/cos of the
// encoding pairs p = 3q..3q+2 (chunks 4-9), p = 4*component + octave.
//
// The kernel is persistent: one 8-wavefront workgroup per CU (LDS holds the
// 88 KB of float32 weights) loops over 32-sample batches until the device-
// side sample count is exhausted.
#include "kernels.h"

namespace cic {

typedef float f4_t __attribute__((ext_vector_type(4)));
typedef float f2_t __attribute__((ext_vector_type(2)));

constexpr int kMlpWaves = 8;
constexpr int kNT = 2;   // 16-sample tiles per wavefront batch
constexpr int kBatch = 16 * kNT;

// float32 LDS layout (in floats)
constexpr int kOffW0 = 0;                          // [t 8][c2 5][lane 64][2]
constexpr int kOffW1 = kOffW0 + 8 * 5 * 64 * 2;    // [t 8][c4 8][lane 64][4]
constexpr int kOffW2 = kOffW1 + 8 * 8 * 64 * 4;    // [q 4][ch 3][t 8][r 4]
constexpr int kOffB0 = kOffW2 + 4 * 3 * 8 * 4;
constexpr int kOffB1 = kOffB0 + 128;
constexpr int kOffB2 = kOffB1 + 128;
constexpr int kLdsF32 = kOffB2 + 4;

int mlp_lds_bytes(int compute)
{
    (void)compute;
    return kLdsF32 * (int)sizeof(float);
}

// Input index (0..38, or -1 for padding) of chunk c for lane group q.
__host__ __device__ __forceinline__ int l0_input(int c, int q)
{
    if (c < 3) return 3 * q + c;
    if (c == 3) return q < 3 ? 12 + q : -1;
    const int jj = (c - 4) >> 1, p = 3 * q + jj;
    return ((c - 4) & 1) ? 27 + p : 15 + p;
}

__device__ void stage_weights_f32(const cic_mlp &m, float *lds)
{
    const int nt = blockDim.x;
    for (int i = threadIdx.x; i < 8 * 10 * 64; i += nt) {
        const int l = i & 63, c = (i >> 6) % 10, t = i / 640;
        const int row = 16 * t + (l & 15), src = l0_input(c, l >> 4);
        lds[kOffW0 + ((t * 5 + (c >> 1)) * 64 + l) * 2 + (c & 1)] = src >= 0 ? m.w0[row * 39 + src] : 0.f;
    }
    for (int i = threadIdx.x; i < 8 * 32 * 64; i += nt) {
        const int l = i & 63, c = (i >> 6) & 31, t = i >> 11;
        const int row = 16 * t + (l & 15), col = 16 * (c >> 2) + 4 * (l >> 4) + (c & 3);
        lds[kOffW1 + ((t * 8 + (c >> 2)) * 64 + l) * 4 + (c & 3)] = m.w1[row * 128 + col];
    }
    for (int i = threadIdx.x; i < 384; i += nt) {
        const int q = i / 96, ch = (i / 32) % 3, t = (i / 4) % 8, r = i & 3;
        lds[kOffW2 + i] = m.w2[ch * 128 + 16 * t + 4 * q + r];
    }
    for (int i = threadIdx.x; i < 128; i += nt) {
        lds[kOffB0 + i] = m.b0[i];
        lds[kOffB1 + i] = m.b1[i];
    }
    if (threadIdx.x < 3) lds[kOffB2 + threadIdx.x] = m.b2[threadIdx.x];
}

__device__ __forceinline__ float pick3(int i, float a, float b, float c) { return i == 0 ? a : (i == 1 ? b : c); }

// Layer-0 inputs of one sample for this lane's group q.
template <typename T>
__device__ __forceinline__ void sample_inputs(const GridK &g, const RenderBufs &b, int64_t rec, int q, float x[10])
{
    const uint32_t ray = b.rec_ray[rec];
    const int k = b.rec_k[rec];
    const RayInfo inf = b.info[ray];
    float o[3], d[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        o[a] = b.rays_o[3 * (int64_t)ray + a];
        d[a] = b.rays_d[3 * (int64_t)ray + a];
    }
    int i0[3];
    float fr[3], tk;
    sample_voxel(o, d, inf.tn, inf.delta, k, g, i0, fr, tk);
    const T *feat = (const T *)g.features;
#pragma unroll
    for (int c = 0; c < 3; ++c) x[c] = trilerp1(feat, g, i0, fr, 12, 3 * q + c);
    x[3] = q < 3 ? pick3(q, d[0], d[1], d[2]) : 0.f;
#pragma unroll
    for (int jj = 0; jj < 3; ++jj) {
        const int p = 3 * q + jj;
        const float a = ldexpf(pick3(p >> 2, d[0], d[1], d[2]), p & 3);
        float sn, cs;
        sincosf(a, &sn, &cs);
        x[4 + 2 * jj] = sn;
        x[5 + 2 * jj] = cs;
    }
}

// STAGE: also write x (with the constant-1 slot), h1 and h2 of every sample
// to its stage row for the adjoint's weight gradients.
template <typename T, bool STAGE>
__global__ __launch_bounds__(kMlpWaves * 64, 1) void k_mlp_fwd_f32(GridK g, cic_mlp m, RenderBufs b, int voxel)
{
    extern __shared__ float lds[];
    stage_weights_f32(m, lds);
    __syncthreads();

    const int lane = lane_id(), q = lane >> 4, j = lane & 15;
    const int wave = threadIdx.x / 64;
    const int64_t total = (int64_t)b.offsets[b.n];
    const int64_t nbatch = (total + kBatch - 1) / kBatch;
    const f2_t *w0f = (const f2_t *)(lds + kOffW0);
    const f4_t *w1f = (const f4_t *)(lds + kOffW1);
    const f4_t *w2l = (const f4_t *)(lds + kOffW2);

    for (int64_t bt = (int64_t)blockIdx.x * kMlpWaves + wave; bt < nbatch; bt += (int64_t)gridDim.x * kMlpWaves) {
        float x[kNT][10];
        int64_t rec[kNT];
        bool valid[kNT];
#pragma unroll
        for (int nt = 0; nt < kNT; ++nt) {
            const int64_t s = bt * kBatch + nt * 16 + j;
            valid[nt] = s < total;
            rec[nt] = valid[nt] ? (voxel ? (int64_t)b.perm[s] : s) : 0;
            if (valid[nt]) {
                sample_inputs<T>(g, b, rec[nt], q, x[nt]);
                if (STAGE) {
                    float *row = b.stage + rec[nt] * kStageStride + kStX;
#pragma unroll
                    for (int c = 0; c < 10; ++c) {
                        const int src = l0_input(c, q);
                        row[src >= 0 ? src : 39] = src >= 0 ? x[nt][c] : 1.0f;
                    }
                }
            } else {
#pragma unroll
                for (int c = 0; c < 10; ++c) x[nt][c] = 0.f;
            }
        }

        // layer 0: 40 -> 128
        f4_t h1[8][kNT];
#pragma unroll
        for (int t = 0; t < 8; ++t) {
            const f4_t bias = *(const f4_t *)(lds + kOffB0 + 16 * t + 4 * q);
#pragma unroll
            for (int nt = 0; nt < kNT; ++nt) h1[t][nt] = bias;
        }
        // A fragments are software-pipelined one step ahead; the scheduling
        // barrier keeps the compiler from hoisting every LDS read (which
        // would exceed the register file).
        {
            f2_t a = w0f[lane];
#pragma unroll
            for (int c2 = 0; c2 < 5; ++c2) {
#pragma unroll
                for (int t = 0; t < 8; ++t) {
                    const int nx = (c2 * 8 + t + 1 < 40) ? (c2 * 8 + t + 1) : (c2 * 8 + t);
                    const f2_t an = w0f[((nx % 8) * 5 + nx / 8) * 64 + lane];
#pragma unroll
                    for (int nt = 0; nt < kNT; ++nt) {
                        h1[t][nt] = __builtin_amdgcn_mfma_f32_16x16x4f32(a.x, x[nt][2 * c2], h1[t][nt], 0, 0, 0);
                        h1[t][nt] = __builtin_amdgcn_mfma_f32_16x16x4f32(a.y, x[nt][2 * c2 + 1], h1[t][nt], 0, 0, 0);
                    }
                    a = an;
                    __builtin_amdgcn_sched_barrier(0);
                }
            }
        }
#pragma unroll
        for (int t = 0; t < 8; ++t)
#pragma unroll
            for (int nt = 0; nt < kNT; ++nt)
#pragma unroll
                for (int r = 0; r < 4; ++r) h1[t][nt][r] = fmaxf(h1[t][nt][r], 0.f);
        if (STAGE) {
#pragma unroll
            for (int nt = 0; nt < kNT; ++nt)
                if (valid[nt])
#pragma unroll
                    for (int t = 0; t < 8; ++t)
                        *(f4_t *)(b.stage + rec[nt] * kStageStride + kStH1 + 16 * t + 4 * q) = h1[t][nt];
        }

        // layer 1: 128 -> 128
        f4_t h2[8][kNT];
#pragma unroll
        for (int t = 0; t < 8; ++t) {
            const f4_t bias = *(const f4_t *)(lds + kOffB1 + 16 * t + 4 * q);
#pragma unroll
            for (int nt = 0; nt < kNT; ++nt) h2[t][nt] = bias;
        }
        {
            f4_t a = w1f[lane];
#pragma unroll
            for (int c4 = 0; c4 < 8; ++c4) {
#pragma unroll
                for (int t = 0; t < 8; ++t) {
                    const int nx = (c4 * 8 + t + 1 < 64) ? (c4 * 8 + t + 1) : (c4 * 8 + t);
                    const f4_t an = w1f[((nx % 8) * 8 + nx / 8) * 64 + lane];
#pragma unroll
                    for (int rr = 0; rr < 4; ++rr)
#pragma unroll
                        for (int nt = 0; nt < kNT; ++nt)
                            h2[t][nt] =
                                __builtin_amdgcn_mfma_f32_16x16x4f32(a[rr], h1[c4][nt][rr], h2[t][nt], 0, 0, 0);
                    a = an;
                    __builtin_amdgcn_sched_barrier(0);
                }
            }
        }

        if (STAGE) {
#pragma unroll
            for (int nt = 0; nt < kNT; ++nt)
                if (valid[nt])
#pragma unroll
                    for (int t = 0; t < 8; ++t) {
                        f4_t v = h2[t][nt];
#pragma unroll
                        for (int r = 0; r < 4; ++r) v[r] = fmaxf(v[r], 0.f);
                        *(f4_t *)(b.stage + rec[nt] * kStageStride + kStH2 + 16 * t + 4 * q) = v;
                    }
        }
        // layer 2: 128 -> 3 on the vector ALUs, then sigmoid
#pragma unroll
        for (int nt = 0; nt < kNT; ++nt) {
            float p0 = 0.f, p1 = 0.f, p2 = 0.f;
#pragma unroll
            for (int t = 0; t < 8; ++t) {
                const f4_t wa = w2l[(q * 3 + 0) * 8 + t];
                const f4_t wb = w2l[(q * 3 + 1) * 8 + t];
                const f4_t wc = w2l[(q * 3 + 2) * 8 + t];
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const float hv = fmaxf(h2[t][nt][r], 0.f);
                    p0 = fmaf(wa[r], hv, p0);
                    p1 = fmaf(wb[r], hv, p1);
                    p2 = fmaf(wc[r], hv, p2);
                }
            }
            p0 += __shfl_xor(p0, 16, kWave);
            p1 += __shfl_xor(p1, 16, kWave);
            p2 += __shfl_xor(p2, 16, kWave);
            p0 += __shfl_xor(p0, 32, kWave);
            p1 += __shfl_xor(p1, 32, kWave);
            p2 += __shfl_xor(p2, 32, kWave);
            if (valid[nt] && q < 3) {
                const float logit = pick3(q, p0, p1, p2) + lds[kOffB2 + q];
                b.rec_c[3 * rec[nt] + q] = sigmoidf(logit);
            }
        }
    }
}

static int num_cus()
{
    int dev = 0, n = 0;
    (void)hipGetDevice(&dev);
    (void)hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, dev);
    return n > 0 ? n : 256;
}

template <typename T, bool STAGE>
static void launch_fwd(const GridK &g, const cic_mlp &m, const RenderBufs &b, bool voxel, hipStream_t s)
{
    const int lds = mlp_lds_bytes(m.compute);
    static bool attr_set = false;   // per process; the attribute is per kernel
    if (!attr_set) {
        (void)hipFuncSetAttribute((const void *)k_mlp_fwd_f32<T, STAGE>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                  lds);
        attr_set = true;
    }
    hipLaunchKernelGGL((k_mlp_fwd_f32<T, STAGE>), dim3(num_cus()), dim3(kMlpWaves * 64), lds, s, g, m, b,
                       voxel ? 1 : 0);
}

template <typename T>
void launch_mlp_forward(const GridK &g, const cic_mlp &m, const RenderBufs &b, bool voxel, hipStream_t s)
{
    launch_fwd<T, false>(g, m, b, voxel, s);
}

void launch_mlp_forward_staged(const GridK &g, const cic_mlp &m, const RenderBufs &b, hipStream_t s)
{
    launch_fwd<float, true>(g, m, b, false, s);
}
template void launch_mlp_forward<float>(const GridK &, const cic_mlp &, const RenderBufs &, bool, hipStream_t);
template void launch_mlp_forward<__half>(const GridK &, const cic_mlp &, const RenderBufs &, bool, hipStream_t);

}  // namespace cic
