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
#include "mlp_common.h"

namespace cic {

// 16-sample tiles per wavefront batch; one tile keeps a wavefront under 128
// VGPRs, so the 16 wavefronts of the CU's single workgroup (the weights take
// 88 KB of LDS) give four per SIMD to overlap gathers with MFMA work.
#ifndef CIC_F32_NT
#define CIC_F32_NT 1
#endif
constexpr int kNT = CIC_F32_NT;

constexpr int kMlpWaves = kNT == 1 ? 16 : 8;
constexpr int kBatch = 16 * kNT;

int mlp_lds_bytes(int compute)
{
    (void)compute;
    return kLdsF32 * (int)sizeof(float);
}

// Per-ray direction term of layer 0: z0[ray][o] = b0[o] + sum_i W0[o][12+i] pe_i
// over the 27 direction inputs (d, sin, cos), once per ray with live samples
// (float32; used by the FP32 MLP in either order).  A block stages the
// inputs of kEmbedRays rays in LDS (one sincosf per argument gives both its
// sine and cosine input), and each of its 128 threads then forms output o for
// every ray with its 27 weights held in registers.
#ifndef CIC_EMBED_RAYS
#define CIC_EMBED_RAYS 64
#endif
constexpr int kEmbedRays = CIC_EMBED_RAYS;

__global__ __launch_bounds__(128) void k_ray_embed(cic_mlp m, RenderBufs b, float *z0)
{
    __shared__ float pe[kEmbedRays][28];
    __shared__ uint32_t live[kEmbedRays];
    const int o = threadIdx.x;
    const int64_t base = (int64_t)blockIdx.x * kEmbedRays;
    // a pass over a device-counted set of rays (the holes of a warped frame)
    // skips the blocks past its count, whose rays have no live samples
    if (b.n_active && (uint64_t)base >= *b.n_active) return;
    for (int r = threadIdx.x; r < kEmbedRays; r += 128) live[r] = base + r < b.n ? b.count[base + r] : 0u;
    __syncthreads();
    // entries 0..2: the direction; argument k = 4c + octave (k < 12): sine at
    // 3 + k, cosine at 15 + k
    for (int e = threadIdx.x; e < kEmbedRays * 15; e += 128) {
        const int r = e / 15, i = e % 15;
        if (!live[r]) continue;
        const float *d = b.rays_d + 3 * (base + r);
        if (i < 3) {
            pe[r][i] = d[i];
        } else {
            const int k = i - 3, c = k >> 2, oc = k & 3;
            float sn, cs;
            sincosf(ldexpf(d[c], oc), &sn, &cs);
            pe[r][3 + k] = sn;
            pe[r][15 + k] = cs;
        }
    }
    __syncthreads();
    float w[27];
#pragma unroll
    for (int i = 0; i < 27; ++i) w[i] = m.w0[o * 39 + 12 + i];
    const float bias = m.b0[o];
    for (int r = 0; r < kEmbedRays; ++r) {
        if (!live[r]) continue;
        float acc = bias;
#pragma unroll
        for (int i = 0; i < 27; ++i) acc = fmaf(w[i], pe[r][i], acc);
        z0[(base + r) * 128 + o] = acc;
    }
}

void launch_ray_embed(const cic_mlp &m, const RenderBufs &b, hipStream_t s)
{
    if (b.n == 0 || m.compute != CIC_F32) return;
    const unsigned blocks = (unsigned)((b.n + kEmbedRays - 1) / kEmbedRays);
    hipLaunchKernelGGL(k_ray_embed, dim3(blocks), dim3(128), 0, s, m, b, b.z0);
}

// PET: the direction half of layer 0 comes from the per-ray table, so layer 0
// only multiplies the 12 interpolated features.
template <typename T, bool PET>
__global__ __launch_bounds__(kMlpWaves * 64, 1) void k_mlp_fwd_f32(GridK g, cic_mlp m, RenderBufs b, int voxel)
{
    extern __shared__ __attribute__((aligned(16))) float lds[];
    stage_weights_f32(m, lds);
    __syncthreads();

    const int lane = lane_id(), q = lane >> 4, j = lane & 15;
    const int wave = threadIdx.x / 64;
    const int64_t total = (int64_t)b.offsets[b.n];
    const int64_t nbatch = (total + kBatch - 1) / kBatch;
    const f2_t *w0f = (const f2_t *)(lds + kOffW0);
    const f4_t *w1f = (const f4_t *)(lds + kOffW1);
    const f4_t *w2l = (const f4_t *)(lds + kOffW2);

    const BatchRange br = xcd_batches(nbatch, kMlpWaves, wave);
    // Sample s of the wave's batch bt (a lane past the last sample works on
    // sample 0: in-bounds inputs, no branches around the loads; its colour is
    // not stored), and its record.
    auto record_of = [&](int64_t bt, int nt) -> uint32_t {
        const int64_t s = bt * kBatch + nt * 16 + j;
        const int64_t sv = s < total ? s : 0;
        return voxel ? b.perm[sv] : (uint32_t)sv;
    };
    // The next batch's record, ray and sample index are loaded during this
    // batch's layer 1 and its ray's origin, direction and interval during
    // layer 2, so a batch starts with only its grid gathers outstanding.
    SampleRay cur[kNT];
    uint32_t crec[kNT];
    if (br.first < br.end) {
#pragma unroll
        for (int nt = 0; nt < kNT; ++nt) {
            crec[nt] = record_of(br.first, nt);
            load_sample_ray(b, b.rec_ray[crec[nt]], b.rec_k[crec[nt]], cur[nt]);
        }
    }
    for (int64_t bt = br.first; bt < br.end; bt += br.stride) {
        // Wave priority (within this kernel's wavefronts on a SIMD): low
        // while gathering the batch's inputs, raised at each layer so that
        // the wavefront furthest through its batch wins the matrix unit.
        // Fair sharing otherwise lets the four wavefronts of a SIMD finish
        // their MFMA phases together and then wait on their gathers together
        // (measured per 800x800 frame: 16.68 ms without priorities, 16.37 ms
        // with one raise at layer 0, 16.23-16.30 ms raising per layer).
        __builtin_amdgcn_s_setprio(0);
        float x[kNT][10];
        uint32_t rec[kNT];
        bool valid[kNT];
#pragma unroll
        for (int nt = 0; nt < kNT; ++nt) {
            valid[nt] = bt * kBatch + nt * 16 + j < total;
            rec[nt] = crec[nt];
            sample_inputs_from<T, !PET>(g, cur[nt], q, x[nt]);
        }
        const bool more = bt + br.stride < br.end;
        uint32_t nrec[kNT], nray[kNT];
        int nk[kNT];

        // layer 0: 40 -> 128 (PET: 12 -> 128 on top of the per-ray term)
        __builtin_amdgcn_s_setprio(1);
        f4_t h1[8][kNT];
        if (PET) {
#pragma unroll
            for (int nt = 0; nt < kNT; ++nt) {
                // (every record's ray has live samples, so its row is written)
                const float *zr = b.z0 + (int64_t)cur[nt].ray * 128 + 4 * q;
#pragma unroll
                for (int t = 0; t < 8; ++t) h1[t][nt] = *(const f4_t *)(zr + 16 * t);
            }
        } else {
#pragma unroll
            for (int t = 0; t < 8; ++t) {
                const f4_t bias = *(const f4_t *)(lds + kOffB0 + 16 * t + 4 * q);
#pragma unroll
                for (int nt = 0; nt < kNT; ++nt) h1[t][nt] = bias;
            }
        }
        // Layer 0: per input chunk pair, the eight output tiles' A fragments
        // are read together and the MFMAs alternate between the eight
        // independent accumulators.  The scheduling barriers keep the
        // compiler from hoisting every LDS read (which would exceed the
        // register budget).
        constexpr int kC2 = PET ? 2 : 5;   // PET: chunks 0..2 (features) only
#pragma unroll
        for (int c2 = 0; c2 < kC2; ++c2) {
            f2_t a[8];
#pragma unroll
            for (int t = 0; t < 8; ++t) a[t] = w0f[(t * 5 + c2) * 64 + lane];
#pragma unroll
            for (int e = 0; e < 2; ++e) {
                if (PET && 2 * c2 + e >= 3) continue;
#pragma unroll
                for (int t = 0; t < 8; ++t)
#pragma unroll
                    for (int nt = 0; nt < kNT; ++nt)
                        h1[t][nt] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[t][e], x[nt][2 * c2 + e], h1[t][nt], 0, 0,
                                                                          0);
            }
            __builtin_amdgcn_sched_barrier(0);
        }
        // ReLU of h1: one input chunk ahead inside layer 1, so the vector
        // work overlaps its MFMAs
#pragma unroll
        for (int nt = 0; nt < kNT; ++nt)
#pragma unroll
            for (int r = 0; r < 4; ++r) h1[0][nt][r] = relu_bits(h1[0][nt][r]);

        // layer 1: 128 -> 128
        __builtin_amdgcn_s_setprio(2);
#pragma unroll
        for (int nt = 0; nt < kNT; ++nt) {
            nrec[nt] = record_of(more ? bt + br.stride : 0, nt);
            nray[nt] = b.rec_ray[nrec[nt]];
            nk[nt] = b.rec_k[nrec[nt]];
        }
        __builtin_amdgcn_sched_barrier(0);
        f4_t h2[8][kNT];
#pragma unroll
        for (int t = 0; t < 8; ++t) {
            const f4_t bias = *(const f4_t *)(lds + kOffB1 + 16 * t + 4 * q);
#pragma unroll
            for (int nt = 0; nt < kNT; ++nt) h2[t][nt] = bias;
        }
        // Layer 1: groups of four output tiles; the next group's fragments
        // are read while the current group's 16 MFMAs (four independent
        // accumulators, one per tile) run.
        {
            f4_t a[4], an[4];
#pragma unroll
            for (int tt = 0; tt < 4; ++tt) a[tt] = w1f[(tt * 8 + 0) * 64 + lane];
#pragma unroll
            for (int c4 = 0; c4 < 8; ++c4) {
#pragma unroll
                for (int tg = 0; tg < 2; ++tg) {
                    const int step = c4 * 2 + tg, nx = step + 1 < 16 ? step + 1 : step;
                    const int nc4 = nx >> 1, ntg = nx & 1;
#pragma unroll
                    for (int tt = 0; tt < 4; ++tt) an[tt] = w1f[((4 * ntg + tt) * 8 + nc4) * 64 + lane];
#pragma unroll
                    for (int rr = 0; rr < 4; ++rr)
#pragma unroll
                        for (int tt = 0; tt < 4; ++tt)
#pragma unroll
                            for (int nt = 0; nt < kNT; ++nt)
                                h2[4 * tg + tt][nt] = __builtin_amdgcn_mfma_f32_16x16x4f32(
                                    a[tt][rr], h1[c4][nt][rr], h2[4 * tg + tt][nt], 0, 0, 0);
                    if (tg == 1 && c4 + 1 < 8) {
#pragma unroll
                        for (int nt = 0; nt < kNT; ++nt)
#pragma unroll
                            for (int r = 0; r < 4; ++r) h1[c4 + 1][nt][r] = relu_bits(h1[c4 + 1][nt][r]);
                    }
#pragma unroll
                    for (int tt = 0; tt < 4; ++tt) a[tt] = an[tt];
                    __builtin_amdgcn_sched_barrier(0);
                }
            }
        }

        // layer 2: 128 -> 3 on the vector ALUs, then sigmoid
        __builtin_amdgcn_s_setprio(3);
#pragma unroll
        for (int nt = 0; nt < kNT; ++nt) {
            crec[nt] = nrec[nt];
            load_sample_ray(b, nray[nt], nk[nt], cur[nt]);
        }
        __builtin_amdgcn_sched_barrier(0);
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
                    const float hv = relu_bits(h2[t][nt][r]);
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
                b.rec_c[3 * (int64_t)rec[nt] + q] = sigmoid_hw(logit);
            }
        }
    }
}

template <typename T, bool PET>
static void launch_fwd(const GridK &g, const cic_mlp &m, const RenderBufs &b, bool voxel, hipStream_t s)
{
    const int lds = mlp_lds_bytes(m.compute);
    static bool attr_set = false;   // per process; the attribute is per kernel
    if (!attr_set) {
        (void)hipFuncSetAttribute((const void *)k_mlp_fwd_f32<T, PET>,
                                  hipFuncAttributeMaxDynamicSharedMemorySize, lds);
        attr_set = true;
    }
    hipLaunchKernelGGL((k_mlp_fwd_f32<T, PET>), dim3(num_cus(b)), dim3(kMlpWaves * 64), lds, s, g, m, b,
                       voxel ? 1 : 0);
}

// FP32, in either order, uses the per-ray direction table (b.z0 must be
// filled by launch_ray_embed first): in voxel order the samples of a ray
// within a brick are consecutive, so the table rows stay cached (measured
// on eight 800x800 views: MLP 145.1 -> 128.3 ms, against 125.8 ms in ray
// order), and both orders then give the same bits.  The BF16 kernel reads a
// per-ray BF16 encoding table instead.
template <typename T>
void launch_mlp_forward(const GridK &g, const cic_mlp &m, const RenderBufs &b, bool voxel, hipStream_t s)
{
    if (m.compute == CIC_BF16) {
        launch_mlp_forward_bf16<T>(g, m, b, voxel, s);
        return;
    }
    launch_fwd<T, true>(g, m, b, voxel, s);
}

template void launch_mlp_forward<float>(const GridK &, const cic_mlp &, const RenderBufs &, bool, hipStream_t);
template void launch_mlp_forward<__half>(const GridK &, const cic_mlp &, const RenderBufs &, bool, hipStream_t);

}  // namespace cic
