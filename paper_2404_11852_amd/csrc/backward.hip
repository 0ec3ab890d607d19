// Adjoint of the rendering quadrature, the MLP and the trilinear gathers.
//
// With C = sum_k w_k c_k + T_stop bg, w_k = T_k (1 - e^{-sigma_k delta}) and
// T_{k+1} = T_k e^{-sigma_k delta}, the derivative with respect to the
// density of live sample k is
//   dC/dsigma_k = delta (T_{k+1} c_k - R_k),  R_k = sum_{j>k} w_j c_j + T_stop bg,
// (every later weight and the background term scale with T_{k+1}), the
// expected distance gives delta (T_{k+1} t_k - D_k) with D_k = sum_{j>k} w_j t_j,
// and the opacity 1 - T_stop gives delta T_stop.  dC/dc_k = w_k.
//
// Kernels (one backward pass over a chunk of rays; the forward has already
// been recomputed into the workspace, with per-sample MLP vectors staged):
//  - k_bwd_composite: one wavefront per ray walks its live samples from the
//    back, 64 at a time, with a reverse wavefront scan for R_k and D_k; it
//    writes dL/dc_k and scatter-adds dL/draw through the trilinear weights.
//  - k_mlp_bwd: per 32-sample batch, the output-layer adjoint on the vector
//    ALUs, then W1^T and W0^T products on FP32 MFMA (transposed weight
//    fragments in LDS); hidden-layer gradients are staged for the weight
//    gradients and the feature gradient is scatter-added to the grid.
//  - k_wgrad: weight gradients as split-K MFMA products over the staged
//    per-sample vectors, one partial per block, reduced in a fixed order by
//    k_wgrad_apply (deterministic).
#include "kernels.h"

namespace cic {

typedef float f4_t __attribute__((ext_vector_type(4)));

// Reverse inclusive scan (sum over lanes >= this lane).
__device__ __forceinline__ float wave_rev_incl_scan(float v)
{
    const int l = lane_id();
#pragma unroll
    for (int off = 1; off < kWave; off <<= 1) {
        const float u = __shfl_down(v, off, kWave);
        if (l + off < kWave) v += u;
    }
    return v;
}

__device__ __forceinline__ void scatter_trilinear(float *grad, const GridK &g, const int i0[3], const float fr[3],
                                                  int stride, int ch, float v)
{
    const float wx[2] = {1.f - fr[0], fr[0]}, wy[2] = {1.f - fr[1], fr[1]}, wz[2] = {1.f - fr[2], fr[2]};
#pragma unroll
    for (int c = 0; c < 8; ++c) {
        const int dx = (c >> 2) & 1, dy = (c >> 1) & 1, dz = c & 1;
        const float w = wx[dx] * wy[dy] * wz[dz];
        atomicAdd(grad + vertex_index(g, i0[0] + dx, i0[1] + dy, i0[2] + dz) * stride + ch, w * v);
    }
}

__global__ __launch_bounds__(256) void k_bwd_composite(GridK g, OptsK op, RenderBufs b, BackwardBufs bb)
{
    const int lane = lane_id();
    const int64_t ray = (int64_t)blockIdx.x * 4 + (threadIdx.x / kWave);
    if (ray >= b.n) return;
    const uint32_t cnt = b.count[ray];
    if (cnt == 0) return;
    const uint32_t off = b.offsets[ray];
    const RayInfo inf = b.info[ray];
    const float gr[3] = {bb.d_rgb[3 * ray], bb.d_rgb[3 * ray + 1], bb.d_rgb[3 * ray + 2]};
    const float gd = bb.d_depth_t ? bb.d_depth_t[ray] : 0.f;
    const float ga = bb.d_acc ? bb.d_acc[ray] : 0.f;
    float o[3], d[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        o[a] = b.rays_o[3 * ray + a];
        d[a] = b.rays_d[3 * ray + a];
    }
    const float *dens = (const float *)g.density;
    float carry[3] = {inf.t_stop * op.bg[0], inf.t_stop * op.bg[1], inf.t_stop * op.bg[2]};
    float carry_d = 0.f;
    const int nch = (int)((cnt + kWave - 1) / kWave);
    for (int chn = nch - 1; chn >= 0; --chn) {
        const uint32_t j = (uint32_t)chn * kWave + lane;
        const bool act = j < cnt;
        float w = 0.f, T = 0.f, c[3] = {0.f, 0.f, 0.f}, tk = 0.f;
        int i0[3] = {0, 0, 0};
        float fr[3] = {0.f, 0.f, 0.f};
        if (act) {
            const int64_t r = (int64_t)off + j;
            w = b.rec_w[r];
            T = b.rec_t[r];
            c[0] = b.rec_c[3 * r];
            c[1] = b.rec_c[3 * r + 1];
            c[2] = b.rec_c[3 * r + 2];
            sample_voxel(o, d, inf.tn, inf.delta, b.rec_k[r], g, i0, fr, tk);
        }
        float R[3], incl[3];
#pragma unroll
        for (int ch = 0; ch < 3; ++ch) {
            incl[ch] = wave_rev_incl_scan(w * c[ch]);
            R[ch] = carry[ch] + (incl[ch] - w * c[ch]);
        }
        const float incl_d = wave_rev_incl_scan(w * tk);
        const float D = carry_d + (incl_d - w * tk);
        if (act) {
            const int64_t r = (int64_t)off + j;
            const float Tn = T - w;   // T_{k+1} = T_k (1 - alpha_k)
            float ds = 0.f;
#pragma unroll
            for (int ch = 0; ch < 3; ++ch) ds = fmaf(gr[ch], fmaf(Tn, c[ch], -R[ch]), ds);
            ds = fmaf(gd, fmaf(Tn, tk, -D), ds);
            ds = fmaf(ga, inf.t_stop, ds);
            ds *= inf.delta;
            const float raw = trilerp1(dens, g, i0, fr, 1, 0);
            const float draw = ds * sigmoidf(raw + g.shift);
            if (bb.rec_draw) bb.rec_draw[r] = draw;   // added per brick with the feature gradients
            else scatter_trilinear(bb.d_density, g, i0, fr, 1, 0, draw);
#pragma unroll
            for (int ch = 0; ch < 3; ++ch) bb.rec_dc[3 * r + ch] = w * gr[ch];
        }
#pragma unroll
        for (int ch = 0; ch < 3; ++ch) carry[ch] += __shfl(incl[ch], 0, kWave);
        carry_d += __shfl(incl_d, 0, kWave);
    }
}

void launch_backward_composite(const GridK &g, const OptsK &o, const RenderBufs &b, const BackwardBufs &bb,
                               hipStream_t s)
{
    if (b.n == 0) return;
    hipLaunchKernelGGL(k_bwd_composite, dim3((unsigned)((b.n + 3) / 4)), dim3(256), 0, s, g, o, b, bb);
}

// ---------------------------------------------------------------------------
// MLP backward
// ---------------------------------------------------------------------------
constexpr int kBwdWaves = 8;
constexpr int kBNT = 2;
// LDS (floats): W1T fragments [ti 8][c4 8][lane 64][4], W0T fragments
// [c4 8][lane 64][4], W2 [q 4][ch 3][t 8][r 4]
constexpr int kBOffW1T = 0;
constexpr int kBOffW0T = kBOffW1T + 8 * 8 * 64 * 4;
constexpr int kBOffW2 = kBOffW0T + 8 * 64 * 4;
constexpr int kBLds = kBOffW2 + 384;

__global__ __launch_bounds__(kBwdWaves * 64, 1) void k_mlp_bwd(GridK g, cic_mlp m, RenderBufs b, BackwardBufs bb,
                                                               int voxel)
{
    extern __shared__ float lds[];
    const int nthr = blockDim.x;
    for (int i = threadIdx.x; i < 8 * 8 * 64 * 4; i += nthr) {
        const int rr = i & 3, l = (i >> 2) & 63, c4 = (i >> 8) & 7, ti = i >> 11;
        lds[kBOffW1T + i] = m.w1[(16 * c4 + 4 * (l >> 4) + rr) * 128 + 16 * ti + (l & 15)];
    }
    for (int i = threadIdx.x; i < 8 * 64 * 4; i += nthr) {
        const int rr = i & 3, l = (i >> 2) & 63, c4 = i >> 8;
        const int col = l & 15;
        lds[kBOffW0T + i] = col < 12 ? m.w0[(16 * c4 + 4 * (l >> 4) + rr) * 39 + col] : 0.f;
    }
    for (int i = threadIdx.x; i < 384; i += nthr) {
        const int q = i / 96, ch = (i / 32) % 3, t = (i / 4) % 8, r = i & 3;
        lds[kBOffW2 + i] = m.w2[ch * 128 + 16 * t + 4 * q + r];
    }
    __syncthreads();

    const int lane = lane_id(), q = lane >> 4, j = lane & 15;
    const int wave = threadIdx.x / 64;
    const int64_t total = (int64_t)b.offsets[b.n];
    const int64_t nbatch = (total + 16 * kBNT - 1) / (16 * kBNT);
    const f4_t *w1t = (const f4_t *)(lds + kBOffW1T);
    const f4_t *w0t = (const f4_t *)(lds + kBOffW0T);
    const f4_t *w2l = (const f4_t *)(lds + kBOffW2);
    float *dfeat_grad = bb.d_features;

    const BatchRange br = xcd_batches(nbatch, kBwdWaves, wave);
    for (int64_t bt = br.first; bt < br.end; bt += br.stride) {
        int64_t rec[kBNT];
        bool valid[kBNT];
        f4_t dp1[8][kBNT];
        f4_t h1m[8][kBNT];   // h1 > 0 masks as values
#pragma unroll
        for (int nt = 0; nt < kBNT; ++nt) {
            const int64_t s = bt * (16 * kBNT) + nt * 16 + j;
            valid[nt] = s < total;
            rec[nt] = valid[nt] ? (voxel ? (int64_t)b.perm[s] : s) : 0;
            const float *row = b.stage + rec[nt] * kStageStride;
            float dl[3] = {0.f, 0.f, 0.f};
            if (valid[nt]) {
#pragma unroll
                for (int ch = 0; ch < 3; ++ch) {
                    const float c = b.rec_c[3 * rec[nt] + ch];
                    dl[ch] = bb.rec_dc[3 * rec[nt] + ch] * c * (1.f - c);
                }
            }
#pragma unroll
            for (int t = 0; t < 8; ++t) {
                const f4_t h2 = valid[nt] ? *(const f4_t *)(row + kStH2 + 16 * t + 4 * q) : f4_t{0.f, 0.f, 0.f, 0.f};
                h1m[t][nt] = valid[nt] ? *(const f4_t *)(row + kStH1 + 16 * t + 4 * q) : f4_t{0.f, 0.f, 0.f, 0.f};
                const f4_t wa = w2l[(q * 3 + 0) * 8 + t], wb = w2l[(q * 3 + 1) * 8 + t], wc = w2l[(q * 3 + 2) * 8 + t];
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const float v = fmaf(wa[r], dl[0], fmaf(wb[r], dl[1], wc[r] * dl[2]));
                    dp1[t][nt][r] = h2[r] > 0.f ? v : 0.f;
                }
            }
            if (valid[nt]) {
                float *wrow = b.stage + rec[nt] * kStageStride;
#pragma unroll
                for (int t = 0; t < 8; ++t) *(f4_t *)(wrow + kStDP1 + 16 * t + 4 * q) = dp1[t][nt];
                *(f4_t *)(wrow + kStDL + 4 * q) = (q == 0) ? f4_t{dl[0], dl[1], dl[2], 0.f} : f4_t{0.f, 0.f, 0.f, 0.f};
            }
        }
        // dh1 = W1^T dp1, dp0 = dh1 * [h1 > 0]
        f4_t dp0[8][kBNT];
#pragma unroll
        for (int ti = 0; ti < 8; ++ti)
#pragma unroll
            for (int nt = 0; nt < kBNT; ++nt) dp0[ti][nt] = f4_t{0.f, 0.f, 0.f, 0.f};
        {
            f4_t a = w1t[lane];
#pragma unroll
            for (int ti = 0; ti < 8; ++ti) {
#pragma unroll
                for (int c4 = 0; c4 < 8; ++c4) {
                    const int nx = (ti * 8 + c4 + 1 < 64) ? (ti * 8 + c4 + 1) : (ti * 8 + c4);
                    const f4_t an = w1t[nx * 64 + lane];
#pragma unroll
                    for (int rr = 0; rr < 4; ++rr)
#pragma unroll
                        for (int nt = 0; nt < kBNT; ++nt)
                            dp0[ti][nt] =
                                __builtin_amdgcn_mfma_f32_16x16x4f32(a[rr], dp1[c4][nt][rr], dp0[ti][nt], 0, 0, 0);
                    a = an;
                    __builtin_amdgcn_sched_barrier(0);
                }
            }
        }
#pragma unroll
        for (int ti = 0; ti < 8; ++ti)
#pragma unroll
            for (int nt = 0; nt < kBNT; ++nt)
#pragma unroll
                for (int r = 0; r < 4; ++r) dp0[ti][nt][r] = h1m[ti][nt][r] > 0.f ? dp0[ti][nt][r] : 0.f;
#pragma unroll
        for (int nt = 0; nt < kBNT; ++nt)
            if (valid[nt]) {
                float *wrow = b.stage + rec[nt] * kStageStride;
#pragma unroll
                for (int t = 0; t < 8; ++t) *(f4_t *)(wrow + kStDP0 + 16 * t + 4 * q) = dp0[t][nt];
            }
        // feature gradient = (W0^T dp0)[0:12], scattered to the grid
        f4_t df[kBNT];
#pragma unroll
        for (int nt = 0; nt < kBNT; ++nt) df[nt] = f4_t{0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int c4 = 0; c4 < 8; ++c4) {
            const f4_t a = w0t[c4 * 64 + lane];
#pragma unroll
            for (int rr = 0; rr < 4; ++rr)
#pragma unroll
                for (int nt = 0; nt < kBNT; ++nt)
                    df[nt] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[rr], dp0[c4][nt][rr], df[nt], 0, 0, 0);
        }
        if (bb.df_sorted) {
            // brick-tile mode: keep the 12 feature gradients of the sample at its
            // position in brick order; k_fgrad_brick accumulates them
#pragma unroll
            for (int nt = 0; nt < kBNT; ++nt) {
                const int64_t s = bt * (16 * kBNT) + nt * 16 + j;
                if (valid[nt] && q < 3) *(f4_t *)(bb.df_sorted + s * 12 + 4 * q) = df[nt];
            }
            continue;
        }
#pragma unroll
        for (int nt = 0; nt < kBNT; ++nt) {
            if (!valid[nt] || q >= 3) continue;
            const uint32_t ray = b.rec_ray[rec[nt]];
            const RayInfo inf = b.info[ray];
            float o[3], d[3];
#pragma unroll
            for (int a = 0; a < 3; ++a) {
                o[a] = b.rays_o[3 * (int64_t)ray + a];
                d[a] = b.rays_d[3 * (int64_t)ray + a];
            }
            int i0[3];
            float fr[3], tk;
            sample_voxel(o, d, inf.tn, inf.delta, b.rec_k[rec[nt]], g, i0, fr, tk);
#pragma unroll
            for (int r = 0; r < 4; ++r) scatter_trilinear(dfeat_grad, g, i0, fr, 12, 4 * q + r, df[nt][r]);
        }
    }
}

static int num_cus_b()
{
    int dev = 0, n = 0;
    (void)hipGetDevice(&dev);
    (void)hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, dev);
    return n > 0 ? n : 256;
}

// Feature and density gradients, one workgroup per brick of 8^3 voxels: the
// brick's samples (contiguous in brick order) add their trilinear shares
// into a 9x9x9-vertex tile of 13 channels (12 features, raw density) in LDS,
// then the tile is added to the gradient grids with one global atomic per
// nonzero entry, consecutive entries on consecutive addresses (vertices on a
// brick face are shared with the neighbour brick, hence atomics).
constexpr int kTileV = kBrick + 1;
constexpr int kTileCh = 13;
constexpr int kTileFloats = kTileV * kTileV * kTileV * kTileCh;

__global__ __launch_bounds__(256) void k_fgrad_brick(GridK g, RenderBufs b, BackwardBufs bb)
{
    __shared__ float tile[kTileFloats];
    const int64_t brick = blockIdx.x;
    const uint32_t start = brick == 0 ? 0u : b.brick_off[brick - 1];
    const uint32_t end = b.brick_off[brick];
    if (start >= end) return;
    for (int e = threadIdx.x; e < kTileFloats; e += blockDim.x) tile[e] = 0.f;
    __syncthreads();
    const int bz = (int)(brick % g.nb2), by = (int)((brick / g.nb2) % g.nb1), bx = (int)(brick / ((int64_t)g.nb2 * g.nb1));
    const int base[3] = {kBrick * bx, kBrick * by, kBrick * bz};
    for (uint32_t s = start + threadIdx.x; s < end; s += blockDim.x) {
        const uint32_t rec = b.perm[s];
        const uint32_t ray = b.rec_ray[rec];
        const RayInfo inf = b.info[ray];
        float o[3], d[3];
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            o[a] = b.rays_o[3 * (int64_t)ray + a];
            d[a] = b.rays_d[3 * (int64_t)ray + a];
        }
        int i0[3];
        float fr[3], tk;
        sample_voxel(o, d, inf.tn, inf.delta, b.rec_k[rec], g, i0, fr, tk);
        const float wx[2] = {1.f - fr[0], fr[0]}, wy[2] = {1.f - fr[1], fr[1]}, wz[2] = {1.f - fr[2], fr[2]};
        const int lx = i0[0] - base[0], ly = i0[1] - base[1], lz = i0[2] - base[2];
        const float *df = bb.df_sorted + (int64_t)s * 12;
        float v[kTileCh];
#pragma unroll
        for (int f = 0; f < 12; ++f) v[f] = df[f];
        v[12] = bb.rec_draw[rec];
#pragma unroll
        for (int c = 0; c < 8; ++c) {
            const int dx = (c >> 2) & 1, dy = (c >> 1) & 1, dz = c & 1;
            const float w = wx[dx] * wy[dy] * wz[dz];
            float *t = tile + (((lx + dx) * kTileV + (ly + dy)) * kTileV + (lz + dz)) * kTileCh;
#pragma unroll
            for (int f = 0; f < kTileCh; ++f) atomicAdd(t + f, w * v[f]);
        }
    }
    __syncthreads();
    for (int e = threadIdx.x; e < kTileFloats; e += blockDim.x) {
        const float val = tile[e];
        if (val == 0.f) continue;
        const int f = e % kTileCh, vtx = e / kTileCh;
        const int vz = base[2] + vtx % kTileV, vy = base[1] + (vtx / kTileV) % kTileV, vx = base[0] + vtx / (kTileV * kTileV);
        if (vx < g.r0 && vy < g.r1 && vz < g.r2) {
            const int64_t vi = vertex_index(g, vx, vy, vz);
            if (f < 12) atomicAdd(bb.d_features + vi * 12 + f, val);
            else atomicAdd(bb.d_density + vi, val);
        }
    }
}

void launch_feature_grads_bricks(const GridK &g, const RenderBufs &b, const BackwardBufs &bb, hipStream_t s)
{
    if (b.n_bricks == 0) return;
    hipLaunchKernelGGL(k_fgrad_brick, dim3((unsigned)b.n_bricks), dim3(256), 0, s, g, b, bb);
}

void launch_mlp_backward(const GridK &g, const cic_mlp &m, const RenderBufs &b, const BackwardBufs &bb, bool voxel,
                         hipStream_t s)
{
    const int lds = kBLds * (int)sizeof(float);
    static bool attr_set = false;
    if (!attr_set) {
        (void)hipFuncSetAttribute((const void *)k_mlp_bwd, hipFuncAttributeMaxDynamicSharedMemorySize, lds);
        attr_set = true;
    }
    hipLaunchKernelGGL(k_mlp_bwd, dim3(num_cus_b()), dim3(kBwdWaves * 64), lds, s, g, m, b, bb, voxel ? 1 : 0);
}

// ---------------------------------------------------------------------------
// Weight gradients: sums over samples of outer products of staged vectors,
//   P0 = dp0^T [x|1|h1[0:8]]   (128 x 48: dW0 and, in column 39, db0)
//   P1 = dp1^T h1              (128 x 128: dW1)
//   P2 = dl^T h2               (16 x 128: dW2 in rows 0..2)
//   P3 = dp1^T [x|1][32:48]    (128 x 16: db1 in column 7)
//   P4 = dl^T [x|1][32:48]     (16 x 16: db2 in column 7)
// one fused pass: each block owns a contiguous range of samples, stages 16
// full rows at a time in LDS and runs all 105 output tiles on FP32 MFMA
// (K = samples), writing one partial per block; k_wgrad_apply adds the
// partials in block order (deterministic).
// ---------------------------------------------------------------------------
constexpr int kWgStep = 16;
constexpr int kWgRow = kStageStride + 4;   // padded LDS row
constexpr int kWgTiles = 24 + 64 + 8 + 8 + 1;
constexpr int kWgWaves = 8;
constexpr int kWgTPW = (kWgTiles + kWgWaves - 1) / kWgWaves;

struct WgTile {
    int a_col, b_col, out;   // stage columns of A and B, offset of the 16x16 tile in the partial
    int ld;                  // row length of the partial matrix
};

__device__ __forceinline__ WgTile wg_tile(int t)
{
    constexpr int P1 = 128 * 48, P2 = P1 + 128 * 128, P3 = P2 + 16 * 128, P4 = P3 + 128 * 16;
    if (t < 24) {
        const int mt = t / 3, nt = t % 3;
        return {kStDP0 + 16 * mt, kStX + 16 * nt, (16 * mt) * 48 + 16 * nt, 48};
    }
    t -= 24;
    if (t < 64) {
        const int mt = t / 8, nt = t % 8;
        return {kStDP1 + 16 * mt, kStH1 + 16 * nt, P1 + (16 * mt) * 128 + 16 * nt, 128};
    }
    t -= 64;
    if (t < 8) return {kStDL, kStH2 + 16 * t, P2 + 16 * t, 128};
    t -= 8;
    if (t < 8) return {kStDP1 + 16 * t, kStX + 32, P3 + (16 * t) * 16, 16};
    return {kStDL, kStX + 32, P4, 16};
}

__global__ __launch_bounds__(kWgWaves * 64, 2) void k_wgrad(const float *stage, const uint32_t *total_p, float *partials,
                                               int64_t slab)
{
    __shared__ float rows[kWgStep * kWgRow];
    const int lane = lane_id(), wave = threadIdx.x / 64;
    const int64_t total = (int64_t)*total_p;
    const int64_t s0 = (int64_t)blockIdx.x * slab;
    const int64_t s1 = (s0 + slab < total) ? s0 + slab : total;
    f4_t acc[kWgTPW];
#pragma unroll
    for (int i = 0; i < kWgTPW; ++i) acc[i] = f4_t{0.f, 0.f, 0.f, 0.f};
    constexpr int kF4Row = kStageStride / 4;
    for (int64_t sb = s0; sb < s1; sb += kWgStep) {
        for (int e = threadIdx.x; e < kWgStep * kF4Row; e += kWgWaves * 64) {
            const int r = e / kF4Row, c4 = e % kF4Row;
            const f4_t v = (sb + r < s1) ? *(const f4_t *)(stage + (sb + r) * kStageStride + 4 * c4)
                                         : f4_t{0.f, 0.f, 0.f, 0.f};
            *(f4_t *)(rows + r * kWgRow + 4 * c4) = v;
        }
        __syncthreads();
#pragma unroll
        for (int kk = 0; kk < kWgStep; kk += 4) {
            const float *rr = rows + (kk + (lane >> 4)) * kWgRow + (lane & 15);
#pragma unroll
            for (int i = 0; i < kWgTPW; ++i) {
                const int t = wave + kWgWaves * i;
                if (t < kWgTiles) {
                    const WgTile w = wg_tile(t);
                    acc[i] = __builtin_amdgcn_mfma_f32_16x16x4f32(rr[w.a_col], rr[w.b_col], acc[i], 0, 0, 0);
                }
            }
        }
        __syncthreads();
    }
    float *out = partials + (int64_t)blockIdx.x * kPartialFloats;
#pragma unroll
    for (int i = 0; i < kWgTPW; ++i) {
        const int t = wave + kWgWaves * i;
        if (t < kWgTiles) {
            const WgTile w = wg_tile(t);
#pragma unroll
            for (int r = 0; r < 4; ++r) out[w.out + (4 * (lane >> 4) + r) * w.ld + (lane & 15)] = acc[i][r];
        }
    }
}

// Sum the per-block partials in block order and add into the gradients.
__global__ __launch_bounds__(256) void k_wgrad_apply(const float *partials, int nblk, BackwardBufs bb)
{
    constexpr int P1 = 128 * 48, P2 = P1 + 128 * 128, P3 = P2 + 16 * 128, P4 = P3 + 128 * 16;
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    int src;
    float *dst;
    if (e < 128 * 39) {
        src = (e / 39) * 48 + e % 39;
        dst = bb.d_w0 + e;
    } else if (e < 128 * 39 + 128) {
        const int o = e - 128 * 39;
        src = o * 48 + 39;
        dst = bb.d_b0 + o;
    } else if (e < 128 * 39 + 128 + 128 * 128) {
        const int k = e - (128 * 39 + 128);
        src = P1 + k;
        dst = bb.d_w1 + k;
    } else if (e < 128 * 39 + 128 + 128 * 128 + 3 * 128) {
        const int k = e - (128 * 39 + 128 + 128 * 128);
        src = P2 + k;
        dst = bb.d_w2 + k;
    } else if (e < 128 * 39 + 128 + 128 * 128 + 3 * 128 + 128) {
        const int o = e - (128 * 39 + 128 + 128 * 128 + 3 * 128);
        src = P3 + o * 16 + 7;
        dst = bb.d_b1 + o;
    } else if (e < 128 * 39 + 128 + 128 * 128 + 3 * 128 + 128 + 3) {
        const int ch = e - (128 * 39 + 128 + 128 * 128 + 3 * 128 + 128);
        src = P4 + ch * 16 + 7;
        dst = bb.d_b2 + ch;
    } else {
        return;
    }
    float sum = 0.f;
    for (int blk = 0; blk < nblk; ++blk) sum += partials[(int64_t)blk * kPartialFloats + src];
    *dst += sum;
}

void launch_weight_grads(const RenderBufs &b, const BackwardBufs &bb, hipStream_t s)
{
    // sample range per block from the pass's maximum sample count
    const int64_t max_s = b.n * (int64_t)b.n_samples;
    const int64_t slab = ((max_s + kWgBlocks - 1) / kWgBlocks + kWgStep - 1) / kWgStep * kWgStep;
    hipLaunchKernelGGL(k_wgrad, dim3(kWgBlocks), dim3(kWgWaves * 64), 0, s, (const float *)b.stage, b.offsets + b.n,
                       bb.partials, slab);
    const int n_out = 128 * 39 + 128 + 128 * 128 + 3 * 128 + 128 + 3;
    hipLaunchKernelGGL(k_wgrad_apply, dim3((n_out + 255) / 256), dim3(256), 0, s, (const float *)bb.partials,
                       kWgBlocks, bb);
}

}  // namespace cic
