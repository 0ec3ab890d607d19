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
// Kernels (one backward pass over a chunk of rays, samples in brick order;
// the forward has already been recomputed into the workspace, with
// per-sample MLP vectors and ReLU sign masks staged):
//  - k_bwd_composite: one wavefront per ray walks its live samples from the
//    back, 64 at a time, with a reverse wavefront scan for R_k and D_k; it
//    writes dL/dc_k and dL/draw per sample.
//  - k_mlp_bwd: per 32-sample batch, the output-layer adjoint on the vector
//    ALUs, then W1^T and W0^T products on FP32 MFMA (transposed weight
//    fragments in LDS); hidden-layer gradients are staged for the weight
//    gradients and the 12 feature gradients written in brick order.
//  - k_fgrad_seg, k_fgrad_gather: the feature and raw-density gradients of
//    each brick segment summed per tile vertex on chip, then added to the
//    grids per vertex in a fixed order (no atomics).
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
            bb.rec_draw[r] = draw;   // added per brick segment with the feature gradients
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

__global__ __launch_bounds__(kBwdWaves * 64, 1) void k_mlp_bwd(GridK g, cic_mlp m, RenderBufs b, BackwardBufs bb)
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

    const BatchRange br = xcd_batches(nbatch, kBwdWaves, wave);
    for (int64_t bt = br.first; bt < br.end; bt += br.stride) {
        int64_t rec[kBNT];
        bool valid[kBNT];
        f4_t dp1[8][kBNT];
        uint32_t h1m[kBNT];   // ReLU mask of h1: bit 4t + r for row 16t + 4q + r
#pragma unroll
        for (int nt = 0; nt < kBNT; ++nt) {
            const int64_t s = bt * (16 * kBNT) + nt * 16 + j;
            valid[nt] = s < total;
            rec[nt] = valid[nt] ? (int64_t)b.perm[s] : 0;
            const uint32_t h2m = valid[nt] ? b.stage_mask[rec[nt] * 8 + 4 + q] : 0u;
            h1m[nt] = valid[nt] ? b.stage_mask[rec[nt] * 8 + q] : 0u;
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
                const f4_t wa = w2l[(q * 3 + 0) * 8 + t], wb = w2l[(q * 3 + 1) * 8 + t], wc = w2l[(q * 3 + 2) * 8 + t];
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const float v = fmaf(wa[r], dl[0], fmaf(wb[r], dl[1], wc[r] * dl[2]));
                    dp1[t][nt][r] = ((h2m >> (4 * t + r)) & 1u) ? v : 0.f;
                }
            }
            // dp1 itself is recomputed by the weight-gradient kernel
            if (valid[nt]) {
                float *wrow = b.stage + rec[nt] * kStageStride;
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
                for (int r = 0; r < 4; ++r) dp0[ti][nt][r] = ((h1m[nt] >> (4 * ti + r)) & 1u) ? dp0[ti][nt][r] : 0.f;
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
        // the 12 feature gradients of the sample at its position in brick order;
        // the brick-segment kernel accumulates them
#pragma unroll
        for (int nt = 0; nt < kBNT; ++nt) {
            const int64_t s = bt * (16 * kBNT) + nt * 16 + j;
            if (valid[nt] && q < 3) *(f4_t *)(bb.df_sorted + s * 12 + 4 * q) = df[nt];
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

// Feature and density gradients in two steps, without atomics on floats.
// The brick-ordered samples are cut into segments of at most kFgSeg samples
// of one brick (a brick crossed by many rays gets several segments, which
// keeps the workgroups' loads even).  k_fgrad_seg: one workgroup per
// segment stages its samples (voxel fractions and the 13 gradient channels:
// 12 features, raw density) in LDS, counting-sorts them by cell of the brick
// (two integer LDS atomics per sample), and then each thread sums, for its
// vertices of the brick's 9x9x9-vertex tile, the trilinear shares of the
// samples in the up-to-8 cells around the vertex, and stores the tile row
// into the segment's slot.  k_fgrad_gather: one workgroup per brick over the
// vertices it owns (its 8^3 lower corner block, and the grid's last vertex
// layer for the last brick of an axis); a vertex on a brick's lower face also
// lies in the lower neighbours' tiles, so each vertex adds the slots of every
// segment of the bricks containing it, in ascending brick and segment order,
// to the gradient grids.
constexpr int kTileV = kBrick + 1;
constexpr int kTileCh = 13;
constexpr int kTileFloats = kTileV * kTileV * kTileV * kTileCh;
constexpr int kCells = kBrick * kBrick * kBrick;
static_assert(kTileFloats == kFgTileFloats, "brick tile size");

// Exclusive scan of cnt[0..kCells) in place (256 threads, kCells = 2 x 256);
// cur receives a copy (the scatter's cursors).
__device__ void cell_scan(int *cnt, int *cur, int *tmp)
{
    const int t = threadIdx.x;
    const int a = cnt[2 * t], c = cnt[2 * t + 1];
    tmp[t] = a + c;
    __syncthreads();
    for (int d = 1; d < 256; d <<= 1) {
        const int v = t >= d ? tmp[t - d] : 0;
        __syncthreads();
        tmp[t] += v;
        __syncthreads();
    }
    const int excl = tmp[t] - (a + c);
    cnt[2 * t] = cur[2 * t] = excl;
    cnt[2 * t + 1] = cur[2 * t + 1] = excl + a;
}

__global__ __launch_bounds__(256) void k_fgrad_seg(GridK g, RenderBufs b, BackwardBufs bb)
{
    static_assert(kCells == 512, "cell_scan assumes 512 cells and 256 threads");
    __shared__ float sfr[3][kFgSeg];
    __shared__ float sv[kTileCh][kFgSeg];
    __shared__ uint16_t scell[kFgSeg];
    __shared__ uint16_t order[kFgSeg];
    __shared__ int cnt[kCells + 1], cur[kCells], tmp[256];
    const uint32_t k = blockIdx.x;
    if (k >= b.seg_off[b.n_bricks]) return;   // uniform per block
    // brick: the last index with seg_off[brick] <= k
    int64_t lo = 0, hi = b.n_bricks;
    while (hi - lo > 1) {
        const int64_t mid = (lo + hi) >> 1;
        if (b.seg_off[mid] <= k) lo = mid;
        else hi = mid;
    }
    const int64_t brick = lo;
    const uint32_t start = (brick == 0 ? 0u : b.brick_off[brick - 1]) + (k - b.seg_off[brick]) * (uint32_t)kFgSeg;
    const int n = (int)(min(b.brick_off[brick], start + (uint32_t)kFgSeg) - start);
    for (int c = threadIdx.x; c <= kCells; c += blockDim.x) cnt[c] = 0;
    __syncthreads();
    const int bz = (int)(brick % g.nb2), by = (int)((brick / g.nb2) % g.nb1), bx = (int)(brick / ((int64_t)g.nb2 * g.nb1));
    const int base[3] = {kBrick * bx, kBrick * by, kBrick * bz};
    for (int e = threadIdx.x; e < n; e += blockDim.x) {
        const uint32_t s = start + (uint32_t)e;
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
        const int cell = ((i0[0] - base[0]) * kBrick + (i0[1] - base[1])) * kBrick + (i0[2] - base[2]);
#pragma unroll
        for (int a = 0; a < 3; ++a) sfr[a][e] = fr[a];
        const float *df = bb.df_sorted + (int64_t)s * 12;
#pragma unroll
        for (int f = 0; f < 12; ++f) sv[f][e] = df[f];
        sv[12][e] = bb.rec_draw[rec];
        scell[e] = (uint16_t)cell;
        atomicAdd(&cnt[cell], 1);
    }
    __syncthreads();
    cell_scan(cnt, cur, tmp);
    if (threadIdx.x == 0) cnt[kCells] = n;
    __syncthreads();
    for (int e = threadIdx.x; e < n; e += blockDim.x) order[atomicAdd(&cur[scell[e]], 1)] = (uint16_t)e;
    __syncthreads();
    // each tile vertex sums the shares of the samples in its up-to-8 cells
    float *slot = bb.seg_tiles + (int64_t)k * kTileFloats;
    for (int vtx = threadIdx.x; vtx < kTileV * kTileV * kTileV; vtx += blockDim.x) {
        const int vz = vtx % kTileV, vy = (vtx / kTileV) % kTileV, vx = vtx / (kTileV * kTileV);
        float acc[kTileCh];
#pragma unroll
        for (int f = 0; f < kTileCh; ++f) acc[f] = 0.f;
        for (int cx = max(vx - 1, 0); cx <= min(vx, kBrick - 1); ++cx)
            for (int cy = max(vy - 1, 0); cy <= min(vy, kBrick - 1); ++cy)
                for (int cz = max(vz - 1, 0); cz <= min(vz, kBrick - 1); ++cz) {
                    const int c = (cx * kBrick + cy) * kBrick + cz;
                    for (int p = cnt[c]; p < cnt[c + 1]; ++p) {
                        const int e = order[p];
                        // the vertex is the cell's lower corner along an axis (weight 1 - fr) or its upper one (fr)
                        const float wx = cx == vx ? 1.f - sfr[0][e] : sfr[0][e];
                        const float wy = cy == vy ? 1.f - sfr[1][e] : sfr[1][e];
                        const float wz = cz == vz ? 1.f - sfr[2][e] : sfr[2][e];
                        const float w = wx * wy * wz;
#pragma unroll
                        for (int f = 0; f < kTileCh; ++f) acc[f] = fmaf(w, sv[f][e], acc[f]);
                    }
                }
#pragma unroll
        for (int f = 0; f < kTileCh; ++f) slot[vtx * kTileCh + f] = acc[f];
    }
}

// Bricks along one axis whose tiles contain vertex coordinate x (nb bricks).
__device__ __forceinline__ void tile_bricks(int x, int nb, int &lo, int &hi)
{
    hi = min(x / kBrick, nb - 1);
    lo = (x % kBrick == 0 && x > 0) ? x / kBrick - 1 : x / kBrick;
    lo = min(lo, hi);
}

__global__ __launch_bounds__(256) void k_fgrad_gather(GridK g, int nb0, RenderBufs b, BackwardBufs bb)
{
    const int64_t brick = blockIdx.x;
    const int nb1 = g.nb1, nb2 = g.nb2;
    const int bz = (int)(brick % nb2), by = (int)((brick / nb2) % nb1), bx = (int)(brick / ((int64_t)nb2 * nb1));
    // nothing to add unless this brick or a lower neighbour has samples (uniform per block)
    bool any = false;
#pragma unroll
    for (int c = 0; c < 8; ++c) {
        const int x = bx - ((c >> 2) & 1), y = by - ((c >> 1) & 1), z = bz - (c & 1);
        if (x >= 0 && y >= 0 && z >= 0) {
            const int64_t nbk = ((int64_t)x * nb1 + y) * nb2 + z;
            any = any || b.seg_off[nbk + 1] > b.seg_off[nbk];
        }
    }
    if (!any) return;
    const int rr[3] = {g.r0, g.r1, g.r2}, nbs[3] = {nb0, nb1, nb2}, bc[3] = {bx, by, bz};
    int lo[3], cnt[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        lo[a] = kBrick * bc[a];
        const int hi = bc[a] == nbs[a] - 1 ? rr[a] - 1 : lo[a] + kBrick - 1;
        cnt[a] = hi - lo[a] + 1;
    }
    const int n = cnt[0] * cnt[1] * cnt[2];
    for (int e = threadIdx.x; e < n; e += blockDim.x) {
        const int z = lo[2] + e % cnt[2], y = lo[1] + (e / cnt[2]) % cnt[1], x = lo[0] + e / (cnt[2] * cnt[1]);
        int xl, xh, yl, yh, zl, zh;
        tile_bricks(x, nb0, xl, xh);
        tile_bricks(y, nb1, yl, yh);
        tile_bricks(z, nb2, zl, zh);
        float acc[kTileCh];
#pragma unroll
        for (int f = 0; f < kTileCh; ++f) acc[f] = 0.f;
        bool hit = false;
        for (int cx = xl; cx <= xh; ++cx)
            for (int cy = yl; cy <= yh; ++cy)
                for (int cz = zl; cz <= zh; ++cz) {
                    const int64_t cb = ((int64_t)cx * nb1 + cy) * nb2 + cz;
                    const uint32_t k0 = b.seg_off[cb], k1 = b.seg_off[cb + 1];
                    const int loc = ((x - kBrick * cx) * kTileV + (y - kBrick * cy)) * kTileV + (z - kBrick * cz);
                    for (uint32_t k = k0; k < k1; ++k) {
                        hit = true;
                        const float *t = bb.seg_tiles + (int64_t)k * kTileFloats + loc * kTileCh;
#pragma unroll
                        for (int f = 0; f < kTileCh; ++f) acc[f] += t[f];
                    }
                }
        if (!hit) continue;
        const int64_t vi = vertex_index(g, x, y, z);
#pragma unroll
        for (int f = 0; f < 12; ++f) bb.d_features[vi * 12 + f] += acc[f];
        bb.d_density[vi] += acc[12];
    }
}

void launch_feature_grads_bricks(const GridK &g, const RenderBufs &b, const BackwardBufs &bb, hipStream_t s)
{
    if (b.n_bricks == 0) return;
    launch_brick_segments(b, kFgSeg, s);
    const int64_t max_seg = fg_max_segments(b.n_bricks, b.n * (int64_t)b.n_samples);
    hipLaunchKernelGGL(k_fgrad_seg, dim3((unsigned)max_seg), dim3(256), 0, s, g, b, bb);
    const int nb0 = (int)(b.n_bricks / ((int64_t)g.nb1 * g.nb2));
    hipLaunchKernelGGL(k_fgrad_gather, dim3((unsigned)b.n_bricks), dim3(256), 0, s, g, nb0, b, bb);
}

void launch_mlp_backward(const GridK &g, const cic_mlp &m, const RenderBufs &b, const BackwardBufs &bb, hipStream_t s)
{
    const int lds = kBLds * (int)sizeof(float);
    static bool attr_set = false;
    if (!attr_set) {
        (void)hipFuncSetAttribute((const void *)k_mlp_bwd, hipFuncAttributeMaxDynamicSharedMemorySize, lds);
        attr_set = true;
    }
    hipLaunchKernelGGL(k_mlp_bwd, dim3(num_cus_b()), dim3(kBwdWaves * 64), lds, s, g, m, b, bb);
}

// ---------------------------------------------------------------------------
// Weight gradients: sums over samples of outer products of staged vectors,
//   P0 = dp0^T [x|1|h1[0:8]]   (128 x 48: dW0 and, in column 39, db0)
//   P1 = dp1^T h1              (128 x 128: dW1)
//   P2 = dl^T h2               (16 x 128: dW2 in rows 0..2)
//   P3 = dp1^T [x|1][32:48]    (128 x 16: db1 in column 7)
//   P4 = dl^T [x|1][32:48]     (16 x 16: db2 in column 7)
// one fused pass: each block owns a contiguous range of samples, stages 16
// stored rows at a time in LDS, recomputes their dp1 there and runs all 105 output tiles on FP32 MFMA
// (K = samples), writing one partial per block; k_wgrad_apply adds the
// partials in block order (deterministic).
// ---------------------------------------------------------------------------
constexpr int kWgStep = 16;
// Padded LDS row (the stored row, then the recomputed dp1): an MFMA operand
// read takes 16 consecutive columns of 4 consecutive rows, so a row stride of
// 16 (mod 64) words puts the 64 lanes on 64 distinct banks.
constexpr int kWgRow = kStDP1 + 128 + 24;
static_assert(kWgRow % 64 == 16, "wgrad LDS row stride");
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

// Two 8-wavefront blocks per CU (four wavefronts per SIMD, at most 128 VGPRs,
// a few spilled): 1.37-1.39 ms per step against 1.42-1.43 ms with one block.
__global__ __launch_bounds__(kWgWaves * 64) __attribute__((amdgpu_waves_per_eu(4))) void k_wgrad(const float *stage, const uint32_t *total_p, float *partials,
                                               int64_t slab, const float *w2)
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
    // The rows of the next step are loaded into registers while this step's
    // MFMAs run, then written to LDS (one step of software pipelining).
    constexpr int kThreads = kWgWaves * 64;
    static_assert(kThreads % 128 == 0, "dp1 fill: whole rows per pass");
    // dp1 fill: thread t owns hidden unit t % 128 of rows t / 128, t / 128 +
    // kThreads / 128, ...; the MLP backward's expression and mask, so the
    // same bits (computing it while storing the rows, from a second load of
    // the logit gradient, measured slower: 1.58 against 1.41 ms per step)
    const int hu = threadIdx.x % 128;
    const float w2a = w2[hu], w2b = w2[128 + hu], w2c = w2[256 + hu];
    constexpr int kPer = (kWgStep * kF4Row + kThreads - 1) / kThreads;
    f4_t pre[kPer];
    auto load_step = [&](int64_t sb) {
#pragma unroll
        for (int i = 0; i < kPer; ++i) {
            const int e = threadIdx.x + i * kThreads;
            const int r = e / kF4Row, c4 = e % kF4Row;
            pre[i] = (e < kWgStep * kF4Row && sb + r < s1) ? *(const f4_t *)(stage + (sb + r) * kStageStride + 4 * c4)
                                                            : f4_t{0.f, 0.f, 0.f, 0.f};
        }
    };
    load_step(s0);
    for (int64_t sb = s0; sb < s1; sb += kWgStep) {
#pragma unroll
        for (int i = 0; i < kPer; ++i) {
            const int e = threadIdx.x + i * kThreads;
            if (e < kWgStep * kF4Row) *(f4_t *)(rows + (e / kF4Row) * kWgRow + 4 * (e % kF4Row)) = pre[i];
        }
        __syncthreads();
        for (int r = threadIdx.x / 128; r < kWgStep; r += kThreads / 128) {
            float *row = rows + r * kWgRow;
            const float v = fmaf(w2a, row[kStDL], fmaf(w2b, row[kStDL + 1], w2c * row[kStDL + 2]));
            row[kStDP1 + hu] = row[kStH2 + hu] > 0.f ? v : 0.f;
        }
        __syncthreads();
        if (sb + kWgStep < s1) load_step(sb + kWgStep);
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
// Sum of the per-block partials of every weight-gradient entry, added to the
// gradient.  A block takes 64 consecutive outputs; its 16 groups of 64
// threads sum contiguous ranges of blocks (coalesced over the outputs), and
// the group sums are added in group order: a fixed order, so the result is
// deterministic.
constexpr int kApplyOut = 64, kApplyGroups = 16;

__device__ __forceinline__ bool wgrad_entry(int e, int &src, float *&dst, const BackwardBufs &bb)
{
    constexpr int P1 = 128 * 48, P2 = P1 + 128 * 128, P3 = P2 + 16 * 128, P4 = P3 + 128 * 16;
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
        return false;
    }
    return true;
}

__global__ __launch_bounds__(kApplyOut * kApplyGroups) void k_wgrad_apply(const float *partials, int nblk,
                                                                          BackwardBufs bb)
{
    __shared__ float part[kApplyGroups][kApplyOut];
    const int o = threadIdx.x % kApplyOut, grp = threadIdx.x / kApplyOut;
    const int e = blockIdx.x * kApplyOut + o;
    int src = 0;
    float *dst = nullptr;
    const bool ok = wgrad_entry(e, src, dst, bb);
    const int per = (nblk + kApplyGroups - 1) / kApplyGroups;
    const int b0 = grp * per, b1 = min(nblk, b0 + per);
    float sum = 0.f;
    if (ok)
        for (int blk = b0; blk < b1; ++blk) sum += partials[(int64_t)blk * kPartialFloats + src];
    part[grp][o] = sum;
    __syncthreads();
    if (grp == 0 && ok) {
        float t = 0.f;
#pragma unroll
        for (int k = 0; k < kApplyGroups; ++k) t += part[k][o];
        *dst += t;
    }
}

void launch_weight_grads(const cic_mlp &m, const RenderBufs &b, const BackwardBufs &bb, hipStream_t s)
{
    // sample range per block from the pass's maximum sample count
    const int64_t max_s = b.n * (int64_t)b.n_samples;
    const int64_t slab = ((max_s + kWgBlocks - 1) / kWgBlocks + kWgStep - 1) / kWgStep * kWgStep;
    hipLaunchKernelGGL(k_wgrad, dim3(kWgBlocks), dim3(kWgWaves * 64), 0, s, (const float *)b.stage, b.offsets + b.n,
                       bb.partials, slab, m.w2);
    const int n_out = 128 * 39 + 128 + 128 * 128 + 3 * 128 + 128 + 3;
    hipLaunchKernelGGL(k_wgrad_apply, dim3((n_out + kApplyOut - 1) / kApplyOut), dim3(kApplyOut * kApplyGroups), 0, s,
                       (const float *)bb.partials, kWgBlocks, bb);
}

}  // namespace cic
