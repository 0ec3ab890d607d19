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
// Kernels (one backward pass over a chunk of rays, after the march and the
// bucketing):
//  - k_mlp_adjoint: per 16-sample batch (ray order), the forward recomputed
//    on chip (its colours c_k kept for the next kernel), the MLP backward
//    from dL/dc_k = w_k dL/dC on FP32 MFMA (the 12 feature gradients written
//    per sample) and the weight-gradient outer products accumulated per
//    workgroup; k_wgrad_apply adds the workgroups' partials in a fixed order
//    (deterministic).
//  - k_bwd_composite: one wavefront per ray walks its live samples from the
//    back, 64 at a time, with a reverse wavefront scan for R_k and D_k; it
//    writes dL/draw per sample.
//  - k_fgrad_seg, k_fgrad_gather: the feature and raw-density gradients of
//    each brick segment summed per tile vertex on chip, then added to the
//    grids per vertex in a fixed order (no atomics).
#include <algorithm>

#include "mlp_common.h"

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
        const float *df = bb.rec_df + (int64_t)rec * 12;
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
    launch_brick_segments(b, kFgSeg, false, s);
    const int64_t max_seg = fg_max_segments(b.n_bricks, b.n * (int64_t)b.n_samples);
    hipLaunchKernelGGL(k_fgrad_seg, dim3((unsigned)max_seg), dim3(256), 0, s, g, b, bb);
    const int nb0 = (int)(b.n_bricks / ((int64_t)g.nb1 * g.nb2));
    hipLaunchKernelGGL(k_fgrad_gather, dim3((unsigned)b.n_bricks), dim3(256), 0, s, g, nb0, b, bb);
}

// ---------------------------------------------------------------------------
// MLP adjoint, fused: per batch of 16 live samples (ray order) a wavefront
// recomputes the forward (full 40-wide layer-0 input, FP32 MFMA), forms the
// output-logit gradient from dL/dc_k = w_k g, and runs the backward: dp1 =
// [h2 > 0] (W2^T dlogit) on the vector ALUs, dh1 = W1^T dp1 and the feature
// gradient (W0^T dp0)[0:12] on FP32 MFMA, dp0 = [h1 > 0] dh1.  Nothing of
// it leaves the chip except the 12 feature gradients per sample (for the
// brick-segment tiles).  Ray order fixes which samples each workgroup sums,
// so the MLP gradients are the same bits on every call (in brick order the
// bucketing's atomic cursors would decide it).  The weight gradients are
// sums over samples of outer products,
//   P0 = dp0^T [x|1|h1[0:8]]   (128 x 48: dW0 and, in column 39, db0)
//   P1 = dp1^T h1              (128 x 128: dW1)
//   P2 = dl^T h2               (16 x 128: dW2 in rows 0..2)
//   P3 = dp1^T [x|1][32:48]    (128 x 16: db1 in column 7)
//   P4 = dl^T [x|1][32:48]     (16 x 16: db2 in column 7)
// on FP32 MFMA with the samples as the reduction index.  Each wavefront
// owns some of the 105 16x16 output tiles and keeps them in registers for
// the workgroup's lifetime; the workgroup's wavefronts take turns writing
// their batch's per-sample rows [x|1, h1, h2, dp0, dlogit, dp1] into one LDS
// row block, and after each write every wavefront adds that block's 16
// samples to its tiles.  One partial per workgroup, summed in a fixed order
// by k_wgrad_apply (deterministic).  LDS: the forward's weight fragments
// (92.6 KB, W1 padded for its transposed reads), W0^T fragments for the
// feature gradients (8 KB), the row block (37.9 KB).
// ---------------------------------------------------------------------------
constexpr int kWgTiles = 24 + 64 + 8 + 8 + 1;
constexpr int kAdjWaves = 8;
constexpr int kAdjTPW = (kWgTiles + kAdjWaves - 1) / kAdjWaves;
// Row of the LDS block: the staged vectors at the offsets below, padded so
// that an MFMA operand read (16 consecutive columns of 4 consecutive rows)
// puts the 64 lanes on 64 distinct banks (row stride 16 mod 64 words).
constexpr int kAdjRow = kStDP1 + 128 + 24;
static_assert(kAdjRow % 64 == 16, "adjoint LDS row stride");
typedef F32Lds<true> AdjLds;                              // forward weights, W1 padded
constexpr int kAOffW0T = AdjLds::kSize;                  // [c4 8][lane 64][4]
constexpr int kAOffRows = kAOffW0T + 8 * 64 * 4;        // [16][kAdjRow]
constexpr int kALds = kAOffRows + 16 * kAdjRow;

struct WgTile {
    int a_col, b_col, out;   // row columns of A and B, offset of the 16x16 tile in the partial
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

// Two wavefronts per SIMD: a wavefront holds its batch's h1, h2, dp0, dp1
// (128 VGPRs) and its output tiles (56) between its turns at the row block.
__global__ __launch_bounds__(kAdjWaves * 64) __attribute__((amdgpu_waves_per_eu(2, 2))) void k_mlp_adjoint(
    GridK g, cic_mlp m, RenderBufs b, BackwardBufs bb)
{
    extern __shared__ __attribute__((aligned(16))) float lds[];
    stage_weights_f32<true>(m, lds);
    for (int i = threadIdx.x; i < 8 * 64 * 4; i += blockDim.x) {
        const int rr = i & 3, l = (i >> 2) & 63, c4 = i >> 8;
        const int col = l & 15;
        lds[kAOffW0T + i] = col < 12 ? m.w0[(16 * c4 + 4 * (l >> 4) + rr) * 39 + col] : 0.f;
    }
    __syncthreads();
    const int lane = lane_id(), q = lane >> 4, j = lane & 15;
    const int wave = threadIdx.x / 64;
    const f2_t *w0f = (const f2_t *)(lds + AdjLds::kW0);
    const f4_t *w2l = (const f4_t *)(lds + AdjLds::kW2);
    const f4_t *w0t = (const f4_t *)(lds + kAOffW0T);
    // this lane's W1 fragment in block 0 (block k at + k * kW1Block floats)
    const float *w1f = lds + AdjLds::w1(0, lane);
    float *rows = lds + kAOffRows;

    // this workgroup's batches: the XCD's contiguous range, interleaved over
    // its workgroups and wavefronts; every wavefront runs the same number of
    // steps (the row-block turns are workgroup-wide)
    const int64_t total = (int64_t)b.offsets[b.n];
    const int64_t nbatch = (total + 15) / 16;
    const int xcd = blockIdx.x % kXcds, slot = blockIdx.x / kXcds, nslots = gridDim.x / kXcds;
    const int64_t per = (nbatch + kXcds - 1) / kXcds;
    const int64_t lo = xcd * per, hi = lo + per < nbatch ? lo + per : nbatch;
    const int64_t first = lo + (int64_t)slot * kAdjWaves, stride = (int64_t)nslots * kAdjWaves;
    const int64_t steps = hi > first ? (hi - first + stride - 1) / stride : 0;

    f4_t acc[kAdjTPW];
#pragma unroll
    for (int i = 0; i < kAdjTPW; ++i) acc[i] = f4_t{0.f, 0.f, 0.f, 0.f};

    for (int64_t st = 0; st < steps; ++st) {
        const int64_t bt = first + st * stride + wave;
        const int64_t s = bt * 16 + j;
        const bool valid = bt < hi && s < total;
        // ray order; a lane past the end works on sample 0 (in-bounds inputs,
        // no branches around the loads) with a zero logit gradient, so it
        // adds nothing to the weight gradients and stores nothing
        const uint32_t rec = valid ? (uint32_t)s : 0u;
        float x[10];
        sample_inputs<float, true>(g, b, rec, q, x);
        // forward: layer 0 (40 -> 128), the same products in the same order
        // as the forward kernel's full-input path
        f4_t h1[8];
#pragma unroll
        for (int t = 0; t < 8; ++t) h1[t] = *(const f4_t *)(lds + AdjLds::kB0 + 16 * t + 4 * q);
#pragma unroll
        for (int c2 = 0; c2 < 5; ++c2) {
            f2_t a[8];
#pragma unroll
            for (int t = 0; t < 8; ++t) a[t] = w0f[(t * 5 + c2) * 64 + lane];
#pragma unroll
            for (int e = 0; e < 2; ++e)
#pragma unroll
                for (int t = 0; t < 8; ++t)
                    h1[t] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[t][e], x[2 * c2 + e], h1[t], 0, 0, 0);
            __builtin_amdgcn_sched_barrier(0);
        }
#pragma unroll
        for (int t = 0; t < 8; ++t)
#pragma unroll
            for (int r = 0; r < 4; ++r) h1[t][r] = relu_bits(h1[t][r]);
        // layer 1 (128 -> 128)
        f4_t h2[8];
#pragma unroll
        for (int t = 0; t < 8; ++t) h2[t] = *(const f4_t *)(lds + AdjLds::kB1 + 16 * t + 4 * q);
        {
            f4_t a[4], an[4];
#pragma unroll
            for (int tt = 0; tt < 4; ++tt) a[tt] = *(const f4_t *)(w1f + (tt * 8 + 0) * AdjLds::kW1Block);
#pragma unroll
            for (int c4 = 0; c4 < 8; ++c4) {
#pragma unroll
                for (int tg = 0; tg < 2; ++tg) {
                    const int step = c4 * 2 + tg, nx = step + 1 < 16 ? step + 1 : step;
                    const int nc4 = nx >> 1, ntg = nx & 1;
#pragma unroll
                    for (int tt = 0; tt < 4; ++tt)
                        an[tt] = *(const f4_t *)(w1f + ((4 * ntg + tt) * 8 + nc4) * AdjLds::kW1Block);
#pragma unroll
                    for (int rr = 0; rr < 4; ++rr)
#pragma unroll
                        for (int tt = 0; tt < 4; ++tt)
                            h2[4 * tg + tt] =
                                __builtin_amdgcn_mfma_f32_16x16x4f32(a[tt][rr], h1[c4][rr], h2[4 * tg + tt], 0, 0, 0);
#pragma unroll
                    for (int tt = 0; tt < 4; ++tt) a[tt] = an[tt];
                    __builtin_amdgcn_sched_barrier(0);
                }
            }
        }
#pragma unroll
        for (int t = 0; t < 8; ++t)
#pragma unroll
            for (int r = 0; r < 4; ++r) h2[t][r] = relu_bits(h2[t][r]);
        // output layer on the vector ALUs (every lane group ends with the
        // three sums), sigmoid, and the logit gradient from dL/dc
        float p0 = 0.f, p1 = 0.f, p2 = 0.f;
#pragma unroll
        for (int t = 0; t < 8; ++t) {
            const f4_t wa = w2l[(q * 3 + 0) * 8 + t], wb = w2l[(q * 3 + 1) * 8 + t], wc = w2l[(q * 3 + 2) * 8 + t];
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                p0 = fmaf(wa[r], h2[t][r], p0);
                p1 = fmaf(wb[r], h2[t][r], p1);
                p2 = fmaf(wc[r], h2[t][r], p2);
            }
        }
        p0 += __shfl_xor(p0, 16, kWave);
        p1 += __shfl_xor(p1, 16, kWave);
        p2 += __shfl_xor(p2, 16, kWave);
        p0 += __shfl_xor(p0, 32, kWave);
        p1 += __shfl_xor(p1, 32, kWave);
        p2 += __shfl_xor(p2, 32, kWave);
        // dL/dc_k = w_k g (g = dL/dC of the sample's ray); the colour is kept
        // for the compositing adjoint, which runs next
        float dl[3];
        {
            const float pp[3] = {p0, p1, p2};
            const float w = b.rec_w[rec];
            const uint32_t ray = b.rec_ray[rec];
#pragma unroll
            for (int ch = 0; ch < 3; ++ch) {
                const float c = sigmoid_hw(pp[ch] + lds[AdjLds::kB2 + ch]);
                const float dc = valid ? w * bb.d_rgb[3 * (int64_t)ray + ch] : 0.f;
                dl[ch] = dc * c * (1.f - c);
                if (valid && q == ch) b.rec_c[3 * (int64_t)rec + ch] = c;
            }
        }
        // dp1 = [h2 > 0] (W2^T dl), for output tile t
        auto dp1_tile = [&](int t) {
            const f4_t wa = w2l[(q * 3 + 0) * 8 + t], wb = w2l[(q * 3 + 1) * 8 + t], wc = w2l[(q * 3 + 2) * 8 + t];
            f4_t v;
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const float u = fmaf(wa[r], dl[0], fmaf(wb[r], dl[1], wc[r] * dl[2]));
                v[r] = h2[t][r] > 0.f ? u : 0.f;
            }
            return v;
        };
        // dh1 = W1^T dp1 (A fragments of W1^T read from the forward's W1
        // layout), dp0 = [h1 > 0] dh1
        f4_t dp0[8];
#pragma unroll
        for (int ti = 0; ti < 8; ++ti) dp0[ti] = f4_t{0.f, 0.f, 0.f, 0.f};
        // kept in registers through the weight-gradient turns below (32 more
        // live registers, some spilled, against recomputing it, W2 reads from
        // LDS included, inside the writing wavefront's turn, where every other
        // wavefront waits: fused adjoint 2.91 -> 2.64 ms per 8192-ray step)
        f4_t dp1[8];
#pragma unroll
        for (int t = 0; t < 8; ++t) dp1[t] = dp1_tile(t);
        {
            // lane l needs W1[16 c4 + 4 (l / 16) + rr][16 ti + l % 16]: float
            // l % 4 of lane 16 g + 4 (l / 16) + rr of block (c4, ti), g =
            // (l % 16) / 4; the next (ti, c4) step's four values are read
            // while this step's MFMAs run
            const float *w1l = lds + AdjLds::w1(0, 16 * ((lane & 15) >> 2) + 4 * (lane >> 4)) + (lane & 3);
            float a[4], an[4];
#pragma unroll
            for (int rr = 0; rr < 4; ++rr) a[rr] = w1l[rr * 4];
#pragma unroll
            for (int idx = 0; idx < 64; ++idx) {
                const int ti = idx >> 3, c4 = idx & 7;
                const int nx = idx + 1 < 64 ? idx + 1 : idx, nti = nx >> 3, nc4 = nx & 7;
#pragma unroll
                for (int rr = 0; rr < 4; ++rr) an[rr] = w1l[(nc4 * 8 + nti) * AdjLds::kW1Block + rr * 4];
#pragma unroll
                for (int rr = 0; rr < 4; ++rr)
                    dp0[ti] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[rr], dp1[c4][rr], dp0[ti], 0, 0, 0);
#pragma unroll
                for (int rr = 0; rr < 4; ++rr) a[rr] = an[rr];
                __builtin_amdgcn_sched_barrier(0);
            }
        }
#pragma unroll
        for (int ti = 0; ti < 8; ++ti)
#pragma unroll
            for (int r = 0; r < 4; ++r) dp0[ti][r] = h1[ti][r] > 0.f ? dp0[ti][r] : 0.f;
        // feature gradient (W0^T dp0)[0:12] of the sample (ray order)
        {
            f4_t df = f4_t{0.f, 0.f, 0.f, 0.f};
#pragma unroll
            for (int c4 = 0; c4 < 8; ++c4) {
                const f4_t a = w0t[c4 * 64 + lane];
#pragma unroll
                for (int rr = 0; rr < 4; ++rr) df = __builtin_amdgcn_mfma_f32_16x16x4f32(a[rr], dp0[c4][rr], df, 0, 0, 0);
            }
            if (valid && q < 3) *(f4_t *)(bb.rec_df + (int64_t)rec * 12 + 4 * q) = df;
        }
        // weight gradients: the wavefronts take turns at the row block
        for (int turn = 0; turn < kAdjWaves; ++turn) {
            __syncthreads();   // the previous block is consumed
            if (wave == turn) {
                float *row = rows + j * kAdjRow;
#pragma unroll
                for (int c = 0; c < 10; ++c) {
                    const int src = l0_input(c, q);
                    row[kStX + (src >= 0 ? src : 39)] = src >= 0 ? x[c] : 1.0f;
                }
#pragma unroll
                for (int t = 0; t < 8; ++t) {
                    *(f4_t *)(row + kStH1 + 16 * t + 4 * q) = h1[t];
                    *(f4_t *)(row + kStH2 + 16 * t + 4 * q) = h2[t];
                    *(f4_t *)(row + kStDP0 + 16 * t + 4 * q) = dp0[t];
                    *(f4_t *)(row + kStDP1 + 16 * t + 4 * q) = dp1[t];
                }
                *(f4_t *)(row + kStDL + 4 * q) = q == 0 ? f4_t{dl[0], dl[1], dl[2], 0.f} : f4_t{0.f, 0.f, 0.f, 0.f};
            }
            __syncthreads();
            // per owned tile, the block's 16 samples in four k-steps (one
            // address pair per tile, the k-step offsets immediate); the
            // compiler may start the next tiles' operand reads during these
            // MFMAs (with a scheduling barrier per tile the adjoint kernel
            // took 3.02 against 2.94 ms per 8192-ray step)
            const float *rl = rows + (lane >> 4) * kAdjRow + (lane & 15);
#pragma unroll
            for (int i = 0; i < kAdjTPW; ++i) {
                const int t = wave + kAdjWaves * i;
                if (t < kWgTiles) {
                    const WgTile w = wg_tile(t);
                    const float *pa = rl + w.a_col, *pb = rl + w.b_col;
#pragma unroll
                    for (int kk = 0; kk < 16; kk += 4)
                        acc[i] = __builtin_amdgcn_mfma_f32_16x16x4f32(pa[kk * kAdjRow], pb[kk * kAdjRow], acc[i], 0, 0,
                                                                      0);
                }
            }
        }
    }
    float *out = bb.partials + (int64_t)blockIdx.x * kPartialFloats;
#pragma unroll
    for (int i = 0; i < kAdjTPW; ++i) {
        const int t = wave + kAdjWaves * i;
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

void launch_mlp_adjoint(const GridK &g, const cic_mlp &m, const RenderBufs &b, const BackwardBufs &bb, hipStream_t s)
{
    const int lds = kALds * (int)sizeof(float);
    static bool attr_set = false;
    if (!attr_set) {
        (void)hipFuncSetAttribute((const void *)k_mlp_adjoint, hipFuncAttributeMaxDynamicSharedMemorySize, lds);
        attr_set = true;
    }
    const int nblk = std::min(num_cus_b(), kWgBlocks);
    hipLaunchKernelGGL(k_mlp_adjoint, dim3(nblk), dim3(kAdjWaves * 64), lds, s, g, m, b, bb);
    const int n_out = 128 * 39 + 128 + 128 * 128 + 3 * 128 + 128 + 3;
    hipLaunchKernelGGL(k_wgrad_apply, dim3((n_out + kApplyOut - 1) / kApplyOut), dim3(kApplyOut * kApplyGroups), 0, s,
                       (const float *)bb.partials, nblk, bb);
}

}  // namespace cic
