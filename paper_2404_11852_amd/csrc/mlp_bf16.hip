// Feature Gathering + Feature Computation (Sec. II-B) with the MLP in BF16
// on MFMA (FP32 accumulation), in ray order or, on dense grids, in voxel
// order from LDS-staged bricks (Sec. IV-A).
#include "mlp_common.h"

namespace cic {

// BF16 compute: lane group q's seven view-encoding inputs of every ray with
// live samples, rounded to BF16 (the rounding the MLP kernel applies to its
// inputs) and packed as 8 BF16 (last slot 0) into words 4q..4q+3 of the ray.
__global__ __launch_bounds__(256) void k_ray_encode_bf16(RenderBufs b)
{
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t ray = t >> 2;
    const int q = (int)(t & 3);
    if (ray >= b.n || b.count[ray] == 0) return;
    float d[3], x[7];
#pragma unroll
    for (int a = 0; a < 3; ++a) d[a] = b.rays_d[3 * ray + a];
    encode_group(d, q, x);
    typedef __bf16 bf8v_t __attribute__((ext_vector_type(8)));
    bf8v_t v;
#pragma unroll
    for (int e = 0; e < 7; ++e) v[e] = (__bf16)x[e];
    v[7] = (__bf16)1.0f;   // the constant input of layer 0's bias
    typedef uint32_t u4_t __attribute__((ext_vector_type(4)));
    *(u4_t *)(b.enc + ray * 16 + 4 * q) = __builtin_bit_cast(u4_t, v);
}

void launch_ray_encode_bf16(const RenderBufs &b, hipStream_t s)
{
    if (b.n == 0) return;
    const int64_t threads = 4 * b.n;
    hipLaunchKernelGGL(k_ray_encode_bf16, dim3((unsigned)((threads + 255) / 256)), dim3(256), 0, s, b);
}

// ---------------------------------------------------------------------------
// Voxel order with LDS-staged bricks (the memory-centric rendering of Sec.
// IV-A): workgroups claim segments of up to kTileSeg samples of one brick of
// 8^3 voxels, stage the brick's 9^3 vertices x 12 feature channels in LDS
// (44 KB as float32) together with the segment's per-sample records (record
// index, ray, voxel fractions and cell within the brick, 24 B per sample),
// and then run the MLP batches from LDS.  Each feature vertex is read from
// the grid once per segment instead of by every sample near it, and the
// dependent loads that locate a sample (its record, its ray, the ray's
// origin and direction) are issued by the whole workgroup at once.
// ---------------------------------------------------------------------------
// Launch shape (measured on the 8-view workload, MLP stage): a BF16 MFMA does
// a 16-sample tile's layer in 1/16 of the FP32 time, so each batch carries
// little MFMA work against its dependent gather loads and its weight reads
// from LDS; 16 wavefronts per CU (a 128-VGPR budget each) with two tiles per
// batch hide the loads best and read each weight fragment for 32 samples
// (43.3 ms; 4 waves x 3 workgroups x 2 tiles 56.6 ms, 16 x 1 x 1 tile 44.4 ms;
// later, with the layers converted pair by pair: 3 tiles x 12 waves 23.95 and
// 4 tiles x 8 waves 25.2 against 23.54 ms).
#ifndef CIC_BF_NT
#define CIC_BF_NT 2
#endif

#ifndef CIC_BF_WAVES
#define CIC_BF_WAVES 16
#endif
#ifndef CIC_BF_WGS
#define CIC_BF_WGS 1
#endif
constexpr int kBfWaves = CIC_BF_WAVES;   // wavefronts per workgroup
constexpr int kBfWgs = CIC_BF_WGS;       // workgroups per CU (each holds its own 53 KB of LDS weights)
constexpr int kBfNT = CIC_BF_NT;         // 16-sample tiles per wavefront batch
constexpr int kBfBatch = 16 * kBfNT;
constexpr int kTileThreads = kBfWaves * 64;   // threads of a workgroup of the LDS-tile kernels

constexpr int kFTileV = kBrick + 1;
// Brick tile: channel ch of vertex (lx, ly, lz) at
// ch * kFTileS + lx * kFTileSX + ly * kFTileSY + lz * kFTileSZ.  One gather
// instruction reads channel 3q + c of the 16 samples' corner for the four
// lane groups q; the samples of a batch lie along one or two rays through
// the brick, so their cells are near neighbours.  The strides are chosen for
// few LDS bank collisions among those 64 words (64 banks): the channel
// stride puts the lane groups 16 banks apart, so two cells collide when
// their offsets differ by a multiple of 16 words.  Among cell steps of at
// most 2 per axis, 10 do so with the dense x stride of 81 (+-(1, 0, -1) among
// them: 80 words) and 6 with the x stride of 102 (+-(1, 1, 1): 112 words,
// and +-(0, 2, -2) as before).  Estimated on
// voxel-ordered samples of an 800x800 view: 1.35 distinct words per bank per
// instruction against 1.82 for the dense 9 x 81 x 752 layout; the 8-view
// pass measured 0.5-1.2% faster over three runs (bank conflicts are not what
// bounds the batches).
#ifndef CIC_TILE_SZ
#define CIC_TILE_SZ 1
#endif
#ifndef CIC_TILE_SY
#define CIC_TILE_SY 9
#endif
#ifndef CIC_TILE_SX
#define CIC_TILE_SX 102
#endif
#ifndef CIC_TILE_CS
#define CIC_TILE_CS 912
#endif
constexpr int kFTileSZ = CIC_TILE_SZ, kFTileSY = CIC_TILE_SY, kFTileSX = CIC_TILE_SX, kFTileS = CIC_TILE_CS;
constexpr int kFTileMax = 11 * kFTileS + (kFTileV - 1) * (kFTileSX + kFTileSY + kFTileSZ);   // largest index
constexpr int kFTileFloats = (kFTileMax + 4) & ~3;
constexpr bool tile_layout_injective()
{
    bool used[kFTileFloats] = {};
    for (int ch = 0; ch < 12; ++ch)
        for (int x = 0; x < kFTileV; ++x)
            for (int y = 0; y < kFTileV; ++y)
                for (int z = 0; z < kFTileV; ++z) {
                    const int i = ch * kFTileS + x * kFTileSX + y * kFTileSY + z * kFTileSZ;
                    if (used[i]) return false;
                    used[i] = true;
                }
    return true;
}
static_assert(tile_layout_injective(), "brick tile layout puts two values in one word");
// Segment records in LDS (structure of arrays, kTileSeg entries each):
// record index, ray, three voxel fractions, packed cell (lx | ly << 4 | lz << 8).
constexpr int kSegWords = 6 * kTileSeg;

// origin vertex of a brick (kept in registers by the callers)
struct BrickBase {
    int x, y, z;
};
__device__ __forceinline__ BrickBase brick_base(const GridK &g, int64_t brick)
{
    const int bz = (int)(brick % g.nb2), by = (int)((brick / g.nb2) % g.nb1);
    const int bx = (int)(brick / ((int64_t)g.nb2 * g.nb1));
    return BrickBase{kBrick * bx, kBrick * by, kBrick * bz};
}

template <typename T>
__device__ void load_feature_tile(const GridK &g, const BrickBase base, float *tile)
{
    const T *feat = (const T *)g.features;
    for (int e = threadIdx.x; e < kFTileV * kFTileV * kFTileV * 3; e += blockDim.x) {
        const int vtx = e / 3, part = e - 3 * vtx;
        const int lz = vtx % kFTileV, ly = (vtx / kFTileV) % kFTileV, lx = vtx / (kFTileV * kFTileV);
        const int vx = base.x + lx, vy = base.y + ly, vz = base.z + lz;
        const int tv = lx * kFTileSX + ly * kFTileSY + lz * kFTileSZ;
        f4_t v = f4_t{0.f, 0.f, 0.f, 0.f};
        if (vx < g.r0 && vy < g.r1 && vz < g.r2) {
            const int64_t off = vertex_index(g, vx, vy, vz) * 12 + 4 * part;
#pragma unroll
            for (int c = 0; c < 4; ++c) v[c] = ldv(feat, off + c);
        }
#pragma unroll
        for (int c = 0; c < 4; ++c) tile[(4 * part + c) * kFTileS + tv] = v[c];
    }
}

// Features 3q..3q+2 of a sample in cell (lx, ly, lz) of the staged brick
// (same interpolation order as the gather from the grid).
__device__ __forceinline__ void tile_gather3(const float *tile, int lx, int ly, int lz, const float fr[3], int q,
                                             float x[3])
{
    const int sx = kFTileSX, sy = kFTileSY, sz = kFTileSZ;
    const float *t = tile + lx * kFTileSX + ly * kFTileSY + lz * kFTileSZ + 3 * q * kFTileS;
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        const float *u = t + c * kFTileS;
        const float v000 = u[0], v001 = u[sz], v010 = u[sy], v011 = u[sy + sz];
        const float v100 = u[sx], v101 = u[sx + sz], v110 = u[sx + sy], v111 = u[sx + sy + sz];
        const float c00 = lerpf(v000, v001, fr[2]), c01 = lerpf(v010, v011, fr[2]);
        const float c10 = lerpf(v100, v101, fr[2]), c11 = lerpf(v110, v111, fr[2]);
        const float c0 = lerpf(c00, c01, fr[1]), c1 = lerpf(c10, c11, fr[1]);
        x[c] = lerpf(c0, c1, fr[0]);
    }
}

// The segment's per-sample records into LDS (every thread of the workgroup;
// same voxel computation as the march, so the cell and fractions are the
// ones the gather from the grid would use).
__device__ void stage_segment(const GridK &g, const RenderBufs &b, uint32_t start, int n, const BrickBase base,
                              uint32_t *seg)
{
    for (int e = threadIdx.x; e < n; e += blockDim.x) {
        const uint32_t rec = b.perm[start + e];
        SampleRay r;
        load_sample_ray(b, b.rec_ray[rec], b.rec_k[rec], r);
        int i0[3];
        float fr[3], tk;
        sample_voxel(r.o, r.d, r.tn, r.delta, r.k, g, i0, fr, tk);
        seg[e] = rec;
        seg[kTileSeg + e] = r.ray;
        seg[2 * kTileSeg + e] = __float_as_uint(fr[0]);
        seg[3 * kTileSeg + e] = __float_as_uint(fr[1]);
        seg[4 * kTileSeg + e] = __float_as_uint(fr[2]);
        seg[5 * kTileSeg + e] =
            (uint32_t)(i0[0] - base.x) | ((uint32_t)(i0[1] - base.y) << 4) | ((uint32_t)(i0[2] - base.z) << 8);
    }
}

// Claim the next segment (up to kTileSeg samples of one brick) for this
// workgroup.  The segment list is split into kXcds contiguous ranges, one
// per XCD, each drained through its own counter: the workgroups sharing an
// L2 then work through neighbouring bricks (and the rays crossing them)
// instead of the whole chip's in-flight window.  Thread 0 claims the
// segment, finds its brick in the segment table and publishes it in LDS
// (a binary search over the segment offsets per claim measured 1.5% slower
// for the whole stage; claiming the next segment while the current one's
// batches run, with batches handed out through an LDS counter, measured the
// same as this); returns false once this XCD's range is exhausted (every
// workgroup of the XCD then ends).  Large bricks are shared by several
// workgroups, each staging the brick's tile.
// With dense brick tiles, segments are claimed kClaimRun consecutive ones at
// a time, so a brick's segments tend to follow each other in one workgroup,
// which then keeps the brick's staged tile (reuse set) instead of loading it
// again (measured on the 8-view pass: 24.4 ms one at a time, 24.1 ms in runs
// of 2, 23.9 ms in runs of 8).  The multi-level boxes depend on each
// segment's samples, so those segments are claimed one at a time.
#ifndef CIC_CLAIM_RUN
#define CIC_CLAIM_RUN 8
#endif
constexpr int kClaimRun = CIC_CLAIM_RUN;
struct TileWork {
    int64_t brick;
    uint32_t start, end;
    int reuse;   // the staged tile is already this brick's
};
// the claiming thread's state: next index of its current run, the run's end, the brick in the tile
struct ClaimState {
    uint64_t next, end;
    int64_t tile_brick;
};
template <int RUN>
__device__ __forceinline__ bool claim_segment(const RenderBufs &b, TileWork *slot, ClaimState &cs, TileWork &w)
{
    __syncthreads();   // every wave is done with the previous segment and tile
    if (threadIdx.x == 0) {
        const int xcd = blockIdx.x % kXcds;
        const uint64_t nseg = b.seg_off[b.n_bricks];
        const uint64_t hi = nseg * (xcd + 1) / kXcds;
        if (cs.next >= cs.end) {
            cs.next = nseg * xcd / kXcds + atomicAdd(b.work_ctr + xcd, (uint32_t)RUN);
            cs.end = min(cs.next + RUN, hi);
        }
        TileWork t{-1, 0u, 0u, 0};
        if (cs.next < cs.end) {
            const uint64_t k = cs.next++;
            const uint32_t brick = b.seg_brick[k];   // from the segment table
            const uint32_t bstart = brick == 0 ? 0u : b.brick_off[brick - 1], bend = b.brick_off[brick];
            t.brick = brick;
            t.start = bstart + ((uint32_t)k - b.seg_off[brick]) * (uint32_t)kTileSeg;
            t.end = min(bend, t.start + (uint32_t)kTileSeg);
            t.reuse = (int64_t)brick == cs.tile_brick;
            cs.tile_brick = brick;
        }
        *slot = t;
    }
    __syncthreads();
    w = *slot;
    return w.brick >= 0;
}

// ---------------------------------------------------------------------------
// Voxel order with the multi-level encoding (hierarchical encodings, Sec.
// IV-A): the segments are still those of the density grid's bricks.  For each
// segment the workgroup stages its samples' records (record index, ray and
// float32 position) and reduces, per level, the bounding box of the cells the
// samples fall in.  Levels are then taken coarse to fine: a level whose box
// of vertices fits the LDS left over and holds no more vertices than the
// segment's gathers would request (8 per sample) is loaded into LDS once and
// its samples interpolate from there; the other levels (typically the finest,
// whose box is large against the samples that use it) are gathered from the
// table per sample, the plain data flow.  Either way a vertex's value is the
// table's, so the features equal the ray-order gather bit for bit.
// ---------------------------------------------------------------------------
// Level staging rule: 0 = levels whose box fits and holds at most 8 vertices
// per sample of the segment; 1 = the densely stored levels only, when they
// fit; 2 = every level that fits.
#ifndef CIC_HASH_STAGE
#define CIC_HASH_STAGE 0
#endif
constexpr int kHSegWords = 5 * kTileSeg;   // record, ray, position x, y, z
constexpr int kHTileBytes = 66 * 1024;     // LDS for the staged levels' vertices

// one staged vertex: the level's 3 features and a pad, in the table's type
template <typename T> struct HashVtx;
template <> struct HashVtx<float> {
    typedef float type __attribute__((ext_vector_type(4)));
};
template <> struct HashVtx<__half> {
    typedef _Float16 type __attribute__((ext_vector_type(4)));
};

struct HashSegInfo {
    float pmin[kBfWaves][3], pmax[kBfWaves][3];   // per wavefront: bounds of its samples' positions
    int lo[4][3], hi[4][3];   // per level: lowest and highest cell of the segment's samples
    int ext[4][3];            // vertices per axis of the staged box (hi - lo + 2)
    int off[4];               // first staged vertex of the level, -1: gathered from the table
};

__device__ __forceinline__ float wave_min_f(float v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = fminf(v, __shfl_xor(v, o, kWave));
    return v;
}
__device__ __forceinline__ float wave_max_f(float v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = fmaxf(v, __shfl_xor(v, o, kWave));
    return v;
}

// Records of the segment's samples into LDS, and each wavefront's bounds of
// their positions.  A level's cell index along an axis is a non-decreasing
// function of that coordinate (subtract, scale by a positive factor, floor,
// clamp, each monotonic in float32), so the cells of the extreme coordinates
// bound every sample's cells exactly.
__device__ void stage_segment_hash(const GridK &g, const RenderBufs &b, uint32_t start, int n, uint32_t *seg,
                                   HashSegInfo &h)
{
    float mn[3] = {INFINITY, INFINITY, INFINITY}, mx[3] = {-INFINITY, -INFINITY, -INFINITY};
    constexpr int kIter = (kTileSeg + kTileThreads - 1) / kTileThreads;
#pragma unroll
    for (int k = 0; k < kIter; ++k) {
        // out-of-range threads repeat the last sample (its cells do not widen the bounds)
        const int e = (int)threadIdx.x + k * kTileThreads;
        const uint32_t rec = b.perm[start + min(e, n - 1)];
        SampleRay r;
        load_sample_ray(b, b.rec_ray[rec], b.rec_k[rec], r);
        float xp[3];
        sample_position(r, xp);
        if (e < n) {
            seg[e] = rec;
            seg[kTileSeg + e] = r.ray;
#pragma unroll
            for (int a = 0; a < 3; ++a) seg[(2 + a) * kTileSeg + e] = __float_as_uint(xp[a]);
        }
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            mn[a] = fminf(mn[a], xp[a]);
            mx[a] = fmaxf(mx[a], xp[a]);
        }
    }
    const int wave = threadIdx.x / kWave;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        const float lo = wave_min_f(mn[a]), hi = wave_max_f(mx[a]);
        if (lane_id() == 0) {
            h.pmin[wave][a] = lo;
            h.pmax[wave][a] = hi;
        }
    }
}

// Where the batches find a level's staged box (off < 0: not staged).
struct LevelTile {
    int off, lo[3], sy, sx;   // sy = ez, sx = ey * ez
};

// Which levels the segment stages, and where (one thread).
template <typename T>
__device__ void plan_hash_levels(const GridK &g, int n, HashSegInfo &h, LevelTile *lt)
{
    constexpr int64_t vb = sizeof(typename HashVtx<T>::type);
    float pmin[3], pmax[3];
    for (int a = 0; a < 3; ++a) {
        pmin[a] = h.pmin[0][a];
        pmax[a] = h.pmax[0][a];
        for (int w = 1; w < kBfWaves; ++w) {
            pmin[a] = fminf(pmin[a], h.pmin[w][a]);
            pmax[a] = fmaxf(pmax[a], h.pmax[w][a]);
        }
    }
    int64_t used = 0;
    for (int l = 0; l < 4; ++l) {
        float fr[3];
        hash_cell(g, l, pmin, h.lo[l], fr);
        hash_cell(g, l, pmax, h.hi[l], fr);
        int64_t nv = 1;
        for (int a = 0; a < 3; ++a) {
            h.ext[l][a] = h.hi[l][a] - h.lo[l][a] + 2;
            nv *= h.ext[l][a];
        }
        const bool want = CIC_HASH_STAGE == 0 ? nv <= 8 * (int64_t)n : CIC_HASH_STAGE == 1 ? g.hdense[l] != 0 : true;
        if (want && used + nv * vb <= kHTileBytes) {
            h.off[l] = (int)(used / vb);
            used += nv * vb;
        } else {
            h.off[l] = -1;
        }
        lt[l] = LevelTile{h.off[l], {h.lo[l][0], h.lo[l][1], h.lo[l][2]}, h.ext[l][2], h.ext[l][1] * h.ext[l][2]};
    }
}

// The staged levels' vertex boxes from the tables into LDS (vertex (dx, dy,
// dz) of the box at off + (dx * ey + dy) * ez + dz).
// The staged boxes are contiguous in level order, so staged vertex t is
// vertex t - off[l] of the level l whose range holds t; each thread loads
// kHLoads of them with independent loads before storing any.
constexpr int kHLoads = 8;
template <typename T>
__device__ void load_hash_tiles(const GridK &g, const HashSegInfo &h, typename HashVtx<T>::type *tile)
{
    typedef typename HashVtx<T>::type V;
    typedef decltype(V{}[0]) E;
    int end[4], tot = 0;
#pragma unroll
    for (int l = 0; l < 4; ++l) {
        if (h.off[l] >= 0) tot = h.off[l] + h.ext[l][0] * h.ext[l][1] * h.ext[l][2];
        end[l] = tot;
    }
    for (int t0 = threadIdx.x; t0 < tot; t0 += kHLoads * kTileThreads) {
        float x[kHLoads][3];
#pragma unroll
        for (int u = 0; u < kHLoads; ++u) {
            const int t = min(t0 + u * kTileThreads, tot - 1);   // past the end: reload the last vertex
            const int l = t < end[0] ? 0 : t < end[1] ? 1 : t < end[2] ? 2 : 3;
            const int v = t - h.off[l], ey = h.ext[l][1], ez = h.ext[l][2];
            const int dz = v % ez, dy = (v / ez) % ey, dx = v / (ez * ey);
            const T *tab = (const T *)g.htab + (size_t)l * ((size_t)g.hmask + 1) * 3;
            load_entry3(tab, hash_entry(g, l, (uint32_t)(h.lo[l][0] + dx), (uint32_t)(h.lo[l][1] + dy),
                                        (uint32_t)(h.lo[l][2] + dz)),
                        x[u]);
        }
#pragma unroll
        for (int u = 0; u < kHLoads; ++u) {
            const int t = t0 + u * kTileThreads;
            if (t < tot) tile[t] = V{(E)x[u][0], (E)x[u][1], (E)x[u][2], (E)0.0f};
        }
    }
}

// Level q's 3 features of a sample at position xp: from the staged box when
// the level is staged, else gathered from the table.
template <typename T>
__device__ __forceinline__ void hash_level3_tiled(const GridK &g, const LevelTile &lt,
                                                  const typename HashVtx<T>::type *tile, int q, const float xp[3],
                                                  float x[3])
{
    int i0[3];
    float fr[3], v[8][3];
    hash_cell(g, q, xp, i0, fr);
    if (lt.off >= 0) {
        const int base = lt.off + (i0[0] - lt.lo[0]) * lt.sx + (i0[1] - lt.lo[1]) * lt.sy + (i0[2] - lt.lo[2]);
#pragma unroll
        for (int c = 0; c < 8; ++c) {
            const auto w = tile[base + ((c >> 2) & 1) * lt.sx + ((c >> 1) & 1) * lt.sy + (c & 1)];
#pragma unroll
            for (int f = 0; f < 3; ++f) v[c][f] = (float)w[f];
        }
    } else {
        hash_corners<T>(g, q, i0, v);
    }
    lerp3_corners(v, fr, x);
}

// ---------------------------------------------------------------------------
// BF16 variant: every layer on v_mfma_f32_16x16x32_bf16 (inputs rounded to
// BF16 with round-to-nearest-even, FP32 accumulation, FP32 bias and
// activations).  K = 32 per instruction: lane (q, j) supplies 8 consecutive
// reduction slots.  Layer 0 uses two K-chunks (64 slots >= 39 inputs, same
// per-lane input assignment as the FP32 kernel: the ten values of lane group
// q fill chunk 0 and the first two slots of chunk 1).  Its bias rides in
// the third slot of chunk 1 of lane groups 0-2: the per-ray encoding row
// carries a constant 1 there, and the weights hold the three BF16 parts of
// the float32 bias, whose sum is the bias exactly, so the layer reads no
// bias from LDS.  Layers 1 and 2 take
// their B operand from two consecutive 16-row result tiles of the previous
// layer: chunk c of lane group q covers rows 32c + 4q + (0..3) and
// 32c + 16 + 4q + (0..3), and the weight fragments are laid out to match.
// The 3-wide output layer is one zero-padded 16-row tile.
// ---------------------------------------------------------------------------
typedef __bf16 bf8_t __attribute__((ext_vector_type(8)));

// LDS layout in 16-byte fragments, then floats
constexpr int kBfW0 = 0;                           // [t 8][c 2][lane 64]
constexpr int kBfW1 = kBfW0 + 8 * 2 * 64;          // [t 8][c 4][lane 64]
constexpr int kBfW2 = kBfW1 + 8 * 4 * 64;          // [c 4][lane 64]
constexpr int kBfFrags = kBfW2 + 4 * 64;
constexpr int kBfB1 = 0, kBfB2 = 128, kBfFloats = 132;
constexpr int kLdsBf16 = kBfFrags * 16 + kBfFloats * 4;
static_assert(kLdsBf16 + (kFTileFloats + kSegWords) * 4 <= 160 * 1024 - 1024, "brick tile kernel LDS");

// reduction index of slot e of chunk c for lane group q in layers 1 and 2
__host__ __device__ __forceinline__ int hid_k(int c, int q, int e)
{
    return e < 4 ? 32 * c + 4 * q + e : 32 * c + 16 + 4 * q + (e - 4);
}

// input index of slot e of chunk c for lane group q in layer 0 (-1 = pad)
__host__ __device__ __forceinline__ int bf_l0_input(int c, int q, int e)
{
    const int slot = 8 * c + e;
    return slot < 10 ? l0_input(slot, q) : -1;
}

// slot of chunk 1 (lane groups 0-2) that carries layer 0's bias: input 1.0
// (encoding slot 7), weight the group's part of the bias
constexpr int kBfBiasSlot = 2;

// part p of float32 b split into three BF16 values b0 + b1 + b2 = b (each
// remainder is exact in float32, and the last has at most 8 significant bits)
__device__ __forceinline__ float bf16_part(float b, int p)
{
    const float hi = (float)(__bf16)b, r1 = b - hi;
    const float mid = (float)(__bf16)r1, r2 = r1 - mid;
    return p == 0 ? hi : p == 1 ? mid : r2;
}

__device__ void stage_weights_bf16(const cic_mlp &m, bf8_t *frag, float *fl)
{
    const int nt = blockDim.x;
    for (int i = threadIdx.x; i < 8 * 2 * 64; i += nt) {
        const int l = i & 63, c = (i >> 6) & 1, t = i >> 7;
        const int row = 16 * t + (l & 15), q = l >> 4;
        bf8_t v;
#pragma unroll
        for (int e = 0; e < 8; ++e) {
            const int src = bf_l0_input(c, q, e);
            float w = src >= 0 ? m.w0[row * 39 + src] : 0.f;
            if (c == 1 && e == kBfBiasSlot) w = q < 3 ? bf16_part(m.b0[row], q) : 0.f;   // exact in BF16
            v[e] = (__bf16)w;
        }
        frag[kBfW0 + i] = v;
    }
    for (int i = threadIdx.x; i < 8 * 4 * 64; i += nt) {
        const int l = i & 63, c = (i >> 6) & 3, t = i >> 8;
        const int row = 16 * t + (l & 15), q = l >> 4;
        bf8_t v;
#pragma unroll
        for (int e = 0; e < 8; ++e) v[e] = (__bf16)m.w1[row * 128 + hid_k(c, q, e)];
        frag[kBfW1 + i] = v;
    }
    for (int i = threadIdx.x; i < 4 * 64; i += nt) {
        const int l = i & 63, c = i >> 6;
        const int row = l & 15, q = l >> 4;
        bf8_t v;
#pragma unroll
        for (int e = 0; e < 8; ++e) v[e] = (__bf16)(row < 3 ? m.w2[row * 128 + hid_k(c, q, e)] : 0.f);
        frag[kBfW2 + i] = v;
    }
    for (int i = threadIdx.x; i < 128; i += nt) fl[kBfB1 + i] = m.b1[i];
    if (threadIdx.x < 4) fl[kBfB2 + threadIdx.x] = threadIdx.x < 3 ? m.b2[threadIdx.x] : 0.f;
}

__device__ __forceinline__ bf8_t pack_bf8(const f4_t a, const f4_t b)
{
    bf8_t v;
#pragma unroll
    for (int e = 0; e < 4; ++e) {
        v[e] = (__bf16)a[e];
        v[4 + e] = (__bf16)b[e];
    }
    return v;
}

// ReLU of BF16 values as 16-bit integers: a negative BF16 (sign bit set) is
// a negative int16, so max(bits, 0) zeroes exactly the negatives (and -0).
// Rounding to BF16 preserves sign, so this equals rounding after the ReLU.
typedef short s8_t __attribute__((ext_vector_type(8)));
__device__ __forceinline__ bf8_t relu_bf8(bf8_t v)
{
    s8_t s = __builtin_bit_cast(s8_t, v);
#pragma unroll
    for (int e = 0; e < 8; ++e) s[e] = s[e] > 0 ? s[e] : (short)0;
    return __builtin_bit_cast(bf8_t, s);
}

// TILE: 0 = gathers from the grid (ray order, or voxel order through the
// sample permutation); 1 = voxel order with the brick's features staged in
// LDS (dense grids); 2 = voxel order with the segment's multi-level encoding
// boxes staged in LDS.
template <typename T, int TILE>
__global__ __launch_bounds__(kBfWaves * 64) void k_mlp_fwd_bf16(GridK g, cic_mlp m, RenderBufs b, int voxel)
{
    typedef typename HashVtx<T>::type HV;
    extern __shared__ __attribute__((aligned(16))) float lds_raw[];   // 16-byte fragments
    bf8_t *frag = (bf8_t *)lds_raw;
    float *fl = lds_raw + kBfFrags * 4;
    float *tile = lds_raw + kBfFrags * 4 + kBfFloats;    // TILE 1: the brick's features
    // TILE 1, 2: the segment's records
    uint32_t *seg = TILE == 1 ? (uint32_t *)(tile + kFTileFloats) : (uint32_t *)tile;
    HV *htile = (HV *)(seg + kHSegWords);                // TILE 2: the staged level boxes
    __shared__ TileWork seg_slot;
    __shared__ HashSegInfo hinfo;
    __shared__ LevelTile ltab[4];
    stage_weights_bf16(m, frag, fl);
    __syncthreads();

    const int lane = lane_id(), q = lane >> 4, j = lane & 15;
    const int wave = threadIdx.x / 64;
    const int64_t total = (int64_t)b.offsets[b.n];

    // one batch of kBfNT tiles: samples s0 + nt*16 + j below send (TILE:
    // positions in the staged segment)
    auto batch = [&](int64_t s0, int64_t send) {
        // wave priority raised at each layer, as in the FP32 kernel (measured:
        // MLP stage 27.0 -> 26.7 ms in voxel order, 45.3 -> 45.0 ms in ray order)
        __builtin_amdgcn_s_setprio(0);
        bf8_t xin[kBfNT][2];
        int64_t rec[kBfNT];
        bool valid[kBfNT];
#pragma unroll
        for (int nt = 0; nt < kBfNT; ++nt) {
            const int64_t s = s0 + nt * 16 + j;
            valid[nt] = s < send;
            // a lane past the batch's last sample works on the first sample of
            // the range (in-bounds inputs, no branches around the loads); its
            // colour is not stored
            const int64_t sv = valid[nt] ? s : 0;
            if (TILE) rec[nt] = (int64_t)seg[sv];
            else rec[nt] = voxel ? (int64_t)b.perm[sv] : sv;
            float x[10];
            uint32_t ray;
            if constexpr (TILE == 2) {
                ray = seg[kTileSeg + sv];
                const float xp[3] = {__uint_as_float(seg[2 * kTileSeg + sv]), __uint_as_float(seg[3 * kTileSeg + sv]),
                                     __uint_as_float(seg[4 * kTileSeg + sv])};
                hash_level3_tiled<T>(g, ltab[q], htile, q, xp, x);
            } else if constexpr (TILE == 1) {
                ray = seg[kTileSeg + sv];
                const float fr[3] = {__uint_as_float(seg[2 * kTileSeg + sv]), __uint_as_float(seg[3 * kTileSeg + sv]),
                                     __uint_as_float(seg[4 * kTileSeg + sv])};
                const uint32_t cell = seg[5 * kTileSeg + sv];
                tile_gather3(tile, (int)(cell & 15u), (int)((cell >> 4) & 15u), (int)(cell >> 8), fr, q, x);
            } else {
                sample_inputs<T, false>(g, b, rec[nt], q, x);
                ray = b.rec_ray[rec[nt]];
            }
            typedef uint32_t u4_t __attribute__((ext_vector_type(4)));
            const bf8_t ev = __builtin_bit_cast(bf8_t, *(const u4_t *)(b.enc + (int64_t)ray * 16 + 4 * q));
            // chunk 0: features 3q..3q+2 then encoding slots 0..4; chunk 1:
            // encoding slots 5, 6 and the bias slot's constant 1 (slot 7)
#pragma unroll
            for (int e = 0; e < 8; ++e) {
                xin[nt][0][e] = e < 3 ? (__bf16)x[e] : ev[e - 3];
                xin[nt][1][e] = e < 3 ? ev[5 + e] : (__bf16)0.0f;
            }

        }
        // layer 0.  A finished pair of row blocks (32 hidden units) becomes
        // one BF16 input chunk of layer 1 while the next pair's MFMAs issue:
        // one row block per scheduling region, the pair before it converted in
        // the region of the next even block.
        __builtin_amdgcn_s_setprio(1);
        // (the bias comes in through input chunk 1)
        bf8_t hb[4][kBfNT];
        f4_t h1[2][2][kBfNT];   // [pair parity][block of the pair][tile]
#pragma unroll
        for (int t = 0; t <= 8; ++t) {
            const f4_t zero = f4_t{0.f, 0.f, 0.f, 0.f};
            if (t < 8) {
#pragma unroll
                for (int c = 0; c < 2; ++c) {
                    const bf8_t a = frag[kBfW0 + (t * 2 + c) * 64 + lane];
#pragma unroll
                    for (int nt = 0; nt < kBfNT; ++nt)
                        h1[(t >> 1) & 1][t & 1][nt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(
                            a, xin[nt][c], c == 0 ? zero : h1[(t >> 1) & 1][t & 1][nt], 0, 0, 0);
                }
            }
            if ((t & 1) == 0 && t > 0) {
                const int pr = (t >> 1) - 1;
#pragma unroll
                for (int nt = 0; nt < kBfNT; ++nt)
                    hb[pr][nt] = relu_bf8(pack_bf8(h1[pr & 1][0][nt], h1[pr & 1][1][nt]));
            }
            __builtin_amdgcn_sched_barrier(0);
        }
        // layer 1, and the output layer (one zero-padded tile) fed pair by
        // pair: the output MFMA of a finished pair of row blocks issues in the
        // region of the next even block (the same sums in the same order as
        // after the whole layer)
        __builtin_amdgcn_s_setprio(2);
        f4_t h2[2][2][kBfNT];
        f4_t o3[kBfNT];
        const f4_t bias2 = *(const f4_t *)(fl + kBfB2);
#pragma unroll
        for (int t = 0; t <= 8; ++t) {
            if (t < 8) {
                const f4_t bias = *(const f4_t *)(fl + kBfB1 + 16 * t + 4 * q);
#pragma unroll
                for (int c = 0; c < 4; ++c) {
                    const bf8_t a = frag[kBfW1 + (t * 4 + c) * 64 + lane];
#pragma unroll
                    for (int nt = 0; nt < kBfNT; ++nt)
                        h2[(t >> 1) & 1][t & 1][nt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(
                            a, hb[c][nt], c == 0 ? bias : h2[(t >> 1) & 1][t & 1][nt], 0, 0, 0);
                }
            }
            if ((t & 1) == 0 && t > 0) {
                const int pr = (t >> 1) - 1;
                const bf8_t a = frag[kBfW2 + pr * 64 + lane];
#pragma unroll
                for (int nt = 0; nt < kBfNT; ++nt)
                    o3[nt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(
                        a, relu_bf8(pack_bf8(h2[pr & 1][0][nt], h2[pr & 1][1][nt])), pr == 0 ? bias2 : o3[nt], 0, 0, 0);
            }
            __builtin_amdgcn_sched_barrier(0);
        }
        __builtin_amdgcn_s_setprio(3);
        // lanes of group 0 hold rows 0..3 (colour channels 0..2) of their sample
#pragma unroll
        for (int nt = 0; nt < kBfNT; ++nt) {
            if (valid[nt] && q == 0) {
                float *out = b.rec_c + 3 * rec[nt];
                out[0] = sigmoid_hw(o3[nt][0]);
                out[1] = sigmoid_hw(o3[nt][1]);
                out[2] = sigmoid_hw(o3[nt][2]);
            }
        }
    };

    if constexpr (TILE != 0) {
        TileWork w;
        ClaimState cs{0, 0, -1};   // used by thread 0 only
        while (claim_segment<TILE == 1 ? kClaimRun : 1>(b, &seg_slot, cs, w)) {
            const int n = (int)(w.end - w.start);
            if constexpr (TILE == 2) {
                stage_segment_hash(g, b, w.start, n, seg, hinfo);
                __syncthreads();
                if (threadIdx.x == 0) plan_hash_levels<T>(g, n, hinfo, ltab);
                __syncthreads();
                load_hash_tiles<T>(g, hinfo, htile);
            } else {
                const BrickBase base = brick_base(g, w.brick);
                if (!w.reuse) load_feature_tile<T>(g, base, tile);
                stage_segment(g, b, w.start, n, base, seg);
            }
            __syncthreads();
            const int nb = (n + kBfBatch - 1) / kBfBatch;
            for (int bi = wave; bi < nb; bi += kBfWaves) batch((int64_t)bi * kBfBatch, (int64_t)n);
        }
    } else {
        const int64_t nbatch = (total + kBfBatch - 1) / kBfBatch;
        const BatchRange br = xcd_batches(nbatch, kBfWaves, wave);
        for (int64_t bt = br.first; bt < br.end; bt += br.stride) batch(bt * kBfBatch, total);
    }
}

#ifndef CIC_VOXEL_TILE
#define CIC_VOXEL_TILE 1
#endif
template <typename T, int TILE>
static void launch_bf16_k(const GridK &g, const cic_mlp &m, const RenderBufs &b, bool voxel, hipStream_t s)
{
    const int lds = kLdsBf16 + (TILE == 1 ? (kFTileFloats + kSegWords) * 4 : TILE == 2 ? kHSegWords * 4 + kHTileBytes : 0);
    static bool attr_set = false;
    if (!attr_set) {
        (void)hipFuncSetAttribute((const void *)k_mlp_fwd_bf16<T, TILE>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                  lds);
        attr_set = true;
    }
    if (TILE) {
        launch_brick_segments(b, kTileSeg, true, s);
        launch_fill_u32(b.work_ctr, 0u, kXcds, s);
    }
    // TILE: at least one workgroup per XCD range of segments
    const int grid = TILE ? std::max(num_cus(b) * kBfWgs, kXcds) : num_cus(b) * kBfWgs;
    hipLaunchKernelGGL((k_mlp_fwd_bf16<T, TILE>), dim3(grid), dim3(kBfWaves * 64), lds, s, g, m, b,
                       voxel ? 1 : 0);
}

template <typename T>
void launch_mlp_forward_bf16(const GridK &g, const cic_mlp &m, const RenderBufs &b, bool voxel, hipStream_t s)
{
    if (CIC_VOXEL_TILE && voxel) {
        if (g.hlevels == 0) launch_bf16_k<T, 1>(g, m, b, true, s);
        else launch_bf16_k<T, 2>(g, m, b, true, s);
    } else {
        launch_bf16_k<T, 0>(g, m, b, voxel, s);
    }
}

template void launch_mlp_forward_bf16<float>(const GridK &, const cic_mlp &, const RenderBufs &, bool, hipStream_t);
template void launch_mlp_forward_bf16<__half>(const GridK &, const cic_mlp &, const RenderBufs &, bool, hipStream_t);

}  // namespace cic
