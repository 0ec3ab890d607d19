// Ray marching, live-sample compaction, voxel-order bucketing and the final
// per-ray accumulation of the rendering quadrature.
//
// March: one wavefront per ray, 64 samples per step (one per lane).  Each
// lane finds its sample's voxel, skips it if unoccupied, interpolates the
// raw density, applies softplus and forms the optical depth sigma*delta.  A
// wavefront inclusive scan of the optical depths gives every lane its
// transmittance T_k = exp(-(carry + exclusive sum)); the first lane whose
// T_k falls below the threshold ends the ray (ballot + find-first-set).
// Live samples (occupied, before termination) are written to per-ray slots
// with their weight w_k = T_k (1 - exp(-sigma_k delta)); sum w_k t_k is a
// wavefront tree sum.  The MLP stage later reads the compacted live samples;
// the per-ray reduction sums w_k c_k in sample order, so results do not
// depend on the order in which the MLP stage visits samples.
#include "kernels.h"

namespace cic {

constexpr int kRayWaves = 4;   // rays (wavefronts) per 256-thread block

// ln(u) for finite u >= 1/2 (the only inputs below whose result is used):
// the hardware log2 times ln 2 rounded to float (3e-9 relative), without the
// library's denormal scaling and extended-precision product
__device__ __forceinline__ float ln_hw(float u)
{
    return __builtin_amdgcn_logf(u) * 0.693147182f;
}

// e^x for x <= 15 (no overflow to guard): 2^(x log2 e) on the hardware exp2,
// the rounding error of the product x log2 e (and of log2 e itself) carried
// as a first-order correction e^lo ~ 1 + lo ln 2 (within 1.2e-7 relative
// when exp2 is correctly rounded)
__device__ __forceinline__ float exp_hw(float x)
{
    constexpr float kL = 1.44269502162933349609375f;    // log2(e) rounded to float
    constexpr float kLlo = 1.925963033500011079e-8f;    // log2(e) - kL
    const float hi = x * kL;
    const float lo = fmaf(x, kLlo, fmaf(x, kL, -hi));
    const float eh = __builtin_amdgcn_exp2f(hi);
    return fmaf(eh, lo * 0.693147182f, eh);
}

// softplus(x) = log(1 + e^x) (x + e^-x above 15), with log1p(e) taken as
// log(u) e / (u - 1), u = 1 + e: Goldberg's form, accurate to a few ulp when
// the logarithm is (3.1e-7 relative over x <= 15 with the hardware exp2, log2
// and reciprocal correctly rounded), where the library's log1pf spends about
// a hundred instructions per call
__device__ __forceinline__ float softplus_fast(float x)
{
    const bool big = x > 15.0f;
    const float e = exp_hw(big ? -x : x), u = 1.0f + e;
    const float l = u == 1.0f ? e : ln_hw(u) * (e * __builtin_amdgcn_rcpf(u - 1.0f));
    return big ? x + e : l;
}

// Opacity 1 - e^-s of optical depth s >= 0: directly where e^-s <= 1/2, and
// in Kahan's form (1 - u) s / -log(u), u = e^-s, near s = 0, where the
// subtraction would cancel (2.4e-7 relative, from the hardware exp2 and log2)
__device__ __forceinline__ float opacity_fast(float s)
{
    const float u = __expf(-s);
    const float k = u == 1.0f ? s : (1.0f - u) * s * __builtin_amdgcn_rcpf(-ln_hw(u));
    return u > 0.5f ? k : 1.0f - u;
}

// Wavefront inclusive prefix sum on DPP lane moves (no LDS round trips):
// within each row of 16 lanes, shifts by 1, 2, 4 and 8 (a lane without a
// source adds 0); then rows 1 and 3 add the last lane of rows 0 and 2, and
// rows 2 and 3 add lane 31.
template <int CTRL, int ROW_MASK, bool BOUND_ZERO>
__device__ __forceinline__ float dpp_add(float v)
{
    return v + __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), CTRL, ROW_MASK, 0xf, BOUND_ZERO));
}
__device__ __forceinline__ float wave_incl_scan_dpp(float v)
{
    v = dpp_add<0x111, 0xf, true>(v);    // row_shr:1
    v = dpp_add<0x112, 0xf, true>(v);    // row_shr:2
    v = dpp_add<0x114, 0xf, true>(v);    // row_shr:4
    v = dpp_add<0x118, 0xf, true>(v);    // row_shr:8
    v = dpp_add<0x142, 0xa, false>(v);   // row_bcast:15 into rows 1, 3
    v = dpp_add<0x143, 0xc, false>(v);   // row_bcast:31 into rows 2, 3
    return v;
}
// the value of the lane below (0 in lane 0): wave_shr:1
__device__ __forceinline__ float wave_shr1(float v)
{
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x138, 0xf, 0xf, true));
}

template <typename T>
__global__ __launch_bounds__(256) void k_march(GridK g, OptsK op, RenderBufs b)
{
    const int lane = lane_id();
    const int64_t ray = (int64_t)blockIdx.x * kRayWaves + (threadIdx.x / kWave);
    if (ray >= b.n) return;
    const uint32_t n_act = b.n_active ? *b.n_active : (uint32_t)b.n;
    if ((uint64_t)ray >= n_act) {
        if (lane == 0) {
            b.count[ray] = 0;
            b.info[ray] = RayInfo{0.f, 0.f, 1.f, 0.f};
        }
        return;
    }
    float o[3], d[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        o[a] = b.rays_o[3 * ray + a];
        d[a] = b.rays_d[3 * ray + a];
    }
    float tn, tf;
    if (!ray_box(o, d, g, tn, tf)) {
        if (lane == 0) {
            b.count[ray] = 0;
            b.info[ray] = RayInfo{tn, 0.f, 1.f, 0.f};
        }
        return;
    }
    const int N = op.n_samples;
    const float delta = (tf - tn) / (float)N;
    const float thr = op.et_threshold;
    const T *dens = (const T *)g.density;
    uint16_t *slot_k = b.slot_k + ray * (int64_t)N;
    float *slot_w = b.slot_w + ray * (int64_t)N;
    float carry = 0.f, depth = 0.f, t_stop = -1.f;
    uint32_t count = 0;
    for (int base = 0; base < N; base += kWave) {
        const int k = base + lane;
        const bool valid = k < N;
        float s = 0.f, tk = 0.f;
        bool occ = false;
        if (valid) {
            int i0[3];
            float fr[3];
            sample_voxel(o, d, tn, delta, k, g, i0, fr, tk);
            occ = g.occ ? (g.occ[cell_index(g, i0)] != 0) : true;
            if (occ) {
                float raw = trilerp1(dens, g, i0, fr, 1, 0);
                s = softplus_fast(raw + g.shift) * delta;
            }
        }
        const float incl = wave_incl_scan_dpp(s);
        const float excl = wave_shr1(incl);
        const float Tk = __expf(-(carry + excl));
        const bool term = valid && thr > 0.f && Tk < thr;
        const uint64_t tmask = __ballot(term);
        const int first = tmask ? (__ffsll((unsigned long long)tmask) - 1) : kWave;
        const bool live = valid && occ && lane < first;
        const float w = live ? Tk * opacity_fast(s) : 0.f;
        const uint64_t lmask = __ballot(live);
        if (live) {
            const uint32_t pos = count + (uint32_t)__popcll(lmask & lanes_below_mask());
            slot_k[pos] = (uint16_t)k;
            slot_w[pos] = w;
            if (b.slot_t) b.slot_t[ray * (int64_t)N + pos] = Tk;
        }
        count += (uint32_t)__popcll(lmask);
        depth += __int_as_float(__builtin_amdgcn_readlane(__float_as_int(wave_incl_scan_dpp(w * tk)), kWave - 1));
        if (first < kWave) {
            t_stop = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(Tk), first));
            break;
        }
        carry += __int_as_float(__builtin_amdgcn_readlane(__float_as_int(incl), kWave - 1));
    }
    if (t_stop < 0.f) t_stop = __expf(-carry);
    if (lane == 0) {
        b.count[ray] = count;
        b.info[ray] = RayInfo{tn, delta, t_stop, depth};
    }
}

template <typename T>
void launch_march(const GridK &g, const OptsK &o, const RenderBufs &b, hipStream_t s)
{
    if (b.n == 0) return;
    const unsigned blocks = (unsigned)((b.n + kRayWaves - 1) / kRayWaves);
    hipLaunchKernelGGL(k_march<T>, dim3(blocks), dim3(256), 0, s, g, o, b);
}
template void launch_march<float>(const GridK &, const OptsK &, const RenderBufs &, hipStream_t);
template void launch_march<__half>(const GridK &, const OptsK &, const RenderBufs &, hipStream_t);

// Head-of-run detection for equal consecutive keys among the first `active`
// lanes: returns the mask of run heads; run length of a head lane is the
// distance to the next head (or to `active`).
__device__ __forceinline__ uint64_t run_heads(uint32_t key, bool active)
{
    const uint32_t prev = __shfl_up(key, 1, kWave);
    const bool head = active && (lane_id() == 0 || prev != key);
    return __ballot(head);
}

__device__ __forceinline__ int run_length(uint64_t heads, int active)
{
    const int l = lane_id();
    const uint64_t above = (l == kWave - 1) ? 0ull : (heads & ~((2ull << l) - 1ull));
    const int next = above ? (__ffsll((unsigned long long)above) - 1) : active;
    return next - l;
}

// One wavefront per ray copies its live samples to their compacted position
// (ray-order), and in voxel mode tags each with its brick and adds each run
// of equal bricks to counts[brick] (global counters or an LDS histogram).
//
// Ray order: the ray's count and offset are loaded together, and the slots
// of two 64-sample chunks before any record of them is stored (as far as the
// compiler knows the stores could alias the slots, so it would not move the
// second chunk's loads above the first chunk's stores by itself): two round
// trips to memory per ray instead of three or four (8-view pass: 2.27 to
// 1.84 ms).  The same form measured slower in voxel mode (4.77 to 6.25 ms with
// the LDS histogram), which keeps one chunk per step.
template <bool WITH_T>
__device__ __forceinline__ void compact_ray_rays(const RenderBufs &b, int64_t ray)
{
    const int lane = lane_id();
    const uint32_t cnt = b.count[ray];
    const uint32_t off = b.offsets[ray];
    if (cnt == 0) return;
    const int64_t slots = ray * (int64_t)b.n_samples;
    for (uint32_t j0 = 0; j0 < cnt; j0 += 2 * kWave) {
        // a lane past the count reads slot 0 (the count is positive); a
        // second chunk past the count stores nothing
        const uint32_t ja = j0 + lane, jb = ja + kWave;
        const int64_t sa = slots + (ja < cnt ? ja : 0u), sb = slots + (jb < cnt ? jb : 0u);
        const uint16_t ka = b.slot_k[sa], kb = b.slot_k[sb];
        const float wa = b.slot_w[sa], wb = b.slot_w[sb];
        float ta = 0.f, tb = 0.f;
        if constexpr (WITH_T) {
            ta = b.slot_t[sa];
            tb = b.slot_t[sb];
        }
        if (ja < cnt) {
            b.rec_ray[off + ja] = (uint32_t)ray;
            b.rec_k[off + ja] = ka;
            b.rec_w[off + ja] = wa;
            if constexpr (WITH_T) b.rec_t[off + ja] = ta;
        }
        if (jb < cnt) {
            b.rec_ray[off + jb] = (uint32_t)ray;
            b.rec_k[off + jb] = kb;
            b.rec_w[off + jb] = wb;
            if constexpr (WITH_T) b.rec_t[off + jb] = tb;
        }
    }
}

__device__ __forceinline__ void compact_ray(const GridK &g, const RenderBufs &b, int64_t ray, bool voxel,
                                            uint32_t *counts)
{
    if (!voxel) {
        if (b.rec_t) compact_ray_rays<true>(b, ray);
        else compact_ray_rays<false>(b, ray);
        return;
    }
    const int lane = lane_id();
    const uint32_t cnt = b.count[ray];
    if (cnt == 0) return;
    const uint32_t off = b.offsets[ray];
    const int N = b.n_samples;
    float o[3], d[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        o[a] = b.rays_o[3 * ray + a];
        d[a] = b.rays_d[3 * ray + a];
    }
    const RayInfo inf = b.info[ray];
    for (uint32_t j0 = 0; j0 < cnt; j0 += kWave) {
        const uint32_t j = j0 + lane;
        const bool act = j < cnt;
        uint32_t key = 0xffffffffu;
        if (act) {
            const uint16_t k = b.slot_k[ray * (int64_t)N + j];
            b.rec_ray[off + j] = (uint32_t)ray;
            b.rec_k[off + j] = k;
            b.rec_w[off + j] = b.slot_w[ray * (int64_t)N + j];
            if (b.rec_t) b.rec_t[off + j] = b.slot_t[ray * (int64_t)N + j];
            int i0[3];
            float fr[3], tk;
            sample_voxel(o, d, inf.tn, inf.delta, k, g, i0, fr, tk);
            key = brick_of(g, i0);
            b.rec_key[off + j] = key;
        }
        const int active = (int)min(cnt - j0, (uint32_t)kWave);
        const uint64_t heads = run_heads(key, act);
        if ((heads >> lane) & 1ull) atomicAdd(&counts[key], (uint32_t)run_length(heads, active));
    }
}

__global__ __launch_bounds__(256) void k_compact(GridK g, RenderBufs b, int voxel)
{
    const int64_t ray = (int64_t)blockIdx.x * kRayWaves + (threadIdx.x / kWave);
    if (ray >= b.n) return;
    compact_ray(g, b, ray, voxel != 0, b.brick_off);
}

// Voxel mode with an LDS histogram of the bricks: a block compacts
// kHistRays consecutive rays, counting their runs in LDS, and then adds each
// brick it touched to the global count once.  The rays of a block cross
// largely the same bricks, so this takes far fewer device-wide atomics than
// one per run.
constexpr int kHistBins = 16384;   // largest brick count of the LDS path (64 KB)
constexpr int kHistRays = 256;     // rays per block
// 16 wavefronts per block, 16 rays each: the rays' dependent load chains
// overlap across wavefronts (measured on eight 800x800 views: compaction +
// sort 6.5 ms with 4 wavefronts per block, 4.9 ms with 8, 4.7 ms with 16)
constexpr int kHistThreads = 1024;
// The LDS path needs enough blocks to fill the chip (small launches, such as
// a training step's few thousand rays, keep the per-run global atomics).
static bool use_hist(const RenderBufs &b)
{
    return b.n_bricks <= kHistBins && b.n >= (int64_t)kHistRays * 512;
}

__global__ __launch_bounds__(kHistThreads) void k_compact_hist(GridK g, RenderBufs b)
{
    extern __shared__ uint32_t hist[];
    for (int64_t i = threadIdx.x; i < b.n_bricks; i += blockDim.x) hist[i] = 0u;
    __syncthreads();
    const int64_t ray0 = (int64_t)blockIdx.x * kHistRays;
    const int64_t ray1 = ray0 + kHistRays < b.n ? ray0 + kHistRays : b.n;
    for (int64_t ray = ray0 + threadIdx.x / kWave; ray < ray1; ray += blockDim.x / kWave)
        compact_ray(g, b, ray, true, hist);
    __syncthreads();
    for (int64_t i = threadIdx.x; i < b.n_bricks; i += blockDim.x) {
        const uint32_t c = hist[i];
        if (c) atomicAdd(&b.brick_off[i], c);
    }
}

void launch_compact(const GridK &g, const RenderBufs &b, bool voxel_keys, hipStream_t s)
{
    if (b.n == 0) return;
    if (voxel_keys && use_hist(b)) {
        const unsigned blocks = (unsigned)((b.n + kHistRays - 1) / kHistRays);
        hipLaunchKernelGGL(k_compact_hist, dim3(blocks), dim3(kHistThreads), b.n_bricks * sizeof(uint32_t), s, g, b);
        return;
    }
    const unsigned blocks = (unsigned)((b.n + kRayWaves - 1) / kRayWaves);
    hipLaunchKernelGGL(k_compact, dim3(blocks), dim3(256), 0, s, g, b, voxel_keys ? 1 : 0);
}

// Bucket scatter: brick_off holds the exclusive scan of brick counts and is
// advanced as a cursor; each run of equal bricks takes one atomic.
__global__ __launch_bounds__(256) void k_brick_scatter(RenderBufs b)
{
    const int lane = lane_id();
    const int64_t ray = (int64_t)blockIdx.x * kRayWaves + (threadIdx.x / kWave);
    if (ray >= b.n) return;
    const uint32_t cnt = b.count[ray];
    if (cnt == 0) return;
    const uint32_t off = b.offsets[ray];
    for (uint32_t j0 = 0; j0 < cnt; j0 += kWave) {
        const uint32_t j = j0 + lane;
        const bool act = j < cnt;
        const uint32_t key = act ? b.rec_key[off + j] : 0xffffffffu;
        const int active = (int)min(cnt - j0, (uint32_t)kWave);
        const uint64_t heads = run_heads(key, act);
        uint32_t base = 0;
        if ((heads >> lane) & 1ull) base = atomicAdd(&b.brick_off[key], (uint32_t)run_length(heads, active));
        // head of my run = highest head at or below my lane
        const uint64_t upto = heads & ((lane == kWave - 1) ? ~0ull : ((2ull << lane) - 1ull));
        const int head = upto ? (63 - __clzll((long long)upto)) : 0;
        const uint32_t hb = __shfl(base, head, kWave);
        if (act) b.perm[hb + (uint32_t)(lane - head)] = off + j;
    }
}

// LDS-histogram scatter over the same blocks of kHistRays rays, whose
// samples are one contiguous range of records: count the block's samples
// per brick in LDS, reserve each touched brick's share of the global cursor
// with one atomic, then hand out positions from the LDS cursors (one LDS
// atomic per run of equal bricks).
__global__ __launch_bounds__(kHistThreads) void k_brick_scatter_hist(RenderBufs b)
{
    extern __shared__ uint32_t hist[];
    const int lane = lane_id(), wave = threadIdx.x / kWave, nwaves = blockDim.x / kWave;
    for (int64_t i = threadIdx.x; i < b.n_bricks; i += blockDim.x) hist[i] = 0u;
    __syncthreads();
    const int64_t ray0 = (int64_t)blockIdx.x * kHistRays;
    const int64_t ray1 = ray0 + kHistRays < b.n ? ray0 + kHistRays : b.n;
    const uint32_t s0 = b.offsets[ray0], s1 = b.offsets[ray1];
    for (uint32_t w0 = s0 + (uint32_t)wave * kWave; w0 < s1; w0 += (uint32_t)nwaves * kWave) {
        const uint32_t sidx = w0 + lane;
        const bool act = sidx < s1;
        const uint32_t key = act ? b.rec_key[sidx] : 0xffffffffu;
        const int active = (int)min(s1 - w0, (uint32_t)kWave);
        const uint64_t heads = run_heads(key, act);
        if ((heads >> lane) & 1ull) atomicAdd(&hist[key], (uint32_t)run_length(heads, active));
    }
    __syncthreads();
    for (int64_t i = threadIdx.x; i < b.n_bricks; i += blockDim.x) {
        const uint32_t c = hist[i];
        if (c) hist[i] = atomicAdd(&b.brick_off[i], c);
    }
    __syncthreads();
    for (uint32_t w0 = s0 + (uint32_t)wave * kWave; w0 < s1; w0 += (uint32_t)nwaves * kWave) {
        const uint32_t sidx = w0 + lane;
        const bool act = sidx < s1;
        const uint32_t key = act ? b.rec_key[sidx] : 0xffffffffu;
        const int active = (int)min(s1 - w0, (uint32_t)kWave);
        const uint64_t heads = run_heads(key, act);
        uint32_t base = 0;
        if ((heads >> lane) & 1ull) base = atomicAdd(&hist[key], (uint32_t)run_length(heads, active));
        const uint64_t upto = heads & ((lane == kWave - 1) ? ~0ull : ((2ull << lane) - 1ull));
        const int head = upto ? (63 - __clzll((long long)upto)) : 0;
        const uint32_t hb = __shfl(base, head, kWave);
        if (act) b.perm[hb + (uint32_t)(lane - head)] = sidx;
    }
}

void launch_brick_scatter(const RenderBufs &b, hipStream_t s)
{
    if (b.n == 0) return;
    if (use_hist(b)) {
        const unsigned blocks = (unsigned)((b.n + kHistRays - 1) / kHistRays);
        hipLaunchKernelGGL(k_brick_scatter_hist, dim3(blocks), dim3(kHistThreads), b.n_bricks * sizeof(uint32_t), s, b);
        return;
    }
    const unsigned blocks = (unsigned)((b.n + kRayWaves - 1) / kRayWaves);
    hipLaunchKernelGGL(k_brick_scatter, dim3(blocks), dim3(256), 0, s, b);
}

__global__ void k_fill_u32(uint32_t *p, uint32_t v, int64_t n)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        p[i] = v;
}
__global__ void k_fill_u64(uint64_t *p, uint64_t v, int64_t n)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        p[i] = v;
}
static unsigned fill_blocks(int64_t n)
{
    int64_t b = (n + 255) / 256;
    return (unsigned)(b < 1 ? 1 : (b > 8192 ? 8192 : b));
}
void launch_fill_u32(uint32_t *p, uint32_t v, int64_t n, hipStream_t s)
{
    if (n > 0) hipLaunchKernelGGL(k_fill_u32, dim3(fill_blocks(n)), dim3(256), 0, s, p, v, n);
}
void launch_fill_u64(uint64_t *p, uint64_t v, int64_t n, hipStream_t s)
{
    if (n > 0) hipLaunchKernelGGL(k_fill_u64, dim3(fill_blocks(n)), dim3(256), 0, s, p, v, n);
}
__global__ void k_fill_u8(uint8_t *p, uint8_t v, int64_t n)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        p[i] = v;
}
// Segments per brick (ceil(count / kTileSeg)) into seg_off, then their
// exclusive scan: brick k owns segments seg_off[k] .. seg_off[k+1]-1.
__global__ void k_brick_segments(RenderBufs b, uint32_t seg)
{
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= b.n_bricks) return;
    const uint32_t start = k == 0 ? 0u : b.brick_off[k - 1], end = b.brick_off[k];
    b.seg_off[k] = (end - start + seg - 1u) / seg;
}

// Brick of every segment: brick k writes its own segments' entries.
__global__ void k_segment_bricks(RenderBufs b)
{
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= b.n_bricks) return;
    for (uint32_t q = b.seg_off[k]; q < b.seg_off[k + 1]; ++q) b.seg_brick[q] = (uint32_t)k;
}

void launch_brick_segments(const RenderBufs &b, int seg, bool table, hipStream_t s)
{
    if (b.n_bricks > 0)
        hipLaunchKernelGGL(k_brick_segments, dim3((unsigned)((b.n_bricks + 255) / 256)), dim3(256), 0, s, b,
                           (uint32_t)seg);
    launch_exclusive_scan(b.seg_off, b.seg_off, b.brick_tmp, b.n_bricks, s);   // also writes the total
    if (table && b.seg_brick && seg == kTileSeg && b.n_bricks > 0)
        hipLaunchKernelGGL(k_segment_bricks, dim3((unsigned)((b.n_bricks + 255) / 256)), dim3(256), 0, s, b);
}

void launch_fill_u8(uint8_t *p, uint8_t v, int64_t n, hipStream_t s)
{
    if (n > 0) hipLaunchKernelGGL(k_fill_u8, dim3(fill_blocks(n)), dim3(256), 0, s, p, v, n);
}

// Per-ray accumulation: rgb = sum_k w_k c_k + T_stop bg, depth_t,
// acc = 1 - T_stop; frame mode converts to z-depth with the void rule.  One
// wavefront per ray: lanes read consecutive live samples (coalesced) and a
// butterfly sum combines them in a fixed order, so the result does not
// depend on the order in which the MLP stage produced the colours.
// Per-ray accumulation, four rays per wavefront (16 lanes each): lane l of a
// ray's group sums w_k c_k over its live samples l, l + 16, l + 32, ... in
// order, then a 16-lane butterfly adds the lanes' partial sums (a fixed
// order, so the result is deterministic and the same in every sample order
// of the MLP stage).  The four rays' loads go out together, which is what a
// stage bound by the latency of its dependent loads needs (measured on eight
// 800x800 views: 1.55 ms with 16 lanes per ray, 1.82 with 8, 1.64 with 32,
// 2.37 with a wavefront per ray).
constexpr int kReduceLanes = 16;
constexpr int kReduceRays = kRayWaves * (kWave / kReduceLanes);   // rays per 256-thread block

// Sum over the 16 lanes of a DPP row, every lane getting it: rotations of
// the row by 8, 4, 2 and 1 lanes (DPP lane moves, no LDS round trips).
__device__ __forceinline__ float group16_sum(float v)
{
    static_assert(kReduceLanes == 16, "one ray per DPP row");
    v = dpp_add<0x128, 0xf, false>(v);   // row_ror:8
    v = dpp_add<0x124, 0xf, false>(v);   // row_ror:4
    v = dpp_add<0x122, 0xf, false>(v);   // row_ror:2
    v = dpp_add<0x121, 0xf, false>(v);   // row_ror:1
    return v;
}

__global__ __launch_bounds__(256) void k_reduce(RenderBufs b, OptsK op, float *rgb, float *depth, float *acc,
                                                const int32_t *out_map, cic_camera cam, int frame,
                                                unsigned long long *n_eval)
{
    const int sub = (int)(threadIdx.x % kReduceLanes);
    const int64_t ray = (int64_t)blockIdx.x * kReduceRays + (threadIdx.x / kReduceLanes);
    if (n_eval && ray == 0 && sub == 0) atomicAdd(n_eval, (unsigned long long)b.offsets[b.n]);
    const uint32_t n_act = b.n_active ? *b.n_active : (uint32_t)b.n;
    const bool active = ray < b.n && (uint64_t)ray < n_act;
    const uint32_t cnt = active ? b.count[ray] : 0u, off = active ? b.offsets[ray] : 0u;
    float r = 0.f, gg = 0.f, bb = 0.f;
    for (uint32_t j = (uint32_t)sub; j < cnt; j += kReduceLanes) {
        const int64_t k = (int64_t)off + j;
        const float w = b.rec_w[k];
        r = fmaf(w, b.rec_c[3 * k], r);
        gg = fmaf(w, b.rec_c[3 * k + 1], gg);
        bb = fmaf(w, b.rec_c[3 * k + 2], bb);
    }
    r = group16_sum(r);
    gg = group16_sum(gg);
    bb = group16_sum(bb);
    if (!active || sub != 0) return;
    const RayInfo inf = b.info[ray];
    const float ts = inf.t_stop;
    const int64_t out = out_map ? (int64_t)out_map[ray] : ray;
    rgb[3 * out + 0] = fmaf(ts, op.bg[0], r);
    rgb[3 * out + 1] = fmaf(ts, op.bg[1], gg);
    rgb[3 * out + 2] = fmaf(ts, op.bg[2], bb);
    const float a = 1.0f - ts;
    if (acc) acc[out] = a;
    if (frame) {
        float dz = INFINITY;
        if (a >= op.void_acc) {
            const float *d = b.rays_d + 3 * ray;
            const float cosang = fmaf(d[0], cam.c2w[2], fmaf(d[1], cam.c2w[6], d[2] * cam.c2w[10]));
            dz = inf.depth_t / a * cosang;
        }
        depth[out] = dz;
    } else {
        depth[out] = inf.depth_t;
    }
}

void launch_reduce(const RenderBufs &b, const OptsK &o, float *rgb, float *depth, float *acc,
                   const int32_t *out_map, const cic_camera *frame_cam, int64_t *n_eval, hipStream_t s)
{
    const int64_t blocks = (b.n + kReduceRays - 1) / kReduceRays;
    cic_camera cam{};
    if (frame_cam) cam = *frame_cam;
    hipLaunchKernelGGL(k_reduce, dim3((unsigned)(blocks < 1 ? 1 : blocks)), dim3(256), 0, s, b, o, rgb, depth, acc,
                       out_map, cam, frame_cam ? 1 : 0, (unsigned long long *)n_eval);
}

// Pixel rays; pixel index from pix (int64), pix32 (int32) or identity.
__global__ __launch_bounds__(256) void k_generate_rays(cic_camera cam, int64_t n, int64_t base, const int64_t *pix,
                                                       const int32_t *pix32, const uint32_t *n_active, float *o,
                                                       float *d)
{
    const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= n) return;
    if (n_active && (uint64_t)r >= *n_active) return;
    const int64_t p = pix ? pix[r] : (pix32 ? (int64_t)pix32[r] : base + r);
    float oo[3], dd[3];
    pixel_ray(cam, (int)(p % cam.width), (int)(p / cam.width), oo, dd);
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        o[3 * r + a] = oo[a];
        d[3 * r + a] = dd[a];
    }
}

void launch_generate_rays(const cic_camera &cam, int64_t n, int64_t base, const int64_t *pix, const int32_t *pix32,
                          const uint32_t *n_active, float *o, float *d, hipStream_t s)
{
    if (n == 0) return;
    hipLaunchKernelGGL(k_generate_rays, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, cam, n, base, pix, pix32,
                       n_active, o, d);
}

// Occupancy: a voxel is occupied iff any vertex has raw + shift > thr
// (thr = log(expm1(occ_sigma)) rounded to float32 on the host).
template <typename T>
__global__ __launch_bounds__(256) void k_build_occupancy(GridK g, float thr, uint8_t *occ)
{
    const int64_t c1 = g.r1 - 1, c2 = g.r2 - 1;
    const int64_t nc = (int64_t)(g.r0 - 1) * c1 * c2;
    const T *dens = (const T *)g.density;
    for (int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; c < nc; c += (int64_t)gridDim.x * blockDim.x) {
        const int x = (int)(c / (c1 * c2)), y = (int)((c / c2) % c1), z = (int)(c % c2);
        bool any = false;
#pragma unroll
        for (int v = 0; v < 8; ++v) {
            const float s = ldv(dens, vertex_index(g, x + ((v >> 2) & 1), y + ((v >> 1) & 1), z + (v & 1))) + g.shift;
            any |= s > thr;
        }
        occ[c] = any ? 1 : 0;
    }
}

template <typename T>
void launch_build_occupancy(const GridK &g, float thr, uint8_t *occ, hipStream_t s)
{
    const int64_t nc = (int64_t)(g.r0 - 1) * (g.r1 - 1) * (g.r2 - 1);
    hipLaunchKernelGGL(k_build_occupancy<T>, dim3(fill_blocks(nc)), dim3(256), 0, s, g, thr, occ);
}
template void launch_build_occupancy<float>(const GridK &, float, uint8_t *, hipStream_t);
template void launch_build_occupancy<__half>(const GridK &, float, uint8_t *, hipStream_t);

}  // namespace cic
