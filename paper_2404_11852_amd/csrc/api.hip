// C interface: argument validation, workspace carving and the launch
// sequences of each entry point (see include/cicero.h for the contract).
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <cmath>
#include <mutex>
#include <string>
#include <vector>

#include "kernels.h"

using namespace cic;

// Z-buffer of warp_frame_noalloc, for callers that cannot allocate device
// memory: one 64-bit key per target pixel, at most kNoAllocPixels target
// pixels (16 MiB per GPU, held until the process ends).  Host code never
// uses this name as an address: each device's copy is reached through the
// pointer hipGetSymbolAddress returns for it (noalloc_zbuf below).
constexpr int64_t kNoAllocPixels = (int64_t)1 << 21;
static __device__ __align__(256) unsigned long long scratch[kNoAllocPixels];

namespace {

thread_local std::string g_err;

int fail(int code, const char *fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    g_err = buf;
    return code;
}

int ok()
{
    g_err.clear();
    return CIC_OK;
}

// Workspace carving: 256-byte aligned sub-buffers from a base pointer; with
// base == nullptr it only measures.
struct Carver {
    char *base;
    size_t off = 0;
    explicit Carver(void *b) : base((char *)b) {}
    template <typename T> T *take(int64_t count)
    {
        off = (off + 255) & ~(size_t)255;
        T *p = base ? (T *)(base + off) : nullptr;
        off += (size_t)(count > 0 ? count : 0) * sizeof(T);
        return p;
    }
};

bool finite_f(float v) { return std::isfinite(v); }

// cos of the warp-angle limit, float32 from a float64 evaluation; < -1 = off.
float cos_limit(float max_angle_deg)
{
    return max_angle_deg > 0.0f ? (float)std::cos((double)max_angle_deg * 3.14159265358979323846 / 180.0) : -2.0f;
}

int check_grid(const cic_grid *g)
{
    if (!g) return fail(CIC_ERR_INVALID, "grid is NULL");
    for (int a = 0; a < 3; ++a) {
        if (g->res[a] < 2 || g->res[a] > 1024) return fail(CIC_ERR_INVALID, "grid.res[%d]=%d outside [2,1024]", a, g->res[a]);
        if (!finite_f(g->box_lo[a]) || !finite_f(g->box_hi[a]) || !(g->box_hi[a] > g->box_lo[a]))
            return fail(CIC_ERR_INVALID, "grid box axis %d is empty or not finite", a);
    }
    if (g->n_feat != 12) return fail(CIC_ERR_INVALID, "grid.n_feat=%d; only 12 channels are supported", g->n_feat);
    if (g->storage != CIC_F32 && g->storage != CIC_F16)
        return fail(CIC_ERR_INVALID, "grid.storage=%d; must be CIC_F32 or CIC_F16", g->storage);
    if (!finite_f(g->density_shift)) return fail(CIC_ERR_INVALID, "grid.density_shift is not finite");
    if (!g->density) return fail(CIC_ERR_INVALID, "grid.density is NULL");
    if (g->hash_levels == 0) {
        if (!g->features) return fail(CIC_ERR_INVALID, "grid.features is NULL");
        if ((uintptr_t)g->features % 4) return fail(CIC_ERR_INVALID, "grid.features must be 4-byte aligned");
    } else {
        if (g->hash_levels != 4) return fail(CIC_ERR_INVALID, "grid.hash_levels=%d; must be 0 or 4", g->hash_levels);
        for (int l = 0; l < 4; ++l)
            if (g->hash_res[l] < 1 || g->hash_res[l] > 4096)
                return fail(CIC_ERR_INVALID, "grid.hash_res[%d]=%d outside [1,4096]", l, g->hash_res[l]);
        if (g->hash_log2_size < 8 || g->hash_log2_size > 24)
            return fail(CIC_ERR_INVALID, "grid.hash_log2_size=%d outside [8,24]", g->hash_log2_size);
        if (!g->hash_tables) return fail(CIC_ERR_INVALID, "grid.hash_tables is NULL");
        if ((uintptr_t)g->hash_tables % 4)
            return fail(CIC_ERR_INVALID, "grid.hash_tables must be 4-byte aligned");
    }
    return CIC_OK;
}

int check_mlp(const cic_mlp *m)
{
    if (!m) return fail(CIC_ERR_INVALID, "mlp is NULL");
    if (m->compute != CIC_F32 && m->compute != CIC_BF16)
        return fail(CIC_ERR_INVALID, "mlp.compute=%d is not CIC_F32 or CIC_BF16", m->compute);
    if (m->in_dim != 39 || m->hidden != 128 || m->pe_freqs != 4)
        return fail(CIC_ERR_INVALID, "mlp shape in_dim=%d hidden=%d pe_freqs=%d; supported 39/128/4", m->in_dim,
                    m->hidden, m->pe_freqs);
    if (!m->w0 || !m->b0 || !m->w1 || !m->b1 || !m->w2 || !m->b2) return fail(CIC_ERR_INVALID, "mlp weight is NULL");
    return CIC_OK;
}

int check_opts(const cic_opts *o, const cic_grid *g)
{
    if (!o) return fail(CIC_ERR_INVALID, "opts is NULL");
    if (o->n_samples < 1 || o->n_samples > kMaxSamples)
        return fail(CIC_ERR_INVALID, "opts.n_samples=%d outside [1,%d]", o->n_samples, kMaxSamples);
    if (!finite_f(o->et_threshold) || o->et_threshold < 0.f || o->et_threshold >= 1.f)
        return fail(CIC_ERR_INVALID, "opts.et_threshold must be in [0,1)");
    if (o->use_occupancy && (!g || !g->occupancy))
        return fail(CIC_ERR_INVALID, "opts.use_occupancy set but grid.occupancy is NULL");
    if (o->order != CIC_ORDER_RAY && o->order != CIC_ORDER_VOXEL)
        return fail(CIC_ERR_INVALID, "opts.order=%d is not CIC_ORDER_RAY/VOXEL", o->order);
    for (int c = 0; c < 3; ++c)
        if (!finite_f(o->bg[c])) return fail(CIC_ERR_INVALID, "opts.bg is not finite");
    if (!finite_f(o->void_acc) || o->void_acc < 0.f) return fail(CIC_ERR_INVALID, "opts.void_acc must be >= 0");
    if (!finite_f(o->warp_max_angle) || o->warp_max_angle < 0.f || o->warp_max_angle > 180.f)
        return fail(CIC_ERR_INVALID, "opts.warp_max_angle must be in [0, 180] degrees");
    return CIC_OK;
}

int check_camera(const cic_camera *c, const char *what)
{
    if (!c) return fail(CIC_ERR_INVALID, "%s camera is NULL", what);
    if (c->width < 1 || c->width > 16384 || c->height < 1 || c->height > 16384)
        return fail(CIC_ERR_INVALID, "%s camera size %dx%d outside [1,16384]", what, c->width, c->height);
    if (!finite_f(c->f) || !(c->f > 0.f) || !finite_f(c->cx) || !finite_f(c->cy))
        return fail(CIC_ERR_INVALID, "%s camera intrinsics invalid", what);
    for (int i = 0; i < 12; ++i)
        if (!finite_f(c->c2w[i])) return fail(CIC_ERR_INVALID, "%s camera pose is not finite", what);
    return CIC_OK;
}

int64_t n_bricks_of(const cic_grid *g)
{
    int64_t nb = 1;
    for (int a = 0; a < 3; ++a) nb *= (g->res[a] - 1 + kBrick - 1) / kBrick;
    return nb;
}

GridK make_gridk(const cic_grid *g, bool use_occ)
{
    GridK k{};
    k.r0 = g->res[0];
    k.r1 = g->res[1];
    k.r2 = g->res[2];
    for (int a = 0; a < 3; ++a) {
        k.lo[a] = g->box_lo[a];
        k.hi[a] = g->box_hi[a];
        k.scale[a] = (float)(g->res[a] - 1) / (g->box_hi[a] - g->box_lo[a]);
    }
    k.shift = g->density_shift;
    k.density = g->density;
    k.features = g->features;
    k.occ = use_occ ? g->occupancy : nullptr;
    k.nb1 = (g->res[1] - 1 + kBrick - 1) / kBrick;
    k.nb2 = (g->res[2] - 1 + kBrick - 1) / kBrick;
    k.hlevels = g->hash_levels;
    if (g->hash_levels) {
        const int64_t T = (int64_t)1 << g->hash_log2_size;
        k.hmask = (uint32_t)(T - 1);
        k.htab = g->hash_tables;
        for (int l = 0; l < 4; ++l) {
            const int64_t n1 = (int64_t)g->hash_res[l] + 1;
            k.hN[l] = g->hash_res[l];
            k.hdense[l] = n1 * n1 * n1 <= T ? 1 : 0;
            for (int a = 0; a < 3; ++a) k.hscale[l][a] = (float)g->hash_res[l] / (g->box_hi[a] - g->box_lo[a]);
        }
    }
    return k;
}

OptsK make_optsk(const cic_opts *o)
{
    OptsK k{};
    k.n_samples = o->n_samples;
    k.et_threshold = o->et_threshold;
    for (int c = 0; c < 3; ++c) k.bg[c] = o->bg[c];
    k.void_acc = o->void_acc;
    return k;
}

// Carve the buffers of one render pass of nc rays; generated rays live in
// the workspace when gen_rays is set.
RenderBufs carve_render(Carver &cv, int64_t nc, int N, int64_t n_bricks, bool voxel, bool gen_rays)
{
    RenderBufs b{};
    b.n = nc;
    b.n_samples = N;
    const int64_t ns = nc * (int64_t)N;
    if (gen_rays) {
        b.rays_o = cv.take<float>(3 * nc);
        b.rays_d = cv.take<float>(3 * nc);
    }
    b.info = cv.take<RayInfo>(nc);
    b.count = cv.take<uint32_t>(nc);
    b.offsets = cv.take<uint32_t>(nc + 1);
    b.scan_tmp = cv.take<uint32_t>((int64_t)scan_tmp_elems(nc));
    // The per-ray slots are read for the last time by the compaction; the
    // colours (ray order) or the sample permutation (voxel order) are written
    // after it, so they take the same bytes.
    const int64_t kbytes = ((2 * ns + 255) / 256) * 256, slot_bytes = kbytes + 4 * ns;
    char *u = cv.take<char>(voxel ? slot_bytes : std::max(slot_bytes, 12 * ns));
    b.slot_k = (uint16_t *)u;
    b.slot_w = u ? (float *)(u + kbytes) : nullptr;
    b.rec_ray = cv.take<uint32_t>(ns);
    b.rec_k = cv.take<uint16_t>(ns);
    b.rec_w = cv.take<float>(ns);
    b.rec_c = voxel ? cv.take<float>(3 * ns) : (float *)u;
    b.z0 = cv.take<float>(128 * nc);
    b.enc = cv.take<uint32_t>(16 * nc);
    if (voxel) {
        b.rec_key = cv.take<uint32_t>(ns);
        b.brick_off = cv.take<uint32_t>(n_bricks + 1);
        b.brick_tmp = cv.take<uint32_t>((int64_t)scan_tmp_elems(n_bricks));
        b.perm = (uint32_t *)u;
        b.work_ctr = cv.take<uint32_t>(kXcds);
        b.seg_off = cv.take<uint32_t>(n_bricks + 1);
        b.seg_brick = cv.take<uint32_t>(tile_max_segments(n_bricks, ns));
    }
    b.n_bricks = n_bricks;
    return b;
}

struct WarpBufs {
    uint64_t *zbuf;
    int32_t *hole_idx;
    uint32_t *n_holes;
};

WarpBufs carve_warp(Carver &cv, int64_t np, bool holes)
{
    WarpBufs w{};
    w.zbuf = cv.take<uint64_t>(np);
    if (holes) {
        w.hole_idx = cv.take<int32_t>(np);
        w.n_holes = cv.take<uint32_t>(1);
    }
    return w;
}

// render_sequence: warp + sparse-render buffers for the target stream,
// render buffers for the reference stream, two reference frame slots.
struct SeqBufs {
    WarpBufs w;
    RenderBufs a, b;
    float *ref_rgb[2], *ref_dz[2];
};

SeqBufs carve_seq(Carver &cv, int64_t np, const cic_opts *o, int64_t nb)
{
    SeqBufs q{};
    const bool voxel = o->order == CIC_ORDER_VOXEL;
    q.w = carve_warp(cv, np, true);
    q.a = carve_render(cv, np, o->n_samples, nb, voxel, true);
    q.b = carve_render(cv, np, o->n_samples, nb, voxel, true);
    for (int k = 0; k < 2; ++k) {
        q.ref_rgb[k] = cv.take<float>(3 * np);
        q.ref_dz[k] = cv.take<float>(np);
    }
    return q;
}

// Adjoint passes of up to 8192 rays.  The samples are processed in brick
// order (the voxel-order bucketing of the forward) so that the grid
// gradients can be accumulated per brick segment on chip and added to the
// grid once per vertex (measured on the 8192-ray training step: 12.05 ms
// with per-sample global atomics in ray order).
constexpr int64_t kChunkRaysBwd = 8192;

// Extra buffers of a backward pass (after carve_render's).
void carve_backward(Carver &cv, int64_t nc, int N, RenderBufs &b, BackwardBufs &bb)
{
    const int64_t ns = nc * (int64_t)N;
    b.slot_t = cv.take<float>(ns);
    b.rec_t = cv.take<float>(ns);
    bb.partials = cv.take<float>((int64_t)kWgBlocks * kPartialFloats);
    bb.rec_df = cv.take<float>(12 * ns);
    bb.rec_draw = cv.take<float>(ns);
    bb.seg_tiles = cv.take<float>(fg_max_segments(b.n_bricks, ns) * kFgTileFloats);
}

size_t bytes_for(int op, int64_t n, const cic_grid *g, const cic_opts *o)
{
    Carver cv(nullptr);
    const bool voxel = o->order == CIC_ORDER_VOXEL;
    const int64_t nb = n_bricks_of(g);
    switch (op) {
    case CIC_OP_RENDER_RAYS: {
        const int64_t nc = n < kChunkRays ? n : kChunkRays;
        carve_render(cv, nc, o->n_samples, nb, voxel, false);
        break;
    }
    case CIC_OP_RENDER_FRAME: {
        const int64_t nc = n < kChunkRays ? n : kChunkRays;
        carve_render(cv, nc, o->n_samples, nb, voxel, true);
        break;
    }
    case CIC_OP_RENDER_FRAME_SPARW:
        carve_warp(cv, n, true);
        carve_render(cv, n, o->n_samples, nb, voxel, true);
        break;
    case CIC_OP_RENDER_SEQUENCE:
        carve_seq(cv, n, o, nb);
        break;
    case CIC_OP_RENDER_FRAME_DS: {   // low-resolution colour and depth, then one render pass (bounded by n)
        cv.take<float>(3 * n);
        cv.take<float>(n);
        cv.off = (cv.off + 255) & ~(size_t)255;
        const int64_t nc = n < kChunkRays ? n : kChunkRays;
        carve_render(cv, nc, o->n_samples, nb, voxel, true);
        break;
    }
    case CIC_OP_RENDER_BACKWARD: {
        const int64_t nc = n < kChunkRaysBwd ? n : kChunkRaysBwd;
        RenderBufs b = carve_render(cv, nc, o->n_samples, nb, true, false);
        BackwardBufs bb{};
        carve_backward(cv, nc, o->n_samples, b, bb);
        break;
    }
    default:
        return 0;
    }
    return cv.off + 256;
}

// Rays per pass that a workspace of ws_bytes holds for `op` (render_rays,
// render_frame, render_backward): the full pass (up to `cap` rays) when it
// fits, else the largest that does (the rays then run in more passes); 0
// when not even one ray fits.  The pass buffers grow with the pass size.
int64_t pass_rays(int op, int64_t n, const cic_grid *g, const cic_opts *o, size_t ws_bytes, int64_t cap)
{
    const int64_t full = n < cap ? n : cap;
    if (bytes_for(op, full, g, o) <= ws_bytes) return full;
    int64_t lo = 0, hi = full;   // lo rays fit (0: none), hi do not
    while (hi - lo > 1) {
        const int64_t mid = lo + (hi - lo) / 2;
        if (bytes_for(op, mid, g, o) <= ws_bytes) lo = mid;
        else hi = mid;
    }
    return lo;
}

int check_pass(int64_t per, int op, const cic_grid *g, const cic_opts *o, void *ws, size_t ws_bytes, size_t full)
{
    if (per < 1)
        return fail(CIC_ERR_WORKSPACE, "workspace too small: need at least %zu bytes (one ray per pass; %zu for the "
                                       "fewest passes), got %zu",
                    bytes_for(op, 1, g, o), full, ws_bytes);
    if (!ws) return fail(CIC_ERR_INVALID, "workspace is NULL");
    return CIC_OK;
}

// gfx950 check, once per device.
std::mutex g_dev_mu;
int g_dev_ok[64];   // 0 unknown, 1 ok, -1 not gfx950

int check_device()
{
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) {
        (void)hipGetLastError();
        return fail(CIC_ERR_HIP, "no HIP device available");
    }
    std::lock_guard<std::mutex> lk(g_dev_mu);
    if (dev >= 0 && dev < 64 && g_dev_ok[dev] == 0) {
        hipDeviceProp_t p;
        if (hipGetDeviceProperties(&p, dev) != hipSuccess) {
            (void)hipGetLastError();
            return fail(CIC_ERR_HIP, "hipGetDeviceProperties failed");
        }
        g_dev_ok[dev] = strncmp(p.gcnArchName, "gfx950", 6) == 0 ? 1 : -1;
    }
    if (dev < 0 || dev >= 64 || g_dev_ok[dev] != 1) return fail(CIC_ERR_DEVICE, "current device is not gfx950");
    return CIC_OK;
}

int after_launch(const char *what)
{
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return fail(CIC_ERR_HIP, "%s: %s", what, hipGetErrorString(e));
    return ok();
}

int check_ws(size_t need, void *ws, size_t ws_bytes)
{
    if (ws_bytes < need) return fail(CIC_ERR_WORKSPACE, "workspace too small: need %zu bytes, got %zu", need, ws_bytes);
    if (need > 0 && !ws) return fail(CIC_ERR_INVALID, "workspace is NULL");
    return CIC_OK;
}

void *align_ws(void *ws) { return (void *)(((uintptr_t)ws + 255) & ~(uintptr_t)255); }

// Stage timing (benchmarks): events recorded around launches while enabled.
struct TimedLaunch {
    int stage;
    hipEvent_t a, b;
};
struct Timing {
    bool on = false;
    std::vector<TimedLaunch> recs;
    std::vector<hipEvent_t> pool;
    hipEvent_t frame0 = nullptr;          // frame clock of the last render_sequence
    std::vector<hipEvent_t> frames;
    void reset_frames()
    {
        if (frame0) pool.push_back(frame0);
        frame0 = nullptr;
        for (auto e : frames) pool.push_back(e);
        frames.clear();
    }
    hipEvent_t get()
    {
        if (!pool.empty()) {
            hipEvent_t e = pool.back();
            pool.pop_back();
            return e;
        }
        hipEvent_t e = nullptr;
        if (hipEventCreate(&e) != hipSuccess) {
            (void)hipGetLastError();
            return nullptr;
        }
        return e;
    }
};
thread_local Timing g_timing;

// Brackets the launches issued during its lifetime.
struct StageTimer {
    int stage;
    hipStream_t s;
    hipEvent_t a = nullptr;
    StageTimer(int st, hipStream_t str) : stage(st), s(str)
    {
        if (g_timing.on) {
            a = g_timing.get();
            if (a) (void)hipEventRecord(a, s);
        }
    }
    ~StageTimer()
    {
        if (a) {
            hipEvent_t b = g_timing.get();
            if (b) {
                (void)hipEventRecord(b, s);
                g_timing.recs.push_back(TimedLaunch{stage, a, b});
            } else {
                g_timing.pool.push_back(a);
            }
        }
    }
};

// Full render pipeline on one pass of rays.
void run_pipeline(const cic_grid *grid, const GridK &gk, const cic_mlp *mlp, const OptsK &ok_, bool voxel,
                  RenderBufs &b, float *rgb, float *depth, float *acc, const int32_t *out_map,
                  const cic_camera *frame_cam, int64_t *n_eval, hipStream_t s)
{
    const bool f16 = grid->storage == CIC_F16;
    {
        StageTimer t(CIC_STAGE_MARCH, s);
        if (f16) launch_march<__half>(gk, ok_, b, s);
        else launch_march<float>(gk, ok_, b, s);
    }
    {
        StageTimer t(CIC_STAGE_COMPACT, s);
        launch_exclusive_scan(b.count, b.offsets, b.scan_tmp, b.n, s);
        if (voxel) launch_fill_u32(b.brick_off, 0u, b.n_bricks + 1, s);
        launch_compact(gk, b, voxel, s);
        if (voxel) {
            launch_exclusive_scan(b.brick_off, b.brick_off, b.brick_tmp, b.n_bricks, s);
            launch_brick_scatter(b, s);
        }
    }
    if (mlp->compute == CIC_F32) {
        StageTimer t(CIC_STAGE_EMBED, s);
        launch_ray_embed(*mlp, b, s);
    }
    if (mlp->compute == CIC_BF16) {
        StageTimer t(CIC_STAGE_EMBED, s);
        launch_ray_encode_bf16(b, s);
    }
    {
        StageTimer t(CIC_STAGE_MLP, s);
        if (f16) launch_mlp_forward<__half>(gk, *mlp, b, voxel, s);
        else launch_mlp_forward<float>(gk, *mlp, b, voxel, s);
    }
    {
        StageTimer t(CIC_STAGE_REDUCE, s);
        launch_reduce(b, ok_, rgb, depth, acc, out_map, frame_cam, n_eval, s);
    }
}

// Full render of one frame that fits one pass (np <= kChunkRays); b carved
// with generated rays.
void full_frame(const cic_grid *grid, const GridK &gk, const cic_mlp *mlp, const OptsK &ok_, bool voxel,
                RenderBufs b, const cic_camera &cam, float *rgb, float *depth_z, int64_t *n_eval, hipStream_t s)
{
    const int64_t np = (int64_t)cam.width * cam.height;
    b.n_active = nullptr;
    {
        StageTimer t(CIC_STAGE_RAYGEN, s);
        launch_generate_rays(cam, np, 0, nullptr, nullptr, nullptr, (float *)b.rays_o, (float *)b.rays_d, s);
    }
    run_pipeline(grid, gk, mlp, ok_, voxel, b, rgb, depth_z, nullptr, nullptr, &cam, n_eval, s);
}

// Warp from a reference, then render the holes in place (Eq. 4).
void sparw_frame(const cic_grid *grid, const GridK &gk, const cic_mlp *mlp, const cic_opts *opts, const OptsK &ok_,
                 bool voxel, const WarpBufs &w, RenderBufs b, const cic_camera &ref, const float *ref_rgb,
                 const float *ref_dz, const cic_camera &tgt, const float T[12], float *out_rgb, float *out_dz,
                 uint8_t *mask, int64_t *n_masked, int64_t *n_eval, hipStream_t s)
{
    const int64_t np = (int64_t)tgt.width * tgt.height;
    b.n_active = w.n_holes;
    {
        StageTimer t(CIC_STAGE_WARP, s);
        launch_warp(ref, tgt, T, cos_limit(opts->warp_max_angle), ref_rgb, ref_dz, w.zbuf, out_rgb, out_dz, mask,
                    nullptr, w.hole_idx, w.n_holes, s);
    }
    {
        StageTimer t(CIC_STAGE_RAYGEN, s);
        launch_generate_rays(tgt, np, 0, nullptr, w.hole_idx, w.n_holes, (float *)b.rays_o, (float *)b.rays_d, s);
    }
    run_pipeline(grid, gk, mlp, ok_, voxel, b, out_rgb, out_dz, nullptr, w.hole_idx, &tgt, n_eval, s);
    if (n_masked) launch_sparw_finish(w.n_holes, n_masked, s);
}

// Events that order render_sequence's two streams.  They live for one call:
// created at its start and destroyed before it returns (HIP keeps a
// destroyed event's pending record and waits alive until they complete).
struct SeqEvents {
    hipEvent_t start = nullptr, side_end = nullptr, f0 = nullptr, win_end[2] = {}, ref_ready[2] = {};
    hipEvent_t *all(int i)
    {
        hipEvent_t *evs[] = {&start, &side_end, &f0, &win_end[0], &win_end[1], &ref_ready[0], &ref_ready[1]};
        return evs[i];
    }
    static constexpr int kCount = 7;
    int create()
    {
        for (int i = 0; i < kCount; ++i)
            if (hipEventCreateWithFlags(all(i), hipEventDisableTiming) != hipSuccess) {
                (void)hipGetLastError();
                destroy();
                return fail(CIC_ERR_HIP, "could not create the sequence's events");
            }
        return CIC_OK;
    }
    void destroy()
    {
        for (int i = 0; i < kCount; ++i)
            if (*all(i)) {
                (void)hipEventDestroy(*all(i));
                *all(i) = nullptr;
            }
    }
    ~SeqEvents() { destroy(); }
};

// CU masks for render_sequence's partitioned overlap: per XCD, `t` CUs for
// the targets and the rest for the references.  The HIP runtime spreads the
// bits of a stream's CU mask over the chip interleaved: bit i goes to XCD
// i % 8, and within the XCD bit i / 8 goes to shader engine (i / 8) % 4.
// The targets take bits [0, 8t) and the references the rest, so every XCD
// gets t target CUs, and with t a multiple of 4 every shader engine gets the
// same number (the dispatcher deals workgroups to the shader engines in
// turn, so an uneven split would leave the persistent kernels' last
// workgroups waiting).
constexpr int kXcdCount = 8;

int device_cus(int *n)
{
    int dev = 0;
    *n = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(n, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) {
        (void)hipGetLastError();
        return fail(CIC_ERR_HIP, "could not read the CU count");
    }
    return CIC_OK;
}

int check_partition(int t, int *ncu_out)
{
    int ncu = 0, rc;
    if ((rc = device_cus(&ncu))) return rc;
    const int per = ncu / kXcdCount;
    if (ncu % kXcdCount != 0 || per % kXcdCount != 0 || ncu > 1024)
        return fail(CIC_ERR_INVALID, "CU partitioning needs 8 XCDs of a multiple of 8 CUs (device has %d CUs)", ncu);
    if (t < 1 || t >= per) return fail(CIC_ERR_INVALID, "target_cus_per_xcd=%d outside [1,%d]", t, per - 1);
    *ncu_out = ncu;
    return CIC_OK;
}

int check_warp_args(const cic_camera *ref, const cic_camera *tgt, const float ref_T_tgt[12], const float *ref_rgb,
                    const float *ref_depth_z, float max_angle_deg, const float *tgt_rgb, const float *tgt_depth_z,
                    const uint8_t *mask)
{
    int rc;
    if ((rc = check_camera(ref, "reference")) || (rc = check_camera(tgt, "target"))) return rc;
    if (!finite_f(max_angle_deg) || max_angle_deg < 0.f || max_angle_deg > 180.f)
        return fail(CIC_ERR_INVALID, "max_angle_deg must be in [0, 180]");
    if (!ref_T_tgt) return fail(CIC_ERR_INVALID, "ref_T_tgt is NULL");
    for (int i = 0; i < 12; ++i)
        if (!finite_f(ref_T_tgt[i])) return fail(CIC_ERR_INVALID, "ref_T_tgt is not finite");
    if ((int64_t)ref->width * ref->height > 0xffffffffll) return fail(CIC_ERR_INVALID, "reference too large");
    if (!ref_rgb || !ref_depth_z || !tgt_rgb || !tgt_depth_z || !mask)
        return fail(CIC_ERR_INVALID, "frame pointer is NULL");
    return CIC_OK;
}

// Device address of this device's copy of `scratch`, looked up once per
// device (with that device current) and kept.
std::mutex g_scratch_mu;
void *g_scratch_ptr[64];

int noalloc_zbuf(uint64_t **out)
{
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) {
        (void)hipGetLastError();
        return fail(CIC_ERR_HIP, "no HIP device");
    }
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p) {
            (void)hipGetLastError();
            return fail(CIC_ERR_HIP, "hipGetSymbolAddress(scratch) failed: %s", hipGetErrorString(e));
        }
        g_scratch_ptr[dev] = p;
    }
    *out = (uint64_t *)g_scratch_ptr[dev];
    return CIC_OK;
}

void frame_mark(hipStream_t s)
{
    if (!g_timing.on) return;
    hipEvent_t e = g_timing.get();
    if (e) {
        (void)hipEventRecord(e, s);
        g_timing.frames.push_back(e);
    }
}

}  // namespace

extern "C" {

const char *cic_last_error_message(void) { return g_err.c_str(); }

size_t cic_workspace_bytes(int op, int64_t n_items, const cic_grid *grid, const cic_opts *opts)
{
    if (n_items < 0) return 0;
    if (op == CIC_OP_WARP_FRAME) {
        Carver cv(nullptr);
        carve_warp(cv, n_items, false);
        return cv.off + 256;
    }
    if (check_grid(grid) != CIC_OK || check_opts(opts, grid) != CIC_OK) return 0;
    return bytes_for(op, n_items, grid, opts);
}

int build_occupancy(const cic_grid *grid, float occ_sigma, uint8_t *occ, cic_stream_t stream)
{
    int rc = check_grid(grid);
    if (rc) return rc;
    if (!occ) return fail(CIC_ERR_INVALID, "occ is NULL");
    if (!finite_f(occ_sigma) || !(occ_sigma > 0.f)) return fail(CIC_ERR_INVALID, "occ_sigma must be > 0");
    if ((rc = check_device())) return rc;
    const float thr = (float)std::log(std::expm1((double)occ_sigma));
    GridK gk = make_gridk(grid, false);
    if (grid->storage == CIC_F16) launch_build_occupancy<__half>(gk, thr, occ, (hipStream_t)stream);
    else launch_build_occupancy<float>(gk, thr, occ, (hipStream_t)stream);
    return after_launch("build_occupancy");
}

int generate_rays(const cic_camera *cam, int64_t n, const int64_t *pix, float *rays_o, float *rays_d,
                  cic_stream_t stream)
{
    int rc = check_camera(cam, "");
    if (rc) return rc;
    if (n < 0) return fail(CIC_ERR_INVALID, "n < 0");
    if (!pix && n != (int64_t)cam->width * cam->height)
        return fail(CIC_ERR_INVALID, "pix is NULL but n != width*height");
    if (n == 0) return ok();
    if (!rays_o || !rays_d) return fail(CIC_ERR_INVALID, "rays_o/rays_d is NULL");
    if ((rc = check_device())) return rc;
    launch_generate_rays(*cam, n, 0, pix, nullptr, nullptr, rays_o, rays_d, (hipStream_t)stream);
    return after_launch("generate_rays");
}

int render_rays(const cic_grid *grid, const cic_mlp *mlp, const cic_opts *opts, int64_t n_rays, const float *rays_o,
                const float *rays_d, float *rgb, float *depth_t, float *acc, int64_t *n_eval, void *ws,
                size_t ws_bytes, cic_stream_t stream)
{
    int rc;
    if ((rc = check_grid(grid)) || (rc = check_mlp(mlp)) || (rc = check_opts(opts, grid))) return rc;
    if (n_rays < 0) return fail(CIC_ERR_INVALID, "n_rays < 0");
    if (n_rays == 0) return ok();
    if (!rays_o || !rays_d || !rgb || !depth_t || !acc) return fail(CIC_ERR_INVALID, "ray or output pointer is NULL");
    const int64_t per = pass_rays(CIC_OP_RENDER_RAYS, n_rays, grid, opts, ws_bytes, kChunkRays);
    if ((rc = check_pass(per, CIC_OP_RENDER_RAYS, grid, opts, ws, ws_bytes,
                         bytes_for(CIC_OP_RENDER_RAYS, n_rays, grid, opts))))
        return rc;
    if ((rc = check_device())) return rc;
    hipStream_t s = (hipStream_t)stream;
    const bool voxel = opts->order == CIC_ORDER_VOXEL;
    const GridK gk = make_gridk(grid, opts->use_occupancy != 0);
    const OptsK ok_ = make_optsk(opts);
    const int64_t nb = n_bricks_of(grid);
    for (int64_t c0 = 0; c0 < n_rays; c0 += per) {
        const int64_t nc = (n_rays - c0) < per ? (n_rays - c0) : per;
        Carver cv(align_ws(ws));
        RenderBufs b = carve_render(cv, nc, opts->n_samples, nb, voxel, false);
        b.rays_o = rays_o + 3 * c0;
        b.rays_d = rays_d + 3 * c0;
        run_pipeline(grid, gk, mlp, ok_, voxel, b, rgb + 3 * c0, depth_t + c0, acc + c0, nullptr, nullptr, n_eval,
                     s);
    }
    return after_launch("render_rays");
}

int render_frame(const cic_grid *grid, const cic_mlp *mlp, const cic_opts *opts, const cic_camera *cam, float *rgb,
                 float *depth_z, float *acc, int64_t *n_eval, void *ws, size_t ws_bytes, cic_stream_t stream)
{
    int rc;
    if ((rc = check_grid(grid)) || (rc = check_mlp(mlp)) || (rc = check_opts(opts, grid)) ||
        (rc = check_camera(cam, "")))
        return rc;
    if (!rgb || !depth_z) return fail(CIC_ERR_INVALID, "rgb/depth_z is NULL");
    const int64_t np = (int64_t)cam->width * cam->height;
    const int64_t per = pass_rays(CIC_OP_RENDER_FRAME, np, grid, opts, ws_bytes, kChunkRays);
    if ((rc = check_pass(per, CIC_OP_RENDER_FRAME, grid, opts, ws, ws_bytes,
                         bytes_for(CIC_OP_RENDER_FRAME, np, grid, opts))))
        return rc;
    if ((rc = check_device())) return rc;
    hipStream_t s = (hipStream_t)stream;
    const bool voxel = opts->order == CIC_ORDER_VOXEL;
    const GridK gk = make_gridk(grid, opts->use_occupancy != 0);
    const OptsK ok_ = make_optsk(opts);
    const int64_t nb = n_bricks_of(grid);
    for (int64_t c0 = 0; c0 < np; c0 += per) {
        const int64_t nc = (np - c0) < per ? (np - c0) : per;
        Carver cv(align_ws(ws));
        RenderBufs b = carve_render(cv, nc, opts->n_samples, nb, voxel, true);
        {
            StageTimer t(CIC_STAGE_RAYGEN, s);
            launch_generate_rays(*cam, nc, c0, nullptr, nullptr, nullptr, (float *)b.rays_o, (float *)b.rays_d, s);
        }
        run_pipeline(grid, gk, mlp, ok_, voxel, b, rgb + 3 * c0, depth_z + c0, acc ? acc + c0 : nullptr, nullptr,
                     cam, n_eval, s);
    }
    return after_launch("render_frame");
}

int warp_frame(const cic_camera *ref, const cic_camera *tgt, const float ref_T_tgt[12], const float *ref_rgb,
               const float *ref_depth_z, float max_angle_deg, float *tgt_rgb, float *tgt_depth_z, uint8_t *mask,
               int32_t *src_index, void *ws, size_t ws_bytes, cic_stream_t stream)
{
    int rc;
    if ((rc = check_warp_args(ref, tgt, ref_T_tgt, ref_rgb, ref_depth_z, max_angle_deg, tgt_rgb, tgt_depth_z, mask)))
        return rc;
    const int64_t np = (int64_t)tgt->width * tgt->height;
    Carver m(nullptr);
    carve_warp(m, np, false);
    const size_t need = m.off + 256;
    if ((rc = check_ws(need, ws, ws_bytes))) return rc;
    if ((rc = check_device())) return rc;
    Carver cv(align_ws(ws));
    WarpBufs w = carve_warp(cv, np, false);
    {
        StageTimer t(CIC_STAGE_WARP, (hipStream_t)stream);
        launch_warp(*ref, *tgt, ref_T_tgt, cos_limit(max_angle_deg), ref_rgb, ref_depth_z, w.zbuf, tgt_rgb,
                    tgt_depth_z, mask, src_index, nullptr, nullptr, (hipStream_t)stream);
    }
    return after_launch("warp_frame");
}

int warp_frame_noalloc(const cic_camera *ref, const cic_camera *tgt, const float ref_T_tgt[12], const float *ref_rgb,
                       const float *ref_depth_z, float max_angle_deg, float *tgt_rgb, float *tgt_depth_z,
                       uint8_t *mask, int32_t *src_index, cic_stream_t stream)
{
    int rc;
    if ((rc = check_warp_args(ref, tgt, ref_T_tgt, ref_rgb, ref_depth_z, max_angle_deg, tgt_rgb, tgt_depth_z, mask)))
        return rc;
    const int64_t np = (int64_t)tgt->width * tgt->height;
    if (np > kNoAllocPixels)
        return fail(CIC_ERR_INVALID, "target frame has %lld pixels; warp_frame_noalloc handles at most %lld",
                    (long long)np, (long long)kNoAllocPixels);
    if ((rc = check_device())) return rc;
    uint64_t *zbuf = nullptr;
    if ((rc = noalloc_zbuf(&zbuf))) return rc;
    // the warp's first kernel fills the z-buffer with the empty key, so no
    // earlier call's contents are read
    launch_warp(*ref, *tgt, ref_T_tgt, cos_limit(max_angle_deg), ref_rgb, ref_depth_z, zbuf, tgt_rgb, tgt_depth_z,
                mask, src_index, nullptr, nullptr, (hipStream_t)stream);
    return after_launch("warp_frame_noalloc");
}

int render_frame_sparw(const cic_grid *grid, const cic_mlp *mlp, const cic_opts *opts, const cic_camera *ref,
                       const float *ref_rgb, const float *ref_depth_z, const cic_camera *tgt,
                       const float ref_T_tgt[12], float *out_rgb, float *out_depth_z, uint8_t *mask,
                       int64_t *n_masked, int64_t *n_eval, void *ws, size_t ws_bytes, cic_stream_t stream)
{
    int rc;
    if ((rc = check_grid(grid)) || (rc = check_mlp(mlp)) || (rc = check_opts(opts, grid)) ||
        (rc = check_camera(ref, "reference")) || (rc = check_camera(tgt, "target")))
        return rc;
    if (!ref_T_tgt) return fail(CIC_ERR_INVALID, "ref_T_tgt is NULL");
    for (int i = 0; i < 12; ++i)
        if (!finite_f(ref_T_tgt[i])) return fail(CIC_ERR_INVALID, "ref_T_tgt is not finite");
    if (!ref_rgb || !ref_depth_z || !out_rgb || !out_depth_z || !mask)
        return fail(CIC_ERR_INVALID, "frame pointer is NULL");
    const int64_t np = (int64_t)tgt->width * tgt->height;
    if (np > kChunkRays) return fail(CIC_ERR_INVALID, "target frame has %lld pixels; at most %lld", (long long)np,
                                     (long long)kChunkRays);
    const size_t need = bytes_for(CIC_OP_RENDER_FRAME_SPARW, np, grid, opts);
    if ((rc = check_ws(need, ws, ws_bytes))) return rc;
    if ((rc = check_device())) return rc;
    hipStream_t s = (hipStream_t)stream;
    const bool voxel = opts->order == CIC_ORDER_VOXEL;
    const GridK gk = make_gridk(grid, opts->use_occupancy != 0);
    const OptsK ok_ = make_optsk(opts);
    Carver cv(align_ws(ws));
    WarpBufs w = carve_warp(cv, np, true);
    RenderBufs b = carve_render(cv, np, opts->n_samples, n_bricks_of(grid), voxel, true);
    sparw_frame(grid, gk, mlp, opts, ok_, voxel, w, b, *ref, ref_rgb, ref_depth_z, *tgt, ref_T_tgt, out_rgb,
                out_depth_z, mask, n_masked, n_eval, s);
    return after_launch("render_frame_sparw");
}

int render_sequence(const cic_grid *grid, const cic_mlp *mlp, const cic_opts *opts, const cic_camera *cams,
                    int32_t n_frames, int32_t window, float lead, int32_t flags, int32_t target_cus_per_xcd,
                    float *rgb, float *depth_z, uint8_t *mask, int64_t *n_masked, float *ref_c2w, int64_t *n_eval,
                    void *ws, size_t ws_bytes, cic_stream_t stream, cic_stream_t ref_stream)
{
    int rc;
    if ((rc = check_grid(grid)) || (rc = check_mlp(mlp)) || (rc = check_opts(opts, grid))) return rc;
    if (n_frames < 0) return fail(CIC_ERR_INVALID, "n_frames < 0");
    if (n_frames == 0) return ok();
    if (window < 1) return fail(CIC_ERR_INVALID, "window must be >= 1");
    if (!finite_f(lead)) return fail(CIC_ERR_INVALID, "lead is not finite");
    if ((flags & ~(CIC_SEQ_OVERLAP | CIC_SEQ_TEMPORAL)) != 0) return fail(CIC_ERR_INVALID, "unknown flags 0x%x", flags);
    const bool temporal = (flags & CIC_SEQ_TEMPORAL) != 0;
    if (temporal && (flags & CIC_SEQ_OVERLAP))
        return fail(CIC_ERR_INVALID, "CIC_SEQ_TEMPORAL cannot be combined with CIC_SEQ_OVERLAP");
    if (target_cus_per_xcd < 0 || (target_cus_per_xcd > 0 && !(flags & CIC_SEQ_OVERLAP)))
        return fail(CIC_ERR_INVALID, "target_cus_per_xcd needs CIC_SEQ_OVERLAP and must be >= 0");
    if ((flags & CIC_SEQ_OVERLAP) && (!ref_stream || ref_stream == stream))
        return fail(CIC_ERR_INVALID, "CIC_SEQ_OVERLAP needs a reference stream other than the target stream");
    if (!cams) return fail(CIC_ERR_INVALID, "cams is NULL");
    for (int32_t k = 0; k < n_frames; ++k) {
        if ((rc = check_camera(&cams[k], "sequence"))) return rc;
        if (cams[k].width != cams[0].width || cams[k].height != cams[0].height)
            return fail(CIC_ERR_INVALID, "camera %d has another size than camera 0", k);
    }
    if (!rgb || !depth_z || !mask) return fail(CIC_ERR_INVALID, "frame pointer is NULL");
    const int64_t np = (int64_t)cams[0].width * cams[0].height;
    if (np > kChunkRays)
        return fail(CIC_ERR_INVALID, "frame has %lld pixels; at most %lld", (long long)np, (long long)kChunkRays);
    const size_t need = bytes_for(CIC_OP_RENDER_SEQUENCE, np, grid, opts);
    if ((rc = check_ws(need, ws, ws_bytes))) return rc;
    if ((rc = check_device())) return rc;

    if (temporal) {
        // Temp-N: full renders every `window` frames, otherwise a warp from the previous output
        hipStream_t s = (hipStream_t)stream;
        const bool voxel = opts->order == CIC_ORDER_VOXEL;
        const GridK gk = make_gridk(grid, opts->use_occupancy != 0);
        const OptsK ok_ = make_optsk(opts);
        Carver cv(align_ws(ws));
        SeqBufs q = carve_seq(cv, np, opts, n_bricks_of(grid));
        if (g_timing.on) {
            g_timing.reset_frames();
            g_timing.frame0 = g_timing.get();
            if (g_timing.frame0) (void)hipEventRecord(g_timing.frame0, s);
        }
        for (int32_t k = 0; k < n_frames; ++k) {
            float *o_rgb = rgb + 3 * np * k, *o_dz = depth_z + np * k;
            if (k % window == 0) {
                full_frame(grid, gk, mlp, ok_, voxel, q.a, cams[k], o_rgb, o_dz, n_eval, s);
                launch_fill_u8(mask + np * k, 1, np, s);
                if (n_masked) launch_fill_u64((uint64_t *)(n_masked + k), (uint64_t)np, 1, s);
            } else {
                float T[12];
                if (cic_relative_pose(cams[k - 1].c2w, cams[k].c2w, T) != CIC_OK)
                    return fail(CIC_ERR_INVALID, "relative pose failed for frame %d", k);
                sparw_frame(grid, gk, mlp, opts, ok_, voxel, q.w, q.a, cams[k - 1], o_rgb - 3 * np, o_dz - np,
                            cams[k], T, o_rgb, o_dz, mask + np * k, n_masked ? n_masked + k : nullptr, n_eval, s);
            }
            frame_mark(s);
        }
        return after_launch("render_sequence");
    }

    // reference poses (host): R_0 = frame 0, R_{w+1} from the poses known when window w starts
    const int32_t n_win = (n_frames - 1 + window - 1) / window;
    const float steps = lead < 0.f ? 0.5f * (float)window : lead;
    std::vector<cic_camera> refs((size_t)(n_win > 0 ? n_win : 1));
    refs[0] = cams[0];
    for (int32_t w = 0; w + 1 < n_win; ++w) {
        const int32_t sw = 1 + w * window;
        refs[w + 1] = cams[sw];
        if (cic_extrapolate_pose(cams[sw - 1].c2w, cams[sw].c2w, steps, refs[w + 1].c2w) != CIC_OK)
            return fail(CIC_ERR_INVALID, "pose extrapolation failed for reference %d", w + 1);
        if ((rc = check_camera(&refs[w + 1], "extrapolated reference"))) return rc;
        if (ref_c2w) memcpy(ref_c2w + 12 * (size_t)w, refs[w + 1].c2w, 12 * sizeof(float));
    }

    const bool overlap = (flags & CIC_SEQ_OVERLAP) != 0;
    const bool part = target_cus_per_xcd > 0;
    int ncu = 0;
    if (part && (rc = check_partition(target_cus_per_xcd, &ncu))) return rc;
    // s: targets (the caller's stream), sb: references
    hipStream_t s = (hipStream_t)stream;
    hipStream_t sb = overlap ? (hipStream_t)ref_stream : s;
    SeqEvents ev;
    if (overlap && (rc = ev.create())) return rc;
    const bool voxel = opts->order == CIC_ORDER_VOXEL;
    const GridK gk = make_gridk(grid, opts->use_occupancy != 0);
    const OptsK ok_ = make_optsk(opts);
    Carver cv(align_ws(ws));
    SeqBufs q = carve_seq(cv, np, opts, n_bricks_of(grid));
    if (part) {
        q.a.grid_cus = kXcdCount * target_cus_per_xcd;
        q.b.grid_cus = ncu - q.a.grid_cus;
    }
    auto ref_rgb = [&](int32_t w) -> const float * { return w == 0 ? rgb : q.ref_rgb[w & 1]; };
    auto ref_dz = [&](int32_t w) -> const float * { return w == 0 ? depth_z : q.ref_dz[w & 1]; };
    auto render_ref = [&](int32_t w, hipStream_t st) {
        full_frame(grid, gk, mlp, ok_, voxel, q.b, refs[w], q.ref_rgb[w & 1], q.ref_dz[w & 1], n_eval, st);
    };

    if (g_timing.on) {
        g_timing.reset_frames();
        g_timing.frame0 = g_timing.get();
        if (g_timing.frame0) (void)hipEventRecord(g_timing.frame0, s);
    }
    if (overlap) {
        (void)hipEventRecord(ev.start, s);
        (void)hipStreamWaitEvent(sb, ev.start, 0);
    }
    // frame 0: rendered in full; it is R_0
    full_frame(grid, gk, mlp, ok_, voxel, q.a, cams[0], rgb, depth_z, n_eval, s);
    launch_fill_u8(mask, 1, np, s);
    if (n_masked) launch_fill_u64((uint64_t *)n_masked, (uint64_t)np, 1, s);
    frame_mark(s);
    if (overlap) (void)hipEventRecord(ev.f0, s);

    for (int32_t w = 0; w < n_win; ++w) {
        if (overlap) {
            // R_{w+1} renders on the reference stream once the poses it needs are known (the
            // frames before window w are done); its slot was last read by window w - 1.
            if (w + 1 < n_win) {
                (void)hipStreamWaitEvent(sb, w == 0 ? ev.f0 : ev.win_end[(w - 1) & 1], 0);
                render_ref(w + 1, sb);
                (void)hipEventRecord(ev.ref_ready[(w + 1) & 1], sb);
            }
            if (w >= 1) (void)hipStreamWaitEvent(s, ev.ref_ready[w & 1], 0);
        } else if (w >= 1) {
            render_ref(w, s);
        }
        const int32_t first = 1 + w * window;
        const int32_t last = first + window < n_frames ? first + window : n_frames;
        for (int32_t k = first; k < last; ++k) {
            float T[12];
            if (cic_relative_pose(refs[w].c2w, cams[k].c2w, T) != CIC_OK)
                return fail(CIC_ERR_INVALID, "relative pose failed for frame %d", k);
            sparw_frame(grid, gk, mlp, opts, ok_, voxel, q.w, q.a, refs[w], ref_rgb(w), ref_dz(w), cams[k], T,
                        rgb + 3 * np * k, depth_z + np * k, mask + np * k, n_masked ? n_masked + k : nullptr,
                        n_eval, s);
            frame_mark(s);
        }
        if (overlap) (void)hipEventRecord(ev.win_end[w & 1], s);
    }
    if (overlap) {
        // the caller's stream waits for the references' last work
        (void)hipEventRecord(ev.side_end, sb);
        (void)hipStreamWaitEvent(s, ev.side_end, 0);
    }
    return after_launch("render_sequence");
}

int render_frame_ds(const cic_grid *grid, const cic_mlp *mlp, const cic_opts *opts, const cic_camera *cam,
                    int32_t factor, float *rgb, int64_t *n_eval, void *ws, size_t ws_bytes, cic_stream_t stream)
{
    int rc;
    if ((rc = check_grid(grid)) || (rc = check_mlp(mlp)) || (rc = check_opts(opts, grid)) ||
        (rc = check_camera(cam, "")))
        return rc;
    if (factor < 1 || factor > 16) return fail(CIC_ERR_INVALID, "factor=%d outside [1,16]", factor);
    if (!rgb) return fail(CIC_ERR_INVALID, "rgb is NULL");
    const int64_t np = (int64_t)cam->width * cam->height;
    const size_t need = bytes_for(CIC_OP_RENDER_FRAME_DS, np, grid, opts);
    if ((rc = check_ws(need, ws, ws_bytes))) return rc;
    if ((rc = check_device())) return rc;
    hipStream_t s = (hipStream_t)stream;
    cic_camera lo = *cam;
    lo.width = (cam->width + factor - 1) / factor;
    lo.height = (cam->height + factor - 1) / factor;
    lo.f = cam->f / (float)factor;
    lo.cx = cam->cx / (float)factor;
    lo.cy = cam->cy / (float)factor;
    const int64_t nl = (int64_t)lo.width * lo.height;
    const bool voxel = opts->order == CIC_ORDER_VOXEL;
    const GridK gk = make_gridk(grid, opts->use_occupancy != 0);
    const OptsK ok_ = make_optsk(opts);
    const int64_t nb = n_bricks_of(grid);
    Carver c0(align_ws(ws));
    float *lo_rgb = c0.take<float>(3 * np);
    float *lo_dz = c0.take<float>(np);
    const size_t render_off = (c0.off + 255) & ~(size_t)255;
    for (int64_t r0 = 0; r0 < nl; r0 += kChunkRays) {
        const int64_t nc = (nl - r0) < kChunkRays ? (nl - r0) : kChunkRays;
        Carver cv((char *)align_ws(ws) + render_off);
        RenderBufs b = carve_render(cv, nc, opts->n_samples, nb, voxel, true);
        {
            StageTimer t(CIC_STAGE_RAYGEN, s);
            launch_generate_rays(lo, nc, r0, nullptr, nullptr, nullptr, (float *)b.rays_o, (float *)b.rays_d, s);
        }
        run_pipeline(grid, gk, mlp, ok_, voxel, b, lo_rgb + 3 * r0, lo_dz + r0, nullptr, nullptr, &lo, n_eval, s);
    }
    launch_upsample_bilinear(lo_rgb, lo.width, lo.height, rgb, cam->width, cam->height, factor, s);
    return after_launch("render_frame_ds");
}

int render_backward(const cic_grid *grid, const cic_mlp *mlp, const cic_opts *opts, int64_t n_rays,
                    const float *rays_o, const float *rays_d, const float *d_rgb, const float *d_depth_t,
                    const float *d_acc, float *d_density, float *d_features, float *d_w0, float *d_b0, float *d_w1,
                    float *d_b1, float *d_w2, float *d_b2, void *ws, size_t ws_bytes, cic_stream_t stream)
{
    int rc;
    if ((rc = check_grid(grid)) || (rc = check_mlp(mlp)) || (rc = check_opts(opts, grid))) return rc;
    if (grid->storage != CIC_F32) return fail(CIC_ERR_INVALID, "render_backward needs a float32 grid");
    if (grid->hash_levels) return fail(CIC_ERR_INVALID, "render_backward does not support the multi-level encoding");
    if (mlp->compute != CIC_F32) return fail(CIC_ERR_INVALID, "render_backward needs CIC_F32 compute");
    if (n_rays < 0) return fail(CIC_ERR_INVALID, "n_rays < 0");
    if (n_rays == 0) return ok();
    if (!rays_o || !rays_d || !d_rgb) return fail(CIC_ERR_INVALID, "rays or d_rgb is NULL");
    if (!d_density || !d_features || !d_w0 || !d_b0 || !d_w1 || !d_b1 || !d_w2 || !d_b2)
        return fail(CIC_ERR_INVALID, "gradient pointer is NULL");
    const int64_t per = pass_rays(CIC_OP_RENDER_BACKWARD, n_rays, grid, opts, ws_bytes, kChunkRaysBwd);
    if ((rc = check_pass(per, CIC_OP_RENDER_BACKWARD, grid, opts, ws, ws_bytes,
                         bytes_for(CIC_OP_RENDER_BACKWARD, n_rays, grid, opts))))
        return rc;
    if ((rc = check_device())) return rc;
    hipStream_t s = (hipStream_t)stream;
    const GridK gk = make_gridk(grid, opts->use_occupancy != 0);
    const OptsK ok_ = make_optsk(opts);
    const int64_t nb = n_bricks_of(grid);
    for (int64_t c0 = 0; c0 < n_rays; c0 += per) {
        const int64_t nc = (n_rays - c0) < per ? (n_rays - c0) : per;
        Carver cv(align_ws(ws));
        RenderBufs b = carve_render(cv, nc, opts->n_samples, nb, true, false);
        BackwardBufs bb{};
        carve_backward(cv, nc, opts->n_samples, b, bb);
        b.rays_o = rays_o + 3 * c0;
        b.rays_d = rays_d + 3 * c0;
        bb.d_rgb = d_rgb + 3 * c0;
        bb.d_depth_t = d_depth_t ? d_depth_t + c0 : nullptr;
        bb.d_acc = d_acc ? d_acc + c0 : nullptr;
        bb.d_density = d_density;
        bb.d_features = d_features;
        bb.d_w0 = d_w0;
        bb.d_b0 = d_b0;
        bb.d_w1 = d_w1;
        bb.d_b1 = d_b1;
        bb.d_w2 = d_w2;
        bb.d_b2 = d_b2;
        {
            StageTimer t(CIC_STAGE_MARCH, s);
            launch_march<float>(gk, ok_, b, s);
        }
        {
            StageTimer t(CIC_STAGE_COMPACT, s);
            launch_exclusive_scan(b.count, b.offsets, b.scan_tmp, b.n, s);
            launch_fill_u32(b.brick_off, 0u, b.n_bricks + 1, s);
            launch_compact(gk, b, true, s);
            {
                launch_exclusive_scan(b.brick_off, b.brick_off, b.brick_tmp, b.n_bricks, s);
                launch_brick_scatter(b, s);
            }
        }
        {
            // recomputed forward (its colours go to the compositing adjoint),
            // MLP backward and weight gradients
            StageTimer t(CIC_STAGE_BWD_MLP, s);
            launch_mlp_adjoint(gk, *mlp, b, bb, s);
        }
        {
            StageTimer t(CIC_STAGE_BACKWARD, s);
            launch_backward_composite(gk, ok_, b, bb, s);
            launch_feature_grads_bricks(gk, b, bb, s);
        }
    }
    return after_launch("render_backward");
}

int cic_timing_enable(int on)
{
    // every event recorded so far is destroyed: while timing is off the
    // library holds no HIP object
    for (auto &r : g_timing.recs) {
        (void)hipEventDestroy(r.a);
        (void)hipEventDestroy(r.b);
    }
    g_timing.recs.clear();
    g_timing.reset_frames();
    for (auto e : g_timing.pool) (void)hipEventDestroy(e);
    g_timing.pool.clear();
    g_timing.on = on != 0;
    return ok();
}

int cic_stream_create_cu_masked(int32_t target_cus_per_xcd, int32_t role, cic_stream_t *out)
{
    if (!out) return fail(CIC_ERR_INVALID, "out is NULL");
    *out = nullptr;
    if (role != 0 && role != 1) return fail(CIC_ERR_INVALID, "role=%d; 0 = targets, 1 = references", role);
    int rc, ncu = 0;
    if ((rc = check_device()) || (rc = check_partition(target_cus_per_xcd, &ncu))) return rc;
    uint32_t mask[32] = {};
    for (int bit = 0; bit < ncu; ++bit)
        if ((bit < kXcdCount * target_cus_per_xcd) == (role == 0)) mask[bit / 32] |= 1u << (bit % 32);
    hipStream_t st = nullptr;
    if (hipExtStreamCreateWithCUMask(&st, (uint32_t)((ncu + 31) / 32), mask) != hipSuccess) {
        (void)hipGetLastError();
        return fail(CIC_ERR_HIP, "could not create a CU-masked stream");
    }
    *out = (cic_stream_t)st;
    return ok();
}

int cic_stream_destroy(cic_stream_t stream)
{
    if (!stream) return ok();
    if (hipStreamDestroy((hipStream_t)stream) != hipSuccess) {
        (void)hipGetLastError();
        return fail(CIC_ERR_HIP, "hipStreamDestroy failed");
    }
    return ok();
}

int cic_timing_read(double *ms, int64_t *launches, int n_stages)
{
    if (n_stages < 0 || (n_stages > 0 && (!ms || !launches))) return fail(CIC_ERR_INVALID, "bad timing arrays");
    for (int i = 0; i < n_stages; ++i) {
        ms[i] = 0.0;
        launches[i] = 0;
    }
    for (auto &r : g_timing.recs) {
        if (hipEventSynchronize(r.b) != hipSuccess) return fail(CIC_ERR_HIP, "hipEventSynchronize failed");
        float t = 0.f;
        if (hipEventElapsedTime(&t, r.a, r.b) != hipSuccess) return fail(CIC_ERR_HIP, "hipEventElapsedTime failed");
        if (r.stage >= 0 && r.stage < n_stages) {
            ms[r.stage] += t;
            launches[r.stage] += 1;
        }
    }
    return ok();
}

int cic_timing_frames(double *ms, int cap)
{
    if (cap < 0 || (cap > 0 && !ms)) return fail(CIC_ERR_INVALID, "bad frame-clock array");
    const int n = (int)g_timing.frames.size();
    if (n == 0 || !g_timing.frame0) return 0;
    for (int i = 0; i < n && i < cap; ++i) {
        if (hipEventSynchronize(g_timing.frames[i]) != hipSuccess) return fail(CIC_ERR_HIP, "hipEventSynchronize failed");
        float t = 0.f;
        if (hipEventElapsedTime(&t, g_timing.frame0, g_timing.frames[i]) != hipSuccess)
            return fail(CIC_ERR_HIP, "hipEventElapsedTime failed");
        ms[i] = t;
    }
    return n;
}

}  // extern "C"
