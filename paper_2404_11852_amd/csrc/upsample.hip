// Bilinear upsampling for the DS-s comparison variant: a frame rendered at
// 1/s resolution is brought back to full size.  Output pixel centre i + 1/2
// sits at (i + 1/2)/s - 1/2 in low-resolution pixel index space; neighbours
// beyond the border are clamped to it.  One thread per output pixel, three
// channels; HBM-bound (12 B written and at most 48 B read per pixel, the
// reads shared through L2 by the s^2 outputs of each input).
#include "kernels.h"

namespace cic {

__global__ __launch_bounds__(256) void k_upsample_bilinear(const float *lo, int w, int h, float *out, int W, int H,
                                                           float inv_s)
{
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= (int64_t)W * H) return;
    const int i = (int)(p % W), j = (int)(p / W);
    const float x = ((float)i + 0.5f) * inv_s - 0.5f;
    const float y = ((float)j + 0.5f) * inv_s - 0.5f;
    const float x0f = floorf(x), y0f = floorf(y);
    const float fx = x - x0f, fy = y - y0f;
    const int x0 = (int)x0f, y0 = (int)y0f;
    const int xa = min(max(x0, 0), w - 1), xb = min(max(x0 + 1, 0), w - 1);
    const int ya = min(max(y0, 0), h - 1), yb = min(max(y0 + 1, 0), h - 1);
    const float *ra = lo + 3 * (int64_t)ya * w, *rb = lo + 3 * (int64_t)yb * w;
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        const float top = (1.0f - fx) * ra[3 * xa + c] + fx * ra[3 * xb + c];
        const float bot = (1.0f - fx) * rb[3 * xa + c] + fx * rb[3 * xb + c];
        out[3 * p + c] = (1.0f - fy) * top + fy * bot;
    }
}

void launch_upsample_bilinear(const float *lo, int w, int h, float *out, int W, int H, int s, hipStream_t st)
{
    const int64_t n = (int64_t)W * H;
    if (n == 0) return;
    hipLaunchKernelGGL(k_upsample_bilinear, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, lo, w, h, out, W, H,
                       1.0f / (float)s);
}

}  // namespace cic
