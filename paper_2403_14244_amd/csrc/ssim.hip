// The loss of the paper (Section 3): the SSIM term and the L1 term.
//
// SSIM: mean structural similarity of a rendered
// image and its target under an 11 x 11 Gaussian window (sigma 1.5, zero outside the
// image), C1 = 0.01^2, C2 = 0.03^2, and its gradient with respect to the rendered image.
//
// Forward: one workgroup per 16 x 16 output tile and channel. The tile's 26 x 26 input
// region is staged in LDS, filtered along rows then columns (the window is separable) for
// the five local statistics (G*x, G*y, G*x^2, G*y^2, G*xy); each pixel forms S and the
// three partial derivatives the backward needs (dS/dm1, dS/de11, dS/de12, with
// m1 = G*x, e11 = G*x^2, e12 = G*xy), which are stored in the workspace. Block sums of S
// are added in FP64 in block order by one workgroup, so the mean is reproducible.
// Backward: the same tiling filters the three derivative maps (the window is symmetric,
// so the transposed filter is the filter) and combines them per pixel:
// dSSIM/dx = (G*dS/dm1 + 2 x G*dS/de11 + y G*dS/de12) / N.
#include "common.h"
#include "kernels.h"

#include <algorithm>

namespace isogs {

namespace {

constexpr int kWin = 11, kHalo = 5, kSpan = kTile + 2 * kHalo;   // 26
constexpr float kC1 = 0.0001f, kC2 = 0.0009f;

struct Window {
    float g[kWin];
};

// Stages a 26 x 26 region of plane `src` around the tile (zero outside the image).
__device__ __forceinline__ void stage_region(float (*dst)[kSpan + 1], const float* __restrict__ src, int x0,
                                             int y0, int width, int height) {
    for (int i = threadIdx.x; i < kSpan * kSpan; i += kTilePixels) {
        const int r = i / kSpan, c = i % kSpan;
        const int y = y0 - kHalo + r, x = x0 - kHalo + c;
        dst[r][c] = (x >= 0 && x < width && y >= 0 && y < height) ? src[(size_t)y * width + x] : 0.0f;
    }
}

struct SsimFwdShared {
    float x[kSpan][kSpan + 1];
    float y[kSpan][kSpan + 1];
    float h[5][kSpan][kTile + 1];   // row-filtered statistics
    double part[kTilePixels / kWave];
};

__global__ void __launch_bounds__(kTilePixels) ssim_fwd_kernel(const float* __restrict__ image,
                                                               const float* __restrict__ target, int width,
                                                               int height, int tiles_x, const Window win,
                                                               float* __restrict__ d_m1, float* __restrict__ d_e11,
                                                               float* __restrict__ d_e12,
                                                               double* __restrict__ block_sum) {
    __shared__ SsimFwdShared sh;
    const uint32_t t = threadIdx.x, tile = blockIdx.x, ch = blockIdx.y;
    const int x0 = (int)(tile % (uint32_t)tiles_x) * kTile, y0 = (int)(tile / (uint32_t)tiles_x) * kTile;
    const size_t plane = (size_t)width * height;
    stage_region(sh.x, image + ch * plane, x0, y0, width, height);
    stage_region(sh.y, target + ch * plane, x0, y0, width, height);
    __syncthreads();
    // rows: 26 rows x 16 output columns
    for (int i = t; i < kSpan * kTile; i += kTilePixels) {
        const int r = i / kTile, c = i % kTile;
        float a[5] = {0.0f, 0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
        for (int k = 0; k < kWin; ++k) {
            const float xv = sh.x[r][c + k], yv = sh.y[r][c + k], g = win.g[k];
            a[0] = fmaf(g, xv, a[0]);
            a[1] = fmaf(g, yv, a[1]);
            a[2] = fmaf(g, xv * xv, a[2]);
            a[3] = fmaf(g, yv * yv, a[3]);
            a[4] = fmaf(g, xv * yv, a[4]);
        }
#pragma unroll
        for (int q = 0; q < 5; ++q) sh.h[q][r][c] = a[q];
    }
    __syncthreads();
    const int r = (int)(t >> 4), c = (int)(t & 15u);
    float m[5] = {0.0f, 0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
    for (int k = 0; k < kWin; ++k) {
        const float g = win.g[k];
#pragma unroll
        for (int q = 0; q < 5; ++q) m[q] = fmaf(g, sh.h[q][r + k][c], m[q]);
    }
    const float m1 = m[0], m2 = m[1];
    const float A1 = 2.0f * m1 * m2 + kC1;
    const float A2 = 2.0f * (m[4] - m1 * m2) + kC2;
    const float B1 = m1 * m1 + m2 * m2 + kC1;
    const float B2 = (m[2] - m1 * m1) + (m[3] - m2 * m2) + kC2;
    const float rB1 = 1.0f / B1, rB2 = 1.0f / B2;
    const float S = A1 * A2 * rB1 * rB2;
    const int px = x0 + c, py = y0 + r;
    const bool in = px < width && py < height;
    if (in) {
        const size_t o = ch * plane + (size_t)py * width + px;
        d_e11[o] = -S * rB2;                      // -A1 A2 / (B1 B2^2)
        d_e12[o] = 2.0f * A1 * rB1 * rB2;         // 2 A1 / (B1 B2)
        d_m1[o] = 2.0f * m2 * (A2 - A1) * rB1 * rB2 - 2.0f * m1 * S * rB1 + 2.0f * m1 * S * rB2;
    }
    double s = in ? (double)S : 0.0;
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o, kWave);
    if ((t & 63u) == 0) sh.part[t >> 6] = s;
    __syncthreads();
    if (t == 0)
        block_sum[(size_t)ch * gridDim.x + tile] = ((sh.part[0] + sh.part[1]) + sh.part[2]) + sh.part[3];
}

// Mean of the block sums, added in block order in FP64 by one workgroup: each thread sums
// a contiguous run, then the runs are added in order.
__global__ void __launch_bounds__(256) ssim_mean_kernel(const double* __restrict__ block_sum, uint32_t n_blocks,
                                                        double inv_n, float* __restrict__ ssim) {
    __shared__ double s_run[256];
    const uint32_t t = threadIdx.x, per = (n_blocks + 255u) / 256u;
    double a = 0.0;
    for (uint32_t i = t * per; i < min(n_blocks, (t + 1u) * per); ++i) a += block_sum[i];
    s_run[t] = a;
    __syncthreads();
    if (t == 0) {
        double tot = 0.0;
        for (int i = 0; i < 256; ++i) tot += s_run[i];
        *ssim = (float)(tot * inv_n);
    }
}

struct SsimBwdShared {
    float d[3][kSpan][kSpan + 1];
    float h[3][kSpan][kTile + 1];
};

__global__ void __launch_bounds__(kTilePixels) ssim_bwd_kernel(const float* __restrict__ image,
                                                               const float* __restrict__ target, int width,
                                                               int height, int tiles_x, const Window win,
                                                               const float* __restrict__ d_m1,
                                                               const float* __restrict__ d_e11,
                                                               const float* __restrict__ d_e12,
                                                               const float* __restrict__ dL_dssim, float inv_n,
                                                               float ssim_w, float l1_w,
                                                               float* __restrict__ dL_dimage) {
    __shared__ SsimBwdShared sh;
    const uint32_t t = threadIdx.x, tile = blockIdx.x, ch = blockIdx.y;
    const int x0 = (int)(tile % (uint32_t)tiles_x) * kTile, y0 = (int)(tile / (uint32_t)tiles_x) * kTile;
    const size_t plane = (size_t)width * height;
    stage_region(sh.d[0], d_m1 + ch * plane, x0, y0, width, height);
    stage_region(sh.d[1], d_e11 + ch * plane, x0, y0, width, height);
    stage_region(sh.d[2], d_e12 + ch * plane, x0, y0, width, height);
    __syncthreads();
    for (int i = t; i < kSpan * kTile; i += kTilePixels) {
        const int r = i / kTile, c = i % kTile;
        float a[3] = {0.0f, 0.0f, 0.0f};
#pragma unroll
        for (int k = 0; k < kWin; ++k) {
            const float g = win.g[k];
#pragma unroll
            for (int q = 0; q < 3; ++q) a[q] = fmaf(g, sh.d[q][r][c + k], a[q]);
        }
#pragma unroll
        for (int q = 0; q < 3; ++q) sh.h[q][r][c] = a[q];
    }
    __syncthreads();
    const int r = (int)(t >> 4), c = (int)(t & 15u);
    const int px = x0 + c, py = y0 + r;
    if (px >= width || py >= height) return;
    float b[3] = {0.0f, 0.0f, 0.0f};
#pragma unroll
    for (int k = 0; k < kWin; ++k) {
        const float g = win.g[k];
#pragma unroll
        for (int q = 0; q < 3; ++q) b[q] = fmaf(g, sh.h[q][r + k][c], b[q]);
    }
    const size_t o = ch * plane + (size_t)py * width + px;
    // dL/dimage = ssim_w g dSSIM/dimage (+ l1_w g sign(image - target) / n for the paper's
    // combined loss), g = dL_dssim[0]
    const float g = *dL_dssim;
    const float scale = ssim_w * g * inv_n;
    float out = scale * (b[0] + 2.0f * image[o] * b[1] + target[o] * b[2]);
    if (l1_w != 0.0f) {
        const float gl = l1_w * g * inv_n, d = image[o] - target[o];
        out += d > 0.0f ? gl : (d < 0.0f ? -gl : 0.0f);
    }
    dL_dimage[o] = out;
}

// The paper's loss (1 - lambda) L1 + lambda (1 - SSIM) from the SSIM mean and the L1 block
// sums (added in block order in FP64, as l1_final_kernel does).
__global__ void __launch_bounds__(256) loss_combine_kernel(const double* __restrict__ l1_blocks, uint32_t n_blocks,
                                                           double inv_n, const float* __restrict__ ssim, double lam,
                                                           float* __restrict__ loss) {
    __shared__ double s_run[256];
    const uint32_t t = threadIdx.x, per = (n_blocks + 255u) / 256u;
    double a = 0.0;
    for (uint32_t i = t * per; i < min(n_blocks, (t + 1u) * per); ++i) a += l1_blocks[i];
    s_run[t] = a;
    __syncthreads();
    if (t == 0) {
        double tot = 0.0;
        for (int i = 0; i < 256; ++i) tot += s_run[i];
        loss[0] = (float)((1.0 - lam) * (tot * inv_n) + lam * (1.0 - (double)*ssim));
        loss[1] = *ssim;
    }
}

Window make_window() {
    Window w{};
    double g[kWin], s = 0.0;
    for (int k = 0; k < kWin; ++k) {
        const double r = (double)(k - kHalo);
        g[k] = exp(-r * r / (2.0 * 1.5 * 1.5));
        s += g[k];
    }
    for (int k = 0; k < kWin; ++k) w.g[k] = (float)(g[k] / s);
    return w;
}

struct SsimWs {
    size_t off_m1, off_e11, off_e12, off_blocks, off_l1, off_scalar, bytes;
};

SsimWs ssim_layout(int32_t channels, int32_t height, int32_t width) {
    const size_t n = (size_t)channels * height * width;
    const size_t blocks = (size_t)channels * ((width + kTile - 1) / kTile) * ((height + kTile - 1) / kTile);
    auto a256 = [](size_t x) { return (x + 255) & ~(size_t)255; };
    SsimWs w{};
    w.off_m1 = 0;
    w.off_e11 = a256(n * 4);
    w.off_e12 = w.off_e11 + a256(n * 4);
    w.off_blocks = w.off_e12 + a256(n * 4);
    w.bytes = w.off_blocks + a256(blocks * 8);
    // the combined loss also keeps the L1 block sums and the SSIM mean
    w.off_l1 = w.bytes;
    w.off_scalar = w.off_l1 + a256(l1_ws_bytes(n));
    return w;
}

}  // namespace

size_t ssim_ws_bytes(int32_t channels, int32_t height, int32_t width) {
    return ssim_layout(channels, height, width).bytes;
}

int launch_ssim_fwd(const float* image, const float* target, int32_t channels, int32_t height, int32_t width,
                    float* ssim, void* ws, hipStream_t stream) {
    const SsimWs L = ssim_layout(channels, height, width);
    char* base = static_cast<char*>(ws);
    const int tx = (width + kTile - 1) / kTile, ty = (height + kTile - 1) / kTile;
    const uint32_t tiles = (uint32_t)(tx * ty);
    double* blocks = reinterpret_cast<double*>(base + L.off_blocks);
    hipLaunchKernelGGL(ssim_fwd_kernel, dim3(tiles, (unsigned)channels), dim3(kTilePixels), 0, stream, image, target,
                       width, height, tx, make_window(), reinterpret_cast<float*>(base + L.off_m1),
                       reinterpret_cast<float*>(base + L.off_e11), reinterpret_cast<float*>(base + L.off_e12),
                       blocks);
    const double n = (double)channels * height * width;
    hipLaunchKernelGGL(ssim_mean_kernel, dim3(1), dim3(256), 0, stream, blocks, tiles * (uint32_t)channels, 1.0 / n,
                       ssim);
    return hipPeekAtLastError() == hipSuccess ? 0 : -1;
}

int launch_ssim_bwd(const float* image, const float* target, int32_t channels, int32_t height, int32_t width,
                    const float* dL_dssim, const void* ws, float* dL_dimage, hipStream_t stream) {
    return launch_ssim_bwd_weighted(image, target, channels, height, width, dL_dssim, ws, 1.0f, 0.0f, dL_dimage,
                                    stream);
}

size_t loss_ws_bytes(int32_t channels, int32_t height, int32_t width) {
    return ssim_layout(channels, height, width).off_scalar + 256;
}

int launch_loss_fwd(const float* image, const float* target, int32_t channels, int32_t height, int32_t width,
                    float lambda, float* loss, void* ws, hipStream_t stream) {
    const SsimWs L = ssim_layout(channels, height, width);
    char* base = static_cast<char*>(ws);
    float* ssim = reinterpret_cast<float*>(base + L.off_scalar);
    if (launch_ssim_fwd(image, target, channels, height, width, ssim, ws, stream)) return -1;
    const uint64_t n = (uint64_t)channels * height * width;
    double* l1b = reinterpret_cast<double*>(base + L.off_l1);
    const uint32_t nb = launch_l1_partial(image, target, n, l1b, stream);
    hipLaunchKernelGGL(loss_combine_kernel, dim3(1), dim3(256), 0, stream, l1b, nb, 1.0 / (double)n, ssim,
                       (double)lambda, loss);
    return hipPeekAtLastError() == hipSuccess ? 0 : -1;
}

int launch_loss_bwd(const float* image, const float* target, int32_t channels, int32_t height, int32_t width,
                    float lambda, const float* dL_dloss, const void* ws, float* dL_dimage, hipStream_t stream) {
    // d/dimage [(1 - lambda) L1 + lambda (1 - SSIM)] = (1 - lambda) dL1 - lambda dSSIM
    return launch_ssim_bwd_weighted(image, target, channels, height, width, dL_dloss, ws, -lambda, 1.0f - lambda,
                                    dL_dimage, stream);
}

int launch_ssim_bwd_weighted(const float* image, const float* target, int32_t channels, int32_t height,
                             int32_t width, const float* dL_dssim, const void* ws, float ssim_w, float l1_w,
                             float* dL_dimage, hipStream_t stream) {
    const SsimWs L = ssim_layout(channels, height, width);
    const char* base = static_cast<const char*>(ws);
    const int tx = (width + kTile - 1) / kTile, ty = (height + kTile - 1) / kTile;
    const float inv_n = (float)(1.0 / ((double)channels * height * width));
    hipLaunchKernelGGL(ssim_bwd_kernel, dim3((unsigned)(tx * ty), (unsigned)channels), dim3(kTilePixels), 0, stream,
                       image, target, width, height, tx, make_window(),
                       reinterpret_cast<const float*>(base + L.off_m1), reinterpret_cast<const float*>(base + L.off_e11),
                       reinterpret_cast<const float*>(base + L.off_e12), dL_dssim, inv_n, ssim_w, l1_w, dL_dimage);
    return hipPeekAtLastError() == hipSuccess ? 0 : -1;
}

}  // namespace isogs

// ---- L1 term of the loss -------------------------------------------------------------
// mean |image - target|: block b sums its contiguous chunk of kL1Chunk values (FP32 per
// lane, then FP64 across the block's lanes in a fixed order); one workgroup adds the block
// sums in FP64 in block order. The backward writes g sign(image - target) / n, sign(0) = 0.
namespace isogs {

namespace {

constexpr int kL1Threads = 256, kL1PerThread = 16;
constexpr uint32_t kL1Chunk = kL1Threads * kL1PerThread;

__global__ void __launch_bounds__(kL1Threads) l1_partial_kernel(const float* __restrict__ image,
                                                                const float* __restrict__ target, uint64_t n,
                                                                double* __restrict__ block_sum) {
    __shared__ double s_w[kL1Threads / kWave];
    const uint64_t base = (uint64_t)blockIdx.x * kL1Chunk;
    float a = 0.0f;
#pragma unroll
    for (int i = 0; i < kL1PerThread; ++i) {
        const uint64_t k = base + (uint64_t)i * kL1Threads + threadIdx.x;
        if (k < n) a += fabsf(image[k] - target[k]);
    }
    double d = (double)a;
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) d += __shfl_xor(d, o, kWave);
    if ((threadIdx.x & 63u) == 0) s_w[threadIdx.x >> 6] = d;
    __syncthreads();
    if (threadIdx.x == 0) block_sum[blockIdx.x] = ((s_w[0] + s_w[1]) + s_w[2]) + s_w[3];
}

__global__ void __launch_bounds__(256) l1_final_kernel(const double* __restrict__ block_sum, uint32_t n_blocks,
                                                       double inv_n, float* __restrict__ loss) {
    __shared__ double s_run[256];
    const uint32_t t = threadIdx.x, per = (n_blocks + 255u) / 256u;
    double a = 0.0;
    for (uint32_t i = t * per; i < min(n_blocks, (t + 1u) * per); ++i) a += block_sum[i];
    s_run[t] = a;
    __syncthreads();
    if (t == 0) {
        double tot = 0.0;
        for (int i = 0; i < 256; ++i) tot += s_run[i];
        *loss = (float)(tot * inv_n);
    }
}

__global__ void __launch_bounds__(kL1Threads) l1_grad_kernel(const float* __restrict__ image,
                                                             const float* __restrict__ target, uint64_t n,
                                                             const float* __restrict__ dL_dloss, float inv_n,
                                                             float* __restrict__ dL_dimage) {
    const float g = *dL_dloss * inv_n;
    for (uint64_t k = (uint64_t)blockIdx.x * kL1Threads + threadIdx.x; k < n; k += (uint64_t)gridDim.x * kL1Threads) {
        const float d = image[k] - target[k];
        dL_dimage[k] = d > 0.0f ? g : (d < 0.0f ? -g : 0.0f);
    }
}

}  // namespace

size_t l1_ws_bytes(uint64_t n) { return ((n + kL1Chunk - 1) / kL1Chunk + 1) * sizeof(double); }

uint32_t launch_l1_partial(const float* image, const float* target, uint64_t n, double* blocks,
                           hipStream_t stream) {
    const uint32_t nb = (uint32_t)((n + kL1Chunk - 1) / kL1Chunk);
    if (nb)
        hipLaunchKernelGGL(l1_partial_kernel, dim3(nb), dim3(kL1Threads), 0, stream, image, target, n, blocks);
    return nb;
}

int launch_l1_fwd(const float* image, const float* target, uint64_t n, float* loss, void* ws, hipStream_t stream) {
    double* blocks = static_cast<double*>(ws);
    const uint32_t nb = launch_l1_partial(image, target, n, blocks, stream);
    hipLaunchKernelGGL(l1_final_kernel, dim3(1), dim3(256), 0, stream, blocks, nb, n ? 1.0 / (double)n : 0.0, loss);
    return hipPeekAtLastError() == hipSuccess ? 0 : -1;
}

int launch_l1_bwd(const float* image, const float* target, uint64_t n, const float* dL_dloss, float* dL_dimage,
                  hipStream_t stream) {
    if (!n) return 0;
    const uint64_t blocks = std::min<uint64_t>((n + kL1Threads - 1) / kL1Threads, 8192);
    hipLaunchKernelGGL(l1_grad_kernel, dim3((unsigned)blocks), dim3(kL1Threads), 0, stream, image, target, n, dL_dloss,
                       (float)(1.0 / (double)n), dL_dimage);
    return hipPeekAtLastError() == hipSuccess ? 0 : -1;
}

}  // namespace isogs
