// The 2D kernel-sum representation of the paper's Section 3 ("Our Method"): an image
// signal as a sum of weighted isotropic kernels (eq. 8) within a support radius (eq. 2),
// with no compositing. It reuses the splatting path's binning and sort: each particle is
// written as a disk of radius D with depth 1, so the stable (tile, depth) sort leaves every
// tile's list in particle order, and every pixel adds its kernels in that fixed order.
#include "common.h"
#include "kernels.h"
#include "raster.h"

namespace isogs {

namespace {

constexpr int kFieldBwdBatch = 64;   // entries staged per step of the backward walk

__device__ __forceinline__ bool bins_ok(const uint32_t* count_p, uint64_t capacity, const int32_t* status) {
    return *status == kStatusOk && (uint64_t)*count_p <= capacity;
}

// Footprint record of every particle, in the layout of the splatting records:
// {mu_x, mu_y, 1/sigma^2, 0} {A_0, A_1, A_2, D}, depth 1 and the member-tile count of the
// disk of radius D (the exact FP32 tile test of the binning). A particle with a
// non-finite parameter or sigma <= 0 gets an all-zero record and no tiles.
__global__ void __launch_bounds__(256) field2d_footprint_kernel(const float* __restrict__ mu,
                                                                const float* __restrict__ sigma,
                                                                const float* __restrict__ amp, uint32_t K,
                                                                int width, int height, float support,
                                                                float4* __restrict__ record,
                                                                float* __restrict__ depth,
                                                                uint32_t* __restrict__ tile_count) {
    const uint32_t k = blockIdx.x * 256u + threadIdx.x;
    if (k >= K) return;
    const float mx = mu[k], my = mu[K + k], s = sigma[k];
    const float a0 = amp[k], a1 = amp[K + k], a2 = amp[2 * (size_t)K + k];
    const bool ok = isfinite(mx) && isfinite(my) && isfinite(s) && s > 0.0f && isfinite(a0) && isfinite(a1) &&
                    isfinite(a2) && isfinite(1.0f / (s * s));
    float4 fp = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
    float4 cr = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
    uint32_t cnt = 0;
    if (ok) {
        fp = make_float4(mx, my, 1.0f / (s * s), 0.0f);
        cr = make_float4(a0, a1, a2, support);
        int tx0, tx1, ty0, ty1;
        const int TX = (width + kTile - 1) / kTile, TY = (height + kTile - 1) / kTile;
        tile_box(mx, my, support, TX, TY, tx0, tx1, ty0, ty1);
        const float r2 = support * support;
        const float w_lim = (float)width - 0.5f, h_lim = (float)height - 0.5f;
        for (int ty = ty0; ty <= ty1; ++ty)
            for (int tx = tx0; tx <= tx1; ++tx) cnt += tile_member(mx, my, r2, tx, ty, w_lim, h_lim) ? 1u : 0u;
    }
    record[2 * (size_t)k] = fp;
    record[2 * (size_t)k + 1] = cr;
    depth[k] = 1.0f;
    tile_count[k] = cnt;
}

// Anisotropic particles (the variant the paper times its kernels against): centre mu,
// rotation angle theta, scales s1, s2; the conic of R(theta) diag(s1^2, s2^2) R(theta)^T
// inverted, in FP64 rounded once: record {mu_x, mu_y, P00, P01} {A_0, A_1, A_2, D} and
// conic_c[k] = P11. Invalid (non-finite parameter, a scale <= 0, a conic entry
// overflowing): all-zero record, no tiles.
__global__ void __launch_bounds__(256) field2d_aniso_footprint_kernel(
    const float* __restrict__ mu, const float* __restrict__ theta, const float* __restrict__ scale,
    const float* __restrict__ amp, uint32_t K, int width, int height, float support, float4* __restrict__ record,
    float* __restrict__ conic_c, float* __restrict__ depth, uint32_t* __restrict__ tile_count) {
    const uint32_t k = blockIdx.x * 256u + threadIdx.x;
    if (k >= K) return;
    const float mx = mu[k], my = mu[K + k], th = theta[k], s1 = scale[k], s2 = scale[K + k];
    const float a0 = amp[k], a1 = amp[K + k], a2 = amp[2 * (size_t)K + k];
    const double c = cos((double)th), sn = sin((double)th);
    const double i1 = 1.0 / ((double)s1 * (double)s1), i2 = 1.0 / ((double)s2 * (double)s2);
    const float p00 = (float)(c * c * i1 + sn * sn * i2), p01 = (float)(c * sn * (i1 - i2));
    const float p11 = (float)(sn * sn * i1 + c * c * i2);
    const bool ok = isfinite(mx) && isfinite(my) && isfinite(th) && isfinite(s1) && isfinite(s2) && s1 > 0.0f &&
                    s2 > 0.0f && isfinite(a0) && isfinite(a1) && isfinite(a2) && isfinite(p00) && isfinite(p01) &&
                    isfinite(p11);
    float4 fp = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
    float4 cr = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
    float pc = 0.0f;
    uint32_t cnt = 0;
    if (ok) {
        fp = make_float4(mx, my, p00, p01);
        cr = make_float4(a0, a1, a2, support);
        pc = p11;
        int tx0, tx1, ty0, ty1;
        const int TX = (width + kTile - 1) / kTile, TY = (height + kTile - 1) / kTile;
        tile_box(mx, my, support, TX, TY, tx0, tx1, ty0, ty1);
        const float r2 = support * support;
        const float w_lim = (float)width - 0.5f, h_lim = (float)height - 0.5f;
        for (int ty = ty0; ty <= ty1; ++ty)
            for (int tx = tx0; tx <= tx1; ++tx) cnt += tile_member(mx, my, r2, tx, ty, w_lim, h_lim) ? 1u : 0u;
    }
    record[2 * (size_t)k] = fp;
    record[2 * (size_t)k + 1] = cr;
    conic_c[k] = pc;
    depth[k] = 1.0f;
    tile_count[k] = cnt;
}

// Kernel value of a staged entry at (dx, dy): isotropic, exp2(-d^2 log2(e)/sigma^2) from
// e.z; anisotropic, exp2(dx (nA dx + nB2 dy) + nC dy^2) from the conic scaled by -log2(e)
// (nA = e.z, nB2 = e.w, nC = the amplitude record's w).
template <bool AN>
__device__ __forceinline__ float field_kernel(float dx, float dy, float d2, const float4& e, float nc) {
    if (!AN) return __builtin_amdgcn_exp2f(-d2 * e.z);
    return __builtin_amdgcn_exp2f(fmaf(dx, fmaf(e.w, dy, e.z * dx), nc * dy * dy));
}

// One workgroup per tile, one lane per pixel. The tile's list is staged through LDS 256
// entries at a time; every lane adds A exp(-d^2/sigma^2) of each staged entry whose support
// holds its pixel centre, in list order. The support decision d2 < D*D is computed one
// rounded operation at a time (the library is built without contraction), as the oracle
// takes it.
template <bool AN>
__device__ __forceinline__ void field_fwd_tile(
    const float4* __restrict__ record, const float* __restrict__ conic_c, const uint32_t* __restrict__ pidx,
    const uint32_t* __restrict__ ranges, const uint32_t* __restrict__ count_p, uint64_t capacity,
    const int32_t* __restrict__ status, int width, int height, int tiles_x, float support, float* __restrict__ image,
    float4* __restrict__ s_pos, float4* __restrict__ s_amp) {
    // s_pos {mu_x, mu_y, log2(e)/sigma^2 or nA, - or nB2}, s_amp {A_0, A_1, A_2, - or nC}
    if (!bins_ok(count_p, capacity, status)) return;
    const uint32_t tile = xcd_swizzle(blockIdx.x, gridDim.x), t = threadIdx.x;
    const int px = (int)(tile % (uint32_t)tiles_x) * kTile + (int)(t & 15u);
    const int py = (int)(tile / (uint32_t)tiles_x) * kTile + (int)(t >> 4);
    const float x = (float)px + 0.5f, y = (float)py + 0.5f;
    const float D2 = support * support;
    const uint32_t start = ranges[2 * tile], end = ranges[2 * tile + 1];
    float c0 = 0.0f, c1 = 0.0f, c2 = 0.0f;
    for (uint32_t b = start; b < end; b += kTilePixels) {
        const uint32_t n = min((uint32_t)kTilePixels, end - b);
        if (t < n) {
            const uint32_t g = pidx[b + t];
            const float4 fp = record[2 * (size_t)g];
            float4 cr = record[2 * (size_t)g + 1];
            if (AN) {
                s_pos[t] = make_float4(fp.x, fp.y, -fp.z * kLog2e, -2.0f * fp.w * kLog2e);
                cr.w = -conic_c[g] * kLog2e;
            } else {
                s_pos[t] = make_float4(fp.x, fp.y, fp.z * kLog2e, 0.0f);
            }
            s_amp[t] = cr;
        }
        __syncthreads();
        for (uint32_t j = 0; j < n; ++j) {
            const float4 e = s_pos[j];
            const float dx = x - e.x, dy = y - e.y;
            const float dx2 = dx * dx, dy2 = dy * dy;
            const float d2 = dx2 + dy2;
            if (d2 < D2) {
                const float4 a = s_amp[j];
                const float g = field_kernel<AN>(dx, dy, d2, e, a.w);
                c0 = fmaf(a.x, g, c0);
                c1 = fmaf(a.y, g, c1);
                c2 = fmaf(a.z, g, c2);
            }
        }
        __syncthreads();
    }
    if (px < width && py < height) {
        const size_t hw = (size_t)width * height, o = (size_t)py * width + px;
        image[o] = c0;
        image[hw + o] = c1;
        image[2 * hw + o] = c2;
    }
}

__global__ void __launch_bounds__(kTilePixels) field2d_fwd_kernel(
    const float4* __restrict__ record, const uint32_t* __restrict__ pidx, const uint32_t* __restrict__ ranges,
    const uint32_t* __restrict__ count_p, uint64_t capacity, const int32_t* __restrict__ status, int width,
    int height, int tiles_x, float support, float* __restrict__ image) {
    __shared__ float4 s_pos[kTilePixels];
    __shared__ float4 s_amp[kTilePixels];
    field_fwd_tile<false>(record, nullptr, pidx, ranges, count_p, capacity, status, width, height, tiles_x, support,
                          image, s_pos, s_amp);
}

__global__ void __launch_bounds__(kTilePixels) field2d_aniso_fwd_kernel(
    const float4* __restrict__ record, const float* __restrict__ conic_c, const uint32_t* __restrict__ pidx,
    const uint32_t* __restrict__ ranges, const uint32_t* __restrict__ count_p, uint64_t capacity,
    const int32_t* __restrict__ status, int width, int height, int tiles_x, float support,
    float* __restrict__ image) {
    __shared__ float4 s_pos[kTilePixels];
    __shared__ float4 s_amp[kTilePixels];
    field_fwd_tile<true>(record, conic_c, pidx, ranges, count_p, capacity, status, width, height, tiles_x, support,
                         image, s_pos, s_amp);
}

// One workgroup per tile; wave w owns the tile's pixels [64 w, 64 w + 64) and the tile's
// list is staged 64 entries at a time. A batch of E entries is spread over the wave's
// lanes entry-major: with E' the power of two >= E, lane l takes entry l mod E' and every
// (64 / E')-th of the wave's pixels from l / E' on, so each lane accumulates the six
// derivative terms (A_0..A_2, mu_x, mu_y, sigma) of one entry over E' pixels in
// registers; the lanes sharing an entry are then summed by a butterfly over the high lane
// bits and the four waves in order. Every sum has a fixed order, so the records are
// bitwise reproducible. Each entry's record {dmu_x, dmu_y, dsigma, 0} {dA_0, dA_1, dA_2, 0}
// is written at its emit position. Pixels outside the image carry dL/dimage = 0.
// Sums per entry: isotropic 6 (the three amplitude terms, then the centre and scale terms
// of dL/dg times 2/sigma^2), anisotropic 8 (the amplitude terms, then t dx, t dy, t dx^2,
// t dx dy, t dy^2 with t = (sum_c w_c A_c) g; the conic enters per particle).
template <bool AN>
constexpr int kFieldTerms = AN ? 8 : 6;

template <bool AN>
struct FieldBwdShared {
    float4 pos[kFieldBwdBatch];   // iso {mu_x, mu_y, 1/sigma^2, log2(e)/sigma^2}; aniso {mu_x, mu_y, nA, nB2}
    float4 amp[kFieldBwdBatch];   // {A_0, A_1, A_2, - or nC}
    uint32_t slot[kFieldBwdBatch];
    float w[3][kTilePixels];      // dL/dimage of the tile's pixels
    float part[kTilePixels / kWave][kFieldBwdBatch][kFieldTerms<AN>];
};

template <bool AN>
__device__ __forceinline__ void field_bwd_tile(
    FieldBwdShared<AN>& sh, const float4* __restrict__ record, const float* __restrict__ conic_c,
    const uint32_t* __restrict__ pidx, const uint32_t* __restrict__ ranges, const uint32_t* __restrict__ offsets,
    const uint32_t* __restrict__ count_p, uint64_t capacity, const int32_t* __restrict__ status, int width,
    int height, int tiles_x, int tiles_y, float support, const float* __restrict__ dL_dimage,
    float4* __restrict__ rec) {
    constexpr int NT = kFieldTerms<AN>;
    float4* s_pos = sh.pos;
    float4* s_amp = sh.amp;
    uint32_t* s_slot = sh.slot;
    auto& s_w = sh.w;
    auto& s_part = sh.part;
    if (!bins_ok(count_p, capacity, status)) return;
    const uint32_t tile = xcd_swizzle(blockIdx.x, gridDim.x), t = threadIdx.x;
    const uint32_t w = t >> 6, lane = t & 63u;
    const int tx = (int)(tile % (uint32_t)tiles_x), ty = (int)(tile / (uint32_t)tiles_x);
    const float D2 = support * support;
    const float w_lim = (float)width - 0.5f, h_lim = (float)height - 0.5f;
    {
        const int px = tx * kTile + (int)(t & 15u), py = ty * kTile + (int)(t >> 4);
        float w0 = 0.0f, w1 = 0.0f, w2 = 0.0f;
        if (px < width && py < height) {
            const size_t hw = (size_t)width * height, o = (size_t)py * width + px;
            w0 = dL_dimage[o];
            w1 = dL_dimage[hw + o];
            w2 = dL_dimage[2 * hw + o];
        }
        s_w[0][t] = w0;
        s_w[1][t] = w1;
        s_w[2][t] = w2;
    }
    const float x0 = (float)(tx * kTile) + 0.5f, y0 = (float)(ty * kTile) + 0.5f;
    const uint32_t start = ranges[2 * tile], end = ranges[2 * tile + 1];
    for (uint32_t b = start; b < end; b += kFieldBwdBatch) {
        const uint32_t n = min((uint32_t)kFieldBwdBatch, end - b);
        if (t < n) {
            const uint32_t g = pidx[b + t];
            const float4 fp = record[2 * (size_t)g];
            float4 cr = record[2 * (size_t)g + 1];
            s_slot[t] = emit_slot(offsets[g], fp.x, fp.y, cr.w, tx, ty, tiles_x, tiles_y, w_lim, h_lim);
            if (AN) {
                s_pos[t] = make_float4(fp.x, fp.y, -fp.z * kLog2e, -2.0f * fp.w * kLog2e);
                cr.w = -conic_c[g] * kLog2e;
            } else {
                s_pos[t] = make_float4(fp.x, fp.y, fp.z, fp.z * kLog2e);
            }
            s_amp[t] = cr;
        }
        __syncthreads();
        // E' = the power of two >= n (uniform), lg = log2(E')
        const uint32_t lg = n > 1 ? 32u - (uint32_t)__builtin_clz(n - 1u) : 0u;
        const uint32_t ep = 1u << lg, e = lane & (ep - 1u), slice = lane >> lg, step = kWave >> lg;
        const bool valid = e < n;
        float4 ent = make_float4(0.0f, 0.0f, 0.0f, 0.0f), amp = ent;
        if (valid) {
            ent = s_pos[e];
            amp = s_amp[e];
        }
        const float inv_s = AN ? 0.0f : sqrtf(ent.z);
        float acc[NT];
#pragma unroll
        for (int q = 0; q < NT; ++q) acc[q] = 0.0f;
        for (uint32_t k = 0; k < ep; ++k) {
            const uint32_t pix = w * kWave + slice + k * step;   // pixel of the tile, row-major
            const float x = x0 + (float)(pix & 15u), y = y0 + (float)(pix >> 4);
            const float dx = x - ent.x, dy = y - ent.y;
            const float dx2 = dx * dx, dy2 = dy * dy;
            const float d2 = dx2 + dy2;
            float g = 0.0f;
            if (valid && d2 < D2) g = AN ? field_kernel<true>(dx, dy, d2, ent, amp.w) : __builtin_amdgcn_exp2f(-d2 * ent.w);
            const float c0 = s_w[0][pix], c1 = s_w[1][pix], c2 = s_w[2][pix];
            acc[0] = fmaf(c0, g, acc[0]);
            acc[1] = fmaf(c1, g, acc[1]);
            acc[2] = fmaf(c2, g, acc[2]);
            if (!AN) {
                // dL/dg times 2/sigma^2: the common factor of the centre and scale terms
                const float k2 = 2.0f * (c0 * amp.x + c1 * amp.y + c2 * amp.z) * g * ent.z;
                acc[3] = fmaf(k2, dx, acc[3]);
                acc[4] = fmaf(k2, dy, acc[4]);
                acc[5] = fmaf(k2 * d2, inv_s, acc[5]);
            } else {
                const float tg = (c0 * amp.x + c1 * amp.y + c2 * amp.z) * g;
                const float tx_ = tg * dx, ty_ = tg * dy;
                acc[3] += tx_;
                acc[4] += ty_;
                acc[5] = fmaf(tx_, dx, acc[5]);
                acc[6] = fmaf(tx_, dy, acc[6]);
                acc[7 % NT] = fmaf(ty_, dy, acc[7 % NT]);
            }
        }
        for (uint32_t o = ep; o < (uint32_t)kWave; o <<= 1) {
#pragma unroll
            for (int q = 0; q < NT; ++q) acc[q] += __shfl_xor(acc[q], (int)o, kWave);
        }
        if (valid && slice == 0) {
#pragma unroll
            for (int q = 0; q < NT; ++q) s_part[w][e][q] = acc[q];
        }
        __syncthreads();
        if (t < n) {
            float r[NT];
#pragma unroll
            for (int q = 0; q < NT; ++q)
                r[q] = ((s_part[0][t][q] + s_part[1][t][q]) + s_part[2][t][q]) + s_part[3][t][q];
            const uint32_t slot = s_slot[t];
            rec[2 * (size_t)slot] = make_float4(r[3], r[4], r[5], AN ? r[6 % NT] : 0.0f);
            rec[2 * (size_t)slot + 1] = make_float4(r[0], r[1], r[2], AN ? r[7 % NT] : 0.0f);
        }
        __syncthreads();
    }
}

__global__ void __launch_bounds__(kTilePixels) field2d_bwd_kernel(
    const float4* __restrict__ record, const uint32_t* __restrict__ pidx, const uint32_t* __restrict__ ranges,
    const uint32_t* __restrict__ offsets, const uint32_t* __restrict__ count_p, uint64_t capacity,
    const int32_t* __restrict__ status, int width, int height, int tiles_x, int tiles_y, float support,
    const float* __restrict__ dL_dimage, float4* __restrict__ rec) {
    __shared__ FieldBwdShared<false> sh;
    field_bwd_tile<false>(sh, record, nullptr, pidx, ranges, offsets, count_p, capacity, status, width, height,
                          tiles_x, tiles_y, support, dL_dimage, rec);
}

__global__ void __launch_bounds__(kTilePixels) field2d_aniso_bwd_kernel(
    const float4* __restrict__ record, const float* __restrict__ conic_c, const uint32_t* __restrict__ pidx,
    const uint32_t* __restrict__ ranges, const uint32_t* __restrict__ offsets, const uint32_t* __restrict__ count_p,
    uint64_t capacity, const int32_t* __restrict__ status, int width, int height, int tiles_x, int tiles_y,
    float support, const float* __restrict__ dL_dimage, float4* __restrict__ rec) {
    __shared__ FieldBwdShared<true> sh;
    field_bwd_tile<true>(sh, record, conic_c, pidx, ranges, offsets, count_p, capacity, status, width, height,
                         tiles_x, tiles_y, support, dL_dimage, rec);
}

// Per particle: the sum of its entries' records in emit order (row-major tiles), written
// as its gradients; a particle with no tiles gets zeros.
__global__ void __launch_bounds__(256) field2d_grad_reduce_kernel(
    const float4* __restrict__ rec, const uint32_t* __restrict__ offsets, const uint32_t* __restrict__ tile_count,
    const uint32_t* __restrict__ count_p, uint64_t capacity, const int32_t* __restrict__ status, uint32_t K,
    float* __restrict__ g_mu, float* __restrict__ g_sigma, float* __restrict__ g_amp) {
    const uint32_t k = blockIdx.x * 256u + threadIdx.x;
    if (k >= K || !bins_ok(count_p, capacity, status)) return;
    const uint32_t e0 = offsets[k], cnt = tile_count[k];
    float a[6] = {0.0f, 0.0f, 0.0f, 0.0f, 0.0f, 0.0f};
    for (uint32_t j = 0; j < cnt; ++j) {
        const float4 p = rec[2 * (size_t)(e0 + j)];
        const float4 q = rec[2 * (size_t)(e0 + j) + 1];
        a[0] += p.x;
        a[1] += p.y;
        a[2] += p.z;
        a[3] += q.x;
        a[4] += q.y;
        a[5] += q.z;
    }
    g_mu[k] = a[0];
    g_mu[K + k] = a[1];
    g_sigma[k] = a[2];
    g_amp[k] = a[3];
    g_amp[K + k] = a[4];
    g_amp[2 * (size_t)K + k] = a[5];
}

// Anisotropic: the sums of the particle's entries (emit order), then the centre and conic
// gradients, dmu_x = 2 (P00 S_x + P01 S_y), dmu_y = 2 (P01 S_x + P11 S_y), dP00 = -S_xx,
// dP01 = -2 S_xy, dP11 = -S_yy, chained in FP64 to theta and the scales through
// P00 = c^2/s1^2 + s^2/s2^2, P01 = c s (1/s1^2 - 1/s2^2), P11 = s^2/s1^2 + c^2/s2^2.
__global__ void __launch_bounds__(256) field2d_aniso_grad_reduce_kernel(
    const float4* __restrict__ rec, const float4* __restrict__ record, const float* __restrict__ conic_c,
    const float* __restrict__ theta, const float* __restrict__ scale, const uint32_t* __restrict__ offsets,
    const uint32_t* __restrict__ tile_count, const uint32_t* __restrict__ count_p, uint64_t capacity,
    const int32_t* __restrict__ status, uint32_t K, float* __restrict__ g_mu, float* __restrict__ g_theta,
    float* __restrict__ g_scale, float* __restrict__ g_amp) {
    const uint32_t k = blockIdx.x * 256u + threadIdx.x;
    if (k >= K || !bins_ok(count_p, capacity, status)) return;
    const uint32_t e0 = offsets[k], cnt = tile_count[k];
    float a[8] = {0.0f, 0.0f, 0.0f, 0.0f, 0.0f, 0.0f, 0.0f, 0.0f};
    for (uint32_t j = 0; j < cnt; ++j) {
        const float4 p = rec[2 * (size_t)(e0 + j)];
        const float4 q = rec[2 * (size_t)(e0 + j) + 1];
        a[0] += p.x;   // t dx
        a[1] += p.y;   // t dy
        a[2] += p.z;   // t dx^2
        a[3] += p.w;   // t dx dy
        a[4] += q.w;   // t dy^2
        a[5] += q.x;
        a[6] += q.y;
        a[7] += q.z;
    }
    float gmx = 0.0f, gmy = 0.0f, gth = 0.0f, gs1 = 0.0f, gs2 = 0.0f;
    if (cnt) {
        const float4 fp = record[2 * (size_t)k];
        const double P00 = fp.z, P01 = fp.w, P11 = conic_c[k];
        const double Sx = a[0], Sy = a[1];
        gmx = (float)(2.0 * (P00 * Sx + P01 * Sy));
        gmy = (float)(2.0 * (P01 * Sx + P11 * Sy));
        const double ga = -(double)a[2], gb = -2.0 * (double)a[3], gc = -(double)a[4];
        const double th = theta[k], s1 = scale[k], s2 = scale[K + k];
        const double c = cos(th), sn = sin(th), i1 = 1.0 / (s1 * s1), i2 = 1.0 / (s2 * s2);
        gth = (float)(ga * 2.0 * c * sn * (i2 - i1) + gb * (c * c - sn * sn) * (i1 - i2) + gc * 2.0 * c * sn * (i1 - i2));
        gs1 = (float)(-2.0 / (s1 * s1 * s1) * (ga * c * c + gb * c * sn + gc * sn * sn));
        gs2 = (float)(-2.0 / (s2 * s2 * s2) * (ga * sn * sn - gb * c * sn + gc * c * c));
    }
    g_mu[k] = gmx;
    g_mu[K + k] = gmy;
    g_theta[k] = gth;
    g_scale[k] = gs1;
    g_scale[K + k] = gs2;
    g_amp[k] = a[5];
    g_amp[K + k] = a[6];
    g_amp[2 * (size_t)K + k] = a[7];
}

isogs_camera field_camera(int32_t width, int32_t height) {
    isogs_camera c{};
    c.width = width;
    c.height = height;
    return c;
}

}  // namespace

BinSortPlan plan_field2d_bin(int32_t K, int32_t width, int32_t height, uint64_t capacity) {
    const isogs_camera cam = field_camera(width, height);
    return plan_bin_sort(&K, &cam, 1, capacity);
}

int launch_field2d_bin(const BinSortPlan& plan, const isogs_field2d* f, int32_t width, int32_t height,
                       float support, const isogs_projected* fp, const isogs_bins* bins, void* ws,
                       hipStream_t stream) {
    const uint32_t K = (uint32_t)f->K;
    if (K)
        hipLaunchKernelGGL(field2d_footprint_kernel, dim3((K + 255) / 256), dim3(256), 0, stream, f->mu, f->sigma,
                           f->amp, K, width, height, support, reinterpret_cast<float4*>(fp->record), fp->depth,
                           fp->tile_count);
    if (hipPeekAtLastError() != hipSuccess) return -1;
    const isogs_camera cam = field_camera(width, height);
    const int32_t n = f->K;
    return launch_bin_sort(plan, fp, &n, &cam, 1, bins, ws, stream);
}

int launch_field2d_fwd(const isogs_projected* fp, const isogs_bins* bins, int32_t width, int32_t height,
                       float support, float* image, hipStream_t stream) {
    const int tx = (width + kTile - 1) / kTile, ty = (height + kTile - 1) / kTile;
    hipLaunchKernelGGL(field2d_fwd_kernel, dim3((unsigned)(tx * ty)), dim3(kTilePixels), 0, stream,
                       reinterpret_cast<const float4*>(fp->record), bins->pidx, bins->ranges, bins->count,
                       bins->capacity, bins->status, width, height, tx, support, image);
    return hipPeekAtLastError() == hipSuccess ? 0 : -1;
}

size_t field2d_bwd_ws(uint64_t capacity) { return (size_t)capacity * 32; }

int launch_field2d_bwd(const isogs_projected* fp, int32_t K, const isogs_bins* bins, int32_t width, int32_t height,
                       float support, const float* dL_dimage, const isogs_field2d* grads, void* ws,
                       hipStream_t stream) {
    const int tx = (width + kTile - 1) / kTile, ty = (height + kTile - 1) / kTile;
    float4* rec = static_cast<float4*>(ws);
    if (bins->capacity)
        hipLaunchKernelGGL(field2d_bwd_kernel, dim3((unsigned)(tx * ty)), dim3(kTilePixels), 0, stream,
                           reinterpret_cast<const float4*>(fp->record), bins->pidx, bins->ranges, bins->offsets,
                           bins->count, bins->capacity, bins->status, width, height, tx, ty, support, dL_dimage,
                           rec);
    if (K > 0)
        hipLaunchKernelGGL(field2d_grad_reduce_kernel, dim3(((uint32_t)K + 255) / 256), dim3(256), 0, stream, rec,
                           bins->offsets, fp->tile_count, bins->count, bins->capacity, bins->status, (uint32_t)K,
                           grads->mu, grads->sigma, grads->amp);
    return hipPeekAtLastError() == hipSuccess ? 0 : -1;
}

int launch_field2d_aniso_bin(const BinSortPlan& plan, const isogs_field2d_aniso* f, int32_t width, int32_t height,
                             float support, const isogs_projected* fp, float* conic_c, const isogs_bins* bins,
                             void* ws, hipStream_t stream) {
    const uint32_t K = (uint32_t)f->K;
    if (K)
        hipLaunchKernelGGL(field2d_aniso_footprint_kernel, dim3((K + 255) / 256), dim3(256), 0, stream, f->mu,
                           f->theta, f->scale, f->amp, K, width, height, support,
                           reinterpret_cast<float4*>(fp->record), conic_c, fp->depth, fp->tile_count);
    if (hipPeekAtLastError() != hipSuccess) return -1;
    const isogs_camera cam = field_camera(width, height);
    const int32_t n = f->K;
    return launch_bin_sort(plan, fp, &n, &cam, 1, bins, ws, stream);
}

int launch_field2d_aniso_fwd(const isogs_projected* fp, const float* conic_c, const isogs_bins* bins, int32_t width,
                             int32_t height, float support, float* image, hipStream_t stream) {
    const int tx = (width + kTile - 1) / kTile, ty = (height + kTile - 1) / kTile;
    hipLaunchKernelGGL(field2d_aniso_fwd_kernel, dim3((unsigned)(tx * ty)), dim3(kTilePixels), 0, stream,
                       reinterpret_cast<const float4*>(fp->record), conic_c, bins->pidx, bins->ranges, bins->count,
                       bins->capacity, bins->status, width, height, tx, support, image);
    return hipPeekAtLastError() == hipSuccess ? 0 : -1;
}

int launch_field2d_aniso_bwd(const isogs_field2d_aniso* f, const isogs_projected* fp, const float* conic_c,
                             const isogs_bins* bins, int32_t width, int32_t height, float support,
                             const float* dL_dimage, const isogs_field2d_aniso* grads, void* ws, hipStream_t stream) {
    const int tx = (width + kTile - 1) / kTile, ty = (height + kTile - 1) / kTile;
    float4* rec = static_cast<float4*>(ws);
    const uint32_t K = (uint32_t)f->K;
    if (bins->capacity)
        hipLaunchKernelGGL(field2d_aniso_bwd_kernel, dim3((unsigned)(tx * ty)), dim3(kTilePixels), 0, stream,
                           reinterpret_cast<const float4*>(fp->record), conic_c, bins->pidx, bins->ranges,
                           bins->offsets, bins->count, bins->capacity, bins->status, width, height, tx, ty, support,
                           dL_dimage, rec);
    if (K)
        hipLaunchKernelGGL(field2d_aniso_grad_reduce_kernel, dim3((K + 255) / 256), dim3(256), 0, stream, rec,
                           reinterpret_cast<const float4*>(fp->record), conic_c, f->theta, f->scale, bins->offsets,
                           fp->tile_count, bins->count, bins->capacity, bins->status, K, grads->mu, grads->theta,
                           grads->scale, grads->amp);
    return hipPeekAtLastError() == hipSuccess ? 0 : -1;
}

}  // namespace isogs
