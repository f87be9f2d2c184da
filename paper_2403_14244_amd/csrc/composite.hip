// Front-to-back compositing (eq. 4) of every pixel over its tile's depth-sorted entries.
#include "raster.h"

namespace isogs {

// Composites one entry into a pixel's running state (branch-free; the dummy pad record
// has log2(o) = -inf, so alpha = 0 and it changes nothing).
__device__ __forceinline__ void composite_entry(const float4& f, const float4& c, float px, float py, uint32_t pos,
                                                float& T, float& cr, float& cg, float& cb, uint32_t& last,
                                                bool& done) {
    float g;
    float a = entry_alpha(px - f.x, py - f.y, f.z, f.w, g);
    const bool use = (a >= kAlphaMin) && !done;
    a = use ? a : 0.0f;
    const float wgt = a * T;
    cr = fmaf(c.x, wgt, cr);
    cg = fmaf(c.y, wgt, cg);
    cb = fmaf(c.z, wgt, cb);
    T = T * (1.0f - a);
    last = use ? pos : last;
    done = done || (T < kTMin);
}

// One 256-thread workgroup per tile, one lane per pixel; wave w owns quadrant w.
__global__ void __launch_bounds__(256) composite_fwd_kernel(
    const RenderPack pk, const float4* __restrict__ record, const uint32_t* __restrict__ pidx,
    const uint32_t* __restrict__ ranges, const int32_t* __restrict__ status,
    float bg_r, float bg_g, float bg_b, float* __restrict__ image, float* __restrict__ T_final,
    uint32_t* __restrict__ n_last) {
    __shared__ StagedBatch sb;
    if (*status != kStatusOk) return;
    int vi, tx, ty;
    locate_tile(pk, xcd_swizzle(blockIdx.x, gridDim.x), vi, tx, ty);
    const ViewDesc& vd = pk.v[vi];
    const uint32_t t = threadIdx.x, w = t >> 6;
    const int x = tx * kTile + quad_x(t), y = ty * kTile + quad_y(t);
    const bool inside = x < vd.width && y < vd.height;
    const float px = (float)x + 0.5f, py = (float)y + 0.5f;
    const uint32_t gt = vd.tile_base + (uint32_t)(ty * vd.tiles_x + tx);
    const uint32_t start = ranges[2 * gt], end = min(ranges[2 * gt + 1], pk.n_entries_cap);
    const float w_lim = (float)vd.width - 0.5f, h_lim = (float)vd.height - 0.5f;

    float T = 1.0f, cr = 0.0f, cg = 0.0f, cb = 0.0f;
    uint32_t last = 0;
    bool done = !inside;
    for (uint32_t b0 = start; b0 < end; b0 += kBatch) {
        if (__syncthreads_and(done)) break;
        const uint32_t nb = min((uint32_t)kBatch, end - b0);
        const uint32_t n4 = stage_batch<false>(sb, record, pidx, pk.n_particles, b0, nb, false, tx * kTile,
                                               ty * kTile, w_lim, h_lim);
        const uint32_t pos0 = b0 - start + 1;   // 1-based list position of staged slot 0
        for (uint32_t k = 0; k < n4; k += 4) {
            uint32_t j[4];
            list4(sb, w, k, j);
            const float4 f0 = sb.fp[j[0]], f1 = sb.fp[j[1]], f2 = sb.fp[j[2]], f3 = sb.fp[j[3]];
            const float4 c0 = sb.col[j[0]], c1 = sb.col[j[1]], c2 = sb.col[j[2]], c3 = sb.col[j[3]];
            composite_entry(f0, c0, px, py, pos0 + j[0], T, cr, cg, cb, last, done);
            composite_entry(f1, c1, px, py, pos0 + j[1], T, cr, cg, cb, last, done);
            composite_entry(f2, c2, px, py, pos0 + j[2], T, cr, cg, cb, last, done);
            composite_entry(f3, c3, px, py, pos0 + j[3], T, cr, cg, cb, last, done);
            if (ballot64(!done) == 0) break;
        }
    }
    if (!inside) return;
    const size_t hw = (size_t)vd.width * vd.height;
    const size_t pix = (size_t)y * vd.width + x;
    float* img = image + (size_t)3 * vd.pix_off;
    img[pix] = fmaf(T, bg_r, cr);
    img[hw + pix] = fmaf(T, bg_g, cg);
    img[2 * hw + pix] = fmaf(T, bg_b, cb);
    T_final[vd.pix_off + pix] = T;
    n_last[vd.pix_off + pix] = last;
}

int launch_render_fwd(const isogs_projected* proj, const int32_t* n_per_view, const isogs_bins* bins,
                      const isogs_camera* cams, int32_t nv, const float* bg, float* image, float* T_final,
                      uint32_t* n_last, hipStream_t stream) {
    uint32_t p_off = 0, tile_base = 0, pix_off = 0;
    for (int v0 = 0; v0 < nv; v0 += kMaxViews) {
        RenderPack pk{};
        uint32_t blocks;
        fill_render_pack(pk, cams, n_per_view, v0, nv, p_off, tile_base, pix_off, blocks);
        set_render_limits(pk, n_per_view, nv, bins->capacity);
        if (!blocks) continue;
        hipLaunchKernelGGL(composite_fwd_kernel, dim3(blocks), dim3(256), 0, stream, pk,
                           reinterpret_cast<const float4*>(proj->record), bins->pidx, bins->ranges,
                           bins->status, bg[0], bg[1], bg[2], image, T_final, n_last);
        if (hipPeekAtLastError() != hipSuccess) return -1;
    }
    return 0;
}

}  // namespace isogs
