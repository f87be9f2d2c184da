// Tile-raster helpers shared by the forward and backward compositing kernels.
#pragma once

#include "common.h"
#include "kernels.h"

namespace isogs {

constexpr int kBatch = 256;   // entries staged in LDS per round (one per thread)

// Stages one batch of a tile's entries in LDS and builds, for each of the four waves, the
// ordered list of entries whose binning disk touches that wave's 16x4 pixel rows. A wave
// then walks only its own list: footprints are small against a tile, so most entries
// concern one or two of the four waves. Contains __syncthreads.
struct StagedBatch {
    float4 fp[kBatch];      // {u, v, q = log2(e)/s^2, o}
    float4 col[kBatch];     // {r, g, b, radius}
    uint8_t list[4][kBatch];
    uint8_t mask[kBatch];   // waves whose rows each staged entry touches
    uint32_t cnt[4][4];     // [loader wave][target wave]
};

__device__ __forceinline__ uint32_t stage_batch(StagedBatch& sb, const float4* __restrict__ footprint,
                                                const float4* __restrict__ color_radius,
                                                const uint32_t* __restrict__ pidx, uint32_t n_particles,
                                                uint32_t first, uint32_t n_in_batch, bool reverse, int tile_x0,
                                                int tile_y0, float w_lim, float h_lim) {
    const uint32_t t = threadIdx.x, w = t >> 6;
    uint32_t mask = 0;
    const uint32_t e = reverse ? first + n_in_batch - 1 - t : first + t;
    const uint32_t g = t < n_in_batch ? pidx[e] : 0xFFFFFFFFu;
    // reverse batches are staged back to front so lists run in decreasing depth order
    if (g < n_particles) {
        float4 f = footprint[g];
        const float4 c = color_radius[g];
        f.z *= kLog2e;
        sb.fp[t] = f;
        sb.col[t] = c;
        const float r2 = c.w * c.w;
        const float x_lo = (float)tile_x0 + 0.5f, x_hi = fminf((float)tile_x0 + 15.5f, w_lim);
#pragma unroll
        for (int ww = 0; ww < 4; ++ww) {
            const float y_lo = (float)(tile_y0 + 4 * ww) + 0.5f;
            const float y_hi = fminf((float)(tile_y0 + 4 * ww) + 3.5f, h_lim);
            const float dx = fmaxf(fmaxf(x_lo - f.x, f.x - x_hi), 0.0f);
            const float dy = fmaxf(fmaxf(y_lo - f.y, f.y - y_hi), 0.0f);
            // rows beyond the image (y_lo > h_lim) have no pixels
            if (y_lo <= h_lim && dx * dx + dy * dy <= r2) mask |= 1u << ww;
        }
    }
    sb.mask[t] = (uint8_t)mask;
    uint64_t bal[4];
#pragma unroll
    for (int ww = 0; ww < 4; ++ww) bal[ww] = ballot64((mask >> ww) & 1u);
    if (lane_id() == 0) {
#pragma unroll
        for (int ww = 0; ww < 4; ++ww) sb.cnt[w][ww] = (uint32_t)__popcll(bal[ww]);
    }
    __syncthreads();
#pragma unroll
    for (int ww = 0; ww < 4; ++ww) {
        if ((mask >> ww) & 1u) {
            uint32_t pos = rank_below(bal[ww]);
            for (uint32_t lw = 0; lw < w; ++lw) pos += sb.cnt[lw][ww];
            sb.list[ww][pos] = (uint8_t)t;
        }
    }
    const uint32_t mine = sb.cnt[0][w] + sb.cnt[1][w] + sb.cnt[2][w] + sb.cnt[3][w];
    __syncthreads();
    return __builtin_amdgcn_readfirstlane(mine);
}

struct RenderPack {
    int32_t nv;
    uint32_t n_particles;                  // packed particles of the whole batch
    uint32_t n_entries_cap;                // entry capacity of the bins
    uint32_t block_begin[kMaxViews + 1];   // tiles of earlier views in this launch
    ViewDesc v[kMaxViews];
};

__device__ __forceinline__ void locate_tile(const RenderPack& pk, uint32_t logical, int& vi, int& tx, int& ty) {
    int v = 0;
    for (int i = 1; i < pk.nv; ++i) v = (logical >= pk.block_begin[i]) ? i : v;
    vi = __builtin_amdgcn_readfirstlane(v);
    const uint32_t local = logical - pk.block_begin[vi];
    tx = (int)(local % (uint32_t)pk.v[vi].tiles_x);
    ty = (int)(local / (uint32_t)pk.v[vi].tiles_x);
}

static inline void fill_render_pack(RenderPack& pk, const isogs_camera* cams, const int32_t* n_per_view, int v0, int nv,
                             uint32_t& p_off, uint32_t& tile_base, uint32_t& pix_off, uint32_t& blocks) {
    pk.nv = min(kMaxViews, nv - v0);
    blocks = 0;
    for (int j = 0; j < pk.nv; ++j) {
        const isogs_camera& cam = cams[v0 + j];
        ViewDesc& d = pk.v[j];
        d.p_off = p_off;
        d.n = (uint32_t)n_per_view[v0 + j];
        d.tile_base = tile_base;
        d.pix_off = pix_off;
        d.width = cam.width;
        d.height = cam.height;
        d.tiles_x = (cam.width + kTile - 1) / kTile;
        d.tiles_y = (cam.height + kTile - 1) / kTile;
        pk.block_begin[j] = blocks;
        blocks += (uint32_t)(d.tiles_x * d.tiles_y);
        p_off += d.n;
        tile_base += (uint32_t)(d.tiles_x * d.tiles_y);
        pix_off += (uint32_t)(cam.width * cam.height);
    }
    pk.block_begin[pk.nv] = blocks;
}

// Sets the batch-wide fields of a render pack.
static inline void set_render_limits(RenderPack& pk, const int32_t* n_per_view, int nv, uint64_t capacity) {
    uint64_t n = 0;
    for (int v = 0; v < nv; ++v) n += (uint64_t)n_per_view[v];
    pk.n_particles = (uint32_t)n;
    pk.n_entries_cap = (uint32_t)(capacity < 0xFFFFFFFFull ? capacity : 0xFFFFFFFFull);
}

}  // namespace isogs
