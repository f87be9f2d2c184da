// Tile-raster helpers shared by the forward and backward compositing kernels.
#pragma once

#include "common.h"
#include "kernels.h"

namespace isogs {

constexpr int kBatch = 256;   // entries staged in LDS per round (one per thread)
constexpr int kDummy = kBatch; // staged slot of a zero-opacity record that pads wave lists

// Pixel of lane l in wave w of a tile workgroup: the four waves own the four 8x8
// quadrants of the 16x16 tile (a square quadrant is touched by fewer small disks than a
// 16x4 strip of the same area).
__device__ __forceinline__ int quad_x(uint32_t t) { return (int)(((t >> 6) & 1u) * 8u + (t & 7u)); }
__device__ __forceinline__ int quad_y(uint32_t t) { return (int)(((t >> 6) >> 1) * 8u + ((t >> 3) & 7u)); }

// One batch of a tile's entries staged in LDS, plus, for each of the four waves, the
// ordered list of staged entries whose binning disk touches that wave's quadrant. A wave
// walks only its own list: footprints are small against a tile, so most entries concern
// one or two quadrants. Lists are padded to a multiple of four with kDummy.
struct StagedBatch {
    float4 fp[kBatch + 1];      // {u, v, q = log2(e)/s^2, log2(o)}
    float4 col[kBatch + 1];     // {r, g, b, o}
    uint16_t list[4][kBatch + 4];
    uint8_t mask[kBatch];       // quadrants each staged entry touches
    uint32_t slot[kBatch];      // emit position of each staged entry (backward only)
    uint32_t cnt[4][4];         // [loader wave][target wave]
};

// Emit position of the entry (particle with footprint u, v, r; tile tx, ty): the
// particle's offset plus the number of its member tiles before (tx, ty) in row-major
// order, counted with the same FP32 test the binning used.
__device__ __forceinline__ uint32_t emit_slot(uint32_t offset, float u, float v, float r, int tx, int ty,
                                              int tiles_x, int tiles_y, float w_lim, float h_lim) {
    int tx0, tx1, ty0, ty1;
    tile_box(u, v, r, tiles_x, tiles_y, tx0, tx1, ty0, ty1);
    const float r2 = r * r;
    uint32_t j = 0;
    for (int yy = ty0; yy <= ty; ++yy) {
        const int xe = (yy == ty) ? tx - 1 : tx1;
        for (int xx = tx0; xx <= xe; ++xx) j += tile_member(u, v, r2, xx, yy, w_lim, h_lim) ? 1u : 0u;
    }
    return offset + j;
}

// Stages entries [first, first + n_in_batch) (reversed when `reverse`, so lists then run
// back to front). Returns the length of the calling wave's padded list (a multiple of 4).
// Contains __syncthreads.
template <bool WITH_SLOT>
__device__ __forceinline__ uint32_t stage_batch(StagedBatch& sb, const float4* __restrict__ record,
                                                const uint32_t* __restrict__ pidx, uint32_t n_particles,
                                                uint32_t first, uint32_t n_in_batch, bool reverse, int tile_x0,
                                                int tile_y0, float w_lim, float h_lim,
                                                const uint32_t* __restrict__ offsets = nullptr,
                                                int tiles_x = 0, int tiles_y = 0) {
    const uint32_t t = threadIdx.x, w = t >> 6;
    uint32_t mask = 0;
    const uint32_t e = reverse ? first + n_in_batch - 1 - t : first + t;
    const uint32_t g = t < n_in_batch ? pidx[e] : 0xFFFFFFFFu;
    if (WITH_SLOT) sb.slot[t] = 0xFFFFFFFFu;
    if (g < n_particles) {
        const float4 f = record[2 * (size_t)g];
        const float4 c = record[2 * (size_t)g + 1];
        if (WITH_SLOT)
            sb.slot[t] = emit_slot(offsets[g], f.x, f.y, c.w, tile_x0 / kTile, tile_y0 / kTile, tiles_x, tiles_y,
                                   w_lim, h_lim);
        sb.fp[t] = make_float4(f.x, f.y, f.z * kLog2e, __builtin_amdgcn_logf(f.w));
        sb.col[t] = make_float4(c.x, c.y, c.z, f.w);
        const float r2 = c.w * c.w;
#pragma unroll
        for (int ww = 0; ww < 4; ++ww) {
            const float x_lo = (float)(tile_x0 + (ww & 1) * 8) + 0.5f;
            const float y_lo = (float)(tile_y0 + (ww >> 1) * 8) + 0.5f;
            const float x_hi = fminf(x_lo + 7.0f, w_lim), y_hi = fminf(y_lo + 7.0f, h_lim);
            const float dx = fmaxf(fmaxf(x_lo - f.x, f.x - x_hi), 0.0f);
            const float dy = fmaxf(fmaxf(y_lo - f.y, f.y - y_hi), 0.0f);
            // a quadrant starting beyond the image has no pixels
            if (x_lo <= w_lim && y_lo <= h_lim && dx * dx + dy * dy <= r2) mask |= 1u << ww;
        }
    }
    if (t == 0) {
        sb.fp[kDummy] = make_float4(0.0f, 0.0f, 0.0f, -__builtin_inff());
        sb.col[kDummy] = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
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
            pos += (w > 0 ? sb.cnt[0][ww] : 0u) + (w > 1 ? sb.cnt[1][ww] : 0u) + (w > 2 ? sb.cnt[2][ww] : 0u);
            sb.list[ww][pos] = (uint16_t)t;
        }
    }
    const uint32_t mine = __builtin_amdgcn_readfirstlane(sb.cnt[0][w] + sb.cnt[1][w] + sb.cnt[2][w] + sb.cnt[3][w]);
    const uint32_t padded = (mine + 3u) & ~3u;
    const uint32_t lane = lane_id();
    if (lane < 4 && mine + lane < padded) sb.list[w][mine + lane] = (uint16_t)kDummy;
    __syncthreads();
    return padded;
}

// Four consecutive entries of a wave's list (uniform: scalar registers).
__device__ __forceinline__ void list4(const StagedBatch& sb, uint32_t w, uint32_t k, uint32_t j[4]) {
    const uint64_t q = *reinterpret_cast<const uint64_t*>(&sb.list[w][k]);
    const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)q);
    const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(q >> 32));
    j[0] = lo & 0xFFFFu;
    j[1] = lo >> 16;
    j[2] = hi & 0xFFFFu;
    j[3] = hi >> 16;
}

// ---- Forward-pass staging with 4x4 sub-blocks -------------------------------------------
// Each wave owns an 8x8 quadrant; its four 16-lane rows own the quadrant's four 4x4
// sub-blocks (lane l: row g = l / 16 covers sub-block g, pixel (l % 4, (l / 4) % 4)). Every
// sub-block gets its own ordered list of the staged entries whose binning disk touches
// it, and the rows of a wave walk their lists side by side: a footprint much smaller than
// a quadrant costs a quarter of a wave step instead of a full one.
__device__ __forceinline__ int sub_x(uint32_t t) {
    return (int)(((t >> 6) & 1u) * 8u + (((t >> 4) & 3u) & 1u) * 4u + (t & 3u));
}
__device__ __forceinline__ int sub_y(uint32_t t) {
    return (int)(((t >> 6) >> 1) * 8u + (((t >> 4) & 3u) >> 1) * 4u + ((t >> 2) & 3u));
}

struct StagedSub {
    float4 fp[kBatch + 1];      // {u, v, q = log2(e)/s^2, log2(o)}
    float4 col[kBatch + 1];     // {r, g, b, o}
    uint16_t list[16][kBatch + 4];
    uint32_t cnt[4][16];        // [loader wave][sub-block]
    uint32_t len[16];           // padded list lengths (multiples of 4)
};

// Stages entries [first, first + n_in_batch) and builds the 16 sub-block lists. Returns the
// number of list steps of the calling wave (the longest of its four rows' padded lists).
// Contains __syncthreads.
__device__ __forceinline__ uint32_t stage_batch_sub(StagedSub& sb, const float4* __restrict__ record,
                                                    const uint32_t* __restrict__ pidx, uint32_t n_particles,
                                                    uint32_t first, uint32_t n_in_batch, int tile_x0, int tile_y0,
                                                    float w_lim, float h_lim) {
    const uint32_t t = threadIdx.x, w = t >> 6;
    uint32_t mask = 0;
    const uint32_t g = t < n_in_batch ? pidx[first + t] : 0xFFFFFFFFu;
    if (g < n_particles) {
        const float4 f = record[2 * (size_t)g];
        const float4 c = record[2 * (size_t)g + 1];
        sb.fp[t] = make_float4(f.x, f.y, f.z * kLog2e, __builtin_amdgcn_logf(f.w));
        sb.col[t] = make_float4(c.x, c.y, c.z, f.w);
        const float r2 = c.w * c.w;
#pragma unroll
        for (int k = 0; k < 16; ++k) {
            // sub-block k = 4 * quadrant + row; quadrant (k/4) at (8 (k/4 % 2), 8 (k/4 / 2))
            const int qx = ((k >> 2) & 1) * 8 + (k & 1) * 4, qy = ((k >> 2) >> 1) * 8 + ((k & 3) >> 1) * 4;
            const float x_lo = (float)(tile_x0 + qx) + 0.5f, y_lo = (float)(tile_y0 + qy) + 0.5f;
            const float x_hi = fminf(x_lo + 3.0f, w_lim), y_hi = fminf(y_lo + 3.0f, h_lim);
            const float dx = fmaxf(fmaxf(x_lo - f.x, f.x - x_hi), 0.0f);
            const float dy = fmaxf(fmaxf(y_lo - f.y, f.y - y_hi), 0.0f);
            if (x_lo <= w_lim && y_lo <= h_lim && dx * dx + dy * dy <= r2) mask |= 1u << k;
        }
    }
    if (t == 0) {
        sb.fp[kDummy] = make_float4(0.0f, 0.0f, 0.0f, -__builtin_inff());
        sb.col[kDummy] = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
    }
    uint64_t bal[16];
#pragma unroll
    for (int k = 0; k < 16; ++k) bal[k] = ballot64((mask >> k) & 1u);
    if (lane_id() < 16) {
        uint32_t c = 0;
#pragma unroll
        for (int k = 0; k < 16; ++k) c = (lane_id() == (uint32_t)k) ? (uint32_t)__popcll(bal[k]) : c;
        sb.cnt[w][lane_id()] = c;
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < 16; ++k) {
        if ((mask >> k) & 1u) {
            uint32_t pos = rank_below(bal[k]);
            pos += (w > 0 ? sb.cnt[0][k] : 0u) + (w > 1 ? sb.cnt[1][k] : 0u) + (w > 2 ? sb.cnt[2][k] : 0u);
            sb.list[k][pos] = (uint16_t)t;
        }
    }
    if (t < 64) {
        // pad sub-block k = t / 4 with dummies up to a multiple of four
        const uint32_t k = t >> 2;
        const uint32_t n = sb.cnt[0][k] + sb.cnt[1][k] + sb.cnt[2][k] + sb.cnt[3][k];
        const uint32_t padded = (n + 3u) & ~3u;
        if (n + (t & 3u) < padded) sb.list[k][n + (t & 3u)] = (uint16_t)kDummy;
        if ((t & 3u) == 0) sb.len[k] = padded;
    }
    __syncthreads();
    const uint32_t a = sb.len[4 * w], b = sb.len[4 * w + 1], c = sb.len[4 * w + 2], d = sb.len[4 * w + 3];
    return __builtin_amdgcn_readfirstlane(max(max(a, b), max(c, d)));
}

// Four consecutive entries of this lane's sub-block list from step k (dummies past its end).
__device__ __forceinline__ void list4_sub(const StagedSub& sb, uint32_t sbk, uint32_t k, uint32_t j[4]) {
    uint64_t q = 0x0100010001000100ull;   // four kDummy (256) indices
    if (k < sb.len[sbk]) q = *reinterpret_cast<const uint64_t*>(&sb.list[sbk][k]);
    j[0] = (uint32_t)q & 0xFFFFu;
    j[1] = (uint32_t)(q >> 16) & 0xFFFFu;
    j[2] = (uint32_t)(q >> 32) & 0xFFFFu;
    j[3] = (uint32_t)(q >> 48);
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
