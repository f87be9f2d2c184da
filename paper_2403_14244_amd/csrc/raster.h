// Tile-raster helpers shared by the forward and backward compositing kernels.
#pragma once

#include "common.h"
#include "kernels.h"

namespace isogs {

constexpr int kBatch = 256;   // forward: entries staged in LDS per round (one per thread)

// Compositing checkpoints: at every kCkptChunk-th position of a long tile list (a multiple
// of the forward batch) the forward can store each pixel's {T, r, g, b} before that entry,
// so that the backward can walk the chunks of the list on different workgroups. The
// checkpoints of the tile whose list starts at global entry `start` occupy slots
// start / kCkptChunk + k (k >= 1), which never overlap between tiles; a slot holds one
// float4 per pixel (thread) of the tile. Lists of at least kChunkedMin entries (length
// class kChunkedClass and up, the class being the bit length) are the long ones.
constexpr uint32_t kCkptChunk = 256;
constexpr uint32_t kChunkedMin = 2 * kCkptChunk;
constexpr int kChunkedClass = 10;
static_assert(kCkptChunk % 256 == 0, "checkpoints sit on forward batch boundaries");
static_assert(kCkptChunk == ISOGS_CKPT_CHUNK, "the header states the checkpoint spacing");
static_assert((1u << (kChunkedClass - 1)) == kChunkedMin, "class of the shortest chunked list");

__host__ __device__ inline uint32_t ckpt_slot(uint32_t start, uint32_t k) { return start / kCkptChunk + k; }
__host__ __device__ inline bool chunked_list(uint32_t len) { return len >= kChunkedMin; }

// Longest-list-first tile queues: list length classes 0, then 32 - clz(length); a queue
// starts with its class histogram (kBuckets words).
constexpr int kBuckets = 33;
constexpr int kDummy = kBatch; // staged slot of a zero-opacity record that pads the lists

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

// ---- Staging with 4x4 sub-blocks -----------------------------------------------------------
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

// Whether the binning disk (centre u, v, radius^2 r2) reaches a pixel centre of sub-block
// k = 4 * quadrant + row of the tile at (tile_x0, tile_y0); quadrant q sits at
// (8 (q % 2), 8 (q / 2)), row g of it at (4 (g % 2), 4 (g / 2)). A sub-block starting
// beyond the image has no pixels. The forward and backward passes share this test, so
// they cull the same entries.
__device__ __forceinline__ bool sub_block_touched(float u, float v, float r2, int k, int tile_x0, int tile_y0,
                                                  float w_lim, float h_lim) {
    const int qx = ((k >> 2) & 1) * 8 + (k & 1) * 4, qy = ((k >> 2) >> 1) * 8 + ((k & 3) >> 1) * 4;
    const float x_lo = (float)(tile_x0 + qx) + 0.5f, y_lo = (float)(tile_y0 + qy) + 0.5f;
    const float x_hi = fminf(x_lo + 3.0f, w_lim), y_hi = fminf(y_lo + 3.0f, h_lim);
    const float dx = fmaxf(fmaxf(x_lo - u, u - x_hi), 0.0f);
    const float dy = fmaxf(fmaxf(y_lo - v, v - y_hi), 0.0f);
    return x_lo <= w_lim && y_lo <= h_lim && dx * dx + dy * dy <= r2;
}

constexpr uint32_t kSlotBytes = 16;   // one staged float4

// The walks serve two kernel families, chosen by the template flag AN: the isotropic
// kernel of eq. 8 (a circle, one scalar 1/s^2 per entry) and the anisotropic kernel of
// eq. 5 (an ellipse: the conic A, B, C of the screen covariance of eq. 7). Staged per entry:
//   isotropic    fp {u, v, q = log2(e)/s^2, log2(o)}
//   anisotropic  fp {u, v, nA = -A log2(e), log2(o)}, cn {nB2 = -2 B log2(e), nC = -C log2(e)}
// and col {r, g, b, slot bits}. Both families share the footprint record's layout for
// what binning reads (centre, radius), so they share the bin sort.
template <bool AN>
struct StagedSubT {
    float4 fp[kBatch + 1];
    float4 col[kBatch + 1];
    float2 cn[AN ? kBatch + 1 : 1];
    uint32_t list[16][kBatch + 4];   // byte offsets (16 x staged slot) into fp and col
    uint32_t cnt[4][16];        // [loader wave][sub-block]
    uint32_t len[16];           // padded list lengths (multiples of 4)
};
using StagedSub = StagedSubT<false>;

// One staged entry as loaded from global memory by its thread (k: the conic's B, C).
struct EntryLoad {
    bool ok;
    float4 f, c;
    float2 k;
};

// Staged form of an entry's kernel parameters (see StagedSubT).
template <bool AN>
__device__ __forceinline__ float4 staged_kernel(const float4& f) {
    return make_float4(f.x, f.y, (AN ? -f.z : f.z) * kLog2e, __builtin_amdgcn_logf(f.w));
}
__device__ __forceinline__ float2 staged_conic(const float2& k) {
    return make_float2(-2.0f * k.x * kLog2e, -k.y * kLog2e);
}

// alpha of a staged entry at pixel offset (dx, dy): the isotropic kernel (entry_alpha) or
// the anisotropic one, min(0.99, o exp(-(A dx^2 + 2 B dx dy + C dy^2))) evaluated as
// exp2(log2(o) + dx (nA dx + nB2 dy) + nC dy^2). `g` returns the value before the clamp.
template <bool AN>
__device__ __forceinline__ float staged_alpha(float dx, float dy, const float4& f, const float2& k, float& g) {
    if (!AN) return entry_alpha(dx, dy, f.z, f.w, g);
    const float t = fmaf(k.x, dy, f.z * dx);
    const float s = fmaf(k.y * dy, dy, f.w);
    g = __builtin_amdgcn_exp2f(fmaf(dx, t, s));
    return fminf(kAlphaMax, g);
}

// Particle index of this thread's entry of the batch at `first` (n_in_batch entries), or
// none past the end.
__device__ __forceinline__ uint32_t batch_pidx(const uint32_t* __restrict__ pidx, uint32_t first,
                                               uint32_t n_in_batch) {
    return threadIdx.x < n_in_batch ? pidx[first + threadIdx.x] : 0xFFFFFFFFu;
}

template <bool AN = false>
__device__ __forceinline__ EntryLoad load_entry(const float4* __restrict__ record, uint32_t g,
                                                uint32_t n_particles, const float2* __restrict__ conic = nullptr) {
    EntryLoad e{false, make_float4(0.f, 0.f, 0.f, 0.f), make_float4(0.f, 0.f, 0.f, 0.f), make_float2(0.f, 0.f)};
    if (g < n_particles) {
        e.ok = true;
        e.f = record[2 * (size_t)g];
        e.c = record[2 * (size_t)g + 1];
        if (AN) e.k = conic[g];
    }
    return e;
}

// Stages the loaded entries of a batch (one per thread) and builds the 16 sub-block lists.
// Returns the number of list steps of the calling wave (the longest of its four rows'
// padded lists). Contains __syncthreads.
template <bool AN>
__device__ __forceinline__ uint32_t stage_loaded(StagedSubT<AN>& sb, const EntryLoad& e, int tile_x0, int tile_y0,
                                                 float w_lim, float h_lim) {
    const uint32_t t = threadIdx.x, w = t >> 6;
    uint32_t mask = 0;
    if (e.ok) {
        const float4 f = e.f, c = e.c;
        sb.fp[t] = staged_kernel<AN>(f);
        if (AN) sb.cn[t] = staged_conic(e.k);
        sb.col[t] = make_float4(c.x, c.y, c.z, __uint_as_float(t));   // w: the slot itself
        const float r2 = c.w * c.w;
#pragma unroll
        for (int k = 0; k < 16; ++k)
            if (sub_block_touched(f.x, f.y, r2, k, tile_x0, tile_y0, w_lim, h_lim)) mask |= 1u << k;
    }
    if (t == 0) {
        sb.fp[kDummy] = make_float4(0.0f, 0.0f, 0.0f, -__builtin_inff());
        if (AN) sb.cn[kDummy] = make_float2(0.0f, 0.0f);
        sb.col[kDummy] = make_float4(0.0f, 0.0f, 0.0f, __uint_as_float((uint32_t)kDummy));
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
            sb.list[k][pos] = t * kSlotBytes;
        }
    }
    if (t < 64) {
        // pad sub-block k = t / 4 with dummies up to a multiple of four
        const uint32_t k = t >> 2;
        const uint32_t n = sb.cnt[0][k] + sb.cnt[1][k] + sb.cnt[2][k] + sb.cnt[3][k];
        const uint32_t padded = (n + 3u) & ~3u;
        if (n + (t & 3u) < padded) sb.list[k][n + (t & 3u)] = kDummy * kSlotBytes;
        sb.list[k][padded + (t & 3u)] = kDummy * kSlotBytes;   // four more: reads past the end
        if ((t & 3u) == 0) sb.len[k] = padded;
    }
    __syncthreads();
    const uint32_t a = sb.len[4 * w], b = sb.len[4 * w + 1], c = sb.len[4 * w + 2], d = sb.len[4 * w + 3];
    return __builtin_amdgcn_readfirstlane(max(max(a, b), max(c, d)));
}

// Loads and stages entries [first, first + n_in_batch). Contains __syncthreads.
template <bool AN>
__device__ __forceinline__ uint32_t stage_batch_sub(StagedSubT<AN>& sb, const float4* __restrict__ record,
                                                    const float2* __restrict__ conic,
                                                    const uint32_t* __restrict__ pidx, uint32_t n_particles,
                                                    uint32_t first, uint32_t n_in_batch, int tile_x0, int tile_y0,
                                                    float w_lim, float h_lim) {
    return stage_loaded(sb, load_entry<AN>(record, batch_pidx(pidx, first, n_in_batch), n_particles, conic),
                        tile_x0, tile_y0, w_lim, h_lim);
}

// Byte offsets of four consecutive entries of this lane's sub-block list (padded length
// `len`) from step k; a step at or past the end reads the four dummies that follow the list.
template <bool AN>
__device__ __forceinline__ uint4 list4_sub(const StagedSubT<AN>& sb, uint32_t sbk, uint32_t k, uint32_t len) {
    return *reinterpret_cast<const uint4*>(&sb.list[sbk][min(k, len)]);
}

// Staged record, colour and conic of the entry at byte offset `off` (16 bytes per slot).
template <bool AN>
__device__ __forceinline__ float4 staged_fp(const StagedSubT<AN>& sb, uint32_t off) {
    return *reinterpret_cast<const float4*>(reinterpret_cast<const char*>(sb.fp) + off);
}
template <bool AN>
__device__ __forceinline__ float4 staged_col(const StagedSubT<AN>& sb, uint32_t off) {
    return *reinterpret_cast<const float4*>(reinterpret_cast<const char*>(sb.col) + off);
}
template <bool AN>
__device__ __forceinline__ float2 staged_cn(const StagedSubT<AN>& sb, uint32_t off) {
    if (!AN) return make_float2(0.0f, 0.0f);
    return *reinterpret_cast<const float2*>(reinterpret_cast<const char*>(sb.cn) + (off >> 1));
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
