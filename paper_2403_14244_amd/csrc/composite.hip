// Front-to-back compositing (eq. 4) of every pixel over its tile's depth-sorted entries.
#include <algorithm>

#include "raster.h"

namespace isogs {

// Composites one staged entry into a pixel's running state (branch-free; the dummy pad
// record has log2(o) = -inf, so alpha = 0 and it changes nothing). T loses the weight it
// gives away, T - alpha T; with LAST, `lastj` keeps the staged slot (carried in c.w) of the
// last entry used in the current batch (slots only increase along a list). TERM: the pixel
// stops after the entry that takes T below kTMin.
template <bool TERM, bool AN, bool LAST = true>
__device__ __forceinline__ void composite_entry(const float4& f, const float4& c, const float2& k, float px, float py,
                                                float& T, float& cr, float& cg, float& cb, uint32_t& lastj,
                                                bool& done) {
    float g;
    float a = staged_alpha<AN>(px - f.x, py - f.y, f, k, g);
    const bool use = (a >= kAlphaMin) && !done;
    a = use ? a : 0.0f;
    const float wgt = a * T;
    cr = fmaf(c.x, wgt, cr);
    cg = fmaf(c.y, wgt, cg);
    cb = fmaf(c.z, wgt, cb);
    T = T - wgt;
    if (LAST) lastj = use ? __float_as_uint(c.w) : lastj;
    if (TERM) done = done || (T < kTMin);
}

// The four entries of one list step: offsets -> staged records (k: conics, anisotropic).
struct Step4 {
    float4 f[4], c[4];
    float2 k[4];
};

template <bool AN>
__device__ __forceinline__ void load_step(const StagedSubT<AN>& sb, const uint4& o, Step4& st) {
    st.f[0] = staged_fp(sb, o.x);
    st.f[1] = staged_fp(sb, o.y);
    st.f[2] = staged_fp(sb, o.z);
    st.f[3] = staged_fp(sb, o.w);
    st.c[0] = staged_col(sb, o.x);
    st.c[1] = staged_col(sb, o.y);
    st.c[2] = staged_col(sb, o.z);
    st.c[3] = staged_col(sb, o.w);
    st.k[0] = staged_cn(sb, o.x);
    st.k[1] = staged_cn(sb, o.y);
    st.k[2] = staged_cn(sb, o.z);
    st.k[3] = staged_cn(sb, o.w);
}

// A lane's pixel in a tile, and the pixel's compositing state.
struct TilePixel {
    int width, height;
    uint32_t pix_off;
    int tx, ty, x, y;
    bool inside;
    float px, py, w_lim, h_lim;
    uint32_t start, len, sbk;
};

struct PixelState {
    float T, cr, cg, cb;
    uint32_t last;   // 1-based tile-list position of the last entry used, 0 if none
    bool done;
};

__device__ __forceinline__ TilePixel tile_pixel(const RenderPack& pk, uint32_t logical,
                                                const uint32_t* __restrict__ ranges) {
    TilePixel p;
    int vi;
    locate_tile(pk, logical, vi, p.tx, p.ty);
    const ViewDesc& vd = pk.v[vi];
    p.width = vd.width;
    p.height = vd.height;
    p.pix_off = vd.pix_off;
    const uint32_t t = threadIdx.x;
    p.x = p.tx * kTile + sub_x(t);
    p.y = p.ty * kTile + sub_y(t);
    p.inside = p.x < vd.width && p.y < vd.height;
    p.px = (float)p.x + 0.5f;
    p.py = (float)p.y + 0.5f;
    p.w_lim = (float)vd.width - 0.5f;
    p.h_lim = (float)vd.height - 0.5f;
    const uint32_t gt = vd.tile_base + (uint32_t)(p.ty * vd.tiles_x + p.tx);
    p.start = ranges[2 * gt];
    const uint32_t end = min(ranges[2 * gt + 1], pk.n_entries_cap);
    p.len = end > p.start ? end - p.start : 0u;
    p.sbk = 4 * (t >> 6) + ((t >> 4) & 3u);   // this lane's sub-block
    return p;
}

// Walks list positions [lo, hi) of the tile (lo a multiple of the batch) with a 256-thread
// workgroup, one lane per pixel, each 16-lane row owning a 4x4 sub-block, and updates the
// lanes' states. With `ckpt`, stores the checkpoints at chunk boundaries inside the range.
// PIPE: the global loads of the next batch are issued while the current one is walked.
// PL (default PIPE): software-pipelined LDS reads as well, for a workgroup with few others
// beside it on its CU (more registers): the reads of the entries of step k + 4 and of the
// list words of step k + 8 are issued while step k is composited, so that the walk does not
// wait on dependent round trips.
// LAST: track the last entry used (s.last); without it s.last stays 0.
// Contains __syncthreads.
template <bool TERM, bool PIPE, bool PL, bool AN, bool LAST = true>
__device__ __forceinline__ void composite_range(StagedSubT<AN>& sb, const RenderPack& pk, const TilePixel& p,
                                                const float4* __restrict__ record, const float2* __restrict__ conic,
                                                const uint32_t* __restrict__ pidx, uint32_t lo, uint32_t hi,
                                                PixelState& s, float4* __restrict__ ckpt) {
    const uint32_t t = threadIdx.x;
    const uint32_t end = p.start + hi;
    auto batch_len = [end](uint32_t b) { return b < end ? min((uint32_t)kBatch, end - b) : 0u; };
    uint32_t b0 = p.start + lo;
    // PIPE also prefetches from global memory: the records of the next batch and the
    // particle indices of the one after are loaded while the current batch is walked
    EntryLoad cur{}, nxt{};
    uint32_t g_next = 0xFFFFFFFFu;
    if (PIPE) {
        cur = load_entry<AN>(record, batch_pidx(pidx, b0, batch_len(b0)), pk.n_particles, conic);
        g_next = batch_pidx(pidx, b0 + kBatch, batch_len(b0 + kBatch));
    }
    for (; b0 < end; b0 += kBatch) {
        if (__syncthreads_and(s.done)) break;
        if (ckpt && chunked_list(p.len) && b0 > p.start && (b0 - p.start) % kCkptChunk == 0)
            ckpt[(size_t)ckpt_slot(p.start, (b0 - p.start) / kCkptChunk) * 256 + t] =
                make_float4(s.T, s.cr, s.cg, s.cb);
        uint32_t steps;
        if (PIPE) {
            nxt = load_entry<AN>(record, g_next, pk.n_particles, conic);
            g_next = batch_pidx(pidx, b0 + 2 * kBatch, batch_len(b0 + 2 * kBatch));
            steps = stage_loaded(sb, cur, p.tx * kTile, p.ty * kTile, p.w_lim, p.h_lim);
        } else {
            steps = stage_batch_sub(sb, record, conic, pidx, pk.n_particles, b0, batch_len(b0), p.tx * kTile,
                                    p.ty * kTile, p.w_lim, p.h_lim);
        }
        const uint32_t pos0 = b0 - p.start + 1;   // 1-based list position of staged slot 0
        const uint32_t len = sb.len[p.sbk];
        uint32_t lastj = 0xFFFFFFFFu;
        auto composite_step = [&](const Step4& st) {
#pragma unroll
            for (int e = 0; e < 4; ++e)
                composite_entry<TERM, AN, LAST>(st.f[e], st.c[e], st.k[e], p.px, p.py, s.T, s.cr, s.cg, s.cb,
                                                lastj, s.done);
        };
        if (!PL) {
            for (uint32_t k = 0; k < steps; k += 4) {
                Step4 st;
                load_step(sb, list4_sub(sb, p.sbk, k, len), st);
                composite_step(st);
                if (TERM && ballot64(!s.done) == 0) break;
            }
        } else {
            // two register sets in turn, unrolled so that neither is copied: while one
            // step is composited, the records of the next and the list words of the one
            // after are in flight (the barriers keep the reads ahead of the arithmetic)
            Step4 sa, sc;
            uint4 o = list4_sub(sb, p.sbk, 0, len);
            load_step(sb, o, sa);
            o = list4_sub(sb, p.sbk, 4, len);
            for (uint32_t k = 0; k < steps; k += 8) {
                load_step(sb, o, sc);
                o = list4_sub(sb, p.sbk, k + 8, len);
                __builtin_amdgcn_sched_barrier(0);
                composite_step(sa);
                if (TERM && ballot64(!s.done) == 0) break;
                load_step(sb, o, sa);
                o = list4_sub(sb, p.sbk, k + 12, len);
                __builtin_amdgcn_sched_barrier(0);
                composite_step(sc);   // past the end of the lists: dummies only
                if (TERM && ballot64(!s.done) == 0) break;
            }
        }
        if (LAST && lastj != 0xFFFFFFFFu) s.last = pos0 + lastj;
        if (PIPE) cur = nxt;
    }
}

__device__ __forceinline__ void write_pixel(const TilePixel& p, const PixelState& s, float bg_r, float bg_g,
                                            float bg_b, float* __restrict__ image, float* __restrict__ T_final,
                                            uint32_t* __restrict__ n_last) {
    if (!p.inside) return;
    const size_t hw = (size_t)p.width * p.height;
    const size_t pix = (size_t)p.y * p.width + p.x;
    float* img = image + (size_t)3 * p.pix_off;
    img[pix] = fmaf(s.T, bg_r, s.cr);
    img[hw + pix] = fmaf(s.T, bg_g, s.cg);
    img[2 * hw + pix] = fmaf(s.T, bg_b, s.cb);
    T_final[p.pix_off + pix] = s.T;
    if (n_last) n_last[p.pix_off + pix] = s.last;
}

// On a capacity overflow the bins hold no valid lists: the tile's pixels get NaN colour
// and transmittance and n_last 0, so that a result whose status was never read cannot
// pass for a render.
__device__ __forceinline__ void write_overflow_tile(const RenderPack& pk, uint32_t logical,
                                                   float* __restrict__ image, float* __restrict__ T_final,
                                                   uint32_t* __restrict__ n_last) {
    int vi, tx, ty;
    locate_tile(pk, logical, vi, tx, ty);
    const ViewDesc& vd = pk.v[vi];
    const int x = tx * kTile + (int)(threadIdx.x & 15u), y = ty * kTile + (int)(threadIdx.x >> 4);
    if (x >= vd.width || y >= vd.height) return;
    const size_t hw = (size_t)vd.width * vd.height, pix = (size_t)y * vd.width + x;
    const float nan = __builtin_nanf("");
    float* img = image + (size_t)3 * vd.pix_off;
    img[pix] = nan;
    img[hw + pix] = nan;
    img[2 * hw + pix] = nan;
    T_final[vd.pix_off + pix] = nan;
    if (n_last) n_last[vd.pix_off + pix] = 0u;
}

// Composites one whole tile (logical index within the launch). Contains __syncthreads.
template <bool PIPE, bool PL, bool AN, bool LAST = true>
__device__ __forceinline__ void composite_tile(StagedSubT<AN>& sb, const RenderPack& pk, uint32_t logical,
                                               const float4* __restrict__ record, const float2* __restrict__ conic,
                                               const uint32_t* __restrict__ pidx,
                                               const uint32_t* __restrict__ ranges, float bg_r, float bg_g,
                                               float bg_b, float* __restrict__ image, float* __restrict__ T_final,
                                               uint32_t* __restrict__ n_last, float4* __restrict__ ckpt) {
    const TilePixel p = tile_pixel(pk, logical, ranges);
    PixelState s{1.0f, 0.0f, 0.0f, 0.0f, 0u, !p.inside};
    composite_range<true, PIPE, PL, AN, LAST>(sb, pk, p, record, conic, pidx, 0, p.len, s, ckpt);
    write_pixel(p, s, bg_r, bg_g, bg_b, image, T_final, n_last);
}

// Register budgets: the compact walk of large launches, six waves per SIMD (80 VGPRs), as
// many resident workgroups as LDS allows hiding the staging gathers; the walk of the
// remaining tiles of small launches also prefetches the next batch from global memory,
// five waves per SIMD (at most 102 VGPRs).
constexpr int kCompactWavesPerSimd = 6;
constexpr int kPrefetchWavesPerSimd = 5;

// One workgroup per tile, tiles in XCD-banded order.
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(kCompactWavesPerSimd))) composite_fwd_kernel(
    const RenderPack pk, const float4* __restrict__ record, const uint32_t* __restrict__ pidx,
    const uint32_t* __restrict__ ranges, const int32_t* __restrict__ status,
    float bg_r, float bg_g, float bg_b, float* __restrict__ image, float* __restrict__ T_final,
    uint32_t* __restrict__ n_last, float4* __restrict__ ckpt) {
    __shared__ StagedSub sb;
    const uint32_t logical = xcd_swizzle(blockIdx.x, gridDim.x);
    if (*status != kStatusOk) return write_overflow_tile(pk, logical, image, T_final, n_last);
    composite_tile<false, false, false>(sb, pk, logical, record, nullptr, pidx, ranges, bg_r, bg_g, bg_b, image,
                                        T_final, n_last, ckpt);
}

// ---- Wide walk for the longest tiles of small launches ------------------------------------
// A launch of one or two views is bound by its few longest tiles: one wave walks a whole
// list for its 64 pixels, one entry after another. The wide walk spreads such a tile over
// four workgroups, one per 8x8 quadrant; wave w walks the list of the quadrant's sub-block
// w with four lanes per pixel (lane l: pixel l / 4 of the 4x4 sub-block, entry l % 4 of
// each four-entry list step). In a step the four lanes form the transmittance products
// of the step's entries with a scan over the pixel's lanes, find the entry that takes T
// below kTMin (the entries after it are not composited), and sum the four colour terms:
// the result is the sequential one up to rounding (products and sums are associated per
// step), at four times the lanes per pixel.

template <bool AN>
struct StagedQuadT {
    float4 fp[kBatch + 1];
    float4 col[kBatch + 1];        // {r, g, b, slot bits}
    float2 cn[AN ? kBatch + 1 : 1];
    uint32_t list[4][kBatch + 4];  // byte offsets, per sub-block of the quadrant
    uint32_t cnt[4][4];            // [loader wave][sub-block]
    uint32_t len[4];
};

// Stages a batch for quadrant `quad` of the tile: records of all entries, lists of the
// quadrant's four sub-blocks only. Returns the padded length of the calling wave's list
// (wave w walks sub-block 4 quad + w). Contains __syncthreads.
template <bool AN>
__device__ __forceinline__ uint32_t stage_quad(StagedQuadT<AN>& sq, const EntryLoad& e, int quad, int tile_x0,
                                               int tile_y0, float w_lim, float h_lim) {
    const uint32_t t = threadIdx.x, w = t >> 6;
    uint32_t mask = 0;
    if (e.ok) {
        const float4 f = e.f, c = e.c;
        sq.fp[t] = staged_kernel<AN>(f);
        if (AN) sq.cn[t] = staged_conic(e.k);
        sq.col[t] = make_float4(c.x, c.y, c.z, __uint_as_float(t));
        const float r2 = c.w * c.w;
#pragma unroll
        for (int r = 0; r < 4; ++r)
            if (sub_block_touched(f.x, f.y, r2, 4 * quad + r, tile_x0, tile_y0, w_lim, h_lim)) mask |= 1u << r;
    }
    if (t == 0) {
        sq.fp[kDummy] = make_float4(0.0f, 0.0f, 0.0f, -__builtin_inff());
        if (AN) sq.cn[kDummy] = make_float2(0.0f, 0.0f);
        sq.col[kDummy] = make_float4(0.0f, 0.0f, 0.0f, __uint_as_float((uint32_t)kDummy));
    }
    uint64_t bal[4];
#pragma unroll
    for (int r = 0; r < 4; ++r) bal[r] = ballot64((mask >> r) & 1u);
    if (lane_id() < 4) {
        const uint32_t r = lane_id();
        sq.cnt[w][r] = (uint32_t)__popcll(r == 0 ? bal[0] : r == 1 ? bal[1] : r == 2 ? bal[2] : bal[3]);
    }
    __syncthreads();
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        if ((mask >> r) & 1u) {
            uint32_t pos = rank_below(bal[r]);
            pos += (w > 0 ? sq.cnt[0][r] : 0u) + (w > 1 ? sq.cnt[1][r] : 0u) + (w > 2 ? sq.cnt[2][r] : 0u);
            sq.list[r][pos] = t * kSlotBytes;
        }
    }
    if (t < 16) {
        const uint32_t r = t >> 2;
        const uint32_t n = sq.cnt[0][r] + sq.cnt[1][r] + sq.cnt[2][r] + sq.cnt[3][r];
        const uint32_t padded = (n + 3u) & ~3u;
        if (n + (t & 3u) < padded) sq.list[r][n + (t & 3u)] = kDummy * kSlotBytes;
        sq.list[r][padded + (t & 3u)] = kDummy * kSlotBytes;
        if ((t & 3u) == 0) sq.len[r] = padded;
    }
    __syncthreads();
    return __builtin_amdgcn_readfirstlane(sq.len[w]);
}

// Composites quadrant `quad` of one tile with the wide walk. Contains __syncthreads.
template <bool AN>
__device__ __forceinline__ void composite_quadrant(StagedQuadT<AN>& sq, const RenderPack& pk, uint32_t logical,
                                                   int quad, const float4* __restrict__ record,
                                                   const float2* __restrict__ conic,
                                                   const uint32_t* __restrict__ pidx,
                                                   const uint32_t* __restrict__ ranges, float bg_r, float bg_g,
                                                   float bg_b, float* __restrict__ image,
                                                   float* __restrict__ T_final, uint32_t* __restrict__ n_last,
                                                   float4* __restrict__ ckpt) {
    int vi, tx, ty;
    locate_tile(pk, logical, vi, tx, ty);
    const ViewDesc& vd = pk.v[vi];
    const uint32_t t = threadIdx.x, w = t >> 6, l = lane_id();
    const uint32_t e_idx = l & 3u;                  // entry of each list step
    const uint32_t pp = l >> 2;                     // pixel of the sub-block
    const uint32_t k = 4u * (uint32_t)quad + w;     // sub-block of the tile
    const uint32_t t_px = 16u * k + pp;             // the pixel's thread in the one-workgroup layout
    const int x = tx * kTile + (int)((k >> 2) & 1u) * 8 + (int)(k & 1u) * 4 + (int)(pp & 3u);
    const int y = ty * kTile + (int)(k >> 3) * 8 + (int)((k & 3u) >> 1) * 4 + (int)(pp >> 2);
    const bool inside = x < vd.width && y < vd.height;
    const float px = (float)x + 0.5f, py = (float)y + 0.5f;
    const float w_lim = (float)vd.width - 0.5f, h_lim = (float)vd.height - 0.5f;
    const uint32_t gt = vd.tile_base + (uint32_t)(ty * vd.tiles_x + tx);
    const uint32_t start = ranges[2 * gt];
    const uint32_t end = min(ranges[2 * gt + 1], pk.n_entries_cap);
    const uint32_t len = end > start ? end - start : 0u;

    float T = 1.0f, cr = 0.0f, cg = 0.0f, cb = 0.0f;
    uint32_t last = 0, lastp1 = 0;   // lastp1: staged slot + 1 of this lane's last entry used
    bool done = !inside;
    auto batch_len = [end](uint32_t b) { return b < end ? min((uint32_t)kBatch, end - b) : 0u; };
    uint32_t b0 = start;
    EntryLoad cur = load_entry<AN>(record, batch_pidx(pidx, b0, batch_len(b0)), pk.n_particles, conic);
    uint32_t g_next = batch_pidx(pidx, b0 + kBatch, batch_len(b0 + kBatch));
    for (; b0 < end; b0 += kBatch) {
        if (__syncthreads_and(done)) break;
        if (ckpt && chunked_list(len) && b0 > start && (b0 - start) % kCkptChunk == 0 && e_idx == 0)
            ckpt[(size_t)ckpt_slot(start, (b0 - start) / kCkptChunk) * 256 + t_px] = make_float4(T, cr, cg, cb);
        const EntryLoad nxt = load_entry<AN>(record, g_next, pk.n_particles, conic);
        g_next = batch_pidx(pidx, b0 + 2 * kBatch, batch_len(b0 + 2 * kBatch));
        const uint32_t n = stage_quad(sq, cur, quad, tx * kTile, ty * kTile, w_lim, h_lim);
        lastp1 = 0;
        for (uint32_t s0 = 0; s0 < n; s0 += 4) {
            const uint32_t off = sq.list[w][s0 + e_idx];
            const float4 f = *reinterpret_cast<const float4*>(reinterpret_cast<const char*>(sq.fp) + off);
            const float4 c = *reinterpret_cast<const float4*>(reinterpret_cast<const char*>(sq.col) + off);
            float2 kc = make_float2(0.0f, 0.0f);
            if (AN) kc = *reinterpret_cast<const float2*>(reinterpret_cast<const char*>(sq.cn) + (off >> 1));
            float g;
            float a = staged_alpha<AN>(px - f.x, py - f.y, f, kc, g);
            const bool use = a >= kAlphaMin;
            a = use ? a : 0.0f;
            const float om = 1.0f - a;
            // products of (1 - alpha) over the pixel's lanes up to this one (quad scan). The
            // cross-lane reads stay outside any condition: a read from a lane that a branch
            // has switched off returns 0
            float incl = om;
            const float from1 = dpp<0x90>(incl);   // lane e - 1
            incl = incl * (e_idx >= 1u ? from1 : 1.0f);
            const float from2 = dpp<0x40>(incl);   // lane e - 2
            incl = incl * (e_idx >= 2u ? from2 : 1.0f);
            const float prev = dpp<0x90>(incl);
            const float excl = e_idx >= 1u ? prev : 1.0f;
            // the entry that takes T below kTMin is the last one composited
            const bool cross = !done && use && (T * incl < kTMin);
            const uint32_t nib = (uint32_t)(ballot64(cross) >> (l & 60u)) & 0xFu;
            const bool muted = done || (nib & ((1u << e_idx) - 1u)) != 0u;
            const float wgt = muted ? 0.0f : a * (T * excl);
            float sr = wgt * c.x, sg = wgt * c.y, sb = wgt * c.z;
            sr += dpp<0xB1>(sr);
            sg += dpp<0xB1>(sg);
            sb += dpp<0xB1>(sb);
            sr += dpp<0x4E>(sr);
            sg += dpp<0x4E>(sg);
            sb += dpp<0x4E>(sb);
            cr += sr;
            cg += sg;
            cb += sb;
            float fac = muted ? 1.0f : om;
            fac *= dpp<0xB1>(fac);
            fac *= dpp<0x4E>(fac);
            T = T * fac;
            lastp1 = (use && !muted) ? __float_as_uint(c.w) + 1u : lastp1;
            done = done || nib != 0u;
            if (ballot64(!done) == 0) break;
        }
        // the pixel's last entry: the largest slot over its four lanes
        uint32_t m = lastp1;
        m = max(m, (uint32_t)__builtin_amdgcn_update_dpp(0, (int)m, 0xB1, 0xF, 0xF, false));
        m = max(m, (uint32_t)__builtin_amdgcn_update_dpp(0, (int)m, 0x4E, 0xF, 0xF, false));
        if (m) last = b0 - start + m;   // 1-based list position
        cur = nxt;
    }
    if (inside && e_idx == 0) {
        const size_t hw = (size_t)vd.width * vd.height;
        const size_t pix = (size_t)y * vd.width + x;
        float* img = image + (size_t)3 * vd.pix_off;
        img[pix] = fmaf(T, bg_r, cr);
        img[hw + pix] = fmaf(T, bg_g, cg);
        img[2 * hw + pix] = fmaf(T, bg_b, cb);
        T_final[vd.pix_off + pix] = T;
        if (n_last) n_last[vd.pix_off + pix] = last;
    }
}

// With the wide flag, every tile of at least 2^kWideMinLog2 entries (length classes above
// kWideMinLog2) takes the wide walk: a decision of the tile alone, so a view's result does
// not depend on the other views of the launch.
constexpr int kWideMinLog2 = 11;

// Longest list first: one workgroup per tile, the tiles taken in the order of a queue
// sorted by list length, so that the dispatcher starts the long tiles of skewed scenes
// first instead of leaving them to trail the launch. Two builds of the walk: with many
// tiles the launch is throughput-bound and the compact one is faster; with few, it is bound
// by its longest tiles and the fully pipelined one is.

// Arguments of the longest-first compositing kernels (both kernel families).
struct OrderedArgs {
    const float4* record;
    const float2* conic;      // anisotropic family: {B, C} per record
    const uint32_t* pidx;
    const uint32_t* ranges;
    const int32_t* status;
    float bg_r, bg_g, bg_b;
    float* image;
    float* T_final;
    uint32_t* n_last;
    float4* ckpt;
    const uint32_t* order;
    const uint32_t* hist;
    uint32_t wide_slots;
    uint64_t* times;          // ISOGS_FWD_TIMES: {start, end} per workgroup of the launch, else NULL
};

// Workgroup clock stamps (ISOGS_FWD_TIMES): the constant 100 MHz clock when the workgroup
// starts and after its last wave has finished, written only by workgroups that composited
// a non-empty list (the others leave zeros).
struct WgStamp {
    uint64_t t0;
    __device__ explicit WgStamp(const OrderedArgs& a) : t0(a.times ? __builtin_amdgcn_s_memrealtime() : 0) {}
    // logical: the tile's index within the launch (queue entries are launch-local)
    __device__ void done(const OrderedArgs& a, const RenderPack& pk, uint32_t logical) const {
        if (!a.times) return;   // uniform: a kernel argument
        __syncthreads();
        const uint32_t gt = pk.v[0].tile_base + logical;   // the launch's tiles are consecutive
        if (threadIdx.x == 0 && a.ranges[2 * gt + 1] > a.ranges[2 * gt]) {
            const uint64_t t1 = __builtin_amdgcn_s_memrealtime();
            a.times[2 * (size_t)blockIdx.x] = t0;
            a.times[2 * (size_t)blockIdx.x + 1] = t1;
        }
    }
};

// LAST: the caller asked for n_last (without it the walk does not track the last entry).
template <bool PIPE, bool AN, bool LAST>
__device__ __forceinline__ void ordered_tile(StagedSubT<AN>& sb, const RenderPack& pk, const OrderedArgs& a) {
    if (*a.status != kStatusOk) return write_overflow_tile(pk, a.order[blockIdx.x], a.image, a.T_final, a.n_last);
    const WgStamp stamp(a);
    composite_tile<PIPE, PIPE, AN, LAST>(sb, pk, a.order[blockIdx.x], a.record, a.conic, a.pidx, a.ranges, a.bg_r, a.bg_g,
                                   a.bg_b, a.image, a.T_final, a.n_last, a.ckpt);
    stamp.done(a, pk, a.order[blockIdx.x]);
}

template <bool LAST>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(kCompactWavesPerSimd)))
composite_fwd_ordered_kernel(const RenderPack pk, const OrderedArgs a) {
    __shared__ StagedSubT<false> sb;
    ordered_tile<false, false, LAST>(sb, pk, a);
}

template <bool LAST>
__global__ void __launch_bounds__(256) composite_fwd_ordered_pipe_kernel(const RenderPack pk, const OrderedArgs a) {
    __shared__ StagedSubT<false> sb;
    ordered_tile<true, false, LAST>(sb, pk, a);
}

// The anisotropic family (eq. 5 kernels): the same walks with the conic staged beside each
// record. Its larger staging (27.5 KB) fits five workgroups per CU, so the compact walk
// gets the registers of five waves per SIMD.
constexpr int kAnisoCompactWavesPerSimd = 5;
constexpr int kAnisoWideWavesPerSimd = 4;

template <bool LAST>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(kAnisoCompactWavesPerSimd)))
aniso_fwd_ordered_kernel(const RenderPack pk, const OrderedArgs a) {
    __shared__ StagedSubT<true> sb;
    ordered_tile<false, true, LAST>(sb, pk, a);
}

template <bool LAST>
__global__ void __launch_bounds__(256) aniso_fwd_ordered_pipe_kernel(const RenderPack pk, const OrderedArgs a) {
    __shared__ StagedSubT<true> sb;
    ordered_tile<true, true, LAST>(sb, pk, a);
}

// Launches of at most this many tiles use the pipelined walk (measured crossover on the
// 1M-particle 1080p views: between two and four views, 16320 and 32640 tiles).
constexpr uint32_t kPipeTileLimit = 24576;

__global__ void __launch_bounds__(128) fill_u32_kernel_c(uint32_t* __restrict__ p, uint32_t n) {
    for (uint32_t i = threadIdx.x; i < n; i += blockDim.x) p[i] = 0u;
}


__device__ __forceinline__ uint32_t length_bucket(const uint32_t* ranges, uint32_t gt, uint32_t cap) {
    const uint32_t s = ranges[2 * gt], e = min(ranges[2 * gt + 1], cap);
    const uint32_t len = e > s ? e - s : 0u;
    return len ? 32u - (uint32_t)__clz(len) : 0u;
}

// Queue order, pass 1: how many tiles fall in each length class.
__global__ void __launch_bounds__(256) tile_class_hist_kernel(const uint32_t* __restrict__ ranges, uint32_t tile0,
                                                              uint32_t n_items, uint32_t cap,
                                                              uint32_t* __restrict__ hist) {
    __shared__ uint32_t h[kBuckets];
    if (threadIdx.x < kBuckets) h[threadIdx.x] = 0u;
    __syncthreads();
    for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < n_items; i += gridDim.x * blockDim.x)
        atomicAdd(&h[length_bucket(ranges, tile0 + i, cap)], 1u);
    __syncthreads();
    if (threadIdx.x < kBuckets && h[threadIdx.x]) atomicAdd(&hist[threadIdx.x], h[threadIdx.x]);
}

// Queue order, pass 2: tiles placed class by class, longest class first (the order inside
// a class is arbitrary; each tile's result does not depend on it).
__global__ void __launch_bounds__(256) tile_class_scatter_kernel(const uint32_t* __restrict__ ranges,
                                                                 uint32_t tile0, uint32_t n_items, uint32_t cap,
                                                                 const uint32_t* __restrict__ hist,
                                                                 uint32_t* __restrict__ cursor,
                                                                 uint32_t* __restrict__ order) {
    __shared__ uint32_t start[kBuckets], cnt[kBuckets], base[kBuckets];
    if (threadIdx.x < kBuckets) {
        uint32_t s = 0;
        for (int b = kBuckets - 1; b > (int)threadIdx.x; --b) s += hist[b];
        start[threadIdx.x] = s;
        cnt[threadIdx.x] = 0u;
    }
    __syncthreads();
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    uint32_t b = 0, local = 0;
    if (i < n_items) {
        b = length_bucket(ranges, tile0 + i, cap);
        local = atomicAdd(&cnt[b], 1u);
    }
    __syncthreads();
    if (threadIdx.x < kBuckets && cnt[threadIdx.x]) base[threadIdx.x] = atomicAdd(&cursor[threadIdx.x], cnt[threadIdx.x]);
    __syncthreads();
    if (i < n_items) order[start[b] + base[b] + local] = i;
}

int launch_render_fwd(const isogs_projected* proj, const int32_t* n_per_view, const isogs_bins* bins,
                      const isogs_camera* cams, int32_t nv, const float* bg, float* image, float* T_final,
                      uint32_t* n_last, float* ckpt, hipStream_t stream) {
    uint32_t p_off = 0, tile_base = 0, pix_off = 0;
    for (int v0 = 0; v0 < nv; v0 += kMaxViews) {
        RenderPack pk{};
        uint32_t blocks;
        fill_render_pack(pk, cams, n_per_view, v0, nv, p_off, tile_base, pix_off, blocks);
        set_render_limits(pk, n_per_view, nv, bins->capacity);
        if (!blocks) continue;
        hipLaunchKernelGGL(composite_fwd_kernel, dim3(blocks), dim3(256), 0, stream, pk,
                           reinterpret_cast<const float4*>(proj->record), bins->pidx, bins->ranges,
                           bins->status, bg[0], bg[1], bg[2], image, T_final, n_last,
                           reinterpret_cast<float4*>(ckpt));
        if (hipPeekAtLastError() != hipSuccess) return -1;
    }
    return 0;
}

// Workspace: the tile queue, then (ISOGS_FWD_TIMES) the clock stamps, 5 workgroups per tile
// of the call at most (the wide launch adds four quadrant workgroups per long tile).
static size_t queue_ws_bytes(const isogs_camera* cams, int32_t nv) {
    return (tile_queue_words(max_group_tiles(cams, nv)) * 4 + 255) & ~(size_t)255;
}

static uint64_t call_tiles(const isogs_camera* cams, int32_t nv) {
    uint64_t tiles = 0;
    for (int j = 0; j < nv; ++j)
        tiles += (uint64_t)(((cams[j].width + kTile - 1) / kTile) * ((cams[j].height + kTile - 1) / kTile));
    return tiles;
}

size_t render_fwd_ordered_ws(const isogs_camera* cams, int32_t nv, uint32_t flags) {
    size_t need = queue_ws_bytes(cams, nv);
    if (flags & ISOGS_FWD_TIMES) need += (size_t)call_tiles(cams, nv) * 5 * 16;
    return need + 256;
}

__global__ void __launch_bounds__(256) fill_stamps_kernel(uint64_t* __restrict__ p, size_t n) {
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
        p[i] = 0u;
}

uint32_t max_group_tiles(const isogs_camera* cams, int32_t nv) {
    uint32_t most = 0;
    for (int v0 = 0; v0 < nv; v0 += kMaxViews) {
        uint32_t tiles = 0;
        for (int j = v0; j < min(nv, v0 + kMaxViews); ++j)
            tiles += (uint32_t)(((cams[j].width + kTile - 1) / kTile) * ((cams[j].height + kTile - 1) / kTile));
        most = tiles > most ? tiles : most;
    }
    return most;
}

// Queue layout: the class histogram (kBuckets words, read by the wide and backward
// kernels), its cursors, then the order.
constexpr size_t kQueueHead = 2 * kBuckets;

size_t tile_queue_words(uint32_t n_tiles) { return kQueueHead + (size_t)n_tiles; }

uint32_t* launch_tile_queue(uint32_t* q, const uint32_t* ranges, uint32_t tile0, uint32_t n_tiles, uint32_t cap,
                            hipStream_t stream) {
    uint32_t* hist = q;
    uint32_t* cursor = q + kBuckets;
    uint32_t* order = q + kQueueHead;
    hipLaunchKernelGGL(fill_u32_kernel_c, dim3(1), dim3(128), 0, stream, q, (uint32_t)kQueueHead);
    const unsigned hb = std::min<unsigned>(256u, (n_tiles + 255u) / 256u);
    hipLaunchKernelGGL(tile_class_hist_kernel, dim3(hb), dim3(256), 0, stream, ranges, tile0, n_tiles, cap, hist);
    hipLaunchKernelGGL(tile_class_scatter_kernel, dim3((n_tiles + 255u) / 256u), dim3(256), 0, stream, ranges, tile0,
                       n_tiles, cap, hist, cursor, order);
    return order;
}

int resident_blocks(const void* kernel, int threads) {
    int dev = 0, cus = 0, per_cu = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kernel, threads, 0) != hipSuccess || per_cu < 1)
        per_cu = 1;
    return cus * per_cu;
}

// Workgroups [0, 4 wide_slots) take the quadrants of the long tiles (those of at least
// 2^kWideMinLog2 entries: the first ones of the queue, counted from its length classes;
// wide_slots bounds their number, and a workgroup past it leaves at once) with the wide
// walk, the others the remaining tiles of the queue with the walk that prefetches the next
// batch.
template <bool AN>
__device__ __forceinline__ void ordered_wide(unsigned char* smem, const RenderPack& pk, const OrderedArgs& a) {
    static_assert(sizeof(StagedQuadT<AN>) <= sizeof(StagedSubT<AN>), "one LDS buffer serves both walks");
    const uint32_t wide_slots = a.wide_slots;
    if (*a.status != kStatusOk) {
        // every tile is one of the remaining ones then (no list is long)
        if (blockIdx.x >= 4 * wide_slots)
            write_overflow_tile(pk, a.order[blockIdx.x - 4 * wide_slots], a.image, a.T_final, a.n_last);
        return;
    }
    uint32_t n_wide = 0;
    for (int c = kWideMinLog2 + 1; c < kBuckets; ++c) n_wide += a.hist[c];
    n_wide = min(n_wide, wide_slots);
    const uint32_t b = blockIdx.x;
    const WgStamp stamp(a);
    if (b < 4 * wide_slots) {
        if ((b >> 2) >= n_wide) return;
        composite_quadrant(*reinterpret_cast<StagedQuadT<AN>*>(smem), pk, a.order[b >> 2], (int)(b & 3u), a.record,
                           a.conic, a.pidx, a.ranges, a.bg_r, a.bg_g, a.bg_b, a.image, a.T_final, a.n_last, a.ckpt);
        stamp.done(a, pk, a.order[b >> 2]);
    } else {
        const uint32_t j = b - 4 * wide_slots;
        if (j < n_wide) return;
        composite_tile<true, false, AN>(*reinterpret_cast<StagedSubT<AN>*>(smem), pk, a.order[j], a.record, a.conic,
                                        a.pidx, a.ranges, a.bg_r, a.bg_g, a.bg_b, a.image, a.T_final, a.n_last,
                                        a.ckpt);
        stamp.done(a, pk, a.order[j]);
    }
}

__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(kPrefetchWavesPerSimd)))
composite_fwd_ordered_wide_kernel(const RenderPack pk, const OrderedArgs a) {
    __shared__ __align__(16) unsigned char smem[sizeof(StagedSubT<false>)];
    ordered_wide<false>(smem, pk, a);
}

__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(kAnisoWideWavesPerSimd)))
aniso_fwd_ordered_wide_kernel(const RenderPack pk, const OrderedArgs a) {
    __shared__ __align__(16) unsigned char smem[sizeof(StagedSubT<true>)];
    ordered_wide<true>(smem, pk, a);
}

int launch_render_fwd_ordered(const isogs_projected* proj, const float* conic, const int32_t* n_per_view,
                              const isogs_bins* bins, const isogs_camera* cams, int32_t nv, const float* bg,
                              float* image, float* T_final, uint32_t* n_last, float* ckpt, uint32_t flags, void* ws,
                              hipStream_t stream) {
    const bool an = conic != nullptr;
    uint32_t* q = static_cast<uint32_t*>(ws);
    uint64_t* stamps = nullptr;
    if (flags & ISOGS_FWD_TIMES) {
        stamps = reinterpret_cast<uint64_t*>(static_cast<char*>(ws) + queue_ws_bytes(cams, nv));
        const size_t n = (size_t)call_tiles(cams, nv) * 5 * 2;
        hipLaunchKernelGGL(fill_stamps_kernel, dim3((unsigned)std::min<size_t>(1024, (n + 255) / 256)), dim3(256), 0,
                           stream, stamps, n);
    }
    uint32_t p_off = 0, tile_base = 0, pix_off = 0;
    for (int v0 = 0; v0 < nv; v0 += kMaxViews) {
        RenderPack pk{};
        uint32_t blocks;
        const uint32_t tile0 = tile_base;
        fill_render_pack(pk, cams, n_per_view, v0, nv, p_off, tile_base, pix_off, blocks);
        set_render_limits(pk, n_per_view, nv, bins->capacity);
        if (!blocks) continue;
        const uint32_t* order = launch_tile_queue(q, bins->ranges, tile0, blocks, pk.n_entries_cap, stream);
        OrderedArgs a{reinterpret_cast<const float4*>(proj->record), reinterpret_cast<const float2*>(conic),
                      bins->pidx, bins->ranges, bins->status, bg[0], bg[1], bg[2], image, T_final, n_last,
                      reinterpret_cast<float4*>(ckpt), order, q, 0u,
                      stamps ? stamps + 2 * 5 * (size_t)tile0 : nullptr};
        if (flags & ISOGS_FWD_WIDE) {
            // a long tile holds at least 2^kWideMinLog2 of the group's entries
            a.wide_slots = (uint32_t)std::min<uint64_t>(blocks, (uint64_t)pk.n_entries_cap / (1u << kWideMinLog2) + 1);
            hipLaunchKernelGGL(an ? aniso_fwd_ordered_wide_kernel : composite_fwd_ordered_wide_kernel,
                               dim3(4 * a.wide_slots + blocks), dim3(256), 0, stream, pk, a);
        } else if (blocks <= kPipeTileLimit) {
            auto k = an ? (n_last ? aniso_fwd_ordered_pipe_kernel<true> : aniso_fwd_ordered_pipe_kernel<false>)
                        : (n_last ? composite_fwd_ordered_pipe_kernel<true> : composite_fwd_ordered_pipe_kernel<false>);
            hipLaunchKernelGGL(k, dim3(blocks), dim3(256), 0, stream, pk, a);
        } else {
            auto k = an ? (n_last ? aniso_fwd_ordered_kernel<true> : aniso_fwd_ordered_kernel<false>)
                        : (n_last ? composite_fwd_ordered_kernel<true> : composite_fwd_ordered_kernel<false>);
            hipLaunchKernelGGL(k, dim3(blocks), dim3(256), 0, stream, pk, a);
        }
        if (hipPeekAtLastError() != hipSuccess) return -1;
    }
    return 0;
}

}  // namespace isogs
