// Backward pass: gradients of a loss through compositing (eq. 4), the isotropic kernel
// (eq. 8), the projection and the spherical-harmonic colour.
//
//   1. composite_bwd  per tile: walk each pixel's entries in reverse from n_last,
//                     recovering T before each entry as T_after / (1 - alpha); reduce each
//                     entry's screen-space gradient over the tile's pixels (wavefront DPP
//                     sums, then the four waves in fixed order) into one record per entry,
//                     stored at the entry's emit position.
//   2. grad_project   per particle: sum its records (consecutive in emit order, views in
//                     order) and chain them to mu, sigma, o and the colour coefficients.
// There are no floating-point atomics: every sum has a fixed order.
#include <algorithm>

#include "raster.h"

namespace isogs {

// Entries staged per round, one per lane of a wave (the other lanes idle in staging): 48
// keeps LDS at about 25 KB per workgroup and measured faster than 32 or 64.
constexpr int kBwdBatch = 48;
static_assert(kBwdBatch <= kWave, "one staged entry per lane");
constexpr int kBwdDummy = kBwdBatch;   // staged slot of the zero-opacity pad record

// Per-entry gradient sums over a tile's pixels (dx = x - u, dy = y - v; k = dL/dalpha
// times the kernel value below the clamp, i.e. -dL/d(exponent); w = alpha T):
//   isotropic (7):    2 k dx / s^2, 2 k dy / s^2, -k d^2, k / o, dr w, dg w, db w
//   anisotropic (9):  k dx, k dy, k dx^2, k dx dy, k dy^2, k / o, dr w, dg w, db w
// (the anisotropic centre and conic gradients are these sums times the entry's conic,
// applied per particle). A record holds them in kRecVec4<AN> float4s at the entry's emit
// position.
template <bool AN>
constexpr int kGradTerms = AN ? 9 : 7;
template <bool AN>
constexpr int kRecVec4 = AN ? 3 : 2;

// One batch of a tile's entries in LDS, back to front, with the 16 sub-block lists.
template <bool AN>
struct StagedBwdT {
    float4 fp[kBwdBatch + 1];            // staged kernel (staged_kernel: {u, v, q or nA, log2(o)})
    float4 col[kBwdBatch + 1];           // {r, g, b, 1/o}
    float2 cn[AN ? kBwdBatch + 1 : 1];   // anisotropic: {nB2, nC}
    uint16_t list[16][kBwdBatch + 4];    // per sub-block, staged slots in walk order
    uint32_t slot[kBwdBatch];            // emit position of each staged entry
    uint8_t mask[4][kBwdBatch];          // [wave] which of its sub-blocks listed the entry
    float part[16][kGradTerms<AN>][kBwdBatch];   // per-sub-block gradient sums of each entry
    uint32_t gmax[16];                   // largest n_last of each sub-block
};

// Stages the nb entries below list position `hi` back to front (staged slot l holds entry
// hi - 1 - l, 1-based tile position pos_hi - l) and builds the 16 sub-block lists. Every
// wave tests the entries against its own quadrant's four sub-blocks, so the lists of a
// wave are built from its own ballots. An entry joins a sub-block's list when its binning
// disk touches the sub-block and its position is at most the sub-block's largest n_last
// (no later entry was composited there). Returns the number of list steps of the calling
// wave; `len` receives the padded length of this lane's row list. Contains __syncthreads.
template <bool AN>
__device__ __forceinline__ uint32_t stage_bwd(StagedBwdT<AN>& sb, const float4* __restrict__ record,
                                              const float2* __restrict__ conic, const uint32_t* __restrict__ pidx,
                                              const uint32_t* __restrict__ offsets, uint32_t n_particles,
                                              uint32_t hi, uint32_t nb, uint32_t pos_hi, int tx, int ty,
                                              int tiles_x, int tiles_y, float w_lim, float h_lim, uint32_t& len) {
    const uint32_t t = threadIdx.x, w = t >> 6, l = lane_id();
    const uint32_t g = l < nb ? pidx[hi - 1 - l] : 0xFFFFFFFFu;
    uint32_t mask = 0;
    if (g < n_particles) {
        const float4 f = record[2 * (size_t)g];
        const float4 c = record[2 * (size_t)g + 1];
        if (w == 0) {
            sb.fp[l] = staged_kernel<AN>(f);
            sb.col[l] = make_float4(c.x, c.y, c.z, __builtin_amdgcn_rcpf(f.w));   // once per entry
        } else if (w == 1) {
            sb.slot[l] = emit_slot(offsets[g], f.x, f.y, c.w, tx, ty, tiles_x, tiles_y, w_lim, h_lim);
        } else if (AN && w == 2) {
            sb.cn[l] = staged_conic(conic[g]);
        }
        const float r2 = c.w * c.w;
        const uint32_t pos1 = pos_hi - l;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int k = 4 * (int)w + r;
            if (pos1 <= sb.gmax[k] && sub_block_touched(f.x, f.y, r2, k, tx * kTile, ty * kTile, w_lim, h_lim))
                mask |= 1u << r;
        }
    } else if (w == 1 && l < (uint32_t)kBwdBatch) {
        sb.slot[l] = 0xFFFFFFFFu;
    }
    if (t == 0) {
        sb.fp[kBwdDummy] = make_float4(0.0f, 0.0f, 0.0f, -__builtin_inff());
        sb.col[kBwdDummy] = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
        if (AN) sb.cn[kBwdDummy] = make_float2(0.0f, 0.0f);
    }
    if (l < (uint32_t)kBwdBatch) sb.mask[w][l] = (uint8_t)mask;
    uint64_t bal[4];
    uint32_t cnt[4];
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        bal[r] = ballot64((mask >> r) & 1u);
        cnt[r] = (uint32_t)__popcll(bal[r]);
        if ((mask >> r) & 1u) sb.list[4 * w + r][rank_below(bal[r])] = (uint16_t)l;
    }
    if (l < 16) {
        // pad row l / 4 of this wave with dummies up to a multiple of four
        const uint32_t r = l >> 2;
        const uint32_t n = r == 0 ? cnt[0] : r == 1 ? cnt[1] : r == 2 ? cnt[2] : cnt[3];
        if (n + (l & 3u) < ((n + 3u) & ~3u)) sb.list[4 * w + r][n + (l & 3u)] = (uint16_t)kBwdDummy;
    }
    const uint32_t row = l >> 4;
    const uint32_t mine = row == 0 ? cnt[0] : row == 1 ? cnt[1] : row == 2 ? cnt[2] : cnt[3];
    len = (mine + 3u) & ~3u;
    const uint32_t most = max(max(cnt[0], cnt[1]), max(cnt[2], cnt[3]));
    __syncthreads();
    return (most + 3u) & ~3u;
}

// Reverse walk of one tile (logical index within the launch) by a 256-thread workgroup,
// one lane per pixel, each 16-lane row owning a 4x4 sub-block (the forward pixel layout).
// Record of an entry: its gradient sums (kGradTerms), at its emit position.
// With checkpoints (`ckpt` non-null) and a list of at least kChunkedMin entries, the
// workgroup walks only chunk `chunk` of the list, positions [chunk * kCkptChunk,
// (chunk + 1) * kCkptChunk); a pixel whose last entry lies beyond the chunk starts from the
// checkpoint at the chunk's end: T from there, and the light from behind = image - colour
// accumulated before the chunk's end. Shorter lists, and every list without checkpoints,
// are one chunk. Contains __syncthreads.
template <bool AN>
__device__ __forceinline__ void composite_bwd_tile(
    StagedBwdT<AN>& sb, const RenderPack& pk, uint32_t logical, uint32_t chunk, const float4* __restrict__ record,
    const float2* __restrict__ conic, const uint32_t* __restrict__ pidx, const uint32_t* __restrict__ offsets, const uint32_t* __restrict__ ranges,
    float bg_r, float bg_g, float bg_b, const float* __restrict__ image, const float* __restrict__ dL_dimage,
    const float* __restrict__ T_final, const uint32_t* __restrict__ n_last, const float4* __restrict__ ckpt,
    float4* __restrict__ rec) {
    int vi, tx, ty;
    locate_tile(pk, logical, vi, tx, ty);
    const ViewDesc& vd = pk.v[vi];
    const uint32_t t = threadIdx.x, w = t >> 6, lane = lane_id();
    const uint32_t sbk = 4 * w + ((t >> 4) & 3u);   // this lane's sub-block
    const int x = tx * kTile + sub_x(t), y = ty * kTile + sub_y(t);
    const bool inside = x < vd.width && y < vd.height;
    const float px = (float)x + 0.5f, py = (float)y + 0.5f;
    const uint32_t gt = vd.tile_base + (uint32_t)(ty * vd.tiles_x + tx);
    const uint32_t start = ranges[2 * gt], end = min(ranges[2 * gt + 1], pk.n_entries_cap);
    const float w_lim = (float)vd.width - 0.5f, h_lim = (float)vd.height - 0.5f;
    const uint32_t len = end > start ? end - start : 0u;
    // this workgroup's positions [c_lo, c_hi) of the list
    const bool chunked = ckpt && chunked_list(len);
    const uint32_t c_lo = chunked ? chunk * kCkptChunk : 0u;
    const uint32_t c_hi = chunked ? min(c_lo + kCkptChunk, len) : len;
    if (c_lo > c_hi) return;   // no such chunk (uniform over the workgroup)

    float T = 1.0f, dr = 0.0f, dg = 0.0f, db = 0.0f;
    float Sr = 0.0f, Sg = 0.0f, Sb = 0.0f;
    uint32_t last = 0;
    if (inside) {
        const size_t hw = (size_t)vd.width * vd.height;
        const size_t pix = (size_t)y * vd.width + x;
        const float* dimg = dL_dimage + (size_t)3 * vd.pix_off;
        dr = dimg[pix];
        dg = dimg[hw + pix];
        db = dimg[2 * hw + pix];
        last = n_last[vd.pix_off + pix];
        if (last > c_hi) {
            // the pixel composited entries beyond this chunk: state at the chunk's end
            const float4 s = ckpt[(size_t)ckpt_slot(start, c_hi / kCkptChunk) * 256 + t];
            const float* im = image + (size_t)3 * vd.pix_off;
            T = s.x;
            Sr = im[pix] - s.y;
            Sg = im[hw + pix] - s.z;
            Sb = im[2 * hw + pix] - s.w;
        } else {
            // light arriving from behind the last entry: T_final bg
            T = T_final[vd.pix_off + pix];
            Sr = T * bg_r;
            Sg = T * bg_g;
            Sb = T * bg_b;
        }
    }

    if (t < 16) sb.gmax[t] = 0u;
    __syncthreads();
    if (last > c_lo) atomicMax(&sb.gmax[sbk], min(last, c_hi));
    __syncthreads();
    uint32_t max_last = 0;
#pragma unroll
    for (int k = 0; k < 16; ++k) max_last = max(max_last, sb.gmax[k]);
    max_last = max(max_last, c_lo);   // 1-based end of the walk inside [c_lo, c_hi]

    // entries of the chunk no pixel reached carry zero gradient
    for (uint32_t e = start + max_last + t; e < start + c_hi; e += 256) {
        const uint32_t g = pidx[e];
        if (g < pk.n_particles) {
            const float4 f = record[2 * (size_t)g];
            const float r = record[2 * (size_t)g + 1].w;
            const uint32_t slot = emit_slot(offsets[g], f.x, f.y, r, tx, ty, vd.tiles_x, vd.tiles_y, w_lim, h_lim);
            if (slot < pk.n_entries_cap) {
#pragma unroll
                for (int q = 0; q < kRecVec4<AN>; ++q)
                    rec[kRecVec4<AN> * (size_t)slot + q] = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
            }
        }
    }

    const uint32_t q8 = rev3(lane & 7u);
    const bool writer = (lane & 15u) < 8u && q8 < (uint32_t)kGradTerms<AN>;
    const bool writer9 = AN && (lane & 15u) == 8u;   // the ninth sum
    for (uint32_t hi = start + max_last; hi > start + c_lo;) {
        const uint32_t nb = min((uint32_t)kBwdBatch, hi - start - c_lo);
        const uint32_t pos_hi = hi - start;
        uint32_t len;
        const uint32_t steps = stage_bwd(sb, record, conic, pidx, offsets, pk.n_particles, hi, nb, pos_hi, tx, ty,
                                         vd.tiles_x, vd.tiles_y, w_lim, h_lim, len);
        for (uint32_t k = 0; k < steps; k += 4) {
            constexpr uint64_t kD = (uint64_t)kBwdDummy;
            uint64_t q4 = kD | (kD << 16) | (kD << 32) | (kD << 48);   // four dummy slots
            if (k < len) q4 = *reinterpret_cast<const uint64_t*>(&sb.list[sbk][k]);
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const uint32_t j = (uint32_t)(q4 >> (16 * r)) & 0xFFFFu;
                const uint32_t pos1 = pos_hi - j;            // 1-based list position
                const float4 f = sb.fp[j];
                const float4 c = sb.col[j];
                const float2 kc = AN ? sb.cn[j] : make_float2(0.0f, 0.0f);
                const float dx = px - f.x, dy = py - f.y;
                float ga;
                float a = staged_alpha<AN>(dx, dy, f, kc, ga);
                // an entry this pixel composited in the forward pass (same decision); the
                // pad record has alpha 0
                const bool use = (pos1 <= last) && (a >= kAlphaMin);
                a = use ? a : 0.0f;
                const float inv_om = __builtin_amdgcn_rcpf(1.0f - a);
                T = T * inv_om;                              // transmittance before this entry
                const float wgt = a * T;
                const float dLda = dr * (c.x * T - Sr * inv_om) + dg * (c.y * T - Sg * inv_om) +
                                   db * (c.z * T - Sb * inv_om);
                Sr = fmaf(c.x, wgt, Sr);
                Sg = fmaf(c.y, wgt, Sg);
                Sb = fmaf(c.z, wgt, Sb);
                // alpha = o exp(-d^2 / s^2) below the clamp: d/du = 2 alpha dx / s^2,
                // d/d(1/s^2) = -alpha d^2, d/do = alpha / o
                const float kk = (use && ga < kAlphaMax) ? dLda * ga : 0.0f;
                float gv[8], g9 = 0.0f;
                if (!AN) {
                    const float inv_s2 = f.z * (1.0f / kLog2e);
                    gv[0] = 2.0f * kk * inv_s2 * dx;
                    gv[1] = 2.0f * kk * inv_s2 * dy;
                    gv[2] = -kk * fmaf(dx, dx, dy * dy);
                    gv[3] = kk * c.w;
                    gv[4] = dr * wgt;
                    gv[5] = dg * wgt;
                    gv[6] = db * wgt;
                    gv[7] = 0.0f;
                } else {
                    // alpha = o exp(-Q) below the clamp: dL/du = k (2 A dx + 2 B dy),
                    // dL/dA = -k dx^2, ...: the conic enters per particle
                    const float kx = kk * dx, ky = kk * dy;
                    gv[0] = kx;
                    gv[1] = ky;
                    gv[2] = kx * dx;
                    gv[3] = kx * dy;
                    gv[4] = ky * dy;
                    gv[5] = kk * c.w;
                    gv[6] = dr * wgt;
                    gv[7] = dg * wgt;
                    g9 = db * wgt;
                }
                const bool any = ballot64(use) != 0;
                const float red = any ? row_sum8(gv, lane) : 0.0f;
                if (writer && j != kBwdDummy) sb.part[sbk][q8][j] = red;
                if (AN) {
                    // the ninth sum over the row: butterfly (quad swaps, row rotations)
                    float r9 = g9;
                    if (any) {
                        r9 += dpp<0xB1>(r9);
                        r9 += dpp<0x4E>(r9);
                        r9 += dpp<0x124>(r9);
                        r9 += dpp<0x128>(r9);
                    }
                    if (writer9 && j != kBwdDummy) sb.part[sbk][kGradTerms<AN> - 1][j] = r9;
                }
            }
        }
        __syncthreads();
        // combine: the sub-blocks that listed an entry, in fixed order; wave w writes
        // float4 w of each record (sums 4w .. 4w + 3)
        const uint32_t l = lane;
        if (w < (uint32_t)kRecVec4<AN> && l < nb) {
            const uint32_t m = (uint32_t)sb.mask[0][l] | ((uint32_t)sb.mask[1][l] << 4) |
                               ((uint32_t)sb.mask[2][l] << 8) | ((uint32_t)sb.mask[3][l] << 12);
            const int q0 = 4 * (int)w;
            float s4[4] = {0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
            for (int k = 0; k < 16; ++k) {
                if ((m >> k) & 1u) {
#pragma unroll
                    for (int e = 0; e < 4; ++e)
                        if (q0 + e < kGradTerms<AN>) s4[e] += sb.part[k][q0 + e][l];
                }
            }
            const uint32_t slot = sb.slot[l];
            if (slot < pk.n_entries_cap)
                rec[kRecVec4<AN> * (size_t)slot + w] = make_float4(s4[0], s4[1], s4[2], s4[3]);
        }
        __syncthreads();
        hi -= nb;
    }
}

__global__ void __launch_bounds__(64) fill_u32_kernel_b(uint32_t* __restrict__ p, uint32_t n) {
    for (uint32_t i = threadIdx.x; i < n; i += blockDim.x) p[i] = 0u;
}

// Work items of the tiles whose list is longer than one checkpoint chunk: one
// (tile, chunk) pair per chunk, appended in any order, with one device-wide add per
// workgroup (adds to one counter from many XCDs are serialised in memory).
__global__ void __launch_bounds__(256) bwd_chunk_list_kernel(const uint32_t* __restrict__ ranges, uint32_t tile0,
                                                             uint32_t n_tiles, uint32_t cap,
                                                             const int32_t* __restrict__ status,
                                                             uint32_t* __restrict__ heavy,
                                                             uint32_t* __restrict__ heavy_count,
                                                             uint32_t heavy_max) {
    __shared__ uint32_t s_wave[4];
    __shared__ uint32_t s_base;
    if (*status != kStatusOk) return;
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x, w = threadIdx.x >> 6, lane = threadIdx.x & 63u;
    uint32_t nch = 0;
    if (i < n_tiles) {
        const uint32_t s = ranges[2 * (tile0 + i)], e = min(ranges[2 * (tile0 + i) + 1], cap);
        const uint32_t len = e > s ? e - s : 0u;
        if (chunked_list(len)) nch = (len + kCkptChunk - 1) / kCkptChunk;
    }
    uint32_t incl = nch;
#pragma unroll
    for (uint32_t o = 1; o < 64; o <<= 1) {
        const uint32_t y = __shfl_up(incl, o, 64);
        if (lane >= o) incl += y;
    }
    if (lane == 63) s_wave[w] = incl;
    __syncthreads();
    uint32_t before = 0, total = 0;
#pragma unroll
    for (uint32_t q = 0; q < 4; ++q) {
        const uint32_t c = s_wave[q];
        before += q < w ? c : 0u;
        total += c;
    }
    if (threadIdx.x == 0) s_base = total ? atomicAdd(heavy_count, total) : 0u;
    __syncthreads();
    const uint32_t base = s_base + before + incl - nch;
    if (!nch || base + nch > heavy_max) return;   // the bound holds for ranges that partition the entries
    for (uint32_t c = 0; c < nch; ++c) {
        heavy[2 * (base + c)] = i;
        heavy[2 * (base + c) + 1] = c;
    }
}

// One workgroup per work item, in dispatch order. With checkpoints: workgroups
// [0, n_chunks) take the chunks of the long tiles (listed by bwd_chunk_list_kernel), the
// next ones the other tiles in longest-list-first order (they follow the long ones in the
// queue, whose length classes tell how many those are); a workgroup past the last item
// leaves at once. Without: workgroup b walks the tile at queue position b whole.
struct BwdArgs {
    const float4* record;
    const float2* conic;     // anisotropic family: {B, C} per record
    const uint32_t* pidx;
    const uint32_t* offsets;
    const uint32_t* ranges;
    const int32_t* status;
    float bg_r, bg_g, bg_b;
    const float* image;
    const float* dL_dimage;
    const float* T_final;
    const uint32_t* n_last;
    const float4* ckpt;
    float4* rec;
    const uint32_t* order;
    const uint32_t* hist;
    uint32_t n_items;
    const uint32_t* heavy;
    const uint32_t* heavy_count;
    uint32_t heavy_max;
};

template <bool AN>
__device__ __forceinline__ void bwd_ordered(StagedBwdT<AN>& sb, const RenderPack& pk, const BwdArgs& A) {
    const float4* __restrict__ ckpt = A.ckpt;
    const uint32_t* __restrict__ heavy = A.heavy;
    const uint32_t* __restrict__ order = A.order;
    const uint32_t* __restrict__ hist = A.hist;
    const uint32_t n_items = A.n_items, heavy_max = A.heavy_max;
    if (*A.status != kStatusOk) return;
    const uint32_t b = blockIdx.x;
    uint32_t logical, chunk = 0;
    if (ckpt) {
        const uint32_t n_heavy = min(*A.heavy_count, heavy_max);
        if (b < n_heavy) {
            logical = heavy[2 * b];
            chunk = heavy[2 * b + 1];
            if (logical >= n_items) return;
        } else {
            uint32_t n_long = 0;
            for (int c = kChunkedClass; c < kBuckets; ++c) n_long += hist[c];
            const uint32_t j = n_long + (b - n_heavy);
            if (j >= n_items) return;
            logical = order[j];
        }
    } else {
        logical = order[b];
    }
    composite_bwd_tile(sb, pk, logical, chunk, A.record, A.conic, A.pidx, A.offsets, A.ranges, A.bg_r, A.bg_g, A.bg_b,
                       A.image, A.dL_dimage, A.T_final, A.n_last, ckpt, A.rec);
}

__global__ void __launch_bounds__(256) composite_bwd_ordered_kernel(const RenderPack pk, const BwdArgs a) {
    __shared__ StagedBwdT<false> sb;
    bwd_ordered(sb, pk, a);
}

// The anisotropic family (eq. 5 kernels).
__global__ void __launch_bounds__(256) aniso_bwd_ordered_kernel(const RenderPack pk, const BwdArgs a) {
    __shared__ StagedBwdT<true> sb;
    bwd_ordered(sb, pk, a);
}

struct GradView {
    uint32_t p_off;
    float R[9], t[3], eye[3], f, cx, cy;
};

// Real SH basis polynomial K (the forms of the forward colour evaluation) and its gradient
// at direction (x, y, z); K is a compile-time constant, so each call folds to its own term.
template <int K>
__device__ __forceinline__ void sh_term(float x, float y, float z, float& Y, float& gx, float& gy, float& gz) {
    constexpr float c1 = 0.48860251190291992f, c2a = 1.09254843059207907f, c2b = 0.31539156525252005f,
                    c2c = 0.54627421529603959f, c3a = 0.59004358992664352f, c3b = 2.89061144264055405f,
                    c3c = 0.45704579946446573f, c3d = 0.37317633259011540f, c3e = 1.44530572132027702f;
    const float xx = x * x, yy = y * y, zz = z * z;
    gx = gy = gz = 0.0f;
    if constexpr (K == 1) { Y = c1 * y; gy = c1; }
    else if constexpr (K == 2) { Y = c1 * z; gz = c1; }
    else if constexpr (K == 3) { Y = c1 * x; gx = c1; }
    else if constexpr (K == 4) { Y = c2a * x * y; gx = c2a * y; gy = c2a * x; }
    else if constexpr (K == 5) { Y = c2a * y * z; gy = c2a * z; gz = c2a * y; }
    else if constexpr (K == 6) { Y = c2b * (3.0f * zz - 1.0f); gz = 6.0f * c2b * z; }
    else if constexpr (K == 7) { Y = c2a * x * z; gx = c2a * z; gz = c2a * x; }
    else if constexpr (K == 8) { Y = c2c * (xx - yy); gx = 2.0f * c2c * x; gy = -2.0f * c2c * y; }
    else if constexpr (K == 9) { Y = c3a * y * (3.0f * xx - yy); gx = 6.0f * c3a * x * y; gy = 3.0f * c3a * (xx - yy); }
    else if constexpr (K == 10) { Y = c3b * x * y * z; gx = c3b * y * z; gy = c3b * x * z; gz = c3b * x * y; }
    else if constexpr (K == 11) { Y = c3c * y * (5.0f * zz - 1.0f); gy = c3c * (5.0f * zz - 1.0f); gz = 10.0f * c3c * y * z; }
    else if constexpr (K == 12) { Y = c3d * z * (5.0f * zz - 3.0f); gz = c3d * (15.0f * zz - 3.0f); }
    else if constexpr (K == 13) { Y = c3c * x * (5.0f * zz - 1.0f); gx = c3c * (5.0f * zz - 1.0f); gz = 10.0f * c3c * x * z; }
    else if constexpr (K == 14) { Y = c3e * z * (xx - yy); gx = 2.0f * c3e * x * z; gy = -2.0f * c3e * y * z; gz = c3e * (xx - yy); }
    else { static_assert(K == 15, "degree 3 at most"); Y = c3a * x * (xx - 3.0f * yy); gx = 3.0f * c3a * (xx - yy); gy = -6.0f * c3a * x * y; }
}

// The coefficients of one particle, held in registers across the views: coefficient k of
// channel ch at c[3 k + ch].
struct CoefRef {
    const float* c;
    __device__ float operator()(int k, int ch) const { return c[3 * k + ch]; }
};

// Colour of one view, rgb = max(0, c_0 + sum_k c_k Y_k(d)) with d = (mu - eye)/|mu - eye|:
// adds the view's gradient (drgb, zero where the colour was clamped) to the coefficients'
// and to the centre's (through the direction's tangential part). Each channel's sum runs
// over k in ascending order, as in the forward evaluation, so the clamp decision agrees.
template <int DEG, int KK = 1>
__device__ __forceinline__ void sh_raw(const CoefRef& coef, float x, float y, float z, float raw[3]) {
    if constexpr (KK < (DEG + 1) * (DEG + 1)) {
        float Y, gx, gy, gz;
        sh_term<KK>(x, y, z, Y, gx, gy, gz);
#pragma unroll
        for (int ch = 0; ch < 3; ++ch) raw[ch] = fmaf(coef(KK, ch), Y, raw[ch]);
        sh_raw<DEG, KK + 1>(coef, x, y, z, raw);
    }
}

template <int DEG, int KK = 1>
__device__ __forceinline__ void sh_back(const CoefRef& coef, float x, float y, float z, const float d[3], float* gcol,
                                        float& wdx, float& wdy, float& wdz) {
    if constexpr (KK < (DEG + 1) * (DEG + 1)) {
        float Y, gx, gy, gz;
        sh_term<KK>(x, y, z, Y, gx, gy, gz);
#pragma unroll
        for (int ch = 0; ch < 3; ++ch) {
            gcol[3 * KK + ch] += d[ch] * Y;
            const float wk = d[ch] * coef(KK, ch);
            wdx = fmaf(wk, gx, wdx);
            wdy = fmaf(wk, gy, wdy);
            wdz = fmaf(wk, gz, wdz);
        }
        sh_back<DEG, KK + 1>(coef, x, y, z, d, gcol, wdx, wdy, wdz);
    }
}

template <int DEG>
__device__ __forceinline__ void color_backward(const CoefRef& coef, const float drgb[3], const float eye[3], float mx,
                                               float my, float mz, float* gcol, float& gmx, float& gmy, float& gmz) {
    const float ex = mx - eye[0], ey = my - eye[1], ez = mz - eye[2];
    const float inv_dist = 1.0f / sqrtf(ex * ex + ey * ey + ez * ez);
    const float dxn = ex * inv_dist, dyn = ey * inv_dist, dzn = ez * inv_dist;
    float raw[3] = {coef(0, 0), coef(0, 1), coef(0, 2)};
    sh_raw<DEG>(coef, dxn, dyn, dzn, raw);
    float d[3];
#pragma unroll
    for (int ch = 0; ch < 3; ++ch) {
        d[ch] = (raw[ch] > 0.0f) ? drgb[ch] : 0.0f;
        gcol[ch] += d[ch];
    }
    float wdx = 0.0f, wdy = 0.0f, wdz = 0.0f;
    sh_back<DEG>(coef, dxn, dyn, dzn, d, gcol, wdx, wdy, wdz);
    const float radial = wdx * dxn + wdy * dyn + wdz * dzn;
    gmx += (wdx - radial * dxn) * inv_dist;
    gmy += (wdy - radial * dyn) * inv_dist;
    gmz += (wdz - radial * dzn) * inv_dist;
}

struct GradPack {
    int32_t nv;            // views of this scene in this launch, in view order
    int32_t accumulate;    // add to the outputs (a previous launch covered earlier views)
    const float* pos;
    const float* scale;
    const float* opacity;
    const float* color;
    uint32_t n;
    int32_t sh_degree;
    float* g_pos;
    float* g_scale;
    float* g_opacity;
    float* g_color;
    GradView v[kMaxViews];
};

// One thread per particle of one scene; DEG is the scene's SH degree.
template <int DEG>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(3))) grad_project_kernel(const GradPack pk, const float4* __restrict__ rec,
                                                           const uint32_t* __restrict__ tile_count,
                                                           const uint32_t* __restrict__ offsets,
                                                           const uint32_t* __restrict__ count_p,
                                                           const int32_t* __restrict__ status) {
    if (*status != kStatusOk) return;
    const uint32_t n_entries = *count_p;
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= pk.n) return;
    const uint32_t n = pk.n;
    constexpr int K = (DEG + 1) * (DEG + 1);
    const float mx = pk.pos[i], my = pk.pos[n + i], mz = pk.pos[2 * n + i];
    const float sigma = pk.scale[i];

    float gmx = 0.0f, gmy = 0.0f, gmz = 0.0f, gsig = 0.0f, gop = 0.0f;
    float gcol[3 * K];
    float coef[3 * K];
#pragma unroll
    for (int k = 0; k < 3 * K; ++k) {
        gcol[k] = 0.0f;
        coef[k] = pk.color[(size_t)k * n + i];
    }

    for (int vv = 0; vv < pk.nv; ++vv) {
        const GradView& gv = pk.v[vv];
        const uint32_t pi = gv.p_off + i;
        const uint32_t cnt = tile_count[pi];
        if (cnt == 0) continue;
        const uint32_t e0 = offsets[pi];
        if ((uint64_t)e0 + cnt > n_entries) continue;
        float du = 0.0f, dv = 0.0f, dis2 = 0.0f, dop = 0.0f, drgb[3] = {0.0f, 0.0f, 0.0f};
        for (uint32_t e = e0; e < e0 + cnt; ++e) {
            const float4 a = rec[2 * (size_t)e];
            const float4 b = rec[2 * (size_t)e + 1];
            du += a.x;
            dv += a.y;
            dis2 += a.z;
            dop += a.w;
            drgb[0] += b.x;
            drgb[1] += b.y;
            drgb[2] += b.z;
        }
        gop += dop;
        // projection: p = R mu + t, u = f p_x/z + cx, v = f p_y/z + cy, s = f sigma/z, 1/s^2
        const double pxd = (double)gv.R[0] * mx + (double)gv.R[1] * my + (double)gv.R[2] * mz + (double)gv.t[0];
        const double pyd = (double)gv.R[3] * mx + (double)gv.R[4] * my + (double)gv.R[5] * mz + (double)gv.t[1];
        const double pzd = (double)gv.R[6] * mx + (double)gv.R[7] * my + (double)gv.R[8] * mz + (double)gv.t[2];
        const float inv_z = (float)(1.0 / pzd);
        const float s = (float)((double)gv.f * (double)sigma / pzd);
        const float inv_s = 1.0f / s;
        // d(1/s^2)/ds = -2/s^3
        const float ds = -2.0f * dis2 * inv_s * inv_s * inv_s;
        gsig += ds * gv.f * inv_z;
        const float gpx = du * gv.f * inv_z, gpy = dv * gv.f * inv_z;
        const float ucx = (float)((double)gv.f * pxd / pzd), vcy = (float)((double)gv.f * pyd / pzd);
        const float gpz = -(ds * s + du * ucx + dv * vcy) * inv_z;
        gmx += gv.R[0] * gpx + gv.R[3] * gpy + gv.R[6] * gpz;
        gmy += gv.R[1] * gpx + gv.R[4] * gpy + gv.R[7] * gpz;
        gmz += gv.R[2] * gpx + gv.R[5] * gpy + gv.R[8] * gpz;
        color_backward<DEG>(CoefRef{coef}, drgb, gv.eye, mx, my, mz, gcol, gmx, gmy, gmz);
    }
    if (pk.accumulate) {
        pk.g_pos[i] += gmx;
        pk.g_pos[n + i] += gmy;
        pk.g_pos[2 * n + i] += gmz;
        pk.g_scale[i] += gsig;
        pk.g_opacity[i] += gop;
#pragma unroll
        for (int k = 0; k < 3 * K; ++k) pk.g_color[(size_t)k * n + i] += gcol[k];
    } else {
        pk.g_pos[i] = gmx;
        pk.g_pos[n + i] = gmy;
        pk.g_pos[2 * n + i] = gmz;
        pk.g_scale[i] = gsig;
        pk.g_opacity[i] = gop;
#pragma unroll
        for (int k = 0; k < 3 * K; ++k) pk.g_color[(size_t)k * n + i] = gcol[k];
    }
}

// ---- Anisotropic chain rule (eq. 5-7) ------------------------------------------------------
struct AnisoGradPack {
    int32_t nv;            // views of this scene in this launch, in view order
    int32_t accumulate;    // add to the outputs (a previous launch covered earlier views)
    const float* pos;
    const float* rot;
    const float* scale;
    const float* opacity;
    const float* color;
    uint32_t n;
    int32_t sh_degree;
    float* g_pos;
    float* g_rot;
    float* g_scale;
    float* g_opacity;
    float* g_color;
    GradView v[kMaxViews];
};

// Rotation matrix of the unit quaternion (w, x, y, z), row-major.
__device__ __forceinline__ void quat_rot(double w, double x, double y, double z, double R[9]) {
    R[0] = 1.0 - 2.0 * (y * y + z * z); R[1] = 2.0 * (x * y - w * z);       R[2] = 2.0 * (x * z + w * y);
    R[3] = 2.0 * (x * y + w * z);       R[4] = 1.0 - 2.0 * (x * x + z * z); R[5] = 2.0 * (y * z - w * x);
    R[6] = 2.0 * (x * z - w * y);       R[7] = 2.0 * (y * z + w * x);       R[8] = 1.0 - 2.0 * (x * x + y * y);
}

// One thread per particle of one scene. Per view: the entry records of the particle are
// summed in emit order (FP32, fixed order), turned into the gradients of the footprint
// centre (u, v), the conic (A, B, C), the opacity and the colour, and chained in FP64
// through Sigma_2D = T Sigma T^T (T = J V, eq. 7; conic = Sigma_2D^-1) to the centre and,
// accumulated over the views, to Sigma = R S S^T R^T (eq. 6), hence to the quaternion
// (through its normalisation) and the three scales.
template <int DEG>
__global__ void __launch_bounds__(256) aniso_grad_project_kernel(const AnisoGradPack pk, const float4* __restrict__ rec,
                                                                 const float4* __restrict__ record,
                                                                 const float2* __restrict__ conic,
                                                                 const uint32_t* __restrict__ tile_count,
                                                                 const uint32_t* __restrict__ offsets,
                                                                 const uint32_t* __restrict__ count_p,
                                                                 const int32_t* __restrict__ status) {
    if (*status != kStatusOk) return;
    const uint32_t n_entries = *count_p;
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= pk.n) return;
    const uint32_t n = pk.n;
    constexpr int K = (DEG + 1) * (DEG + 1);
    const float mx = pk.pos[i], my = pk.pos[n + i], mz = pk.pos[2 * n + i];
    const double qw = pk.rot[i], qx = pk.rot[n + i], qy = pk.rot[2 * n + i], qz = pk.rot[3 * n + i];
    const double sc[3] = {(double)pk.scale[i], (double)pk.scale[n + i], (double)pk.scale[2 * n + i]};
    const double qn = sqrt(qw * qw + qx * qx + qy * qy + qz * qz);
    const double hw = qw / qn, hx = qx / qn, hy = qy / qn, hz = qz / qn;
    double Rq[9];
    quat_rot(hw, hx, hy, hz, Rq);
    // Sigma = R diag(s^2) R^T
    double Sig[9];
#pragma unroll
    for (int a = 0; a < 3; ++a)
#pragma unroll
        for (int b = 0; b < 3; ++b) {
            double acc = 0.0;
#pragma unroll
            for (int c = 0; c < 3; ++c) acc += Rq[3 * a + c] * sc[c] * sc[c] * Rq[3 * b + c];
            Sig[3 * a + b] = acc;
        }

    float gmx = 0.0f, gmy = 0.0f, gmz = 0.0f, gop = 0.0f;
    double GS[9];   // dL/dSigma, summed over the views
#pragma unroll
    for (int k = 0; k < 9; ++k) GS[k] = 0.0;
    double gmu64[3] = {0.0, 0.0, 0.0};
    bool any = false;
    float gcol[3 * K];
    float coef[3 * K];
#pragma unroll
    for (int k = 0; k < 3 * K; ++k) {
        gcol[k] = 0.0f;
        coef[k] = pk.color[(size_t)k * n + i];
    }

    for (int vv = 0; vv < pk.nv; ++vv) {
        const GradView& gv = pk.v[vv];
        const uint32_t pi = gv.p_off + i;
        const uint32_t cnt = tile_count[pi];
        if (cnt == 0) continue;
        const uint32_t e0 = offsets[pi];
        if ((uint64_t)e0 + cnt > n_entries) continue;
        any = true;
        float S[12];
#pragma unroll
        for (int k = 0; k < 12; ++k) S[k] = 0.0f;
        for (uint32_t e = e0; e < e0 + cnt; ++e) {
#pragma unroll
            for (int q = 0; q < 3; ++q) {
                const float4 r = rec[3 * (size_t)e + q];
                S[4 * q] += r.x;
                S[4 * q + 1] += r.y;
                S[4 * q + 2] += r.z;
                S[4 * q + 3] += r.w;
            }
        }
        gop += S[5];
        const double A = (double)record[2 * (size_t)pi].z;
        const float2 bc = conic[pi];
        const double B = (double)bc.x, C = (double)bc.y;
        // sums k dx, k dy, k dx^2, k dx dy, k dy^2 -> gradients of u, v and the conic
        const double du = 2.0 * (A * S[0] + B * S[1]), dv = 2.0 * (B * S[0] + C * S[1]);
        const double dA = -(double)S[2], dB = -2.0 * (double)S[3], dC = -(double)S[4];
        // dL/dSigma_2D = -Ci Gc Ci, Ci = [[A, B], [B, C]], Gc = [[dA, dB/2], [dB/2, dC]]
        const double m00 = A * dA + B * 0.5 * dB, m01 = A * 0.5 * dB + B * dC;
        const double m10 = B * dA + C * 0.5 * dB, m11 = B * 0.5 * dB + C * dC;
        const double G00 = -(m00 * A + m01 * B), G01 = -(m00 * B + m01 * C), G11 = -(m10 * B + m11 * C);
        // camera-space centre and T = J V
        double V[9];
#pragma unroll
        for (int k = 0; k < 9; ++k) V[k] = (double)gv.R[k];
        const double px = V[0] * mx + V[1] * my + V[2] * mz + (double)gv.t[0];
        const double py = V[3] * mx + V[4] * my + V[5] * mz + (double)gv.t[1];
        const double pz = V[6] * mx + V[7] * my + V[8] * mz + (double)gv.t[2];
        const double f = (double)gv.f, iz = 1.0 / pz;
        const double J00 = f * iz, J02 = -f * px * iz * iz, J12 = -f * py * iz * iz;
        double T[6];
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            T[c] = J00 * V[c] + J02 * V[6 + c];
            T[3 + c] = J00 * V[3 + c] + J12 * V[6 + c];
        }
        // dL/dSigma += T^T G T
#pragma unroll
        for (int a = 0; a < 3; ++a)
#pragma unroll
            for (int b = 0; b < 3; ++b)
                GS[3 * a + b] += T[a] * (G00 * T[b] + G01 * T[3 + b]) + T[3 + a] * (G01 * T[b] + G11 * T[3 + b]);
        // dL/dT = 2 G T Sigma, dL/dJ = dL/dT V^T
        double TS[6];
#pragma unroll
        for (int r = 0; r < 2; ++r)
#pragma unroll
            for (int c = 0; c < 3; ++c)
                TS[3 * r + c] = T[3 * r] * Sig[c] + T[3 * r + 1] * Sig[3 + c] + T[3 * r + 2] * Sig[6 + c];
        double GT[6];
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            GT[c] = 2.0 * (G00 * TS[c] + G01 * TS[3 + c]);
            GT[3 + c] = 2.0 * (G01 * TS[c] + G11 * TS[3 + c]);
        }
        double GJ[6];
#pragma unroll
        for (int r = 0; r < 2; ++r)
#pragma unroll
            for (int c = 0; c < 3; ++c)
                GJ[3 * r + c] = GT[3 * r] * V[3 * c] + GT[3 * r + 1] * V[3 * c + 1] + GT[3 * r + 2] * V[3 * c + 2];
        // J = [[f/z, 0, -f p_x/z^2], [0, f/z, -f p_y/z^2]]; u = f p_x / z + cx, v likewise
        const double iz2 = iz * iz;
        double dpx = -GJ[2] * f * iz2 + du * f * iz;
        double dpy = -GJ[5] * f * iz2 + dv * f * iz;
        double dpz = -(GJ[0] + GJ[4]) * f * iz2 + 2.0 * f * (GJ[2] * px + GJ[5] * py) * iz2 * iz -
                     (du * f * px + dv * f * py) * iz2;
        gmu64[0] += V[0] * dpx + V[3] * dpy + V[6] * dpz;
        gmu64[1] += V[1] * dpx + V[4] * dpy + V[7] * dpz;
        gmu64[2] += V[2] * dpx + V[5] * dpy + V[8] * dpz;
        const float drgb[3] = {S[6], S[7], S[8]};
        color_backward<DEG>(CoefRef{coef}, drgb, gv.eye, mx, my, mz, gcol, gmx, gmy, gmz);
    }
    float grot[4] = {0.0f, 0.0f, 0.0f, 0.0f}, gsc[3] = {0.0f, 0.0f, 0.0f};
    if (any) {
        // Sigma = R diag(s^2) R^T: dL/dR = 2 GS R diag(s^2), dL/ds_b = 2 s_b (R^T GS R)_bb
        double GR[9];
#pragma unroll
        for (int a = 0; a < 3; ++a)
#pragma unroll
            for (int b = 0; b < 3; ++b)
                GR[3 * a + b] = 2.0 * (GS[3 * a] * Rq[b] + GS[3 * a + 1] * Rq[3 + b] + GS[3 * a + 2] * Rq[6 + b]) *
                                sc[b] * sc[b];
#pragma unroll
        for (int b = 0; b < 3; ++b) {
            double acc = 0.0;
#pragma unroll
            for (int a = 0; a < 3; ++a)
#pragma unroll
                for (int c = 0; c < 3; ++c) acc += Rq[3 * a + b] * GS[3 * a + c] * Rq[3 * c + b];
            gsc[b] = (float)(2.0 * sc[b] * acc);
        }
        // dR/d(w, x, y, z) of the rotation formula, at the unit quaternion
        const double w = hw, x = hx, y = hy, z = hz;
        const double dRw[9] = {0.0, -2 * z, 2 * y, 2 * z, 0.0, -2 * x, -2 * y, 2 * x, 0.0};
        const double dRx[9] = {0.0, 2 * y, 2 * z, 2 * y, -4 * x, -2 * w, 2 * z, 2 * w, -4 * x};
        const double dRy[9] = {-4 * y, 2 * x, 2 * w, 2 * x, 0.0, 2 * z, -2 * w, 2 * z, -4 * y};
        const double dRz[9] = {-4 * z, -2 * w, 2 * x, 2 * w, -4 * z, 2 * y, 2 * x, 2 * y, 0.0};
        double dq[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
        for (int k = 0; k < 9; ++k) {
            dq[0] += GR[k] * dRw[k];
            dq[1] += GR[k] * dRx[k];
            dq[2] += GR[k] * dRy[k];
            dq[3] += GR[k] * dRz[k];
        }
        // through the normalisation q / |q|
        const double radial = hw * dq[0] + hx * dq[1] + hy * dq[2] + hz * dq[3];
        grot[0] = (float)((dq[0] - hw * radial) / qn);
        grot[1] = (float)((dq[1] - hx * radial) / qn);
        grot[2] = (float)((dq[2] - hy * radial) / qn);
        grot[3] = (float)((dq[3] - hz * radial) / qn);
        gmx += (float)gmu64[0];
        gmy += (float)gmu64[1];
        gmz += (float)gmu64[2];
    }
    if (pk.accumulate) {
        pk.g_pos[i] += gmx;
        pk.g_pos[n + i] += gmy;
        pk.g_pos[2 * n + i] += gmz;
#pragma unroll
        for (int k = 0; k < 4; ++k) pk.g_rot[(size_t)k * n + i] += grot[k];
#pragma unroll
        for (int k = 0; k < 3; ++k) pk.g_scale[(size_t)k * n + i] += gsc[k];
        pk.g_opacity[i] += gop;
#pragma unroll
        for (int k = 0; k < 3 * K; ++k) pk.g_color[(size_t)k * n + i] += gcol[k];
    } else {
        pk.g_pos[i] = gmx;
        pk.g_pos[n + i] = gmy;
        pk.g_pos[2 * n + i] = gmz;
#pragma unroll
        for (int k = 0; k < 4; ++k) pk.g_rot[(size_t)k * n + i] = grot[k];
#pragma unroll
        for (int k = 0; k < 3; ++k) pk.g_scale[(size_t)k * n + i] = gsc[k];
        pk.g_opacity[i] = gop;
#pragma unroll
        for (int k = 0; k < 3 * K; ++k) pk.g_color[(size_t)k * n + i] = gcol[k];
    }
}

static size_t round256(size_t b) { return (b + 255) & ~(size_t)255; }

// Workspace: gradient records (32 B per entry of capacity, 48 B for the anisotropic
// family), the tile queue, the chunk item count and the chunk items (two words each; at
// most capacity / kCkptChunk + tiles).
static size_t bwd_heavy_items(uint64_t capacity, uint32_t tiles) {
    return (size_t)(capacity / kCkptChunk) + tiles + 1;
}

static size_t rec_bytes(bool an) { return an ? 48 : 32; }

size_t render_bwd_ws(uint64_t capacity, const isogs_camera* cams, int32_t nv, bool an) {
    const uint32_t tiles = max_group_tiles(cams, nv);
    return round256((size_t)capacity * rec_bytes(an)) + round256(tile_queue_words(tiles) * 4) + 256 +
           bwd_heavy_items(capacity, tiles) * 8 + 256;
}

// Reverse compositing of every view into the entry records (both families): chunks of
// long tiles (with checkpoints), then tiles longest first. Returns the records.
static float4* launch_composite_bwd(bool an, const int32_t* n_all, const isogs_camera* cams, int32_t nv,
                                    const isogs_projected* proj, const float* conic, const isogs_bins* bins,
                                    const float* bg, const float* image, const float* dL_dimage,
                                    const float* T_final, const uint32_t* n_last, const float* ckpt, void* ws,
                                    hipStream_t stream) {
    const uint32_t max_tiles = max_group_tiles(cams, nv);
    char* base = static_cast<char*>(ws);
    float4* rec = reinterpret_cast<float4*>(base);
    base += round256((size_t)bins->capacity * rec_bytes(an));
    uint32_t* q = reinterpret_cast<uint32_t*>(base);
    base += round256(tile_queue_words(max_tiles) * 4);
    uint32_t* heavy_count = reinterpret_cast<uint32_t*>(base);
    uint32_t* heavy = reinterpret_cast<uint32_t*>(base + 256);
    const uint32_t heavy_max = (uint32_t)bwd_heavy_items(bins->capacity, max_tiles);
    // a long tile of len entries has ceil(len / kCkptChunk) chunks, at most len / kCkptChunk
    // more items than tiles; over ranges that partition the entries, at most
    // capacity / kCkptChunk more in all
    const uint32_t extra_items = ckpt ? (uint32_t)(bins->capacity / kCkptChunk) + 1u : 0u;
    uint32_t p_off = 0, tile_base = 0, pix_off = 0;
    for (int v0 = 0; v0 < nv; v0 += kMaxViews) {
        const int m = min(kMaxViews, nv - v0);
        RenderPack pk{};
        uint32_t blocks;
        const uint32_t tile0 = tile_base;
        fill_render_pack(pk, cams + v0, n_all + v0, 0, m, p_off, tile_base, pix_off, blocks);
        set_render_limits(pk, n_all, nv, bins->capacity);
        if (!blocks) continue;
        uint32_t* order = launch_tile_queue(q, bins->ranges, tile0, blocks, pk.n_entries_cap, stream);
        if (ckpt) {
            hipLaunchKernelGGL(fill_u32_kernel_b, dim3(1), dim3(64), 0, stream, heavy_count, 1u);
            hipLaunchKernelGGL(bwd_chunk_list_kernel, dim3((blocks + 255) / 256), dim3(256), 0, stream, bins->ranges,
                               tile0, blocks, pk.n_entries_cap, bins->status, heavy, heavy_count, heavy_max);
        }
        const BwdArgs a{reinterpret_cast<const float4*>(proj->record), reinterpret_cast<const float2*>(conic),
                        bins->pidx, bins->offsets, bins->ranges, bins->status, bg[0], bg[1], bg[2], image, dL_dimage,
                        T_final, n_last, reinterpret_cast<const float4*>(ckpt), rec, order, q, blocks, heavy,
                        heavy_count, heavy_max};
        hipLaunchKernelGGL(an ? aniso_bwd_ordered_kernel : composite_bwd_ordered_kernel, dim3(blocks + extra_items),
                           dim3(256), 0, stream, pk, a);
        if (hipPeekAtLastError() != hipSuccess) return nullptr;
    }
    return rec;
}

// Views grouped by scene (equal position buffers), in view order; calls fn(first view of
// the scene, views[], count) for each scene.
template <typename Fn>
static void for_each_scene(const float* const* pos, int32_t nv, Fn fn) {
    bool handled[4096] = {false};
    for (int v = 0; v < nv; ++v) {
        if (handled[v]) continue;
        int pending[4096];
        int np = 0;
        for (int u = v; u < nv; ++u)
            if (!handled[u] && pos[u] == pos[v]) {
                handled[u] = true;
                pending[np++] = u;
            }
        fn(v, pending, np);
    }
}

static void fill_grad_view(GradView& g, const isogs_camera& c, uint32_t p_off) {
    g.p_off = p_off;
    for (int k = 0; k < 9; ++k) g.R[k] = c.R[k];
    for (int k = 0; k < 3; ++k) g.t[k] = c.t[k], g.eye[k] = c.eye[k];
    g.f = c.f;
    g.cx = c.cx;
    g.cy = c.cy;
}

int launch_render_bwd(const isogs_scene* scenes, const isogs_camera* cams, int32_t nv,
                      const isogs_projected* proj, const isogs_bins* bins, const float* bg,
                      const float* image, const float* dL_dimage, const float* T_final, const uint32_t* n_last,
                      const float* ckpt, const isogs_scene* grads, void* ws, hipStream_t stream) {
    if (nv > 4096) return -1;
    int32_t n_all[4096];
    uint32_t view_off[4096];
    const float* pos[4096];
    uint32_t o = 0;
    for (int v = 0; v < nv; ++v) {
        n_all[v] = scenes[v].n;
        view_off[v] = o;
        o += (uint32_t)scenes[v].n;
        pos[v] = scenes[v].pos;
    }
    // 1. reverse compositing
    const float4* rec = launch_composite_bwd(false, n_all, cams, nv, proj, nullptr, bins, bg, image, dL_dimage, T_final,
                                             n_last, ckpt, ws, stream);
    if (!rec) return -1;
    // 2. per scene: reduce records over its views (in view order) and chain to parameters
    int rc = 0;
    for_each_scene(pos, nv, [&](int v, const int* pending, int np) {
        const isogs_scene& sc = scenes[v];
        const isogs_scene& gs = grads[v];
        for (int b0 = 0; b0 < np && !rc; b0 += kMaxViews) {
            GradPack gp{};
            gp.nv = min(kMaxViews, np - b0);
            gp.accumulate = b0 > 0;
            gp.pos = sc.pos;
            gp.scale = sc.scale;
            gp.opacity = sc.opacity;
            gp.color = sc.color;
            gp.n = (uint32_t)sc.n;
            gp.sh_degree = sc.sh_degree;
            gp.g_pos = const_cast<float*>(gs.pos);
            gp.g_scale = const_cast<float*>(gs.scale);
            gp.g_opacity = const_cast<float*>(gs.opacity);
            gp.g_color = const_cast<float*>(gs.color);
            for (int j = 0; j < gp.nv; ++j) fill_grad_view(gp.v[j], cams[pending[b0 + j]], view_off[pending[b0 + j]]);
            if (sc.n > 0) {
                const dim3 grid((sc.n + 255) / 256);
                switch (sc.sh_degree) {
                    case 0: hipLaunchKernelGGL(grad_project_kernel<0>, grid, dim3(256), 0, stream, gp, rec, proj->tile_count, bins->offsets, bins->count, bins->status); break;
                    case 1: hipLaunchKernelGGL(grad_project_kernel<1>, grid, dim3(256), 0, stream, gp, rec, proj->tile_count, bins->offsets, bins->count, bins->status); break;
                    case 2: hipLaunchKernelGGL(grad_project_kernel<2>, grid, dim3(256), 0, stream, gp, rec, proj->tile_count, bins->offsets, bins->count, bins->status); break;
                    default: hipLaunchKernelGGL(grad_project_kernel<3>, grid, dim3(256), 0, stream, gp, rec, proj->tile_count, bins->offsets, bins->count, bins->status); break;
                }
            }
            if (hipPeekAtLastError() != hipSuccess) rc = -1;
        }
    });
    return rc;
}

int launch_aniso_render_bwd(const isogs_aniso_scene* scenes, const isogs_camera* cams, int32_t nv,
                            const isogs_aniso_projected* proj, const isogs_bins* bins, const float* bg,
                            const float* image, const float* dL_dimage, const float* T_final,
                            const uint32_t* n_last, const float* ckpt, const isogs_aniso_scene* grads, void* ws,
                            hipStream_t stream) {
    if (nv > 4096) return -1;
    int32_t n_all[4096];
    uint32_t view_off[4096];
    const float* pos[4096];
    uint32_t o = 0;
    for (int v = 0; v < nv; ++v) {
        n_all[v] = scenes[v].n;
        view_off[v] = o;
        o += (uint32_t)scenes[v].n;
        pos[v] = scenes[v].pos;
    }
    const float4* rec = launch_composite_bwd(true, n_all, cams, nv, &proj->fp, proj->conic, bins, bg, image, dL_dimage,
                                             T_final, n_last, ckpt, ws, stream);
    if (!rec) return -1;
    int rc = 0;
    for_each_scene(pos, nv, [&](int v, const int* pending, int np) {
        const isogs_aniso_scene& sc = scenes[v];
        const isogs_aniso_scene& gs = grads[v];
        for (int b0 = 0; b0 < np && !rc; b0 += kMaxViews) {
            AnisoGradPack gp{};
            gp.nv = min(kMaxViews, np - b0);
            gp.accumulate = b0 > 0;
            gp.pos = sc.pos;
            gp.rot = sc.rot;
            gp.scale = sc.scale;
            gp.opacity = sc.opacity;
            gp.color = sc.color;
            gp.n = (uint32_t)sc.n;
            gp.sh_degree = sc.sh_degree;
            gp.g_pos = const_cast<float*>(gs.pos);
            gp.g_rot = const_cast<float*>(gs.rot);
            gp.g_scale = const_cast<float*>(gs.scale);
            gp.g_opacity = const_cast<float*>(gs.opacity);
            gp.g_color = const_cast<float*>(gs.color);
            for (int j = 0; j < gp.nv; ++j) fill_grad_view(gp.v[j], cams[pending[b0 + j]], view_off[pending[b0 + j]]);
            if (sc.n > 0) {
                const dim3 grid((sc.n + 255) / 256);
                const float4* r = reinterpret_cast<const float4*>(proj->fp.record);
                const float2* k = reinterpret_cast<const float2*>(proj->conic);
                const uint32_t* tc = proj->fp.tile_count;
                switch (sc.sh_degree) {
                    case 0: hipLaunchKernelGGL(aniso_grad_project_kernel<0>, grid, dim3(256), 0, stream, gp, rec, r, k, tc, bins->offsets, bins->count, bins->status); break;
                    case 1: hipLaunchKernelGGL(aniso_grad_project_kernel<1>, grid, dim3(256), 0, stream, gp, rec, r, k, tc, bins->offsets, bins->count, bins->status); break;
                    case 2: hipLaunchKernelGGL(aniso_grad_project_kernel<2>, grid, dim3(256), 0, stream, gp, rec, r, k, tc, bins->offsets, bins->count, bins->status); break;
                    default: hipLaunchKernelGGL(aniso_grad_project_kernel<3>, grid, dim3(256), 0, stream, gp, rec, r, k, tc, bins->offsets, bins->count, bins->status); break;
                }
            }
            if (hipPeekAtLastError() != hipSuccess) rc = -1;
        }
    });
    return rc;
}

}  // namespace isogs
