// Device-side definitions shared by the isotropic-splatting kernels (gfx950, wave64).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace isogs {

constexpr int kTile = 16;                  // tile edge in pixels
constexpr int kTilePixels = kTile * kTile; // one workgroup per tile, one lane per pixel
constexpr int kWave = 64;
constexpr float kAlphaMin = 1.0f / 255.0f; // support of a particle: alpha >= 1/255 (eq. 2)
constexpr float kAlphaMax = 0.99f;         // alpha clamp: 1 - alpha >= 0.01
constexpr float kTMin = 1e-4f;             // a pixel stops after T falls below this
constexpr float kLog2e = 1.4426950408889634f;
constexpr int kMaxViews = 16;              // views per launch (kernel-argument pack)

// Error words written to the device status of a bin set.
constexpr int32_t kStatusOk = 0;
constexpr int32_t kStatusCapacity = -2;
constexpr int32_t kStatusDevice = -4;

// Per-view constants, passed by value in kernel arguments.
struct ViewDesc {
    uint32_t p_off;      // first packed particle of the view
    uint32_t n;          // particles of the view
    uint32_t tile_base;  // first global tile id of the view
    uint32_t pix_off;    // first pixel of the view (H*W units)
    int32_t width, height, tiles_x, tiles_y;
};

struct ViewPack {
    int32_t nv;
    uint32_t block_begin[kMaxViews + 1];  // first block of each view in this launch
    ViewDesc v[kMaxViews];
};

// View of a block in a launch whose blocks are grouped by view (uniform per block).
__device__ __forceinline__ int view_of_block(const ViewPack& pk, uint32_t b) {
    int v = 0;
    for (int i = 1; i < pk.nv; ++i) v = (b >= pk.block_begin[i]) ? i : v;
    return __builtin_amdgcn_readfirstlane(v);
}

// Blocks are dispatched round-robin over the 8 XCDs (block b runs on XCD b mod 8). This
// bijection gives each XCD a contiguous range of logical work items, so neighbouring
// tiles, which share particles, are served from the same L2.
__device__ __forceinline__ uint32_t xcd_swizzle(uint32_t b, uint32_t nb) {
    const uint32_t q = nb >> 3, r = nb & 7u, x = b & 7u, i = b >> 3;
    return (x < r) ? x * (q + 1u) + i : r * (q + 1u) + (x - r) * q + i;
}

// Exact FP32 disk-versus-tile test. Evaluated one rounded operation at a time (this
// library is compiled with -ffp-contract=off), so the decision is bit-reproducible by any
// IEEE FP32 implementation of the same expression:
//   dx = max(max(x_lo - u, u - x_hi), 0), dy likewise, member iff dx*dx + dy*dy <= r2,
// where [x_lo, x_hi] spans the tile's pixel centres and r2 = radius * radius.
__device__ __forceinline__ bool tile_member(float u, float v, float r2, int tx, int ty, float w_lim,
                                            float h_lim) {
    const float x0 = (float)(tx * kTile), y0 = (float)(ty * kTile);
    const float x_lo = x0 + 0.5f, y_lo = y0 + 0.5f;
    const float x_hi = fminf(x0 + 15.5f, w_lim), y_hi = fminf(y0 + 15.5f, h_lim);
    const float dx = fmaxf(fmaxf(x_lo - u, u - x_hi), 0.0f);
    const float dy = fmaxf(fmaxf(y_lo - v, v - y_hi), 0.0f);
    const float d2 = dx * dx + dy * dy;
    return d2 <= r2;
}

// Candidate tile box of a footprint: every tile that can pass tile_member lies inside.
// A tile left of u needs 16 tx + 15.5 >= u - r, one right of u needs 16 tx + 0.5 <= u + r;
// the extra half pixel absorbs FP32 rounding of the test: a tile below the lower bound has
// its last pixel centre more than r + 0.5 from u, far outside any rounding of tile_member.
__device__ __forceinline__ void tile_box(float u, float v, float r, int tiles_x, int tiles_y, int& tx0,
                                         int& tx1, int& ty0, int& ty1) {
    tx0 = max(0, (int)ceilf((u - r - 16.0f) * (1.0f / kTile)));
    ty0 = max(0, (int)ceilf((v - r - 16.0f) * (1.0f / kTile)));
    tx1 = min(tiles_x - 1, (int)floorf((u + r) * (1.0f / kTile)));
    ty1 = min(tiles_y - 1, (int)floorf((v + r) * (1.0f / kTile)));
}

// alpha of an entry at a pixel: min(0.99, o exp(-d^2 / s^2)), evaluated as
// exp2(log2(o) - d^2 log2(e)/s^2) with lo = log2(o) and q = log2(e)/s^2. `g` returns the
// value before the clamp (o times the kernel). The forward and backward kernels call this
// one function, so they take identical threshold decisions.
__device__ __forceinline__ float entry_alpha(float dx, float dy, float q, float lo, float& g) {
    const float d2 = fmaf(dx, dx, dy * dy);
    g = __builtin_amdgcn_exp2f(fmaf(-d2, q, lo));
    return fminf(kAlphaMax, g);
}

template <int CTRL>
__device__ __forceinline__ float dpp(float x) {
    return __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, x), CTRL, 0xF, 0xF, false));
}

// Sums eight per-lane values over each 16-lane row of a wave with a transposing
// butterfly: each exchange step halves the values a lane carries (two quad swaps, then
// row rotations by 4 and by 8). Afterwards lanes l and l + 8 of a row both hold the row
// total of value rev3(l), where rev3 reverses the three low bits of l < 8. About twenty
// instructions for all eight sums; the combination order is fixed, so results are
// bitwise reproducible.
__device__ __forceinline__ float row_sum8(const float v[8], uint32_t lane) {
    const bool p = lane & 1u, q = lane & 2u, b = lane & 4u;
    float a[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) a[k] = (p ? v[k + 4] : v[k]) + dpp<0xB1>(p ? v[k] : v[k + 4]);
    float c[2];
#pragma unroll
    for (int k = 0; k < 2; ++k) c[k] = (q ? a[k + 2] : a[k]) + dpp<0x4E>(q ? a[k] : a[k + 2]);
    float d = (b ? c[1] : c[0]) + dpp<0x124>(b ? c[0] : c[1]);   // row_ror:4
    d += dpp<0x128>(d);                                             // row_ror:8
    return d;
}

__device__ __forceinline__ uint32_t rev3(uint32_t l) { return ((l & 1u) << 2) | (l & 2u) | ((l >> 2) & 1u); }

__device__ __forceinline__ uint64_t ballot64(bool p) { return __ballot(p); }

__device__ __forceinline__ uint32_t lane_id() { return __lane_id(); }

// Number of set bits of m in lanes below this one.
__device__ __forceinline__ uint32_t rank_below(uint64_t m) {
    return __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
}

}  // namespace isogs
