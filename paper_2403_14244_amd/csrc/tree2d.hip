// Quadtree initialisation and multiscale edits of 2D particles (the paper's Section 3,
// "Initial with Tree Structure", and Section 2, "Multiscale").
//
// Quadtree: the tree's levels are complete cell grids (level l: square cells of side
// root >> l, clipped at the image borders), so every cell's colour statistics come from
// one pyramid: the finest level sums its pixels, each coarser cell sums its (up to four)
// children, in FP64. The tree is then decided top-down, one launch per level, all on the
// device: a cell is active if it is a root cell or its parent split; an active cell may
// split when its colour variance exceeds tau and its quadrants are at least min_side
// wide; a one-workgroup budget step refuses the whole level's splits if they would let
// the leaf count exceed K. Leaves (active cells that do not split) are compacted level by
// level, row-major within a level, into particles: centre of the in-image rectangle,
// sigma = side / 2, amplitude = mean colour.
//
// Prune and split: every particle maps to 0, 1 or 4 outputs; a block count, a one-
// workgroup scan and a scatter keep the input order.
#include "common.h"
#include "kernels.h"

#include <algorithm>

namespace isogs {

namespace {

constexpr int kTreeThreads = 256;

struct LevelGeom {
    int side, gx, gy;
    uint32_t first;   // index of the level's first cell in the concatenated levels
};

struct TreeGeom {
    int n_levels;
    LevelGeom lv[32];
    uint32_t n_cells;
};

TreeGeom tree_geom(int32_t width, int32_t height, int32_t root, int32_t min_side) {
    TreeGeom g{};
    uint32_t first = 0;
    for (int side = root; side >= min_side && g.n_levels < 32; side >>= 1) {
        LevelGeom& L = g.lv[g.n_levels++];
        L.side = side;
        L.gx = (width + side - 1) / side;
        L.gy = (height + side - 1) / side;
        L.first = first;
        first += (uint32_t)(L.gx * L.gy);
        if (side == 1) break;
    }
    g.n_cells = first;
    return g;
}

// Per cell: S1[3], S2[3] (sums of colour and squared colour) and the pixel count.
struct CellSums {
    double s1[3], s2[3], n;
};

__global__ void __launch_bounds__(kTreeThreads) tree_finest_kernel(const float* __restrict__ target, int width,
                                                                   int height, LevelGeom L,
                                                                   CellSums* __restrict__ sums) {
    const uint32_t c = blockIdx.x * kTreeThreads + threadIdx.x;
    if (c >= (uint32_t)(L.gx * L.gy)) return;
    const int x0 = (int)(c % (uint32_t)L.gx) * L.side, y0 = (int)(c / (uint32_t)L.gx) * L.side;
    const int x1 = min(x0 + L.side, width), y1 = min(y0 + L.side, height);
    const size_t plane = (size_t)width * height;
    CellSums s{};
    for (int y = y0; y < y1; ++y)
        for (int x = x0; x < x1; ++x)
            for (int ch = 0; ch < 3; ++ch) {
                const double v = (double)target[ch * plane + (size_t)y * width + x];
                s.s1[ch] += v;
                s.s2[ch] += v * v;
            }
    s.n = (double)((x1 - x0) * (y1 - y0));
    sums[L.first + c] = s;
}

__global__ void __launch_bounds__(kTreeThreads) tree_up_kernel(LevelGeom C, LevelGeom F,
                                                               CellSums* __restrict__ sums) {
    const uint32_t c = blockIdx.x * kTreeThreads + threadIdx.x;
    if (c >= (uint32_t)(C.gx * C.gy)) return;
    const int i = (int)(c % (uint32_t)C.gx), j = (int)(c / (uint32_t)C.gx);
    CellSums s{};
    for (int dy = 0; dy < 2; ++dy)
        for (int dx = 0; dx < 2; ++dx) {
            const int fi = 2 * i + dx, fj = 2 * j + dy;
            if (fi >= F.gx || fj >= F.gy) continue;
            const CellSums& k = sums[F.first + (uint32_t)(fj * F.gx + fi)];
            for (int ch = 0; ch < 3; ++ch) {
                s.s1[ch] += k.s1[ch];
                s.s2[ch] += k.s2[ch];
            }
            s.n += k.n;
        }
    sums[C.first + c] = s;
}

__device__ __forceinline__ double cell_variance(const CellSums& s) {
    double v = 0.0;
    for (int ch = 0; ch < 3; ++ch) {
        const double m = s.s1[ch] / s.n;
        v += s.s2[ch] / s.n - m * m;
    }
    return v / 3.0;
}

// Per level: active / can-split flags and per-block counts {active, active and not
// splitting, in-image quadrants of the splitting ones}.
__global__ void __launch_bounds__(kTreeThreads) tree_decide_kernel(int l, LevelGeom L, LevelGeom P, LevelGeom N,
                                                                   int has_next, double tau, int min_side,
                                                                   const CellSums* __restrict__ sums,
                                                                   uint8_t* __restrict__ active,
                                                                   uint8_t* __restrict__ can,
                                                                   const int32_t* __restrict__ stop,
                                                                   uint32_t* __restrict__ block_counts) {
    __shared__ uint32_t s_cnt[3][kTreeThreads / kWave];
    const uint32_t c = blockIdx.x * kTreeThreads + threadIdx.x;
    uint32_t a = 0, leaf = 0, kids = 0;
    if (c < (uint32_t)(L.gx * L.gy)) {
        const int i = (int)(c % (uint32_t)L.gx), j = (int)(c / (uint32_t)L.gx);
        bool act = true;
        if (l > 0) {
            const uint32_t p = P.first + (uint32_t)((j / 2) * P.gx + i / 2);
            act = active[p] && can[p] && !stop[l - 1];
        }
        bool cs = false;
        if (act && has_next && L.side / 2 >= min_side) cs = cell_variance(sums[L.first + c]) > tau;
        active[L.first + c] = act;
        can[L.first + c] = cs;
        a = act;
        leaf = act && !cs;
        if (cs)
            for (int dy = 0; dy < 2; ++dy)
                for (int dx = 0; dx < 2; ++dx) kids += (2 * i + dx < N.gx && 2 * j + dy < N.gy) ? 1u : 0u;
    }
    const uint32_t w = threadIdx.x >> 6;
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        a += __shfl_xor(a, o, kWave);
        leaf += __shfl_xor(leaf, o, kWave);
        kids += __shfl_xor(kids, o, kWave);
    }
    if ((threadIdx.x & 63u) == 0) {
        s_cnt[0][w] = a;
        s_cnt[1][w] = leaf;
        s_cnt[2][w] = kids;
    }
    __syncthreads();
    if (threadIdx.x < 3) {
        uint32_t t = 0;
        for (int q = 0; q < kTreeThreads / kWave; ++q) t += s_cnt[threadIdx.x][q];
        block_counts[3 * blockIdx.x + threadIdx.x] = t;
    }
}

// One workgroup: totals of the level and the budget rule. state[0] = leaves so far.
__global__ void __launch_bounds__(kTreeThreads) tree_budget_kernel(int l, uint32_t n_blocks,
                                                                   const uint32_t* __restrict__ block_counts,
                                                                   uint32_t K, int32_t* __restrict__ stop,
                                                                   uint32_t* __restrict__ state) {
    __shared__ uint64_t s_t[3][kTreeThreads];
    uint64_t t[3] = {0, 0, 0};
    for (uint32_t b = threadIdx.x; b < n_blocks; b += kTreeThreads)
        for (int q = 0; q < 3; ++q) t[q] += block_counts[3 * b + q];
    for (int q = 0; q < 3; ++q) s_t[q][threadIdx.x] = t[q];
    __syncthreads();
    if (threadIdx.x == 0) {
        uint64_t a = 0, leaf = 0, kids = 0;
        for (int i = 0; i < kTreeThreads; ++i) {
            a += s_t[0][i];
            leaf += s_t[1][i];
            kids += s_t[2][i];
        }
        const uint64_t done = state[0];
        const bool refuse = done + leaf + kids > (uint64_t)K;
        stop[l] = refuse ? 1 : 0;
        state[0] = (uint32_t)(done + (refuse ? a : leaf));
    }
}

__global__ void tree_reset_kernel(uint32_t* __restrict__ state) {
    if (threadIdx.x == 0) state[0] = 0u;
}

// Leaf flag of a cell of the concatenated levels.
__device__ __forceinline__ bool tree_leaf(uint32_t g, const TreeGeom& T, const uint8_t* active, const uint8_t* can,
                                          const int32_t* stop, int& level) {
    int l = 0;
    for (int q = 1; q < T.n_levels; ++q) l = (g >= T.lv[q].first) ? q : l;
    level = l;
    return active[g] && !(can[g] && !stop[l]);
}

__global__ void __launch_bounds__(kTreeThreads) tree_leaf_count_kernel(TreeGeom T, const uint8_t* __restrict__ active,
                                                                       const uint8_t* __restrict__ can,
                                                                       const int32_t* __restrict__ stop,
                                                                       uint32_t* __restrict__ block_sums) {
    __shared__ uint32_t s_w[kTreeThreads / kWave];
    const uint32_t g = blockIdx.x * kTreeThreads + threadIdx.x;
    int l;
    uint32_t m = (g < T.n_cells && tree_leaf(g, T, active, can, stop, l)) ? 1u : 0u;
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) m += __shfl_xor(m, o, kWave);
    if ((threadIdx.x & 63u) == 0) s_w[threadIdx.x >> 6] = m;
    __syncthreads();
    if (threadIdx.x == 0) block_sums[blockIdx.x] = s_w[0] + s_w[1] + s_w[2] + s_w[3];
}

// Exclusive scan of n block sums in place by one workgroup (chunks of 256, in order);
// the total goes to *total.
__global__ void __launch_bounds__(kTreeThreads) tree_scan_kernel(uint32_t* __restrict__ sums, uint32_t n,
                                                                 int32_t* __restrict__ total) {
    __shared__ uint32_t s_w[kTreeThreads / kWave];
    __shared__ uint32_t s_carry;
    if (threadIdx.x == 0) s_carry = 0;
    __syncthreads();
    const uint32_t lane = threadIdx.x & 63u, w = threadIdx.x >> 6;
    for (uint32_t c0 = 0; c0 < n; c0 += kTreeThreads) {
        const uint32_t i = c0 + threadIdx.x;
        const uint32_t x = i < n ? sums[i] : 0u;
        uint32_t incl = x;
#pragma unroll
        for (uint32_t o = 1; o < 64; o <<= 1) {
            const uint32_t y = __shfl_up(incl, o, kWave);
            if (lane >= o) incl += y;
        }
        if (lane == 63) s_w[w] = incl;
        __syncthreads();
        uint32_t before = s_carry;
        for (uint32_t q = 0; q < w; ++q) before += s_w[q];
        if (i < n) sums[i] = before + incl - x;
        __syncthreads();
        if (threadIdx.x == kTreeThreads - 1) s_carry = before + incl;
        __syncthreads();
    }
    if (threadIdx.x == 0) *total = (int32_t)s_carry;
}

__global__ void __launch_bounds__(kTreeThreads) tree_emit_kernel(TreeGeom T, int width, int height,
                                                                 const CellSums* __restrict__ sums,
                                                                 const uint8_t* __restrict__ active,
                                                                 const uint8_t* __restrict__ can,
                                                                 const int32_t* __restrict__ stop,
                                                                 const uint32_t* __restrict__ block_offsets,
                                                                 uint32_t cap, float* __restrict__ mu,
                                                                 float* __restrict__ sigma, float* __restrict__ amp) {
    __shared__ uint32_t s_w[kTreeThreads / kWave];
    const uint32_t g = blockIdx.x * kTreeThreads + threadIdx.x;
    int l = 0;
    const bool leaf = g < T.n_cells && tree_leaf(g, T, active, can, stop, l);
    const uint64_t m = ballot64(leaf);
    const uint32_t w = threadIdx.x >> 6;
    if ((threadIdx.x & 63u) == 0) s_w[w] = (uint32_t)__popcll(m);
    __syncthreads();
    if (!leaf) return;
    uint32_t pos = block_offsets[blockIdx.x] + rank_below(m);
    for (uint32_t q = 0; q < w; ++q) pos += s_w[q];
    if (pos >= cap) return;
    const LevelGeom& L = T.lv[l];
    const uint32_t c = g - L.first;
    const int x0 = (int)(c % (uint32_t)L.gx) * L.side, y0 = (int)(c / (uint32_t)L.gx) * L.side;
    const int x1 = min(x0 + L.side, width), y1 = min(y0 + L.side, height);
    const CellSums& s = sums[g];
    mu[pos] = 0.5f * (float)(x0 + x1);
    mu[cap + pos] = 0.5f * (float)(y0 + y1);
    sigma[pos] = 0.5f * (float)L.side;
    for (int ch = 0; ch < 3; ++ch) amp[(size_t)ch * cap + pos] = (float)(s.s1[ch] / s.n);
}

// ---- prune and split ----------------------------------------------------------------

__device__ __forceinline__ uint32_t edit_outputs(int mode, float thr, const float* mu, const float* sigma,
                                                 const float* amp, uint32_t K, uint32_t k) {
    const float mx = mu[k], my = mu[K + k], s = sigma[k];
    const float a0 = amp[k], a1 = amp[K + k], a2 = amp[2 * (size_t)K + k];
    if (mode == 0) {   // prune
        const bool ok = isfinite(mx) && isfinite(my) && isfinite(s) && s > 0.0f && isfinite(a0) && isfinite(a1) &&
                        isfinite(a2);
        return (ok && fmaxf(fmaxf(fabsf(a0), fabsf(a1)), fabsf(a2)) >= thr) ? 1u : 0u;
    }
    return s > thr ? 4u : 1u;   // split
}

__global__ void __launch_bounds__(kTreeThreads) edit_count_kernel(int mode, float thr, const float* __restrict__ mu,
                                                                  const float* __restrict__ sigma,
                                                                  const float* __restrict__ amp, uint32_t K,
                                                                  uint32_t* __restrict__ block_sums) {
    __shared__ uint32_t s_w[kTreeThreads / kWave];
    const uint32_t k = blockIdx.x * kTreeThreads + threadIdx.x;
    uint32_t m = k < K ? edit_outputs(mode, thr, mu, sigma, amp, K, k) : 0u;
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) m += __shfl_xor(m, o, kWave);
    if ((threadIdx.x & 63u) == 0) s_w[threadIdx.x >> 6] = m;
    __syncthreads();
    if (threadIdx.x == 0) block_sums[blockIdx.x] = s_w[0] + s_w[1] + s_w[2] + s_w[3];
}

__global__ void __launch_bounds__(kTreeThreads) edit_scatter_kernel(
    int mode, float thr, const float* __restrict__ mu, const float* __restrict__ sigma, const float* __restrict__ amp,
    uint32_t K, const uint32_t* __restrict__ block_offsets, uint32_t cap, float* __restrict__ omu,
    float* __restrict__ osigma, float* __restrict__ oamp) {
    __shared__ uint32_t s_w[kTreeThreads / kWave];
    const uint32_t k = blockIdx.x * kTreeThreads + threadIdx.x;
    const uint32_t m = k < K ? edit_outputs(mode, thr, mu, sigma, amp, K, k) : 0u;
    uint32_t incl = m;
    const uint32_t lane = threadIdx.x & 63u, w = threadIdx.x >> 6;
#pragma unroll
    for (uint32_t o = 1; o < 64; o <<= 1) {
        const uint32_t y = __shfl_up(incl, o, kWave);
        if (lane >= o) incl += y;
    }
    if (lane == 63) s_w[w] = incl;
    __syncthreads();
    if (!m) return;
    uint32_t pos = block_offsets[blockIdx.x] + incl - m;
    for (uint32_t q = 0; q < w; ++q) pos += s_w[q];
    const float mx = mu[k], my = mu[K + k], s = sigma[k];
    const float a0 = amp[k], a1 = amp[K + k], a2 = amp[2 * (size_t)K + k];
    for (uint32_t j = 0; j < m; ++j) {
        const uint32_t o = pos + j;
        if (o >= cap) return;
        float ox = mx, oy = my, os = s;
        if (m == 4) {
            const float h = s * 0.5f;
            ox = (j & 1u) ? mx + h : mx - h;
            oy = (j & 2u) ? my + h : my - h;
            os = h;
        }
        omu[o] = ox;
        omu[cap + o] = oy;
        osigma[o] = os;
        oamp[o] = a0;
        oamp[cap + o] = a1;
        oamp[2 * (size_t)cap + o] = a2;
    }
}

struct TreeWs {
    size_t off_sums, off_active, off_can, off_stop, off_state, off_blocks, bytes;
};

size_t a256(size_t x) { return (x + 255) & ~(size_t)255; }

TreeWs tree_layout(const TreeGeom& T) {
    TreeWs w{};
    size_t max_level = 0;
    for (int l = 0; l < T.n_levels; ++l) max_level = std::max(max_level, (size_t)T.lv[l].gx * T.lv[l].gy);
    const size_t blocks = std::max((T.n_cells + kTreeThreads - 1) / kTreeThreads,
                                   (uint32_t)((max_level + kTreeThreads - 1) / kTreeThreads));
    w.off_sums = 0;
    w.off_active = a256((size_t)T.n_cells * sizeof(CellSums));
    w.off_can = w.off_active + a256(T.n_cells);
    w.off_stop = w.off_can + a256(T.n_cells);
    w.off_state = w.off_stop + 256;
    w.off_blocks = w.off_state + 256;
    w.bytes = w.off_blocks + a256(blocks * 3 * 4);
    return w;
}

}  // namespace

int tree_levels_ok(int32_t width, int32_t height, int32_t root, int32_t min_side, uint64_t* root_cells) {
    if (root < 1 || (root & (root - 1)) || min_side < 1 || min_side > root) return 0;
    const TreeGeom T = tree_geom(width, height, root, min_side);
    *root_cells = (uint64_t)T.lv[0].gx * T.lv[0].gy;
    return T.n_cells < (1u << 30) ? 1 : 0;
}

size_t tree_init_ws(int32_t width, int32_t height, int32_t root, int32_t min_side) {
    return tree_layout(tree_geom(width, height, root, min_side)).bytes;
}

int launch_tree_init(const float* target, int32_t width, int32_t height, int32_t root, int32_t min_side, float tau,
                     int32_t K, const isogs_field2d* out, int32_t* count, void* ws, hipStream_t stream) {
    const TreeGeom T = tree_geom(width, height, root, min_side);
    const TreeWs W = tree_layout(T);
    char* base = static_cast<char*>(ws);
    CellSums* sums = reinterpret_cast<CellSums*>(base + W.off_sums);
    uint8_t* active = reinterpret_cast<uint8_t*>(base + W.off_active);
    uint8_t* can = reinterpret_cast<uint8_t*>(base + W.off_can);
    int32_t* stop = reinterpret_cast<int32_t*>(base + W.off_stop);
    uint32_t* state = reinterpret_cast<uint32_t*>(base + W.off_state);
    uint32_t* blocks = reinterpret_cast<uint32_t*>(base + W.off_blocks);
    auto grid = [](uint32_t n) { return dim3((n + kTreeThreads - 1) / kTreeThreads); };
    // pyramid, finest level first
    const LevelGeom& F = T.lv[T.n_levels - 1];
    hipLaunchKernelGGL(tree_finest_kernel, grid((uint32_t)(F.gx * F.gy)), dim3(kTreeThreads), 0, stream, target, width,
                       height, F, sums);
    for (int l = T.n_levels - 2; l >= 0; --l)
        hipLaunchKernelGGL(tree_up_kernel, grid((uint32_t)(T.lv[l].gx * T.lv[l].gy)), dim3(kTreeThreads), 0, stream,
                           T.lv[l], T.lv[l + 1], sums);
    // top-down decisions
    hipLaunchKernelGGL(tree_reset_kernel, dim3(1), dim3(64), 0, stream, state);
    for (int l = 0; l < T.n_levels; ++l) {
        const LevelGeom& L = T.lv[l];
        const LevelGeom P = l > 0 ? T.lv[l - 1] : L;
        const int has_next = l + 1 < T.n_levels;
        const LevelGeom N = has_next ? T.lv[l + 1] : L;
        const uint32_t nb = ((uint32_t)(L.gx * L.gy) + kTreeThreads - 1) / kTreeThreads;
        hipLaunchKernelGGL(tree_decide_kernel, dim3(nb), dim3(kTreeThreads), 0, stream, l, L, P, N, has_next,
                           (double)tau, min_side, sums, active, can, stop, blocks);
        hipLaunchKernelGGL(tree_budget_kernel, dim3(1), dim3(kTreeThreads), 0, stream, l, nb, blocks, (uint32_t)K,
                           stop, state);
    }
    // leaves, level by level, row-major
    const uint32_t nb = (T.n_cells + kTreeThreads - 1) / kTreeThreads;
    hipLaunchKernelGGL(tree_leaf_count_kernel, dim3(nb), dim3(kTreeThreads), 0, stream, T, active, can, stop, blocks);
    hipLaunchKernelGGL(tree_scan_kernel, dim3(1), dim3(kTreeThreads), 0, stream, blocks, nb, count);
    hipLaunchKernelGGL(tree_emit_kernel, dim3(nb), dim3(kTreeThreads), 0, stream, T, width, height, sums, active, can,
                       stop, blocks, (uint32_t)K, out->mu, out->sigma, out->amp);
    return hipPeekAtLastError() == hipSuccess ? 0 : -1;
}

size_t edit_ws(int32_t K) { return a256((size_t)((K + kTreeThreads - 1) / kTreeThreads + 1) * 4); }

int launch_edit(int mode, float thr, const isogs_field2d* in, const isogs_field2d* out, int32_t cap, int32_t* count,
                void* ws, hipStream_t stream) {
    const uint32_t K = (uint32_t)in->K;
    const uint32_t nb = (K + kTreeThreads - 1) / kTreeThreads;
    uint32_t* blocks = static_cast<uint32_t*>(ws);
    if (nb)
        hipLaunchKernelGGL(edit_count_kernel, dim3(nb), dim3(kTreeThreads), 0, stream, mode, thr, in->mu, in->sigma,
                           in->amp, K, blocks);
    hipLaunchKernelGGL(tree_scan_kernel, dim3(1), dim3(kTreeThreads), 0, stream, blocks, nb, count);
    if (nb)
        hipLaunchKernelGGL(edit_scatter_kernel, dim3(nb), dim3(kTreeThreads), 0, stream, mode, thr, in->mu, in->sigma,
                           in->amp, K, blocks, (uint32_t)cap, out->mu, out->sigma, out->amp);
    return hipPeekAtLastError() == hipSuccess ? 0 : -1;
}

}  // namespace isogs
