// Tree initialisation and multiscale edits (the paper's Section 3, "Initial with Tree
// Structure", and Section 2, "Multiscale"): the quadtree of 2D particles over an image,
// the octree of 3D particles over a coloured point cloud, and the prune, split and merge
// of 2D particles.
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
#include <cmath>

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

namespace {

// ---- octree initialisation of 3D particles ----------------------------------------------
// The tree over a coloured point cloud: levels are complete cell grids over the root grid
// (level l: cubic cells of edge root_side / 2^l). Colour statistics are exact integers (each
// channel clamped to [0, 1] and quantised to rint(65535 c)), so the finest cells gather their
// points with 64-bit integer atomics in any order and the variance computed from them in
// FP64 is the same whatever that order; coarser cells add their eight children. Decisions
// top-down as for the quadtree, empty cells carrying nothing; leaves become isotropic
// particles (cell centre, scale = edge / 2, the given opacity, mean colour as the
// degree-0 coefficient).

struct OctLevel {
    int gx, gy, gz;
    uint32_t first;
    double edge;
};

struct OctGeom {
    int n_levels;
    OctLevel lv[16];
    uint32_t n_cells;
    double lo[3];
};

struct OctSums {
    unsigned long long n, s1[3], s2[3];
};

constexpr double kColorQ = 65535.0;

OctGeom oct_geom(const isogs_octree_grid& g) {
    OctGeom G{};
    G.n_levels = g.levels;
    uint64_t first = 0;
    for (int l = 0; l < g.levels && l < 16; ++l) {
        OctLevel& L = G.lv[l];
        L.gx = g.roots[0] << l;
        L.gy = g.roots[1] << l;
        L.gz = g.roots[2] << l;
        L.first = (uint32_t)first;
        L.edge = (double)g.root_side / (double)(1u << l);
        first += (uint64_t)L.gx * L.gy * L.gz;
    }
    G.n_cells = (uint32_t)(first < 0xFFFFFFFFull ? first : 0xFFFFFFFFull);
    for (int a = 0; a < 3; ++a) G.lo[a] = (double)g.lo[a];
    return G;
}

__global__ void __launch_bounds__(kTreeThreads) oct_clear_kernel(OctSums* __restrict__ sums, uint32_t n) {
    for (uint32_t c = blockIdx.x * kTreeThreads + threadIdx.x; c < n; c += gridDim.x * kTreeThreads)
        sums[c] = OctSums{};
}

__global__ void __launch_bounds__(kTreeThreads) oct_points_kernel(const float* __restrict__ pts,
                                                                  const float* __restrict__ col, uint32_t P,
                                                                  OctGeom G, OctSums* __restrict__ sums) {
    const uint32_t k = blockIdx.x * kTreeThreads + threadIdx.x;
    if (k >= P) return;
    const OctLevel& F = G.lv[G.n_levels - 1];
    const int dims[3] = {F.gx, F.gy, F.gz};
    int idx[3];
    for (int a = 0; a < 3; ++a) {
        const double q = floor(((double)pts[(size_t)a * P + k] - G.lo[a]) / F.edge);
        if (!(q >= 0.0 && q < (double)dims[a])) return;   // outside the grid, or not finite
        idx[a] = (int)q;
    }
    OctSums* c = sums + F.first + ((uint64_t)idx[2] * F.gy + idx[1]) * F.gx + idx[0];
    atomicAdd(&c->n, 1ull);
    for (int ch = 0; ch < 3; ++ch) {
        const double v = fmin(fmax((double)col[(size_t)ch * P + k], 0.0), 1.0);
        const unsigned long long q = (unsigned long long)rint(v * kColorQ);
        atomicAdd(&c->s1[ch], q);
        atomicAdd(&c->s2[ch], q * q);
    }
}

__global__ void __launch_bounds__(kTreeThreads) oct_up_kernel(OctLevel C, OctLevel F, OctSums* __restrict__ sums) {
    const uint32_t c = blockIdx.x * kTreeThreads + threadIdx.x;
    if (c >= (uint32_t)(C.gx * C.gy * C.gz)) return;
    const int i = (int)(c % (uint32_t)C.gx), j = (int)((c / (uint32_t)C.gx) % (uint32_t)C.gy);
    const int k = (int)(c / (uint32_t)(C.gx * C.gy));
    OctSums s{};
    for (int dz = 0; dz < 2; ++dz)
        for (int dy = 0; dy < 2; ++dy)
            for (int dx = 0; dx < 2; ++dx) {
                const OctSums& f =
                    sums[F.first + ((uint32_t)(2 * k + dz) * F.gy + (uint32_t)(2 * j + dy)) * F.gx + 2 * i + dx];
                s.n += f.n;
                for (int ch = 0; ch < 3; ++ch) {
                    s.s1[ch] += f.s1[ch];
                    s.s2[ch] += f.s2[ch];
                }
            }
    sums[C.first + c] = s;
}

// (1/3) sum_ch (S2/n - (S1/n)^2), FP64 from the exact integer sums (n > 0).
__device__ __forceinline__ double oct_variance(const OctSums& s) {
    const double n = (double)s.n;
    double v = 0.0;
    for (int ch = 0; ch < 3; ++ch) {
        const double m = (double)s.s1[ch] / n;
        v = v + ((double)s.s2[ch] / n - m * m);
    }
    return v / 3.0;
}

// Per level: active and split flags, per-block counts {active non-empty, leaves if the
// level splits, non-empty children of the splitting cells}.
__global__ void __launch_bounds__(kTreeThreads) oct_decide_kernel(int l, OctLevel L, OctLevel P, OctLevel N,
                                                                  int has_next, double thr,
                                                                  const OctSums* __restrict__ sums,
                                                                  uint8_t* __restrict__ active,
                                                                  uint8_t* __restrict__ can,
                                                                  const int32_t* __restrict__ stop,
                                                                  uint32_t* __restrict__ block_counts) {
    __shared__ uint32_t s_cnt[3][kTreeThreads / kWave];
    const uint32_t c = blockIdx.x * kTreeThreads + threadIdx.x;
    uint32_t a = 0, leaf = 0, kids = 0;
    if (c < (uint32_t)(L.gx * L.gy * L.gz)) {
        const int i = (int)(c % (uint32_t)L.gx), j = (int)((c / (uint32_t)L.gx) % (uint32_t)L.gy);
        const int k = (int)(c / (uint32_t)(L.gx * L.gy));
        bool act = true;
        if (l > 0) {
            const uint32_t p = P.first + ((uint32_t)(k / 2) * P.gy + (uint32_t)(j / 2)) * P.gx + i / 2;
            act = active[p] && can[p] && !stop[l - 1];
        }
        const OctSums& s = sums[L.first + c];
        const bool nonempty = s.n > 0;
        const bool cs = act && nonempty && has_next && oct_variance(s) > thr;
        active[L.first + c] = act;
        can[L.first + c] = cs;
        a = act && nonempty;
        leaf = act && nonempty && !cs;
        if (cs)
            for (int dz = 0; dz < 2; ++dz)
                for (int dy = 0; dy < 2; ++dy)
                    for (int dx = 0; dx < 2; ++dx)
                        kids += sums[N.first + ((uint32_t)(2 * k + dz) * N.gy + (uint32_t)(2 * j + dy)) * N.gx +
                                     2 * i + dx].n > 0 ? 1u : 0u;
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

__device__ __forceinline__ bool oct_leaf(uint32_t g, const OctGeom& G, const OctSums* sums, const uint8_t* active,
                                         const uint8_t* can, const int32_t* stop, int& level) {
    int l = 0;
    for (int q = 1; q < G.n_levels; ++q) l = (g >= G.lv[q].first) ? q : l;
    level = l;
    return active[g] && sums[g].n > 0 && !(can[g] && !stop[l]);
}

__global__ void __launch_bounds__(kTreeThreads) oct_leaf_count_kernel(OctGeom G, const OctSums* __restrict__ sums,
                                                                      const uint8_t* __restrict__ active,
                                                                      const uint8_t* __restrict__ can,
                                                                      const int32_t* __restrict__ stop,
                                                                      uint32_t* __restrict__ block_sums) {
    __shared__ uint32_t s_w[kTreeThreads / kWave];
    const uint32_t g = blockIdx.x * kTreeThreads + threadIdx.x;
    int l;
    uint32_t m = (g < G.n_cells && oct_leaf(g, G, sums, active, can, stop, l)) ? 1u : 0u;
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) m += __shfl_xor(m, o, kWave);
    if ((threadIdx.x & 63u) == 0) s_w[threadIdx.x >> 6] = m;
    __syncthreads();
    if (threadIdx.x == 0) block_sums[blockIdx.x] = s_w[0] + s_w[1] + s_w[2] + s_w[3];
}

__global__ void __launch_bounds__(kTreeThreads) oct_emit_kernel(OctGeom G, const OctSums* __restrict__ sums,
                                                                const uint8_t* __restrict__ active,
                                                                const uint8_t* __restrict__ can,
                                                                const int32_t* __restrict__ stop,
                                                                const uint32_t* __restrict__ block_offsets,
                                                                uint32_t K, uint32_t stride, int n_coef,
                                                                float opacity, float* __restrict__ pos,
                                                                float* __restrict__ scale, float* __restrict__ opa,
                                                                float* __restrict__ color) {
    __shared__ uint32_t s_w[kTreeThreads / kWave];
    const uint32_t g = blockIdx.x * kTreeThreads + threadIdx.x;
    int l = 0;
    const bool leaf = g < G.n_cells && oct_leaf(g, G, sums, active, can, stop, l);
    const uint64_t m = ballot64(leaf);
    const uint32_t w = threadIdx.x >> 6;
    if ((threadIdx.x & 63u) == 0) s_w[w] = (uint32_t)__popcll(m);
    __syncthreads();
    if (!leaf) return;
    uint32_t p = block_offsets[blockIdx.x] + rank_below(m);
    for (uint32_t q = 0; q < w; ++q) p += s_w[q];
    if (p >= K) return;
    const OctLevel& L = G.lv[l];
    const uint32_t c = g - L.first;
    const int i = (int)(c % (uint32_t)L.gx), j = (int)((c / (uint32_t)L.gx) % (uint32_t)L.gy);
    const int k = (int)(c / (uint32_t)(L.gx * L.gy));
    const int ijk[3] = {i, j, k};
    for (int a = 0; a < 3; ++a) pos[(size_t)a * stride + p] = (float)(G.lo[a] + ((double)ijk[a] + 0.5) * L.edge);
    scale[p] = (float)(0.5 * L.edge);
    opa[p] = opacity;
    const OctSums& s = sums[g];
    for (int ch = 0; ch < 3; ++ch) color[(size_t)ch * stride + p] = (float)((double)s.s1[ch] / (double)s.n / kColorQ);
    for (int q = 3; q < 3 * n_coef; ++q) color[(size_t)q * stride + p] = 0.0f;
}

struct OctWs {
    size_t off_sums, off_active, off_can, off_stop, off_state, off_blocks, bytes;
};

OctWs oct_layout(const OctGeom& G) {
    OctWs w{};
    size_t max_level = 0;
    for (int l = 0; l < G.n_levels; ++l) max_level = std::max(max_level, (size_t)G.lv[l].gx * G.lv[l].gy * G.lv[l].gz);
    const size_t blocks = std::max((size_t)(G.n_cells + kTreeThreads - 1) / kTreeThreads,
                                   (max_level + kTreeThreads - 1) / kTreeThreads);
    w.off_sums = 0;
    w.off_active = a256((size_t)G.n_cells * sizeof(OctSums));
    w.off_can = w.off_active + a256(G.n_cells);
    w.off_stop = w.off_can + a256(G.n_cells);
    w.off_state = w.off_stop + 256;
    w.off_blocks = w.off_state + 256;
    w.bytes = w.off_blocks + a256(blocks * 3 * 4);
    return w;
}

// ---- merge of 2D particles ------------------------------------------------------------
// Particles with sigma <= sigma_max (finite, sigma > 0, centre in the image) are grouped by
// the cell of edge `cell` holding their centre; every group of two or more becomes one
// particle keeping the kernels' mass per channel (sigma_m^2 = sum sigma^2, centre and
// amplitude the sigma^2-weighted means), at the position of the group's first member.
// The group sums are FP64 atomics (the order of at most a few terms changes only their
// last FP64 bits); membership and output order are integer work.
struct MergeCell {
    uint32_t count, leader;
    double w, wx, wy, wa[3];
};

__global__ void __launch_bounds__(kTreeThreads) merge_clear_kernel(MergeCell* __restrict__ cells, uint32_t n) {
    for (uint32_t c = blockIdx.x * kTreeThreads + threadIdx.x; c < n; c += gridDim.x * kTreeThreads)
        cells[c] = MergeCell{0u, 0xFFFFFFFFu, 0.0, 0.0, 0.0, {0.0, 0.0, 0.0}};
}

// Cell of particle k, or -1 when it does not take part.
__device__ __forceinline__ int64_t merge_cell(const float* mu, const float* sigma, const float* amp, uint32_t K,
                                              uint32_t k, int width, int height, double cell, int gx,
                                              float sigma_max) {
    const float mx = mu[k], my = mu[K + k], s = sigma[k];
    const float a0 = amp[k], a1 = amp[K + k], a2 = amp[2 * (size_t)K + k];
    if (!(isfinite(mx) && isfinite(my) && isfinite(s) && isfinite(a0) && isfinite(a1) && isfinite(a2))) return -1;
    if (!(s > 0.0f && s <= sigma_max)) return -1;
    const double x = (double)mx, y = (double)my;
    if (!(x >= 0.0 && x < (double)width && y >= 0.0 && y < (double)height)) return -1;
    return (int64_t)floor(y / cell) * gx + (int64_t)floor(x / cell);
}

__global__ void __launch_bounds__(kTreeThreads) merge_accum_kernel(const float* __restrict__ mu,
                                                                   const float* __restrict__ sigma,
                                                                   const float* __restrict__ amp, uint32_t K,
                                                                   int width, int height, double cell, int gx,
                                                                   float sigma_max, MergeCell* __restrict__ cells) {
    const uint32_t k = blockIdx.x * kTreeThreads + threadIdx.x;
    if (k >= K) return;
    const int64_t c = merge_cell(mu, sigma, amp, K, k, width, height, cell, gx, sigma_max);
    if (c < 0) return;
    MergeCell* m = cells + c;
    const double s = (double)sigma[k], w = s * s;
    atomicAdd(&m->count, 1u);
    atomicMin(&m->leader, k);
    atomicAdd(&m->w, w);
    atomicAdd(&m->wx, w * (double)mu[k]);
    atomicAdd(&m->wy, w * (double)mu[K + k]);
    for (int ch = 0; ch < 3; ++ch) atomicAdd(&m->wa[ch], w * (double)amp[(size_t)ch * K + k]);
}

// 1 if particle k appears in the output (alone or as its group's merged particle), else 0.
__device__ __forceinline__ uint32_t merge_outputs(const float* mu, const float* sigma, const float* amp, uint32_t K,
                                                  uint32_t k, int width, int height, double cell, int gx,
                                                  float sigma_max, const MergeCell* cells, int64_t& c) {
    c = merge_cell(mu, sigma, amp, K, k, width, height, cell, gx, sigma_max);
    if (c < 0 || cells[c].count < 2) return 1u;
    return cells[c].leader == k ? 1u : 0u;
}

__global__ void __launch_bounds__(kTreeThreads) merge_count_kernel(const float* __restrict__ mu,
                                                                   const float* __restrict__ sigma,
                                                                   const float* __restrict__ amp, uint32_t K,
                                                                   int width, int height, double cell, int gx,
                                                                   float sigma_max, const MergeCell* __restrict__ cells,
                                                                   uint32_t* __restrict__ block_sums) {
    __shared__ uint32_t s_w[kTreeThreads / kWave];
    const uint32_t k = blockIdx.x * kTreeThreads + threadIdx.x;
    int64_t c;
    uint32_t m = k < K ? merge_outputs(mu, sigma, amp, K, k, width, height, cell, gx, sigma_max, cells, c) : 0u;
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) m += __shfl_xor(m, o, kWave);
    if ((threadIdx.x & 63u) == 0) s_w[threadIdx.x >> 6] = m;
    __syncthreads();
    if (threadIdx.x == 0) block_sums[blockIdx.x] = s_w[0] + s_w[1] + s_w[2] + s_w[3];
}

__global__ void __launch_bounds__(kTreeThreads) merge_scatter_kernel(
    const float* __restrict__ mu, const float* __restrict__ sigma, const float* __restrict__ amp, uint32_t K, int width,
    int height, double cell, int gx, float sigma_max, const MergeCell* __restrict__ cells,
    const uint32_t* __restrict__ block_offsets, uint32_t cap, float* __restrict__ omu, float* __restrict__ osigma,
    float* __restrict__ oamp) {
    __shared__ uint32_t s_w[kTreeThreads / kWave];
    const uint32_t k = blockIdx.x * kTreeThreads + threadIdx.x;
    int64_t c = -1;
    const uint32_t m = k < K ? merge_outputs(mu, sigma, amp, K, k, width, height, cell, gx, sigma_max, cells, c) : 0u;
    const uint64_t bal = ballot64(m != 0u);
    const uint32_t w = threadIdx.x >> 6;
    if ((threadIdx.x & 63u) == 0) s_w[w] = (uint32_t)__popcll(bal);
    __syncthreads();
    if (!m) return;
    uint32_t o = block_offsets[blockIdx.x] + rank_below(bal);
    for (uint32_t q = 0; q < w; ++q) o += s_w[q];
    if (o >= cap) return;
    if (c >= 0 && cells[c].count >= 2) {
        const MergeCell& g = cells[c];
        omu[o] = (float)(g.wx / g.w);
        omu[cap + o] = (float)(g.wy / g.w);
        osigma[o] = (float)sqrt(g.w);
        for (int ch = 0; ch < 3; ++ch) oamp[(size_t)ch * cap + o] = (float)(g.wa[ch] / g.w);
    } else {
        omu[o] = mu[k];
        omu[cap + o] = mu[K + k];
        osigma[o] = sigma[k];
        for (int ch = 0; ch < 3; ++ch) oamp[(size_t)ch * cap + o] = amp[(size_t)ch * K + k];
    }
}

}  // namespace

int octree_grid_ok(const isogs_octree_grid* g) {
    if (!(g->root_side > 0.0f) || !std::isfinite(g->root_side)) return 0;
    for (int a = 0; a < 3; ++a)
        if (!std::isfinite(g->lo[a]) || g->roots[a] < 1) return 0;
    if (g->levels < 1 || g->levels > 12) return 0;
    uint64_t cells = 0;
    for (int l = 0; l < g->levels; ++l)
        cells += ((uint64_t)g->roots[0] << l) * ((uint64_t)g->roots[1] << l) * ((uint64_t)g->roots[2] << l);
    return cells < (1ull << 28) ? 1 : 0;
}

size_t octree_init_ws(const isogs_octree_grid* g) { return oct_layout(oct_geom(*g)).bytes; }

int launch_octree_init(const float* points, const float* colors, int32_t P, const isogs_octree_grid* grid, float tau,
                       int32_t K, float opacity, const isogs_scene* out, int32_t* count, void* ws,
                       hipStream_t stream) {
    const OctGeom G = oct_geom(*grid);
    const OctWs W = oct_layout(G);
    char* base = static_cast<char*>(ws);
    OctSums* sums = reinterpret_cast<OctSums*>(base + W.off_sums);
    uint8_t* active = reinterpret_cast<uint8_t*>(base + W.off_active);
    uint8_t* can = reinterpret_cast<uint8_t*>(base + W.off_can);
    int32_t* stop = reinterpret_cast<int32_t*>(base + W.off_stop);
    uint32_t* state = reinterpret_cast<uint32_t*>(base + W.off_state);
    uint32_t* blocks = reinterpret_cast<uint32_t*>(base + W.off_blocks);
    auto grid_of = [](uint32_t n) { return dim3(std::max(1u, std::min(65535u, (n + kTreeThreads - 1) / kTreeThreads))); };
    const OctLevel& F = G.lv[G.n_levels - 1];
    const uint32_t nf = (uint32_t)(F.gx * F.gy * F.gz);
    hipLaunchKernelGGL(oct_clear_kernel, grid_of(nf), dim3(kTreeThreads), 0, stream, sums + F.first, nf);
    if (P > 0)
        hipLaunchKernelGGL(oct_points_kernel, dim3(((uint32_t)P + kTreeThreads - 1) / kTreeThreads), dim3(kTreeThreads),
                           0, stream, points, colors, (uint32_t)P, G, sums);
    for (int l = G.n_levels - 2; l >= 0; --l) {
        const uint32_t nc = (uint32_t)(G.lv[l].gx * G.lv[l].gy * G.lv[l].gz);
        hipLaunchKernelGGL(oct_up_kernel, dim3((nc + kTreeThreads - 1) / kTreeThreads), dim3(kTreeThreads), 0, stream,
                           G.lv[l], G.lv[l + 1], sums);
    }
    hipLaunchKernelGGL(tree_reset_kernel, dim3(1), dim3(64), 0, stream, state);
    const double thr = (double)tau * kColorQ * kColorQ;
    for (int l = 0; l < G.n_levels; ++l) {
        const OctLevel& L = G.lv[l];
        const OctLevel P0 = l > 0 ? G.lv[l - 1] : L;
        const int has_next = l + 1 < G.n_levels;
        const OctLevel N = has_next ? G.lv[l + 1] : L;
        const uint32_t nb = ((uint32_t)(L.gx * L.gy * L.gz) + kTreeThreads - 1) / kTreeThreads;
        hipLaunchKernelGGL(oct_decide_kernel, dim3(nb), dim3(kTreeThreads), 0, stream, l, L, P0, N, has_next, thr,
                           sums, active, can, stop, blocks);
        hipLaunchKernelGGL(tree_budget_kernel, dim3(1), dim3(kTreeThreads), 0, stream, l, nb, blocks, (uint32_t)K,
                           stop, state);
    }
    const uint32_t nb = (G.n_cells + kTreeThreads - 1) / kTreeThreads;
    hipLaunchKernelGGL(oct_leaf_count_kernel, dim3(nb), dim3(kTreeThreads), 0, stream, G, sums, active, can, stop,
                       blocks);
    hipLaunchKernelGGL(tree_scan_kernel, dim3(1), dim3(kTreeThreads), 0, stream, blocks, nb, count);
    hipLaunchKernelGGL(oct_emit_kernel, dim3(nb), dim3(kTreeThreads), 0, stream, G, sums, active, can, stop, blocks,
                       (uint32_t)K, (uint32_t)out->n, (out->sh_degree + 1) * (out->sh_degree + 1), opacity,
                       const_cast<float*>(out->pos), const_cast<float*>(out->scale), const_cast<float*>(out->opacity),
                       const_cast<float*>(out->color));
    return hipPeekAtLastError() == hipSuccess ? 0 : -1;
}

static int merge_grid(int32_t width, int32_t height, float cell, int* gx, int* gy) {
    const double c = (double)cell;
    const double fx = ceil((double)width / c), fy = ceil((double)height / c);
    if (!(fx * fy < (double)(1u << 26))) return 0;
    *gx = (int)fx;
    *gy = (int)fy;
    return 1;
}

int merge_cells_ok(int32_t width, int32_t height, float cell) {
    int gx, gy;
    return merge_grid(width, height, cell, &gx, &gy);
}

size_t merge_ws(int32_t K, int32_t width, int32_t height, float cell) {
    int gx = 0, gy = 0;
    merge_grid(width, height, cell, &gx, &gy);
    return a256((size_t)gx * gy * sizeof(MergeCell)) + edit_ws(K);
}

int launch_merge(const isogs_field2d* in, int32_t width, int32_t height, float cell, float sigma_max,
                 const isogs_field2d* out, int32_t* count, void* ws, hipStream_t stream) {
    int gx, gy;
    merge_grid(width, height, cell, &gx, &gy);
    const uint32_t nc = (uint32_t)(gx * gy);
    MergeCell* cells = static_cast<MergeCell*>(ws);
    uint32_t* blocks = reinterpret_cast<uint32_t*>(static_cast<char*>(ws) + a256((size_t)nc * sizeof(MergeCell)));
    const uint32_t K = (uint32_t)in->K;
    const uint32_t nb = (K + kTreeThreads - 1) / kTreeThreads;
    const double c = (double)cell;
    hipLaunchKernelGGL(merge_clear_kernel, dim3(std::max(1u, std::min(65535u, (nc + kTreeThreads - 1) / kTreeThreads))),
                       dim3(kTreeThreads), 0, stream, cells, nc);
    if (nb) {
        hipLaunchKernelGGL(merge_accum_kernel, dim3(nb), dim3(kTreeThreads), 0, stream, in->mu, in->sigma, in->amp, K,
                           width, height, c, gx, sigma_max, cells);
        hipLaunchKernelGGL(merge_count_kernel, dim3(nb), dim3(kTreeThreads), 0, stream, in->mu, in->sigma, in->amp, K,
                           width, height, c, gx, sigma_max, cells, blocks);
    }
    hipLaunchKernelGGL(tree_scan_kernel, dim3(1), dim3(kTreeThreads), 0, stream, blocks, nb, count);
    if (nb)
        hipLaunchKernelGGL(merge_scatter_kernel, dim3(nb), dim3(kTreeThreads), 0, stream, in->mu, in->sigma, in->amp,
                           K, width, height, c, gx, sigma_max, cells, blocks, (uint32_t)out->K, out->mu, out->sigma,
                           out->amp);
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
