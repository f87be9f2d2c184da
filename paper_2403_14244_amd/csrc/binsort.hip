// Binning of footprints into 16x16 tiles and the stable (tile, depth) key sort.
//
// Steps (all on the caller's stream, no host synchronisation):
//   1. fill        zero tile ranges, radix histograms, tickets and look-back words
//   2. scan        exclusive scan of per-particle tile counts -> emit offsets, total, status
//   3. emit        one (key, particle index) pair per (particle, member tile), row-major tiles
//   4. histogram   digit counts of every radix pass in one read of the keys
//   5. passes      LSD radix passes over the compacted key (31 depth bits + tile bits),
//                  8-bit digits, each a single kernel with decoupled look-back
//   6. finalize    tile ranges [start, end)
#include "common.h"
#include <algorithm>

#include "kernels.h"

namespace isogs {

constexpr int kScanThreads = 256;
constexpr int kScanItems = 8;
constexpr int kScanBlock = kScanThreads * kScanItems;   // particles per scan block
constexpr int kSortThreads = 256;
constexpr int kSortItems = 16;
constexpr int kSortTile = kSortThreads * kSortItems;    // entries per sort workgroup
constexpr int kRadixBits = 8;
constexpr int kRadix = 1 << kRadixBits;
constexpr int kMaxPasses = 8;
constexpr uint32_t kLbAggregate = 1u << 30;              // look-back word: tile's own count
constexpr uint32_t kLbInclusive = 2u << 30;              // look-back word: prefix through tile
constexpr uint32_t kLbValue = (1u << 30) - 1u;
constexpr uint32_t kSpinLimit = 1u << 22;

// (tile << 32 | depth bits) -> (tile << 31 | depth bits): depth > 0, so its sign bit is 0.
__device__ __forceinline__ uint64_t compact_key(uint64_t k) {
    return ((k >> 32) << 31) | (k & 0x7FFFFFFFull);
}

__device__ __forceinline__ uint32_t digit_of(uint64_t k, int shift) {
    return (uint32_t)(compact_key(k) >> shift) & (kRadix - 1);
}

// Inclusive scan over the 64 lanes of a wave.
__device__ __forceinline__ uint32_t wave_inclusive_scan(uint32_t x) {
    const int lane = (int)lane_id();
#pragma unroll
    for (int o = 1; o < kWave; o <<= 1) {
        const uint32_t y = __shfl_up(x, o, kWave);
        if (lane >= o) x += y;
    }
    return x;
}

// Exclusive scan over a 256-thread block; s_tmp holds 4 words. Returns the block total
// in `total`. Contains __syncthreads.
__device__ __forceinline__ uint32_t block_exclusive_scan(uint32_t x, uint32_t* s_tmp, uint32_t& total) {
    const uint32_t w = threadIdx.x >> 6;
    const uint32_t inc = wave_inclusive_scan(x);
    if (lane_id() == kWave - 1) s_tmp[w] = inc;
    __syncthreads();
    uint32_t before = 0;
    for (uint32_t j = 0; j < w; ++j) before += s_tmp[j];
    total = s_tmp[0] + s_tmp[1] + s_tmp[2] + s_tmp[3];
    __syncthreads();
    return before + inc - x;
}

__global__ void __launch_bounds__(256) fill_u32_kernel(uint32_t* __restrict__ p, size_t n, uint32_t value) {
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
        p[i] = value;
}

// Step 2a: per-block sums of tile counts.
__global__ void __launch_bounds__(kScanThreads) scan_reduce_kernel(const uint32_t* __restrict__ cnt, uint32_t n,
                                                                   uint32_t* __restrict__ block_sums) {
    __shared__ uint32_t s_tmp[4];
    const uint32_t base = blockIdx.x * kScanBlock;
    uint32_t acc = 0;
#pragma unroll
    for (int k = 0; k < kScanItems; ++k) {
        const uint32_t i = base + k * kScanThreads + threadIdx.x;
        acc += (i < n) ? cnt[i] : 0u;
    }
    uint32_t total;
    block_exclusive_scan(acc, s_tmp, total);
    if (threadIdx.x == 0) block_sums[blockIdx.x] = total;
}

// Step 2b: exclusive scan of the block sums (one workgroup), total and capacity status.
__global__ void __launch_bounds__(kScanThreads) scan_top_kernel(uint32_t* __restrict__ block_sums, uint32_t nb,
                                                                uint64_t capacity, uint32_t* __restrict__ count,
                                                                int32_t* __restrict__ status) {
    __shared__ uint32_t s_tmp[4];
    uint64_t carry = 0;
    for (uint32_t b0 = 0; b0 < nb; b0 += kScanThreads) {
        const uint32_t i = b0 + threadIdx.x;
        const uint32_t x = (i < nb) ? block_sums[i] : 0u;
        uint32_t total;
        const uint32_t ex = block_exclusive_scan(x, s_tmp, total);
        if (i < nb) block_sums[i] = (uint32_t)(carry + ex);
        carry += total;
    }
    if (threadIdx.x == 0) {
        const bool fits = carry <= capacity && carry < (uint64_t)kLbValue;
        *count = (uint32_t)(carry > 0xFFFFFFFFull ? 0xFFFFFFFFull : carry);
        *status = fits ? kStatusOk : kStatusCapacity;
    }
}

// Step 2c: emit offsets = block prefix + in-block exclusive scan.
__global__ void __launch_bounds__(kScanThreads) scan_down_kernel(const uint32_t* __restrict__ cnt, uint32_t n,
                                                                 const uint32_t* __restrict__ block_prefix,
                                                                 uint32_t* __restrict__ offsets) {
    __shared__ uint32_t s_tmp[4];
    // each thread scans kScanItems consecutive particles (blocked), lanes then threads
    const uint32_t base = blockIdx.x * kScanBlock + threadIdx.x * kScanItems;
    uint32_t v[kScanItems];
    uint32_t acc = 0;
#pragma unroll
    for (int k = 0; k < kScanItems; ++k) {
        v[k] = (base + k < n) ? cnt[base + k] : 0u;
        acc += v[k];
    }
    uint32_t total;
    uint32_t run = block_exclusive_scan(acc, s_tmp, total) + block_prefix[blockIdx.x];
#pragma unroll
    for (int k = 0; k < kScanItems; ++k) {
        if (base + k < n) offsets[base + k] = run;
        run += v[k];
    }
}

// Step 3: one entry per (particle, member tile); entries of a particle are consecutive
// from its offset, tiles in row-major order. A particle writes no more entries than its
// tile count says (the count may come from elsewhere); missing ones get a sentinel key.
__global__ void __launch_bounds__(256) emit_kernel(const ViewPack pk, const float4* __restrict__ record,
                                                   const float* __restrict__ depth,
                                                   const uint32_t* __restrict__ tile_count,
                                                   const uint32_t* __restrict__ offsets,
                                                   const uint32_t* __restrict__ count_p, uint64_t capacity,
                                                   uint64_t* __restrict__ keys, uint32_t* __restrict__ vals) {
    const uint32_t count = *count_p;
    if ((uint64_t)count > capacity) return;
    const int vi = view_of_block(pk, blockIdx.x);
    const ViewDesc& vd = pk.v[vi];
    const uint32_t li = (blockIdx.x - pk.block_begin[vi]) * blockDim.x + threadIdx.x;
    if (li >= vd.n) return;
    const uint32_t i = vd.p_off + li;
    const uint32_t want = tile_count[i];
    if (want == 0) return;
    const uint32_t e0 = offsets[i];
    if ((uint64_t)e0 + want > count) return;
    const float4 fp = record[2 * (size_t)i];
    const float r = record[2 * (size_t)i + 1].w;
    const uint64_t zbits = (uint64_t)__float_as_uint(depth[i]);
    int tx0, tx1, ty0, ty1;
    tile_box(fp.x, fp.y, r, vd.tiles_x, vd.tiles_y, tx0, tx1, ty0, ty1);
    const float r2 = r * r;
    const float w_lim = (float)vd.width - 0.5f, h_lim = (float)vd.height - 0.5f;
    uint32_t j = 0;
    for (int ty = ty0; ty <= ty1 && j < want; ++ty) {
        for (int tx = tx0; tx <= tx1 && j < want; ++tx) {
            if (!tile_member(fp.x, fp.y, r2, tx, ty, w_lim, h_lim)) continue;
            const uint32_t e = e0 + j++;
            const uint64_t tid = (uint64_t)(vd.tile_base + (uint32_t)(ty * vd.tiles_x + tx));
            keys[e] = (tid << 32) | zbits;
            vals[e] = i;
        }
    }
    for (; j < want; ++j) {
        const uint32_t e = e0 + j;
        keys[e] = ~0ull;
        vals[e] = i;
    }
}

// Step 4: digit histograms of all passes in one sweep over the keys.
__global__ void __launch_bounds__(256) sort_hist_kernel(const uint64_t* __restrict__ keys,
                                                        const uint32_t* __restrict__ count_p, uint64_t capacity,
                                                        int passes, uint32_t* __restrict__ hist) {
    __shared__ uint32_t s_h[kMaxPasses][kRadix];
    for (int p = 0; p < kMaxPasses; ++p) s_h[p][threadIdx.x] = 0u;
    __syncthreads();
    const uint32_t count = *count_p;
    if ((uint64_t)count > capacity) return;
    for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < count; i += gridDim.x * blockDim.x) {
        const uint64_t c = compact_key(keys[i]);
        for (int p = 0; p < passes; ++p) atomicAdd(&s_h[p][(uint32_t)(c >> (p * kRadixBits)) & (kRadix - 1)], 1u);
    }
    __syncthreads();
    for (int p = 0; p < passes; ++p) {
        const uint32_t h = s_h[p][threadIdx.x];
        if (h) atomicAdd(&hist[p * kRadix + threadIdx.x], h);
    }
}

// Step 5: one stable LSD pass. Each workgroup takes the next 4096-entry tile in ticket
// order, ranks its entries per digit with wavefront ballots (lanes with equal digits are
// matched bit by bit; the rank is the count of matching lanes below), publishes its digit
// counts and resolves its global offsets by looking back over earlier tiles' words, then
// reorders the tile in LDS so the scatter writes contiguous runs per digit.
__global__ void __launch_bounds__(kSortThreads) sort_pass_kernel(
    const uint64_t* __restrict__ kin, const uint32_t* __restrict__ vin, uint64_t* __restrict__ kout,
    uint32_t* __restrict__ vout, const uint32_t* __restrict__ count_p, uint64_t capacity, int pass,
    const uint32_t* __restrict__ hist, uint32_t* __restrict__ lookback, uint32_t* __restrict__ ticket,
    int32_t* __restrict__ status) {
    __shared__ uint64_t s_buf[kSortTile];   // tile reordered by digit: keys, then values
    __shared__ uint32_t s_wcnt[4][kRadix];
    __shared__ uint32_t s_local[kRadix];
    __shared__ uint32_t s_base[kRadix];
    __shared__ uint32_t s_tmp[4];
    __shared__ uint32_t s_ticket;

    const uint32_t count = *count_p;
    if ((uint64_t)count > capacity) return;
    const uint32_t ntiles = (count + kSortTile - 1) / kSortTile;
    const uint32_t t = threadIdx.x, w = t >> 6, lane = t & 63;
    if (t == 0) s_ticket = atomicAdd(ticket, 1u);
    for (int k = 0; k < 4; ++k) s_wcnt[k][t] = 0u;
    __syncthreads();
    const uint32_t tile = s_ticket;
    if (tile >= ntiles) return;
    const int shift = pass * kRadixBits;

    // load: wave w owns entries [tile*4096 + w*1024, +1024), item i of lane l at i*64 + l
    const uint32_t wbase = tile * kSortTile + w * (kSortTile / 4);
    uint64_t k[kSortItems];
    uint32_t v[kSortItems];
    uint32_t rk[kSortItems];
#pragma unroll
    for (int i = 0; i < kSortItems; ++i) {
        const uint32_t idx = wbase + i * kWave + lane;
        if (idx < count) {
            k[i] = kin[idx];
            v[i] = vin[idx];
        } else {
            k[i] = 0;
            v[i] = 0;
        }
    }
    // rank within the wave, rounds in entry order
#pragma unroll
    for (int i = 0; i < kSortItems; ++i) {
        const bool valid = wbase + i * kWave + lane < count;
        const uint32_t d = digit_of(k[i], shift);
        uint64_t m = ballot64(valid);
#pragma unroll
        for (int b = 0; b < kRadixBits; ++b) {
            const bool bit = (d >> b) & 1u;
            const uint64_t bal = ballot64(bit);
            m &= bit ? bal : ~bal;
        }
        const uint32_t below = rank_below(m);
        const uint32_t prior = s_wcnt[w][d];
        rk[i] = prior + below;
        if (valid && below == 0) s_wcnt[w][d] = prior + (uint32_t)__popcll(m);
    }
    __syncthreads();

    // thread t owns digit t: wave prefixes, tile total, look-back
    const uint32_t c0 = s_wcnt[0][t], c1 = s_wcnt[1][t], c2 = s_wcnt[2][t], c3 = s_wcnt[3][t];
    const uint32_t mine = c0 + c1 + c2 + c3;
    s_wcnt[0][t] = 0u;
    s_wcnt[1][t] = c0;
    s_wcnt[2][t] = c0 + c1;
    s_wcnt[3][t] = c0 + c1 + c2;
    uint32_t* lb = lookback;  // this pass's region
    __hip_atomic_store(&lb[(size_t)tile * kRadix + t], (tile == 0 ? kLbInclusive : kLbAggregate) | mine,
                       __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    uint32_t excl = 0;
    if (tile > 0) {
        int32_t j = (int32_t)tile - 1;
        uint32_t spins = 0;
        while (j >= 0) {
            const uint32_t word = __hip_atomic_load(&lb[(size_t)j * kRadix + t], __ATOMIC_RELAXED,
                                                    __HIP_MEMORY_SCOPE_AGENT);
            const uint32_t flag = word & ~kLbValue;
            if (flag == 0u) {
                if (++spins > kSpinLimit) {
                    *status = kStatusDevice;
                    break;
                }
                __builtin_amdgcn_s_sleep(1);
                continue;
            }
            excl += word & kLbValue;
            if (flag == kLbInclusive) break;
            --j;
        }
        __hip_atomic_store(&lb[(size_t)tile * kRadix + t], kLbInclusive | (excl + mine), __ATOMIC_RELAXED,
                           __HIP_MEMORY_SCOPE_AGENT);
    }
    uint32_t tot;
    const uint32_t gbase = block_exclusive_scan(hist[pass * kRadix + t], s_tmp, tot);
    const uint32_t lbase = block_exclusive_scan(mine, s_tmp, tot);
    s_base[t] = gbase + excl;
    s_local[t] = lbase;
    __syncthreads();

    // reorder in LDS by digit (stable), then write runs: keys first, then the values
    // through the same buffer (halves the LDS a workgroup needs)
    uint32_t lpos[kSortItems];
#pragma unroll
    for (int i = 0; i < kSortItems; ++i) {
        lpos[i] = 0xFFFFFFFFu;
        if (wbase + i * kWave + lane < count) {
            const uint32_t d = digit_of(k[i], shift);
            lpos[i] = s_local[d] + s_wcnt[w][d] + rk[i];
            s_buf[lpos[i]] = k[i];
        }
    }
    __syncthreads();
    const uint32_t n_here = min((uint32_t)kSortTile, count - tile * kSortTile);
    uint32_t dst[kSortItems];
#pragma unroll
    for (int i = 0; i < kSortItems; ++i) {
        const uint32_t j = t + i * kSortThreads;
        dst[i] = 0xFFFFFFFFu;
        if (j < n_here) {
            const uint64_t key = s_buf[j];
            const uint32_t d = digit_of(key, shift);
            dst[i] = s_base[d] + (j - s_local[d]);
            if (dst[i] < count) kout[dst[i]] = key;
        }
    }
    __syncthreads();
    uint32_t* s_val = reinterpret_cast<uint32_t*>(s_buf);
#pragma unroll
    for (int i = 0; i < kSortItems; ++i)
        if (lpos[i] != 0xFFFFFFFFu) s_val[lpos[i]] = v[i];
    __syncthreads();
#pragma unroll
    for (int i = 0; i < kSortItems; ++i) {
        const uint32_t j = t + i * kSortThreads;
        if (j < n_here && dst[i] < count) vout[dst[i]] = s_val[j];
    }
}

// Step 6: tile ranges.
__global__ void __launch_bounds__(256) finalize_kernel(const uint64_t* __restrict__ keys,
                                                       const uint32_t* __restrict__ count_p, uint64_t capacity,
                                                       uint32_t tiles_total, uint32_t* __restrict__ ranges) {
    const uint32_t count = *count_p;
    if ((uint64_t)count > capacity) return;
    for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < count; i += gridDim.x * blockDim.x) {
        const uint32_t tl = (uint32_t)(keys[i] >> 32);
        const uint32_t prev = i > 0 ? (uint32_t)(keys[i - 1] >> 32) : 0xFFFFFFFFu;
        const uint32_t next = i + 1 < count ? (uint32_t)(keys[i + 1] >> 32) : 0xFFFFFFFFu;
        if (tl < tiles_total) {
            if (tl != prev) ranges[2 * tl] = i;
            if (tl != next) ranges[2 * tl + 1] = i + 1;
        }
    }
}

static size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

BinSortPlan plan_bin_sort(const int32_t* n_per_view, const isogs_camera* cams, int32_t nv, uint64_t capacity) {
    BinSortPlan p{};
    p.capacity = capacity;
    uint64_t n = 0, tiles = 0;
    for (int v = 0; v < nv; ++v) {
        n += (uint64_t)n_per_view[v];
        tiles += (uint64_t)((cams[v].width + kTile - 1) / kTile) * (uint64_t)((cams[v].height + kTile - 1) / kTile);
    }
    p.n_total = (uint32_t)n;
    p.tiles_total = (uint32_t)tiles;
    int tile_bits = 0;
    while (tile_bits < 32 && (1ull << tile_bits) < tiles) ++tile_bits;
    p.passes = (31 + tile_bits + kRadixBits - 1) / kRadixBits;
    p.sort_tiles = (uint32_t)((capacity + kSortTile - 1) / kSortTile);
    p.scan_blocks = (uint32_t)((n + kScanBlock - 1) / kScanBlock);
    size_t off = 0;
    p.off_keys_alt = off;   off = align256(off + capacity * 8);
    p.off_vals_alt = off;   off = align256(off + capacity * 4);
    // zero-initialised region: histograms, tickets, look-back words (contiguous)
    p.off_hist = off;       off += (size_t)kMaxPasses * kRadix * 4;
    p.off_tickets = off;    off += (size_t)kMaxPasses * 4;
    p.off_lookback = off;   off = align256(off + (size_t)p.passes * p.sort_tiles * kRadix * 4);
    p.off_block_sums = off; off = align256(off + (size_t)(p.scan_blocks + 1) * 4);
    p.off_flags = off;      off = align256(off + 64);
    p.bytes = off;
    return p;
}

int launch_bin_sort(const BinSortPlan& plan, const isogs_projected* proj, const int32_t* n_per_view,
                    const isogs_camera* cams, int32_t nv, const isogs_bins* bins, void* ws, hipStream_t stream) {
    char* base = static_cast<char*>(ws);
    uint64_t* keys_alt = reinterpret_cast<uint64_t*>(base + plan.off_keys_alt);
    uint32_t* vals_alt = reinterpret_cast<uint32_t*>(base + plan.off_vals_alt);
    uint32_t* hist = reinterpret_cast<uint32_t*>(base + plan.off_hist);
    uint32_t* tickets = reinterpret_cast<uint32_t*>(base + plan.off_tickets);
    uint32_t* lookback = reinterpret_cast<uint32_t*>(base + plan.off_lookback);
    uint32_t* block_sums = reinterpret_cast<uint32_t*>(base + plan.off_block_sums);

    // 1. zero ranges and the sort's bookkeeping
    {
        const size_t nz = (plan.off_block_sums - plan.off_hist) / 4;
        hipLaunchKernelGGL(fill_u32_kernel, dim3((unsigned)std::min<size_t>(1024, (nz + 255) / 256 + 1)), dim3(256), 0,
                           stream, hist, nz, 0u);
        const size_t nr = (size_t)plan.tiles_total * 2;
        if (nr)
            hipLaunchKernelGGL(fill_u32_kernel, dim3((unsigned)std::min<size_t>(1024, (nr + 255) / 256)), dim3(256), 0,
                               stream, bins->ranges, nr, 0u);
    }
    // 2. scan of tile counts
    const uint32_t n = plan.n_total;
    if (plan.scan_blocks) {
        hipLaunchKernelGGL(scan_reduce_kernel, dim3(plan.scan_blocks), dim3(kScanThreads), 0, stream,
                           proj->tile_count, n, block_sums);
    }
    hipLaunchKernelGGL(scan_top_kernel, dim3(1), dim3(kScanThreads), 0, stream, block_sums, plan.scan_blocks,
                       plan.capacity, bins->count, bins->status);
    if (plan.scan_blocks) {
        hipLaunchKernelGGL(scan_down_kernel, dim3(plan.scan_blocks), dim3(kScanThreads), 0, stream,
                           proj->tile_count, n, block_sums, bins->offsets);
    }
    if (hipPeekAtLastError() != hipSuccess) return -1;

    // ping-pong so that the last pass lands in the caller's arrays
    const bool odd = plan.passes & 1;
    uint64_t* k_emit = odd ? keys_alt : bins->keys;
    uint32_t* v_emit = odd ? vals_alt : bins->pidx;
    uint64_t* k_other = odd ? bins->keys : keys_alt;
    uint32_t* v_other = odd ? bins->pidx : vals_alt;

    // 3. emit, per group of views
    uint32_t p_off = 0, tile_base = 0;
    for (int v0 = 0; v0 < nv; v0 += kMaxViews) {
        ViewPack pk{};
        pk.nv = min(kMaxViews, nv - v0);
        uint32_t blocks = 0;
        for (int j = 0; j < pk.nv; ++j) {
            const isogs_camera& cam = cams[v0 + j];
            ViewDesc& d = pk.v[j];
            d.p_off = p_off;
            d.n = (uint32_t)n_per_view[v0 + j];
            d.tile_base = tile_base;
            d.width = cam.width;
            d.height = cam.height;
            d.tiles_x = (cam.width + kTile - 1) / kTile;
            d.tiles_y = (cam.height + kTile - 1) / kTile;
            pk.block_begin[j] = blocks;
            blocks += (d.n + 255u) / 256u;
            p_off += d.n;
            tile_base += (uint32_t)(d.tiles_x * d.tiles_y);
        }
        pk.block_begin[pk.nv] = blocks;
        if (blocks)
            hipLaunchKernelGGL(emit_kernel, dim3(blocks), dim3(256), 0, stream, pk,
                               reinterpret_cast<const float4*>(proj->record), proj->depth, proj->tile_count,
                               bins->offsets, bins->count, plan.capacity, k_emit, v_emit);
    }
    if (plan.capacity == 0) return hipPeekAtLastError() == hipSuccess ? 0 : -1;

    // 4. histograms
    const unsigned hist_blocks = (unsigned)std::min<uint64_t>(512, (plan.capacity + 255) / 256);
    hipLaunchKernelGGL(sort_hist_kernel, dim3(hist_blocks), dim3(256), 0, stream, k_emit, bins->count,
                       plan.capacity, plan.passes, hist);
    // 5. radix passes
    const uint64_t* kin = k_emit;
    const uint32_t* vin = v_emit;
    uint64_t* kout = k_other;
    uint32_t* vout = v_other;
    for (int p = 0; p < plan.passes; ++p) {
        hipLaunchKernelGGL(sort_pass_kernel, dim3(plan.sort_tiles), dim3(kSortThreads), 0, stream, kin, vin, kout,
                           vout, bins->count, plan.capacity, p, hist,
                           lookback + (size_t)p * plan.sort_tiles * kRadix, tickets + p, bins->status);
        const uint64_t* tk = kin;
        const uint32_t* tv = vin;
        kin = kout;
        vin = vout;
        kout = const_cast<uint64_t*>(tk);
        vout = const_cast<uint32_t*>(tv);
    }
    // 6. ranges
    const unsigned fin_blocks = (unsigned)std::min<uint64_t>(2048, (plan.capacity + 255) / 256);
    hipLaunchKernelGGL(finalize_kernel, dim3(fin_blocks), dim3(256), 0, stream, bins->keys, bins->count,
                       plan.capacity, plan.tiles_total, bins->ranges);
    return hipPeekAtLastError() == hipSuccess ? 0 : -1;
}

}  // namespace isogs
