// Binning of footprints into 16x16 tiles and the stable (tile, depth) sort.
//
// The sort is split by key part. Entries are emitted in particle order, which is the tie
// order of the (tile, depth) sort; a stable sort on the tile id alone therefore leaves
// each tile's entries in emit order, and a stable sort of every tile's segment on depth
// then yields exactly the stable (tile, depth) order. The global passes rank only the tile
// bits (ceil(tile bits / 8) passes instead of ceil((tile bits + 31) / 8)), carrying the
// particle index and the depth bits along so that the per-tile depth sort, which runs in
// LDS, reads its keys sequentially instead of gathering them.
//
// Steps (all on the caller's stream, no host synchronisation):
//   1. fill        zero tile ranges and counters
//   2. scan        exclusive scan of per-particle tile counts -> emit offsets, total, status
//   3. emit        one (tile id, particle index, depth bits) per (particle, member tile)
//   4. passes      stable LSD radix passes over the tile id, digits of up to 9 bits, each
//                  as count / scan / scatter kernels; the per-digit scan over the sort tiles
//                  also yields each digit's total, from which the scatter forms the bases
//   5. finalize    tile ranges [start, end)
//   6. segments    stable sort of each tile's segment on the depth bits (and the 64-bit
//                  (tile, depth) keys, when the caller asks for them): one wave per short
//                  segment, two, four or eight waves per longer one (several segments to a
//                  workgroup), the whole workgroup beyond 4096 entries
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
constexpr int kRadixBits = 8;                 // digits of the per-tile depth sorts
constexpr int kRadix = 1 << kRadixBits;
constexpr int kTileRadixBits = 9;             // digits of the global tile-id passes
constexpr int kTileRadix = 1 << kTileRadixBits;
constexpr int kMaxPasses = 4;                             // tile ids have at most 32 bits
constexpr int kBigThreads = 512;                          // workgroup of the long-segment sort
constexpr int kBigWaves = kBigThreads / kWave;
constexpr int kBigItems = 8;
constexpr uint32_t kSegMax = kBigThreads * kBigItems;    // longest segment sorted in LDS
constexpr uint32_t kCountLimit = (1u << 30) - 1u;       // entries per batch must stay below

// Splits the key bits [lo, hi) into the fewest passes of at most `maxw` bits, widths as
// equal as possible (ballot ranking costs one ballot per digit bit, so no pass ranks unused
// bits).
struct DigitSplit {
    int passes, base, extra, lo;
    __host__ __device__ DigitSplit(int lo_, int hi_, int maxw = kRadixBits) : lo(lo_) {
        const int span = hi_ > lo_ ? hi_ - lo_ : 0;
        passes = (span + maxw - 1) / maxw;
        base = passes ? span / passes : 0;
        extra = passes ? span % passes : 0;
    }
    __host__ __device__ int width(int p) const { return base + (p < extra ? 1 : 0); }
    __host__ __device__ int shift(int p) const { return lo + p * base + (p < extra ? p : extra); }
};

// The segment sorts rank fixed 8-bit digits, [lo, lo + 8 passes) covering the differing
// bits [lo, hi): bits at and above hi are equal within the segment, so ranking them too
// leaves the order unchanged, and a compile-time width keeps the ballot chain free of
// per-bit conditions (their masks otherwise take scalar registers the kernel runs short of).
struct Split8 {
    int passes, lo;
    __device__ Split8(int lo_, int hi_) : passes(hi_ > lo_ ? (hi_ - lo_ + kRadixBits - 1) / kRadixBits : 0), lo(lo_) {}
    __device__ int shift(int p) const { return lo + p * kRadixBits; }
};

// Digit of key k at (shift, bits).
__device__ __forceinline__ uint32_t digit_at(uint32_t k, int shift, int bits) {
    return (k >> shift) & ((1u << bits) - 1u);
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

// Exclusive scan over a block of NW waves; s_tmp holds NW words. Returns the block total
// in `total`. Contains __syncthreads.
template <int NW = 4>
__device__ __forceinline__ uint32_t block_exclusive_scan(uint32_t x, uint32_t* s_tmp, uint32_t& total) {
    const uint32_t w = threadIdx.x >> 6;
    const uint32_t inc = wave_inclusive_scan(x);
    if (lane_id() == kWave - 1) s_tmp[w] = inc;
    __syncthreads();
    uint32_t before = 0;
    total = 0;
#pragma unroll
    for (int j = 0; j < NW; ++j) {
        before += ((uint32_t)j < w) ? s_tmp[j] : 0u;
        total += s_tmp[j];
    }
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
    const uint32_t base = blockIdx.x * kScanBlock + threadIdx.x * kScanItems;
    uint32_t acc = 0;
    if (base + kScanItems <= n && (reinterpret_cast<uintptr_t>(cnt) & 15u) == 0) {
        const uint4 a = *reinterpret_cast<const uint4*>(cnt + base);
        const uint4 b = *reinterpret_cast<const uint4*>(cnt + base + 4);
        acc = a.x + a.y + a.z + a.w + b.x + b.y + b.z + b.w;
    } else {
#pragma unroll
        for (int k = 0; k < kScanItems; ++k) acc += (base + k < n) ? cnt[base + k] : 0u;
    }
    uint32_t total;
    block_exclusive_scan(acc, s_tmp, total);
    if (threadIdx.x == 0) block_sums[blockIdx.x] = total;
}

// Step 2b: exclusive scan of the block sums (one workgroup), total and capacity status.
// Each thread takes a run of consecutive sums, so one workgroup scan covers up to
// kScanThreads * kTopItems of them at a time (a 10-view call of 1M particles has about 5000).
constexpr uint32_t kTopItems = 32;
__global__ void __launch_bounds__(kScanThreads) scan_top_kernel(uint32_t* __restrict__ block_sums, uint32_t nb,
                                                                uint64_t capacity, uint32_t* __restrict__ count,
                                                                int32_t* __restrict__ status) {
    __shared__ uint32_t s_tmp[4];
    uint64_t carry = 0;
    for (uint32_t b0 = 0; b0 < nb; b0 += kScanThreads * kTopItems) {
        const uint32_t per = (min(nb - b0, kScanThreads * kTopItems) + kScanThreads - 1) / kScanThreads;
        const uint32_t i0 = b0 + threadIdx.x * per, i1 = min(i0 + per, nb);
        uint32_t sum = 0;
        for (uint32_t i = i0; i < i1; ++i) sum += block_sums[i];
        uint32_t total;
        uint64_t run = carry + block_exclusive_scan(sum, s_tmp, total);
        for (uint32_t i = i0; i < i1; ++i) {
            const uint32_t x = block_sums[i];
            block_sums[i] = (uint32_t)run;
            run += x;
        }
        carry += total;
    }
    if (threadIdx.x == 0) {
        const bool fits = carry <= capacity && carry < (uint64_t)kCountLimit;
        *count = (uint32_t)(carry > 0xFFFFFFFFull ? 0xFFFFFFFFull : carry);
        *status = fits ? kStatusOk : kStatusCapacity;
    }
}

// Step 2c: emit offsets = block prefix + in-block exclusive scan.
__global__ void __launch_bounds__(kScanThreads) scan_down_kernel(const uint32_t* __restrict__ cnt, uint32_t n,
                                                                 const uint32_t* __restrict__ block_prefix,
                                                                 uint32_t* __restrict__ offsets) {
    __shared__ uint32_t s_tmp[4];
    // each thread scans kScanItems consecutive particles (blocked), lanes then threads; whole
    // runs move as two 16-byte loads and stores when both arrays allow it
    static_assert(kScanItems == 8, "two 16-byte vectors per thread");
    const uint32_t base = blockIdx.x * kScanBlock + threadIdx.x * kScanItems;
    const bool vec = base + kScanItems <= n && ((reinterpret_cast<uintptr_t>(cnt) | reinterpret_cast<uintptr_t>(offsets)) & 15u) == 0;
    uint32_t v[kScanItems];
    if (vec) {
        const uint4 a = *reinterpret_cast<const uint4*>(cnt + base);
        const uint4 b = *reinterpret_cast<const uint4*>(cnt + base + 4);
        v[0] = a.x; v[1] = a.y; v[2] = a.z; v[3] = a.w;
        v[4] = b.x; v[5] = b.y; v[6] = b.z; v[7] = b.w;
    } else {
#pragma unroll
        for (int k = 0; k < kScanItems; ++k) v[k] = (base + k < n) ? cnt[base + k] : 0u;
    }
    uint32_t acc = 0;
#pragma unroll
    for (int k = 0; k < kScanItems; ++k) acc += v[k];
    uint32_t total;
    const uint32_t run = block_exclusive_scan(acc, s_tmp, total) + block_prefix[blockIdx.x];
    uint32_t o[kScanItems];
    o[0] = run;
#pragma unroll
    for (int k = 1; k < kScanItems; ++k) o[k] = o[k - 1] + v[k - 1];
    if (vec) {
        *reinterpret_cast<uint4*>(offsets + base) = make_uint4(o[0], o[1], o[2], o[3]);
        *reinterpret_cast<uint4*>(offsets + base + 4) = make_uint4(o[4], o[5], o[6], o[7]);
    } else {
#pragma unroll
        for (int k = 0; k < kScanItems; ++k)
            if (base + k < n) offsets[base + k] = o[k];
    }
}


// Step 3: one entry per (particle, member tile); entries of a particle are consecutive
// from its offset, tiles in row-major order. A particle writes no more entries than its
// tile count says (the count may come from elsewhere; here it is the difference of
// consecutive offsets, which the scan made from those counts, the last one's from the
// total); missing ones get the sentinel id 0xFFFFFFFF, which sorts last and belongs to no
// tile. One workgroup per chunk of 256 particles of a view. The chunk's entries are one
// run of the output; when it holds at most kEmitStage entries they are gathered in LDS
// (tile id and owner) and written as whole runs, else each particle writes its own.
constexpr uint32_t kEmitStage = 2048;

__global__ void __launch_bounds__(256) emit_kernel(const ViewPack pk, const float4* __restrict__ record,
                                                   const uint32_t* __restrict__ offsets, uint32_t n_total,
                                                   const float* __restrict__ depth,
                                                   const uint32_t* __restrict__ count_p, uint64_t capacity,
                                                   uint32_t* __restrict__ keys, uint32_t* __restrict__ vals,
                                                   uint32_t* __restrict__ zbits) {
    __shared__ uint32_t s_key[kEmitStage];
    __shared__ uint8_t s_own[kEmitStage];
    __shared__ uint32_t s_z[256];
    const uint32_t count = *count_p;
    if ((uint64_t)count > capacity) return;
    const uint32_t c = blockIdx.x;
    const int vi = view_of_block(pk, c);
    const ViewDesc& vd = pk.v[vi];
    const uint32_t first = vd.p_off + (c - pk.block_begin[vi]) * 256u;
    const uint32_t last = min(first + 255u, vd.p_off + vd.n - 1u);
    // the chunk's run [E0, E1), uniform over the workgroup
    const uint32_t E0 = offsets[first];
    const uint32_t E1 = last + 1 < n_total ? offsets[last + 1] : count;
    const bool staged = E1 >= E0 && E1 <= count && E1 - E0 <= kEmitStage;
    const uint32_t i = first + threadIdx.x;
    uint32_t e0 = 0, want = 0;
    if (i <= last) {
        e0 = offsets[i];
        want = (i + 1 < n_total ? offsets[i + 1] : count) - e0;
        if ((uint64_t)e0 + want > count) want = 0;
    }
    uint32_t z = 0;
    int tx0 = 0, tx1 = -1, ty0 = 0, ty1 = -1;
    float fx = 0.f, fy = 0.f, r2 = 0.f;
    if (want) {
        const float4 fp = record[2 * (size_t)i];
        const float r = record[2 * (size_t)i + 1].w;
        z = __float_as_uint(depth[i]);
        fx = fp.x;
        fy = fp.y;
        r2 = r * r;
        tile_box(fp.x, fp.y, r, vd.tiles_x, vd.tiles_y, tx0, tx1, ty0, ty1);
    }
    const float w_lim = (float)vd.width - 0.5f, h_lim = (float)vd.height - 0.5f;
    if (!staged) {
        uint32_t j = 0;
        for (int ty = ty0; ty <= ty1 && j < want; ++ty) {
            for (int tx = tx0; tx <= tx1 && j < want; ++tx) {
                if (!tile_member(fx, fy, r2, tx, ty, w_lim, h_lim)) continue;
                const uint32_t e = e0 + j++;
                keys[e] = vd.tile_base + (uint32_t)(ty * vd.tiles_x + tx);
                vals[e] = i;
                zbits[e] = z;
            }
        }
        for (; j < want; ++j) {
            const uint32_t e = e0 + j;
            keys[e] = 0xFFFFFFFFu;
            vals[e] = i;
            zbits[e] = z;
        }
        return;
    }
    // staged: every entry of the run belongs to one particle of the chunk (the offsets are
    // non-decreasing), so each LDS slot is written once
    s_z[threadIdx.x] = z;
    const uint32_t l0 = e0 - E0;
    uint32_t j = 0;
    for (int ty = ty0; ty <= ty1 && j < want; ++ty) {
        for (int tx = tx0; tx <= tx1 && j < want; ++tx) {
            if (!tile_member(fx, fy, r2, tx, ty, w_lim, h_lim)) continue;
            s_key[l0 + j] = vd.tile_base + (uint32_t)(ty * vd.tiles_x + tx);
            s_own[l0 + j] = (uint8_t)threadIdx.x;
            ++j;
        }
    }
    for (; j < want; ++j) {
        s_key[l0 + j] = 0xFFFFFFFFu;
        s_own[l0 + j] = (uint8_t)threadIdx.x;
    }
    __syncthreads();
    for (uint32_t q = threadIdx.x; q < E1 - E0; q += 256u) {
        const uint32_t o = s_own[q];
        keys[E0 + q] = s_key[q];
        vals[E0 + q] = first + o;
        zbits[E0 + q] = s_z[o];
    }
}

// Ranks up to ITEMS items per lane within the wave by a digit of `bits` <= MAXB bits. Items are taken in
// rounds (item i of every lane in round i, lanes in order), so ranks follow the order
// (round, lane). Lanes with equal digits are matched bit by bit with ballots; an item's
// rank is the wave's count of its digit in earlier rounds plus the matching lanes below
// it. `cnt` holds the wave's 256 digit counters (zero on entry) and ends with the wave's
// digit totals. Bit i of `valid` marks item i as present; `items` (uniform) bounds the
// rounds.
template <int ITEMS, int MAXB = kRadixBits>
__device__ __forceinline__ void wave_rank(const uint32_t (&k)[ITEMS], int shift, int bits, uint32_t valid,
                                          int items, uint32_t* __restrict__ cnt, uint32_t (&rk)[ITEMS]) {
#pragma unroll
    for (int i = 0; i < ITEMS; ++i) {
        if (i < items) {
            const uint32_t d = digit_at(k[i], shift, bits);
            const bool ok = (valid >> i) & 1u;
            const uint64_t okm = ballot64(ok);
            uint32_t m_lo = (uint32_t)okm, m_hi = (uint32_t)(okm >> 32);
#pragma unroll
            for (int b = 0; b < MAXB; ++b) {
                if (b < bits) {
                    // keep the lanes whose bit b equals this lane's: m &= ~(ballot ^ sign(bit))
                    // (one three-input bitwise instruction per half)
                    const uint32_t sx = (uint32_t)((int32_t)(d << (31 - b)) >> 31);   // bit b, sign-extended
                    const uint64_t bal = ballot64(sx != 0u);
                    m_lo &= ~((uint32_t)bal ^ sx);
                    m_hi &= ~((uint32_t)(bal >> 32) ^ sx);
                }
            }
            const uint64_t m = ((uint64_t)m_hi << 32) | m_lo;
            const uint32_t below = rank_below(m);
            const uint32_t prior = cnt[d];
            rk[i] = prior + below;
            if (ok && below == 0) cnt[d] = prior + (uint32_t)__popcll(m);
        }
    }
}

// Step 4: stable LSD passes over the tile ids (digit of `bits` <= 9 bits at `shift`), each
// in three kernels over 4096-entry sort tiles, with no waiting between workgroups:
//   4a  count     each sort tile's digit counts, stored digit-major
//   4b  scan      per digit, the exclusive prefix over the sort tiles and the total
//   4c  scatter   each sort tile ranks its entries per digit within each wave (ballots),
//                 places them at digit base + earlier tiles' count + rank, reorders in LDS
//                 so that the stores are contiguous runs per digit
// Count and scatter give each XCD a contiguous range of sort tiles (xcd_swizzle over the
// tiles in use): neighbouring sort tiles write neighbouring words of the digit-major counts
// and, for a digit, adjacent pieces of its output run, so the partial cache lines they
// leave are completed in one L2 instead of being written back separately from several.
__global__ void __launch_bounds__(kSortThreads) tile_count_kernel(const uint32_t* __restrict__ kin,
                                                                  const uint32_t* __restrict__ count_p,
                                                                  uint64_t capacity, int shift, int bits,
                                                                  uint32_t* __restrict__ tcount, uint32_t stride) {
    // four copies of the counters, lane l adding to copy l mod 4: lanes of one instruction
    // that share a digit (many do in the second pass, whose input is ordered by the low
    // digit) mostly hit different copies, at different banks (copies kTileRadix + 1 apart)
    constexpr uint32_t kCopy = kTileRadix + 1;
    __shared__ uint32_t s_h[4 * kCopy];
    const uint32_t count = *count_p;
    if ((uint64_t)count > capacity) return;
    const uint32_t n_tiles = (count + kSortTile - 1) / kSortTile;
    if (blockIdx.x >= n_tiles) return;
    const uint32_t tile = xcd_swizzle(blockIdx.x, n_tiles), t = threadIdx.x;
    for (uint32_t q = t; q < 4 * kCopy; q += kSortThreads) s_h[q] = 0u;
    __syncthreads();
    uint32_t k[kSortItems];
#pragma unroll
    for (int i = 0; i < kSortItems; ++i) k[i] = kin[min(tile * kSortTile + i * kSortThreads + t, count - 1)];
    uint32_t* h = s_h + (lane_id() & 3u) * kCopy;
#pragma unroll
    for (int i = 0; i < kSortItems; ++i) {
        const bool ok = tile * kSortTile + i * kSortThreads + t < count;
        const uint32_t d = digit_at(k[i], shift, bits);
        // neighbouring entries mostly share a digit: then one add per wave
        const uint32_t d0 = __builtin_amdgcn_readfirstlane(d);
        const uint64_t act = ballot64(ok);
        if (ballot64(ok && d != d0) == 0) {
            if (lane_id() == 0 && act) atomicAdd(&s_h[d0], (uint32_t)__popcll(act));
        } else if (ok) {
            atomicAdd(&h[d], 1u);
        }
    }
    __syncthreads();
#pragma unroll
    for (uint32_t d = t; d < (uint32_t)kTileRadix; d += kSortThreads)
        tcount[(size_t)d * stride + tile] = s_h[d] + s_h[kCopy + d] + s_h[2 * kCopy + d] + s_h[3 * kCopy + d];
}

__global__ void __launch_bounds__(256) tile_scan_kernel(uint32_t* __restrict__ tcount, uint32_t stride,
                                                        const uint32_t* __restrict__ count_p, uint64_t capacity,
                                                        uint32_t* __restrict__ hist) {
    __shared__ uint32_t s_tmp[4];
    constexpr uint32_t kItems = 16;   // consecutive sort tiles per thread and chunk
    const uint32_t count = *count_p;
    if ((uint64_t)count > capacity) return;
    const uint32_t ntiles = (count + kSortTile - 1) / kSortTile;
    uint32_t* row = tcount + (size_t)blockIdx.x * stride;
    uint32_t carry = 0;
    for (uint32_t c0 = 0; c0 < ntiles; c0 += 256 * kItems) {
        const uint32_t i0 = c0 + threadIdx.x * kItems;
        uint32_t x[kItems], sum = 0;
#pragma unroll
        for (uint32_t q = 0; q < kItems; ++q) {
            x[q] = i0 + q < ntiles ? row[i0 + q] : 0u;
            sum += x[q];
        }
        uint32_t total;
        uint32_t run = carry + block_exclusive_scan(sum, s_tmp, total);
#pragma unroll
        for (uint32_t q = 0; q < kItems; ++q) {
            if (i0 + q < ntiles) row[i0 + q] = run;
            run += x[q];
        }
        carry += total;
    }
    if (threadIdx.x == 0) hist[blockIdx.x] = carry;   // this digit's count over all entries
}

// BITS: the pass's digit width, a compile-time constant (the ballot chain then carries no
// per-bit condition). Positions past the last entry (the final sort tile only) carry the
// all-ones key, whose digit is the largest, so they sort behind every entry of the tile
// and no step needs a per-item validity mask; only positions below n_here are written.
template <int BITS>
__global__ void __launch_bounds__(kSortThreads) sort_scatter_kernel(
    const uint32_t* __restrict__ kin, const uint32_t* __restrict__ vin, const uint32_t* __restrict__ zin,
    uint32_t* __restrict__ kout, uint32_t* __restrict__ vout, uint32_t* __restrict__ zout,
    const uint32_t* __restrict__ count_p, uint64_t capacity, int shift,
    const uint32_t* __restrict__ hist, const uint32_t* __restrict__ tcount, uint32_t stride) {
    __shared__ uint32_t s_buf[kSortTile];   // tile reordered by digit: keys, values, depth bits
    __shared__ uint16_t s_dig[kSortTile];    // digit at each reordered position
    __shared__ uint32_t s_wcnt[4][kTileRadix];
    __shared__ uint32_t s_local[kTileRadix];
    __shared__ uint32_t s_base[kTileRadix];
    __shared__ uint32_t s_tmp[4];

    const uint32_t count = *count_p;
    if ((uint64_t)count > capacity) return;
    const uint32_t n_tiles = (count + kSortTile - 1) / kSortTile;
    if (blockIdx.x >= n_tiles) return;
    const uint32_t tile = xcd_swizzle(blockIdx.x, n_tiles);
    const uint32_t t = threadIdx.x, w = t >> 6, lane = t & 63;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        s_wcnt[k][t] = 0u;
        s_wcnt[k][t + 256] = 0u;
    }
    __syncthreads();

    // load: wave w owns entries [tile*4096 + w*1024, +1024), item i of lane l at i*64 + l
    const uint32_t wbase = tile * kSortTile + w * (kSortTile / 4);
    const uint32_t n_here = min((uint32_t)kSortTile, count - tile * kSortTile);
    uint32_t k[kSortItems], v[kSortItems], rk[kSortItems];
#pragma unroll
    for (int i = 0; i < kSortItems; ++i) {
        const uint32_t idx = wbase + i * kWave + lane;
        k[i] = idx < count ? kin[idx] : 0xFFFFFFFFu;
    }
    // this tile's start of digits 2t, 2t+1: digit base over all entries + earlier tiles' count
    const uint32_t h0 = hist[2 * t], h1 = hist[2 * t + 1];
    const uint32_t e0 = tcount[(size_t)(2 * t) * stride + tile], e1 = tcount[(size_t)(2 * t + 1) * stride + tile];
    wave_rank<kSortItems, BITS>(k, shift, BITS, 0xFFFFFFFFu, kSortItems, s_wcnt[w], rk);
    // values are needed only after the keys are placed: their loads overlap the scans
#pragma unroll
    for (int i = 0; i < kSortItems; ++i) v[i] = vin[min(wbase + i * kWave + lane, count - 1)];
    __syncthreads();

    uint32_t mine[2];
#pragma unroll
    for (int h = 0; h < 2; ++h) {
        const uint32_t d = 2 * t + h;
        const uint32_t c0 = s_wcnt[0][d], c1 = s_wcnt[1][d], c2 = s_wcnt[2][d], c3 = s_wcnt[3][d];
        mine[h] = c0 + c1 + c2 + c3;
        s_wcnt[0][d] = 0u;
        s_wcnt[1][d] = c0;
        s_wcnt[2][d] = c0 + c1;
        s_wcnt[3][d] = c0 + c1 + c2;
    }
    uint32_t tot;
    const uint32_t gbase = block_exclusive_scan(h0 + h1, s_tmp, tot);
    const uint32_t lbase = block_exclusive_scan(mine[0] + mine[1], s_tmp, tot);
    s_base[2 * t] = gbase + e0;
    s_base[2 * t + 1] = gbase + h0 + e1;
    s_local[2 * t] = lbase;
    s_local[2 * t + 1] = lbase + mine[0];
    __syncthreads();

    // reorder in LDS by digit (stable), then write runs: keys first, then the values and
    // the depth bits through the same buffer
    uint32_t lpos[kSortItems];
#pragma unroll
    for (int i = 0; i < kSortItems; ++i) {
        const uint32_t d = digit_at(k[i], shift, BITS);
        lpos[i] = s_local[d] + s_wcnt[w][d] + rk[i];
        s_buf[lpos[i]] = k[i];
    }
    __syncthreads();
#pragma unroll
    for (int i = 0; i < kSortItems; ++i) {
        const uint32_t j = t + i * kSortThreads;
        if (j < n_here) {
            const uint32_t key = s_buf[j];
            const uint32_t dd = digit_at(key, shift, BITS);
            s_dig[j] = (uint16_t)dd;
            const uint32_t dst = s_base[dd] + (j - s_local[dd]);
            if (dst < count) kout[dst] = key;
        }
    }
    __syncthreads();
#pragma unroll
    for (int i = 0; i < kSortItems; ++i) s_buf[lpos[i]] = v[i];
    __syncthreads();
#pragma unroll
    for (int i = 0; i < kSortItems; ++i) {
        const uint32_t j = t + i * kSortThreads;
        if (j < n_here) {
            const uint32_t dd = s_dig[j];
            const uint32_t dst = s_base[dd] + (j - s_local[dd]);
            if (dst < count) vout[dst] = s_buf[j];
        }
    }
    // the depth bits follow the same path (loaded late to keep registers free)
#pragma unroll
    for (int i = 0; i < kSortItems; ++i) v[i] = zin[min(wbase + i * kWave + lane, count - 1)];
    __syncthreads();
#pragma unroll
    for (int i = 0; i < kSortItems; ++i) s_buf[lpos[i]] = v[i];
    __syncthreads();
#pragma unroll
    for (int i = 0; i < kSortItems; ++i) {
        const uint32_t j = t + i * kSortThreads;
        if (j < n_here) {
            const uint32_t dd = s_dig[j];
            const uint32_t dst = s_base[dd] + (j - s_local[dd]);
            if (dst < count) zout[dst] = s_buf[j];
        }
    }
}

// Step 5: tile ranges from the sorted tile ids, four consecutive entries per thread (one
// 16-byte load; the workspace and its sections are 256-byte aligned) and the two
// neighbours of the run.
__global__ void __launch_bounds__(256) finalize_kernel(const uint32_t* __restrict__ keys,
                                                       const uint32_t* __restrict__ count_p, uint64_t capacity,
                                                       uint32_t tiles_total, uint32_t* __restrict__ ranges) {
    const uint32_t count = *count_p;
    if ((uint64_t)count > capacity) return;
    const uint32_t groups = (count + 3) / 4;
    for (uint32_t g = blockIdx.x * blockDim.x + threadIdx.x; g < groups; g += gridDim.x * blockDim.x) {
        const uint32_t i0 = 4 * g;
        uint32_t k[6];   // ids of entries i0 - 1 .. i0 + 4; none past the ends (all ones)
        k[0] = i0 > 0 ? keys[i0 - 1] : 0xFFFFFFFFu;
        if (i0 + 4 <= count) {
            const uint4 q = *reinterpret_cast<const uint4*>(keys + i0);
            k[1] = q.x;
            k[2] = q.y;
            k[3] = q.z;
            k[4] = q.w;
        } else {
#pragma unroll
            for (uint32_t j = 0; j < 4; ++j) k[1 + j] = i0 + j < count ? keys[i0 + j] : 0xFFFFFFFFu;
        }
        k[5] = i0 + 4 < count ? keys[i0 + 4] : 0xFFFFFFFFu;
#pragma unroll
        for (uint32_t j = 0; j < 4; ++j) {
            const uint32_t i = i0 + j, tl = k[1 + j];
            if (i < count && tl < tiles_total) {
                if (tl != k[j]) ranges[2 * tl] = i;
                if (tl != k[j + 2]) ranges[2 * tl + 1] = i + 1;
            }
        }
    }
}

// OR and AND of x over the workgroup (s_tmp: 2 * kBigWaves words). Contains __syncthreads.
__device__ __forceinline__ void block_or_and(uint32_t x_or, uint32_t x_and, uint32_t* s_tmp, uint32_t& r_or,
                                             uint32_t& r_and) {
#pragma unroll
    for (int o = 1; o < kWave; o <<= 1) {
        x_or |= __shfl_xor(x_or, o, kWave);
        x_and &= __shfl_xor(x_and, o, kWave);
    }
    const uint32_t w = threadIdx.x >> 6;
    if (lane_id() == 0) {
        s_tmp[w] = x_or;
        s_tmp[kBigWaves + w] = x_and;
    }
    __syncthreads();
    r_or = 0u;
    r_and = 0xFFFFFFFFu;
#pragma unroll
    for (int j = 0; j < kBigWaves; ++j) {
        r_or |= s_tmp[j];
        r_and &= s_tmp[kBigWaves + j];
    }
    __syncthreads();
}

struct SegShared {
    uint32_t buf[kSegMax];                      // segments reordered by digit: keys, then values
    uint32_t wcnt[kBigWaves][kRadix];
    uint32_t local[kBigWaves / 2][kRadix];      // group path: each group's digit bases; global
                                                // path: digit histogram [0], next output position [1]
    uint32_t tmp[2 * kBigWaves];
};

__device__ __forceinline__ void zero_wcnt(SegShared& sh, uint32_t t) {
#pragma unroll
    for (int q = 0; q < kBigWaves * kRadix / kBigThreads; ++q) (&sh.wcnt[0][0])[q * kBigThreads + t] = 0u;
}

// Digit d (< kRadix): wave prefixes written back into wcnt, returns the total over waves.
__device__ __forceinline__ uint32_t digit_wave_prefix(SegShared& sh, uint32_t d) {
    uint32_t run = 0;
#pragma unroll
    for (int q = 0; q < kBigWaves; ++q) {
        const uint32_t c = sh.wcnt[q][d];
        sh.wcnt[q][d] = run;
        run += c;
    }
    return run;
}

// Segments of up to 512 G entries sorted in LDS by groups of G waves (G = 2, 4 or 8, the
// same for the whole workgroup): the workgroup sorts kBigWaves / G segments side by side,
// group g (waves gG .. gG + G - 1) the segment (tile, start, n) that its threads pass
// (n = 0: none), so that the barriers and latencies of a pass are shared by several
// segments. Items stay in registers between passes; each pass ranks by one 8-bit digit of
// the depth bits within each wave (ballots), turns the group's digit counts into bases,
// reorders the keys and then the values through the group's part of LDS and reloads them
// in position order. Only the bits that differ within a segment are sorted on. Positions
// past the segment's end, up to the group's whole rounds, carry the key with all bits set:
// its digit is the largest of every pass and those positions come after every entry, so
// stability keeps them at the end and no pass needs a per-item validity mask. G is a
// parameter rather than a template argument so that the kernel holds one copy of this
// code (three copies take more registers than the kernel may use).
__device__ __forceinline__ void segment_sort_groups(SegShared& sh, uint32_t G, uint32_t tile, uint32_t start,
                                                    uint32_t n, const uint32_t* __restrict__ zs,
                                                    uint32_t* __restrict__ pidx, uint64_t* __restrict__ keys64) {
    static_assert(kBigWaves == 8 && kRadix == 256 && kBigItems * kWave * kBigWaves == (int)kSegMax, "group layout");
    // the segment is the same for every lane of a wave, G for the whole workgroup: scalars
    G = __builtin_amdgcn_readfirstlane(G);
    tile = __builtin_amdgcn_readfirstlane(tile);
    start = __builtin_amdgcn_readfirstlane(start);
    n = __builtin_amdgcn_readfirstlane(n);
    const uint32_t t = threadIdx.x, w = __builtin_amdgcn_readfirstlane(t >> 6), l = lane_id();
    const uint32_t group_threads = kWave * G;
    const uint32_t g = w / G, g0 = g * G, tg = t - g * group_threads;
    uint32_t* buf = sh.buf + g * group_threads * kBigItems;
    const int items = (int)((n + group_threads - 1) / group_threads);   // uniform within the group
    const uint32_t wbase = (w - g0) * kWave * (uint32_t)items;          // this wave's first position
    uint32_t k[kBigItems], v[kBigItems], rk[kBigItems];
    uint32_t k_or = 0u, k_and = 0xFFFFFFFFu;
    if (n) {
        // loads clamped into the segment rather than predicated, so that all of them are in
        // flight at once
#pragma unroll
        for (int i = 0; i < kBigItems; ++i) {
            const uint32_t p = min(wbase + (uint32_t)i * kWave + l, n - 1);
            v[i] = pidx[start + p];
            k[i] = zs[start + p];
        }
    }
#pragma unroll
    for (int i = 0; i < kBigItems; ++i) {
        const bool ok = i < items && wbase + (uint32_t)i * kWave + l < n;
        k_or |= ok ? k[i] : 0u;
        k_and &= ok ? k[i] : 0xFFFFFFFFu;
        k[i] = ok ? k[i] : 0xFFFFFFFFu;
    }
#pragma unroll
    for (int o = 1; o < kWave; o <<= 1) {
        k_or |= __shfl_xor(k_or, o, kWave);
        k_and &= __shfl_xor(k_and, o, kWave);
    }
    if (l == 0) {
        sh.tmp[w] = k_or;
        sh.tmp[kBigWaves + w] = k_and;
    }
    __syncthreads();
    // the differing bits of every group (its waves' OR and AND; an empty group has OR 0 and
    // AND all ones: no differing bit): this group's first bit, the most passes of any group
    int lo = 0, passes = 0;
    {
        uint32_t a_or = 0u, a_and = 0xFFFFFFFFu;
#pragma unroll
        for (uint32_t q = 0; q < (uint32_t)kBigWaves; ++q) {
            a_or |= sh.tmp[q];
            a_and &= sh.tmp[kBigWaves + q];
            if (((q + 1) & (G - 1)) == 0) {   // q is the last wave of group q / G
                const uint32_t diff = a_or & ~a_and;
                const int glo = diff ? __builtin_ctz(diff) : 0;
                const int ghi = diff ? 32 - __builtin_clz(diff) : 0;
                passes = max(passes, (ghi - glo + kRadixBits - 1) / kRadixBits);
                if (q / G == g) lo = glo;
                a_or = 0u;
                a_and = 0xFFFFFFFFu;
            }
        }
    }
    lo = __builtin_amdgcn_readfirstlane(lo);
    passes = __builtin_amdgcn_readfirstlane(passes);
    // digits of this thread in the group's scan: 2 tg, 2 tg + 1 for G = 2, tg otherwise
    const uint32_t nd = G == 2 ? 2u : 1u, d0 = tg * nd;
    // Every group makes the most passes any group needs, pass p on bits [min(lo + 8 p, 24),
    // +8). A group's extra passes rank bits above its differing ones (equal within the
    // segment) or its most significant differing bits again: stable passes over keys
    // already in that order, which change nothing. Where the clamp makes a group's own last
    // pass overlap the one before, the stable LSD order is still the sorted one.
    for (int pass = 0; pass < passes; ++pass) {
        const int shift = min(lo + pass * kRadixBits, 32 - kRadixBits);
        // each wave clears its own counters: LDS operations of one wave complete in order
#pragma unroll
        for (int q = 0; q < kRadix / kWave; ++q) sh.wcnt[w][q * kWave + l] = 0u;
        wave_rank<kBigItems>(k, shift, kRadixBits, 0xFFFFFFFFu, items, sh.wcnt[w], rk);
        __syncthreads();
        // this thread's digits: prefixes over the group's waves, the group's totals
        uint32_t tot[2], mine = 0u;
#pragma unroll
        for (uint32_t j = 0; j < 2; ++j) {
            const uint32_t d = d0 + j;
            uint32_t run = 0u;
            if (j < nd && d < (uint32_t)kRadix) {
#pragma unroll
                for (uint32_t q = 0; q < (uint32_t)kBigWaves; ++q) {
                    if (q < G) {
                        const uint32_t c = sh.wcnt[g0 + q][d];
                        sh.wcnt[g0 + q][d] = run;
                        run += c;
                    }
                }
            }
            tot[j] = run;
            mine += run;
        }
        // exclusive scan of the totals over the group's threads (digit order)
        const uint32_t inc = wave_inclusive_scan(mine);
        if (l == kWave - 1) sh.tmp[w] = inc;
        __syncthreads();
        uint32_t base = inc - mine;
#pragma unroll
        for (uint32_t q = 0; q < (uint32_t)kBigWaves; ++q) base += (g0 + q < w) ? sh.tmp[g0 + q] : 0u;
#pragma unroll
        for (uint32_t j = 0; j < 2; ++j) {
            const uint32_t d = d0 + j;
            if (j < nd && d < (uint32_t)kRadix) sh.local[g][d] = base;
            base += tot[j];
        }
        __syncthreads();
        uint32_t pos[kBigItems];
#pragma unroll
        for (int i = 0; i < kBigItems; ++i) {
            if (i < items) {
                const uint32_t d = digit_at(k[i], shift, kRadixBits);
                pos[i] = sh.local[g][d] + sh.wcnt[w][d] + rk[i];
                buf[pos[i]] = k[i];
            }
        }
        __syncthreads();
#pragma unroll
        for (int i = 0; i < kBigItems; ++i)
            if (i < items) k[i] = buf[wbase + (uint32_t)i * kWave + l];
        __syncthreads();
#pragma unroll
        for (int i = 0; i < kBigItems; ++i)
            if (i < items) buf[pos[i]] = v[i];
        __syncthreads();
#pragma unroll
        for (int i = 0; i < kBigItems; ++i)
            if (i < items) v[i] = buf[wbase + (uint32_t)i * kWave + l];
    }
    // every read of the segment happened before the first barrier: in place is safe
#pragma unroll
    for (int i = 0; i < kBigItems; ++i) {
        const uint32_t p = wbase + (uint32_t)i * kWave + l;
        if (i >= items || p >= n) continue;
        if (passes) pidx[start + p] = v[i];
        if (keys64) keys64[start + p] = ((uint64_t)tile << 32) | k[i];
    }
}

// Segment longer than kSegMax, sorted by one workgroup through global scratch. A first
// sweep copies (depth bits, particle index) to (sk0, sv) and reduces the differing bits;
// each pass then scatters chunk after chunk straight to its place, counting the next
// pass's digits on the way. Every sweep issues kBigItems independent loads per thread.
__device__ __forceinline__ void segment_sort_global(SegShared& sh, uint32_t tile, uint32_t start, uint32_t n,
                                                    const uint32_t* __restrict__ zs, uint32_t* __restrict__ pidx,
                                                    uint64_t* __restrict__ keys64, uint32_t* __restrict__ sk0,
                                                    uint32_t* __restrict__ sk1, uint32_t* __restrict__ sv) {
    const uint32_t t = threadIdx.x, w = t >> 6, l = lane_id();
    uint32_t k_or = 0u, k_and = 0xFFFFFFFFu;
    for (uint32_t c0 = 0; c0 < n; c0 += kSegMax) {
        uint32_t g[kBigItems], key[kBigItems];
#pragma unroll
        for (int i = 0; i < kBigItems; ++i) {
            const uint32_t pc = min(c0 + (uint32_t)i * kBigThreads + t, n - 1);
            g[i] = pidx[start + pc];
            key[i] = zs[start + pc];
        }
#pragma unroll
        for (int i = 0; i < kBigItems; ++i) {
            const uint32_t p = c0 + (uint32_t)i * kBigThreads + t;
            if (p < n) {
                sk0[start + p] = key[i];
                sv[start + p] = g[i];
                k_or |= key[i];
                k_and &= key[i];
            }
        }
    }
    uint32_t all_or, all_and;
    block_or_and(k_or, k_and, sh.tmp, all_or, all_and);   // also orders the sweep's writes
    const uint32_t diff = all_or ^ all_and;
    // uniform by construction; readfirstlane tells the compiler, so the digit loops branch
    // on scalars
    const int lo = __builtin_amdgcn_readfirstlane(diff ? __builtin_ctz(diff) : 0);
    const int hi = __builtin_amdgcn_readfirstlane(diff ? 32 - __builtin_clz(diff) : 0);
    const Split8 split(lo, hi);
    const int passes = split.passes;
    uint32_t *src_k = sk0, *src_v = sv, *dst_k = sk1, *dst_v = pidx;
    if (passes > 0) {
        // digit histogram of the first pass
        if (t < kRadix) sh.local[0][t] = 0u;
        __syncthreads();
        for (uint32_t c0 = 0; c0 < n; c0 += kSegMax) {
            uint32_t kk[kBigItems];
#pragma unroll
            for (int i = 0; i < kBigItems; ++i) kk[i] = src_k[start + min(c0 + (uint32_t)i * kBigThreads + t, n - 1)];
#pragma unroll
            for (int i = 0; i < kBigItems; ++i)
                if (c0 + (uint32_t)i * kBigThreads + t < n) atomicAdd(&sh.local[0][digit_at(kk[i], split.shift(0), kRadixBits)], 1u);
        }
        __syncthreads();
    }
    for (int pass = 0; pass < passes; ++pass) {
        const int shift = split.shift(pass), bits = kRadixBits;
        const bool has_next = pass + 1 < passes;
        const int next_shift = has_next ? split.shift(pass + 1) : 0, next_bits = kRadixBits;
        uint32_t all;
        const uint32_t h = t < kRadix ? sh.local[0][t] : 0u;
        const uint32_t rb = block_exclusive_scan<kBigWaves>(h, sh.tmp, all);
        if (t < kRadix) {
            sh.local[1][t] = rb;
            sh.local[0][t] = 0u;   // now the next pass's histogram
        }
        for (uint32_t c0 = 0; c0 < n; c0 += kSegMax) {
            const uint32_t cn = min(kSegMax, n - c0);
            const int items = (int)((cn + kBigThreads - 1) / kBigThreads);
            const uint32_t wbase = c0 + w * kWave * (uint32_t)items;
            zero_wcnt(sh, t);
            __syncthreads();
            uint32_t k[kBigItems], v[kBigItems], rk[kBigItems];
            uint32_t valid = 0;
#pragma unroll
            for (int i = 0; i < kBigItems; ++i) {
                const uint32_t p = wbase + (uint32_t)i * kWave + l;
                valid |= (uint32_t)(i < items && p < c0 + cn) << i;
                const uint32_t pc = min(p, n - 1);
                k[i] = src_k[start + pc];
                v[i] = src_v[start + pc];
            }
            wave_rank<kBigItems>(k, shift, bits, valid, items, sh.wcnt[w], rk);
            __syncthreads();
            const uint32_t tot = t < kRadix ? digit_wave_prefix(sh, t) : 0u;
            __syncthreads();
#pragma unroll
            for (int i = 0; i < kBigItems; ++i) {
                if (!((valid >> i) & 1u)) continue;
                const uint32_t d = digit_at(k[i], shift, bits);
                const uint32_t o = sh.local[1][d] + sh.wcnt[w][d] + rk[i];
                dst_k[start + o] = k[i];
                dst_v[start + o] = v[i];
                if (has_next) atomicAdd(&sh.local[0][digit_at(k[i], next_shift, next_bits)], 1u);
            }
            __syncthreads();
            if (t < kRadix) sh.local[1][t] += tot;
        }
        __syncthreads();
        uint32_t* tk = src_k;
        uint32_t* tv = src_v;
        src_k = dst_k;
        src_v = dst_v;
        dst_k = tk;
        dst_v = tv;
    }
    // sorted data in (src_k, src_v): (sk1, pidx) after an odd pass count, else (sk0, sv)
    const bool in_place = src_v == pidx;
    if (!in_place && passes == 0 && !keys64) return;   // order unchanged, pidx untouched
    for (uint32_t c0 = 0; c0 < n; c0 += kSegMax) {
#pragma unroll
        for (int i = 0; i < kBigItems; ++i) {
            const uint32_t p = c0 + (uint32_t)i * kBigThreads + t;
            if (p >= n) continue;
            if (!in_place) pidx[start + p] = src_v[start + p];
            if (keys64) keys64[start + p] = ((uint64_t)tile << 32) | src_k[start + p];
        }
    }
}

// Wave-level segment sort, for segments of up to kWaveSegMax entries: one wave per tile,
// items in registers (item i of lane l at position 64 i + l), each pass ranks by one 8-bit
// digit with ballots, turns the wave's 256 digit counts into bases with a wave scan and
// reorders through the wave's own LDS region. No workgroup barrier is involved: LDS
// operations of one wave complete in order.
constexpr int kWaveItems = 8;
constexpr uint32_t kWaveSegMax = kWave * kWaveItems;

struct WaveSegShared {
    uint32_t buf[4][kWaveSegMax];
    uint32_t cnt[4][kRadix];
};

__device__ __forceinline__ void wave_sort_segment(uint32_t* __restrict__ buf, uint32_t* __restrict__ cnt,
                                                  uint32_t tile, uint32_t start, uint32_t n,
                                                  const uint32_t* __restrict__ zs, uint32_t* __restrict__ pidx,
                                                  uint64_t* __restrict__ keys64) {
    const uint32_t l = lane_id();
    const int items = (int)((n + kWave - 1) / kWave);
    uint32_t k[kWaveItems], v[kWaveItems], rk[kWaveItems], pos[kWaveItems];
    uint32_t valid = 0, k_or = 0u, k_and = 0xFFFFFFFFu;
    // loads clamped into the segment rather than predicated, so that all of them are in
    // flight at once
#pragma unroll
    for (int i = 0; i < kWaveItems; ++i) {
        const uint32_t p = (uint32_t)i * kWave + l;
        valid |= (uint32_t)(i < items && p < n) << i;
        v[i] = pidx[start + min(p, n - 1)];
        k[i] = zs[start + min(p, n - 1)];
    }
#pragma unroll
    for (int i = 0; i < kWaveItems; ++i) {
        const bool ok = (valid >> i) & 1u;
        k_or |= ok ? k[i] : 0u;
        k_and &= ok ? k[i] : 0xFFFFFFFFu;
    }
#pragma unroll
    for (int o = 1; o < kWave; o <<= 1) {
        k_or |= __shfl_xor(k_or, o, kWave);
        k_and &= __shfl_xor(k_and, o, kWave);
    }
    const uint32_t diff = k_or ^ k_and;
    if (n <= kWave && diff) {
        // one entry per lane: the rank is the number of smaller keys plus the number of
        // equal keys at lower positions (about four instructions per entry)
        const uint32_t key = k[0];
        uint32_t rank = 0;
        for (uint32_t j = 0; j < n; ++j) {
            const uint32_t kj = __builtin_amdgcn_readlane(key, (int)j);
            rank += (kj < key || (kj == key && j < l)) ? 1u : 0u;
        }
        if (valid & 1u) {
            pidx[start + rank] = v[0];
            if (keys64) keys64[start + rank] = ((uint64_t)tile << 32) | key;
        }
        return;
    }
    // uniform by construction; readfirstlane tells the compiler, so the digit loops branch
    // on scalars
    const int lo = __builtin_amdgcn_readfirstlane(diff ? __builtin_ctz(diff) : 0);
    const int hi = __builtin_amdgcn_readfirstlane(diff ? 32 - __builtin_clz(diff) : 0);
    const Split8 split(lo, hi);
    for (int pass = 0; pass < split.passes; ++pass) {
        const int shift = split.shift(pass), bits = kRadixBits;
#pragma unroll
        for (int q = 0; q < 4; ++q) cnt[4 * l + q] = 0u;
        __builtin_amdgcn_wave_barrier();
        wave_rank<kWaveItems>(k, shift, bits, valid, items, cnt, rk);
        __builtin_amdgcn_wave_barrier();
        // lane l owns digits 4l .. 4l+3: counts -> exclusive bases
        const uint32_t c0 = cnt[4 * l], c1 = cnt[4 * l + 1], c2 = cnt[4 * l + 2], c3 = cnt[4 * l + 3];
        const uint32_t sum = c0 + c1 + c2 + c3;
        const uint32_t ex = wave_inclusive_scan(sum) - sum;
        __builtin_amdgcn_wave_barrier();
        cnt[4 * l] = ex;
        cnt[4 * l + 1] = ex + c0;
        cnt[4 * l + 2] = ex + c0 + c1;
        cnt[4 * l + 3] = ex + c0 + c1 + c2;
        __builtin_amdgcn_wave_barrier();
#pragma unroll
        for (int i = 0; i < kWaveItems; ++i) {
            if ((valid >> i) & 1u) {
                pos[i] = cnt[digit_at(k[i], shift, bits)] + rk[i];
                buf[pos[i]] = k[i];
            }
        }
        __builtin_amdgcn_wave_barrier();
#pragma unroll
        for (int i = 0; i < kWaveItems; ++i)
            if ((valid >> i) & 1u) k[i] = buf[(uint32_t)i * kWave + l];
        __builtin_amdgcn_wave_barrier();
#pragma unroll
        for (int i = 0; i < kWaveItems; ++i)
            if ((valid >> i) & 1u) buf[pos[i]] = v[i];
        __builtin_amdgcn_wave_barrier();
#pragma unroll
        for (int i = 0; i < kWaveItems; ++i)
            if ((valid >> i) & 1u) v[i] = buf[(uint32_t)i * kWave + l];
        __builtin_amdgcn_wave_barrier();
    }
#pragma unroll
    for (int i = 0; i < kWaveItems; ++i) {
        if (!((valid >> i) & 1u)) continue;
        const uint32_t p = (uint32_t)i * kWave + l;
        if (hi > lo) pidx[start + p] = v[i];
        if (keys64) keys64[start + p] = ((uint64_t)tile << 32) | k[i];
    }
}

// The long segments are listed for step 6b by size class: class 0 up to kSegMax entries
// (sorted by a whole workgroup), class 1 up to kSegMax / 2 (two at once), class 2 up to
// kSegMax / 4 (four at once). Each class has kLongLists lists, tile t in list t mod
// kLongLists, each with its own counter on its own 128-byte line: appends to one
// device-wide counter are serialised in memory (the XCDs' L2s are not coherent), while
// appends to different lines proceed in parallel. List j of class c is list c kLongLists + j
// at (c kLongLists + j) * per words.
constexpr uint32_t kLongLists = 64;
constexpr uint32_t kClasses = 3;
constexpr uint32_t kClassLists = kClasses * kLongLists;
constexpr uint32_t kLongCounterStride = 32;   // words: one counter per 128-byte line
// Segments longer than kSegMax (sorted through the workspace, several times the work of
// the others) go to one more list, at kClassLists * per words, counted in counter slot
// kHugeSlot; slot kWorkSlot is the work counter of step 6b. Segments longer than kChunkMin
// are sorted by all workgroups together (step 6c): they are listed after that, at
// kClassLists * per + tiles words, counted in slot kChunkSlot; slot kChunkTotalSlot receives
// their number of 4096-entry chunks.
constexpr uint32_t kHugeSlot = kClassLists, kWorkSlot = kClassLists + 1, kChunkSlot = kClassLists + 2,
                   kChunkTotalSlot = kClassLists + 3, kLongCounters = kClassLists + 4;
constexpr uint32_t kChunkMin = 16384;

// Size class of a segment of kWaveSegMax < n <= kSegMax entries.
__device__ __forceinline__ uint32_t seg_class(uint32_t n) {
    return n > kSegMax / 2 ? 0u : n > kSegMax / 4 ? 1u : 2u;
}

// Step 6a: one wave per tile sorts segments of up to kWaveSegMax entries and appends the
// longer ones to the lists for step 6b.
__global__ void __launch_bounds__(kSortThreads) segment_sort_small_kernel(
    const uint32_t* __restrict__ ranges, uint32_t tiles_total, const uint32_t* __restrict__ zs,
    uint32_t* __restrict__ pidx, uint64_t* __restrict__ keys64, const uint32_t* __restrict__ count_p,
    uint64_t capacity, const int32_t* __restrict__ status, uint32_t* __restrict__ long_lists,
    uint32_t* __restrict__ long_counts) {
    __shared__ WaveSegShared sh;
    if (*status != kStatusOk) return;
    if ((uint64_t)*count_p > capacity) return;
    const uint32_t w = threadIdx.x >> 6;
    const uint32_t tile = 4 * xcd_swizzle(blockIdx.x, gridDim.x) + w;
    if (tile >= tiles_total) return;
    const uint32_t start = ranges[2 * tile], end = ranges[2 * tile + 1];
    if (end <= start) return;
    const uint32_t n = end - start;
    if (n > kWaveSegMax) {
        if (lane_id() == 0) {
            const uint32_t per = (tiles_total + kLongLists - 1) / kLongLists;
            if (n > kChunkMin) {
                long_lists[kClassLists * per + tiles_total +
                           atomicAdd(&long_counts[kChunkSlot * kLongCounterStride], 1u)] = tile;
            } else {
                const uint32_t j = n > kSegMax ? kHugeSlot : seg_class(n) * kLongLists + tile % kLongLists;
                long_lists[j * per + atomicAdd(&long_counts[j * kLongCounterStride], 1u)] = tile;
            }
        }
        return;
    }
    wave_sort_segment(sh.buf[w], sh.cnt[w], tile, start, n, zs, pidx, keys64);
}

// Tile of item r of class c: list j holds the class's items [first[j], first[j + 1]), so j
// is the number of lists that end at or before r (one ballot of the wave).
__device__ __forceinline__ uint32_t class_item(const uint32_t* __restrict__ long_lists, uint32_t per, uint32_t c,
                                               const uint32_t* first, uint32_t r) {
    const uint32_t j = (uint32_t)__popcll(ballot64(first[lane_id() + 1] <= r));
    return long_lists[(c * kLongLists + j) * per + (r - first[j])];
}

// Step 6b: a resident grid sorts the listed long segments, with stable LSD radix passes: in
// LDS up to kSegMax entries, through the workspace beyond. Workgroups take the next item
// from a device-wide counter (one atomic per item: a few thousand per call, against tens of
// microseconds of work each), the longest segments first, so that no workgroup is left with
// a run of long ones while the others have finished: the segments sorted through the
// workspace, then class 0 one per item, class 1 two per item, class 2 four per item. The
// sort is bound by its ballot chains and the latency of its barriers, not by bytes, so the
// kernel is held to 80 VGPRs: three workgroups per CU (at 64 the group sort spills to
// scratch memory, without a limit two workgroups fit).
__global__ void __launch_bounds__(kBigThreads) __attribute__((amdgpu_waves_per_eu(6))) segment_sort_big_kernel(
    const uint32_t* __restrict__ ranges, uint32_t tiles_total, const uint32_t* __restrict__ zs,
    uint32_t* __restrict__ pidx, uint64_t* __restrict__ keys64, const uint32_t* __restrict__ count_p,
    uint64_t capacity, const int32_t* __restrict__ status, const uint32_t* __restrict__ long_lists,
    uint32_t* __restrict__ long_counts, uint32_t* __restrict__ sk0, uint32_t* __restrict__ sk1,
    uint32_t* __restrict__ sv) {
    __shared__ SegShared sh;
    __shared__ uint32_t s_first[kClasses][kLongLists + 1];   // each list's first item within its class
    __shared__ uint32_t s_item;
    if (*status != kStatusOk) return;
    if ((uint64_t)*count_p > capacity) return;
    const uint32_t t = threadIdx.x;
    static_assert(kLongLists == kWave, "one lane per list");
    if (t < kClasses * kWave) {
        const uint32_t c = t / kWave, lane = lane_id();
        const uint32_t incl = wave_inclusive_scan(long_counts[(c * kLongLists + lane) * kLongCounterStride]);
        s_first[c][lane + 1] = incl;
        if (lane == 0) s_first[c][0] = 0u;
    }
    __syncthreads();
    const uint32_t per = (tiles_total + kLongLists - 1) / kLongLists;
    const uint32_t n_huge = long_counts[kHugeSlot * kLongCounterStride];
    const uint32_t n0 = s_first[0][kLongLists], n1 = s_first[1][kLongLists], n2 = s_first[2][kLongLists];
    const uint32_t e0 = n_huge + n0, e1 = e0 + (n1 + 1) / 2, total = e1 + (n2 + 3) / 4;
    uint32_t* work = long_counts + kWorkSlot * kLongCounterStride;
    const uint32_t w = t >> 6;
    for (;;) {
        if (t == 0) s_item = atomicAdd(work, 1u);
        __syncthreads();
        const uint32_t i = s_item;
        if (i >= total) break;   // uniform: every thread read the same item
        if (i < n_huge) {
            const uint32_t tile = long_lists[kHugeSlot * per + i];
            const uint32_t start = ranges[2 * tile], n = ranges[2 * tile + 1] - start;
            segment_sort_global(sh, tile, start, n, zs, pidx, keys64, sk0, sk1, sv);
        } else {
            // class 0: one segment per item (groups of 8 waves), class 1: two (4 waves each),
            // class 2: four (2 waves each)
            const uint32_t c = i < e0 ? 0u : i < e1 ? 1u : 2u;
            const uint32_t G = kBigWaves >> c;
            const uint32_t r = c == 0 ? i - n_huge : c == 1 ? 2 * (i - e0) + w / G : 4 * (i - e1) + w / G;
            const uint32_t nc = c == 0 ? n0 : c == 1 ? n1 : n2;
            uint32_t tile = 0, start = 0, n = 0;
            if (r < nc) {
                tile = class_item(long_lists, per, c, s_first[c], r);
                start = ranges[2 * tile];
                n = ranges[2 * tile + 1] - start;
            }
            segment_sort_groups(sh, G, tile, start, n, zs, pidx, keys64);
        }
        __syncthreads();   // also orders every read of s_item before the next write
    }
}

// Step 6c: the segments longer than kChunkMin, sorted by every workgroup together: each is
// cut into 4096-entry chunks and sorted by stable LSD passes over the four bytes of the
// depth bits, each pass as count (a digit histogram per chunk), scan (per segment: for each
// digit, the prefix over its chunks, placed after the smaller digits' entries) and scatter
// (each chunk ranks its entries per digit with ballots and writes them to their places,
// reordered in LDS into runs). A pass whose byte is the same for every entry of a segment
// would leave it unchanged: the scan marks it skipped and the segment stays where it is, so
// each segment keeps its own record of which buffer holds it. Buffers: A = (depth bits,
// pidx) as the tile passes left them, B = workspace. The grids are resident and stride over
// the chunks (or segments); with no long segment every kernel leaves at once.
struct ChunkPlan {
    uint32_t* seg_start;    // [h] first entry of segment s
    uint32_t* seg_n;        // [h] its length
    uint32_t* chunk_first;  // [h + 1] index of its first chunk
    uint32_t* seg_loc;      // [5][h] buffer holding segment s before pass p (0 = A, 1 = B)
    uint32_t* seg_tile;     // [h] its tile
    uint32_t* chunk_seg;    // [chunks] segment of each chunk
    uint32_t* cnt;          // [chunks][kRadix] digit counts, then output bases
    uint32_t h_max;
};

// One workgroup: the segment table, the chunk table and the chunk total.
__global__ void __launch_bounds__(256) chunk_setup_kernel(const uint32_t* __restrict__ ranges, uint32_t tiles_total,
                                                          const uint32_t* __restrict__ long_lists,
                                                          uint32_t* __restrict__ long_counts, ChunkPlan cp) {
    __shared__ uint32_t s_tmp[4];
    const uint32_t per = (tiles_total + kLongLists - 1) / kLongLists;
    const uint32_t h = min(long_counts[kChunkSlot * kLongCounterStride], cp.h_max);
    const uint32_t* list = long_lists + kClassLists * per + tiles_total;
    uint32_t carry = 0;
    for (uint32_t s0 = 0; s0 < h; s0 += 256) {
        const uint32_t sid = s0 + threadIdx.x;
        uint32_t start = 0, n = 0, tile = 0;
        if (sid < h) {
            tile = list[sid];
            start = ranges[2 * tile];
            n = ranges[2 * tile + 1] - start;
        }
        const uint32_t nch = (n + kSortTile - 1) / kSortTile;
        uint32_t total;
        const uint32_t first = carry + block_exclusive_scan(nch, s_tmp, total);
        if (sid < h) {
            cp.seg_start[sid] = start;
            cp.seg_n[sid] = n;
            cp.seg_tile[sid] = tile;
            cp.chunk_first[sid] = first;
            cp.seg_loc[sid] = 0u;
            for (uint32_t c = 0; c < nch; ++c) cp.chunk_seg[first + c] = sid;
        }
        carry += total;
    }
    if (threadIdx.x == 0) {
        cp.chunk_first[h] = carry;
        long_counts[kChunkTotalSlot * kLongCounterStride] = carry;
    }
}

__device__ __forceinline__ uint32_t chunk_count_of(const uint32_t* long_counts) {
    return long_counts[kChunkTotalSlot * kLongCounterStride];
}

// Entries [lo, hi) of chunk c, its segment and the buffer holding it before pass p.
struct ChunkSpan {
    uint32_t s, lo, hi, loc;
};

__device__ __forceinline__ ChunkSpan chunk_span(const ChunkPlan& cp, uint32_t c, int pass) {
    ChunkSpan r;
    r.s = cp.chunk_seg[c];
    const uint32_t start = cp.seg_start[r.s], end = start + cp.seg_n[r.s];
    r.lo = start + (c - cp.chunk_first[r.s]) * kSortTile;
    r.hi = min(r.lo + kSortTile, end);
    r.loc = cp.seg_loc[pass * cp.h_max + r.s];
    return r;
}

__global__ void __launch_bounds__(kSortThreads) chunk_count_kernel(const uint32_t* __restrict__ a_key,
                                                                   const uint32_t* __restrict__ b_key,
                                                                   const uint32_t* __restrict__ long_counts,
                                                                   ChunkPlan cp, int pass) {
    __shared__ uint32_t s_h[kRadix];
    const uint32_t nc = chunk_count_of(long_counts), t = threadIdx.x;
    const int shift = 8 * pass;
    for (uint32_t c = blockIdx.x; c < nc; c += gridDim.x) {
        const ChunkSpan sp = chunk_span(cp, c, pass);
        const uint32_t* key = sp.loc ? b_key : a_key;
        s_h[t] = 0u;
        // all of the chunk's loads in flight at once (clamped into the chunk), then the counts
        uint32_t k[kSortItems];
#pragma unroll
        for (int i = 0; i < kSortItems; ++i) k[i] = key[min(sp.lo + i * kSortThreads + t, sp.hi - 1)];
        __syncthreads();
#pragma unroll
        for (int i = 0; i < kSortItems; ++i) {
            if (sp.lo + i * kSortThreads + t >= sp.hi) continue;
            const uint32_t d = digit_at(k[i], shift, 8);
            // a byte shared by the whole wave (the leading bytes of close depths): one add
            const uint32_t d0 = __builtin_amdgcn_readfirstlane(d);
            const uint64_t act = ballot64(true);
            if (ballot64(d != d0) == 0) {
                if (lane_id() == (uint32_t)__builtin_ctzll(act)) atomicAdd(&s_h[d0], (uint32_t)__popcll(act));
            } else {
                atomicAdd(&s_h[d], 1u);
            }
        }
        __syncthreads();
        cp.cnt[(size_t)c * kRadix + t] = s_h[t];
        __syncthreads();
    }
}

// One segment per workgroup iteration, thread d for digit d.
__global__ void __launch_bounds__(256) chunk_scan_kernel(const uint32_t* __restrict__ long_counts, ChunkPlan cp,
                                                         int pass) {
    __shared__ uint32_t s_tmp[4];
    __shared__ uint32_t s_nz[4];
    static_assert(kRadix == 256, "one thread per digit");
    const uint32_t h = min(long_counts[kChunkSlot * kLongCounterStride], cp.h_max), d = threadIdx.x;
    for (uint32_t sid = blockIdx.x; sid < h; sid += gridDim.x) {
        const uint32_t c0 = cp.chunk_first[sid], c1 = cp.chunk_first[sid + 1];
        uint32_t run = 0;
        for (uint32_t c = c0; c < c1; ++c) {
            const uint32_t x = cp.cnt[(size_t)c * kRadix + d];
            cp.cnt[(size_t)c * kRadix + d] = run;
            run += x;
        }
        // a byte the same for every entry: the pass would not move anything
        const uint32_t nz = (uint32_t)__popcll(ballot64(run != 0u));
        if (lane_id() == 0) s_nz[d >> 6] = nz;
        uint32_t total;
        const uint32_t base = block_exclusive_scan(run, s_tmp, total) + cp.seg_start[sid];
        const bool skip = s_nz[0] + s_nz[1] + s_nz[2] + s_nz[3] <= 1u;
        const uint32_t loc = cp.seg_loc[pass * cp.h_max + sid];
        if (d == 0) cp.seg_loc[(pass + 1) * cp.h_max + sid] = skip ? loc : loc ^ 1u;
        if (!skip)
            for (uint32_t c = c0; c < c1; ++c) cp.cnt[(size_t)c * kRadix + d] += base;
        __syncthreads();   // s_nz and s_tmp are reused by the next segment
    }
}

__global__ void __launch_bounds__(kSortThreads) chunk_scatter_kernel(uint32_t* __restrict__ a_key,
                                                                     uint32_t* __restrict__ a_val,
                                                                     uint32_t* __restrict__ b_key,
                                                                     uint32_t* __restrict__ b_val,
                                                                     const uint32_t* __restrict__ long_counts,
                                                                     ChunkPlan cp, int pass) {
    __shared__ uint32_t s_buf[kSortTile];
    __shared__ uint32_t s_wcnt[4][kRadix];
    __shared__ uint32_t s_local[kRadix];
    __shared__ uint32_t s_base[kRadix];
    __shared__ uint32_t s_tmp[4];
    const uint32_t nc = chunk_count_of(long_counts), t = threadIdx.x, w = t >> 6, lane = t & 63;
    const int shift = 8 * pass;
    for (uint32_t c = blockIdx.x; c < nc; c += gridDim.x) {
        const ChunkSpan sp = chunk_span(cp, c, pass);
        const uint32_t loc_next = cp.seg_loc[(pass + 1) * cp.h_max + sp.s];
        if (loc_next == sp.loc) continue;   // skipped pass: uniform over the workgroup
        const uint32_t* skey = sp.loc ? b_key : a_key;
        const uint32_t* sval = sp.loc ? b_val : a_val;
        uint32_t* dkey = sp.loc ? a_key : b_key;
        uint32_t* dval = sp.loc ? a_val : b_val;
        const uint32_t n_here = sp.hi - sp.lo;
#pragma unroll
        for (int k = 0; k < 4; ++k) s_wcnt[k][t] = 0u;
        // wave w owns chunk positions [w * 1024, +1024), item i of lane l at i * 64 + l;
        // positions past the chunk's end carry the all-ones key (largest digit, placed last)
        uint32_t k[kSortItems], v[kSortItems], rk[kSortItems];
#pragma unroll
        for (int i = 0; i < kSortItems; ++i) {
            const uint32_t j = w * (kSortTile / 4) + i * kWave + lane;
            const uint32_t idx = sp.lo + min(j, n_here - 1);
            k[i] = j < n_here ? skey[idx] : 0xFFFFFFFFu;
            v[i] = sval[idx];
        }
        s_base[t] = cp.cnt[(size_t)c * kRadix + t];
        __syncthreads();
        wave_rank<kSortItems>(k, shift, kRadixBits, 0xFFFFFFFFu, kSortItems, s_wcnt[w], rk);
        __syncthreads();
        const uint32_t c0 = s_wcnt[0][t], c1 = s_wcnt[1][t], c2 = s_wcnt[2][t], c3 = s_wcnt[3][t];
        s_wcnt[0][t] = 0u;
        s_wcnt[1][t] = c0;
        s_wcnt[2][t] = c0 + c1;
        s_wcnt[3][t] = c0 + c1 + c2;
        uint32_t tot;
        const uint32_t lb = block_exclusive_scan(c0 + c1 + c2 + c3, s_tmp, tot);
        s_local[t] = lb;
        __syncthreads();
        uint32_t lpos[kSortItems];
#pragma unroll
        for (int i = 0; i < kSortItems; ++i) {
            const uint32_t d = digit_at(k[i], shift, kRadixBits);
            lpos[i] = s_local[d] + s_wcnt[w][d] + rk[i];
            s_buf[lpos[i]] = k[i];
        }
        __syncthreads();
        // runs per digit: position j of the reordered chunk goes to base[d] + (j - local[d])
        uint32_t dig[kSortItems];
#pragma unroll
        for (int i = 0; i < kSortItems; ++i) {
            const uint32_t j = t + i * kSortThreads;
            const uint32_t key = s_buf[j];
            dig[i] = digit_at(key, shift, kRadixBits);
            if (j < n_here) dkey[s_base[dig[i]] + (j - s_local[dig[i]])] = key;
        }
        __syncthreads();
#pragma unroll
        for (int i = 0; i < kSortItems; ++i) s_buf[lpos[i]] = v[i];
        __syncthreads();
#pragma unroll
        for (int i = 0; i < kSortItems; ++i) {
            const uint32_t j = t + i * kSortThreads;
            if (j < n_here) dval[s_base[dig[i]] + (j - s_local[dig[i]])] = s_buf[j];
        }
        __syncthreads();   // LDS is reused by the next chunk
    }
}

// The sorted segments into pidx (those left in B) and keys64.
__global__ void __launch_bounds__(256) chunk_final_kernel(const uint32_t* __restrict__ b_key,
                                                          const uint32_t* __restrict__ b_val,
                                                          const uint32_t* __restrict__ a_key,
                                                          uint32_t* __restrict__ pidx, uint64_t* __restrict__ keys64,
                                                          const uint32_t* __restrict__ long_counts, ChunkPlan cp) {
    const uint32_t nc = chunk_count_of(long_counts);
    for (uint32_t c = blockIdx.x; c < nc; c += gridDim.x) {
        const ChunkSpan sp = chunk_span(cp, c, 4);
        if (!sp.loc && !keys64) continue;   // already in place
        const uint64_t tile = cp.seg_tile[sp.s];
        const uint32_t* key = sp.loc ? b_key : a_key;
        static_assert(kSortTile == 16 * 256, "sixteen entries per thread");
        uint32_t v[16], k[16];
#pragma unroll
        for (int i = 0; i < 16; ++i) {
            const uint32_t j = min(sp.lo + i * 256 + threadIdx.x, sp.hi - 1);
            v[i] = sp.loc ? b_val[j] : 0u;
            k[i] = keys64 ? key[j] : 0u;
        }
#pragma unroll
        for (int i = 0; i < 16; ++i) {
            const uint32_t j = sp.lo + i * 256 + threadIdx.x;
            if (j >= sp.hi) continue;
            if (sp.loc) pidx[j] = v[i];
            if (keys64) keys64[j] = (tile << 32) | k[i];
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
    // 2^tile_bits > tiles: the sentinel id 0xFFFFFFFF, cut to the sorted bits, still sorts
    // after every real tile id
    int tile_bits = 0;
    while (tile_bits < 32 && (1ull << tile_bits) <= tiles) ++tile_bits;
    p.passes = DigitSplit(0, tile_bits, kTileRadixBits).passes;
    p.tile_bits = tile_bits;
    p.sort_tiles = (uint32_t)((capacity + kSortTile - 1) / kSortTile);
    p.scan_blocks = (uint32_t)((n + kScanBlock - 1) / kScanBlock);
    size_t off = 0;
    p.off_keys_a = off;     off = align256(off + capacity * 4);
    p.off_keys_b = off;     off = align256(off + capacity * 4);
    p.off_vals_alt = off;   off = align256(off + capacity * 4);
    p.off_z_a = off;        off = align256(off + capacity * 4);
    p.off_z_b = off;        off = align256(off + capacity * 4);
    // zero-initialised region: the digit totals of the passes and the long-segment counts
    p.off_hist = off;       off += (size_t)kMaxPasses * kTileRadix * 4;
    p.off_long_counts = off; off = align256(off + (size_t)kLongCounters * kLongCounterStride * 4);
    p.off_block_sums = off; off = align256(off + (size_t)(p.scan_blocks + 1) * 4);
    // kClassLists lists of at most `per` tiles, the list of the segments sorted through the
    // workspace, the list of the chunk-sorted ones
    p.off_long_lists = off; off = align256(off + (size_t)(5 * tiles + 2 * kClassLists) * 4);
    // the chunk sort's tables: at most h_max segments (longer than kChunkMin each) and
    // capacity / 4096 + h_max chunks
    p.chunk_h_max = (uint32_t)std::min<uint64_t>(tiles, capacity / (kChunkMin + 1) + 1);
    p.chunk_max = (uint32_t)(capacity / kSortTile + p.chunk_h_max);
    p.off_chunk_tables = off; off = align256(off + (size_t)(10 * (uint64_t)p.chunk_h_max + 1) * 4);
    p.off_chunk_seg = off;   off = align256(off + (size_t)p.chunk_max * 4);
    p.off_chunk_cnt = off;   off = align256(off + (size_t)p.chunk_max * kRadix * 4);
    p.off_tcount = off;     off = align256(off + (size_t)p.sort_tiles * kTileRadix * 4);
    p.bytes = off;
    return p;
}

int launch_bin_sort(const BinSortPlan& plan, const isogs_projected* proj, const int32_t* n_per_view,
                    const isogs_camera* cams, int32_t nv, const isogs_bins* bins, void* ws, hipStream_t stream) {
    char* base = static_cast<char*>(ws);
    uint32_t* keys_a = reinterpret_cast<uint32_t*>(base + plan.off_keys_a);
    uint32_t* keys_b = reinterpret_cast<uint32_t*>(base + plan.off_keys_b);
    uint32_t* vals_alt = reinterpret_cast<uint32_t*>(base + plan.off_vals_alt);
    uint32_t* z_a = reinterpret_cast<uint32_t*>(base + plan.off_z_a);
    uint32_t* z_b = reinterpret_cast<uint32_t*>(base + plan.off_z_b);
    uint32_t* hist = reinterpret_cast<uint32_t*>(base + plan.off_hist);
    uint32_t* tcount = reinterpret_cast<uint32_t*>(base + plan.off_tcount);
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

    // ping-pong so that the last tile pass lands the values in the caller's pidx
    const bool odd = plan.passes & 1;
    uint32_t* v_emit = odd ? vals_alt : bins->pidx;
    uint32_t* v_other = odd ? bins->pidx : vals_alt;

    // 3. emit (per group of views)
    const DigitSplit tsplit(0, plan.tile_bits, kTileRadixBits);
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
        if (!blocks) continue;
        hipLaunchKernelGGL(emit_kernel, dim3(blocks), dim3(256), 0, stream, pk,
                           reinterpret_cast<const float4*>(proj->record), bins->offsets, plan.n_total,
                           proj->depth, bins->count, plan.capacity, keys_a, v_emit, z_a);
    }
    if (plan.capacity == 0) return hipPeekAtLastError() == hipSuccess ? 0 : -1;

    // 4. radix passes over the tile id
    const uint32_t* kin = keys_a;
    const uint32_t* vin = v_emit;
    const uint32_t* zin = z_a;
    uint32_t* kout = keys_b;
    uint32_t* vout = v_other;
    uint32_t* zout = z_b;
    for (int p = 0; p < plan.passes; ++p) {
        const int sh = tsplit.shift(p), wd = tsplit.width(p);
        hipLaunchKernelGGL(tile_count_kernel, dim3(plan.sort_tiles), dim3(kSortThreads), 0, stream, kin, bins->count,
                           plan.capacity, sh, wd, tcount, plan.sort_tiles);
        hipLaunchKernelGGL(tile_scan_kernel, dim3(kTileRadix), dim3(256), 0, stream, tcount, plan.sort_tiles,
                           bins->count, plan.capacity, hist + p * kTileRadix);
        // digit widths of the tile passes: 8 or 9 bits (DigitSplit of at most 32 bits, 9 at most)
        static_assert(kTileRadixBits == 9, "scatter instantiated for 8- and 9-bit digits");
        auto scatter = wd == 9 ? sort_scatter_kernel<9> : wd == 8 ? sort_scatter_kernel<8> : wd == 7 ? sort_scatter_kernel<7>
                     : wd == 6 ? sort_scatter_kernel<6> : wd == 5 ? sort_scatter_kernel<5> : wd == 4 ? sort_scatter_kernel<4>
                     : wd == 3 ? sort_scatter_kernel<3> : wd == 2 ? sort_scatter_kernel<2> : sort_scatter_kernel<1>;
        hipLaunchKernelGGL(scatter, dim3(plan.sort_tiles), dim3(kSortThreads), 0, stream, kin, vin, zin, kout, vout,
                           zout, bins->count, plan.capacity, sh, hist + p * kTileRadix, tcount, plan.sort_tiles);
        const uint32_t* tk = kin;
        const uint32_t* tv = vin;
        const uint32_t* tz = zin;
        kin = kout;
        vin = vout;
        zin = zout;
        kout = const_cast<uint32_t*>(tk);
        vout = const_cast<uint32_t*>(tv);
        zout = const_cast<uint32_t*>(tz);
    }
    // 5. ranges
    const unsigned fin_blocks = (unsigned)std::min<uint64_t>(2048, (plan.capacity + 1023) / 1024);
    hipLaunchKernelGGL(finalize_kernel, dim3(fin_blocks), dim3(256), 0, stream, kin, bins->count, plan.capacity,
                       plan.tiles_total, bins->ranges);
    // 6. depth order within every tile (zin: depth bits in the order of pidx; the tile-id
    // arrays and vals_alt are scratch now)
    if (plan.tiles_total) {
        static int big_grid = 0;
        if (!big_grid) big_grid = resident_blocks(reinterpret_cast<const void*>(segment_sort_big_kernel), kBigThreads);
        if (!big_grid) return -1;
        uint32_t* long_counts = reinterpret_cast<uint32_t*>(base + plan.off_long_counts);
        uint32_t* long_lists = reinterpret_cast<uint32_t*>(base + plan.off_long_lists);
        hipLaunchKernelGGL(segment_sort_small_kernel, dim3((plan.tiles_total + 3) / 4), dim3(kSortThreads), 0, stream,
                           bins->ranges, plan.tiles_total, zin, bins->pidx, bins->keys, bins->count,
                           plan.capacity, bins->status, long_lists, long_counts);
        hipLaunchKernelGGL(segment_sort_big_kernel, dim3((unsigned)std::min<uint32_t>(plan.tiles_total, big_grid)),
                           dim3(kBigThreads), 0, stream, bins->ranges, plan.tiles_total, zin, bins->pidx,
                           bins->keys, bins->count, plan.capacity, bins->status, long_lists, long_counts, keys_a,
                           keys_b, vals_alt);
        // 6c. the longest segments, by all workgroups (A = (zin, pidx), B = (keys_a, vals_alt)).
        // A tile's list holds each particle of its view at most once, so without a view of
        // more than kChunkMin particles there is no such segment and nothing is launched.
        int32_t most = 0;
        for (int v = 0; v < nv; ++v) most = std::max(most, n_per_view[v]);
        if ((uint32_t)most <= kChunkMin) return hipPeekAtLastError() == hipSuccess ? 0 : -1;
        static int chunk_grid = 0;
        if (!chunk_grid) chunk_grid = resident_blocks(reinterpret_cast<const void*>(chunk_scatter_kernel), kSortThreads);
        if (!chunk_grid) return -1;
        uint32_t* tables = reinterpret_cast<uint32_t*>(base + plan.off_chunk_tables);
        const uint32_t hm = plan.chunk_h_max;
        ChunkPlan cp{tables, tables + hm, tables + 2 * hm, tables + 3 * hm + 1, tables + 8 * hm + 1,
                     reinterpret_cast<uint32_t*>(base + plan.off_chunk_seg),
                     reinterpret_cast<uint32_t*>(base + plan.off_chunk_cnt), hm};
        uint32_t* zmut = const_cast<uint32_t*>(zin);
        const unsigned cg = (unsigned)std::min<uint32_t>(plan.chunk_max, (uint32_t)chunk_grid);
        const unsigned sg = (unsigned)std::min<uint32_t>(hm, 1024u);
        hipLaunchKernelGGL(chunk_setup_kernel, dim3(1), dim3(256), 0, stream, bins->ranges, plan.tiles_total,
                           long_lists, long_counts, cp);
        for (int pass = 0; pass < 4; ++pass) {
            hipLaunchKernelGGL(chunk_count_kernel, dim3(cg), dim3(kSortThreads), 0, stream, zin, keys_a, long_counts,
                               cp, pass);
            hipLaunchKernelGGL(chunk_scan_kernel, dim3(sg), dim3(256), 0, stream, long_counts, cp, pass);
            hipLaunchKernelGGL(chunk_scatter_kernel, dim3(cg), dim3(kSortThreads), 0, stream, zmut, bins->pidx, keys_a,
                               vals_alt, long_counts, cp, pass);
        }
        hipLaunchKernelGGL(chunk_final_kernel, dim3(cg), dim3(256), 0, stream, keys_a, vals_alt, zin, bins->pidx,
                           bins->keys, long_counts, cp);
    }
    return hipPeekAtLastError() == hipSuccess ? 0 : -1;
}

}  // namespace isogs
