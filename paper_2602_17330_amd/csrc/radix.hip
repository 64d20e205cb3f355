// Device-wide stable LSD radix sort of 64-bit records (8-bit digits) and exclusive scan.
//
// Each pass is three launches: a per-tile digit histogram, an exclusive scan of the
// digit-major histogram (so tile t's bucket d starts after every earlier tile's bucket d and
// every smaller bucket), and a scatter.  The scatter ranks records stably inside a tile
// with wave ballots (the eight digit bits give each lane the mask of lanes holding the same
// digit; its rank is the popcount of the lower lanes in that mask) and per-wave digit
// counters in LDS, stages the tile in LDS in sorted order, and then writes each digit's run
// with consecutive threads so that global stores are contiguous.  The scan itself is two
// launches, chunk totals and then the chunks, each block of the second adding up the totals
// before its chunk (a third launch scans the totals first when there are more than 1024).
#include "radix.h"

namespace subquad {

constexpr int kScanThreads = 256;
constexpr int kScanItems = 16;
constexpr int kScanChunk = kScanThreads * kScanItems;
constexpr int64_t kScanSumChunks = 1024;  // up to this many chunks, apply blocks add up their prefix

// idx, or the last valid index when idx is past the end (count >= 1): lets a loop issue all
// of its loads unconditionally, masking the values afterwards.
__device__ __forceinline__ int64_t clamp_index(int64_t idx, int64_t count) { return idx < count ? idx : count - 1; }

__device__ __forceinline__ uint64_t lanemask_lt(int lane) {
    return lane == 0 ? 0ull : (~0ull >> (64 - lane));
}

// Inclusive scan of one value per thread over a block of kScanThreads (= 4 waves).
__device__ __forceinline__ uint32_t block_inclusive_scan(uint32_t v, uint32_t *wave_tot) {
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        uint32_t o = __shfl_up(v, off, 64);
        if (lane >= off) v += o;
    }
    if (lane == 63) wave_tot[w] = v;
    __syncthreads();
    uint32_t add = 0;
    for (int k = 0; k < w; ++k) add += wave_tot[k];
    __syncthreads();
    return v + add;
}

// (live, when given, is a record count on the device: with none, the scan has nothing to do
// and each of its kernels returns at once; the whole block takes the same branch.)
__global__ __launch_bounds__(kScanThreads) void scan_reduce_kernel(const uint32_t *__restrict__ data,
                                                                   int64_t count, uint32_t *__restrict__ partial,
                                                                   const int64_t *__restrict__ live) {
    if (live && *live <= 0) return;
    __shared__ uint32_t wt[4];
    int64_t base = (int64_t)blockIdx.x * kScanChunk;
    uint32_t v[kScanItems], s = 0;
#pragma unroll
    for (int k = 0; k < kScanItems; ++k) v[k] = data[clamp_index(base + (int64_t)k * kScanThreads + threadIdx.x, count)];
#pragma unroll
    for (int k = 0; k < kScanItems; ++k)
        if (base + (int64_t)k * kScanThreads + threadIdx.x < count) s += v[k];
    uint32_t inc = block_inclusive_scan(s, wt);
    if (threadIdx.x == kScanThreads - 1) partial[blockIdx.x] = inc;
}

// Single block: exclusive scan of the chunk totals, any length.
__global__ __launch_bounds__(kScanThreads) void scan_partials_kernel(uint32_t *__restrict__ partial, int64_t m,
                                                                     const int64_t *__restrict__ live) {
    if (live && *live <= 0) return;
    __shared__ uint32_t wt[4];
    __shared__ uint32_t carry_s;
    if (threadIdx.x == 0) carry_s = 0;
    __syncthreads();
    for (int64_t base = 0; base < m; base += kScanThreads) {
        int64_t idx = base + threadIdx.x;
        uint32_t v = idx < m ? partial[idx] : 0;
        uint32_t inc = block_inclusive_scan(v, wt);
        uint32_t carry = carry_s;
        if (idx < m) partial[idx] = carry + inc - v;
        __syncthreads();
        if (threadIdx.x == kScanThreads - 1) carry_s = carry + inc;
        __syncthreads();
    }
}

// VEC: data is 16-byte aligned, so a thread moves its entries as 16-byte words (a wave's
// loads then cover whole lines instead of one word in every 64 bytes).
// SUM: partial holds the chunks' raw totals (no scan_partials_kernel ran) and each block adds
// up those before its own; for at most kScanSumChunks chunks that costs less than a launch.
template <bool VEC, bool SUM>
__global__ __launch_bounds__(kScanThreads) void scan_apply_kernel(uint32_t *__restrict__ data, int64_t count,
                                                                  const uint32_t *__restrict__ partial,
                                                                  const int64_t *__restrict__ live) {
    if (live && *live <= 0) return;
    __shared__ uint32_t wt[4];
    __shared__ uint32_t before;
    if (SUM) {  // the chunks before this block's, summed over the block
        uint32_t acc = 0;
        for (int c = threadIdx.x; c < (int)blockIdx.x; c += kScanThreads) acc += partial[c];
        const uint32_t ps = block_inclusive_scan(acc, wt);
        if (threadIdx.x == kScanThreads - 1) before = ps;
        __syncthreads();
    }
    // thread t owns kScanItems consecutive entries
    int64_t base = (int64_t)blockIdx.x * kScanChunk + (int64_t)threadIdx.x * kScanItems;
    const bool whole = VEC && base + kScanItems <= count;
    uint32_t v[kScanItems];
    uint32_t s = 0;
    if (whole) {
        const uint4 *d4 = reinterpret_cast<const uint4 *>(data + base);
#pragma unroll
        for (int k = 0; k < kScanItems / 4; ++k) {
            const uint4 q = d4[k];
            v[4 * k] = q.x;
            v[4 * k + 1] = q.y;
            v[4 * k + 2] = q.z;
            v[4 * k + 3] = q.w;
        }
    } else {
#pragma unroll
        for (int k = 0; k < kScanItems; ++k) v[k] = base + k < count ? data[base + k] : 0u;
    }
#pragma unroll
    for (int k = 0; k < kScanItems; ++k) s += v[k];
    uint32_t inc = block_inclusive_scan(s, wt);
    uint32_t run = (SUM ? before : partial[blockIdx.x]) + inc - s;
    uint32_t out[kScanItems];
#pragma unroll
    for (int k = 0; k < kScanItems; ++k) {
        out[k] = run;
        run += v[k];
    }
    if (whole) {
        uint4 *d4 = reinterpret_cast<uint4 *>(data + base);
#pragma unroll
        for (int k = 0; k < kScanItems / 4; ++k) d4[k] = make_uint4(out[4 * k], out[4 * k + 1], out[4 * k + 2], out[4 * k + 3]);
    } else {
#pragma unroll
        for (int k = 0; k < kScanItems; ++k)
            if (base + k < count) data[base + k] = out[k];
    }
}

size_t scan_scratch_bytes(int64_t count) {
    return align_up(sizeof(uint32_t) * (size_t)std::max<int64_t>(1, ceil_div(count, kScanChunk)), 256);
}

static int scan_exclusive_u32_live(uint32_t *data, int64_t count, const int64_t *live, void *scratch,
                                   hipStream_t st) {
    if (count <= 0) return SUBQUAD_OK;
    int64_t chunks = ceil_div(count, kScanChunk);
    uint32_t *partial = static_cast<uint32_t *>(scratch);
    scan_reduce_kernel<<<(unsigned)chunks, kScanThreads, 0, st>>>(data, count, partial, live);
    SQ_LAUNCHED("scan_reduce_kernel");
    const bool vec = ((uintptr_t)data & 15) == 0;
    const unsigned g = (unsigned)chunks;
    if (chunks <= kScanSumChunks) {
        if (vec) scan_apply_kernel<true, true><<<g, kScanThreads, 0, st>>>(data, count, partial, live);
        else scan_apply_kernel<false, true><<<g, kScanThreads, 0, st>>>(data, count, partial, live);
    } else {
        scan_partials_kernel<<<1, kScanThreads, 0, st>>>(partial, chunks, live);
        SQ_LAUNCHED("scan_partials_kernel");
        if (vec) scan_apply_kernel<true, false><<<g, kScanThreads, 0, st>>>(data, count, partial, live);
        else scan_apply_kernel<false, false><<<g, kScanThreads, 0, st>>>(data, count, partial, live);
    }
    SQ_LAUNCHED("scan_apply_kernel");
    return SUBQUAD_OK;
}

int scan_exclusive_u32(uint32_t *data, int64_t count, void *scratch, hipStream_t st) {
    return scan_exclusive_u32_live(data, count, nullptr, scratch, st);
}

// ---- 64-bit exclusive scan (device-side element count) ----
__device__ __forceinline__ uint64_t block_inclusive_scan64(uint64_t v, uint64_t *wave_tot) {
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        uint64_t o = __shfl_up(v, off, 64);
        if (lane >= off) v += o;
    }
    if (lane == 63) wave_tot[w] = v;
    __syncthreads();
    uint64_t add = 0;
    for (int k = 0; k < w; ++k) add += wave_tot[k];
    __syncthreads();
    return v + add;
}

__device__ __forceinline__ int64_t count_of(int64_t cap, const uint64_t *count_dev) {
    if (!count_dev) return cap;
    uint64_t c = *count_dev;
    return c < (uint64_t)cap ? (int64_t)c : cap;
}

__global__ __launch_bounds__(kScanThreads) void scan64_reduce_kernel(const uint64_t *__restrict__ data, int64_t cap,
                                                                     const uint64_t *__restrict__ count_dev,
                                                                     uint64_t *__restrict__ partial) {
    __shared__ uint64_t wt[4];
    const int64_t count = count_of(cap, count_dev);
    int64_t base = (int64_t)blockIdx.x * kScanChunk;
    uint64_t s = 0;
    if (base < count) {  // count may be below the launch's capacity
        uint64_t v[kScanItems];
#pragma unroll
        for (int k = 0; k < kScanItems; ++k)
            v[k] = data[clamp_index(base + (int64_t)k * kScanThreads + threadIdx.x, count)];
#pragma unroll
        for (int k = 0; k < kScanItems; ++k)
            if (base + (int64_t)k * kScanThreads + threadIdx.x < count) s += v[k];
    }
    uint64_t inc = block_inclusive_scan64(s, wt);
    if (threadIdx.x == kScanThreads - 1) partial[blockIdx.x] = inc;
}

__global__ __launch_bounds__(kScanThreads) void scan64_partials_kernel(uint64_t *__restrict__ partial, int64_t m) {
    __shared__ uint64_t wt[4];
    __shared__ uint64_t carry_s;
    if (threadIdx.x == 0) carry_s = 0;
    __syncthreads();
    for (int64_t base = 0; base < m; base += kScanThreads) {
        int64_t idx = base + threadIdx.x;
        uint64_t v = idx < m ? partial[idx] : 0;
        uint64_t inc = block_inclusive_scan64(v, wt);
        uint64_t carry = carry_s;
        if (idx < m) partial[idx] = carry + inc - v;
        __syncthreads();
        if (threadIdx.x == kScanThreads - 1) carry_s = carry + inc;
        __syncthreads();
    }
}

// SUM as in scan_apply_kernel: partial holds raw chunk totals, added up here.
template <bool SUM>
__global__ __launch_bounds__(kScanThreads) void scan64_apply_kernel(uint64_t *__restrict__ data, int64_t cap,
                                                                    const uint64_t *__restrict__ count_dev,
                                                                    const uint64_t *__restrict__ partial) {
    __shared__ uint64_t wt[4];
    __shared__ uint64_t before;
    if (SUM) {
        uint64_t acc = 0;
        for (int c = threadIdx.x; c < (int)blockIdx.x; c += kScanThreads) acc += partial[c];
        const uint64_t ps = block_inclusive_scan64(acc, wt);
        if (threadIdx.x == kScanThreads - 1) before = ps;
        __syncthreads();
    }
    const int64_t count = count_of(cap, count_dev);
    int64_t base = (int64_t)blockIdx.x * kScanChunk + (int64_t)threadIdx.x * kScanItems;
    uint64_t v[kScanItems];
    uint64_t s = 0;
    if (count > 0) {
#pragma unroll
        for (int k = 0; k < kScanItems; ++k) v[k] = data[clamp_index(base + k, count)];
    }
#pragma unroll
    for (int k = 0; k < kScanItems; ++k) {
        if (base + k >= count) v[k] = 0;
        s += v[k];
    }
    uint64_t inc = block_inclusive_scan64(s, wt);
    uint64_t run = (SUM ? before : partial[blockIdx.x]) + inc - s;
#pragma unroll
    for (int k = 0; k < kScanItems; ++k) {
        int64_t idx = base + k;
        if (idx < count) data[idx] = run;
        run += v[k];
    }
}

size_t scan64_scratch_bytes(int64_t count_cap) {
    return align_up(sizeof(uint64_t) * (size_t)std::max<int64_t>(1, ceil_div(count_cap, kScanChunk)), 256);
}

int scan_exclusive_u64(uint64_t *data, int64_t count_cap, const uint64_t *count_dev, void *scratch, hipStream_t st) {
    if (count_cap <= 0) return SUBQUAD_OK;
    int64_t chunks = ceil_div(count_cap, kScanChunk);
    uint64_t *partial = static_cast<uint64_t *>(scratch);
    scan64_reduce_kernel<<<(unsigned)chunks, kScanThreads, 0, st>>>(data, count_cap, count_dev, partial);
    SQ_LAUNCHED("scan64_reduce_kernel");
    if (chunks <= kScanSumChunks) {
        scan64_apply_kernel<true><<<(unsigned)chunks, kScanThreads, 0, st>>>(data, count_cap, count_dev, partial);
    } else {
        scan64_partials_kernel<<<1, kScanThreads, 0, st>>>(partial, chunks);
        SQ_LAUNCHED("scan64_partials_kernel");
        scan64_apply_kernel<false><<<(unsigned)chunks, kScanThreads, 0, st>>>(data, count_cap, count_dev, partial);
    }
    SQ_LAUNCHED("scan64_apply_kernel");
    return SUBQUAD_OK;
}

__device__ __forceinline__ int64_t live_count(int64_t n_cap, const int64_t *n_dev) {
    if (!n_dev) return n_cap;
    int64_t v = *n_dev;
    return v < n_cap ? (v < 0 ? 0 : v) : n_cap;
}

// One tile's digit counts into column tb of hist (zero past the live records).
__device__ __forceinline__ void radix_hist_tile(const uint64_t *__restrict__ in, int64_t n, int shift, uint32_t dmask,
                                                uint32_t *__restrict__ hist, int64_t nblocks, int64_t tb, uint32_t *h) {
    h[threadIdx.x] = 0;  // (this thread read its counter of any previous tile already)
    __syncthreads();
    const int64_t base = tb * kRadixTile;
    if (base < n) {
        // all loads in flight before any is used (an index past the end reads the last record
        // and is not counted)
        uint64_t v[kRadixItems];
#pragma unroll
        for (int k = 0; k < kRadixItems; ++k) {
            const int64_t idx = base + (int64_t)k * kRadixThreads + threadIdx.x;
            v[k] = in[idx < n ? idx : n - 1];
        }
#pragma unroll
        for (int k = 0; k < kRadixItems; ++k) {
            const int64_t idx = base + (int64_t)k * kRadixThreads + threadIdx.x;
            if (idx < n) atomicAdd(&h[(uint32_t)(v[k] >> shift) & dmask], 1u);
        }
    }
    __syncthreads();
    hist[(int64_t)threadIdx.x * nblocks + tb] = h[threadIdx.x];
}

// LOOP (the few-live form): blocks take tiles blockIdx.x, blockIdx.x + gridDim.x, ...;
// otherwise one tile per block.  Every tile's column is written, zero past the live records.
template <bool LOOP>
__global__ __launch_bounds__(kRadixThreads) void radix_hist_kernel(const uint64_t *__restrict__ in, int64_t n_cap,
                                                                   const int64_t *__restrict__ n_dev, int shift,
                                                                   uint32_t dmask, uint32_t *__restrict__ hist,
                                                                   int64_t nblocks) {
    __shared__ uint32_t h[kRadixBuckets];
    const int64_t n = live_count(n_cap, n_dev);
    if (n_dev && n == 0) return;  // no records: the scan and the scatter skip this pass too
    if (!LOOP) {
        radix_hist_tile(in, n, shift, dmask, hist, nblocks, blockIdx.x, h);
        return;
    }
    for (int64_t tb = blockIdx.x; tb < nblocks; tb += gridDim.x) radix_hist_tile(in, n, shift, dmask, hist, nblocks, tb, h);
}

// One tile of the scatter (the block's LDS passed in); tile0 < n.
__device__ __forceinline__ void radix_scatter_tile(const uint64_t *__restrict__ in, uint64_t *__restrict__ out,
                                                   int64_t n, int shift, uint32_t dmask,
                                                   const uint32_t *__restrict__ hist, int64_t nblocks, int64_t tb,
                                                   uint32_t (*wc)[kRadixBuckets], uint32_t *tile_off, uint32_t *gbase,
                                                   uint32_t *wt, uint64_t *stage) {
    constexpr int kWaves = kRadixThreads / 64;
    const int t = threadIdx.x, lane = t & 63, w = t >> 6;
    const int64_t tile0 = tb * kRadixTile;
    for (int k = t; k < kWaves * kRadixBuckets; k += kRadixThreads) (&wc[0][0])[k] = 0;
    __syncthreads();

    const int64_t base = tile0 + (int64_t)w * (64 * kRadixItems);
    const uint64_t lt = lanemask_lt(lane);
    uint64_t rec[kRadixItems];
    uint32_t rank[kRadixItems];
    // the tile's loads all issue before the ranking starts (an index past the end reads the
    // last record; it is not ranked or written)
#pragma unroll
    for (int k = 0; k < kRadixItems; ++k) {
        const int64_t idx = base + (int64_t)k * 64 + lane;
        rec[k] = in[idx < n ? idx : n - 1];
    }
    const uint32_t my_base = hist[(int64_t)t * nblocks + tb];  // kRadixThreads == kRadixBuckets
#pragma unroll
    for (int k = 0; k < kRadixItems; ++k) {
        int64_t idx = base + (int64_t)k * 64 + lane;
        bool valid = idx < n;
        uint32_t d = (uint32_t)(rec[k] >> shift) & dmask;
        // lanes holding the same digit: for every bit, those whose bit equals this lane's
        // (the ballot XNOR the lane's bit replicated), as two 32-bit halves
        uint64_t m = __ballot(valid);
        uint32_t mlo = (uint32_t)m, mhi = (uint32_t)(m >> 32);
#pragma unroll
        for (int bit = 0; bit < kRadixBits; ++bit) {
            const uint32_t rep = (uint32_t)((int32_t)(d << (31 - bit)) >> 31);  // 0 or ~0
            const uint64_t bal = __ballot(rep != 0u);
            mlo &= ~((uint32_t)bal ^ rep);
            mhi &= ~((uint32_t)(bal >> 32) ^ rep);
        }
        m = ((uint64_t)mhi << 32) | mlo;
        uint32_t r = 0;
        if (valid) {
            uint32_t before = wc[w][d];
            r = before + (uint32_t)__popcll(m & lt);
            if ((m & lt) == 0) wc[w][d] = before + (uint32_t)__popcll(m);
        }
        rank[k] = valid ? r : 0xFFFFFFFFu;
    }
    __syncthreads();
    // wave-exclusive offsets per digit, then the tile-exclusive digit offsets
    uint32_t tot = 0;
    {
        const int d = t;  // kRadixThreads == kRadixBuckets
#pragma unroll
        for (int ww = 0; ww < kWaves; ++ww) {
            uint32_t c = wc[ww][d];
            wc[ww][d] = tot;
            tot += c;
        }
        gbase[d] = my_base;
    }
    uint32_t inc = block_inclusive_scan(tot, wt);
    tile_off[t] = inc - tot;
    __syncthreads();
#pragma unroll
    for (int k = 0; k < kRadixItems; ++k) {
        if (rank[k] != 0xFFFFFFFFu) {
            uint32_t d = (uint32_t)(rec[k] >> shift) & dmask;
            stage[tile_off[d] + wc[w][d] + rank[k]] = rec[k];
        }
    }
    __syncthreads();
    const int tile_n = (int)std::min<int64_t>(kRadixTile, n - tile0);
    for (int s = t; s < tile_n; s += kRadixThreads) {
        uint64_t v = stage[s];
        uint32_t d = (uint32_t)(v >> shift) & dmask;
        const int64_t pos = (int64_t)gbase[d] + (s - (int64_t)tile_off[d]);
        if (pos >= 0 && pos < n) out[pos] = v;
    }
}

// LOOP (the few-live form): blocks take tiles blockIdx.x, blockIdx.x + gridDim.x, ...;
// otherwise one tile per block.
template <bool LOOP>
__global__ __launch_bounds__(kRadixThreads) void radix_scatter_kernel(
    const uint64_t *__restrict__ in, uint64_t *__restrict__ out, int64_t n_cap, const int64_t *__restrict__ n_dev,
    int shift, uint32_t dmask, const uint32_t *__restrict__ hist, int64_t nblocks) {
    constexpr int kWaves = kRadixThreads / 64;
    __shared__ uint32_t wc[kWaves][kRadixBuckets];
    __shared__ uint32_t tile_off[kRadixBuckets];
    __shared__ uint32_t gbase[kRadixBuckets];
    __shared__ uint32_t wt[4];
    __shared__ uint64_t stage[kRadixTile];
    const int64_t n = live_count(n_cap, n_dev);
    if (!LOOP) {
        if ((int64_t)blockIdx.x * kRadixTile >= n) return;  // whole block
        radix_scatter_tile(in, out, n, shift, dmask, hist, nblocks, blockIdx.x, wc, tile_off, gbase, wt, stage);
        return;
    }
    for (int64_t tb = blockIdx.x; tb < nblocks; tb += gridDim.x) {
        if (tb * kRadixTile >= n) break;  // this tile and every later one hold no live record
        radix_scatter_tile(in, out, n, shift, dmask, hist, nblocks, tb, wc, tile_off, gbase, wt, stage);
        __syncthreads();  // the LDS counters and the staged tile are reused by the next tile
    }
}

size_t radix_scratch_bytes(int64_t n_cap) {
    int64_t nblocks = std::max<int64_t>(1, ceil_div(n_cap, kRadixTile));
    int64_t hist = nblocks * kRadixBuckets;
    return align_up(sizeof(uint32_t) * (size_t)hist, 256) + scan_scratch_bytes(hist);
}

int radix_sort_u64(uint64_t *a, uint64_t *b, int64_t n_cap, const int64_t *n_dev, int lo_bit, int key_bits,
                   void *scratch, size_t scratch_bytes, hipStream_t st, uint64_t **result, const char *tag,
                   bool few_live) {
    const std::string hist_name = std::string(tag) + "_hist", scan_name = std::string(tag) + "_scan",
                      scatter_name = std::string(tag) + "_scatter";
    *result = a;
    if (n_cap <= 1 || key_bits <= 0) return SUBQUAD_OK;
    SQ_REQUIRE(scratch_bytes >= radix_scratch_bytes(n_cap), SUBQUAD_ERR_WORKSPACE, "radix scratch too small");
    const int64_t nblocks = ceil_div(n_cap, kRadixTile);  // tiles
    // one tile per block, unless few records are expected to be live (the device count is
    // usually zero): then at most as many blocks as the chip holds at once, striding by the
    // grid, so that an empty pass dispatches few blocks whatever the capacity (a full pass in
    // this form is slower: its tiles in flight spread further apart than dispatch order keeps
    // them, and their scattered writes lose locality)
    int64_t grid_h = nblocks, grid_s = nblocks;
    if (few_live) {
        grid_h = std::min<int64_t>(
            nblocks, (int64_t)resident_blocks_per_cu((const void *)radix_hist_kernel<true>) * device_cus());
        grid_s = std::min<int64_t>(
            nblocks, (int64_t)resident_blocks_per_cu((const void *)radix_scatter_kernel<true>) * device_cus());
    }
    const int64_t hist_n = nblocks * kRadixBuckets;
    SQ_REQUIRE(n_cap < (int64_t(1) << 32), SUBQUAD_ERR_ARG, "radix sort limited to 2^32 records");
    uint32_t *hist = static_cast<uint32_t *>(scratch);
    void *scan_scratch = static_cast<char *>(scratch) + align_up(sizeof(uint32_t) * (size_t)hist_n, 256);
    uint64_t *src = a, *dst = b;
    for (int done = 0; done < key_bits; done += kRadixBits) {
        const int bits = std::min(kRadixBits, key_bits - done);
        const int shift = lo_bit + done;
        const uint32_t dmask = (1u << bits) - 1u;
        {
            ProfScope prof(hist_name.c_str(), st);
            if (few_live)
                radix_hist_kernel<true><<<(unsigned)grid_h, kRadixThreads, 0, st>>>(src, n_cap, n_dev, shift, dmask,
                                                                                hist, nblocks);
            else
                radix_hist_kernel<false><<<(unsigned)grid_h, kRadixThreads, 0, st>>>(src, n_cap, n_dev, shift, dmask,
                                                                                 hist, nblocks);
        }
        SQ_LAUNCHED("radix_hist_kernel");
        int rc;
        {
            ProfScope prof(scan_name.c_str(), st);
            rc = scan_exclusive_u32_live(hist, hist_n, n_dev, scan_scratch, st);
        }
        if (rc != SUBQUAD_OK) return rc;
        {
            ProfScope prof(scatter_name.c_str(), st);
            if (few_live)
                radix_scatter_kernel<true><<<(unsigned)grid_s, kRadixThreads, 0, st>>>(src, dst, n_cap, n_dev, shift,
                                                                                    dmask, hist, nblocks);
            else
                radix_scatter_kernel<false><<<(unsigned)grid_s, kRadixThreads, 0, st>>>(src, dst, n_cap, n_dev, shift,
                                                                                     dmask, hist, nblocks);
        }
        SQ_LAUNCHED("radix_scatter_kernel");
        std::swap(src, dst);
    }
    *result = src;
    return SUBQUAD_OK;
}

}  // namespace subquad
