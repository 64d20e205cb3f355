// MinHash LSH banding into the candidate list (Algorithm 1, preprocessing: build the MinHash
// index and generate CAND; index of Sec. 4.2; retrieval cost O(|C|) + O(n log n),
// Appendix B).
//
// A pair (i, j), i < j, of one repertoire is a candidate iff for some band beta the r-tuples
// sig[i][beta*r .. beta*r + r) and sig[j][...] are exactly equal.  Steps:
//   1. band records: for every (beta, i) a 64-bit mix of (tuple, repertoire); the record is
//      (top bits of the mix | beta) << 32 | (beta * n + i), written band-major (beta in the
//      word's low bits when the sort key leaves them free).  Every (i, beta) also gets a
//      class id in a row-major table C[n][b], at first its own record number beta * n + i.
//   2. stable radix sort of the records on their mix bits (log2 n + 4 rounded up to whole
//      bytes, at most 32: 24 for n <= 2^20; the bits below are cleared).  Stability keeps
//      records with equal mix bits in (beta, i) order, so each bucket (equal mix bits, equal
//      band) is a contiguous run with ascending i.
//   3. runs: every run of >= 2 records is listed.  Equal tuples (of one repertoire) always
//      share a run, so exact classes are formed inside runs: a member whose tuple and
//      repertoire equal those of its run's first record takes that record's number as its
//      class id, any other member the number of the first member equal to it.  Afterwards
//      C[i][e] == C[j][e] holds exactly when i and j (of one repertoire) have equal tuples
//      in band e.
//   4. emission: every pair of records of a run is a potential partner; it is kept only in
//      the FIRST band in which its tuples are equal (class ids equal in the run's band and
//      different in every earlier one), so each candidate is emitted exactly once.  Kept
//      pairs are appended as keys (i << nb) | j.
//   5. radix sort of the pair keys gives the canonical (i, j) order; then the pair list and
//      the CSR row offsets are written.
// The mixing function only decides which records meet; equality is always decided on the
// signature words themselves, so results never depend on hash collisions.
#include "radix.h"

namespace subquad {

constexpr int kKeysTileSeqs = 64;
constexpr int kKeysThreads = 256;
constexpr int kKeysUnroll = 8;

// Words per row of the class-id table C: b rounded up to whole 16-byte words, so that every
// row is 16-byte aligned.
__host__ __device__ inline int class_stride(int b) { return (b + 3) & ~3; }

// 64-bit finaliser of MurmurHash3 (fmix64, Austin Appleby's published constants): a
// bijective mix whose every output bit depends on every input bit.
__device__ __forceinline__ uint64_t mix64(uint64_t z) {
    z = (z ^ (z >> 33)) * 0xFF51AFD7ED558CCDull;
    z = (z ^ (z >> 33)) * 0xC4CEB9FE1A85EC53ull;
    return z ^ (z >> 33);
}

// Step 1. Block = 64 sequences x b bands.  Reads of the signature rows are contiguous
// (item e = s * b + beta), record stores are contiguous per band (staged through LDS), and
// the class-id rows C[i][0..b) are written in the same item order (contiguous).
// R4: r == 4 with 16-byte aligned tuples, each read as two 16-byte loads.
template <bool R4>
__global__ __launch_bounds__(kKeysThreads) void lsh_keys_kernel(
    const uint64_t *__restrict__ sig, int64_t n, int32_t M, int32_t b, int32_t r,
    const int64_t *__restrict__ offs, int64_t R, uint32_t keep, uint32_t band_in_key, uint64_t *__restrict__ rec,
    uint32_t *__restrict__ C) {
    extern __shared__ uint32_t keyhi[];  // [b][kKeysTileSeqs + 1] (rows padded: a wave's writes, one band apart, hit
                                         // different banks)
    const int64_t i0 = (int64_t)blockIdx.x * kKeysTileSeqs;
    const int items = kKeysTileSeqs * b;
    // kKeysUnroll items per thread at a time, so that their signature loads are in flight
    // together
    for (int e0 = 0; e0 < items; e0 += kKeysThreads * kKeysUnroll) {
        uint64_t h[kKeysUnroll];
        const uint64_t *tup[kKeysUnroll];
#pragma unroll
        for (int u = 0; u < kKeysUnroll; ++u) {
            const int e = e0 + u * kKeysThreads + threadIdx.x;
            const int s = e / b, beta = e - s * b;
            const int64_t i = i0 + s;
            const bool ok = e < items && i < n;
            tup[u] = ok ? sig + i * (int64_t)M + (int64_t)beta * r : nullptr;
            const uint64_t rep = ok && R > 1 ? (uint64_t)rep_of(offs, R, i) : 0ull;
            h[u] = mix64(rep * 0x9E3779B97F4A7C15ull + 0x632BE59BD9B4E019ull + (uint64_t)beta);
        }
        if (R4) {
            ulonglong2 w[kKeysUnroll][2];
#pragma unroll
            for (int u = 0; u < kKeysUnroll; ++u) {
                const ulonglong2 *t2 = reinterpret_cast<const ulonglong2 *>(tup[u] ? tup[u] : sig);
                w[u][0] = t2[0];
                w[u][1] = t2[1];
            }
#pragma unroll
            for (int u = 0; u < kKeysUnroll; ++u) {
                h[u] = mix64(h[u] ^ w[u][0].x);
                h[u] = mix64(h[u] ^ w[u][0].y);
                h[u] = mix64(h[u] ^ w[u][1].x);
                h[u] = mix64(h[u] ^ w[u][1].y);
            }
        } else {
            for (int k = 0; k < r; ++k) {
                uint64_t w[kKeysUnroll];
#pragma unroll
                for (int u = 0; u < kKeysUnroll; ++u) w[u] = tup[u] ? tup[u][k] : 0ull;
#pragma unroll
                for (int u = 0; u < kKeysUnroll; ++u) h[u] = mix64(h[u] ^ w[u]);
            }
        }
#pragma unroll
        for (int u = 0; u < kKeysUnroll; ++u) {
            if (!tup[u]) continue;
            const int e = e0 + u * kKeysThreads + threadIdx.x;
            const int s = e / b, beta = e - s * b;
            keyhi[beta * (kKeysTileSeqs + 1) + s] = ((uint32_t)(h[u] >> 32) & keep) | (band_in_key ? (uint32_t)beta : 0u);
            C[(i0 + s) * class_stride(b) + beta] = (uint32_t)beta * (uint32_t)n + (uint32_t)(i0 + s);  // own class
        }
    }
    __syncthreads();
    for (int e = threadIdx.x; e < items; e += blockDim.x) {
        int beta = e / kKeysTileSeqs, s = e - beta * kKeysTileSeqs;
        int64_t i = i0 + s;
        if (i >= n) continue;
        uint64_t q = (uint64_t)beta * (uint64_t)n + (uint64_t)i;
        rec[q] = ((uint64_t)keyhi[beta * (kKeysTileSeqs + 1) + s] << 32) | q;
    }
}

// Number of mix bits (a multiple of 8, at most 32) that the record sort orders by.
static int record_mix_bits(int64_t n) {
    int lg = 0;
    while ((int64_t(1) << lg) < n) ++lg;
    return std::min(32, (int)ceil_div(lg + 4, 8) * 8);
}

// Step 3a.  Runs: a record that starts a run of >= 2 records (equal mix bits, equal band)
// appends (start << 32 | length) to the run list and adds its pair count.
// BAND_IN_KEY: bits 32.. of a record hold its band as well as its mix bits (the sort key
// leaves them room), so no division is needed.
template <bool BAND_IN_KEY>
__device__ __forceinline__ bool same_bucket(uint64_t a, uint64_t c, uint32_t n32) {
    if (BAND_IN_KEY) return (a >> 32) == (c >> 32);
    return (a >> 32) == (c >> 32) && ((uint32_t)a / n32) == ((uint32_t)c / n32);
}

constexpr int kRunsThreads = 256;
constexpr int kRunsItems = 16;
constexpr int kRunsTile = kRunsThreads * kRunsItems;
constexpr int kSmallRun = 8;  // runs up to this many records: all their pairs in one thread

// End of a bucket's run in sorted records: `good` is known to be in the run whose record
// is `me`, and a bucket's records are contiguous, so gallop forward, then bisect: O(log m)
// loads.  Returns the first index past the run (at most `end`).  `at(x)` reads record x.
template <bool BAND_IN_KEY, typename At>
__device__ __forceinline__ int64_t run_end(At at, int64_t good, int64_t end, uint64_t me, uint32_t n32) {
    int64_t bad = end, stride = 1;
    while (good + stride < end) {
        if (!same_bucket<BAND_IN_KEY>(at(good + stride), me, n32)) {
            bad = good + stride;
            break;
        }
        good += stride;
        stride <<= 1;
    }
    while (bad - good > 1) {
        const int64_t mid = good + ((bad - good) >> 1);
        if (same_bucket<BAND_IN_KEY>(at(mid), me, n32)) good = mid;
        else bad = mid;
    }
    return bad;
}

// Per tile of kRunsTile sorted records: room for its run starts (at most kRunsTile / 2,
// since a run has >= 2 records) from the front, and for its long runs (each starts at least
// kSmallRun + 1 records after the previous one) from the back.
constexpr int kRunsCap = kRunsTile / 2 + kRunsTile / (kSmallRun + 1) + 1;

// A block takes tiles of kRunsTile sorted records; thread t holds records t, t + 256, ...
// of the tile in registers (so a wave's neighbour reads in LDS are consecutive words).
// Pass 1 marks the run starts and a block scan gives each thread its slots in the tile's
// region; pass 2 measures the runs.  Every run start takes a slot at the front: its record
// (start << 32 | length) when the run has at most kSmallRun records (one thread will walk
// all its pairs), else an empty record (length 0), the run itself going to the back of the
// region (its pairs are spread over threads).  No global atomics: the tile writes its
// counts, tmeta[tile] = (starts, long runs), tcount[tile] = starts | long runs << 32 and
// tpairs[tile] = pairs of its long runs, which a scan over tiles turns into list offsets.
template <bool BAND_IN_KEY>
__global__ __launch_bounds__(kRunsThreads) void lsh_runs_kernel(const uint64_t *__restrict__ srec, int64_t total,
                                                                int64_t n, uint64_t *__restrict__ region,
                                                                uint2 *__restrict__ tmeta,
                                                                uint64_t *__restrict__ tcount,
                                                                uint64_t *__restrict__ tpairs) {
    const uint32_t n32 = (uint32_t)n;
    const int t = threadIdx.x;
    __shared__ uint32_t scan[kRunsThreads];
    __shared__ uint32_t nlong;
    __shared__ unsigned long long lpairs;
    __shared__ uint64_t tile_sh[kRunsTile + 2];  // records tile-1 .. tile+kRunsTile
    for (int64_t tile = (int64_t)blockIdx.x * kRunsTile; tile < total; tile += (int64_t)gridDim.x * kRunsTile) {
        const int64_t ti = tile / kRunsTile;
        uint64_t *reg = region + ti * kRunsCap;
        // the tile's loads all issue before any is used (absent records read as ~0)
        uint64_t v[kRunsItems];
#pragma unroll
        for (int k = 0; k < kRunsItems; ++k) {
            const int64_t q = tile + k * kRunsThreads + t;
            v[k] = q < total ? srec[q] : ~0ull;
        }
        if (t < 2) {
            const int64_t q = t == 0 ? tile - 1 : tile + kRunsTile;
            tile_sh[t == 0 ? 0 : kRunsTile + 1] = q >= 0 && q < total ? srec[q] : ~0ull;
        }
        if (t == 0) {
            nlong = 0u;
            lpairs = 0ull;
        }
#pragma unroll
        for (int k = 0; k < kRunsItems; ++k) tile_sh[1 + k * kRunsThreads + t] = v[k];
        __syncthreads();
        // run starts of >= 2 records among this thread's items: bit k for item k
        uint32_t starts = 0;
#pragma unroll
        for (int k = 0; k < kRunsItems; ++k) {
            const int e = k * kRunsThreads + t;  // place in the tile
            const int64_t q = tile + e;
            if (q + 1 < total) {  // the last record starts no run of two
                const bool start = q == 0 || !same_bucket<BAND_IN_KEY>(tile_sh[e], v[k], n32);
                if (start && same_bucket<BAND_IN_KEY>(tile_sh[e + 2], v[k], n32)) starts |= 1u << k;
            }
        }
        const uint32_t cnt = __builtin_popcount(starts);
        scan[t] = cnt;
        __syncthreads();
        for (int off = 1; off < kRunsThreads; off <<= 1) {  // inclusive scan
            const uint32_t x = t >= off ? scan[t - off] : 0u;
            __syncthreads();
            scan[t] += x;
            __syncthreads();
        }
        uint32_t slot = scan[t] - cnt;
        while (starts) {
            const int k = __builtin_ctz(starts);
            starts &= starts - 1;
            const int e0 = k * kRunsThreads + t;
            const int64_t q = tile + e0;
            // the run is measured in the staged tile; only one that reaches the tile's end
            // goes on in global memory
            const uint64_t me = tile_sh[1 + e0];
            const int64_t tend = min<int64_t>(kRunsTile, total - tile);  // records in the tile
            int64_t end = run_end<BAND_IN_KEY>([&](int64_t x) { return tile_sh[1 + x]; }, e0 + 1, tend, me, n32);
            if (end == tend && tile + tend < total)
                end = run_end<BAND_IN_KEY>([&](int64_t x) { return srec[x]; }, tile + tend - 1, total, me, n32) - tile;
            const int64_t m = end - e0;
            const uint64_t rec = ((uint64_t)q << 32) | (uint64_t)m;
            if (m <= kSmallRun) {
                reg[slot] = rec;
            } else {
                reg[slot] = 0ull;
                const uint32_t l = atomicAdd(&nlong, 1u);
                reg[kRunsCap - 1 - l] = rec;
                atomicAdd(&lpairs, (unsigned long long)((uint64_t)m * (uint64_t)(m - 1) / 2));
            }
            ++slot;
        }
        __syncthreads();
        if (t == 0) {
            const uint32_t ns = scan[kRunsThreads - 1];
            tmeta[ti] = make_uint2(ns, nlong);
            tcount[ti] = (uint64_t)ns | ((uint64_t)nlong << 32);
            tpairs[ti] = lpairs;
        }
        __syncthreads();  // scan, the LDS counters and the tile are reused by the next tile
    }
}

// After the scan over tiles (tcount, tpairs exclusive): tile ti's run starts go to
// runs[starts before ti ...], its long runs to bruns[long runs before ti ...] with their
// first flattened pair index in bpoff.  The last tile publishes the totals: counters [0] run
// starts, [1] pairs of the long runs, [2] long runs.
__global__ __launch_bounds__(kRunsThreads) void lsh_compact_kernel(
    const uint64_t *__restrict__ region, const uint2 *__restrict__ tmeta, const uint64_t *__restrict__ tcount,
    const uint64_t *__restrict__ tpairs, int64_t T, uint64_t *__restrict__ runs, uint64_t *__restrict__ bruns,
    uint64_t *__restrict__ bpoff, unsigned long long *__restrict__ counters) {
    for (int64_t ti = blockIdx.x; ti < T; ti += gridDim.x) {
        const uint2 meta = tmeta[ti];
        const uint64_t base = tcount[ti];
        const uint64_t sbase = base & 0xFFFFFFFFull, lbase = base >> 32;
        const uint64_t *reg = region + ti * kRunsCap;
        for (uint32_t x = threadIdx.x; x < meta.x; x += kRunsThreads) runs[sbase + x] = reg[x];
        if (threadIdx.x == 0) {
            uint64_t acc = tpairs[ti];
            for (uint32_t l = 0; l < meta.y; ++l) {
                const uint64_t rec = reg[kRunsCap - 1 - l];
                const uint64_t m = rec & 0xFFFFFFFFull;
                bruns[lbase + l] = rec;
                bpoff[lbase + l] = acc;
                acc += m * (m - 1) / 2;
            }
            if (ti == T - 1) {
                counters[0] = sbase + meta.x;
                counters[1] = acc;
                counters[2] = lbase + meta.y;
            }
        }
    }
}

// Tuples of rows i and j equal in band beta, and i and j in one repertoire.
__device__ __forceinline__ bool same_class(const uint64_t *__restrict__ sig, int64_t M, int r, int beta, int64_t i,
                                           int64_t j, const int64_t *__restrict__ offs, int64_t R) {
    const uint64_t *a = sig + i * M + (int64_t)beta * r;
    const uint64_t *c = sig + j * M + (int64_t)beta * r;
    bool eq = true;
    if (r == 4 && (M & 1) == 0 && ((reinterpret_cast<uintptr_t>(sig) & 15) == 0)) {
        const ulonglong2 *a2 = reinterpret_cast<const ulonglong2 *>(a), *c2 = reinterpret_cast<const ulonglong2 *>(c);
        const ulonglong2 x0 = a2[0], x1 = a2[1], y0 = c2[0], y1 = c2[1];
        eq = x0.x == y0.x && x0.y == y0.y && x1.x == y1.x && x1.y == y1.y;
    } else {
        for (int k = 0; k < r; ++k) eq &= a[k] == c[k];
    }
    return eq && (R <= 1 || rep_of(offs, R, i) == rep_of(offs, R, j));
}

// Step 3b, class ids of the members of one run (records start .. start + m - 1 of the sorted
// list, all of band beta): member k > 0 equal to the first record takes its record number;
// a member that differs from it (two tuples met by chance in the mix bits) looks for the
// first earlier member equal to it (whose own id is then the class's), else keeps its own.
__device__ __forceinline__ void class_member(const uint64_t *__restrict__ srec, int64_t start, int64_t k, uint32_t la0,
                                             int beta, uint32_t n32, const uint64_t *__restrict__ sig, int32_t M,
                                             int32_t b, int32_t r, const int64_t *__restrict__ offs, int64_t R,
                                             uint32_t *__restrict__ C) {
    const uint32_t base = (uint32_t)beta * n32;
    const uint32_t la = (uint32_t)srec[start + k];
    const int64_t i = (int64_t)(la - base);
    const int64_t i0 = (int64_t)(la0 - base);
    uint32_t cls = la;
    if (same_class(sig, M, r, beta, i, i0, offs, R)) {
        cls = la0;
    } else {
        for (int64_t q = 1; q < k; ++q) {
            const uint32_t lq = (uint32_t)srec[start + q];
            if (same_class(sig, M, r, beta, i, (int64_t)(lq - base), offs, R)) {
                cls = lq;
                break;
            }
        }
    }
    if (cls != la) C[i * class_stride(b) + beta] = cls;
}

// Short runs (the run list: (start << 32 | m), m = 0 for a slot whose run is long): one
// thread per run.  The run's records, then every member's tuple, are loaded before any
// comparison; member k's class is the first member k' < k with an equal tuple (k' = 0 but
// in runs whose tuples met by chance in the mix bits), else its own record number.
__global__ __launch_bounds__(256) void lsh_class_small_kernel(const uint64_t *__restrict__ srec, int64_t n,
                                                              const uint64_t *__restrict__ sig, int32_t M, int32_t b,
                                                              int32_t r, const int64_t *__restrict__ offs, int64_t R,
                                                              const uint64_t *__restrict__ runs,
                                                              const unsigned long long *__restrict__ counters,
                                                              uint32_t *__restrict__ C) {
    const int64_t nruns = (int64_t)counters[0];
    const uint32_t n32 = (uint32_t)n;
    const bool r4 = r == 4 && (M & 1) == 0 && ((reinterpret_cast<uintptr_t>(sig) & 15) == 0) && R <= 1;
    for (int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; q < nruns; q += (int64_t)gridDim.x * blockDim.x) {
        const uint64_t run = runs[q];
        const int m = (int)(uint32_t)run;
        if (m < 2) continue;
        const int64_t start = (int64_t)(run >> 32);
        if (!r4) {
            const uint32_t la0 = (uint32_t)srec[start];
            const int beta = (int)(la0 / n32);
            for (int k = 1; k < m; ++k) class_member(srec, start, k, la0, beta, n32, sig, M, b, r, offs, R, C);
            continue;
        }
        uint32_t la[kSmallRun];
#pragma unroll
        for (int k = 0; k < kSmallRun; ++k) la[k] = k < m ? (uint32_t)srec[start + k] : 0u;
        const int beta = (int)(la[0] / n32);
        const uint32_t base = (uint32_t)beta * n32;
        ulonglong2 t[kSmallRun][2];
#pragma unroll
        for (int k = 0; k < kSmallRun; ++k) {
            if (k < m) {
                const ulonglong2 *p = reinterpret_cast<const ulonglong2 *>(sig + (int64_t)(la[k] - base) * M + beta * 4);
                t[k][0] = p[0];
                t[k][1] = p[1];
            } else {
                t[k][0] = t[k][1] = make_ulonglong2(0ull, 0ull);
            }
        }
#pragma unroll
        for (int k = 1; k < kSmallRun; ++k) {
            if (k >= m) break;
            uint32_t cls = la[k];
#pragma unroll
            for (int q2 = 0; q2 < k; ++q2) {
                const bool eq = t[k][0].x == t[q2][0].x && t[k][0].y == t[q2][0].y && t[k][1].x == t[q2][1].x &&
                                t[k][1].y == t[q2][1].y;
                if (eq) {
                    cls = la[q2];
                    break;
                }
            }
            if (cls != la[k]) C[(int64_t)(la[k] - base) * class_stride(b) + beta] = cls;
        }
    }
}

// Long runs: one wave per run, lanes over its members.
__global__ __launch_bounds__(256) void lsh_class_long_kernel(const uint64_t *__restrict__ srec, int64_t n,
                                                             const uint64_t *__restrict__ sig, int32_t M, int32_t b,
                                                             int32_t r, const int64_t *__restrict__ offs, int64_t R,
                                                             const uint64_t *__restrict__ bruns,
                                                             const unsigned long long *__restrict__ counters,
                                                             uint32_t *__restrict__ C) {
    const int64_t nruns = (int64_t)counters[2];
    const uint32_t n32 = (uint32_t)n;
    const int lane = threadIdx.x & 63;
    const int64_t wave = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    const int64_t nwaves = ((int64_t)gridDim.x * blockDim.x) >> 6;
    for (int64_t q = wave; q < nruns; q += nwaves) {
        const uint64_t run = bruns[q];
        const int64_t m = (int64_t)(uint32_t)run;
        const int64_t start = (int64_t)(run >> 32);
        const uint32_t la0 = (uint32_t)srec[start];
        const int beta = (int)(la0 / n32);
        for (int64_t k = 1 + lane; k < m; k += 64) class_member(srec, start, k, la0, beta, n32, sig, M, b, r, offs, R, C);
    }
}

// Whether records la < lb of one run (band beta) make a candidate pair first found in this
// band: equal classes in beta, different classes in every earlier band.  i < j on return.
__device__ __forceinline__ bool pair_first_here(uint32_t la, uint32_t lb, uint32_t n32, int32_t b,
                                                const uint32_t *__restrict__ C, int64_t &i, int64_t &j) {
    const int beta = (int)(la / n32);
    if (beta >= b) return false;
    i = (int64_t)(la - (uint32_t)beta * n32);
    j = (int64_t)(lb - (uint32_t)beta * n32);  // i < j within a run
    const uint32_t *ci = C + i * class_stride(b), *cj = C + j * class_stride(b);
    {
        // the rows' words 0 .. beta as 16-byte loads, all issued before any test (rows are
        // padded to whole 16-byte words)
        const int wl = beta >> 2;
        uint4 x[8], y[8];
        const bool fits = b <= 32;
        if (fits) {
#pragma unroll
            for (int w = 0; w < 8; ++w) {
                if (w <= wl) {
                    x[w] = reinterpret_cast<const uint4 *>(ci)[w];
                    y[w] = reinterpret_cast<const uint4 *>(cj)[w];
                } else {
                    x[w] = y[w] = make_uint4(1u, 1u, 1u, 1u);  // past beta: never looked at
                }
            }
            // equal in band beta and in no earlier band: word e of the rows' XOR is zero for
            // e == beta and nonzero for every e < beta
            bool ok = true;
#pragma unroll
            for (int w = 0; w < 8; ++w) {
                const uint32_t e[4] = {x[w].x ^ y[w].x, x[w].y ^ y[w].y, x[w].z ^ y[w].z, x[w].w ^ y[w].w};
#pragma unroll
                for (int k = 0; k < 4; ++k) {
                    const int band = 4 * w + k;
                    if (band < beta) ok &= e[k] != 0u;
                    else if (band == beta) ok &= e[k] == 0u;
                }
            }
            return ok;
        }
    }
    if (ci[beta] != cj[beta]) return false;
    for (int e = 0; e < beta; ++e)
        if (ci[e] == cj[e]) return false;
    return true;
}

// Slots in the pair-key list for the threads of a block that want one: an LDS counter
// hands out block-local ranks, then one global atomic per block reserves them.  Every
// thread of the block must call it (it synchronises the block).
__device__ __forceinline__ unsigned long long block_slot(unsigned long long *count, bool want, uint32_t *lcount,
                                                         unsigned long long *gbase) {
    if (threadIdx.x == 0) *lcount = 0u;
    __syncthreads();
    const uint32_t local = want ? atomicAdd(lcount, 1u) : 0u;
    __syncthreads();
    if (threadIdx.x == 0) *gbase = *lcount ? atomicAdd(count, (unsigned long long)*lcount) : 0ull;
    __syncthreads();
    return *gbase + local;
}

constexpr int kEmitThreads = 256;

constexpr int kEmitPer = 4;                           // runs per thread of a chunk
constexpr int kEmitRuns = kEmitThreads * kEmitPer;    // runs per chunk
constexpr int kEmitBuf = 1024;                        // kept keys buffered per block

// Step 3b, short runs (<= kSmallRun records): a block takes chunks of kEmitRuns runs, scans
// their pair counts in LDS, and its threads walk the chunk's pairs in rounds of 256 (a pair
// finds its run by bisection in LDS; k-th pair of a run: y = the largest y with
// y(y-1)/2 <= k, x = k - y(y-1)/2).  Kept keys collect in LDS and leave in batches, one
// global atomic per batch.
__global__ __launch_bounds__(kEmitThreads) void lsh_emit_small_kernel(
    const uint64_t *__restrict__ srec, int64_t n, int32_t b, const uint32_t *__restrict__ C, int nb,
    const uint64_t *__restrict__ runs, const unsigned long long *__restrict__ counters, uint64_t *__restrict__ pkeys,
    int64_t cap, unsigned long long *__restrict__ count) {
    __shared__ uint32_t vend[kEmitRuns];  // inclusive prefix of the runs' pair counts
    __shared__ uint32_t rsh[kEmitRuns];  // first record of each run
    __shared__ uint64_t kbuf[kEmitBuf];
    __shared__ uint32_t wt[kEmitThreads / 64];
    __shared__ uint32_t kn;
    __shared__ unsigned long long gbase;
    const int64_t nruns = (int64_t)counters[0];
    const uint32_t n32 = (uint32_t)n;
    const int t = threadIdx.x, lane = t & 63, w = t >> 6;
    if (t == 0) kn = 0u;
    // moves the buffered keys out (all threads call it)
    auto flush = [&]() {
        __syncthreads();
        const uint32_t cnt = kn;
        if (t == 0 && cnt) gbase = atomicAdd(count, (unsigned long long)cnt);
        __syncthreads();
        for (uint32_t x = t; x < cnt; x += kEmitThreads)
            if ((int64_t)(gbase + x) < cap) pkeys[gbase + x] = kbuf[x];
        __syncthreads();
        if (t == 0) kn = 0u;
        __syncthreads();
    };
    for (int64_t tile = (int64_t)blockIdx.x * kEmitRuns; tile < nruns; tile += (int64_t)gridDim.x * kEmitRuns) {
        // thread t takes runs 4t .. 4t+3 of the chunk
        uint32_t c[kEmitPer], sum = 0;
#pragma unroll
        for (int k = 0; k < kEmitPer; ++k) {
            const int64_t q = tile + t * kEmitPer + k;
            const uint64_t run = q < nruns ? runs[q] : 0ull;
            const uint32_t m = (uint32_t)run;  // 0 for a slot whose run is long
            rsh[t * kEmitPer + k] = (uint32_t)(run >> 32);
            c[k] = m * (m - (m > 0)) / 2;
            sum += c[k];
        }
        // block inclusive scan of the thread sums: wave scan, then the wave totals
        uint32_t inc = sum;
#pragma unroll
        for (int off = 1; off < 64; off <<= 1) {
            const uint32_t o = __shfl_up(inc, off, 64);
            if (lane >= off) inc += o;
        }
        if (lane == 63) wt[w] = inc;
        __syncthreads();
        for (int ww = 0; ww < w; ++ww) inc += wt[ww];
        uint32_t run_end = inc - sum;
#pragma unroll
        for (int k = 0; k < kEmitPer; ++k) {
            run_end += c[k];
            vend[t * kEmitPer + k] = run_end;
        }
        __syncthreads();
        const uint32_t V = vend[kEmitRuns - 1];
        for (uint32_t v0 = 0; v0 < V; v0 += kEmitThreads) {
            const uint32_t v = v0 + t;
            if (v < V) {
                int lo = 0, hi = kEmitRuns - 1;  // first run with vend > v
                while (lo < hi) {
                    const int mid = (lo + hi) >> 1;
                    if (vend[mid] > v) hi = mid; else lo = mid + 1;
                }
                const uint32_t k = v - (lo ? vend[lo - 1] : 0u);
                uint32_t y = 1;
                while ((y + 1) * y / 2 <= k) ++y;  // y < kSmallRun
                const uint32_t x = k - y * (y - 1) / 2;
                const int64_t start = (int64_t)rsh[lo];
                int64_t i = 0, j = 0;
                const uint32_t la = (uint32_t)srec[start + x], lb = (uint32_t)srec[start + y];
                if (pair_first_here(la, lb, n32, b, C, i, j))
                    kbuf[atomicAdd(&kn, 1u)] = ((uint64_t)i << nb) | (uint64_t)j;
            }
            __syncthreads();
            if (kn > kEmitBuf - kEmitThreads) flush();  // room for one more round
        }
        __syncthreads();  // vend, rsh and wt are reused by the next chunk
    }
    flush();
}

// Long runs (more than kSmallRun records): one thread per (run, x < y) pair of records, the
// long runs' pairs flattened by the prefix sum of their pair counts; k-th pair of a run:
// y = the largest y with y(y-1)/2 <= k, x = k - y(y-1)/2.  A window of kEmitWin runs always
// covers a round's pairs (a long run has at least kSmallRun (kSmallRun + 1) / 2 of them).
// With at most one round of pairs per block, block b takes pairs b blockDim.x + threadIdx.x:
// one thread finds the block's first run in the global prefix, the window after it is
// staged in LDS and every thread finds its run there.  With more pairs each block takes one
// contiguous range in rounds: its first run is searched once and each next round's first
// run is found in the staged window (no round waits on the global prefix), and kept keys
// collect in LDS and leave in batches (one global atomic per batch rather than per round:
// atomics on one address serialise).  A run's pairs are consecutive, so its members'
// class-id rows are read from the cache by the threads that share them.  The kernel waits on
// loads: it is held to six waves per SIMD (80 registers) rather than the five its registers
// would otherwise allow.
constexpr int kEmitWin = 64;        // runs staged per window
constexpr int kEmitLongBuf = 4096;  // kept keys of long runs buffered per block

// Pair t of the flattened long runs, given the staged window of runs (t falls in one of
// them): its run by bisection over the staged offsets, its (x, y) by the triangular root,
// then the first-band test.
__device__ __forceinline__ bool long_pair_test(uint64_t t, const uint64_t *wpoff, const uint64_t *wrun,
                                               const uint64_t *__restrict__ srec, uint32_t n32, int32_t b,
                                               const uint32_t *__restrict__ C, int64_t &i, int64_t &j) {
    int lo = 0, hi = kEmitWin - 1;  // last staged run with poff <= t
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (wpoff[mid] <= t) lo = mid; else hi = mid - 1;
    }
    const uint64_t start = wrun[lo] >> 32;
    const uint64_t k = t - wpoff[lo];
    uint64_t y = (uint64_t)((1.0f + sqrtf(1.0f + 8.0f * (float)k)) * 0.5f);
    while (y * (y - 1) / 2 > k) --y;
    while ((y + 1) * y / 2 <= k) ++y;
    const uint64_t x = k - y * (y - 1) / 2;
    const uint32_t la = (uint32_t)srec[start + x], lb = (uint32_t)srec[start + y];
    return pair_first_here(la, lb, n32, b, C, i, j);
}

__global__ __launch_bounds__(1024) __attribute__((amdgpu_waves_per_eu(6))) void lsh_emit_long_kernel(
    const uint64_t *__restrict__ srec, int64_t n, int32_t b, const uint32_t *__restrict__ C, int nb,
    const uint64_t *__restrict__ runs, const uint64_t *__restrict__ poff, const unsigned long long *__restrict__ counters,
    uint64_t *__restrict__ pkeys, int64_t cap, unsigned long long *__restrict__ count) {
    static_assert((kSmallRun + 1) * kSmallRun / 2 * (kEmitWin - 1) >= 1024, "a window may span more runs");
    __shared__ uint32_t kn;
    __shared__ unsigned long long gbase;
    __shared__ uint64_t wrun[kEmitWin], wpoff[kEmitWin];
    __shared__ uint64_t kbuf[kEmitLongBuf];
    __shared__ int64_t wfirst;
    const int64_t nruns = (int64_t)counters[2];
    const uint64_t visits = (uint64_t)counters[1];
    const uint32_t n32 = (uint32_t)n;
    if (visits <= (uint64_t)gridDim.x * blockDim.x) {  // (uniform) at most one round per block
        const uint64_t t = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
        if ((uint64_t)blockIdx.x * blockDim.x >= visits) return;  // (the whole block)
        if (threadIdx.x == 0) {
            int64_t lo = 0, hi = nruns - 1;  // last run with poff <= the block's first pair
            const uint64_t base = (uint64_t)blockIdx.x * blockDim.x;
            while (lo < hi) {
                const int64_t mid = (lo + hi + 1) >> 1;
                if (poff[mid] <= base) lo = mid; else hi = mid - 1;
            }
            wfirst = lo;
        }
        __syncthreads();
        for (int k = threadIdx.x; k < kEmitWin; k += blockDim.x) {
            const int64_t q = wfirst + k;
            wpoff[k] = q < nruns ? poff[q] : ~0ull;
            wrun[k] = q < nruns ? runs[q] : 0ull;
        }
        __syncthreads();
        bool want = false;
        int64_t i = 0, j = 0;
        if (t < visits) want = long_pair_test(t, wpoff, wrun, srec, n32, b, C, i, j);
        const unsigned long long slot = block_slot(count, want, &kn, &gbase);  // (synchronises the block)
        if (want && (int64_t)slot < cap) pkeys[slot] = ((uint64_t)i << nb) | (uint64_t)j;
        return;
    }
    // many pairs: equal contiguous ranges
    const uint64_t per = (visits + gridDim.x - 1) / gridDim.x;
    const uint64_t v0 = (uint64_t)blockIdx.x * per, v1 = min(visits, v0 + per);
    if (v0 >= v1) return;  // (the whole block) no pairs left for it
    // kept keys collect in LDS and leave in batches: one global atomic and contiguous stores
    // per batch (all threads call it)
    auto flush = [&]() {
        __syncthreads();
        const uint32_t cnt = kn;
        if (threadIdx.x == 0 && cnt) gbase = atomicAdd(count, (unsigned long long)cnt);
        __syncthreads();
        for (uint32_t x = threadIdx.x; x < cnt; x += blockDim.x)
            if ((int64_t)(gbase + x) < cap) pkeys[gbase + x] = kbuf[x];
        __syncthreads();
        if (threadIdx.x == 0) kn = 0u;
        __syncthreads();
    };
    if (threadIdx.x == 0) {
        kn = 0u;
        int64_t lo = 0, hi = nruns - 1;  // last run with poff <= v0
        while (lo < hi) {
            const int64_t mid = (lo + hi + 1) >> 1;
            if (poff[mid] <= v0) lo = mid; else hi = mid - 1;
        }
        wfirst = lo;
    }
    __syncthreads();
    // block-uniform trip count: every thread reaches every round's barriers
    for (uint64_t base = v0; base < v1; base += blockDim.x) {
        const int64_t first = wfirst;
        for (int k = threadIdx.x; k < kEmitWin; k += blockDim.x) {
            const int64_t q = first + k;
            wpoff[k] = q < nruns ? poff[q] : ~0ull;
            wrun[k] = q < nruns ? runs[q] : 0ull;
        }
        __syncthreads();
        const uint64_t t = base + threadIdx.x;
        bool want = false;
        int64_t i = 0, j = 0;
        if (t < v1) want = long_pair_test(t, wpoff, wrun, srec, n32, b, C, i, j);
        if (want) kbuf[atomicAdd(&kn, 1u)] = ((uint64_t)i << nb) | (uint64_t)j;
        __syncthreads();  // every thread is done with the staged runs and the buffer count
        if (threadIdx.x == 0) {  // the next round's first run, among the staged ones
            const uint64_t next = base + blockDim.x;
            int lo = 0, hi = kEmitWin - 1;
            while (lo < hi) {
                const int mid = (lo + hi + 1) >> 1;
                if (wpoff[mid] <= next) lo = mid; else hi = mid - 1;
            }
            wfirst = first + lo;
        }
        __syncthreads();  // wfirst is set and the staged runs are free again
        if (kn > kEmitLongBuf - blockDim.x) flush();  // (uniform) room for one more round
    }
    flush();
}

__global__ void lsh_init_kernel(unsigned long long *count) {
    // [0] pairs, [1] spare, [2] short runs, [3] long-run pairs, [4] long runs, [5] spare
    if (blockIdx.x == 0 && threadIdx.x < 6) count[threadIdx.x] = 0ull;
}

// Publishes P, the capacity status, and the clamped pair count used by the pair sort.
__global__ void lsh_count_kernel(const unsigned long long *__restrict__ count, int64_t cap,
                                 int64_t *__restrict__ n_pairs, int32_t *__restrict__ status,
                                 int64_t *__restrict__ clamped) {
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        int64_t P = (int64_t)*count;
        if (n_pairs) *n_pairs = P;
        if (status) *status = P > cap ? SUBQUAD_ERR_CAPACITY : 0;
        *clamped = P > cap ? 0 : P;  // on overflow nothing is sorted or written
    }
}

__global__ void lsh_pairs_kernel(const uint64_t *__restrict__ skeys, const int64_t *__restrict__ clamped,
                                 int64_t cap, int nb, int32_t *__restrict__ pairs) {
    const int64_t P = *clamped;
    const uint64_t jmask = (1ull << nb) - 1ull;
    for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < P; p += (int64_t)gridDim.x * blockDim.x) {
        uint64_t k = skeys[p];
        pairs[2 * p] = (int32_t)(k >> nb);
        pairs[2 * p + 1] = (int32_t)(k & jmask);
    }
}

// row_offsets[i] = number of pairs whose first index is < i (lower bound in sorted keys).
__global__ void lsh_rows_kernel(const uint64_t *__restrict__ skeys, const int64_t *__restrict__ clamped,
                                int64_t n, int nb, int64_t *__restrict__ row_offsets) {
    const int64_t P = *clamped;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i <= n; i += (int64_t)gridDim.x * blockDim.x) {
        uint64_t key = (uint64_t)i << nb;
        int64_t lo = 0, hi = P;
        while (lo < hi) {
            int64_t mid = (lo + hi) >> 1;
            if (skeys[mid] < key) lo = mid + 1; else hi = mid;
        }
        row_offsets[i] = lo;
    }
}

struct LshLayout {
    size_t rec_a, rec_b, fp, runs, poff, pk_a, pk_b, misc, radix, total;
};

static int bits_for(int64_t n) {
    int nb = 1;
    while ((int64_t(1) << nb) < n) ++nb;
    return nb;
}

static int64_t runs_tiles(int64_t recs) { return ceil_div(recs, kRunsTile); }
// long runs (>= kSmallRun + 1 records each) in `recs` records
static int64_t long_cap(int64_t recs) { return recs / (kSmallRun + 1) + 1; }

static LshLayout lsh_layout(int64_t n, int32_t b, int64_t cap) {
    LshLayout L{};
    const int64_t recs = n * b;
    size_t off = 0;
    auto take = [&](size_t bytes) { size_t o = off; off += align_up(std::max<size_t>(bytes, 1), 256); return o; };
    L.rec_a = take(sizeof(uint64_t) * recs);
    L.rec_b = take(sizeof(uint64_t) * recs);
    L.fp = take(sizeof(uint32_t) * (size_t)n * class_stride(b));  // class ids C[n][b], rows padded
    const int64_t T = runs_tiles(recs);
    L.runs = take(sizeof(uint64_t) * (size_t)T * kRunsCap);
    L.poff = take(sizeof(uint64_t) * (size_t)(2 * long_cap(recs) + 3 * T));
    L.pk_a = take(sizeof(uint64_t) * cap);
    L.pk_b = take(sizeof(uint64_t) * cap);
    L.misc = take(128);
    L.radix = take(std::max(radix_scratch_bytes(std::max<int64_t>(recs, cap)), scan64_scratch_bytes(T)));
    L.total = off;
    return L;
}

static int lsh_validate(const uint64_t *sig, int64_t n, int32_t M, int32_t b, int32_t r, const int64_t *offs,
                        int64_t R, void *ws, size_t ws_bytes, int32_t *pairs, int64_t cap) {
    SQ_REQUIRE(n >= 0 && cap >= 0, SUBQUAD_ERR_ARG, "n and cap must be >= 0");
    SQ_REQUIRE(b >= 1 && b <= 256 && r >= 1 && (int64_t)b * r <= M && M <= 4096, SUBQUAD_ERR_ARG,
               "need 1 <= b <= 256, r >= 1, b*r <= M (b=%d r=%d M=%d)", b, r, M);
    SQ_REQUIRE(n * (int64_t)b < (int64_t(1) << 32), SUBQUAD_ERR_ARG, "n*b must be below 2^32");
    SQ_REQUIRE(n < (int64_t(1) << 31), SUBQUAD_ERR_ARG, "n must be below 2^31");
    SQ_REQUIRE(R >= 1 && (R == 1 || offs), SUBQUAD_ERR_ARG, "R >= 1 and rep_offsets required when R > 1");
    SQ_REQUIRE(n == 0 || sig, SUBQUAD_ERR_ARG, "null signature pointer");
    SQ_REQUIRE(cap == 0 || pairs, SUBQUAD_ERR_ARG, "null pairs pointer");
    SQ_REQUIRE(ws || n == 0, SUBQUAD_ERR_ARG, "null workspace");
    SQ_REQUIRE(((uintptr_t)ws & 255) == 0, SUBQUAD_ERR_ARG, "workspace must be 256-byte aligned");
    size_t need = lsh_layout(n, b, cap).total;
    SQ_REQUIRE(ws_bytes >= need, SUBQUAD_ERR_WORKSPACE, "workspace of %zu bytes, %zu needed", ws_bytes, need);
    return SUBQUAD_OK;
}

// Steps 1-3: records, sort, emission.  Leaves the raw pair keys in L.pk_a and the count in misc.
static int lsh_front(const uint64_t *sig, int64_t n, int32_t M, int32_t b, int32_t r, const int64_t *offs,
                     int64_t R, char *ws, const LshLayout &L, int64_t cap, int nb, hipStream_t st) {
    const int64_t recs = n * b;
    uint64_t *rec_a = reinterpret_cast<uint64_t *>(ws + L.rec_a);
    uint64_t *rec_b = reinterpret_cast<uint64_t *>(ws + L.rec_b);
    uint32_t *C = reinterpret_cast<uint32_t *>(ws + L.fp);
    unsigned long long *count = reinterpret_cast<unsigned long long *>(ws + L.misc);
    void *rscratch = ws + L.radix;
    const size_t rscratch_bytes = radix_scratch_bytes(std::max<int64_t>(recs, cap));

    lsh_init_kernel<<<1, 64, 0, st>>>(count);
    SQ_LAUNCHED("lsh_init_kernel");
    // Mix bits kept in the sort key: enough that a band's n records rarely share them by
    // chance (n / 2^bits <= 1/16, each such meeting costing one tuple comparison), in whole
    // radix digits, so a small repertoire sorts in fewer passes.
    const int mix_bits = record_mix_bits(n);
    const uint32_t keep = mix_bits >= 32 ? ~0u : ~((1u << (32 - mix_bits)) - 1u);
    // the band (b <= 256) goes into the cleared bits when there are any: runs then compare
    // whole key words, with no division by n
    const uint32_t band_in_key = mix_bits <= 24 ? 1u : 0u;
    const size_t lds = sizeof(uint32_t) * (kKeysTileSeqs + 1) * b;  // at most 65 KiB (b <= 256)
    static bool lds_attr = false;  // above 64 KiB the kernels must allow it (once per process)
    if (lds > 65536 && !lds_attr) {
        const int most = (int)(sizeof(uint32_t) * (kKeysTileSeqs + 1) * 256);
        SQ_HIP(hipFuncSetAttribute((const void *)lsh_keys_kernel<true>, hipFuncAttributeMaxDynamicSharedMemorySize, most));
        SQ_HIP(hipFuncSetAttribute((const void *)lsh_keys_kernel<false>, hipFuncAttributeMaxDynamicSharedMemorySize, most));
        lds_attr = true;
    }
    {
        ProfScope prof("lsh_keys_kernel", st);
        const unsigned g = (unsigned)ceil_div(n, kKeysTileSeqs);
        if (r == 4 && M % 2 == 0 && ((uintptr_t)sig & 15) == 0)
            lsh_keys_kernel<true><<<g, kKeysThreads, lds, st>>>(sig, n, M, b, r, offs, R, keep, band_in_key, rec_a, C);
        else
            lsh_keys_kernel<false><<<g, kKeysThreads, lds, st>>>(sig, n, M, b, r, offs, R, keep, band_in_key, rec_a, C);
    }
    SQ_LAUNCHED("lsh_keys_kernel");
    uint64_t *sorted = nullptr;
    int rc = radix_sort_u64(rec_a, rec_b, recs, nullptr, 64 - mix_bits, mix_bits, rscratch, rscratch_bytes, st, &sorted,
                            "sort_records");
    if (rc != SUBQUAD_OK) return rc;
    // per-tile regions, then the compact lists: the run starts in the record buffer the sort
    // left free, the long runs and their pair offsets in the poff region
    const int64_t T = runs_tiles(recs);
    uint64_t *region = reinterpret_cast<uint64_t *>(ws + L.runs);
    uint64_t *runs = sorted == rec_a ? rec_b : rec_a;
    const int64_t big_cap = long_cap(recs);
    uint64_t *bruns = reinterpret_cast<uint64_t *>(ws + L.poff);
    uint64_t *bpoff = bruns + big_cap;
    uint64_t *tcount = bpoff + big_cap;
    uint64_t *tpairs = tcount + T;
    uint2 *tmeta = reinterpret_cast<uint2 *>(tpairs + T);
    unsigned long long *counters = count + 2;  // [0] run starts, [1] long-run pairs, [2] long runs
    if (T > 0) {
        const unsigned g = (unsigned)std::min<int64_t>(T, (int64_t)device_cus() * 8);
        {
            ProfScope prof("lsh_runs_kernel", st);
            if (band_in_key)
                lsh_runs_kernel<true><<<g, kRunsThreads, 0, st>>>(sorted, recs, n, region, tmeta, tcount, tpairs);
            else
                lsh_runs_kernel<false><<<g, kRunsThreads, 0, st>>>(sorted, recs, n, region, tmeta, tcount, tpairs);
        }
        SQ_LAUNCHED("lsh_runs_kernel");
        rc = scan_exclusive_u64(tcount, T, nullptr, rscratch, st);
        if (rc != SUBQUAD_OK) return rc;
        rc = scan_exclusive_u64(tpairs, T, nullptr, rscratch, st);
        if (rc != SUBQUAD_OK) return rc;
        {
            ProfScope prof("lsh_compact_kernel", st);
            lsh_compact_kernel<<<g, kRunsThreads, 0, st>>>(region, tmeta, tcount, tpairs, T, runs, bruns, bpoff,
                                                           counters);
        }
        SQ_LAUNCHED("lsh_compact_kernel");
    }
    // exact classes inside the runs, then the emission of the short and the long runs
    {
        const unsigned g = (unsigned)((int64_t)device_cus() * 8);
        {
            // one thread per run: up to half the records start one
            const unsigned gs = (unsigned)std::min<int64_t>(ceil_div(recs / 2 + 1, 256), (int64_t)device_cus() * 64);
            ProfScope prof("lsh_class_small_kernel", st);
            lsh_class_small_kernel<<<gs, 256, 0, st>>>(sorted, n, sig, M, b, r, offs, R, runs, counters, C);
        }
        SQ_LAUNCHED("lsh_class_small_kernel");
        {
            ProfScope prof("lsh_class_long_kernel", st);
            lsh_class_long_kernel<<<g, 256, 0, st>>>(sorted, n, sig, M, b, r, offs, R, bruns, counters, C);
        }
        SQ_LAUNCHED("lsh_class_long_kernel");
    }
    uint64_t *pk = reinterpret_cast<uint64_t *>(ws + L.pk_a);
    {
        ProfScope prof("lsh_emit_small_kernel", st);
        const unsigned g = (unsigned)((int64_t)device_cus() * 8);
        lsh_emit_small_kernel<<<g, kEmitThreads, 0, st>>>(sorted, n, b, C, nb, runs, counters, pk, cap, count);
    }
    SQ_LAUNCHED("lsh_emit_small_kernel");
    {
        const int emit_threads = knob(SUBQUAD_KNOB_EMIT_THREADS);
        ProfScope prof("lsh_emit_long_kernel", st);
        const unsigned g = (unsigned)((int64_t)device_cus() * 16);
        lsh_emit_long_kernel<<<g, emit_threads, 0, st>>>(sorted, n, b, C, nb, bruns, bpoff, counters, pk, cap, count);
    }
    SQ_LAUNCHED("lsh_emit_long_kernel");
    return SUBQUAD_OK;
}

// Step 4 on `P_host` keys (or the device count when P_host < 0, sized for cap).
static int lsh_back(int64_t n, char *ws, const LshLayout &L, int64_t cap, int64_t sort_n, int nb, int32_t *pairs,
                    int64_t *row_offsets, int64_t *n_pairs_dev, int32_t *status_dev, hipStream_t st) {
    unsigned long long *count = reinterpret_cast<unsigned long long *>(ws + L.misc);
    int64_t *clamped = reinterpret_cast<int64_t *>(ws + L.misc + 64);
    lsh_count_kernel<<<1, 64, 0, st>>>(count, cap, n_pairs_dev, status_dev, clamped);
    SQ_LAUNCHED("lsh_count_kernel");
    uint64_t *sorted = reinterpret_cast<uint64_t *>(ws + L.pk_a);
    if (sort_n > 0) {
        int rc = radix_sort_u64(reinterpret_cast<uint64_t *>(ws + L.pk_a), reinterpret_cast<uint64_t *>(ws + L.pk_b),
                                sort_n, clamped, 0, 2 * nb, ws + L.radix, L.total - L.radix, st, &sorted,
                                "sort_pairs");
        if (rc != SUBQUAD_OK) return rc;
        int64_t blocks = std::min<int64_t>(ceil_div(sort_n, 256), (int64_t)device_cus() * 16);
        lsh_pairs_kernel<<<(unsigned)blocks, 256, 0, st>>>(sorted, clamped, cap, nb, pairs);
        SQ_LAUNCHED("lsh_pairs_kernel");
    }
    if (row_offsets) {
        int64_t blocks = std::min<int64_t>(ceil_div(n + 1, 256), (int64_t)device_cus() * 16);
        lsh_rows_kernel<<<(unsigned)blocks, 256, 0, st>>>(sorted, clamped, n, nb, row_offsets);
        SQ_LAUNCHED("lsh_rows_kernel");
    }
    return SUBQUAD_OK;
}

}  // namespace subquad

using namespace subquad;

extern "C" size_t subquad_lsh_workspace_bytes(int64_t n, int32_t b, int64_t cap) {
    if (n < 0 || b < 1 || cap < 0 || n * (int64_t)b >= (int64_t(1) << 32)) return 0;
    return lsh_layout(n, b, cap).total;
}

extern "C" int subquad_lsh_candidates(const uint64_t *sig, int64_t n, int32_t M, int32_t b, int32_t r,
                                      const int64_t *rep_offsets, int64_t R, void *ws, size_t ws_bytes,
                                      int32_t *pairs, int64_t *row_offsets, int64_t cap, int64_t *n_pairs,
                                      void *stream) {
    clear_error();
    SQ_REQUIRE(n_pairs, SUBQUAD_ERR_ARG, "null n_pairs");
    int rc = lsh_validate(sig, n, M, b, r, rep_offsets, R, ws, ws_bytes, pairs, cap);
    if (rc != SUBQUAD_OK) return rc;
    *n_pairs = 0;
    hipStream_t st = as_stream(stream);
    const LshLayout L = lsh_layout(n, b, cap);
    char *w = static_cast<char *>(ws);
    if (n == 0) {
        if (row_offsets) SQ_HIP(hipMemsetAsync(row_offsets, 0, sizeof(int64_t), st));
        return SUBQUAD_OK;
    }
    const int nb = bits_for(n);
    rc = lsh_front(sig, n, M, b, r, rep_offsets, R, w, L, cap, nb, st);
    if (rc != SUBQUAD_OK) return rc;
    unsigned long long P = 0;
    SQ_HIP(hipMemcpyAsync(&P, w + L.misc, sizeof(P), hipMemcpyDeviceToHost, st));
    SQ_HIP(hipStreamSynchronize(st));
    *n_pairs = (int64_t)P;
    SQ_REQUIRE((int64_t)P <= cap, SUBQUAD_ERR_CAPACITY, "%llu candidate pairs exceed the capacity %lld", P,
               (long long)cap);
    return lsh_back(n, w, L, cap, (int64_t)P, nb, pairs, row_offsets, nullptr, nullptr, st);
}

extern "C" int subquad_lsh_candidates_async(const uint64_t *sig, int64_t n, int32_t M, int32_t b, int32_t r,
                                            const int64_t *rep_offsets, int64_t R, void *ws, size_t ws_bytes,
                                            int32_t *pairs, int64_t *row_offsets, int64_t cap, int64_t *n_pairs_dev,
                                            int32_t *status_dev, void *stream) {
    clear_error();
    SQ_REQUIRE(n_pairs_dev && status_dev, SUBQUAD_ERR_ARG, "null device count or status pointer");
    int rc = lsh_validate(sig, n, M, b, r, rep_offsets, R, ws, ws_bytes, pairs, cap);
    if (rc != SUBQUAD_OK) return rc;
    SQ_REQUIRE(n > 0, SUBQUAD_ERR_ARG, "the asynchronous variant needs n > 0");
    hipStream_t st = as_stream(stream);
    const LshLayout L = lsh_layout(n, b, cap);
    char *w = static_cast<char *>(ws);
    const int nb = bits_for(n);
    rc = lsh_front(sig, n, M, b, r, rep_offsets, R, w, L, cap, nb, st);
    if (rc != SUBQUAD_OK) return rc;
    return lsh_back(n, w, L, cap, cap, nb, pairs, row_offsets, n_pairs_dev, status_dev, st);
}
