// Local alignment channel on candidate pairs: Smith-Waterman score with Gotoh affine gaps
// (the alignment affinity of Algorithm 1's affinity computation; the paper's own kernel,
// Appendix F.3, is a global edit distance, here replaced by the local alignment score).
//
//   H = max(0, H_diag + S(a_x, b_y), E, F)
//   E = max(E_left - ge, H_left - go),  F = max(F_up - ge, H_up - go),  score = max H.
//
// Formulation used on the GPU: E' = max(E, 0) and F' = max(F, 0) obey
//   E' = max(E'_left - ge, H_left - go, 0),  F' = max(F'_up - ge, H_up - go, 0),
//   H = max(H_diag + S, E', F'),
// which is the recurrence above with the 0 of H folded into the gap states (by induction:
// a negative E can only lower a maximum that already contains 0).  Every cell is then
// two v_max3, one add and three subtractions, with no minus-infinity sentinel.
//
// Mapping to CDNA4: one lane per pair (inter-pair parallelism; CDR3s are short, so a pair
// fits in registers).  The shorter sequence runs down the unrolled, register-resident
// rows (ROWS = its length rounded up to 4), the longer one across the column loop.
// Pairs are first radix-sorted by (rows bucket, longer length), so the lanes of a wave
// have the same unroll and nearly the same trip count.  Substitution scores come from an
// LDS table that packs S(a_x, c) and S(a_x+1, c) for a row pair and a column residue c
// into one 32-bit word (one ds_read per two cells).
#include <mutex>
#include <vector>

#include "common.h"
#include "radix.h"

namespace subquad {

constexpr int kAlignThreads = 256;
// Rows per bucket: a kernel of ROWS rows takes the shorter lengths in (ROWS - step, ROWS],
// step 4 from kAlignFinePairs pairs (less row padding), 8 below (half the launches).
constexpr int kAlignFinePairs = 1 << 24;
constexpr int kAlignKeyBins = 16 * 64;  // rows bucket (1..16) x longer length (1..stride <= 64)
constexpr int kMaskCode = 20;          // rows past the shorter sequence's end
constexpr int kMaskScore = -4096;
constexpr int kCodes = 21;
constexpr int kS2Words = 20 * kCodes * kCodes;

__device__ __forceinline__ int max3i(int a, int b, int c) { return max(max(a, b), c); }

// One v_max3_i32 (the compiler otherwise splits a max whose operands it knows to be
// non-negative into a signed and an unsigned max).
__device__ __forceinline__ int max3_asm(int a, int b, int c) {
    int r;
    asm("v_max3_i32 %0, %1, %2, %3" : "=v"(r) : "v"(a), "v"(b), "v"(c));
    return r;
}

__device__ __forceinline__ void pair_lengths(const int32_t *__restrict__ pairs, const int32_t *__restrict__ lens,
                                             int64_t p, int &lmin, int &lmax) {
    int la = lens[pairs[2 * p]], lb = lens[pairs[2 * p + 1]];
    lmin = min(max(la, 0), 64);
    lmax = min(max(lb, 0), 64);
    if (lmin > lmax) { int t = lmin; lmin = lmax; lmax = t; }
}

__device__ __forceinline__ bool pair_ok(const int32_t *__restrict__ pairs, int64_t n, int64_t p) {
    int32_t i = pairs[2 * p], j = pairs[2 * p + 1];
    return i >= 0 && j >= 0 && i < n && j < n;
}

// Sort key of a pair: its rows bucket (shorter length in (step(rb-1), step rb]) times
// W = stride, plus the longer length - 1 (lengths clamped to 1..W): at stride 32, 7 bits
// (step 8) or 8 (step 4), one radix pass.
__device__ __forceinline__ int align_key(int lmin, int lmax, int W, int step) {
    const int rb = (min(max(lmin, 1), W) + step - 1) / step;  // 1..ceil(W / step)
    return (rb - 1) * W + (min(max(lmax, 1), W) - 1);
}

// Bits of the largest key at stride W.
static int align_key_bits(int W, int step) {
    const int top = ((W + step - 1) / step) * W - 1;
    int b = 1;
    while ((1 << b) <= top) ++b;
    return b;
}

// Pairs to process: cap, or min(*count_dev, cap) when a producer left the count on the device.
__device__ __forceinline__ int64_t align_count(int64_t cap, const int64_t *__restrict__ count_dev) {
    if (!count_dev) return cap;
    const int64_t c = *count_dev;
    return c < 0 ? 0 : (c < cap ? c : cap);
}

__global__ __launch_bounds__(256) void align_keys_kernel(const int32_t *__restrict__ pairs,
                                                         const int32_t *__restrict__ lens, int64_t n, int64_t cap,
                                                         const int64_t *__restrict__ P_dev, int W, int step,
                                                         uint64_t *__restrict__ rec) {
    const int64_t P = align_count(cap, P_dev);
    for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < P; p += (int64_t)gridDim.x * blockDim.x) {
        int lmin = 1, lmax = 1;
        if (pair_ok(pairs, n, p)) pair_lengths(pairs, lens, p, lmin, lmax);
        rec[p] = ((uint64_t)align_key(lmin, lmax, W, step) << 32) | (uint64_t)p;
    }
}

// bin_end[k] = number of sorted records with key <= k (one thread per key, binary search).
__global__ __launch_bounds__(kAlignKeyBins) void align_bins_kernel(const uint64_t *__restrict__ srec, int64_t cap,
                                                                   const int64_t *__restrict__ P_dev,
                                                                   uint32_t *__restrict__ bin_end) {
    const int64_t P = align_count(cap, P_dev);
    const uint64_t k = threadIdx.x;
    int64_t lo = 0, hi = P;
    while (lo < hi) {
        int64_t mid = (lo + hi) >> 1;
        if ((srec[mid] >> 32) <= k) lo = mid + 1; else hi = mid;
    }
    bin_end[k] = (uint32_t)lo;
}

// Per sorted position: the pair's rows and lengths with the shorter sequence first,
// meta = (row a, row b, la | lb << 8 | swapped << 16, p), or z = ~0 for a pair with an
// index out of range.  One gather pass, so that the alignment kernel reads one coalesced
// record per pair instead of a chain of dependent loads.
constexpr uint32_t kMetaBad = 0xFFFFFFFFu;
__global__ __launch_bounds__(256) void align_meta_kernel(const uint64_t *__restrict__ srec,
                                                         const int32_t *__restrict__ pairs,
                                                         const int32_t *__restrict__ lens, int64_t n, int32_t stride,
                                                         int64_t cap, const int64_t *__restrict__ P_dev,
                                                         uint4 *__restrict__ meta) {
    const int64_t P = align_count(cap, P_dev);
    for (int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; q < P; q += (int64_t)gridDim.x * blockDim.x) {
        const uint32_t p = (uint32_t)srec[q];
        const int32_t i = pairs[2 * (int64_t)p], j = pairs[2 * (int64_t)p + 1];
        uint4 m = make_uint4(0u, 0u, kMetaBad, p);
        if (i >= 0 && j >= 0 && i < n && j < n) {
            const int li = min(max(lens[i], 0), stride), lj = min(max(lens[j], 0), stride);
            const bool swap = li > lj;
            m.x = (uint32_t)(swap ? j : i);
            m.y = (uint32_t)(swap ? i : j);
            m.z = (uint32_t)(swap ? lj : li) | (uint32_t)(swap ? li : lj) << 8 | (swap ? 1u << 16 : 0u);
        }
        meta[q] = m;
    }
}

struct AlignLayout {
    size_t ra, rb, bins, meta, radix, total;
};

static AlignLayout align_layout(int64_t P) {
    AlignLayout L{};
    size_t off = 0;
    auto take = [&](size_t bytes) { size_t o = off; off += align_up(std::max<size_t>(bytes, 1), 256); return o; };
    L.ra = take(sizeof(uint64_t) * P);
    L.rb = take(sizeof(uint64_t) * P);
    L.bins = take(sizeof(uint32_t) * kAlignKeyBins);
    L.meta = take(sizeof(uint4) * P);
    L.radix = take(radix_scratch_bytes(P));
    L.total = off;
    return L;
}

// Table offsets of the row pairs (x, x+1) of the shorter sequence: its first ROWS bytes are
// read as words, all loads issued together (word indices clamped to the row's last word,
// aw_max; bytes at x >= la are masked), instead of one dependent byte load per row.
template <int ROWS>
__device__ __forceinline__ void row_pair_codes(const uint8_t *__restrict__ arow, int la, int aw_max,
                                               uint32_t (&idx2)[ROWS / 2]) {
    constexpr int NW = (ROWS + 3) / 4;
    const uint32_t *aw = reinterpret_cast<const uint32_t *>(arow);
    uint32_t w[NW];
#pragma unroll
    for (int k = 0; k < NW; ++k) w[k] = aw[min(k, aw_max)];
#pragma unroll
    for (int k = 0; k < ROWS / 2; ++k) {
        const int x0 = 2 * k, x1 = 2 * k + 1;
        const int b0 = (int)((w[x0 >> 2] >> (8 * (x0 & 3))) & 0xFFu);
        const int b1 = (int)((w[x1 >> 2] >> (8 * (x1 & 3))) & 0xFFu);
        const int c0 = x0 < la ? min(b0, 19) : kMaskCode;
        const int c1 = x1 < la ? min(b1, 19) : kMaskCode;
        idx2[k] = (uint32_t)(c0 * kCodes + c1);
    }
}

// DP of one pair in one lane.  a: the shorter sequence (rows), b: the longer (columns).
template <int ROWS>
__device__ __forceinline__ int sw_lane(const uint8_t *__restrict__ arow, int la, const uint8_t *__restrict__ brow,
                                       int lb, const uint32_t *__restrict__ S2, int go, int ge, int aw_max) {
    // byte offsets into S2 of the row pair (x, x+1), without the column-residue part
    uint32_t idx2[ROWS / 2];
    row_pair_codes<ROWS>(arow, la, aw_max, idx2);
    int Hp[ROWS], E[ROWS], HG[ROWS];
#pragma unroll
    for (int x = 0; x < ROWS; ++x) {
        Hp[x] = 0;
        E[x] = 0;
        HG[x] = -go;
    }
    int best = 0;
    const uint32_t *bw = reinterpret_cast<const uint32_t *>(brow);
    uint32_t word = bw[0];
    for (int y0 = 0; y0 < lb; y0 += 4) {
        uint32_t cur = word;
        if (y0 + 4 < lb) word = bw[(y0 >> 2) + 1];
#pragma unroll
        for (int k4 = 0; k4 < 4; ++k4) {
            if (y0 + k4 < lb) {
                int c = min((int)((cur >> (8 * k4)) & 0xFFu), 19);
                const uint32_t *col = S2 + c * (kCodes * kCodes);
                int diag = 0, f = 0, hup_go = -go;
#pragma unroll
                for (int k = 0; k < ROWS / 2; ++k) {
                    uint32_t w = col[idx2[k]];
                    int s0 = (int)(int16_t)(w & 0xFFFFu);
                    int s1 = (int)w >> 16;
                    int hh[2];
#pragma unroll
                    for (int h2 = 0; h2 < 2; ++h2) {
                        const int x = 2 * k + h2;
                        const int s = h2 ? s1 : s0;
                        int e = max3i(E[x] - ge, HG[x], 0);
                        f = max3i(f - ge, hup_go, 0);
                        int h = max3_asm(diag + s, e, f);
                        diag = Hp[x];
                        Hp[x] = h;
                        E[x] = e;
                        HG[x] = h - go;
                        hup_go = HG[x];
                        hh[h2] = h;
                    }
                    best = max3_asm(best, hh[0], hh[1]);
                }
            }
        }
    }
    return best;
}

// Two pairs per lane in packed half precision: pair A in the low halves, pair B in the high
// halves of every register, each cell update two packed adds and one three-way packed
// maximum (v_pk_maximum3_f16) for E, F and H.  Every value the recurrence produces is an
// integer in [-(gap_open + 128), bound] with bound = (largest substitution score) x ROWS;
// the caller takes this path only when bound <= 2048, where half precision represents every
// such integer exactly, so the scores are the int32 recurrence's bit for bit.  Rows past a
// pair's shorter sequence and columns past its longer one read the mask score -2048, which
// no diagonal can lift above the non-negative gap states (bound - 2048 <= 0).
typedef _Float16 half2_t __attribute__((ext_vector_type(2)));

__device__ __forceinline__ half2_t max3h(half2_t a, half2_t b, half2_t c) {
    half2_t r;
    asm("v_pk_maximum3_f16 %0, %1, %2, %3" : "=v"(r) : "v"(a), "v"(b), "v"(c));
    return r;
}

__device__ __forceinline__ half2_t as_h2(uint32_t w) { return __builtin_bit_cast(half2_t, w); }

constexpr int kMaskCol = 20;   // column code past a pair's longer sequence (packed path)
constexpr int kHalfMask = -2048;
constexpr int kHalfBound = 2048;

// Row-pair table offsets from a shorter sequence's words already in registers (bytes at
// x >= la masked), as row_pair_codes.
template <int ROWS>
__device__ __forceinline__ void row_pair_codes_w(const uint32_t (&w)[(ROWS + 3) / 4], int la,
                                                 uint32_t (&idx2)[ROWS / 2]) {
#pragma unroll
    for (int k = 0; k < ROWS / 2; ++k) {
        const int x0 = 2 * k, x1 = 2 * k + 1;
        const int b0 = (int)((w[x0 >> 2] >> (8 * (x0 & 3))) & 0xFFu);
        const int b1 = (int)((w[x1 >> 2] >> (8 * (x1 & 3))) & 0xFFu);
        const int c0 = x0 < la ? min(b0, 19) : kMaskCode;
        const int c1 = x1 < la ? min(b1, 19) : kMaskCode;
        idx2[k] = (uint32_t)(c0 * kCodes + c1);
    }
}

constexpr int kPackedWords = 8;  // longer-sequence words held in registers (stride <= 32)

// The two pairs' DP: shorter sequences' words aw, longer sequences' words bw (registers).
template <int ROWS>
__device__ __forceinline__ void sw_lane2(const uint32_t (&awA)[(ROWS + 3) / 4], int laA,
                                         const uint32_t (&bwA0)[kPackedWords], int lbA,
                                         const uint32_t (&awB)[(ROWS + 3) / 4], int laB,
                                         const uint32_t (&bwB0)[kPackedWords], int lbB,
                                         const uint32_t *__restrict__ S2, int go, int ge, int &outA, int &outB) {
    uint32_t idxA[ROWS / 2], idxB[ROWS / 2];
    row_pair_codes_w<ROWS>(awA, laA, idxA);
    row_pair_codes_w<ROWS>(awB, laB, idxB);
    uint32_t bwA[kPackedWords], bwB[kPackedWords];
#pragma unroll
    for (int k = 0; k < kPackedWords; ++k) {
        bwA[k] = bwA0[k];
        bwB[k] = bwB0[k];
    }
    const half2_t zero = {(_Float16)0, (_Float16)0};
    const half2_t ngo = {(_Float16)(-go), (_Float16)(-go)}, nge = {(_Float16)(-ge), (_Float16)(-ge)};
    half2_t Hp[ROWS], E[ROWS], HG[ROWS];
#pragma unroll
    for (int x = 0; x < ROWS; ++x) {
        Hp[x] = zero;
        E[x] = zero;
        HG[x] = ngo;
    }
    half2_t best = zero;
    const int lb = max(lbA, lbB);
    for (int y0 = 0; y0 < lb; y0 += 4) {
        const uint32_t curA = bwA[0], curB = bwB[0];
#pragma unroll
        for (int k = 0; k + 1 < kPackedWords; ++k) {  // the next word moves to the front
            bwA[k] = bwA[k + 1];
            bwB[k] = bwB[k + 1];
        }
#pragma unroll
        for (int k4 = 0; k4 < 4; ++k4) {
            const int y = y0 + k4;
            if (y < lb) {
                const int cA = y < lbA ? min((int)((curA >> (8 * k4)) & 0xFFu), 19) : kMaskCol;
                const int cB = y < lbB ? min((int)((curB >> (8 * k4)) & 0xFFu), 19) : kMaskCol;
                const uint32_t *colA = S2 + cA * (kCodes * kCodes);
                const uint32_t *colB = S2 + cB * (kCodes * kCodes);
                half2_t diag = zero, f = zero, hup_go = ngo;
#pragma unroll
                for (int k = 0; k < ROWS / 2; ++k) {
                    const uint32_t wA = colA[idxA[k]], wB = colB[idxB[k]];
                    // row 2k: (A's score, B's score); row 2k + 1 likewise
                    const half2_t sc[2] = {as_h2(__builtin_amdgcn_perm(wB, wA, 0x05040100u)),
                                           as_h2(__builtin_amdgcn_perm(wB, wA, 0x07060302u))};
                    half2_t hh[2];
#pragma unroll
                    for (int h2 = 0; h2 < 2; ++h2) {
                        const int x = 2 * k + h2;
                        const half2_t e = max3h(E[x] + nge, HG[x], zero);
                        f = max3h(f + nge, hup_go, zero);
                        const half2_t h = max3h(diag + sc[h2], e, f);
                        diag = Hp[x];
                        Hp[x] = h;
                        E[x] = e;
                        HG[x] = h + ngo;
                        hup_go = HG[x];
                        hh[h2] = h;
                    }
                    best = max3h(best, hh[0], hh[1]);
                }
            }
        }
    }
    outA = (int)best.x;
    outB = (int)best.y;
}

// Weighted global edit distance of one pair in one lane (the paper's Appendix F.3
// recurrence with caller-given substitution costs and indel cost):
//   D[x][y] = min(D[x-1][y] + indel, D[x][y-1] + indel, D[x-1][y-1] + cost(a_x, b_y)).
// a (the shorter sequence) runs down the unrolled rows, b across the column loop; the
// answer D[la][lb] is picked out of the register column by an unrolled select.
template <int ROWS>
__device__ __forceinline__ int ed_lane(const uint8_t *__restrict__ arow, int la, const uint8_t *__restrict__ brow,
                                       int lb, const uint32_t *__restrict__ C2, int indel, int aw_max) {
    uint32_t idx2[ROWS / 2];
    row_pair_codes<ROWS>(arow, la, aw_max, idx2);
    int D[ROWS];  // D[x] holds row x + 1 of the current column
#pragma unroll
    for (int x = 0; x < ROWS; ++x) D[x] = (x + 1) * indel;  // column 0
    const uint32_t *bw = reinterpret_cast<const uint32_t *>(brow);
    uint32_t word = bw[0];
    for (int y0 = 0; y0 < lb; y0 += 4) {
        uint32_t cur = word;
        if (y0 + 4 < lb) word = bw[(y0 >> 2) + 1];
#pragma unroll
        for (int k4 = 0; k4 < 4; ++k4) {
            const int y = y0 + k4;
            if (y < lb) {
                int c = min((int)((cur >> (8 * k4)) & 0xFFu), 19);
                const uint32_t *col = C2 + c * (kCodes * kCodes);
                int diag = y * indel;        // D[0][y]
                int up = (y + 1) * indel;    // D[0][y+1]
#pragma unroll
                for (int k = 0; k < ROWS / 2; ++k) {
                    uint32_t w = col[idx2[k]];
#pragma unroll
                    for (int h2 = 0; h2 < 2; ++h2) {
                        const int x = 2 * k + h2;
                        const int cost = h2 ? (int)(w >> 16) : (int)(w & 0xFFFFu);
                        int v = min(min(diag + cost, up + indel), D[x] + indel);
                        diag = D[x];
                        D[x] = v;
                        up = v;
                    }
                }
            }
        }
    }
    int res = 0;
#pragma unroll
    for (int x = 0; x < ROWS; ++x) res = (x + 1 == la) ? D[x] : res;
    return la == 0 ? lb * indel : res;
}

// Pairs of one rows bucket (shorter length in (ROWS - step, ROWS]), taken in the length order
// (one metadata record per sorted position): the bucket's range is read from the sort's
// end offsets on the device, so the launch needs no host synchronisation.
template <int ROWS, int MODE>
__global__ __launch_bounds__(kAlignThreads) void align_kernel(const uint8_t *__restrict__ seqs,
                                                              const int32_t *__restrict__ lens, int64_t n,
                                                              int32_t stride, const int32_t *__restrict__ pairs,
                                                              int64_t P, const uint4 *__restrict__ meta,
                                                              const uint32_t *__restrict__ bin_end,
                                                              const int8_t *__restrict__ subst, int go, int ge,
                                                              int32_t *__restrict__ scores, int step) {
    const int g = ROWS / step;  // 1..16 (ROWS a multiple of step)
    int64_t lo = g > 1 ? (int64_t)bin_end[(g - 1) * stride - 1] : 0;
    int64_t hi = (int64_t)bin_end[g * stride - 1];
    if (hi > P) hi = P;
    if (lo >= hi) return;  // whole grid
    if ((int64_t)blockIdx.x * (kAlignThreads / 64) >= ceil_div(hi - lo, 64)) return;  // whole block
    __shared__ uint32_t S2[kS2Words + kCodes * kCodes];  // (+ the mask column of the packed path)
    __shared__ int8_t sub_sh[20 * 20];  // the 400 scores, loaded once (one load per thread)
    __shared__ int smax;
    if (threadIdx.x == 0) smax = -128;
    __syncthreads();
    int asym = 0, lmax = -128;
    for (int e = threadIdx.x; e < 20 * 20; e += blockDim.x) {
        const int8_t v = subst[e], vt = subst[(e % 20) * 20 + e / 20];
        sub_sh[e] = v;
        asym |= v != vt;
        lmax = max(lmax, (int)v);
    }
    atomicMax(&smax, lmax);
    // A symmetric matrix (BLOSUM, PAM) needs one pass.  An asymmetric one takes a second pass
    // over the block's pairs: the first aligns the pairs kept in (i, j) order, the second
    // those whose operands were swapped (the longer i runs across the columns), with the
    // table of the transposed matrix, since S(a_x, b_y) then reads S(col, row).
    asym = __syncthreads_or(asym);
    const int lane = threadIdx.x & 63;
    // Two pairs per lane in packed half precision when every score of the bucket is an
    // integer half precision holds exactly (symmetric matrix, ROWS <= 32 for the registers).
    if (MODE == 0 && !asym && ROWS <= 32 && stride <= 4 * kPackedWords && max(smax, 0) * ROWS <= kHalfBound) {
        for (int e = threadIdx.x; e < kS2Words + kCodes * kCodes; e += blockDim.x) {
            const int c = e / (kCodes * kCodes);
            const int rem = e - c * (kCodes * kCodes);
            const int a0 = rem / kCodes, a1 = rem - a0 * kCodes;
            const int s0 = (a0 < 20 && c < 20) ? (int)sub_sh[a0 * 20 + c] : kHalfMask;
            const int s1 = (a1 < 20 && c < 20) ? (int)sub_sh[a1 * 20 + c] : kHalfMask;
            const half2_t v = {(_Float16)s0, (_Float16)s1};
            S2[e] = __builtin_bit_cast(uint32_t, v);
        }
        __syncthreads();
        const int64_t nw2 = ceil_div(hi - lo, 128);
        const int64_t wave0h = (int64_t)blockIdx.x * (kAlignThreads / 64) + (threadIdx.x >> 6);
        const int64_t wsteph = (int64_t)gridDim.x * (kAlignThreads / 64);
        constexpr int NA = (ROWS + 3) / 4;
        const int D = stride >> 2;  // words per row (<= kPackedWords here)
        // lane l takes sorted positions 2l and 2l + 1 of its wave's 128 (neighbours in the
        // length order, so the two pairs' loops have nearly the same trip counts)
        auto meta_at = [&](int64_t wv, int u) {
            const int64_t idx = lo + wv * 128 + 2 * lane + u;
            return (wv < nw2 && idx < hi) ? meta[idx] : make_uint4(0u, 0u, kMetaBad, 0u);
        };
        // the rows' words (a pair out of range reads row 0; its result is not stored)
        auto rows_for = [&](const uint4 (&m)[2], uint32_t (&aw)[2][NA], uint32_t (&bw)[2][kPackedWords]) {
#pragma unroll
            for (int u = 0; u < 2; ++u) {
                const bool ok = m[u].z != kMetaBad;
                const uint32_t *ra = reinterpret_cast<const uint32_t *>(seqs + (ok ? (int64_t)m[u].x : 0) * stride);
                const uint32_t *rb = reinterpret_cast<const uint32_t *>(seqs + (ok ? (int64_t)m[u].y : 0) * stride);
#pragma unroll
                for (int w = 0; w < NA; ++w) aw[u][w] = ra[min(w, D - 1)];
#pragma unroll
                for (int w = 0; w < kPackedWords; ++w) bw[u][w] = w < D ? rb[w] : 0u;
            }
        };
        // software pipeline: the next iteration's rows and the one after's records are loaded
        // while this one computes
        uint4 mc[2] = {meta_at(wave0h, 0), meta_at(wave0h, 1)};
        uint4 mn[2] = {meta_at(wave0h + wsteph, 0), meta_at(wave0h + wsteph, 1)};
        uint32_t ac[2][NA], bc[2][kPackedWords];
        rows_for(mc, ac, bc);
        for (int64_t wv = wave0h; wv < nw2; wv += wsteph) {
            uint32_t an[2][NA], bn[2][kPackedWords];
            rows_for(mn, an, bn);
            const uint4 mnn[2] = {meta_at(wv + 2 * wsteph, 0), meta_at(wv + 2 * wsteph, 1)};
            const bool ok0 = mc[0].z != kMetaBad, ok1 = mc[1].z != kMetaBad;
            // a pair with an index out of range scores -1 (positions past the bucket carry no pair)
            const int64_t i0 = lo + wv * 128 + 2 * lane;
            if (!ok0 && i0 < hi) scores[mc[0].w] = -1;
            if (!ok1 && i0 + 1 < hi) scores[mc[1].w] = -1;
            if (ok0 || ok1) {
                const int laA = ok0 ? min((int)(mc[0].z & 0xFFu), ROWS) : 0, lbA = ok0 ? (int)((mc[0].z >> 8) & 0xFFu) : 0;
                const int laB = ok1 ? min((int)(mc[1].z & 0xFFu), ROWS) : 0, lbB = ok1 ? (int)((mc[1].z >> 8) & 0xFFu) : 0;
                int sa = 0, sb = 0;
                sw_lane2<ROWS>(ac[0], laA, bc[0], lbA, ac[1], laB, bc[1], lbB, S2, go, ge, sa, sb);
                if (ok0) scores[mc[0].w] = sa;
                if (ok1) scores[mc[1].w] = sb;
            }
#pragma unroll
            for (int u = 0; u < 2; ++u) {
                mc[u] = mn[u];
                mn[u] = mnn[u];
#pragma unroll
                for (int w = 0; w < NA; ++w) ac[u][w] = an[u][w];
#pragma unroll
                for (int w = 0; w < kPackedWords; ++w) bc[u][w] = bn[u][w];
            }
        }
        return;
    }
    const int64_t nw = ceil_div(hi - lo, 64);
    const int64_t wave0 = (int64_t)blockIdx.x * (kAlignThreads / 64) + (threadIdx.x >> 6);
    const int64_t wstep = (int64_t)gridDim.x * (kAlignThreads / 64);
    for (int pass = 0; pass <= asym; ++pass) {
        if (pass) __syncthreads();  // every wave is done with the first pass's table
        for (int e = threadIdx.x; e < kS2Words; e += blockDim.x) {
            int c = e / (kCodes * kCodes);
            int rem = e - c * (kCodes * kCodes);
            int a0 = rem / kCodes, a1 = rem - a0 * kCodes;
            const int i0 = pass ? c * 20 + a0 : a0 * 20 + c, i1 = pass ? c * 20 + a1 : a1 * 20 + c;
            int s0, s1;
            if (MODE == 0) {
                s0 = a0 < 20 ? (int)sub_sh[i0] : kMaskScore;
                s1 = a1 < 20 ? (int)sub_sh[i1] : kMaskScore;
            } else {  // costs; rows past the end are never read back
                s0 = a0 < 20 ? (int)sub_sh[i0] : 0;
                s1 = a1 < 20 ? (int)sub_sh[i1] : 0;
            }
            S2[e] = ((uint32_t)(uint16_t)(int16_t)s0) | ((uint32_t)(uint16_t)(int16_t)s1 << 16);
        }
        __syncthreads();
        for (int64_t wv = wave0; wv < nw; wv += wstep) {
            const int64_t idx = lo + wv * 64 + lane;
            if (idx >= hi) continue;
            const uint4 m = meta[idx];
            const int64_t p = m.w;
            if (m.z == kMetaBad) {
                if (pass == 0) scores[p] = -1;
                continue;
            }
            const bool swap = (m.z >> 16) & 1u;
            if (asym && swap != (pass == 1)) continue;
            const uint8_t *arow = seqs + (int64_t)m.x * stride, *brow = seqs + (int64_t)m.y * stride;
            const int la = (int)(m.z & 0xFFu), lb = (int)((m.z >> 8) & 0xFFu);
            if (MODE == 0) scores[p] = sw_lane<ROWS>(arow, min(la, ROWS), brow, lb, S2, go, ge, (stride >> 2) - 1);
            else scores[p] = ed_lane<ROWS>(arow, min(la, ROWS), brow, lb, S2, go, (stride >> 2) - 1);
        }
    }
}

__global__ __launch_bounds__(256) void self_scores_kernel(const uint8_t *__restrict__ seqs,
                                                          const int32_t *__restrict__ lens, int64_t n,
                                                          int32_t stride, const int8_t *__restrict__ subst,
                                                          int32_t *__restrict__ self) {
    __shared__ int diag[20];
    if (threadIdx.x < 20) diag[threadIdx.x] = subst[threadIdx.x * 21];
    __syncthreads();
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        const uint8_t *row = seqs + i * stride;
        int L = min(lens[i], stride), s = 0;
        for (int x = 0; x < L; ++x) s += diag[min((int)row[x], 19)];
        self[i] = s;
    }
}

}  // namespace subquad

using namespace subquad;

extern "C" int subquad_self_scores(const uint8_t *seqs, const int32_t *lens, int64_t n, int32_t stride,
                                   const int8_t *subst, int32_t *self, void *stream) {
    clear_error();
    SQ_REQUIRE(n >= 0, SUBQUAD_ERR_ARG, "n must be >= 0");
    SQ_REQUIRE(n == 0 || (seqs && lens && subst && self), SUBQUAD_ERR_ARG, "null pointer argument");
    SQ_REQUIRE(stride >= 1 && stride <= 4096, SUBQUAD_ERR_ARG, "stride out of range");
    if (n == 0) return SUBQUAD_OK;
    hipStream_t st = as_stream(stream);
    int64_t blocks = std::min<int64_t>(ceil_div(n, 256), (int64_t)device_cus() * 16);
    self_scores_kernel<<<(unsigned)blocks, 256, 0, st>>>(seqs, lens, n, stride, subst, self);
    SQ_LAUNCHED("self_scores_kernel");
    return SUBQUAD_OK;
}

// The length sort needs P + 512 words of scratch; it is taken from a stream-ordered
// allocation only when the caller passes no workspace (the plain entry point below).
// P is the number of pairs, or with P_dev the capacity and *P_dev (read on the device) the
// number.
static int align_run(const uint8_t *seqs, const int32_t *lens, int64_t n, int32_t stride, const int32_t *pairs, int64_t P,
                     const int8_t *subst, int go, int ge, int32_t *scores, uint32_t *scratch, hipStream_t st,
                     int mode = 0, const int64_t *P_dev = nullptr) {
    // Length sort: records (bucket key << 32 | p) sorted on their key bits (7 at stride 32)
    // by the stable radix sort; then bin_end[k] = first position whose key exceeds k.
    char *base = reinterpret_cast<char *>(scratch);
    const AlignLayout L = align_layout(P);
    uint64_t *ra = reinterpret_cast<uint64_t *>(base + L.ra);
    uint64_t *rb = reinterpret_cast<uint64_t *>(base + L.rb);
    uint32_t *hist = reinterpret_cast<uint32_t *>(base + L.bins);
    const int64_t blocks = std::min<int64_t>(ceil_div(P, 256), (int64_t)device_cus() * 8);
    const int step = P >= kAlignFinePairs ? 4 : 8;  // rows per bucket
    align_keys_kernel<<<(unsigned)blocks, 256, 0, st>>>(pairs, lens, n, P, P_dev, stride, step, ra);
    SQ_LAUNCHED("align_keys_kernel");
    uint64_t *sorted = nullptr;
    int rc = radix_sort_u64(ra, rb, P, P_dev, 32, align_key_bits(stride, step), base + L.radix, L.total - L.radix, st,
                            &sorted, "sort_lengths");
    if (rc != SUBQUAD_OK) return rc;
    align_bins_kernel<<<1, kAlignKeyBins, 0, st>>>(sorted, P, P_dev, hist);
    SQ_LAUNCHED("align_bins_kernel");
    uint4 *meta = reinterpret_cast<uint4 *>(base + L.meta);
    align_meta_kernel<<<(unsigned)blocks, 256, 0, st>>>(sorted, pairs, lens, n, stride, P, P_dev, meta);
    SQ_LAUNCHED("align_meta_kernel");
    const int64_t waves = ceil_div(P, 64);
    // persistent blocks: no more than the chip holds at once for the bucket's kernel (a second
    // round of blocks would leave a tail), and no more than the knob asks for
    auto ablocks = [&](const void *kernel) {
        const int per_cu = std::min(knob(SUBQUAD_KNOB_ALIGN_BLOCKS_PER_CU), resident_blocks_per_cu(kernel));
        return (unsigned)std::min<int64_t>(ceil_div(waves, kAlignThreads / 64), (int64_t)device_cus() * per_cu);
    };
    const uint32_t *bin_end = hist;
    if (mode == 0) {
        ProfScope prof("align_kernel", st);
#define SQ_ROWS(R)                                                                                             \
    align_kernel<R, 0><<<ablocks((const void *)align_kernel<R, 0>), kAlignThreads, 0, st>>>(                   \
        seqs, lens, n, stride, pairs, P, meta, bin_end, subst, go, ge, scores, step);
        if (step == 4) { SQ_ROWS(4) SQ_ROWS(12) SQ_ROWS(20) SQ_ROWS(28) }
        SQ_ROWS(8) SQ_ROWS(16) SQ_ROWS(24) SQ_ROWS(32)
        if (stride > 32) {
            if (step == 4) { SQ_ROWS(36) SQ_ROWS(44) SQ_ROWS(52) SQ_ROWS(60) }
            SQ_ROWS(40) SQ_ROWS(48) SQ_ROWS(56) SQ_ROWS(64)
        }
#undef SQ_ROWS
    } else {
        ProfScope prof("edit_kernel", st);
#define SQ_ROWS(R)                                                                                             \
    align_kernel<R, 1><<<ablocks((const void *)align_kernel<R, 1>), kAlignThreads, 0, st>>>(                   \
        seqs, lens, n, stride, pairs, P, meta, bin_end, subst, go, ge, scores, step);
        if (step == 4) { SQ_ROWS(4) SQ_ROWS(12) SQ_ROWS(20) SQ_ROWS(28) }
        SQ_ROWS(8) SQ_ROWS(16) SQ_ROWS(24) SQ_ROWS(32)
        if (stride > 32) {
            if (step == 4) { SQ_ROWS(36) SQ_ROWS(44) SQ_ROWS(52) SQ_ROWS(60) }
            SQ_ROWS(40) SQ_ROWS(48) SQ_ROWS(56) SQ_ROWS(64)
        }
#undef SQ_ROWS
    }
    SQ_LAUNCHED("align_kernel");
    return SUBQUAD_OK;
}

extern "C" size_t subquad_align_workspace_bytes(int64_t P) {
    if (P < 0) return 0;
    return align_layout(std::max<int64_t>(P, 1)).total;
}

extern "C" int subquad_align_batch_ws(const uint8_t *seqs, const int32_t *lens, int64_t n, int32_t stride,
                                      const int32_t *pairs, int64_t P, const int8_t *subst, int32_t gap_open,
                                      int32_t gap_extend, int32_t *scores, void *ws, size_t ws_bytes,
                                      void *stream) {
    clear_error();
    SQ_REQUIRE(n >= 0 && P >= 0, SUBQUAD_ERR_ARG, "n and P must be >= 0");
    SQ_REQUIRE(P == 0 || (seqs && lens && pairs && subst && scores), SUBQUAD_ERR_ARG, "null pointer argument");
    SQ_REQUIRE(stride >= 4 && stride <= 64 && stride % 4 == 0, SUBQUAD_ERR_ARG,
               "stride must be a multiple of 4 in 4..64 (got %d)", stride);
    SQ_REQUIRE(gap_extend >= 0 && gap_open >= gap_extend && gap_open <= 1000, SUBQUAD_ERR_ARG,
               "need 0 <= gap_extend <= gap_open <= 1000");
    SQ_REQUIRE(P < (int64_t(1) << 32), SUBQUAD_ERR_ARG, "P must be below 2^32");
    if (P == 0) return SUBQUAD_OK;
    SQ_REQUIRE(ws && ws_bytes >= subquad_align_workspace_bytes(P), SUBQUAD_ERR_WORKSPACE,
               "alignment workspace too small");
    return align_run(seqs, lens, n, stride, pairs, P, subst, gap_open, gap_extend, scores, static_cast<uint32_t *>(ws),
                     as_stream(stream));
}

extern "C" int subquad_align_batch(const uint8_t *seqs, const int32_t *lens, int64_t n, int32_t stride,
                                   const int32_t *pairs, int64_t P, const int8_t *subst, int32_t gap_open,
                                   int32_t gap_extend, int32_t *scores, void *stream) {
    clear_error();
    SQ_REQUIRE(n >= 0 && P >= 0, SUBQUAD_ERR_ARG, "n and P must be >= 0");
    if (P == 0) return SUBQUAD_OK;
    hipStream_t st = as_stream(stream);
    size_t bytes = subquad_align_workspace_bytes(P);
    void *ws = nullptr;
    SQ_HIP(hipMallocAsync(&ws, bytes, st));
    int rc = subquad_align_batch_ws(seqs, lens, n, stride, pairs, P, subst, gap_open, gap_extend, scores, ws, bytes,
                                    stream);
    hipError_t fe = hipFreeAsync(ws, st);
    if (rc != SUBQUAD_OK) return rc;
    SQ_HIP(fe);
    return SUBQUAD_OK;
}

extern "C" int subquad_align_batch_dev(const uint8_t *seqs, const int32_t *lens, int64_t n, int32_t stride,
                                       const int32_t *pairs, int64_t cap, const int64_t *n_pairs_dev,
                                       const int8_t *subst, int32_t gap_open, int32_t gap_extend, int32_t *scores,
                                       void *ws, size_t ws_bytes, void *stream) {
    clear_error();
    SQ_REQUIRE(n >= 0 && cap >= 0, SUBQUAD_ERR_ARG, "n and cap must be >= 0");
    SQ_REQUIRE(cap == 0 || (seqs && lens && pairs && subst && scores && n_pairs_dev), SUBQUAD_ERR_ARG,
               "null pointer argument");
    SQ_REQUIRE(stride >= 4 && stride <= 64 && stride % 4 == 0, SUBQUAD_ERR_ARG,
               "stride must be a multiple of 4 in 4..64 (got %d)", stride);
    SQ_REQUIRE(gap_extend >= 0 && gap_open >= gap_extend && gap_open <= 1000, SUBQUAD_ERR_ARG,
               "need 0 <= gap_extend <= gap_open <= 1000");
    SQ_REQUIRE(cap < (int64_t(1) << 32), SUBQUAD_ERR_ARG, "cap must be below 2^32");
    if (cap == 0) return SUBQUAD_OK;
    SQ_REQUIRE(ws && ws_bytes >= subquad_align_workspace_bytes(cap), SUBQUAD_ERR_WORKSPACE,
               "alignment workspace too small");
    return align_run(seqs, lens, n, stride, pairs, cap, subst, gap_open, gap_extend, scores, static_cast<uint32_t *>(ws),
                     as_stream(stream), 0, n_pairs_dev);
}

// Allocation-free variant: the length sort's scratch is a file-scope device array that each
// GPU holds from the library's first use on it until the process ends.  In host code the
// array's name is only a stand-in, so its device address is looked up once per device
// (hipGetSymbolAddress, with that device current) and only that address reaches kernels.
constexpr int64_t kNoAllocMaxPairs = SUBQUAD_ALIGN_NOALLOC_MAX_PAIRS;
constexpr size_t kNoAllocScratchBytes = size_t(33) << 20;  // >= align_layout(kNoAllocMaxPairs).total
static __device__ __align__(256) uint8_t scratch[kNoAllocScratchBytes];

static int noalloc_scratch(uint32_t **out) {
    static std::mutex mu;
    static std::vector<void *> ptrs;
    int dev = 0;
    SQ_HIP(hipGetDevice(&dev));
    std::lock_guard<std::mutex> lk(mu);
    if ((int)ptrs.size() <= dev) ptrs.resize(dev + 1, nullptr);
    if (!ptrs[dev]) {
        void *ptr = nullptr;
        SQ_HIP(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)));
        SQ_REQUIRE(ptr != nullptr, SUBQUAD_ERR_HIP, "no device address for the alignment scratch array");
        ptrs[dev] = ptr;
    }
    *out = static_cast<uint32_t *>(ptrs[dev]);
    return SUBQUAD_OK;
}

extern "C" int subquad_align_batch_noalloc(const uint8_t *seqs, const int32_t *lens, int64_t n, int32_t stride,
                                           const int32_t *pairs, int64_t P, const int8_t *subst, int32_t gap_open,
                                           int32_t gap_extend, int32_t *scores, void *stream) {
    clear_error();
    SQ_REQUIRE(n >= 0 && P >= 0, SUBQUAD_ERR_ARG, "n and P must be >= 0");
    SQ_REQUIRE(P <= kNoAllocMaxPairs, SUBQUAD_ERR_ARG,
               "subquad_align_batch_noalloc takes at most %lld pairs (got %lld); use subquad_align_batch_ws",
               (long long)kNoAllocMaxPairs, (long long)P);
    SQ_REQUIRE(P == 0 || (seqs && lens && pairs && subst && scores), SUBQUAD_ERR_ARG, "null pointer argument");
    SQ_REQUIRE(stride >= 4 && stride <= 64 && stride % 4 == 0, SUBQUAD_ERR_ARG,
               "stride must be a multiple of 4 in 4..64 (got %d)", stride);
    SQ_REQUIRE(gap_extend >= 0 && gap_open >= gap_extend && gap_open <= 1000, SUBQUAD_ERR_ARG,
               "need 0 <= gap_extend <= gap_open <= 1000");
    if (P == 0) return SUBQUAD_OK;
    SQ_REQUIRE(align_layout(P).total <= kNoAllocScratchBytes, SUBQUAD_ERR_WORKSPACE,
               "alignment scratch array too small for %lld pairs", (long long)P);
    uint32_t *ws = nullptr;
    const int rc = noalloc_scratch(&ws);
    if (rc != SUBQUAD_OK) return rc;
    return align_run(seqs, lens, n, stride, pairs, P, subst, gap_open, gap_extend, scores, ws, as_stream(stream));
}

extern "C" int subquad_edit_cost_matrix(const int8_t *subst, int8_t *cost) {
    clear_error();
    SQ_REQUIRE(subst && cost, SUBQUAD_ERR_ARG, "null pointer argument");
    for (int a = 0; a < 20; ++a)
        for (int b = 0; b < 20; ++b) cost[a * 20 + b] = (int8_t)(a == b ? 0 : (subst[a * 20 + b] > 0 ? 1 : 2));
    return SUBQUAD_OK;
}

extern "C" int subquad_edit_batch_ws(const uint8_t *seqs, const int32_t *lens, int64_t n, int32_t stride,
                                     const int32_t *pairs, int64_t P, const int8_t *cost, int32_t indel,
                                     int32_t *dist, void *ws, size_t ws_bytes, void *stream) {
    clear_error();
    SQ_REQUIRE(n >= 0 && P >= 0, SUBQUAD_ERR_ARG, "n and P must be >= 0");
    SQ_REQUIRE(P == 0 || (seqs && lens && pairs && cost && dist), SUBQUAD_ERR_ARG, "null pointer argument");
    SQ_REQUIRE(stride >= 4 && stride <= 64 && stride % 4 == 0, SUBQUAD_ERR_ARG,
               "stride must be a multiple of 4 in 4..64 (got %d)", stride);
    SQ_REQUIRE(indel >= 0 && indel <= 1000, SUBQUAD_ERR_ARG, "indel must be in 0..1000");
    SQ_REQUIRE(P < (int64_t(1) << 32), SUBQUAD_ERR_ARG, "P must be below 2^32");
    if (P == 0) return SUBQUAD_OK;
    SQ_REQUIRE(ws && ws_bytes >= subquad_align_workspace_bytes(P), SUBQUAD_ERR_WORKSPACE,
               "alignment workspace too small");
    return align_run(seqs, lens, n, stride, pairs, P, cost, indel, 0, dist, static_cast<uint32_t *>(ws),
                     as_stream(stream), 1);
}
