// MinHash sketches of 3-mer shingle sets (Algorithm 1, preprocessing; sketch size M,
// Sec. 4.1; Jaccard sampling error 1/sqrt(M), Appendix B).
//
// Hash family: simple tabulation h_t(a, b, c) = T[t][0][a] ^ T[t][1][b] ^ T[t][2][c] over
// 64-bit words, T filled with consecutive SplitMix64 outputs (t, then position, then
// residue) from the caller's seed.  The signature is the unsigned minimum over the set of
// distinct 3-mers; taking the minimum over every 3-mer position gives the same value.
//
// Mapping to CDNA4: one wave per sequence, lane l owns hash functions l + 64 j (j < J).
// Every block regenerates the 60*M table words into LDS as separate hi and lo 32-bit
// planes, laid out [pos][residue][lane][j], so that a lookup with a wave-uniform residue
// reads consecutive 4*J-byte words (no bank conflicts).  The sequence row is wave-uniform;
// it is fetched one sequence ahead with vector loads and kept in registers.  Stores are
// 512-byte coalesced rows of sig.
#include "common.h"

namespace subquad {

__device__ __forceinline__ uint64_t splitmix64_at(uint64_t seed, uint64_t q) {
    // Output number q (0-based) of SplitMix64 started at state `seed`: the state after
    // q + 1 golden-gamma increments, through the variant-13 finaliser.
    uint64_t z = seed + (q + 1) * 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

constexpr int kMinhashBlock = 512;

// Median of three unsigned words (one VALU instruction).
__device__ __forceinline__ uint32_t umed3(uint32_t a, uint32_t b, uint32_t c) {
    uint32_t r;
    asm("v_med3_u32 %0, %1, %2, %3" : "=v"(r) : "v"(a), "v"(b), "v"(c));
    return r;
}

// The signature word is compared as (hi, lo) 32-bit halves.  The streaming pass reads only
// the hi halves of the tables and keeps, per hash function, the smallest hi value m1, the
// second smallest m2 (v_med3 of m1, m2 and the new value) and the position of m1.  When
// m1 != m2 the minimum hash is unique in its hi half, so its lo half is the lo half at that
// position, read once at the end.  When m1 == m2 (a repeated 3-mer, or two 3-mers whose
// hashes share the hi half) that lane redoes the sequence with full 64-bit words.
template <int J>
__global__ __launch_bounds__(kMinhashBlock) void minhash3_kernel(
    const uint8_t *__restrict__ seqs, const int32_t *__restrict__ lens, int64_t n, int32_t stride,
    int32_t M, uint64_t seed, uint64_t *__restrict__ sig) {
    extern __shared__ uint32_t lds[];
    constexpr int kEntries = 3 * 20 * 64 * J;  // [pos][residue][lane][j]
    uint32_t *Thi = lds;
    uint32_t *Tlo = lds + kEntries;
    for (int e = threadIdx.x; e < kEntries; e += blockDim.x) {
        int j = e % J;
        int l = (e / J) % 64;
        int pr = e / (J * 64);  // pos * 20 + residue
        int t = l + 64 * j;
        uint64_t v = ~0ull;
        if (t < M) {
            int pos = pr / 20, res = pr % 20;
            v = splitmix64_at(seed, ((uint64_t)t * 3 + pos) * 20 + res);
        }
        Thi[e] = (uint32_t)(v >> 32);
        Tlo[e] = (uint32_t)v;
    }
    __syncthreads();

    const int lane = threadIdx.x & 63;
    const int64_t wave = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6)) +
                         (int64_t)blockIdx.x * (blockDim.x >> 6);
    const int64_t nwaves = (int64_t)gridDim.x * (blockDim.x >> 6);
    constexpr int kRole = 20 * 64 * J;  // words between position tables
    const uint32_t *Hl = Thi + lane * J;
    const uint32_t *Ll = Tlo + lane * J;

    // The sequence row (at most 64 bytes) and length come through vector loads issued one
    // sequence ahead: they wait on the vector-memory counter, which the LDS lookups of the
    // current sequence never wait on, so the next row arrives while this one is hashed.
    const int words = stride >> 2;
    uint32_t nrow[16];
    int nlen = 0;
    auto fetch = [&](int64_t k) {
        if (k < n) {
            const uint32_t *r32 = reinterpret_cast<const uint32_t *>(seqs + k * (int64_t)stride);
#pragma unroll
            for (int q = 0; q < 16; ++q) nrow[q] = q < words ? r32[q] : 0u;  // never past the row
            nlen = lens[k];
        }
    };
    fetch(wave);
    for (int64_t i = wave; i < n; i += nwaves) {
        uint32_t row[16];
#pragma unroll
        for (int q = 0; q < 16; ++q) row[q] = __builtin_amdgcn_readfirstlane(nrow[q]);
        const int L = __builtin_amdgcn_readfirstlane(nlen);
        fetch(i + nwaves);
        const int nsh = L - 2;  // shingles
        uint32_t m1[J], m2[J], arg[J];
#pragma unroll
        for (int j = 0; j < J; ++j) {
            m1[j] = ~0u;
            m2[j] = ~0u;
            arg[j] = 0;
        }
        // Four shingles per iteration: residues q .. q+5 come from two row words, and all
        // twelve lookups are issued before any is used.
#pragma unroll 1
        for (int q = 0; q < nsh; q += 4) {
            const int w = q >> 2;
            uint32_t w0 = row[0], w1 = row[1];
#pragma unroll
            for (int k = 1; k < 15; ++k) {  // wave-uniform selects of row[w], row[w + 1]
                w0 = w == k ? row[k] : w0;
                w1 = w == k ? row[k + 1] : w1;
            }
            if (w == 15) { w0 = row[15]; w1 = 0u; }
            uint32_t off[6];
#pragma unroll
            for (int k = 0; k < 6; ++k) {
                uint32_t c = k < 4 ? (w0 >> (8 * k)) & 0xFFu : (w1 >> (8 * (k - 4))) & 0xFFu;
                off[k] = (c < 20u ? c : 19u) * (64 * J);
            }
            uint32_t h[4][J];
#pragma unroll
            for (int sh = 0; sh < 4; ++sh) {
#pragma unroll
                for (int j = 0; j < J; ++j)
                    h[sh][j] = Hl[off[sh] + j] ^ Hl[kRole + off[sh + 1] + j] ^ Hl[2 * kRole + off[sh + 2] + j];
            }
            const int live = min(4, nsh - q);  // wave-uniform
#pragma unroll
            for (int sh = 0; sh < 4; ++sh) {
                if (sh < live) {
#pragma unroll
                    for (int j = 0; j < J; ++j) {
                        const uint32_t v = h[sh][j];
                        arg[j] = v < m1[j] ? (uint32_t)(q + sh) : arg[j];
                        m2[j] = umed3(m1[j], m2[j], v);
                        m1[j] = min(m1[j], v);
                    }
                }
            }
        }
        uint64_t *out = sig + i * (int64_t)M;
#pragma unroll
        for (int j = 0; j < J; ++j) {
            const int t = lane + 64 * j;
            // lo half of the winning shingle: its three residues from the row words in registers
            const uint32_t a = arg[j], wa = a >> 2;
            uint32_t lo0 = row[0], hi0 = row[1];
#pragma unroll
            for (int k = 1; k < 16; ++k) {
                lo0 = wa == (uint32_t)k ? row[k] : lo0;
                hi0 = wa == (uint32_t)k ? (k + 1 < 16 ? row[k + 1] : 0u) : hi0;
            }
            const uint32_t tri = (uint32_t)((((uint64_t)hi0 << 32) | lo0) >> (8 * (a & 3u)));
            const uint32_t a0 = min(tri & 0xFFu, 19u), a1 = min((tri >> 8) & 0xFFu, 19u), a2 = min((tri >> 16) & 0xFFu, 19u);
            uint32_t lo = Ll[a0 * (64 * J) + j] ^ Ll[kRole + a1 * (64 * J) + j] ^ Ll[2 * kRole + a2 * (64 * J) + j];
            uint64_t best = ((uint64_t)m1[j] << 32) | lo;
            if (m1[j] == m2[j]) {  // rare: exact 64-bit minimum over every position
                const uint8_t *row8 = seqs + i * (int64_t)stride;
                best = ~0ull;
                for (int q = 0; q + 3 <= L; ++q) {
                    const uint32_t b0 = min((uint32_t)row8[q], 19u);
                    const uint32_t b1 = min((uint32_t)row8[q + 1], 19u);
                    const uint32_t b2 = min((uint32_t)row8[q + 2], 19u);
                    const int o0 = b0 * (64 * J) + j, o1 = kRole + b1 * (64 * J) + j, o2 = 2 * kRole + b2 * (64 * J) + j;
                    uint64_t h = ((uint64_t)(Hl[o0] ^ Hl[o1] ^ Hl[o2]) << 32) | (Ll[o0] ^ Ll[o1] ^ Ll[o2]);
                    best = h < best ? h : best;
                }
            }
            if (t < M) out[t] = best;
        }
    }
}

template <int J>
static int launch_minhash(const uint8_t *seqs, const int32_t *lens, int64_t n, int32_t stride, int32_t M,
                          uint64_t seed, uint64_t *sig, hipStream_t st) {
    const size_t lds = 2 * sizeof(uint32_t) * 3 * 20 * 64 * J;
    static bool attr_set = false;
    if (!attr_set) {
        SQ_HIP(hipFuncSetAttribute((const void *)minhash3_kernel<J>,
                                   hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
        attr_set = true;
    }
    const int waves_per_block = kMinhashBlock / kWave;
    const int per_cu = J <= 2 ? std::min(knob(SUBQUAD_KNOB_MINHASH_BLOCKS_PER_CU), 2) : 1;  // LDS bound
    int64_t blocks = std::min<int64_t>(ceil_div(n, waves_per_block), (int64_t)device_cus() * per_cu);
    ProfScope prof("minhash3_kernel", st);
    minhash3_kernel<J><<<(unsigned)blocks, kMinhashBlock, lds, st>>>(seqs, lens, n, stride, M, seed, sig);
    SQ_LAUNCHED("minhash3_kernel");
    return SUBQUAD_OK;
}

}  // namespace subquad

using namespace subquad;

extern "C" int subquad_minhash(const uint8_t *seqs, const int32_t *lens, int64_t n, int32_t stride,
                               int32_t k, int32_t M, uint64_t seed, uint64_t *sig, void *stream) {
    clear_error();
    SQ_REQUIRE(n >= 0, SUBQUAD_ERR_ARG, "n must be >= 0");
    SQ_REQUIRE(n == 0 || (seqs && lens && sig), SUBQUAD_ERR_ARG, "null pointer argument");
    SQ_REQUIRE(k == 3, SUBQUAD_ERR_ARG, "only k = 3 shingles are implemented (got %d)", k);
    SQ_REQUIRE(M >= 1 && M <= 256, SUBQUAD_ERR_ARG, "M must be in 1..256 (got %d)", M);
    SQ_REQUIRE(stride >= 4 && stride <= 64 && stride % 4 == 0, SUBQUAD_ERR_ARG,
               "stride must be a multiple of 4 in 4..64 (got %d)", stride);
    SQ_REQUIRE(((uintptr_t)seqs & 3) == 0, SUBQUAD_ERR_ARG, "seqs must be 4-byte aligned");
    if (n == 0) return SUBQUAD_OK;
    hipStream_t st = as_stream(stream);
    if (M <= 64) return launch_minhash<1>(seqs, lens, n, stride, M, seed, sig, st);
    if (M <= 128) return launch_minhash<2>(seqs, lens, n, stride, M, seed, sig, st);
    return launch_minhash<4>(seqs, lens, n, stride, M, seed, sig, st);
}
