// MinHash sketches of 3-mer shingle sets (Algorithm 1, preprocessing; sketch size M,
// Sec. 4.1; Jaccard sampling error 1/sqrt(M), Appendix B).
//
// Hash family: simple tabulation h_t(a, b, c) = T[t][0][a] ^ T[t][1][b] ^ T[t][2][c] over
// 64-bit words, T filled with consecutive SplitMix64 outputs (t, then position, then
// residue) from the caller's seed.  The signature is the unsigned minimum over the set of
// distinct 3-mers; taking the minimum over every 3-mer position gives the same value.
//
// Mapping to CDNA4: one wave per sequence, lane l owns hash functions l + 64 j (j < J).
// Every block regenerates the 60*M table words into LDS, laid out [pos][residue][lane][j]
// so that a lookup with a wave-uniform residue reads consecutive 8*J-byte words (no bank
// conflicts, one ds_read_b64/b128 per lookup).  The sequence row is wave-uniform and comes
// through scalar loads.  Stores are 512-byte coalesced rows of sig.
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

template <int J>
__global__ __launch_bounds__(kMinhashBlock) void minhash3_kernel(
    const uint8_t *__restrict__ seqs, const int32_t *__restrict__ lens, int64_t n, int32_t stride,
    int32_t M, uint64_t seed, uint64_t *__restrict__ sig) {
    extern __shared__ uint64_t T[];  // [3][20][64][J]
    constexpr int kEntries = 3 * 20 * 64 * J;
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
        T[e] = v;
    }
    __syncthreads();

    const int lane = threadIdx.x & 63;
    const int64_t wave = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6)) +
                         (int64_t)blockIdx.x * (blockDim.x >> 6);
    const int64_t nwaves = (int64_t)gridDim.x * (blockDim.x >> 6);
    const uint64_t *Tl = T + lane * J;
    constexpr int kRole = 20 * 64 * J;  // words between position tables

    for (int64_t i = wave; i < n; i += nwaves) {
        const uint32_t *row = reinterpret_cast<const uint32_t *>(seqs + i * (int64_t)stride);
        const int L = __builtin_amdgcn_readfirstlane(lens[i]);
        const int words = stride >> 2;
        uint64_t mn[J], x01[J], r0p[J];
#pragma unroll
        for (int j = 0; j < J; ++j) { mn[j] = ~0ull; x01[j] = 0; r0p[j] = 0; }
        int p = 0;
#pragma unroll 1
        for (int w = 0; w < words && p < L; ++w) {
            uint32_t word = __builtin_amdgcn_readfirstlane(row[w]);
#pragma unroll
            for (int k = 0; k < 4; ++k, ++p) {
                if (p >= L) break;
                uint32_t c = (word >> (8 * k)) & 0xFFu;
                c = c < 20u ? c : 19u;
                const uint64_t *base = Tl + c * (64 * J);
#pragma unroll
                for (int j = 0; j < J; ++j) {
                    uint64_t r0 = base[j];
                    uint64_t r1 = base[kRole + j];
                    uint64_t r2 = base[2 * kRole + j];
                    if (p >= 2) {
                        uint64_t h = x01[j] ^ r2;  // shingle starting at p - 2
                        mn[j] = h < mn[j] ? h : mn[j];
                    }
                    x01[j] = r0p[j] ^ r1;  // R0[p-1] ^ R1[p], shingle starting at p - 1
                    r0p[j] = r0;
                }
            }
        }
        uint64_t *out = sig + i * (int64_t)M;
#pragma unroll
        for (int j = 0; j < J; ++j) {
            int t = lane + 64 * j;
            if (t < M) out[t] = mn[j];
        }
    }
}

template <int J>
static int launch_minhash(const uint8_t *seqs, const int32_t *lens, int64_t n, int32_t stride, int32_t M,
                          uint64_t seed, uint64_t *sig, hipStream_t st) {
    const size_t lds = sizeof(uint64_t) * 3 * 20 * 64 * J;
    static bool attr_set = false;
    if (!attr_set) {
        SQ_HIP(hipFuncSetAttribute((const void *)minhash3_kernel<J>,
                                   hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
        attr_set = true;
    }
    const int waves_per_block = kMinhashBlock / kWave;
    const int per_cu = J <= 2 ? 2 : 1;
    int64_t blocks = std::min<int64_t>(ceil_div(n, waves_per_block), (int64_t)device_cus() * per_cu);
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
    if (n == 0) return SUBQUAD_OK;
    hipStream_t st = as_stream(stream);
    if (M <= 64) return launch_minhash<1>(seqs, lens, n, stride, M, seed, sig, st);
    if (M <= 128) return launch_minhash<2>(seqs, lens, n, stride, M, seed, sig, st);
    return launch_minhash<4>(seqs, lens, n, stride, M, seed, sig, st);
}
