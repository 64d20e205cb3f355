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
// reads consecutive 4*J-byte words (no bank conflicts).  Rows reach a wave in groups of
// consecutive sequences, one coalesced load per group issued a group ahead.  Stores are
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

constexpr int kMinhashBlock = 1024;
constexpr uint32_t kPosMask = 63u;  // shingle positions 0..61 (stride <= 64)

// Median of three unsigned words (one VALU instruction).
__device__ __forceinline__ uint32_t umed3(uint32_t a, uint32_t b, uint32_t c) {
    uint32_t r;
    asm("v_med3_u32 %0, %1, %2, %3" : "=v"(r) : "v"(a), "v"(b), "v"(c));
    return r;
}

// A lane's J consecutive table words in one LDS access (8 or 16 bytes for J = 2 or 4).
template <int J>
__device__ __forceinline__ void lds_words(const uint32_t *p, uint32_t (&v)[J]) {
    if constexpr (J == 1) {
        v[0] = p[0];
    } else if constexpr (J == 2) {
        const uint2 t = *reinterpret_cast<const uint2 *>(p);
        v[0] = t.x;
        v[1] = t.y;
    } else {
        const uint4 t = *reinterpret_cast<const uint4 *>(p);
        v[0] = t.x;
        v[1] = t.y;
        v[2] = t.z;
        v[3] = t.w;
    }
}

// The signature word is compared as (hi, lo) 32-bit halves.  The streaming pass reads only
// the hi halves of the tables; per hash function it keeps the smallest and second smallest
// of the words (top 26 bits of hi | shingle position): m1 and m2 (v_med3 of m1, m2 and the
// new word), so m1 carries its own position.  When m1 and m2 differ in the top 26 bits, the
// shingle at m1's position has the strictly smallest hi half, hence the minimum hash, whose
// full 64 bits are read once at the end.  Otherwise (a repeated 3-mer, or two 3-mers whose
// hashes agree in those bits) that lane redoes the sequence with full 64-bit words, taking
// the residues from the row words the wave already holds.
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

    // Sequences go to waves in groups of G consecutive rows, G = 64 / D with D = stride / 4
    // words per row: one coalesced dword load per lane brings a whole group (lane k D + w holds
    // word w of row k), issued a group ahead; the hashing loop reads words with readlane at
    // wave-uniform indices, and each lane fetches the words around its winning shingle from
    // the lane that holds them (ds_bpermute).  The wait for that load (which on this ISA also
    // waits for the signature stores) thus comes once per group.
    const int D = stride >> 2;
    const int G = 64 / D;
    const int64_t ngroups = ceil_div(n, (int64_t)G);
    uint32_t nrow = 0u;
    int nlen = 0;
    auto fetch = [&](int64_t g) {
        nrow = 0u;
        nlen = 0;
        if (g < ngroups) {
            const int64_t base = g * G;
            const int k = lane / D;
            if (k < G && base + k < n) nrow = reinterpret_cast<const uint32_t *>(seqs + base * (int64_t)stride)[lane];
            if (lane < G && base + lane < n) nlen = lens[base + lane];
        }
    };
    fetch(wave);
    for (int64_t g = wave; g < ngroups; g += nwaves) {
        const uint32_t rowv = nrow;
        const int lenv = nlen;
        fetch(g + nwaves);
        const int64_t base = g * G;
        const int gn = (int)min((int64_t)G, n - base);
        for (int k = 0; k < gn; ++k) {
            const int64_t i = base + k;
            const int L = __builtin_amdgcn_readlane(lenv, k);
            const int kD = k * D;
            const int nsh = L - 2;  // shingles
            uint32_t m1[J], m2[J];
#pragma unroll
            for (int j = 0; j < J; ++j) {
                m1[j] = ~0u;
                m2[j] = ~0u;
            }
            // Four shingles per iteration: residues q .. q+5 come from two row words, and all
            // twelve lookups are issued before any is used.
#pragma unroll 1
            for (int q = 0; q < nsh; q += 4) {
                const int w = q >> 2;
                const uint32_t w0 = __builtin_amdgcn_readlane(rowv, kD + w);
                const uint32_t w1 = w + 1 < D ? __builtin_amdgcn_readlane(rowv, kD + w + 1) : 0u;
                uint32_t off[6];
#pragma unroll
                for (int e = 0; e < 6; ++e) {
                    uint32_t c = e < 4 ? (w0 >> (8 * e)) & 0xFFu : (w1 >> (8 * (e - 4))) & 0xFFu;
                    off[e] = (c < 20u ? c : 19u) * (64 * J);
                }
                uint32_t h[4][J];
#pragma unroll
                for (int sh = 0; sh < 4; ++sh) {
                    uint32_t t0[J], t1[J], t2[J];
                    lds_words<J>(Hl + off[sh], t0);
                    lds_words<J>(Hl + kRole + off[sh + 1], t1);
                    lds_words<J>(Hl + 2 * kRole + off[sh + 2], t2);
#pragma unroll
                    for (int j = 0; j < J; ++j) h[sh][j] = t0[j] ^ t1[j] ^ t2[j];
                }
                const int live = min(4, nsh - q);  // wave-uniform
#pragma unroll
                for (int sh = 0; sh < 4; ++sh) {
                    if (sh < live) {
#pragma unroll
                        for (int j = 0; j < J; ++j) {
                            // top 26 bits of the hi half, shingle position in the low 6
                            const uint32_t v = (h[sh][j] & ~kPosMask) | (uint32_t)(q + sh);
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
                // lo half of the winning shingle: its three residues, from the lanes holding
                // words position/4 and position/4 + 1 of this row
                const uint32_t a = m1[j] & kPosMask, wa = a >> 2;
                const uint32_t lo0 = (uint32_t)__builtin_amdgcn_ds_bpermute((int)((kD + wa) * 4), (int)rowv);
                uint32_t hi0 = (uint32_t)__builtin_amdgcn_ds_bpermute((int)((kD + wa + 1) * 4), (int)rowv);
                if (wa + 1 >= (uint32_t)D) hi0 = 0u;
                const uint32_t tri = (uint32_t)((((uint64_t)hi0 << 32) | lo0) >> (8 * (a & 3u)));
                const uint32_t a0 = min(tri & 0xFFu, 19u), a1 = min((tri >> 8) & 0xFFu, 19u),
                               a2 = min((tri >> 16) & 0xFFu, 19u);
                const int o0 = a0 * (64 * J) + j, o1 = kRole + a1 * (64 * J) + j, o2 = 2 * kRole + a2 * (64 * J) + j;
                const uint32_t hi = Hl[o0] ^ Hl[o1] ^ Hl[o2];  // the full hi half (its low 6 bits were replaced)
                const uint32_t lo = Ll[o0] ^ Ll[o1] ^ Ll[o2];
                uint64_t best = ((uint64_t)hi << 32) | lo;
                if ((m1[j] >> 6) == (m2[j] >> 6)) {  // a tie in the top bits: exact 64-bit minimum over every position
                    best = ~0ull;
                    for (int q = 0; q + 3 <= L; ++q) {  // residues from the row words (no memory access)
                        const int w = q >> 2;
                        const uint32_t wl = __builtin_amdgcn_readlane(rowv, kD + w);
                        const uint32_t wh = w + 1 < D ? __builtin_amdgcn_readlane(rowv, kD + w + 1) : 0u;
                        const uint32_t tq = (uint32_t)((((uint64_t)wh << 32) | wl) >> (8 * (q & 3)));
                        const uint32_t b0 = min(tq & 0xFFu, 19u);
                        const uint32_t b1 = min((tq >> 8) & 0xFFu, 19u);
                        const uint32_t b2 = min((tq >> 16) & 0xFFu, 19u);
                        const int e0 = b0 * (64 * J) + j, e1 = kRole + b1 * (64 * J) + j,
                                  e2 = 2 * kRole + b2 * (64 * J) + j;
                        uint64_t hh = ((uint64_t)(Hl[e0] ^ Hl[e1] ^ Hl[e2]) << 32) | (Ll[e0] ^ Ll[e1] ^ Ll[e2]);
                        best = hh < best ? hh : best;
                    }
                }
                if (t < M) out[t] = best;
            }
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
    const int64_t groups = ceil_div(n, (int64_t)(64 / (stride / 4)));  // rows per wave group: 64 / (stride / 4)
    int64_t blocks = std::min<int64_t>(ceil_div(groups, waves_per_block), (int64_t)device_cus() * per_cu);
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
