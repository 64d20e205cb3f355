// MinHash sketches of 3-mer shingle sets (Algorithm 1, preprocessing; sketch size M,
// Sec. 4.1; Jaccard sampling error 1/sqrt(M), Appendix B).
//
// Hash family: simple tabulation h_t(a, b, c) = T[t][0][a] ^ T[t][1][b] ^ T[t][2][c] over
// 64-bit words, T filled with consecutive SplitMix64 outputs (t, then position, then
// residue) from the caller's seed.  The signature is the unsigned minimum over the set of
// distinct 3-mers; taking the minimum over every 3-mer position gives the same value.
//
// Mapping to CDNA4: one wave per sequence, lane l owns hash functions l + 64 q.  Every block
// regenerates the 60*M table words into LDS (full hi and lo planes, plus the top 16 bits of
// the hi halves packed two hash functions to a word), laid out [residue][position][lane] so
// that a lookup with a wave-uniform residue reads consecutive words (no bank conflicts) and
// one address per residue serves all three positions.  Rows reach a wave in groups of
// consecutive sequences, one coalesced load per group issued a group ahead.  Stores are
// 512-byte coalesced rows of sig.
#include <type_traits>

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

// Median of three unsigned words (one VALU instruction).
__device__ __forceinline__ uint32_t umed3(uint32_t a, uint32_t b, uint32_t c) {
    uint32_t r;
    asm("v_med3_u32 %0, %1, %2, %3" : "=v"(r) : "v"(a), "v"(b), "v"(c));
    return r;
}

// a ^ b ^ c as one VALU instruction (v_bitop3 with the three-way XOR truth table).
__device__ __forceinline__ uint32_t xor3(uint32_t a, uint32_t b, uint32_t c) {
    uint32_t r;
    asm("v_bitop3_b32 %0, %1, %2, %3 bitop3:0x96" : "=v"(r) : "v"(a), "v"(b), "v"(c));
    return r;
}
// A lane's JP consecutive table words in one LDS access (4 or 8 bytes).
template <int JP>
__device__ __forceinline__ void lds_words(const uint32_t *p, uint32_t (&v)[JP]) {
    if constexpr (JP == 1) {
        v[0] = p[0];
    } else {
        const uint2 t = *reinterpret_cast<const uint2 *>(p);
        v[0] = t.x;
        v[1] = t.y;
    }
}

// Lane l owns the 2 JP hash functions t = l + 64 q (q < 2 JP).  Three LDS tables, each
// laid out [residue][position][lane][...] so that one address per residue serves the three
// position tables (their offsets are immediates):
//   Q  [20][3][64][JP]   packed top halves: word jp holds the top 16 bits of the hi half of
//                        hash q = 2 jp (low 16 bits) and of hash q = 2 jp + 1 (high 16 bits);
//   Hh, Hl [20][3][2 JP][64]   the full hi and lo halves of every hash (a lane's words 4
//                        bytes apart, so that the winners' lookups are conflict-free).
// The streaming pass XORs three packed words per shingle (two hash functions at once) and
// keeps, per hash function, the smallest and second smallest of the keys
// (16 top bits << 16 | the shingle's 3-mer code a << 10 | b << 5 | c): m1 and m2 (v_med3
// of m1, m2 and the new key).  When m1 and m2 differ in their top 16 bits, m1's 3-mer has
// strictly the smallest hi half of all the sequence's 3-mers, hence the minimum hash, whose
// full 64 bits are read once from its code.  Otherwise (the same 3-mer twice, or two 3-mers
// whose hashes share those 16 bits) that lane redoes the sequence with full 64-bit words.
template <int JP>
__global__ __launch_bounds__(kMinhashBlock) void minhash3_kernel(
    const uint8_t *__restrict__ seqs, const int32_t *__restrict__ lens, int64_t n, int32_t stride,
    int32_t M, uint64_t seed, uint64_t *__restrict__ sig) {
    constexpr int J = 2 * JP;                     // hash functions per lane
    constexpr int kHWords = 20 * 3 * 64 * J;      // one full plane
    constexpr int kQWords = 20 * 3 * 64 * JP;
    constexpr int kResH = 3 * 64 * J, kPosH = 64 * J;    // strides (words) in Hh / Hl
    constexpr int kResQ = 3 * 64 * JP, kPosQ = 64 * JP;  // strides (words) in Q
    extern __shared__ uint32_t lds[];
    uint32_t *Hh = lds;
    uint32_t *Hl = lds + kHWords;
    uint32_t *Q = lds + 2 * kHWords;
    for (int e = threadIdx.x; e < kHWords; e += blockDim.x) {
        const int l = e % 64;
        const int q = (e / 64) % J;
        const int rp = e / (J * 64);  // residue * 3 + position
        const int t = l + 64 * q;
        uint64_t v = ~0ull;
        if (t < M) {
            const int res = rp / 3, pos = rp % 3;
            v = splitmix64_at(seed, ((uint64_t)t * 3 + pos) * 20 + res);
        }
        Hh[e] = (uint32_t)(v >> 32);
        Hl[e] = (uint32_t)v;
    }
    __syncthreads();
    for (int e = threadIdx.x; e < kQWords; e += blockDim.x) {
        const int jp = e % JP;
        const int l = (e / JP) % 64;
        const int base = (e / (JP * 64)) * (64 * J) + 2 * jp * 64 + l;  // hash q = 2 jp of that row in Hh
        Q[e] = (Hh[base] >> 16) | (Hh[base + 64] & 0xFFFF0000u);
    }
    __syncthreads();

    const int lane = threadIdx.x & 63;
    const int64_t wave = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6)) +
                         (int64_t)blockIdx.x * (blockDim.x >> 6);
    const int64_t nwaves = (int64_t)gridDim.x * (blockDim.x >> 6);
    const uint32_t *Ql = Q + lane * JP;
    const uint32_t *Hhl = Hh + lane;
    const uint32_t *Hll = Hl + lane;

    // Sequences go to waves in groups of G consecutive rows, G = 64 / D with D = stride / 4
    // words per row: one coalesced dword load per lane brings a whole group (lane k D + w holds
    // word w of row k), issued a group ahead.  Each lane then prepares, for the four residue
    // positions of its word, the LDS byte offsets of their table rows and the 3-mer codes of
    // the shingles starting there (two 16-bit values per word); the hashing loop broadcasts
    // them with readlane, so the per-shingle work is vector work with scalar operands.
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
    // key = (16 hash bits << 16) | 3-mer code, from a packed hash word h and a packed code
    // word s (v_perm byte selectors: bytes 4..7 are h's, 0..3 are s's)
    const uint32_t sel_lo_c0 = 0x05040100u, sel_lo_c1 = 0x05040302u;  // hash q = 2 jp
    const uint32_t sel_hi_c0 = 0x07060100u, sel_hi_c1 = 0x07060302u;  // hash q = 2 jp + 1
    const char *Qb = reinterpret_cast<const char *>(Ql);
    fetch(wave);
    for (int64_t g = wave; g < ngroups; g += nwaves) {
        const uint32_t rowv = nrow;
        const int lenv = nlen;
        fetch(g + nwaves);
        // this lane's residue positions 4w .. 4w + 5 (the next word from the next lane;
        // positions past a row only ever feed shingles past its length)
        const uint32_t nxt = (uint32_t)__shfl_down((int)rowv, 1, 64);
        uint32_t r[6];
#pragma unroll
        for (int e = 0; e < 6; ++e) r[e] = min(((e < 4 ? rowv >> (8 * e) : nxt >> (8 * (e - 4)))) & 0xFFu, 19u);
        constexpr uint32_t kRowBytes = 4u * kResQ;  // one residue's table rows
        const uint32_t off01 = r[0] * kRowBytes | (r[1] * kRowBytes) << 16;
        const uint32_t off23 = r[2] * kRowBytes | (r[3] * kRowBytes) << 16;
        uint32_t cd[4];
#pragma unroll
        for (int e = 0; e < 4; ++e) cd[e] = (r[e] << 10) | (r[e + 1] << 5) | r[e + 2];
        const uint32_t code01 = cd[0] | cd[1] << 16, code23 = cd[2] | cd[3] << 16;
        const int64_t base = g * G;
        const int gn = (int)min((int64_t)G, n - base);
        for (int k = 0; k < gn; ++k) {
            const int64_t i = base + k;
            const int L = min(max(__builtin_amdgcn_readlane(lenv, k), 0), stride);
            const int kD = k * D;
            const int nsh = L - 2;  // shingles
            uint64_t *out = sig + i * (int64_t)M;
            if (nsh <= 0) {  // no 3-mer (a length below 3 breaks the contract): the empty minimum
#pragma unroll
                for (int q = 0; q < J; ++q)
                    if (lane + 64 * q < M) out[lane + 64 * q] = ~0ull;
                continue;
            }
            uint32_t m1[J], m2[J];
#pragma unroll
            for (int q = 0; q < J; ++q) {
                m1[q] = ~0u;
                m2[q] = ~0u;
            }
            // Four shingles per iteration (positions q0 .. q0+5, from row words w and w + 1):
            // one LDS address per position serves its three position tables, and all twelve
            // lookups are issued before any is used.  `live` shingles of the four count.
            auto iter = [&](int q0, auto live) {
                const int w = q0 >> 2;
                const uint32_t so01 = __builtin_amdgcn_readlane(off01, kD + w);
                const uint32_t so23 = __builtin_amdgcn_readlane(off23, kD + w);
                const uint32_t so45 = w + 1 < D ? __builtin_amdgcn_readlane(off01, kD + w + 1) : 0u;
                const uint32_t sc01 = __builtin_amdgcn_readlane(code01, kD + w);
                const uint32_t sc23 = __builtin_amdgcn_readlane(code23, kD + w);
                const uint32_t so[6] = {so01 & 0xFFFFu, so01 >> 16, so23 & 0xFFFFu, so23 >> 16, so45 & 0xFFFFu,
                                        so45 >> 16};
                const uint32_t *A[6];
#pragma unroll
                for (int e = 0; e < 6; ++e) A[e] = reinterpret_cast<const uint32_t *>(Qb + so[e]);
                uint32_t h[4][JP];
#pragma unroll
                for (int sh = 0; sh < 4; ++sh) {
                    uint32_t t0[JP], t1[JP], t2[JP];
                    lds_words<JP>(A[sh], t0);
                    lds_words<JP>(A[sh + 1] + kPosQ, t1);
                    lds_words<JP>(A[sh + 2] + 2 * kPosQ, t2);
#pragma unroll
                    for (int jp = 0; jp < JP; ++jp) h[sh][jp] = xor3(t0[jp], t1[jp], t2[jp]);
                }
#pragma unroll
                for (int sh = 0; sh < 4; ++sh) {
                    if (sh < live) {
                        const uint32_t sc = sh < 2 ? sc01 : sc23;
                        const uint32_t sa = (sh & 1) ? sel_lo_c1 : sel_lo_c0, sb = (sh & 1) ? sel_hi_c1 : sel_hi_c0;
#pragma unroll
                        for (int jp = 0; jp < JP; ++jp) {
                            const uint32_t ka = __builtin_amdgcn_perm(h[sh][jp], sc, sa);  // hash q = 2 jp
                            const uint32_t kb = __builtin_amdgcn_perm(h[sh][jp], sc, sb);  // hash q = 2 jp + 1
                            m2[2 * jp] = umed3(m1[2 * jp], m2[2 * jp], ka);
                            m1[2 * jp] = min(m1[2 * jp], ka);
                            m2[2 * jp + 1] = umed3(m1[2 * jp + 1], m2[2 * jp + 1], kb);
                            m1[2 * jp + 1] = min(m1[2 * jp + 1], kb);
                        }
                    }
                }
            };
            int q0 = 0;
#pragma unroll 1
            for (; q0 + 4 <= nsh; q0 += 4) iter(q0, std::integral_constant<int, 4>{});
            if (q0 < nsh) iter(q0, nsh - q0);  // the last, partial, iteration
#pragma unroll
            for (int q = 0; q < J; ++q) {
                const int t = lane + 64 * q;
                // the winner's full 64 bits from its code (nsh >= 1, so m1 holds a real key
                // and every field is a residue code below 20)
                const uint32_t a0 = (m1[q] >> 10) & 31u, a1 = (m1[q] >> 5) & 31u, a2 = m1[q] & 31u;
                const char *hb = reinterpret_cast<const char *>(Hhl + 64 * q);
                const uint32_t *p0 = reinterpret_cast<const uint32_t *>(hb + a0 * (4 * kResH));
                const uint32_t *p1 = reinterpret_cast<const uint32_t *>(hb + a1 * (4 * kResH)) + kPosH;
                const uint32_t *p2 = reinterpret_cast<const uint32_t *>(hb + a2 * (4 * kResH)) + 2 * kPosH;
                uint64_t best = ((uint64_t)xor3(p0[0], p1[0], p2[0]) << 32) |
                                xor3(p0[kHWords], p1[kHWords], p2[kHWords]);  // hi, then the lo plane
                if ((m1[q] ^ m2[q]) < 0x10000u) {  // a tie in the top bits: exact 64-bit minimum
                    best = ~0ull;
                    for (int p = 0; p + 3 <= L; ++p) {  // residues from the row words (no memory access)
                        const int w = p >> 2;
                        const uint32_t wl = __builtin_amdgcn_readlane(rowv, kD + w);
                        const uint32_t wh = w + 1 < D ? __builtin_amdgcn_readlane(rowv, kD + w + 1) : 0u;
                        const uint32_t tq = (uint32_t)((((uint64_t)wh << 32) | wl) >> (8 * (p & 3)));
                        const uint32_t b0 = min(tq & 0xFFu, 19u);
                        const uint32_t b1 = min((tq >> 8) & 0xFFu, 19u);
                        const uint32_t b2 = min((tq >> 16) & 0xFFu, 19u);
                        const int e0 = b0 * kResH + 64 * q, e1 = b1 * kResH + kPosH + 64 * q,
                                  e2 = b2 * kResH + 2 * kPosH + 64 * q;
                        const uint64_t hh = ((uint64_t)(Hhl[e0] ^ Hhl[e1] ^ Hhl[e2]) << 32) | (Hll[e0] ^ Hll[e1] ^ Hll[e2]);
                        best = hh < best ? hh : best;
                    }
                }
                if (t < M) out[t] = best;
            }
        }
    }
}

template <int JP>
static int launch_minhash(const uint8_t *seqs, const int32_t *lens, int64_t n, int32_t stride, int32_t M,
                          uint64_t seed, uint64_t *sig, hipStream_t st) {
    const size_t lds = sizeof(uint32_t) * (2 * 20 * 3 * 64 * 2 * JP + 20 * 3 * 64 * JP);
    static bool attr_set = false;
    if (!attr_set) {
        SQ_HIP(hipFuncSetAttribute((const void *)minhash3_kernel<JP>,
                                   hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
        attr_set = true;
    }
    const int waves_per_block = kMinhashBlock / kWave;
    const int per_cu = JP == 1 ? std::min(knob(SUBQUAD_KNOB_MINHASH_BLOCKS_PER_CU), 2) : 1;  // LDS bound
    const int64_t groups = ceil_div(n, (int64_t)(64 / (stride / 4)));  // rows per wave group: 64 / (stride / 4)
    int64_t blocks = std::min<int64_t>(ceil_div(groups, waves_per_block), (int64_t)device_cus() * per_cu);
    ProfScope prof("minhash3_kernel", st);
    minhash3_kernel<JP><<<(unsigned)blocks, kMinhashBlock, lds, st>>>(seqs, lens, n, stride, M, seed, sig);
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
    if (M <= 128) return launch_minhash<1>(seqs, lens, n, stride, M, seed, sig, st);
    return launch_minhash<2>(seqs, lens, n, stride, M, seed, sig, st);
}
