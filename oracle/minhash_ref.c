/*
 * Oracle: MinHash signatures in plain C -- TEST INFRASTRUCTURE ONLY.
 * sig[i][t] = min over 3-mer positions p of T[t][0][a_p] ^ T[t][1][a_{p+1}] ^ T[t][2][a_{p+2}]
 * (the minimum over the shingle set; a repeated 3-mer repeats a value).  The tables T come
 * from the Python oracle (SplitMix64 outputs), laid out [M][3][20].
 */
#include <stdint.h>

void oracle_minhash3(const uint8_t *seqs, const int32_t *lens, int64_t n, int32_t stride,
                     const uint64_t *T, int32_t M, uint64_t *sig)
{
    for (int64_t i = 0; i < n; ++i) {
        const uint8_t *s = seqs + i * stride;
        for (int t = 0; t < M; ++t) {
            const uint64_t *Tt = T + (int64_t)t * 60;
            uint64_t best = UINT64_MAX;
            for (int p = 0; p + 3 <= lens[i]; ++p) {
                uint64_t h = Tt[s[p]] ^ Tt[20 + s[p + 1]] ^ Tt[40 + s[p + 2]];
                if (h < best) best = h;
            }
            sig[i * M + t] = best;
        }
    }
}
