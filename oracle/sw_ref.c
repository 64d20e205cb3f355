/*
 * Oracle: Smith-Waterman local alignment score with affine gaps (Gotoh's recurrence),
 * plain textbook C over the full dynamic-programming matrices.  TEST INFRASTRUCTURE ONLY.
 *
 * The paper's affinity kernel is a global edit distance (Appendix F.3); the alignment
 * channel computed here is a local alignment with a substitution matrix and affine gaps.
 * Reading of the gap convention: a gap of length k costs gap_open + (k - 1) * gap_extend,
 * i.e. its first residue costs gap_open and every further residue gap_extend.
 *
 *   H[x][y] = max(0, H[x-1][y-1] + S(a_x, b_y), E[x][y], F[x][y])
 *   E[x][y] = max(E[x][y-1] - gap_extend, H[x][y-1] - gap_open)   (gap in a)
 *   F[x][y] = max(F[x-1][y] - gap_extend, H[x-1][y] - gap_open)   (gap in b)
 *   H[0][.] = H[.][0] = 0, E and F start at minus infinity; score = max over all H.
 *
 * Residue codes are 0..19; subst is int8[20][20] in the same order.
 */
#include <stdint.h>
#include <stdlib.h>

#define NEG_INF (-1000000000)

static int imax(int a, int b) { return a > b ? a : b; }

int oracle_sw_score(const uint8_t *a, int la, const uint8_t *b, int lb,
                    const int8_t *subst, int gap_open, int gap_extend)
{
    int rows = la + 1, cols = lb + 1;
    int *H = (int *)malloc(sizeof(int) * rows * cols);
    int *E = (int *)malloc(sizeof(int) * rows * cols);
    int *F = (int *)malloc(sizeof(int) * rows * cols);
    int best = 0;
    for (int x = 0; x < rows; ++x) {
        for (int y = 0; y < cols; ++y) {
            int idx = x * cols + y;
            if (x == 0 || y == 0) {
                H[idx] = 0;
                E[idx] = NEG_INF;
                F[idx] = NEG_INF;
                continue;
            }
            int e = imax(E[idx - 1] - gap_extend, H[idx - 1] - gap_open);
            int f = imax(F[idx - cols] - gap_extend, H[idx - cols] - gap_open);
            int d = H[idx - cols - 1] + subst[a[x - 1] * 20 + b[y - 1]];
            int h = imax(imax(0, d), imax(e, f));
            E[idx] = e;
            F[idx] = f;
            H[idx] = h;
            if (h > best) best = h;
        }
    }
    free(H);
    free(E);
    free(F);
    return best;
}

/* Scores for a list of pairs (i, j) of rows of a padded batch seqs[n][stride]. */
void oracle_sw_pairs(const uint8_t *seqs, const int32_t *lens, int32_t stride,
                     const int32_t *pairs, int64_t P, const int8_t *subst,
                     int gap_open, int gap_extend, int32_t *out)
{
    for (int64_t p = 0; p < P; ++p) {
        int i = pairs[2 * p], j = pairs[2 * p + 1];
        out[p] = oracle_sw_score(seqs + (int64_t)i * stride, lens[i],
                                 seqs + (int64_t)j * stride, lens[j],
                                 subst, gap_open, gap_extend);
    }
}

/*
 * Weighted global edit distance (the paper's Appendix F.3 recurrence):
 *   d[x][y] = min(d[x-1][y] + indel, d[x][y-1] + indel, d[x-1][y-1] + cost[a_x][b_y]),
 *   d[x][0] = x * indel, d[0][y] = y * indel; result d[la][lb].
 */
int oracle_edit_distance(const uint8_t *a, int la, const uint8_t *b, int lb, const int8_t *cost, int indel)
{
    int cols = lb + 1;
    int *d = (int *)malloc(sizeof(int) * (la + 1) * cols);
    for (int x = 0; x <= la; ++x) {
        for (int y = 0; y <= lb; ++y) {
            int idx = x * cols + y;
            if (x == 0) { d[idx] = y * indel; continue; }
            if (y == 0) { d[idx] = x * indel; continue; }
            int best = d[idx - cols] + indel;
            int v = d[idx - 1] + indel;
            if (v < best) best = v;
            v = d[idx - cols - 1] + cost[a[x - 1] * 20 + b[y - 1]];
            if (v < best) best = v;
            d[idx] = best;
        }
    }
    int out = d[la * cols + lb];
    free(d);
    return out;
}

void oracle_edit_pairs(const uint8_t *seqs, const int32_t *lens, int32_t stride, const int32_t *pairs, int64_t P,
                       const int8_t *cost, int indel, int32_t *out)
{
    for (int64_t p = 0; p < P; ++p) {
        int i = pairs[2 * p], j = pairs[2 * p + 1];
        out[p] = oracle_edit_distance(seqs + (int64_t)i * stride, lens[i], seqs + (int64_t)j * stride, lens[j],
                                      cost, indel);
    }
}
