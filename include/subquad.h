/*
 * subquad.h -- C ABI of the SubQuad hot path on AMD Instinct MI355X (gfx950).
 *
 * The library computes, for a batch of immune-receptor sequences, the candidate-pair
 * affinity stage of SubQuad (arXiv 2602.17330): MinHash sketches, an LSH index that
 * yields the candidate list, a local-alignment channel on every candidate pair and the
 * per-pair gated fusion of that channel with an embedding-cosine channel, forward and
 * backward.  The paper's problem statement (Sec. 3.1) maps sequences to a sparse weighted
 * graph; this library stops at the sparse list of fused pair affinities that populates it
 * (Algorithm 1, preprocessing and affinity computation).
 *
 * Conventions shared by every entry point
 *   - Every array argument is DEVICE memory on the current HIP device unless it is marked
 *     "host".  The caller owns all memory and the library keeps no data between calls
 *     (it keeps a second stream per device and host thread, see below, and the static
 *     array of the allocation-free alignment entry point).
 *     Entry points that take a workspace allocate nothing; subquad_check_seqs and
 *     subquad_align_batch (the variant without a workspace) take a small stream-ordered
 *     allocation (hipMallocAsync) and release it before returning.
 *   - `stream` is a hipStream_t (NULL = the default stream).  Work is enqueued on it and the
 *     call returns without waiting, except where a host output is documented.  The gate
 *     backward and training calls run one independent part (the pairs' order by j) on a
 *     second stream the library creates once per device and host thread (non-blocking,
 *     default priority): forked from `stream` by an event and joined back to it before the
 *     call returns, so all of a call's work stays ordered on `stream`, and a graph captured
 *     from `stream` holds it as a parallel branch.  The first such call on a device and host
 *     thread creates that stream and its events: make it outside a graph capture.
 *   - Sequences are rows of `stride` bytes: residue codes 0..19 in the order
 *     ACDEFGHIKLMNPQRSTVWY, any value past the row's length (pad 0xFF by convention).
 *     `lens[i]` is the length of row i.
 *   - Return value: SUBQUAD_OK or one of the error codes below.  Arguments are validated on
 *     the host before anything is enqueued; on an error nothing is enqueued and
 *     subquad_last_error() describes it (thread-local, valid until the next call on the
 *     same thread).  Device contents (residue codes, lengths) are validated only by
 *     subquad_check_seqs; other kernels clamp out-of-range codes so that bad data can give
 *     wrong results but never an out-of-bounds access.
 */
#ifndef SUBQUAD_H
#define SUBQUAD_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum subquad_status {
    SUBQUAD_OK = 0,
    SUBQUAD_ERR_ARG = 1,        /* null pointer, negative or out-of-range size or parameter  */
    SUBQUAD_ERR_RESIDUE = 2,    /* a residue code >= 20 within a sequence's length           */
    SUBQUAD_ERR_LENGTH = 3,     /* a length below k or above stride                          */
    SUBQUAD_ERR_CAPACITY = 4,   /* more candidate pairs than the output capacity             */
    SUBQUAD_ERR_WORKSPACE = 5,  /* workspace smaller than the size function returns          */
    SUBQUAD_ERR_HIP = 6         /* the HIP runtime reported an error                         */
};

/* Message for the last non-OK status returned on this thread ("" if none). */
const char *subquad_last_error(void);

/* Library version string. */
const char *subquad_version(void);

/*
 * Launch-shape knobs (process-wide, every GPU).  They choose grid and block shapes only and
 * never change any result; an autotuner may set them.  Values <= 0 restore the default.
 */
enum subquad_knob {
    SUBQUAD_KNOB_MINHASH_BLOCKS_PER_CU = 0,  /* persistent MinHash blocks per CU (default 2) */
    SUBQUAD_KNOB_ALIGN_BLOCKS_PER_CU = 1,    /* alignment blocks per CU, at most the resident ones (16) */
    SUBQUAD_KNOB_GATE_GROUPS_PER_CU = 2,     /* 16-lane pair groups per CU (default 64)       */
    SUBQUAD_KNOB_EMIT_THREADS = 3,           /* LSH long-run emission block size (512)         */
    SUBQUAD_KNOB_COUNT = 4
};
int subquad_set_knob(int32_t knob, int32_t value);  /* SUBQUAD_ERR_ARG for an unknown knob */
int32_t subquad_get_knob(int32_t knob);             /* current value, -1 if unknown        */

/*
 * Per-kernel timing (tracing).  While enabled, every main kernel launch is bracketed by two
 * HIP events recorded on its own stream.  subquad_profile_report synchronises those events
 * and writes one line per kernel name, "name launches total_ms\n", into buf (host, len
 * bytes, always NUL-terminated); it returns the bytes needed (excluding the NUL).
 * Enabling (on != 0) or disabling clears the records.  Not for use under graph capture.
 * subquad_profile_only limits the timing to the launches of the kernel named `name` (host
 * string, copied), so that the rest of the work runs with no events between its launches;
 * null or "" times every kernel again.  It clears the records too.
 */
int subquad_profile_enable(int32_t on);
int subquad_profile_only(const char *name);
int64_t subquad_profile_report(char *buf, size_t len);

/*
 * subquad_check_seqs -- validate a sequence batch (Algorithm 1, preprocessing: the padded
 * sequence rows every later stage reads).
 *   seqs [n][stride] u8, lens [n] i32: the batch.  k: shingle length (1..5).
 *   n_bad (host, may be NULL): receives the number of rows that fail.
 * Synchronises `stream`.  Returns SUBQUAD_ERR_LENGTH if some k <= lens[i] <= stride fails,
 * else SUBQUAD_ERR_RESIDUE if some code within a length is >= 20, else SUBQUAD_OK.
 */
int subquad_check_seqs(const uint8_t *seqs, const int32_t *lens, int64_t n, int32_t stride,
                       int32_t k, int64_t *n_bad, void *stream);

/*
 * subquad_minhash -- MinHash sketch of every sequence (Algorithm 1, preprocessing; sketch
 * size M as in Sec. 4.1 and the sampling-error bound of Appendix B).
 *   sig [n][M] u64, row-major (out): sig[i][t] = min over the set of distinct k-mers x of
 *   row i of h_t(x), with simple tabulation h_t(x) = XOR_p T[t][p][x_p] and the 20*k*M table
 *   words T taken, in the order t, p, residue, from the SplitMix64 sequence started at
 *   `seed`.  Requires k == 3 (the hot path's shingle length), 1 <= M <= 256, 3 <= stride
 *   <= 64, stride % 4 == 0, seqs 4-byte aligned.  Row lengths must lie in [k, stride]
 *   (subquad_check_seqs).
 */
int subquad_minhash(const uint8_t *seqs, const int32_t *lens, int64_t n, int32_t stride,
                    int32_t k, int32_t M, uint64_t seed, uint64_t *sig, void *stream);

/*
 * subquad_lsh_workspace_bytes -- bytes of device workspace subquad_lsh_candidates needs
 * for n sequences, b bands and an output capacity of `cap` pairs.  Returns 0 if the sizes
 * are out of range (n * b >= 2^32, cap < 0).
 */
size_t subquad_lsh_workspace_bytes(int64_t n, int32_t b, int64_t cap);

/*
 * subquad_lsh_candidates -- candidate list CAND of the MinHash LSH index (Algorithm 1,
 * preprocessing; index of Sec. 4.2; cost O(|C|) + O(n log n), Appendix B).
 *   sig [n][M] u64: signatures from subquad_minhash.  b bands of r rows, 1 <= b <= 256,
 *   b * r <= M; band beta covers signature rows beta*r .. beta*r + r - 1.
 *   rep_offsets [R+1] i64 (may be NULL, then R must be 1): repertoire r is rows
 *   rep_offsets[r] .. rep_offsets[r+1]-1; rep_offsets[0] = 0, rep_offsets[R] = n, ascending.
 *   ws / ws_bytes: workspace of at least subquad_lsh_workspace_bytes(n, b, cap) bytes,
 *   256-byte aligned.
 *   pairs [cap][2] i32 (out): the pairs (i, j), i < j, of rows of one repertoire whose
 *   r-tuples are exactly equal in at least one band; each pair once, sorted by (i, j).
 *   row_offsets [n+1] i64 (out, may be NULL): CSR offsets into `pairs` by first index.
 *   n_pairs (host out): the number of candidate pairs P.
 * Synchronises `stream` once (to read P).  If P > cap, returns SUBQUAD_ERR_CAPACITY with
 * *n_pairs = P; then `pairs` and `row_offsets` are unspecified and the call can be repeated
 * with a larger capacity.
 */
int subquad_lsh_candidates(const uint64_t *sig, int64_t n, int32_t M, int32_t b, int32_t r,
                           const int64_t *rep_offsets, int64_t R, void *ws, size_t ws_bytes,
                           int32_t *pairs, int64_t *row_offsets, int64_t cap,
                           int64_t *n_pairs, void *stream);

/*
 * subquad_lsh_candidates_async -- as subquad_lsh_candidates, but never synchronises, so it
 * can be captured in a HIP graph.  n_pairs_dev (device out, i64): P.  status_dev (device
 * out, i32): 0, or SUBQUAD_ERR_CAPACITY when P > cap (then pairs and row_offsets are
 * unspecified).  The sort is sized for `cap` pairs, so cap should be a tight bound.
 */
int subquad_lsh_candidates_async(const uint64_t *sig, int64_t n, int32_t M, int32_t b,
                                 int32_t r, const int64_t *rep_offsets, int64_t R, void *ws,
                                 size_t ws_bytes, int32_t *pairs, int64_t *row_offsets,
                                 int64_t cap, int64_t *n_pairs_dev, int32_t *status_dev,
                                 void *stream);

/*
 * subquad_self_scores -- self[i] = sum over x < lens[i] of subst[a_x][a_x], the local
 * alignment score of a sequence with itself whenever every off-diagonal entry of subst is
 * below every diagonal entry (as for BLOSUM62).  Used to normalise the alignment channel.
 *   subst [20][20] i8, rows and columns in residue-code order.
 */
int subquad_self_scores(const uint8_t *seqs, const int32_t *lens, int64_t n, int32_t stride,
                        const int8_t *subst, int32_t *self, void *stream);

/*
 * subquad_align_batch -- local alignment channel on every candidate pair (Algorithm 1,
 * affinity computation: the alignment affinity a^(1) of Eq. (afused)).  The paper's own
 * kernel is a global edit distance (Appendix F.3); this channel is the Smith-Waterman local
 * alignment score with Gotoh's affine gaps:
 *   H = max(0, H_diag + subst[a_x][b_y], E, F), E = max(E_left - gap_extend,
 *   H_left - gap_open), F = max(F_up - gap_extend, H_up - gap_open); score = max H,
 * so a gap of length k costs gap_open + (k - 1) * gap_extend.
 *   pairs [P][2] i32 (rows of seqs, any order, i == j allowed), scores [P] i32 (out).
 *   gap_open, gap_extend: positive costs, 0 <= gap_extend <= gap_open <= 1000.
 *   subst [20][20] i8: subst[a][b] scores residue a of sequence i against residue b of
 *   sequence j (a = pairs[p][0]'s residue); it need not be symmetric.  Each pair is aligned
 *   with its shorter sequence down the register-resident rows; when that is sequence j the
 *   transposed matrix is used (an asymmetric matrix costs a second pass over the pairs).
 *   Requires stride % 4 == 0, 4 <= stride <= 64.
 */
int subquad_align_batch(const uint8_t *seqs, const int32_t *lens, int64_t n, int32_t stride,
                        const int32_t *pairs, int64_t P, const int8_t *subst,
                        int32_t gap_open, int32_t gap_extend, int32_t *scores, void *stream);

/*
 * subquad_align_batch_ws -- as subquad_align_batch, with caller-provided scratch for the
 * length sort that groups pairs of similar lengths into the same wavefront.
 *   ws / ws_bytes: at least subquad_align_workspace_bytes(P) bytes, 4-byte aligned.
 */
size_t subquad_align_workspace_bytes(int64_t P);
int subquad_align_batch_ws(const uint8_t *seqs, const int32_t *lens, int64_t n, int32_t stride,
                           const int32_t *pairs, int64_t P, const int8_t *subst,
                           int32_t gap_open, int32_t gap_extend, int32_t *scores, void *ws,
                           size_t ws_bytes, void *stream);

/*
 * subquad_align_batch_dev -- subquad_align_batch_ws on a pair count that a producer left in
 * device memory (the candidate count of subquad_lsh_candidates_async): no host
 * synchronisation, so the call can be captured in a HIP graph and replayed on new inputs.
 *   pairs [cap][2] i32; n_pairs_dev [1] i64 (device): the number of pairs P, read on the
 *   device and clamped to [0, cap]; scores [cap] i32 (out; entries p >= P are not written).
 *   ws / ws_bytes: at least subquad_align_workspace_bytes(cap) bytes.
 */
int subquad_align_batch_dev(const uint8_t *seqs, const int32_t *lens, int64_t n, int32_t stride,
                            const int32_t *pairs, int64_t cap, const int64_t *n_pairs_dev,
                            const int8_t *subst, int32_t gap_open, int32_t gap_extend,
                            int32_t *scores, void *ws, size_t ws_bytes, void *stream);

/*
 * subquad_align_batch_noalloc -- for callers that cannot allocate device memory (code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * scores as subquad_align_batch, with the length sort's scratch taken from a fixed device
 * array inside the library instead of an allocation.  No hipMalloc, hipFree or allocating
 * call is made.
 *   Arguments and results as subquad_align_batch.  P must be at most
 *   SUBQUAD_ALIGN_NOALLOC_MAX_PAIRS, else SUBQUAD_ERR_ARG and nothing is enqueued.
 *   The array (33 MiB) is held by every GPU the library runs on until the process ends.
 *   All calls on one GPU share it: calls that overlap in time on one GPU (other streams,
 *   other threads) race and give wrong scores; calls ordered on one stream are safe.
 *   Nothing in the array needs to start at zero, so a call never reads what an earlier
 *   call left there.
 */
#define SUBQUAD_ALIGN_NOALLOC_MAX_PAIRS (1 << 20)
int subquad_align_batch_noalloc(const uint8_t *seqs, const int32_t *lens, int64_t n,
                                int32_t stride, const int32_t *pairs, int64_t P,
                                const int8_t *subst, int32_t gap_open, int32_t gap_extend,
                                int32_t *scores, void *stream);

/*
 * subquad_gate_fwd -- per-pair dynamic affinity fusion, Sec. 3.6, Eq. (wm) and (afused),
 * with the sigmoid channel weight of Eq. (alpha).  For pair p = (i, j):
 *   s = align[p] / sqrt(self[i] * self[j])      (alignment channel)
 *   c = <e_i, e_j> / (|e_i| |e_j|)               (embedding channel; 0 if a norm is 0)
 *   x = (s, c, |lens[i] - lens[j]|, [vgene[i] == vgene[j]])
 *   g = sigmoid(w2 . relu(W1 x + b1) + b2)       (= softmax weight of channel 1 over the
 *                                                  channel logits (u, 0))
 *   fused[p] = g * s + (1 - g) * c
 *   emb [n][d] f32 row-major, d % 4 == 0, 4 <= d <= 1024.  self [n] i32 (> 0).
 *   W1 [H][4], b1 [H], w2 [H], b2 [1] f32; H % 16 == 0, 16 <= H <= 256.
 *   fused [P] f32 (out); gate [P] f32 (out, may be NULL): g.
 */
int subquad_gate_fwd(const float *emb, int64_t n, int32_t d, const int32_t *lens,
                     const int32_t *vgene, const int32_t *self, const int32_t *pairs,
                     const int32_t *align, int64_t P, const float *W1, const float *b1,
                     const float *w2, const float *b2, int32_t H, float *fused, float *gate,
                     void *stream);

/* Bytes of device workspace subquad_gate_bwd and subquad_gate_train need for H hidden units,
 * P pairs and n nodes (0 when H <= 0, P < 0, n < 0 or P >= 2^32). */
size_t subquad_gate_bwd_workspace_bytes(int32_t H, int64_t P, int64_t n);

/*
 * subquad_gate_bwd -- gradient of L = sum_p grad_fused[p] * fused[p] (the backward of
 * subquad_gate_fwd, same arguments), recomputing every per-pair intermediate instead of
 * storing it.  Gradients ACCUMULATE into the outputs (zero them first for a plain
 * gradient): dW1 [H][4], db1 [H], dw2 [H], db2 [1], demb [n][d] (may be NULL: then the
 * embedding gradient is skipped).  The alignment, length and V-gene inputs get no gradient.
 * Weight gradients are summed in float32 over each run of 16 consecutive pairs, then in
 * float64 per block and over blocks in a fixed order (reproducible bit for bit).  The embedding gradient is gathered in two
 * passes over the pairs, stably sorted by i and then by j: a row whose pairs all fall in one
 * worker's chunk is updated with a plain read-modify-write, a row split between chunks with
 * float32 atomics (summation order, and last bits, may then vary between runs).  demb must
 * be 16-byte aligned.
 *   ws / ws_bytes: at least subquad_gate_bwd_workspace_bytes(H, P, n) bytes, 256-byte aligned.
 */
int subquad_gate_bwd(const float *emb, int64_t n, int32_t d, const int32_t *lens,
                     const int32_t *vgene, const int32_t *self, const int32_t *pairs,
                     const int32_t *align, int64_t P, const float *W1, const float *b1,
                     const float *w2, const float *b2, int32_t H, const float *grad_fused,
                     float *dW1, float *db1, float *dw2, float *db2, float *demb, void *ws,
                     size_t ws_bytes, void *stream);

/*
 * subquad_gate_train -- one training pass of the gate: the forward of subquad_gate_fwd, the
 * loss of subquad_contrastive_grad on label[] (margin contrastive, averaged over P) and the
 * backward of subquad_gate_bwd with that loss's gradient, in one pass over the pairs (each
 * pair's fused value, loss term and gradient are formed where the backward recomputes the
 * forward, so the forward is evaluated once).  Arguments as subquad_gate_bwd, plus
 * label [n] i32 (device) and margin; fused [P] f32 (out, may be NULL) receives the forward;
 * loss [1] f64 (device out) the mean loss, summed in a fixed order of blocks.  Gradients
 * ACCUMULATE as in subquad_gate_bwd.  ws: subquad_gate_bwd_workspace_bytes(H, P, n) bytes.
 */
int subquad_gate_train(const float *emb, int64_t n, int32_t d, const int32_t *lens,
                       const int32_t *vgene, const int32_t *self, const int32_t *pairs,
                       const int32_t *align, int64_t P, const float *W1, const float *b1,
                       const float *w2, const float *b2, int32_t H, const int32_t *label,
                       float margin, float *fused, double *loss, float *dW1, float *db1,
                       float *dw2, float *db2, float *demb, void *ws, size_t ws_bytes, void *stream);

/*
 * subquad_gate_train_set -- subquad_gate_train with the embedding gradient WRITTEN rather
 * than accumulated: on return demb [n][d] holds d loss / d emb (rows of nodes in no pair
 * are zero), so a training step needs no zero fill of demb first, and the first pass reads
 * no old gradient rows.  demb's prior contents (NaN included) are never read.  The weight
 * gradients, the loss and fused are as in subquad_gate_train (weight gradients ACCUMULATE).
 * Same arguments, workspace and error codes.
 */
int subquad_gate_train_set(const float *emb, int64_t n, int32_t d, const int32_t *lens,
                           const int32_t *vgene, const int32_t *self, const int32_t *pairs,
                           const int32_t *align, int64_t P, const float *W1, const float *b1,
                           const float *w2, const float *b2, int32_t H, const int32_t *label,
                           float margin, float *fused, double *loss, float *dW1, float *db1,
                           float *dw2, float *db2, float *demb, void *ws, size_t ws_bytes,
                           void *stream);

/*
 * subquad_gate_train_set_dev -- subquad_gate_train_set on a pair count that a producer
 * left in device memory (the candidate count of subquad_lsh_candidates_async), so that the
 * candidate, alignment and gate stages run with no host synchronisation and can be
 * captured once in a HIP graph and replayed on new inputs (Eq. (batch): a batch sized
 * against device memory, processed with launches sized for its capacity).
 *   cap: the capacity the launches and the workspace are sized for (pairs has cap rows);
 *   n_pairs_dev [1] i64 (device): the number of pairs P, read on the device and clamped to
 *   [0, cap].  Entries p >= P of fused are not written.  Otherwise as
 *   subquad_gate_train_set, with ws of subquad_gate_bwd_workspace_bytes(H, cap, n) bytes.
 */
int subquad_gate_train_set_dev(const float *emb, int64_t n, int32_t d, const int32_t *lens,
                               const int32_t *vgene, const int32_t *self, const int32_t *pairs,
                               const int32_t *align, int64_t cap, const int64_t *n_pairs_dev,
                               const float *W1, const float *b1, const float *w2, const float *b2,
                               int32_t H, const int32_t *label, float margin, float *fused,
                               double *loss, float *dW1, float *db1, float *dw2, float *db2,
                               float *demb, void *ws, size_t ws_bytes, void *stream);

/*
 * subquad_edit_cost_matrix -- the substitution costs of the edit-distance channel (Appendix
 * F.3 asks for costs "based on biochemical similarity" and gives no table), doubled so
 * that the dynamic program runs in integers: cost[a][b] = 0 for a == b, 1 for a
 * conservative substitution (subst[a][b] > 0), 2 for any other; the matching indel cost is
 * 2.  subst [20][20] i8 and cost [20][20] i8 are HOST pointers, row-major in residue-code
 * order; no HIP call is made.  Returns SUBQUAD_ERR_ARG for a null pointer.
 */
int subquad_edit_cost_matrix(const int8_t *subst, int8_t *cost);

/*
 * subquad_edit_batch_ws -- the paper's own affinity recurrence (Appendix F.3), a weighted
 * global edit distance, on every pair:
 *   D[x][y] = min(D[x-1][y] + indel, D[x][y-1] + indel, D[x-1][y-1] + cost[a_x][b_y]),
 *   D[x][0] = x * indel, D[0][y] = y * indel; dist[p] = D[L_i][L_j] (i32).
 *   cost [20][20] i8 (device), >= 0, cost[a][b] for residue a of sequence i against b of
 *   sequence j (need not be symmetric); 0 <= indel <= 1000.  The workspace is the
 *   alignment one (subquad_align_workspace_bytes(P)).  Requires stride % 4 == 0, <= 64.
 */
int subquad_edit_batch_ws(const uint8_t *seqs, const int32_t *lens, int64_t n, int32_t stride,
                          const int32_t *pairs, int64_t P, const int8_t *cost, int32_t indel,
                          int32_t *dist, void *ws, size_t ws_bytes, void *stream);

/*
 * subquad_gate3_fwd / subquad_gate3_bwd -- per-pair fusion over three channels, Sec. 3.6
 * Eq. (wm) and (afused) with a softmax over M = 3 channel logits:
 *   a = (s, c, e): s and c as in subquad_gate_fwd, e = 1 - dist[p] / (2 max(L_i, L_j))
 *   (dist from subquad_edit_batch_ws with doubled costs);
 *   x = (s, c, e, |L_i - L_j|, [V_i == V_j]); z = W1 x + b1; g = W2 relu(z) + b2;
 *   w = softmax(g); fused[p] = sum_m w_m a_m; weights [P][3] (out, may be NULL): w.
 *   W1 [H][5], b1 [H], W2 [3][H], b2 [3] f32; H in {16, 32, 64}; d % 4 == 0, d <= 512.
 * The backward accumulates dW1, db1, dW2, db2 (float64 per block, added into the workspace
 * with atomics, so the last bits may vary between runs) and, if non-NULL, demb (float32
 * atomics per pair), with the semantics of subquad_gate_bwd otherwise;
 * ws: subquad_gate3_bwd_workspace_bytes(H) bytes, 256-byte aligned.
 */
int subquad_gate3_fwd(const float *emb, int64_t n, int32_t d, const int32_t *lens,
                      const int32_t *vgene, const int32_t *self, const int32_t *pairs,
                      const int32_t *align, const int32_t *dist, int64_t P, const float *W1,
                      const float *b1, const float *W2, const float *b2, int32_t H, float *fused,
                      float *weights, void *stream);
size_t subquad_gate3_bwd_workspace_bytes(int32_t H);
int subquad_gate3_bwd(const float *emb, int64_t n, int32_t d, const int32_t *lens,
                      const int32_t *vgene, const int32_t *self, const int32_t *pairs,
                      const int32_t *align, const int32_t *dist, int64_t P, const float *W1,
                      const float *b1, const float *W2, const float *b2, int32_t H,
                      const float *grad_fused, float *dW1, float *db1, float *dW2, float *db2,
                      float *demb, void *ws, size_t ws_bytes, void *stream);

/*
 * subquad_graph_topk -- sparse similarity graph from the fused affinities (Algorithm 1,
 * graph construction; Sec. 3.7; the evaluation links receptors whose fused similarity
 * exceeds tau = 0.7, Appendix B sensitivity study).  Every pair (i, j) of `pairs` with
 * w[p] >= tau gives the directed edges i -> j and j -> i of weight w[p]; each node's edges
 * are ordered by weight descending, then neighbour id ascending, and the first k are kept
 * (k = 0: all).  NaN weights never pass.
 *   pairs [P][2] i32, w [P] f32 (e.g. the output of subquad_gate_fwd), n nodes.
 *   ws / ws_bytes: at least subquad_graph_workspace_bytes(n, P) bytes, 256-byte aligned.
 *   row_offsets [n+1] i64, cols [cap] i32, vals [cap] f32 (out): the CSR graph.
 *   nnz (host out): number of entries.  cap >= 2 * P always suffices.
 * Synchronises `stream` once.  SUBQUAD_ERR_CAPACITY (with *nnz set) if nnz > cap.
 */
size_t subquad_graph_workspace_bytes(int64_t n, int64_t P);
int subquad_graph_topk(const int32_t *pairs, const float *w, int64_t P, int64_t n, float tau,
                       int32_t k, void *ws, size_t ws_bytes, int64_t *row_offsets, int32_t *cols,
                       float *vals, int64_t cap, int64_t *nnz, void *stream);

/*
 * subquad_contrastive_grad -- the training signal of the gate: margin contrastive loss in
 * similarity form (Hadsell, Chopra and LeCun, 2006) on pair labels y_p = [label[i] = label[j]]:
 *   loss = (1/P) sum_p  y_p (1 - f_p)^2 + (1 - y_p) max(0, f_p - margin)^2,
 *   grad[p] = d loss / d f_p.
 * (The paper trains with a prototype-level loss, Eq. (proto); this per-pair form gives the
 * gate backward an upstream gradient.)  fused [P] f32, pairs [P][2] i32, label [n] i32
 * (device); grad [P] f32 (out); loss [1] f64 (device out, may be NULL), summed in a fixed
 * order.  Pairs with an index outside [0, n) get grad 0 and add 0.
 *   ws / ws_bytes: subquad_contrastive_workspace_bytes() bytes, 8-byte aligned.
 */
size_t subquad_contrastive_workspace_bytes(void);
int subquad_contrastive_grad(const float *fused, const int32_t *pairs, int64_t P, const int32_t *label,
                             int64_t n, float margin, float *grad, double *loss, void *ws,
                             size_t ws_bytes, void *stream);

/*
 * Prototype-contrastive loss (Sec. 3, prototype-contrastive consolidation; Eq. (pc), (proto)):
 *   p_c = mean of the rows of emb with label c (S_c);
 *   loss = sum over x in the batch of  log sum_{c : S_c non-empty} exp(<e_x, p_c> / tau)
 *                                    - <e_x, p_{y(x)}> / tau.
 * The denominator runs over every non-empty class, the positive one included.
 *   emb [n][d] f32 (16-byte aligned), d in {32, 64, 128}; labels [n] i32, classes 0..C-1
 *   (a row with a label outside that range belongs to no class); batch [B] i32 row indices
 *   (repeats allowed; an index outside [0, n) or of an unlabelled row contributes nothing);
 *   tau > 0.  Logits are float32 matrix-core products; per-row log-sum-exp in float32; the
 *   sum over the batch in float64 in a fixed order.
 * subquad_proto_fwd: loss [1] f64 (device, out); row_loss [B] f32 (device, out, may be NULL);
 *   protos [C][d] f32 (device, out, may be NULL): the prototypes.  It leaves the prototypes,
 *   class sizes and per-row log-sum-exp in ws.
 * subquad_proto_bwd: ACCUMULATES grad_loss * d loss / d emb into demb [n][d] (16-byte
 *   aligned); grad_loss is a device f32 scalar (NULL: 1).  It reads what subquad_proto_fwd
 *   left in ws: call it with the same inputs and the same, unmodified ws.  With
 *   through_prototypes != 0 the gradient also flows through Eq. (pc) into every labelled row;
 *   with 0 the prototypes are held constant.  Batch-row gradients are added with float32
 *   atomics (summation order, and last bits, may vary between runs).
 *   ws / ws_bytes: at least subquad_proto_workspace_bytes(n, d, C, B) bytes, 256-byte aligned.
 */
size_t subquad_proto_workspace_bytes(int64_t n, int32_t d, int64_t C, int64_t B);
int subquad_proto_fwd(const float *emb, int64_t n, int32_t d, const int32_t *labels, int64_t C,
                      const int32_t *batch, int64_t B, float tau, double *loss, float *row_loss,
                      float *protos, void *ws, size_t ws_bytes, void *stream);
int subquad_proto_bwd(const float *emb, int64_t n, int32_t d, const int32_t *labels, int64_t C,
                      const int32_t *batch, int64_t B, float tau, const float *grad_loss,
                      int32_t through_prototypes, float *demb, void *ws, size_t ws_bytes,
                      void *stream);

/*
 * RMT edge threshold of the similarity graph (Sec. 3.7; Algorithm 1: the eigenvalue spectrum
 * of the fused-affinity matrix gives a bulk cutoff; edges below the threshold it implies are
 * dropped).  Input: the symmetric CSR graph of subquad_graph_topk built with tau = 0, k = 0
 * (every positive affinity, both directions): row_offsets [n+1] i64, cols [nnz] i32,
 * vals [nnz] f32 (device).  Readings (the paper names no estimator):
 *   lambda_plus = 2 sqrt(sum of vals^2 / n), the Wigner semicircle edge at A's mean squared
 *   row norm; tau* = the largest tau whose lighter edges (0 < a < tau) keep the largest
 *   eigenvalue inside the bulk (<= lambda_plus), by `iters` bisection steps on [0, max a]
 *   with float64 midpoints; tau* = max a + 1 (no edge kept) when lambda_max(A) <= lambda_plus.
 * Each largest eigenvalue comes from `steps` Lanczos steps (float32 vectors, float64 dots,
 * full reorthogonalisation) from a start vector drawn from SplitMix64 with `seed`.
 * Outputs are host doubles; the call synchronises `stream` once per Lanczos run.  Keep the
 * edges with a >= tau* (subquad_graph_topk with tau = tau*).
 *   steps in 2..128, iters in 0..60;
 *   ws / ws_bytes: subquad_rmt_workspace_bytes(n, steps) bytes, 256-byte aligned.
 * subquad_rmt_lambda_max: the largest eigenvalue of A_low(tau) alone (tau = INFINITY: of A).
 */
size_t subquad_rmt_workspace_bytes(int64_t n, int32_t steps);
int subquad_rmt_threshold(const int64_t *row_offsets, const int32_t *cols, const float *vals,
                          int64_t n, int64_t nnz, int32_t steps, int32_t iters, uint64_t seed,
                          double *tau, double *lambda_plus, double *lambda_max, void *ws,
                          size_t ws_bytes, void *stream);
int subquad_rmt_lambda_max(const int64_t *row_offsets, const int32_t *cols, const float *vals,
                           int64_t n, int64_t nnz, double tau, int32_t steps, uint64_t seed,
                           double *lambda_max, void *ws, size_t ws_bytes, void *stream);

#ifdef __cplusplus
}
#endif

#endif /* SUBQUAD_H */
