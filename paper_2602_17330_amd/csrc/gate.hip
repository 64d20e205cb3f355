// Per-pair dynamic affinity fusion (Sec. 3.6, Eq. (wm) and (afused); sigmoid channel weight
// as in Eq. (alpha)), forward and backward.
//
//   s = A / sqrt(S_i S_j), c = cos(e_i, e_j), x = (s, c, |L_i - L_j|, [V_i == V_j])
//   z = W1 x + b1, h = relu(z), u = w2 . h + b2, g = sigmoid(u)   (softmax over (u, 0))
//   f = g s + (1 - g) c
// Backward of L = sum_p gf_p f_p, recomputing every intermediate:
//   u_bar = gf (s - c) g (1 - g);  dw2 += u_bar h;  db2 += u_bar
//   z_bar = u_bar w2 [z > 0];      dW1 += z_bar x^T; db1 += z_bar
//   c_bar = gf (1 - g) + (W1^T z_bar)_c
//   de_i += c_bar (e_j / (|e_i||e_j|) - c e_i / |e_i|^2), and symmetrically for e_j.
//
// Mapping to CDNA4: a group of 16 lanes per pair; lane l of the group loads float4 slices
// l, l + 16, ... of both embeddings (256-byte coalesced segments) and owns hidden units
// l, l + 16, ...; dot products and the logit are reduced with 16-wide shuffles.  A group
// walks a contiguous chunk of the (row-sorted) pair list, so e_i, |e_i| and, in the
// backward, the gradient of e_i stay in registers while the first index repeats.  Weight
// gradients are summed in float32 over each batch of 16 pairs, in float64 per block, and over
// blocks in a fixed order (gate_wgrad_kernel, gate_ws_reduce_kernel).
#include "gate_util.h"
#include "radix.h"

namespace subquad {

constexpr int kGateRing = 2;  // load slots of the first backward pass (3 or 4 cost a wave per SIMD)
static_assert(kGateRing <= 16, "lane u of a pair group stores ring slot u's records");
constexpr int kWeightStride = 8;  // floats per hidden unit of the LDS weight tables (two float4)
constexpr int kGateMaxH = 256;

struct GateIn {
    const float *emb;
    int64_t n;
    int32_t d;
    const int32_t *lens, *vgene, *self, *pairs, *align;
    int64_t P;
    const float *W1, *b1, *w2, *b2;
    int32_t H;
    // (self score, length, V-gene, label) per node, one 16-byte record: a partner costs one
    // gather instead of four.  NULL: the separate arrays above are read.
    const int4 *node;
    // When set, the number of pairs is min(*P_dev, P) read on the device (P is then the
    // capacity the launches are sized for).
    const int64_t *P_dev;
};

__device__ __forceinline__ int64_t live_pairs(const GateIn &in) { return live_count(in.P, in.P_dev); }

// node[k] = (self[k], lens[k], vgene[k], label ? label[k] : 0).
__global__ void gate_node_pack_kernel(const int32_t *__restrict__ self, const int32_t *__restrict__ lens,
                                      const int32_t *__restrict__ vgene, const int32_t *__restrict__ label, int64_t n,
                                      int4 *__restrict__ node) {
    for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < n; k += (int64_t)gridDim.x * blockDim.x)
        node[k] = make_int4(self[k], lens[k], vgene[k], label ? label[k] : 0);
}

// The MLP's weights in LDS, so that the gather kernels keep their registers for loads in
// flight: two tables of one 16-byte word per hidden unit, A[u] = W1's row u and
// B[u] = (b1[u], w2[u], W1[u][c] w2[u] (the unit's weight in the gradient by c), 0).  Lane l
// of a pair group reads unit l + 16 k, so a group's 16 reads cover 256 contiguous bytes
// (no bank conflicts; the groups of a wave read the same words).  The whole block calls it.
__device__ __forceinline__ void stage_weights(const GateIn &in, float *wsh) {
    float4 *A = reinterpret_cast<float4 *>(wsh), *B = A + kGateMaxH;
    for (int e = threadIdx.x; e < in.H; e += blockDim.x) {
        const float w0 = in.W1[e * 4 + 0], w1 = in.W1[e * 4 + 1], w2v = in.w2[e];
        A[e] = make_float4(w0, w1, in.W1[e * 4 + 2], in.W1[e * 4 + 3]);
        B[e] = make_float4(in.b1[e], w2v, w1 * w2v, 0.f);
    }
    __syncthreads();
}

__device__ __forceinline__ float4 weight_row(const float *wsh, int unit) {
    return reinterpret_cast<const float4 *>(wsh)[unit];
}
__device__ __forceinline__ float4 weight_aux(const float *wsh, int unit) {
    return reinterpret_cast<const float4 *>(wsh)[kGateMaxH + unit];
}

// One pair's inputs as loaded by a group, before any of them is used: the partner row e_j,
// the partner's node record and the pair's alignment score.  Loading is branch-free (an
// out-of-range pair loads node 0 and row 0), so a batch's loads are all in flight together.
template <int NV>
struct PairLoad {
    int32_t i;  // i < 0: no pair (past the chunk, or out of range)
    int4 nj;          // (self score, length, V-gene, label) of j (label 0 without packed records)
    int32_t al;
    float4 ej[NV];
};

// Node record of k: the packed one, or assembled from the separate arrays.
__device__ __forceinline__ int4 node_record(const GateIn &in, int64_t k) {
    return in.node ? in.node[k] : make_int4(in.self[k], in.lens[k], in.vgene[k], 0);
}

// PACKED: in.node is set (the backward packs the records first), and the loads go out with
// no branch between them.
template <int NV, bool PACKED = false>
__device__ __forceinline__ void load_pair(const GateIn &in, int64_t p, int64_t i, int64_t j, int d4, int l,
                                          PairLoad<NV> &pl) {
    const bool ok = p >= 0 && i >= 0 && j >= 0 && i < in.n && j < in.n;
    pl.i = ok ? (int32_t)i : -1;
    // no row to stand in when there are none (every pair is out of range; a PACKED caller
    // handles that case before it loads anything)
    if (!PACKED && in.n == 0) return;
    const int64_t js = ok ? j : 0, ps = ok ? p : 0;
    pl.nj = PACKED ? in.node[js] : node_record(in, js);
    pl.al = in.align[ps];
    if (PACKED) load_row_flat<NV>(in.emb, js, d4, l, pl.ej);
    else load_row<NV>(in.emb, js, d4, l, pl.ej);
}

// The pair's integer features: s = A / sqrt(S_i S_j), |L_i - L_j|, [V_i = V_j], same label.
struct PairFeat {
    float s, x2, x3;
    bool same_label;
};

template <int NV>
__device__ __forceinline__ PairFeat pair_features(const PairLoad<NV> &pl, int4 ni) {
    PairFeat f;
    f.s = (float)pl.al * rsqrt_fast((float)ni.x * (float)pl.nj.x);
    f.x2 = fabsf((float)(ni.y - pl.nj.y));
    f.x3 = ni.z == pl.nj.z ? 1.f : 0.f;
    f.same_label = ni.w == pl.nj.w;
    return f;
}

// Pre-activation of one hidden unit as one fixed fma chain, so that every kernel that
// evaluates it takes the same ReLU decision bit for bit.
__device__ __forceinline__ float unit_preact(const float (&w)[4], float b, float s, float c, float x2, float x3) {
    return fmaf(w[3], x3, fmaf(w[2], x2, fmaf(w[1], c, fmaf(w[0], s, b))));
}

// Forward quantities of one pair (all lanes of the group hold the same values on return,
// except z, the lane's own hidden units).
template <int UNITS>
struct PairState {
    float c, ni, nj, inv, g, gm, u;  // inv = 1 / (|e_i| |e_j|), 0 for a zero row
    bool ok;
    float z[UNITS];
};

template <int NV, int UNITS>
__device__ __forceinline__ void pair_forward(const float4 (&ei)[NV], float ni2, const PairLoad<NV> &pl,
                                             const PairFeat &ft, const float *wsh, int l, float b2,
                                             PairState<UNITS> &st) {
    float dot = 0.f, nj2 = 0.f;
#pragma unroll
    for (int k = 0; k < NV; ++k) {
        dot += dot4(ei[k], pl.ej[k]);
        nj2 += dot4(pl.ej[k], pl.ej[k]);
    }
    dot = group_sum(dot);
    nj2 = group_sum(nj2);
    st.ni = sqrt_fast(ni2);
    st.nj = sqrt_fast(nj2);
    const float den = st.ni * st.nj;
    st.ok = den >= 1e-12f;
    st.inv = st.ok ? rcp_fast(den) : 0.f;
    st.c = dot * st.inv;
    float part = 0.f;
#pragma unroll
    for (int k = 0; k < UNITS; ++k) {
        const float4 w = weight_row(wsh, l + kGroup * k), aux = weight_aux(wsh, l + kGroup * k);
        const float wv[4] = {w.x, w.y, w.z, w.w};
        st.z[k] = unit_preact(wv, aux.x, ft.s, st.c, ft.x2, ft.x3);
        part = fmaf(aux.y, fmaxf(st.z[k], 0.f), part);
    }
    st.u = group_sum(part) + b2;
    // g = sigmoid(u) and gm = 1 - g from one exponential of -|u| (no overflow, and gm
    // without the cancellation of 1 - g)
    const float t = exp2_fast(-fabsf(st.u) * 1.44269504f);
    const float r = rcp_fast(1.f + t);
    st.g = st.u >= 0.f ? r : t * r;
    st.gm = st.u >= 0.f ? t * r : r;
}

// f = g s + (1 - g) c as one fixed fma (the forward and the training pass agree bit for bit).
template <int UNITS>
__device__ __forceinline__ float fused_value(const PairState<UNITS> &st, const PairFeat &ft) {
    return fmaf(st.g, ft.s, st.gm * st.c);
}

template <int UNITS>
__device__ __forceinline__ void load_weights(const GateIn &in, int l, float (&W1)[UNITS][4], float (&b1)[UNITS],
                                             float (&w2)[UNITS], float &b2) {
#pragma unroll
    for (int k = 0; k < UNITS; ++k) {
        int unit = l + kGroup * k;
#pragma unroll
        for (int q = 0; q < 4; ++q) W1[k][q] = in.W1[unit * 4 + q];
        b1[k] = in.b1[unit];
        w2[k] = in.w2[unit];
    }
    b2 = in.b2[0];
}

template <int NV>
__device__ __forceinline__ void load_row_norm(const GateIn &in, int64_t i, int d4, int l, float4 (&ei)[NV], float &ni2) {
    load_row<NV>(in.emb, i, d4, l, ei);
    float a = 0.f;
#pragma unroll
    for (int k = 0; k < NV; ++k) a += dot4(ei[k], ei[k]);
    ni2 = group_sum(a);
}

template <int NV, int UNITS>
__global__ __launch_bounds__(kGateThreads) void gate_fwd_kernel(GateIn in, float *__restrict__ fused,
                                                                float *__restrict__ gate) {
    const int l = threadIdx.x & (kGroup - 1);
    const int64_t group = ((int64_t)blockIdx.x * kGateThreads + threadIdx.x) / kGroup;
    const int64_t ngroups = (int64_t)gridDim.x * (kGateThreads / kGroup);
    const int64_t P = live_pairs(in);
    const int64_t chunk = ceil_div(P, ngroups);
    const int64_t p0 = group * chunk, p1 = min(P, p0 + chunk);
    __shared__ __align__(16) float wsh[kGateMaxH * kWeightStride];
    stage_weights(in, wsh);
    if (p0 >= p1) return;
    const int d4 = in.d >> 2;
    const float b2 = in.b2[0];
    float4 ei[NV];
    float ni2 = 0.f;
    int4 ni = make_int4(0, 0, 0, 0);
    int64_t cur_i = -1;
    for (int64_t p = p0; p < p1; p += kGateBatch) {
        int64_t ib[kGateBatch], jb[kGateBatch];
#pragma unroll
        for (int u = 0; u < kGateBatch; ++u) {
            ib[u] = p + u < p1 ? in.pairs[2 * (p + u)] : -1;
            jb[u] = p + u < p1 ? in.pairs[2 * (p + u) + 1] : -1;
        }
        PairLoad<NV> pl[kGateBatch];
#pragma unroll
        for (int u = 0; u < kGateBatch; ++u) load_pair<NV>(in, p + u < p1 ? p + u : -1, ib[u], jb[u], d4, l, pl[u]);
#pragma unroll
        for (int u = 0; u < kGateBatch; ++u) {
            if (p + u >= p1) break;
            if (pl[u].i < 0) {  // out-of-range pair: no access
                if (l == 0) {
                    fused[p + u] = __builtin_nanf("");
                    if (gate) gate[p + u] = __builtin_nanf("");
                }
                continue;
            }
            if (pl[u].i != cur_i) {
                ni = node_record(in, pl[u].i);
                load_row_norm<NV>(in, pl[u].i, d4, l, ei, ni2);
                cur_i = pl[u].i;
            }
            const PairFeat ft = pair_features<NV>(pl[u], ni);
            PairState<UNITS> st;
            pair_forward<NV, UNITS>(ei, ni2, pl[u], ft, wsh, l, b2, st);
            if (l == 0) {
                fused[p + u] = fused_value(st, ft);
                if (gate) gate[p + u] = st.g;
            }
        }
    }
}

// The training signal of the fused pass: with TRAIN, grad_fused[p] is not read but formed
// from the pair's own fused value: the margin contrastive loss in similarity form on
// same-label pairs (y (1 - f)^2 + (1 - y) max(0, f - margin)^2, averaged over P), whose sum
// goes to one float64 partial per block; fused[p] is written when non-NULL.
struct TrainOut {
    float margin, inv_P;
    float *fused;
    double *loss_partial;
    bool set_demb;  // demb is written, not accumulated (rows without pairs are zeroed)
};

// First pass of the backward, over the pairs in order of their first index i (order_i: the
// records (i << 32 | p) sorted, or in their natural order when the pairs are sorted already):
// recomputes the forward, accumulates e_i's gradient in registers over its row, and stores
// per pair pack[p] = (cbar, c, 1 / (|e_i||e_j|), ubar) for the second pass and
// feat[p] = (s, c, |dL|, [V = V]) for the weight gradients.
//
// The gathers run ahead of the arithmetic through a ring of kGateRing slots: slot u holds
// the loads of one pair (e_j, j's node record, the alignment score and, when the pair starts
// a new row, e_i and i's node record), and as soon as its pair is computed the slot is
// refilled with the pair kGateRing places further on.  Every gather, including the row of
// the next i, is thus in flight while the pairs before it compute; the pair indices are
// fetched one ring turn further ahead still.
template <int NV>
struct RingSlot {
    int32_t p;  // pair number, -1: past the chunk
    int32_t i;  // -1: an out-of-range pair
    int4 nj, ni;  // node records of j and (new row only) of i
    int32_t al;
    float gf;   // upstream gradient (not TRAIN)
    float4 ej[NV], ei[NV];  // ei: new row only
};

// The walk of gate_bwd_kernel over the chunk [q0, q1) of one lane group (NATURAL: the pairs
// are in order of i, p = q; SET: demb is written, not added to); returns the group's sum of
// loss terms (TRAIN, lane 0).
template <int NV, int UNITS, bool TRAIN, bool NATURAL, bool SET>
__device__ __forceinline__ double gate_bwd_walk(const GateIn &in, const float *__restrict__ gfused,
                                                const uint64_t *__restrict__ order_i, const float *wsh,
                                                float4 *__restrict__ pack, float4 *__restrict__ feat,
                                                float *__restrict__ demb, const TrainOut &tr, int64_t P, int64_t q0,
                                                int64_t q1, int l, int d4, float b2, float4 (*stage)[2],
                                                float *fstage) {
    constexpr int R = kGateRing;
    double loss_acc = 0.0;
    if (q0 >= q1) return loss_acc;
    if (in.n == 0) {  // no rows: every pair is out of range
        for (int64_t q = q0 + l; q < q1; q += kGroup) {
            const int64_t p = NATURAL ? q : (int64_t)(uint32_t)order_i[q];
            pack[p] = make_float4(0.f, 0.f, 0.f, 0.f);
            feat[p] = make_float4(0.f, 0.f, 0.f, 0.f);
            if (TRAIN && tr.fused) tr.fused[p] = __builtin_nanf("");
        }
        return loss_acc;
    }
    const int64_t n = in.n;
    // the row of the record before the chunk: a first row equal to it started in another chunk
    const int64_t key_before = q0 > 0 ? (int64_t)(order_i[q0 - 1] >> 32) : -1;
    // e_i's gradient over its row is sum_p a_p e_j(p) - B e_i with a_p = cbar_p / (|e_i||e_j|)
    // and B = sum_p cbar_p c_p / |e_i|^2: gi holds the first sum, bsum the scalar B, and the
    // e_i term is applied once when the row is flushed.
    float4 ei[NV], gi[NV], old[NV];
#pragma unroll
    for (int k = 0; k < NV; ++k) {
        gi[k] = make_float4(0.f, 0.f, 0.f, 0.f);
        old[k] = make_float4(0.f, 0.f, 0.f, 0.f);
    }
    float bsum = 0.f;
    int64_t cur_i = -1;
    auto flush = [&](bool owned) {
#pragma unroll
        for (int k = 0; k < NV; ++k) {
            gi[k].x = fmaf(-bsum, ei[k].x, gi[k].x);
            gi[k].y = fmaf(-bsum, ei[k].y, gi[k].y);
            gi[k].z = fmaf(-bsum, ei[k].z, gi[k].z);
            gi[k].w = fmaf(-bsum, ei[k].w, gi[k].w);
        }
        bsum = 0.f;
        flush_row_pre<NV>(demb, cur_i, d4, l, gi, old, owned);
    };
    float ni2 = 0.f;
    int4 ni = make_int4(0, 0, 0, 0);
    bool started_here = false;
    // indices of the next ring turn: pair number, i and j of walk positions qb .. qb + R - 1
    // (clamped to the chunk's last pair, so that every load is unconditional)
    uint32_t pn[R];
    int32_t inx[R], jnx[R];
    auto fetch = [&](int64_t qb) {
#pragma unroll
        for (int u = 0; u < R; ++u) {
            const int64_t qq = min(qb + u, q1 - 1);
            const uint32_t pp = NATURAL ? (uint32_t)qq : (uint32_t)order_i[qq];
            pn[u] = pp;
            inx[u] = in.pairs[2 * (int64_t)pp];
            jnx[u] = in.pairs[2 * (int64_t)pp + 1];
        }
    };
    int32_t last_i = -1;  // i of the last pair put in the ring (-1: none, or out of range)
    RingSlot<NV> slot[R];
    // Slot u takes the pair at walk position q (its indices in pn[u], inx[u], jnx[u]).  The
    // loads of a live pair are unconditional; e_i and i's record are loaded when the pair's
    // row differs from the previous pair's.
    auto issue = [&](int u, int64_t q) {
        RingSlot<NV> &s = slot[u];
        const bool live = q < q1;
        const int32_t ii = inx[u], jj = jnx[u];
        const bool ok = live && ii >= 0 && jj >= 0 && ii < n && jj < n;
        s.p = live ? (int32_t)pn[u] : -1;
        s.i = ok ? ii : -1;
        const int64_t js = ok ? jj : 0, ps = pn[u];
        s.nj = in.node[js];
        s.al = in.align[ps];
        if (!TRAIN) s.gf = gfused[ps];
        load_row_flat<NV>(in.emb, js, d4, l, s.ej);
        if (ok && ii != last_i) {
            s.ni = in.node[ii];
            load_row_flat<NV>(in.emb, ii, d4, l, s.ei);
        }
        if (live) last_i = ok ? ii : -1;
    };
    fetch(q0);
#pragma unroll
    for (int u = 0; u < R; ++u) issue(u, q0 + u);
    fetch(q0 + R);
    for (int64_t q = q0; q < q1; q += R) {
        int32_t pb[R];
#pragma unroll
        for (int u = 0; u < R; ++u) {
            const RingSlot<NV> &s = slot[u];
            pb[u] = s.p;
            if (s.p >= 0) {
                if (s.i < 0) {  // out-of-range pair: skipped
                    if (l == 0) {
                        stage[u][0] = make_float4(0.f, 0.f, 0.f, 0.f);
                        stage[u][1] = make_float4(0.f, 0.f, 0.f, 0.f);
                        fstage[u] = __builtin_nanf("");
                    }
                } else {
                    const int64_t i = s.i;
                    if (i != cur_i) {
                        if (cur_i >= 0 && demb) flush(started_here);
                        // the row starts inside this chunk unless the record before the chunk is in it too
                        started_here = cur_i >= 0 || q0 == 0 || key_before != i;
                        cur_i = i;
                        if (demb && !SET) load_grad_row<NV>(demb, i, d4, l, old);
                        ni = s.ni;
                        float a = 0.f;
#pragma unroll
                        for (int k = 0; k < NV; ++k) {
                            ei[k] = s.ei[k];
                            a += dot4(ei[k], ei[k]);
                        }
                        ni2 = group_sum(a);
                    }
                    PairLoad<NV> pl;
                    pl.i = s.i;
                    pl.nj = s.nj;
                    pl.al = s.al;
#pragma unroll
                    for (int k = 0; k < NV; ++k) pl.ej[k] = s.ej[k];
                    const PairFeat ft = pair_features<NV>(pl, ni);
                    PairState<UNITS> st;
                    pair_forward<NV, UNITS>(ei, ni2, pl, ft, wsh, l, b2, st);
                    float gf;
                    if (TRAIN) {
                        const float f = fused_value(st, ft);
                        float lp;
                        if (ft.same_label) {
                            const float e = 1.f - f;
                            lp = e * e;
                            gf = -2.f * e * tr.inv_P;
                        } else {
                            const float h = fmaxf(f - tr.margin, 0.f);
                            lp = h * h;
                            gf = 2.f * h * tr.inv_P;
                        }
                        if (l == 0) {
                            loss_acc += (double)lp;
                            fstage[u] = f;
                        }
                    } else {
                        gf = s.gf;
                    }
                    const float ubar = gf * (ft.s - st.c) * st.g * st.gm;
                    float xc = 0.f;
#pragma unroll
                    for (int k = 0; k < UNITS; ++k) {
                        xc += st.z[k] > 0.f ? weight_aux(wsh, l + kGroup * k).z : 0.f;
                    }
                    const float cbar = gf * st.gm + ubar * group_sum(xc);
                    const float inv = st.inv;
                    if (l == 0) {
                        stage[u][0] = make_float4(st.ok ? cbar : 0.f, st.c, inv, ubar);
                        stage[u][1] = make_float4(ft.s, st.c, ft.x2, ft.x3);
                    }
                    if (demb && st.ok) {
                        const float a = cbar * inv;
                        bsum = fmaf(cbar * st.c, rcp_fast(ni2), bsum);
#pragma unroll
                        for (int k = 0; k < NV; ++k) {
                            gi[k].x = fmaf(a, pl.ej[k].x, gi[k].x);
                            gi[k].y = fmaf(a, pl.ej[k].y, gi[k].y);
                            gi[k].z = fmaf(a, pl.ej[k].z, gi[k].z);
                            gi[k].w = fmaf(a, pl.ej[k].w, gi[k].w);
                        }
                    }
                }
            }
            issue(u, q + R + u);  // the slot takes the pair one ring turn ahead
        }
        if (q + 2 * R < q1) fetch(q + 2 * R);
        // the turn's per-pair records leave together: lane u stores pair u's (consecutive
        // pairs give one contiguous store per array)
        int32_t mine = -1;
#pragma unroll
        for (int u = 0; u < R; ++u) mine = l == u ? pb[u] : mine;
        if (mine >= 0) {
            pack[mine] = stage[l][0];
            feat[mine] = stage[l][1];
            if (TRAIN && tr.fused) tr.fused[mine] = fstage[l];
        }
    }
    if (cur_i >= 0 && demb) {
        const bool ends_here = q1 == P || (int64_t)(order_i[q1] >> 32) != cur_i;
        flush(started_here && ends_here);
    }
    return loss_acc;
}

// (Three waves per SIMD: the register budget is capped at 168 so that the TRAIN variant
// keeps that occupancy.)
template <int NV, int UNITS, bool TRAIN, bool SET>
__global__ __launch_bounds__(kGateThreads) __attribute__((amdgpu_waves_per_eu(3))) void gate_bwd_kernel(
    GateIn in, const float *__restrict__ gfused, const uint64_t *__restrict__ order_nat,
    const uint64_t *__restrict__ order_sorted, const int64_t *__restrict__ unsorted, float4 *__restrict__ pack,
    float4 *__restrict__ feat, float *__restrict__ demb, TrainOut tr) {
    // Pairs already in order of i (the candidate lists are): walk them as they are, p = q.
    const bool natural = unsorted[0] == 0;
    const uint64_t *__restrict__ order_i = natural ? order_nat : order_sorted;
    const int64_t P = live_pairs(in);
    if (in.P_dev) tr.inv_P = 1.f / (float)(P > 0 ? P : 1);  // (the host forms it when P is known there)
    const int l = threadIdx.x & (kGroup - 1);
    const int64_t group = ((int64_t)blockIdx.x * kGateThreads + threadIdx.x) / kGroup;
    const int64_t ngroups = (int64_t)gridDim.x * (kGateThreads / kGroup);
    const int64_t chunk = gate_chunk(P, ngroups);
    const int d4 = in.d >> 2;
    __shared__ __align__(16) float wsh[kGateMaxH * kWeightStride];
    stage_weights(in, wsh);
    const float b2 = in.b2[0];
    // per lane group: the current batch's pack and feat records and fused values
    __shared__ float4 stage[kGateThreads / kGroup][kGateRing][2];
    __shared__ float fstage[kGateThreads / kGroup][kGateRing];
    const int g = threadIdx.x / kGroup;
    double loss_acc = 0.0;
    for (int64_t q0 = group * chunk; q0 < P; q0 += ngroups * chunk) {
        const int64_t q1 = min(P, q0 + chunk);
        loss_acc += natural ? gate_bwd_walk<NV, UNITS, TRAIN, true, SET>(in, gfused, order_i, wsh, pack, feat, demb, tr,
                                                                         P, q0, q1, l, d4, b2, stage[g], fstage[g])
                            : gate_bwd_walk<NV, UNITS, TRAIN, false, SET>(in, gfused, order_i, wsh, pack, feat, demb,
                                                                          tr, P, q0, q1, l, d4, b2, stage[g], fstage[g]);
    }
    if (TRAIN) {  // block sum of the loss terms (held by lane 0 of each group)
        __shared__ double red[kGateThreads];
        red[threadIdx.x] = loss_acc;
        __syncthreads();
        for (int o = kGateThreads / 2; o > 0; o >>= 1) {
            if (threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
            __syncthreads();
        }
        if (threadIdx.x == 0) tr.loss_partial[blockIdx.x] = red[0];
    }
}

// Weight gradients from the per-pair record of the first pass (a stream of 32 bytes per
// pair, no gathers): with ubar = dL/du and z = W1 x + b1 recomputed from x,
//   dW1[k] += ubar w2_k [z_k > 0] x,  db1[k] += ubar w2_k [z_k > 0],
//   dw2[k] += ubar relu(z_k),          db2 += ubar.
// Lane l of a 16-lane group owns units l + 16 m; each batch of 16 pairs is summed in
// float32 and added to float64 accumulators (a sixteenth of the float64 adds of one per
// term, which bound this kernel), reduced per block
// into column-major partials wpart[col][block] over the 6H + 1 values (dW1[H][4], db1[H],
// dw2[H], db2), which gate_ws_reduce_kernel sums in a fixed order (no atomics: the weight
// gradients are reproducible bit for bit).
template <int UNITS>
__global__ __launch_bounds__(kGateThreads) void gate_wgrad_kernel(GateIn in, const float4 *__restrict__ pack,
                                                                  const float4 *__restrict__ feat,
                                                                  double *__restrict__ wpart) {
    const int64_t P = live_pairs(in);
    const int l = threadIdx.x & (kGroup - 1);
    const int64_t group = ((int64_t)blockIdx.x * kGateThreads + threadIdx.x) / kGroup;
    const int64_t ngroups = (int64_t)gridDim.x * (kGateThreads / kGroup);
    const int64_t chunk = ceil_div(P, ngroups);
    const int64_t p0 = group * chunk, p1 = min(P, p0 + chunk);
    float W1[UNITS][4], b1[UNITS], w2[UNITS], b2;
    load_weights<UNITS>(in, l, W1, b1, w2, b2);
    double aW1[UNITS][4], ab1[UNITS], aw2[UNITS], ab2 = 0.0;
#pragma unroll
    for (int k = 0; k < UNITS; ++k) {
        ab1[k] = 0.0;
        aw2[k] = 0.0;
#pragma unroll
        for (int q = 0; q < 4; ++q) aW1[k][q] = 0.0;
    }
    for (int64_t pb = p0; pb < p1; pb += kGroup) {
        // lane t of the group loads pair pb + t; the group then walks the 16 pairs
        const int64_t mine = pb + l;
        const float4 f = mine < p1 ? feat[mine] : make_float4(0.f, 0.f, 0.f, 0.f);
        const float ub = mine < p1 ? pack[mine].w : 0.f;
        const int cnt = (int)min((int64_t)kGroup, p1 - pb);
        // the batch's (at most 16) terms are summed in float32, then added to the float64
        // accumulators once per batch
        float fW1[UNITS][4], fb1[UNITS], fw2[UNITS], fb2 = 0.f;
#pragma unroll
        for (int k = 0; k < UNITS; ++k) {
            fb1[k] = 0.f;
            fw2[k] = 0.f;
#pragma unroll
            for (int qq = 0; qq < 4; ++qq) fW1[k][qq] = 0.f;
        }
        for (int t = 0; t < cnt; ++t) {
            const float s = __shfl(f.x, t, kGroup), c = __shfl(f.y, t, kGroup);
            const float x2 = __shfl(f.z, t, kGroup), x3 = __shfl(f.w, t, kGroup);
            const float ubar = __shfl(ub, t, kGroup);
            const float x[4] = {s, c, x2, x3};
#pragma unroll
            for (int k = 0; k < UNITS; ++k) {
                const float z = unit_preact(W1[k], b1[k], s, c, x2, x3);
                fw2[k] = fmaf(ubar, fmaxf(z, 0.f), fw2[k]);
                const float zbar = z > 0.f ? ubar * w2[k] : 0.f;
#pragma unroll
                for (int qq = 0; qq < 4; ++qq) fW1[k][qq] = fmaf(zbar, x[qq], fW1[k][qq]);
                fb1[k] += zbar;
            }
            fb2 += ubar;
        }
#pragma unroll
        for (int k = 0; k < UNITS; ++k) {
            aw2[k] += (double)fw2[k];
            ab1[k] += (double)fb1[k];
#pragma unroll
            for (int qq = 0; qq < 4; ++qq) aW1[k][qq] += (double)fW1[k][qq];
        }
        if (l == 0) ab2 += (double)fb2;
    }

    // Block reduction: lanes with equal l hold the same units.
    constexpr int kVals = 6 * UNITS;
    double v[kVals];
#pragma unroll
    for (int k = 0; k < UNITS; ++k) {
#pragma unroll
        for (int qq = 0; qq < 4; ++qq) v[k * 6 + qq] = aW1[k][qq];
        v[k * 6 + 4] = ab1[k];
        v[k * 6 + 5] = aw2[k];
    }
#pragma unroll
    for (int m = 0; m < kVals; ++m) {
        v[m] += __shfl_xor(v[m], 16, 64);
        v[m] += __shfl_xor(v[m], 32, 64);
    }
    ab2 += __shfl_xor(ab2, 16, 64);
    ab2 += __shfl_xor(ab2, 32, 64);
    __shared__ double red[kGateThreads / 64][kGroup][kVals + 1];
    const int w = threadIdx.x >> 6, lw = threadIdx.x & 63;
    if (lw < kGroup) {
#pragma unroll
        for (int m = 0; m < kVals; ++m) red[w][lw][m] = v[m];
        red[w][lw][kVals] = ab2;
    }
    __syncthreads();
    for (int e = threadIdx.x; e < kGroup * (kVals + 1); e += kGateThreads) {
        const int ll = e / (kVals + 1), m = e - ll * (kVals + 1);
        double sacc = 0.0;
#pragma unroll
        for (int ww = 0; ww < kGateThreads / 64; ++ww) sacc += red[ww][ll][m];
        int col;
        if (m == kVals) {
            if (ll != 0) continue;  // every lane group holds the same db2 sum
            col = in.H * 6;
        } else {
            const int k = m / 6, qq = m - k * 6;
            const int unit = ll + kGroup * k;
            col = qq < 4 ? unit * 4 + qq : (qq == 4 ? in.H * 4 + unit : in.H * 5 + unit);
        }
        wpart[(int64_t)col * gridDim.x + blockIdx.x] = sacc;
    }
}

constexpr int kReduceThreads = 256;

// Column col of the weight-gradient partials summed over the nblocks blocks in a fixed
// order, rounded to float32 and added to its output.
__global__ __launch_bounds__(kReduceThreads) void gate_ws_reduce_kernel(const double *__restrict__ wpart,
                                                                        int64_t nblocks, int H,
                                                                        float *__restrict__ dW1,
                                                                        float *__restrict__ db1,
                                                                        float *__restrict__ dw2,
                                                                        float *__restrict__ db2) {
    __shared__ double red[kReduceThreads];
    const int col = blockIdx.x;
    const double *row = wpart + (int64_t)col * nblocks;
    double acc = 0.0;
    for (int64_t b = threadIdx.x; b < nblocks; b += kReduceThreads) acc += row[b];
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int half = kReduceThreads / 2; half > 0; half >>= 1) {
        if (threadIdx.x < half) red[threadIdx.x] += red[threadIdx.x + half];
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        const float v = (float)red[0];
        if (col < H * 4) dW1[col] += v;
        else if (col < H * 5) db1[col - H * 4] += v;
        else if (col < H * 6) dw2[col - H * 5] += v;
        else db2[0] += v;
    }
}

static int gate_validate(const GateIn &in) {
    SQ_REQUIRE(in.n >= 0 && in.P >= 0, SUBQUAD_ERR_ARG, "n and P must be >= 0");
    SQ_REQUIRE(in.d >= 4 && in.d <= 1024 && in.d % 4 == 0, SUBQUAD_ERR_ARG, "d must be a multiple of 4 in 4..1024");
    SQ_REQUIRE(in.H >= 16 && in.H <= 256 && in.H % 16 == 0, SUBQUAD_ERR_ARG, "H must be a multiple of 16 in 16..256");
    SQ_REQUIRE(in.P == 0 || (in.emb && in.lens && in.vgene && in.self && in.pairs && in.align), SUBQUAD_ERR_ARG,
               "null input pointer");
    SQ_REQUIRE(in.W1 && in.b1 && in.w2 && in.b2, SUBQUAD_ERR_ARG, "null weight pointer");
    SQ_REQUIRE(((uintptr_t)in.emb & 15) == 0, SUBQUAD_ERR_ARG, "emb must be 16-byte aligned");
    return SUBQUAD_OK;
}

static int64_t gate_max_blocks();

static int64_t gate_blocks(int64_t P, const void *kernel) {
    return std::min<int64_t>(gate_blocks_resident(P, knob(SUBQUAD_KNOB_GATE_GROUPS_PER_CU), kernel), gate_max_blocks());
}

template <int NV>
static int gate_fwd_nv(const GateIn &in, float *fused, float *gate, hipStream_t st) {
    ProfScope prof("gate_fwd_kernel", st);
    switch (in.H / kGroup) {
#define SQ_CASE(U)                                                                                                \
    case U:                                                                                                       \
        gate_fwd_kernel<NV, U><<<(unsigned)gate_blocks(in.P, (const void *)gate_fwd_kernel<NV, U>), kGateThreads, 0, \
                                 st>>>(in, fused, gate);                                                          \
        break;
        SQ_CASE(1) SQ_CASE(2) SQ_CASE(4) SQ_CASE(8) SQ_CASE(16)
#undef SQ_CASE
        default:
            set_error("H = %d is not one of 16, 32, 64, 128, 256", in.H);
            return SUBQUAD_ERR_ARG;
    }
    SQ_LAUNCHED("gate_fwd_kernel");
    return SUBQUAD_OK;
}

struct GateOrders {
    const uint64_t *order_nat;  // (i << 32 | p) in natural order
    const uint64_t *order_i;    // the same sorted by i (meaningful only when unsorted[0] != 0)
    const uint64_t *order_j;    // (j << 32 | p) sorted by j
    const int64_t *unsorted;    // [0]: 1 when the pairs are not in order of i, [1]: records the i sort takes
    hipEvent_t j_ready;         // recorded on the second stream once order_j is built
};

__global__ void fill_f32_kernel(float *__restrict__ x, int64_t count, float v) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count; i += (int64_t)gridDim.x * blockDim.x)
        x[i] = v;
}

// For a first pass that writes demb rather than adding to it: the rows it does not write are
// set to zero beforehand.  The i keys are in order (sorted, or the natural order the in-order
// check accepted), so the rows with no pair are the gaps between consecutive keys; and a row
// whose records straddle the start of a lane group's chunk (q = g * chunk) is added to
// atomically from both sides, so it starts from zero.  One lane per record q in [0, P]
// finds its rows to zero: the gap (key[q-1], key[q]) (with key[-1] = -1, key[P] = n), or at
// a chunk start the straddling row; then the whole wave zeroes each lane's rows in turn with
// contiguous stores.
__global__ __launch_bounds__(256) void gate_set_rows_prep_kernel(const uint64_t *__restrict__ order_nat,
                                                                 const uint64_t *__restrict__ order_sorted,
                                                                 const int64_t *__restrict__ unsorted, int64_t cap,
                                                                 const int64_t *__restrict__ P_dev, int64_t n,
                                                                 int64_t ngroups, int d4, float *__restrict__ demb) {
    const uint64_t *order_i = unsorted[0] == 0 ? order_nat : order_sorted;
    const int64_t P = live_count(cap, P_dev);
    const int64_t chunk = gate_chunk(P, ngroups);  // the first pass's chunk of pairs
    const int lane = threadIdx.x & 63;
    const int64_t nwaves = (int64_t)gridDim.x * (blockDim.x / 64);
    const float4 z = make_float4(0.f, 0.f, 0.f, 0.f);
    float4 *__restrict__ rows = reinterpret_cast<float4 *>(demb);
    // q0 is the same for every lane of a wave, so all lanes run the same iterations
    for (int64_t q0 = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / 64 * 64; q0 <= P; q0 += nwaves * 64) {
        const int64_t q = q0 + lane;
        int64_t lo = 0, hi = 0;  // rows [lo, hi) to zero
        if (q <= P) {
            const int64_t ka = q == 0 ? -1 : (int64_t)(order_i[q - 1] >> 32);
            const int64_t kb = q == P ? n : (int64_t)(order_i[q] >> 32);
            const int64_t a = ka < n ? ka : n, b = kb < n ? kb : n;
            lo = a + 1;
            hi = b;
            if (q > 0 && q < P && q % chunk == 0 && a == b && b < n) {  // the straddling row
                lo = b;
                hi = b + 1;
            }
        }
        uint64_t todo = __ballot(hi > lo);
        while (todo) {
            const int src = __builtin_ctzll(todo);
            todo &= todo - 1;
            const int64_t rlo = __shfl(lo, src), rhi = __shfl(hi, src);
            float4 *__restrict__ dst = rows + rlo * d4;
            const int64_t count = (rhi - rlo) * d4;
            for (int64_t e = lane; e < count; e += 64) dst[e] = z;
        }
    }
}

template <int NV, bool TRAIN>
static int gate_bwd_nv(const GateIn &in, const float *gf, const TrainOut &tr, int64_t *lblocks, const GateOrders &o,
                       float4 *pack, float4 *feat, float *demb, double *wpart, float *dW1, float *db1, float *dw2,
                       float *db2, hipStream_t st) {
    const uint64_t *order_j = o.order_j;
    switch (in.H / kGroup) {
#define SQ_CASE(U)                                                                                                 \
    case U: {                                                                                                      \
        {                                                                                                          \
            const auto kern = tr.set_demb ? gate_bwd_kernel<NV, U, TRAIN, true> : gate_bwd_kernel<NV, U, TRAIN, false>; \
            const int64_t blocks = gate_blocks(in.P, (const void *)kern);                                          \
            if (lblocks) *lblocks = blocks;                                                                        \
            if (demb && tr.set_demb) {                                                                             \
                const int64_t pblocks = std::min<int64_t>(ceil_div(in.P + 1, 256), gate_max_blocks() * 4);          \
                gate_set_rows_prep_kernel<<<(unsigned)pblocks, 256, 0, st>>>(o.order_nat, o.order_i, o.unsorted, in.P, \
                                                                             in.P_dev, in.n,                       \
                                                                             blocks * (kGateThreads / kGroup),    \
                                                                             in.d >> 2, demb);                     \
                SQ_LAUNCHED("gate_set_rows_prep_kernel");                                                          \
            }                                                                                                      \
            SQ_HIP(hipStreamWaitEvent(st, o.j_ready, 0)); /* the j order, built on the second stream */           \
            ProfScope prof("gate_bwd_kernel", st);                                                                 \
            kern<<<(unsigned)blocks, kGateThreads, 0, st>>>(in, gf, o.order_nat, o.order_i, o.unsorted, pack, feat,  \
                                                            demb, tr);                                             \
        }                                                                                                          \
        SQ_LAUNCHED("gate_bwd_kernel");                                                                            \
        {                                                                                                          \
            const int64_t blocks = gate_blocks(in.P, (const void *)gate_wgrad_kernel<U>);                          \
            ProfScope prof("gate_wgrad_kernel", st);                                                               \
            gate_wgrad_kernel<U><<<(unsigned)blocks, kGateThreads, 0, st>>>(in, pack, feat, wpart);                \
            SQ_LAUNCHED("gate_wgrad_kernel");                                                                      \
            gate_ws_reduce_kernel<<<(unsigned)(in.H * 6 + 1), kReduceThreads, 0, st>>>(wpart, blocks, in.H, dW1,     \
                                                                                       db1, dw2, db2);             \
        }                                                                                                          \
        SQ_LAUNCHED("gate_ws_reduce_kernel");                                                                      \
        break;                                                                                                     \
    }
        SQ_CASE(1) SQ_CASE(2) SQ_CASE(4) SQ_CASE(8) SQ_CASE(16)
#undef SQ_CASE
        default:
            set_error("H = %d is not one of 16, 32, 64, 128, 256", in.H);
            return SUBQUAD_ERR_ARG;
    }
    if (demb) {
        // one chunk per lane group unless the capacity needs several capped ones
        auto kern = gate_cos_bwd_j_kernel<NV, false>;
        int64_t blocks = gate_blocks(in.P, (const void *)kern);
        if (in.P > blocks * (kGateThreads / kGroup) * kGateChunkMax) {
            kern = gate_cos_bwd_j_kernel<NV, true>;
            blocks = gate_blocks(in.P, (const void *)kern);
        }
        ProfScope prof("gate_cos_bwd_j_kernel", st);
        kern<<<(unsigned)blocks, kGateThreads, 0, st>>>(in.emb, in.n, in.d, in.pairs, in.P, in.P_dev, order_j, pack,
                                                         demb);
    }
    SQ_LAUNCHED("gate_cos_bwd_j_kernel");
    return SUBQUAD_OK;
}

// Most blocks any chunked gate kernel is launched with (the resident-round cap).
static int64_t gate_max_blocks() { return (int64_t)device_cus() * 8; }

struct GateBwdLayout {
    size_t wpart, ra, rb, rc, rd, pack, feat, node, lpart, flags, radix, radix_j, total;
};

static GateBwdLayout gate_bwd_layout(int32_t H, int64_t P, int64_t n) {
    GateBwdLayout L{};
    size_t off = 0;
    auto take = [&](size_t bytes) { size_t o = off; off += align_up(std::max<size_t>(bytes, 1), 256); return o; };
    L.wpart = take(sizeof(double) * (size_t)(H * 6 + 1) * (size_t)gate_max_blocks());
    L.ra = take(sizeof(uint64_t) * P);
    L.rb = take(sizeof(uint64_t) * P);
    L.rc = take(sizeof(uint64_t) * P);
    L.rd = take(sizeof(uint64_t) * P);
    L.pack = take(sizeof(float4) * P);
    L.feat = take(sizeof(float4) * P);
    L.node = take(sizeof(int4) * n);
    L.lpart = take(sizeof(double) * (size_t)gate_max_blocks());
    L.flags = take(sizeof(int64_t) * 2);
    L.radix = take(radix_scratch_bytes(std::max<int64_t>(P, 1)));
    L.radix_j = take(radix_scratch_bytes(std::max<int64_t>(P, 1)));
    L.total = off;
    return L;
}

// flags[0] = 1 when some pair's i key (n for an out-of-range pair) exceeds the next one's.
__global__ void gate_sorted_init_kernel(int64_t *__restrict__ flags) {
    if (threadIdx.x == 0 && blockIdx.x == 0) flags[0] = 0;
}

__global__ void gate_sorted_check_kernel(const int32_t *__restrict__ pairs, int64_t cap,
                                         const int64_t *__restrict__ P_dev, int64_t n, int64_t *__restrict__ flags) {
    const int64_t P = live_count(cap, P_dev);
    for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p + 1 < P; p += (int64_t)gridDim.x * blockDim.x) {
        const int32_t a = pairs[2 * p], b = pairs[2 * p + 2];
        const int64_t ka = (a < 0 || a >= n || pairs[2 * p + 1] < 0 || pairs[2 * p + 1] >= n) ? n : a;
        const int64_t kb = (b < 0 || b >= n || pairs[2 * p + 3] < 0 || pairs[2 * p + 3] >= n) ? n : b;
        if (ka > kb) flags[0] = 1;  // every writer stores the same value
    }
}

// flags[1] = records the sort by i takes: P when the pairs are out of order, else none.
__global__ void gate_sorted_count_kernel(int64_t *__restrict__ flags, int64_t cap, const int64_t *__restrict__ P_dev) {
    if (threadIdx.x == 0 && blockIdx.x == 0) flags[1] = flags[0] ? live_count(cap, P_dev) : 0;
}

// Orders of the pair indices by their first and by their second index (stable, so each row
// keeps the input order) for the two backward passes.  When the pairs already come in order
// of i (the candidate lists do), the i sort is given no records and the first pass walks the
// pairs as they are.  The two orders depend only on the pairs: the j order is built on a
// second stream (its own sort scratch) while this one builds the i order and zeroes rows;
// the first pass waits for both (o.j_ready), so the two chains of small launches overlap.
static int gate_pair_orders(const int32_t *pairs, int64_t P, const int64_t *P_dev, int64_t n, char *ws,
                            const GateBwdLayout &L, hipStream_t st, GateOrders &o) {
    uint64_t *ra = reinterpret_cast<uint64_t *>(ws + L.ra), *rb = reinterpret_cast<uint64_t *>(ws + L.rb);
    uint64_t *rc = reinterpret_cast<uint64_t *>(ws + L.rc), *rd = reinterpret_cast<uint64_t *>(ws + L.rd);
    int64_t *flags = reinterpret_cast<int64_t *>(ws + L.flags);
    const int64_t blocks = std::min<int64_t>(ceil_div(P, 256), (int64_t)device_cus() * 16);
    const int bits = key_bits_for(n);
    const size_t sort_scratch = radix_scratch_bytes(std::max<int64_t>(P, 1));
    SideStream *side = nullptr;
    int rc_ = side_stream(&side);
    if (rc_ != SUBQUAD_OK) return rc_;
    SQ_HIP(hipEventRecord(side->fork, st));
    SQ_HIP(hipStreamWaitEvent(side->s, side->fork, 0));
    uint64_t *order_i = nullptr, *order_j = nullptr;
    gate_order_keys_kernel<<<(unsigned)blocks, 256, 0, side->s>>>(pairs, P, P_dev, n, 1, rc);
    SQ_LAUNCHED("gate_order_keys_kernel");
    rc_ = radix_sort_u64(rc, rd, P, P_dev, 32, bits, ws + L.radix_j, sort_scratch, side->s, &order_j, "sort_gate_j");
    if (rc_ != SUBQUAD_OK) return rc_;
    SQ_HIP(hipEventRecord(side->done, side->s));
    gate_sorted_init_kernel<<<1, 64, 0, st>>>(flags);
    SQ_LAUNCHED("gate_sorted_init_kernel");
    gate_sorted_check_kernel<<<(unsigned)blocks, 256, 0, st>>>(pairs, P, P_dev, n, flags);
    SQ_LAUNCHED("gate_sorted_check_kernel");
    gate_sorted_count_kernel<<<1, 64, 0, st>>>(flags, P, P_dev);
    SQ_LAUNCHED("gate_sorted_count_kernel");
    gate_order_keys_kernel<<<(unsigned)blocks, 256, 0, st>>>(pairs, P, P_dev, n, 0, ra);
    SQ_LAUNCHED("gate_order_keys_kernel");
    // With no records to sort (pairs already in order) the sort writes nothing and ra keeps
    // the natural order, which is then the one used; otherwise its result is.
    rc_ = radix_sort_u64(ra, rb, P, flags + 1, 32, bits, ws + L.radix, sort_scratch, st, &order_i, "sort_gate_i",
                         true);
    if (rc_ != SUBQUAD_OK) return rc_;
    o = GateOrders{ra, order_i, order_j, flags, side->done};
    return SUBQUAD_OK;
}

// ------------------------------------------------------------------ training signal

constexpr int kLossThreads = 256;

// Margin contrastive loss in similarity form on same-label pairs: per pair
// y (1 - f)^2 + (1 - y) max(0, f - margin)^2 with y = [label_i = label_j], averaged over P;
// grad[p] = its derivative by f_p.  One float64 partial per block (fixed order).
__global__ __launch_bounds__(kLossThreads) void contrastive_kernel(const float *__restrict__ fused,
                                                                   const int32_t *__restrict__ pairs, int64_t P,
                                                                   const int32_t *__restrict__ label, int64_t n,
                                                                   float margin, float *__restrict__ grad,
                                                                   double *__restrict__ partial) {
    const float invP = 1.f / (float)(P > 0 ? P : 1);
    double acc = 0.0;
    for (int64_t p = (int64_t)blockIdx.x * kLossThreads + threadIdx.x; p < P; p += (int64_t)gridDim.x * kLossThreads) {
        const int64_t i = pairs[2 * p], j = pairs[2 * p + 1];
        const bool ok = i >= 0 && j >= 0 && i < n && j < n;
        const float f = fused[p];
        float g = 0.f, l = 0.f;
        if (ok) {
            if (label[i] == label[j]) {
                const float e = 1.f - f;
                l = e * e;
                g = -2.f * e;
            } else {
                const float h = fmaxf(f - margin, 0.f);
                l = h * h;
                g = 2.f * h;
            }
        }
        grad[p] = g * invP;
        acc += (double)l;
    }
    __shared__ double red[kLossThreads];
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int o = kLossThreads / 2; o > 0; o >>= 1) {
        if (threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0) partial[blockIdx.x] = red[0];
}

__global__ void contrastive_final_kernel(const double *__restrict__ partial, int nb, int64_t cap,
                                         const int64_t *__restrict__ P_dev, double *__restrict__ loss) {
    const int64_t P = live_count(cap, P_dev);
    __shared__ double red[kLossThreads];
    double a = 0.0;
    for (int k = threadIdx.x; k < nb; k += kLossThreads) a += partial[k];
    red[threadIdx.x] = a;
    __syncthreads();
    for (int o = kLossThreads / 2; o > 0; o >>= 1) {
        if (threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0) loss[0] = red[0] / (double)(P > 0 ? P : 1);
}

static int contrastive_blocks() { return device_cus() * 4; }

}  // namespace subquad

using namespace subquad;

extern "C" int subquad_gate_fwd(const float *emb, int64_t n, int32_t d, const int32_t *lens, const int32_t *vgene,
                                const int32_t *self, const int32_t *pairs, const int32_t *align, int64_t P,
                                const float *W1, const float *b1, const float *w2, const float *b2, int32_t H,
                                float *fused, float *gate, void *stream) {
    clear_error();
    GateIn in{emb, n, d, lens, vgene, self, pairs, align, P, W1, b1, w2, b2, H};
    int rc = gate_validate(in);
    if (rc != SUBQUAD_OK) return rc;
    SQ_REQUIRE(P == 0 || fused, SUBQUAD_ERR_ARG, "null output pointer");
    if (P == 0) return SUBQUAD_OK;
    hipStream_t st = as_stream(stream);
    const int nv = (int)ceil_div(d / 4, kGroup);
    if (nv <= 1) return gate_fwd_nv<1>(in, fused, gate, st);
    if (nv <= 2) return gate_fwd_nv<2>(in, fused, gate, st);
    if (nv <= 4) return gate_fwd_nv<4>(in, fused, gate, st);
    if (nv <= 8) return gate_fwd_nv<8>(in, fused, gate, st);
    return gate_fwd_nv<16>(in, fused, gate, st);
}

extern "C" size_t subquad_gate_bwd_workspace_bytes(int32_t H, int64_t P, int64_t n) {
    if (H <= 0 || P < 0 || n < 0 || P >= (int64_t(1) << 32)) return 0;
    return gate_bwd_layout(H, P, n).total;
}

// The backward (TRAIN = false: upstream gradient given) or the fused training pass.
template <bool TRAIN>
static int gate_backward(const GateIn &in0, const int32_t *label, const float *grad_fused, float margin, float *fused,
                         double *loss, float *dW1, float *db1, float *dw2, float *db2, float *demb, void *ws,
                         size_t ws_bytes, void *stream, bool set_demb = false) {
    GateIn in = in0;
    int rc = gate_validate(in);
    if (rc != SUBQUAD_OK) return rc;
    SQ_REQUIRE(dW1 && db1 && dw2 && db2, SUBQUAD_ERR_ARG, "null weight-gradient pointer");
    if (TRAIN) {
        SQ_REQUIRE(loss, SUBQUAD_ERR_ARG, "null loss pointer");
        SQ_REQUIRE(in.P == 0 || label, SUBQUAD_ERR_ARG, "null label pointer");
        SQ_REQUIRE(margin == margin, SUBQUAD_ERR_ARG, "margin is NaN");
    } else {
        SQ_REQUIRE(in.P == 0 || grad_fused, SUBQUAD_ERR_ARG, "null grad_fused");
    }
    SQ_REQUIRE(in.P < (int64_t(1) << 32), SUBQUAD_ERR_ARG, "P must be below 2^32");
    const GateBwdLayout L = gate_bwd_layout(in.H, in.P, in.n);
    SQ_REQUIRE(ws && ws_bytes >= L.total, SUBQUAD_ERR_WORKSPACE, "gate workspace of %zu bytes, %zu needed", ws_bytes,
               L.total);
    SQ_REQUIRE(((uintptr_t)ws & 255) == 0, SUBQUAD_ERR_ARG, "workspace must be 256-byte aligned");
    SQ_REQUIRE(demb == nullptr || ((uintptr_t)demb & 15) == 0, SUBQUAD_ERR_ARG, "demb must be 16-byte aligned");
    hipStream_t st = as_stream(stream);
    char *w = static_cast<char *>(ws);
    double *lpart = reinterpret_cast<double *>(w + L.lpart);
    if (in.P == 0) {
        if (TRAIN) {
            contrastive_final_kernel<<<1, kLossThreads, 0, st>>>(lpart, 0, 0, nullptr, loss);
            SQ_LAUNCHED("contrastive_final_kernel");
        }
        if (set_demb && demb && in.n > 0) {  // no pairs: the written gradient is zero
            fill_f32_kernel<<<(unsigned)std::min<int64_t>(ceil_div(in.n * in.d, 256), (int64_t)device_cus() * 16), 256,
                              0, st>>>(demb, in.n * (int64_t)in.d, 0.f);
            SQ_LAUNCHED("fill_f32_kernel");
        }
        return SUBQUAD_OK;
    }
    double *wpart = reinterpret_cast<double *>(w + L.wpart);
    int4 *node = reinterpret_cast<int4 *>(w + L.node);
    if (in.n > 0) {
        gate_node_pack_kernel<<<(unsigned)std::min<int64_t>(ceil_div(in.n, 256), (int64_t)device_cus() * 16), 256, 0,
                                st>>>(in.self, in.lens, in.vgene, TRAIN ? label : nullptr, in.n, node);
        SQ_LAUNCHED("gate_node_pack_kernel");
    }
    in.node = node;
    GateOrders orders{};
    rc = gate_pair_orders(in.pairs, in.P, in.P_dev, in.n, w, L, st, orders);
    if (rc != SUBQUAD_OK) return rc;
    float4 *pack = reinterpret_cast<float4 *>(w + L.pack);
    float4 *feat = reinterpret_cast<float4 *>(w + L.feat);
    const TrainOut tr{margin, 1.f / (float)in.P, fused, lpart, set_demb};
    int64_t lblocks = 0;
    const int nv = (int)ceil_div(in.d / 4, kGroup);
    if (nv <= 1) rc = gate_bwd_nv<1, TRAIN>(in, grad_fused, tr, &lblocks, orders, pack, feat, demb, wpart, dW1, db1, dw2,
                                               db2, st);
    else if (nv <= 2) rc = gate_bwd_nv<2, TRAIN>(in, grad_fused, tr, &lblocks, orders, pack, feat, demb, wpart, dW1, db1, dw2,
                                               db2, st);
    else if (nv <= 4) rc = gate_bwd_nv<4, TRAIN>(in, grad_fused, tr, &lblocks, orders, pack, feat, demb, wpart, dW1, db1, dw2,
                                               db2, st);
    else if (nv <= 8) rc = gate_bwd_nv<8, TRAIN>(in, grad_fused, tr, &lblocks, orders, pack, feat, demb, wpart, dW1, db1, dw2,
                                               db2, st);
    else rc = gate_bwd_nv<16, TRAIN>(in, grad_fused, tr, &lblocks, orders, pack, feat, demb, wpart, dW1, db1, dw2,
                                               db2, st);
    if (rc != SUBQUAD_OK) return rc;
    if (TRAIN) {
        contrastive_final_kernel<<<1, kLossThreads, 0, st>>>(lpart, (int)lblocks, in.P, in.P_dev, loss);
        SQ_LAUNCHED("contrastive_final_kernel");
    }
    return SUBQUAD_OK;
}

extern "C" int subquad_gate_bwd(const float *emb, int64_t n, int32_t d, const int32_t *lens, const int32_t *vgene,
                                const int32_t *self, const int32_t *pairs, const int32_t *align, int64_t P,
                                const float *W1, const float *b1, const float *w2, const float *b2, int32_t H,
                                const float *grad_fused, float *dW1, float *db1, float *dw2, float *db2, float *demb,
                                void *ws, size_t ws_bytes, void *stream) {
    clear_error();
    const GateIn in{emb, n, d, lens, vgene, self, pairs, align, P, W1, b1, w2, b2, H, nullptr};
    return gate_backward<false>(in, nullptr, grad_fused, 0.f, nullptr, nullptr, dW1, db1, dw2, db2, demb, ws, ws_bytes,
                                stream);
}

extern "C" int subquad_gate_train(const float *emb, int64_t n, int32_t d, const int32_t *lens, const int32_t *vgene,
                                  const int32_t *self, const int32_t *pairs, const int32_t *align, int64_t P,
                                  const float *W1, const float *b1, const float *w2, const float *b2, int32_t H,
                                  const int32_t *label, float margin, float *fused, double *loss, float *dW1,
                                  float *db1, float *dw2, float *db2, float *demb, void *ws, size_t ws_bytes,
                                  void *stream) {
    clear_error();
    const GateIn in{emb, n, d, lens, vgene, self, pairs, align, P, W1, b1, w2, b2, H, nullptr};
    return gate_backward<true>(in, label, nullptr, margin, fused, loss, dW1, db1, dw2, db2, demb, ws, ws_bytes, stream);
}

extern "C" int subquad_gate_train_set(const float *emb, int64_t n, int32_t d, const int32_t *lens,
                                      const int32_t *vgene, const int32_t *self, const int32_t *pairs,
                                      const int32_t *align, int64_t P, const float *W1, const float *b1,
                                      const float *w2, const float *b2, int32_t H, const int32_t *label, float margin,
                                      float *fused, double *loss, float *dW1, float *db1, float *dw2, float *db2,
                                      float *demb, void *ws, size_t ws_bytes, void *stream) {
    clear_error();
    const GateIn in{emb, n, d, lens, vgene, self, pairs, align, P, W1, b1, w2, b2, H, nullptr};
    return gate_backward<true>(in, label, nullptr, margin, fused, loss, dW1, db1, dw2, db2, demb, ws, ws_bytes, stream,
                               true);
}

extern "C" int subquad_gate_train_set_dev(const float *emb, int64_t n, int32_t d, const int32_t *lens,
                                          const int32_t *vgene, const int32_t *self, const int32_t *pairs,
                                          const int32_t *align, int64_t cap, const int64_t *n_pairs_dev,
                                          const float *W1, const float *b1, const float *w2, const float *b2, int32_t H,
                                          const int32_t *label, float margin, float *fused, double *loss, float *dW1,
                                          float *db1, float *dw2, float *db2, float *demb, void *ws, size_t ws_bytes,
                                          void *stream) {
    clear_error();
    SQ_REQUIRE(n_pairs_dev, SUBQUAD_ERR_ARG, "null n_pairs_dev");
    const GateIn in{emb, n, d, lens, vgene, self, pairs, align, cap, W1, b1, w2, b2, H, nullptr, n_pairs_dev};
    return gate_backward<true>(in, label, nullptr, margin, fused, loss, dW1, db1, dw2, db2, demb, ws, ws_bytes, stream,
                               true);
}

extern "C" size_t subquad_contrastive_workspace_bytes(void) { return sizeof(double) * (size_t)contrastive_blocks(); }

extern "C" int subquad_contrastive_grad(const float *fused, const int32_t *pairs, int64_t P, const int32_t *label,
                                        int64_t n, float margin, float *grad, double *loss, void *ws, size_t ws_bytes,
                                        void *stream) {
    clear_error();
    SQ_REQUIRE(P >= 0 && n >= 0, SUBQUAD_ERR_ARG, "P and n must be >= 0");
    SQ_REQUIRE(P == 0 || (fused && pairs && label && grad), SUBQUAD_ERR_ARG, "null pointer argument");
    SQ_REQUIRE(margin == margin, SUBQUAD_ERR_ARG, "margin is NaN");
    const int nb = contrastive_blocks();
    SQ_REQUIRE(ws && ws_bytes >= sizeof(double) * (size_t)nb, SUBQUAD_ERR_WORKSPACE,
               "contrastive workspace of %zu bytes, %zu needed", ws_bytes, sizeof(double) * (size_t)nb);
    SQ_REQUIRE(((uintptr_t)ws & 7) == 0, SUBQUAD_ERR_ARG, "workspace must be 8-byte aligned");
    if (P == 0 && !loss) return SUBQUAD_OK;
    hipStream_t st = as_stream(stream);
    double *partial = static_cast<double *>(ws);
    contrastive_kernel<<<(unsigned)nb, kLossThreads, 0, st>>>(fused, pairs, P, label, n, margin, grad, partial);
    SQ_LAUNCHED("contrastive_kernel");
    if (loss) {
        contrastive_final_kernel<<<1, kLossThreads, 0, st>>>(partial, nb, P, nullptr, loss);
        SQ_LAUNCHED("contrastive_final_kernel");
    }
    return SUBQUAD_OK;
}
