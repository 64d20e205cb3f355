// Per-pair fusion over M = 3 channels (Sec. 3.6, Eq. (wm) and (afused) with a softmax over M
// channel logits): a = (s, c, e) with s the normalised alignment score, c the embedding
// cosine and e = 1 - d / (2 max(L_i, L_j)) the similarity of the doubled-cost edit distance
// d (Appendix F.3 recurrence).  Features x = (s, c, e, |L_i - L_j|, [V_i == V_j]).
//   z = W1 x + b1 (H), h = relu(z), g = W2 h + b2 (3), w = softmax(g), f = sum_m w_m a_m.
// Backward of L = sum_p gf_p f_p:
//   g_bar_m = gf w_m (a_m - f);  dW2 += g_bar h^T;  db2 += g_bar
//   z_bar = (W2^T g_bar) [z > 0];  dW1 += z_bar x^T;  db1 += z_bar
//   c_bar = gf w_c + (W1^T z_bar)_c, then the cosine gradient to both embeddings.
// Same CDNA4 mapping as the two-channel gate (16-lane groups, contiguous pair chunks,
// float64 weight-gradient accumulators).
#include "gate_util.h"

namespace subquad {

constexpr int kM = 3;  // channels
constexpr int kF = 5;  // features

struct GateMIn {
    const float *emb;
    int64_t n;
    int32_t d;
    const int32_t *lens, *vgene, *self, *pairs, *align, *dist;
    int64_t P;
    const float *W1, *b1, *W2, *b2;  // W1 [H][5], b1 [H], W2 [3][H], b2 [3]
    int32_t H;
};

template <int UNITS>
struct MWeights {
    float W1[UNITS][kF], b1[UNITS], W2[kM][UNITS], b2[kM];
};

template <int UNITS>
__device__ __forceinline__ void load_mweights(const GateMIn &in, int l, MWeights<UNITS> &w) {
#pragma unroll
    for (int k = 0; k < UNITS; ++k) {
        const int unit = l + kGroup * k;
#pragma unroll
        for (int q = 0; q < kF; ++q) w.W1[k][q] = in.W1[unit * kF + q];
        w.b1[k] = in.b1[unit];
#pragma unroll
        for (int m = 0; m < kM; ++m) w.W2[m][k] = in.W2[m * in.H + unit];
    }
#pragma unroll
    for (int m = 0; m < kM; ++m) w.b2[m] = in.b2[m];
}

template <int UNITS>
struct MState {
    float a[kM], x[kF], wm[kM], f, ni, nj;
    bool ok;
    float z[UNITS], h[UNITS];
};

template <int NV, int UNITS>
__device__ __forceinline__ void mpair_forward(const GateMIn &in, int64_t p, const float4 (&ei)[NV], float ni2,
                                              const float4 (&ej)[NV], int64_t i, int64_t j,
                                              const MWeights<UNITS> &w, MState<UNITS> &st) {
    float dot = 0.f, nj2 = 0.f;
#pragma unroll
    for (int k = 0; k < NV; ++k) {
        dot += dot4(ei[k], ej[k]);
        nj2 += dot4(ej[k], ej[k]);
    }
    dot = group_sum(dot);
    nj2 = group_sum(nj2);
    st.ni = sqrtf(ni2);
    st.nj = sqrtf(nj2);
    const float den = st.ni * st.nj;
    st.ok = den >= 1e-12f;
    const float c = st.ok ? dot / den : 0.f;
    const int Li = in.lens[i], Lj = in.lens[j];
    const float s = (float)in.align[p] / sqrtf((float)in.self[i] * (float)in.self[j]);
    const float e = 1.f - (float)in.dist[p] / (2.f * (float)max(Li, Lj));
    st.a[0] = s;
    st.a[1] = c;
    st.a[2] = e;
    st.x[0] = s;
    st.x[1] = c;
    st.x[2] = e;
    st.x[3] = fabsf((float)(Li - Lj));
    st.x[4] = in.vgene[i] == in.vgene[j] ? 1.f : 0.f;
    float g[kM] = {0.f, 0.f, 0.f};
#pragma unroll
    for (int k = 0; k < UNITS; ++k) {
        float z = w.b1[k];
#pragma unroll
        for (int q = 0; q < kF; ++q) z += w.W1[k][q] * st.x[q];
        st.z[k] = z;
        st.h[k] = fmaxf(z, 0.f);
#pragma unroll
        for (int m = 0; m < kM; ++m) g[m] += w.W2[m][k] * st.h[k];
    }
    float gmax = -INFINITY;
#pragma unroll
    for (int m = 0; m < kM; ++m) {
        g[m] = group_sum(g[m]) + w.b2[m];
        gmax = fmaxf(gmax, g[m]);
    }
    float den_s = 0.f;
#pragma unroll
    for (int m = 0; m < kM; ++m) {
        st.wm[m] = expf(g[m] - gmax);
        den_s += st.wm[m];
    }
    const float inv = 1.f / den_s;
    st.f = 0.f;
#pragma unroll
    for (int m = 0; m < kM; ++m) {
        st.wm[m] *= inv;
        st.f += st.wm[m] * st.a[m];
    }
}

__device__ __forceinline__ bool pair_in_range(int64_t i, int64_t j, int64_t n) {
    return i >= 0 && j >= 0 && i < n && j < n;
}

template <int NV, int UNITS>
__global__ __launch_bounds__(kGateThreads) void gate_m_fwd_kernel(GateMIn in, float *__restrict__ fused,
                                                                  float *__restrict__ weights) {
    const int l = threadIdx.x & (kGroup - 1);
    const int64_t group = ((int64_t)blockIdx.x * kGateThreads + threadIdx.x) / kGroup;
    const int64_t ngroups = (int64_t)gridDim.x * (kGateThreads / kGroup);
    const int64_t chunk = ceil_div(in.P, ngroups);
    const int64_t p0 = group * chunk, p1 = min(in.P, p0 + chunk);
    if (p0 >= p1) return;
    const int d4 = in.d >> 2;
    MWeights<UNITS> w;
    load_mweights<UNITS>(in, l, w);
    float4 ei[NV], ej[NV];
    float ni2 = 0.f;
    int64_t cur_i = -1;
    for (int64_t p = p0; p < p1; ++p) {
        const int64_t i = in.pairs[2 * p], j = in.pairs[2 * p + 1];
        if (!pair_in_range(i, j, in.n)) {
            if (l == 0) fused[p] = __builtin_nanf("");
            continue;
        }
        if (i != cur_i) {
            load_row<NV>(in.emb, i, d4, l, ei);
            float a = 0.f;
#pragma unroll
            for (int k = 0; k < NV; ++k) a += dot4(ei[k], ei[k]);
            ni2 = group_sum(a);
            cur_i = i;
        }
        load_row<NV>(in.emb, j, d4, l, ej);
        MState<UNITS> st;
        mpair_forward<NV, UNITS>(in, p, ei, ni2, ej, i, j, w, st);
        if (l == 0) {
            fused[p] = st.f;
            if (weights) {
#pragma unroll
                for (int m = 0; m < kM; ++m) weights[p * kM + m] = st.wm[m];
            }
        }
    }
}

// Workspace (doubles): dW1[H][5], db1[H], dW2[3][H], db2[3].
template <int NV, int UNITS>
__global__ __launch_bounds__(kGateThreads) void gate_m_bwd_kernel(GateMIn in, const float *__restrict__ gfused,
                                                                  float *__restrict__ demb, double *__restrict__ wacc) {
    const int l = threadIdx.x & (kGroup - 1);
    const int64_t group = ((int64_t)blockIdx.x * kGateThreads + threadIdx.x) / kGroup;
    const int64_t ngroups = (int64_t)gridDim.x * (kGateThreads / kGroup);
    const int64_t chunk = ceil_div(in.P, ngroups);
    const int64_t p0 = group * chunk, p1 = min(in.P, p0 + chunk);
    const int d4 = in.d >> 2;
    MWeights<UNITS> w;
    load_mweights<UNITS>(in, l, w);
    constexpr int kVals = UNITS * (kF + 1 + kM);  // per lane: dW1 row, db1, dW2 column
    double acc[kVals];
#pragma unroll
    for (int m = 0; m < kVals; ++m) acc[m] = 0.0;
    double ab2[kM] = {0.0, 0.0, 0.0};
    float4 ei[NV], ej[NV], gi[NV];
#pragma unroll
    for (int k = 0; k < NV; ++k) gi[k] = make_float4(0.f, 0.f, 0.f, 0.f);
    float ni2 = 0.f;
    int64_t cur_i = -1;
    auto flush_i = [&](int64_t row) {
        if (!demb || row < 0) return;
        float *base = demb + row * (int64_t)in.d;
#pragma unroll
        for (int k = 0; k < NV; ++k) {
            int c = l + kGroup * k;
            if (c < d4) {
                atomicAdd(base + 4 * c + 0, gi[k].x);
                atomicAdd(base + 4 * c + 1, gi[k].y);
                atomicAdd(base + 4 * c + 2, gi[k].z);
                atomicAdd(base + 4 * c + 3, gi[k].w);
            }
            gi[k] = make_float4(0.f, 0.f, 0.f, 0.f);
        }
    };
    for (int64_t p = p0; p < p1; ++p) {
        const int64_t i = in.pairs[2 * p], j = in.pairs[2 * p + 1];
        if (!pair_in_range(i, j, in.n)) continue;
        if (i != cur_i) {
            flush_i(cur_i);
            load_row<NV>(in.emb, i, d4, l, ei);
            float a = 0.f;
#pragma unroll
            for (int k = 0; k < NV; ++k) a += dot4(ei[k], ei[k]);
            ni2 = group_sum(a);
            cur_i = i;
        }
        load_row<NV>(in.emb, j, d4, l, ej);
        MState<UNITS> st;
        mpair_forward<NV, UNITS>(in, p, ei, ni2, ej, i, j, w, st);
        const float gf = gfused[p];
        float gbar[kM];
#pragma unroll
        for (int m = 0; m < kM; ++m) {
            gbar[m] = gf * st.wm[m] * (st.a[m] - st.f);
            if (l == 0) ab2[m] += (double)gbar[m];
        }
        float xc = 0.f;
#pragma unroll
        for (int k = 0; k < UNITS; ++k) {
            float hbar = 0.f;
#pragma unroll
            for (int m = 0; m < kM; ++m) {
                acc[k * (kF + 1 + kM) + kF + 1 + m] += (double)(gbar[m] * st.h[k]);
                hbar += w.W2[m][k] * gbar[m];
            }
            const float zbar = st.z[k] > 0.f ? hbar : 0.f;
#pragma unroll
            for (int q = 0; q < kF; ++q) acc[k * (kF + 1 + kM) + q] += (double)(zbar * st.x[q]);
            acc[k * (kF + 1 + kM) + kF] += (double)zbar;
            xc += zbar * w.W1[k][1];
        }
        const float cbar = gf * st.wm[1] + group_sum(xc);
        if (demb && st.ok) {
            const float c = st.a[1];
            const float inv = 1.f / (st.ni * st.nj);
            const float ci = c / (st.ni * st.ni), cj = c / (st.nj * st.nj);
            float *bj = demb + j * (int64_t)in.d;
#pragma unroll
            for (int k = 0; k < NV; ++k) {
                int cc = l + kGroup * k;
                if (cc < d4) {
                    gi[k].x += cbar * (ej[k].x * inv - ci * ei[k].x);
                    gi[k].y += cbar * (ej[k].y * inv - ci * ei[k].y);
                    gi[k].z += cbar * (ej[k].z * inv - ci * ei[k].z);
                    gi[k].w += cbar * (ej[k].w * inv - ci * ei[k].w);
                    atomicAdd(bj + 4 * cc + 0, cbar * (ei[k].x * inv - cj * ej[k].x));
                    atomicAdd(bj + 4 * cc + 1, cbar * (ei[k].y * inv - cj * ej[k].y));
                    atomicAdd(bj + 4 * cc + 2, cbar * (ei[k].z * inv - cj * ej[k].z));
                    atomicAdd(bj + 4 * cc + 3, cbar * (ei[k].w * inv - cj * ej[k].w));
                }
            }
        }
    }
    flush_i(cur_i);

    // block reduction: lanes with equal l own the same hidden units
#pragma unroll
    for (int m = 0; m < kVals; ++m) {
        acc[m] += __shfl_xor(acc[m], 16, 64);
        acc[m] += __shfl_xor(acc[m], 32, 64);
    }
#pragma unroll
    for (int m = 0; m < kM; ++m) {
        ab2[m] += __shfl_xor(ab2[m], 16, 64);
        ab2[m] += __shfl_xor(ab2[m], 32, 64);
    }
    __shared__ double red[kGateThreads / 64][kGroup][kVals + kM];
    const int wv = threadIdx.x >> 6, lw = threadIdx.x & 63;
    if (lw < kGroup) {
#pragma unroll
        for (int m = 0; m < kVals; ++m) red[wv][lw][m] = acc[m];
#pragma unroll
        for (int m = 0; m < kM; ++m) red[wv][lw][kVals + m] = ab2[m];
    }
    __syncthreads();
    const int H = in.H;
    for (int e = threadIdx.x; e < kGroup * (kVals + kM); e += kGateThreads) {
        const int ll = e / (kVals + kM), m = e - ll * (kVals + kM);
        double s = 0.0;
#pragma unroll
        for (int ww = 0; ww < kGateThreads / 64; ++ww) s += red[ww][ll][m];
        if (m >= kVals) {
            if (ll == 0) atomicAdd(&wacc[H * kF + H + kM * H + (m - kVals)], s);
            continue;
        }
        const int k = m / (kF + 1 + kM), q = m - k * (kF + 1 + kM);
        const int unit = ll + kGroup * k;
        double *dst;
        if (q < kF) dst = &wacc[unit * kF + q];
        else if (q == kF) dst = &wacc[H * kF + unit];
        else dst = &wacc[H * kF + H + (q - kF - 1) * H + unit];
        atomicAdd(dst, s);
    }
}

__global__ void gate_m_ws_zero_kernel(double *__restrict__ wacc, int count) {
    for (int k = threadIdx.x; k < count; k += blockDim.x) wacc[k] = 0.0;
}

__global__ void gate_m_ws_finish_kernel(const double *__restrict__ wacc, int H, float *__restrict__ dW1,
                                        float *__restrict__ db1, float *__restrict__ dW2, float *__restrict__ db2) {
    const int total = H * kF + H + kM * H + kM;
    for (int k = threadIdx.x; k < total; k += blockDim.x) {
        float v = (float)wacc[k];
        if (k < H * kF) dW1[k] += v;
        else if (k < H * kF + H) db1[k - H * kF] += v;
        else if (k < H * kF + H + kM * H) dW2[k - H * kF - H] += v;
        else db2[k - H * kF - H - kM * H] += v;
    }
}

static int gate_m_validate(const GateMIn &in) {
    SQ_REQUIRE(in.n >= 0 && in.P >= 0, SUBQUAD_ERR_ARG, "n and P must be >= 0");
    SQ_REQUIRE(in.d >= 4 && in.d <= 512 && in.d % 4 == 0, SUBQUAD_ERR_ARG, "d must be a multiple of 4 in 4..512");
    SQ_REQUIRE(in.H == 16 || in.H == 32 || in.H == 64, SUBQUAD_ERR_ARG, "H must be 16, 32 or 64");
    SQ_REQUIRE(in.P == 0 || (in.emb && in.lens && in.vgene && in.self && in.pairs && in.align && in.dist),
               SUBQUAD_ERR_ARG, "null input pointer");
    SQ_REQUIRE(in.W1 && in.b1 && in.W2 && in.b2, SUBQUAD_ERR_ARG, "null weight pointer");
    SQ_REQUIRE(((uintptr_t)in.emb & 15) == 0, SUBQUAD_ERR_ARG, "emb must be 16-byte aligned");
    return SUBQUAD_OK;
}

template <int NV, int UNITS>
static void launch_m(bool fwd, const GateMIn &in, float *fused, float *weights, const float *gf, float *demb,
                     double *wacc, hipStream_t st) {
    const int64_t blocks = gate_blocks_for(in.P, knob(SUBQUAD_KNOB_GATE_GROUPS_PER_CU));
    if (fwd) gate_m_fwd_kernel<NV, UNITS><<<(unsigned)blocks, kGateThreads, 0, st>>>(in, fused, weights);
    else gate_m_bwd_kernel<NV, UNITS><<<(unsigned)blocks, kGateThreads, 0, st>>>(in, gf, demb, wacc);
}

template <int NV>
static void launch_m_h(bool fwd, const GateMIn &in, float *fused, float *weights, const float *gf, float *demb,
                       double *wacc, hipStream_t st) {
    if (in.H == 16) launch_m<NV, 1>(fwd, in, fused, weights, gf, demb, wacc, st);
    else if (in.H == 32) launch_m<NV, 2>(fwd, in, fused, weights, gf, demb, wacc, st);
    else launch_m<NV, 4>(fwd, in, fused, weights, gf, demb, wacc, st);
}

static void launch_m_any(bool fwd, const GateMIn &in, float *fused, float *weights, const float *gf, float *demb,
                         double *wacc, hipStream_t st) {
    const int nv = (int)ceil_div(in.d / 4, kGroup);
    if (nv <= 1) launch_m_h<1>(fwd, in, fused, weights, gf, demb, wacc, st);
    else if (nv <= 2) launch_m_h<2>(fwd, in, fused, weights, gf, demb, wacc, st);
    else if (nv <= 4) launch_m_h<4>(fwd, in, fused, weights, gf, demb, wacc, st);
    else launch_m_h<8>(fwd, in, fused, weights, gf, demb, wacc, st);
}

}  // namespace subquad

using namespace subquad;

extern "C" int subquad_gate3_fwd(const float *emb, int64_t n, int32_t d, const int32_t *lens, const int32_t *vgene,
                                 const int32_t *self, const int32_t *pairs, const int32_t *align,
                                 const int32_t *dist, int64_t P, const float *W1, const float *b1, const float *W2,
                                 const float *b2, int32_t H, float *fused, float *weights, void *stream) {
    clear_error();
    GateMIn in{emb, n, d, lens, vgene, self, pairs, align, dist, P, W1, b1, W2, b2, H};
    int rc = gate_m_validate(in);
    if (rc != SUBQUAD_OK) return rc;
    SQ_REQUIRE(P == 0 || fused, SUBQUAD_ERR_ARG, "null output pointer");
    if (P == 0) return SUBQUAD_OK;
    hipStream_t st = as_stream(stream);
    {
        ProfScope prof("gate3_fwd_kernel", st);
        launch_m_any(true, in, fused, weights, nullptr, nullptr, nullptr, st);
    }
    SQ_LAUNCHED("gate_m_fwd_kernel");
    return SUBQUAD_OK;
}

extern "C" size_t subquad_gate3_bwd_workspace_bytes(int32_t H) {
    if (H <= 0) return 0;
    return align_up(sizeof(double) * (size_t)(H * kF + H + kM * H + kM), 256);
}

extern "C" int subquad_gate3_bwd(const float *emb, int64_t n, int32_t d, const int32_t *lens, const int32_t *vgene,
                                 const int32_t *self, const int32_t *pairs, const int32_t *align,
                                 const int32_t *dist, int64_t P, const float *W1, const float *b1, const float *W2,
                                 const float *b2, int32_t H, const float *grad_fused, float *dW1, float *db1,
                                 float *dW2, float *db2, float *demb, void *ws, size_t ws_bytes, void *stream) {
    clear_error();
    GateMIn in{emb, n, d, lens, vgene, self, pairs, align, dist, P, W1, b1, W2, b2, H};
    int rc = gate_m_validate(in);
    if (rc != SUBQUAD_OK) return rc;
    SQ_REQUIRE(dW1 && db1 && dW2 && db2, SUBQUAD_ERR_ARG, "null weight-gradient pointer");
    SQ_REQUIRE(P == 0 || grad_fused, SUBQUAD_ERR_ARG, "null grad_fused");
    SQ_REQUIRE(ws && ws_bytes >= subquad_gate3_bwd_workspace_bytes(H), SUBQUAD_ERR_WORKSPACE,
               "gate workspace too small");
    SQ_REQUIRE(((uintptr_t)ws & 255) == 0, SUBQUAD_ERR_ARG, "workspace must be 256-byte aligned");
    if (P == 0) return SUBQUAD_OK;
    hipStream_t st = as_stream(stream);
    double *wacc = static_cast<double *>(ws);
    const int total = H * kF + H + kM * H + kM;
    gate_m_ws_zero_kernel<<<1, 256, 0, st>>>(wacc, total);
    SQ_LAUNCHED("gate_m_ws_zero_kernel");
    {
        ProfScope prof("gate3_bwd_kernel", st);
        launch_m_any(false, in, nullptr, nullptr, grad_fused, demb, wacc, st);
    }
    SQ_LAUNCHED("gate_m_bwd_kernel");
    gate_m_ws_finish_kernel<<<1, 256, 0, st>>>(wacc, H, dW1, db1, dW2, db2);
    SQ_LAUNCHED("gate_m_ws_finish_kernel");
    return SUBQUAD_OK;
}
