// Prototype-contrastive loss and its gradient (Sec. 3, prototype-contrastive consolidation,
// Eq. (pc) and Eq. (proto)):
//   p_c = mean of the embedding rows with label c;
//   L   = sum over batch rows x of  logsumexp_c <e_x, p_c> / tau  -  <e_x, p_y(x)> / tau,
// the log-sum-exp running over every non-empty class (the positive one included).
//
// The logits form a B x C x d contraction, done on the matrix cores in float32
// (v_mfma_f32_32x32x2f32) with the transposed product Z^T = P E_B^T, so that each lane holds
// one batch row (a column of the 32 x 32 tile) and 16 of the tile's classes: the softmax
// statistics of a row stay inside one lane until the two lane halves are merged.
//   * forward: online (max, sum-exp) over class tiles, split over class ranges, merged per row;
//   * backward, like the backward of attention, recomputes each Z tile and forms
//     G = (softmax - onehot) * grad / tau in registers, then feeds G straight back into the
//     matrix cores: dE_B^T += P^T G^T for the batch rows and dP^T += E_B^T G for the classes;
//   * through Eq. (pc) every row r gets dP[y_r] / |S_y|.
// Operands stream through LDS in 32-row tiles with rows padded to d + 4 floats (conflict-free
// 16-byte reads); the fixed operand of each product stays in registers for the whole launch.
#include <algorithm>

#include "gate_util.h"
#include "radix.h"

namespace subquad {

typedef float f32x16 __attribute__((ext_vector_type(16)));

constexpr int kProtoThreads = 256;  // four waves, 32 fixed rows each
constexpr int kProtoRows = 128;     // fixed rows per block
constexpr int kMaxSplits = 32;

__device__ __forceinline__ f32x16 mfma32(float a, float b, f32x16 c) {
    return __builtin_amdgcn_mfma_f32_32x32x2f32(a, b, c, 0, 0, 0);
}

// Row of the 32 x 32 result held in accumulator v by lane half h (column = lane % 32).
__device__ __forceinline__ int acc_row(int v, int h) { return 8 * (v >> 2) + 4 * h + (v & 3); }

struct ProtoIn {
    const float *emb;
    int64_t n;
    const int32_t *labels;
    int64_t C;
    const int32_t *batch;
    int64_t B;
    float inv_tau;
};

// Batch row x -> table row, or -1 when x, its row index or its label is out of range.
__device__ __forceinline__ int64_t batch_row(const ProtoIn &in, int64_t x, int32_t &y) {
    y = -1;
    if (x >= in.B) return -1;
    const int64_t r = in.batch[x];
    if (r < 0 || r >= in.n) return -1;
    const int32_t c = in.labels[r];
    if (c < 0 || c >= in.C) return -1;
    y = c;
    return r;
}

// The 32-row operand held in registers: lane (column j, half h) keeps row j's elements
// [h d/2, (h+1) d/2).  Missing rows are zero.
template <int D>
__device__ __forceinline__ void load_fixed(const float *__restrict__ src, int64_t row, int h, float (&r)[D / 2]) {
    if (row < 0) {
#pragma unroll
        for (int q = 0; q < D / 2; ++q) r[q] = 0.f;
        return;
    }
    const float4 *p = reinterpret_cast<const float4 *>(src + row * D + h * (D / 2));
#pragma unroll
    for (int q = 0; q < D / 8; ++q) {
        const float4 v = p[q];
        r[4 * q] = v.x;
        r[4 * q + 1] = v.y;
        r[4 * q + 2] = v.z;
        r[4 * q + 3] = v.w;
    }
}

// Stages 32 rows (src row of tile entry i = rowof(i), -1 for zeros) into LDS.
template <int D>
constexpr int tile_per() { return (32 * (D / 4) + kProtoThreads - 1) / kProtoThreads; }  // float4 per thread

// A tile's rows loaded into registers, every load issued before any is used: an absent row
// (rowof < 0) reads row 0 and is zeroed with a bit mask (a select would let the compiler put
// the load behind a branch, with a wait after each).
template <int D, typename RowOf>
__device__ __forceinline__ void tile_load(const float *__restrict__ src, RowOf rowof, float4 (&v)[tile_per<D>()]) {
    constexpr int Q = D / 4;
#pragma unroll
    for (int u = 0; u < tile_per<D>(); ++u) {
        const int e = threadIdx.x + u * kProtoThreads;
        const int i = min(e / Q, 31), q = e - (e / Q) * Q;
        const int64_t row = rowof(i);
        v[u] = reinterpret_cast<const float4 *>(src + (row >= 0 ? row : 0) * D)[q];
        const int m = (row >= 0 && e < 32 * Q) ? -1 : 0;
        v[u] = make_float4(__int_as_float(__float_as_int(v[u].x) & m), __int_as_float(__float_as_int(v[u].y) & m),
                           __int_as_float(__float_as_int(v[u].z) & m), __int_as_float(__float_as_int(v[u].w) & m));
    }
}

template <int D>
__device__ __forceinline__ void tile_store(float *tile, const float4 (&v)[tile_per<D>()]) {
    constexpr int LD = D + 4, Q = D / 4;
#pragma unroll
    for (int u = 0; u < tile_per<D>(); ++u) {
        const int e = threadIdx.x + u * kProtoThreads;
        if (e < 32 * Q) *reinterpret_cast<float4 *>(tile + (e / Q) * LD + 4 * (e % Q)) = v[u];
    }
}

// Rows rowof(0..31) of src (D floats each; rowof < 0: zeros) into the LDS tile, rows padded
// to D + 4 floats.
template <int D, typename RowOf>
__device__ __forceinline__ void stage_tile(float *tile, const float *__restrict__ src, RowOf rowof) {
    float4 v[tile_per<D>()];
    tile_load<D>(src, rowof, v);
    tile_store<D>(tile, v);
}

// acc = sum_k tile[i][k] * fixed[j][k] for the 32 x 32 tile (i = tile row, j = lane column).
template <int D>
__device__ __forceinline__ f32x16 tile_product(const float *tile, const float (&r)[D / 2], int j, int h) {
    constexpr int LD = D + 4;
    const float *a = tile + j * LD + h * (D / 2);
    f32x16 acc = {};
#pragma unroll
    for (int q = 0; q < D / 2; q += 4) {
        const float4 av = *reinterpret_cast<const float4 *>(a + q);
        acc = mfma32(av.x, r[q], acc);
        acc = mfma32(av.y, r[q + 1], acc);
        acc = mfma32(av.z, r[q + 2], acc);
        acc = mfma32(av.w, r[q + 3], acc);
    }
    return acc;
}

// out[kb] (rows k = 32 kb + acc_row, column j) += sum_i tile[i][k] * g[i][j], where lane
// (j, h) holds g[acc_row(v, h)][j] in g[v]: the contraction runs over the tile rows in the
// order the accumulator layout gives them.
template <int D>
__device__ __forceinline__ void tile_product_t(const float *tile, const f32x16 &g, int j, int h, f32x16 (&out)[D / 32]) {
    constexpr int LD = D + 4;
#pragma unroll
    for (int s = 0; s < 16; ++s) {
        const float *a = tile + acc_row(s, h) * LD + j;
#pragma unroll
        for (int kb = 0; kb < D / 32; ++kb) out[kb] = mfma32(a[32 * kb], g[s], out[kb]);
    }
}

// ------------------------------------------------------------------ prototypes, Eq. (pc)

__global__ void proto_keys_kernel(const int32_t *__restrict__ labels, int64_t n, int64_t C, uint64_t *__restrict__ rec) {
    for (int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; r < n; r += (int64_t)gridDim.x * blockDim.x) {
        const int32_t c = labels[r];
        const uint64_t key = (c < 0 || c >= C) ? (uint64_t)C : (uint64_t)c;  // unlabelled rows sort last
        rec[r] = (key << 32) | (uint64_t)r;
    }
}

// Class sums over the rows sorted by label: a 16-lane group walks a contiguous chunk and
// keeps the current class's sum in registers; a class lying wholly in the chunk is stored,
// a class split between chunks is added atomically (float64).
template <int D>
__global__ __launch_bounds__(kGateThreads) void proto_sum_kernel(const float *__restrict__ emb, const uint64_t *__restrict__ sorted,
                                                                 int64_t n, int64_t C, double *__restrict__ psum,
                                                                 int32_t *__restrict__ count) {
    constexpr int NV = D / 64 > 0 ? D / 64 : 1, D4 = D / 4;
    const int l = threadIdx.x & (kGroup - 1);
    const int64_t group = ((int64_t)blockIdx.x * kGateThreads + threadIdx.x) / kGroup;
    const int64_t ngroups = (int64_t)gridDim.x * (kGateThreads / kGroup);
    const int64_t chunk = ceil_div(n, ngroups);
    const int64_t q0 = group * chunk, q1 = min(n, q0 + chunk);
    float4 acc[NV];
#pragma unroll
    for (int k = 0; k < NV; ++k) acc[k] = make_float4(0.f, 0.f, 0.f, 0.f);
    int64_t cur = -1, members = 0;
    bool started_here = false;
    auto flush = [&](bool owned) {
        double *base = psum + cur * D;
#pragma unroll
        for (int k = 0; k < NV; ++k) {
            const int c4 = l + kGroup * k;
            if (c4 < D4) {
                const float v[4] = {acc[k].x, acc[k].y, acc[k].z, acc[k].w};
#pragma unroll
                for (int e = 0; e < 4; ++e) {
                    if (owned) base[4 * c4 + e] = (double)v[e];
                    else atomicAdd(base + 4 * c4 + e, (double)v[e]);
                }
            }
            acc[k] = make_float4(0.f, 0.f, 0.f, 0.f);
        }
        if (l == 0) atomicAdd(count + cur, (int32_t)members);
        members = 0;
    };
    for (int64_t q = q0; q < q1; ++q) {
        const uint64_t rec = sorted[q];
        const int64_t c = (int64_t)(rec >> 32);
        if (c >= C) break;  // unlabelled rows are last
        if (c != cur) {
            if (cur >= 0) flush(started_here);
            cur = c;
            started_here = q0 == 0 || (int64_t)(sorted[q0 - 1] >> 32) != c;
        }
        const int64_t r = (int64_t)(uint32_t)rec;
        const float4 *row = reinterpret_cast<const float4 *>(emb + r * D);
#pragma unroll
        for (int k = 0; k < NV; ++k) {
            const int c4 = l + kGroup * k;
            if (c4 < D4) {
                const float4 v = row[c4];
                acc[k].x += v.x;
                acc[k].y += v.y;
                acc[k].z += v.z;
                acc[k].w += v.w;
            }
        }
        ++members;
    }
    if (cur >= 0) {
        const bool ends_here = q1 == n || (int64_t)(sorted[q1] >> 32) != cur;
        flush(started_here && ends_here);
    }
}

// p_c = sum / |S_c| in float32; inv[c] = 1 / |S_c| (0 for an empty class, which has no prototype).
__global__ void proto_scale_kernel(const double *__restrict__ psum, const int32_t *__restrict__ count, int64_t C, int D,
                                   float *__restrict__ P, float *__restrict__ inv) {
    const int64_t total = C * D;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += (int64_t)gridDim.x * blockDim.x) {
        const int64_t c = e / D;
        const int32_t m = count[c];
        P[e] = m > 0 ? (float)(psum[e] / (double)m) : 0.f;
        if (e - c * D == 0) inv[c] = m > 0 ? 1.f / (float)m : 0.f;
    }
}

template <class T>
__global__ void proto_fill_kernel(T *__restrict__ p, int64_t count, T v) {
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < count; e += (int64_t)gridDim.x * blockDim.x) p[e] = v;
}

// ------------------------------------------------------------------ forward, Eq. (proto)

// Per batch row and class split: (max logit m, sum over the negative classes of
// exp(logit - m), positive logit).  The positive class is kept out of the sum so that the
// loss and 1 - softmax(positive) can be formed without cancellation.
template <int D>
__global__ __launch_bounds__(kProtoThreads) void proto_fwd_kernel(ProtoIn in, const float *__restrict__ P,
                                                                  const float *__restrict__ inv, int64_t tiles_per_split,
                                                                  float4 *__restrict__ part) {
    constexpr int LD = D + 4;
    __shared__ __align__(16) float tile[32 * LD];
    __shared__ float tvalid[32];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6, h = lane >> 5, j = lane & 31;
    const int64_t x = (int64_t)blockIdx.x * kProtoRows + w * 32 + j;
    int32_t y;
    const int64_t row = batch_row(in, x, y);
    float r[D / 2];
    load_fixed<D>(in.emb, row, h, r);
    const int64_t ntiles = ceil_div(in.C, 32);
    const int64_t t0 = (int64_t)blockIdx.y * tiles_per_split, t1 = min(ntiles, t0 + tiles_per_split);
    float m = -INFINITY, s = 0.f, pos = -INFINITY;
    // the next tile's rows are loaded into registers while the current one is multiplied
    float4 nx[tile_per<D>()];
    float nvalid = 0.f;
    auto fetch = [&](int64_t t) {
        const int64_t c0 = t * 32;
        tile_load<D>(P, [&](int i) { return c0 + i < in.C ? c0 + i : (int64_t)-1; }, nx);
        if (threadIdx.x < 32) nvalid = (c0 + threadIdx.x < in.C && inv[c0 + threadIdx.x] > 0.f) ? 1.f : 0.f;
    };
    if (t0 < t1) fetch(t0);
    for (int64_t t = t0; t < t1; ++t) {
        __syncthreads();
        const int64_t c0 = t * 32;
        tile_store<D>(tile, nx);
        if (threadIdx.x < 32) tvalid[threadIdx.x] = nvalid;
        __syncthreads();
        if (t + 1 < t1) fetch(t + 1);
        const f32x16 acc = tile_product<D>(tile, r, j, h);
        float z[16], mt = -INFINITY;
#pragma unroll
        for (int v = 0; v < 16; ++v) {
            const int i = acc_row(v, h);
            z[v] = tvalid[i] > 0.f ? acc[v] * in.inv_tau : -INFINITY;
            if (c0 + i == y) pos = z[v];
            mt = fmaxf(mt, z[v]);
        }
        if (mt > m) {
            s *= expf(m - mt);
            m = mt;
        }
#pragma unroll
        for (int v = 0; v < 16; ++v)  // negatives only; exp(-inf) = 0 for missing classes
            if (c0 + acc_row(v, h) != y) s += expf(z[v] - m);
    }
    // merge the two lane halves of each column
    const float m2 = __shfl_xor(m, 32, 64), s2 = __shfl_xor(s, 32, 64), p2 = __shfl_xor(pos, 32, 64);
    const float M = fmaxf(m, m2);
    float S = 0.f;
    if (M > -INFINITY) S = (m > -INFINITY ? s * expf(m - M) : 0.f) + (m2 > -INFINITY ? s2 * expf(m2 - M) : 0.f);
    if (h == 0 && x < in.B) part[(int64_t)blockIdx.y * in.B + x] = make_float4(M, S, fmaxf(pos, p2), 0.f);
}

// Merges the class splits of every batch row.  With R = sum_{c != y} exp(z_c - z_y):
//   row loss = log(1 + R),  lse = z_y + log(1 + R),  1 - softmax_y = R / (1 + R),
// none of which cancels when the positive class dominates (a nearly perfect prediction).
// Writes lse and 1 - softmax_y for the backward, the row loss (0 for an excluded row) and
// one float64 partial sum per block.
__global__ __launch_bounds__(256) void proto_combine_kernel(ProtoIn in, const float4 *__restrict__ part, int splits,
                                                            float *__restrict__ lse, float *__restrict__ omp,
                                                            float *__restrict__ row_loss,
                                                            double *__restrict__ block_sum) {
    const int64_t x = (int64_t)blockIdx.x * 256 + threadIdx.x;
    double lx = 0.0;
    if (x < in.B) {
        int32_t y;
        const bool ok = batch_row(in, x, y) >= 0;
        float M = -INFINITY, pos = -INFINITY;
        for (int k = 0; k < splits; ++k) {
            const float4 p = part[(int64_t)k * in.B + x];
            M = fmaxf(M, p.x);
            pos = fmaxf(pos, p.z);
        }
        float Sneg = 0.f;
        for (int k = 0; k < splits; ++k) {
            const float4 p = part[(int64_t)k * in.B + x];
            if (p.x > -INFINITY) Sneg += p.y * expf(p.x - M);
        }
        float rl = 0.f, one_minus = 0.f;
        if (ok) {
            const float gap = M - pos;  // >= 0
            if (gap < 80.f) {
                const float R = Sneg * expf(gap);
                rl = log1pf(R);
                one_minus = R / (1.f + R);
            } else {  // the positive class is negligible: R overflows, softmax_y ~ e^-gap
                rl = gap + logf(Sneg);
                one_minus = 1.f;
            }
        }
        lse[x] = ok ? pos + rl : 0.f;
        omp[x] = one_minus;
        if (row_loss) row_loss[x] = rl;
        lx = (double)rl;
    }
    __shared__ double red[256];
    red[threadIdx.x] = lx;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if (threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0) block_sum[blockIdx.x] = red[0];
}

__global__ void proto_loss_final_kernel(const double *__restrict__ block_sum, int64_t nb, double *__restrict__ loss) {
    __shared__ double red[256];
    double a = 0.0;
    for (int64_t k = threadIdx.x; k < nb; k += 256) a += block_sum[k];
    red[threadIdx.x] = a;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if (threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0) loss[0] = red[0];
}

// ------------------------------------------------------------------ backward

// G[c][x] = (softmax_c(x) - [c = y(x)]) * grad / tau from a recomputed Z^T tile entry; for
// the positive class the stored 1 - softmax_y (no cancellation).
__device__ __forceinline__ float grad_logit(float zdot, float inv_tau, float lse_x, float omp_x, bool valid,
                                           bool positive, float gs) {
    if (positive) return -omp_x * gs;
    return valid ? expf(zdot * inv_tau - lse_x) * gs : 0.f;
}

// Batch-row side: dE[batch[x]] += sum_c G[c][x] p_c.  Fixed operand: the block's 128 batch
// rows; streamed: the class tiles of one split.
template <int D>
__global__ __launch_bounds__(kProtoThreads) void proto_bwd_rows_kernel(ProtoIn in, const float *__restrict__ P,
                                                                       const float *__restrict__ inv,
                                                                       const float *__restrict__ lse,
                                                                       const float *__restrict__ omp,
                                                                       const float *__restrict__ grad_loss,
                                                                       int64_t tiles_per_split, float *__restrict__ demb) {
    constexpr int LD = D + 4;
    __shared__ __align__(16) float tile[32 * LD];
    __shared__ float tvalid[32];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6, h = lane >> 5, j = lane & 31;
    const int64_t x = (int64_t)blockIdx.x * kProtoRows + w * 32 + j;
    int32_t y;
    const int64_t row = batch_row(in, x, y);
    float r[D / 2];
    load_fixed<D>(in.emb, row, h, r);
    const float lse_x = row >= 0 ? lse[x] : 0.f, omp_x = row >= 0 ? omp[x] : 0.f;
    const float gs = (grad_loss ? grad_loss[0] : 1.f) * in.inv_tau;
    f32x16 out[D / 32];
#pragma unroll
    for (int kb = 0; kb < D / 32; ++kb) out[kb] = f32x16{};
    const int64_t ntiles = ceil_div(in.C, 32);
    const int64_t t0 = (int64_t)blockIdx.y * tiles_per_split, t1 = min(ntiles, t0 + tiles_per_split);
    float4 nx[tile_per<D>()];  // the next tile, loaded during the current one's products
    float nvalid = 0.f;
    auto fetch = [&](int64_t t) {
        const int64_t c0 = t * 32;
        tile_load<D>(P, [&](int i) { return c0 + i < in.C ? c0 + i : (int64_t)-1; }, nx);
        if (threadIdx.x < 32) nvalid = (c0 + threadIdx.x < in.C && inv[c0 + threadIdx.x] > 0.f) ? 1.f : 0.f;
    };
    if (t0 < t1) fetch(t0);
    for (int64_t t = t0; t < t1; ++t) {
        __syncthreads();
        const int64_t c0 = t * 32;
        tile_store<D>(tile, nx);
        if (threadIdx.x < 32) tvalid[threadIdx.x] = nvalid;
        __syncthreads();
        if (t + 1 < t1) fetch(t + 1);
        f32x16 g = tile_product<D>(tile, r, j, h);
#pragma unroll
        for (int v = 0; v < 16; ++v) {
            const int i = acc_row(v, h);
            g[v] = grad_logit(g[v], in.inv_tau, lse_x, omp_x, row >= 0 && tvalid[i] > 0.f, c0 + i == y, gs);
        }
        tile_product_t<D>(tile, g, j, h, out);
    }
    if (row < 0) return;
    float *dst = demb + row * D;
#pragma unroll
    for (int kb = 0; kb < D / 32; ++kb)
#pragma unroll
        for (int v = 0; v < 16; ++v) atomicAdd(dst + 32 * kb + acc_row(v, h), out[kb][v]);
}

// Class side: dP[c] = sum_x G[c][x] e_x.  Fixed operand: the block's 128 prototypes;
// streamed: the batch-row tiles of one split.  With one split every class is written
// once (plain store), otherwise added atomically into a zeroed dP.
template <int D>
__global__ __launch_bounds__(kProtoThreads) void proto_bwd_protos_kernel(ProtoIn in, const float *__restrict__ P,
                                                                         const float *__restrict__ inv,
                                                                         const float *__restrict__ lse,
                                                                         const float *__restrict__ omp,
                                                                         const float *__restrict__ grad_loss,
                                                                         int64_t tiles_per_split, bool atomic,
                                                                         float *__restrict__ dP) {
    constexpr int LD = D + 4;
    __shared__ __align__(16) float tile[32 * LD];
    __shared__ float tlse[32], tomp[32];
    __shared__ int32_t tlab[32];
    __shared__ int64_t trow[32];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6, h = lane >> 5, j = lane & 31;
    const int64_t c = (int64_t)blockIdx.x * kProtoRows + w * 32 + j;
    const bool cvalid = c < in.C && inv[c] > 0.f;
    float r[D / 2];
    load_fixed<D>(P, cvalid ? c : -1, h, r);
    const float gs = (grad_loss ? grad_loss[0] : 1.f) * in.inv_tau;
    f32x16 out[D / 32];
#pragma unroll
    for (int kb = 0; kb < D / 32; ++kb) out[kb] = f32x16{};
    const int64_t ntiles = ceil_div(in.B, 32);
    const int64_t t0 = (int64_t)blockIdx.y * tiles_per_split, t1 = min(ntiles, t0 + tiles_per_split);
    for (int64_t t = t0; t < t1; ++t) {
        __syncthreads();
        const int64_t x0 = t * 32;
        if (threadIdx.x < 32) {
            int32_t y;
            const int64_t rr = batch_row(in, x0 + threadIdx.x, y);
            trow[threadIdx.x] = rr;
            tlab[threadIdx.x] = rr >= 0 ? y : -1;
            tlse[threadIdx.x] = rr >= 0 ? lse[x0 + threadIdx.x] : 0.f;
            tomp[threadIdx.x] = rr >= 0 ? omp[x0 + threadIdx.x] : 0.f;
        }
        __syncthreads();
        stage_tile<D>(tile, in.emb, [&](int i) { return trow[i]; });
        __syncthreads();
        f32x16 g = tile_product<D>(tile, r, j, h);
#pragma unroll
        for (int v = 0; v < 16; ++v) {
            const int i = acc_row(v, h);
            g[v] = grad_logit(g[v], in.inv_tau, tlse[i], tomp[i], cvalid && tlab[i] >= 0, tlab[i] == c, gs);
        }
        tile_product_t<D>(tile, g, j, h, out);
    }
    if (c >= in.C) return;
    float *dst = dP + c * D;
#pragma unroll
    for (int kb = 0; kb < D / 32; ++kb)
#pragma unroll
        for (int v = 0; v < 16; ++v) {
            if (atomic) atomicAdd(dst + 32 * kb + acc_row(v, h), out[kb][v]);
            else dst[32 * kb + acc_row(v, h)] = out[kb][v];
        }
}

// Through Eq. (pc): dE[r] += dP[y_r] / |S_y| for every labelled row.
template <int D>
__global__ void proto_route_kernel(const int32_t *__restrict__ labels, int64_t n, int64_t C, const float *__restrict__ dP,
                                   const float *__restrict__ inv, float *__restrict__ demb) {
    constexpr int Q = D / 4;
    const int64_t total = n * Q;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += (int64_t)gridDim.x * blockDim.x) {
        const int64_t r = e / Q;
        const int q = (int)(e - r * Q);
        const int32_t c = labels[r];
        if (c < 0 || c >= C) continue;
        const float s = inv[c];
        const float4 g = reinterpret_cast<const float4 *>(dP + (int64_t)c * D)[q];
        float4 *d = reinterpret_cast<float4 *>(demb) + e;
        float4 v = *d;
        v.x += g.x * s;
        v.y += g.y * s;
        v.z += g.z * s;
        v.w += g.w * s;
        *d = v;
    }
}

// ------------------------------------------------------------------ host side

struct ProtoLayout {
    size_t ra, rb, radix, psum, P, count, inv, part, lse, omp, bsum, dP, total;
};

static ProtoLayout proto_layout(int64_t n, int32_t d, int64_t C, int64_t B) {
    ProtoLayout L{};
    size_t off = 0;
    auto take = [&](size_t bytes) { size_t o = off; off += align_up(std::max<size_t>(bytes, 1), 256); return o; };
    const int64_t n1 = std::max<int64_t>(n, 1);
    L.ra = take(sizeof(uint64_t) * n1);
    L.rb = take(sizeof(uint64_t) * n1);
    L.radix = take(radix_scratch_bytes(n1));
    L.psum = take(sizeof(double) * C * d);
    L.P = take(sizeof(float) * C * d);
    L.count = take(sizeof(int32_t) * C);
    L.inv = take(sizeof(float) * C);
    L.part = take(sizeof(float4) * kMaxSplits * B);
    L.lse = take(sizeof(float) * B);
    L.omp = take(sizeof(float) * B);
    L.bsum = take(sizeof(double) * ceil_div(std::max<int64_t>(B, 1), 256));
    L.dP = take(sizeof(float) * C * d);
    L.total = off;
    return L;
}

static int64_t grid1d(int64_t work, int threads) {
    return std::max<int64_t>(1, std::min<int64_t>(ceil_div(work, threads), (int64_t)device_cus() * 16));
}

// Splits of the streamed dimension so that a launch has about four blocks per CU.
static void plan_splits(int64_t fixed_blocks, int64_t stream_tiles, int64_t &splits, int64_t &tiles_per_split) {
    const int64_t want = ceil_div((int64_t)device_cus() * 4, std::max<int64_t>(fixed_blocks, 1));
    splits = std::max<int64_t>(1, std::min<int64_t>({want, (int64_t)kMaxSplits, std::max<int64_t>(stream_tiles, 1)}));
    tiles_per_split = ceil_div(std::max<int64_t>(stream_tiles, 1), splits);
    splits = ceil_div(std::max<int64_t>(stream_tiles, 1), tiles_per_split);
}

static int proto_validate(const float *emb, int64_t n, int32_t d, const int32_t *labels, int64_t C, const int32_t *batch,
                          int64_t B, float tau, void *ws, size_t ws_bytes, ProtoLayout &L) {
    SQ_REQUIRE(n >= 0 && B >= 0 && C >= 1, SUBQUAD_ERR_ARG, "need n >= 0, B >= 0, C >= 1");
    SQ_REQUIRE(n < (int64_t(1) << 32) && C < (int64_t(1) << 31) && B < (int64_t(1) << 40), SUBQUAD_ERR_ARG,
               "n must be below 2^32 and C below 2^31");
    SQ_REQUIRE(d == 32 || d == 64 || d == 128, SUBQUAD_ERR_ARG, "d must be 32, 64 or 128 (got %d)", d);
    SQ_REQUIRE(tau > 0.f && tau < INFINITY, SUBQUAD_ERR_ARG, "tau must be positive and finite");
    SQ_REQUIRE((n == 0 || (emb && labels)) && (B == 0 || batch), SUBQUAD_ERR_ARG, "null pointer argument");
    SQ_REQUIRE(((uintptr_t)emb & 15) == 0, SUBQUAD_ERR_ARG, "emb must be 16-byte aligned");
    L = proto_layout(n, d, C, B);
    SQ_REQUIRE(ws && ws_bytes >= L.total, SUBQUAD_ERR_WORKSPACE, "proto workspace of %zu bytes, %zu needed", ws_bytes,
               L.total);
    SQ_REQUIRE(((uintptr_t)ws & 255) == 0, SUBQUAD_ERR_ARG, "workspace must be 256-byte aligned");
    return SUBQUAD_OK;
}

template <int D>
static int proto_fwd_d(const ProtoIn &in, char *w, const ProtoLayout &L, double *loss, float *row_loss, float *protos,
                       hipStream_t st) {
    double *psum = reinterpret_cast<double *>(w + L.psum);
    float *P = reinterpret_cast<float *>(w + L.P), *inv = reinterpret_cast<float *>(w + L.inv);
    int32_t *count = reinterpret_cast<int32_t *>(w + L.count);
    {
        ProfScope prof("proto_prototypes", st);
        proto_fill_kernel<double><<<(unsigned)grid1d(in.C * D, 256), 256, 0, st>>>(psum, in.C * D, 0.0);
        SQ_LAUNCHED("proto_fill_kernel");
        proto_fill_kernel<int32_t><<<(unsigned)grid1d(in.C, 256), 256, 0, st>>>(count, in.C, 0);
        SQ_LAUNCHED("proto_fill_kernel");
        if (in.n > 0) {
            uint64_t *ra = reinterpret_cast<uint64_t *>(w + L.ra), *rb = reinterpret_cast<uint64_t *>(w + L.rb);
            proto_keys_kernel<<<(unsigned)grid1d(in.n, 256), 256, 0, st>>>(in.labels, in.n, in.C, ra);
            SQ_LAUNCHED("proto_keys_kernel");
            uint64_t *sorted = nullptr;
            int rc = radix_sort_u64(ra, rb, in.n, nullptr, 32, key_bits_for(in.C), w + L.radix, L.psum - L.radix, st,
                                    &sorted, "sort_labels");
            if (rc != SUBQUAD_OK) return rc;
            proto_sum_kernel<D><<<(unsigned)gate_blocks_for(in.n, 64), kGateThreads, 0, st>>>(in.emb, sorted, in.n, in.C,
                                                                                               psum, count);
            SQ_LAUNCHED("proto_sum_kernel");
        }
        proto_scale_kernel<<<(unsigned)grid1d(in.C * D, 256), 256, 0, st>>>(psum, count, in.C, D, P, inv);
        SQ_LAUNCHED("proto_scale_kernel");
    }
    if (protos) SQ_HIP(hipMemcpyAsync(protos, P, sizeof(float) * in.C * D, hipMemcpyDeviceToDevice, st));
    const int64_t nb = ceil_div(std::max<int64_t>(in.B, 1), 256);
    double *bsum = reinterpret_cast<double *>(w + L.bsum);
    if (in.B > 0) {
        float4 *part = reinterpret_cast<float4 *>(w + L.part);
        const int64_t bx = ceil_div(in.B, kProtoRows);
        int64_t splits, tps;
        plan_splits(bx, ceil_div(in.C, 32), splits, tps);
        {
            ProfScope prof("proto_fwd_kernel", st);
            proto_fwd_kernel<D><<<dim3((unsigned)bx, (unsigned)splits), kProtoThreads, 0, st>>>(in, P, inv, tps, part);
        }
        SQ_LAUNCHED("proto_fwd_kernel");
        proto_combine_kernel<<<(unsigned)nb, 256, 0, st>>>(in, part, (int)splits, reinterpret_cast<float *>(w + L.lse),
                                                           reinterpret_cast<float *>(w + L.omp), row_loss, bsum);
        SQ_LAUNCHED("proto_combine_kernel");
    } else {
        proto_fill_kernel<double><<<1, 256, 0, st>>>(bsum, 1, 0.0);
        SQ_LAUNCHED("proto_fill_kernel");
    }
    proto_loss_final_kernel<<<1, 256, 0, st>>>(bsum, in.B > 0 ? nb : 1, loss);
    SQ_LAUNCHED("proto_loss_final_kernel");
    return SUBQUAD_OK;
}

template <int D>
static int proto_bwd_d(const ProtoIn &in, char *w, const ProtoLayout &L, const float *grad_loss, bool through,
                       float *demb, hipStream_t st) {
    if (in.B == 0) return SUBQUAD_OK;
    const float *P = reinterpret_cast<const float *>(w + L.P), *inv = reinterpret_cast<const float *>(w + L.inv);
    const float *lse = reinterpret_cast<const float *>(w + L.lse), *omp = reinterpret_cast<const float *>(w + L.omp);
    {
        const int64_t bx = ceil_div(in.B, kProtoRows);
        int64_t splits, tps;
        plan_splits(bx, ceil_div(in.C, 32), splits, tps);
        ProfScope prof("proto_bwd_rows_kernel", st);
        proto_bwd_rows_kernel<D><<<dim3((unsigned)bx, (unsigned)splits), kProtoThreads, 0, st>>>(in, P, inv, lse, omp,
                                                                                                 grad_loss, tps, demb);
    }
    SQ_LAUNCHED("proto_bwd_rows_kernel");
    if (!through || in.n == 0) return SUBQUAD_OK;  // (no rows: nothing routes back; tiles stage emb rows)
    float *dP = reinterpret_cast<float *>(w + L.dP);
    {
        const int64_t bx = ceil_div(in.C, kProtoRows);
        int64_t splits, tps;
        plan_splits(bx, ceil_div(in.B, 32), splits, tps);
        if (splits > 1) {
            proto_fill_kernel<float><<<(unsigned)grid1d(in.C * D, 256), 256, 0, st>>>(dP, in.C * D, 0.f);
            SQ_LAUNCHED("proto_fill_kernel");
        }
        ProfScope prof("proto_bwd_protos_kernel", st);
        proto_bwd_protos_kernel<D><<<dim3((unsigned)bx, (unsigned)splits), kProtoThreads, 0, st>>>(
            in, P, inv, lse, omp, grad_loss, tps, splits > 1, dP);
    }
    SQ_LAUNCHED("proto_bwd_protos_kernel");
    if (in.n > 0) {
        ProfScope prof("proto_route_kernel", st);
        proto_route_kernel<D><<<(unsigned)grid1d(in.n * (D / 4), 256), 256, 0, st>>>(in.labels, in.n, in.C, dP, inv, demb);
    }
    SQ_LAUNCHED("proto_route_kernel");
    return SUBQUAD_OK;
}

}  // namespace subquad

using namespace subquad;

extern "C" size_t subquad_proto_workspace_bytes(int64_t n, int32_t d, int64_t C, int64_t B) {
    if (n < 0 || d <= 0 || C < 1 || B < 0) return 0;
    return proto_layout(n, d, C, B).total;
}

extern "C" int subquad_proto_fwd(const float *emb, int64_t n, int32_t d, const int32_t *labels, int64_t C,
                                 const int32_t *batch, int64_t B, float tau, double *loss, float *row_loss,
                                 float *protos, void *ws, size_t ws_bytes, void *stream) {
    clear_error();
    ProtoLayout L;
    int rc = proto_validate(emb, n, d, labels, C, batch, B, tau, ws, ws_bytes, L);
    if (rc != SUBQUAD_OK) return rc;
    SQ_REQUIRE(loss, SUBQUAD_ERR_ARG, "null loss pointer");
    const ProtoIn in{emb, n, labels, C, batch, B, 1.f / tau};
    char *w = static_cast<char *>(ws);
    hipStream_t st = as_stream(stream);
    if (d == 32) return proto_fwd_d<32>(in, w, L, loss, row_loss, protos, st);
    if (d == 64) return proto_fwd_d<64>(in, w, L, loss, row_loss, protos, st);
    return proto_fwd_d<128>(in, w, L, loss, row_loss, protos, st);
}

extern "C" int subquad_proto_bwd(const float *emb, int64_t n, int32_t d, const int32_t *labels, int64_t C,
                                 const int32_t *batch, int64_t B, float tau, const float *grad_loss,
                                 int32_t through_prototypes, float *demb, void *ws, size_t ws_bytes, void *stream) {
    clear_error();
    ProtoLayout L;
    int rc = proto_validate(emb, n, d, labels, C, batch, B, tau, ws, ws_bytes, L);
    if (rc != SUBQUAD_OK) return rc;
    SQ_REQUIRE(demb || n == 0, SUBQUAD_ERR_ARG, "null demb pointer");
    SQ_REQUIRE(((uintptr_t)demb & 15) == 0, SUBQUAD_ERR_ARG, "demb must be 16-byte aligned");
    const ProtoIn in{emb, n, labels, C, batch, B, 1.f / tau};
    char *w = static_cast<char *>(ws);
    hipStream_t st = as_stream(stream);
    if (d == 32) return proto_bwd_d<32>(in, w, L, grad_loss, through_prototypes != 0, demb, st);
    if (d == 64) return proto_bwd_d<64>(in, w, L, grad_loss, through_prototypes != 0, demb, st);
    return proto_bwd_d<128>(in, w, L, grad_loss, through_prototypes != 0, demb, st);
}
