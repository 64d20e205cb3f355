// Helpers shared by the gate kernels: 16-lane pair groups, float4 row gathers, reductions.
#pragma once

#include "common.h"

namespace subquad {

constexpr int kGateThreads = 256;
constexpr int kGroup = 16;
// Pairs whose index and row loads a lane group issues together before computing any of
// them: more gathers in flight per group.
constexpr int kGateBatch = 4;

// Hardware reciprocal, square root, reciprocal square root and 2^x (about 1 ulp each; the
// gate's tolerance against the float64 reference is 1e-5 relative).  Every gate kernel uses
// the same ones, so the forward and the backward take the same ReLU decisions.
__device__ __forceinline__ float rcp_fast(float x) { return __builtin_amdgcn_rcpf(x); }
__device__ __forceinline__ float sqrt_fast(float x) { return __builtin_amdgcn_sqrtf(x); }
__device__ __forceinline__ float rsqrt_fast(float x) { return __builtin_amdgcn_rsqf(x); }
__device__ __forceinline__ float exp2_fast(float x) { return __builtin_amdgcn_exp2f(x); }

// v moved across the lanes of each 16-lane row by the DPP control `ctrl`.
template <int ctrl>
__device__ __forceinline__ float dpp_f32(float v) {
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), ctrl, 0xF, 0xF, false));
}

// Sum over the 16 lanes of a group (a DPP row), in every lane, with no LDS traffic: swap
// within pairs (quad_perm 1,0,3,2), within quads (quad_perm 2,3,0,1), across the quads of
// each half row (row_half_mirror), across the half rows (row_mirror).  Each step adds two
// equal partial sums in either order, so all 16 lanes end with the same bits.
__device__ __forceinline__ float group_sum(float v) {
    static_assert(kGroup == 16, "group_sum works on DPP rows of 16 lanes");
    v += dpp_f32<0xB1>(v);
    v += dpp_f32<0x4E>(v);
    v += dpp_f32<0x141>(v);
    v += dpp_f32<0x140>(v);
    return v;
}

// Pairs per chunk of a lane group: P split evenly over the groups, but at most
// kGateChunkMax; a group then takes chunks g, g + ngroups, ... so that at any time all
// groups work inside one window of ngroups x chunk consecutive pairs, whose partner rows
// (one repertoire's, or a few) stay in the caches while it is walked.
constexpr int64_t kGateChunkMax = 4096;
__host__ __device__ inline int64_t gate_chunk(int64_t P, int64_t ngroups) {
    const int64_t c = (P + ngroups - 1) / ngroups;
    return c < 1 ? 1 : (c < kGateChunkMax ? c : kGateChunkMax);
}

// Pairs to process: `cap`, or the count a producer left in device memory (clamped to
// [0, cap]) when `count_dev` is set, so that a launch sized for the capacity needs no host
// synchronisation.
__device__ __forceinline__ int64_t live_count(int64_t cap, const int64_t *__restrict__ count_dev) {
    if (!count_dev) return cap;
    const int64_t c = *count_dev;
    return c < 0 ? 0 : (c < cap ? c : cap);
}

template <int NV>
__device__ __forceinline__ void load_row(const float *__restrict__ emb, int64_t row, int d4, int l, float4 (&v)[NV]) {
    const float4 *r = reinterpret_cast<const float4 *>(emb) + row * d4;
#pragma unroll
    for (int k = 0; k < NV; ++k) {
        int c = l + kGroup * k;
        v[k] = c < d4 ? r[c] : make_float4(0.f, 0.f, 0.f, 0.f);
    }
}

// load_row with no branch around the loads: slots past the row are clamped into it and
// zeroed after the load, so that a batch's row loads can all be in flight together.
template <int NV>
__device__ __forceinline__ void load_row_flat(const float *__restrict__ emb, int64_t row, int d4, int l,
                                              float4 (&v)[NV]) {
    const float4 *r = reinterpret_cast<const float4 *>(emb) + row * d4;
#pragma unroll
    for (int k = 0; k < NV; ++k) {
        const int c = l + kGroup * k;
        const float4 x = r[min(c, d4 - 1)];
        // a bit mask rather than a select, so the compiler cannot move the load under a branch
        const int m = c < d4 ? -1 : 0;
        v[k] = make_float4(__int_as_float(__float_as_int(x.x) & m), __int_as_float(__float_as_int(x.y) & m),
                           __int_as_float(__float_as_int(x.z) & m), __int_as_float(__float_as_int(x.w) & m));
    }
}

// One fixed fma chain (with contraction left to the compiler, two kernels could round the
// same dot product differently).
__device__ __forceinline__ float dot4(float4 a, float4 b) {
    return fmaf(a.w, b.w, fmaf(a.z, b.z, fmaf(a.y, b.y, a.x * b.x)));
}

// Adds a row's accumulated gradient slice into demb.  A row whose pairs all lie inside one
// group's chunk is owned by that group (plain read-modify-write); a row split across
// chunks is added atomically.
template <int NV>
__device__ __forceinline__ void flush_row(float *__restrict__ demb, int64_t row, int d4, int l, float4 (&acc)[NV],
                                          bool owned) {
    float4 *base = reinterpret_cast<float4 *>(demb) + row * d4;
#pragma unroll
    for (int k = 0; k < NV; ++k) {
        const int c = l + kGroup * k;
        if (c < d4) {
            if (owned) {
                float4 v = base[c];
                v.x += acc[k].x;
                v.y += acc[k].y;
                v.z += acc[k].z;
                v.w += acc[k].w;
                base[c] = v;
            } else {
                float *f = reinterpret_cast<float *>(base + c);
                atomicAdd(f + 0, acc[k].x);
                atomicAdd(f + 1, acc[k].y);
                atomicAdd(f + 2, acc[k].z);
                atomicAdd(f + 3, acc[k].w);
            }
        }
        acc[k] = make_float4(0.f, 0.f, 0.f, 0.f);
    }
}

// Loads a row's current gradient slice (issued when the row starts, used when it is flushed).
template <int NV>
__device__ __forceinline__ void load_grad_row(const float *__restrict__ demb, int64_t row, int d4, int l,
                                              float4 (&old)[NV]) {
    load_row<NV>(demb, row, d4, l, old);
}

// flush_row with the row's old value already in registers: an owned row is stored as
// old + acc (no load on the flush path), a split row is added atomically.
template <int NV>
__device__ __forceinline__ void flush_row_pre(float *__restrict__ demb, int64_t row, int d4, int l, float4 (&acc)[NV],
                                              const float4 (&old)[NV], bool owned) {
    float4 *base = reinterpret_cast<float4 *>(demb) + row * d4;
#pragma unroll
    for (int k = 0; k < NV; ++k) {
        const int c = l + kGroup * k;
        if (c < d4) {
            if (owned) {
                base[c] = make_float4(old[k].x + acc[k].x, old[k].y + acc[k].y, old[k].z + acc[k].z, old[k].w + acc[k].w);
            } else {
                float *f = reinterpret_cast<float *>(base + c);
                atomicAdd(f + 0, acc[k].x);
                atomicAdd(f + 1, acc[k].y);
                atomicAdd(f + 2, acc[k].z);
                atomicAdd(f + 3, acc[k].w);
            }
        }
        acc[k] = make_float4(0.f, 0.f, 0.f, 0.f);
    }
}

// Second pass of the cosine gradient: pairs in order of their second index j; each row u
// gathers its partners e_i and adds sum_p cbar_p (e_i inv_p - c_p e_u / |e_u|^2) to demb[u].
// pack[p] = (cbar_p, c_p, inv_p = 1 / (|e_i| |e_j|), 0), written by the first pass.
// One chunk [q0, q1) of gate_cos_bwd_j_kernel's walk.
template <int NV>
__device__ __forceinline__ void cos_bwd_j_chunk(const float *__restrict__ emb, int64_t n, int32_t d,
                                                const int32_t *__restrict__ pairs, int64_t P,
                                                const uint64_t *__restrict__ order_j, const float4 *__restrict__ pack,
                                                float *__restrict__ demb, int64_t q0, int64_t q1, int l) {
    if (q0 >= q1) return;
    const int d4 = d >> 2;
    float4 eu[NV], acc[NV], old[NV];
#pragma unroll
    for (int k = 0; k < NV; ++k) acc[k] = make_float4(0.f, 0.f, 0.f, 0.f);
    float inv_nu2 = 0.f;
    int64_t cur = -1;
    bool started_here = false;
    // the row's gradient is sum_p a_p e_i(p) - B e_u (a_p = cbar_p inv_p, B = sum_p cbar_p c_p
    // / |e_u|^2): acc holds the sum, bsum the scalar B, and the e_u term is applied at the flush
    float bsum = 0.f;
    auto flush = [&](bool owned) {
#pragma unroll
        for (int k = 0; k < NV; ++k) {
            acc[k].x = fmaf(-bsum, eu[k].x, acc[k].x);
            acc[k].y = fmaf(-bsum, eu[k].y, acc[k].y);
            acc[k].z = fmaf(-bsum, eu[k].z, acc[k].z);
            acc[k].w = fmaf(-bsum, eu[k].w, acc[k].w);
        }
        bsum = 0.f;
        flush_row_pre<NV>(demb, cur, d4, l, acc, old, owned);
    };
    // the next batch's order records are fetched while the current one is computed
    uint64_t nrec[kGateBatch];
#pragma unroll
    for (int t = 0; t < kGateBatch; ++t) nrec[t] = q0 + t < q1 ? order_j[q0 + t] : ~0ull;
    for (int64_t qb = q0; qb < q1; qb += kGateBatch) {
        int64_t ub[kGateBatch], ib[kGateBatch];
        float4 pk[kGateBatch];
        uint64_t recs[kGateBatch];
#pragma unroll
        for (int t = 0; t < kGateBatch; ++t) recs[t] = nrec[t];
#pragma unroll
        for (int t = 0; t < kGateBatch; ++t) {
            // loads with no branch around them (a dead entry reads pair 0; its values are
            // masked out), so that the batch's loads are in flight together
            const uint64_t rec = recs[t];
            ub[t] = qb + t < q1 ? (int64_t)(rec >> 32) : -1;
            const int64_t pr = (int64_t)(uint32_t)rec;
            const bool live = ub[t] >= 0 && ub[t] < n && pr < P;
            const int64_t p = live ? pr : 0;
            const float4 pv = pack[p];
            const int32_t iv = pairs[2 * p];
            const int m = live ? -1 : 0;
            pk[t] = make_float4(__int_as_float(__float_as_int(pv.x) & m), __int_as_float(__float_as_int(pv.y) & m),
                                __int_as_float(__float_as_int(pv.z) & m), __int_as_float(__float_as_int(pv.w) & m));
            ib[t] = live ? iv : -1;
        }
        float4 ep[kGateBatch][NV];
#pragma unroll
        for (int t = 0; t < kGateBatch; ++t) {
            const bool use = pk[t].x != 0.f && ib[t] >= 0 && ib[t] < n;
            if (!use) ib[t] = -1;
            if (use) load_row<NV>(emb, ib[t], d4, l, ep[t]);
        }
#pragma unroll
        for (int t = 0; t < kGateBatch; ++t) {
            const int64_t qn = qb + kGateBatch + t;
            nrec[t] = qn < q1 ? order_j[qn] : ~0ull;
        }
#pragma unroll
        for (int t = 0; t < kGateBatch; ++t) {
            if (ub[t] < 0) break;
            const int64_t u = ub[t];
            if (u != cur) {
                if (cur >= 0 && cur < n) flush(started_here);
                cur = u;
                // The row starts inside this chunk unless the record before the chunk is in it too.
                started_here = q0 == 0 || (int64_t)(order_j[q0 - 1] >> 32) != u;
                if (u < n) {
                    load_grad_row<NV>(demb, u, d4, l, old);
                    load_row<NV>(emb, u, d4, l, eu);
                    float a = 0.f;
#pragma unroll
                    for (int k = 0; k < NV; ++k) a += dot4(eu[k], eu[k]);
                    a = group_sum(a);
                    inv_nu2 = a > 0.f ? 1.f / a : 0.f;
                }
            }
            if (ib[t] < 0) continue;
            const float a = pk[t].x * pk[t].z;
            bsum = fmaf(pk[t].x * pk[t].y, inv_nu2, bsum);
#pragma unroll
            for (int k = 0; k < NV; ++k) {
                acc[k].x = fmaf(a, ep[t][k].x, acc[k].x);
                acc[k].y = fmaf(a, ep[t][k].y, acc[k].y);
                acc[k].z = fmaf(a, ep[t][k].z, acc[k].z);
                acc[k].w = fmaf(a, ep[t][k].w, acc[k].w);
            }
        }
    }
    if (cur >= 0 && cur < n) {
        const bool ends_here = q1 == P || (int64_t)(order_j[q1] >> 32) != cur;
        flush(started_here && ends_here);
    }
}

// LOOP: a lane group walks several capped chunks (a capacity above ngroups x
// kGateChunkMax pairs); otherwise its one chunk (fewer registers live).
template <int NV, bool LOOP>
__global__ __launch_bounds__(kGateThreads) void gate_cos_bwd_j_kernel(const float *__restrict__ emb, int64_t n,
                                                                      int32_t d, const int32_t *__restrict__ pairs,
                                                                      int64_t cap, const int64_t *__restrict__ P_dev,
                                                                      const uint64_t *__restrict__ order_j,
                                                                      const float4 *__restrict__ pack,
                                                                      float *__restrict__ demb) {
    const int64_t P = live_count(cap, P_dev);
    const int l = threadIdx.x & (kGroup - 1);
    const int64_t group = ((int64_t)blockIdx.x * kGateThreads + threadIdx.x) / kGroup;
    const int64_t ngroups = (int64_t)gridDim.x * (kGateThreads / kGroup);
    const int64_t chunk = gate_chunk(P, ngroups);
    if (LOOP) {
        for (int64_t c0 = group * chunk; c0 < P; c0 += ngroups * chunk)
            cos_bwd_j_chunk<NV>(emb, n, d, pairs, P, order_j, pack, demb, c0, min(P, c0 + chunk), l);
    } else {
        const int64_t c0 = group * chunk;
        cos_bwd_j_chunk<NV>(emb, n, d, pairs, P, order_j, pack, demb, c0, min(P, c0 + chunk), l);
    }
}

// Records (key << 32 | p) for the pair-order sorts: key = pairs[p][side], or n for a pair
// with either index out of range (such pairs sort last on both sides; the same key as the
// in-order check of the pairs gives them, so that a natural order passed by that check is
// in order of these keys too).
static __global__ void gate_order_keys_kernel(const int32_t *__restrict__ pairs, int64_t cap,
                                              const int64_t *__restrict__ P_dev, int64_t n, int side,
                                              uint64_t *__restrict__ rec) {
    const int64_t P = live_count(cap, P_dev);
    for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < P; p += (int64_t)gridDim.x * blockDim.x) {
        const int32_t i = pairs[2 * p], j = pairs[2 * p + 1];
        const bool ok = i >= 0 && i < n && j >= 0 && j < n;
        const uint64_t key = ok ? (uint64_t)(side ? j : i) : (uint64_t)n;
        rec[p] = (key << 32) | (uint64_t)p;
    }
}

inline int key_bits_for(int64_t n) {  // bits holding 0..n
    int b = 1;
    while ((int64_t(1) << b) <= n) ++b;
    return b;
}

// Groups of 16 lanes, each owning a contiguous chunk of pairs.
inline int64_t gate_blocks_for(int64_t P, int groups_per_cu) {
    int64_t groups = std::max<int64_t>(1, std::min<int64_t>(ceil_div(P, 4), (int64_t)device_cus() * groups_per_cu));
    return ceil_div(groups, kGateThreads / kGroup);
}

// As gate_blocks_for, but never more blocks than the chip holds at once for `kernel`: a
// chunked kernel then runs in one round instead of leaving a tail of late groups.
inline int64_t gate_blocks_resident(int64_t P, int groups_per_cu, const void *kernel) {
    return std::min<int64_t>(gate_blocks_for(P, groups_per_cu), (int64_t)device_cus() * resident_blocks_per_cu(kernel));
}

}  // namespace subquad
