// Helpers shared by the gate kernels: 16-lane pair groups, float4 row gathers, reductions.
#pragma once

#include "common.h"

namespace subquad {

constexpr int kGateThreads = 256;
constexpr int kGroup = 16;

__device__ __forceinline__ float group_sum(float v) {
#pragma unroll
    for (int off = kGroup / 2; off >= 1; off >>= 1) v += __shfl_xor(v, off, kGroup);
    return v;
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

__device__ __forceinline__ float dot4(float4 a, float4 b) { return a.x * b.x + a.y * b.y + a.z * b.z + a.w * b.w; }

// Groups of 16 lanes, each owning a contiguous chunk of pairs.
inline int64_t gate_blocks_for(int64_t P, int groups_per_cu) {
    int64_t groups = std::max<int64_t>(1, std::min<int64_t>(ceil_div(P, 4), (int64_t)device_cus() * groups_per_cu));
    return ceil_div(groups, kGateThreads / kGroup);
}

}  // namespace subquad
