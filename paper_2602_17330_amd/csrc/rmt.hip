// Random-matrix-theory edge threshold of the similarity graph (Sec. 3.7, Algorithm 1: the
// eigenvalue spectrum of the fused-affinity matrix A gives a bulk cutoff, and edges below the
// threshold it implies are dropped).
//
//   lambda_plus = 2 sqrt(sum_ij a_ij^2 / n)   (Wigner semicircle edge at A's mean squared row norm)
//   tau* = the largest tau with lambda_max(A_low(tau)) <= lambda_plus, A_low(tau) = {0 < a_ij < tau},
//          by bisection on [0, max a_ij] with float64 midpoints (lambda_max(A_low) grows with tau
//          since A >= 0); tau* = max a_ij + 1 when lambda_max(A) <= lambda_plus.
//
// lambda_max of each masked matrix comes from K steps of Lanczos on the device: a masked CSR
// product (16 lanes per row), float32 Lanczos vectors, float64 dot products, full
// reorthogonalisation by two rounds of classical Gram-Schmidt (which also give alpha_k and
// beta_k), and the largest eigenvalue of the tridiagonal T_K by Sturm-count bisection.
#include <algorithm>
#include <cmath>
#include <vector>

#include "gate_util.h"

namespace subquad {

constexpr int kRmtThreads = 256;
constexpr int kRmtMaxSteps = 128;
constexpr int kRmtChunk = kRmtThreads * 16;  // vector entries per block of a dot product

struct RmtScalars {  // device-resident Lanczos state
    double alpha[kRmtMaxSteps + 1];
    double beta[kRmtMaxSteps + 2];  // beta[k] couples V_{k-1} and V_k; beta[0] = 0
    double lambda;                  // largest Ritz value of the last run
    double sumsq, wmax;             // of the CSR values (bulk edge)
    int32_t steps;                  // Lanczos steps actually taken (breakdown stops early)
    int32_t pad;
};

// y = A_tau x: entries with 0 < v < tau (compared in float64).  16 lanes per row (four per
// row measured slower: rows of the similarity graph vary widely in length).
__global__ __launch_bounds__(kRmtThreads) void rmt_spmv_kernel(const int64_t *__restrict__ ro,
                                                               const int32_t *__restrict__ cols,
                                                               const float *__restrict__ vals, int64_t n, double tau,
                                                               const float *__restrict__ x, float *__restrict__ y,
                                                               const RmtScalars *__restrict__ sc, int k) {
    if (sc->steps <= k) return;  // the run stopped at an invariant subspace
    const int l = threadIdx.x & (kGroup - 1);
    const int64_t g0 = ((int64_t)blockIdx.x * kRmtThreads + threadIdx.x) / kGroup;
    const int64_t gs = (int64_t)gridDim.x * (kRmtThreads / kGroup);
    for (int64_t r = g0; r < n; r += gs) {
        float acc = 0.f;
        for (int64_t e = ro[r] + l; e < ro[r + 1]; e += kGroup) {
            const float v = vals[e];
            if (v > 0.f && (double)v < tau) acc += v * x[cols[e]];
        }
        acc = group_sum(acc);
        if (l == 0) y[r] = acc;
    }
}

// partial[j * nchunks + c] = sum over chunk c of V_j . w  (j = 0..k), blockIdx.y = j.
__global__ __launch_bounds__(kRmtThreads) void rmt_mdot_kernel(const float *__restrict__ V, const float *__restrict__ w,
                                                               int64_t n, int64_t nchunks, double *__restrict__ partial,
                                                               const RmtScalars *__restrict__ sc, int k) {
    if (sc->steps <= k) return;
    const int j = blockIdx.y;
    const float *v = V + (int64_t)j * n;
    double acc = 0.0;
    for (int64_t c = blockIdx.x; c < nchunks; c += gridDim.x) {
        const int64_t base = c * kRmtChunk;
        // the chunk's loads all issue before the products (indices past n are clamped and
        // their terms skipped; the sum runs in the same order as a plain loop)
        float vv[kRmtChunk / kRmtThreads], ww[kRmtChunk / kRmtThreads];
#pragma unroll
        for (int u = 0; u < kRmtChunk / kRmtThreads; ++u) {
            const int64_t i = min(base + u * kRmtThreads + threadIdx.x, n - 1);
            vv[u] = v[i];
            ww[u] = w[i];
        }
        double part = 0.0;
#pragma unroll
        for (int u = 0; u < kRmtChunk / kRmtThreads; ++u)
            if (base + u * kRmtThreads + threadIdx.x < n) part += (double)vv[u] * (double)ww[u];
        acc += part;
    }
    __shared__ double red[kRmtThreads];
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int o = kRmtThreads / 2; o > 0; o >>= 1) {
        if (threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0) partial[(int64_t)j * gridDim.x + blockIdx.x] = red[0];
}

// h[j] = sum of the partials of j; in the first round alpha_k = h[k] (the projection of
// A V_k on V_k), in the second its correction is added.
__global__ void rmt_mdot_reduce_kernel(const double *__restrict__ partial, int nparts, double *__restrict__ h,
                                       RmtScalars *__restrict__ sc, int k, int round) {
    if (sc->steps <= k) return;
    const int j = blockIdx.x;
    __shared__ double red[kRmtThreads];
    double a = 0.0;
    for (int t = threadIdx.x; t < nparts; t += kRmtThreads) a += partial[(int64_t)j * nparts + t];
    red[threadIdx.x] = a;
    __syncthreads();
    for (int o = kRmtThreads / 2; o > 0; o >>= 1) {
        if (threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        h[j] = red[0];
        if (j == k) sc->alpha[k] = round == 0 ? red[0] : sc->alpha[k] + red[0];
    }
}

// w -= sum_j h[j] V_j (j = 0..k); block partial sums of w^2 for the norm.
__global__ __launch_bounds__(kRmtThreads) void rmt_msub_kernel(const float *__restrict__ V, float *__restrict__ w,
                                                               int64_t n, const double *__restrict__ h,
                                                               double *__restrict__ partial,
                                                               const RmtScalars *__restrict__ sc, int k) {
    if (sc->steps <= k) return;
    double acc = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * kRmtThreads + threadIdx.x; i < n; i += (int64_t)gridDim.x * kRmtThreads) {
        double s = (double)w[i];
        // eight basis entries in flight at a time (same subtraction order as one by one)
        int j = 0;
        for (; j + 8 <= k + 1; j += 8) {
            float vv[8];
#pragma unroll
            for (int u = 0; u < 8; ++u) vv[u] = V[(int64_t)(j + u) * n + i];
#pragma unroll
            for (int u = 0; u < 8; ++u) s -= h[j + u] * (double)vv[u];
        }
        for (; j <= k; ++j) s -= h[j] * (double)V[(int64_t)j * n + i];
        const float f = (float)s;
        w[i] = f;
        acc += (double)f * (double)f;
    }
    __shared__ double red[kRmtThreads];
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int o = kRmtThreads / 2; o > 0; o >>= 1) {
        if (threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0) partial[blockIdx.x] = red[0];
}

// beta_{k+1} = |w|; a breakdown (|w| <= 1e-10 |A V_k| scale) ends the run after step k.
__global__ void rmt_norm_kernel(const double *__restrict__ partial, int nparts, RmtScalars *__restrict__ sc, int k,
                                int K) {
    if (sc->steps <= k) return;
    __shared__ double red[kRmtThreads];
    double a = 0.0;
    for (int t = threadIdx.x; t < nparts; t += kRmtThreads) a += partial[t];
    red[threadIdx.x] = a;
    __syncthreads();
    for (int o = kRmtThreads / 2; o > 0; o >>= 1) {
        if (threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        const double b = sqrt(red[0]);
        sc->beta[k + 1] = b;
        const double scale = fabs(sc->alpha[k]) + sc->beta[k] + 1e-300;
        if (k + 1 >= K || b <= 1e-10 * scale) sc->steps = k + 1;
    }
}

// V_{k+1} = w / beta_{k+1}
__global__ __launch_bounds__(kRmtThreads) void rmt_scale_kernel(const float *__restrict__ w, float *__restrict__ vnext,
                                                                int64_t n, const RmtScalars *__restrict__ sc, int k) {
    if (sc->steps <= k + 1) return;
    const double inv = 1.0 / sc->beta[k + 1];
    for (int64_t i = (int64_t)blockIdx.x * kRmtThreads + threadIdx.x; i < n; i += (int64_t)gridDim.x * kRmtThreads)
        vnext[i] = (float)((double)w[i] * inv);
}

// Start vector: entries uniform in [-1, 1) from SplitMix64 outputs keyed by (seed, i), then
// normalised (the norm by the same two-stage sum).
__device__ __forceinline__ uint64_t mix64_at(uint64_t seed, uint64_t q) {
    uint64_t z = seed + (q + 1) * 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

__global__ __launch_bounds__(kRmtThreads) void rmt_start_kernel(float *__restrict__ w, int64_t n, uint64_t seed,
                                                                double *__restrict__ partial) {
    double acc = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * kRmtThreads + threadIdx.x; i < n; i += (int64_t)gridDim.x * kRmtThreads) {
        const float f = (float)((double)(mix64_at(seed, (uint64_t)i) >> 11) * 0x1.0p-52 - 1.0);
        w[i] = f;
        acc += (double)f * (double)f;
    }
    __shared__ double red[kRmtThreads];
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int o = kRmtThreads / 2; o > 0; o >>= 1) {
        if (threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0) partial[blockIdx.x] = red[0];
}

__global__ void rmt_start_norm_kernel(const double *__restrict__ partial, int nparts, RmtScalars *__restrict__ sc,
                                      int K) {
    __shared__ double red[kRmtThreads];
    double a = 0.0;
    for (int t = threadIdx.x; t < nparts; t += kRmtThreads) a += partial[t];
    red[threadIdx.x] = a;
    __syncthreads();
    for (int o = kRmtThreads / 2; o > 0; o >>= 1) {
        if (threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        sc->beta[0] = sqrt(red[0]);  // the start vector's norm, used once to normalise it
        sc->steps = K;
        sc->lambda = 0.0;
    }
}

__global__ __launch_bounds__(kRmtThreads) void rmt_start_scale_kernel(const float *__restrict__ w, float *__restrict__ v0,
                                                                      int64_t n, RmtScalars *__restrict__ sc) {
    const double inv = sc->beta[0] > 0.0 ? 1.0 / sc->beta[0] : 0.0;
    for (int64_t i = (int64_t)blockIdx.x * kRmtThreads + threadIdx.x; i < n; i += (int64_t)gridDim.x * kRmtThreads)
        v0[i] = (float)((double)w[i] * inv);
}

// beta[0] held the start vector's norm; it is not a coupling of T (reset after every block
// of the scaling kernel has read it).
__global__ void rmt_start_done_kernel(RmtScalars *__restrict__ sc) {
    if (threadIdx.x == 0 && blockIdx.x == 0) sc->beta[0] = 0.0;
}

// Largest eigenvalue of T_m (diagonal alpha[0..m), off-diagonal beta[1..m)): multisection
// on the Sturm count (the number of eigenvalues below x, from the LDL^T pivots) by the 64
// lanes of one wave, each testing one of 64 interior points, from the Gershgorin interval
// down to a width of 1e-15 relative; returns the interval's upper end (every lane the same).
__device__ double ritz_max(const RmtScalars *__restrict__ sc, int m) {
    const int t = threadIdx.x & 63;
    double lo = 0.0, hi = 0.0;
    for (int i = 0; i < m; ++i) {
        const double r = (i > 0 ? fabs(sc->beta[i]) : 0.0) + (i + 1 < m ? fabs(sc->beta[i + 1]) : 0.0);
        lo = i == 0 ? sc->alpha[i] - r : fmin(lo, sc->alpha[i] - r);
        hi = i == 0 ? sc->alpha[i] + r : fmax(hi, sc->alpha[i] + r);
    }
    for (int it = 0; it < 64 && hi - lo > 1e-15 * fmax(fabs(lo), fabs(hi)); ++it) {
        const double x = lo + (hi - lo) * (double)(t + 1) / 65.0;
        int below = 0;
        double q = 1.0;
        for (int i = 0; i < m; ++i) {
            const double b2 = i > 0 ? sc->beta[i] * sc->beta[i] : 0.0;
            q = sc->alpha[i] - x - (i > 0 ? b2 / q : 0.0);
            if (q == 0.0) q = -1e-300;
            below += q < 0.0;
        }
        // the first point above every eigenvalue bounds the largest one from above; the
        // point before it (or lo) bounds it from below
        const uint64_t above = __ballot(below == m);
        const int f = above ? __builtin_ctzll(above) : 64;
        const double nlo = lo + (hi - lo) * (double)f / 65.0;
        const double nhi = f == 64 ? hi : lo + (hi - lo) * (double)(f + 1) / 65.0;
        lo = nlo;
        hi = nhi;
    }
    return hi;
}

// lambda = largest eigenvalue of T over the steps taken (one wave).
__global__ __launch_bounds__(64) void rmt_tridiag_kernel(RmtScalars *__restrict__ sc) {
    const double lam = ritz_max(sc, sc->steps);
    if (threadIdx.x == 0) sc->lambda = lam;
}

// After step k: when the largest Ritz value of T_{k+1} already exceeds `target`, the run
// stops there (later steps return at once).  Ritz values of Lanczos only grow with the
// step count, so the run's answer to "is lambda_max above target?" is the one all steps
// would give.  One wave.
__global__ __launch_bounds__(64) void rmt_check_kernel(RmtScalars *__restrict__ sc, int k, double target) {
    if (sc->steps <= k) return;
    const double theta = ritz_max(sc, k + 1);
    if (threadIdx.x == 0 && theta > target) sc->steps = k + 1;
}

// sumsq and max of the values (two-stage: block partials, then one block).
__global__ __launch_bounds__(kRmtThreads) void rmt_stats_kernel(const float *__restrict__ vals, int64_t nnz,
                                                                double *__restrict__ partial) {
    double s = 0.0, m = 0.0;
    for (int64_t e = (int64_t)blockIdx.x * kRmtThreads + threadIdx.x; e < nnz; e += (int64_t)gridDim.x * kRmtThreads) {
        const float v = vals[e];
        if (v > 0.f) {
            s += (double)v * (double)v;
            m = fmax(m, (double)v);
        }
    }
    __shared__ double rs[kRmtThreads], rm[kRmtThreads];
    rs[threadIdx.x] = s;
    rm[threadIdx.x] = m;
    __syncthreads();
    for (int o = kRmtThreads / 2; o > 0; o >>= 1) {
        if (threadIdx.x < o) {
            rs[threadIdx.x] += rs[threadIdx.x + o];
            rm[threadIdx.x] = fmax(rm[threadIdx.x], rm[threadIdx.x + o]);
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        partial[2 * blockIdx.x] = rs[0];
        partial[2 * blockIdx.x + 1] = rm[0];
    }
}

__global__ void rmt_stats_reduce_kernel(const double *__restrict__ partial, int nparts, RmtScalars *__restrict__ sc) {
    __shared__ double rs[kRmtThreads], rm[kRmtThreads];
    double s = 0.0, m = 0.0;
    for (int t = threadIdx.x; t < nparts; t += kRmtThreads) {
        s += partial[2 * t];
        m = fmax(m, partial[2 * t + 1]);
    }
    rs[threadIdx.x] = s;
    rm[threadIdx.x] = m;
    __syncthreads();
    for (int o = kRmtThreads / 2; o > 0; o >>= 1) {
        if (threadIdx.x < o) {
            rs[threadIdx.x] += rs[threadIdx.x + o];
            rm[threadIdx.x] = fmax(rm[threadIdx.x], rm[threadIdx.x + o]);
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        sc->sumsq = rs[0];
        sc->wmax = rm[0];
    }
}

struct RmtLayout {
    size_t V, w, h, partial, sc, total;
};

static int64_t rmt_blocks(int64_t work) {
    return std::max<int64_t>(1, std::min<int64_t>(ceil_div(work, kRmtThreads), (int64_t)device_cus() * 4));
}

static RmtLayout rmt_layout(int64_t n, int32_t K) {
    RmtLayout L{};
    size_t off = 0;
    auto take = [&](size_t bytes) { size_t o = off; off += align_up(std::max<size_t>(bytes, 1), 256); return o; };
    const int64_t n1 = std::max<int64_t>(n, 1);
    const int64_t nchunks = ceil_div(n1, (int64_t)kRmtChunk);
    const int64_t parts = std::max<int64_t>(std::min<int64_t>(nchunks, (int64_t)device_cus() * 4) * (K + 1),
                                            2 * rmt_blocks(std::max<int64_t>(n1, 1)));
    L.V = take(sizeof(float) * (size_t)(K + 1) * n1);
    L.w = take(sizeof(float) * n1);
    L.h = take(sizeof(double) * (K + 1));
    L.partial = take(sizeof(double) * (size_t)std::max<int64_t>(parts, 2 * (int64_t)device_cus() * 4 * 2));
    L.sc = take(sizeof(RmtScalars));
    L.total = off;
    return L;
}

// lambda_max(A_tau) by K Lanczos steps; leaves it in sc->lambda (device).
constexpr int kRmtCheckEvery = 8;  // steps between early-stop checks

// stop_above: finite for a threshold decision (stop once a Ritz value exceeds it), INFINITY
// for the eigenvalue itself.
static int rmt_lanczos(const int64_t *ro, const int32_t *cols, const float *vals, int64_t n, double tau, int K,
                       uint64_t seed, char *ws, const RmtLayout &L, hipStream_t st,
                       double stop_above = INFINITY) {
    float *V = reinterpret_cast<float *>(ws + L.V);
    float *w = reinterpret_cast<float *>(ws + L.w);
    double *h = reinterpret_cast<double *>(ws + L.h);
    double *partial = reinterpret_cast<double *>(ws + L.partial);
    RmtScalars *sc = reinterpret_cast<RmtScalars *>(ws + L.sc);
    const int64_t vb = rmt_blocks(n);
    const int64_t nchunks = ceil_div(n, (int64_t)kRmtChunk);
    const int64_t cb = std::min<int64_t>(nchunks, (int64_t)device_cus() * 4);
    const int64_t spmv_blocks = std::max<int64_t>(1, std::min<int64_t>(ceil_div(n, kRmtThreads / kGroup),
                                                                       (int64_t)device_cus() * 16));
    rmt_start_kernel<<<(unsigned)vb, kRmtThreads, 0, st>>>(w, n, seed, partial);
    SQ_LAUNCHED("rmt_start_kernel");
    rmt_start_norm_kernel<<<1, kRmtThreads, 0, st>>>(partial, (int)vb, sc, K);
    SQ_LAUNCHED("rmt_start_norm_kernel");
    rmt_start_scale_kernel<<<(unsigned)vb, kRmtThreads, 0, st>>>(w, V, n, sc);
    SQ_LAUNCHED("rmt_start_scale_kernel");
    rmt_start_done_kernel<<<1, 64, 0, st>>>(sc);
    SQ_LAUNCHED("rmt_start_done_kernel");
    for (int k = 0; k < K; ++k) {
        {
            ProfScope prof("rmt_spmv_kernel", st);
            rmt_spmv_kernel<<<(unsigned)spmv_blocks, kRmtThreads, 0, st>>>(ro, cols, vals, n, tau, V + (int64_t)k * n,
                                                                          w, sc, k);
        }
        SQ_LAUNCHED("rmt_spmv_kernel");
        for (int round = 0; round < 2; ++round) {  // classical Gram-Schmidt, twice
            rmt_mdot_kernel<<<dim3((unsigned)cb, (unsigned)(k + 1)), kRmtThreads, 0, st>>>(V, w, n, nchunks, partial, sc,
                                                                                          k);
            SQ_LAUNCHED("rmt_mdot_kernel");
            rmt_mdot_reduce_kernel<<<(unsigned)(k + 1), kRmtThreads, 0, st>>>(partial, (int)cb, h, sc, k, round);
            SQ_LAUNCHED("rmt_mdot_reduce_kernel");
            rmt_msub_kernel<<<(unsigned)vb, kRmtThreads, 0, st>>>(V, w, n, h, partial, sc, k);
            SQ_LAUNCHED("rmt_msub_kernel");
        }
        rmt_norm_kernel<<<1, kRmtThreads, 0, st>>>(partial, (int)vb, sc, k, K);
        SQ_LAUNCHED("rmt_norm_kernel");
        rmt_scale_kernel<<<(unsigned)vb, kRmtThreads, 0, st>>>(w, V + (int64_t)(k + 1) * n, n, sc, k);
        SQ_LAUNCHED("rmt_scale_kernel");
        if (std::isfinite(stop_above) && (k + 1) % kRmtCheckEvery == 0 && k + 1 < K) {
            rmt_check_kernel<<<1, 64, 0, st>>>(sc, k, stop_above);
            SQ_LAUNCHED("rmt_check_kernel");
        }
    }
    rmt_tridiag_kernel<<<1, 64, 0, st>>>(sc);
    SQ_LAUNCHED("rmt_tridiag_kernel");
    return SUBQUAD_OK;
}

}  // namespace subquad

using namespace subquad;

extern "C" size_t subquad_rmt_workspace_bytes(int64_t n, int32_t steps) {
    if (n < 0 || steps < 2 || steps > kRmtMaxSteps) return 0;
    return rmt_layout(n, steps).total;
}

extern "C" int subquad_rmt_threshold(const int64_t *row_offsets, const int32_t *cols, const float *vals, int64_t n,
                                     int64_t nnz, int32_t steps, int32_t iters, uint64_t seed, double *tau_out,
                                     double *lambda_plus, double *lambda_max, void *ws, size_t ws_bytes,
                                     void *stream) {
    clear_error();
    SQ_REQUIRE(n >= 0 && nnz >= 0, SUBQUAD_ERR_ARG, "n and nnz must be >= 0");
    SQ_REQUIRE(steps >= 2 && steps <= kRmtMaxSteps, SUBQUAD_ERR_ARG, "steps must be in 2..%d", kRmtMaxSteps);
    SQ_REQUIRE(iters >= 0 && iters <= 60, SUBQUAD_ERR_ARG, "iters must be in 0..60");
    SQ_REQUIRE(tau_out && lambda_plus && lambda_max, SUBQUAD_ERR_ARG, "null output pointer");
    SQ_REQUIRE(n == 0 || row_offsets, SUBQUAD_ERR_ARG, "null row_offsets");
    SQ_REQUIRE(nnz == 0 || (cols && vals), SUBQUAD_ERR_ARG, "null cols or vals");
    const RmtLayout L = rmt_layout(n, steps);
    SQ_REQUIRE(ws && ws_bytes >= L.total, SUBQUAD_ERR_WORKSPACE, "rmt workspace of %zu bytes, %zu needed", ws_bytes,
               L.total);
    SQ_REQUIRE(((uintptr_t)ws & 255) == 0, SUBQUAD_ERR_ARG, "workspace must be 256-byte aligned");
    if (n == 0 || nnz == 0) {
        *lambda_plus = 0.0;
        *lambda_max = 0.0;
        *tau_out = 1.0;  // max a_ij + 1 with max a_ij read as 0: no edge
        return SUBQUAD_OK;
    }
    hipStream_t st = as_stream(stream);
    char *w = static_cast<char *>(ws);
    RmtScalars *sc = reinterpret_cast<RmtScalars *>(w + L.sc);
    double *partial = reinterpret_cast<double *>(w + L.partial);
    const int64_t sb = rmt_blocks(nnz);
    rmt_stats_kernel<<<(unsigned)sb, kRmtThreads, 0, st>>>(vals, nnz, partial);
    SQ_LAUNCHED("rmt_stats_kernel");
    rmt_stats_reduce_kernel<<<1, kRmtThreads, 0, st>>>(partial, (int)sb, sc);
    SQ_LAUNCHED("rmt_stats_reduce_kernel");
    int rc = rmt_lanczos(row_offsets, cols, vals, n, INFINITY, steps, seed, w, L, st);
    if (rc != SUBQUAD_OK) return rc;
    RmtScalars host{};
    SQ_HIP(hipMemcpyAsync(&host, sc, sizeof(RmtScalars), hipMemcpyDeviceToHost, st));
    SQ_HIP(hipStreamSynchronize(st));
    const double lp = 2.0 * std::sqrt(host.sumsq / (double)n);
    const double lmax = host.lambda;
    const double wmax = host.wmax;
    *lambda_plus = lp;
    *lambda_max = lmax;
    if (lmax <= lp) {
        *tau_out = wmax + 1.0;
        return SUBQUAD_OK;
    }
    double lo = 0.0, hi = wmax;
    for (int it = 0; it < iters; ++it) {
        const double mid = 0.5 * (lo + hi);
        rc = rmt_lanczos(row_offsets, cols, vals, n, mid, steps, seed, w, L, st, lp);
        if (rc != SUBQUAD_OK) return rc;
        double lam = 0.0;
        SQ_HIP(hipMemcpyAsync(&lam, &sc->lambda, sizeof(double), hipMemcpyDeviceToHost, st));
        SQ_HIP(hipStreamSynchronize(st));
        if (lam <= lp) lo = mid;
        else hi = mid;
    }
    *tau_out = lo;
    return SUBQUAD_OK;
}

extern "C" int subquad_rmt_lambda_max(const int64_t *row_offsets, const int32_t *cols, const float *vals, int64_t n,
                                      int64_t nnz, double tau, int32_t steps, uint64_t seed, double *lambda_max,
                                      void *ws, size_t ws_bytes, void *stream) {
    clear_error();
    SQ_REQUIRE(n >= 0 && nnz >= 0, SUBQUAD_ERR_ARG, "n and nnz must be >= 0");
    SQ_REQUIRE(steps >= 2 && steps <= kRmtMaxSteps, SUBQUAD_ERR_ARG, "steps must be in 2..%d", kRmtMaxSteps);
    SQ_REQUIRE(lambda_max, SUBQUAD_ERR_ARG, "null output pointer");
    SQ_REQUIRE(n == 0 || row_offsets, SUBQUAD_ERR_ARG, "null row_offsets");
    SQ_REQUIRE(nnz == 0 || (cols && vals), SUBQUAD_ERR_ARG, "null cols or vals");
    const RmtLayout L = rmt_layout(n, steps);
    SQ_REQUIRE(ws && ws_bytes >= L.total, SUBQUAD_ERR_WORKSPACE, "rmt workspace of %zu bytes, %zu needed", ws_bytes,
               L.total);
    SQ_REQUIRE(((uintptr_t)ws & 255) == 0, SUBQUAD_ERR_ARG, "workspace must be 256-byte aligned");
    if (n == 0 || nnz == 0) {
        *lambda_max = 0.0;
        return SUBQUAD_OK;
    }
    hipStream_t st = as_stream(stream);
    char *w = static_cast<char *>(ws);
    int rc = rmt_lanczos(row_offsets, cols, vals, n, tau, steps, seed, w, L, st);
    if (rc != SUBQUAD_OK) return rc;
    RmtScalars *sc = reinterpret_cast<RmtScalars *>(w + L.sc);
    SQ_HIP(hipMemcpyAsync(lambda_max, &sc->lambda, sizeof(double), hipMemcpyDeviceToHost, st));
    SQ_HIP(hipStreamSynchronize(st));
    return SUBQUAD_OK;
}
