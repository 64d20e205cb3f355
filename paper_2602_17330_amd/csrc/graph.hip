// Sparse similarity graph from the fused pair affinities (Algorithm 1, graph construction;
// Sec. 3.7): every candidate pair (i, j) whose fused weight w >= tau gives the edges i -> j
// and j -> i; each node's neighbours are ordered by weight descending, then neighbour id
// ascending, and the first k are kept (k = 0 keeps all).  Output is CSR.
//
// Mapping to CDNA4: the order (row, weight desc, neighbour asc) is built by three stable
// LSD radix sorts of 64-bit records (key << 32 | directed-edge index), least significant
// key first, so hub nodes of any degree need no special path; a per-node pass then copies
// the first min(k, degree) entries of each row.
#include "radix.h"

namespace subquad {

// Orderable unsigned image of a float: ascending in the float's value.
__device__ __forceinline__ uint32_t float_key(float x) {
    uint32_t u = __float_as_uint(x);
    return (u & 0x80000000u) ? ~u : (u | 0x80000000u);
}

// Directed edge e = 2p + side of pair p: side 0 is i -> j, side 1 is j -> i.
__device__ __forceinline__ void edge_ends(const int32_t *__restrict__ pairs, int64_t e, int32_t &row, int32_t &col) {
    const int64_t p = e >> 1;
    const int32_t a = pairs[2 * p], b = pairs[2 * p + 1];
    row = (e & 1) ? b : a;
    col = (e & 1) ? a : b;
}

// key 0: neighbour id; key 1: weight descending; key 2: row (n for edges below tau).
__global__ void graph_key_kernel(const uint64_t *__restrict__ in, uint64_t *__restrict__ out, int64_t E,
                                 const int32_t *__restrict__ pairs, const float *__restrict__ w, int64_t n,
                                 float tau, int which) {
    for (int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; q < E; q += (int64_t)gridDim.x * blockDim.x) {
        const uint64_t e = in ? (in[q] & 0xFFFFFFFFull) : (uint64_t)q;
        int32_t row, col;
        edge_ends(pairs, (int64_t)e, row, col);
        const float x = w[e >> 1];
        uint32_t key;
        if (which == 0) key = (uint32_t)col;
        else if (which == 1) key = ~float_key(x);
        else key = (x >= tau && row >= 0 && row < n && col >= 0 && col < n) ? (uint32_t)row : (uint32_t)n;
        out[q] = ((uint64_t)key << 32) | e;
    }
}

// full[u] = first sorted position with row >= u (u = 0..n); the live edges end at full[n].
__global__ void graph_rows_kernel(const uint64_t *__restrict__ srec, int64_t E, int64_t n,
                                  uint32_t *__restrict__ full) {
    for (int64_t u = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; u <= n; u += (int64_t)gridDim.x * blockDim.x) {
        int64_t lo = 0, hi = E;
        while (lo < hi) {
            int64_t mid = (lo + hi) >> 1;
            if ((srec[mid] >> 32) < (uint64_t)u) lo = mid + 1; else hi = mid;
        }
        full[u] = (uint32_t)lo;
    }
}

__global__ void graph_len_kernel(const uint32_t *__restrict__ full, int64_t n, int32_t k, uint32_t *__restrict__ len) {
    for (int64_t u = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; u <= n; u += (int64_t)gridDim.x * blockDim.x) {
        if (u == n) { len[u] = 0; continue; }
        uint32_t d = full[u + 1] - full[u];
        len[u] = (k > 0 && d > (uint32_t)k) ? (uint32_t)k : d;
    }
}

// One thread per output slot of each row (rows are walked by a grid-stride over nodes,
// their entries by the inner loop).
__global__ void graph_copy_kernel(const uint64_t *__restrict__ srec, const uint32_t *__restrict__ full,
                                  const uint32_t *__restrict__ outoff, int64_t n, const int32_t *__restrict__ pairs,
                                  const float *__restrict__ w, int64_t cap, int32_t *__restrict__ cols,
                                  float *__restrict__ vals, int64_t *__restrict__ row_offsets) {
    for (int64_t u = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; u <= n; u += (int64_t)gridDim.x * blockDim.x) {
        row_offsets[u] = outoff[u];
        if (u == n) continue;
        const uint32_t o = outoff[u], m = outoff[u + 1] - outoff[u], f = full[u];
        for (uint32_t t = 0; t < m; ++t) {
            if ((int64_t)o + t >= cap) break;
            const uint64_t e = srec[f + t] & 0xFFFFFFFFull;
            int32_t row, col;
            edge_ends(pairs, (int64_t)e, row, col);
            cols[o + t] = col;
            vals[o + t] = w[e >> 1];
        }
    }
}

struct GraphLayout {
    size_t ra, rb, full, len, radix, total;
};

static GraphLayout graph_layout(int64_t n, int64_t P) {
    GraphLayout L{};
    const int64_t E = 2 * P;
    size_t off = 0;
    auto take = [&](size_t bytes) { size_t o = off; off += align_up(std::max<size_t>(bytes, 1), 256); return o; };
    L.ra = take(sizeof(uint64_t) * E);
    L.rb = take(sizeof(uint64_t) * E);
    L.full = take(sizeof(uint32_t) * (n + 1));
    L.len = take(sizeof(uint32_t) * (n + 1));
    L.radix = take(std::max(radix_scratch_bytes(E), scan_scratch_bytes(n + 1)));
    L.total = off;
    return L;
}

static int bits_of(int64_t v) {
    int b = 1;
    while ((int64_t(1) << b) <= v) ++b;
    return b;
}

}  // namespace subquad

using namespace subquad;

extern "C" size_t subquad_graph_workspace_bytes(int64_t n, int64_t P) {
    if (n < 0 || P < 0 || 2 * P >= (int64_t(1) << 32)) return 0;
    return graph_layout(n, P).total;
}

extern "C" int subquad_graph_topk(const int32_t *pairs, const float *w, int64_t P, int64_t n, float tau, int32_t k,
                                  void *ws, size_t ws_bytes, int64_t *row_offsets, int32_t *cols, float *vals,
                                  int64_t cap, int64_t *nnz, void *stream) {
    clear_error();
    SQ_REQUIRE(n >= 0 && P >= 0 && cap >= 0 && k >= 0, SUBQUAD_ERR_ARG, "n, P, cap and k must be >= 0");
    SQ_REQUIRE(n < (int64_t(1) << 31) - 1 && 2 * P < (int64_t(1) << 32), SUBQUAD_ERR_ARG, "n or P too large");
    SQ_REQUIRE(nnz && row_offsets, SUBQUAD_ERR_ARG, "null nnz or row_offsets");
    SQ_REQUIRE(P == 0 || (pairs && w), SUBQUAD_ERR_ARG, "null pairs or weights");
    SQ_REQUIRE(cap == 0 || (cols && vals), SUBQUAD_ERR_ARG, "null output arrays");
    SQ_REQUIRE(ws && ((uintptr_t)ws & 255) == 0, SUBQUAD_ERR_ARG, "workspace must be non-null and 256-byte aligned");
    const GraphLayout L = graph_layout(n, P);
    SQ_REQUIRE(ws_bytes >= L.total, SUBQUAD_ERR_WORKSPACE, "graph workspace of %zu bytes, %zu needed", ws_bytes,
               L.total);
    *nnz = 0;
    hipStream_t st = as_stream(stream);
    char *base = static_cast<char *>(ws);
    uint64_t *ra = reinterpret_cast<uint64_t *>(base + L.ra);
    uint64_t *rb = reinterpret_cast<uint64_t *>(base + L.rb);
    uint32_t *full = reinterpret_cast<uint32_t *>(base + L.full);
    uint32_t *len = reinterpret_cast<uint32_t *>(base + L.len);
    void *scratch = base + L.radix;
    const size_t scratch_bytes = L.total - L.radix;
    const int64_t E = 2 * P;
    const int blocks = (int)std::max<int64_t>(1, std::min<int64_t>(ceil_div(std::max<int64_t>(E, n + 1), 256),
                                                                   (int64_t)device_cus() * 16));
    const int nbits = bits_of(n);
    uint64_t *cur = nullptr;
    if (E > 0) {
        // three stable sorts, least significant key first: neighbour, weight (desc), row
        const uint64_t *prev = nullptr;
        uint64_t *a = ra, *b = rb;
        const int key_bits[3] = {nbits, 32, nbits};
        for (int which = 0; which < 3; ++which) {
            graph_key_kernel<<<blocks, 256, 0, st>>>(prev, a, E, pairs, w, n, tau, which);
            SQ_LAUNCHED("graph_key_kernel");
            uint64_t *sorted = nullptr;
            int rc = radix_sort_u64(a, b, E, nullptr, 32, key_bits[which], scratch, scratch_bytes, st, &sorted,
                                    "sort_graph");
            if (rc != SUBQUAD_OK) return rc;
            prev = sorted;
            uint64_t *other = sorted == a ? b : a;
            a = other;
            b = sorted;
        }
        cur = const_cast<uint64_t *>(prev);
    }
    if (E > 0) {
        graph_rows_kernel<<<blocks, 256, 0, st>>>(cur, E, n, full);
        SQ_LAUNCHED("graph_rows_kernel");
    } else {
        SQ_HIP(hipMemsetAsync(full, 0, sizeof(uint32_t) * (n + 1), st));
    }
    graph_len_kernel<<<blocks, 256, 0, st>>>(full, n, k, len);
    SQ_LAUNCHED("graph_len_kernel");
    int rc = scan_exclusive_u32(len, n + 1, scratch, st);
    if (rc != SUBQUAD_OK) return rc;
    uint32_t total = 0;
    SQ_HIP(hipMemcpyAsync(&total, len + n, sizeof(uint32_t), hipMemcpyDeviceToHost, st));
    SQ_HIP(hipStreamSynchronize(st));
    *nnz = (int64_t)total;
    SQ_REQUIRE((int64_t)total <= cap, SUBQUAD_ERR_CAPACITY, "%u graph entries exceed the capacity %lld", total,
               (long long)cap);
    graph_copy_kernel<<<blocks, 256, 0, st>>>(cur, full, len, n, pairs, w, cap, cols, vals, row_offsets);
    SQ_LAUNCHED("graph_copy_kernel");
    return SUBQUAD_OK;
}
