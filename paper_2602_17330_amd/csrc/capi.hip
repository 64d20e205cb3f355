// Library-wide entry points: error reporting, version, sequence validation.
#include <atomic>
#include <cstdarg>
#include <cstring>
#include <mutex>
#include <unordered_map>
#include <vector>

#include "common.h"

namespace subquad {

static thread_local std::string g_last_error;

void set_error(const char *fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    g_last_error = buf;
}

void clear_error() { g_last_error.clear(); }

int device_cus() {
    static std::mutex mu;
    static std::vector<int> cache;
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 256;
    std::lock_guard<std::mutex> lk(mu);
    if ((int)cache.size() <= dev) cache.resize(dev + 1, 0);
    if (cache[dev] == 0) {
        int cus = 0;
        if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus <= 0)
            cus = 256;
        cache[dev] = cus;
    }
    return cache[dev];
}

int resident_blocks_per_cu(const void *kernel) {
    static std::mutex mu;
    static std::unordered_map<const void *, int> cache;
    std::lock_guard<std::mutex> lk(mu);
    auto it = cache.find(kernel);
    if (it != cache.end()) return it->second;
    int nb = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, kernel, 256, 0) != hipSuccess || nb < 1) {
        (void)hipGetLastError();
        nb = 1;
    }
    cache.emplace(kernel, nb);
    return nb;
}

// One thread per row: bit 0 = bad length, bit 1 = bad residue; counts go to out[0], out[1].
__global__ void check_seqs_kernel(const uint8_t *__restrict__ seqs, const int32_t *__restrict__ lens,
                                  int64_t n, int32_t stride, int32_t k,
                                  unsigned long long *__restrict__ out) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    int32_t L = lens[i];
    if (L < k || L > stride) {
        atomicAdd(&out[0], 1ull);
        return;
    }
    const uint8_t *row = seqs + i * (int64_t)stride;
    for (int32_t p = 0; p < L; ++p) {
        if (row[p] >= 20) {
            atomicAdd(&out[1], 1ull);
            return;
        }
    }
}

static std::atomic<int> g_knobs[SUBQUAD_KNOB_COUNT] = {};
static const int kKnobDefault[SUBQUAD_KNOB_COUNT] = {2, 16, 64, 512};

int knob(int which) {
    int v = g_knobs[which].load(std::memory_order_relaxed);
    return v > 0 ? v : kKnobDefault[which];
}

struct ProfRec {
    std::string name;
    hipEvent_t a = nullptr, b = nullptr;
};
static std::mutex g_prof_mu;
static std::vector<ProfRec> g_prof;
static std::vector<hipEvent_t> g_prof_pool;  // events are reused, so timing adds no creation cost
static std::atomic<bool> g_prof_on{false};
static std::string g_prof_only;  // when not empty, only launches of this kernel are timed

static void prof_clear_locked() {
    for (auto &r : g_prof) {
        if (r.a) g_prof_pool.push_back(r.a);
        if (r.b) g_prof_pool.push_back(r.b);
    }
    g_prof.clear();
}

static hipEvent_t prof_event_locked() {
    if (!g_prof_pool.empty()) {
        hipEvent_t e = g_prof_pool.back();
        g_prof_pool.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
}

int side_stream(SideStream **out) {
    constexpr int kMaxDevices = 64;
    int dev = 0;
    SQ_HIP(hipGetDevice(&dev));
    SQ_REQUIRE(dev >= 0 && dev < kMaxDevices, SUBQUAD_ERR_HIP, "device %d out of range", dev);
    static thread_local SideStream side[kMaxDevices];
    SideStream &ss = side[dev];
    if (!ss.s) {
        SideStream made;
        SQ_HIP(hipStreamCreateWithFlags(&made.s, hipStreamNonBlocking));
        SQ_HIP(hipEventCreateWithFlags(&made.fork, hipEventDisableTiming));
        SQ_HIP(hipEventCreateWithFlags(&made.done, hipEventDisableTiming));
        ss = made;
    }
    *out = &ss;
    return SUBQUAD_OK;
}

int prof_begin(const char *name, hipStream_t st) {
    if (!g_prof_on.load(std::memory_order_relaxed)) return -1;
    std::lock_guard<std::mutex> lk(g_prof_mu);
    if (!g_prof_only.empty() && g_prof_only != name) return -1;
    ProfRec r;
    r.a = prof_event_locked();
    r.b = prof_event_locked();
    if (!r.a || !r.b || hipEventRecord(r.a, st) != hipSuccess) {
        if (r.a) g_prof_pool.push_back(r.a);
        if (r.b) g_prof_pool.push_back(r.b);
        return -1;
    }
    g_prof.push_back(r);
    return (int)g_prof.size() - 1;
}

void prof_end(int token, const char *name, hipStream_t st) {
    if (token < 0) return;
    std::lock_guard<std::mutex> lk(g_prof_mu);
    if (token >= (int)g_prof.size()) return;
    g_prof[token].name = name;
    (void)hipEventRecord(g_prof[token].b, st);
}

__global__ void fill_u64_kernel(unsigned long long *p, int64_t n, unsigned long long v) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

}  // namespace subquad

using namespace subquad;

extern "C" const char *subquad_last_error(void) { return g_last_error.c_str(); }

extern "C" const char *subquad_version(void) { return "subquad 0.1 (gfx950)"; }

extern "C" int subquad_set_knob(int32_t which, int32_t value) {
    clear_error();
    SQ_REQUIRE(which >= 0 && which < SUBQUAD_KNOB_COUNT, SUBQUAD_ERR_ARG, "unknown knob %d", which);
    if (which == SUBQUAD_KNOB_EMIT_THREADS && value > 0)
        SQ_REQUIRE(value % 64 == 0 && value <= 1024, SUBQUAD_ERR_ARG, "emit threads must be a multiple of 64 <= 1024");
    g_knobs[which].store(value > 0 ? value : 0, std::memory_order_relaxed);
    return SUBQUAD_OK;
}

extern "C" int32_t subquad_get_knob(int32_t which) {
    if (which < 0 || which >= SUBQUAD_KNOB_COUNT) return -1;
    return knob(which);
}

extern "C" int subquad_profile_enable(int32_t on) {
    clear_error();
    std::lock_guard<std::mutex> lk(g_prof_mu);
    prof_clear_locked();
    g_prof_on.store(on != 0);
    return SUBQUAD_OK;
}

extern "C" int subquad_profile_only(const char *name) {
    clear_error();
    std::lock_guard<std::mutex> lk(g_prof_mu);
    prof_clear_locked();
    g_prof_only = name ? name : "";
    return SUBQUAD_OK;
}

extern "C" int64_t subquad_profile_report(char *buf, size_t len) {
    std::lock_guard<std::mutex> lk(g_prof_mu);
    std::vector<std::pair<std::string, std::pair<int, double>>> agg;
    for (auto &r : g_prof) {
        if (r.name.empty()) continue;
        float ms = 0.f;
        if (hipEventSynchronize(r.b) != hipSuccess || hipEventElapsedTime(&ms, r.a, r.b) != hipSuccess) continue;
        bool found = false;
        for (auto &e : agg)
            if (e.first == r.name) { e.second.first += 1; e.second.second += ms; found = true; break; }
        if (!found) agg.push_back({r.name, {1, (double)ms}});
    }
    std::string out;
    char line[256];
    for (auto &e : agg) {
        snprintf(line, sizeof(line), "%s %d %.6f\n", e.first.c_str(), e.second.first, e.second.second);
        out += line;
    }
    if (buf && len) {
        size_t k = std::min(len - 1, out.size());
        memcpy(buf, out.data(), k);
        buf[k] = 0;
    }
    return (int64_t)out.size();
}

extern "C" int subquad_check_seqs(const uint8_t *seqs, const int32_t *lens, int64_t n, int32_t stride,
                                  int32_t k, int64_t *n_bad, void *stream) {
    clear_error();
    SQ_REQUIRE(n >= 0, SUBQUAD_ERR_ARG, "n must be >= 0");
    SQ_REQUIRE(n == 0 || (seqs && lens), SUBQUAD_ERR_ARG, "null sequence or length pointer");
    SQ_REQUIRE(stride >= 1 && stride <= 4096, SUBQUAD_ERR_ARG, "stride out of range");
    SQ_REQUIRE(k >= 1 && k <= 5, SUBQUAD_ERR_ARG, "k must be in 1..5");
    if (n_bad) *n_bad = 0;
    if (n == 0) return SUBQUAD_OK;
    hipStream_t st = as_stream(stream);
    unsigned long long *dcount = nullptr;
    SQ_HIP(hipMallocAsync((void **)&dcount, 2 * sizeof(unsigned long long), st));
    fill_u64_kernel<<<1, 64, 0, st>>>(dcount, 2, 0ull);
    check_seqs_kernel<<<(unsigned)ceil_div(n, 256), 256, 0, st>>>(seqs, lens, n, stride, k, dcount);
    unsigned long long host[2] = {0, 0};
    hipError_t e1 = hipMemcpyAsync(host, dcount, sizeof(host), hipMemcpyDeviceToHost, st);
    hipError_t e2 = hipStreamSynchronize(st);
    hipError_t e3 = hipFreeAsync(dcount, st);
    SQ_HIP(e1);
    SQ_HIP(e2);
    SQ_HIP(e3);
    if (n_bad) *n_bad = (int64_t)(host[0] + host[1]);
    SQ_REQUIRE(host[0] == 0, SUBQUAD_ERR_LENGTH, "%llu sequence(s) with length outside [k, stride]", host[0]);
    SQ_REQUIRE(host[1] == 0, SUBQUAD_ERR_RESIDUE, "%llu sequence(s) with a residue code >= 20", host[1]);
    return SUBQUAD_OK;
}
