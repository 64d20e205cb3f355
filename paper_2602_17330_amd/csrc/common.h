// Shared host/device helpers of libsubquad: status handling, launch checks, wave helpers.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstdio>
#include <string>

#include "subquad.h"

namespace subquad {

// Thread-local message for subquad_last_error().
void set_error(const char *fmt, ...);
void clear_error();

inline hipStream_t as_stream(void *s) { return reinterpret_cast<hipStream_t>(s); }

#define SQ_REQUIRE(cond, code, ...)             \
    do {                                        \
        if (!(cond)) {                          \
            ::subquad::set_error(__VA_ARGS__);  \
            return (code);                      \
        }                                       \
    } while (0)

#define SQ_HIP(expr)                                                                     \
    do {                                                                                 \
        hipError_t err__ = (expr);                                                       \
        if (err__ != hipSuccess) {                                                       \
            ::subquad::set_error("%s failed: %s", #expr, hipGetErrorString(err__));      \
            return SUBQUAD_ERR_HIP;                                                      \
        }                                                                                \
    } while (0)

// Checks the launch that was just enqueued.
#define SQ_LAUNCHED(name)                                                                \
    do {                                                                                 \
        hipError_t err__ = hipGetLastError();                                            \
        if (err__ != hipSuccess) {                                                       \
            ::subquad::set_error("launch of %s failed: %s", name, hipGetErrorString(err__)); \
            return SUBQUAD_ERR_HIP;                                                      \
        }                                                                                \
    } while (0)

constexpr int kWave = 64;

__host__ __device__ inline int64_t ceil_div(int64_t a, int64_t b) { return (a + b - 1) / b; }
inline size_t align_up(size_t v, size_t a) { return (v + a - 1) / a * a; }

// Number of compute units of the current device (cached per process per device).
int device_cus();

// Blocks of 256 threads that one CU holds at once for `kernel` (cached per kernel).
int resident_blocks_per_cu(const void *kernel);

// Launch-shape knob value (default when unset).
int knob(int which);

// A second stream on the current device for the calling host thread (non-blocking, default
// priority), with events to fork work off a caller's stream and join it back: record on one
// stream, wait on the other.  Created on first use and kept until the process ends.  Work
// forked this way joins the caller's stream before the entry point returns, so a captured
// graph gets it as a parallel branch.
struct SideStream {
    hipStream_t s = nullptr;
    hipEvent_t fork = nullptr, done = nullptr;
};
int side_stream(SideStream **out);

// Opt-in per-kernel event timing: prof_begin returns a token (or -1 when timing is off, or
// limited to another kernel) and prof_end records the closing event for it.
int prof_begin(const char *name, hipStream_t st);
void prof_end(int token, const char *name, hipStream_t st);

struct ProfScope {
    int tok;
    const char *name;
    hipStream_t st;
    ProfScope(const char *n, hipStream_t s) : tok(prof_begin(n, s)), name(n), st(s) {}
    ~ProfScope() { prof_end(tok, name, st); }
};

// Upper bound of a repertoire id: the r with rep_offsets[r] <= i < rep_offsets[r+1].
__device__ __forceinline__ int64_t rep_of(const int64_t *__restrict__ offs, int64_t R, int64_t i) {
    int64_t lo = 0, hi = R;  // answer in [lo, hi)
    while (hi - lo > 1) {
        int64_t mid = (lo + hi) >> 1;
        if (offs[mid] <= i) lo = mid; else hi = mid;
    }
    return lo;
}

}  // namespace subquad
