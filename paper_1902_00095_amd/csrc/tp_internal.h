// tp_internal.h -- shared host-side plumbing of the tpsolve library (gfx950).
//
// Errors travel as tp::Error exceptions inside the library and are turned
// into status codes at every extern "C" entry point (TP_GUARD).  Device
// memory comes from the allocator registered with tp_init.
#pragma once

#include <hip/hip_runtime.h>
#include <hip/hip_ext.h>

#include <cstdarg>
#include <cstdint>
#include <cstdio>
#include <vector>

#include "tpsolve.h"

namespace tp {

struct Error {
    int code;
};

void set_error(const char* fmt, ...);
[[noreturn]] void fail(int code, const char* fmt, ...);

#define TP_HIP(call)                                                                  \
    do {                                                                              \
        hipError_t e_ = (call);                                                       \
        if (e_ != hipSuccess) {                                                       \
            (void)hipGetLastError(); /* reported here: do not leave it to the next call */ \
            ::tp::fail(TP_ERR_HIP, "%s failed: %s (%s:%d)", #call, hipGetErrorString(e_), \
                       __FILE__, __LINE__);                                           \
        }                                                                             \
    } while (0)

#define TP_CHECK_ARG(cond, ...)                                                       \
    do {                                                                              \
        if (!(cond)) ::tp::fail(TP_ERR_ARG, __VA_ARGS__);                             \
    } while (0)

// Launch with an immediate check of the launch itself.
#define TP_LAUNCH(kernel, grid, block, shmem, stream, ...)                            \
    do {                                                                              \
        hipLaunchKernelGGL(kernel, dim3(grid), dim3(block), shmem, stream, __VA_ARGS__); \
        TP_HIP(hipGetLastError());                                                    \
    } while (0)

// Wrap an extern "C" body: exceptions become status codes.
#define TP_GUARD(...)                                                                 \
    try {                                                                             \
        __VA_ARGS__;                                                                  \
    } catch (const ::tp::Error& e_) {                                                 \
        return e_.code;                                                               \
    } catch (...) {                                                                   \
        ::tp::set_error("unexpected C++ exception");                                  \
        return TP_ERR_HIP;                                                            \
    }

void* dalloc(size_t bytes, hipStream_t s);
void dfree(void* p, hipStream_t s);
int current_device();

// Bump allocator over large device chunks.  While an ArenaScope is active on
// a host thread, every DBuf allocation of that thread is carved from the
// arena and its individual free is a no-op; the arena returns its chunks
// when it is destroyed.  Used for AMG setups (no frees during setup, a few
// frees at teardown).
struct ArenaChunk {
    void* p;
    size_t bytes;
};
struct Arena {
    std::vector<ArenaChunk> chunks;
    char* cur = nullptr;
    size_t left = 0;
    hipStream_t s = nullptr;
    size_t bytes_used = 0;
    ~Arena();
};
bool arena_active();
void release_chunk_cache();  // frees every cached arena chunk
void release_ws_cache();     // frees every idle FGMRES workspace
struct ArenaScope {
    Arena* prev;
    explicit ArenaScope(Arena* a);
    ~ArenaScope();
};

// Owning device buffer (stream-ordered free).
template <typename T>
struct DBuf {
    T* p = nullptr;
    size_t n = 0;
    hipStream_t s = nullptr;
    bool in_arena = false;
    DBuf() = default;
    DBuf(size_t count, hipStream_t st) { alloc(count, st); }
    void alloc(size_t count, hipStream_t st) {
        release();
        s = st;
        n = count;
        in_arena = arena_active();
        p = count ? static_cast<T*>(dalloc(count * sizeof(T), st)) : nullptr;
    }
    void release() {
        if (p && !in_arena) dfree(p, s);
        p = nullptr;
        n = 0;
    }
    ~DBuf() { release(); }
    DBuf(const DBuf&) = delete;
    DBuf& operator=(const DBuf&) = delete;
    DBuf(DBuf&& o) noexcept : p(o.p), n(o.n), s(o.s), in_arena(o.in_arena) { o.p = nullptr; o.n = 0; }
    DBuf& operator=(DBuf&& o) noexcept {
        if (this != &o) {
            release();
            p = o.p; n = o.n; s = o.s; in_arena = o.in_arena;
            o.p = nullptr; o.n = 0;
        }
        return *this;
    }
    T* get() const { return p; }
};

struct Csr {
    int32_t n = 0, m = 0, nnz = 0;  // n rows, m columns
    DBuf<int32_t> rowptr, col;
    DBuf<double> val;
};

// Pinned host scalar mailbox for the few device->host reads of a solve.
struct HostMail {
    void* p = nullptr;
    HostMail();
    ~HostMail();
    template <typename T> T* as() { return static_cast<T*>(p); }
};

inline int cdiv(int64_t a, int64_t b) { return static_cast<int>((a + b - 1) / b); }

// Exclusive prefix sum of n int32 counts into out[0..n] (out[n] = total).
// `in` and `out` may alias (in-place with out == in works when out has n+1
// slots).  Returns nothing; read out[n] with read_i32 when the host needs it.
void scan_exclusive(const int32_t* in, int32_t* out, int32_t n, hipStream_t s);
int32_t read_i32(const int32_t* dptr, hipStream_t s);   // synchronises s

// Fine-level smoother timer (dominant kernel); see tp_timer_enable.
struct KernelTimer {
    bool on = false;
    int64_t launches = 0;
    double ms = 0.0, bytes = 0.0;
    std::vector<hipEvent_t> ev;  // pairs
    std::vector<double> ev_bytes;
    size_t used = 0;
};
KernelTimer& timer();
// The current device's copy of the fixed scratch array of the allocation-free
// preconditioner apply (resolved once per device; defined with the array).
double* scratch_ptr();
// When the timer is on, reserve an event pair for one launch of the timed
// kernel (returns false when off).  The pair is handed to
// hipExtLaunchKernelGGL, which stamps the kernel's own dispatch start and
// completion, so the interval is the kernel's execution time.
bool timer_events(double bytes, hipEvent_t* start, hipEvent_t* stop);
void timer_collect();  // fold recorded pairs into totals (synchronises events)

// Launch, with the timer's event pair when `timed` (null events otherwise).
#define TP_LAUNCH_TIMED(timed, bytes, kernel, grid, block, shmem, stream, ...)           \
    do {                                                                              \
        if (timed) {                                                                  \
            hipEvent_t e0_ = nullptr, e1_ = nullptr;                                  \
            ::tp::timer_events((bytes), &e0_, &e1_);                                  \
            hipExtLaunchKernelGGL(kernel, dim3(grid), dim3(block), shmem, stream, e0_, e1_, 0, \
                                  __VA_ARGS__);                                       \
        } else {                                                                      \
            hipLaunchKernelGGL(kernel, dim3(grid), dim3(block), shmem, stream, __VA_ARGS__); \
        }                                                                             \
        TP_HIP(hipGetLastError());                                                    \
    } while (0)

}  // namespace tp
