// tp_runtime.hip -- errors, device memory, prefix sums and kernel timers.
#include "tp_internal.h"

#include <cstring>
#include <mutex>

namespace tp {

static thread_local char g_err[1024] = "";
static tp_allocator g_alloc = {nullptr, nullptr, nullptr};
static bool g_has_alloc = false;
static int g_device = -1;

void set_error(const char* fmt, ...) {
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_err, sizeof(g_err), fmt, ap);
    va_end(ap);
}

void fail(int code, const char* fmt, ...) {
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_err, sizeof(g_err), fmt, ap);
    va_end(ap);
    throw Error{code};
}

int current_device() { return g_device; }

static thread_local Arena* g_arena = nullptr;
constexpr size_t ARENA_CHUNK = size_t(64) << 20;
constexpr size_t ARENA_ALIGN = 256;

bool arena_active() { return g_arena != nullptr; }
ArenaScope::ArenaScope(Arena* a) : prev(g_arena) { g_arena = a; }
ArenaScope::~ArenaScope() { g_arena = prev; }

static void* raw_alloc(size_t bytes, hipStream_t s);

// Released arena chunks are kept for the next hierarchy (up to CACHE_MAX
// bytes): one hierarchy per operator is built and dropped every Newton step,
// and returning its chunks to the device allocator is slow for the large ones.
// A chunk enters the cache only after the arena's stream has drained.
constexpr size_t CACHE_MAX = size_t(32) << 30;  // of 288 GB
static std::mutex g_cache_mu;
static std::vector<ArenaChunk> g_cache;
static size_t g_cache_bytes = 0;

// a cached chunk of at least `bytes` and at most twice that, else a new one
static ArenaChunk chunk_get(size_t bytes, hipStream_t s) {
    {
        std::lock_guard<std::mutex> lk(g_cache_mu);
        int best = -1;
        for (int i = 0; i < (int)g_cache.size(); ++i) {
            const size_t b = g_cache[i].bytes;
            if (b >= bytes && b <= 2 * bytes && (best < 0 || b < g_cache[best].bytes)) best = i;
        }
        if (best >= 0) {
            const ArenaChunk c = g_cache[best];
            g_cache.erase(g_cache.begin() + best);
            g_cache_bytes -= c.bytes;
            return c;
        }
    }
    return ArenaChunk{raw_alloc(bytes, s), bytes};
}

static void chunk_put(const ArenaChunk& c, hipStream_t s) {
    {
        std::lock_guard<std::mutex> lk(g_cache_mu);
        if (g_cache_bytes + c.bytes <= CACHE_MAX) {
            g_cache.push_back(c);
            g_cache_bytes += c.bytes;
            return;
        }
    }
    dfree(c.p, s);
}

void release_chunk_cache() {
    std::vector<ArenaChunk> all;
    {
        std::lock_guard<std::mutex> lk(g_cache_mu);
        all.swap(g_cache);
        g_cache_bytes = 0;
    }
    for (const ArenaChunk& c : all) dfree(c.p, nullptr);
}

static void* arena_alloc(Arena* a, size_t bytes, hipStream_t s) {
    bytes = (bytes + ARENA_ALIGN - 1) / ARENA_ALIGN * ARENA_ALIGN;
    if (bytes > a->left) {
        const size_t sz = bytes > ARENA_CHUNK / 4 ? bytes : ARENA_CHUNK;
        const ArenaChunk ch = chunk_get(sz, s);
        void* c = ch.p;
        a->chunks.push_back(ch);
        if (a->chunks.size() == 1) a->s = s;
        if (bytes > ARENA_CHUNK / 4) {  // dedicated chunk, keep the open one
            a->bytes_used += bytes;
            return c;
        }
        a->cur = static_cast<char*>(c);
        a->left = ch.bytes;
    }
    void* p = a->cur;
    a->cur += bytes;
    a->left -= bytes;
    a->bytes_used += bytes;
    return p;
}

Arena::~Arena() {
    if (chunks.empty()) return;
    (void)hipStreamSynchronize(s);  // the chunks may be handed to another stream next
    for (const ArenaChunk& c : chunks) chunk_put(c, s);
}

void* dalloc(size_t bytes, hipStream_t s) {
    if (g_device < 0) fail(TP_ERR_ARG, "tp_init has not been called");
    if (bytes == 0) bytes = 1;
    if (g_arena) return arena_alloc(g_arena, bytes, s);
    return raw_alloc(bytes, s);
}

static void* raw_alloc(size_t bytes, hipStream_t s) {
    void* p = nullptr;
    if (g_has_alloc) {
        p = g_alloc.alloc(bytes, (void*)s, g_alloc.ctx);
    } else {
        hipError_t e = hipMallocAsync(&p, bytes, s);
        if (e != hipSuccess) p = nullptr;
    }
    if (!p) fail(TP_ERR_OOM, "device allocation of %zu bytes failed", bytes);
    return p;
}

void dfree(void* p, hipStream_t s) {
    if (!p) return;
    if (g_has_alloc) g_alloc.free(p, (void*)s, g_alloc.ctx);
    else (void)hipFreeAsync(p, s);
}

HostMail::HostMail() {
    TP_HIP(hipHostMalloc(&p, 256, hipHostMallocDefault));
    memset(p, 0, 256);
}
HostMail::~HostMail() {
    if (p) (void)hipHostFree(p);
}

// ---- prefix sum ------------------------------------------------------------
// Three-phase scan over tiles of 1024 (256 threads x 4 items).
constexpr int SCAN_BLOCK = 256;
constexpr int SCAN_ITEMS = 4;
constexpr int SCAN_TILE = SCAN_BLOCK * SCAN_ITEMS;

__device__ inline int32_t block_exclusive_scan(int32_t v, int32_t* sh, int32_t* total) {
    // Hillis-Steele over the block in LDS (256 entries)
    const int t = threadIdx.x;
    sh[t] = v;
    __syncthreads();
    for (int off = 1; off < SCAN_BLOCK; off <<= 1) {
        int32_t a = (t >= off) ? sh[t - off] : 0;
        __syncthreads();
        sh[t] += a;
        __syncthreads();
    }
    int32_t incl = sh[t];
    *total = sh[SCAN_BLOCK - 1];
    __syncthreads();
    return incl - v;
}

__global__ void __launch_bounds__(SCAN_BLOCK)
k_scan_tiles(const int32_t* in, int32_t* out,  // may alias (in-place scan)
             int32_t* __restrict__ tile_sums, int32_t n) {
    __shared__ int32_t sh[SCAN_BLOCK];
    const int64_t base = (int64_t)blockIdx.x * SCAN_TILE + threadIdx.x * SCAN_ITEMS;
    int32_t v[SCAN_ITEMS];
    int32_t local = 0;
#pragma unroll
    for (int k = 0; k < SCAN_ITEMS; ++k) {
        v[k] = (base + k < n) ? in[base + k] : 0;
        local += v[k];
    }
    int32_t total;
    int32_t ex = block_exclusive_scan(local, sh, &total);
#pragma unroll
    for (int k = 0; k < SCAN_ITEMS; ++k) {
        if (base + k < n) out[base + k] = ex;
        ex += v[k];
    }
    if (threadIdx.x == 0) tile_sums[blockIdx.x] = total;
}

// single block: exclusive scan of the tile sums in place, total to *grand
__global__ void __launch_bounds__(SCAN_BLOCK)
k_scan_sums(int32_t* __restrict__ sums, int32_t ntiles, int32_t* __restrict__ grand) {
    __shared__ int32_t sh[SCAN_BLOCK];
    int32_t carry = 0;
    for (int32_t start = 0; start < ntiles; start += SCAN_BLOCK) {
        int32_t i = start + threadIdx.x;
        int32_t v = (i < ntiles) ? sums[i] : 0;
        int32_t total;
        int32_t ex = block_exclusive_scan(v, sh, &total);
        if (i < ntiles) sums[i] = carry + ex;
        carry += total;
    }
    if (threadIdx.x == 0) *grand = carry;
}

__global__ void __launch_bounds__(SCAN_BLOCK)
k_scan_add(int32_t* __restrict__ out, const int32_t* __restrict__ sums, int32_t n) {
    const int64_t base = (int64_t)blockIdx.x * SCAN_TILE + threadIdx.x * SCAN_ITEMS;
    const int32_t add = sums[blockIdx.x];
#pragma unroll
    for (int k = 0; k < SCAN_ITEMS; ++k)
        if (base + k < n) out[base + k] += add;
}

// Up to 16384 entries: one workgroup (1024 threads x 16 consecutive items;
// wavefront scans by shuffles, then the 16 wavefront totals), one launch
// instead of three. Every thread reads its items before the first barrier and
// writes after it, so in-place use is safe.
constexpr int SS_T = 1024;
constexpr int SS_ITEMS = 16;
constexpr int SS_MAX = SS_T * SS_ITEMS;

__global__ void __launch_bounds__(SS_T)
k_scan_small(const int32_t* in, int32_t* out, int32_t n) {
    __shared__ int32_t wsum[SS_T / 64];
    const int t = threadIdx.x, lane = t & 63, w = t >> 6;
    const int32_t base = t * SS_ITEMS;
    int32_t v[SS_ITEMS];
    int32_t local = 0;
#pragma unroll
    for (int k = 0; k < SS_ITEMS; ++k) {
        v[k] = base + k < n ? in[base + k] : 0;
        local += v[k];
    }
    int32_t x = local;  // inclusive scan over the wavefront
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        const int32_t y = __shfl_up(x, d, 64);
        if (lane >= d) x += y;
    }
    if (lane == 63) wsum[w] = x;
    __syncthreads();
    if (w == 0) {
        int32_t y = lane < SS_T / 64 ? wsum[lane] : 0;
#pragma unroll
        for (int d = 1; d < SS_T / 64; d <<= 1) {
            const int32_t z = __shfl_up(y, d, 64);
            if (lane >= d) y += z;
        }
        if (lane < SS_T / 64) wsum[lane] = y;
    }
    __syncthreads();
    int32_t ex = (w > 0 ? wsum[w - 1] : 0) + x - local;
#pragma unroll
    for (int k = 0; k < SS_ITEMS; ++k) {
        if (base + k < n) out[base + k] = ex;
        ex += v[k];
    }
    if (t == 0) out[n] = wsum[SS_T / 64 - 1];
}

void scan_exclusive(const int32_t* in, int32_t* out, int32_t n, hipStream_t s) {
    if (n <= SS_MAX) {
        TP_LAUNCH(k_scan_small, 1, SS_T, 0, s, in, out, n);
        return;
    }
    int ntiles = n > 0 ? cdiv(n, SCAN_TILE) : 1;
    DBuf<int32_t> sums(ntiles, s);
    if (n > 0) TP_LAUNCH(k_scan_tiles, ntiles, SCAN_BLOCK, 0, s, in, out, sums.p, n);
    TP_LAUNCH(k_scan_sums, 1, SCAN_BLOCK, 0, s, sums.p, n > 0 ? ntiles : 0, out + n);
    if (n > 0) TP_LAUNCH(k_scan_add, ntiles, SCAN_BLOCK, 0, s, out, sums.p, n);
}

int32_t read_i32(const int32_t* dptr, hipStream_t s) {
    int32_t v = 0;
    TP_HIP(hipMemcpyAsync(&v, dptr, sizeof(int32_t), hipMemcpyDeviceToHost, s));
    TP_HIP(hipStreamSynchronize(s));
    return v;
}

// ---- kernel timer ------------------------------------------------------------
KernelTimer& timer() {
    static KernelTimer t;
    return t;
}

bool timer_events(double bytes, hipEvent_t* start, hipEvent_t* stop) {
    KernelTimer& t = timer();
    if (!t.on) return false;
    if (t.used * 2 + 2 > t.ev.size()) {
        size_t old = t.ev.size();
        t.ev.resize(old == 0 ? 512 : old * 2);
        for (size_t i = old; i < t.ev.size(); ++i) TP_HIP(hipEventCreate(&t.ev[i]));
        t.ev_bytes.resize(t.ev.size() / 2);
    }
    size_t idx = t.used++;
    t.ev_bytes[idx] = bytes;
    *start = t.ev[2 * idx];
    *stop = t.ev[2 * idx + 1];
    return true;
}

void timer_collect() {
    KernelTimer& t = timer();
    for (size_t i = 0; i < t.used; ++i) {
        TP_HIP(hipEventSynchronize(t.ev[2 * i + 1]));
        float ms = 0.f;
        TP_HIP(hipEventElapsedTime(&ms, t.ev[2 * i], t.ev[2 * i + 1]));
        t.ms += ms;
        t.bytes += t.ev_bytes[i];
        t.launches += 1;
    }
    t.used = 0;
}

}  // namespace tp

extern "C" {

const char* tp_last_error(void) { return tp::g_err; }

int tp_init(const tp_allocator* alloc, int device) {
    TP_GUARD({
        int count = 0;
        TP_HIP(hipGetDeviceCount(&count));
        TP_CHECK_ARG(device >= 0 && device < count, "device %d out of range (%d devices)", device, count);
        // cached arena chunks belong to the previous device and allocator
        if (tp::g_device >= 0) {
            tp::release_chunk_cache();
            tp::release_ws_cache();
        }
        TP_HIP(hipSetDevice(device));
        tp::g_device = device;
        (void)tp::scratch_ptr();  // the device's copy of the allocation-free apply's scratch
        // keep freed blocks in the device's stream-ordered pool instead of
        // returning them to the driver at every synchronisation
        hipMemPool_t pool = nullptr;
        if (hipDeviceGetDefaultMemPool(&pool, device) == hipSuccess && pool) {
            uint64_t keep = UINT64_MAX;
            TP_HIP(hipMemPoolSetAttribute(pool, hipMemPoolAttrReleaseThreshold, &keep));
        }
        if (alloc) {
            TP_CHECK_ARG(alloc->alloc && alloc->free, "allocator needs alloc and free");
            tp::g_alloc = *alloc;
            tp::g_has_alloc = true;
        } else {
            tp::g_has_alloc = false;
        }
    });
    return TP_OK;
}

int tp_timer_enable(int32_t on) {
    TP_GUARD({
        tp::KernelTimer& t = tp::timer();
        if (t.on) tp::timer_collect();
        t.on = on != 0;
        t.launches = 0;
        t.ms = 0.0;
        t.bytes = 0.0;
        t.used = 0;
    });
    return TP_OK;
}

int tp_timer_read(int64_t* launches, double* ms, double* bytes) {
    TP_GUARD({
        TP_CHECK_ARG(launches && ms && bytes, "null output");
        tp::timer_collect();
        tp::KernelTimer& t = tp::timer();
        *launches = t.launches;
        *ms = t.ms;
        *bytes = t.bytes;
    });
    return TP_OK;
}

}  // extern "C"
