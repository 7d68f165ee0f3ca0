// tp_amg_setup.hip -- AMG hierarchy construction on the GPU, FP64.
//
// The paper applies A_pp^{-1} and the inverse of its Schur approximation by
// one AMG V-cycle each (Section 3.2, Section 4).  The components:
//   strength      j in S_i iff j != i, m_i > 0 and -s_i a_ij >= theta m_i,
//                 s_i = sign(a_ii), m_i = max_{k != i} -s_i a_ik;
//   coarsening    PMIS (De Sterck, Yang & Heys, SIMAX 2006): measure
//                 lambda_i = |S^T_i|, key (lambda_i, splitmix64(seed ^
//                 level << 40 ^ i), i) compared lexicographically; each round
//                 selects, from a snapshot, the undecided points whose key
//                 beats every undecided strong neighbour (S_i u S^T_i), then
//                 marks undecided points depending on a C point as F;
//   interpolation direct interpolation (Stueben 2001) with same-sign
//                 couplings lumped into the diagonal;
//   restriction   R = P^T, or R = Q^T with Q the direct interpolation of A^T
//                 on the same C/F split (Petrov-Galerkin);
//   coarse op.    A_c = R (A P), each entry summed in ascending inner index;
//   coarsest      explicit inverse by blocked Gauss-Jordan elimination with partial
//                 pivoting (same pivot rule as an LU: largest modulus, lowest row).
// PMIS decisions are integer comparisons, so the C/F split is exact on any
// hardware.  Floating-point steps are written in one fixed operation order
// and compiled without contraction, so the hierarchy values follow a single
// rounding sequence.  There are no floating-point atomics.
#include "tp_amg.h"

#include <cfloat>

#include <algorithm>

namespace tp {

constexpr int B = 256;

// Lanes cooperating on a row: the power of two at or above the mean row
// length; on levels of 65536 rows or more (bandwidth-bound) half of that, so
// a wavefront serves twice the rows with the same loads in flight (on the
// 128 x 128 x 64 workload the preconditioner apply drops from 1.28 to 1.20 ms;
// small levels are launch-bound and keep the wider groups).
int lanes_for(int32_t n, int64_t nnz) {
    double avg = n > 0 ? (double)nnz / n : 1.0;
    if (n >= 65536) avg /= 2.0;
    int g = 1;
    while (g < avg && g < 64) g <<= 1;
    // Large levels take at most 8 lanes a row (16 for rows of more than 32
    // entries): more rows per wavefront keep more independent loads in
    // flight.  Measured on the 256x256x64 hierarchies' first coarse levels
    // (18-29 entries a row): 8 lanes fastest, 16 lanes +4% time per
    // preconditioner apply, 32 lanes +13%, 4 lanes +2%; on the second
    // levels (46-60 entries) 16 lanes are 1% faster than 8.
    if (n >= 65536 && g > 8) g = avg > 16.0 ? 16 : 8;
    return g;
}

// ---- transpose ------------------------------------------------------------------
__global__ void __launch_bounds__(B)
k_fill_i32(int32_t* __restrict__ a, int32_t v, int64_t n) {
    int64_t i = (int64_t)blockIdx.x * B + threadIdx.x;
    if (i < n) a[i] = v;
}

// Sorted copy of each row: one 64-lane workgroup per row; an entry's
// destination is its rank (number of smaller column indices in the row;
// columns within a row are distinct).
__global__ void __launch_bounds__(64)
k_sort_rows(int32_t n, const int32_t* __restrict__ rowptr, const int32_t* __restrict__ col_in,
            const double* __restrict__ val_in, int32_t* __restrict__ col, double* __restrict__ val) {
    for (int32_t i = blockIdx.x; i < n; i += gridDim.x) {
        const int32_t a = rowptr[i], L = rowptr[i + 1] - a;
        for (int32_t e = threadIdx.x; e < L; e += 64) {
            const int32_t key = col_in[a + e];
            int32_t rank = 0;
            for (int32_t q = 0; q < L; ++q) rank += col_in[a + q] < key;
            col[a + rank] = key;
            if (val) val[a + rank] = val_in[a + e];
        }
    }
}

// ---- a lane group per row: strength, direct interpolation, transpose -------------------
// Each row gets a group of lanes sized to the level's rows (row_group: 8 on
// the finest levels, whose rows hold about 7 entries, up to 32 on coarse
// ones; a thread per row would make every load instruction of a wavefront
// touch a cache line per lane).  Entries are loaded lane-parallel;
// a floating-point sum is still taken in row order (each entry's term is
// broadcast to the group in turn, all lanes adding the same sequence), and
// outputs are compacted in row order by ballot, so the results equal those
// of one thread walking the row, bit for bit.
constexpr int WR = 64;
constexpr int WR_ROWS = B / WR;

// Lane l's value broadcast to the wavefront, l uniform (v_readlane: no
// LDS round trip, unlike a shuffle -- the row sums below broadcast their
// terms one by one)
__device__ inline int32_t bcast_i(int32_t v, int l) { return __builtin_amdgcn_readlane(v, l); }
__device__ inline double bcast_d(double v, int l) {
    const long long b = __double_as_longlong(v);
    const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int32_t)(uint32_t)b, l);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int32_t)(uint32_t)(b >> 32), l);
    return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}
constexpr double WR_MIN_AVG = 10.0;  // mean row length from which a level uses them

__device__ inline int below_count(uint64_t mask, int lane) {
    return __popcll(mask & ((1ull << lane) - 1ull));
}

// Lane groups of G lanes per row (G a power of two dividing 64): the
// group's mask of a predicate (bit l: lane l of the group), and a value of
// lane l of the group (l the same in all lanes of the group).
template <int G>
__device__ inline uint64_t gballot(bool p) {
    const uint64_t b = __ballot(p);
    if constexpr (G == 64) return b;
    else return (b >> ((threadIdx.x & 63) & ~(G - 1))) & ((1ull << G) - 1ull);
}
template <int G>
__device__ inline int32_t gbcast_i(int32_t v, int l) {
    if constexpr (G == 64) return bcast_i(v, l);
    else return __shfl(v, l, G);
}
template <int G>
__device__ inline double gbcast_d(double v, int l) {
    if constexpr (G == 64) return bcast_d(v, l);
    else return __shfl(v, l, G);
}

template <int G>
__device__ inline void row_sign_max_w(const int32_t* rowptr, const int32_t* col, const double* val, int32_t i,
                                      int lane, double* s_out, double* m_out) {
    const int32_t a = rowptr[i], e = rowptr[i + 1];
    double aii = 0.0;
    bool has = false;
    for (int32_t q = a + lane; q < e; q += G)
        if (col[q] == i) { aii = val[q]; has = true; }
    const uint64_t hm = gballot<G>(has);
    aii = hm ? gbcast_d<G>(aii, __ffsll((unsigned long long)hm) - 1) : 0.0;
    const double s = aii < 0.0 ? -1.0 : 1.0;
    double m = 0.0;
    for (int32_t q = a + lane; q < e; q += G)
        if (col[q] != i && -s * val[q] > m) m = -s * val[q];
#pragma unroll
    for (int d = G / 2; d > 0; d >>= 1) m = fmax(m, __shfl_xor(m, d, G));
    *s_out = s;
    *m_out = m;
}

template <int G>
__global__ void __launch_bounds__(B)
k_strength_w(int32_t n, const int32_t* __restrict__ rowptr, const int32_t* __restrict__ col,
             const double* __restrict__ val, double theta, int32_t* __restrict__ cnt,
             const int32_t* __restrict__ Srowptr, int32_t* __restrict__ Scol) {
    const int32_t i = blockIdx.x * (B / G) + threadIdx.x / G;
    const int lane = threadIdx.x % G;
    if (i >= n) return;  // whole wavefront
    double s, m;
    row_sign_max_w<G>(rowptr, col, val, i, lane, &s, &m);
    int32_t c = 0;
    const int32_t out = Scol ? Srowptr[i] : 0;
    if (m > 0.0) {
        for (int32_t b = rowptr[i]; b < rowptr[i + 1]; b += G) {
            const int32_t q = b + lane;
            const bool strong = q < rowptr[i + 1] && col[q] != i && -s * val[q] >= theta * m;
            const uint64_t mk = gballot<G>(strong);
            if (Scol && strong) Scol[out + c + below_count(mk, lane)] = col[q];
            c += __popcll(mk);
        }
    }
    if (cnt && lane == 0) cnt[i] = c;
}

template <int G>
__global__ void __launch_bounds__(B)
k_interp_count_w(int32_t n, const int32_t* __restrict__ Srp, const int32_t* __restrict__ Sc,
                 const int32_t* __restrict__ cf, int32_t* __restrict__ cnt) {
    const int32_t i = blockIdx.x * (B / G) + threadIdx.x / G;
    const int lane = threadIdx.x % G;
    if (i >= n) return;
    int32_t c = 0;
    for (int32_t q = Srp[i] + lane; q < Srp[i + 1]; q += G) c += cf[Sc[q]];
#pragma unroll
    for (int d = G / 2; d > 0; d >>= 1) c += __shfl_xor(c, d, G);
    if (lane == 0) cnt[i] = cf[i] ? 1 : c;
}

// is j among the sorted strong columns Sc[a, e)?
__device__ inline bool in_sorted(const int32_t* Sc, int32_t a, int32_t e, int32_t j) {
    int32_t lo = a, hi = e;  // first position in [a, e) whose column is >= j
    while (lo < hi) {
        const int32_t mid = lo + (hi - lo) / 2;
        if (Sc[mid] < j) lo = mid + 1;
        else hi = mid;
    }
    return lo < e && Sc[lo] == j;
}

template <int G>
__global__ void __launch_bounds__(B)
k_interp_fill_w(int32_t n, const int32_t* __restrict__ rowptr, const int32_t* __restrict__ col,
                const double* __restrict__ val, const int32_t* __restrict__ Srp,
                const int32_t* __restrict__ Sc, const int32_t* __restrict__ cf,
                const int32_t* __restrict__ cmap, const int32_t* __restrict__ Prp,
                int32_t* __restrict__ Pc, double* __restrict__ Pv) {
    const int32_t i = blockIdx.x * (B / G) + threadIdx.x / G;
    const int lane = threadIdx.x % G;
    if (i >= n) return;
    const int32_t q0 = Prp[i];
    if (cf[i]) {
        if (lane == 0) { Pc[q0] = cmap[i]; Pv[q0] = 1.0; }
        return;
    }
    if (Prp[i + 1] == q0) return;  // no strong C neighbour: empty row
    const int32_t a = rowptr[i], e = rowptr[i + 1], sa = Srp[i], se = Srp[i + 1];
    double aii = 0.0;
    bool has = false;
    for (int32_t q = a + lane; q < e; q += G)
        if (col[q] == i) { aii = val[q]; has = true; }
    const uint64_t hm = gballot<G>(has);
    aii = hm ? gbcast_d<G>(aii, __ffsll((unsigned long long)hm) - 1) : 0.0;
    const double s = aii < 0.0 ? -1.0 : 1.0;
    // the three sums in row order, exactly as one thread would take them
    double sum_all = 0.0, lump = 0.0, sum_p = 0.0;
    for (int32_t b = a; b < e; b += G) {
        const int32_t q = b + lane;
        const bool ok = q < e;
        const int32_t j = ok ? col[q] : -1;
        const double v = ok ? val[q] : 0.0;
        const bool sc = ok && j != i && cf[j] && in_sorted(Sc, sa, se, j);
        const uint64_t scm = gballot<G>(sc);
        const int len = min(G, (int)(e - b));
        for (int l = 0; l < len; ++l) {
            const int32_t jl = gbcast_i<G>(j, l);
            const double vl = gbcast_d<G>(v, l);
            if (jl != i) {
                if (s * vl < 0.0) sum_all += vl;
                else lump += vl;
            }
            if ((scm >> l) & 1ull) sum_p += vl;
        }
    }
    const double alpha = sum_all / sum_p;
    const double dtil = aii + lump;
    int32_t c = 0;
    for (int32_t b = a; b < e; b += G) {
        const int32_t q = b + lane;
        const bool ok = q < e;
        const int32_t j = ok ? col[q] : -1;
        const bool sc = ok && j != i && cf[j] && in_sorted(Sc, sa, se, j);
        const uint64_t scm = gballot<G>(sc);
        if (sc) {
            const int32_t pos = q0 + c + below_count(scm, lane);
            Pc[pos] = cmap[j];
            Pv[pos] = -(alpha * val[q]) / dtil;
        }
        c += __popcll(scm);
    }
}

template <int G>
__global__ void __launch_bounds__(B)
k_col_count_w(int32_t n, const int32_t* __restrict__ rowptr, const int32_t* __restrict__ col,
              int32_t* __restrict__ cnt) {
    const int32_t i = blockIdx.x * (B / G) + threadIdx.x / G;
    const int lane = threadIdx.x % G;
    if (i >= n) return;
    for (int32_t q = rowptr[i] + lane; q < rowptr[i + 1]; q += G) atomicAdd(&cnt[col[q]], 1);
}

template <int G>
__global__ void __launch_bounds__(B)
k_transpose_fill_w(int32_t n, const int32_t* __restrict__ rowptr, const int32_t* __restrict__ col,
                   const double* __restrict__ val, int32_t* __restrict__ cursor,
                   int32_t* __restrict__ Tcol, double* __restrict__ Tval) {
    const int32_t i = blockIdx.x * (B / G) + threadIdx.x / G;
    const int lane = threadIdx.x % G;
    if (i >= n) return;
    for (int32_t q = rowptr[i] + lane; q < rowptr[i + 1]; q += G) {
        const int32_t pos = atomicAdd(&cursor[col[q]], 1);
        Tcol[pos] = i;
        if (Tval) Tval[pos] = val[q];
    }
}

// Values of A^T on A's own pattern, for a square A whose pattern is
// symmetric: entry (i, j) goes to the position of column i in row j (binary
// search).  *asym is set when some (i, j) has no (j, i).
template <int G>
__global__ void __launch_bounds__(B)
k_transpose_sym(int32_t n, const int32_t* __restrict__ rowptr, const int32_t* __restrict__ col,
                const double* __restrict__ val, double* __restrict__ Tval, int32_t* __restrict__ asym) {
    const int32_t i = blockIdx.x * (B / G) + threadIdx.x / G;
    const int lane = threadIdx.x % G;
    if (i >= n) return;
    for (int32_t q = rowptr[i] + lane; q < rowptr[i + 1]; q += G) {
        const int32_t j = col[q];
        int32_t lo = rowptr[j], hi = rowptr[j + 1];
        while (lo < hi) {
            const int32_t mid = lo + (hi - lo) / 2;
            if (col[mid] < i) lo = mid + 1;
            else hi = mid;
        }
        if (lo < rowptr[j + 1] && col[lo] == i) Tval[lo] = val[q];
        else *asym = 1;
    }
}

static bool long_rows(int32_t n, int32_t nnz) { return n > 0 && (double)nnz / n >= WR_MIN_AVG; }

// Lanes per row for the row kernels: the mean row length rounded up to a
// power of two, at least 4 and at most 32 (a group then loads a row, or a
// 32-entry piece of it, in one contiguous access; wider groups left most
// lanes idle on the coarse levels' rows of 18-60 entries).
static int row_group(int32_t n, int64_t nnz) {
    const double avg = n > 0 ? (double)nnz / n : 1.0;
    int g = 4;
    while (g < avg && g < 32) g <<= 1;
    return g;
}

// A row kernel templated on its lane-group size G, launched with the group
// size g of row_group.
#define TP_ROWS_LAUNCH(kernel, g, n, stream, ...)                                             \
    do {                                                                                      \
        switch (g) {                                                                          \
        case 4: TP_LAUNCH(kernel<4>, cdiv((n), B / 4), B, 0, stream, __VA_ARGS__); break;     \
        case 8: TP_LAUNCH(kernel<8>, cdiv((n), B / 8), B, 0, stream, __VA_ARGS__); break;     \
        case 16: TP_LAUNCH(kernel<16>, cdiv((n), B / 16), B, 0, stream, __VA_ARGS__); break;  \
        default: TP_LAUNCH(kernel<32>, cdiv((n), B / 32), B, 0, stream, __VA_ARGS__); break;  \
        }                                                                                     \
    } while (0)

// T = A^T (m rows); values optional; rows sorted when `sorted`.  nnz is the
// entry count or an upper bound of it: it only sizes the allocations (the
// counts come from rowptr), and T.nnz keeps the value passed.
void transpose(const int32_t* rowptr, const int32_t* col, const double* val, int32_t n,
                      int32_t m, int32_t nnz, bool sorted, Csr& T, hipStream_t s) {
    T.n = m;
    T.m = n;
    T.nnz = nnz;
    T.rowptr.alloc(m + 1, s);
    T.col.alloc(nnz, s);
    if (val) T.val.alloc(nnz, s);
    DBuf<int32_t> cursor(m + 1, s);
    TP_LAUNCH(k_fill_i32, cdiv(m + 1, B), B, 0, s, T.rowptr.p, 0, (int64_t)m + 1);
    const int g = row_group(n, nnz);
    if (n > 0) TP_ROWS_LAUNCH(k_col_count_w, g, n, s, n, rowptr, col, T.rowptr.p);
    auto fill = [&](int32_t* tc, double* tv) {
        if (n > 0) TP_ROWS_LAUNCH(k_transpose_fill_w, g, n, s, n, rowptr, col, val, cursor.p, tc, tv);
    };
    scan_exclusive(T.rowptr.p, T.rowptr.p, m, s);
    TP_HIP(hipMemcpyAsync(cursor.p, T.rowptr.p, sizeof(int32_t) * (m + 1), hipMemcpyDeviceToDevice, s));
    if (!sorted) {
        fill(T.col.p, val ? T.val.p : nullptr);
        return;
    }
    DBuf<int32_t> tcol(nnz, s);
    DBuf<double> tval(val ? nnz : 0, s);
    fill(tcol.p, val ? tval.p : nullptr);
    if (m > 0)
        TP_LAUNCH(k_sort_rows, std::min(m, 65536), 64, 0, s, m, T.rowptr.p, tcol.p,
                  val ? tval.p : nullptr, T.col.p, val ? T.val.p : nullptr);
}

// T = A^T (square A, values, sorted rows).  The finest operators share a
// symmetric stencil pattern: when `try_sym`, A^T is first formed on A's own
// pattern (no atomics, no sort); a pattern found asymmetric falls back to the
// general transpose.
static void transpose_square(const Csr& A, bool try_sym, Csr& T, hipStream_t s) {
    if (try_sym && A.n > 0) {
        T.n = T.m = A.n;
        T.nnz = A.nnz;
        T.rowptr.alloc(A.n + 1, s);
        T.col.alloc(A.nnz, s);
        T.val.alloc(A.nnz, s);
        DBuf<int32_t> asym(1, s);
        TP_LAUNCH(k_fill_i32, 1, B, 0, s, asym.p, 0, (int64_t)1);
        TP_ROWS_LAUNCH(k_transpose_sym, row_group(A.n, A.nnz), A.n, s, A.n, A.rowptr.p, A.col.p, A.val.p, T.val.p,
                       asym.p);
        if (read_i32(asym.p, s) == 0) {
            TP_HIP(hipMemcpyAsync(T.rowptr.p, A.rowptr.p, sizeof(int32_t) * (A.n + 1), hipMemcpyDeviceToDevice, s));
            TP_HIP(hipMemcpyAsync(T.col.p, A.col.p, sizeof(int32_t) * A.nnz, hipMemcpyDeviceToDevice, s));
            return;
        }
    }
    transpose(A.rowptr.p, A.col.p, A.val.p, A.n, A.n, A.nnz, true, T, s);
}

// ---- PMIS -------------------------------------------------------------------------
__device__ inline uint64_t splitmix64(uint64_t x) {
    // SplitMix64 (Steele, Lea & Flood 2014): golden-gamma increment, then the
    // variant-13 finaliser.
    uint64_t z = x + 0x9E3779B97F4A7C15ULL;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
    return z ^ (z >> 31);
}

__device__ inline bool key_gt(int32_t li, uint64_t hi, int32_t i, int32_t lj, uint64_t hj, int32_t j) {
    if (li != lj) return li > lj;
    if (hi != hj) return hi > hj;
    return i > j;
}

__global__ void __launch_bounds__(B)
k_pmis_init(int32_t n, const int32_t* __restrict__ STrowptr, int8_t* __restrict__ st) {
    int32_t i = blockIdx.x * B + threadIdx.x;
    if (i >= n) return;
    st[i] = (STrowptr[i + 1] - STrowptr[i]) == 0 ? (int8_t)-1 : (int8_t)0;
}

__global__ void __launch_bounds__(B)
k_pmis_select(int32_t n, uint64_t hseed, const int32_t* __restrict__ Srp, const int32_t* __restrict__ Sc,
              const int32_t* __restrict__ STrp, const int32_t* __restrict__ STc,
              const int8_t* __restrict__ old, int8_t* __restrict__ nxt) {
    int32_t i = blockIdx.x * B + threadIdx.x;
    if (i >= n) return;
    int8_t o = old[i];
    if (o != 0) { nxt[i] = o; return; }
    int32_t li = STrp[i + 1] - STrp[i];
    uint64_t hi = splitmix64(hseed ^ (uint64_t)i);
    bool isC = true;
    for (int32_t q = Srp[i]; q < Srp[i + 1] && isC; ++q) {
        int32_t j = Sc[q];
        if (old[j] == 0) {
            int32_t lj = STrp[j + 1] - STrp[j];
            if (!key_gt(li, hi, i, lj, splitmix64(hseed ^ (uint64_t)j), j)) isC = false;
        }
    }
    for (int32_t q = STrp[i]; q < STrp[i + 1] && isC; ++q) {
        int32_t j = STc[q];
        if (old[j] == 0) {
            int32_t lj = STrp[j + 1] - STrp[j];
            if (!key_gt(li, hi, i, lj, splitmix64(hseed ^ (uint64_t)j), j)) isC = false;
        }
    }
    nxt[i] = isC ? (int8_t)1 : (int8_t)0;
}

// undecided points with a strong C dependence become F; *undecided is set
// to 1 when some point stays undecided (a plain store by one lane of each
// such wavefront: a same-address atomic per wavefront serialised across
// the chip and cost up to 0.75 ms per round on 4M points)
__global__ void __launch_bounds__(B)
k_pmis_fmark(int32_t n, const int32_t* __restrict__ Srp, const int32_t* __restrict__ Sc,
             int8_t* st, int32_t* __restrict__ undecided) {
    const int32_t i = blockIdx.x * B + threadIdx.x;
    bool und = false;
    if (i < n && st[i] == 0) {
        und = true;
        for (int32_t q = Srp[i]; q < Srp[i + 1]; ++q)
            if (st[Sc[q]] == 1) {
                st[i] = -1;
                und = false;
                break;
            }
    }
    const uint64_t m = __ballot(und);  // (all lanes take part)
    if ((threadIdx.x & 63) == 0 && m) *undecided = 1;
}

__global__ void __launch_bounds__(B)
k_cf_flags(int32_t n, const int8_t* __restrict__ st, int32_t* __restrict__ cf) {
    int32_t i = blockIdx.x * B + threadIdx.x;
    if (i < n) cf[i] = st[i] == 1 ? 1 : 0;
}

// ---- extended+i interpolation -----------------------------------------------------------
// F point i interpolates from C^_i, its strong C neighbours and the strong C
// neighbours of its strong F neighbours (De Sterck, Falgout, Nolting, Yang,
// Numer. Linear Algebra Appl. 15, 2008).  C^_i is the pattern of row i of
// X Y with X(i,:) = {i} and the strong F neighbours of i (F rows only) and
// Y(k,:) = the strong C neighbours of k (F rows only), formed by the SpGEMM
// below (sorted columns).
__global__ void __launch_bounds__(B)
k_ext_xy_count(int32_t n, const int32_t* __restrict__ Srp, const int32_t* __restrict__ Sc,
               const int32_t* __restrict__ cf, int32_t* __restrict__ xc, int32_t* __restrict__ yc) {
    const int32_t i = blockIdx.x * B + threadIdx.x;
    if (i >= n) return;
    int32_t f = 0, c = 0;
    if (!cf[i]) {
        for (int32_t q = Srp[i]; q < Srp[i + 1]; ++q) {
            if (cf[Sc[q]]) ++c;
            else ++f;
        }
        ++f;  // i itself
    }
    xc[i] = f;
    yc[i] = c;
}

__global__ void __launch_bounds__(B)
k_ext_xy_fill(int32_t n, const int32_t* __restrict__ Srp, const int32_t* __restrict__ Sc,
              const int32_t* __restrict__ cf, const int32_t* __restrict__ Xrp, int32_t* __restrict__ Xc,
              double* __restrict__ Xv, const int32_t* __restrict__ Yrp, int32_t* __restrict__ Yc,
              double* __restrict__ Yv) {
    const int32_t i = blockIdx.x * B + threadIdx.x;
    if (i >= n || cf[i]) return;
    int32_t x = Xrp[i], y = Yrp[i];
    bool self = false;
    for (int32_t q = Srp[i]; q < Srp[i + 1]; ++q) {
        const int32_t j = Sc[q];
        if (!self && j > i) {  // keep X's row ascending
            Xc[x] = i;
            Xv[x++] = 1.0;
            self = true;
        }
        if (cf[j]) {
            Yc[y] = j;
            Yv[y++] = 1.0;
        } else {
            Xc[x] = j;
            Xv[x++] = 1.0;
        }
    }
    if (!self) {
        Xc[x] = i;
        Xv[x] = 1.0;
    }
}

__global__ void __launch_bounds__(B)
k_ext_count(int32_t n, const int32_t* __restrict__ cf, const int32_t* __restrict__ Trp, int pmax,
            int32_t* __restrict__ cnt) {
    const int32_t i = blockIdx.x * B + threadIdx.x;
    if (i >= n) return;
    const int32_t len = Trp[i + 1] - Trp[i];
    cnt[i] = cf[i] ? 1 : (pmax > 0 && len > pmax ? pmax : len);
}

constexpr int EXT_PMAX = 16;  // largest accepted interp_pmax

// index of x in the ascending v[0..len), or -1
__device__ inline int32_t find_sorted(const int32_t* __restrict__ v, int32_t len, int32_t x) {
    int32_t lo = 0, hi = len;
    while (lo < hi) {
        const int32_t mid = lo + (hi - lo) / 2;
        if (v[mid] < x) lo = mid + 1;
        else hi = mid;
    }
    return (lo < len && v[lo] == x) ? lo : -1;
}

__device__ inline double opposite(double a, double akk) { return (akk > 0.0 ? a < 0.0 : a > 0.0) ? a : 0.0; }

// Weights of row i: with den_k = sum of hat a_kl over l in C^_i and l = i
// for each strong F neighbour k (hat a_kl = a_kl where its sign is opposite
// to a_kk's, else 0),
//   a~_ii = a_ii + (weak couplings outside C^_i) + sum_k a_ik hat a_ki / den_k,
//   w_ij  = -(a_ij + sum_k a_ik hat a_kj / den_k) / a~_ii,
// summed in the row's column order, then k ascending over row k's order; a
// strong F neighbour with den_k = 0 is lumped like a weak one.
// Row i's weights are formed in w (scratch of the row's interpolatory-set
// length), then written to P, truncated as described at k_ext_fill_w.
// refresh != 0: P's pattern is frozen (a numeric refresh) -- a row shorter
// than its interpolatory set keeps its frozen columns instead of the pmax of
// largest magnitude, and only values are written.
__device__ void ext_row(int32_t i, const int32_t* __restrict__ rowptr, const int32_t* __restrict__ col,
                        const double* __restrict__ val, const int32_t* __restrict__ Srp,
                        const int32_t* __restrict__ Sc, const int32_t* __restrict__ cf,
                        const int32_t* __restrict__ cmap, const int32_t* __restrict__ Trp,
                        const int32_t* __restrict__ Tc, const int32_t* __restrict__ Prp, int32_t* __restrict__ Pc,
                        double* __restrict__ Pv, double* __restrict__ wbuf, int pmax, int refresh) {
    const int32_t p0 = Prp[i];
    if (cf[i]) {
        if (refresh) return;  // the unit row is kept
        Pc[p0] = cmap[i];
        Pv[p0] = 1.0;
        return;
    }
    const int32_t* list = Tc + Trp[i];
    const int32_t len = Trp[i + 1] - Trp[i];
    if (len == 0) return;
    const int32_t* Si = Sc + Srp[i];
    const int32_t slen = Srp[i + 1] - Srp[i];
    double* w = wbuf + Trp[i];
    for (int32_t t = 0; t < len; ++t) w[t] = 0.0;
    double aii = 0.0;
    for (int32_t t = rowptr[i]; t < rowptr[i + 1]; ++t)
        if (col[t] == i) aii = val[t];
    double at = aii;
    for (int32_t t = rowptr[i]; t < rowptr[i + 1]; ++t) {
        const int32_t j = col[t];
        if (j == i) continue;
        const int32_t pos = find_sorted(list, len, j);
        if (pos >= 0) w[pos] += val[t];
        else if (find_sorted(Si, slen, j) < 0) at += val[t];
    }
    for (int32_t t = rowptr[i]; t < rowptr[i + 1]; ++t) {
        const int32_t k = col[t];
        if (k == i || cf[k] || find_sorted(Si, slen, k) < 0) continue;
        const double aik = val[t];
        double akk = 0.0, den = 0.0;
        const int32_t kb = rowptr[k], ke = rowptr[k + 1];
        for (int32_t u = kb; u < ke; ++u)
            if (col[u] == k) akk = val[u];
        for (int32_t u = kb; u < ke; ++u) {
            const int32_t l = col[u];
            if (l == i || find_sorted(list, len, l) >= 0) den += opposite(val[u], akk);
        }
        if (den == 0.0) {
            at += aik;
            continue;
        }
        for (int32_t u = kb; u < ke; ++u) {
            const int32_t l = col[u];
            const double c = (aik * opposite(val[u], akk)) / den;
            const int32_t pos = find_sorted(list, len, l);
            if (pos >= 0) w[pos] += c;
            else if (l == i) at += c;
        }
    }
    for (int32_t t = 0; t < len; ++t) w[t] = -w[t] / at;
    if (refresh) {
        const int32_t plen = Prp[i + 1] - p0;
        if (plen >= len) {
            for (int32_t t = 0; t < len; ++t) Pv[p0 + t] = w[t];
            return;
        }
        double all = 0.0, kept = 0.0;
        for (int32_t t = 0; t < len; ++t) all += w[t];
        for (int32_t t = 0; t < len; ++t)
            if (find_sorted(Pc + p0, plen, cmap[list[t]]) >= 0) kept += w[t];
        const double f = kept != 0.0 ? all / kept : 1.0;
        int32_t r = 0;
        for (int32_t t = 0; t < len; ++t)
            if (find_sorted(Pc + p0, plen, cmap[list[t]]) >= 0) Pv[p0 + r++] = kept != 0.0 ? w[t] * f : w[t];
        return;
    }
    if (pmax > 0 && len > pmax) {
        int32_t sel[EXT_PMAX];
        for (int r = 0; r < pmax; ++r) {  // largest magnitude first, ties: smaller column
            int32_t best = -1;
            for (int32_t t = 0; t < len; ++t) {
                bool taken = false;
                for (int q = 0; q < r; ++q) taken |= sel[q] == t;
                if (!taken && (best < 0 || fabs(w[t]) > fabs(w[best]))) best = t;
            }
            sel[r] = best;
        }
        for (int r = 1; r < pmax; ++r)  // ascending column order
            for (int q = r; q > 0 && sel[q - 1] > sel[q]; --q) {
                const int32_t x = sel[q];
                sel[q] = sel[q - 1];
                sel[q - 1] = x;
            }
        double all = 0.0, kept = 0.0;
        for (int32_t t = 0; t < len; ++t) all += w[t];
        for (int r = 0; r < pmax; ++r) kept += w[sel[r]];
        const double f = kept != 0.0 ? all / kept : 1.0;
        for (int r = 0; r < pmax; ++r) {
            Pc[p0 + r] = cmap[list[sel[r]]];
            Pv[p0 + r] = kept != 0.0 ? w[sel[r]] * f : w[sel[r]];
        }
    } else {
        for (int32_t t = 0; t < len; ++t) {
            Pc[p0 + t] = cmap[list[t]];
            Pv[p0 + t] = w[t];
        }
    }
}

__global__ void __launch_bounds__(B)
k_ext_fill(int32_t n, const int32_t* __restrict__ rowptr, const int32_t* __restrict__ col,
           const double* __restrict__ val, const int32_t* __restrict__ Srp, const int32_t* __restrict__ Sc,
           const int32_t* __restrict__ cf, const int32_t* __restrict__ cmap, const int32_t* __restrict__ Trp,
           const int32_t* __restrict__ Tc, const int32_t* __restrict__ Prp, int32_t* __restrict__ Pc,
           double* __restrict__ Pv, double* __restrict__ wbuf, int pmax, int refresh) {
    const int32_t i = blockIdx.x * B + threadIdx.x;
    if (i < n) ext_row(i, rowptr, col, val, Srp, Sc, cf, cmap, Trp, Tc, Prp, Pc, Pv, wbuf, pmax, refresh);
}

// Wavefront-per-row form for levels of long rows.  Weight slot t of the row
// lives in a register of lane t mod 64, and that lane forms the slot's sum:
// the row's own coupling, then for each strong F neighbour k in the row's
// order the term of row k's entry in the slot's column, as the one-thread
// form adds them (the neighbours' rows are processed in chunks, see the
// loop).  a~_ii is a sum over the row: its terms are broadcast to the
// wavefront one by one in row order; each den_k is summed in row k's order
// by one lane.  So every slot, a~_ii and every den_k receive the same
// operations in the same order (identical results).  Rows of more than
// EXT_SLOTS slots take the one-thread form on lane 0.  Truncation (pmax > 0, longer rows): pmax rounds of a
// wavefront arg-max over (|w|, then the smaller slot) select the kept slots,
// the full and the kept sums run slot by slot in column order, and the kept
// weights, scaled by their ratio, are written in column order.  A refresh
// (frozen P pattern, see ext_row) marks the kept slots by membership in the
// row's frozen columns instead and writes values only.
constexpr int EXT_NW = 4;
constexpr int EXT_SLOTS = WR * EXT_NW;
// Chunk sizes: LDS per workgroup stays near 26 KB, so that six workgroups
// fit a CU, and the kernel is compiled for six wavefronts a SIMD (80
// registers; the row loops are latency-bound).  Measured on the 256x256x64
// pressure hierarchy (ms a setup): 4 wavefronts, 256-entry chunks, 9.4; 5
// wavefronts 8.3; 6 wavefronts with 192-entry chunks and strength rows up to
// 128 staged 8.0, with 128-entry chunks 8.4, 160-entry chunks 9.5 (five
// workgroups fit); 512-entry chunks were 25% slower than 256.  The term
// matrix holds a whole row's slots (a chunk always takes its first
// neighbour, and the slots' starting sums live there too): EXT_TC >= EXT_SLOTS.
constexpr int EXT_EC = 192;  // staged neighbour-row entries per chunk
constexpr int EXT_TC = 256;  // entries of the chunk's term matrix (neighbours x slots)
static_assert(EXT_TC >= EXT_SLOTS, "the term matrix must hold one neighbour's row of slots");
constexpr int EXT_KC = 16;   // neighbours per chunk
constexpr int EXT_SI = 128;  // strength rows up to this long are staged in LDS

__global__ void __launch_bounds__(B) __attribute__((amdgpu_waves_per_eu(6)))
k_ext_fill_w(int32_t n, const int32_t* __restrict__ rowptr, const int32_t* __restrict__ col,
             const double* __restrict__ val, const int32_t* __restrict__ Srp, const int32_t* __restrict__ Sc,
             const int32_t* __restrict__ cf, const int32_t* __restrict__ cmap, const int32_t* __restrict__ Trp,
             const int32_t* __restrict__ Tc, const int32_t* __restrict__ Prp, int32_t* __restrict__ Pc,
             double* __restrict__ Pv, double* __restrict__ wbuf, int pmax, int refresh) {
    const int32_t i = blockIdx.x * WR_ROWS + threadIdx.x / WR;
    const int lane = threadIdx.x % WR;
    if (i >= n) return;
    // The loads are grouped by what they depend on, so that each group is
    // one round trip: the row's extents; then its set, strong set and first
    // WR entries; then those entries' points' C/F flags and row extents.
    const int32_t p0 = Prp[i], ci = cf[i], ta = Trp[i], tb = Trp[i + 1], sa = Srp[i], sb = Srp[i + 1];
    const int32_t a = rowptr[i], e = rowptr[i + 1];
    if (ci) {
        if (lane == 0 && !refresh) {
            Pc[p0] = cmap[i];
            Pv[p0] = 1.0;
        }
        return;
    }
    const int32_t* list = Tc + ta;
    const int32_t len = tb - ta;
    if (len == 0) return;
    if (len > EXT_SLOTS) {
        if (lane == 0) ext_row(i, rowptr, col, val, Srp, Sc, cf, cmap, Trp, Tc, Prp, Pc, Pv, wbuf, pmax, refresh);
        return;
    }
    const int32_t* Si = Sc + sa;
    const int32_t slen = sb - sa;
    const bool ok0 = a + lane < e;
    const int32_t j0 = ok0 ? col[a + lane] : i;
    const double v0 = ok0 ? val[a + lane] : 0.0;
    // the row's interpolatory set in LDS (binary searches of the den sums)
    __shared__ int32_t s_list[WR_ROWS][EXT_SLOTS];
    // one chunk of strong F neighbours: their rows (columns, then slot
    // positions; values, then hat values), offsets, and per-row data
    __shared__ int32_t s_ec[WR_ROWS][EXT_EC];
    __shared__ double s_ev[WR_ROWS][EXT_EC];
    __shared__ double s_t[WR_ROWS][EXT_TC];  // T[k][slot]
    __shared__ int32_t s_ko[WR_ROWS][EXT_KC + 1], s_kb[WR_ROWS][EXT_KC], s_kk[WR_ROWS][EXT_KC],
        s_kf[WR_ROWS][EXT_KC];
    __shared__ double s_ka[WR_ROWS][EXT_KC], s_kd[WR_ROWS][EXT_KC], s_kn[WR_ROWS][EXT_KC], s_kt[WR_ROWS][EXT_KC];
    __shared__ int32_t s_si[WR_ROWS][EXT_SI];
    double* const s_w0 = s_t[threadIdx.x / WR];  // (the slots' starting sums, before T is used)
    const int wv = threadIdx.x / WR;
    int32_t* const sl = s_list[wv];
    for (int32_t t = lane; t < len; t += WR) {
        sl[t] = list[t];
        s_w0[t] = 0.0;
    }
    // row i's strong set in LDS when it fits (membership tests below)
    const bool si_lds = slen <= EXT_SI;
    if (si_lds)
        for (int32_t t = lane; t < slen; t += WR) s_si[wv][t] = Si[t];
    const int32_t* const si = si_lds ? s_si[wv] : Si;
    // (j0 = i on lanes past the row: a valid index)
    const int32_t cfj0 = cf[j0], kbj0 = rowptr[j0], kej0 = rowptr[j0 + 1];
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    // slot t = r * WR + lane lives in w[r] of its lane; its column, and that
    // column's coarse index (used at the end)
    int32_t lc[EXT_NW], lcm[EXT_NW];
#pragma unroll
    for (int r = 0; r < EXT_NW; ++r) lc[r] = r * WR + lane < len ? sl[r * WR + lane] : -1;
#pragma unroll
    for (int r = 0; r < EXT_NW; ++r) lcm[r] = lc[r] >= 0 ? cmap[lc[r]] : 0;
    // entry b + lane of row i (the first WR are held in registers)
    auto entry = [&](int32_t b, int32_t* j, double* v) {
        if (b == a) {
            *j = j0;
            *v = v0;
        } else {
            const bool ok = b + lane < e;
            *j = ok ? col[b + lane] : i;
            *v = ok ? val[b + lane] : 0.0;
        }
    };
    double aii = 0.0;
    bool has = false;
    for (int32_t b = a; b < e; b += WR) {
        int32_t j;
        double v;
        entry(b, &j, &v);
        if (b + lane < e && j == i) { aii = v; has = true; }
    }
    const uint64_t hm = __ballot(has);
    aii = hm ? bcast_d(aii, __ffsll((unsigned long long)hm) - 1) : 0.0;
    double at = aii;
    // The row's own couplings: a coupling in the set starts its slot's sum
    // (0.0 + a_ij, placed by the entry's lane: a row holds a column once);
    // weak couplings outside the set are lumped into a~_ii in row order.
    for (int32_t b = a; b < e; b += WR) {
        const bool ok = b + lane < e;
        int32_t j;
        double v;
        entry(b, &j, &v);
        const int32_t pos = j != i ? find_sorted(sl, len, j) : -1;
        if (pos >= 0) s_w0[pos] = 0.0 + v;
        const bool lump = ok && j != i && pos < 0 && find_sorted(si, slen, j) < 0;
        // the lumped terms in lane (row) order
        for (uint64_t lm = __ballot(lump); lm; lm &= lm - 1) at += bcast_d(v, __ffsll((unsigned long long)lm) - 1);
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    double w[EXT_NW];
#pragma unroll
    for (int r = 0; r < EXT_NW; ++r) w[r] = lc[r] >= 0 ? s_w0[r * WR + lane] : 0.0;
    // Strong F neighbours k in the row's order, in chunks.  A chunk's rows
    // are staged in LDS together (one pass of loads for all of them); for
    // all of them at once each row's diagonal, the values hat a_kl of its
    // entries with l in C^_i or l = i (0 for the others) and den_k, their
    // sum in row k's order, are formed; the terms a_ik hat a_kl / den_k go
    // to an LDS matrix T[k][slot] (+0.0 where row k lacks the slot's
    // column).  Then every slot adds its column of T over the chunk's k in
    // order, and a~_ii its terms likewise: each sum receives the terms of
    // the one-row-at-a-time form in the same order (adding +0.0 leaves these
    // sums, which are never -0.0, unchanged).  A neighbour row of more than
    // EXT_EC entries is a chunk of its own, read in place.
    auto wsync = [] {
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    };
    int32_t* const ko = s_ko[wv];
    int32_t* const ec = s_ec[wv];
    double* const ev = s_ev[wv];
    double* const tm = s_t[wv];
    // the chunk row that holds staged entry x
    auto owner = [&](int32_t cnt, int32_t x) -> int {
        int lo = 0, hi = cnt - 1;
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (ko[mid] <= x) lo = mid;
            else hi = mid - 1;
        }
        return lo;
    };
    // one strong F neighbour k (row kc/kv of length kl): its den_k, then its
    // terms to the slots and to a~_ii, the row's sums broadcast in order
    auto one_row = [&](int32_t k, double aik, const int32_t* kc, const double* kv, int32_t kl) {
        double akk = 0.0;
        bool hk = false;
        for (int32_t u = lane; u < kl; u += WR)
            if (kc[u] == k) { akk = kv[u]; hk = true; }
        const uint64_t km = __ballot(hk);
        akk = km ? bcast_d(akk, __ffsll((unsigned long long)km) - 1) : 0.0;
        double den = 0.0;
        for (int32_t c0 = 0; c0 < kl; c0 += WR) {
            const int32_t u = c0 + lane;
            const bool inr = u < kl;
            const int32_t lcu = inr ? kc[u] : -1;
            const bool mem = inr && (lcu == i || find_sorted(sl, len, lcu) >= 0);
            const double h = mem ? opposite(kv[u], akk) : 0.0;
            for (uint64_t mm2 = __ballot(mem); mm2; mm2 &= mm2 - 1)
                den += bcast_d(h, __ffsll((unsigned long long)mm2) - 1);
        }
        if (den == 0.0) {
            at += aik;
            return;
        }
#pragma unroll
        for (int r = 0; r < EXT_NW; ++r) {
            if (lc[r] < 0) continue;
            const int32_t u = find_sorted(kc, kl, lc[r]);
            if (u >= 0) w[r] += (aik * opposite(kv[u], akk)) / den;
        }
        const int32_t ui = find_sorted(kc, kl, i);
        if (ui >= 0) at += (aik * opposite(kv[ui], akk)) / den;
    };
    for (int32_t b = a; b < e; b += WR) {
        const bool ok = b + lane < e;
        int32_t k0;
        double v;
        entry(b, &k0, &v);
        int32_t cfk, kbk, kek;
        if (b == a) {
            cfk = cfj0;
            kbk = kbj0;
            kek = kej0;
        } else {
            cfk = cf[k0];
            kbk = rowptr[k0];
            kek = rowptr[k0 + 1];
        }
        const bool sf = ok && k0 != i && !cfk && find_sorted(si, slen, k0) >= 0;
        const int32_t kb0 = sf ? kbk : 0, ke0 = sf ? kek : 0;
        const double aik0 = sf ? v : 0.0;
        const int32_t kl0 = ke0 - kb0;
        uint64_t m = __ballot(sf);
        while (m) {
            uint64_t cm = 0;  // the chunk: the next neighbours while they fit
            int cnt = 0;
            int32_t tot = 0;
            for (uint64_t mm = m; mm; mm &= mm - 1) {
                const int l = __ffsll((unsigned long long)mm) - 1;
                const int32_t kl = bcast_i(kl0, l);
                if (cnt > 0 && (tot + kl > EXT_EC || cnt == EXT_KC || (cnt + 1) * len > EXT_TC)) break;
                cm |= 1ull << l;
                ++cnt;
                tot += kl;
                if (kl > EXT_EC) break;
            }
            m &= ~cm;
            if (tot > EXT_EC) {  // one long neighbour row, read in place
                const int l = __ffsll((unsigned long long)cm) - 1;
                const int32_t kb = bcast_i(kb0, l);
                one_row(bcast_i(k0, l), bcast_d(aik0, l), col + kb, val + kb, bcast_i(kl0, l));
                continue;
            }
            const bool in = (cm >> lane) & 1ull;
            const int kx = __popcll(cm & ((1ull << lane) - 1ull));
            int32_t inc = in ? kl0 : 0;  // inclusive scan of the rows' lengths
#pragma unroll
            for (int d = 1; d < WR; d <<= 1) {
                const int32_t o = __shfl_up(inc, d, WR);
                if (lane >= d) inc += o;
            }
            if (in) {
                ko[kx] = inc - kl0;
                s_kb[wv][kx] = kb0;
                s_kk[wv][kx] = k0;
                s_ka[wv][kx] = aik0;
                s_kd[wv][kx] = 0.0;
                s_kf[wv][kx] = 0;
            }
            if (lane == 0) ko[cnt] = tot;
            wsync();
            for (int32_t x = lane; x < tot; x += WR) {  // stage the rows
                const int kk = owner(cnt, x);
                const int32_t src = s_kb[wv][kk] + (x - ko[kk]);
                ec[x] = col[src];
                ev[x] = val[src];
            }
            for (int32_t x = lane; x < cnt * len; x += WR) tm[x] = 0.0;
            wsync();
            for (int32_t x = lane; x < tot; x += WR) {  // each row's diagonal (a row holds it once)
                const int kk = owner(cnt, x);
                if (ec[x] == s_kk[wv][kk]) s_kd[wv][kk] = ev[x];
            }
            wsync();
            for (int32_t x = lane; x < tot; x += WR) {  // hat values; slot positions (-2: column i)
                const int kk = owner(cnt, x);
                const int32_t l = ec[x];
                const int32_t pos = l == i ? -2 : find_sorted(sl, len, l);
                ev[x] = pos != -1 ? opposite(ev[x], s_kd[wv][kk]) : 0.0;
                ec[x] = pos;
            }
            wsync();
            if (in) {  // den_k over row k in its order
                double den = 0.0;
                for (int32_t x = ko[kx]; x < ko[kx + 1]; ++x) den += ev[x];
                s_kn[wv][kx] = den;
            }
            wsync();
            for (int32_t x = lane; x < tot; x += WR) {  // the terms
                const int kk = owner(cnt, x);
                const double den = s_kn[wv][kk];
                const int32_t pos = ec[x];
                if (den != 0.0 && pos != -1) {
                    const double c = (s_ka[wv][kk] * ev[x]) / den;
                    if (pos >= 0) {
                        tm[kk * len + pos] = c;
                    } else {
                        s_kt[wv][kk] = c;
                        s_kf[wv][kk] = 1;
                    }
                }
            }
            wsync();
            for (int kk = 0; kk < cnt; ++kk) {  // the sums, k in order
                if (s_kn[wv][kk] == 0.0) {
                    at += s_ka[wv][kk];
                    continue;
                }
#pragma unroll
                for (int r = 0; r < EXT_NW; ++r)
                    if (lc[r] >= 0) w[r] += tm[kk * len + r * WR + lane];
                if (s_kf[wv][kk]) at += s_kt[wv][kk];
            }
            wsync();  // (the next chunk reuses the arrays)
        }
    }
#pragma unroll
    for (int r = 0; r < EXT_NW; ++r) w[r] = -w[r] / at;
    const int32_t plen = Prp[i + 1] - p0;
    if (refresh ? plen >= len : !(pmax > 0 && len > pmax)) {
#pragma unroll
        for (int r = 0; r < EXT_NW; ++r) {
            const int32_t t = r * WR + lane;
            if (t < len) {
                if (!refresh) Pc[p0 + t] = lcm[r];
                Pv[p0 + t] = w[r];
            }
        }
        return;
    }
    unsigned selm = 0;  // bit r: slot r * WR + lane kept
    if (refresh) {
#pragma unroll
        for (int r = 0; r < EXT_NW; ++r)
            if (lc[r] >= 0 && find_sorted(Pc + p0, plen, lcm[r]) >= 0) selm |= 1u << r;
    }
    if (!refresh) {
        // slot t is kept when fewer than pmax slots precede it in the order
        // (|w| descending, then slot ascending) -- the slots that pmax rounds
        // of an arg-max over that order would pick; each slot's rank is
        // counted over the broadcast magnitudes of all slots
        double aw[EXT_NW];
        int32_t rank[EXT_NW];
#pragma unroll
        for (int r = 0; r < EXT_NW; ++r) {
            aw[r] = fabs(w[r]);
            rank[r] = 0;
        }
#pragma unroll
        for (int r2 = 0; r2 < EXT_NW; ++r2) {
            if (r2 * WR >= len) continue;  // (uniform)
            const int cnt = min(WR, (int)(len - r2 * WR));
            for (int l = 0; l < cnt; ++l) {
                const double au = bcast_d(aw[r2], l);
                const int32_t u = r2 * WR + l;
#pragma unroll
                for (int r = 0; r < EXT_NW; ++r) {
                    if (r * WR >= len) continue;  // (uniform)
                    if (au > aw[r] || (au == aw[r] && u < r * WR + lane)) ++rank[r];
                }
            }
        }
#pragma unroll
        for (int r = 0; r < EXT_NW; ++r)
            if (r * WR + lane < len && rank[r] < pmax) selm |= 1u << r;
    }
    double all = 0.0, kept = 0.0;
    int32_t below = 0;  // kept slots before this lane's, register by register
#pragma unroll
    for (int r = 0; r < EXT_NW; ++r) {
        const int cnt = min(WR, (int)(len - r * WR));
        for (int l = 0; l < cnt; ++l) {
            const double v = bcast_d(w[r], l);
            const bool k = (bcast_i((int)selm, l) >> r) & 1;
            all += v;
            if (k) kept += v;
        }
    }
    const double f = kept != 0.0 ? all / kept : 1.0;
#pragma unroll
    for (int r = 0; r < EXT_NW; ++r) {
        const bool k = (selm >> r) & 1u;
        const uint64_t km = __ballot(k);
        if (k) {
            const int32_t pos = below + __popcll(km & ((1ull << lane) - 1ull));
            if (!refresh) Pc[p0 + pos] = lcm[r];
            Pv[p0 + pos] = kept != 0.0 ? w[r] * f : w[r];
        }
        below += __popcll(km);
    }
}

// ---- SpGEMM C = A B with an LDS hash per row --------------------------------------------
constexpr int HASH = 2048;
constexpr int HASH_LOG = 11;
constexpr int SG_WAVE = 64;

// Table size for one row: a power of two >= twice the product count
// (bounded by HASH); rows with more distinct columns than HASH overflow.
__device__ inline int row_table_log(const int32_t* Arp, const int32_t* Ac, const int32_t* Brp, int32_t i,
                                    int32_t* sh_bound) {
    int32_t b = 0;
    for (int32_t kk = Arp[i] + threadIdx.x; kk < Arp[i + 1]; kk += SG_WAVE) {
        int32_t r = Ac[kk];
        b += Brp[r + 1] - Brp[r];
    }
    for (int off = 32; off > 0; off >>= 1) b += __shfl_down(b, off, 64);
    if (threadIdx.x == 0) *sh_bound = b;
    __syncthreads();
    b = *sh_bound;
    int lg = 6;
    while (lg < HASH_LOG && (1 << lg) < 2 * b) ++lg;
    return lg;
}

__device__ inline int32_t hslot(int32_t c, int lg) {
    return (int32_t)(((uint32_t)c * 2654435761u) >> (32 - lg));
}

// Insert the column set of row i of A*B into tab (size 1 << lg).
__device__ inline void sg_insert_row(const int32_t* Arp, const int32_t* Ac, const int32_t* Brp,
                                     const int32_t* Bc, int32_t i, int32_t* tab, int lg, int32_t* count,
                                     int32_t* overflow) {
    const int32_t mask = (1 << lg) - 1;
    for (int32_t kk = Arp[i] + threadIdx.x; kk < Arp[i + 1]; kk += SG_WAVE) {
        int32_t r = Ac[kk];
        for (int32_t q = Brp[r]; q < Brp[r + 1]; ++q) {
            int32_t c = Bc[q];
            int32_t h = hslot(c, lg);
            int probes = 0;
            while (true) {
                int32_t old = atomicCAS(&tab[h], -1, c);
                if (old == -1) { atomicAdd(count, 1); break; }
                if (old == c) break;
                h = (h + 1) & mask;
                if (++probes > mask) { *overflow = 1; break; }
            }
        }
    }
}

// The two kernels below take the rows listed in rows[0 .. *nrows) (the rows
// the short-row path handed over).
__global__ void __launch_bounds__(SG_WAVE)
k_spgemm_count(const int32_t* __restrict__ rows, const int32_t* __restrict__ nrows,
               const int32_t* __restrict__ Arp, const int32_t* __restrict__ Ac,
               const int32_t* __restrict__ Brp, const int32_t* __restrict__ Bc,
               int32_t* __restrict__ cnt, int32_t* __restrict__ gflag) {
    __shared__ int32_t tab[HASH];
    __shared__ int32_t count, overflow, bound;
    const int32_t nr = *nrows;
    for (int32_t idx = blockIdx.x; idx < nr; idx += gridDim.x) {
        const int32_t i = rows[idx];
        const int lg = row_table_log(Arp, Ac, Brp, i, &bound);
        for (int h = threadIdx.x; h < (1 << lg); h += SG_WAVE) tab[h] = -1;
        if (threadIdx.x == 0) { count = 0; overflow = 0; }
        __syncthreads();
        sg_insert_row(Arp, Ac, Brp, Bc, i, tab, lg, &count, &overflow);
        __syncthreads();
        if (threadIdx.x == 0) {
            cnt[i] = count;
            if (overflow) *gflag = 1;
        }
        __syncthreads();
    }
}

__global__ void __launch_bounds__(SG_WAVE)
k_spgemm_fill(const int32_t* __restrict__ rows, const int32_t* __restrict__ nrows,
              const int32_t* __restrict__ Arp, const int32_t* __restrict__ Ac,
              const double* __restrict__ Av, const int32_t* __restrict__ Brp,
              const int32_t* __restrict__ Bc, const double* __restrict__ Bv,
              const int32_t* __restrict__ Crp, int32_t* __restrict__ Cc, double* __restrict__ Cv,
              int32_t* __restrict__ gflag) {
    __shared__ int32_t tab[HASH];
    __shared__ int32_t list[HASH];
    __shared__ int32_t count, overflow, ncomp, bound;
    const int32_t nr = *nrows;
    for (int32_t idx = blockIdx.x; idx < nr; idx += gridDim.x) {
        const int32_t i = rows[idx];
        const int lg = row_table_log(Arp, Ac, Brp, i, &bound);
        for (int h = threadIdx.x; h < (1 << lg); h += SG_WAVE) tab[h] = -1;
        if (threadIdx.x == 0) { count = 0; overflow = 0; ncomp = 0; }
        __syncthreads();
        sg_insert_row(Arp, Ac, Brp, Bc, i, tab, lg, &count, &overflow);
        __syncthreads();
        if (overflow) {
            // keep the row's slots valid (column 0, value 0) for the kernels
            // that follow; the flag fails the setup at its end
            for (int32_t q = Crp[i] + threadIdx.x; q < Crp[i + 1]; q += SG_WAVE) {
                Cc[q] = 0;
                Cv[q] = 0.0;
            }
            if (threadIdx.x == 0) *gflag = 1;
            __syncthreads();
            continue;
        }
        // compact the keys
        for (int h = threadIdx.x; h < (1 << lg); h += SG_WAVE) {
            int32_t c = tab[h];
            if (c != -1) list[atomicAdd(&ncomp, 1)] = c;
        }
        __syncthreads();
        const int32_t u = ncomp;
        const int32_t base = Crp[i];
        if (u != Crp[i + 1] - base) {  // must equal the symbolic count
            for (int32_t q = base + threadIdx.x; q < Crp[i + 1]; q += SG_WAVE) {
                Cc[q] = 0;
                Cv[q] = 0.0;
            }
            if (threadIdx.x == 0) *gflag = 2;
            __syncthreads();
            continue;
        }
        // rank sort into tab[0..u)
        for (int32_t e = threadIdx.x; e < u; e += SG_WAVE) {
            int32_t key = list[e], rank = 0;
            for (int32_t x = 0; x < u; ++x) rank += list[x] < key;
            tab[rank] = key;
        }
        __syncthreads();
        // one lane per output entry: sum over k ascending (the row of A is sorted)
        for (int32_t e = threadIdx.x; e < u; e += SG_WAVE) {
            int32_t c = tab[e];
            double acc = 0.0;
            for (int32_t kk = Arp[i]; kk < Arp[i + 1]; ++kk) {
                int32_t r = Ac[kk];
                int32_t lo = Brp[r], hi = Brp[r + 1] - 1;
                while (lo <= hi) {
                    int32_t mid = (lo + hi) >> 1;
                    int32_t v = Bc[mid];
                    if (v == c) { acc += Av[kk] * Bv[mid]; break; }
                    if (v < c) lo = mid + 1; else hi = mid - 1;
                }
            }
            Cc[base + e] = c;
            Cv[base + e] = acc;
        }
        __syncthreads();
    }
}

// list[0 .. n) = 0 .. n-1 and *count = n
__global__ void __launch_bounds__(B)
k_iota_i32(int32_t n, int32_t* __restrict__ list, int32_t* __restrict__ count) {
    const int32_t i = blockIdx.x * B + threadIdx.x;
    if (i < n) list[i] = i;
    if (i == 0) *count = n;
}

// ---- long rows: a workgroup per output row ------------------------------------------------
// The rows the short path hands over (more A entries than its lane group, or
// more products than it sorts).  A workgroup of LG_T threads takes a row:
// the B-row lengths of its A entries are scanned into first-product slots,
// every thread loads product slots e, e + LG_T, ... (slot e belongs to the
// last A entry whose first slot is <= e) and inserts the column into the
// LDS hash table (a slot already holding the column is seen by a plain
// read; only an empty slot takes an atomic).  The numeric pass sorts the
// distinct columns (rank sort), then sends every product a_iq b_qc to
// M[p][q], p the output position of c (binary search in the sorted
// columns), in LDS -- each A entry's B row holds a column at most once, and
// absent pairs hold +0.0 -- and sums each output's row of M over q
// ascending from +0.0.  That is the sum of the hash-table kernels above, in
// their order (a +0.0 term never changes a sum that starts at +0.0), so the
// values are identical.  Rows whose M would exceed LG_M entries search the
// B rows in global memory instead, as those kernels do; rows with more than
// LA_MAX A entries are listed for them.
constexpr int LG_T = 256;
constexpr int LG_W = LG_T / 64;
constexpr int LG_M = 2048;
constexpr int LA_MAX = 128;

// exclusive prefix of v over the workgroup (thread order) and the total
__device__ inline int32_t block_exscan(int32_t v, int32_t* s_wave, int32_t* total) {
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    int32_t inc = v;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        const int32_t o = __shfl_up(inc, d, 64);
        if (lane >= d) inc += o;
    }
    if (lane == 63) s_wave[w] = inc;
    __syncthreads();
    int32_t before = 0, all = 0;
    for (int q = 0; q < LG_W; ++q) {
        if (q < w) before += s_wave[q];
        all += s_wave[q];
    }
    __syncthreads();
    *total = all;
    return before + inc - v;
}

// index of the last A entry whose first product slot is <= e
__device__ inline int32_t owner_entry(const int32_t* s_off, int32_t la, int32_t e) {
    int32_t lo = 0, hi = la - 1;
    while (lo < hi) {
        const int32_t mid = (lo + hi + 1) >> 1;
        if (s_off[mid] <= e) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

// insert c into the open-addressed table (size mask + 1); counts new keys
__device__ inline void lg_insert(int32_t* tab, int32_t c, int lg, int32_t mask, int32_t* count,
                                 int32_t* overflow) {
    int32_t hh = hslot(c, lg);
    int probes = 0;
    while (true) {
        const int32_t cur = __hip_atomic_load(&tab[hh], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
        if (cur == c) return;
        if (cur == -1) {
            const int32_t old = atomicCAS(&tab[hh], -1, c);
            if (old == -1) {
                atomicAdd(count, 1);
                return;
            }
            if (old == c) return;
        }
        hh = (hh + 1) & mask;
        if (++probes > mask) {
            *overflow = 1;
            return;
        }
    }
}

// (six workgroups a CU: the LDS allows six, and 80 registers a lane keep
// the numeric pass unspilled; 16% faster than the five that 92 registers gave)
template <bool NUMERIC>
__global__ void __launch_bounds__(LG_T) __attribute__((amdgpu_waves_per_eu(6)))
k_spgemm_long(const int32_t* __restrict__ rows, const int32_t* __restrict__ nrows,
              const int32_t* __restrict__ Arp, const int32_t* __restrict__ Ac, const double* __restrict__ Av,
              const int32_t* __restrict__ Brp, const int32_t* __restrict__ Bc, const double* __restrict__ Bv,
              int32_t* __restrict__ cnt, const int32_t* __restrict__ Crp, int32_t* __restrict__ Cc,
              double* __restrict__ Cv, int32_t* __restrict__ vlong, int32_t* __restrict__ nvlong,
              int32_t* __restrict__ gflag) {
    __shared__ int32_t tab[HASH];
    // the compacted keys (before the sort) and M (after it) share this space
    __shared__ double s_m[NUMERIC ? (LG_M > HASH / 2 ? LG_M : HASH / 2) : 1];
    int32_t* const list = reinterpret_cast<int32_t*>(s_m);
    __shared__ int32_t s_off[LA_MAX + 1];
    __shared__ int32_t s_b0[LA_MAX];
    __shared__ double s_av[NUMERIC ? LA_MAX : 1];
    __shared__ int32_t s_wave[LG_W];
    __shared__ int32_t count, overflow, ncomp;
    constexpr int LG_U = 4;  // products a thread loads before it uses them
    const int t = threadIdx.x;
    const int32_t nr = *nrows;
    for (int32_t idx = blockIdx.x; idx < nr; idx += gridDim.x) {
        const int32_t i = rows[idx];
        const int32_t a0 = Arp[i], la = Arp[i + 1] - a0;
        if (la > LA_MAX) {  // (uniform across the workgroup)
            if (t == 0) vlong[atomicAdd(nvlong, 1)] = i;
            continue;
        }
        // entries 2t, 2t + 1: B-row starts and lengths, scanned into first slots
        int32_t len2[2] = {0, 0};
#pragma unroll
        for (int k = 0; k < 2; ++k) {
            const int32_t q = 2 * t + k;
            if (q < la) {
                const int32_t r = Ac[a0 + q];
                const int32_t b0 = Brp[r];
                s_b0[q] = b0;
                len2[k] = Brp[r + 1] - b0;
                if (NUMERIC) s_av[q] = Av[a0 + q];
            }
        }
        int32_t total = 0;
        const int32_t ex = block_exscan(len2[0] + len2[1], s_wave, &total);
        if (2 * t < la) s_off[2 * t] = ex;
        if (2 * t + 1 < la) s_off[2 * t + 1] = ex + len2[0];
        if (t == 0) {
            s_off[la] = total;
            count = 0;
            overflow = 0;
            ncomp = 0;
        }
        int lg = 6;
        while (lg < HASH_LOG && (1 << lg) < 2 * total) ++lg;
        const int32_t mask = (1 << lg) - 1;
        for (int h = t; h < (1 << lg); h += LG_T) tab[h] = -1;
        __syncthreads();
        for (int32_t e0 = t; e0 < total; e0 += LG_U * LG_T) {
            int32_t cc[LG_U];
#pragma unroll
            for (int u = 0; u < LG_U; ++u) {
                const int32_t e = e0 + u * LG_T;
                cc[u] = -1;
                if (e < total) {
                    const int32_t q = owner_entry(s_off, la, e);
                    cc[u] = Bc[s_b0[q] + (e - s_off[q])];
                }
            }
#pragma unroll
            for (int u = 0; u < LG_U; ++u)
                if (e0 + u * LG_T < total) lg_insert(tab, cc[u], lg, mask, &count, &overflow);
        }
        __syncthreads();
        if (!NUMERIC) {
            if (t == 0) {
                cnt[i] = count;
                if (overflow) *gflag = 1;
            }
            __syncthreads();
            continue;
        }
        const int32_t base = Crp[i];
        if (overflow || count != Crp[i + 1] - base) {
            // keep the row's slots valid (column 0, value 0) for the kernels
            // that follow; the flag fails the setup at its end
            for (int32_t q = base + t; q < Crp[i + 1]; q += LG_T) {
                Cc[q] = 0;
                Cv[q] = 0.0;
            }
            if (t == 0) *gflag = overflow ? 1 : 2;
            __syncthreads();
            continue;
        }
        for (int h = t; h < (1 << lg); h += LG_T) {
            const int32_t c = tab[h];
            if (c != -1) list[atomicAdd(&ncomp, 1)] = c;
        }
        __syncthreads();
        const int32_t u = ncomp;
        for (int32_t e = t; e < u; e += LG_T) {  // rank sort into tab[0 .. u)
            const int32_t key = list[e];
            int32_t rank = 0;
            for (int32_t x = 0; x < u; ++x) rank += list[x] < key;
            tab[rank] = key;
        }
        __syncthreads();  // (list is read until here; M takes its space)
        // The A entries in chunks of qc, each chunk's products placed in
        // the LDS product matrix M[e][q - q0] (+0.0 where row q of B lacks
        // column e) and added to the entries' sums chunk after chunk: every
        // output entry is summed over q ascending from 0.0, as in the
        // one-pass form (adding +0.0 leaves a sum that is never -0.0
        // unchanged).
        const int32_t qc = u > 0 ? max(1, LG_M / u) : la;
        constexpr int LG_E = HASH / LG_T;  // output entries per thread
        double acc[LG_E];
#pragma unroll
        for (int j = 0; j < LG_E; ++j) acc[j] = 0.0;
        for (int32_t q0 = 0; q0 < la; q0 += qc) {
            const int32_t q1 = min(la, q0 + qc), wq = q1 - q0;
            for (int32_t m = t; m < u * wq; m += LG_T) s_m[m] = 0.0;
            __syncthreads();
            const int32_t e_end = s_off[q1];
            for (int32_t e0 = s_off[q0] + t; e0 < e_end; e0 += LG_U * LG_T) {
                int32_t cc[LG_U], qq[LG_U];
                double vv[LG_U];
#pragma unroll
                for (int uu = 0; uu < LG_U; ++uu) {
                    const int32_t e = e0 + uu * LG_T;
                    qq[uu] = -1;
                    if (e < e_end) {
                        const int32_t q = owner_entry(s_off, la, e);
                        const int32_t src = s_b0[q] + (e - s_off[q]);
                        qq[uu] = q;
                        cc[uu] = Bc[src];
                        vv[uu] = s_av[q] * Bv[src];
                    }
                }
#pragma unroll
                for (int uu = 0; uu < LG_U; ++uu) {
                    if (qq[uu] < 0) continue;
                    int32_t lo = 0, hi = u - 1;  // the column's output position
                    while (lo < hi) {
                        const int32_t mid = (lo + hi) >> 1;
                        if (tab[mid] < cc[uu]) lo = mid + 1;
                        else hi = mid;
                    }
                    s_m[lo * wq + (qq[uu] - q0)] = vv[uu];
                }
            }
            __syncthreads();
#pragma unroll
            for (int j = 0; j < LG_E; ++j) {
                const int32_t e = t + j * LG_T;
                if (e < u)
                    for (int32_t q = 0; q < wq; ++q) acc[j] += s_m[e * wq + q];
            }
            __syncthreads();
        }
#pragma unroll
        for (int j = 0; j < LG_E; ++j) {
            const int32_t e = t + j * LG_T;
            if (e < u) {
                Cc[base + e] = tab[e];
                Cv[base + e] = acc[j];
            }
        }
        __syncthreads();
    }
}

// ---- short rows: a lane group per output row ---------------------------------------------
// A row with at most SR_G entries whose products number at most SR_MAX is
// expanded into LDS in A-entry-major order (inner index ascending, and within
// it B's sorted columns): product e has column c_e and value a_ik b_kc.  The
// keys c_e * SR_MAX + e are sorted in LDS by a bitonic network (padded to a
// power of two), which groups each column's products in ascending e.  A
// column's output position is the number of distinct smaller columns (heads
// of the sorted runs before it); its value is the sum of its products in
// ascending e from 0, i.e. in ascending inner index, the order of the
// hash-table path.  The row's columns and values go to its staging offset
// Crp[i], their count to cnt[i].  Other rows are appended to a list for the
// long-row kernels.  Products with long rows (coarse levels, the Galerkin product)
// take 64-lane groups with room for 256 products; the fine-level A P takes
// 16 lanes, 128 products, or 64 when the mean product count is at most 24
// (half the LDS: eight wavefronts a SIMD instead of five).  All give the same
// values, in the same order.
// The keys need c < 2^31 / SR_MAX (the caller sends every row of a wider B
// to the long-row kernels).
constexpr int SR_T = 256;

template <int SR_G, int SR_MAX>
__global__ void __launch_bounds__(SR_T)
k_spgemm_short(int32_t n, const int32_t* __restrict__ Arp, const int32_t* __restrict__ Ac,
               const double* __restrict__ Av, const int32_t* __restrict__ Brp, const int32_t* __restrict__ Bc,
               const double* __restrict__ Bv, int32_t* __restrict__ cnt, const int32_t* __restrict__ Crp,
               int32_t* __restrict__ Cc, double* __restrict__ Cv, int32_t* __restrict__ long_rows,
               int32_t* __restrict__ nlong) {
    constexpr int SR_ROWS = SR_T / SR_G;
    constexpr int SHIFT = __builtin_ctz(SR_MAX);  // key = c << SHIFT | e
    __shared__ uint32_t s_k[SR_ROWS][SR_MAX];
    __shared__ double s_v[SR_ROWS][SR_MAX];
    __shared__ int32_t s_off[SR_ROWS][SR_G];  // per A entry: first product slot, B-row start, value
    __shared__ int32_t s_b0[SR_ROWS][SR_G];
    __shared__ double s_av[SR_ROWS][SR_G];
    const int g = threadIdx.x / SR_G, lane = threadIdx.x % SR_G;
    const int32_t i = blockIdx.x * SR_ROWS + g;
    const bool valid = i < n;
    const int32_t a0 = valid ? Arp[i] : 0, la = valid ? Arp[i + 1] - a0 : 0;
    // this lane's inner index and its B row
    int32_t b0 = 0, lb = 0;
    double av = 0.0;
    if (lane < la && la <= SR_G) {
        const int32_t r = Ac[a0 + lane];
        b0 = Brp[r];
        lb = Brp[r + 1] - b0;
        av = Av[a0 + lane];
    }
    // exclusive scan of the B-row lengths across the row's lanes
    int32_t off = lb;
#pragma unroll
    for (int d = 1; d < SR_G; d <<= 1) {
        const int32_t o = __shfl_up(off, d, SR_G);
        if (lane >= d) off += o;
    }
    const int32_t total = __shfl(off, SR_G - 1, SR_G);
    off -= lb;
    const bool is_short = valid && la <= SR_G && total <= SR_MAX;
    if (valid && !is_short) {
        if (lane == 0) long_rows[atomicAdd(nlong, 1)] = i;
        return;  // the whole group leaves together (uniform across its lanes)
    }
    if (!valid) return;
    // Expansion, product slot e on lane e mod SR_G: its A entry t is the last
    // one whose first slot is <= e (entries with empty B rows share their
    // successor's first slot and are never the last such one), and its
    // product is B's entry e - off_t of that row.  Every lane loads its own
    // slots, so the row's loads are in flight together.
    if (lane < la) {
        s_off[g][lane] = off;
        s_b0[g][lane] = b0;
        s_av[g][lane] = av;
    }
    int np = 2;  // sorted length: a power of two >= total
    while (np < total) np <<= 1;
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    for (int32_t e = lane; e < np; e += SR_G) {
        if (e >= total) {
            s_k[g][e] = 0xFFFFFFFFu;
            continue;
        }
        int32_t lo = 0, hi = la - 1;
        while (lo < hi) {
            const int32_t mid = (lo + hi + 1) >> 1;
            if (s_off[g][mid] <= e) lo = mid;
            else hi = mid - 1;
        }
        const int32_t src = s_b0[g][lo] + (e - s_off[g][lo]);
        s_k[g][e] = ((uint32_t)Bc[src] << SHIFT) | (uint32_t)e;
        s_v[g][e] = s_av[g][lo] * Bv[src];
    }
    // bitonic sort of the np keys, ascending: stage (size 2^ls, stride 2^lt)
    // compares the pairs (lo, lo + stride), lo = pair index pi with a zero
    // bit inserted at position lt
    for (int ls = 1; (1 << ls) <= np; ++ls) {
        for (int lt = ls - 1; lt >= 0; --lt) {
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
            for (int pi = lane; pi < np / 2; pi += SR_G) {
                const int lo = ((pi >> lt) << (lt + 1)) | (pi & ((1 << lt) - 1));
                const int hi = lo + (1 << lt);
                const uint32_t x = s_k[g][lo], y = s_k[g][hi];
                const bool up = (lo & (1 << ls)) == 0;
                if ((x > y) == up) {
                    s_k[g][lo] = y;
                    s_k[g][hi] = x;
                }
            }
        }
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    // heads of the column runs, counted round by round (lanes of one round
    // hold consecutive sorted elements)
    const int gshift = (int)((threadIdx.x % 64) / SR_G) * SR_G;  // the group's first lane in its wavefront
    const uint64_t gmask = SR_G == 64 ? ~0ull : ((1ull << SR_G) - 1ull) << gshift;
    int32_t heads_before = 0;
    const int32_t base = Crp[i];
    for (int32_t e0 = 0; e0 < total; e0 += SR_G) {
        const int32_t e = e0 + lane;
        const bool in = e < total;
        const uint32_t key = in ? s_k[g][e] : 0u;
        const uint32_t c = key >> SHIFT;
        const bool head = in && (e == 0 || (s_k[g][e - 1] >> SHIFT) != c);
        const uint64_t hm = __ballot(head) & gmask;
        if (head) {
            const int32_t pos = heads_before + __popcll(hm & ((1ull << (threadIdx.x % 64)) - 1ull));
            double acc = 0.0;
            for (int32_t e2 = e; e2 < total; ++e2) {
                const uint32_t k2 = s_k[g][e2];
                if ((k2 >> SHIFT) != c) break;
                acc += s_v[g][k2 & (SR_MAX - 1)];
            }
            Cc[base + pos] = (int32_t)c;
            Cv[base + pos] = acc;
        }
        heads_before += __popcll(hm);
    }
    if (lane == 0) cnt[i] = heads_before;
}

// Staging offsets of the short path: ub[i] = the row's product count when
// k_spgemm_short<SR_G, SR_MAX> takes it (at most SR_G A entries and SR_MAX
// products), else 0.  (Its distinct columns number at most that.)
template <int SR_G, int SR_MAX>
__global__ void __launch_bounds__(B)
k_spgemm_ub(int32_t n, const int32_t* __restrict__ Arp, const int32_t* __restrict__ Ac,
            const int32_t* __restrict__ Brp, int32_t* __restrict__ ub) {
    const int32_t i = blockIdx.x * B + threadIdx.x;
    if (i >= n) return;
    const int32_t a0 = Arp[i], la = Arp[i + 1] - a0;
    int32_t total = 0;
    if (la <= SR_G)
        for (int32_t q = 0; q < la; ++q) {
            const int32_t r = Ac[a0 + q];
            total += Brp[r + 1] - Brp[r];
        }
    ub[i] = (la <= SR_G && total <= SR_MAX) ? total : 0;
}

// C's rows from the short path's staging (rows of nonzero staging length;
// the long rows were written in place), SR_C lanes a row
constexpr int SR_C = 16;
__global__ void __launch_bounds__(B)
k_spgemm_compact(int32_t n, const int32_t* __restrict__ ubp, const int32_t* __restrict__ Tc,
                 const double* __restrict__ Tv, const int32_t* __restrict__ Crp, int32_t* __restrict__ Cc,
                 double* __restrict__ Cv) {
    const int64_t tid = (int64_t)blockIdx.x * B + threadIdx.x;
    const int32_t i = (int32_t)(tid / SR_C);
    const int lane = (int)(tid % SR_C);
    if (i >= n || ubp[i + 1] == ubp[i]) return;
    const int32_t src = ubp[i], dst = Crp[i], len = Crp[i + 1] - dst;
    for (int32_t q = lane; q < len; q += SR_C) {
        Cc[dst + q] = Tc[src + q];
        Cv[dst + q] = Tv[src + q];
    }
}

// C = A B; a row whose distinct columns exceed the LDS table sets *flag
// (checked by the caller once the whole setup is queued)
static void spgemm(const Csr& A, const Csr& Bm, Csr& C, int32_t* flag, hipStream_t s) {
    C.n = A.n;
    C.m = Bm.m;
    C.rowptr.alloc(A.n + 1, s);
    DBuf<int32_t> long_rows(std::max(A.n, 1), s), nlong(1, s), vlong(std::max(A.n, 1), s), nvlong(1, s);
    DBuf<int32_t> ubp(A.n + 1, s);
    TP_LAUNCH(k_fill_i32, 1, B, 0, s, nlong.p, 0, (int64_t)1);
    TP_LAUNCH(k_fill_i32, 1, B, 0, s, nvlong.p, 0, (int64_t)1);
    const int grid = std::min<int>(std::max<int>(A.n, 1), 16384);
    // products per output row, estimated from the operands' mean row lengths
    // (host sizes: exact for level operators, upper bounds for P and R)
    const double est = ((double)A.nnz / std::max(A.n, 1)) * ((double)Bm.nnz / std::max(Bm.n, 1));
    const bool wide = est >= 64.0;
    const bool narrow = est <= 24.0;  // rows of a few short B rows: 64 product slots
    // the short kernels' sort keys hold a column in 23 bits, and their
    // staging offsets (at most SR_MAX a row) are 32-bit; otherwise every row
    // takes the long-row kernels
    const bool keys_fit =
        Bm.m < (1 << 23) && (int64_t)A.n * (wide ? 256 : narrow ? 64 : 128) < ((int64_t)1 << 31);
    const bool all_long = !keys_fit;
    // Short rows in one pass: each writes its sorted distinct columns and
    // values to a staging area at its product-count offset and its count to
    // C.rowptr; the long rows are counted by the long-row kernels; once the
    // counts are scanned, the staged rows are compacted into C and the long
    // rows computed in place.
    if (A.n > 0) {
        if (all_long)
            TP_LAUNCH(k_fill_i32, cdiv(A.n, B), B, 0, s, ubp.p, 0, (int64_t)A.n);
        else if (wide)
            TP_LAUNCH((k_spgemm_ub<64, 256>), cdiv(A.n, B), B, 0, s, A.n, A.rowptr.p, A.col.p, Bm.rowptr.p, ubp.p);
        else if (narrow)
            TP_LAUNCH((k_spgemm_ub<16, 64>), cdiv(A.n, B), B, 0, s, A.n, A.rowptr.p, A.col.p, Bm.rowptr.p, ubp.p);
        else
            TP_LAUNCH((k_spgemm_ub<16, 128>), cdiv(A.n, B), B, 0, s, A.n, A.rowptr.p, A.col.p, Bm.rowptr.p, ubp.p);
    }
    scan_exclusive(ubp.p, ubp.p, A.n, s);
    const int32_t staged = read_i32(ubp.p + A.n, s);
    DBuf<int32_t> Tc(std::max(staged, 1), s);
    DBuf<double> Tv(std::max(staged, 1), s);
    // long rows: a workgroup per row (k_spgemm_long); rows of more than
    // LA_MAX A entries go on to the one-wavefront hash-table kernels
    const int lgrid = std::min<int>(std::max<int>(A.n, 1), 8192);
    if (A.n > 0) {
        if (all_long)  // every row to the long-row kernels
            TP_LAUNCH(k_iota_i32, cdiv(A.n, B), B, 0, s, A.n, long_rows.p, nlong.p);
        else if (wide)
            TP_LAUNCH((k_spgemm_short<64, 256>), cdiv(A.n, SR_T / 64), SR_T, 0, s, A.n, A.rowptr.p, A.col.p,
                      A.val.p, Bm.rowptr.p, Bm.col.p, Bm.val.p, C.rowptr.p, (const int32_t*)ubp.p, Tc.p, Tv.p,
                      long_rows.p, nlong.p);
        else if (narrow)
            TP_LAUNCH((k_spgemm_short<16, 64>), cdiv(A.n, SR_T / 16), SR_T, 0, s, A.n, A.rowptr.p, A.col.p,
                      A.val.p, Bm.rowptr.p, Bm.col.p, Bm.val.p, C.rowptr.p, (const int32_t*)ubp.p, Tc.p, Tv.p,
                      long_rows.p, nlong.p);
        else
            TP_LAUNCH((k_spgemm_short<16, 128>), cdiv(A.n, SR_T / 16), SR_T, 0, s, A.n, A.rowptr.p, A.col.p,
                      A.val.p, Bm.rowptr.p, Bm.col.p, Bm.val.p, C.rowptr.p, (const int32_t*)ubp.p, Tc.p, Tv.p,
                      long_rows.p, nlong.p);
        TP_LAUNCH(k_spgemm_long<false>, lgrid, LG_T, 0, s, (const int32_t*)long_rows.p, (const int32_t*)nlong.p,
                  A.rowptr.p, A.col.p, A.val.p, Bm.rowptr.p, Bm.col.p, Bm.val.p, C.rowptr.p, (const int32_t*)nullptr,
                  (int32_t*)nullptr, (double*)nullptr, vlong.p, nvlong.p, flag);
        TP_LAUNCH(k_spgemm_count, grid, SG_WAVE, 0, s, (const int32_t*)vlong.p, (const int32_t*)nvlong.p,
                  A.rowptr.p, A.col.p, Bm.rowptr.p, Bm.col.p, C.rowptr.p, flag);
    }
    scan_exclusive(C.rowptr.p, C.rowptr.p, A.n, s);
    // (an overflowing row is caught by the numeric pass, which only writes
    // rows whose distinct-column count matches the symbolic one)
    C.nnz = read_i32(C.rowptr.p + A.n, s);
    C.col.alloc(C.nnz, s);
    C.val.alloc(C.nnz, s);
    if (A.n > 0) {
        TP_LAUNCH(k_spgemm_compact, cdiv((int64_t)A.n * SR_C, B), B, 0, s, A.n, (const int32_t*)ubp.p,
                  (const int32_t*)Tc.p, (const double*)Tv.p, (const int32_t*)C.rowptr.p, C.col.p, C.val.p);
        // the long-row pass lists the longest rows again: start that list afresh
        TP_LAUNCH(k_fill_i32, 1, B, 0, s, nvlong.p, 0, (int64_t)1);
        TP_LAUNCH(k_spgemm_long<true>, lgrid, LG_T, 0, s, (const int32_t*)long_rows.p, (const int32_t*)nlong.p,
                  A.rowptr.p, A.col.p, A.val.p, Bm.rowptr.p, Bm.col.p, Bm.val.p, (int32_t*)nullptr,
                  (const int32_t*)C.rowptr.p, C.col.p, C.val.p, vlong.p, nvlong.p, flag);
        TP_LAUNCH(k_spgemm_fill, grid, SG_WAVE, 0, s, (const int32_t*)vlong.p, (const int32_t*)nvlong.p,
                  A.rowptr.p, A.col.p, A.val.p, Bm.rowptr.p, Bm.col.p, Bm.val.p, C.rowptr.p, C.col.p, C.val.p,
                  flag);
    }
}

// ---- l1 diagonal, precision copies ----------------------------------------------------
// 1 / sum_j |a_ij| (0 for an empty or zero row), the sum in row order; a
// lane group per row (row_group), each entry broadcast to the group in turn
template <int G>
__global__ void __launch_bounds__(B)
k_l1_dinv(int32_t n, const int32_t* __restrict__ rowptr, const double* __restrict__ val,
          double* __restrict__ dinv) {
    const int32_t i = blockIdx.x * (B / G) + threadIdx.x / G;
    const int lane = threadIdx.x % G;
    if (i >= n) return;
    const int32_t a = rowptr[i], e = rowptr[i + 1];
    double d = 0.0;
    for (int32_t b = a; b < e; b += G) {
        const double v = b + lane < e ? fabs(val[b + lane]) : 0.0;
        const int cnt = min(G, (int)(e - b));
        for (int l = 0; l < cnt; ++l) d += gbcast_d<G>(v, l);
    }
    if (lane == 0) dinv[i] = d > 0.0 ? 1.0 / d : 0.0;
}

__global__ void __launch_bounds__(B)
k_to_f32(int64_t n, const double* __restrict__ a, float* __restrict__ b) {
    int64_t i = (int64_t)blockIdx.x * B + threadIdx.x;
    if (i < n) b[i] = (float)a[i];
}

// storage 2: off-diagonal entries to BF16 (through FP32, round to nearest
// even), the diagonal entry stored as 0 and kept in FP32 in diag
__global__ void __launch_bounds__(B)
k_split_bf16_csr(int32_t n, const int32_t* __restrict__ rowptr, const int32_t* __restrict__ col,
                 const double* __restrict__ val, __bf16* __restrict__ a16, float* __restrict__ diag) {
    const int32_t i = blockIdx.x * B + threadIdx.x;
    if (i >= n) return;
    float dg = 0.f;
    for (int32_t q = rowptr[i]; q < rowptr[i + 1]; ++q) {
        const float v = (float)val[q];
        if (col[q] == i) {
            dg = v;
            a16[q] = (__bf16)0.f;
        } else {
            a16[q] = (__bf16)v;
        }
    }
    diag[i] = dg;
}

// the same for the DIA copy: diagonal d0 (offset 0) stored as 0
__global__ void __launch_bounds__(B)
k_split_bf16_dia(int64_t total, int32_t n, int d0, const double* __restrict__ dia, __bf16* __restrict__ d16) {
    const int64_t e = (int64_t)blockIdx.x * B + threadIdx.x;
    if (e >= total) return;
    d16[e] = (e / n == d0) ? (__bf16)0.f : (__bf16)(float)dia[e];
}

// ---- coarsest level: explicit inverse by blocked Gauss-Jordan elimination --------------
// The inverse is formed with partial (row) pivoting, NB columns at a time.
// For the panel K = [k, k+NB) with pivot rows B (after interchanges) and the
// other rows O, one step turns
//   M_BK -> M_BK^{-1},  M_OK -> -M_OK M_BK^{-1}                  (panel kernel: T)
//   M_BR -> M_BK^{-1} M_BR,  M_OR -> M_OR - M_OK M_BK^{-1} M_BR  (update kernel)
// for every other column R; both are T M_BR(old), plus M_OR for the O rows.
// The update reads the previous matrix X and writes the next one Y, applying
// the panel's row interchanges as a gather (row i of Y comes from row
// rowsrc[i] of X), so no step works in place.  After the last panel the
// interchanges are undone as column interchanges in reverse order.
__global__ void __launch_bounds__(B)
k_fill_f64(int64_t n, double* __restrict__ x, double v) {
    for (int64_t i = (int64_t)blockIdx.x * B + threadIdx.x; i < n; i += (int64_t)gridDim.x * B) x[i] = v;
}

__global__ void __launch_bounds__(B)
k_csr_to_dense(int32_t n, const int32_t* __restrict__ rowptr, const int32_t* __restrict__ col,
               const double* __restrict__ val, double* __restrict__ Dm) {
    int32_t i = blockIdx.x * B + threadIdx.x;
    if (i >= n) return;
    for (int32_t q = rowptr[i]; q < rowptr[i + 1]; ++q) Dm[(int64_t)i * n + col[q]] = val[q];
}


// One workgroup of GJ_T = 256 threads (one wavefront per SIMD); thread t
// holds rows t, t + GJ_T, ... of the panel columns in registers (the column
// loop is unrolled, so every register index is fixed; RPT * NB <= 64 keeps
// the array in registers).
// Per column: each wavefront finds its largest |a_ic| among rows not yet used
// as pivots (ties -> lowest row) and publishes that row; the owner of row
// k+c publishes it too; one barrier; every thread then knows the pivot row
// and applies the interchange and the elimination to its rows.
template <int NB, int RPT, int GJ_T>
__global__ void __launch_bounds__(GJ_T) __attribute__((amdgpu_waves_per_eu(1, 1)))  // a lone workgroup: registers over occupancy
k_gj_panel(int32_t n, int32_t k, const double* __restrict__ X, double* __restrict__ T,
           int32_t* __restrict__ piv, int32_t* __restrict__ rowsrc, int32_t* __restrict__ bad) {
    constexpr int GJ_W = GJ_T / 64;
    static_assert(RPT * NB <= 64, "panel rows must stay in registers");
    __shared__ double s_row[2][GJ_W][NB];
    __shared__ double s_val[2][GJ_W];
    __shared__ int32_t s_idx[2][GJ_W];
    __shared__ double s_kc[2][NB];
    __shared__ int32_t s_piv[NB];
    __shared__ int32_t s_pos[2 * NB], s_from[2 * NB];
    __shared__ int s_m;
    const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
    const int nb = min(NB, n - k);
    double v[RPT][NB];
#pragma unroll
    for (int q = 0; q < RPT; ++q) {
        const int32_t i = t + q * GJ_T;
#pragma unroll
        for (int c = 0; c < NB; ++c) v[q][c] = (i < n && c < nb) ? X[(int64_t)i * n + k + c] : 0.0;
    }
#pragma unroll
    for (int c = 0; c < NB; ++c) {
        if (c >= nb) break;
        const int par = c & 1;
        const int32_t kc = k + c;
        double best = -1.0;
        int32_t bi = n;
#pragma unroll
        for (int q = 0; q < RPT; ++q) {
            const int32_t i = t + q * GJ_T;
            const double x = fabs(v[q][c]);
            if (i < n && i >= kc && x > best) {
                best = x;
                bi = i;
            }
        }
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) {
            const double ob = __shfl_xor(best, off, 64);
            const int32_t oi = __shfl_xor(bi, off, 64);
            if (ob > best || (ob == best && oi < bi)) {
                best = ob;
                bi = oi;
            }
        }
#pragma unroll
        for (int q = 0; q < RPT; ++q) {
            const int32_t i = t + q * GJ_T;
            if (i == bi) {
#pragma unroll
                for (int c2 = 0; c2 < NB; ++c2) s_row[par][wave][c2] = v[q][c2];
            }
            if (i == kc) {
#pragma unroll
                for (int c2 = 0; c2 < NB; ++c2) s_kc[par][c2] = v[q][c2];
            }
        }
        if (lane == 0) {
            s_val[par][wave] = best;
            s_idx[par][wave] = bi;
        }
        __syncthreads();
        double pb = -1.0;
        int32_t p = n;
        int pw = 0;
#pragma unroll
        for (int w = 0; w < GJ_W; ++w) {
            const double x = s_val[par][w];
            const int32_t iw = s_idx[par][w];
            if (x > pb || (x == pb && iw < p)) {
                pb = x;
                p = iw;
                pw = w;
            }
        }
        const bool ok = p < n && pb > 0.0;
        if (!ok) p = kc;  // singular: keep every index in range, the host sees the flag
        if (t == 0) {
            s_piv[c] = p;
            if (!ok) *bad = 1;
        }
        const double* prow = ok ? s_row[par][pw] : s_kc[par];
        const double d = 1.0 / prow[c];
#pragma unroll
        for (int q = 0; q < RPT; ++q) {
            const int32_t i = t + q * GJ_T;
            if (i == kc) {
#pragma unroll
                for (int c2 = 0; c2 < NB; ++c2) v[q][c2] = c2 == c ? d : prow[c2] * d;
            } else {
                if (i == p) {
#pragma unroll
                    for (int c2 = 0; c2 < NB; ++c2) v[q][c2] = s_kc[par][c2];
                }
                const double f = v[q][c];
#pragma unroll
                for (int c2 = 0; c2 < NB; ++c2) v[q][c2] = c2 == c ? -(f * d) : v[q][c2] - f * (prow[c2] * d);
            }
        }
    }
#pragma unroll
    for (int q = 0; q < RPT; ++q) {
        const int32_t i = t + q * GJ_T;
        if (i < n)
#pragma unroll
            for (int c = 0; c < NB; ++c) T[(int64_t)i * NB + c] = v[q][c];
    }
    // the panel's interchanges composed: the rows they touch are pos[0..m)
    // (the pivot positions k..k+nb first); afterwards row pos[e] holds what
    // row pos[from[e]] held before
    __syncthreads();
    if (t < nb) piv[k + t] = s_piv[t];
    if (t == 0) {
        int m = nb;
        for (int c = 0; c < nb; ++c) s_pos[c] = k + c;
        for (int c = 0; c < nb; ++c) {
            const int32_t p = s_piv[c];
            bool seen = false;
            for (int e = 0; e < m; ++e) seen = seen || s_pos[e] == p;
            if (!seen) s_pos[m++] = p;
        }
        for (int e = 0; e < m; ++e) s_from[e] = e;
        for (int c = 0; c < nb; ++c) {
            int ep = 0;
            for (int e = 0; e < m; ++e) ep = s_pos[e] == s_piv[c] ? e : ep;
            const int32_t x = s_from[c];
            s_from[c] = s_from[ep];
            s_from[ep] = x;
        }
        s_m = m;
    }
    __syncthreads();
    const int m = s_m;
    for (int32_t i = t; i < n; i += GJ_T) {
        int32_t src = i;
        for (int e = 0; e < m; ++e) src = s_pos[e] == i ? s_pos[s_from[e]] : src;
        rowsrc[i] = src;
    }
}

// Y_ij = T_i,j-k (j in the panel), else [row i not a pivot row] X_rowsrc[i],j
// + sum_c T_ic X_rowsrc[k+c],j.  64 x 64 tiles, each thread one column and
// 16 rows, all loads issued before the first store.
constexpr int GU_T = 256;
template <int NB>
__global__ void __launch_bounds__(GU_T)
k_gj_update(int32_t n, int32_t k, int32_t nb, const double* __restrict__ X, const double* __restrict__ T,
            const int32_t* __restrict__ rowsrc, double* __restrict__ Y) {
    __shared__ double s_T[64][NB];
    __shared__ double s_B[NB][64];
    __shared__ int32_t s_src[64];
    const int t = threadIdx.x, tx = t & 63, ty = t >> 6;
    const int32_t j0 = blockIdx.x * 64, i0 = blockIdx.y * 64;
    for (int e = t; e < 64 * NB; e += GU_T) {
        const int r = e / NB, c = e % NB;
        const int32_t i = i0 + r;
        s_T[r][c] = (i < n && c < nb) ? T[(int64_t)i * NB + c] : 0.0;
    }
    for (int e = t; e < NB * 64; e += GU_T) {
        const int c = e / 64, x = e % 64;
        const int32_t j = j0 + x;
        s_B[c][x] = (j < n && c < nb) ? X[(int64_t)rowsrc[k + c] * n + j] : 0.0;
    }
    if (t < 64) s_src[t] = i0 + t < n ? rowsrc[i0 + t] : 0;
    __syncthreads();
    const int32_t j = j0 + tx;
    if (j >= n) return;
    const bool inK = j >= k && j < k + nb;
    constexpr int RT = 64 / (GU_T / 64);  // rows per thread
    double acc[RT];
#pragma unroll
    for (int q = 0; q < RT; ++q) {
        const int r = ty + q * (GU_T / 64);
        const int32_t i = i0 + r;
        acc[q] = (i < n && !inK && !(i >= k && i < k + nb)) ? X[(int64_t)s_src[r] * n + j] : 0.0;
    }
#pragma unroll
    for (int q = 0; q < RT; ++q) {
        const int r = ty + q * (GU_T / 64);
        const int32_t i = i0 + r;
        if (i >= n) break;
        if (inK) {
            Y[(int64_t)i * n + j] = s_T[r][j - k];
        } else {
#pragma unroll
            for (int c = 0; c < NB; ++c) acc[q] += s_T[r][c] * s_B[c][tx];
            Y[(int64_t)i * n + j] = acc[q];
        }
    }
}

// source column of every column of the inverse: the interchanges replayed on
// an index vector in reverse order (one thread; piv and src in LDS)
constexpr int GS_T = 1024;
__global__ void __launch_bounds__(GS_T)
k_gj_src(int32_t n, const int32_t* __restrict__ piv, int32_t* __restrict__ src) {
    __shared__ int32_t s_piv[4096], s_src[4096];
    for (int32_t i = threadIdx.x; i < n; i += GS_T) {
        s_piv[i] = piv[i];
        s_src[i] = i;
    }
    __syncthreads();
    if (threadIdx.x == 0)
        for (int32_t l = n - 1; l >= 0; --l) {
            const int32_t p = s_piv[l];
            const int32_t x = s_src[l];
            s_src[l] = s_src[p];
            s_src[p] = x;
        }
    __syncthreads();
    for (int32_t i = threadIdx.x; i < n; i += GS_T) src[i] = s_src[i];
}

__global__ void __launch_bounds__(B)
k_gj_gather(int32_t n, const double* __restrict__ a, const int32_t* __restrict__ src, double* __restrict__ inv) {
    const int64_t e = (int64_t)blockIdx.x * B + threadIdx.x;
    if (e >= (int64_t)n * n) return;
    const int32_t i = (int32_t)(e / n), j = (int32_t)(e % n);
    inv[e] = a[(int64_t)i * n + src[j]];
}

// returns the buffer holding the result
template <int NB, int RPT, int GJ_T>
static double* gj_run(int32_t n, double* X, double* Y, double* T, int32_t* rowsrc, int32_t* piv, int32_t* bad,
                      hipStream_t s) {
    const dim3 g(cdiv(n, 64), cdiv(n, 64));
    for (int32_t k = 0; k < n; k += NB) {
        TP_LAUNCH((k_gj_panel<NB, RPT, GJ_T>), 1, GJ_T, 0, s, n, k, (const double*)X, T, piv, rowsrc, bad);
        TP_LAUNCH((k_gj_update<NB>), g, GU_T, 0, s, n, k, std::min(NB, n - k), (const double*)X,
                  (const double*)T, (const int32_t*)rowsrc, Y);
        std::swap(X, Y);
    }
    return X;
}

// ---- the same elimination without interchanges, verified -------------------------------
// Partial pivoting leaves the rows in place exactly when, at every column, the
// diagonal entry is the largest candidate (ties go to the lowest row, i.e. the
// diagonal).  The coarse operators met here (Galerkin products of the TPFA
// blocks) satisfy this, so the steps above run with diagonal pivots: the
// NB x NB pivot block is inverted by one workgroup (recording its LU upper
// factor), and the update kernel, besides forming the next matrix, re-runs the
// forward elimination of every candidate row below the block against that
// factor and flags a column where the row would beat the pivot.  A flag sends
// the whole inverse through the row-pivoted kernels instead, so the pivot
// sequence is always the one partial pivoting would choose.
constexpr int BG_NB = 32;

// One workgroup inverts the pivot block in LDS (Gauss-Jordan with diagonal
// pivots, recording the LU upper factor); thread t owns column t % BG_NB of
// rows t / BG_NB + (BK_T / BG_NB) q.  Rows and columns past nb carry the
// identity and stay untouched.
constexpr int BK_T = 1024;
__global__ void __launch_bounds__(BK_T)
k_bgj_block(int32_t n, int32_t k, const double* __restrict__ X, double* __restrict__ binv, double* __restrict__ U,
            int32_t* __restrict__ need_piv) {
    __shared__ double s_a[BG_NB][BG_NB + 1];
    constexpr int RQ = BG_NB * BG_NB / BK_T;
    const int t = threadIdx.x, j = t % BG_NB, r0 = t / BG_NB;
    const int nb = min(BG_NB, n - k);
#pragma unroll
    for (int q = 0; q < RQ; ++q) {
        const int r = r0 + q * (BK_T / BG_NB);
        s_a[r][j] = (r < nb && j < nb) ? X[(int64_t)(k + r) * n + k + j] : (r == j ? 1.0 : 0.0);
    }
    __syncthreads();
    bool flag = false;
    for (int c = 0; c < nb; ++c) {
        const double p = s_a[c][c];
        if (t == 0) flag = flag || !(fabs(p) > 0.0 && fabs(p) <= DBL_MAX);  // zero or non-finite pivot
        const double u = s_a[c][j];
        double m[RQ];
#pragma unroll
        for (int q = 0; q < RQ; ++q) {
            const int r = r0 + q * (BK_T / BG_NB);
            m[q] = s_a[r][c];
            if (j == c && r > c && r < nb) flag = flag || !(fabs(m[q]) <= fabs(p));
            if (r == c && j >= c && j < nb) U[c * BG_NB + j] = u;
        }
        __syncthreads();
        const double d = 1.0 / p;
#pragma unroll
        for (int q = 0; q < RQ; ++q) {
            const int r = r0 + q * (BK_T / BG_NB);
            if (r == c) s_a[r][j] = j == c ? d : u * d;
            else s_a[r][j] = j == c ? -(m[q] * d) : s_a[r][j] - m[q] * (u * d);
        }
        __syncthreads();
    }
#pragma unroll
    for (int q = 0; q < RQ; ++q) {
        const int r = r0 + q * (BK_T / BG_NB);
        if (r < nb && j < nb) binv[r * BG_NB + j] = s_a[r][j];
    }
    if (flag) *need_piv = 1;
}

// W = Binv on the block's rows and W = -X_iK Binv on the others (n x BG_NB,
// one thread per entry, a row's BG_NB entries in one wavefront).  The
// same wavefront re-runs the forward elimination of a candidate row
// below the block against the block's U (lanes hold the row's entries, the
// pivot entry is broadcast by a shuffle) and flags a column where the row
// would beat the pivot.
constexpr int BW_T = 256;
__global__ void __launch_bounds__(BW_T)
k_bgj_w(int32_t n, int32_t k, int32_t nb, const double* __restrict__ X, const double* __restrict__ binv,
        const double* __restrict__ U, double* __restrict__ W, int32_t* __restrict__ need_piv) {
    __shared__ double s_bi[BG_NB][BG_NB + 1];
    __shared__ double s_U[BG_NB][BG_NB + 1];
    __shared__ double s_x[BW_T / BG_NB][BG_NB + 1];
    const int t = threadIdx.x, c = t % BG_NB, rr = t / BG_NB;
    const int32_t i = blockIdx.x * (BW_T / BG_NB) + rr;
    for (int e = t; e < BG_NB * BG_NB; e += BW_T) {
        const int r = e / BG_NB, q = e % BG_NB;
        s_bi[r][q] = (r < nb && q < nb) ? binv[r * BG_NB + q] : 0.0;
        s_U[r][q] = (r < nb && q < nb && q >= r) ? U[r * BG_NB + q] : 0.0;
    }
    const double xv = (i < n && c < nb) ? X[(int64_t)i * n + k + c] : 0.0;
    s_x[rr][c] = xv;
    __syncthreads();
    if (i >= n) return;
    double w;
    if (i >= k && i < k + nb) {
        w = s_bi[i - k][c];
    } else {
        w = 0.0;
        for (int q = 0; q < nb; ++q) w += s_x[rr][q] * s_bi[q][c];
        w = -w;
    }
    W[(int64_t)i * BG_NB + c] = w;
    if (i >= k + nb) {
        double v = xv;
        bool flag = false;
        for (int q = 0; q < nb; ++q) {
            const double vq = __shfl(v, (t & ~(BG_NB - 1) & 63) + q, 64);
            const double p = s_U[q][q];
            flag = flag || !(fabs(vq) <= fabs(p));
            if (c > q) v -= (vq / p) * s_U[q][c];
        }
        if (flag) *need_piv = 1;
    }
}

// Y_ij = W_i,j-k (j in the block), else [i not in the block] X_ij + sum_c W_ic X_k+c,j.
// TS x TS tiles (TS = 16 MT); each thread an MT x MT micro-tile, all its loads
// of X before its stores.  Every output sums its terms in the same order for
// any TS, so the tile size changes only the launch shape.
constexpr int BU_T = 256;
template <int MT>
__global__ void __launch_bounds__(BU_T)
k_bgj_update(int32_t n, int32_t k, int32_t nb, const double* __restrict__ X, const double* __restrict__ W,
             double* __restrict__ Y) {
    constexpr int TS = 16 * MT;
    __shared__ double s_W[TS][BG_NB + 1];
    __shared__ double s_B[BG_NB][TS + 2];
    const int t = threadIdx.x, tx = t % 16, ty = t / 16;
    const int32_t j0 = blockIdx.x * TS, i0 = blockIdx.y * TS;
    for (int e = t; e < TS * BG_NB; e += BU_T) {
        const int r = e / BG_NB, c = e % BG_NB;
        const int32_t i = i0 + r;
        s_W[r][c] = (i < n && c < nb) ? W[(int64_t)i * BG_NB + c] : 0.0;
    }
    for (int e = t; e < BG_NB * TS; e += BU_T) {
        const int c = e / TS, x = e % TS;
        const int32_t j = j0 + x;
        s_B[c][x] = (j < n && c < nb) ? X[(int64_t)(k + c) * n + j] : 0.0;
    }
    double acc[MT][MT];
#pragma unroll
    for (int a = 0; a < MT; ++a) {
        const int32_t i = i0 + MT * ty + a;
        const bool keep = i < n && !(i >= k && i < k + nb);
#pragma unroll
        for (int q = 0; q < MT; ++q) {
            const int32_t j = j0 + MT * tx + q;
            acc[a][q] = (keep && j < n && !(j >= k && j < k + nb)) ? X[(int64_t)i * n + j] : 0.0;
        }
    }
    __syncthreads();
#pragma unroll 8
    for (int c = 0; c < BG_NB; ++c) {
        double wv[MT], bv[MT];
#pragma unroll
        for (int a = 0; a < MT; ++a) wv[a] = s_W[MT * ty + a][c];
#pragma unroll
        for (int q = 0; q < MT; ++q) bv[q] = s_B[c][MT * tx + q];
#pragma unroll
        for (int a = 0; a < MT; ++a)
#pragma unroll
            for (int q = 0; q < MT; ++q) acc[a][q] += wv[a] * bv[q];
    }
#pragma unroll
    for (int a = 0; a < MT; ++a) {
        const int32_t i = i0 + MT * ty + a;
        if (i >= n) continue;
#pragma unroll
        for (int q = 0; q < MT; ++q) {
            const int32_t j = j0 + MT * tx + q;
            if (j >= n) continue;
            Y[(int64_t)i * n + j] = (j >= k && j < k + nb) ? s_W[MT * ty + a][j - k] : acc[a][q];
        }
    }
}

static void build_coarse_inverse(tp_amg* h, const Csr& A, hipStream_t s) {
    const int32_t n = A.n;
    h->nc = n;
    if (n > 4096) fail(TP_ERR_NUMERIC, "coarsening stalled at %d rows (> 4096), no dense factorisation", n);
    if (h->cinv.n != (size_t)n * n) h->cinv.alloc((size_t)n * n, s);  // kept on a refresh (graphs hold it)
    if (n == 0) return;
    DBuf<double> W((size_t)n * n, s), T((size_t)16 * n, s), binv(BG_NB * BG_NB, s), U(BG_NB * BG_NB, s),
        Wk((size_t)BG_NB * n, s);
    DBuf<int32_t> piv(n, s), rowsrc(n, s), src(n, s), flags(2, s);
    const int64_t nn = (int64_t)n * n;
    const int fill_grid = (int)std::min<int64_t>(cdiv(nn, B), 4096);
    TP_LAUNCH(k_fill_i32, 1, B, 0, s, flags.p, 0, (int64_t)2);
    // diagonal pivots: ping-pong so that the last step writes cinv
    const int steps = cdiv(n, BG_NB);
    double* X = steps % 2 == 0 ? h->cinv.p : W.p;
    double* Y = steps % 2 == 0 ? W.p : h->cinv.p;
    TP_LAUNCH(k_fill_f64, fill_grid, B, 0, s, nn, X, 0.0);
    TP_LAUNCH(k_csr_to_dense, cdiv(n, B), B, 0, s, n, A.rowptr.p, A.col.p, A.val.p, X);
    // 32 x 32 tiles while 64 x 64 ones would leave the chip under-filled
    const bool small_tiles = n <= 2048;
    const dim3 g = small_tiles ? dim3(cdiv(n, 32), cdiv(n, 32)) : dim3(cdiv(n, 64), cdiv(n, 64));
    for (int32_t k = 0; k < n; k += BG_NB) {
        TP_LAUNCH(k_bgj_block, 1, BK_T, 0, s, n, k, (const double*)X, binv.p, U.p, flags.p);
        const int32_t nb = std::min(BG_NB, n - k);
        TP_LAUNCH(k_bgj_w, cdiv(n, BW_T / BG_NB), BW_T, 0, s, n, k, nb, (const double*)X, (const double*)binv.p,
                  (const double*)U.p, Wk.p, flags.p);
        if (small_tiles)
            TP_LAUNCH(k_bgj_update<2>, g, BU_T, 0, s, n, k, nb, (const double*)X, (const double*)Wk.p, Y);
        else
            TP_LAUNCH(k_bgj_update<4>, g, BU_T, 0, s, n, k, nb, (const double*)X, (const double*)Wk.p, Y);
        std::swap(X, Y);
    }
    if (read_i32(flags.p, s) == 0) return;  // no interchange needed: cinv holds the inverse
    // partial pivoting would interchange rows: the row-pivoted elimination
    X = W.p;
    Y = h->cinv.p;
    TP_LAUNCH(k_fill_f64, fill_grid, B, 0, s, nn, X, 0.0);
    TP_LAUNCH(k_csr_to_dense, cdiv(n, B), B, 0, s, n, A.rowptr.p, A.col.p, A.val.p, X);
    int32_t* bad = flags.p + 1;
    double* res;
    if (n <= 512) res = gj_run<16, 2, 256>(n, X, Y, T.p, rowsrc.p, piv.p, bad, s);
    else if (n <= 1024) res = gj_run<16, 4, 256>(n, X, Y, T.p, rowsrc.p, piv.p, bad, s);
    else if (n <= 1280) res = gj_run<12, 5, 256>(n, X, Y, T.p, rowsrc.p, piv.p, bad, s);
    else if (n <= 2048) res = gj_run<8, 8, 256>(n, X, Y, T.p, rowsrc.p, piv.p, bad, s);
    else res = gj_run<4, 16, 256>(n, X, Y, T.p, rowsrc.p, piv.p, bad, s);
    if (read_i32(bad, s)) fail(TP_ERR_NUMERIC, "zero pivot in the coarsest-level elimination (n=%d)", n);
    // res is one of W, cinv: gather into the other, then make sure cinv holds it
    double* out = res == W.p ? h->cinv.p : W.p;
    TP_LAUNCH(k_gj_src, 1, GS_T, 0, s, n, piv.p, src.p);
    TP_LAUNCH(k_gj_gather, cdiv(nn, B), B, 0, s, n, (const double*)res, src.p, out);
    if (out != h->cinv.p)
        TP_HIP(hipMemcpyAsync(h->cinv.p, out, sizeof(double) * nn, hipMemcpyDeviceToDevice, s));
}

// ---- setup driver ---------------------------------------------------------------------
static void copy_csr_in(Csr& A, int32_t n, const int32_t* rowptr, const int32_t* col, const double* val,
                        hipStream_t s) {
    A.n = A.m = n;
    A.nnz = read_i32(rowptr + n, s);
    TP_CHECK_ARG(A.nnz >= n, "amg_setup: nnz %d < n %d (diagonal missing)", A.nnz, n);
    A.rowptr.alloc(n + 1, s);
    A.col.alloc(A.nnz, s);
    A.val.alloc(A.nnz, s);
    TP_HIP(hipMemcpyAsync(A.rowptr.p, rowptr, sizeof(int32_t) * (n + 1), hipMemcpyDeviceToDevice, s));
    TP_HIP(hipMemcpyAsync(A.col.p, col, sizeof(int32_t) * A.nnz, hipMemcpyDeviceToDevice, s));
    TP_HIP(hipMemcpyAsync(A.val.p, val, sizeof(double) * A.nnz, hipMemcpyDeviceToDevice, s));
}

// strength matrix (pattern) of A
static void strength(const Csr& A, double theta, Csr& S, hipStream_t s) {
    S.n = S.m = A.n;
    S.rowptr.alloc(A.n + 1, s);
    const int g = row_group(A.n, A.nnz);
    auto pass = [&](int32_t* cnt, const int32_t* srp, int32_t* scol) {
        if (A.n == 0) return;
        TP_ROWS_LAUNCH(k_strength_w, g, A.n, s, A.n, A.rowptr.p, A.col.p, A.val.p, theta, cnt, srp, scol);
    };
    pass(S.rowptr.p, nullptr, nullptr);
    scan_exclusive(S.rowptr.p, S.rowptr.p, A.n, s);
    S.nnz = A.nnz;  // an upper bound (S is a subset of A's pattern): no host read
    S.col.alloc(S.nnz, s);
    pass(nullptr, S.rowptr.p, S.col.p);
}

static void direct_interp(const Csr& A, const Csr& S, const int32_t* cf, const int32_t* cmap, int32_t nc,
                          Csr& P, hipStream_t s) {
    P.n = A.n;
    P.m = nc;
    P.rowptr.alloc(A.n + 1, s);
    const int g = row_group(A.n, A.nnz);
    if (A.n > 0) TP_ROWS_LAUNCH(k_interp_count_w, g, A.n, s, A.n, S.rowptr.p, S.col.p, cf, P.rowptr.p);
    scan_exclusive(P.rowptr.p, P.rowptr.p, A.n, s);
    // an upper bound (an F row interpolates from its strong C neighbours, a
    // C row has one entry); the exact count is read once at the end of setup
    P.nnz = A.nnz;
    P.col.alloc(P.nnz, s);
    P.val.alloc(P.nnz, s);
    if (A.n > 0)
        TP_ROWS_LAUNCH(k_interp_fill_w, g, A.n, s, A.n, A.rowptr.p, A.col.p, A.val.p, S.rowptr.p, S.col.p, cf,
                       cmap, P.rowptr.p, P.col.p, P.val.p);
}

// Extended+i weights of every row of A over its interpolatory set (row i of
// T) written to P: at setup (refresh 0) P's columns too, truncated to the
// pmax of largest magnitude; in a numeric refresh (refresh 1) P's pattern is
// frozen and only its values are rewritten.
static void ext_fill(const Csr& A, const Csr& S, const Csr& T, const int32_t* cf, const int32_t* cmap, Csr& P,
                     int pmax, int refresh, hipStream_t s) {
    const int32_t n = A.n;
    if (n == 0) return;
    DBuf<double> wbuf(std::max(T.nnz, 1), s);  // one weight per interpolatory-set entry
    if (long_rows(A.n, A.nnz))
        TP_LAUNCH(k_ext_fill_w, cdiv(n, WR_ROWS), B, 0, s, n, A.rowptr.p, A.col.p, A.val.p, S.rowptr.p, S.col.p, cf,
                  cmap, T.rowptr.p, T.col.p, P.rowptr.p, P.col.p, P.val.p, wbuf.p, pmax, refresh);
    else
        TP_LAUNCH(k_ext_fill, cdiv(n, B), B, 0, s, n, A.rowptr.p, A.col.p, A.val.p, S.rowptr.p, S.col.p, cf, cmap,
                  T.rowptr.p, T.col.p, P.rowptr.p, P.col.p, P.val.p, wbuf.p, pmax, refresh);
}

// T (out): the interpolatory sets C^_i, one row per point (fine columns,
// ascending), kept by the caller for numeric refreshes.
static void ext_interp(const Csr& A, const Csr& S, const int32_t* cf, const int32_t* cmap, int32_t nc,
                       int pmax, Csr& P, Csr& T, int32_t* flag, hipStream_t s) {
    const int32_t n = A.n;
    Csr X, Y;
    X.n = Y.n = n;
    X.m = Y.m = n;
    X.rowptr.alloc(n + 1, s);
    Y.rowptr.alloc(n + 1, s);
    if (n > 0) TP_LAUNCH(k_ext_xy_count, cdiv(n, B), B, 0, s, n, S.rowptr.p, S.col.p, cf, X.rowptr.p, Y.rowptr.p);
    scan_exclusive(X.rowptr.p, X.rowptr.p, n, s);
    scan_exclusive(Y.rowptr.p, Y.rowptr.p, n, s);
    // upper bounds (one entry of S, or i itself, per entry of X and Y); the
    // SpGEMM reads the exact sizes from the row pointers
    X.nnz = S.nnz + n;
    Y.nnz = S.nnz;
    X.col.alloc(std::max(X.nnz, 1), s);
    X.val.alloc(std::max(X.nnz, 1), s);
    Y.col.alloc(std::max(Y.nnz, 1), s);
    Y.val.alloc(std::max(Y.nnz, 1), s);
    if (n > 0)
        TP_LAUNCH(k_ext_xy_fill, cdiv(n, B), B, 0, s, n, S.rowptr.p, S.col.p, cf, X.rowptr.p, X.col.p, X.val.p,
                  Y.rowptr.p, Y.col.p, Y.val.p);
    spgemm(X, Y, T, flag, s);
    P.n = n;
    P.m = nc;
    P.rowptr.alloc(n + 1, s);
    if (n > 0) TP_LAUNCH(k_ext_count, cdiv(n, B), B, 0, s, n, cf, T.rowptr.p, pmax, P.rowptr.p);
    scan_exclusive(P.rowptr.p, P.rowptr.p, n, s);
    P.nnz = read_i32(P.rowptr.p + n, s);
    P.col.alloc(std::max(P.nnz, 1), s);
    P.val.alloc(std::max(P.nnz, 1), s);
    ext_fill(A, S, T, cf, cmap, P, pmax, 0, s);
}

static void make_f32(DBuf<float>& dst, const DBuf<double>& src, size_t n, hipStream_t s) {
    dst.alloc(n, s);
    if (n) TP_LAUNCH(k_to_f32, cdiv(n, B), B, 0, s, (int64_t)n, src.p, dst.p);
}

// ---- DIA detection --------------------------------------------------------------------
__global__ void __launch_bounds__(B)
k_dia_fill(int32_t n, const int32_t* __restrict__ rowptr, const int32_t* __restrict__ col,
           const double* __restrict__ val, int nd, const int32_t* __restrict__ offs,
           double* __restrict__ dia) {
    int32_t i = blockIdx.x * B + threadIdx.x;
    if (i >= n) return;
    for (int d = 0; d < nd; ++d) dia[(int64_t)d * n + i] = 0.0;
    for (int32_t q = rowptr[i]; q < rowptr[i + 1]; ++q) {
        int32_t o = col[q] - i;
        for (int d = 0; d < nd; ++d)
            if (offs[d] == o) dia[(int64_t)d * n + i] = val[q];
    }
}

// One wavefront: lanes 1..15 measure 15 hashed rows; lane 0 takes the
// longest (ties: the first probed) and, when its length is odd in 3..7, writes
// its column offsets: out[0] = number of diagonals (0: not a stencil level),
// out[1..] = offsets.
__global__ void __launch_bounds__(64)
k_dia_probe(int32_t n, const int32_t* __restrict__ rowptr, const int32_t* __restrict__ col,
            int32_t* __restrict__ out) {
    __shared__ int32_t lens[16];
    const uint32_t k = threadIdx.x;
    if (k < 16) {
        const int32_t r = (int32_t)((k * 2654435761u) % (uint32_t)n);
        lens[k] = k >= 1 ? rowptr[r + 1] - rowptr[r] : -1;
    }
    __syncthreads();
    if (k != 0) return;
    int32_t best_len = -1, best_row = 0;
    for (uint32_t q = 1; q <= 15; ++q)
        if (lens[q] > best_len) {
            best_len = lens[q];
            best_row = (int32_t)((q * 2654435761u) % (uint32_t)n);
        }
    const int nd = (best_len >= 3 && best_len <= 7 && best_len % 2 == 1) ? best_len : 0;
    out[0] = nd;
    const int32_t rp0 = rowptr[best_row];
    for (int d = 0; d < nd; ++d) out[1 + d] = col[rp0 + d] - best_row;
}

// Every entry's offset col - row must belong to the probe row's offsets.
__global__ void __launch_bounds__(B)
k_dia_check(int32_t n, const int32_t* __restrict__ rowptr, const int32_t* __restrict__ col,
            const int32_t* __restrict__ probe, int32_t* __restrict__ bad) {
    int32_t i = blockIdx.x * B + threadIdx.x;
    if (i >= n) return;
    const int nd = probe[0];
    if (nd == 0) {
        if (i == 0) *bad = 1;
        return;
    }
    for (int32_t q = rowptr[i]; q < rowptr[i + 1]; ++q) {
        int32_t o = col[q] - i;
        bool found = false;
        for (int d = 0; d < nd; ++d) found |= (probe[1 + d] == o);
        if (!found) *bad = 1;
    }
}

// DIA copy of a stencil level: one device probe and check, one host read.
// most entries in any block of rb consecutive rows
__global__ void __launch_bounds__(B)
k_block_nnz_max(int32_t n, const int32_t* __restrict__ rowptr, int32_t rb, int32_t* __restrict__ out) {
    const int32_t b = blockIdx.x * B + threadIdx.x;
    const int64_t r0 = (int64_t)b * rb;
    if (r0 >= n) return;
    const int32_t r1 = r0 + rb < n ? (int32_t)(r0 + rb) : n;
    atomicMax(out, rowptr[r1] - rowptr[r0]);
}

// Row-block form of a large CSR level (n >= 65536): 64-row blocks (32 when
// those would hold more products than the LDS budget) whose products fit in
// 48 KB of LDS; else the level keeps the lane-group kernels.  Measured on the
// 256x256x64 hierarchies (18-60 entries a row), time per preconditioner
// apply against the lane-group kernels: 64 rows -2.0% (FP32) / -1.4%
// (FP64), 32 rows -1.2% / -1.5%, 128 rows -1.6% / 0, 256 rows +1.8% / +0.2%.
// The first block size of rbs whose blocks of rb consecutive rows of X hold at
// most `cap` entries: its rows and that maximum (0, 0 when none fits).
static void stream_blocks(const Csr& X, int32_t cap, std::initializer_list<int32_t> rbs, int* rows, int* lds,
                          hipStream_t s) {
    *rows = *lds = 0;
    DBuf<int32_t> mx(1, s);
    for (int32_t rb : rbs) {
        TP_LAUNCH(k_fill_i32, 1, B, 0, s, mx.p, 0, (int64_t)1);
        TP_LAUNCH(k_block_nnz_max, cdiv(cdiv(X.n, rb), B), B, 0, s, X.n, X.rowptr.p, rb, mx.p);
        const int32_t m = read_i32(mx.p, s);
        if (m <= cap) {
            *rows = rb;
            *lds = std::max(m, 1);
            return;
        }
    }
}

static void try_stream(tp_amg* h, Level& L, hipStream_t s) {
    L.sb_rows = L.sb_lds = L.sbP_rows = L.sbP_lds = L.sbR_rows = L.sbR_lds = 0;
    const int32_t cap = (int32_t)(48 * 1024 / storage_bytes(h));
    if (!L.ndia && L.A.n >= 65536) stream_blocks(L.A, cap, {64, 32}, &L.sb_rows, &L.sb_lds, s);
    // P's rows are short (a few entries), R's a few tens: blocks of a whole
    // workgroup's rows
    if (L.P.n >= 65536) stream_blocks(L.P, cap, {256, 128}, &L.sbP_rows, &L.sbP_lds, s);
    if (L.R.n >= 65536) stream_blocks(L.R, cap, {256, 128, 64}, &L.sbR_rows, &L.sbR_lds, s);
}

static void try_dia(tp_amg* h, Level& L, hipStream_t s) {
    const int32_t n = L.A.n;
    if (n < 1024 || L.A.nnz > 8LL * n) return;
    DBuf<int32_t> res(9, s);  // [0] bad, [1] nd, [2..8] offsets
    TP_LAUNCH(k_fill_i32, 1, B, 0, s, res.p, 0, (int64_t)1);
    TP_LAUNCH(k_dia_probe, 1, 64, 0, s, n, L.A.rowptr.p, L.A.col.p, res.p + 1);
    TP_LAUNCH(k_dia_check, cdiv(n, B), B, 0, s, n, L.A.rowptr.p, L.A.col.p, (const int32_t*)(res.p + 1), res.p);
    int32_t hres[9] = {0};
    TP_HIP(hipMemcpyAsync(hres, res.p, sizeof(hres), hipMemcpyDeviceToHost, s));
    TP_HIP(hipStreamSynchronize(s));
    if (hres[0] || hres[1] == 0) return;
    const int nd = hres[1];
    L.ndia = nd;
    for (int d = 0; d < nd; ++d) L.dia_off[d] = hres[2 + d];
    L.dia.alloc((size_t)nd * n, s);
    TP_LAUNCH(k_dia_fill, cdiv(n, B), B, 0, s, n, L.A.rowptr.p, L.A.col.p, L.A.val.p, nd,
              (const int32_t*)(res.p + 2), L.dia.p);
    if (h->prm.storage == 1) {
        L.dia32.alloc((size_t)nd * n, s);
        TP_LAUNCH(k_to_f32, cdiv((int64_t)nd * n, B), B, 0, s, (int64_t)nd * n, L.dia.p, L.dia32.p);
    } else if (h->prm.storage == 2) {
        int d0 = -1;
        for (int d = 0; d < nd; ++d)
            if (L.dia_off[d] == 0) d0 = d;
        L.dia16.alloc((size_t)nd * n, s);
        TP_LAUNCH(k_split_bf16_dia, cdiv((int64_t)nd * n, B), B, 0, s, (int64_t)nd * n, n, d0, L.dia.p,
                  (__bf16*)L.dia16.p);
    }
}

static void alloc_work(tp_amg* h, hipStream_t s) {
    size_t es = storage_bytes(h);
    for (auto& L : h->lev) {
        size_t n = (size_t)std::max(L.A.n, 1);
        L.b.alloc(n * es, s);
        L.x.alloc(n * es, s);
        L.x2.alloc(n * es, s);
        L.r.alloc(n * es, s);
        L.d.alloc(n * es, s);
        L.gA = lanes_for(L.A.n, L.A.nnz);
        L.gP = lanes_for(L.P.n, L.P.nnz);
        L.gR = lanes_for(L.R.n, L.R.nnz);
        if (&L != &h->lev.back()) {
            try_dia(h, L, s);
            try_stream(h, L, s);
        }
        if (h->prm.storage >= 1) {
            if (h->prm.storage == 1) {
                make_f32(L.A32, L.A.val, L.A.nnz, s);
            } else {
                L.A16.alloc(std::max(L.A.nnz, 1), s);
                L.diag32.alloc(n, s);
                if (L.A.n > 0)
                    TP_LAUNCH(k_split_bf16_csr, cdiv(L.A.n, B), B, 0, s, L.A.n, L.A.rowptr.p, L.A.col.p, L.A.val.p,
                              (__bf16*)L.A16.p, L.diag32.p);
            }
            make_f32(L.dinv32, L.dinv, L.A.n, s);
            if (L.P.nnz) make_f32(L.P32, L.P.val, L.P.nnz, s);
            if (L.R.nnz) make_f32(L.R32, L.R.val, L.R.nnz, s);
        }
    }
}

// The sizes of P and R were allocated from upper bounds during the level
// loop; their exact entry counts (rowptr[n]) and the SpGEMM overflow flag are
// gathered by one kernel and read once.
struct SizeSrc {
    const int32_t* p[64];
    int32_t count;
};

__global__ void k_gather_i32(SizeSrc src, int32_t* __restrict__ out) {
    const int t = threadIdx.x;
    if (t < src.count) out[t] = *src.p[t];
}

static void exact_sizes(tp_amg* h, const int32_t* flag, hipStream_t s) {
    SizeSrc src{};
    int c = 0;
    for (size_t l = 0; l + 1 < h->lev.size(); ++l) {
        Level& L = h->lev[l];
        src.p[c++] = L.P.rowptr.p + L.P.n;
        src.p[c++] = L.R.rowptr.p + L.R.n;
    }
    src.p[c++] = flag;
    src.count = c;
    DBuf<int32_t> out(c, s);
    TP_LAUNCH(k_gather_i32, 1, 64, 0, s, src, out.p);
    std::vector<int32_t> v(c);
    TP_HIP(hipMemcpyAsync(v.data(), out.p, sizeof(int32_t) * c, hipMemcpyDeviceToHost, s));
    TP_HIP(hipStreamSynchronize(s));
    if (v[c - 1]) fail(TP_ERR_CAPACITY, "SpGEMM row exceeded the %d-entry LDS hash table (code %d)", HASH, v[c - 1]);
    for (size_t l = 0; l + 1 < h->lev.size(); ++l) {
        h->lev[l].P.nnz = v[2 * l];
        h->lev[l].R.nnz = v[2 * l + 1];
    }
}

static void setup(tp_amg* h, int32_t n, const int32_t* rowptr, const int32_t* col, const double* val,
                  hipStream_t s) {
    const tp_amg_params& prm = h->prm;
    h->lev.emplace_back();
    copy_csr_in(h->lev[0].A, n, rowptr, col, val, s);
    DBuf<int32_t> undecided(512, s), sg_flag(1, s);
    TP_LAUNCH(k_fill_i32, 1, B, 0, s, sg_flag.p, 0, (int64_t)1);
    for (int32_t l = 0;; ++l) {
        Level& L = h->lev[l];
        Csr& A = L.A;
        L.dinv.alloc(std::max(A.n, 1), s);
        if (A.n > 0) TP_ROWS_LAUNCH(k_l1_dinv, row_group(A.n, A.nnz), A.n, s, A.n, A.rowptr.p, A.val.p, L.dinv.p);
        if (A.n <= prm.coarse_max || l + 1 >= prm.max_levels) break;
        Csr S, ST;
        strength(A, prm.theta, S, s);
        transpose(S.rowptr.p, S.col.p, nullptr, S.n, S.n, S.nnz, false, ST, s);
        // PMIS rounds
        DBuf<int8_t> st(A.n, s), st2(A.n, s);
        TP_LAUNCH(k_pmis_init, cdiv(A.n, B), B, 0, s, A.n, ST.rowptr.p, st.p);
        const uint64_t hseed = prm.seed ^ ((uint64_t)l << 40);
        // Rounds are idempotent once every point is decided, so the host
        // reads the undecided flag only after every third round.
        int round = 0;
        TP_LAUNCH(k_fill_i32, 2, B, 0, s, undecided.p, 0, (int64_t)512);  // one flag per round
        for (;; ++round) {
            if (round >= 510) fail(TP_ERR_NUMERIC, "PMIS did not finish in 510 rounds");
            TP_LAUNCH(k_pmis_select, cdiv(A.n, B), B, 0, s, A.n, hseed, S.rowptr.p, S.col.p, ST.rowptr.p,
                      ST.col.p, st.p, st2.p);
            TP_LAUNCH(k_pmis_fmark, cdiv(A.n, B), B, 0, s, A.n, S.rowptr.p, S.col.p, st2.p,
                      undecided.p + round);
            std::swap(st.p, st2.p);
            if (round % 3 == 2 && read_i32(undecided.p + round, s) == 0) break;
        }
        L.cf.alloc(A.n, s);
        TP_LAUNCH(k_cf_flags, cdiv(A.n, B), B, 0, s, A.n, st.p, L.cf.p);
        DBuf<int32_t> cmap(A.n + 1, s);
        scan_exclusive(L.cf.p, cmap.p, A.n, s);
        const int32_t nc = read_i32(cmap.p + A.n, s);
        if (nc == 0 || (double)nc > 0.9 * (double)A.n) {  // empty or stalled coarsening
            L.cf.release();
            break;
        }
        if (prm.interp == 1) {
            ext_interp(A, S, L.cf.p, cmap.p, nc, prm.interp_pmax, L.P, L.T, sg_flag.p, s);
            L.S = std::move(S);
        } else {
            direct_interp(A, S, L.cf.p, cmap.p, nc, L.P, s);
        }
        if (prm.restriction == 1) {
            Csr At, St, Q;
            transpose_square(A, l == 0, At, s);
            strength(At, prm.theta, St, s);
            if (prm.interp == 1) {
                ext_interp(At, St, L.cf.p, cmap.p, nc, prm.interp_pmax, Q, L.Tq, sg_flag.p, s);
                L.Sq = std::move(St);
            } else {
                direct_interp(At, St, L.cf.p, cmap.p, nc, Q, s);
            }
            transpose(Q.rowptr.p, Q.col.p, Q.val.p, Q.n, nc, Q.nnz, true, L.R, s);
        } else {
            transpose(L.P.rowptr.p, L.P.col.p, L.P.val.p, L.P.n, nc, L.P.nnz, true, L.R, s);
        }
        spgemm(A, L.P, L.AP, sg_flag.p, s);
        h->lev.emplace_back();
        Level& Ln = h->lev[l + 1];        // (reference after emplace_back)
        spgemm(h->lev[l].R, h->lev[l].AP, Ln.A, sg_flag.p, s);
        Ln.A.m = nc;
    }
    exact_sizes(h, sg_flag.p, s);
    build_coarse_inverse(h, h->lev.back().A, s);
    alloc_work(h, s);
    TP_HIP(hipStreamSynchronize(s));
}

// ---- the diagonal Schur approximation ----------------------------------------------------
// rows of A_pT (a copy, v) scaled by 1 / (A_pp)_ii; a zero or non-finite
// pivot sets *bad
__global__ void __launch_bounds__(B)
k_scale_rows_inv_diag(int32_t n, const int32_t* __restrict__ rowptr, const int32_t* __restrict__ col,
                      const double* __restrict__ pp, double* __restrict__ v, int32_t* __restrict__ bad) {
    const int32_t i = blockIdx.x * B + threadIdx.x;
    if (i >= n) return;
    double d = 0.0;
    for (int32_t q = rowptr[i]; q < rowptr[i + 1]; ++q)
        if (col[q] == i) d = pp[q];
    if (!(fabs(d) > 0.0 && fabs(d) <= DBL_MAX)) {
        *bad = 1;
        return;
    }
    for (int32_t q = rowptr[i]; q < rowptr[i + 1]; ++q) v[q] = v[q] / d;
}

// C <- A - C on C's pattern (sorted rows); an entry of A outside it sets *bad
__global__ void __launch_bounds__(B)
k_sub_from(int32_t n, const int32_t* __restrict__ crp, const int32_t* __restrict__ ccol, double* __restrict__ cval,
           const int32_t* __restrict__ arp, const int32_t* __restrict__ acol, const double* __restrict__ aval,
           int32_t* __restrict__ bad) {
    const int32_t i = blockIdx.x * B + threadIdx.x;
    if (i >= n) return;
    const int32_t e = crp[i + 1];
    for (int32_t q = crp[i]; q < e; ++q) cval[q] = -cval[q];
    int32_t qc = crp[i];
    for (int32_t k = arp[i]; k < arp[i + 1]; ++k) {
        const int32_t j = acol[k];
        while (qc < e && ccol[qc] < j) ++qc;
        if (qc < e && ccol[qc] == j) cval[qc] += aval[k];
        else *bad = 1;
    }
}

// S_diag = A_TT - A_Tp diag(A_pp)^{-1} A_pT on the distance-two pattern of the stencil
static void schur_diag(const tp_jacobian& J, Csr& S, hipStream_t s) {
    const int32_t n = J.n;
    Csr Tp, DpT;
    copy_csr_in(Tp, n, J.rowptr, J.col, J.Tp, s);
    copy_csr_in(DpT, n, J.rowptr, J.col, J.pT, s);
    DBuf<int32_t> flags(2, s);
    TP_LAUNCH(k_fill_i32, 1, B, 0, s, flags.p, 0, (int64_t)2);
    TP_LAUNCH(k_scale_rows_inv_diag, cdiv(n, B), B, 0, s, n, J.rowptr, J.col, J.pp, DpT.val.p, flags.p);
    spgemm(Tp, DpT, S, flags.p + 1, s);
    TP_LAUNCH(k_sub_from, cdiv(n, B), B, 0, s, n, S.rowptr.p, S.col.p, S.val.p, J.rowptr, J.col, J.TT, flags.p);
    int32_t f[2] = {0, 0};
    TP_HIP(hipMemcpyAsync(f, flags.p, sizeof(f), hipMemcpyDeviceToHost, s));
    TP_HIP(hipStreamSynchronize(s));
    if (f[1]) fail(TP_ERR_NUMERIC, "schur_diag: product row exceeds the SpGEMM table");
    if (f[0]) fail(TP_ERR_NUMERIC, "schur_diag: zero or non-finite A_pp diagonal, or A_TT outside the product pattern");
}

// ---- refreshing the finest level (hierarchy reuse across Newton iterations) -------------
struct DiaOffs {
    int32_t o[7];
};

__global__ void __launch_bounds__(B)
k_dia_refill(int32_t n, const int32_t* __restrict__ rowptr, const int32_t* __restrict__ col,
             const double* __restrict__ val, int nd, DiaOffs offs, double* __restrict__ dia) {
    int32_t i = blockIdx.x * B + threadIdx.x;
    if (i >= n) return;
    for (int d = 0; d < nd; ++d) dia[(int64_t)d * n + i] = 0.0;
    for (int32_t q = rowptr[i]; q < rowptr[i + 1]; ++q) {
        const int32_t o = col[q] - i;
        for (int d = 0; d < nd; ++d)
            if (offs.o[d] == o) dia[(int64_t)d * n + i] = val[q];
    }
}

// New values for level 0 (same pattern as at setup): the operator and
// everything derived from it alone (l1 diagonal, DIA copy, reduced-precision
// copies, the learned smoother's static features; the dense inverse when
// level 0 is the coarsest), all rewritten in place so that captured graphs of
// the V-cycle stay valid. Coarser levels, P and R are kept.
static void refresh_fine(tp_amg* h, const double* val, hipStream_t s) {
    Level& L = h->lev[0];
    const int32_t n = L.A.n;
    const int64_t nnz = L.A.nnz;
    TP_HIP(hipMemcpyAsync(L.A.val.p, val, sizeof(double) * nnz, hipMemcpyDeviceToDevice, s));
    TP_ROWS_LAUNCH(k_l1_dinv, row_group(n, nnz), n, s, n, L.A.rowptr.p, L.A.val.p, L.dinv.p);
    const int64_t nd_n = (int64_t)L.ndia * n;
    if (L.ndia) {
        DiaOffs o{};
        for (int d = 0; d < L.ndia; ++d) o.o[d] = L.dia_off[d];
        TP_LAUNCH(k_dia_refill, cdiv(n, B), B, 0, s, n, L.A.rowptr.p, L.A.col.p, L.A.val.p, L.ndia, o, L.dia.p);
    }
    if (h->prm.storage >= 1) {
        TP_LAUNCH(k_to_f32, cdiv(n, B), B, 0, s, (int64_t)n, L.dinv.p, L.dinv32.p);
        if (h->prm.storage == 1) {
            TP_LAUNCH(k_to_f32, cdiv(nnz, B), B, 0, s, nnz, L.A.val.p, L.A32.p);
            if (L.ndia) TP_LAUNCH(k_to_f32, cdiv(nd_n, B), B, 0, s, nd_n, L.dia.p, L.dia32.p);
        } else {
            TP_LAUNCH(k_split_bf16_csr, cdiv(n, B), B, 0, s, n, L.A.rowptr.p, L.A.col.p, L.A.val.p,
                      (__bf16*)L.A16.p, L.diag32.p);
            if (L.ndia) {
                int d0 = -1;
                for (int d = 0; d < L.ndia; ++d)
                    if (L.dia_off[d] == 0) d0 = d;
                TP_LAUNCH(k_split_bf16_dia, cdiv(nd_n, B), B, 0, s, nd_n, n, d0, L.dia.p, (__bf16*)L.dia16.p);
            }
        }
    }
    if (h->lev.size() == 1) build_coarse_inverse(h, L.A, s);
    if (h->cnn) cnn_attach_refresh(h->cnn.get(), L.A.rowptr.p, L.A.col.p, L.A.val.p, s);
}

// ---- numeric refresh: new level-0 values on a frozen hierarchy -------------------------
// Setup reuse across Newton iterations.  The C/F splits and every sparsity
// pattern (P, R, the kept A P and the coarse operators) stay; values are
// recomputed from the new finest-level operator in the setup's own order:
//   interpolation  direct interpolation restricted to the frozen set P_i:
//                  sum_all and lump as at setup; sum_p = sum of a_ij over the
//                  frozen j with s a_ij < 0 (row order); w_ij = -(alpha a_ij)
//                  / (a_ii + lump) for those j, an explicit zero for the
//                  other frozen entries, and a zero row where sum_p = 0.
//                  With the frozen set equal to the new strong C set this is
//                  the setup's direct interpolation, bit for bit;
//   restriction    R = P^T; or (Petrov-Galerkin) Q = the same construction
//                  on A^T over the frozen pattern of R^T, and R = Q^T;
//   coarse op.     A P and R (A P) on their kept patterns, each entry summed
//                  in ascending inner index from zero (the SpGEMM's order).
__global__ void __launch_bounds__(B)
k_refresh_interp(int32_t n, const int32_t* __restrict__ rowptr, const int32_t* __restrict__ col,
                 const double* __restrict__ val, const int32_t* __restrict__ cf,
                 const int32_t* __restrict__ cmap, const int32_t* __restrict__ Prp,
                 const int32_t* __restrict__ Pc, double* __restrict__ Pv) {
    const int32_t i = blockIdx.x * B + threadIdx.x;
    if (i >= n || cf[i]) return;  // C rows keep their unit entry
    const int32_t pa = Prp[i], pe = Prp[i + 1];
    if (pa == pe) return;
    const int32_t a = rowptr[i], e = rowptr[i + 1];
    double aii = 0.0;
    for (int32_t k = a; k < e; ++k)
        if (col[k] == i) aii = val[k];
    const double s = aii < 0.0 ? -1.0 : 1.0;
    double sum_all = 0.0, lump = 0.0;
    for (int32_t k = a; k < e; ++k) {
        if (col[k] == i) continue;
        const double v = val[k];
        if (s * v < 0.0) sum_all += v;
        else lump += v;
    }
    double sum_p = 0.0;
    int32_t q = pa;
    for (int32_t k = a; k < e; ++k) {
        const int32_t j = col[k];
        if (j == i || !cf[j]) continue;
        const int32_t c = cmap[j];
        while (q < pe && Pc[q] < c) ++q;
        if (q < pe && Pc[q] == c && s * val[k] < 0.0) sum_p += val[k];
    }
    for (int32_t t = pa; t < pe; ++t) Pv[t] = 0.0;
    if (sum_p == 0.0) return;
    const double alpha = sum_all / sum_p;
    const double dtil = aii + lump;
    q = pa;
    for (int32_t k = a; k < e; ++k) {
        const int32_t j = col[k];
        if (j == i || !cf[j]) continue;
        const int32_t c = cmap[j];
        while (q < pe && Pc[q] < c) ++q;
        if (q < pe && Pc[q] == c && s * val[k] < 0.0) Pv[q] = -(alpha * val[k]) / dtil;
    }
}

// T = X^T on T's kept (sorted) pattern: entry (i, J) of X goes to row J of T
// at column i, found by bisection.
__global__ void __launch_bounds__(B)
k_scatter_transpose(int32_t n, const int32_t* __restrict__ Xrp, const int32_t* __restrict__ Xc,
                    const double* __restrict__ Xv, const int32_t* __restrict__ Trp,
                    const int32_t* __restrict__ Tc, double* __restrict__ Tv) {
    const int32_t i = blockIdx.x * B + threadIdx.x;
    if (i >= n) return;
    for (int32_t q = Xrp[i]; q < Xrp[i + 1]; ++q) {
        const int32_t J = Xc[q];
        int32_t lo = Trp[J], hi = Trp[J + 1];
        while (lo < hi) {
            const int32_t mid = lo + (hi - lo) / 2;
            if (Tc[mid] < i) lo = mid + 1;
            else hi = mid;
        }
        Tv[lo] = Xv[q];
    }
}

// C = A B on C's kept pattern.  A group of G lanes per output row i: the
// row's output columns are staged in LDS; every product a_iq b_qc is placed
// at M[p][q] (p the position of c in the row, found by binary search; +0.0
// where row q of B lacks column p's), and each output entry sums its row of
// M over q ascending from 0.0 -- the order in which the SpGEMM sums it (an
// added +0.0 leaves a sum that is never -0.0 unchanged); the A entries are
// taken in chunks whose part of M fits, each output entry's sum carried in a
// register from chunk to chunk.  A row with more columns or A entries than
// fit takes the form of one lane per output entry, which searches row q of B
// for the entry's column in global memory.
template <int G, int VM, int VU, int VLA>
__global__ void __launch_bounds__(B)
k_spgemm_values(int32_t n, const int32_t* __restrict__ Crp, const int32_t* __restrict__ Cc,
                double* __restrict__ Cv, const int32_t* __restrict__ Arp, const int32_t* __restrict__ Ac,
                const double* __restrict__ Av, const int32_t* __restrict__ Brp,
                const int32_t* __restrict__ Bc, const double* __restrict__ Bv) {
    constexpr int NG = B / G;
    __shared__ double s_m[NG][VM];
    __shared__ int32_t s_c[NG][VU];
    __shared__ int32_t s_b0[NG][VLA], s_off[NG][VLA + 1];
    __shared__ double s_av[NG][VLA];
    const int g = threadIdx.x / G, lane = threadIdx.x % G;
    const int32_t i = blockIdx.x * NG + g;
    if (i >= n) return;  // (the whole group)
    const int32_t a0 = Arp[i], la = Arp[i + 1] - a0, c0 = Crp[i], u = Crp[i + 1] - c0;
    auto sync = [] {
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    };
    if (la > VLA || u > VU) {
        for (int32_t p = lane; p < u; p += G) {
            const int32_t c = Cc[c0 + p];
            double acc = 0.0;
            for (int32_t kk = a0; kk < a0 + la; ++kk) {
                const int32_t r = Ac[kk];
                int32_t l2 = Brp[r], h2 = Brp[r + 1] - 1;
                while (l2 <= h2) {
                    const int32_t mid = (l2 + h2) >> 1;
                    const int32_t v = Bc[mid];
                    if (v == c) { acc += Av[kk] * Bv[mid]; break; }
                    if (v < c) l2 = mid + 1;
                    else h2 = mid - 1;
                }
            }
            Cv[c0 + p] = acc;
        }
        return;
    }
    // the row's columns, and per A entry its B row and value with the
    // products' offsets (a scan over the group, VLA / G entries a lane)
    for (int32_t p = lane; p < u; p += G) s_c[g][p] = Cc[c0 + p];
    int32_t carry = 0;
    for (int32_t q0 = 0; q0 < la; q0 += G) {
        const int32_t q = q0 + lane;
        int32_t len = 0;
        if (q < la) {
            const int32_t r = Ac[a0 + q];
            const int32_t b0 = Brp[r];
            len = Brp[r + 1] - b0;
            s_b0[g][q] = b0;
            s_av[g][q] = Av[a0 + q];
        }
        int32_t inc = len;
#pragma unroll
        for (int d = 1; d < G; d <<= 1) {
            const int32_t o = __shfl_up(inc, d, G);
            if (lane >= d) inc += o;
        }
        if (q < la) s_off[g][q] = carry + inc - len;
        carry += __shfl(inc, G - 1, G);
    }
    if (lane == 0) s_off[g][la] = carry;
    constexpr int NE = VU / G;  // output entries a lane
    double acc[NE];
#pragma unroll
    for (int j = 0; j < NE; ++j) acc[j] = 0.0;
    const int32_t qc = u > 0 ? max(1, VM / u) : la;  // A entries a chunk
    for (int32_t q0 = 0; q0 < la; q0 += qc) {
        const int32_t q1 = min(la, q0 + qc), wq = q1 - q0;
        for (int32_t m = lane; m < u * wq; m += G) s_m[g][m] = 0.0;
        sync();
        const int32_t e1 = s_off[g][q1];
        for (int32_t e = s_off[g][q0] + lane; e < e1; e += G) {
            int32_t lo = q0, hi = q1 - 1;  // the last A entry whose first product is <= e
            while (lo < hi) {
                const int32_t mid = (lo + hi + 1) >> 1;
                if (s_off[g][mid] <= e) lo = mid;
                else hi = mid - 1;
            }
            const int32_t src = s_b0[g][lo] + (e - s_off[g][lo]);
            const int32_t c = Bc[src];
            int32_t pl = 0, ph = u - 1;  // its output position
            while (pl < ph) {
                const int32_t mid = (pl + ph) >> 1;
                if (s_c[g][mid] < c) pl = mid + 1;
                else ph = mid;
            }
            if (s_c[g][pl] == c) s_m[g][pl * wq + (lo - q0)] = s_av[g][lo] * Bv[src];
        }
        sync();
#pragma unroll
        for (int j = 0; j < NE; ++j) {
            const int32_t p = lane + j * G;
            if (p < u)
                for (int32_t q = 0; q < wq; ++q) acc[j] += s_m[g][p * wq + q];
        }
        sync();
    }
#pragma unroll
    for (int j = 0; j < NE; ++j) {
        const int32_t p = lane + j * G;
        if (p < u) Cv[c0 + p] = acc[j];
    }
}

static void spgemm_values(const Csr& A, const Csr& Bm, Csr& C, hipStream_t s) {
    if (C.nnz == 0 || C.n == 0) return;
    // products per output row, from the operands' mean row lengths
    const double est = ((double)A.nnz / std::max(A.n, 1)) * ((double)Bm.nnz / std::max(Bm.n, 1));
    if (est <= 48.0)
        TP_LAUNCH((k_spgemm_values<16, 256, 64, 16>), cdiv(C.n, B / 16), B, 0, s, C.n, C.rowptr.p, C.col.p,
                  C.val.p, A.rowptr.p, A.col.p, A.val.p, Bm.rowptr.p, Bm.col.p, Bm.val.p);
    else
        TP_LAUNCH((k_spgemm_values<64, 1024, 256, 64>), cdiv(C.n, B / 64), B, 0, s, C.n, C.rowptr.p, C.col.p,
                  C.val.p, A.rowptr.p, A.col.p, A.val.p, Bm.rowptr.p, Bm.col.p, Bm.val.p);
}

// Everything a level derives from its values alone: the DIA copy and the
// reduced-precision copies of A, 1/D, P and R (rewritten in place).
static void refresh_level_copies(tp_amg* h, Level& L, bool transfers, hipStream_t s) {
    const int32_t n = L.A.n;
    const int64_t nnz = L.A.nnz;
    const int64_t nd_n = (int64_t)L.ndia * n;
    if (L.ndia) {
        DiaOffs o{};
        for (int d = 0; d < L.ndia; ++d) o.o[d] = L.dia_off[d];
        TP_LAUNCH(k_dia_refill, cdiv(n, B), B, 0, s, n, L.A.rowptr.p, L.A.col.p, L.A.val.p, L.ndia, o, L.dia.p);
    }
    if (h->prm.storage == 0 || n == 0) return;
    TP_LAUNCH(k_to_f32, cdiv(n, B), B, 0, s, (int64_t)n, L.dinv.p, L.dinv32.p);
    if (h->prm.storage == 1) {
        TP_LAUNCH(k_to_f32, cdiv(nnz, B), B, 0, s, nnz, L.A.val.p, L.A32.p);
        if (L.ndia) TP_LAUNCH(k_to_f32, cdiv(nd_n, B), B, 0, s, nd_n, L.dia.p, L.dia32.p);
    } else {
        TP_LAUNCH(k_split_bf16_csr, cdiv(n, B), B, 0, s, n, L.A.rowptr.p, L.A.col.p, L.A.val.p, (__bf16*)L.A16.p,
                  L.diag32.p);
        if (L.ndia) {
            int d0 = -1;
            for (int d = 0; d < L.ndia; ++d)
                if (L.dia_off[d] == 0) d0 = d;
            TP_LAUNCH(k_split_bf16_dia, cdiv(nd_n, B), B, 0, s, nd_n, n, d0, L.dia.p, (__bf16*)L.dia16.p);
        }
    }
    if (transfers) {
        if (L.P.nnz) TP_LAUNCH(k_to_f32, cdiv(L.P.nnz, B), B, 0, s, (int64_t)L.P.nnz, L.P.val.p, L.P32.p);
        if (L.R.nnz) TP_LAUNCH(k_to_f32, cdiv(L.R.nnz, B), B, 0, s, (int64_t)L.R.nnz, L.R.val.p, L.R32.p);
    }
}

static void refresh_numeric(tp_amg* h, const double* val, hipStream_t s) {
    const bool ext = h->prm.interp == 1;
    const int nl = (int)h->lev.size();
    TP_HIP(hipMemcpyAsync(h->lev[0].A.val.p, val, sizeof(double) * h->lev[0].A.nnz, hipMemcpyDeviceToDevice, s));
    for (int l = 0; l < nl; ++l) {
        Level& L = h->lev[l];
        const int32_t n = L.A.n;
        if (n > 0) TP_ROWS_LAUNCH(k_l1_dinv, row_group(n, L.A.nnz), n, s, n, L.A.rowptr.p, L.A.val.p, L.dinv.p);
        if (l == nl - 1) break;
        DBuf<int32_t> cmap(n + 1, s);
        scan_exclusive(L.cf.p, cmap.p, n, s);
        if (ext) ext_fill(L.A, L.S, L.T, L.cf.p, cmap.p, L.P, h->prm.interp_pmax, 1, s);
        else
            TP_LAUNCH(k_refresh_interp, cdiv(n, B), B, 0, s, n, L.A.rowptr.p, L.A.col.p, L.A.val.p, L.cf.p, cmap.p,
                      L.P.rowptr.p, L.P.col.p, L.P.val.p);
        if (h->prm.restriction == 1) {
            Csr At, Q;
            transpose_square(L.A, l == 0, At, s);
            transpose(L.R.rowptr.p, L.R.col.p, L.R.val.p, L.R.n, n, L.R.nnz, true, Q, s);  // pattern of R^T
            if (ext) ext_fill(At, L.Sq, L.Tq, L.cf.p, cmap.p, Q, h->prm.interp_pmax, 1, s);
            else
                TP_LAUNCH(k_refresh_interp, cdiv(n, B), B, 0, s, n, At.rowptr.p, At.col.p, At.val.p, L.cf.p, cmap.p,
                          Q.rowptr.p, Q.col.p, Q.val.p);
            TP_LAUNCH(k_scatter_transpose, cdiv(n, B), B, 0, s, n, Q.rowptr.p, Q.col.p, Q.val.p, L.R.rowptr.p,
                      L.R.col.p, L.R.val.p);
        } else {
            TP_LAUNCH(k_scatter_transpose, cdiv(n, B), B, 0, s, n, L.P.rowptr.p, L.P.col.p, L.P.val.p,
                      L.R.rowptr.p, L.R.col.p, L.R.val.p);
        }
        spgemm_values(L.A, L.P, L.AP, s);
        spgemm_values(L.R, L.AP, h->lev[l + 1].A, s);
    }
    for (int l = 0; l < nl; ++l) refresh_level_copies(h, h->lev[l], l < nl - 1, s);
    build_coarse_inverse(h, h->lev.back().A, s);
    if (h->cnn) cnn_attach_refresh(h->cnn.get(), h->lev[0].A.rowptr.p, h->lev[0].A.col.p, h->lev[0].A.val.p, s);
}

}  // namespace tp

extern "C" {

int amg_setup(int32_t n, const int32_t* rowptr, const int32_t* col, const double* val,
              const tp_amg_params* params, tp_amg_t* out, void* stream) {
    TP_GUARD({
        TP_CHECK_ARG(out && params, "amg_setup: null argument");
        *out = nullptr;
        TP_CHECK_ARG(n >= 1 && rowptr && col && val, "amg_setup: empty or null matrix");
        const tp_amg_params& p = *params;
        TP_CHECK_ARG(p.theta > 0.0 && p.theta < 1.0, "amg_setup: theta must be in (0,1)");
        TP_CHECK_ARG(p.max_levels >= 1 && p.max_levels <= 25, "amg_setup: max_levels must be in [1,25]");
        TP_CHECK_ARG(p.coarse_max >= 0 && p.coarse_max <= 4096, "amg_setup: coarse_max must be in [0,4096]");
        TP_CHECK_ARG(p.smoother == 0 || p.smoother == 1, "amg_setup: smoother must be 0 or 1");
        TP_CHECK_ARG(p.smoother == 0 || (p.cheb_degree >= 1 && p.cheb_degree <= 16),
                     "amg_setup: cheb_degree must be in [1,16]");
        TP_CHECK_ARG(p.cheb_degree_coarse >= 0 && p.cheb_degree_coarse <= 16,
                     "amg_setup: cheb_degree_coarse must be in [0,16]");
        TP_CHECK_ARG(p.smoother == 0 || (p.cheb_lo > 0.0 && p.cheb_lo < 1.0), "amg_setup: cheb_lo in (0,1)");
        TP_CHECK_ARG(p.nu_pre >= 0 && p.nu_pre <= 8 && p.nu_post >= 0 && p.nu_post <= 8,
                     "amg_setup: sweeps must be in [0,8]");
        TP_CHECK_ARG(p.restriction == 0 || p.restriction == 1, "amg_setup: restriction must be 0 or 1");
        TP_CHECK_ARG(p.storage >= 0 && p.storage <= 2, "amg_setup: storage must be 0, 1 or 2");
        TP_CHECK_ARG(p.interp == 0 || p.interp == 1, "amg_setup: interp must be 0 or 1");
        TP_CHECK_ARG(p.interp_pmax >= 0 && p.interp_pmax <= tp::EXT_PMAX, "amg_setup: interp_pmax must be in [0,%d]",
                     tp::EXT_PMAX);
        hipStream_t s = (hipStream_t)stream;
        tp_amg* h = new tp_amg();
        h->prm = p;
        h->stream = s;
        try {
            tp::ArenaScope scope(&h->arena);
            tp::setup(h, n, rowptr, col, val, s);
        } catch (...) {
            delete h;
            throw;
        }
        *out = h;
    });
    return TP_OK;
}

int amg_setup_schur_diag(const tp_jacobian* J, const tp_amg_params* params, tp_amg_t* out, void* stream) {
    TP_GUARD({
        TP_CHECK_ARG(J && out && params, "amg_setup_schur_diag: null argument");
        *out = nullptr;
        TP_CHECK_ARG(J->n >= 1 && J->rowptr && J->col && J->pp && J->pT && J->Tp && J->TT,
                     "amg_setup_schur_diag: empty or null Jacobian");
        hipStream_t s = (hipStream_t)stream;
        tp::Csr S;
        tp::schur_diag(*J, S, s);
        return amg_setup(J->n, S.rowptr.p, S.col.p, S.val.p, params, out, stream);  // copies S
    });
    return TP_OK;
}

int amg_refresh_fine(tp_amg_t amg, const double* val, void* stream) {
    TP_GUARD({
        TP_CHECK_ARG(amg && val, "amg_refresh_fine: null argument");
        hipStream_t s = (hipStream_t)stream;
        tp::refresh_fine(amg, val, s);
        TP_HIP(hipStreamSynchronize(s));
    });
    return TP_OK;
}

int amg_refresh(tp_amg_t amg, const double* val, void* stream) {
    TP_GUARD({
        TP_CHECK_ARG(amg && val, "amg_refresh: null argument");
        hipStream_t s = (hipStream_t)stream;
        tp::refresh_numeric(amg, val, s);
        TP_HIP(hipStreamSynchronize(s));
    });
    return TP_OK;
}

int amg_num_levels(tp_amg_t amg, int32_t* nlev) {
    TP_GUARD({
        TP_CHECK_ARG(amg && nlev, "null argument");
        *nlev = (int32_t)amg->lev.size();
    });
    return TP_OK;
}

int amg_level_info(tp_amg_t amg, int32_t level, int32_t* n, int32_t* nnzA, int32_t* nnzP, int32_t* nnzR) {
    TP_GUARD({
        TP_CHECK_ARG(amg && n && nnzA && nnzP && nnzR, "null argument");
        TP_CHECK_ARG(level >= 0 && level < (int32_t)amg->lev.size(), "level out of range");
        const tp::Level& L = amg->lev[level];
        *n = L.A.n;
        *nnzA = L.A.nnz;
        *nnzP = L.P.nnz;
        *nnzR = L.R.nnz;
    });
    return TP_OK;
}

int amg_level_format(tp_amg_t amg, int32_t level, int32_t* ndia, int32_t* lanes) {
    TP_GUARD({
        TP_CHECK_ARG(amg && ndia && lanes, "null argument");
        TP_CHECK_ARG(level >= 0 && level < (int32_t)amg->lev.size(), "level out of range");
        *ndia = amg->lev[level].ndia;
        *lanes = amg->lev[level].gA;
    });
    return TP_OK;
}

int amg_level_copy(tp_amg_t amg, int32_t level, int32_t* A_rowptr, int32_t* A_col, double* A_val,
                   int32_t* cf, int32_t* P_rowptr, int32_t* P_col, double* P_val, int32_t* R_rowptr,
                   int32_t* R_col, double* R_val, void* stream) {
    TP_GUARD({
        TP_CHECK_ARG(amg, "null handle");
        TP_CHECK_ARG(level >= 0 && level < (int32_t)amg->lev.size(), "level out of range");
        hipStream_t s = (hipStream_t)stream;
        const tp::Level& L = amg->lev[level];
        auto cp = [&](void* dst, const void* src, size_t bytes) {
            if (dst && src && bytes) TP_HIP(hipMemcpyAsync(dst, src, bytes, hipMemcpyDeviceToDevice, s));
        };
        cp(A_rowptr, L.A.rowptr.p, sizeof(int32_t) * (L.A.n + 1));
        cp(A_col, L.A.col.p, sizeof(int32_t) * L.A.nnz);
        cp(A_val, L.A.val.p, sizeof(double) * L.A.nnz);
        cp(cf, L.cf.p, sizeof(int32_t) * L.A.n);
        if (L.P.nnz || L.P.n) {
            cp(P_rowptr, L.P.rowptr.p, sizeof(int32_t) * (L.P.n + 1));
            cp(P_col, L.P.col.p, sizeof(int32_t) * L.P.nnz);
            cp(P_val, L.P.val.p, sizeof(double) * L.P.nnz);
            cp(R_rowptr, L.R.rowptr.p, sizeof(int32_t) * (L.R.n + 1));
            cp(R_col, L.R.col.p, sizeof(int32_t) * L.R.nnz);
            cp(R_val, L.R.val.p, sizeof(double) * L.R.nnz);
        }
    });
    return TP_OK;
}

int amg_destroy(tp_amg_t amg) {
    TP_GUARD({
        if (!amg) return TP_OK;
        // the hierarchy may have been used on streams other than its setup
        // stream: wait for all device work before returning its memory
        TP_HIP(hipDeviceSynchronize());
        delete amg;
        TP_HIP(hipDeviceSynchronize());
    });
    return TP_OK;
}

}  // extern "C"
