// tp_vcycle.hip -- the AMG V(nu_pre, nu_post)-cycle on the GPU.
//
// One cycle from a zero guess on level l:
//   pre-smooth, r = b - A x, b_{l+1} = R r, recurse (explicit dense inverse
//   on the coarsest level), x += P x_{l+1}, post-smooth.
// Smoothers act on D^{-1} A with D_ii = sum_j |a_ij| (l1 diagonal):
//   l1-Jacobi   x <- x + w D^{-1}(b - A x)
//   Chebyshev   the polynomial iteration on [lo, 1] (Saad, Iterative
//               Methods for Sparse Linear Systems, 2nd ed., Sec. 12.3); by
//               Gershgorin the spectrum of D^{-1}A lies in the disc touching
//               1 from the left, so no eigenvalue estimate is needed.
// Every kernel streams its CSR arrays once: G lanes cooperate on a row (G
// a power of two near the mean row length, 64-lane wavefronts hold 64/G
// rows) so consecutive lanes read consecutive values and column indices.
// Vector type T is double (storage 0) or float (storage 1, 2); the level
// operator's values have type V = T, or, for storage 2, BF16 off-diagonal
// entries (V = __bf16, the diagonal entry stored as 0) with the diagonal in a
// separate FP32 array `diag` that the kernels add in (a null diag: none).
#include "tp_amg.h"

namespace tp {

constexpr int VB = 256;

// Workgroup -> tile map of the one-row-per-thread stencil kernels: the
// hardware hands workgroups to the 8 XCDs round-robin, so tile w would land
// on XCD w % 8 and every XCD's L2 would see every z-plane; here XCD x takes
// the contiguous tile range [x q + min(x, r), ...) (q = W / 8, r = W % 8),
// and the +-nx*ny neighbour planes a tile reads are mostly the ones its own
// XCD just streamed.  Measured on the FP32 hierarchies of the 256x256x64
// workload: -9% time per preconditioner apply (the two-row FP64 kernels got
// slower with it and keep the plain order).
__device__ inline int32_t xcd_tile() {
    const int32_t w = blockIdx.x, nw = gridDim.x, x = w % 8, q = nw / 8, r = nw % 8;
    return (x < r ? x * (q + 1) : r * (q + 1) + (x - r) * q) + w / 8;
}

template <typename T, int G>
__device__ inline T group_sum(T v) {
#pragma unroll
    for (int off = G / 2; off > 0; off >>= 1) v += __shfl_down(v, off, G);
    return v;
}

template <typename T, typename V, int G>
__device__ inline T row_dot(const int32_t* __restrict__ rp, const int32_t* __restrict__ ci,
                            const V* __restrict__ v, const T* __restrict__ x, int32_t i, int lane,
                            bool valid) {
    T s = 0;
    if (valid) {
        const int32_t e = rp[i + 1];
        for (int32_t q = rp[i] + lane; q < e; q += G) s += (T)v[q] * x[ci[q]];
    }
    return group_sum<T, G>(s);
}

// Chebyshev sweep step: r = D^{-1}(b - A x_in); d = first ? r/theta : c1 d + c2 r;
// x_out = x_in + d
template <typename T, typename V, int G>
__global__ void __launch_bounds__(VB)
k_cheb_step(int32_t n, const int32_t* __restrict__ rp, const int32_t* __restrict__ ci,
            const V* __restrict__ av, const T* __restrict__ diag, const T* __restrict__ dinv,
            const T* __restrict__ b, const T* __restrict__ xin, T* __restrict__ xout, T* __restrict__ d,
            int first, T theta, T c1, T c2) {
    const int64_t tid = (int64_t)blockIdx.x * VB + threadIdx.x;
    const int32_t i = (int32_t)(tid / G);
    const int lane = (int)(tid % G);
    const bool valid = i < n;
    const bool head = valid && lane == 0;
    // the row's own operands do not depend on the product: load them first
    T bi = 0, di = 0, xi = 0, dprev = 0;
    if (head) {
        bi = b[i];
        di = dinv[i];
        xi = xin[i];
        if (!first) dprev = d[i];
    }
    T ax = row_dot<T, V, G>(rp, ci, av, xin, i, lane, valid);
    if (head) {
        if (diag) ax += diag[i] * xi;
        T r = di * (bi - ax);
        T dn = first ? r / theta : c1 * dprev + c2 * r;
        d[i] = dn;
        xout[i] = xi + dn;
    }
}

template <typename T, typename V, int G>
__global__ void __launch_bounds__(VB)
k_jac_step(int32_t n, const int32_t* __restrict__ rp, const int32_t* __restrict__ ci,
           const V* __restrict__ av, const T* __restrict__ diag, const T* __restrict__ dinv,
           const T* __restrict__ b, const T* __restrict__ xin, T* __restrict__ xout, T w) {
    const int64_t tid = (int64_t)blockIdx.x * VB + threadIdx.x;
    const int32_t i = (int32_t)(tid / G);
    const int lane = (int)(tid % G);
    const bool valid = i < n;
    const bool head = valid && lane == 0;
    T bi = 0, di = 0, xi = 0;
    if (head) {
        bi = b[i];
        di = dinv[i];
        xi = xin[i];
    }
    T ax = row_dot<T, V, G>(rp, ci, av, xin, i, lane, valid);
    if (head && diag) ax += diag[i] * xi;
    if (head) xout[i] = xi + w * di * (bi - ax);
}

// r = b - A x
template <typename T, typename V, int G>
__global__ void __launch_bounds__(VB)
k_residual(int32_t n, const int32_t* __restrict__ rp, const int32_t* __restrict__ ci,
           const V* __restrict__ av, const T* __restrict__ diag, const T* __restrict__ b,
           const T* __restrict__ x, T* __restrict__ r) {
    const int64_t tid = (int64_t)blockIdx.x * VB + threadIdx.x;
    const int32_t i = (int32_t)(tid / G);
    const int lane = (int)(tid % G);
    const bool valid = i < n;
    const bool head = valid && lane == 0;
    const T bi = head ? b[i] : T(0);
    const T xd = head && diag ? diag[i] * x[i] : T(0);
    T ax = row_dot<T, V, G>(rp, ci, av, x, i, lane, valid);
    if (head) r[i] = bi - (diag ? ax + xd : ax);
}

// y = M x (restriction), or y += M x (prolongation, add = 1)
template <typename T, int G>
__global__ void __launch_bounds__(VB)
k_spmv(int32_t n, const int32_t* __restrict__ rp, const int32_t* __restrict__ ci,
       const T* __restrict__ av, const T* __restrict__ x, T* __restrict__ y, int add) {
    const int64_t tid = (int64_t)blockIdx.x * VB + threadIdx.x;
    const int32_t i = (int32_t)(tid / G);
    const int lane = (int)(tid % G);
    const bool valid = i < n;
    const bool head = valid && lane == 0;
    const T yi = head && add ? y[i] : T(0);
    T s = row_dot<T, T, G>(rp, ci, av, x, i, lane, valid);
    if (head) y[i] = add ? yi + s : s;
}

// ---- DIA (stencil-level) kernels: one thread per row, no column indices --------
template <int ND>
struct DiaOff {
    int32_t o[ND];
};

template <typename T, typename V, int ND>
__device__ inline T dia_dot(int32_t n, const V* __restrict__ dv, DiaOff<ND> off, const T* __restrict__ diag,
                            const T* __restrict__ x, int32_t i) {
    T s = 0;
#pragma unroll
    for (int d = 0; d < ND; ++d) {
        int32_t j = i + off.o[d];
        j = j < 0 ? 0 : (j >= n ? n - 1 : j);  // out-of-range slots hold 0
        s += (T)dv[(int64_t)d * n + i] * x[j];
    }
    if (diag) s += diag[i] * x[i];
    return s;
}

template <typename T, typename V, int ND>
__global__ void __launch_bounds__(VB)
k_cheb_step_dia(int32_t n, const V* __restrict__ dv, DiaOff<ND> off, const T* __restrict__ diag,
                const T* __restrict__ dinv, const T* __restrict__ b, const T* __restrict__ xin,
                T* __restrict__ xout, T* __restrict__ d, int first, T theta, T c1, T c2) {
    const int32_t i = xcd_tile() * VB + threadIdx.x;
    if (i >= n) return;
    T ax = dia_dot<T, V, ND>(n, dv, off, diag, xin, i);
    T r = dinv[i] * (b[i] - ax);
    T dn = first ? r / theta : c1 * d[i] + c2 * r;
    d[i] = dn;
    xout[i] = xin[i] + dn;
}

template <typename T, typename V, int ND>
__global__ void __launch_bounds__(VB)
k_jac_step_dia(int32_t n, const V* __restrict__ dv, DiaOff<ND> off, const T* __restrict__ diag,
               const T* __restrict__ dinv, const T* __restrict__ b, const T* __restrict__ xin,
               T* __restrict__ xout, T w) {
    const int32_t i = xcd_tile() * VB + threadIdx.x;
    if (i >= n) return;
    T ax = dia_dot<T, V, ND>(n, dv, off, diag, xin, i);
    xout[i] = xin[i] + w * dinv[i] * (b[i] - ax);
}

template <typename T, typename V, int ND>
__global__ void __launch_bounds__(VB)
k_residual_dia(int32_t n, const V* __restrict__ dv, DiaOff<ND> off, const T* __restrict__ diag,
               const T* __restrict__ b, const T* __restrict__ x, T* __restrict__ r) {
    const int32_t i = xcd_tile() * VB + threadIdx.x;
    if (i >= n) return;
    r[i] = b[i] - dia_dot<T, V, ND>(n, dv, off, diag, x, i);
}

// R consecutive rows per thread (2, in FP64): every row-indexed stream
// (diagonals, b, 1/D, d, x at the rows, the outputs) is read and written R
// elements at a time (16 bytes), which moves the same
// bytes with 1/R of the memory instructions; the neighbour reads x[i + off]
// stay per row. Each row's arithmetic is the one-row kernels', term for term,
// so the results are equal. Used when n is a multiple of R and every
// row-indexed array is aligned to R elements.
template <typename X, int R> struct VecR;
template <> struct VecR<double, 2> { using type = double2; };
template <typename X, int R>
__device__ inline void ldr(const X* p, X (&a)[R]) {
    const typename VecR<X, R>::type v = *(const typename VecR<X, R>::type*)p;
    const X* e = (const X*)&v;
#pragma unroll
    for (int r = 0; r < R; ++r) a[r] = e[r];
}
template <typename X, int R>
__device__ inline void str(X* p, const X (&a)[R]) {
    typename VecR<X, R>::type v;
    X* e = (X*)&v;
#pragma unroll
    for (int r = 0; r < R; ++r) e[r] = a[r];
    *(typename VecR<X, R>::type*)p = v;
}

// (A x)_{i+r}, r < R
template <typename T, typename V, int ND, int R>
__device__ inline void dia_dot_r(int32_t n, const V* __restrict__ dv, DiaOff<ND> off, const T* __restrict__ diag,
                                 const T* __restrict__ x, int32_t i, T (&s)[R]) {
#pragma unroll
    for (int r = 0; r < R; ++r) s[r] = 0;
#pragma unroll
    for (int d = 0; d < ND; ++d) {
        V a[R];
        ldr<V, R>(&dv[(int64_t)d * n + i], a);
#pragma unroll
        for (int r = 0; r < R; ++r) {
            int32_t j = i + r + off.o[d];
            j = j < 0 ? 0 : (j >= n ? n - 1 : j);  // out-of-range slots hold 0
            s[r] += (T)a[r] * x[j];
        }
    }
    if (diag) {
        T g[R], xi[R];
        ldr<T, R>(&diag[i], g);
        ldr<T, R>(&x[i], xi);
#pragma unroll
        for (int r = 0; r < R; ++r) s[r] += g[r] * xi[r];
    }
}

template <typename T, typename V, int ND, int VBk, int R>
__global__ void __launch_bounds__(VBk)
k_cheb_step_dia_r(int32_t n, const V* __restrict__ dv, DiaOff<ND> off, const T* __restrict__ diag,
                  const T* __restrict__ dinv, const T* __restrict__ b, const T* __restrict__ xin,
                  T* __restrict__ xout, T* __restrict__ d, int first, T theta, T c1, T c2) {
    const int32_t i = R * (blockIdx.x * VBk + threadIdx.x);
    if (i >= n) return;  // n is a multiple of R: rows i .. i + R - 1 exist
    T ax[R], di[R], bi[R], xi[R], dp[R], dn[R], xo[R];
    dia_dot_r<T, V, ND, R>(n, dv, off, diag, xin, i, ax);
    ldr<T, R>(&dinv[i], di);
    ldr<T, R>(&b[i], bi);
    ldr<T, R>(&xin[i], xi);
    if (!first) ldr<T, R>(&d[i], dp);
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const T rr = di[r] * (bi[r] - ax[r]);
        dn[r] = first ? rr / theta : c1 * dp[r] + c2 * rr;
        xo[r] = xi[r] + dn[r];
    }
    str<T, R>(&d[i], dn);
    str<T, R>(&xout[i], xo);
}

template <typename T, typename V, int ND, int VBk, int R>
__global__ void __launch_bounds__(VBk)
k_residual_dia_r(int32_t n, const V* __restrict__ dv, DiaOff<ND> off, const T* __restrict__ diag,
                 const T* __restrict__ b, const T* __restrict__ x, T* __restrict__ res) {
    const int32_t i = R * (blockIdx.x * VBk + threadIdx.x);
    if (i >= n) return;
    T ax[R], bi[R], o[R];
    dia_dot_r<T, V, ND, R>(n, dv, off, diag, x, i, ax);
    ldr<T, R>(&b[i], bi);
#pragma unroll
    for (int r = 0; r < R; ++r) o[r] = bi[r] - ax[r];
    str<T, R>(&res[i], o);
}

#define TP_ND_DISPATCH(nd, ...)                                 \
    switch (nd) {                                               \
    case 3: { constexpr int NDD = 3; __VA_ARGS__; } break;      \
    case 5: { constexpr int NDD = 5; __VA_ARGS__; } break;      \
    default: { constexpr int NDD = 7; __VA_ARGS__; } break;     \
    }

template <int ND>
static DiaOff<ND> dia_offsets(const Level& L) {
    DiaOff<ND> o;
    for (int d = 0; d < ND; ++d) o.o[d] = L.dia_off[d];
    return o;
}

// ---- fused kernels ----------------------------------------------------------------
// Chebyshev steps 0 and 1 from a zero guess in one pass: x0_j = (D^{-1} b)_j / theta
// is formed on the fly for every neighbour, then
//   r = D^{-1}(b - A x0); d = c1 x0_i + c2 r; x = x0_i + d.
template <typename T, typename V, int G>
__global__ void __launch_bounds__(VB)
k_cheb01(int32_t n, const int32_t* __restrict__ rp, const int32_t* __restrict__ ci, const V* __restrict__ av,
         const T* __restrict__ diag, const T* __restrict__ dinv, const T* __restrict__ b, T* __restrict__ xout,
         T* __restrict__ d, T theta, T c1, T c2) {
    const int64_t tid = (int64_t)blockIdx.x * VB + threadIdx.x;
    const int32_t i = (int32_t)(tid / G);
    const int lane = (int)(tid % G);
    const bool valid = i < n;
    const bool head = valid && lane == 0;
    T bi = 0, di = 0;
    if (head) {
        bi = b[i];
        di = dinv[i];
    }
    T s = 0;
    if (valid) {
        const int32_t e = rp[i + 1];
        for (int32_t q = rp[i] + lane; q < e; q += G) {
            const int32_t j = ci[q];
            s += (T)av[q] * ((dinv[j] * b[j]) / theta);
        }
    }
    s = group_sum<T, G>(s);
    if (head) {
        const T x0 = (di * bi) / theta;
        if (diag) s += diag[i] * x0;
        const T r = di * (bi - s);
        const T dn = c1 * x0 + c2 * r;
        d[i] = dn;
        xout[i] = x0 + dn;
    }
}

template <typename T, typename V, int ND>
__global__ void __launch_bounds__(VB)
k_cheb01_dia(int32_t n, const V* __restrict__ dv, DiaOff<ND> off, const T* __restrict__ diag,
             const T* __restrict__ dinv, const T* __restrict__ b, T* __restrict__ xout, T* __restrict__ d, T theta,
             T c1, T c2) {
    const int32_t i = xcd_tile() * VB + threadIdx.x;
    if (i >= n) return;
    T s = 0;
#pragma unroll
    for (int q = 0; q < ND; ++q) {
        int32_t j = i + off.o[q];
        j = j < 0 ? 0 : (j >= n ? n - 1 : j);
        s += (T)dv[(int64_t)q * n + i] * ((dinv[j] * b[j]) / theta);
    }
    const T x0 = (dinv[i] * b[i]) / theta;
    if (diag) s += diag[i] * x0;
    const T r = dinv[i] * (b[i] - s);
    const T dn = c1 * x0 + c2 * r;
    d[i] = dn;
    xout[i] = x0 + dn;
}

template <typename T, typename V, int ND, int VBk, int R>
__global__ void __launch_bounds__(VBk)
k_cheb01_dia_r(int32_t n, const V* __restrict__ dv, DiaOff<ND> off, const T* __restrict__ diag,
               const T* __restrict__ dinv, const T* __restrict__ b, T* __restrict__ xout, T* __restrict__ d,
               T theta, T c1, T c2) {
    const int32_t i = R * (blockIdx.x * VBk + threadIdx.x);
    if (i >= n) return;
    T sm[R], di[R], bi[R], x0[R], dn[R], xo[R];
#pragma unroll
    for (int r = 0; r < R; ++r) sm[r] = 0;
#pragma unroll
    for (int q = 0; q < ND; ++q) {
        V a[R];
        ldr<V, R>(&dv[(int64_t)q * n + i], a);
#pragma unroll
        for (int r = 0; r < R; ++r) {
            int32_t j = i + r + off.o[q];
            j = j < 0 ? 0 : (j >= n ? n - 1 : j);
            sm[r] += (T)a[r] * ((dinv[j] * b[j]) / theta);
        }
    }
    ldr<T, R>(&dinv[i], di);
    ldr<T, R>(&b[i], bi);
#pragma unroll
    for (int r = 0; r < R; ++r) x0[r] = (di[r] * bi[r]) / theta;
    if (diag) {
        T g[R];
        ldr<T, R>(&diag[i], g);
#pragma unroll
        for (int r = 0; r < R; ++r) sm[r] += g[r] * x0[r];
    }
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const T rr = di[r] * (bi[r] - sm[r]);
        dn[r] = c1 * x0[r] + c2 * rr;
        xo[r] = x0[r] + dn[r];
    }
    str<T, R>(&d[i], dn);
    str<T, R>(&xout[i], xo);
}

// Pre-smoothing by one step from a zero guess fused with the residual on a
// CSR level: x0 = (D^{-1} b)/theta (Chebyshev) or w D^{-1} b (l1-Jacobi) is
// formed on the fly for every neighbour, x = x0 (and d = x0) written for the
// row, and r = b - A x0 -- the products and sums of the two separate passes
// in the same order; one launch instead of two.
template <typename T, typename V, int G>
__global__ void __launch_bounds__(VB)
k_smooth0_res(int32_t n, const int32_t* __restrict__ rp, const int32_t* __restrict__ ci, const V* __restrict__ av,
              const T* __restrict__ diag, const T* __restrict__ dinv, const T* __restrict__ b, T* __restrict__ x,
              T* __restrict__ d, T* __restrict__ r, int cheb, T theta, T w) {
    const int64_t tid = (int64_t)blockIdx.x * VB + threadIdx.x;
    const int32_t i = (int32_t)(tid / G);
    const int lane = (int)(tid % G);
    const bool valid = i < n;
    const bool head = valid && lane == 0;
    T bi = 0, x0 = 0;
    if (head) {
        bi = b[i];
        x0 = cheb ? (dinv[i] * bi) / theta : w * dinv[i] * bi;
    }
    const T xd = head && diag ? diag[i] * x0 : T(0);
    T s = 0;
    if (valid) {
        const int32_t e = rp[i + 1];
        for (int32_t q = rp[i] + lane; q < e; q += G) {
            const int32_t j = ci[q];
            const T xj = cheb ? (dinv[j] * b[j]) / theta : w * dinv[j] * b[j];
            s += (T)av[q] * xj;
        }
    }
    s = group_sum<T, G>(s);
    if (head) {
        x[i] = x0;
        if (cheb) d[i] = x0;
        r[i] = bi - (diag ? s + xd : s);
    }
}

// Row-block (stream) form of the row products on a large CSR level: the
// workgroup takes rows [r0, r0 + rb); its threads stream the block's entries
// (consecutive threads, consecutive entries: every index and value load is
// coalesced across the wavefront) and put the products a_ij x_j in LDS;
// then thread t sums row r0 + t's products in entry order.  (The lane-group
// kernels read each row's entries through a group of lanes, so a wavefront's
// load touches a cache line per row it serves.)  MODE 0: a Chebyshev step
// as k_cheb_step; MODE 1: the residual r = b - A x as k_residual.
template <typename T, typename V, int MODE>
__global__ void __launch_bounds__(VB)
k_rows_stream(int32_t n, int32_t rb, const int32_t* __restrict__ rp, const int32_t* __restrict__ ci,
              const V* __restrict__ av, const T* __restrict__ diag, const T* __restrict__ dinv,
              const T* __restrict__ b, const T* __restrict__ xin, T* __restrict__ xout, T* __restrict__ d,
              int first, T theta, T c1, T c2) {
    extern __shared__ double s_raw[];  // (typed double for its alignment)
    T* const prod = reinterpret_cast<T*>(s_raw);
    const int32_t r0 = blockIdx.x * rb;
    const int32_t r1 = r0 + rb < n ? r0 + rb : n;
    const int32_t base = rp[r0], end = rp[r1];
    // the thread's own row (its extent and vector entries), loaded before
    // the products
    const int32_t i = r0 + (int32_t)threadIdx.x;
    const bool mine = (int32_t)threadIdx.x < rb && i < r1;
    const int32_t qa = mine ? rp[i] : 0, qe = mine ? rp[i + 1] : 0;
    const T bi = mine ? b[i] : T(0), xi = mine ? xin[i] : T(0);
    const T di = mine && diag ? diag[i] : T(0);
    const T dvi = mine && MODE == 0 ? dinv[i] : T(0);
    const T dprev = mine && MODE == 0 && !first ? d[i] : T(0);
    // four entries a thread before any product is formed: their loads are in
    // flight together
    for (int32_t e0 = base + threadIdx.x; e0 < end; e0 += 4 * VB) {
        int32_t cc[4];
        T aa[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int32_t e = e0 + u * VB;
            cc[u] = e < end ? ci[e] : 0;
            aa[u] = e < end ? (T)av[e] : T(0);
        }
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int32_t e = e0 + u * VB;
            if (e < end) prod[e - base] = aa[u] * xin[cc[u]];
        }
    }
    __syncthreads();
    if (!mine) return;
    T s = 0;
    for (int32_t q = qa - base; q < qe - base; ++q) s += prod[q];
    if (diag) s += di * xi;
    if (MODE == 1) {
        xout[i] = bi - s;
        return;
    }
    const T r = dvi * (bi - s);
    const T dn = first ? r / theta : c1 * dprev + c2 * r;
    d[i] = dn;
    xout[i] = xi + dn;
}

// y = A x, or y += A x (add), in the row-block form of k_rows_stream: the
// block's products in LDS, then one thread per row sums them in entry order
// (the transfers P and R on large levels; rb <= VB)
template <typename T>
__global__ void __launch_bounds__(VB)
k_spmv_stream(int32_t n, int32_t rb, const int32_t* __restrict__ rp, const int32_t* __restrict__ ci,
              const T* __restrict__ av, const T* __restrict__ x, T* __restrict__ y, int add) {
    extern __shared__ double s_raw[];  // (typed double for its alignment)
    T* const prod = reinterpret_cast<T*>(s_raw);
    const int32_t r0 = blockIdx.x * rb;
    const int32_t r1 = r0 + rb < n ? r0 + rb : n;
    const int32_t base = rp[r0], end = rp[r1];
    // the thread's own row: its extent and y, loaded before the products
    const int32_t i = r0 + (int32_t)threadIdx.x;
    const bool mine = (int32_t)threadIdx.x < rb && i < r1;
    const int32_t qa = mine ? rp[i] : 0, qe = mine ? rp[i + 1] : 0;
    const T yi = mine && add ? y[i] : T(0);
    for (int32_t e0 = base + threadIdx.x; e0 < end; e0 += 4 * VB) {
        int32_t cc[4];
        T aa[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int32_t e = e0 + u * VB;
            cc[u] = e < end ? ci[e] : 0;
            aa[u] = e < end ? av[e] : T(0);
        }
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int32_t e = e0 + u * VB;
            if (e < end) prod[e - base] = aa[u] * x[cc[u]];
        }
    }
    __syncthreads();
    if (!mine) return;
    T sum = 0;
    for (int32_t q = qa - base; q < qe - base; ++q) sum += prod[q];
    y[i] = add ? yi + sum : sum;
}

// first sweep from a zero guess
template <typename T>
__global__ void __launch_bounds__(VB)
k_smooth0(int32_t n, const T* __restrict__ dinv, const T* __restrict__ b, T* __restrict__ x,
          T* __restrict__ d, int cheb, T theta, T w) {
    int32_t i = blockIdx.x * VB + threadIdx.x;
    if (i >= n) return;
    if (cheb) {
        T r = dinv[i] * b[i];
        T dn = r / theta;
        d[i] = dn;
        x[i] = dn;
    } else {
        x[i] = w * dinv[i] * b[i];
    }
}

template <typename T>
__global__ void __launch_bounds__(VB)
k_zero(int32_t n, T* __restrict__ x) {
    int32_t i = blockIdx.x * VB + threadIdx.x;
    if (i < n) x[i] = 0;
}

// coarsest level: x = inv * b, one wavefront per row, FP64 accumulation
template <typename T>
__global__ void __launch_bounds__(VB)
k_coarse_solve(int32_t n, const double* __restrict__ inv, const T* __restrict__ b, T* __restrict__ x) {
    const int64_t tid = (int64_t)blockIdx.x * VB + threadIdx.x;
    const int32_t i = (int32_t)(tid / 64);
    const int lane = (int)(tid % 64);
    double s = 0.0;
    if (i < n)
        for (int32_t j = lane; j < n; j += 64) s += inv[(int64_t)i * n + j] * (double)b[j];
    s = group_sum<double, 64>(s);
    if (i < n && lane == 0) x[i] = (T)s;
}

// ---- dispatch ---------------------------------------------------------------------
#define TP_G_DISPATCH(G, ...)                                  \
    switch (G) {                                               \
    case 1: { constexpr int GG = 1; __VA_ARGS__; } break;      \
    case 2: { constexpr int GG = 2; __VA_ARGS__; } break;      \
    case 4: { constexpr int GG = 4; __VA_ARGS__; } break;      \
    case 8: { constexpr int GG = 8; __VA_ARGS__; } break;      \
    case 16: { constexpr int GG = 16; __VA_ARGS__; } break;    \
    case 32: { constexpr int GG = 32; __VA_ARGS__; } break;    \
    default: { constexpr int GG = 64; __VA_ARGS__; } break;    \
    }

// Storage modes: vector type T, level-operator value type V, and where each
// level array lives (diag: the separate FP32 diagonal of storage 2).
struct M64 { using T = double; using V = double; };
struct M32 { using T = float; using V = float; };
struct M16 { using T = float; using V = __bf16; };
template <typename M> struct LevelVals;
template <> struct LevelVals<M64> {
    static const double* D(const Level& L) { return L.dia.p; }
    static const double* A(const Level& L) { return L.A.val.p; }
    static const double* diag(const Level&) { return nullptr; }
    static const double* P(const Level& L) { return L.P.val.p; }
    static const double* R(const Level& L) { return L.R.val.p; }
    static const double* dinv(const Level& L) { return L.dinv.p; }
};
template <> struct LevelVals<M32> {
    static const float* D(const Level& L) { return L.dia32.p; }
    static const float* A(const Level& L) { return L.A32.p; }
    static const float* diag(const Level&) { return nullptr; }
    static const float* P(const Level& L) { return L.P32.p; }
    static const float* R(const Level& L) { return L.R32.p; }
    static const float* dinv(const Level& L) { return L.dinv32.p; }
};
template <> struct LevelVals<M16> {
    static const __bf16* D(const Level& L) { return (const __bf16*)L.dia16.p; }
    static const __bf16* A(const Level& L) { return (const __bf16*)L.A16.p; }
    static const float* diag(const Level& L) { return L.diag32.p; }
    static const float* P(const Level& L) { return L.P32.p; }
    static const float* R(const Level& L) { return L.R32.p; }
    static const float* dinv(const Level& L) { return L.dinv32.p; }
};

// ---- DIA launches: R rows per thread when n and the arrays allow it -------------------
template <typename X, int R>
static inline bool alr(const X* p) { return p == nullptr || ((uintptr_t)p % (R * sizeof(X))) == 0; }
// measured: 128-thread workgroups are faster up to ~131k threads, 256 above
static inline bool small_grid(int32_t n, int R) { return n / R <= 131072; }
// rows per thread: 2 in FP64 (16-byte accesses, 8-16% faster sweeps); in FP32 and
// with BF16 values several rows per thread measured no faster (W3 apply 0.92 ms
// either way; BF16 0.86 -> 0.96 ms with 4 rows), so one row
template <typename T>
static constexpr int rows_per_thread() { return sizeof(T) == 8 ? 2 : 1; }

#define TP_DIA_R_DISPATCH(R_, LAUNCH_R, LAUNCH_1)                                        \
    do {                                                                                \
        constexpr int RR = R_;                                                          \
        if constexpr (RR > 1) {                                                         \
            if (rows_ok) {                                                              \
                if (small_grid(n, RR)) { constexpr int BK = 128; LAUNCH_R; }            \
                else { constexpr int BK = 256; LAUNCH_R; }                              \
            } else {                                                                    \
                LAUNCH_1;                                                               \
            }                                                                           \
        } else {                                                                        \
            (void)rows_ok;                                                              \
            LAUNCH_1;                                                                   \
        }                                                                               \
    } while (0)

template <typename T, typename V>
static void dia_cheb_step(const Level& L, int32_t n, const V* D, const T* dg, const T* dv, const T* b, const T* xin,
                          T* xout, T* d, int first, T theta, T c1, T c2, hipStream_t s, bool timed, double bytes) {
    constexpr int R = rows_per_thread<T>();
    const bool rows_ok = n % R == 0 && alr<V, R>(D) && alr<T, R>(dg) && alr<T, R>(dv) && alr<T, R>(b) &&
                         alr<T, R>(xin) && alr<T, R>(xout) && alr<T, R>(d);
    TP_DIA_R_DISPATCH(
        R,
        TP_ND_DISPATCH(L.ndia, TP_LAUNCH_TIMED(timed, bytes, (k_cheb_step_dia_r<T, V, NDD, BK, RR>),
                                               cdiv(n / RR, BK), BK, 0, s, n, D, dia_offsets<NDD>(L), dg, dv, b,
                                               xin, xout, d, first, theta, c1, c2)),
        TP_ND_DISPATCH(L.ndia, TP_LAUNCH_TIMED(timed, bytes, (k_cheb_step_dia<T, V, NDD>), cdiv(n, VB), VB, 0, s, n, D,
                                               dia_offsets<NDD>(L), dg, dv, b, xin, xout, d, first, theta, c1, c2)));
}

template <typename T, typename V>
static void dia_cheb01(const Level& L, int32_t n, const V* D, const T* dg, const T* dv, const T* b, T* xout, T* d,
                       T theta, T c1, T c2, hipStream_t s, bool timed, double bytes) {
    constexpr int R = rows_per_thread<T>();
    const bool rows_ok = n % R == 0 && alr<V, R>(D) && alr<T, R>(dg) && alr<T, R>(dv) && alr<T, R>(b) &&
                         alr<T, R>(xout) && alr<T, R>(d);
    TP_DIA_R_DISPATCH(
        R,
        TP_ND_DISPATCH(L.ndia, TP_LAUNCH_TIMED(timed, bytes, (k_cheb01_dia_r<T, V, NDD, BK, RR>), cdiv(n / RR, BK),
                                               BK, 0, s, n, D, dia_offsets<NDD>(L), dg, dv, b, xout, d, theta, c1,
                                               c2)),
        TP_ND_DISPATCH(L.ndia, TP_LAUNCH_TIMED(timed, bytes, (k_cheb01_dia<T, V, NDD>), cdiv(n, VB), VB, 0, s, n, D,
                                               dia_offsets<NDD>(L), dg, dv, b, xout, d, theta, c1, c2)));
}

template <typename T, typename V>
static void dia_residual(const Level& L, int32_t n, const V* D, const T* dg, const T* b, const T* x, T* r,
                         hipStream_t s) {
    constexpr int R = rows_per_thread<T>();
    const bool rows_ok =
        n % R == 0 && alr<V, R>(D) && alr<T, R>(dg) && alr<T, R>(b) && alr<T, R>(x) && alr<T, R>(r);
    TP_DIA_R_DISPATCH(
        R,
        TP_ND_DISPATCH(L.ndia, TP_LAUNCH((k_residual_dia_r<T, V, NDD, BK, RR>), cdiv(n / RR, BK), BK, 0, s, n, D,
                                         dia_offsets<NDD>(L), dg, b, x, r)),
        TP_ND_DISPATCH(L.ndia, TP_LAUNCH((k_residual_dia<T, V, NDD>), cdiv(n, VB), VB, 0, s, n, D,
                                         dia_offsets<NDD>(L), dg, b, x, r)));
}

static inline int grid_rows(int32_t n, int G) { return cdiv((int64_t)std::max(n, 1) * G, VB); }

// smoothing sweeps on level L; x_cur in/out (ping-pong between x and x2)
// final_out (optional): buffer for the sweep's last step, so the result can
// land in the caller's vector; the returned pointer says where it is.
template <typename M>
static typename M::T* smooth(tp_amg* h, int l, const typename M::T* b, typename M::T* xc, bool zero, int nu,
                             hipStream_t s, typename M::T* final_out = nullptr) {
    using T = typename M::T;
    using V = typename M::V;
    Level& L = h->lev[l];
    const tp_amg_params& p = h->prm;
    const int32_t n = L.A.n;
    const V* av = LevelVals<M>::A(L);
    const T* dg = LevelVals<M>::diag(L);
    const T* dv = LevelVals<M>::dinv(L);
    T* xa = (T*)L.x.p;
    T* xb = (T*)L.x2.p;
    T* d = (T*)L.d.p;
    T* cur = xc;
    auto other = [&](T* q) { return q == xa ? xb : xa; };
    auto target = [&](T* q, bool last) { return last && final_out ? final_out : other(q); };
    const double lo = p.cheb_lo, theta = 0.5 * (1.0 + lo), delta = 0.5 * (1.0 - lo);
    const double sigma = theta / delta;
    const size_t es = sizeof(T), vs = sizeof(V);
    // bytes of one pass over the level operator (values, indices, separate diagonal)
    const double abytes = (L.ndia ? (double)L.ndia * n * vs : (double)L.A.nnz * (vs + 4) + 4.0 * (n + 1)) +
                          (dg ? (double)es * n : 0.0);
    const int deg = (l > 0 && p.cheb_degree_coarse > 0) ? p.cheb_degree_coarse : p.cheb_degree;
    for (int sw = 0; sw < nu; ++sw) {
        bool z = zero && sw == 0;
        bool fused01 = false;
        if (z && p.smoother == 1 && deg >= 2) {
            // steps 0 and 1 in one pass
            const double rho1 = 1.0 / (2.0 * sigma - 1.0 / sigma);
            const double c1 = rho1 * (1.0 / sigma), c2 = 2.0 * rho1 / delta;
            T* nx = target(cur, sw == nu - 1 && deg == 2);
            const bool timed = false;  // the timer follows the Chebyshev step kernel alone
            const double bytes = abytes + 4.0 * es * n;
            if (L.ndia) {
                dia_cheb01<T, V>(L, n, LevelVals<M>::D(L), dg, dv, b, nx, d, (T)theta, (T)c1, (T)c2, s, timed,
                                 bytes);
            } else {
                TP_G_DISPATCH(L.gA, TP_LAUNCH_TIMED(timed, bytes, (k_cheb01<T, V, GG>), grid_rows(n, GG), VB, 0, s, n,
                                                    L.A.rowptr.p, L.A.col.p, av, dg, dv, b, nx, d, (T)theta, (T)c1,
                                                    (T)c2));
            }
            cur = nx;
            fused01 = true;
        } else if (z) {
            TP_LAUNCH(k_smooth0<T>, cdiv(n, VB), VB, 0, s, n, dv, b, cur, d, p.smoother == 1, (T)theta,
                      (T)p.omega);
        }
        if (p.smoother == 0) {
            if (z) continue;
            T* nx = target(cur, sw == nu - 1);
            double bytes = abytes + 4.0 * es * n;
            const bool timed = l == 0;
            if (L.ndia) {
                TP_ND_DISPATCH(L.ndia, TP_LAUNCH_TIMED(timed, bytes, (k_jac_step_dia<T, V, NDD>), cdiv(n, VB), VB, 0,
                                                       s, n, LevelVals<M>::D(L), dia_offsets<NDD>(L), dg, dv, b, cur,
                                                       nx, (T)p.omega));
            } else {
                TP_G_DISPATCH(L.gA, TP_LAUNCH_TIMED(timed, bytes, (k_jac_step<T, V, GG>), grid_rows(n, GG), VB, 0, s,
                                                    n, L.A.rowptr.p, L.A.col.p, av, dg, dv, b, cur, nx, (T)p.omega));
            }
            cur = nx;
            continue;
        }
        double rho0 = 1.0 / sigma;
        int k0 = 0;
        if (z) k0 = 1;  // first Chebyshev step done by k_smooth0
        if (fused01) {  // steps 0 and 1 done by k_cheb01
            k0 = 2;
            rho0 = 1.0 / (2.0 * sigma - rho0);
        }
        for (int k = k0; k < deg; ++k) {
            T* nx = target(cur, sw == nu - 1 && k == deg - 1);
            int first = (k == 0);
            double c1 = 0.0, c2 = 0.0;
            if (!first) {
                double rho1 = 1.0 / (2.0 * sigma - rho0);
                c1 = rho1 * rho0;
                c2 = 2.0 * rho1 / delta;
                rho0 = rho1;
            }
            double bytes = abytes + (first ? 5.0 : 6.0) * es * n;
            const bool timed = l == 0;
            if (L.ndia) {
                dia_cheb_step<T, V>(L, n, LevelVals<M>::D(L), dg, dv, b, cur, nx, d, first, (T)theta, (T)c1, (T)c2,
                                    s, timed, bytes);
            } else if (L.sb_rows) {
                TP_LAUNCH((k_rows_stream<T, V, 0>), cdiv(n, L.sb_rows), VB, (size_t)L.sb_lds * sizeof(T), s, n,
                          L.sb_rows, L.A.rowptr.p, L.A.col.p, av, dg, dv, b, cur, nx, d, first, (T)theta, (T)c1,
                          (T)c2);
            } else {
                TP_G_DISPATCH(L.gA, TP_LAUNCH_TIMED(timed, bytes, (k_cheb_step<T, V, GG>), grid_rows(n, GG), VB, 0, s,
                                                    n, L.A.rowptr.p, L.A.col.p, av, dg, dv, b, cur, nx, d, first,
                                                    (T)theta, (T)c1, (T)c2));
            }
            cur = nx;
        }
    }
    return cur;
}

template <typename M>
static typename M::T* vcycle_level(tp_amg* h, int l, const typename M::T* b, hipStream_t s,
                                   typename M::T* final_out = nullptr) {
    using T = typename M::T;
    using V = typename M::V;
    Level& L = h->lev[l];
    const int32_t n = L.A.n;
    const int last = (int)h->lev.size() - 1;
    T* x = (T*)L.x.p;
    if (l == last) {
        TP_LAUNCH(k_coarse_solve<T>, cdiv((int64_t)std::max(n, 1) * 64, VB), VB, 0, s, n, h->cinv.p, b, x);
        return x;
    }
    const tp_amg_params& p = h->prm;
    T* cur = x;
    T* r = (T*)L.r.p;
    // a pre-smoothing that is a single step from zero on a small CSR level
    // (the coarse levels of the degree-1 schedule) runs fused with the
    // residual: one launch fewer.  On levels of >= 65536 rows the two passes
    // are cheaper than the fused one, which gathers D^{-1} and b at every
    // neighbour instead of x (first coarse level of the 256x256x64 pressure
    // hierarchy: 186 us fused against ~145 us for the pair).
    const int deg = (l > 0 && p.cheb_degree_coarse > 0) ? p.cheb_degree_coarse : p.cheb_degree;
    if (p.nu_pre == 1 && !L.ndia && (p.smoother == 0 || deg == 1) && n < 65536) {
        const double theta = 0.5 * (1.0 + p.cheb_lo);
        TP_G_DISPATCH(L.gA, TP_LAUNCH((k_smooth0_res<T, V, GG>), grid_rows(n, GG), VB, 0, s, n, L.A.rowptr.p,
                                      L.A.col.p, LevelVals<M>::A(L), LevelVals<M>::diag(L), LevelVals<M>::dinv(L),
                                      b, cur, (T*)L.d.p, r, p.smoother == 1, (T)theta, (T)p.omega));
    } else {
        if (p.nu_pre > 0) cur = smooth<M>(h, l, b, cur, true, p.nu_pre, s);
        else TP_LAUNCH(k_zero<T>, cdiv(n, VB), VB, 0, s, n, cur);
        // (residual and restriction stay two row-parallel passes: forming the
        // residual entries inside the restriction recomputes each fine row for
        // every coarse row that holds it and serialises its gathers)
        if (L.ndia) {
            dia_residual<T, V>(L, n, LevelVals<M>::D(L), LevelVals<M>::diag(L), b, cur, r, s);
        } else if (L.sb_rows) {
            TP_LAUNCH((k_rows_stream<T, V, 1>), cdiv(n, L.sb_rows), VB, (size_t)L.sb_lds * sizeof(T), s, n,
                      L.sb_rows, L.A.rowptr.p, L.A.col.p, LevelVals<M>::A(L), LevelVals<M>::diag(L),
                      (const T*)nullptr, b, cur, r, (T*)nullptr, 0, (T)0, (T)0, (T)0);
        } else {
            TP_G_DISPATCH(L.gA, TP_LAUNCH((k_residual<T, V, GG>), grid_rows(n, GG), VB, 0, s, n, L.A.rowptr.p,
                                          L.A.col.p, LevelVals<M>::A(L), LevelVals<M>::diag(L), b, cur, r));
        }
    }
    Level& Ln = h->lev[l + 1];
    T* bc = (T*)Ln.b.p;
    if (L.sbR_rows)
        TP_LAUNCH(k_spmv_stream<T>, cdiv(L.R.n, L.sbR_rows), VB, (size_t)L.sbR_lds * sizeof(T), s, L.R.n,
                  L.sbR_rows, L.R.rowptr.p, L.R.col.p, LevelVals<M>::R(L), r, bc, 0);
    else
        TP_G_DISPATCH(L.gR, TP_LAUNCH((k_spmv<T, GG>), grid_rows(L.R.n, GG), VB, 0, s, L.R.n, L.R.rowptr.p,
                                      L.R.col.p, LevelVals<M>::R(L), r, bc, 0));
    T* xc = vcycle_level<M>(h, l + 1, bc, s);
    // (prolongation stays a separate row-parallel pass: fusing it into the
    // first post-smoothing step recomputes P x_c for every neighbour and
    // turns the step latency-bound)
    if (L.sbP_rows)
        TP_LAUNCH(k_spmv_stream<T>, cdiv(n, L.sbP_rows), VB, (size_t)L.sbP_lds * sizeof(T), s, n, L.sbP_rows,
                  L.P.rowptr.p, L.P.col.p, LevelVals<M>::P(L), xc, cur, 1);
    else
        TP_G_DISPATCH(L.gP, TP_LAUNCH((k_spmv<T, GG>), grid_rows(n, GG), VB, 0, s, n, L.P.rowptr.p, L.P.col.p,
                                      LevelVals<M>::P(L), xc, cur, 1));
    if (l == 0 && h->stop_before_post) return cur;
    if (l == 0 && h->cnn && h->cnn->enabled) {
        // learned post-smoother: r = b - A x; x += s * CNN(features(r))
        if (L.ndia) {
            dia_residual<T, V>(L, n, LevelVals<M>::D(L), LevelVals<M>::diag(L), b, cur, r, s);
        } else {
            TP_G_DISPATCH(L.gA, TP_LAUNCH((k_residual<T, V, GG>), grid_rows(n, GG), VB, 0, s, n, L.A.rowptr.p,
                                          L.A.col.p, LevelVals<M>::A(L), LevelVals<M>::diag(L), b, cur, r));
        }
        tp_cnn_attach* a = h->cnn.get();
        cnn_features_into<T>(a, r, a->feat.p, s, false);
        cnn_smooth_fused<T>(a, cur, s);
        return cur;
    }
    if (p.nu_post > 0) cur = smooth<M>(h, l, b, cur, false, p.nu_post, s, final_out);
    return cur;
}

const void* vcycle_run(tp_amg* h, const void* b_ext, hipStream_t s, void* x_ext) {
    const void* b = b_ext ? b_ext : (const void*)h->lev[0].b.p;
    if (h->prm.storage == 2) return vcycle_level<M16>(h, 0, (const float*)b, s, (float*)x_ext);
    if (h->prm.storage == 1) return vcycle_level<M32>(h, 0, (const float*)b, s, (float*)x_ext);
    return vcycle_level<M64>(h, 0, (const double*)b, s, (double*)x_ext);
}

template <typename Ti, typename To>
__global__ void __launch_bounds__(VB)
k_cast(int32_t n, const Ti* __restrict__ a, To* __restrict__ b) {
    int32_t i = blockIdx.x * VB + threadIdx.x;
    if (i < n) b[i] = (To)a[i];
}

// host helpers used by the preconditioner (kernels only, so the apply can
// be captured in a graph without copy or fill nodes)
void cast_d2s(int32_t n, const double* a, void* b, size_t es, hipStream_t s) {
    if (es == 4) TP_LAUNCH((k_cast<double, float>), cdiv(n, VB), VB, 0, s, n, a, (float*)b);
    else TP_LAUNCH((k_cast<double, double>), cdiv(n, VB), VB, 0, s, n, a, (double*)b);
}
void cast_s2d(int32_t n, const void* a, double* b, size_t es, hipStream_t s) {
    if (es == 4) TP_LAUNCH((k_cast<float, double>), cdiv(n, VB), VB, 0, s, n, (const float*)a, b);
    else TP_LAUNCH((k_cast<double, double>), cdiv(n, VB), VB, 0, s, n, (const double*)a, b);
}

}  // namespace tp

namespace tp {

__global__ void __launch_bounds__(VB)
k_pair_finish(int32_t n, const double* __restrict__ y, const double* __restrict__ x, double* __restrict__ e) {
    int32_t i = blockIdx.x * VB + threadIdx.x;
    if (i < n) e[i] = y[i] - x[i];
}

}  // namespace tp

extern "C" int amg_presmoothed_pair(tp_amg_t amg, const double* y, double* r, double* e, void* stream) {
    TP_GUARD({
        TP_CHECK_ARG(amg && y && r && e, "amg_presmoothed_pair: null argument");
        TP_CHECK_ARG(amg->lev.size() >= 2, "amg_presmoothed_pair: needs at least two levels");
        hipStream_t s = (hipStream_t)stream;
        tp::Level& L = amg->lev[0];
        const int32_t n = L.A.n;
        // b = A y (FP64 level operator)
        tp::DBuf<double> b(n, s), x(n, s);
        TP_G_DISPATCH(L.gA, TP_LAUNCH((tp::k_spmv<double, GG>), tp::grid_rows(n, GG), tp::VB, 0, s, n,
                                      L.A.rowptr.p, L.A.col.p, L.A.val.p, y, b.p, 0));
        const size_t es = tp::storage_bytes(amg);
        tp::cast_d2s(n, b.p, amg->lev[0].b.p, es, s);
        amg->stop_before_post = true;
        const void* xv = nullptr;
        try {
            xv = tp::vcycle_run(amg, nullptr, s);
        } catch (...) {
            amg->stop_before_post = false;
            throw;
        }
        amg->stop_before_post = false;
        tp::cast_s2d(n, xv, x.p, es, s);
        TP_G_DISPATCH(L.gA, TP_LAUNCH((tp::k_residual<double, double, GG>), tp::grid_rows(n, GG), tp::VB, 0, s, n,
                                      L.A.rowptr.p, L.A.col.p, L.A.val.p, (const double*)nullptr, b.p, x.p, r));
        TP_LAUNCH(tp::k_pair_finish, tp::cdiv(n, tp::VB), tp::VB, 0, s, n, y, x.p, e);
        TP_HIP(hipStreamSynchronize(s));
    });
    return TP_OK;
}

extern "C" int amg_attach_post_smoother(tp_amg_t amg, tp_cnn_t net, const tp_grid* grid) {
    TP_GUARD({
        TP_CHECK_ARG(amg, "amg_attach_post_smoother: null hierarchy");
        ++amg->cnn_gen;  // a graph captured with the previous attachment is stale
        if (!net) {
            amg->cnn.reset();
            return TP_OK;
        }
        TP_CHECK_ARG(grid, "amg_attach_post_smoother: null grid");
        const int64_t n = (int64_t)grid->nx * grid->ny * grid->nz;
        TP_CHECK_ARG(n == amg->lev[0].A.n, "amg_attach_post_smoother: grid has %lld cells, level 0 has %d rows",
                     (long long)n, amg->lev[0].A.n);
        TP_CHECK_ARG(amg->lev.size() >= 2, "amg_attach_post_smoother: needs at least two levels");
        hipStream_t s = amg->stream;
        auto a = std::make_unique<tp::tp_cnn_attach>();
        a->net = net;
        const tp::Level& L = amg->lev[0];
        tp::cnn_attach_build(a.get(), *grid, L.A.rowptr.p, L.A.col.p, L.A.val.p, s);
        TP_LAUNCH(tp::k_zero<int32_t>, 1, tp::VB, 0, s, 1, a->bad.p);
        TP_HIP(hipStreamSynchronize(s));
        amg->cnn = std::move(a);
    });
    return TP_OK;
}

extern "C" int amg_features(tp_amg_t amg, const double* r, float* feat, float* scale, void* stream) {
    TP_GUARD({
        TP_CHECK_ARG(amg && r && feat, "amg_features: null argument");
        TP_CHECK_ARG(amg->cnn, "amg_features: no network attached (amg_attach_post_smoother)");
        hipStream_t s = (hipStream_t)stream;
        tp::tp_cnn_attach* a = amg->cnn.get();
        const int32_t n = amg->lev[0].A.n;
        TP_HIP(hipMemcpyAsync(feat + n, a->feat.p + n, sizeof(float) * 7 * (size_t)n, hipMemcpyDeviceToDevice, s));
        tp::cnn_features_into<double>(a, r, feat, s);
        if (scale) {
            TP_HIP(hipMemcpyAsync(scale, a->scale.p, sizeof(float), hipMemcpyDeviceToHost, s));
            TP_HIP(hipStreamSynchronize(s));
        }
    });
    return TP_OK;
}

extern "C" int amg_cnn_loss_grad(tp_amg_t amg, const float* feat, const float* target, float err_weight,
                                 double* loss, void* stream) {
    TP_GUARD({
        TP_CHECK_ARG(amg && feat && target, "amg_cnn_loss_grad: null argument");
        TP_CHECK_ARG(amg->cnn, "amg_cnn_loss_grad: no network attached");
        TP_CHECK_ARG(err_weight >= 0.f && std::isfinite(err_weight), "amg_cnn_loss_grad: err_weight must be finite and >= 0");
        hipStream_t s = (hipStream_t)stream;
        const tp::Level& L = amg->lev[0];
        tp::cnn_op_loss_grad(amg->cnn.get(), L.A.rowptr.p, L.A.col.p, L.A.val.p, L.A.nnz, feat, target, err_weight,
                             s);
        if (loss) {
            TP_HIP(hipMemcpyAsync(loss, amg->cnn->net->loss.p, sizeof(double), hipMemcpyDeviceToHost, s));
            TP_HIP(hipStreamSynchronize(s));
        }
    });
    return TP_OK;
}

namespace tp {
// a read pass over fl[0, n) that evicts the last-level cache and leaves it
// holding clean lines (no write-back competes with the timed launch); the
// store never happens for finite data and only keeps the loads
__global__ void __launch_bounds__(VB)
k_flush(int64_t n, double* __restrict__ fl) {
    const int64_t i = (int64_t)blockIdx.x * VB + threadIdx.x;
    const double v = i < n ? fl[i] : 0.0;
    if (v != v) fl[0] = 0.0;
}

// With fl (flush_n doubles): every launch follows a sweep of fl and is timed
// by an event pair of its own; the mean of those times is returned.
template <typename M>
static double replay_fine_smoother(tp_amg* h, int reps, hipStream_t s, double* bytes, double* fl = nullptr,
                                   int64_t flush_n = 0) {
    using T = typename M::T;
    using V = typename M::V;
    Level& L = h->lev[0];
    const int32_t n = L.A.n;
    const size_t es = sizeof(T), vs = sizeof(V);
    const T* dg = LevelVals<M>::diag(L);
    T* xa = (T*)L.x.p;
    T* xb = (T*)L.x2.p;
    T* d = (T*)L.d.p;
    T* b = (T*)L.b.p;
    for (T* v : {xa, xb, d, b}) TP_LAUNCH(k_zero<T>, cdiv(n, VB), VB, 0, s, n, v);
    const T* dv = LevelVals<M>::dinv(L);
    const double lo = h->prm.cheb_lo, theta = 0.5 * (1.0 + lo), delta = 0.5 * (1.0 - lo), sigma = theta / delta;
    const double rho1 = 1.0 / (2.0 * sigma - 1.0 / sigma), c1 = rho1 / sigma, c2 = 2.0 * rho1 / delta;
    hipEvent_t e0, e1;
    TP_HIP(hipEventCreate(&e0));
    TP_HIP(hipEventCreate(&e1));
    std::vector<hipEvent_t> ev;  // (flushed: a pair per launch)
    if (fl)
        for (int k = 0; k < 2 * reps; ++k) {
            hipEvent_t e;
            TP_HIP(hipEventCreate(&e));
            ev.push_back(e);
        }
    TP_HIP(hipEventRecord(e0, s));
    for (int k = 0; k < reps; ++k) {
        T* in = (k & 1) ? xb : xa;
        T* out = (k & 1) ? xa : xb;
        if (fl) {
            TP_LAUNCH(k_flush, cdiv(flush_n, VB), VB, 0, s, flush_n, fl);
            TP_HIP(hipEventRecord(ev[2 * k], s));
        }
        if (L.ndia) {
            dia_cheb_step<T, V>(L, n, LevelVals<M>::D(L), dg, dv, b, in, out, d, 0, (T)theta, (T)c1, (T)c2, s,
                                false, 0.0);
        } else {
            TP_G_DISPATCH(L.gA, TP_LAUNCH((k_cheb_step<T, V, GG>), grid_rows(n, GG), VB, 0, s, n, L.A.rowptr.p,
                                          L.A.col.p, LevelVals<M>::A(L), dg, dv, b, in, out, d, 0, (T)theta,
                                          (T)c1, (T)c2));
        }
        if (fl) TP_HIP(hipEventRecord(ev[2 * k + 1], s));
    }
    TP_HIP(hipEventRecord(e1, s));
    TP_HIP(hipEventSynchronize(e1));
    float ms = 0.f;
    TP_HIP(hipEventElapsedTime(&ms, e0, e1));
    if (fl) {
        ms = 0.f;
        for (int k = 0; k < reps; ++k) {
            float t = 0.f;
            TP_HIP(hipEventElapsedTime(&t, ev[2 * k], ev[2 * k + 1]));
            ms += t;
        }
        for (hipEvent_t e : ev) (void)hipEventDestroy(e);
    }
    TP_HIP(hipEventDestroy(e0));
    TP_HIP(hipEventDestroy(e1));
    *bytes = (L.ndia ? (double)L.ndia * n * vs : (double)L.A.nnz * (vs + 4) + 4.0 * (n + 1)) +
             (dg ? (double)es * n : 0.0) + 6.0 * es * n;
    return (double)ms / reps;
}
}  // namespace tp

extern "C" int amg_time_fine_smoother(tp_amg_t amg, int32_t reps, double* ms_per_launch,
                                      double* bytes_per_launch, void* stream) {
    TP_GUARD({
        TP_CHECK_ARG(amg && ms_per_launch && bytes_per_launch, "amg_time_fine_smoother: null argument");
        TP_CHECK_ARG(reps >= 1 && reps <= 100000, "amg_time_fine_smoother: reps out of range");
        TP_CHECK_ARG(amg->lev.size() >= 2, "amg_time_fine_smoother: needs at least two levels");
        hipStream_t s = (hipStream_t)stream;
        *ms_per_launch = amg->prm.storage == 2   ? tp::replay_fine_smoother<tp::M16>(amg, reps, s, bytes_per_launch)
                         : amg->prm.storage == 1 ? tp::replay_fine_smoother<tp::M32>(amg, reps, s, bytes_per_launch)
                                                 : tp::replay_fine_smoother<tp::M64>(amg, reps, s, bytes_per_launch);
    });
    return TP_OK;
}

extern "C" int amg_time_fine_smoother_flushed(tp_amg_t amg, int32_t reps, double* flush_buf, int64_t flush_doubles,
                                              double* ms_per_launch, double* bytes_per_launch, void* stream) {
    TP_GUARD({
        TP_CHECK_ARG(amg && flush_buf && ms_per_launch && bytes_per_launch,
                     "amg_time_fine_smoother_flushed: null argument");
        TP_CHECK_ARG(reps >= 1 && reps <= 1000, "amg_time_fine_smoother_flushed: reps out of range");
        TP_CHECK_ARG(flush_doubles >= 1, "amg_time_fine_smoother_flushed: empty flush buffer");
        TP_CHECK_ARG(amg->lev.size() >= 2, "amg_time_fine_smoother_flushed: needs at least two levels");
        hipStream_t s = (hipStream_t)stream;
        double* const fl = flush_buf;
        const int64_t fn = flush_doubles;
        *ms_per_launch =
            amg->prm.storage == 2   ? tp::replay_fine_smoother<tp::M16>(amg, reps, s, bytes_per_launch, fl, fn)
            : amg->prm.storage == 1 ? tp::replay_fine_smoother<tp::M32>(amg, reps, s, bytes_per_launch, fl, fn)
                                    : tp::replay_fine_smoother<tp::M64>(amg, reps, s, bytes_per_launch, fl, fn);
    });
    return TP_OK;
}

extern "C" int amg_vcycle(tp_amg_t amg, const double* b, double* x, void* stream) {
    TP_GUARD({
        TP_CHECK_ARG(amg && b && x, "amg_vcycle: null argument");
        hipStream_t s = (hipStream_t)stream;
        const int32_t n = amg->lev[0].A.n;
        const size_t es = tp::storage_bytes(amg);
        tp::cast_d2s(n, b, amg->lev[0].b.p, es, s);
        const void* r = tp::vcycle_run(amg, nullptr, s);
        tp::cast_s2d(n, r, x, es, s);
    });
    return TP_OK;
}
