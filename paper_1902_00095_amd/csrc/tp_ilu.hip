// tp_ilu.hip -- ILU(0) factorisation and level-scheduled triangular solves.
//
// ILU(0) (Section 3, the incomplete factorisations named there): A ~ L U
// with L unit lower and U upper triangular on the sparsity pattern of A,
// computed by row-by-row (IKJ) Gaussian elimination in which every update
// outside the pattern is dropped.  It is the second stage of the CPR
// preconditioner of Section 3.1 (Section 4 uses ILU(0) on the whole
// Jacobian).
//
// GPU schedule.  Row i of the elimination, and of the forward solve, needs
// the finished rows k < i that its pattern holds; row i of the backward
// solve needs the rows k > i.  A host pass over the pattern (once per
// pattern) gives every row its level, 1 + the largest level among those
// rows, and groups the rows level by level; one kernel launch then handles
// every row of one level.  On a Cartesian grid in field-by-field order the
// levels are the grid's wavefront planes (about nx + ny + nz of them), so a
// solve is a few hundred short launches: it is bound by launch and memory
// latency, not by HBM bandwidth.  The elimination runs one thread per row
// with the operations and order of the definition (bit-identical to a
// sequential elimination); the solves give each row a lane group whose
// partial sums are reduced by shuffles.
#include "tp_internal.h"

#include <algorithm>
#include <cmath>
#include <vector>

struct tp_ilu {
    int32_t N = 0, nnz = 0;
    int32_t n_cells = 0;                 // > 0: built from a Jacobian (N = 2 n_cells)
    tp::DBuf<int32_t> rowptr, col, dg;  // pattern (sorted rows) and the slot of each diagonal
    tp::DBuf<double> lu;                 // L below the diagonal (unit diagonal implied), U on and above
    tp::DBuf<int32_t> lrows, urows;      // rows grouped by forward and by backward level
    std::vector<int32_t> lptr, uptr;     // level offsets into lrows / urows (host)
    tp::DBuf<int32_t> bad;               // zero-pivot flag of the last factorisation
    int32_t maxrow = 0;                  // longest row (the lane-per-entry elimination needs <= 16)
    // Solve copies in level order, fixed width per row (position t of lrows /
    // urows holds its row's entries at [t * W, t * W + W), column -1 padding):
    // the strictly lower part, the strictly upper part and U's diagonal.
    int32_t wl = 0, wu = 0;
    tp::DBuf<int32_t> lci, uci;
    tp::DBuf<double> lval, uval, udiag;
};

namespace tp {

constexpr int IB = 256;  // threads per block of the level kernels
constexpr int IG = 16;   // lanes per row in the solves (a field-ordered TPFA row holds 14 entries)

// ---- whole Jacobian in field-by-field order ---------------------------------------------
// row p_i = [A_pp(i,:), A_pT(i,:)] (columns j, n + j), row T_i = [A_Tp(i,:), A_TT(i,:)];
// every stored entry of the four blocks is kept (structural zeros included)
__global__ void __launch_bounds__(IB)
k_jac_fieldwise(int32_t n, int32_t nnz, const int32_t* __restrict__ rp, const int32_t* __restrict__ ci,
                const double* __restrict__ pp, const double* __restrict__ pT, const double* __restrict__ Tp,
                const double* __restrict__ TT, int32_t* __restrict__ orp, int32_t* __restrict__ oci,
                double* __restrict__ ov) {
    const int64_t r = (int64_t)blockIdx.x * IB + threadIdx.x;
    if (r >= 2 * (int64_t)n) return;
    const int f = r >= n;
    const int32_t i = (int32_t)(f ? r - n : r);
    const double* left = f ? Tp : pp;
    const double* right = f ? TT : pT;
    const int32_t b = rp[i], len = rp[i + 1] - b;
    const int64_t o = (int64_t)f * 2 * nnz + 2 * (int64_t)b;
    for (int32_t k = 0; k < len; ++k) {
        if (oci) {
            oci[o + k] = ci[b + k];
            oci[o + len + k] = n + ci[b + k];
        }
        ov[o + k] = left[b + k];
        ov[o + len + k] = right[b + k];
    }
    if (orp) {
        orp[r] = (int32_t)o;
        if (r == 2 * (int64_t)n - 1) orp[2 * n] = 4 * nnz;
    }
}

// ---- elimination of the rows of one level ------------------------------------------------
// Row i: for each k < i held by the row, in increasing k, l_ik = a_ik / u_kk,
// then a_ij -= l_ik u_kj for every j > k held by both row k and row i.
__global__ void __launch_bounds__(IB)
k_ilu_factor_level(int32_t cnt, const int32_t* __restrict__ rows, const int32_t* __restrict__ rp,
                   const int32_t* __restrict__ ci, const int32_t* __restrict__ dg, double* __restrict__ lu,
                   int32_t* __restrict__ bad) {
    const int32_t t = blockIdx.x * IB + threadIdx.x;
    if (t >= cnt) return;
    const int32_t i = rows[t];
    const int32_t e = rp[i + 1], d = dg[i];
    for (int32_t q = rp[i]; q < d; ++q) {
        const int32_t k = ci[q];
        const int32_t dk = dg[k], ke = rp[k + 1];
        const double lik = lu[q] / lu[dk];
        lu[q] = lik;
        int32_t p = q + 1;
        for (int32_t u = dk + 1; u < ke && p < e; ++u) {
            const int32_t j = ci[u];
            while (p < e && ci[p] < j) ++p;
            if (p < e && ci[p] == j) lu[p] -= lik * lu[u];
        }
    }
    const double piv = lu[d];
    if (!(piv != 0.0) || !std::isfinite(piv)) bad[0] = 1;
}

// Lane-per-entry form of the same elimination (rows of at most G entries):
// lane l holds entry l of row i.  The columns k of the row's lower part are
// taken in increasing order as before; the lanes load row k's upper part in
// one coalesced read and each finds its own column there by shuffles.  Every
// entry sees the same operations in the same order as in the thread-per-row
// kernel, so the factors are identical.
template <int G>
__global__ void __launch_bounds__(IB)
k_ilu_factor_level_w(int32_t cnt, const int32_t* __restrict__ rows, const int32_t* __restrict__ rp,
                     const int32_t* __restrict__ ci, const int32_t* __restrict__ dg, double* __restrict__ lu,
                     int32_t* __restrict__ bad) {
    const int64_t tid = (int64_t)blockIdx.x * IB + threadIdx.x;
    const int32_t t = (int32_t)(tid / G);
    const int lane = (int)(tid % G);
    const bool valid = t < cnt;
    int32_t b = 0, len = 0, nl = 0;
    if (valid) {
        const int32_t i = rows[t];
        b = rp[i];
        len = rp[i + 1] - b;
        nl = dg[i] - b;
    }
    const bool mine = lane < len;
    int32_t c = -1;
    double a = 0.0;
    int32_t dk = 0, ke = 0;
    if (mine) {
        c = ci[b + lane];
        a = lu[b + lane];
        if (lane < nl) {  // prefetch where row c's upper part lies
            dk = dg[c];
            ke = rp[c + 1];
        }
    }
    for (int m = 0; m < nl; ++m) {  // uniform within the row's lanes
        const int32_t k = __shfl(c, m, G);
        const int32_t dkk = __shfl(dk, m, G), kee = __shfl(ke, m, G);
        const double ukk = lu[dkk];
        const double lik = __shfl(a, m, G) / ukk;
        const int32_t u = dkk + 1 + lane;
        int32_t cu = -1;
        double vu = 0.0;
        if (u < kee) {
            cu = ci[u];
            vu = lu[u];
        }
        double ukj = 0.0;
        bool hit = false;
#pragma unroll
        for (int w = 0; w < G; ++w) {
            const int32_t cw = __shfl(cu, w, G);
            const double vw = __shfl(vu, w, G);
            if (cw == c && cw >= 0) {
                ukj = vw;
                hit = true;
            }
        }
        if (lane == m) a = lik;
        else if (mine && c > k && hit) a -= lik * ukj;
    }
    if (mine) lu[b + lane] = a;
    if (mine && lane == nl && (!(a != 0.0) || !std::isfinite(a))) bad[0] = 1;
}

// Level-ordered fixed-width copies of the factors for the solves: for
// position t of a level ordering (row i = rows[t]), entries of the chosen part
// go to [t * W, t * W + W) with column -1 after the last; with `ud`, also
// U's diagonal ud[t] = u_ii.
__global__ void __launch_bounds__(IB)
k_ilu_ell(int32_t N, const int32_t* __restrict__ rows, const int32_t* __restrict__ rp,
          const int32_t* __restrict__ ci, const int32_t* __restrict__ dg, const double* __restrict__ lu, int upper,
          int32_t W, int32_t* __restrict__ oci, double* __restrict__ oval, double* __restrict__ ud) {
    const int32_t t = blockIdx.x * IB + threadIdx.x;
    if (t >= N) return;
    const int32_t i = rows[t];
    const int32_t q0 = upper ? dg[i] + 1 : rp[i];
    const int32_t q1 = upper ? rp[i + 1] : dg[i];
    const int64_t o = (int64_t)t * W;
    for (int32_t k = 0; k < W; ++k) {
        const int32_t q = q0 + k;
        const bool in = q < q1;
        if (oci) oci[o + k] = in ? ci[q] : -1;
        oval[o + k] = in ? lu[q] : 0.0;
    }
    if (ud) ud[t] = lu[dg[i]];
}

// ---- triangular solves, one level per launch ------------------------------------------------
// forward: y_i = b_i - sum_{k<i} l_ik y_k (b and y may alias); the level's
// rows in the fixed-width level-ordered copy of L
__global__ void __launch_bounds__(IB)
k_ilu_lower_level(int32_t cnt, const int32_t* __restrict__ rows, int32_t W, const int32_t* __restrict__ lci,
                  const double* __restrict__ lval, const double* b, double* y) {
    const int64_t tid = (int64_t)blockIdx.x * IB + threadIdx.x;
    const int32_t t = (int32_t)(tid / IG);
    const int lane = (int)(tid % IG);
    int32_t i = 0;
    double s = 0.0;
    if (t < cnt) {
        i = rows[t];
        const int64_t o = (int64_t)t * W;
        for (int32_t k = lane; k < W; k += IG) {
            const int32_t c = lci[o + k];
            if (c >= 0) s += lval[o + k] * y[c];
        }
    }
#pragma unroll
    for (int off = IG / 2; off > 0; off >>= 1) s += __shfl_down(s, off, IG);
    if (t < cnt && lane == 0) y[i] = b[i] - s;
}

// backward, in place: x_i = (y_i - sum_{k>i} u_ik x_k) / u_ii
__global__ void __launch_bounds__(IB)
k_ilu_upper_level(int32_t cnt, const int32_t* __restrict__ rows, int32_t W, const int32_t* __restrict__ uci,
                  const double* __restrict__ uval, const double* __restrict__ ud, double* x) {
    const int64_t tid = (int64_t)blockIdx.x * IB + threadIdx.x;
    const int32_t t = (int32_t)(tid / IG);
    const int lane = (int)(tid % IG);
    int32_t i = 0;
    double s = 0.0;
    if (t < cnt) {
        i = rows[t];
        const int64_t o = (int64_t)t * W;
        for (int32_t k = lane; k < W; k += IG) {
            const int32_t c = uci[o + k];
            if (c >= 0) s += uval[o + k] * x[c];
        }
    }
#pragma unroll
    for (int off = IG / 2; off > 0; off >>= 1) s += __shfl_down(s, off, IG);
    if (t < cnt && lane == 0) x[i] = (x[i] - s) / ud[t];
}

__global__ void k_ilu_clear(int32_t* p) {
    if (threadIdx.x == 0 && blockIdx.x == 0) p[0] = 0;
}

// ---- host side -------------------------------------------------------------------------------
// Levels of the forward and backward dependency graphs, rows grouped by level.
static void analyse(tp_ilu* F, hipStream_t s) {
    const int32_t N = F->N;
    std::vector<int32_t> rp(N + 1), ci(F->nnz);
    TP_HIP(hipMemcpyAsync(rp.data(), F->rowptr.p, sizeof(int32_t) * (N + 1), hipMemcpyDeviceToHost, s));
    if (F->nnz) TP_HIP(hipMemcpyAsync(ci.data(), F->col.p, sizeof(int32_t) * F->nnz, hipMemcpyDeviceToHost, s));
    TP_HIP(hipStreamSynchronize(s));
    TP_CHECK_ARG(rp[0] == 0 && rp[N] == F->nnz, "ilu0: rowptr does not span nnz");
    for (int32_t i = 0; i < N; ++i) TP_CHECK_ARG(rp[i + 1] >= rp[i], "ilu0: rowptr is not monotone at row %d", i);
    std::vector<int32_t> dg(N), lev(N);
    for (int32_t i = 0; i < N; ++i) {
        dg[i] = -1;
        for (int32_t q = rp[i]; q < rp[i + 1]; ++q) {
            TP_CHECK_ARG(ci[q] >= 0 && ci[q] < N, "ilu0: column index out of range in row %d", i);
            TP_CHECK_ARG(q == rp[i] || ci[q] > ci[q - 1], "ilu0: row %d is not sorted or has duplicates", i);
            if (ci[q] == i) dg[i] = q;
        }
        TP_CHECK_ARG(dg[i] >= 0, "ilu0: row %d has no diagonal entry", i);
    }
    auto group = [&](std::vector<int32_t>& ptr, DBuf<int32_t>& rows) {
        int32_t nl = 0;
        for (int32_t i = 0; i < N; ++i) nl = std::max(nl, lev[i] + 1);
        ptr.assign(nl + 1, 0);
        for (int32_t i = 0; i < N; ++i) ++ptr[lev[i] + 1];
        for (int32_t l = 0; l < nl; ++l) ptr[l + 1] += ptr[l];
        std::vector<int32_t> fill(ptr.begin(), ptr.end() - 1), out(N);
        for (int32_t i = 0; i < N; ++i) out[fill[lev[i]]++] = i;
        rows.alloc(N, s);
        TP_HIP(hipMemcpyAsync(rows.p, out.data(), sizeof(int32_t) * N, hipMemcpyHostToDevice, s));
        TP_HIP(hipStreamSynchronize(s));  // `out` is a host temporary
    };
    for (int32_t i = 0; i < N; ++i) {
        int32_t l = 0;
        for (int32_t q = rp[i]; q < dg[i]; ++q) l = std::max(l, lev[ci[q]] + 1);
        lev[i] = l;
    }
    group(F->lptr, F->lrows);
    for (int32_t i = N - 1; i >= 0; --i) {
        int32_t l = 0;
        for (int32_t q = dg[i] + 1; q < rp[i + 1]; ++q) l = std::max(l, lev[ci[q]] + 1);
        lev[i] = l;
    }
    group(F->uptr, F->urows);
    F->maxrow = F->wl = F->wu = 0;
    for (int32_t i = 0; i < N; ++i) {
        F->maxrow = std::max(F->maxrow, rp[i + 1] - rp[i]);
        F->wl = std::max(F->wl, dg[i] - rp[i]);
        F->wu = std::max(F->wu, rp[i + 1] - dg[i] - 1);
    }
    F->wl = std::max(F->wl, 1);
    F->wu = std::max(F->wu, 1);
    F->lci.alloc((size_t)N * F->wl, s);
    F->lval.alloc((size_t)N * F->wl, s);
    F->uci.alloc((size_t)N * F->wu, s);
    F->uval.alloc((size_t)N * F->wu, s);
    F->udiag.alloc(N, s);
    F->dg.alloc(N, s);
    TP_HIP(hipMemcpyAsync(F->dg.p, dg.data(), sizeof(int32_t) * N, hipMemcpyHostToDevice, s));
    TP_HIP(hipStreamSynchronize(s));
}

static void factorise(tp_ilu* F, bool pattern, hipStream_t s) {
    TP_LAUNCH(k_ilu_clear, 1, 64, 0, s, F->bad.p);
    for (size_t l = 0; l + 1 < F->lptr.size(); ++l) {
        const int32_t b = F->lptr[l], cnt = F->lptr[l + 1] - b;
        if (F->maxrow <= 16)
            TP_LAUNCH(k_ilu_factor_level_w<16>, cdiv((int64_t)cnt * 16, IB), IB, 0, s, cnt, F->lrows.p + b,
                      F->rowptr.p, F->col.p, F->dg.p, F->lu.p, F->bad.p);
        else
            TP_LAUNCH(k_ilu_factor_level, cdiv(cnt, IB), IB, 0, s, cnt, F->lrows.p + b, F->rowptr.p, F->col.p,
                      F->dg.p, F->lu.p, F->bad.p);
    }
    const int g = cdiv(F->N, IB);
    TP_LAUNCH(k_ilu_ell, g, IB, 0, s, F->N, F->lrows.p, F->rowptr.p, F->col.p, F->dg.p, F->lu.p, 0, F->wl,
              pattern ? F->lci.p : nullptr, F->lval.p, (double*)nullptr);
    TP_LAUNCH(k_ilu_ell, g, IB, 0, s, F->N, F->urows.p, F->rowptr.p, F->col.p, F->dg.p, F->lu.p, 1, F->wu,
              pattern ? F->uci.p : nullptr, F->uval.p, F->udiag.p);
    if (read_i32(F->bad.p, s))
        fail(TP_ERR_NUMERIC, "ilu0: zero or non-finite pivot in the incomplete factorisation");
}

void ilu_solve(tp_ilu* F, const double* b, double* x, hipStream_t s) {
    for (size_t l = 0; l + 1 < F->lptr.size(); ++l) {
        const int32_t o = F->lptr[l], cnt = F->lptr[l + 1] - o;
        TP_LAUNCH(k_ilu_lower_level, cdiv((int64_t)cnt * IG, IB), IB, 0, s, cnt, F->lrows.p + o, F->wl,
                  F->lci.p + (int64_t)o * F->wl, F->lval.p + (int64_t)o * F->wl, b, x);
    }
    for (size_t l = 0; l + 1 < F->uptr.size(); ++l) {
        const int32_t o = F->uptr[l], cnt = F->uptr[l + 1] - o;
        TP_LAUNCH(k_ilu_upper_level, cdiv((int64_t)cnt * IG, IB), IB, 0, s, cnt, F->urows.p + o, F->wu,
                  F->uci.p + (int64_t)o * F->wu, F->uval.p + (int64_t)o * F->wu, F->udiag.p + o, x);
    }
}

int32_t ilu_size(const tp_ilu* F) { return F->N; }
int32_t ilu_cells(const tp_ilu* F) { return F->n_cells; }

static void check_jacobian(const tp_jacobian* J) {
    TP_CHECK_ARG(J, "ilu0: null Jacobian");
    TP_CHECK_ARG(J->n >= 1 && J->nnz >= 1 && J->rowptr && J->col && J->pp && J->pT && J->Tp && J->TT,
                 "ilu0: empty Jacobian or null block array");
    TP_CHECK_ARG((int64_t)J->nnz * 4 <= INT32_MAX && (int64_t)J->n * 2 <= INT32_MAX,
                 "ilu0: the whole Jacobian would exceed 2^31-1 entries");
}

static void fill_fieldwise(tp_ilu* F, const tp_jacobian* J, bool pattern, hipStream_t s) {
    TP_LAUNCH(k_jac_fieldwise, cdiv(2 * (int64_t)J->n, IB), IB, 0, s, J->n, J->nnz, J->rowptr, J->col, J->pp, J->pT,
              J->Tp, J->TT, pattern ? F->rowptr.p : nullptr, pattern ? F->col.p : nullptr, F->lu.p);
}

}  // namespace tp

extern "C" {

int ilu0_create(int32_t N, const int32_t* rowptr, const int32_t* col, const double* val, void* stream,
                tp_ilu_t* out) {
    TP_GUARD({
        TP_CHECK_ARG(out, "ilu0_create: null argument");
        *out = nullptr;
        TP_CHECK_ARG(N >= 1 && rowptr && col && val, "ilu0_create: empty or null matrix");
        hipStream_t s = (hipStream_t)stream;
        int32_t nnz = tp::read_i32(rowptr + N, s);
        TP_CHECK_ARG(nnz >= N, "ilu0_create: fewer entries than rows (a diagonal is missing)");
        tp_ilu* F = new tp_ilu();
        try {
            F->N = N;
            F->nnz = nnz;
            F->rowptr.alloc(N + 1, s);
            F->col.alloc(nnz, s);
            F->lu.alloc(nnz, s);
            F->bad.alloc(1, s);
            TP_HIP(hipMemcpyAsync(F->rowptr.p, rowptr, sizeof(int32_t) * (N + 1), hipMemcpyDeviceToDevice, s));
            TP_HIP(hipMemcpyAsync(F->col.p, col, sizeof(int32_t) * nnz, hipMemcpyDeviceToDevice, s));
            TP_HIP(hipMemcpyAsync(F->lu.p, val, sizeof(double) * nnz, hipMemcpyDeviceToDevice, s));
            tp::analyse(F, s);
            tp::factorise(F, true, s);
        } catch (...) {
            (void)hipStreamSynchronize(s);
            delete F;
            throw;
        }
        *out = F;
    });
    return TP_OK;
}

int ilu0_create_jacobian(const tp_jacobian* J, void* stream, tp_ilu_t* out) {
    TP_GUARD({
        TP_CHECK_ARG(out, "ilu0_create_jacobian: null argument");
        *out = nullptr;
        tp::check_jacobian(J);
        hipStream_t s = (hipStream_t)stream;
        tp_ilu* F = new tp_ilu();
        try {
            F->N = 2 * J->n;
            F->nnz = 4 * J->nnz;
            F->n_cells = J->n;
            F->rowptr.alloc(F->N + 1, s);
            F->col.alloc(F->nnz, s);
            F->lu.alloc(F->nnz, s);
            F->bad.alloc(1, s);
            tp::fill_fieldwise(F, J, true, s);
            tp::analyse(F, s);
            tp::factorise(F, true, s);
        } catch (...) {
            (void)hipStreamSynchronize(s);
            delete F;
            throw;
        }
        *out = F;
    });
    return TP_OK;
}

int ilu0_refactor_jacobian(tp_ilu_t F, const tp_jacobian* J, void* stream) {
    TP_GUARD({
        TP_CHECK_ARG(F, "ilu0_refactor_jacobian: null handle");
        tp::check_jacobian(J);
        TP_CHECK_ARG(F->n_cells == J->n && F->nnz == 4 * J->nnz,
                     "ilu0_refactor_jacobian: the handle was not built from a Jacobian of this size");
        hipStream_t s = (hipStream_t)stream;
        tp::fill_fieldwise(F, J, false, s);
        tp::factorise(F, false, s);
    });
    return TP_OK;
}

int ilu0_solve(tp_ilu_t F, const double* b, double* x, void* stream) {
    TP_GUARD({
        TP_CHECK_ARG(F && b && x, "ilu0_solve: null argument");
        tp::ilu_solve(F, b, x, (hipStream_t)stream);
    });
    return TP_OK;
}

int ilu0_info(tp_ilu_t F, int32_t* N, int32_t* nnz, int32_t* levels_lower, int32_t* levels_upper) {
    TP_GUARD({
        TP_CHECK_ARG(F, "ilu0_info: null handle");
        if (N) *N = F->N;
        if (nnz) *nnz = F->nnz;
        if (levels_lower) *levels_lower = (int32_t)F->lptr.size() - 1;
        if (levels_upper) *levels_upper = (int32_t)F->uptr.size() - 1;
    });
    return TP_OK;
}

int ilu0_copy(tp_ilu_t F, int32_t* rowptr, int32_t* col, double* lu, void* stream) {
    TP_GUARD({
        TP_CHECK_ARG(F, "ilu0_copy: null handle");
        hipStream_t s = (hipStream_t)stream;
        if (rowptr)
            TP_HIP(hipMemcpyAsync(rowptr, F->rowptr.p, sizeof(int32_t) * (F->N + 1), hipMemcpyDeviceToDevice, s));
        if (col) TP_HIP(hipMemcpyAsync(col, F->col.p, sizeof(int32_t) * F->nnz, hipMemcpyDeviceToDevice, s));
        if (lu) TP_HIP(hipMemcpyAsync(lu, F->lu.p, sizeof(double) * F->nnz, hipMemcpyDeviceToDevice, s));
    });
    return TP_OK;
}

int ilu0_destroy(tp_ilu_t F) {
    TP_GUARD({
        if (!F) return TP_OK;
        // the factors may be in use on streams other than the creating one
        TP_HIP(hipDeviceSynchronize());
        delete F;
        TP_HIP(hipDeviceSynchronize());
    });
    return TP_OK;
}

}  // extern "C"
