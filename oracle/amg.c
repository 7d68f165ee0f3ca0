/*
 * amg.c -- oracle algebraic multigrid: setup and V(nu_pre, nu_post) cycle.
 *
 * TEST INFRASTRUCTURE ONLY (see tp_oracle.h).  Plain FP64, sequential.
 *
 * The paper applies A_pp^{-1} and the Schur approximation's inverse by one
 * AMG V-cycle each (Section 3.2, Section 4).  The components are:
 *   strength     classical Ruge-Stueben test, sign-aware: j in S_i iff
 *                -s_i a_ij >= theta * max_{k != i} (-s_i a_ik) > 0, s_i = sign(a_ii);
 *   coarsening   PMIS (De Sterck, Yang, Heys, SIAM J. Matrix Anal. Appl. 2006)
 *                with measure lambda_i = |S^T_i| and ties broken by the key
 *                (lambda_i, splitmix64(seed ^ (level << 40) ^ i), i);
 *   interpolation direct interpolation (Stueben, "An introduction to
 *                algebraic multigrid", 2001), positive couplings lumped into
 *                the diagonal; or (interp = 1) extended+i interpolation
 *                (De Sterck, Falgout, Nolting, Yang, "Distance-two
 *                interpolation for parallel algebraic multigrid", Numer.
 *                Linear Algebra Appl. 15, 2008), see ext_interp;
 *   coarse op.   Galerkin A_c = R (A P) with R = P^T, every entry summed
 *                sequentially in ascending inner index, structural pattern kept;
 *   restriction  Galerkin R = P^T, or Petrov-Galerkin R = Q^T where Q is the
 *                direct interpolation built from A^T on the same C/F split
 *                (used for the non-symmetric Schur approximation, whose
 *                columns, not rows, are diagonally dominant);
 *   smoother     l1-Jacobi (Baker, Falgout, Kolev, Yang 2011), D_ii = sum_j |a_ij|,
 *                or the Chebyshev polynomial iteration (Saad, "Iterative
 *                methods for sparse linear systems", 2nd ed., Sec. 12.3) on
 *                D^{-1} A over [lo, 1]: by Gershgorin every eigenvalue of
 *                D^{-1} A lies in the disc touching 1 from the left, so the
 *                upper end needs no estimate;
 *   coarsest     dense LU with partial pivoting.
 */
#include "tp_oracle.h"
#include <math.h>
#include <stdlib.h>
#include <string.h>

#define OR_MAXLEV 32

typedef struct { int32_t n, m, nnz; int32_t* rowptr; int32_t* col; double* val; } csr_t;

struct or_amg {
    or_amg_params prm;
    int32_t nlev;
    csr_t A[OR_MAXLEV], P[OR_MAXLEV], R[OR_MAXLEV];
    /* extended+i: the strength patterns of A_l (and of A_l^T when R = Q^T),
     * kept for the numeric refresh */
    csr_t S[OR_MAXLEV], Sq[OR_MAXLEV];
    double* dinv[OR_MAXLEV];
    int32_t* cf[OR_MAXLEV];
    int32_t nc;
    double* lu;
    int32_t* piv;
};

static void csr_free(csr_t* a)
{
    free(a->rowptr);
    free(a->col);
    free(a->val);
    memset(a, 0, sizeof(*a));
}

static void csr_alloc(csr_t* a, int32_t n, int32_t m, int32_t nnz)
{
    a->n = n;
    a->m = m;
    a->nnz = nnz;
    a->rowptr = calloc((size_t)n + 1, sizeof(int32_t));
    a->col = malloc(sizeof(int32_t) * (size_t)(nnz > 0 ? nnz : 1));
    a->val = malloc(sizeof(double) * (size_t)(nnz > 0 ? nnz : 1));
}

uint64_t or_splitmix64(uint64_t x)
{
    /* SplitMix64 (Steele, Lea, Flood, OOPSLA 2014): advance the state by the
     * golden-ratio increment, then apply the variant-13 finaliser. */
    uint64_t z = x + 0x9E3779B97F4A7C15ULL;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
    return z ^ (z >> 31);
}

void or_spmv(int32_t n, const int32_t* rowptr, const int32_t* col, const double* val,
             const double* x, double* y)
{
    for (int32_t i = 0; i < n; ++i) {
        double s = 0.0;
        for (int32_t k = rowptr[i]; k < rowptr[i + 1]; ++k) s += val[k] * x[col[k]];
        y[i] = s;
    }
}

/* strength matrix S (pattern only), rows list j in S_i ascending */
static void strength(const csr_t* A, double theta, csr_t* S)
{
    int32_t n = A->n;
    csr_alloc(S, n, n, A->nnz);
    int32_t k = 0;
    for (int32_t i = 0; i < n; ++i) {
        double aii = 0.0;
        for (int32_t q = A->rowptr[i]; q < A->rowptr[i + 1]; ++q)
            if (A->col[q] == i) aii = A->val[q];
        double s = aii < 0.0 ? -1.0 : 1.0;
        double m = 0.0;
        for (int32_t q = A->rowptr[i]; q < A->rowptr[i + 1]; ++q)
            if (A->col[q] != i && -s * A->val[q] > m) m = -s * A->val[q];
        S->rowptr[i] = k;
        if (m > 0.0) {
            for (int32_t q = A->rowptr[i]; q < A->rowptr[i + 1]; ++q)
                if (A->col[q] != i && -s * A->val[q] >= theta * m) S->col[k++] = A->col[q];
        }
    }
    S->rowptr[n] = k;
    S->nnz = k;
}

/* transpose of a pattern/values CSR with sorted rows (stable counting sort) */
static void transpose(const csr_t* A, csr_t* T)
{
    csr_alloc(T, A->m, A->n, A->nnz);
    for (int32_t k = 0; k < A->nnz; ++k) T->rowptr[A->col[k] + 1]++;
    for (int32_t i = 0; i < A->m; ++i) T->rowptr[i + 1] += T->rowptr[i];
    int32_t* pos = malloc(sizeof(int32_t) * ((size_t)A->m + 1));
    memcpy(pos, T->rowptr, sizeof(int32_t) * ((size_t)A->m + 1));
    for (int32_t i = 0; i < A->n; ++i)
        for (int32_t k = A->rowptr[i]; k < A->rowptr[i + 1]; ++k) {
            int32_t d = pos[A->col[k]]++;
            T->col[d] = i;
            if (A->val) T->val[d] = A->val[k];
        }
    free(pos);
}

static int key_greater(int32_t li, uint64_t hi, int32_t i, int32_t lj, uint64_t hj, int32_t j)
{
    if (li != lj) return li > lj;
    if (hi != hj) return hi > hj;
    return i > j;
}

/* PMIS: cf[i] = 1 (C) or 0 (F) */
static void pmis(const csr_t* S, uint64_t seed, int32_t level, int32_t* cf)
{
    int32_t n = S->n;
    csr_t ST;
    transpose(S, &ST);
    int32_t* lam = malloc(sizeof(int32_t) * (size_t)(n > 0 ? n : 1));
    uint64_t* h = malloc(sizeof(uint64_t) * (size_t)(n > 0 ? n : 1));
    int8_t* st = malloc((size_t)(n > 0 ? n : 1));   /* 0 undecided, 1 C, -1 F */
    int8_t* old = malloc((size_t)(n > 0 ? n : 1));
    for (int32_t i = 0; i < n; ++i) {
        lam[i] = ST.rowptr[i + 1] - ST.rowptr[i];
        h[i] = or_splitmix64(seed ^ ((uint64_t)level << 40) ^ (uint64_t)i);
        st[i] = lam[i] == 0 ? -1 : 0;
    }
    for (;;) {
        int32_t und = 0;
        for (int32_t i = 0; i < n; ++i) und += st[i] == 0;
        if (und == 0) break;
        memcpy(old, st, (size_t)n);
        /* C selection from the snapshot */
        for (int32_t i = 0; i < n; ++i) {
            if (old[i] != 0) continue;
            int isC = 1;
            for (int32_t k = S->rowptr[i]; k < S->rowptr[i + 1] && isC; ++k) {
                int32_t j = S->col[k];
                if (old[j] == 0 && !key_greater(lam[i], h[i], i, lam[j], h[j], j)) isC = 0;
            }
            for (int32_t k = ST.rowptr[i]; k < ST.rowptr[i + 1] && isC; ++k) {
                int32_t j = ST.col[k];
                if (old[j] == 0 && !key_greater(lam[i], h[i], i, lam[j], h[j], j)) isC = 0;
            }
            if (isC) st[i] = 1;
        }
        /* undecided points that strongly depend on a C point become F */
        for (int32_t j = 0; j < n; ++j) {
            if (st[j] != 0) continue;
            for (int32_t k = S->rowptr[j]; k < S->rowptr[j + 1]; ++k)
                if (st[S->col[k]] == 1) { st[j] = -1; break; }
        }
    }
    for (int32_t i = 0; i < n; ++i) cf[i] = st[i] == 1;
    free(lam); free(h); free(st); free(old);
    csr_free(&ST);
}

/* direct interpolation; cmap = coarse index of C points (rank among C) */
static void direct_interp(const csr_t* A, const csr_t* S, const int32_t* cf,
                          const int32_t* cmap, int32_t nc, csr_t* P)
{
    int32_t n = A->n;
    /* count */
    int32_t nnz = 0;
    for (int32_t i = 0; i < n; ++i) {
        if (cf[i]) { nnz += 1; continue; }
        for (int32_t k = S->rowptr[i]; k < S->rowptr[i + 1]; ++k) nnz += cf[S->col[k]];
    }
    csr_alloc(P, n, nc, nnz);
    int32_t q = 0;
    for (int32_t i = 0; i < n; ++i) {
        P->rowptr[i] = q;
        if (cf[i]) { P->col[q] = cmap[i]; P->val[q] = 1.0; ++q; continue; }
        double aii = 0.0;
        for (int32_t k = A->rowptr[i]; k < A->rowptr[i + 1]; ++k)
            if (A->col[k] == i) aii = A->val[k];
        double s = aii < 0.0 ? -1.0 : 1.0;
        /* sums over all off-diagonal couplings of the sign opposite to the
         * diagonal, and the lumped same-sign couplings */
        double sum_all = 0.0, lump = 0.0;
        for (int32_t k = A->rowptr[i]; k < A->rowptr[i + 1]; ++k) {
            if (A->col[k] == i) continue;
            double a = A->val[k];
            if (s * a < 0.0) sum_all += a;
            else lump += a;
        }
        /* interpolatory set: strong C neighbours (ascending) */
        double sum_p = 0.0;
        int32_t k2 = S->rowptr[i];
        for (int32_t k = A->rowptr[i]; k < A->rowptr[i + 1]; ++k) {
            int32_t j = A->col[k];
            while (k2 < S->rowptr[i + 1] && S->col[k2] < j) ++k2;
            if (k2 < S->rowptr[i + 1] && S->col[k2] == j && cf[j]) sum_p += A->val[k];
        }
        if (sum_p == 0.0) continue;          /* no C neighbour: empty row */
        double alpha = sum_all / sum_p;
        double dtil = aii + lump;
        k2 = S->rowptr[i];
        for (int32_t k = A->rowptr[i]; k < A->rowptr[i + 1]; ++k) {
            int32_t j = A->col[k];
            while (k2 < S->rowptr[i + 1] && S->col[k2] < j) ++k2;
            if (k2 < S->rowptr[i + 1] && S->col[k2] == j && cf[j]) {
                P->col[q] = cmap[j];
                P->val[q] = -(alpha * A->val[k]) / dtil;
                ++q;
            }
        }
    }
    P->rowptr[n] = q;
    P->nnz = q;
}

/* hat a_kl: a_kl where its sign is opposite to the diagonal a_kk's, else 0 */
static double opp(double a, double akk)
{
    return (akk > 0.0 ? a < 0.0 : a > 0.0) ? a : 0.0;
}

static int in_sorted(const int32_t* v, int32_t len, int32_t x)
{
    int32_t lo = 0, hi = len;
    while (lo < hi) {
        int32_t mid = lo + (hi - lo) / 2;
        if (v[mid] < x) lo = mid + 1; else hi = mid;
    }
    return lo < len && v[lo] == x ? lo : -1;
}

static int cmp_i32(const void* a, const void* b)
{
    int32_t x = *(const int32_t*)a, y = *(const int32_t*)b;
    return (x > y) - (x < y);
}

/* Interpolatory set of F point i: its strong C neighbours and the strong C
 * neighbours of its strong F neighbours, ascending; returns the count. */
static int32_t ext_set(const csr_t* S, const int32_t* cf, int32_t i, int32_t* mark, int32_t* list)
{
    int32_t len = 0;
    for (int32_t q = S->rowptr[i]; q < S->rowptr[i + 1]; ++q) {
        int32_t k = S->col[q];
        if (cf[k]) {
            if (mark[k] != i) { mark[k] = i; list[len++] = k; }
        } else {
            for (int32_t t = S->rowptr[k]; t < S->rowptr[k + 1]; ++t) {
                int32_t j = S->col[t];
                if (cf[j] && mark[j] != i) { mark[j] = i; list[len++] = j; }
            }
        }
    }
    qsort(list, (size_t)len, sizeof(int32_t), cmp_i32);
    return len;
}

/* Extended+i interpolation.  For F point i with interpolatory set C^_i (see
 * ext_set), and for each strong F neighbour k the sum
 * den_k = sum of hat a_kl over l in C^_i and l = i:
 *   a~_ii = a_ii + (sum of a_in over neighbours n that are neither strong nor
 *           in C^_i) + sum_k a_ik hat a_ki / den_k,
 *   w_ij  = -(a_ij + sum_k a_ik hat a_kj / den_k) / a~_ii,   j in C^_i
 * (a_ij = 0 when j is not a neighbour).  A strong F neighbour with den_k = 0
 * is lumped into a~_ii like a weak one.  Sums run in ascending column order
 * (the row's own entries first, then the strong F neighbours k ascending,
 * each over row k ascending).  C points interpolate themselves; an F point
 * with an empty set gets an empty row.
 * Truncation (pmax > 0): a row of more than pmax weights keeps the pmax of
 * largest magnitude (ties: the smaller column), scaled by
 * f = (sum of all its weights) / (sum of the kept ones), both sums in
 * ascending column order (no scaling when the kept sum is 0): the row sum
 * is preserved. */

/* the weights w[0..len) of F row i over its set list[0..len) */
static void ext_weights(const csr_t* A, const csr_t* S, const int32_t* cf, int32_t i,
                        const int32_t* list, int32_t len, double* w)
{
    const int32_t* Si = S->col + S->rowptr[i];
    int32_t slen = S->rowptr[i + 1] - S->rowptr[i];
    double aii = 0.0;
    for (int32_t t = A->rowptr[i]; t < A->rowptr[i + 1]; ++t)
        if (A->col[t] == i) aii = A->val[t];
    for (int32_t s = 0; s < len; ++s) w[s] = 0.0;
    double at = aii;
    /* the row's own couplings: interpolatory ones to w, weak others lumped */
    for (int32_t t = A->rowptr[i]; t < A->rowptr[i + 1]; ++t) {
        int32_t j = A->col[t];
        if (j == i) continue;
        int32_t pos = in_sorted(list, len, j);
        if (pos >= 0) w[pos] += A->val[t];
        else if (in_sorted(Si, slen, j) < 0) at += A->val[t];
    }
    /* strong F neighbours, distributed over C^_i and i */
    for (int32_t t = A->rowptr[i]; t < A->rowptr[i + 1]; ++t) {
        int32_t k = A->col[t];
        if (k == i || cf[k] || in_sorted(Si, slen, k) < 0) continue;
        double aik = A->val[t], akk = 0.0, den = 0.0;
        for (int32_t u = A->rowptr[k]; u < A->rowptr[k + 1]; ++u)
            if (A->col[u] == k) akk = A->val[u];
        for (int32_t u = A->rowptr[k]; u < A->rowptr[k + 1]; ++u) {
            int32_t l = A->col[u];
            if (l == i || in_sorted(list, len, l) >= 0) den += opp(A->val[u], akk);
        }
        if (den == 0.0) { at += aik; continue; }
        for (int32_t u = A->rowptr[k]; u < A->rowptr[k + 1]; ++u) {
            int32_t l = A->col[u];
            double c = (aik * opp(A->val[u], akk)) / den;
            int32_t pos = in_sorted(list, len, l);
            if (pos >= 0) w[pos] += c;
            else if (l == i) at += c;
        }
    }
    for (int32_t s = 0; s < len; ++s) w[s] = -w[s] / at;
}

/* the kept weights of a truncated row, scaled to the full row sum, written
 * in ascending column order to val (keep[s] marks the kept slots) */
static void ext_scale_kept(const double* w, const char* keep, int32_t len, double* val)
{
    double all = 0.0, kept = 0.0;
    for (int32_t s = 0; s < len; ++s) all += w[s];
    for (int32_t s = 0; s < len; ++s) if (keep[s]) kept += w[s];
    double f = kept != 0.0 ? all / kept : 1.0;
    int32_t q = 0;
    for (int32_t s = 0; s < len; ++s)
        if (keep[s]) val[q++] = kept != 0.0 ? w[s] * f : w[s];
}

static void ext_interp(const csr_t* A, const csr_t* S, const int32_t* cf,
                       const int32_t* cmap, int32_t nc, int32_t pmax, csr_t* P)
{
    int32_t n = A->n;
    int32_t* mark = malloc(sizeof(int32_t) * (size_t)(n > 0 ? n : 1));
    int32_t* list = malloc(sizeof(int32_t) * (size_t)(n > 0 ? n : 1));
    double* w = malloc(sizeof(double) * (size_t)(n > 0 ? n : 1));
    char* keep = malloc((size_t)(n > 0 ? n : 1));
    for (int32_t j = 0; j < n; ++j) mark[j] = -1;
    int64_t nnz = 0;
    for (int32_t i = 0; i < n; ++i) {
        int32_t len = cf[i] ? 1 : ext_set(S, cf, i, mark, list);
        nnz += (pmax > 0 && len > pmax) ? pmax : len;
    }
    csr_alloc(P, n, nc, (int32_t)nnz);
    for (int32_t j = 0; j < n; ++j) mark[j] = -1;
    int32_t q = 0;
    for (int32_t i = 0; i < n; ++i) {
        P->rowptr[i] = q;
        if (cf[i]) { P->col[q] = cmap[i]; P->val[q] = 1.0; ++q; continue; }
        int32_t len = ext_set(S, cf, i, mark, list);
        if (len == 0) continue;
        ext_weights(A, S, cf, i, list, len, w);
        if (pmax > 0 && len > pmax) {
            for (int32_t s = 0; s < len; ++s) keep[s] = 0;
            for (int32_t r = 0; r < pmax; ++r) {
                int32_t best = -1;
                for (int32_t s = 0; s < len; ++s)
                    if (!keep[s] && (best < 0 || fabs(w[s]) > fabs(w[best]))) best = s;
                keep[best] = 1;
            }
            for (int32_t s = 0; s < len; ++s)
                if (keep[s]) P->col[q++] = cmap[list[s]];
            ext_scale_kept(w, keep, len, P->val + q - pmax);
        } else {
            for (int32_t s = 0; s < len; ++s) {
                P->col[q] = cmap[list[s]];
                P->val[q] = w[s];
                ++q;
            }
        }
    }
    P->rowptr[n] = q;
    P->nnz = q;
    free(mark); free(list); free(w); free(keep);
}

/* Extended+i interpolation on a frozen hierarchy: the strength pattern S,
 * the split and P's pattern (the kept set of each row) are those of the
 * setup; the weights of each F row are formed over its full interpolatory
 * set C^_i (from the frozen S and split) as in ext_interp, from the new
 * values, and a row that the setup truncated keeps its frozen columns,
 * scaled to the full row sum as in ext_interp.  When S, the split and the
 * kept sets are those that a fresh setup on the new values would choose,
 * this is exactly that setup's interpolation. */
static void ext_refresh(const csr_t* A, const csr_t* S, const int32_t* cf, const int32_t* cmap, csr_t* P)
{
    int32_t n = A->n;
    int32_t* mark = malloc(sizeof(int32_t) * (size_t)(n > 0 ? n : 1));
    int32_t* list = malloc(sizeof(int32_t) * (size_t)(n > 0 ? n : 1));
    double* w = malloc(sizeof(double) * (size_t)(n > 0 ? n : 1));
    char* keep = malloc((size_t)(n > 0 ? n : 1));
    for (int32_t j = 0; j < n; ++j) mark[j] = -1;
    for (int32_t i = 0; i < n; ++i) {
        if (cf[i]) continue;                       /* C row: the unit vector, kept */
        int32_t len = ext_set(S, cf, i, mark, list);
        if (len == 0) continue;
        const int32_t pa = P->rowptr[i], plen = P->rowptr[i + 1] - pa;
        ext_weights(A, S, cf, i, list, len, w);
        if (plen < len) {
            for (int32_t s = 0; s < len; ++s) keep[s] = in_sorted(P->col + pa, plen, cmap[list[s]]) >= 0;
            ext_scale_kept(w, keep, len, P->val + pa);
        } else {
            for (int32_t s = 0; s < len; ++s) P->val[pa + s] = w[s];
        }
    }
    free(mark); free(list); free(w); free(keep);
}

/* C = A B (Gustavson, dense accumulator); each output entry is summed in
 * ascending inner index; output columns ascending; structural zeros kept */
static void spgemm(const csr_t* A, const csr_t* B, csr_t* C)
{
    int32_t n = A->n, m = B->m;
    int32_t* mark = malloc(sizeof(int32_t) * (size_t)(m > 0 ? m : 1));
    double* acc = malloc(sizeof(double) * (size_t)(m > 0 ? m : 1));
    int32_t* list = malloc(sizeof(int32_t) * (size_t)(m > 0 ? m : 1));
    for (int32_t j = 0; j < m; ++j) mark[j] = -1;
    /* symbolic */
    int64_t nnz = 0;
    for (int32_t i = 0; i < n; ++i)
        for (int32_t k = A->rowptr[i]; k < A->rowptr[i + 1]; ++k) {
            int32_t r = A->col[k];
            for (int32_t q = B->rowptr[r]; q < B->rowptr[r + 1]; ++q)
                if (mark[B->col[q]] != i) { mark[B->col[q]] = i; ++nnz; }
        }
    csr_alloc(C, n, m, (int32_t)nnz);
    for (int32_t j = 0; j < m; ++j) mark[j] = -1;
    int32_t pos = 0;
    for (int32_t i = 0; i < n; ++i) {
        int32_t len = 0;
        C->rowptr[i] = pos;
        for (int32_t k = A->rowptr[i]; k < A->rowptr[i + 1]; ++k) {
            int32_t r = A->col[k];
            double a = A->val[k];
            for (int32_t q = B->rowptr[r]; q < B->rowptr[r + 1]; ++q) {
                int32_t c = B->col[q];
                if (mark[c] != i) { mark[c] = i; acc[c] = 0.0; list[len++] = c; }
                acc[c] += a * B->val[q];
            }
        }
        /* insertion sort of the row's columns */
        for (int32_t u = 1; u < len; ++u) {
            int32_t v = list[u], w = u - 1;
            while (w >= 0 && list[w] > v) { list[w + 1] = list[w]; --w; }
            list[w + 1] = v;
        }
        for (int32_t u = 0; u < len; ++u) {
            C->col[pos] = list[u];
            C->val[pos] = acc[list[u]];
            ++pos;
        }
    }
    C->rowptr[n] = pos;
    free(mark); free(acc); free(list);
}

static void l1_dinv(const csr_t* A, double* dinv)
{
    for (int32_t i = 0; i < A->n; ++i) {
        double d = 0.0;
        for (int32_t k = A->rowptr[i]; k < A->rowptr[i + 1]; ++k) d += fabs(A->val[k]);
        dinv[i] = d > 0.0 ? 1.0 / d : 0.0;
    }
}

/* dense LU, partial pivoting (largest |a|, ties -> lowest row) */
static int dense_lu(int32_t n, double* a, int32_t* piv)
{
    for (int32_t k = 0; k < n; ++k) {
        int32_t p = k;
        double best = fabs(a[(size_t)k * n + k]);
        for (int32_t i = k + 1; i < n; ++i)
            if (fabs(a[(size_t)i * n + k]) > best) { best = fabs(a[(size_t)i * n + k]); p = i; }
        piv[k] = p;
        if (best == 0.0) return -4;
        if (p != k)
            for (int32_t j = 0; j < n; ++j) {
                double t = a[(size_t)k * n + j];
                a[(size_t)k * n + j] = a[(size_t)p * n + j];
                a[(size_t)p * n + j] = t;
            }
        for (int32_t i = k + 1; i < n; ++i) {
            double l = a[(size_t)i * n + k] / a[(size_t)k * n + k];
            a[(size_t)i * n + k] = l;
            for (int32_t j = k + 1; j < n; ++j) a[(size_t)i * n + j] -= l * a[(size_t)k * n + j];
        }
    }
    return 0;
}

static void dense_lu_solve(int32_t n, const double* a, const int32_t* piv, const double* b, double* x)
{
    for (int32_t i = 0; i < n; ++i) x[i] = b[i];
    for (int32_t k = 0; k < n; ++k)
        if (piv[k] != k) { double t = x[k]; x[k] = x[piv[k]]; x[piv[k]] = t; }
    for (int32_t i = 0; i < n; ++i)
        for (int32_t j = 0; j < i; ++j) x[i] -= a[(size_t)i * n + j] * x[j];
    for (int32_t i = n - 1; i >= 0; --i) {
        for (int32_t j = i + 1; j < n; ++j) x[i] -= a[(size_t)i * n + j] * x[j];
        x[i] /= a[(size_t)i * n + i];
    }
}

static void csr_copy_in(csr_t* dst, int32_t n, const int32_t* rowptr, const int32_t* col, const double* val)
{
    csr_alloc(dst, n, n, rowptr[n]);
    memcpy(dst->rowptr, rowptr, sizeof(int32_t) * ((size_t)n + 1));
    memcpy(dst->col, col, sizeof(int32_t) * (size_t)rowptr[n]);
    memcpy(dst->val, val, sizeof(double) * (size_t)rowptr[n]);
}

int or_amg_setup(int32_t n, const int32_t* rowptr, const int32_t* col,
                 const double* val, const or_amg_params* prm, or_amg** out)
{
    or_amg* h = calloc(1, sizeof(or_amg));
    h->prm = *prm;
    csr_copy_in(&h->A[0], n, rowptr, col, val);
    int32_t l = 0;
    int maxl = prm->max_levels < OR_MAXLEV ? prm->max_levels : OR_MAXLEV;
    for (;;) {
        csr_t* A = &h->A[l];
        h->dinv[l] = malloc(sizeof(double) * (size_t)(A->n > 0 ? A->n : 1));
        l1_dinv(A, h->dinv[l]);
        if (A->n <= prm->coarse_max || l + 1 >= maxl) break;
        csr_t S;
        strength(A, prm->theta, &S);
        int32_t* cf = malloc(sizeof(int32_t) * (size_t)(A->n > 0 ? A->n : 1));
        pmis(&S, prm->seed, l, cf);
        int32_t* cmap = malloc(sizeof(int32_t) * (size_t)(A->n > 0 ? A->n : 1));
        int32_t nc = 0;
        for (int32_t i = 0; i < A->n; ++i) cmap[i] = cf[i] ? nc++ : -1;
        if (nc == 0 || nc > 0.9 * (double)A->n) {   /* stalled or empty */
            free(cf); free(cmap); csr_free(&S);
            break;
        }
        h->cf[l] = cf;
        if (prm->interp == 1) ext_interp(A, &S, cf, cmap, nc, prm->interp_pmax, &h->P[l]);
        else direct_interp(A, &S, cf, cmap, nc, &h->P[l]);
        if (prm->restriction == 1) {
            /* Q = the same interpolation built from A^T on the same split; R = Q^T */
            csr_t At, St, Q;
            transpose(A, &At);
            strength(&At, prm->theta, &St);
            if (prm->interp == 1) ext_interp(&At, &St, cf, cmap, nc, prm->interp_pmax, &Q);
            else direct_interp(&At, &St, cf, cmap, nc, &Q);
            transpose(&Q, &h->R[l]);
            if (prm->interp == 1) h->Sq[l] = St;
            else csr_free(&St);
            csr_free(&At); csr_free(&Q);
        } else {
            transpose(&h->P[l], &h->R[l]);
        }
        csr_t AP;
        spgemm(A, &h->P[l], &AP);
        spgemm(&h->R[l], &AP, &h->A[l + 1]);
        csr_free(&AP);
        if (prm->interp == 1) h->S[l] = S;
        else csr_free(&S);
        free(cmap);
        ++l;
    }
    h->nlev = l + 1;
    if (!prm->skip_lu) {
        csr_t* A = &h->A[l];
        if (A->n > 4096) { *out = h; return -4; }
        h->nc = A->n;
        h->lu = calloc((size_t)A->n * (size_t)A->n + 1, sizeof(double));
        h->piv = malloc(sizeof(int32_t) * (size_t)(A->n > 0 ? A->n : 1));
        for (int32_t i = 0; i < A->n; ++i)
            for (int32_t k = A->rowptr[i]; k < A->rowptr[i + 1]; ++k)
                h->lu[(size_t)i * A->n + A->col[k]] = A->val[k];
        if (dense_lu(A->n, h->lu, h->piv) != 0) { *out = h; return -4; }
    }
    *out = h;
    return 0;
}

/* ---- numeric refresh: new level-0 values on a frozen hierarchy ------------
 * Setup reuse across Newton iterations: the C/F splits and the sparsity
 * patterns of every P, R and A_l are kept from the setup, and only values
 * are recomputed from the new level-0 operator, in the setup's order:
 *   interpolation  extended+i: see ext_refresh (the strength patterns are
 *                  kept too).  Direct: interpolation restricted to the frozen set P_i of
 *                  row i: with s = sign(a_ii), sum_all = sum of the
 *                  off-diagonal a_ik with s a_ik < 0, lump = sum of the
 *                  other off-diagonal a_ik, sum_p = sum of a_ij over j in
 *                  P_i with s a_ij < 0 (row order throughout),
 *                  w_ij = -(alpha a_ij) / (a_ii + lump), alpha = sum_all /
 *                  sum_p, for j in P_i with s a_ij < 0 and 0 for the other
 *                  entries of the frozen row (kept as explicit zeros); a row
 *                  with sum_p = 0 keeps its pattern with zero weights.  When
 *                  the frozen P_i is the strong C set of the new operator
 *                  (every such coupling has s a_ij < 0) this is exactly the
 *                  setup's direct interpolation;
 *   restriction    R = P^T, or R = Q^T with Q the same refresh applied to A^T
 *                  on the frozen pattern of Q = R^T (Petrov-Galerkin);
 *   coarse op.     A_{l+1} = R (A P), each entry summed in ascending inner
 *                  index; its pattern equals the frozen one;
 *   coarsest       dense LU with partial pivoting, as at setup.
 * Returns -4 on a zero pivot. */
static void refresh_interp(const csr_t* A, const int32_t* cf, const int32_t* cmap, csr_t* P)
{
    for (int32_t i = 0; i < A->n; ++i) {
        if (cf[i]) continue;                       /* C row: the unit vector, kept */
        const int32_t pa = P->rowptr[i], pe = P->rowptr[i + 1];
        if (pa == pe) continue;
        double aii = 0.0;
        for (int32_t k = A->rowptr[i]; k < A->rowptr[i + 1]; ++k)
            if (A->col[k] == i) aii = A->val[k];
        double s = aii < 0.0 ? -1.0 : 1.0;
        double sum_all = 0.0, lump = 0.0, sum_p = 0.0;
        for (int32_t k = A->rowptr[i]; k < A->rowptr[i + 1]; ++k) {
            if (A->col[k] == i) continue;
            double a = A->val[k];
            if (s * a < 0.0) sum_all += a;
            else lump += a;
        }
        for (int32_t k = A->rowptr[i]; k < A->rowptr[i + 1]; ++k) {
            int32_t j = A->col[k];
            if (j == i || !cf[j] || !(s * A->val[k] < 0.0)) continue;
            if (in_sorted(P->col + pa, pe - pa, cmap[j]) >= 0) sum_p += A->val[k];
        }
        for (int32_t q = pa; q < pe; ++q) P->val[q] = 0.0;
        if (sum_p == 0.0) continue;
        double alpha = sum_all / sum_p;
        double dtil = aii + lump;
        for (int32_t k = A->rowptr[i]; k < A->rowptr[i + 1]; ++k) {
            int32_t j = A->col[k];
            if (j == i || !cf[j] || !(s * A->val[k] < 0.0)) continue;
            int32_t t = in_sorted(P->col + pa, pe - pa, cmap[j]);
            if (t >= 0) P->val[pa + t] = -(alpha * A->val[k]) / dtil;
        }
    }
}

int or_amg_refresh(or_amg* h, const double* val)
{
    memcpy(h->A[0].val, val, sizeof(double) * (size_t)h->A[0].nnz);
    for (int32_t l = 0; l < h->nlev; ++l) {
        csr_t* A = &h->A[l];
        l1_dinv(A, h->dinv[l]);
        if (l == h->nlev - 1) break;
        int32_t* cmap = malloc(sizeof(int32_t) * (size_t)(A->n > 0 ? A->n : 1));
        int32_t nc = 0;
        for (int32_t i = 0; i < A->n; ++i) cmap[i] = h->cf[l][i] ? nc++ : -1;
        if (h->prm.interp == 1) ext_refresh(A, &h->S[l], h->cf[l], cmap, &h->P[l]);
        else refresh_interp(A, h->cf[l], cmap, &h->P[l]);
        csr_t T;
        if (h->prm.restriction == 1) {
            csr_t At, Q;
            transpose(A, &At);
            transpose(&h->R[l], &Q);               /* the frozen pattern of Q = R^T */
            if (h->prm.interp == 1) ext_refresh(&At, &h->Sq[l], h->cf[l], cmap, &Q);
            else refresh_interp(&At, h->cf[l], cmap, &Q);
            transpose(&Q, &T);
            csr_free(&At); csr_free(&Q);
        } else {
            transpose(&h->P[l], &T);
        }
        memcpy(h->R[l].val, T.val, sizeof(double) * (size_t)T.nnz);
        csr_free(&T);
        csr_t AP, Ac;
        spgemm(A, &h->P[l], &AP);
        spgemm(&h->R[l], &AP, &Ac);
        csr_t* An = &h->A[l + 1];
        if (Ac.nnz != An->nnz || memcmp(Ac.col, An->col, sizeof(int32_t) * (size_t)Ac.nnz) != 0) {
            csr_free(&AP); csr_free(&Ac); free(cmap);
            return -1;                                 /* cannot happen: patterns are frozen */
        }
        memcpy(An->val, Ac.val, sizeof(double) * (size_t)Ac.nnz);
        csr_free(&AP); csr_free(&Ac); free(cmap);
    }
    if (!h->prm.skip_lu) {
        csr_t* A = &h->A[h->nlev - 1];
        memset(h->lu, 0, sizeof(double) * (size_t)A->n * (size_t)A->n);
        for (int32_t i = 0; i < A->n; ++i)
            for (int32_t k = A->rowptr[i]; k < A->rowptr[i + 1]; ++k)
                h->lu[(size_t)i * A->n + A->col[k]] = A->val[k];
        if (dense_lu(A->n, h->lu, h->piv) != 0) return -4;
    }
    return 0;
}

void or_amg_free(or_amg* h)
{
    if (!h) return;
    for (int32_t l = 0; l < OR_MAXLEV; ++l) {
        csr_free(&h->A[l]); csr_free(&h->P[l]); csr_free(&h->R[l]);
        csr_free(&h->S[l]); csr_free(&h->Sq[l]);
        free(h->dinv[l]); free(h->cf[l]);
    }
    free(h->lu); free(h->piv);
    free(h);
}

int32_t or_amg_nlev(const or_amg* h) { return h->nlev; }

void or_amg_level_sizes(const or_amg* h, int32_t l, int32_t* n, int32_t* nnzA, int32_t* nnzP)
{
    *n = h->A[l].n;
    *nnzA = h->A[l].nnz;
    *nnzP = (l + 1 < h->nlev) ? h->P[l].nnz : 0;
}

void or_amg_level_copy(const or_amg* h, int32_t l, int32_t* A_rowptr, int32_t* A_col,
                       double* A_val, int32_t* cf, int32_t* P_rowptr, int32_t* P_col,
                       double* P_val, double* dinv)
{
    const csr_t* A = &h->A[l];
    if (A_rowptr) memcpy(A_rowptr, A->rowptr, sizeof(int32_t) * ((size_t)A->n + 1));
    if (A_col) memcpy(A_col, A->col, sizeof(int32_t) * (size_t)A->nnz);
    if (A_val) memcpy(A_val, A->val, sizeof(double) * (size_t)A->nnz);
    if (dinv) memcpy(dinv, h->dinv[l], sizeof(double) * (size_t)A->n);
    if (l + 1 < h->nlev) {
        const csr_t* P = &h->P[l];
        if (cf) memcpy(cf, h->cf[l], sizeof(int32_t) * (size_t)A->n);
        if (P_rowptr) memcpy(P_rowptr, P->rowptr, sizeof(int32_t) * ((size_t)P->n + 1));
        if (P_col) memcpy(P_col, P->col, sizeof(int32_t) * (size_t)P->nnz);
        if (P_val) memcpy(P_val, P->val, sizeof(double) * (size_t)P->nnz);
    }
}

/* One smoothing sweep on A x = b starting from x (x_is_zero: x == 0).
 * l1-Jacobi: x += w D^{-1}(b - A x), repeated nu times.
 * Chebyshev of degree k on D^{-1} A with eigenvalues in [lo, 1]:
 *   theta = (1+lo)/2, delta = (1-lo)/2, sigma = theta/delta, rho_0 = 1/sigma;
 *   r = D^{-1}(b - A x); d = r/theta; x += d;
 *   then k-1 times: r = D^{-1}(b - A x); rho_1 = 1/(2 sigma - rho_0);
 *                   d = rho_1 rho_0 d + (2 rho_1/delta) r; x += d; rho_0 = rho_1. */
static void smooth(const or_amg* h, int32_t l, const double* b, double* x, int x_is_zero,
                   int32_t nu, double* r, double* d)
{
    const csr_t* A = &h->A[l];
    int32_t n = A->n;
    const double* dinv = h->dinv[l];
    for (int32_t s = 0; s < nu; ++s) {
        int zero = x_is_zero && s == 0;
        if (h->prm.smoother == 0) {
            double w = h->prm.omega;
            if (zero) {
                for (int32_t i = 0; i < n; ++i) x[i] = w * dinv[i] * b[i];
            } else {
                or_spmv(n, A->rowptr, A->col, A->val, x, r);
                for (int32_t i = 0; i < n; ++i) x[i] += w * dinv[i] * (b[i] - r[i]);
            }
            continue;
        }
        double lo = h->prm.cheb_lo;
        double theta = 0.5 * (1.0 + lo), delta = 0.5 * (1.0 - lo);
        double sigma = theta / delta, rho0 = 1.0 / sigma;
        if (zero) {
            for (int32_t i = 0; i < n; ++i) r[i] = dinv[i] * b[i];
        } else {
            or_spmv(n, A->rowptr, A->col, A->val, x, r);
            for (int32_t i = 0; i < n; ++i) r[i] = dinv[i] * (b[i] - r[i]);
        }
        for (int32_t i = 0; i < n; ++i) { d[i] = r[i] / theta; x[i] = (zero ? 0.0 : x[i]) + d[i]; }
        const int32_t deg = (l > 0 && h->prm.cheb_degree_coarse > 0) ? h->prm.cheb_degree_coarse
                                                                      : h->prm.cheb_degree;
        for (int32_t k = 1; k < deg; ++k) {
            double rho1 = 1.0 / (2.0 * sigma - rho0);
            double c1 = rho1 * rho0, c2 = 2.0 * rho1 / delta;
            or_spmv(n, A->rowptr, A->col, A->val, x, r);
            for (int32_t i = 0; i < n; ++i) r[i] = dinv[i] * (b[i] - r[i]);
            for (int32_t i = 0; i < n; ++i) { d[i] = c1 * d[i] + c2 * r[i]; x[i] += d[i]; }
            rho0 = rho1;
        }
    }
}

int32_t or_amg_level_R_nnz(const or_amg* h, int32_t l)
{
    return (l + 1 < h->nlev) ? h->R[l].nnz : 0;
}

void or_amg_level_R_copy(const or_amg* h, int32_t l, int32_t* rowptr, int32_t* col, double* val)
{
    if (l + 1 >= h->nlev) return;
    const csr_t* R = &h->R[l];
    if (rowptr) memcpy(rowptr, R->rowptr, sizeof(int32_t) * ((size_t)R->n + 1));
    if (col) memcpy(col, R->col, sizeof(int32_t) * (size_t)R->nnz);
    if (val) memcpy(val, R->val, sizeof(double) * (size_t)R->nnz);
}

static void vcycle_level(const or_amg* h, int32_t l, const double* b, double* x)
{
    const csr_t* A = &h->A[l];
    int32_t n = A->n;
    if (l == h->nlev - 1) {
        dense_lu_solve(h->nc, h->lu, h->piv, b, x);
        return;
    }
    double* r = malloc(sizeof(double) * (size_t)(n > 0 ? n : 1));
    double* d = malloc(sizeof(double) * (size_t)(n > 0 ? n : 1));
    /* pre-smoothing from a zero guess */
    smooth(h, l, b, x, 1, h->prm.nu_pre, r, d);
    if (h->prm.nu_pre == 0) for (int32_t i = 0; i < n; ++i) x[i] = 0.0;
    /* residual, restriction, coarse correction */
    or_spmv(n, A->rowptr, A->col, A->val, x, r);
    for (int32_t i = 0; i < n; ++i) r[i] = b[i] - r[i];
    int32_t nc = h->A[l + 1].n;
    double* bc = malloc(sizeof(double) * (size_t)(nc > 0 ? nc : 1));
    double* xc = malloc(sizeof(double) * (size_t)(nc > 0 ? nc : 1));
    or_spmv(nc, h->R[l].rowptr, h->R[l].col, h->R[l].val, r, bc);
    vcycle_level(h, l + 1, bc, xc);
    const csr_t* P = &h->P[l];
    for (int32_t i = 0; i < n; ++i) {
        double s = 0.0;
        for (int32_t k = P->rowptr[i]; k < P->rowptr[i + 1]; ++k) s += P->val[k] * xc[P->col[k]];
        x[i] += s;
    }
    /* post-smoothing */
    smooth(h, l, b, x, 0, h->prm.nu_post, r, d);
    free(r); free(d); free(bc); free(xc);
}

void or_vcycle(const or_amg* h, const double* b, double* x)
{
    vcycle_level(h, 0, b, x);
}
