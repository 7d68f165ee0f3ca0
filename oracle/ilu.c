/*
 * ilu.c -- oracle ILU(0) and the two-stage CPR preconditioner.
 *
 * TEST INFRASTRUCTURE ONLY (see tp_oracle.h).  Plain FP64, sequential.
 *
 * ILU(0) (Section 3, the incomplete factorisations named there; Saad,
 * "Iterative Methods for Sparse Linear Systems", 2003, Section 10.3):
 * A ~ L U with L unit lower triangular and U upper triangular, both on the
 * sparsity pattern of A.  Gaussian elimination is run row by row (the IKJ
 * ordering): row i subtracts multiples of the finished rows k < i that its
 * pattern holds, in increasing k, and every update whose position lies
 * outside the pattern of A is dropped.  L (below the diagonal, unit
 * diagonal implied) and U (diagonal and above) overwrite a copy of A's
 * values in place.
 *
 * Two-stage preconditioner (Section 3.1): x1 = M1^{-1} b; b1 = b - A x1;
 * x = M2^{-1} b1 + x1.  For CPR, M1^{-1} is one AMG V-cycle on A_pp in the
 * pressure rows and zero in the temperature rows, and M2 is ILU(0) of the
 * whole Jacobian (Section 4: PETSc's ILU(0) in serial).  The whole Jacobian
 * is factorised in the field-by-field order of eq. AXR ([p_0..p_{n-1},
 * T_0..T_{n-1}]), the numbering of a mixed space assembled as one matrix;
 * the vectors of the solver interface stay interleaved [p_i, T_i].
 */
#include "tp_oracle.h"
#include <math.h>
#include <stdlib.h>
#include <string.h>

int or_ilu0(int32_t N, const int32_t* rowptr, const int32_t* col, const double* a, double* lu)
{
    memcpy(lu, a, sizeof(double) * (size_t)rowptr[N]);
    int32_t* pos = malloc(sizeof(int32_t) * (size_t)(N > 0 ? N : 1));  /* column -> slot in row i */
    int32_t* dg = malloc(sizeof(int32_t) * (size_t)(N > 0 ? N : 1));   /* slot of the diagonal */
    for (int32_t j = 0; j < N; ++j) pos[j] = -1;
    int status = 0;
    for (int32_t i = 0; i < N && status == 0; ++i) {
        dg[i] = -1;
        for (int32_t q = rowptr[i]; q < rowptr[i + 1]; ++q) {
            pos[col[q]] = q;
            if (col[q] == i) dg[i] = q;
        }
        if (dg[i] < 0) status = -1;
        for (int32_t q = rowptr[i]; q < rowptr[i + 1] && status == 0; ++q) {
            int32_t k = col[q];
            if (k >= i) continue;
            /* multiplier l_ik = a_ik / u_kk */
            double lik = lu[q] / lu[dg[k]];
            lu[q] = lik;
            /* a_ij -= l_ik u_kj for j > k, kept only where (i, j) is in the pattern */
            for (int32_t t = rowptr[k]; t < rowptr[k + 1]; ++t) {
                int32_t j = col[t];
                if (j <= k) continue;
                if (pos[j] >= 0) lu[pos[j]] -= lik * lu[t];
            }
        }
        if (status == 0 && lu[dg[i]] == 0.0) status = -4;
        for (int32_t q = rowptr[i]; q < rowptr[i + 1]; ++q) pos[col[q]] = -1;
    }
    free(pos);
    free(dg);
    return status;
}

void or_ilu0_solve(int32_t N, const int32_t* rowptr, const int32_t* col, const double* lu,
                   const double* b, double* x)
{
    /* L y = b (unit diagonal), in increasing row order */
    for (int32_t i = 0; i < N; ++i) {
        double s = b[i];
        for (int32_t q = rowptr[i]; q < rowptr[i + 1]; ++q)
            if (col[q] < i) s -= lu[q] * x[col[q]];
        x[i] = s;
    }
    /* U x = y, in decreasing row order */
    for (int32_t i = N - 1; i >= 0; --i) {
        double s = x[i], d = 0.0;
        for (int32_t q = rowptr[i]; q < rowptr[i + 1]; ++q) {
            if (col[q] > i) s -= lu[q] * x[col[q]];
            else if (col[q] == i) d = lu[q];
        }
        x[i] = s / d;
    }
}

/* The whole Jacobian in field-by-field order: row p_i holds A_pp(i,:) then
 * A_pT(i,:) (columns j and n + j), row T_i holds A_Tp(i,:) then A_TT(i,:);
 * every stored entry of the four blocks is kept, zeros included. */
void or_jac_fieldwise(const or_jac* J, int32_t* rowptr, int32_t* col, double* val)
{
    int32_t n = J->n, q = 0;
    rowptr[0] = 0;
    for (int32_t f = 0; f < 2; ++f) {
        const double* left = f == 0 ? J->pp : J->Tp;
        const double* right = f == 0 ? J->pT : J->TT;
        for (int32_t i = 0; i < n; ++i) {
            for (int32_t k = J->rowptr[i]; k < J->rowptr[i + 1]; ++k) {
                col[q] = J->col[k];
                val[q++] = left[k];
            }
            for (int32_t k = J->rowptr[i]; k < J->rowptr[i + 1]; ++k) {
                col[q] = n + J->col[k];
                val[q++] = right[k];
            }
            rowptr[f * n + i + 1] = q;
        }
    }
}

/* x = M^{-1} r for the CPR two-stage preconditioner; r and x interleaved. */
void or_cpr_apply(const or_jac* J, const or_amg* amg_pp, const or_ilu* F, const double* r, double* x)
{
    int32_t n = J->n;
    double* rp = malloc(sizeof(double) * (size_t)n);
    double* x1p = malloc(sizeof(double) * (size_t)n);
    double* t = malloc(sizeof(double) * (size_t)n);
    double* b1 = malloc(sizeof(double) * 2 * (size_t)n);
    double* y = malloc(sizeof(double) * 2 * (size_t)n);
    /* stage 1: x1 = [V_pp(r_p); 0] */
    for (int32_t i = 0; i < n; ++i) rp[i] = r[2 * i];
    or_vcycle(amg_pp, rp, x1p);
    /* b1 = r - A x1 (only the pressure columns of A meet x1), field order */
    or_spmv(n, J->rowptr, J->col, J->pp, x1p, t);
    for (int32_t i = 0; i < n; ++i) b1[i] = r[2 * i] - t[i];
    or_spmv(n, J->rowptr, J->col, J->Tp, x1p, t);
    for (int32_t i = 0; i < n; ++i) b1[n + i] = r[2 * i + 1] - t[i];
    /* stage 2: x = M2^{-1} b1 + x1 */
    or_ilu0_solve(F->N, F->rowptr, F->col, F->lu, b1, y);
    for (int32_t i = 0; i < n; ++i) {
        x[2 * i] = y[i] + x1p[i];
        x[2 * i + 1] = y[n + i];
    }
    free(rp); free(x1p); free(t); free(b1); free(y);
}
