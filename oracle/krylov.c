/*
 * krylov.c -- oracle block preconditioner and restarted GMRES.
 *
 * TEST INFRASTRUCTURE ONLY (see tp_oracle.h).  Plain FP64, sequential,
 * vectors interleaved [p_0, T_0, p_1, T_1, ...] as the Jacobian of eq. AXR is
 * ordered cell by cell.
 *
 * Preconditioner (Section 3.2, the five-step application list):
 *   lower  : steps 1-3  x_p = V_pp(b_p); b~_T = b_T - A_Tp x_p; d_T = V_S(b~_T)
 *   full   : steps 1-5, reading step 4 as b~_p = b_p - A_pT d_T (the printed
 *            x_p there is taken as a typo for b_p); step 5 solves A_pp again
 *   upper  : d_T = V_S(b_T); x_p = V_pp(b_p - A_pT d_T)
 * GMRES (Saad & Schultz 1986) right-preconditioned, restarted every
 * `restart` steps (Section 4: restart 30), with classical Gram-Schmidt
 * applied twice (CGS2), Givens rotations on the Hessenberg matrix, and an
 * FP64 true residual ||b - A x|| / ||b|| after each cycle.
 */
#include "tp_oracle.h"
#include <math.h>
#include <stdlib.h>
#include <string.h>

static void blk_spmv(const or_jac* J, const double* pp_or_Tp, const double* x, double* y)
{
    or_spmv(J->n, J->rowptr, J->col, pp_or_Tp, x, y);
}

/* y = J x, interleaved */
static void jac_apply(const or_jac* J, const double* x, double* y)
{
    for (int32_t i = 0; i < J->n; ++i) {
        double sm = 0.0, se = 0.0;
        for (int32_t k = J->rowptr[i]; k < J->rowptr[i + 1]; ++k) {
            int32_t j = J->col[k];
            sm += J->pp[k] * x[2 * j] + J->pT[k] * x[2 * j + 1];
            se += J->Tp[k] * x[2 * j] + J->TT[k] * x[2 * j + 1];
        }
        y[2 * i] = sm;
        y[2 * i + 1] = se;
    }
}

void or_precond_apply(const or_jac* J, const or_amg* amg_pp, const or_amg* amg_S,
                      int32_t variant, const double* r, double* z)
{
    int32_t n = J->n;
    if (variant < 0) { memcpy(z, r, sizeof(double) * 2 * (size_t)n); return; }
    double* rp = malloc(sizeof(double) * (size_t)n);
    double* rT = malloc(sizeof(double) * (size_t)n);
    double* zp = malloc(sizeof(double) * (size_t)n);
    double* zT = malloc(sizeof(double) * (size_t)n);
    double* t = malloc(sizeof(double) * (size_t)n);
    for (int32_t i = 0; i < n; ++i) { rp[i] = r[2 * i]; rT[i] = r[2 * i + 1]; }
    if (variant == 1) {
        or_vcycle(amg_S, rT, zT);
        blk_spmv(J, J->pT, zT, t);
        for (int32_t i = 0; i < n; ++i) t[i] = rp[i] - t[i];
        or_vcycle(amg_pp, t, zp);
    } else {
        /* step 1 */
        or_vcycle(amg_pp, rp, zp);
        /* step 2 */
        blk_spmv(J, J->Tp, zp, t);
        for (int32_t i = 0; i < n; ++i) t[i] = rT[i] - t[i];
        /* step 3 */
        or_vcycle(amg_S, t, zT);
        if (variant == 2) {
            /* step 4 and 5 */
            blk_spmv(J, J->pT, zT, t);
            for (int32_t i = 0; i < n; ++i) t[i] = rp[i] - t[i];
            or_vcycle(amg_pp, t, zp);
        }
    }
    for (int32_t i = 0; i < n; ++i) { z[2 * i] = zp[i]; z[2 * i + 1] = zT[i]; }
    free(rp); free(rT); free(zp); free(zT); free(t);
}

static double dot(int32_t m, const double* a, const double* b)
{
    double s = 0.0;
    for (int32_t i = 0; i < m; ++i) s += a[i] * b[i];
    return s;
}

/* the preconditioner as z = apply(ctx, r) */
typedef void (*prec_fn)(const void* ctx, const double* r, double* z);

struct blk_ctx { const or_jac* J; const or_amg* pp; const or_amg* S; int32_t variant; };
static void blk_prec(const void* c, const double* r, double* z)
{
    const struct blk_ctx* b = c;
    or_precond_apply(b->J, b->pp, b->S, b->variant, r, z);
}

struct cpr_ctx { const or_jac* J; const or_amg* pp; const or_ilu* F; };
static void cpr_prec(const void* c, const double* r, double* z)
{
    const struct cpr_ctx* b = c;
    or_cpr_apply(b->J, b->pp, b->F, r, z);
}

static int gmres_core(const or_jac* J, prec_fn prec, const void* ctx, const double* b, double* x,
                      double rtol, int32_t restart, int32_t maxit, int32_t* iters,
                      double* rel_true, double* history)
{
    int32_t m = 2 * J->n, it = 0, mr = restart;
    double* V = malloc(sizeof(double) * (size_t)m * (size_t)(mr + 1));
    double* Z = malloc(sizeof(double) * (size_t)m * (size_t)mr);
    double* H = calloc((size_t)(mr + 1) * (size_t)mr, sizeof(double));  /* H[i*mr + j] */
    double* cs = malloc(sizeof(double) * (size_t)mr);
    double* sn = malloc(sizeof(double) * (size_t)mr);
    double* gv = malloc(sizeof(double) * (size_t)(mr + 1));
    double* y = malloc(sizeof(double) * (size_t)mr);
    double* h1 = malloc(sizeof(double) * (size_t)(mr + 1));
    double* w = malloc(sizeof(double) * (size_t)m);
    double* r = malloc(sizeof(double) * (size_t)m);
    double bnorm = sqrt(dot(m, b, b));
    int converged = 0;
    double rel = 0.0;
    if (bnorm == 0.0) {
        memset(x, 0, sizeof(double) * (size_t)m);
        *iters = 0; *rel_true = 0.0;
        if (history) history[0] = 0.0;
        converged = 1;
        goto done;
    }
    jac_apply(J, x, r);
    for (int32_t i = 0; i < m; ++i) r[i] = b[i] - r[i];
    rel = sqrt(dot(m, r, r)) / bnorm;
    if (history) history[0] = rel;
    while (rel > rtol && it < maxit) {
        double beta = sqrt(dot(m, r, r));
        for (int32_t i = 0; i < m; ++i) V[i] = r[i] / beta;
        memset(gv, 0, sizeof(double) * (size_t)(mr + 1));
        gv[0] = beta;
        int32_t j, k = 0;
        for (j = 0; j < mr && it < maxit; ++j) {
            double* vj = V + (size_t)j * m;
            double* zj = Z + (size_t)j * m;
            prec(ctx, vj, zj);
            jac_apply(J, zj, w);
            /* CGS2: two classical Gram-Schmidt passes */
            for (int32_t i = 0; i <= j; ++i) H[(size_t)i * mr + j] = 0.0;
            for (int pass = 0; pass < 2; ++pass) {
                for (int32_t i = 0; i <= j; ++i) h1[i] = dot(m, V + (size_t)i * m, w);
                for (int32_t i = 0; i <= j; ++i) {
                    const double* vi = V + (size_t)i * m;
                    for (int32_t q = 0; q < m; ++q) w[q] -= h1[i] * vi[q];
                    H[(size_t)i * mr + j] += h1[i];
                }
            }
            double hn = sqrt(dot(m, w, w));
            H[(size_t)(j + 1) * mr + j] = hn;
            if (hn > 0.0)
                for (int32_t q = 0; q < m; ++q) V[(size_t)(j + 1) * m + q] = w[q] / hn;
            /* apply previous rotations, then a new one */
            for (int32_t i = 0; i < j; ++i) {
                double a = H[(size_t)i * mr + j], c = H[(size_t)(i + 1) * mr + j];
                H[(size_t)i * mr + j] = cs[i] * a + sn[i] * c;
                H[(size_t)(i + 1) * mr + j] = -sn[i] * a + cs[i] * c;
            }
            double a = H[(size_t)j * mr + j], c = H[(size_t)(j + 1) * mr + j];
            double den = hypot(a, c);
            cs[j] = a / den;
            sn[j] = c / den;
            H[(size_t)j * mr + j] = den;
            H[(size_t)(j + 1) * mr + j] = 0.0;
            gv[j + 1] = -sn[j] * gv[j];
            gv[j] = cs[j] * gv[j];
            ++it;
            k = j + 1;
            double est = fabs(gv[j + 1]) / bnorm;
            if (history) history[it] = est;
            if (est <= rtol || hn == 0.0) break;
        }
        /* y = H^{-1} g (upper triangular k x k), x += Z y */
        for (int32_t i = k - 1; i >= 0; --i) {
            double s = gv[i];
            for (int32_t q = i + 1; q < k; ++q) s -= H[(size_t)i * mr + q] * y[q];
            y[i] = s / H[(size_t)i * mr + i];
        }
        for (int32_t i = 0; i < k; ++i) {
            const double* zi = Z + (size_t)i * m;
            for (int32_t q = 0; q < m; ++q) x[q] += y[i] * zi[q];
        }
        jac_apply(J, x, r);
        for (int32_t i = 0; i < m; ++i) r[i] = b[i] - r[i];
        rel = sqrt(dot(m, r, r)) / bnorm;
    }
    converged = rel <= rtol;
    *iters = it;
    *rel_true = rel;
done:
    free(V); free(Z); free(H); free(cs); free(sn); free(gv); free(y); free(h1); free(w); free(r);
    return converged ? 0 : 1;
}

int or_gmres(const or_jac* J, const or_amg* amg_pp, const or_amg* amg_S,
             int32_t variant, const double* b, double* x, double rtol,
             int32_t restart, int32_t maxit, int32_t* iters, double* rel_true,
             double* history)
{
    struct blk_ctx c = { J, amg_pp, amg_S, variant };
    return gmres_core(J, blk_prec, &c, b, x, rtol, restart, maxit, iters, rel_true, history);
}

int or_gmres_cpr(const or_jac* J, const or_amg* amg_pp, const or_ilu* F, const double* b,
                 double* x, double rtol, int32_t restart, int32_t maxit, int32_t* iters,
                 double* rel_true, double* history)
{
    struct cpr_ctx c = { J, amg_pp, F };
    return gmres_core(J, cpr_prec, &c, b, x, rtol, restart, maxit, iters, rel_true, history);
}
