/*
 * tp_oracle.h -- plain, slow, single-threaded FP64 CPU oracle.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library links, calls or
 * includes this code; only the test-suite, the smoke check and the CPU
 * baseline leg of the benchmark load it.  It shares no source with the HIP
 * path.  Every routine follows a passage of Roy, Jonsthovel, Lemon & Wathen,
 * "A block preconditioner for non-isothermal flow in porous media" (2019), or
 * a published algorithm named at the routine, written in the order of that
 * description without blocking, fusion or reordering.
 *
 * Build: gcc -std=c99 -O2 -ffp-contract=off -fPIC -shared (no fast-math).
 */
#ifndef TP_ORACLE_H
#define TP_ORACLE_H

#include <stdint.h>
#include <complex.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct { int32_t nx, ny, nz; double dx, dy, dz; } or_grid;
/* api > 0 selects the Bennison viscosity (Section 2.1, eq. bennison) in
 * place of mu0 exp(mu_B (1/T - 1/T0)). */
typedef struct { double rho0, p0, T0, c_p, c_T, mu0, mu_B, cv, rho_r, c_r, g, api; } or_props;
/* kind 0 injector, 1 producer (rate in m^3/s); kind 2 heater: rate is the
 * heat-transfer coefficient U (W/K) and T_inj the heater temperature */
/* kind 0 injector, 1 producer (rate m^3/s), 2 heater (rate = U, T_inj =
 * T_heater), 3 / 4 Peaceman injector / producer (Section 2.1: rate
 * wi (p_bh - p) / mu or wi (p - p_bh) / mu, clamped to [0, rate]). */
typedef struct { int32_t cell, kind; double rate, T_inj, p_bh, wi; } or_well;

/* ---- Section 2.2: TPFA discretisation ---------------------------------- */
int32_t or_stencil_nnz(const or_grid* g);
/* Sorted 5/7-point stencil pattern; returns nnz. */
int32_t or_stencil_pattern(const or_grid* g, int32_t* rowptr, int32_t* col);

/* K is the permeability: kstride 0 for a scalar per cell (n values), or
 * kstride n for the diagonal tensor diag(K_x, K_y, K_z) of the Peaceman
 * discussion in Section 2.1, stored as [K_x(n), K_y(n), K_z(n)]; a face
 * normal to axis a takes the harmonic mean of its two cells' K_a.
 * Residual G(x) of eq. (Fm)/(Fe) on complex states (complex-step checks). */
void or_residual_c(const or_grid* g, const or_props* pr, const double* K,
                   int32_t kstride, const double* phi, const double* kappa, int32_t nw,
                   const or_well* w, double dt, const double* x_prev,
                   const double complex* x, double complex* G);
/* Residual on real states (interleaved [p_i, T_i]). */
void or_residual(const or_grid* g, const or_props* pr, const double* K,
                 int32_t kstride, const double* phi, const double* kappa, int32_t nw,
                 const or_well* w, double dt, const double* x_prev,
                 const double* x, double* G);
/* Jacobian blocks (eq. AXR) and the Schur approximation of eq. (Se), all on
 * the stencil pattern. */
void or_jacobian(const or_grid* g, const or_props* pr, const double* K,
                 int32_t kstride, const double* phi, const double* kappa, int32_t nw,
                 const or_well* w, double dt, const double* x_prev,
                 const double* x, const int32_t* rowptr, const int32_t* col,
                 double* App, double* ApT, double* ATp, double* ATT, double* S);

/* ---- AMG (Section 3 background; components per the method description) */
typedef struct {
    double theta;        /* strength threshold (0.25) */
    uint64_t seed;       /* PMIS hash seed */
    int32_t max_levels;  /* 25 */
    int32_t coarse_max;  /* stop at n_l <= coarse_max (256) */
    double omega;        /* l1-Jacobi weight (1.0) */
    int32_t nu_pre, nu_post;
    int32_t skip_lu;     /* 1: build levels only (coarsening tests) */
    int32_t smoother;    /* 0 l1-Jacobi, 1 Chebyshev on the l1-scaled operator */
    int32_t cheb_degree; /* polynomial degree per smoothing sweep (3) */
    double cheb_lo;      /* interval [cheb_lo, 1] of D_l1^{-1} A (0.3) */
    int32_t restriction; /* 0 Galerkin R = P^T; 1 Petrov-Galerkin R = P(A^T)^T */
    int32_t cheb_degree_coarse; /* degree on levels >= 1 (0: cheb_degree) */
    int32_t interp;      /* 0 direct interpolation; 1 extended+i */
    int32_t interp_pmax; /* extended+i: keep at most this many weights per row (0: all) */
} or_amg_params;

typedef struct or_amg or_amg;
/* returns 0 on success, -4 on numeric failure (zero pivot / stalled large level) */
int or_amg_setup(int32_t n, const int32_t* rowptr, const int32_t* col,
                 const double* val, const or_amg_params* prm, or_amg** out);
void or_amg_free(or_amg* h);
int32_t or_amg_nlev(const or_amg* h);
/* sizes of level l: n, nnz(A_l), nnz(P_l) (0 on the coarsest) */
void or_amg_level_sizes(const or_amg* h, int32_t l, int32_t* n, int32_t* nnzA, int32_t* nnzP);
/* copy level arrays out (any pointer may be NULL) */
void or_amg_level_copy(const or_amg* h, int32_t l, int32_t* A_rowptr, int32_t* A_col,
                       double* A_val, int32_t* cf, int32_t* P_rowptr, int32_t* P_col,
                       double* P_val, double* dinv);
/* restriction R_l (n_{l+1} x n_l): nnz, then copy (pointers may be NULL) */
int32_t or_amg_level_R_nnz(const or_amg* h, int32_t l);
void or_amg_level_R_copy(const or_amg* h, int32_t l, int32_t* rowptr, int32_t* col, double* val);
/* Numeric refresh for a new level-0 operator on the same pattern: C/F
 * splits, strength patterns (extended+i) and every sparsity pattern frozen,
 * values recomputed (see amg.c).  0 on success, -4 on a zero pivot. */
int or_amg_refresh(or_amg* h, const double* val);
/* one V-cycle with zero initial guess: x = V(b) */
void or_vcycle(const or_amg* h, const double* b, double* x);
void or_spmv(int32_t n, const int32_t* rowptr, const int32_t* col, const double* val,
             const double* x, double* y);
/* SplitMix64 output for state x (PMIS tie-break hash) */
uint64_t or_splitmix64(uint64_t x);

/* ---- Block preconditioner (Section 3.2) and GMRES --------------------- */
typedef struct {
    int32_t n;
    const int32_t *rowptr, *col;
    const double *pp, *pT, *Tp, *TT;
} or_jac;

/* variant: 0 lower (steps 1-3), 1 upper, 2 full five-step, -1 identity.
 * r and z are interleaved [p_i, T_i]. */
void or_precond_apply(const or_jac* J, const or_amg* amg_pp, const or_amg* amg_S,
                      int32_t variant, const double* r, double* z);
/* Right-preconditioned restarted GMRES with CGS2; interleaved vectors.
 * x: in initial guess, out solution.  history (optional): maxit+1 entries of
 * the relative residual estimate.  Returns 0 if converged, 1 otherwise. */
int or_gmres(const or_jac* J, const or_amg* amg_pp, const or_amg* amg_S,
             int32_t variant, const double* b, double* x, double rtol,
             int32_t restart, int32_t maxit, int32_t* iters, double* rel_true,
             double* history);

/* ---- ILU(0) and the two-stage CPR preconditioner (see ilu.c) ---------- */
typedef struct {
    int32_t N;
    const int32_t *rowptr, *col;  /* pattern of the factorised matrix, sorted rows */
    const double* lu;             /* L (strictly lower, unit diagonal implied) and U */
} or_ilu;

/* ILU(0) of the N x N CSR matrix (sorted columns, diagonal stored) into lu
 * (same pattern).  Returns 0, -1 if a row has no diagonal entry, -4 on a zero
 * pivot. */
int or_ilu0(int32_t N, const int32_t* rowptr, const int32_t* col, const double* a, double* lu);
/* x = U^{-1} L^{-1} b */
void or_ilu0_solve(int32_t N, const int32_t* rowptr, const int32_t* col, const double* lu,
                   const double* b, double* x);
/* The 2n x 2n Jacobian in field-by-field order ([p; T]) from its four blocks:
 * rowptr (2n+1), col and val (4 nnz). */
void or_jac_fieldwise(const or_jac* J, int32_t* rowptr, int32_t* col, double* val);
/* CPR: x1 = [V_pp(r_p); 0]; x = ILU0^{-1}(r - J x1) + x1, with F the ILU(0) of
 * the field-by-field Jacobian; r and x interleaved. */
void or_cpr_apply(const or_jac* J, const or_amg* amg_pp, const or_ilu* F, const double* r, double* x);
/* GMRES (as or_gmres) right-preconditioned by CPR */
int or_gmres_cpr(const or_jac* J, const or_amg* amg_pp, const or_ilu* F, const double* b,
                 double* x, double rtol, int32_t restart, int32_t maxit, int32_t* iters,
                 double* rel_true, double* history);

/* ---- Learned post-smoother network (see cnn.c) ------------------------ */
void or_cnn_forward(const or_grid* g, const double* W1, const double* b1, const double* W2,
                    double b2, const double* f, double* h, double* out);
double or_cnn_backward(const or_grid* g, const double* W1, const double* b1, const double* W2,
                       double b2, const double* f, const double* y, double* grad);
double or_cnn_features(const or_grid* g, const int32_t* rowptr, const int32_t* col,
                       const double* val, const double* r, double* f);

#ifdef __cplusplus
}
#endif
#endif
