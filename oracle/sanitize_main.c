/*
 * sanitize_main.c -- drives every oracle routine once on small grids, for a
 * build with AddressSanitizer and UndefinedBehaviorSanitizer (test
 * infrastructure: the CPU test-suite compiles it with the oracle sources and
 * runs it; any out-of-bounds access, leak-free misuse or undefined operation
 * aborts the run).  Inputs are deterministic: a linear congruential sequence
 * (Knuth's MMIX constants) stands in for the seeded fields of the workloads.
 */
#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include "tp_oracle.h"

static uint64_t lcg_state = 88172645463325252ull;

/* uniform in [0, 1) */
static double lcg_u(void)
{
    lcg_state = lcg_state * 6364136223846793005ull + 1442695040888963407ull;
    return (double)(lcg_state >> 11) * (1.0 / 9007199254740992.0);
}

static void* xmalloc(size_t n)
{
    void* p = calloc(n > 0 ? n : 1, 1);
    if (!p) { fprintf(stderr, "out of memory\n"); exit(2); }
    return p;
}

static int check_finite(const char* what, const double* v, size_t n)
{
    for (size_t i = 0; i < n; ++i)
        if (!isfinite(v[i])) { fprintf(stderr, "%s: non-finite at %zu\n", what, i); return 1; }
    return 0;
}

/* one grid: assembly, both hierarchies under several parameter sets, the
 * block preconditioner variants, GMRES, ILU(0)/CPR and the network */
static int run_grid(int32_t nx, int32_t ny, int32_t nz, double api, int aniso)
{
    or_grid g = {nx, ny, nz, 1.0, 1.5, 2.0};
    or_props pr = {1000.0, 1e7, 350.0, 4.5e-10, -3e-4, 1e-3, 1500.0, 2093.4, 2500.0, 920.0, 9.80665, api};
    const int32_t n = nx * ny * nz;
    int bad = 0;
    double* K = xmalloc(sizeof(double) * 3 * (size_t)n);
    double* phi = xmalloc(sizeof(double) * (size_t)n);
    double* kap = xmalloc(sizeof(double) * (size_t)n);
    double* xp = xmalloc(sizeof(double) * 2 * (size_t)n);
    double* xk = xmalloc(sizeof(double) * 2 * (size_t)n);
    for (int32_t i = 0; i < 3 * n; ++i) K[i] = pow(10.0, -14.0 + 2.0 * lcg_u());
    for (int32_t i = 0; i < n; ++i) {
        phi[i] = 0.1 + 0.2 * lcg_u();
        kap[i] = 2.0;
        xp[2 * i] = 1e7; xp[2 * i + 1] = 350.0;
        xk[2 * i] = 1e7 + 1e5 * (lcg_u() - 0.5);
        xk[2 * i + 1] = 350.0 + 5.0 * (lcg_u() - 0.5);
    }
    or_well w[5] = {
        {0, 0, 1e-5, 450.0, 0.0, 0.0},
        {n - 1, 1, 1e-5, 0.0, 0.0, 0.0},
        {n / 2, 2, 150.0, 420.0, 0.0, 0.0},
        {n / 3, 3, 1e-3, 420.0, 1.05e7, 1e-12},
        {(2 * n) / 3, 4, 1e-3, 0.0, 0.95e7, 1e-12},
    };
    const int32_t kstride = aniso ? n : 0;
    const double dt = 86400.0;

    const int32_t nnz = or_stencil_nnz(&g);
    int32_t* rowptr = xmalloc(sizeof(int32_t) * ((size_t)n + 1));
    int32_t* col = xmalloc(sizeof(int32_t) * (size_t)nnz);
    if (or_stencil_pattern(&g, rowptr, col) != nnz) { fprintf(stderr, "stencil nnz\n"); return 1; }

    double* G = xmalloc(sizeof(double) * 2 * (size_t)n);
    or_residual(&g, &pr, K, kstride, phi, kap, 5, w, dt, xp, xk, G);
    bad |= check_finite("G", G, 2 * (size_t)n);
    double complex* xc = xmalloc(sizeof(double complex) * 2 * (size_t)n);
    double complex* Gc = xmalloc(sizeof(double complex) * 2 * (size_t)n);
    for (int32_t i = 0; i < 2 * n; ++i) xc[i] = xk[i] + (i == 3 ? 1e-20 * I : 0.0);
    or_residual_c(&g, &pr, K, kstride, phi, kap, 5, w, dt, xp, xc, Gc);

    double* blk[5];
    for (int b = 0; b < 5; ++b) blk[b] = xmalloc(sizeof(double) * (size_t)nnz);
    or_jacobian(&g, &pr, K, kstride, phi, kap, 5, w, dt, xp, xk, rowptr, col, blk[0], blk[1], blk[2], blk[3],
                blk[4]);
    for (int b = 0; b < 5; ++b) bad |= check_finite("J", blk[b], (size_t)nnz);
    or_jac J = {n, rowptr, col, blk[0], blk[1], blk[2], blk[3]};

    double* b = xmalloc(sizeof(double) * 2 * (size_t)n);
    double* z = xmalloc(sizeof(double) * 2 * (size_t)n);
    double* x = xmalloc(sizeof(double) * 2 * (size_t)n);
    for (int32_t i = 0; i < 2 * n; ++i) b[i] = -G[i];

    /* parameter sets: smoother, degree schedule, restriction, interpolation */
    const struct { int32_t smoother, deg, degc, interp, pmax, cmax; } sets[] = {
        {0, 3, 0, 0, 0, 16}, {1, 10, 1, 0, 0, 16}, {1, 3, 2, 1, 4, 16}, {1, 4, 0, 1, 0, 40}, {1, 10, 1, 0, 4, 4096},
    };
    for (size_t s = 0; s < sizeof(sets) / sizeof(sets[0]); ++s) {
        or_amg_params p = {0.25, 12345u, 25, sets[s].cmax, 1.0, 1, 1, 0, sets[s].smoother, sets[s].deg, 0.03, 0,
                           sets[s].degc, sets[s].interp, sets[s].pmax};
        or_amg *hpp = NULL, *hS = NULL;
        if (or_amg_setup(n, rowptr, col, blk[0], &p, &hpp) != 0) { fprintf(stderr, "setup pp\n"); return 1; }
        p.restriction = 1;
        if (or_amg_setup(n, rowptr, col, blk[4], &p, &hS) != 0) { fprintf(stderr, "setup S\n"); return 1; }
        for (int32_t l = 0; l < or_amg_nlev(hpp); ++l) {
            int32_t ln, la, lp;
            or_amg_level_sizes(hpp, l, &ln, &la, &lp);
            int32_t* arp = xmalloc(sizeof(int32_t) * ((size_t)ln + 1));
            int32_t* acol = xmalloc(sizeof(int32_t) * (size_t)la);
            double* aval = xmalloc(sizeof(double) * (size_t)la);
            int32_t* cf = xmalloc(sizeof(int32_t) * (size_t)ln);
            int32_t* prp = xmalloc(sizeof(int32_t) * ((size_t)ln + 1));
            int32_t* pcol = xmalloc(sizeof(int32_t) * (size_t)lp);
            double* pval = xmalloc(sizeof(double) * (size_t)lp);
            double* dinv = xmalloc(sizeof(double) * (size_t)ln);
            or_amg_level_copy(hpp, l, arp, acol, aval, cf, prp, pcol, pval, dinv);
            const int32_t rn = or_amg_level_R_nnz(hpp, l);
            if (l + 1 < or_amg_nlev(hpp)) {
                int32_t cn, ca, cp;
                or_amg_level_sizes(hpp, l + 1, &cn, &ca, &cp);
                int32_t* rrp = xmalloc(sizeof(int32_t) * ((size_t)cn + 1));
                int32_t* rcol = xmalloc(sizeof(int32_t) * (size_t)rn);
                double* rval = xmalloc(sizeof(double) * (size_t)rn);
                or_amg_level_R_copy(hpp, l, rrp, rcol, rval);
                free(rrp); free(rcol); free(rval);
            }
            free(arp); free(acol); free(aval); free(cf); free(prp); free(pcol); free(pval); free(dinv);
        }
        or_vcycle(hpp, b, x);
        bad |= check_finite("vcycle", x, (size_t)n);
        for (int32_t v = -1; v <= 2; ++v) {
            or_precond_apply(&J, hpp, hS, v, b, z);
            bad |= check_finite("precond", z, 2 * (size_t)n);
        }
        int32_t its;
        double rel;
        double* hist = xmalloc(sizeof(double) * 201);
        memset(x, 0, sizeof(double) * 2 * (size_t)n);
        or_gmres(&J, hpp, hS, 0, b, x, 1e-10, 30, 200, &its, &rel, hist);
        bad |= check_finite("gmres", x, 2 * (size_t)n);
        /* restarts: a short restart length */
        memset(x, 0, sizeof(double) * 2 * (size_t)n);
        or_gmres(&J, hpp, hS, 1, b, x, 1e-10, 3, 200, &its, &rel, hist);

        /* CPR: ILU(0) of the field-by-field Jacobian */
        int32_t* frp = xmalloc(sizeof(int32_t) * (2 * (size_t)n + 1));
        int32_t* fcol = xmalloc(sizeof(int32_t) * 4 * (size_t)nnz);
        double* fval = xmalloc(sizeof(double) * 4 * (size_t)nnz);
        double* flu = xmalloc(sizeof(double) * 4 * (size_t)nnz);
        or_jac_fieldwise(&J, frp, fcol, fval);
        if (or_ilu0(2 * n, frp, fcol, fval, flu) != 0) { fprintf(stderr, "ilu0\n"); return 1; }
        or_ilu0_solve(2 * n, frp, fcol, flu, b, z);
        or_ilu F = {2 * n, frp, fcol, flu};
        or_cpr_apply(&J, hpp, &F, b, z);
        memset(x, 0, sizeof(double) * 2 * (size_t)n);
        or_gmres_cpr(&J, hpp, &F, b, x, 1e-10, 30, 200, &its, &rel, hist);
        bad |= check_finite("gmres cpr", x, 2 * (size_t)n);
        free(frp); free(fcol); free(fval); free(flu); free(hist);
        or_amg_free(hpp);
        or_amg_free(hS);
    }

    /* learned smoother network: features, forward, loss and gradient */
    const int32_t np1 = 16 * 8 * 27, np2 = 16 * 27;
    double* W1 = xmalloc(sizeof(double) * (size_t)np1);
    double* b1 = xmalloc(sizeof(double) * 16);
    double* W2 = xmalloc(sizeof(double) * (size_t)np2);
    for (int32_t i = 0; i < np1; ++i) W1[i] = 0.1 * (lcg_u() - 0.5);
    for (int32_t i = 0; i < 16; ++i) b1[i] = 0.01 * (lcg_u() - 0.5);
    for (int32_t i = 0; i < np2; ++i) W2[i] = 0.1 * (lcg_u() - 0.5);
    double* f = xmalloc(sizeof(double) * 8 * (size_t)n);
    double* h = xmalloc(sizeof(double) * 16 * (size_t)n);
    double* out = xmalloc(sizeof(double) * (size_t)n);
    double* grad = xmalloc(sizeof(double) * (size_t)(np1 + 16 + np2 + 1));
    double* r = xmalloc(sizeof(double) * (size_t)n);
    for (int32_t i = 0; i < n; ++i) r[i] = lcg_u() - 0.5;
    or_cnn_features(&g, rowptr, col, blk[4], r, f);
    or_cnn_forward(&g, W1, b1, W2, 0.01, f, h, out);
    double loss = or_cnn_backward(&g, W1, b1, W2, 0.01, f, r, grad);
    bad |= check_finite("cnn", out, (size_t)n) | !isfinite(loss);

    free(W1); free(b1); free(W2); free(f); free(h); free(out); free(grad); free(r);
    for (int k = 0; k < 5; ++k) free(blk[k]);
    free(K); free(phi); free(kap); free(xp); free(xk); free(rowptr); free(col); free(G); free(xc); free(Gc);
    free(b); free(z); free(x);
    return bad;
}

int main(void)
{
    int bad = 0;
    bad |= run_grid(7, 5, 4, 0.0, 0);      /* 3-D, the workloads' fluid laws */
    bad |= run_grid(9, 6, 1, 10.0, 1);     /* 2-D slab, Bennison viscosity, diagonal tensor */
    bad |= run_grid(13, 1, 1, 0.0, 0);     /* a single row of cells */
    /* SplitMix64 over a few states */
    uint64_t acc = 0;
    for (uint64_t s = 0; s < 64; ++s) acc ^= or_splitmix64(s * 0x9e3779b97f4a7c15ull);
    if (bad) { fprintf(stderr, "sanitize: a result was not finite\n"); return 1; }
    printf("sanitize ok %016llx\n", (unsigned long long)acc);
    return 0;
}
