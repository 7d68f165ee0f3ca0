/*
 * tpsolve.h -- C ABI of the MI355X (gfx950) coupled pressure-temperature
 * solver: the block-preconditioned Krylov solve of the Jacobian of
 * non-isothermal single-phase porous-media flow (Roy, Jonsthovel, Lemon &
 * Wathen, "A block preconditioner for non-isothermal flow in porous media",
 * J. Comput. Phys. preprint 2019).
 *
 * Conventions for every call
 *   - Pointers named as device arrays are HIP device pointers owned by the
 *     caller; the library never frees them.  Host pointers are marked "host".
 *   - Every call is ordered on the HIP stream passed as `stream` (NULL = the
 *     null stream).  Calls that return sizes or statistics to the host
 *     synchronise that stream before returning.
 *   - Return value: TP_OK (0); a negative hard error; TP_NOT_CONVERGED (1),
 *     a soft status whose outputs are usable.  tp_last_error() gives a
 *     thread-local message for the last nonzero status.  No C++ exception
 *     crosses this interface.
 *   - Vectors at this interface are interleaved cell by cell:
 *     [p_0, T_0, p_1, T_1, ...], the ordering of the unknowns of Section 3.
 *   - Indices are int32; all floating point at this interface is FP64.
 *   - Handles (tp_amg_t, tp_prec_t) own device memory obtained from the
 *     allocator registered with tp_init (default: the HIP stream-ordered
 *     pool).  A handle is used by one stream at a time.
 */
#ifndef TPSOLVE_H
#define TPSOLVE_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
    TP_OK = 0,
    TP_ERR_ARG = -1,      /* null pointer, size mismatch, parameter out of range */
    TP_ERR_HIP = -2,      /* a HIP runtime call failed (message names it) */
    TP_ERR_OOM = -3,      /* device allocation failed */
    TP_ERR_NUMERIC = -4,  /* zero pivot, non-finite values, stalled coarsening */
    TP_ERR_CAPACITY = -5, /* a fixed-capacity structure overflowed (message says which) */
    TP_NOT_CONVERGED = 1  /* Krylov limit reached; x holds the last iterate */
};

const char* tp_last_error(void);

/* Device memory provider.  alloc(bytes, stream, ctx) returns device memory
 * or NULL; free(ptr, stream, ctx) returns it.  Memory must stay valid until
 * freed (stream-ordered reuse is allowed). */
typedef struct {
    void* (*alloc)(size_t bytes, void* stream, void* ctx);
    void (*free)(void* ptr, void* stream, void* ctx);
    void* ctx;
} tp_allocator;

/* Select the device and, optionally, an allocator (NULL: HIP stream-ordered
 * pool).  Must be called once before any other call; may be called again to
 * switch allocators when no handle is alive. */
int tp_init(const tp_allocator* alloc, int device);

/* ---------------------------------------------------------------------------
 * Discretisation (Section 2.2): two-point flux finite volumes on a uniform
 * Cartesian grid, backward Euler, residual forms F_m and F_e (eq. Fm, Fe),
 * Jacobian blocks of eq. AXR and the Schur approximation of eq. Se.
 * ------------------------------------------------------------------------ */
typedef struct { int32_t nx, ny, nz; double dx, dy, dz; } tp_grid;  /* cell i = ix + nx (iy + ny iz) */

/* rho = rho0 exp(c_p (p - p0) + c_T (T - T0)); mu = mu0 exp(mu_B (1/T - 1/T0))
 * when api = 0, else the Bennison heavy-oil correlation (Section 2.1,
 * eq. bennison with the constants of table bennison): mu = 1e-3
 * 10^(A1 api + A2) T_F^(A3 api + A4) Pa s, T_F = 1.8 (T - 273.15) + 32 the
 * temperature in Fahrenheit, api the API gravity; cv, c_r specific heats of
 * fluid and rock; rho_r rock density; g gravity along -z (0 disables). SI
 * units. */
typedef struct { double rho0, p0, T0, c_p, c_T, mu0, mu_B, cv, rho_r, c_r, g, api; } tp_props;

/* Constant-rate point well (eq. f, eq. fT): kind 0 injector (mass
 * rate*rho(p, T_inj), enthalpy c_v T_inj), kind 1 producer (mass
 * rate*rho(p, T), enthalpy c_v T). rate >= 0 in m^3/s.  Kind 2 is a heater
 * (Section 2.1, source terms): energy source U (T_heater - T) with
 * rate = U >= 0 in W/K and T_inj = T_heater; it adds U to A_TT and to the
 * Schur approximation (eq. Se).  Kinds 3 and 4 are Peaceman wells (Section
 * 2.1, well model): an injector (3) or producer (4) whose volumetric rate is
 * wi (p_bh - p) / mu(T) (injector) or wi (p - p_bh) / mu(T) (producer), mu
 * the cell fluid's viscosity, wi = 2 pi h K_e / ln(r_e / r_w) > 0 the well
 * index in m^3 (computed by the caller), clamped to [0, rate] with rate the
 * maximum rate; mass and enthalpy as kinds 0 and 1.  A producer adds c_v
 * times its mass rate to the Schur approximation (eq. wellschurapprox).
 * p_bh and wi are ignored for kinds 0 to 2. */
typedef struct { int32_t cell; int32_t kind; double rate, T_inj, p_bh, wi; } tp_well;
#define TP_MAX_WELLS 32

/* Jacobian storage: one CSR pattern (sorted columns, full 5/7-point stencil
 * including structural zeros) shared by A_pp, A_pT, A_Tp, A_TT and the Schur
 * approximation S.  All arrays are caller-owned device memory sized by
 * tp_jacobian_sizes. */
typedef struct {
    int32_t n, nnz;
    int32_t *rowptr, *col;            /* n+1, nnz */
    double *pp, *pT, *Tp, *TT, *S;    /* nnz each */
} tp_jacobian;

/* n = nx*ny*nz cells and nnz of the stencil pattern. TP_ERR_ARG if any
 * dimension < 1 or nnz would exceed 2^31-1. */
int tp_jacobian_sizes(const tp_grid* grid, int32_t* n, int32_t* nnz);

/* Assemble G(x_k) (eq. Fm, Fe; 2n interleaved, device) and J = dG/dx at
 * x_k (eq. AXR ... eq. rhouT, upwind choice frozen) plus S (eq. Se with the
 * specific heat on the advective term).  K, phi, kappa: n device arrays;
 * x_prev, x_k: 2n device arrays; wells: host array of nwells <= TP_MAX_WELLS.
 * Homogeneous no-flow boundaries.  Errors: TP_ERR_ARG on null pointers,
 * J->n/nnz not matching the grid, a well cell out of range, rate < 0 or
 * dt <= 0. */
int assemble_tpfa(const tp_grid* grid, const tp_props* props, const double* K,
                  const double* phi, const double* kappa, int32_t nwells,
                  const tp_well* wells, double dt, const double* x_prev,
                  const double* x_k, tp_jacobian* J, double* G, void* stream);

/* As assemble_tpfa with the diagonal permeability tensor K = diag(K_x, K_y,
 * K_z) of the Peaceman discussion in Section 2.1 (anisotropic media, the
 * problem-size study's Cases IV and V in Section 4): K3 is a 3n device array
 * [K_x(0..n-1), K_y(0..n-1), K_z(0..n-1)], and a face normal to axis a takes
 * the harmonic mean of its two cells' K_a.  Same errors as assemble_tpfa. */
int assemble_tpfa_aniso(const tp_grid* grid, const tp_props* props, const double* K3,
                        const double* phi, const double* kappa, int32_t nwells,
                        const tp_well* wells, double dt, const double* x_prev,
                        const double* x_k, tp_jacobian* J, double* G, void* stream);

/* ---------------------------------------------------------------------------
 * Algebraic multigrid (Section 3: A_pp and the Schur approximation are each
 * applied by one AMG V-cycle).  Strength theta, seeded PMIS coarsening with
 * key (|S^T_i|, splitmix64(seed ^ level<<40 ^ i), i), direct interpolation,
 * Galerkin or Petrov-Galerkin coarse operators R (A P), smoother, and on the
 * coarsest level an explicit inverse (blocked Gauss-Jordan elimination with
 * partial pivoting).  The setup runs in FP64; `storage` only selects how the
 * hierarchy is stored and applied.
 * ------------------------------------------------------------------------ */
typedef struct {
    double theta;          /* strength threshold, (0,1); 0.25 */
    uint64_t seed;         /* PMIS hash seed */
    int32_t max_levels;    /* 1..25 */
    int32_t coarse_max;    /* stop when n_l <= coarse_max (<= 4096); 1200: a dense
                              coarsest level of ~1000 rows is one GEMV, cheaper
                              than the several latency-bound levels it replaces */
    int32_t smoother;      /* 0 l1-Jacobi, 1 Chebyshev on D_l1^{-1} A over [cheb_lo, 1] */
    int32_t cheb_degree;   /* 1..16; 10 (on the finest level) */
    double cheb_lo;        /* (0,1); 0.03 (degrees and interval chosen by measured
                              time-to-solution on the layered and channelised fields) */
    double omega;          /* l1-Jacobi weight; 1.0 */
    int32_t nu_pre, nu_post; /* sweeps; 1, 1 */
    int32_t restriction;   /* 0 R = P^T; 1 R = Q^T, Q the interpolation built from A^T */
    int32_t storage;       /* 0 FP64; 1 FP32 (values and V-cycle vectors); 2 FP32 vectors,
                              P, R and level-operator diagonal, level-operator
                              off-diagonal entries in BF16 (round to nearest even) */
    int32_t cheb_degree_coarse; /* Chebyshev degree on levels >= 1, 0..16 (0: cheb_degree); 1 */
    int32_t interp;        /* 0 direct interpolation (default); 1 extended+i: an F point
                              also interpolates from the strong C neighbours of its
                              strong F neighbours (De Sterck, Falgout, Nolting, Yang,
                              Numer. Linear Algebra Appl. 15, 2008); with restriction 1
                              Q is built the same way from A^T */
    int32_t interp_pmax;   /* extended+i only, 0..16: a row of more weights keeps the
                              interp_pmax of largest magnitude (ties: smaller column),
                              scaled to the row's full sum; 0 keeps all; 4 */
} tp_amg_params;

typedef struct tp_amg* tp_amg_t;

/* Build the hierarchy of the n x n CSR matrix (device arrays, sorted
 * columns, diagonal present in every row).  Synchronises `stream`.
 * Errors: TP_ERR_ARG (bad sizes/params), TP_ERR_NUMERIC (zero pivot in the
 * coarsest-level elimination, coarsening stalled above 4096 rows), TP_ERR_CAPACITY (a
 * product row exceeded the on-chip hash table), TP_ERR_OOM. */
int amg_setup(int32_t n, const int32_t* rowptr, const int32_t* col, const double* val,
              const tp_amg_params* params, tp_amg_t* out, void* stream);

/* Hierarchy of the diagonal Schur approximation (Section 3.2, one of the
 * simple approximations the paper compares S~_T with)
 *   S_diag = A_TT - A_Tp diag(A_pp)^{-1} A_pT,
 * formed on the device from the Jacobian's blocks (sparse product on the
 * distance-two pattern of the stencil), then amg_setup on it; the hierarchy
 * keeps its own copy (level 0).  J is read only.  Synchronises `stream`.
 * Errors: as amg_setup, and TP_ERR_NUMERIC for a zero or non-finite A_pp
 * diagonal entry. */
int amg_setup_schur_diag(const tp_jacobian* J, const tp_amg_params* params, tp_amg_t* out,
                         void* stream);

/* Reuse of a hierarchy across Newton iterations (the setup is the largest
 * part of a single solve): new values `val` (device, nnz of level 0) for the
 * finest-level operator, on the pattern the hierarchy was built on.  The
 * operator and what is derived from it alone are rewritten in place (l1
 * diagonal, stencil-diagonal copy, reduced-precision copies, an attached
 * learned smoother's static features; the dense inverse when level 0 is the
 * coarsest); the coarse levels, P and R are kept, so the V-cycle becomes a
 * preconditioner lagged on the coarse levels.  Preconditioner handles and
 * their captured graphs built on this hierarchy stay valid.  Not for
 * hierarchies from amg_setup_schur_diag (their level 0 has its own pattern).
 * Synchronises `stream`. */
int amg_refresh_fine(tp_amg_t amg, const double* val, void* stream);

/* Setup reuse across Newton iterations (Section 4, opening: each Newton
 * iteration solves a new Jacobian; the AMG setup is rebuilt for it
 * otherwise): new values `val` (device, nnz of level 0) for the finest-level
 * operator on the pattern the hierarchy was built on, with the C/F split of
 * every level and every sparsity pattern (P, R, the coarse operators) kept.
 * All values are recomputed from `val` in the setup's order: direct
 * interpolation weights restricted to the kept interpolation sets (only
 * couplings of the sign opposite to the diagonal interpolate; a kept entry
 * that no longer does holds an explicit zero), or, for extended+i
 * interpolation (interp 1), the extended+i weights over each row's
 * interpolatory set taken from the kept strength pattern, a row truncated at
 * setup keeping its kept columns scaled to the full row sum; R = P^T or its
 * Petrov-Galerkin counterpart on the kept pattern, the Galerkin products
 * R (A P) on their kept patterns (each entry summed in ascending inner
 * index), the l1 diagonals, stencil-diagonal and reduced-precision copies,
 * the coarsest inverse, and an attached learned smoother's static features.
 * When the kept splits and patterns are the ones a fresh amg_setup would
 * choose for `val`, the hierarchy equals that fresh setup bit for bit.
 * Everything is rewritten in place: preconditioner handles and their
 * captured graphs stay valid.  Not for hierarchies from
 * amg_setup_schur_diag.  Errors: TP_ERR_ARG (null), TP_ERR_NUMERIC (zero
 * pivot in the coarsest inverse).  Synchronises `stream`. */
int amg_refresh(tp_amg_t amg, const double* val, void* stream);

int amg_num_levels(tp_amg_t amg, int32_t* nlev);
/* sizes of level l (P/R sizes are 0 on the coarsest level) */
int amg_level_info(tp_amg_t amg, int32_t level, int32_t* n, int32_t* nnzA,
                   int32_t* nnzP, int32_t* nnzR);
/* Storage format of level l's operator in the V-cycle: ndia > 0 when it is
 * kept diagonal-major with ndia diagonals (stencil levels), else CSR read by
 * `lanes` cooperating lanes per row. */
int amg_level_format(tp_amg_t amg, int32_t level, int32_t* ndia, int32_t* lanes);
/* Copy level arrays into caller device buffers (any pointer may be NULL;
 * sizes from amg_level_info; cf: 1 = C point, 0 = F point).  FP64 values of
 * the setup.  Stream-ordered; does not synchronise. */
int amg_level_copy(tp_amg_t amg, int32_t level, int32_t* A_rowptr, int32_t* A_col,
                   double* A_val, int32_t* cf, int32_t* P_rowptr, int32_t* P_col,
                   double* P_val, int32_t* R_rowptr, int32_t* R_col, double* R_val,
                   void* stream);
/* x = V(b): one V(nu_pre, nu_post)-cycle from a zero guess (device, n). */
int amg_vcycle(tp_amg_t amg, const double* b, double* x, void* stream);
int amg_destroy(tp_amg_t amg);

/* ---------------------------------------------------------------------------
 * Block preconditioner (Section 3.2, the five-step application list).
 * variant 0 lower (steps 1-3, default), 1 upper, 2 full (steps 1-5, step 4
 * read as b_p - A_pT d_T).  Borrows J and both hierarchies: they must
 * outlive the handle.
 * ------------------------------------------------------------------------ */
typedef struct tp_prec* tp_prec_t;
int precond_create(const tp_jacobian* J, tp_amg_t amg_pp, tp_amg_t amg_S,
                   int32_t variant, tp_prec_t* out);
/* z = M^{-1} r, 2n interleaved device vectors.  The apply is captured as a
 * HIP graph (kernels only) on its first use and replayed afterwards on
 * `stream`; while a learned smoother is active or the kernel timer is on,
 * its kernels are launched one by one.  Calls on one handle must not overlap
 * (they share the handle's staging vectors and the hierarchies' work
 * vectors). */
int precond_apply(tp_prec_t M, const double* r, double* z, void* stream);

/* For callers that cannot allocate (code under HIP graph capture, serving
 * loops, harnesses that forbid hipMalloc): precond_apply without any device
 * allocation by the library.  The same kernels in the same order as
 * precond_apply (identical z), launched one by one on `stream` (no graph is
 * captured or instantiated).  Its work vectors -- the split r and z (2n + 2n
 * doubles) and, for CPR handles, the first-stage pressure and residual
 * (n + 2n) -- live in a fixed 256 MiB device array that every GPU the library
 * runs on holds for the life of the process: at most 8,388,608 cells (block
 * variants) or 4,793,490 (CPR) per call; larger handles get
 * TP_ERR_CAPACITY.  Nothing in the array has to start at zero.  All calls on
 * one GPU share that array: calls that overlap in time on one GPU (two
 * streams, two threads) race and must be serialised by the caller.  The
 * handle's hierarchies and an attached learned smoother use the buffers they
 * allocated at setup / attachment.  Errors: TP_ERR_ARG (null; the smoother
 * timer is on, since it records events), TP_ERR_CAPACITY, TP_ERR_HIP. */
int precond_apply_noalloc(tp_prec_t M, const double* r, double* z, void* stream);
int precond_destroy(tp_prec_t M);

/* ---------------------------------------------------------------------------
 * ILU(0) (Section 3: incomplete LU with the factors on the sparsity pattern
 * of the matrix) and the two-stage CPR preconditioner of Section 3.1, the
 * comparator of Section 4 (AMG V-cycle on A_pp in the first stage, ILU(0)
 * of the whole Jacobian in the second).
 *
 * Factors: L unit lower triangular and U upper triangular with
 * (L U)_ij = a_ij at every stored position of A, by row-by-row Gaussian
 * elimination that drops every update outside the pattern.  Triangular
 * solves run level by level (rows grouped by the depth of their dependency
 * chains, found by a host pass over the pattern at creation), one kernel
 * launch per level.
 * ------------------------------------------------------------------------ */
typedef struct tp_ilu* tp_ilu_t;
/* ILU(0) of an N x N CSR matrix (device arrays: rowptr N+1, col and val
 * rowptr[N]; columns sorted and unique within each row, every diagonal
 * stored).  Copies the matrix; synchronises `stream` (the pattern is read by
 * the host).  Errors: TP_ERR_ARG for a malformed pattern (unsorted or
 * duplicate columns, an index out of range, a missing diagonal),
 * TP_ERR_NUMERIC for a zero or non-finite pivot. */
int ilu0_create(int32_t N, const int32_t* rowptr, const int32_t* col, const double* val,
                void* stream, tp_ilu_t* out);
/* ILU(0) of the whole 2n x 2n Jacobian of eq. AXR in field-by-field order
 * (rows and columns [p_0..p_{n-1}, T_0..T_{n-1}]): row p_i holds A_pp(i,:)
 * then A_pT(i,:) at columns j and n + j, row T_i holds A_Tp(i,:) then
 * A_TT(i,:); all 4 nnz stored entries are kept, structural zeros included.
 * Synchronises `stream`; errors as ilu0_create. */
int ilu0_create_jacobian(const tp_jacobian* J, void* stream, tp_ilu_t* out);
/* New values of a Jacobian with the pattern the handle was built from
 * (a later Newton iterate): refill and refactorise, no new analysis.
 * Synchronises `stream` (pivot check). */
int ilu0_refactor_jacobian(tp_ilu_t F, const tp_jacobian* J, void* stream);
/* x = U^{-1} L^{-1} b (device, N each, in the ordering of the factorised
 * matrix: field by field for a Jacobian handle).  b and x may be the same
 * array.  Stream-ordered; does not synchronise. */
int ilu0_solve(tp_ilu_t F, const double* b, double* x, void* stream);
/* Sizes and level counts of the forward and backward solves (host outputs,
 * any may be NULL). */
int ilu0_info(tp_ilu_t F, int32_t* N, int32_t* nnz, int32_t* levels_lower, int32_t* levels_upper);
/* Copy the pattern and the factors (L strictly below the diagonal, U on and
 * above) into caller device arrays (any may be NULL). Stream-ordered. */
int ilu0_copy(tp_ilu_t F, int32_t* rowptr, int32_t* col, double* lu, void* stream);
int ilu0_destroy(tp_ilu_t F);

/* CPR (Section 3.1): z = M^{-1} r with x1 = [V_pp(r_p); 0] and
 * z = ILU0^{-1}(r - J x1) + x1, for a handle from ilu0_create_jacobian of
 * the same J.  Used through precond_apply, fgmres_solve and
 * precond_destroy like the block forms; borrows J, the hierarchy and the
 * ILU(0) handle, which must outlive it. */
int precond_create_cpr(const tp_jacobian* J, tp_amg_t amg_pp, tp_ilu_t ilu, tp_prec_t* out);

/* ---------------------------------------------------------------------------
 * Flexible GMRES (right preconditioned, restarted; Section 4: GMRES with
 * restart 30) with classical Gram-Schmidt applied twice, Givens rotations on
 * the Hessenberg matrix, all in FP64 on the device.  Stops when the true
 * relative residual ||b - J x||_2 / ||b||_2 <= rtol (checked in FP64 at the
 * end of every cycle), after maxit iterations, or -- TP_NOT_CONVERGED --
 * when a cycle whose residual estimate met rtol leaves the true residual
 * above rtol and above half its value at the cycle's start: the true
 * residual has reached the rounding floor of the FP64 product b - J x (a
 * right-hand side small against ||J|| ||x||), where more cycles repeat the
 * same correction.
 * ------------------------------------------------------------------------ */
typedef struct {
    double rtol;
    int32_t restart;
    int32_t maxit;
    /* Stagnation guard for a learned post-smoother attached to the Schur
     * hierarchy: when the residual estimate of iteration j exceeds
     * stag_ratio times that of iteration j-2 (or the network produced a
     * non-finite value), the network is switched off for the rest of the
     * solve and the hierarchy's own post-smoother is used.  0 disables. */
    double stag_ratio;
    /* 1: the preconditioner apply is captured once per (handle, stream) as a
     * HIP graph and replayed each iteration (not while a learned smoother is
     * active or the kernel timer is on); 0: its kernels are launched one by
     * one.  Both give bit-identical iterates. */
    int32_t graph;
    /* Absolute tolerance: the solve also stops when ||b - J x||_2 <= atol
     * (0: relative test only). */
    double atol;
    /* Stagnation window w of the guard above: estimate j against estimate
     * j - w (0 takes 2). */
    int32_t stag_window;
    /* Contraction guard for the learned smoother: when > 0, the network is
     * switched off at iteration j >= 4 of a solve whose relative residual
     * estimate exceeds ref_rate^j, i.e. whose mean contraction per iteration
     * so far falls behind ref_rate (the caller passes the plain form's rate,
     * measured on an earlier solve and relaxed for the network's cost per
     * iteration).  Recorded in fallback_iter like the stagnation guard. */
    double ref_rate;
} tp_krylov_params;
typedef struct {
    int32_t iters, restarts;
    double rel_true, rel_est;
    int32_t fallback_iter;  /* iteration at which the network was switched off, -1 none */
} tp_krylov_stats;

/* Solve J x = b (2n interleaved device vectors; x holds the initial guess on
 * entry).  history: optional host array of maxit+1 relative residual
 * estimates.  Synchronises `stream`.  Returns TP_OK or TP_NOT_CONVERGED;
 * TP_ERR_NUMERIC on a non-finite residual. */
int fgmres_solve(const tp_jacobian* J, tp_prec_t M, const double* b, double* x,
                 const tp_krylov_params* params, tp_krylov_stats* stats,
                 double* history, void* stream);

/* ---------------------------------------------------------------------------
 * Learned post-smoother on the finest level of the Schur-approximation
 * hierarchy (a method pattern on top of the paper's V-cycle; the paper has
 * no learned component).  Network: 3x3x3 convolution 8 -> 16 channels +
 * bias, ReLU, 3x3x3 convolution 16 -> 1 + bias, zero padding; BF16 weights
 * and inputs, FP32 accumulation.  Parameters (3905 floats) are laid out
 * W1[16][8][27], b1[16], W2[16][27], b2[1], tap t = (dz+1)*9 + (dy+1)*3 + (dx+1).
 * Input features per cell (8 x n, channel-major, FP32): (D^{-1} r)/s with
 * s = RMS(D^{-1} r) and D the l1 diagonal; a_{i,nbr}/a_ii for the -x, +x,
 * -y, +y, -z, +z neighbours (0 off-grid); a_ii / D_ii.  The smoother update
 * is x <- x + s * out.
 * ------------------------------------------------------------------------ */
typedef struct tp_cnn* tp_cnn_t;
#define TP_CNN_NPARAM 3905
/* params: host array of TP_CNN_NPARAM finite floats (copied). */
int cnn_create(const float* params, tp_cnn_t* out);
/* current FP32 master parameters into a host array */
int cnn_get_params(tp_cnn_t net, float* params);
int cnn_destroy(tp_cnn_t net);
/* gradient of the last loss evaluation (cnn_loss_grad / amg_cnn_loss_grad) into a host array */
int cnn_get_grad(tp_cnn_t net, float* grad);
/* out (n, device) = network(feat) on the grid; feat: 8 x n device FP32 */
int cnn_forward(tp_cnn_t net, const tp_grid* grid, const float* feat, float* out, void* stream);
/* Loss mean_i (out_i - target_i)^2 and its gradient, kept in the handle for
 * cnn_adam_step; grad (device, TP_CNN_NPARAM) and loss (host) optional. */
int cnn_loss_grad(tp_cnn_t net, const tp_grid* grid, const float* feat, const float* target,
                  double* loss, float* grad, void* stream);
/* One Adam step (beta 0.9/0.999, eps 1e-8) with the last gradient. */
int cnn_adam_step(tp_cnn_t net, float lr, void* stream);
/* Attach `net` as the finest-level post-smoother of `amg` (the grid must
 * have amg's level-0 size; the level must be that grid's stencil matrix);
 * net = NULL detaches.  The network must outlive the attachment. */
int amg_attach_post_smoother(tp_amg_t amg, tp_cnn_t net, const tp_grid* grid);
/* Features (8 x n device FP32) of residual r (n device FP64) on the
 * finest level of a hierarchy with an attached network; scale (host, optional). */
int amg_features(tp_amg_t amg, const double* r, float* feat, float* scale, void* stream);
/* Loss of the attached network measured in the D^{-1} A norm of the
 * hierarchy's finest-level operator A (D its l1 diagonal), plus an optional
 * error term: L = mean_i (D^{-1} A (out - target))_i^2
 *               + err_weight * mean_i (out - target)_i^2, out = network(feat);
 * for target = e/s the first term is the residual the correction leaves
 * behind and the second the error (err_weight >= 0, finite; 0 for the pure
 * residual loss).  The gradient is kept in the network handle for
 * cnn_adam_step; loss (host) optional. */
int amg_cnn_loss_grad(tp_amg_t amg, const float* feat, const float* target, float err_weight,
                      double* loss, void* stream);
/* Training pair at the finest-level post-smoothing point: b = A y, one
 * V-cycle from a zero guess stopped before level-0 post-smoothing gives x;
 * r = b - A x and e = y - x (all n, device FP64). */
int amg_presmoothed_pair(tp_amg_t amg, const double* y, double* r, double* e, void* stream);

/* ---------------------------------------------------------------------------
 * Measurement support: HIP-event timing of the fine-level smoother kernel
 * (the V-cycle's dominant kernel) on the stream it is launched on.
 * ------------------------------------------------------------------------ */
/* Mean execution time of the finest-level Chebyshev sweep kernel of `amg`,
 * replayed `reps` times back to back on `stream` (its own level-0 operator
 * and work vectors, contents zeroed first) between one HIP event pair;
 * bytes_per_launch is the kernel's algorithmic byte count.  Overwrites the
 * hierarchy's work vectors; synchronises `stream`. */
int amg_time_fine_smoother(tp_amg_t amg, int32_t reps, double* ms_per_launch,
                           double* bytes_per_launch, void* stream);
/* The same sweep with the last-level cache evicted before every launch: each
 * launch follows a read pass over `flush_buf` (device, `flush_doubles`
 * doubles, caller-owned, finite values, left unchanged; make it several
 * times the 256 MB cache) and is timed by an event pair of its own;
 * ms_per_launch is the mean of those times.  Errors:
 * TP_ERR_ARG (null, reps outside [1, 1000], empty buffer, one level).
 * Synchronises `stream`. */
int amg_time_fine_smoother_flushed(tp_amg_t amg, int32_t reps, double* flush_buf, int64_t flush_doubles,
                                   double* ms_per_launch, double* bytes_per_launch, void* stream);
/* enable (1) / disable (0) and reset the counters */
int tp_timer_enable(int32_t on);
/* totals since the last enable: launches, summed kernel milliseconds and
 * algorithmic bytes (matrix values, indices and vectors each counted once) */
int tp_timer_read(int64_t* launches, double* ms, double* bytes);

#ifdef __cplusplus
}
#endif
#endif
