/*
 * physics.c -- oracle TPFA residual, Jacobian and Schur approximation.
 *
 * TEST INFRASTRUCTURE ONLY (see tp_oracle.h).  Plain FP64, one cell at a time.
 *
 * Follows Section 2.2 of the paper: DG0 = two-point flux finite volumes on a
 * uniform Cartesian grid, harmonic-mean transmissibilities, arithmetic-mean
 * face density, upwinded mobility rho/mu and upwinded temperature (Section
 * 2.2.2), point wells through the cell-indicator delta (Section 2.2.2), and
 * the backward-Euler forms F_m and F_e (eq. Fm, eq. Fe).  Readings taken
 * where the text is silent or garbled:
 *   - the advective energy flux carries the specific heat c_v (as in the
 *     strong form of Section 2.1.2); eq. Fe and eq. Se print it without;
 *   - the upwind side is decided on the physical potential difference
 *     dPhi = (p_i - p_j) + rho_bar g (z_i - z_j) of the face oriented from
 *     the lower to the higher cell index; dPhi >= 0 picks the lower cell;
 *   - homogeneous Neumann (no-flow) on every boundary face.
 */
#include "tp_oracle.h"
#include <math.h>
#include <stdlib.h>
#include <string.h>

/* neighbour offsets in ascending column order: -z, -y, -x, (self), +x, +y, +z */
static int nb_cell(const or_grid* g, int32_t i, int d, int* axis)
{
    int32_t ix = i % g->nx, iy = (i / g->nx) % g->ny, iz = i / (g->nx * g->ny);
    switch (d) {
    case 0: *axis = 2; return iz > 0 ? i - g->nx * g->ny : -1;
    case 1: *axis = 1; return iy > 0 ? i - g->nx : -1;
    case 2: *axis = 0; return ix > 0 ? i - 1 : -1;
    case 3: *axis = 0; return ix < g->nx - 1 ? i + 1 : -1;
    case 4: *axis = 1; return iy < g->ny - 1 ? i + g->nx : -1;
    default: *axis = 2; return iz < g->nz - 1 ? i + g->nx * g->ny : -1;
    }
}

int32_t or_stencil_nnz(const or_grid* g)
{
    int64_t nx = g->nx, ny = g->ny, nz = g->nz;
    int64_t n = nx * ny * nz;
    int64_t faces = (nx - 1) * ny * nz + nx * (ny - 1) * nz + nx * ny * (nz - 1);
    return (int32_t)(n + 2 * faces);
}

int32_t or_stencil_pattern(const or_grid* g, int32_t* rowptr, int32_t* col)
{
    int32_t n = g->nx * g->ny * g->nz, k = 0, ax;
    rowptr[0] = 0;
    for (int32_t i = 0; i < n; ++i) {
        for (int d = 0; d < 6; ++d) {
            if (d == 3) col[k++] = i;
            int j = nb_cell(g, i, d, &ax);
            if (j >= 0) col[k++] = j;
        }
        rowptr[i + 1] = k;
    }
    return k;
}

/* area / centre distance of a face normal to an axis */
static double area_over_dist(const or_grid* g, int axis)
{
    if (axis == 0) return g->dy * g->dz / g->dx;
    if (axis == 1) return g->dx * g->dz / g->dy;
    return g->dx * g->dy / g->dz;
}

static double harmonic(double a, double b)
{
    double s = a + b;
    return s > 0.0 ? 2.0 * a * b / s : 0.0;
}

/* cell-centre height (z up) */
static double zc(const or_grid* g, int32_t i) { return ((double)(i / (g->nx * g->ny)) + 0.5) * g->dz; }

/* ---- residual on complex states ----------------------------------------- */

static double complex rho_c(const or_props* pr, double complex p, double complex T)
{
    return pr->rho0 * cexp(pr->c_p * (p - pr->p0) + pr->c_T * (T - pr->T0));
}

/* Bennison's heavy-oil correlation (Section 2.1, eq. bennison; constants of
 * table bennison): viscosity in centipoise 10^(A1 api + A2) T_F^(A3 api + A4)
 * with T_F the temperature in degrees Fahrenheit; returned in Pa s. */
static const double BEN_A1 = -0.8021, BEN_A2 = 23.8765, BEN_A3 = 0.31458, BEN_A4 = -9.21592;

static double complex mu_c(const or_props* pr, double complex T)
{
    if (pr->api > 0.0) {
        double complex TF = (T - 273.15) * 9.0 / 5.0 + 32.0;
        double centipoise_scale = pow(10.0, BEN_A1 * pr->api + BEN_A2);
        return 1e-3 * centipoise_scale * cpow(TF, BEN_A3 * pr->api + BEN_A4);
    }
    return pr->mu0 * cexp(pr->mu_B * (1.0 / T - 1.0 / pr->T0));
}

/* mass flux from lo to hi across one face and the upwinded temperature */
static void face_flux_c(const or_grid* g, const or_props* pr, const double* K,
                        int32_t kstride, const double* kappa, const double complex* x, int32_t lo,
                        int32_t hi, int axis, double complex* F, double complex* Tup,
                        double* Th)
{
    double ad = area_over_dist(g, axis);
    const double* Ka = K + (size_t)axis * (size_t)kstride;  /* K's diagonal entry along this axis */
    double Ups = ad * harmonic(Ka[lo], Ka[hi]);
    *Th = ad * harmonic(kappa[lo], kappa[hi]);
    double complex pl = x[2 * lo], Tl = x[2 * lo + 1], ph = x[2 * hi], Thh = x[2 * hi + 1];
    double complex rl = rho_c(pr, pl, Tl), rh = rho_c(pr, ph, Thh);
    double complex dphi = (pl - ph) + 0.5 * (rl + rh) * pr->g * (zc(g, lo) - zc(g, hi));
    if (creal(dphi) >= 0.0) {
        *F = Ups * (rl / mu_c(pr, Tl)) * dphi;
        *Tup = Tl;
    } else {
        *F = Ups * (rh / mu_c(pr, Thh)) * dphi;
        *Tup = Thh;
    }
}

void or_residual_c(const or_grid* g, const or_props* pr, const double* K,
                   int32_t kstride, const double* phi, const double* kappa, int32_t nw,
                   const or_well* w, double dt, const double* x_prev,
                   const double complex* x, double complex* G)
{
    int32_t n = g->nx * g->ny * g->nz, ax;
    double V = g->dx * g->dy * g->dz;
    for (int32_t i = 0; i < n; ++i) {
        double complex p = x[2 * i], T = x[2 * i + 1];
        double complex r = rho_c(pr, p, T);
        double rn = creal(rho_c(pr, x_prev[2 * i], x_prev[2 * i + 1]));
        double Tn = x_prev[2 * i + 1];
        /* accumulation (eq. Fm, eq. Fe) */
        double complex Rm = V * phi[i] * (r - rn) / dt;
        double complex Re = V * (phi[i] * pr->cv * (r * T - rn * Tn)
                                 + (1.0 - phi[i]) * pr->rho_r * pr->c_r * (T - Tn)) / dt;
        /* interior faces: flux out of cell i */
        for (int d = 0; d < 6; ++d) {
            int32_t j = nb_cell(g, i, d, &ax);
            if (j < 0) continue;
            int32_t lo = i < j ? i : j, hi = i < j ? j : i;
            double complex F, Tup;
            double Th;
            face_flux_c(g, pr, K, kstride, kappa, x, lo, hi, ax, &F, &Tup, &Th);
            double complex Fout = (i == lo) ? F : -F;
            Rm += Fout;
            Re += pr->cv * Tup * Fout + Th * (T - x[2 * j + 1]);
        }
        /* wells: cell-indicator delta times the cell volume (eq. f, eq. fT) */
        for (int32_t k = 0; k < nw; ++k) {
            if (w[k].cell != i) continue;
            if (w[k].kind == 0) {
                double complex Qm = w[k].rate * rho_c(pr, p, w[k].T_inj);
                Rm -= Qm;
                Re -= pr->cv * w[k].T_inj * Qm;
            } else if (w[k].kind == 1) {
                double complex Qm = -w[k].rate * r;
                Rm -= Qm;
                Re -= pr->cv * T * Qm;
            } else if (w[k].kind == 2) {
                /* heater (Section 2.1, source terms): f_T = U (T_heater - T) */
                Re -= w[k].rate * (w[k].T_inj - T);
            } else {
                /* Peaceman well (Section 2.1): volumetric rate from the pressure
                 * difference to the bottom hole, the cell fluid's viscosity, and the
                 * limits 0 (no backflow) and the maximum rate */
                double complex dpw = w[k].kind == 3 ? w[k].p_bh - p : p - w[k].p_bh;
                double complex qv = w[k].wi * dpw / mu_c(pr, T);
                if (creal(qv) >= w[k].rate) qv = w[k].rate;
                if (creal(qv) <= 0.0) qv = 0.0;
                double complex Qm = w[k].kind == 3 ? qv * rho_c(pr, p, w[k].T_inj) : -qv * r;
                Rm -= Qm;
                Re -= pr->cv * (w[k].kind == 3 ? w[k].T_inj : T) * Qm;
            }
        }
        G[2 * i] = Rm;
        G[2 * i + 1] = Re;
    }
}

void or_residual(const or_grid* g, const or_props* pr, const double* K,
                 int32_t kstride, const double* phi, const double* kappa, int32_t nw,
                 const or_well* w, double dt, const double* x_prev,
                 const double* x, double* G)
{
    int32_t n = g->nx * g->ny * g->nz;
    double complex* xc = (double complex*)malloc(sizeof(double complex) * 2 * (size_t)n);
    double complex* Gc = malloc(sizeof(double complex) * 2 * (size_t)n);
    for (int32_t i = 0; i < 2 * n; ++i) xc[i] = x[i];
    or_residual_c(g, pr, K, kstride, phi, kappa, nw, w, dt, x_prev, xc, Gc);
    for (int32_t i = 0; i < 2 * n; ++i) G[i] = creal(Gc[i]);
    free(xc);
    free(Gc);
}

/* ---- Jacobian (eq. AXR ... eq. rhouT), upwind choice frozen ------------- */

static double rho_r(const or_props* pr, double p, double T)
{
    return pr->rho0 * exp(pr->c_p * (p - pr->p0) + pr->c_T * (T - pr->T0));
}

static double mu_r(const or_props* pr, double T)
{
    if (pr->api > 0.0) {
        double TF = (T - 273.15) * 9.0 / 5.0 + 32.0;
        return 1e-3 * pow(10.0, BEN_A1 * pr->api + BEN_A2) * pow(TF, BEN_A3 * pr->api + BEN_A4);
    }
    return pr->mu0 * exp(pr->mu_B * (1.0 / T - 1.0 / pr->T0));
}

/* -d ln(mu) / dT by hand: mu_B / T^2 for the exponential law; for Bennison's,
 * ln mu = const + (A3 api + A4) ln T_F and dT_F/dT = 9/5 */
static double minus_dlnmu_dT(const or_props* pr, double T)
{
    if (pr->api > 0.0) {
        double TF = (T - 273.15) * 9.0 / 5.0 + 32.0;
        return -(BEN_A3 * pr->api + BEN_A4) * (9.0 / 5.0) / TF;
    }
    return pr->mu_B / (T * T);
}

/* Face oriented lo->hi: flux F and its partial derivatives with respect to
 * (p_lo, p_hi, T_lo, T_hi); up = 0 if the lower cell is upwind. */
typedef struct {
    double F, dF_plo, dF_phi, dF_Tlo, dF_Thi, Tup, Th;
    int up_is_lo;
} face_t;

static face_t face_real(const or_grid* g, const or_props* pr, const double* K,
                        int32_t kstride, const double* kappa, const double* x, int32_t lo, int32_t hi,
                        int axis)
{
    face_t f;
    double ad = area_over_dist(g, axis);
    const double* Ka = K + (size_t)axis * (size_t)kstride;
    double Ups = ad * harmonic(Ka[lo], Ka[hi]);
    f.Th = ad * harmonic(kappa[lo], kappa[hi]);
    double pl = x[2 * lo], Tl = x[2 * lo + 1], ph = x[2 * hi], Thv = x[2 * hi + 1];
    double rl = rho_r(pr, pl, Tl), rh = rho_r(pr, ph, Thv);
    double dz = zc(g, lo) - zc(g, hi);
    double dphi = (pl - ph) + 0.5 * (rl + rh) * pr->g * dz;
    /* derivatives of dPhi */
    double dd_plo = 1.0 + 0.5 * pr->c_p * rl * pr->g * dz;
    double dd_phi = -1.0 + 0.5 * pr->c_p * rh * pr->g * dz;
    double dd_Tlo = 0.5 * pr->c_T * rl * pr->g * dz;
    double dd_Thi = 0.5 * pr->c_T * rh * pr->g * dz;
    f.up_is_lo = dphi >= 0.0;
    double lam, Tup;
    if (f.up_is_lo) { lam = rl / mu_r(pr, Tl); Tup = Tl; }
    else            { lam = rh / mu_r(pr, Thv); Tup = Thv; }
    double dlam_dp = pr->c_p * lam;
    double dlam_dT = (pr->c_T + minus_dlnmu_dT(pr, Tup)) * lam;
    f.F = Ups * lam * dphi;
    f.Tup = Tup;
    f.dF_plo = Ups * ((f.up_is_lo ? dlam_dp : 0.0) * dphi + lam * dd_plo);
    f.dF_phi = Ups * ((f.up_is_lo ? 0.0 : dlam_dp) * dphi + lam * dd_phi);
    f.dF_Tlo = Ups * ((f.up_is_lo ? dlam_dT : 0.0) * dphi + lam * dd_Tlo);
    f.dF_Thi = Ups * ((f.up_is_lo ? 0.0 : dlam_dT) * dphi + lam * dd_Thi);
    return f;
}

void or_jacobian(const or_grid* g, const or_props* pr, const double* K,
                 int32_t kstride, const double* phi, const double* kappa, int32_t nw,
                 const or_well* w, double dt, const double* x_prev,
                 const double* x, const int32_t* rowptr, const int32_t* col,
                 double* App, double* ApT, double* ATp, double* ATT, double* S)
{
    (void)x_prev;
    int32_t n = g->nx * g->ny * g->nz, ax;
    double V = g->dx * g->dy * g->dz;
    const double cv = pr->cv;
    for (int32_t i = 0; i < n; ++i) {
        double p = x[2 * i], T = x[2 * i + 1];
        double r = rho_r(pr, p, T);
        /* find diagonal slot */
        int32_t kd = -1;
        for (int32_t k = rowptr[i]; k < rowptr[i + 1]; ++k) {
            App[k] = ApT[k] = ATp[k] = ATT[k] = S[k] = 0.0;
            if (col[k] == i) kd = k;
        }
        /* accumulation terms */
        App[kd] = V * phi[i] * pr->c_p * r / dt;
        ApT[kd] = V * phi[i] * pr->c_T * r / dt;
        ATp[kd] = V * phi[i] * cv * pr->c_p * r * T / dt;
        ATT[kd] = V * (phi[i] * cv * (r + T * pr->c_T * r)
                       + (1.0 - phi[i]) * pr->rho_r * pr->c_r) / dt;
        S[kd] = V * (phi[i] * cv * r + (1.0 - phi[i]) * pr->rho_r * pr->c_r) / dt;
        /* faces, in ascending neighbour order */
        for (int d = 0; d < 6; ++d) {
            int32_t j = nb_cell(g, i, d, &ax);
            if (j < 0) continue;
            int32_t kj = -1;
            for (int32_t k = rowptr[i]; k < rowptr[i + 1]; ++k)
                if (col[k] == j) kj = k;
            int32_t lo = i < j ? i : j, hi = i < j ? j : i;
            face_t f = face_real(g, pr, K, kstride, kappa, x, lo, hi, ax);
            /* flux out of i and its derivatives w.r.t. (own, neighbour) */
            double s = (i == lo) ? 1.0 : -1.0;
            double Fout = s * f.F;
            double dFo_pi = s * ((i == lo) ? f.dF_plo : f.dF_phi);
            double dFo_pj = s * ((i == lo) ? f.dF_phi : f.dF_plo);
            double dFo_Ti = s * ((i == lo) ? f.dF_Tlo : f.dF_Thi);
            double dFo_Tj = s * ((i == lo) ? f.dF_Thi : f.dF_Tlo);
            int up_i = ((i == lo) == (f.up_is_lo != 0));
            /* mass rows */
            App[kd] += dFo_pi;
            App[kj] += dFo_pj;
            ApT[kd] += dFo_Ti;
            ApT[kj] += dFo_Tj;
            /* energy rows: c_v T_up F + Theta (T_i - T_j) */
            ATp[kd] += cv * f.Tup * dFo_pi;
            ATp[kj] += cv * f.Tup * dFo_pj;
            ATT[kd] += cv * ((up_i ? Fout : 0.0) + f.Tup * dFo_Ti) + f.Th;
            ATT[kj] += cv * ((up_i ? 0.0 : Fout) + f.Tup * dFo_Tj) - f.Th;
            /* eq. Se: frozen flux, upwinded dT, conduction */
            S[kd] += cv * (up_i ? Fout : 0.0) + f.Th;
            S[kj] += cv * (up_i ? 0.0 : Fout) - f.Th;
        }
        /* wells */
        for (int32_t k = 0; k < nw; ++k) {
            if (w[k].cell != i) continue;
            double q = w[k].rate;
            if (w[k].kind == 0) {
                double Qm = q * rho_r(pr, p, w[k].T_inj);
                App[kd] -= pr->c_p * Qm;
                ATp[kd] -= cv * w[k].T_inj * pr->c_p * Qm;
            } else if (w[k].kind == 1) {
                /* Q^m = -q rho_i, Q^e = -c_v T_i q rho_i */
                App[kd] += q * pr->c_p * r;
                ApT[kd] += q * pr->c_T * r;
                ATp[kd] += cv * T * q * pr->c_p * r;
                ATT[kd] += cv * q * (r + T * pr->c_T * r);
                S[kd] += cv * q * r;
            } else if (w[k].kind == 2) {
                /* heater: d(-U (T_h - T))/dT = U, in A_TT and in eq. Se (U D_heaters) */
                ATT[kd] += q;
                S[kd] += q;
            } else {
                /* Peaceman well: q_v = wi s (p_bh - p) / mu(T), s = +1 injector, -1
                 * producer; between its limits dq_v/dp = -s wi / mu and
                 * dq_v/dT = -q_v dln(mu)/dT, at a limit both vanish */
                int inj = w[k].kind == 3;
                double mu = mu_r(pr, T);
                double qv = w[k].wi * (inj ? w[k].p_bh - p : p - w[k].p_bh) / mu;
                double dq_dp = (inj ? -w[k].wi : w[k].wi) / mu;
                double dq_dT = qv * minus_dlnmu_dT(pr, T);
                if (qv >= q) { qv = q; dq_dp = 0.0; dq_dT = 0.0; }
                if (qv <= 0.0) { qv = 0.0; dq_dp = 0.0; dq_dT = 0.0; }
                if (inj) {
                    /* Q^m = q_v rho(p, T_inj), Q^e = c_v T_inj Q^m; G gets -Q */
                    double ri = rho_r(pr, p, w[k].T_inj);
                    double dQ_dp = dq_dp * ri + qv * pr->c_p * ri, dQ_dT = dq_dT * ri;
                    App[kd] -= dQ_dp;
                    ApT[kd] -= dQ_dT;
                    ATp[kd] -= cv * w[k].T_inj * dQ_dp;
                    ATT[kd] -= cv * w[k].T_inj * dQ_dT;
                } else {
                    /* Q^m = -q_v rho(p, T), Q^e = c_v T Q^m; eq. wellschurapprox keeps
                     * -c_v f_prod with the derivatives of the rate dropped */
                    double dM_dp = dq_dp * r + qv * pr->c_p * r;   /* d(q_v rho)/dp */
                    double dM_dT = dq_dT * r + qv * pr->c_T * r;   /* d(q_v rho)/dT */
                    App[kd] += dM_dp;
                    ApT[kd] += dM_dT;
                    ATp[kd] += cv * T * dM_dp;
                    ATT[kd] += cv * (qv * r + T * dM_dT);
                    S[kd] += cv * qv * r;
                }
            }
        }
    }
}
