// tp_assemble.hip -- TPFA residual, Jacobian blocks and Schur approximation.
//
// Section 2.2 of the paper: DG0 on a uniform Cartesian grid is the two-point
// flux finite-volume scheme.  Face transmissibilities use harmonic means of
// K and k_T, the face density is the arithmetic mean, mobility rho/mu and the
// advected temperature are upwinded on the potential difference
// dPhi = (p_lo - p_hi) + rho_bar g (z_lo - z_hi) of the face oriented from the
// lower to the higher cell index (dPhi >= 0 picks the lower cell).  The
// backward-Euler forms are eq. Fm and eq. Fe (with c_v on the advective
// energy flux), the Jacobian blocks those of eq. AXR with the upwind choice
// frozen, and S is the operator of eq. Se (frozen flux, upwinded dT,
// conduction, accumulation phi c_v rho + (1-phi) rho_r c_r, producer term
// c_v q rho).  Wells are point sources through the cell-indicator delta.
//
// One thread per cell writes its CSR row of all five matrices and its two
// residual entries.  Each face is evaluated by both of its cells from the
// same inputs in the same order, so the two flux values are bitwise equal
// and opposite: the scheme conserves mass and energy exactly, with no atomics.
#include "tp_internal.h"

namespace tp {

struct WellSet {
    int32_t n;
    tp_well w[TP_MAX_WELLS];
};

struct FaceOut {
    double F, dplo, dphi, dTlo, dThi, Tup, Th;
    bool up_lo;
};

__device__ inline double harmonic(double a, double b) {
    double s = a + b;
    return s > 0.0 ? 2.0 * a * b / s : 0.0;
}

__device__ inline double rho_of(const tp_props& pr, double p, double T) {
    return pr.rho0 * exp(pr.c_p * (p - pr.p0) + pr.c_T * (T - pr.T0));
}

// Bennison correlation (table bennison): log10 of the viscosity in cp is
// (A1 api + A2) + (A3 api + A4) log10(T_F)
constexpr double kBenA1 = -0.8021, kBenA2 = 23.8765, kBenA3 = 0.31458, kBenA4 = -9.21592;
constexpr double kLn10 = 2.302585092994045684;

__device__ inline double fahrenheit(double T) { return 1.8 * (T - 273.15) + 32.0; }

__device__ inline double mu_of(const tp_props& pr, double T) {
    if (pr.api > 0.0)
        return 1e-3 * exp(kLn10 * (kBenA1 * pr.api + kBenA2)
                          + (kBenA3 * pr.api + kBenA4) * log(fahrenheit(T)));
    return pr.mu0 * exp(pr.mu_B * (1.0 / T - 1.0 / pr.T0));
}

// d ln(mu) / dT
__device__ inline double dlnmu_dT(const tp_props& pr, double T) {
    if (pr.api > 0.0) return (kBenA3 * pr.api + kBenA4) * 1.8 / fahrenheit(T);
    return -pr.mu_B / (T * T);
}

// flux of one face oriented lo -> hi and its partial derivatives
__device__ inline FaceOut face_eval(const tp_props& pr, double ad, double Klo, double Khi,
                                    double klo, double khi, double pl, double Tl, double ph,
                                    double Th, double dz) {
    FaceOut f;
    double Ups = ad * harmonic(Klo, Khi);
    f.Th = ad * harmonic(klo, khi);
    double rl = rho_of(pr, pl, Tl), rh = rho_of(pr, ph, Th);
    double dphi = (pl - ph) + 0.5 * (rl + rh) * pr.g * dz;
    double dd_plo = 1.0 + 0.5 * pr.c_p * rl * pr.g * dz;
    double dd_phi = -1.0 + 0.5 * pr.c_p * rh * pr.g * dz;
    double dd_Tlo = 0.5 * pr.c_T * rl * pr.g * dz;
    double dd_Thi = 0.5 * pr.c_T * rh * pr.g * dz;
    f.up_lo = dphi >= 0.0;
    double lam, Tup;
    if (f.up_lo) { lam = rl / mu_of(pr, Tl); Tup = Tl; }
    else         { lam = rh / mu_of(pr, Th); Tup = Th; }
    double dlam_dp = pr.c_p * lam;
    double dlam_dT = (pr.c_T - dlnmu_dT(pr, Tup)) * lam;
    f.F = Ups * lam * dphi;
    f.Tup = Tup;
    f.dplo = Ups * ((f.up_lo ? dlam_dp : 0.0) * dphi + lam * dd_plo);
    f.dphi = Ups * ((f.up_lo ? 0.0 : dlam_dp) * dphi + lam * dd_phi);
    f.dTlo = Ups * ((f.up_lo ? dlam_dT : 0.0) * dphi + lam * dd_Tlo);
    f.dThi = Ups * ((f.up_lo ? 0.0 : dlam_dT) * dphi + lam * dd_Thi);
    return f;
}

__global__ void __launch_bounds__(256)
k_stencil_counts(tp_grid g, int32_t* __restrict__ cnt) {
    int32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    int32_t n = g.nx * g.ny * g.nz;
    if (i >= n) return;
    int32_t ix = i % g.nx, iy = (i / g.nx) % g.ny, iz = i / (g.nx * g.ny);
    cnt[i] = 1 + (iz > 0) + (iy > 0) + (ix > 0) + (ix < g.nx - 1) + (iy < g.ny - 1) + (iz < g.nz - 1);
}

__global__ void __launch_bounds__(256)
k_assemble(tp_grid g, tp_props pr, WellSet ws, double dt, const double* __restrict__ K,
           int32_t kstride, const double* __restrict__ phi, const double* __restrict__ kap,
           const double* __restrict__ xprev, const double* __restrict__ x,
           const int32_t* __restrict__ rowptr, int32_t* __restrict__ col,
           double* __restrict__ App, double* __restrict__ ApT, double* __restrict__ ATp,
           double* __restrict__ ATT, double* __restrict__ S, double* __restrict__ G) {
    const int32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    const int32_t nxy = g.nx * g.ny;
    const int32_t n = nxy * g.nz;
    if (i >= n) return;
    const int32_t ix = i % g.nx, iy = (i / g.nx) % g.ny, iz = i / nxy;
    const double V = g.dx * g.dy * g.dz;
    const double cv = pr.cv;
    const double p = x[2 * i], T = x[2 * i + 1];
    const double r = rho_of(pr, p, T);
    const double phi_i = phi[i];
    const double rn = rho_of(pr, xprev[2 * i], xprev[2 * i + 1]);
    const double Tn = xprev[2 * i + 1];

    double Rm = V * phi_i * (r - rn) / dt;
    double Re = V * (phi_i * cv * (r * T - rn * Tn) + (1.0 - phi_i) * pr.rho_r * pr.c_r * (T - Tn)) / dt;
    double dpp = V * phi_i * pr.c_p * r / dt;
    double dpT = V * phi_i * pr.c_T * r / dt;
    double dTp = V * phi_i * cv * pr.c_p * r * T / dt;
    double dTT = V * (phi_i * cv * (r + T * pr.c_T * r) + (1.0 - phi_i) * pr.rho_r * pr.c_r) / dt;
    double dS = V * (phi_i * cv * r + (1.0 - phi_i) * pr.rho_r * pr.c_r) / dt;

    const int32_t base = rowptr[i];
    const int nlow = (iz > 0) + (iy > 0) + (ix > 0);
    const int32_t kd = base + nlow;
    col[kd] = i;
    int32_t k = base;
    const double zi = (iz + 0.5) * g.dz;
    const double ad_axis[3] = {g.dy * g.dz / g.dx, g.dx * g.dz / g.dy, g.dx * g.dy / g.dz};

#pragma unroll
    for (int d = 0; d < 6; ++d) {
        int32_t j;
        int axis;
        bool ok;
        switch (d) {
        case 0: ok = iz > 0; j = i - nxy; axis = 2; break;
        case 1: ok = iy > 0; j = i - g.nx; axis = 1; break;
        case 2: ok = ix > 0; j = i - 1; axis = 0; break;
        case 3: ok = ix < g.nx - 1; j = i + 1; axis = 0; break;
        case 4: ok = iy < g.ny - 1; j = i + g.nx; axis = 1; break;
        default: ok = iz < g.nz - 1; j = i + nxy; axis = 2; break;
        }
        if (d == 3) k = kd + 1;
        if (!ok) continue;
        const bool i_lo = i < j;
        const int32_t lo = i_lo ? i : j, hi = i_lo ? j : i;
        const double zlo = (lo / nxy + 0.5) * g.dz, zhi = (hi / nxy + 0.5) * g.dz;
        (void)zi;
        const double* Ka = K + (size_t)axis * (size_t)kstride;
        FaceOut f = face_eval(pr, ad_axis[axis], Ka[lo], Ka[hi], kap[lo], kap[hi], x[2 * lo],
                              x[2 * lo + 1], x[2 * hi], x[2 * hi + 1], zlo - zhi);
        const double s = i_lo ? 1.0 : -1.0;
        const double Fout = s * f.F;
        const double dFo_pi = s * (i_lo ? f.dplo : f.dphi);
        const double dFo_pj = s * (i_lo ? f.dphi : f.dplo);
        const double dFo_Ti = s * (i_lo ? f.dTlo : f.dThi);
        const double dFo_Tj = s * (i_lo ? f.dThi : f.dTlo);
        const bool up_i = (i_lo == f.up_lo);
        const double Tj = x[2 * j + 1];
        // residual
        Rm += Fout;
        Re += cv * f.Tup * Fout + f.Th * (T - Tj);
        // Jacobian
        dpp += dFo_pi;
        dpT += dFo_Ti;
        dTp += cv * f.Tup * dFo_pi;
        dTT += cv * ((up_i ? Fout : 0.0) + f.Tup * dFo_Ti) + f.Th;
        dS += cv * (up_i ? Fout : 0.0) + f.Th;
        col[k] = j;
        App[k] = dFo_pj;
        ApT[k] = dFo_Tj;
        ATp[k] = cv * f.Tup * dFo_pj;
        ATT[k] = cv * ((up_i ? 0.0 : Fout) + f.Tup * dFo_Tj) - f.Th;
        S[k] = cv * (up_i ? 0.0 : Fout) - f.Th;
        ++k;
    }
    for (int32_t w = 0; w < ws.n; ++w) {
        if (ws.w[w].cell != i) continue;
        const double q = ws.w[w].rate;
        if (ws.w[w].kind == 0) {
            const double Qm = q * rho_of(pr, p, ws.w[w].T_inj);
            Rm -= Qm;
            Re -= cv * ws.w[w].T_inj * Qm;
            dpp -= pr.c_p * Qm;
            dTp -= cv * ws.w[w].T_inj * pr.c_p * Qm;
        } else if (ws.w[w].kind == 1) {
            const double Qm = -q * r;
            Rm -= Qm;
            Re -= cv * T * Qm;
            dpp += q * pr.c_p * r;
            dpT += q * pr.c_T * r;
            dTp += cv * T * q * pr.c_p * r;
            dTT += cv * q * (r + T * pr.c_T * r);
            dS += cv * q * r;
        } else if (ws.w[w].kind == 2) {  // heater: energy source U (T_heater - T)
            Re -= q * (ws.w[w].T_inj - T);
            dTT += q;
            dS += q;
        } else {  // Peaceman well: rate from the bottom-hole pressure, within [0, q]
            const bool inj = ws.w[w].kind == 3;
            const double mu = mu_of(pr, T);
            double qv = ws.w[w].wi * (inj ? ws.w[w].p_bh - p : p - ws.w[w].p_bh) / mu;
            double dq_dp = (inj ? -ws.w[w].wi : ws.w[w].wi) / mu;
            double dq_dT = -qv * dlnmu_dT(pr, T);
            if (qv >= q) { qv = q; dq_dp = 0.0; dq_dT = 0.0; }
            if (qv <= 0.0) { qv = 0.0; dq_dp = 0.0; dq_dT = 0.0; }
            if (inj) {
                const double ri = rho_of(pr, p, ws.w[w].T_inj);
                const double Qm = qv * ri;
                const double dQp = dq_dp * ri + pr.c_p * Qm, dQT = dq_dT * ri;
                Rm -= Qm;
                Re -= cv * ws.w[w].T_inj * Qm;
                dpp -= dQp;
                dpT -= dQT;
                dTp -= cv * ws.w[w].T_inj * dQp;
                dTT -= cv * ws.w[w].T_inj * dQT;
            } else {
                const double M = qv * r;  // produced mass rate
                const double dMp = dq_dp * r + pr.c_p * M, dMT = dq_dT * r + pr.c_T * M;
                Rm += M;
                Re += cv * T * M;
                dpp += dMp;
                dpT += dMT;
                dTp += cv * T * dMp;
                dTT += cv * (M + T * dMT);
                dS += cv * M;
            }
        }
    }
    App[kd] = dpp;
    ApT[kd] = dpT;
    ATp[kd] = dTp;
    ATT[kd] = dTT;
    S[kd] = dS;
    G[2 * i] = Rm;
    G[2 * i + 1] = Re;
}

static int64_t stencil_nnz(const tp_grid& g) {
    int64_t nx = g.nx, ny = g.ny, nz = g.nz;
    return nx * ny * nz + 2 * ((nx - 1) * ny * nz + nx * (ny - 1) * nz + nx * ny * (nz - 1));
}

}  // namespace tp

extern "C" {

int tp_jacobian_sizes(const tp_grid* grid, int32_t* n, int32_t* nnz) {
    TP_GUARD({
        TP_CHECK_ARG(grid && n && nnz, "null argument");
        TP_CHECK_ARG(grid->nx >= 1 && grid->ny >= 1 && grid->nz >= 1, "grid dimensions must be >= 1");
        int64_t nn = (int64_t)grid->nx * grid->ny * grid->nz;
        int64_t z = tp::stencil_nnz(*grid);
        TP_CHECK_ARG(z < INT32_MAX && nn < INT32_MAX, "grid too large for int32 indices");
        *n = (int32_t)nn;
        *nnz = (int32_t)z;
    });
    return TP_OK;
}

namespace {

int assemble(const tp_grid* grid, const tp_props* props, const double* K, bool diag_tensor,
             const double* phi, const double* kappa, int32_t nwells, const tp_well* wells,
             double dt, const double* x_prev, const double* x_k, tp_jacobian* J, double* G,
             void* stream) {
    TP_GUARD({
        TP_CHECK_ARG(grid && props && K && phi && kappa && x_prev && x_k && J && G,
                     "assemble_tpfa: null argument");
        int32_t n, nnz;
        int st = tp_jacobian_sizes(grid, &n, &nnz);
        if (st != TP_OK) return st;
        TP_CHECK_ARG(J->n == n && J->nnz == nnz, "assemble_tpfa: J sized n=%d nnz=%d, grid needs n=%d nnz=%d",
                     J->n, J->nnz, n, nnz);
        TP_CHECK_ARG(J->rowptr && J->col && J->pp && J->pT && J->Tp && J->TT && J->S,
                     "assemble_tpfa: null Jacobian array");
        TP_CHECK_ARG(dt > 0.0, "assemble_tpfa: dt must be > 0");
        TP_CHECK_ARG(grid->dx > 0 && grid->dy > 0 && grid->dz > 0, "assemble_tpfa: spacing must be > 0");
        TP_CHECK_ARG(nwells >= 0 && nwells <= TP_MAX_WELLS, "assemble_tpfa: nwells %d outside [0,%d]",
                     nwells, TP_MAX_WELLS);
        TP_CHECK_ARG(nwells == 0 || wells, "assemble_tpfa: wells is null");
        tp::WellSet ws;
        ws.n = nwells;
        for (int32_t w = 0; w < nwells; ++w) {
            TP_CHECK_ARG(wells[w].cell >= 0 && wells[w].cell < n, "well %d cell %d out of range", w, wells[w].cell);
            TP_CHECK_ARG(wells[w].kind >= 0 && wells[w].kind <= 4, "well %d kind must be 0 to 4", w);
            TP_CHECK_ARG(wells[w].kind < 3 || wells[w].wi > 0.0, "well %d: Peaceman well index must be > 0", w);
            TP_CHECK_ARG(wells[w].rate >= 0.0, "well %d rate must be >= 0", w);
            ws.w[w] = wells[w];
        }
        hipStream_t s = (hipStream_t)stream;
        const int B = 256;
        TP_LAUNCH(tp::k_stencil_counts, tp::cdiv(n, B), B, 0, s, *grid, J->rowptr);
        tp::scan_exclusive(J->rowptr, J->rowptr, n, s);
        TP_LAUNCH(tp::k_assemble, tp::cdiv(n, B), B, 0, s, *grid, *props, ws, dt, K,
                  diag_tensor ? n : 0, phi, kappa, x_prev, x_k, J->rowptr, J->col, J->pp, J->pT,
                  J->Tp, J->TT, J->S, G);
    });
    return TP_OK;
}

}  // namespace

int assemble_tpfa(const tp_grid* grid, const tp_props* props, const double* K,
                  const double* phi, const double* kappa, int32_t nwells,
                  const tp_well* wells, double dt, const double* x_prev,
                  const double* x_k, tp_jacobian* J, double* G, void* stream) {
    return assemble(grid, props, K, false, phi, kappa, nwells, wells, dt, x_prev, x_k, J, G,
                    stream);
}

int assemble_tpfa_aniso(const tp_grid* grid, const tp_props* props, const double* K3,
                        const double* phi, const double* kappa, int32_t nwells,
                        const tp_well* wells, double dt, const double* x_prev,
                        const double* x_k, tp_jacobian* J, double* G, void* stream) {
    return assemble(grid, props, K3, true, phi, kappa, nwells, wells, dt, x_prev, x_k, J, G,
                    stream);
}

}  // extern "C"
