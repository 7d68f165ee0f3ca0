// tp_krylov.hip -- block preconditioner and flexible GMRES on the GPU.
//
// Preconditioner: the five-step application list of Section 3.2.  The lower
// form (steps 1-3) solves A_pp x_p = b_p, forms b~_T = b_T - A_Tp x_p and
// solves S~ d_T = b~_T, each solve being one AMG V-cycle; the full form adds
// steps 4-5 with b~_p = b_p - A_pT d_T; the upper form runs the Schur solve
// first.  The CPR comparator (Section 3.1) is the two-stage form
// x1 = [V_pp(r_p); 0], x = ILU0^{-1}(r - J x1) + x1.  Internally the p and T halves of a vector are stored split
// ([p_0..p_{n-1}, T_0..T_{n-1}]), a symmetric permutation of the
// interleaved ordering at the interface.
//
// FGMRES (Saad 1993; right preconditioning as in Section 4, restart 30):
// classical Gram-Schmidt applied twice (CGS2) with all inner products
// reduced over a fixed grid in a fixed order, so results are run-to-run
// deterministic; Hessenberg, Givens rotations and the small triangular solve
// stay on the device in FP64.  One 8-byte device->host read per iteration
// carries the residual estimate for the stopping test.
#include "tp_amg.h"

#include <cmath>
#include <mutex>

namespace tp {
void cast_d2s(int32_t n, const double* a, void* b, size_t es, hipStream_t s);
void cast_s2d(int32_t n, const void* a, double* b, size_t es, hipStream_t s);
}  // namespace tp

namespace tp {
struct Gmres;
void gmres_free(Gmres* g);
void ilu_solve(tp_ilu* F, const double* b, double* x, hipStream_t s);
int32_t ilu_cells(const tp_ilu* F);
}  // namespace tp

struct tp_prec {
    tp::Gmres* ws = nullptr;  // FGMRES workspace kept across solves of the same size
    // The split-vector apply captured once as a HIP graph (kernels only, no
    // stream-specific state) on fixed staging vectors rin -> zout.
    hipGraphExec_t gexec = nullptr;
    // the same with the learned post-smoother of the Schur hierarchy enabled,
    // valid for the attachment numbered gen_cnn
    hipGraphExec_t gexec_cnn = nullptr;
    uint64_t gen_cnn = 0;
    // the stream of the handle's last launch (one stream so far: its
    // synchronisation suffices at destruction; several: the device's)
    hipStream_t last = nullptr;
    bool used = false, multi = false;
    tp::DBuf<double> rin, zout;
    tp_jacobian J;
    tp_amg* pp = nullptr;
    tp_amg* S = nullptr;  // null for CPR
    tp_ilu* ilu = nullptr;  // CPR second stage (ILU(0) of the field-ordered Jacobian)
    int variant = 0;      // 0 lower, 1 upper, 2 full, 3 CPR
    tp::DBuf<double> cw, cb;  // CPR: first-stage pressure x1 (n) and the residual r - J x1 (2n)
    tp::DBuf<double> rs, zs;  // split work vectors (2n) for the interleaved entry point
    // The Jacobian's stencil, for the sparse products with implied columns:
    // st_nd offsets (column - row, ascending) from which every entry of the
    // pattern is drawn, so that a row of st_nd entries holds all of them;
    // st_nd = 0 when the pattern is not of that form (st_done: examined).
    int32_t st_nd = 0;
    int32_t st_off[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    bool st_done = false;
};

namespace tp {

constexpr int KB = 256;
constexpr int MAXK = 32;      // restart length bound (H has MAXK+1 rows)

// ---- layout ----------------------------------------------------------------------
__global__ void __launch_bounds__(KB)
k_deinterleave(int32_t n, const double* __restrict__ in, double* __restrict__ out) {
    int32_t i = blockIdx.x * KB + threadIdx.x;
    if (i >= n) return;
    out[i] = in[2 * i];
    out[n + i] = in[2 * i + 1];
}

__global__ void __launch_bounds__(KB)
k_interleave(int32_t n, const double* __restrict__ in, double* __restrict__ out) {
    int32_t i = blockIdx.x * KB + threadIdx.x;
    if (i >= n) return;
    out[2 * i] = in[i];
    out[2 * i + 1] = in[n + i];
}

__global__ void k_zero_u32(unsigned int* p) {
    if (threadIdx.x == 0 && blockIdx.x == 0) *p = 0u;
}

__global__ void k_zero_i32(int32_t* p) {
    if (threadIdx.x == 0 && blockIdx.x == 0) *p = 0;
}

__global__ void __launch_bounds__(KB)
k_zero_d(int64_t N, double* __restrict__ x) {
    int64_t i = (int64_t)blockIdx.x * KB + threadIdx.x;
    if (i < N) x[i] = 0.0;
}

// ---- sparse products on the Jacobian -----------------------------------------------
// Lanes per stencil row (at most 7 entries: two passes of 4).  Measured on
// the 256x256x64 Jacobian: 4 lanes take 1.5% less time per FGMRES
// iteration than 8 or 2, and 20% less than one lane per row.
constexpr int JG = 4;

// out = rhs - M x (rhs may be null: out = -M x is never needed; null -> M x)
template <typename To>
__global__ void __launch_bounds__(KB)
k_spmv_sub(int32_t n, const int32_t* __restrict__ rp, const int32_t* __restrict__ ci,
           const double* __restrict__ av, const double* __restrict__ x, const double* __restrict__ rhs,
           To* __restrict__ out) {
    const int64_t tid = (int64_t)blockIdx.x * KB + threadIdx.x;
    const int32_t i = (int32_t)(tid / JG);
    const int lane = (int)(tid % JG);
    double s = 0.0;
    if (i < n)
        for (int32_t q = rp[i] + lane; q < rp[i + 1]; q += JG) s += av[q] * x[ci[q]];
#pragma unroll
    for (int off = JG / 2; off > 0; off >>= 1) s += __shfl_down(s, off, JG);
    if (i < n && lane == 0) out[i] = (To)(rhs[i] - s);
}

// w = J z (split vectors); with b: w = b - J z
__global__ void __launch_bounds__(KB)
k_block_spmv(int32_t n, const int32_t* __restrict__ rp, const int32_t* __restrict__ ci,
             const double* __restrict__ pp, const double* __restrict__ pT, const double* __restrict__ Tp,
             const double* __restrict__ TT, const double* __restrict__ z, const double* __restrict__ b,
             double* __restrict__ w, double* __restrict__ zcopy) {
    const int64_t tid = (int64_t)blockIdx.x * KB + threadIdx.x;
    const int32_t i = (int32_t)(tid / JG);
    const int lane = (int)(tid % JG);
    double sm = 0.0, se = 0.0;
    if (i < n) {
        const double* zp = z;
        const double* zT = z + n;
        for (int32_t q = rp[i] + lane; q < rp[i + 1]; q += JG) {
            const int32_t j = ci[q];
            const double a = zp[j], c = zT[j];
            sm += pp[q] * a + pT[q] * c;
            se += Tp[q] * a + TT[q] * c;
        }
    }
#pragma unroll
    for (int off = JG / 2; off > 0; off >>= 1) {
        sm += __shfl_down(sm, off, JG);
        se += __shfl_down(se, off, JG);
    }
    if (i < n && lane == 0) {
        if (b) {
            w[i] = b[i] - sm;
            w[n + i] = b[n + i] - se;
        } else {
            w[i] = sm;
            w[n + i] = se;
        }
        if (zcopy) {
            zcopy[i] = z[i];
            zcopy[n + i] = z[n + i];
        }
    }
}

// ---- the same products on a stencil pattern --------------------------------------------
// Every entry's column is row + one of ND offsets (ascending), so a row of ND
// entries holds them all and its columns need not be loaded.  A workgroup
// takes ST_ROWS consecutive rows: it loads their values into LDS in one
// coalesced sweep, then each thread sums its row in entry order (rows of
// fewer entries, at the domain's faces, read their columns).
constexpr int ST_ROWS = 256;
struct StencilOffs {
    int32_t off[8];
};

// stage the values of rows [i0, iend) (q0 = rp[i0], q1 = rp[iend], at most
// ST_ROWS * ND of them) in s_a: every load is issued before the stores
template <int ND>
__device__ inline void stage_rows(const double* __restrict__ av, int32_t q0, int32_t q1, double* s_a) {
    double v[ND];
#pragma unroll
    for (int k = 0; k < ND; ++k) {
        const int32_t q = q0 + (int32_t)threadIdx.x + k * ST_ROWS;
        v[k] = q < q1 ? av[q] : 0.0;
    }
#pragma unroll
    for (int k = 0; k < ND; ++k) {
        const int32_t q = q0 + (int32_t)threadIdx.x + k * ST_ROWS;
        if (q < q1) s_a[q - q0] = v[k];
    }
}

template <typename To, int ND>
__global__ void __launch_bounds__(ST_ROWS)
k_spmv_sub_st(int32_t n, const int32_t* __restrict__ rp, const int32_t* __restrict__ ci,
              const double* __restrict__ av, const double* __restrict__ x, const double* __restrict__ rhs,
              To* __restrict__ out, StencilOffs st) {
    __shared__ double s_a[ST_ROWS * ND];
    const int32_t i0 = blockIdx.x * ST_ROWS, i = i0 + (int32_t)threadIdx.x;
    const bool in = i < n;
    // everything that does not wait for the staged values is loaded first
    const int32_t q0 = rp[i0], q1 = rp[min(n, i0 + ST_ROWS)];
    const int32_t a = in ? rp[i] : 0, e = in ? rp[i + 1] : 0;
    const double r = in ? rhs[i] : 0.0;
    double xv[ND];  // the stencil's x (a full row's; clamped indices elsewhere)
#pragma unroll
    for (int d = 0; d < ND; ++d) xv[d] = x[min(max(i + st.off[d], 0), n - 1)];
    stage_rows<ND>(av, q0, q1, s_a);
    __syncthreads();
    if (!in) return;
    double sum = 0.0;
    if (e - a == ND) {
#pragma unroll
        for (int d = 0; d < ND; ++d) sum += s_a[a - q0 + d] * xv[d];
    } else {
        for (int32_t q = a; q < e; ++q) sum += s_a[q - q0] * x[ci[q]];
    }
    out[i] = (To)(r - sum);
}

// w = J z (split vectors), with b: w = b - J z; the pressure rows' two
// blocks are staged first, then the temperature rows'
template <int ND>
__global__ void __launch_bounds__(ST_ROWS)
k_block_spmv_st(int32_t n, const int32_t* __restrict__ rp, const int32_t* __restrict__ ci,
                const double* __restrict__ pp, const double* __restrict__ pT, const double* __restrict__ Tp,
                const double* __restrict__ TT, const double* __restrict__ z, const double* __restrict__ b,
                double* __restrict__ w, double* __restrict__ zcopy, StencilOffs st) {
    __shared__ double s_a[ST_ROWS * ND], s_c[ST_ROWS * ND];
    const int32_t i0 = blockIdx.x * ST_ROWS, i = i0 + (int32_t)threadIdx.x;
    const int32_t q0 = rp[i0], q1 = rp[min(n, i0 + ST_ROWS)];
    const bool in = i < n;
    const int32_t a = in ? rp[i] : 0, e = in ? rp[i + 1] : 0;
    const bool full = e - a == ND;
    const double* zp = z;
    const double* zT = z + n;
    double za[ND], zc[ND];  // the stencil's z (a full row's; clamped indices elsewhere)
#pragma unroll
    for (int d = 0; d < ND; ++d) {
        const int32_t j = min(max(i + st.off[d], 0), n - 1);
        za[d] = zp[j];
        zc[d] = zT[j];
    }
    double res[2];
#pragma unroll
    for (int half = 0; half < 2; ++half) {
        if (half) __syncthreads();  // (the first half's values are read until here)
        stage_rows<ND>(half ? Tp : pp, q0, q1, s_a);
        stage_rows<ND>(half ? TT : pT, q0, q1, s_c);
        __syncthreads();
        double sum = 0.0;
        if (in) {
            if (full) {
#pragma unroll
                for (int d = 0; d < ND; ++d) sum += s_a[a - q0 + d] * za[d] + s_c[a - q0 + d] * zc[d];
            } else {
                for (int32_t q = a; q < e; ++q) {
                    const int32_t j = ci[q];
                    sum += s_a[q - q0] * zp[j] + s_c[q - q0] * zT[j];
                }
            }
        }
        res[half] = sum;
    }
    if (!in) return;
    if (b) {
        w[i] = b[i] - res[0];
        w[n + i] = b[n + i] - res[1];
    } else {
        w[i] = res[0];
        w[n + i] = res[1];
    }
    if (zcopy) {
        zcopy[i] = z[i];
        zcopy[n + i] = z[n + i];
    }
}

// *bad = 1 when some entry's column - row is not among the nd offsets
__global__ void __launch_bounds__(KB)
k_stencil_check(int32_t n, const int32_t* __restrict__ rp, const int32_t* __restrict__ ci, int32_t nd,
                StencilOffs st, int32_t* __restrict__ bad) {
    const int32_t i = blockIdx.x * KB + threadIdx.x;
    if (i >= n) return;
    for (int32_t q = rp[i]; q < rp[i + 1]; ++q) {
        const int32_t o = ci[q] - i;
        bool hit = false;
        for (int d = 0; d < nd; ++d) hit |= o == st.off[d];
        if (!hit) {
            *bad = 1;
            return;
        }
    }
}

// CPR stage residual, field order: b1 = r - J [x1; 0] (x1 in the pressure rows)
__global__ void __launch_bounds__(KB)
k_cpr_resid(int32_t n, const int32_t* __restrict__ rp, const int32_t* __restrict__ ci,
            const double* __restrict__ pp, const double* __restrict__ Tp, const double* __restrict__ x1,
            const double* __restrict__ r, double* __restrict__ b1) {
    const int64_t tid = (int64_t)blockIdx.x * KB + threadIdx.x;
    const int32_t i = (int32_t)(tid / JG);
    const int lane = (int)(tid % JG);
    double sm = 0.0, se = 0.0;
    if (i < n) {
        for (int32_t q = rp[i] + lane; q < rp[i + 1]; q += JG) {
            const double a = x1[ci[q]];
            sm += pp[q] * a;
            se += Tp[q] * a;
        }
    }
#pragma unroll
    for (int off = JG / 2; off > 0; off >>= 1) {
        sm += __shfl_down(sm, off, JG);
        se += __shfl_down(se, off, JG);
    }
    if (i < n && lane == 0) {
        b1[i] = r[i] - sm;
        b1[n + i] = r[n + i] - se;
    }
}

// z_p += x1 (the correction of the second stage plus the first stage)
__global__ void __launch_bounds__(KB)
k_add_into(int32_t n, const double* __restrict__ a, double* __restrict__ z) {
    const int32_t i = blockIdx.x * KB + threadIdx.x;
    if (i < n) z[i] += a[i];
}

// ---- CGS2 building blocks -------------------------------------------------------------
// One pass over the basis V_0..V_{k-1} (each column read once):
//   mode 0: out[i] = V_i . w
//   mode 1: w <- w - sum_i h_i V_i, then out[i] = V_i . w_new
//   mode 2: w <- w - sum_i h_i V_i (k may be 0), then out[0] = w_new . w_new
// Elements are assigned to threads by a fixed grid-stride pattern; each
// block writes partial sums (vector-major), and the last block to finish
// reduces them in a fixed order, so the result is run-to-run deterministic.
// With `arn` set (mode 2), that last block also performs the Arnoldi column
// update (Givens rotations) for column j.
constexpr int CG_T = 256;
constexpr int CG_W = CG_T / 64;

struct ArnoldiArgs {
    int j, m;
    const double* h1;
    const double* h2;
    double* H;
    double* cs;
    double* sn;
    double* g;
    double* sc;  // [0] ||w||, [1] |g[j+1]|
};

__device__ inline double wave_sum(double v) {
    for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
    return v;
}

// Givens update of Hessenberg column j; the column, the previous rotations
// and g are staged in LDS by the whole workgroup, rotated by one thread,
// then written back in parallel.
__device__ void arnoldi_update_block(const ArnoldiArgs& a, double nrm2, double* hc, double* cs, double* sn,
                                     double* gg) {
    const int j = a.j, m = a.m, t = threadIdx.x;
    for (int i = t; i <= j; i += blockDim.x) {
        hc[i] = a.h1[i] + a.h2[i];
        if (i < j) { cs[i] = a.cs[i]; sn[i] = a.sn[i]; }
    }
    if (t == 0) { gg[0] = a.g[j]; }
    __syncthreads();
    if (t == 0) {
        const double hn = sqrt(nrm2);
        hc[j + 1] = hn;
        for (int i = 0; i < j; ++i) {
            double x = hc[i], y = hc[i + 1];
            hc[i] = cs[i] * x + sn[i] * y;
            hc[i + 1] = -sn[i] * x + cs[i] * y;
        }
        double x = hc[j], y = hc[j + 1];
        double den = hypot(x, y);
        cs[j] = x / den;
        sn[j] = y / den;
        hc[j] = den;
        hc[j + 1] = 0.0;
        const double gj = gg[0];
        a.g[j + 1] = -sn[j] * gj;
        a.g[j] = cs[j] * gj;
        a.cs[j] = cs[j];
        a.sn[j] = sn[j];
        a.sc[0] = hn;
        a.sc[1] = fabs(-sn[j] * gj);
    }
    __syncthreads();
    for (int i = t; i <= j + 1; i += blockDim.x) a.H[i * m + j] = hc[i];
}

template <int K>
__global__ void __launch_bounds__(CG_T)
k_cgs(int64_t N, const double* __restrict__ V, const double* __restrict__ h, double* __restrict__ w,
      int mode, double* __restrict__ part) {
    constexpr int KA = K > 0 ? K : 1;
    __shared__ double red[CG_W][KA];
    const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
    const int nb = gridDim.x;
    double acc[KA];
    double hh[KA];
#pragma unroll
    for (int i = 0; i < KA; ++i) {
        acc[i] = 0.0;
        hh[i] = (mode >= 1 && i < K) ? h[i] : 0.0;
    }
    const int64_t stride = (int64_t)nb * CG_T;
    for (int64_t e = (int64_t)blockIdx.x * CG_T + t; e < N; e += stride) {
        double we = w[e];
        double v[KA];
#pragma unroll
        for (int i = 0; i < K; ++i) v[i] = V[(int64_t)i * N + e];
        if (mode >= 1) {
#pragma unroll
            for (int i = 0; i < K; ++i) we -= hh[i] * v[i];
            w[e] = we;
        }
        if (mode == 2) {
            acc[0] += we * we;
        } else {
#pragma unroll
            for (int i = 0; i < K; ++i) acc[i] += v[i] * we;
        }
    }
    const int cnt = mode == 2 ? 1 : K;
#pragma unroll
    for (int i = 0; i < KA; ++i) {
        if (i < cnt) {
            double s = wave_sum(acc[i]);
            if (lane == 0) red[wave][i] = s;
        }
    }
    __syncthreads();
    if (t < cnt) {
        double s = 0.0;
        for (int q = 0; q < CG_W; ++q) s += red[q][t];
        part[(int64_t)t * nb + blockIdx.x] = s;
    }
}

// Sum the per-block partials (one wavefront per vector, fixed order); with
// `arn`, thread 0 then performs the Arnoldi column update.
constexpr int FIN_T = 1024;
__global__ void __launch_bounds__(FIN_T)
k_cgs_finish(int nb, int cnt, const double* __restrict__ part, double* __restrict__ out, int arn,
             ArnoldiArgs aa) {
    __shared__ double hc[MAXK + 1], cs[MAXK], sn[MAXK], gg[1], nrm;
    const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
    for (int i = wave; i < cnt; i += FIN_T / 64) {
        double s = 0.0;
        for (int b = lane; b < nb; b += 64) s += part[(int64_t)i * nb + b];
        s = wave_sum(s);
        if (lane == 0) {
            out[i] = s;
            if (i == 0) nrm = s;
        }
    }
    if (!arn) return;
    __syncthreads();
    arnoldi_update_block(aa, nrm, hc, cs, sn, gg);
}

// v = w / nrm (nrm on device); optionally also into v2 (the graph's input);
// flag (when given) = the learned smoother's failure flag bad (0 without one)
__global__ void __launch_bounds__(KB)
k_scale_div(int64_t N, const double* __restrict__ w, const double* __restrict__ nrm, double* __restrict__ v,
            double* __restrict__ v2, const int32_t* __restrict__ bad, double* __restrict__ flag) {
    int64_t i = (int64_t)blockIdx.x * KB + threadIdx.x;
    if (i == 0 && flag) flag[0] = bad ? (double)bad[0] : 0.0;
    if (i >= N) return;
    const double q = w[i] / nrm[0];
    v[i] = q;
    if (v2) v2[i] = q;
}

// start of a cycle: beta = sqrt(nrm2); g = [beta, 0, ...]; sc[0] = beta
__global__ void k_cycle_init(int m, const double* __restrict__ nrm2, double* __restrict__ g,
                             double* __restrict__ sc) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    double beta = sqrt(nrm2[0]);
    for (int i = 0; i <= m; ++i) g[i] = 0.0;
    g[0] = beta;
    sc[0] = beta;
}

// y = H(0:k,0:k)^{-1} g(0:k)
__global__ void k_hess_solve(int k, int m, const double* __restrict__ H, const double* __restrict__ g,
                             double* __restrict__ y) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    for (int i = k - 1; i >= 0; --i) {
        double s = g[i];
        for (int q = i + 1; q < k; ++q) s -= H[i * m + q] * y[q];
        y[i] = s / H[i * m + i];
    }
}

// x += sum_i y_i Z_i
__global__ void __launch_bounds__(KB)
k_xupdate(int64_t N, int k, const double* __restrict__ Z, const double* __restrict__ y, double* __restrict__ x) {
    int64_t e = (int64_t)blockIdx.x * KB + threadIdx.x;
    if (e >= N) return;
    double v = x[e];
    for (int i = 0; i < k; ++i) v += y[i] * Z[(int64_t)i * N + e];
    x[e] = v;
}

// ---- preconditioner on split vectors ------------------------------------------------------
// One V-cycle of h on rhs into out.  With FP64 storage the cycle reads rhs
// and writes out directly; with FP32 storage both are converted.
static void vsolve(tp_amg* h, const double* rhs, double* out, int32_t n, hipStream_t s) {
    const size_t es = storage_bytes(h);
    if (es == 8) {
        const void* x = vcycle_run(h, rhs, s, out);
        if (x != out) cast_s2d(n, x, out, es, s);
        return;
    }
    cast_d2s(n, rhs, h->lev[0].b.p, es, s);
    const void* x = vcycle_run(h, nullptr, s);
    cast_s2d(n, x, out, es, s);
}

// The Jacobian's stencil offsets (tp_prec::st_nd), examined once per handle
// before its first product: the longest of up to 1024 rows from the middle
// of the grid (an interior cell when there is one) gives the candidate
// offsets, and a check over the whole pattern confirms them.  Stencils of 5
// (2-D) or 7 (3-D) offsets take the implied-column kernels.
static void stencil_detect(tp_prec* P, hipStream_t s) {
    P->st_done = true;
    const tp_jacobian& J = P->J;
    const int32_t n = J.n, i0 = n / 2, w = std::min(n - i0, 1024);
    std::vector<int32_t> ext(w + 1);
    TP_HIP(hipMemcpyAsync(ext.data(), J.rowptr + i0, sizeof(int32_t) * (w + 1), hipMemcpyDeviceToHost, s));
    TP_HIP(hipStreamSynchronize(s));
    int32_t i = i0, nd = 0;
    for (int32_t k = 0; k < w; ++k)
        if (ext[k + 1] - ext[k] > nd) {
            nd = ext[k + 1] - ext[k];
            i = i0 + k;
        }
    if (nd != 5 && nd != 7) return;
    int32_t cols[8];
    TP_HIP(hipMemcpyAsync(cols, J.col + ext[i - i0], sizeof(int32_t) * nd, hipMemcpyDeviceToHost, s));
    TP_HIP(hipStreamSynchronize(s));
    StencilOffs st{};
    for (int d = 0; d < nd; ++d) st.off[d] = cols[d] - i;
    DBuf<int32_t> bad(1, s);
    TP_LAUNCH(k_zero_i32, 1, 1, 0, s, bad.p);
    TP_LAUNCH(k_stencil_check, cdiv(n, KB), KB, 0, s, n, J.rowptr, J.col, nd, st, bad.p);
    if (read_i32(bad.p, s)) return;
    P->st_nd = nd;
    for (int d = 0; d < nd; ++d) P->st_off[d] = st.off[d];
}

static StencilOffs stencil_of(const tp_prec* P) {
    StencilOffs st{};
    for (int d = 0; d < 8; ++d) st.off[d] = P->st_off[d];
    return st;
}

// rhs - M x written in the storage precision of h's level-0 right-hand side
static void sub_into_b(const tp_prec* P, const double* M, const double* x, const double* rhs, tp_amg* h,
                       hipStream_t s) {
    const tp_jacobian& J = P->J;
    const int32_t n = J.n;
    const int grid = cdiv((int64_t)n * JG, KB);
    const bool f32 = storage_bytes(h) == 4;
    if (P->st_nd == 7 || P->st_nd == 5) {
        const int gs = cdiv(n, ST_ROWS);
        const StencilOffs st = stencil_of(P);
        if (P->st_nd == 7 && f32)
            TP_LAUNCH((k_spmv_sub_st<float, 7>), gs, ST_ROWS, 0, s, n, J.rowptr, J.col, M, x, rhs,
                      (float*)h->lev[0].b.p, st);
        else if (P->st_nd == 7)
            TP_LAUNCH((k_spmv_sub_st<double, 7>), gs, ST_ROWS, 0, s, n, J.rowptr, J.col, M, x, rhs,
                      (double*)h->lev[0].b.p, st);
        else if (f32)
            TP_LAUNCH((k_spmv_sub_st<float, 5>), gs, ST_ROWS, 0, s, n, J.rowptr, J.col, M, x, rhs,
                      (float*)h->lev[0].b.p, st);
        else
            TP_LAUNCH((k_spmv_sub_st<double, 5>), gs, ST_ROWS, 0, s, n, J.rowptr, J.col, M, x, rhs,
                      (double*)h->lev[0].b.p, st);
        return;
    }
    if (f32)
        TP_LAUNCH(k_spmv_sub<float>, grid, KB, 0, s, n, J.rowptr, J.col, M, x, rhs, (float*)h->lev[0].b.p);
    else
        TP_LAUNCH(k_spmv_sub<double>, grid, KB, 0, s, n, J.rowptr, J.col, M, x, rhs, (double*)h->lev[0].b.p);
}

// w = J z (or b - J z), zcopy <- z when given; the implied-column form when J
// is the handle's own Jacobian and its stencil was found
static void block_spmv(const tp_jacobian& J, const tp_prec* P, const double* z, const double* b, double* w,
                       double* zcopy, hipStream_t s) {
    const int32_t n = J.n;
    const bool own = J.rowptr == P->J.rowptr && J.col == P->J.col;
    if (own && (P->st_nd == 7 || P->st_nd == 5)) {
        const int gs = cdiv(n, ST_ROWS);
        if (P->st_nd == 7)
            TP_LAUNCH(k_block_spmv_st<7>, gs, ST_ROWS, 0, s, n, J.rowptr, J.col, J.pp, J.pT, J.Tp, J.TT, z, b, w,
                      zcopy, stencil_of(P));
        else
            TP_LAUNCH(k_block_spmv_st<5>, gs, ST_ROWS, 0, s, n, J.rowptr, J.col, J.pp, J.pT, J.Tp, J.TT, z, b, w,
                      zcopy, stencil_of(P));
        return;
    }
    TP_LAUNCH(k_block_spmv, cdiv((int64_t)n * JG, KB), KB, 0, s, n, J.rowptr, J.col, J.pp, J.pT, J.Tp, J.TT, z, b,
              w, zcopy);
}

static void run_from_b(tp_amg* h, double* out, int32_t n, hipStream_t s) {
    const size_t es = storage_bytes(h);
    const void* x = vcycle_run(h, nullptr, s, es == 8 ? out : nullptr);
    if (x != out) cast_s2d(n, x, out, es, s);
}

// work vectors of the CPR form, allocated outside any capture, and the
// stencil examined
static void prec_buffers(tp_prec* M, hipStream_t s) {
    const int32_t n = M->J.n;
    if (!M->st_done) stencil_detect(M, s);
    if (M->variant == 3 && M->cw.n != (size_t)n) {
        M->cw.alloc(n, s);
        M->cb.alloc(2 * (size_t)n, s);
    }
}

// cw, cb: CPR work vectors (n and 2n); null takes the handle's own
void prec_apply_split(tp_prec* M, const double* r, double* z, hipStream_t s, double* cw = nullptr,
                      double* cb = nullptr) {
    const int32_t n = M->J.n;
    const double* rp = r;
    const double* rT = r + n;
    double* zp = z;
    double* zT = z + n;
    if (M->variant == 3) {
        if (!cw) cw = M->cw.p;
        if (!cb) cb = M->cb.p;
        vsolve(M->pp, rp, cw, n, s);  // stage 1: x1 = V_pp(r_p)
        TP_LAUNCH(k_cpr_resid, cdiv((int64_t)n * JG, KB), KB, 0, s, n, M->J.rowptr, M->J.col, M->J.pp, M->J.Tp,
                  cw, r, cb);
        ilu_solve(M->ilu, cb, z, s);  // stage 2
        TP_LAUNCH(k_add_into, cdiv(n, KB), KB, 0, s, n, cw, z);
        return;
    }
    if (M->variant == 1) {
        vsolve(M->S, rT, zT, n, s);
        sub_into_b(M, M->J.pT, zT, rp, M->pp, s);
        run_from_b(M->pp, zp, n, s);
        return;
    }
    vsolve(M->pp, rp, zp, n, s);                 // step 1
    sub_into_b(M, M->J.Tp, zp, rT, M->S, s);  // step 2
    run_from_b(M->S, zT, n, s);                  // step 3
    if (M->variant == 2) {
        sub_into_b(M, M->J.pT, zT, rp, M->pp, s);  // step 4
        run_from_b(M->pp, zp, n, s);                  // step 5
    }
}

// ---- graph of the preconditioner apply -------------------------------------------------------
static void note_stream(tp_prec* M, hipStream_t s) {
    if (M->used && s != M->last) M->multi = true;
    M->last = s;
    M->used = true;
}

// Capture runs on a non-blocking stream of its own (capture is not allowed on
// the legacy null stream that callers often pass): one per host thread and
// device, created on first use and kept for the process lifetime (creating
// and destroying one per preconditioner cost ~0.2 ms a solve).
static hipStream_t capture_stream() {
    int dev = 0;
    TP_HIP(hipGetDevice(&dev));
    thread_local std::vector<hipStream_t> cs;
    if ((int)cs.size() <= dev) cs.resize(dev + 1, nullptr);
    if (!cs[dev]) TP_HIP(hipStreamCreateWithFlags(&cs[dev], hipStreamNonBlocking));
    return cs[dev];
}

// (a learned smoother on the pressure hierarchy, which the solver never
// switches off, and the smoother timer keep the apply eager)
static bool graph_usable(tp_prec* M) { return !(M->pp->cnn && M->pp->cnn->enabled) && !timer().on; }

static bool schur_cnn_on(tp_prec* M) { return M->S && M->S->cnn && M->S->cnn->enabled; }

// Graph of prec_apply_split(rin -> zout), with or without the Schur hierarchy's
// learned post-smoother (captured the first time each is needed, the learned one
// again after every new attachment; staging vectors allocated on the solve
// stream s). The instantiated graph is launched on whatever stream the solve
// runs on.
static hipGraphExec_t graph_ensure(tp_prec* M, hipStream_t s, bool with_cnn) {
    hipGraphExec_t& slot = with_cnn ? M->gexec_cnn : M->gexec;
    if (with_cnn && slot && M->gen_cnn != M->S->cnn_gen) {
        TP_HIP(hipDeviceSynchronize());  // a replay of the stale graph may still run
        (void)hipGraphExecDestroy(slot);
        slot = nullptr;
    }
    if (slot) return slot;
    const int32_t n = M->J.n;
    if (M->rin.n != 2 * (size_t)n) {
        M->rin.alloc(2 * (size_t)n, s);
        M->zout.alloc(2 * (size_t)n, s);
    }
    prec_buffers(M, s);
    const hipStream_t c = capture_stream();
    tp_cnn_attach* a = M->S ? M->S->cnn.get() : nullptr;
    const bool was = a && a->enabled;
    if (a) a->enabled = with_cnn;
    hipGraph_t g = nullptr;
    TP_HIP(hipStreamBeginCapture(c, hipStreamCaptureModeThreadLocal));
    try {
        prec_apply_split(M, M->rin.p, M->zout.p, c);
    } catch (...) {
        hipGraph_t junk = nullptr;
        (void)hipStreamEndCapture(c, &junk);
        if (junk) (void)hipGraphDestroy(junk);
        if (a) a->enabled = was;
        throw;
    }
    if (a) a->enabled = was;
    TP_HIP(hipStreamEndCapture(c, &g));
    hipGraphExec_t ex = nullptr;
    hipError_t e = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    TP_HIP(e);
    slot = ex;
    if (with_cnn) M->gen_cnn = M->S->cnn_gen;
    return ex;
}

// ---- FGMRES driver ------------------------------------------------------------------------------
struct Gmres {
    int32_t n;
    int64_t N;
    int m;
    int nb;
    DBuf<double> V, Z, w, b, x, r, H, cs, sn, g, y, h1, h2, nrm2, part, sc;
    DBuf<unsigned int> ticket;
    hipEvent_t ev[2] = {nullptr, nullptr};  // one per mailbox slot (pipelined iterations)
    static HostMail& host_mail() {
        // one pinned mailbox per host thread, kept for the process lifetime
        static thread_local HostMail* box = new HostMail();
        return *box;
    }
    Gmres(int32_t n_, int m_, hipStream_t s) : n(n_), N(2 * (int64_t)n_), m(m_) {
        nb = (int)std::min<int64_t>(512, std::max<int64_t>(1, (N + 2 * CG_T - 1) / (2 * CG_T)));
        V.alloc((size_t)(m + 1) * N, s);
        Z.alloc((size_t)m * N, s);
        w.alloc(N, s);
        b.alloc(N, s);
        x.alloc(N, s);
        r.alloc(N, s);
        H.alloc((size_t)(m + 1) * m, s);
        cs.alloc(m, s);
        sn.alloc(m, s);
        g.alloc(m + 1, s);
        y.alloc(m, s);
        h1.alloc(MAXK + 1, s);
        h2.alloc(MAXK + 1, s);
        nrm2.alloc(1, s);
        part.alloc((size_t)nb * MAXK, s);
        sc.alloc(4, s);
        ticket.alloc(1, s);
        TP_LAUNCH(k_zero_u32, 1, 64, 0, s, ticket.p);
        for (auto& e : ev) TP_HIP(hipEventCreateWithFlags(&e, hipEventDisableTiming));
    }
    ~Gmres() {
        for (auto& e : ev)
            if (e) (void)hipEventDestroy(e);
    }
    // after the device work on the buffers has finished: free them on the
    // null stream later (the stream they were allocated on may be gone)
    void detach_streams() {
        for (DBuf<double>* q : {&V, &Z, &w, &b, &x, &r, &H, &cs, &sn, &g, &y, &h1, &h2, &nrm2, &part, &sc}) q->s = nullptr;
        ticket.s = nullptr;
    }
};

// Idle workspaces, kept per device for the next preconditioner of the same
// size: a Newton loop creates a preconditioner per iteration, and allocating
// the Krylov basis anew each time (4 GB at 8.4M unknowns) is slow.  A
// workspace enters the list only after its handle's streams have drained.
constexpr size_t WS_KEEP = 2;  // per device
static std::mutex g_ws_mu;
static std::vector<std::pair<int, Gmres*>> g_ws;

static Gmres* ws_take(int32_t n, int m) {
    std::lock_guard<std::mutex> lk(g_ws_mu);
    const int dev = current_device();
    for (size_t i = 0; i < g_ws.size(); ++i)
        if (g_ws[i].first == dev && g_ws[i].second->n == n && g_ws[i].second->m == m) {
            Gmres* g = g_ws[i].second;
            g_ws.erase(g_ws.begin() + i);
            return g;
        }
    return nullptr;
}

void ws_give(Gmres* g) {
    if (!g) return;
    g->detach_streams();
    std::lock_guard<std::mutex> lk(g_ws_mu);
    const int dev = current_device();
    size_t held = 0;
    for (auto& e : g_ws) held += e.first == dev;
    if (held >= WS_KEEP) {  // drop the oldest of this device
        for (size_t i = 0; i < g_ws.size(); ++i)
            if (g_ws[i].first == dev) {
                delete g_ws[i].second;
                g_ws.erase(g_ws.begin() + i);
                break;
            }
    }
    g_ws.emplace_back(dev, g);
}

void release_ws_cache() {
    std::lock_guard<std::mutex> lk(g_ws_mu);
    for (auto& e : g_ws) delete e.second;
    g_ws.clear();
}

static void dots(Gmres& G, int k, const double* h, double* w, int mode, double* out, hipStream_t s,
                 int arn = 0, int j = 0) {
    ArnoldiArgs aa{j, G.m, G.h1.p, G.h2.p, G.H.p, G.cs.p, G.sn.p, G.g.p, G.sc.p};
#define TP_CGS_CASE(KK)                                                                                 \
    case KK:                                                                                            \
        TP_LAUNCH(k_cgs<KK>, G.nb, CG_T, 0, s, G.N, G.V.p, h, w, mode, G.part.p);                       \
        break;
    switch (k) {
        TP_CGS_CASE(0) TP_CGS_CASE(1) TP_CGS_CASE(2) TP_CGS_CASE(3) TP_CGS_CASE(4) TP_CGS_CASE(5)
        TP_CGS_CASE(6) TP_CGS_CASE(7) TP_CGS_CASE(8) TP_CGS_CASE(9) TP_CGS_CASE(10) TP_CGS_CASE(11)
        TP_CGS_CASE(12) TP_CGS_CASE(13) TP_CGS_CASE(14) TP_CGS_CASE(15) TP_CGS_CASE(16) TP_CGS_CASE(17)
        TP_CGS_CASE(18) TP_CGS_CASE(19) TP_CGS_CASE(20) TP_CGS_CASE(21) TP_CGS_CASE(22) TP_CGS_CASE(23)
        TP_CGS_CASE(24) TP_CGS_CASE(25) TP_CGS_CASE(26) TP_CGS_CASE(27) TP_CGS_CASE(28) TP_CGS_CASE(29)
        TP_CGS_CASE(30) TP_CGS_CASE(31)
    default: fail(TP_ERR_ARG, "basis size %d exceeds %d", k, MAXK - 1);
    }
#undef TP_CGS_CASE
    TP_LAUNCH(k_cgs_finish, 1, FIN_T, 0, s, G.nb, mode == 2 ? 1 : k, G.part.p, out, arn, aa);
}

static double read_d(const double* dptr, HostMail& mail, hipStream_t s) {
    TP_HIP(hipMemcpyAsync(mail.p, dptr, sizeof(double), hipMemcpyDeviceToHost, s));
    TP_HIP(hipStreamSynchronize(s));
    return *mail.as<double>();
}

void gmres_free(Gmres* g) { ws_give(g); }

static int fgmres(const tp_jacobian& J, tp_prec* M, const double* b_il, double* x_il,
                  const tp_krylov_params& kp, tp_krylov_stats* st, double* history, hipStream_t s) {
    const int32_t n = J.n;
    const int m = kp.restart;
    note_stream(M, s);
    prec_buffers(M, s);
    if (!M->ws || M->ws->n != n || M->ws->m != m) {
        if (M->ws) {
            TP_HIP(hipDeviceSynchronize());
            ws_give(M->ws);
            M->ws = nullptr;
        }
        M->ws = ws_take(n, m);
        if (!M->ws) M->ws = new Gmres(n, m, s);
    }
    Gmres& G = *M->ws;
    HostMail& mail = Gmres::host_mail();  // the calling thread's pinned mailbox
    const int gn = cdiv(n, KB);
    const int gN = cdiv(G.N, KB);
    TP_LAUNCH(k_deinterleave, gn, KB, 0, s, n, b_il, G.b.p);
    TP_LAUNCH(k_deinterleave, gn, KB, 0, s, n, x_il, G.x.p);
    dots(G, 0, nullptr, G.b.p, 2, G.nrm2.p, s);
    const double bnorm = std::sqrt(read_d(G.nrm2.p, mail, s));
    // the stopping test on relative quantities: ||r|| <= max(rtol ||b||, atol)
    const double tol = bnorm > 0.0 ? std::max(kp.rtol, kp.atol / bnorm) : kp.rtol;
    int it = 0, restarts = 0;
    double rel = 0.0, est = 0.0;
    std::vector<double> ests;
    bool cnn_on = schur_cnn_on(M);
    int fallback_iter = -1;
    bool floor_hit = false;
    if (cnn_on) TP_LAUNCH(k_zero_i32, 1, 64, 0, s, M->S->cnn->bad.p);
    int status = TP_OK;
    if (bnorm == 0.0) {
        TP_LAUNCH(k_zero_d, gN, KB, 0, s, G.N, G.x.p);
        if (history) history[0] = 0.0;
        rel = est = 0.0;
    } else {
        block_spmv(J, M, G.x.p, G.b.p, G.r.p, nullptr, s);
        dots(G, 0, nullptr, G.r.p, 2, G.nrm2.p, s);
        rel = std::sqrt(read_d(G.nrm2.p, mail, s)) / bnorm;
        est = rel;
        if (history) history[0] = rel;
        double prev_rel = rel;
        while (rel > tol && it < kp.maxit) {
            if (!std::isfinite(rel)) fail(TP_ERR_NUMERIC, "non-finite residual in FGMRES");
            // v_0 = r / beta (nrm2 holds ||r||^2)
            const bool use_graph = kp.graph != 0 && graph_usable(M);
            if (use_graph) graph_ensure(M, s, cnn_on);
            TP_LAUNCH(k_cycle_init, 1, 1, 0, s, m, G.nrm2.p, G.g.p, G.sc.p);
            TP_LAUNCH(k_scale_div, gN, KB, 0, s, G.N, G.r.p, G.sc.p, G.V.p, use_graph ? M->rin.p : nullptr,
                      (const int32_t*)nullptr, (double*)nullptr);
            // Arnoldi step j: z_j = M^{-1} v_j, w = J z_j, CGS2 against v_0..v_j, Givens on
            // column j, v_{j+1} = w / h_{j+1,j}; (h_{j+1,j}, |g_{j+1}|, the learned smoother's
            // failure flag) go to mailbox slot `slot`
            auto enqueue = [&](int j, int slot) {
                double* vj = G.V.p + (int64_t)j * G.N;
                double* zj = G.Z.p + (int64_t)j * G.N;
                if (use_graph) {
                    // rin already holds v_j; the product kernel copies zout into Z_j
                    TP_HIP(hipGraphLaunch(graph_ensure(M, s, cnn_on), s));
                    block_spmv(J, M, M->zout.p, nullptr, G.w.p, zj, s);
                } else {
                    prec_apply_split(M, vj, zj, s);
                    block_spmv(J, M, zj, nullptr, G.w.p, nullptr, s);
                }
                dots(G, j + 1, nullptr, G.w.p, 0, G.h1.p, s);
                dots(G, j + 1, G.h1.p, G.w.p, 1, G.h2.p, s);
                dots(G, j + 1, G.h2.p, G.w.p, 2, G.nrm2.p, s, 1, j);
                TP_LAUNCH(k_scale_div, gN, KB, 0, s, G.N, G.w.p, G.sc.p, G.V.p + (int64_t)(j + 1) * G.N,
                          use_graph ? M->rin.p : nullptr, cnn_on ? (const int32_t*)M->S->cnn->bad.p : nullptr,
                          G.sc.p + 2);
                TP_HIP(hipMemcpyAsync(mail.as<double>() + 4 * slot, G.sc.p, 3 * sizeof(double),
                                      hipMemcpyDeviceToHost, s));
                TP_HIP(hipEventRecord(G.ev[slot], s));
            };
            // Step j+1 is queued before the host waits for step j's values, so the
            // device never idles on the host's check. If step j ends the cycle, step
            // j+1 has only written column j+1 of H, V_{j+2}, Z_{j+1} and the rotation
            // j+1 (g_{j+1}, g_{j+2}); the update below uses columns 0..j and g_0..g_j,
            // so it is discarded. When the host switches the learned smoother off
            // after step j, step j+1 has already run with it: FGMRES keeps each
            // step's own z, so a preconditioner that changes between steps is valid.
            const bool pipelined = true;
            int k = 0;
            if (it < kp.maxit) enqueue(0, 0);
            for (int j = 0; j < m && it < kp.maxit; ++j) {
                const int slot = j & 1;
                // no step ahead when the last two estimates' ratio predicts that
                // step j already meets the tolerance (the step would be wasted)
                const size_t q = ests.size();
                const bool likely_last =
                    q >= 2 && ests[q - 2] > 0.0 && ests[q - 1] * (ests[q - 1] / ests[q - 2]) <= tol;
                const bool ahead = pipelined && !likely_last && j + 1 < m && it + 1 < kp.maxit;
                if (ahead) enqueue(j + 1, slot ^ 1);
                TP_HIP(hipEventSynchronize(G.ev[slot]));
                const double hn = mail.as<double>()[4 * slot];
                est = mail.as<double>()[4 * slot + 1] / bnorm;
                const bool bad = mail.as<double>()[4 * slot + 2] != 0.0;
                ++it;
                k = j + 1;
                if (history) history[it] = est;
                ests.push_back(est);
                if (cnn_on) {
                    tp_cnn_attach* a = M->S->cnn.get();
                    const size_t q = ests.size();
                    const size_t w = kp.stag_window > 0 ? (size_t)kp.stag_window : 2;
                    const bool stag = kp.stag_ratio > 0.0 && q >= w + 1 && ests[q - 1] > kp.stag_ratio * ests[q - 1 - w];
                    const bool slow = kp.ref_rate > 0.0 && q >= 4 && ests[q - 1] > std::pow(kp.ref_rate, (double)q);
                    if (bad || stag || slow) {
                        a->enabled = false;
                        cnn_on = false;
                        fallback_iter = it;
                    }
                }
                if (!std::isfinite(est)) fail(TP_ERR_NUMERIC, "non-finite Arnoldi value in FGMRES");
                if (est <= tol || hn == 0.0) break;
                if (!ahead && j + 1 < m && it < kp.maxit) enqueue(j + 1, slot ^ 1);
            }
            TP_LAUNCH(k_hess_solve, 1, 1, 0, s, k, m, G.H.p, G.g.p, G.y.p);
            TP_LAUNCH(k_xupdate, gN, KB, 0, s, G.N, k, G.Z.p, G.y.p, G.x.p);
            block_spmv(J, M, G.x.p, G.b.p, G.r.p, nullptr, s);
            dots(G, 0, nullptr, G.r.p, 2, G.nrm2.p, s);
            rel = std::sqrt(read_d(G.nrm2.p, mail, s)) / bnorm;
            ++restarts;
            // The cycle's estimate met the tolerance but the true residual
            // neither did nor fell by half since the previous cycle: it sits
            // at the rounding floor of the FP64 product b - J x (small ||b||
            // against ||J|| ||x||, e.g. a nearly converged Newton residual),
            // and further cycles repeat the same correction.  Stop there.
            if (est <= tol && rel > tol && rel > 0.5 * prev_rel) {
                floor_hit = true;
                break;
            }
            prev_rel = rel;
        }
    }
    TP_LAUNCH(k_interleave, gn, KB, 0, s, n, G.x.p, x_il);
    TP_HIP(hipStreamSynchronize(s));
    if (!std::isfinite(rel)) fail(TP_ERR_NUMERIC, "non-finite true residual in FGMRES");
    if (M->S && M->S->cnn) M->S->cnn->enabled = true;  // the switch lasts for one solve
    if (st) {
        st->fallback_iter = fallback_iter;
        st->iters = it;
        st->restarts = restarts > 0 ? restarts - 1 : 0;
        st->rel_true = rel;
        st->rel_est = est;
    }
    status = rel <= tol ? TP_OK : TP_NOT_CONVERGED;
    if (status != TP_OK) {
        if (floor_hit)
            set_error("FGMRES: true relative residual stalled at %.3e above the tolerance %.3e after %d "
                      "iterations (rounding floor of b - J x)", rel, tol, it);
        else
            set_error("FGMRES reached maxit=%d with relative residual %.3e", kp.maxit, rel);
    }
    return status;
}

// ---- allocation-free apply: fixed device scratch ---------------------------------------
// precond_apply_noalloc keeps its work vectors (the split right-hand side and
// result, 2n + 2n doubles, and for CPR the first-stage pressure and residual,
// n + 2n) in this array instead of buffers the library allocates: 256 MiB,
// enough for 4.79M cells (the 256 x 256 x 64 grid's 4.19M fit).  Each device
// holds its own copy for the life of the process.  In host code the name is
// a host-side stand-in: device code reaches the array only through the
// address hipGetSymbolAddress returns for the current device (kept below).
constexpr size_t SCRATCH_DOUBLES = (size_t)32 << 20;
__device__ __align__(256) double scratch[SCRATCH_DOUBLES];

constexpr int SCRATCH_MAX_DEV = 64;
static double* g_scratch[SCRATCH_MAX_DEV] = {nullptr};

// The current device's copy of `scratch` (resolved once per device, with
// that device current; tp_init calls it, the entry point too on a device
// tp_init has not seen).
double* scratch_ptr() {
    int dev = 0;
    TP_HIP(hipGetDevice(&dev));
    TP_CHECK_ARG(dev >= 0 && dev < SCRATCH_MAX_DEV, "device %d beyond the scratch table", dev);
    if (!g_scratch[dev]) {
        void* p = nullptr;
        TP_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
        g_scratch[dev] = static_cast<double*>(p);
    }
    return g_scratch[dev];
}

}  // namespace tp


extern "C" {

int precond_create(const tp_jacobian* J, tp_amg_t amg_pp, tp_amg_t amg_S, int32_t variant, tp_prec_t* out) {
    TP_GUARD({
        TP_CHECK_ARG(J && amg_pp && amg_S && out, "precond_create: null argument");
        TP_CHECK_ARG(variant >= 0 && variant <= 2, "precond_create: variant must be 0, 1 or 2");
        TP_CHECK_ARG(J->rowptr && J->col && J->pp && J->pT && J->Tp && J->TT, "precond_create: null Jacobian array");
        TP_CHECK_ARG(amg_pp->lev[0].A.n == J->n && amg_S->lev[0].A.n == J->n,
                     "precond_create: hierarchy size does not match J->n");
        tp_prec* M = new tp_prec();
        M->J = *J;
        M->pp = amg_pp;
        M->S = amg_S;
        M->variant = variant;
        *out = M;
    });
    return TP_OK;
}

int precond_create_cpr(const tp_jacobian* J, tp_amg_t amg_pp, tp_ilu_t ilu, tp_prec_t* out) {
    TP_GUARD({
        TP_CHECK_ARG(J && amg_pp && ilu && out, "precond_create_cpr: null argument");
        TP_CHECK_ARG(J->rowptr && J->col && J->pp && J->pT && J->Tp && J->TT, "precond_create_cpr: null Jacobian array");
        TP_CHECK_ARG(amg_pp->lev[0].A.n == J->n, "precond_create_cpr: hierarchy size does not match J->n");
        TP_CHECK_ARG(tp::ilu_cells(ilu) == J->n,
                     "precond_create_cpr: the ILU(0) handle was not built from a Jacobian of this size");
        tp_prec* M = new tp_prec();
        M->J = *J;
        M->pp = amg_pp;
        M->ilu = ilu;
        M->variant = 3;
        *out = M;
    });
    return TP_OK;
}

int precond_apply(tp_prec_t M, const double* r, double* z, void* stream) {
    TP_GUARD({
        TP_CHECK_ARG(M && r && z, "precond_apply: null argument");
        hipStream_t s = (hipStream_t)stream;
        const int32_t n = M->J.n;
        tp::note_stream(M, s);
        tp::prec_buffers(M, s);
        if (tp::graph_usable(M)) {
            hipGraphExec_t ex = tp::graph_ensure(M, s, tp::schur_cnn_on(M));
            TP_LAUNCH(tp::k_deinterleave, tp::cdiv(n, tp::KB), tp::KB, 0, s, n, r, M->rin.p);
            TP_HIP(hipGraphLaunch(ex, s));
            TP_LAUNCH(tp::k_interleave, tp::cdiv(n, tp::KB), tp::KB, 0, s, n, M->zout.p, z);
        } else {
            if (M->rs.n != (size_t)2 * n) {
                M->rs.alloc(2 * (size_t)n, s);
                M->zs.alloc(2 * (size_t)n, s);
            }
            TP_LAUNCH(tp::k_deinterleave, tp::cdiv(n, tp::KB), tp::KB, 0, s, n, r, M->rs.p);
            tp::prec_apply_split(M, M->rs.p, M->zs.p, s);
            TP_LAUNCH(tp::k_interleave, tp::cdiv(n, tp::KB), tp::KB, 0, s, n, M->zs.p, z);
        }
    });
    return TP_OK;
}

int precond_apply_noalloc(tp_prec_t M, const double* r, double* z, void* stream) {
    TP_GUARD({
        TP_CHECK_ARG(M && r && z, "precond_apply_noalloc: null argument");
        TP_CHECK_ARG(!tp::timer().on, "precond_apply_noalloc: the smoother timer is on (it records events)");
        hipStream_t s = (hipStream_t)stream;
        const int32_t n = M->J.n;
        const size_t need = 4 * (size_t)n + (M->variant == 3 ? 3 * (size_t)n : 0);
        if (need > tp::SCRATCH_DOUBLES)
            tp::fail(TP_ERR_CAPACITY,
                     "precond_apply_noalloc: %zu doubles of work space needed, the fixed scratch holds %zu "
                     "(n = %d cells; at most %zu cells, %zu for CPR)",
                     need, tp::SCRATCH_DOUBLES, n, tp::SCRATCH_DOUBLES / 4, tp::SCRATCH_DOUBLES / 7);
        double* w = tp::scratch_ptr();
        double* rs = w;
        double* zs = w + 2 * (size_t)n;
        double* cw = M->variant == 3 ? w + 4 * (size_t)n : nullptr;
        double* cb = M->variant == 3 ? w + 5 * (size_t)n : nullptr;
        tp::note_stream(M, s);
        TP_LAUNCH(tp::k_deinterleave, tp::cdiv(n, tp::KB), tp::KB, 0, s, n, r, rs);
        tp::prec_apply_split(M, rs, zs, s, cw, cb);
        TP_LAUNCH(tp::k_interleave, tp::cdiv(n, tp::KB), tp::KB, 0, s, n, zs, z);
    });
    return TP_OK;
}

int precond_destroy(tp_prec_t M) {
    TP_GUARD({
        if (M) {
            // work of this handle may still run on the streams it was used on
            if (M->multi) TP_HIP(hipDeviceSynchronize());
            else if (M->used) TP_HIP(hipStreamSynchronize(M->last));
            tp::gmres_free(M->ws);
            if (M->gexec) (void)hipGraphExecDestroy(M->gexec);
            if (M->gexec_cnn) (void)hipGraphExecDestroy(M->gexec_cnn);
            delete M;
        }
    });
    return TP_OK;
}

int fgmres_solve(const tp_jacobian* J, tp_prec_t M, const double* b, double* x,
                 const tp_krylov_params* params, tp_krylov_stats* stats, double* history, void* stream) {
    TP_GUARD({
        TP_CHECK_ARG(J && M && b && x && params, "fgmres_solve: null argument");
        TP_CHECK_ARG(params->restart >= 1 && params->restart <= tp::MAXK - 1,
                     "fgmres_solve: restart must be in [1,%d]", tp::MAXK - 1);
        TP_CHECK_ARG(params->maxit >= 0, "fgmres_solve: maxit must be >= 0");
        TP_CHECK_ARG(params->rtol >= 0.0, "fgmres_solve: rtol must be >= 0");
        TP_CHECK_ARG(params->atol >= 0.0, "fgmres_solve: atol must be >= 0");
        TP_CHECK_ARG(params->stag_window >= 0 && params->stag_window <= 16, "fgmres_solve: stag_window must be in [0,16]");
        TP_CHECK_ARG(params->ref_rate >= 0.0 && params->ref_rate < 1.0, "fgmres_solve: ref_rate must be in [0,1)");
        TP_CHECK_ARG(J->n == M->J.n, "fgmres_solve: J and preconditioner sizes differ");
        return tp::fgmres(*J, M, b, x, *params, stats, history, (hipStream_t)stream);
    });
    return TP_OK;
}

}  // extern "C"
