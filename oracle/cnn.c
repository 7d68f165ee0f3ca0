/*
 * cnn.c -- oracle for the learned post-smoother network.
 *
 * TEST INFRASTRUCTURE ONLY (see tp_oracle.h).  Plain FP64 loops.
 *
 * The network (a method pattern built on top of the paper's V-cycle; the
 * paper itself has no learned component): on the nx x ny x nz cell grid,
 *   h_o(i)  = b1_o + sum_c sum_t W1[o][c][t] f_c(i + t)      (8 -> 16 channels)
 *   a_o(i)  = max(h_o(i), 0)
 *   out(i)  = b2 + sum_o sum_t W2[o][t] a_o(i + t)          (16 -> 1 channel)
 * with t running over the 27 offsets of a 3x3x3 neighbourhood, tap index
 * t = (dz+1)*9 + (dy+1)*3 + (dx+1), and zero padding outside the grid.
 * Loss = mean_i (out(i) - y(i))^2.  The backward pass is the chain rule of
 * these sums written out.
 */
#include "tp_oracle.h"
#include <stdlib.h>
#include <string.h>

#define CIN 8
#define CH 16
#define NT 27

static int32_t nbr(const or_grid* g, int32_t i, int t)
{
    int dz = t / 9 - 1, dy = (t / 3) % 3 - 1, dx = t % 3 - 1;
    int32_t ix = i % g->nx + dx, iy = (i / g->nx) % g->ny + dy, iz = i / (g->nx * g->ny) + dz;
    if (ix < 0 || iy < 0 || iz < 0 || ix >= g->nx || iy >= g->ny || iz >= g->nz) return -1;
    return ix + g->nx * (iy + g->ny * iz);
}

/* h (CH x n) pre-activation, out (n) */
void or_cnn_forward(const or_grid* g, const double* W1, const double* b1, const double* W2,
                    double b2, const double* f, double* h, double* out)
{
    int32_t n = g->nx * g->ny * g->nz;
    for (int o = 0; o < CH; ++o)
        for (int32_t i = 0; i < n; ++i) {
            double s = b1[o];
            for (int c = 0; c < CIN; ++c)
                for (int t = 0; t < NT; ++t) {
                    int32_t j = nbr(g, i, t);
                    if (j >= 0) s += W1[(o * CIN + c) * NT + t] * f[(size_t)c * n + j];
                }
            h[(size_t)o * n + i] = s;
        }
    for (int32_t i = 0; i < n; ++i) {
        double s = b2;
        for (int o = 0; o < CH; ++o)
            for (int t = 0; t < NT; ++t) {
                int32_t j = nbr(g, i, t);
                if (j >= 0) {
                    double a = h[(size_t)o * n + j];
                    s += W2[o * NT + t] * (a > 0.0 ? a : 0.0);
                }
            }
        out[i] = s;
    }
}

/* loss and gradients for target y; grads laid out W1 (3456), b1 (16), W2 (432), b2 (1) */
double or_cnn_backward(const or_grid* g, const double* W1, const double* b1, const double* W2,
                       double b2, const double* f, const double* y, double* grad)
{
    int32_t n = g->nx * g->ny * g->nz;
    double* h = malloc(sizeof(double) * (size_t)CH * n);
    double* out = malloc(sizeof(double) * (size_t)n);
    double* dout = malloc(sizeof(double) * (size_t)n);
    double* dh = malloc(sizeof(double) * (size_t)CH * n);
    or_cnn_forward(g, W1, b1, W2, b2, f, h, out);
    double loss = 0.0;
    for (int32_t i = 0; i < n; ++i) {
        double d = out[i] - y[i];
        loss += d * d;
        dout[i] = 2.0 * d / n;
    }
    loss /= n;
    double* gW1 = grad;
    double* gb1 = grad + CH * CIN * NT;
    double* gW2 = gb1 + CH;
    double* gb2 = gW2 + CH * NT;
    memset(grad, 0, sizeof(double) * (CH * CIN * NT + CH + CH * NT + 1));
    /* layer 2 */
    for (int32_t i = 0; i < n; ++i) {
        gb2[0] += dout[i];
        for (int o = 0; o < CH; ++o)
            for (int t = 0; t < NT; ++t) {
                int32_t j = nbr(g, i, t);
                if (j >= 0) {
                    double a = h[(size_t)o * n + j];
                    gW2[o * NT + t] += dout[i] * (a > 0.0 ? a : 0.0);
                }
            }
    }
    /* dL/da_o(j) = sum over i with j = i + t of W2[o][t] dout(i); then ReLU mask */
    for (int o = 0; o < CH; ++o)
        for (int32_t j = 0; j < n; ++j) {
            double s = 0.0;
            for (int t = 0; t < NT; ++t) {
                int32_t i = nbr(g, j, NT - 1 - t);   /* i = j - offset(t) */
                if (i >= 0) s += W2[o * NT + t] * dout[i];
            }
            dh[(size_t)o * n + j] = h[(size_t)o * n + j] > 0.0 ? s : 0.0;
        }
    /* layer 1 */
    for (int o = 0; o < CH; ++o)
        for (int32_t i = 0; i < n; ++i) {
            double d = dh[(size_t)o * n + i];
            gb1[o] += d;
            for (int c = 0; c < CIN; ++c)
                for (int t = 0; t < NT; ++t) {
                    int32_t j = nbr(g, i, t);
                    if (j >= 0) gW1[(o * CIN + c) * NT + t] += d * f[(size_t)c * n + j];
                }
        }
    free(h); free(out); free(dout); free(dh);
    return loss;
}

/* Input features on the finest level of the Schur-approximation hierarchy
 * (a stencil matrix on the grid) for residual r:
 *   ch0 = (D^{-1} r)_i / s,  s = sqrt(mean_i (D^{-1} r)_i^2),  D_ii = sum_j |a_ij|
 *   ch1..ch6 = a_{i,j} / a_ii for the -x, +x, -y, +y, -z, +z neighbour (0 off-grid)
 *   ch7 = a_ii / D_ii
 * Returns s. */
double or_cnn_features(const or_grid* g, const int32_t* rowptr, const int32_t* col,
                       const double* val, const double* r, double* f)
{
    int32_t n = g->nx * g->ny * g->nz, nxy = g->nx * g->ny;
    double ss = 0.0;
    double* z = malloc(sizeof(double) * (size_t)n);
    for (int32_t i = 0; i < n; ++i) {
        double d = 0.0, aii = 0.0;
        for (int32_t k = rowptr[i]; k < rowptr[i + 1]; ++k) {
            d += val[k] < 0.0 ? -val[k] : val[k];
            if (col[k] == i) aii = val[k];
        }
        z[i] = r[i] / d;
        ss += z[i] * z[i];
        const int32_t off[6] = {-1, 1, -g->nx, g->nx, -nxy, nxy};
        int32_t ix = i % g->nx, iy = (i / g->nx) % g->ny, iz = i / nxy;
        const int ok[6] = {ix > 0, ix < g->nx - 1, iy > 0, iy < g->ny - 1, iz > 0, iz < g->nz - 1};
        for (int q = 0; q < 6; ++q) {
            double a = 0.0;
            if (ok[q])
                for (int32_t k = rowptr[i]; k < rowptr[i + 1]; ++k)
                    if (col[k] == i + off[q]) a = val[k];
            f[(size_t)(1 + q) * n + i] = a / aii;
        }
        f[(size_t)7 * n + i] = aii / d;
    }
    double s = n > 0 ? __builtin_sqrt(ss / n) : 0.0;
    for (int32_t i = 0; i < n; ++i) f[i] = s > 0.0 ? z[i] / s : 0.0;
    free(z);
    return s;
}
