// tp_cnn.hip -- learned post-smoother: a two-layer 3-D convolutional network
// applied on the finest level of the Schur-approximation hierarchy.
//
// Network (zero padding, 27-point 3x3x3 taps, tap t = (dz+1)*9 + (dy+1)*3 + (dx+1)):
//   h_o(i) = b1_o + sum_{c<8} sum_t W1[o][c][t] f_c(i + t)      (16 outputs)
//   out(i) = b2 + sum_{o<16} sum_t W2[o][t] max(h_o(i + t), 0)
// Inputs per cell: f_0 = (D^{-1} r)_i / s with s = RMS(D^{-1} r) and D the
// l1 diagonal, f_1..f_6 = a_{i,nbr}/a_ii (-x,+x,-y,+y,-z,+z), f_7 = a_ii/D_ii.
// The smoother update is x <- x + s * out.  Weights are stored in BF16 and
// features rounded to BF16; products accumulate in FP32 (the hidden
// activations stay FP32).  A FP32 master copy
// of the weights is kept for training (Adam).  All reductions (scale,
// loss, gradients) use a fixed assignment of cells to threads and a fixed
// combination order: results are run-to-run deterministic.
#include "tp_cnn.h"

#include <cmath>

namespace tp {

constexpr int CB = 256;

__device__ inline float bf16_round(float x) {
    // round to nearest even on the upper 16 bits (finite inputs)
    uint32_t u = __float_as_uint(x);
    uint32_t lsb = (u >> 16) & 1u;
    u += 0x7FFFu + lsb;
    return __uint_as_float(u & 0xFFFF0000u);
}

__device__ inline int32_t tap_nbr(int32_t ix, int32_t iy, int32_t iz, int t, int32_t nx, int32_t ny,
                                  int32_t nz) {
    int dz = t / 9 - 1, dy = (t / 3) % 3 - 1, dx = t % 3 - 1;
    int32_t x = ix + dx, y = iy + dy, z = iz + dz;
    if (x < 0 || y < 0 || z < 0 || x >= nx || y >= ny || z >= nz) return -1;
    return x + nx * (y + ny * z);
}

// ---- features -----------------------------------------------------------------------
// static channels 1..7 from the stencil matrix (FP64 CSR)
__global__ void __launch_bounds__(CB)
k_feat_static(tp_grid g, const int32_t* __restrict__ rowptr, const int32_t* __restrict__ col,
              const double* __restrict__ val, float* __restrict__ f, float* __restrict__ dinv) {
    const int32_t n = g.nx * g.ny * g.nz, nxy = g.nx * g.ny;
    const int32_t i = blockIdx.x * CB + threadIdx.x;
    if (i >= n) return;
    double d = 0.0, aii = 0.0;
    for (int32_t k = rowptr[i]; k < rowptr[i + 1]; ++k) {
        d += fabs(val[k]);
        if (col[k] == i) aii = val[k];
    }
    const int32_t ix = i % g.nx, iy = (i / g.nx) % g.ny, iz = i / nxy;
    const int32_t off[6] = {-1, 1, -g.nx, g.nx, -nxy, nxy};
    const bool ok[6] = {ix > 0, ix < g.nx - 1, iy > 0, iy < g.ny - 1, iz > 0, iz < g.nz - 1};
    for (int q = 0; q < 6; ++q) {
        double a = 0.0;
        if (ok[q])
            for (int32_t k = rowptr[i]; k < rowptr[i + 1]; ++k)
                if (col[k] == i + off[q]) a = val[k];
        f[(int64_t)(1 + q) * n + i] = (float)(a / aii);
    }
    f[(int64_t)7 * n + i] = (float)(aii / d);
    dinv[i] = (float)(1.0 / d);
}

// z = D^{-1} r into channel 0 (unscaled); per-block partial sums of z^2
template <typename T>
__global__ void __launch_bounds__(CB)
k_feat_resid(int32_t n, const T* __restrict__ r, const float* __restrict__ dinv, float* __restrict__ f0,
             double* __restrict__ part) {
    __shared__ double sh[CB];
    double acc = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * CB + threadIdx.x; i < n; i += (int64_t)gridDim.x * CB) {
        float z = (float)r[i] * dinv[i];
        f0[i] = z;
        acc += (double)z * (double)z;
    }
    sh[threadIdx.x] = acc;
    __syncthreads();
    for (int off = CB / 2; off > 0; off >>= 1) {
        if (threadIdx.x < off) sh[threadIdx.x] += sh[threadIdx.x + off];
        __syncthreads();
    }
    if (threadIdx.x == 0) part[blockIdx.x] = sh[0];
}

// s = sqrt(sum part / n); f0 /= s  (single block sums the partials, then all scale)
__global__ void __launch_bounds__(CB)
k_feat_scale_sum(int nb, int32_t n, const double* __restrict__ part, float* __restrict__ scale) {
    __shared__ double sh[CB];
    double a = 0.0;
    for (int b = threadIdx.x; b < nb; b += CB) a += part[b];
    sh[threadIdx.x] = a;
    __syncthreads();
    for (int off = CB / 2; off > 0; off >>= 1) {
        if (threadIdx.x < off) sh[threadIdx.x] += sh[threadIdx.x + off];
        __syncthreads();
    }
    if (threadIdx.x == 0) scale[0] = n > 0 ? (float)sqrt(sh[0] / n) : 0.f;
}

__global__ void __launch_bounds__(CB)
k_feat_normalise(int32_t n, const float* __restrict__ scale, float* __restrict__ f0) {
    const int32_t i = blockIdx.x * CB + threadIdx.x;
    if (i >= n) return;
    const float s = scale[0];
    f0[i] = s > 0.f ? f0[i] / s : 0.f;
}

// ---- forward ------------------------------------------------------------------------------
// Layer 1 as an implicit GEMM on the matrix cores: for a row of 16 cells along x,
// H (16 channels x 16 cells) = W1 (16 x 216) * F (216 x 16) + b1 with
// F[k][cell] = bf16(f_c(neighbour t of cell)) (0 off the grid), in seven
// v_mfma_f32_16x16x32_bf16 steps with FP32 accumulation. Lane layout of that
// instruction (16 lanes per group q = lane / 16): A[m][k] at lane m + 16 (k / 8 % 4),
// element k % 8; B[k][n] at lane n + 16 (k / 8 % 4); D[m][n] at lane n + 16 (m / 4),
// element m % 4. The contraction index runs tap-major, k = 8 t + c, so the eight
// values a lane contributes to B are the eight channels of one cell at one tap:
// with the features of the tile and its one-cell halo staged in LDS channel-
// interleaved (16 bytes per cell) each B fragment is a single 16-byte LDS read.
// Group q of K-step st takes tap 4 st + q (tap 27, past the end, contributes 0).
typedef __attribute__((__vector_size__(8 * sizeof(__bf16)))) __bf16 bf16x8;
typedef __attribute__((__vector_size__(4 * sizeof(float)))) float float4v;
constexpr int MF_K = CNN_CIN * CNN_NT;   // 216
constexpr int MF_KS = (MF_K + 31) / 32;  // 7 K-steps of 32
// cell tile of one workgroup (16 x 4 x 4 cells: sixteen 16-cell rows along x)
// and its one-cell halo (zero outside the grid)
constexpr int TX = 16, TY = 4, TZ = 4, HX = TX + 2, HY = TY + 2, HZ = TZ + 2;
constexpr int HCELLS = HX * HY * HZ;
constexpr int MF_T = 256;

__device__ inline int halo_tap(int t) { return ((t / 9) * HY + (t / 3) % 3) * HX + t % 3; }

__global__ void __launch_bounds__(MF_T)
k_cnn_l1(tp_grid g, const float* __restrict__ f, const float* __restrict__ w1, const float* __restrict__ b1,
         float* __restrict__ h) {
    __shared__ bf16x8 s_f[HCELLS];  // [halo cell][channel]
    const int32_t n = g.nx * g.ny * g.nz;
    const int32_t tx = (g.nx + TX - 1) / TX, ty = (g.ny + TY - 1) / TY;
    const int32_t bz = blockIdx.x / (tx * ty), by = (blockIdx.x / tx) % ty, bx = blockIdx.x % tx;
    const int32_t x0 = bx * TX, y0 = by * TY, z0 = bz * TZ;
    for (int r = threadIdx.x; r < HCELLS; r += MF_T) {
        const int hz = r / (HX * HY), hy = (r / HX) % HY, hx = r % HX;
        const int32_t x = x0 + hx - 1, y = y0 + hy - 1, z = z0 + hz - 1;
        const bool in = x >= 0 && y >= 0 && z >= 0 && x < g.nx && y < g.ny && z < g.nz;
        const int64_t cell = x + (int64_t)g.nx * (y + (int64_t)g.ny * z);
        bf16x8 v;
#pragma unroll
        for (int c = 0; c < CNN_CIN; ++c) v[c] = (__bf16)(in ? bf16_round(f[(int64_t)c * n + cell]) : 0.f);
        s_f[r] = v;  // the conversions are exact: BF16 values
    }
    const int lane = threadIdx.x & 63, q = lane >> 4, col = lane & 15, wv = threadIdx.x >> 6;
    bf16x8 a[MF_KS];
    int toff[MF_KS];
#pragma unroll
    for (int st = 0; st < MF_KS; ++st) {
        const int t = 4 * st + q;
#pragma unroll
        for (int c = 0; c < CNN_CIN; ++c)
            a[st][c] = (__bf16)(t < CNN_NT ? w1[col * MF_K + c * CNN_NT + t] : 0.f);  // BF16 values: exact
        toff[st] = t < CNN_NT ? halo_tap(t) : -1;
    }
    float4v bias;
#pragma unroll
    for (int r = 0; r < 4; ++r) bias[r] = b1[4 * q + r];
    __syncthreads();
#pragma unroll 1
    for (int row = wv; row < TY * TZ; row += MF_T / 64) {
        const int ly = row % TY, lz = row / TY;
        const int cb = (lz * HY + ly) * HX + col;
        float4v acc = bias;
#pragma unroll
        for (int st = 0; st < MF_KS; ++st) {
            bf16x8 b = s_f[toff[st] < 0 ? 0 : cb + toff[st]];
            if (toff[st] < 0) b = bf16x8{};  // A is zero there too; keep B finite
            acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[st], b, acc, 0, 0, 0);
        }
        const int32_t x = x0 + col, y = y0 + ly, z = z0 + lz;
        if (x < g.nx && y < g.ny && z < g.nz) {
            const int64_t cell = x + (int64_t)g.nx * (y + (int64_t)g.ny * z);
#pragma unroll
            for (int r = 0; r < 4; ++r) h[(int64_t)(4 * q + r) * n + cell] = acc[r];
        }
    }
}

// Layer 2 (FP32): out = b2 + W2 * relu(h); with x: x += scale * out. relu(h) of the
// tile and its halo is staged in LDS channel-planar (conflict-free), one thread per cell.
template <typename T>
__global__ void __launch_bounds__(MF_T)
k_cnn_l2(tp_grid g, const float* __restrict__ h, const float* __restrict__ w2, const float* __restrict__ b2,
         float* __restrict__ out, T* __restrict__ x, const float* __restrict__ scale,
         int32_t* __restrict__ bad) {
    __shared__ float s_h[CNN_CH * HCELLS];                             // [o][halo cell]
    __shared__ __attribute__((aligned(16))) float s_w[CNN_NT * CNN_CH];  // [t][o]
    const int32_t n = g.nx * g.ny * g.nz;
    const int32_t tx = (g.nx + TX - 1) / TX, ty = (g.ny + TY - 1) / TY;
    const int32_t bz = blockIdx.x / (tx * ty), by = (blockIdx.x / tx) % ty, bx = blockIdx.x % tx;
    const int32_t x0 = bx * TX, y0 = by * TY, z0 = bz * TZ;
    for (int k = threadIdx.x; k < CNN_NT * CNN_CH; k += MF_T) s_w[k] = w2[(k % CNN_CH) * CNN_NT + k / CNN_CH];
    for (int e = threadIdx.x; e < CNN_CH * HCELLS; e += MF_T) {
        const int o = e / HCELLS, r = e % HCELLS;
        const int hz = r / (HX * HY), hy = (r / HX) % HY, hx = r % HX;
        const int32_t xx = x0 + hx - 1, y = y0 + hy - 1, z = z0 + hz - 1;
        float v = 0.f;
        if (xx >= 0 && y >= 0 && z >= 0 && xx < g.nx && y < g.ny && z < g.nz)
            v = h[(int64_t)o * n + xx + (int64_t)g.nx * (y + (int64_t)g.ny * z)];
        s_h[e] = v > 0.f ? v : 0.f;
    }
    __syncthreads();
    const int lx = threadIdx.x % TX, ly = (threadIdx.x / TX) % TY, lz = threadIdx.x / (TX * TY);
    const int32_t xi = x0 + lx, yi = y0 + ly, zi = z0 + lz;
    if (xi >= g.nx || yi >= g.ny || zi >= g.nz) return;
    const int cb = (lz * HY + ly) * HX + lx;
    float acc = b2[0];
    for (int t = 0; t < CNN_NT; ++t) {
        const int j = cb + halo_tap(t);
        const float4v* wt = (const float4v*)&s_w[t * CNN_CH];
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            const float4v w = wt[k];
#pragma unroll
            for (int r = 0; r < 4; ++r) acc += w[r] * s_h[(4 * k + r) * HCELLS + j];
        }
    }
    const int64_t i = xi + (int64_t)g.nx * (yi + (int64_t)g.ny * zi);
    if (out) out[i] = acc;
    if (x) {
        if (!isfinite(acc)) *bad = 1;
        else x[i] = x[i] + (T)(scale[0] * acc);
    }
}

// ---- fused forward (inference) ------------------------------------------------------------
// Both layers in one pass, the hidden activations never leaving the chip.  A
// workgroup owns an 8 x 8 x 8 output tile; layer 2 needs relu(h) on the tile
// and a one-cell halo (10 x 10 x 10 cells, "H"), and those need the features
// on a two-cell halo (12 x 12 x 12, "F", staged in LDS as eight BF16 channels
// per cell, zero outside the grid).
//   Layer 1 runs on the H cells in groups of 16 (any 16 cells: each lane
//   addresses its own cell's taps), as k_cnn_l1 does: H (16 channels x 16
//   cells) = W1 F + b1 in seven v_mfma_f32_16x16x32_bf16 steps.
//   Layer 2 is regrouped by tap: out(i) = b2 + sum_t G_t(i + off_t) with
//   G_t(c) = sum_o W2[o][t] relu(h_o(c)).  G (taps x cells) = W2^T relu(H)
//   is a second contraction, over the 16 channels, on v_mfma_f32_16x16x16_bf16:
//   the first instruction leaves channel 4q + e of cell n in element e of
//   lane n + 16 q, which is exactly where the second one takes operand
//   B[k = channel][n], so relu(H) passes from accumulator to operand in
//   registers.  relu(h) enters split in two BF16 parts (hi + lo, relative
//   remainder <= 2^-18), taps in two blocks of 16 (27 used): four
//   instructions per group.  H cells outside the grid get G = 0 (layer 2's
//   zero padding).  G goes to LDS tap-major, one block of 16 taps at a time
//   (16 x 1008 FP32), into the space the features held (layer 1 is done by
//   then: every wavefront keeps its groups' relu(h) in registers); after a
//   barrier every thread adds its output cell's taps of the block, in tap
//   order, to its sum.
// LDS: max(27.6 KB of features, 64.5 KB of G) -- two workgroups per CU.
// Feature sources: FS 0, eight FP32 channel planes (channel 0 already
// scaled); FS 1, the attachment's BF16 static channels (8 per cell, slot 0
// unused) and the unscaled channel-0 plane z, divided by scale[0] when
// staged (the same FP32 division as the planar path).
typedef __attribute__((__vector_size__(4 * sizeof(short)))) short short4v;
typedef __attribute__((__vector_size__(4 * sizeof(__bf16)))) __bf16 bf16x4;
constexpr int FT = 8;                 // output tile edge
constexpr int FH = FT + 2, FF = FT + 4;
constexpr int FHC = FH * FH * FH;     // 1000 H cells
constexpr int FFC = FF * FF * FF;     // 1728 F cells
constexpr int FGROUPS = (FHC + 15) / 16;  // 63
constexpr int FGN = FGROUPS * 16;     // 1008 G columns (the last 8 unused)
constexpr int FU_T = 512;

__device__ inline int f_tap(int t) { return ((t / 9) * FF + (t / 3) % 3) * FF + t % 3; }
__device__ inline int h_tap(int t) { return ((t / 9) * FH + (t / 3) % 3) * FH + t % 3; }

__device__ inline short4v bf16x4_bits(float a, float b, float c, float d) {
    short4v v;
    v[0] = (short)(__float_as_uint(a) >> 16);  // arguments are BF16 values: exact
    v[1] = (short)(__float_as_uint(b) >> 16);
    v[2] = (short)(__float_as_uint(c) >> 16);
    v[3] = (short)(__float_as_uint(d) >> 16);
    return v;
}

template <typename T, int FS>
__global__ void __launch_bounds__(FU_T) __attribute__((amdgpu_waves_per_eu(4)))  // two workgroups a CU
k_cnn_fused(tp_grid g, const float* __restrict__ f, const uint16_t* __restrict__ fstat,
            const float* __restrict__ w1, const float* __restrict__ b1, const float* __restrict__ w2,
            const float* __restrict__ b2, float* __restrict__ out, T* __restrict__ x,
            const float* __restrict__ scale, int32_t* __restrict__ bad) {
    constexpr int FBYTES = FFC * (int)sizeof(bf16x8), GBYTES = 16 * FGN * (int)sizeof(float);
    __shared__ __attribute__((aligned(16))) unsigned char s_raw[FBYTES > GBYTES ? FBYTES : GBYTES];
    bf16x8* const s_f = reinterpret_cast<bf16x8*>(s_raw);  // features (layer 1)
    float* const s_g = reinterpret_cast<float*>(s_raw);     // then one tap block of G
    const int32_t n = g.nx * g.ny * g.nz;
    const int32_t tx = (g.nx + FT - 1) / FT, ty = (g.ny + FT - 1) / FT, tz = (g.nz + FT - 1) / FT;
    const int32_t ntiles = tx * ty * tz;
    // XCD-aware order: consecutive workgroups go to different XCDs (round
    // robin over 8), so tile k of XCD j is tile j * (ntiles / 8) + k and each
    // XCD walks a contiguous run of neighbouring tiles (shared halos in its L2)
    int32_t tile = blockIdx.x;
    if (ntiles % 8 == 0) tile = (blockIdx.x % 8) * (ntiles / 8) + blockIdx.x / 8;
    const int32_t bz = tile / (tx * ty), by = (tile / tx) % ty, bx = tile % tx;
    const int32_t x0 = bx * FT, y0 = by * FT, z0 = bz * FT;
    // weight fragments first: their loads overlap the staging's
    const int lane = threadIdx.x & 63, q = lane >> 4, col = lane & 15, wv = threadIdx.x >> 6;
    bf16x8 a[MF_KS];
    int ftoff[MF_KS];
#pragma unroll
    for (int st = 0; st < MF_KS; ++st) {
        const int t = 4 * st + q;
#pragma unroll
        for (int c = 0; c < CNN_CIN; ++c) {  // (padded taps load a real one, then take 0)
            const float w = w1[col * MF_K + c * CNN_NT + min(t, CNN_NT - 1)];
            a[st][c] = (__bf16)(t < CNN_NT ? w : 0.f);
        }
        ftoff[st] = t < CNN_NT ? f_tap(t) : 0;  // the padded tap reads a real cell, times zero weights
    }
    // W2^T tap blocks: A[m = tap - 16 blk][k = channel] at lane m + 16 (k / 4), element k % 4
    short4v a2[2];
#pragma unroll
    for (int blk = 0; blk < 2; ++blk) {
        const int t = 16 * blk + col;
        float w[4];
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            const float v = w2[(4 * q + e) * CNN_NT + min(t, CNN_NT - 1)];
            w[e] = t < CNN_NT ? v : 0.f;
        }
        a2[blk] = bf16x4_bits(w[0], w[1], w[2], w[3]);
    }
    float4v bias;
#pragma unroll
    for (int r = 0; r < 4; ++r) bias[r] = b1[4 * q + r];
    const float inv_s = FS == 1 ? scale[0] : 1.f;
    // staging: a thread's cells (at most FR) are loaded all at once, then
    // converted and stored (one round trip to memory instead of FR); a cell
    // outside the grid loads cell 0 and takes zeros (no masked, serialised loads)
    constexpr int FR = (FFC + FU_T - 1) / FU_T;
    bool fin[FR];
    int64_t fcell[FR];
#pragma unroll
    for (int k = 0; k < FR; ++k) {
        const int r = threadIdx.x + k * FU_T;
        const int fz = r / (FF * FF), fy = (r / FF) % FF, fx = r % FF;
        const int32_t cx = x0 + fx - 2, cy = y0 + fy - 2, cz = z0 + fz - 2;
        fin[k] = r < FFC && cx >= 0 && cy >= 0 && cz >= 0 && cx < g.nx && cy < g.ny && cz < g.nz;
        fcell[k] = fin[k] ? cx + (int64_t)g.nx * (cy + (int64_t)g.ny * cz) : 0;
    }
    if (FS == 0) {
        float fv[FR][CNN_CIN];
#pragma unroll
        for (int k = 0; k < FR; ++k)
#pragma unroll
            for (int c = 0; c < CNN_CIN; ++c) fv[k][c] = f[(int64_t)c * n + fcell[k]];
#pragma unroll
        for (int k = 0; k < FR; ++k) {
            const int r = threadIdx.x + k * FU_T;
            bf16x8 v{};
#pragma unroll
            for (int c = 0; c < CNN_CIN; ++c) v[c] = (__bf16)(fin[k] ? fv[k][c] : 0.f);  // nearest even
            if (r < FFC) s_f[r] = v;
        }
    } else {
        bf16x8 sv[FR];
        float zv[FR];
#pragma unroll
        for (int k = 0; k < FR; ++k) {
            sv[k] = *reinterpret_cast<const bf16x8*>(fstat + 8 * fcell[k]);
            zv[k] = f[fcell[k]];
        }
#pragma unroll
        for (int k = 0; k < FR; ++k) {
            const int r = threadIdx.x + k * FU_T;
            bf16x8 v = fin[k] ? sv[k] : bf16x8{};
            v[0] = (__bf16)(fin[k] && inv_s > 0.f ? zv[k] / inv_s : 0.f);
            if (r < FFC) s_f[r] = v;
        }
    }
    // this thread's output cell, and what its update reads, loaded now
    const int lx = threadIdx.x % FT, ly = (threadIdx.x / FT) % FT, lz = threadIdx.x / (FT * FT);
    const int32_t xi = x0 + lx, yi = y0 + ly, zi = z0 + lz;
    const bool mine = xi < g.nx && yi < g.ny && zi < g.nz;
    const int hb = (lz * FH + ly) * FH + lx;  // H index of tap (-1,-1,-1)
    const int64_t i = mine ? xi + (int64_t)g.nx * (yi + (int64_t)g.ny * zi) : 0;
    float o = b2[0];
    const T xold = x && mine ? x[i] : T(0);
    const float sc = x ? scale[0] : 0.f;
    __syncthreads();
    // layer 1 on this wavefront's groups: relu(h) split in two BF16 parts,
    // kept in registers (the features' LDS space is reused for G below)
    constexpr int FW = FU_T / 64;                   // wavefronts
    constexpr int KG = (FGROUPS + FW - 1) / FW;     // groups a wavefront
    short4v bh[KG], bl[KG];
#pragma unroll
    for (int k = 0; k < KG; ++k) {
        const int grp = wv + FW * k;
        bh[k] = bl[k] = short4v{0, 0, 0, 0};
        if (grp >= FGROUPS) continue;
        const int hl = 16 * grp + col;             // this lane's H cell
        const bool real = hl < FHC;
        const int hx = hl % FH, hy = (hl / FH) % FH, hz = hl / (FH * FH);
        const int fb = real ? (hz * FF + hy) * FF + hx : 0;  // F index of tap (-1,-1,-1)
        float4v acc = bias;
#pragma unroll
        for (int st = 0; st < MF_KS; ++st) {
            const bf16x8 b = s_f[fb + ftoff[st]];
            acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[st], b, acc, 0, 0, 0);
        }
        const int32_t cx = x0 + hx - 1, cy = y0 + hy - 1, cz = z0 + hz - 1;
        const bool live = real & (cx >= 0) & (cy >= 0) & (cz >= 0) & (cx < g.nx) & (cy < g.ny) & (cz < g.nz);
        bf16x4 hi, lo;
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            const float v = live & (acc[e] > 0.f) ? acc[e] : 0.f;
            hi[e] = (__bf16)v;                   // round to nearest even
            lo[e] = (__bf16)(v - (float)hi[e]);  // v - hi is exact in FP32
        }
        bh[k] = __builtin_bit_cast(short4v, hi);
        bl[k] = __builtin_bit_cast(short4v, lo);
    }
#pragma unroll
    for (int blk = 0; blk < 2; ++blk) {
        __syncthreads();  // (the features, then the previous block, are read until here)
#pragma unroll
        for (int k = 0; k < KG; ++k) {
            const int grp = wv + FW * k;
            if (grp >= FGROUPS) continue;
            float4v gt = {0.f, 0.f, 0.f, 0.f};
            gt = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a2[blk], bh[k], gt, 0, 0, 0);
            gt = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a2[blk], bl[k], gt, 0, 0, 0);
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                // D[m = tap][n = cell] at lane n + 16 (m / 4); rows past the last tap are never read
                s_g[(4 * q + e) * FGN + 16 * grp + col] = gt[e];
            }
        }
        __syncthreads();
        if (mine)
#pragma unroll
            for (int tl = 0; tl < 16; ++tl) {
                const int t = 16 * blk + tl;
                if (t < CNN_NT) o += s_g[tl * FGN + hb + h_tap(t)];
            }
    }
    if (!mine) return;
    if (out) out[i] = o;
    if (x) {
        if (!isfinite(o)) *bad = 1;
        else x[i] = xold + (T)(sc * o);
    }
}

// static channels 1..7 as BF16, eight per cell (slot 0 left zero)
__global__ void __launch_bounds__(CB)
k_feat_pack(int32_t n, const float* __restrict__ f, uint16_t* __restrict__ fs) {
    const int32_t i = blockIdx.x * CB + threadIdx.x;
    if (i >= n) return;
    uint16_t v[8];
    v[0] = 0;
#pragma unroll
    for (int c = 1; c < CNN_CIN; ++c) v[c] = (uint16_t)(__float_as_uint(bf16_round(f[(int64_t)c * n + i])) >> 16);
#pragma unroll
    for (int c = 0; c < CNN_CIN; ++c) fs[8 * (int64_t)i + c] = v[c];
}

// ---- loss and gradients ------------------------------------------------------------------
// dout = 2 (out - y) / n; per-block partial sums of (out - y)^2
__global__ void __launch_bounds__(CB)
k_cnn_dout(int32_t n, const float* __restrict__ out, const float* __restrict__ y, float* __restrict__ dout,
           double* __restrict__ part) {
    __shared__ double sh[CB];
    double acc = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * CB + threadIdx.x; i < n; i += (int64_t)gridDim.x * CB) {
        const float d = out[i] - y[i];
        dout[i] = 2.f * d / (float)n;
        acc += (double)d * (double)d;
    }
    sh[threadIdx.x] = acc;
    __syncthreads();
    for (int off = CB / 2; off > 0; off >>= 1) {
        if (threadIdx.x < off) sh[threadIdx.x] += sh[threadIdx.x + off];
        __syncthreads();
    }
    if (threadIdx.x == 0) part[blockIdx.x] = sh[0];
}

// ---- weight and bias gradients --------------------------------------------------------------
// Per cell tile (the forward pass's 16 x 4 x 4 tiling) and with the one-cell halo of the
// features and of dout staged in LDS:
//   dh_o(j)      = [h_o(j) > 0] sum_t W2[o][t] dout(j - off_t)            (FP32, in the tile)
//   dW1[o][c][t] = sum_j dh_o(j) f_c(j + off_t)     db1[o] = sum_j dh_o(j)
//   dW2[o][t]    = sum_j relu(h_o(j)) dout(j - off_t)                   db2 = sum_j dout(j)
// (the second is the first layer's gradient sum with i = j + off_t substituted). The three
// cell sums are contractions over the tile's 256 cells, run on 16x16x32 BF16 MFMA with FP32
// accumulation: [W1 | b1] as 14 column blocks of 16 (216 im2col columns of the BF16 features,
// a column of ones, 7 zero columns) against dh, and W2 as 2 blocks (27 taps of dout) against
// relu(h), four blocks per wave. FP32 operands that are not BF16 values enter split in two
// BF16 parts v = hi + lo (|v - hi - lo| <= 2^-18 |v|): dh x feature takes 2 products,
// relu(h) x dout takes 3 (hi.hi, hi.lo, lo.hi). Each workgroup accumulates over the tiles it
// visits and writes its own partial gradient; k_cnn_grad_reduce sums the partials in a fixed
// order, so the result is deterministic.
constexpr int GT_CELLS = TX * TY * TZ;  // 256 = one cell per thread
constexpr int GW_MAX = 512;             // partial-gradient workgroups at most

__device__ inline void split_bf16(float v, __bf16& hi, __bf16& lo) {
    const float a = bf16_round(v);
    hi = (__bf16)a;                   // exact
    lo = (__bf16)bf16_round(v - a);   // v - a is exact in FP32
}

__global__ void __launch_bounds__(MF_T)
k_cnn_wgrad(tp_grid g, const float* __restrict__ f, const float* __restrict__ h,
            const float* __restrict__ dout, const float* __restrict__ w2, float* __restrict__ part) {
    __shared__ __bf16 s_f[CNN_CIN * HCELLS];
    __shared__ float s_do[HCELLS];
    __shared__ __bf16 s_doh[HCELLS], s_dol[HCELLS];
    __shared__ __attribute__((aligned(16))) __bf16 s_dh[2][CNN_CH * GT_CELLS];  // [hi|lo][o][cell]
    __shared__ __attribute__((aligned(16))) __bf16 s_rh[2][CNN_CH * GT_CELLS];
    __shared__ __attribute__((aligned(16))) float s_w2[CNN_NT * CNN_CH];          // [t][o]
    __shared__ float s_red[MF_T / 64];
    const int32_t n = g.nx * g.ny * g.nz;
    const int32_t tx = (g.nx + TX - 1) / TX, ty = (g.ny + TY - 1) / TY, tz = (g.nz + TZ - 1) / TZ;
    const int32_t ntiles = tx * ty * tz;
    for (int k = threadIdx.x; k < CNN_NT * CNN_CH; k += MF_T) s_w2[k] = w2[(k % CNN_CH) * CNN_NT + k / CNN_CH];
    const int lane = threadIdx.x & 63, q = lane >> 4, col = lane & 15, wv = threadIdx.x >> 6;
    // per-lane operand source of each of the wave's four column blocks: an LDS offset of the
    // tap (relative to the cell's place in the halo), or a constant column (1 or 0)
    int boff[4], bconst[4];  // bconst: -1 gather, else the constant value
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const int job = wv + 4 * i;
        if (job < 14) {
            const int p = 16 * job + col;
            const int c = p / CNN_NT, t = p % CNN_NT;
            boff[i] = c * HCELLS + ((t / 9) * HY + (t / 3) % 3) * HX + t % 3;
            bconst[i] = p < MF_K ? -1 : (p == MF_K ? 1 : 0);
            if (bconst[i] >= 0) boff[i] = 0;
        } else {
            const int t = 16 * (job - 14) + col;
            boff[i] = ((2 - t / 9) * HY + (2 - (t / 3) % 3)) * HX + 2 - t % 3;
            bconst[i] = t < CNN_NT ? -1 : 0;
            if (bconst[i] >= 0) boff[i] = 0;
        }
    }
    float4v acc[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) acc[i] = float4v{0.f, 0.f, 0.f, 0.f};
    float db2 = 0.f;
    const int lx = threadIdx.x % TX, ly = (threadIdx.x / TX) % TY, lz = threadIdx.x / (TX * TY);
    for (int32_t tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
        const int32_t bz = tile / (tx * ty), by = (tile / tx) % ty, bx = tile % tx;
        const int32_t x0 = bx * TX, y0 = by * TY, z0 = bz * TZ;
        __syncthreads();  // the previous tile's operands are consumed; s_w2 is written
        for (int e = threadIdx.x; e < CNN_CIN * HCELLS; e += MF_T) {
            const int c = e / HCELLS, r = e % HCELLS;
            const int hz = r / (HX * HY), hy = (r / HX) % HY, hx = r % HX;
            const int32_t x = x0 + hx - 1, y = y0 + hy - 1, z = z0 + hz - 1;
            const bool in = x >= 0 && y >= 0 && z >= 0 && x < g.nx && y < g.ny && z < g.nz;
            const int64_t cell = x + (int64_t)g.nx * (y + (int64_t)g.ny * z);
            s_f[e] = (__bf16)(in ? bf16_round(f[(int64_t)c * n + cell]) : 0.f);
            if (c == 0) s_do[r] = in ? dout[cell] : 0.f;
        }
        __syncthreads();
        for (int e = threadIdx.x; e < HCELLS; e += MF_T) split_bf16(s_do[e], s_doh[e], s_dol[e]);
        {
            const int32_t x = x0 + lx, y = y0 + ly, z = z0 + lz;
            const bool in = x < g.nx && y < g.ny && z < g.nz;
            const int64_t cell = x + (int64_t)g.nx * (y + (int64_t)g.ny * z);
            const int hb = ((lz + 2) * HY + ly + 2) * HX + lx + 2;  // halo index of j - off_t at t = 0
            float d[CNN_CH];
#pragma unroll
            for (int o = 0; o < CNN_CH; ++o) d[o] = 0.f;
#pragma unroll 1
            for (int t = 0; t < CNN_NT; ++t) {
                const float dv = s_do[hb - ((t / 9) * HY + (t / 3) % 3) * HX - t % 3];
                const float4v* wt = (const float4v*)&s_w2[t * CNN_CH];
#pragma unroll
                for (int k = 0; k < 4; ++k) {
                    const float4v w = wt[k];
#pragma unroll
                    for (int r = 0; r < 4; ++r) d[4 * k + r] += w[r] * dv;
                }
            }
#pragma unroll
            for (int o = 0; o < CNN_CH; ++o) {
                const float hv = in ? h[(int64_t)o * n + cell] : 0.f;
                const float dh = hv > 0.f ? d[o] : 0.f;
                split_bf16(dh, s_dh[0][o * GT_CELLS + threadIdx.x], s_dh[1][o * GT_CELLS + threadIdx.x]);
                split_bf16(hv > 0.f ? hv : 0.f, s_rh[0][o * GT_CELLS + threadIdx.x],
                           s_rh[1][o * GT_CELLS + threadIdx.x]);
            }
            db2 += s_do[((lz + 1) * HY + ly + 1) * HX + lx + 1];  // zero outside the grid
        }
        __syncthreads();
#pragma unroll 1
        for (int st = 0; st < GT_CELLS / 32; ++st) {
            // this lane's cells in the K-step: 8 consecutive x of tile row 2 st + q / 2
            const int row = 2 * st + (q >> 1);
            const int cb = ((row / TY) * HY + row % TY) * HX + 8 * (q & 1);  // halo index, tap (0,0,0)
            const int ka = col * GT_CELLS + 32 * st + 8 * q;
            const bf16x8 dhh = *(const bf16x8*)&s_dh[0][ka], dhl = *(const bf16x8*)&s_dh[1][ka];
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                if (i < 3 || wv < 2) {  // job wv + 4 i: 0..13 [W1 | b1]; 14, 15 W2
                    bf16x8 b;
#pragma unroll
                    for (int j = 0; j < 8; ++j)
                        b[j] = bconst[i] < 0 ? s_f[boff[i] + cb + j] : (__bf16)(float)bconst[i];
                    acc[i] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(dhh, b, acc[i], 0, 0, 0);
                    acc[i] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(dhl, b, acc[i], 0, 0, 0);
                } else {
                    const bf16x8 rhh = *(const bf16x8*)&s_rh[0][ka], rhl = *(const bf16x8*)&s_rh[1][ka];
                    bf16x8 bh, bl;
#pragma unroll
                    for (int j = 0; j < 8; ++j) {
                        const bool gth = bconst[i] < 0;
                        bh[j] = gth ? s_doh[boff[i] + cb + j] : (__bf16)0.f;
                        bl[j] = gth ? s_dol[boff[i] + cb + j] : (__bf16)0.f;
                    }
                    acc[i] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(rhh, bh, acc[i], 0, 0, 0);
                    acc[i] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(rhh, bl, acc[i], 0, 0, 0);
                    acc[i] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(rhl, bh, acc[i], 0, 0, 0);
                }
            }
        }
    }
    float* pw = part + (int64_t)blockIdx.x * CNN_NPARAM;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const int job = wv + 4 * i;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int o = 4 * q + r;
            if (job < 14) {
                const int p = 16 * job + col;
                if (p < MF_K) pw[o * MF_K + p] = acc[i][r];
                else if (p == MF_K) pw[CNN_OFF_B1 + o] = acc[i][r];
            } else {
                const int t = 16 * (job - 14) + col;
                if (t < CNN_NT) pw[CNN_OFF_W2 + o * CNN_NT + t] = acc[i][r];
            }
        }
    }
    for (int off = 32; off > 0; off >>= 1) db2 += __shfl_down(db2, off);
    if (lane == 0) s_red[wv] = db2;
    __syncthreads();
    if (threadIdx.x == 0) pw[CNN_OFF_B2] = (s_red[0] + s_red[1]) + (s_red[2] + s_red[3]);
}

// grad[p] = sum over workgroups of the partials, in workgroup order
__global__ void __launch_bounds__(CB)
k_cnn_grad_reduce(int nwg, const float* __restrict__ part, float* __restrict__ grad) {
    const int p = blockIdx.x * CB + threadIdx.x;
    if (p >= CNN_NPARAM) return;
    float a0 = 0.f, a1 = 0.f, a2 = 0.f, a3 = 0.f;
    int b = 0;
    for (; b + 4 <= nwg; b += 4) {
        a0 += part[(int64_t)b * CNN_NPARAM + p];
        a1 += part[(int64_t)(b + 1) * CNN_NPARAM + p];
        a2 += part[(int64_t)(b + 2) * CNN_NPARAM + p];
        a3 += part[(int64_t)(b + 3) * CNN_NPARAM + p];
    }
    for (; b < nwg; ++b) a0 += part[(int64_t)b * CNN_NPARAM + p];
    grad[p] = (a0 + a1) + (a2 + a3);
}

// Adam (Kingma & Ba 2015) on the FP32 master weights; refresh the BF16 copies
__global__ void __launch_bounds__(CB)
k_adam(int np, const float* __restrict__ grad, float* __restrict__ w, float* __restrict__ m,
       float* __restrict__ v, float* __restrict__ wbf, float lr, float b1, float b2, float eps, float c1,
       float c2) {
    const int p = blockIdx.x * CB + threadIdx.x;
    if (p >= np) return;
    const float gr = grad[p];
    const float mm = b1 * m[p] + (1.f - b1) * gr;
    const float vv = b2 * v[p] + (1.f - b2) * gr * gr;
    m[p] = mm;
    v[p] = vv;
    const float wn = w[p] - lr * (mm / c1) / (sqrtf(vv / c2) + eps);
    w[p] = wn;
    wbf[p] = bf16_round(wn);
}

__global__ void __launch_bounds__(CB)
k_bf16_copy(int np, const float* __restrict__ w, float* __restrict__ wbf) {
    const int p = blockIdx.x * CB + threadIdx.x;
    if (p < np) wbf[p] = bf16_round(w[p]);
}

__global__ void __launch_bounds__(CB)
k_loss_sum(int nb, int32_t n, const double* __restrict__ part, double* __restrict__ loss) {
    __shared__ double sh[CB];
    double a = 0.0;
    for (int b = threadIdx.x; b < nb; b += CB) a += part[b];
    sh[threadIdx.x] = a;
    __syncthreads();
    for (int off = CB / 2; off > 0; off >>= 1) {
        if (threadIdx.x < off) sh[threadIdx.x] += sh[threadIdx.x + off];
        __syncthreads();
    }
    if (threadIdx.x == 0) loss[0] = sh[0] / n;
}

// ---- loss in the D^{-1} A norm --------------------------------------------------------------
// v = D^{-1} A (out - target); per-block partial sums of v^2 + w (out - target)^2 (w: weight
// of the error term); v overwritten by dL/dv = 2 v / n
__global__ void __launch_bounds__(CB)
k_op_forward(int32_t n, const int32_t* __restrict__ rowptr, const int32_t* __restrict__ col,
             const double* __restrict__ val, const float* __restrict__ dinv, const float* __restrict__ out,
             const float* __restrict__ target, float w, float* __restrict__ dv, double* __restrict__ part) {
    __shared__ double sh[CB];
    double acc = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * CB + threadIdx.x; i < n; i += (int64_t)gridDim.x * CB) {
        double s = 0.0;
        for (int32_t k = rowptr[i]; k < rowptr[i + 1]; ++k) {
            const int32_t j = col[k];
            s += val[k] * (double)(out[j] - target[j]);
        }
        const float v = (float)(s * (double)dinv[i]);
        const float e = out[i] - target[i];
        acc += (double)v * (double)v + (double)w * ((double)e * (double)e);
        dv[i] = 2.f * v / (float)n;
    }
    sh[threadIdx.x] = acc;
    __syncthreads();
    for (int off = CB / 2; off > 0; off >>= 1) {
        if (threadIdx.x < off) sh[threadIdx.x] += sh[threadIdx.x + off];
        __syncthreads();
    }
    if (threadIdx.x == 0) part[blockIdx.x] = sh[0];
}

// dout = A^T (D^{-1} dv) + 2 w (out - target) / n, with A^T given explicitly (sorted CSR)
__global__ void __launch_bounds__(CB)
k_op_backward(int32_t n, const int32_t* __restrict__ trp, const int32_t* __restrict__ tcol,
              const double* __restrict__ tval, const float* __restrict__ dinv, const float* __restrict__ dv,
              const float* __restrict__ out, const float* __restrict__ target, float w,
              float* __restrict__ dout) {
    const int32_t j = blockIdx.x * CB + threadIdx.x;
    if (j >= n) return;
    double s = 0.0;
    for (int32_t k = trp[j]; k < trp[j + 1]; ++k) {
        const int32_t i = tcol[k];
        s += tval[k] * (double)(dinv[i] * dv[i]);
    }
    if (w != 0.f) s += (double)(2.f * w * (out[j] - target[j]) / (float)n);
    dout[j] = (float)s;
}

// ---- host helpers ---------------------------------------------------------------------------
static int red_blocks(int32_t n) { return std::max(1, std::min(1024, cdiv(n, CB * 4))); }

void cnn_work_reserve(tp_cnn* c, int32_t n, hipStream_t s) {
    if (c->n_work >= n) return;
    c->h.alloc((size_t)CNN_CH * n, s);
    c->dh.alloc((size_t)CNN_CH * n, s);
    c->out.alloc(n, s);
    c->dout.alloc(n, s);
    c->part.alloc(1024, s);
    if (!c->gpart.p) c->gpart.alloc((size_t)GW_MAX * CNN_NPARAM, s);
    c->n_work = n;
}

// forward on given features; out may be null; with x: smoother update x += scale * out;
// hidden activations in hw (16 x n) or, when null, in the network's own work buffer
static int fused_tiles(const tp_grid& g) {
    return ((g.nx + FT - 1) / FT) * ((g.ny + FT - 1) / FT) * ((g.nz + FT - 1) / FT);
}

// inference: both layers in one pass (planar FP32 features, channel 0 scaled)
template <typename T>
void cnn_forward_fused(tp_cnn* c, const tp_grid& g, const float* f, float* out, T* x, const float* scale,
                       int32_t* bad, hipStream_t s) {
    const int tiles = fused_tiles(g);
    if (tiles > 0)
        TP_LAUNCH((k_cnn_fused<T, 0>), tiles, FU_T, 0, s, g, f, (const uint16_t*)nullptr, c->wbf.p,
                  c->w.p + CNN_OFF_B1, c->wbf.p + CNN_OFF_W2, c->w.p + CNN_OFF_B2, out, x, scale, bad);
}
template void cnn_forward_fused<float>(tp_cnn*, const tp_grid&, const float*, float*, float*, const float*,
                                       int32_t*, hipStream_t);

// the smoother update on the finest level: features from the attachment's
// packed static channels and its unscaled channel-0 plane
template <typename T>
void cnn_smooth_fused(tp_cnn_attach* a, T* x, hipStream_t s) {
    const int tiles = fused_tiles(a->g);
    tp_cnn* c = a->net;
    if (tiles > 0)
        TP_LAUNCH((k_cnn_fused<T, 1>), tiles, FU_T, 0, s, a->g, a->feat.p, a->fstat.p, c->wbf.p,
                  c->w.p + CNN_OFF_B1, c->wbf.p + CNN_OFF_W2, c->w.p + CNN_OFF_B2, (float*)nullptr, x, a->scale.p,
                  a->bad.p);
}
template void cnn_smooth_fused<double>(tp_cnn_attach*, double*, hipStream_t);
template void cnn_smooth_fused<float>(tp_cnn_attach*, float*, hipStream_t);

// training forward: the two layers apart, keeping the hidden activations
// (hw, or the network's own work buffer) for the gradient
template <typename T>
void cnn_forward_into(tp_cnn* c, const tp_grid& g, const float* f, float* out, T* x, const float* scale,
                      int32_t* bad, hipStream_t s, float* hw) {
    const int32_t n = g.nx * g.ny * g.nz;
    if (!hw) {
        cnn_work_reserve(c, n, s);
        hw = c->h.p;
    }
    {
        const int64_t tiles = (int64_t)((g.nx + TX - 1) / TX) * ((g.ny + TY - 1) / TY) * ((g.nz + TZ - 1) / TZ);
        if (tiles > 0) {
            TP_LAUNCH(k_cnn_l1, (int)tiles, MF_T, 0, s, g, f, c->wbf.p, c->w.p + CNN_OFF_B1, hw);
            TP_LAUNCH(k_cnn_l2<T>, (int)tiles, MF_T, 0, s, g, hw, c->wbf.p + CNN_OFF_W2, c->w.p + CNN_OFF_B2,
                      out, x, scale, bad);
        }
    }
}
template void cnn_forward_into<double>(tp_cnn*, const tp_grid&, const float*, float*, double*, const float*,
                                       int32_t*, hipStream_t, float*);
template void cnn_forward_into<float>(tp_cnn*, const tp_grid&, const float*, float*, float*, const float*,
                                      int32_t*, hipStream_t, float*);

// features for residual r on the finest level of a hierarchy with an attached smoother
// (normalise false: channel 0 is left as z = D^{-1} r, the fused smoother
// divides by the scale when it stages it)
template <typename T>
void cnn_features_into(tp_cnn_attach* a, const T* r, float* f, hipStream_t s, bool normalise) {
    const int32_t n = a->g.nx * a->g.ny * a->g.nz;
    const int nb = red_blocks(n);
    TP_LAUNCH(k_feat_resid<T>, nb, CB, 0, s, n, r, a->dinv.p, f, a->part.p);
    TP_LAUNCH(k_feat_scale_sum, 1, CB, 0, s, nb, n, a->part.p, a->scale.p);
    if (normalise) TP_LAUNCH(k_feat_normalise, cdiv(n, CB), CB, 0, s, n, a->scale.p, f);
}
template void cnn_features_into<double>(tp_cnn_attach*, const double*, float*, hipStream_t, bool);
template void cnn_features_into<float>(tp_cnn_attach*, const float*, float*, hipStream_t, bool);

// gradient of the loss from c->dout (set by the caller) and c->h of the last forward
void cnn_backward_from_dout(tp_cnn* c, const tp_grid& g, const float* feat, hipStream_t s) {
    const int64_t tiles = (int64_t)((g.nx + TX - 1) / TX) * ((g.ny + TY - 1) / TY) * ((g.nz + TZ - 1) / TZ);
    const int nwg = (int)std::max<int64_t>(1, std::min<int64_t>(tiles, GW_MAX));
    TP_LAUNCH(k_cnn_wgrad, nwg, MF_T, 0, s, g, feat, c->h.p, c->dout.p, c->wbf.p + CNN_OFF_W2, c->gpart.p);
    TP_LAUNCH(k_cnn_grad_reduce, cdiv(CNN_NPARAM, CB), CB, 0, s, nwg, c->gpart.p, c->grad.p);
}

// loss in the D^{-1} A norm of the attached finest level (A^T built on first use)
void cnn_op_loss_grad(tp_cnn_attach* a, const int32_t* rowptr, const int32_t* col, const double* val,
                      int32_t nnz, const float* feat, const float* target, float err_weight, hipStream_t s) {
    tp_cnn* c = a->net;
    const tp_grid& g = a->g;
    const int32_t n = g.nx * g.ny * g.nz;
    if (!a->At.rowptr.p) transpose(rowptr, col, val, n, n, nnz, true, a->At, s);
    cnn_work_reserve(c, n, s);
    cnn_forward_into<float>(c, g, feat, c->out.p, nullptr, nullptr, nullptr, s);
    const int nb = red_blocks(n);
    TP_LAUNCH(k_op_forward, nb, CB, 0, s, n, rowptr, col, val, a->dinv.p, c->out.p, target, err_weight, c->dh.p,
              c->part.p);
    TP_LAUNCH(k_loss_sum, 1, CB, 0, s, nb, n, c->part.p, c->loss.p);
    TP_LAUNCH(k_op_backward, cdiv(n, CB), CB, 0, s, n, a->At.rowptr.p, a->At.col.p, a->At.val.p, a->dinv.p,
              c->dh.p, c->out.p, target, err_weight, c->dout.p);
    cnn_backward_from_dout(c, g, feat, s);
}

void cnn_attach_build(tp_cnn_attach* a, const tp_grid& g, const int32_t* rowptr, const int32_t* col,
                      const double* val, hipStream_t s) {
    const int32_t n = g.nx * g.ny * g.nz;
    a->g = g;
    a->feat.alloc((size_t)CNN_CIN * n, s);
    a->dinv.alloc(n, s);
    a->part.alloc(1024, s);
    a->scale.alloc(1, s);
    a->bad.alloc(1, s);
    a->fstat.alloc((size_t)CNN_CIN * n, s);
    TP_LAUNCH(k_feat_static, cdiv(n, CB), CB, 0, s, g, rowptr, col, val, a->feat.p, a->dinv.p);
    TP_LAUNCH(k_feat_pack, cdiv(n, CB), CB, 0, s, n, a->feat.p, a->fstat.p);
}

// new values of the level operator (same pattern): static feature channels and
// 1/D again, in place; the transpose kept for the training loss is dropped
void cnn_attach_refresh(tp_cnn_attach* a, const int32_t* rowptr, const int32_t* col, const double* val,
                        hipStream_t s) {
    const int32_t n = a->g.nx * a->g.ny * a->g.nz;
    TP_LAUNCH(k_feat_static, cdiv(n, CB), CB, 0, s, a->g, rowptr, col, val, a->feat.p, a->dinv.p);
    TP_LAUNCH(k_feat_pack, cdiv(n, CB), CB, 0, s, n, a->feat.p, a->fstat.p);
    a->At = Csr{};
}

}  // namespace tp

extern "C" {

int cnn_create(const float* params, tp_cnn_t* out) {
    TP_GUARD({
        TP_CHECK_ARG(params && out, "cnn_create: null argument");
        for (int p = 0; p < CNN_NPARAM; ++p)
            TP_CHECK_ARG(std::isfinite(params[p]), "cnn_create: parameter %d is not finite", p);
        hipStream_t s = nullptr;
        tp_cnn* c = new tp_cnn();
        c->w.alloc(CNN_NPARAM, s);
        c->wbf.alloc(CNN_NPARAM, s);
        c->m.alloc(CNN_NPARAM, s);
        c->v.alloc(CNN_NPARAM, s);
        c->grad.alloc(CNN_NPARAM, s);
        c->loss.alloc(1, s);
        TP_HIP(hipMemcpyAsync(c->w.p, params, sizeof(float) * CNN_NPARAM, hipMemcpyHostToDevice, s));
        TP_HIP(hipMemsetAsync(c->m.p, 0, sizeof(float) * CNN_NPARAM, s));
        TP_HIP(hipMemsetAsync(c->v.p, 0, sizeof(float) * CNN_NPARAM, s));
        TP_LAUNCH(tp::k_bf16_copy, tp::cdiv(CNN_NPARAM, tp::CB), tp::CB, 0, s, CNN_NPARAM, c->w.p, c->wbf.p);
        TP_HIP(hipStreamSynchronize(s));
        *out = c;
    });
    return TP_OK;
}

int cnn_get_params(tp_cnn_t c, float* params) {
    TP_GUARD({
        TP_CHECK_ARG(c && params, "cnn_get_params: null argument");
        TP_HIP(hipMemcpy(params, c->w.p, sizeof(float) * CNN_NPARAM, hipMemcpyDeviceToHost));
    });
    return TP_OK;
}

int cnn_get_grad(tp_cnn_t c, float* grad) {
    TP_GUARD({
        TP_CHECK_ARG(c && grad, "cnn_get_grad: null argument");
        TP_HIP(hipDeviceSynchronize());
        TP_HIP(hipMemcpy(grad, c->grad.p, sizeof(float) * CNN_NPARAM, hipMemcpyDeviceToHost));
    });
    return TP_OK;
}

int cnn_destroy(tp_cnn_t c) {
    TP_GUARD({
        if (c) {
            TP_HIP(hipDeviceSynchronize());
            delete c;
            TP_HIP(hipDeviceSynchronize());
        }
    });
    return TP_OK;
}

int cnn_forward(tp_cnn_t c, const tp_grid* grid, const float* feat, float* out, void* stream) {
    TP_GUARD({
        TP_CHECK_ARG(c && grid && feat && out, "cnn_forward: null argument");
        TP_CHECK_ARG(grid->nx >= 1 && grid->ny >= 1 && grid->nz >= 1, "cnn_forward: bad grid");
        tp::cnn_forward_fused<float>(c, *grid, feat, out, nullptr, nullptr, nullptr, (hipStream_t)stream);
    });
    return TP_OK;
}

int cnn_loss_grad(tp_cnn_t c, const tp_grid* grid, const float* feat, const float* target, double* loss,
                  float* grad, void* stream) {
    TP_GUARD({
        TP_CHECK_ARG(c && grid && feat && target, "cnn_loss_grad: null argument");
        hipStream_t s = (hipStream_t)stream;
        const tp_grid g = *grid;
        const int32_t n = g.nx * g.ny * g.nz;
        TP_CHECK_ARG(n >= 1, "cnn_loss_grad: bad grid");
        tp::cnn_work_reserve(c, n, s);  // before taking c->out.p
        tp::cnn_forward_into<float>(c, g, feat, c->out.p, nullptr, nullptr, nullptr, s);
        const int nb = tp::red_blocks(n);
        TP_LAUNCH(tp::k_cnn_dout, nb, tp::CB, 0, s, n, c->out.p, target, c->dout.p, c->part.p);
        TP_LAUNCH(tp::k_loss_sum, 1, tp::CB, 0, s, nb, n, c->part.p, c->loss.p);
        tp::cnn_backward_from_dout(c, g, feat, s);
        if (grad)
            TP_HIP(hipMemcpyAsync(grad, c->grad.p, sizeof(float) * CNN_NPARAM, hipMemcpyDeviceToDevice, s));
        if (loss) {
            TP_HIP(hipMemcpyAsync(loss, c->loss.p, sizeof(double), hipMemcpyDeviceToHost, s));
            TP_HIP(hipStreamSynchronize(s));
        }
    });
    return TP_OK;
}

int cnn_adam_step(tp_cnn_t c, float lr, void* stream) {
    TP_GUARD({
        TP_CHECK_ARG(c, "cnn_adam_step: null handle");
        TP_CHECK_ARG(lr > 0.f && std::isfinite(lr), "cnn_adam_step: lr must be > 0");
        c->step += 1;
        const float b1 = 0.9f, b2 = 0.999f;
        const float c1 = 1.f - std::pow(b1, (float)c->step), c2 = 1.f - std::pow(b2, (float)c->step);
        TP_LAUNCH(tp::k_adam, tp::cdiv(CNN_NPARAM, tp::CB), tp::CB, 0, (hipStream_t)stream, CNN_NPARAM, c->grad.p,
                  c->w.p, c->m.p, c->v.p, c->wbf.p, lr, b1, b2, 1e-8f, c1, c2);
    });
    return TP_OK;
}

}  // extern "C"
