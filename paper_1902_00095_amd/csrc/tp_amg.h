// tp_amg.h -- AMG hierarchy object shared by the setup, the V-cycle and the
// block preconditioner.
#pragma once

#include "tp_cnn.h"

#include <memory>

namespace tp {

// Lanes cooperating on one CSR row in the row-group SpMV kernels.
int lanes_for(int32_t n, int64_t nnz);

struct Level {
    Csr A, P, R;          // FP64 setup results (P, R empty on the coarsest level)
    Csr AP;               // the product A P formed for the Galerkin operator (kept for numeric refreshes)
    // extended+i interpolation, kept for numeric refreshes: the strength
    // pattern of A and the interpolatory sets (S, T), and the same for A^T
    // when R = Q^T (Sq, Tq)
    Csr S, T, Sq, Tq;
    DBuf<int32_t> cf;     // 1 C, 0 F
    DBuf<double> dinv;    // 1 / sum_j |a_ij|
    DBuf<float> A32, P32, R32, dinv32;  // storage 1 copies (storage 2: P32, R32, dinv32)
    // storage 2: BF16 values of A with the diagonal entries stored as 0 (CSR
    // and DIA layouts) and the diagonal itself in FP32
    DBuf<uint16_t> A16, dia16;
    DBuf<float> diag32;
    int gA = 1, gP = 1, gR = 1;
    // Row-block (stream) form of A's row products on large CSR levels: blocks
    // of sb_rows consecutive rows whose products are staged in LDS (at most
    // sb_lds of them per block); sb_rows = 0 when the level does not use it.
    int sb_rows = 0, sb_lds = 0;
    // the same form for the products with P and R (sbP_rows = 0: not used)
    int sbP_rows = 0, sbP_lds = 0, sbR_rows = 0, sbR_lds = 0;
    // Diagonal (DIA) copy of A when its column offsets form a small set
    // (stencil levels): dia[d * n + i] = a(i, i + off[d]), zero outside.
    int ndia = 0;
    int dia_off[7] = {0, 0, 0, 0, 0, 0, 0};
    DBuf<double> dia;
    DBuf<float> dia32;
    // V-cycle work vectors (element type follows the storage)
    DBuf<char> b, x, x2, r, d;
};

}  // namespace tp

struct tp_amg {
    tp::Arena arena;             // owns every setup allocation (declared first: destroyed last)
    tp_amg_params prm;
    std::vector<tp::Level> lev;  // lev.back() is the coarsest level
    int32_t nc = 0;              // coarsest size
    tp::DBuf<double> cinv;       // nc x nc inverse of the coarsest operator
    hipStream_t stream = nullptr;
    std::unique_ptr<tp::tp_cnn_attach> cnn;  // learned finest-level post-smoother (optional)
    uint64_t cnn_gen = 0;                    // attachments made so far (identifies the current one)
    bool stop_before_post = false;           // pair generation: end the cycle before post-smoothing
};

namespace tp {
// Run one V-cycle on the level-0 right-hand side already placed in lev[0].b
// (or at `b_ext` when non-null, same element type as the storage).  Returns
// a device pointer to the level-0 solution (element type of the storage):
// `x_ext` when non-null and the cycle ends in a smoothing step that can
// write there, else one of the level's work vectors.
const void* vcycle_run(tp_amg* h, const void* b_ext, hipStream_t s, void* x_ext = nullptr);
// element size of the hierarchy's storage
inline size_t storage_bytes(const tp_amg* h) { return h->prm.storage == 0 ? 8 : 4; }
}  // namespace tp
