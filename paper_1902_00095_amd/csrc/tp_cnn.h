// tp_cnn.h -- learned post-smoother objects (network weights, attachment to
// the finest level of a hierarchy).
#pragma once

#include "tp_internal.h"

#define CNN_CIN 8
#define CNN_CH 16
#define CNN_NT 27
#define CNN_OFF_B1 (CNN_CH * CNN_CIN * CNN_NT)           // 3456
#define CNN_OFF_W2 (CNN_OFF_B1 + CNN_CH)                  // 3472
#define CNN_OFF_B2 (CNN_OFF_W2 + CNN_CH * CNN_NT)         // 3904
#define CNN_NPARAM (CNN_OFF_B2 + 1)                       // 3905

struct tp_cnn {
    tp::DBuf<float> w;      // FP32 master parameters (W1, b1, W2, b2)
    tp::DBuf<float> wbf;    // the same rounded to BF16 (values used by the kernels)
    tp::DBuf<float> m, v, grad;
    tp::DBuf<double> loss;
    int64_t step = 0;
    // work (grown on demand)
    int32_t n_work = 0;
    tp::DBuf<float> h, dh, out, dout;
    tp::DBuf<double> part;
    tp::DBuf<float> gpart;  // per-workgroup partial gradients
};

namespace tp {
// A network attached to the finest level of a hierarchy (grid geometry,
// static feature channels 1..7, l1 diagonal inverse, scale, failure flag).
struct tp_cnn_attach {
    tp_cnn* net = nullptr;
    tp_grid g{};
    DBuf<float> feat;   // 8 x n; channel 0 rewritten per application
    DBuf<float> dinv;
    DBuf<double> part;
    DBuf<float> scale;
    DBuf<int32_t> bad;
    DBuf<uint16_t> fstat;  // static channels 1..7 as BF16, 8 per cell (slot 0 unused): the fused smoother's input
    Csr At;             // transpose of the level operator (operator-norm training loss)
    bool enabled = true;
};

void cnn_work_reserve(tp_cnn* c, int32_t n, hipStream_t s);
template <typename T>
void cnn_forward_into(tp_cnn* c, const tp_grid& g, const float* f, float* out, T* x, const float* scale,
                      int32_t* bad, hipStream_t s, float* hw = nullptr);
template <typename T>
void cnn_features_into(tp_cnn_attach* a, const T* r, float* f, hipStream_t s, bool normalise = true);
template <typename T>
void cnn_forward_fused(tp_cnn* c, const tp_grid& g, const float* f, float* out, T* x, const float* scale,
                       int32_t* bad, hipStream_t s);
template <typename T>
void cnn_smooth_fused(tp_cnn_attach* a, T* x, hipStream_t s);
void cnn_backward_from_dout(tp_cnn* c, const tp_grid& g, const float* feat, hipStream_t s);
void cnn_op_loss_grad(tp_cnn_attach* a, const int32_t* rowptr, const int32_t* col, const double* val,
                      int32_t nnz, const float* feat, const float* target, float err_weight, hipStream_t s);
void transpose(const int32_t* rowptr, const int32_t* col, const double* val, int32_t n, int32_t m,
               int32_t nnz, bool sorted, Csr& T, hipStream_t s);
void cnn_attach_build(tp_cnn_attach* a, const tp_grid& g, const int32_t* rowptr, const int32_t* col,
                      const double* val, hipStream_t s);
void cnn_attach_refresh(tp_cnn_attach* a, const int32_t* rowptr, const int32_t* col, const double* val,
                        hipStream_t s);
}  // namespace tp
