// mlp.h -- learned refinement flags (host interface of mlp.hip).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "kernels.h"

#ifndef IC_MLP_IN
#define IC_MLP_IN 512
#endif
#define IC_MLP_HID 128
// parameter vector (fp32 master copy): W1 [512][128], b1 [128], W2 [128][128], b2 [128], w3 [128], b3
#define IC_MLP_OFF_W1 0
#define IC_MLP_OFF_B1 (IC_MLP_OFF_W1 + IC_MLP_IN * IC_MLP_HID)
#define IC_MLP_OFF_W2 (IC_MLP_OFF_B1 + IC_MLP_HID)
#define IC_MLP_OFF_B2 (IC_MLP_OFF_W2 + IC_MLP_HID * IC_MLP_HID)
#define IC_MLP_OFF_W3 (IC_MLP_OFF_B2 + IC_MLP_HID)
#define IC_MLP_OFF_B3 (IC_MLP_OFF_W3 + IC_MLP_HID)
#define IC_MLP_NPARAM_ (IC_MLP_OFF_B3 + 1)
#ifndef IC_MLP_NPARAM
#define IC_MLP_NPARAM IC_MLP_NPARAM_
#endif
static_assert(IC_MLP_NPARAM == IC_MLP_NPARAM_, "parameter count");

struct MlpHparams {
    int epochs;
    int batch;
    float lr, beta1, beta2, eps;
    unsigned seed;
    float pos_weight;   // <= 0: N_neg / N_pos of the training set
};

// device copy of a trained network for inference inside a sim
struct MlpDevice {
    float *w = nullptr;       // fp32 parameters
    uint16_t *wb = nullptr;   // bf16 copies
    float *mean = nullptr, *istd = nullptr;
    uint16_t *xb = nullptr, *h1 = nullptr, *h2 = nullptr;
    float *prob = nullptr;
    int8_t *flags_tmp = nullptr;
    int cap = 0;
    bool ready = false;
    MlpDevice();
    ~MlpDevice();
    void set(const float *params, const float *mean, const float *std);
    void reserve(int n);
    void forward(hipStream_t s, int n);
};

void mlp_features(hipStream_t s, const KArgs &a, int bi, int bj, int bk, const int *items, const int *nitems, int n,
                  float *raw, const float *mean, const float *istd, uint16_t *xb);
void mlp_prob_flags(hipStream_t s, const float *prob, const int *items, int n, float threshold, int8_t *flags);
void mlp_grad(const float *xnorm, const uint8_t *y, int n, float pw, const float *params, float *grad_out,
              float *loss_out);
void mlp_train(const float *raw, const uint8_t *y, long n, const MlpHparams &hp, float *params, float *mean_out,
               float *std_out, float *loss_epochs);
void mlp_infer(const float *raw, long n, const float *params, const float *mean, const float *std, float *prob);

// rows of one allocation-free inference call (the fixed device scratch holds
// their bf16 inputs and hidden layers)
#ifndef IC_MLP_NOALLOC_ROWS
#define IC_MLP_NOALLOC_ROWS 4096
#endif
// Inference on device arrays with no allocation: scratch is a file-scope
// device array of mlp.hip, shared by every call on a device.  Enqueued on s.
void mlp_infer_noalloc(const float *raw, long n, const float *params, const float *mean, const float *std,
                       float *prob, hipStream_t s);
