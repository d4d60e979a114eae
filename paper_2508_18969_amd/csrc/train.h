// Training path of the chemistry net (FP32): forward with saved
// pre-activations, MSE loss, hand-written backward and Adam.  Host-side
// declarations shared with the C-ABI layer.
#pragma once
#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

namespace chemdnn {

// Device scratch carved from the caller's workspace, sized for max_batch.
struct TrainScratch {
  int64_t cap;            // max batch
  float *x;               // [D][cap] normalised inputs
  float *z;               // [H1+H2+H3][cap] pre-activations
  float *out;             // [S][cap] network output
  float *dz[2];           // [max hidden or S][cap] ping-pong gradients
  float *part;            // weight-gradient partials: 32 copies of the largest layer's weights
  float *bpart;           // bias-gradient partials [up to 256 splits][max layer width]
  float *lpart;           // [1024] loss partial sums
};

size_t train_scratch_bytes(const int *widths, int64_t max_batch);
void train_scratch_layout(TrainScratch *t, uint8_t *base, const int *widths, int64_t max_batch);
hipError_t train_prepare();

hipError_t train_mlp_forward(const int *widths, int64_t B, int64_t ld, const float *x,
                             const float *params, float *out, float *saved, TrainScratch *t,
                             hipStream_t s);
hipError_t train_mlp_backward(const int *widths, int64_t B, int64_t ld, const float *x,
                              const float *params, const float *saved, const float *grad_out,
                              float *grad_params, float *grad_x, TrainScratch *t, hipStream_t s);
hipError_t train_step(const int *widths, int64_t B, int64_t ld, const double *T, const double *P,
                      const double *Y, const float *target, float *params, float *grads,
                      float *adam_m, float *adam_v, int64_t step, float lr, bool recompute,
                      float *loss, const float *fc, const double *dc, TrainScratch *t,
                      hipStream_t s);

}  // namespace chemdnn
