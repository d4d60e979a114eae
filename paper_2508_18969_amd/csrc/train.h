// Training path of the chemistry net (FP32): forward with saved
// pre-activations, MSE loss, hand-written backward and Adam.  Host-side
// declarations shared with the C-ABI layer.
#pragma once
#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

namespace chemdnn {

// Device scratch carved from the caller's workspace.  The per-sample
// buffers hold one chunk of `ld` samples: the whole batch (ld = max_batch),
// or, with activation recomputation, recompute_chunk samples - a training
// step then runs forward and backward chunk by chunk and accumulates the
// gradient, and only one chunk's pre-activations ever exist.
struct TrainScratch {
  int64_t cap;            // max batch
  int64_t ld;             // samples per chunk (leading dimension of the buffers below)
  float *x;               // [D][ld] normalised inputs
  float *z;               // [H1+H2+H3][ld] pre-activations
  float *out;             // [S][ld] network output
  float *dz[2];           // [max hidden or S][ld] ping-pong gradients
  float *part;            // weight-gradient partials: 32 copies of the largest layer's weights
  float *bpart;           // bias-gradient partials [up to 256 splits][max layer width]
  float *lpart;           // [1024] loss partial sums of a chunk
  double *closs;          // [ceil(cap / ld)] loss sum of each chunk
};

// chunk = 0: the whole batch at once; > 0: chunks of that many samples.
size_t train_scratch_bytes(const int *widths, int64_t max_batch, int64_t chunk);
void train_scratch_layout(TrainScratch *t, uint8_t *base, const int *widths, int64_t max_batch,
                          int64_t chunk);
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
