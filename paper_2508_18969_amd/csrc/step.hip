// Shape lookup of the fused chemistry-update kernel (its instantiations live
// in step_<format>.hip) and the weight-packing kernels.
#include "common.h"
#include "internal.h"

namespace chemdnn {

bool find_layout(int p, int h1, int h2, int h3, NetLayout *out) {
  switch (p) {
    case P_FP32: return find_layout_fp32(h1, h2, h3, out);
    case P_BF16: return find_layout_bf16(h1, h2, h3, out);
    case P_FP16: return find_layout_fp16(h1, h2, h3, out);
    case P_FP8: return find_layout_fp8(h1, h2, h3, out);
    default: return false;
  }
}

bool find_prop_layout(int p, int h1, int h2, int h3, NetLayout *out) {
  switch (p) {
    case P_FP32: return find_prop_layout_fp32(h1, h2, h3, out);
    case P_BF16: return find_prop_layout_bf16(h1, h2, h3, out);
    case P_FP16: return find_prop_layout_fp16(h1, h2, h3, out);
    default: return false;
  }
}

__device__ __forceinline__ float umaxf(float a, float b) { return a > b ? a : b; }

// ------------------------------------------------------------------ packing
__global__ void weight_amax_kernel(const float *W, int64_t count, uint32_t *amax_bits) {
  float m = 0.0f;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < count;
       i += (int64_t)gridDim.x * blockDim.x)
    m = umaxf(m, __builtin_fabsf(W[i]));
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) m = umaxf(m, __shfl_xor(m, o));
  if ((threadIdx.x & 63) == 0) atomicMax(amax_bits, __builtin_bit_cast(uint32_t, m));
}

// Weight scales: the smallest power of two s with amax / s <= 448 (FP8),
// computed in FP64; 1 for the other formats.  Also forms the accumulator
// multipliers act_scale * w_scale.  Writes into the FConst block.
__global__ void pow2_scale_kernel(const uint32_t *amax_bits, float *fc, int nl, int fp8) {
  int l = threadIdx.x;
  if (l >= nl) return;
  float s = 1.0f;
  if (fp8) {
    double amax = (double)__builtin_bit_cast(float, amax_bits[l]);
    if (amax > 0.0) {
      int e;
      double m = frexp(amax / 448.0, &e);
      int k = (m == 0.5) ? e - 1 : e;
      s = (float)ldexp(1.0, k);
    }
  }
  fc[FConst::WSCALE + l] = s;
  fc[FConst::SOUT + l] = fc[FConst::ASCALE + l] * s;
}

// Packs W [N][K] (row-major FP32) into fragment order: fragment (rb, q) of
// lane l, slot j holds W[16 rb + l%16 - rowshift][frag_feature(q, l/16, j)] / s,
// zero outside the matrix.  fmt: 0 FP32, 1 BF16, 2 FP16, 3 FP8 E4M3.
__global__ void pack_kernel(const float *W, int N, int K, int rowshift, int R, int NQ, int KS,
                            int fmt, const float *w_scale, uint8_t *dst) {
  const int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;   // (rb, q, lane)
  if (t >= (int64_t)R * NQ * 64) return;
  const int lane = (int)(t % 64);
  const int q = (int)((t / 64) % NQ);
  const int rb = (int)(t / (64 * (int64_t)NQ));
  const int row = 16 * rb + (lane & 15) - rowshift;
  const float inv = fmt == 3 ? 1.0f / *w_scale : 1.0f;
  const int ne = KS / 4;
  for (int j = 0; j < ne; ++j) {
    const int k = frag_feature(KS, q, lane >> 4, j);
    float v = (row >= 0 && row < N && k < K) ? W[(int64_t)row * K + k] * inv : 0.0f;
    const int64_t e = t * ne + j;
    switch (fmt) {
      case 0: ((float *)dst)[e] = v; break;
      case 1: ((__bf16 *)dst)[e] = (__bf16)v; break;
      case 2: ((_Float16 *)dst)[e] = (_Float16)v; break;
      default: {
        float c = __builtin_amdgcn_fmed3f(v, -448.0f, 448.0f);
        dst[e] = (uint8_t)(__builtin_amdgcn_cvt_pk_fp8_f32(c, 0.0f, 0, false) & 0xff);
      }
    }
  }
}

__global__ void pad_bias_kernel(const float *b, int N, int rowshift, int NP, float *dst) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= NP) return;
  int r = i - rowshift;
  dst[i] = (r >= 0 && r < N) ? b[r] : 0.0f;
}

__global__ void fill_u32_kernel(uint32_t *p, uint32_t v, int64_t n) {
  int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}

hipError_t launch_weight_amax(const float *W, int64_t count, uint32_t *amax_bits, hipStream_t s) {
  int blocks = (int)((count + 255) / 256);
  if (blocks > 1024) blocks = 1024;
  if (blocks < 1) blocks = 1;
  hipLaunchKernelGGL(weight_amax_kernel, dim3(blocks), dim3(256), 0, s, W, count, amax_bits);
  return hipGetLastError();
}
hipError_t launch_pow2_scales(const uint32_t *amax_bits, float *fc, int nl, int fp8,
                              hipStream_t s) {
  hipLaunchKernelGGL(pow2_scale_kernel, dim3(1), dim3(64), 0, s, amax_bits, fc, nl, fp8);
  return hipGetLastError();
}
hipError_t launch_pack(const float *W, int N, int K, int rowshift, int R, int NQ, int KS, int fmt,
                       const float *w_scale, void *dst, hipStream_t s) {
  int64_t threads = (int64_t)R * NQ * 64;
  hipLaunchKernelGGL(pack_kernel, dim3((unsigned)((threads + 255) / 256)), dim3(256), 0, s, W, N,
                     K, rowshift, R, NQ, KS, fmt, w_scale, (uint8_t *)dst);
  return hipGetLastError();
}
hipError_t launch_pad_bias(const float *b, int N, int rowshift, int NP, float *dst, hipStream_t s) {
  hipLaunchKernelGGL(pad_bias_kernel, dim3((NP + 255) / 256), dim3(256), 0, s, b, N, rowshift, NP,
                     dst);
  return hipGetLastError();
}
hipError_t launch_fill_u32(uint32_t *p, uint32_t v, int64_t n, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(fill_u32_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, p, v, n);
  return hipGetLastError();
}

}  // namespace chemdnn
