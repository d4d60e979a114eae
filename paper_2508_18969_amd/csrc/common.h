// Device-side building blocks of the chemistry-update kernels (gfx950 only).
//
// Matrix-core fragment layout used throughout
// -------------------------------------------
// Every dense layer is computed transposed, Z^T = W A^T: the weights are the
// MFMA "A" operand (16 output features x KS input features per instruction
// group) and the activations are the "B" operand (KS input features x 16
// cells).  A 16x16 accumulator tile holds, in lane l, cell (l % 16) and output
// features 4*(l / 16) + r, r = 0..3.
//
// A k-step covers KS input features.  In both operands lane l owns a
// fragment of KS/4 elements; slot j of lane-group g = l / 16 carries input
// feature
//        f(q, g, j) = KS*q + 16*(j / 4) + 4*g + (j % 4)
// (any bijection works as long as both operands use the same one).  With this
// map the four accumulator values a lane holds for an output row-block are
// exactly four consecutive slots of the next layer's B fragment of the same
// lane, so a layer's result is written to LDS by the lane that computed it,
// without any shuffle, and read back by the next layer as one 16-byte
// (32-byte for FP8) LDS load per lane.  Weights are packed into the same
// per-lane fragment order once at initialisation, so each wave streams them
// from L2 with fully coalesced 1 KiB (2 KiB) loads.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace chemdnn {

typedef float f4 __attribute__((ext_vector_type(4)));
typedef int i4 __attribute__((ext_vector_type(4)));
typedef int i8v __attribute__((ext_vector_type(8)));
typedef __bf16 bf8 __attribute__((ext_vector_type(8)));
typedef _Float16 h8 __attribute__((ext_vector_type(8)));
typedef double double2v __attribute__((ext_vector_type(2)));

// tanh-form GELU, 0.5 x (1 + tanh(v)), v = sqrt(2/pi)(x + 0.044715 x^3),
// evaluated as x / (1 + 2^(-2 v log2 e)) (the identity 0.5(1 + tanh v) =
// 1/(1 + e^(-2v))): one exp2 and one reciprocal, no cancellation, and the
// correct limits 0 and x for large |x|.
constexpr double kSqrt2OverPi = 0.7978845608028654;
constexpr double kGeluCubic = 0.044715;
// Molar gas constant, J/(mol K) (exact in the SI: N_A k_B).
constexpr double kRGas = 8.31446261815324;
constexpr float kLog2e = 1.4426950408889634f;
constexpr float kLn2 = 0.6931471805599453f;
constexpr float kG1 = (float)(-2.0 * kSqrt2OverPi * 1.4426950408889634);
constexpr float kG3 = (float)(-2.0 * kSqrt2OverPi * 1.4426950408889634 * kGeluCubic);

__device__ __forceinline__ float gelu(float x) {
  float p = __builtin_fmaf(x * x, kG3, kG1);
  float e = __builtin_amdgcn_exp2f(x * p);
  return x * __builtin_amdgcn_rcpf(1.0f + e);
}

// The same GELU of the first n tiles of z (four values each, n <= NT), in
// place, one operation at a time across all the values: each value's chain
// of seven dependent operations (two of them transcendental) is interleaved
// with the other values' instead of issuing back to back.  The empty asm
// statements after each stage keep that order.  Bitwise equal to gelu().
template <int NT> __device__ __forceinline__ void gelu_stages(f4 (&z)[NT], int n) {
  f4 t[NT];
  auto pin = [&]() {
#pragma unroll
    for (int u = 0; u < NT; ++u)
      if (u < n) asm volatile("" : "+v"(t[u]));
  };
#pragma unroll
  for (int u = 0; u < NT; ++u)
    if (u < n) t[u] = z[u] * z[u];
  pin();
#pragma unroll
  for (int u = 0; u < NT; ++u)
#pragma unroll
    for (int r = 0; r < 4; ++r)
      if (u < n) t[u][r] = __builtin_fmaf(t[u][r], kG3, kG1);
  pin();
#pragma unroll
  for (int u = 0; u < NT; ++u)
    if (u < n) t[u] = z[u] * t[u];
  pin();
#pragma unroll
  for (int u = 0; u < NT; ++u)
#pragma unroll
    for (int r = 0; r < 4; ++r)
      if (u < n) t[u][r] = __builtin_amdgcn_exp2f(t[u][r]);
  pin();
#pragma unroll
  for (int u = 0; u < NT; ++u)
    if (u < n) t[u] = 1.0f + t[u];
  pin();
#pragma unroll
  for (int u = 0; u < NT; ++u)
#pragma unroll
    for (int r = 0; r < 4; ++r)
      if (u < n) t[u][r] = __builtin_amdgcn_rcpf(t[u][r]);
  pin();
#pragma unroll
  for (int u = 0; u < NT; ++u)
    if (u < n) z[u] = z[u] * t[u];
}

// Tabulated GELU (Sec. 3.3.2): 0 below -3, x above 3; in between, the
// interval i = floor((x + 3) / 0.01) holds the second-order expansion
// c0 + c1 d + c2 d^2 about its midpoint (d = x - midpoint).  `tab` is the
// LDS copy of the table, (c0, c1, c2, 0) per interval.
__device__ __forceinline__ float gelu_tab(float x, const f4 *tab) {
  int i = (int)((x + 3.0f) * 100.0f);
  i = i < 0 ? 0 : (i > 599 ? 599 : i);
  const float d = x - __builtin_fmaf((float)i, 0.01f, -2.995f);
  const f4 c = tab[i];
  const float y = __builtin_fmaf(__builtin_fmaf(c[2], d, c[1]), d, c[0]);
  return x < -3.0f ? 0.0f : (x > 3.0f ? x : y);
}

// The same table with FP16 coefficients (c0, c1, c2, 0) per interval (the
// paper implements FP32 and FP16 tabulation, Sec. 3.3.2): 8 bytes per
// interval, converted to FP32 on use; the polynomial is evaluated in FP32.
typedef _Float16 h4v __attribute__((ext_vector_type(4)));
__device__ __forceinline__ float gelu_tab16(float x, const h4v *tab) {
  int i = (int)((x + 3.0f) * 100.0f);
  i = i < 0 ? 0 : (i > 599 ? 599 : i);
  const float d = x - __builtin_fmaf((float)i, 0.01f, -2.995f);
  const h4v c = tab[i];
  const float y = __builtin_fmaf(__builtin_fmaf((float)c[2], d, (float)c[1]), d, (float)c[0]);
  return x < -3.0f ? 0.0f : (x > 3.0f ? x : y);
}

// Y^lam in FP32 from an FP64 mass fraction, via the exponent split
// y = m 2^e (m in [1, 2)) so that values far below FLT_MIN keep their
// magnitude.  Non-positive, NaN or subnormal-double inputs give 0
// (y^lam < 1e-30 for subnormal doubles).
__device__ __forceinline__ float ypow(double y, float lam) {
  const uint64_t bits = __builtin_bit_cast(uint64_t, y);
  const int ef = (int)((bits >> 52) & 0x7ff);
  const double m = __builtin_bit_cast(double, (bits & 0x000fffffffffffffull) | 0x3ff0000000000000ull);
  const float l2 = __builtin_amdgcn_logf((float)m) + (float)(ef - 1023);
  const float r = __builtin_amdgcn_exp2f(lam * l2);
  // selects, no branches: 0 for y <= 0, NaN or subnormal; inf for +inf
  return (y > 0.0 && ef != 0) ? (ef == 0x7ff ? __builtin_inff() : r) : 0.0f;
}

// The change Y* - Y of one mass fraction y whose Box-Cox value moves by
// wv = lam delta (delta = the network output after the output statistics):
// Y* = (max(0, y^lam + wv))^(1/lam).  For a small step it is taken relative to
// y, Y* - y = y ((1 + t)^(1/lam) - 1) with t = wv / y^lam, so the change keeps
// its relative accuracy.  The caller adds y back: y + y e with e = (1 + t)^(1/lam)
// - 1 cancels by 1/(1 + e), so the relative form is used only for t >= -0.1
// (1 + e >= 0.9^10 = 0.35, at most a 1.9x loss; for t > 0 nothing cancels);
// a larger decrease takes Y* itself.  Both forms are evaluated without
// branches on the hardware log2 / exp2.
__device__ __forceinline__ double inv_change(double y, float wv, float lam, float inv_lam) {
  const float b = ypow(y, lam);
  const float t = wv * __builtin_amdgcn_rcpf(b);
  const bool small = b > 0.0f && t >= -0.1f && t <= 0.5f;
  const float u = 1.0f + t;
  // log2(1 + t) = log2(u) t / (u - 1) for the rounded u (exact when u == 1)
  // (both arms of each choice are computed and pinned, so that the choice is
  // a select, not a branch)
  float l1a = t * kLog2e, l1b = __builtin_amdgcn_logf(u) * (t * __builtin_amdgcn_rcpf(u - 1.0f));
  const float base = b + wv;
  float lb = __builtin_amdgcn_logf(base);
  asm volatile("" : "+v"(l1a), "+v"(l1b), "+v"(lb));
  const float z = (small ? (u == 1.0f ? l1a : l1b) : lb) * inv_lam;
  const float e = __builtin_amdgcn_exp2f(z);
  // 2^z - 1 = (e - 1) z / log2(e) for the rounded e = 2^z
  float ema = z * kLn2, emb = (e - 1.0f) * (z * __builtin_amdgcn_rcpf(__builtin_amdgcn_logf(e)));
  asm volatile("" : "+v"(ema), "+v"(emb));
  const float em1 = e == 1.0f ? ema : emb;
  double dys = y * (double)em1, dyl = (base > 0.0f ? (double)e : 0.0) - y;
  asm volatile("" : "+v"(dys), "+v"(dyl));
  return small ? dys : dyl;
}

// Sums and reductions over the lane quartet {l, l ^ 16, l ^ 32, l ^ 48} (the
// four lanes of one cell) with the row-swap permutes: swapping odd rows of
// one copy with even rows of another leaves, per lane, its own row's value
// in one result and the partner row's in the other.
__device__ __forceinline__ double quad_sum(double v) {
  uint64_t u = __builtin_bit_cast(uint64_t, v);
  auto l = __builtin_amdgcn_permlane16_swap((uint32_t)u, (uint32_t)u, false, false);
  auto h = __builtin_amdgcn_permlane16_swap((uint32_t)(u >> 32), (uint32_t)(u >> 32), false, false);
  v = __builtin_bit_cast(double, (uint64_t)l[0] | ((uint64_t)h[0] << 32)) +
      __builtin_bit_cast(double, (uint64_t)l[1] | ((uint64_t)h[1] << 32));
  u = __builtin_bit_cast(uint64_t, v);
  l = __builtin_amdgcn_permlane32_swap((uint32_t)u, (uint32_t)u, false, false);
  h = __builtin_amdgcn_permlane32_swap((uint32_t)(u >> 32), (uint32_t)(u >> 32), false, false);
  return __builtin_bit_cast(double, (uint64_t)l[0] | ((uint64_t)h[0] << 32)) +
         __builtin_bit_cast(double, (uint64_t)l[1] | ((uint64_t)h[1] << 32));
}
__device__ __forceinline__ uint32_t quad_or(uint32_t v) {
  auto a = __builtin_amdgcn_permlane16_swap(v, v, false, false);
  v = a[0] | a[1];
  auto b = __builtin_amdgcn_permlane32_swap(v, v, false, false);
  return b[0] | b[1];
}

// ---------------------------------------------------------------- operand formats
// KS: input features per k-step; FRAG: bytes per lane per fragment;
// EB: bytes per element; SCALED: operands carry power-of-two scales.
struct OpF32 {
  static constexpr int KS = 16, FRAG = 16, EB = 4;
  static constexpr bool SCALED = false;
  typedef i4 frag_t;
  static __device__ __forceinline__ f4 mma(const frag_t &a, const frag_t &b, f4 c) {
    // bit-cast whole vectors: a bit-cast of a single vector element collapses
    // every element to the first one in this compiler
    const f4 af = __builtin_bit_cast(f4, a), bf = __builtin_bit_cast(f4, b);
#pragma unroll
    for (int r = 0; r < 4; ++r) c = __builtin_amdgcn_mfma_f32_16x16x4f32(af[r], bf[r], c, 0, 0, 0);
    return c;
  }
  // store 4 values (already scaled) into 4 consecutive slots
  static __device__ __forceinline__ void store4(uint8_t *p, f4 v) { *(f4 *)p = v; }
  // the operand value a stored v becomes, as FP32
  static __device__ __forceinline__ float q(float v) { return v; }
  static __device__ __forceinline__ void store4s(uint8_t *p, f4 v, float) { store4(p, v); }
};

struct OpBF16 {
  static constexpr int KS = 32, FRAG = 16, EB = 2;
  static constexpr bool SCALED = false;
  typedef i4 frag_t;
  static __device__ __forceinline__ f4 mma(const frag_t &a, const frag_t &b, f4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf8, a),
                                                   __builtin_bit_cast(bf8, b), c, 0, 0, 0);
  }
  static __device__ __forceinline__ void store4(uint8_t *p, f4 v) {
    typedef __bf16 b4 __attribute__((ext_vector_type(4)));
    b4 o;
    o[0] = (__bf16)v[0]; o[1] = (__bf16)v[1]; o[2] = (__bf16)v[2]; o[3] = (__bf16)v[3];
    *(b4 *)p = o;
  }
  static __device__ __forceinline__ float q(float v) { return (float)(__bf16)v; }
  static __device__ __forceinline__ void store4s(uint8_t *p, f4 v, float) { store4(p, v); }
};

struct OpF16 {
  static constexpr int KS = 32, FRAG = 16, EB = 2;
  static constexpr bool SCALED = false;
  typedef i4 frag_t;
  static __device__ __forceinline__ f4 mma(const frag_t &a, const frag_t &b, f4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x32_f16(__builtin_bit_cast(h8, a),
                                                  __builtin_bit_cast(h8, b), c, 0, 0, 0);
  }
  static __device__ __forceinline__ void store4(uint8_t *p, f4 v) {
    typedef _Float16 q4 __attribute__((ext_vector_type(4)));
    q4 o;
    o[0] = (_Float16)v[0]; o[1] = (_Float16)v[1]; o[2] = (_Float16)v[2]; o[3] = (_Float16)v[3];
    *(q4 *)p = o;
  }
  static __device__ __forceinline__ float q(float v) { return (float)(_Float16)v; }
  static __device__ __forceinline__ void store4s(uint8_t *p, f4 v, float) { store4(p, v); }
};

// OCP FP8 E4M3 with the K=128 f8f6f4 matrix instruction (unit block scales:
// the E8M0 scale operand 127 encodes 2^0).  The hardware conversion does not
// saturate (values past 464 become NaN), so values are clamped to +-448 first.
struct OpF8 {
  static constexpr int KS = 128, FRAG = 32, EB = 1;
  static constexpr bool SCALED = true;
  typedef i8v frag_t;
  static __device__ __forceinline__ f4 mma(const frag_t &a, const frag_t &b, f4 c) {
    return __builtin_amdgcn_mfma_scale_f32_16x16x128_f8f6f4(a, b, c, 0, 0, 0, 127, 0, 127);
  }
  static __device__ __forceinline__ uint32_t pack4(f4 v) {
    float a = __builtin_amdgcn_fmed3f(v[0], -448.0f, 448.0f);
    float b = __builtin_amdgcn_fmed3f(v[1], -448.0f, 448.0f);
    float c = __builtin_amdgcn_fmed3f(v[2], -448.0f, 448.0f);
    float d = __builtin_amdgcn_fmed3f(v[3], -448.0f, 448.0f);
    uint32_t w = __builtin_amdgcn_cvt_pk_fp8_f32(a, b, 0, false);
    return __builtin_amdgcn_cvt_pk_fp8_f32(c, d, w, true);
  }
  static __device__ __forceinline__ void store4(uint8_t *p, f4 v) { *(uint32_t *)p = pack4(v); }
  // pack4 of v / a for a power of two a, with the division done by the
  // scaled conversion: the clamp moves to +-448 a, and every value rounds as
  // in pack4(v / a) (checked on the device over the whole FP32 range)
  static __device__ __forceinline__ void store4s(uint8_t *p, f4 v, float a) {
    typedef short s2 __attribute__((ext_vector_type(2)));
    const float b = 448.0f * a;
    s2 w = {0, 0};
    w = __builtin_amdgcn_cvt_scalef32_pk_fp8_f32(w, __builtin_amdgcn_fmed3f(v[0], -b, b),
                                                 __builtin_amdgcn_fmed3f(v[1], -b, b), a, false);
    w = __builtin_amdgcn_cvt_scalef32_pk_fp8_f32(w, __builtin_amdgcn_fmed3f(v[2], -b, b),
                                                 __builtin_amdgcn_fmed3f(v[3], -b, b), a, true);
    *(s2 *)p = w;
  }
  // the same clamp and conversion as pack4, decoded back to FP32
  static __device__ __forceinline__ float q(float v) {
    const uint32_t w = __builtin_amdgcn_cvt_pk_fp8_f32(__builtin_amdgcn_fmed3f(v, -448.0f, 448.0f),
                                                       0.0f, 0, false);
    return __builtin_amdgcn_cvt_f32_fp8((int)w, 0);
  }
};

template <int A, int B> struct Max { static constexpr int v = A > B ? A : B; };
constexpr int roundup(int x, int m) { return (x + m - 1) / m * m; }

// Input feature held in slot j of lane-group g in k-step q.
__host__ __device__ constexpr int frag_feature(int KS, int q, int g, int j) {
  return KS * q + 16 * (j >> 2) + 4 * g + (j & 3);
}

}  // namespace chemdnn
