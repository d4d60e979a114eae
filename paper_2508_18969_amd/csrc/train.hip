// Training kernels (FP32): a strided MFMA GEMM with fused epilogues,
// deterministic split-K weight gradients, MSE loss and Adam.
//
// Forward  z_l = W_l a_(l-1) + b_l, a_l = GELU(z_l) (GELU is applied inside
//          the next GEMM's operand loader, so only z_l is stored);
// backward dW_l = dZ_l a_(l-1)^T (split over the batch, partials summed in a
//          fixed order), db_l = row sums of dZ_l, dZ_(l-1) = (W_l^T dZ_l) *
//          GELU'(z_(l-1)) fused in the GEMM epilogue.  No floating-point
//          atomics anywhere, so gradients are bitwise reproducible.
#include "common.h"
#include "internal.h"
#include "train.h"

namespace chemdnn {

namespace {

// Weight-gradient batch splits: the partials scratch holds kMaxSplit copies
// of the largest layer; smaller layers use up to kMaxSplitAll splits of the
// same scratch, at least kMinSplitBatch batch entries each.
constexpr int kMaxSplit = 32;
constexpr int kMaxSplitAll = 256;
constexpr int kMinSplitBatch = 256;
constexpr int kSplitTarget = 1024;     // workgroups to aim for

// d/dx of the tanh-form GELU with s = 0.5 (1 + tanh v) = 1/(1 + e^(-2v)):
// GELU' = s + x * 2 s (1 - s) * sqrt(2/pi) (1 + 3 * 0.044715 x^2).
__device__ __forceinline__ float gelu_grad(float x) {
  float p = __builtin_fmaf(x * x, kG3, kG1);
  float s = __builtin_amdgcn_rcpf(1.0f + __builtin_amdgcn_exp2f(x * p));
  float dv = (float)kSqrt2OverPi * __builtin_fmaf(3.0f * (float)kGeluCubic, x * x, 1.0f);
  return __builtin_fmaf(x * 2.0f * s * (1.0f - s), dv, s);
}

enum { EPI_FWD = 0, EPI_DA = 1, EPI_PART = 2 };

// Workgroup ids are dealt round-robin to the 8 XCDs, each with its own L2.
// Tile (x, y) of workgroup id in an nx x ny grid such that the ny tiles of a
// column x run back to back on one XCD (when nx is a multiple of 8): the
// operand panel they share is fetched into that XCD's L2 once.
__device__ __forceinline__ void xcd_tile(int id, int nx, int ny, int &x, int &y) {
  if (nx % 8 == 0) {
    const int xcd = id & 7, j = id >> 3;
    y = j % ny;
    x = (j / ny) * 8 + xcd;
  } else {
    x = id % nx;
    y = id / nx;
  }
}

struct GemmArgs {
  const float *A, *B;
  float *C;
  int64_t sam, sak, sbk, sbn, scm, scn;
  int M, N;
  int64_t K, kchunk;
  int gelu_b;              // apply GELU to B operand values on load
  const float *bias;       // EPI_FWD: [M]
  const float *zprev;      // EPI_DA: multiply by GELU'(zprev[m * scm + n * scn]) if set
  int64_t part_stride;     // EPI_PART: offset of split z's partial block
  float *bpart;            // weight-gradient partials: also the row sums of A, [split][M], or NULL
};

// C = A B over one K-split; 64x64 output tile, four waves of 32x32, the
// 16x16x4 FP32 matrix instruction.
template <int EPI>
__global__ __launch_bounds__(256) void gemm_kernel(GemmArgs g) {
  __shared__ float As[16][65], Bs[16][65];
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6, wm = w >> 1, wn = w & 1;
  const int64_t m0 = (int64_t)blockIdx.y * 64, n0 = (int64_t)blockIdx.x * 64;
  const int64_t k0 = (int64_t)blockIdx.z * g.kchunk;
  const int64_t k1 = (k0 + g.kchunk < g.K) ? k0 + g.kchunk : g.K;
  f4 acc[2][2];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) acc[i][j] = f4{0.f, 0.f, 0.f, 0.f};
  const bool a_kfast = g.sak == 1, b_nfast = g.sbn == 1;
  for (int64_t kb = k0; kb < k1; kb += 16) {
#pragma unroll
    for (int e0 = 0; e0 < 1024; e0 += 256) {
      const int e = e0 + tid;
      int m, k;
      if (a_kfast) { m = e >> 4; k = e & 15; } else { m = e & 63; k = e >> 6; }
      const int64_t gm = m0 + m, gk = kb + k;
      As[k][m] = (gm < g.M && gk < k1) ? g.A[gm * g.sam + gk * g.sak] : 0.0f;
    }
#pragma unroll
    for (int e0 = 0; e0 < 1024; e0 += 256) {
      const int e = e0 + tid;
      int n, k;
      if (b_nfast) { k = e >> 6; n = e & 63; } else { n = e >> 4; k = e & 15; }
      const int64_t gn = n0 + n, gk = kb + k;
      float v = (gn < g.N && gk < k1) ? g.B[gk * g.sbk + gn * g.sbn] : 0.0f;
      Bs[k][n] = g.gelu_b ? gelu(v) : v;
    }
    __syncthreads();
#pragma unroll
    for (int k4 = 0; k4 < 4; ++k4) {
      const int kk = 4 * k4 + (lane >> 4);
      const float a0 = As[kk][wm * 32 + (lane & 15)], a1 = As[kk][wm * 32 + 16 + (lane & 15)];
      const float b0 = Bs[kk][wn * 32 + (lane & 15)], b1 = Bs[kk][wn * 32 + 16 + (lane & 15)];
      acc[0][0] = __builtin_amdgcn_mfma_f32_16x16x4f32(a0, b0, acc[0][0], 0, 0, 0);
      acc[0][1] = __builtin_amdgcn_mfma_f32_16x16x4f32(a0, b1, acc[0][1], 0, 0, 0);
      acc[1][0] = __builtin_amdgcn_mfma_f32_16x16x4f32(a1, b0, acc[1][0], 0, 0, 0);
      acc[1][1] = __builtin_amdgcn_mfma_f32_16x16x4f32(a1, b1, acc[1][1], 0, 0, 0);
    }
    __syncthreads();
  }
  float *C = g.C + (EPI == EPI_PART ? blockIdx.z * g.part_stride : 0);
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int64_t m = m0 + wm * 32 + i * 16 + 4 * (lane >> 4) + r;
        const int64_t n = n0 + wn * 32 + j * 16 + (lane & 15);
        if (m < g.M && n < g.N) {
          float v = acc[i][j][r];
          const int64_t o = m * g.scm + n * g.scn;
          if (EPI == EPI_FWD) v += g.bias[m];
          if (EPI == EPI_DA && g.zprev) v *= gelu_grad(g.zprev[o]);
          C[o] = v;
        }
      }
}

// Weight-gradient partial of one K-split, for operands whose reduction index
// (the batch) is contiguous: C[m][n] = sum_k A[m][k] B'[n][k], B' = GELU(B) if
// gelu_b.  The workgroup's 64x64 tile is computed by each of its four waves
// over a quarter of the split (straight from global memory: each lane loads 4
// consecutive k of one row, and the four 16x16x4 products of a 16-k block take
// them in turn - the same k permutation on both operands), then the four
// partial tiles are summed in LDS in wave order.  Requires A and B rows 16-byte
// aligned (leading dimensions multiples of 4).
//
// One-dimensional grid of tn x tm tiles x nsplit splits: the tiles of a split
// (which read the same batch range) run back to back on one XCD.
__global__ __launch_bounds__(256) void dw_kernel(GemmArgs g, int tn, int tm, int nsplit) {
  __shared__ float red[2][64][65];
  __shared__ float rsl[4][4][64];       // row sums of A per wave and lane group
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6, g4 = lane >> 4, c16 = lane & 15;
  int zt, tile;
  xcd_tile(blockIdx.x, nsplit, tn * tm, zt, tile);
  const int bx = tile % tn, by = tile / tn;
  const int64_t m0 = (int64_t)by * 64, n0 = (int64_t)bx * 64;
  const int64_t k0 = (int64_t)zt * g.kchunk;
  const int64_t k1 = (k0 + g.kchunk < g.K) ? k0 + g.kchunk : g.K;
  const int64_t ks = ((g.kchunk + 3) / 4 + 15) / 16 * 16;          // per wave, whole 16-k blocks
  const int64_t kb0 = k0 + w * ks;
  const int64_t kb1 = (kb0 + ks < k1) ? kb0 + ks : k1;
  f4 acc[4][4];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) acc[i][j] = f4{0.f, 0.f, 0.f, 0.f};
  // the rows this lane reads (clamped into range; their values are zeroed)
  int64_t ra[4], rb[4];
  bool va[4], vb[4];
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const int64_t m = m0 + 16 * i + c16, n = n0 + 16 * i + c16;
    va[i] = m < g.M;
    vb[i] = n < g.N;
    ra[i] = (va[i] ? m : 0) * g.sam;
    rb[i] = (vb[i] ? n : 0) * g.sbn;
  }
  float rs[4] = {0.f, 0.f, 0.f, 0.f};        // row sums of A (the bias gradient)
  for (int64_t kb = kb0; kb < kb1; kb += 16) {
    const int64_t k = kb + 4 * g4;
    f4 a[4], b[4];
    if (kb + 16 <= kb1) {
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        a[i] = *(const f4 *)(g.A + ra[i] + k);
        b[i] = *(const f4 *)(g.B + rb[i] + k);
      }
    } else {
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          a[i][e] = k + e < kb1 ? g.A[ra[i] + k + e] : 0.0f;
          b[i][e] = k + e < kb1 ? g.B[rb[i] + k + e] : 0.0f;
        }
    }
#pragma unroll
    for (int i = 0; i < 4; ++i) {
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        if (!va[i]) a[i][e] = 0.0f;
        float v = vb[i] ? b[i][e] : 0.0f;
        if (g.gelu_b) v = gelu(v);
        // zero past the batch (gelu(0) = 0 as well)
        b[i][e] = (k + e < kb1) ? v : 0.0f;
      }
      rs[i] += (a[i][0] + a[i][1]) + (a[i][2] + a[i][3]);
    }
#pragma unroll
    for (int e = 0; e < 4; ++e)
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j)
          acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[i][e], b[j][e], acc[i][j], 0, 0, 0);
  }
  // row sums: per row, the 16 (wave, lane group) partials in that order
  if (g.bpart && bx == 0) {
#pragma unroll
    for (int i = 0; i < 4; ++i) rsl[w][g4][16 * i + c16] = rs[i];
    __syncthreads();
    if (tid < 64 && m0 + tid < g.M) {
      float t = 0.0f;
      for (int ww = 0; ww < 4; ++ww)
        for (int gg = 0; gg < 4; ++gg) t += rsl[ww][gg][tid];
      g.bpart[zt * (int64_t)g.M + m0 + tid] = t;
    }
  }
  // the waves' partial tiles, summed in wave order ((w0 + w1) + w2) + w3,
  // through LDS in two halves
  auto put = [&](int slot) {
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
      for (int j = 0; j < 4; ++j)
#pragma unroll
        for (int r = 0; r < 4; ++r) red[slot][16 * i + 4 * g4 + r][16 * j + c16] = acc[i][j][r];
  };
  if (w < 2) put(w);
  __syncthreads();
  float v[16];
#pragma unroll
  for (int t = 0; t < 16; ++t) {
    const int e = tid + 256 * t, mm = e >> 6, nn = e & 63;
    v[t] = red[0][mm][nn] + red[1][mm][nn];
  }
  __syncthreads();
  if (w >= 2) put(w - 2);
  __syncthreads();
  float *C = g.C + zt * g.part_stride;
#pragma unroll
  for (int t = 0; t < 16; ++t) {
    const int e = tid + 256 * t, mm = e >> 6, nn = e & 63;
    const int64_t m = m0 + mm, n = n0 + nn;
    float x = v[t];
    x += red[0][mm][nn];
    x += red[1][mm][nn];
    if (m < g.M && n < g.N) C[m * g.scm + n * g.scn] = x;
  }
}

// C = A B (+ epilogue) with the batch as the fast index of B and C, for the
// forward (EPI_FWD: + bias) and the activation gradient (EPI_DA: times
// GELU'(zprev)).  Workgroup tile 64 rows x 256 columns; wave w takes columns
// 64 w .. 64 w + 63 of it as four interleaved 16-column blocks (block j holds
// the columns 4 c + j, c = 0..15), so that every lane loads and stores four
// consecutive columns with one 16-byte access.  Per 16-k step the operand A
// (weights, 64 x 16) is loaded once by the whole workgroup with coalesced
// loads and read from LDS (double-buffered, one barrier per step); B comes
// straight from global memory.  The loads of step k + 1 are issued before the
// products of step k.  Requires B and C rows 16-byte aligned (leading
// dimensions multiples of 4).  One-dimensional grid of nx column tiles x ny
// row tiles: the row tiles of a column tile (which share its B panel) run
// back to back on one XCD.
template <int EPI>
__global__ __launch_bounds__(256) void fc_kernel(GemmArgs g, int nx, int ny) {
  __shared__ __align__(16) float As[2][64][20];   // [buffer][row][k], rows padded to 80 bytes
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6, g4 = lane >> 4, c16 = lane & 15;
  int bx, by;
  xcd_tile(blockIdx.x, nx, ny, bx, by);
  const int64_t m0 = (int64_t)by * 64;
  const int64_t nc = (int64_t)bx * 256 + 64 * w + 4 * c16;   // this lane's first column
  const bool full = nc + 3 < g.N;
  const bool a_kfast = g.sak == 1;
  // element tid + 256 j of the A tile: (row, k) with the contiguous index fastest
  auto a_row = [&](int j) { const int e = tid + 256 * j; return a_kfast ? e >> 4 : e & 63; };
  auto a_k = [&](int j) { const int e = tid + 256 * j; return a_kfast ? e & 15 : e >> 6; };
  float ra[4];
  auto load_a = [&](int64_t k0) {
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int64_t gm = m0 + a_row(j), gk = k0 + a_k(j);
      ra[j] = (gm < g.M && gk < g.K) ? g.A[gm * g.sam + gk * g.sak] : 0.0f;
    }
  };
  auto store_a = [&](int buf) {
#pragma unroll
    for (int j = 0; j < 4; ++j) As[buf][a_row(j)][a_k(j)] = ra[j];
  };
  // raw B of a step: rb[e] = B[k0 + 4 g4 + e][nc .. nc + 3] (zero past K and N)
  f4 rb[4];
  auto load_b = [&](int64_t k0) {
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const int64_t k = k0 + 4 * g4 + e;
      const bool kv = k < g.K;
      const float *bp = g.B + (kv ? k : 0) * g.sbk;
      f4 v;
      if (full) {
        v = *(const f4 *)(bp + nc);
      } else {
#pragma unroll
        for (int j = 0; j < 4; ++j) v[j] = nc + j < g.N ? bp[nc + j] : 0.0f;
      }
      rb[e] = kv ? v : f4{0.f, 0.f, 0.f, 0.f};
    }
  };
  f4 acc[4][4];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) acc[i][j] = f4{0.f, 0.f, 0.f, 0.f};
  load_a(0);
  load_b(0);
  store_a(0);
  __syncthreads();
  int buf = 0;
  for (int64_t k0 = 0; k0 < g.K; k0 += 16) {
    f4 b[4];
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      b[e] = rb[e];
      if (g.gelu_b)
#pragma unroll
        for (int j = 0; j < 4; ++j) b[e][j] = gelu(b[e][j]);
    }
    const bool more = k0 + 16 < g.K;
    if (more) {
      load_a(k0 + 16);
      load_b(k0 + 16);
    }
    // a[i][e] = A[m0 + 16 i + c16][k0 + 4 g4 + e]
    f4 a[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) a[i] = *(const f4 *)&As[buf][16 * i + c16][4 * g4];
#pragma unroll
    for (int e = 0; e < 4; ++e)
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j)
          acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[i][e], b[e][j], acc[i][j], 0, 0, 0);
    // the other buffer was last read before the previous barrier
    if (more) store_a(buf ^ 1);
    __syncthreads();
    buf ^= 1;
  }
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int64_t m = m0 + 16 * i + 4 * g4 + r;
      if (m >= g.M) continue;
      f4 v = {acc[i][0][r], acc[i][1][r], acc[i][2][r], acc[i][3][r]};
      if (EPI == EPI_FWD) v += g.bias[m];
      float *cp = g.C + m * g.scm;
      if (EPI == EPI_DA && g.zprev) {
        const float *zp = g.zprev + m * g.scm;
        if (full) {
          const f4 z = *(const f4 *)(zp + nc);
#pragma unroll
          for (int j = 0; j < 4; ++j) v[j] *= gelu_grad(z[j]);
        } else {
#pragma unroll
          for (int j = 0; j < 4; ++j)
            if (nc + j < g.N) v[j] *= gelu_grad(zp[nc + j]);
        }
      }
      if (full) {
        *(f4 *)(cp + nc) = v;
      } else {
#pragma unroll
        for (int j = 0; j < 4; ++j)
          if (nc + j < g.N) cp[nc + j] = v[j];
      }
    }
}

// Sums of split partials for two outputs in one launch: output o < n0 is
// o0[o] = sum_z p0[z * s0 + o], the next n1 are o1 from p1 likewise.  A
// workgroup takes 64 outputs; its four waves sum a quarter of the splits each,
// in increasing z, and the four quarter sums are added in wave order.  With
// `acc` the sum is added to the output (the gradient of a later chunk).
__global__ __launch_bounds__(256) void reduce_parts2_kernel(const float *p0, int64_t s0, int64_t n0,
                                                            float *o0, const float *p1, int64_t s1,
                                                            int64_t n1, float *o1, int nz, int accum) {
  __shared__ float q[4][64];
  const int l = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int64_t o = blockIdx.x * (int64_t)64 + l;
  const bool first = o < n0, valid = o < n0 + n1;
  const float *p = first ? p0 + o : p1 + (valid ? o - n0 : 0);
  const int64_t st = first ? s0 : s1;
  const int zq = (nz + 3) / 4, z0 = w * zq, z1 = z0 + zq < nz ? z0 + zq : nz;
  float acc = 0.0f;
  if (valid)
    for (int z = z0; z < z1; ++z) acc += p[z * st];
  q[w][l] = acc;
  __syncthreads();
  if (w == 0 && valid) {
    const float t = ((q[0][l] + q[1][l]) + q[2][l]) + q[3][l];
    float *dst = first ? o0 + o : o1 + (o - n0);
    *dst = accum ? *dst + t : t;
  }
}

// out[m] = sum_b dz[m * ld + b] (+= with acc): one workgroup per row, fixed-order tree.
__global__ void rowsum_kernel(const float *dz, int64_t ld, int64_t B, float *out, int acc) {
  __shared__ float red[256];
  const int64_t m = blockIdx.x;
  float s = 0.0f;
  for (int64_t b = threadIdx.x; b < B; b += 256) s += dz[m * ld + b];
  red[threadIdx.x] = s;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[m] = acc ? out[m] + red[0] : red[0];
}

// dO = 2 (o - t) / denom over B samples (denom = batch x species of the whole
// step); per-block partial sums of (o - t)^2.
__global__ void mse_kernel(const float *o, int64_t ldo, const float *t, int64_t ldt, int S,
                           int64_t B, double denom, float *dO, float *lpart) {
  __shared__ float red[256];
  const int64_t n = (int64_t)S * B;
  const float inv = 2.0f / (float)denom;
  float s = 0.0f;
  for (int64_t e = blockIdx.x * 256 + threadIdx.x; e < n; e += (int64_t)gridDim.x * 256) {
    const int64_t sp = e / B, b = e % B;
    const float d = o[sp * ldo + b] - t[sp * ldt + b];
    dO[sp * ldo + b] = d * inv;
    s = __builtin_fmaf(d, d, s);
  }
  red[threadIdx.x] = s;
  __syncthreads();
  for (int off = 128; off > 0; off >>= 1) {
    if ((int)threadIdx.x < off) red[threadIdx.x] += red[threadIdx.x + off];
    __syncthreads();
  }
  if (threadIdx.x == 0) lpart[blockIdx.x] = red[0];
}

// One wave: lane l sums partials l, l + 64, ... in order, then a fixed
// butterfly over the lanes (lane 0's order is the same on every run): the
// loss sum of one chunk.
__global__ void loss_chunk_kernel(const float *lpart, int nb, double *chunk_sum) {
  const int l = threadIdx.x;
  double s = 0.0;
  for (int i = l; i < nb; i += 64) s += (double)lpart[i];
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) s += __shfl_xor(s, o);
  if (l == 0) *chunk_sum = s;
}
// The step's loss: the chunk sums in chunk order, over batch x species.
__global__ void loss_final_kernel(const double *chunk_sum, int nchunks, double denom, float *loss) {
  if (threadIdx.x != 0) return;
  double s = 0.0;
  for (int k = 0; k < nchunks; ++k) s += chunk_sum[k];
  *loss = (float)(s / denom);
}

// Normalised network input from the FP64 state, the same arithmetic as the
// inference kernel's preprocessing.
__global__ void features_kernel(const double *T, const double *P, const double *Y, int64_t ld,
                                int64_t B, int S, const float *fc, const double *dc, float *x,
                                int64_t ldx) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= B) return;
  const float lam = fc[FConst::LAM];
  x[i] = (float)((T[i] - dc[DConst::T_MU]) * dc[DConst::T_IS]);
  x[ldx + i] = (float)((P[i] - dc[DConst::P_MU]) * dc[DConst::P_IS]);
  for (int s = 0; s < S; ++s)
    x[(int64_t)(s + 2) * ldx + i] =
        __builtin_fmaf(ypow(Y[(int64_t)s * ld + i], lam), fc[FConst::ZA + s + 2], fc[FConst::ZC + s + 2]);
}

__global__ void adam_kernel(float *p, const float *g, float *m, float *v, int64_t n, float lr,
                            float c1, float c2) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= n) return;
  const float gi = g[i];
  const float mi = 0.9f * m[i] + 0.1f * gi;
  const float vi = 0.999f * v[i] + 0.001f * gi * gi;
  m[i] = mi;
  v[i] = vi;
  p[i] -= lr * (mi * c1) / (__builtin_sqrtf(vi * c2) + 1e-8f);
}

unsigned blocks_for(int64_t n, int per = 256) { return (unsigned)((n + per - 1) / per); }

hipError_t gemm(int epi, const GemmArgs &g, int nsplit, hipStream_t s) {
  // batch-fast products with 16-byte aligned rows: the direct kernel
  if ((epi == EPI_FWD || epi == EPI_DA) && nsplit == 1 && g.sbn == 1 && g.scn == 1 &&
      g.sbk % 4 == 0 && g.scm % 4 == 0 && ((uintptr_t)g.B | (uintptr_t)g.C) % 16 == 0 &&
      (!g.zprev || (uintptr_t)g.zprev % 16 == 0)) {
    const int nx = (int)blocks_for(g.N, 256), ny = (int)blocks_for(g.M, 64);
    const dim3 grid((unsigned)nx * ny);
    if (epi == EPI_FWD) hipLaunchKernelGGL(fc_kernel<EPI_FWD>, grid, dim3(256), 0, s, g, nx, ny);
    else hipLaunchKernelGGL(fc_kernel<EPI_DA>, grid, dim3(256), 0, s, g, nx, ny);
    return hipGetLastError();
  }
  dim3 grid(blocks_for(g.N, 64), blocks_for(g.M, 64), nsplit);
  switch (epi) {
    case EPI_FWD: hipLaunchKernelGGL(gemm_kernel<EPI_FWD>, grid, dim3(256), 0, s, g); break;
    case EPI_DA: hipLaunchKernelGGL(gemm_kernel<EPI_DA>, grid, dim3(256), 0, s, g); break;
    default: hipLaunchKernelGGL(gemm_kernel<EPI_PART>, grid, dim3(256), 0, s, g); break;
  }
  return hipGetLastError();
}

size_t param_off(const int *w, int l) {
  size_t o = 0;
  for (int i = 0; i < l; ++i) o += (size_t)w[i] * w[i + 1] + w[i + 1];
  return o;
}

int64_t max_layer_weights(const int *w) {
  int64_t m = 0;
  for (int l = 0; l < 4; ++l) m = m > (int64_t)w[l] * w[l + 1] ? m : (int64_t)w[l] * w[l + 1];
  return m;
}

// Batch splits of the weight gradient of an N x K layer: about kSplitTarget
// workgroups of 64 x 64 tiles, at least kMinSplitBatch entries per split, the
// partials within the scratch.  Depends on the shapes only, so results are
// reproducible.
int split_count(const int *w, int64_t B, int N, int K) {
  const int64_t tiles = (int64_t)blocks_for(N, 64) * blocks_for(K, 64);
  int64_t n = (kSplitTarget + tiles - 1) / tiles;
  const int64_t by_batch = (B + kMinSplitBatch - 1) / kMinSplitBatch;
  const int64_t by_space = (int64_t)kMaxSplit * max_layer_weights(w) / ((int64_t)N * K);
  n = n < by_batch ? n : by_batch;
  n = n < by_space ? n : by_space;
  n = n < kMaxSplitAll ? n : kMaxSplitAll;
  n = n >= 8 ? n / 8 * 8 : n;          // whole rounds over the 8 XCDs
  return (int)(n < 1 ? 1 : n);
}

// Forward of the 4-layer net.  z: pre-activations [H1+H2+H3][ldz]; out [S][ldo].
hipError_t forward(const int *w, int64_t B, const float *x, int64_t ldx, const float *params,
                   float *z, int64_t ldz, float *out, int64_t ldo, hipStream_t s) {
  int64_t zoff = 0;
  const float *in = x;
  int64_t ldin = ldx;
  int gelu_in = 0;
  for (int l = 0; l < 4; ++l) {
    const int N = w[l + 1], K = w[l];
    GemmArgs g{};
    g.A = params + param_off(w, l);
    g.sam = K; g.sak = 1;
    g.B = in; g.sbk = ldin; g.sbn = 1;
    g.gelu_b = gelu_in;
    float *dst = (l < 3) ? z + zoff * ldz : out;
    const int64_t ldd = (l < 3) ? ldz : ldo;
    g.C = dst; g.scm = ldd; g.scn = 1;
    g.M = N; g.N = (int)B; g.K = K; g.kchunk = K;
    g.bias = params + param_off(w, l) + (size_t)N * K;
    hipError_t e = gemm(EPI_FWD, g, 1, s);
    if (e != hipSuccess) return e;
    in = dst;
    ldin = ldd;
    gelu_in = 1;
    zoff += (l < 3) ? N : 0;
  }
  return hipSuccess;
}

// Backward given dL/d out (gout [S][ldg]) and the pre-activations z; the
// weight and bias gradients are written, or with `acc` added to gparams.
hipError_t backward(const int *w, int64_t B, const float *x, int64_t ldx, const float *params,
                    const float *z, int64_t ldz, const float *gout, int64_t ldg, float *gparams,
                    float *gx, int64_t ldgx, TrainScratch *t, hipStream_t s, int acc) {
  int64_t zoffs[4] = {0, w[1], (int64_t)w[1] + w[2], 0};
  const float *dZ = gout;
  int64_t lddz = ldg;
  int pp = 0;
  for (int l = 3; l >= 0; --l) {
    const int N = w[l + 1], K = w[l];
    const int nsplit = split_count(w, B, N, K);
    const int64_t kchunk = ((B + nsplit - 1) / nsplit + 15) / 16 * 16;
    const float *ain = (l == 0) ? x : z + zoffs[l - 1] * ldz;
    const int64_t ldain = (l == 0) ? ldx : ldz;
    // dW_l = dZ_l a_(l-1)^T over the batch, split in fixed chunks
    GemmArgs g{};
    g.A = dZ; g.sam = lddz; g.sak = 1;
    g.B = ain; g.sbk = 1; g.sbn = ldain;
    g.gelu_b = (l > 0);
    g.C = t->part; g.scm = K; g.scn = 1;
    g.M = N; g.N = K; g.K = B; g.kchunk = kchunk;
    g.part_stride = (int64_t)N * K;
    hipError_t e;
    float *gW = gparams + param_off(w, l);
    const bool direct = lddz % 4 == 0 && ldain % 4 == 0 && ((uintptr_t)dZ | (uintptr_t)ain) % 16 == 0;
    if (direct) {
      // weight and bias partials in one pass
      g.bpart = t->bpart;
      const int tn = (int)blocks_for(K, 64), tm = (int)blocks_for(N, 64);
      hipLaunchKernelGGL(dw_kernel, dim3((unsigned)(tn * tm * nsplit)), dim3(256), 0, s, g, tn, tm,
                         nsplit);
      e = hipGetLastError();
    } else {
      e = gemm(EPI_PART, g, nsplit, s);
    }
    if (e != hipSuccess) return e;
    // weights and (direct path) biases in one launch
    const int64_t nw = (int64_t)N * K, nb = direct ? N : 0;
    hipLaunchKernelGGL(reduce_parts2_kernel, dim3(blocks_for(nw + nb, 64)), dim3(256), 0, s,
                       (const float *)t->part, nw, nw, gW, (const float *)t->bpart, (int64_t)N, nb,
                       gW + (size_t)N * K, nsplit, acc);
    if (!direct)
      hipLaunchKernelGGL(rowsum_kernel, dim3(N), dim3(256), 0, s, dZ, lddz, B, gW + (size_t)N * K, acc);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    // dZ_(l-1) = (W_l^T dZ_l) * GELU'(z_(l-1)), or grad_x for l = 0
    if (l > 0 || gx) {
      GemmArgs d{};
      d.A = params + param_off(w, l); d.sam = 1; d.sak = K;    // W^T: (k, n) -> W[n][k]
      d.B = dZ; d.sbk = lddz; d.sbn = 1;
      float *dst = (l > 0) ? t->dz[pp] : gx;
      const int64_t ldd = (l > 0) ? t->ld : ldgx;
      d.C = dst; d.scm = ldd; d.scn = 1;
      d.M = K; d.N = (int)B; d.K = N; d.kchunk = N;
      d.zprev = (l > 0) ? z + zoffs[l - 1] * ldz : nullptr;
      if (l > 0 && ldz != ldd) return hipErrorInvalidValue;   // epilogue indexes z like C
      e = gemm(EPI_DA, d, 1, s);
      if (e != hipSuccess) return e;
      dZ = dst;
      lddz = ldd;
      pp ^= 1;
    }
  }
  return hipSuccess;
}

}  // namespace

namespace {

// Samples the per-sample buffers hold: the whole batch, or one chunk.
int64_t chunk_of(int64_t cap, int64_t chunk) { return chunk > 0 && chunk < cap ? chunk : cap; }
int64_t n_chunks(int64_t B, int64_t ld) { return (B + ld - 1) / ld; }

}  // namespace

size_t train_scratch_bytes(const int *w, int64_t cap, int64_t chunk) {
  if (cap <= 0) return 0;
  const int64_t ld = chunk_of(cap, chunk);
  const int64_t H = (int64_t)w[1] + w[2] + w[3];
  int64_t mx = w[4];
  for (int l = 1; l < 4; ++l) mx = mx > w[l] ? mx : w[l];
  size_t f = (size_t)ld * (w[0] + H + w[4] + 2 * mx) + (size_t)kMaxSplit * max_layer_weights(w) +
             (size_t)kMaxSplitAll * mx + 1024;
  return f * sizeof(float) + (size_t)n_chunks(cap, ld) * sizeof(double) + 10 * 256;
}

void train_scratch_layout(TrainScratch *t, uint8_t *base, const int *w, int64_t cap, int64_t chunk) {
  *t = TrainScratch{};
  t->cap = cap;
  if (cap <= 0) return;
  const int64_t ld = chunk_of(cap, chunk);
  t->ld = ld;
  const int64_t H = (int64_t)w[1] + w[2] + w[3];
  int64_t mx = w[4];
  for (int l = 1; l < 4; ++l) mx = mx > w[l] ? mx : w[l];
  auto take = [&](size_t bytes) {
    uint8_t *p = base;
    base += (bytes + 255) / 256 * 256;
    return p;
  };
  t->x = (float *)take((size_t)ld * w[0] * sizeof(float));
  t->z = (float *)take((size_t)ld * H * sizeof(float));
  t->out = (float *)take((size_t)ld * w[4] * sizeof(float));
  t->dz[0] = (float *)take((size_t)ld * mx * sizeof(float));
  t->dz[1] = (float *)take((size_t)ld * mx * sizeof(float));
  t->part = (float *)take((size_t)kMaxSplit * max_layer_weights(w) * sizeof(float));
  t->bpart = (float *)take((size_t)kMaxSplitAll * mx * sizeof(float));
  t->lpart = (float *)take(1024 * sizeof(float));
  t->closs = (double *)take((size_t)n_chunks(cap, ld) * sizeof(double));
}

hipError_t train_prepare() { return hipSuccess; }

// Forward over B samples of x [D][ld]: with `saved` the pre-activations of the
// whole batch go there ([H][ld]); without, chunk by chunk through the scratch.
hipError_t train_mlp_forward(const int *w, int64_t B, int64_t ld, const float *x,
                             const float *params, float *out, float *saved, TrainScratch *t,
                             hipStream_t s) {
  if (saved) return forward(w, B, x, ld, params, saved, ld, out, ld, s);
  if (B > t->cap) return hipErrorInvalidValue;
  for (int64_t c0 = 0; c0 < B; c0 += t->ld) {
    const int64_t bc = B - c0 < t->ld ? B - c0 : t->ld;
    hipError_t e = forward(w, bc, x + c0, ld, params, t->z, t->ld, out + c0, ld, s);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

// Backward over B samples, chunk by chunk (one chunk when the scratch holds
// the whole batch): the chunk's pre-activations are copied from `saved`
// ([H][ld]) or, without it, recomputed from x; the weight and bias gradients
// of later chunks are added in chunk order.  The schedule and the arithmetic
// per chunk are the same whether the pre-activations were saved or
// recomputed, so both give the same gradient bit for bit.
hipError_t train_mlp_backward(const int *w, int64_t B, int64_t ld, const float *x,
                              const float *params, const float *saved, const float *grad_out,
                              float *grad_params, float *grad_x, TrainScratch *t, hipStream_t s) {
  if (B > t->cap) return hipErrorInvalidValue;
  const int64_t H = (int64_t)w[1] + w[2] + w[3];
  int k = 0;
  for (int64_t c0 = 0; c0 < B; c0 += t->ld, ++k) {
    const int64_t bc = B - c0 < t->ld ? B - c0 : t->ld;
    const float *z = t->z;
    hipError_t e = hipSuccess;
    if (saved && c0 == 0 && bc == B && ld == t->ld) {
      z = saved;                 // (already in the scratch's layout)
    } else if (saved) {
      // the fused GELU' epilogue reads z with the scratch leading dimension
      e = hipMemcpy2DAsync(t->z, t->ld * sizeof(float), saved + c0, ld * sizeof(float),
                           bc * sizeof(float), H, hipMemcpyDeviceToDevice, s);
    } else {
      e = forward(w, bc, x + c0, ld, params, t->z, t->ld, t->out, t->ld, s);
    }
    if (e != hipSuccess) return e;
    e = backward(w, bc, x + c0, ld, params, z, t->ld, grad_out + c0, ld, grad_params,
                 grad_x ? grad_x + c0 : nullptr, ld, t, s, k > 0);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

// One training step: chunk by chunk, features -> forward -> loss gradient ->
// backward, the gradient of later chunks added in chunk order; then the loss
// (the chunk sums in order) and Adam.  With the whole batch in one chunk
// this is the plain step; with smaller chunks only one chunk's activations
// exist at a time (nothing has to be recomputed: a sample's loss gradient
// does not depend on the other samples).
hipError_t train_step(const int *w, int64_t B, int64_t ld, const double *T, const double *P,
                      const double *Y, const float *target, float *params, float *grads,
                      float *adam_m, float *adam_v, int64_t step, float lr, bool recompute,
                      float *loss, const float *fc, const double *dc, TrainScratch *t,
                      hipStream_t s) {
  (void)recompute;
  if (B > t->cap) return hipErrorInvalidValue;
  const int S = w[4];
  const int64_t cc = t->ld;
  const double denom = (double)B * S;
  hipError_t e = hipSuccess;
  int k = 0;
  for (int64_t c0 = 0; c0 < B; c0 += cc, ++k) {
    const int64_t bc = B - c0 < cc ? B - c0 : cc;
    hipLaunchKernelGGL(features_kernel, dim3(blocks_for(bc)), dim3(256), 0, s, T + c0, P + c0,
                       Y + c0, ld, bc, S, fc, dc, t->x, cc);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    e = forward(w, bc, t->x, cc, params, t->z, cc, t->out, cc, s);
    if (e != hipSuccess) return e;
    // dL/do into dz[1] (the backward ping-pong starts writing dz[0])
    int nb = (int)blocks_for((int64_t)S * bc);
    if (nb > 1024) nb = 1024;
    hipLaunchKernelGGL(mse_kernel, dim3(nb), dim3(256), 0, s, (const float *)t->out, cc,
                       target + c0, ld, S, bc, denom, t->dz[1], t->lpart);
    hipLaunchKernelGGL(loss_chunk_kernel, dim3(1), dim3(64), 0, s, (const float *)t->lpart, nb,
                       t->closs + k);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    // mse_kernel wrote dO with the output's leading dimension (cc)
    e = backward(w, bc, t->x, cc, params, t->z, cc, t->dz[1], cc, grads, nullptr, 0, t, s, k > 0);
    if (e != hipSuccess) return e;
  }
  hipLaunchKernelGGL(loss_final_kernel, dim3(1), dim3(64), 0, s, (const double *)t->closs, k, denom,
                     loss);
  const int64_t np = (int64_t)param_off(w, 4);
  const double c1 = 1.0 / (1.0 - pow(0.9, (double)step));
  const double c2 = 1.0 / (1.0 - pow(0.999, (double)step));
  hipLaunchKernelGGL(adam_kernel, dim3(blocks_for(np)), dim3(256), 0, s, params, (const float *)grads,
                     adam_m, adam_v, np, lr, (float)c1, (float)c2);
  return hipGetLastError();
}

}  // namespace chemdnn
