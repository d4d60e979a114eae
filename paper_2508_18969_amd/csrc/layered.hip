// Layer-by-layer path of the chemistry update for networks whose weights do
// not fit the on-chip design of the fused kernel - e.g. the ODENet of the
// paper's runs, 20-2048-4096-2048-1024-512-17 (Sec. 4, network sizes table;
// 38.9 MFLOP and 19.4M parameters per cell): its 38.9 MB of BF16 weights
// exceed the 4 MB L2 of an XCD, so every 64-cell tile of the fused kernel
// would stream them from the Infinity Cache.  Here each layer is one large
// matrix product over a chunk of cells, with 256 x 256 output tiles whose
// operands are staged in LDS, so every weight byte fetched serves 256 cells.
//
//   prep_kernel    steps 1-2 (power transform, Z-score) -> layer-1 B fragments
//   layer_kernel   one layer, Zt = W At (+ b, GELU for hidden layers); the
//                  output goes straight into the next layer's B fragments
//   post_kernel    steps 4-7 per cell (one thread per cell, FP64 update)
//
// The property networks of the supercritical flame (PRNet, Sec. 2 and the
// network sizes of Sec. 4: 3-1024-512-256-1 and 3-2048-1024-512-4) run on the
// same layer kernel between their own input and output maps
// (prop_prep_kernel: Z-score of the input fields; prop_post_kernel: the
// output affine map in FP64).
//
// Activations live in HBM between layers as "B fragments": for k-step q and
// cell-block cb (16 cells) a 1 KiB block of 64 lanes x 16 bytes, lane
// (cell cl, group g) holding input features frag_feature(KS, q, g, j); blocks
// are ordered [q][cb], so the 16 cell-blocks of a tile are 16 consecutive
// KiB.  Weights use the fused kernel's packed layout ([row-block][k-step]).
#include "common.h"
#include "internal.h"

namespace chemdnn {

namespace {

constexpr int FB = 64 * 16;        // bytes of one fragment (64 lanes x 16 bytes)
constexpr int STAGES = 4;          // LDS k-step buffers in flight

// Waits until at most N vector-memory operations of this wave are in flight.
// Direct-to-LDS copies are not tracked by the compiler's own wait insertion;
// the memory clobber keeps LDS reads from moving above the wait.
template <int N>
__device__ __forceinline__ void wait_vmem() {
  static_assert(N >= 0 && N < 64, "vmcnt range");
  asm volatile("s_waitcnt vmcnt(%0)" ::"n"(N) : "memory");
}
// Waits until at most PER * min(k, MAXK) vector-memory operations are in
// flight (k >= 0 at run time; PER, MAXK compile-time).
template <int PER, int MAXK>
__device__ __forceinline__ void wait_vmem_upto(int k) {
  if constexpr (MAXK <= 0) {
    wait_vmem<0>();
  } else {
    if (k >= MAXK) wait_vmem<PER * MAXK>();
    else wait_vmem_upto<PER, MAXK - 1>(k);
  }
}
__device__ __forceinline__ void lds_barrier_all() {
  asm volatile("s_waitcnt lgkmcnt(0)\n\ts_barrier" ::: "memory");
}

// One wave copies the 1 KiB fragment at src (global) to dst (LDS), lane l's
// 16 bytes to dst + 16 l, without passing through registers.
__device__ __forceinline__ void dma_frag(const uint8_t *src, uint8_t *dst, int lane) {
  __builtin_amdgcn_global_load_lds(
      (const __attribute__((address_space(1))) void *)(src + (uint32_t)(lane * 16)),
      (__attribute__((address_space(3))) void *)dst, 16, 0, 0);
}

}  // namespace

// ------------------------------------------------------------------ layer
// Workgroup tile: TRB = WRB*WR row-blocks x TCB = WCB*WC cell-blocks; eight
// waves in a WR x WC grid, each computing WRB x WCB 16x16 output blocks.  Per
// k-step the tile's TRB weight fragments and TCB activation fragments are
// copied to an LDS stage (every wave copies every eighth fragment); each wave
// then reads its WRB + WCB fragments from LDS into registers one k-step ahead,
// so that the reads of k-step q + 1 overlap the products of k-step q.  Four
// stages: the copies of k-step q + 3 are issued once every wave has read the
// fragments of k-step q (and so is done with the stage of q - 1).
// DBG (hidden layers): the accumulators are also written to a.dbg_acc.
template <class Op, int WRB, int WR, int WCB, int WC, bool ACT, bool DBG = false>
__global__ __launch_bounds__(WR * WC * 64, 1) void layer_kernel(LayerArgs a) {
  constexpr int NW = WR * WC;                         // waves
  static_assert(Op::FRAG == 16, "16-byte fragments");
  using frag_t = typename Op::frag_t;
  constexpr int TRB = WRB * WR, TCB = WCB * WC, NF = TRB + TCB;
  constexpr int PERW = NF % NW == 0 ? NF / NW : -1;  // copies per wave per k-step, if even
  extern __shared__ __align__(16) uint8_t smem[];
  const int lane = threadIdx.x & 63, g = lane >> 4, cl = lane & 15;
  const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int wr = w % WR, wc = w / WR;
  const int nrt = a.R / TRB;
  const int rt = blockIdx.x % nrt, ct = blockIdx.x / nrt;
  const int rb0 = rt * TRB, cb0 = ct * TCB;
  const uint8_t *const Wt = a.W + (size_t)rb0 * a.NQ * FB;
  const uint8_t *const Xt = a.X + (size_t)cb0 * FB;

  // this wave's copies: fragments f = w + NW k of the NF of a k-step
  auto issue = [&](int q, int s) {
    uint8_t *dst = smem + s * NF * FB;
    if constexpr (TRB % NW == 0 && TCB % NW == 0) {
#pragma unroll
      for (int k = 0; k < NF / NW; ++k) {
        const int f = w + NW * k;
        const uint8_t *src = k < TRB / NW ? Wt + ((size_t)f * a.NQ + q) * FB
                                          : Xt + ((size_t)q * a.NCB + (f - TRB)) * FB;
        dma_frag(src, dst + f * FB, lane);
      }
    } else {
      for (int f = w; f < NF; f += NW) {
        const uint8_t *src = f < TRB ? Wt + ((size_t)f * a.NQ + q) * FB
                                     : Xt + ((size_t)q * a.NCB + (f - TRB)) * FB;
        dma_frag(src, dst + f * FB, lane);
      }
    }
  };
  auto read = [&](int q, frag_t (&af)[WRB], frag_t (&bf)[WCB]) {
    const uint8_t *st = smem + (q % STAGES) * NF * FB + lane * 16;
#pragma unroll
    for (int i = 0; i < WRB; ++i) af[i] = *(const frag_t *)(st + (wr * WRB + i) * FB);
#pragma unroll
    for (int j = 0; j < WCB; ++j) bf[j] = *(const frag_t *)(st + (TRB + wc * WCB + j) * FB);
  };

  // accumulators start at the bias (rows 16 rb + 4 g + r)
  f4 acc[WRB][WCB];
#pragma unroll
  for (int i = 0; i < WRB; ++i) {
    const f4 b = *(const f4 *)(a.bias + 16 * (rb0 + wr * WRB + i) + 4 * g);
#pragma unroll
    for (int j = 0; j < WCB; ++j) acc[i][j] = b;
  }

  // k-steps 0 .. STAGES - 2 in flight; k-step 0 in registers (the copies of
  // the later ones may stay in flight)
  for (int q = 0; q < STAGES - 1 && q < a.NQ; ++q) issue(q, q);
  if constexpr (PERW > 0) {
    const int issued = a.NQ < STAGES - 1 ? a.NQ : STAGES - 1;
    wait_vmem_upto<PERW, STAGES - 2>(issued - 1);
  } else {
    wait_vmem<0>();
  }
  lds_barrier_all();
  frag_t af[2][WRB], bf[2][WCB];
  read(0, af[0], bf[0]);
  for (int q = 0; q < a.NQ; q += 2) {
    // two k-steps per trip, so the register buffers need no dynamic index
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const int qq = q + h;
      if (qq < a.NQ) {
        if (qq + 1 < a.NQ) {
          // k-step qq + 1: this wave's copies (those of qq + 2 .. qq +
          // STAGES - 2 may be in flight), then every wave's; every wave has
          // read k-step qq, so the stage of qq - 1 is free for k-step
          // qq + STAGES - 1
          if constexpr (PERW > 0) {
            const int last = qq + STAGES - 2 < a.NQ - 1 ? qq + STAGES - 2 : a.NQ - 1;
            wait_vmem_upto<PERW, STAGES - 3>(last - (qq + 1));
          } else {
            wait_vmem<0>();
          }
          lds_barrier_all();
          if (qq + STAGES - 1 < a.NQ) issue(qq + STAGES - 1, (qq + STAGES - 1) % STAGES);
          read(qq + 1, af[h ^ 1], bf[h ^ 1]);
        }
#pragma unroll
        for (int i = 0; i < WRB; ++i)
#pragma unroll
          for (int j = 0; j < WCB; ++j) acc[i][j] = Op::mma(af[h][i], bf[h][j], acc[i][j]);
      }
    }
  }

  if constexpr (DBG) {
#pragma unroll
    for (int i = 0; i < WRB; ++i)
#pragma unroll
      for (int j = 0; j < WCB; ++j)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int row = 16 * (rb0 + wr * WRB + i) + 4 * g + r;
          const int cell = 16 * (cb0 + wc * WCB + j) + cl;
          if (row < a.dbg_rows && cell < a.dbg_n) a.dbg_acc[(size_t)row * a.dbg_n + cell] = acc[i][j][r];
        }
  }
  if constexpr (ACT) {
    // GELU, then the next layer's B fragments: output row 16 rb + 4 g + r is
    // input feature of k-step rb / RPQ, slot 4 (rb % RPQ) + r
    constexpr int RPQ = Op::KS / 16;
    static_assert(WRB % RPQ == 0, "row-blocks of a k-step in one wave");
#pragma unroll
    for (int i = 0; i < WRB; i += RPQ) {
      const int rb = rb0 + wr * WRB + i;
#pragma unroll
      for (int j = 0; j < WCB; ++j) {
        const int cb = cb0 + wc * WCB + j;
        __attribute__((aligned(16))) uint8_t buf[16];
#pragma unroll
        for (int k = 0; k < RPQ; ++k) {
          f4 y;
#pragma unroll
          for (int r = 0; r < 4; ++r) y[r] = gelu(acc[i + k][j][r]);
          Op::store4(buf + 4 * k * Op::EB, y);
        }
        *(i4 *)(a.Y + ((size_t)(rb / RPQ) * a.NCB + cb) * FB + lane * 16) = *(const i4 *)buf;
      }
    }
  } else {
    // output layer: FP32 [row][cell]
#pragma unroll
    for (int i = 0; i < WRB; ++i)
#pragma unroll
      for (int j = 0; j < WCB; ++j)
#pragma unroll
        for (int r = 0; r < 4; ++r)
          a.O[(size_t)(16 * (rb0 + wr * WRB + i) + 4 * g + r) * a.ldo + 16 * (cb0 + wc * WCB + j) + cl] =
              acc[i][j][r];
  }
}

// ------------------------------------------------------------------ prep
// Writes the 32 features z of cell c of the chunk into the layer-1 B
// fragments X ([32 / KS][NCB] fragments).
template <class Op>
__device__ __forceinline__ void store_layer1(const float (&z)[32], uint8_t *X, int NCB, int c) {
  const int cb = c >> 4, cl = c & 15;
  constexpr int NE = 16 / Op::EB;                          // slots per lane
#pragma unroll
  for (int q = 0; q < 32 / Op::KS; ++q)
#pragma unroll
    for (int g = 0; g < 4; ++g) {
      __attribute__((aligned(16))) uint8_t buf[16];
#pragma unroll
      for (int j0 = 0; j0 < NE; j0 += 4) {
        f4 y;
#pragma unroll
        for (int r = 0; r < 4; ++r) y[r] = z[frag_feature(Op::KS, q, g, j0 + r)];
        Op::store4(buf + j0 * Op::EB, y);
      }
      *(i4 *)(X + ((size_t)q * NCB + cb) * FB + (g * 16 + cl) * 16) = *(const i4 *)buf;
    }
}

// Thread per cell c of the chunk (cells past the chunk give zero features):
// z_f of steps 1-2 for f < 32, written into the layer-1 B fragments.
template <class Op>
__global__ __launch_bounds__(256) void prep_kernel(PrepArgs a) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= 16 * a.NCB) return;
  const int64_t i = a.n0 + c;
  const bool valid = c < a.nc;
  const int64_t ii = valid ? i : 0;
  const float lam = a.fc[FConst::LAM];
  float z[32];
#pragma unroll
  for (int f = 0; f < 32; ++f) {
    float v = 0.0f;
    if (valid) {
      if (f == 0) {
        v = (float)((a.T[ii] - a.dc[DConst::T_MU]) * a.dc[DConst::T_IS]);
      } else if (f == 1) {
        v = (float)((a.P[ii] - a.dc[DConst::P_MU]) * a.dc[DConst::P_IS]);
      } else if (f - 2 < a.S) {
        v = __builtin_fmaf(ypow(a.Y[(int64_t)(f - 2) * a.ld + ii], lam), a.fc[FConst::ZA + f],
                           a.fc[FConst::ZC + f]);
      }
    }
    z[f] = v;
  }
  store_layer1<Op>(z, a.X, a.NCB, c);
}

// Property network input: thread per cell c of the chunk, z_f = (x_f - mu_f) /
// sigma_f in FP64 for the n_in input fields (zero for f >= n_in and for cells
// past the chunk), rounded to FP32 and written into the layer-1 B fragments.
template <class Op>
__global__ __launch_bounds__(256) void prop_prep_kernel(PropPrepArgs a) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= 16 * a.NCB) return;
  const bool valid = c < a.nc;
  const int64_t i = valid ? a.n0 + c : 0;
  float z[32];
#pragma unroll
  for (int f = 0; f < 32; ++f)
    z[f] = (valid && f < a.D)
               ? (float)((a.x[(int64_t)f * a.ld + i] - a.pc[PConst::IN_MU + f]) * a.pc[PConst::IN_IS + f])
               : 0.0f;
  store_layer1<Op>(z, a.X, a.NCB, c);
}

// ------------------------------------------------------------------ post
// Thread per cell: steps 4-7 from the FP32 network output O[s][cell].  The
// species loops are unrolled to the 30-species maximum (guarded by S), so
// the updated fractions stay in registers between the passes.
__global__ __launch_bounds__(256) void post_kernel(PostArgs a) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= a.nc) return;
  const int64_t i = a.n0 + c;
  const float lam = a.fc[FConst::LAM], inv_lam = a.fc[FConst::INV_LAM];
  const double T = a.T[i], P = a.P[i], t_ref = a.dc[DConst::T_REF];
  bool bad = !__builtin_isfinite(T) || !__builtin_isfinite(P);
  constexpr int SMAX = 30;
  double y[SMAX], yh[SMAX];
  double ssum = 0.0, h0 = 0.0, ry = 0.0;
#pragma unroll
  for (int s = 0; s < SMAX; ++s) {
    y[s] = 0.0;
    yh[s] = 0.0;
    if (s >= a.S) continue;
    const int rho = s + 2;
    y[s] = a.Y[(int64_t)s * a.ld + i];
    bad |= !__builtin_isfinite(y[s]);
    const float o = a.O[(size_t)s * a.ldo + c];
    const float wv = __builtin_fmaf(o, a.fc[FConst::PA + rho], a.fc[FConst::PB + rho]);
    const double v = y[s] + inv_change(y[s], wv, lam, inv_lam);
    // a NaN network output or a non-finite result flags the cell (the inverse
    // transform takes a NaN base like a negative one; the clamp turns NaN into 0)
    bad |= __builtin_isnan(wv) || !__builtin_isfinite(v);
    yh[s] = v > 0.0 ? v : 0.0;
    ssum += yh[s];
    h0 += y[s] * (a.dc[DConst::HF + rho] + a.dc[DConst::CP + rho] * (T - t_ref));
    ry += y[s] * a.dc[DConst::WINV + rho];
  }
  const double rsum = 1.0 / ssum;
  double hn = 0.0, cn = 0.0;
  bool nonfin = false;
#pragma unroll
  for (int s = 0; s < SMAX; ++s) {
    if (s >= a.S) continue;
    const double yn = yh[s] * rsum;
    nonfin |= !__builtin_isfinite(yn);
    hn += yn * a.dc[DConst::HF + s + 2];
    cn += yn * a.dc[DConst::CP + s + 2];
  }
  const double Tn = a.thermo ? t_ref + (h0 - hn) / cn : T;
  const bool okc = !bad && !nonfin && ssum > 0.0 && __builtin_isfinite(ssum) && __builtin_isfinite(Tn);
  const double rho_dt = a.omega && okc ? P / (kRGas * T * ry) * a.inv_dt : 0.0;
#pragma unroll
  for (int s = 0; s < SMAX; ++s) {
    if (s >= a.S) continue;
    const double yn = okc ? yh[s] * rsum : y[s];
    a.Y_out[(int64_t)s * a.ld + i] = yn;
    if (a.omega) a.omega[(int64_t)s * a.ld + i] = okc ? rho_dt * (yn - y[s]) : 0.0;
  }
  if (a.T_out) a.T_out[i] = okc ? Tn : T;
  if (!okc && a.n_bad) atomicAdd(a.n_bad, 1u);
}

// Property network output: y_k = o_k sigma_k + mu_k in FP64, thread per
// (output k, cell c); FP32 network output O[k][ldo] of the chunk.
__global__ __launch_bounds__(256) void prop_post_kernel(PropPostArgs a) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x, k = blockIdx.y;
  if (c >= a.nc) return;
  const double o = a.O[(size_t)k * a.ldo + c];
  a.y[(int64_t)k * a.ld + a.n0 + c] = __builtin_fma(o, a.pc[PConst::OUT_SD + k], a.pc[PConst::OUT_MU + k]);
}

// ------------------------------------------------------------------ debug
// Operand value of feature f < K of cell c < n in the B fragments X
// ([NQ][NCB] fragments of 64 lanes x 16 bytes), decoded to FP32: the
// inverse of frag_feature within a k-step, f = KS q + 16 (j / 4) + 4 g + j % 4.
template <class Op>
__global__ __launch_bounds__(256) void frag_decode_kernel(const uint8_t *X, int NCB, int K, int n,
                                                          float *out) {
  const int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (t >= (int64_t)K * n) return;
  const int f = (int)(t / n), c = (int)(t % n);
  const int q = f / Op::KS, rr = f % Op::KS;
  const int j = 4 * (rr / 16) + rr % 4, g = (rr % 16) / 4;
  const uint8_t *p = X + ((size_t)(q * NCB + c / 16) * 64 + g * 16 + c % 16) * 16 + j * Op::EB;
  float v;
  if constexpr (__is_same(Op, OpF32)) v = *(const float *)p;
  else if constexpr (__is_same(Op, OpBF16)) v = (float)*(const __bf16 *)p;
  else v = (float)*(const _Float16 *)p;
  out[t] = v;
}

__global__ __launch_bounds__(256) void copy_rows_kernel(const float *src, int ld_src, int rows, int n,
                                                        float *dst) {
  const int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (t >= (int64_t)rows * n) return;
  dst[t] = src[(t / n) * (int64_t)ld_src + t % n];
}

// ------------------------------------------------------------------ launchers
namespace {

template <class K>
hipError_t set_lds(K kern, int bytes) {
  return hipFuncSetAttribute((const void *)kern, hipFuncAttributeMaxDynamicSharedMemorySize, bytes);
}

// hidden layers: 256 x 256 tiles (16 row-blocks x 16 cell-blocks) over
// HWR x HWC waves of HWRB x HWCB blocks each
constexpr int HWRB = 4, HWR = 4, HWCB = 8, HWC = 2;
static_assert(HWRB * HWR == 16 && HWCB * HWC == 16, "256 x 256 tiles");
constexpr int LDS_HIDDEN = STAGES * (16 + 16) * FB;
constexpr int LDS_OUT = STAGES * (2 + 16) * FB;
static_assert(LDS_HIDDEN <= 160 * 1024, "LDS budget");

template <class Op>
hipError_t launch_layer_op(const LayerArgs &a, bool hidden, hipStream_t s) {
  if (hidden) {
    auto k = layer_kernel<Op, HWRB, HWR, HWCB, HWC, true>;
    const int grid = (a.R / 16) * (a.NCB / 16);
    constexpr int LDS = LDS_HIDDEN, NT = 64 * HWR * HWC;
    hipLaunchKernelGGL(k, dim3(grid), dim3(NT), LDS, s, a);
  } else {
    // output layer, 32 rows: 2 row-blocks x 16 cell-blocks (2 per wave)
    constexpr int LDS = LDS_OUT;
    auto k = layer_kernel<Op, 2, 1, 2, 8, false>;
    const int grid = (a.R / 2) * (a.NCB / 16);
    hipLaunchKernelGGL(k, dim3(grid), dim3(512), LDS, s, a);
  }
  return hipGetLastError();
}

template <class Op>
hipError_t launch_layer_dbg_op(const LayerArgs &a, hipStream_t s) {
  auto k = layer_kernel<Op, HWRB, HWR, HWCB, HWC, true, true>;
  const int grid = (a.R / 16) * (a.NCB / 16);
  hipLaunchKernelGGL(k, dim3(grid), dim3(64 * HWR * HWC), LDS_HIDDEN, s, a);
  return hipGetLastError();
}

}  // namespace

hipError_t launch_layer_dbg(int fmt, const LayerArgs &a, hipStream_t s) {
  switch (fmt) {
    case 0: return launch_layer_dbg_op<OpF32>(a, s);
    case 1: return launch_layer_dbg_op<OpBF16>(a, s);
    case 2: return launch_layer_dbg_op<OpF16>(a, s);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_frag_decode(int fmt, const uint8_t *X, int NCB, int K, int n, float *out,
                              hipStream_t s) {
  const int64_t total = (int64_t)K * n;
  if (total <= 0) return hipSuccess;
  const dim3 grid((unsigned)((total + 255) / 256));
  switch (fmt) {
    case 0: hipLaunchKernelGGL(frag_decode_kernel<OpF32>, grid, dim3(256), 0, s, X, NCB, K, n, out); break;
    case 1: hipLaunchKernelGGL(frag_decode_kernel<OpBF16>, grid, dim3(256), 0, s, X, NCB, K, n, out); break;
    case 2: hipLaunchKernelGGL(frag_decode_kernel<OpF16>, grid, dim3(256), 0, s, X, NCB, K, n, out); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_copy_rows(const float *src, int ld_src, int rows, int n, float *dst, hipStream_t s) {
  const int64_t total = (int64_t)rows * n;
  if (total <= 0) return hipSuccess;
  hipLaunchKernelGGL(copy_rows_kernel, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, s, src,
                     ld_src, rows, n, dst);
  return hipGetLastError();
}

// The layer kernels use more than the default 64 KiB of LDS.
hipError_t layered_prepare() {
  hipError_t e = set_lds(layer_kernel<OpF32, HWRB, HWR, HWCB, HWC, true>, LDS_HIDDEN);
  if (e == hipSuccess) e = set_lds(layer_kernel<OpF32, HWRB, HWR, HWCB, HWC, true, true>, LDS_HIDDEN);
  if (e == hipSuccess) e = set_lds(layer_kernel<OpBF16, HWRB, HWR, HWCB, HWC, true, true>, LDS_HIDDEN);
  if (e == hipSuccess) e = set_lds(layer_kernel<OpF16, HWRB, HWR, HWCB, HWC, true, true>, LDS_HIDDEN);
  if (e == hipSuccess) e = set_lds(layer_kernel<OpBF16, HWRB, HWR, HWCB, HWC, true>, LDS_HIDDEN);
  if (e == hipSuccess) e = set_lds(layer_kernel<OpF16, HWRB, HWR, HWCB, HWC, true>, LDS_HIDDEN);
  if (e == hipSuccess) e = set_lds(layer_kernel<OpF32, 2, 1, 2, 8, false>, LDS_OUT);
  if (e == hipSuccess) e = set_lds(layer_kernel<OpBF16, 2, 1, 2, 8, false>, LDS_OUT);
  if (e == hipSuccess) e = set_lds(layer_kernel<OpF16, 2, 1, 2, 8, false>, LDS_OUT);
  return e;
}

hipError_t launch_layer(int fmt, const LayerArgs &a, bool hidden, hipStream_t s) {
  switch (fmt) {
    case 0: return launch_layer_op<OpF32>(a, hidden, s);
    case 1: return launch_layer_op<OpBF16>(a, hidden, s);
    case 2: return launch_layer_op<OpF16>(a, hidden, s);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_prep(int fmt, const PrepArgs &a, hipStream_t s) {
  const int blocks = (16 * a.NCB + 255) / 256;
  switch (fmt) {
    case 0: hipLaunchKernelGGL(prep_kernel<OpF32>, dim3(blocks), dim3(256), 0, s, a); break;
    case 1: hipLaunchKernelGGL(prep_kernel<OpBF16>, dim3(blocks), dim3(256), 0, s, a); break;
    case 2: hipLaunchKernelGGL(prep_kernel<OpF16>, dim3(blocks), dim3(256), 0, s, a); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_prop_prep(int fmt, const PropPrepArgs &a, hipStream_t s) {
  const int blocks = (16 * a.NCB + 255) / 256;
  switch (fmt) {
    case 0: hipLaunchKernelGGL(prop_prep_kernel<OpF32>, dim3(blocks), dim3(256), 0, s, a); break;
    case 1: hipLaunchKernelGGL(prop_prep_kernel<OpBF16>, dim3(blocks), dim3(256), 0, s, a); break;
    case 2: hipLaunchKernelGGL(prop_prep_kernel<OpF16>, dim3(blocks), dim3(256), 0, s, a); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_prop_post(const PropPostArgs &a, hipStream_t s) {
  if (a.nc <= 0 || a.K <= 0) return hipSuccess;
  hipLaunchKernelGGL(prop_post_kernel, dim3((a.nc + 255) / 256, a.K), dim3(256), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_post(const PostArgs &a, hipStream_t s) {
  if (a.nc <= 0) return hipSuccess;
  hipLaunchKernelGGL(post_kernel, dim3((a.nc + 255) / 256), dim3(256), 0, s, a);
  return hipGetLastError();
}

}  // namespace chemdnn
