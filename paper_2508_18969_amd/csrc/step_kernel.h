// Fused, persistent chemistry-update kernel (gfx950): the kernel template,
// its configurations and launchers.  Instantiated per operand format in
// step_fp32.hip, step_bf16.hip, step_fp16.hip and step_fp8.hip.
//
// One workgroup of NW waves (four: one per SIMD; eight: two per SIMD) owns a
// tile of MC cells at a time and loops over tiles with a grid stride (grid =
// number of CUs).  Per tile:
//   pre     FP64 state -> Box-Cox + Z-score (FP32) -> layer-1 B fragments (LDS);
//           the state itself stays in LDS for the post-processing
//   L1+L2   layer 1 is produced in super-chunks of its output rows; each chunk
//           (bias + GELU + quantise) goes to a ring of LDS slots and is
//           consumed as a K-slice of layer 2, whose accumulators stay in
//           registers: the wide layer-1 activation never exists whole
//   L3      layer-2 GELU output sits in LDS; layer 3 streams it
//   L4      layer-3 output reuses that LDS region; linear output layer
//   post    inverse transform in FP32, update, renormalisation and optional
//           temperature in FP64, written by the lane that holds the values
// Waves split every layer's output rows, so each wave reads weight rows no
// other wave reads: weights stream from L2 straight into registers, fetched
// one or more k-steps ahead of their use, and cross the L2->CU path once per
// tile.  LDS holds activations, the tile's state, biases and constants.
#pragma once
#include "common.h"
#include "internal.h"

namespace chemdnn {

// Split of R output row-blocks x CB cell-blocks over NW waves: each wave
// owns F whole row-blocks (all cell-blocks) plus NREM leftover tiles.
template <int R, int CB, int NW> struct Split {
  static constexpr int F = R / NW;
  static constexpr int RR = R % NW;
  static constexpr int NREM = RR * CB / NW;
  static constexpr int T = F * CB + NREM;
  static_assert((RR * CB) % NW == 0, "row-blocks must split evenly over the waves");
  // (I unsigned: the wave index is often an opaque copy, whose sign the
  // compiler can not see; signed division adds a sign fix-up)
  template <class I> static __device__ __forceinline__ int rem_rb(I w, int k) { return NW * F + (w * NREM + (I)k) / CB; }
  template <class I> static __device__ __forceinline__ int rem_cb(I w, int k) { return (w * NREM + (I)k) % CB; }
};

// Output rows a layer computes: h rounded up to row-blocks of 16 such that
// the row-blocks split evenly over the nw waves (see Split); with `whole`,
// to a multiple of nw row-blocks, so that no wave has leftover tiles.
constexpr int padN(int h, int cb, bool whole, int nw) {
  int p = roundup(h, whole ? 16 * nw : 16);
  while ((((p / 16) % nw) * cb) % nw) p += 16;
  return p;
}

template <class Op_, int CB_, int NW_, int H1_, int H2_, int H3_> struct Cfg {
  using Op = Op_;
  static constexpr int H1 = H1_, H2 = H2_, H3 = H3_;
  // NW waves per workgroup (4: one per SIMD; 8: two per SIMD, which hides
  // one wave's memory waits behind the other's work, at half the registers)
  static constexpr int NW = NW_;
  using frag_t = typename Op::frag_t;
  static constexpr int KS = Op::KS, FRAG = Op::FRAG, EB = Op::EB, CB = CB_, MC = 16 * CB_;
  static constexpr int NQ1 = (32 + KS - 1) / KS;    // layer-1 k-steps (inputs <= 32)
  static constexpr int SC = KS > 64 ? KS : 64;      // layer-1 rows per super-chunk
  static constexpr int H1P = roundup(H1_, SC);
  // layers 2 and 3 compute H2N / H3N rows; as the next layer's input they
  // are zero-padded to whole k-steps (H2P / H3P)
  // FP8 fragments take twice the registers: no leftover tiles there
  static constexpr int H2N = padN(H2_, CB_, FRAG == 32 && NW_ <= 4, NW_), H3N = padN(H3_, CB_, FRAG == 32 && NW_ <= 4, NW_);
  static constexpr int H2P = roundup(H2N, KS), H3P = roundup(H3N, KS);
  static constexpr int R1 = H1P / 16, R2 = H2N / 16, R3 = H3N / 16, R4 = 2;
  static constexpr int NQ2 = H1P / KS, NQ3 = H2P / KS, NQ4 = H3P / KS;
  static constexpr int NSC = H1P / SC, RB1W = SC / 64, QSC = SC / KS, RPQ = KS / 16;
  using S2 = Split<R2, CB_, NW_>;
  using S3 = Split<R3, CB_, NW_>;
  static constexpr int QBYTES = CB * 64 * FRAG;     // one k-step of a tile's activations
  static constexpr int NW1 = RB1W * NQ1;             // layer-1 fragments per wave per chunk
  // A chunk's layer-1 tiles: SC / 16 / RB1W row groups x CB cell-blocks.  With
  // more waves than row groups, the waves of a row group split its
  // cell-blocks (CBW each).
  static constexpr int L1G = SC / 16 / RB1W;
  static constexpr int CBW = NW_ > L1G ? CB_ * L1G / NW_ : CB_;
  static constexpr int NBIAS = H1P + H2N + H3N + 32; // biases of all layers, FP32
  static constexpr int LDS_BIAS = 0;
  static constexpr int LDS_DC = roundup(NBIAS * 4, 16);          // DConst or PConst block (FP64)
  static constexpr int LDS_FC = LDS_DC + Max<DConst::N, PConst::N>::v * 8;   // FConst block (FP32)
  // The FP64 state of the tile (8 values per lane of the CB preprocess
  // waves), kept from the preprocess for the post-processing.
  static constexpr int ST_BYTES = CB * 64 * 8 * 8;
  static constexpr int LDS_ST = roundup(LDS_FC + FConst::N * 4, 256);
  static constexpr int LDS_A0 = roundup(LDS_ST + ST_BYTES, 256);
  static constexpr int LDS_A1 = LDS_A0 + NQ1 * QBYTES;
  // A2 (layers 3 and 4 inputs) shares the space of A0 and A1 (layers 1 and 2
  // inputs): they are never in use at the same time
  static constexpr int LDS_A2 = LDS_A0;
  // Layer 1 runs LA chunks ahead of layer 2, into a ring of 2 LA chunk
  // buffers; with LA = 2 the loop needs a barrier after every second chunk
  // only (BF16/FP16 on eight waves)
  static constexpr int LA = NW_ > 4 && KS == 32 ? 2 : 1;
  static constexpr int A01_BYTES = NQ1 * QBYTES + 2 * LA * QSC * QBYTES;
  static constexpr int NW2 = S2::F + S2::NREM;               // layer-2 fragments per wave per k-step
  static constexpr int NB2 = NW_ > 4 ? 1 : QSC % 2 == 0 ? 2 : 1;   // layer-2 register buffers
  static constexpr int A2_BYTES = Max<NQ3, NQ4>::v * QBYTES;
  // The LDS tail holds the GELU table (tabulated form only), then the
  // output-layer weights, copied once per workgroup when they fit.
  static constexpr int W4_BYTES = R4 * NQ4 * 64 * FRAG;
  // bytes of packed layer l (row-blocks x k-steps x 64 lane fragments)
  static constexpr int wbytes(int l) {
    return (l == 0 ? R1 * NQ1 : l == 1 ? R2 * NQ2 : l == 2 ? R3 * NQ3 : R4 * NQ4) * 64 * FRAG;
  }
  // gt: 0 tanh form, 1 FP32 table (16 bytes per interval), 2 FP16 table (8)
  static constexpr int tab_bytes(int gt) { return gt == 1 ? GTAB_N * 16 : gt == 2 ? GTAB_N * 8 : 0; }
  static constexpr int LDS_TAIL = LDS_A2 + (A2_BYTES > A01_BYTES ? A2_BYTES : A01_BYTES);
  static constexpr int lds_w4(int gt) { return LDS_TAIL + tab_bytes(gt); }
  static constexpr bool w4_lds(int gt) { return lds_w4(gt) + W4_BYTES <= 160 * 1024; }
  static constexpr int lds_bytes(int gt) { return lds_w4(gt) + (w4_lds(gt) ? W4_BYTES : 0); }
  static constexpr int LDS_BYTES = lds_bytes(0);
  static_assert(lds_bytes(1) <= 160 * 1024 && lds_bytes(2) <= 160 * 1024, "LDS budget");
};

// Weight fragments are read through buffer resources: the address of a load
// is the resource base, one per-lane byte offset (a single VGPR for the whole
// kernel) and a wave-uniform byte offset in an SGPR, so a load costs no
// vector address arithmetic and keeps no 64-bit addresses live.  Loads past
// num_records return zero instead of touching memory.
typedef __amdgpu_buffer_rsrc_t rsrc_t;
// word 3 of a raw (stride 0) gfx9 buffer resource: 32-bit data format
constexpr int kBufWord3 = 0x00020000;
__device__ __forceinline__ rsrc_t weight_rsrc(const void *p, int bytes) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void *>(p), (short)0, bytes, kBufWord3);
}

// Workgroup barrier for LDS traffic only: unlike __syncthreads it does not
// wait for outstanding global loads, so weight loads stay in flight.  Every
// barrier of the tile loop is of this kind: the waves of a workgroup share
// only LDS (each wave's global loads are waited for where it uses them), and
// a full barrier would stall on the state loads of the post-processing and of
// the next tile, which are issued early to hide their HBM latency.
__device__ __forceinline__ void lds_barrier() {
  asm volatile("s_waitcnt lgkmcnt(0)\n\ts_barrier" ::: "memory");
}

// Fragment idx of a packed weight matrix (blocks of 64 lane fragments);
// voff = lane * sizeof(frag_t).
template <class frag_t>
__device__ __forceinline__ frag_t ldb_frag(rsrc_t r, int idx, int voff) {
  const int soff = idx * (64 * (int)sizeof(frag_t));
  if constexpr (sizeof(frag_t) == 16) {
    return __builtin_bit_cast(frag_t, __builtin_amdgcn_raw_buffer_load_b128(r, voff, soff, 0));
  } else {
    static_assert(sizeof(frag_t) == 32, "fragment size");
    typedef uint32_t u4 __attribute__((ext_vector_type(4)));
    typedef uint32_t u8v __attribute__((ext_vector_type(8)));
    const u4 lo = __builtin_amdgcn_raw_buffer_load_b128(r, voff, soff, 0);
    const u4 hi = __builtin_amdgcn_raw_buffer_load_b128(r, voff + 16, soff, 0);
    return __builtin_bit_cast(frag_t, u8v{lo[0], lo[1], lo[2], lo[3], hi[0], hi[1], hi[2], hi[3]});
  }
}
template <class frag_t>
__device__ __forceinline__ frag_t lds_frag(const uint8_t *base, int idx, int lane) {
  return *(const frag_t *)(base + (idx * 64 + lane) * (int)sizeof(frag_t));
}

__device__ __forceinline__ float umaxf(float a, float b) { return a > b ? a : b; }

// A copy of a uniform value that the optimisers can not see through: offsets
// derived from it are recomputed where they are used (one scalar add each)
// instead of being precomputed for every load of a loop and spilled.
__device__ __forceinline__ int opaque(int v) {
  asm volatile("" : "+s"(v));
  return v;
}
// An opaque copy of an index known to be non-negative (a wave index): its
// divisions and remainders by powers of two are plain shifts and masks.
__device__ __forceinline__ unsigned opaque_u(unsigned v) {
  asm volatile("" : "+s"(v));
  return v;
}
// The same for a per-lane value: LDS addresses built on it keep their
// constant parts in the instruction's offset field.
__device__ __forceinline__ int opaque_v(int v) {
  asm volatile("" : "+v"(v));
  return v;
}

// PROP: property mode - the input features are the Z-scored fields x[f]
// (f < D) and the output rows 2 .. K+1 are scaled to y[k] = o sigma_k + mu_k;
// dc is then a PConst block.
// DBG: layer dump - every layer's input operand values (decoded to FP32) and
// FP32 accumulators go to a.dbg_in / a.dbg_acc (rows of real features and
// cells only); the post-processing is skipped.  The products, activations
// and their schedules are those of the plain kernel.
// GT: the hidden activation - 0 the tanh form, 1 the FP32 table, 2 the FP16 table.
template <class C, bool CALIB, int GT, bool PROP = false, bool DBG = false>
__global__ __launch_bounds__(C::NW * 64, 1) void chem_step_kernel(StepArgs a) {
  using Op = typename C::Op;
  using frag_t = typename C::frag_t;
  using S2 = typename C::S2;
  using S3 = typename C::S3;
  constexpr int CB = C::CB, KS = C::KS, FRAG = C::FRAG, EB = C::EB, RPQ = C::RPQ;
  extern __shared__ __align__(16) uint8_t smem[];
  uint8_t *const A0 = smem + C::LDS_A0;
  uint8_t *const A1 = smem + C::LDS_A1;
  uint8_t *const A2 = smem + C::LDS_A2;
  // the wave index is uniform: keeping it scalar lets every weight address be a
  // scalar base plus one per-lane offset
  const int lane = threadIdx.x & 63, g = lane >> 4, cl = lane & 15;
  const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const float *fc = a.fc;
  const double *dc = a.dc;
  const uint8_t *const W1g = (const uint8_t *)a.w[0], *const W2g = (const uint8_t *)a.w[1];
  const uint8_t *const W3g = (const uint8_t *)a.w[2], *const W4g = (const uint8_t *)a.w[3];
  const float lam = fc[FConst::LAM], inv_lam = fc[FConst::INV_LAM];
  float inv_sa[4], sout[4], sa[4];
#pragma unroll
  for (int l = 0; l < 4; ++l) {
    inv_sa[l] = Op::SCALED ? fc[FConst::INV_SA + l] : 1.0f;
    sa[l] = Op::SCALED ? fc[FConst::ASCALE + l] : 1.0f;
    sout[l] = Op::SCALED ? fc[FConst::SOUT + l] : 1.0f;
  }
  float amx[4] = {0.f, 0.f, 0.f, 0.f};

  // all biases live in LDS for the whole kernel: no global loads in the
  // weight-streaming loops besides the direct-to-LDS copies
  float *const Bl = (float *)(smem + C::LDS_BIAS);
  for (int i = threadIdx.x; i < C::NBIAS; i += blockDim.x) {
    const int l = i < C::H1P ? 0 : i < C::H1P + C::H2N ? 1 : i < C::H1P + C::H2N + C::H3N ? 2 : 3;
    const int o = l == 0 ? 0 : l == 1 ? C::H1P : l == 2 ? C::H1P + C::H2N : C::H1P + C::H2N + C::H3N;
    Bl[i] = a.b[l][i - o];
  }
  const float *const B1 = Bl, *const B2 = Bl + C::H1P, *const B3 = Bl + C::H1P + C::H2N;
  const float *const B4 = Bl + C::H1P + C::H2N + C::H3N;
  // transform and thermodynamic constants too
  double *const dcl = (double *)(smem + C::LDS_DC);
  float *const fcl = (float *)(smem + C::LDS_FC);
  for (int i = threadIdx.x; i < (PROP ? PConst::N : DConst::N); i += blockDim.x) dcl[i] = a.dc[i];
  for (int i = threadIdx.x; i < FConst::N; i += blockDim.x) fcl[i] = a.fc[i];
  constexpr bool W4L = C::w4_lds(GT);
  constexpr int LW4 = C::lds_w4(GT);
  if constexpr (W4L)
    for (int i = threadIdx.x; i < C::W4_BYTES / 16; i += blockDim.x)
      ((i4 *)(smem + LW4))[i] = ((const i4 *)W4g)[i];
  const f4 *const tabl = (const f4 *)(smem + C::LDS_TAIL);
  const h4v *const tabl16 = (const h4v *)(smem + C::LDS_TAIL);
  if constexpr (GT != 0)   // (the table as bytes: 16 or 8 per interval)
    for (int i = threadIdx.x; i < C::tab_bytes(GT) / 16; i += blockDim.x)
      ((i4 *)(smem + C::LDS_TAIL))[i] = ((const i4 *)a.gtab)[i];
  // hidden-layer activation: the tanh form, or a table
  auto act = [&](float x) {
    if constexpr (GT == 1) return gelu_tab(x, tabl);
    else if constexpr (GT == 2) return gelu_tab16(x, tabl16);
    else return gelu(x);
  };
  // debug mode: value v of output row `row` (< rows) of a cell into
  // buf[(row0 + row) * n + cell]
  auto dbg_put = [&](float *buf, int row0, int row, int rows, int64_t cell, float v) {
    if (row < rows && cell < a.n) buf[(int64_t)(row0 + row) * a.n + cell] = v;
  };
  __syncthreads();

  // The preprocess state is loaded one tile ahead: lane (cell 16w + cl,
  // group g) holds input features f = 16h + 4g + r (T, P, Y_(f-2)), as
  // xin[4h + r], from clamped (always valid) addresses.
  double xin[8];
  // The field offsets of these loads are recomputed where they are issued,
  // from an opaque copy of the lane group: hoisted out of the tile loop they
  // would be spilled, and the reload of each - counted with the loads in issue
  // order - would make every load wait for the HBM load before it.
  auto load_xin = [&](int64_t t) {
    const int64_t i = t * C::MC + 16 * w + cl;
    const int64_t ii = (t < a.ntiles && i < a.n) ? i : 0;
    const int go = opaque_v(g);
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      const int f = 16 * (j >> 2) + 4 * go + (j & 3);
      if constexpr (PROP) {
        // fields past the inputs read the last one (zeroed below)
        xin[j] = __builtin_nontemporal_load(&a.x[(int64_t)(f < a.D ? f : a.D - 1) * a.ld + ii]);
      } else {
        const int s = f - 2 < a.S ? f - 2 : a.S - 1;
        xin[j] = __builtin_nontemporal_load(f == 0 ? &a.T[ii] : f == 1 ? &a.P[ii] : &a.Y[(int64_t)(s > 0 ? s : 0) * a.ld + ii]);
      }
    }
  };
  if (C::NW == CB || w < CB) load_xin(blockIdx.x);

  for (int64_t tile = blockIdx.x; tile < a.ntiles; tile += gridDim.x) {
    const int64_t cell0 = tile * C::MC;
    // Opaque copies of the weight bases: the resources are rebuilt per tile
    // instead of being hoisted out of the tile loop and kept live (spilled).
    const uint8_t *W1o = W1g, *W2o = W2g, *W3o = W3g, *W4o = W4g;
    asm volatile("" : "+s"(W1o), "+s"(W2o), "+s"(W3o), "+s"(W4o));
    const rsrc_t W1 = weight_rsrc(W1o, C::wbytes(0)), W2 = weight_rsrc(W2o, C::wbytes(1));
    const rsrc_t W3 = weight_rsrc(W3o, C::wbytes(2)), W4 = weight_rsrc(W4o, C::wbytes(3));
    const int voff = lane * (int)sizeof(frag_t);

    // ------------------------------------------------------------ preprocess
    // Lane (cell 16w + cl, group g) computes input features f = 16h + 4g + r.
    // (Every wave has finished the previous tile's layer 4, which reads A2,
    // and post-processing, which reads the staged state, before the
    // preprocess overwrites both.)
    lds_barrier();
    if (C::NW == CB || w < CB) {
      const int64_t i = cell0 + 16 * w + cl;
      // the state stays in LDS for the post-processing (the same lane then
      // holds the same fields), instead of a second read from HBM
      if constexpr (!CALIB && !PROP) {
        double *st = (double *)(smem + C::LDS_ST) + (w * 64 + lane) * 8;
#pragma unroll
        for (int j = 0; j < 8; j += 2) *(double2v *)(st + j) = double2v{xin[j], xin[j + 1]};
      }
      const bool valid = i < a.n;
      f4 v[2];
#pragma unroll
      for (int h = 0; h < 2; ++h)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          // selects instead of branches: feature f is T or P only in the
          // first two slots of the lanes with g == 0
          const int f = 16 * h + 4 * g + r;
          const double x = xin[4 * h + r];
          float z;
          if constexpr (PROP) {
            z = (float)((x - dcl[PConst::IN_MU + f]) * dcl[PConst::IN_IS + f]);
            z = f < a.D ? z : 0.0f;
          } else {
            z = __builtin_fmaf(ypow(x, lam), fcl[FConst::ZA + f], fcl[FConst::ZC + f]);
            z = f - 2 < a.S ? z : 0.0f;
            if (h == 0 && r < 2) {
              const float ztp = r == 0 ? (float)((x - dcl[DConst::T_MU]) * dcl[DConst::T_IS])
                                       : (float)((x - dcl[DConst::P_MU]) * dcl[DConst::P_IS]);
              z = g == 0 ? ztp : z;
            }
          }
          z = valid ? z : 0.0f;
          if (CALIB) amx[0] = umaxf(amx[0], __builtin_fabsf(z));
          v[h][r] = z * inv_sa[0];
          if constexpr (DBG)
            if (valid && f < a.S + 2) a.dbg_in[(int64_t)(a.dbg_in_row[0] + f) * a.n + i] = Op::q(v[h][r]);
        }
      if constexpr (KS == 16) {
        // two k-steps of 16: feature 16h + 4g + r sits in k-step h, slot r
        Op::store4(A0 + ((0 * CB + w) * 64 + lane) * FRAG, v[0]);
        Op::store4(A0 + ((1 * CB + w) * 64 + lane) * FRAG, v[1]);
      } else {
        uint8_t *p = A0 + (w * 64 + lane) * FRAG;
        Op::store4(p, v[0]);
        Op::store4(p + 4 * EB, v[1]);
        // slots 8.. (features >= 32) are zero padding
#pragma unroll
        for (int o = 8 * EB; o < FRAG; o += 4) *(uint32_t *)(p + o) = 0u;
      }
    }
    lds_barrier();


    // Layer 1, super-chunk sc, in two steps: the products (into acc1) and the
    // activation of values [v0, v1) (bias + GELU + quantise into A1 buffer
    // `buf`).  Value v of the chunk is output value v % 4 of tile v / 4:
    // row-block v / (4 CB) of this wave, cell-block (v / 4) % CB.
    // Wave w computes row group w / NCG of the chunk, cell-blocks
    // CBW (w % NCG) .. + CBW - 1.
    constexpr int CBW = C::CBW, NCG = CB / CBW;
    constexpr int NV1 = C::RB1W * CBW * 4;             // activation values per lane per chunk
    // layer 1 is computed by the first L1W waves
    constexpr int L1W = C::L1G * NCG;
    const bool l1wave = C::NW == L1W || w < L1W;
    f4 acc1[C::RB1W][CBW];
    f4 y1[C::RB1W][CBW];
    // opaque copy of the wave index, renewed per k-step (unsigned: shifts
    // and masks for its divisions; FP8 keeps the signed form, with which its
    // registers spill less)
    using widx_t = std::conditional_t<FRAG == 32, int, unsigned>;
    widx_t wo = w;
    // the layer-1 input fragments, re-read per chunk (cheaper than keeping
    // them live through the layer-2 loop)
    auto layer1_in = [&](frag_t (&a0)[C::NQ1][CBW]) {
      if (!l1wave) return;
#pragma unroll
      for (int q = 0; q < C::NQ1; ++q)
#pragma unroll
        for (int c = 0; c < CBW; ++c) a0[q][c] = lds_frag<frag_t>(A0, q * CB + (wo % NCG) * CBW + c, lane);
    };
    auto layer1_mma = [&](int sc, const frag_t (&w1f)[C::NW1], const frag_t (&a0)[C::NQ1][CBW]) {
      if (!l1wave) return;
#pragma unroll
      for (int ii = 0; ii < C::RB1W; ++ii) {
        const f4 bias = *(const f4 *)(B1 + 16 * (sc * (C::SC / 16) + (wo / NCG) * C::RB1W + ii) + 4 * g);
#pragma unroll
        for (int c = 0; c < CBW; ++c) {
          acc1[ii][c] = Op::SCALED ? f4{0.f, 0.f, 0.f, 0.f} : bias;
#pragma unroll
          for (int q = 0; q < C::NQ1; ++q) acc1[ii][c] = Op::mma(w1f[ii * C::NQ1 + q], a0[q][c], acc1[ii][c]);
        }
      }
    };
    // activation values [v0, v1) of chunk sc; a tile is stored with its last value
    auto layer1_act = [&](int sc, int buf, int v0, int v1) {
      if (!l1wave) return;
      const int dv = opaque_v(buf * C::QSC * C::QBYTES + lane * FRAG);
#pragma unroll
      for (int v = 0; v < NV1; ++v) {
        if (v < v0 || v >= v1) continue;
        const int ii = v / (4 * CBW), c = (v / 4) % CBW, r = v % 4;
        const int cb = (wo % NCG) * CBW + c;
        const int rbl = (wo / NCG) * C::RB1W + ii;     // row-block within the chunk
        const int rb = sc * (C::SC / 16) + rbl;
        const float bias = B1[16 * rb + 4 * g + r];
        const float zz = Op::SCALED ? __builtin_fmaf(acc1[ii][c][r], sout[0], bias) : acc1[ii][c][r];
        if constexpr (DBG) dbg_put(a.dbg_acc, a.dbg_acc_row[0], 16 * rb + 4 * g + r, C::H1, cell0 + 16 * cb + cl, acc1[ii][c][r]);
        y1[ii][c][r] = act(zz);
        if (r == 3) {
          f4 y = y1[ii][c];
          if (CALIB && cell0 + 16 * cb + cl < a.n)
#pragma unroll
            for (int k = 0; k < 4; ++k) amx[1] = umaxf(amx[1], __builtin_fabsf(y[k]));
          // (scaled formats: y / a_1 is quantised by the store)
          if constexpr (DBG)
#pragma unroll
            for (int k = 0; k < 4; ++k) dbg_put(a.dbg_in, a.dbg_in_row[1], 16 * rb + 4 * g + k, C::H1, cell0 + 16 * cb + cl, Op::q(y[k] * inv_sa[1]));
          const int q2l = rbl / RPQ, j0 = 4 * (rbl % RPQ);
          Op::store4s((A1 + cb * 64 * FRAG) + (dv + (q2l * CB * 64 * FRAG + j0 * EB)), y, sa[1]);
        }
      }
    };

    // The same activation (tanh form) in stages, spread over the layer-2
    // fragment groups of the loop.  The operations form a stage-major list:
    // operation k is stage k / NV1 of value k % NV1, so that two dependent
    // operations are a whole stage apart (their latency is covered), and each
    // group takes a few of them, placed between its matrix products, whose
    // execution they overlap.
    // (BF16 / FP16 operands; the FP32 and FP8 loops keep one activation block,
    // measured faster there)
    constexpr bool STAGED = GT == 0 && KS == 32;
    constexpr int NOPS1 = 8 * NV1;
    float xs[NV1], ts[NV1];
    auto layer1_ops = [&](int sc, int buf, int k0, int k1) {
      if (!l1wave) return;
#pragma unroll
      for (int k = 0; k < NOPS1; ++k) {
        if (k < k0 || k >= k1) continue;
        const int st = k / NV1, v = k % NV1;
        const int ii = v / (4 * CBW), c = (v / 4) % CBW, r = v % 4;
        const int cb = (wo % NCG) * CBW + c;
        const int rbl = (wo / NCG) * C::RB1W + ii;     // row-block within the chunk
        if (st == 0) {
          if constexpr (Op::SCALED) {
            const float bias = B1[16 * (sc * (C::SC / 16) + rbl) + 4 * g + r];
            xs[v] = __builtin_fmaf(acc1[ii][c][r], sout[0], bias);
          } else {
            xs[v] = acc1[ii][c][r];
          }
          if constexpr (DBG)
            dbg_put(a.dbg_acc, a.dbg_acc_row[0], 16 * (sc * (C::SC / 16) + rbl) + 4 * g + r,
                    C::H1, cell0 + 16 * cb + cl, acc1[ii][c][r]);
          ts[v] = xs[v] * xs[v];
        } else if (st == 1) {
          ts[v] = __builtin_fmaf(ts[v], kG3, kG1);
        } else if (st == 2) {
          ts[v] = xs[v] * ts[v];
        } else if (st == 3) {
          ts[v] = __builtin_amdgcn_exp2f(ts[v]);
        } else if (st == 4) {
          ts[v] = 1.0f + ts[v];
        } else if (st == 5) {
          ts[v] = __builtin_amdgcn_rcpf(ts[v]);
        } else if (st == 6) {
          ts[v] = xs[v] * ts[v];
        } else if (r == 3) {
          f4 y = {ts[v - 3], ts[v - 2], ts[v - 1], ts[v]};
          if (CALIB && cell0 + 16 * cb + cl < a.n)
#pragma unroll
            for (int j = 0; j < 4; ++j) amx[1] = umaxf(amx[1], __builtin_fabsf(y[j]));
          if constexpr (DBG)
#pragma unroll
            for (int k = 0; k < 4; ++k)
              dbg_put(a.dbg_in, a.dbg_in_row[1], 16 * (sc * (C::SC / 16) + rbl) + 4 * g + k, C::H1, cell0 + 16 * cb + cl, Op::q(y[k] * inv_sa[1]));
          const int q2l = rbl / RPQ, j0 = 4 * (rbl % RPQ);
          // (the store's lane offset is taken here, where it is used: an
          // opaque copy per call of this function costs a move per group;
          // scaled formats: y / a_1 is quantised by the store)
          const int dv = opaque_v(buf * C::QSC * C::QBYTES + lane * FRAG);
          Op::store4s((A1 + cb * 64 * FRAG) + (dv + (q2l * CB * 64 * FRAG + j0 * EB)), y, sa[1]);
        }
        // keeps the operation in its group
        asm volatile("" : "+v"(ts[v]));
      }
    };

    // ------------------------------------------------------------ layers 1+2
    f4 acc2[S2::T];
#pragma unroll
    for (int i = 0; i < S2::F; ++i) {
      const f4 bias = Op::SCALED ? f4{0.f, 0.f, 0.f, 0.f} : *(const f4 *)(B2 + 16 * (w * S2::F + i) + 4 * g);
#pragma unroll
      for (int cb = 0; cb < CB; ++cb) acc2[i * CB + cb] = bias;
    }
#pragma unroll
    for (int k = 0; k < S2::NREM; ++k)
      acc2[S2::F * CB + k] = Op::SCALED ? f4{0.f, 0.f, 0.f, 0.f} : *(const f4 *)(B2 + 16 * S2::rem_rb(w, k) + 4 * g);

    // Weight streaming.  Every wave reads only its own weight rows, so the
    // fragments go from L2 straight into registers.  Layer 2 keeps NB2
    // register buffers (one on eight waves, whose registers are halved):
    // fragment i of k-step q + NB2 is loaded as soon as the products of
    // k-step q have read fragment i, which gives each load about NB2 k-steps
    // of matrix work to land.  Layer-1 fragments of chunk c + 1 + LA are
    // loaded once chunk c + LA has used them.  Past the end the indices are
    // clamped, so the loop body is uniform.
    constexpr int NW2 = C::NW2;
    constexpr int NB2 = C::NB2;
    constexpr int NA2 = CB + (S2::NREM > 0 ? S2::NREM : 1);
    frag_t wb[NB2][NW2];
    auto w2_load = [&](frag_t &dst, int i, int q) {
      const int rb = i < S2::F ? wo * S2::F + i : S2::rem_rb(wo, i - S2::F);
      dst = ldb_frag<frag_t>(W2, rb * C::NQ2 + (q < C::NQ2 ? q : C::NQ2 - 1), voff);
    };
    frag_t w1r[C::NW1];
    auto w1_load = [&](int c) {
      if (!l1wave) return;
      const int cs = c < C::NSC ? c : c - C::NSC;
#pragma unroll
      for (int ii = 0; ii < C::RB1W; ++ii)
#pragma unroll
        for (int q = 0; q < C::NQ1; ++q) {
          const int rb = cs * (C::SC / 16) + (wo / NCG) * C::RB1W + ii;
          w1r[ii * C::NQ1 + q] = ldb_frag<frag_t>(W1, rb * C::NQ1 + q, voff);
        }
    };
    frag_t a0[C::NQ1][CBW];
    constexpr int LA = C::LA;
    static_assert(C::NSC >= LA, "layer-1 lead");
#pragma unroll
    for (int c = 0; c < LA; ++c) {
      w1_load(c);
      layer1_in(a0);
      layer1_mma(c, w1r, a0);
      layer1_act(c, c, 0, NV1);
    }
    w1_load(LA);
#pragma unroll
    for (int b = 0; b < NB2; ++b)
#pragma unroll
      for (int i = 0; i < NW2; ++i) w2_load(wb[b][i], i, b);
    lds_barrier();

#pragma nounroll
    for (int sc = 0; sc < C::NSC; ++sc) {
      // Layer 1 of chunk sc + LA: its products follow the first fragment
      // group's, its activation is spread over the later groups (staged form)
      // or follows as one block (the last LA iterations recompute the first
      // chunks into idle buffers, which keeps the loop body uniform).
      const int nsc = sc + LA < C::NSC ? sc + LA : sc + LA - C::NSC;
      const int nbuf = (sc + LA) & (2 * LA - 1);
      const int sv = opaque_v((sc & (2 * LA - 1)) * C::QSC * C::QBYTES + lane * FRAG);
      const widx_t wa = FRAG == 32 ? (widx_t)opaque(w) : (widx_t)opaque_u(w);
      // The chunk's activation fragments, read once (constant offsets first,
      // so that they land in the instructions' offset fields).  Only the
      // first k-step's fragments and the layer-1 inputs are read before the
      // first products: every wave reads the same fragments at the same time
      // here, and the later k-steps' reads go out behind the first products
      // instead of delaying them.
      frag_t act[C::QSC][NA2];
      auto act_load = [&](int ql) {
#pragma unroll
        for (int cb = 0; cb < CB; ++cb) act[ql][cb] = *(const frag_t *)((A1 + (ql * CB + cb) * 64 * FRAG) + sv);
#pragma unroll
        for (int k = 0; k < S2::NREM; ++k)
          act[ql][CB + k] = *(const frag_t *)((A1 + ql * CB * 64 * FRAG) + (sv + S2::rem_cb(wa, k) * 64 * FRAG));
      };
      act_load(0);
      layer1_in(a0);
#pragma unroll
      for (int ql = 0; ql < C::QSC; ++ql) {
        const int q = sc * C::QSC + ql;
        wo = FRAG == 32 ? (widx_t)opaque(w) : (widx_t)opaque_u(w);
        frag_t(&wc)[NW2] = wb[ql % NB2];
        // the scheduling barriers keep each refill right behind the products
        // that read the fragment (the scheduler would otherwise sink the
        // loads towards their next use and shorten their lead)
#pragma unroll
        for (int i = 0; i < NW2; ++i) {
          if (i < S2::F) {
#pragma unroll
            for (int cb = 0; cb < CB; ++cb) acc2[i * CB + cb] = Op::mma(wc[i], act[ql][cb], acc2[i * CB + cb]);
          } else {
            const int k = i - S2::F;
            acc2[S2::F * CB + k] = Op::mma(wc[i], act[ql][CB + k], acc2[S2::F * CB + k]);
          }
          w2_load(wc[i], i, q + NB2);
          const int gi = ql * NW2 + i;                 // fragment group of the chunk
          if (gi == 0) {
            layer1_mma(nsc, w1r, a0);
#pragma unroll
            for (int ql = 1; ql < C::QSC; ++ql) act_load(ql);
            w1_load(sc + 1 + LA);
            if constexpr (!STAGED) layer1_act(nsc, nbuf, 0, NV1);
          }
          if constexpr (STAGED) {
            // the activation's operations from the third group on (the
            // layer-1 products have finished by then)
            // operations in proportion to the group's products
            constexpr int G0 = 2, MK = S2::F * CB + S2::NREM;     // products per k-step
            auto mcum = [](int gq) {                   // products before group gq
              const int qq = gq / NW2, ig = gq % NW2;
              return qq * MK + (ig < S2::F ? ig * CB : S2::F * CB + (ig - S2::F));
            };
            constexpr int MT = C::QSC * MK - (G0 / NW2) * MK - (G0 % NW2 < S2::F ? (G0 % NW2) * CB : S2::F * CB + (G0 % NW2 - S2::F));
            static_assert(C::QSC * NW2 > G0 && MT > 0, "fragment groups for the layer-1 activation");
            if (gi >= G0) {
              const int m0 = mcum(gi) - mcum(G0), m1 = m0 + (i < S2::F ? CB : 1);
              const int k0 = m0 * NOPS1 / MT, k1 = m1 * NOPS1 / MT;
              layer1_ops(nsc, nbuf, k0, k1);
              // products and activation operations alternate
              constexpr int PER = (NOPS1 + MT - 1) / MT + 1;
#pragma unroll
              for (int m = 0; m < (i < S2::F ? CB : 1); ++m) {
                __builtin_amdgcn_sched_group_barrier(0x008, 1, 0);
                __builtin_amdgcn_sched_group_barrier(0x002, PER, 0);
              }
            }
          }
          __builtin_amdgcn_sched_barrier(0);
        }
      }
      // (LA = 2: chunks sc + 1 and sc + 2, written during sc - 1 and sc, are
      // complete at the barrier after every odd chunk, and the buffers they
      // overwrite were last read before the barrier before that)
      if (LA == 1 || (sc & 1)) lds_barrier();
    }
    lds_barrier();

    // The next tile's state is fetched at the end of the layer-3 products
    // (BF16/FP16) or after them (FP32), so its latency overlaps the rest of
    // the tile - or, with FP8 operands, whose registers are scarcer, after
    // the layer-4 products (it is then held through the post-processing only;
    // calibration ends the tile here).
    constexpr bool LATE_XIN = FRAG == 32 && !CALIB;

    // The first k-step of layer-3 weights is requested now, so its latency
    // overlaps the layer-2 activation phase; the next ones follow it.
    constexpr int NW3 = S3::F + S3::NREM;              // fragments per wave per k-step
    constexpr int NB3 = FRAG == 32 ? 1 : 3;            // k-steps in flight (FP8 k-steps are 4x longer)
    // BF16/FP16: the next tile's state loads go out in the layer-3 loop, at
    // k-step XQ (FP32's registers are too few for them there)
    constexpr bool XIN_L3 = !LATE_XIN && NB3 > 1 && KS == 32;
    constexpr int XQ = C::NQ3 > NB3 ? C::NQ3 - NB3 : 0;
    constexpr int NA3 = CB + (S3::NREM > 0 ? S3::NREM : 1);
    frag_t w3b[NB3][NW3];
    auto w3_load = [&](frag_t &dst, int i, int q) {
      const int rb = i < S3::F ? w * S3::F + i : S3::rem_rb(w, i - S3::F);
      dst = ldb_frag<frag_t>(W3, rb * C::NQ3 + q, voff);
    };
#pragma unroll
    for (int i = 0; i < NW3; ++i) w3_load(w3b[0][i], i, 0);

    // layer-2 activation -> LDS (layer-3 B fragments)
    // FP8: the per-lane LDS addresses of the layer-2/3/4 activations are
    // recomputed at each use from an opaque copy of the lane index (past the
    // 16-bit offset field the compiler keeps one base register per address,
    // which it spills with 32-byte fragments)
    auto lane_a = [&]() { return FRAG == 32 ? opaque_v(lane) : lane; };
    // (scaled formats: y / as is quantised by the store)
    auto put = [&](uint8_t *base, int rb, int cb, f4 y, float as) {
      Op::store4s(base + (((rb / RPQ) * CB + cb) * 64 + lane_a()) * FRAG + 4 * (rb % RPQ) * EB, y, as);
    };
    // rows past the computed ones, up to the next k-step boundary, are zero
    auto zero_pad = [&](int r0, int r1) {
#pragma unroll
      for (int t = w; t < (r1 - r0) * CB; t += C::NW) put(A2, r0 + t / CB, t % CB, f4{0.f, 0.f, 0.f, 0.f}, 1.0f);
    };
    // The activation phases take ATG tiles at a time; with the tanh form
    // their GELUs are evaluated stage by stage across the group
    // (gelu_stages), which interleaves their dependent operations.
    constexpr int ATG = GT == 0 ? 2 : 1;
    auto act_group = [&](f4 (&z)[ATG], int n) {
      if constexpr (ATG > 1) {
        gelu_stages(z, n);
      } else {
#pragma unroll
        for (int r = 0; r < 4; ++r) z[0][r] = act(z[0][r]);
      }
    };
    {
#pragma unroll
      for (int t0 = 0; t0 < S2::T; t0 += ATG) {
        const int n = S2::T - t0 < ATG ? S2::T - t0 : ATG;
        f4 z[ATG];
#pragma unroll
        for (int u = 0; u < ATG; ++u) {
          if (u >= n) continue;
          const int t = t0 + u;
          const int rb = t < S2::F * CB ? w * S2::F + t / CB : S2::rem_rb(w, t - S2::F * CB);
          f4 bias = Op::SCALED ? *(const f4 *)(B2 + 16 * rb + 4 * g) : f4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
          for (int r = 0; r < 4; ++r) z[u][r] = Op::SCALED ? __builtin_fmaf(acc2[t][r], sout[1], bias[r]) : acc2[t][r];
        }
        act_group(z, n);
#pragma unroll
        for (int u = 0; u < ATG; ++u) {
          if (u >= n) continue;
          const int t = t0 + u;
          const int rb = t < S2::F * CB ? w * S2::F + t / CB : S2::rem_rb(w, t - S2::F * CB);
          const int cb = t < S2::F * CB ? t % CB : S2::rem_cb(w, t - S2::F * CB);
          const f4 y = z[u];
          if (CALIB && cell0 + 16 * cb + cl < a.n)
#pragma unroll
            for (int r = 0; r < 4; ++r) amx[2] = umaxf(amx[2], __builtin_fabsf(y[r]));
          if constexpr (DBG)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
              dbg_put(a.dbg_acc, a.dbg_acc_row[1], 16 * rb + 4 * g + r, C::H2, cell0 + 16 * cb + cl, acc2[t][r]);
              dbg_put(a.dbg_in, a.dbg_in_row[2], 16 * rb + 4 * g + r, C::H2, cell0 + 16 * cb + cl, Op::q(y[r] * inv_sa[2]));
            }
          put(A2, rb, cb, y, sa[2]);
        }
        // FP8: two tiles at a time, which keeps the accumulators where they
        // are instead of letting the scheduler copy them all out of the
        // accumulation registers up front (the register file is full there)
        if (FRAG == 32 && (t0 & 1)) __builtin_amdgcn_sched_barrier(0);
      }
      zero_pad(C::R2, C::H2P / 16);
    }
    lds_barrier();

    // ------------------------------------------------------------ layer 3
    f4 acc3[S3::T];
#pragma unroll
    for (int i = 0; i < S3::F; ++i) {
      const f4 bias = Op::SCALED ? f4{0.f, 0.f, 0.f, 0.f}
                                 : *(const f4 *)(B3 + 16 * (w * S3::F + i) + 4 * g);
#pragma unroll
      for (int cb = 0; cb < CB; ++cb) acc3[i * CB + cb] = bias;
    }
#pragma unroll
    for (int k = 0; k < S3::NREM; ++k)
      acc3[S3::F * CB + k] = Op::SCALED ? f4{0.f, 0.f, 0.f, 0.f}
                                        : *(const f4 *)(B3 + 16 * S3::rem_rb(w, k) + 4 * g);
    {
      // Fully unrolled: every load index is a constant, so the compiler's
      // wait counts are exact.  Fragment i of k-step q + NB3 is loaded as
      // soon as the products of k-step q have read fragment i; activations
      // are read one k-step ahead.
      frag_t a3r[2][NA3];
      auto load_a3 = [&](frag_t (&dst)[NA3], int q) {
#pragma unroll
        for (int cb = 0; cb < CB; ++cb) dst[cb] = lds_frag<frag_t>(A2, q * CB + cb, lane_a());
#pragma unroll
        for (int k = 0; k < S3::NREM; ++k) dst[CB + k] = lds_frag<frag_t>(A2, q * CB + S3::rem_cb(w, k), lane_a());
      };
      if constexpr (NB3 == 1) {
        // one buffer: a rolled loop, one k-step per iteration (a basic block
        // each, which keeps every refill behind the products of its k-step)
#pragma nounroll
        for (int q = 0; q < C::NQ3; ++q) {
          frag_t ac[NA3];
          load_a3(ac, q);
          const int qn = q + 1 < C::NQ3 ? q + 1 : q;
#pragma unroll
          for (int i = 0; i < S3::F; ++i) {
#pragma unroll
            for (int cb = 0; cb < CB; ++cb) acc3[i * CB + cb] = Op::mma(w3b[0][i], ac[cb], acc3[i * CB + cb]);
            w3_load(w3b[0][i], i, qn);
            __builtin_amdgcn_sched_barrier(0);
          }
#pragma unroll
          for (int k = 0; k < S3::NREM; ++k) {
            acc3[S3::F * CB + k] = Op::mma(w3b[0][S3::F + k], ac[CB + k], acc3[S3::F * CB + k]);
            w3_load(w3b[0][S3::F + k], S3::F + k, qn);
            __builtin_amdgcn_sched_barrier(0);
          }
        }
      } else {
#pragma unroll
        for (int b = 1; b < NB3; ++b)
#pragma unroll
          for (int i = 0; i < NW3; ++i)
            if (b < C::NQ3) w3_load(w3b[b][i], i, b);
        load_a3(a3r[0], 0);
#pragma unroll
        for (int q = 0; q < C::NQ3; ++q) {
          if (q + 1 < C::NQ3) load_a3(a3r[(q + 1) & 1], q + 1);
          frag_t(&wc)[NW3] = w3b[q % NB3];
          const auto &ac = a3r[q & 1];
#pragma unroll
          for (int i = 0; i < S3::F; ++i) {
#pragma unroll
            for (int cb = 0; cb < CB; ++cb) acc3[i * CB + cb] = Op::mma(wc[i], ac[cb], acc3[i * CB + cb]);
            if (q + NB3 < C::NQ3) w3_load(wc[i], i, q + NB3);
            // the next tile's state, requested once the last weight loads
            // have gone out (loads complete in order: a weight load behind
            // it would wait for HBM), its address arithmetic beside the
            // remaining products
            if (XIN_L3 && q == XQ && i == 0 && (C::NW == CB || w < CB)) load_xin(tile + gridDim.x);
            __builtin_amdgcn_sched_barrier(0);
          }
#pragma unroll
          for (int k = 0; k < S3::NREM; ++k) {
            acc3[S3::F * CB + k] = Op::mma(wc[S3::F + k], ac[CB + k], acc3[S3::F * CB + k]);
            if (q + NB3 < C::NQ3) w3_load(wc[S3::F + k], S3::F + k, q + NB3);
            __builtin_amdgcn_sched_barrier(0);
          }
        }
      }
    }
    const int64_t ipost = cell0 + 16 * w + cl;
    const bool vpost = ipost < a.n;
    // (single-buffered layer-3 loop, or fewer than two k-steps: the next
    // tile's state is fetched here, unless it comes after layer 4)
    if (!LATE_XIN && !XIN_L3 && (C::NW == CB || w < CB)) load_xin(tile + gridDim.x);
    lds_barrier();  // every wave is done reading the layer-2 activation
    {
#pragma unroll
      for (int t0 = 0; t0 < S3::T; t0 += ATG) {
        const int n = S3::T - t0 < ATG ? S3::T - t0 : ATG;
        f4 z[ATG];
#pragma unroll
        for (int u = 0; u < ATG; ++u) {
          if (u >= n) continue;
          const int t = t0 + u;
          const int rb = t < S3::F * CB ? w * S3::F + t / CB : S3::rem_rb(w, t - S3::F * CB);
          f4 bias = Op::SCALED ? *(const f4 *)(B3 + 16 * rb + 4 * g) : f4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
          for (int r = 0; r < 4; ++r) z[u][r] = Op::SCALED ? __builtin_fmaf(acc3[t][r], sout[2], bias[r]) : acc3[t][r];
        }
        act_group(z, n);
#pragma unroll
        for (int u = 0; u < ATG; ++u) {
          if (u >= n) continue;
          const int t = t0 + u;
          const int rb = t < S3::F * CB ? w * S3::F + t / CB : S3::rem_rb(w, t - S3::F * CB);
          const int cb = t < S3::F * CB ? t % CB : S3::rem_cb(w, t - S3::F * CB);
          const f4 y = z[u];
          if (CALIB && cell0 + 16 * cb + cl < a.n)
#pragma unroll
            for (int r = 0; r < 4; ++r) amx[3] = umaxf(amx[3], __builtin_fabsf(y[r]));
          if constexpr (DBG)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
              dbg_put(a.dbg_acc, a.dbg_acc_row[2], 16 * rb + 4 * g + r, C::H3, cell0 + 16 * cb + cl, acc3[t][r]);
              dbg_put(a.dbg_in, a.dbg_in_row[3], 16 * rb + 4 * g + r, C::H3, cell0 + 16 * cb + cl, Op::q(y[r] * inv_sa[3]));
            }
          put(A2, rb, cb, y, sa[3]);
        }
        if (FRAG == 32 && (t0 & 1)) __builtin_amdgcn_sched_barrier(0);
      }
      zero_pad(C::R3, C::H3P / 16);
    }
    lds_barrier();
    if (CALIB) continue;

    // ------------------------------------------------------------ layer 4 + post
    if (w < CB) {
      f4 o[2];
#pragma unroll
      for (int rb = 0; rb < 2; ++rb)
        o[rb] = Op::SCALED ? f4{0.f, 0.f, 0.f, 0.f} : *(const f4 *)(B4 + 16 * rb + 4 * g);
      // all layer-4 fragments in flight at once (FP8: one k-step at a time,
      // its fragments are twice as large)
      constexpr int NQ4L = FRAG == 32 ? 1 : C::NQ4;
#pragma unroll
      for (int q0 = 0; q0 < C::NQ4; q0 += NQ4L) {
        frag_t w4r[2][NQ4L];
#pragma unroll
        for (int rb = 0; rb < 2; ++rb)
#pragma unroll
          for (int q = 0; q < NQ4L; ++q)
            w4r[rb][q] = W4L ? lds_frag<frag_t>(smem + LW4, rb * C::NQ4 + q0 + q, lane)
                             : ldb_frag<frag_t>(W4, rb * C::NQ4 + q0 + q, voff);
#pragma unroll
        for (int q = 0; q < NQ4L; ++q) {
          const frag_t af = lds_frag<frag_t>(A2, (q0 + q) * CB + w, lane_a());
#pragma unroll
          for (int rb = 0; rb < 2; ++rb) o[rb] = Op::mma(w4r[rb][q], af, o[rb]);
        }
      }
      if constexpr (LATE_XIN) load_xin(tile + gridDim.x);
      if constexpr (DBG) {
        // output row rho = 16 h + 4 g + r holds species rho - 2
#pragma unroll
        for (int h = 0; h < 2; ++h)
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            const int s = 16 * h + 4 * g + r - 2;
            if (vpost && s >= 0 && s < a.S) a.dbg_acc[(int64_t)(a.dbg_acc_row[3] + s) * a.n + ipost] = o[h][r];
          }
        continue;
      }
      if (Op::SCALED)
#pragma unroll
        for (int rb = 0; rb < 2; ++rb) {
          const f4 bias = *(const f4 *)(B4 + 16 * rb + 4 * g);
#pragma unroll
          for (int r = 0; r < 4; ++r) o[rb][r] = __builtin_fmaf(o[rb][r], sout[3], bias[r]);
        }

      if constexpr (PROP) {
        // output k = rho - 2 of row rho = 16h + 4g + r, scaled in FP64
        if (vpost) {
#pragma unroll
          for (int h = 0; h < 2; ++h)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
              const int k = 16 * h + 4 * g + r - 2;
              if (k >= 0 && k < a.K)
                __builtin_nontemporal_store(
                    __builtin_fma((double)o[h][r], dcl[PConst::OUT_SD + k], dcl[PConst::OUT_MU + k]),
                    &a.y[(int64_t)k * a.ld + ipost]);
            }
        }
        continue;
      }
      // post: lane holds output rows rho = 16h + 4g + r, species s = rho - 2;
      // the state from LDS (slot j of the lane: field 16 (j / 4) + 4g + j % 4,
      // i.e. species row rho; T and P are fields 0 and 1 of lane cl)
      const int64_t i = ipost;
      const bool valid = vpost;
      const double *st = (const double *)(smem + C::LDS_ST) + w * 64 * 8;
      const double T = st[cl * 8], P = st[cl * 8 + 1];
      double Yc[8];
#pragma unroll
      for (int j = 0; j < 8; j += 2) {
        const double2v y2 = *(const double2v *)(st + lane * 8 + j);
        Yc[j] = y2[0];
        Yc[j + 1] = y2[1];
      }
      bool bad = !__builtin_isfinite(T) || !__builtin_isfinite(P);
      double Y[8], Yh[8];
      double ssum = 0.0, h0 = 0.0;
      const double t_ref = dcl[DConst::T_REF];
#pragma unroll
      for (int h = 0; h < 2; ++h)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          // every row is evaluated (no branches); rows that are not species
          // take y = 0 and are zeroed at the end
          const int rho = 16 * h + 4 * g + r, s = rho - 2, j = 4 * h + r;
          const bool sp = s >= 0 && s < a.S;
          {
            const double y = sp ? Yc[j] : 0.0;
            Y[j] = y;
            bad |= !__builtin_isfinite(y);
            const float wv = __builtin_fmaf(o[h][r], fcl[FConst::PA + rho], fcl[FConst::PB + rho]);
            double yh = y + inv_change(y, wv, lam, inv_lam);
            // a NaN network output or a non-finite result flags the cell (the
            // inverse transform takes a NaN base like a negative one, and the
            // clamp below would turn a NaN into 0)
            bad |= sp && (__builtin_isnan(wv) || !__builtin_isfinite(yh));
            yh = sp && yh > 0.0 ? yh : 0.0;
            Yh[j] = yh;
            ssum += yh;
            // (the tables are zero past the species rows and without thermo data)
            h0 += y * (dcl[DConst::HF + rho] + dcl[DConst::CP + rho] * (T - t_ref));
          }
        }
      // the cell's four lanes: l, l^16, l^32, l^48
      ssum = quad_sum(ssum);
      double Yn[8];
      double hn = 0.0, cn = 0.0;
      const double rsum = 1.0 / ssum;
      uint32_t nonfin = 0u;
#pragma unroll
      for (int j = 0; j < 8; ++j) {
        Yn[j] = Yh[j] * rsum;
        nonfin |= __builtin_isfinite(Yn[j]) ? 0u : 1u;
        const int rho = 16 * (j >> 2) + 4 * g + (j & 3);
        hn += Yn[j] * dcl[DConst::HF + rho];
        cn += Yn[j] * dcl[DConst::CP + rho];
      }
      double Tn = T;
      if (a.thermo) {
        h0 = quad_sum(h0);
        hn = quad_sum(hn);
        cn = quad_sum(cn);
        Tn = t_ref + (h0 - hn) / cn;
      }
      const uint32_t badq = quad_or((bad ? 1u : 0u) | nonfin);
      const bool okc = !badq && ssum > 0.0 && __builtin_isfinite(ssum) && __builtin_isfinite(Tn);
      // species source terms: ideal-gas density of the state before the step
      double rho_dt = 0.0;
      if (a.omega) {
        double ry = 0.0;
#pragma unroll
        for (int j = 0; j < 8; ++j) ry += Y[j] * dcl[DConst::WINV + 16 * (j >> 2) + 4 * g + (j & 3)];
        ry = quad_sum(ry);
        rho_dt = okc ? P / (kRGas * T * ry) * a.inv_dt : 0.0;
      }
      if (valid) {
        // (FP8: row offsets from an opaque copy of the lane group, recomputed
        // here instead of being kept, or spilled, across the tile loop)
        const int go = FRAG == 32 ? opaque_v(g) : g;
#pragma unroll
        for (int h = 0; h < 2; ++h)
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            const int s = 16 * h + 4 * go + r - 2, j = 4 * h + r;
            if (s >= 0 && s < a.S) {
              __builtin_nontemporal_store(okc ? Yn[j] : Y[j], &a.Y_out[(int64_t)s * a.ld + i]);
              if (a.omega) __builtin_nontemporal_store(okc ? rho_dt * (Yn[j] - Y[j]) : 0.0, &a.omega[(int64_t)s * a.ld + i]);
            }
          }
        if (g == 0) {
          if (a.T_out) __builtin_nontemporal_store(okc ? Tn : T, &a.T_out[i]);
          if (!okc && a.n_bad) atomicAdd(a.n_bad, 1u);
        }
      }
    }
  }

  if (CALIB) {
#pragma unroll
    for (int l = 0; l < 4; ++l) {
      float m = amx[l];
#pragma unroll
      for (int o = 32; o >= 1; o >>= 1) m = umaxf(m, __shfl_xor(m, o));
      if (lane == 0) atomicMax((unsigned int *)(a.amax + l), __builtin_bit_cast(unsigned int, m));
    }
  }
}

// ------------------------------------------------------------------ launchers
template <class C, int GT, bool PROP = false>
static hipError_t launch_step(const StepArgs &a, int grid, hipStream_t s) {
  hipLaunchKernelGGL((chem_step_kernel<C, false, GT, PROP>), dim3(grid), dim3(C::NW * 64),
                     C::lds_bytes(GT), s, a);
  return hipGetLastError();
}
template <class C, int GT>
static hipError_t launch_calib(const StepArgs &a, int grid, hipStream_t s) {
  hipLaunchKernelGGL((chem_step_kernel<C, true, GT>), dim3(grid), dim3(C::NW * 64),
                     C::lds_bytes(GT), s, a);
  return hipGetLastError();
}
template <class C>
static hipError_t launch_dbg(const StepArgs &a, int grid, hipStream_t s) {
  hipLaunchKernelGGL((chem_step_kernel<C, false, 0, false, true>), dim3(grid), dim3(C::NW * 64),
                     C::lds_bytes(0), s, a);
  return hipGetLastError();
}
template <class C, bool CALIB, int GT, bool PROP = false, bool DBG = false>
static hipError_t set_lds_limit() {
  return hipFuncSetAttribute((const void *)chem_step_kernel<C, CALIB, GT, PROP, DBG>,
                             hipFuncAttributeMaxDynamicSharedMemorySize, C::lds_bytes(GT));
}
template <class C, bool WITH_CALIB>
static hipError_t prepare() {
  hipError_t e = set_lds_limit<C, false, 0>();
  if (e == hipSuccess) e = set_lds_limit<C, false, 1>();
  if (e == hipSuccess) e = set_lds_limit<C, false, 2>();
  if (e == hipSuccess) e = set_lds_limit<C, false, 0, false, true>();
  if constexpr (WITH_CALIB) {
    if (e == hipSuccess) e = set_lds_limit<C, true, 0>();
    if (e == hipSuccess) e = set_lds_limit<C, true, 1>();
    if (e == hipSuccess) e = set_lds_limit<C, true, 2>();
  }
  return e;
}

template <class C>
static hipError_t prepare_prop() {
  return set_lds_limit<C, false, 0, true>();
}

template <class C, bool WITH_CALIB>
static void fill_layout(NetLayout *L) {
  L->KS = C::KS;
  L->FRAG = C::FRAG;
  L->EB = C::EB;
  L->MC = C::MC;
  L->R[0] = C::R1; L->R[1] = C::R2; L->R[2] = C::R3; L->R[3] = C::R4;
  L->NQ[0] = C::NQ1; L->NQ[1] = C::NQ2; L->NQ[2] = C::NQ3; L->NQ[3] = C::NQ4;
  L->lds_bytes = C::LDS_BYTES;
  L->step = launch_step<C, 0>;
  L->step_tab = launch_step<C, 1>;
  L->step_tab16 = launch_step<C, 2>;
  L->dbg = launch_dbg<C>;
  L->calib = L->calib_tab = L->calib_tab16 = nullptr;
  if constexpr (WITH_CALIB) {      // (only then are the calibration kernels instantiated)
    L->calib = launch_calib<C, 0>;
    L->calib_tab = launch_calib<C, 1>;
    L->calib_tab16 = launch_calib<C, 2>;
  }
  L->prepare = prepare<C, WITH_CALIB>;
}

template <class C>
static void fill_prop_layout(NetLayout *L) {
  *L = NetLayout{};
  L->KS = C::KS;
  L->FRAG = C::FRAG;
  L->EB = C::EB;
  L->MC = C::MC;
  L->R[0] = C::R1; L->R[1] = C::R2; L->R[2] = C::R3; L->R[3] = C::R4;
  L->NQ[0] = C::NQ1; L->NQ[1] = C::NQ2; L->NQ[2] = C::NQ3; L->NQ[3] = C::NQ4;
  L->lds_bytes = C::LDS_BYTES;
  L->step = launch_step<C, 0, true>;
  L->prepare = prepare_prop<C>;
}

}  // namespace chemdnn
