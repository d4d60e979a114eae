// Host-side structures shared by the C-ABI layer and the kernel translation
// units.  Not part of the public interface.
#pragma once
#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

namespace chemdnn {

enum Prec { P_FP32 = 0, P_BF16 = 1, P_FP16 = 2, P_FP8 = 3 };

// Device constants of a handle, FP32 block (indices in floats).
struct FConst {
  enum {
    ZA = 0,        // [32] z = Y^lam * ZA[f] + ZC[f] for species feature f = s + 2
    ZC = 32,       // [32]
    PA = 64,       // [32] lam * delta = o * PA[rho] + PB[rho], output row rho = s + 2
    PB = 96,       // [32]
    INV_SA = 128,  // [4] 1 / act_scale[l]: multiplier applied before quantising layer l's input
    SOUT = 132,    // [4] act_scale[l] * w_scale[l]: multiplier of layer l's accumulator
    WSCALE = 136,  // [4] w_scale[l]
    ASCALE = 140,  // [4] act_scale[l]
    LAM = 144,     // lam
    INV_LAM = 145, // 1 / lam (rounded from FP64)
    N = 160
  };
};
// FP64 block (indices in doubles).
struct DConst {
  enum {
    T_MU = 0, T_IS = 1, P_MU = 2, P_IS = 3, T_REF = 4, LAM = 5,
    HF = 8,    // [32] by output row rho = s + 2
    CP = 40,   // [32]
    WINV = 72, // [32] 1 / molar mass, mol/kg, by output row (0 past the species)
    N = 104
  };
};

struct StepArgs {
  const double *T, *P, *Y;
  double *Y_out, *T_out;
  uint32_t *n_bad;
  int64_t n, ld, ntiles;
  const void *w[4];      // packed weights
  const float *b[4];     // padded biases (layer 4 shifted by two rows)
  const float *fc;       // FConst block
  const double *dc;      // DConst block
  float *amax;           // calibration output [4] (bit pattern max)
  const void *gtab;      // tabulated GELU: [GTAB_N][4] (c0, c1, c2, 0) per interval,
                         // FP32 or FP16
  double *omega;         // species source terms [S][ld], or NULL
  double inv_dt;         // 1 / dt of the source terms
  int S, thermo;
  // property networks (the kernel's property mode; dc is then a PConst block)
  const double *x;       // input fields [D][ld]
  double *y;             // outputs [K][ld] (output k on row k + 2 of layer 4)
  int D, K;
  // layer dump (the kernel's debug mode): per layer l, its input operand
  // values (decoded to FP32) in rows dbg_in_row[l] .. + widths[l] of dbg_in
  // and its FP32 accumulators in rows dbg_acc_row[l] .. + widths[l+1] of
  // dbg_acc, both [rows][n]
  float *dbg_in, *dbg_acc;
  int dbg_in_row[4], dbg_acc_row[4];
};

// Tabulated GELU: GTAB_N intervals of width 1/GTAB_INV_H from GTAB_LO.
constexpr int GTAB_N = 600;
constexpr float GTAB_LO = -3.0f, GTAB_HI = 3.0f, GTAB_INV_H = 100.0f, GTAB_H = 0.01f;

// Layer-by-layer path (layered.hip): arguments of its three kernels.
struct LayerArgs {
  const uint8_t *W;      // packed weights [R][NQ] fragments
  const float *bias;     // [16 R]
  const uint8_t *X;      // input B fragments [NQ][NCB]
  uint8_t *Y;            // hidden layers: output B fragments [16 R / KS][NCB]
  float *O;              // output layer: FP32 [16 R][ldo]
  int R, NQ, NCB, ldo;   // row-blocks, input k-steps, cell-blocks of the chunk, O's stride
  // debug mode of hidden layers: FP32 accumulators of rows < dbg_rows and
  // cells < dbg_n into dbg_acc[row * dbg_n + cell]
  float *dbg_acc;
  int dbg_rows, dbg_n;
};
struct PrepArgs {
  const double *T, *P, *Y;
  int64_t ld, n0;        // field stride; first cell of the chunk
  int nc, NCB;           // cells of the chunk; cell-blocks written (>= nc / 16)
  uint8_t *X;            // layer-1 B fragments [32 / KS][NCB]
  const float *fc;
  const double *dc;
  int S;
};
struct PostArgs {
  const double *T, *P, *Y;
  double *Y_out, *T_out, *omega;
  uint32_t *n_bad;
  int64_t ld, n0;
  int nc, ldo;
  const float *O;        // network output [S][ldo] of the chunk
  const float *fc;
  const double *dc;
  double inv_dt;
  int S, thermo;
};
// Property networks: FP64 constants of the input and output affine maps.
struct PConst {
  enum {
    IN_MU = 0,     // [32] input mean
    IN_IS = 32,    // [32] 1 / input standard deviation
    OUT_MU = 64,   // [32] output mean
    OUT_SD = 96,   // [32] output standard deviation
    N = 128
  };
};
struct PropPrepArgs {
  const double *x;       // input fields [D][ld]
  int64_t ld, n0;        // field stride; first cell of the chunk
  int nc, NCB, D;        // cells of the chunk; cell-blocks written; input count
  uint8_t *X;            // layer-1 B fragments [32 / KS][NCB]
  const double *pc;      // PConst block
};
struct PropPostArgs {
  double *y;             // outputs [K][ld]
  int64_t ld, n0;
  int nc, K, ldo;        // cells of the chunk; outputs; O's stride
  const float *O;        // network output [K][ldo] of the chunk
  const double *pc;
};
// fmt: 0 FP32, 1 BF16, 2 FP16 operands
hipError_t layered_prepare();
hipError_t launch_prep(int fmt, const PrepArgs &a, hipStream_t s);
hipError_t launch_layer(int fmt, const LayerArgs &a, bool hidden, hipStream_t s);
hipError_t launch_post(const PostArgs &a, hipStream_t s);
hipError_t launch_prop_prep(int fmt, const PropPrepArgs &a, hipStream_t s);
hipError_t launch_prop_post(const PropPostArgs &a, hipStream_t s);
// debug: hidden layer with its accumulators dumped; the operand values of B
// fragments X ([NQ][NCB], features < K, cells < n) decoded into out[f * n + c]
hipError_t launch_layer_dbg(int fmt, const LayerArgs &a, hipStream_t s);
hipError_t launch_frag_decode(int fmt, const uint8_t *X, int NCB, int K, int n, float *out,
                              hipStream_t s);
hipError_t launch_copy_rows(const float *src, int ld_src, int rows, int n, float *dst,
                            hipStream_t s);

// Shape and layout of one compiled network configuration.
struct NetLayout {
  int KS, FRAG, EB;            // operand format of the hidden layers
  int MC;                      // cells per tile
  int R[4], NQ[4];             // row-blocks and k-steps per layer
  int lds_bytes;
  // launches
  hipError_t (*step)(const StepArgs &, int grid, hipStream_t);
  hipError_t (*step_tab)(const StepArgs &, int grid, hipStream_t);   // tabulated GELU
  hipError_t (*step_tab16)(const StepArgs &, int grid, hipStream_t); // ... FP16 table
  hipError_t (*calib)(const StepArgs &, int grid, hipStream_t);  // FP32 only, else null
  hipError_t (*calib_tab)(const StepArgs &, int grid, hipStream_t);
  hipError_t (*calib_tab16)(const StepArgs &, int grid, hipStream_t);
  hipError_t (*dbg)(const StepArgs &, int grid, hipStream_t);    // layer dump
  hipError_t (*prepare)();     // one-time function attributes
};
// The same for the kernel's property mode (hidden widths h1, h2, h3); only
// `step` and `prepare` are set.
bool find_prop_layout(int p, int h1, int h2, int h3, NetLayout *out);

// Finds the compiled configuration for hidden widths (h1, h2, h3) in
// precision p; returns false when the library has none.
bool find_layout(int p, int h1, int h2, int h3, NetLayout *out);
// (per operand format, in step_<format>.hip)
bool find_layout_fp32(int h1, int h2, int h3, NetLayout *out);
bool find_layout_bf16(int h1, int h2, int h3, NetLayout *out);
bool find_layout_fp16(int h1, int h2, int h3, NetLayout *out);
bool find_layout_fp8(int h1, int h2, int h3, NetLayout *out);
bool find_prop_layout_fp32(int h1, int h2, int h3, NetLayout *out);
bool find_prop_layout_bf16(int h1, int h2, int h3, NetLayout *out);
bool find_prop_layout_fp16(int h1, int h2, int h3, NetLayout *out);

// Weight packing (kernels in step.hip).
hipError_t launch_weight_amax(const float *W, int64_t count, uint32_t *amax_bits, hipStream_t s);
hipError_t launch_pow2_scales(const uint32_t *amax_bits, float *fc, int nl, int fp8,
                              hipStream_t s);
hipError_t launch_pack(const float *W, int N, int K, int rowshift, int R, int NQ, int KS,
                       int fmt, const float *w_scale, void *dst, hipStream_t s);
hipError_t launch_pad_bias(const float *b, int N, int rowshift, int NP, float *dst,
                           hipStream_t s);
hipError_t launch_fill_u32(uint32_t *p, uint32_t v, int64_t n, hipStream_t s);

}  // namespace chemdnn
