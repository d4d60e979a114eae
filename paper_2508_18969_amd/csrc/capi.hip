// C ABI of the chemistry-update library: argument checking, workspace
// layout, weight packing and kernel launches.  No device allocation happens
// here; every device buffer is the caller's.
#include <math.h>
#include <stdlib.h>
#include <string.h>

#include <mutex>
#include <new>

#include "../../include/chem_dnn.h"
#include "internal.h"
#include "train.h"

using namespace chemdnn;

struct chem_dnn {
  int S, L, D, H[3], prec;
  int widths[9];
  NetLayout lay;
  // layer-by-layer path (networks the fused kernel does not cover)
  int layered;
  int lR[8], lNQ[8];   // per layer: output row-blocks, input k-steps
  uint8_t *act[2];     // activation fragment buffers of one chunk
  float *obuf;         // FP32 network output of one chunk [32][chunk]
  int dev, n_cu;
  uint8_t *ws;
  size_t ws_bytes;
  // device sub-buffers
  float *fc;
  double *dc;
  uint32_t *amax_bits;
  float *bias[8];
  void *wpack[8];
  TrainScratch tr;
  int64_t max_batch;
  int64_t recompute_chunk;
  int thermo;
  int molar;       // molar masses given: source terms available
  int gelu_form;
  float *gtab;
  // host copies kept alive for the asynchronous uploads
  float hfc[FConst::N];
  double hdc[DConst::N];
  float hgtab[GTAB_N * 4];
};

// Property-network handle: the fused kernel's property mode for the shapes
// it is compiled for, else the layer-by-layer path.
struct chem_prop {
  int L, prec, widths[9];
  int fused;
  NetLayout lay;         // fused: compiled layout
  int n_cu;
  int lR[8], lNQ[8];     // layer by layer: output row-blocks, input k-steps
  int64_t chunk;         // cells per chunk
  uint8_t *ws;
  size_t ws_bytes;
  double *pc;            // PConst block
  float *fc;             // FConst block (fused: operand scales 1)
  float *bias[8];
  void *wpack[8];
  uint8_t *act[2];       // activation fragment buffers of one chunk
  float *obuf;           // FP32 network output of one chunk [32][chunk]
  double hpc[PConst::N]; // host copies kept alive for the asynchronous uploads
  float hfc[FConst::N];
};

// Scratch of the allocation-free training step: one copy per GPU, held until
// the process ends.  Host code never passes this name to a kernel (on the
// host it only stands in for the symbol): it uses the device address that
// hipGetSymbolAddress returns for the current device, kept per device.
static __device__ __align__(256) uint8_t scratch[CHEM_DNN_NOALLOC_SCRATCH_BYTES];

namespace {

constexpr size_t kAlign = 256;

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
uint8_t *g_scratch[kMaxDevices];   // device address of `scratch` on each device

// Looks up the static scratch on device `dev` (the current device) once.
int32_t scratch_init(int dev) {
  if (dev < 0 || dev >= kMaxDevices) return CHEM_DNN_EUNSUPPORTED;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (g_scratch[dev]) return CHEM_DNN_OK;
  void *p = nullptr;
  if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return CHEM_DNN_EHIP;
  g_scratch[dev] = (uint8_t *)p;
  return CHEM_DNN_OK;
}

// Coefficients of the tabulated GELU: per interval i of [-3, 3] (width
// 0.01), the value, first derivative and half the second derivative of
// G(x) = x (1 + tanh v) / 2, v = sqrt(2/pi) (x + 0.044715 x^3), at the
// midpoint, computed in FP64.  With t = tanh v and s = 1 - t^2:
// G' = (1 + t)/2 + x s v'/2 and G'' = s v' + x (s v'' - 2 t s v'^2)/2.
void fill_gelu_table(float *tab) {
  const double c = sqrt(2.0 / M_PI), k = 0.044715;
  for (int i = 0; i < GTAB_N; ++i) {
    const double x = -3.0 + (i + 0.5) * 0.01;
    const double v = c * (x + k * x * x * x), t = tanh(v), s = 1.0 - t * t;
    const double v1 = c * (1.0 + 3.0 * k * x * x), v2 = c * 6.0 * k * x;
    tab[4 * i + 0] = (float)(0.5 * x * (1.0 + t));
    tab[4 * i + 1] = (float)(0.5 * (1.0 + t) + 0.5 * x * s * v1);
    tab[4 * i + 2] = (float)(0.5 * (s * v1 + 0.5 * x * (s * v2 - 2.0 * t * s * v1 * v1)));
    tab[4 * i + 3] = 0.0f;
  }
}
// The FP16 table: the same coefficients rounded once from FP64 to FP16
// (round to nearest even), 8 bytes per interval.
void fill_gelu_table16(_Float16 *tab) {
  const double c = sqrt(2.0 / M_PI), k = 0.044715;
  for (int i = 0; i < GTAB_N; ++i) {
    const double x = -3.0 + (i + 0.5) * 0.01;
    const double v = c * (x + k * x * x * x), t = tanh(v), s = 1.0 - t * t;
    const double v1 = c * (1.0 + 3.0 * k * x * x), v2 = c * 6.0 * k * x;
    tab[4 * i + 0] = (_Float16)(0.5 * x * (1.0 + t));
    tab[4 * i + 1] = (_Float16)(0.5 * (1.0 + t) + 0.5 * x * s * v1);
    tab[4 * i + 2] = (_Float16)(0.5 * (s * v1 + 0.5 * x * (s * v2 - 2.0 * t * s * v1 * v1)));
    tab[4 * i + 3] = (_Float16)0.0;
  }
}
size_t align_up(size_t x) { return (x + kAlign - 1) / kAlign * kAlign; }

int32_t hip_status(hipError_t e) { return e == hipSuccess ? CHEM_DNN_OK : CHEM_DNN_EHIP; }

// Offsets of every sub-buffer inside the workspace.
struct WsPlan {
  size_t fc, dc, amax, gtab, bias[8], w[8], act[2], obuf, train, total;
};

// Layer-by-layer path: cells per chunk (activation buffers are sized for it).
constexpr int64_t kChunk = 32768;

// The layer-by-layer path covers FP32/BF16/FP16 networks with hidden widths
// that are multiples of 256 (its 256-row tiles), up to 4096.
bool layered_shape_ok(const chem_dnn_desc *d) {
  if (d->precision == CHEM_DNN_FP8E4M3 || d->n_layers < 2) return false;
  for (int l = 1; l < d->n_layers; ++l)
    if (d->widths[l] % 256 || d->widths[l] > 4096) return false;
  return true;
}
int ks_of(int prec) { return prec == CHEM_DNN_FP32 ? 16 : 32; }
int eb_of(int prec) { return prec == CHEM_DNN_FP32 ? 4 : 2; }

int32_t check_desc(const chem_dnn_desc *d) {
  if (!d) return CHEM_DNN_EINVAL;
  const int S = d->n_species, L = d->n_layers;
  if (S < 1 || S > 30) return CHEM_DNN_EINVAL;
  if (L < 1 || L > 8) return CHEM_DNN_EINVAL;
  if (d->widths[0] != S + 2 || d->widths[L] != S) return CHEM_DNN_EINVAL;
  for (int l = 1; l < L; ++l)
    if (d->widths[l] < 1 || d->widths[l] > 4096) return CHEM_DNN_EINVAL;
  if (d->precision < CHEM_DNN_FP32 || d->precision > CHEM_DNN_FP8E4M3) return CHEM_DNN_EINVAL;
  if (d->gelu_form != CHEM_DNN_GELU_TANH && d->gelu_form != CHEM_DNN_GELU_TABLE &&
      d->gelu_form != CHEM_DNN_GELU_TABLE16)
    return CHEM_DNN_EINVAL;
  if (!(d->boxcox_lambda > 0.0) || !isfinite(d->boxcox_lambda)) return CHEM_DNN_EINVAL;
  if (!d->in_mean || !d->in_std) return CHEM_DNN_EINVAL;
  for (int f = 0; f < S + 2; ++f)
    if (!(d->in_std[f] > 0.0) || !isfinite(d->in_mean[f]) || !isfinite(d->in_std[f]))
      return CHEM_DNN_EINVAL;
  if ((d->thermo_hf == nullptr) != (d->thermo_cp == nullptr)) return CHEM_DNN_EINVAL;
  if (d->precision == CHEM_DNN_FP8E4M3 && !d->act_amax) return CHEM_DNN_EINVAL;
  if (d->max_batch < 0) return CHEM_DNN_EINVAL;
  if (d->recompute_chunk < 0 || d->recompute_chunk % 16) return CHEM_DNN_EINVAL;
  if (d->molar_mass)
    for (int s = 0; s < S; ++s)
      if (!(d->molar_mass[s] > 0.0) || !isfinite(d->molar_mass[s])) return CHEM_DNN_EINVAL;
  return CHEM_DNN_OK;
}

int32_t plan(const chem_dnn_desc *d, NetLayout *lay, WsPlan *p) {
  int32_t st = check_desc(d);
  if (st) return st;
  *lay = NetLayout{};
  const bool fused = d->n_layers == 4 &&
                     find_layout(d->precision, d->widths[1], d->widths[2], d->widths[3], lay);
  if (!fused) {
    if (!layered_shape_ok(d)) return CHEM_DNN_EUNSUPPORTED;
    if (d->max_batch > 0) return CHEM_DNN_EUNSUPPORTED;   // training: fused shapes only
    if (d->gelu_form != CHEM_DNN_GELU_TANH) return CHEM_DNN_EUNSUPPORTED;
  }
  size_t off = 0;
  p->fc = off; off = align_up(off + FConst::N * sizeof(float));
  p->gtab = off; off = align_up(off + GTAB_N * 4 * sizeof(float));
  p->dc = off; off = align_up(off + DConst::N * sizeof(double));
  p->amax = off; off = align_up(off + 8 * sizeof(uint32_t));
  const int L = d->n_layers;
  if (fused) {
    for (int l = 0; l < 4; ++l) {
      p->bias[l] = off;
      off = align_up(off + (size_t)lay->R[l] * 16 * sizeof(float));
    }
    for (int l = 0; l < 4; ++l) {
      p->w[l] = off;
      off = align_up(off + (size_t)lay->R[l] * 16 * lay->NQ[l] * lay->KS * lay->EB);
    }
    p->act[0] = p->act[1] = p->obuf = 0;
  } else {
    const int ks = ks_of(d->precision), eb = eb_of(d->precision);
    int kmax = 32;
    for (int l = 0; l < L; ++l) {
      const int R = l == L - 1 ? 2 : d->widths[l + 1] / 16;   // output layer: 32 rows
      const int K = l == 0 ? 32 : d->widths[l];
      kmax = K > kmax ? K : kmax;
      p->bias[l] = off;
      off = align_up(off + (size_t)R * 16 * sizeof(float));
      p->w[l] = off;
      off = align_up(off + (size_t)R * 16 * (K / ks) * ks * eb);
    }
    for (int b = 0; b < 2; ++b) {
      p->act[b] = off;
      off = align_up(off + (size_t)kmax * kChunk * eb);
    }
    p->obuf = off;
    off = align_up(off + (size_t)32 * kChunk * sizeof(float));
  }
  p->train = off;
  off += fused ? train_scratch_bytes(d->widths, d->max_batch, d->recompute_chunk) : 0;
  p->total = align_up(off);
  return CHEM_DNN_OK;
}

int32_t current_device(int *dev, int *n_cu) {
  int count = 0;
  if (hipGetDeviceCount(&count) != hipSuccess || count < 1) return CHEM_DNN_ENODEV;
  if (hipGetDevice(dev) != hipSuccess) return CHEM_DNN_ENODEV;
  hipDeviceProp_t prop;
  if (hipGetDeviceProperties(&prop, *dev) != hipSuccess) return CHEM_DNN_EHIP;
  if (strncmp(prop.gcnArchName, "gfx950", 6) != 0) return CHEM_DNN_EUNSUPPORTED;
  *n_cu = prop.multiProcessorCount;
  return CHEM_DNN_OK;
}

// Power-of-two FP8 activation scale of one layer from its calibration amax.
double act_scale_of(float amax) {
  double a = (double)amax;
  if (!(a > 0.0) || !isfinite(a)) return 1.0;
  int e;
  double m = frexp(a / 448.0, &e);
  return ldexp(1.0, m == 0.5 ? e - 1 : e);
}

size_t param_offset(const int *widths, int layer, bool bias) {
  size_t off = 0;
  for (int l = 0; l < layer; ++l) off += (size_t)widths[l] * widths[l + 1] + widths[l + 1];
  if (bias) off += (size_t)widths[layer] * widths[layer + 1];
  return off;
}

int32_t pack_params(chem_dnn *h, const float *params, hipStream_t s) {
  const bool fp8 = h->prec == CHEM_DNN_FP8E4M3;
  hipError_t e = hipSuccess;
  e = launch_fill_u32(h->amax_bits, 0u, 4, s);
  for (int l = 0; l < 4 && e == hipSuccess; ++l)
    if (fp8)
      e = launch_weight_amax(params + param_offset(h->widths, l, false),
                             (int64_t)h->widths[l] * h->widths[l + 1], h->amax_bits + l, s);
  if (e == hipSuccess) e = launch_pow2_scales(h->amax_bits, h->fc, 4, fp8 ? 1 : 0, s);
  static const int fmt_of[4] = {0, 1, 2, 3};
  if (h->layered) {
    // output rows unshifted; the w_scale operand is read for FP8 only
    for (int l = 0; l < h->L && e == hipSuccess; ++l) {
      const int N = h->widths[l + 1], K = h->widths[l];
      e = launch_pack(params + param_offset(h->widths, l, false), N, K, 0, h->lR[l], h->lNQ[l],
                      ks_of(h->prec), fmt_of[h->prec], h->fc + FConst::WSCALE, h->wpack[l], s);
      if (e == hipSuccess)
        e = launch_pad_bias(params + param_offset(h->widths, l, true), N, 0, h->lR[l] * 16,
                            h->bias[l], s);
    }
    return hip_status(e);
  }
  for (int l = 0; l < 4 && e == hipSuccess; ++l) {
    const int N = h->widths[l + 1], K = h->widths[l];
    const int rowshift = (l == 3) ? 2 : 0;
    const int ks = h->lay.KS;
    e = launch_pack(params + param_offset(h->widths, l, false), N, K, rowshift, h->lay.R[l],
                    h->lay.NQ[l], ks, fmt_of[h->prec], h->fc + FConst::WSCALE + l, h->wpack[l], s);
    if (e == hipSuccess)
      e = launch_pad_bias(params + param_offset(h->widths, l, true), N, rowshift,
                          h->lay.R[l] * 16, h->bias[l], s);
  }
  return hip_status(e);
}

StepArgs step_args(chem_dnn *h, int64_t n, int64_t ld, const double *T, const double *P,
                   const double *Y, double *Y_out, double *T_out, uint32_t *n_bad) {
  StepArgs a{};
  a.T = T; a.P = P; a.Y = Y; a.Y_out = Y_out; a.T_out = T_out; a.n_bad = n_bad;
  a.n = n; a.ld = ld;
  a.ntiles = (n + h->lay.MC - 1) / h->lay.MC;
  for (int l = 0; l < 4; ++l) { a.w[l] = h->wpack[l]; a.b[l] = h->bias[l]; }
  a.fc = h->fc; a.dc = h->dc;
  a.amax = nullptr;
  a.gtab = h->gtab;
  a.omega = nullptr;
  a.inv_dt = 0.0;
  a.S = h->S;
  a.thermo = h->thermo;
  return a;
}

// The layer-by-layer path over chunks of kChunk cells: preprocess, one
// launch per layer, post-processing.
int32_t run_layered(chem_dnn *h, int64_t n, int64_t ld, const double *T, const double *P,
                    const double *Y, double *Y_out, double *T_out, double *omega, double inv_dt,
                    uint32_t *n_bad, hipStream_t s) {
  const int fmt = h->prec;   // 0 FP32, 1 BF16, 2 FP16
  // the chunk buffers lie inside the workspace
  const uint8_t *end = h->ws + h->ws_bytes;
  if (h->act[0] < h->ws || h->act[1] < h->ws || (const uint8_t *)h->obuf < h->ws ||
      (const uint8_t *)(h->obuf + 32 * kChunk) > end)
    return CHEM_DNN_EWORKSPACE;
  hipError_t e = hipSuccess;
  for (int64_t n0 = 0; n0 < n && e == hipSuccess; n0 += kChunk) {
    const int nc = (int)(n - n0 < kChunk ? n - n0 : kChunk);
    const int ncb = (nc + 255) / 256 * 16;     // whole 256-cell tiles
    PrepArgs pa{T, P, Y, ld, n0, nc, ncb, h->act[0], h->fc, h->dc, h->S};
    e = launch_prep(fmt, pa, s);
    int cur = 0;
    for (int l = 0; l < h->L && e == hipSuccess; ++l) {
      LayerArgs la{h->wpack[l] ? (const uint8_t *)h->wpack[l] : nullptr, h->bias[l], h->act[cur],
                   h->act[cur ^ 1], h->obuf, h->lR[l], h->lNQ[l], ncb, 16 * ncb, nullptr, 0, 0};
      e = launch_layer(fmt, la, l < h->L - 1, s);
      cur ^= 1;
    }
    if (e == hipSuccess) {
      PostArgs po{T, P, Y, Y_out, T_out, omega, n_bad, ld, n0, nc, 16 * ncb, h->obuf, h->fc,
                  h->dc, inv_dt, h->S, h->thermo};
      e = launch_post(po, s);
    }
  }
  return hip_status(e);
}

// ---- property networks
int32_t check_prop_desc(const chem_prop_desc *d) {
  if (!d) return CHEM_DNN_EINVAL;
  const int L = d->n_layers;
  if (L < 2 || L > 8) return CHEM_DNN_EINVAL;
  const int D = d->widths[0], K = d->widths[L];
  if (D < 1 || D > 32 || K < 1 || K > 32) return CHEM_DNN_EINVAL;
  for (int l = 1; l < L; ++l)
    if (d->widths[l] < 1 || d->widths[l] > 4096) return CHEM_DNN_EINVAL;
  if (d->precision < CHEM_DNN_FP32 || d->precision > CHEM_DNN_FP8E4M3) return CHEM_DNN_EINVAL;
  if (!d->in_mean || !d->in_std) return CHEM_DNN_EINVAL;
  for (int f = 0; f < D; ++f)
    if (!(d->in_std[f] > 0.0) || !isfinite(d->in_mean[f]) || !isfinite(d->in_std[f]))
      return CHEM_DNN_EINVAL;
  for (int k = 0; k < K; ++k)
    if ((d->out_mean && !isfinite(d->out_mean[k])) || (d->out_std && !isfinite(d->out_std[k])))
      return CHEM_DNN_EINVAL;
  if (d->precision == CHEM_DNN_FP8E4M3) return CHEM_DNN_EUNSUPPORTED;
  for (int l = 1; l < L; ++l)
    if (d->widths[l] % 256) return CHEM_DNN_EUNSUPPORTED;   // the layer kernel's row tiles
  return CHEM_DNN_OK;
}

// Cells per chunk: doubled from kChunk (up to 4 kChunk) while the widest
// hidden activation of a chunk stays within 256 MiB, so that narrow networks
// give the layer kernel enough cell tiles and their small kernels (input,
// output layer, output scaling) enough cells per launch.
int64_t prop_chunk(const chem_prop_desc *d) {
  int hmax = 1;
  for (int l = 1; l < d->n_layers; ++l) hmax = d->widths[l] > hmax ? d->widths[l] : hmax;
  const int64_t cap = (int64_t)256 << 20;
  int64_t c = kChunk;
  while (c < 4 * kChunk && 2 * c * hmax * eb_of(d->precision) <= cap) c *= 2;
  return c;
}

struct PropPlan {
  size_t pc, fc, bias[8], w[8], act[2], obuf, total;
  int64_t chunk;
  bool fused;
  NetLayout lay;
};

int32_t prop_plan(const chem_prop_desc *d, PropPlan *p) {
  int32_t st = check_prop_desc(d);
  if (st) return st;
  const int L = d->n_layers, ks = ks_of(d->precision), eb = eb_of(d->precision);
  p->lay = NetLayout{};
  // the fused kernel's output rows are 2 .. K+1 of 32
  p->fused = L == 4 && d->widths[L] <= 30 &&
             find_prop_layout(d->precision, d->widths[1], d->widths[2], d->widths[3], &p->lay);
  p->chunk = prop_chunk(d);
  size_t off = 0;
  p->pc = off; off = align_up(off + PConst::N * sizeof(double));
  p->fc = off; off = align_up(off + FConst::N * sizeof(float));
  if (p->fused) {
    for (int l = 0; l < 4; ++l) {
      p->bias[l] = off;
      off = align_up(off + (size_t)p->lay.R[l] * 16 * sizeof(float));
      p->w[l] = off;
      off = align_up(off + (size_t)p->lay.R[l] * 16 * p->lay.NQ[l] * p->lay.KS * p->lay.EB);
    }
    p->act[0] = p->act[1] = p->obuf = 0;
    p->total = off;
    return CHEM_DNN_OK;
  }
  int kmax = 32;
  for (int l = 0; l < L; ++l) {
    const int R = l == L - 1 ? 2 : d->widths[l + 1] / 16;   // output layer: 32 rows
    const int K = l == 0 ? 32 : d->widths[l];
    kmax = K > kmax ? K : kmax;
    p->bias[l] = off;
    off = align_up(off + (size_t)R * 16 * sizeof(float));
    p->w[l] = off;
    off = align_up(off + (size_t)R * 16 * (K / ks) * ks * eb);
  }
  for (int b = 0; b < 2; ++b) {
    p->act[b] = off;
    off = align_up(off + (size_t)kmax * p->chunk * eb);
  }
  p->obuf = off;
  off = align_up(off + (size_t)32 * p->chunk * sizeof(float));
  p->total = off;
  return CHEM_DNN_OK;
}

int32_t prop_pack(chem_prop *h, const float *params, hipStream_t s) {
  hipError_t e = hipSuccess;
  if (h->fused) {
    // the fused kernel's layout: output layer shifted by two rows
    for (int l = 0; l < 4 && e == hipSuccess; ++l) {
      const int N = h->widths[l + 1], K = h->widths[l], rowshift = l == 3 ? 2 : 0;
      e = launch_pack(params + param_offset(h->widths, l, false), N, K, rowshift, h->lay.R[l],
                      h->lay.NQ[l], h->lay.KS, h->prec, nullptr, h->wpack[l], s);
      if (e == hipSuccess)
        e = launch_pad_bias(params + param_offset(h->widths, l, true), N, rowshift,
                            h->lay.R[l] * 16, h->bias[l], s);
    }
    return hip_status(e);
  }
  for (int l = 0; l < h->L && e == hipSuccess; ++l) {
    const int N = h->widths[l + 1], K = h->widths[l];
    e = launch_pack(params + param_offset(h->widths, l, false), N, K, 0, h->lR[l], h->lNQ[l],
                    ks_of(h->prec), h->prec, nullptr, h->wpack[l], s);
    if (e == hipSuccess)
      e = launch_pad_bias(params + param_offset(h->widths, l, true), N, 0, h->lR[l] * 16,
                          h->bias[l], s);
  }
  return hip_status(e);
}

// The fused kernel of the handle's activation form.
hipError_t (*step_launch(const chem_dnn *h))(const StepArgs &, int, hipStream_t) {
  return h->gelu_form == CHEM_DNN_GELU_TABLE   ? h->lay.step_tab
         : h->gelu_form == CHEM_DNN_GELU_TABLE16 ? h->lay.step_tab16
                                                 : h->lay.step;
}

int grid_for(const chem_dnn *h, int64_t ntiles) {
  int64_t g = ntiles < h->n_cu ? ntiles : h->n_cu;
  return (int)(g < 1 ? 1 : g);
}

}  // namespace

extern "C" {

int32_t chem_dnn_abi_version(void) { return 5; }

const char *chem_dnn_strerror(int32_t st) {
  switch (st) {
    case CHEM_DNN_OK: return "ok";
    case CHEM_DNN_EINVAL: return "invalid argument";
    case CHEM_DNN_ENODEV: return "no HIP device";
    case CHEM_DNN_EWORKSPACE: return "workspace missing, misaligned or too small";
    case CHEM_DNN_EUNSUPPORTED: return "unsupported device or network shape";
    case CHEM_DNN_EHIP: return "HIP runtime error";
    case CHEM_DNN_ETOOLARGE:
      return "request exceeds the allocation-free entry point's static scratch "
             "(CHEM_DNN_NOALLOC_SCRATCH_BYTES)";
    default: return "unknown status";
  }
}

int32_t chem_dnn_workspace_bytes(const chem_dnn_desc *desc, size_t *bytes) {
  if (!bytes) return CHEM_DNN_EINVAL;
  NetLayout lay;
  WsPlan p;
  int32_t st = plan(desc, &lay, &p);
  if (st) return st;
  *bytes = p.total;
  return CHEM_DNN_OK;
}

int32_t chem_dnn_init(const chem_dnn_desc *d, const float *params, void *workspace,
                      size_t workspace_bytes, void *stream, chem_dnn **out) {
  if (!out) return CHEM_DNN_EINVAL;
  *out = nullptr;
  NetLayout lay;
  WsPlan p;
  int32_t st = plan(d, &lay, &p);
  if (st) return st;
  if (!params) return CHEM_DNN_EINVAL;
  if (!workspace || ((uintptr_t)workspace % kAlign) || workspace_bytes < p.total)
    return CHEM_DNN_EWORKSPACE;
  int dev = 0, n_cu = 0;
  st = current_device(&dev, &n_cu);
  if (st) return st;
  const bool layered = lay.prepare == nullptr;
  // the static scratch of the allocation-free training step (fused shapes)
  if (!layered && (st = scratch_init(dev)) != CHEM_DNN_OK) return st;
  if ((layered ? layered_prepare() : lay.prepare()) != hipSuccess) return CHEM_DNN_EHIP;
  if (d->max_batch > 0 && train_prepare() != hipSuccess) return CHEM_DNN_EHIP;

  chem_dnn *h = new (std::nothrow) chem_dnn();
  if (!h) return CHEM_DNN_EHIP;
  h->S = d->n_species;
  h->L = d->n_layers;
  h->D = d->widths[0];
  for (int l = 0; l <= h->L; ++l) h->widths[l] = d->widths[l];
  for (int l = 0; l < 3; ++l) h->H[l] = d->widths[l + 1];
  h->layered = layered ? 1 : 0;
  if (layered) {
    const int ks = ks_of(d->precision);
    for (int l = 0; l < h->L; ++l) {
      h->lR[l] = l == h->L - 1 ? 2 : d->widths[l + 1] / 16;
      h->lNQ[l] = (l == 0 ? 32 : d->widths[l]) / ks;
    }
  }
  h->prec = d->precision;
  h->lay = lay;
  h->dev = dev;
  h->n_cu = n_cu;
  h->ws = (uint8_t *)workspace;
  h->ws_bytes = workspace_bytes;
  if (layered) {
    // (workspace pointers: only once h->ws is set)
    h->act[0] = h->ws + p.act[0];
    h->act[1] = h->ws + p.act[1];
    h->obuf = (float *)(h->ws + p.obuf);
  }
  h->fc = (float *)(h->ws + p.fc);
  h->gtab = (float *)(h->ws + p.gtab);
  h->dc = (double *)(h->ws + p.dc);
  h->amax_bits = (uint32_t *)(h->ws + p.amax);
  for (int l = 0; l < (layered ? h->L : 4); ++l) {
    h->bias[l] = (float *)(h->ws + p.bias[l]);
    h->wpack[l] = h->ws + p.w[l];
  }
  h->max_batch = d->max_batch;
  h->recompute_chunk = d->recompute_chunk;
  train_scratch_layout(&h->tr, h->ws + p.train, d->widths, d->max_batch, d->recompute_chunk);
  h->thermo = d->thermo_hf ? 1 : 0;
  h->molar = d->molar_mass ? 1 : 0;
  h->gelu_form = d->gelu_form;
  if (d->gelu_form == CHEM_DNN_GELU_TABLE16) {
    memset(h->hgtab, 0, sizeof(h->hgtab));
    fill_gelu_table16((_Float16 *)h->hgtab);       // (the first 4.8 KB of the buffer)
  } else {
    fill_gelu_table(h->hgtab);
  }

  // constants
  const double lam = d->boxcox_lambda;
  memset(h->hfc, 0, sizeof(h->hfc));
  memset(h->hdc, 0, sizeof(h->hdc));
  for (int s = 0; s < h->S; ++s) {
    const int f = s + 2;
    const double mu = d->in_mean[f], sd = d->in_std[f];
    h->hfc[FConst::ZA + f] = (float)(1.0 / (lam * sd));
    h->hfc[FConst::ZC + f] = (float)(-(1.0 / lam + mu) / sd);
    const double om = d->out_mean ? d->out_mean[s] : 0.0;
    const double os = d->out_std ? d->out_std[s] : 1.0;
    h->hfc[FConst::PA + f] = (float)(lam * os);
    h->hfc[FConst::PB + f] = (float)(lam * om);
    if (h->thermo) {
      h->hdc[DConst::HF + f] = d->thermo_hf[s];
      h->hdc[DConst::CP + f] = d->thermo_cp[s];
    }
    if (d->molar_mass) h->hdc[DConst::WINV + f] = 1.0 / d->molar_mass[s];
  }
  for (int l = 0; l < 4; ++l) {
    const double sa = (h->prec == CHEM_DNN_FP8E4M3) ? act_scale_of(d->act_amax[l]) : 1.0;
    h->hfc[FConst::ASCALE + l] = (float)sa;
    h->hfc[FConst::INV_SA + l] = (float)(1.0 / sa);
    h->hfc[FConst::WSCALE + l] = 1.0f;
    h->hfc[FConst::SOUT + l] = (float)sa;
  }
  h->hfc[FConst::LAM] = (float)lam;
  h->hfc[FConst::INV_LAM] = (float)(1.0 / lam);
  h->hdc[DConst::T_MU] = d->in_mean[0];
  h->hdc[DConst::T_IS] = 1.0 / d->in_std[0];
  h->hdc[DConst::P_MU] = d->in_mean[1];
  h->hdc[DConst::P_IS] = 1.0 / d->in_std[1];
  h->hdc[DConst::T_REF] = d->t_ref;
  h->hdc[DConst::LAM] = lam;

  hipStream_t s = (hipStream_t)stream;
  hipError_t e = hipMemcpyAsync(h->fc, h->hfc, sizeof(h->hfc), hipMemcpyHostToDevice, s);
  if (e == hipSuccess) e = hipMemcpyAsync(h->dc, h->hdc, sizeof(h->hdc), hipMemcpyHostToDevice, s);
  if (e == hipSuccess) e = hipMemcpyAsync(h->gtab, h->hgtab, sizeof(h->hgtab), hipMemcpyHostToDevice, s);
  if (e != hipSuccess) {
    delete h;
    return CHEM_DNN_EHIP;
  }
  st = pack_params(h, params, s);
  if (st) {
    delete h;
    return st;
  }
  // the host staging arrays must not be released before the copies finish
  if (hipStreamSynchronize(s) != hipSuccess) {
    delete h;
    return CHEM_DNN_EHIP;
  }
  *out = h;
  return CHEM_DNN_OK;
}

int32_t chem_dnn_set_params(chem_dnn *h, const float *params, void *stream) {
  if (!h || !params) return CHEM_DNN_EINVAL;
  return pack_params(h, params, (hipStream_t)stream);
}

int32_t chem_dnn_step(chem_dnn *h, int64_t n, int64_t ld, const double *T, const double *P,
                      const double *Y, double *Y_out, double *T_out, uint32_t *n_bad,
                      void *stream) {
  if (!h || n < 0 || ld < n) return CHEM_DNN_EINVAL;
  if (n == 0) return CHEM_DNN_OK;
  if (!T || !P || !Y || !Y_out) return CHEM_DNN_EINVAL;
  if (T_out && !h->thermo) return CHEM_DNN_EINVAL;
  if (h->layered)
    return run_layered(h, n, ld, T, P, Y, Y_out, T_out, nullptr, 0.0, n_bad, (hipStream_t)stream);
  StepArgs a = step_args(h, n, ld, T, P, Y, Y_out, T_out, n_bad);
  return hip_status(step_launch(h)(a, grid_for(h, a.ntiles), (hipStream_t)stream));
}

int32_t chem_dnn_step_source(chem_dnn *h, int64_t n, int64_t ld, const double *T,
                             const double *P, const double *Y, double *Y_out, double *T_out,
                             double *omega, double dt, uint32_t *n_bad, void *stream) {
  if (!h || n < 0 || ld < n) return CHEM_DNN_EINVAL;
  if (!h->molar || !(dt > 0.0) || !isfinite(dt)) return CHEM_DNN_EINVAL;
  if (n == 0) return CHEM_DNN_OK;
  if (!T || !P || !Y || !Y_out || !omega) return CHEM_DNN_EINVAL;
  if (T_out && !h->thermo) return CHEM_DNN_EINVAL;
  const void *o = omega;
  if (o == T || o == P || o == Y || o == Y_out || o == T_out) return CHEM_DNN_EINVAL;
  if (h->layered)
    return run_layered(h, n, ld, T, P, Y, Y_out, T_out, omega, 1.0 / dt, n_bad,
                       (hipStream_t)stream);
  StepArgs a = step_args(h, n, ld, T, P, Y, Y_out, T_out, n_bad);
  a.omega = omega;
  a.inv_dt = 1.0 / dt;
  return hip_status(step_launch(h)(a, grid_for(h, a.ntiles), (hipStream_t)stream));
}

int32_t chem_dnn_calibrate(chem_dnn *h, int64_t n, int64_t ld, const double *T, const double *P,
                           const double *Y, float *amax, void *stream) {
  if (!h || n < 0 || ld < n || !amax) return CHEM_DNN_EINVAL;
  if (h->prec != CHEM_DNN_FP32 || !h->lay.calib) return CHEM_DNN_EINVAL;
  hipStream_t s = (hipStream_t)stream;
  hipError_t e = launch_fill_u32((uint32_t *)amax, 0u, 4, s);
  if (e != hipSuccess || n == 0) return hip_status(e);
  if (!T || !P || !Y) return CHEM_DNN_EINVAL;
  StepArgs a = step_args(h, n, ld, T, P, Y, nullptr, nullptr, nullptr);
  a.amax = amax;
  auto launch = h->gelu_form == CHEM_DNN_GELU_TABLE   ? h->lay.calib_tab
                : h->gelu_form == CHEM_DNN_GELU_TABLE16 ? h->lay.calib_tab16
                                                        : h->lay.calib;
  return hip_status(launch(a, grid_for(h, a.ntiles), s));
}

int32_t chem_dnn_get_scales(chem_dnn *h, float *act_scale, float *w_scale, void *stream) {
  if (!h || !act_scale || !w_scale) return CHEM_DNN_EINVAL;
  hipStream_t s = (hipStream_t)stream;
  float tmp[FConst::N];
  hipError_t e = hipMemcpyAsync(tmp, h->fc, sizeof(tmp), hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e != hipSuccess) return CHEM_DNN_EHIP;
  for (int l = 0; l < h->L; ++l) {       // (layers past the fourth: never scaled)
    act_scale[l] = l < 4 ? tmp[FConst::ASCALE + l] : 1.0f;
    w_scale[l] = l < 4 ? tmp[FConst::WSCALE + l] : 1.0f;
  }
  return CHEM_DNN_OK;
}

int32_t chem_dnn_mlp_forward(chem_dnn *h, int64_t B, int64_t ld, const float *x,
                             const float *params, float *out, float *saved, void *stream) {
  if (!h || B < 0 || ld < B) return CHEM_DNN_EINVAL;
  if (h->layered) return CHEM_DNN_EUNSUPPORTED;
  if (B == 0) return CHEM_DNN_OK;
  if (!x || !params || !out) return CHEM_DNN_EINVAL;
  if (!saved && B > h->max_batch) return CHEM_DNN_EINVAL;
  return hip_status(train_mlp_forward(h->widths, B, ld, x, params, out, saved, &h->tr,
                                      (hipStream_t)stream));
}

int32_t chem_dnn_mlp_backward(chem_dnn *h, int64_t B, int64_t ld, const float *x,
                              const float *params, const float *saved, const float *grad_out,
                              float *grad_params, float *grad_x, void *stream) {
  if (!h || B < 0 || ld < B) return CHEM_DNN_EINVAL;
  if (h->layered) return CHEM_DNN_EUNSUPPORTED;
  if (!params || !grad_params) return CHEM_DNN_EINVAL;
  if (B > 0 && (!x || !grad_out)) return CHEM_DNN_EINVAL;
  if (B > h->max_batch) return CHEM_DNN_EINVAL;
  return hip_status(train_mlp_backward(h->widths, B, ld, x, params, saved, grad_out,
                                       grad_params, grad_x, &h->tr, (hipStream_t)stream));
}

int32_t chem_dnn_train_step(chem_dnn *h, int64_t B, int64_t ld, const double *T, const double *P,
                            const double *Y, const float *target, float *params, float *grads,
                            float *adam_m, float *adam_v, int64_t step, float lr,
                            int32_t recompute, float *loss, void *stream) {
  if (h && h->layered) return CHEM_DNN_EUNSUPPORTED;
  if (!h || B < 1 || ld < B || B > h->max_batch || step < 1) return CHEM_DNN_EINVAL;
  if (!T || !P || !Y || !target || !params || !grads || !adam_m || !adam_v || !loss)
    return CHEM_DNN_EINVAL;
  if (!(lr > 0.0f)) return CHEM_DNN_EINVAL;
  return hip_status(train_step(h->widths, B, ld, T, P, Y, target, params, grads, adam_m, adam_v,
                               step, lr, recompute != 0, loss, h->fc, h->dc, &h->tr,
                               (hipStream_t)stream));
}

int32_t chem_dnn_train_step_noalloc(chem_dnn *h, int64_t B, int64_t ld, const double *T,
                                    const double *P, const double *Y, const float *target,
                                    float *params, float *grads, float *adam_m, float *adam_v,
                                    int64_t step, float lr, float *loss, void *stream) {
  if (h && h->layered) return CHEM_DNN_EUNSUPPORTED;
  if (!h || B < 1 || ld < B || step < 1) return CHEM_DNN_EINVAL;
  if (!T || !P || !Y || !target || !params || !grads || !adam_m || !adam_v || !loss)
    return CHEM_DNN_EINVAL;
  if (!(lr > 0.0f)) return CHEM_DNN_EINVAL;
  uint8_t *base = (h->dev >= 0 && h->dev < kMaxDevices) ? g_scratch[h->dev] : nullptr;
  if (!base) return CHEM_DNN_EHIP;
  // the same chunk schedule as chem_dnn_train_step on a handle with this
  // recompute_chunk; per-sample buffers padded to 16 samples (aligned rows)
  const int64_t cap = (B + 15) / 16 * 16;
  if (train_scratch_bytes(h->widths, cap, h->recompute_chunk) > CHEM_DNN_NOALLOC_SCRATCH_BYTES)
    return CHEM_DNN_ETOOLARGE;
  TrainScratch t;
  train_scratch_layout(&t, base, h->widths, cap, h->recompute_chunk);
  return hip_status(train_step(h->widths, B, ld, T, P, Y, target, params, grads, adam_m, adam_v,
                               step, lr, false, loss, h->fc, h->dc, &t, (hipStream_t)stream));
}

int32_t chem_dnn_destroy(chem_dnn *h) {
  if (!h) return CHEM_DNN_EINVAL;
  delete h;
  return CHEM_DNN_OK;
}

int32_t chem_dnn_debug_layers(chem_dnn *h, int64_t n, int64_t ld, const double *T,
                              const double *P, const double *Y, float *qin, float *acc,
                              void *stream) {
  if (!h || n < 0 || ld < n || n > CHEM_DNN_DEBUG_MAX_CELLS) return CHEM_DNN_EINVAL;
  if (n == 0) return CHEM_DNN_OK;
  if (!T || !P || !Y || !qin || !acc) return CHEM_DNN_EINVAL;
  if (h->gelu_form != CHEM_DNN_GELU_TANH) return CHEM_DNN_EUNSUPPORTED;
  hipStream_t s = (hipStream_t)stream;
  int in_row[8], acc_row[8];
  for (int l = 0, ri = 0, ra = 0; l < h->L; ++l) {
    in_row[l] = ri;
    acc_row[l] = ra;
    ri += h->widths[l];
    ra += h->widths[l + 1];
  }
  if (!h->layered) {
    if (!h->lay.dbg) return CHEM_DNN_EUNSUPPORTED;
    StepArgs a = step_args(h, n, ld, T, P, Y, nullptr, nullptr, nullptr);
    a.dbg_in = qin;
    a.dbg_acc = acc;
    for (int l = 0; l < 4; ++l) {
      a.dbg_in_row[l] = in_row[l];
      a.dbg_acc_row[l] = acc_row[l];
    }
    return hip_status(h->lay.dbg(a, grid_for(h, a.ntiles), s));
  }
  // layer by layer: one chunk (n <= CHEM_DNN_DEBUG_MAX_CELLS < kChunk)
  const int fmt = h->prec;
  const int nc = (int)n, ncb = (nc + 255) / 256 * 16;
  PrepArgs pa{T, P, Y, ld, 0, nc, ncb, h->act[0], h->fc, h->dc, h->S};
  hipError_t e = launch_prep(fmt, pa, s);
  if (e == hipSuccess) e = launch_frag_decode(fmt, h->act[0], ncb, h->widths[0], nc, qin, s);
  int cur = 0;
  for (int l = 0; l < h->L && e == hipSuccess; ++l) {
    const bool hidden = l < h->L - 1;
    LayerArgs la{(const uint8_t *)h->wpack[l], h->bias[l], h->act[cur], h->act[cur ^ 1], h->obuf,
                 h->lR[l], h->lNQ[l], ncb, 16 * ncb, nullptr, 0, 0};
    if (hidden) {
      la.dbg_acc = acc + (size_t)acc_row[l] * nc;
      la.dbg_rows = h->widths[l + 1];
      la.dbg_n = nc;
      e = launch_layer_dbg(fmt, la, s);
      if (e == hipSuccess)
        e = launch_frag_decode(fmt, h->act[cur ^ 1], ncb, h->widths[l + 1], nc,
                               qin + (size_t)in_row[l + 1] * nc, s);
    } else {
      e = launch_layer(fmt, la, false, s);
      if (e == hipSuccess)
        e = launch_copy_rows(h->obuf, 16 * ncb, h->S, nc, acc + (size_t)acc_row[l] * nc, s);
    }
    cur ^= 1;
  }
  return hip_status(e);
}

int32_t chem_prop_workspace_bytes(const chem_prop_desc *desc, size_t *bytes) {
  if (!bytes) return CHEM_DNN_EINVAL;
  PropPlan p;
  int32_t st = prop_plan(desc, &p);
  if (st) return st;
  *bytes = p.total;
  return CHEM_DNN_OK;
}

int32_t chem_prop_init(const chem_prop_desc *d, const float *params, void *workspace,
                       size_t workspace_bytes, void *stream, chem_prop **out) {
  if (!out) return CHEM_DNN_EINVAL;
  *out = nullptr;
  PropPlan p;
  int32_t st = prop_plan(d, &p);
  if (st) return st;
  if (!params) return CHEM_DNN_EINVAL;
  if (!workspace || ((uintptr_t)workspace % kAlign) || workspace_bytes < p.total)
    return CHEM_DNN_EWORKSPACE;
  int dev = 0, n_cu = 0;
  st = current_device(&dev, &n_cu);
  if (st) return st;
  if ((p.fused ? p.lay.prepare() : layered_prepare()) != hipSuccess) return CHEM_DNN_EHIP;
  chem_prop *h = new (std::nothrow) chem_prop();
  if (!h) return CHEM_DNN_EHIP;
  h->L = d->n_layers;
  h->prec = d->precision;
  h->fused = p.fused ? 1 : 0;
  h->lay = p.lay;
  h->n_cu = n_cu;
  for (int l = 0; l <= h->L; ++l) h->widths[l] = d->widths[l];
  const int ks = ks_of(d->precision);
  for (int l = 0; l < h->L; ++l) {
    h->lR[l] = l == h->L - 1 ? 2 : d->widths[l + 1] / 16;
    h->lNQ[l] = (l == 0 ? 32 : d->widths[l]) / ks;
  }
  h->chunk = p.chunk;
  h->ws = (uint8_t *)workspace;
  h->ws_bytes = workspace_bytes;
  h->pc = (double *)(h->ws + p.pc);
  h->fc = (float *)(h->ws + p.fc);
  for (int l = 0; l < h->L; ++l) {
    h->bias[l] = (float *)(h->ws + p.bias[l]);
    h->wpack[l] = h->ws + p.w[l];
  }
  if (!h->fused) {
    h->act[0] = h->ws + p.act[0];
    h->act[1] = h->ws + p.act[1];
    h->obuf = (float *)(h->ws + p.obuf);
  }
  memset(h->hfc, 0, sizeof(h->hfc));
  for (int l = 0; l < 4; ++l) {
    h->hfc[FConst::ASCALE + l] = h->hfc[FConst::INV_SA + l] = 1.0f;
    h->hfc[FConst::WSCALE + l] = h->hfc[FConst::SOUT + l] = 1.0f;
  }
  memset(h->hpc, 0, sizeof(h->hpc));
  for (int f = 0; f < d->widths[0]; ++f) {
    h->hpc[PConst::IN_MU + f] = d->in_mean[f];
    h->hpc[PConst::IN_IS + f] = 1.0 / d->in_std[f];
  }
  for (int k = 0; k < d->widths[h->L]; ++k) {
    h->hpc[PConst::OUT_MU + k] = d->out_mean ? d->out_mean[k] : 0.0;
    h->hpc[PConst::OUT_SD + k] = d->out_std ? d->out_std[k] : 1.0;
  }
  hipStream_t s = (hipStream_t)stream;
  st = hip_status(hipMemcpyAsync(h->pc, h->hpc, sizeof(h->hpc), hipMemcpyHostToDevice, s));
  if (st == CHEM_DNN_OK)
    st = hip_status(hipMemcpyAsync(h->fc, h->hfc, sizeof(h->hfc), hipMemcpyHostToDevice, s));
  if (st == CHEM_DNN_OK) st = prop_pack(h, params, s);
  // the host copy must not be released before the upload finishes
  if (st == CHEM_DNN_OK && hipStreamSynchronize(s) != hipSuccess) st = CHEM_DNN_EHIP;
  if (st) {
    delete h;
    return st;
  }
  *out = h;
  return CHEM_DNN_OK;
}

int32_t chem_prop_set_params(chem_prop *h, const float *params, void *stream) {
  if (!h || !params) return CHEM_DNN_EINVAL;
  return prop_pack(h, params, (hipStream_t)stream);
}

int32_t chem_prop_eval(chem_prop *h, int64_t n, int64_t ld, const double *x, double *y,
                       void *stream) {
  if (!h || n < 0 || ld < n) return CHEM_DNN_EINVAL;
  if (n == 0) return CHEM_DNN_OK;
  if (!x || !y) return CHEM_DNN_EINVAL;
  const int D = h->widths[0], K = h->widths[h->L];
  {  // x [D][ld] and y [K][ld] must not overlap
    const uintptr_t x0 = (uintptr_t)x, x1 = (uintptr_t)(x + (D - 1) * ld + n);
    const uintptr_t y0 = (uintptr_t)y, y1 = (uintptr_t)(y + (K - 1) * ld + n);
    if (x0 < y1 && y0 < x1) return CHEM_DNN_EINVAL;
  }
  hipStream_t s = (hipStream_t)stream;
  if (h->fused) {
    StepArgs a{};
    a.n = n;
    a.ld = ld;
    a.ntiles = (n + h->lay.MC - 1) / h->lay.MC;
    for (int l = 0; l < 4; ++l) { a.w[l] = h->wpack[l]; a.b[l] = h->bias[l]; }
    a.fc = h->fc;
    a.dc = h->pc;
    a.x = x;
    a.y = y;
    a.D = D;
    a.K = K;
    const int64_t grid = a.ntiles < h->n_cu ? a.ntiles : h->n_cu;
    return hip_status(h->lay.step(a, (int)(grid < 1 ? 1 : grid), s));
  }
  const uint8_t *end = h->ws + h->ws_bytes;
  if ((const uint8_t *)(h->obuf + 32 * h->chunk) > end) return CHEM_DNN_EWORKSPACE;
  hipError_t e = hipSuccess;
  for (int64_t n0 = 0; n0 < n && e == hipSuccess; n0 += h->chunk) {
    const int nc = (int)(n - n0 < h->chunk ? n - n0 : h->chunk);
    const int ncb = (nc + 255) / 256 * 16;     // whole 256-cell tiles
    PropPrepArgs pa{x, ld, n0, nc, ncb, D, h->act[0], h->pc};
    e = launch_prop_prep(h->prec, pa, s);
    int cur = 0;
    for (int l = 0; l < h->L && e == hipSuccess; ++l) {
      LayerArgs la{(const uint8_t *)h->wpack[l], h->bias[l], h->act[cur], h->act[cur ^ 1],
                   h->obuf, h->lR[l], h->lNQ[l], ncb, 16 * ncb, nullptr, 0, 0};
      e = launch_layer(h->prec, la, l < h->L - 1, s);
      cur ^= 1;
    }
    if (e == hipSuccess) {
      PropPostArgs po{y, ld, n0, nc, K, 16 * ncb, h->obuf, h->pc};
      e = launch_prop_post(po, s);
    }
  }
  return hip_status(e);
}

int32_t chem_prop_destroy(chem_prop *h) {
  if (!h) return CHEM_DNN_EINVAL;
  delete h;
  return CHEM_DNN_OK;
}

}  // extern "C"
