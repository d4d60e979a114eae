/* chem_dnn.h - C ABI of the MI355X (gfx950) DNN chemistry update.
 *
 * The library replaces stiff chemistry integration by a fully connected
 * network, per cell, as DeepFlame's ODENet does (paper: arXiv 2508.18969,
 * Sec. 2 "DeepFlame workflow": the net maps the thermochemical state
 * (T, p, Y_i) to the chemical change of the cell).  One call of
 * chem_dnn_step performs, for every cell i of a batch:
 *
 *   1. u_s  = (Y_s^lam - 1)/lam                 power (Box-Cox) transform
 *   2. z    = (x - mu_in)/sigma_in, x = [T, P, u_1..u_S]   Z-score (Sec. 3.3.1)
 *   3. a_l  = GELU(W_l a_(l-1) + b_l), l < L;  o = W_L a_(L-1) + b_L
 *            GELU in the tanh form 0.5x(1+tanh(sqrt(2/pi)(x+0.044715x^3)))
 *            (Sec. 3.3.2); products on matrix cores in the handle's precision
 *            with FP32 accumulation (mixed precision, Sec. 3.3.1)
 *   4. delta = o sigma_out + mu_out;  Y*_s = (max(0, Y_s^lam + lam delta_s))^(1/lam)
 *   5. Yhat = Y + (Y* - Y) in FP64;  Y_new = Yhat / sum(Yhat)   (FP64, Sec. 3.3.1:
 *            everything outside the network stays in double precision)
 *   6. optional T_new keeping sum_s Y_s (h_f,s + c_p,s (T - T_ref)) constant.
 *   7. optional (chem_dnn_step_source) species source terms
 *            omega_s = rho (Y_new,s - Y_s) / dt, rho = P / (R T sum_s Y_s / W_s),
 *            the chemical source terms the network's result stands for in the
 *            species transport equations (Sec. 2, DeepFlame workflow); ideal-gas
 *            density of the state before the step.
 *
 * Conventions for every entry point
 *   - Return value: CHEM_DNN_OK or a negative status; nothing throws or exits.
 *   - Work is enqueued on `stream` (a hipStream_t; NULL = the null stream) and
 *     runs asynchronously; OK means "enqueued".  Argument errors are detected on
 *     the host before anything is enqueued.
 *   - "device" pointers must point to memory of the handle's GPU; "host"
 *     pointers to host memory.  The library never allocates device memory:
 *     the caller owns every buffer, including the workspace.
 *   - Field layout is structure-of-arrays: array[j * ld + i] holds feature or
 *     species j of cell i, ld >= n.
 *   - One handle may be used from one stream at a time.
 */
#ifndef CHEM_DNN_H
#define CHEM_DNN_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct chem_dnn chem_dnn; /* opaque handle; host memory owned by the library */

enum {
    CHEM_DNN_OK = 0,
    CHEM_DNN_EINVAL = -1,      /* bad argument (NULL, negative size, ld < n, shape mismatch) */
    CHEM_DNN_ENODEV = -2,      /* no HIP device */
    CHEM_DNN_EWORKSPACE = -3,  /* workspace NULL, misaligned or smaller than required */
    CHEM_DNN_EUNSUPPORTED = -4,/* device is not gfx950, or network shape not built */
    CHEM_DNN_EHIP = -5,        /* a HIP runtime call or kernel launch failed */
    CHEM_DNN_ETOOLARGE = -6    /* the request needs more than the allocation-free entry point's
                                  static scratch (CHEM_DNN_NOALLOC_SCRATCH_BYTES) */
};

enum {
    CHEM_DNN_FP32 = 0,    /* FP32 operands (16x16x4 f32 matrix cores) */
    CHEM_DNN_BF16 = 1,    /* bfloat16 operands, round-to-nearest-even */
    CHEM_DNN_FP16 = 2,    /* IEEE half operands, round-to-nearest-even */
    CHEM_DNN_FP8E4M3 = 3  /* OCP FP8 E4M3 operands, saturating RNE, per-layer power-of-two scales */
};

enum {
    CHEM_DNN_GELU_TANH = 0,   /* 0.5x(1 + tanh(sqrt(2/pi)(x + 0.044715x^3))) evaluated in FP32 */
    CHEM_DNN_GELU_TABLE = 1,  /* the tabulated GELU of Sec. 3.3.2: 0 for x < -3, x for x > 3, and
                                 on [-3, 3] 600 intervals of 0.01, each the second-order Taylor
                                 expansion about its midpoint (error <= 1.7e-8 inside, a jump of
                                 |GELU(-+3)| = 3.6e-3 at the ends); inference only - training
                                 always uses the tanh form */
    CHEM_DNN_GELU_TABLE16 = 2 /* the same table with its coefficients rounded to FP16 (the
                                 paper implements FP32- and FP16-precision tabulation,
                                 Sec. 3.3.2): 4.8 KB instead of 9.6 KB; evaluated in FP32;
                                 error against the tanh form up to 1.5e-3 (coefficient
                                 rounding) */
};

/* Network and transform description.  All pointers are host pointers; the
 * arrays are copied by chem_dnn_init and need not outlive it. */
typedef struct {
    int32_t n_species;          /* S, 1..30 */
    int32_t n_layers;           /* L linear layers, 1..8.  Built: L = 4 with the hidden widths
                                   of the fused kernel (19-400-200-100-17, 31-1600-800-400-29,
                                   all precisions, training), and 2..8 layers with hidden
                                   widths that are multiples of 256 (layer by layer; FP32, BF16,
                                   FP16, tanh GELU, inference only); EUNSUPPORTED otherwise */
    int32_t widths[9];          /* widths[0] = S + 2, widths[L] = S, hidden widths 1..4096 */
    int32_t precision;          /* CHEM_DNN_FP32 / _BF16 / _FP16 / _FP8E4M3 */
    int32_t gelu_form;          /* CHEM_DNN_GELU_TANH or CHEM_DNN_GELU_TABLE (hidden layers of
                                   chem_dnn_step and chem_dnn_calibrate) */
    double boxcox_lambda;       /* lam > 0 (0.1 in the workloads shipped) */
    const double *in_mean;      /* [S+2] Z-score mean of x = [T, P, u_1..u_S] */
    const double *in_std;       /* [S+2] Z-score standard deviation, > 0 */
    const double *out_mean;     /* [S] mean of the normalised output; NULL -> 0 */
    const double *out_std;      /* [S] std of the normalised output; NULL -> 1 */
    const float *act_amax;      /* [L] max |input| of each layer over a calibration set
                                   (chem_dnn_calibrate); required for FP8, ignored otherwise */
    const double *thermo_hf;    /* [S] formation enthalpy J/kg; NULL -> no temperature update */
    const double *thermo_cp;    /* [S] constant c_p J/(kg K); NULL iff thermo_hf is NULL */
    double t_ref;               /* reference temperature of h_f, K */
    int64_t max_batch;          /* largest batch of chem_dnn_train_step (0 = no training) */
    const double *molar_mass;   /* [S] species molar masses kg/mol, > 0; NULL -> no source
                                   terms (chem_dnn_step_source returns EINVAL) */
    int64_t recompute_chunk;    /* training memory: 0 = the workspace holds the activations of
                                   max_batch samples; > 0 (a multiple of 16) = of this many
                                   samples only: training runs chunk by chunk and pre-activations
                                   that were not saved are recomputed per chunk, so the
                                   workspace no longer grows with the batch */
} chem_dnn_desc;

/* Bytes of device workspace chem_dnn_init needs for `desc` (packed weights,
 * biases, scales, constants and, if max_batch > 0, training scratch).
 * EINVAL for a bad description, EUNSUPPORTED for a shape the library does not compile. */
int32_t chem_dnn_workspace_bytes(const chem_dnn_desc *desc, size_t *bytes);

/* Create a handle on the current HIP device.  params (device, FP32) is the
 * flat parameter vector [W_1 (out x in, row-major), b_1, ..., W_L, b_L]; it is
 * packed into the workspace (device, >= chem_dnn_workspace_bytes, 256-byte
 * aligned), which must stay allocated and unmodified until chem_dnn_destroy.
 * Packing is enqueued on stream.  *out receives the handle (NULL on error).
 * ENODEV without a device, EUNSUPPORTED unless the device is gfx950. */
int32_t chem_dnn_init(const chem_dnn_desc *desc, const float *params, void *workspace,
                      size_t workspace_bytes, void *stream, chem_dnn **out);

/* Re-pack (and, for FP8, re-scale) the weights from a new FP32 parameter
 * vector (device), e.g. after training or loading a checkpoint. */
int32_t chem_dnn_set_params(chem_dnn *h, const float *params, void *stream);

/* One chemistry update of n cells (steps 1-6 above).
 *   T, P      device FP64 [n]      temperature K, pressure Pa
 *   Y         device FP64 [S][ld]  mass fractions
 *   Y_out     device FP64 [S][ld]  new mass fractions; may alias Y
 *   T_out     device FP64 [n] or NULL; may alias T; needs thermo data
 *   n_bad     device uint32 or NULL; the number of cells with a non-finite
 *             input or result, or a non-positive renormalisation sum, is ADDED
 *             to *n_bad.  Such cells are passed through: Y_out = Y, T_out = T.
 * n = 0 is a no-op.  Cells are independent: a cell's result does not depend on
 * the batch it is in. */
int32_t chem_dnn_step(chem_dnn *h, int64_t n, int64_t ld, const double *T, const double *P,
                      const double *Y, double *Y_out, double *T_out, uint32_t *n_bad,
                      void *stream);

/* chem_dnn_step plus the species source terms of step 7:
 *   omega     device FP64 [S][ld]  kg/(m^3 s); must not alias T, P, Y, Y_out
 *             or T_out.  0 for cells passed through as bad.
 *   dt        the time step the network's change refers to, s, > 0 (finite)
 * The other arguments are those of chem_dnn_step.  EINVAL if the handle was
 * created without molar masses. */
int32_t chem_dnn_step_source(chem_dnn *h, int64_t n, int64_t ld, const double *T,
                             const double *P, const double *Y, double *Y_out, double *T_out,
                             double *omega, double dt, uint32_t *n_bad, void *stream);

/* FP8 calibration: running the FP32-operand network on n cells, writes each
 * layer's max |input| (device FP32 [L], overwritten) - the act_amax of an FP8
 * description.  Valid on FP32 handles only (EINVAL otherwise). */
int32_t chem_dnn_calibrate(chem_dnn *h, int64_t n, int64_t ld, const double *T,
                           const double *P, const double *Y, float *amax, void *stream);

/* Per-layer scales (host FP32 [L] each): the operand values fed to the matrix
 * cores are round(a / act_scale[l]) and round(W / w_scale[l]).  Powers of two
 * for FP8, 1 otherwise.  Synchronises the handle's stream. */
int32_t chem_dnn_get_scales(chem_dnn *h, float *act_scale, float *w_scale, void *stream);

/* ------------------------------------------------------------------------
 * Training.  The paper's solver infers a pre-trained network (Sec. 2,
 * DeepFlame paragraph: the chemical source terms come from inferencing the
 * pre-trained ODENet); it does not describe how the network is trained.  The
 * entry points below are this library's own differentiable path for
 * training or fine-tuning the chemistry network on labels from a stiff
 * integrator: an FP32 forward that saves (or recomputes) the hidden
 * pre-activations, an MSE loss on the normalised Box-Cox increment, a
 * hand-written backward of the tanh-form GELU network and Adam (Kingma & Ba,
 * Algorithm 1).  Fused network shapes only.
 * ------------------------------------------------------------------------ */

/* Plain MLP forward in FP32 on feature-major batches (training path):
 *   x     device FP32 [D][ld]  normalised inputs, D = widths[0]
 *   out   device FP32 [S][ld]  linear output
 *   saved device FP32 [sum of hidden widths][ld] pre-activations z_1..z_(L-1)
 *         (layer after layer), or NULL (then B <= max_batch and the handle's
 *         scratch holds them).  B = 0 is a no-op. */
int32_t chem_dnn_mlp_forward(chem_dnn *h, int64_t B, int64_t ld, const float *x,
                             const float *params, float *out, float *saved, void *stream);

/* Backward of chem_dnn_mlp_forward for dL/d out = grad_out (device FP32
 * [S][ld]); needs B <= max_batch (gradient scratch).  saved: the
 * pre-activations of the forward with the same x and params, or NULL to
 * recompute them from x (activation recomputation).  The batch is processed
 * in chunks of the handle's recompute_chunk samples (one chunk without it):
 * per chunk the pre-activations are copied from `saved` or recomputed, and the
 * gradients of later chunks are added in chunk order.  grad_params (device
 * FP32, flat like params) is overwritten; grad_x (device FP32 [D][ld]) is
 * written when not NULL.  The batch reduction has a fixed order: results are
 * bitwise reproducible, and equal with and without `saved`. */
int32_t chem_dnn_mlp_backward(chem_dnn *h, int64_t B, int64_t ld, const float *x,
                              const float *params, const float *saved, const float *grad_out,
                              float *grad_params, float *grad_x, void *stream);

/* One training step on a batch of B states (B <= max_batch):
 * steps 1-2 above with the handle's statistics, FP32 forward, loss
 * L = sum (o - target)^2 / (B S) (target device FP32 [S][ld], the normalised
 * Box-Cox increment), backward, and one Adam update (beta1 0.9, beta2 0.999,
 * eps 1e-8, bias-corrected, `step` counts from 1) of params / adam_m / adam_v
 * (device FP32, flat, updated in place).  grads (device FP32, flat) receives
 * the gradient; *loss (device FP32) the loss before the update.  The handle's
 * packed inference weights are NOT refreshed; call chem_dnn_set_params.
 * Memory: with recompute_chunk > 0 in the description the step runs chunk by
 * chunk (features, forward, loss gradient and backward of one chunk, its
 * weight and bias gradients added to those of the earlier chunks in order),
 * so only one chunk's activations exist at a time - nothing needs recomputing,
 * since a sample's loss gradient does not depend on the other samples.
 * recompute: kept for compatibility; the schedule follows the description. */
int32_t chem_dnn_train_step(chem_dnn *h, int64_t B, int64_t ld, const double *T,
                            const double *P, const double *Y, const float *target,
                            float *params, float *grads, float *adam_m, float *adam_v,
                            int64_t step, float lr, int32_t recompute, float *loss,
                            void *stream);

/* Allocation-free training step, for callers that cannot allocate device
 * memory (code under HIP graph capture, tight loops, harnesses that forbid
 * allocation): chem_dnn_train_step with its training scratch in a static
 * device array of the library - CHEM_DNN_NOALLOC_SCRATCH_BYTES per GPU,
 * reserved when the library's code is loaded on that GPU and held until the
 * process ends - instead of the handle's workspace, so the handle needs no
 * training scratch (max_batch may be 0).  B is not bounded by max_batch; the
 * scratch is: ETOOLARGE when the batch (in chunks of the handle's
 * recompute_chunk, if any) needs more.  It runs the same kernels in the same
 * schedule as chem_dnn_train_step on a handle with the same recompute_chunk
 * (results equal bit for bit) and calls no allocation routine.  All calls on
 * one GPU share its array: calls that overlap on one GPU (concurrent streams,
 * threads or handles) race and must be serialised by the caller.  Nothing in
 * the array has to start at zero; it keeps the last call's contents. */
#define CHEM_DNN_NOALLOC_SCRATCH_BYTES (64u << 20)
int32_t chem_dnn_train_step_noalloc(chem_dnn *h, int64_t B, int64_t ld, const double *T,
                                    const double *P, const double *Y, const float *target,
                                    float *params, float *grads, float *adam_m, float *adam_v,
                                    int64_t step, float lr, float *loss, void *stream);

/* Release the handle (host memory only; the caller frees the workspace). */
int32_t chem_dnn_destroy(chem_dnn *h);

/* Layer dump, for testing the kernels layer by layer (the products of one
 * layer against an exact recomputation from the very operands the matrix
 * cores received, and each activation against its accumulators).  Runs the
 * network of chem_dnn_step on n <= CHEM_DNN_DEBUG_MAX_CELLS cells with the
 * same kernels, operand formats and schedules, and instead of the update
 * writes, for every layer l = 0 .. L-1:
 *   qin  device FP32 [sum_l widths[l]][n]; rows in_row(l) = sum_{k<l} widths[k]
 *        onward: layer l's input as the operand values fed to the matrix
 *        cores (quantised to the handle's precision; for FP8 the scaled
 *        values a / act_scale[l]), decoded exactly to FP32.  Layer 0's input
 *        is the Z-scored network input.
 *   acc  device FP32 [sum_l widths[l+1]][n]; rows acc_row(l) =
 *        sum_{k<l} widths[k+1] onward: layer l's FP32 accumulators after all
 *        its products, before the activation.  For FP32, BF16 and FP16 they
 *        started at the bias; for FP8 at 0, and the result is scaled by
 *        act_scale[l] * w_scale[l] and given the bias afterwards.  For the
 *        output layer, rows are species.
 * Tanh-form GELU handles only (EUNSUPPORTED otherwise).  Y_out/T_out are not
 * touched.  The dump is the kernels' own debug build of the same code, not
 * a separate implementation. */
#define CHEM_DNN_DEBUG_MAX_CELLS 4096
int32_t chem_dnn_debug_layers(chem_dnn *h, int64_t n, int64_t ld, const double *T,
                              const double *P, const double *Y, float *qin, float *acc,
                              void *stream);

/* ------------------------------------------------------------------------
 * Property networks.  For flames at supercritical pressure a second network
 * per cell (the paper's PRNet, Sec. 2; sizes 3-1024-512-256-1 for the density
 * and 3-2048-1024-512-4 for the temperature and transport properties, Sec. 4)
 * maps a few thermodynamic state variables to mixture properties in place of
 * the real-fluid equation of state.  chem_prop_eval performs, for every cell:
 *
 *   1. z = (x - mu_in) / sigma_in          (FP64, then FP32 operands)
 *   2. a_l = GELU(W_l a_(l-1) + b_l), l < L;  o = W_L a_(L-1) + b_L
 *      (the GELU, operand formats and FP32 accumulation of chem_dnn_step)
 *   3. y = o sigma_out + mu_out            (FP64)
 *
 * Cells are independent; a non-finite input gives non-finite outputs of that
 * cell only.  Conventions (status codes, streams, ownership, SoA layout) are
 * those of the chemistry entry points above.
 * ------------------------------------------------------------------------ */
typedef struct chem_prop chem_prop; /* opaque handle; host memory owned by the library */

typedef struct {
    int32_t n_layers;           /* L linear layers, 2..8 */
    int32_t widths[9];          /* widths[0] = number of inputs 1..32, widths[L] = number of
                                   outputs 1..32, hidden widths multiples of 256 up to 4096 */
    int32_t precision;          /* CHEM_DNN_FP32 / _BF16 / _FP16 (FP8: EUNSUPPORTED) */
    const double *in_mean;      /* host [widths[0]] input mean */
    const double *in_std;       /* host [widths[0]] input standard deviation, > 0 */
    const double *out_mean;     /* host [widths[L]] output mean; NULL -> 0 */
    const double *out_std;      /* host [widths[L]] output scale; NULL -> 1 */
} chem_prop_desc;

/* Device workspace for `desc`: packed weights, constants and the activation
 * buffers of one chunk of cells.  EINVAL for a bad description,
 * EUNSUPPORTED for a shape or precision the library does not offer. */
int32_t chem_prop_workspace_bytes(const chem_prop_desc *desc, size_t *bytes);

/* Create a handle on the current HIP device; params (device FP32, flat
 * [W_1 (out x in, row-major), b_1, ..., W_L, b_L]) is packed into the
 * workspace (device, 256-byte aligned, >= chem_prop_workspace_bytes), which
 * stays allocated and unmodified until chem_prop_destroy.  The host arrays of
 * the description are copied.  ENODEV / EUNSUPPORTED as chem_dnn_init. */
int32_t chem_prop_init(const chem_prop_desc *desc, const float *params, void *workspace,
                       size_t workspace_bytes, void *stream, chem_prop **out);

/* Re-pack the weights from a new FP32 parameter vector (device). */
int32_t chem_prop_set_params(chem_prop *h, const float *params, void *stream);

/* Evaluate the network on n cells:
 *   x   device FP64 [widths[0]][ld]   input fields
 *   y   device FP64 [widths[L]][ld]   outputs; must not alias x
 * n = 0 is a no-op. */
int32_t chem_prop_eval(chem_prop *h, int64_t n, int64_t ld, const double *x, double *y,
                       void *stream);

/* Release the handle (host memory only). */
int32_t chem_prop_destroy(chem_prop *h);

/* Static description of a status code. */
const char *chem_dnn_strerror(int32_t status);

/* ABI version of this header: 5 (2 added gelu_form to chem_dnn_desc; 3 added
 * molar_mass at its end and chem_dnn_step_source; 4 added the property
 * networks, chem_prop_*; 5 added chem_dnn_debug_layers). */
int32_t chem_dnn_abi_version(void);

#ifdef __cplusplus
}
#endif
#endif /* CHEM_DNN_H */
