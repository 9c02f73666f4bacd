/*
 * halftone.h -- C ABI of libhalftone, the MI355X (gfx950) implementation of
 * the halftoning method of "Efficient Halftoning via Deep Reinforcement
 * Learning" (Jiang et al., IEEE TIP; arXiv 2304.12152).
 *
 * General conventions (every entry point):
 *   - Returns HS_OK (0) or a negative HS_E* code; halftone_last_error()
 *     returns a thread-local message for the last failure of the calling
 *     thread. No exception crosses the ABI.
 *   - Every pointer argument is DEVICE memory unless its name ends in _host.
 *     The caller owns all memory: inputs, outputs and the workspace whose
 *     size comes from the matching *_workspace_size call. The library never
 *     allocates device memory.
 *   - `stream` is a hipStream_t passed as void*. All device work is enqueued
 *     asynchronously on it; no call synchronises the host unless noted.
 *   - Images are dense row-major [B][H][W]; contone values are float in
 *     [0, 1] with 1 = white. Halftone bits are uint8 0/1 with 1 = white.
 *     Within image b pixel a = y*W + x.
 *   - Policy weights are FP32, one flat array of HS_PARAM_COUNT floats:
 *     layer after layer, W[cout][cin][3][3] then bias[cout]; layers are
 *     2->32, four 32->32, 32->1 (3x3, stride 1, zero 'same' padding, ReLU
 *     after all but the last).
 *   - Random draws are Philox4x32-10 keyed by (seed of the image) with
 *     counter (a_lo, a_hi, stream, step): stream 0 = Bernoulli actions,
 *     stream 1 = noise map z. u = (w0 >> 8) * 2^-24; Gaussian z by
 *     Box-Muller on (w0, w1).
 *   - On error, outputs are unspecified but nothing is written out of bounds;
 *     argument errors are detected before any launch.
 */
#ifndef HALFTONE_H
#define HALFTONE_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define HS_OK 0
#define HS_EINVAL (-1)       /* null pointer, bad enum, bad parameter      */
#define HS_ESHAPE (-2)       /* bad B/H/W (non-positive, or too small)     */
#define HS_EUNSUPPORTED (-3) /* precision or device not supported          */
#define HS_EWORKSPACE (-4)   /* workspace smaller than *_workspace_size    */
#define HS_EHIP (-5)         /* a HIP call or kernel launch failed          */
#define HS_ENONFINITE (-6)   /* an input holds NaN or +-inf (checked only
                                when HS_CHECK_FINITE is requested)        */

/* Optional input check, OR-ed into the `noise_kind` argument of the
 * inference calls, into hs_loss_params.flags, or into the flags of
 * halftone_policy_pack: before any other launch the call counts the NaN and
 * infinite values of its floating-point inputs on the device, waits for the
 * count (so the call synchronises its stream) and returns HS_ENONFINITE if
 * there is one. Without it non-finite inputs give unspecified outputs, but
 * nothing is written out of bounds. */
#define HS_CHECK_FINITE 0x100

#define HS_FP32 0 /* FP32 arithmetic throughout                           */
#define HS_BF16 1 /* BF16 MFMA with FP32 accumulation                      */
#define HS_FP16 2 /* FP16 MFMA with FP32 accumulation (inference only)     */
#define HS_FP8 3  /* FP8 (E4M3) MFMA for the 32->32 layers, FP32
                     accumulation (packed policies with FP8 scales only)   */

#define HS_NOISE_GAUSS 0   /* z ~ N(0,1) (Sec. III, "State")               */
#define HS_NOISE_UNIFORM 1 /* z ~ U(0,1), the variant of Sec. VI-D         */

#define HS_WRT_PROB 0  /* gradients with respect to pi_a(h=1)              */
#define HS_WRT_LOGIT 1 /* gradients with respect to the logit x_a          */

#define HS_EST_LE 0   /* Local Expectation estimator (Sec. III-B, Eq. le)    */
#define HS_EST_COMA 1 /* REINFORCE with the COMA baseline (Sec. III-A,
                         Eqs. baseline and coma)                            */

#define HS_PARAM_COUNT 37889
#define HS_MAX_LEVELS 8 /* most output levels of the multitoning variant  */

/* Parameters of the reward and of the anisotropy-suppressing loss.
 * Defaults (halftone_default_loss_params): w_s = 0.06 and w_a = 0.002
 * (Sec. VI-A), HVS = 11x11 Gaussian sigma 2 (stand-in for the Nasanen
 * filter of Sec. V), SSIM window 11x11 Gaussian sigma 1.5 and k = 2
 * (Sec. V, contrast map), C1 = 1e-4, C2 = 9e-4 (SSIM constants of Wang et
 * al. 2004 for L = 1), anisotropy patches of 32x32, the Local Expectation
 * estimator, 2 output levels (binary halftoning).
 *
 * levels > 2 selects the multitoning prototype of Sec. VI-E (its
 * unnumbered rounding equation): the network keeps its one sigmoid output v, the L levels are
 * k / (L-1), and agent a's two actions are the levels k_f and k_f + 1 around
 * v_a (k_f = min(floor(v_a (L-1)), L-2)), the upper one drawn with
 * probability v_a (L-1) - k_f. Actions are then level indices k (one byte,
 * image value k / (L-1)); only the Local Expectation estimator is
 * supported (HS_EUNSUPPORTED otherwise). */
typedef struct hs_loss_params {
  float w_s;
  float w_a;
  float hvs_sigma;
  int hvs_radius;  /* 1..7 */
  float ssim_sigma;
  int ssim_radius; /* 1..7 */
  float k;
  float c1;
  float c2;
  int as_patch;  /* only 32 is supported */
  int estimator; /* HS_EST_LE or HS_EST_COMA */
  int levels;    /* 2 (binary) .. HS_MAX_LEVELS (multitoning) */
  int flags;     /* 0 or HS_CHECK_FINITE (contone and probabilities) */
} hs_loss_params;

/* Optimiser and sampling parameters of one TRAIN iteration (Algorithm 1).
 * Defaults: Adam beta1 0.9, beta2 0.999, eps 1e-8; cosine learning rate
 * from lr_max 3e-4 to lr_min 1e-5 over total_steps (Sec. VI-A); all
 * activations kept for the backward (recompute = 0).
 *
 * recompute = 1 keeps two activation maps instead of five: the backward
 * rebuilds the input of each 32->32 layer by re-running layers 1..k-1 on the
 * same input and noise (the same kernels, so the same values and the same
 * gradient), for large crops. It costs ten more layer launches per batch
 * and saves three NHWC activation maps (3 x 64 B per pixel in BF16). */
typedef struct hs_train_params {
  hs_loss_params loss;
  float lr_max;
  float lr_min;
  float beta1;
  float beta2;
  float eps;
  int noise_kind; /* HS_NOISE_* */
  int recompute;  /* 0: keep activations; 1: recompute them in the backward */
} hs_train_params;

void halftone_default_loss_params(hs_loss_params* p);
void halftone_default_train_params(hs_train_params* p);
int halftone_version(void);
const char* halftone_last_error(void);
int64_t halftone_param_count(void);

/* ---------------------------------------------------------------------
 * Inference: the TEST procedure of Algorithm 1 (Sec. IV). z is drawn from
 * Philox (stream 1, step 0) for image b keyed by seeds[b]; the policy
 * network gives the logit x_a; bit_a = [x_a >= 0] (threshold of
 * pi_a(h=1) at 0.5; a tie is white).
 *
 * weights  [HS_PARAM_COUNT] FP32.
 * contone  [B][H][W] FP32.
 * seeds    [B] uint64.
 * precision HS_FP32: FP32 arithmetic. HS_BF16: BF16 MFMA with FP32
 *          accumulation; every pixel whose BF16 logit satisfies
 *          |x| < recheck_tau is recomputed over its 13x13 receptive field
 *          with split-BF16 products (hi*hi + lo*hi + hi*lo, FP32
 *          accumulation, about 2^-8 of the BF16 error), and every pixel
 *          whose split |x| is still below tau2 = max(recheck_tau/64,
 *          1.5e-4) once more in FP32, decided from that value (when tau2
 *          <= 2e-4 there is no FP32 stage: such a pixel's exact logit is
 *          within 2 tau2 <= 4e-4 of the threshold, inside the margin
 *          |p - 1/2| <= 1e-4 where either bit is the oracle's, and the
 *          split stage decides it from its own logit)
 *          (recheck_tau >= 0; it must exceed the largest BF16 logit error
 *          for the bits to equal FP32's off-margin, and tau2 the split
 *          stage's). halftone_policy_infer takes tau2 explicitly and can
 *          put an FP16 cone stage (FP16 products, about 1/8 of the BF16
 *          error) with its own band tau16 in front of the split stage.
 *          The BF16 error
 *          depends on the weights (0.042 for a He-initialised policy, 4.5
 *          for a trained one on the same images): measure it by comparing
 *          the logits of a call with recheck_tau = 0 against HS_FP32's.
 *          HS_FP16: the same with FP16 in place of BF16 in the fused pass,
 *          so recheck_tau can be about 8 times smaller (and there is no
 *          FP16 cone stage); FP16 holds at most 65504, and if any
 *          activation of the pass overflows, the pass is run again in BF16
 *          with 8 * recheck_tau, decided on the device (no host
 *          synchronisation), and stats[3] reads 1.
 * noise_kind HS_NOISE_GAUSS or HS_NOISE_UNIFORM, optionally OR-ed with
 *          HS_CHECK_FINITE (the contone is then checked first).
 * bits     [B][H][W] uint8 out.
 * logits_or_null [B][H][W] FP32 out: the logit each bit was decided from.
 * stats_or_null  int32[8] out: {pixels rechecked (|x_bf16| < recheck_tau),
 *          bits changed by the rechecks, pixels recomputed in FP32,
 *          1 if an HS_FP16 pass overflowed and was run again in BF16,
 *          pixels recomputed by the split stage, 0, 0, 0}; zeros for
 *          HS_FP32.
 * Shapes: B >= 1, H >= 1, W >= 1, B*H*W < 2^31.
 * --------------------------------------------------------------------- */
size_t halftone_infer_workspace_size(int B, int H, int W, int precision);
int halftone_infer(const float* weights, const float* contone, const uint64_t* seeds, int B,
                   int H, int W, int noise_kind, int precision, float recheck_tau, uint8_t* bits,
                   float* logits_or_null, int32_t* stats_or_null, void* workspace,
                   size_t workspace_bytes, void* stream);

/* ---------------------------------------------------------------------
 * halftone_infer for callers that cannot allocate device memory (code
 * under HIP graph capture, tight serving loops, harnesses that forbid
 * allocation): the same call without the workspace argument. Its
 * workspace is a static device array of HS_NOALLOC_SCRATCH_BYTES (64 MiB)
 * that the library holds on each GPU it runs on until the process ends;
 * the call allocates nothing and, without HS_CHECK_FINITE, does not
 * synchronise.
 *
 * Arguments, results and errors as for halftone_infer, plus HS_EWORKSPACE
 * when halftone_infer_workspace_size(B, H, W, precision) exceeds the
 * scratch: about 3.6 Mpx for HS_BF16 and HS_FP16 (e.g. 3 x 1024 x 1024),
 * about 250 kpx for HS_FP32 (256 B per pixel). Every call on one GPU uses
 * that GPU's one array (its counters are cleared by each call), so calls
 * that overlap on one GPU -- on different streams or from different host
 * threads -- race and must be serialised by the caller.
 * --------------------------------------------------------------------- */
#define HS_NOALLOC_SCRATCH_BYTES (64u << 20)
int halftone_infer_noalloc(const float* weights, const float* contone, const uint64_t* seeds,
                           int B, int H, int W, int noise_kind, int precision, float recheck_tau,
                           uint8_t* bits, float* logits_or_null, int32_t* stats_or_null,
                           void* stream);

/* ---------------------------------------------------------------------
 * Inference over pages of different sizes (the TEST procedure of
 * Algorithm 1 on an uneven batch), with HS_BF16 or HS_FP16 in ONE persistent launch
 * of the fused kernel whose workgroups split all pages' strips evenly,
 * followed by the same two recheck stages as halftone_infer; with HS_FP32
 * page by page.
 *
 * shapes_host [npages][2] int32 in HOST memory: (H, W) of each page; read
 *          during the call only.
 * contone  FP32, the pages concatenated: page p at offset
 *          sum_{q < p} H_q W_q, row-major within the page.
 * seeds    [npages] uint64: page p's noise map is keyed by seeds[p]
 *          (pixel a = y W_p + x within the page).
 * bits, logits_or_null: the same concatenated layout; stats_or_null as for
 *          halftone_infer. Every page at least 1 x 1; total < 2^31 pixels.
 * --------------------------------------------------------------------- */
size_t halftone_infer_pages_workspace_size(int npages, const int32_t* shapes_host,
                                           int precision);
int halftone_infer_pages(const float* weights, const float* contone, const uint64_t* seeds,
                         int npages, const int32_t* shapes_host, int noise_kind, int precision,
                         float recheck_tau, uint8_t* bits, float* logits_or_null,
                         int32_t* stats_or_null, void* workspace, size_t workspace_bytes,
                         void* stream);

/* ---------------------------------------------------------------------
 * Multitoning inference (Sec. VI-E, the TEST phase with L output levels):
 * the level nearest to v = sigmoid(x), a tie going up, i.e. the number of
 * thresholds logit((j + 1/2)/(L-1)), j = 0..L-2, that the logit x reaches
 * (levels = 2 is halftone_infer_pages exactly). Arguments as for
 * halftone_infer_pages, with
 * levels   2..HS_MAX_LEVELS (HS_EINVAL otherwise);
 * levels_out the level index k in 0..L-1 per pixel (image value k/(L-1)).
 * With HS_BF16 or HS_FP16 the recheck band is |x - nearest threshold| < recheck_tau
 * (the split stage: < tau2), so every level equals the FP32 one wherever v
 * is farther than the BF16 error from the midpoints; stats as for
 * halftone_infer ("bits changed" counts changed levels). Workspace from
 * halftone_infer_pages_workspace_size.
 * --------------------------------------------------------------------- */
int halftone_infer_levels(const float* weights, const float* contone, const uint64_t* seeds,
                          int npages, const int32_t* shapes_host, int levels, int noise_kind,
                          int precision, float recheck_tau, uint8_t* levels_out,
                          float* logits_or_null, int32_t* stats_or_null, void* workspace,
                          size_t workspace_bytes, void* stream);

/* ---------------------------------------------------------------------
 * A packed inference policy (the network of the TEST procedure, Algorithm
 * 1): a copy of the FP32 weights together with every derived copy the
 * inference calls use -- the BF16 and FP16 MFMA fragments of the fused
 * pass, its FP16 layer bounds, the split hi/lo BF16 and transposed FP32
 * copies of the recheck stages, and the FP32 per-layer fragments -- made
 * once per weight update instead of on every call.
 *
 * halftone_policy_bytes: device memory one packed policy needs.
 * halftone_policy_pack: packs `weights` (device FP32 [HS_PARAM_COUNT])
 *          into `mem` (device memory of at least halftone_policy_bytes(),
 *          256-byte aligned, owned by the caller and left untouched by it
 *          while the policy is used) and fills the host struct *policy.
 *          The copy is taken on `stream`: later changes to `weights` do
 *          not affect the policy until it is packed again. flags: 0 or
 *          HS_CHECK_FINITE (then the weights are checked and the call
 *          waits for the stream).
 * halftone_policy_infer: halftone_infer_levels (levels = 2: the bits of
 *          halftone_infer_pages) with the policy's packed copies, so the
 *          call launches no packing kernel. Arguments and results as for
 *          halftone_infer_levels, plus the bands of the cone stages, each
 *          >= 0 or -1 for the default rule of halftone_infer:
 *          recheck_tau16 the FP16 stage's after an HS_BF16 pass (pixels
 *          whose FP16 |x| is below it go on to the split stage; it must
 *          exceed the FP16 stage's largest logit error for the weights; 0
 *          skips the stage) and recheck_tau2 the split stage's (pixels
 *          below it go to the FP32 stage; it must exceed the split
 *          stage's largest error). A large recheck_tau with
 *          recheck_tau16 = 0 and recheck_tau2 = 0 returns the split
 *          stage's logits for every pixel, and with recheck_tau2 = 0 and a
 *          huge recheck_tau16 all pass the FP16 stage undecided: that is
 *          how the errors are measured. Workspace from
 *          halftone_infer_pages_workspace_size. Calls on the same policy
 *          may overlap (the policy is only read); the work must be
 *          enqueued after the pack on a stream ordered after `stream`.
 * --------------------------------------------------------------------- */
typedef struct hs_policy {
  void* mem;    /* the caller's device memory holding the packed copies */
  size_t bytes; /* its size */
  int packed;   /* 1 once halftone_policy_pack has succeeded */
  int fp8;      /* 1 once halftone_policy_set_fp8 has succeeded (a new
                   pack clears it) */
} hs_policy;
size_t halftone_policy_bytes(void);
int halftone_policy_pack(hs_policy* policy, const float* weights, void* mem, size_t bytes,
                         int flags, void* stream);
int halftone_policy_infer(const hs_policy* policy, const float* contone, const uint64_t* seeds,
                          int npages, const int32_t* shapes_host, int levels, int noise_kind,
                          int precision, float recheck_tau, float recheck_tau16,
                          float recheck_tau2, uint8_t* out, float* logits_or_null,
                          int32_t* stats_or_null, void* workspace, size_t workspace_bytes,
                          void* stream);

/* ---------------------------------------------------------------------
 * The FP8 pass of a packed policy: the TEST procedure of Algorithm 1 with
 * the four 32->32 convolutions of the policy network (Sec. VI-A; 97.7% of
 * its multiply-adds) on the FP8 E4M3 matrix cores. The paper reports FP32
 * runtimes only (Sec. VI-C); this precision is the library's own, and the
 * recheck stages keep the bits those of FP32 off the margin.
 *
 * halftone_layer_max: the FP32 forward of `weights` (noise and shapes as
 *          in halftone_infer with HS_FP32); layer_max [5] FP32 DEVICE out:
 *          the largest activation (after the ReLU) of layers 1..5 over the
 *          batch. Workspace halftone_infer_workspace_size(B, H, W,
 *          HS_FP32). For calibration on images other than those to be
 *          halftoned.
 * halftone_policy_set_fp8: the FP8 copy of a packed policy from
 *          act_max_host [4] (HOST FP32, finite, >= 0): calibrated maxima
 *          of layers 1..4's activations. Layer k's activations are stored
 *          as E4M3 codes of a / s_k, s_k the smallest power of two with
 *          4 act_max[k] <= 448 s_k; each output channel of layers 2..5 has
 *          its own power-of-two weight scale (largest |w| at most 448
 *          times it). Layers 1 and 6 stay BF16. Enqueued on `stream`;
 *          packing the policy again clears it. Errors: HS_EINVAL (policy
 *          not packed, a bad maximum).
 * halftone_policy_infer with precision HS_FP8: the fused pass in FP8, then
 *          the split and FP32 stages as after HS_FP16 (recheck_tau16 is
 *          ignored). recheck_tau must exceed the FP8 pass's largest logit
 *          error, measured like the BF16 one. If an activation exceeds 448
 *          s_k (saturation), the pass is run again in BF16 with
 *          recheck_tau / 8, decided on the device, and stats[3] reads 1.
 * --------------------------------------------------------------------- */
int halftone_layer_max(const float* weights, const float* contone, const uint64_t* seeds, int B,
                       int H, int W, int noise_kind, float* layer_max, void* workspace,
                       size_t workspace_bytes, void* stream);
int halftone_policy_set_fp8(hs_policy* policy, const float* act_max_host, void* stream);

/* ---------------------------------------------------------------------
 * Training-mode policy forward and its backward (the conv stack of
 * Sec. VI-A with its chain rule), for torch.autograd wrappers.
 *
 * halftone_policy_forward: z from Philox (stream 1, `step`);
 *   probs [B][H][W] FP32 out = sigmoid(logit). Keeps every layer's
 *   activations in `workspace` for the backward.
 * halftone_policy_backward: grad_probs [B][H][W] FP32 in (dLoss/dprobs),
 *   probs as returned by the forward; grad_weights [HS_PARAM_COUNT] FP32
 *   out (overwritten). `workspace` must be the one given to the matching
 *   forward, with the same weights and shapes, untouched in between.
 * --------------------------------------------------------------------- */
size_t halftone_policy_workspace_size(int B, int H, int W, int precision);
int halftone_policy_forward(const float* weights, const float* contone, const uint64_t* seeds,
                            int B, int H, int W, int noise_kind, uint32_t step, int precision,
                            float* probs, void* workspace, size_t workspace_bytes, void* stream);
int halftone_policy_backward(const float* weights, const float* grad_probs, const float* probs,
                             int B, int H, int W, int precision, float* grad_weights,
                             void* workspace, size_t workspace_bytes, void* stream);

/* ---------------------------------------------------------------------
 * Reward and anisotropy loss (Sec. III "Rewards", Eq. final_reward;
 * Sec. V Eq. cssim; Sec. IV Eq. as with the probability proxy).
 *
 * actions  [B][H][W] uint8 (the sampled halftone h; level indices when
 *          prm->levels > 2, image value k / (levels - 1)).
 * contone  [B][H][W] FP32.
 * probs_gray_or_null [Bg][Hg][Wg] FP32: pi(h=1) of the constant-gray side
 *          batch; L_AS is computed over its non-overlapping 32x32 patches
 *          (remainders dropped). Pass NULL (and Bg = 0) to skip L_AS.
 * out      FP32, 3*B + 2 values: per image {MSE(HVS(h), HVS(c)), mean
 *          CSSIM, R = -MSE + w_s*CSSIM}, then L_AS (mean over patches; 0 if
 *          no patch), then the total training loss of the batch,
 *          -mean_b R_b + w_a * L_AS (the value whose gradient the
 *          estimators of halftone_loss_backward stand in for, Sec. III-B
 *          and Sec. IV). MSE and CSSIM are means over the valid region
 *          [m, H-m) x [m, W-m), m = max(hvs_radius, ssim_radius).
 * Shapes: H, W >= 2m+1.
 * --------------------------------------------------------------------- */
size_t halftone_loss_workspace_size(int B, int H, int W, int Bg, int Hg, int Wg,
                                    const hs_loss_params* prm);
int halftone_loss(const uint8_t* actions, const float* contone, int B, int H, int W,
                  const float* probs_gray_or_null, int Bg, int Hg, int Wg,
                  const hs_loss_params* prm, float* out, void* workspace, size_t workspace_bytes,
                  void* stream);

/* ---------------------------------------------------------------------
 * Gradients of the training loss (Eq. marl with the Local Expectation
 * estimator of Sec. III-B, computed locally as in Sec. III-C; Eq. as).
 *
 * grad_probs [B][H][W] FP32 out: dL_MARL/dp_a = -dR_a / B where
 *          dR_a = R(h_a = 1, h_-a) - R(h_a = 0, h_-a) (prm->estimator =
 *          HS_EST_LE). With HS_EST_COMA: the one-sample COMA estimate
 *          -(d/dp_a log pi_a(h_a)) (R(h) - b_a) / B, b_a = p_a R(h_a = 1,
 *          h_-a) + (1 - p_a) R(h_a = 0, h_-a), i.e. -dR_a (1-p_a)/p_a / B
 *          where h_a = 1 and -dR_a p_a/(1-p_a) / B where h_a = 0; it needs
 *          probs_or_null in both gradient spaces.
 *          With prm->levels = L > 2 (multitoning): dL_MARL/dv_a =
 *          -dR_a (L-1) / B, dR_a = R(h_a = level k_f + 1) - R(h_a = level
 *          k_f) with k_f from v_a = probs_or_null (required); each h_a must
 *          be one of its two levels (the sampled actions are).
 * grad_probs_gray_or_null [Bg][Hg][Wg] FP32 out: w_a * dL_AS/dp_g (zero
 *          outside the patches).
 * grad_space HS_WRT_PROB, or HS_WRT_LOGIT to multiply both by p(1 - p)
 *          (for COMA: -dR_a (1-p_a)^2 / B where h_a = 1, -dR_a p_a^2 / B
 *          where h_a = 0);
 *          HS_WRT_LOGIT needs probs_or_null (for the main batch) and uses
 *          probs_gray_or_null for the gray batch.
 * --------------------------------------------------------------------- */
int halftone_loss_backward(const uint8_t* actions, const float* contone,
                           const float* probs_or_null, int B, int H, int W,
                           const float* probs_gray_or_null, int Bg, int Hg, int Wg,
                           const hs_loss_params* prm, int grad_space, float* grad_probs,
                           float* grad_probs_gray_or_null, void* workspace,
                           size_t workspace_bytes, void* stream);

/* ---------------------------------------------------------------------
 * One TRAIN iteration of Algorithm 1 on one GPU:
 *   forward of the batch (z from stream 1 at `step`), p = sigmoid(x),
 *   actions h_a = [u_a < p_a] (stream 0 at `step`; with tp->loss.levels
 *   = L > 2 the level index k_f + [u_a < p_a (L-1) - k_f]), dL_MARL/dp from the
 *   estimator tp->loss.estimator (Local Expectation or COMA); forward of the constant-gray side batch,
 *   w_a * dL_AS/dp_g; backward of both through the conv stack; Adam on the
 *   FP32 master weights with lr_t = lr_min + (lr_max - lr_min)(1 +
 *   cos(pi step / total_steps))/2 and bias corrections at t = step + 1.
 *
 * weights, adam_m, adam_v [HS_PARAM_COUNT] FP32, updated in place.
 * contones [B][H][W], seeds [B]; gray [Bg][Hg][Wg], gray_seeds [Bg]
 *          (Bg = 0 and NULLs to skip the anisotropy term).
 * precision HS_FP32 or HS_BF16 (BF16 activations and MFMA, FP32 master
 *          weights, FP32 gradients accumulated in FP32).
 * metrics  FP32[8] out: mean MSE, mean CSSIM, mean R, L_AS, lr, |grad|_2,
 *          fill (the mean of h: the fraction of ones for binary actions),
 *          the total loss -mean R + w_a L_AS.
 * tp->loss.flags & HS_CHECK_FINITE checks the contones (and gray levels).
 * actions_out_or_null [B][H][W] uint8: the sampled actions.
 * grad_out_or_null [HS_PARAM_COUNT] FP32: the total gradient before Adam.
 * Streams: with Bg > 0 the side batch runs on a second stream that the
 *          library owns per device (default priority), forked from
 *          `stream` after the step's weight packing and joined back into
 *          it before the gradient is summed, so every output is ordered on
 *          `stream`; calls on one device take turns on that second stream.
 * --------------------------------------------------------------------- */
size_t halftone_train_workspace_size(int B, int H, int W, int Bg, int Hg, int Wg,
                                     int precision);
/* the same for the given parameters (smaller with tp->recompute = 1; a NULL
 * tp is the defaults) */
size_t halftone_train_workspace_size_params(int B, int H, int W, int Bg, int Hg, int Wg,
                                            int precision, const hs_train_params* tp);
int policy_train_step(float* weights, float* adam_m, float* adam_v, const float* contones,
                      const uint64_t* seeds, int B, int H, int W, const float* gray,
                      const uint64_t* gray_seeds, int Bg, int Hg, int Wg, int64_t step,
                      int64_t total_steps, const hs_train_params* tp, int precision,
                      float* metrics, uint8_t* actions_out_or_null, float* grad_out_or_null,
                      void* workspace, size_t workspace_bytes, void* stream);

/* ---------------------------------------------------------------------
 * Timing of the dominant kernel, for benchmarks. Between
 * halftone_profile_start() and halftone_profile_stop(), every
 * halftone_infer call records a pair of hipEvents on its stream around its
 * dominant kernel (the fused BF16 kernel; for HS_FP32 the four 32->32
 * convolution launches taken together), at most 4096 pairs.
 * halftone_profile_stop waits for the recorded events and returns their
 * summed duration (ms) and the number of recorded calls (host pointers).
 * --------------------------------------------------------------------- */
int halftone_profile_start(void);
int halftone_profile_stop(double* ms_total_host, int* launches_host);

/* ---------------------------------------------------------------------
 * Blue-noise evaluation (Sec. IV, Eqs. psd, rapsd, anis): the power spectrum
 * of a batch of halftones estimated as the mean of the periodograms
 * |DFT|^2 / P^2 (no mean removal) of all non-overlapping P x P patches of the
 * B images, tiled from (0, 0) with the remainders dropped; then per ring rho
 * (frequency (u, v) folded to ub = min(u, P-u), vb = min(v, P-v), rho the
 * unique integer with (2rho-1)^2 <= 4(ub^2+vb^2) < (2rho+1)^2, the DC term is
 * ring 0) the radially averaged power RAPSD[rho] (mean over the ring) and
 * the anisotropy anis[rho] = sum (P(f) - RAPSD)^2 / ((n-1) RAPSD^2), 0 for
 * rings with one frequency or zero power.
 *   bits [B][H][W] uint8 in device memory, each 0 or 1 (any byte value is
 *        taken as its number);
 *   P    32 or 64 (HS_EUNSUPPORTED otherwise); H >= P and W >= P
 *        (HS_ESHAPE otherwise);
 *   rapsd_out, anis_out: device FP32 arrays of halftone_spectrum_rings(P)
 *        entries (24 for P = 32, 46 for P = 64).
 * Rings are in linear power; the caller takes 10 log10 for dB. The mean over
 * patches runs in a fixed order, so results are deterministic. Workspace
 * from halftone_spectrum_workspace_size (0 for invalid shapes).
 * --------------------------------------------------------------------- */
int halftone_spectrum_rings(int P);
size_t halftone_spectrum_workspace_size(int B, int H, int W, int P);
int halftone_spectrum(const uint8_t* bits, int B, int H, int W, int P, float* rapsd_out,
                      float* anis_out, void* workspace, size_t workspace_bytes, void* stream);

/* ---------------------------------------------------------------------
 * Floyd-Steinberg error diffusion on the host (the classic error diffusion
 * cited in Sec. I): the halftoner a trained policy is judged against, and
 * a host-side halftoner for callers without a GPU; no GPU call uses it.
 * Definition:
 * raster order, threshold v >= 0.5, weights 7/16 right, 3/16 down-left,
 * 5/16 down, 1/16 down-right, error leaving the image dropped.
 * contone_host [B][H][W] FP32 in host memory; bits_host [B][H][W] out.
 * --------------------------------------------------------------------- */
int halftone_error_diffusion_host(const float* contone_host, int B, int H, int W,
                                  uint8_t* bits_host);
/* The same with L output levels k / (L-1), the serial fallback beside the
 * multitoning variant (Sec. VI-E): each pixel takes the level nearest to
 * v = c + diffused error (a tie going up, clamped to 0..L-1) and diffuses
 * v - k / (L-1) with the same weights; levels = 2 gives the bits of
 * halftone_error_diffusion_host. levels_host [B][H][W] level indices out;
 * HS_EINVAL for levels outside 2..HS_MAX_LEVELS. */
int halftone_error_diffusion_levels_host(const float* contone_host, int B, int H, int W,
                                         int levels, uint8_t* levels_host);

#ifdef __cplusplus
}
#endif
#endif /* HALFTONE_H */
