// hs_internal.h -- host-side launchers shared by the translation units of
// libhalftone. Not part of the public ABI (include/halftone.h is).
#pragma once
#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include "../../include/halftone.h"

// Offsets of the layers in the flat weight array (layer after layer,
// W[cout][cin][3][3] then bias[cout]): 2 -> 32, four 32 -> 32, 32 -> 1.
constexpr int HS_C = 32;
constexpr int HS_W1 = 0;                       // W1[32][2][9]
constexpr int HS_B1 = HS_W1 + 32 * 2 * 9;      // 576
constexpr int HS_L32_SIZE = 32 * 32 * 9 + 32;  // 9248
constexpr int HS_W2 = HS_B1 + 32;              // 608
constexpr int hs_wk(int k) { return HS_W2 + (k - 2) * HS_L32_SIZE; }  // k = 2..5
constexpr int hs_bk(int k) { return hs_wk(k) + 32 * 32 * 9; }
constexpr int HS_W6 = HS_W2 + 4 * HS_L32_SIZE;  // 37600
constexpr int HS_B6 = HS_W6 + 32 * 9;           // 37888
static_assert(HS_B6 + 1 == HS_PARAM_COUNT, "parameter layout");

namespace hs {

constexpr int NPARAM = HS_PARAM_COUNT;

// One page (image) of an inference call: pixels [off, off + H W) of the
// concatenated buffers, its first virtual strip row in the fused kernel's
// work partition, and its strip count. Its seed is seeds[page].
struct Page {
  long long off;
  long long vstart;
  int H, W, nstrip, pad;
};
// A recheck-list entry: pixel index (bits 0-30), page (31-62), the bit
// decided so far (63).
constexpr uint64_t ENTRY_PIXEL = 0x7FFFFFFFull;
inline __host__ __device__ uint32_t entry_pixel(uint64_t e) { return (uint32_t)(e & ENTRY_PIXEL); }
inline __host__ __device__ int entry_page(uint64_t e) { return (int)((e >> 31) & 0xFFFFFFFFull); }
inline __host__ __device__ int entry_bit(uint64_t e) { return (int)(e >> 63); }
constexpr int WGRAD_BLOCKS = 512;  // rows of weight-gradient partial sums

// Output levels of the test phase (Sec. VI-E multitoning; binary = 2 levels):
// level = #{j : x >= thr[j]} over the logit midpoints
// thr[j] = logit((j + 1/2) / (L - 1)), j = 0..L-2; binary: thr = {0}.
constexpr int MAX_LEVELS = 8;
struct Levels {
  int n;  // L - 1 thresholds, ascending
  float thr[MAX_LEVELS - 1];
};
Levels make_levels(int L);
// level of logit x, the distance to the nearest threshold and the side of it
inline __host__ __device__ int level_of(const Levels& q, float x, float* dist, int* side) {
  int lev = 0;
  float best = 3.0e38f;
  int sd = 0;
  for (int j = 0; j < q.n; ++j) {
    const float d = x - q.thr[j];
    lev += d >= 0.0f ? 1 : 0;
    const float ad = d < 0.0f ? -d : d;
    if (ad < best) {
      best = ad;
      sd = d >= 0.0f ? 1 : 0;
    }
  }
  *dist = best;
  *side = sd;
  return lev;
}
// index of the threshold nearest to x
inline __host__ __device__ int nearest_threshold(const Levels& q, float x) {
  int k = 0;
  float best = 3.0e38f;
  for (int j = 0; j < q.n; ++j) {
    const float d = x - q.thr[j], ad = d < 0.0f ? -d : d;
    if (ad < best) {
      best = ad;
      k = j;
    }
  }
  return k;
}

// Bytes of one NHWC 32-channel activation map of n pixels.
inline size_t act_bytes(size_t n, int precision) {
  return n * 32 * (precision == HS_BF16 ? 2 : 4);
}
inline size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

// Packed weights of the four 32->32 layers in MFMA operand order
// (9 taps x 2 row tiles x 64 lanes x 8 values per layer).
constexpr int PACK32_PER_LAYER = 9 * 2 * 64 * 8;  // 9216
inline size_t pack_bytes(int precision) {
  return 4 * (size_t)PACK32_PER_LAYER * (precision == HS_BF16 ? 2 : 4);
}

// conv.hip
hipError_t launch_pack32(const float* w, void* out, int precision, int transposed, hipStream_t s);
// Both copies (forward into outF, transposed into outT) in one launch.
hipError_t launch_pack32_both(const float* w, void* outF, void* outT, int precision,
                              hipStream_t s);
hipError_t launch_conv_first(const float* contone, const uint64_t* seeds, const float* w, int B,
                             int H, int W, int kind, uint32_t step, int precision, void* out,
                             float* zout, float* cout, hipStream_t s);
hipError_t launch_conv32(const void* in, const void* wpack, const float* bias, const void* mask,
                         void* out, int B, int H, int W, int precision, int mode, hipStream_t s);
// mode 0: bits or levels (+ logits); mode 1: probs + actions sampled from
// stream 0 at step (bits, or level indices when lv.n > 1)
hipError_t launch_conv_last(const void* in, const float* w, int B, int H, int W, int precision,
                            int mode, const uint64_t* seeds, uint32_t step, uint8_t* bits,
                            float* logits, float* probs, float tau, uint32_t* list, int* count,
                            const Levels& lv, hipStream_t s);
// infer.hip: the fused BF16 pass
hipError_t launch_zero_ints(int* p, int n, hipStream_t s);
// *count (zeroed beforehand) += the NaN and infinite values of x[0, n)
hipError_t launch_count_nonfinite(const float* x, size_t n, int* count, hipStream_t s);
size_t fused_frag_bytes();
// Set-up folded into the fragment packing launch: zero0[0..n0) and
// zero1[0..n1) cleared (null / 0 to skip), and when pages is set the page
// table of a uniform batch of B images of H x W.
struct PackPrologue {
  int* zero0;
  int n0;
  int* zero1;
  int n1;
  Page* pages;
  int B, H, W;
};
// BF16 fragments into frags and, when frags16 is not null, the same in FP16
// and *needs_all: 1 unless a priori bounds keep FP16 layers 1..4 in range
hipError_t launch_fused_pack(const float* w, void* frags, void* frags16, int* needs_all,
                             const PackPrologue& pro, hipStream_t s);
// the prologue alone (weights packed beforehand)
hipError_t launch_prologue(const PackPrologue& pro, hipStream_t s);
// persistent fused inference over pages (one launch for all of them;
// shapes_host = [npages][H, W] as in the device page table); the recheck
// list is segmented (two segments per workgroup, counts in seg_count; list
// may be null). form FUSED_BF16, or FP16 fragments and activations with
// *ovf set to 1 when a tested value overflows FP16: FUSED_FP16_L5 tests
// layer 5 and the contone range, FUSED_FP16_ALL every layer. guard (may be
// null): the launch does nothing unless (*guard != 0) == guard_nonzero
int fused_strips(int W);
int fused_fill();
hipError_t launch_uniform_pages(Page* pages, int B, int H, int W, hipStream_t s);
hipError_t launch_put_pages(Page* dst, const Page* src_host, int n, hipStream_t s);
size_t fused_list_entries(const int* shapes_host, int npages, int num_cus);
hipError_t launch_fused_infer(const float* w, const float* contone, const uint64_t* seeds,
                              const Page* pages, const int* shapes_host, int npages, int kind,
                              float tau, const Levels& lv, uint8_t* bits, float* logits,
                              uint64_t* list, int* seg_count, int* nseg, long long* seg_cap,
                              const void* frags, const void* frags8, int form, int* ovf,
                              const int* guard, int guard_nonzero, int num_cus, hipStream_t s);
// FUSED_FP8: layers 2..5 in FP8 from frags8 (the FP8 block), layers 1 and 6
// in BF16 (layer 6 from frags), *ovf set to 1 when an activation saturated
enum { FUSED_BF16 = 0, FUSED_FP16_L5 = 1, FUSED_FP16_ALL = 2, FUSED_FP8 = 3 };
// the FP8 block: FP8 fragments of layers 2..5 with per-output-channel
// power-of-two scales, layer 1 in BF16, the row scales and biases for the
// activation scales 2^act_exp[0..3] of layers 1..4
size_t fp8_block_bytes();
hipError_t launch_fp8_pack(const float* w, void* blk, const int* act_exp, hipStream_t s);
// *out = max(*out, x[0, n)) for non-negative floats, n a multiple of 4
hipError_t launch_layer_max(const float* x, size_t n, float* out, hipStream_t s);
// recheck.hip: re-evaluation of listed pixels over their receptive field
// (wt: layers 2..5 transposed for the FP32 stage, fp32_pack_bytes())
hipError_t launch_recheck_fp32(const float* w, const float* contone, const uint64_t* seeds,
                               const Page* pages, int kind, const uint64_t* list,
                               const int* count, const void* wt, const Levels& lv, uint8_t* bits,
                               float* logits, int32_t* stats, int count_slot, int num_cus,
                               hipStream_t s);
size_t split_frag_bytes();
size_t half_frag_bytes();
size_t fp32_pack_bytes();
// the weight copies of the cone stages: split hi / lo (BF16), FP16, FP32
// transposed, and a flag set when a weight of layers 1..5 overflows FP16
struct ConeWeights {
  void *whi, *wlo, *w16, *wt;
  int* wflag;
};
// wflag must be zero before the launch
hipError_t launch_split_pack(const float* w, const ConeWeights& cw, hipStream_t s);
// one cone stage over a segmented list: the FP16 form (half) or the split
// form; pixels at least `band` from the nearest threshold are decided, the
// others appended to list_out (count_out); stats[total_slot] = the number
// of input entries
hipError_t launch_recheck_cones(bool half, const float* w, const float* contone,
                                const uint64_t* seeds, const Page* pages, int kind,
                                const uint64_t* seglist, const int* seg_count, int nseg,
                                long long seg_cap, const ConeWeights& cw, float band,
                                const Levels& lv, uint64_t* list_out, int* count_out,
                                uint8_t* bits, float* logits, int32_t* stats, int total_slot,
                                int num_cus, hipStream_t s);
// g6 = grad (if probs == null) or grad * p (1 - p); writes g6 and the
// masked input gradient of layer 6.
hipError_t launch_dgrad_last(const float* grad, const float* probs, const void* a5,
                             const float* w, int B, int H, int W, int precision, float* g6,
                             void* g5, hipStream_t s);
// The head's and layer 6's backward: the input gradient g5 as
// launch_dgrad_last and the weight-gradient partial rows as
// launch_wgrad_last (BF16: one pass that writes no g6; FP32: those two)
hipError_t launch_bwd_last(const float* grad, const float* probs, const void* a5, const float* w,
                           int B, int H, int W, int precision, float* g6, void* g5,
                           float* partials, int accumulate, hipStream_t s);
hipError_t launch_wgrad_first(const float* contone, const float* z, const void* g1, int B, int H,
                              int W, int precision, float* partials, int accumulate,
                              hipStream_t s);
// BF16 only: the input gradient g_in of a 32->32 layer (through the ReLU
// mask of a_in) and its weight-gradient partial rows in one pass
hipError_t launch_bwd32(const void* a_in, const void* g_out, const void* wpackT, void* g_in,
                        int layer, int B, int H, int W, float* partials, int accumulate,
                        int num_cus, hipStream_t s);
hipError_t launch_wgrad32(const void* a_in, const void* g_out, int layer, int B, int H, int W,
                          int precision, float* partials, int accumulate, hipStream_t s);
hipError_t launch_wgrad_last(const void* a5, const float* g6, int B, int H, int W, int precision,
                             float* partials, int accumulate, hipStream_t s);
// sums `rows` rows of NPARAM partial sums in a fixed order; `tmp` holds
// REDUCE_GROUPS * NPARAM + REDUCE_BLOCKS floats, the last REDUCE_BLOCKS of
// which receive partial sums of grad^2 (launch_train_metrics' gsq)
constexpr int REDUCE_GROUPS = 16;
constexpr int REDUCE_BLOCKS = (NPARAM + 255) / 256;
// the grid (and partial rows) of launch_bwd32 on a device with num_cus CUs
int bwd32_grid(int num_cus);
hipError_t launch_reduce_partials(const float* partials, int rows, int rows32, float* tmp,
                                  float* grad, hipStream_t s);
// The two levels apart, for the train step: the group sums of the rows into
// tmp[0..REDUCE_GROUPS) (launch_reduce_rows), then the gradient as tmp0's
// group sums and then tmp1's (null: none) into grad, the per-block sums of
// grad^2 into gsq, and the Adam update of w, m, v with it (train.hip; c1,
// c2 the bias corrections 1 - beta^t).
hipError_t launch_reduce_rows(const float* partials, int rows, int rows32, float* tmp,
                              hipStream_t s);
hipError_t launch_reduce_adam(const float* tmp0, const float* tmp1, float* grad, float* gsq,
                              float* w, float* m, float* v, float lr, float b1, float b2,
                              float eps, float c1, float c2, hipStream_t s);

// loss.hip
struct LossDev {  // the two normalised windows, passed to kernels by value
  float G[15 * 15];
  float w[15 * 15];
  float g1[15], w1[15];  // their normalised 1-D factors (G = g1 g1^T, w = w1 w1^T)
};
void make_windows(const hs_loss_params& p, LossDev* host_out);
hipError_t launch_loss_stats(const uint8_t* h, const float* c, int B, int H, int W,
                             const hs_loss_params& p, const LossDev& win, float* maps,
                             float* tile_partials, int ntiles_per_img, hipStream_t s);
hipError_t launch_loss_reduce(const float* tile_partials, int B, int ntiles_per_img,
                              const float* as_partials, int npatch, float w_s, long M, float* out,
                              hipStream_t s);
// out[3B + 1] = -mean_b out[3b + 2] + w_a out[3B] (after launch_loss_reduce)
hipError_t launch_loss_total(int B, float w_a, float* out, hipStream_t s);
// per-pixel policy gradient from the toggle differences dR (Local Expectation
// or COMA, p.estimator); probs may be null only for LE in probability space
hipError_t launch_le_grad(const uint8_t* h, const float* c, const float* probs, int logit_space,
                          int B, int H, int W, const hs_loss_params& p, const LossDev& win,
                          const float* maps, float* grad, hipStream_t s);
hipError_t launch_as(const float* pg, int Bg, int Hg, int Wg, float scale, int logit_space,
                     float* patch_loss, float* grad_or_null, hipStream_t s);
hipError_t launch_fill(float* p, size_t n, float v, hipStream_t s);

// train.hip
// the number of actions' ones (levels: the sum of the level indices) into
// *counter
hipError_t launch_count_actions(const uint8_t* actions, size_t nact,
                                unsigned long long* counter, hipStream_t s);
// metrics[8] from the loss sums, the REDUCE_BLOCKS partial sums of grad^2
// (gsq) and the action count (after launch_count_actions)
hipError_t launch_train_metrics(const float* loss_out, int B, const float* gsq,
                                const unsigned long long* counter, size_t nact, int levels,
                                float lr, float w_a, float* metrics, hipStream_t s);

// spectrum.hip
int spectrum_rings(int P);
size_t spectrum_patches(int B, int H, int W, int P);
hipError_t launch_spectrum(const uint8_t* bits, int B, int H, int W, int P, float* spec,
                           float* avg, float* rapsd, float* anis, hipStream_t s);

}  // namespace hs
