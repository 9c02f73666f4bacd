// abi.cpp -- the C entry points of libhalftone (declared in include/halftone.h):
// argument validation, workspace layout and the launch sequence of each call.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <cmath>
#include <initializer_list>
#include <mutex>
#include <string>
#include <utility>
#include <vector>

#include "hs_internal.h"

using namespace hs;

namespace {

thread_local std::string g_err;

int fail(int code, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_err = buf;
  return code;
}

#define HS_TRY(expr)                                                                    \
  do {                                                                                  \
    hipError_t e_ = (expr);                                                             \
    if (e_ != hipSuccess) return fail(HS_EHIP, "%s: %s", #expr, hipGetErrorString(e_)); \
  } while (0)

// The library is built for gfx950 only; refuse other devices up front.
int check_device() {
  static std::mutex mu;
  static std::vector<int> state;  // per device: 0 unknown, 1 ok, 2 unsupported
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return fail(HS_EHIP, "hipGetDevice failed");
  std::lock_guard<std::mutex> lk(mu);
  if ((int)state.size() <= dev) state.resize(dev + 1, 0);
  if (state[dev] == 0) {
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, dev) != hipSuccess)
      return fail(HS_EHIP, "hipGetDeviceProperties failed");
    state[dev] = strncmp(prop.gcnArchName, "gfx950", 6) == 0 ? 1 : 2;
  }
  if (state[dev] != 1) return fail(HS_EUNSUPPORTED, "device %d is not gfx950", dev);
  return HS_OK;
}

// Bump allocator over the caller's workspace; with base == nullptr it only
// measures, so the *_workspace_size functions and the entry points share one
// layout description.
struct Carve {
  char* base;
  size_t off = 0;
  explicit Carve(void* b) : base((char*)b) {}
  template <typename T> T* take(size_t bytes) {
    T* p = base ? (T*)(base + off) : nullptr;
    off = align256(off + bytes);
    return p;
  }
};

bool shape_ok(int B, int H, int W) {
  return B >= 1 && H >= 1 && W >= 1 && (long long)B * H * W < (1ll << 31);
}

int check_params(const hs_loss_params* p) {
  if (!p) return fail(HS_EINVAL, "null loss parameters");
  if (p->hvs_radius < 1 || p->hvs_radius > 7 || p->ssim_radius < 1 || p->ssim_radius > 7)
    return fail(HS_EINVAL, "window radii must be in 1..7");
  if (!(p->hvs_sigma > 0.0f) || !(p->ssim_sigma > 0.0f)) return fail(HS_EINVAL, "sigma <= 0");
  if (p->as_patch != 32) return fail(HS_EUNSUPPORTED, "only 32x32 anisotropy patches");
  if (p->estimator != HS_EST_LE && p->estimator != HS_EST_COMA)
    return fail(HS_EINVAL, "estimator %d", p->estimator);
  if (p->levels < 2 || p->levels > HS_MAX_LEVELS)
    return fail(HS_EINVAL, "levels %d (2..%d)", p->levels, HS_MAX_LEVELS);
  if (p->levels > 2 && p->estimator != HS_EST_LE)
    return fail(HS_EUNSUPPORTED, "multitone levels need the Local Expectation estimator");
  if (p->flags & ~HS_CHECK_FINITE) return fail(HS_EINVAL, "loss flags 0x%x", p->flags);
  return HS_OK;
}

// HS_CHECK_FINITE: count the NaN / infinite values of the given inputs on
// the device (counter: one device int of the call's workspace), wait for the
// count and fail with HS_ENONFINITE if there is any.
struct FloatSpan {
  const float* p;
  size_t n;
};
int check_finite(std::initializer_list<FloatSpan> spans, int* counter, hipStream_t s,
                 const char* who) {
  if (launch_zero_ints(counter, 1, s) != hipSuccess)
    return fail(HS_EHIP, "%s: clearing the finite-check counter failed", who);
  for (const FloatSpan& sp : spans)
    if (sp.p && launch_count_nonfinite(sp.p, sp.n, counter, s) != hipSuccess)
      return fail(HS_EHIP, "%s: finite check launch failed", who);
  int bad = 0;
  if (hipMemcpyAsync(&bad, counter, sizeof(int), hipMemcpyDeviceToHost, s) != hipSuccess ||
      hipStreamSynchronize(s) != hipSuccess)
    return fail(HS_EHIP, "%s: reading the finite-check counter failed", who);
  if (bad) return fail(HS_ENONFINITE, "%s: %d non-finite input values", who, bad);
  return HS_OK;
}

int margin(const hs_loss_params* p) {
  return p->hvs_radius > p->ssim_radius ? p->hvs_radius : p->ssim_radius;
}

// ---------------------------------------------------------------- layouts --
// Activations of the training forward: act(j) is the output of layer j + 1
// (j = 0..4). Kept in five buffers, or, with recomputation, in two that
// alternate (act(j) in buffer j % 2): the backward then rebuilds act(j)
// from the input by re-running layers 1..j+1 when it needs it.
struct PolicyWs {
  void *packF, *packT, *buf[5], *gA, *gB;
  float *z, *c, *g6, *partials, *rtmp;
  unsigned long long* counter;
  bool recompute;
  void* act(int j) const { return buf[recompute ? j % 2 : j]; }
};
// partials: the rows of weight-gradient partial sums to use, or null to
// carve WGRAD_BLOCKS x rows of them
PolicyWs carve_policy(Carve& cv, size_t N, int prec, bool recompute = false,
                      float* partials = nullptr, int rows = WGRAD_BLOCKS) {
  PolicyWs w;
  w.recompute = recompute;
  w.packF = cv.take<char>(pack_bytes(prec));
  w.packT = cv.take<char>(pack_bytes(prec));
  for (int k = 0; k < 5; ++k) w.buf[k] = k < (recompute ? 2 : 5) ? cv.take<char>(act_bytes(N, prec)) : nullptr;
  w.gA = cv.take<char>(act_bytes(N, prec));
  w.gB = cv.take<char>(act_bytes(N, prec));
  w.z = cv.take<float>(N * 4);
  w.c = cv.take<float>(N * 4);
  w.g6 = cv.take<float>(N * 4);
  w.partials = partials ? partials : cv.take<float>((size_t)rows * NPARAM * 4);
  w.rtmp = cv.take<float>(((size_t)REDUCE_GROUPS * NPARAM + REDUCE_BLOCKS) * 4);
  w.counter = cv.take<unsigned long long>(64);
  return w;
}

struct LossWs {
  float *maps, *tiles, *patches;
  int* flag;  // the finite check's counter
  int ntiles;
};
LossWs carve_loss(Carve& cv, int B, int H, int W, int Bg, int Hg, int Wg, int m, bool maps) {
  LossWs w;
  const int vh = H - 2 * m, vw = W - 2 * m;
  w.ntiles = ((vh + 15) / 16) * ((vw + 15) / 16);
  w.maps = maps ? cv.take<float>((size_t)6 * B * H * W * 4) : nullptr;
  w.tiles = cv.take<float>((size_t)B * w.ntiles * 2 * 4);
  const size_t np = (size_t)Bg * (Hg / 32) * (Wg / 32);
  w.patches = cv.take<float>((np > 0 ? np : 1) * 4);
  w.flag = cv.take<int>(64);
  return w;
}

struct InferWs {
  void *pack, *a0, *a1;
};
InferWs carve_infer(Carve& cv, size_t N, int prec) {
  InferWs w;
  w.pack = cv.take<char>(pack_bytes(prec));
  w.a0 = cv.take<char>(act_bytes(N, prec));
  w.a1 = cv.take<char>(act_bytes(N, prec));
  return w;
}

// Forward of the stack on one batch: pack -> first -> four 32->32 -> last,
// keeping the activations, with probs (+ actions) out. pack = false: the
// caller has already packed w into pw.packF on this stream.
hipError_t run_forward_train(const float* w, const float* contone, const uint64_t* seeds, int B,
                             int H, int W, int kind, uint32_t step, int prec, const PolicyWs& pw,
                             float* probs, uint8_t* actions, int levels, hipStream_t s,
                             bool pack = true) {
  hipError_t e;
  if (pack && (e = launch_pack32(w, pw.packF, prec, 0, s)) != hipSuccess) return e;
  if ((e = launch_conv_first(contone, seeds, w, B, H, W, kind, step, prec, pw.act(0), pw.z, pw.c,
                             s)) != hipSuccess)
    return e;
  const size_t per_layer = (size_t)PACK32_PER_LAYER * (prec == HS_BF16 ? 2 : 4);
  for (int k = 2; k <= 5; ++k) {
    if ((e = launch_conv32(pw.act(k - 2), (const char*)pw.packF + (k - 2) * per_layer,
                           w + hs_bk(k), nullptr, pw.act(k - 1), B, H, W, prec, 0, s)) !=
        hipSuccess)
      return e;
  }
  return launch_conv_last(pw.act(4), w, B, H, W, prec, 1, seeds, step, actions, nullptr, probs,
                          0.0f, nullptr, nullptr, make_levels(levels), s);
}

// Recomputation: act(j) again from the input (layers 1..j+1, the same
// kernels and inputs as the forward, so the same values); z and c are kept.
struct FwdInput {
  const float* contone;
  const uint64_t* seeds;
  int kind;
  uint32_t step;
};
hipError_t recompute_act(const float* w, const FwdInput& in, int j, int B, int H, int W, int prec,
                         const PolicyWs& pw, hipStream_t s) {
  hipError_t e;
  if ((e = launch_conv_first(in.contone, in.seeds, w, B, H, W, in.kind, in.step, prec, pw.act(0),
                             nullptr, nullptr, s)) != hipSuccess)
    return e;
  const size_t per_layer = (size_t)PACK32_PER_LAYER * (prec == HS_BF16 ? 2 : 4);
  for (int k = 2; k <= j + 1; ++k) {
    if ((e = launch_conv32(pw.act(k - 2), (const char*)pw.packF + (k - 2) * per_layer,
                           w + hs_bk(k), nullptr, pw.act(k - 1), B, H, W, prec, 0, s)) !=
        hipSuccess)
      return e;
  }
  return hipSuccess;
}

int num_cus();  // compute units of the current device (below)

// Backward of the stack given dL/dprobs (probs != null) or dL/dlogit
// (probs == null); accumulates into the weight-gradient partial rows.
// With pw.recompute, `in` must be the forward's input (act(4) is still in
// its buffer from the forward; the others are rebuilt layer by layer).
hipError_t run_backward(const float* w, const float* grad, const float* probs, int B, int H,
                        int W, int prec, const PolicyWs& pw, int accumulate, hipStream_t s,
                        const FwdInput* in = nullptr, bool pack = true) {
  hipError_t e;
  if (pack && (e = launch_pack32(w, pw.packT, prec, 1, s)) != hipSuccess) return e;
  if ((e = launch_bwd_last(grad, probs, pw.act(4), w, B, H, W, prec, pw.g6, pw.gA, pw.partials,
                           accumulate, s)) != hipSuccess)
    return e;
  const size_t per_layer = (size_t)PACK32_PER_LAYER * (prec == HS_BF16 ? 2 : 4);
  void* g = pw.gA;  // gradient at the pre-activation of layer k
  void* other = pw.gB;
  for (int k = 5; k >= 2; --k) {
    if (pw.recompute && (e = recompute_act(w, *in, k - 2, B, H, W, prec, pw, s)) != hipSuccess)
      return e;
    if (prec == HS_BF16) {
      // input and weight gradients in one pass over g and a
      if ((e = launch_bwd32(pw.act(k - 2), g, (const char*)pw.packT + (k - 2) * per_layer, other,
                            k, B, H, W, pw.partials, accumulate, num_cus(), s)) != hipSuccess)
        return e;
    } else {
      if ((e = launch_wgrad32(pw.act(k - 2), g, k, B, H, W, prec, pw.partials, accumulate, s)) !=
          hipSuccess)
        return e;
      if ((e = launch_conv32(g, (const char*)pw.packT + (k - 2) * per_layer, nullptr,
                             pw.act(k - 2), other, B, H, W, prec, 1, s)) != hipSuccess)
        return e;
    }
    void* t = g;
    g = other;
    other = t;
  }
  return launch_wgrad_first(pw.c, pw.z, g, B, H, W, prec, pw.partials, accumulate, s);
}

int num_cus() {
  static std::mutex mu;
  static std::vector<int> cache;
  int dev = 0;
  (void)hipGetDevice(&dev);
  std::lock_guard<std::mutex> lk(mu);
  if ((int)cache.size() <= dev) cache.resize(dev + 1, 0);
  if (cache[dev] == 0) {
    int n = 0;
    if (hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || n <= 0)
      n = 256;
    cache[dev] = n;
  }
  return cache[dev];
}

// Event pairs around the dominant kernel of each inference call, recorded
// only between halftone_profile_start and halftone_profile_stop.
struct Profiler {
  std::mutex mu;
  bool on = false;
  std::vector<hipEvent_t> ev;  // pairs: 2i begin, 2i + 1 end
  int used = 0;
} g_prof;
constexpr int PROF_MAX = 4096;

void prof_begin(hipStream_t s) {
  std::lock_guard<std::mutex> lk(g_prof.mu);
  if (!g_prof.on || g_prof.used >= PROF_MAX) return;
  while ((int)g_prof.ev.size() < 2 * (g_prof.used + 1)) {
    hipEvent_t e;
    if (hipEventCreate(&e) != hipSuccess) return;
    g_prof.ev.push_back(e);
  }
  (void)hipEventRecord(g_prof.ev[2 * g_prof.used], s);
}

void prof_end(hipStream_t s) {
  std::lock_guard<std::mutex> lk(g_prof.mu);
  if (!g_prof.on || g_prof.used >= PROF_MAX || (int)g_prof.ev.size() < 2 * (g_prof.used + 1))
    return;
  (void)hipEventRecord(g_prof.ev[2 * g_prof.used + 1], s);
  ++g_prof.used;
}

}  // namespace

namespace hs {
// thr[j] = logit((j + 1/2) / (L - 1)) = log((2j + 1) / (2L - 3 - 2j)), in
// double then rounded; L = 2 gives exactly {0}
Levels make_levels(int L) {
  Levels q;
  q.n = L - 1;
  for (int j = 0; j < MAX_LEVELS - 1; ++j)
    q.thr[j] = j < q.n ? (float)log((2.0 * j + 1.0) / (2.0 * L - 3.0 - 2.0 * j)) : 0.0f;
  return q;
}
}  // namespace hs

// ===================================================================== ABI ==
extern "C" {

void halftone_default_loss_params(hs_loss_params* p) {
  if (!p) return;
  p->w_s = 0.06f;
  p->w_a = 0.002f;
  p->hvs_sigma = 2.0f;
  p->hvs_radius = 5;
  p->ssim_sigma = 1.5f;
  p->ssim_radius = 5;
  p->k = 2.0f;
  p->c1 = 1e-4f;
  p->c2 = 9e-4f;
  p->as_patch = 32;
  p->estimator = HS_EST_LE;
  p->levels = 2;
  p->flags = 0;
}

void halftone_default_train_params(hs_train_params* p) {
  if (!p) return;
  halftone_default_loss_params(&p->loss);
  p->lr_max = 3e-4f;
  p->lr_min = 1e-5f;
  p->beta1 = 0.9f;
  p->beta2 = 0.999f;
  p->eps = 1e-8f;
  p->noise_kind = HS_NOISE_GAUSS;
  p->recompute = 0;
}

int halftone_version(void) { return 200; }

int halftone_profile_start(void) {
  std::lock_guard<std::mutex> lk(g_prof.mu);
  g_prof.on = true;
  g_prof.used = 0;
  return HS_OK;
}

int halftone_profile_stop(double* ms_total, int* launches) {
  if (!ms_total || !launches) return fail(HS_EINVAL, "halftone_profile_stop: null pointer");
  std::lock_guard<std::mutex> lk(g_prof.mu);
  g_prof.on = false;
  double sum = 0.0;
  for (int i = 0; i < g_prof.used; ++i) {
    HS_TRY(hipEventSynchronize(g_prof.ev[2 * i + 1]));
    float ms = 0.0f;
    HS_TRY(hipEventElapsedTime(&ms, g_prof.ev[2 * i], g_prof.ev[2 * i + 1]));
    sum += ms;
  }
  *ms_total = sum;
  *launches = g_prof.used;
  g_prof.used = 0;
  return HS_OK;
}
const char* halftone_last_error(void) { return g_err.c_str(); }
int64_t halftone_param_count(void) { return HS_PARAM_COUNT; }

// ------------------------------------------------------------- inference --
// The cone stages' weight copies in one region: split hi | lo, FP32
// transposed, FP16.
static size_t cone_region_bytes() {
  return split_frag_bytes() + fp32_pack_bytes() + half_frag_bytes();
}
static ConeWeights cone_weights(char* region, int* wflag) {
  ConeWeights cw;
  cw.whi = region;
  cw.wlo = region + split_frag_bytes() / 2;
  cw.wt = region + split_frag_bytes();
  cw.w16 = region + split_frag_bytes() + fp32_pack_bytes();
  cw.wflag = wflag;
  return cw;
}

// The packed copies of one weight set: the FP32 weights, the fused pass's
// BF16 and FP16 fragments, its FP16 layer bounds flag, the split hi/lo and
// transposed FP32 copies of the recheck stages, and the FP32 per-layer
// fragments. They live in a packed policy's memory, or in the workspace of a
// call that packs for itself.
struct Packed {
  float* w;
  char *frags, *frags16, *split, *pack32, *frags8;
  int* needs_all;
};
static size_t policy_layout(void* base, Packed* out) {
  Carve cv(base);
  Packed p;
  p.w = cv.take<float>((size_t)NPARAM * 4);
  p.frags = cv.take<char>(fused_frag_bytes());
  p.frags16 = cv.take<char>(fused_frag_bytes());
  p.split = cv.take<char>(cone_region_bytes());
  p.pack32 = cv.take<char>(pack_bytes(HS_FP32));
  p.needs_all = cv.take<int>(64 * sizeof(int));
  p.frags8 = cv.take<char>(fp8_block_bytes());
  if (out) *out = p;
  return cv.off;
}

// Workspace of the 16-bit paths (sizes in bytes) for pages of the given
// shapes: packed BF16 and FP16 fragments, the split and FP32 weight copies,
// the page table, the segmented recheck list and its counts, the FP32-stage
// list, counters.
struct Bf16Ws {
  char *pack, *pack16, *split;
  Page* pages;
  uint64_t *seglist, *list2;
  int *seg_count, *cnt;
};
static size_t bf16_ws(const int* shapes, int npages, size_t N, Bf16Ws* out, void* base) {
  Carve cv(base);
  Bf16Ws w;
  w.pack = cv.take<char>(fused_frag_bytes());
  w.pack16 = cv.take<char>(fused_frag_bytes());
  w.split = cv.take<char>(cone_region_bytes());
  w.pages = cv.take<Page>((size_t)npages * sizeof(Page));
  const size_t ne = fused_list_entries(shapes, npages, num_cus());
  w.seglist = cv.take<uint64_t>(ne * sizeof(uint64_t));
  w.seg_count = cv.take<int>((2 * (size_t)num_cus() + 16) * sizeof(int));
  w.list2 = cv.take<uint64_t>(N * sizeof(uint64_t));
  w.cnt = cv.take<int>(64);
  if (out) *out = w;
  return cv.off;
}
// counters of the 16-bit workspace: [0, 24) cleared by the prologue (1 and 2
// the lengths of the lists between the cone stages, 3 the FP16 weight flag
// of a self-packing call, [16, 24) the statistics when the caller passes
// none), 24 the FP16 bounds flag of a self-packing call, 40 the finite
// check's counter
constexpr int CNT_FINITE = 40;
constexpr int NSTATS = 8;  // entries of the statistics array

// Workspace of the FP32 path for one batch of B images of H x W.
static size_t fp32_ws(int B, int H, int W, InferWs* out, int** cnt, void* base) {
  Carve cv(base);
  InferWs w = carve_infer(cv, (size_t)B * H * W, HS_FP32);
  int* c = cv.take<int>(64);
  if (out) *out = w;
  if (cnt) *cnt = c;
  return cv.off;
}

static std::vector<int> uniform_shapes(int B, int H, int W) {
  std::vector<int> s(2 * (size_t)B);
  for (int b = 0; b < B; ++b) {
    s[2 * b] = H;
    s[2 * b + 1] = W;
  }
  return s;
}

size_t halftone_infer_workspace_size(int B, int H, int W, int precision) {
  if (!shape_ok(B, H, W)) return 0;
  if (precision != HS_FP32) {
    const std::vector<int> sh = uniform_shapes(B, H, W);
    return bf16_ws(sh.data(), B, (size_t)B * H * W, nullptr, nullptr);
  }
  return fp32_ws(B, H, W, nullptr, nullptr, nullptr);
}

// The split stage decides |x| >= tau2 and must err by less than tau2: the
// default is tau / 64 (the split products carry about 2^-8 of the 16-bit
// error, so this keeps the factor 1.3..1.5 of tau over the 16-bit error
// about 16 times over the split error whatever the weights), and at least
// 1.5e-4, which is under the 4e-4 margin and 2.8 times the largest split
// error measured for the He policy.
static float default_tau2(float tau) { return fmaxf(tau / 64.0f, 1.5e-4f); }
// The bits must equal the oracle's wherever |p - 1/2| > 1e-4, i.e. |x| >
// 2 atanh(2e-4) = 4.0e-4. A pixel the split stage leaves undecided has
// |x_split| < tau2 and so, its error being below tau2, an exact |x| below
// 2 tau2: with tau2 <= 2e-4 it is inside that margin, where either bit is
// the oracle's, and the split stage decides it from its own logit; only a
// larger tau2 needs the FP32 stage.
constexpr float HALF_MARGIN_X = 2.0e-4f;
// The FP16 cone stage after a BF16 pass decides |x| >= tau16 (FP16 rounds 8
// times finer than BF16, so a quarter of the BF16 band would leave it twice
// its share of the error). Per listed pixel it costs about as much as the
// split stage it would spare, so by default it is off; a packed policy's
// call can set its band.
static float default_tau16(float) { return 0.0f; }

// The fused pass's arithmetic.
enum Pass { PASS_BF16, PASS_FP16, PASS_FP8 };

// The 16-bit path over a page table (one persistent fused launch for all pages):
//   stage 1: fused BF16 (or FP16, or FP8) pass, pixels with |x| < tau listed
//   stage 1b (FP16 and FP8): if an activation overflowed FP16 or saturated
//            FP8, the fused BF16 pass again, with 8 tau after FP16 (BF16
//            rounds 8 times coarser) and tau / 8 after FP8 (E4M3 keeps 4
//            significant bits to BF16's 8, and its measured logit error is
//            12 to 16 times BF16's); a launch that returns at once
//            otherwise, so no host synchronisation
//   stage 2: split-BF16 receptive-field recompute, |x| < tau2 listed again
//   stage 3: FP32 receptive-field recompute
// The page table is built on the device (uniform batch) or from pages_host.
// pp: the weights packed beforehand (a packed policy), or null to pack them
// into the workspace in this call.
static int infer_bf16(const float* weights, const Packed* pp, const float* contone,
                      const uint64_t* seeds, const int* shapes, int npages, size_t N,
                      const Page* pages_host, int noise_kind, float recheck_tau, float tau16,
                      float tau2, const Levels& lv, Pass pass, uint8_t* bits, float* logits,
                      int32_t* stats_or_null, void* workspace, hipStream_t s) {
  const bool fp16 = pass == PASS_FP16;
  Bf16Ws w;
  bf16_ws(shapes, npages, N, &w, workspace);
  int32_t* stats = stats_or_null ? stats_or_null : (int32_t*)(w.cnt + 16);
  // counters cleared and the uniform page table written by the first launch
  PackPrologue pro{w.cnt, 24, stats_or_null, stats_or_null ? NSTATS : 0,
                   pages_host ? nullptr : w.pages, npages, shapes[0], shapes[1]};
  if (pages_host) HS_TRY(launch_put_pages(w.pages, pages_host, npages, s));
  ConeWeights cw;
  const int* needs_all;  // FP16: layers 1..4 not cleared by their bounds
  const char *frags, *frags16;
  if (pp) {
    weights = pp->w;
    cw = cone_weights(pp->split, pp->needs_all + 16);
    needs_all = pp->needs_all;
    frags = pp->frags;
    frags16 = pp->frags16;
    HS_TRY(launch_prologue(pro, s));
  } else {
    cw = cone_weights(w.split, w.cnt + 3);  // the flag cleared by the pack's prologue
    needs_all = w.cnt + 24;
    frags = w.pack;
    frags16 = w.pack16;
    HS_TRY(launch_fused_pack(weights, w.pack, fp16 ? w.pack16 : nullptr, w.cnt + 24, pro, s));
    HS_TRY(launch_split_pack(weights, cw, s));
  }
  int nseg = 0;
  long long seg_cap = 0;
  int* ovf = stats + 3;  // zeroed above
  prof_begin(s);
  if (pass == PASS_FP8) {
    HS_TRY(launch_fused_infer(weights, contone, seeds, w.pages, shapes, npages, noise_kind,
                              recheck_tau, lv, bits, logits, w.seglist, w.seg_count, &nseg,
                              &seg_cap, frags, pp->frags8, FUSED_FP8, ovf, nullptr, 0, num_cus(),
                              s));
  } else if (!fp16) {
    HS_TRY(launch_fused_infer(weights, contone, seeds, w.pages, shapes, npages, noise_kind,
                              recheck_tau, lv, bits, logits, w.seglist, w.seg_count, &nseg,
                              &seg_cap, frags, nullptr, FUSED_BF16, nullptr, nullptr, 0,
                              num_cus(), s));
  } else {
    // the device picks the FP16 form: of the two launches, the one whose
    // gate does not match needs_all returns at once
    for (int form : {FUSED_FP16_L5, FUSED_FP16_ALL})
      HS_TRY(launch_fused_infer(weights, contone, seeds, w.pages, shapes, npages, noise_kind,
                                recheck_tau, lv, bits, logits, w.seglist, w.seg_count, &nseg,
                                &seg_cap, frags16, nullptr, form, ovf, needs_all,
                                form == FUSED_FP16_ALL, num_cus(), s));
  }
  prof_end(s);
  if (pass != PASS_BF16)
    HS_TRY(launch_fused_infer(weights, contone, seeds, w.pages, shapes, npages, noise_kind,
                              fp16 ? 8.0f * recheck_tau : 0.125f * recheck_tau, lv, bits, logits,
                              w.seglist, w.seg_count, &nseg, &seg_cap, frags, nullptr,
                              FUSED_BF16, nullptr, ovf, 1, num_cus(), s));
  const bool fp32_stage = tau2 > HALF_MARGIN_X;
  const float split_band = fp32_stage ? tau2 : 0.0f;  // 0: the split stage decides all
  if (pass == PASS_BF16 && tau16 > 0.0f) {
    // FP16 cones over the fused pass's list (into list2), split cones over
    // theirs (into the fused list's memory, which is free by then), FP32
    HS_TRY(launch_recheck_cones(true, weights, contone, seeds, w.pages, noise_kind, w.seglist,
                                w.seg_count, nseg, seg_cap, cw, tau16, lv, w.list2, w.cnt + 1,
                                bits, logits, stats, 0, num_cus(), s));
    HS_TRY(launch_recheck_cones(false, weights, contone, seeds, w.pages, noise_kind, w.list2,
                                w.cnt + 1, 1, (long long)N, cw, split_band, lv, w.seglist,
                                w.cnt + 2, bits, logits, stats, 4, num_cus(), s));
    if (fp32_stage)
      HS_TRY(launch_recheck_fp32(weights, contone, seeds, w.pages, noise_kind, w.seglist,
                                 w.cnt + 2, cw.wt, lv, bits, logits, stats, 2, num_cus(), s));
    return HS_OK;
  }
  // after an FP16 or FP8 pass (or with tau16 = 0): split cones over the fused
  // pass's list, then FP32
  HS_TRY(launch_recheck_cones(false, weights, contone, seeds, w.pages, noise_kind, w.seglist,
                              w.seg_count, nseg, seg_cap, cw, split_band, lv, w.list2, w.cnt + 1,
                              bits, logits, stats, 0, num_cus(), s));
  if (fp32_stage)
    HS_TRY(launch_recheck_fp32(weights, contone, seeds, w.pages, noise_kind, w.list2, w.cnt + 1,
                               cw.wt, lv, bits, logits, stats, 2, num_cus(), s));
  return HS_OK;
}

// The FP32 path (per-layer kernels) on one uniform batch; pack32: the FP32
// fragments packed beforehand, or null to pack them into the workspace.
static int infer_fp32(const float* weights, const char* pack32, const float* contone,
                      const uint64_t* seeds, int B, int H, int W, int noise_kind,
                      const Levels& lv, uint8_t* bits, float* logits, void* workspace,
                      hipStream_t s) {
  InferWs iw;
  int* cnt;
  fp32_ws(B, H, W, &iw, &cnt, workspace);
  const size_t per_layer = (size_t)PACK32_PER_LAYER * 4;
  HS_TRY(launch_zero_ints(cnt, 16, s));
  const char* pack = pack32;
  if (!pack) {
    HS_TRY(launch_pack32(weights, iw.pack, HS_FP32, 0, s));
    pack = (const char*)iw.pack;
  }
  HS_TRY(launch_conv_first(contone, seeds, weights, B, H, W, noise_kind, 0u, HS_FP32, iw.a0,
                           nullptr, nullptr, s));
  void* src = iw.a0;
  void* dst = iw.a1;
  for (int k = 2; k <= 5; ++k) {
    if (k == 2) prof_begin(s);
    HS_TRY(launch_conv32(src, pack + (k - 2) * per_layer, weights + hs_bk(k), nullptr, dst, B, H,
                         W, HS_FP32, 0, s));
    if (k == 5) prof_end(s);
    void* t = src;
    src = dst;
    dst = t;
  }
  HS_TRY(launch_conv_last(src, weights, B, H, W, HS_FP32, 0, seeds, 0u, bits, logits, nullptr,
                          0.0f, nullptr, cnt, lv, s));
  return HS_OK;
}

static int check_infer_args(const float* weights, const float* contone, const uint64_t* seeds,
                            const uint8_t* bits, const void* workspace, int noise_kind,
                            int precision, float recheck_tau, const char* who,
                            bool fp8_ok = false) {
  if (!weights || !contone || !seeds || !bits || !workspace)
    return fail(HS_EINVAL, "%s: null pointer", who);
  if (precision == HS_FP8 && !fp8_ok)
    return fail(HS_EUNSUPPORTED, "%s: HS_FP8 needs a packed policy with FP8 scales "
                "(halftone_policy_set_fp8)", who);
  if (precision != HS_FP32 && precision != HS_BF16 && precision != HS_FP16 &&
      precision != HS_FP8)
    return fail(HS_EUNSUPPORTED, "%s: precision %d", who, precision);
  const int kind = noise_kind & ~HS_CHECK_FINITE;
  if (kind != HS_NOISE_GAUSS && kind != HS_NOISE_UNIFORM)
    return fail(HS_EINVAL, "%s: noise kind %d", who, noise_kind);
  if (!(recheck_tau >= 0.0f)) return fail(HS_EINVAL, "%s: recheck_tau < 0", who);
  return HS_OK;
}

int halftone_infer(const float* weights, const float* contone, const uint64_t* seeds, int B,
                   int H, int W, int noise_kind, int precision, float recheck_tau, uint8_t* bits,
                   float* logits_or_null, int32_t* stats_or_null, void* workspace,
                   size_t workspace_bytes, void* stream) {
  int rc = check_infer_args(weights, contone, seeds, bits, workspace, noise_kind, precision,
                            recheck_tau, "halftone_infer");
  if (rc) return rc;
  if (!shape_ok(B, H, W)) return fail(HS_ESHAPE, "halftone_infer: bad shape %d x %d x %d", B, H, W);
  if (workspace_bytes < halftone_infer_workspace_size(B, H, W, precision))
    return fail(HS_EWORKSPACE, "halftone_infer: workspace too small");
  if ((rc = check_device())) return rc;
  hipStream_t s = (hipStream_t)stream;
  const int kind = noise_kind & ~HS_CHECK_FINITE;
  const size_t N = (size_t)B * H * W;
  if (precision != HS_FP32) {
    const std::vector<int> sh = uniform_shapes(B, H, W);
    if (noise_kind & HS_CHECK_FINITE) {
      Bf16Ws w;
      bf16_ws(sh.data(), B, N, &w, workspace);
      if ((rc = check_finite({{contone, N}}, w.cnt + CNT_FINITE, s, "halftone_infer"))) return rc;
    }
    return infer_bf16(weights, nullptr, contone, seeds, sh.data(), B, N, nullptr, kind,
                      recheck_tau, default_tau16(recheck_tau), default_tau2(recheck_tau),
                      make_levels(2), precision == HS_FP16 ? PASS_FP16 : PASS_BF16, bits,
                      logits_or_null, stats_or_null, workspace, s);
  }
  if (noise_kind & HS_CHECK_FINITE) {
    int* cnt;
    fp32_ws(B, H, W, nullptr, &cnt, workspace);
    if ((rc = check_finite({{contone, N}}, cnt + CNT_FINITE, s, "halftone_infer"))) return rc;
  }
  if (stats_or_null) HS_TRY(launch_zero_ints(stats_or_null, NSTATS, s));
  return infer_fp32(weights, nullptr, contone, seeds, B, H, W, kind, make_levels(2), bits,
                    logits_or_null, workspace, s);
}

// ------------------------------------------------ inference, no allocation --
// The workspace of halftone_infer_noalloc: one array per device, kept until
// the process ends. In host code `scratch` names a host-side stand-in, so
// its device address is looked up once per device (hipGetSymbolAddress with
// that device current) and only that address is ever handed to kernels.
static __device__ __align__(256) unsigned char scratch[HS_NOALLOC_SCRATCH_BYTES];

static int scratch_address(void** out) {
  static std::mutex mu;
  static std::vector<void*> addr;  // per device; null until looked up
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return fail(HS_EHIP, "hipGetDevice failed");
  std::lock_guard<std::mutex> lk(mu);
  if ((int)addr.size() <= dev) addr.resize(dev + 1, nullptr);
  if (!addr[dev]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p)
      return fail(HS_EHIP, "hipGetSymbolAddress(scratch): %s", hipGetErrorString(e));
    addr[dev] = p;
  }
  *out = addr[dev];
  return HS_OK;
}

int halftone_infer_noalloc(const float* weights, const float* contone, const uint64_t* seeds,
                           int B, int H, int W, int noise_kind, int precision, float recheck_tau,
                           uint8_t* bits, float* logits_or_null, int32_t* stats_or_null,
                           void* stream) {
  // the same checks as halftone_infer, before the scratch is looked up
  const int dummy = 0;
  int rc = check_infer_args(weights, contone, seeds, bits, &dummy, noise_kind, precision,
                            recheck_tau, "halftone_infer_noalloc");
  if (rc) return rc;
  if (!shape_ok(B, H, W))
    return fail(HS_ESHAPE, "halftone_infer_noalloc: bad shape %d x %d x %d", B, H, W);
  const size_t need = halftone_infer_workspace_size(B, H, W, precision);
  if (need > (size_t)HS_NOALLOC_SCRATCH_BYTES)
    return fail(HS_EWORKSPACE,
                "halftone_infer_noalloc: %d x %d x %d needs %zu bytes of workspace, more than "
                "the %zu-byte static scratch",
                B, H, W, need, (size_t)HS_NOALLOC_SCRATCH_BYTES);
  if ((rc = check_device())) return rc;
  void* ws = nullptr;
  if ((rc = scratch_address(&ws))) return rc;
  return halftone_infer(weights, contone, seeds, B, H, W, noise_kind, precision, recheck_tau, bits,
                        logits_or_null, stats_or_null, ws, (size_t)HS_NOALLOC_SCRATCH_BYTES,
                        stream);
}

// Page shapes: every page at least 1 x 1 and the total under 2^31 pixels.
static bool pages_ok(int npages, const int32_t* shapes, size_t* N) {
  if (npages < 1 || !shapes) return false;
  long long n = 0;
  for (int p = 0; p < npages; ++p) {
    if (shapes[2 * p] < 1 || shapes[2 * p + 1] < 1) return false;
    n += (long long)shapes[2 * p] * shapes[2 * p + 1];
    if (n >= (1ll << 31)) return false;
  }
  *N = (size_t)n;
  return true;
}

size_t halftone_infer_pages_workspace_size(int npages, const int32_t* shapes_host,
                                           int precision) {
  size_t N = 0;
  if (!pages_ok(npages, shapes_host, &N)) return 0;
  if (precision != HS_FP32) return bf16_ws(shapes_host, npages, N, nullptr, nullptr);
  size_t m = 0;  // the FP32 path runs page by page
  for (int p = 0; p < npages; ++p) {
    const size_t b = fp32_ws(1, shapes_host[2 * p], shapes_host[2 * p + 1], nullptr, nullptr,
                             nullptr);
    if (b > m) m = b;
  }
  return m;
}

// pp: packed weights (a packed policy) or null; tau16, tau2 < 0: the default
// rules.
static int infer_pages(const float* weights, const Packed* pp, const float* contone,
                       const uint64_t* seeds, int npages, const int32_t* shapes_host, int levels,
                       int noise_kind, int precision, float recheck_tau, float tau16, float tau2,
                       uint8_t* out,
                       float* logits_or_null, int32_t* stats_or_null, void* workspace,
                       size_t workspace_bytes, void* stream, const char* who,
                       bool fp8_ok = false) {
  int rc = check_infer_args(weights, contone, seeds, out, workspace, noise_kind, precision,
                            recheck_tau, who, fp8_ok);
  if (rc) return rc;
  if (levels < 2 || levels > HS_MAX_LEVELS)
    return fail(HS_EINVAL, "%s: levels %d (2..%d)", who, levels, HS_MAX_LEVELS);
  size_t N = 0;
  if (!pages_ok(npages, shapes_host, &N))
    return fail(HS_ESHAPE, "%s: bad page shapes or more than 2^31 pixels", who);
  if (workspace_bytes < halftone_infer_pages_workspace_size(npages, shapes_host, precision))
    return fail(HS_EWORKSPACE, "%s: workspace too small", who);
  if ((rc = check_device())) return rc;
  hipStream_t s = (hipStream_t)stream;
  const Levels lv = make_levels(levels);
  const int kind = noise_kind & ~HS_CHECK_FINITE;
  if (precision != HS_FP32) {
    if (noise_kind & HS_CHECK_FINITE) {
      Bf16Ws w;
      bf16_ws(shapes_host, npages, N, &w, workspace);
      if ((rc = check_finite({{contone, N}}, w.cnt + CNT_FINITE, s, who))) return rc;
    }
    bool uniform = true;
    for (int p = 1; p < npages; ++p)
      uniform = uniform && shapes_host[2 * p] == shapes_host[0] &&
                shapes_host[2 * p + 1] == shapes_host[1];
    std::vector<Page> pages;
    if (!uniform) {  // a uniform batch's table is written on the device
      pages.resize(npages);
      long long off = 0, vstart = 0;
      for (int p = 0; p < npages; ++p) {
        const int H = shapes_host[2 * p], W = shapes_host[2 * p + 1];
        pages[p].off = off;
        pages[p].vstart = vstart;
        pages[p].H = H;
        pages[p].W = W;
        pages[p].nstrip = fused_strips(W);
        pages[p].pad = 0;
        off += (long long)H * W;
        vstart += (long long)fused_strips(W) * (H + fused_fill());
      }
    }
    return infer_bf16(weights, pp, contone, seeds, shapes_host, npages, N,
                      uniform ? nullptr : pages.data(), kind, recheck_tau,
                      tau16 < 0.0f ? default_tau16(recheck_tau) : tau16,
                      tau2 < 0.0f ? default_tau2(recheck_tau) : tau2, lv,
                      precision == HS_FP16 ? PASS_FP16
                                           : (precision == HS_FP8 ? PASS_FP8 : PASS_BF16),
                      out, logits_or_null, stats_or_null, workspace, s);
  }
  if (noise_kind & HS_CHECK_FINITE) {
    int* cnt;
    fp32_ws(1, shapes_host[0], shapes_host[1], nullptr, &cnt, workspace);
    if ((rc = check_finite({{contone, N}}, cnt + CNT_FINITE, s, who))) return rc;
  }
  if (stats_or_null) HS_TRY(launch_zero_ints(stats_or_null, NSTATS, s));
  if (pp) weights = pp->w;
  long long off = 0;
  for (int p = 0; p < npages; ++p) {
    const int H = shapes_host[2 * p], W = shapes_host[2 * p + 1];
    rc = infer_fp32(weights, pp ? pp->pack32 : nullptr, contone + off, seeds + p, 1, H, W, kind,
                    lv, out + off, logits_or_null ? logits_or_null + off : nullptr, workspace, s);
    if (rc) return rc;
    off += (long long)H * W;
  }
  return HS_OK;
}

int halftone_infer_pages(const float* weights, const float* contone, const uint64_t* seeds,
                         int npages, const int32_t* shapes_host, int noise_kind, int precision,
                         float recheck_tau, uint8_t* bits, float* logits_or_null,
                         int32_t* stats_or_null, void* workspace, size_t workspace_bytes,
                         void* stream) {
  return infer_pages(weights, nullptr, contone, seeds, npages, shapes_host, 2, noise_kind,
                     precision, recheck_tau, -1.0f, -1.0f, bits, logits_or_null, stats_or_null,
                     workspace, workspace_bytes, stream, "halftone_infer_pages");
}

int halftone_infer_levels(const float* weights, const float* contone, const uint64_t* seeds,
                          int npages, const int32_t* shapes_host, int levels, int noise_kind,
                          int precision, float recheck_tau, uint8_t* levels_out,
                          float* logits_or_null, int32_t* stats_or_null, void* workspace,
                          size_t workspace_bytes, void* stream) {
  return infer_pages(weights, nullptr, contone, seeds, npages, shapes_host, levels, noise_kind,
                     precision, recheck_tau, -1.0f, -1.0f, levels_out, logits_or_null,
                     stats_or_null, workspace, workspace_bytes, stream, "halftone_infer_levels");
}

// ------------------------------------------------------ packed policies --
size_t halftone_policy_bytes(void) { return policy_layout(nullptr, nullptr); }

int halftone_policy_pack(hs_policy* policy, const float* weights, void* mem, size_t bytes,
                         int flags, void* stream) {
  if (!policy || !weights || !mem) return fail(HS_EINVAL, "halftone_policy_pack: null pointer");
  if (flags & ~HS_CHECK_FINITE) return fail(HS_EINVAL, "halftone_policy_pack: flags 0x%x", flags);
  if ((uintptr_t)mem & 255) return fail(HS_EINVAL, "halftone_policy_pack: mem not 256-byte aligned");
  if (bytes < halftone_policy_bytes())
    return fail(HS_EWORKSPACE, "halftone_policy_pack: %zu bytes, %zu needed", bytes,
                halftone_policy_bytes());
  int rc = check_device();
  if (rc) return rc;
  hipStream_t s = (hipStream_t)stream;
  policy->packed = 0;
  Packed pk;
  policy_layout(mem, &pk);
  if ((flags & HS_CHECK_FINITE) &&
      (rc = check_finite({{weights, (size_t)NPARAM}}, pk.needs_all + 8, s, "halftone_policy_pack")))
    return rc;
  HS_TRY(hipMemcpyAsync(pk.w, weights, (size_t)NPARAM * 4, hipMemcpyDeviceToDevice, s));
  const PackPrologue none{nullptr, 0, nullptr, 0, nullptr, 0, 0, 0};
  HS_TRY(launch_zero_ints(pk.needs_all, 64, s));
  HS_TRY(launch_fused_pack(pk.w, pk.frags, pk.frags16, pk.needs_all, none, s));
  HS_TRY(launch_split_pack(pk.w, cone_weights(pk.split, pk.needs_all + 16), s));
  HS_TRY(launch_pack32(pk.w, pk.pack32, HS_FP32, 0, s));
  policy->mem = mem;
  policy->bytes = bytes;
  policy->packed = 1;
  policy->fp8 = 0;
  return HS_OK;
}

// Activation scales of the FP8 pass: s_k = 2^e, the smallest power of two
// with FP8_HEADROOM * act_max[k] <= 448 s_k, so an image may reach 4 times
// the calibration maximum before the pass saturates (it then runs again in
// BF16). Values below 2^-6 s_k lose precision as E4M3 subnormals, but their
// absolute error (at most 2^-10 s_k, under 1e-4 of the maximum) stays far
// below that of the largest values.
constexpr float FP8_HEADROOM = 4.0f;

int halftone_policy_set_fp8(hs_policy* policy, const float* act_max_host, void* stream) {
  if (!policy || !policy->packed || !policy->mem)
    return fail(HS_EINVAL, "halftone_policy_set_fp8: policy not packed");
  if (!act_max_host) return fail(HS_EINVAL, "halftone_policy_set_fp8: null act_max");
  int ex[4];
  for (int k = 0; k < 4; ++k) {
    const float m = act_max_host[k];
    if (!(m >= 0.0f) || !std::isfinite(m) || m > 1e15f)
      return fail(HS_EINVAL, "halftone_policy_set_fp8: act_max[%d] = %g", k, (double)m);
    int e = 0;
    if (m > 0.0f) {
      const double need = (double)FP8_HEADROOM * m / 448.0;
      e = (int)std::ceil(std::log2(need));
      while (std::ldexp(448.0, e - 1) >= FP8_HEADROOM * (double)m) --e;
      while (std::ldexp(448.0, e) < FP8_HEADROOM * (double)m) ++e;
      e = std::max(-60, std::min(60, e));
    }
    ex[k] = e;
  }
  int rc = check_device();
  if (rc) return rc;
  Packed pk;
  policy_layout(policy->mem, &pk);
  policy->fp8 = 0;
  HS_TRY(launch_fp8_pack(pk.w, pk.frags8, ex, (hipStream_t)stream));
  policy->fp8 = 1;
  return HS_OK;
}

int halftone_layer_max(const float* weights, const float* contone, const uint64_t* seeds, int B,
                       int H, int W, int noise_kind, float* layer_max, void* workspace,
                       size_t workspace_bytes, void* stream) {
  if (!weights || !contone || !seeds || !layer_max || !workspace)
    return fail(HS_EINVAL, "halftone_layer_max: null pointer");
  if (noise_kind != HS_NOISE_GAUSS && noise_kind != HS_NOISE_UNIFORM)
    return fail(HS_EINVAL, "halftone_layer_max: noise kind %d", noise_kind);
  if (!shape_ok(B, H, W))
    return fail(HS_ESHAPE, "halftone_layer_max: bad shape %d x %d x %d", B, H, W);
  if (workspace_bytes < halftone_infer_workspace_size(B, H, W, HS_FP32))
    return fail(HS_EWORKSPACE, "halftone_layer_max: workspace too small");
  int rc = check_device();
  if (rc) return rc;
  hipStream_t s = (hipStream_t)stream;
  InferWs iw;
  fp32_ws(B, H, W, &iw, nullptr, workspace);
  const size_t n = (size_t)B * H * W * 32;
  const size_t per_layer = (size_t)PACK32_PER_LAYER * 4;
  HS_TRY(launch_zero_ints((int*)layer_max, 5, s));
  HS_TRY(launch_pack32(weights, iw.pack, HS_FP32, 0, s));
  HS_TRY(launch_conv_first(contone, seeds, weights, B, H, W, noise_kind, 0u, HS_FP32, iw.a0,
                           nullptr, nullptr, s));
  HS_TRY(launch_layer_max((const float*)iw.a0, n, layer_max, s));
  void* src = iw.a0;
  void* dst = iw.a1;
  for (int k = 2; k <= 5; ++k) {
    HS_TRY(launch_conv32(src, (const char*)iw.pack + (k - 2) * per_layer, weights + hs_bk(k),
                         nullptr, dst, B, H, W, HS_FP32, 0, s));
    HS_TRY(launch_layer_max((const float*)dst, n, layer_max + (k - 1), s));
    std::swap(src, dst);
  }
  return HS_OK;
}

int halftone_policy_infer(const hs_policy* policy, const float* contone, const uint64_t* seeds,
                          int npages, const int32_t* shapes_host, int levels, int noise_kind,
                          int precision, float recheck_tau, float recheck_tau16,
                          float recheck_tau2, uint8_t* out, float* logits_or_null,
                          int32_t* stats_or_null, void* workspace, size_t workspace_bytes,
                          void* stream) {
  if (!policy || !policy->packed || !policy->mem)
    return fail(HS_EINVAL, "halftone_policy_infer: policy not packed");
  if (!(recheck_tau2 >= 0.0f) && recheck_tau2 != -1.0f)
    return fail(HS_EINVAL, "halftone_policy_infer: recheck_tau2 must be >= 0 or -1");
  if (!(recheck_tau16 >= 0.0f) && recheck_tau16 != -1.0f)
    return fail(HS_EINVAL, "halftone_policy_infer: recheck_tau16 must be >= 0 or -1");
  Packed pk;
  policy_layout(policy->mem, &pk);
  return infer_pages(pk.w, &pk, contone, seeds, npages, shapes_host, levels, noise_kind,
                     precision, recheck_tau, recheck_tau16, recheck_tau2, out, logits_or_null,
                     stats_or_null, workspace, workspace_bytes, stream, "halftone_policy_infer",
                     policy->fp8 == 1);
}

// ------------------------------------------------------- policy fwd / bwd --
size_t halftone_policy_workspace_size(int B, int H, int W, int precision) {
  if (!shape_ok(B, H, W)) return 0;
  Carve cv(nullptr);
  carve_policy(cv, (size_t)B * H * W, precision);
  return cv.off;
}

int halftone_policy_forward(const float* weights, const float* contone, const uint64_t* seeds,
                            int B, int H, int W, int noise_kind, uint32_t step, int precision,
                            float* probs, void* workspace, size_t workspace_bytes, void* stream) {
  if (!weights || !contone || !seeds || !probs || !workspace)
    return fail(HS_EINVAL, "halftone_policy_forward: null pointer");
  if (!shape_ok(B, H, W)) return fail(HS_ESHAPE, "halftone_policy_forward: bad shape");
  if (precision != HS_FP32 && precision != HS_BF16)
    return fail(HS_EUNSUPPORTED, "halftone_policy_forward: precision %d", precision);
  if (noise_kind != HS_NOISE_GAUSS && noise_kind != HS_NOISE_UNIFORM)
    return fail(HS_EINVAL, "halftone_policy_forward: noise kind %d", noise_kind);
  if (workspace_bytes < halftone_policy_workspace_size(B, H, W, precision))
    return fail(HS_EWORKSPACE, "halftone_policy_forward: workspace too small");
  int rc = check_device();
  if (rc) return rc;
  Carve cv(workspace);
  PolicyWs pw = carve_policy(cv, (size_t)B * H * W, precision);
  HS_TRY(run_forward_train(weights, contone, seeds, B, H, W, noise_kind, step, precision, pw,
                           probs, nullptr, 2, (hipStream_t)stream));
  return HS_OK;
}

int halftone_policy_backward(const float* weights, const float* grad_probs, const float* probs,
                             int B, int H, int W, int precision, float* grad_weights,
                             void* workspace, size_t workspace_bytes, void* stream) {
  if (!weights || !grad_probs || !probs || !grad_weights || !workspace)
    return fail(HS_EINVAL, "halftone_policy_backward: null pointer");
  if (!shape_ok(B, H, W)) return fail(HS_ESHAPE, "halftone_policy_backward: bad shape");
  if (precision != HS_FP32 && precision != HS_BF16)
    return fail(HS_EUNSUPPORTED, "halftone_policy_backward: precision %d", precision);
  if (workspace_bytes < halftone_policy_workspace_size(B, H, W, precision))
    return fail(HS_EWORKSPACE, "halftone_policy_backward: workspace too small");
  int rc = check_device();
  if (rc) return rc;
  hipStream_t s = (hipStream_t)stream;
  Carve cv(workspace);
  PolicyWs pw = carve_policy(cv, (size_t)B * H * W, precision);
  HS_TRY(run_backward(weights, grad_probs, probs, B, H, W, precision, pw, 0, s));
  HS_TRY(launch_reduce_partials(pw.partials, WGRAD_BLOCKS,
                                precision == HS_BF16 ? bwd32_grid(num_cus()) : WGRAD_BLOCKS,
                                pw.rtmp, grad_weights, s));
  return HS_OK;
}

// ------------------------------------------------------------------ loss --
static int check_loss_args(const uint8_t* actions, const float* contone, int B, int H, int W,
                           const float* pg, int Bg, int Hg, int Wg, const hs_loss_params* prm,
                           const char* who) {
  if (!actions || !contone) return fail(HS_EINVAL, "%s: null pointer", who);
  int rc = check_params(prm);
  if (rc) return rc;
  const int m = margin(prm);
  if (!shape_ok(B, H, W) || H < 2 * m + 1 || W < 2 * m + 1)
    return fail(HS_ESHAPE, "%s: images must be at least %d x %d", who, 2 * m + 1, 2 * m + 1);
  if (pg) {
    if (!shape_ok(Bg, Hg, Wg)) return fail(HS_ESHAPE, "%s: bad gray-batch shape", who);
  } else if (Bg != 0) {
    return fail(HS_EINVAL, "%s: Bg > 0 with a null gray batch", who);
  }
  return HS_OK;
}

size_t halftone_loss_workspace_size(int B, int H, int W, int Bg, int Hg, int Wg,
                                    const hs_loss_params* prm) {
  if (!prm || !shape_ok(B, H, W)) return 0;
  Carve cv(nullptr);
  carve_loss(cv, B, H, W, Bg, Hg, Wg, margin(prm), true);
  return cv.off;
}

int halftone_loss(const uint8_t* actions, const float* contone, int B, int H, int W,
                  const float* probs_gray_or_null, int Bg, int Hg, int Wg,
                  const hs_loss_params* prm, float* out, void* workspace, size_t workspace_bytes,
                  void* stream) {
  int rc = check_loss_args(actions, contone, B, H, W, probs_gray_or_null, Bg, Hg, Wg, prm,
                           "halftone_loss");
  if (rc) return rc;
  if (!out || !workspace) return fail(HS_EINVAL, "halftone_loss: null pointer");
  if (!probs_gray_or_null) Bg = Hg = Wg = 0;
  if (workspace_bytes < halftone_loss_workspace_size(B, H, W, Bg, Hg, Wg, prm))
    return fail(HS_EWORKSPACE, "halftone_loss: workspace too small");
  if ((rc = check_device())) return rc;
  hipStream_t s = (hipStream_t)stream;
  const int m = margin(prm);
  Carve cv(workspace);
  LossWs lw = carve_loss(cv, B, H, W, Bg, Hg, Wg, m, true);
  if ((prm->flags & HS_CHECK_FINITE) &&
      (rc = check_finite({{contone, (size_t)B * H * W}, {probs_gray_or_null, (size_t)Bg * Hg * Wg}},
                         lw.flag, s, "halftone_loss")))
    return rc;
  LossDev win;
  make_windows(*prm, &win);
  HS_TRY(launch_loss_stats(actions, contone, B, H, W, *prm, win, nullptr, lw.tiles, lw.ntiles, s));
  const int npatch = Bg * (Hg / 32) * (Wg / 32);
  if (npatch > 0)
    HS_TRY(launch_as(probs_gray_or_null, Bg, Hg, Wg, 1.0f, 0, lw.patches, nullptr, s));
  HS_TRY(launch_loss_reduce(lw.tiles, B, lw.ntiles, lw.patches, npatch, prm->w_s,
                            (long)(H - 2 * m) * (W - 2 * m), out, s));
  HS_TRY(launch_loss_total(B, prm->w_a, out, s));
  return HS_OK;
}

int halftone_loss_backward(const uint8_t* actions, const float* contone,
                           const float* probs_or_null, int B, int H, int W,
                           const float* probs_gray_or_null, int Bg, int Hg, int Wg,
                           const hs_loss_params* prm, int grad_space, float* grad_probs,
                           float* grad_probs_gray_or_null, void* workspace,
                           size_t workspace_bytes, void* stream) {
  int rc = check_loss_args(actions, contone, B, H, W, probs_gray_or_null, Bg, Hg, Wg, prm,
                           "halftone_loss_backward");
  if (rc) return rc;
  if (!grad_probs || !workspace) return fail(HS_EINVAL, "halftone_loss_backward: null pointer");
  if (grad_space != HS_WRT_PROB && grad_space != HS_WRT_LOGIT)
    return fail(HS_EINVAL, "halftone_loss_backward: grad_space %d", grad_space);
  if (grad_space == HS_WRT_LOGIT && !probs_or_null)
    return fail(HS_EINVAL, "halftone_loss_backward: logit space needs probs");
  if (prm->estimator == HS_EST_COMA && !probs_or_null)
    return fail(HS_EINVAL, "halftone_loss_backward: the COMA estimator needs probs");
  if (prm->levels > 2 && !probs_or_null)
    return fail(HS_EINVAL, "halftone_loss_backward: multitone levels need probs");
  if (probs_gray_or_null && !grad_probs_gray_or_null)
    return fail(HS_EINVAL, "halftone_loss_backward: gray batch without its gradient buffer");
  if (!probs_gray_or_null) Bg = Hg = Wg = 0;
  if (workspace_bytes < halftone_loss_workspace_size(B, H, W, Bg, Hg, Wg, prm))
    return fail(HS_EWORKSPACE, "halftone_loss_backward: workspace too small");
  if ((rc = check_device())) return rc;
  hipStream_t s = (hipStream_t)stream;
  const int m = margin(prm);
  Carve cv(workspace);
  LossWs lw = carve_loss(cv, B, H, W, Bg, Hg, Wg, m, true);
  if ((prm->flags & HS_CHECK_FINITE) &&
      (rc = check_finite({{contone, (size_t)B * H * W},
                          {probs_or_null, probs_or_null ? (size_t)B * H * W : 0},
                          {probs_gray_or_null, (size_t)Bg * Hg * Wg}},
                         lw.flag, s, "halftone_loss_backward")))
    return rc;
  LossDev win;
  make_windows(*prm, &win);
  HS_TRY(launch_loss_stats(actions, contone, B, H, W, *prm, win, lw.maps, lw.tiles, lw.ntiles, s));
  HS_TRY(launch_le_grad(actions, contone, probs_or_null, grad_space == HS_WRT_LOGIT, B, H, W,
                        *prm, win, lw.maps, grad_probs, s));
  if (probs_gray_or_null) {
    const int npatch = Bg * (Hg / 32) * (Wg / 32);
    HS_TRY(launch_fill(grad_probs_gray_or_null, (size_t)Bg * Hg * Wg, 0.0f, s));
    if (npatch > 0)
      HS_TRY(launch_as(probs_gray_or_null, Bg, Hg, Wg, prm->w_a / (float)npatch,
                       grad_space == HS_WRT_LOGIT, lw.patches, grad_probs_gray_or_null, s));
  }
  return HS_OK;
}

// ------------------------------------------------------------ train step --
// The second stream of a device (default priority, non-blocking) and the two
// events that fork the gray side batch onto it and join it back; created on
// first use, kept until the process ends. The mutex keeps each caller's
// record / wait / launch sequence on them whole.
struct SideStream {
  hipStream_t s = nullptr;
  hipEvent_t fork = nullptr, join = nullptr, stats = nullptr;
  std::mutex mu;
};
static int side_stream(SideStream** out) {
  static std::mutex mu;
  static std::vector<SideStream*> per_dev;
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return fail(HS_EHIP, "hipGetDevice failed");
  std::lock_guard<std::mutex> lk(mu);
  if ((int)per_dev.size() <= dev) per_dev.resize(dev + 1, nullptr);
  if (!per_dev[dev]) {
    SideStream* ss = new SideStream;
    if (hipStreamCreateWithFlags(&ss->s, hipStreamNonBlocking) != hipSuccess ||
        hipEventCreateWithFlags(&ss->fork, hipEventDisableTiming) != hipSuccess ||
        hipEventCreateWithFlags(&ss->join, hipEventDisableTiming) != hipSuccess ||
        hipEventCreateWithFlags(&ss->stats, hipEventDisableTiming) != hipSuccess) {
      delete ss;
      return fail(HS_EHIP, "policy_train_step: creating the side stream failed");
    }
    per_dev[dev] = ss;
  }
  *out = per_dev[dev];
  return HS_OK;
}

// The batch and the gray side batch have workspaces of their own, so that
// the side batch runs on a second stream beside the batch; the side batch's
// weight-gradient partial sums are the second WGRAD_BLOCKS rows.
static size_t train_ws(int B, int H, int W, int Bg, int Hg, int Wg, int prec, bool recompute,
                       void* base, PolicyWs* pw, PolicyWs* pwg, LossWs* lw, float** probs,
                       float** probs_g, uint8_t** act, float** gradp, float** gradg,
                       float** grad, float** loss_out) {
  Carve cv(base);
  const size_t N = (size_t)B * H * W, Ng = (size_t)Bg * Hg * Wg;
  PolicyWs p = carve_policy(cv, N, prec, recompute, nullptr, Ng ? 2 * WGRAD_BLOCKS : WGRAD_BLOCKS);
  PolicyWs q{};
  if (Ng) q = carve_policy(cv, Ng, prec, recompute, p.partials + (size_t)WGRAD_BLOCKS * NPARAM);
  // sized for the smallest margin (most tiles); the caller sets the real count
  LossWs l = carve_loss(cv, B, H, W, Bg, Hg, Wg, 1, true);
  float* pr = cv.take<float>(N * 4);
  float* pg = cv.take<float>((Ng ? Ng : 1) * 4);
  uint8_t* a = cv.take<uint8_t>(N);
  float* gp = cv.take<float>(N * 4);
  float* gg = cv.take<float>((Ng ? Ng : 1) * 4);
  float* g = cv.take<float>((size_t)NPARAM * 4);
  float* lo = cv.take<float>((size_t)(3 * B + 2) * 4);
  if (pw) *pw = p;
  if (pwg) *pwg = q;
  if (lw) *lw = l;
  if (probs) *probs = pr;
  if (probs_g) *probs_g = pg;
  if (act) *act = a;
  if (gradp) *gradp = gp;
  if (gradg) *gradg = gg;
  if (grad) *grad = g;
  if (loss_out) *loss_out = lo;
  return cv.off;
}

size_t halftone_train_workspace_size_params(int B, int H, int W, int Bg, int Hg, int Wg,
                                            int precision, const hs_train_params* tp) {
  if (!shape_ok(B, H, W) || Bg < 0) return 0;
  if (Bg > 0 && !shape_ok(Bg, Hg, Wg)) return 0;
  if (Bg == 0) Hg = Wg = 0;
  return train_ws(B, H, W, Bg, Hg, Wg, precision, tp && tp->recompute, nullptr, nullptr, nullptr,
                  nullptr, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr);
}

size_t halftone_train_workspace_size(int B, int H, int W, int Bg, int Hg, int Wg,
                                     int precision) {
  return halftone_train_workspace_size_params(B, H, W, Bg, Hg, Wg, precision, nullptr);
}

int policy_train_step(float* weights, float* adam_m, float* adam_v, const float* contones,
                      const uint64_t* seeds, int B, int H, int W, const float* gray,
                      const uint64_t* gray_seeds, int Bg, int Hg, int Wg, int64_t step,
                      int64_t total_steps, const hs_train_params* tp, int precision,
                      float* metrics, uint8_t* actions_out_or_null, float* grad_out_or_null,
                      void* workspace, size_t workspace_bytes, void* stream) {
  if (!weights || !adam_m || !adam_v || !contones || !seeds || !tp || !metrics || !workspace)
    return fail(HS_EINVAL, "policy_train_step: null pointer");
  if (precision != HS_FP32 && precision != HS_BF16)
    return fail(HS_EUNSUPPORTED, "policy_train_step: precision %d", precision);
  if (tp->noise_kind != HS_NOISE_GAUSS && tp->noise_kind != HS_NOISE_UNIFORM)
    return fail(HS_EINVAL, "policy_train_step: noise kind %d", tp->noise_kind);
  if (step < 0 || total_steps < 0) return fail(HS_EINVAL, "policy_train_step: negative step");
  if (gray && (!gray_seeds || Bg <= 0))
    return fail(HS_EINVAL, "policy_train_step: gray batch needs seeds and Bg > 0");
  if (!gray) Bg = Hg = Wg = 0;
  int rc = check_params(&tp->loss);
  if (rc) return rc;
  const int m = margin(&tp->loss);
  if (!shape_ok(B, H, W) || H < 2 * m + 1 || W < 2 * m + 1)
    return fail(HS_ESHAPE, "policy_train_step: images must be at least %d x %d", 2 * m + 1,
                2 * m + 1);
  if (Bg > 0 && !shape_ok(Bg, Hg, Wg))
    return fail(HS_ESHAPE, "policy_train_step: bad gray-batch shape");
  if (tp->recompute != 0 && tp->recompute != 1)
    return fail(HS_EINVAL, "policy_train_step: recompute %d", tp->recompute);
  if (workspace_bytes < halftone_train_workspace_size_params(B, H, W, Bg, Hg, Wg, precision, tp))
    return fail(HS_EWORKSPACE, "policy_train_step: workspace too small");
  if ((rc = check_device())) return rc;
  hipStream_t s = (hipStream_t)stream;
  PolicyWs pw, pwg;
  LossWs lw;
  float *probs, *probs_g, *gradp, *gradg, *grad, *loss_out;
  uint8_t* act;
  train_ws(B, H, W, Bg, Hg, Wg, precision, tp->recompute != 0, workspace, &pw, &pwg, &lw, &probs,
           &probs_g, &act, &gradp, &gradg, &grad, &loss_out);
  lw.ntiles = ((H - 2 * m + 15) / 16) * ((W - 2 * m + 15) / 16);
  const hs_loss_params& lp = tp->loss;
  if ((lp.flags & HS_CHECK_FINITE) &&
      (rc = check_finite({{contones, (size_t)B * H * W}, {gray, (size_t)Bg * Hg * Wg}}, lw.flag,
                         s, "policy_train_step")))
    return rc;
  const int kind = tp->noise_kind;
  const uint32_t st = (uint32_t)step;
  LossDev win;
  make_windows(lp, &win);
  // the layers' packed weights, forward and transposed, once for both batches
  HS_TRY(launch_pack32_both(weights, pw.packF, pw.packT, precision, s));
  pwg.packF = pw.packF;
  pwg.packT = pw.packT;
  SideStream* side = nullptr;
  std::unique_lock<std::mutex> side_lock;
  if (Bg > 0) {
    if ((rc = side_stream(&side))) return rc;
    side_lock = std::unique_lock<std::mutex>(side->mu);
    HS_TRY(hipEventRecord(side->fork, s));
  }
  // batch: forward and actions
  HS_TRY(run_forward_train(weights, contones, seeds, B, H, W, kind, st, precision, pw, probs, act,
                           lp.levels, s, false));
  // the constant-gray side batch (forward, anisotropy gradient, backward
  // into its own partial rows) on a second stream, forked before the
  // batch's forward and beside it and the batch's loss kernels; the batch
  // waits for it before the partial sums are added. The batch's forward and
  // loss kernels are launched first, so that its stream is not left idle
  // while the host issues the side batch's many small launches.
  const int npatch = Bg * (Hg / 32) * (Wg / 32);
  // batch: policy gradient (logit space)
  HS_TRY(launch_loss_stats(act, contones, B, H, W, lp, win, lw.maps, lw.tiles, lw.ntiles, s));
  if (Bg > 0) HS_TRY(hipEventRecord(side->stats, s));
  HS_TRY(launch_le_grad(act, contones, probs, 1, B, H, W, lp, win, lw.maps, gradp, s));
  const long M = (long)(H - 2 * m) * (W - 2 * m);
  const size_t nact = (size_t)B * H * W;
  // the rows of the 32->32 layers' weight-gradient partial sums per batch
  const int rows32 = precision == HS_BF16 ? bwd32_grid(num_cus()) : WGRAD_BLOCKS;
  if (Bg > 0) {
    // the second stream also takes the reported metrics' action count and
    // the loss sums (both after the batch's loss statistics), off the
    // batch's path
    HS_TRY(hipStreamWaitEvent(side->s, side->fork, 0));
    hipStream_t s2 = side->s;
    HS_TRY(run_forward_train(weights, gray, gray_seeds, Bg, Hg, Wg, kind, st, precision, pwg,
                             probs_g, nullptr, lp.levels, s2, false));
    HS_TRY(launch_fill(gradg, (size_t)Bg * Hg * Wg, 0.0f, s2));
    if (npatch > 0)
      HS_TRY(launch_as(probs_g, Bg, Hg, Wg, lp.w_a / (float)npatch, 1, lw.patches, gradg, s2));
    HS_TRY(hipStreamWaitEvent(s2, side->stats, 0));
    HS_TRY(launch_count_actions(act, nact, pw.counter, s2));
    HS_TRY(launch_loss_reduce(lw.tiles, B, lw.ntiles, lw.patches, npatch, lp.w_s, M, loss_out,
                              s2));
    const FwdInput gin{gray, gray_seeds, kind, st};
    HS_TRY(run_backward(weights, gradg, nullptr, Bg, Hg, Wg, precision, pwg, 0, s2, &gin, false));
    // its weight-gradient rows' group sums, beside the batch's backward
    HS_TRY(launch_reduce_rows(pwg.partials, WGRAD_BLOCKS, rows32, pwg.rtmp, s2));
    HS_TRY(hipEventRecord(side->join, s2));
  }
  // batch: backward
  const FwdInput fin{contones, seeds, kind, st};
  HS_TRY(run_backward(weights, gradp, nullptr, B, H, W, precision, pw, 0, s, &fin, false));
  HS_TRY(launch_reduce_rows(pw.partials, WGRAD_BLOCKS, rows32, pw.rtmp, s));
  if (Bg > 0) HS_TRY(hipStreamWaitEvent(s, side->join, 0));
  if (Bg == 0) {
    HS_TRY(launch_loss_reduce(lw.tiles, B, lw.ntiles, lw.patches, npatch, lp.w_s, M, loss_out,
                              s));
    HS_TRY(launch_count_actions(act, nact, pw.counter, s));
  }
  // Adam with the cosine learning rate of this step, bias corrections at t = step + 1
  const double T = (double)total_steps;
  const double lr = T > 0 ? tp->lr_min + 0.5 * ((double)tp->lr_max - tp->lr_min) *
                                             (1.0 + cos(M_PI * (double)step / T))
                          : (double)tp->lr_max;
  const double c1 = 1.0 - pow((double)tp->beta1, (double)(step + 1));
  const double c2 = 1.0 - pow((double)tp->beta2, (double)(step + 1));
  // the gradient (the batch's group sums, then the side batch's) and Adam
  float* gsq = pw.rtmp + (size_t)REDUCE_GROUPS * NPARAM;
  HS_TRY(launch_reduce_adam(pw.rtmp, Bg > 0 ? pwg.rtmp : nullptr, grad, gsq, weights, adam_m,
                            adam_v, (float)lr, tp->beta1, tp->beta2, tp->eps, (float)c1,
                            (float)c2, s));
  if (grad_out_or_null)
    HS_TRY(hipMemcpyAsync(grad_out_or_null, grad, (size_t)NPARAM * 4, hipMemcpyDeviceToDevice, s));
  HS_TRY(launch_train_metrics(loss_out, B, gsq, pw.counter, nact, lp.levels, (float)lr, lp.w_a,
                              metrics, s));
  if (actions_out_or_null)
    HS_TRY(hipMemcpyAsync(actions_out_or_null, act, (size_t)B * H * W, hipMemcpyDeviceToDevice, s));
  return HS_OK;
}

// ------------------------------------------------------------- spectrum --
int halftone_spectrum_rings(int P) { return (P == 32 || P == 64) ? spectrum_rings(P) : 0; }

static bool spectrum_shape_ok(int B, int H, int W, int P) {
  return (P == 32 || P == 64) && shape_ok(B, H, W) && H >= P && W >= P;
}

size_t halftone_spectrum_workspace_size(int B, int H, int W, int P) {
  if (!spectrum_shape_ok(B, H, W, P)) return 0;
  Carve cv(nullptr);
  cv.take<float>(spectrum_patches(B, H, W, P) * P * P * sizeof(float));
  cv.take<float>((size_t)P * P * sizeof(float));
  return cv.off;
}

int halftone_spectrum(const uint8_t* bits, int B, int H, int W, int P, float* rapsd_out,
                      float* anis_out, void* workspace, size_t workspace_bytes, void* stream) {
  if (P != 32 && P != 64) return fail(HS_EUNSUPPORTED, "halftone_spectrum: P=%d (32 or 64)", P);
  if (!spectrum_shape_ok(B, H, W, P))
    return fail(HS_ESHAPE, "halftone_spectrum: bad shape %dx%dx%d for P=%d", B, H, W, P);
  if (!bits || !rapsd_out || !anis_out || !workspace)
    return fail(HS_EINVAL, "halftone_spectrum: null pointer");
  if (workspace_bytes < halftone_spectrum_workspace_size(B, H, W, P))
    return fail(HS_EWORKSPACE, "halftone_spectrum: workspace too small");
  int rc = check_device();
  if (rc) return rc;
  Carve cv(workspace);
  float* spec = cv.take<float>(spectrum_patches(B, H, W, P) * P * P * sizeof(float));
  float* avg = cv.take<float>((size_t)P * P * sizeof(float));
  HS_TRY(launch_spectrum(bits, B, H, W, P, spec, avg, rapsd_out, anis_out, (hipStream_t)stream));
  return HS_OK;
}

// ---------------------------------------------------- host error diffusion --
int halftone_error_diffusion_host(const float* contone_host, int B, int H, int W,
                                  uint8_t* bits_host) {
  if (!contone_host || !bits_host) return fail(HS_EINVAL, "error diffusion: null pointer");
  if (!shape_ok(B, H, W)) return fail(HS_ESHAPE, "error diffusion: bad shape");
  // two rows of pending error (current and next), with one guard column each side
  std::vector<double> cur(W + 2), nxt(W + 2);
  for (int b = 0; b < B; ++b) {
    std::fill(cur.begin(), cur.end(), 0.0);
    std::fill(nxt.begin(), nxt.end(), 0.0);
    const float* c = contone_host + (size_t)b * H * W;
    uint8_t* h = bits_host + (size_t)b * H * W;
    for (int y = 0; y < H; ++y) {
      for (int x = 0; x < W; ++x) {
        const double v = (double)c[(size_t)y * W + x] + cur[x + 1];
        const uint8_t bit = v >= 0.5 ? 1 : 0;
        const double q = v - (double)bit;
        h[(size_t)y * W + x] = bit;
        if (x + 1 < W) cur[x + 2] += q * (7.0 / 16.0);
        if (x > 0) nxt[x] += q * (3.0 / 16.0);
        nxt[x + 1] += q * (5.0 / 16.0);
        if (x + 1 < W) nxt[x + 2] += q * (1.0 / 16.0);
      }
      std::swap(cur, nxt);
      std::fill(nxt.begin(), nxt.end(), 0.0);
    }
  }
  return HS_OK;
}

int halftone_error_diffusion_levels_host(const float* contone_host, int B, int H, int W,
                                         int levels, uint8_t* levels_host) {
  if (!contone_host || !levels_host) return fail(HS_EINVAL, "error diffusion: null pointer");
  if (!shape_ok(B, H, W)) return fail(HS_ESHAPE, "error diffusion: bad shape");
  if (levels < 2 || levels > HS_MAX_LEVELS)
    return fail(HS_EINVAL, "error diffusion: levels %d (2..%d)", levels, HS_MAX_LEVELS);
  const double step = 1.0 / (levels - 1);
  std::vector<double> cur(W + 2), nxt(W + 2);
  for (int b = 0; b < B; ++b) {
    std::fill(cur.begin(), cur.end(), 0.0);
    std::fill(nxt.begin(), nxt.end(), 0.0);
    const float* c = contone_host + (size_t)b * H * W;
    uint8_t* k = levels_host + (size_t)b * H * W;
    for (int y = 0; y < H; ++y) {
      for (int x = 0; x < W; ++x) {
        const double v = (double)c[(size_t)y * W + x] + cur[x + 1];
        int lev = (int)floor(v * (levels - 1) + 0.5);
        lev = lev < 0 ? 0 : (lev > levels - 1 ? levels - 1 : lev);
        const double q = v - lev * step;
        k[(size_t)y * W + x] = (uint8_t)lev;
        if (x + 1 < W) cur[x + 2] += q * (7.0 / 16.0);
        if (x > 0) nxt[x] += q * (3.0 / 16.0);
        nxt[x + 1] += q * (5.0 / 16.0);
        if (x + 1 < W) nxt[x + 2] += q * (1.0 / 16.0);
      }
      std::swap(cur, nxt);
      std::fill(nxt.begin(), nxt.end(), 0.0);
    }
  }
  return HS_OK;
}

}  // extern "C"
