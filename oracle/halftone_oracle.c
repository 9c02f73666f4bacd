/*
 * halftone_oracle.c -- plain, slow, double-precision CPU oracle for the
 * halftoning method of "Efficient Halftoning via Deep Reinforcement
 * Learning" (Jiang et al., IEEE TIP; arXiv 2304.12152).
 *
 * TEST INFRASTRUCTURE ONLY. The test-suite, the smoke check and the
 * benchmark's CPU-baseline leg are the only users of this file. The HIP
 * product library shares no code, header, table or helper with it.
 *
 * Everything below is the plain definition of each step: nested loops in
 * natural order, FP64, no blocking, no fusion, no reordering. Each function
 * names the passage of the paper it follows. Where the paper is silent the
 * reading taken is stated next to the code.
 *
 * Layout conventions (shared with the product only through the documented
 * interface, never through code):
 *   - images are row-major [B][H][W]; within image b, pixel a = y*W + x;
 *   - 1 = white (Sec. VI-A: the sigmoid outputs the probability of white);
 *   - policy weights are one flat array, layer after layer, each layer being
 *     W[cout][cin][3][3] followed by bias[cout].
 */
#include <math.h>
#include <pthread.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#ifndef M_PI
#define M_PI 3.14159265358979323846
#endif

/* ------------------------------------------------------------------------
 * Counter-based random numbers: Philox4x32 with 10 rounds, written from the
 * published definition (Salmon, Moraes, Dror and Shaw, "Parallel random
 * numbers: as easy as 1, 2, 3", SC'11). Each round multiplies counter words
 * 0 and 2 by two fixed odd constants, swaps the halves and folds in the key;
 * the key is advanced by the Weyl increments between rounds.
 *
 * The paper draws its noise map and actions from torch's generator; keying
 * the draws by (seed, pixel, stream, step) is this project's reading, so
 * that every draw can be replayed on either side independently.
 * ---------------------------------------------------------------------- */
void or_philox4x32_10(const uint32_t ctr_in[4], const uint32_t key_in[2],
                      uint32_t out[4]) {
  uint32_t c0 = ctr_in[0], c1 = ctr_in[1], c2 = ctr_in[2], c3 = ctr_in[3];
  uint32_t k0 = key_in[0], k1 = key_in[1];
  for (int round = 0; round < 10; ++round) {
    if (round > 0) {
      k0 += 0x9E3779B9u;
      k1 += 0xBB67AE85u;
    }
    uint64_t p0 = (uint64_t)0xD2511F53u * (uint64_t)c0;
    uint64_t p1 = (uint64_t)0xCD9E8D57u * (uint64_t)c2;
    uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
    uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
    uint32_t n0 = hi1 ^ c1 ^ k0;
    uint32_t n1 = lo1;
    uint32_t n2 = hi0 ^ c3 ^ k1;
    uint32_t n3 = lo0;
    c0 = n0; c1 = n1; c2 = n2; c3 = n3;
  }
  out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

static void draw_words(uint64_t seed, uint64_t a, uint32_t stream,
                       uint32_t step, uint32_t w[4]) {
  uint32_t ctr[4] = {(uint32_t)a, (uint32_t)(a >> 32), stream, step};
  uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
  or_philox4x32_10(ctr, key, w);
}

/* u in [0,1): the top 24 bits of word 0, scaled by 2^-24 (exact in FP32). */
double or_uniform(uint64_t seed, uint64_t a, uint32_t stream, uint32_t step) {
  uint32_t w[4];
  draw_words(seed, a, stream, step, w);
  return (double)(w[0] >> 8) * (1.0 / 16777216.0);
}

/* Standard normal by the Box-Muller transform (Box and Muller, 1958):
 * u1 in (0,1] from word 0, u2 in [0,1) from word 1,
 * z = sqrt(-2 ln u1) cos(2 pi u2). */
double or_normal(uint64_t seed, uint64_t a, uint32_t stream, uint32_t step) {
  uint32_t w[4];
  draw_words(seed, a, stream, step, w);
  double u1 = (double)((w[0] >> 8) + 1u) * (1.0 / 16777216.0);
  double u2 = (double)(w[1] >> 8) * (1.0 / 16777216.0);
  return sqrt(-2.0 * log(u1)) * cos(2.0 * M_PI * u2);
}

/* Noise map z of the state s = concat(c, z) (Sec. III, "State"): white
 * Gaussian by default (kind 0); kind 1 is the uniform U(0,1) variant of the
 * noise-type study (Sec. VI-D). Stream 1 by convention. */
void or_noise_map(const uint64_t* seeds, int B, int H, int W, int kind,
                  uint32_t stream, uint32_t step, double* z) {
  for (int b = 0; b < B; ++b)
    for (int y = 0; y < H; ++y)
      for (int x = 0; x < W; ++x) {
        uint64_t a = (uint64_t)y * (uint64_t)W + (uint64_t)x;
        double v = kind == 0 ? or_normal(seeds[b], a, stream, step)
                             : or_uniform(seeds[b], a, stream, step);
        z[((size_t)b * H + y) * W + x] = v;
      }
}

/* Stochastic actions of the agents, h_a ~ Bernoulli(pi_a(h=1))
 * (Eq. independent; Algorithm 1, TRAIN): h_a = [u_a < p_a], stream 0. */
void or_bernoulli(const double* p, const uint64_t* seeds, int B, int H, int W,
                  uint32_t step, uint8_t* h) {
  for (int b = 0; b < B; ++b)
    for (int y = 0; y < H; ++y)
      for (int x = 0; x < W; ++x) {
        uint64_t a = (uint64_t)y * (uint64_t)W + (uint64_t)x;
        size_t i = ((size_t)b * H + y) * W + x;
        h[i] = or_uniform(seeds[b], a, 0, step) < p[i] ? 1 : 0;
      }
}

/* ------------------------------------------------------------------------
 * Optional threads, for speed only. or_set_threads(n) lets the channel loops
 * of the conv stack (forward: output channels; backward: output channels for
 * the weight gradient, input channels for the input gradient) run on n POSIX
 * threads. Each thread owns whole output elements and adds their terms in the
 * order of the serial loop, so every result is bit-identical for any n. The
 * default is one thread.
 * ---------------------------------------------------------------------- */
static int g_threads = 1;

void or_set_threads(int n) { g_threads = n < 1 ? 1 : (n > 256 ? 256 : n); }
int or_get_threads(void) { return g_threads; }

typedef void (*range_fn)(int lo, int hi, void* ctx);
typedef struct { range_fn fn; void* ctx; int lo, hi; } range_job;

static void* run_range(void* p) {
  range_job* j = (range_job*)p;
  j->fn(j->lo, j->hi, j->ctx);
  return NULL;
}

/* fn over [0, n) split into contiguous ranges, one per thread; a range whose
 * thread cannot be started runs on the calling thread */
static void parallel_ranges(int n, range_fn fn, void* ctx) {
  int T = g_threads < n ? g_threads : n;
  if (T <= 1) {
    fn(0, n, ctx);
    return;
  }
  pthread_t* tid = (pthread_t*)malloc(sizeof(pthread_t) * T);
  range_job* job = (range_job*)malloc(sizeof(range_job) * T);
  int* started = (int*)calloc(T, sizeof(int));
  for (int t = 0; t < T; ++t) {
    job[t].fn = fn;
    job[t].ctx = ctx;
    job[t].lo = (int)((long)n * t / T);
    job[t].hi = (int)((long)n * (t + 1) / T);
    if (t > 0) started[t] = pthread_create(&tid[t], NULL, run_range, &job[t]) == 0;
  }
  fn(job[0].lo, job[0].hi, ctx);
  for (int t = 1; t < T; ++t) {
    if (started[t]) pthread_join(tid[t], NULL);
    else fn(job[t].lo, job[t].hi, ctx);
  }
  free(tid);
  free(job);
  free(started);
}

/* ------------------------------------------------------------------------
 * Policy network (Sec. VI-A "Details of Our Method"; Sec. III "Agents"):
 * a fully convolutional stack of 3x3 convolutions, stride 1, zero 'same'
 * padding, with bias, ReLU after every layer but the last, and a pixel-wise
 * sigmoid on the last layer's single channel giving pi_a(h=1).
 * ch[0..L] are the channel counts; ch[0] = 2 for the state (c, z).
 * ---------------------------------------------------------------------- */
long or_param_count(const int* ch, int L) {
  long n = 0;
  for (int l = 0; l < L; ++l) n += (long)ch[l + 1] * ch[l] * 9 + ch[l + 1];
  return n;
}

static long layer_offset(const int* ch, int l) {
  long n = 0;
  for (int k = 0; k < l; ++k) n += (long)ch[k + 1] * ch[k] * 9 + ch[k + 1];
  return n;
}

typedef struct { int y0, y1, x0, x1; } region;

static region grow(region r, int m, int H, int W) {
  region g = {r.y0 - m, r.y1 + m, r.x0 - m, r.x1 + m};
  if (g.y0 < 0) g.y0 = 0;
  if (g.x0 < 0) g.x0 = 0;
  if (g.y1 > H) g.y1 = H;
  if (g.x1 > W) g.x1 = W;
  return g;
}

/* One conv layer of the stack, output channels [o0, o1): out[o](y, x) =
 * b[o] + sum_{i, dy, dx} W[o][i][dy][dx] s_i(y + dy - 1, x + dx - 1), zero
 * outside the image, then the ReLU (all layers but the last). `prev` holds
 * the input on region prev_r (ph x pw), `cur` the output on region r. */
typedef struct {
  const double *Wk, *bk, *prev;
  double* cur;
  int ci_n, relu, H, W;
  region r, prev_r;
  int ph, pw;
} conv_layer;

static void conv_channels(int o0, int o1, void* ctx) {
  const conv_layer* c = (const conv_layer*)ctx;
  const double* Wk = c->Wk;
  const double* bk = c->bk;
  const double* prev = c->prev;
  double* cur = c->cur;
  const int ci_n = c->ci_n, H = c->H, W = c->W, ph = c->ph, pw = c->pw;
  const region r = c->r, prev_r = c->prev_r;
  const int rh = r.y1 - r.y0, rw = r.x1 - r.x0;
  for (int o = o0; o < o1; ++o)
    for (int y = 0; y < rh; ++y)
      for (int x = 0; x < rw; ++x) {
        double acc = bk[o];
        int gy = r.y0 + y, gx = r.x0 + x;
        for (int i = 0; i < ci_n; ++i)
          for (int dy = 0; dy < 3; ++dy)
            for (int dx = 0; dx < 3; ++dx) {
              int sy = gy + dy - 1, sx = gx + dx - 1;
              if (sy < 0 || sy >= H || sx < 0 || sx >= W) continue;
              double s = prev[((size_t)i * ph + (sy - prev_r.y0)) * pw + (sx - prev_r.x0)];
              acc += Wk[(((size_t)o * ci_n + i) * 3 + dy) * 3 + dx] * s;
            }
        if (c->relu && acc < 0.0) acc = 0.0; /* ReLU */
        cur[((size_t)o * rh + y) * rw + x] = acc;
      }
}

/* One image. Layer k (1..L) is evaluated on the output region grown by
 * (L - k) pixels and clipped to the image, so every value a later layer reads
 * inside the image has been computed; reads outside the image are the zero
 * padding. If `keep` is non-null (only for the full image) the output of
 * each layer k is copied to keep[k-1] as [ch[k]][H][W] (post-ReLU; the last
 * one is the logit map). */
static void forward_one(const double* w, const int* ch, int L,
                        const double* c, const double* z, int H, int W,
                        region out, double* logits, double** keep) {
  region prev_r = grow(out, L, H, W);
  int ph = prev_r.y1 - prev_r.y0, pw = prev_r.x1 - prev_r.x0;
  double* prev = (double*)malloc(sizeof(double) * 2 * (size_t)ph * pw);
  for (int y = 0; y < ph; ++y)
    for (int x = 0; x < pw; ++x) {
      size_t src = (size_t)(prev_r.y0 + y) * W + (prev_r.x0 + x);
      prev[(size_t)y * pw + x] = c[src];
      prev[(size_t)ph * pw + (size_t)y * pw + x] = z[src];
    }
  for (int k = 1; k <= L; ++k) {
    region r = grow(out, L - k, H, W);
    int rh = r.y1 - r.y0, rw = r.x1 - r.x0;
    int ci_n = ch[k - 1], co_n = ch[k];
    const double* Wk = w + layer_offset(ch, k - 1);
    const double* bk = Wk + (long)co_n * ci_n * 9;
    double* cur = (double*)malloc(sizeof(double) * (size_t)co_n * rh * rw);
    conv_layer lay = {Wk, bk, prev, cur, ci_n, k < L, H, W, r, prev_r, ph, pw};
    parallel_ranges(co_n, conv_channels, &lay);
    if (keep) memcpy(keep[k - 1], cur, sizeof(double) * (size_t)co_n * rh * rw);
    free(prev);
    prev = cur;
    prev_r = r;
    ph = rh;
    pw = rw;
  }
  /* the last layer has one channel: the logit x_a; pi_a(h=1) = sigmoid(x_a) */
  for (int y = 0; y < out.y1 - out.y0; ++y)
    for (int x = 0; x < out.x1 - out.x0; ++x)
      logits[(size_t)y * (out.x1 - out.x0) + x] = prev[(size_t)y * pw + x];
  free(prev);
}

/* Logits of B images over the whole image. */
void or_policy_forward(const double* w, const int* ch, int L, const double* c,
                       const double* z, int B, int H, int W, double* logits) {
  region full = {0, H, 0, W};
  for (int b = 0; b < B; ++b)
    forward_one(w, ch, L, c + (size_t)b * H * W, z + (size_t)b * H * W, H, W,
                full, logits + (size_t)b * H * W, NULL);
}

/* Logits of image (c, z) (H x W) over an output window only: the same
 * definition evaluated on the window's receptive field. */
void or_policy_forward_window(const double* w, const int* ch, int L,
                              const double* c, const double* z, int H, int W,
                              int y0, int y1, int x0, int x1, double* logits) {
  region r = {y0, y1, x0, x1};
  forward_one(w, ch, L, c, z, H, W, r, logits, NULL);
}

/* Test phase of Algorithm 1: h = Thresholding(CNN(c, z), 0.5). A tie
 * (p exactly 0.5) is not specified by the paper; it is read as white. */
void or_threshold(const double* logits, long n, uint8_t* bits) {
  for (long i = 0; i < n; ++i) bits[i] = logits[i] >= 0.0 ? 1 : 0;
}

/* Gradients of one conv layer y = b + W * s given g = dLoss/dy (C x H x W):
 *   dLoss/dW[o][i][dy][dx] += sum_{y,x} g[o](y, x) s_i(y + dy - 1, x + dx - 1),
 *   dLoss/db[o]            += sum_{y,x} g[o](y, x),
 *   dLoss/ds_i(sy, sx)     += sum_{o, dy, dx} g[o](sy - dy + 1, sx - dx + 1) W[o][i][dy][dx],
 * terms outside the image dropped. Both sums visit their terms in the order
 * (o, y, x, dy, dx) of one loop over the output, so splitting the first over
 * o and the second over i changes no rounding. */
typedef struct {
  const double *Wk, *in, *g;
  double *gW, *gb, *gin;
  int ci_n, co_n, H, W;
} conv_grad;

static void conv_grad_weights(int o0, int o1, void* ctx) {
  const conv_grad* c = (const conv_grad*)ctx;
  const double* in = c->in;
  const double* g = c->g;
  double* gW = c->gW;
  double* gb = c->gb;
  const int H = c->H, W = c->W, ci_n = c->ci_n;
  const size_t HW = (size_t)H * W;
  for (int o = o0; o < o1; ++o)
    for (int y = 0; y < H; ++y)
      for (int x = 0; x < W; ++x) {
        double go = g[(size_t)o * HW + (size_t)y * W + x];
        if (go == 0.0) continue;
        gb[o] += go;
        for (int i = 0; i < ci_n; ++i)
          for (int dy = 0; dy < 3; ++dy)
            for (int dx = 0; dx < 3; ++dx) {
              int sy = y + dy - 1, sx = x + dx - 1;
              if (sy < 0 || sy >= H || sx < 0 || sx >= W) continue;
              gW[(((size_t)o * ci_n + i) * 3 + dy) * 3 + dx] +=
                  go * in[(size_t)i * HW + (size_t)sy * W + sx];
            }
      }
}

static void conv_grad_input(int i0, int i1, void* ctx) {
  const conv_grad* c = (const conv_grad*)ctx;
  const double* Wk = c->Wk;
  const double* g = c->g;
  double* gin = c->gin;
  const int H = c->H, W = c->W, ci_n = c->ci_n, co_n = c->co_n;
  const size_t HW = (size_t)H * W;
  for (int i = i0; i < i1; ++i)
    for (int o = 0; o < co_n; ++o)
      for (int y = 0; y < H; ++y)
        for (int x = 0; x < W; ++x) {
          double go = g[(size_t)o * HW + (size_t)y * W + x];
          if (go == 0.0) continue;
          for (int dy = 0; dy < 3; ++dy)
            for (int dx = 0; dx < 3; ++dx) {
              int sy = y + dy - 1, sx = x + dx - 1;
              if (sy < 0 || sy >= H || sx < 0 || sx >= W) continue;
              gin[(size_t)i * HW + (size_t)sy * W + sx] +=
                  go * Wk[(((size_t)o * ci_n + i) * 3 + dy) * 3 + dx];
            }
        }
}

/* Backward pass of the conv stack (the chain rule through Sec. VI-A's
 * network): given g = dLoss/dlogit for every pixel, accumulate dLoss/dtheta
 * into grad_w (same layout as w; the caller zeroes it) and, if requested,
 * dLoss/ds for the 2-channel input into grad_in [B][2][H][W]. The forward is
 * recomputed and each layer's output kept. ReLU'(0) is taken as 0. */
void or_policy_backward(const double* w, const int* ch, int L, const double* c,
                        const double* z, int B, int H, int W,
                        const double* g_logit, double* grad_w, double* grad_in) {
  size_t HW = (size_t)H * W;
  double** keep = (double**)malloc(sizeof(double*) * L);
  for (int k = 0; k < L; ++k)
    keep[k] = (double*)malloc(sizeof(double) * ch[k + 1] * HW);
  double* logit = (double*)malloc(sizeof(double) * HW);
  double* s0 = (double*)malloc(sizeof(double) * 2 * HW);
  region full = {0, H, 0, W};
  for (int b = 0; b < B; ++b) {
    const double* cb = c + b * HW;
    const double* zb = z + b * HW;
    forward_one(w, ch, L, cb, zb, H, W, full, logit, keep);
    memcpy(s0, cb, sizeof(double) * HW);
    memcpy(s0 + HW, zb, sizeof(double) * HW);
    /* g holds dLoss/d(output of layer k), starting with the logits */
    double* g = (double*)malloc(sizeof(double) * HW);
    memcpy(g, g_logit + b * HW, sizeof(double) * HW);
    for (int k = L; k >= 1; --k) {
      int ci_n = ch[k - 1], co_n = ch[k];
      long off = layer_offset(ch, k - 1);
      const double* Wk = w + off;
      double* gW = grad_w + off;
      double* gb = gW + (long)co_n * ci_n * 9;
      const double* in = k >= 2 ? keep[k - 2] : s0;
      double* gin = (double*)calloc((size_t)ci_n * HW, sizeof(double));
      conv_grad cg = {Wk, in, g, gW, gb, gin, ci_n, co_n, H, W};
      parallel_ranges(co_n, conv_grad_weights, &cg);
      parallel_ranges(ci_n, conv_grad_input, &cg);
      if (k >= 2) {
        /* through the ReLU of layer k-1: zero where its output is 0 */
        for (size_t i = 0; i < (size_t)ci_n * HW; ++i)
          if (!(keep[k - 2][i] > 0.0)) gin[i] = 0.0;
      } else if (grad_in) {
        memcpy(grad_in + (size_t)b * 2 * HW, gin, sizeof(double) * 2 * HW);
      }
      free(g);
      g = gin;
    }
    free(g);
  }
  free(s0);
  free(logit);
  for (int k = 0; k < L; ++k) free(keep[k]);
  free(keep);
}

/* ------------------------------------------------------------------------
 * Halftone metrics (Sec. III "Rewards"; Sec. V).
 * prm[] = {w_s, w_a, hvs_sigma, hvs_r, ssim_sigma, ssim_r, k, C1, C2,
 *          as_patch, estimator, levels}.
 * ---------------------------------------------------------------------- */
enum { P_WS, P_WA, P_HVS_SIGMA, P_HVS_R, P_SSIM_SIGMA, P_SSIM_R, P_K, P_C1,
       P_C2, P_AS_PATCH, P_ESTIMATOR, P_LEVELS };

/* (2r+1)^2 Gaussian window, exp(-(i^2+j^2)/(2 sigma^2)) normalised to sum 1.
 * Used as the HVS low-pass filter (BASELINE's Gaussian sigma = 2 stands in
 * for the paper's Nasanen model) and as the SSIM window (11x11, sigma 1.5,
 * Sec. V). */
void or_gauss_window(double sigma, int r, double* g) {
  int n = 2 * r + 1;
  double sum = 0.0;
  for (int i = -r; i <= r; ++i)
    for (int j = -r; j <= r; ++j) {
      double v = exp(-(double)(i * i + j * j) / (2.0 * sigma * sigma));
      g[(i + r) * n + (j + r)] = v;
      sum += v;
    }
  for (int i = 0; i < n * n; ++i) g[i] /= sum;
}

/* Valid-mode correlation (no padding, Sec. VI-A: metrics are computed
 * without padding): out[y][x] = sum_{i,j} g[i][j] img[y+i][x+j],
 * out is (H-2r) x (W-2r). */
void or_filter_valid(const double* img, int H, int W, const double* g, int r,
                     double* out) {
  int n = 2 * r + 1, oh = H - 2 * r, ow = W - 2 * r;
  for (int y = 0; y < oh; ++y)
    for (int x = 0; x < ow; ++x) {
      double acc = 0.0;
      for (int i = 0; i < n; ++i)
        for (int j = 0; j < n; ++j) acc += g[i * n + j] * img[(size_t)(y + i) * W + (x + j)];
      out[(size_t)y * ow + x] = acc;
    }
}

/* Margin of the common valid region V = [m, H-m) x [m, W-m) on which both the
 * MSE map and the CSSIM map are averaged (paper: the reward is a mean over
 * the reward map). With the default radii (5 and 5) both are the same. */
static int valid_margin(const double* prm) {
  int a = (int)prm[P_HVS_R], b = (int)prm[P_SSIM_R];
  return a > b ? a : b;
}

/* Local SSIM statistics at pixel (cy, cx) of the image over the window w of
 * radius r, in the plain two-pass weighted form of Wang et al. (2004):
 * means, variances and covariance with weights w. */
typedef struct { double mu_h, mu_c, var_h, var_c, cov; } ssim_stats;

static ssim_stats window_stats(const double* h, const double* c, int W,
                               int cy, int cx, const double* w, int r) {
  int n = 2 * r + 1;
  ssim_stats s = {0, 0, 0, 0, 0};
  for (int i = -r; i <= r; ++i)
    for (int j = -r; j <= r; ++j) {
      double wi = w[(i + r) * n + (j + r)];
      size_t p = (size_t)(cy + i) * W + (cx + j);
      s.mu_h += wi * h[p];
      s.mu_c += wi * c[p];
    }
  for (int i = -r; i <= r; ++i)
    for (int j = -r; j <= r; ++j) {
      double wi = w[(i + r) * n + (j + r)];
      size_t p = (size_t)(cy + i) * W + (cx + j);
      double dh = h[p] - s.mu_h, dc = c[p] - s.mu_c;
      s.var_h += wi * dh * dh;
      s.var_c += wi * dc * dc;
      s.cov += wi * dh * dc;
    }
  return s;
}

/* SSIM index from the local statistics (Wang et al. 2004, with C1, C2). */
static double ssim_from(double mu_h, double mu_c, double var_h, double var_c,
                        double cov, double C1, double C2) {
  return (2.0 * mu_h * mu_c + C1) * (2.0 * cov + C2) /
         ((mu_h * mu_h + mu_c * mu_c + C1) * (var_h + var_c + C2));
}

/* Per image b: out[3b+0] = MSE(HVS(h), HVS(c)) over V (Sec. III, Eq. reward;
 * Eq. final_reward), out[3b+1] = mean CSSIM over V (Eq. cssim: contrast map
 * sigma_a = k * sqrt(sum w (c - mu)^2)), out[3b+2] = R = -MSE + w_s * CSSIM
 * (Eq. final_reward). h may be real-valued (used by derivative checks). */
void or_reward(const double* h, const double* c, int B, int H, int W,
               const double* prm, double* out) {
  int rh = (int)prm[P_HVS_R], rs = (int)prm[P_SSIM_R], m = valid_margin(prm);
  double* G = (double*)malloc(sizeof(double) * (2 * rh + 1) * (2 * rh + 1));
  double* w = (double*)malloc(sizeof(double) * (2 * rs + 1) * (2 * rs + 1));
  or_gauss_window(prm[P_HVS_SIGMA], rh, G);
  or_gauss_window(prm[P_SSIM_SIGMA], rs, w);
  int nh = 2 * rh + 1;
  for (int b = 0; b < B; ++b) {
    const double* hb = h + (size_t)b * H * W;
    const double* cb = c + (size_t)b * H * W;
    double se = 0.0, cs = 0.0;
    long M = 0;
    for (int y = m; y < H - m; ++y)
      for (int x = m; x < W - m; ++x) {
        double fh = 0.0, fc = 0.0;
        for (int i = -rh; i <= rh; ++i)
          for (int j = -rh; j <= rh; ++j) {
            double g = G[(i + rh) * nh + (j + rh)];
            fh += g * hb[(size_t)(y + i) * W + (x + j)];
            fc += g * cb[(size_t)(y + i) * W + (x + j)];
          }
        se += (fh - fc) * (fh - fc);
        ssim_stats s = window_stats(hb, cb, W, y, x, w, rs);
        double ssim = ssim_from(s.mu_h, s.mu_c, s.var_h, s.var_c, s.cov,
                                prm[P_C1], prm[P_C2]);
        double sig = prm[P_K] * sqrt(s.var_c);
        cs += sig * ssim + (1.0 - sig);
        ++M;
      }
    double mse = M ? se / (double)M : 0.0;
    double cssim = M ? cs / (double)M : 0.0;
    out[3 * b + 0] = mse;
    out[3 * b + 1] = cssim;
    out[3 * b + 2] = -mse + prm[P_WS] * cssim;
  }
  free(G);
  free(w);
}

/* ------------------------------------------------------------------------
 * Local Expectation gradient (Sec. III-B, Eqs. le and marl; Sec. III-C).
 * For every pixel a, dR[a] = R({h_a = 1, h_-a}) - R({h_a = 0, h_-a}).
 * Then dL_MARL/dp_a = -dR[a] / B.
 * ---------------------------------------------------------------------- */

/* (i) Brute force: evaluate R for both values of h_a from scratch. */
void or_le_delta_brute(const double* h, const double* c, int B, int H, int W,
                       const double* prm, double* dR) {
  size_t HW = (size_t)H * W;
  double* t = (double*)malloc(sizeof(double) * HW);
  double r1[3], r0[3];
  for (int b = 0; b < B; ++b) {
    memcpy(t, h + b * HW, sizeof(double) * HW);
    for (size_t a = 0; a < HW; ++a) {
      double keep = t[a];
      t[a] = 1.0;
      or_reward(t, c + b * HW, 1, H, W, prm, r1);
      t[a] = 0.0;
      or_reward(t, c + b * HW, 1, H, W, prm, r0);
      t[a] = keep;
      dR[b * HW + a] = r1[2] - r0[2];
    }
  }
  free(t);
}

/* (ii) The paper's efficient form (Sec. III-C): all agents share the filtered
 * maps of the sampled h; toggling h_a only changes the reward map inside the
 * filter window around a, by plus/minus the filter. For binary h:
 *   delta = 1 - 2 h_a (the toggle's sign),
 *   MSE part:   F(h)_j moves by delta*G_{a-j}, so the change of the squared
 *               error at j is 2 delta G e_j + G^2;
 *   CSSIM part: mu_h,j moves by delta*w_{a-j}; var_h stays mu_h (1 - mu_h)
 *               because h stays binary and w sums to 1; cov_j moves by
 *               delta*w_{a-j}(c_a - mu_c,j); var_c and sigma_c do not move.
 * dR[a] = delta * (R(toggled) - R(h)). */
void or_le_delta_local(const double* h, const double* c, int B, int H, int W,
                       const double* prm, double* dR) {
  int rh = (int)prm[P_HVS_R], rs = (int)prm[P_SSIM_R], m = valid_margin(prm);
  int nh = 2 * rh + 1, ns = 2 * rs + 1;
  double* G = (double*)malloc(sizeof(double) * nh * nh);
  double* w = (double*)malloc(sizeof(double) * ns * ns);
  or_gauss_window(prm[P_HVS_SIGMA], rh, G);
  or_gauss_window(prm[P_SSIM_SIGMA], rs, w);
  size_t HW = (size_t)H * W;
  double* e = (double*)calloc(HW, sizeof(double));
  ssim_stats* st = (ssim_stats*)calloc(HW, sizeof(ssim_stats));
  double* ssim = (double*)calloc(HW, sizeof(double));
  double* sig = (double*)calloc(HW, sizeof(double));
  double C1 = prm[P_C1], C2 = prm[P_C2];
  long M = (long)(H - 2 * m) * (W - 2 * m);
  for (int b = 0; b < B; ++b) {
    const double* hb = h + b * HW;
    const double* cb = c + b * HW;
    for (int y = m; y < H - m; ++y)
      for (int x = m; x < W - m; ++x) {
        double fh = 0.0, fc = 0.0;
        for (int i = -rh; i <= rh; ++i)
          for (int j = -rh; j <= rh; ++j) {
            double g = G[(i + rh) * nh + (j + rh)];
            fh += g * hb[(size_t)(y + i) * W + (x + j)];
            fc += g * cb[(size_t)(y + i) * W + (x + j)];
          }
        size_t p = (size_t)y * W + x;
        e[p] = fh - fc;
        st[p] = window_stats(hb, cb, W, y, x, w, rs);
        ssim[p] = ssim_from(st[p].mu_h, st[p].mu_c, st[p].var_h, st[p].var_c,
                            st[p].cov, C1, C2);
        sig[p] = prm[P_K] * sqrt(st[p].var_c);
      }
    for (int ay = 0; ay < H; ++ay)
      for (int ax = 0; ax < W; ++ax) {
        size_t a = (size_t)ay * W + ax;
        double delta = 1.0 - 2.0 * hb[a];
        double dmse = 0.0, dcs = 0.0;
        /* reward-map pixels j whose HVS window contains a */
        for (int jy = ay - rh; jy <= ay + rh; ++jy)
          for (int jx = ax - rh; jx <= ax + rh; ++jx) {
            if (jy < m || jy >= H - m || jx < m || jx >= W - m) continue;
            double g = G[(ay - jy + rh) * nh + (ax - jx + rh)];
            dmse += 2.0 * delta * g * e[(size_t)jy * W + jx] + g * g;
          }
        /* reward-map pixels j whose SSIM window contains a */
        for (int jy = ay - rs; jy <= ay + rs; ++jy)
          for (int jx = ax - rs; jx <= ax + rs; ++jx) {
            if (jy < m || jy >= H - m || jx < m || jx >= W - m) continue;
            size_t j = (size_t)jy * W + jx;
            double wa = w[(ay - jy + rs) * ns + (ax - jx + rs)];
            double mu_h = st[j].mu_h + delta * wa;
            double var_h = mu_h * (1.0 - mu_h);
            double cov = st[j].cov + delta * wa * (cb[a] - st[j].mu_c);
            double s1 = ssim_from(mu_h, st[j].mu_c, var_h, st[j].var_c, cov, C1, C2);
            dcs += sig[j] * (s1 - ssim[j]);
          }
        dR[b * HW + a] =
            delta * (-dmse / (double)M + prm[P_WS] * dcs / (double)M);
      }
  }
  free(G); free(w); free(e); free(st); free(ssim); free(sig);
}

/* ------------------------------------------------------------------------
 * Multitoning (Sec. VI-E, the deep multitoning prototype). There are L ink
 * levels l_k = k Delta, k = 0..L-1, Delta = 1/(L-1). The network keeps its
 * single sigmoid output v_a, and agent a chooses between the two levels
 * around v_a: the upper one with probability (v_a - floor(v_a)) / Delta and
 * the lower one otherwise (the unnumbered rounding equation of Sec. VI-E).
 * So every agent still has two actions, and E[h_a] = v_a.
 * Readings where the paper is silent:
 *   - the pair around v is (k_f, k_f + 1) with k_f = min(floor(v / Delta),
 *     L - 2), so v = 1 picks level L-1 with probability one;
 *   - the test phase rounds v to the nearest level, a tie going up (the
 *     binary threshold at 0.5 is the case L = 2);
 *   - the anisotropy proxy is v itself, the expectation of the rounding;
 *   - a level is stored as its index k (one byte), the image value is k Delta.
 * With L = 2 each function below is the binary one.
 * ---------------------------------------------------------------------- */
static int pair_low(double v, int L) {
  int k = (int)floor(v * (L - 1));
  if (k > L - 2) k = L - 2;
  if (k < 0) k = 0;
  return k;
}

/* Actions h_a = l_{k_f} or l_{k_f + 1}; the upper one iff u_a < q_a with
 * q_a = v_a (L-1) - k_f and u_a the stream-0 uniform of or_bernoulli. */
void or_multitone_actions(const double* v, const uint64_t* seeds, int B, int H, int W,
                          int L, uint32_t step, uint8_t* k) {
  for (int b = 0; b < B; ++b)
    for (int y = 0; y < H; ++y)
      for (int x = 0; x < W; ++x) {
        uint64_t a = (uint64_t)y * (uint64_t)W + (uint64_t)x;
        size_t i = ((size_t)b * H + y) * W + x;
        int kf = pair_low(v[i], L);
        double q = v[i] * (L - 1) - kf;
        k[i] = (uint8_t)(kf + (or_uniform(seeds[b], a, 0, step) < q ? 1 : 0));
      }
}

/* Test phase: the level nearest to v = sigmoid(x), a tie going up. The
 * sigmoid is monotone, so this is the number of midpoints (j + 1/2) Delta,
 * j = 0..L-2, that v reaches, decided on the logit against
 * logit((j + 1/2) Delta) = log((2j + 1) / (2L - 3 - 2j)); for L = 2 that is
 * the binary threshold x >= 0 exactly. */
void or_multitone_levels(const double* logits, long n, int L, uint8_t* k) {
  for (long i = 0; i < n; ++i) {
    int kk = 0;
    for (int j = 0; j + 1 < L; ++j)
      if (logits[i] >= log((2.0 * j + 1.0) / (2.0 * L - 3.0 - 2.0 * j))) ++kk;
    k[i] = (uint8_t)kk;
  }
}

/* The Local Expectation difference of the two actions of every agent:
 * dR[a] = R({h_a = l_{k_f+1}, h_-a}) - R({h_a = l_{k_f}, h_-a}), with k_f
 * from v_a; then dE[R]/dv_a = dR[a] / Delta. h holds image values.
 * (i) Brute force: both rewards from scratch. */
void or_multitone_delta_brute(const double* h, const double* c, const double* v, int B,
                              int H, int W, int L, const double* prm, double* dR) {
  size_t HW = (size_t)H * W;
  double* t = (double*)malloc(sizeof(double) * HW);
  double r1[3], r0[3];
  for (int b = 0; b < B; ++b) {
    memcpy(t, h + b * HW, sizeof(double) * HW);
    for (size_t a = 0; a < HW; ++a) {
      double keep = t[a];
      int kf = pair_low(v[b * HW + a], L);
      t[a] = (double)(kf + 1) / (L - 1);
      or_reward(t, c + b * HW, 1, H, W, prm, r1);
      t[a] = (double)kf / (L - 1);
      or_reward(t, c + b * HW, 1, H, W, prm, r0);
      t[a] = keep;
      dR[b * HW + a] = r1[2] - r0[2];
    }
  }
  free(t);
}

/* (ii) The local toggle of Sec. III-C with a step of one level: h_a is one
 * of the pair (k_f, k_f + 1) and moves to the other one, by d = +Delta
 * (from the lower) or -Delta (from the upper). At a reward-map pixel j
 * whose window holds a:
 *   HVS error e_j moves by d G_{a-j}: the squared error by 2 d G e + d^2 G^2;
 *   mu_h,j moves by d w_{a-j}; the weighted second moment of h by
 *   w_{a-j} ((h_a + d)^2 - h_a^2), so var_h' = var_h + w d (2 h_a + d)
 *   - (mu_h'^2 - mu_h^2) (binary h keeps var_h = mu_h (1 - mu_h));
 *   cov_j moves by d w_{a-j} (c_a - mu_c,j); var_c and sigma_c stay.
 * dR[a] = sign(d) (R(moved) - R(h)). Agents whose h_a is not in the pair
 * are not defined here (the sampled actions always are). */
void or_multitone_delta_local(const double* h, const double* c, const double* v, int B,
                              int H, int W, int L, const double* prm, double* dR) {
  int rh = (int)prm[P_HVS_R], rs = (int)prm[P_SSIM_R], m = valid_margin(prm);
  int nh = 2 * rh + 1, ns = 2 * rs + 1;
  double* G = (double*)malloc(sizeof(double) * nh * nh);
  double* w = (double*)malloc(sizeof(double) * ns * ns);
  or_gauss_window(prm[P_HVS_SIGMA], rh, G);
  or_gauss_window(prm[P_SSIM_SIGMA], rs, w);
  size_t HW = (size_t)H * W;
  double* e = (double*)calloc(HW, sizeof(double));
  ssim_stats* st = (ssim_stats*)calloc(HW, sizeof(ssim_stats));
  double* ssim = (double*)calloc(HW, sizeof(double));
  double* sig = (double*)calloc(HW, sizeof(double));
  double C1 = prm[P_C1], C2 = prm[P_C2], step = 1.0 / (L - 1);
  long M = (long)(H - 2 * m) * (W - 2 * m);
  for (int b = 0; b < B; ++b) {
    const double* hb = h + b * HW;
    const double* cb = c + b * HW;
    for (int y = m; y < H - m; ++y)
      for (int x = m; x < W - m; ++x) {
        double fh = 0.0, fc = 0.0;
        for (int i = -rh; i <= rh; ++i)
          for (int j = -rh; j <= rh; ++j) {
            double g = G[(i + rh) * nh + (j + rh)];
            fh += g * hb[(size_t)(y + i) * W + (x + j)];
            fc += g * cb[(size_t)(y + i) * W + (x + j)];
          }
        size_t p = (size_t)y * W + x;
        e[p] = fh - fc;
        st[p] = window_stats(hb, cb, W, y, x, w, rs);
        ssim[p] = ssim_from(st[p].mu_h, st[p].mu_c, st[p].var_h, st[p].var_c,
                            st[p].cov, C1, C2);
        sig[p] = prm[P_K] * sqrt(st[p].var_c);
      }
    for (int ay = 0; ay < H; ++ay)
      for (int ax = 0; ax < W; ++ax) {
        size_t a = (size_t)ay * W + ax;
        int kf = pair_low(v[b * HW + a], L);
        double lo = kf * step;
        /* from the lower level up, else from the upper level down */
        double d = fabs(hb[a] - lo) < 0.5 * step ? step : -step;
        double ha = hb[a];
        double dmse = 0.0, dcs = 0.0;
        for (int jy = ay - rh; jy <= ay + rh; ++jy)
          for (int jx = ax - rh; jx <= ax + rh; ++jx) {
            if (jy < m || jy >= H - m || jx < m || jx >= W - m) continue;
            double g = G[(ay - jy + rh) * nh + (ax - jx + rh)];
            dmse += 2.0 * d * g * e[(size_t)jy * W + jx] + d * d * g * g;
          }
        for (int jy = ay - rs; jy <= ay + rs; ++jy)
          for (int jx = ax - rs; jx <= ax + rs; ++jx) {
            if (jy < m || jy >= H - m || jx < m || jx >= W - m) continue;
            size_t j = (size_t)jy * W + jx;
            double wa = w[(ay - jy + rs) * ns + (ax - jx + rs)];
            double mu_h = st[j].mu_h + d * wa;
            double var_h = st[j].var_h + wa * d * (2.0 * ha + d) -
                           (mu_h * mu_h - st[j].mu_h * st[j].mu_h);
            double cov = st[j].cov + d * wa * (cb[a] - st[j].mu_c);
            double s1 = ssim_from(mu_h, st[j].mu_c, var_h, st[j].var_c, cov, C1, C2);
            dcs += sig[j] * (s1 - ssim[j]);
          }
        double sgn = d > 0.0 ? 1.0 : -1.0;
        dR[b * HW + a] = sgn * (-dmse / (double)M + prm[P_WS] * dcs / (double)M);
      }
  }
  free(G); free(w); free(e); free(st); free(ssim); free(sig);
}

/* ------------------------------------------------------------------------
 * REINFORCE with the counterfactual (COMA) baseline (Sec. III-A, Eqs.
 * baseline and coma), the estimator the Local Expectation one is compared
 * with. For the sampled h and every agent a:
 *   b_a = sum over h'_a of pi_a(h'_a) R({h'_a, h_-a})
 *       = p_a R(h^1) + (1 - p_a) R(h^0),   h^v = h with h_a := v,
 *   g_a = d/dx_a log pi_a(h_a) * (R(h) - b_a),
 * where pi_a(1) = p_a = sigmoid(x_a), so d/dx_a log pi_a(h_a) = h_a - p_a.
 * R(h^1) - R(h^0) is the toggle difference dR of the Local Expectation
 * estimator and R(h) is R(h^{h_a}), so R(h) - b_a needs no further reward
 * evaluation. Output: dL/dx_a = -g_a / B (the loss is -J, averaged over the
 * batch).
 * ---------------------------------------------------------------------- */
void or_coma_grad_logit(const double* h, const double* c, const double* p, int B, int H,
                        int W, const double* prm, double* grad) {
  size_t N = (size_t)B * H * W;
  double* dR = (double*)malloc(sizeof(double) * N);
  or_le_delta_local(h, c, B, H, W, prm, dR);
  for (size_t a = 0; a < N; ++a) {
    /* R(h^1) = R0 + dR and R(h^0) = R0 for any common R0, which cancels */
    double r1 = dR[a], r0 = 0.0;
    double r_h = h[a] != 0.0 ? r1 : r0;
    double b_a = p[a] * r1 + (1.0 - p[a]) * r0;
    double dlogpi = h[a] - p[a];
    grad[a] = -dlogpi * (r_h - b_a) / (double)B;
  }
  free(dR);
}

/* ------------------------------------------------------------------------
 * Anisotropy-suppressing loss (Sec. IV, Eqs. psd, rapsd, as; the probability
 * proxy of Sec. IV). Readings where the paper is silent: the map is cut into
 * non-overlapping P x P patches from (0,0) (remainders dropped); the
 * periodogram of a patch is |DFT|^2 / P^2 with no mean removal; the ring of a
 * frequency (u, v) is rho = round-half-up(sqrt(ub^2 + vb^2)) with
 * ub = min(u, P-u), vb = min(v, P-v), decided exactly in integers; every ring
 * (DC included) takes part; L_AS is the mean over patches.
 * ---------------------------------------------------------------------- */
int or_ring_index(int u, int v, int P) {
  int ub = u < P - u ? u : P - u, vb = v < P - v ? v : P - v;
  long q = 4L * (ub * ub + vb * vb);
  int rho = 0;
  while ((long)(2 * rho + 1) * (2 * rho + 1) <= q) ++rho;
  return rho;
}

/* Returns L_AS = mean over patches of sum_rho sum_{f in ring} (Phat - Pbar)^2.
 * If grad is non-null it receives dL_AS/dx (zero outside the patches). */
double or_as_loss(const double* xmap, int Bg, int Hg, int Wg, int P,
                  double* grad) {
  int N = P * P;
  int nrings = or_ring_index(P / 2, P / 2, P) + 1;
  double* cs = (double*)malloc(sizeof(double) * P);
  double* sn = (double*)malloc(sizeof(double) * P);
  for (int k = 0; k < P; ++k) {
    cs[k] = cos(2.0 * M_PI * k / P);
    sn[k] = sin(2.0 * M_PI * k / P);
  }
  double* re = (double*)malloc(sizeof(double) * N);
  double* im = (double*)malloc(sizeof(double) * N);
  double* ph = (double*)malloc(sizeof(double) * N);
  double* ring_sum = (double*)malloc(sizeof(double) * nrings);
  int* ring_n = (int*)malloc(sizeof(int) * nrings);
  int py = Hg / P, px = Wg / P;
  long npatch = (long)Bg * py * px;
  if (grad) memset(grad, 0, sizeof(double) * (size_t)Bg * Hg * Wg);
  double total = 0.0;
  for (int b = 0; b < Bg; ++b)
    for (int ty = 0; ty < py; ++ty)
      for (int tx = 0; tx < px; ++tx) {
        const double* base = xmap + (size_t)b * Hg * Wg + (size_t)ty * P * Wg + tx * P;
        /* X(u,v) = sum_{y,x} x[y][x] exp(-2 pi i (u y + v x) / P) */
        for (int u = 0; u < P; ++u)
          for (int v = 0; v < P; ++v) {
            double sr = 0.0, si = 0.0;
            for (int y = 0; y < P; ++y)
              for (int x = 0; x < P; ++x) {
                int k = (u * y + v * x) % P;
                double val = base[(size_t)y * Wg + x];
                sr += val * cs[k];
                si -= val * sn[k];
              }
            re[u * P + v] = sr;
            im[u * P + v] = si;
            ph[u * P + v] = (sr * sr + si * si) / (double)N;
          }
        for (int r = 0; r < nrings; ++r) { ring_sum[r] = 0.0; ring_n[r] = 0; }
        for (int u = 0; u < P; ++u)
          for (int v = 0; v < P; ++v) {
            int r = or_ring_index(u, v, P);
            ring_sum[r] += ph[u * P + v];
            ring_n[r] += 1;
          }
        double L = 0.0;
        for (int u = 0; u < P; ++u)
          for (int v = 0; v < P; ++v) {
            int r = or_ring_index(u, v, P);
            double d = ph[u * P + v] - ring_sum[r] / ring_n[r];
            L += d * d;
          }
        total += L;
        if (grad) {
          /* dL/dPhat_f = 2 (Phat_f - Pbar_rho(f)) (the ring-mean terms cancel
           * because deviations within a ring sum to zero);
           * dPhat_f/dx_n = (2/N) Re(conj(X_f) exp(-2 pi i f.n / P)). */
          for (int y = 0; y < P; ++y)
            for (int x = 0; x < P; ++x) {
              double acc = 0.0;
              for (int u = 0; u < P; ++u)
                for (int v = 0; v < P; ++v) {
                  int r = or_ring_index(u, v, P);
                  double gf = 2.0 * (ph[u * P + v] - ring_sum[r] / ring_n[r]);
                  int k = (u * y + v * x) % P;
                  /* Re(conj(X) e^{-i t}) = re cos t - im sin t */
                  double dphat = (2.0 / N) * (re[u * P + v] * cs[k] - im[u * P + v] * sn[k]);
                  acc += gf * dphat;
                }
              grad[(size_t)b * Hg * Wg + (size_t)(ty * P + y) * Wg + tx * P + x] =
                  acc / (double)npatch;
            }
        }
      }
  free(cs); free(sn); free(re); free(im); free(ph); free(ring_sum); free(ring_n);
  return npatch ? total / (double)npatch : 0.0;
}

/* Periodogram of one P x P patch (Eq. psd): |DFT|^2 / P^2 by the direct sum. */
static void periodogram(const double* patch, int ld, int P, double* ph) {
  int N = P * P;
  for (int u = 0; u < P; ++u)
    for (int v = 0; v < P; ++v) {
      double sr = 0.0, si = 0.0;
      for (int y = 0; y < P; ++y)
        for (int x = 0; x < P; ++x) {
          double t = 2.0 * M_PI * (double)((u * y + v * x) % P) / P;
          sr += patch[(size_t)y * ld + x] * cos(t);
          si -= patch[(size_t)y * ld + x] * sin(t);
        }
      ph[u * P + v] = (sr * sr + si * si) / N;
    }
}

/* RAPSD (Eq. rapsd) and anisotropy (Eq. anis) of a power spectrum estimate:
 * for every ring rho, the mean of the estimate over the ring and the
 * variance about it over the squared mean, with n - 1 in the denominator
 * (rings with one sample, or zero mean, get anisotropy 0). */
static void ring_stats(const double* ph, int P, double* rapsd, double* anis) {
  int nrings = or_ring_index(P / 2, P / 2, P) + 1;
  for (int r = 0; r < nrings; ++r) {
    double s = 0.0;
    int n = 0;
    for (int u = 0; u < P; ++u)
      for (int v = 0; v < P; ++v)
        if (or_ring_index(u, v, P) == r) { s += ph[u * P + v]; ++n; }
    double mean = s / n, a = 0.0;
    for (int u = 0; u < P; ++u)
      for (int v = 0; v < P; ++v)
        if (or_ring_index(u, v, P) == r) {
          double d = ph[u * P + v] - mean;
          a += d * d;
        }
    rapsd[r] = mean;
    anis[r] = (n > 1 && mean != 0.0) ? a / ((n - 1) * mean * mean) : 0.0;
  }
}

/* Anisotropy A(f_rho) of one P x P patch (Eq. anis), for the blue-noise
 * evaluation: out[rho] for every ring (rings with one sample get 0). */
void or_anisotropy(const double* patch, int P, double* rapsd, double* anis) {
  double* ph = (double*)malloc(sizeof(double) * P * P);
  periodogram(patch, P, P, ph);
  ring_stats(ph, P, rapsd, anis);
  free(ph);
}

/* Blue-noise evaluation of halftones (the spectral measures of Sec. IV,
 * Eqs. psd, rapsd, anis): the power spectrum is estimated as the mean of the
 * periodograms of all non-overlapping P x P patches of the B images (from
 * (0, 0), remainders dropped), then reduced to RAPSD and anisotropy per
 * ring. Returns the number of patches. */
int or_spectrum(const double* img, int B, int H, int W, int P, double* rapsd, double* anis) {
  int py = H / P, px = W / P, np = B * py * px;
  double* ph = (double*)malloc(sizeof(double) * P * P);
  double* avg = (double*)calloc((size_t)P * P, sizeof(double));
  for (int b = 0; b < B; ++b)
    for (int ty = 0; ty < py; ++ty)
      for (int tx = 0; tx < px; ++tx) {
        periodogram(img + (size_t)b * H * W + (size_t)ty * P * W + tx * P, W, P, ph);
        for (int i = 0; i < P * P; ++i) avg[i] += ph[i];
      }
  if (np > 0) {
    for (int i = 0; i < P * P; ++i) avg[i] /= np;
    ring_stats(avg, P, rapsd, anis);
  }
  free(ph);
  free(avg);
  return np;
}

/* ------------------------------------------------------------------------
 * Optimiser (Sec. VI-A): Adam (Kingma and Ba) with the textbook defaults,
 * learning rate annealed from lr_max to lr_min by a cosine schedule.
 * ---------------------------------------------------------------------- */
double or_lr_cosine(long t, long T, double lr_max, double lr_min) {
  if (T <= 0) return lr_max;
  return lr_min + 0.5 * (lr_max - lr_min) * (1.0 + cos(M_PI * (double)t / (double)T));
}

/* t is the 1-based step count used by the bias corrections. */
void or_adam_step(double* theta, double* m, double* v, const double* g, long n,
                  long t, double lr, double b1, double b2, double eps) {
  double c1 = 1.0 - pow(b1, (double)t), c2 = 1.0 - pow(b2, (double)t);
  for (long i = 0; i < n; ++i) {
    m[i] = b1 * m[i] + (1.0 - b1) * g[i];
    v[i] = b2 * v[i] + (1.0 - b2) * g[i] * g[i];
    double mh = m[i] / c1, vh = v[i] / c2;
    theta[i] -= lr * mh / (sqrt(vh) + eps);
  }
}

/* ------------------------------------------------------------------------
 * One TRAIN iteration of Algorithm 1:
 *   z ~ N(0, I) (stream 1, this step); p = sigmoid(CNN(c, z));
 *   h ~ Bernoulli(p) (stream 0, this step) unless `actions_in` is given;
 *   dL_MARL/dp = -dR/B (Local Expectation), or the COMA estimator's
 *   dL/dx when prm[P_ESTIMATOR] = 1; back through the sigmoid and the conv
 *   stack;
 *   with prm[P_LEVELS] = L > 2 (multitoning): actions are level indices
 *   drawn by or_multitone_actions, the reward is taken on h = k / (L-1), and
 *   dL_MARL/dv = -dR (L-1) / B with dR from or_multitone_delta_local (Local
 *   Expectation only);
 *   the constant-gray side batch: p_g = sigmoid(CNN(c_g, z_g)),
 *   dL_AS/dp_g, back through the sigmoid and the conv stack, weighted by w_a;
 *   Adam step with the cosine learning rate of `step` (0-based) out of
 *   `total`.
 * tprm[] = {lr_max, lr_min, beta1, beta2, eps}.
 * metrics[] = {mean MSE, mean CSSIM, mean R, L_AS, lr, |grad|, fill}, fill
 * being the mean of h.
 * ---------------------------------------------------------------------- */
void or_train_step(double* w, double* m, double* v, const int* ch, int L,
                   const double* c, const uint64_t* seeds, int B, int H, int W,
                   const double* cg, const uint64_t* gseeds, int Bg, int Hg,
                   int Wg, long step, long total, const double* prm,
                   const double* tprm, int noise_kind,
                   const uint8_t* actions_in, uint8_t* actions_out,
                   double* grad_out, double* metrics) {
  long np = or_param_count(ch, L);
  size_t HW = (size_t)H * W, N = (size_t)B * HW;
  double* z = (double*)malloc(sizeof(double) * N);
  double* x = (double*)malloc(sizeof(double) * N);
  double* p = (double*)malloc(sizeof(double) * N);
  double* hd = (double*)malloc(sizeof(double) * N);
  double* dR = (double*)malloc(sizeof(double) * N);
  uint8_t* h = (uint8_t*)malloc(N);
  double* grad = (double*)calloc((size_t)np, sizeof(double));
  or_noise_map(seeds, B, H, W, noise_kind, 1, (uint32_t)step, z);
  or_policy_forward(w, ch, L, c, z, B, H, W, x);
  for (size_t i = 0; i < N; ++i) p[i] = 1.0 / (1.0 + exp(-x[i]));
  int levels = (int)prm[P_LEVELS];
  if (levels < 2) levels = 2;
  if (actions_in) memcpy(h, actions_in, N);
  else if (levels > 2) or_multitone_actions(p, seeds, B, H, W, levels, (uint32_t)step, h);
  else or_bernoulli(p, seeds, B, H, W, (uint32_t)step, h);
  if (actions_out) memcpy(actions_out, h, N);
  double fill = 0.0;
  for (size_t i = 0; i < N; ++i) { hd[i] = (double)h[i] / (levels - 1); fill += hd[i]; }
  double* rew = (double*)malloc(sizeof(double) * 3 * B);
  or_reward(hd, c, B, H, W, prm, rew);
  if (levels > 2) {
    or_multitone_delta_local(hd, c, p, B, H, W, levels, prm, dR);
    /* dL/dx_a = dL/dv_a * v_a (1 - v_a), dL/dv_a = -dR_a (L-1) / B */
    for (size_t i = 0; i < N; ++i) dR[i] = (-dR[i] * (levels - 1) / B) * p[i] * (1.0 - p[i]);
  } else if ((int)prm[P_ESTIMATOR] == 1) {
    or_coma_grad_logit(hd, c, p, B, H, W, prm, dR);
  } else {
    or_le_delta_local(hd, c, B, H, W, prm, dR);
    /* dL/dx_a = dL/dp_a * p_a (1 - p_a), dL/dp_a = -dR_a / B */
    for (size_t i = 0; i < N; ++i) dR[i] = (-dR[i] / B) * p[i] * (1.0 - p[i]);
  }
  or_policy_backward(w, ch, L, c, z, B, H, W, dR, grad, NULL);
  double las = 0.0;
  if (Bg > 0) {
    size_t NG = (size_t)Bg * Hg * Wg;
    double* zg = (double*)malloc(sizeof(double) * NG);
    double* xg = (double*)malloc(sizeof(double) * NG);
    double* pg = (double*)malloc(sizeof(double) * NG);
    double* gg = (double*)malloc(sizeof(double) * NG);
    or_noise_map(gseeds, Bg, Hg, Wg, noise_kind, 1, (uint32_t)step, zg);
    or_policy_forward(w, ch, L, cg, zg, Bg, Hg, Wg, xg);
    for (size_t i = 0; i < NG; ++i) pg[i] = 1.0 / (1.0 + exp(-xg[i]));
    las = or_as_loss(pg, Bg, Hg, Wg, (int)prm[P_AS_PATCH], gg);
    for (size_t i = 0; i < NG; ++i) gg[i] = prm[P_WA] * gg[i] * pg[i] * (1.0 - pg[i]);
    or_policy_backward(w, ch, L, cg, zg, Bg, Hg, Wg, gg, grad, NULL);
    free(zg); free(xg); free(pg); free(gg);
  }
  double lr = or_lr_cosine(step, total, tprm[0], tprm[1]);
  double gn = 0.0;
  for (long i = 0; i < np; ++i) gn += grad[i] * grad[i];
  if (grad_out) memcpy(grad_out, grad, sizeof(double) * np);
  or_adam_step(w, m, v, grad, np, step + 1, lr, tprm[2], tprm[3], tprm[4]);
  double smse = 0, scs = 0, sr = 0;
  for (int b = 0; b < B; ++b) { smse += rew[3 * b]; scs += rew[3 * b + 1]; sr += rew[3 * b + 2]; }
  metrics[0] = smse / B;
  metrics[1] = scs / B;
  metrics[2] = sr / B;
  metrics[3] = las;
  metrics[4] = lr;
  metrics[5] = sqrt(gn);
  metrics[6] = fill / (double)N;
  free(z); free(x); free(p); free(hd); free(dR); free(h); free(grad); free(rew);
}

/* ------------------------------------------------------------------------
 * Floyd-Steinberg error diffusion (Floyd and Steinberg 1976, cited in Sec. I
 * as the classic error diffusion): raster order, v = c + diffused error,
 * h = [v >= 0.5], error q = v - h pushed 7/16 right, 3/16 down-left,
 * 5/16 down, 1/16 down-right; error leaving the image is dropped.
 * ---------------------------------------------------------------------- */
void or_floyd_steinberg(const double* c, int B, int H, int W, uint8_t* h) {
  double* v = (double*)malloc(sizeof(double) * (size_t)H * W);
  for (int b = 0; b < B; ++b) {
    memcpy(v, c + (size_t)b * H * W, sizeof(double) * (size_t)H * W);
    for (int y = 0; y < H; ++y)
      for (int x = 0; x < W; ++x) {
        double val = v[(size_t)y * W + x];
        uint8_t bit = val >= 0.5 ? 1 : 0;
        double q = val - (double)bit;
        h[(size_t)b * H * W + (size_t)y * W + x] = bit;
        if (x + 1 < W) v[(size_t)y * W + x + 1] += q * 7.0 / 16.0;
        if (y + 1 < H) {
          if (x > 0) v[(size_t)(y + 1) * W + x - 1] += q * 3.0 / 16.0;
          v[(size_t)(y + 1) * W + x] += q * 5.0 / 16.0;
          if (x + 1 < W) v[(size_t)(y + 1) * W + x + 1] += q * 1.0 / 16.0;
        }
      }
  }
  free(v);
}

/* Floyd-Steinberg with L output levels k / (L-1), the error diffusion that
 * stands beside the multitoning variant (Sec. VI-E) as its serial fallback:
 * v = c + diffused error, k = the level nearest to v (a tie going up, clamped
 * to 0..L-1), error v - k / (L-1) pushed with the same weights and borders
 * as or_floyd_steinberg, which is the case L = 2. */
void or_floyd_steinberg_levels(const double* c, int B, int H, int W, int L, uint8_t* k) {
  double* v = (double*)malloc(sizeof(double) * (size_t)H * W);
  for (int b = 0; b < B; ++b) {
    memcpy(v, c + (size_t)b * H * W, sizeof(double) * (size_t)H * W);
    for (int y = 0; y < H; ++y)
      for (int x = 0; x < W; ++x) {
        double val = v[(size_t)y * W + x];
        int lev = (int)floor(val * (L - 1) + 0.5);
        if (lev < 0) lev = 0;
        if (lev > L - 1) lev = L - 1;
        double q = val - (double)lev / (L - 1);
        k[(size_t)b * H * W + (size_t)y * W + x] = (uint8_t)lev;
        if (x + 1 < W) v[(size_t)y * W + x + 1] += q * 7.0 / 16.0;
        if (y + 1 < H) {
          if (x > 0) v[(size_t)(y + 1) * W + x - 1] += q * 3.0 / 16.0;
          v[(size_t)(y + 1) * W + x] += q * 5.0 / 16.0;
          if (x + 1 < W) v[(size_t)(y + 1) * W + x + 1] += q * 1.0 / 16.0;
        }
      }
  }
  free(v);
}
