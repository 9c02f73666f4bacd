// loss.hip -- reward, Local Expectation gradient and anisotropy-suppressing
// loss on gfx950 (FP32 on the vector ALUs, tiles staged in LDS).
//
// Reward (Sec. III "Rewards", Eq. final_reward; Sec. V, Eq. cssim): over the
// valid region V = [m, H-m) x [m, W-m), e = HVS(h) - HVS(c) and
// CSSIM = sigma_c SSIM + 1 - sigma_c with sigma_c = k sqrt(var_c);
// R = -mean(e^2) + w_s mean(CSSIM). Local statistics use the weighted
// two-pass form (means first, then centred second moments) for accuracy.
//
// Local Expectation gradient (Sec. III-B, Eq. le; Sec. III-C): for every
// pixel a, the reward change of toggling h_a only involves the reward-map
// pixels j whose windows contain a. With delta = 1 - 2 h_a the HVS error at
// j moves by delta G_{a-j}; the SSIM statistics at j move by
// dmu_h = delta w_{a-j}, dcov = delta w_{a-j} (c_a - mu_c), and var_h stays
// mu_h (1 - mu_h) for binary h. The SSIM change is evaluated as a difference
// of products expanded in those increments, so no two O(1) values are
// subtracted. dR_a = delta (R(toggled) - R(h)); dL_MARL/dp_a = -dR_a / B.
//
// Multitoning (Sec. VI-E, its unnumbered rounding equation; L levels spaced s = 1/(L-1)): an
// action byte is a level index k, h = k s. Agent a's two actions are the
// levels kf, kf + 1 around its output v_a (kf = min(floor(v (L-1)), L-2)),
// and its toggle moves h_a by delta = +s (from kf) or -s (from kf + 1). Then
// var_h is no longer mu_h (1 - mu_h): it is kept as a map, and moves by
// w delta (2 h_a + delta) - (mu_h'^2 - mu_h^2) = dw (2 h_a + delta - 2 mu_h
// - dw), dw = delta w_{a-j}. dR_a = R(kf + 1) - R(kf) and
// dL_MARL/dv_a = -dR_a (L-1) / B.
//
// Anisotropy-suppressing loss (Sec. IV, Eqs. psd, rapsd, as): per 32 x 32
// patch of the probability map, Phat = |DFT|^2 / 1024, ring means over
// rings of width 1 (ring of (u, v) = rounded radius of the folded
// frequency), L = sum (Phat - ring mean)^2. Its adjoint: with
// g = dL/dPhat = 2 (Phat - ring mean), dL/dx = (2/1024) Re(sum_{u,v} g X
// e^{+2 pi i (u y + v x)/32}), an inverse transform of g X.
#include <math.h>

#include "hs_common.h"
#include "hs_internal.h"

namespace {

constexpr int LT = 16;   // output tile edge
constexpr int MAXR = 7;  // largest supported window radius
constexpr int LS = LT + 2 * MAXR;

struct LossConst {
  int rh, rs, m;
  float k, c1, c2, w_s;
  int est;
  int levels;   // 2 = binary
  float hstep;  // 1 / (levels - 1)
};

__global__ __launch_bounds__(256) void loss_stats_kernel(const uint8_t* __restrict__ h,
                                                         const float* __restrict__ c, int H,
                                                         int W, LossConst q,
                                                         const hs::LossDev win,
                                                         float* __restrict__ maps,
                                                         float* __restrict__ partials,
                                                         int ntiles_per_img) {
  __shared__ float sh[LS * LS], sc[LS * LS];
  __shared__ float sG[15 * 15], sw[15 * 15];
  __shared__ float red[2][4];
  const int b = blockIdx.z, m = q.m, R = q.m;
  const int vy0 = m + blockIdx.y * LT, vx0 = m + blockIdx.x * LT;
  const size_t img = (size_t)b * H * W;
  const int ls = LT + 2 * R;
  for (int i = threadIdx.x; i < 15 * 15; i += 256) {
    sG[i] = win.G[i];
    sw[i] = win.w[i];
  }
  for (int i = threadIdx.x; i < ls * ls; i += 256) {
    const int ly = i / ls, lx = i - ly * ls, gy = vy0 - R + ly, gx = vx0 - R + lx;
    const bool in = gy < H && gx < W;  // gy, gx >= 0 because vy0 >= R
    sh[i] = in ? (float)h[img + (size_t)gy * W + gx] * q.hstep : 0.0f;
    sc[i] = in ? c[img + (size_t)gy * W + gx] : 0.0f;
  }
  __syncthreads();
  const int ty = threadIdx.x >> 4, tx = threadIdx.x & 15;
  const int jy = vy0 + ty, jx = vx0 + tx;
  const bool valid = jy < H - m && jx < W - m;
  float e2 = 0.0f, cs = 0.0f;
  if (valid) {
    const int cy = ty + R, cx = tx + R;
    const int nh = 2 * q.rh + 1, ns = 2 * q.rs + 1;
    float e = 0.0f;
    for (int i = -q.rh; i <= q.rh; ++i)
      for (int j = -q.rh; j <= q.rh; ++j) {
        const int p = (cy + i) * ls + cx + j;
        e = fmaf(sG[(i + q.rh) * nh + j + q.rh], sh[p] - sc[p], e);
      }
    float mu_h = 0.0f, mu_c = 0.0f;
    for (int i = -q.rs; i <= q.rs; ++i)
      for (int j = -q.rs; j <= q.rs; ++j) {
        const int p = (cy + i) * ls + cx + j;
        const float wv = sw[(i + q.rs) * ns + j + q.rs];
        mu_h = fmaf(wv, sh[p], mu_h);
        mu_c = fmaf(wv, sc[p], mu_c);
      }
    float var_h = 0.0f, var_c = 0.0f, cov = 0.0f;
    for (int i = -q.rs; i <= q.rs; ++i)
      for (int j = -q.rs; j <= q.rs; ++j) {
        const int p = (cy + i) * ls + cx + j;
        const float wv = sw[(i + q.rs) * ns + j + q.rs];
        const float dh = sh[p] - mu_h, dc = sc[p] - mu_c;
        var_h = fmaf(wv * dh, dh, var_h);
        var_c = fmaf(wv * dc, dc, var_c);
        cov = fmaf(wv * dh, dc, cov);
      }
    const float ssim = ((2.0f * mu_h * mu_c + q.c1) * (2.0f * cov + q.c2)) /
                       ((mu_h * mu_h + mu_c * mu_c + q.c1) * (var_h + var_c + q.c2));
    const float sig = q.k * sqrtf(var_c);
    e2 = e * e;
    cs = sig * ssim + (1.0f - sig);
    if (maps) {
      const size_t n = (size_t)gridDim.z * H * W, o = img + (size_t)jy * W + jx;
      maps[o] = e;
      maps[n + o] = mu_h;
      maps[2 * n + o] = mu_c;
      maps[3 * n + o] = var_c;
      maps[4 * n + o] = cov;
      if (q.levels > 2) maps[5 * n + o] = var_h;
    }
  }
  e2 = hs_wave_sum(e2);
  cs = hs_wave_sum(cs);
  const int wave = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 0) {
    red[0][wave] = e2;
    red[1][wave] = cs;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    const int tile = blockIdx.y * gridDim.x + blockIdx.x;
    float* d = partials + ((size_t)b * ntiles_per_img + tile) * 2;
    d[0] = ((red[0][0] + red[0][1]) + red[0][2]) + red[0][3];
    d[1] = ((red[1][0] + red[1][1]) + red[1][2]) + red[1][3];
  }
}

// The same statistics for compile-time window radii RH (HVS) and RS (SSIM),
// register-blocked: a thread computes four horizontally adjacent outputs.
// The first pass (e = G * (h - c), mu_h = w * h, mu_c = w * c) uses the
// separability of the Gaussian windows (G = g g^T, w = w1 w1^T): row sums
// over the taps j of every staged row into LDS, then column sums over the
// taps i, 4 (2r + 1) operations per output instead of 2 (2r + 1)^2. The
// second pass (the centred second moments, which do not separate) reads
// each staged row segment (4 + 2R values of h and of c) once per kernel row
// for all four outputs, with the same taps in the same order as in
// loss_stats_kernel; the per-tile sums are added in another order. A block
// covers 16 x 64 outputs, i.e. four of the 16 x 16 tiles whose partial sums
// loss_reduce_kernel adds.
constexpr int LB_TY = 16, LB_TX = 64;

template <int RH, int RS>
__global__ __launch_bounds__(256) void loss_stats_rb_kernel(const uint8_t* __restrict__ h,
                                                            const float* __restrict__ c, int H,
                                                            int W, LossConst q,
                                                            const hs::LossDev win,
                                                            float* __restrict__ maps,
                                                            float* __restrict__ partials,
                                                            int ntiles_per_img) {
  constexpr int R = RH > RS ? RH : RS, SY = LB_TY + 2 * R, SX = LB_TX + 2 * R, NS = 4 + 2 * R;
  __shared__ float sh[SY * SX], sc[SY * SX];
  __shared__ float sw[(2 * RS + 1) * (2 * RS + 1)];
  __shared__ float red[2][256];
  // the first pass's row sums: e, mu_h, mu_c of every staged row at the
  // tile's output columns (the windows are separable Gaussians)
  __shared__ __attribute__((aligned(16))) float rE[SY * LB_TX], rH[SY * LB_TX], rC[SY * LB_TX];
  const int b = blockIdx.z;
  const int vy0 = R + blockIdx.y * LB_TY, vx0 = R + blockIdx.x * LB_TX;
  const size_t img = (size_t)b * H * W;
  // the SSIM window's rows of 2 r + 1 taps, stored densely (win holds 15 x 15)
  for (int i = threadIdx.x; i < (2 * RS + 1) * (2 * RS + 1); i += 256)
    sw[i] = win.w[(i / (2 * RS + 1)) * (2 * RS + 1) + i % (2 * RS + 1)];
  for (int i = threadIdx.x; i < SY * SX; i += 256) {
    const int ly = i / SX, lx = i - ly * SX, gy = vy0 - R + ly, gx = vx0 - R + lx;
    const bool in = gy < H && gx < W;  // gy, gx >= 0 because vy0, vx0 >= R
    sh[i] = in ? (float)h[img + (size_t)gy * W + gx] * q.hstep : 0.0f;
    sc[i] = in ? c[img + (size_t)gy * W + gx] : 0.0f;
  }
  __syncthreads();
  // ---- first pass, separable: row sums over the taps j (item = a staged
  // row and four output columns), then column sums over the taps i
  for (int it = threadIdx.x; it < SY * (LB_TX / 4); it += 256) {
    const int ly = it / (LB_TX / 4), x4 = 4 * (it % (LB_TX / 4));
    float hv[NS], cv[NS];
#pragma unroll
    for (int j = 0; j < NS; ++j) {
      hv[j] = sh[ly * SX + x4 + j];
      cv[j] = sc[ly * SX + x4 + j];
    }
    f32x4_t re = {0.f, 0.f, 0.f, 0.f}, rh = {0.f, 0.f, 0.f, 0.f}, rc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int j = 0; j < 2 * RH + 1; ++j) {
      const float g = win.g1[j];
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        const int p = k + j + (R - RH);
        re[k] = fmaf(g, hv[p] - cv[p], re[k]);
      }
    }
#pragma unroll
    for (int j = 0; j < 2 * RS + 1; ++j) {
      const float wv = win.w1[j];
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        const int p = k + j + (R - RS);
        rh[k] = fmaf(wv, hv[p], rh[k]);
        rc[k] = fmaf(wv, cv[p], rc[k]);
      }
    }
    *(f32x4_t*)(rE + ly * LB_TX + x4) = re;
    *(f32x4_t*)(rH + ly * LB_TX + x4) = rh;
    *(f32x4_t*)(rC + ly * LB_TX + x4) = rc;
  }
  __syncthreads();
  const int ty = threadIdx.x >> 4, tx = threadIdx.x & 15;
  const int jy = vy0 + ty, jx0 = vx0 + 4 * tx;
  // row segment of kernel row i: staged columns 4 tx .. 4 tx + 2R + 3
  const float* hr0 = sh + ty * SX + 4 * tx;
  const float* cr0 = sc + ty * SX + 4 * tx;
  float e[4] = {0.f, 0.f, 0.f, 0.f}, mh[4] = {0.f, 0.f, 0.f, 0.f}, mc[4] = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
  for (int i = 0; i < 2 * RH + 1; ++i) {
    const f32x4_t v = *(const f32x4_t*)(rE + (ty + i + (R - RH)) * LB_TX + 4 * tx);
    const float g = win.g1[i];
#pragma unroll
    for (int k = 0; k < 4; ++k) e[k] = fmaf(g, v[k], e[k]);
  }
#pragma unroll
  for (int i = 0; i < 2 * RS + 1; ++i) {
    const f32x4_t vh4 = *(const f32x4_t*)(rH + (ty + i + (R - RS)) * LB_TX + 4 * tx);
    const f32x4_t vc4 = *(const f32x4_t*)(rC + (ty + i + (R - RS)) * LB_TX + 4 * tx);
    const float wv = win.w1[i];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      mh[k] = fmaf(wv, vh4[k], mh[k]);
      mc[k] = fmaf(wv, vc4[k], mc[k]);
    }
  }
  float vh[4] = {0.f, 0.f, 0.f, 0.f}, vc[4] = {0.f, 0.f, 0.f, 0.f}, cov[4] = {0.f, 0.f, 0.f, 0.f};
  if (q.levels == 2) {
    // binary h (0 or 1) and window weights summing to 1: var_h = mu_h (1 -
    // mu_h) and cov = sum w h (c - mu_c), the h - mu_h centring adding
    // mu_h sum w (c - mu_c) = 0; c stays centred for var_c and cov
#pragma unroll 1
    for (int i = R - RS; i <= R + RS; ++i) {
      const int wi = i - (R - RS);
      float hv[NS], cv[NS];
#pragma unroll
      for (int j = 0; j < NS; ++j) {
        hv[j] = hr0[i * SX + j];
        cv[j] = cr0[i * SX + j];
      }
#pragma unroll
      for (int j = 0; j < 2 * RS + 1; ++j) {
        const float wv = sw[wi * (2 * RS + 1) + j];
#pragma unroll
        for (int k = 0; k < 4; ++k) {
          const int p = k + j + (R - RS);
          const float dc = cv[p] - mc[k], wdc = wv * dc;
          vc[k] = fmaf(wdc, dc, vc[k]);
          cov[k] = fmaf(wdc, hv[p], cov[k]);
        }
      }
    }
#pragma unroll
    for (int k = 0; k < 4; ++k) vh[k] = mh[k] * (1.0f - mh[k]);
  } else {
#pragma unroll 1
    for (int i = R - RS; i <= R + RS; ++i) {
      const int wi = i - (R - RS);
      float hv[NS], cv[NS];
#pragma unroll
      for (int j = 0; j < NS; ++j) {
        hv[j] = hr0[i * SX + j];
        cv[j] = cr0[i * SX + j];
      }
#pragma unroll
      for (int j = 0; j < 2 * RS + 1; ++j) {
        const float wv = sw[wi * (2 * RS + 1) + j];
#pragma unroll
        for (int k = 0; k < 4; ++k) {
          const int p = k + j + (R - RS);
          const float dh = hv[p] - mh[k], dc = cv[p] - mc[k];
          vh[k] = fmaf(wv * dh, dh, vh[k]);
          vc[k] = fmaf(wv * dc, dc, vc[k]);
          cov[k] = fmaf(wv * dh, dc, cov[k]);
        }
      }
    }
  }
  float e2 = 0.0f, cs = 0.0f;
  const size_t n = (size_t)gridDim.z * H * W;
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    const int jx = jx0 + k;
    if (jy < H - R && jx < W - R) {
      const float ssim = ((2.0f * mh[k] * mc[k] + q.c1) * (2.0f * cov[k] + q.c2)) /
                         ((mh[k] * mh[k] + mc[k] * mc[k] + q.c1) * (vh[k] + vc[k] + q.c2));
      const float sig = q.k * sqrtf(vc[k]);
      e2 += e[k] * e[k];
      cs += sig * ssim + (1.0f - sig);
      if (maps) {
        const size_t o = img + (size_t)jy * W + jx;
        maps[o] = e[k];
        maps[n + o] = mh[k];
        maps[2 * n + o] = mc[k];
        maps[3 * n + o] = vc[k];
        maps[4 * n + o] = cov[k];
        if (q.levels > 2) maps[5 * n + o] = vh[k];
      }
    }
  }
  red[0][threadIdx.x] = e2;
  red[1][threadIdx.x] = cs;
  __syncthreads();
  // the four 16 x 16 tiles: thread t < 4 adds tile t's 64 threads in order
  const int tiles_x = (W - 2 * R + 15) / 16;
  if (threadIdx.x < 4) {
    const int tcol = blockIdx.x * 4 + threadIdx.x;
    if (tcol < tiles_x) {
      float a = 0.0f, d = 0.0f;
      for (int r = 0; r < 16; ++r)
        for (int u = 0; u < 4; ++u) {
          const int t = r * 16 + 4 * threadIdx.x + u;
          a += red[0][t];
          d += red[1][t];
        }
      float* dp = partials + ((size_t)b * ntiles_per_img + blockIdx.y * tiles_x + tcol) * 2;
      dp[0] = a;
      dp[1] = d;
    }
  }
}

__global__ void loss_reduce_kernel(const float* __restrict__ partials, int B, int ntiles,
                                   const float* __restrict__ as_partials, int npatch, float w_s,
                                   float invM, float* __restrict__ out) {
  __shared__ float red[2][4];
  const int b = blockIdx.x;
  float s0 = 0.0f, s1 = 0.0f;
  if (b < B) {
    for (int t = threadIdx.x; t < ntiles; t += 256) {
      s0 += partials[((size_t)b * ntiles + t) * 2];
      s1 += partials[((size_t)b * ntiles + t) * 2 + 1];
    }
  } else {
    for (int t = threadIdx.x; t < npatch; t += 256) s0 += as_partials[t];
  }
  s0 = hs_wave_sum(s0);
  s1 = hs_wave_sum(s1);
  const int wave = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 0) {
    red[0][wave] = s0;
    red[1][wave] = s1;
  }
  __syncthreads();
  if (threadIdx.x != 0) return;
  const float a = ((red[0][0] + red[0][1]) + red[0][2]) + red[0][3];
  const float cc = ((red[1][0] + red[1][1]) + red[1][2]) + red[1][3];
  if (b < B) {
    const float mse = a * invM, cssim = cc * invM;
    out[3 * b + 0] = mse;
    out[3 * b + 1] = cssim;
    out[3 * b + 2] = -mse + w_s * cssim;
  } else {
    out[3 * B] = npatch > 0 ? a / (float)npatch : 0.0f;
  }
}

// The total training loss of the batch, -mean_b R_b + w_a L_AS, after the
// per-image rewards and L_AS are in out (images summed in order).
__global__ void loss_total_kernel(int B, float w_a, float* __restrict__ out) {
  if (threadIdx.x != 0) return;
  float r = 0.0f;
  for (int b = 0; b < B; ++b) r += out[3 * b + 2];
  out[3 * B + 1] = -r / (float)B + w_a * out[3 * B];
}

// MULTI: multitone levels (q.levels > 2), with the var_h map; otherwise the
// binary form, whose var_h is mu_h (1 - mu_h)
template <bool MULTI>
__global__ __launch_bounds__(256) void le_grad_kernel(const uint8_t* __restrict__ h,
                                                      const float* __restrict__ c,
                                                      const float* __restrict__ probs,
                                                      int logit_space, int B, int H, int W,
                                                      LossConst q,
                                                      const hs::LossDev win,
                                                      const float* __restrict__ maps, float invM,
                                                      float* __restrict__ grad) {
  __shared__ float se[LS * LS], smh[LS * LS], smc[LS * LS], svc[LS * LS], scv[LS * LS],
      ssg[LS * LS];
  __shared__ float svh[MULTI ? LS * LS : 1];
  __shared__ float sG[15 * 15], sw[15 * 15];
  const int b = blockIdx.z, R = q.m;
  const int ay0 = blockIdx.y * LT, ax0 = blockIdx.x * LT;
  const size_t img = (size_t)b * H * W, n = (size_t)B * H * W;
  const int ls = LT + 2 * R;
  for (int i = threadIdx.x; i < 15 * 15; i += 256) {
    sG[i] = win.G[i];
    sw[i] = win.w[i];
  }
  for (int i = threadIdx.x; i < ls * ls; i += 256) {
    const int ly = i / ls, lx = i - ly * ls, gy = ay0 - R + ly, gx = ax0 - R + lx;
    const bool in = gy >= q.m && gy < H - q.m && gx >= q.m && gx < W - q.m;
    float v0 = 0.f, v1 = 0.f, v2 = 0.f, v3 = 0.f, v4 = 0.f, v5 = 0.f;
    if (in) {
      const size_t o = img + (size_t)gy * W + gx;
      v0 = maps[o];
      v1 = maps[n + o];
      v2 = maps[2 * n + o];
      v3 = maps[3 * n + o];
      v4 = maps[4 * n + o];
      if (MULTI) v5 = maps[5 * n + o];
    }
    se[i] = v0;
    smh[i] = v1;
    smc[i] = v2;
    svc[i] = v3;
    scv[i] = v4;
    ssg[i] = q.k * sqrtf(v3);
    if (MULTI) svh[i] = v5;
  }
  __syncthreads();
  const int ty = threadIdx.x >> 4, tx = threadIdx.x & 15;
  const int ay = ay0 + ty, ax = ax0 + tx;
  if (ay >= H || ax >= W) return;
  const size_t oa = img + (size_t)ay * W + ax;
  float delta = h[oa] ? -1.0f : 1.0f;
  const float ha = (float)h[oa] * q.hstep;
  if (MULTI) {
    const float t = probs[oa] * (float)(q.levels - 1);
    const int kf = min((int)floorf(t), q.levels - 2);
    delta = (int)h[oa] == kf ? q.hstep : -q.hstep;
  }
  const float ca = c[oa];
  const int cy = ty + R, cx = tx + R;
  const int nh = 2 * q.rh + 1, ns = 2 * q.rs + 1;
  float dmse = 0.0f;
  for (int i = -q.rh; i <= q.rh; ++i) {
    const int jy = ay + i;
    if (jy < q.m || jy >= H - q.m) continue;
    for (int j = -q.rh; j <= q.rh; ++j) {
      const int jx = ax + j;
      if (jx < q.m || jx >= W - q.m) continue;
      const float dG = delta * sG[(q.rh - i) * nh + (q.rh - j)];  // delta G_{a-j}
      dmse = fmaf(2.0f * dG, se[(cy + i) * ls + cx + j], fmaf(dG, dG, dmse));
    }
  }
  float dcs = 0.0f;
  for (int i = -q.rs; i <= q.rs; ++i) {
    const int jy = ay + i;
    if (jy < q.m || jy >= H - q.m) continue;
    for (int j = -q.rs; j <= q.rs; ++j) {
      const int jx = ax + j;
      if (jx < q.m || jx >= W - q.m) continue;
      const int p = (cy + i) * ls + cx + j;
      const float wa = sw[(q.rs - i) * ns + (q.rs - j)];  // w_{a-j}
      const float mh = smh[p], mc = smc[p];
      const float A = 2.0f * mh * mc + q.c1;
      const float Bc = 2.0f * scv[p] + q.c2;
      const float C = mh * mh + mc * mc + q.c1;
      const float D = (MULTI ? svh[p] : mh * (1.0f - mh)) + svc[p] + q.c2;
      const float dw = delta * wa;
      const float dA = 2.0f * dw * mc;
      const float dB = 2.0f * dw * (ca - mc);
      const float dC = dw * (2.0f * mh + dw);
      // binary: 2 h_a + delta = 1 for either toggle
      const float dD = dw * ((MULTI ? 2.0f * ha + delta : 1.0f) - 2.0f * mh - dw);
      const float num = C * D * (A * dB + Bc * dA + dA * dB) - A * Bc * (C * dD + D * dC + dC * dD);
      const float den = (C + dC) * (D + dD) * (C * D);
      // hardware reciprocal (1 ulp) instead of the IEEE division sequence
      dcs = fmaf(ssg[p], num * __builtin_amdgcn_rcpf(den), dcs);
    }
  }
  // the sign of the toggle: dR = R(upper) - R(lower)
  const float sgn = delta > 0.0f ? 1.0f : -1.0f;
  const float dR = sgn * (-dmse * invM + q.w_s * dcs * invM);
  float gv = -dR * (float)(q.levels - 1) / (float)B;
  if (q.est == HS_EST_COMA) {
    // score function times (R(h) - b_a) = (h_a ? (1 - p) : -p) dR: in logit
    // space (h_a - p)(R(h) - b_a), in probability space divided by p (h_a = 1)
    // or 1 - p (h_a = 0); a sampled h_a = 1 implies p > 0 and h_a = 0, p < 1
    const float pa = probs[oa];
    const bool one = h[oa] != 0;
    if (logit_space) gv *= one ? (1.0f - pa) * (1.0f - pa) : pa * pa;
    else gv *= one ? (1.0f - pa) / pa : pa / (1.0f - pa);
  } else if (logit_space) {
    gv *= probs[oa] * (1.0f - probs[oa]);
  }
  grad[oa] = gv;
}

// The binary form of le_grad_kernel for compile-time window radii RH and RS,
// register-blocked: a thread computes the gradient of four horizontally
// adjacent pixels. The HVS part, sum over valid centres j of 2 delta
// G_{a-j} e_j + G_{a-j}^2, is 2 delta (G * e)_a plus the sum of G^2 over
// the valid centres, both separable (G = g g^T, and the valid region is a
// rectangle): row sums of e into LDS, then column sums. For the SSIM part
// it walks each kernel row's segment of 4 + 2R window centres once, with
// the centre's own terms A, B = 2 cov + c2, C, D = var_h + var_c + c2,
// SSIM_j = A B / (C D), 2 mu_h and 2 mu_c staged once per block as float
// pairs, and for each of the up to
// four pixels whose windows hold the centre takes the toggled factors
// A', B', C', D' and the change A'B' / (C'D') - SSIM_j, in the same centre
// order as le_grad_kernel. (The difference of the two ratios has the FP32
// error of the cancellation-free form of le_grad_kernel: both are set by
// the rounding of the FP32 statistics, about 3e-7 of the largest change;
// it takes 14 instead of about 26 operations per term.) A centre outside
// the valid region has zero maps, zero sigma_c and a staged D of 1, so its
// SSIM term adds exactly zero. A block covers 16 x 64 pixels.
template <int RH, int RS>
__global__ __launch_bounds__(256) void le_grad_rb_kernel(const uint8_t* __restrict__ h,
                                                         const float* __restrict__ c,
                                                         const float* __restrict__ probs,
                                                         int logit_space, int B, int H, int W,
                                                         LossConst q, const hs::LossDev win,
                                                         const float* __restrict__ maps,
                                                         float invM, float* __restrict__ grad) {
  constexpr int R = RH > RS ? RH : RS, SY = LB_TY + 2 * R, SX = LB_TX + 2 * R;
  constexpr int NSW = 2 * RS + 1;
  // per staged centre: (A, C), (B, D), (e then SSIM_j, sigma_c), (2 mu_h,
  // 2 mu_c); e is replaced by SSIM_j once its row sums are taken
  __shared__ float2 sAC[SY * SX], sBD[SY * SX], sSG[SY * SX], sM2[SY * SX];
  __shared__ float sw[NSW * NSW];
  __shared__ __attribute__((aligned(16))) float rS[SY * LB_TX];  // row sums of g * e
  const int b = blockIdx.z;
  const int ay0 = blockIdx.y * LB_TY, ax0 = blockIdx.x * LB_TX;
  const size_t img = (size_t)b * H * W, n = (size_t)B * H * W;
  for (int i = threadIdx.x; i < NSW * NSW; i += 256) sw[i] = win.w[i];
  for (int i = threadIdx.x; i < SY * SX; i += 256) {
    const int ly = i / SX, lx = i - ly * SX, gy = ay0 - R + ly, gx = ax0 - R + lx;
    const bool in = gy >= q.m && gy < H - q.m && gx >= q.m && gx < W - q.m;
    float v0 = 0.f, v1 = 0.f, v2 = 0.f, v3 = 0.f, v4 = 0.f;
    if (in) {
      const size_t o = img + (size_t)gy * W + gx;
      v0 = maps[o];
      v1 = maps[n + o];
      v2 = maps[2 * n + o];
      v3 = maps[3 * n + o];
      v4 = maps[4 * n + o];
    }
    const float twomh = 2.0f * v1;
    sAC[i] = make_float2(fmaf(twomh, v2, q.c1), fmaf(v1, v1, fmaf(v2, v2, q.c1)));
    // binary: var_h = mu_h (1 - mu_h); outside the valid region D = 1 keeps
    // the toggled C'D' away from zero (such a centre's term has sigma_c = 0)
    sBD[i] = make_float2(fmaf(2.0f, v4, q.c2), in ? fmaf(v1, 1.0f - v1, v3 + q.c2) : 1.0f);
    sSG[i] = make_float2(v0, q.k * sqrtf(v3));
    sM2[i] = make_float2(twomh, 2.0f * v2);
  }
  __syncthreads();
  // row sums of g * e at the tile's pixel columns (item: a staged row and
  // four columns)
  for (int it = threadIdx.x; it < SY * (LB_TX / 4); it += 256) {
    const int ly = it / (LB_TX / 4), x4 = 4 * (it % (LB_TX / 4));
    f32x4_t rs = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int t = 0; t < 2 * RH + 4; ++t) {
      const float ev = sSG[ly * SX + x4 + (R - RH) + t].x;
#pragma unroll
      for (int k = 0; k < 4; ++k)
        if (t - k >= 0 && t - k <= 2 * RH) rs[k] = fmaf(win.g1[t - k], ev, rs[k]);
    }
    *(f32x4_t*)(rS + ly * LB_TX + x4) = rs;
  }
  __syncthreads();
  // SSIM_j of every staged centre
  for (int i = threadIdx.x; i < SY * SX; i += 256) {
    const float2 ac = sAC[i], bd = sBD[i];
    sSG[i].x = (ac.x * bd.x) * __builtin_amdgcn_rcpf(ac.y * bd.y);
  }
  __syncthreads();
  const int ty = threadIdx.x >> 4, tx = threadIdx.x & 15;
  const int ay = ay0 + ty, axb = ax0 + 4 * tx;
  if (ay >= H || axb >= W) return;
  float delta[4], tca[4];  // the toggle, 2 c_a
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    const bool ok = axb + k < W;
    const size_t oa = img + (size_t)ay * W + (ok ? axb + k : axb);
    delta[k] = h[oa] ? -1.0f : 1.0f;
    tca[k] = 2.0f * c[oa];
  }
  // HVS: 2 delta (G * e)_a + sum of G^2 over the valid centres (the product
  // of the valid rows' and the valid columns' sums of g^2)
  float dmse[4];
  {
    f32x4_t ge = {0.f, 0.f, 0.f, 0.f};
    float rowg2 = 0.0f;
#pragma unroll
    for (int i = 0; i <= 2 * RH; ++i) {
      const f32x4_t v = *(const f32x4_t*)(rS + (ty + (R - RH) + i) * LB_TX + 4 * tx);
      const float g = win.g1[i];
#pragma unroll
      for (int k = 0; k < 4; ++k) ge[k] = fmaf(g, v[k], ge[k]);
      const int jy = ay - RH + i;
      if (jy >= q.m && jy < H - q.m) rowg2 = fmaf(g, g, rowg2);
    }
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      float colg2 = 0.0f;
#pragma unroll
      for (int j = 0; j <= 2 * RH; ++j) {
        const int jx = axb + k - RH + j;
        if (jx >= q.m && jx < W - q.m) colg2 = fmaf(win.g1[j], win.g1[j], colg2);
      }
      dmse[k] = fmaf(2.0f * delta[k], ge[k], rowg2 * colg2);
    }
  }
  float dcs[4] = {0.f, 0.f, 0.f, 0.f};
#pragma unroll 1
  for (int i = -RS; i <= RS; ++i) {
    const int jy = ay + i;
    if (jy < q.m || jy >= H - q.m) continue;
    const int rowo = (ty + R + i) * SX + 4 * tx + (R - RS);
#pragma unroll
    for (int jc = 0; jc < 2 * RS + 4; ++jc) {
      const int p = rowo + jc;
      const float2 ac = sAC[p], bd = sBD[p], ss = sSG[p], m2 = sM2[p];
      const float A = ac.x, C = ac.y, Bc = bd.x, D = bd.y, S = ss.x, sg = ss.y;
      const float twomh = m2.x, tmc = m2.y;
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        const int jt = jc - k;
        if (jt < 0 || jt > 2 * RS) continue;
        const float wa = sw[(RS - i) * NSW + (2 * RS - jt)];
        const float dw = delta[k] * wa;  // the change of mu_h
        const float u = twomh + dw;
        const float A2 = fmaf(dw, tmc, A);                // + 2 dw mu_c
        const float B2 = fmaf(dw, tca[k] - tmc, Bc);      // + 2 dw (c_a - mu_c)
        const float C2 = fmaf(dw, u, C);                  // + dw (2 mu_h + dw)
        const float D2 = fmaf(dw, 1.0f - u, D);           // + dw (1 - 2 mu_h - dw)
        const float t = fmaf(A2 * B2, __builtin_amdgcn_rcpf(C2 * D2), -S);
        dcs[k] = fmaf(sg, t, dcs[k]);
      }
    }
  }
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    if (axb + k >= W) break;
    const size_t oa = img + (size_t)ay * W + axb + k;
    const float sgn = delta[k] > 0.0f ? 1.0f : -1.0f;
    const float dR = sgn * (-dmse[k] * invM + q.w_s * dcs[k] * invM);
    float gv = -dR / (float)B;
    if (q.est == HS_EST_COMA) {
      const float pa = probs[oa];
      const bool one = h[oa] != 0;
      if (logit_space) gv *= one ? (1.0f - pa) * (1.0f - pa) : pa * pa;
      else gv *= one ? (1.0f - pa) / pa : pa / (1.0f - pa);
    } else if (logit_space) {
      gv *= probs[oa] * (1.0f - probs[oa]);
    }
    grad[oa] = gv;
  }
}

constexpr int NRING = 24;

// Ring of frequency (u, v) of a 32 x 32 periodogram: the rho with
// (2 rho - 1)^2 <= 4 (ub^2 + vb^2) < (2 rho + 1)^2, ub = min(u, 32 - u).
constexpr int ring_of(int u, int v) {
  const int ub = u < 32 - u ? u : 32 - u, vb = v < 32 - v ? v : 32 - v;
  const int q4 = 4 * (ub * ub + vb * vb);
  int rho = 0;
  while ((2 * rho + 1) * (2 * rho + 1) <= q4) ++rho;
  return rho;
}

// The frequencies grouped by ring (row-major order inside a ring) and the
// ring of each frequency; the same for every patch, so built at compile time.
struct RingTable {
  unsigned short idx[1024];
  unsigned short start[NRING + 1];
  unsigned char ring[1024];
};

constexpr RingTable make_ring_table() {
  RingTable t{};
  for (int i = 0; i < 1024; ++i) t.ring[i] = (unsigned char)ring_of(i >> 5, i & 31);
  int n = 0;
  for (int r = 0; r < NRING; ++r) {
    t.start[r] = (unsigned short)n;
    for (int i = 0; i < 1024; ++i)
      if (t.ring[i] == r) t.idx[n++] = (unsigned short)i;
  }
  t.start[NRING] = (unsigned short)n;
  return t;
}

__constant__ RingTable kRings = make_ring_table();
static_assert(make_ring_table().start[NRING] == 1024, "every frequency lies in a ring");

__global__ __launch_bounds__(256) void as_kernel(const float* __restrict__ pg, int Bg, int Hg,
                                                 int Wg, float scale, int logit_space,
                                                 float* __restrict__ patch_loss,
                                                 float* __restrict__ grad) {
  __shared__ float x[32 * 33];
  __shared__ float rr[32 * 33], ri[32 * 33];  // row transforms, then inverse column pass
  __shared__ float xr[32 * 33], xi[32 * 33];  // spectrum X
  __shared__ float ph[32 * 32];
  __shared__ float cs[32], sn[32];
  __shared__ float ring_part[NRING][8];
  __shared__ float ring_mean[NRING];
  __shared__ float red[4];
  const int py = Hg / 32, px = Wg / 32;
  const int patch = blockIdx.x;
  const int b = patch / (py * px), rem = patch - b * py * px;
  const int oy = (rem / px) * 32, ox = (rem % px) * 32;
  const float* base = pg + (size_t)b * Hg * Wg + (size_t)oy * Wg + ox;
  const int t = threadIdx.x;
  if (t < 32) {
    float sv, cv;
    sincospif((float)t / 16.0f, &sv, &cv);  // angle 2 pi t / 32
    cs[t] = cv;
    sn[t] = sv;
  }
  for (int i = t; i < 1024; i += 256) x[(i >> 5) * 33 + (i & 31)] = base[(size_t)(i >> 5) * Wg + (i & 31)];
  __syncthreads();
  // forward transform along x: rr + i ri = sum_x x[y][x] e^{-2 pi i v x / 32}
  for (int i = t; i < 1024; i += 256) {
    const int y = i >> 5, v = i & 31;
    float sr = 0.f, si = 0.f;
    for (int xx = 0; xx < 32; ++xx) {
      const int k = (v * xx) & 31;
      const float val = x[y * 33 + xx];
      sr = fmaf(val, cs[k], sr);
      si = fmaf(-val, sn[k], si);
    }
    rr[y * 33 + v] = sr;
    ri[y * 33 + v] = si;
  }
  __syncthreads();
  // along y: X[u][v] = sum_y (rr + i ri)[y][v] e^{-2 pi i u y / 32}
  for (int i = t; i < 1024; i += 256) {
    const int u = i >> 5, v = i & 31;
    float sr = 0.f, si = 0.f;
    for (int y = 0; y < 32; ++y) {
      const int k = (u * y) & 31;
      const float a = rr[y * 33 + v], bb = ri[y * 33 + v];
      // (a + i bb)(cos - i sin)
      sr = fmaf(a, cs[k], fmaf(bb, sn[k], sr));
      si = fmaf(bb, cs[k], fmaf(-a, sn[k], si));
    }
    xr[u * 33 + v] = sr;
    xi[u * 33 + v] = si;
    ph[i] = (sr * sr + si * si) * (1.0f / 1024.0f);
  }
  __syncthreads();
  // ring means, fixed summation order: 8 interleaved partial sums per ring
  if (t < NRING * 8) {
    const int r = t >> 3, sub = t & 7;
    float s = 0.f;
    const int e = kRings.start[r + 1];
    for (int j = kRings.start[r] + sub; j < e; j += 8) s += ph[kRings.idx[j]];
    ring_part[r][sub] = s;
  }
  __syncthreads();
  if (t < NRING) {
    float s = 0.f;
    for (int k = 0; k < 8; ++k) s += ring_part[t][k];
    ring_mean[t] = s / (float)(kRings.start[t + 1] - kRings.start[t]);
  }
  __syncthreads();
  float lsum = 0.f;
  for (int i = t; i < 1024; i += 256) {
    const float d = ph[i] - ring_mean[kRings.ring[i]];
    lsum = fmaf(d, d, lsum);
    ph[i] = 2.0f * d;  // dL/dPhat
  }
  lsum = hs_wave_sum(lsum);
  if ((t & 63) == 0) red[t >> 6] = lsum;
  __syncthreads();
  if (t == 0) patch_loss[patch] = ((red[0] + red[1]) + red[2]) + red[3];
  if (!grad) return;
  // gradient: dL/dx = (2 / 1024) Re( sum_{u,v} g X e^{+2 pi i (u y + v x) / 32} )
  for (int i = t; i < 1024; i += 256) {
    const int u = i >> 5, v = i & 31;
    xr[u * 33 + v] *= ph[i];
    xi[u * 33 + v] *= ph[i];
  }
  __syncthreads();
  for (int i = t; i < 1024; i += 256) {  // inverse along u -> y
    const int y = i >> 5, v = i & 31;
    float sr = 0.f, si = 0.f;
    for (int u = 0; u < 32; ++u) {
      const int k = (u * y) & 31;
      const float a = xr[u * 33 + v], bb = xi[u * 33 + v];
      // (a + i bb)(cos + i sin)
      sr = fmaf(a, cs[k], fmaf(-bb, sn[k], sr));
      si = fmaf(bb, cs[k], fmaf(a, sn[k], si));
    }
    rr[y * 33 + v] = sr;
    ri[y * 33 + v] = si;
  }
  __syncthreads();
  float* gbase = grad + (size_t)b * Hg * Wg + (size_t)oy * Wg + ox;
  for (int i = t; i < 1024; i += 256) {  // inverse along v -> x, real part
    const int y = i >> 5, xx = i & 31;
    float sr = 0.f;
    for (int v = 0; v < 32; ++v) {
      const int k = (v * xx) & 31;
      sr = fmaf(rr[y * 33 + v], cs[k], fmaf(-ri[y * 33 + v], sn[k], sr));
    }
    float gv = sr * (2.0f / 1024.0f) * scale;
    if (logit_space) {
      const float p = x[y * 33 + xx];
      gv *= p * (1.0f - p);
    }
    gbase[(size_t)y * Wg + xx] = gv;
  }
}

__global__ void fill_kernel(float* __restrict__ p, size_t n, float v) {
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n;
       i += (size_t)gridDim.x * blockDim.x)
    p[i] = v;
}

}  // namespace

namespace hs {

void make_windows(const hs_loss_params& p, LossDev* out) {
  auto gauss = [](double sigma, int r, float* dst) {
    const int n = 2 * r + 1;
    double tmp[15 * 15], sum = 0.0;
    for (int i = -r; i <= r; ++i)
      for (int j = -r; j <= r; ++j) {
        const double v = exp(-(double)(i * i + j * j) / (2.0 * sigma * sigma));
        tmp[(i + r) * n + (j + r)] = v;
        sum += v;
      }
    for (int i = 0; i < 15 * 15; ++i) dst[i] = 0.0f;
    for (int i = 0; i < n * n; ++i) dst[i] = (float)(tmp[i] / sum);
  };
  gauss(p.hvs_sigma, p.hvs_radius, out->G);
  gauss(p.ssim_sigma, p.ssim_radius, out->w);
  // the 1-D factors: exp(-(i^2 + j^2) / 2 s^2) / Z = f_i f_j with f_i =
  // exp(-i^2 / 2 s^2) / sqrt(Z), sqrt(Z) the 1-D sum
  auto gauss1 = [](double sigma, int r, float* dst) {
    double tmp[15], sum = 0.0;
    for (int i = -r; i <= r; ++i) sum += (tmp[i + r] = exp(-(double)(i * i) / (2.0 * sigma * sigma)));
    for (int i = 0; i < 15; ++i) dst[i] = i < 2 * r + 1 ? (float)(tmp[i] / sum) : 0.0f;
  };
  gauss1(p.hvs_sigma, p.hvs_radius, out->g1);
  gauss1(p.ssim_sigma, p.ssim_radius, out->w1);
}

static LossConst make_const(const hs_loss_params& p) {
  LossConst q;
  q.rh = p.hvs_radius;
  q.rs = p.ssim_radius;
  q.m = p.hvs_radius > p.ssim_radius ? p.hvs_radius : p.ssim_radius;
  q.k = p.k;
  q.c1 = p.c1;
  q.c2 = p.c2;
  q.w_s = p.w_s;
  q.est = p.estimator;
  q.levels = p.levels < 2 ? 2 : p.levels;
  q.hstep = 1.0f / (float)(q.levels - 1);
  return q;
}

hipError_t launch_loss_stats(const uint8_t* h, const float* c, int B, int H, int W,
                             const hs_loss_params& p, const LossDev& win, float* maps,
                             float* tile_partials, int ntiles_per_img, hipStream_t s) {
  const LossConst q = make_const(p);
  const int vh = H - 2 * q.m, vw = W - 2 * q.m;
  if (q.rh == 5 && q.rs == 5) {  // the default windows
    const dim3 grid((vw + LB_TX - 1) / LB_TX, (vh + LB_TY - 1) / LB_TY, B);
    loss_stats_rb_kernel<5, 5><<<grid, 256, 0, s>>>(h, c, H, W, q, win, maps, tile_partials,
                                                    ntiles_per_img);
    return hipGetLastError();
  }
  const dim3 grid((vw + LT - 1) / LT, (vh + LT - 1) / LT, B);
  loss_stats_kernel<<<grid, 256, 0, s>>>(h, c, H, W, q, win, maps, tile_partials,
                                         ntiles_per_img);
  return hipGetLastError();
}

hipError_t launch_loss_reduce(const float* tile_partials, int B, int ntiles_per_img,
                              const float* as_partials, int npatch, float w_s, long M, float* out,
                              hipStream_t s) {
  loss_reduce_kernel<<<B + 1, 256, 0, s>>>(tile_partials, B, ntiles_per_img, as_partials, npatch,
                                           w_s, (float)(1.0 / (double)M), out);
  return hipGetLastError();
}

hipError_t launch_loss_total(int B, float w_a, float* out, hipStream_t s) {
  loss_total_kernel<<<1, 64, 0, s>>>(B, w_a, out);
  return hipGetLastError();
}

hipError_t launch_le_grad(const uint8_t* h, const float* c, const float* probs, int logit_space,
                          int B, int H, int W, const hs_loss_params& p, const LossDev& win,
                          const float* maps, float* grad, hipStream_t s) {
  const LossConst q = make_const(p);
  const long M = (long)(H - 2 * q.m) * (W - 2 * q.m);
  if (q.levels == 2 && q.rh == 5 && q.rs == 5) {  // binary, the default windows
    const dim3 grid((W + LB_TX - 1) / LB_TX, (H + LB_TY - 1) / LB_TY, B);
    le_grad_rb_kernel<5, 5><<<grid, 256, 0, s>>>(h, c, probs, logit_space, B, H, W, q, win, maps,
                                                 (float)(1.0 / (double)M), grad);
    return hipGetLastError();
  }
  const dim3 grid((W + LT - 1) / LT, (H + LT - 1) / LT, B);
  auto kern = q.levels > 2 ? le_grad_kernel<true> : le_grad_kernel<false>;
  kern<<<grid, 256, 0, s>>>(h, c, probs, logit_space, B, H, W, q, win, maps,
                                      (float)(1.0 / (double)M), grad);
  return hipGetLastError();
}

hipError_t launch_as(const float* pg, int Bg, int Hg, int Wg, float scale, int logit_space,
                     float* patch_loss, float* grad_or_null, hipStream_t s) {
  const int npatch = Bg * (Hg / 32) * (Wg / 32);
  if (npatch == 0) return hipSuccess;
  as_kernel<<<npatch, 256, 0, s>>>(pg, Bg, Hg, Wg, scale, logit_space, patch_loss, grad_or_null);
  return hipGetLastError();
}

hipError_t launch_fill(float* p, size_t n, float v, hipStream_t s) {
  if (n == 0) return hipSuccess;
  size_t blocks = (n + 255) / 256;
  if (blocks > 4096) blocks = 4096;
  fill_kernel<<<(unsigned)blocks, 256, 0, s>>>(p, n, v);
  return hipGetLastError();
}

}  // namespace hs
