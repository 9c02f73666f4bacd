// conv.hip -- the policy's conv stack on gfx950, one layer per launch.
//
// The policy (Sec. VI-A of the paper, with the 6 x 32 geometry of this
// library) is 3x3 conv 2->32, four 3x3 conv 32->32, 3x3 conv 32->1, zero
// 'same' padding, ReLU after all but the last, sigmoid head. Activations are
// NHWC with 32 channels (BF16 or FP32). The 32->32 layers are implicit GEMMs
// on the matrix cores: D[cout][pixel] = sum over taps of W_tap[cout][cin] x
// act[pixel + tap][cin], with the weights as the A operand (held in
// registers) and 16-pixel runs of the LDS-staged input tile as the B
// operand. The input gradient of a layer is the same conv with weights
// transposed in (cin, cout) and flipped in the taps. Weight gradients are
// reductions over pixels with one row of partial sums per block, summed in
// a fixed order afterwards (deterministic).
#include "hs_common.h"
#include "hs_internal.h"

namespace {

// ---------------------------------------------------------------------------
// Weight packing into MFMA A-operand order [tap][row tile][lane][8].
// forward:    element (t, m, l, j) = W[16m + l%16][8(l/16) + j][t]
// transposed: element (t, m, l, j) = W[8(l/16) + j][16m + l%16][8 - t]
// ---------------------------------------------------------------------------
// blockIdx.y + y0 = 4 x (transposed) + layer, layer 0..3 being conv layer 2..5;
// the forward copy goes to outF, the transposed one to outT.
template <typename T>
__global__ void pack32_kernel(const float* __restrict__ w, T* __restrict__ outF,
                              T* __restrict__ outT, int y0) {
  const int y = blockIdx.y + y0, layer = y & 3, transposed = y >> 2;
  T* __restrict__ out = transposed ? outT : outF;
  const float* Wk = w + hs_wk(layer + 2);
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < hs::PACK32_PER_LAYER;
       i += gridDim.x * blockDim.x) {
    const int j = i & 7, l = (i >> 3) & 63, m = (i >> 9) & 1, t = i >> 10;
    const int r = l & 15, g = l >> 4;
    const float v = transposed ? Wk[((8 * g + j) * 32 + 16 * m + r) * 9 + (8 - t)]
                               : Wk[((16 * m + r) * 32 + 8 * g + j) * 9 + t];
    out[layer * hs::PACK32_PER_LAYER + i] = hs_from_f<T>(v);
  }
}

// B-operand fragment of lane group g (channels 8g..8g+7) of the pixel stored
// at `px` (LDS column `col`) in a chunk-swizzled tile.
HS_DEV void lds_frag(frag8<__bf16>& f, const __bf16* px, int col, int g) {
  f.v = *(const bf16x8_t*)(px + hs_swz<__bf16>(col, g) * 8);
}
HS_DEV void lds_frag(frag8<float>& f, const float* px, int col, int g) {
  f.lo = *(const f32x4_t*)(px + hs_swz<float>(col, 2 * g) * 4);
  f.hi = *(const f32x4_t*)(px + hs_swz<float>(col, 2 * g + 1) * 4);
}

// ---------------------------------------------------------------------------
// 32 -> 32 conv layer. Block = 4 waves over a (4 RPW) x 64 pixel tile; wave
// w owns tile rows RPW w .. RPW w + RPW - 1 as four 16-pixel runs each, both
// 16-channel row tiles of the output. With two rows per wave (BF16) every
// staged input row fragment feeds both output rows (taps dy and dy - 1), so
// a wave reads 4 x 3 x 4 fragments from LDS for 144 MFMAs instead of
// 2 x 36 for the same work; each output still sums its taps in the order
// t = 0..8. MODE 0: + bias, ReLU.  MODE 1: x [mask > 0] (input gradient
// through ReLU).
// ---------------------------------------------------------------------------
constexpr int CT_W = 64, CL_W = CT_W + 2;
template <typename T>
struct conv_rows {
  static constexpr int RPW = sizeof(T) == 2 ? 2 : 1;  // output rows per wave
  static constexpr int CT_H = 4 * RPW, CL_H = CT_H + 2;
};

template <typename T, int MODE>
__global__ __launch_bounds__(256) void conv32_kernel(const T* __restrict__ in,
                                                     const T* __restrict__ wp,
                                                     const float* __restrict__ bias,
                                                     const T* __restrict__ mask,
                                                     T* __restrict__ out, int H, int W) {
  constexpr int CPP = act_traits<T>::chunks_per_px, EPC = act_traits<T>::elems_per_chunk;
  constexpr int RPW = conv_rows<T>::RPW, CT_H = conv_rows<T>::CT_H, CL_H = conv_rows<T>::CL_H;
  __shared__ __attribute__((aligned(16))) T lds[CL_H * CL_W * 32];
  const int b = blockIdx.z, y0 = blockIdx.y * CT_H, x0 = blockIdx.x * CT_W;
  const size_t img = (size_t)b * H * W;
  // all of the tile's 16-byte loads are issued before the first LDS store
  constexpr int NCH = CL_H * CL_W * CPP, NIT = (NCH + 255) / 256;
  uint4 v[NIT];
#pragma unroll
  for (int k = 0; k < NIT; ++k) {
    const int i = (int)threadIdx.x + 256 * k;
    const int p = i / CPP, c = i - p * CPP;
    const int ly = p / CL_W, lx = p - ly * CL_W;
    const int gy = y0 + ly - 1, gx = x0 + lx - 1;
    v[k] = make_uint4(0u, 0u, 0u, 0u);
    if (i < NCH && gy >= 0 && gy < H && gx >= 0 && gx < W)
      v[k] = *(const uint4*)(in + (img + (size_t)gy * W + gx) * 32 + c * EPC);
  }
#pragma unroll
  for (int k = 0; k < NIT; ++k) {
    const int i = (int)threadIdx.x + 256 * k;
    const int p = i / CPP, c = i - p * CPP;
    const int lx = p - (p / CL_W) * CL_W;
    if (i < NCH) *(uint4*)(lds + p * 32 + hs_swz<T>(lx, c) * EPC) = v[k];
  }
  __syncthreads();
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, g = lane >> 4, r = lane & 15;
  f32x4_t acc[RPW][2][4];
#pragma unroll
  for (int q = 0; q < RPW; ++q)
#pragma unroll
    for (int m = 0; m < 2; ++m)
#pragma unroll
      for (int n = 0; n < 4; ++n) acc[q][m][n] = f32x4_t{0.f, 0.f, 0.f, 0.f};
  // input row RPW w + d (d = 0..RPW+1) feeds output row q with tap dy = d - q
#pragma unroll
  for (int d = 0; d < RPW + 2; ++d) {
#pragma unroll
    for (int dx = 0; dx < 3; ++dx) {
      frag8<T> a[RPW][2];
#pragma unroll
      for (int q = 0; q < RPW; ++q) {
        const int dy = d - q;
        if (dy < 0 || dy > 2) continue;
        const int t = dy * 3 + dx;
        hs_load_frag(a[q][0], wp + ((t * 2 + 0) * 64 + lane) * 8);
        hs_load_frag(a[q][1], wp + ((t * 2 + 1) * 64 + lane) * 8);
      }
#pragma unroll
      for (int n = 0; n < 4; ++n) {
        const int lx = n * 16 + r + dx, ly = RPW * wave + d;
        frag8<T> bf;
        lds_frag(bf, lds + (ly * CL_W + lx) * 32, lx, g);
#pragma unroll
        for (int q = 0; q < RPW; ++q) {
          const int dy = d - q;
          if (dy < 0 || dy > 2) continue;
          acc[q][0][n] = hs_mma(a[q][0], bf, acc[q][0][n]);
          acc[q][1][n] = hs_mma(a[q][1], bf, acc[q][1][n]);
        }
      }
    }
  }
#pragma unroll
  for (int q = 0; q < RPW; ++q) {
    const int gy = y0 + RPW * wave + q;
    if (gy >= H) break;
#pragma unroll
    for (int n = 0; n < 4; ++n) {
      const int gx = x0 + n * 16 + r;
      if (gx >= W) continue;
      const size_t o = (img + (size_t)gy * W + gx) * 32;
#pragma unroll
      for (int m = 0; m < 2; ++m) {
        const int co = 16 * m + 4 * g;
        float vv[4];
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          vv[i] = acc[q][m][n][i];
          if (MODE == 0) {
            vv[i] = fmaxf(vv[i] + bias[co + i], 0.0f);
          } else {
            vv[i] = hs_to_f(mask[o + co + i]) > 0.0f ? vv[i] : 0.0f;
          }
        }
        hs_store4(out + o + co, vv[0], vv[1], vv[2], vv[3]);
      }
    }
  }
}

// ---------------------------------------------------------------------------
// The forward 32 -> 32 layer on BF16 activations as a persistent kernel: the
// tiles, fragments and MFMA order of conv32_kernel (each output sums its taps
// t = 0..8 in order, bias first), with the layer's 18 weight fragments and
// the lane's biases held in registers for the whole kernel and the next
// tile's loads issued before this tile's matrix work, so that the loads of
// one tile overlap the MFMAs of the previous one. Staging is arranged to cost
// few vector instructions: thread (column sc, chunk c) loads column sc of
// the tile's ten staged rows (threads < 80 also one of the two extra
// columns) from clamped, always valid addresses, and positions outside the
// image are zeroed when the registers are stored to LDS; the row checks
// are uniform over the block. Two blocks per CU.
// ---------------------------------------------------------------------------
constexpr int CF_BLOCKS = 512;  // 2 per CU on 256 CUs

__global__ __launch_bounds__(256, 2) void conv32_fwd_bf16_kernel(
    const __bf16* __restrict__ in, const __bf16* __restrict__ wp, const float* __restrict__ bias,
    __bf16* __restrict__ out, int B, int H, int W) {
  constexpr int RPW = conv_rows<__bf16>::RPW, CT_H = conv_rows<__bf16>::CT_H;
  constexpr int CL_H = conv_rows<__bf16>::CL_H;
  constexpr int NEX = CL_H * 2 * 4;  // chunks of the two extra columns
  static_assert(CT_W == 64 && CL_W == 66 && NEX <= 256, "staging assumes 64 + 2 columns");
  __shared__ __attribute__((aligned(16))) __bf16 lds[CL_H * CL_W * 32];
  const int tiles_x = (W + CT_W - 1) / CT_W, tiles_y = (H + CT_H - 1) / CT_H;
  const int ntiles = B * tiles_x * tiles_y;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, g = lane >> 4, r = lane & 15;
  frag8<__bf16> wf[9][2];
#pragma unroll
  for (int t = 0; t < 9; ++t)
#pragma unroll
    for (int m = 0; m < 2; ++m) hs_load_frag(wf[t][m], wp + ((t * 2 + m) * 64 + lane) * 8);
  float bv[2][4];
#pragma unroll
  for (int m = 0; m < 2; ++m)
#pragma unroll
    for (int i = 0; i < 4; ++i) bv[m][i] = bias[16 * m + 4 * g + i];
  // staging geometry (element offsets in LDS of staged row 0)
  const int c = threadIdx.x & 3, sc = threadIdx.x >> 2;
  const int st_off = sc * 32 + hs_swz<__bf16>(sc, c) * 8;
  const bool has_ex = (int)threadIdx.x < NEX;
  const int ex_ly = (int)threadIdx.x >> 3, ex_lx = CT_W + (((int)threadIdx.x >> 2) & 1);
  const int ex_off = (ex_ly * CL_W + ex_lx) * 32 + hs_swz<__bf16>(ex_lx, c) * 8;
  // B-fragment offsets of this lane for dx = 0, 1, 2 (the swizzle depends on
  // the column's bits 1..2, which the run offset n * 16 leaves alone)
  int boff[3];
#pragma unroll
  for (int dx = 0; dx < 3; ++dx) boff[dx] = (r + dx) * 32 + hs_swz<__bf16>(r + dx, g) * 8;
  uint4 v[CL_H], vx;
  auto load = [&](int tile) {
    const int b = tile / (tiles_x * tiles_y), rem = tile - b * tiles_x * tiles_y;
    const int y0 = (rem / tiles_x) * CT_H, x0 = (rem % tiles_x) * CT_W;
    const __bf16* base = in + (size_t)b * H * W * 32 + c * 8;
    const int gxc = min(max(x0 + sc - 1, 0), W - 1);
#pragma unroll
    for (int ly = 0; ly < CL_H; ++ly) {
      const int gyc = min(max(y0 + ly - 1, 0), H - 1);
      v[ly] = *(const uint4*)(base + ((size_t)gyc * W + gxc) * 32);
    }
    const int eyc = min(max(y0 + ex_ly - 1, 0), H - 1), exc = min(x0 + ex_lx - 1, W - 1);
    vx = *(const uint4*)(base + ((size_t)eyc * W + exc) * 32);
  };
  if ((int)blockIdx.x < ntiles) load(blockIdx.x);
  for (int tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
    const int b = tile / (tiles_x * tiles_y), rem = tile - b * tiles_x * tiles_y;
    const int y0 = (rem / tiles_x) * CT_H, x0 = (rem % tiles_x) * CT_W;
    __syncthreads();  // the previous tile's LDS reads are done
    {
      const int gx = x0 + sc - 1;
      const bool xin = gx >= 0 && gx < W;
#pragma unroll
      for (int ly = 0; ly < CL_H; ++ly) {
        const int gy = y0 + ly - 1;
        const bool in_img = xin && gy >= 0 && gy < H;
        const uint32_t k = in_img ? ~0u : 0u;
        *(uint4*)(lds + st_off + ly * CL_W * 32) =
            make_uint4(v[ly].x & k, v[ly].y & k, v[ly].z & k, v[ly].w & k);
      }
      const int ey = y0 + ex_ly - 1, ex = x0 + ex_lx - 1;
      const uint32_t k = (ey >= 0 && ey < H && ex < W) ? ~0u : 0u;
      if (has_ex) *(uint4*)(lds + ex_off) = make_uint4(vx.x & k, vx.y & k, vx.z & k, vx.w & k);
    }
    __syncthreads();
    if (tile + (int)gridDim.x < ntiles) load(tile + gridDim.x);
    f32x4_t acc[RPW][2][4];
#pragma unroll
    for (int q = 0; q < RPW; ++q)
#pragma unroll
      for (int m = 0; m < 2; ++m)
#pragma unroll
        for (int n = 0; n < 4; ++n) acc[q][m][n] = f32x4_t{bv[m][0], bv[m][1], bv[m][2], bv[m][3]};
#pragma unroll
    for (int d = 0; d < RPW + 2; ++d) {
#pragma unroll
      for (int dx = 0; dx < 3; ++dx) {
#pragma unroll
        for (int n = 0; n < 4; ++n) {
          frag8<__bf16> bf;
          bf.v = *(const bf16x8_t*)(lds + boff[dx] + ((RPW * wave + d) * CL_W + n * 16) * 32);
#pragma unroll
          for (int q = 0; q < RPW; ++q) {
            const int dy = d - q;
            if (dy < 0 || dy > 2) continue;
            acc[q][0][n] = hs_mma(wf[dy * 3 + dx][0], bf, acc[q][0][n]);
            acc[q][1][n] = hs_mma(wf[dy * 3 + dx][1], bf, acc[q][1][n]);
          }
        }
      }
    }
    const bool full_x = x0 + CT_W <= W;
#pragma unroll
    for (int q = 0; q < RPW; ++q) {
      const int gy = y0 + RPW * wave + q;
      if (gy >= H) break;
      __bf16* rowp = out + (((size_t)b * H + gy) * W + x0 + r) * 32 + 4 * g;
#pragma unroll
      for (int n = 0; n < 4; ++n) {
        if (!full_x && x0 + n * 16 + r >= W) continue;
#pragma unroll
        for (int m = 0; m < 2; ++m)
          hs_store4(rowp + n * 16 * 32 + 16 * m, fmaxf(acc[q][m][n][0], 0.0f),
                    fmaxf(acc[q][m][n][1], 0.0f), fmaxf(acc[q][m][n][2], 0.0f),
                    fmaxf(acc[q][m][n][3], 0.0f));
      }
    }
  }
}

// ---------------------------------------------------------------------------
// First layer 2 -> 32 on the state s = (c, z); z from Philox stream 1.
// 16 x 16 pixel tile per block, one pixel per thread, 32 outputs each.
// ---------------------------------------------------------------------------
template <typename T>
__global__ __launch_bounds__(256) void conv_first_kernel(const float* __restrict__ contone,
                                                         const uint64_t* __restrict__ seeds,
                                                         const float* __restrict__ w, int H,
                                                         int W, int kind, uint32_t step,
                                                         T* __restrict__ out,
                                                         float* __restrict__ zout,
                                                         float* __restrict__ cout) {
  // weights as [tap][co][channel c, z], so one 16-byte LDS read brings the
  // four weights of two output channels (the same for every lane)
  __shared__ __attribute__((aligned(16))) float swt[9 * 32 * 2];
  __shared__ float sc[18 * 18], sz[18 * 18], sb[32];
  const int b = blockIdx.z, y0 = blockIdx.y * 16, x0 = blockIdx.x * 16;
  const size_t img = (size_t)b * H * W;
  const uint64_t seed = seeds[b];
  for (int i = threadIdx.x; i < 32 * 2 * 9; i += 256) {
    const int co = i / 18, ch = (i / 9) % 2, t = i % 9;  // source W1[co][ch][t]
    swt[(t * 32 + co) * 2 + ch] = w[HS_W1 + i];
  }
  if (threadIdx.x < 32) sb[threadIdx.x] = w[HS_B1 + threadIdx.x];
  for (int i = threadIdx.x; i < 18 * 18; i += 256) {
    const int ly = i / 18, lx = i - ly * 18, gy = y0 + ly - 1, gx = x0 + lx - 1;
    float cv = 0.0f, zv = 0.0f;
    if (gy >= 0 && gy < H && gx >= 0 && gx < W) {
      const uint64_t a = (uint64_t)gy * W + gx;
      cv = contone[img + a];
      zv = hs_noise<true>(seed, a, step, kind);
    }
    sc[i] = cv;
    sz[i] = zv;
  }
  __syncthreads();
  const int ty = threadIdx.x >> 4, tx = threadIdx.x & 15, gy = y0 + ty, gx = x0 + tx;
  if (gy >= H || gx >= W) return;
  if (zout) zout[img + (size_t)gy * W + gx] = sz[(ty + 1) * 18 + tx + 1];
  if (cout) cout[img + (size_t)gy * W + gx] = sc[(ty + 1) * 18 + tx + 1];
  float acc[32];
#pragma unroll
  for (int co = 0; co < 32; ++co) acc[co] = sb[co];
#pragma unroll
  for (int t = 0; t < 9; ++t) {
    const int dy = t / 3, dx = t - (t / 3) * 3;
    const float c = sc[(ty + dy) * 18 + tx + dx], z = sz[(ty + dy) * 18 + tx + dx];
#pragma unroll
    for (int co = 0; co < 32; co += 2) {
      const f32x4_t q = *(const f32x4_t*)(swt + (t * 32 + co) * 2);
      acc[co] = fmaf(q[1], z, fmaf(q[0], c, acc[co]));
      acc[co + 1] = fmaf(q[3], z, fmaf(q[2], c, acc[co + 1]));
    }
  }
  T* o = out + (img + (size_t)gy * W + gx) * 32;
#pragma unroll
  for (int co = 0; co < 32; co += 4)
    hs_store4(o + co, fmaxf(acc[co], 0.f), fmaxf(acc[co + 1], 0.f), fmaxf(acc[co + 2], 0.f),
              fmaxf(acc[co + 3], 0.f));
}

// ---------------------------------------------------------------------------
// First layer 2 -> 32 of the training forward on BF16 activations, on the
// FP32 matrix cores: a1[px][co] = relu(sum_k W[co][k] U[k][px]), where column
// k = 9 ci + t (k < 18) takes U = s_ci[px + tap t] (s_0 the contone, s_1 the
// noise z of Philox stream 1), column 18 takes U = 1 against the bias and
// column 19 is zero: five K-steps of four. The products are FP32 as in the
// per-pixel form, so the BF16 rounding of a1 sees the same values up to
// FP32 summation order. The weight rows are permuted so that lane (g, r) of
// the two results holds channels 8 g .. 8 g + 7 of pixel r: one 16-byte
// store. A block computes 16 x 64 pixels from the state of its 18 x 66
// window, staged in LDS.
// ---------------------------------------------------------------------------
constexpr int CFM_TY = 16, CFM_TX = 64, CFM_SX = CFM_TX + 2, CFM_SN = (CFM_TY + 2) * CFM_SX;
constexpr int CFM_RUNS = CFM_TY * CFM_TX / 16 / 4;  // 16-pixel runs per wave

__global__ __launch_bounds__(256) void conv_first_mfma_kernel(
    const float* __restrict__ contone, const uint64_t* __restrict__ seeds,
    const float* __restrict__ w, int H, int W, int kind, uint32_t step,
    __bf16* __restrict__ out, float* __restrict__ zout, float* __restrict__ cout) {
  __shared__ float sst[2 * CFM_SN + 2];  // contone, noise; then the constants 1 and 0
  const int b = blockIdx.z, y0 = blockIdx.y * CFM_TY, x0 = blockIdx.x * CFM_TX;
  const size_t img = (size_t)b * H * W;
  const uint64_t seed = seeds[b];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, g = lane >> 4, r = lane & 15;
  // K-step q: lane (g, r) holds A[r][k] and B[k][r] with k = 4 q + g; row r of
  // tile c is channel 8 (r / 4) + 4 c + r % 4
  float wa[2][5];
  int off[5], stp[5];
#pragma unroll
  for (int q = 0; q < 5; ++q) {
    const int k = 4 * q + g, ci = k / 9, t = k - 9 * ci;
#pragma unroll
    for (int c = 0; c < 2; ++c) {
      const int co = 8 * (r >> 2) + 4 * c + (r & 3);
      wa[c][q] = k < 18 ? w[HS_W1 + co * 18 + k] : k == 18 ? w[HS_B1 + co] : 0.0f;
    }
    off[q] = k < 18 ? ci * CFM_SN + (t / 3) * CFM_SX + t % 3 : k == 18 ? 2 * CFM_SN : 2 * CFM_SN + 1;
    stp[q] = k < 18 ? 1 : 0;
  }
  for (int i = threadIdx.x; i < CFM_SN; i += 256) {
    const int sy = i / CFM_SX, sx = i - sy * CFM_SX, gy = y0 + sy - 1, gx = x0 + sx - 1;
    float cv = 0.0f, zv = 0.0f;
    if (gy >= 0 && gy < H && gx >= 0 && gx < W) {
      const uint64_t a = (uint64_t)gy * W + gx;
      cv = contone[img + a];
      zv = hs_noise<true>(seed, a, step, kind);
      if (sy >= 1 && sy <= CFM_TY && sx >= 1 && sx <= CFM_TX) {
        if (zout) zout[img + a] = zv;
        if (cout) cout[img + a] = cv;
      }
    }
    sst[i] = cv;
    sst[CFM_SN + i] = zv;
  }
  if (threadIdx.x == 0) {
    sst[2 * CFM_SN] = 1.0f;
    sst[2 * CFM_SN + 1] = 0.0f;
  }
  __syncthreads();
#pragma unroll 2
  for (int n = 0; n < CFM_RUNS; ++n) {
    const int run = wave + 4 * n, ly = run >> 2, lx = (run & 3) * 16 + r;
    const int pos = ly * CFM_SX + lx;
    float u[5];
#pragma unroll
    for (int q = 0; q < 5; ++q) u[q] = sst[off[q] + pos * stp[q]];
    f32x4_t acc[2];
#pragma unroll
    for (int c = 0; c < 2; ++c) {
      acc[c] = f32x4_t{0.f, 0.f, 0.f, 0.f};
#pragma unroll
      for (int q = 0; q < 5; ++q)
        acc[c] = __builtin_amdgcn_mfma_f32_16x16x4f32(wa[c][q], u[q], acc[c], 0, 0, 0);
    }
    const int gy = y0 + ly, gx = x0 + lx;
    if (gy < H && gx < W) {
      bf16x8_t o;
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        o[e] = (__bf16)fmaxf(acc[0][e], 0.0f);
        o[4 + e] = (__bf16)fmaxf(acc[1][e], 0.0f);
      }
      *(bf16x8_t*)(out + (img + (size_t)gy * W + gx) * 32 + 8 * g) = o;
    }
  }
}

__device__ __forceinline__ uint32_t split_bf16(float v) {
  const __bf16 hi = (__bf16)v, lo = (__bf16)(v - (float)hi);
  return (uint32_t)__builtin_bit_cast(unsigned short, hi) |
         ((uint32_t)__builtin_bit_cast(unsigned short, lo) << 16);
}

// ---------------------------------------------------------------------------
// Last layer 32 -> 1 and the head. MODE 0: bit = [x >= 0] (+ logit), or
// with multitone levels (lv.n > 1) the level of x among lv's thresholds.
// MODE 1: p = sigmoid(x), action = [u < p] with u from stream 0 at `step`;
// with L = lv.n + 1 > 2 levels the index kf + [u < q] of the stochastic
// rounding between the levels around p (Sec. VI-E, its unnumbered rounding equation):
// kf = min(floor(p (L-1)), L-2), q = p (L-1) - kf.
// ---------------------------------------------------------------------------
constexpr int LP = 33;  // padded pixel stride (floats) of the staged tile

template <typename T, int MODE>
__global__ __launch_bounds__(256) void conv_last_kernel(const T* __restrict__ in,
                                                        const float* __restrict__ w, int H, int W,
                                                        const uint64_t* __restrict__ seeds,
                                                        uint32_t step, uint8_t* __restrict__ bits,
                                                        float* __restrict__ logits,
                                                        float* __restrict__ probs, float tau,
                                                        uint32_t* __restrict__ list,
                                                        int* __restrict__ count,
                                                        const hs::Levels lv) {
  // staged positions 16-byte aligned (stride LQ = 36 floats: the 16 lanes of
  // a tile row read 16 distinct groups of 4 banks), weights as [tap][ci]
  constexpr int LQ = 36;
  __shared__ __attribute__((aligned(16))) float s[18 * 18 * LQ];
  __shared__ __attribute__((aligned(16))) float sw[9 * 32 + 4];
  const int b = blockIdx.z, y0 = blockIdx.y * 16, x0 = blockIdx.x * 16;
  const size_t img = (size_t)b * H * W;
  for (int i = threadIdx.x; i < 32 * 9; i += 256) sw[(i % 9) * 32 + i / 9] = w[HS_W6 + i];
  if (threadIdx.x == 0) sw[9 * 32] = w[HS_B6];
  for (int i = threadIdx.x; i < 18 * 18 * 8; i += 256) {
    const int p = i >> 3, q = (i & 7) * 4;
    const int ly = p / 18, lx = p - ly * 18, gy = y0 + ly - 1, gx = x0 + lx - 1;
    float v[4] = {0.f, 0.f, 0.f, 0.f};
    if (gy >= 0 && gy < H && gx >= 0 && gx < W) {
      const T* src = in + (img + (size_t)gy * W + gx) * 32 + q;
#pragma unroll
      for (int k = 0; k < 4; ++k) v[k] = hs_to_f(src[k]);
    }
    *(f32x4_t*)(s + p * LQ + q) = f32x4_t{v[0], v[1], v[2], v[3]};
  }
  __syncthreads();
  const int ty = threadIdx.x >> 4, tx = threadIdx.x & 15, gy = y0 + ty, gx = x0 + tx;
  if (gy >= H || gx >= W) return;
  float x = sw[32 * 9];
#pragma unroll
  for (int t = 0; t < 9; ++t) {
    const int dy = t / 3, dx = t - (t / 3) * 3;
    const float* sp = s + ((ty + dy) * 18 + tx + dx) * LQ;
#pragma unroll
    for (int c4 = 0; c4 < 32; c4 += 4) {
      const f32x4_t a = *(const f32x4_t*)(sp + c4);
      const f32x4_t wv = *(const f32x4_t*)(sw + t * 32 + c4);
      x = fmaf(wv[0], a[0], x);
      x = fmaf(wv[1], a[1], x);
      x = fmaf(wv[2], a[2], x);
      x = fmaf(wv[3], a[3], x);
    }
  }
  const size_t o = img + (size_t)gy * W + gx;
  if (MODE == 0) {
    float dist;
    int side;
    bits[o] = (uint8_t)hs::level_of(lv, x, &dist, &side);
    if (logits) logits[o] = x;
    if (list && dist < tau) list[atomicAdd(count, 1)] = (uint32_t)o;
  } else {
    const float p = hs_sigmoid(x);
    probs[o] = p;
    if (bits) {
      const float u = hs_action_u(seeds[b], (uint64_t)gy * W + gx, step);
      if (lv.n == 1) {
        bits[o] = u < p ? 1 : 0;
      } else {
        const float t = p * (float)lv.n;
        const int kf = min((int)floorf(t), lv.n - 1);
        bits[o] = (uint8_t)(kf + (u < t - (float)kf ? 1 : 0));
      }
    }
  }
}

// ---------------------------------------------------------------------------
// Layer 6 and the head of the training forward (MODE 1 of conv_last_kernel)
// on BF16 activations, on the matrix cores: one MFMA pair per 16-pixel run
// of the tile and its halo gives the nine taps' 32-channel sums
// T[tap][pixel] = sum_ci W6[ci][tap] a5[pixel][ci] (the FP32 weights split
// into BF16 hi + lo parts, about 16 significant bits; a5 is BF16 already),
// and each output adds its neighbours' taps, x = b6 + sum_t T[t][pixel +
// tap t], in tap order. A block covers 16 x 64 outputs (four per thread),
// with T of the 18 x 66 positions in LDS.
// ---------------------------------------------------------------------------
constexpr int CLM_TY = 16, CLM_TX = 64, CLM_RY = CLM_TY + 2, CLM_RX = CLM_TX + 2;
constexpr int CLM_RUNS = (CLM_RX + 15) / 16;  // 16-pixel runs per halo row
constexpr int CLM_NP = CLM_RY * CLM_RX;      // positions of the tile and its halo
constexpr int CLM_WRUNS = (CLM_RY * CLM_RUNS + 3) / 4;  // runs per wave

__global__ __launch_bounds__(256) void conv_last_mfma_kernel(const __bf16* __restrict__ in,
                                                             const float* __restrict__ w, int H,
                                                             int W,
                                                             const uint64_t* __restrict__ seeds,
                                                             uint32_t step,
                                                             uint8_t* __restrict__ bits,
                                                             float* __restrict__ probs,
                                                             const hs::Levels lv) {
  // T tap-major, [tap][position]: a wave's stores of one tap are 16
  // consecutive positions, and the 16 lanes of a row read positions 4 apart,
  // both free of bank conflicts
  __shared__ float sT[9 * CLM_NP];
  const int b = blockIdx.z, y0 = blockIdx.y * CLM_TY, x0 = blockIdx.x * CLM_TX;
  const size_t img = (size_t)b * H * W;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, g = lane >> 4, r = lane & 15;
  // A operands: row r = tap r (rows 9..15 zero), K = channels 8g .. 8g + 7
  bf16x8_t whi, wlo;
#pragma unroll
  for (int e = 0; e < 8; ++e) {
    const float v = r < 9 ? w[HS_W6 + (8 * g + e) * 9 + r] : 0.0f;
    const __bf16 hi = (__bf16)v;
    whi[e] = hi;
    wlo[e] = (__bf16)(v - (float)hi);
  }
  // all of a wave's runs are loaded before the first MFMA
  bf16x8_t a[CLM_WRUNS];
#pragma unroll
  for (int k = 0; k < CLM_WRUNS; ++k) {
    const int run = wave + 4 * k, ry = run / CLM_RUNS, rc = (run - ry * CLM_RUNS) * 16;
    const int gy = y0 + ry - 1, gx = x0 + rc + r - 1;
#pragma unroll
    for (int e = 0; e < 8; ++e) a[k][e] = (__bf16)0.0f;
    if (run < CLM_RY * CLM_RUNS && rc + r < CLM_RX && gy >= 0 && gy < H && gx >= 0 && gx < W)
      a[k] = *(const bf16x8_t*)(in + (img + (size_t)gy * W + gx) * 32 + 8 * g);
  }
#pragma unroll
  for (int k = 0; k < CLM_WRUNS; ++k) {
    const int run = wave + 4 * k, ry = run / CLM_RUNS, rc = (run - ry * CLM_RUNS) * 16;
    f32x4_t t = __builtin_amdgcn_mfma_f32_16x16x32_bf16(whi, a[k], f32x4_t{0.f, 0.f, 0.f, 0.f},
                                                         0, 0, 0);
    t = __builtin_amdgcn_mfma_f32_16x16x32_bf16(wlo, a[k], t, 0, 0, 0);
    // lane (g, r) holds taps 4g .. 4g + 3 of position (ry, rc + r)
    if (run < CLM_RY * CLM_RUNS && g < 3 && rc + r < CLM_RX)
#pragma unroll
      for (int e = 0; e < 4; ++e)
        if (4 * g + e < 9) sT[(4 * g + e) * CLM_NP + ry * CLM_RX + rc + r] = t[e];
  }
  __syncthreads();
  const float b6 = w[HS_B6];
  const int ty = threadIdx.x >> 4, tx = threadIdx.x & 15, gy = y0 + ty;
  if (gy >= H) return;
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    const int cx = 4 * tx + k, gx = x0 + cx;
    if (gx >= W) break;
    float x = b6;
#pragma unroll
    for (int t = 0; t < 9; ++t) x += sT[t * CLM_NP + (ty + t / 3) * CLM_RX + cx + t % 3];
    const size_t o = img + (size_t)gy * W + gx;
    const float p = hs_sigmoid(x);
    probs[o] = p;
    if (bits) {
      const float u = hs_action_u(seeds[b], (uint64_t)gy * W + gx, step);
      if (lv.n == 1) {
        bits[o] = u < p ? 1 : 0;
      } else {
        const float tl = p * (float)lv.n;
        const int kf = min((int)floorf(tl), lv.n - 1);
        bits[o] = (uint8_t)(kf + (u < tl - (float)kf ? 1 : 0));
      }
    }
  }
}

// ---------------------------------------------------------------------------
// Backward through the head and layer 6: g6 = dL/dlogit, and
// g5[y][x][ci] = [a5 > 0] * sum_t W6[ci][t] g6[y - dy + 1][x - dx + 1].
// ---------------------------------------------------------------------------
template <typename T>
__global__ __launch_bounds__(256) void dgrad_last_kernel(const float* __restrict__ grad,
                                                         const float* __restrict__ probs,
                                                         const T* __restrict__ a5,
                                                         const float* __restrict__ w, int H,
                                                         int W, float* __restrict__ g6out,
                                                         T* __restrict__ g5) {
  // weights as [tap][ci]: one 16-byte LDS read brings four channels' weights
  __shared__ __attribute__((aligned(16))) float sw[9 * 32];
  __shared__ float sg[18 * 18];
  const int b = blockIdx.z, y0 = blockIdx.y * 16, x0 = blockIdx.x * 16;
  const size_t img = (size_t)b * H * W;
  for (int i = threadIdx.x; i < 32 * 9; i += 256) sw[(i % 9) * 32 + i / 9] = w[HS_W6 + i];
  for (int i = threadIdx.x; i < 18 * 18; i += 256) {
    const int ly = i / 18, lx = i - ly * 18, gy = y0 + ly - 1, gx = x0 + lx - 1;
    float v = 0.0f;
    if (gy >= 0 && gy < H && gx >= 0 && gx < W) {
      const size_t o = img + (size_t)gy * W + gx;
      v = grad[o];
      if (probs) v *= probs[o] * (1.0f - probs[o]);
    }
    sg[i] = v;
  }
  __syncthreads();
  const int ty = threadIdx.x >> 4, tx = threadIdx.x & 15, gy = y0 + ty, gx = x0 + tx;
  if (gy >= H || gx >= W) return;
  const size_t o = img + (size_t)gy * W + gx;
  g6out[o] = sg[(ty + 1) * 18 + tx + 1];
  float acc[32];
#pragma unroll
  for (int ci = 0; ci < 32; ++ci) acc[ci] = 0.0f;
#pragma unroll
  for (int t = 0; t < 9; ++t) {
    const int dy = t / 3, dx = t - (t / 3) * 3;
    const float gv = sg[(ty + 2 - dy) * 18 + tx + 2 - dx];
#pragma unroll
    for (int ci = 0; ci < 32; ci += 4) {
      const f32x4_t q = *(const f32x4_t*)(sw + t * 32 + ci);
#pragma unroll
      for (int k = 0; k < 4; ++k) acc[ci + k] = fmaf(q[k], gv, acc[ci + k]);
    }
  }
  const T* m = a5 + o * 32;
  T* dst = g5 + o * 32;
#pragma unroll
  for (int ci = 0; ci < 32; ci += 4) {
    float v[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) v[k] = hs_to_f(m[ci + k]) > 0.0f ? acc[ci + k] : 0.0f;
    hs_store4(dst + ci, v[0], v[1], v[2], v[3]);
  }
}

// ---------------------------------------------------------------------------
// Weight gradient of a 32->32 layer on the FP32 matrix cores:
// dW[co][ci][t] = sum_px g[px][co] a[px + tap t][ci]; db[co] = sum_px g[px][co].
// Tile = 2 x 64 pixels (the K dimension); block = 4 waves, wave w owns the
// (co tile, ci tile) = (w >> 1, w & 1) output block for all nine taps.
// Blocks stride over tiles; each block writes one row of partial sums.
// ---------------------------------------------------------------------------
constexpr int WT_H = 2, WT_W = 64, WT_PX = WT_H * WT_W, WL_H = WT_H + 2, WL_W = WT_W + 2;
constexpr int WG_STRIDE = 132;  // floats per channel row of the staged gradient (128 + 4)
constexpr int WA_STRIDE = 268;  // floats per channel row of the staged input (264 + 4)

template <typename T>
__global__ __launch_bounds__(256) void wgrad32_kernel(const T* __restrict__ a_in,
                                                      const T* __restrict__ g_out, int B, int H,
                                                      int W, int layer,
                                                      float* __restrict__ partials,
                                                      int accumulate) {
  __shared__ float sg[32 * WG_STRIDE];
  __shared__ float sa[32 * WA_STRIDE];
  const int tiles_x = (W + WT_W - 1) / WT_W, tiles_y = (H + WT_H - 1) / WT_H;
  const int ntiles = B * tiles_x * tiles_y;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, g = lane >> 4, r = lane & 15;
  const int mt = wave >> 1, nt = wave & 1;
  f32x4_t acc[9];
#pragma unroll
  for (int t = 0; t < 9; ++t) acc[t] = f32x4_t{0.f, 0.f, 0.f, 0.f};
  float bacc = 0.0f;
  for (int tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
    const int b = tile / (tiles_x * tiles_y), rem = tile - b * tiles_x * tiles_y;
    const int y0 = (rem / tiles_x) * WT_H, x0 = (rem % tiles_x) * WT_W;
    const size_t img = (size_t)b * H * W;
    __syncthreads();
    // gradient tile, transposed to [co][px]; zero outside the image
    for (int i = threadIdx.x; i < WT_PX * 8; i += 256) {
      const int p = i >> 3, q = (i & 7) * 4;
      const int gy = y0 + p / WT_W, gx = x0 + (p % WT_W);
      float v[4] = {0.f, 0.f, 0.f, 0.f};
      if (gy < H && gx < W) {
        const T* src = g_out + (img + (size_t)gy * W + gx) * 32 + q;
#pragma unroll
        for (int k = 0; k < 4; ++k) v[k] = hs_to_f(src[k]);
      }
#pragma unroll
      for (int k = 0; k < 4; ++k) sg[(q + k) * WG_STRIDE + p] = v[k];
    }
    // input tile with a one-pixel halo, transposed to [ci][halo px]
    for (int i = threadIdx.x; i < WL_H * WL_W * 8; i += 256) {
      const int p = i >> 3, q = (i & 7) * 4;
      const int ly = p / WL_W, lx = p - ly * WL_W, gy = y0 + ly - 1, gx = x0 + lx - 1;
      float v[4] = {0.f, 0.f, 0.f, 0.f};
      if (gy >= 0 && gy < H && gx >= 0 && gx < W) {
        const T* src = a_in + (img + (size_t)gy * W + gx) * 32 + q;
#pragma unroll
        for (int k = 0; k < 4; ++k) v[k] = hs_to_f(src[k]);
      }
#pragma unroll
      for (int k = 0; k < 4; ++k) sa[(q + k) * WA_STRIDE + p] = v[k];
    }
    __syncthreads();
    if (threadIdx.x < 32) {
      float s = 0.0f;
      for (int p = 0; p < WT_PX; ++p) s += sg[threadIdx.x * WG_STRIDE + p];
      bacc += s;
    }
    // K loop: 4 pixels per MFMA step; lane group g takes pixel 4s + g
    for (int s4 = 0; s4 < WT_PX / 4; ++s4) {
      const int p = 4 * s4 + g, py = p / WT_W, px = p - py * WT_W;
      const float av = sg[(16 * mt + r) * WG_STRIDE + p];
      const float* brow = sa + (16 * nt + r) * WA_STRIDE;
#pragma unroll
      for (int t = 0; t < 9; ++t) {
        const int dy = t / 3, dx = t - (t / 3) * 3;
        const float bv = brow[(py + dy) * WL_W + px + dx];
        acc[t] = __builtin_amdgcn_mfma_f32_16x16x4f32(av, bv, acc[t], 0, 0, 0);
      }
    }
  }
  // acc[t][i] = dW[co = 16 mt + 4 g + i][ci = 16 nt + r][t]
  float* row = partials + (size_t)blockIdx.x * hs::NPARAM + hs_wk(layer);
#pragma unroll
  for (int t = 0; t < 9; ++t)
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int co = 16 * mt + 4 * g + i, ci = 16 * nt + r;
      float* d = row + (co * 32 + ci) * 9 + t;
      *d = accumulate ? *d + acc[t][i] : acc[t][i];
    }
  if (threadIdx.x < 32) {
    float* d = row + 32 * 32 * 9 + threadIdx.x;
    *d = accumulate ? *d + bacc : bacc;
  }
}

// 8 consecutive bf16 starting `dx` elements into the 16 loaded ones
HS_DEV bf16x8_t shift_frag(const bf16x8_t lo, const bf16x8_t hi, int dx) {
  uint32_t d[8], o[4];
  __builtin_memcpy(d, &lo, 16);
  __builtin_memcpy(d + 4, &hi, 16);
  if (dx == 0) {
    return lo;
  } else if (dx == 1) {
#pragma unroll
    for (int j = 0; j < 4; ++j) o[j] = __builtin_amdgcn_alignbyte(d[j + 1], d[j], 2);
  } else {
#pragma unroll
    for (int j = 0; j < 4; ++j) o[j] = d[j + 1];
  }
  bf16x8_t v;
  __builtin_memcpy(&v, o, 16);
  return v;
}

// ---------------------------------------------------------------------------
// Backward of a 32->32 layer in BF16 in one pass over the pixels: the input
// gradient (the conv of g with the transposed, flipped weights, times the
// ReLU mask [a > 0]) and the weight and bias gradients (sums over pixels of
// g[px][co] a[px + tap][ci] and of g[px][co]). A block of 8 waves strides
// over 8 x 64 pixel tiles; each tile of g and of a, with its one-pixel halo,
// is read from HBM once and staged in LDS three ways:
//   gP[row][col][chunk]  g pixel-major with the chunk swizzle of conv32
//                        (10 x 66 pixels): the input gradient's B operands;
//   gT[co][px]           g's 8 x 64 interior transposed: the weight
//                        gradient's A operands (K = 8 consecutive pixels);
//   aT[ci][row][col]     a transposed (10 rows x 68 columns): the weight
//                        gradient's B operands (the K-slice of tap dx cut out
//                        of two aligned 16-byte reads) and the ReLU mask.
// Wave w computes row w of the input gradient (both channel tiles, four
// 16-pixel runs) and the weight-gradient block (co tile, ci tile) = ((w >>
// 1) & 1, w & 1) over tile rows 4 (w >> 2) .. 4 (w >> 2) + 3; the two row
// halves are added in a fixed order at the end, so each block's row of
// partial sums is deterministic. It computes what conv32_kernel (MODE 1)
// and wgrad32_kernel compute in FP32, reading g and a once: a separate
// input-gradient pass and weight-gradient pass read them three times (the
// conv's tile, its mask, and the weight gradient's own staging with a
// halo twice its tile's height), about twice the bytes.
// Staging operations: "g" = 4 consecutive columns x 8 channels of one row
// of g (rows -1..8, columns 0..63), "h" = one 16-byte chunk of g's halo
// columns -1 and 64, "a" = 4 columns x 8 channels of a (rows -1..8, columns
// -1..66); thread i owns operations i, i + 512 and i + 1024 of the 1,400.
// All of a tile's global loads are issued together into registers, and the
// next tile's loads are in flight while the current tile's MFMAs run.
// ---------------------------------------------------------------------------
constexpr int FB_H = 8, FB_W = 64, FB_PX = FB_H * FB_W;
constexpr int FB_LH = FB_H + 2, FB_LW = FB_W + 2;  // gP: 10 x 66 pixels
constexpr int FB_GS = FB_PX + 8;                   // gT channel stride (65 x 16 B: odd)
constexpr int FB_AC = FB_W + 4;                    // aT staged columns (68)
constexpr int FB_RS = FB_W + 8;                    // aT row stride (72)
constexpr int FB_CS = FB_LH * FB_RS + 8;           // aT channel stride (91 x 16 B: odd)
constexpr int FB_GOPS = FB_LH * (FB_W / 4) * 4;    // 640
constexpr int FB_HOPS = FB_LH * 2 * 4;             // 80
constexpr int FB_AOPS = FB_LH * (FB_AC / 4) * 4;   // 680
constexpr int FB_OPS = FB_GOPS + FB_HOPS + FB_AOPS;
constexpr int FB_NT = 512, FB_NOP = (FB_OPS + FB_NT - 1) / FB_NT;
static_assert(FB_NOP == 3, "bwd32 staging split");
static_assert(4 * 64 * 40 * 4 <= FB_LH * FB_LW * 32 * 2, "bwd32 combine scratch fits in gP");

__global__ __launch_bounds__(FB_NT, 1) void bwd32_bf16_kernel(
    const __bf16* __restrict__ a_in, const __bf16* __restrict__ g_out,
    const __bf16* __restrict__ wpT, __bf16* __restrict__ g_in, int B, int H, int W, int layer,
    float* __restrict__ partials, int accumulate) {
  __shared__ __attribute__((aligned(16))) __bf16 gP[FB_LH * FB_LW * 32];
  __shared__ __attribute__((aligned(16))) __bf16 gT[32 * FB_GS];
  __shared__ __attribute__((aligned(16))) __bf16 aT[32 * FB_CS];
  // the input gradient's weight fragments [tap][row tile][lane], in LDS so
  // that the tile loop issues no global load besides the next tile's
  // prefetch (a wait on the vector memory counter for a weight load would
  // also wait for the prefetch)
  __shared__ bf16x8_t wS[9 * 2 * 64];
  const int tiles_x = (W + FB_W - 1) / FB_W, tiles_y = (H + FB_H - 1) / FB_H;
  const int ntiles = B * tiles_x * tiles_y;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6, g = lane >> 4, r = lane & 15;
  const int mt = (wave >> 1) & 1, nt = wave & 1, kh = wave >> 2;
  for (int i = tid; i < 9 * 2 * 64; i += FB_NT) wS[i] = *(const bf16x8_t*)(wpT + i * 8);
  f32x4_t accw[9], accb = f32x4_t{0.f, 0.f, 0.f, 0.f};
#pragma unroll
  for (int t = 0; t < 9; ++t) accw[t] = f32x4_t{0.f, 0.f, 0.f, 0.f};
  bf16x8_t ones;
#pragma unroll
  for (int e = 0; e < 8; ++e) ones[e] = (__bf16)1.0f;
  // staging operation k of this thread, the same for every tile: kind (0
  // none, 1 g, 2 a, 3 halo chunk of g), source row and first column
  // relative to (y0, x0), channel group. Thread t: operation 0 is g at row
  // t / 64 - 1, columns 4 ((t / 4) % 16) + 0..3, channel group t % 4;
  // operation 1 is a at the same row and channel group, columns one to the
  // left; operation 2 covers the rest (g and a at rows 7 and 8, a's last
  // column group, g's halo chunks). Decoded where it is used from a thread
  // number the compiler cannot hoist (a volatile copy), which keeps registers
  // free across the tile loop.
  struct Op {
    int kind, row, col, c8;
  };
  auto op = [&](int k) {
    int q;
    asm volatile("v_mov_b32 %0, %1" : "=v"(q) : "v"(tid));
    Op o{0, 0, 0, q & 3};
    const int cg = (q >> 2) & 15;
    if (k < 2) {
      o.kind = k + 1;
      o.row = (q >> 6) - 1;
      o.col = 4 * cg - k;
    } else if (q < 256) {
      o.kind = q < 128 ? 1 : 2;
      o.row = 7 + ((q >> 6) & 1);
      o.col = 4 * cg - (q < 128 ? 0 : 1);
    } else if (q < 296) {
      o.kind = 2;
      o.row = ((q - 256) >> 2) - 1;
      o.col = FB_AC - 5;
    } else if (q < 376) {
      q -= 296;
      o.kind = 3;
      o.col = ((q >> 2) & 1) ? FB_W : -1;
      o.row = (q >> 3) - 1;
    }
    return o;
  };
  // loads from clamped (always valid) addresses; positions outside the image
  // are zeroed when the registers are stored to LDS
  bf16x8_t v[FB_NOP][4];
  auto load = [&](int tile) {
    const int b = tile / (tiles_x * tiles_y), rem = tile - b * tiles_x * tiles_y;
    const int y0 = (rem / tiles_x) * FB_H, x0 = (rem % tiles_x) * FB_W;
    const size_t img = (size_t)b * H * W;
#pragma unroll
    for (int k = 0; k < FB_NOP; ++k) {
      const Op o = op(k);
      if (o.kind == 0) continue;
      const __bf16* src = (o.kind == 2 ? a_in : g_out) + img * 32 + 8 * o.c8;
      const int gyc = min(max(y0 + o.row, 0), H - 1);
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int gxc = min(max(x0 + o.col + u, 0), W - 1);
        v[k][u] = *(const bf16x8_t*)(src + ((size_t)gyc * W + gxc) * 32);
      }
    }
  };
  auto store = [&](int y0, int x0, auto masked) {
    bf16x8_t zero;
#pragma unroll
    for (int e = 0; e < 8; ++e) zero[e] = (__bf16)0.0f;
#pragma unroll
    for (int k = 0; k < FB_NOP; ++k) {
      const Op o = op(k);
      const int row = o.row + 1, c8 = o.c8;
      bf16x8_t w4[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        w4[u] = v[k][u];
        if (decltype(masked)::value) {
          const bool ok = (unsigned)(y0 + o.row) < (unsigned)H &&
                          (unsigned)(x0 + o.col + u) < (unsigned)W;
          w4[u] = ok ? w4[u] : zero;
        }
      }
      if (o.kind == 1 || o.kind == 3) {
        const int nu = o.kind == 1 ? 4 : 1;
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          if (u >= nu) break;
          const int lx = o.col + u + 1;
          *(bf16x8_t*)(gP + (row * FB_LW + lx) * 32 + hs_swz<__bf16>(lx, c8) * 8) = w4[u];
        }
        if (o.kind == 1 && row >= 1 && row <= FB_H) {
          __bf16* base = gT + (8 * c8) * FB_GS + (row - 1) * FB_W + o.col;
#pragma unroll
          for (int e = 0; e < 8; ++e)
            *(bf16x4_t*)(base + e * FB_GS) = bf16x4_t{w4[0][e], w4[1][e], w4[2][e], w4[3][e]};
        }
      } else if (o.kind == 2) {
        __bf16* base = aT + (8 * c8) * FB_CS + row * FB_RS + (o.col + 1);
#pragma unroll
        for (int e = 0; e < 8; ++e)
          *(bf16x4_t*)(base + e * FB_CS) = bf16x4_t{w4[0][e], w4[1][e], w4[2][e], w4[3][e]};
      }
    }
  };
  if ((int)blockIdx.x < ntiles) load(blockIdx.x);
  for (int tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
    const int b = tile / (tiles_x * tiles_y), rem = tile - b * tiles_x * tiles_y;
    const int y0 = (rem / tiles_x) * FB_H, x0 = (rem % tiles_x) * FB_W;
    const size_t img = (size_t)b * H * W;
    __syncthreads();  // the previous tile's operands have been read
    // a tile whose staged window lies inside the image needs no zeroing
    if (y0 >= 1 && y0 + FB_H + 1 <= H && x0 >= 1 && x0 + FB_AC - 1 <= W)
      store(y0, x0, std::false_type{});
    else
      store(y0, x0, std::true_type{});
    __syncthreads();
    if (tile + (int)gridDim.x < ntiles) load(tile + gridDim.x);
    // ---- input gradient, row `wave` of the tile: input row wave + d of gP
    // (tap dy = d), both 16-channel tiles, four 16-pixel runs. The weight
    // fragments are read from LDS where they are used; the lane number comes
    // from a volatile statement so that the compiler does not hoist all
    // eighteen out of the tile loop (72 registers it does not have)
    int ln;
    asm volatile("v_mbcnt_lo_u32_b32 %0, -1, 0\n\tv_mbcnt_hi_u32_b32 %0, -1, %0" : "=v"(ln));
    f32x4_t acc[2][4];
#pragma unroll
    for (int m = 0; m < 2; ++m)
#pragma unroll
      for (int n = 0; n < 4; ++n) acc[m][n] = f32x4_t{0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int d = 0; d < 3; ++d) {
#pragma unroll
      for (int dx = 0; dx < 3; ++dx) {
        const int t = d * 3 + dx;
        frag8<__bf16> w0, w1;
        w0.v = wS[(t * 2 + 0) * 64 + ln];
        w1.v = wS[(t * 2 + 1) * 64 + ln];
#pragma unroll
        for (int n = 0; n < 4; ++n) {
          const int lx = n * 16 + r + dx;
          frag8<__bf16> bf;
          lds_frag(bf, gP + ((wave + d) * FB_LW + lx) * 32, lx, g);
          acc[0][n] = hs_mma(w0, bf, acc[0][n]);
          acc[1][n] = hs_mma(w1, bf, acc[1][n]);
        }
      }
    }
    // ---- weight gradient: K = 32 pixels of one tile row per MFMA
#pragma unroll
    for (int kc = 0; kc < 8; ++kc) {
      const int py = 4 * kh + (kc >> 1), pc = (kc & 1) * 32 + 8 * g;
      const bf16x8_t af = *(const bf16x8_t*)(gT + (16 * mt + r) * FB_GS + py * FB_W + pc);
#pragma unroll
      for (int dy = 0; dy < 3; ++dy) {
        const __bf16* rowp = aT + (16 * nt + r) * FB_CS + (py + dy) * FB_RS + pc;
        const bf16x8_t lo = *(const bf16x8_t*)rowp;
        const bf16x8_t hi = *(const bf16x8_t*)(rowp + 8);
#pragma unroll
        for (int dx = 0; dx < 3; ++dx)
          accw[dy * 3 + dx] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(
              af, shift_frag(lo, hi, dx), accw[dy * 3 + dx], 0, 0, 0);
      }
      if (nt == 0) accb = __builtin_amdgcn_mfma_f32_16x16x32_bf16(af, ones, accb, 0, 0, 0);
    }
    // ---- input gradient out, times the ReLU mask of a (from aT)
    const int gy = y0 + wave;
    if (gy < H) {
#pragma unroll
      for (int n = 0; n < 4; ++n) {
        const int gx = x0 + n * 16 + r;
        if (gx >= W) continue;
        const size_t o = (img + (size_t)gy * W + gx) * 32;
        const __bf16* mk = aT + (wave + 1) * FB_RS + (n * 16 + r + 1);
#pragma unroll
        for (int m = 0; m < 2; ++m) {
          const int co = 16 * m + 4 * g;
          float vv[4];
#pragma unroll
          for (int i = 0; i < 4; ++i)
            vv[i] = (float)mk[(co + i) * FB_CS] > 0.0f ? acc[m][n][i] : 0.0f;
          hs_store4(g_in + o + co, vv[0], vv[1], vv[2], vv[3]);
        }
      }
    }
  }
  // ---- the two row halves of each weight-gradient block, in a fixed order
  __syncthreads();
  float* scratch = (float*)gP;
  if (kh == 1) {
    float* sp = scratch + ((wave - 4) * 64 + lane) * 40;
#pragma unroll
    for (int t = 0; t < 9; ++t)
#pragma unroll
      for (int i = 0; i < 4; ++i) sp[4 * t + i] = accw[t][i];
#pragma unroll
    for (int i = 0; i < 4; ++i) sp[36 + i] = accb[i];
  }
  __syncthreads();
  if (kh == 1) return;
  {
    const float* sp = scratch + (wave * 64 + lane) * 40;
#pragma unroll
    for (int t = 0; t < 9; ++t)
#pragma unroll
      for (int i = 0; i < 4; ++i) accw[t][i] += sp[4 * t + i];
#pragma unroll
    for (int i = 0; i < 4; ++i) accb[i] += sp[36 + i];
  }
  // accw[t][i] = dW[co = 16 mt + 4 g + i][ci = 16 nt + r][t]
  float* prow = partials + (size_t)blockIdx.x * hs::NPARAM + hs_wk(layer);
#pragma unroll
  for (int t = 0; t < 9; ++t)
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int co = 16 * mt + 4 * g + i, ci = 16 * nt + r;
      float* dd = prow + (co * 32 + ci) * 9 + t;
      *dd = accumulate ? *dd + accw[t][i] : accw[t][i];
    }
  if (nt == 0 && r == 0) {
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      float* dd = prow + 32 * 32 * 9 + 16 * mt + 4 * g + i;
      *dd = accumulate ? *dd + accb[i] : accb[i];
    }
  }
  // with fewer than WGRAD_BLOCKS blocks the layer's other rows are left
  // alone: the reduction reads only the first gridDim.x rows of the 32->32
  // layers (launch_reduce_partials, rows32)
}

// ---------------------------------------------------------------------------
// Weight gradient of layer 1 (2 -> 32) on BF16 activations, on the matrix
// cores: dW1[co][n] = sum_px g1[px][co] u_n(px), where column n = 9 ci + t
// (n < 18) takes u_n(px) = in_ci[px + tap t] (ci 0 the contone, 1 the noise)
// and column 18 takes u = 1 (the bias gradient). One MFMA sums over 32
// pixels of a tile row. g1's pixel-major 16-byte fragments become
// channel-major ones through an MFMA with a unit matrix (every output is a
// single product by 1, so exact); the contone and noise values are split
// into BF16 hi + lo parts (about 16 significant bits), staged in LDS as
// one dword per value and position. A block takes 8 x 32 tiles in turn, wave
// w rows 2w and 2w + 1, and loads the next tile during this one's work;
// the four waves' sums are added in a fixed order at the end.
// ---------------------------------------------------------------------------
constexpr int WF_TY = 8, WF_TX = 32;
constexpr int WF_SX = WF_TX + 2, WF_SN = (WF_TY + 2) * WF_SX;  // staged window with its halo
constexpr int WF_SPT = (WF_SN + 255) / 256;                   // staged positions per thread

__global__ __launch_bounds__(256) void wgrad_first_bf16_kernel(
    const float* __restrict__ contone, const float* __restrict__ z,
    const __bf16* __restrict__ g1, int B, int H, int W, float* __restrict__ partials,
    int accumulate) {
  __shared__ uint32_t sin[2][WF_SN];
  __shared__ float sred[4][32 * 19];
  const int tiles_x = (W + WF_TX - 1) / WF_TX, tiles_y = (H + WF_TY - 1) / WF_TY;
  const int ntiles = B * tiles_x * tiles_y;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, g = lane >> 4, r = lane & 15;
  // unit B operands: channel tile c, lane (g, r) holds [8 g + j == 16 c + r]
  bf16x8_t unit[2];
#pragma unroll
  for (int c = 0; c < 2; ++c)
#pragma unroll
    for (int j = 0; j < 8; ++j) unit[c][j] = (__bf16)(8 * g + j == 16 * c + r ? 1.0f : 0.0f);
  // this lane's columns: n = r in column tile 0, n = 16 + r in tile 1
  // (16, 17: the noise's taps 7, 8; 18: the bias; beyond: zero)
  const int n1 = 16 + r;
  const int ci0 = r / 9, t0 = r % 9, ci1 = n1 < 18 ? 1 : 0, t1 = n1 < 18 ? n1 - 9 : 0;
  const int base0 = ci0 * WF_SN + (t0 / 3) * WF_SX + t0 % 3;
  const int base1 = ci1 * WF_SN + (t1 / 3) * WF_SX + t1 % 3;
  const uint32_t fixed1 = n1 == 18 ? (uint32_t)__builtin_bit_cast(unsigned short, (__bf16)1.0f)
                                   : 0u;
  f32x4_t acc[2][2];
#pragma unroll
  for (int c = 0; c < 2; ++c)
#pragma unroll
    for (int nt = 0; nt < 2; ++nt) acc[c][nt] = f32x4_t{0.f, 0.f, 0.f, 0.f};
  bf16x8_t gv[2][2];
  float cv[WF_SPT], zv[WF_SPT];
  auto load = [&](int tile) {
    const int b = tile / (tiles_x * tiles_y), rem = tile - b * tiles_x * tiles_y;
    const int y0 = (rem / tiles_x) * WF_TY, x0 = (rem % tiles_x) * WF_TX;
    const size_t img = (size_t)b * H * W;
#pragma unroll
    for (int j = 0; j < WF_SPT; ++j) {
      const int i = (int)threadIdx.x + 256 * j;
      const int sy = i / WF_SX, sx = i - sy * WF_SX, gy = y0 + sy - 1, gx = x0 + sx - 1;
      const bool in = i < WF_SN && gy >= 0 && gy < H && gx >= 0 && gx < W;
      cv[j] = in ? contone[img + (size_t)gy * W + gx] : 0.0f;
      zv[j] = in ? z[img + (size_t)gy * W + gx] : 0.0f;
    }
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        const int gy = y0 + 2 * wave + i, gx = x0 + 16 * h + r;
#pragma unroll
        for (int e = 0; e < 8; ++e) gv[i][h][e] = (__bf16)0.0f;
        if (gy < H && gx < W)
          gv[i][h] = *(const bf16x8_t*)(g1 + (img + (size_t)gy * W + gx) * 32 + 8 * g);
      }
  };
  if ((int)blockIdx.x < ntiles) load(blockIdx.x);
  for (int tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
    __syncthreads();  // the previous tile's reads of sin are done
#pragma unroll
    for (int j = 0; j < WF_SPT; ++j) {
      const int i = (int)threadIdx.x + 256 * j;
      if (i < WF_SN) {
        sin[0][i] = split_bf16(cv[j]);
        sin[1][i] = split_bf16(zv[j]);
      }
    }
    bf16x8_t cur[2][2];
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int h = 0; h < 2; ++h) cur[i][h] = gv[i][h];
    __syncthreads();
    if (tile + (int)gridDim.x < ntiles) load(tile + gridDim.x);
    const uint32_t* s0 = &sin[0][0];
#pragma unroll
    for (int i = 0; i < 2; ++i) {
      // K slot j of lane group g is pixel 4 g + j (j < 4) or 16 + 4 g + j - 4
      bf16x8_t a[2];
#pragma unroll
      for (int c = 0; c < 2; ++c) {
#pragma unroll
        for (int h = 0; h < 2; ++h) {
          const f32x4_t t = __builtin_amdgcn_mfma_f32_16x16x32_bf16(
              cur[i][h], unit[c], f32x4_t{0.f, 0.f, 0.f, 0.f}, 0, 0, 0);
#pragma unroll
          for (int e = 0; e < 4; ++e) a[c][4 * h + e] = (__bf16)t[e];
        }
      }
      const int row = (2 * wave + i) * WF_SX + 4 * g;
      uint32_t d0[8], d1[8];
#pragma unroll
      for (int j = 0; j < 8; ++j) {
        const int p = row + (j < 4 ? j : 12 + j);
        d0[j] = s0[base0 + p];
        d1[j] = n1 < 18 ? s0[base1 + p] : fixed1;
      }
      bf16x8_t bh[2], bl[2];
#pragma unroll
      for (int j = 0; j < 8; ++j) {
        bh[0][j] = __builtin_bit_cast(__bf16, (unsigned short)(d0[j] & 0xffffu));
        bl[0][j] = __builtin_bit_cast(__bf16, (unsigned short)(d0[j] >> 16));
        bh[1][j] = __builtin_bit_cast(__bf16, (unsigned short)(d1[j] & 0xffffu));
        bl[1][j] = __builtin_bit_cast(__bf16, (unsigned short)(d1[j] >> 16));
      }
#pragma unroll
      for (int c = 0; c < 2; ++c)
#pragma unroll
        for (int nt = 0; nt < 2; ++nt) {
          acc[c][nt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[c], bh[nt], acc[c][nt], 0, 0, 0);
          acc[c][nt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[c], bl[nt], acc[c][nt], 0, 0, 0);
        }
    }
  }
  // lane (g, r) of (c, nt) holds output channels 16 c + 4 g + e, column 16 nt + r
#pragma unroll
  for (int c = 0; c < 2; ++c)
#pragma unroll
    for (int nt = 0; nt < 2; ++nt) {
      const int n = 16 * nt + r;
      if (n <= 18)
#pragma unroll
        for (int e = 0; e < 4; ++e) sred[wave][(16 * c + 4 * g + e) * 19 + n] = acc[c][nt][e];
    }
  __syncthreads();
  // W1[co][ci][t] at co * 18 + ci * 9 + t, then the biases at 576 + co
  float* rowp = partials + (size_t)blockIdx.x * hs::NPARAM + HS_W1;
  for (int q = threadIdx.x; q < 32 * 19; q += 256) {
    const int co = q / 19, n = q - co * 19;
    const float s = ((sred[0][q] + sred[1][q]) + sred[2][q]) + sred[3][q];
    const int prm = n < 18 ? co * 18 + n : 576 + co;
    rowp[prm] = accumulate ? rowp[prm] + s : s;
  }
}

// ---------------------------------------------------------------------------
// Weight gradient of the first layer (2 -> 32) on the vector ALUs.
// Tile = 16 x 16 pixels; thread i < 608 owns parameter i of layer 1.
// ---------------------------------------------------------------------------
// Weight gradient of layer 1 (2 -> 32): thread (co = tid % 32, pixel group
// pg = tid / 32) of a 16 x 16 tile owns the 18 weights (channel, tap) of
// output channel co and its bias over the tile's rows 2 pg, 2 pg + 1, sliding
// 3 x 3 register windows of c and z along each row. The eight pixel groups
// are summed in a fixed order at the end.
template <typename T>
__global__ __launch_bounds__(256) void wgrad_first_kernel(const float* __restrict__ contone,
                                                          const float* __restrict__ z,
                                                          const T* __restrict__ g1, int B, int H,
                                                          int W, float* __restrict__ partials,
                                                          int accumulate) {
  __shared__ float sg[256 * 33];
  __shared__ float sc[18 * 18], sz[18 * 18];
  __shared__ float sred[8][609];
  const int tiles_x = (W + 15) / 16, tiles_y = (H + 15) / 16, ntiles = B * tiles_x * tiles_y;
  const int co = threadIdx.x & 31, pg = threadIdx.x >> 5;
  float ac[9], az[9], accb = 0.0f;
#pragma unroll
  for (int t = 0; t < 9; ++t) ac[t] = az[t] = 0.0f;
  // staging of a tile: 256 pixels x 8 groups of 4 channels of g1 (8 per
  // thread) and the 18 x 18 c and z values (up to 2 per thread); the next
  // tile's loads are issued before this tile's arithmetic
  float vg[8][4], vc[2], vz[2];
  auto load = [&](int tile) {
    const int b = tile / (tiles_x * tiles_y), rem = tile - b * tiles_x * tiles_y;
    const int y0 = (rem / tiles_x) * 16, x0 = (rem % tiles_x) * 16;
    const size_t img = (size_t)b * H * W;
#pragma unroll
    for (int k = 0; k < 8; ++k) {
      const int i = (int)threadIdx.x + 256 * k;
      const int p = i >> 3, q = (i & 7) * 4, gy = y0 + (p >> 4), gx = x0 + (p & 15);
#pragma unroll
      for (int e = 0; e < 4; ++e) vg[k][e] = 0.0f;
      if (gy < H && gx < W) {
        const T* src = g1 + (img + (size_t)gy * W + gx) * 32 + q;
#pragma unroll
        for (int e = 0; e < 4; ++e) vg[k][e] = hs_to_f(src[e]);
      }
    }
#pragma unroll
    for (int k = 0; k < 2; ++k) {
      const int i = (int)threadIdx.x + 256 * k;
      const int ly = i / 18, lx = i - ly * 18, gy = y0 + ly - 1, gx = x0 + lx - 1;
      const bool in = i < 18 * 18 && gy >= 0 && gy < H && gx >= 0 && gx < W;
      vc[k] = in ? contone[img + (size_t)gy * W + gx] : 0.0f;
      vz[k] = in ? z[img + (size_t)gy * W + gx] : 0.0f;
    }
  };
  if ((int)blockIdx.x < ntiles) load(blockIdx.x);
  for (int tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
    __syncthreads();
#pragma unroll
    for (int k = 0; k < 8; ++k) {
      const int i = (int)threadIdx.x + 256 * k;
      const int p = i >> 3, q = (i & 7) * 4;
#pragma unroll
      for (int e = 0; e < 4; ++e) sg[p * 33 + q + e] = vg[k][e];
    }
#pragma unroll
    for (int k = 0; k < 2; ++k) {
      const int i = (int)threadIdx.x + 256 * k;
      if (i < 18 * 18) {
        sc[i] = vc[k];
        sz[i] = vz[k];
      }
    }
    __syncthreads();
    if (tile + (int)gridDim.x < ntiles) load(tile + gridDim.x);
#pragma unroll
    for (int rr = 0; rr < 2; ++rr) {
      const int py = 2 * pg + rr;
      float wc[3][3], wz[3][3];
#pragma unroll
      for (int dy = 0; dy < 3; ++dy)
#pragma unroll
        for (int dx = 0; dx < 2; ++dx) {
          wc[dy][dx + 1] = sc[(py + dy) * 18 + dx];
          wz[dy][dx + 1] = sz[(py + dy) * 18 + dx];
        }
      for (int px = 0; px < 16; ++px) {
#pragma unroll
        for (int dy = 0; dy < 3; ++dy) {
          wc[dy][0] = wc[dy][1];
          wc[dy][1] = wc[dy][2];
          wc[dy][2] = sc[(py + dy) * 18 + px + 2];
          wz[dy][0] = wz[dy][1];
          wz[dy][1] = wz[dy][2];
          wz[dy][2] = sz[(py + dy) * 18 + px + 2];
        }
        const float gv = sg[(py * 16 + px) * 33 + co];
#pragma unroll
        for (int t = 0; t < 9; ++t) {
          ac[t] = fmaf(gv, wc[t / 3][t % 3], ac[t]);
          az[t] = fmaf(gv, wz[t / 3][t % 3], az[t]);
        }
        accb += gv;
      }
    }
  }
  // W1[co][ci][t] at co * 18 + ci * 9 + t, then the biases at 576 + co
  __syncthreads();
#pragma unroll
  for (int t = 0; t < 9; ++t) {
    sred[pg][co * 18 + t] = ac[t];
    sred[pg][co * 18 + 9 + t] = az[t];
  }
  sred[pg][576 + co] = accb;
  __syncthreads();
  float* row = partials + (size_t)blockIdx.x * hs::NPARAM + HS_W1;
  for (int prm = threadIdx.x; prm < 608; prm += 256) {
    float s = 0.0f;
#pragma unroll
    for (int k = 0; k < 8; ++k) s += sred[k][prm];
    row[prm] = accumulate ? row[prm] + s : s;
  }
}

// ---------------------------------------------------------------------------
// Weight gradient of the last layer (32 -> 1): dW6[ci][t] = sum g6 a5[+t][ci].
// ---------------------------------------------------------------------------
// Thread (ci = tid % 32, pixel group pg = tid / 32) of a 16 x 16 tile owns
// the nine taps of input channel ci over the tile's rows 2 pg, 2 pg + 1; it
// slides a 3 x 3 register window of the staged activations along each row
// (three new LDS reads per pixel for nine FMAs). The eight pixel groups are
// summed in a fixed order at the end.
template <typename T>
__global__ __launch_bounds__(256) void wgrad_last_kernel(const T* __restrict__ a5,
                                                         const float* __restrict__ g6, int B,
                                                         int H, int W,
                                                         float* __restrict__ partials,
                                                         int accumulate) {
  __shared__ float sa[18 * 18 * LP];
  __shared__ float sg[256];
  __shared__ float sred[8][289];
  const int tiles_x = (W + 15) / 16, tiles_y = (H + 15) / 16, ntiles = B * tiles_x * tiles_y;
  const int ci = threadIdx.x & 31, pg = threadIdx.x >> 5;
  float acc[9], accb = 0.0f;
#pragma unroll
  for (int t = 0; t < 9; ++t) acc[t] = 0.0f;
  // staging of a tile: 18 x 18 positions x 8 groups of 4 channels, NIT per
  // thread, plus one g6 value; the next tile's loads are issued before this
  // tile's arithmetic
  constexpr int NA = 18 * 18 * 8, NIT = (NA + 255) / 256;
  float v[NIT][4], gv6 = 0.0f;
  auto load = [&](int tile) {
    const int b = tile / (tiles_x * tiles_y), rem = tile - b * tiles_x * tiles_y;
    const int y0 = (rem / tiles_x) * 16, x0 = (rem % tiles_x) * 16;
    const size_t img = (size_t)b * H * W;
#pragma unroll
    for (int k = 0; k < NIT; ++k) {
      const int i = (int)threadIdx.x + 256 * k;
      const int p = i >> 3, q = (i & 7) * 4;
      const int ly = p / 18, lx = p - ly * 18, gy = y0 + ly - 1, gx = x0 + lx - 1;
#pragma unroll
      for (int e = 0; e < 4; ++e) v[k][e] = 0.0f;
      if (i < NA && gy >= 0 && gy < H && gx >= 0 && gx < W) {
        const T* src = a5 + (img + (size_t)gy * W + gx) * 32 + q;
#pragma unroll
        for (int e = 0; e < 4; ++e) v[k][e] = hs_to_f(src[e]);
      }
    }
    const int gy = y0 + ((int)threadIdx.x >> 4), gx = x0 + ((int)threadIdx.x & 15);
    gv6 = (gy < H && gx < W) ? g6[img + (size_t)gy * W + gx] : 0.0f;
  };
  if ((int)blockIdx.x < ntiles) load(blockIdx.x);
  for (int tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
    __syncthreads();
#pragma unroll
    for (int k = 0; k < NIT; ++k) {
      const int i = (int)threadIdx.x + 256 * k;
      const int p = i >> 3, q = (i & 7) * 4;
      if (i < NA) {
#pragma unroll
        for (int e = 0; e < 4; ++e) sa[p * LP + q + e] = v[k][e];
      }
    }
    sg[threadIdx.x] = gv6;
    __syncthreads();
    if (tile + (int)gridDim.x < ntiles) load(tile + gridDim.x);
#pragma unroll
    for (int rr = 0; rr < 2; ++rr) {
      const int py = 2 * pg + rr;
      // window columns px .. px + 2 of staged rows py .. py + 2
      float win[3][3];
#pragma unroll
      for (int dy = 0; dy < 3; ++dy)
#pragma unroll
        for (int dx = 0; dx < 2; ++dx) win[dy][dx + 1] = sa[((py + dy) * 18 + dx) * LP + ci];
      for (int px = 0; px < 16; ++px) {
#pragma unroll
        for (int dy = 0; dy < 3; ++dy) {
          win[dy][0] = win[dy][1];
          win[dy][1] = win[dy][2];
          win[dy][2] = sa[((py + dy) * 18 + px + 2) * LP + ci];
        }
        const float gv = sg[py * 16 + px];
#pragma unroll
        for (int t = 0; t < 9; ++t) acc[t] = fmaf(gv, win[t / 3][t % 3], acc[t]);
        accb += gv;
      }
    }
  }
  __syncthreads();
#pragma unroll
  for (int t = 0; t < 9; ++t) sred[pg][ci * 9 + t] = acc[t];
  if (ci == 0) sred[pg][288] = accb;
  __syncthreads();
  for (int prm = threadIdx.x; prm <= 288; prm += blockDim.x) {
    float s = 0.0f;
#pragma unroll
    for (int k = 0; k < 8; ++k) s += sred[k][prm];
    float* d = partials + (size_t)blockIdx.x * hs::NPARAM + HS_W6 + prm;
    *d = accumulate ? *d + s : s;
  }
}

// ---------------------------------------------------------------------------
// Backward through the head and layer 6 in one pass (BF16 activations).
// With G_t(q) = g6[q_y - dy + 1][q_x - dx + 1] for tap t = (dy, dx) (zero
// outside the image), the input gradient
//   g5[q][ci] = [a5[q][ci] > 0] sum_t W6[ci][t] G_t(q)
// and the weight gradient, re-indexed by q = px + tap t,
//   dW6[ci][t] = sum_px g6[px] a5[px + tap t][ci] = sum_q a5[q][ci] G_t(q)
// take the same nine values of g6 around q and a5 at q only, so a5 is read
// once and with no halo. A block takes 8 x 32 tiles in turn: the tile's g6
// with a one-pixel halo is formed in LDS from dL/dp and p, and thread
// (c4, seg) owns channels 4 c4 .. 4 c4 + 3 of the 8-pixel row segment seg,
// with those channels' 36 weights and 36 weight-gradient sums in
// registers, sliding the 3 x 3 window of g6 along the segment. The next
// tile's loads are issued before this tile's arithmetic; the 32 segments'
// sums are added in a fixed order at the end.
// ---------------------------------------------------------------------------
constexpr int BL_TY = 8, BL_TX = 32, BL_SEG = 8;               // tile rows, columns; segment
constexpr int BL_GX = BL_TX + 2, BL_GN = (BL_TY + 2) * BL_GX;  // staged g6 with its halo
constexpr int BL_GPT = (BL_GN + 255) / 256;                    // staged values per thread

__global__ __launch_bounds__(256) void bwd_last_bf16_kernel(
    const float* __restrict__ grad, const float* __restrict__ probs,
    const __bf16* __restrict__ a5, const float* __restrict__ w, int B, int H, int W,
    __bf16* __restrict__ g5, float* __restrict__ partials, int accumulate) {
  __shared__ float sg[BL_GN];
  __shared__ float sred[32][289];
  const int tiles_x = (W + BL_TX - 1) / BL_TX, tiles_y = (H + BL_TY - 1) / BL_TY;
  const int ntiles = B * tiles_x * tiles_y;
  const int c4 = threadIdx.x & 7, seg = threadIdx.x >> 3;
  const int ly = seg >> 2, lx0 = (seg & 3) * BL_SEG;
  float wr[4][9], acc[4][9], accb = 0.0f;
#pragma unroll
  for (int k = 0; k < 4; ++k)
#pragma unroll
    for (int t = 0; t < 9; ++t) {
      wr[k][t] = w[HS_W6 + (4 * c4 + k) * 9 + t];
      acc[k][t] = 0.0f;
    }
  bf16x4_t av[BL_SEG];
  float gq[BL_GPT], pq[BL_GPT];
  auto load = [&](int tile) {
    const int b = tile / (tiles_x * tiles_y), rem = tile - b * tiles_x * tiles_y;
    const int y0 = (rem / tiles_x) * BL_TY, x0 = (rem % tiles_x) * BL_TX;
    const size_t img = (size_t)b * H * W;
#pragma unroll
    for (int j = 0; j < BL_GPT; ++j) {
      const int i = (int)threadIdx.x + 256 * j;
      const int sy = i / BL_GX, sx = i - sy * BL_GX, gy = y0 + sy - 1, gx = x0 + sx - 1;
      gq[j] = 0.0f;
      pq[j] = 0.0f;
      if (i < BL_GN && gy >= 0 && gy < H && gx >= 0 && gx < W) {
        const size_t o = img + (size_t)gy * W + gx;
        gq[j] = grad[o];
        if (probs) pq[j] = probs[o];
      }
    }
    const int gy = y0 + ly;
#pragma unroll
    for (int e = 0; e < BL_SEG; ++e) {
      const int gx = x0 + lx0 + e;
      av[e] = bf16x4_t{(__bf16)0.0f, (__bf16)0.0f, (__bf16)0.0f, (__bf16)0.0f};
      if (gy < H && gx < W)
        av[e] = *(const bf16x4_t*)(a5 + (img + (size_t)gy * W + gx) * 32 + 4 * c4);
    }
  };
  if ((int)blockIdx.x < ntiles) load(blockIdx.x);
  for (int tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
    const int b = tile / (tiles_x * tiles_y), rem = tile - b * tiles_x * tiles_y;
    const int y0 = (rem / tiles_x) * BL_TY, x0 = (rem % tiles_x) * BL_TX;
    const size_t img = (size_t)b * H * W;
    __syncthreads();  // the previous tile's reads of sg are done
#pragma unroll
    for (int j = 0; j < BL_GPT; ++j) {
      const int i = (int)threadIdx.x + 256 * j;
      if (i < BL_GN) sg[i] = probs ? gq[j] * (pq[j] * (1.0f - pq[j])) : gq[j];
    }
    bf16x4_t cur[BL_SEG];
#pragma unroll
    for (int e = 0; e < BL_SEG; ++e) cur[e] = av[e];
    __syncthreads();
    if (tile + (int)gridDim.x < ntiles) load(tile + gridDim.x);
    // window columns lx .. lx + 2 of staged rows ly .. ly + 2; G_t = win[2 - dy][2 - dx]
    float win[3][3];
#pragma unroll
    for (int r = 0; r < 3; ++r)
#pragma unroll
      for (int c = 0; c < 2; ++c) win[r][c + 1] = sg[(ly + r) * BL_GX + lx0 + c];
    const int gy = y0 + ly;
#pragma unroll
    for (int e = 0; e < BL_SEG; ++e) {
#pragma unroll
      for (int r = 0; r < 3; ++r) {
        win[r][0] = win[r][1];
        win[r][1] = win[r][2];
        win[r][2] = sg[(ly + r) * BL_GX + lx0 + e + 2];
      }
      float a[4], o[4];
#pragma unroll
      for (int k = 0; k < 4; ++k) a[k] = (float)cur[e][k];
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        float x = 0.0f;
#pragma unroll
        for (int t = 0; t < 9; ++t) x = fmaf(wr[k][t], win[2 - t / 3][2 - t % 3], x);
        o[k] = a[k] > 0.0f ? x : 0.0f;
#pragma unroll
        for (int t = 0; t < 9; ++t) acc[k][t] = fmaf(a[k], win[2 - t / 3][2 - t % 3], acc[k][t]);
      }
      accb += win[1][1];
      const int gx = x0 + lx0 + e;
      if (gy < H && gx < W)
        hs_store4(g5 + (img + (size_t)gy * W + gx) * 32 + 4 * c4, o[0], o[1], o[2], o[3]);
    }
  }
#pragma unroll
  for (int k = 0; k < 4; ++k)
#pragma unroll
    for (int t = 0; t < 9; ++t) sred[seg][(4 * c4 + k) * 9 + t] = acc[k][t];
  if (c4 == 0) sred[seg][288] = accb;
  __syncthreads();
  for (int prm = threadIdx.x; prm <= 288; prm += blockDim.x) {
    float s = 0.0f;
#pragma unroll
    for (int k = 0; k < 32; ++k) s += sred[k][prm];
    float* d = partials + (size_t)blockIdx.x * hs::NPARAM + HS_W6 + prm;
    *d = accumulate ? *d + s : s;
  }
}

// Two-level fixed-order sum of the partial rows: group gi sums rows
// gi, gi + G, gi + 2G, ... into tmp[gi]; then the G group sums in order.
// rows: a multiple of WGRAD_BLOCKS (one set of rows per batch); the 32->32
// layers' parameters have partial sums only in the first rows32 rows of each
// set (their weight-gradient kernel's grid), the other rows are skipped
__global__ void reduce_partials_kernel(const float* __restrict__ partials, int rows, int rows32,
                                       float* __restrict__ tmp) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x, gi = blockIdx.y;
  if (p >= hs::NPARAM) return;
  const bool l32 = p >= hs_wk(2) && p < hs_bk(5) + 32;
  constexpr int G = hs::REDUCE_GROUPS;
  const float* col = partials + p;
  float s = 0.0f;
  // rows gi, gi + G, ... of each set in increasing order, four loads in flight
  for (int set = 0; set < rows; set += hs::WGRAD_BLOCKS) {
    const int end = set + (l32 ? rows32 : hs::WGRAD_BLOCKS);
    int r = set + gi;
    for (; r + 3 * G < end; r += 4 * G) {
      const float a = col[(size_t)r * hs::NPARAM], b = col[(size_t)(r + G) * hs::NPARAM];
      const float c = col[(size_t)(r + 2 * G) * hs::NPARAM];
      const float d = col[(size_t)(r + 3 * G) * hs::NPARAM];
      s += a;
      s += b;
      s += c;
      s += d;
    }
    for (; r < end; r += G) s += col[(size_t)r * hs::NPARAM];
  }
  tmp[(size_t)gi * hs::NPARAM + p] = s;
}

// also the block's sum of grad^2 into gsq[blockIdx.x] (waves in order)
__global__ __launch_bounds__(256) void reduce_groups_kernel(const float* __restrict__ tmp,
                                                            float* __restrict__ grad,
                                                            float* __restrict__ gsq) {
  __shared__ float part[4];
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  float s = 0.0f;
  if (p < hs::NPARAM) {
    for (int gi = 0; gi < hs::REDUCE_GROUPS; ++gi) s += tmp[(size_t)gi * hs::NPARAM + p];
    grad[p] = s;
  }
  float q = s * s;
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) q += __shfl_xor(q, o, 64);
  if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = q;
  __syncthreads();
  if (threadIdx.x == 0) gsq[blockIdx.x] = ((part[0] + part[1]) + part[2]) + part[3];
}

inline dim3 tiles16(int B, int H, int W) { return dim3((W + 15) / 16, (H + 15) / 16, B); }

}  // namespace

namespace hs {

hipError_t launch_pack32(const float* w, void* out, int precision, int transposed,
                         hipStream_t s) {
  const int y0 = transposed ? 4 : 0;
  if (precision == HS_BF16)
    pack32_kernel<__bf16><<<dim3(36, 4), 256, 0, s>>>(w, (__bf16*)out, (__bf16*)out, y0);
  else
    pack32_kernel<float><<<dim3(36, 4), 256, 0, s>>>(w, (float*)out, (float*)out, y0);
  return hipGetLastError();
}

hipError_t launch_pack32_both(const float* w, void* outF, void* outT, int precision,
                              hipStream_t s) {
  if (precision == HS_BF16)
    pack32_kernel<__bf16><<<dim3(36, 8), 256, 0, s>>>(w, (__bf16*)outF, (__bf16*)outT, 0);
  else
    pack32_kernel<float><<<dim3(36, 8), 256, 0, s>>>(w, (float*)outF, (float*)outT, 0);
  return hipGetLastError();
}

hipError_t launch_conv_first(const float* contone, const uint64_t* seeds, const float* w, int B,
                             int H, int W, int kind, uint32_t step, int precision, void* out,
                             float* zout, float* cout, hipStream_t s) {
  if (precision == HS_BF16)
    conv_first_mfma_kernel<<<dim3((W + CFM_TX - 1) / CFM_TX, (H + CFM_TY - 1) / CFM_TY, B), 256,
                             0, s>>>(contone, seeds, w, H, W, kind, step, (__bf16*)out, zout,
                                     cout);
  else
    conv_first_kernel<float><<<tiles16(B, H, W), 256, 0, s>>>(contone, seeds, w, H, W, kind,
                                                              step, (float*)out, zout, cout);
  return hipGetLastError();
}

hipError_t launch_conv32(const void* in, const void* wpack, const float* bias, const void* mask,
                         void* out, int B, int H, int W, int precision, int mode, hipStream_t s) {
  const int ct_h = precision == HS_BF16 ? conv_rows<__bf16>::CT_H : conv_rows<float>::CT_H;
  const dim3 grid((W + CT_W - 1) / CT_W, (H + ct_h - 1) / ct_h, B);
  if (precision == HS_BF16) {
    // the input gradient of a BF16 layer comes from the fused backward
    if (mode != 0) return hipErrorInvalidValue;
    const int ntiles = (int)(grid.x * grid.y * grid.z);
    conv32_fwd_bf16_kernel<<<ntiles < CF_BLOCKS ? ntiles : CF_BLOCKS, 256, 0, s>>>(
        (const __bf16*)in, (const __bf16*)wpack, bias, (__bf16*)out, B, H, W);
  } else {
    if (mode == 0)
      conv32_kernel<float, 0><<<grid, 256, 0, s>>>((const float*)in, (const float*)wpack, bias,
                                                   nullptr, (float*)out, H, W);
    else
      conv32_kernel<float, 1><<<grid, 256, 0, s>>>((const float*)in, (const float*)wpack, nullptr,
                                                   (const float*)mask, (float*)out, H, W);
  }
  return hipGetLastError();
}

hipError_t launch_conv_last(const void* in, const float* w, int B, int H, int W, int precision,
                            int mode, const uint64_t* seeds, uint32_t step, uint8_t* bits,
                            float* logits, float* probs, float tau, uint32_t* list, int* count,
                            const Levels& lv, hipStream_t s) {
  const dim3 grid = tiles16(B, H, W);
  if (precision == HS_BF16) {
    if (mode == 0)
      conv_last_kernel<__bf16, 0><<<grid, 256, 0, s>>>((const __bf16*)in, w, H, W, seeds, step,
                                                       bits, logits, probs, tau, list, count, lv);
    else
      conv_last_mfma_kernel<<<dim3((W + CLM_TX - 1) / CLM_TX, (H + CLM_TY - 1) / CLM_TY, B), 256,
                              0, s>>>((const __bf16*)in, w, H, W, seeds, step, bits, probs, lv);
  } else {
    if (mode == 0)
      conv_last_kernel<float, 0><<<grid, 256, 0, s>>>((const float*)in, w, H, W, seeds, step,
                                                      bits, logits, probs, tau, list, count, lv);
    else
      conv_last_kernel<float, 1><<<grid, 256, 0, s>>>((const float*)in, w, H, W, seeds, step,
                                                      bits, logits, probs, tau, list, count, lv);
  }
  return hipGetLastError();
}

hipError_t launch_dgrad_last(const float* grad, const float* probs, const void* a5,
                             const float* w, int B, int H, int W, int precision, float* g6,
                             void* g5, hipStream_t s) {
  const dim3 grid = tiles16(B, H, W);
  if (precision == HS_BF16)
    dgrad_last_kernel<__bf16><<<grid, 256, 0, s>>>(grad, probs, (const __bf16*)a5, w, H, W, g6,
                                                   (__bf16*)g5);
  else
    dgrad_last_kernel<float><<<grid, 256, 0, s>>>(grad, probs, (const float*)a5, w, H, W, g6,
                                                  (float*)g5);
  return hipGetLastError();
}

hipError_t launch_bwd_last(const float* grad, const float* probs, const void* a5, const float* w,
                           int B, int H, int W, int precision, float* g6, void* g5,
                           float* partials, int accumulate, hipStream_t s) {
  if (precision == HS_BF16) {
    bwd_last_bf16_kernel<<<WGRAD_BLOCKS, 256, 0, s>>>(grad, probs, (const __bf16*)a5, w, B, H, W,
                                                      (__bf16*)g5, partials, accumulate);
    return hipGetLastError();
  }
  hipError_t e = launch_dgrad_last(grad, probs, a5, w, B, H, W, precision, g6, g5, s);
  if (e != hipSuccess) return e;
  return launch_wgrad_last(a5, g6, B, H, W, precision, partials, accumulate, s);
}

hipError_t launch_wgrad_first(const float* contone, const float* z, const void* g1, int B, int H,
                              int W, int precision, float* partials, int accumulate,
                              hipStream_t s) {
  if (precision == HS_BF16)
    wgrad_first_bf16_kernel<<<WGRAD_BLOCKS, 256, 0, s>>>(contone, z, (const __bf16*)g1, B, H, W,
                                                         partials, accumulate);
  else
    wgrad_first_kernel<float><<<WGRAD_BLOCKS, 256, 0, s>>>(contone, z, (const float*)g1, B, H, W,
                                                           partials, accumulate);
  return hipGetLastError();
}

hipError_t launch_wgrad32(const void* a_in, const void* g_out, int layer, int B, int H, int W,
                          int precision, float* partials, int accumulate, hipStream_t s) {
  // BF16 layers take the fused backward (launch_bwd32)
  if (precision == HS_BF16) return hipErrorInvalidValue;
  wgrad32_kernel<float><<<WGRAD_BLOCKS, 256, 0, s>>>((const float*)a_in, (const float*)g_out, B,
                                                     H, W, layer, partials, accumulate);
  return hipGetLastError();
}

hipError_t launch_bwd32(const void* a_in, const void* g_out, const void* wpackT, void* g_in,
                        int layer, int B, int H, int W, float* partials, int accumulate,
                        int num_cus, hipStream_t s) {
  // one block per CU (its LDS allows no second), all resident at once
  const int grid = bwd32_grid(num_cus);
  bwd32_bf16_kernel<<<grid, FB_NT, 0, s>>>((const __bf16*)a_in, (const __bf16*)g_out,
                                                   (const __bf16*)wpackT, (__bf16*)g_in, B, H, W,
                                                   layer, partials, accumulate);
  return hipGetLastError();
}

hipError_t launch_wgrad_last(const void* a5, const float* g6, int B, int H, int W, int precision,
                             float* partials, int accumulate, hipStream_t s) {
  if (precision == HS_BF16)
    wgrad_last_kernel<__bf16><<<WGRAD_BLOCKS, 256, 0, s>>>((const __bf16*)a5, g6, B, H, W,
                                                           partials, accumulate);
  else
    wgrad_last_kernel<float><<<WGRAD_BLOCKS, 256, 0, s>>>((const float*)a5, g6, B, H, W, partials,
                                                          accumulate);
  return hipGetLastError();
}

int bwd32_grid(int num_cus) {
  return num_cus < WGRAD_BLOCKS ? (num_cus > 0 ? num_cus : 1) : WGRAD_BLOCKS;
}

hipError_t launch_reduce_partials(const float* partials, int rows, int rows32, float* tmp,
                                  float* grad, hipStream_t s) {
  if (rows <= 0 || rows % WGRAD_BLOCKS != 0 || rows32 <= 0 || rows32 > WGRAD_BLOCKS)
    return hipErrorInvalidValue;
  reduce_partials_kernel<<<dim3((NPARAM + 255) / 256, REDUCE_GROUPS), 256, 0, s>>>(
      partials, rows, rows32, tmp);
  reduce_groups_kernel<<<REDUCE_BLOCKS, 256, 0, s>>>(tmp, grad,
                                                     tmp + (size_t)REDUCE_GROUPS * NPARAM);
  return hipGetLastError();
}

hipError_t launch_reduce_rows(const float* partials, int rows, int rows32, float* tmp,
                              hipStream_t s) {
  if (rows <= 0 || rows % WGRAD_BLOCKS != 0 || rows32 <= 0 || rows32 > WGRAD_BLOCKS)
    return hipErrorInvalidValue;
  reduce_partials_kernel<<<dim3((NPARAM + 255) / 256, REDUCE_GROUPS), 256, 0, s>>>(
      partials, rows, rows32, tmp);
  return hipGetLastError();
}


}  // namespace hs
