// infer.hip -- the TEST procedure of Algorithm 1 on gfx950: FP32
// re-evaluation of the pixels whose low-precision logit falls near the 0.5
// threshold.
//
// A listed pixel is recomputed exactly as the FP32 network would compute it,
// over its 13 x 13 receptive field only: layer k is evaluated on the
// (13 - 2k) x (13 - 2k) window centred on the pixel, with every activation
// outside the image forced to zero (the zero 'same' padding of each layer).
#include "hs_common.h"
#include "hs_internal.h"

namespace {

constexpr int RS = 33;  // padded channel stride of a staged pixel (floats)

__global__ void zero_ints_kernel(int* p, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = 0;
}

// One block re-evaluates one listed pixel at a time (grid-stride over the
// list, whose length is read on the device).
__global__ __launch_bounds__(256) void recheck_fp32_kernel(
    const float* __restrict__ w, const float* __restrict__ contone,
    const uint64_t* __restrict__ seeds, int H, int W, int kind, const uint32_t* __restrict__ list,
    const int* __restrict__ count, uint8_t* __restrict__ bits, float* __restrict__ logits,
    int32_t* __restrict__ stats, int count_slot) {
  __shared__ float s0[13 * 13 * 2];
  __shared__ float bufA[11 * 11 * RS], bufB[9 * 9 * RS];
  __shared__ float sw[9 * 32 * 32];  // [ci][t][co]: consecutive lanes read consecutive co
  __shared__ float sb[32];
  const int n = *count;
  const int tid = threadIdx.x;
  for (int it = blockIdx.x; it < n; it += gridDim.x) {
    const uint32_t o = list[it];
    const int b = (int)(o / ((uint32_t)H * W));
    const int rem = (int)(o - (uint32_t)b * H * W), y = rem / W, x = rem - (rem / W) * W;
    const size_t img = (size_t)b * H * W;
    __syncthreads();
    for (int i = tid; i < 169; i += 256) {
      const int gy = y - 6 + i / 13, gx = x - 6 + i % 13;
      float cv = 0.f, zv = 0.f;
      if (gy >= 0 && gy < H && gx >= 0 && gx < W) {
        const uint64_t a = (uint64_t)gy * W + gx;
        cv = contone[img + a];
        zv = hs_noise(seeds[b], a, 0u, kind);
      }
      s0[i * 2] = cv;
      s0[i * 2 + 1] = zv;
    }
    for (int i = tid; i < 32 * 2 * 9; i += 256) {
      const int co = i / 18, ci = (i / 9) & 1, t = i % 9;
      sw[(ci * 9 + t) * 32 + co] = w[HS_W1 + i];
    }
    if (tid < 32) sb[tid] = w[HS_B1 + tid];
    __syncthreads();
    // layer 1 on the 11 x 11 window
    for (int i = tid; i < 121 * 32; i += 256) {
      const int co = i & 31, p = i >> 5, py = p / 11, px = p % 11;
      const int gy = y - 5 + py, gx = x - 5 + px;
      float acc = 0.f;
      if (gy >= 0 && gy < H && gx >= 0 && gx < W) {
        acc = sb[co];
        for (int t = 0; t < 9; ++t) {
          const int q = (py + t / 3) * 13 + px + t % 3;
          acc = fmaf(sw[(0 * 9 + t) * 32 + co], s0[q * 2], acc);
          acc = fmaf(sw[(1 * 9 + t) * 32 + co], s0[q * 2 + 1], acc);
        }
        acc = fmaxf(acc, 0.f);
      }
      bufA[p * RS + co] = acc;
    }
    // layers 2..5: window edges 9, 7, 5, 3
    for (int k = 2; k <= 5; ++k) {
      const int e_in = 13 - 2 * (k - 1), e_out = 13 - 2 * k;
      const float* src = (k & 1) ? bufB : bufA;
      float* dst = (k & 1) ? bufA : bufB;
      __syncthreads();
      const float* Wk = w + hs_wk(k);
      for (int i = tid; i < 9 * 32 * 32; i += 256) {
        const int co = i / 288, ci = (i / 9) & 31, t = i % 9;
        sw[(ci * 9 + t) * 32 + co] = Wk[i];
      }
      if (tid < 32) sb[tid] = w[hs_bk(k) + tid];
      __syncthreads();
      for (int i = tid; i < e_out * e_out * 32; i += 256) {
        const int co = i & 31, p = i >> 5, py = p / e_out, px = p % e_out;
        const int gy = y - (6 - k) + py, gx = x - (6 - k) + px;
        float acc = 0.f;
        if (gy >= 0 && gy < H && gx >= 0 && gx < W) {
          acc = sb[co];
          for (int t = 0; t < 9; ++t) {
            const float* sp = src + ((py + t / 3) * e_in + px + t % 3) * RS;
            const float* wp = sw + t * 32 + co;
#pragma unroll 8
            for (int ci = 0; ci < 32; ++ci) acc = fmaf(wp[ci * 9 * 32], sp[ci], acc);
          }
          acc = fmaxf(acc, 0.f);
        }
        dst[p * RS + co] = acc;
      }
    }
    __syncthreads();
    // layer 6 at the centre of the 3 x 3 window (in bufA)
    if (tid < 64) {
      float part = 0.f;
      for (int i = tid; i < 288; i += 64) {
        const int ci = i / 9, t = i % 9;
        part = fmaf(w[HS_W6 + i], bufA[((t / 3) * 3 + t % 3) * RS + ci], part);
      }
      part = hs_wave_sum(part);
      if (tid == 0) {
        const float xl = part + w[HS_B6];
        const uint8_t nb = xl >= 0.f ? 1 : 0;
        if (bits[o] != nb) atomicAdd(&stats[1], 1);
        bits[o] = nb;
        if (logits) logits[o] = xl;
      }
    }
  }
  if (blockIdx.x == 0 && tid == 0) stats[count_slot] = n;
}

}  // namespace

namespace hs {

hipError_t launch_zero_ints(int* p, int n, hipStream_t s) {
  zero_ints_kernel<<<(n + 255) / 256, 256, 0, s>>>(p, n);
  return hipGetLastError();
}

hipError_t launch_recheck_fp32(const float* w, const float* contone, const uint64_t* seeds,
                               int H, int W, int kind, const uint32_t* list, const int* count,
                               uint8_t* bits, float* logits, int32_t* stats, int count_slot,
                               hipStream_t s) {
  recheck_fp32_kernel<<<1024, 256, 0, s>>>(w, contone, seeds, H, W, kind, list, count, bits,
                                           logits, stats, count_slot);
  return hipGetLastError();
}

}  // namespace hs

// ===========================================================================
// Fused BF16 inference: one persistent kernel runs all six layers of the
// policy over vertical strips of the image, streaming down the rows.
//
// A strip is FW = 128 computed columns, of which the central FS = 116 are
// valid outputs (the 13 x 13 receptive field eats 6 columns on each side).
// Every layer keeps a ring of three rows of its output in LDS (BF16, 32
// channels, 64 B per pixel), so activations never leave the chip. Each step
// advances every stage by one row: the input stage (contone + Philox noise),
// conv layers 1..5, the per-tap partial sums T of layer 6 (one MFMA gives the
// nine taps' 32-channel dot products of a pixel), and the output stage (the
// nine-tap shift-add of T, the threshold and the recheck flag). A stage reads
// rows written at earlier steps only (phase A), then all stages write their
// new row (phase B); so consecutive stages lag by two rows (one for T).
//
// Work per step: eight waves; conv layer k (2..5) belongs to waves
// 2(k-2), 2(k-2)+1, each owning four 16-pixel runs of the row and holding
// its layer's weights in registers for the whole kernel. Layer 1 runs on
// waves 0-1, the T stage on waves 6-7, the input stage on waves 2-3 and the
// output stage on waves 4-5.
//
// Channel order in the rings: the MFMA result of lane (g, r) holds output
// channels {4g..4g+3, 16+4g..16+4g+3} of pixel r; those eight channels are
// stored as the lane's 16-byte chunk and read back as the same lane group's
// K-slice by the next layer, whose weights are packed in that order.
// ===========================================================================
namespace {

constexpr int FW = 128, FS = FW - 12, RWID = FW + 2, FNT = FW / 16;
constexpr int LAG_OUT = 19;  // steps from input row Y0-6 to output row Y0
constexpr int FRAG_L1 = 0, FRAG_L32 = 128, FRAG_T = 128 + 4 * 9 * 2 * 64;
constexpr int FRAG_TOTAL = FRAG_T + 64;

// channel held by slot e of lane group g in the ring order
HS_DEV int ring_channel(int g, int e) { return e < 4 ? 4 * g + e : 16 + 4 * g + (e - 4); }

__global__ void pack_fused_kernel(const float* __restrict__ w, __bf16* __restrict__ out) {
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < FRAG_TOTAL * 8;
       i += gridDim.x * blockDim.x) {
    const int f = i >> 3, e = i & 7;
    float v = 0.0f;
    if (f < FRAG_L32) {  // layer 1: slot j = 8g + e holds (tap j/2, channel j%2)
      const int m = f >> 6, l = f & 63, g = l >> 4, r = l & 15;
      const int j = 8 * g + e, co = 16 * m + r;
      if (j < 18) v = w[HS_W1 + (co * 2 + (j & 1)) * 9 + (j >> 1)];
    } else if (f < FRAG_T) {  // layers 2..5: [layer][tap][m][lane]
      const int q = f - FRAG_L32, l = q & 63, m = (q >> 6) & 1, t = (q >> 7) % 9,
                layer = (q >> 7) / 9;
      const int g = l >> 4, r = l & 15;
      v = w[hs_wk(layer + 2) + ((16 * m + r) * 32 + ring_channel(g, e)) * 9 + t];
    } else {  // layer 6 as T[tap][pixel] = sum_ci W6[ci][tap] a5[pixel][ci]
      const int l = f - FRAG_T, g = l >> 4, r = l & 15;
      if (r < 9) v = w[HS_W6 + ring_channel(g, e) * 9 + r];
    }
    out[i] = (__bf16)v;
  }
}

struct FusedArgs {
  const float* contone;
  const uint64_t* seeds;
  const bf16x8_t* frags;
  const float* w;
  int B, H, W, kind, nstrip;
  long long total_rows, rows_per_wg;
  float tau;
  uint8_t* bits;
  float* logits;
  uint32_t* list;
  int* count;
};

HS_DEV int slot3(int row) { return ((row % 3) + 3) % 3; }

__global__ __launch_bounds__(512, 1) void fused_infer_kernel(FusedArgs a) {
  __shared__ __attribute__((aligned(16))) __bf16 ring[5 * 3 * RWID * 32];
  __shared__ uint32_t inring[3 * RWID];
  __shared__ __attribute__((aligned(16))) float tring[3 * RWID * 12];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6, g = lane >> 4, r = lane & 15;
  const int half = wave & 1, k = 2 + (wave >> 1);  // conv layer owned by this wave
  for (int i = tid; i < 5 * 3 * RWID * 32 / 8; i += 512) ((uint4*)ring)[i] = make_uint4(0, 0, 0, 0);
  for (int i = tid; i < 3 * RWID; i += 512) inring[i] = 0u;
  for (int i = tid; i < 3 * RWID * 12; i += 512) tring[i] = 0.0f;
  // weights of the owned layer (A operands) and its bias for this lane's channels
  bf16x8_t wA[9][2];
#pragma unroll
  for (int t = 0; t < 9; ++t)
#pragma unroll
    for (int m = 0; m < 2; ++m) wA[t][m] = a.frags[FRAG_L32 + (((k - 2) * 9 + t) * 2 + m) * 64 + lane];
  float bk[2][4];
#pragma unroll
  for (int m = 0; m < 2; ++m)
#pragma unroll
    for (int i = 0; i < 4; ++i) bk[m][i] = a.w[hs_bk(k) + 16 * m + 4 * g + i];
  // role-specific operands share registers: waves 0-1 hold layer 1's two A
  // operands and bias, waves 6-7 the layer-6 tap matrix
  bf16x8_t wx[2];
  float b1[2][4];
  if (wave < 2) {
    wx[0] = a.frags[FRAG_L1 + lane];
    wx[1] = a.frags[FRAG_L1 + 64 + lane];
#pragma unroll
    for (int m = 0; m < 2; ++m)
#pragma unroll
      for (int i = 0; i < 4; ++i) b1[m][i] = a.w[HS_B1 + 16 * m + 4 * g + i];
  } else {
    wx[0] = a.frags[FRAG_T + lane];
    wx[1] = wx[0];
#pragma unroll
    for (int m = 0; m < 2; ++m)
#pragma unroll
      for (int i = 0; i < 4; ++i) b1[m][i] = 0.0f;
  }
  const float b6 = a.w[HS_B6];
  __syncthreads();

  const long long Lbeg = (long long)blockIdx.x * a.rows_per_wg;
  const long long Lend = Lbeg + a.rows_per_wg < a.total_rows ? Lbeg + a.rows_per_wg : a.total_rows;
  const int H = a.H, W = a.W;
  for (long long L = Lbeg; L < Lend;) {
    const long long strip_id = L / H;
    const int Y0 = (int)(L - strip_id * H);
    const long long seg_end = (strip_id + 1) * H < Lend ? (strip_id + 1) * H : Lend;
    const int Y1 = Y0 + (int)(seg_end - L);
    const int b = (int)(strip_id / a.nstrip), s = (int)(strip_id % a.nstrip);
    const int X = s * FS - 6;
    const size_t img = (size_t)b * H * W;
    const uint64_t seed = a.seeds[b];
    const int nsteps = (Y1 - Y0) + LAG_OUT;
    for (int t = 0; t < nsteps; ++t) {
      // ------------------------------------------------------------ phase A
      const int rk = Y0 - 6 - 2 * k + t;  // row of the owned conv layer
      f32x4_t acc[4][2];
      const int rin = rk - 1;  // first input row of the owned layer
      const __bf16* src = ring + (size_t)(k - 2) * 3 * RWID * 32;
#pragma unroll
      for (int n = 0; n < 4; ++n) {
        acc[n][0] = f32x4_t{0.f, 0.f, 0.f, 0.f};
        acc[n][1] = f32x4_t{0.f, 0.f, 0.f, 0.f};
      }
#pragma unroll
      for (int dy = 0; dy < 3; ++dy) {
        const __bf16* rowp = src + (size_t)slot3(rin + dy) * RWID * 32;
#pragma unroll
        for (int dx = 0; dx < 3; ++dx) {
#pragma unroll
          for (int n = 0; n < 4; ++n) {
            const int col = 16 * (4 * half + n) + r + dx;
            const bf16x8_t bf = *(const bf16x8_t*)(rowp + col * 32 + hs_swz<__bf16>(col, g) * 8);
            acc[n][0] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(wA[dy * 3 + dx][0], bf, acc[n][0], 0, 0, 0);
            acc[n][1] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(wA[dy * 3 + dx][1], bf, acc[n][1], 0, 0, 0);
          }
        }
      }
      // extra duty of each wave pair
      f32x4_t accx[4][2];  // layer 1 (waves 0-1) or the T stage (waves 6-7, [n][0])
      float cval = 0.f, zval = 0.f;
      const int r1 = Y0 - 8 + t, r0 = Y0 - 6 + t, r6 = Y0 - 17 + t, r7 = Y0 - 19 + t;
      if (wave < 2) {  // layer 1 from the input ring
#pragma unroll
        for (int n = 0; n < 4; ++n) {
          const int c0 = 16 * (4 * half + n) + r;  // column of tap dx = 0
          uint32_t u[4] = {0u, 0u, 0u, 0u};
#pragma unroll
          for (int e = 0; e < 4; ++e) {
            const int tap = 4 * g + e;
            if (tap < 9) {
              const int dy = tap / 3, dx = tap - 3 * (tap / 3);
              u[e] = inring[slot3(r1 - 1 + dy) * RWID + c0 + dx];
            }
          }
          bf16x8_t bf;
          __builtin_memcpy(&bf, u, 16);
          accx[n][0] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(wx[0], bf, f32x4_t{0.f, 0.f, 0.f, 0.f}, 0, 0, 0);
          accx[n][1] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(wx[1], bf, f32x4_t{0.f, 0.f, 0.f, 0.f}, 0, 0, 0);
        }
      } else if (wave < 4) {  // input stage: contone and noise of row r0
        const int Lx = (wave - 2) * 64 + lane, x = X + Lx;
        if (r0 >= 0 && r0 < H && x >= 0 && x < W) {
          const uint64_t ap = (uint64_t)r0 * W + x;
          cval = a.contone[img + ap];
          zval = hs_noise(seed, ap, 0u, a.kind);
        }
      } else if (wave < 6) {  // output stage: row r7
        const int Lx = (wave - 4) * 64 + lane, x = X + Lx;
        const bool valid = Lx >= 6 && Lx < 6 + FS && x < W && r7 >= Y0 && r7 < Y1;
        bool flag = false;
        size_t o = 0;
        if (valid) {
          float xl = b6;
#pragma unroll
          for (int dy = 0; dy < 3; ++dy) {
            const float* trow = tring + (size_t)slot3(r7 - 1 + dy) * RWID * 12;
#pragma unroll
            for (int dx = 0; dx < 3; ++dx) xl += trow[(Lx + dx) * 12 + dy * 3 + dx];
          }
          o = img + (size_t)r7 * W + x;
          a.bits[o] = xl >= 0.0f ? 1 : 0;
          if (a.logits) a.logits[o] = xl;
          flag = a.list && fabsf(xl) < a.tau;
        }
        const uint64_t mask = __ballot(flag);
        if (mask) {
          const int cnt = __popcll(mask);
          int base = 0;
          const int leader = __ffsll((unsigned long long)mask) - 1;
          if (lane == leader) base = atomicAdd(a.count, cnt);
          base = __shfl(base, leader, 64);
          if (flag) {
            const uint64_t lower = lane ? (mask & ((~0ull) >> (64 - lane))) : 0ull;
            a.list[base + __popcll(lower)] = (uint32_t)o;
          }
        }
      } else {  // T stage: nine taps of layer 6 on row r6 of layer 5
        const __bf16* rowp = ring + ((size_t)4 * 3 + slot3(r6)) * RWID * 32;
#pragma unroll
        for (int n = 0; n < 4; ++n) {
          const int col = 16 * (4 * half + n) + r + 1;
          const bf16x8_t bf = *(const bf16x8_t*)(rowp + col * 32 + hs_swz<__bf16>(col, g) * 8);
          accx[n][0] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(wx[0], bf, f32x4_t{0.f, 0.f, 0.f, 0.f}, 0, 0, 0);
        }
      }
      __syncthreads();
      // ------------------------------------------------------------ phase B
      {
        __bf16* dst = ring + ((size_t)(k - 1) * 3 + slot3(rk)) * RWID * 32;
        const bool row_in = rk >= 0 && rk < H;
#pragma unroll
        for (int n = 0; n < 4; ++n) {
          const int col = 16 * (4 * half + n) + r + 1, x = X + col - 1;
          const bool in = row_in && x >= 0 && x < W;
          bf16x8_t v;
#pragma unroll
          for (int m = 0; m < 2; ++m)
#pragma unroll
            for (int i = 0; i < 4; ++i)
              v[4 * m + i] = (__bf16)(in ? fmaxf(acc[n][m][i] + bk[m][i], 0.0f) : 0.0f);
          *(bf16x8_t*)(dst + col * 32 + hs_swz<__bf16>(col, g) * 8) = v;
        }
      }
      if (wave < 2) {
        __bf16* dst = ring + (size_t)slot3(r1) * RWID * 32;
        const bool row_in = r1 >= 0 && r1 < H;
#pragma unroll
        for (int n = 0; n < 4; ++n) {
          const int col = 16 * (4 * half + n) + r + 1, x = X + col - 1;
          const bool in = row_in && x >= 0 && x < W;
          bf16x8_t v;
#pragma unroll
          for (int m = 0; m < 2; ++m)
#pragma unroll
            for (int i = 0; i < 4; ++i)
              v[4 * m + i] = (__bf16)(in ? fmaxf(accx[n][m][i] + b1[m][i], 0.0f) : 0.0f);
          *(bf16x8_t*)(dst + col * 32 + hs_swz<__bf16>(col, g) * 8) = v;
        }
      } else if (wave < 4) {
        const int Lx = (wave - 2) * 64 + lane;
        const __bf16 cz[2] = {(__bf16)cval, (__bf16)zval};
        uint32_t u;
        __builtin_memcpy(&u, cz, 4);
        inring[slot3(r0) * RWID + Lx + 1] = u;
      } else if (wave >= 6) {
        float* trow = tring + (size_t)slot3(r6) * RWID * 12;
#pragma unroll
        for (int n = 0; n < 4; ++n) {
          const int col = 16 * (4 * half + n) + r + 1;
          if (g < 3) *(f32x4_t*)(trow + col * 12 + 4 * g) = accx[n][0];
        }
      }
      __syncthreads();
    }
    L = seg_end;
  }
}

}  // namespace

namespace hs {

size_t fused_frag_bytes() { return (size_t)FRAG_TOTAL * 16; }

hipError_t launch_fused_pack(const float* w, void* frags, hipStream_t s) {
  pack_fused_kernel<<<38, 256, 0, s>>>(w, (__bf16*)frags);
  return hipGetLastError();
}

hipError_t launch_fused_infer(const float* w, const float* contone, const uint64_t* seeds, int B,
                              int H, int W, int kind, float tau, uint8_t* bits, float* logits,
                              uint32_t* list, int* count, const void* frags, int num_cus,
                              hipStream_t s) {
  FusedArgs a;
  a.contone = contone;
  a.seeds = seeds;
  a.frags = (const bf16x8_t*)frags;
  a.w = w;
  a.B = B;
  a.H = H;
  a.W = W;
  a.kind = kind;
  a.nstrip = (W + FS - 1) / FS;
  a.total_rows = (long long)B * a.nstrip * H;
  long long per = (a.total_rows + num_cus - 1) / num_cus;
  if (per < 32) per = 32;
  a.rows_per_wg = per;
  a.tau = tau;
  a.bits = bits;
  a.logits = logits;
  a.list = list;
  a.count = count;
  const int grid = (int)((a.total_rows + per - 1) / per);
  fused_infer_kernel<<<grid, 512, 0, s>>>(a);
  return hipGetLastError();
}

}  // namespace hs

// ===========================================================================
// Second-stage recheck: the listed pixels' receptive fields recomputed with
// split-BF16 products on the matrix cores. Every FP32 value v is carried as
// hi + lo with hi = bf16(v), lo = bf16(v - hi); a product is taken as
// hi*hi' + lo*hi' + hi*lo' (the lo*lo' term, ~2^-16 relative, is dropped),
// accumulated in FP32. Layer 1 and layer 6 are evaluated in plain FP32. The
// result's error is ~2^-8 of the BF16 pass's, so a pixel is decided here
// when |x| >= tau2; the rest go to the FP32 stage.
//
// A block takes CB = 4 listed pixels at a time. For layer k the four cones'
// (13-2k)^2 output positions are cut into 16-position runs (the N operand);
// the layer's hi and lo weight fragments sit in LDS for all runs.
// ===========================================================================
namespace {

constexpr int CB = 4;                 // cones per block
constexpr int CREC = 128;             // bytes per staged pixel: 4 groups x (hi, lo) x 16 B
constexpr int CBUF_A = 121, CBUF_B = 81;

__global__ void pack_split_kernel(const float* __restrict__ w, __bf16* __restrict__ hi,
                                  __bf16* __restrict__ lo) {
  // layers 2..5 in the ring channel order of the fused kernel: [layer][tap][m][lane][8]
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < 4 * 9 * 2 * 64 * 8;
       i += gridDim.x * blockDim.x) {
    const int e = i & 7, l = (i >> 3) & 63, m = (i >> 9) & 1, t = (i >> 10) % 9,
              layer = (i >> 10) / 9;
    const int g = l >> 4, r = l & 15;
    const float v = w[hs_wk(layer + 2) + ((16 * m + r) * 32 + ring_channel(g, e)) * 9 + t];
    const __bf16 h = (__bf16)v;
    hi[i] = h;
    lo[i] = (__bf16)(v - (float)h);
  }
}

HS_DEV int crec_slot(int p, int c) { return c ^ (p & 7); }

__global__ __launch_bounds__(256) void recheck_split_kernel(
    const float* __restrict__ w, const float* __restrict__ contone,
    const uint64_t* __restrict__ seeds, int H, int W, int kind, const uint32_t* __restrict__ list,
    const int* __restrict__ count, const bf16x8_t* __restrict__ whi,
    const bf16x8_t* __restrict__ wlo, float tau2, uint32_t* __restrict__ list2,
    int* __restrict__ count2, uint8_t* __restrict__ bits, float* __restrict__ logits,
    int32_t* __restrict__ stats) {
  __shared__ __attribute__((aligned(16))) bf16x8_t swh[9 * 2 * 64], swl[9 * 2 * 64];
  __shared__ __attribute__((aligned(16))) char bufA[CB][CBUF_A * CREC];
  __shared__ __attribute__((aligned(16))) char bufB[CB][CBUF_B * CREC];
  __shared__ float s0[CB][169 * 2];
  __shared__ float sw1[32 * 2 * 9 + 32];
  __shared__ float l5f[CB][9 * 32];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6, g = lane >> 4, r = lane & 15;
  const int n = *count;
  for (int i = tid; i < 608; i += 256) sw1[i] = w[HS_W1 + i];
  for (int base = blockIdx.x * CB; base < n; base += gridDim.x * CB) {
    const int ncone = n - base < CB ? n - base : CB;
    __syncthreads();
    // stage the 13 x 13 state (c, z) of each cone, zero outside the image
    for (int i = tid; i < CB * 169; i += 256) {
      const int cidx = i / 169, q = i - cidx * 169;
      float cv = 0.f, zv = 0.f;
      if (cidx < ncone) {
        const uint32_t o = list[base + cidx];
        const int b = (int)(o / ((uint32_t)H * W));
        const int rem = (int)(o - (uint32_t)b * H * W), y = rem / W, x = rem - (rem / W) * W;
        const int gy = y - 6 + q / 13, gx = x - 6 + q % 13;
        if (gy >= 0 && gy < H && gx >= 0 && gx < W) {
          const uint64_t a = (uint64_t)gy * W + gx;
          cv = contone[(size_t)b * H * W + a];
          zv = hs_noise(seeds[b], a, 0u, kind);
        }
      }
      s0[cidx][q * 2] = cv;
      s0[cidx][q * 2 + 1] = zv;
    }
    __syncthreads();
    // layer 1 in FP32 on the 11 x 11 windows; outputs stored split, in the
    // ring channel order (chunk g holds channels 4g..4g+3, 16+4g..16+4g+3)
    for (int i = tid; i < CB * 121 * 4; i += 256) {
      const int cidx = i / 484, rem = i - cidx * 484, p = rem >> 2, cg = rem & 3;
      const int py = p / 11, px = p - (p / 11) * 11;
      const uint32_t o = list[base + (cidx < ncone ? cidx : 0)];
      const int b = (int)(o / ((uint32_t)H * W));
      const int rr = (int)(o - (uint32_t)b * H * W), y = rr / W, x = rr - (rr / W) * W;
      const int gy = y - 5 + py, gx = x - 5 + px;
      const bool in = cidx < ncone && gy >= 0 && gy < H && gx >= 0 && gx < W;
      bf16x8_t vh, vl;
#pragma unroll
      for (int e = 0; e < 8; ++e) {
        const int co = ring_channel(cg, e);
        float acc = 0.f;
        if (in) {
          acc = sw1[HS_B1 + co];
#pragma unroll
          for (int t = 0; t < 9; ++t) {
            const int q = (py + t / 3) * 13 + px + t % 3;
            acc = fmaf(sw1[(co * 2) * 9 + t], s0[cidx][q * 2], acc);
            acc = fmaf(sw1[(co * 2 + 1) * 9 + t], s0[cidx][q * 2 + 1], acc);
          }
          acc = fmaxf(acc, 0.f);
        }
        const __bf16 h = (__bf16)acc;
        vh[e] = h;
        vl[e] = (__bf16)(acc - (float)h);
      }
      char* rec = bufA[cidx] + p * CREC;
      *(bf16x8_t*)(rec + crec_slot(p, 2 * cg) * 16) = vh;
      *(bf16x8_t*)(rec + crec_slot(p, 2 * cg + 1) * 16) = vl;
    }
    // layers 2..5 on the matrix cores
    for (int k = 2; k <= 5; ++k) {
      const int e_out = 13 - 2 * k, e_in = e_out + 2, npos = e_out * e_out;
      const int runs = (npos + 15) / 16;
      __syncthreads();
      for (int i = tid; i < 9 * 2 * 64; i += 256) {
        swh[i] = whi[(k - 2) * 9 * 2 * 64 + i];
        swl[i] = wlo[(k - 2) * 9 * 2 * 64 + i];
      }
      __syncthreads();
      const bool from_a = (k & 1) == 0;  // layer 2 reads A, 3 reads B, ...
      float bk[2][4];
#pragma unroll
      for (int m = 0; m < 2; ++m)
#pragma unroll
        for (int i = 0; i < 4; ++i) bk[m][i] = w[hs_bk(k) + 16 * m + 4 * g + i];
      for (int job = wave; job < CB * runs; job += 4) {
        const int cidx = job / runs, run = job - cidx * runs;
        const char* src = from_a ? bufA[cidx] : bufB[cidx];
        char* dst = from_a ? bufB[cidx] : bufA[cidx];
        const int pos = run * 16 + r;  // this lane's output position
        const int pi = pos < npos ? pos / e_out : 0, pj = pos < npos ? pos - pi * e_out : 0;
        f32x4_t acc[2] = {f32x4_t{0.f, 0.f, 0.f, 0.f}, f32x4_t{0.f, 0.f, 0.f, 0.f}};
#pragma unroll
        for (int t = 0; t < 9; ++t) {
          const int q = (pi + t / 3) * e_in + pj + t % 3;
          const char* rec = src + q * CREC;
          const bf16x8_t bh = *(const bf16x8_t*)(rec + crec_slot(q, 2 * g) * 16);
          const bf16x8_t bl = *(const bf16x8_t*)(rec + crec_slot(q, 2 * g + 1) * 16);
#pragma unroll
          for (int m = 0; m < 2; ++m) {
            const bf16x8_t ah = swh[(t * 2 + m) * 64 + lane], al = swl[(t * 2 + m) * 64 + lane];
            acc[m] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, bh, acc[m], 0, 0, 0);
            acc[m] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(al, bh, acc[m], 0, 0, 0);
            acc[m] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, bl, acc[m], 0, 0, 0);
          }
        }
        if (pos < npos && cidx < ncone) {
          const uint32_t o = list[base + cidx];
          const int b = (int)(o / ((uint32_t)H * W));
          const int rr = (int)(o - (uint32_t)b * H * W), y = rr / W, x = rr - (rr / W) * W;
          const int gy = y - (6 - k) + pi, gx = x - (6 - k) + pj;
          const bool in = gy >= 0 && gy < H && gx >= 0 && gx < W;
          float v[2][4];
#pragma unroll
          for (int m = 0; m < 2; ++m)
#pragma unroll
            for (int i = 0; i < 4; ++i) v[m][i] = in ? fmaxf(acc[m][i] + bk[m][i], 0.f) : 0.f;
          if (k == 5) {  // keep layer 5 in FP32 for the head
#pragma unroll
            for (int m = 0; m < 2; ++m)
#pragma unroll
              for (int i = 0; i < 4; ++i) l5f[cidx][pos * 32 + 16 * m + 4 * g + i] = v[m][i];
          } else {
            bf16x8_t vh, vl;
#pragma unroll
            for (int m = 0; m < 2; ++m)
#pragma unroll
              for (int i = 0; i < 4; ++i) {
                const __bf16 h = (__bf16)v[m][i];
                vh[4 * m + i] = h;
                vl[4 * m + i] = (__bf16)(v[m][i] - (float)h);
              }
            char* rec = dst + pos * CREC;
            *(bf16x8_t*)(rec + crec_slot(pos, 2 * g) * 16) = vh;
            *(bf16x8_t*)(rec + crec_slot(pos, 2 * g + 1) * 16) = vl;
          }
        }
      }
    }
    __syncthreads();
    // layer 6 in FP32, one wave per cone
    if (wave < ncone) {
      float part = 0.f;
      for (int i = lane; i < 288; i += 64) {
        const int ci = i / 9, t = i % 9;
        part = fmaf(w[HS_W6 + i], l5f[wave][t * 32 + ci], part);
      }
      part = hs_wave_sum(part);
      if (lane == 0) {
        const uint32_t o = list[base + wave];
        const float xl = part + w[HS_B6];
        if (fabsf(xl) >= tau2) {
          const uint8_t nb = xl >= 0.f ? 1 : 0;
          if (bits[o] != nb) atomicAdd(&stats[1], 1);
          bits[o] = nb;
          if (logits) logits[o] = xl;
        } else {
          list2[atomicAdd(count2, 1)] = o;
        }
      }
    }
  }
  if (blockIdx.x == 0 && tid == 0) stats[0] = n;
}

}  // namespace

namespace hs {

// bytes of the hi and the lo copy together (each 4 layers x 9 taps x 2 row
// tiles x 64 lanes x 8 BF16 values)
size_t split_frag_bytes() { return 2 * (size_t)(4 * 9 * 2 * 64 * 8) * sizeof(__bf16); }

hipError_t launch_split_pack(const float* w, void* whi, void* wlo, hipStream_t s) {
  pack_split_kernel<<<36, 256, 0, s>>>(w, (__bf16*)whi, (__bf16*)wlo);
  return hipGetLastError();
}

hipError_t launch_recheck_split(const float* w, const float* contone, const uint64_t* seeds,
                                int H, int W, int kind, const uint32_t* list, const int* count,
                                const void* whi, const void* wlo, float tau2, uint32_t* list2,
                                int* count2, uint8_t* bits, float* logits, int32_t* stats,
                                int num_cus, hipStream_t s) {
  recheck_split_kernel<<<num_cus, 256, 0, s>>>(w, contone, seeds, H, W, kind, list, count,
                                               (const bf16x8_t*)whi, (const bf16x8_t*)wlo, tau2,
                                               list2, count2, bits, logits, stats);
  return hipGetLastError();
}

}  // namespace hs
