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
    int32_t* __restrict__ stats) {
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
  if (blockIdx.x == 0 && tid == 0) stats[0] = n;
}

}  // namespace

namespace hs {

hipError_t launch_zero_ints(int* p, int n, hipStream_t s) {
  zero_ints_kernel<<<(n + 255) / 256, 256, 0, s>>>(p, n);
  return hipGetLastError();
}

hipError_t launch_recheck_fp32(const float* w, const float* contone, const uint64_t* seeds,
                               int H, int W, int kind, const uint32_t* list, const int* count,
                               uint8_t* bits, float* logits, int32_t* stats, hipStream_t s) {
  recheck_fp32_kernel<<<1024, 256, 0, s>>>(w, contone, seeds, H, W, kind, list, count, bits,
                                           logits, stats);
  return hipGetLastError();
}

}  // namespace hs
