// train.hip -- optimiser step and training metrics on gfx950.
//
// Adam (Kingma and Ba) on the FP32 master weights, as used in Sec. VI-A of
// the paper; the host supplies the cosine-annealed learning rate and the
// bias-correction factors of the step.
#include "hs_common.h"
#include "hs_internal.h"

namespace {

// The train step's last reduction level fused with Adam: parameter p's
// gradient is the sum of the group sums tmp0[0..G) and then, if tmp1 is
// given (the side batch's), tmp1[0..G), in that order; it goes to grad[p],
// the block's sum of grad^2 to gsq[blockIdx.x] (waves in order), and Adam
// updates w, m, v at p with it.
__global__ __launch_bounds__(256) void reduce_groups_adam_kernel(
    const float* __restrict__ tmp0, const float* __restrict__ tmp1, float* __restrict__ grad,
    float* __restrict__ gsq, float* __restrict__ w, float* __restrict__ m, float* __restrict__ v,
    float lr, float b1, float b2, float eps, float inv_c1, float inv_c2) {
  __shared__ float part[4];
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  float s = 0.0f;
  if (p < hs::NPARAM) {
    for (int gi = 0; gi < hs::REDUCE_GROUPS; ++gi) s += tmp0[(size_t)gi * hs::NPARAM + p];
    if (tmp1)
      for (int gi = 0; gi < hs::REDUCE_GROUPS; ++gi) s += tmp1[(size_t)gi * hs::NPARAM + p];
    grad[p] = s;
    const float mi = b1 * m[p] + (1.0f - b1) * s;
    const float vi = b2 * v[p] + (1.0f - b2) * s * s;
    m[p] = mi;
    v[p] = vi;
    const float mh = mi * inv_c1, vh = vi * inv_c2;
    w[p] -= lr * mh / (sqrtf(vh) + eps);
  }
  float q = s * s;
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) q += __shfl_xor(q, o, 64);
  if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = q;
  __syncthreads();
  if (threadIdx.x == 0) gsq[blockIdx.x] = ((part[0] + part[1]) + part[2]) + part[3];
}

// Sum of the action bytes (bits, or level indices below 64). Each block sums
// a slice with 16-byte loads (the byte sum of a 32-bit word v of such bytes
// is (v * 0x01010101) >> 24: no partial sum reaches 256) and adds it to a
// 64-bit counter; integer sums are order-independent.
__global__ __launch_bounds__(256) void count_ones_kernel(const uint8_t* __restrict__ act,
                                                         size_t nact,
                                                         unsigned long long* __restrict__ out) {
  __shared__ unsigned long long part[4];
  unsigned long long c = 0;
  const size_t nvec = nact / 16;
  const uint4* av = (const uint4*)act;
  for (size_t i = blockIdx.x * (size_t)256 + threadIdx.x; i < nvec; i += (size_t)gridDim.x * 256) {
    const uint4 v = av[i];
    c += ((v.x * 0x01010101u) >> 24) + ((v.y * 0x01010101u) >> 24) +
         ((v.z * 0x01010101u) >> 24) + ((v.w * 0x01010101u) >> 24);
  }
  if (blockIdx.x == 0)
    for (size_t i = nvec * 16 + threadIdx.x; i < nact; i += 256) c += act[i];
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) c += __shfl_xor(c, o, 64);
  if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = c;
  __syncthreads();
  if (threadIdx.x == 0) atomicAdd(out, part[0] + part[1] + part[2] + part[3]);
}

// metrics = {mean MSE, mean CSSIM, mean R, L_AS, lr, |grad|_2, fill, 0}; fill
// is the mean of h = action / (levels - 1)
// one workgroup of 1024 threads: the gradient norm is a single pass of 37
// loads per thread, summed per wave and then over the 16 waves in order
__global__ __launch_bounds__(256) void metrics_kernel(const float* __restrict__ loss_out, int B,
                                                     const float* __restrict__ gsq,
                                                     const unsigned long long* __restrict__ ones,
                                                     size_t nact, int levels, float lr,
                                                     float w_a, float* __restrict__ metrics) {
  __shared__ float red[4];
  float s = threadIdx.x < hs::REDUCE_BLOCKS ? gsq[threadIdx.x] : 0.0f;
  s = hs_wave_sum(s);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x != 0) return;
  float mse = 0.f, cs = 0.f, r = 0.f;
  for (int b = 0; b < B; ++b) {
    mse += loss_out[3 * b];
    cs += loss_out[3 * b + 1];
    r += loss_out[3 * b + 2];
  }
  metrics[0] = mse / B;
  metrics[1] = cs / B;
  metrics[2] = r / B;
  metrics[3] = loss_out[3 * B];
  metrics[4] = lr;
  float g2 = 0.0f;
  for (int k = 0; k < 4; ++k) g2 += red[k];
  metrics[5] = sqrtf(g2);
  metrics[6] = (float)((double)*ones / ((double)nact * (levels - 1)));
  metrics[7] = -metrics[2] + w_a * metrics[3];
}

__global__ void zero_u64_kernel(unsigned long long* p) { *p = 0ull; }

}  // namespace

namespace hs {

hipError_t launch_reduce_adam(const float* tmp0, const float* tmp1, float* grad, float* gsq,
                              float* w, float* m, float* v, float lr, float b1, float b2,
                              float eps, float c1, float c2, hipStream_t s) {
  reduce_groups_adam_kernel<<<REDUCE_BLOCKS, 256, 0, s>>>(tmp0, tmp1, grad, gsq, w, m, v, lr, b1,
                                                          b2, eps, 1.0f / c1, 1.0f / c2);
  return hipGetLastError();
}

hipError_t launch_count_actions(const uint8_t* actions, size_t nact,
                                unsigned long long* counter, hipStream_t s) {
  zero_u64_kernel<<<1, 1, 0, s>>>(counter);
  size_t blocks = (nact / 16 + 255) / 256;
  if (blocks < 1) blocks = 1;
  if (blocks > 1024) blocks = 1024;
  count_ones_kernel<<<(unsigned)blocks, 256, 0, s>>>(actions, nact, counter);
  return hipGetLastError();
}

hipError_t launch_train_metrics(const float* loss_out, int B, const float* gsq,
                                const unsigned long long* counter, size_t nact, int levels,
                                float lr, float w_a, float* metrics, hipStream_t s) {
  static_assert(REDUCE_BLOCKS <= 256, "one block sums the partial sums of grad^2");
  metrics_kernel<<<1, 256, 0, s>>>(loss_out, B, gsq, counter, nact, levels, lr, w_a, metrics);
  return hipGetLastError();
}

}  // namespace hs
