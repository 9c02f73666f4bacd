// spectrum.hip -- the blue-noise measures of Sec. IV (Eqs. psd, rapsd, anis)
// on halftones: the power spectrum estimated as the mean periodogram of the
// non-overlapping P x P patches of a batch of bit maps, reduced to the
// radially averaged power (RAPSD) and the anisotropy per ring.
//
// Three launches, all with a fixed summation order:
//   spectrum_patch_kernel  one workgroup per patch: separable direct DFT in
//                          LDS (rows, then columns), periodogram |X|^2 / P^2
//                          written to the patch's row of the workspace;
//   spectrum_mean_kernel   per frequency, the mean over patches in order;
//   spectrum_rings_kernel  per ring, mean and variance over its frequencies.
#include "hs_common.h"
#include "hs_internal.h"

namespace {

// Ring of frequency (u, v) of a P x P spectrum: the unique rho with
// (2 rho - 1)^2 <= 4 (ub^2 + vb^2) < (2 rho + 1)^2 (the folded radius
// rounded half up), ub = min(u, P - u), vb = min(v, P - v).
HS_DEV int ring_index(int u, int v, int P) {
  const int ub = u < P - u ? u : P - u, vb = v < P - v ? v : P - v;
  const int q4 = 4 * (ub * ub + vb * vb);
  int rho = (int)sqrtf((float)(ub * ub + vb * vb));
  while ((2 * rho + 1) * (2 * rho + 1) <= q4) ++rho;
  while (rho > 0 && (2 * rho - 1) * (2 * rho - 1) > q4) --rho;
  return rho;
}

template <int P>
__global__ __launch_bounds__(256) void spectrum_patch_kernel(const uint8_t* __restrict__ bits,
                                                             int H, int W,
                                                             float* __restrict__ spec) {
  constexpr int LD = P + 1;
  __shared__ float x[P * LD], rr[P * LD], ri[P * LD];
  __shared__ float cs[P], sn[P];
  const int py = H / P, px = W / P;
  const int patch = blockIdx.x;
  const int b = patch / (py * px), rem = patch - b * py * px;
  const int oy = (rem / px) * P, ox = (rem % px) * P;
  const uint8_t* base = bits + (size_t)b * H * W + (size_t)oy * W + ox;
  const int t = threadIdx.x;
  for (int k = t; k < P; k += 256) {
    float sv, cv;
    sincospif(2.0f * (float)k / (float)P, &sv, &cv);  // angle 2 pi k / P
    cs[k] = cv;
    sn[k] = sv;
  }
  for (int i = t; i < P * P; i += 256) x[(i / P) * LD + i % P] = (float)base[(size_t)(i / P) * W + i % P];
  __syncthreads();
  // along x: (rr + i ri)[y][v] = sum_x x[y][x] e^{-2 pi i v x / P}
  for (int i = t; i < P * P; i += 256) {
    const int y = i / P, v = i % P;
    float sr = 0.f, si = 0.f;
    for (int xx = 0; xx < P; ++xx) {
      const int k = (v * xx) % P;
      const float val = x[y * LD + xx];
      sr = fmaf(val, cs[k], sr);
      si = fmaf(-val, sn[k], si);
    }
    rr[y * LD + v] = sr;
    ri[y * LD + v] = si;
  }
  __syncthreads();
  // along y, then |X|^2 / P^2
  float* out = spec + (size_t)patch * P * P;
  for (int i = t; i < P * P; i += 256) {
    const int u = i / P, v = i % P;
    float sr = 0.f, si = 0.f;
    for (int y = 0; y < P; ++y) {
      const int k = (u * y) % P;
      const float a = rr[y * LD + v], bb = ri[y * LD + v];
      sr = fmaf(a, cs[k], fmaf(bb, sn[k], sr));
      si = fmaf(bb, cs[k], fmaf(-a, sn[k], si));
    }
    out[i] = (sr * sr + si * si) * (1.0f / (float)(P * P));
  }
}

__global__ void spectrum_mean_kernel(const float* __restrict__ spec, int npatch, int n,
                                     float* __restrict__ avg) {
  const int f = blockIdx.x * blockDim.x + threadIdx.x;
  if (f >= n) return;
  float s = 0.f;
  for (int p = 0; p < npatch; ++p) s += spec[(size_t)p * n + f];
  avg[f] = s / (float)npatch;
}

// one workgroup; thread rho handles ring rho (two passes over the spectrum)
__global__ __launch_bounds__(256) void spectrum_rings_kernel(const float* __restrict__ avg, int P,
                                                             int nrings, float* __restrict__ rapsd,
                                                             float* __restrict__ anis) {
  const int rho = threadIdx.x;
  if (rho >= nrings) return;
  float s = 0.f;
  int n = 0;
  for (int i = 0; i < P * P; ++i)
    if (ring_index(i / P, i % P, P) == rho) {
      s += avg[i];
      ++n;
    }
  const float mean = s / (float)n;
  float a = 0.f;
  for (int i = 0; i < P * P; ++i)
    if (ring_index(i / P, i % P, P) == rho) {
      const float d = avg[i] - mean;
      a = fmaf(d, d, a);
    }
  rapsd[rho] = mean;
  anis[rho] = (n > 1 && mean != 0.f) ? a / ((float)(n - 1) * mean * mean) : 0.f;
}

}  // namespace

namespace hs {

int spectrum_rings(int P) {
  const int h = P / 2, q4 = 4 * (h * h + h * h);
  int rho = 0;
  while ((2 * rho + 1) * (2 * rho + 1) <= q4) ++rho;
  return rho + 1;
}

size_t spectrum_patches(int B, int H, int W, int P) { return (size_t)B * (H / P) * (W / P); }

hipError_t launch_spectrum(const uint8_t* bits, int B, int H, int W, int P, float* spec,
                           float* avg, float* rapsd, float* anis, hipStream_t s) {
  const size_t np = spectrum_patches(B, H, W, P);
  if (P == 32)
    spectrum_patch_kernel<32><<<(unsigned)np, 256, 0, s>>>(bits, H, W, spec);
  else
    spectrum_patch_kernel<64><<<(unsigned)np, 256, 0, s>>>(bits, H, W, spec);
  spectrum_mean_kernel<<<(P * P + 255) / 256, 256, 0, s>>>(spec, (int)np, P * P, avg);
  spectrum_rings_kernel<<<1, 256, 0, s>>>(avg, P, spectrum_rings(P), rapsd, anis);
  return hipGetLastError();
}

}  // namespace hs
