// hs_common.h -- device-side building blocks of libhalftone (gfx950).
//
// Counter-based random numbers, fragment types for the CDNA4 matrix cores,
// and small helpers shared by the kernels of this library.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#define HS_DEV __device__ __forceinline__

typedef __attribute__((__vector_size__(8 * sizeof(__bf16)))) __bf16 bf16x8_t;
typedef __attribute__((__vector_size__(4 * sizeof(__bf16)))) __bf16 bf16x4_t;
typedef __attribute__((__vector_size__(4 * sizeof(float)))) float f32x4_t;
typedef __attribute__((__vector_size__(2 * sizeof(float)))) float f32x2_t;
typedef __attribute__((__vector_size__(2 * sizeof(__bf16)))) __bf16 bf16x2_t;
typedef __attribute__((__vector_size__(2 * sizeof(short)))) short i16x2_t;
typedef __attribute__((__vector_size__(2 * sizeof(unsigned short)))) unsigned short u16x2_t;
typedef __attribute__((__vector_size__(8 * sizeof(_Float16)))) _Float16 f16x8_t;
typedef __attribute__((__vector_size__(2 * sizeof(_Float16)))) _Float16 f16x2_t;
typedef __attribute__((__vector_size__(16 * sizeof(float)))) float f32x16_t;
typedef __attribute__((__vector_size__(8 * sizeof(int)))) int i32x8_t;

// ---------------------------------------------------------------------------
// Philox4x32-10 (Salmon et al., SC'11): ten rounds of a multiply-and-swap
// bijection on four 32-bit words keyed by two words, the key advanced by the
// Weyl constants between rounds. Integer-only, so every implementation of
// the published definition gives the same bits.
// ---------------------------------------------------------------------------
// WIDE takes each 32 x 32 -> 64-bit product in one multiply
// (v_mad_u64_u32) instead of separate low and high halves: fewer
// quarter-rate instructions, but one more 64-bit temporary, so kernels at
// the edge of their register budget use the narrow form. Both give the same
// bits.
template <bool WIDE = false>
HS_DEV uint4 hs_philox(uint4 c, uint32_t k0, uint32_t k1) {
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    if (r) {
      k0 += 0x9E3779B9u;
      k1 += 0xBB67AE85u;
    }
    uint32_t lo0, hi0, lo1, hi1;
    if constexpr (WIDE) {
      const uint64_t p0 = (uint64_t)0xD2511F53u * c.x, p1 = (uint64_t)0xCD9E8D57u * c.z;
      lo0 = (uint32_t)p0;
      hi0 = (uint32_t)(p0 >> 32);
      lo1 = (uint32_t)p1;
      hi1 = (uint32_t)(p1 >> 32);
    } else {
      lo0 = 0xD2511F53u * c.x;
      hi0 = __umulhi(0xD2511F53u, c.x);
      lo1 = 0xCD9E8D57u * c.z;
      hi1 = __umulhi(0xCD9E8D57u, c.z);
    }
    c = make_uint4(hi1 ^ c.y ^ k0, lo1, hi0 ^ c.w ^ k1, lo0);
  }
  return c;
}

template <bool WIDE = false>
HS_DEV uint4 hs_draw(uint64_t seed, uint64_t a, uint32_t stream, uint32_t step) {
  return hs_philox<WIDE>(make_uint4((uint32_t)a, (uint32_t)(a >> 32), stream, step),
                         (uint32_t)seed, (uint32_t)(seed >> 32));
}

// u in [0,1) with 24 random bits (exact in FP32).
HS_DEV float hs_u24(uint32_t w) { return (float)(w >> 8) * (1.0f / 16777216.0f); }

// Noise map value of pixel a (stream 1): Gaussian by Box-Muller on words 0
// and 1 (u1 in (0,1], so the log is finite), or the uniform variant.
template <bool WIDE = false>
HS_DEV float hs_noise(uint64_t seed, uint64_t a, uint32_t step, int kind) {
  const uint4 w = hs_draw<WIDE>(seed, a, 1u, step);
  if (kind == 1) return hs_u24(w.x);
  const float u1 = (float)((w.x >> 8) + 1u) * (1.0f / 16777216.0f);
  const float u2 = hs_u24(w.y);
  return sqrtf(-2.0f * logf(u1)) * cospif(2.0f * u2);
}

// Action draw of pixel a (stream 0): h = [u < p].
HS_DEV float hs_action_u(uint64_t seed, uint64_t a, uint32_t step) {
  return hs_u24(hs_draw<true>(seed, a, 0u, step).x);
}

// ---------------------------------------------------------------------------
// Activation element types. Activations are NHWC with 32 channels. A "chunk"
// is 16 bytes; one MFMA operand fragment per lane is 8 channels (one chunk
// in BF16, two in FP32).
// ---------------------------------------------------------------------------
template <typename T> struct act_traits;
template <> struct act_traits<__bf16> {
  static constexpr int chunks_per_px = 4;  // 64 B per pixel
  static constexpr int elems_per_chunk = 8;
};
template <> struct act_traits<float> {
  static constexpr int chunks_per_px = 8;  // 128 B per pixel
  static constexpr int elems_per_chunk = 4;
};

// LDS chunk swizzle: the lanes of one operand read the same chunk of
// consecutive pixels; XOR-ing the chunk slot with the pixel's column bits
// spreads those reads over all banks.
template <typename T> HS_DEV int hs_swz(int col, int chunk);
template <> HS_DEV int hs_swz<__bf16>(int col, int chunk) { return chunk ^ ((col >> 1) & 3); }
template <> HS_DEV int hs_swz<float>(int col, int chunk) { return chunk ^ (col & 7); }

HS_DEV float hs_to_f(float v) { return v; }
HS_DEV float hs_to_f(__bf16 v) { return (float)v; }
template <typename T> HS_DEV T hs_from_f(float v);
template <> HS_DEV float hs_from_f<float>(float v) { return v; }
template <> HS_DEV __bf16 hs_from_f<__bf16>(float v) { return (__bf16)v; }

// 8-channel operand fragment of one lane.
template <typename T> struct frag8;
template <> struct frag8<__bf16> {
  bf16x8_t v;
};
template <> struct frag8<float> {
  f32x4_t lo, hi;
};

HS_DEV void hs_load_frag(frag8<__bf16>& f, const __bf16* p) { f.v = *(const bf16x8_t*)p; }
HS_DEV void hs_load_frag(frag8<float>& f, const float* p) {
  f.lo = *(const f32x4_t*)p;
  f.hi = *(const f32x4_t*)(p + 4);
}

// acc[16x16] += A[16 x 32-slice] * B[32-slice x 16] where lane l holds row
// (l % 16) of A and column (l % 16) of B over the same 8 k-values.
HS_DEV f32x4_t hs_mma(const frag8<__bf16>& a, const frag8<__bf16>& b, f32x4_t acc) {
  return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a.v, b.v, acc, 0, 0, 0);
}
HS_DEV f32x4_t hs_mma(const frag8<float>& a, const frag8<float>& b, f32x4_t acc) {
  acc = __builtin_amdgcn_mfma_f32_16x16x4f32(a.lo[0], b.lo[0], acc, 0, 0, 0);
  acc = __builtin_amdgcn_mfma_f32_16x16x4f32(a.lo[1], b.lo[1], acc, 0, 0, 0);
  acc = __builtin_amdgcn_mfma_f32_16x16x4f32(a.lo[2], b.lo[2], acc, 0, 0, 0);
  acc = __builtin_amdgcn_mfma_f32_16x16x4f32(a.lo[3], b.lo[3], acc, 0, 0, 0);
  acc = __builtin_amdgcn_mfma_f32_16x16x4f32(a.hi[0], b.hi[0], acc, 0, 0, 0);
  acc = __builtin_amdgcn_mfma_f32_16x16x4f32(a.hi[1], b.hi[1], acc, 0, 0, 0);
  acc = __builtin_amdgcn_mfma_f32_16x16x4f32(a.hi[2], b.hi[2], acc, 0, 0, 0);
  acc = __builtin_amdgcn_mfma_f32_16x16x4f32(a.hi[3], b.hi[3], acc, 0, 0, 0);
  return acc;
}

// Store 4 consecutive channels.
HS_DEV void hs_store4(float* p, float a, float b, float c, float d) {
  *(f32x4_t*)p = f32x4_t{a, b, c, d};
}
HS_DEV void hs_store4(__bf16* p, float a, float b, float c, float d) {
  *(bf16x4_t*)p = bf16x4_t{(__bf16)a, (__bf16)b, (__bf16)c, (__bf16)d};
}

HS_DEV float hs_sigmoid(float x) { return 1.0f / (1.0f + expf(-x)); }

// Channel order of the matrix-core convolutions: the 16x16 MFMA result of
// lane (g, r) holds channels 4g..4g+3 of both 16-channel row tiles for
// pixel r; those eight channels, stored as the lane's 16-byte chunk, are the
// next layer's K-slice for lane group g. Slot e of that chunk holds channel
// hs_ring_channel(g, e), and the next layer's weights are packed to match.
HS_DEV int hs_ring_channel(int g, int e) { return e < 4 ? 4 * g + e : 16 + 4 * g + (e - 4); }

// Workgroup barrier that orders LDS accesses only: unlike __syncthreads()
// it does not wait for the wave's outstanding global loads and stores, so a
// load issued for a later step stays in flight across it. Only for kernels
// whose waves do not communicate through global memory within a launch.
HS_DEV void hs_lds_barrier() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
  __builtin_amdgcn_s_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

// Wave-wide sum (64 lanes) with a fixed reduction order.
HS_DEV float hs_wave_sum(float v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}
