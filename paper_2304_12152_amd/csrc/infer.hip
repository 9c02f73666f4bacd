// infer.hip -- the TEST procedure of Algorithm 1 on gfx950: the fused BF16
// (or FP16) pass of the policy network over whole images, with each pixel's
// logit thresholded at 0 (p = 0.5) and the near-threshold pixels listed for
// the recheck stages (recheck.hip). FP16 has 11 significant bits to BF16's 8
// at the same matrix-core rate, so its logit error and recheck band are about
// 8 times smaller; its range ends at 65504, so the FP16 pass tests the
// activations it stores (only layer 5's and the contone range when a priori
// bounds clear layers 1..4) and records an overflow, and a BF16 launch that
// does nothing otherwise then redoes the pass.
#include "hs_common.h"
#include "hs_internal.h"

namespace {

__global__ void zero_ints_kernel(int* p, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = 0;
}

// *count (zeroed before) += number of NaN / infinite values in x[0, n):
// exponent bits all ones. One atomic per wave that found any.
__global__ void count_nonfinite_kernel(const float* __restrict__ x, size_t n, int* count) {
  int bad = 0;
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (size_t)gridDim.x * blockDim.x)
    bad += ((__float_as_uint(x[i]) & 0x7F800000u) == 0x7F800000u) ? 1 : 0;
  for (int o = 32; o > 0; o >>= 1) bad += __shfl_xor(bad, o);
  if ((threadIdx.x & 63) == 0 && bad) atomicAdd(count, bad);
}

}  // namespace

namespace hs {

hipError_t launch_zero_ints(int* p, int n, hipStream_t s) {
  zero_ints_kernel<<<(n + 255) / 256, 256, 0, s>>>(p, n);
  return hipGetLastError();
}

hipError_t launch_count_nonfinite(const float* x, size_t n, int* count, hipStream_t s) {
  if (n == 0) return hipSuccess;
  size_t blocks = (n + 255) / 256;
  if (blocks > 2048) blocks = 2048;
  count_nonfinite_kernel<<<(unsigned)blocks, 256, 0, s>>>(x, n, count);
  return hipGetLastError();
}

}  // namespace hs

// ===========================================================================
// Fused BF16 inference: one persistent kernel runs all six layers of the
// policy over vertical strips of the image, streaming down the rows.
//
// A strip is FW = 128 computed columns, of which the central FS = 116 are
// valid outputs (the 13 x 13 receptive field eats 6 columns on each side).
// Each step advances every stage by one row, with a single barrier per step:
//   input stage   contone + Philox noise of one row -> input ring (4 slots)
//   layer 1       three input rows -> one output row (MFMA, K = 9 taps x 2)
//   layers 2..5   ONE new input row per step: its three tap rows dy = 0, 1, 2
//                 feed three accumulator sets (output rows q+1, q, q-1), so
//                 each set sees its three input rows on consecutive steps and
//                 every input row is read from LDS once. The set finished in
//                 a step is stored in the next one, so the store never waits
//                 on the MFMA pipeline.
//   layer 6       layer 5's finished row goes straight from registers into
//                 one MFMA giving, per pixel, the nine taps' 32-channel dot
//                 products T; the output stage slides the same way over T
//                 rows, adds the bias, thresholds and flags near-ties.
// A row is written into a slot that no stage reads in the same step, and
// read in the next step, so the rings of layers 1..4 and T hold two rows.
//
// Work per step: eight waves; conv layer k (2..5) belongs to waves
// 2(k-2), 2(k-2)+1, each owning four 16-pixel runs of the row and holding
// its layer's weights in registers for the whole kernel. Besides that,
// waves 0-1 run layer 1, waves 2-3 the input stage, waves 4-5 the output
// stage and waves 6-7 (layer 5) the layer-6 taps.
//
// Channel order in the rings: the MFMA result of lane (g, r) holds output
// channels {4g..4g+3, 16+4g..16+4g+3} of pixel r; those eight channels are
// stored as the lane's 16-byte chunk and read back as the same lane group's
// K-slice by the next layer, whose weights are packed in that order. A ring
// row is [column][chunk][16 B] with the chunk index XOR-ed by bits 1..2 of
// the column, which makes the 16-byte reads and writes of a wave free of LDS
// bank conflicts; runs of 16 columns are immediate offsets from one base.
// ===========================================================================
namespace {

constexpr int FW = 128, FS = FW - 12, RWID = FW + 2;
constexpr int LAG_OUT = 22;  // steps from the first input row Y0-6 to output row Y0
// A strip segment costs its rows plus about FILL steps of pipeline fill, so
// the workgroups split a sequence in which every strip is preceded by FILL
// virtual rows into equal parts: each workgroup then runs about the same
// number of steps, whether or not its rows cross a strip boundary.
constexpr int FILL = LAG_OUT + 2;
constexpr int FRAG_L1 = 0, FRAG_L32 = 128, FRAG_T = 128 + 4 * 9 * 2 * 64;
constexpr int FRAG_TOTAL = FRAG_T + 64;
constexpr int FUSED_NW = 2;  // waves per conv layer in the fused kernel
constexpr int ROWE = RWID * 32;         // elements per ring row
constexpr int RUNE = 16 * 32;           // elements per 16-column run

// element offset of chunk g of column col in a ring row
HS_DEV int ring_off(int col, int g) { return (col * 4 + (g ^ ((col >> 1) & 3))) * 8; }

HS_DEV int ring_channel(int g, int e) { return hs_ring_channel(g, e); }

// ---- the FP8 form: layers 2..5 on the 16x16x128 FP8 (E4M3) matrix-core
// instruction, whose K of 128 takes the three taps dx of one kernel row
// (32 channels each; the fourth K slice meets zero weights). Layers 1..4
// store their activations as E4M3 codes q = a / s_k with a per-layer power
// of two s_k; the weights of layers 2..5 are codes W / sw with a power of
// two sw per output channel, and the instruction's per-row E8M0 scale
// applies sw * s_(k-1) / s_k, so the accumulator holds q_k (a_5 for layer
// 5, which feeds the BF16 layer-6 taps). Layer 1 stays BF16 (weights and
// bias divided by s_1).
//
// An FP8 ring row is RWID 32-byte records, a record being the column's 32
// channels in ring order (8-byte piece q = the producing lane group); the
// two 16-byte halves are swapped in columns with bit 3 set, so that the
// 8-byte stores of a 32-lane half-wave (16 columns) and the 16-byte loads
// of 8 consecutive columns fall in distinct LDS banks.
constexpr int ROWB8 = RWID * 32;  // bytes per FP8 ring row
constexpr int RUNB8 = 16 * 32;    // bytes per 16-column run
HS_DEV int ring8_off(int col, int q) {
  return col * 32 + ((((q >> 1) ^ (col >> 3)) & 1) << 4) + ((q & 1) << 3);
}
HS_DEV int ring8_half(int col, int h) { return col * 32 + (((h ^ (col >> 3)) & 1) << 4); }
// the largest finite E4M3 value; the conversion gives NaN above 464
constexpr float FP8_MAX = 448.0f;
// the FP8 block of a packed policy (byte offsets)
constexpr int F8_L32 = 0;                      // layers 2..5: [layer][dy][m][lane] x 32 B
constexpr int F8_L1 = 4 * 3 * 2 * 64 * 32;     // layer 1, BF16: [m][lane] x 16 B
constexpr int F8_SCALE = F8_L1 + 2 * 64 * 16;  // int32 [layer][lane]: byte m = row 16m + lane%16
constexpr int F8_BIAS = F8_SCALE + 4 * 64 * 4;  // float [5][32]: b_k / s_k (s_5 = 1)
constexpr int F8_TOTAL = F8_BIAS + 5 * 32 * 4;

template <int M>  // M: the byte of the scale word that holds this m-tile's row scale
HS_DEV f32x4_t mma8(const i32x8_t& a, const i32x8_t& b, f32x4_t c, int sc) {
  return __builtin_amdgcn_mfma_scale_f32_16x16x128_f8f6f4(a, b, c, 0, 0, M, sc, 0, 127);
}

// ReLU, saturation test and E4M3 conversion (round to nearest even) of one
// finished 16-pixel run: the lane's eight channels, ring order, as 8 bytes,
// zero where the pixel is padding. amax keeps the largest value before the
// clamp; one above 448 means the pass saturated.
HS_DEV uint2 relu_pack8(const f32x4_t (&acc)[2], bool in, float& amax) {
  float v[8];
#pragma unroll
  for (int m = 0; m < 2; ++m)
#pragma unroll
    for (int i = 0; i < 4; ++i) v[4 * m + i] = acc[m][i];
#pragma unroll
  for (int j = 0; j < 4; ++j) amax = fmaxf(amax, fmaxf(v[2 * j], v[2 * j + 1]));
#pragma unroll
  for (int j = 0; j < 8; ++j) v[j] = __builtin_amdgcn_fmed3f(v[j], 0.0f, FP8_MAX);
  uint32_t lo = (uint32_t)__builtin_amdgcn_cvt_pk_fp8_f32(v[0], v[1], 0, false);
  lo = (uint32_t)__builtin_amdgcn_cvt_pk_fp8_f32(v[2], v[3], (int)lo, true);
  uint32_t hi = (uint32_t)__builtin_amdgcn_cvt_pk_fp8_f32(v[4], v[5], 0, false);
  hi = (uint32_t)__builtin_amdgcn_cvt_pk_fp8_f32(v[6], v[7], (int)hi, true);
  const uint32_t keep = 0u - (uint32_t)in;
  return make_uint2(lo & keep, hi & keep);
}

// Activation bound below which FP16 carries a layer safely: the FP16 pass
// rounds weights and activations (relative 2^-11 each, at most ten roundings
// up to layer 5) and accumulates in FP32, all within 1% of the bound; 65504
// is FP16's largest finite value.
constexpr float FP16_SAFE = 60000.0f;
// The Gaussian noise takes u1 >= 2^-24 in the Box-Muller transform, so
// |z| <= sqrt(48 ln 2) = 5.77; the uniform noise lies in [0, 1).
constexpr float NOISE_MAX = 5.8f;

// Page of a uniform batch: image b of B images of H x W.
HS_DEV hs::Page uniform_page(int b, int H, int W) {
  const int nstrip = (W + FS - 1) / FS;
  hs::Page p;
  p.off = (long long)b * H * W;
  p.vstart = (long long)b * nstrip * (H + FILL);
  p.H = H;
  p.W = W;
  p.nstrip = nstrip;
  p.pad = 0;
  return p;
}

// The call's other set-up in the same launch: counters to clear and, for a
// uniform batch, the page table (one kernel instead of three).
// out: BF16 fragments; out16 (may be null): the same fragments in FP16, and
// then *needs_all = 1 unless a priori bounds keep layers 1..4 inside FP16's
// range. With contones in [0, 1] (which the FP16 pass verifies) every
// layer's inputs are non-negative after the ReLU, so output channel co is at
// most the sum over its inputs of max(w, 0) times the input's bound, plus the
// bias (layer 1 takes |w| for the noise channel).
__global__ void pack_fused_kernel(const float* __restrict__ w, __bf16* __restrict__ out,
                                  _Float16* __restrict__ out16, int* __restrict__ needs_all,
                                  const hs::PackPrologue pro) {
  const int gid = blockIdx.x * blockDim.x + threadIdx.x;
  if (gid < pro.n0) pro.zero0[gid] = 0;
  if (gid < pro.n1) pro.zero1[gid] = 0;
  if (pro.pages)
    for (int b = gid; b < pro.B; b += gridDim.x * blockDim.x) pro.pages[b] = uniform_page(b, pro.H, pro.W);
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < FRAG_TOTAL * 8;
       i += gridDim.x * blockDim.x) {
    const int f = i >> 3, e = i & 7;
    float v = 0.0f;
    if (f < FRAG_L32) {  // layer 1: lane group g = kernel row dy, slot e = (dx = e/2, channel e%2)
      const int m = f >> 6, l = f & 63, g = l >> 4, r = l & 15;
      const int co = 16 * m + r;
      if (g < 3 && e < 6) v = w[HS_W1 + (co * 2 + (e & 1)) * 9 + g * 3 + (e >> 1)];
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
    if (out16) out16[i] = (_Float16)v;
  }
  if (!out16 || blockIdx.x != 0) return;  // block-uniform: the barriers below are safe
  // thread t: output channel co = t / 8, input channels ci = 4 (t % 8) .. +3
  __shared__ float bound[32], part[256];
  const int t = threadIdx.x, co = t >> 3, q = t & 7;
  bool over = false;
  for (int k = 1; k <= 4; ++k) {
    const int cin = k == 1 ? 2 : 32;
    const float* wk = w + (k == 1 ? HS_W1 : hs_wk(k));
    float sum = 0.0f;
    for (int ci = 4 * q; ci < 4 * q + 4 && ci < cin; ++ci) {
      float sp = 0.0f;  // over the taps
      for (int tp = 0; tp < 9; ++tp) {
        const float wv = wk[(co * cin + ci) * 9 + tp];
        sp += (k == 1 && ci == 1) ? fabsf(wv) : fmaxf(wv, 0.0f);
      }
      sum += sp * (k == 1 ? (ci == 0 ? 1.0f : NOISE_MAX) : bound[ci]);
    }
    part[t] = sum;
    __syncthreads();
    if (t < 32) {
      float b = w[(k == 1 ? HS_B1 : hs_bk(k)) + t];
      for (int j = 0; j < 8; ++j) b += part[8 * t + j];
      bound[t] = fmaxf(b, 0.0f);
    }
    __syncthreads();
    for (int c = 0; c < 32; ++c) over = over || !(bound[c] < FP16_SAFE);
  }
  if (t == 0) *needs_all = over ? 1 : 0;
}

// The set-up of a call whose weights are already packed: the counters and
// the uniform page table of the pack prologue, without the packing.
__global__ void prologue_kernel(const hs::PackPrologue pro) {
  const int gid = blockIdx.x * blockDim.x + threadIdx.x;
  if (gid < pro.n0) pro.zero0[gid] = 0;
  if (gid < pro.n1) pro.zero1[gid] = 0;
  if (pro.pages)
    for (int b = gid; b < pro.B; b += gridDim.x * blockDim.x) pro.pages[b] = uniform_page(b, pro.H, pro.W);
}

// Exponents (base 2) of the FP8 form's activation scales s_1..s_4.
struct Fp8Exp {
  int e[4];
};

// the smallest e in [-60, 60] with mx <= 448 * 2^e (0 for mx = 0)
HS_DEV int fp8_exp(float mx) {
  if (!(mx > 0.0f)) return 0;
  int e = 0;
  frexpf(mx / FP8_MAX, &e);
  while (e > -60 && ldexpf(FP8_MAX, e - 1) >= mx) --e;
  while (e < 60 && ldexpf(FP8_MAX, e) < mx) ++e;
  return e;
}

// The FP8 block from the FP32 weights, one workgroup of 256 threads: each
// output channel of layers 2..5 gets the power-of-two weight scale that
// brings its largest |w| to at most 448, and each row's E8M0 scale combines
// it with the activation scales around the layer.
__global__ __launch_bounds__(256) void pack_fp8_kernel(const float* __restrict__ w,
                                                       uint8_t* __restrict__ blk, Fp8Exp ex) {
  __shared__ int ew[4][32];  // [layer 2..5][output channel]
  const int t = threadIdx.x;
  if (t < 128) {
    const int L = t >> 5, co = t & 31;
    const float* wk = w + hs_wk(L + 2) + co * 32 * 9;
    float mx = 0.0f;
    for (int i = 0; i < 32 * 9; ++i) mx = fmaxf(mx, fabsf(wk[i]));
    ew[L][co] = fp8_exp(mx);
  }
  __syncthreads();
  auto es = [&](int k) { return k >= 5 ? 0 : ex.e[k - 1]; };  // exponent of s_k
  // layers 2..5, one 32-bit word (4 codes) per thread and iteration: word
  // i & 7 of the 32-byte slice of lane (i >> 3) & 63 of fragment i >> 9 =
  // ((layer * 3 + dy) * 2 + m); lane (g, r): row 16m + r, tap dx = g
  for (int i = t; i < F8_L1 / 4; i += 256) {
    const int lane = (i >> 3) & 63, f = i >> 9;
    const int m = f & 1, dy = (f >> 1) % 3, L = (f >> 1) / 3;
    const int g = lane >> 4, co = 16 * m + (lane & 15);
    float v[4] = {0.0f, 0.0f, 0.0f, 0.0f};
    if (g < 3) {
#pragma unroll
      for (int b = 0; b < 4; ++b) {
        const int j = 4 * (i & 7) + b;  // byte of the slice = ring position
        const int ci = ring_channel(j >> 3, j & 7);
        v[b] = ldexpf(w[hs_wk(L + 2) + (co * 32 + ci) * 9 + dy * 3 + g], -ew[L][co]);
      }
    }
    uint32_t u = (uint32_t)__builtin_amdgcn_cvt_pk_fp8_f32(v[0], v[1], 0, false);
    u = (uint32_t)__builtin_amdgcn_cvt_pk_fp8_f32(v[2], v[3], (int)u, true);
    ((uint32_t*)(blk + F8_L32))[i] = u;
  }
  // layer 1 in BF16 as in the 16-bit fragments, divided by s_1
  __bf16* l1 = (__bf16*)(blk + F8_L1);
  for (int i = t; i < 128 * 8; i += 256) {
    const int f = i >> 3, e = i & 7, m = f >> 6, l = f & 63, g = l >> 4;
    const int co = 16 * m + (l & 15);
    float v = 0.0f;
    if (g < 3 && e < 6) v = ldexpf(w[HS_W1 + (co * 2 + (e & 1)) * 9 + g * 3 + (e >> 1)], -es(1));
    l1[i] = (__bf16)v;
  }
  {  // scale words: thread t = layer * 64 + lane
    const int L = t >> 6, r = t & 15, k = L + 2;
    uint32_t word = 0x7F7F0000u;
#pragma unroll
    for (int m = 0; m < 2; ++m) {
      const int e = min(max(127 + ew[L][16 * m + r] + es(k - 1) - es(k), 1), 254);
      word |= (uint32_t)e << (8 * m);
    }
    ((uint32_t*)(blk + F8_SCALE))[t] = word;
  }
  float* bias = (float*)(blk + F8_BIAS);
  for (int i = t; i < 5 * 32; i += 256) {
    const int k = 1 + i / 32, c = i & 31;
    bias[i] = ldexpf(w[(k == 1 ? HS_B1 : hs_bk(k)) + c], -es(k));
  }
}

// *out = max(*out, x[0, n)) for non-negative x, n a multiple of 4 (*out
// zeroed before): such floats order like their bit patterns as unsigned
// integers. One atomic per wave.
__global__ void layer_max_kernel(const float4* __restrict__ x, size_t n4, unsigned* out) {
  float m = 0.0f;
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n4;
       i += (size_t)gridDim.x * blockDim.x) {
    const float4 v = x[i];
    m = fmaxf(m, fmaxf(fmaxf(v.x, v.y), fmaxf(v.z, v.w)));
  }
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) m = fmaxf(m, __shfl_xor(m, o));
  if ((threadIdx.x & 63) == 0 && m > 0.0f) atomicMax(out, __float_as_uint(m));
}

// The 16-bit element type of the fused pass: BF16, or FP16 (three more
// mantissa bits at the same matrix-core rate, a range of 65504).
template <typename E>
struct Elem;
template <>
struct Elem<__bf16> {
  using v8 = bf16x8_t;
  using v2 = bf16x2_t;
  static HS_DEV f32x4_t mma(v8 a, v8 b, f32x4_t c) {
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
  }
};
template <>
struct Elem<_Float16> {
  using v8 = f16x8_t;
  using v2 = f16x2_t;
  static HS_DEV f32x4_t mma(v8 a, v8 b, f32x4_t c) {
    return __builtin_amdgcn_mfma_f32_16x16x32_f16(a, b, c, 0, 0, 0);
  }
};

struct FusedArgs {
  const float* contone;
  const uint64_t* seeds;
  const void* frags;  // 16-bit fragments of the element type
  const uint8_t* frags8;  // the FP8 form's block (FP8 form only)
  const float* w;
  const hs::Page* pages;
  int npages, kind;
  long long vtotal;   // sum over pages of strips x (H + FILL): the partition's extent
  float tau;
  hs::Levels lv;      // thresholds of the multitone levels (MULTI only)
  uint8_t* bits;      // bit, or level index (MULTI)
  float* logits;
  uint64_t* list;     // per output wave a segment of seg_cap entries
  int* seg_count;     // entries written per segment
  long long seg_cap;
  int* ovf;           // FP16: set to 1 when an activation left the FP16 range;
                      // FP8: when one saturated
  const int* guard;   // when set: run only if (*guard != 0) == guard_nonzero
  int guard_nonzero;
};

// Overflow tests of an FP16 pass: none (BF16), layer 5 only plus the range
// of the contones (when the a priori bounds clear layers 1..4), or every layer.
enum Check { CHECK_NONE = 0, CHECK_L5 = 1, CHECK_ALL = 2 };

template <int V>
struct StepIndex {
  static constexpr int value = V;
};

// two floats -> packed 16-bit pair (round to nearest even), then ReLU on the
// packed bits: a BF16 or FP16 value with its sign bit set is a negative
// int16, so a 16-bit integer max with 0 is the ReLU (and equals ReLU before
// rounding)
template <typename E>
HS_DEV uint32_t relu_x2(float lo, float hi) {
  const f32x2_t v = {lo, hi};
  const typename Elem<E>::v2 h = __builtin_convertvector(v, typename Elem<E>::v2);
  i16x2_t q;
  __builtin_memcpy(&q, &h, 4);
  q = __builtin_elementwise_max(q, (i16x2_t){0, 0});
  uint32_t u;
  __builtin_memcpy(&u, &q, 4);
  return u;
}

// ReLU + conversion of one finished 16-pixel run in the ring channel order;
// zero where the pixel lies outside the image (the next layer's zero
// padding). CHECK: ovf keeps the running maximum of the packed results as
// unsigned 16-bit pairs; a non-negative FP16 at or above 0x7C00 is inf or
// NaN, so a maximum that reaches it means an activation overflowed.
template <typename E, bool CHECK>
HS_DEV typename Elem<E>::v8 relu_pack(const f32x4_t (&acc)[2], bool in, u16x2_t& ovf) {
  // branch-free: the pairs are packed for every lane and masked (a select
  // per pair instead of a divergent branch around each)
  const uint32_t keep = 0u - (uint32_t)in;
  uint32_t u[4];
#pragma unroll
  for (int m = 0; m < 2; ++m) {
    u[2 * m] = relu_x2<E>(acc[m][0], acc[m][1]) & keep;
    u[2 * m + 1] = relu_x2<E>(acc[m][2], acc[m][3]) & keep;
  }
  if constexpr (CHECK) {
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      u16x2_t q;
      __builtin_memcpy(&q, &u[j], 4);
      ovf = __builtin_elementwise_max(ovf, q);
    }
  }
  typename Elem<E>::v8 v;
  __builtin_memcpy(&v, u, 16);
  return v;
}

// The waves of a workgroup never read each other's global writes, so the
// per-step barrier orders LDS only (hs_lds_barrier): it need not wait for
// the bits, logits and list stores (nor the contone prefetch) to complete.

// MULTI: the output is the level of the logit among a.lv's thresholds
// (multitoning), and the recheck band is around the nearest threshold;
// otherwise the bit [x >= 0] with the band around 0.
// E: the 16-bit element type of activations and weights (BF16 or FP16);
// CHK: the overflow tests (CHECK_NONE for BF16). F8: the FP8 form (E is
// then BF16, the type of layer 1 and of the layer-6 taps).
template <int NW, bool MULTI, typename E, int CHK, bool F8 = false>
__global__ __launch_bounds__(64 * 4 * NW, 1) void fused_infer_kernel(FusedArgs a) {
  static_assert(!F8 || (CHK == CHECK_NONE && sizeof(E) == 2), "the FP8 form runs BF16 layers 1, 6");
  using V8 = typename Elem<E>::v8;
  using V2 = typename Elem<E>::v2;
  constexpr int RPW = 8 / NW, NT = 64 * 4 * NW, HPW = 2 / NW;  // runs, threads, 64-px halves per wave
  // a gated launch exits at once unless its condition holds (the BF16 re-run
  // after an FP16 overflow, the FP16 form the layer bounds select)
  if (a.guard && ((__builtin_amdgcn_readfirstlane(*a.guard) != 0) != (a.guard_nonzero != 0)))
    return;
  __shared__ __attribute__((aligned(16))) E ring[4 * 2 * ROWE];   // layers 1..4
  // input rows as per-column records [(c, z) of columns j, j+1, j+2, 0],
  // each (c, z) a 16-bit pair: one record is a layer-1 operand row
  __shared__ __attribute__((aligned(16))) uint32_t inring[4 * RWID * 4];
  __shared__ __attribute__((aligned(16))) float tring[2 * RWID * 12];  // T, 12 floats per column
  __shared__ V8 cfrag[3 * 64];  // layer-1 A operands (m = 0, 1), layer-6 tap matrix
  __shared__ __attribute__((aligned(16))) float cbias[5 * 32];  // biases of layers 1..5
  __shared__ float osum[3][FW];  // the output stage's running sums, per strip column
  const int tid = threadIdx.x, lane = tid & 63, g = lane >> 4, r = lane & 15;
  // wave-uniform values are kept in scalar registers
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int part = wave % NW, role = wave / NW, k = 2 + role;  // conv layer owned by this wave
  for (int i = tid; i < 4 * 2 * ROWE / 8; i += NT) ((uint4*)ring)[i] = make_uint4(0, 0, 0, 0);
  for (int i = tid; i < 4 * RWID * 4; i += NT) inring[i] = 0u;
  for (int i = tid; i < 2 * RWID * 12; i += NT) tring[i] = 0.0f;
  for (int i = tid; i < 3 * FW; i += NT) osum[i / FW][i % FW] = 0.0f;
  // weights of the owned layer stay in registers (A operands, [dy][dx][m]);
  // the biases and the role operands (layer 1's two A operands, the layer-6
  // tap matrix) are read from LDS where they are used
  const V8* frags = (const V8*)a.frags;
  V8 wA[3][3][2];
  i32x8_t w8[3][2];  // FP8 form: [dy][m], K = the taps dx of kernel row dy
  int sc8 = 0;       // FP8 form: E8M0 row scales of the owned layer, byte m
  if constexpr (F8) {
    const i32x8_t* f8 = (const i32x8_t*)(a.frags8 + F8_L32);
#pragma unroll
    for (int dy = 0; dy < 3; ++dy)
#pragma unroll
      for (int m = 0; m < 2; ++m) w8[dy][m] = f8[(((k - 2) * 3 + dy) * 2 + m) * 64 + lane];
    sc8 = ((const int*)(a.frags8 + F8_SCALE))[(k - 2) * 64 + lane];
    const V8* l1 = (const V8*)(a.frags8 + F8_L1);
    const float* b8 = (const float*)(a.frags8 + F8_BIAS);
    for (int i = tid; i < 3 * 64; i += NT) cfrag[i] = i < 128 ? l1[i] : frags[FRAG_T + (i - 128)];
    for (int i = tid; i < 5 * 32; i += NT) cbias[i] = b8[i];
  } else {
#pragma unroll
    for (int t = 0; t < 9; ++t)
#pragma unroll
      for (int m = 0; m < 2; ++m)
        wA[t / 3][t % 3][m] = frags[FRAG_L32 + (((k - 2) * 9 + t) * 2 + m) * 64 + lane];
    for (int i = tid; i < 3 * 64; i += NT)
      cfrag[i] = frags[i < 128 ? FRAG_L1 + i : FRAG_T + (i - 128)];
    for (int i = tid; i < 5 * 32; i += NT)
      cbias[i] = a.w[i < 32 ? HS_B1 + i : hs_bk(2 + (i - 32) / 32) + (i & 31)];
  }
  uint8_t* const ring8 = (uint8_t*)ring;  // the FP8 form's rings (ROWB8 bytes a row)
  float amax8 = 0.0f;                     // FP8: the largest value before a clamp
  const float b6 = a.w[HS_B6];
  // this lane's element offset in a ring row: chunk g, first column of its
  // runs (tap dx and run n are added as immediates)
  const int col0 = 16 * RPW * part;  // first strip column of this wave's runs
  // three accumulator sets of the owned layer, and the output stage's three
  // running sums per 64-pixel half
  f32x4_t S[3][RPW][2];
#pragma unroll
  for (int j = 0; j < 3; ++j)
#pragma unroll
    for (int n = 0; n < RPW; ++n) S[j][n][0] = S[j][n][1] = f32x4_t{0.f, 0.f, 0.f, 0.f};
  u16x2_t ovf = {0, 0};  // running maximum of the tested FP16 values

  int nflag[HPW];
#pragma unroll
  for (int h = 0; h < HPW; ++h) nflag[h] = 0;
  __syncthreads();

  // This workgroup's equal share [v, vend) of the virtual sequence (page,
  // strip, row), in which every strip has FILL virtual rows before its H
  // real ones; it is cut into segments of one strip each. The divisions and
  // the page lookup are wave-uniform and kept scalar.
  long long v = (long long)blockIdx.x * a.vtotal / gridDim.x;
  const long long vend = (long long)(blockIdx.x + 1) * a.vtotal / gridDim.x;
  while (v < vend) {
    int pg = 0;  // the last page with vstart <= v
    {
      int hi = a.npages - 1;
      while (pg < hi) {
        const int mid = (pg + hi + 1) >> 1;
        if (a.pages[mid].vstart <= v) pg = mid;
        else hi = mid - 1;
      }
    }
    pg = __builtin_amdgcn_readfirstlane(pg);
    const hs::Page P = a.pages[pg];
    const int H = P.H, W = P.W;
    const long long local = v - P.vstart;
    const int strip = (int)(local / (H + FILL));
    const long long sv0 = P.vstart + (long long)strip * (H + FILL);  // the strip's first virtual row
    const long long sv1 = min(sv0 + H + FILL, vend);
    const int Y0 = max((int)(v - sv0) - FILL, 0);
    const int Y1 = max((int)(sv1 - sv0) - FILL, 0);
    v = sv1;
    if (Y1 <= Y0) continue;
    const int X = strip * FS - 6;
    const bool cols_inside = X >= 0 && X + FW <= W;  // no column of the strip is padding
    const size_t img = (size_t)P.off;
    const uint64_t pgbits = (uint64_t)pg << 31;
    const uint64_t seed = a.seeds[pg];
    const int A = Y0 - 6;  // input row of step 0
    const int nsteps = ((Y1 - Y0) + LAG_OUT + 2) / 3 * 3;

    auto step = [&](const int t, auto jc) {
      constexpr int J = decltype(jc)::value;  // == t % 3
      constexpr int M1 = (J + 2) % 3, M2 = (J + 1) % 3;
      const int cur = t & 1, prev = cur ^ 1;
      // per-lane offsets are rebuilt in every step from the lane number (a
      // few VALU operations) instead of being held in registers across the
      // loop; the volatile statement keeps the compiler from hoisting them
      int ln;
      asm volatile("v_mbcnt_lo_u32_b32 %0, -1, 0\n\tv_mbcnt_hi_u32_b32 %0, -1, %0" : "=v"(ln));
      const int lr = ln & 15, lg = ln >> 4;
      // this lane's chunk of its first column written (tap centre) and read
      const int woff = ring_off(col0 + lr + 1, lg);
      // ---- the input waves issue their contone loads first and use them
      // after their MFMAs, which hide the latency
      float cin[HPW];
      if (role == 1) {
        const int ri = A + t;
#pragma unroll
        for (int h = 0; h < HPW; ++h) {
          const int xin = X + 64 * (HPW * part + h) + ln;
          cin[h] = 0.f;
          if (xin >= 0 && xin < W && ri >= 0 && ri < H) cin[h] = a.contone[img + (size_t)ri * W + xin];
        }
      }
      // ---- output stage (waves 2NW..3NW-1), first in the step so that its
      // global stores have drained before anything in a later step waits on
      // the vector memory counter: T row q = A+t-15 finishes output row q-1
      if (role == 2) {
        const int y = A + t - 16;
        const bool row_out = y >= Y0 && y < Y1;
#pragma unroll
        for (int h = 0; h < HPW; ++h) {
          const int Lx = 64 * (HPW * part + h) + ln, x = X + Lx;
          const float* trow = tring + (size_t)prev * RWID * 12 + Lx * 12;
          float sdy[3] = {0.f, 0.f, 0.f};
#pragma unroll
          for (int dy = 0; dy < 3; ++dy)
#pragma unroll
            for (int dx = 0; dx < 3; ++dx) sdy[dy] += trow[dx * 12 + dy * 3 + dx];
          const float xl = osum[M2][Lx] + sdy[2] + b6;
          osum[M1][Lx] += sdy[1];
          osum[J][Lx] = sdy[0];
          if (row_out) {
            const bool valid = Lx >= 6 && Lx < 6 + FS && x < W;
            bool flag = false;
            size_t o = 0;
            int side = xl >= 0.0f ? 1 : 0;
            if (valid) {
              o = img + (size_t)y * W + x;
              if constexpr (MULTI) {
                float dist;
                a.bits[o] = (uint8_t)hs::level_of(a.lv, xl, &dist, &side);
                flag = a.list && dist < a.tau;
              } else {
                a.bits[o] = (uint8_t)side;
                flag = a.list && fabsf(xl) < a.tau;
              }
              if (a.logits) a.logits[o] = xl;
            }
            const uint64_t mask = __ballot(flag);
            if (mask) {
              if (flag) {
                // flagged lanes below this one
                const int below = __builtin_amdgcn_mbcnt_hi((uint32_t)(mask >> 32),
                                                             __builtin_amdgcn_mbcnt_lo((uint32_t)mask, 0u));
                const long long seg = 2LL * blockIdx.x + HPW * part + h;
                // entry: pixel (bits 0-30), page (31-62), the side of the
                // (nearest) threshold written (63)
                a.list[seg * a.seg_cap + nflag[h] + below] =
                    (uint64_t)o | pgbits | (side ? (1ull << 63) : 0ull);
              }
              nflag[h] += __popcll(mask);
            }
          }
        }
      }
      // ---- the set finished in the previous step (row rs) leaves the registers
      if (k < 5) {
        const int rs = A + t + 1 - 3 * k;
        const bool row_in = rs >= 0 && rs < H;
        if constexpr (F8) {
          uint8_t* dst8 = ring8 + ((k - 1) * 2 + cur) * ROWB8 + ring8_off(col0 + lr + 1, lg);
#pragma unroll
          for (int n = 0; n < RPW; ++n) {
            const int x = X + col0 + 16 * n + lr;
            const bool in = row_in && (cols_inside || (x >= 0 && x < W));
            *(uint2*)(dst8 + n * RUNB8) = relu_pack8(S[J][n], in, amax8);
          }
        } else {
          E* dst = ring + ((size_t)(k - 1) * 2 + cur) * ROWE + woff;
#pragma unroll
          for (int n = 0; n < RPW; ++n) {
            const int x = X + col0 + 16 * n + lr;
            const bool in = row_in && (cols_inside || (x >= 0 && x < W));
            *(V8*)(dst + n * RUNE) = relu_pack<E, CHK == CHECK_ALL>(S[J][n], in, ovf);
          }
        }
      } else {  // layer 5: the nine layer-6 taps of row rs into the T ring
        const int rs = A + t - 14;
        const bool row_in = rs >= 0 && rs < H;
        float* trow = tring + (size_t)cur * RWID * 12;
        const V8 w6 = cfrag[128 + ln];
#pragma unroll
        for (int n = 0; n < RPW; ++n) {
          const int c = col0 + 16 * n + lr, x = X + c;
          const bool in = row_in && (cols_inside || (x >= 0 && x < W));
          const f32x4_t tv = Elem<E>::mma(
              w6, relu_pack<E, CHK != CHECK_NONE>(S[J][n], in, ovf), f32x4_t{0.f, 0.f, 0.f, 0.f});
          if (lg < 3) *(f32x4_t*)(trow + (c + 1) * 12 + 4 * lg) = tv;
        }
      }
      {
        const f32x4_t bk0 = *(const f32x4_t*)(cbias + 32 * (k - 1) + 4 * lg);
        const f32x4_t bk1 = *(const f32x4_t*)(cbias + 32 * (k - 1) + 16 + 4 * lg);
#pragma unroll
        for (int n = 0; n < RPW; ++n) {
          S[J][n][0] = bk0;
          S[J][n][1] = bk1;
        }
      }
      // ---- one input row q (written by layer k-1 in the previous step)
      if constexpr (F8) {
        // lane group g reads the record of tap dx = g (group 3 meets zero
        // weights and reads tap 2's); half 1 of a record sits 16 bytes after
        // or before half 0
        const uint8_t* src8 = ring8 + ((k - 2) * 2 + prev) * ROWB8;
        const int cr = col0 + lr + (lg < 3 ? lg : 2);
        const uint8_t* p0 = src8 + ring8_half(cr, 0);
        const uint8_t* p1 = src8 + ring8_half(cr, 1);
#pragma unroll
        for (int n = 0; n < RPW; ++n) {
          const uint4 h0 = *(const uint4*)(p0 + n * RUNB8);
          const uint4 h1 = *(const uint4*)(p1 + n * RUNB8);
          i32x8_t bf;
          __builtin_memcpy(&bf, &h0, 16);
          __builtin_memcpy((char*)&bf + 16, &h1, 16);
          S[J][n][0] = mma8<0>(w8[0][0], bf, S[J][n][0], sc8);
          S[M1][n][0] = mma8<0>(w8[1][0], bf, S[M1][n][0], sc8);
          S[M2][n][0] = mma8<0>(w8[2][0], bf, S[M2][n][0], sc8);
          S[J][n][1] = mma8<1>(w8[0][1], bf, S[J][n][1], sc8);
          S[M1][n][1] = mma8<1>(w8[1][1], bf, S[M1][n][1], sc8);
          S[M2][n][1] = mma8<1>(w8[2][1], bf, S[M2][n][1], sc8);
        }
      } else {
      const E* src = ring + ((size_t)(k - 2) * 2 + prev) * ROWE;
#pragma unroll
      for (int dx = 0; dx < 3; ++dx) {
        const E* srcd = src + ring_off(col0 + lr + dx, lg);
#pragma unroll
        for (int n = 0; n < RPW; ++n) {
          const V8 bf = *(const V8*)(srcd + n * RUNE);
#pragma unroll
          for (int m = 0; m < 2; ++m) {
            S[J][n][m] = Elem<E>::mma(wA[0][dx][m], bf, S[J][n][m]);
            S[M1][n][m] = Elem<E>::mma(wA[1][dx][m], bf, S[M1][n][m]);
            S[M2][n][m] = Elem<E>::mma(wA[2][dx][m], bf, S[M2][n][m]);
          }
        }
      }
      }
      // ---- layer 1 (waves 0..NW-1), after their MFMAs: the wave sharing the
      // SIMD runs the output stage before its own, so the two stages overlap
      // the other wave's matrix-core work. Output row A+t-2 from input rows
      // A+t-3 .. A+t-1
      if (role == 0) {
        const int r1 = A + t - 2;
        const bool row_in = r1 >= 0 && r1 < H;
        // lane group g reads kernel row dy = g (group 3 meets zero weights)
        const int dyl = lg < 3 ? lg : 2;
        const uint4* rec = (const uint4*)inring + ((t + 1 + dyl) & 3) * RWID + col0 + lr;
        E* dst = ring + (size_t)cur * ROWE + woff;
        const V8 w10 = cfrag[ln], w11 = cfrag[64 + ln];
        const f32x4_t b10 = *(const f32x4_t*)(cbias + 4 * lg), b11 = *(const f32x4_t*)(cbias + 16 + 4 * lg);
        auto layer1 = [&]() {
#pragma unroll
          for (int n = 0; n < RPW; ++n) {
            const int c0 = col0 + 16 * n + lr;  // column of tap dx = 0
            const uint4 u = rec[16 * n];
            V8 bf;
            __builtin_memcpy(&bf, &u, 16);
            f32x4_t l1[2];
            l1[0] = Elem<E>::mma(w10, bf, b10);
            l1[1] = Elem<E>::mma(w11, bf, b11);
            const int x = X + c0;
            *(V8*)(dst + n * RUNE) =
                relu_pack<E, CHK == CHECK_ALL>(l1, row_in && x >= 0 && x < W, ovf);
          }
        };
        // the same loop, spelled inline for the multitone forms and as a lambda
        // for the binary ones: with these spellings neither form's step loop
        // spills registers (each spelling spills in the other form)
        if constexpr (F8) {
          uint8_t* dst8 = ring8 + cur * ROWB8 + ring8_off(col0 + lr + 1, lg);
#pragma unroll
          for (int n = 0; n < RPW; ++n) {
            const int c0 = col0 + 16 * n + lr;  // column of tap dx = 0
            const uint4 u = rec[16 * n];
            V8 bf;
            __builtin_memcpy(&bf, &u, 16);
            f32x4_t l1[2];
            l1[0] = Elem<E>::mma(w10, bf, b10);
            l1[1] = Elem<E>::mma(w11, bf, b11);
            const int x = X + c0;
            *(uint2*)(dst8 + n * RUNB8) = relu_pack8(l1, row_in && x >= 0 && x < W, amax8);
          }
        } else if constexpr (MULTI) {
#pragma unroll
          for (int n = 0; n < RPW; ++n) {
            const int c0 = col0 + 16 * n + lr;  // column of tap dx = 0
            const uint4 u = rec[16 * n];
            V8 bf;
            __builtin_memcpy(&bf, &u, 16);
            f32x4_t l1[2];
            l1[0] = Elem<E>::mma(w10, bf, b10);
            l1[1] = Elem<E>::mma(w11, bf, b11);
            const int x = X + c0;
            *(V8*)(dst + n * RUNE) =
                relu_pack<E, CHK == CHECK_ALL>(l1, row_in && x >= 0 && x < W, ovf);
          }
        } else {
          layer1();
        }
      }
      // ---- input stage (waves NW..2NW-1): row A+t into slot t % 4
      if (role == 1) {
        const int ri = A + t;
#pragma unroll
        for (int h = 0; h < HPW; ++h) {
          const int Lx = 64 * (HPW * part + h) + ln, xin = X + Lx;
          const bool xin_ok = xin >= 0 && xin < W;
          const float cval = cin[h];

          // the 64-bit-product Philox only where it does not cost spills:
          // the binary FP16 form that tests layer 5 (the BF16 forms went
          // from 1 to 30 spilled registers with it)
          constexpr bool WIDE = CHK == CHECK_L5 && !MULTI;
          float zval = 0.f;
          if (xin_ok && ri >= 0 && ri < H)
            zval = hs_noise<WIDE>(seed, (uint64_t)ri * W + xin, 0u, a.kind);
          const V2 cz = __builtin_convertvector((f32x2_t){cval, zval}, V2);
          uint32_t u;
          __builtin_memcpy(&u, &cz, 4);
          if constexpr (CHK == CHECK_L5) {
            // the contone range the layer bounds assume: c in [0, 1], i.e. FP16
            // bits at most 0x3C00 (negative c sets bit 15); adding 0x3FFF with
            // saturation reaches 0x7C00 exactly when c lies outside
            const uint32_t hi = u << 16;  // c into the upper half, 0 below
            u16x2_t cv;
            __builtin_memcpy(&cv, &hi, 4);
            ovf = __builtin_elementwise_max(ovf, __builtin_elementwise_add_sat(cv, (u16x2_t){0, 0x3FFF}));
          }
          // column j = Lx + 1 is element e of the record of column j - e
          uint32_t* rrow = inring + (t & 3) * RWID * 4;
          rrow[(Lx + 1) * 4] = u;
          rrow[Lx * 4 + 1] = u;
          if (Lx >= 1) rrow[(Lx - 1) * 4 + 2] = u;
        }
      }
      hs_lds_barrier();
    };
    for (int t = 0; t < nsteps; t += 3) {
      step(t, StepIndex<0>{});
      step(t + 1, StepIndex<1>{});
      step(t + 2, StepIndex<2>{});
    }
  }
  if constexpr (CHK != CHECK_NONE) {
    // a packed half at or above 0x7C00 is inf or NaN; no wave reads the flag
    const bool bad = ovf[0] >= 0x7C00 || ovf[1] >= 0x7C00;
    if (__ballot(bad) && lane == 0 && a.ovf) *a.ovf = 1;
  }
  if constexpr (F8) {
    if (__ballot(amax8 > FP8_MAX) && lane == 0 && a.ovf) *a.ovf = 1;
  }
  // recheck list: the output stage's 64-pixel halves each own a segment
  if (role == 2 && lane == 0 && a.seg_count) {
#pragma unroll
    for (int h = 0; h < HPW; ++h) a.seg_count[2 * blockIdx.x + HPW * part + h] = nflag[h];
  }
}

// A page table travels to the device in kernel arguments, 48 pages at a
// time (no host buffer has to outlive the call).
constexpr int PAGE_CHUNK = 48;
struct PageChunk {
  hs::Page p[PAGE_CHUNK];
  int first, n;
};
__global__ void put_pages_kernel(hs::Page* pages, PageChunk c) {
  if ((int)threadIdx.x < c.n) pages[c.first + threadIdx.x] = c.p[threadIdx.x];
}

// Pages of a uniform batch: B images of H x W.
__global__ void uniform_pages_kernel(hs::Page* pages, int B, int H, int W) {
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b < B) pages[b] = uniform_page(b, H, W);
}

}  // namespace

namespace hs {

size_t fused_frag_bytes() { return (size_t)FRAG_TOTAL * 16; }
size_t fp8_block_bytes() { return (size_t)F8_TOTAL; }

hipError_t launch_fp8_pack(const float* w, void* blk, const int* act_exp, hipStream_t s) {
  Fp8Exp ex;
  for (int k = 0; k < 4; ++k) ex.e[k] = act_exp[k];
  pack_fp8_kernel<<<1, 256, 0, s>>>(w, (uint8_t*)blk, ex);
  return hipGetLastError();
}

hipError_t launch_layer_max(const float* x, size_t n, float* out, hipStream_t s) {
  const size_t n4 = n / 4;
  size_t blocks = (n4 + 255) / 256;
  if (blocks > 2048) blocks = 2048;
  if (blocks < 1) blocks = 1;
  layer_max_kernel<<<(unsigned)blocks, 256, 0, s>>>((const float4*)x, n4, (unsigned*)out);
  return hipGetLastError();
}

hipError_t launch_fused_pack(const float* w, void* frags, void* frags16, int* needs_all,
                             const PackPrologue& pro, hipStream_t s) {
  pack_fused_kernel<<<38, 256, 0, s>>>(w, (__bf16*)frags, (_Float16*)frags16, needs_all, pro);
  return hipGetLastError();
}

hipError_t launch_prologue(const PackPrologue& pro, hipStream_t s) {
  prologue_kernel<<<1, 256, 0, s>>>(pro);
  return hipGetLastError();
}

int fused_strips(int W) { return (W + FS - 1) / FS; }
int fused_fill() { return FILL; }

hipError_t launch_put_pages(Page* dst, const Page* src_host, int n, hipStream_t s) {
  for (int first = 0; first < n; first += PAGE_CHUNK) {
    PageChunk c;
    c.first = first;
    c.n = n - first < PAGE_CHUNK ? n - first : PAGE_CHUNK;
    for (int i = 0; i < c.n; ++i) c.p[i] = src_host[first + i];
    put_pages_kernel<<<1, 64, 0, s>>>(dst, c);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

hipError_t launch_uniform_pages(Page* pages, int B, int H, int W, hipStream_t s) {
  uniform_pages_kernel<<<(B + 255) / 256, 256, 0, s>>>(pages, B, H, W);
  return hipGetLastError();
}

// Geometry of the persistent launch over pages of the given shapes:
// workgroups (one per CU, fewer when there are under 32 strip rows per CU),
// the virtual extent, and an upper bound on the real strip rows of one
// workgroup's share.
void fused_geometry(const int* shapes_host, int npages, int num_cus, int* grid,
                    long long* vtotal, long long* max_rows) {
  long long total = 0, vt = 0;
  for (int p = 0; p < npages; ++p) {
    const int H = shapes_host[2 * p], W = shapes_host[2 * p + 1];
    total += (long long)fused_strips(W) * H;
    vt += (long long)fused_strips(W) * (H + FILL);
  }
  long long per = (total + num_cus - 1) / num_cus;
  if (per < 32) per = 32;
  const int g = (int)((total + per - 1) / per);
  *grid = g;
  *vtotal = vt;
  *max_rows = (vt + g - 1) / g + 1;
}

// Entries of the segmented recheck list: two segments per workgroup, each
// able to hold every pixel its wave writes.
size_t fused_list_entries(const int* shapes_host, int npages, int num_cus) {
  int grid;
  long long vt, rows;
  fused_geometry(shapes_host, npages, num_cus, &grid, &vt, &rows);
  return (size_t)grid * 2 * (size_t)rows * 64;
}

hipError_t launch_fused_infer(const float* w, const float* contone, const uint64_t* seeds,
                              const Page* pages, const int* shapes_host, int npages, int kind,
                              float tau, const Levels& lv, uint8_t* bits, float* logits,
                              uint64_t* list, int* seg_count, int* nseg, long long* seg_cap,
                              const void* frags, const void* frags8, int form, int* ovf,
                              const int* guard, int guard_nonzero, int num_cus, hipStream_t s) {
  FusedArgs a;
  a.contone = contone;
  a.seeds = seeds;
  a.frags = frags;
  a.frags8 = (const uint8_t*)frags8;
  a.ovf = ovf;
  a.guard = guard;
  a.guard_nonzero = guard_nonzero;
  a.w = w;
  a.pages = pages;
  a.npages = npages;
  a.kind = kind;
  int grid;
  long long rows;
  fused_geometry(shapes_host, npages, num_cus, &grid, &a.vtotal, &rows);
  a.tau = tau;
  a.lv = lv;
  a.bits = bits;
  a.logits = logits;
  a.list = list;
  a.seg_count = seg_count;
  a.seg_cap = rows * 64;
  *nseg = 2 * grid;
  *seg_cap = a.seg_cap;
  const bool binary = lv.n == 1 && lv.thr[0] == 0.0f;
  const dim3 block(64 * 4 * FUSED_NW);
  constexpr int N = FUSED_NW;
  if (form == FUSED_FP8) {
    if (binary) fused_infer_kernel<N, false, __bf16, CHECK_NONE, true><<<grid, block, 0, s>>>(a);
    else fused_infer_kernel<N, true, __bf16, CHECK_NONE, true><<<grid, block, 0, s>>>(a);
  } else if (form == FUSED_FP16_L5) {
    if (binary) fused_infer_kernel<N, false, _Float16, CHECK_L5><<<grid, block, 0, s>>>(a);
    else fused_infer_kernel<N, true, _Float16, CHECK_L5><<<grid, block, 0, s>>>(a);
  } else if (form == FUSED_FP16_ALL) {
    if (binary) fused_infer_kernel<N, false, _Float16, CHECK_ALL><<<grid, block, 0, s>>>(a);
    else fused_infer_kernel<N, true, _Float16, CHECK_ALL><<<grid, block, 0, s>>>(a);
  } else {
    if (binary) fused_infer_kernel<N, false, __bf16, CHECK_NONE><<<grid, block, 0, s>>>(a);
    else fused_infer_kernel<N, true, __bf16, CHECK_NONE><<<grid, block, 0, s>>>(a);
  }
  return hipGetLastError();
}

}  // namespace hs

