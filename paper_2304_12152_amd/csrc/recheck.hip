// recheck.hip -- the exact decision of near-threshold pixels (the TEST
// procedure of Algorithm 1 at p = 0.5) after the fused BF16 pass.
//
// A listed pixel is recomputed over its 13 x 13 receptive field only: layer
// k is evaluated on the (13 - 2k) x (13 - 2k) window centred on the pixel
// (its "cone"), with every activation outside the image forced to zero (the
// zero 'same' padding of each layer). Up to three stages:
//   FP16 stage   (after a BF16 pass) every pixel the fused pass listed
//                (|x_bf16| < tau); layers 1..5 with FP16 products on the
//                matrix cores, layer 6 in FP32. Pixels with |x| >= tau16 are
//                decided here, the rest listed again.
//   split stage  the pixels still listed; the same with split-BF16
//                products, decided at |x| >= tau2.
//   FP32 stage   the pixels listed by the split stage, in plain FP32.
// With multitone levels (Sec. VI-E) the same holds with |x| replaced by the
// distance to the nearest level threshold; the output is the level.
#include "hs_common.h"
#include "hs_internal.h"

namespace {

// ===========================================================================
// Cone stages. A listed pixel's receptive field is recomputed in one of two
// precisions by the same pipelined kernel:
//   split (HALF = false): every FP32 value v is carried as hi + lo with
//     hi = bf16(v) and lo = bf16(v - hi); a product is taken as
//     hi*hi' + lo*hi' + hi*lo' (lo*lo', ~2^-16 relative, is dropped), each of
//     the three in its own FP32 accumulator. The result's error is ~2^-8 of
//     the BF16 pass's.
//   FP16 (HALF = true): weights and activations of layers 1..5 rounded to
//     FP16 (11 significant bits to BF16's 8), one product per operand pair,
//     FP32 accumulation, layer 5's output and layer 6 in FP32: about 1/8 of
//     the BF16 pass's error for a third of the split stage's matrix work.
//     FP16 holds at most 65504: a cone in which any stored activation (or
//     the contone, or a weight) would round to infinity is not decided here
//     but passed on to the split stage.
// Each stage decides the pixels whose recomputed logit is at least its band
// from the nearest threshold and lists the rest for the next stage.
//
// The kernel is a pipeline over the listed pixels, one cone per step. Each
// wave owns one layer (its A fragments stay in registers for the whole
// kernel; in the split form the lo fragments of all four layers sit in LDS)
// and up to two of that layer's 16-position runs, which it computes together
// (independent MFMA chains, the next tap's operands loaded while a tap's
// MFMAs run). In step t the stage of layer k works on cone t - k:
//   stage 0    the (c, z) state of the 13 x 13 window (z drawn from Philox
//              exactly as the fused pass drew it)
//   stage 1-5  layers 1..5 (layer 5's output kept in FP32)
//   stage 6    layer 6 in FP32 and the decision
// Stage k reads the buffer stage k-1 wrote in the previous step and writes
// its own; every buffer has two slots (cone parity), so one barrier per step
// orders all of it. The barrier orders LDS only: the global loads issued for
// a later step (list entries, window values) stay in flight across it.
//
// Waves (w and w+4 share a SIMD), split form (balanced by measured step
// times):
//   w0, w1, w2  layer 2, runs 0-1 / 2-3 / 4-5; layer 1, run 0 / 1 / 2
//   w3          layer 3, runs 0-1; staging of window positions 0-63; layer 6
//   w4          layer 3, runs 2-3
//   w5          layer 4, runs 0-1
//   w6          layer 5, run 0; layer 1, runs 3-5
//   w7          layer 1, runs 6-7; staging of positions 64-168; the cone list
// FP16 form (a third of the matrix work, so the staging is spread out):
//   w0, w1, w2  as above
//   w3          layer 3, runs 0-1; staging of positions 0-63; layer 6
//   w4          layer 3, runs 2-3; layer 1, runs 3-4; staging of 128-168
//   w5          layer 4, runs 0-1; layer 1, runs 5-6
//   w6          layer 5, run 0; layer 1, run 7; staging of 64-127
//   w7          the cone list
// (a layer-1 run is 2 products of 16x16x32 per precision term, a
// layer-2..5 run 18)
// ===========================================================================
constexpr int SPLIT_MAXSEG = 1024;    // list segments the stage accepts
constexpr int NSTAGE = 7;             // staging, layers 1..5, layer 6
constexpr int SPLIT_THREADS = 512;
constexpr float F16_INF_AT = 65520.0f;  // smallest value that rounds to FP16 infinity

// the element type of a form: operand fragments, record size (bytes per
// staged position: 4 lane groups x (hi, lo) x 16 B, or 4 x 16 B) and the
// record's chunk swizzle (spreads a run's reads over the banks)
template <bool HALF> struct ConeForm;
template <> struct ConeForm<false> {
  using op = bf16x8_t;
  static constexpr int REC = 128;
  // 16 consecutive positions read one chunk each: adding bit 3 of the
  // position spreads positions 8 apart over different banks (measured: 356
  // -> 332 us for the 25,094 cones of the 8 x 1024 x 1024 batch)
  static HS_DEV int slot(int p, int c) { return c ^ ((p + (p >> 3)) & 7); }
  static HS_DEV f32x4_t mma(op a, op b, f32x4_t c) {
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
  }
};
template <> struct ConeForm<true> {
  using op = f16x8_t;
  static constexpr int REC = 64;
  static HS_DEV int slot(int p, int c) { return c ^ (p & 3); }
  static HS_DEV f32x4_t mma(op a, op b, f32x4_t c) {
    return __builtin_amdgcn_mfma_f32_16x16x32_f16(a, b, c, 0, 0, 0);
  }
};

// cone record: pixel (-1: none), row, column, bit of the fused pass, page,
// page height and width, seed (two words)
enum { CI_O, CI_Y, CI_X, CI_BIT, CI_PG, CI_H, CI_W, CI_SLO, CI_SHI, CI_N };

constexpr int win_edge(int k) { return 13 - 2 * k; }           // layer k's output window edge
constexpr int win_pos(int k) { return win_edge(k) * win_edge(k); }
constexpr int win_runs(int k) { return (win_pos(k) + 15) / 16; }
static_assert(win_runs(1) == 8 && win_runs(2) == 6 && win_runs(3) == 4 && win_runs(4) == 2 &&
                  win_runs(5) == 1,
              "wave roles assume these run counts");

// element i of the cone fragments: layers 2..5 in the ring channel order,
// [layer][tap][m][lane][8]
constexpr int SPLIT_ELEMS = 4 * 9 * 2 * 64 * 8;
HS_DEV float cone_weight(const float* __restrict__ w, int i) {
  const int e = i & 7, l = (i >> 3) & 63, m = (i >> 9) & 1, t = (i >> 10) % 9,
            layer = (i >> 10) / 9;
  const int g = l >> 4, r = l & 15;
  return w[hs_wk(layer + 2) + ((16 * m + r) * 32 + hs_ring_channel(g, e)) * 9 + t];
}

struct SplitArgs {
  const float* w;
  const float* contone;
  const uint64_t* seeds;
  const hs::Page* pages;
  int kind, nseg;
  const uint64_t* seglist;
  const int* seg_count;
  long long seg_cap;
  const void* whi;        // hi (split) or FP16 fragments of layers 2..5
  const bf16x8_t* wlo;    // lo fragments (split form)
  const int* wflag;       // FP16 form: nonzero if a weight of layers 1..5 overflows FP16
  float tau2;             // the band of this stage
  hs::Levels lv;          // output thresholds (binary: {0})
  uint64_t* list2;
  int* count2;
  uint8_t* bits;
  float* logits;
  int32_t* stats;
  int total_slot;         // stats entry that receives this stage's input count
};

template <bool HALF>
struct SplitSmem {
  static constexpr int REC = ConeForm<HALF>::REC;
  __attribute__((aligned(16))) float s0[2][169 * 2];  // (c, z) of the 13 x 13 window
  __attribute__((aligned(16))) char b1[2][121 * REC];  // layer outputs
  __attribute__((aligned(16))) char b2[2][81 * REC];
  __attribute__((aligned(16))) char b3[2][49 * REC];
  __attribute__((aligned(16))) char b4[2][25 * REC];
  float l5[2][9 * 32];                                   // layer 5 in FP32
  bf16x8_t wlo[HALF ? 1 : 4][9][2][HALF ? 1 : 64];       // layers 2..5, lo parts (split)
  typename ConeForm<HALF>::op w1[2][2][64];              // layer 1: [hi, lo][m][lane]
  float w6[288];                                         // layer 6, [channel][tap]
  __attribute__((aligned(16))) float b1v[32];           // layer 1 bias
  int spre[SPLIT_MAXSEG + 1];                            // exclusive prefix of the segment counts
  int cinfo[16][CI_N];  // per cone, the CI_* fields
  int covf[16];         // per cone: an FP16 activation overflowed
};

// one position's 32 channels (lane group g's 8 of them) into a record
template <bool HALF>
HS_DEV void cone_store(char* rec_base, int p, int g, const float (&v)[2][4], bool& ovf) {
  using F = ConeForm<HALF>;
  char* rec = rec_base + p * F::REC;
  if constexpr (HALF) {
    f16x8_t vh;
#pragma unroll
    for (int m = 0; m < 2; ++m)
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        vh[4 * m + i] = (_Float16)v[m][i];
        ovf = ovf || v[m][i] >= F16_INF_AT;  // ReLU'd: never negative or NaN
      }
    *(f16x8_t*)(rec + F::slot(p, g) * 16) = vh;
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
    *(bf16x8_t*)(rec + F::slot(p, 2 * g) * 16) = vh;
    *(bf16x8_t*)(rec + F::slot(p, 2 * g + 1) * 16) = vl;
  }
}

// Layer K (2..5) on runs run0 .. run0 + NR - 1 of one cone (ci); src / dst
// are the cone's input and output slots; returns whether a stored value
// overflowed FP16 (FP16 form).
template <bool HALF, int K, int NR>
HS_DEV bool cone_layer(const typename ConeForm<HALF>::op (&wh)[9][2], const bf16x8_t* wl,
                       const f32x4_t (&bias)[2], const char* src, char* dst, float* dst5,
                       const int* ci, int run0, int lane) {
  using F = ConeForm<HALF>;
  using op = typename F::op;
  constexpr int EO = win_edge(K), EI = EO + 2, NP = EO * EO;
  const int H = ci[CI_H], W = ci[CI_W];
  const int g = lane >> 4, r = lane & 15;
  int ln = lane;
  asm volatile("" : "+v"(ln));
  int p[NR], q0[NR];
  f32x4_t a0[NR][2], a1[NR][2], a2[NR][2];
  // the per-tap LDS addresses are recomputed in every call (a few VALU
  // operations) rather than hoisted out of the step loop, where they would
  // occupy registers for the whole kernel; the empty asm hides q0's value
#pragma unroll
  for (int j = 0; j < NR; ++j) {
    const int P = (run0 + j) * 16 + r;
    p[j] = P < NP ? P : -1;
    const int pp = P < NP ? P : 0;
    q0[j] = (pp / EO) * EI + pp % EO;
    asm volatile("" : "+v"(q0[j]));
#pragma unroll
    for (int m = 0; m < 2; ++m) a0[j][m] = a1[j][m] = a2[j][m] = f32x4_t{0.f, 0.f, 0.f, 0.f};
  }
  // the operands of tap t + PD are loaded while tap t's MFMAs run (PD = 2
  // in the FP16 form, whose 4 MFMAs per tap are too short to cover one load
  // latency; 1 in the split form, with 12); the scheduling barrier at the
  // end of each tap keeps the compiler from hoisting every tap's loads to
  // the top (which would exhaust the registers)
  constexpr int PD = HALF ? 2 : 1, NS = PD + 1;
  op bh[NS][NR], bl[NS][NR];
  bf16x8_t wlo[NS][2];
  auto load_tap = [&](int t, int s) {
#pragma unroll
    for (int j = 0; j < NR; ++j) {
      const int q = q0[j] + (t / 3) * EI + t % 3;
      const char* rec = src + q * F::REC;
      if constexpr (HALF) {
        bh[s][j] = *(const op*)(rec + F::slot(q, g) * 16);
      } else {
        bh[s][j] = *(const op*)(rec + F::slot(q, 2 * g) * 16);
        bl[s][j] = *(const op*)(rec + F::slot(q, 2 * g + 1) * 16);
      }
    }
    if constexpr (!HALF) {
      wlo[s][0] = wl[(t * 2 + 0) * 64 + ln];
      wlo[s][1] = wl[(t * 2 + 1) * 64 + ln];
    }
  };
#pragma unroll
  for (int t = 0; t < PD; ++t) load_tap(t, t);
#pragma unroll
  for (int t = 0; t < 9; ++t) {
    const int s = t % NS;
    if (t + PD < 9) load_tap(t + PD, (t + PD) % NS);
#pragma unroll
    for (int j = 0; j < NR; ++j)
#pragma unroll
      for (int m = 0; m < 2; ++m) {
        a0[j][m] = F::mma(wh[t][m], bh[s][j], a0[j][m]);
        if constexpr (!HALF) {
          a1[j][m] = F::mma(wlo[s][m], bh[s][j], a1[j][m]);
          a2[j][m] = F::mma(wh[t][m], bl[s][j], a2[j][m]);
        }
      }
    __builtin_amdgcn_sched_barrier(0);
  }
  const bool cone = ci[CI_O] >= 0;
  bool ovf = false;
#pragma unroll
  for (int j = 0; j < NR; ++j) {
    if (p[j] < 0) continue;
    const int pi = p[j] / EO, pj = p[j] % EO;
    const int gy = ci[CI_Y] - (6 - K) + pi, gx = ci[CI_X] - (6 - K) + pj;
    const bool in_img = cone && gy >= 0 && gy < H && gx >= 0 && gx < W;
    float v[2][4];
#pragma unroll
    for (int m = 0; m < 2; ++m) {
      const f32x4_t s = HALF ? a0[j][m] : a0[j][m] + (a1[j][m] + a2[j][m]);
#pragma unroll
      for (int i = 0; i < 4; ++i) v[m][i] = in_img ? fmaxf(s[i] + bias[m][i], 0.f) : 0.f;
    }
    if (K < 5) {
      cone_store<HALF>(dst, p[j], g, v, ovf);
    } else {
      float* d = dst5 + p[j] * 32;
#pragma unroll
      for (int m = 0; m < 2; ++m)
#pragma unroll
        for (int i = 0; i < 4; ++i) d[16 * m + 4 * g + i] = v[m][i];
    }
  }
  return ovf;
}

template <bool HALF>
__global__ __launch_bounds__(SPLIT_THREADS, 1) void recheck_split_kernel(SplitArgs a) {
  using F = ConeForm<HALF>;
  using op = typename F::op;
  __shared__ SplitSmem<HALF> sm;
  const int tid = threadIdx.x, lane = tid & 63, g = lane >> 4, r = lane & 15;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  // ---- wave roles (see the table above); wave 7 owns no layer
  const int K = wave < 3 ? 2 : wave < 5 ? 3 : wave == 5 ? 4 : wave == 6 ? 5 : 0;
  const int run0 = (wave < 3) ? 2 * wave : (wave == 4) ? 2 : 0;
  // the owned layer's A operands (hi or FP16) and biases, for the whole
  // kernel; the lo A operands of all four layers in LDS
  op wh[9][2];
  f32x4_t bias[2];
  if constexpr (!HALF)
    for (int i = tid; i < 4 * 9 * 2 * 64; i += SPLIT_THREADS) (&sm.wlo[0][0][0][0])[i] = a.wlo[i];
  {
    const int kk = K ? K : 2;
    const op* whi = (const op*)a.whi;
#pragma unroll
    for (int t = 0; t < 9; ++t)
#pragma unroll
      for (int m = 0; m < 2; ++m) wh[t][m] = whi[(((kk - 2) * 9 + t) * 2 + m) * 64 + lane];
#pragma unroll
    for (int m = 0; m < 2; ++m)
#pragma unroll
      for (int i = 0; i < 4; ++i) bias[m][i] = a.w[hs_bk(kk) + 16 * m + 4 * g + i];
  }
  // layer 1's A operands in LDS: K = 9 taps x 2 channels, lane group g =
  // kernel row, slot e = (dx = e / 2, channel e % 2); zero in the padding slots
  if (wave < 2) {
    const int m = wave;
    op vh, vl;
#pragma unroll
    for (int e = 0; e < 8; ++e) {
      const float v =
          (g < 3 && e < 6) ? a.w[HS_W1 + ((16 * m + r) * 2 + (e & 1)) * 9 + g * 3 + (e >> 1)] : 0.0f;
      if constexpr (HALF) {
        vh[e] = (_Float16)v;
        vl[e] = (_Float16)0.0f;
      } else {
        const __bf16 h = (__bf16)v;
        vh[e] = h;
        vl[e] = (__bf16)(v - (float)h);
      }
    }
    sm.w1[0][m][lane] = vh;
    sm.w1[1][m][lane] = vl;
  }
  if (tid < 32) sm.b1v[tid] = a.w[HS_B1 + tid];
  // ---- concatenate the segments: wave 0 scans the counts (per lane a
  // chunk of consecutive segments, then a wave-wide scan of the chunk sums)
  if (wave == 0) {
    constexpr int PER = (SPLIT_MAXSEG + 63) / 64;
    int cs = 0;
#pragma unroll
    for (int j = 0; j < PER; ++j) {
      const int q = lane * PER + j;
      cs += q < a.nseg ? a.seg_count[q] : 0;
    }
    int incl = cs;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
      const int v = __shfl_up(incl, d);
      if (lane >= d) incl += v;
    }
    int run = incl - cs;
#pragma unroll
    for (int j = 0; j < PER; ++j) {
      const int q = lane * PER + j;
      if (q <= a.nseg) sm.spre[q] = run;
      run += q < a.nseg ? a.seg_count[q] : 0;
    }
  }
  __syncthreads();
  const int total = sm.spre[a.nseg];
  const int cb0 = (int)((long long)blockIdx.x * total / gridDim.x);
  const int cb1 = (int)((long long)(blockIdx.x + 1) * total / gridDim.x);
  const int nloc = cb1 - cb0;
  if (blockIdx.x == 0 && tid == 0) {
    a.stats[a.total_slot] = total;
    if (!HALF) a.stats[4] = total;  // the pixels the split stage recomputes
  }
  if (nloc <= 0) return;  // uniform over the block
  // FP16 form: weights outside FP16's range send every cone on
  const bool wbad = HALF && *a.wflag != 0;

  // Cone i's record goes to cinfo[i % 16] (wave 7, lane 0), three steps
  // before cone i is staged. Wave 7 loads the list entries 64 at a time (one
  // per lane, 64 cones before they are decoded) and hands them to lane 0
  // with readlane, so no step waits on a list load; the page record is
  // loaded when the page changes. The segment of entry e is the last with
  // spre <= e.
  int cpage = -1;
  hs::Page cp = {};
  uint64_t cseed = 0;
  auto load_batch = [&](int j) -> uint64_t {  // entry of cone 64 j + lane
    const int i = 64 * j + lane;
    if (i >= nloc) return 0;
    const int e = cb0 + i;
    int lo = 0, hi = a.nseg - 1;  // spre[lo] <= e < spre[hi + 1]
    while (lo < hi) {
      const int mid = (lo + hi + 1) >> 1;
      if (sm.spre[mid] <= e) lo = mid;
      else hi = mid - 1;
    }
    return a.seglist[(size_t)lo * a.seg_cap + (e - sm.spre[lo])];
  };
  auto put_cone = [&](int i, uint64_t u) {
    int* d = sm.cinfo[i & 15];
    sm.covf[i & 15] = 0;
    if (i >= nloc) {
      d[CI_O] = -1;
      d[CI_Y] = d[CI_X] = d[CI_BIT] = d[CI_PG] = d[CI_SLO] = d[CI_SHI] = 0;
      d[CI_H] = d[CI_W] = 1;
      return;
    }
    const int page = hs::entry_page(u);
    if (page != cpage) {
      cpage = page;
      cp = a.pages[page];
      cseed = a.seeds[page];
    }
    const int o = (int)hs::entry_pixel(u);
    const int local = (int)(o - cp.off);
    d[CI_O] = o;
    d[CI_Y] = local / cp.W;
    d[CI_X] = local - (local / cp.W) * cp.W;
    d[CI_BIT] = hs::entry_bit(u);
    d[CI_PG] = page;
    d[CI_H] = cp.H;
    d[CI_W] = cp.W;
    d[CI_SLO] = (int)(uint32_t)cseed;
    d[CI_SHI] = (int)(uint32_t)(cseed >> 32);
  };
  uint64_t ebuf0 = 0, ebuf1 = 0;  // entries of batches 2j and 2j + 1
  auto decode = [&](int i) {      // wave 7: cone i's record; refills the batch of i - 64
    const uint64_t b = ((i >> 6) & 1) ? ebuf1 : ebuf0;
    const uint32_t ulo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)b, i & 63);
    const uint32_t uhi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(b >> 32), i & 63);
    if (lane == 0) put_cone(i, (uint64_t)ulo | ((uint64_t)uhi << 32));
    if ((i & 63) == 63 && i + 65 < nloc) {  // batch i >> 6 is used up: load i >> 6 + 2
      if ((i >> 6) & 1) ebuf1 = load_batch((i >> 6) + 2);
      else ebuf0 = load_batch((i >> 6) + 2);
    }
  };
  // staging: window positions j = 64 s + lane for the wave's slots s. The
  // split form stages on waves 3 (slot 0) and 7 (slots 1, 2); the FP16 form,
  // whose layer waves have slack, on waves 3, 6 and 4 (one slot each). The
  // contone values are loaded a step ahead, always from a valid address
  // (the same loads every step, no branch), and masked where they are used
  // (a select on the loaded value would wait for it at once).
  constexpr int NSTG = 2;
  const int slot0 = HALF ? (wave == 3 ? 0 : wave == 6 ? 1 : wave == 4 ? 2 : -1)
                         : (wave == 3 ? 0 : wave == 7 ? 1 : -1);
  const int nslot = slot0 < 0 ? 0 : (!HALF && wave == 7) ? 2 : 1;
  const bool stager = nslot > 0;
  auto stage_pos = [&](int k) { return k < nslot ? 64 * (slot0 + k) + lane : 999; };
  float pcv[NSTG];
  auto prefetch_window = [&](int i) {
    const int* ci = sm.cinfo[i & 15];
    const int H = ci[CI_H], W = ci[CI_W], o = ci[CI_O];
#pragma unroll
    for (int k = 0; k < NSTG; ++k) {
      const int j = stage_pos(k);
      const int dy = j / 13 - 6, dx = j % 13 - 6;
      const int gy = ci[CI_Y] + dy, gx = ci[CI_X] + dx;
      const bool ok = j < 169 && i < nloc && o >= 0 && gy >= 0 && gy < H && gx >= 0 && gx < W;
      pcv[k] = a.contone[ok ? o + dy * W + dx : 0];
    }
  };
  for (int i = tid; i < 288; i += SPLIT_THREADS) sm.w6[i] = a.w[HS_W6 + i];
  const float b6 = a.w[HS_B6];
  // prologue: the first two batches of entries, cones 0..2 decoded, the
  // window values of cone 0 in flight
  if (wave == 7) {
    ebuf0 = load_batch(0);
    ebuf1 = load_batch(1);
    for (int i = 0; i < 3; ++i) decode(i);
  }
  __syncthreads();
  if (stager) prefetch_window(0);

  for (int t = 0; t < nloc + NSTAGE - 1; ++t) {
    // ---- stage 0: the (c, z) window of cone t from the prefetched values,
    // then the loads of cone t + 1's window
    if (stager) {
      if (t < nloc) {
        const int* ci = sm.cinfo[t & 15];
        const int H = ci[CI_H], W = ci[CI_W];
        const uint64_t sd = (uint64_t)(uint32_t)ci[CI_SLO] | ((uint64_t)(uint32_t)ci[CI_SHI] << 32);
#pragma unroll
        for (int k = 0; k < NSTG; ++k) {
          const int j = stage_pos(k);
          if (j < 169) {
            const int gy = ci[CI_Y] - 6 + j / 13, gx = ci[CI_X] - 6 + j % 13;
            const bool in = ci[CI_O] >= 0 && gy >= 0 && gy < H && gx >= 0 && gx < W;
            float zv = 0.f;
            if (in) zv = hs_noise<true>(sd, (uint64_t)gy * W + gx, 0u, a.kind);
            sm.s0[t & 1][j * 2] = in ? pcv[k] : 0.f;
            sm.s0[t & 1][j * 2 + 1] = zv;
          }
        }
      }
      prefetch_window(t + 1);
    }
    // ---- cone t + 3 decoded
    if (wave == 7) decode(t + 3);
    // ---- stage 1: layer 1 of cone t - 1, one run at a time (split: waves
    // 0-2 one run each, wave 6 three, wave 7 two; FP16: waves 0-2 one each,
    // waves 4 and 5 two, wave 6 one)
    const int l1run0 = wave < 3 ? wave
                       : HALF ? (wave == 4 ? 3 : wave == 5 ? 5 : wave == 6 ? 7 : 0)
                              : (wave == 6 ? 3 : 6);
    const int l1runs = wave < 3 ? 1
                       : HALF ? (wave == 4 || wave == 5 ? 2 : wave == 6 ? 1 : 0)
                              : (wave == 6 ? 3 : wave == 7 ? 2 : 0);
    if (l1runs && t >= 1 && t - 1 < nloc) {
      const int i = t - 1, sl = i & 1;
      const int* ci = sm.cinfo[i & 15];
      const bool cone = ci[CI_O] >= 0;
      const int H = ci[CI_H], W = ci[CI_W];
      const op ah0 = sm.w1[0][0][lane], al0 = sm.w1[1][0][lane];
      const op ah1 = sm.w1[0][1][lane], al1 = sm.w1[1][1][lane];
      const f32x4_t bb0 = *(const f32x4_t*)&sm.b1v[4 * g];
      const f32x4_t bb1 = *(const f32x4_t*)&sm.b1v[16 + 4 * g];
      bool ovf = false;
      for (int run = l1run0; run < l1run0 + l1runs; ++run) {
        const int P = run * 16 + r;
        const int p = P < 121 ? P : 0;
        const int pi = p / 11, pj = p - (p / 11) * 11;
        // six consecutive floats: (c, z) of columns pj .. pj + 2 of row pi + dy
        const f32x2_t* sp = (const f32x2_t*)&sm.s0[sl][((pi + (g < 3 ? g : 2)) * 13 + pj) * 2];
        const f32x2_t v0 = sp[0], v1 = sp[1], v2 = sp[2];
        const float vv[8] = {v0[0], v0[1], v1[0], v1[1], v2[0], v2[1], 0.f, 0.f};
        const f32x4_t z4 = {0.f, 0.f, 0.f, 0.f};
        f32x4_t s0v, s1v;
        if constexpr (HALF) {
          f16x8_t bh;
#pragma unroll
          for (int e = 0; e < 8; ++e) {
            bh[e] = (_Float16)vv[e];
            ovf = ovf || !(fabsf(vv[e]) < F16_INF_AT);  // also NaN
          }
          s0v = F::mma(ah0, bh, z4);
          s1v = F::mma(ah1, bh, z4);
        } else {
          bf16x8_t bh, bl;
#pragma unroll
          for (int e = 0; e < 8; ++e) {
            const __bf16 h = (__bf16)vv[e];
            bh[e] = h;
            bl[e] = (__bf16)(vv[e] - (float)h);
          }
          s0v = F::mma(ah0, bh, z4) + (F::mma(al0, bh, z4) + F::mma(ah0, bl, z4));
          s1v = F::mma(ah1, bh, z4) + (F::mma(al1, bh, z4) + F::mma(ah1, bl, z4));
        }
        const int gy = ci[CI_Y] - 5 + pi, gx = ci[CI_X] - 5 + pj;
        const bool in_img = cone && gy >= 0 && gy < H && gx >= 0 && gx < W;
        float v[2][4];
#pragma unroll
        for (int ii = 0; ii < 4; ++ii) {
          v[0][ii] = in_img ? fmaxf(s0v[ii] + bb0[ii], 0.f) : 0.f;
          v[1][ii] = in_img ? fmaxf(s1v[ii] + bb1[ii], 0.f) : 0.f;
        }
        if (P < 121) cone_store<HALF>(sm.b1[sl], p, g, v, ovf);
      }
      if (HALF && ovf) sm.covf[i & 15] = 1;
    }
    // ---- stages 2..5: the owned layer on cone t - K
    if (K) {
      const int i = t - K;
      if (i >= 0 && i < nloc) {
        const int sl = i & 1;
        const int* ci = sm.cinfo[i & 15];
        const bf16x8_t* wl = &sm.wlo[0][0][0][0];
        constexpr int LS = HALF ? 0 : 9 * 2 * 64;  // lo fragments per layer
        bool ovf;
        switch (K) {
          case 2:
            ovf = cone_layer<HALF, 2, 2>(wh, wl, bias, sm.b1[sl], sm.b2[sl], nullptr, ci, run0,
                                         lane);
            break;
          case 3:
            ovf = cone_layer<HALF, 3, 2>(wh, wl + LS, bias, sm.b2[sl], sm.b3[sl], nullptr, ci,
                                         run0, lane);
            break;
          case 4:
            ovf = cone_layer<HALF, 4, 2>(wh, wl + 2 * LS, bias, sm.b3[sl], sm.b4[sl], nullptr, ci,
                                         run0, lane);
            break;
          default:
            ovf = cone_layer<HALF, 5, 1>(wh, wl + 3 * LS, bias, sm.b4[sl], nullptr, sm.l5[sl], ci,
                                         run0, lane);
            break;
        }
        if (HALF && ovf) sm.covf[i & 15] = 1;
      }
    }
    // ---- stage 6 (wave 3): layer 6 in FP32 and the decision
    if (wave == 3 && t >= 6 && t - 6 < nloc) {
      const int i = t - 6;
      const int* ci = sm.cinfo[i & 15];
      const int o = ci[CI_O];
      if (o >= 0) {
        const float* l5 = sm.l5[i & 1];
        float part = 0.f;
#pragma unroll
        for (int k = 0; k < 5; ++k) {
          const int j = lane + 64 * k;
          if (j < 288) part = fmaf(sm.w6[j], l5[(j % 9) * 32 + j / 9], part);
        }
        part = hs_wave_sum(part);
        if (lane == 0) {
          const float xl = part + b6;
          float dist;
          int side;
          const int nb = hs::level_of(a.lv, xl, &dist, &side);
          const bool trusted = !HALF || (!wbad && sm.covf[i & 15] == 0);
          if (trusted && dist >= a.tau2) {
            // the level decided before: the side of the same nearest threshold
            const int old = hs::nearest_threshold(a.lv, xl) + ci[CI_BIT];
            if (old != nb) atomicAdd(&a.stats[1], 1);
            a.bits[o] = (uint8_t)nb;
            if (a.logits) a.logits[o] = xl;
          } else {
            a.list2[atomicAdd(a.count2, 1)] = (uint64_t)(uint32_t)o |
                                              ((uint64_t)(uint32_t)ci[CI_PG] << 31) |
                                              ((uint64_t)ci[CI_BIT] << 63);
          }
        }
      }
    }
    hs_lds_barrier();
  }
}

// ===========================================================================
// FP32 stage: one workgroup per listed pixel (grid-stride over the list,
// whose length is read on the device). Layer k's window outputs are
// register-blocked: thread (cg, pg) computes channels 4cg..4cg+3 of the
// window positions pg, pg + 32, ..., so each weight quad read from LDS
// feeds several positions and each activation read feeds four channels.
// The next layer's weights are loaded into registers while a layer computes.
// ===========================================================================
constexpr int RS = 33;  // padded channel stride of a staged position (floats)
constexpr int F32_THREADS = 256;
constexpr int F32_LAYER = 9 * 32 * 32;                // weights of one 32 -> 32 layer
constexpr int F32_VPT = F32_LAYER / 4 / F32_THREADS;  // 16-byte vectors per thread per layer

// element i of layers 2..5 as [layer][tap][ci][co] FP32, so a thread's four
// output channels are one 16-byte read
HS_DEV void pack_fp32_elem(const float* __restrict__ w, float* __restrict__ out, int i) {
  const int layer = i / F32_LAYER, rem = i - layer * F32_LAYER;
  const int t = rem / 1024, ci = (rem >> 5) & 31, co = rem & 31;
  out[i] = w[hs_wk(layer + 2) + (co * 32 + ci) * 9 + t];
}

// the weight copies of the recheck stages in one launch: split hi and lo,
// FP16, FP32 transposed; *wflag (zeroed before) set if a weight of layers
// 1..5 rounds to infinity in FP16
__global__ void pack_recheck_kernel(const float* __restrict__ w, __bf16* __restrict__ hi,
                                    __bf16* __restrict__ lo, _Float16* __restrict__ h16,
                                    float* __restrict__ wt, int* __restrict__ wflag) {
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < SPLIT_ELEMS + 4 * F32_LAYER;
       i += gridDim.x * blockDim.x) {
    if (i < SPLIT_ELEMS) {
      const float v = cone_weight(w, i);
      const __bf16 h = (__bf16)v;
      hi[i] = h;
      lo[i] = (__bf16)(v - (float)h);
      h16[i] = (_Float16)v;
    } else {
      pack_fp32_elem(w, wt, i - SPLIT_ELEMS);
    }
  }
  bool bad = false;
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < HS_W6; i += gridDim.x * blockDim.x)
    bad = bad || !(fabsf(w[i]) < F16_INF_AT);
  if (bad) atomicOr(wflag, 1);
}

template <int K>
HS_DEV void fp32_layer(const float* __restrict__ src, float* __restrict__ dst,
                       const float* __restrict__ sw, const float* __restrict__ sb, int y, int x,
                       int H, int W, int tid) {
  constexpr int EO = win_edge(K), EI = EO + 2, NP = EO * EO, J = (NP + 31) / 32;
  const int cg = tid & 7, pg = tid >> 3;
  int q0[J];
  float acc[J][4];
#pragma unroll
  for (int j = 0; j < J; ++j) {
    const int p = pg + 32 * j < NP ? pg + 32 * j : 0;
    q0[j] = (p / EO) * EI + p % EO;
#pragma unroll
    for (int i = 0; i < 4; ++i) acc[j][i] = sb[4 * cg + i];
  }
#pragma unroll 1
  for (int t = 0; t < 9; ++t) {
    const int dq = (t / 3) * EI + t % 3;
#pragma unroll 4
    for (int ci = 0; ci < 32; ++ci) {
      const f32x4_t wv = *(const f32x4_t*)(sw + (t * 32 + ci) * 32 + 4 * cg);
#pragma unroll
      for (int j = 0; j < J; ++j) {
        const float av = src[(q0[j] + dq) * RS + ci];
#pragma unroll
        for (int i = 0; i < 4; ++i) acc[j][i] = fmaf(wv[i], av, acc[j][i]);
      }
    }
  }
#pragma unroll
  for (int j = 0; j < J; ++j) {
    const int p = pg + 32 * j;
    if (p < NP) {
      const int gy = y - (6 - K) + p / EO, gx = x - (6 - K) + p % EO;
      const bool in = gy >= 0 && gy < H && gx >= 0 && gx < W;
#pragma unroll
      for (int i = 0; i < 4; ++i) dst[p * RS + 4 * cg + i] = in ? fmaxf(acc[j][i], 0.f) : 0.f;
    }
  }
}

__global__ __launch_bounds__(F32_THREADS, 2) void recheck_fp32_kernel(
    const float* __restrict__ w, const float* __restrict__ contone,
    const uint64_t* __restrict__ seeds, const hs::Page* __restrict__ pages, int kind,
    const uint64_t* __restrict__ list, const int* __restrict__ count,
    const f32x4_t* __restrict__ wt, const hs::Levels lv, uint8_t* __restrict__ bits,
    float* __restrict__ logits, int32_t* __restrict__ stats, int count_slot) {
  __shared__ float s0[13 * 13 * 2];
  __shared__ float bufA[11 * 11 * RS], bufB[9 * 9 * RS];
  __shared__ __attribute__((aligned(16))) float sw[F32_LAYER];  // [t][ci][co]
  __shared__ float sb[32];
  __shared__ float w1[32 * 2 * 9 + 32];
  const int n = *count;
  const int tid = threadIdx.x;
  if (blockIdx.x == 0 && tid == 0) stats[count_slot] = n;
  // the next layer's weights travel in registers while a layer computes
  f32x4_t pw[F32_VPT];
  auto fetch = [&](int k) {
#pragma unroll
    for (int j = 0; j < F32_VPT; ++j) pw[j] = wt[(k - 2) * (F32_LAYER / 4) + tid + F32_THREADS * j];
  };
  auto commit = [&]() {
#pragma unroll
    for (int j = 0; j < F32_VPT; ++j) ((f32x4_t*)sw)[tid + F32_THREADS * j] = pw[j];
  };
  for (int it = blockIdx.x; it < n; it += gridDim.x) {
    const uint64_t u = list[it];
    const uint32_t o = hs::entry_pixel(u);
    const int page = hs::entry_page(u);
    const hs::Page P = pages[page];
    const int H = P.H, W = P.W;
    const int rem = (int)(o - P.off), y = rem / W, x = rem - (rem / W) * W;
    const size_t img = (size_t)P.off;
    const uint64_t seed = seeds[page];
    fetch(2);
    __syncthreads();
    for (int i = tid; i < 169; i += F32_THREADS) {
      const int gy = y - 6 + i / 13, gx = x - 6 + i % 13;
      float cv = 0.f, zv = 0.f;
      if (gy >= 0 && gy < H && gx >= 0 && gx < W) {
        const uint64_t a = (uint64_t)gy * W + gx;
        cv = contone[img + a];
        zv = hs_noise<true>(seed, a, 0u, kind);
      }
      s0[i * 2] = cv;
      s0[i * 2 + 1] = zv;
    }
    for (int i = tid; i < 32 * 2 * 9 + 32; i += F32_THREADS) w1[i] = w[HS_W1 + i];
    __syncthreads();
    // layer 1 on the 11 x 11 window
    for (int i = tid; i < 121 * 32; i += F32_THREADS) {
      const int co = i & 31, p = i >> 5, py = p / 11, px = p % 11;
      const int gy = y - 5 + py, gx = x - 5 + px;
      float acc = 0.f;
      if (gy >= 0 && gy < H && gx >= 0 && gx < W) {
        acc = w1[HS_B1 + co];
#pragma unroll
        for (int t = 0; t < 9; ++t) {
          const int q = (py + t / 3) * 13 + px + t % 3;
          acc = fmaf(w1[(co * 2) * 9 + t], s0[q * 2], acc);
          acc = fmaf(w1[(co * 2 + 1) * 9 + t], s0[q * 2 + 1], acc);
        }
        acc = fmaxf(acc, 0.f);
      }
      bufA[p * RS + co] = acc;
    }
    // layers 2..5: bufA -> bufB -> bufA -> bufB -> bufA
    for (int k = 2; k <= 5; ++k) {
      __syncthreads();
      commit();
      if (tid < 32) sb[tid] = w[hs_bk(k) + tid];
      __syncthreads();
      if (k < 5) fetch(k + 1);
      switch (k) {
        case 2: fp32_layer<2>(bufA, bufB, sw, sb, y, x, H, W, tid); break;
        case 3: fp32_layer<3>(bufB, bufA, sw, sb, y, x, H, W, tid); break;
        case 4: fp32_layer<4>(bufA, bufB, sw, sb, y, x, H, W, tid); break;
        default: fp32_layer<5>(bufB, bufA, sw, sb, y, x, H, W, tid); break;
      }
    }
    __syncthreads();
    // layer 6 at the centre of the 3 x 3 window (in bufA)
    if (tid < 64) {
      float part = 0.f;
      for (int i = tid; i < 288; i += 64) {
        const int ci = i / 9, t = i % 9;
        part = fmaf(w[HS_W6 + i], bufA[t * RS + ci], part);
      }
      part = hs_wave_sum(part);
      if (tid == 0) {
        const float xl = part + w[HS_B6];
        float dist;
        int side;
        const int nb = hs::level_of(lv, xl, &dist, &side);
        if (nb != hs::nearest_threshold(lv, xl) + hs::entry_bit(u)) atomicAdd(&stats[1], 1);
        bits[o] = (uint8_t)nb;
        if (logits) logits[o] = xl;
      }
    }
  }
}

}  // namespace

namespace hs {

// bytes of the hi and the lo copy together (each 4 layers x 9 taps x 2 row
// tiles x 64 lanes x 8 BF16 values)
size_t split_frag_bytes() { return 2 * (size_t)SPLIT_ELEMS * sizeof(__bf16); }
size_t half_frag_bytes() { return (size_t)SPLIT_ELEMS * sizeof(_Float16); }
size_t fp32_pack_bytes() { return (size_t)4 * F32_LAYER * sizeof(float); }

hipError_t launch_split_pack(const float* w, const ConeWeights& cw, hipStream_t s) {
  pack_recheck_kernel<<<72, 256, 0, s>>>(w, (__bf16*)cw.whi, (__bf16*)cw.wlo, (_Float16*)cw.w16,
                                         (float*)cw.wt, cw.wflag);
  return hipGetLastError();
}

hipError_t launch_recheck_cones(bool half, const float* w, const float* contone,
                                const uint64_t* seeds, const Page* pages, int kind,
                                const uint64_t* seglist, const int* seg_count, int nseg,
                                long long seg_cap, const ConeWeights& cw, float band,
                                const Levels& lv, uint64_t* list_out, int* count_out,
                                uint8_t* bits, float* logits, int32_t* stats, int total_slot,
                                int num_cus, hipStream_t s) {
  if (nseg < 1 || nseg > SPLIT_MAXSEG) return hipErrorInvalidValue;
  SplitArgs a;
  a.w = w;
  a.contone = contone;
  a.seeds = seeds;
  a.pages = pages;
  a.kind = kind;
  a.nseg = nseg;
  a.seglist = seglist;
  a.seg_count = seg_count;
  a.seg_cap = seg_cap;
  a.whi = half ? cw.w16 : cw.whi;
  a.wlo = (const bf16x8_t*)cw.wlo;
  a.wflag = cw.wflag;
  a.tau2 = band;
  a.lv = lv;
  a.list2 = list_out;
  a.count2 = count_out;
  a.bits = bits;
  a.logits = logits;
  a.stats = stats;
  a.total_slot = total_slot;
  if (half) recheck_split_kernel<true><<<num_cus, SPLIT_THREADS, 0, s>>>(a);
  else recheck_split_kernel<false><<<num_cus, SPLIT_THREADS, 0, s>>>(a);
  return hipGetLastError();
}

hipError_t launch_recheck_fp32(const float* w, const float* contone, const uint64_t* seeds,
                               const Page* pages, int kind, const uint64_t* list,
                               const int* count, const void* wt, const Levels& lv, uint8_t* bits,
                               float* logits, int32_t* stats, int count_slot, int num_cus,
                               hipStream_t s) {
  recheck_fp32_kernel<<<2 * num_cus, F32_THREADS, 0, s>>>(w, contone, seeds, pages, kind, list,
                                                          count, (const f32x4_t*)wt, lv, bits,
                                                          logits, stats, count_slot);
  return hipGetLastError();
}

}  // namespace hs
