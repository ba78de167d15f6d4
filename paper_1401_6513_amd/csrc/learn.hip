// Learned start vector for the pressure Poisson solve: a small convolutional
// network on the lattice image of the node set, trained on the GPU on
// (residual, right-hand side) -> correction pairs captured from the solver's
// own steps.
//
// Network: 3x3 convolutions 3 -> 32 -> 32 -> 32 -> 1, ReLU after the first
// three, zero padding, NHWC images.  Inputs (per lattice pixel): the residual
// of the previous increment r = b - L phi_prev scaled by s = rms(r h^2) / h^2,
// the right-hand side scaled by its own rms, and the lattice mask; target:
// (phi - phi_prev) / (s h^2).  Weights and activations are BF16, every sum is
// FP32; the two 32 -> 32 layers (9 taps x 32 x 32 per pixel) run on MFMA
// (v_mfma_f32_16x16x32_bf16, one tap = one K step), the thin first and last
// layers as direct FP32 loops.  Training uses Adam on FP32 master weights.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <type_traits>
#include <vector>

#include "vip_internal.h"

namespace vip {

namespace {

typedef __attribute__((ext_vector_type(8))) __bf16 bf16x8;
typedef __attribute__((ext_vector_type(4))) float f32x4;
typedef unsigned short bf16_t;   // storage type of one bfloat16

constexpr int kC = 32;          // hidden channels
constexpr int kCin = 3;         // input channels
constexpr int kMargin = 4;      // receptive-field radius of the 4 layers (loss mask margin)

// Parameter offsets in the flat FP32 vector (same layout as the checker's):
// W1 [9][3][32], b1 [32], W2 [9][32][32], b2, W3 [9][32][32], b3, W4 [9][32], b4 [1]
constexpr int kW1 = 0, kB1 = kW1 + 9 * kCin * kC, kW2 = kB1 + kC, kB2 = kW2 + 9 * kC * kC,
              kW3 = kB2 + kC, kB3 = kW3 + 9 * kC * kC, kW4 = kB3 + kC, kB4 = kW4 + 9 * kC,
              kNParams = kB4 + 1;

__device__ __forceinline__ float bf2f(bf16_t v) { return __uint_as_float(static_cast<unsigned>(v) << 16); }

__device__ __forceinline__ bf16_t f2bf(float f) {   // round to nearest even
  unsigned u = __float_as_uint(f);
  if ((u & 0x7f800000u) == 0x7f800000u) return static_cast<bf16_t>(u >> 16);   // inf / nan
  u += 0x7fffu + ((u >> 16) & 1u);
  return static_cast<bf16_t>(u >> 16);
}

struct Img {
  int B, H, W;
};

__device__ __forceinline__ bool inside(const Img& g, int i, int j) {
  return i >= 0 && i < g.H && j >= 0 && j < g.W;
}

// ---- forward ------------------------------------------------------------------------------------

// two FP32 values to BF16 (round to nearest even) in one v_cvt_pk_bf16_f32, a in the low half
typedef __attribute__((ext_vector_type(2))) float f32x2;
typedef __attribute__((ext_vector_type(2))) __bf16 bf16x2;
__device__ __forceinline__ uint32_t pack_bf2(float a, float b) {
  const f32x2 v = {a, b};
  return __builtin_bit_cast(uint32_t, __builtin_convertvector(v, bf16x2));
}

// ReLU of a layer's four sums (the bias already in them, as the MFMA's initial accumulator),
// rounded to BF16 first: a BF16 value is negative exactly when its 16-bit pattern is a
// negative integer, so one packed integer max with 0 (v_pk_max_i16) per two values clears the
// negatives (and -0).  For finite sums this is bit for bit the BF16 rounding of the FP32 ReLU.
typedef short __attribute__((ext_vector_type(2))) s16x2;
__device__ __forceinline__ uint32_t relu_bf2(uint32_t w) {
  const s16x2 zero = {0, 0};
  return __builtin_bit_cast(uint32_t, __builtin_elementwise_max(__builtin_bit_cast(s16x2, w), zero));
}
__device__ __forceinline__ uint2 relu_pack4(const f32x4& d) {
  return make_uint2(relu_bf2(pack_bf2(d[0], d[1])), relu_bf2(pack_bf2(d[2], d[3])));
}

// Layer 1 (3 -> 32) as one MFMA K-step over the 9 taps and 3 channels (27 of the 32 K slots,
// the rest 0).  Slot k = 8 G + j: for G = 0, 1, 2 tap row dy = G, tap column dx = j / 3,
// channel j % 3 (j < 8); G = 3 holds tap column 2, channel 2 of the tap rows j = 0, 1, 2.  So
// each 8-slot group is one contiguous run of input values (three pixels' channels of one row,
// or the three left over), which the fused kernel reads with one load.  A = weights (16 output
// channels x 32 k for this lane's row), B = the pixel's 27 tap values (lane: the 8 slots of
// group l / 16 of pixel l % 16).  in(t, ci) returns the BF16 bits of tap t = 3 dy + dx,
// channel ci (0 outside the image).
__device__ __forceinline__ bool l1_slot(int k, int& t, int& ci) {
  const int G = k >> 3, j = k & 7;
  if (G < 3) {
    t = 3 * G + j / 3;
    ci = j % 3;
    return true;
  }
  t = 3 * j + 2;
  ci = 2;
  return j < 3;
}

__device__ __forceinline__ bf16x8 l1_weights(const bf16_t* w1, int m, int n, int kq) {
  uint32_t w[4] = {0u, 0u, 0u, 0u};
#pragma unroll
  for (int j = 0; j < 8; ++j) {
    int t = 0, ci = 0;
    const uint32_t v = l1_slot(kq + j, t, ci) ? w1[(t * kCin + ci) * kC + m * 16 + n] : 0u;
    w[j / 2] |= v << (16 * (j % 2));
  }
  return __builtin_bit_cast(bf16x8, make_uint4(w[0], w[1], w[2], w[3]));
}

template <class In>
__device__ __forceinline__ bf16x8 l1_operand(int kq, In&& in) {
  uint32_t w[4] = {0u, 0u, 0u, 0u};
#pragma unroll
  for (int j = 0; j < 8; ++j) {
    int t = 0, ci = 0;
    const uint32_t v = l1_slot(kq + j, t, ci) ? static_cast<uint32_t>(in(t, ci)) : 0u;
    w[j / 2] |= v << (16 * (j % 2));
  }
  return __builtin_bit_cast(bf16x8, make_uint4(w[0], w[1], w[2], w[3]));
}

// Layer 4 (32 -> 1): one MFMA K-step per tap with only output row 0 of the A tile nonzero; lane
// l < 16 ends with the output of pixel l.
__device__ __forceinline__ bf16x8 l4_weights(const bf16_t* w4, int t, int n, int kq) {
  if (n != 0) return __builtin_bit_cast(bf16x8, make_uint4(0u, 0u, 0u, 0u));
  return __builtin_bit_cast(bf16x8, *reinterpret_cast<const uint4*>(w4 + t * kC + kq));
}

// 16-pixel strips of image rows handled by one wavefront each pass (layers 1, 2, 3 and 4)
constexpr int kStripsPerWave = 8;

// layer 1 (3 -> 32) on MFMA, strips of 16 pixels of one image row; lane l ends with 4
// consecutive output channels of pixel l % 16 per output-channel tile
__global__ __launch_bounds__(256) void k_conv_in(Img g, const bf16_t* x, const bf16_t* w1, const float* b1,
                                                 bf16_t* out, int64_t nstrips) {
  const int64_t wv = (blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x) / 64;
  const int64_t s0 = wv * kStripsPerWave;
  if (s0 >= nstrips) return;
  const int l = threadIdx.x & 63;
  const int kq = (l >> 4) * 8;
  const int n = l & 15;
  const int cq = (l >> 4) * 4;
  const bf16x8 wa0 = l1_weights(w1, 0, n, kq), wa1 = l1_weights(w1, 1, n, kq);
  const f32x4 bv0 = {b1[cq], b1[cq + 1], b1[cq + 2], b1[cq + 3]};
  const f32x4 bv1 = {b1[16 + cq], b1[16 + cq + 1], b1[16 + cq + 2], b1[16 + cq + 3]};
  const int strips_w = (g.W + 15) / 16;
  for (int64_t s = s0; s < s0 + kStripsPerWave && s < nstrips; ++s) {
    const int j0 = static_cast<int>(s % strips_w) * 16;
    const int i = static_cast<int>((s / strips_w) % g.H);
    const int b = static_cast<int>(s / (static_cast<int64_t>(strips_w) * g.H));
    const int j = j0 + n;
    const bf16x8 xb = l1_operand(kq, [&](int t, int ci) -> bf16_t {
      const int ii = i + t / 3 - 1, jj = j + t % 3 - 1;
      return inside(g, ii, jj) ? x[((static_cast<int64_t>(b) * g.H + ii) * g.W + jj) * kCin + ci] : bf16_t(0);
    });
    const f32x4 d0 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(wa0, xb, bv0, 0, 0, 0);
    const f32x4 d1 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(wa1, xb, bv1, 0, 0, 0);
    if (j < g.W) {
      bf16_t* op = out + ((static_cast<int64_t>(b) * g.H + i) * g.W + j) * kC + cq;
      *reinterpret_cast<uint2*>(op) = relu_pack4(d0);
      *reinterpret_cast<uint2*>(op + 16) = relu_pack4(d1);
    }
  }
}

// MFMA tile over 16 pixels of one image row: D[pixel][n] += sum_taps A_tap[pixel][k] B_tap[k][n]
// where A_tap reads `src` at the pixel shifted by sign*(tap offset) and B_tap = wt[tap][n][k].
// Lane l: A row l%16 (pixel j0 + l%16), K chunk (l/16)*8; D rows (l/16)*4 + r, column l%16.
__device__ __forceinline__ void mfma_strip(const Img& g, int b, int i, int j0, const bf16_t* src, int sign,
                                           const bf16_t* wt, f32x4& d0, f32x4& d1) {
  const int l = threadIdx.x & 63;
  const int kq = (l >> 4) * 8;
  const int n = l & 15;
  for (int t = 0; t < 9; ++t) {
    const int ii = i + sign * (t / 3 - 1), jj = j0 + n + sign * (t % 3 - 1);
    bf16x8 a;
    if (inside(g, ii, jj)) {
      const uint4 raw = *reinterpret_cast<const uint4*>(src + ((static_cast<int64_t>(b) * g.H + ii) * g.W + jj) * kC + kq);
      a = __builtin_bit_cast(bf16x8, raw);
    } else {
      a = __builtin_bit_cast(bf16x8, make_uint4(0u, 0u, 0u, 0u));
    }
    const uint4 w0 = *reinterpret_cast<const uint4*>(wt + (t * kC + n) * kC + kq);
    const uint4 w1 = *reinterpret_cast<const uint4*>(wt + (t * kC + 16 + n) * kC + kq);
    d0 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, __builtin_bit_cast(bf16x8, w0), d0, 0, 0, 0);
    d1 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, __builtin_bit_cast(bf16x8, w1), d1, 0, 0, 0);
  }
}

// layers 2 and 3 (32 -> 32) on MFMA, D[co][pixel] = sum over taps W_t[co][ci] x[pixel + d_t][ci]
// per 16-pixel strip: A = weights (16 output channels x 32 input channels of one tap, held in
// registers for the whole wave), B = activations (32 channels x 16 pixels, one 16-byte load
// per lane), two output-channel tiles.  Lane l ends with 4 consecutive output channels of
// pixel l % 16, stored as one 8-byte write per tile.
__global__ __launch_bounds__(256) void k_conv_mid(Img g, const bf16_t* x, const bf16_t* wt, const float* bias,
                                                  bf16_t* out, int64_t nstrips) {
  const int64_t wv = (blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x) / 64;
  const int64_t s0 = wv * kStripsPerWave;
  if (s0 >= nstrips) return;
  const int l = threadIdx.x & 63;
  const int kq = (l >> 4) * 8;
  const int n = l & 15;
  const int cq = (l >> 4) * 4;
  bf16x8 wa[9][2];
#pragma unroll
  for (int t = 0; t < 9; ++t)
#pragma unroll
    for (int m = 0; m < 2; ++m)
      wa[t][m] = __builtin_bit_cast(bf16x8, *reinterpret_cast<const uint4*>(wt + (t * kC + m * 16 + n) * kC + kq));
  const f32x4 bv0 = {bias[cq], bias[cq + 1], bias[cq + 2], bias[cq + 3]};
  const f32x4 bv1 = {bias[16 + cq], bias[16 + cq + 1], bias[16 + cq + 2], bias[16 + cq + 3]};
  const int strips_w = (g.W + 15) / 16;
  for (int64_t s = s0; s < s0 + kStripsPerWave && s < nstrips; ++s) {
    const int j0 = static_cast<int>(s % strips_w) * 16;
    const int i = static_cast<int>((s / strips_w) % g.H);
    const int b = static_cast<int>(s / (static_cast<int64_t>(strips_w) * g.H));
    f32x4 d0 = bv0, d1 = bv1;   // the bias is the accumulators' start
#pragma unroll
    for (int t = 0; t < 9; ++t) {
      const int ii = i + (t / 3 - 1), jj = j0 + n + (t % 3 - 1);
      uint4 raw = make_uint4(0u, 0u, 0u, 0u);
      if (inside(g, ii, jj))
        raw = *reinterpret_cast<const uint4*>(x + ((static_cast<int64_t>(b) * g.H + ii) * g.W + jj) * kC + kq);
      const bf16x8 xb = __builtin_bit_cast(bf16x8, raw);
      d0 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(wa[t][0], xb, d0, 0, 0, 0);
      d1 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(wa[t][1], xb, d1, 0, 0, 0);
    }
    const int j = j0 + n;
    if (j < g.W) {
      bf16_t* op = out + ((static_cast<int64_t>(b) * g.H + i) * g.W + j) * kC + cq;
      *reinterpret_cast<uint2*>(op) = relu_pack4(d0);
      *reinterpret_cast<uint2*>(op + 16) = relu_pack4(d1);
    }
  }
}

// layer 4 (32 -> 1) on MFMA, strips of 16 pixels of one image row
__global__ __launch_bounds__(256) void k_conv_out(Img g, const bf16_t* x, const bf16_t* w4, const float* b4,
                                                  float* y, int64_t nstrips) {
  const int64_t wv = (blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x) / 64;
  const int64_t s0 = wv * kStripsPerWave;
  if (s0 >= nstrips) return;
  const int l = threadIdx.x & 63;
  const int kq = (l >> 4) * 8;
  const int n = l & 15;
  bf16x8 wa[9];
#pragma unroll
  for (int t = 0; t < 9; ++t) wa[t] = l4_weights(w4, t, n, kq);
  const f32x4 bias = {b4[0], 0.f, 0.f, 0.f};   // output row 0 starts from the bias
  const int strips_w = (g.W + 15) / 16;
  for (int64_t s = s0; s < s0 + kStripsPerWave && s < nstrips; ++s) {
    const int j0 = static_cast<int>(s % strips_w) * 16;
    const int i = static_cast<int>((s / strips_w) % g.H);
    const int b = static_cast<int>(s / (static_cast<int64_t>(strips_w) * g.H));
    f32x4 d = bias;
#pragma unroll
    for (int t = 0; t < 9; ++t) {
      const int ii = i + (t / 3 - 1), jj = j0 + n + (t % 3 - 1);
      uint4 raw = make_uint4(0u, 0u, 0u, 0u);
      if (inside(g, ii, jj))
        raw = *reinterpret_cast<const uint4*>(x + ((static_cast<int64_t>(b) * g.H + ii) * g.W + jj) * kC + kq);
      d = __builtin_amdgcn_mfma_f32_16x16x32_bf16(wa[t], __builtin_bit_cast(bf16x8, raw), d, 0, 0, 0);
    }
    const int j = j0 + n;
    if (l < 16 && j < g.W) y[(static_cast<int64_t>(b) * g.H + i) * g.W + j] = d[0];
  }
}

// ---- fused inference ---------------------------------------------------------------------------------

// All four layers in one launch.  A block owns a strip of kSW output columns and th <= kMaxTH
// output rows and walks down it one row per step: at step k layer 1 computes its row k from
// the input staged in LDS, and each later layer takes one row of the layer below from a
// two-row ring in LDS, adds that row's three taps (one per horizontal shift) into each of the
// three output rows it feeds, and writes the row that is then complete into its own ring.  A
// row of activations is read from LDS once per consuming layer (three shifted loads), not
// once per tap, and only the strip's top and bottom margins are computed twice.  For every
// output pixel and channel the nine taps are still added in tap order starting from the
// layer's bias, with the layer-by-layer kernels' MFMA operands and the BF16 rounding of each
// layer's output, so the result has the same bits.  Pixels outside the image hold 0 after
// every layer.
//
// Columns: the output covers kSW = 58 columns from the strip origin ox, layer 3 the 60 from
// ox - 1, layer 2 the 62 from ox - 2, layer 1 the 64 from ox - 3 and the staged input the 66
// from ox - 4; every layer is four groups of 16 columns (one MFMA pixel block each), and a
// lane past its layer's width stores 0 (its bias is -inf, so the ReLU gives 0).
// Rows, for a strip of th output rows from oy: layer 1 has th + 6 rows from oy - 3 (row k at
// step k), layer 2 th + 4 from oy - 2, layer 3 th + 2 from oy - 1, the output th from oy.  A
// layer loads a row of the layer below into registers in the step after it was written and
// uses it in the next one: layer 2 uses layer-1 row i at step i + 2 (and completes its own
// row i - 2), layer 3 layer-2 row i at step i + 6, layer 4 layer-3 row i at step i + 10; the
// last output row is done at step th + 11.  Layer 1's row k is multiplied at the end of step
// k - 1 and written at the start of step k, which keeps its LDS reads, MFMA wait and epilogue
// off the end of the step.  Input row r (image row oy - 4 + r) is loaded from HBM at step
// r - 8 and written to LDS at step r - 7 (channel planes of a row apart, so that the 4 lane
// groups of one layer-1 load read distinct banks), well before layer 1 reads it at step r - 3.
// One barrier per step.
// Waves: 0-3 layer 2 and 4-7 layer 3 (column group wave % 4), 8-11 layers 1 and 4 of group
// wave - 8; wave w runs on SIMD w % 4, so every SIMD holds one of each (18 + 18 + 11 MFMA a
// step).  The step loop is unrolled six times so that the three accumulator rows rotate and
// the ring slots alternate by renaming instead of copies.
constexpr int kSW = 58;             // output columns per strip
constexpr int kRingPx = 68;         // ring row: 64 region columns + 2 read by the shifted loads, padded
constexpr int kInW = kSW + 8;       // staged input columns
constexpr int kInPlane = 80;        // LDS stride of one channel's columns in a staged row (the 4
                                    // planes one layer-1 load touches fall 8 banks apart or more)
constexpr int kInRow = kCin * kInPlane;   // one staged input row: 3 channel planes
constexpr int kMaxTH = 160;         // output rows per strip at most
constexpr int kPx = 40;             // LDS stride of one pixel's 32 channels (80 bytes: the 16-byte
                                    // reads of 16 consecutive pixels hit 64 distinct banks)
constexpr int kRingLen = kRingPx * kPx;
constexpr int kCnnBlock = 768;      // 12 wavefronts, 3 per SIMD
constexpr int kInPre = 7;           // input rows staged before the first step

template <int U>
using Step = std::integral_constant<int, U>;

__global__ __launch_bounds__(kCnnBlock) void k_cnn_fused(Img g, int th, const bf16_t* x, const bf16_t* w1,
                                                       const float* b1, const bf16_t* w2t, const float* b2,
                                                       const bf16_t* w3t, const float* b3, const bf16_t* w4,
                                                       const float* b4, float* y) {
  __shared__ bf16_t s_in[(kMaxTH + 8) * kInRow];
  __shared__ __attribute__((aligned(16))) bf16_t s_ring[3][2][kRingLen];   // layers 1, 2, 3
  const int tid = static_cast<int>(threadIdx.x);
  const int b = static_cast<int>(blockIdx.z);
  const int ox = static_cast<int>(blockIdx.x) * kSW, oy = static_cast<int>(blockIdx.y) * th;
  const int nin = th + 8;                             // staged input rows
  // input value tid of a staged row: column ox - 4 + tid / 3, channel tid % 3, kept at
  // sdst = channel plane + column in LDS
  const bool stager = tid < kInW * kCin;
  const int sq = tid / kCin, sci = tid - (tid / kCin) * kCin;
  const bool scol = stager && ox - 4 + sq >= 0 && ox - 4 + sq < g.W;
  const int sdst = sci * kInPlane + sq;
  const int soff = (ox - 4) * kCin + tid;             // offset of this value in its image row
  auto in_load = [&](int r) -> bf16_t {
    const int ii = oy - 4 + r;
    if (r >= nin || ii < 0 || ii >= g.H) return bf16_t(0);
    const bf16_t* row = x + (static_cast<int64_t>(b) * g.H + ii) * g.W * kCin;   // uniform
    return scol ? row[soff] : bf16_t(0);
  };
  {
    bf16_t v[kInPre];
#pragma unroll
    for (int r = 0; r < kInPre; ++r) v[r] = in_load(r);
    if (stager)
#pragma unroll
      for (int r = 0; r < kInPre; ++r) s_in[r * kInRow + sdst] = v[r];
    // ring columns 64..67 feed only discarded lanes; keep them finite
    for (int e = tid; e < 3 * 2 * 4 * kPx; e += kCnnBlock)
      (&s_ring[0][0][0])[(e / (4 * kPx)) * kRingLen + 64 * kPx + e % (4 * kPx)] = 0;
    // column kInW of every staged row's first plane is never staged: 0, read by layer 1's
    // empty K slots
    for (int r = tid; r < nin; r += kCnnBlock) s_in[r * kInRow + kInW] = 0;
  }
  bf16_t pend = in_load(kInPre);                      // row kInPre, written at step 0
  const int l = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);   // uniform: role branches are scalar
  const int kq = (l >> 4) * 8;
  const int n = l & 15;
  const int cq = (l >> 4) * 4;
  const int role = wave >> 2;        // 0: layer 2, 1: layer 3, 2: layers 1 and 4
  const int c = (wave & 3) * 16 + n; // this lane's column in its layer's region
  const int hal = 2 - role;          // region origin ox - hal, oy - hal (layers 2, 3, 4)
  // role 0 / 1: wa[t][m] = the layer's weights of tap t, output channels 16 m ..; role 2:
  // wa[t][0] = layer 4 (A row 0 only), wa[0][1], wa[1][1] = layer 1's two channel tiles.
  // bv: the bias of this lane's 8 channels (layer 2 or 3; layer 1 for role 2), the start of a
  // row's accumulators; -inf in a column outside the layer's region or the image, so that the
  // ReLU stores 0 there.  bv4: layer 4's start (row 0: its bias).
  bf16x8 wa[9][2];
  f32x4 bv[2];
  {
    const int jc = role < 2 ? ox - hal + c : ox - 3 + c;
    const bool colok = (role < 2 ? c < 62 - 2 * role : true) && jc >= 0 && jc < g.W;
    const float* bias = role == 0 ? b2 : role == 1 ? b3 : b1;
#pragma unroll
    for (int m = 0; m < 2; ++m)
#pragma unroll
      for (int r = 0; r < 4; ++r) bv[m][r] = colok ? bias[m * 16 + cq + r] : -INFINITY;
  }
  if (role < 2) {
    const bf16_t* wt = role == 0 ? w2t : w3t;
#pragma unroll
    for (int t = 0; t < 9; ++t)
#pragma unroll
      for (int m = 0; m < 2; ++m)
        wa[t][m] = __builtin_bit_cast(bf16x8, *reinterpret_cast<const uint4*>(wt + (t * kC + m * 16 + n) * kC + kq));
  } else {
#pragma unroll
    for (int t = 0; t < 9; ++t) {
      wa[t][0] = l4_weights(w4, t, n, kq);
      wa[t][1] = __builtin_bit_cast(bf16x8, make_uint4(0u, 0u, 0u, 0u));
    }
    wa[0][1] = l1_weights(w1, 0, n, kq);
    wa[1][1] = l1_weights(w1, 1, n, kq);
  }
  const f32x4 bv4 = {b4[0], 0.f, 0.f, 0.f};
  const bool ystore = l < 16 && c < kSW && ox + c < g.W;
  // layer 1: slot j of this lane's group is tap row dy, tap column dx, channel ci (l1_slot), at
  // goff[j] + row * kInRow in the staged input; the empty slots (k >= 27) read the row's zero
  // at column kInW, so the 8 values are the operand as loaded
  int goff[8];
#pragma unroll
  for (int j = 0; j < 8; ++j) {
    int t = 0, ci = 0;
    goff[j] = l1_slot(kq + j, t, ci) ? (t / 3) * kInRow + ci * kInPlane + c + t % 3 : kInW;
  }
  typedef unsigned short __attribute__((ext_vector_type(8))) u16x8;
  auto gather = [&](int row) -> bf16x8 {
    u16x8 h;
#pragma unroll
    for (int j = 0; j < 8; ++j) h[j] = s_in[goff[j] + row * kInRow];
    return __builtin_bit_cast(bf16x8, h);
  };
  const int lag = 2 + 4 * role;                       // step at which row 0 of the layer below is used
  const int nsrc = th + 6 - 2 * role;                 // rows of the layer below
  const bf16_t* srcp = &s_ring[role][0][0] + c * kPx + kq;            // role r reads layer r + 1
  bf16_t* dstp = &s_ring[role < 2 ? role + 1 : 0][0][0] + c * kPx + cq;   // role 2: layer 1's ring
  const f32x4 z = {0.f, 0.f, 0.f, 0.f};
  const bf16x8 zb = __builtin_bit_cast(bf16x8, make_uint4(0u, 0u, 0u, 0u));
  f32x4 aX[2] = {z, z}, aY[2] = {z, z}, aZ[2] = {z, z};
  bf16x8 bP[3] = {zb, zb, zb}, bQ[3] = {zb, zb, zb};
  // One step of each role.  F: accumulator of the row that starts now (row i of the layer),
  // M: row i - 1, L: row i - 2 (completed now); BC: this step's operands, BN: the next step's.
  // The slot parity of every ring access equals that of k (all lags are even), which the
  // unrolling makes a constant.  The roles run separate loops with the same barriers, so
  // that neither role's registers shape the other's.
  auto fetch = [&](auto u, int k, bf16x8 (&BN)[3]) __attribute__((always_inline)) {
    constexpr int par = decltype(u)::value & 1;
    const int ip = k - lag + 1;
    if (ip >= 0 && ip < nsrc) {
#pragma unroll
      for (int d = 0; d < 3; ++d)
        BN[d] = __builtin_bit_cast(bf16x8, *reinterpret_cast<const uint4*>(srcp + (1 - par) * kRingLen + d * kPx));
    }
  };
  // a completed row into this layer's ring slot; a row outside the image (only near the
  // image's top and bottom edges) is then overwritten with zeros
  auto store_row = [&](auto u, const f32x4& d0, const f32x4& d1, bool rowok) __attribute__((always_inline)) {
    constexpr int par = decltype(u)::value & 1;
    bf16_t* wp = dstp + par * kRingLen;
    *reinterpret_cast<uint2*>(wp) = relu_pack4(d0);
    *reinterpret_cast<uint2*>(wp + 16) = relu_pack4(d1);
    if (!rowok) {
      __builtin_amdgcn_sched_barrier(0);
      *reinterpret_cast<uint2*>(wp) = make_uint2(0u, 0u);
      *reinterpret_cast<uint2*>(wp + 16) = make_uint2(0u, 0u);
    }
  };
  auto step_mid = [&](auto u, int k, f32x4 (&F)[2], f32x4 (&M)[2], f32x4 (&L)[2], bf16x8 (&BC)[3],
                      bf16x8 (&BN)[3]) __attribute__((always_inline)) {
    const bf16_t nxt = in_load(k + kInPre + 1);
    fetch(u, k, BN);
    const int i = k - lag;
    if (i >= 0 && i < nsrc) {
#pragma unroll
      for (int d = 0; d < 3; ++d)
#pragma unroll
        for (int m = 0; m < 2; ++m) L[m] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(wa[6 + d][m], BC[d], L[m], 0, 0, 0);
      const int j = i - 2;             // the row completed now
      if (j >= 0) store_row(u, L[0], L[1], oy - hal + j >= 0 && oy - hal + j < g.H);
#pragma unroll
      for (int d = 0; d < 3; ++d)
#pragma unroll
        for (int m = 0; m < 2; ++m) {
          M[m] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(wa[3 + d][m], BC[d], M[m], 0, 0, 0);
          F[m] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(wa[d][m], BC[d], d == 0 ? bv[m] : F[m], 0, 0, 0);
        }
    }
    if (stager && k + kInPre < nin) s_in[(k + kInPre) * kInRow + sdst] = pend;
    pend = nxt;
    __syncthreads();
  };
  // layer 1's row k + 1 is multiplied at the end of step k (D0, D1) and stored at the start of
  // step k + 1, so that neither the MFMA queue nor the epilogue sits on the step's critical path
  auto step_edge = [&](auto u, int k, f32x4 (&F)[2], f32x4 (&M)[2], f32x4 (&L)[2], bf16x8 (&BC)[3],
                       bf16x8 (&BN)[3], f32x4& D0, f32x4& D1, f32x4& E0, f32x4& E1) __attribute__((always_inline)) {
    if (k < th + 6) store_row(u, D0, D1, oy - 3 + k >= 0 && oy - 3 + k < g.H);
    fetch(u, k, BN);
    const int i = k - lag;
    const bool live = i >= 0 && i < nsrc;
    const bf16x8 xn = gather(k + 1 < th + 6 ? k + 1 : th + 5);
    if (live) {
#pragma unroll
      for (int d = 0; d < 3; ++d) L[0] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(wa[6 + d][0], BC[d], L[0], 0, 0, 0);
      // layer 4: output row i - 2 is complete
      const int o = i - 2;
      if (o >= 0 && oy + o < g.H && ystore)
        y[(static_cast<int64_t>(b) * g.H + oy + o) * g.W + ox + c] = L[0][0];
#pragma unroll
      for (int d = 0; d < 3; ++d) {
        M[0] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(wa[3 + d][0], BC[d], M[0], 0, 0, 0);
        F[0] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(wa[d][0], BC[d], d == 0 ? bv4 : F[0], 0, 0, 0);
      }
    }
    E0 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(wa[0][1], xn, bv[0], 0, 0, 0);
    E1 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(wa[1][1], xn, bv[1], 0, 0, 0);
    __syncthreads();
  };
  __syncthreads();
  const int nsteps = th + 12;
  // accumulators (F, M, L) rotate (X, Y, Z) -> (Z, X, Y) -> (Y, Z, X); operands alternate P, Q
  if (role < 2) {
    for (int k0 = 0; k0 < nsteps; k0 += 6) {
      step_mid(Step<0>{}, k0, aX, aY, aZ, bP, bQ);
      if (k0 + 1 < nsteps) step_mid(Step<1>{}, k0 + 1, aZ, aX, aY, bQ, bP);
      if (k0 + 2 < nsteps) step_mid(Step<2>{}, k0 + 2, aY, aZ, aX, bP, bQ);
      if (k0 + 3 < nsteps) step_mid(Step<3>{}, k0 + 3, aX, aY, aZ, bQ, bP);
      if (k0 + 4 < nsteps) step_mid(Step<4>{}, k0 + 4, aZ, aX, aY, bP, bQ);
      if (k0 + 5 < nsteps) step_mid(Step<5>{}, k0 + 5, aY, aZ, aX, bQ, bP);
    }
  } else {
    const bf16x8 x0 = gather(0);
    f32x4 dP0 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(wa[0][1], x0, bv[0], 0, 0, 0);
    f32x4 dP1 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(wa[1][1], x0, bv[1], 0, 0, 0);
    f32x4 dQ0 = z, dQ1 = z;
    for (int k0 = 0; k0 < nsteps; k0 += 6) {
      step_edge(Step<0>{}, k0, aX, aY, aZ, bP, bQ, dP0, dP1, dQ0, dQ1);
      if (k0 + 1 < nsteps) step_edge(Step<1>{}, k0 + 1, aZ, aX, aY, bQ, bP, dQ0, dQ1, dP0, dP1);
      if (k0 + 2 < nsteps) step_edge(Step<2>{}, k0 + 2, aY, aZ, aX, bP, bQ, dP0, dP1, dQ0, dQ1);
      if (k0 + 3 < nsteps) step_edge(Step<3>{}, k0 + 3, aX, aY, aZ, bQ, bP, dQ0, dQ1, dP0, dP1);
      if (k0 + 4 < nsteps) step_edge(Step<4>{}, k0 + 4, aZ, aX, aY, bP, bQ, dP0, dP1, dQ0, dQ1);
      if (k0 + 5 < nsteps) step_edge(Step<5>{}, k0 + 5, aY, aZ, aX, bQ, bP, dQ0, dQ1, dP0, dP1);
    }
  }
}

// ---- loss -----------------------------------------------------------------------------------------

// block sums of mask and of mask * (y - t)^2
__global__ void k_loss_partial(int64_t np, const float* y, const float* t, const float* m, double* part) {
  __shared__ double s0[256], s1[256];
  double a = 0.0, c = 0.0;
  for (int64_t p = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x; p < np;
       p += static_cast<int64_t>(gridDim.x) * blockDim.x) {
    const double d = static_cast<double>(y[p]) - static_cast<double>(t[p]);
    a += static_cast<double>(m[p]) * d * d;
    c += m[p];
  }
  s0[threadIdx.x] = a;
  s1[threadIdx.x] = c;
  __syncthreads();
  for (int off = blockDim.x / 2; off > 0; off >>= 1) {
    if (static_cast<int>(threadIdx.x) < off) {
      s0[threadIdx.x] += s0[threadIdx.x + off];
      s1[threadIdx.x] += s1[threadIdx.x + off];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    part[2 * blockIdx.x] = s0[0];
    part[2 * blockIdx.x + 1] = s1[0];
  }
}

// loss = sum / count (fixed block order); out[0] = loss, out[1] = count
__global__ void k_loss_finish(int nb, const double* part, double* out) {
  if (threadIdx.x != 0) return;
  double a = 0.0, c = 0.0;
  for (int k = 0; k < nb; ++k) {
    a += part[2 * k];
    c += part[2 * k + 1];
  }
  out[0] = c > 0.0 ? a / c : 0.0;
  out[1] = c;
}

// dL/dy = 2 m (y - t) / count
__global__ void k_loss_grad(int64_t np, const float* y, const float* t, const float* m, const double* lc,
                            float* gy) {
  const int64_t p = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x;
  if (p >= np) return;
  const double c = lc[1] > 0.0 ? lc[1] : 1.0;
  gy[p] = static_cast<float>(2.0 * m[p] * (static_cast<double>(y[p]) - t[p]) / c);
}

// ---- backward ---------------------------------------------------------------------------------------

// dA3 = conv^T(gy, W4), times relu'(A3): one thread per pixel, BF16 output
__global__ void k_out_bwd(Img g, const float* gy, const bf16_t* w4, const bf16_t* a3, bf16_t* gz3) {
  const int64_t p = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x;
  const int64_t np = static_cast<int64_t>(g.B) * g.H * g.W;
  if (p >= np) return;
  const int j = static_cast<int>(p % g.W), i = static_cast<int>((p / g.W) % g.H);
  const int64_t b = p / (static_cast<int64_t>(g.H) * g.W);
  float acc[kC];
#pragma unroll
  for (int c = 0; c < kC; ++c) acc[c] = 0.0f;
  for (int t = 0; t < 9; ++t) {
    // output pixel q = p - d_t contributed to p through tap t
    const int ii = i - (t / 3 - 1), jj = j - (t % 3 - 1);
    if (!inside(g, ii, jj)) continue;
    const float gv = gy[(b * g.H + ii) * g.W + jj];
    const bf16_t* wp = w4 + t * kC;
#pragma unroll
    for (int c = 0; c < kC; ++c) acc[c] += gv * bf2f(wp[c]);
  }
  const bf16_t* ap = a3 + p * kC;
  bf16_t* op = gz3 + p * kC;
#pragma unroll
  for (int c = 0; c < kC; ++c) op[c] = f2bf(bf2f(ap[c]) > 0.0f ? acc[c] : 0.0f);
}

// dA_{l-1} = conv^T(gz_l, W_l) on MFMA, times relu'(A_{l-1}); wb = [tap][ci][co]
__global__ void k_mid_bwd(Img g, const bf16_t* gz, const bf16_t* wb, const bf16_t* aprev, bf16_t* gzprev,
                          int64_t nstrips) {
  const int64_t s = (blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x) / 64;
  if (s >= nstrips) return;
  const int strips_w = (g.W + 15) / 16;
  const int j0 = static_cast<int>(s % strips_w) * 16;
  const int i = static_cast<int>((s / strips_w) % g.H);
  const int b = static_cast<int>(s / (static_cast<int64_t>(strips_w) * g.H));
  f32x4 d0 = {0.f, 0.f, 0.f, 0.f}, d1 = {0.f, 0.f, 0.f, 0.f};
  mfma_strip(g, b, i, j0, gz, -1, wb, d0, d1);
  const int l = threadIdx.x & 63;
  const int n = l & 15;
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    const int j = j0 + (l >> 4) * 4 + r;
    if (j >= g.W) continue;
    const int64_t o = ((static_cast<int64_t>(b) * g.H + i) * g.W + j) * kC;
    gzprev[o + n] = f2bf(bf2f(aprev[o + n]) > 0.0f ? d0[r] : 0.0f);
    gzprev[o + 16 + n] = f2bf(bf2f(aprev[o + 16 + n]) > 0.0f ? d1[r] : 0.0f);
  }
}

// Weight gradient of a 32 -> 32 layer on MFMA: dW[tap][ci][co] = sum_p x[p + d_tap][ci] gz[p][co].
// One wave per chunk of pixels; M = ci (2 tiles), N = co (2 tiles), K = 32 pixels per step.
// Lane l: A row ci = mt*16 + l%16 over pixels kq..kq+7; B pixels kq..kq+7, column co = nt*16 + l%16.
__global__ __launch_bounds__(256) void k_mid_wgrad(Img g, const bf16_t* x, const bf16_t* gz,
                                                   int64_t chunk, float* part) {
  const int64_t wave = (blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x) / 64;
  const int64_t np = static_cast<int64_t>(g.B) * g.H * g.W;
  const int l = threadIdx.x & 63;
  const int kq = (l >> 4) * 8;
  const int n = l & 15;
  f32x4 acc[9][4];
#pragma unroll
  for (int t = 0; t < 9; ++t)
#pragma unroll
    for (int q = 0; q < 4; ++q) acc[t][q] = f32x4{0.f, 0.f, 0.f, 0.f};
  const int64_t p0 = wave * chunk;
  for (int64_t base = p0; base < p0 + chunk && base < np; base += 32) {
    // B operands (gz) for the 8 pixels of this lane, both co tiles
    bf16x8 bv[2];
    int pi[8], pj[8];
    int64_t pb[8];
    bool pv[8];
#pragma unroll
    for (int e = 0; e < 8; ++e) {
      const int64_t p = base + kq + e;
      pv[e] = p < np && p < p0 + chunk;
      const int64_t pp = pv[e] ? p : 0;
      pj[e] = static_cast<int>(pp % g.W);
      pi[e] = static_cast<int>((pp / g.W) % g.H);
      pb[e] = pp / (static_cast<int64_t>(g.H) * g.W);
    }
#pragma unroll
    for (int nt = 0; nt < 2; ++nt)
#pragma unroll
      for (int e = 0; e < 8; ++e) {
        const int64_t p = base + kq + e;
        const bf16_t v = pv[e] ? gz[p * kC + nt * 16 + n] : static_cast<bf16_t>(0);
        bv[nt][e] = __builtin_bit_cast(__bf16, v);
      }
#pragma unroll
    for (int t = 0; t < 9; ++t) {
      const int dy = t / 3 - 1, dx = t % 3 - 1;
#pragma unroll
      for (int mt = 0; mt < 2; ++mt) {
        bf16x8 av;
#pragma unroll
        for (int e = 0; e < 8; ++e) {
          const int ii = pi[e] + dy, jj = pj[e] + dx;
          bf16_t v = 0;
          if (pv[e] && inside(g, ii, jj))
            v = x[((pb[e] * g.H + ii) * g.W + jj) * kC + mt * 16 + n];
          av[e] = __builtin_bit_cast(__bf16, v);
        }
        acc[t][mt * 2 + 0] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av, bv[0], acc[t][mt * 2 + 0], 0, 0, 0);
        acc[t][mt * 2 + 1] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av, bv[1], acc[t][mt * 2 + 1], 0, 0, 0);
      }
    }
  }
  // D layout: lane l holds rows (l/16)*4 + r (ci within the tile), column l%16 (co within the tile)
  float* pw = part + wave * (9 * kC * kC);
#pragma unroll
  for (int t = 0; t < 9; ++t)
#pragma unroll
    for (int mt = 0; mt < 2; ++mt)
#pragma unroll
      for (int nt = 0; nt < 2; ++nt)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int ci = mt * 16 + (l >> 4) * 4 + r, co = nt * 16 + n;
          pw[(t * kC + ci) * kC + co] = acc[t][mt * 2 + nt][r];
        }
}

// Weight and bias gradients of a thin layer (cin -> cout, direct): thread k of the block owns
// parameter k (tap, ci, co) or bias co; each block sums over one chunk of pixels.
// x has cin channels (BF16), gz has cout channels (FP32 if gzf != null, else BF16).
__global__ void k_thin_wgrad(Img g, int cin, int cout, const bf16_t* x, const bf16_t* gzb, const float* gzf,
                             int64_t chunk, float* part) {
  const int k = threadIdx.x;
  const int nw = 9 * cin * cout, nparam = nw + cout;
  const int64_t np = static_cast<int64_t>(g.B) * g.H * g.W;
  if (k >= nparam) return;
  int t = 0, ci = 0, co;
  if (k < nw) {
    t = k / (cin * cout);
    ci = (k / cout) % cin;
    co = k % cout;
  } else {
    co = k - nw;
  }
  const int dy = t / 3 - 1, dx = t % 3 - 1;
  float acc = 0.0f;
  const int64_t p0 = blockIdx.x * chunk;
  for (int64_t p = p0; p < p0 + chunk && p < np; ++p) {
    const float gv = gzf ? gzf[p * cout + co] : bf2f(gzb[p * cout + co]);
    if (gv == 0.0f) continue;
    if (k >= nw) {
      acc += gv;
      continue;
    }
    const int j = static_cast<int>(p % g.W), i = static_cast<int>((p / g.W) % g.H);
    const int64_t b = p / (static_cast<int64_t>(g.H) * g.W);
    const int ii = i + dy, jj = j + dx;
    if (!inside(g, ii, jj)) continue;
    acc += bf2f(x[((b * g.H + ii) * g.W + jj) * cin + ci]) * gv;
  }
  part[blockIdx.x * static_cast<int64_t>(nparam) + k] = acc;
}

// bias gradient of a 32-channel BF16 gradient image: block partial sums per channel
__global__ void k_bias_grad(int64_t np, const bf16_t* gz, int64_t chunk, float* part) {
  const int c = threadIdx.x;
  if (c >= kC) return;
  float acc = 0.0f;
  const int64_t p0 = blockIdx.x * chunk;
  for (int64_t p = p0; p < p0 + chunk && p < np; ++p) acc += bf2f(gz[p * kC + c]);
  part[blockIdx.x * static_cast<int64_t>(kC) + c] = acc;
}

// grad[off + k] = sum over nb partial rows of part[row * stride + k], k < count (fixed order)
__global__ void k_sum_parts(const float* part, int nb, int stride, int count, float* grad, int off) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= count) return;
  double s = 0.0;
  for (int r = 0; r < nb; ++r) s += part[static_cast<int64_t>(r) * stride + k];
  grad[off + k] = static_cast<float>(s);
}

// ---- optimiser and weight packing ---------------------------------------------------------------------

__global__ void k_adam(int n, float* w, const float* g, float* m, float* v, float lr, float b1, float b2,
                       float eps, float c1, float c2) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= n) return;
  const float gk = g[k];
  const float mk = b1 * m[k] + (1.0f - b1) * gk;
  const float vk = b2 * v[k] + (1.0f - b2) * gk * gk;
  m[k] = mk;
  v[k] = vk;
  w[k] -= lr * (mk / c1) / (sqrtf(vk / c2) + eps);
}

// BF16 copies: W1 as [tap][ci][co]; W2, W3 as [tap][co][ci] (forward) and [tap][ci][co]
// (backward); W4 as [tap][ci]
__global__ void k_pack(const float* th, bf16_t* w1, bf16_t* w2f, bf16_t* w2b, bf16_t* w3f, bf16_t* w3b,
                       bf16_t* w4) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k < 9 * kCin * kC) w1[k] = f2bf(th[kW1 + k]);
  if (k < 9 * kC * kC) {
    const int t = k / (kC * kC), ci = (k / kC) % kC, co = k % kC;
    w2b[k] = f2bf(th[kW2 + k]);
    w3b[k] = f2bf(th[kW3 + k]);
    w2f[(t * kC + co) * kC + ci] = f2bf(th[kW2 + k]);
    w3f[(t * kC + co) * kC + ci] = f2bf(th[kW3 + k]);
  }
  if (k < 9 * kC) w4[k] = f2bf(th[kW4 + k]);
}

// ---- lattice raster ------------------------------------------------------------------------------------

// training crop `sample` of the batch from one snapshot image; loss mask = lattice node
// and at least `margin` pixels inside the crop
__global__ void k_make_crop(const bf16_t* sx, const float* st, int W, int H, int oy, int ox, int crop,
                            int sample, bf16_t* X, float* T, float* M, int margin) {
  const int64_t q = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x;
  if (q >= static_cast<int64_t>(crop) * crop) return;
  const int cy = static_cast<int>(q / crop), cx = static_cast<int>(q % crop);
  const int iy = oy + cy, ix = ox + cx;
  const int64_t o = static_cast<int64_t>(sample) * crop * crop + q;
  bf16_t v0 = 0, v1 = 0, v2 = 0;
  float tv = 0.0f;
  if (iy >= 0 && iy < H && ix >= 0 && ix < W) {
    const int64_t src = static_cast<int64_t>(iy) * W + ix;
    v0 = sx[3 * src];
    v1 = sx[3 * src + 1];
    v2 = sx[3 * src + 2];
    tv = st[src];
  }
  X[3 * o] = v0;
  X[3 * o + 1] = v1;
  X[3 * o + 2] = v2;
  T[o] = tv;
  const bool core = cy >= margin && cy < crop - margin && cx >= margin && cx < crop - margin;
  M[o] = (v2 != 0 && core) ? 1.0f : 0.0f;
}

// input image: channels r h^2 / s_r, b h^2 / s_b, lattice mask (s_r, s_b: rms of r h^2 and
// b h^2 over lattice nodes, in scal[0], scal[1])
__global__ void k_make_image(int64_t npix, const int32_t* node_of, const double* r, const double* b,
                             const double* scal, double h2, bf16_t* X) {
  const int64_t q = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x;
  if (q >= npix) return;
  const int32_t node = node_of[q];
  const bool in = node >= 0;
  const double sr = scal[0], sb = scal[1];
  X[q * 3 + 0] = f2bf(in && sr > 0.0 ? static_cast<float>(r[node] * h2 / sr) : 0.0f);
  X[q * 3 + 1] = f2bf(in && sb > 0.0 ? static_cast<float>(b[node] * h2 / sb) : 0.0f);
  X[q * 3 + 2] = f2bf(in ? 1.0f : 0.0f);
}

// training target image: (phi - phi_prev - e) h^2 / s_r
__global__ void k_make_target(int64_t npix, const int32_t* node_of, const double* phi, const double* phi_prev,
                              const double* e, const double* scal, double h2, float* T) {
  const int64_t q = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x;
  if (q >= npix) return;
  const int32_t node = node_of[q];
  const double sr = scal[0];
  T[q] = node >= 0 && sr > 0.0 ? static_cast<float>((phi[node] - phi_prev[node] - e[node]) * h2 / sr) : 0.0f;
}

// predicted correction: s_r y / h^2 at lattice nodes, 0 elsewhere
__global__ void k_direction(int64_t n, const int32_t* pix, const float* y, const double* scal, double h2,
                            double* d) {
  const int64_t i = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x;
  if (i >= n) return;
  const int32_t p = pix[i];
  const double sr = scal[0];
  d[i] = p >= 0 && sr > 0.0 ? sr / h2 * static_cast<double>(y[p]) : 0.0;
}

// e = phi - phi_prev
__global__ void k_diff(int64_t n, const double* phi, const double* phi_prev, double* e) {
  const int64_t i = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x;
  if (i >= n) return;
  e[i] = phi[i] - phi_prev[i];
}

__global__ void k_f2d(int64_t n, const float* a, double* b) {
  const int64_t i = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x;
  if (i >= n) return;
  b[i] = static_cast<double>(a[i]);
}

// x += alpha d + beta c (c may be null)
__global__ void k_add2(int64_t n, double* x, const double* d, const double* cv, double alpha, double beta) {
  const int64_t i = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x;
  if (i >= n) return;
  x[i] += alpha * d[i] + (cv ? beta * cv[i] : 0.0);
}

// block partials of the squared sums of a h^2 and c h^2 over lattice nodes and their count
__global__ void k_rms_part(int64_t n, const int32_t* pix, const double* a, const double* cv, double h2,
                           double* part) {
  __shared__ double s0[256], s1[256], s2[256];
  double x0 = 0.0, x1 = 0.0, x2 = 0.0;
  for (int64_t i = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x; i < n;
       i += static_cast<int64_t>(gridDim.x) * blockDim.x) {
    if (pix[i] < 0) continue;
    const double u = a[i] * h2, v = cv[i] * h2;
    x0 += u * u;
    x1 += v * v;
    x2 += 1.0;
  }
  s0[threadIdx.x] = x0;
  s1[threadIdx.x] = x1;
  s2[threadIdx.x] = x2;
  __syncthreads();
  for (int off = blockDim.x / 2; off > 0; off >>= 1) {
    if (static_cast<int>(threadIdx.x) < off) {
      s0[threadIdx.x] += s0[threadIdx.x + off];
      s1[threadIdx.x] += s1[threadIdx.x + off];
      s2[threadIdx.x] += s2[threadIdx.x + off];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    part[3 * blockIdx.x] = s0[0];
    part[3 * blockIdx.x + 1] = s1[0];
    part[3 * blockIdx.x + 2] = s2[0];
  }
}

// scal[0], scal[1] = the two rms values (fixed block order)
// Sums of NV values over nb block partials part[k * NV + a], in a fixed order (thread t adds
// blocks t, t + 256, ..., then a tree over the threads), valid in thread 0.  256 threads.
template <int NV>
__device__ __forceinline__ void sum_partials(int nb, const double* part, double (&tot)[NV]) {
  __shared__ double sh[NV][256];
  double acc[NV];
#pragma unroll
  for (int a = 0; a < NV; ++a) acc[a] = 0.0;
  for (int k = threadIdx.x; k < nb; k += 256)
#pragma unroll
    for (int a = 0; a < NV; ++a) acc[a] += part[NV * k + a];
#pragma unroll
  for (int a = 0; a < NV; ++a) sh[a][threadIdx.x] = acc[a];
  __syncthreads();
  for (int off = 128; off > 0; off >>= 1) {
    if (static_cast<int>(threadIdx.x) < off)
#pragma unroll
      for (int a = 0; a < NV; ++a) sh[a][threadIdx.x] += sh[a][threadIdx.x + off];
    __syncthreads();
  }
#pragma unroll
  for (int a = 0; a < NV; ++a) tot[a] = sh[a][0];
}

__global__ void k_rms_finish(int nb, const double* part, double* scal) {
  double t[3];
  sum_partials<3>(nb, part, t);
  if (threadIdx.x != 0) return;
  scal[0] = t[2] > 0.0 ? sqrt(t[0] / t[2]) : 0.0;
  scal[1] = t[2] > 0.0 ? sqrt(t[1] / t[2]) : 0.0;
}

// block partials of q1.q1, q1.q2, q2.q2, q1.r, q2.r, r.r (q2 may be null: its terms are 0)
__global__ void k_dots6_part(int64_t n, const double* q1, const double* q2, const double* r, double* part) {
  __shared__ double sh[6][256];
  double acc[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
  for (int64_t i = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x; i < n;
       i += static_cast<int64_t>(gridDim.x) * blockDim.x) {
    const double a = q1[i], c = q2 ? q2[i] : 0.0, rv = r[i];
    acc[0] += a * a;
    acc[1] += a * c;
    acc[2] += c * c;
    acc[3] += a * rv;
    acc[4] += c * rv;
    acc[5] += rv * rv;
  }
  for (int k = 0; k < 6; ++k) sh[k][threadIdx.x] = acc[k];
  __syncthreads();
  for (int off = blockDim.x / 2; off > 0; off >>= 1) {
    if (static_cast<int>(threadIdx.x) < off)
      for (int k = 0; k < 6; ++k) sh[k][threadIdx.x] += sh[k][threadIdx.x + off];
    __syncthreads();
  }
  if (threadIdx.x < 6) part[6 * blockIdx.x + threadIdx.x] = sh[threadIdx.x][0];
}

// block partials of the Gram matrix of three directions and their dots with r:
// q1.q1, q1.q2, q1.q3, q2.q2, q2.q3, q3.q3, q1.r, q2.r, q3.r, r.r (a null q gives zero terms)
__global__ void k_dots10_part(int64_t n, const double* q1, const double* q2, const double* q3, const double* r,
                              double* part) {
  __shared__ double sh[10][256];
  double acc[10] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
  for (int64_t i = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x; i < n;
       i += static_cast<int64_t>(gridDim.x) * blockDim.x) {
    const double a = q1[i], b = q2 ? q2[i] : 0.0, c = q3 ? q3[i] : 0.0, rv = r[i];
    acc[0] += a * a;
    acc[1] += a * b;
    acc[2] += a * c;
    acc[3] += b * b;
    acc[4] += b * c;
    acc[5] += c * c;
    acc[6] += a * rv;
    acc[7] += b * rv;
    acc[8] += c * rv;
    acc[9] += rv * rv;
  }
  for (int k = 0; k < 10; ++k) sh[k][threadIdx.x] = acc[k];
  __syncthreads();
  for (int off = blockDim.x / 2; off > 0; off >>= 1) {
    if (static_cast<int>(threadIdx.x) < off)
      for (int k = 0; k < 10; ++k) sh[k][threadIdx.x] += sh[k][threadIdx.x + off];
    __syncthreads();
  }
  if (threadIdx.x < 10) part[10 * blockIdx.x + threadIdx.x] = sh[threadIdx.x][0];
}

// scal[2 + k] = sum over blocks of dot k of k_dots10_part (fixed block order)
__global__ void k_dots10_finish(int nb, const double* part, double* scal) {
  double t[10];
  sum_partials<10>(nb, part, t);
  if (threadIdx.x < 10) scal[2 + threadIdx.x] = t[threadIdx.x];
}

// phi = phi_prev + a1 d1 + a2 d2 + a3 d3 (a null direction is skipped)
// The start-vector fit: minimise ||r - sum_k a_k q_k||_2 over the directions in use (e; the
// network's c; e - e_old) from the Gram sums s[2..11] (q1.q1, q1.q2, q1.q3, q2.q2, q2.q3,
// q3.q3, q1.r, q2.r, q3.r, r.r): normal equations by Gaussian elimination with partial
// pivoting; a direction whose pivot vanishes against its Gram diagonal is dropped and the
// system solved again without it.  The fit is accepted if it lowers the residual; out[0..2] =
// the coefficients (all 0 if not accepted), out[3] = the residual ratio.  One thread, on the
// device, so that the step does not wait for the host here; no contraction into FMAs, so the
// arithmetic is the plain sequence written.
__global__ void k_fit3(const double* s, int learned, int second, double* out) {
#pragma clang fp contract(off)
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  const double G[3][3] = {{s[2], s[3], s[4]}, {s[3], s[5], s[6]}, {s[4], s[6], s[7]}};
  const double g[3] = {s[8], s[9], s[10]};
  const double rr = s[11];
  bool use[3] = {s[2] > 0.0, learned && s[5] > 0.0, second && s[7] > 0.0};
  double coef[3] = {0.0, 0.0, 0.0};
  for (int attempt = 0; attempt < 3; ++attempt) {
    int idx[3] = {0, 0, 0}, m = 0;
    for (int k = 0; k < 3; ++k)
      if (use[k]) idx[m++] = k;
    coef[0] = coef[1] = coef[2] = 0.0;
    if (m == 0) break;
    double A[3][4];
    for (int a = 0; a < m; ++a) {
      for (int b2 = 0; b2 < m; ++b2) A[a][b2] = G[idx[a]][idx[b2]];
      A[a][m] = g[idx[a]];
    }
    int bad = -1;
    for (int col = 0; col < m && bad < 0; ++col) {
      int piv = col;
      for (int r2 = col + 1; r2 < m; ++r2)
        if (fabs(A[r2][col]) > fabs(A[piv][col])) piv = r2;
      for (int k = 0; k <= m; ++k) {
        const double t = A[col][k];
        A[col][k] = A[piv][k];
        A[piv][k] = t;
      }
      if (!(fabs(A[col][col]) > 1e-10 * G[idx[col]][idx[col]])) {
        bad = col;
        break;
      }
      for (int r2 = col + 1; r2 < m; ++r2) {
        const double f = A[r2][col] / A[col][col];
        for (int k = col; k <= m; ++k) A[r2][k] -= f * A[col][k];
      }
    }
    if (bad >= 0) {   // drop the last direction in use (e stays) and solve again
      for (int k = 2; k >= 1; --k)
        if (use[k]) {
          use[k] = false;
          break;
        }
      if (m == 1) use[0] = false;
      continue;
    }
    double sol[3] = {0.0, 0.0, 0.0};
    for (int a = m - 1; a >= 0; --a) {
      double v = A[a][m];
      for (int k = a + 1; k < m; ++k) v -= A[a][k] * sol[k];
      sol[a] = v / A[a][a];
    }
    for (int a = 0; a < m; ++a) coef[idx[a]] = sol[a];
    break;
  }
  const double alpha = coef[0], beta = coef[1], gamma = coef[2];
  const double ratio2 = rr > 0.0 ? (rr - alpha * g[0] - beta * g[1] - gamma * g[2]) / rr : 1.0;
  const double ratio = sqrt(fmax(ratio2, 0.0));
  const bool accept = isfinite(alpha) && isfinite(beta) && isfinite(gamma) && isfinite(ratio) && ratio < 1.0 &&
                      (alpha != 0.0 || beta != 0.0 || gamma != 0.0);
  out[0] = accept ? alpha : 0.0;
  out[1] = accept ? beta : 0.0;
  out[2] = accept ? gamma : 0.0;
  out[3] = ratio;
}

// phi = phi_prev + a1 d1 + a2 d2 + a3 d3 with the coefficients of k_fit3 (a term whose
// coefficient is 0 is left out; all 0: the fit was not accepted and phi stays)
__global__ void k_combine3(int64_t n, const double* phi_prev, const double* d1, const double* d2, const double* d3,
                           const double* a, double* phi) {
  const int64_t i = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x;
  const double a1 = a[0], a2 = a[1], a3 = a[2];
  if (i >= n || (a1 == 0.0 && a2 == 0.0 && a3 == 0.0)) return;
  phi[i] = phi_prev[i] + a1 * d1[i] + (d2 && a2 != 0.0 ? a2 * d2[i] : 0.0) + (d3 && a3 != 0.0 ? a3 * d3[i] : 0.0);
}

// scal[2 + k] = sum over blocks of dot k (fixed block order)
__global__ void k_dots6_finish(int nb, const double* part, double* scal) {
  double t[6];
  sum_partials<6>(nb, part, t);
  if (threadIdx.x < 6) scal[2 + threadIdx.x] = t[threadIdx.x];
}

// splitmix64 (Steele, Lea and Flood 2014): a counter-based 64-bit generator
uint64_t splitmix64(uint64_t x) {
  x += 0x9E3779B97F4A7C15ull;
  x = (x ^ (x >> 30)) * 0xBF58476D1CE4E5B9ull;
  x = (x ^ (x >> 27)) * 0x94D049BB133111EBull;
  return x ^ (x >> 31);
}

constexpr int kSumBlocks = 256;
constexpr int kRedBlocks = 1024;   // blocks of the whole-node-set reductions (8 wavefronts per SIMD)

}  // namespace

// ---- host side -------------------------------------------------------------------------------------------

struct Net {
  float* theta = nullptr;     // FP32 master parameters [kNParams]
  float* grad = nullptr;
  float* m = nullptr;
  float* v = nullptr;
  bf16_t* w1 = nullptr;       // packed BF16 weights
  bf16_t* w2f = nullptr;
  bf16_t* w2b = nullptr;
  bf16_t* w3f = nullptr;
  bf16_t* w3b = nullptr;
  bf16_t* w4 = nullptr;
  int step = 0;
  bool ready = false;
  // activation and work buffers for up to `cap` pixels
  int64_t cap = 0;
  bf16_t *x = nullptr, *a1 = nullptr, *a2 = nullptr, *a3 = nullptr, *g3 = nullptr, *g2 = nullptr,
         *g1 = nullptr;
  float *y = nullptr, *t = nullptr, *mask = nullptr, *gy = nullptr, *part = nullptr;
  int64_t part_len = 0;
  double* dscal = nullptr;    // [0] loss, [1] mask count, then partials
  int64_t dscal_len = 0;
  // inference on a whole lattice image (fused kernel): input and output only
  bf16_t* ix = nullptr;
  float* iy = nullptr;
  int64_t icap = 0;
  int ncu = 0;                // compute units of the device (strip height of the fused inference)
};

void learn_clear(Ctx* c) {
  for (auto& s : c->learn.snaps) {
    dfree(s.x);
    dfree(s.t);
  }
  c->learn.snaps.clear();
}

void learn_free_nodeset(Ctx* c) {
  Learn& L = c->learn;
  L.fit_pending = false;
  for (double** p : {&L.r, &L.phi_prev, &L.eprev, &L.q1, &L.rx, &L.dir, &L.q2, &L.scal, &L.pc_r, &L.pc_d, &L.pc_c,
                     &L.pc_q1, &L.pc_q2, &L.pc_scal, &L.eprev2, &L.dir2, &L.q3})
    dfree(*p);
  L.have_eprev = false;
  L.have_eprev2 = false;
}

void learn_free(Ctx* c) {
  Learn& L = c->learn;
  if (L.fit_host) (void)hipHostFree(L.fit_host);
  if (L.fit_event) (void)hipEventDestroy(L.fit_event);
  L.fit_host = nullptr;
  L.fit_event = nullptr;
  L.fit_pending = false;
  if (L.net) {
    Net* N = static_cast<Net*>(L.net);
    for (float** p : {&N->theta, &N->grad, &N->m, &N->v, &N->y, &N->t, &N->mask, &N->gy, &N->part}) dfree(*p);
    for (bf16_t** p : {&N->w1, &N->w2f, &N->w2b, &N->w3f, &N->w3b, &N->w4, &N->x, &N->a1, &N->a2, &N->a3,
                       &N->g3, &N->g2, &N->g1, &N->ix})
      dfree(*p);
    dfree(N->iy);
    dfree(N->dscal);
    delete N;
    L.net = nullptr;
  }
  learn_clear(c);
  learn_free_nodeset(c);
}

bool learn_ready(const Ctx* c) {
  return c->learn.net && static_cast<const Net*>(c->learn.net)->ready;
}

namespace {

Net* net_of(Ctx* c) {
  if (!c->learn.net) c->learn.net = new Net();
  return static_cast<Net*>(c->learn.net);
}

int net_alloc(Ctx* c) {
  Net* N = net_of(c);
  if (N->theta) return VIP_OK;
  VIP_TRY(dalloc(c, &N->theta, kNParams));
  VIP_TRY(dalloc(c, &N->grad, kNParams));
  VIP_TRY(dalloc(c, &N->m, kNParams));
  VIP_TRY(dalloc(c, &N->v, kNParams));
  VIP_TRY(dalloc(c, &N->w1, 9 * kCin * kC));
  VIP_TRY(dalloc(c, &N->w2f, 9 * kC * kC));
  VIP_TRY(dalloc(c, &N->w2b, 9 * kC * kC));
  VIP_TRY(dalloc(c, &N->w3f, 9 * kC * kC));
  VIP_TRY(dalloc(c, &N->w3b, 9 * kC * kC));
  VIP_TRY(dalloc(c, &N->w4, 9 * kC));
  return VIP_OK;
}

int net_buffers(Ctx* c, int64_t npix) {
  Net* N = net_of(c);
  if (N->cap >= npix) return VIP_OK;
  VIP_HIP_TRY(c, hipStreamSynchronize(c->stream));
  for (bf16_t** p : {&N->x, &N->a1, &N->a2, &N->a3, &N->g3, &N->g2, &N->g1}) dfree(*p);
  for (float** p : {&N->y, &N->t, &N->mask, &N->gy}) dfree(*p);
  const int64_t cap = npix;
  VIP_TRY(dalloc(c, &N->x, cap * kCin));
  VIP_TRY(dalloc(c, &N->a1, cap * kC));
  VIP_TRY(dalloc(c, &N->a2, cap * kC));
  VIP_TRY(dalloc(c, &N->a3, cap * kC));
  VIP_TRY(dalloc(c, &N->g3, cap * kC));
  VIP_TRY(dalloc(c, &N->g2, cap * kC));
  VIP_TRY(dalloc(c, &N->g1, cap * kC));
  VIP_TRY(dalloc(c, &N->y, cap));
  VIP_TRY(dalloc(c, &N->t, cap));
  VIP_TRY(dalloc(c, &N->mask, cap));
  VIP_TRY(dalloc(c, &N->gy, cap));
  N->cap = npix;
  return VIP_OK;
}

int infer_buffers(Ctx* c, int64_t npix) {
  Net* N = net_of(c);
  if (N->icap >= npix) return VIP_OK;
  VIP_HIP_TRY(c, hipStreamSynchronize(c->stream));
  dfree(N->ix);
  dfree(N->iy);
  VIP_TRY(dalloc(c, &N->ix, npix * kCin));
  VIP_TRY(dalloc(c, &N->iy, npix));
  N->icap = npix;
  return VIP_OK;
}

int ensure_part(Ctx* c, int64_t floats, int64_t doubles) {
  Net* N = net_of(c);
  if (N->part_len < floats || N->dscal_len < doubles) VIP_HIP_TRY(c, hipStreamSynchronize(c->stream));
  if (N->part_len < floats) {
    dfree(N->part);
    VIP_TRY(dalloc(c, &N->part, floats));
    N->part_len = floats;
  }
  if (N->dscal_len < doubles) {
    dfree(N->dscal);
    VIP_TRY(dalloc(c, &N->dscal, doubles));
    N->dscal_len = doubles;
  }
  return VIP_OK;
}

int pack(Ctx* c) {
  Net* N = net_of(c);
  k_pack<<<(9 * kC * kC + kBlock - 1) / kBlock, kBlock, 0, c->stream>>>(N->theta, N->w1, N->w2f, N->w2b,
                                                                        N->w3f, N->w3b, N->w4);
  VIP_HIP_TRY(c, hipGetLastError());
  return VIP_OK;
}

int64_t blocks_for(int64_t items) { return (items + kBlock - 1) / kBlock; }

// forward pass over g (input already in N->x); prediction in N->y.  timed: HIP events around
// the two MFMA layers into c->conv_timing (harvested by the caller after a synchronisation).
int forward(Ctx* c, const Img& g, bool timed = false) {
  Net* N = net_of(c);
  hipStream_t st = c->stream;
  const int64_t nstrips = static_cast<int64_t>(g.B) * g.H * ((g.W + 15) / 16);
  const int64_t cwaves = (nstrips + kStripsPerWave - 1) / kStripsPerWave;
  const int64_t cblocks = blocks_for(cwaves * 64);
  timed = timed && c->conv_timing.enabled;
  k_conv_in<<<cblocks, kBlock, 0, st>>>(g, N->x, N->w1, N->theta + kB1, N->a1, nstrips);
  for (int layer = 0; layer < 2; ++layer) {
    std::pair<hipEvent_t, hipEvent_t> ev{};
    if (timed) {
      if (c->conv_timing.pool.empty()) {
        hipEvent_t a, b;
        VIP_HIP_TRY(c, hipEventCreateWithFlags(&a, hipEventDisableSystemFence));
        VIP_HIP_TRY(c, hipEventCreateWithFlags(&b, hipEventDisableSystemFence));
        c->conv_timing.pool.push_back({a, b});
      }
      ev = c->conv_timing.pool.back();
      c->conv_timing.pool.pop_back();
      VIP_HIP_TRY(c, hipEventRecord(ev.first, st));
    }
    if (layer == 0)
      k_conv_mid<<<cblocks, kBlock, 0, st>>>(g, N->a1, N->w2f, N->theta + kB2, N->a2, nstrips);
    else
      k_conv_mid<<<cblocks, kBlock, 0, st>>>(g, N->a2, N->w3f, N->theta + kB3, N->a3, nstrips);
    if (timed) {
      VIP_HIP_TRY(c, hipEventRecord(ev.second, st));
      c->conv_timing.pending.push_back(ev);
    }
  }
  k_conv_out<<<cblocks, kBlock, 0, st>>>(g, N->a3, N->w4, N->theta + kB4, N->y, nstrips);
  VIP_HIP_TRY(c, hipGetLastError());
  return VIP_OK;
}

// Output rows per strip of the fused inference.  A block takes th + 12 steps (the first and last
// are the layers' pipeline filling and draining) and runs alone on a CU, so the launch takes
// about ceil(blocks / CUs) x (th + 12) steps; the smallest such estimate wins.
int cnn_strip_rows(const Img& g, int ncu) {
  const int64_t strips = static_cast<int64_t>((g.W + kSW - 1) / kSW) * g.B;
  int best = 1;
  int64_t best_cost = INT64_MAX;
  for (int cand = 1; cand <= kMaxTH; ++cand) {
    const int th = std::min(cand, g.H);
    const int64_t blocks = strips * ((g.H + th - 1) / th);
    const int64_t cost = (blocks + ncu - 1) / ncu * (th + 12);
    if (cost < best_cost) {
      best_cost = cost;
      best = th;
    }
  }
  return best;
}

// inference over g in one launch (k_cnn_fused), input in N->ix, prediction in N->iy; timed: HIP
// events around the launch into c->conv_timing
int forward_fused(Ctx* c, const Img& g, bool timed) {
  Net* N = net_of(c);
  hipStream_t st = c->stream;
  timed = timed && c->conv_timing.enabled;
  std::pair<hipEvent_t, hipEvent_t> ev{};
  if (timed) {
    if (c->conv_timing.pool.empty()) {
      hipEvent_t a, b;
      VIP_HIP_TRY(c, hipEventCreateWithFlags(&a, hipEventDisableSystemFence));
      VIP_HIP_TRY(c, hipEventCreateWithFlags(&b, hipEventDisableSystemFence));
      c->conv_timing.pool.push_back({a, b});
    }
    ev = c->conv_timing.pool.back();
    c->conv_timing.pool.pop_back();
    VIP_HIP_TRY(c, hipEventRecord(ev.first, st));
  }
  if (N->ncu <= 0) {
    int ncu = 0;
    VIP_HIP_TRY(c, hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, c->device));
    N->ncu = std::max(ncu, 1);
  }
  const int th = cnn_strip_rows(g, N->ncu);
  if ((g.H + th - 1) / th > 65535)
    return set_error(c, VIP_E_INVALID, "image too tall for the fused inference (more than 65535 strips of rows)");
  const dim3 grid((g.W + kSW - 1) / kSW, (g.H + th - 1) / th, g.B);
  k_cnn_fused<<<grid, kCnnBlock, 0, st>>>(g, th, N->ix, N->w1, N->theta + kB1, N->w2f, N->theta + kB2,
                                       N->w3f, N->theta + kB3, N->w4, N->theta + kB4, N->iy);
  VIP_HIP_TRY(c, hipGetLastError());
  if (timed) {
    VIP_HIP_TRY(c, hipEventRecord(ev.second, st));
    c->conv_timing.pending.push_back(ev);
  }
  return VIP_OK;
}

// add the finished MFMA-layer timings (call after the stream has synchronised)
void harvest_conv_timing(Ctx* c) {
  Timing& T = c->conv_timing;
  for (auto& e : T.pending) {
    float ms = 0.0f;
    if (hipEventElapsedTime(&ms, e.first, e.second) == hipSuccess) {
      T.total_ms += ms;
      T.count += 1;
    }
    T.pool.push_back(e);
  }
  T.pending.clear();
}

// loss and gradient (targets and mask in N->t, N->mask); gradient in N->grad, loss in N->dscal[0]
int backward(Ctx* c, const Img& g) {
  Net* N = net_of(c);
  hipStream_t st = c->stream;
  const int64_t np = static_cast<int64_t>(g.B) * g.H * g.W;
  const int64_t nstrips = static_cast<int64_t>(g.B) * g.H * ((g.W + 15) / 16);
  const int64_t sblocks = blocks_for(nstrips * 64);
  const int lblocks = kSumBlocks;
  const int64_t thin_chunk = 128;        // pixels per block of the thin layers' gradients
  const int64_t thin_blocks = (np + thin_chunk - 1) / thin_chunk;
  const int64_t wave_chunk = 128;        // pixels per wave in the MFMA weight gradient
  const int64_t waves = (np + wave_chunk - 1) / wave_chunk;
  const int64_t wblocks = (waves * 64 + kBlock - 1) / kBlock;
  const int64_t mid_part = wblocks * 4 * 9 * kC * kC;
  const int64_t thin_part = thin_blocks * (9 * kCin * kC + kC);
  VIP_TRY(ensure_part(c, std::max(mid_part, thin_part), 2 + 2 * lblocks));
  k_loss_partial<<<lblocks, 256, 0, st>>>(np, N->y, N->t, N->mask, N->dscal + 2);
  k_loss_finish<<<1, 64, 0, st>>>(lblocks, N->dscal + 2, N->dscal);
  k_loss_grad<<<blocks_for(np), kBlock, 0, st>>>(np, N->y, N->t, N->mask, N->dscal, N->gy);
  // layer 4
  k_thin_wgrad<<<thin_blocks, 320, 0, st>>>(g, kC, 1, N->a3, nullptr, N->gy, thin_chunk, N->part);
  k_sum_parts<<<2, 256, 0, st>>>(N->part, static_cast<int>(thin_blocks), 9 * kC + 1, 9 * kC + 1, N->grad, kW4);
  k_out_bwd<<<blocks_for(np), kBlock, 0, st>>>(g, N->gy, N->w4, N->a3, N->g3);
  // layer 3
  k_mid_wgrad<<<wblocks, kBlock, 0, st>>>(g, N->a2, N->g3, wave_chunk, N->part);
  k_sum_parts<<<(9 * kC * kC + 255) / 256, 256, 0, st>>>(N->part, static_cast<int>(wblocks * 4), 9 * kC * kC,
                                                         9 * kC * kC, N->grad, kW3);
  k_bias_grad<<<thin_blocks, 64, 0, st>>>(np, N->g3, thin_chunk, N->part);
  k_sum_parts<<<1, 64, 0, st>>>(N->part, static_cast<int>(thin_blocks), kC, kC, N->grad, kB3);
  k_mid_bwd<<<sblocks, kBlock, 0, st>>>(g, N->g3, N->w3b, N->a2, N->g2, nstrips);
  // layer 2
  k_mid_wgrad<<<wblocks, kBlock, 0, st>>>(g, N->a1, N->g2, wave_chunk, N->part);
  k_sum_parts<<<(9 * kC * kC + 255) / 256, 256, 0, st>>>(N->part, static_cast<int>(wblocks * 4), 9 * kC * kC,
                                                         9 * kC * kC, N->grad, kW2);
  k_bias_grad<<<thin_blocks, 64, 0, st>>>(np, N->g2, thin_chunk, N->part);
  k_sum_parts<<<1, 64, 0, st>>>(N->part, static_cast<int>(thin_blocks), kC, kC, N->grad, kB2);
  k_mid_bwd<<<sblocks, kBlock, 0, st>>>(g, N->g2, N->w2b, N->a1, N->g1, nstrips);
  // layer 1
  k_thin_wgrad<<<thin_blocks, 9 * kCin * kC + kC, 0, st>>>(g, kCin, kC, N->x, N->g1, nullptr, thin_chunk,
                                                           N->part);
  k_sum_parts<<<(9 * kCin * kC + kC + 255) / 256, 256, 0, st>>>(N->part, static_cast<int>(thin_blocks),
                                                                9 * kCin * kC + kC, 9 * kCin * kC + kC, N->grad,
                                                                kW1);
  VIP_HIP_TRY(c, hipGetLastError());
  return VIP_OK;
}

int adam(Ctx* c, double lr) {
  Net* N = net_of(c);
  const float b1 = 0.9f, b2 = 0.999f, eps = 1e-8f;
  N->step += 1;
  const float c1 = static_cast<float>(1.0 - std::pow(0.9, N->step));
  const float c2 = static_cast<float>(1.0 - std::pow(0.999, N->step));
  k_adam<<<(kNParams + kBlock - 1) / kBlock, kBlock, 0, c->stream>>>(kNParams, N->theta, N->grad, N->m, N->v,
                                                                    static_cast<float>(lr), b1, b2, eps, c1, c2);
  VIP_HIP_TRY(c, hipGetLastError());
  return pack(c);
}

uint16_t host_bf16(double x) {
  const float f = static_cast<float>(x);
  uint32_t u;
  std::memcpy(&u, &f, 4);
  if ((u & 0x7f800000u) == 0x7f800000u) return static_cast<uint16_t>(u >> 16);
  u += 0x7fffu + ((u >> 16) & 1u);
  return static_cast<uint16_t>(u >> 16);
}

constexpr int kScalHead = 16;
constexpr int kScalFit = 12;   // scal[12..15]: the start-vector fit's coefficients and residual ratio

// rms of a h^2 and c h^2 over lattice nodes into scal[0], scal[1]
int lattice_rms(Ctx* c, const double* a, const double* cv) {
  Learn& L = c->learn;
  k_rms_part<<<kRedBlocks, 256, 0, c->stream>>>(c->n, c->lat.pix, a, cv, c->h * c->h, L.scal + kScalHead);
  k_rms_finish<<<1, 256, 0, c->stream>>>(kRedBlocks, L.scal + kScalHead, L.scal);
  VIP_HIP_TRY(c, hipGetLastError());
  return VIP_OK;
}

int ensure_vectors(Ctx* c) {
  Learn& L = c->learn;
  if (L.r) return VIP_OK;
  for (double** p : {&L.r, &L.phi_prev, &L.eprev, &L.q1, &L.rx, &L.dir, &L.q2, &L.pc_r, &L.pc_d, &L.pc_c,
                     &L.pc_q1, &L.pc_q2, &L.eprev2, &L.dir2, &L.q3})
    VIP_TRY(dalloc(c, p, c->n));
  VIP_TRY(dalloc(c, &L.scal, kScalHead + 10 * kRedBlocks));
  VIP_TRY(dalloc(c, &L.pc_scal, kScalHead + 6 * kRedBlocks));
  return VIP_OK;
}

// q1 = L eprev and rx = r - q1
int extrapolation_residual(Ctx* c) {
  Learn& L = c->learn;
  // q1 = L e and rx = r - q1 in one pass
  SysApply P;
  P.x = L.eprev;
  P.y = L.q1;
  P.b = L.r;
  P.r = L.rx;
  return pressure_apply(c, P);
}

}  // namespace

// ---- entry points used by api.hip and step.hip ----------------------------------------------------------------

int learn_n_params() { return kNParams; }

int learn_set_params(Ctx* c, const double* theta) {
  VIP_TRY(net_alloc(c));
  std::vector<float> h(kNParams);
  for (int k = 0; k < kNParams; ++k) {
    if (!std::isfinite(theta[k])) return set_error(c, VIP_E_INVALID, "non-finite network parameter");
    h[k] = static_cast<float>(theta[k]);
  }
  Net* N = net_of(c);
  VIP_HIP_TRY(c, hipMemcpyAsync(N->theta, h.data(), sizeof(float) * kNParams, hipMemcpyHostToDevice, c->stream));
  VIP_HIP_TRY(c, hipMemsetAsync(N->m, 0, sizeof(float) * kNParams, c->stream));
  VIP_HIP_TRY(c, hipMemsetAsync(N->v, 0, sizeof(float) * kNParams, c->stream));
  N->step = 0;
  VIP_TRY(pack(c));
  VIP_HIP_TRY(c, hipStreamSynchronize(c->stream));
  N->ready = true;
  return VIP_OK;
}

// He-uniform weights U(-sqrt(6/fan_in), sqrt(6/fan_in)) from splitmix64, zero biases
int learn_init(Ctx* c, uint64_t seed) {
  std::vector<double> th(kNParams, 0.0);
  const struct {
    int off, count, fan_in;
  } layers[4] = {{kW1, 9 * kCin * kC, 9 * kCin}, {kW2, 9 * kC * kC, 9 * kC}, {kW3, 9 * kC * kC, 9 * kC},
                 {kW4, 9 * kC, 9 * kC}};
  uint64_t ctr = seed * 0x9E3779B97F4A7C15ull;
  for (const auto& l : layers) {
    const double lim = std::sqrt(6.0 / l.fan_in);
    for (int k = 0; k < l.count; ++k) {
      const double u = static_cast<double>(splitmix64(ctr++) >> 11) * (1.0 / 9007199254740992.0);
      th[l.off + k] = (2.0 * u - 1.0) * lim;
    }
  }
  return learn_set_params(c, th.data());
}

int learn_get_params(Ctx* c, double* theta) {
  if (!learn_ready(c)) return set_error(c, VIP_E_NOT_BUILT, "network parameters not set");
  Net* N = net_of(c);
  std::vector<float> h(kNParams);
  VIP_HIP_TRY(c, hipMemcpyAsync(h.data(), N->theta, sizeof(float) * kNParams, hipMemcpyDeviceToHost, c->stream));
  VIP_HIP_TRY(c, hipStreamSynchronize(c->stream));
  for (int k = 0; k < kNParams; ++k) theta[k] = h[k];
  return VIP_OK;
}

// host images in, host results out; lr > 0 also takes one Adam step with the gradient
int learn_eval(Ctx* c, const double* x, const double* t, const double* m, int B, int H, int W, double* y,
               double* loss, double* grad, double lr) {
  if (!learn_ready(c)) return set_error(c, VIP_E_NOT_BUILT, "network parameters not set");
  if (B <= 0 || H <= 0 || W <= 0 || static_cast<int64_t>(B) * H * W > (int64_t{1} << 28))
    return set_error(c, VIP_E_INVALID, "image sizes must be positive and at most 2^28 pixels");
  if (!x) return set_error(c, VIP_E_INVALID, "input image is NULL");
  const bool need_bwd = grad || loss || lr > 0.0;
  if (need_bwd && (!t || !m)) return set_error(c, VIP_E_INVALID, "targets and mask are needed for the loss");
  Net* N = net_of(c);
  const int64_t np = static_cast<int64_t>(B) * H * W;
  VIP_TRY(net_buffers(c, np));
  hipStream_t st = c->stream;
  std::vector<uint16_t> hx(np * kCin);
  for (int64_t k = 0; k < np * kCin; ++k) hx[k] = host_bf16(x[k]);
  VIP_HIP_TRY(c, hipMemcpyAsync(N->x, hx.data(), sizeof(uint16_t) * np * kCin, hipMemcpyHostToDevice, st));
  const Img g{B, H, W};
  VIP_TRY(forward(c, g));
  std::vector<float> hy(np), ht, hm;
  VIP_HIP_TRY(c, hipMemcpyAsync(hy.data(), N->y, sizeof(float) * np, hipMemcpyDeviceToHost, st));
  double lc[2] = {0.0, 0.0};
  std::vector<float> hg;
  if (need_bwd) {
    ht.resize(np);
    hm.resize(np);
    for (int64_t k = 0; k < np; ++k) {
      ht[k] = static_cast<float>(t[k]);
      hm[k] = static_cast<float>(m[k]);
    }
    VIP_HIP_TRY(c, hipMemcpyAsync(N->t, ht.data(), sizeof(float) * np, hipMemcpyHostToDevice, st));
    VIP_HIP_TRY(c, hipMemcpyAsync(N->mask, hm.data(), sizeof(float) * np, hipMemcpyHostToDevice, st));
    VIP_TRY(backward(c, g));
    hg.resize(kNParams);
    VIP_HIP_TRY(c, hipMemcpyAsync(lc, N->dscal, sizeof(lc), hipMemcpyDeviceToHost, st));
    VIP_HIP_TRY(c, hipMemcpyAsync(hg.data(), N->grad, sizeof(float) * kNParams, hipMemcpyDeviceToHost, st));
    if (lr > 0.0) VIP_TRY(adam(c, lr));
  }
  VIP_HIP_TRY(c, hipStreamSynchronize(st));
  if (y)
    for (int64_t k = 0; k < np; ++k) y[k] = hy[k];
  if (loss) *loss = lc[0];
  if (grad)
    for (int k = 0; k < kNParams; ++k) grad[k] = hg[k];
  return VIP_OK;
}

// the fused inference launch that vip_step runs, on host images (checks and tools)
int learn_infer(Ctx* c, const double* x, int B, int H, int W, double* y) {
  if (!learn_ready(c)) return set_error(c, VIP_E_NOT_BUILT, "network parameters not set");
  if (B <= 0 || H <= 0 || W <= 0 || B > 65535 || static_cast<int64_t>(B) * H * W > (int64_t{1} << 28))
    return set_error(c, VIP_E_INVALID, "image sizes must be positive, batch at most 65535, at most 2^28 pixels");
  if (!x || !y) return set_error(c, VIP_E_INVALID, "input or output image is NULL");
  Net* N = net_of(c);
  const int64_t np = static_cast<int64_t>(B) * H * W;
  VIP_TRY(infer_buffers(c, np));
  hipStream_t st = c->stream;
  std::vector<uint16_t> hx(np * kCin);
  for (int64_t k = 0; k < np * kCin; ++k) hx[k] = host_bf16(x[k]);
  VIP_HIP_TRY(c, hipMemcpyAsync(N->ix, hx.data(), sizeof(uint16_t) * np * kCin, hipMemcpyHostToDevice, st));
  const Img g{B, H, W};
  VIP_TRY(forward_fused(c, g, true));
  std::vector<float> hy(np);
  VIP_HIP_TRY(c, hipMemcpyAsync(hy.data(), N->iy, sizeof(float) * np, hipMemcpyDeviceToHost, st));
  VIP_HIP_TRY(c, hipStreamSynchronize(st));
  harvest_conv_timing(c);
  for (int64_t k = 0; k < np; ++k) y[k] = hy[k];
  return VIP_OK;
}

// lattice image of the node set; the learned start vector needs one
static int learn_map(Ctx* c) {
  bool ok = false;
  VIP_TRY(lattice_map(c, &ok));
  if (!ok) return set_error(c, VIP_E_INVALID, "node set is not lattice based (image much larger than the node count)");
  return VIP_OK;
}

int learn_prepare(Ctx* c, const double* b, const double* phi, bool with_map) {
  Learn& L = c->learn;
  if (with_map) VIP_TRY(learn_map(c));
  VIP_TRY(ensure_vectors(c));
  // phi_prev = phi and r = b - L phi in one pass
  SysApply P;
  P.x = phi;
  P.cp = L.phi_prev;
  P.b = b;
  P.r = L.r;
  return pressure_apply(c, P);
}

int learn_warm_start(Ctx* c, int mode, const double* b, double* phi, vip_step_stats* stats) {
  Learn& L = c->learn;
  L.fit_pending = false;
  if (!L.have_eprev) return VIP_OK;   // no previous change yet: start from phi_prev
  hipStream_t st = c->stream;
  const double h2 = c->h * c->h;
  const bool learned = mode == VIP_WS_LEARNED;
  if (learned && !learn_ready(c))
    return set_error(c, VIP_E_NOT_BUILT, "learned start vector requested without network parameters");
  VIP_TRY(extrapolation_residual(c));
  if (learned) {
    Net* N = net_of(c);
    const int64_t npix = static_cast<int64_t>(c->lat.W) * c->lat.H;
    const Img g{1, c->lat.H, c->lat.W};
    VIP_TRY(lattice_rms(c, L.rx, b));
    const float* yv = nullptr;
    if (c->cnn_layered) {
      // layer-by-layer kernels (the training forward pass), for comparison
      VIP_TRY(net_buffers(c, npix));
      k_make_image<<<blocks_for(npix), kBlock, 0, st>>>(npix, c->lat.node_of, L.rx, b, L.scal, h2, N->x);
      VIP_TRY(forward(c, g, true));
      yv = N->y;
    } else {
      VIP_TRY(infer_buffers(c, npix));
      k_make_image<<<blocks_for(npix), kBlock, 0, st>>>(npix, c->lat.node_of, L.rx, b, L.scal, h2, N->ix);
      VIP_TRY(forward_fused(c, g, true));
      yv = N->iy;
    }
    k_direction<<<blocks_for(c->n), kBlock, 0, st>>>(c->n, c->lat.pix, yv, L.scal, h2, L.dir);
    VIP_TRY(pressure_apply(c, L.dir, L.q2));
  }
  // second difference of the increments, e - e_old (the quadratic extrapolation adds it)
  const bool second = L.have_eprev2;
  if (second) {
    // dir2 = e - e_old and q3 = L dir2 in one pass
    SysApply P;
    P.x = L.eprev;
    P.x2 = L.eprev2;
    P.xd = L.dir2;
    P.y = L.q3;
    VIP_TRY(pressure_apply(c, P));
  }
  k_dots10_part<<<kRedBlocks, 256, 0, st>>>(c->n, L.q1, learned ? L.q2 : nullptr, second ? L.q3 : nullptr, L.r,
                                            L.scal + kScalHead);
  k_dots10_finish<<<1, 256, 0, st>>>(kRedBlocks, L.scal + kScalHead, L.scal);
  k_fit3<<<1, 64, 0, st>>>(L.scal, learned ? 1 : 0, second ? 1 : 0, L.scal + kScalFit);
  k_combine3<<<blocks_for(c->n), kBlock, 0, st>>>(c->n, L.phi_prev, L.eprev, learned ? L.dir : nullptr,
                                                  second ? L.dir2 : nullptr, L.scal + kScalFit, phi);
  VIP_HIP_TRY(c, hipGetLastError());
  // the fit's outcome reaches the host with the pressure solve's first convergence check
  if (!L.fit_host) VIP_HIP_TRY(c, hipHostMalloc(reinterpret_cast<void**>(&L.fit_host), 4 * sizeof(double),
                                                hipHostMallocDefault));
  if (!L.fit_event) VIP_HIP_TRY(c, hipEventCreateWithFlags(&L.fit_event, hipEventDisableTiming));
  VIP_HIP_TRY(c, hipMemcpyAsync(L.fit_host, L.scal + kScalFit, 4 * sizeof(double), hipMemcpyDeviceToHost, st));
  VIP_HIP_TRY(c, hipEventRecord(L.fit_event, st));
  L.fit_pending = true;
  L.fit_mode = mode;
  (void)stats;
  return VIP_OK;
}

int learn_warm_stats(Ctx* c, vip_step_stats* stats) {
  Learn& L = c->learn;
  if (!L.fit_pending) return VIP_OK;
  L.fit_pending = false;
  VIP_HIP_TRY(c, hipEventSynchronize(L.fit_event));   // complete already after the solve's checks
  harvest_conv_timing(c);
  if (stats) {
    const double* f = L.fit_host;
    const bool accept = f[0] != 0.0 || f[1] != 0.0 || f[2] != 0.0;
    stats->warm_start = accept ? L.fit_mode : VIP_WS_PREV;
    stats->warm_ratio = f[3];
    stats->warm_alpha = f[0];
    stats->warm_beta = f[1];
    stats->warm_gamma = f[2];
  }
  return VIP_OK;
}

bool learn_precond_active(Ctx* c) {
  if (!c->opt.learned_precond || c->opt.warmstart != VIP_WS_LEARNED || c->opt.precision != VIP_P_MIXED) return false;
  if (c->singular || !learn_ready(c) || !c->lat.ok) return false;
  return true;
}

// One flexible refinement pass with the network as a second preconditioner: c = the network's
// correction of the pass residual r (the image of r h^2 / s, b h^2 / rms(b h^2) and the lattice
// mask, as for the start vector: the network approximates L^-1 on a residual), then
// x += alpha d + beta c with (alpha, beta) minimising ||r - alpha L d - beta L c||_2; if the
// network's direction does not beat the best multiple of d alone, x += d.
int learn_precond_pass(Ctx* c, const float* r32, const double* b, const float* d32, double* x, int* used,
                       double* gain) {
  Learn& L = c->learn;
  VIP_TRY(ensure_vectors(c));
  Net* N = net_of(c);
  hipStream_t st = c->stream;
  const int64_t n = c->n;
  const double h2 = c->h * c->h;
  const int64_t npix = static_cast<int64_t>(c->lat.W) * c->lat.H;
  const Img g{1, c->lat.H, c->lat.W};
  k_f2d<<<blocks_for(n), kBlock, 0, st>>>(n, r32, L.pc_r);
  k_f2d<<<blocks_for(n), kBlock, 0, st>>>(n, d32, L.pc_d);
  k_rms_part<<<kRedBlocks, 256, 0, st>>>(n, c->lat.pix, L.pc_r, b, h2, L.pc_scal + kScalHead);
  k_rms_finish<<<1, 256, 0, st>>>(kRedBlocks, L.pc_scal + kScalHead, L.pc_scal);
  VIP_TRY(infer_buffers(c, npix));
  k_make_image<<<blocks_for(npix), kBlock, 0, st>>>(npix, c->lat.node_of, L.pc_r, b, L.pc_scal, h2, N->ix);
  VIP_TRY(forward_fused(c, g, true));
  k_direction<<<blocks_for(n), kBlock, 0, st>>>(n, c->lat.pix, N->iy, L.pc_scal, h2, L.pc_c);
  VIP_TRY(pressure_apply(c, L.pc_d, L.pc_q1));
  VIP_TRY(pressure_apply(c, L.pc_c, L.pc_q2));
  k_dots6_part<<<kRedBlocks, 256, 0, st>>>(n, L.pc_q1, L.pc_q2, L.pc_r, L.pc_scal + kScalHead);
  k_dots6_finish<<<1, 256, 0, st>>>(kRedBlocks, L.pc_scal + kScalHead, L.pc_scal);
  VIP_HIP_TRY(c, hipGetLastError());
  double sv[8];
  VIP_HIP_TRY(c, hipMemcpyAsync(sv, L.pc_scal, sizeof(sv), hipMemcpyDeviceToHost, st));
  VIP_HIP_TRY(c, hipStreamSynchronize(st));
  harvest_conv_timing(c);
  const double a11 = sv[2], a12 = sv[3], a22 = sv[4], g1 = sv[5], g2 = sv[6], rr = sv[7];
  double alpha = 1.0, beta = 0.0;
  bool take = false;
  const double det = a11 * a22 - a12 * a12;
  if (a11 > 0.0 && a22 > 0.0 && rr > 0.0 && det > 1e-10 * a11 * a22) {
    const double al = (g1 * a22 - g2 * a12) / det, be = (a11 * g2 - a12 * g1) / det;
    const double r2 = (rr - al * g1 - be * g2) / rr;    // with the network's direction
    const double r1 = (rr - g1 * g1 / a11) / rr;         // best multiple of d alone
    if (std::isfinite(al) && std::isfinite(be) && r2 < r1 && r1 > 0.0) {
      alpha = al;
      beta = be;
      take = true;
      if (gain) *gain *= std::sqrt(std::max(r2, 0.0) / r1);
    }
  }
  if (take) {
    k_add2<<<blocks_for(n), kBlock, 0, st>>>(n, x, L.pc_d, L.pc_c, alpha, beta);
    if (used) ++*used;
  } else {
    k_add2<<<blocks_for(n), kBlock, 0, st>>>(n, x, L.pc_d, nullptr, 1.0, 0.0);
  }
  VIP_HIP_TRY(c, hipGetLastError());
  return VIP_OK;
}

int learn_finish(Ctx* c, const double* b, const double* phi, bool capture) {
  Learn& L = c->learn;
  hipStream_t st = c->stream;
  if (capture && L.have_eprev && static_cast<int>(L.snaps.size()) < L.capacity) {
    const int64_t npix = static_cast<int64_t>(c->lat.W) * c->lat.H;
    Snapshot s;
    s.W = c->lat.W;
    s.H = c->lat.H;
    VIP_TRY(dalloc(c, &s.x, 3 * npix));
    if (dalloc(c, &s.t, npix) != VIP_OK) {
      dfree(s.x);
      return VIP_E_HIP;
    }
    L.snaps.push_back(s);
    const double h2 = c->h * c->h;
    VIP_TRY(extrapolation_residual(c));
    VIP_TRY(lattice_rms(c, L.rx, b));
    k_make_image<<<blocks_for(npix), kBlock, 0, st>>>(npix, c->lat.node_of, L.rx, b, L.scal, h2, s.x);
    k_make_target<<<blocks_for(npix), kBlock, 0, st>>>(npix, c->lat.node_of, phi, L.phi_prev, L.eprev, L.scal, h2,
                                                       s.t);
  }
  if (L.have_eprev) {
    std::swap(L.eprev, L.eprev2);   // the change before (its buffer swapped in, no copy)
    L.have_eprev2 = true;
  }
  k_diff<<<blocks_for(c->n), kBlock, 0, st>>>(c->n, phi, L.phi_prev, L.eprev);
  VIP_HIP_TRY(c, hipGetLastError());
  L.have_eprev = true;
  return VIP_OK;
}

int learn_train(Ctx* c, int iters, int batch, int crop, double lr, uint64_t seed, double* last_loss) {
  Learn& L = c->learn;
  if (!learn_ready(c)) return set_error(c, VIP_E_NOT_BUILT, "network parameters not set");
  if (L.snaps.empty()) return set_error(c, VIP_E_INVALID, "no captured snapshots to train on");
  if (iters <= 0 || batch <= 0 || batch > 1024 || crop < 2 * kMargin + 4 || crop > 1024 || !(lr > 0.0))
    return set_error(c, VIP_E_INVALID, "bad training arguments");
  Net* N = net_of(c);
  const int64_t np = static_cast<int64_t>(batch) * crop * crop;
  VIP_TRY(net_buffers(c, np));
  hipStream_t st = c->stream;
  const Img g{batch, crop, crop};
  double loss = 0.0;
  for (int it = 0; it < iters; ++it) {
    for (int k = 0; k < batch; ++k) {
      const uint64_t key = splitmix64(seed) + (static_cast<uint64_t>(N->step) << 20) + static_cast<uint64_t>(k);
      const uint64_t r0 = splitmix64(3 * key), r1 = splitmix64(3 * key + 1), r2 = splitmix64(3 * key + 2);
      const Snapshot& s = L.snaps[r0 % L.snaps.size()];
      const int oy = static_cast<int>(r1 % static_cast<uint64_t>(std::max(1, s.H - crop + 1)));
      const int ox = static_cast<int>(r2 % static_cast<uint64_t>(std::max(1, s.W - crop + 1)));
      k_make_crop<<<blocks_for(static_cast<int64_t>(crop) * crop), kBlock, 0, st>>>(
          s.x, s.t, s.W, s.H, oy, ox, crop, k, N->x, N->t, N->mask, kMargin);
    }
    VIP_TRY(forward(c, g));
    VIP_TRY(backward(c, g));
    VIP_TRY(adam(c, lr));
    if (it == iters - 1 || (it + 1) % 50 == 0) {
      double lc[2];
      VIP_HIP_TRY(c, hipMemcpyAsync(lc, N->dscal, sizeof(lc), hipMemcpyDeviceToHost, st));
      VIP_HIP_TRY(c, hipStreamSynchronize(st));
      loss = lc[0];
      if (!std::isfinite(loss)) return set_error(c, VIP_E_NONFINITE, "training loss is not finite");
      if (c->debug) std::fprintf(stderr, "[vip] train iter %d loss %.4e\n", it + 1, loss);
    }
  }
  if (last_loss) *last_loss = loss;
  return VIP_OK;
}

}  // namespace vip
