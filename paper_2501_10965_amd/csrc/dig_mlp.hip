// Learned closure network on the CDNA4 matrix cores: forward, back-propagation
// and Adam for a 4-layer perceptron (9 -> 128 -> 128 -> 128 -> 7, padded to
// 32 inputs and 16 outputs, tanh hidden layers).  Products use gfx950's
// v_mfma_f32_16x16x32_bf16: BF16 operands, FP32 accumulation.  A workgroup of
// four waves carries a tile of 64 samples through all layers with the
// activations in LDS.  Inference runs a persistent grid whose waves keep
// their share of every weight matrix (88 VGPRs of BF16) in registers for the
// whole launch; training kernels read the BF16 weights from L2.
#include <math.h>
#include <string.h>

#include <string>

#include "dig_internal.h"

namespace dig {
namespace {

typedef short bf16x4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

constexpr int kIn = 32, kH = 128, kOutP = 16, kNIn = 9, kNOut = 7;
constexpr int kTile = 64;      // samples per workgroup
constexpr int kThreads = 256;  // four waves
constexpr int kLds = kH + 8;   // LDS row stride of an activation tile (bf16)
constexpr int kNW = 38912;     // weights (no biases)

// offsets of W_l and b_l in the FP32 parameter array, and of W_l in the BF16
// copies (forward [out][in] and transposed [in][out])
__host__ __device__ constexpr int pw(int l) { return l == 0 ? 0 : l == 1 ? 4224 : l == 2 ? 20736 : 37248; }
__host__ __device__ constexpr int pb(int l) { return l == 0 ? 4096 : l == 1 ? 20608 : l == 2 ? 37120 : 39296; }
__host__ __device__ constexpr int qw(int l) { return l == 0 ? 0 : l == 1 ? 4096 : l == 2 ? 20480 : 36864; }
__host__ __device__ constexpr int din(int l) { return l == 0 ? kIn : kH; }
__host__ __device__ constexpr int dout(int l) { return l == 3 ? kOutP : kH; }
static_assert(pb(3) + kOutP == DIG_MLP_NPARAM, "parameter layout");
static_assert(qw(3) + kOutP * kH == kNW, "weight layout");

// bfloat16 from float, round to nearest even (the gfx950 conversion
// instruction, two values per instruction where the compiler pairs them)
__device__ __forceinline__ uint16_t to_bf16(float f) {
  return __builtin_bit_cast(uint16_t, (__bf16)f);
}
__device__ __forceinline__ float from_bf16(uint16_t h) {
  return __uint_as_float((uint32_t)h << 16);
}

// tanh for activations that are rounded to bfloat16 right after:
// 1 - 2 / (e^{2x} + 1) with the hardware base-2 exponential and reciprocal
// (both about 1 ulp; saturates to +-1 through e^{2x} -> inf or 0), and
// x (1 - x^2/3) for |x| < 2^-6, where the quotient form loses relative
// accuracy; within about 1e-6 relative of tanh, far below half a bfloat16
// unit (2^-9).
__device__ __forceinline__ float tanh_act(float x) {
  const float e = __builtin_amdgcn_exp2f(x * 2.8853900817779268f);  // e^{2x}
  const float big = 1.0f - 2.0f * __builtin_amdgcn_rcpf(e + 1.0f);
  const float small = x * (1.0f - 0.33333333333333333f * (x * x));
  return fabsf(x) < 0.015625f ? small : big;
}

// gfx950 MFMA, 16 x 16 outputs, K = 32.  Lane l supplies A[l%16][8(l/16)+j]
// and B[8(l/16)+j][l%16] (j = 0..7) and receives D[4(l/16)+r][l%16].
__device__ __forceinline__ f32x4 mfma32(bf16x8 a, bf16x8 b, f32x4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
}

__device__ __forceinline__ bf16x8 ld8(const uint16_t* p) { return *(const bf16x8*)p; }

__device__ __forceinline__ f32x4 mfma(bf16x4 a, bf16x4 b, f32x4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, c, 0, 0, 0);
}

__device__ __forceinline__ bf16x4 ld4(const uint16_t* p) { return *(const bf16x4*)p; }

__device__ __forceinline__ void st4(uint16_t* p, uint16_t a, uint16_t b, uint16_t c,
                                    uint16_t d) {
  bf16x4 v;
  v[0] = (short)a;
  v[1] = (short)b;
  v[2] = (short)c;
  v[3] = (short)d;
  *(bf16x4*)p = v;
}

struct MlpDev {
  float* p;        // master parameters
  float* g;        // gradients
  float* m;        // Adam first moment
  float* v;        // Adam second moment
  float* loss;
  uint16_t* wb;    // BF16 weights [out][in]
  uint16_t* wbt;   // BF16 weights [in][out]
  // training batch, feature-major (row f holds feature f of all B samples):
  // activations a0 [32][B], a1..a3 [128][B]; pre-activation gradients
  // g2, g1, g0 [128][B] and g3T [16][B]; g3 [B][16] sample-major
  uint16_t *a0, *a1, *a2, *a3;
  uint16_t *g3, *g2, *g1, *g0, *g3T;
  float* lpart;    // per-wave loss partial sums of a training batch
  float* wpart;    // [kWMaxChunks][DIG_MLP_NPARAM] gradient partial sums
  int64_t B;       // rows of the training arrays
};

// One 128-wide layer for a tile of 64 samples: out = act(W in + b), with
// in [64][K] and out [64][128] in LDS.  Wave w computes neurons 32w..32w+31
// (two 16-row MFMA tiles) for all four 16-sample column tiles.
// Lane layout of the 16x16x16 MFMA: lane l supplies A[l%16][4(l/16)+j] and
// B[4(l/16)+j][l%16] and receives D[4(l/16)+r][l%16].
template <int K>
__device__ __forceinline__ void mma_rows(const uint16_t* __restrict__ W, const uint16_t* in,
                                         int wave, int lane, f32x4 acc[2][4]) {
  const int li = lane & 15;
#pragma unroll
  for (int rt = 0; rt < 2; ++rt)
#pragma unroll
    for (int ct = 0; ct < 4; ++ct) acc[rt][ct] = f32x4{0.0f, 0.0f, 0.0f, 0.0f};
  if constexpr (K % 32 == 0) {
    const int lk = 8 * (lane >> 4);
#pragma unroll
    for (int k0 = 0; k0 < K; k0 += 32) {
      const bf16x8 a0 = ld8(W + (32 * wave + li) * K + k0 + lk);
      const bf16x8 a1 = ld8(W + (32 * wave + 16 + li) * K + k0 + lk);
#pragma unroll
      for (int ct = 0; ct < 4; ++ct) {
        const bf16x8 b = ld8(in + (16 * ct + li) * kLds + k0 + lk);
        acc[0][ct] = mfma32(a0, b, acc[0][ct]);
        acc[1][ct] = mfma32(a1, b, acc[1][ct]);
      }
    }
  } else {  // K = 16 (the padded output layer's back-propagation)
    const int lk = 4 * (lane >> 4);
    const bf16x4 a0 = ld4(W + (32 * wave + li) * K + lk);
    const bf16x4 a1 = ld4(W + (32 * wave + 16 + li) * K + lk);
#pragma unroll
    for (int ct = 0; ct < 4; ++ct) {
      const bf16x4 b = ld4(in + (16 * ct + li) * kLds + lk);
      acc[0][ct] = mfma(a0, b, acc[0][ct]);
      acc[1][ct] = mfma(a1, b, acc[1][ct]);
    }
  }
}

template <int K>
__device__ void hidden_layer(const uint16_t* __restrict__ W, const float* __restrict__ b,
                             const uint16_t* in, uint16_t* out, uint16_t* gact, int64_t B,
                             int64_t s0, int wave, int lane) {
  f32x4 acc[2][4];
  mma_rows<K>(W, in, wave, lane, acc);
  const int li = lane & 15, lg = lane >> 4;
#pragma unroll
  for (int rt = 0; rt < 2; ++rt) {
    const int n0 = 32 * wave + 16 * rt + 4 * lg;
    const float b0 = b[n0], b1 = b[n0 + 1], b2 = b[n0 + 2], b3 = b[n0 + 3];
#pragma unroll
    for (int ct = 0; ct < 4; ++ct) {
      const int s = 16 * ct + li;
      const uint16_t h0 = to_bf16(tanh_act(acc[rt][ct][0] + b0));
      const uint16_t h1 = to_bf16(tanh_act(acc[rt][ct][1] + b1));
      const uint16_t h2 = to_bf16(tanh_act(acc[rt][ct][2] + b2));
      const uint16_t h3 = to_bf16(tanh_act(acc[rt][ct][3] + b3));
      st4(out + s * kLds + n0, h0, h1, h2, h3);
      if (gact) {
        gact[(int64_t)n0 * B + s0 + s] = h0;
        gact[(int64_t)(n0 + 1) * B + s0 + s] = h1;
        gact[(int64_t)(n0 + 2) * B + s0 + s] = h2;
        gact[(int64_t)(n0 + 3) * B + s0 + s] = h3;
      }
    }
  }
}

// Back-propagation through one layer: gout = bf16(W^T gin * (1 - a^2)), with
// WT = W^T [128][K], gin [64][K] in LDS and a the layer's output activation.
template <int K>
__device__ void back_layer(const uint16_t* __restrict__ WT, const uint16_t* gin, uint16_t* gout,
                           const uint16_t* __restrict__ a, uint16_t* gglob, int64_t B,
                           int64_t s0, int wave, int lane) {
  f32x4 acc[2][4];
  mma_rows<K>(WT, gin, wave, lane, acc);
  const int li = lane & 15, lg = lane >> 4;
#pragma unroll
  for (int rt = 0; rt < 2; ++rt) {
    const int n0 = 32 * wave + 16 * rt + 4 * lg;
#pragma unroll
    for (int ct = 0; ct < 4; ++ct) {
      const int s = 16 * ct + li;
      uint16_t h[4];
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int64_t at = (int64_t)(n0 + r) * B + s0 + s;
        const float x = from_bf16(a[at]);
        h[r] = to_bf16(acc[rt][ct][r] * (1.0f - x * x));
        gglob[at] = h[r];
      }
      st4(gout + s * kLds + n0, h[0], h[1], h[2], h[3]);
    }
  }
}

// Forward pass of a tile of 64 samples.  TRAIN: also stores every activation,
// the loss contribution and the output gradient bf16(2 (y - t) / (7 n)).
template <bool TRAIN>
__global__ __launch_bounds__(kThreads) void k_mlp_fwd(MlpDev d, const float* __restrict__ x,
                                                      const float* __restrict__ t,
                                                      float* __restrict__ y, int64_t n) {
  __shared__ __attribute__((aligned(16))) uint16_t bufA[kTile * kLds];
  __shared__ __attribute__((aligned(16))) uint16_t bufB[kTile * kLds];
  const int64_t s0 = (int64_t)blockIdx.x * kTile;
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  for (int i = threadIdx.x; i < kTile * kIn; i += kThreads) {
    const int s = i / kIn, k = i % kIn;
    const int64_t gs = s0 + s;
    const float v = (k < kNIn && gs < n) ? x[gs * kNIn + k] : 0.0f;
    const uint16_t h = to_bf16(v);
    bufA[s * kLds + k] = h;
    if (TRAIN) d.a0[(int64_t)k * d.B + gs] = h;
  }
  __syncthreads();
  hidden_layer<kIn>(d.wb + qw(0), d.p + pb(0), bufA, bufB, TRAIN ? d.a1 : nullptr, d.B, s0,
                    wave, lane);
  __syncthreads();
  hidden_layer<kH>(d.wb + qw(1), d.p + pb(1), bufB, bufA, TRAIN ? d.a2 : nullptr, d.B, s0,
                   wave, lane);
  __syncthreads();
  hidden_layer<kH>(d.wb + qw(2), d.p + pb(2), bufA, bufB, TRAIN ? d.a3 : nullptr, d.B, s0,
                   wave, lane);
  __syncthreads();
  // output layer: wave w takes samples 16w..16w+15, all 16 (padded) outputs
  const int li = lane & 15, lg = lane >> 4;
  const uint16_t* W3 = d.wb + qw(3);
  f32x4 acc = {0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
  for (int k0 = 0; k0 < kH; k0 += 32)
    acc = mfma32(ld8(W3 + li * kH + k0 + 8 * lg),
                 ld8(bufB + (16 * wave + li) * kLds + k0 + 8 * lg), acc);
  const int s = 16 * wave + li;
  const int64_t gs = s0 + s;
  float lsum = 0.0f;
  const float scale = 2.0f / (7.0f * (float)n);
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    const int j = 4 * lg + r;
    const float yv = acc[r] + d.p[pb(3) + j];
    const bool real = j < kNOut && gs < n;
    if (!TRAIN) {
      if (real) y[gs * kNOut + j] = yv;
    } else {
      const float dv = real ? yv - t[gs * kNOut + j] : 0.0f;
      lsum += dv * dv;
      const uint16_t gv = to_bf16(dv * scale);
      d.g3[gs * kOutP + j] = gv;
      d.g3T[(int64_t)j * d.B + gs] = gv;
    }
  }
  if (TRAIN) {
    for (int off = 32; off > 0; off >>= 1) lsum += __shfl_xor(lsum, off);
    if (lane == 0) d.lpart[blockIdx.x * (kThreads / 64) + wave] = lsum;
  }
}

// Loss of a training batch: the per-wave partial sums of the forward pass
// added in a fixed order (deterministic), over 7 n.
// Loss of a training batch from the per-wave partial sums, in a fixed order
// (a 256-thread workgroup, every thread taking part).
__device__ __forceinline__ void loss_sum(const MlpDev& d, int nparts, int64_t n) {
  __shared__ float sh[4];
  float v = 0.0f;
  for (int i = threadIdx.x; i < nparts; i += 256) v += d.lpart[i];
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
  if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = v;
  __syncthreads();
  if (threadIdx.x == 0) d.loss[0] = (((sh[0] + sh[1]) + sh[2]) + sh[3]) / (7.0f * (float)n);
}

__global__ __launch_bounds__(256) void k_mlp_loss(MlpDev d, int nparts, int64_t n) {
  loss_sum(d, nparts, n);
}

// One hidden layer of the inference kernel from register-resident weights:
// out = bf16(tanh(W in + b)) for 64 samples, wave w computing neurons
// 32w..32w+31.  W[rt][kb]: rows 32w + 16 rt + (l % 16), inputs 32 kb + 8 (l / 16) + j.
template <int KB>
__device__ __forceinline__ void infer_layer(const bf16x8 (&W)[2][KB], const float* __restrict__ b,
                                            const uint16_t* in, uint16_t* out, int wave,
                                            int lane) {
  const int li = lane & 15, lg = lane >> 4;
  f32x4 acc[2][4];
#pragma unroll
  for (int rt = 0; rt < 2; ++rt)
#pragma unroll
    for (int ct = 0; ct < 4; ++ct) acc[rt][ct] = f32x4{0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
  for (int kb = 0; kb < KB; ++kb)
#pragma unroll
    for (int ct = 0; ct < 4; ++ct) {
      const bf16x8 bv = ld8(in + (16 * ct + li) * kLds + 32 * kb + 8 * lg);
      acc[0][ct] = mfma32(W[0][kb], bv, acc[0][ct]);
      acc[1][ct] = mfma32(W[1][kb], bv, acc[1][ct]);
    }
#pragma unroll
  for (int rt = 0; rt < 2; ++rt) {
    const int n0 = 32 * wave + 16 * rt + 4 * lg;
    const float b0 = b[n0], b1 = b[n0 + 1], b2 = b[n0 + 2], b3 = b[n0 + 3];
#pragma unroll
    for (int ct = 0; ct < 4; ++ct)
      st4(out + (16 * ct + li) * kLds + n0, to_bf16(tanh_act(acc[rt][ct][0] + b0)),
          to_bf16(tanh_act(acc[rt][ct][1] + b1)), to_bf16(tanh_act(acc[rt][ct][2] + b2)),
          to_bf16(tanh_act(acc[rt][ct][3] + b3)));
  }
}

// Inference over n samples: a persistent grid, tiles of 64 samples taken in
// a grid stride.  Each wave loads once the BF16 weights it multiplies by
// (rows 32w..32w+31 of the three hidden layers, all 16 padded rows of the
// output layer: 22 x 8 values per lane) and keeps them in registers.
__global__ __launch_bounds__(kThreads, 2) void k_mlp_infer(MlpDev d, const float* __restrict__ x,
                                                         float* __restrict__ y, int64_t n,
                                                         int64_t ntiles) {
  __shared__ __attribute__((aligned(16))) uint16_t bufA[kTile * kLds];
  __shared__ __attribute__((aligned(16))) uint16_t bufB[kTile * kLds];
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63, li = lane & 15, lg = lane >> 4;
  bf16x8 w0[2][1], w1[2][4], w2[2][4], w3[4];
#pragma unroll
  for (int rt = 0; rt < 2; ++rt) {
    const int row = 32 * wave + 16 * rt + li;
    w0[rt][0] = ld8(d.wb + qw(0) + row * kIn + 8 * lg);
#pragma unroll
    for (int kb = 0; kb < 4; ++kb) {
      w1[rt][kb] = ld8(d.wb + qw(1) + row * kH + 32 * kb + 8 * lg);
      w2[rt][kb] = ld8(d.wb + qw(2) + row * kH + 32 * kb + 8 * lg);
    }
  }
#pragma unroll
  for (int kb = 0; kb < 4; ++kb) w3[kb] = ld8(d.wb + qw(3) + li * kH + 32 * kb + 8 * lg);
  for (int64_t tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
    const int64_t s0 = tile * kTile;
    for (int i = threadIdx.x; i < kTile * kIn; i += kThreads) {
      const int sl = i / kIn, k = i % kIn;
      const int64_t gs = s0 + sl;
      bufA[sl * kLds + k] = to_bf16((k < kNIn && gs < n) ? x[gs * kNIn + k] : 0.0f);
    }
    __syncthreads();
    infer_layer<1>(w0, d.p + pb(0), bufA, bufB, wave, lane);
    __syncthreads();
    infer_layer<4>(w1, d.p + pb(1), bufB, bufA, wave, lane);
    __syncthreads();
    infer_layer<4>(w2, d.p + pb(2), bufA, bufB, wave, lane);
    __syncthreads();
    // output layer: wave w takes samples 16w..16w+15, all 16 (padded) outputs
    f32x4 acc = {0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
    for (int kb = 0; kb < 4; ++kb)
      acc = mfma32(w3[kb], ld8(bufB + (16 * wave + li) * kLds + 32 * kb + 8 * lg), acc);
    const int64_t gs = s0 + 16 * wave + li;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int j = 4 * lg + r;
      if (j < kNOut && gs < n) y[gs * kNOut + j] = acc[r] + d.p[pb(3) + j];
    }
    // the next tile's input goes to bufA, last read before the barrier above;
    // bufB is rewritten only after the barrier that follows that input
  }
}

// Back-propagation of a tile: g3 -> g2 -> g1 -> g0 (pre-activation gradients).
__global__ __launch_bounds__(kThreads) void k_mlp_bwd(MlpDev d) {
  __shared__ __attribute__((aligned(16))) uint16_t gA[kTile * kLds];
  __shared__ __attribute__((aligned(16))) uint16_t gB[kTile * kLds];
  const int64_t s0 = (int64_t)blockIdx.x * kTile;
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  for (int i = threadIdx.x; i < kTile * kOutP; i += kThreads) {
    const int s = i / kOutP, j = i % kOutP;
    gA[s * kLds + j] = d.g3[(s0 + s) * kOutP + j];
  }
  __syncthreads();
  back_layer<kOutP>(d.wbt + qw(3), gA, gB, d.a3, d.g2, d.B, s0, wave, lane);
  __syncthreads();
  back_layer<kH>(d.wbt + qw(2), gB, gA, d.a2, d.g1, d.B, s0, wave, lane);
  __syncthreads();
  back_layer<kH>(d.wbt + qw(1), gA, gB, d.a1, d.g0, d.B, s0, wave, lane);
}

// Weight and bias gradients of a batch: dW_l[o][i] = sum_s g_l[s][o] a_l[s][i]
// and db_l[o] = sum_s g_l[s][o], from the feature-major activations and
// gradients.  Split over samples: workgroup (l, chunk) takes all of layer l's
// weights for one chunk of samples.  Its rows of g^T and a^T are staged in
// LDS kWStage samples at a time (each row read from memory once, rather than
// once per 32 x 32 output block), and wave w computes its tiles from there
// with 16 x 16 MFMA tiles and the samples as the reduction axis (A = rows of
// g^T, B = rows of a^T: 8 consecutive samples per lane, one 16-byte read
// each): layers 0-2 rows 32w..32w+31 (two row tiles) against every input
// tile, layer 3 (16 padded outputs, one row tile) input tiles 2w and 2w+1.
// It writes its partial block (and the bias sums of its rows); k_mlp_wred
// adds the chunks' partials in chunk order, so the result does not depend
// on timing.
constexpr int kWMaxChunks = 128;
constexpr int kWStage = 64;           // samples per LDS stage
constexpr int kWRow = kWStage + 8;    // LDS row stride in bf16 (padded)
constexpr int kWPieces = kWStage / 8; // 16-byte pieces per staged row
static_assert(kWStage % 32 == 0, "whole 32-sample MFMA steps per stage");
constexpr size_t kWLds = 2 * 128 * kWRow * sizeof(uint16_t);

// One workgroup's share of layer l: RT row tiles from rt0, CT input tiles
// from ct0 per wave; BIAS: the wave also sums its rows' bias gradients.
template <int RT, int CT>
__device__ __forceinline__ void wgrad_layer(const MlpDev& d, int l, int64_t s_lo, int64_t s_hi,
                                            int ck, int rt0, int ct0, bool bias,
                                            uint16_t* sA, uint16_t* sB) {
  const int lane = threadIdx.x & 63, li = lane & 15, lg = lane >> 4;
  const int O = dout(l), I = din(l);
  const uint16_t* gT = l == 3 ? d.g3T : l == 2 ? d.g2 : l == 1 ? d.g1 : d.g0;
  const uint16_t* aT = l == 3 ? d.a3 : l == 2 ? d.a2 : l == 1 ? d.a1 : d.a0;
  f32x4 acc[RT][CT];
#pragma unroll
  for (int rt = 0; rt < RT; ++rt)
#pragma unroll
    for (int ct = 0; ct < CT; ++ct) acc[rt][ct] = f32x4{0.0f, 0.0f, 0.0f, 0.0f};
  float bs[RT];
#pragma unroll
  for (int rt = 0; rt < RT; ++rt) bs[rt] = 0.0f;
  const bf16x8 zero = {};
  for (int64_t s0 = s_lo; s0 < s_hi; s0 += kWStage) {
    __syncthreads();  // the previous stage has been read
    // 16-byte pieces, kWPieces per row of the stage; a 32-sample step is
    // read when it starts before the chunk's end, later steps are zeros
    for (int pc = threadIdx.x; pc < (O + I) * kWPieces; pc += blockDim.x) {
      const bool isA = pc < O * kWPieces;
      const int q = isA ? pc : pc - O * kWPieces;
      const int row = q / kWPieces, c8 = (q % kWPieces) * 8;
      const bool ok = s0 + (c8 & ~31) < s_hi;
      const bf16x8 v = ok ? ld8((isA ? gT : aT) + (int64_t)row * d.B + s0 + c8) : zero;
      *(bf16x8*)((isA ? sA : sB) + row * kWRow + c8) = v;
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < kWStage / 32; ++k) {
      bf16x8 A[RT], Bv[CT];
#pragma unroll
      for (int rt = 0; rt < RT; ++rt)
        A[rt] = ld8(sA + (16 * (rt0 + rt) + li) * kWRow + 32 * k + 8 * lg);
#pragma unroll
      for (int ct = 0; ct < CT; ++ct)
        Bv[ct] = ld8(sB + (16 * (ct0 + ct) + li) * kWRow + 32 * k + 8 * lg);
#pragma unroll
      for (int rt = 0; rt < RT; ++rt)
#pragma unroll
        for (int ct = 0; ct < CT; ++ct) acc[rt][ct] = mfma32(A[rt], Bv[ct], acc[rt][ct]);
      if (bias) {
#pragma unroll
        for (int rt = 0; rt < RT; ++rt)
#pragma unroll
          for (int j = 0; j < 8; ++j) bs[rt] += (float)A[rt][j];
      }
    }
  }
  float* part = d.wpart + (int64_t)ck * DIG_MLP_NPARAM;
#pragma unroll
  for (int rt = 0; rt < RT; ++rt) {
#pragma unroll
    for (int ct = 0; ct < CT; ++ct)
#pragma unroll
      for (int r = 0; r < 4; ++r)
        part[pw(l) + (16 * (rt0 + rt) + 4 * lg + r) * I + 16 * (ct0 + ct) + li] = acc[rt][ct][r];
    if (bias) {
      float v = bs[rt];
      v += __shfl_xor(v, 16);
      v += __shfl_xor(v, 32);
      if (lg == 0) part[pb(l) + 16 * (rt0 + rt) + li] = v;
    }
  }
}

__global__ __launch_bounds__(256) void k_mlp_wgrad(MlpDev d, int64_t rows, int nchunks,
                                                   int64_t chunk) {
  extern __shared__ __align__(16) unsigned char smem_w[];
  uint16_t* sA = (uint16_t*)smem_w;
  uint16_t* sB = sA + 128 * kWRow;
  const int wave = threadIdx.x >> 6;
  const int l = (int)blockIdx.x / nchunks, ck = (int)blockIdx.x % nchunks;
  const int64_t s_lo = (int64_t)ck * chunk;
  const int64_t s_hi = s_lo + chunk < rows ? s_lo + chunk : rows;
  if (l == 3) {
    wgrad_layer<1, 2>(d, l, s_lo, s_hi, ck, 0, 2 * wave, wave == 0, sA, sB);
  } else if (l == 0) {
    wgrad_layer<2, 2>(d, l, s_lo, s_hi, ck, 2 * wave, 0, true, sA, sB);
  } else {
    wgrad_layer<2, 8>(d, l, s_lo, s_hi, ck, 2 * wave, 0, true, sA, sB);
  }
}

// Gradient of every parameter: the chunk partials added in chunk order.
__global__ void k_mlp_wred(MlpDev d, int nchunks) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= DIG_MLP_NPARAM) return;
  float v = 0.0f;
  // loads of sixteen chunks in flight, added in chunk order
#pragma unroll 16
  for (int c = 0; c < nchunks; ++c) v += d.wpart[(int64_t)c * DIG_MLP_NPARAM + i];
  d.g[i] = v;
}

// BF16 copies of parameter i (no-op for biases).
__device__ __forceinline__ void write_copies(const MlpDev& d, int i, float val) {
#pragma unroll
  for (int l = 0; l < 4; ++l) {
    if (i >= pw(l) && i < pb(l)) {
      const int k = i - pw(l), o = k / din(l), c = k % din(l);
      const uint16_t h = to_bf16(val);
      d.wb[qw(l) + o * din(l) + c] = h;
      d.wbt[qw(l) + c * dout(l) + o] = h;
    }
  }
}

// Adam update of parameter i with gradient g (no contraction, so the
// separate and the fused launches round alike).
__device__ __forceinline__ void adam_update(const MlpDev& d, int i, float g, float lr, float b1,
                                            float b2, float eps, float c1, float c2) {
#pragma clang fp contract(off)
  const float m = b1 * d.m[i] + (1.0f - b1) * g;
  const float v = b2 * d.v[i] + (1.0f - b2) * g * g;
  d.m[i] = m;
  d.v[i] = v;
  const float p = d.p[i] - lr * (m / c1) / (sqrtf(v / c2) + eps);
  d.p[i] = p;
  write_copies(d, i, p);
}

__global__ void k_mlp_adam(MlpDev d, float lr, float b1, float b2, float eps, float c1,
                           float c2) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= DIG_MLP_NPARAM) return;
  adam_update(d, i, d.g[i], lr, b1, b2, eps, c1, c2);
}

// A training step's tail in one launch: workgroup 0 also sums the loss; each
// parameter's gradient is the chunk partials added in chunk order (as the
// plain reduction adds them), stored, and applied by Adam.
__global__ __launch_bounds__(256) void k_mlp_wred_adam(MlpDev d, int nchunks, int nparts,
                                                       int64_t n, float lr, float b1, float b2,
                                                       float eps, float c1, float c2) {
  if (blockIdx.x == 0) loss_sum(d, nparts, n);
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= DIG_MLP_NPARAM) return;
  float v = 0.0f;
#pragma unroll 16
  for (int c = 0; c < nchunks; ++c) v += d.wpart[(int64_t)c * DIG_MLP_NPARAM + i];
  d.g[i] = v;
  adam_update(d, i, v, lr, b1, b2, eps, c1, c2);
}

__global__ void k_mlp_sync(MlpDev d) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < DIG_MLP_NPARAM) write_copies(d, i, d.p[i]);
}

__global__ void k_mlp_zero(float* p, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = 0.0f;
}

constexpr size_t kAlignM = 256;
size_t up(size_t v) { return (v + kAlignM - 1) / kAlignM * kAlignM; }

struct MlpOffsets {
  size_t wb, wbt, a0, a1, a2, a3, g3, g2, g1, g0, g3T, lpart, wpart;
};

void plan(int32_t max_batch, dig_mlp_layout* L, MlpOffsets* O) {
  const size_t B = (size_t)((max_batch + kTile - 1) / kTile) * kTile;
  size_t o = 0;
  auto take = [&](size_t bytes) {
    const size_t r = o;
    o = up(o + bytes);
    return r;
  };
  memset(L, 0, sizeof(*L));
  L->max_batch = (int32_t)B;
  L->params = take(4 * DIG_MLP_NPARAM);
  L->grads = take(4 * DIG_MLP_NPARAM);
  L->adam_m = take(4 * DIG_MLP_NPARAM);
  L->adam_v = take(4 * DIG_MLP_NPARAM);
  L->loss = take(4);
  O->wb = take(2 * kNW);
  O->wbt = take(2 * kNW);
  O->a0 = take(2 * B * kIn);
  O->a1 = take(2 * B * kH);
  O->a2 = take(2 * B * kH);
  O->a3 = take(2 * B * kH);
  O->g3 = take(2 * B * kOutP);
  O->g2 = take(2 * B * kH);
  O->g1 = take(2 * B * kH);
  O->g0 = take(2 * B * kH);
  O->g3T = take(2 * B * kOutP);
  O->lpart = take(4 * (B / kTile) * (kThreads / 64));
  O->wpart = take(4 * (size_t)kWMaxChunks * DIG_MLP_NPARAM);
  L->total_bytes = o;
}

}  // namespace
}  // namespace dig

using namespace dig;

struct dig_mlp {
  unsigned char* ws;
  dig_mlp_layout L;
  MlpOffsets O;
  int64_t infer_grid;  // workgroups of the persistent inference launch
  MlpDev dev() const {
    MlpDev d;
    d.p = (float*)(ws + L.params);
    d.g = (float*)(ws + L.grads);
    d.m = (float*)(ws + L.adam_m);
    d.v = (float*)(ws + L.adam_v);
    d.loss = (float*)(ws + L.loss);
    d.wb = (uint16_t*)(ws + O.wb);
    d.wbt = (uint16_t*)(ws + O.wbt);
    d.a0 = (uint16_t*)(ws + O.a0);
    d.a1 = (uint16_t*)(ws + O.a1);
    d.a2 = (uint16_t*)(ws + O.a2);
    d.a3 = (uint16_t*)(ws + O.a3);
    d.g3 = (uint16_t*)(ws + O.g3);
    d.g2 = (uint16_t*)(ws + O.g2);
    d.g1 = (uint16_t*)(ws + O.g1);
    d.g0 = (uint16_t*)(ws + O.g0);
    d.lpart = (float*)(ws + O.lpart);
    d.g3T = (uint16_t*)(ws + O.g3T);
    d.wpart = (float*)(ws + O.wpart);
    d.B = L.max_batch;
    return d;
  }
};

namespace {
dig_status hip_check(const char* where) {
  const hipError_t e = hipGetLastError();
  if (e == hipSuccess) return DIG_OK;
  return report(DIG_ERR_HIP, (std::string(where) + ": " + hipGetErrorString(e)).c_str());
}
}  // namespace

extern "C" {

dig_status mlp_plan(int32_t max_batch, dig_mlp_layout* out) {
  if (!out) return report(DIG_ERR_INVALID, "null layout");
  if (max_batch < 1 || max_batch > (1 << 24))
    return report(DIG_ERR_INVALID, "max_batch must lie in [1, 2^24]");
  MlpOffsets O;
  plan(max_batch, out, &O);
  return DIG_OK;
}

dig_status mlp_create(void* ws, size_t bytes, int32_t max_batch, dig_stream_t stream,
                      dig_mlp** out) {
  if (!out) return report(DIG_ERR_INVALID, "null output");
  *out = nullptr;
  if (!ws || ((uintptr_t)ws) % kAlignM)
    return report(DIG_ERR_INVALID, "workspace null or not 256-byte aligned");
  if (max_batch < 1 || max_batch > (1 << 24))
    return report(DIG_ERR_INVALID, "max_batch must lie in [1, 2^24]");
  dig_mlp* m = new dig_mlp;
  m->ws = (unsigned char*)ws;
  plan(max_batch, &m->L, &m->O);
  {
    // two workgroups per compute unit (register-resident weights)
    int dev = 0, cus = 256;
    if (hipGetDevice(&dev) == hipSuccess)
      (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    m->infer_grid = 2 * (int64_t)(cus > 0 ? cus : 256);
  }
  if (bytes < m->L.total_bytes) {
    delete m;
    return report(DIG_ERR_INVALID, "workspace too small");
  }
  // the weight-gradient kernel stages its rows in LDS (kWLds bytes)
  if (hipFuncSetAttribute((const void*)k_mlp_wgrad, hipFuncAttributeMaxDynamicSharedMemorySize,
                          (int)kWLds) != hipSuccess) {
    delete m;
    return report(DIG_ERR_HIP, "mlp_create: LDS attribute of the weight-gradient kernel");
  }
  MlpDev d = m->dev();
  hipStream_t s = (hipStream_t)stream;
  for (float* p : {d.g, d.m, d.v, d.loss}) {
    const int64_t n = p == d.loss ? 1 : DIG_MLP_NPARAM;
    hipLaunchKernelGGL(k_mlp_zero, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, p, n);
  }
  const dig_status st = hip_check("mlp_create");
  if (st != DIG_OK) {
    delete m;
    return st;
  }
  *out = m;
  return DIG_OK;
}

dig_status mlp_sync(dig_mlp* m, dig_stream_t stream) {
  if (!m) return report(DIG_ERR_INVALID, "null network");
  hipLaunchKernelGGL(k_mlp_sync, dim3((DIG_MLP_NPARAM + 255) / 256), dim3(256), 0,
                     (hipStream_t)stream, m->dev());
  return hip_check("mlp_sync");
}

dig_status mlp_forward(dig_mlp* m, const float* x, float* y, int64_t n, dig_stream_t stream) {
  if (!m || (n > 0 && (!x || !y))) return report(DIG_ERR_INVALID, "null argument");
  if (n < 0 || n > ((int64_t)1 << 36)) return report(DIG_ERR_INVALID, "bad sample count");
  if (n == 0) return DIG_OK;
  const int64_t tiles = (n + kTile - 1) / kTile;
  const int64_t grid = tiles < m->infer_grid ? tiles : m->infer_grid;
  hipLaunchKernelGGL(k_mlp_infer, dim3((unsigned)grid), dim3(kThreads), 0, (hipStream_t)stream,
                     m->dev(), x, y, n, tiles);
  return hip_check("mlp_forward");
}

}  // extern "C"

namespace {
struct AdamArgs {
  float lr, b1, b2, eps, c1, c2;
};

// Forward, backward and weight gradients of a batch. With `adam` the loss,
// the gradient reduction and the Adam update run as one launch; without it
// the loss and the reduction run on their own.
dig_status launch_grad(dig_mlp* m, const float* x, const float* t, int64_t n, hipStream_t s,
                       const AdamArgs* adam) {
  MlpDev d = m->dev();
  const unsigned tiles = (unsigned)((n + kTile - 1) / kTile);
  const int nparts = (int)(tiles * (kThreads / 64));
  hipLaunchKernelGGL(k_mlp_fwd<true>, dim3(tiles), dim3(kThreads), 0, s, d, x, t, (float*)nullptr,
                     n);
  if (!adam) hipLaunchKernelGGL(k_mlp_loss, dim3(1), dim3(256), 0, s, d, nparts, n);
  hipLaunchKernelGGL(k_mlp_bwd, dim3(tiles), dim3(kThreads), 0, s, d);
  // sample chunks of the weight gradients: a multiple of 32 samples, at most
  // kWMaxChunks chunks, about 256 samples or more each
  const int64_t rows = (int64_t)tiles * kTile;
  int64_t nch = rows / 256;
  nch = nch < 1 ? 1 : (nch > kWMaxChunks ? kWMaxChunks : nch);
  int64_t chunk = (rows + nch - 1) / nch;
  chunk = (chunk + 31) / 32 * 32;
  nch = (rows + chunk - 1) / chunk;
  hipLaunchKernelGGL(k_mlp_wgrad, dim3((unsigned)(4 * nch)), dim3(256), kWLds, s, d, rows,
                     (int)nch, chunk);
  const dim3 pgrid((DIG_MLP_NPARAM + 255) / 256);
  if (adam)
    hipLaunchKernelGGL(k_mlp_wred_adam, pgrid, dim3(256), 0, s, d, (int)nch, nparts, n, adam->lr,
                       adam->b1, adam->b2, adam->eps, adam->c1, adam->c2);
  else
    hipLaunchKernelGGL(k_mlp_wred, pgrid, dim3(256), 0, s, d, (int)nch);
  return hip_check(adam ? "mlp_train_step" : "mlp_grad");
}

// Adam's hyper-parameters lie in range (NaN fails every comparison).
bool adam_args_ok(float lr, float beta1, float beta2, float eps, int64_t t) {
  return t >= 1 && beta1 >= 0.0f && beta1 < 1.0f && beta2 >= 0.0f && beta2 < 1.0f &&
         eps > 0.0f && lr >= 0.0f;
}
}  // namespace

extern "C" {

dig_status mlp_grad(dig_mlp* m, const float* x, const float* t, int64_t n, dig_stream_t stream) {
  if (!m || !x || !t) return report(DIG_ERR_INVALID, "null argument");
  if (n < 1 || n > m->L.max_batch) return report(DIG_ERR_INVALID, "n outside [1, max_batch]");
  return launch_grad(m, x, t, n, (hipStream_t)stream, nullptr);
}

dig_status mlp_adam(dig_mlp* m, float lr, float beta1, float beta2, float eps, int64_t t,
                    dig_stream_t stream) {
  if (!m) return report(DIG_ERR_INVALID, "null network");
  if (!adam_args_ok(lr, beta1, beta2, eps, t))
    return report(DIG_ERR_INVALID, "bad Adam hyper-parameters");
  const float c1 = (float)(1.0 - pow((double)beta1, (double)t));
  const float c2 = (float)(1.0 - pow((double)beta2, (double)t));
  hipLaunchKernelGGL(k_mlp_adam, dim3((DIG_MLP_NPARAM + 255) / 256), dim3(256), 0,
                     (hipStream_t)stream, m->dev(), lr, beta1, beta2, eps, c1, c2);
  return hip_check("mlp_adam");
}

dig_status mlp_train_step(dig_mlp* m, const float* x, const float* t, int64_t n, float lr,
                          int64_t step, dig_stream_t stream) {
  if (!m || !x || !t) return report(DIG_ERR_INVALID, "null argument");
  if (n < 1 || n > m->L.max_batch) return report(DIG_ERR_INVALID, "n outside [1, max_batch]");
  const float b1 = 0.9f, b2 = 0.999f, eps = 1e-8f;
  if (!adam_args_ok(lr, b1, b2, eps, step))
    return report(DIG_ERR_INVALID, "bad Adam hyper-parameters");
  const AdamArgs A{lr, b1, b2, eps, (float)(1.0 - pow((double)b1, (double)step)),
                   (float)(1.0 - pow((double)b2, (double)step))};
  return launch_grad(m, x, t, n, (hipStream_t)stream, &A);
}

void mlp_destroy(dig_mlp* m) { delete m; }

}  // extern "C"
