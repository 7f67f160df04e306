// Learned closure network on the CDNA4 matrix cores: forward, back-propagation
// and Adam for a 4-layer perceptron (9 -> 128 -> 128 -> 128 -> 7, padded to
// 32 inputs and 16 outputs, tanh hidden layers).  Products use
// v_mfma_f32_16x16x16_bf16: BF16 operands, FP32 accumulation.  A workgroup of
// four waves carries a tile of 64 samples through all layers with the
// activations in LDS; weights (78 KB in BF16) stay in L2.
#include <math.h>
#include <string.h>

#include <string>

#include "dig_internal.h"

namespace dig {
namespace {

typedef short bf16x4 __attribute__((ext_vector_type(4)));
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

// tanh for activations that are rounded to bfloat16 right after: from the
// identity tanh x = sign(x) (1 - e^{-2|x|}) / (1 + e^{-2|x|}) with the
// hardware exponential and reciprocal, and from the Taylor series
// x - x^3/3 + 2x^5/15 - 17x^7/315 for |x| < 2^-4, where the identity loses
// relative accuracy; the result is within a few FP32 ulps of tanh, far below
// half a bfloat16 unit.
__device__ __forceinline__ float tanh_act(float x) {
  const float ax = fabsf(x);
  const float e = __expf(-2.0f * ax);
  const float big = (1.0f - e) * __builtin_amdgcn_rcpf(1.0f + e);
  const float x2 = x * x;
  const float small = ax * (1.0f + x2 * (-1.0f / 3.0f + x2 * (2.0f / 15.0f - x2 * (17.0f / 315.0f))));
  return copysignf(ax < 0.0625f ? small : big, x);
}

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
  uint16_t *a0, *a1, *a2, *a3;  // activations [B][32], [B][128] x3
  uint16_t *g3, *g2, *g1, *g0;  // pre-activation gradients [B][16], [B][128] x3
};

// One 128-wide layer for a tile of 64 samples: out = act(W in + b), with
// in [64][K] and out [64][128] in LDS.  Wave w computes neurons 32w..32w+31
// (two 16-row MFMA tiles) for all four 16-sample column tiles.
// Lane layout of the 16x16x16 MFMA: lane l supplies A[l%16][4(l/16)+j] and
// B[4(l/16)+j][l%16] and receives D[4(l/16)+r][l%16].
template <int K>
__device__ __forceinline__ void mma_rows(const uint16_t* __restrict__ W, const uint16_t* in,
                                         int wave, int lane, f32x4 acc[2][4]) {
  const int li = lane & 15, lk = 4 * (lane >> 4);
#pragma unroll
  for (int rt = 0; rt < 2; ++rt)
#pragma unroll
    for (int ct = 0; ct < 4; ++ct) acc[rt][ct] = f32x4{0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
  for (int k0 = 0; k0 < K; k0 += 16) {
    const bf16x4 a0 = ld4(W + (32 * wave + li) * K + k0 + lk);
    const bf16x4 a1 = ld4(W + (32 * wave + 16 + li) * K + k0 + lk);
#pragma unroll
    for (int ct = 0; ct < 4; ++ct) {
      const bf16x4 b = ld4(in + (16 * ct + li) * kLds + k0 + lk);
      acc[0][ct] = mfma(a0, b, acc[0][ct]);
      acc[1][ct] = mfma(a1, b, acc[1][ct]);
    }
  }
}

template <int K>
__device__ void hidden_layer(const uint16_t* __restrict__ W, const float* __restrict__ b,
                             const uint16_t* in, uint16_t* out, uint16_t* gact, int wave,
                             int lane) {
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
      if (gact) st4(gact + s * kH + n0, h0, h1, h2, h3);
    }
  }
}

// Back-propagation through one layer: gout = bf16(W^T gin * (1 - a^2)), with
// WT = W^T [128][K], gin [64][K] in LDS and a the layer's output activation.
template <int K>
__device__ void back_layer(const uint16_t* __restrict__ WT, const uint16_t* gin, uint16_t* gout,
                           const uint16_t* __restrict__ a, uint16_t* gglob, int wave,
                           int lane) {
  f32x4 acc[2][4];
  mma_rows<K>(WT, gin, wave, lane, acc);
  const int li = lane & 15, lg = lane >> 4;
#pragma unroll
  for (int rt = 0; rt < 2; ++rt) {
    const int n0 = 32 * wave + 16 * rt + 4 * lg;
#pragma unroll
    for (int ct = 0; ct < 4; ++ct) {
      const int s = 16 * ct + li;
      const bf16x4 av = ld4(a + s * kH + n0);
      uint16_t h[4];
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const float x = from_bf16((uint16_t)av[r]);
        h[r] = to_bf16(acc[rt][ct][r] * (1.0f - x * x));
      }
      st4(gout + s * kLds + n0, h[0], h[1], h[2], h[3]);
      st4(gglob + s * kH + n0, h[0], h[1], h[2], h[3]);
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
    if (TRAIN) d.a0[gs * kIn + k] = h;
  }
  __syncthreads();
  hidden_layer<kIn>(d.wb + qw(0), d.p + pb(0), bufA, bufB, TRAIN ? d.a1 + s0 * kH : nullptr,
                    wave, lane);
  __syncthreads();
  hidden_layer<kH>(d.wb + qw(1), d.p + pb(1), bufB, bufA, TRAIN ? d.a2 + s0 * kH : nullptr,
                   wave, lane);
  __syncthreads();
  hidden_layer<kH>(d.wb + qw(2), d.p + pb(2), bufA, bufB, TRAIN ? d.a3 + s0 * kH : nullptr,
                   wave, lane);
  __syncthreads();
  // output layer: wave w takes samples 16w..16w+15, all 16 (padded) outputs
  const int li = lane & 15, lg = lane >> 4;
  const uint16_t* W3 = d.wb + qw(3);
  f32x4 acc = {0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
  for (int k0 = 0; k0 < kH; k0 += 16)
    acc = mfma(ld4(W3 + li * kH + k0 + 4 * lg), ld4(bufB + (16 * wave + li) * kLds + k0 + 4 * lg),
               acc);
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
      d.g3[gs * kOutP + j] = to_bf16(dv * scale);
    }
  }
  if (TRAIN) {
    for (int off = 32; off > 0; off >>= 1) lsum += __shfl_xor(lsum, off);
    if (lane == 0) atomicAdd(d.loss, lsum / (7.0f * (float)n));
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
  back_layer<kOutP>(d.wbt + qw(3), gA, gB, d.a3 + s0 * kH, d.g2 + s0 * kH, wave, lane);
  __syncthreads();
  back_layer<kH>(d.wbt + qw(2), gB, gA, d.a2 + s0 * kH, d.g1 + s0 * kH, wave, lane);
  __syncthreads();
  back_layer<kH>(d.wbt + qw(1), gA, gB, d.a1 + s0 * kH, d.g0 + s0 * kH, wave, lane);
}

// Weight and bias gradients: dW_l = sum over samples of g_l (x) a_l, one
// workgroup per 16x16 block of a weight matrix, the samples as the MFMA
// reduction axis.  The kGradWaves waves of a workgroup each reduce a
// contiguous share of the samples (loads issued kGradAhead MFMA steps ahead),
// then wave 0 adds the shares in wave order: deterministic, no atomics.
// Tiles: layer 3 (8), layer 2 (64), layer 1 (64), layer 0 (16).
constexpr int kGradTiles = 8 + 64 + 64 + 16;
constexpr int kGradWaves = 8;
constexpr int kGradAhead = 4;

__global__ __launch_bounds__(64 * kGradWaves) void k_mlp_wgrad(MlpDev d, int64_t rows) {
  __shared__ f32x4 s_acc[kGradWaves][64];
  __shared__ float s_b[kGradWaves][64];
  int tile = blockIdx.x, l;
  if (tile < 8) {
    l = 3;
  } else if (tile < 72) {
    l = 2;
    tile -= 8;
  } else if (tile < 136) {
    l = 1;
    tile -= 72;
  } else {
    l = 0;
    tile -= 136;
  }
  const int ni = din(l) / 16;
  const int ot = tile / ni, it = tile % ni;
  const uint16_t* g = l == 3 ? d.g3 : l == 2 ? d.g2 : l == 1 ? d.g1 : d.g0;
  const uint16_t* a = l == 3 ? d.a3 : l == 2 ? d.a2 : l == 1 ? d.a1 : d.a0;
  const int ldo = dout(l), ldi = din(l);
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63, li = lane & 15, lg = lane >> 4;
  // this wave's steps of 16 samples: [k0, k1)
  const int64_t steps = rows / 16;
  const int64_t share = (steps + kGradWaves - 1) / kGradWaves;
  const int64_t k0 = min(steps, wave * share), k1 = min(steps, k0 + share);
  f32x4 acc = {0.0f, 0.0f, 0.0f, 0.0f};
  float bsum = 0.0f;
  for (int64_t kb = k0; kb < k1; kb += kGradAhead) {
    bf16x4 A[kGradAhead], B[kGradAhead];
#pragma unroll
    for (int u = 0; u < kGradAhead; ++u) {
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const int64_t s = (kb + u) * 16 + 4 * lg + j;
        const bool ok = kb + u < k1;
        A[u][j] = ok ? (short)g[s * ldo + ot * 16 + li] : (short)0;
        B[u][j] = ok ? (short)a[s * ldi + it * 16 + li] : (short)0;
      }
    }
#pragma unroll
    for (int u = 0; u < kGradAhead; ++u) {
#pragma unroll
      for (int j = 0; j < 4; ++j) bsum += from_bf16((uint16_t)A[u][j]);
      acc = mfma(A[u], B[u], acc);
    }
  }
  s_acc[wave][lane] = acc;
  s_b[wave][lane] = bsum;
  __syncthreads();
  if (wave != 0) return;
  for (int w = 1; w < kGradWaves; ++w) {
    const f32x4 o = s_acc[w][lane];
#pragma unroll
    for (int r = 0; r < 4; ++r) acc[r] += o[r];
    bsum += s_b[w][lane];
  }
#pragma unroll
  for (int r = 0; r < 4; ++r)
    d.g[pw(l) + (ot * 16 + 4 * lg + r) * ldi + it * 16 + li] = acc[r];
  if (it == 0) {
    bsum += __shfl_xor(bsum, 16);
    bsum += __shfl_xor(bsum, 32);
    if (lg == 0) d.g[pb(l) + ot * 16 + li] = bsum;
  }
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

__global__ void k_mlp_adam(MlpDev d, float lr, float b1, float b2, float eps, float c1,
                           float c2) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= DIG_MLP_NPARAM) return;
  const float g = d.g[i];
  const float m = b1 * d.m[i] + (1.0f - b1) * g;
  const float v = b2 * d.v[i] + (1.0f - b2) * g * g;
  d.m[i] = m;
  d.v[i] = v;
  const float p = d.p[i] - lr * (m / c1) / (sqrtf(v / c2) + eps);
  d.p[i] = p;
  write_copies(d, i, p);
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
  size_t wb, wbt, a0, a1, a2, a3, g3, g2, g1, g0;
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
  L->total_bytes = o;
}

}  // namespace
}  // namespace dig

using namespace dig;

struct dig_mlp {
  unsigned char* ws;
  dig_mlp_layout L;
  MlpOffsets O;
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
  if (bytes < m->L.total_bytes) {
    delete m;
    return report(DIG_ERR_INVALID, "workspace too small");
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
  hipLaunchKernelGGL(k_mlp_fwd<false>, dim3((unsigned)((n + kTile - 1) / kTile)), dim3(kThreads),
                     0, (hipStream_t)stream, m->dev(), x, (const float*)nullptr, y, n);
  return hip_check("mlp_forward");
}

dig_status mlp_grad(dig_mlp* m, const float* x, const float* t, int64_t n, dig_stream_t stream) {
  if (!m || !x || !t) return report(DIG_ERR_INVALID, "null argument");
  if (n < 1 || n > m->L.max_batch) return report(DIG_ERR_INVALID, "n outside [1, max_batch]");
  hipStream_t s = (hipStream_t)stream;
  MlpDev d = m->dev();
  const unsigned tiles = (unsigned)((n + kTile - 1) / kTile);
  hipLaunchKernelGGL(k_mlp_zero, dim3(1), dim3(64), 0, s, d.loss, (int64_t)1);
  hipLaunchKernelGGL(k_mlp_fwd<true>, dim3(tiles), dim3(kThreads), 0, s, d, x, t, (float*)nullptr,
                     n);
  hipLaunchKernelGGL(k_mlp_bwd, dim3(tiles), dim3(kThreads), 0, s, d);
  hipLaunchKernelGGL(k_mlp_wgrad, dim3(kGradTiles), dim3(64 * kGradWaves), 0, s, d,
                     (int64_t)tiles * kTile);
  return hip_check("mlp_grad");
}

dig_status mlp_adam(dig_mlp* m, float lr, float beta1, float beta2, float eps, int64_t t,
                    dig_stream_t stream) {
  if (!m) return report(DIG_ERR_INVALID, "null network");
  if (t < 1 || !(beta1 >= 0.0f && beta1 < 1.0f) || !(beta2 >= 0.0f && beta2 < 1.0f) ||
      !(eps > 0.0f) || !(lr >= 0.0f))
    return report(DIG_ERR_INVALID, "bad Adam hyper-parameters");
  const float c1 = (float)(1.0 - pow((double)beta1, (double)t));
  const float c2 = (float)(1.0 - pow((double)beta2, (double)t));
  hipLaunchKernelGGL(k_mlp_adam, dim3((DIG_MLP_NPARAM + 255) / 256), dim3(256), 0,
                     (hipStream_t)stream, m->dev(), lr, beta1, beta2, eps, c1, c2);
  return hip_check("mlp_adam");
}

dig_status mlp_train_step(dig_mlp* m, const float* x, const float* t, int64_t n, float lr,
                          int64_t step, dig_stream_t stream) {
  const dig_status st = mlp_grad(m, x, t, n, stream);
  if (st != DIG_OK) return st;
  return mlp_adam(m, lr, 0.9f, 0.999f, 1e-8f, step, stream);
}

void mlp_destroy(dig_mlp* m) { delete m; }

}  // extern "C"
