// Learned control proposal for gfx950: a three-layer network
// (16 -> 128 -> 128 -> 8) on MFMA, BF16 operands and FP32 accumulation.
//
// Alg. 2 draws every control uniformly from U.  The learned proposal keeps
// that draw for a fixed share of the samples and otherwise draws from a
// Gaussian whose mean and spread the network predicts from the parent node;
// the uniform share keeps a positive density on all of U, which is what the
// completeness argument of Sec. V needs.
//
//   k_mlp_pack     FP32 parameters -> BF16 A-operand fragments + FP32 biases
//   k_mlp_forward  raw network outputs for rows of features
//   k_mlp_head     per frontier entry of the planner: the node's features,
//                  the network, and the Gaussian mean / std in control units
//   k_mlp_grad     minibatch forward and backward of the Gaussian negative
//                  log-likelihood; one partial gradient per 64-row block
//   k_mlp_adam     fixed-order sum of the partial gradients, one Adam step
//                  (Kingma & Ba, 2015)
//   k_log_path     training rows (parent features, normalised control) from
//                  the edges of a root-to-node path
//   k_edge_count,  training rows from every tree edge whose child lies closer
//   k_edge_write   to the goal centre than its parent, in node id order
//
// Layout of the network in registers.  Every product is computed transposed,
// out^T = W * in^T, so the weights are the A operand (16 x 32 per MFMA) and
// the activations of 16 rows are the B operand.  v_mfma_f32_16x16x32_bf16
// leaves lane l holding outputs 16 t + 4 (l / 16) + r (r = 0..3) of row
// l % 16 for output tile t.  Packing tiles 2s and 2s+1 of that accumulator to
// BF16 gives, unchanged, the B operand of K-step s of the next layer when the
// next layer's weights are stored with the matching K order (hid_k below), so
// activations never leave registers between layers.
#include "kp_internal.h"

#include <hip/hip_ext.h>

#include "kp.h"
#include "kp_device.h"

namespace kp {
namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));

constexpr int OFF_W1 = 0;
constexpr int OFF_B1 = OFF_W1 + kMlpHid * kMlpIn;
constexpr int OFF_W2 = OFF_B1 + kMlpHid;
constexpr int OFF_B2 = OFF_W2 + kMlpHid * kMlpHid;
constexpr int OFF_W3 = OFF_B2 + kMlpHid;
constexpr int OFF_B3 = OFF_W3 + kMlpOut * kMlpHid;
static_assert(OFF_B3 + kMlpOut == kMlpParams, "parameter layout");

constexpr float kLsMin = -4.0f, kLsMax = 0.0f;  // clip of the log standard deviation
constexpr uint32_t kTagBatch = 6u;              // Philox tag of the minibatch draws

// Fragment entries (16 bytes: 8 BF16 values of one lane's A operand):
//   F1  W1        8 tiles x 1 K-step       F2T  W2^T  8 tiles x 4 K-steps
//   F2  W2        8 tiles x 4 K-steps      F3T  W3^T  8 tiles x 1 K-step
//   F3  W3 (pad)  1 tile  x 4 K-steps
// followed by the biases b1, b2, b3 as FP32.
constexpr int E_F1 = 0;
constexpr int E_F2 = E_F1 + 8 * 1 * 64;
constexpr int E_F3 = E_F2 + 8 * 4 * 64;
constexpr int E_F2T = E_F3 + 1 * 4 * 64;
constexpr int E_F3T = E_F2T + 8 * 4 * 64;
constexpr int E_END = E_F3T + 8 * 1 * 64;
constexpr int E_FWD = E_F2T;  // entries of the forward pass (F1, F2, F3)
constexpr int N_BIAS = kMlpHid + kMlpHid + kMlpOut;
constexpr size_t kPackedBytes = (size_t)E_END * 16 + (size_t)N_BIAS * 4;
static_assert(kPackedBytes == KP_MLP_PACKED_BYTES, "packed size in kp.h");
static_assert(kMlpParams == KP_MLP_PARAMS, "parameter count in kp.h");

// K index held in slot j of lane group g at K-step s, for a 128-long hidden
// vector held in the accumulator layout (tiles 2s and 2s+1, four each)
__host__ __device__ constexpr int hid_k(int s, int g, int j) {
  return 16 * (2 * s + (j >> 2)) + 4 * g + (j & 3);
}

// parameter held by slot j of fragment entry e, or -1 for a zero
__device__ int frag_param(int e, int j) {
  const int lane = e & 63, i = lane & 15, g = lane >> 4;
  if (e < E_F2) {  // F1: W1[16t + i][8g + j]; inputs 16..31 of the K-step are zero
    const int t = (e - E_F1) >> 6;
    return g < 2 ? OFF_W1 + (16 * t + i) * kMlpIn + 8 * g + j : -1;
  }
  if (e < E_F3) {  // F2: W2[16t + i][hid_k(s, g, j)]
    const int ts = (e - E_F2) >> 6, t = ts >> 2, s = ts & 3;
    return OFF_W2 + (16 * t + i) * kMlpHid + hid_k(s, g, j);
  }
  if (e < E_F2T) {  // F3: W3[i][hid_k(s, g, j)], rows 8..15 zero
    const int s = (e - E_F3) >> 6;
    return i < kMlpOut ? OFF_W3 + i * kMlpHid + hid_k(s, g, j) : -1;
  }
  if (e < E_F3T) {  // F2T: W2^T[16t + i][hid_k(s, g, j)] = W2[hid_k][16t + i]
    const int ts = (e - E_F2T) >> 6, t = ts >> 2, s = ts & 3;
    return OFF_W2 + hid_k(s, g, j) * kMlpHid + 16 * t + i;
  }
  // F3T: W3^T[16t + i][4g + j] for output 4g + j < 8 (lane groups 0, 1, slots 0..3)
  const int t = (e - E_F3T) >> 6;
  return (g < 2 && j < 4) ? OFF_W3 + (4 * g + j) * kMlpHid + 16 * t + i : -1;
}

// round to nearest BF16, ties to even (finite inputs)
__device__ __forceinline__ uint32_t bf16_bits(float v) {
  uint32_t b = __float_as_uint(v);
  b += 0x7FFFu + ((b >> 16) & 1u);
  return b >> 16;
}
__device__ __forceinline__ float bf16_value(uint32_t bits) { return __uint_as_float(bits << 16); }

__device__ __forceinline__ bf16x8 as_bf16x8(u32x4 w) { return __builtin_bit_cast(bf16x8, w); }
__device__ __forceinline__ u32x4 as_u32x4(bf16x8 v) { return __builtin_bit_cast(u32x4, v); }

// eight FP32 values to BF16, round to nearest even (the hardware's packed
// conversion on gfx950)
__device__ __forceinline__ bf16x8 pack8(const float* f) {
  bf16x8 v;
#pragma unroll
  for (int j = 0; j < 8; ++j) v[j] = (__bf16)f[j];
  return v;
}

// BF16 relu of accumulator tiles a (slots 0..3) and b (slots 4..7)
__device__ __forceinline__ bf16x8 pack_relu(const f32x4& a, const f32x4& b) {
  float f[8];
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    f[r] = fmaxf(a[r], 0.0f);
    f[4 + r] = fmaxf(b[r], 0.0f);
  }
  return pack8(f);
}

// slot j of a packed operand, as BF16 bits
__device__ __forceinline__ uint32_t slot_bits(bf16x8 v, int j) {
  const u32x4 w = as_u32x4(v);
  return (w[j >> 1] >> (16 * (j & 1))) & 0xFFFFu;
}

__device__ __forceinline__ f32x4 mfma(u32x4 a, bf16x8 b, f32x4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x32_bf16(as_bf16x8(a), b, c, 0, 0, 0);
}

struct Fwd {
  f32x4 o;        // lane group 0: outputs 0..3, group 1: outputs 4..7 (row lane % 16)
  bf16x8 h1[4];   // BF16 relu(layer 1), B operand of layer 2 per K-step
  bf16x8 h2[4];   // BF16 relu(layer 2), B operand of layer 3 per K-step
};

// The network on the 16 rows whose layer-1 operand is xb.  frag: fragment
// entries (LDS or global); bias: b1, b2, b3 (FP32).
__device__ __forceinline__ void forward_wave(const u32x4* frag, const float* bias, bf16x8 xb,
                                             Fwd& r) {
  const int lane = __lane_id(), g = lane >> 4;
  f32x4 acc[8];
#pragma unroll
  for (int t = 0; t < 8; ++t) {
#pragma unroll
    for (int q = 0; q < 4; ++q) acc[t][q] = bias[16 * t + 4 * g + q];
    acc[t] = mfma(frag[E_F1 + t * 64 + lane], xb, acc[t]);
  }
#pragma unroll
  for (int s = 0; s < 4; ++s) r.h1[s] = pack_relu(acc[2 * s], acc[2 * s + 1]);
#pragma unroll
  for (int t = 0; t < 8; ++t)
#pragma unroll
    for (int q = 0; q < 4; ++q) acc[t][q] = bias[kMlpHid + 16 * t + 4 * g + q];
#pragma unroll
  for (int s = 0; s < 4; ++s)
#pragma unroll
    for (int t = 0; t < 8; ++t) acc[t] = mfma(frag[E_F2 + (t * 4 + s) * 64 + lane], r.h1[s], acc[t]);
#pragma unroll
  for (int s = 0; s < 4; ++s) r.h2[s] = pack_relu(acc[2 * s], acc[2 * s + 1]);
  f32x4 o;
#pragma unroll
  for (int q = 0; q < 4; ++q) o[q] = g < 2 ? bias[2 * kMlpHid + 4 * g + q] : 0.0f;
#pragma unroll
  for (int s = 0; s < 4; ++s) o = mfma(frag[E_F3 + s * 64 + lane], r.h2[s], o);
  r.o = o;
}

// The network on NG groups of 16 rows at once (layer-1 operands xb[0..NG-1]):
// each weight fragment read from LDS feeds NG products, and layer 2 is
// computed one pair of output tiles at a time, so only 8 NG accumulators
// are live.  Raw outputs in o[] (same layout as Fwd::o).
template <int NG>
__device__ __forceinline__ void forward_rows(const u32x4* frag, const float* bias,
                                             const bf16x8* xb, f32x4* o) {
  const int lane = __lane_id(), g = lane >> 4;
  bf16x8 h1[NG][4], h2[NG][4];
#pragma unroll
  for (int s = 0; s < 4; ++s) {
    const u32x4 A0 = frag[E_F1 + (2 * s) * 64 + lane];
    const u32x4 A1 = frag[E_F1 + (2 * s + 1) * 64 + lane];
    f32x4 b0, b1;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      b0[q] = bias[16 * (2 * s) + 4 * g + q];
      b1[q] = bias[16 * (2 * s + 1) + 4 * g + q];
    }
#pragma unroll
    for (int k = 0; k < NG; ++k) h1[k][s] = pack_relu(mfma(A0, xb[k], b0), mfma(A1, xb[k], b1));
  }
  __builtin_amdgcn_sched_barrier(0);
#pragma unroll
  for (int s2 = 0; s2 < 4; ++s2) {
    f32x4 b0, b1;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      b0[q] = bias[kMlpHid + 16 * (2 * s2) + 4 * g + q];
      b1[q] = bias[kMlpHid + 16 * (2 * s2 + 1) + 4 * g + q];
    }
    f32x4 a0[NG], a1[NG];
#pragma unroll
    for (int k = 0; k < NG; ++k) {
      a0[k] = b0;
      a1[k] = b1;
    }
#pragma unroll
    for (int s = 0; s < 4; ++s) {
      const u32x4 A0 = frag[E_F2 + ((2 * s2) * 4 + s) * 64 + lane];
      const u32x4 A1 = frag[E_F2 + ((2 * s2 + 1) * 4 + s) * 64 + lane];
#pragma unroll
      for (int k = 0; k < NG; ++k) {
        a0[k] = mfma(A0, h1[k][s], a0[k]);
        a1[k] = mfma(A1, h1[k][s], a1[k]);
      }
    }
#pragma unroll
    for (int k = 0; k < NG; ++k) h2[k][s2] = pack_relu(a0[k], a1[k]);
    // keep the next tile pair's weight loads below this point: hoisting all
    // of them ahead would need the whole weight set in registers
    __builtin_amdgcn_sched_barrier(0);
  }
  f32x4 b3;
#pragma unroll
  for (int q = 0; q < 4; ++q) b3[q] = g < 2 ? bias[2 * kMlpHid + 4 * g + q] : 0.0f;
#pragma unroll
  for (int k = 0; k < NG; ++k) o[k] = b3;
#pragma unroll
  for (int s = 0; s < 4; ++s) {
    const u32x4 A = frag[E_F3 + s * 64 + lane];
#pragma unroll
    for (int k = 0; k < NG; ++k) o[k] = mfma(A, h2[k][s], o[k]);
  }
}

// raw feature k of a tree node: state, P_accept of its region, goal offset
__device__ __forceinline__ float raw_feature(const Params& p, const Dev& d, int32_t node, int k,
                                             float pacc) {
  const int n = p.n;
  if (k < n) return d.x[(size_t)k * d.capP + node];
  if (k == n) return pacc;
  if (k <= n + 3) {
    const int a = k - n - 1;
    return p.goal_c[a] - d.x[(size_t)a * d.capP + node];
  }
  return 0.0f;
}

__device__ __forceinline__ float node_pacc(const Dev& d, int32_t node) {
  const unsigned long long thr = d.thr[d.cell[node] >> 6];
  const unsigned long long t = thr < (1ull << 32) ? thr : (1ull << 32);
  return (float)t * 0x1p-32f;
}

// layer-1 operand of row `node` for this lane: features 8g .. 8g+7 (g < 2)
__device__ __forceinline__ bf16x8 node_operand(const Params& p, const Dev& d, int32_t node,
                                               bool valid) {
  const int g = __lane_id() >> 4;
  float f[8];
  if (valid && g < 2) {
    const float pacc = node_pacc(d, node);
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      const int k = 8 * g + j;
      f[j] = (raw_feature(p, d, node, k, pacc) - p.fc[k]) * p.fs[k];
    }
  } else {
#pragma unroll
    for (int j = 0; j < 8; ++j) f[j] = 0.0f;
  }
  return pack8(f);
}

__device__ __forceinline__ bf16x8 row_operand(const float* x, int32_t row, bool valid) {
  const int g = __lane_id() >> 4;
  float f[8];
  if (valid && g < 2) {
    const float4 a = reinterpret_cast<const float4*>(x + (size_t)row * kMlpIn + 8 * g)[0];
    const float4 b = reinterpret_cast<const float4*>(x + (size_t)row * kMlpIn + 8 * g)[1];
    f[0] = a.x; f[1] = a.y; f[2] = a.z; f[3] = a.w;
    f[4] = b.x; f[5] = b.y; f[6] = b.z; f[7] = b.w;
  } else {
#pragma unroll
    for (int j = 0; j < 8; ++j) f[j] = 0.0f;
  }
  return pack8(f);
}

// forward-pass weights and biases into LDS.  Every load of a thread is
// issued before its first store, so the copy costs one memory latency
// rather than one per entry.
template <int BLOCK>
__device__ __forceinline__ void stage_forward(const u32x4* packed, u32x4* sfrag, float* sbias) {
  constexpr int kPer = (E_FWD + BLOCK - 1) / BLOCK;
  u32x4 v[kPer];
#pragma unroll
  for (int i = 0; i < kPer; ++i) {
    const int k = (int)threadIdx.x + i * BLOCK;
    if (k < E_FWD) v[i] = packed[k];
  }
  const float* b = reinterpret_cast<const float*>(packed + E_END);
  const float bv = (int)threadIdx.x < N_BIAS ? b[threadIdx.x] : 0.0f;
#pragma unroll
  for (int i = 0; i < kPer; ++i) {
    const int k = (int)threadIdx.x + i * BLOCK;
    if (k < E_FWD) sfrag[k] = v[i];
  }
  if ((int)threadIdx.x < N_BIAS) sbias[threadIdx.x] = bv;
  __syncthreads();
}

constexpr int kMlpBlock = 256;   // training: 4 waves of 16 rows (one 64-row block)
constexpr int kInfBlock = 512;   // inference: 8 waves (2 per SIMD) share one LDS copy
static_assert(kInfBlock >= 264, "one bias per thread when staging");
constexpr int kInfWaves = kInfBlock / 64;
constexpr int kInfNG = 4;        // 16-row groups per wave pass
constexpr int kInfRows = 16 * kInfNG;  // rows per wave pass

// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_mlp_pack(const float* __restrict__ prm,
                                                  u32x4* __restrict__ packed) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e < E_END) {
    u32x4 w;
#pragma unroll
    for (int h = 0; h < 4; ++h) {
      const int a = frag_param(e, 2 * h), b = frag_param(e, 2 * h + 1);
      const uint32_t lo = a >= 0 ? bf16_bits(prm[a]) : 0u;
      const uint32_t hi = b >= 0 ? bf16_bits(prm[b]) : 0u;
      w[h] = lo | (hi << 16);
    }
    packed[e] = w;
  } else if (e < E_END + N_BIAS) {
    const int k = e - E_END;
    const int src = k < kMlpHid       ? OFF_B1 + k
                    : k < 2 * kMlpHid ? OFF_B2 + (k - kMlpHid)
                                      : OFF_B3 + (k - 2 * kMlpHid);
    reinterpret_cast<float*>(packed + E_END)[k] = prm[src];
  }
}

__global__ __launch_bounds__(kInfBlock) void k_mlp_forward(const u32x4* __restrict__ packed,
                                                           const float* __restrict__ x,
                                                           int32_t rows, float* __restrict__ out) {
  __shared__ u32x4 sfrag[E_FWD];
  __shared__ float sbias[N_BIAS];
  const int passes = (rows + kInfRows - 1) / kInfRows;
  if ((int)blockIdx.x * kInfWaves >= passes) return;
  const int wave = threadIdx.x >> 6, lane = __lane_id(), g = lane >> 4;
  // the first pass's inputs load while the weights are staged
  bf16x8 xb[kInfNG];
  int q = blockIdx.x * kInfWaves + wave;
#pragma unroll
  for (int k = 0; k < kInfNG; ++k) {
    const int32_t row = q * kInfRows + 16 * k + (lane & 15);
    xb[k] = row_operand(x, row, row < rows);
  }
  stage_forward<kInfBlock>(packed, sfrag, sbias);
  for (; q < passes; q += gridDim.x * kInfWaves) {
    if (q != (int)blockIdx.x * kInfWaves + wave) {
#pragma unroll
      for (int k = 0; k < kInfNG; ++k) {
        const int32_t row = q * kInfRows + 16 * k + (lane & 15);
        xb[k] = row_operand(x, row, row < rows);
      }
    }
    f32x4 o[kInfNG];
    forward_rows<kInfNG>(sfrag, sbias, xb, o);
#pragma unroll
    for (int k = 0; k < kInfNG; ++k) {
      const int32_t row = q * kInfRows + 16 * k + (lane & 15);
      if (row < rows && g < 2)
        reinterpret_cast<float4*>(out + (size_t)row * kMlpOut)[g] =
            make_float4(o[k][0], o[k][1], o[k][2], o[k][3]);
    }
  }
}

// Per frontier entry e (the layout the expansion lanes index by e = lane /
// lambda): Gaussian mean (4 floats) and standard deviation (4 floats).
__device__ __forceinline__ void head_body(const Env* __restrict__ env) {
  __shared__ u32x4 sfrag[E_FWD];
  __shared__ float sbias[N_BIAS];
  const Params& p = env->p;
  const Dev& d = env->d;
  const Ctl* c = d.ctl;
  if (c->done || p.mix_thr == 0ull) return;
  const int32_t nF = c->nF, f_expl = c->f_expl, f_base = c->f_base;
  const int passes = (nF + kInfRows - 1) / kInfRows;
  if ((int)blockIdx.x * kInfWaves >= passes) return;
  const int wave = threadIdx.x >> 6, lane = __lane_id(), g = lane >> 4;
  const int m = p.m;
  // the first pass's node features load while the weights are staged
  bf16x8 xb[kInfNG];
  int q = blockIdx.x * kInfWaves + wave;
#pragma unroll
  for (int k = 0; k < kInfNG; ++k) {
    const int32_t e = q * kInfRows + 16 * k + (lane & 15);
    const bool valid = e < nF;
    const int32_t node = valid ? frontier_node(d.F, e, f_expl, f_base) : 0;
    xb[k] = node_operand(p, d, node, valid);
  }
  stage_forward<kInfBlock>(reinterpret_cast<const u32x4*>(d.mlp), sfrag, sbias);
  for (; q < passes; q += gridDim.x * kInfWaves) {
    if (q != (int)blockIdx.x * kInfWaves + wave) {
#pragma unroll
      for (int k = 0; k < kInfNG; ++k) {
        const int32_t e = q * kInfRows + 16 * k + (lane & 15);
        const bool valid = e < nF;
        const int32_t node = valid ? frontier_node(d.F, e, f_expl, f_base) : 0;
        xb[k] = node_operand(p, d, node, valid);
      }
    }
    f32x4 o[kInfNG];
    forward_rows<kInfNG>(sfrag, sbias, xb, o);
#pragma unroll
    for (int k = 0; k < kInfNG; ++k) {
      const int32_t e = q * kInfRows + 16 * k + (lane & 15);
      if (e < nF && g < 2) {
        float v[4];
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          const float lo = p.u_lo[j], hi = p.u_hi[j];
          const float ctr = 0.5f * (lo + hi), half = 0.5f * (hi - lo);
          if (j >= m) v[j] = 0.0f;
          else if (g == 0) v[j] = ctr + half * tanhf(o[k][j]);
          else v[j] = half * expf(fminf(fmaxf(o[k][j], kLsMin), kLsMax));
        }
        reinterpret_cast<float4*>(d.head + (size_t)e * 8)[g] = make_float4(v[0], v[1], v[2], v[3]);
      }
    }
  }
}

__global__ __launch_bounds__(kInfBlock) void k_mlp_head(const Env* __restrict__ env) {
  head_body(env);
}
// one grid row per problem of a batch; problems without a proposal return at once
__global__ __launch_bounds__(kInfBlock) void k_mlp_head_batch(const Env* const* __restrict__ envs) {
  head_body(envs[blockIdx.y]);
}

// ---------------------------------------------------------------------------
// training
// ---------------------------------------------------------------------------
constexpr int kTrStride = 72;  // BF16 per row of a transposed activation tile (64 rows + pad)

__device__ __forceinline__ u32x4 lds_frag(const uint16_t* base, int row, int col) {
  return *reinterpret_cast<const u32x4*>(base + row * kTrStride + col);
}

// One 64-row block of a minibatch: forward, the loss gradient at the
// outputs, backward through both hidden layers (register resident, weights
// as A operands), then the weight gradients as products over the block's rows
// with activations transposed through LDS.  Writes the block's gradient of
// the mean loss (all kMlpParams entries) and its share of the mean loss.
__global__ __launch_bounds__(kMlpBlock) void k_mlp_grad(const u32x4* __restrict__ packed,
                                                        const float* __restrict__ X,
                                                        const float* __restrict__ T,
                                                        int32_t n_rows, int32_t m, int32_t batch,
                                                        uint32_t key0, uint32_t key1,
                                                        int32_t step, float* __restrict__ partials,
                                                        float* __restrict__ loss_out) {
  // phase A: H1T, DZ2T, DZ1T [128][kTrStride], XT [16][kTrStride]
  // phase B: H2T [128][kTrStride], DOT [16][kTrStride]
  __shared__ uint16_t tr[(3 * kMlpHid + kMlpIn) * kTrStride];
  __shared__ float wloss[4];
  uint16_t* H1T = tr;
  uint16_t* DZ2T = tr + kMlpHid * kTrStride;
  uint16_t* DZ1T = tr + 2 * kMlpHid * kTrStride;
  uint16_t* XT = tr + 3 * kMlpHid * kTrStride;
  uint16_t* H2T = tr;
  uint16_t* DOT = tr + kMlpHid * kTrStride;

  const int wave = threadIdx.x >> 6, lane = __lane_id(), g = lane >> 4, n = lane & 15;
  const int col = wave * 16 + n;  // row of the block
  const int32_t k = (int32_t)blockIdx.x * kMlpRowsPerBlock + col;
  const bool valid = k < batch;
  int32_t row = k;
  if ((key0 | key1) != 0u) {
    const U4 w = philox((uint32_t)step, (uint32_t)k, 0u, kTagBatch, key0, key1);
    row = (int32_t)(((unsigned long long)w.w[0] * (unsigned long long)n_rows) >> 32);
  }
  const float* bias = reinterpret_cast<const float*>(packed + E_END);
  const bf16x8 xb = row_operand(X, row, valid);
  Fwd r;
  forward_wave(packed, bias, xb, r);

  // outputs: lane groups 0 and 1 of a row swap halves, so both see mean and log-std
  float tj[4];
#pragma unroll
  for (int j = 0; j < 4; ++j) tj[j] = (valid && j < m) ? T[(size_t)row * 4 + j] : 0.0f;
  float dv[4];
  float lrow = 0.0f;
  const float inv_b = 1.0f / (float)batch;
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    const float other = __shfl_xor(r.o[j], 16);
    const float om = (g == 0) ? r.o[j] : other;
    const float ol = (g == 0) ? other : r.o[j];
    const float a = tanhf(om);
    const float ls = fminf(fmaxf(ol, kLsMin), kLsMax);
    const float e2 = expf(-2.0f * ls);
    const float rr = tj[j] - a;
    const bool use = valid && j < m && g < 2;
    if (g == 0) {
      dv[j] = use ? -rr * (1.0f - a * a) * e2 * inv_b : 0.0f;
      if (use) lrow += 0.5f * rr * rr * e2 + ls;
    } else {
      const bool inside = ol > kLsMin && ol < kLsMax;
      dv[j] = (use && inside) ? (1.0f - rr * rr * e2) * inv_b : 0.0f;
    }
  }
  // d loss / d outputs as the B operand of the W3^T products: slots 0..3 of
  // lane group g hold outputs 4g .. 4g+3
  u32x4 dw = {0u, 0u, 0u, 0u};
  if (g < 2) {
    dw[0] = bf16_bits(dv[0]) | (bf16_bits(dv[1]) << 16);
    dw[1] = bf16_bits(dv[2]) | (bf16_bits(dv[3]) << 16);
  }
  const bf16x8 dob = as_bf16x8(dw);

  // layer 3 backward: d h2 = W3^T d o, masked by relu
  bf16x8 dz2[4];
  {
    f32x4 acc[8];
#pragma unroll
    for (int t = 0; t < 8; ++t) {
      acc[t] = f32x4{0.0f, 0.0f, 0.0f, 0.0f};
      acc[t] = mfma(packed[E_F3T + t * 64 + lane], dob, acc[t]);
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const uint32_t hb = slot_bits(r.h2[t >> 1], 4 * (t & 1) + q);
        if (!(hb != 0u && hb < 0x8000u)) acc[t][q] = 0.0f;
      }
    }
#pragma unroll
    for (int s = 0; s < 4; ++s) {
      float f[8];
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        f[q] = acc[2 * s][q];
        f[4 + q] = acc[2 * s + 1][q];
      }
      dz2[s] = pack8(f);
    }
  }
  // layer 2 backward: d h1 = W2^T d z2, masked by relu
  bf16x8 dz1[4];
  {
    f32x4 acc[8];
#pragma unroll
    for (int t = 0; t < 8; ++t) acc[t] = f32x4{0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
    for (int s = 0; s < 4; ++s)
#pragma unroll
      for (int t = 0; t < 8; ++t) acc[t] = mfma(packed[E_F2T + (t * 4 + s) * 64 + lane], dz2[s], acc[t]);
#pragma unroll
    for (int t = 0; t < 8; ++t)
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const uint32_t hb = slot_bits(r.h1[t >> 1], 4 * (t & 1) + q);
        if (!(hb != 0u && hb < 0x8000u)) acc[t][q] = 0.0f;
      }
#pragma unroll
    for (int s = 0; s < 4; ++s) {
      float f[8];
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        f[q] = acc[2 * s][q];
        f[4 + q] = acc[2 * s + 1][q];
      }
      dz1[s] = pack8(f);
    }
  }

  // phase A: transposes of h1, d z2, d z1, x
#pragma unroll
  for (int t = 0; t < 8; ++t)
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int f = 16 * t + 4 * g + q, j = 4 * (t & 1) + q;
      H1T[f * kTrStride + col] = (uint16_t)slot_bits(r.h1[t >> 1], j);
      DZ2T[f * kTrStride + col] = (uint16_t)slot_bits(dz2[t >> 1], j);
      DZ1T[f * kTrStride + col] = (uint16_t)slot_bits(dz1[t >> 1], j);
    }
  if (g < 2)
#pragma unroll
    for (int j = 0; j < 8; ++j) XT[(8 * g + j) * kTrStride + col] = (uint16_t)slot_bits(xb, j);
  {
    float lw = lrow;
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) lw += __shfl_xor(lw, o);
    if (lane == 0) wloss[wave] = lw;
  }
  __syncthreads();

  float* gout = partials + (size_t)blockIdx.x * kMlpParams;
  // W2 gradient: out feature tiles 2*wave, 2*wave+1; input feature tiles 0..7
#pragma unroll
  for (int a = 0; a < 2; ++a) {
    const int tm = 2 * wave + a;
    for (int tn = 0; tn < 8; ++tn) {
      f32x4 acc = {0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
      for (int s = 0; s < 2; ++s)
        acc = mfma(lds_frag(DZ2T, 16 * tm + n, 32 * s + 8 * g),
                   as_bf16x8(lds_frag(H1T, 16 * tn + n, 32 * s + 8 * g)), acc);
#pragma unroll
      for (int q = 0; q < 4; ++q)
        gout[OFF_W2 + (16 * tm + 4 * g + q) * kMlpHid + 16 * tn + n] = acc[q];
    }
    // W1 gradient: the same out tiles, the 16 inputs
    f32x4 acc = {0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
    for (int s = 0; s < 2; ++s)
      acc = mfma(lds_frag(DZ1T, 16 * tm + n, 32 * s + 8 * g),
                 as_bf16x8(lds_frag(XT, n, 32 * s + 8 * g)), acc);
#pragma unroll
    for (int q = 0; q < 4; ++q) gout[OFF_W1 + (16 * tm + 4 * g + q) * kMlpIn + n] = acc[q];
  }
  {
    // bias gradients of the hidden layers: sums over the block's rows
    const int f = threadIdx.x & (kMlpHid - 1);
    const uint16_t* src = (threadIdx.x < kMlpHid) ? DZ1T : DZ2T;
    float sum = 0.0f;
    for (int c2 = 0; c2 < kMlpRowsPerBlock; ++c2) sum += bf16_value(src[f * kTrStride + c2]);
    gout[(threadIdx.x < kMlpHid ? OFF_B1 : OFF_B2) + f] = sum;
  }
  if (threadIdx.x == 0) loss_out[blockIdx.x] = (wloss[0] + wloss[1] + wloss[2] + wloss[3]) * inv_b;
  __syncthreads();

  // phase B: transposes of h2 and d o
#pragma unroll
  for (int t = 0; t < 8; ++t)
#pragma unroll
    for (int q = 0; q < 4; ++q)
      H2T[(16 * t + 4 * g + q) * kTrStride + col] = (uint16_t)slot_bits(r.h2[t >> 1], 4 * (t & 1) + q);
#pragma unroll
  for (int q = 0; q < 4; ++q) DOT[(4 * g + q) * kTrStride + col] = (uint16_t)slot_bits(dob, q);
  __syncthreads();
  // W3 gradient: outputs 0..7 (rows 8..15 of the tile are zero), inputs in
  // tiles 2*wave, 2*wave+1
#pragma unroll
  for (int a = 0; a < 2; ++a) {
    const int tn = 2 * wave + a;
    f32x4 acc = {0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
    for (int s = 0; s < 2; ++s)
      acc = mfma(lds_frag(DOT, n, 32 * s + 8 * g), as_bf16x8(lds_frag(H2T, 16 * tn + n, 32 * s + 8 * g)),
                 acc);
    if (g < 2)
#pragma unroll
      for (int q = 0; q < 4; ++q) gout[OFF_W3 + (4 * g + q) * kMlpHid + 16 * tn + n] = acc[q];
  }
  if (threadIdx.x < kMlpOut) {
    float sum = 0.0f;
    for (int c2 = 0; c2 < kMlpRowsPerBlock; ++c2) sum += bf16_value(DOT[threadIdx.x * kTrStride + c2]);
    gout[OFF_B3 + threadIdx.x] = sum;
  }
}

__global__ __launch_bounds__(256) void k_mlp_adam(float* __restrict__ prm, float* __restrict__ m1,
                                                  float* __restrict__ m2,
                                                  const float* __restrict__ partials, int32_t nb,
                                                  float lr, float beta1, float beta2, float eps,
                                                  float inv_bc1, float inv_bc2) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= kMlpParams) return;
  float g = 0.0f;
  for (int b = 0; b < nb; ++b) g += partials[(size_t)b * kMlpParams + i];
  const float a = beta1 * m1[i] + (1.0f - beta1) * g;
  const float v = beta2 * m2[i] + (1.0f - beta2) * (g * g);
  m1[i] = a;
  m2[i] = v;
  prm[i] = prm[i] - lr * (a * inv_bc1) / (sqrtf(v * inv_bc2) + eps);
}

// training rows from the path that k_path left in d.path (root first):
// row k = features of the parent of edge k, targets = the edge's control
// in units of the control box's half-width around its centre
__global__ __launch_bounds__(256) void k_log_path(const Env* __restrict__ env, float* __restrict__ X,
                                                  float* __restrict__ T, int32_t cap_rows,
                                                  int32_t row0) {
  const Params& p = env->p;
  const Dev& d = env->d;
  const int32_t len = d.path[0];
  if (len < 2 || len > kMaxPath) return;
  for (int32_t k = threadIdx.x; k < len - 1; k += blockDim.x) {
    const int32_t row = row0 + k;
    if (row >= cap_rows) break;
    const int32_t parent = d.path[1 + k], child = d.path[2 + k];
    const float pacc = node_pacc(d, parent);
    for (int j = 0; j < kMlpIn; ++j)
      X[(size_t)row * kMlpIn + j] = (raw_feature(p, d, parent, j, pacc) - p.fc[j]) * p.fs[j];
    for (int j = 0; j < 4; ++j) {
      const float lo = p.u_lo[j], hi = p.u_hi[j];
      const float ctr = 0.5f * (lo + hi), half = 0.5f * (hi - lo);
      T[(size_t)row * 4 + j] =
          (j < p.m && half > 0.0f) ? (d.u[(size_t)j * d.capP + child] - ctr) / half : 0.0f;
    }
  }
}

// Tree edges that move towards the goal: edge (parent(i), i) qualifies when
// node i's position is strictly closer to the goal centre than its parent's.
// Rows are written in node id order (a count pass per 4096-node tile, then a
// write pass that sums the earlier tiles' counts), so the row set and its
// order do not depend on the schedule.
constexpr int kEdgeTile = 4096;
constexpr int kEdgeBlock = 256;
constexpr int kEdgePerThread = kEdgeTile / kEdgeBlock;  // 16 consecutive nodes per thread

__device__ __forceinline__ bool edge_closer(const Params& p, const Dev& d, int32_t i) {
  const int32_t a = d.parent[i];
  if (a < 0) return false;
  float dc = 0.0f, da = 0.0f;
  for (int k = 0; k < 3; ++k) {
    const float ec = d.x[(size_t)k * d.capP + i] - p.goal_c[k];
    const float ea = d.x[(size_t)k * d.capP + a] - p.goal_c[k];
    dc = __builtin_fmaf(ec, ec, dc);
    da = __builtin_fmaf(ea, ea, da);
  }
  return dc < da;
}

__device__ __forceinline__ uint32_t edge_bits(const Params& p, const Dev& d, int32_t N,
                                              int32_t base) {
  uint32_t bits = 0;
  for (int k = 0; k < kEdgePerThread; ++k) {
    const int32_t i = base + k;
    if (i < N && edge_closer(p, d, i)) bits |= 1u << k;
  }
  return bits;
}

// block-wide exclusive prefix of per-thread counts; *total gets the sum
__device__ __forceinline__ uint32_t edge_block_prefix(uint32_t v, uint32_t* total) {
  __shared__ uint32_t s_w[kEdgeBlock / 64];
  const int w = threadIdx.x >> 6;
  const unsigned long long below = (1ull << __lane_id()) - 1ull;
  uint32_t ex = 0, tot = 0;
  for (int b = 0; b < 5; ++b) {   // counts are at most 16
    const unsigned long long m = __ballot((v >> b) & 1u);
    ex += (uint32_t)__popcll(m & below) << b;
    tot += (uint32_t)__popcll(m) << b;
  }
  if (__lane_id() == 0) s_w[w] = tot;
  __syncthreads();
  uint32_t off = 0, all = 0;
  for (int k = 0; k < kEdgeBlock / 64; ++k) {
    off += (k < w) ? s_w[k] : 0u;
    all += s_w[k];
  }
  *total = all;
  return off + ex;
}

__global__ __launch_bounds__(kEdgeBlock) void k_edge_count(const Env* __restrict__ env,
                                                           uint32_t* __restrict__ tcount) {
  const Params& p = env->p;
  const Dev& d = env->d;
  const int32_t N = d.ctl->N;
  const int32_t base = blockIdx.x * kEdgeTile + threadIdx.x * kEdgePerThread;
  const uint32_t bits = edge_bits(p, d, N, base);
  uint32_t total;
  (void)edge_block_prefix((uint32_t)__popc(bits), &total);
  if (threadIdx.x == 0) tcount[blockIdx.x] = total;
}

__global__ __launch_bounds__(kEdgeBlock) void k_edge_write(const Env* __restrict__ env,
                                                           const uint32_t* __restrict__ tcount,
                                                           float* __restrict__ X,
                                                           float* __restrict__ T,
                                                           int32_t cap_rows, int32_t row0) {
  const Params& p = env->p;
  const Dev& d = env->d;
  const int32_t N = d.ctl->N;
  __shared__ uint32_t s_pre;
  if (threadIdx.x < 64) {
    uint32_t part = 0;
    for (uint32_t t = threadIdx.x; t < blockIdx.x; t += 64) part += tcount[t];
    for (int o = 32; o > 0; o >>= 1) part += __shfl_xor(part, o);
    if (threadIdx.x == 0) s_pre = part;
  }
  __syncthreads();
  const int32_t base = blockIdx.x * kEdgeTile + threadIdx.x * kEdgePerThread;
  uint32_t bits = edge_bits(p, d, N, base);
  uint32_t total;
  const uint32_t off = edge_block_prefix((uint32_t)__popc(bits), &total);
  int64_t row = (int64_t)row0 + s_pre + off;
  while (bits) {
    const int k = __ffs(bits) - 1;
    bits &= bits - 1u;
    if (row >= cap_rows) break;
    const int32_t child = base + k, parent = d.parent[child];
    const float pacc = node_pacc(d, parent);
    for (int j = 0; j < kMlpIn; ++j)
      X[(size_t)row * kMlpIn + j] = (raw_feature(p, d, parent, j, pacc) - p.fc[j]) * p.fs[j];
    for (int j = 0; j < 4; ++j) {
      const float lo = p.u_lo[j], hi = p.u_hi[j];
      const float ctr = 0.5f * (lo + hi), half = 0.5f * (hi - lo);
      T[(size_t)row * 4 + j] =
          (j < p.m && half > 0.0f) ? (d.u[(size_t)j * d.capP + child] - ctr) / half : 0.0f;
    }
    ++row;
  }
}

}  // namespace

size_t mlp_packed_bytes() { return kPackedBytes; }

hipError_t launch_mlp_pack(const float* params, uint4* packed, hipStream_t s) {
  const int n = E_END + N_BIAS;
  hipLaunchKernelGGL(k_mlp_pack, dim3((n + 255) / 256), dim3(256), 0, s, params,
                     reinterpret_cast<u32x4*>(packed));
  return hipGetLastError();
}

hipError_t launch_mlp_forward(const uint4* packed, const float* x, int32_t rows, float* out,
                              hipStream_t s) {
  const int passes = (rows + kInfRows - 1) / kInfRows;
  int grid = (passes + kInfWaves - 1) / kInfWaves;
  if (grid > 1024) grid = 1024;
  if (grid < 1) grid = 1;
  hipLaunchKernelGGL(k_mlp_forward, dim3(grid), dim3(kInfBlock), 0, s,
                     reinterpret_cast<const u32x4*>(packed), x, rows, out);
  return hipGetLastError();
}

int mlp_head_rows_per_block() { return kInfRows * kInfWaves; }
int mlp_head_grid_max(int cu_count) { return cu_count; }

hipError_t launch_mlp_head(const Env* env, int grid, hipStream_t s, Timing t) {
  if (grid < 1) grid = 1;
  hipExtLaunchKernelGGL(k_mlp_head, dim3(grid), dim3(kInfBlock), 0, s, t.start, t.stop, 0, env);
  return hipGetLastError();
}

hipError_t launch_mlp_head_batch(const Env* const* envs, int n, int grid, hipStream_t s) {
  if (grid < 1) grid = 1;
  hipLaunchKernelGGL(k_mlp_head_batch, dim3(grid, n), dim3(kInfBlock), 0, s, envs);
  return hipGetLastError();
}

hipError_t launch_mlp_grad(const uint4* packed, const float* x, const float* t, int32_t n_rows,
                           int32_t m, int32_t batch, uint64_t key, int32_t step, float* partials,
                           float* loss, hipStream_t s) {
  const int grid = (batch + kMlpRowsPerBlock - 1) / kMlpRowsPerBlock;
  hipLaunchKernelGGL(k_mlp_grad, dim3(grid), dim3(kMlpBlock), 0, s,
                     reinterpret_cast<const u32x4*>(packed), x, t, n_rows, m, batch,
                     (uint32_t)key, (uint32_t)(key >> 32), step, partials, loss);
  return hipGetLastError();
}

hipError_t launch_mlp_adam(float* params, float* m1, float* m2, const float* partials,
                           int32_t n_partials, float lr, float beta1, float beta2, float eps,
                           float inv_bc1, float inv_bc2, hipStream_t s) {
  hipLaunchKernelGGL(k_mlp_adam, dim3((kMlpParams + 255) / 256), dim3(256), 0, s, params, m1, m2,
                     partials, n_partials, lr, beta1, beta2, eps, inv_bc1, inv_bc2);
  return hipGetLastError();
}

int edge_tiles(int32_t n_nodes) { return (n_nodes + kEdgeTile - 1) / kEdgeTile; }

hipError_t launch_edge_count(const Env* env, int tiles, uint32_t* tcount, hipStream_t s) {
  if (tiles < 1) return hipSuccess;
  hipLaunchKernelGGL(k_edge_count, dim3(tiles), dim3(kEdgeBlock), 0, s, env, tcount);
  return hipGetLastError();
}

hipError_t launch_edge_write(const Env* env, int tiles, const uint32_t* tcount, float* x, float* t,
                             int32_t cap_rows, int32_t row0, hipStream_t s) {
  if (tiles < 1) return hipSuccess;
  hipLaunchKernelGGL(k_edge_write, dim3(tiles), dim3(kEdgeBlock), 0, s, env, tcount, x, t,
                     cap_rows, row0);
  return hipGetLastError();
}

hipError_t launch_log_path(const Env* env, float* x, float* t, int32_t cap_rows, int32_t row0,
                           hipStream_t s) {
  hipLaunchKernelGGL(k_log_path, dim3(1), dim3(256), 0, s, env, x, t, cap_rows, row0);
  return hipGetLastError();
}

}  // namespace kp
