// mlp.hip -- kernels of the learned sign-distribution proposal: a small MLP
// (inputs = the +-1 signs of one mask, outputs = logits of scheme features)
// trained on masks labelled by the exact scheme kernels, then used to rank
// mutated candidate masks before the exact kernels judge them.
//
// Dense products use gfx950 matrix cores (v_mfma_f32_16x16x32_bf16: BF16
// operands, FP32 accumulation).  Everything else is elementwise or a small
// reduction on the vector units.  bfloat16 values are kept as uint16_t bit
// patterns; conversion rounds to nearest-even from the IEEE-754 binary32
// layout (the upper 16 bits of a float are a bfloat16).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdint>

#include "patchwork.h"
#include "pw_host.h"

namespace pw {

typedef float float4_t __attribute__((ext_vector_type(4)));

__device__ __forceinline__ float bf16_to_f32(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }

__device__ __forceinline__ uint16_t f32_to_bf16(float f) {
  const uint32_t u = __float_as_uint(f);
  const uint32_t rounding = 0x7FFFu + ((u >> 16) & 1u);  // ties to even
  return (uint16_t)((u + rounding) >> 16);
}

// --------------------------------------------------------------------- GEMM
//
// C[M x N] = A[M x K] * B[K x N] with arbitrary element strides (so the
// same kernel serves X W, dY W^T and X^T dY).  A block of four waves owns a
// BM x BN tile (BM, BN in {64, 128}); each wave a (BM/2) x (BN/2) quarter
// made of 16 x 16 MFMA tiles.  K advances TK = 64 (or 32 where K is not a
// multiple of 64) at a time through LDS,
// the next slab being fetched into registers while the current one is
// multiplied.  Tall-K products with few output tiles (the weight gradients
// X^T dY, K = batch) split K over blockIdx.z and add their partial tiles
// into C32 with FP32 atomics.
//
// gfx950 MFMA v_mfma_f32_16x16x32_bf16 operand layout (l = lane):
//   X: lane l holds X[l % 16][8 (l / 16) + 0..7]
//   Y: lane l holds Y[8 (l / 16) + 0..7][l % 16]
//   Z: lane l holds Z[4 (l / 16) + 0..3][l % 16]     (Z = X Y)
// Both tiles sit in LDS k-contiguous ([m][k] and [n][k]), so each operand
// fragment is one 16-byte LDS read.  The product is issued as C^T = B^T A^T
// (X = the B fragment, Y = the A fragment): lane l then holds
// C[l % 16][4 (l / 16) + 0..3], four consecutive columns of one row, and
// the epilogue (+ bias[n], ReLU, times [gate > 0], fp32 and/or bf16
// stores) moves 4 columns per access.

typedef __bf16 bf16x8_t __attribute__((ext_vector_type(8)));

constexpr int TBK = 32;  // K granularity of the API; slabs of TK = 32 or 64

struct GemmArgs {
  const uint16_t* A;
  int64_t a_m, a_k;
  const uint16_t* B;
  int64_t b_k, b_n;
  int M, N, K;
  int k_split;           // K range of one blockIdx.z (multiple of the slab width)
  const float* bias;     // N or null
  const uint16_t* gate;  // M x N (ld g_m) or null: multiply by [gate > 0]
  int64_t g_m;
  int relu;
  float* C32;  // or null
  uint16_t* C16;  // or null
  int64_t c_m;
  int accumulate;  // C32 += result
  int atomic;      // partial tiles of a split K: C32 += result atomically
  float* colsum;   // N or null: colsum[n] += sum over m of the final C[m][n]
  int vec;         // bias, gate, C32 and C16 allow 4-column vector accesses
};

// One ROWS x TK slab of an operand X (element (r, k) at X[r s_row + k s_k])
// moves HBM -> registers -> LDS tile T[ROWS][LDK] in 16-byte chunks.
// MODE 1: contiguous along k (s_k == 1): a chunk is 8 consecutive k of one
// row.  MODE 2: contiguous along r (s_row == 1): chunks of 8 consecutive
// rows of one k, four k at a time, transposed in registers (below).  MODE
// 0: element by element.
typedef uint32_t u32x4_t __attribute__((ext_vector_type(4)));  // 8 bf16

template <int ROWS, int MODE, int TK>
struct Slab {
  static constexpr int CHUNKS = ROWS * TK / 8 / 256;  // per thread
  static constexpr int CPR = TK / 8;                  // 16-byte chunks per row
  static constexpr int LDK = TK + 8;                  // padded LDS row
  // MODE 2: a thread takes a group of 4 k x 8 r (four 16-byte loads, one
  // per k), transposes it in registers and stores 8 rows of 4 consecutive
  // k (8 bytes each); consecutive lanes take consecutive k quads, so a
  // store instruction covers whole bank rows
  static constexpr int KQ = TK / 4, GROUPS = KQ * (ROWS / 8);
  static_assert(MODE != 2 || GROUPS <= 256, "one group per thread");
  static constexpr int NQ = MODE == 2 ? 4 : CHUNKS;
  u32x4_t q[NQ];

  __device__ __forceinline__ void load(const uint16_t* __restrict__ X, int64_t s_row, int64_t s_k, int r0, int k0,
                                       int tid) {
    if (MODE == 2) {
      if (tid < GROUPS) {
        const int k = 4 * (tid % KQ), r = 8 * (tid / KQ);
#pragma unroll
        for (int kk = 0; kk < 4; ++kk)
          q[kk] = *reinterpret_cast<const u32x4_t*>(&X[(int64_t)(k0 + k + kk) * s_k + (int64_t)(r0 + r)]);
      }
      return;
    }
#pragma unroll
    for (int c = 0; c < CHUNKS; ++c) {
      const int id = tid + 256 * c;
      const int r = id / CPR, k = (id % CPR) * 8;
      if (MODE == 1) {
        q[c] = *reinterpret_cast<const u32x4_t*>(&X[(int64_t)(r0 + r) * s_row + (int64_t)(k0 + k)]);
      } else {
        const uint16_t* x = &X[(int64_t)(r0 + r) * s_row + (int64_t)k0 * s_k];
#pragma unroll
        for (int e = 0; e < 4; ++e)
          q[c][e] = (uint32_t)x[(k + 2 * e) * s_k] | ((uint32_t)x[(k + 2 * e + 1) * s_k] << 16);
      }
    }
  }

  __device__ __forceinline__ void store(uint16_t (*T)[LDK], int tid) const {
    if (MODE == 2) {
      if (tid < GROUPS) {
        const int k = 4 * (tid % KQ), r = 8 * (tid / KQ);
#pragma unroll
        for (int e = 0; e < 8; ++e) {
          // row r + e: the low (e even) or high (e odd) halves of word e / 2
          // of the four k loads, paired k, k+1 and k+2, k+3
          const uint32_t sel = (e & 1) ? 0x07060302u : 0x05040100u;
          uint2 d;
          d.x = __builtin_amdgcn_perm(q[1][e >> 1], q[0][e >> 1], sel);
          d.y = __builtin_amdgcn_perm(q[3][e >> 1], q[2][e >> 1], sel);
          *reinterpret_cast<uint2*>(&T[r + e][k]) = d;
        }
      }
      return;
    }
#pragma unroll
    for (int c = 0; c < CHUNKS; ++c) {
      const int id = tid + 256 * c;
      const int r = id / CPR, k = (id % CPR) * 8;
      *reinterpret_cast<u32x4_t*>(&T[r][k]) = q[c];
    }
  }
};

// (compiled for 3 waves per SIMD -- at most 168 registers -- when both
// operands move in 16-byte chunks: those tiles fit without spilling, and two
// waves left the matrix cores idle more often; the element-wise staging of
// unaligned operands keeps 2)
template <int BM, int BN, int AM, int BM_, int TK>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu((AM != 0 && BM_ != 0) ? 3 : 2))) void k_gemm_bf16(
    GemmArgs g) {
  constexpr int FM = BM / 32, FN = BN / 32;  // 16 x 16 tiles per wave along m and n
  constexpr int LDK = TK + 8;
  __shared__ __attribute__((aligned(16))) uint16_t As[BM][LDK];  // [m][k]
  __shared__ __attribute__((aligned(16))) uint16_t Bs[BN][LDK];  // [n][k]
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int m0 = blockIdx.y * BM, n0 = blockIdx.x * BN;
  const int wm = (wave >> 1) * (BM / 2), wn = (wave & 1) * (BN / 2);
  const int kb = blockIdx.z * g.k_split;
  const int ke = kb + g.k_split < g.K ? kb + g.k_split : g.K;
  float4_t acc[FM][FN];
#pragma unroll
  for (int a = 0; a < FM; ++a)
#pragma unroll
    for (int b = 0; b < FN; ++b) acc[a][b] = float4_t{0.f, 0.f, 0.f, 0.f};
  Slab<BM, AM, TK> sa;
  Slab<BN, BM_, TK> sb;
  if (kb < ke) {
    sa.load(g.A, g.a_m, g.a_k, m0, kb, tid);
    sb.load(g.B, g.b_n, g.b_k, n0, kb, tid);
  }
  for (int k0 = kb; k0 < ke; k0 += TK) {
    sa.store(As, tid);
    sb.store(Bs, tid);
    __syncthreads();
    if (k0 + TK < ke) {  // next slab in flight during the products
      sa.load(g.A, g.a_m, g.a_k, m0, k0 + TK, tid);
      sb.load(g.B, g.b_n, g.b_k, n0, k0 + TK, tid);
    }
#pragma unroll
    for (int ks = 0; ks < TK; ks += 32) {
      const int kk = ks + 8 * (lane >> 4);
      bf16x8_t af[FM], bfr[FN];
#pragma unroll
      for (int a = 0; a < FM; ++a) af[a] = *reinterpret_cast<const bf16x8_t*>(&As[wm + 16 * a + (lane & 15)][kk]);
#pragma unroll
      for (int b = 0; b < FN; ++b) bfr[b] = *reinterpret_cast<const bf16x8_t*>(&Bs[wn + 16 * b + (lane & 15)][kk]);
#pragma unroll
      for (int a = 0; a < FM; ++a)
#pragma unroll
        for (int b = 0; b < FN; ++b)
          acc[a][b] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(bfr[b], af[a], acc[a][b], 0, 0, 0);
    }
    __syncthreads();
  }
  // lane: row m = m0 + wm + 16 a + (lane % 16), columns n .. n + 3 with
  // n = n0 + wn + 16 b + 4 (lane / 16)
  float4_t csum[FN];
#pragma unroll
  for (int b = 0; b < FN; ++b) csum[b] = float4_t{0.f, 0.f, 0.f, 0.f};
#pragma unroll
  for (int a = 0; a < FM; ++a) {
    const int m = m0 + wm + 16 * a + (lane & 15);
#pragma unroll
    for (int b = 0; b < FN; ++b) {
      const int n = n0 + wn + 16 * b + 4 * (lane >> 4);
      float4_t v = acc[a][b];
      if (g.atomic) {
        float* o = g.C32 + (int64_t)m * g.c_m + n;
#pragma unroll
        for (int r = 0; r < 4; ++r) unsafeAtomicAdd(o + r, v[r]);
        continue;
      }
      if (g.vec) {
        if (g.bias) v += *reinterpret_cast<const float4_t*>(g.bias + n);
        if (g.relu) {
#pragma unroll
          for (int r = 0; r < 4; ++r) v[r] = v[r] > 0.f ? v[r] : 0.f;
        }
        if (g.gate) {
          const uint2 q = *reinterpret_cast<const uint2*>(g.gate + (int64_t)m * g.g_m + n);
          const uint32_t h[4] = {q.x << 16, q.x & 0xFFFF0000u, q.y << 16, q.y & 0xFFFF0000u};
#pragma unroll
          for (int r = 0; r < 4; ++r) v[r] = __uint_as_float(h[r]) > 0.f ? v[r] : 0.f;
        }
        csum[b] += v;
        if (g.C32) {
          float4_t* o = reinterpret_cast<float4_t*>(g.C32 + (int64_t)m * g.c_m + n);
          *o = g.accumulate ? *o + v : v;
        }
        if (g.C16) {
          uint2 q;
          q.x = (uint32_t)f32_to_bf16(v[0]) | ((uint32_t)f32_to_bf16(v[1]) << 16);
          q.y = (uint32_t)f32_to_bf16(v[2]) | ((uint32_t)f32_to_bf16(v[3]) << 16);
          *reinterpret_cast<uint2*>(g.C16 + (int64_t)m * g.c_m + n) = q;
        }
        continue;
      }
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        float x = v[r];
        if (g.bias) x += g.bias[n + r];
        if (g.relu) x = x > 0.f ? x : 0.f;
        if (g.gate && !(bf16_to_f32(g.gate[(int64_t)m * g.g_m + n + r]) > 0.f)) x = 0.f;
        csum[b][r] += x;
        if (g.C32) {
          float* o = &g.C32[(int64_t)m * g.c_m + n + r];
          *o = g.accumulate ? *o + x : x;
        }
        if (g.C16) g.C16[(int64_t)m * g.c_m + n + r] = f32_to_bf16(x);
      }
    }
  }
  if (g.colsum) {  // the 16 lanes with one lane / 16 hold the same 4 columns
#pragma unroll
    for (int b = 0; b < FN; ++b) {
      float4_t v = csum[b];
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        v[r] += __shfl_xor(v[r], 1);
        v[r] += __shfl_xor(v[r], 2);
        v[r] += __shfl_xor(v[r], 4);
        v[r] += __shfl_xor(v[r], 8);
      }
      if ((lane & 15) == 0) {
        const int n = n0 + wn + 16 * b + 4 * (lane >> 4);
#pragma unroll
        for (int r = 0; r < 4; ++r) unsafeAtomicAdd(&g.colsum[n + r], v[r]);
      }
    }
  }
}

// ------------------------------------------------------------- elementwise

// X[k][j] = +1 if bit j of mask k is 0 ('+'), -1 if it is 1, for j < n_bits;
// 0 for the padding columns n_bits <= j < width.
__global__ void k_encode(const uint64_t* __restrict__ masks, int64_t n, int n_bits, int width,
                         uint16_t* __restrict__ X) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n * width) return;
  const int64_t k = e / width;
  const int j = (int)(e % width);
  float v = 0.f;
  if (j < n_bits) v = ((masks[2 * k + (j >> 6)] >> (j & 63)) & 1) ? -1.f : 1.f;
  X[e] = f32_to_bf16(v);
}

// Feature classes of a scheme code (targets of the six softmax heads):
//   0: number of ovals, clamped to 22          (23 classes, logits 0..22)
//   1: deepest nesting level, clamped to 4     (5 classes,  logits 23..27)
//   2..5: number of ovals at depth 1..4, in buckets
//         0,1,2,3,4,5-6,7-9,10-14,15+          (9 classes each, logits 28..63)
// The depth of an oval is the running balance of the code word at its '1'
// (outermost = 1).
__device__ __forceinline__ int bucket9(int c) {
  return c <= 4 ? c : (c <= 6 ? 5 : (c <= 9 ? 6 : (c <= 14 ? 7 : 8)));
}

__global__ void k_features(const uint64_t* __restrict__ codes, int64_t n, int32_t* __restrict__ labels) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= n) return;
  const uint64_t lo = codes[2 * k], hi = codes[2 * k + 1] & ~(1ull << 63);
  const int len = hi ? 128 - __clzll((long long)hi) : 64 - __clzll((long long)lo);  // bit length of 2^|W| + W
  const int wl = len - 1;
  int depth = 0, maxd = 0, ovals = 0, cnt[4] = {0, 0, 0, 0};
  for (int b = wl - 1; b >= 0; --b) {
    const int bit = b >= 64 ? (int)((hi >> (b - 64)) & 1) : (int)((lo >> b) & 1);
    if (bit) {
      ++depth;
      ++ovals;
      maxd = depth > maxd ? depth : maxd;
      if (depth <= 4) ++cnt[depth - 1];
    } else {
      --depth;
    }
  }
  int32_t* o = labels + 6 * k;
  o[0] = ovals < 22 ? ovals : 22;
  o[1] = maxd < 4 ? maxd : 4;
  for (int h = 0; h < 4; ++h) o[2 + h] = bucket9(cnt[h]);
}

// Softmax cross-entropy over the six heads, averaged over the batch:
// loss += sum_h -log softmax(Y[k, head h])[label_h] / n and
// dY[k, head h] = (softmax - onehot) / n (fp32 and bf16 copies).
__constant__ int kHeadStart[7] = {0, 23, 28, 37, 46, 55, 64};

__global__ void k_softmax_xent(const float* __restrict__ Y, const int32_t* __restrict__ labels, int64_t n,
                               float* __restrict__ dY32, uint16_t* __restrict__ dY16, float* __restrict__ loss) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= n) return;
  const float* y = Y + 64 * k;
  float l = 0.f;
  for (int h = 0; h < 6; ++h) {
    const int s = kHeadStart[h], e = kHeadStart[h + 1];
    float mx = -INFINITY;
    for (int j = s; j < e; ++j) mx = fmaxf(mx, y[j]);
    float z = 0.f;
    for (int j = s; j < e; ++j) z += expf(y[j] - mx);
    const int t = labels[6 * k + h];
    l += logf(z) - (y[s + t] - mx);
    for (int j = s; j < e; ++j) {
      const float g = (expf(y[j] - mx) / z - (j - s == t ? 1.f : 0.f)) / (float)n;
      if (dY32) dY32[64 * k + j] = g;
      if (dY16) dY16[64 * k + j] = f32_to_bf16(g);
    }
  }
  atomicAdd(loss, l / (float)n);
}

// out[j] = sum_k X[k][j]  (bias gradients): block (x, y) sums rows
// [256 y, 256 y + 256) of columns [256 x, 256 x + 256) and adds its partial
// sums to out, which k_fill zeroed first.
constexpr int kColRows = 256;

__global__ void k_fill(float* __restrict__ x, int64_t n, float v) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) x[i] = v;
}

// C[m][n] = 0 for an M x N matrix with row stride ld
__global__ void k_fill2d(float* __restrict__ C, int M, int N, int64_t ld) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < (int64_t)M * N) C[(i / N) * ld + i % N] = 0.f;
}

__global__ void k_colsum(const float* __restrict__ X, int64_t n, int cols, float* __restrict__ out) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= cols) return;
  const int64_t r0 = (int64_t)blockIdx.y * kColRows;
  const int64_t r1 = r0 + kColRows < n ? r0 + kColRows : n;
  float s = 0.f;
  for (int64_t k = r0; k < r1; ++k) s += X[k * cols + j];
  atomicAdd(&out[j], s);
}

// Adam (Kingma & Ba, 2015) on fp32 master weights, refreshing the bf16 copy.
__global__ void k_adam(float* __restrict__ w, const float* __restrict__ g, float* __restrict__ m,
                       float* __restrict__ v, int64_t n, float lr, float b1, float b2, float eps, float bc1,
                       float bc2, uint16_t* __restrict__ w16) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const float gi = g[i];
  const float mi = b1 * m[i] + (1.f - b1) * gi;
  const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
  m[i] = mi;
  v[i] = vi;
  const float wi = w[i] - lr * (mi / bc1) / (sqrtf(vi / bc2) + eps);
  w[i] = wi;
  if (w16) w16[i] = f32_to_bf16(wi);
}

// Novelty score of a candidate: sum over heads of the expected rarity of
// its predicted class, sum_j softmax(Y)_j * rarity_j.
__global__ void k_score(const float* __restrict__ Y, const float* __restrict__ rarity, int64_t n,
                        float* __restrict__ score) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= n) return;
  const float* y = Y + 64 * k;
  float s = 0.f;
  for (int h = 0; h < 6; ++h) {
    const int a = kHeadStart[h], e = kHeadStart[h + 1];
    float mx = -INFINITY;
    for (int j = a; j < e; ++j) mx = fmaxf(mx, y[j]);
    float z = 0.f, acc = 0.f;
    for (int j = a; j < e; ++j) {
      const float p = expf(y[j] - mx);
      z += p;
      acc += p * rarity[j];
    }
    s += acc / z;
  }
  score[k] = s;
}

// counts[kHeadStart[h] + labels[k][h]] += 1 for every row k and head h
__global__ void k_label_counts(const int32_t* __restrict__ labels, int64_t n, uint32_t* __restrict__ counts) {
  __shared__ uint32_t c[64];
  if (threadIdx.x < 64) c[threadIdx.x] = 0;
  __syncthreads();
  for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < n; k += (int64_t)gridDim.x * blockDim.x)
    for (int h = 0; h < 6; ++h) atomicAdd(&c[kHeadStart[h] + labels[6 * k + h]], 1u);
  __syncthreads();
  if (threadIdx.x < 64 && c[threadIdx.x]) atomicAdd(&counts[threadIdx.x], c[threadIdx.x]);
}

// Gradient of the novelty score with respect to the logits: for head h with
// p = softmax(Y_h) and s_h = sum_j p_j rarity_j, d s_h / d Y_j =
// p_j (rarity_j - s_h).  Written as bf16 (the operand of the backward
// products).
__global__ void k_score_grad(const float* __restrict__ Y, const float* __restrict__ rarity, int64_t n,
                             uint16_t* __restrict__ dY16) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= n) return;
  const float* y = Y + 64 * k;
  for (int h = 0; h < 6; ++h) {
    const int a = kHeadStart[h], e = kHeadStart[h + 1];
    float mx = -INFINITY;
    for (int j = a; j < e; ++j) mx = fmaxf(mx, y[j]);
    float z = 0.f, acc = 0.f;
    for (int j = a; j < e; ++j) {
      const float p = expf(y[j] - mx);
      z += p;
      acc += p * rarity[j];
    }
    const float sh = acc / z;
    for (int j = a; j < e; ++j) dY16[64 * k + j] = f32_to_bf16(expf(y[j] - mx) / z * (rarity[j] - sh));
  }
}

// SplitMix64 finaliser as a counter-based generator: out(key) depends only
// on key (Steele, Lea, Flood 2014).
__device__ __forceinline__ uint64_t mix64(uint64_t z) {
  z += 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

// Candidate k = parent[k % n_parents] with `flips` random bits in
// [1, n_bits) toggled (bit 0, sigma(0,0), stays '+').
__global__ void k_mutate(const uint64_t* __restrict__ parents, int64_t n_parents, int64_t n, int n_bits, int flips,
                         uint64_t seed, uint64_t* __restrict__ out) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= n) return;
  const int64_t p = k % n_parents;
  uint64_t lo = parents[2 * p], hi = parents[2 * p + 1];
  for (int f = 0; f < flips; ++f) {
    const uint64_t r = mix64(seed ^ mix64((uint64_t)k * 0x100000001B3ull + (uint64_t)f));
    const int b = 1 + (int)(r % (uint64_t)(n_bits - 1));
    if (b < 64)
      lo ^= 1ull << b;
    else
      hi ^= 1ull << (b - 64);
  }
  out[2 * k] = lo;
  out[2 * k + 1] = hi;
}

// Flip distribution of each parent: cdf[p][j] = P(bit <= j) over bits
// 1 .. n_bits-1 with P(j) = (1 - explore) softmax_j(gain / (temp max|gain|))
// + explore / (n_bits - 1), where gain_j = -2 x_j dX[p][j] is the
// first-order change of the network's novelty score when bit j of the parent
// flips (x_j = +1 for '+', -1 for '-'; dX = d score / d input).  cdf[p][0] =
// 0; entries past n_bits - 1 are 1.
__global__ void k_flip_cdf(const uint64_t* __restrict__ parents, const float* __restrict__ dX, int64_t ldx,
                           int64_t n_parents, int n_bits, float temp, float explore, float* __restrict__ cdf) {
  const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= n_parents) return;
  const uint64_t lo = parents[2 * p], hi = parents[2 * p + 1];
  const float* g = dX + p * ldx;
  auto gain = [&](int j) {
    const uint64_t b = j < 64 ? (lo >> j) & 1 : (hi >> (j - 64)) & 1;
    return (b ? 2.f : -2.f) * g[j];
  };
  float gmax = -INFINITY, amax = 0.f;
  for (int j = 1; j < n_bits; ++j) {
    const float a = gain(j);
    gmax = fmaxf(gmax, a);
    amax = fmaxf(amax, fabsf(a));
  }
  const float inv = 1.f / (temp * amax + 1e-30f);
  float z = 0.f;
  for (int j = 1; j < n_bits; ++j) z += expf((gain(j) - gmax) * inv);
  float* c = cdf + p * 64;
  const float u = explore / (float)(n_bits - 1);
  float acc = 0.f;
  c[0] = 0.f;
  for (int j = 1; j < 64; ++j) {
    if (j < n_bits) acc += (1.f - explore) * expf((gain(j) - gmax) * inv) / z + u;
    c[j] = j < n_bits - 1 ? acc : 1.f;
  }
}

// Guided mutants: candidate k = parent p = k % n_parents with `flips` bits
// toggled, bit j drawn with probability cdf[p][j] - cdf[p][j-1] (inverse
// transform of a 24-bit uniform by binary search over the 64 entries).
__global__ void k_mutate_cdf(const uint64_t* __restrict__ parents, const float* __restrict__ cdf,
                             int64_t n_parents, int64_t n, int flips, uint64_t seed, uint64_t* __restrict__ out) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= n) return;
  const int64_t p = k % n_parents;
  uint64_t lo = parents[2 * p], hi = parents[2 * p + 1];
  const float* c = cdf + p * 64;
  for (int f = 0; f < flips; ++f) {
    const uint64_t r = mix64(seed ^ mix64((uint64_t)k * 0x100000001B3ull + (uint64_t)f));
    const float u = (float)(r >> 40) * (1.f / 16777216.f);
    int j = 0;  // largest j with c[j] <= u, then bit j + 1
#pragma unroll
    for (int step = 32; step > 0; step >>= 1)
      if (c[j + step] <= u) j += step;
    const int b = j + 1 < 64 ? j + 1 : 63;
    if (b < 64)
      lo ^= 1ull << b;
    else
      hi ^= 1ull << (b - 64);
  }
  out[2 * k] = lo;
  out[2 * k + 1] = hi;
}

// Uniform masks: word w of mask k is SplitMix64 output 2k + w of the stream
// started at `seed` (state seed + (i+1) * golden gamma), bits >= n_bits and
// bit 0 (sigma(0,0) = '+') cleared.
__global__ void k_random_masks(uint64_t seed, uint64_t offset, int64_t n, int n_bits, uint64_t* __restrict__ out) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= n) return;
  const uint64_t i = 2 * (offset + (uint64_t)k);
  uint64_t lo = mix64(seed + i * 0x9E3779B97F4A7C15ull);
  uint64_t hi = mix64(seed + (i + 1) * 0x9E3779B97F4A7C15ull);
  if (n_bits < 64) lo &= (1ull << n_bits) - 1;
  hi = n_bits <= 64 ? 0 : (n_bits < 128 ? hi & ((1ull << (n_bits - 64)) - 1) : hi);
  out[2 * k] = lo & ~1ull;
  out[2 * k + 1] = hi;
}

// counts[b] += #{k : lo + b w <= x[k] < lo + (b+1) w}, w = (hi - lo) / bins,
// values outside [lo, hi) clamped into the end bins
__global__ void k_bin_floats(const float* __restrict__ x, int64_t n, float lo, float hi, int bins,
                             unsigned int* __restrict__ counts) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= n) return;
  int b = (int)floorf((x[k] - lo) / (hi - lo) * (float)bins);
  b = b < 0 ? 0 : (b >= bins ? bins - 1 : b);
  atomicAdd(&counts[b], 1u);
}

// Keep the candidates scoring above `threshold`, in any order, up to cap.
__global__ void k_select(const float* __restrict__ score, const uint64_t* __restrict__ cand, int64_t n,
                         float threshold, uint64_t* __restrict__ out, int64_t cap,
                         unsigned long long* __restrict__ count) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= n || !(score[k] > threshold)) return;
  const unsigned long long slot = atomicAdd(count, 1ull);
  if ((int64_t)slot < cap) {
    out[2 * slot] = cand[2 * k];
    out[2 * slot + 1] = cand[2 * k + 1];
  }
}

__global__ void k_to_bf16(const float* __restrict__ x, int64_t n, uint16_t* __restrict__ y) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) y[i] = f32_to_bf16(x[i]);
}

// out[c][r] = in[r][c] for a rows x cols bf16 matrix, through 32 x 32 LDS
// tiles (reads and writes along rows of 32 consecutive elements)
__global__ void k_transpose_bf16(const uint16_t* __restrict__ in, int64_t rows, int64_t cols,
                                 uint16_t* __restrict__ out) {
  __shared__ uint16_t t[32][33];
  const int64_t r0 = (int64_t)blockIdx.y * 32, c0 = (int64_t)blockIdx.x * 32;
  const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;  // 256 threads: 8 rows at a time
  for (int k = ty; k < 32; k += 8)
    if (r0 + k < rows && c0 + tx < cols) t[k][tx] = in[(r0 + k) * cols + c0 + tx];
  __syncthreads();
  for (int k = ty; k < 32; k += 8)
    if (c0 + k < cols && r0 + tx < rows) out[(c0 + k) * rows + r0 + tx] = t[tx][k];
}

int grid1d(int64_t n, int threads) { return (int)((n + threads - 1) / threads); }

}  // namespace pw

using namespace pw;

extern "C" {

pw_status pw_mlp_gemm(const uint16_t* A, int64_t a_m, int64_t a_k, const uint16_t* B, int64_t b_k, int64_t b_n,
                      int32_t M, int32_t N, int32_t K, const float* bias, const uint16_t* gate, int64_t g_m,
                      int32_t relu, float* C32, uint16_t* C16, int64_t c_m, int32_t accumulate, float* colsum,
                      hipStream_t s) {
  if (!A || !B || (!C32 && !C16)) return set_err(PW_ERR_ARG, "null operand");
  if (M <= 0 || N <= 0 || K <= 0 || M % 64 || N % 64 || K % TBK)
    return set_err(PW_ERR_ARG, "gemm sizes must be positive multiples of 64 (M, N) and 32 (K): %d %d %d", M, N, K);
  if (accumulate && !C32) return set_err(PW_ERR_ARG, "accumulate needs the fp32 output");
  GemmArgs g{A, a_m, a_k, B, b_k, b_n, M, N, K, K, bias, gate, g_m, relu, C32, C16, c_m, accumulate, 0, colsum, 0};
  // 16-byte staging needs 8-element alignment of the base and the strides
  auto al = [](const void* p, int64_t s1) { return ((uintptr_t)p % 16 == 0) && (s1 % 8 == 0); };
  // 4-column epilogue accesses: 16 bytes of fp32, 8 bytes of bf16
  g.vec = (!bias || (uintptr_t)bias % 16 == 0) && (!gate || ((uintptr_t)gate % 8 == 0 && g_m % 4 == 0)) &&
          (!C32 || ((uintptr_t)C32 % 16 == 0 && c_m % 4 == 0)) && (!C16 || ((uintptr_t)C16 % 8 == 0 && c_m % 4 == 0));
  const int am = (a_k == 1 && al(A, a_m)) ? 1 : ((a_m == 1 && al(A, a_k)) ? 2 : 0);
  const int bm = (b_k == 1 && al(B, b_n)) ? 1 : ((b_n == 1 && al(B, b_k)) ? 2 : 0);
  const int tm = M % 128 == 0 ? 128 : 64, tn = N % 128 == 0 ? 128 : 64;
  const int tiles = (M / tm) * (N / tn);
  // split K when the output has too few tiles to fill 256 CUs and there is
  // no element-wise epilogue (partial sums are added atomically)
  // K slabs of 64 where K allows (half the global round trips), else 32
  const int tk = K % 64 == 0 ? 64 : 32;
  int splits = 1;
  const int ksteps = K / tk;
  if (C32 && !C16 && !bias && !gate && !relu && !colsum && tiles < 512 && ksteps >= 8) {
    splits = std::min(ksteps / 4, (1024 + tiles - 1) / tiles);
    const int per = (ksteps + splits - 1) / splits;
    g.k_split = per * tk;
    splits = (ksteps + per - 1) / per;
  }
  if (splits > 1) {
    g.atomic = 1;
    if (!accumulate) {
      hipLaunchKernelGGL(k_fill2d, dim3(grid1d((int64_t)M * N, 256)), dim3(256), 0, s, C32, M, N, c_m);
    }
  }
  const dim3 grid(N / tn, M / tm, splits);
#define PW_GEMM_MODES(BM_, BN_, TK_)                                                                   \
  switch (am * 3 + bm) {                                                                               \
    case 0: hipLaunchKernelGGL((k_gemm_bf16<BM_, BN_, 0, 0, TK_>), grid, dim3(256), 0, s, g); break; \
    case 1: hipLaunchKernelGGL((k_gemm_bf16<BM_, BN_, 0, 1, TK_>), grid, dim3(256), 0, s, g); break; \
    case 2: hipLaunchKernelGGL((k_gemm_bf16<BM_, BN_, 0, 2, TK_>), grid, dim3(256), 0, s, g); break; \
    case 3: hipLaunchKernelGGL((k_gemm_bf16<BM_, BN_, 1, 0, TK_>), grid, dim3(256), 0, s, g); break; \
    case 4: hipLaunchKernelGGL((k_gemm_bf16<BM_, BN_, 1, 1, TK_>), grid, dim3(256), 0, s, g); break; \
    case 5: hipLaunchKernelGGL((k_gemm_bf16<BM_, BN_, 1, 2, TK_>), grid, dim3(256), 0, s, g); break; \
    case 6: hipLaunchKernelGGL((k_gemm_bf16<BM_, BN_, 2, 0, TK_>), grid, dim3(256), 0, s, g); break; \
    case 7: hipLaunchKernelGGL((k_gemm_bf16<BM_, BN_, 2, 1, TK_>), grid, dim3(256), 0, s, g); break; \
    default: hipLaunchKernelGGL((k_gemm_bf16<BM_, BN_, 2, 2, TK_>), grid, dim3(256), 0, s, g); break; \
  }
#define PW_GEMM_CASES(BM_, BN_)    \
  if (tk == 64) {                  \
    PW_GEMM_MODES(BM_, BN_, 64)    \
  } else {                         \
    PW_GEMM_MODES(BM_, BN_, 32)    \
  }
  if (tm == 128 && tn == 128) {
    PW_GEMM_CASES(128, 128)
  } else if (tm == 128) {
    PW_GEMM_CASES(128, 64)
  } else if (tn == 128) {
    PW_GEMM_CASES(64, 128)
  } else {
    PW_GEMM_CASES(64, 64)
  }
#undef PW_GEMM_CASES
#undef PW_GEMM_MODES
  PW_HIP(hipGetLastError());
  return PW_OK;
}

pw_status pw_mlp_encode(const uint64_t* masks, int64_t n, int32_t n_bits, int32_t width, uint16_t* X,
                        hipStream_t s) {
  if (n < 0 || n_bits < 1 || n_bits > 128 || width < n_bits) return set_err(PW_ERR_ARG, "bad encode sizes");
  if (n == 0) return PW_OK;
  if (!masks || !X) return set_err(PW_ERR_ARG, "null buffer");
  hipLaunchKernelGGL(k_encode, dim3(grid1d(n * width, 256)), dim3(256), 0, s, masks, n, n_bits, width, X);
  PW_HIP(hipGetLastError());
  return PW_OK;
}

pw_status pw_features(const uint64_t* codes, int64_t n, int32_t* labels, hipStream_t s) {
  if (n < 0) return set_err(PW_ERR_ARG, "negative count");
  if (n == 0) return PW_OK;
  if (!codes || !labels) return set_err(PW_ERR_ARG, "null buffer");
  hipLaunchKernelGGL(k_features, dim3(grid1d(n, 256)), dim3(256), 0, s, codes, n, labels);
  PW_HIP(hipGetLastError());
  return PW_OK;
}

pw_status pw_mlp_softmax_xent(const float* Y, const int32_t* labels, int64_t n, float* dY32, uint16_t* dY16,
                              float* loss, hipStream_t s) {
  if (n <= 0 || !Y || !labels || !loss) return set_err(PW_ERR_ARG, "bad loss arguments");
  hipLaunchKernelGGL(k_softmax_xent, dim3(grid1d(n, 256)), dim3(256), 0, s, Y, labels, n, dY32, dY16, loss);
  PW_HIP(hipGetLastError());
  return PW_OK;
}

pw_status pw_mlp_colsum(const float* X, int64_t n, int32_t cols, float* out, int32_t accumulate, hipStream_t s) {
  if (n < 0 || cols <= 0 || !X || !out) return set_err(PW_ERR_ARG, "bad colsum arguments");
  if (!accumulate) hipLaunchKernelGGL(k_fill, dim3(grid1d(cols, 256)), dim3(256), 0, s, out, (int64_t)cols, 0.f);
  if (n == 0) return PW_OK;
  hipLaunchKernelGGL(k_colsum, dim3(grid1d(cols, 256), (unsigned)((n + kColRows - 1) / kColRows)), dim3(256), 0, s,
                     X, n, cols, out);
  PW_HIP(hipGetLastError());
  return PW_OK;
}

pw_status pw_mlp_adam(float* w, const float* g, float* m, float* v, int64_t n, float lr, float beta1, float beta2,
                      float eps, int32_t step, uint16_t* w16, hipStream_t s) {
  if (n <= 0 || step < 1 || !w || !g || !m || !v) return set_err(PW_ERR_ARG, "bad adam arguments");
  const float bc1 = 1.f - std::pow(beta1, (float)step), bc2 = 1.f - std::pow(beta2, (float)step);
  hipLaunchKernelGGL(k_adam, dim3(grid1d(n, 256)), dim3(256), 0, s, w, g, m, v, n, lr, beta1, beta2, eps, bc1, bc2,
                     w16);
  PW_HIP(hipGetLastError());
  return PW_OK;
}

pw_status pw_label_counts(const int32_t* labels, int64_t n, uint32_t* counts, hipStream_t s) {
  if (n < 0 || !labels || !counts) return set_err(PW_ERR_ARG, "bad label-count arguments");
  if (n == 0) return PW_OK;
  const int blocks = (int)std::min<int64_t>(grid1d(n, 256), 1024);
  hipLaunchKernelGGL(k_label_counts, dim3(blocks), dim3(256), 0, s, labels, n, counts);
  PW_HIP(hipGetLastError());
  return PW_OK;
}

pw_status pw_fill_f32(float* x, int64_t n, float v, hipStream_t s) {
  if (n < 0 || (n > 0 && !x)) return set_err(PW_ERR_ARG, "bad fill arguments");
  if (n == 0) return PW_OK;
  hipLaunchKernelGGL(k_fill, dim3(grid1d(n, 256)), dim3(256), 0, s, x, n, v);
  PW_HIP(hipGetLastError());
  return PW_OK;
}

pw_status pw_mlp_score_grad(const float* Y, const float* rarity, int64_t n, uint16_t* dY16, hipStream_t s) {
  if (n < 0 || !Y || !rarity || !dY16) return set_err(PW_ERR_ARG, "bad score-gradient arguments");
  if (n == 0) return PW_OK;
  hipLaunchKernelGGL(k_score_grad, dim3(grid1d(n, 256)), dim3(256), 0, s, Y, rarity, n, dY16);
  PW_HIP(hipGetLastError());
  return PW_OK;
}

pw_status pw_flip_cdf(const uint64_t* parents, const float* dX, int64_t ldx, int64_t n_parents, int32_t n_bits,
                      float temp, float explore, float* cdf, hipStream_t s) {
  if (n_parents < 0 || n_bits < 2 || n_bits > 64 || ldx < n_bits || !(temp > 0.f) || !(explore >= 0.f) ||
      !(explore <= 1.f) || !parents || !dX || !cdf)
    return set_err(PW_ERR_ARG, "bad flip-distribution arguments");
  if (n_parents == 0) return PW_OK;
  hipLaunchKernelGGL(k_flip_cdf, dim3(grid1d(n_parents, 64)), dim3(64), 0, s, parents, dX, ldx, n_parents, n_bits,
                     temp, explore, cdf);
  PW_HIP(hipGetLastError());
  return PW_OK;
}

pw_status pw_mutate_cdf(const uint64_t* parents, const float* cdf, int64_t n_parents, int64_t n, int32_t flips,
                        uint64_t seed, uint64_t* out, hipStream_t s) {
  if (n < 0 || n_parents <= 0 || flips < 0 || !parents || !cdf || !out)
    return set_err(PW_ERR_ARG, "bad guided-mutation arguments");
  if (n == 0) return PW_OK;
  hipLaunchKernelGGL(k_mutate_cdf, dim3(grid1d(n, 256)), dim3(256), 0, s, parents, cdf, n_parents, n, flips, seed,
                     out);
  PW_HIP(hipGetLastError());
  return PW_OK;
}

pw_status pw_to_bf16(const float* x, int64_t n, uint16_t* y, hipStream_t s) {
  if (n < 0 || !x || !y) return set_err(PW_ERR_ARG, "bad conversion arguments");
  if (n == 0) return PW_OK;
  hipLaunchKernelGGL(k_to_bf16, dim3(grid1d(n, 256)), dim3(256), 0, s, x, n, y);
  PW_HIP(hipGetLastError());
  return PW_OK;
}

pw_status pw_bf16_transpose(const uint16_t* in, int64_t rows, int64_t cols, uint16_t* out, hipStream_t s) {
  if (rows < 0 || cols < 0 || rows > 65535ll * 32 || cols > 2147483647ll * 32)
    return set_err(PW_ERR_ARG, "bad transpose sizes %lld x %lld", (long long)rows, (long long)cols);
  if (rows == 0 || cols == 0) return PW_OK;
  if (!in || !out || in == out) return set_err(PW_ERR_ARG, "null or aliased buffers");
  const dim3 grid((unsigned)((cols + 31) / 32), (unsigned)((rows + 31) / 32));
  hipLaunchKernelGGL(k_transpose_bf16, grid, dim3(256), 0, s, in, rows, cols, out);
  PW_HIP(hipGetLastError());
  return PW_OK;
}

pw_status pw_mlp_score(const float* Y, const float* rarity, int64_t n, float* score, hipStream_t s) {
  if (n < 0 || !Y || !rarity || !score) return set_err(PW_ERR_ARG, "bad score arguments");
  if (n == 0) return PW_OK;
  hipLaunchKernelGGL(k_score, dim3(grid1d(n, 256)), dim3(256), 0, s, Y, rarity, n, score);
  PW_HIP(hipGetLastError());
  return PW_OK;
}

pw_status pw_mutate(const uint64_t* parents, int64_t n_parents, int64_t n, int32_t n_bits, int32_t flips,
                    uint64_t seed, uint64_t* out, hipStream_t s) {
  if (n < 0 || n_parents <= 0 || n_bits < 2 || n_bits > 128 || flips < 0 || !parents || !out)
    return set_err(PW_ERR_ARG, "bad mutate arguments");
  if (n == 0) return PW_OK;
  hipLaunchKernelGGL(k_mutate, dim3(grid1d(n, 256)), dim3(256), 0, s, parents, n_parents, n, n_bits, flips, seed,
                     out);
  PW_HIP(hipGetLastError());
  return PW_OK;
}

pw_status pw_random_masks(uint64_t seed, uint64_t offset, int64_t n, int32_t n_bits, uint64_t* out, hipStream_t s) {
  if (n < 0 || n_bits < 1 || n_bits > 128 || !out) return set_err(PW_ERR_ARG, "bad random mask arguments");
  if (n == 0) return PW_OK;
  hipLaunchKernelGGL(k_random_masks, dim3(grid1d(n, 256)), dim3(256), 0, s, seed, offset, n, n_bits, out);
  PW_HIP(hipGetLastError());
  return PW_OK;
}

pw_status pw_bin_floats(const float* x, int64_t n, float lo, float hi, int32_t bins, uint32_t* counts,
                        hipStream_t s) {
  if (n < 0 || bins < 1 || !(hi > lo) || !x || !counts) return set_err(PW_ERR_ARG, "bad binning arguments");
  if (n == 0) return PW_OK;
  hipLaunchKernelGGL(k_bin_floats, dim3(grid1d(n, 256)), dim3(256), 0, s, x, n, lo, hi, bins, counts);
  PW_HIP(hipGetLastError());
  return PW_OK;
}

pw_status pw_select(const float* score, const uint64_t* cand, int64_t n, float threshold, uint64_t* out,
                    int64_t cap, unsigned long long* count, hipStream_t s) {
  if (n < 0 || cap < 0 || !score || !cand || !out || !count) return set_err(PW_ERR_ARG, "bad select arguments");
  if (n == 0) return PW_OK;
  hipLaunchKernelGGL(k_select, dim3(grid1d(n, 256)), dim3(256), 0, s, score, cand, n, threshold, out, cap, count);
  PW_HIP(hipGetLastError());
  return PW_OK;
}

}  // extern "C"
