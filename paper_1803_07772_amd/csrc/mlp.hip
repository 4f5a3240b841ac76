// Warm-start network for the allocator (include/alloc_mlp.h): features,
// BF16 matrix-core GEMMs with fused bias/GELU epilogues, backward pass,
// AdamW, pooling into a warm start, and the warm-started solves.
//
// GEMMs run on the gfx950 matrix cores (v_mfma_f32_16x16x32_bf16): a
// workgroup of four waves computes a 64x64 tile of C = X Y, each wave a 32x32
// quarter as 2x2 blocks of 16x16.  Operand tiles of 64x32 are staged in LDS
// with the contraction index contiguous, so each lane reads its eight bf16
// operands as one 16-byte load.  Operand strides are arbitrary (the same
// kernel serves X W^T, dZ W and dZ^T A), and the global loads walk whichever
// index is contiguous in memory so they coalesce.  Weight gradients reduce
// over rows with a fixed split into chunks and an ordered sum of the chunk
// partials, so training steps are deterministic.

#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <string>
#include <vector>

#include "alloc.h"
#include "alloc_mlp.h"
#include "ctx.h"

namespace {

typedef __bf16 bf16;
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

constexpr int kIn = ALLOC_MLP_NIN, kHid = ALLOC_MLP_HID, kOut = ALLOC_MLP_NOUT;
// offsets of the FP32 parameter vector
constexpr int64_t kOW[5] = {0, 0, 1280, 67072, 132864};
constexpr int64_t kOB[5] = {0, 1024, 66816, 132608, 133632};
constexpr int64_t kNP = ALLOC_MLP_NPARAMS;
// offsets of the BF16 weight copies
constexpr int64_t kQW[5] = {0, 0, 1024, 66560, 132096};
constexpr int64_t kNQ = 132864;
constexpr int kLayerIn[5] = {0, kIn, kHid, kHid, kHid};
constexpr int kLayerOut[5] = {0, kHid, kHid, kHid, kOut};
constexpr float kGc = 0.7978845608028654f;  // sqrt(2/pi)
constexpr double kQMin = 0.1, kLogClip = 30.0;
constexpr double kDecades = 6.0;  // power code: 1 + log10(p/pmask)/kDecades
constexpr int64_t kChunk = 1 << 20;  // rows per inference chunk

// ----------------------------------------------------------------- helpers

// GELU, tanh form: 0.5 z (1 + tanh u) = z sigmoid(2u), u = sqrt(2/pi)(z + 0.044715 z^3).
__device__ inline float gelu(float z) {
  const float u = kGc * (z + 0.044715f * z * z * z);
  return z / (1.0f + __expf(-2.0f * u));
}

// d/dz of the tanh-form GELU: s + 2 z s (1 - s) u'(z), s = sigmoid(2u).
__device__ inline float gelu_grad(float z) {
  const float u = kGc * (z + 0.044715f * z * z * z);
  const float s = 1.0f / (1.0f + __expf(-2.0f * u));
  return s + 2.0f * z * s * (1.0f - s) * kGc * (1.0f + 3.0f * 0.044715f * z * z);
}

__device__ inline bf16 to_bf16(float x) { return (bf16)x; }  // round to nearest even

// ------------------------------------------------------------------- GEMM

enum Epi : int {
  kEpiHidTrain = 0,  // z = acc + b -> Zf (fp32) and Ab = bf16(gelu(z))
  kEpiHidInfer = 1,  // Ab = bf16(gelu(acc + b))
  kEpiOut = 2,       // Zf = acc + b
  kEpiBwd = 3,       // Ab = bf16(acc * gelu'(Zprev))
  kEpiPart = 4,      // Zf[split][i][j] = acc
};

struct GemmArgs {
  const bf16* X;
  int64_t xs_i, xs_p;  // X(i, p) = X[i xs_i + p xs_p]
  const bf16* Y;
  int64_t ys_p, ys_j;  // Y(p, j) = Y[p ys_p + j ys_j]
  int64_t I, J, P;     // C is I x J, contraction over P
  int64_t ones_col;    // column j == ones_col reads Y(p, j) = 1 (or -1: none)
  int64_t pchunk;      // contraction range of one split (multiple of 32)
  int epi;
  const float* bias;   // [J]
  float* Zf;
  bf16* Ab;
  const float* Zprev;
  int64_t ldc;
};

constexpr int kTile = 64, kKs = 32, kPad = 40;  // LDS row: 32 bf16 + 8 pad (80 bytes)

__device__ inline bf16 load_x(const GemmArgs& a, int64_t i, int64_t p, int64_t pend) {
  return (i < a.I && p < pend) ? a.X[i * a.xs_i + p * a.xs_p] : to_bf16(0.0f);
}

__device__ inline bf16 load_y(const GemmArgs& a, int64_t p, int64_t j, int64_t pend) {
  if (p >= pend || j >= a.J) return to_bf16(0.0f);
  if (j == a.ones_col) return to_bf16(1.0f);
  return a.Y[p * a.ys_p + j * a.ys_j];
}

// Tile element e of this thread (0..7): row r in [0,64), contraction c in [0,32).
// When the contraction index is contiguous in memory, consecutive threads walk
// it; otherwise they walk the row index.
__device__ inline void tile_pos(bool c_fast, int e, int& r, int& c) {
  const int lin = threadIdx.x + 256 * e;
  if (c_fast) {
    r = lin >> 5;
    c = lin & 31;
  } else {
    c = lin >> 6;
    r = lin & 63;
  }
}

__global__ void __launch_bounds__(256) gemm_kernel(GemmArgs a) {
  __shared__ __align__(16) bf16 xs[kTile][kPad];
  __shared__ __align__(16) bf16 ys[kTile][kPad];  // ys[j][p]: transposed
  const int64_t i0 = (int64_t)blockIdx.x * kTile, j0 = (int64_t)blockIdx.y * kTile;
  const int64_t pbeg = (int64_t)blockIdx.z * a.pchunk;
  const int64_t pend = std::min(a.P, pbeg + a.pchunk);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int wr = wave >> 1, wc = wave & 1;
  const bool xc = a.xs_p == 1, yc = a.ys_p == 1;
  f32x4 acc[2][2];
  for (int u = 0; u < 2; ++u)
    for (int v = 0; v < 2; ++v) acc[u][v] = f32x4{0.0f, 0.0f, 0.0f, 0.0f};
  bf16 rx[8], ry[8];
  auto fetch = [&](int64_t p0) {
    for (int e = 0; e < 8; ++e) {
      int r, c;
      tile_pos(xc, e, r, c);
      rx[e] = load_x(a, i0 + r, p0 + c, pend);
      tile_pos(yc, e, r, c);
      ry[e] = load_y(a, p0 + c, j0 + r, pend);
    }
  };
  if (pbeg < pend) fetch(pbeg);
  for (int64_t p0 = pbeg; p0 < pend; p0 += kKs) {
    for (int e = 0; e < 8; ++e) {
      int r, c;
      tile_pos(xc, e, r, c);
      xs[r][c] = rx[e];
      tile_pos(yc, e, r, c);
      ys[r][c] = ry[e];
    }
    __syncthreads();
    if (p0 + kKs < pend) fetch(p0 + kKs);  // next tile's loads overlap the products
    bf16x8 fa[2], fb[2];
    for (int u = 0; u < 2; ++u)
      fa[u] = *reinterpret_cast<const bf16x8*>(&xs[wr * 32 + u * 16 + (lane & 15)][8 * (lane >> 4)]);
    for (int v = 0; v < 2; ++v)
      fb[v] = *reinterpret_cast<const bf16x8*>(&ys[wc * 32 + v * 16 + (lane & 15)][8 * (lane >> 4)]);
    for (int u = 0; u < 2; ++u)
      for (int v = 0; v < 2; ++v) acc[u][v] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(fa[u], fb[v], acc[u][v], 0, 0, 0);
    __syncthreads();
  }
  // lane holds C[row 4 (lane/16) + q][col lane % 16] of each 16x16 block
  for (int u = 0; u < 2; ++u)
    for (int v = 0; v < 2; ++v)
      for (int q = 0; q < 4; ++q) {
        const int64_t i = i0 + wr * 32 + u * 16 + 4 * (lane >> 4) + q;
        const int64_t j = j0 + wc * 32 + v * 16 + (lane & 15);
        if (i >= a.I || j >= a.J) continue;
        const float c = acc[u][v][q];
        const int64_t o = i * a.ldc + j;
        switch (a.epi) {
          case kEpiHidTrain: {
            const float z = c + a.bias[j];
            a.Zf[o] = z;
            a.Ab[o] = to_bf16(gelu(z));
            break;
          }
          case kEpiHidInfer:
            a.Ab[o] = to_bf16(gelu(c + a.bias[j]));
            break;
          case kEpiOut:
            a.Zf[o] = c + a.bias[j];
            break;
          case kEpiBwd:
            a.Ab[o] = to_bf16(c * gelu_grad(a.Zprev[o]));
            break;
          default:
            a.Zf[(int64_t)blockIdx.z * a.I * a.ldc + o] = c;
            break;
        }
      }
}

// ------------------------------------------------------ fused inference
//
// One wave carries 32 rows (two blocks of 16) through all four layers with
// the activations in registers.  Each product is computed transposed,
// H^T = W A^T: the weights are the matrix cores' A operand (16 outputs x 32
// inputs) and the activations the B operand (32 inputs x 16 rows).  A 16x16
// output block leaves lane l holding outputs 4(l/16)+q (q < 4) of row l%16;
// two consecutive blocks give that lane 8 values of one row, which is its B
// operand for a 32-input chunk of the next layer once the chunk's inputs are
// taken in the order (32c + 4g + j, j < 4; 32c + 16 + 4g + j - 4, j >= 4),
// g = l/16.  The weight fragments are stored in that order, 16 bytes per
// lane, so each operand is one coalesced load.

// Input of k-slot j of lane group g in chunk c.
__host__ __device__ inline int frag_in(int c, int g, int j) {
  return 32 * c + (j < 4 ? 4 * g + j : 16 + 4 * g + j - 4);
}

constexpr int64_t kFragHid = 16 * 8 * 64;  // bf16x8 fragments of a 256x256 layer
constexpr int64_t kFragOut = 8 * 64;       // of the 256 -> 3 layer, outputs padded to 16

// Fragments of W2, W3 (kFragHid each) and W4 (kFragOut) from the master weights.
__global__ void pack_frags_kernel(const float* master, bf16x8* frag) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= 2 * kFragHid + kFragOut) return;
  int layer;
  int64_t f;
  if (t < 2 * kFragHid) {
    layer = t < kFragHid ? 2 : 3;
    f = t % kFragHid;
  } else {
    layer = 4;
    f = t - 2 * kFragHid;
  }
  const int lane = (int)(f % 64), c = (int)((f / 64) % 8), ob = layer == 4 ? 0 : (int)(f / (64 * 8));
  const int g = lane >> 4, out = 16 * ob + (lane & 15);
  bf16x8 v;
  for (int j = 0; j < 8; ++j) {
    const int in = frag_in(c, g, j);
    float w = 0.0f;
    if (layer < 4)
      w = master[kOW[layer] + (int64_t)out * kHid + in];
    else if (out < kOut)
      w = master[kOW[4] + (int64_t)out * kHid + in];
    v[j] = to_bf16(w);
  }
  frag[t] = v;
}

// GELU of the fused inference: the same tanh form with a hardware reciprocal.
__device__ inline float gelu_rcp(float z) {
  const float u = kGc * (z + 0.044715f * z * z * z);
  return z * __frcp_rn(1.0f + __expf(-2.0f * u));
}

__device__ inline f32x4 mfma16(const bf16x8& a, const bf16x8& b, const f32x4& c) {
  return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
}

// One hidden layer on kR row blocks: out[r][chunk] from in[r][chunk].
template <int kR>
__device__ inline void fused_hidden(const bf16x8* __restrict__ wl, const float* __restrict__ bias, int lane,
                                    const bf16x8 (&in)[kR][8], bf16x8 (&out)[kR][8]) {
  const int g = lane >> 4;
#pragma unroll
  for (int ob = 0; ob < 16; ++ob) {
    f32x4 acc[kR];
#pragma unroll
    for (int r = 0; r < kR; ++r) acc[r] = f32x4{0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
    for (int c = 0; c < 8; ++c) {
      const bf16x8 a = wl[(ob * 8 + c) * 64];
#pragma unroll
      for (int r = 0; r < kR; ++r) acc[r] = mfma16(a, in[r][c], acc[r]);
    }
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const float b = bias[16 * ob + 4 * g + q];
#pragma unroll
      for (int r = 0; r < kR; ++r) out[r][ob >> 1][(ob & 1) * 4 + q] = to_bf16(gelu_rcp(acc[r][q] + b));
    }
    // keep each output block's fragment loads next to their products (the
    // unrolled layer would otherwise hoist all 128 loads and spill)
    __builtin_amdgcn_sched_barrier(0);
  }
}

// Row blocks of 16 per wave: each weight fragment loaded feeds kFusedR
// products.  Two take 168 VGPRs and no scratch (three waves per SIMD); one
// or three were slower on 16.8 M rows (13.0 and 12.2 ms against 10.7).
constexpr int kFusedR = 2;

// y [n][3] from bf16 inputs x0 [n][4]; persistent over blocks of 16 kFusedR
// rows per wave.
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2))) mlp_fused_kernel(const bf16* __restrict__ x0, int64_t n,
                                                        const float* __restrict__ master,
                                                        const bf16x8* __restrict__ frag, float* __restrict__ y) {
  constexpr int R = kFusedR, RB = 16 * kFusedR;
  const int lane = threadIdx.x & 63, g = lane >> 4, rl = lane & 15;
  const int64_t wave = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6), nw = (int64_t)gridDim.x * 4;
  const float* W1 = master + kOW[1];
  const float* b1 = master + kOB[1];
  for (int64_t base = wave * RB; base < n; base += nw * RB) {
    // the weights are invariant in this loop: a compiler barrier keeps them
    // loaded where they are used instead of hoisted (and spilled) ahead of it
    asm volatile("" ::: "memory");
    // the lane's fragment offset, opaque to the compiler inside each pass:
    // addresses are formed where they are used
    int lo = lane;
    asm volatile("" : "+v"(lo));
    const bf16x8* wl = frag + lo;
    const int go = lo >> 4;  // g, opaque too: the bias and W1 addresses stay in the pass
    bf16x8 a[R][8], b[R][8];
    // layer 1 (4 inputs) on the vector units, into the B-operand layout
    float x[R][4];
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const int64_t row = base + 16 * r + rl;
#pragma unroll
      for (int p = 0; p < 4; ++p) x[r][p] = row < n ? (float)x0[row * 4 + p] : 0.0f;
    }
#pragma unroll
    for (int f = 0; f < 16; ++f) {
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int o = 16 * f + 4 * go + q;
        const float4 w = *reinterpret_cast<const float4*>(W1 + o * 4);
        const float wb[4] = {(float)to_bf16(w.x), (float)to_bf16(w.y), (float)to_bf16(w.z), (float)to_bf16(w.w)};
        const float bo = b1[o];
#pragma unroll
        for (int r = 0; r < R; ++r) {
          float z = bo;
#pragma unroll
          for (int p = 0; p < 4; ++p) z = fmaf(wb[p], x[r][p], z);
          a[r][f >> 1][(f & 1) * 4 + q] = to_bf16(gelu_rcp(z));
        }
      }
      __builtin_amdgcn_sched_barrier(0);
    }
    fused_hidden<R>(wl, master + kOB[2], lo, a, b);
    fused_hidden<R>(wl + kFragHid, master + kOB[3], lo, b, a);
    // layer 4: outputs padded to 16, the first three kept
    f32x4 acc[R];
#pragma unroll
    for (int r = 0; r < R; ++r) acc[r] = f32x4{0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
    for (int c = 0; c < 8; ++c) {
      const bf16x8 w = wl[2 * kFragHid + c * 64];
#pragma unroll
      for (int r = 0; r < R; ++r) acc[r] = mfma16(w, a[r][c], acc[r]);
    }
    if (g == 0) {
      const float* b4 = master + kOB[4];
#pragma unroll
      for (int r = 0; r < R; ++r) {
        const int64_t row = base + 16 * r + rl;
        if (row < n)
          for (int q = 0; q < kOut; ++q) y[row * 3 + q] = acc[r][q] + b4[q];
      }
    }
  }
}

// Weight gradient of one layer from its split partials [S][out][in+1], summed
// in split order; column `in` is the bias gradient.
__global__ void reduce_split_kernel(const float* part, int S, int out, int in, float* gW, float* gb) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  const int J = in + 1;
  if (t >= out * J) return;
  float s = 0.0f;
  for (int z = 0; z < S; ++z) s += part[(int64_t)z * out * J + t];
  const int o = t / J, j = t - o * J;
  if (j < in)
    gW[(int64_t)o * in + j] = s;
  else
    gb[o] = s;
}

// ------------------------------------------------------ elementwise kernels

__global__ void cast_weights_kernel(const float* master, bf16* q) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  for (int l = 1; l <= 4; ++l) {
    const int64_t n = (int64_t)kLayerIn[l] * kLayerOut[l];
    if (t < n) q[kQW[l] + t] = to_bf16(master[kOW[l] + t]);
  }
}

__global__ void cast_rows_kernel(const float* x, bf16* out, int64_t n) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t < n) out[t] = to_bf16(x[t]);
}

// Per-row loss and dL/dy / R (bf16); per-block loss sums in a fixed order.
__global__ void __launch_bounds__(256) loss_kernel(const float* y, const float* T, const float* W, int64_t R,
                                                   bf16* dy, double* block_loss) {
  __shared__ double red[256];
  const int64_t r = (int64_t)blockIdx.x * 256 + threadIdx.x;
  double l = 0.0;
  if (r < R) {
    const float y0 = y[r * 3], t0 = T[r * 3];
    const float sig = 1.0f / (1.0f + __expf(-y0));
    const float bce = fmaxf(y0, 0.0f) - y0 * t0 + log1pf(__expf(-fabsf(y0)));
    const float e1 = y[r * 3 + 1] - T[r * 3 + 1], e2 = y[r * 3 + 2] - T[r * 3 + 2];
    const float w0 = W[r * 3], w1 = W[r * 3 + 1], w2 = W[r * 3 + 2];
    l = (double)(w0 * bce) + (double)(w1 * e1 * e1) + (double)(w2 * e2 * e2);
    const float inv = 1.0f / (float)R;
    dy[r * 3] = to_bf16(w0 * (sig - t0) * inv);
    dy[r * 3 + 1] = to_bf16(2.0f * w1 * e1 * inv);
    dy[r * 3 + 2] = to_bf16(2.0f * w2 * e2 * inv);
  }
  red[threadIdx.x] = l;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if (threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
    __syncthreads();
  }
  if (threadIdx.x == 0) block_loss[blockIdx.x] = red[0];
}

__global__ void __launch_bounds__(256) sum_kernel(const double* x, int64_t n, double* out) {
  __shared__ double red[256];
  double s = 0.0;
  for (int64_t i = threadIdx.x; i < n; i += 256) s += x[i];
  red[threadIdx.x] = s;
  __syncthreads();
  for (int k = 128; k > 0; k >>= 1) {
    if (threadIdx.x < k) red[threadIdx.x] += red[threadIdx.x + k];
    __syncthreads();
  }
  if (threadIdx.x == 0) *out = red[0];
}

// AdamW with decoupled weight decay on the weight matrices.
__global__ void adamw_kernel(float* theta, float* m, float* v, const float* g, float lr, float b1, float b2,
                             float eps, float wd, float bc1, float bc2) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= kNP) return;
  const bool is_bias = (t >= kOB[1] && t < kOW[2]) || (t >= kOB[2] && t < kOW[3]) ||
                       (t >= kOB[3] && t < kOW[4]) || t >= kOB[4];
  const float gt = g[t];
  const float mt = b1 * m[t] + (1.0f - b1) * gt;
  const float vt = b2 * v[t] + (1.0f - b2) * gt * gt;
  m[t] = mt;
  v[t] = vt;
  const float mh = mt / bc1, vh = vt / bc2;
  const float th = theta[t];
  theta[t] = th - lr * (mh / (sqrtf(vh) + eps) + (is_bias ? 0.0f : wd) * th);
}

// Per-drop constants of the feature map.
struct FeatDrop {
  int M, N, K;
  const float* G;          // [M][N][K]
  const double* snr_scale; // [M] pmask_m / sigma
  const float* f3;         // [M] centred budget in dBm
  const float* f1;         // [K] streaming flag
  const float* f2;         // [K] minimum rate
  const double* pmask;     // [M]
};

__device__ inline void triple_features(const FeatDrop& d, int64_t idx, float out[4]) {
  const int64_t NK = (int64_t)d.N * d.K;
  const int m = (int)(idx / NK), k = (int)(idx % d.K);
  out[0] = (float)((10.0 * log10((double)d.G[idx] * d.snr_scale[m]) - 20.0) / 20.0);
  out[1] = d.f1[k];
  out[2] = d.f2[k];
  out[3] = d.f3[m];
}

// Features of rows [r0, r0 + n) of the drop; fp32 out and/or bf16 out.
__global__ void features_kernel(FeatDrop d, int64_t r0, int64_t n, float* outf, bf16* outb) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= n) return;
  float f[4];
  triple_features(d, r0 + t, f);
  for (int c = 0; c < 4; ++c) {
    if (outf) outf[t * 4 + c] = f[c];
    if (outb) outb[t * 4 + c] = to_bf16(f[c]);
  }
}

// Training rows: features, targets and loss weights of sampled triples.
__global__ void rows_kernel(FeatDrop d, const float* power, const double* xi, const double* zeta, int64_t R,
                            const int64_t* idx, float* feat, float* target, float* weight) {
  const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= R) return;
  const int64_t i = idx[r];
  const int64_t NK = (int64_t)d.N * d.K;
  if (i < 0 || i >= (int64_t)d.M * NK) {  // out-of-range index: an all-zero row
    for (int c = 0; c < 4; ++c) feat[r * 4 + c] = 0.0f;
    for (int c = 0; c < 3; ++c) target[r * 3 + c] = weight[r * 3 + c] = 0.0f;
    return;
  }
  const int m = (int)(i / NK), k = (int)(i % d.K);
  float f[4];
  triple_features(d, i, f);
  for (int c = 0; c < 4; ++c) feat[r * 4 + c] = f[c];
  const double pw = power[i];
  target[r * 3] = pw > 0.0 ? (float)fmin(fmax(1.0 + log10(pw / d.pmask[m]) / kDecades, 0.0), 1.0) : 0.0f;
  target[r * 3 + 1] = (float)log1p(xi[m]);
  target[r * 3 + 2] = (float)log1p(zeta[k]);
  weight[r * 3] = 1.0f;
  weight[r * 3 + 1] = 1.0f;
  weight[r * 3 + 2] = f[1];
}

// Initial powers: q = sigmoid(y0); p0 = pmask 10^(6 (q - 1)) where q >= 0.1, else 0.
__global__ void p0_kernel(FeatDrop d, const float* y, double* p0) {
  const int64_t n = (int64_t)d.M * d.N * d.K;
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= n) return;
  const int m = (int)(t / ((int64_t)d.N * d.K));
  const double q = 1.0 / (1.0 + exp(-(double)y[t * 3]));
  p0[t] = q >= kQMin ? d.pmask[m] * exp10(kDecades * (q - 1.0)) : 0.0;
}

// xi0_m = expm1(clip(mean_{n,k} y1, 0, 30)): one workgroup per RRH, fixed order.
__global__ void __launch_bounds__(256) xi_pool_kernel(FeatDrop d, const float* y, double* xi0) {
  __shared__ double red[256];
  const int m = blockIdx.x;
  const int64_t NK = (int64_t)d.N * d.K;
  double s = 0.0;
  for (int64_t i = threadIdx.x; i < NK; i += 256) s += (double)y[((int64_t)m * NK + i) * 3 + 1];
  red[threadIdx.x] = s;
  __syncthreads();
  for (int k = 128; k > 0; k >>= 1) {
    if (threadIdx.x < k) red[threadIdx.x] += red[threadIdx.x + k];
    __syncthreads();
  }
  if (threadIdx.x == 0) xi0[m] = expm1(fmin(fmax(red[0] / (double)NK, 0.0), kLogClip));
}

// zeta0_k = expm1(clip(mean_{m,n} y2, 0, 30)) for streaming users, else 0.
__global__ void __launch_bounds__(256) zeta_pool_kernel(FeatDrop d, const float* y, double* zeta0) {
  __shared__ double red[256];
  const int k = blockIdx.x;
  const int64_t MN = (int64_t)d.M * d.N;
  double s = 0.0;
  for (int64_t i = threadIdx.x; i < MN; i += 256) s += (double)y[(i * d.K + k) * 3 + 2];
  red[threadIdx.x] = s;
  __syncthreads();
  for (int q = 128; q > 0; q >>= 1) {
    if (threadIdx.x < q) red[threadIdx.x] += red[threadIdx.x + q];
    __syncthreads();
  }
  if (threadIdx.x == 0)
    zeta0[k] = d.f1[k] != 0.0f ? expm1(fmin(fmax(red[0] / (double)MN, 0.0), kLogClip)) : 0.0;
}

// One drop of a batched inference: its rows are [row0, row0 + M N K) of the
// batch, its multipliers start at moff (xi) and koff (zeta).
struct BatchFeat {
  int64_t row0, moff, koff;
  FeatDrop fd;
};

// Largest b with tab[b].row0 <= r (tab sorted by row0).
__device__ inline int find_drop(const BatchFeat* tab, int B, int64_t r) {
  int lo = 0, hi = B - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (tab[mid].row0 <= r)
      lo = mid;
    else
      hi = mid - 1;
  }
  return lo;
}

// bf16 features of batch rows [r0, r0 + n).
__global__ void features_batch_kernel(const BatchFeat* tab, int B, int64_t r0, int64_t n, bf16* out) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= n) return;
  const int64_t r = r0 + t;
  const int b = find_drop(tab, B, r);
  float f[4];
  triple_features(tab[b].fd, r - tab[b].row0, f);
  for (int c = 0; c < 4; ++c) out[t * 4 + c] = to_bf16(f[c]);
}

// Initial powers of batch rows [r0, r0 + n); y holds rows from y0.
__global__ void p0_batch_kernel(const BatchFeat* tab, int B, int64_t r0, int64_t n, const float* y, int64_t y0,
                                double* p0) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= n) return;
  const int64_t r = r0 + t;
  const int b = find_drop(tab, B, r);
  const FeatDrop& d = tab[b].fd;
  const int m = (int)((r - tab[b].row0) / ((int64_t)d.N * d.K));
  const double q = 1.0 / (1.0 + exp(-(double)y[(r - y0) * 3]));
  p0[r] = q >= kQMin ? d.pmask[m] * exp10(kDecades * (q - 1.0)) : 0.0;
}

// xi0 of item (drop b, RRH m) per workgroup: mean over (n,k), fixed order.
__global__ void __launch_bounds__(256) xi_pool_batch_kernel(const BatchFeat* tab, const int2* items,
                                                            const float* y, int64_t y0, double* xi0) {
  __shared__ double red[256];
  const int2 it = items[blockIdx.x];
  const BatchFeat& e = tab[it.x];
  const int64_t NK = (int64_t)e.fd.N * e.fd.K;
  const float* yb = y + (e.row0 - y0 + (int64_t)it.y * NK) * 3;
  double s = 0.0;
  for (int64_t i = threadIdx.x; i < NK; i += 256) s += (double)yb[i * 3 + 1];
  red[threadIdx.x] = s;
  __syncthreads();
  for (int k = 128; k > 0; k >>= 1) {
    if (threadIdx.x < k) red[threadIdx.x] += red[threadIdx.x + k];
    __syncthreads();
  }
  if (threadIdx.x == 0) xi0[e.moff + it.y] = expm1(fmin(fmax(red[0] / (double)NK, 0.0), kLogClip));
}

// zeta0 of item (drop b, user k): mean over (m,n), 0 for elastic users.
__global__ void __launch_bounds__(256) zeta_pool_batch_kernel(const BatchFeat* tab, const int2* items,
                                                              const float* y, int64_t y0, double* zeta0) {
  __shared__ double red[256];
  const int2 it = items[blockIdx.x];
  const BatchFeat& e = tab[it.x];
  const int K = e.fd.K;
  const int64_t MN = (int64_t)e.fd.M * e.fd.N;
  const float* yb = y + (e.row0 - y0) * 3;
  double s = 0.0;
  for (int64_t i = threadIdx.x; i < MN; i += 256) s += (double)yb[(i * K + it.y) * 3 + 2];
  red[threadIdx.x] = s;
  __syncthreads();
  for (int q = 128; q > 0; q >>= 1) {
    if (threadIdx.x < q) red[threadIdx.x] += red[threadIdx.x + q];
    __syncthreads();
  }
  if (threadIdx.x == 0)
    zeta0[e.koff + it.y] =
        e.fd.f1[it.y] != 0.0f ? expm1(fmin(fmax(red[0] / (double)MN, 0.0), kLogClip)) : 0.0;
}

double min_rate(double arrival_bps, double delay_s, double packet_bits, double bw_hz) {
  const double lambda = arrival_bps / packet_bits;
  const double x = lambda * delay_s;
  return (arrival_bps / (1.0 - 1.0 / (x + sqrt(1.0 + x * x)))) / bw_hz;
}

int64_t cdiv(int64_t a, int64_t b) { return (a + b - 1) / b; }

}  // namespace

// ==================================================================== host

struct alloc_mlp {
  alloc_ctx* ctx;
  float* master;  // [kNP]
  float* grad;    // [kNP]
  float* m1;      // [kNP] AdamW first moment
  float* m2;      // [kNP] second moment
  bf16* q;        // [kNQ] bf16 weight matrices (training GEMMs)
  bf16x8* frag;   // [2 kFragHid + kFragOut] fused-inference weight fragments
  int64_t step;
  char* ws;       // scratch (rows, activations, partials, warm-start arrays)
  size_t ws_bytes;
  double last_ms;
};

namespace {

struct Scratch {
  size_t total = 0;
  size_t add(size_t bytes) {
    const size_t o = total;
    total += (bytes + 255) & ~size_t(255);
    return o;
  }
};

int ensure_ws(alloc_mlp* net, size_t bytes) {
  if (bytes <= net->ws_bytes) return ALLOC_OK;
  if (net->ws) (void)hipFree(net->ws);
  net->ws = nullptr;
  net->ws_bytes = 0;
  if (hipMalloc((void**)&net->ws, bytes) != hipSuccess) return ALLOC_ENOMEM;
  net->ws_bytes = bytes;
  return ALLOC_OK;
}

// Launches C = X Y with the contraction split into `splits` chunks (partials
// epilogue) or whole; *used receives the number of chunks launched.
int launch_gemm(hipStream_t st, GemmArgs a, int splits, int* used = nullptr) {
  if (a.I <= 0 || a.J <= 0) return ALLOC_OK;
  a.pchunk = cdiv(cdiv(a.P, splits), kKs) * kKs;
  const int64_t gz = std::max<int64_t>(1, cdiv(a.P, a.pchunk));
  if (used) *used = (int)gz;
  hipLaunchKernelGGL(gemm_kernel, dim3((unsigned)cdiv(a.I, kTile), (unsigned)cdiv(a.J, kTile), (unsigned)gz),
                     dim3(256), 0, st, a);
  return hipGetLastError() == hipSuccess ? ALLOC_OK : ALLOC_EDEVICE;
}

// Forward pass of n rows whose bf16 inputs are at x0 [n][4].  Training keeps
// the pre-activations Z1..Z3 [n][256] (fp32) and activations A1..A3 (bf16);
// inference ping-pongs two activation buffers.  y [n][3] fp32.
struct Acts {
  float* Z[4];
  bf16* A[4];
};

int forward_rows(alloc_mlp* net, int64_t n, const bf16* x0, const Acts& s, bool train, float* y) {
  hipStream_t st = net->ctx->stream;
  const bf16* in = x0;
  int64_t in_w = kIn;
  for (int l = 1; l <= 4; ++l) {
    GemmArgs a;
    memset(&a, 0, sizeof a);
    a.X = in;
    a.xs_i = in_w;
    a.xs_p = 1;
    a.Y = net->q + kQW[l];
    a.ys_p = 1;
    a.ys_j = kLayerIn[l];
    a.I = n;
    a.J = kLayerOut[l];
    a.P = kLayerIn[l];
    a.ones_col = -1;
    a.bias = net->master + kOB[l];
    a.ldc = kLayerOut[l];
    if (l < 4) {
      a.epi = train ? kEpiHidTrain : kEpiHidInfer;
      a.Zf = train ? s.Z[l] : nullptr;
      a.Ab = s.A[l];
    } else {
      a.epi = kEpiOut;
      a.Zf = y;
    }
    const int rc = launch_gemm(st, a, 1);
    if (rc) return rc;
    in = s.A[l];
    in_w = kHid;
  }
  return ALLOC_OK;
}

int grad_rows(alloc_mlp* net, int64_t R, const float* feat, const float* target, const float* weight,
              double* loss_host) {
  if (!net || R < 1 || !feat || !target || !weight) return ALLOC_EINVAL;
  hipStream_t st = net->ctx->stream;
  const int S = (int)std::min<int64_t>(64, std::max<int64_t>(1, R / 2048));
  const int64_t nblk = cdiv(R, 256);
  Scratch L;
  const size_t oX0 = L.add(sizeof(bf16) * R * kIn);
  size_t oZ[4], oA[4];
  for (int l = 1; l <= 3; ++l) {
    oZ[l] = L.add(sizeof(float) * R * kHid);
    oA[l] = L.add(sizeof(bf16) * R * kHid);
  }
  const size_t oY = L.add(sizeof(float) * R * kOut);
  const size_t oDy = L.add(sizeof(bf16) * R * kOut);
  const size_t oD0 = L.add(sizeof(bf16) * R * kHid);
  const size_t oD1 = L.add(sizeof(bf16) * R * kHid);
  const size_t oPart = L.add(sizeof(float) * S * kHid * (kHid + 1));
  const size_t oBl = L.add(sizeof(double) * nblk);
  const size_t oLs = L.add(sizeof(double));
  int rc = ensure_ws(net, L.total);
  if (rc) return rc;
  char* w = net->ws;
  bf16* x0 = (bf16*)(w + oX0);
  Acts s;
  s.A[0] = x0;
  s.Z[0] = nullptr;
  for (int l = 1; l <= 3; ++l) {
    s.Z[l] = (float*)(w + oZ[l]);
    s.A[l] = (bf16*)(w + oA[l]);
  }
  float* y = (float*)(w + oY);
  bf16* dy = (bf16*)(w + oDy);
  bf16* dz[2] = {(bf16*)(w + oD0), (bf16*)(w + oD1)};
  float* part = (float*)(w + oPart);
  double* bl = (double*)(w + oBl);
  double* ls = (double*)(w + oLs);

  hipLaunchKernelGGL(cast_rows_kernel, dim3((unsigned)cdiv(R * kIn, 256)), dim3(256), 0, st, feat, x0, R * kIn);
  if ((rc = forward_rows(net, R, x0, s, true, y))) return rc;
  hipLaunchKernelGGL(loss_kernel, dim3((unsigned)nblk), dim3(256), 0, st, y, target, weight, R, dy, bl);
  hipLaunchKernelGGL(sum_kernel, dim3(1), dim3(256), 0, st, bl, nblk, ls);

  // backward: layer l's upstream gradient g (bf16 [R][out_l], row stride out_l)
  const bf16* g = dy;
  for (int l = 4; l >= 1; --l) {
    const int out = kLayerOut[l], in = kLayerIn[l];
    const bf16* act_in = s.A[l - 1];
    // dW_l | db_l = g^T [A_{l-1} | 1]
    GemmArgs a;
    memset(&a, 0, sizeof a);
    a.X = g;
    a.xs_i = 1;
    a.xs_p = out;
    a.Y = act_in;
    a.ys_p = in;
    a.ys_j = 1;
    a.I = out;
    a.J = in + 1;
    a.P = R;
    a.ones_col = in;
    a.epi = kEpiPart;
    a.Zf = part;
    a.ldc = in + 1;
    int S_used = 0;
    if ((rc = launch_gemm(st, a, S, &S_used))) return rc;
    hipLaunchKernelGGL(reduce_split_kernel, dim3((unsigned)cdiv((int64_t)out * (in + 1), 256)), dim3(256), 0,
                       st, (const float*)part, S_used, out, in, net->grad + kOW[l], net->grad + kOB[l]);
    if (l == 1) break;
    // dA_{l-1} = g W_l, then dz_{l-1} = bf16(dA * gelu'(Z_{l-1}))
    bf16* gn = dz[l & 1];
    memset(&a, 0, sizeof a);
    a.X = g;
    a.xs_i = out;
    a.xs_p = 1;
    a.Y = net->q + kQW[l];
    a.ys_p = in;
    a.ys_j = 1;
    a.I = R;
    a.J = in;
    a.P = out;
    a.ones_col = -1;
    a.epi = kEpiBwd;
    a.Ab = gn;
    a.Zprev = s.Z[l - 1];
    a.ldc = in;
    if ((rc = launch_gemm(st, a, 1))) return rc;
    g = gn;
  }
  if (hipGetLastError() != hipSuccess) return ALLOC_EDEVICE;
  double lsum = 0.0;
  if (hipMemcpyAsync(&lsum, ls, sizeof(double), hipMemcpyDeviceToHost, st) != hipSuccess ||
      hipStreamSynchronize(st) != hipSuccess)
    return ALLOC_EDEVICE;
  if (loss_host) *loss_host = lsum / (double)R;
  return ALLOC_OK;
}

// bf16 copies of the weights for the training GEMMs and the fused inference.
void refresh_weights(alloc_mlp* net, hipStream_t st) {
  hipLaunchKernelGGL(cast_weights_kernel, dim3((unsigned)cdiv((int64_t)kHid * kHid, 256)), dim3(256), 0, st,
                     (const float*)net->master, net->q);
  hipLaunchKernelGGL(pack_frags_kernel, dim3((unsigned)cdiv(2 * kFragHid + kFragOut, 256)), dim3(256), 0, st,
                     (const float*)net->master, net->frag);
}

// Inference of n rows (bf16 inputs x0 [n][4]) into y [n][3] by the fused kernel.
int infer_rows(alloc_mlp* net, int64_t n, const bf16* x0, float* y) {
  if (n <= 0) return ALLOC_OK;
  // persistent grid of 8 workgroups per compute unit, more than are resident
  // at once (three at 168 VGPRs): sized to the resident count it ran 6%
  // slower (11.37 against 10.70 ms for 16.8 M rows)
  const int64_t grid = std::min<int64_t>(cdiv(n, 4 * 16 * kFusedR), (int64_t)net->ctx->cus * 8);
  hipLaunchKernelGGL(mlp_fused_kernel, dim3((unsigned)grid), dim3(256), 0, net->ctx->stream, x0, n,
                     (const float*)net->master, (const bf16x8*)net->frag, y);
  return hipGetLastError() == hipSuccess ? ALLOC_OK : ALLOC_EDEVICE;
}

int adamw(alloc_mlp* net, const float* g, const alloc_mlp_opt* o) {
  if (!net || !g || !o) return ALLOC_EINVAL;
  hipStream_t st = net->ctx->stream;
  net->step += 1;
  const double bc1 = 1.0 - pow((double)o->beta1, (double)net->step);
  const double bc2 = 1.0 - pow((double)o->beta2, (double)net->step);
  hipLaunchKernelGGL(adamw_kernel, dim3((unsigned)cdiv(kNP, 256)), dim3(256), 0, st, net->master, net->m1,
                     net->m2, g, o->lr, o->beta1, o->beta2, o->eps, o->weight_decay, (float)bc1, (float)bc2);
  refresh_weights(net, st);
  return hipGetLastError() == hipSuccess ? ALLOC_OK : ALLOC_EDEVICE;
}

// Per-drop feature constants (host side), uploaded into the scratch at off.
struct FeatHost {
  std::vector<double> snr_scale, pmask;
  std::vector<float> f1, f2, f3;
};

int feat_drop(alloc_mlp* net, const alloc_problem* pb, uint32_t flags, size_t off, FeatDrop* d,
              const float** gain_dev_out, size_t gain_off) {
  const int M = pb->M, N = pb->N, K = pb->K;
  if (M < 1 || N < 1 || K < 1 || !pb->gain || !pb->user_type || !pb->pmax_w) return ALLOC_EINVAL;
  if (!(pb->noise_w > 0) || !(pb->bw_hz > 0) || !(pb->packet_bits > 0)) return ALLOC_EINVAL;
  std::vector<char> img(sizeof(double) * 2 * M + sizeof(float) * (M + 2 * K) + 64, 0);
  double* sc = (double*)img.data();
  double* pm = sc + M;
  float* f3 = (float*)(pm + M);
  float* f1 = f3 + M;
  float* f2 = f1 + K;
  for (int m = 0; m < M; ++m) {
    if (!(pb->pmax_w[m] > 0)) return ALLOC_EINVAL;
    pm[m] = pb->pmask_w ? pb->pmask_w[m] : pb->pmax_w[m] / N;
    sc[m] = pm[m] / pb->noise_w;
    f3[m] = (float)((10.0 * log10(1000.0 * pb->pmax_w[m]) - 40.0) / 10.0);
  }
  for (int k = 0; k < K; ++k) {
    const bool s = pb->user_type[k] == 1;
    if (s && (!pb->arrival_bps || !pb->delay_s || !(pb->arrival_bps[k] > 0) || !(pb->delay_s[k] > 0)))
      return ALLOC_EINVAL;
    f1[k] = s ? 1.0f : 0.0f;
    f2[k] = s ? (float)min_rate(pb->arrival_bps[k], pb->delay_s[k], pb->packet_bits, pb->bw_hz) : 0.0f;
  }
  hipStream_t st = net->ctx->stream;
  char* base = net->ws + off;
  if (hipMemcpyAsync(base, img.data(), img.size(), hipMemcpyHostToDevice, st) != hipSuccess)
    return ALLOC_EDEVICE;
  d->M = M;
  d->N = N;
  d->K = K;
  d->snr_scale = (const double*)base;
  d->pmask = (const double*)base + M;
  d->f3 = (const float*)((const double*)base + 2 * M);
  d->f1 = d->f3 + M;
  d->f2 = d->f1 + K;
  if (flags & ALLOC_GAIN_ON_DEVICE) {
    d->G = pb->gain;
  } else {
    const size_t n3 = (size_t)M * N * K;
    if (hipMemcpyAsync(net->ws + gain_off, pb->gain, sizeof(float) * n3, hipMemcpyHostToDevice, st) !=
        hipSuccess)
      return ALLOC_EDEVICE;
    d->G = (const float*)(net->ws + gain_off);
  }
  if (gain_dev_out) *gain_dev_out = d->G;
  return ALLOC_OK;
}

size_t feat_bytes(int M, int K) { return sizeof(double) * 2 * M + sizeof(float) * (M + 2 * K) + 64; }

// Host image of one drop's feature constants (layout of feat_bytes):
// snr_scale [M], pmask [M] (double), f3 [M], f1 [K], f2 [K] (float).
int feat_image(const alloc_problem* pb, char* img) {
  const int M = pb->M, N = pb->N, K = pb->K;
  if (M < 1 || N < 1 || K < 1 || !pb->gain || !pb->user_type || !pb->pmax_w) return ALLOC_EINVAL;
  if (!(pb->noise_w > 0) || !(pb->bw_hz > 0) || !(pb->packet_bits > 0)) return ALLOC_EINVAL;
  double* sc = (double*)img;
  double* pm = sc + M;
  float* f3 = (float*)(pm + M);
  float* f1 = f3 + M;
  float* f2 = f1 + K;
  for (int m = 0; m < M; ++m) {
    if (!(pb->pmax_w[m] > 0)) return ALLOC_EINVAL;
    pm[m] = pb->pmask_w ? pb->pmask_w[m] : pb->pmax_w[m] / N;
    sc[m] = pm[m] / pb->noise_w;
    f3[m] = (float)((10.0 * log10(1000.0 * pb->pmax_w[m]) - 40.0) / 10.0);
  }
  for (int k = 0; k < K; ++k) {
    const bool st = pb->user_type[k] == 1;
    if (st && (!pb->arrival_bps || !pb->delay_s || !(pb->arrival_bps[k] > 0) || !(pb->delay_s[k] > 0)))
      return ALLOC_EINVAL;
    f1[k] = st ? 1.0f : 0.0f;
    f2[k] = st ? (float)min_rate(pb->arrival_bps[k], pb->delay_s[k], pb->packet_bits, pb->bw_hz) : 0.0f;
  }
  return ALLOC_OK;
}

void feat_ptrs(const alloc_problem* pb, const char* base, const float* gain, FeatDrop* d) {
  d->M = pb->M;
  d->N = pb->N;
  d->K = pb->K;
  d->G = gain;
  d->snr_scale = (const double*)base;
  d->pmask = (const double*)base + pb->M;
  d->f3 = (const float*)((const double*)base + 2 * pb->M);
  d->f1 = d->f3 + pb->M;
  d->f2 = d->f1 + pb->K;
}

// Warm-start arrays of a whole batch, from one inference pass over every
// drop's rows (drops in groups of at most kGroupRows rows share the output
// buffer).  Offsets into the network's scratch; per drop its first row and
// multiplier offsets.
constexpr int64_t kGroupRows = int64_t(1) << 26;

struct WarmBatch {
  size_t p0 = 0, xi = 0, zeta = 0;
  std::vector<int64_t> row0, moff, koff;
};

int warm_batch(alloc_mlp* net, int B, const alloc_problem* probs, uint32_t gflag, WarmBatch* wb) {
  std::vector<int64_t>& row0 = wb->row0;
  std::vector<int64_t>& moff = wb->moff;
  std::vector<int64_t>& koff = wb->koff;
  row0.assign(B + 1, 0);
  moff.assign(B + 1, 0);
  koff.assign(B + 1, 0);
  std::vector<size_t> cimg(B + 1, 0);
  for (int b = 0; b < B; ++b) {
    const alloc_problem& pb = probs[b];
    if (pb.M < 1 || pb.N < 1 || pb.K < 1) return ALLOC_EINVAL;
    row0[b + 1] = row0[b] + (int64_t)pb.M * pb.N * pb.K;
    moff[b + 1] = moff[b] + pb.M;
    koff[b + 1] = koff[b] + pb.K;
    cimg[b + 1] = cimg[b] + ((feat_bytes(pb.M, pb.K) + 255) & ~size_t(255));
  }
  const int64_t R = row0[B];
  // groups of consecutive drops
  std::vector<int> gstart{0};
  int64_t ymax = 0;
  for (int b = 0; b < B; ++b) {
    const int g0 = gstart.back();
    if (b > g0 && row0[b + 1] - row0[g0] > kGroupRows) gstart.push_back(b);
  }
  gstart.push_back(B);
  for (size_t g = 0; g + 1 < gstart.size(); ++g) ymax = std::max(ymax, row0[gstart[g + 1]] - row0[gstart[g]]);
  const int64_t chunk = std::min<int64_t>(ymax, kChunk);

  Scratch L;
  const size_t oC = L.add(cimg[B]);
  const size_t oTab = L.add(sizeof(BatchFeat) * B);
  const size_t oMi = L.add(sizeof(int2) * moff[B]);
  const size_t oKi = L.add(sizeof(int2) * koff[B]);
  const size_t oG = L.add(gflag ? 0 : sizeof(float) * R);
  const size_t oX0 = L.add(sizeof(bf16) * chunk * kIn);
  const size_t oA1 = L.add(sizeof(bf16) * chunk * kHid);
  const size_t oA2 = L.add(sizeof(bf16) * chunk * kHid);
  const size_t oY = L.add(sizeof(float) * ymax * kOut);
  wb->p0 = L.add(sizeof(double) * R);
  wb->xi = L.add(sizeof(double) * moff[B]);
  wb->zeta = L.add(sizeof(double) * koff[B]);
  int rc = ensure_ws(net, L.total);
  if (rc) return rc;
  char* w = net->ws;
  hipStream_t st = net->ctx->stream;

  std::vector<char> img(cimg[B], 0);
  std::vector<BatchFeat> tab(B);
  std::vector<int2> mi(moff[B]), ki(koff[B]);
  for (int b = 0; b < B; ++b) {
    const alloc_problem& pb = probs[b];
    if ((rc = feat_image(&pb, img.data() + cimg[b]))) return rc;
    const float* g = gflag ? pb.gain : (const float*)(w + oG) + row0[b];
    tab[b].row0 = row0[b];
    tab[b].moff = moff[b];
    tab[b].koff = koff[b];
    feat_ptrs(&pb, w + oC + cimg[b], g, &tab[b].fd);
    for (int m = 0; m < pb.M; ++m) mi[moff[b] + m] = make_int2(b, m);
    for (int k = 0; k < pb.K; ++k) ki[koff[b] + k] = make_int2(b, k);
    if (!gflag && hipMemcpyAsync((float*)(w + oG) + row0[b], pb.gain, sizeof(float) * (row0[b + 1] - row0[b]),
                                 hipMemcpyHostToDevice, st) != hipSuccess)
      return ALLOC_EDEVICE;
  }
  if (hipMemcpyAsync(w + oC, img.data(), img.size(), hipMemcpyHostToDevice, st) != hipSuccess ||
      hipMemcpyAsync(w + oTab, tab.data(), sizeof(BatchFeat) * B, hipMemcpyHostToDevice, st) != hipSuccess ||
      hipMemcpyAsync(w + oMi, mi.data(), sizeof(int2) * mi.size(), hipMemcpyHostToDevice, st) != hipSuccess ||
      hipMemcpyAsync(w + oKi, ki.data(), sizeof(int2) * ki.size(), hipMemcpyHostToDevice, st) != hipSuccess)
    return ALLOC_EDEVICE;
  const BatchFeat* dtab = (const BatchFeat*)(w + oTab);
  Acts s;
  s.A[0] = (bf16*)(w + oX0);
  s.A[1] = (bf16*)(w + oA1);
  s.A[2] = (bf16*)(w + oA2);
  s.A[3] = s.A[1];
  for (int l = 0; l < 4; ++l) s.Z[l] = nullptr;
  float* y = (float*)(w + oY);
  for (size_t g = 0; g + 1 < gstart.size(); ++g) {
    const int ga = gstart[g], gb = gstart[g + 1];
    const int64_t R0 = row0[ga], R1 = row0[gb];
    for (int64_t r0 = R0; r0 < R1; r0 += chunk) {
      const int64_t n = std::min(chunk, R1 - r0);
      hipLaunchKernelGGL(features_batch_kernel, dim3((unsigned)cdiv(n, 256)), dim3(256), 0, st, dtab, B, r0, n,
                         s.A[0]);
      if ((rc = infer_rows(net, n, s.A[0], y + (r0 - R0) * kOut))) return rc;
    }
    hipLaunchKernelGGL(p0_batch_kernel, dim3((unsigned)cdiv(R1 - R0, 256)), dim3(256), 0, st, dtab, B, R0, R1 - R0,
                       (const float*)y, R0, (double*)(w + wb->p0));
    const int64_t nm = moff[gb] - moff[ga], nk = koff[gb] - koff[ga];
    hipLaunchKernelGGL(xi_pool_batch_kernel, dim3((unsigned)nm), dim3(256), 0, st, dtab,
                       (const int2*)(w + oMi) + moff[ga], (const float*)y, R0, (double*)(w + wb->xi));
    hipLaunchKernelGGL(zeta_pool_batch_kernel, dim3((unsigned)nk), dim3(256), 0, st, dtab,
                       (const int2*)(w + oKi) + koff[ga], (const float*)y, R0, (double*)(w + wb->zeta));
  }
  return hipGetLastError() == hipSuccess ? ALLOC_OK : ALLOC_EDEVICE;
}

// Scratch of warm_drop from offset base: feature constants, optional host
// gain staging, chunk activations, y [n3][3].
struct WarmScratch {
  size_t F, G, X0, A1, A2, Y, end;
};

WarmScratch warm_scratch(const alloc_problem* pb, uint32_t flags, size_t base) {
  const int64_t n3 = (int64_t)pb->M * pb->N * pb->K;
  const int64_t chunk = std::min(n3, kChunk);
  Scratch L;
  L.total = base;
  WarmScratch w;
  w.F = L.add(feat_bytes(pb->M, pb->K));
  w.G = L.add((flags & ALLOC_GAIN_ON_DEVICE) ? 0 : sizeof(float) * n3);
  w.X0 = L.add(sizeof(bf16) * chunk * kIn);
  w.A1 = L.add(sizeof(bf16) * chunk * kHid);
  w.A2 = L.add(sizeof(bf16) * chunk * kHid);
  w.Y = L.add(sizeof(float) * n3 * kOut);
  w.end = L.total;
  return w;
}

// Inference of one drop into p0/xi0/zeta0 (device).  The caller has sized
// the scratch to warm_scratch(...).end, so it is not reallocated here.
int warm_drop(alloc_mlp* net, const alloc_problem* pb, uint32_t flags, double* p0, double* xi0,
              double* zeta0, size_t base) {
  const int64_t n3 = (int64_t)pb->M * pb->N * pb->K;
  const int64_t chunk = std::min(n3, kChunk);
  const WarmScratch ws = warm_scratch(pb, flags, base);
  if (ws.end > net->ws_bytes) return ALLOC_EINVAL;
  const size_t oF = ws.F, oG = ws.G, oX0 = ws.X0, oA1 = ws.A1, oA2 = ws.A2, oY = ws.Y;
  int rc;
  FeatDrop d;
  if ((rc = feat_drop(net, pb, flags, oF, &d, nullptr, oG))) return rc;
  hipStream_t st = net->ctx->stream;
  char* w = net->ws;
  Acts s;
  s.A[0] = (bf16*)(w + oX0);
  s.A[1] = (bf16*)(w + oA1);
  s.A[2] = (bf16*)(w + oA2);
  s.A[3] = (bf16*)(w + oA1);
  for (int l = 0; l < 4; ++l) s.Z[l] = nullptr;
  float* y = (float*)(w + oY);
  for (int64_t r0 = 0; r0 < n3; r0 += chunk) {
    const int64_t n = std::min(chunk, n3 - r0);
    hipLaunchKernelGGL(features_kernel, dim3((unsigned)cdiv(n, 256)), dim3(256), 0, st, d, r0, n,
                       (float*)nullptr, s.A[0]);
    if ((rc = infer_rows(net, n, s.A[0], y + r0 * kOut))) return rc;
  }
  hipLaunchKernelGGL(p0_kernel, dim3((unsigned)cdiv(n3, 256)), dim3(256), 0, st, d, (const float*)y, p0);
  hipLaunchKernelGGL(xi_pool_kernel, dim3(pb->M), dim3(256), 0, st, d, (const float*)y, xi0);
  hipLaunchKernelGGL(zeta_pool_kernel, dim3(pb->K), dim3(256), 0, st, d, (const float*)y, zeta0);
  return hipGetLastError() == hipSuccess ? ALLOC_OK : ALLOC_EDEVICE;
}

// Scratch offset where warm_drop's own area starts, after the warm-start
// arrays of one drop (p0 [n3], xi0 [M], zeta0 [K]).
struct WarmArrays {
  size_t p0, xi0, zeta0, end;
};

WarmArrays warm_arrays(int64_t n3, int M, int K) {
  Scratch L;
  WarmArrays w;
  w.p0 = L.add(sizeof(double) * n3);
  w.xi0 = L.add(sizeof(double) * M);
  w.zeta0 = L.add(sizeof(double) * K);
  w.end = L.total;
  return w;
}

// The warm-started solve is replaced by the cold one when it ended
// non-finite, with no allocation at all (EE not positive), or infeasible for
// the constraints the method meets when it converges: a streaming user below
// its minimum rate (C13) or an RRH over its budget (C12).  C14 is enforced
// through its multiplier and reported, as on the cold path.
bool needs_fallback(const alloc_result& r, bool capped) {
  const uint32_t bad = ALLOC_NONFINITE | ALLOC_QOS_INFEASIBLE | ALLOC_BUDGET_INFEASIBLE |
                       (capped ? ALLOC_NOT_CONVERGED : 0u);
  return (r.status_flags & bad) || !(r.ee > 0.0);
}

// The warm attempt's schedule: max_dinkelbach cut to warm_max_dinkelbach
// when that is set and smaller (then *capped).
alloc_params warm_params(const alloc_params& p, bool* capped) {
  alloc_params w = p;
  *capped = p.warm_max_dinkelbach > 0 && p.warm_max_dinkelbach < p.max_dinkelbach;
  if (*capped) w.max_dinkelbach = p.warm_max_dinkelbach;
  return w;
}

}  // namespace

namespace {

// Finds `"key"` at object depth 1 of the header and returns the position after
// its colon, or npos.
size_t json_key(const std::string& h, const char* key) {
  const std::string k = std::string("\"") + key + "\"";
  int depth = 0;
  bool str = false;
  for (size_t i = 0; i < h.size(); ++i) {
    const char c = h[i];
    if (str) {
      if (c == '\\') ++i;
      else if (c == '"') str = false;
      continue;
    }
    if (c == '{' || c == '[') ++depth;
    else if (c == '}' || c == ']') --depth;
    else if (c == '"') {
      if (depth == 1 && h.compare(i, k.size(), k) == 0) {
        size_t j = i + k.size();
        while (j < h.size() && (h[j] == ' ' || h[j] == ':')) ++j;
        return j;
      }
      str = true;
    }
  }
  return std::string::npos;
}

// The integers of a JSON array starting at h[pos] == '['.
bool json_ints(const std::string& h, size_t pos, std::vector<long long>* out) {
  if (pos >= h.size() || h[pos] != '[') return false;
  size_t i = pos + 1;
  while (i < h.size()) {
    while (i < h.size() && (h[i] == ' ' || h[i] == ',')) ++i;
    if (i < h.size() && h[i] == ']') return true;
    char* end = nullptr;
    const long long v = strtoll(h.c_str() + i, &end, 10);
    if (end == h.c_str() + i) return false;
    out->push_back(v);
    i = (size_t)(end - h.c_str());
  }
  return false;
}

}  // namespace

extern "C" {

int alloc_mlp_create(alloc_ctx* ctx, alloc_mlp** out) {
  if (!ctx || !out || ctx->closed) return ALLOC_EINVAL;
  if (hipSetDevice(ctx->device) != hipSuccess) return ALLOC_EDEVICE;
  alloc_mlp* n = new alloc_mlp;
  memset(n, 0, sizeof *n);
  n->ctx = ctx;
  n->last_ms = -1.0;
  const size_t fbytes = sizeof(bf16x8) * (2 * kFragHid + kFragOut);
  const size_t bytes = sizeof(float) * kNP * 4 + sizeof(bf16) * kNQ + 256 + fbytes;
  char* p = nullptr;
  if (hipMalloc((void**)&p, bytes) != hipSuccess) {
    delete n;
    return ALLOC_ENOMEM;
  }
  n->master = (float*)p;
  n->grad = n->master + kNP;
  n->m1 = n->grad + kNP;
  n->m2 = n->m1 + kNP;
  n->q = (bf16*)(n->m2 + kNP);
  n->frag = (bf16x8*)(((uintptr_t)(n->q + kNQ) + 255) & ~(uintptr_t)255);
  if (hipMemsetAsync(p, 0, bytes, ctx->stream) != hipSuccess || hipStreamSynchronize(ctx->stream) != hipSuccess) {
    (void)hipFree(p);
    delete n;
    return ALLOC_EDEVICE;
  }
  alloc_internal::ctx_retain(ctx);
  *out = n;
  return ALLOC_OK;
}

void alloc_mlp_destroy(alloc_mlp* net) {
  if (!net) return;
  (void)hipSetDevice(net->ctx->device);
  (void)hipFree(net->master);
  if (net->ws) (void)hipFree(net->ws);
  alloc_internal::ctx_release(net->ctx);
  delete net;
}

int alloc_mlp_set_params(alloc_mlp* net, const float* host, int64_t n) {
  if (!net || !host || n != kNP) return ALLOC_EINVAL;
  for (int64_t i = 0; i < n; ++i)
    if (!std::isfinite(host[i])) return ALLOC_EINVAL;
  hipStream_t st = net->ctx->stream;
  if (hipMemcpyAsync(net->master, host, sizeof(float) * kNP, hipMemcpyHostToDevice, st) != hipSuccess ||
      hipMemsetAsync(net->m1, 0, sizeof(float) * kNP * 2, st) != hipSuccess)
    return ALLOC_EDEVICE;
  net->step = 0;
  refresh_weights(net, st);
  if (hipGetLastError() != hipSuccess || hipStreamSynchronize(st) != hipSuccess) return ALLOC_EDEVICE;
  return ALLOC_OK;
}

int alloc_mlp_get_params(alloc_mlp* net, float* host, int64_t n) {
  if (!net || !host || n != kNP) return ALLOC_EINVAL;
  hipStream_t st = net->ctx->stream;
  if (hipMemcpyAsync(host, net->master, sizeof(float) * kNP, hipMemcpyDeviceToHost, st) != hipSuccess ||
      hipStreamSynchronize(st) != hipSuccess)
    return ALLOC_EDEVICE;
  return ALLOC_OK;
}

// The safetensors layout of a saved network: little-endian uint64 header
// length, a JSON header (space-padded to a multiple of 8 bytes), the data.
int alloc_mlp_save(alloc_mlp* net, const char* path) {
  if (!net || !path) return ALLOC_EINVAL;
  std::vector<float> w(kNP);
  int rc = alloc_mlp_get_params(net, w.data(), kNP);
  if (rc) return rc;
  char buf[256];
  snprintf(buf, sizeof buf,
           "{\"__metadata__\":{\"n_params\":\"%lld\",\"layers\":\"4-256-256-256-3\"},"
           "\"params\":{\"dtype\":\"F32\",\"shape\":[%lld],\"data_offsets\":[0,%lld]}}",
           (long long)kNP, (long long)kNP, (long long)(kNP * sizeof(float)));
  std::string hdr(buf);
  while (hdr.size() % 8) hdr += ' ';
  unsigned char len[8];
  for (int i = 0; i < 8; ++i) len[i] = (unsigned char)(((uint64_t)hdr.size() >> (8 * i)) & 0xff);
  FILE* f = fopen(path, "wb");
  if (!f) return ALLOC_EFILE;
  bool ok = fwrite(len, 1, 8, f) == 8 && fwrite(hdr.data(), 1, hdr.size(), f) == hdr.size() &&
            fwrite(w.data(), sizeof(float), kNP, f) == (size_t)kNP;
  // the data are written as the host holds them: little-endian IEEE floats
  ok = (fclose(f) == 0) && ok;
  return ok ? ALLOC_OK : ALLOC_EFILE;
}

int alloc_mlp_load(alloc_mlp* net, const char* path) {
  if (!net || !path) return ALLOC_EINVAL;
  FILE* f = fopen(path, "rb");
  if (!f) return ALLOC_EFILE;
  unsigned char len[8];
  uint64_t n = 0;
  std::string hdr;
  std::vector<float> w;
  bool ok = fread(len, 1, 8, f) == 8;
  if (ok) {
    for (int i = 0; i < 8; ++i) n |= (uint64_t)len[i] << (8 * i);
    ok = n > 0 && n < (1u << 20);
  }
  if (ok) {
    hdr.resize(n);
    ok = fread(&hdr[0], 1, n, f) == n;
  }
  // the one tensor "params": F32 of shape [kNP] at the start of the data
  size_t at = ok ? json_key(hdr, "params") : std::string::npos;
  if (at == std::string::npos || hdr[at] != '{') ok = false;
  std::vector<long long> shape, offs;
  if (ok) {
    const std::string t = hdr.substr(at, hdr.find('}', at) - at + 1);
    const size_t dt = json_key(t, "dtype"), sh = json_key(t, "shape"), of = json_key(t, "data_offsets");
    ok = dt != std::string::npos && t.compare(dt, 5, "\"F32\"") == 0 && sh != std::string::npos &&
         of != std::string::npos && json_ints(t, sh, &shape) && json_ints(t, of, &offs) && shape.size() == 1 &&
         shape[0] == kNP && offs.size() == 2 && offs[1] - offs[0] == (long long)(kNP * sizeof(float)) &&
         offs[0] >= 0;
  }
  if (ok) ok = fseek(f, (long)(8 + n + offs[0]), SEEK_SET) == 0;
  if (ok) {
    w.resize(kNP);
    ok = fread(w.data(), sizeof(float), kNP, f) == (size_t)kNP;
  }
  fclose(f);
  if (!ok) return ALLOC_EFILE;
  return alloc_mlp_set_params(net, w.data(), kNP);
}

int alloc_mlp_features(alloc_mlp* net, const alloc_problem* pb, uint32_t flags, float* feat) {
  if (!net || !pb || !feat) return ALLOC_EINVAL;
  const int64_t n3 = (int64_t)pb->M * pb->N * pb->K;
  Scratch L;
  const size_t oF = L.add(feat_bytes(pb->M, pb->K));
  const size_t oG = L.add((flags & ALLOC_GAIN_ON_DEVICE) ? 0 : sizeof(float) * n3);
  int rc = ensure_ws(net, L.total);
  if (rc) return rc;
  FeatDrop d;
  if ((rc = feat_drop(net, pb, flags, oF, &d, nullptr, oG))) return rc;
  hipStream_t st = net->ctx->stream;
  hipLaunchKernelGGL(features_kernel, dim3((unsigned)cdiv(n3, 256)), dim3(256), 0, st, d, (int64_t)0, n3, feat,
                     (bf16*)nullptr);
  if (hipGetLastError() != hipSuccess || hipStreamSynchronize(st) != hipSuccess) return ALLOC_EDEVICE;
  return ALLOC_OK;
}

int alloc_mlp_forward(alloc_mlp* net, int64_t R, const float* feat, float* y) {
  if (!net || R < 1 || !feat || !y) return ALLOC_EINVAL;
  const int64_t chunk = std::min(R, kChunk);
  Scratch L;
  const size_t oX0 = L.add(sizeof(bf16) * chunk * kIn);
  const size_t oA1 = L.add(sizeof(bf16) * chunk * kHid);
  const size_t oA2 = L.add(sizeof(bf16) * chunk * kHid);
  int rc = ensure_ws(net, L.total);
  if (rc) return rc;
  hipStream_t st = net->ctx->stream;
  Acts s;
  s.A[0] = (bf16*)(net->ws + oX0);
  s.A[1] = (bf16*)(net->ws + oA1);
  s.A[2] = (bf16*)(net->ws + oA2);
  s.A[3] = s.A[1];
  for (int l = 0; l < 4; ++l) s.Z[l] = nullptr;
  alloc_ctx* c = net->ctx;
  if (c->timing && hipEventRecord(c->ev0, st) != hipSuccess) return ALLOC_EDEVICE;
  for (int64_t r0 = 0; r0 < R; r0 += chunk) {
    const int64_t n = std::min(chunk, R - r0);
    hipLaunchKernelGGL(cast_rows_kernel, dim3((unsigned)cdiv(n * kIn, 256)), dim3(256), 0, st, feat + r0 * kIn,
                       s.A[0], n * kIn);
    if ((rc = infer_rows(net, n, s.A[0], y + r0 * kOut))) return rc;
  }
  if (c->timing && hipEventRecord(c->ev1, st) != hipSuccess) return ALLOC_EDEVICE;
  if (hipStreamSynchronize(st) != hipSuccess) return ALLOC_EDEVICE;
  net->last_ms = -1.0;
  if (c->timing) {
    float ms = 0.0f;
    if (hipEventElapsedTime(&ms, c->ev0, c->ev1) != hipSuccess) return ALLOC_EDEVICE;
    net->last_ms = ms;
  }
  return ALLOC_OK;
}

int alloc_mlp_grad(alloc_mlp* net, int64_t R, const float* feat, const float* target, const float* weight,
                   float* grad, double* loss) {
  const int rc = grad_rows(net, R, feat, target, weight, loss);
  if (rc) return rc;
  if (grad) {
    hipStream_t st = net->ctx->stream;
    if (hipMemcpyAsync(grad, net->grad, sizeof(float) * kNP, hipMemcpyDeviceToDevice, st) != hipSuccess ||
        hipStreamSynchronize(st) != hipSuccess)
      return ALLOC_EDEVICE;
  }
  return ALLOC_OK;
}

int alloc_mlp_train_step(alloc_mlp* net, int64_t R, const float* feat, const float* target, const float* weight,
                         const alloc_mlp_opt* opt, double* loss) {
  if (!opt) return ALLOC_EINVAL;
  int rc = grad_rows(net, R, feat, target, weight, loss);
  if (rc) return rc;
  if ((rc = adamw(net, net->grad, opt))) return rc;
  return hipStreamSynchronize(net->ctx->stream) == hipSuccess ? ALLOC_OK : ALLOC_EDEVICE;
}

int alloc_mlp_adamw(alloc_mlp* net, const float* grad, const alloc_mlp_opt* opt) {
  const int rc = adamw(net, grad, opt);
  if (rc) return rc;
  return hipStreamSynchronize(net->ctx->stream) == hipSuccess ? ALLOC_OK : ALLOC_EDEVICE;
}

int alloc_mlp_rows(alloc_mlp* net, const alloc_problem* pb, uint32_t flags, const float* power, const double* xi,
                   const double* zeta, int64_t R, const int64_t* idx, float* feat, float* target, float* weight) {
  if (!net || !pb || !power || !xi || !zeta || R < 1 || !idx || !feat || !target || !weight) return ALLOC_EINVAL;
  const int64_t n3 = (int64_t)pb->M * pb->N * pb->K;
  Scratch L;
  const size_t oF = L.add(feat_bytes(pb->M, pb->K));
  const size_t oG = L.add((flags & ALLOC_GAIN_ON_DEVICE) ? 0 : sizeof(float) * n3);
  int rc = ensure_ws(net, L.total);
  if (rc) return rc;
  FeatDrop d;
  if ((rc = feat_drop(net, pb, flags, oF, &d, nullptr, oG))) return rc;
  hipStream_t st = net->ctx->stream;
  hipLaunchKernelGGL(rows_kernel, dim3((unsigned)cdiv(R, 256)), dim3(256), 0, st, d, power, xi, zeta, R, idx, feat,
                     target, weight);
  if (hipGetLastError() != hipSuccess || hipStreamSynchronize(st) != hipSuccess) return ALLOC_EDEVICE;
  return ALLOC_OK;
}

int alloc_mlp_warm(alloc_mlp* net, const alloc_problem* pb, uint32_t flags, double* p0, double* xi0,
                   double* zeta0) {
  if (!net || !pb || !p0 || !xi0 || !zeta0) return ALLOC_EINVAL;
  if (pb->M < 1 || pb->N < 1 || pb->K < 1) return ALLOC_EINVAL;
  int rc = ensure_ws(net, warm_scratch(pb, flags, 0).end);
  if (rc) return rc;
  rc = warm_drop(net, pb, flags, p0, xi0, zeta0, 0);
  if (rc) return rc;
  return hipStreamSynchronize(net->ctx->stream) == hipSuccess ? ALLOC_OK : ALLOC_EDEVICE;
}

int alloc_solve_mlp(alloc_mlp* net, const alloc_problem* pb, const alloc_params* prm, alloc_result* res) {
  if (!net || !pb || !prm || !res) return ALLOC_EINVAL;
  const int64_t n3 = (int64_t)pb->M * pb->N * pb->K;
  if (pb->M < 1 || pb->N < 1 || pb->K < 1) return ALLOC_EINVAL;
  const WarmArrays wa = warm_arrays(n3, pb->M, pb->K);
  alloc_ctx* c = net->ctx;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  if (c->timing && (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess)) return ALLOC_EDEVICE;
  if (e0 && hipEventRecord(e0, c->stream) != hipSuccess) return ALLOC_EDEVICE;
  const uint32_t gflag = prm->flags & ALLOC_GAIN_ON_DEVICE;
  int rc = ensure_ws(net, warm_scratch(pb, gflag, wa.end).end);
  if (rc == ALLOC_OK)
    rc = warm_drop(net, pb, gflag, (double*)(net->ws + wa.p0), (double*)(net->ws + wa.xi0),
                   (double*)(net->ws + wa.zeta0), wa.end);
  if (rc == ALLOC_OK && e1 && hipEventRecord(e1, c->stream) != hipSuccess) rc = ALLOC_EDEVICE;
  double mlp_ms = -1.0;
  if (rc == ALLOC_OK && e1) {
    float ms = 0.0f;
    if (hipEventSynchronize(e1) != hipSuccess || hipEventElapsedTime(&ms, e0, e1) != hipSuccess) rc = ALLOC_EDEVICE;
    mlp_ms = ms;
  }
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  if (rc) return rc;
  net->last_ms = mlp_ms;
  const alloc_internal::DevWarm dw{(const double*)(net->ws + wa.p0), (const double*)(net->ws + wa.xi0),
                                   (const double*)(net->ws + wa.zeta0)};
  bool capped;
  const alloc_params wp = warm_params(*prm, &capped);
  rc = alloc_internal::solve_one(c, pb, &wp, nullptr, &dw, res);
  if (rc) return rc;
  if (needs_fallback(*res, capped)) {
    rc = alloc_internal::solve_one(c, pb, prm, nullptr, nullptr, res);
    if (rc) return rc;
    res->status_flags |= ALLOC_WARM_FALLBACK;
  }
  return ALLOC_OK;
}

int alloc_solve_batch_mlp(alloc_mlp* net, int32_t B, const alloc_problem* probs, const alloc_params* prm,
                          alloc_result* results) {
  if (!net || B < 1 || !probs || !prm || !results) return ALLOC_EINVAL;
  alloc_ctx* c = net->ctx;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  if (c->timing && (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess)) return ALLOC_EDEVICE;
  if (e0 && hipEventRecord(e0, c->stream) != hipSuccess) return ALLOC_EDEVICE;
  WarmBatch wb;
  int rc = warm_batch(net, B, probs, prm->flags & ALLOC_GAIN_ON_DEVICE, &wb);
  double mlp_ms = -1.0;
  if (rc == ALLOC_OK && e1) {
    float ms = 0.0f;
    if (hipEventRecord(e1, c->stream) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
        hipEventElapsedTime(&ms, e0, e1) != hipSuccess)
      rc = ALLOC_EDEVICE;
    mlp_ms = ms;
  }
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  if (rc) return rc;
  net->last_ms = mlp_ms;
  const char* w = net->ws;
  const alloc_internal::WarmFn fn = [&](int b, alloc_internal::DevWarm* dw) {
    dw->p0 = (const double*)(w + wb.p0) + wb.row0[b];
    dw->xi0 = (const double*)(w + wb.xi) + wb.moff[b];
    dw->zeta0 = (const double*)(w + wb.zeta) + wb.koff[b];
    return ALLOC_OK;
  };
  bool capped;
  const alloc_params wp = warm_params(*prm, &capped);
  rc = alloc_internal::solve_batch(c, B, probs, &wp, nullptr, &fn, results);
  if (rc) return rc;
  std::vector<int> redo;
  for (int b = 0; b < B; ++b)
    if (needs_fallback(results[b], capped)) redo.push_back(b);
  if (redo.empty()) return ALLOC_OK;
  std::vector<alloc_problem> rp;
  std::vector<alloc_result> rr;
  for (int b : redo) {
    rp.push_back(probs[b]);
    rr.push_back(results[b]);
  }
  rc = alloc_internal::solve_batch(c, (int)redo.size(), rp.data(), prm, nullptr, nullptr, rr.data());
  if (rc) return rc;
  for (size_t i = 0; i < redo.size(); ++i) {
    results[redo[i]] = rr[i];
    results[redo[i]].status_flags |= ALLOC_WARM_FALLBACK;
  }
  return ALLOC_OK;
}

double alloc_mlp_last_ms(alloc_mlp* net) { return net ? net->last_ms : -1.0; }

}  // extern "C"
