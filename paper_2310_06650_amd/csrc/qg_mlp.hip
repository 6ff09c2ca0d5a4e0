// Multilayer perceptron of the learned warm start (qg_mlp.h): FP32 training
// on MFMA (v_mfma_f32_16x16x4f32) and BF16 inference (v_mfma_f32_16x16x32_bf16
// with FP32 accumulation), GELU activations, mean squared error, Adam.
//
// Every matrix product goes through one tiled kernel per operand type: a
// 256-thread block computes a 64 x 64 tile of op(A) op(B) over a slice of the
// reduction dimension (grid.z splits it when the output has few tiles) and
// writes raw sums; a second kernel adds the slices in a fixed order and
// applies the layer's epilogue (bias, GELU, GELU derivative, BF16 rounding).
// With one slice and no epilogue the product is written in place.  No
// floating-point atomics: results are bitwise reproducible.
//
// MFMA operand layouts (gfx950): lane l holds A[l%16][KPL*(l/16) + i] and
// B[KPL*(l/16) + i][l%16] for i < KPL (KPL = 1 for FP32, 8 for BF16); the
// 16 x 16 result sits at D[4*(l/16) + r][l%16] in register r of lane l.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <string>

#include "qg_internal.h"
#include "qg_mlp.h"

namespace qg {
qg_status fail(qg_status s, const std::string& msg);
}

namespace {

typedef float v4f __attribute__((ext_vector_type(4)));
typedef __bf16 v8bf __attribute__((ext_vector_type(8)));

constexpr int kT = 64;        // output tile edge
constexpr int kThreads = 256;
constexpr int kLossBlocks = 256;

enum Epi { kStore = 0, kBiasGelu = 1, kBias = 2, kGeluBwd = 3, kBiasGeluBf16 = 4 };

__device__ __forceinline__ float gelu(float z) {
  return 0.5f * z * (1.0f + erff(z * 0.70710678118654752f));
}
// d gelu / dz = Phi(z) + z phi(z)
__device__ __forceinline__ float gelu_d(float z) {
  const float phi = 0.39894228040143268f * expf(-0.5f * z * z);
  return 0.5f * (1.0f + erff(z * 0.70710678118654752f)) + z * phi;
}
// FP32 -> BF16 bits, round to nearest even (finite inputs)
__device__ __forceinline__ uint16_t to_bf16(float f) {
  const unsigned u = __float_as_uint(f);
  return (uint16_t)((u + 0x7fffu + ((u >> 16) & 1u)) >> 16);
}
__device__ __forceinline__ float from_bf16(uint16_t h) { return __uint_as_float((unsigned)h << 16); }

// C (+ z * M * ldc) = op(A) op(B) over the z-th reduction slice.
// op(A)[m][k] = TA ? A[k*lda + m] : A[m*lda + k]; op(B)[k][n] likewise.
// Software-pipelined: the operands of the next 16-wide k-step are loaded
// into registers while the current one is multiplied from one of two LDS
// buffers (one barrier per k-step: a buffer is refilled only after every
// wavefront has passed the barrier that follows its last use).
template <int TA, int TB>
__global__ __launch_bounds__(kThreads) void k_gemm_f32(const float* __restrict__ A, int lda,
                                                      const float* __restrict__ B, int ldb,
                                                      float* __restrict__ C, int ldc, int M,
                                                      int N, int K, int kslice) {
  __shared__ float As[2][kT][17];
  __shared__ float Bs[2][16][kT + 1];
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int m0 = blockIdx.y * kT, n0 = blockIdx.x * kT;
  const int kb = blockIdx.z * kslice, ke = min(K, kb + kslice);
  const int wm = (wv >> 1) * 32, wn = (wv & 1) * 32;
  v4f acc[2][2];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) acc[i][j] = v4f{0.f, 0.f, 0.f, 0.f};
  float ra[4], rb[4];  // this thread's elements of the next k-step
  auto gload = [&](int k0) {
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int e = tid + q * kThreads;
      const int mm = TA ? (e & 63) : (e >> 4), kk = TA ? (e >> 6) : (e & 15);
      const int gm = m0 + mm, gk = k0 + kk;
      ra[q] = (gm < M && gk < ke) ? (TA ? A[(size_t)gk * lda + gm] : A[(size_t)gm * lda + gk]) : 0.f;
    }
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int e = tid + q * kThreads;
      const int kk = TB ? (e & 15) : (e >> 6), nn = TB ? (e >> 4) : (e & 63);
      const int gk = k0 + kk, gn = n0 + nn;
      rb[q] = (gn < N && gk < ke) ? (TB ? B[(size_t)gn * ldb + gk] : B[(size_t)gk * ldb + gn]) : 0.f;
    }
  };
  if (kb < ke) gload(kb);
  for (int k0 = kb, buf = 0; k0 < ke; k0 += 16, buf ^= 1) {
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int e = tid + q * kThreads;
      As[buf][TA ? (e & 63) : (e >> 4)][TA ? (e >> 6) : (e & 15)] = ra[q];
      Bs[buf][TB ? (e & 15) : (e >> 6)][TB ? (e >> 4) : (e & 63)] = rb[q];
    }
    __syncthreads();
    if (k0 + 16 < ke) gload(k0 + 16);
#pragma unroll
    for (int ks = 0; ks < 16; ks += 4) {
      float a[2], b[2];
#pragma unroll
      for (int i = 0; i < 2; ++i) a[i] = As[buf][wm + i * 16 + (lane & 15)][ks + (lane >> 4)];
#pragma unroll
      for (int j = 0; j < 2; ++j) b[j] = Bs[buf][ks + (lane >> 4)][wn + j * 16 + (lane & 15)];
#pragma unroll
      for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j)
          acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[i], b[j], acc[i][j], 0, 0, 0);
    }
  }
  float* Cz = C + (size_t)blockIdx.z * M * ldc;
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int row = m0 + wm + i * 16 + 4 * (lane >> 4) + r;
        const int col = n0 + wn + j * 16 + (lane & 15);
        if (row < M && col < N) Cz[(size_t)row * ldc + col] = acc[i][j][r];
      }
}

// BF16 operands, row-major A [M][K] and B [K][N], FP32 sums; pipelined like
// k_gemm_f32 with 32-wide k-steps.
__global__ __launch_bounds__(kThreads) void k_gemm_bf16(const uint16_t* __restrict__ A, int lda,
                                                       const uint16_t* __restrict__ B, int ldb,
                                                       float* __restrict__ C, int ldc, int M,
                                                       int N, int K, int kslice) {
  __shared__ uint16_t As[2][kT][32 + 8];  // [m][k]
  __shared__ uint16_t Bs[2][kT][32 + 8];  // [n][k] (transposed for 8 consecutive k per lane)
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int m0 = blockIdx.y * kT, n0 = blockIdx.x * kT;
  const int kb = blockIdx.z * kslice, ke = min(K, kb + kslice);
  const int wm = (wv >> 1) * 32, wn = (wv & 1) * 32;
  v4f acc[2][2];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) acc[i][j] = v4f{0.f, 0.f, 0.f, 0.f};
  uint16_t ra[8], rb[8];
  auto gload = [&](int k0) {
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      const int e = tid + q * kThreads;  // 64 x 32 tile
      const int mm = e >> 5, kk = e & 31;
      const int gm = m0 + mm, gk = k0 + kk;
      ra[q] = (gm < M && gk < ke) ? A[(size_t)gm * lda + gk] : (uint16_t)0;
    }
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      const int e = tid + q * kThreads;  // 32 x 64 tile, coalesced along n
      const int kk = e >> 6, nn = e & 63;
      const int gk = k0 + kk, gn = n0 + nn;
      rb[q] = (gn < N && gk < ke) ? B[(size_t)gk * ldb + gn] : (uint16_t)0;
    }
  };
  if (kb < ke) gload(kb);
  for (int k0 = kb, buf = 0; k0 < ke; k0 += 32, buf ^= 1) {
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      const int e = tid + q * kThreads;
      As[buf][e >> 5][e & 31] = ra[q];
      Bs[buf][e & 63][e >> 6] = rb[q];
    }
    __syncthreads();
    if (k0 + 32 < ke) gload(k0 + 32);
    v8bf a[2], b[2];
#pragma unroll
    for (int i = 0; i < 2; ++i) {
      const uint16_t* src = &As[buf][wm + i * 16 + (lane & 15)][8 * (lane >> 4)];
#pragma unroll
      for (int u = 0; u < 8; ++u) a[i][u] = __builtin_bit_cast(__bf16, src[u]);
    }
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      const uint16_t* src = &Bs[buf][wn + j * 16 + (lane & 15)][8 * (lane >> 4)];
#pragma unroll
      for (int u = 0; u < 8; ++u) b[j][u] = __builtin_bit_cast(__bf16, src[u]);
    }
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int j = 0; j < 2; ++j)
        acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[i], b[j], acc[i][j], 0, 0, 0);
  }
  float* Cz = C + (size_t)blockIdx.z * M * ldc;
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int row = m0 + wm + i * 16 + 4 * (lane >> 4) + r;
        const int col = n0 + wn + j * 16 + (lane & 15);
        if (row < M && col < N) Cz[(size_t)row * ldc + col] = acc[i][j][r];
      }
}

// out = epilogue(sum over slices of P[s][m][n]) for an M x N matrix (ld N).
struct EpiArgs {
  int kind;
  const float* bias;  // [N]
  float* z;           // kBiasGelu: pre-activation out; kGeluBwd: pre-activation in
  float* out;         // float result
  uint16_t* out16;    // kBiasGeluBf16
};

// The slices of 32 elements are summed by 8 groups of threads (group g takes
// slices g, g + 8, ...), the group sums then added in group order: a fixed
// order, with 8 independent chains of loads in flight per element.
__global__ __launch_bounds__(kThreads) void k_reduce_epi(const float* __restrict__ P, int slices,
                                                         int M, int N, EpiArgs ep) {
  __shared__ float red[8][33];
  const size_t MN = (size_t)M * N;
  const int c = threadIdx.x & 31, g = threadIdx.x >> 5;
  for (size_t e0 = (size_t)blockIdx.x * 32; e0 < MN; e0 += (size_t)gridDim.x * 32) {
    const size_t ec = e0 + c;
    float part = 0.f;
    if (ec < MN)
      for (int q = g; q < slices; q += 8) part += P[(size_t)q * MN + ec];
    red[g][c] = part;
    __syncthreads();
    const size_t e = ec;
    const bool mine = g == 0 && e < MN;
    float s = 0.f;
    if (mine)
      for (int q = 0; q < 8; ++q) s += red[q][c];
    __syncthreads();  // red is refilled by the next round
    if (!mine) continue;
    const int n = (int)(e % N);
    switch (ep.kind) {
      case kBiasGelu: {
        const float z = s + ep.bias[n];
        ep.z[e] = z;
        ep.out[e] = gelu(z);
        break;
      }
      case kBias: ep.out[e] = s + ep.bias[n]; break;
      case kGeluBwd: ep.out[e] = s * gelu_d(ep.z[e]); break;
      case kBiasGeluBf16: ep.out16[e] = to_bf16(gelu(s + ep.bias[n])); break;
      default: ep.out[e] = s; break;
    }
  }
}

// db[n] = sum_m dZ[m][n]: 64 columns a block, each column's rows in four
// interleaved quarters (thread q takes rows q, q + 4, ...), the quarters
// then added in order
__global__ __launch_bounds__(kThreads) void k_colsum(const float* __restrict__ dZ, int M, int N,
                                                     float* __restrict__ db) {
  __shared__ float red[4][64];
  const int c = threadIdx.x & 63, q = threadIdx.x >> 6;
  const int n = blockIdx.x * 64 + c;
  float s = 0.f;
  if (n < N)
    for (int m = q; m < M; m += 4) s += dZ[(size_t)m * N + n];
  red[q][c] = s;
  __syncthreads();
  if (q == 0 && n < N) db[n] = ((red[0][c] + red[1][c]) + red[2][c]) + red[3][c];
}

// dY = 2 (Y - T) / (M N); per-block partial sums of (Y - T)^2
__global__ __launch_bounds__(kThreads) void k_mse(const float* __restrict__ Y,
                                                  const float* __restrict__ T, size_t n, float inv,
                                                  float* __restrict__ dY, float* __restrict__ part) {
  __shared__ float red[kThreads];
  float acc = 0.f;
  for (size_t e = (size_t)blockIdx.x * kThreads + threadIdx.x; e < n;
       e += (size_t)gridDim.x * kThreads) {
    const float d = Y[e] - T[e];
    dY[e] = 2.f * d * inv;
    acc += d * d;
  }
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int s = kThreads / 2; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[blockIdx.x] = red[0];
}

// loss = inv * sum of the n <= kThreads block partials, by a tree in a fixed order
__global__ __launch_bounds__(kThreads) void k_loss_final(const float* __restrict__ part, int n,
                                                         float inv, float* loss) {
  __shared__ float red[kThreads];
  red[threadIdx.x] = (int)threadIdx.x < n ? part[threadIdx.x] : 0.f;
  __syncthreads();
  for (int s = kThreads / 2; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
    __syncthreads();
  }
  if (threadIdx.x == 0) *loss = red[0] * inv;
}

__global__ __launch_bounds__(kThreads) void k_adam_f32(float* __restrict__ p, float* __restrict__ m,
                                                       float* __restrict__ v,
                                                       const float* __restrict__ g, size_t n,
                                                       float lr, float bc1, float bc2) {
  for (size_t e = (size_t)blockIdx.x * kThreads + threadIdx.x; e < n;
       e += (size_t)gridDim.x * kThreads) {
    const float ge = g[e];
    const float mm = 0.9f * m[e] + 0.1f * ge;
    const float vv = 0.999f * v[e] + 0.001f * ge * ge;
    m[e] = mm;
    v[e] = vv;
    p[e] -= lr * (mm / bc1) / (sqrtf(vv / bc2) + 1e-8f);
  }
}

__global__ __launch_bounds__(kThreads) void k_from_bf16_bias(const uint16_t* __restrict__ b16,
                                                             int n, float* __restrict__ b) {
  const int e = blockIdx.x * kThreads + threadIdx.x;
  if (e < n) b[e] = from_bf16(b16[e]);
}

__global__ __launch_bounds__(kThreads) void k_to_bf16(const float* __restrict__ x, size_t n,
                                                      uint16_t* __restrict__ y) {
  for (size_t e = (size_t)blockIdx.x * kThreads + threadIdx.x; e < n;
       e += (size_t)gridDim.x * kThreads)
    y[e] = to_bf16(x[e]);
}

// ---------------------------------------------------------------------------
// host side

struct Ws {
  float* z[QG_MLP_MAX_DEPTH];  // pre-activations [B][width]
  float* h[QG_MLP_MAX_DEPTH];  // activations [B][width]
  float* y;                    // [B][d_out]
  float* dy;                   // [B][d_out]
  float* da;                   // [B][width]
  float* dz;                   // [B][width]
  float* part;                 // product slices
  float* loss_part;            // [kLossBlocks]
  uint16_t* a16[2];            // BF16 activations [B][max(d_in, width)]
  size_t part_floats;
  size_t total;
};

constexpr int kMaxSlices = 128;

bool valid(const qg_mlp_desc* d) {
  return d && d->d_in > 0 && d->width > 0 && d->d_out > 0 && d->depth >= 1 &&
         d->depth <= QG_MLP_MAX_DEPTH;
}

size_t al(size_t v) { return (v + 63) / 64 * 64; }

void layout(const qg_mlp_desc* d, qg_mlp_layout* L) {
  int64_t o = 0;
  int64_t fan_in = d->d_in;
  for (int i = 0; i <= d->depth; ++i) {
    const int64_t out = (i == d->depth) ? d->d_out : d->width;
    L->w_off[i] = o;
    o = (int64_t)al((size_t)(o + fan_in * out));
    L->b_off[i] = o;
    o = (int64_t)al((size_t)(o + out));
    fan_in = d->width;
  }
  for (int i = d->depth + 1; i <= QG_MLP_MAX_DEPTH; ++i) L->w_off[i] = L->b_off[i] = -1;
  L->n_params = o;
}

// product slices: about four blocks per CU when the output has few tiles,
// each slice at least 32 deep (the pipelined k-loop needs a few k-steps)
int slices_for(int M, int N, int K) {
  const int tiles = ((M + kT - 1) / kT) * ((N + kT - 1) / kT);
  int s = 1;
  while (s < kMaxSlices && tiles * s < 1024 && K / (s * 2) >= 32) s *= 2;
  return s;
}

Ws carve(const qg_mlp_desc* d, int B, void* base) {
  Ws w;
  size_t o = 0;
  auto take = [&](size_t bytes) {
    const size_t at = o;
    o = (o + bytes + 255) / 256 * 256;
    return base ? static_cast<unsigned char*>(base) + at : nullptr;
  };
  const size_t BW = (size_t)B * d->width, BO = (size_t)B * d->d_out;
  for (int i = 0; i < d->depth; ++i) {
    w.z[i] = reinterpret_cast<float*>(take(BW * 4));
    w.h[i] = reinterpret_cast<float*>(take(BW * 4));
  }
  w.y = reinterpret_cast<float*>(take(BO * 4));
  w.dy = reinterpret_cast<float*>(take(BO * 4));
  w.da = reinterpret_cast<float*>(take(BW * 4));
  w.dz = reinterpret_cast<float*>(take(BW * 4));
  // the largest sliced product: B x width outputs with up to kMaxSlices
  // slices, or one B x d_out slice
  w.part_floats = std::max((size_t)kMaxSlices * BW, BO);
  w.part = reinterpret_cast<float*>(take(w.part_floats * 4));
  w.loss_part = reinterpret_cast<float*>(take(kLossBlocks * 4));
  const size_t wide = (size_t)B * std::max(d->d_in, d->width);
  w.a16[0] = reinterpret_cast<uint16_t*>(take(wide * 2));
  w.a16[1] = reinterpret_cast<uint16_t*>(take(wide * 2));
  w.total = o;
  return w;
}

int grid1(size_t n) { return (int)std::min<size_t>(4096, (n + kThreads - 1) / kThreads); }
// k_reduce_epi: 32 elements a block and round
int grid_red(size_t n) { return (int)std::min<size_t>(4096, (n + 31) / 32); }

// C = op(A) op(B) with epilogue; slices go through ws.part
int fit_slices(int sl, int M, int N, const Ws& w) {
  while (sl > 1 && (size_t)sl * M * N > w.part_floats) sl /= 2;
  return sl;
}

hipError_t product(hipStream_t s, int ta, int tb, const float* A, int lda, const float* B, int ldb,
                   int M, int N, int K, const EpiArgs& ep, const Ws& w) {
  const int sl = fit_slices(slices_for(M, N, K), M, N, w);
  const bool direct = (sl == 1 && ep.kind == kStore);
  float* dst = direct ? ep.out : w.part;
  const int kslice = ((K + sl - 1) / sl + 15) / 16 * 16;
  const dim3 grid((N + kT - 1) / kT, (M + kT - 1) / kT, sl);
  if (!ta && !tb) hipLaunchKernelGGL((k_gemm_f32<0, 0>), grid, dim3(kThreads), 0, s, A, lda, B, ldb, dst, N, M, N, K, kslice);
  else if (ta && !tb) hipLaunchKernelGGL((k_gemm_f32<1, 0>), grid, dim3(kThreads), 0, s, A, lda, B, ldb, dst, N, M, N, K, kslice);
  else if (!ta && tb) hipLaunchKernelGGL((k_gemm_f32<0, 1>), grid, dim3(kThreads), 0, s, A, lda, B, ldb, dst, N, M, N, K, kslice);
  else hipLaunchKernelGGL((k_gemm_f32<1, 1>), grid, dim3(kThreads), 0, s, A, lda, B, ldb, dst, N, M, N, K, kslice);
  if (!direct)
    hipLaunchKernelGGL(k_reduce_epi, dim3(grid_red((size_t)M * N)), dim3(kThreads), 0, s, w.part,
                       sl, M, N, ep);
  return hipGetLastError();
}

hipError_t product16(hipStream_t s, const uint16_t* A, int lda, const uint16_t* B, int ldb, int M,
                     int N, int K, const EpiArgs& ep, const Ws& w) {
  const int sl = fit_slices(slices_for(M, N, K), M, N, w);
  const int kslice = ((K + sl - 1) / sl + 31) / 32 * 32;
  const dim3 grid((N + kT - 1) / kT, (M + kT - 1) / kT, sl);
  hipLaunchKernelGGL(k_gemm_bf16, grid, dim3(kThreads), 0, s, A, lda, B, ldb, w.part, N, M, N, K,
                     kslice);
  hipLaunchKernelGGL(k_reduce_epi, dim3(grid_red((size_t)M * N)), dim3(kThreads), 0, s, w.part, sl,
                     M, N, ep);
  return hipGetLastError();
}

bool al256(const void* p) { return (reinterpret_cast<uintptr_t>(p) & 255u) == 0; }

qg_status check_common(const qg_mlp_desc* d, int batch, const void* ws) {
  if (!valid(d)) return qg::fail(QG_ERR_ARG, "bad network description");
  if (batch < 1) return qg::fail(QG_ERR_ARG, "batch must be >= 1");
  if (!ws || !al256(ws)) return qg::fail(QG_ERR_ARG, "workspace must be non-null and 256-byte aligned");
  return QG_OK;
}

qg_status dev_fail(hipError_t e, const char* where) {
  return qg::fail(QG_ERR_DEVICE, std::string(where) + ": " + hipGetErrorString(e));
}

// forward in FP32, activations kept for the reverse pass
hipError_t forward(hipStream_t s, const qg_mlp_desc* d, const qg_mlp_layout& L, const float* P,
                   const float* x, int B, const Ws& w) {
  const float* in = x;
  int fan_in = d->d_in;
  for (int i = 0; i < d->depth; ++i) {
    EpiArgs ep{kBiasGelu, P + L.b_off[i], w.z[i], w.h[i], nullptr};
    hipError_t e = product(s, 0, 0, in, fan_in, P + L.w_off[i], d->width, B, d->width, fan_in, ep, w);
    if (e != hipSuccess) return e;
    in = w.h[i];
    fan_in = d->width;
  }
  EpiArgs ep{kBias, P + L.b_off[d->depth], nullptr, w.y, nullptr};
  return product(s, 0, 0, in, fan_in, P + L.w_off[d->depth], d->d_out, B, d->d_out, fan_in, ep, w);
}

}  // namespace

extern "C" {

qg_status qg_mlp_sizes(const qg_mlp_desc* desc, int32_t max_batch, qg_mlp_layout* lay,
                       size_t* workspace_bytes) {
  if (!valid(desc)) return qg::fail(QG_ERR_ARG, "bad network description");
  if (max_batch < 1 || !lay || !workspace_bytes) return qg::fail(QG_ERR_ARG, "bad arguments");
  layout(desc, lay);
  *workspace_bytes = carve(desc, max_batch, nullptr).total;
  return QG_OK;
}

qg_status qg_mlp_forward(const qg_mlp_desc* desc, const float* d_params, const float* d_x,
                         int32_t batch, float* d_y, void* d_ws, void* stream) {
  qg_status st = check_common(desc, batch, d_ws);
  if (st != QG_OK) return st;
  if (!d_params || !d_x || !d_y) return qg::fail(QG_ERR_ARG, "null buffer");
  qg_mlp_layout L;
  layout(desc, &L);
  const Ws w = carve(desc, batch, d_ws);
  hipStream_t s = static_cast<hipStream_t>(stream);
  hipError_t e = forward(s, desc, L, d_params, d_x, batch, w);
  if (e == hipSuccess)
    e = hipMemcpyAsync(d_y, w.y, (size_t)batch * desc->d_out * 4, hipMemcpyDeviceToDevice, s);
  return e == hipSuccess ? QG_OK : dev_fail(e, "mlp forward");
}

qg_status qg_mlp_grad(const qg_mlp_desc* desc, const float* d_params, const float* d_x,
                      const float* d_t, int32_t batch, float* d_grad, float* d_loss, void* d_ws,
                      void* stream) {
  qg_status st = check_common(desc, batch, d_ws);
  if (st != QG_OK) return st;
  if (!d_params || !d_x || !d_t || !d_grad || !d_loss) return qg::fail(QG_ERR_ARG, "null buffer");
  qg_mlp_layout L;
  layout(desc, &L);
  const Ws w = carve(desc, batch, d_ws);
  hipStream_t s = static_cast<hipStream_t>(stream);
  const int B = batch, D = desc->depth, W = desc->width;
  hipError_t e = forward(s, desc, L, d_params, d_x, B, w);
  if (e != hipSuccess) return dev_fail(e, "mlp forward");
  const size_t BO = (size_t)B * desc->d_out;
  const float inv = 1.0f / (float)BO;
  hipLaunchKernelGGL(k_mse, dim3(kLossBlocks), dim3(kThreads), 0, s, w.y, d_t, BO, inv, w.dy,
                     w.loss_part);
  hipLaunchKernelGGL(k_loss_final, dim3(1), dim3(kThreads), 0, s, w.loss_part, kLossBlocks, inv,
                     d_loss);
  // output layer: dW_out = h_D^T dY, db_out = colsum dY, dh_D = dY W_out^T
  const float* dcur = w.dy;  // gradient at the current layer's output
  int n_out = desc->d_out;
  for (int i = D; i >= 0; --i) {
    const float* in = (i == 0) ? d_x : w.h[i - 1];
    const int fan_in = (i == 0) ? desc->d_in : W;
    EpiArgs ew{kStore, nullptr, nullptr, d_grad + L.w_off[i], nullptr};
    e = product(s, 1, 0, in, fan_in, dcur, n_out, fan_in, n_out, B, ew, w);
    if (e != hipSuccess) return dev_fail(e, "mlp weight gradient");
    hipLaunchKernelGGL(k_colsum, dim3((n_out + 63) / 64), dim3(kThreads), 0, s, dcur, B, n_out,
                       d_grad + L.b_off[i]);
    if (i == 0) break;
    // dz_{i-1} = (dcur W_i^T) * gelu'(z_{i-1}), W_i is [fan_in][n_out]
    float* dst = (dcur == w.dz) ? w.da : w.dz;
    EpiArgs eb{kGeluBwd, nullptr, w.z[i - 1], dst, nullptr};
    e = product(s, 0, 1, dcur, n_out, d_params + L.w_off[i], n_out, B, fan_in, n_out, eb, w);
    if (e != hipSuccess) return dev_fail(e, "mlp activation gradient");
    dcur = dst;
    n_out = W;
  }
  e = hipGetLastError();
  return e == hipSuccess ? QG_OK : dev_fail(e, "mlp reverse");
}

qg_status qg_mlp_train_step(const qg_mlp_desc* desc, float* d_params, float* d_m, float* d_v,
                            float* d_grad, const float* d_x, const float* d_t, int32_t batch,
                            int64_t iter, float lr, float* d_loss, void* d_ws, void* stream) {
  if (!d_m || !d_v || iter < 1 || !(lr > 0.f)) return qg::fail(QG_ERR_ARG, "bad Adam arguments");
  qg_status st = qg_mlp_grad(desc, d_params, d_x, d_t, batch, d_grad, d_loss, d_ws, stream);
  if (st != QG_OK) return st;
  qg_mlp_layout L;
  layout(desc, &L);
  const float bc1 = 1.0f - std::pow(0.9f, (float)iter);
  const float bc2 = 1.0f - std::pow(0.999f, (float)iter);
  hipStream_t s = static_cast<hipStream_t>(stream);
  hipLaunchKernelGGL(k_adam_f32, dim3(grid1((size_t)L.n_params)), dim3(kThreads), 0, s, d_params,
                     d_m, d_v, d_grad, (size_t)L.n_params, lr, bc1, bc2);
  hipError_t e = hipGetLastError();
  return e == hipSuccess ? QG_OK : dev_fail(e, "mlp Adam");
}

qg_status qg_mlp_to_bf16(const qg_mlp_desc* desc, const float* d_params, uint16_t* d_params16,
                         void* stream) {
  if (!valid(desc) || !d_params || !d_params16) return qg::fail(QG_ERR_ARG, "bad arguments");
  qg_mlp_layout L;
  layout(desc, &L);
  hipStream_t s = static_cast<hipStream_t>(stream);
  hipLaunchKernelGGL(k_to_bf16, dim3(grid1((size_t)L.n_params)), dim3(kThreads), 0, s, d_params,
                     (size_t)L.n_params, d_params16);
  hipError_t e = hipGetLastError();
  return e == hipSuccess ? QG_OK : dev_fail(e, "bf16 conversion");
}

qg_status qg_mlp_forward_bf16(const qg_mlp_desc* desc, const uint16_t* d_params16,
                              const float* d_x, int32_t batch, float* d_y, void* d_ws,
                              void* stream) {
  qg_status st = check_common(desc, batch, d_ws);
  if (st != QG_OK) return st;
  if (!d_params16 || !d_x || !d_y) return qg::fail(QG_ERR_ARG, "null buffer");
  qg_mlp_layout L;
  layout(desc, &L);
  const Ws w = carve(desc, batch, d_ws);
  hipStream_t s = static_cast<hipStream_t>(stream);
  const int B = batch;
  hipLaunchKernelGGL(k_to_bf16, dim3(grid1((size_t)B * desc->d_in)), dim3(kThreads), 0, s, d_x,
                     (size_t)B * desc->d_in, w.a16[0]);
  // the epilogue adds each layer's bias widened from its BF16 image (scratch:
  // ws.dz for hidden layers, ws.dy for the output layer)
  int cur = 0, fan_in = desc->d_in;
  hipError_t e = hipSuccess;
  for (int i = 0; i < desc->depth && e == hipSuccess; ++i) {
    hipLaunchKernelGGL(k_from_bf16_bias, dim3((desc->width + kThreads - 1) / kThreads),
                       dim3(kThreads), 0, s, d_params16 + L.b_off[i], desc->width, w.dz);
    EpiArgs ep{kBiasGeluBf16, w.dz, nullptr, nullptr, w.a16[cur ^ 1]};
    e = product16(s, w.a16[cur], fan_in, d_params16 + L.w_off[i], desc->width, B, desc->width,
                  fan_in, ep, w);
    cur ^= 1;
    fan_in = desc->width;
  }
  if (e == hipSuccess) {
    hipLaunchKernelGGL(k_from_bf16_bias, dim3((desc->d_out + kThreads - 1) / kThreads),
                       dim3(kThreads), 0, s, d_params16 + L.b_off[desc->depth], desc->d_out, w.dy);
    EpiArgs ep{kBias, w.dy, nullptr, d_y, nullptr};
    e = product16(s, w.a16[cur], fan_in, d_params16 + L.w_off[desc->depth], desc->d_out, B,
                  desc->d_out, fan_in, ep, w);
  }
  if (e == hipSuccess) e = hipGetLastError();
  return e == hipSuccess ? QG_OK : dev_fail(e, "mlp bf16 forward");
}

}  // extern "C"
