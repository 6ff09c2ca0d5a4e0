// Contingency screening of the contingency solver (Alg. 2) for gfx950.
//
// An exact step scores every contingency; from its penalties z_tk the set
// scored by the following screened steps is chosen on the device, with no
// host round trip:
//   k_scr_sev      severity sev_k = max_t (z_tk - d_t c_s beta (L - 1) eps), the
//                  penalty above the no-overload value (exactly zero for an
//                  outage that overloads nothing), and the draw key of k
//   k_scr_top      worst set: contingencies with sev_k > zeta ranked by
//                  decreasing severity (smaller index first on ties); ranks
//                  by counting, every lane against all K
//   k_scr_draw     the other slots go to the contingencies outside the worst
//                  set with the smallest keys (smaller index first on ties):
//                  a uniform draw without replacement
//   k_scr_compact  slots in increasing contingency order (one block, ballot
//                  prefix sums): slot -> contingency and contingency -> slot
//   k_scr_gather   the slots' outage-factor columns into contiguous rows of
//                  the screening buffer, NaN past the set so that padding
//                  lanes never test overloaded
// Keys: output r 2^32 + k + 1 of SplitMix64 (Steele, Lea and Flood, OOPSLA
// 2014) seeded with the screening seed, r the index of the refresh.
#include <hip/hip_runtime.h>

#include <cstdint>

#include "qg_internal.h"

namespace qg {

namespace {

constexpr int kScrBlock = 256;
constexpr int kScrScan = 1024;

__device__ __forceinline__ uint64_t splitmix_key(uint64_t seed, uint64_t r, int k) {
  uint64_t z = seed + 0x9E3779B97F4A7C15ull * ((r << 32) + (uint64_t)k + 1ull);
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

// r_arg >= 0: refresh index r_arg; otherwise it follows from the solve
// schedule: the row of the step just taken holds its 0-based iteration index,
// and r = index / refresh.
__global__ __launch_bounds__(kScrBlock) void k_scr_sev(DevProblem p, const double* zval,
                                                       const double* params, const double* sched,
                                                       const int64_t* step, int64_t refresh,
                                                       uint64_t seed, int64_t r_arg, double* sev,
                                                       uint64_t* key) {
  // the no-overload value is formed exactly as in the per-contingency
  // reduction, so an outage without overload has severity exactly zero
#pragma clang fp contract(off)
  const int k = blockIdx.x * kScrBlock + threadIdx.x;
  if (k >= p.K) return;
  int64_t r = r_arg;
  if (r < 0) r = (int64_t)sched[(size_t)(step[0] - 1) * kSchedStride + 11] / refresh;
  const double eps = params[PB_EPS], beta = params[PB_BETA];
  double s = 0.0;
  for (int t = 0; t < p.T; ++t) {
    const double kt = p.dt[t] * p.c_s * beta;
    const double base = kt * ((double)(p.L - 1) * eps);
    s = fmax(s, zval[(size_t)t * p.Kp + k] - base);
  }
  sev[k] = s;
  key[k] = splitmix_key(seed, (uint64_t)r, k);
}

// Ranks by counting.  A block of 16 wavefronts owns 64 contingencies k (one
// per lane); wavefront w compares them with the chunks of 64 j's w, w + 16,
// ...: each lane loads one j of the chunk and the 64 values reach every lane
// through readlane, so the inner loop runs on registers.  The 16 partial
// counts are summed in LDS.
__device__ __forceinline__ double bcast_f64(double v, int lane) {
  const uint64_t b = (uint64_t)__double_as_longlong(v);
  const uint32_t lo = __builtin_amdgcn_readlane((int)(uint32_t)b, lane);
  const uint32_t hi = __builtin_amdgcn_readlane((int)(uint32_t)(b >> 32), lane);
  return __longlong_as_double((long long)(((uint64_t)hi << 32) | lo));
}
__device__ __forceinline__ uint64_t bcast_u64(uint64_t v, int lane) {
  const uint32_t lo = __builtin_amdgcn_readlane((int)(uint32_t)v, lane);
  const uint32_t hi = __builtin_amdgcn_readlane((int)(uint32_t)(v >> 32), lane);
  return ((uint64_t)hi << 32) | lo;
}

constexpr int kRankWaves = kScrScan / 64;

__global__ __launch_bounds__(kScrScan) void k_scr_top(const double* sev, int K, int n_top,
                                                      double zeta, int* top) {
  __shared__ int part[kRankWaves][64];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int k = blockIdx.x * 64 + lane;
  const double my = k < K ? sev[k] : 0.0;
  int rank = 0;
  for (int j0 = wv * 64; j0 < K; j0 += kRankWaves * 64) {
    const int j = j0 + lane;
    // past K: -inf, never above zeta, so it counts for nobody
    const double vj = j < K ? sev[j] : -__builtin_inf();
#pragma unroll 16
    for (int u = 0; u < 64; ++u) {
      const double v = bcast_f64(vj, u);
      rank += (v > zeta) && (v > my || (v == my && j0 + u < k));
    }
  }
  part[wv][lane] = rank;
  __syncthreads();
  if (wv == 0 && k < K) {
    int r = 0;
    for (int q = 0; q < kRankWaves; ++q) r += part[q][lane];
    top[k] = (my > zeta && r < n_top) ? 1 : 0;
  }
}

__global__ __launch_bounds__(kScrScan) void k_scr_draw(const uint64_t* key, const int* top,
                                                       int K, int n_act, int* sel) {
  __shared__ int part[kRankWaves][64];
  __shared__ int ntops[kRankWaves];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int k = blockIdx.x * 64 + lane;
  const uint64_t my = k < K ? key[k] : 0ull;
  const int mine = k < K ? top[k] : 0;
  int ntop = 0, rank = 0;
  for (int j0 = wv * 64; j0 < K; j0 += kRankWaves * 64) {
    const int j = j0 + lane;
    // past K: treated as worst-set members, which the draw skips
    const int tj = j < K ? top[j] : 1;
    const uint64_t kj = j < K ? key[j] : 0ull;
    ntop += __popcll(__builtin_amdgcn_ballot_w64(j < K && tj != 0));
#pragma unroll 16
    for (int u = 0; u < 64; ++u) {
      const int t = __builtin_amdgcn_readlane(tj, u);
      const uint64_t kk = bcast_u64(kj, u);
      rank += !t && (kk < my || (kk == my && j0 + u < k));
    }
  }
  part[wv][lane] = rank;
  if (lane == 0) ntops[wv] = ntop;
  __syncthreads();
  if (wv == 0 && k < K) {
    int r = 0, nt = 0;
    for (int q = 0; q < kRankWaves; ++q) {
      r += part[q][lane];
      nt += ntops[q];
    }
    sel[k] = (mine || r < n_act - nt) ? 1 : 0;
  }
}

__global__ __launch_bounds__(kScrScan) void k_scr_compact(const int* sel, int K, int Kp,
                                                          int* act_k, int* act_slot) {
  __shared__ int wsum[kScrScan / 64];
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  int base = 0;
  for (int c0 = 0; c0 < K; c0 += kScrScan) {
    const int k = c0 + tid;
    const bool f = k < K && sel[k] != 0;
    const uint64_t b = __builtin_amdgcn_ballot_w64(f);
    const int pre = __popcll(b & ((1ull << lane) - 1ull));
    if (lane == 0) wsum[wv] = __popcll(b);
    __syncthreads();
    int off = 0, tot = 0;
    for (int q = 0; q < kScrScan / 64; ++q) {
      const int c = wsum[q];
      off += q < wv ? c : 0;
      tot += c;
    }
    if (k < K) {
      const int slot = base + off + pre;
      act_slot[k] = f ? slot : -1;
      if (f) act_k[slot] = k;
    }
    base += tot;
    __syncthreads();
  }
  for (int s = base + tid; s < Kp; s += kScrScan) act_k[s] = 0;
}

template <typename LT> __device__ __forceinline__ LT nan_of();
template <> __device__ __forceinline__ double nan_of<double>() { return __builtin_nan(""); }
template <> __device__ __forceinline__ float nan_of<float>() { return __builtin_nanf(""); }
template <> __device__ __forceinline__ uint16_t nan_of<uint16_t>() { return 0x7FC0; }

template <typename LT>
__global__ __launch_bounds__(kScrBlock) void k_scr_gather(const LT* lodf, int Kp, int Lp,
                                                          const int* act_k, int na, int Ka,
                                                          LT* out) {
  const int s = blockIdx.x * kScrBlock + threadIdx.x;
  if (s >= Ka) return;
  const int k = s < na ? act_k[s] : 0;
  for (int l = blockIdx.y; l < Lp; l += gridDim.y)
    out[(size_t)l * Ka + s] = s < na ? lodf[(size_t)l * Kp + k] : nan_of<LT>();
}

}  // namespace

int launch_screen_gather(const Problem* pr, void* stream) {
  hipStream_t st = static_cast<hipStream_t>(stream);
  const Screen& sc = pr->scr;
  const DevProblem& dp = pr->dp;
  const dim3 grid((sc.Ka + kScrBlock - 1) / kScrBlock, pr->Lp < 65535 ? pr->Lp : 65535);
  if (dp.lodf_kind == kLodfF64)
    hipLaunchKernelGGL(k_scr_gather<double>, grid, dim3(kScrBlock), 0, st, dp.lodf, pr->Kp,
                       pr->Lp, sc.act_k, sc.n_act, sc.Ka, static_cast<double*>(sc.lodf_act));
  else if (dp.lodf_kind == kLodfF32)
    hipLaunchKernelGGL(k_scr_gather<float>, grid, dim3(kScrBlock), 0, st, dp.lodf32, pr->Kp,
                       pr->Lp, sc.act_k, sc.n_act, sc.Ka, static_cast<float*>(sc.lodf_act));
  else
    hipLaunchKernelGGL(k_scr_gather<uint16_t>, grid, dim3(kScrBlock), 0, st, dp.lodf16, pr->Kp,
                       pr->Lp, sc.act_k, sc.n_act, sc.Ka, static_cast<uint16_t*>(sc.lodf_act));
  return (int)hipGetLastError();
}

int launch_screen_select(const Problem* pr, const DevWork& w, int64_t round, void* stream) {
  hipStream_t st = static_cast<hipStream_t>(stream);
  const Screen& sc = pr->scr;
  const int K = pr->K, nb = (K + kScrBlock - 1) / kScrBlock;
  hipLaunchKernelGGL(k_scr_sev, dim3(nb), dim3(kScrBlock), 0, st, pr->dp, w.zval, w.params,
                     (const double*)w.sched, (const int64_t*)w.step, (int64_t)sc.refresh, sc.seed,
                     (int64_t)round, sc.sev, sc.key);
  const int nr = (K + 63) / 64;
  hipLaunchKernelGGL(k_scr_top, dim3(nr), dim3(kScrScan), 0, st, sc.sev, K, sc.n_top, sc.zeta,
                     sc.top);
  hipLaunchKernelGGL(k_scr_draw, dim3(nr), dim3(kScrScan), 0, st, sc.key, sc.top, K, sc.n_act,
                     sc.sel);
  hipLaunchKernelGGL(k_scr_compact, dim3(1), dim3(kScrScan), 0, st, sc.sel, K, pr->Kp, sc.act_k,
                     sc.act_slot);
  const int e = (int)hipGetLastError();
  if (e != 0) return e;
  return launch_screen_gather(pr, stream);
}

}  // namespace qg
