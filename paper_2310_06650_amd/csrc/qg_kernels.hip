// HIP kernels of one solver step for gfx950 (MI355X).
//
// Stage map (one launch each, in stream order):
//   k_forward       per-(t, branch) AC flows and penalties          (Section II-B Ex. 1, 4; II-G)
//                   + base-case DC flows on FP64 MFMA:                 (eqs. (Yb_solve)-(p_flow))
//                     F_t = ISF[:, gen] p_t - ISF load_t - mean_t ISF 1 (uniform slack)
//   k_ctg_main      per-(t, l, k) outage flows F_l + LODF_lk F_k, their (eqs. (rank_correct),
//                     penalties and partial reductions                   (sfr_pen)-(zctg), (2nd_lin_sys))
//                     (k_ctg_pm: the same stage with period-split blocks)
//   k_ctg_zred      per-(t, k) penalties z_tk, per-chunk worst and sum
//   k_ctg_asm       per-(t, l) dL/dF and dL/dqmax2 (mean + worst-contingency weights)
//                   + per-(t, bus) power balance from bus-sorted endpoint flows
//                     (LDS-staged segmented sums)                      (Ex. 4)
//                   + one block per period: device terms, reserve     (Ex. 2, 3; eq. (nlp_updated))
//                     shortfall
//   k_adjoint       dL/dp_tj (DC part) = sum_l dL/dF_tl (ISF[l][bus(j)] - rowsum_l/N)
//                     on FP64 MFMA, split over the branch dimension      (eqs. (2nd_lin_sys), (correction))
//                   + per-(t, branch) reverse of the AC flows into bus-sorted endpoint slots
//   k_final         per-(t, bus) segmented sums of endpoint adjoints and per-(t, generator)
//                     gradient assembly, then either the gradient or the fused Adam
//                     update with clip (Alg. 3), and the deterministic sum of the terms.
//
// Every reduction has a fixed order (no floating-point atomics), so a step is
// bitwise reproducible run to run.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <array>
#include <cfloat>
#include <climits>
#include <cstring>
#include <string>
#include <type_traits>
#include <vector>

#include "qg_internal.h"

namespace qg {

typedef double v4d __attribute__((ext_vector_type(4)));

struct StepParams {
  double eps, beta, rho_s;
  double alpha[QG_NCLASS];
  double bc1, bc2;
};

struct EvalArgs {
  DevProblem p;
  DevWork w;
  const double* x;
  double* grad;
  double* terms_out;
  double* m;
  double* v;
  EvalMode mode;
  int fuse_adam;
  int nb_br, nb_bus, bus_chunks, nb_gen, nsplit;
  int nLb, nKb, nKc, nLc, tc, lt;
  // partials stored sparsely with flags (the period-split map-reduce);
  // strides of w.zflag (k-blocks, l-blocks per row) and w.rflag (k-blocks)
  int sparse, zfk, zfs, rfs;
  TermOffsets toff;
  // contingencies scored this step (Alg. 2): slot s of the map-reduce holds
  // contingency act_k[s] (the identity when act_k is null), na slots in use,
  // outage factors of the slots in rows of kst entries at lodf_sel;
  // act_slot maps a contingency back to its slot (-1 when not scored)
  const int* act_k;
  const int* act_slot;
  int na, kst;
  const void* lodf_sel;
};

// ---------------------------------------------------------------------------
// small device helpers

__device__ __forceinline__ double soft_relu(double e, double eps) {
  const double m = fmax(e, 0.0);
  return sqrt(m * m + eps * eps);
}

// d sigma/de = max(e,0)/sigma(e), 0 where max(e,0) = 0
__device__ __forceinline__ double soft_relu_d(double e, double eps) {
  const double m = fmax(e, 0.0);
  if (!(m > 0.0)) return 0.0;
  return m / sqrt(m * m + eps * eps);
}

// 1/sqrt(x) for x > 0: the hardware estimate refined by two Newton steps on
// y^-2 = x (y <- y + y (1 - x y^2) / 2), which restores FP64 accuracy.
__device__ __forceinline__ double rsqrt_nr(double x) {
  double y = __builtin_amdgcn_rsq(x);
  double r = fma(-x * y, y, 1.0);
  y = fma(0.5 * y, r, y);
  r = fma(-x * y, y, 1.0);
  return fma(0.5 * y, r, y);
}

// sigma(e) = sqrt(max(e,0)^2 + eps^2) and d sigma/de = max(e,0)/sigma (0 where
// max(e,0) = 0) from one reciprocal square root, for the per-generator
// penalties: a dependent sqrt and division per term cost more than the
// whole rest of a period block at 18 periods.  Both 0 when eps = 0 and e <= 0.
__device__ __forceinline__ double soft_relu_pair(double e, double eps, double& d) {
  const double m = fmax(e, 0.0);
  const double x = fma(m, m, eps * eps);
  if (!(x > 0.0)) {
    d = 0.0;
    return 0.0;
  }
  const double r = rsqrt_nr(x);
  d = m * r;
  return x * r;
}

template <int CTRL, int ROWS>
__device__ __forceinline__ double dpp_f64(double v) {
  const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(v), CTRL, ROWS, 0xF, false);
  const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(v), CTRL, ROWS, 0xF, false);
  return __hiloint2double(hi, lo);
}

__device__ __forceinline__ double readlane_f64(double v, int lane) {
  const int lo = __builtin_amdgcn_readlane(__double2loint(v), lane);
  const int hi = __builtin_amdgcn_readlane(__double2hiint(v), lane);
  return __hiloint2double(hi, lo);
}

// Sum over the 64 lanes of a wavefront (all lanes active), returned in every
// lane.  Butterflies inside each row of 16 lanes (quad swaps, half-row and
// row mirrors) give every lane its row sum; row_bcast15 then adds row 0's
// sum into row 1 and row 2's into row 3, and row_bcast31 adds rows 0+1 into
// row 3, so lane 63 holds ((r0 + r1) + (r2 + r3)).
__device__ __forceinline__ double wave_sum(double v) {
  v += dpp_f64<0xB1, 0xF>(v);    // quad_perm [1,0,3,2]
  v += dpp_f64<0x4E, 0xF>(v);    // quad_perm [2,3,0,1]
  v += dpp_f64<0x141, 0xF>(v);   // row_half_mirror
  v += dpp_f64<0x140, 0xF>(v);   // row_mirror
  v += dpp_f64<0x142, 0xA>(v);   // row_bcast15 into rows 1 and 3
  v += dpp_f64<0x143, 0xC>(v);   // row_bcast31 into rows 2 and 3
  return readlane_f64(v, 63);
}

// Cross-half exchanges of gfx950: permlane32_swap trades lanes 32..63 of
// its first operand with lanes 0..31 of its second, permlane16_swap the odd
// 16-lane rows of the first with the even rows of the second.  After either,
// the sum of the two results holds, in the lanes whose exchanged bit is 0,
// a summed over the lane pair, and in the others b summed over the pair.
template <int W>
__device__ __forceinline__ double swap_add(double a, double b) {
  const unsigned alo = __double2loint(a), ahi = __double2hiint(a);
  const unsigned blo = __double2loint(b), bhi = __double2hiint(b);
  unsigned xlo, ylo, xhi, yhi;
  if constexpr (W == 32) {
    const auto l = __builtin_amdgcn_permlane32_swap(alo, blo, false, false);
    const auto h = __builtin_amdgcn_permlane32_swap(ahi, bhi, false, false);
    xlo = l[0]; ylo = l[1]; xhi = h[0]; yhi = h[1];
  } else {
    const auto l = __builtin_amdgcn_permlane16_swap(alo, blo, false, false);
    const auto h = __builtin_amdgcn_permlane16_swap(ahi, bhi, false, false);
    xlo = l[0]; ylo = l[1]; xhi = h[0]; yhi = h[1];
  }
  return __hiloint2double((int)xhi, (int)xlo) + __hiloint2double((int)yhi, (int)ylo);
}

// dpp_f64 for patterns that read a lane of the same row for every lane
// (quad permutations, mirrors): no lane keeps its old value, so none is set.
template <int CTRL>
__device__ __forceinline__ double dpp_f64_row(double v) {
  const int lo = __builtin_amdgcn_mov_dpp(__double2loint(v), CTRL, 0xF, 0xF, false);
  const int hi = __builtin_amdgcn_mov_dpp(__double2hiint(v), CTRL, 0xF, 0xF, false);
  return __hiloint2double(hi, lo);
}

// Wavefront totals of two per-lane values at once (all lanes active): lanes
// 0..31 return the sum of a over the 64 lanes, lanes 32..63 the sum of b.
// The 32-lane swap leaves a's pair sums in the low half and b's in the high
// half, the 16-lane swap adds the two rows of each half, and four DPP steps
// finish inside each row.
__device__ __forceinline__ double pair_sum(double a, double b) {
  double v = swap_add<32>(a, b);
  v = swap_add<16>(v, v);
  v += dpp_f64_row<0xB1>(v);     // quad_perm [1,0,3,2]
  v += dpp_f64_row<0x4E>(v);     // quad_perm [2,3,0,1]
  v += dpp_f64_row<0x141>(v);    // row_half_mirror
  v += dpp_f64_row<0x140>(v);    // row_mirror
  return v;
}

// Largest value over the 64 lanes of a wavefront (all lanes active), in every
// lane: butterflies inside each row of 16 lanes, then the two cross-row
// exchanges.  NaN inputs are dropped (fmax).
__device__ __forceinline__ double wave_max(double v) {
  v = fmax(v, dpp_f64_row<0xB1>(v));   // quad_perm [1,0,3,2]
  v = fmax(v, dpp_f64_row<0x4E>(v));   // quad_perm [2,3,0,1]
  v = fmax(v, dpp_f64_row<0x141>(v));  // row_half_mirror
  v = fmax(v, dpp_f64_row<0x140>(v));  // row_mirror
  const unsigned lo = __double2loint(v), hi = __double2hiint(v);
  auto l = __builtin_amdgcn_permlane16_swap(lo, lo, false, false);
  auto h = __builtin_amdgcn_permlane16_swap(hi, hi, false, false);
  v = fmax(__hiloint2double((int)h[0], (int)l[0]), __hiloint2double((int)h[1], (int)l[1]));
  const unsigned lo2 = __double2loint(v), hi2 = __double2hiint(v);
  l = __builtin_amdgcn_permlane32_swap(lo2, lo2, false, false);
  h = __builtin_amdgcn_permlane32_swap(hi2, hi2, false, false);
  return fmax(__hiloint2double((int)h[0], (int)l[0]), __hiloint2double((int)h[1], (int)l[1]));
}

// Read-only view of device memory in the constant address space: loads at
// wavefront-uniform addresses through it become scalar loads into SGPRs.
// Only for data that no kernel of the same launch writes.
typedef __attribute__((address_space(4))) const double cdouble;
__device__ __forceinline__ const cdouble* as_const(const double* q) {
  return (const cdouble*)q;
}

// a * b + c with c wavefront-uniform, read straight from its SGPR pair (one
// VOP3 instruction instead of a copy into VGPRs and an accumulate).
__device__ __forceinline__ double fma_uniform_c(double a, double b, double c) {
  double d;
  asm("v_fma_f64 %0, %1, %2, %3" : "=v"(d) : "v"(a), "v"(b), "s"(c));
  return d;
}
__device__ __forceinline__ float fma_uniform_c(float a, float b, float c) {
  float d;
  asm("v_fma_f32 %0, %1, %2, %3" : "=v"(d) : "v"(a), "v"(b), "s"(c));
  return d;
}

// Branch-tiled copy of F and thr (w.fh): per 8-branch tile and period one
// 128-byte row of two 64-byte halves, [F0..F3 thr0..thr3][F4..F7 thr4..thr7],
// so that one 16-dword scalar load brings the F and thr of four branches.
__device__ __forceinline__ constexpr int fh_col_f(int g) { return (g >> 2) * 8 + (g & 3); }
__device__ __forceinline__ constexpr int fh_col_h(int g) { return (g >> 2) * 8 + 4 + (g & 3); }

// ---- FP32 counterparts for the reduced-precision contingency map-reduce

// 1/sqrt(x) for x > 0 in FP32: the hardware estimate and one Newton step.
__device__ __forceinline__ float rsqrt_nr(float x) {
  float y = __builtin_amdgcn_rsqf(x);
  const float r = fmaf(-x * y, y, 1.0f);
  return fmaf(0.5f * y, r, y);
}

__device__ __forceinline__ float readlane_any(float v, int lane) {
  return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), lane));
}
__device__ __forceinline__ double readlane_any(double v, int lane) { return readlane_f64(v, lane); }
// v with lane `lane` replaced by the wavefront-uniform x
template <typename R>
__device__ __forceinline__ R writelane_any(R v, R x, int lane) {
  return (int)(threadIdx.x & 63) == lane ? x : v;
}

// The same with v_writelane (one per 32-bit half), for lanes known at compile
// time after unrolling (an immediate lane select, which also leaves the one
// scalar operand the instruction may read to x): the select form would keep
// one lane mask per constant live in SGPRs.
__device__ __forceinline__ unsigned writelane_u32(unsigned v, unsigned x, int lane) {
  asm("v_writelane_b32 %0, %1, %2" : "+v"(v) : "s"(x), "i"(lane));
  return v;
}
__device__ __forceinline__ double writelane_set(double v, double x, int lane) {
  const unsigned lo = writelane_u32((unsigned)__double2loint(v), (unsigned)__double2loint(x), lane);
  const unsigned hi = writelane_u32((unsigned)__double2hiint(v), (unsigned)__double2hiint(x), lane);
  return __hiloint2double((int)hi, (int)lo);
}
__device__ __forceinline__ float writelane_set(float v, float x, int lane) {
  return __uint_as_float(writelane_u32(__float_as_uint(v), __float_as_uint(x), lane));
}

template <int CTRL>
__device__ __forceinline__ float dpp_f32(float v) {
  return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), CTRL, 0xF, 0xF, false));
}

// FP32 form of pair_sum (the same lane pattern, one register per value).
__device__ __forceinline__ float pair_sum(float a, float b) {
  const auto x = __builtin_amdgcn_permlane32_swap(__float_as_uint(a), __float_as_uint(b), false,
                                                  false);
  float v = __uint_as_float(x[0]) + __uint_as_float(x[1]);
  const auto y = __builtin_amdgcn_permlane16_swap(__float_as_uint(v), __float_as_uint(v), false,
                                                  false);
  v = __uint_as_float(y[0]) + __uint_as_float(y[1]);
  v += dpp_f32<0xB1>(v);
  v += dpp_f32<0x4E>(v);
  v += dpp_f32<0x141>(v);
  v += dpp_f32<0x140>(v);
  return v;
}

// Raw buffer resource over `bytes` bytes from `base` (gfx9 word 3): the
// address of a buffer access is base + the lane's 32-bit offset (VGPR) + a
// wavefront-uniform offset (SGPR), so a loop that advances the uniform offset
// needs no per-lane address arithmetic.  Loads past the end return 0 and
// stores past it are dropped.
__device__ __forceinline__ __amdgpu_buffer_rsrc_t buf_rsrc(const void* base, uint32_t bytes) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(base), 0, (int)bytes, 0x00020000);
}
__device__ __forceinline__ double lodf_buf(__amdgpu_buffer_rsrc_t r, const double*, unsigned v,
                                           unsigned s) {
  return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, v, s, 0));
}
__device__ __forceinline__ float lodf_buf(__amdgpu_buffer_rsrc_t r, const float*, unsigned v,
                                          unsigned s) {
  return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, v, s, 0));
}
__device__ __forceinline__ float lodf_buf(__amdgpu_buffer_rsrc_t r, const uint16_t*, unsigned v,
                                          unsigned s) {
  return __uint_as_float((unsigned)__builtin_amdgcn_raw_buffer_load_b16(r, v, s, 0) << 16);
}

// Outage factor of the stored kind, widened to the arithmetic type.
__device__ __forceinline__ double lodf_load(const double* q, size_t e) { return q[e]; }
__device__ __forceinline__ float lodf_load(const float* q, size_t e) { return q[e]; }
__device__ __forceinline__ float lodf_load(const uint16_t* q, size_t e) {
  return __uint_as_float((unsigned)q[e] << 16);
}
__device__ __forceinline__ double lodf_value(const DevProblem& p, int l, int k) {
  const size_t e = (size_t)l * p.Kp + k;
  if (p.lodf_kind == kLodfF64) return p.lodf[e];
  if (p.lodf_kind == kLodfF32) return (double)p.lodf32[e];
  return (double)lodf_load(p.lodf16, e);
}

// Largest value over the 64 lanes of a wavefront, ties to the smaller index
// (a total order, so the combination order does not matter); every lane gets
// the winner.  Entries with index INT_MAX are empty.
__device__ __forceinline__ bool better(double v2, int i2, double v, int i) {
  if (i2 == INT_MAX) return false;
  if (i == INT_MAX) return true;
  return v2 > v || (v2 == v && i2 < i);
}

template <int CTRL>
__device__ __forceinline__ void argmax_step(double& v, int& i) {
  const double v2 = dpp_f64<CTRL, 0xF>(v);
  const int i2 = __builtin_amdgcn_update_dpp(0, i, CTRL, 0xF, 0xF, false);
  if (better(v2, i2, v, i)) { v = v2; i = i2; }
}

__device__ __forceinline__ void wave_argmax(double& v, int& i) {
  argmax_step<0xB1>(v, i);
  argmax_step<0x4E>(v, i);
  argmax_step<0x141>(v, i);
  argmax_step<0x140>(v, i);
  // every lane of a row holds the row's winner; combine rows 0..3 in order
  double bv = readlane_f64(v, 0);
  int bi = __builtin_amdgcn_readlane(i, 0);
  for (int r = 16; r < 64; r += 16) {
    const double v2 = readlane_f64(v, r);
    const int i2 = __builtin_amdgcn_readlane(i, r);
    if (better(v2, i2, bv, bi)) { bv = v2; bi = i2; }
  }
  v = bv;
  i = bi;
}

// Deterministic block sum of NV values; every thread returns the totals.
// Each wavefront reduces with DPP, then the per-wavefront sums are added in
// wavefront order.  lds holds NV * 16 doubles; ends with a barrier so that
// lds can be reused.
template <int NV>
__device__ __forceinline__ void block_sum(double (&v)[NV], double* lds) {
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6, nw = blockDim.x >> 6;
#pragma unroll
  for (int q = 0; q < NV; ++q) {
    const double ws = wave_sum(v[q]);
    if (lane == 0) lds[q * 16 + wv] = ws;
  }
  __syncthreads();
#pragma unroll
  for (int q = 0; q < NV; ++q) {
    double s = 0.0;
    for (int w = 0; w < nw; ++w) s += lds[q * 16 + w];
    v[q] = s;
  }
  __syncthreads();
}

// Block argmax (ties to the smaller index); lds holds 16 doubles and 16 ints.
__device__ __forceinline__ void block_argmax(double& v, int& i, double* ldsv, int* ldsi) {
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6, nw = blockDim.x >> 6;
  wave_argmax(v, i);
  if (lane == 0) { ldsv[wv] = v; ldsi[wv] = i; }
  __syncthreads();
  double bv = ldsv[0];
  int bi = ldsi[0];
  for (int w = 1; w < nw; ++w)
    if (better(ldsv[w], ldsi[w], bv, bi)) { bv = ldsv[w]; bi = ldsi[w]; }
  v = bv;
  i = bi;
  __syncthreads();
}

// sum_{q < n} src[q * stride] in ascending q, with up to U loads in flight.
template <int U>
__device__ __forceinline__ double strided_sum(const double* src, int n, size_t stride) {
  double acc = 0.0;
  for (int q0 = 0; q0 < n; q0 += U) {
    double v[U];
#pragma unroll
    for (int u = 0; u < U; ++u) v[u] = (q0 + u < n) ? src[(size_t)(q0 + u) * stride] : 0.0;
#pragma unroll
    for (int u = 0; u < U; ++u) acc += v[u];
  }
  return acc;
}

// Homotopy and step sizes of this step: from the arguments, or from the row
// of the schedule table (eqs. (norm_t)-(step_size), evaluated on the host per
// iteration) that the step counter points at.
__device__ void resolve_params(const EvalArgs& a, StepParams& sp) {
  if (a.mode.schedule == 0) {
    sp.eps = a.mode.eps;
    sp.beta = a.mode.beta;
    sp.rho_s = a.mode.rho_s;
    for (int c = 0; c < QG_NCLASS; ++c) sp.alpha[c] = 0.0;
    sp.bc1 = sp.bc2 = 1.0;
    return;
  }
  // the row of this step, copied ahead by the previous step (k_ctg_asm) or
  // by k_set_step: one load instead of the counter and then the row
  const double* row = a.w.snext;
  sp.eps = row[0];
  sp.beta = row[1];
  sp.rho_s = row[2];
  for (int c = 0; c < QG_NCLASS; ++c) sp.alpha[c] = row[3 + c];
  sp.bc1 = row[9];
  sp.bc2 = row[10];
}

// Contribution of one overloaded outage element: with s = sqrt(s2),
// e = s - s_ctg and sigma = sqrt(max(e,0)^2 + eps^2), returns sigma - eps (the
// penalty above its floor), and dC/dP, dC/dqmax2 scaled by kt.
template <typename R>
__device__ __forceinline__ R ctg_overload(R P, R s2, R smx, R eps, R eps2, R kt, R& dP, R& dq) {
  const R rs = rsqrt_nr(s2);
  const R s = s2 * rs;
  const R em = fmax(s - smx, R(0));
  const R w2 = fma(em, em, eps2);
  // w2 = 0 only when eps = 0 and s sits exactly on the rating: sigma = 0
  // there and the one-sided derivative is taken as 0
  const bool pos = w2 > R(0);
  const R rw = rsqrt_nr(pos ? w2 : R(1));
  const R sig = w2 * rw;
  const R gs = pos ? kt * em * rw : R(0);
  dP = gs * P * rs;
  dq = R(0.5) * gs * rs;
  return sig - eps;
}

// ---------------------------------------------------------------------------
// LDS-staged segmented sums over bus-sorted endpoint slots.  The block owns
// buses [i0, i0 + nbus) of one period; their slots are contiguous, so they are
// loaded with coalesced reads in chunks and each thread sums its own segment
// in ascending slot order.

constexpr int kSegChunk = 1024;

template <int NV>
__device__ __forceinline__ void bus_segsum(const double* const (&src)[NV], const int* bptr,
                                           int i0, int nbus, double* lds, double (&acc)[NV]) {
  const int tid = threadIdx.x;
  const int s_lo = bptr[i0], s_hi = bptr[i0 + nbus];
  int a = 0, b = 0;
  if (tid < nbus) { a = bptr[i0 + tid]; b = bptr[i0 + tid + 1]; }
#pragma unroll
  for (int q = 0; q < NV; ++q) acc[q] = 0.0;
  for (int c0 = s_lo; c0 < s_hi; c0 += kSegChunk) {
    const int c1 = min(c0 + kSegChunk, s_hi);
    for (int s = c0 + tid; s < c1; s += kBlock) {
#pragma unroll
      for (int q = 0; q < NV; ++q) lds[q * kSegChunk + (s - c0)] = src[q][s];
    }
    __syncthreads();
    const int lo = max(a, c0), hi = min(b, c1);
    for (int s = lo; s < hi; ++s) {
#pragma unroll
      for (int q = 0; q < NV; ++q) acc[q] += lds[q * kSegChunk + (s - c0)];
    }
    __syncthreads();
  }
}

// ---------------------------------------------------------------------------
// FP64 MFMA slab product.  A 256-thread block computes the 16 output columns
// [n0, n0+16) of C = A * B over the reduction range [k0, k1) (multiples of 4)
// for all MT*16 rows; aload(k, row) supplies A[row][k] (zero outside A) and B
// is row-major (ldb).  The range is split over the four wavefronts; operands
// of NB consecutive k-steps are loaded before their MFMAs so that their
// memory latencies overlap.  The partial tiles are summed in LDS in wavefront order.
// v_mfma_f64_16x16x4f64 operands: lane l holds A[l%16][l/16] and
// B[l/16][l%16]; the result D[l/16 + 4r][l%16] sits in register r of lane l.
template <int MT, int NB, class ALoad, class Epi>
__device__ __forceinline__ void mfma_slab(ALoad aload, const double* __restrict__ B, int ldb,
                                          int k0, int k1, int n0, double* lds, Epi epi) {
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wv = tid >> 6;
  const int steps = (k1 - k0) >> 2;
  const int s0 = (steps * wv) >> 2, s1 = (steps * (wv + 1)) >> 2;
  v4d acc[MT];
#pragma unroll
  for (int mt = 0; mt < MT; ++mt) acc[mt] = v4d{0.0, 0.0, 0.0, 0.0};
  const int kr = lane >> 4, cc = lane & 15;
  int st = s0;
  for (; st + NB <= s1; st += NB) {
    double bb[NB], aa[NB][MT];
#pragma unroll
    for (int u = 0; u < NB; ++u) {
      const int k = k0 + (st + u) * 4 + kr;
      bb[u] = B[(size_t)k * ldb + n0 + cc];
#pragma unroll
      for (int mt = 0; mt < MT; ++mt) aa[u][mt] = aload(k, mt * 16 + cc);
    }
#pragma unroll
    for (int u = 0; u < NB; ++u)
#pragma unroll
      for (int mt = 0; mt < MT; ++mt)
        acc[mt] = __builtin_amdgcn_mfma_f64_16x16x4f64(aa[u][mt], bb[u], acc[mt], 0, 0, 0);
  }
  if (st < s1) {
    // the last, partial batch: its loads in flight together as well (the
    // step range is wavefront-uniform, so the guards do not diverge)
    double bb[NB], aa[NB][MT];
#pragma unroll
    for (int u = 0; u < NB; ++u) {
      const bool in = st + u < s1;
      const int k = k0 + (st + u) * 4 + kr;
      bb[u] = in ? B[(size_t)k * ldb + n0 + cc] : 0.0;
#pragma unroll
      for (int mt = 0; mt < MT; ++mt) aa[u][mt] = in ? aload(k, mt * 16 + cc) : 0.0;
    }
#pragma unroll
    for (int u = 0; u < NB; ++u)
      if (st + u < s1)
#pragma unroll
        for (int mt = 0; mt < MT; ++mt)
          acc[mt] = __builtin_amdgcn_mfma_f64_16x16x4f64(aa[u][mt], bb[u], acc[mt], 0, 0, 0);
  }
#pragma unroll
  for (int mt = 0; mt < MT; ++mt)
#pragma unroll
    for (int r = 0; r < 4; ++r) lds[((wv * MT + mt) * 4 + r) * 64 + lane] = acc[mt][r];
  __syncthreads();
  for (int e = tid; e < MT * 256; e += kBlock) {
    double s = 0.0;
#pragma unroll
    for (int w = 0; w < 4; ++w) s += lds[w * MT * 256 + e];
    const int mt = e >> 8, rem = e & 255, r = rem >> 6, ln = rem & 63;
    const int row = mt * 16 + (ln >> 4) + 4 * r;
    const int col = n0 + (ln & 15);
    epi(row, col, s);
  }
  __syncthreads();
}

// NB: k-steps whose operands are loaded together; more steps in flight
// cost registers (the flow product shares its kernel with the branch and
// period blocks, so it takes 4 with 3-4 row tiles).
template <int NB34, class ALoad, class Epi>
__device__ __forceinline__ void mfma_slab_dispatch(int mtiles, ALoad aload, const double* B,
                                                   int ldb, int k0, int k1, int n0, double* lds,
                                                   Epi epi) {
  switch (mtiles) {
    case 1: mfma_slab<1, 8>(aload, B, ldb, k0, k1, n0, lds, epi); break;
    case 2: mfma_slab<2, 8>(aload, B, ldb, k0, k1, n0, lds, epi); break;
    case 3: mfma_slab<3, NB34>(aload, B, ldb, k0, k1, n0, lds, epi); break;
    default: mfma_slab<4, NB34>(aload, B, ldb, k0, k1, n0, lds, epi); break;
  }
}

// ---------------------------------------------------------------------------
// K1: branch forward, reserve and padding blocks, flow slabs

// Consecutive block indices go to the eight XCDs in turn.  xcd_group(p, n)
// renumbers block p of n so that the blocks of one XCD take one contiguous
// range of the logical order (the first n % 8 ranges one block longer), so
// that neighbouring logical blocks share an L2: the consecutive branches of
// a period store their bus-sorted endpoint slots through it (which merges
// the scattered stores into whole lines), and the blocks that read one
// operand fetch it from memory once per XCD.  Used by the branch blocks of
// the forward and adjoint kernels, the flow-adjoint assembly and the
// adjoint product's slabs.
__device__ __forceinline__ int xcd_group(int p, int n) {
  const int q = n >> 3, rem = n & 7, x = p & 7, i = p >> 3;
  return x * q + min(x, rem) + i;
}

__device__ void branch_forward(const EvalArgs& a, const StepParams& sp, int blk, double* lds) {
  const DevProblem& p = a.p;
  const DevWork& w = a.w;
  const int T = p.T, L = p.L, N = p.N;
  const int idx = blk * kBlock + threadIdx.x;
  double part[2] = {0.0, 0.0};
  if (idx < T * L) {
    const int t = idx / L, l = idx - t * L;
    const double* V = a.x;
    const double* TH = a.x + (size_t)T * N;
    const int f = p.br_from[l], o = p.br_to[l];
    const double vf = V[(size_t)t * N + f], vt = V[(size_t)t * N + o];
    const double d = TH[(size_t)t * N + f] - TH[(size_t)t * N + o];
    double sn, cs;
    sincos(d, &sn, &cs);
    const double g = p.br_g[l], b = p.br_b[l], bh = p.br_bh[l];
    const double vv = vf * vt;
    const double pf = g * vf * vf + vv * (-g * cs - b * sn);
    const double qf = -(b + bh) * vf * vf + vv * (b * cs - g * sn);
    const double pt = g * vt * vt + vv * (-g * cs + b * sn);
    const double qt = -(b + bh) * vt * vt + vv * (b * cs + g * sn);
    const size_t ep = (size_t)t * p.twoL;
    w.epP[ep + p.slot_fr[l]] = pf;
    w.epP[ep + p.slot_to[l]] = pt;
    w.epQ[ep + p.slot_fr[l]] = qf;
    w.epQ[ep + p.slot_to[l]] = qt;
    // thermal penalty on the larger side (ties: from side), Example 1
    const double sf = sqrt(pf * pf + qf * qf), st = sqrt(pt * pt + qt * qt);
    const bool use_f = sf >= st;
    const double eb = (use_f ? sf : st) - p.br_smax[l];
    const double kbr = p.dt[t] * p.c_s * sp.beta;
    double kth;
    part[0] = kbr * soft_relu_pair(eb, sp.eps, kth);
    kth *= kbr;
    double kpf = 0.0, kqf = 0.0, kpt = 0.0, kqt = 0.0;
    if (use_f) {
      if (sf > 0.0) { kpf = kth * pf / sf; kqf = kth * qf / sf; }
    } else {
      if (st > 0.0) { kpt = kth * pt / st; kqt = kth * qt / st; }
    }
    // angle-difference penalty
    const double ea = fabs(d) - p.ang_max;
    const double kang = p.dt[t] * p.c_ang * sp.beta;
    double ka;
    part[1] = kang * soft_relu_pair(ea, sp.eps, ka);
    const double sgn = d > 0.0 ? 1.0 : (d < 0.0 ? -1.0 : 0.0);
    const double kd = kang * ka * sgn;
    // reactive part of the contingency flows: max(q_fr^2, q_to^2), ties: from
    const double qf2 = qf * qf, qt2 = qt * qt;
    const bool qfr = qf2 >= qt2;
    const double qm2 = qfr ? qf2 : qt2;
    w.q2[(size_t)t * p.Lp + l] = qm2;
    // radius of the map-reduce's first test: with margins of 2^-40 on s_ctg^2
    // and 2^-50 on the root, fl(P^2 + qmax2) > s_ctg^2 implies |P| > thr
    // under FP64 rounding; -1 (every flow passes) where qmax2 alone comes
    // within the margin of the rating
    const double A = p.ctg_smax2[l] * (1.0 - 0x1p-40) - qm2;
    const double thr = A > 0.0 ? sqrt(A) * (1.0 - 0x1p-50) : -1.0;
    w.thr[(size_t)t * p.Lp + l] = thr;
    w.fh[((size_t)(l >> 3) * T + t) * 16 + fh_col_h(l & 7)] = thr;
    const size_t TL = (size_t)T * L, e = (size_t)t * L + l;
    w.bco[0 * TL + e] = cs;
    w.bco[1 * TL + e] = sn;
    w.bco[2 * TL + e] = kpf;
    w.bco[3 * TL + e] = kqf;
    w.bco[4 * TL + e] = kpt;
    w.bco[5 * TL + e] = kqt;
    w.bco[6 * TL + e] = kd;
    w.bco[7 * TL + e] = qfr ? 2.0 * qf : 0.0;
    w.bco[8 * TL + e] = qfr ? 0.0 : 2.0 * qt;
  }
  block_sum<2>(part, lds);
  if (threadIdx.x == 0) {
    w.tpart[a.toff.br + blk] = part[0];
    w.tpart[a.toff.ang + blk] = part[1];
  }
}

// One block per period t and slice sl of 256 generators, one thread per
// generator: block-bid cost, no-load, start-up/shut-down and reserve costs
// (Examples 2-3), the penalised device constraints of eq. (nlp_updated) and
// their partials, and the slice's sums of the cost and penalty terms.  The
// next period's terms that depend on this period's p and u are included, so
// each thread writes only its own partials; the reserve shortfall, which
// needs the whole period's reserve, is reserve_pad_block's.  Only the final
// kernel reads what it writes, so it runs in k_ctg_asm's launch, beside the
// contingency reductions: in the forward kernel its registers (the most of
// any block there) held that kernel to four wavefronts per SIMD.
__device__ void period_block(const EvalArgs& a, const StepParams& sp, int t, int sl,
                             double* lds) {
  const DevProblem& p = a.p;
  const DevWork& w = a.w;
  const int T = p.T, N = p.N, G = p.G, M = p.M;
  const int tid = threadIdx.x;
  const double* xP = a.x + 2 * (size_t)T * N;
  const double* xQ = xP + (size_t)T * G;
  const double* xR = xQ + (size_t)T * G;
  const double* xU = xR + (size_t)T * G;
  const size_t TG = (size_t)T * G;
  const double dtt = p.dt[t];
  const double kpen = sp.rho_s * p.rho * sp.beta * dtt;
  const double eps = sp.eps;
  double acc[2] = {0.0, 0.0};  // dev, pen
  const int j = sl * kBlock + tid;
  if (j < G) {
    const size_t e = (size_t)t * G + j;
    // every load of the generator first, so that their latencies overlap
    const double pj = xP[e], qj = xQ[e], rj = xR[e], uj = xU[e];
    const double pm1 = t > 0 ? xP[e - G] : p.p0[j];
    const double um1 = t > 0 ? xU[e - G] : p.u0[j];
    const bool nxt = t + 1 < T;
    const double p1 = nxt ? xP[e + G] : 0.0, u1 = nxt ? xU[e + G] : 0.0;
    const double pmax = p.pmax[j], pmin = p.pmin[j], qmax = p.qmax[j], qmin = p.qmin[j];
    const double rmax = p.rmax[j], ru = p.ru[j], rd = p.rd[j], rusu = p.rusu[j];
    const double rdsd = p.rdsd[j], con = p.con[j], csu = p.csu[j], csd = p.csd[j];
    const double cr = p.cr[j];
    double sz4[4], cm4[4], pc4[4];
#pragma unroll
    for (int m = 0; m < 4; ++m) {
      const bool in = m < M;
      sz4[m] = in ? p.seg_size[j * M + m] : 0.0;
      cm4[m] = in ? p.seg_cost[j * M + m] : 0.0;
      pc4[m] = in ? p.pcum[j * M + m] : 0.0;
    }
    // block-bid energy cost, eq. (costs): sum_m c_m max(min(p - Pcum_{m-1}, D_m), 0)
    double cost = 0.0, dcost = 0.0, lo = 0.0;
#pragma unroll
    for (int m = 0; m < 4; ++m) {
      if (m < M) {
        const double am = pj - lo;
        cost += cm4[m] * fmax(fmin(am, sz4[m]), 0.0);
        if (am > 0.0 && am <= sz4[m]) dcost += cm4[m];
        lo = pc4[m];
      }
    }
    for (int m = 4; m < M; ++m) {
      const double am = pj - lo;
      const double sz = p.seg_size[j * M + m], cm = p.seg_cost[j * M + m];
      cost += cm * fmax(fmin(am, sz), 0.0);
      if (am > 0.0 && am <= sz) dcost += cm;
      lo = p.pcum[j * M + m];
    }
    const double du = uj - um1;
    const double dev = dtt * cost + dtt * con * uj + csu * fmax(du, 0.0) +
                       csd * fmax(-du, 0.0) + dtt * cr * rj;
    double gp = dtt * dcost;
    double gu = dtt * con + (du > 0.0 ? csu : 0.0) - (-du > 0.0 ? csd : 0.0);
    double gr = dtt * cr;
    double gq = 0.0;
    if (nxt) {
      const double du1 = u1 - uj;
      gu -= (du1 > 0.0 ? csu : 0.0) - (-du1 > 0.0 ? csd : 0.0);
    }
    double pen = 0.0, a_, dd;
    a_ = pj + rj - pmax * uj;                             // headroom
    pen += soft_relu_pair(a_, eps, dd); dd *= kpen;
    gp += dd; gr += dd; gu -= dd * pmax;
    a_ = pmin * uj - pj;                                  // minimum output
    pen += soft_relu_pair(a_, eps, dd); dd *= kpen;
    gu += dd * pmin; gp -= dd;
    a_ = pj - pm1 - dtt * (ru * uj + rusu * (1.0 - uj));  // ramp up
    pen += soft_relu_pair(a_, eps, dd); dd *= kpen;
    gp += dd; gu -= dd * dtt * (ru - rusu);
    a_ = pm1 - pj - dtt * (rd * uj + rdsd * (1.0 - uj));  // ramp down
    pen += soft_relu_pair(a_, eps, dd); dd *= kpen;
    gp -= dd; gu -= dd * dtt * (rd - rdsd);
    a_ = qj - qmax * uj;                                  // reactive upper
    pen += soft_relu_pair(a_, eps, dd); dd *= kpen;
    gq += dd; gu -= dd * qmax;
    a_ = qmin * uj - qj;                                  // reactive lower
    pen += soft_relu_pair(a_, eps, dd); dd *= kpen;
    gu += dd * qmin; gq -= dd;
    a_ = rj - rmax * uj;                                  // reserve capability
    pen += soft_relu_pair(a_, eps, dd); dd *= kpen;
    gr += dd; gu -= dd * rmax;
    if (nxt) {  // the next period's ramp constraints depend on p_t
      const double dt1 = p.dt[t + 1];
      const double k1 = sp.rho_s * p.rho * sp.beta * dt1;
      a_ = p1 - pj - dt1 * (ru * u1 + rusu * (1.0 - u1));
      double d1;
      (void)soft_relu_pair(a_, eps, d1);
      gp -= k1 * d1;
      a_ = pj - p1 - dt1 * (rd * u1 + rdsd * (1.0 - u1));
      (void)soft_relu_pair(a_, eps, d1);
      gp += k1 * d1;
    }
    w.gdev[0 * TG + e] = gp;
    w.gdev[1 * TG + e] = gq;
    w.gdev[2 * TG + e] = gr;
    w.gdev[3 * TG + e] = gu;
    acc[0] = dev;
    acc[1] = kpen * pen;
  }
  block_sum<2>(acc, lds);
  if (tid == 0) {
    const int q = t * ((G + kBlock - 1) / kBlock) + sl;
    w.tpart[a.toff.dev + q] = acc[0];
    w.tpart[a.toff.pen + q] = acc[1];
  }
}

// Period t's reserve shortfall penalty and its derivative (eq.
// (nlp_updated)), which every generator's reserve partial needs; and the
// padding of period t that the map-reduce reads: branches past L pass
// every test (q2 = 0, radius -1), outages past K have no flow.
__device__ void reserve_pad_block(const EvalArgs& a, const StepParams& sp, int t, double* lds) {
  const DevProblem& p = a.p;
  const DevWork& w = a.w;
  const int tid = threadIdx.x, T = p.T, G = p.G;
  const double* xR = a.x + 2 * (size_t)T * p.N + 2 * (size_t)T * G;
  double acc[1] = {0.0};
  for (int j = tid; j < G; j += kBlock) acc[0] += xR[(size_t)t * G + j];
  block_sum<1>(acc, lds);
  if (tid == 0) {
    const double short_ = p.rsv_req[t] - acc[0];
    const double krs = p.dt[t] * p.c_rsv * sp.beta;
    w.tpart[a.toff.rsv + t] = krs * soft_relu(short_, sp.eps);
    w.drs[t] = krs * soft_relu_d(short_, sp.eps);
  }
  for (int l = p.L + tid; l < p.Lp; l += kBlock) {
    w.q2[(size_t)t * p.Lp + l] = 0.0;
    w.thr[(size_t)t * p.Lp + l] = -1.0;
    w.fh[((size_t)(l >> 3) * p.T + t) * 16 + fh_col_h(l & 7)] = -1.0;
  }
  for (int k = p.K + tid; k < p.Kp; k += kBlock) w.Fk[(size_t)t * p.Kp + k] = 0.0;
}

// LDS of a kernel that runs both segmented sums and an MFMA slab: the slab
// keeps four wavefronts x up to 4 row tiles x 256 partial results.
constexpr int kSlabLds = 4 * 4 * 256;
static_assert(kSlabLds >= 2 * kSegChunk + 8 * kBlock, "LDS carve");
// LDS of the forward kernel: the flow slab's single row tile (its block sums
// need 32 doubles), so that LDS does not limit its blocks per CU.
constexpr int kFwdLds = 4 * 1 * 256;
static_assert(kFwdLds >= 2 * 16, "LDS carve");

// Base-case DC flows of 16 branches for 16 periods, on FP64 MFMA, with the
// uniform slack folded into the operand: F[t][l] = sum_j p_tj (ISF[l][bus(j)]
// - rowsum_l / N) - c[t][l], where the per-grid constant c holds the loads'
// part (ISF load_t - rowsum_l sum_i load_ti / N).  Also the outaged branches'
// flows.  One block per (16 branches, 16 periods): a single row tile keeps
// eight k-steps of operands in flight (the k-loop's load round trips, not
// the MFMAs, set a slab's time).
__device__ void flow_slab(const EvalArgs& a, int blk, double* smem) {
  const DevProblem& p = a.p;
  const DevWork& w = a.w;
  const int T = p.T, G = p.G, Lp = p.Lp, Kp = p.Kp, N = p.N;
  const int mtiles = p.Tp / 16;
  // consecutive blocks go to the eight XCDs in turn: the period tiles of a
  // slab take block indices eight apart, so they run on one XCD and its L2
  // fetches the slab's ISF columns once (the last group of fewer than eight
  // slabs spreads them over its own slabs' count)
  const int nsl = Lp / 16, grp = 8 * mtiles;
  const int q = blk / grp, r = blk - q * grp;
  const int ns = min(8, nsl - 8 * q);
  const int slab = 8 * q + r % ns, r0 = (r / ns) * 16;
  const double* xP = a.x + 2 * (size_t)T * N;
  const int n0 = slab * 16;
  double* F = w.F;
  double* Fk = w.Fk;
  double* FH = w.fh;
  const int* kof = p.kof;
  const double* cload = p.cload;
  auto aload = [=](int k, int row) -> double {
    const int t = r0 + row;
    return (t < T && k < G) ? xP[(size_t)t * G + k] : 0.0;
  };
  auto epi = [=](int row, int col, double v) {
    const int t = r0 + row;
    if (t < T) {
      const double f = v - cload[(size_t)t * Lp + col];
      F[(size_t)t * Lp + col] = f;
      FH[((size_t)(col >> 3) * T + t) * 16 + fh_col_f(col & 7)] = f;
      const int k = kof[col];
      if (k >= 0) Fk[(size_t)t * Kp + k] = f;
    }
  };
  mfma_slab<1, 8>(aload, p.isf_gT, Lp, 0, p.G4, n0, smem, epi);
}

// Blocks [0, T): the reserve shortfall and the padding of one period each;
// [T, T + nb_br): branch forward; then (Lp / 16) x (Tp / 16) flow slabs.
__device__ __forceinline__ void forward_body(const EvalArgs& a, int b, double* smem) {
  StepParams sp;
  resolve_params(a, sp);
  if (b == 0 && threadIdx.x == 0) {
    double* pb = a.w.params;
    pb[PB_EPS] = sp.eps;
    pb[PB_BETA] = sp.beta;
    pb[PB_RHO] = sp.rho_s;
    for (int c = 0; c < QG_NCLASS; ++c) pb[PB_ALPHA + c] = sp.alpha[c];
    pb[PB_BC1] = sp.bc1;
    pb[PB_BC2] = sp.bc2;
  }
  if (b < a.p.T)
    reserve_pad_block(a, sp, b, smem);
  else if (b < a.nb_br + a.p.T)
    branch_forward(a, sp, xcd_group(b - a.p.T, a.nb_br), smem);
  else
    flow_slab(a, b - a.nb_br - a.p.T, smem);
}

__global__ __launch_bounds__(kBlock) void k_forward(EvalArgs a) {
  __shared__ double smem[kFwdLds];
  forward_body(a, blockIdx.x, smem);
}

// Per-(t, bus) power balance (Example 4): segmented sums of the bus's
// endpoint flows staged through LDS, minus its generators; multipliers and
// the soft-abs value.
__device__ void bus_balance(const EvalArgs& a, int blk, double* smem) {
  const DevProblem& p = a.p;
  const DevWork& w = a.w;
  const int tid = threadIdx.x;
  const int t = blk / a.bus_chunks;
  const int c = blk - t * a.bus_chunks;
  const int i0 = c * kBlock;
  const int nbus = min(kBlock, p.N - i0);
  const double eps = w.params[PB_EPS], beta = w.params[PB_BETA];
  const double* src[2] = {w.epP + (size_t)t * p.twoL, w.epQ + (size_t)t * p.twoL};
  double fl[2];
  bus_segsum<2>(src, p.bptr, i0, nbus, smem, fl);
  double part[1] = {0.0};
  if (tid < nbus) {
    const int i = i0 + tid;
    const double* xP = a.x + 2 * (size_t)p.T * p.N;
    const double* xQ = xP + (size_t)p.T * p.G;
    double sp_ = 0.0, sq = 0.0;
    for (int g = p.gptr[i]; g < p.gptr[i + 1]; ++g) {
      const size_t e = (size_t)t * p.G + p.glist[g];
      sp_ += xP[e];
      sq += xQ[e];
    }
    const size_t ti = (size_t)t * p.N + i;
    const double dp = p.load_p[ti] + fl[0] - sp_;
    const double dq = p.load_q[ti] + fl[1] - sq;
    const double kb = p.dt[t] * beta;
    // |.|_eps = sqrt(v^2 + eps^2) and its derivative v / |.|_eps from one
    // reciprocal square root each (0 where both vanish)
    const double xp = fma(dp, dp, eps * eps), xq = fma(dq, dq, eps * eps);
    const double rp = xp > 0.0 ? rsqrt_nr(xp) : 0.0, rq = xq > 0.0 ? rsqrt_nr(xq) : 0.0;
    const double lp = kb * p.c_p * (dp * rp), lq = kb * p.c_q * (dq * rq);
    w.lamp[ti] = lp;
    w.lamq[ti] = lq;
    // the same multipliers per generator of the bus (read by k_final)
    for (int g = p.gptr[i]; g < p.gptr[i + 1]; ++g) {
      const size_t e = (size_t)t * p.G + p.glist[g];
      w.lamg[e] = lp;
      w.lamqg[e] = lq;
    }
    part[0] = kb * (p.c_p * (xp * rp) + p.c_q * (xq * rq));
  }
  block_sum<1>(part, smem);
  if (tid == 0) w.tpart[a.toff.bal + blk] = part[0];
}

// ---------------------------------------------------------------------------
// K3: contingency map-reduce over (t, l, k).
//
// A wavefront owns 64 contingencies (one per lane) and BL consecutive
// branches; its BL outage factors stay in registers.  A block stacks WL
// wavefronts along l and covers the periods [t0, t0 + TC) (grid.z splits
// the periods).  The branch quantities F_tl, qmax2_tl and s_ctg^2 are the
// same for every lane, so they are read with scalar loads into SGPRs; the
// flows of the block's 64 outaged branches are staged in LDS.  For each
// period and group of 8 branches every lane forms the post-outage flows
// P = F_tl + LODF_lk F_tk and tests P^2 + qmax2_tl > s_ctg^2 (one compare
// into a ballot per branch).  Only a branch with an overloaded lane
// evaluates soft-ReLUs and sums dP (-> R, d/dF_tl) and dq (-> Q,
// d/dqmax2_tl) over its 64 lanes; the other branches store zero partials.
// z_tk and S_tk (the derivative through F_tk) accumulate in the lane over l
// and are summed over the block's wavefronts in LDS.  The outaged branch
// itself and the padding carry a NaN factor, so they never test overloaded.

// LT: storage type of the outage factors (double, float, or BF16 bits);
// R: arithmetic type (double with FP64 factors, float otherwise).
template <int BL, typename LT>
__global__ __launch_bounds__(512) void k_ctg_main(EvalArgs a, const LT* __restrict__ lodf) {
  static_assert(BL % 8 == 0 && BL <= 32, "branches per wavefront");
  typedef typename std::conditional<std::is_same<LT, double>::value, double, float>::type R;
  constexpr bool kF64 = std::is_same<R, double>::value;
  // LDS: sFk[TC][64] (outaged branches' flows), then per period and
  // wavefront the lanes' z and S: zsh[TC][WL][64], ssh[TC][WL][64]
  extern __shared__ double dyn[];
  const DevProblem& p = a.p;
  const DevWork& w = a.w;
  const int lane = threadIdx.x & 63;
  const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int WL = blockDim.x >> 6;
  const int lb = blockIdx.x, kb = blockIdx.y;
  const int T = p.T, Lp = p.Lp, Kp = p.Kp;
  const int TC = a.tc;
  const int t0 = blockIdx.z * TC;
  const int nt = min(TC, T - t0);
  const int k = kb * 64 + lane;  // slot of the lane
  double* sFk = dyn;
  double* zsh = dyn + TC * 64;
  double* ssh = zsh + TC * WL * 64;
  for (int e = threadIdx.x; e < nt * 64; e += blockDim.x) {
    const int tt = e >> 6, s = kb * 64 + (e & 63);
    sFk[e] = w.Fk[(size_t)(t0 + tt) * Kp + (a.act_k ? a.act_k[s] : s)];
  }
  const cdouble* Sc = as_const(p.ctg_smax2);
  const cdouble* Mc = as_const(p.ctg_smax);
  const cdouble* Dc = as_const(p.dt);
  const double beta = w.params[PB_BETA];
  const R eps = (R)w.params[PB_EPS];
  const R eps2 = eps * eps;
  // the block covers a.lt consecutive tiles of WL * BL branches; z and S of
  // each (period, wavefront, lane) accumulate over them in LDS
  for (int it = 0; it < a.lt; ++it) {
    const int lbase = __builtin_amdgcn_readfirstlane((lb * a.lt + it) * BL * WL + wv * BL);
    const bool on = lbase < Lp;
    R lod[BL], smx2[BL];
    // lane e of chunk c holds F, qmax2 and (FP64) the test radius thr of
    // period t0 + e / 8, branch lbase + 8 c + e % 8 (TC * 8 <= 64 entries)
    R fv[BL / 8], qv[BL / 8], hv[BL / 8];
    if (on) {
#pragma unroll
      for (int j = 0; j < BL; ++j) {
        lod[j] = lodf_load(lodf, (size_t)(lbase + j) * a.kst + k);
        smx2[j] = (R)Sc[lbase + j];
      }
      const int et = lane >> 3, eg = lane & 7;
#pragma unroll
      for (int c = 0; c < BL / 8; ++c) {
        fv[c] = R(0);
        qv[c] = R(0);
        hv[c] = R(0);
        if (et < nt) {
          const size_t e = (size_t)(t0 + et) * Lp + lbase + c * 8 + eg;
          fv[c] = (R)w.F[e];
          qv[c] = (R)w.q2[e];
          if constexpr (kF64) hv[c] = w.thr[e];
        }
      }
    }
    if (it == 0) __syncthreads();  // sFk staged
    // R and Q of (period t0 + e / 8, branch lbase + 8 c + e % 8) gather in
    // lane e of racc[c], qacc[c] (zero where nothing is overloaded) and go
    // out once per tile, so the period loop itself stores nothing
    R racc[BL / 8], qacc[BL / 8];
#pragma unroll
    for (int c = 0; c < BL / 8; ++c) {
      racc[c] = R(0);
      qacc[c] = R(0);
    }
    for (int tt = 0; tt < nt; ++tt) {
      const int t = t0 + tt;
      R zacc = R(0), sacc = R(0);
      if (on) {
        const R fk = (R)sFk[tt * 64 + lane];
#pragma unroll
        for (int c = 0; c < BL / 8; ++c) {
          R Fr[8], Qr[8], P[8];
          unsigned rows = 0;
          if constexpr (kF64) {
            // FP64: |P| > thr, which every element of the exact test passes
            // (the radius of k_forward); the exact test follows per branch
#pragma unroll
            for (int g = 0; g < 8; ++g) {
              Fr[g] = readlane_any(fv[c], tt * 8 + g);
              const R Hr = readlane_any(hv[c], tt * 8 + g);
              P[g] = fma_uniform_c(lod[c * 8 + g], fk, Fr[g]);
              if (__builtin_amdgcn_ballot_w64(fabs(P[g]) > Hr)) rows |= 1u << g;
            }
          } else {
#pragma unroll
            for (int g = 0; g < 8; ++g) {
              Fr[g] = readlane_any(fv[c], tt * 8 + g);
              Qr[g] = readlane_any(qv[c], tt * 8 + g);
            }
#pragma unroll
            for (int g = 0; g < 8; ++g) {
              const int j = c * 8 + g;
              P[g] = fma_uniform_c(lod[j], fk, Fr[g]);
              const R s2 = fma_uniform_c(P[g], P[g], Qr[g]);
              if (__builtin_amdgcn_ballot_w64(s2 > smx2[j])) rows |= 1u << g;
            }
          }
          if (rows) {
            const R kt = (R)(Dc[t] * p.c_s * beta);
#pragma unroll
            for (int g = 0; g < 8; ++g) {
              if ((rows >> g) & 1u) {
                const int j = c * 8 + g;
                if constexpr (kF64) Qr[g] = readlane_any(qv[c], tt * 8 + g);
                // the square is formed again (the same fused operation, so
                // the same value) rather than kept across the test of all
                // eight branches: fewer live registers
                const R s2 = fma(P[g], P[g], Qr[g]);
                R dP = R(0), dq = R(0);
                if (s2 > smx2[j]) {
                  zacc += ctg_overload(P[g], s2, (R)Mc[lbase + j], eps, eps2, kt, dP, dq);
                  sacc = fma(lod[j], dP, sacc);
                }
                const R r = pair_sum(dP, dq);  // lane 0: sum of dP, lane 32: of dq
                racc[c] = writelane_any(racc[c], readlane_any(r, 0), tt * 8 + g);
                qacc[c] = writelane_any(qacc[c], readlane_any(r, 32), tt * 8 + g);
              }
            }
          }
        }
      }
      const int zi = (tt * WL + wv) * 64 + lane;
      if (it == 0) {
        zsh[zi] = (double)zacc;
        ssh[zi] = (double)sacc;
      } else {
        zsh[zi] += (double)zacc;
        ssh[zi] += (double)sacc;
      }
    }
    if (on && lane < nt * 8) {
      const size_t o = ((size_t)kb * T + t0 + (lane >> 3)) * Lp + lbase + (lane & 7);
#pragma unroll
      for (int c = 0; c < BL / 8; ++c) {
        w.rpart[o + c * 8] = (double)racc[c];
        w.qpart[o + c * 8] = (double)qacc[c];
      }
    }
  }
  // sum z and S over the block's wavefronts (wavefront order), every
  // (period, contingency) of the block by one thread
  __syncthreads();
  for (int e = threadIdx.x; e < nt * 64; e += blockDim.x) {
    const int tt = e >> 6, kk = e & 63;
    double z = 0.0, s2 = 0.0;
    for (int q = 0; q < WL; ++q) {
      z += zsh[(tt * WL + q) * 64 + kk];
      s2 += ssh[(tt * WL + q) * 64 + kk];
    }
    const size_t o = ((size_t)lb * T + t0 + tt) * Kp + kb * 64 + kk;
    w.zpart[o] = z;
    w.spart[o] = s2;
  }
}

// Skip test of the period-split map-reduce (FP64 factors, every contingency
// scored).  For a half row h (branches 4h..4h+3 of an 8-branch tile) of one
// period, |P_tlk| = |F_tl + LODF_lk F_tk| <= |F_tl| + Lm Fm, where Lm is the
// largest |LODF| of the 4 branches over the wave's 64 contingencies (a
// per-grid table) and Fm the largest |F_tk| of the wave's lanes and periods.
// When |F_tl| (1 + 2^-40) + Lm Fm <= thr_tl (1 - 2^-40) holds in floating
// point for each of the 4 branches, no element of the half row passes the
// test |fl(P)| > thr_tl: the margins cover the rounding of the bound, of its
// comparison and of fl(P) (a few units of 2^-53), so the half row is skipped.
// NaN in F or thr makes the comparison false (the half row is tested).  Lane
// e of the wavefront decides half row (period tw + i, tile t0 + j) with
// j = e / (2 TCW), i = (e / 2) % TCW, h = e % 2; periods past the wave's last
// are skipped (their verdicts are dropped anyway).  Returns the ballot.
//
// FP32 arithmetic (FP32 or BF16 factors) tests fl(P^2 + qmax2) > s_ctg^2 in
// FP32 on FP32 roundings of F, qmax2 and s_ctg^2, and Lm is the largest
// stored factor.  There |fl(P)| <= (Lm Fm + |F|)(1 + u)^2 and the test's
// left side is at most ((Lm Fm + |F|)^2 + qmax2)(1 + u)^5 (u = 2^-24), so a
// half row is skipped when (Lm Fm + |F|)^2 (1 + 2^-18) + qmax2 (1 + 2^-18)
// <= s_ctg^2 (1 - 2^-18), computed in FP64, for each of its branches.
template <int TCW, bool F64>
__device__ __forceinline__ uint64_t ctg_cold_mask(const double* __restrict__ fh,
                                                  const double* __restrict__ lmaxh, int T,
                                                  int tw, int ntw, int tile0, int ntile, int kb,
                                                  int nkb, double fkm,
                                                  const double* __restrict__ q2,
                                                  const double* __restrict__ smax2, int Lp) {
  constexpr int CT = 32 / TCW;  // tiles per mask
  const int e = threadIdx.x & 63;
  const int j = e / (2 * TCW), i = (e >> 1) % TCW, h = e & 1;
  bool cold = false;
  if (j < CT && j < ntile) {
    if (i >= ntw) {
      cold = true;
    } else {
      const int tile = tile0 + j;
      const double* r = fh + ((size_t)tile * T + tw + i) * 16 + 8 * h;
      const double lm = lmaxh[(size_t)(2 * tile + h) * nkb + kb];
      double f[4], t[4];
#pragma unroll
      for (int g = 0; g < 4; ++g) {
        f[g] = r[g];
        t[g] = r[4 + g];
      }
      cold = true;
      if constexpr (F64) {
#pragma unroll
        for (int g = 0; g < 4; ++g) {
          const double s = fabs(f[g]) * (1.0 + 0x1p-40) - t[g] * (1.0 - 0x1p-40);
          cold = cold && fma(lm, fkm, s) <= 0.0;
        }
      } else {
        const int l = tile * 8 + 4 * h;
#pragma unroll
        for (int g = 0; g < 4; ++g) {
          const double b = fma(lm, fkm, fabs(f[g]));
          const double lhs = (b * b + q2[(size_t)(tw + i) * Lp + l + g]) * (1.0 + 0x1p-18);
          cold = cold && lhs <= smax2[l + g] * (1.0 - 0x1p-18);
        }
      }
    }
  }
  return __builtin_amdgcn_ballot_w64(cold);
}

// Period-split form of the same map-reduce.  The wavefronts of a block share
// one range of lt * 8 branches and split the periods: wavefront w owns the
// periods [t0 + w TCW, t0 + (w + 1) TCW), so z_tk and S_tk of its lanes need
// no sum over wavefronts and stay with the wavefront (in its own LDS slice)
// over the whole branch range, and with wl * TCW >= T every outage factor is
// read from memory once per evaluation (the block's wavefronts read the same
// tile, served by the L1 cache).  Per period the eight tests of a tile are
// combined before one branch; a period with a flagged lane takes the
// per-branch path of k_ctg_main.  A group of 64 z/S partials or of 8 R/Q
// partials is stored only when not all zero, with a byte flag per group
// (w.zflag, w.rflag) that the readers consult first.
//
// FP64: the test is |P| > thr_tl with thr_tl from k_forward, a radius a
// little below sqrt(s_ctg^2 - qmax2_tl), so that every element the exact
// test P^2 + qmax2 > s_ctg^2 accepts passes it (one FMA and one compare per
// element); the exact test is applied again on the per-branch path.  F_tl
// and thr_tl reach SGPRs by scalar loads issued one period ahead.  FP32
// arithmetic keeps the exact test with F and qmax2 moved to SGPRs by
// v_readlane from a per-tile lane load (lane e: period e / 8, branch e % 8).
//
// The batched launch (k_ctg_pm_b) runs the same block code for each work
// item; it is written out in both kernels rather than shared through an
// inlined function, which made the compiler spill about three times as many
// SGPRs and the map-reduce 1.5x slower.  Batched and single steps are checked
// to agree bit for bit.
template <int TCW, typename LT, bool SKIP>
__global__ __launch_bounds__(512) void k_ctg_pm(EvalArgs a, const LT* __restrict__ lodf) {
  typedef typename std::conditional<std::is_same<LT, double>::value, double, float>::type R;
  constexpr bool kF64 = std::is_same<R, double>::value;
  const DevProblem& p = a.p;
  const DevWork& w = a.w;
  const int lane = threadIdx.x & 63;
  const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int WL = blockDim.x >> 6;
  const int lb = blockIdx.x, kb = blockIdx.y;
  const int T = p.T, Lp = p.Lp, Kp = p.Kp;
  const int tw = (blockIdx.z * WL + wv) * TCW;  // first period of the wavefront
  const int ntw = min(TCW, T - tw);
  if (ntw <= 0) return;  // no barrier follows
  const int k = kb * 64 + lane;  // slot of the lane
  const int kc = a.act_k ? a.act_k[k] : k;
  // z and S of the wavefront's (period, lane) pairs live in its own slice
  // of LDS: only the per-branch path and the final store touch them
  extern __shared__ double dyn[];
  double* zsh = dyn + (size_t)wv * TCW * 128;
  double* ssh = zsh + TCW * 64;
  R fk[TCW];
#pragma unroll
  for (int i = 0; i < TCW; ++i) {
    fk[i] = i < ntw ? (R)w.Fk[(size_t)(tw + i) * Kp + kc] : R(0);
    zsh[i * 64 + lane] = 0.0;
    ssh[i * 64 + lane] = 0.0;
  }
  const cdouble* Sc = as_const(p.ctg_smax2);
  const cdouble* Mc = as_const(p.ctg_smax);
  const cdouble* Dc = as_const(p.dt);
  const cdouble* Qc = as_const(w.q2);
  const cdouble* FH = as_const(w.fh);
  const double beta = w.params[PB_BETA];
  const R eps = (R)w.params[PB_EPS];
  const R eps2 = eps * eps;
  const int ei = lane >> 3, eg = lane & 7;
  const int l0 = lb * a.lt * 8;
  const int l1 = min(Lp, l0 + a.lt * 8);
  // The factor loads of the tile loop go through a buffer resource over
  // the block's rows: the lane's fixed 32-bit byte offset (its slot k) plus
  // a uniform row offset that advances with the tile, so the loop needs no
  // per-lane address arithmetic.
  unsigned rowb = (unsigned)a.kst * (unsigned)sizeof(LT);  // bytes per factor row
  const __amdgpu_buffer_rsrc_t lrs =
      buf_rsrc(lodf + (size_t)l0 * a.kst, (unsigned)(l1 - l0) * rowb);
  const unsigned koff = (unsigned)k * (unsigned)sizeof(LT);
  // R/Q flags of the lane's period (lane e < ntw: period tw + e), bit i for
  // tile i of the block, stored after the loop
  uint64_t fbits = 0;
  // SKIP: half rows proved free of overloads are skipped (ctg_cold_mask),
  // with FP64 factors, every contingency scored and a block of at most
  // 64 / TCW tiles (two masks of 32 / TCW tiles cover them; the host
  // launches the SKIP form only then, and a block outside it tests
  // everything); the F and thr of a tested half row are loaded when it is
  // reached.  Otherwise they are prefetched one half row ahead.
  // Bit ((ti mod CT) TCW + i) 2 + h of mask ti / CT (CT = 32 / TCW): half
  // row h of period tw + i of tile ti skipped.
  uint64_t coldm = 0, coldm1 = 0;
  if constexpr (SKIP) {
    constexpr int CT = 32 / TCW;  // tiles per mask
    const int ntile = (l1 - l0) >> 3;
    if (p.lmaxh != nullptr && a.act_k == nullptr && ntile <= 2 * CT) {
      double fkm = 0.0;  // largest |F_tk| of the wave's lanes and periods
#pragma unroll
      for (int i = 0; i < TCW; ++i) fkm = fmax(fkm, fabs(fk[i]));
      fkm = wave_max(fkm);
      coldm = ctg_cold_mask<TCW, kF64>(w.fh, p.lmaxh, T, tw, ntw, l0 >> 3, ntile, kb, Kp >> 6,
                                       fkm, w.q2, p.ctg_smax2, Lp);
      if (ntile > CT)
        coldm1 = ctg_cold_mask<TCW, kF64>(w.fh, p.lmaxh, T, tw, ntw, (l0 >> 3) + CT, ntile - CT,
                                          kb, Kp >> 6, fkm, w.q2, p.ctg_smax2, Lp);
    }
  }
  // F and thr of the next half row (four branches of one period) to be
  // tested, from the branch-tiled copy, so that every prefetch is a fixed
  // offset from the tile's row of period tw
  double Fn[4], Hn[4];
  if constexpr (kF64 && !SKIP) {
    const cdouble* r = FH + ((size_t)(l0 >> 3) * T + tw) * 16;
#pragma unroll
    for (int g = 0; g < 4; ++g) {
      Fn[g] = r[g];
      Hn[g] = r[4 + g];
    }
  }
  const uint32_t live = (1u << ntw) - 1u;  // the wave's periods among the TCW tested
  unsigned lso = 0;  // uniform offset of the tile's factor rows
  int ti = 0;        // tile index in the block
  // rows of the branch-tiled copy: period tw of the tile, of the next tile
  const cdouble* cur = FH + ((size_t)(l0 >> 3) * T + tw) * 16;
  unsigned fstep = (unsigned)T * 16u;
  for (int lbase = l0; lbase < l1; lbase += 8, lso += 8 * rowb, ++ti, cur += fstep) {
    // the strides are taken as changing in every tile, so that nothing
    // derived from them is hoisted out of the loop (such values took SGPRs
    // that were then spilled, and reloading them costs vector instructions)
    asm volatile("" : "+s"(rowb), "+s"(fstep));
    const cdouble* nxt = cur + fstep;
    // the tile's half rows that are tested (bit 2 i + h); a tile without
    // any is passed over, and only the factor rows of tested halves are loaded
    const uint32_t need =
        ~(uint32_t)((ti < 32 / TCW ? coldm : coldm1) >> ((ti % (32 / TCW)) * TCW * 2)) &
        ((1u << (2 * TCW)) - 1u);
    if (need == 0) continue;
    R lod[8];
#pragma unroll
    for (int j = 0; j < 8; ++j)
      lod[j] = (need & (j < 4 ? 0x5555u : 0xAAAAu)) ? lodf_buf(lrs, lodf, koff, lso + j * rowb) : R(0);
    R fv = R(0), qv = R(0), smx2[8];
    if constexpr (!kF64) {
      if (ei < ntw) {
        const size_t e = (size_t)(tw + ei) * Lp + lbase + eg;
        fv = (R)w.F[e];
        qv = (R)w.q2[e];
      }
#pragma unroll
      for (int j = 0; j < 8; ++j) smx2[j] = (R)Sc[lbase + j];
    }
    // The test of every (period, branch, lane) of the tile, without a
    // branch: all TCW periods are tested (the rows past the wave's last
    // period are spare rows of the array, and their verdicts are dropped
    // with the mask), and each period's verdict is one bit of hotm.
    uint32_t hotm = 0;
#pragma unroll
    for (int i = 0; i < TCW; ++i) {
      uint64_t hot = 0;
      if constexpr (SKIP && kF64) {
#pragma unroll
        for (int h = 0; h < 2; ++h) {
          if ((need >> (2 * i + h)) & 1u) {
            double Fr[4], Hr[4];
            const cdouble* q = cur + 16 * i + 8 * h;
#pragma unroll
            for (int g = 0; g < 4; ++g) {
              Fr[g] = q[g];
              Hr[g] = q[4 + g];
            }
#pragma unroll
            for (int g = 0; g < 4; ++g) {
              const double P = fma_uniform_c(lod[4 * h + g], fk[i], Fr[g]);
              hot |= __builtin_amdgcn_ballot_w64(fabs(P) > Hr[g]);
            }
          }
        }
      } else if constexpr (kF64) {
#pragma unroll
        for (int h = 0; h < 2; ++h) {
          double Fr[4], Hr[4];
#pragma unroll
          for (int g = 0; g < 4; ++g) {
            Fr[g] = Fn[g];
            Hr[g] = Hn[g];
          }
          // prefetch: the other half of this period's row, else the next
          // period of this tile, else period tw of the next tile (rows past
          // the tile or the last tile are spare rows)
          const cdouble* q = h == 0 ? cur + 16 * i + 8 : (i + 1 < TCW) ? cur + 16 * (i + 1) : nxt;
#pragma unroll
          for (int g = 0; g < 4; ++g) {
            Fn[g] = q[g];
            Hn[g] = q[4 + g];
          }
#pragma unroll
          for (int g = 0; g < 4; ++g) {
            const double P = fma_uniform_c(lod[4 * h + g], fk[i], Fr[g]);
            hot |= __builtin_amdgcn_ballot_w64(fabs(P) > Hr[g]);
          }
        }
      } else {
        // FP32 arithmetic; with SKIP only the half rows that are tested
#pragma unroll
        for (int h = 0; h < 2; ++h) {
          if ((need >> (2 * i + h)) & 1u) {
#pragma unroll
            for (int gg = 0; gg < 4; ++gg) {
              const int g = 4 * h + gg;
              const R Fr = readlane_any(fv, i * 8 + g);
              const R P = fma_uniform_c(lod[g], fk[i], Fr);
              const R s2 = fma_uniform_c(P, P, readlane_any(qv, i * 8 + g));
              hot |= __builtin_amdgcn_ballot_w64(s2 > smx2[g]);
            }
          }
        }
      }
      hotm |= (hot != 0 ? 1u : 0u) << i;
    }
    hotm &= live;
    // a wave with fewer than TCW periods prefetched a spare row for the
    // next tile: load its first period's row again
    if constexpr (kF64 && !SKIP) {
      if (ntw < TCW) {
#pragma unroll
        for (int g = 0; g < 4; ++g) {
          Fn[g] = nxt[g];
          Hn[g] = nxt[4 + g];
        }
      }
    }
    if (hotm) {
      // R and Q of (period tw + e / 8, branch lbase + e % 8) gather in lane e
      R racc = R(0), qacc = R(0);
      // the overloaded periods of the tile: the per-branch path, with F,
      // qmax2 and the ratings loaded again
#pragma unroll
      for (int i = 0; i < TCW; ++i) {
        if ((hotm >> i) & 1u) {
          const R kt = (R)(Dc[tw + i] * p.c_s * beta);
          R Fr[8], Qr[8], Sr[8];
#pragma unroll
          for (int g = 0; g < 8; ++g) {
            if constexpr (kF64) {
              Fr[g] = cur[16 * i + fh_col_f(g)];
              Qr[g] = Qc[(size_t)(tw + i) * Lp + lbase + g];
              Sr[g] = Sc[lbase + g];
            } else {
              Fr[g] = readlane_any(fv, i * 8 + g);
              Qr[g] = readlane_any(qv, i * 8 + g);
              Sr[g] = smx2[g];
            }
          }
          R zt = R(0), st = R(0);
#pragma unroll
          for (int g = 0; g < 8; ++g) {
            // a skipped half row holds no overload (and its factors were
            // not loaded)
            if (((need >> (2 * i + (g >> 2))) & 1u) == 0) continue;
            // the flow formed again (the same fused operation, so the same
            // value as in the test)
            const R P = fma_uniform_c(lod[g], fk[i], Fr[g]);
            const R s2 = fma_uniform_c(P, P, Qr[g]);
            if (__builtin_amdgcn_ballot_w64(s2 > Sr[g])) {
              R dP = R(0), dq = R(0);
              if (s2 > Sr[g]) {
                zt += ctg_overload(P, s2, (R)Mc[lbase + g], eps, eps2, kt, dP, dq);
                st = fma(lod[g], dP, st);
              }
              const R r = pair_sum(dP, dq);  // lane 0: sum of dP, lane 32: of dq
              racc = writelane_set(racc, readlane_any(r, 0), i * 8 + g);
              qacc = writelane_set(qacc, readlane_any(r, 32), i * 8 + g);
            }
          }
          zsh[i * 64 + lane] += (double)zt;
          ssh[i * 64 + lane] += (double)st;
        }
      }
      // per (period, 8 branches): stored only when not all zero, and flagged
      const uint64_t b = __builtin_amdgcn_ballot_w64(racc != R(0) || qacc != R(0));
      if (lane < ntw && ((b >> (8 * lane)) & 0xFF) != 0) fbits |= (uint64_t)1 << ti;
      if (b != 0 && lane < ntw * 8 && ((b >> (lane & ~7)) & 0xFF) != 0) {
        const size_t o = ((size_t)kb * T + tw + ei) * Lp + lbase + eg;
        w.rpart[o] = (double)racc;
        w.qpart[o] = (double)qacc;
      }
    }
  }
  if (lane < ntw) {
    uint8_t* f = w.rflag + ((size_t)(tw + lane) * (Lp / 8) + (l0 >> 3)) * a.rfs + kb;
    for (int i = 0; i < ti; ++i) f[(size_t)i * a.rfs] = (uint8_t)((fbits >> i) & 1u);
  }
#pragma unroll
  for (int i = 0; i < TCW; ++i) {
    if (i < ntw) {
      // stored only when not all zero, and flagged
      const double z = zsh[i * 64 + lane], s2 = ssh[i * 64 + lane];
      const bool nz = __builtin_amdgcn_ballot_w64(z != 0.0 || s2 != 0.0) != 0;
      if (lane == 0) w.zflag[((size_t)(tw + i) * a.zfk + kb) * a.zfs + lb] = (uint8_t)nz;
      if (nz) {
        const size_t o = ((size_t)lb * T + tw + i) * Kp + k;
        w.zpart[o] = z;
        w.spart[o] = s2;
      }
    }
  }
}


// ---------------------------------------------------------------------------
// K4: per-(t, k) penalties z_tk (the l-block partials plus the floor
// (L-1) eps), the mean outage-correction derivative, and per 64-contingency
// chunk the worst penalty (smallest index on ties) and the sum.  One 64-thread
// block per (chunk, t); all partial loads of a lane are in flight together.

// flagged l-block partials loaded together by the sparse reduction
constexpr int kZredBatch = 32;

template <bool SPARSE>
__device__ __forceinline__ void ctg_zred_body(const EvalArgs& a, int kc, int t) {
  const DevProblem& p = a.p;
  const DevWork& w = a.w;
  const int lane = threadIdx.x;
  const int T = p.T, L = p.L, K = p.K, Kp = p.Kp;
  const double eps = w.params[PB_EPS], beta = w.params[PB_BETA];
  const double kt = p.dt[t] * p.c_s * beta;
  const int s = kc * 64 + lane;  // slot
  const size_t o = (size_t)t * Kp + s;
  const size_t stride = (size_t)T * Kp;
  // the l-block partials in l-block order; after the period-split
  // map-reduce only the flagged ones (the others are all zero), up to 32 of
  // each in flight
  double zs = 0.0, ss = 0.0;
  if constexpr (!SPARSE) {
    zs = strided_sum<16>(w.zpart + o, a.nLb, stride);
    ss = strided_sum<16>(w.spart + o, a.nLb, stride);
  }
  const uint8_t* zf = w.zflag + ((size_t)t * a.zfk + kc) * a.zfs;
  for (int b0 = 0; SPARSE && b0 < a.nLb; b0 += 64) {
    uint64_t m = __builtin_amdgcn_ballot_w64(b0 + lane < a.nLb && zf[b0 + lane] != 0);
    while (m) {
      int idx[kZredBatch];
#pragma unroll
      for (int u = 0; u < kZredBatch; ++u) {
        idx[u] = m ? b0 + __builtin_ctzll(m) : -1;
        m &= m - 1;
      }
      double vz[kZredBatch], vs[kZredBatch];
#pragma unroll
      for (int u = 0; u < kZredBatch; ++u) {
        vz[u] = idx[u] >= 0 ? w.zpart[o + (size_t)idx[u] * stride] : 0.0;
        vs[u] = idx[u] >= 0 ? w.spart[o + (size_t)idx[u] * stride] : 0.0;
      }
#pragma unroll
      for (int u = 0; u < kZredBatch; ++u) {
        zs += vz[u];
        ss += vs[u];
      }
    }
  }
  double z = -DBL_MAX, zsum = 0.0;
  int idx = INT_MAX;
  if (s < a.na) {
    const int k = a.act_k ? a.act_k[s] : s;
    z = kt * ((double)(L - 1) * eps + zs);
    w.zval[(size_t)t * Kp + k] = z;
    w.smean[o] = p.ctg_sum ? ss : ss / (double)K;
    idx = k;
    zsum = z;
  }
  const double tot = wave_sum(zsum);
  wave_argmax(z, idx);
  if (lane == 0) {
    const size_t c = (size_t)t * a.nKc + kc;
    w.zmaxp[c] = z;
    w.zargp[c] = (double)idx;
    w.zsump[c] = tot;
  }
}

template <bool SPARSE>
__global__ __launch_bounds__(64) void k_ctg_zred(EvalArgs a) {
  ctg_zred_body<SPARSE>(a, blockIdx.x, blockIdx.y);
}

// ---------------------------------------------------------------------------
// K5: per-(t, l) adjoint of the flows: dL/dF_tl (transposed, the A operand of
// the adjoint product) and dL/dqmax2_tl, with weight 1/K for every
// contingency plus 1 for the worst of the period (Table 1's two contingency
// rows).  The worst contingency's own column is re-evaluated here; its
// outage-correction term S* = sum_l LODF_lk* dP_tlk* belongs to dL/dF at the
// outaged branch and is applied in k_final as a rank-1 term (per-chunk sums).

template <bool SPARSE>
__device__ void ctg_assemble(const EvalArgs& a, int t, int lc, double* red) {
  const DevProblem& p = a.p;
  const DevWork& w = a.w;
  const int tid = threadIdx.x;
  const int T = p.T, L = p.L, K = p.K, Lp = p.Lp, Kp = p.Kp, Tp = p.Tp;
  const double eps = w.params[PB_EPS], beta = w.params[PB_BETA];
  const double kt = p.dt[t] * p.c_s * beta;
  const int l = lc * kBlock + tid;
  const bool hasl = l < L;
  // independent loads first
  double r = 0.0, q = 0.0, Fl = 0.0, q2l = 0.0, sm2 = 0.0, sm = 0.0;
  int kk = -1;
  const size_t o = (size_t)t * Lp + l;
  if (hasl) {
    Fl = w.F[o];
    q2l = w.q2[o];
    sm2 = p.ctg_smax2[l];
    sm = p.ctg_smax[l];
    kk = p.kof[l];
  }
  double sacc[1] = {0.0};
  if (K > 0) {
    // per-chunk worst penalties and sums: chunk c0 + u in lane u (vector
    // loads, issued first), combined by wavefront reductions (the argmax is
    // a total order, the sum has a fixed order); then the k-block partials
    // of R and Q in k-block order, 16 of each in flight together.  Without
    // contingencies the partials were never written.
    const int lane = tid & 63;
    double zmax = -DBL_MAX, zsum = 0.0;
    int kstar = INT_MAX;
    const size_t ob = (size_t)t * a.nKc;
    double cz = -DBL_MAX, cs = 0.0;
    int ci = INT_MAX;
    if (lane < a.nKc) {
      cz = w.zmaxp[ob + lane];
      ci = (int)w.zargp[ob + lane];
      cs = w.zsump[ob + lane];
    }
    // after the period-split map-reduce only the flagged k-block partials
    // were stored (the others are zero): the flags of the branch's group of
    // 8 first, 16 k-blocks per load
    const size_t st = (size_t)T * Lp;
    const uint8_t* rf = w.rflag + ((size_t)t * (Lp / 8) + l / 8) * a.rfs;
    for (int c0 = 0; c0 < a.nKb; c0 += 16) {
      uint4 f4 = make_uint4(~0u, ~0u, ~0u, ~0u);
      if constexpr (SPARSE)
        f4 = hasl ? *reinterpret_cast<const uint4*>(rf + c0) : make_uint4(0u, 0u, 0u, 0u);
      const uint32_t fw[4] = {f4.x, f4.y, f4.z, f4.w};
      double vr[16], vq[16];
#pragma unroll
      for (int u = 0; u < 16; ++u) {
        const bool ib = hasl && c0 + u < a.nKb && ((fw[u >> 2] >> (8 * (u & 3))) & 0xFFu) != 0;
        vr[u] = ib ? w.rpart[o + (size_t)(c0 + u) * st] : 0.0;
        vq[u] = ib ? w.qpart[o + (size_t)(c0 + u) * st] : 0.0;
      }
#pragma unroll
      for (int u = 0; u < 16; ++u) {
        r += vr[u];
        q += vq[u];
      }
    }
    for (int c0 = 0; c0 < a.nKc; c0 += 64) {
      if (c0 > 0) {
        const int c = c0 + lane;
        cz = c < a.nKc ? w.zmaxp[ob + c] : -DBL_MAX;
        ci = c < a.nKc ? (int)w.zargp[ob + c] : INT_MAX;
        cs = c < a.nKc ? w.zsump[ob + c] : 0.0;
      }
      wave_argmax(cz, ci);
      const double ssum = wave_sum(cs);
      if (better(cz, ci, zmax, kstar)) { zmax = cz; kstar = ci; }
      zsum += ssum;
    }
    if (!(kstar >= 0 && kstar < K)) kstar = 0;  // NaN penalties: keep every index in range
    // weight of every scored contingency: 1/K for the mean (plus 1 for the
    // period's worst), or 1 for the plain sum
    const double invK = 1.0 / (double)K;
    const double wk = p.ctg_sum ? 1.0 : invK;
    if (hasl) {
      r *= wk;
      q *= wk;
      // the outaged branch's own factor is NaN: it never tests overloaded
      const double lo = lodf_value(p, l, kstar);
      const double P = fma(lo, w.Fk[(size_t)t * Kp + kstar], Fl);
      const double s2 = fma(P, P, q2l);
      if (!p.ctg_sum && s2 > sm2) {
        double dP, dq;
        ctg_overload(P, s2, sm, eps, eps * eps, kt, dP, dq);
        r += dP;
        q += dq;
        sacc[0] = lo * dP;
      }
      if (kk >= 0) {
        const int sl = a.act_slot ? a.act_slot[kk] : kk;
        if (sl >= 0) r += w.smean[(size_t)t * Kp + sl];
      }
    }
    if (lc == 0 && tid == 0) {
      w.tpart[a.toff.cmax + t] = p.ctg_sum ? 0.0 : zmax;
      // contingencies not scored this step take their no-overload penalty
      const double rest = (double)(K - a.na) * (kt * ((double)(L - 1) * eps));
      w.tpart[a.toff.cmean + t] = (zsum + rest) * wk;
      w.kstar[t] = (double)kstar;
    }
  } else if (lc == 0 && tid == 0) {
    w.tpart[a.toff.cmax + t] = 0.0;
    w.tpart[a.toff.cmean + t] = 0.0;
    w.kstar[t] = 0.0;
  }
  if (l < Lp) {
    w.gfT[(size_t)l * Tp + t] = hasl ? r : 0.0;
    w.qtot[(size_t)t * Lp + l] = hasl ? q : 0.0;
  }
  block_sum<1>(sacc, red);
  if (tid == 0) w.smaxp[(size_t)t * a.nLc + lc] = sacc[0];
}

// Blocks [0, T nsl): the device terms of one period and one slice of 256
// generators each (period_block, with the step's parameters as the forward
// kernel resolved them; nsl slices per period); then nLc T blocks of flow
// adjoints of (period, 256-branch chunk); then the nb_bus power-balance
// blocks, which only need the forward flows.
template <bool SPARSE>
__device__ __forceinline__ void ctg_asm_body(const EvalArgs& a, int b, int nblocks,
                                             double* smem) {
  const int T = a.p.T, nasm = a.nLc * T;
  const int nsl = (a.p.G + kBlock - 1) / kBlock, nper = T * nsl;
  // scheduled steps: the next step's schedule row (the counter is advanced
  // by k_final, after this kernel), clamped to the table; a new table comes
  // with k_set_step, which copies its own row
  if (a.mode.schedule && b == nblocks - 1 && threadIdx.x < kSchedStride) {
    const int64_t s1 = min(a.w.step[0] + 1, (int64_t)kSchedCap - 1);
    a.w.snext[threadIdx.x] = a.w.sched[s1 * kSchedStride + threadIdx.x];
  }
  if (b < nper) {
    StepParams sp{};
    sp.eps = a.w.params[PB_EPS];
    sp.beta = a.w.params[PB_BETA];
    sp.rho_s = a.w.params[PB_RHO];
    period_block(a, sp, b / nsl, b % nsl, smem);
  } else if (b < nper + nasm) {
    // XCD-grouped: the blocks of consecutive periods store the transposed
    // flow adjoints gfT[l][t] of the same branches through one L2
    const int g = xcd_group(b - nper, nasm);
    ctg_assemble<SPARSE>(a, g / a.nLc, g % a.nLc, smem);
  } else {
    bus_balance(a, b - nper - nasm, smem);
  }
}

template <bool SPARSE>
__global__ __launch_bounds__(kBlock) void k_ctg_asm(EvalArgs a) {
  __shared__ double smem[2 * kSegChunk + 16];
  ctg_asm_body<SPARSE>(a, blockIdx.x, gridDim.x, smem);
}

// ---------------------------------------------------------------------------
// K6: adjoint DC product + branch reverse

__device__ void branch_reverse(const EvalArgs& a, int blk) {
  const DevProblem& p = a.p;
  const DevWork& w = a.w;
  const int T = p.T, L = p.L, N = p.N;
  const int idx = blk * kBlock + threadIdx.x;
  if (idx >= T * L) return;
  const int t = idx / L, l = idx - t * L;
  const size_t TL = (size_t)T * L, e = (size_t)t * L + l;
  const double cs = w.bco[0 * TL + e], sn = w.bco[1 * TL + e];
  const int f = p.br_from[l], o = p.br_to[l];
  const double vf = a.x[(size_t)t * N + f], vt = a.x[(size_t)t * N + o];
  const double Qc = w.qtot[(size_t)t * p.Lp + l];
  const double lpf = w.lamp[(size_t)t * N + f] + w.bco[2 * TL + e];
  const double lqf = w.lamq[(size_t)t * N + f] + w.bco[3 * TL + e] + Qc * w.bco[7 * TL + e];
  const double lpt = w.lamp[(size_t)t * N + o] + w.bco[4 * TL + e];
  const double lqt = w.lamq[(size_t)t * N + o] + w.bco[5 * TL + e] + Qc * w.bco[8 * TL + e];
  const double g = p.br_g[l], b = p.br_b[l], bh = p.br_bh[l];
  const double A = -g * cs - b * sn;   // p_fr cross coefficient
  const double Bq = b * cs - g * sn;   // q_fr
  const double Ct = -g * cs + b * sn;  // p_to
  const double Dq = b * cs + g * sn;   // q_to
  const double gvf = lpf * (2.0 * g * vf + vt * A) + lqf * (-2.0 * (b + bh) * vf + vt * Bq) +
                     lpt * (vt * Ct) + lqt * (vt * Dq);
  const double gvt = lpf * (vf * A) + lqf * (vf * Bq) + lpt * (2.0 * g * vt + vf * Ct) +
                     lqt * (-2.0 * (b + bh) * vt + vf * Dq);
  const double vv = vf * vt;
  const double gd = w.bco[6 * TL + e] + lpf * vv * (g * sn - b * cs) +
                    lqf * vv * (-b * sn - g * cs) + lpt * vv * (g * sn + b * cs) +
                    lqt * vv * (-b * sn + g * cs);
  const size_t ep = (size_t)t * p.twoL;
  w.epGV[ep + p.slot_fr[l]] = gvf;
  w.epGT[ep + p.slot_fr[l]] = gd;
  w.epGV[ep + p.slot_to[l]] = gvt;
  w.epGT[ep + p.slot_to[l]] = -gd;
}

// Blocks [0, nslab * nsplit): the DC part of dL/dp, one 16-generator slab and
// one slice of the branch dimension each (partials summed in k_final); then
// nb_br branch-reverse blocks; then the worst outage's ISF rows.
__device__ __forceinline__ void adjoint_body(const EvalArgs& a, int bx, double* smem) {
  const DevProblem& p = a.p;
  const int nslab = p.G16 / 16;
  if (bx < nslab * a.nsplit) {
    // XCD-grouped: the slabs of one slice, which read the same rows of the
    // flow adjoints, mostly share an L2
    const int g = xcd_group(bx, nslab * a.nsplit);
    const int slab = g % nslab, sp = g / nslab;
    const int n0 = slab * 16;
    const int steps = p.Lp / 4;
    const int per = (steps + a.nsplit - 1) / a.nsplit;
    const int k0 = min(steps, sp * per) * 4, k1 = min(steps, (sp + 1) * per) * 4;
    const int T = p.T, Tp = p.Tp, G16 = p.G16;
    double* out = a.w.gpdc + (size_t)sp * T * G16;
    const double* gfT = a.w.gfT;
    // rows past T of gfT are never written: they enter as zeros
    auto aload = [=](int k, int row) -> double {
      return row < T ? gfT[(size_t)k * Tp + row] : 0.0;
    };
    auto epi = [=](int row, int col, double v) {
      if (row < T) out[(size_t)row * G16 + col] = v;
    };
    mfma_slab_dispatch<8>(p.Tp / 16, aload, p.isf_ga, G16, k0, k1, n0, smem, epi);
    return;
  }
  const int b = bx - nslab * a.nsplit;
  if (b < a.nb_br) {
    branch_reverse(a, xcd_group(b, a.nb_br));
    return;
  }
  // the worst outage's ISF row of each period (generator columns), for the
  // rank-1 outage-correction term that k_final adds to dL/dp
  const int idx = (b - a.nb_br) * kBlock + threadIdx.x;
  if (idx < p.T * p.G16) {
    const int t = idx / p.G16, j = idx - t * p.G16;
    const int bks = p.brk[(int)a.w.kstar[t]];
    a.w.isfk[idx] = p.isf_ga[(size_t)bks * p.G16 + j];
  }
}

__global__ __launch_bounds__(kBlock) void k_adjoint(EvalArgs a) {
  __shared__ double smem[kSlabLds];
  adjoint_body(a, blockIdx.x, smem);
}

// ---------------------------------------------------------------------------
// K7: bus reduce, generator assembly, gradient or fused Adam, terms

struct AdamCtx {
  double b1, b2, eps, bc1, bc2;
  int eps_num;
};

// x, m, v of one variable.  The loads of every variable a thread updates are
// issued before its first store: x, m and v may alias as far as the compiler
// knows, so a load after a store would wait for it.
struct AdamVar {
  double x, m, v;
};
__device__ __forceinline__ AdamVar adam_load(const double* x, const double* m, const double* v,
                                             size_t e) {
  return AdamVar{x[e], m[e], v[e]};
}
__device__ __forceinline__ void adam_store(double* x, double* m, double* v, size_t e,
                                           const AdamVar& s, double g, double lr, double lo,
                                           double hi, const AdamCtx& c) {
  const double mm = c.b1 * s.m + (1.0 - c.b1) * g;
  const double vv = c.b2 * s.v + (1.0 - c.b2) * g * g;
  const double mh = mm / c.bc1;
  const double vh = vv / c.bc2;
  const double num = c.eps_num ? mh + c.eps : mh;
  double xn = s.x - lr * num / (sqrt(vh) + c.eps);
  xn = fmin(fmax(xn, lo), hi);
  m[e] = mm;
  v[e] = vv;
  x[e] = xn;
}
__device__ __forceinline__ void adam_entry(double* x, double* m, double* v, size_t e, double g,
                                           double lr, double lo, double hi, const AdamCtx& c) {
  adam_store(x, m, v, e, adam_load(x, m, v, e), g, lr, lo, hi, c);
}

__device__ __forceinline__ void final_body(const EvalArgs& a, int bx, double* smem) {
  const DevProblem& p = a.p;
  const DevWork& w = a.w;
  const int tid = threadIdx.x;
  const int T = p.T, N = p.N, G = p.G;
  AdamCtx ac;
  double alpha[QG_NCLASS];
  if (a.fuse_adam) {
    ac.b1 = a.mode.adam_b1; ac.b2 = a.mode.adam_b2; ac.eps = a.mode.adam_eps;
    ac.eps_num = a.mode.eps_in_num;
    ac.bc1 = w.params[PB_BC1]; ac.bc2 = w.params[PB_BC2];
    for (int c = 0; c < QG_NCLASS; ++c) alpha[c] = w.params[PB_ALPHA + c];
  }
  double* xm = const_cast<double*>(a.x);
  if (bx < a.nb_bus) {
    const int t = bx / a.bus_chunks;
    const int c = bx - t * a.bus_chunks;
    const int i0 = c * kBlock;
    const int nbus = min(kBlock, N - i0);
    const double* src[2] = {w.epGV + (size_t)t * p.twoL, w.epGT + (size_t)t * p.twoL};
    // the bus's Adam state, loaded while the endpoint sums are formed
    const int i = i0 + tid;
    const size_t ev = (size_t)t * N + i, et = (size_t)T * N + ev;
    const bool upd = a.fuse_adam && tid < nbus;
    const AdamVar sv = upd ? adam_load(xm, a.m, a.v, ev) : AdamVar{0.0, 0.0, 0.0};
    const AdamVar st = upd ? adam_load(xm, a.m, a.v, et) : AdamVar{0.0, 0.0, 0.0};
    const double vlo = upd ? p.vmin[i] : 0.0, vhi = upd ? p.vmax[i] : 0.0;
    double gsum[2];
    bus_segsum<2>(src, p.bptr, i0, nbus, smem, gsum);
    if (tid < nbus) {
      if (a.fuse_adam) {
        adam_store(xm, a.m, a.v, ev, sv, gsum[0], alpha[QG_C_V], vlo, vhi, ac);
        adam_store(xm, a.m, a.v, et, st, gsum[1], alpha[QG_C_TH], -DBL_MAX, DBL_MAX, ac);
      } else if (a.grad) {
        a.grad[ev] = gsum[0];
        a.grad[et] = gsum[1];
      }
    }
    return;
  }
  const int gb = bx - a.nb_bus;
  if (gb < a.nb_gen) {
    // dL/dp: device partials, balance multiplier, and the DC part: the MFMA
    // split partials plus the worst contingency's rank-1 term
    // S*_t (ISF[br(k*)][bus(j)] - rowsum/N).
    const int idx = gb * kBlock + tid;
    if (idx >= T * G) return;
    const int t = idx / G, j = idx - t * G;
    const size_t TG = (size_t)T * G;
    const size_t base = 2 * (size_t)T * N;
    const size_t e = (size_t)t * G + j;
    // every single load first (the Adam state of the four variables too),
    // then the partial sums
    AdamVar s4[4];
    if (a.fuse_adam)
#pragma unroll
      for (int q = 0; q < 4; ++q) s4[q] = adam_load(xm, a.m, a.v, base + q * TG + e);
    const double gd0 = w.gdev[e], gd1 = w.gdev[TG + e], gd2 = w.gdev[2 * TG + e];
    const double gd3 = w.gdev[3 * TG + e];
    const double lg = w.lamg[e], lqg = w.lamqg[e], drs = w.drs[t];
    const double isk = w.isfk[(size_t)t * p.G16 + j];
    const double pmax = p.pmax[j], qmin = p.qmin[j], qmax = p.qmax[j], rmax = p.rmax[j];
    const double smax = strided_sum<16>(w.smaxp + (size_t)t * a.nLc, a.nLc, 1);
    double dc = smax * isk;
    dc += strided_sum<16>(w.gpdc + (size_t)t * p.G16 + j, a.nsplit, (size_t)T * p.G16);
    const double gp = gd0 - lg + dc;
    const double gq = gd1 - lqg;
    const double gr = gd2 - drs;
    const double gu = gd3;
    if (a.fuse_adam) {
      adam_store(xm, a.m, a.v, base + e, s4[0], gp, alpha[QG_C_P], 0.0, pmax, ac);
      adam_store(xm, a.m, a.v, base + TG + e, s4[1], gq, alpha[QG_C_Q], qmin, qmax, ac);
      adam_store(xm, a.m, a.v, base + 2 * TG + e, s4[2], gr, alpha[QG_C_R], 0.0, rmax, ac);
      adam_store(xm, a.m, a.v, base + 3 * TG + e, s4[3], gu, alpha[QG_C_U], 0.0, 1.0, ac);
    } else if (a.grad) {
      a.grad[base + e] = gp;
      a.grad[base + TG + e] = gq;
      a.grad[base + 2 * TG + e] = gr;
      a.grad[base + 3 * TG + e] = gu;
    }
    return;
  }
  // terms: deterministic sums of the partials (one pass, so that all of a
  // thread's loads are in flight together)
  const TermOffsets& to = a.toff;
  double v[8] = {0, 0, 0, 0, 0, 0, 0, 0};
  const int ndev = T * ((G + kBlock - 1) / kBlock);  // device-term slices
  const int nq = max(max(a.nb_br, ndev), a.nb_bus);
  for (int q = tid; q < nq; q += kBlock) {
    const bool ib = q < a.nb_br, it = q < T, iu = q < a.nb_bus, id = q < ndev;
    const double br = ib ? w.tpart[to.br + q] : 0.0, an = ib ? w.tpart[to.ang + q] : 0.0;
    const double dv = id ? w.tpart[to.dev + q] : 0.0, pn = id ? w.tpart[to.pen + q] : 0.0;
    const double rs = it ? w.tpart[to.rsv + q] : 0.0, cx = it ? w.tpart[to.cmax + q] : 0.0;
    const double cm = it ? w.tpart[to.cmean + q] : 0.0, bl = iu ? w.tpart[to.bal + q] : 0.0;
    v[0] += dv; v[1] += bl; v[2] += br; v[3] += an;
    v[4] += pn; v[5] += rs; v[6] += cx; v[7] += cm;
  }
  block_sum<8>(v, smem);
  if (tid == 0) {
    double out[QG_NTERMS];
    for (int q = 0; q < 8; ++q) out[q] = v[q];
    out[QG_T_LOADVAL] = p.vload;
    out[QG_T_TOTAL] = v[0] + v[1] + v[2] + v[3] + v[4] + v[5] + v[6] + v[7] - p.vload;
    for (int q = 0; q < QG_NTERMS; ++q) {
      w.terms[q] = out[q];
      if (a.terms_out) a.terms_out[q] = out[q];
    }
    if (a.mode.schedule) w.step[0] = w.step[0] + 1;
  }
}

__global__ __launch_bounds__(kBlock) void k_final(EvalArgs a) {
  __shared__ double smem[2 * kSegChunk + 8 * kBlock];
  final_body(a, blockIdx.x, smem);
}

// ---------------------------------------------------------------------------
// standalone Adam (qg_adam_step) and helpers

__global__ __launch_bounds__(kBlock) void k_adam(DevProblem p, double* x, double* m, double* v,
                                                 const double* g, double lr0, double lr1,
                                                 double lr2, double lr3, double lr4, double lr5,
                                                 AdamCtx ac) {
  const size_t TN = (size_t)p.T * p.N, TG = (size_t)p.T * p.G;
  const size_t n = 2 * TN + 4 * TG;
  const size_t e = (size_t)blockIdx.x * kBlock + threadIdx.x;
  if (e >= n) return;
  double lr, lo, hi;
  if (e < TN) {
    const int i = (int)(e % p.N);
    lr = lr0; lo = p.vmin[i]; hi = p.vmax[i];
  } else if (e < 2 * TN) {
    lr = lr1; lo = -DBL_MAX; hi = DBL_MAX;
  } else {
    const size_t r = e - 2 * TN;
    const int cls = (int)(r / TG);
    const int j = (int)((r - cls * TG) % p.G);
    switch (cls) {
      case 0: lr = lr2; lo = 0.0; hi = p.pmax[j]; break;
      case 1: lr = lr3; lo = p.qmin[j]; hi = p.qmax[j]; break;
      case 2: lr = lr4; lo = 0.0; hi = p.rmax[j]; break;
      default: lr = lr5; lo = 0.0; hi = 1.0; break;
    }
  }
  adam_entry(x, m, v, e, g[e], lr, lo, hi, ac);
}

__global__ void k_set_step(int64_t* step, int64_t value, const double* sched, double* snext) {
  if (blockIdx.x != 0) return;
  if (threadIdx.x == 0) step[0] = value;
  if (threadIdx.x < kSchedStride) snext[threadIdx.x] = sched[value * kSchedStride + threadIdx.x];
}

__global__ void k_clear_flag(int* flag) {
  if (threadIdx.x == 0 && blockIdx.x == 0) flag[0] = 0;
}

__global__ __launch_bounds__(kBlock) void k_check_finite(const double* x, size_t n, int* flag) {
  const size_t e = (size_t)blockIdx.x * kBlock + threadIdx.x;
  if (e < n && !isfinite(x[e])) flag[0] = 1;
}

// ---------------------------------------------------------------------------
// launchers

template <typename LT>
void launch_ctg_main(int bl, dim3 grid, dim3 block, hipStream_t s, const EvalArgs& a,
                     const LT* lodf) {
  // sFk[tc][64] + z and S of every (period, wavefront, lane)
  const size_t lds = (size_t)a.tc * 64 * (1 + 2 * (block.x / 64)) * sizeof(double);
  switch (bl) {
    case 8: hipLaunchKernelGGL((k_ctg_main<8, LT>), grid, block, lds, s, a, lodf); break;
    case 16: hipLaunchKernelGGL((k_ctg_main<16, LT>), grid, block, lds, s, a, lodf); break;
    default: hipLaunchKernelGGL((k_ctg_main<32, LT>), grid, block, lds, s, a, lodf); break;
  }
}

// The map-reduce takes the skip test (ctg_cold_mask) with every contingency
// scored and blocks of 4 to 64 / TCW branch tiles: with fewer tiles per
// block the mask's cost is not recovered.
constexpr int kSkipMinTiles = 4;
inline bool ctg_skip(const EvalArgs& a, int tcw) {
  return a.p.lmaxh != nullptr && a.act_k == nullptr && a.lt >= kSkipMinTiles && a.lt <= 64 / tcw;
}

template <int TCW, typename LT>
void launch_ctg_pm_t(dim3 grid, dim3 block, hipStream_t s, const EvalArgs& a, const LT* lodf) {
  // z and S of every (wavefront, period, lane)
  const size_t lds = (size_t)(block.x / 64) * TCW * 128 * sizeof(double);
  if (ctg_skip(a, TCW)) {
    hipLaunchKernelGGL((k_ctg_pm<TCW, LT, true>), grid, block, lds, s, a, lodf);
    return;
  }
  hipLaunchKernelGGL((k_ctg_pm<TCW, LT, false>), grid, block, lds, s, a, lodf);
}

template <typename LT>
void launch_ctg_pm(int tcw, dim3 grid, dim3 block, hipStream_t s, const EvalArgs& a,
                   const LT* lodf) {
  switch (tcw) {
    case 1: launch_ctg_pm_t<1>(grid, block, s, a, lodf); break;
    case 2: launch_ctg_pm_t<2>(grid, block, s, a, lodf); break;
    case 3: launch_ctg_pm_t<3>(grid, block, s, a, lodf); break;
    case 4: launch_ctg_pm_t<4>(grid, block, s, a, lodf); break;
    case 5: launch_ctg_pm_t<5>(grid, block, s, a, lodf); break;
    case 6: launch_ctg_pm_t<6>(grid, block, s, a, lodf); break;
    case 7: launch_ctg_pm_t<7>(grid, block, s, a, lodf); break;
    default: launch_ctg_pm_t<8>(grid, block, s, a, lodf); break;
  }
}

template <typename LT>
void launch_ctg(const Problem* pr, hipStream_t s, const EvalArgs& a, const LT* lodf) {
  const CtgTile& t = pr->tile;
  const int span = t.split ? t.wl * t.tc : t.tc;
  const dim3 grid(pr->nLb, a.nKb, (pr->T + span - 1) / span), block(64 * t.wl);
  if (t.split)
    launch_ctg_pm(t.tc, grid, block, s, a, lodf);
  else
    launch_ctg_main(t.bl, grid, block, s, a, lodf);
}

static EvalArgs make_args(const Problem* pr, const DevWork& w, const double* x, double* grad,
                          double* terms_out, const EvalMode& mode, int fuse_adam, double* m,
                          double* v) {
  EvalArgs a;
  a.p = pr->dp;
  a.w = w;
  a.x = x;
  a.grad = grad;
  a.terms_out = terms_out;
  a.m = m;
  a.v = v;
  a.mode = mode;
  a.fuse_adam = fuse_adam;
  a.nb_br = pr->nb_br;
  a.nb_bus = pr->nb_bus;
  a.bus_chunks = pr->bus_chunks;
  a.nb_gen = pr->nb_gen;
  a.nsplit = pr->nsplit;
  a.nLb = pr->nLb;
  a.nKb = pr->nKb;
  a.nKc = pr->nKc;
  a.nLc = pr->nLc;
  a.tc = pr->tile.tc;
  a.lt = pr->tile.lt;
  a.sparse = pr->tile.split;
  a.zfk = pr->nKb_max;
  a.zfs = pr->nLb_max;
  a.rfs = rflag_stride(pr->nKb_max);
  a.toff = pr->toff;
  const Screen& sc = pr->scr;
  if (mode.screened) {
    a.act_k = sc.act_k;
    a.act_slot = sc.act_slot;
    a.na = sc.n_act;
    a.kst = sc.Ka;
    a.nKb = a.nKc = sc.Ka / kCtgLanes;
    a.lodf_sel = sc.lodf_act;
  } else {
    a.act_k = nullptr;
    a.act_slot = nullptr;
    a.na = pr->K;
    a.kst = pr->Kp;
    const DevProblem& dp = pr->dp;
    a.lodf_sel = dp.lodf_kind == kLodfF64 ? (const void*)dp.lodf
                 : dp.lodf_kind == kLodfF32 ? (const void*)dp.lodf32 : (const void*)dp.lodf16;
  }
  return a;
}

// Blocks of k_ctg_asm: the device-term slices, the flow-adjoint chunks and
// the bus-balance blocks.
static int asm_blocks(const Problem* pr) {
  return pr->T * ((pr->G + kBlock - 1) / kBlock) + pr->nLc * pr->T + pr->nb_bus;
}

// One kernel of the step, in stream order 0..kStages-1.
static void launch_stage(const Problem* pr, const EvalArgs& a, int stage, hipStream_t s) {
  switch (stage) {
    case 0:
      hipLaunchKernelGGL(k_forward, dim3(pr->nb_br + pr->T + pr->Lp / 16 * (pr->Tp / 16)),
                         dim3(kBlock), 0, s, a);
      break;
    case 1:
      if (pr->K > 0) {
        const int kind = pr->dp.lodf_kind;
        if (kind == kLodfF64)
          launch_ctg(pr, s, a, static_cast<const double*>(a.lodf_sel));
        else if (kind == kLodfF32)
          launch_ctg(pr, s, a, static_cast<const float*>(a.lodf_sel));
        else
          launch_ctg(pr, s, a, static_cast<const uint16_t*>(a.lodf_sel));
      }
      break;
    case 2:
      if (pr->K > 0) {
        if (a.sparse)
          hipLaunchKernelGGL(k_ctg_zred<true>, dim3(a.nKc, pr->T), dim3(64), 0, s, a);
        else
          hipLaunchKernelGGL(k_ctg_zred<false>, dim3(a.nKc, pr->T), dim3(64), 0, s, a);
      }
      break;
    case 3:
      if (a.sparse)
        hipLaunchKernelGGL(k_ctg_asm<true>, dim3(asm_blocks(pr)), dim3(kBlock), 0,
                           s, a);
      else
        hipLaunchKernelGGL(k_ctg_asm<false>, dim3(asm_blocks(pr)), dim3(kBlock), 0,
                           s, a);
      break;
    case 4:
      hipLaunchKernelGGL(k_adjoint,
                         dim3(pr->G16 / 16 * pr->nsplit + pr->nb_br +
                              (pr->T * pr->G16 + kBlock - 1) / kBlock),
                         dim3(kBlock), 0,
                         s, a);
      break;
    default:
      hipLaunchKernelGGL(k_final, dim3(pr->nb_bus + pr->nb_gen + 1), dim3(kBlock), 0, s, a);
      break;
  }
}

int launch_eval(const Problem* pr, const DevWork& w, const double* x, double* grad,
                double* terms_out, const EvalMode& mode, int fuse_adam, double* m, double* v,
                void* stream, void** events) {
  hipStream_t s = static_cast<hipStream_t>(stream);
  const EvalArgs a = make_args(pr, w, x, grad, terms_out, mode, fuse_adam, m, v);
  for (int i = 0; i < kStages; ++i) {
    if (events) (void)hipEventRecord(static_cast<hipEvent_t>(events[i]), s);
    launch_stage(pr, a, i, s);
  }
  if (events) (void)hipEventRecord(static_cast<hipEvent_t>(events[kStages]), s);
  return (int)hipGetLastError();
}

// ---------------------------------------------------------------------------
// Batched step: the same six stages for many independent problems, one launch
// per stage.  A block finds its problem and its block of that problem in the
// stage's table (one scalar load); the kernel arguments of every problem sit
// in the batch buffer.  Each problem's blocks do exactly what they do in a
// launch of its own, so a batched step gives bitwise the points of the
// problems' own steps.

__device__ __forceinline__ void batch_entry(const uint32_t* __restrict__ tab, uint32_t i, int& s,
                                            int& loc) {
  const uint32_t e = tab[i];
  s = (int)(e >> kBatchLocBits);
  loc = (int)(e & ((1u << kBatchLocBits) - 1u));
}

__global__ __launch_bounds__(kBlock) void k_forward_b(const EvalArgs* __restrict__ args,
                                                      const uint32_t* __restrict__ tab, int* ctr) {
  __shared__ double smem[kFwdLds];
  // the work counter of this step's map-reduce (the previous step's has
  // finished: the launches are ordered)
  if (blockIdx.x == 0 && threadIdx.x == 0) *ctr = 0;
  int s, b;
  batch_entry(tab, blockIdx.x, s, b);
  forward_body(args[s], b, smem);
}

// Persistent contingency map-reduce: every block takes work items (one
// period-split block of one problem: l-block, k-block, period chunk) from the
// counter until none is left, and runs k_ctg_pm's block code on each (a
// wavefront without periods skips it, as every wavefront must reach the
// barriers of the loop).  Items are ordered by decreasing work, so the
// last ones to be taken are short.  Tiles: 4 wavefronts of 4 periods (the
// problem's tile), its branch tiles per block free.
template <typename LT, bool SKIP>
__global__ __launch_bounds__(kBatchWl * 64) void k_ctg_pm_b(const EvalArgs* __restrict__ args,
                                                            const uint32_t* __restrict__ items,
                                                            int nitems, int* ctr) {
  extern __shared__ double dyn[];
  __shared__ int next;
  for (;;) {
    if (threadIdx.x == 0) next = atomicAdd(ctr, 1);
    __syncthreads();
    const int it = next;
    __syncthreads();  // every wave has read the item before it is replaced
    if (it >= nitems) break;
    int s, loc;
    batch_entry(items, (uint32_t)it, s, loc);
    const EvalArgs& a = args[s];
    const int nLb = a.nLb, nKb = a.nKb;
    const int lb = loc % nLb, kb = (loc / nLb) % nKb, bz = loc / (nLb * nKb);
    constexpr int TCW = kBatchTcw;
    const int WL = kBatchWl;
    const LT* __restrict__ lodf = static_cast<const LT*>(a.lodf_sel);
    {
      typedef typename std::conditional<std::is_same<LT, double>::value, double, float>::type R;
      constexpr bool kF64 = std::is_same<R, double>::value;
      const DevProblem& p = a.p;
      const DevWork& w = a.w;
      const int lane = threadIdx.x & 63;
      const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
      const int T = p.T, Lp = p.Lp, Kp = p.Kp;
      const int tw = (bz * WL + wv) * TCW;  // first period of the wavefront
      const int ntw = min(TCW, T - tw);
      if (ntw > 0) {
      const int k = kb * 64 + lane;  // slot of the lane
      const int kc = a.act_k ? a.act_k[k] : k;
      // z and S of the wavefront's (period, lane) pairs live in its own slice
      // of LDS: only the per-branch path and the final store touch them
      double* zsh = dyn + (size_t)wv * TCW * 128;
      double* ssh = zsh + TCW * 64;
      R fk[TCW];
    #pragma unroll
      for (int i = 0; i < TCW; ++i) {
        fk[i] = i < ntw ? (R)w.Fk[(size_t)(tw + i) * Kp + kc] : R(0);
        zsh[i * 64 + lane] = 0.0;
        ssh[i * 64 + lane] = 0.0;
      }
      const cdouble* Sc = as_const(p.ctg_smax2);
      const cdouble* Mc = as_const(p.ctg_smax);
      const cdouble* Dc = as_const(p.dt);
      const cdouble* Qc = as_const(w.q2);
      const cdouble* FH = as_const(w.fh);
      const double beta = w.params[PB_BETA];
      const R eps = (R)w.params[PB_EPS];
      const R eps2 = eps * eps;
      const int ei = lane >> 3, eg = lane & 7;
      const int l0 = lb * a.lt * 8;
      const int l1 = min(Lp, l0 + a.lt * 8);
      // The factor loads of the tile loop go through a buffer resource over
      // the block's rows: the lane's fixed 32-bit byte offset (its slot k) plus
      // a uniform row offset that advances with the tile, so the loop needs no
      // per-lane address arithmetic.
      unsigned rowb = (unsigned)a.kst * (unsigned)sizeof(LT);  // bytes per factor row
      const __amdgpu_buffer_rsrc_t lrs =
          buf_rsrc(lodf + (size_t)l0 * a.kst, (unsigned)(l1 - l0) * rowb);
      const unsigned koff = (unsigned)k * (unsigned)sizeof(LT);
      // R/Q flags of the lane's period (lane e < ntw: period tw + e), bit i for
      // tile i of the block, stored after the loop
      uint64_t fbits = 0;
      // SKIP: half rows proved free of overloads are skipped (ctg_cold_mask),
      // with FP64 factors, every contingency scored and a block of at most
      // 64 / TCW tiles (two masks of 32 / TCW tiles cover them; the host
      // launches the SKIP form only then, and a block outside it tests
      // everything); the F and thr of a tested half row are loaded when it is
      // reached.  Otherwise they are prefetched one half row ahead.
      // Bit ((ti mod CT) TCW + i) 2 + h of mask ti / CT (CT = 32 / TCW): half
      // row h of period tw + i of tile ti skipped.
      uint64_t coldm = 0, coldm1 = 0;
      if constexpr (SKIP) {
        constexpr int CT = 32 / TCW;  // tiles per mask
        const int ntile = (l1 - l0) >> 3;
        if (p.lmaxh != nullptr && a.act_k == nullptr && ntile <= 2 * CT) {
          double fkm = 0.0;  // largest |F_tk| of the wave's lanes and periods
    #pragma unroll
          for (int i = 0; i < TCW; ++i) fkm = fmax(fkm, fabs(fk[i]));
          fkm = wave_max(fkm);
          coldm = ctg_cold_mask<TCW, kF64>(w.fh, p.lmaxh, T, tw, ntw, l0 >> 3, ntile, kb, Kp >> 6,
                                           fkm, w.q2, p.ctg_smax2, Lp);
          if (ntile > CT)
            coldm1 = ctg_cold_mask<TCW, kF64>(w.fh, p.lmaxh, T, tw, ntw, (l0 >> 3) + CT, ntile - CT,
                                              kb, Kp >> 6, fkm, w.q2, p.ctg_smax2, Lp);
        }
      }
      // F and thr of the next half row (four branches of one period) to be
      // tested, from the branch-tiled copy, so that every prefetch is a fixed
      // offset from the tile's row of period tw
      double Fn[4], Hn[4];
      if constexpr (kF64 && !SKIP) {
        const cdouble* r = FH + ((size_t)(l0 >> 3) * T + tw) * 16;
    #pragma unroll
        for (int g = 0; g < 4; ++g) {
          Fn[g] = r[g];
          Hn[g] = r[4 + g];
        }
      }
      const uint32_t live = (1u << ntw) - 1u;  // the wave's periods among the TCW tested
      unsigned lso = 0;  // uniform offset of the tile's factor rows
      int ti = 0;        // tile index in the block
      // rows of the branch-tiled copy: period tw of the tile, of the next tile
      const cdouble* cur = FH + ((size_t)(l0 >> 3) * T + tw) * 16;
      unsigned fstep = (unsigned)T * 16u;
      for (int lbase = l0; lbase < l1; lbase += 8, lso += 8 * rowb, ++ti, cur += fstep) {
        // the strides are taken as changing in every tile, so that nothing
        // derived from them is hoisted out of the loop (such values took SGPRs
        // that were then spilled, and reloading them costs vector instructions)
        asm volatile("" : "+s"(rowb), "+s"(fstep));
        const cdouble* nxt = cur + fstep;
        // the tile's half rows that are tested (bit 2 i + h); a tile without
        // any is passed over, and only the factor rows of tested halves are loaded
        const uint32_t need =
            ~(uint32_t)((ti < 32 / TCW ? coldm : coldm1) >> ((ti % (32 / TCW)) * TCW * 2)) &
            ((1u << (2 * TCW)) - 1u);
        if (need == 0) continue;
        R lod[8];
    #pragma unroll
        for (int j = 0; j < 8; ++j)
          lod[j] = (need & (j < 4 ? 0x5555u : 0xAAAAu)) ? lodf_buf(lrs, lodf, koff, lso + j * rowb) : R(0);
        R fv = R(0), qv = R(0), smx2[8];
        if constexpr (!kF64) {
          if (ei < ntw) {
            const size_t e = (size_t)(tw + ei) * Lp + lbase + eg;
            fv = (R)w.F[e];
            qv = (R)w.q2[e];
          }
    #pragma unroll
          for (int j = 0; j < 8; ++j) smx2[j] = (R)Sc[lbase + j];
        }
        // The test of every (period, branch, lane) of the tile, without a
        // branch: all TCW periods are tested (the rows past the wave's last
        // period are spare rows of the array, and their verdicts are dropped
        // with the mask), and each period's verdict is one bit of hotm.
        uint32_t hotm = 0;
    #pragma unroll
        for (int i = 0; i < TCW; ++i) {
          uint64_t hot = 0;
          if constexpr (SKIP && kF64) {
    #pragma unroll
            for (int h = 0; h < 2; ++h) {
              if ((need >> (2 * i + h)) & 1u) {
                double Fr[4], Hr[4];
                const cdouble* q = cur + 16 * i + 8 * h;
    #pragma unroll
                for (int g = 0; g < 4; ++g) {
                  Fr[g] = q[g];
                  Hr[g] = q[4 + g];
                }
    #pragma unroll
                for (int g = 0; g < 4; ++g) {
                  const double P = fma_uniform_c(lod[4 * h + g], fk[i], Fr[g]);
                  hot |= __builtin_amdgcn_ballot_w64(fabs(P) > Hr[g]);
                }
              }
            }
          } else if constexpr (kF64) {
    #pragma unroll
            for (int h = 0; h < 2; ++h) {
              double Fr[4], Hr[4];
    #pragma unroll
              for (int g = 0; g < 4; ++g) {
                Fr[g] = Fn[g];
                Hr[g] = Hn[g];
              }
              // prefetch: the other half of this period's row, else the next
              // period of this tile, else period tw of the next tile (rows past
              // the tile or the last tile are spare rows)
              const cdouble* q = h == 0 ? cur + 16 * i + 8 : (i + 1 < TCW) ? cur + 16 * (i + 1) : nxt;
    #pragma unroll
              for (int g = 0; g < 4; ++g) {
                Fn[g] = q[g];
                Hn[g] = q[4 + g];
              }
    #pragma unroll
              for (int g = 0; g < 4; ++g) {
                const double P = fma_uniform_c(lod[4 * h + g], fk[i], Fr[g]);
                hot |= __builtin_amdgcn_ballot_w64(fabs(P) > Hr[g]);
              }
            }
          } else {
            // FP32 arithmetic; with SKIP only the half rows that are tested
    #pragma unroll
            for (int h = 0; h < 2; ++h) {
              if ((need >> (2 * i + h)) & 1u) {
    #pragma unroll
                for (int gg = 0; gg < 4; ++gg) {
                  const int g = 4 * h + gg;
                  const R Fr = readlane_any(fv, i * 8 + g);
                  const R P = fma_uniform_c(lod[g], fk[i], Fr);
                  const R s2 = fma_uniform_c(P, P, readlane_any(qv, i * 8 + g));
                  hot |= __builtin_amdgcn_ballot_w64(s2 > smx2[g]);
                }
              }
            }
          }
          hotm |= (hot != 0 ? 1u : 0u) << i;
        }
        hotm &= live;
        // a wave with fewer than TCW periods prefetched a spare row for the
        // next tile: load its first period's row again
        if constexpr (kF64 && !SKIP) {
          if (ntw < TCW) {
    #pragma unroll
            for (int g = 0; g < 4; ++g) {
              Fn[g] = nxt[g];
              Hn[g] = nxt[4 + g];
            }
          }
        }
        if (hotm) {
          // R and Q of (period tw + e / 8, branch lbase + e % 8) gather in lane e
          R racc = R(0), qacc = R(0);
          // the overloaded periods of the tile: the per-branch path, with F,
          // qmax2 and the ratings loaded again
    #pragma unroll
          for (int i = 0; i < TCW; ++i) {
            if ((hotm >> i) & 1u) {
              const R kt = (R)(Dc[tw + i] * p.c_s * beta);
              R Fr[8], Qr[8], Sr[8];
    #pragma unroll
              for (int g = 0; g < 8; ++g) {
                if constexpr (kF64) {
                  Fr[g] = cur[16 * i + fh_col_f(g)];
                  Qr[g] = Qc[(size_t)(tw + i) * Lp + lbase + g];
                  Sr[g] = Sc[lbase + g];
                } else {
                  Fr[g] = readlane_any(fv, i * 8 + g);
                  Qr[g] = readlane_any(qv, i * 8 + g);
                  Sr[g] = smx2[g];
                }
              }
              R zt = R(0), st = R(0);
    #pragma unroll
              for (int g = 0; g < 8; ++g) {
                // a skipped half row holds no overload (and its factors were
                // not loaded)
                if (((need >> (2 * i + (g >> 2))) & 1u) == 0) continue;
                // the flow formed again (the same fused operation, so the same
                // value as in the test)
                const R P = fma_uniform_c(lod[g], fk[i], Fr[g]);
                const R s2 = fma_uniform_c(P, P, Qr[g]);
                if (__builtin_amdgcn_ballot_w64(s2 > Sr[g])) {
                  R dP = R(0), dq = R(0);
                  if (s2 > Sr[g]) {
                    zt += ctg_overload(P, s2, (R)Mc[lbase + g], eps, eps2, kt, dP, dq);
                    st = fma(lod[g], dP, st);
                  }
                  const R r = pair_sum(dP, dq);  // lane 0: sum of dP, lane 32: of dq
                  racc = writelane_set(racc, readlane_any(r, 0), i * 8 + g);
                  qacc = writelane_set(qacc, readlane_any(r, 32), i * 8 + g);
                }
              }
              zsh[i * 64 + lane] += (double)zt;
              ssh[i * 64 + lane] += (double)st;
            }
          }
          // per (period, 8 branches): stored only when not all zero, and flagged
          const uint64_t b = __builtin_amdgcn_ballot_w64(racc != R(0) || qacc != R(0));
          if (lane < ntw && ((b >> (8 * lane)) & 0xFF) != 0) fbits |= (uint64_t)1 << ti;
          if (b != 0 && lane < ntw * 8 && ((b >> (lane & ~7)) & 0xFF) != 0) {
            const size_t o = ((size_t)kb * T + tw + ei) * Lp + lbase + eg;
            w.rpart[o] = (double)racc;
            w.qpart[o] = (double)qacc;
          }
        }
      }
      if (lane < ntw) {
        uint8_t* f = w.rflag + ((size_t)(tw + lane) * (Lp / 8) + (l0 >> 3)) * a.rfs + kb;
        for (int i = 0; i < ti; ++i) f[(size_t)i * a.rfs] = (uint8_t)((fbits >> i) & 1u);
      }
    #pragma unroll
      for (int i = 0; i < TCW; ++i) {
        if (i < ntw) {
          // stored only when not all zero, and flagged
          const double z = zsh[i * 64 + lane], s2 = ssh[i * 64 + lane];
          const bool nz = __builtin_amdgcn_ballot_w64(z != 0.0 || s2 != 0.0) != 0;
          if (lane == 0) w.zflag[((size_t)(tw + i) * a.zfk + kb) * a.zfs + lb] = (uint8_t)nz;
          if (nz) {
            const size_t o = ((size_t)lb * T + tw + i) * Kp + k;
            w.zpart[o] = z;
            w.spart[o] = s2;
          }
        }
      }
      }

    }
  }
}

__global__ __launch_bounds__(64) void k_ctg_zred_b(const EvalArgs* __restrict__ args,
                                                   const uint32_t* __restrict__ tab) {
  int s, b;
  batch_entry(tab, blockIdx.x, s, b);
  const EvalArgs& a = args[s];
  ctg_zred_body<true>(a, b % a.nKc, b / a.nKc);
}

__global__ __launch_bounds__(kBlock) void k_ctg_asm_b(const EvalArgs* __restrict__ args,
                                                      const uint32_t* __restrict__ tab) {
  __shared__ double smem[2 * kSegChunk + 16];
  int s, b;
  batch_entry(tab, blockIdx.x, s, b);
  const EvalArgs& a = args[s];
  ctg_asm_body<true>(a, b, a.p.T * ((a.p.G + kBlock - 1) / kBlock) + a.nLc * a.p.T + a.nb_bus,
                     smem);
}

__global__ __launch_bounds__(kBlock) void k_adjoint_b(const EvalArgs* __restrict__ args,
                                                      const uint32_t* __restrict__ tab) {
  __shared__ double smem[kSlabLds];
  int s, b;
  batch_entry(tab, blockIdx.x, s, b);
  adjoint_body(args[s], b, smem);
}

__global__ __launch_bounds__(kBlock) void k_final_b(const EvalArgs* __restrict__ args,
                                                    const uint32_t* __restrict__ tab) {
  __shared__ double smem[2 * kSegChunk + 8 * kBlock];
  int s, b;
  batch_entry(tab, blockIdx.x, s, b);
  final_body(args[s], b, smem);
}

// Blocks of each stage of one problem (stage 1: map-reduce work items).
static void stage_blocks(const Problem* pr, const EvalArgs& a, int out[kStages]) {
  const int span = pr->tile.wl * pr->tile.tc;
  out[0] = pr->nb_br + pr->T + pr->Lp / 16 * (pr->Tp / 16);
  out[1] = pr->K > 0 ? pr->nLb * a.nKb * ((pr->T + span - 1) / span) : 0;
  out[2] = pr->K > 0 ? a.nKc * pr->T : 0;
  out[3] = asm_blocks(pr);
  out[4] = pr->G16 / 16 * pr->nsplit + pr->nb_br + (pr->T * pr->G16 + kBlock - 1) / kBlock;
  out[5] = pr->nb_bus + pr->nb_gen + 1;
}

static size_t align_up(size_t v) { return (v + kAlign - 1) / kAlign * kAlign; }

int plan_batch(const Problem* const* prs, const DevWork* ws, int n, const double* const* x,
               double* const* m, double* const* v, const EvalMode& mode, BatchPlan* plan,
               std::vector<unsigned char>* image, std::string* err) {
  BatchPlan P;
  P.n = n;
  std::vector<EvalArgs> args((size_t)n);
  std::vector<std::array<int, kStages>> nb((size_t)n);
  for (int i = 0; i < n; ++i) {
    const Problem* pr = prs[i];
    const CtgTile& t = pr->tile;
    if (pr->K > 0 && !(t.split && t.wl == kBatchWl && t.tc == kBatchTcw)) {
      *err = "problem " + std::to_string(i) +
             ": the batched step needs a period-split tile of 4 wavefronts of 4 periods";
      return 1;
    }
    if (pr->scr.on) {
      *err = "problem " + std::to_string(i) + ": screening is not supported in a batch";
      return 1;
    }
    if (i > 0 && pr->dp.lodf_kind != prs[0]->dp.lodf_kind) {
      *err = "every problem of a batch needs the same storage of the outage factors";
      return 1;
    }
    args[i] = make_args(pr, ws[i], x[i], nullptr, nullptr, mode, 1, m[i], v[i]);
    int b[kStages];
    stage_blocks(pr, args[i], b);
    for (int q = 0; q < kStages; ++q) {
      if (b[q] >= (1 << kBatchLocBits)) {
        *err = "problem " + std::to_string(i) + " has too many blocks for a batch";
        return 1;
      }
      nb[i][q] = b[q];
      P.nblk[q] += b[q];
    }
  }
  P.lodf_kind = n > 0 ? prs[0]->dp.lodf_kind : 0;
  size_t o = 0;
  P.off_args = o;
  o = align_up(o + (size_t)n * sizeof(EvalArgs));
  for (int q = 0; q < kStages; ++q) {
    P.off_tab[q] = o;
    o = align_up(o + (size_t)P.nblk[q] * sizeof(uint32_t));
  }
  P.off_ctr = o;
  o = align_up(o + sizeof(int));
  P.bytes = o;
  if (image) {
    image->assign(P.bytes, 0);
    std::memcpy(image->data() + P.off_args, args.data(), (size_t)n * sizeof(EvalArgs));
    // map-reduce items: problems by decreasing work per item (periods and
    // branch tiles of a block), each problem's items in its grid order
    std::vector<int> order((size_t)n);
    for (int i = 0; i < n; ++i) order[i] = i;
    auto item_work = [&](int i) {
      const Problem* pr = prs[i];
      return (int64_t)std::min(pr->T, kBatchWl * pr->tile.tc) * pr->tile.lt;
    };
    std::stable_sort(order.begin(), order.end(),
                     [&](int a2, int b2) { return item_work(a2) > item_work(b2); });
    for (int q = 0; q < kStages; ++q) {
      uint32_t* tab = reinterpret_cast<uint32_t*>(image->data() + P.off_tab[q]);
      size_t k = 0;
      for (int j = 0; j < n; ++j) {
        const int i = q == 1 ? order[j] : j;
        for (int b = 0; b < nb[i][q]; ++b)
          tab[k++] = ((uint32_t)i << kBatchLocBits) | (uint32_t)b;
      }
    }
  }
  // persistent map-reduce: as many blocks as fit on the chip at once
  int dev = 0, ncu = 256, per_cu = 1;
  const size_t lds = (size_t)kBatchWl * kBatchTcw * 128 * sizeof(double);
  if (hipGetDevice(&dev) == hipSuccess)
    (void)hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev);
  // the skip test (FP64) when a problem's blocks qualify for it; the SKIP
  // kernel tests every half row of the others
  P.skip = false;
  for (int i = 0; i < n; ++i)
    P.skip = P.skip || (prs[i]->dp.lmaxh != nullptr && prs[i]->tile.lt >= kSkipMinTiles &&
                        prs[i]->tile.lt <= 64 / kBatchTcw);
  hipError_t e;
  if (P.lodf_kind == kLodfF64)
    e = P.skip ? hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_ctg_pm_b<double, true>,
                                                              kBatchWl * 64, lds)
               : hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_ctg_pm_b<double, false>,
                                                              kBatchWl * 64, lds);
  else if (P.lodf_kind == kLodfF32)
    e = P.skip ? hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_ctg_pm_b<float, true>,
                                                              kBatchWl * 64, lds)
               : hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_ctg_pm_b<float, false>,
                                                              kBatchWl * 64, lds);
  else
    e = P.skip
            ? hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_ctg_pm_b<uint16_t, true>,
                                                           kBatchWl * 64, lds)
            : hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_ctg_pm_b<uint16_t, false>,
                                                           kBatchWl * 64, lds);
  if (e != hipSuccess || per_cu < 1) per_cu = 1;
  P.pm_grid = std::max(1, std::min(P.nblk[1], ncu * per_cu));
  *plan = P;
  return 0;
}

int launch_eval_batch(const BatchPlan& P, void* d_buf, void* stream) {
  hipStream_t s = static_cast<hipStream_t>(stream);
  unsigned char* b = static_cast<unsigned char*>(d_buf);
  const EvalArgs* args = reinterpret_cast<const EvalArgs*>(b + P.off_args);
  auto tab = [&](int q) { return reinterpret_cast<const uint32_t*>(b + P.off_tab[q]); };
  int* ctr = reinterpret_cast<int*>(b + P.off_ctr);
  hipLaunchKernelGGL(k_forward_b, dim3(P.nblk[0]), dim3(kBlock), 0, s, args, tab(0), ctr);
  if (P.nblk[1] > 0) {
    const size_t lds = (size_t)kBatchWl * kBatchTcw * 128 * sizeof(double);
    const dim3 g(P.pm_grid), blk(kBatchWl * 64);
    if (P.lodf_kind == kLodfF64 && P.skip)
      hipLaunchKernelGGL((k_ctg_pm_b<double, true>), g, blk, lds, s, args, tab(1), P.nblk[1], ctr);
    else if (P.lodf_kind == kLodfF64)
      hipLaunchKernelGGL((k_ctg_pm_b<double, false>), g, blk, lds, s, args, tab(1), P.nblk[1], ctr);
    else if (P.lodf_kind == kLodfF32 && P.skip)
      hipLaunchKernelGGL((k_ctg_pm_b<float, true>), g, blk, lds, s, args, tab(1), P.nblk[1], ctr);
    else if (P.lodf_kind == kLodfF32)
      hipLaunchKernelGGL((k_ctg_pm_b<float, false>), g, blk, lds, s, args, tab(1), P.nblk[1], ctr);
    else if (P.skip)
      hipLaunchKernelGGL((k_ctg_pm_b<uint16_t, true>), g, blk, lds, s, args, tab(1), P.nblk[1],
                         ctr);
    else
      hipLaunchKernelGGL((k_ctg_pm_b<uint16_t, false>), g, blk, lds, s, args, tab(1), P.nblk[1],
                         ctr);
  }
  if (P.nblk[2] > 0)
    hipLaunchKernelGGL(k_ctg_zred_b, dim3(P.nblk[2]), dim3(64), 0, s, args, tab(2));
  hipLaunchKernelGGL(k_ctg_asm_b, dim3(P.nblk[3]), dim3(kBlock), 0, s, args, tab(3));
  hipLaunchKernelGGL(k_adjoint_b, dim3(P.nblk[4]), dim3(kBlock), 0, s, args, tab(4));
  hipLaunchKernelGGL(k_final_b, dim3(P.nblk[5]), dim3(kBlock), 0, s, args, tab(5));
  return (int)hipGetLastError();
}

int time_stage(const Problem* pr, const DevWork& w, const double* x, const EvalMode& mode,
               int stage, int reps, void* stream, double* mean_ms) {
  hipStream_t s = static_cast<hipStream_t>(stream);
  const EvalArgs a = make_args(pr, w, x, nullptr, nullptr, mode, 0, nullptr, nullptr);
  for (int i = 0; i < kStages; ++i) launch_stage(pr, a, i, s);  // inputs of every stage
  hipEvent_t e0, e1;
  hipError_t err = hipEventCreate(&e0);
  if (err != hipSuccess) return (int)err;
  err = hipEventCreate(&e1);
  if (err != hipSuccess) { (void)hipEventDestroy(e0); return (int)err; }
  launch_stage(pr, a, stage, s);  // warm
  (void)hipEventRecord(e0, s);
  for (int r = 0; r < reps; ++r) launch_stage(pr, a, stage, s);
  (void)hipEventRecord(e1, s);
  err = hipEventSynchronize(e1);
  float ms = 0.f;
  if (err == hipSuccess) err = hipEventElapsedTime(&ms, e0, e1);
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (err != hipSuccess) return (int)err;
  *mean_ms = (double)ms / reps;
  return (int)hipGetLastError();
}

int launch_adam(const Problem* pr, double* x, double* m, double* v, const double* g,
                const double lr[QG_NCLASS], double bc1, double bc2, double b1, double b2,
                double eps, int eps_in_num, void* stream) {
  hipStream_t s = static_cast<hipStream_t>(stream);
  AdamCtx ac{b1, b2, eps, bc1, bc2, eps_in_num};
  const int nb = (int)((pr->n_x + kBlock - 1) / kBlock);
  hipLaunchKernelGGL(k_adam, dim3(nb), dim3(kBlock), 0, s, pr->dp, x, m, v, g, lr[0], lr[1],
                     lr[2], lr[3], lr[4], lr[5], ac);
  return (int)hipGetLastError();
}

int launch_set_step(const Problem* pr, const DevWork& w, int64_t value, void* stream) {
  (void)pr;
  if (value < 0 || value >= kSchedCap) return (int)hipErrorInvalidValue;
  hipLaunchKernelGGL(k_set_step, dim3(1), dim3(64), 0, static_cast<hipStream_t>(stream),
                     w.step, value, (const double*)w.sched, w.snext);
  return (int)hipGetLastError();
}

int launch_check_finite(const Problem* pr, const double* x, int* flag, void* stream) {
  const int nb = (int)((pr->n_x + kBlock - 1) / kBlock);
  hipStream_t s = static_cast<hipStream_t>(stream);
  hipLaunchKernelGGL(k_clear_flag, dim3(1), dim3(64), 0, s, flag);
  hipLaunchKernelGGL(k_check_finite, dim3(nb), dim3(kBlock), 0, s, x, (size_t)pr->n_x, flag);
  return (int)hipGetLastError();
}

}  // namespace qg
