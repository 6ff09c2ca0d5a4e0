// HIP kernels of one solver step for gfx950 (MI355X).
//
// Stage map (one launch each, in stream order):
//   k_forward       per-(t, branch) AC flows and penalties        (Section II-B Ex. 1, 4; II-G)
//                   + one block per period for device terms and   (Ex. 2, 3; eq. (nlp_updated))
//                     the slack-balanced DC injections            (Section II-E)
//   k_balance_flow  per-(t, bus) power balance from bus-sorted    (Ex. 4)
//                     endpoint flows (LDS-staged segmented sums)
//                   + base-case DC flows F = Pbar ISF^T on MFMA   (eqs. (Yb_solve)-(p_flow))
//   k_ctg_main      per-(t, l, k) outage flows F_l + LODF_lk F_k,  (eqs. (rank_correct),
//                     penalties and their partial reductions        (sfr_pen)-(zctg), (2nd_lin_sys))
//   k_ctg_finalize  per period: worst + mean aggregation, weights, the
//                     adjoint of the flows dL/dF
//   k_adjoint       dL/dPbar = (dL/dF) ISF on MFMA                (eqs. (2nd_lin_sys), (correction))
//                   + per-(t, branch) reverse of the AC flows into bus-sorted endpoint slots
//   k_final         per-(t, bus) segmented sums of endpoint adjoints, per-generator
//                     gradient assembly (uniform-slack correction, eq. (correction)),
//                     then either the gradient or the fused Adam update with clip (Alg. 3),
//                     and the deterministic sum of the objective terms.
//
// Every reduction has a fixed order (no floating-point atomics), so a step is
// bitwise reproducible run to run.
#include <hip/hip_runtime.h>

#include <cfloat>
#include <climits>

#include "qg_internal.h"

namespace qg {

typedef double v4d __attribute__((ext_vector_type(4)));

struct StepParams {
  double eps, beta, rho_s;
  double alpha[QG_NCLASS];
  double bc1, bc2;
};

// Parameter block layout (DevWork::params)
enum { PB_EPS = 0, PB_BETA = 1, PB_RHO = 2, PB_ALPHA = 4, PB_BC1 = 10, PB_BC2 = 11 };

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
  int nb_br, nb_bus, bus_chunks, nLb, nKb;
  TermOffsets toff;
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

__device__ __forceinline__ double soft_abs_d(double v, double eps) {
  const double s = sqrt(v * v + eps * eps);
  return s > 0.0 ? v / s : 0.0;
}

template <int CTRL>
__device__ __forceinline__ double dpp_f64(double v) {
  const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(v), CTRL, 0xF, 0xF, false);
  const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(v), CTRL, 0xF, 0xF, false);
  return __hiloint2double(hi, lo);
}

__device__ __forceinline__ double readlane_f64(double v, int lane) {
  const int lo = __builtin_amdgcn_readlane(__double2loint(v), lane);
  const int hi = __builtin_amdgcn_readlane(__double2hiint(v), lane);
  return __hiloint2double(hi, lo);
}

// Sum over the 64 lanes of a wavefront (all lanes active).  Butterflies
// inside each row of 16 lanes with DPP (quad swaps, half-row and row
// mirrors), then the four row sums in lane order.  Every lane gets the same
// bits.
__device__ __forceinline__ double wave_sum(double v) {
  v += dpp_f64<0xB1>(v);   // quad_perm [1,0,3,2]
  v += dpp_f64<0x4E>(v);   // quad_perm [2,3,0,1]
  v += dpp_f64<0x141>(v);  // row_half_mirror
  v += dpp_f64<0x140>(v);  // row_mirror
  return ((readlane_f64(v, 0) + readlane_f64(v, 16)) + readlane_f64(v, 32)) +
         readlane_f64(v, 48);
}

// Deterministic block sum of NV values over a 256-thread block; every
// thread returns the totals.  lds holds NV*256 doubles.
template <int NV>
__device__ __forceinline__ void block_sum(double (&v)[NV], double* lds) {
  const int tid = threadIdx.x;
#pragma unroll
  for (int q = 0; q < NV; ++q) lds[q * kBlock + tid] = v[q];
  __syncthreads();
  for (int s = kBlock / 2; s > 0; s >>= 1) {
    if (tid < s) {
#pragma unroll
      for (int q = 0; q < NV; ++q) lds[q * kBlock + tid] += lds[q * kBlock + tid + s];
    }
    __syncthreads();
  }
#pragma unroll
  for (int q = 0; q < NV; ++q) v[q] = lds[q * kBlock];
  __syncthreads();
}

__device__ double sched_scale(double i, double n) {
  const double th = 2.0 * i / n - 1.0;
  const double e = exp(4.0 * th);
  return e / (0.6 + e);
}

__device__ double sched_log(double a0, double af, double s) {
  return a0 * pow(10.0, s * log10(af / a0));
}

// Homotopy and step sizes of this step: from the arguments, or from the
// iteration-indexed schedule of the solve loop (eqs. (norm_t)-(step_size)).
__device__ void resolve_params(const EvalArgs& a, StepParams& sp) {
  if (a.mode.schedule == 0) {
    sp.eps = a.mode.eps;
    sp.beta = a.mode.beta;
    sp.rho_s = a.mode.rho_s;
    for (int c = 0; c < QG_NCLASS; ++c) sp.alpha[c] = 0.0;
    sp.bc1 = sp.bc2 = 1.0;
    return;
  }
  const double i = (double)(a.w.step[0] + 1);
  const double n = (double)a.mode.n_total;
  const double s = sched_scale(i, n);
  sp.eps = sched_log(a.mode.eps0, a.mode.epsf, s);
  sp.beta = a.mode.beta0 + (a.mode.betaf - a.mode.beta0) * (i / n);
  sp.rho_s = a.mode.rho0 + (a.mode.rhof - a.mode.rho0) * (i / n);
  for (int c = 0; c < QG_NCLASS; ++c) sp.alpha[c] = sched_log(a.mode.alpha0[c], a.mode.alphaf[c], s);
  sp.bc1 = 1.0 - pow(a.mode.adam_b1, i);
  sp.bc2 = 1.0 - pow(a.mode.adam_b2, i);
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
// [n0, n0+16) of C = A * B for all MT*16 rows, where A is stored transposed
// (AT[k][row], row stride Tp) and B row-major (ldb).  The reduction depth kd
// (a multiple of 4) is split over the four wavefronts; their partial tiles
// are summed in LDS in wavefront order.  v_mfma_f64_16x16x4f64 operands:
// lane l holds A[l%16][l/16] and B[l/16][l%16]; the result D[l/16 + 4r][l%16]
// sits in register r of lane l.
template <int MT, class Epi>
__device__ __forceinline__ void mfma_slab(const double* __restrict__ AT, int Tp,
                                          const double* __restrict__ B, int ldb, int kd,
                                          int n0, double* lds, Epi epi) {
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wv = tid >> 6;
  const int steps = kd >> 2;
  const int s0 = (steps * wv) >> 2, s1 = (steps * (wv + 1)) >> 2;
  v4d acc[MT];
#pragma unroll
  for (int mt = 0; mt < MT; ++mt) acc[mt] = v4d{0.0, 0.0, 0.0, 0.0};
  const int kr = lane >> 4, cc = lane & 15;
  for (int st = s0; st < s1; ++st) {
    const int k = st * 4 + kr;
    const double b = B[(size_t)k * ldb + n0 + cc];
#pragma unroll
    for (int mt = 0; mt < MT; ++mt) {
      const double av = AT[(size_t)k * Tp + mt * 16 + cc];
      acc[mt] = __builtin_amdgcn_mfma_f64_16x16x4f64(av, b, acc[mt], 0, 0, 0);
    }
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

template <class Epi>
__device__ __forceinline__ void mfma_slab_dispatch(int mtiles, const double* AT, int Tp,
                                                   const double* B, int ldb, int kd, int n0,
                                                   double* lds, Epi epi) {
  switch (mtiles) {
    case 1: mfma_slab<1>(AT, Tp, B, ldb, kd, n0, lds, epi); break;
    case 2: mfma_slab<2>(AT, Tp, B, ldb, kd, n0, lds, epi); break;
    case 3: mfma_slab<3>(AT, Tp, B, ldb, kd, n0, lds, epi); break;
    default: mfma_slab<4>(AT, Tp, B, ldb, kd, n0, lds, epi); break;
  }
}

// ---------------------------------------------------------------------------
// K1: branch forward + period blocks

__device__ void branch_forward(const EvalArgs& a, const StepParams& sp, double* lds) {
  const DevProblem& p = a.p;
  const DevWork& w = a.w;
  const int T = p.T, L = p.L, N = p.N;
  const int idx = blockIdx.x * kBlock + threadIdx.x;
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
    part[0] = kbr * soft_relu(eb, sp.eps);
    const double kth = kbr * soft_relu_d(eb, sp.eps);
    double kpf = 0.0, kqf = 0.0, kpt = 0.0, kqt = 0.0;
    if (use_f) {
      if (sf > 0.0) { kpf = kth * pf / sf; kqf = kth * qf / sf; }
    } else {
      if (st > 0.0) { kpt = kth * pt / st; kqt = kth * qt / st; }
    }
    // angle-difference penalty
    const double ea = fabs(d) - p.ang_max;
    const double kang = p.dt[t] * p.c_ang * sp.beta;
    part[1] = kang * soft_relu(ea, sp.eps);
    const double sgn = d > 0.0 ? 1.0 : (d < 0.0 ? -1.0 : 0.0);
    const double kd = kang * soft_relu_d(ea, sp.eps) * sgn;
    // reactive part of the contingency flows: max(q_fr^2, q_to^2), ties: from
    const double qf2 = qf * qf, qt2 = qt * qt;
    const bool qfr = qf2 >= qt2;
    w.q2[(size_t)t * p.Lp + l] = qfr ? qf2 : qt2;
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
    w.tpart[a.toff.br + blockIdx.x] = part[0];
    w.tpart[a.toff.ang + blockIdx.x] = part[1];
  }
}

// One block per period t: device costs and penalised device constraints
// (Examples 2-3, eq. (nlp_updated)), reserve shortfall, device-only partials,
// and the uniform-slack DC injections (Section II-E, eq. (correction)).
__device__ void period_block(const EvalArgs& a, const StepParams& sp, int t, double* lds) {
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
  double acc[4] = {0.0, 0.0, 0.0, 0.0};  // dev, pen, sum p, sum r
  for (int j = tid; j < G; j += kBlock) {
    const size_t e = (size_t)t * G + j;
    const double pj = xP[e], qj = xQ[e], rj = xR[e], uj = xU[e];
    const double pm1 = t > 0 ? xP[e - G] : p.p0[j];
    const double um1 = t > 0 ? xU[e - G] : p.u0[j];
    // block-bid energy cost, eq. (costs): sum_m c_m max(min(p - Pcum_{m-1}, D_m), 0)
    double cost = 0.0, dcost = 0.0, lo = 0.0;
    for (int m = 0; m < M; ++m) {
      const double am = pj - lo;
      const double sz = p.seg_size[j * M + m], cm = p.seg_cost[j * M + m];
      cost += cm * fmax(fmin(am, sz), 0.0);
      if (am > 0.0 && am <= sz) dcost += cm;
      lo = p.pcum[j * M + m];
    }
    const double du = uj - um1;
    double dev = dtt * cost + dtt * p.con[j] * uj + p.csu[j] * fmax(du, 0.0) +
                 p.csd[j] * fmax(-du, 0.0) + dtt * p.cr[j] * rj;
    double gp = dtt * dcost;
    double gu = dtt * p.con[j] + (du > 0.0 ? p.csu[j] : 0.0) - (-du > 0.0 ? p.csd[j] : 0.0);
    double gr = dtt * p.cr[j];
    double gq = 0.0;
    if (t + 1 < T) {
      const double du1 = xU[e + G] - uj;
      gu -= (du1 > 0.0 ? p.csu[j] : 0.0) - (-du1 > 0.0 ? p.csd[j] : 0.0);
    }
    // penalised device constraints at t
    double pen = 0.0, a_, dd;
    a_ = pj + rj - p.pmax[j] * uj;                        // headroom
    pen += soft_relu(a_, eps); dd = kpen * soft_relu_d(a_, eps);
    gp += dd; gr += dd; gu -= dd * p.pmax[j];
    a_ = p.pmin[j] * uj - pj;                             // minimum output
    pen += soft_relu(a_, eps); dd = kpen * soft_relu_d(a_, eps);
    gu += dd * p.pmin[j]; gp -= dd;
    a_ = pj - pm1 - dtt * (p.ru[j] * uj + p.rusu[j] * (1.0 - uj));   // ramp up
    pen += soft_relu(a_, eps); dd = kpen * soft_relu_d(a_, eps);
    gp += dd; gu -= dd * dtt * (p.ru[j] - p.rusu[j]);
    a_ = pm1 - pj - dtt * (p.rd[j] * uj + p.rdsd[j] * (1.0 - uj));   // ramp down
    pen += soft_relu(a_, eps); dd = kpen * soft_relu_d(a_, eps);
    gp -= dd; gu -= dd * dtt * (p.rd[j] - p.rdsd[j]);
    a_ = qj - p.qmax[j] * uj;                             // reactive upper
    pen += soft_relu(a_, eps); dd = kpen * soft_relu_d(a_, eps);
    gq += dd; gu -= dd * p.qmax[j];
    a_ = p.qmin[j] * uj - qj;                             // reactive lower
    pen += soft_relu(a_, eps); dd = kpen * soft_relu_d(a_, eps);
    gu += dd * p.qmin[j]; gq -= dd;
    a_ = rj - p.rmax[j] * uj;                             // reserve capability
    pen += soft_relu(a_, eps); dd = kpen * soft_relu_d(a_, eps);
    gr += dd; gu -= dd * p.rmax[j];
    // the next period's ramp constraints depend on p_t
    if (t + 1 < T) {
      const double dt1 = p.dt[t + 1];
      const double k1 = sp.rho_s * p.rho * sp.beta * dt1;
      const double p1 = xP[e + G], u1 = xU[e + G];
      a_ = p1 - pj - dt1 * (p.ru[j] * u1 + p.rusu[j] * (1.0 - u1));
      gp -= k1 * soft_relu_d(a_, eps);
      a_ = pj - p1 - dt1 * (p.rd[j] * u1 + p.rdsd[j] * (1.0 - u1));
      gp += k1 * soft_relu_d(a_, eps);
    }
    w.gdev[0 * TG + e] = gp;
    w.gdev[1 * TG + e] = gq;
    w.gdev[2 * TG + e] = gr;
    w.gdev[3 * TG + e] = gu;
    acc[0] += dev;
    acc[1] += kpen * pen;
    acc[2] += pj;
    acc[3] += rj;
  }
  block_sum<4>(acc, lds);
  // zonal reserve shortfall
  const double short_ = p.rsv_req[t] - acc[3];
  const double krs = dtt * p.c_rsv * sp.beta;
  const double drs = krs * soft_relu_d(short_, eps);
  if (drs != 0.0)
    for (int j = tid; j < G; j += kBlock) w.gdev[2 * TG + (size_t)t * G + j] -= drs;
  if (tid == 0) {
    w.tpart[a.toff.dev + t] = acc[0];
    w.tpart[a.toff.pen + t] = acc[1];
    w.tpart[a.toff.rsv + t] = krs * soft_relu(short_, eps);
  }
  // uniform-slack DC injections, written transposed for the MFMA A operand
  const double mean = (acc[2] - p.sum_load[t]) / (double)N;
  for (int i = tid; i < p.N4; i += kBlock) {
    double v = 0.0;
    if (i < N) {
      double s = 0.0;
      for (int g = p.gptr[i]; g < p.gptr[i + 1]; ++g) s += xP[(size_t)t * G + p.glist[g]];
      v = (s - p.load_p[(size_t)t * N + i]) - mean;
    }
    w.pbarT[(size_t)i * p.Tp + t] = v;
  }
  // zero the padding read by later stages
  for (int l = p.L + tid; l < p.Lp; l += kBlock) w.q2[(size_t)t * p.Lp + l] = 0.0;
  for (int k = p.K + tid; k < p.Kp; k += kBlock) w.Fk[(size_t)t * p.Kp + k] = 0.0;
  if (t == 0) {
    const int padc = p.Tp - T;
    for (int e = tid; e < p.N4 * padc; e += kBlock) {
      const int i = e / padc, c = T + e % padc;
      w.pbarT[(size_t)i * p.Tp + c] = 0.0;
    }
    for (int e = tid; e < p.Lp * padc; e += kBlock) {
      const int l = e / padc, c = T + e % padc;
      w.gfT[(size_t)l * p.Tp + c] = 0.0;
    }
  }
}

__global__ __launch_bounds__(kBlock) void k_forward(EvalArgs a) {
  __shared__ double lds[4 * kBlock];
  StepParams sp;
  resolve_params(a, sp);
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    double* pb = a.w.params;
    pb[PB_EPS] = sp.eps;
    pb[PB_BETA] = sp.beta;
    pb[PB_RHO] = sp.rho_s;
    for (int c = 0; c < QG_NCLASS; ++c) pb[PB_ALPHA + c] = sp.alpha[c];
    pb[PB_BC1] = sp.bc1;
    pb[PB_BC2] = sp.bc2;
  }
  if ((int)blockIdx.x < a.nb_br)
    branch_forward(a, sp, lds);
  else
    period_block(a, sp, blockIdx.x - a.nb_br, lds);
}

// ---------------------------------------------------------------------------
// K2: bus balance + base-case DC flows

// LDS of a kernel that runs both segmented sums and an MFMA slab: the slab
// keeps four wavefronts x up to 4 row tiles x 256 partial results.
constexpr int kSlabLds = 4 * 4 * 256;
static_assert(kSlabLds >= 2 * kSegChunk + 8 * kBlock, "LDS carve");

__global__ __launch_bounds__(kBlock) void k_balance_flow(EvalArgs a) {
  __shared__ double smem[kSlabLds];
  const DevProblem& p = a.p;
  const DevWork& w = a.w;
  const int tid = threadIdx.x;
  if ((int)blockIdx.x < a.nb_bus) {
    const int t = blockIdx.x / a.bus_chunks;
    const int c = blockIdx.x - t * a.bus_chunks;
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
      w.lamp[ti] = kb * p.c_p * soft_abs_d(dp, eps);
      w.lamq[ti] = kb * p.c_q * soft_abs_d(dq, eps);
      part[0] = kb * (p.c_p * sqrt(dp * dp + eps * eps) + p.c_q * sqrt(dq * dq + eps * eps));
    }
    block_sum<1>(part, smem);
    if (tid == 0) w.tpart[a.toff.bal + blockIdx.x] = part[0];
    return;
  }
  // F[t][l] = sum_i Pbar[t][i] ISF[l][i]; also the outaged branches' flows
  const int slab = blockIdx.x - a.nb_bus;
  const int n0 = slab * 16;
  double* F = w.F;
  double* Fk = w.Fk;
  const int T = p.T, Lp = p.Lp, Kp = p.Kp;
  const int* kof = p.kof;
  auto epi = [=](int row, int col, double v) {
    if (row < T) {
      F[(size_t)row * Lp + col] = v;
      const int k = kof[col];
      if (k >= 0) Fk[(size_t)row * Kp + k] = v;
    }
  };
  mfma_slab_dispatch(p.Tp / 16, w.pbarT, p.Tp, p.isft, Lp, p.N4, n0, smem, epi);
}

// ---------------------------------------------------------------------------
// K3: contingency map-reduce over (t, l, k).
//
// A wavefront owns 64 contingencies (one per lane) and BL consecutive
// branches; its BL outage factors stay in registers for all T periods.  For
// each (t, l) every lane forms the post-outage flow P = F_tl + LODF_lk F_tk
// and tests P^2 + qmax2_tl > s_ctg^2.  Only when some lane of the wavefront
// is overloaded does it compute the soft-ReLU, its derivative and the
// wavefront sums over k (R: d/dF_tl, Q: d/dqmax2_tl); z_tk and S_tk (the
// derivative through F_tk) accumulate in the lane over l.  The outaged branch
// itself and the padding carry a NaN factor, so they never test overloaded.
// Blocks stack WL wavefronts along l; their z and S are summed in LDS.

template <int BL>
__global__ __launch_bounds__(512) void k_ctg_main(EvalArgs a) {
  __shared__ double zsh[2][8][64];
  __shared__ double ssh[2][8][64];
  const DevProblem& p = a.p;
  const DevWork& w = a.w;
  const int lane = threadIdx.x & 63;
  const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int WL = blockDim.x >> 6;
  const int lb = blockIdx.x, kb = blockIdx.y;
  const int lbase = __builtin_amdgcn_readfirstlane(lb * BL * WL + wv * BL);
  const bool on = lbase < p.Lp;
  const int k = kb * 64 + lane;
  const int T = p.T, Lp = p.Lp, Kp = p.Kp;
  const double eps = w.params[PB_EPS], beta = w.params[PB_BETA];
  const double eps2 = eps * eps;
  double lod[BL], smx[BL], smx2[BL];
  if (on) {
#pragma unroll
    for (int j = 0; j < BL; ++j) {
      lod[j] = p.lodf[(size_t)(lbase + j) * Kp + k];
      smx[j] = p.ctg_smax[lbase + j];
      smx2[j] = p.ctg_smax2[lbase + j];
    }
  }
  for (int t = 0; t < T; ++t) {
    double zacc = 0.0, sacc = 0.0, racc = 0.0, qacc = 0.0;
    if (on) {
      const double kt = p.dt[t] * p.c_s * beta;
      const double fk = w.Fk[(size_t)t * Kp + k];
      const double* Ft = w.F + (size_t)t * Lp + lbase;
      const double* Qt = w.q2 + (size_t)t * Lp + lbase;
#pragma unroll
      for (int j = 0; j < BL; ++j) {
        const double P = fma(lod[j], fk, Ft[j]);
        const double s2 = fma(P, P, Qt[j]);
        const bool over = s2 > smx2[j];
        if (__builtin_amdgcn_ballot_w64(over)) {
          double dP = 0.0, dq = 0.0;
          if (over) {
            const double s = sqrt(s2);
            const double em = fmax(s - smx[j], 0.0);
            const double sig = sqrt(em * em + eps2);
            if (sig > 0.0) {
              zacc += em * em / (sig + eps);
              const double gs = kt * em / sig;
              const double inv_s = 1.0 / s;
              dP = gs * P * inv_s;
              dq = 0.5 * gs * inv_s;
              sacc += lod[j] * dP;
            }
          }
          const double rs = wave_sum(dP);
          const double qs = wave_sum(dq);
          if (lane == j) { racc = rs; qacc = qs; }
        }
      }
      if (lane < BL) {
        const size_t o = ((size_t)kb * T + t) * Lp + lbase + lane;
        w.rpart[o] = racc;
        w.qpart[o] = qacc;
      }
    }
    const int par = t & 1;
    zsh[par][wv][lane] = zacc;
    ssh[par][wv][lane] = sacc;
    __syncthreads();
    if (wv == 0) {
      double z = 0.0, s = 0.0;
      for (int q = 0; q < WL; ++q) { z += zsh[par][q][lane]; s += ssh[par][q][lane]; }
      const size_t o = ((size_t)lb * T + t) * Kp + k;
      w.zpart[o] = z;
      w.spart[o] = s;
    }
  }
}

// ---------------------------------------------------------------------------
// K4: per-period aggregation over contingencies (worst + mean, Table 1 rows),
// the worst contingency's own column, and dL/dF, dL/dqmax2.

__global__ __launch_bounds__(kBlock) void k_ctg_finalize(EvalArgs a) {
  __shared__ double sv[kBlock];
  __shared__ int si[kBlock];
  __shared__ double red[kBlock];
  const DevProblem& p = a.p;
  const DevWork& w = a.w;
  const int t = blockIdx.x, tid = threadIdx.x;
  const int T = p.T, L = p.L, K = p.K, Lp = p.Lp, Kp = p.Kp, Tp = p.Tp;
  const double eps = w.params[PB_EPS], beta = w.params[PB_BETA];
  const double kt = p.dt[t] * p.c_s * beta;
  if (K == 0) {
    for (int l = tid; l < Lp; l += kBlock) {
      w.gfT[(size_t)l * Tp + t] = 0.0;
      w.qtot[(size_t)t * Lp + l] = 0.0;
    }
    if (tid == 0) { w.tpart[a.toff.cmax + t] = 0.0; w.tpart[a.toff.cmean + t] = 0.0; }
    return;
  }
  const double floor_ = (double)(L - 1) * eps;
  const double invK = 1.0 / (double)K;
  double best = -DBL_MAX;
  int bi = INT_MAX;
  double zs_local[1] = {0.0};
  for (int k = tid; k < K; k += kBlock) {
    double zs = 0.0, ss = 0.0;
    for (int q = 0; q < a.nLb; ++q) {
      const size_t o = ((size_t)q * T + t) * Kp + k;
      zs += w.zpart[o];
      ss += w.spart[o];
    }
    const double z = kt * (floor_ + zs);
    w.zval[(size_t)t * Kp + k] = z;
    w.smean[(size_t)t * Kp + k] = ss * invK;
    if (z > best) { best = z; bi = k; }
    zs_local[0] += z;
  }
  sv[tid] = best;
  si[tid] = bi;
  __syncthreads();
  for (int s = kBlock / 2; s > 0; s >>= 1) {
    if (tid < s) {
      const double v2 = sv[tid + s];
      const int i2 = si[tid + s];
      if (v2 > sv[tid] || (v2 == sv[tid] && i2 < si[tid])) { sv[tid] = v2; si[tid] = i2; }
    }
    __syncthreads();
  }
  // a NaN penalty never wins a comparison; fall back to contingency 0 so that
  // every index below stays in range
  const int kstar = si[0] < K ? si[0] : 0;
  const double zmax = sv[0];
  block_sum<1>(zs_local, red);
  if (tid == 0) {
    w.tpart[a.toff.cmax + t] = zmax;
    w.tpart[a.toff.cmean + t] = zs_local[0] * invK;
  }
  const double fks = w.Fk[(size_t)t * Kp + kstar];
  const int bks = p.brk[kstar];
  double sacc[1] = {0.0};
  for (int l = tid; l < Lp; l += kBlock) {
    double r = 0.0, q = 0.0;
    if (l < L) {
      for (int kb = 0; kb < a.nKb; ++kb) {
        const size_t o = ((size_t)kb * T + t) * Lp + l;
        r += w.rpart[o];
        q += w.qpart[o];
      }
      r *= invK;
      q *= invK;
      if (l != bks) {
        const double lo = p.lodf[(size_t)l * Kp + kstar];
        const double P = fma(lo, fks, w.F[(size_t)t * Lp + l]);
        const double s2 = fma(P, P, w.q2[(size_t)t * Lp + l]);
        if (s2 > p.ctg_smax2[l]) {
          const double s = sqrt(s2);
          const double em = fmax(s - p.ctg_smax[l], 0.0);
          const double sig = sqrt(em * em + eps * eps);
          if (sig > 0.0) {
            const double gs = kt * em / sig;
            const double dP = gs * P / s;
            r += dP;
            q += 0.5 * gs / s;
            sacc[0] += lo * dP;
          }
        }
      }
      const int kk = p.kof[l];
      if (kk >= 0) r += w.smean[(size_t)t * Kp + kk];
    }
    w.gfT[(size_t)l * Tp + t] = r;
    w.qtot[(size_t)t * Lp + l] = q;
  }
  block_sum<1>(sacc, red);
  if (tid == 0) w.gfT[(size_t)bks * Tp + t] += sacc[0];
}

// ---------------------------------------------------------------------------
// K5: adjoint DC product + branch reverse

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

__global__ __launch_bounds__(kBlock) void k_adjoint(EvalArgs a) {
  __shared__ double smem[kSlabLds];
  const DevProblem& p = a.p;
  const int nslab = p.Np / 16;
  if ((int)blockIdx.x < nslab) {
    const int n0 = blockIdx.x * 16;
    double* gpb = a.w.gpb;
    const int T = p.T, Np = p.Np;
    auto epi = [=](int row, int col, double v) {
      if (row < T) gpb[(size_t)row * Np + col] = v;
    };
    mfma_slab_dispatch(p.Tp / 16, a.w.gfT, p.Tp, p.isf, Np, p.Lp, n0, smem, epi);
    return;
  }
  branch_reverse(a, blockIdx.x - nslab);
}

// ---------------------------------------------------------------------------
// K6: bus reduce, generator assembly, gradient or fused Adam, terms

struct AdamCtx {
  double b1, b2, eps, bc1, bc2;
  int eps_num;
};

__device__ __forceinline__ void adam_entry(double* x, double* m, double* v, size_t e, double g,
                                           double lr, double lo, double hi, const AdamCtx& c) {
  const double mm = c.b1 * m[e] + (1.0 - c.b1) * g;
  const double vv = c.b2 * v[e] + (1.0 - c.b2) * g * g;
  m[e] = mm;
  v[e] = vv;
  const double mh = mm / c.bc1;
  const double vh = vv / c.bc2;
  const double num = c.eps_num ? mh + c.eps : mh;
  double xn = x[e] - lr * num / (sqrt(vh) + c.eps);
  xn = fmin(fmax(xn, lo), hi);
  x[e] = xn;
}

__global__ __launch_bounds__(kBlock) void k_final(EvalArgs a) {
  __shared__ double smem[2 * kSegChunk + 8 * kBlock];
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
  if ((int)blockIdx.x < a.nb_bus) {
    const int t = blockIdx.x / a.bus_chunks;
    const int c = blockIdx.x - t * a.bus_chunks;
    const int i0 = c * kBlock;
    const int nbus = min(kBlock, N - i0);
    const double* src[2] = {w.epGV + (size_t)t * p.twoL, w.epGT + (size_t)t * p.twoL};
    double gsum[2];
    bus_segsum<2>(src, p.bptr, i0, nbus, smem, gsum);
    if (tid < nbus) {
      const int i = i0 + tid;
      const size_t ev = (size_t)t * N + i, et = (size_t)T * N + ev;
      if (a.fuse_adam) {
        adam_entry(xm, a.m, a.v, ev, gsum[0], alpha[QG_C_V], p.vmin[i], p.vmax[i], ac);
        adam_entry(xm, a.m, a.v, et, gsum[1], alpha[QG_C_TH], -DBL_MAX, DBL_MAX, ac);
      } else if (a.grad) {
        a.grad[ev] = gsum[0];
        a.grad[et] = gsum[1];
      }
    }
    return;
  }
  const int gb = blockIdx.x - a.nb_bus;
  if (gb < T) {
    const int t = gb;
    double s[1] = {0.0};
    for (int i = tid; i < N; i += kBlock) s[0] += w.gpb[(size_t)t * p.Np + i];
    block_sum<1>(s, smem);
    const double meanG = s[0] / (double)N;
    const size_t TG = (size_t)T * G;
    const size_t base = 2 * (size_t)T * N;
    for (int j = tid; j < G; j += kBlock) {
      const size_t e = (size_t)t * G + j;
      const int bus = p.gen_bus[j];
      const size_t tb = (size_t)t * N + bus;
      const double gp = w.gdev[e] - w.lamp[tb] + (w.gpb[(size_t)t * p.Np + bus] - meanG);
      const double gq = w.gdev[TG + e] - w.lamq[tb];
      const double gr = w.gdev[2 * TG + e];
      const double gu = w.gdev[3 * TG + e];
      if (a.fuse_adam) {
        adam_entry(xm, a.m, a.v, base + e, gp, alpha[QG_C_P], 0.0, p.pmax[j], ac);
        adam_entry(xm, a.m, a.v, base + TG + e, gq, alpha[QG_C_Q], p.qmin[j], p.qmax[j], ac);
        adam_entry(xm, a.m, a.v, base + 2 * TG + e, gr, alpha[QG_C_R], 0.0, p.rmax[j], ac);
        adam_entry(xm, a.m, a.v, base + 3 * TG + e, gu, alpha[QG_C_U], 0.0, 1.0, ac);
      } else if (a.grad) {
        a.grad[base + e] = gp;
        a.grad[base + TG + e] = gq;
        a.grad[base + 2 * TG + e] = gr;
        a.grad[base + 3 * TG + e] = gu;
      }
    }
    return;
  }
  // terms: deterministic sums of the partials
  const TermOffsets& to = a.toff;
  double v[8] = {0, 0, 0, 0, 0, 0, 0, 0};
  for (int q = tid; q < a.nb_br; q += kBlock) { v[2] += w.tpart[to.br + q]; v[3] += w.tpart[to.ang + q]; }
  for (int q = tid; q < T; q += kBlock) {
    v[0] += w.tpart[to.dev + q];
    v[4] += w.tpart[to.pen + q];
    v[5] += w.tpart[to.rsv + q];
    v[6] += w.tpart[to.cmax + q];
    v[7] += w.tpart[to.cmean + q];
  }
  for (int q = tid; q < a.nb_bus; q += kBlock) v[1] += w.tpart[to.bal + q];
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

__global__ void k_set_step(int64_t* step, int64_t value) {
  if (threadIdx.x == 0 && blockIdx.x == 0) step[0] = value;
}

__global__ __launch_bounds__(kBlock) void k_check_finite(const double* x, size_t n, int* flag) {
  const size_t e = (size_t)blockIdx.x * kBlock + threadIdx.x;
  if (e < n && !isfinite(x[e])) flag[0] = 1;
}

// ---------------------------------------------------------------------------
// launchers

int launch_eval(const Problem* pr, const DevWork& w, const double* x, double* grad,
                double* terms_out, const EvalMode& mode, int fuse_adam, double* m, double* v,
                void* stream, void** events) {
  hipStream_t s = static_cast<hipStream_t>(stream);
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
  a.nLb = pr->nLb;
  a.nKb = pr->nKb;
  a.toff = pr->toff;
  auto rec = [&](int i) {
    if (events) (void)hipEventRecord(static_cast<hipEvent_t>(events[i]), s);
  };
  rec(0);
  hipLaunchKernelGGL(k_forward, dim3(pr->nb_br + pr->T), dim3(kBlock), 0, s, a);
  rec(1);
  hipLaunchKernelGGL(k_balance_flow, dim3(pr->nb_bus + pr->Lp / 16), dim3(kBlock), 0, s, a);
  rec(2);
  if (pr->K > 0) {
    const dim3 grid(pr->nLb, pr->nKb), block(64 * pr->tile.wl);
    switch (pr->tile.bl) {
      case 8: hipLaunchKernelGGL(k_ctg_main<8>, grid, block, 0, s, a); break;
      case 16: hipLaunchKernelGGL(k_ctg_main<16>, grid, block, 0, s, a); break;
      default: hipLaunchKernelGGL(k_ctg_main<32>, grid, block, 0, s, a); break;
    }
  }
  rec(3);
  hipLaunchKernelGGL(k_ctg_finalize, dim3(pr->T), dim3(kBlock), 0, s, a);
  rec(4);
  hipLaunchKernelGGL(k_adjoint, dim3(pr->Np / 16 + pr->nb_br), dim3(kBlock), 0, s, a);
  rec(5);
  hipLaunchKernelGGL(k_final, dim3(pr->nb_bus + pr->T + 1), dim3(kBlock), 0, s, a);
  rec(6);
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
  hipLaunchKernelGGL(k_set_step, dim3(1), dim3(64), 0, static_cast<hipStream_t>(stream),
                     w.step, value);
  return (int)hipGetLastError();
}

int launch_check_finite(const Problem* pr, const double* x, int* flag, void* stream) {
  const int nb = (int)((pr->n_x + kBlock - 1) / kBlock);
  hipLaunchKernelGGL(k_check_finite, dim3(nb), dim3(kBlock), 0,
                     static_cast<hipStream_t>(stream), x, (size_t)pr->n_x, flag);
  return (int)hipGetLastError();
}

}  // namespace qg
