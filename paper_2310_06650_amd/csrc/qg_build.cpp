// Host side of problem construction: validation, topology, the FP64 factor of
// the reduced susceptance matrix, injection shift factors, line outage
// distribution factors and the constant-arena image.
//
// Section II-E of the paper evaluates each contingency by a base-case solve of
// the reduced DC system (eq. (Yb_solve)) followed by a rank-1 correction
// (eq. (rank_correct)).  Here the reduced matrix is factored once per grid
// (Cholesky, FP64) and its inverse is applied to unit injections to give the
// injection shift factors ISF = diag(y) Ehat Yhat^{-1}; the rank-1 correction,
// mapped from angles to flows, is the outage factor
// LODF[l][k] = PTDF[l][k] / (1 - PTDF[k][k]),
// PTDF[l][k] = ISF[l][from(k)] - ISF[l][to(k)].
#include <algorithm>
#include <cmath>
#include <cstring>
#include <limits>
#include <thread>

#include "qg_internal.h"

namespace qg {

namespace {

thread_local std::string g_err;

template <class F>
void parallel_for(int n, F&& f) {
  unsigned hw = std::thread::hardware_concurrency();
  int nt = (int)std::max(1u, std::min(hw ? hw : 1u, 32u));
  if (n < 64 || nt == 1) {
    for (int i = 0; i < n; ++i) f(i);
    return;
  }
  std::vector<std::thread> th;
  th.reserve(nt);
  for (int w = 0; w < nt; ++w) {
    th.emplace_back([&, w] {
      for (int i = w; i < n; i += nt) f(i);  // interleaved for balance
    });
  }
  for (auto& t : th) t.join();
}

bool finite(double v) { return std::isfinite(v); }

// Bridges by Tarjan's low-link on an iterative DFS (edge ids distinguish
// parallel branches).  Returns false if the graph is disconnected.
bool find_bridges(int N, int L, const int32_t* fr, const int32_t* to,
                  std::vector<char>* bridge) {
  std::vector<int> deg(N + 1, 0);
  for (int l = 0; l < L; ++l) { deg[fr[l] + 1]++; deg[to[l] + 1]++; }
  for (int i = 0; i < N; ++i) deg[i + 1] += deg[i];
  std::vector<int> adj_v(2 * L), adj_e(2 * L), pos(deg.begin(), deg.end() - 1);
  for (int l = 0; l < L; ++l) {
    adj_v[pos[fr[l]]] = to[l]; adj_e[pos[fr[l]]++] = l;
    adj_v[pos[to[l]]] = fr[l]; adj_e[pos[to[l]]++] = l;
  }
  std::vector<int> disc(N, -1), low(N, 0), it(N, 0), pe(N, -1);
  bridge->assign(L, 0);
  int timer = 0;
  std::vector<int> st;
  st.push_back(0);
  disc[0] = low[0] = timer++;
  it[0] = deg[0];
  while (!st.empty()) {
    int u = st.back();
    if (it[u] < deg[u + 1]) {
      int k = it[u]++;
      int v = adj_v[k], e = adj_e[k];
      if (e == pe[u]) continue;
      if (disc[v] < 0) {
        disc[v] = low[v] = timer++;
        pe[v] = e;
        it[v] = deg[v];
        st.push_back(v);
      } else {
        low[u] = std::min(low[u], disc[v]);
      }
    } else {
      st.pop_back();
      if (!st.empty()) {
        int p = st.back();
        low[p] = std::min(low[p], low[u]);
        if (low[u] > disc[p]) (*bridge)[pe[u]] = 1;
      }
    }
  }
  return timer == N;
}

// Byte layout of the constant arena.  The same walk gives the size (for
// qg_problem_sizes) and the offsets (for the image).
constexpr int kNConst = 47;

// FP32 -> BF16 with round to nearest even; NaN stays a (quiet) NaN.
uint16_t to_bf16(float f) {
  uint32_t u;
  std::memcpy(&u, &f, 4);
  if ((u & 0x7f800000u) == 0x7f800000u && (u & 0x007fffffu)) return (uint16_t)((u >> 16) | 0x40u);
  const uint32_t r = u + 0x7fffu + ((u >> 16) & 1u);
  return (uint16_t)(r >> 16);
}

struct ConstLayout {
  size_t off[kNConst];
  size_t total;
};

ConstLayout const_layout(const Problem& p) {
  const size_t I = sizeof(int32_t), D = sizeof(double);
  const size_t N = p.N, L = p.L, G = p.G, T = p.T, M = p.M;
  const size_t cnt[kNConst] = {
      L * I, L * I, L * I, L * I,                 // from, to, slot_fr, slot_to
      L * D, L * D, L * D, L * D,                 // g, b, bh, smax
      (size_t)p.Lp * D, (size_t)p.Lp * D,         // ctg_smax, ctg_smax2
      (size_t)p.Lp * I, (size_t)p.Kp * I,         // kof, brk
      (N + 1) * I, (N + 1) * I, G * I,            // bptr, gptr, glist
      N * D, N * D,                               // vmin, vmax
      G * I,                                      // gen_bus
      G * D, G * D, G * D, G * D, G * D, G * D, G * D, G * D, G * D, G * D, G * D,
      G * D, G * D, G * D, G * D,                 // con csu csd cr
      G * M * D, G * M * D, G * M * D,            // seg_cost, seg_size, pcum
      T * N * D, T * N * D,                       // load_p, load_q
      T * D, T * D, T * D,                        // dt, rsv_req, sum_load
      (size_t)p.G4 * p.Lp * D,                    // isf_gT
      (size_t)p.Lp * p.G16 * D,                   // isf_ga
      (size_t)p.Lp * p.Kp * lodf_elem_bytes(lodf_kind_of(p.flags)),  // lodf (FP64/FP32/BF16)
      T * (size_t)p.Lp * D,                       // cload
      (size_t)p.Lp * D,                           // rsum
      (size_t)(p.Lp / 4) * (p.Kp / 64) * D};      // lmaxh
  ConstLayout c;
  size_t o = 0;
  for (int i = 0; i < kNConst; ++i) {
    o = (size_t)round_up((int64_t)o, kAlign);
    c.off[i] = o;
    o += cnt[i];
  }
  c.total = (size_t)round_up((int64_t)o, kAlign);
  return c;
}

struct WorkLayout {
  size_t off[40];
  size_t total;
};

WorkLayout work_layout(const Problem& p) {
  const size_t D = sizeof(double);
  const size_t T = p.T, L = p.L, N = p.N, G = p.G;
  const size_t twoL = 2 * L;
  const size_t nterm = (size_t)p.toff.total;
  const size_t cnt[] = {
      kParams * D, 8,                                   // params, step
      (size_t)kSchedCap * kSchedStride * D,             // sched
      T * twoL * D, T * twoL * D,                       // epP, epQ
      9 * T * L * D,                                    // bco
      T * p.Lp * D,                                     // q2
      T * p.Lp * D, T * p.Kp * D,                       // F, Fk
      T * N * D, T * N * D,                             // lamp, lamq
      4 * T * G * D,                                    // gdev
      (size_t)p.nLb_max * T * p.Kp * D, (size_t)p.nLb_max * T * p.Kp * D,
      (size_t)p.nKb_max * T * p.Lp * D, (size_t)p.nKb_max * T * p.Lp * D,
      T * p.Kp * D, T * p.Kp * D,                       // smean, zval
      (size_t)p.Lp * p.Tp * D,                          // gfT
      T * p.Lp * D,                                     // qtot
      (size_t)p.nsplit * T * p.G16 * D,                 // gpdc
      T * twoL * D, T * twoL * D,                       // epGV, epGT
      nterm * D,                                        // tpart
      QG_NTERMS * D,                                    // terms
      T * D,                                            // drs
      T * (size_t)p.nKc * D, T * (size_t)p.nKc * D,     // zmaxp, zargp
      T * (size_t)p.nKc * D,                            // zsump
      T * D,                                            // kstar
      T * (size_t)p.nLc * D,                            // smaxp
      T * G * D, T * G * D,                             // lamg, lamqg
      T * (size_t)p.G16 * D,                            // isfk
      T * p.Lp * D,                                     // thr
      T * (size_t)p.nKb_max * p.nLb_max,                // zflag
      T * (size_t)(p.Lp / 8) * rflag_stride(p.nKb_max),   // rflag
      kSchedStride * D,                                 // snext
      ((size_t)(p.Lp / 8 + 1) * T + 8) * 16 * D};       // fh
  WorkLayout w;
  const int n = (int)(sizeof(cnt) / sizeof(cnt[0]));
  size_t o = 0;
  for (int i = 0; i < n; ++i) {
    o = (size_t)round_up((int64_t)o, kAlign);
    w.off[i] = o;
    o += cnt[i];
  }
  w.total = (size_t)round_up((int64_t)o, kAlign);
  return w;
}

}  // namespace

int default_ctg_tc(const Problem& p, int wl) {
  // periods per block of the contingency map-reduce.  Short chunks give the
  // chip more blocks and shorter per-block tails, but every chunk re-reads
  // the outage factors: take 4 periods while the re-reads stay within a
  // 64 MB budget per step, else the longest chunk (8 periods).
  const double lodf_bytes = (double)p.Lp * p.Kp * lodf_elem_bytes(lodf_kind_of(p.flags));
  const int chunks4 = (p.T + 3) / 4;
  int tc = (lodf_bytes * chunks4 <= 64.0 * (1 << 20)) ? 4 : kCtgMaxTc;
  tc = std::min(tc, ctg_tc_cap(wl));
  return std::max(1, std::min(tc, p.T));
}

int default_ctg_lt(const Problem& p, const CtgTile& t) {
  // branch tiles per block: more tiles per block amortise the block's
  // prologue and epilogue and divide the (t, k) partial sums of z and S,
  // while at least 2048 blocks remain to fill the chip
  const int span = t.split ? 8 : t.bl * t.wl;
  const int nl1 = (p.Lp + span - 1) / span;
  const int tspan = t.split ? t.wl * t.tc : t.tc;
  const int ntc = (p.T + tspan - 1) / tspan;
  int lt = t.split ? 2 : 1;
  while (lt < 8) {
    const int nl = (nl1 + 2 * lt - 1) / (2 * lt);
    if ((int64_t)nl * p.nKb * ntc < 2048) break;
    lt *= 2;
  }
  return lt;
}

CtgTile default_ctg_tile(const Problem& p) {
  // period-split blocks: below 32 periods four, three or two wavefronts of
  // two periods, whichever leaves the fewest padded periods in the last
  // period chunk (ties to more wavefronts); from 32 periods one wavefront
  // of four.  Branch tiles per block by the rule of default_ctg_lt.
  // Measured as whole graph-replayed steps: against the best branch-stacked
  // tile 4.8 % faster at 18 periods, 1.6x at 48; at 18 periods (617 buses)
  // three wavefronts run 31.1k steps/s against 30.8k for four (whose last
  // chunk holds 2 of 8 periods); at 48 periods (2000 buses) one wavefront
  // runs 10.15k against 9.99k for two and 9.72k for four.
  int wl = 1, tc = 4;
  if (p.T < 32) {
    tc = 2;
    int fewest = 1 << 30;
    for (int w = 4; w >= 2; --w) {
      const int span = w * tc, pad = (p.T + span - 1) / span * span - p.T;
      if (pad < fewest) {
        fewest = pad;
        wl = w;
      }
    }
  }
  CtgTile t{8, wl, tc, 2};
  t.split = 1;
  t.lt = default_ctg_lt(p, t);
  return t;
}

void apply_ctg_tile(Problem* p, const CtgTile& t) {
  p->tile = t;
  const int span = t.split ? 8 * t.lt : t.bl * t.wl * t.lt;
  p->nLb = (p->Lp + span - 1) / span;
}

int ctg_tc_cap(int wl) {
  // LDS of the map-reduce block: tc * 64 doubles of outaged-branch flows and
  // tc * wl * 64 each of z and S
  const int per_tc = 64 * (1 + 2 * wl) * (int)sizeof(double);
  return std::max(1, std::min(kCtgMaxTc, kCtgLdsBytes / per_tc));
}

qg_status fail(qg_status s, const std::string& msg) {
  g_err = msg;
  return s;
}

const char* last_error_text() { return g_err.c_str(); }

qg_status plan_problem(const qg_grid_desc* d, const qg_build_opts* o, Problem* p) {
  if (!d || !o || !p) return fail(QG_ERR_ARG, "null descriptor, options or output");
  const int N = d->n_bus, L = d->n_branch, G = d->n_gen, T = d->n_period, M = d->n_seg;
  if (N < 2 || L < 1 || G < 1 || T < 1 || M < 1)
    return fail(QG_ERR_ARG, "sizes must satisfy n_bus>=2, n_branch>=1, n_gen>=1, n_period>=1, n_seg>=1");
  if (T > kMaxT) return fail(QG_ERR_ARG, "n_period above 64 is not supported");
  if (N > (1 << 24) || L > (1 << 24) || G > (1 << 24))
    return fail(QG_ERR_ARG, "sizes above 2^24 are not supported");
  const void* req[] = {d->br_from, d->br_to, d->br_r, d->br_x, d->br_bch, d->br_smax,
                       d->br_smax_ctg, d->gen_bus, d->gen_pmin, d->gen_pmax, d->gen_qmin,
                       d->gen_qmax, d->gen_rmax, d->gen_ru, d->gen_rd, d->gen_ru_su,
                       d->gen_rd_sd, d->gen_p0, d->gen_u0, d->gen_c_on, d->gen_c_su,
                       d->gen_c_sd, d->gen_c_r, d->gen_seg_cost, d->gen_seg_size,
                       d->load_p, d->load_q, d->reserve_req, d->dt, d->v_min, d->v_max};
  for (const void* r : req)
    if (!r) return fail(QG_ERR_ARG, "a required descriptor array is null");
  if (o->ref_bus < 0 || o->ref_bus >= N) return fail(QG_ERR_ARG, "ref_bus out of range");
  for (int l = 0; l < L; ++l) {
    if (d->br_from[l] < 0 || d->br_from[l] >= N || d->br_to[l] < 0 || d->br_to[l] >= N)
      return fail(QG_ERR_ARG, "branch " + std::to_string(l) + " has an endpoint out of range");
    if (d->br_from[l] == d->br_to[l])
      return fail(QG_ERR_ARG, "branch " + std::to_string(l) + " is a self loop");
    if (!(d->br_x[l] > 0.0) || !(d->br_r[l] >= 0.0) || !finite(d->br_x[l]) || !finite(d->br_r[l]))
      return fail(QG_ERR_ARG, "branch " + std::to_string(l) + " needs x > 0 and r >= 0");
    if (!(d->br_smax[l] > 0.0) || !(d->br_smax_ctg[l] > 0.0) || !finite(d->br_bch[l]))
      return fail(QG_ERR_ARG, "branch " + std::to_string(l) + " needs positive ratings");
  }
  for (int j = 0; j < G; ++j) {
    if (d->gen_bus[j] < 0 || d->gen_bus[j] >= N)
      return fail(QG_ERR_ARG, "generator " + std::to_string(j) + " bus out of range");
    if (!(d->gen_pmax[j] > 0.0) || !(d->gen_pmin[j] >= 0.0) || d->gen_pmin[j] > d->gen_pmax[j] ||
        !(d->gen_qmin[j] <= d->gen_qmax[j]) || !(d->gen_rmax[j] >= 0.0) ||
        !(d->gen_u0[j] >= 0.0 && d->gen_u0[j] <= 1.0))
      return fail(QG_ERR_ARG, "generator " + std::to_string(j) + " has inconsistent limits");
    for (int m = 0; m < M; ++m)
      if (!(d->gen_seg_size[j * M + m] > 0.0) || !finite(d->gen_seg_cost[j * M + m]))
        return fail(QG_ERR_ARG, "generator " + std::to_string(j) + " has a bad cost block");
  }
  for (int t = 0; t < T; ++t)
    if (!(d->dt[t] > 0.0)) return fail(QG_ERR_ARG, "durations must be positive");
  for (int i = 0; i < N; ++i)
    if (!(d->v_min[i] <= d->v_max[i])) return fail(QG_ERR_ARG, "v_min > v_max");

  std::vector<char> bridge;
  if (!find_bridges(N, L, d->br_from, d->br_to, &bridge))
    return fail(QG_ERR_TOPOLOGY, "the grid is not connected");
  p->ctg.clear();
  if (o->ctg_mode == QG_CTG_ALL_NONBRIDGE) {
    for (int l = 0; l < L; ++l)
      if (!bridge[l]) p->ctg.push_back(l);
  } else if (o->ctg_mode == QG_CTG_LIST) {
    if (o->n_ctg < 0 || (o->n_ctg > 0 && !o->ctg_list))
      return fail(QG_ERR_ARG, "bad contingency list");
    std::vector<char> seen(L, 0);
    for (int k = 0; k < o->n_ctg; ++k) {
      int l = o->ctg_list[k];
      if (l < 0 || l >= L) return fail(QG_ERR_ARG, "contingency branch index out of range");
      if (seen[l]) return fail(QG_ERR_ARG, "duplicate contingency branch");
      seen[l] = 1;
      if (bridge[l])
        return fail(QG_ERR_TOPOLOGY, "outage of branch " + std::to_string(l) + " islands the grid");
      p->ctg.push_back(l);
    }
  } else {
    return fail(QG_ERR_ARG, "unknown ctg_mode");
  }

  p->N = N; p->L = L; p->G = G; p->T = T; p->M = M;
  p->K = (int)p->ctg.size();
  p->Lp = (int)round_up(L, 64);
  p->Kp = (int)round_up(std::max(p->K, 1), 64);
  p->G16 = (int)round_up(G, 16);
  p->G4 = (int)round_up(G, 4);
  p->Tp = (int)round_up(T, 16);
  p->n_x = 2LL * T * N + 4LL * T * G;
  if ((o->flags & QG_FLAG_CTG_FP32) && (o->flags & QG_FLAG_CTG_BF16))
    return fail(QG_ERR_ARG, "at most one contingency precision flag");
  if (o->flags & ~(uint32_t)(QG_FLAG_CHECK_FINITE | QG_FLAG_CTG_FP32 | QG_FLAG_CTG_BF16 |
                             QG_FLAG_CTG_SUM | QG_FLAG_CTG_NO_SKIP))
    return fail(QG_ERR_ARG, "unknown build flag");
  p->flags = o->flags;
  p->nb_br = (int)((int64_t(T) * L + kBlock - 1) / kBlock);
  p->bus_chunks = (N + kBlock - 1) / kBlock;
  p->nb_bus = T * p->bus_chunks;
  p->nb_gen = (int)((int64_t(T) * G + kBlock - 1) / kBlock);
  {
    // splits of the adjoint product's reduction: about one block per CU in
    // all, each with at least kAdjStepsPerBlock MFMA k-steps when there are
    // enough
    const int steps = p->Lp / 4;
    const int nslab = (int)(round_up(G, 16) / 16);
    const int most = std::max(1, (steps + kAdjStepsPerBlock - 1) / kAdjStepsPerBlock);
    p->nsplit = std::min(most, std::max(1, (256 + nslab - 1) / nslab));
  }
  p->nKc = p->Kp / kCtgLanes;
  p->nLc = (p->Lp + kBlock - 1) / kBlock;
  p->nLb_max = p->Lp / 16;
  p->nKb_max = p->Kp / kCtgLanes;
  p->nKb = p->Kp / kCtgLanes;
  const CtgTile tile = default_ctg_tile(*p);
  apply_ctg_tile(p, tile);
  TermOffsets& to = p->toff;
  int o2 = 0;
  to.br = o2; o2 += p->nb_br;
  to.ang = o2; o2 += p->nb_br;
  // device terms: one partial per period and slice of kBlock generators
  const int ndev = T * ((p->G + kBlock - 1) / kBlock);
  to.dev = o2; o2 += ndev;
  to.pen = o2; o2 += ndev;
  to.rsv = o2; o2 += T;
  to.bal = o2; o2 += p->nb_bus;
  to.cmax = o2; o2 += T;
  to.cmean = o2; o2 += T;
  to.total = o2;
  p->const_bytes = const_layout(*p).total;
  p->work_bytes = work_layout(*p).total;
  return QG_OK;
}

namespace {

// In-place lower Cholesky of the n x n row-major matrix A (blocked,
// right-looking; the trailing update runs on host threads).
bool cholesky(std::vector<double>& A, int n) {
  const int nb = 64;
  for (int k0 = 0; k0 < n; k0 += nb) {
    const int k1 = std::min(n, k0 + nb);
    // factor the diagonal block and the panel below it, column by column
    for (int j = k0; j < k1; ++j) {
      double s = A[(size_t)j * n + j];
      for (int k = k0; k < j; ++k) s -= A[(size_t)j * n + k] * A[(size_t)j * n + k];
      if (!(s > 0.0) || !std::isfinite(s)) return false;
      const double djj = std::sqrt(s);
      A[(size_t)j * n + j] = djj;
      const double inv = 1.0 / djj;
      const int rows = n - (j + 1);
      auto col = [&](int r) {
        const int i = j + 1 + r;
        double v = A[(size_t)i * n + j];
        const double* ai = &A[(size_t)i * n];
        const double* aj = &A[(size_t)j * n];
        for (int k = k0; k < j; ++k) v -= ai[k] * aj[k];
        A[(size_t)i * n + j] = v * inv;
      };
      if (rows > 4096) parallel_for(rows, col); else for (int r = 0; r < rows; ++r) col(r);
    }
    // trailing update A[i][j] -= sum_k L[i][k] L[j][k], i >= j >= k1, k in panel
    const int rem = n - k1;
    if (rem <= 0) continue;
    parallel_for(rem, [&](int r) {
      const int i = k1 + r;
      const double* li = &A[(size_t)i * n + k0];
      for (int j = k1; j <= i; ++j) {
        const double* lj = &A[(size_t)j * n + k0];
        double s = 0.0;
        for (int k = 0; k < k1 - k0; ++k) s += li[k] * lj[k];
        A[(size_t)i * n + j] -= s;
      }
    });
  }
  return true;
}

// Inverse of the reduced matrix from its Cholesky factor: W = Lc^{-1}
// (stored transposed, WT[c][i] = W[i][c]), then Yinv = W^T W.
void inverse_from_cholesky(const std::vector<double>& Lc, int n, std::vector<double>* Yinv) {
  std::vector<double> WT((size_t)n * n, 0.0);
  parallel_for(n, [&](int c) {
    double* w = &WT[(size_t)c * n];
    w[c] = 1.0 / Lc[(size_t)c * n + c];
    for (int i = c + 1; i < n; ++i) {
      const double* li = &Lc[(size_t)i * n];
      double s = 0.0;
      for (int k = c; k < i; ++k) s += li[k] * w[k];
      w[i] = -s / li[i];
    }
  });
  Yinv->assign((size_t)n * n, 0.0);
  parallel_for(n, [&](int a) {
    const double* wa = &WT[(size_t)a * n];
    for (int b = a; b < n; ++b) {
      const double* wb = &WT[(size_t)b * n];
      double s = 0.0;
      for (int k = b; k < n; ++k) s += wa[k] * wb[k];
      (*Yinv)[(size_t)a * n + b] = s;
      (*Yinv)[(size_t)b * n + a] = s;
    }
  });
}

template <class T>
void put(std::vector<unsigned char>& img, size_t off, const T* src, size_t n) {
  std::memcpy(img.data() + off, src, n * sizeof(T));
}

}  // namespace

qg_status build_arena(const qg_grid_desc* d, const qg_build_opts* o, Problem* p,
                      HostBuild* hb) {
  (void)o;
  const int N = p->N, L = p->L, G = p->G, T = p->T, M = p->M, K = p->K;
  const int Lp = p->Lp, Kp = p->Kp, G16 = p->G16, G4 = p->G4;
  const int Np = (int)round_up(N, 16);  // row stride of the host ISF
  const ConstLayout cl = const_layout(*p);
  hb->const_bytes = cl.total;
  hb->image.assign(cl.total, 0);
  auto& img = hb->image;

  // ---- branches
  std::vector<double> g(L), b(L), bh(L), y(L);
  for (int l = 0; l < L; ++l) {
    const double r = d->br_r[l], x = d->br_x[l], z2 = r * r + x * x;
    g[l] = r / z2;
    b[l] = -x / z2;
    bh[l] = 0.5 * d->br_bch[l];
    y[l] = x / z2;  // -b: series susceptance of the DC flow model
  }
  // endpoint slots sorted by bus, ascending branch index within a bus
  std::vector<int32_t> bptr(N + 1, 0), slot_fr(L), slot_to(L);
  for (int l = 0; l < L; ++l) { bptr[d->br_from[l] + 1]++; bptr[d->br_to[l] + 1]++; }
  for (int i = 0; i < N; ++i) bptr[i + 1] += bptr[i];
  {
    std::vector<int32_t> pos(bptr.begin(), bptr.end() - 1);
    for (int l = 0; l < L; ++l) {
      slot_fr[l] = pos[d->br_from[l]]++;
      slot_to[l] = pos[d->br_to[l]]++;
    }
  }
  std::vector<int32_t> gptr(N + 1, 0), glist(G);
  for (int j = 0; j < G; ++j) gptr[d->gen_bus[j] + 1]++;
  for (int i = 0; i < N; ++i) gptr[i + 1] += gptr[i];
  {
    std::vector<int32_t> pos(gptr.begin(), gptr.end() - 1);
    for (int j = 0; j < G; ++j) glist[pos[d->gen_bus[j]]++] = j;
  }
  std::vector<double> cs(Lp, 1.0), cs2(Lp, 1.0);
  for (int l = 0; l < L; ++l) { cs[l] = d->br_smax_ctg[l]; cs2[l] = cs[l] * cs[l]; }
  std::vector<int32_t> kof(Lp, -1), brk(Kp, 0);
  for (int k = 0; k < K; ++k) { kof[p->ctg[k]] = k; brk[k] = p->ctg[k]; }

  put(img, cl.off[0], d->br_from, L);
  put(img, cl.off[1], d->br_to, L);
  put(img, cl.off[2], slot_fr.data(), L);
  put(img, cl.off[3], slot_to.data(), L);
  put(img, cl.off[4], g.data(), L);
  put(img, cl.off[5], b.data(), L);
  put(img, cl.off[6], bh.data(), L);
  put(img, cl.off[7], d->br_smax, L);
  put(img, cl.off[8], cs.data(), Lp);
  put(img, cl.off[9], cs2.data(), Lp);
  put(img, cl.off[10], kof.data(), Lp);
  put(img, cl.off[11], brk.data(), Kp);
  put(img, cl.off[12], bptr.data(), N + 1);
  put(img, cl.off[13], gptr.data(), N + 1);
  put(img, cl.off[14], glist.data(), G);
  put(img, cl.off[15], d->v_min, N);
  put(img, cl.off[16], d->v_max, N);
  put(img, cl.off[17], d->gen_bus, G);
  const double* gen_arrays[] = {d->gen_pmin, d->gen_pmax, d->gen_qmin, d->gen_qmax,
                                d->gen_rmax, d->gen_ru, d->gen_rd, d->gen_ru_su,
                                d->gen_rd_sd, d->gen_p0, d->gen_u0, d->gen_c_on,
                                d->gen_c_su, d->gen_c_sd, d->gen_c_r};
  for (int a = 0; a < 15; ++a) put(img, cl.off[18 + a], gen_arrays[a], G);
  // cumulative block ends, summed left to right per generator
  std::vector<double> pcum((size_t)G * M);
  for (int j = 0; j < G; ++j) {
    double acc = 0.0;
    for (int m = 0; m < M; ++m) { acc += d->gen_seg_size[j * M + m]; pcum[j * M + m] = acc; }
  }
  put(img, cl.off[33], d->gen_seg_cost, (size_t)G * M);
  put(img, cl.off[34], d->gen_seg_size, (size_t)G * M);
  put(img, cl.off[35], pcum.data(), (size_t)G * M);
  put(img, cl.off[36], d->load_p, (size_t)T * N);
  put(img, cl.off[37], d->load_q, (size_t)T * N);
  put(img, cl.off[38], d->dt, T);
  put(img, cl.off[39], d->reserve_req, T);
  std::vector<double> sum_load(T, 0.0);
  double vload = 0.0;
  for (int t = 0; t < T; ++t) {
    double s = 0.0;
    for (int i = 0; i < N; ++i) s += d->load_p[(size_t)t * N + i];
    sum_load[t] = s;
    vload += d->dt[t] * d->load_value * s;
  }
  put(img, cl.off[40], sum_load.data(), T);

  // ---- reduced susceptance matrix, factor and inverse
  const int ref = o->ref_bus;
  const int n = N - 1;
  std::vector<int> red(N);
  for (int i = 0, c = 0; i < N; ++i) red[i] = (i == ref) ? -1 : c++;
  std::vector<double> Y((size_t)n * n, 0.0);
  for (int l = 0; l < L; ++l) {
    const int a = red[d->br_from[l]], c = red[d->br_to[l]];
    if (a >= 0) Y[(size_t)a * n + a] += y[l];
    if (c >= 0) Y[(size_t)c * n + c] += y[l];
    if (a >= 0 && c >= 0) {
      Y[(size_t)a * n + c] -= y[l];
      Y[(size_t)c * n + a] -= y[l];
    }
  }
  if (!cholesky(Y, n)) return fail(QG_ERR_SINGULAR, "reduced susceptance matrix is not positive definite");
  std::vector<double> Yinv;
  inverse_from_cholesky(Y, n, &Yinv);
  Y.clear();
  Y.shrink_to_fit();

  // ---- injection shift factors: ISF[l][i] = y_l (Yinv[f][i] - Yinv[t][i])
  std::vector<double> isf((size_t)L * Np, 0.0);
  parallel_for(L, [&](int l) {
    const int a = red[d->br_from[l]], c = red[d->br_to[l]];
    double* row = &isf[(size_t)l * Np];
    for (int i = 0; i < N; ++i) {
      const int ri = red[i];
      if (ri < 0) continue;
      const double va = a >= 0 ? Yinv[(size_t)a * n + ri] : 0.0;
      const double vc = c >= 0 ? Yinv[(size_t)c * n + ri] : 0.0;
      row[i] = y[l] * (va - vc);
    }
  });
  Yinv.clear();
  Yinv.shrink_to_fit();
  // ---- the ISF restricted to generator buses, its row sums and the load term.
  // With the uniform slack, F_t = ISF p_bar_t = ISF[:, bus(j)] p_t - ISF load_t
  // - mean_t ISF 1 and mean_t = (sum_j p_tj - sum_i load_ti) / N, so
  // F_tl = sum_j p_tj (ISF[l][bus(j)] - rsum_l / N) - c_tl with the per-grid
  // constant c_tl = ISF load_t - rsum_l sum_i load_ti / N; the slack-corrected
  // injection gradient (eq. (correction)) of generator j is the transpose:
  // sum_l dL/dF_tl (ISF[l][bus(j)] - rsum_l / N).
  {
    std::vector<double> rsum(Lp, 0.0);
    for (int l = 0; l < L; ++l) {
      double s = 0.0;
      for (int i = 0; i < N; ++i) s += isf[(size_t)l * Np + i];
      rsum[l] = s;
    }
    double* gT = reinterpret_cast<double*>(img.data() + cl.off[41]);   // [G4][Lp]
    double* ga = reinterpret_cast<double*>(img.data() + cl.off[42]);   // [Lp][G16]
    for (int j = 0; j < G; ++j) {
      const int bj = d->gen_bus[j];
      for (int l = 0; l < L; ++l) {
        const double v = isf[(size_t)l * Np + bj];
        gT[(size_t)j * Lp + l] = v - rsum[l] / (double)N;
        ga[(size_t)l * G16 + j] = v - rsum[l] / (double)N;
      }
    }
    put(img, cl.off[45], rsum.data(), Lp);
    (void)G4;
    p->rsum_host = rsum;
  }

  // ---- outage factors, NaN on the outaged branch itself and on padding
  {
    const int kind = lodf_kind_of(p->flags);
    std::vector<double> lo_buf;
    double* lo;
    if (kind == kLodfF64) {
      lo = reinterpret_cast<double*>(img.data() + cl.off[43]);
    } else {
      lo_buf.resize((size_t)Lp * Kp);
      lo = lo_buf.data();
    }
    const double qnan = std::numeric_limits<double>::quiet_NaN();
    std::fill(lo, lo + (size_t)Lp * Kp, qnan);
    std::vector<double> denom(K);
    for (int k = 0; k < K; ++k) {
      const int bk = p->ctg[k];
      const double pkk = isf[(size_t)bk * Np + d->br_from[bk]] - isf[(size_t)bk * Np + d->br_to[bk]];
      denom[k] = 1.0 - pkk;
      if (!(denom[k] > 1e-10))
        return fail(QG_ERR_TOPOLOGY, "outage of branch " + std::to_string(bk) +
                                         " islands the grid (1 - PTDF_kk <= 1e-10)");
    }
    parallel_for(L, [&](int l) {
      const double* row = &isf[(size_t)l * Np];
      double* out = lo + (size_t)l * Kp;
      for (int k = 0; k < K; ++k) {
        const int bk = p->ctg[k];
        if (bk == l) continue;  // stays NaN: the outaged branch carries no flow
        out[k] = (row[d->br_from[bk]] - row[d->br_to[bk]]) / denom[k];
      }
    });
    // largest |factor| of every 4-branch group over every 64-contingency
    // block (NaN entries left out), of the factors as stored (FP32 or BF16
    // rounding included): the bound of the map-reduce's skip test
    {
      double* lm = reinterpret_cast<double*>(img.data() + cl.off[46]);
      const int nkb = Kp / 64;
      auto stored = [&](double v) -> double {
        if (kind == kLodfF32) return (double)(float)v;
        if (kind == kLodfBF16) {
          const uint32_t u = (uint32_t)to_bf16((float)v) << 16;
          float f;
          std::memcpy(&f, &u, 4);
          return (double)f;
        }
        return v;
      };
      parallel_for(Lp / 4, [&](int q) {
        for (int kb = 0; kb < nkb; ++kb) {
          double m = 0.0;
          for (int l = 4 * q; l < 4 * q + 4; ++l)
            for (int k = 64 * kb; k < 64 * kb + 64; ++k) {
              const double v = std::fabs(stored(lo[(size_t)l * Kp + k]));
              if (v > m) m = v;  // false for NaN
            }
          lm[(size_t)q * nkb + kb] = m;
        }
      });
    }
    if (kind == kLodfF32) {
      float* o32 = reinterpret_cast<float*>(img.data() + cl.off[43]);
      for (size_t e = 0; e < (size_t)Lp * Kp; ++e) o32[e] = (float)lo[e];
    } else if (kind == kLodfBF16) {
      uint16_t* o16 = reinterpret_cast<uint16_t*>(img.data() + cl.off[43]);
      for (size_t e = 0; e < (size_t)Lp * Kp; ++e) o16[e] = to_bf16((float)lo[e]);
    }
  }

  // ---- host data for load updates, and the load-dependent flow constant
  p->isf_host = std::move(isf);
  p->isf_np = Np;
  p->dt_host.assign(d->dt, d->dt + T);
  p->load_value = d->load_value;
  {
    LoadBlock lb;
    load_block(p, d->load_p, &lb);
    put(img, lb.off_cload, lb.cload.data(), (size_t)T * Lp);
  }

  // ---- scalars
  DevProblem& dp = p->dp;
  dp.N = N; dp.L = L; dp.G = G; dp.T = T; dp.M = M; dp.K = K;
  dp.Lp = Lp; dp.Kp = Kp; dp.G16 = G16; dp.G4 = G4; dp.Tp = p->Tp; dp.twoL = 2 * L;
  dp.c_p = d->c_p; dp.c_q = d->c_q; dp.c_s = d->c_s; dp.c_ang = d->c_ang;
  dp.ang_max = d->ang_max; dp.c_rsv = d->c_rsv; dp.rho = d->rho; dp.vload = vload;
  return QG_OK;
}

void load_block(const Problem* p, const double* load_p, LoadBlock* out) {
  const ConstLayout cl = const_layout(*p);
  const int N = p->N, L = p->L, T = p->T, Lp = p->Lp, Np = p->isf_np;
  out->off_lp = cl.off[36];
  out->off_lq = cl.off[37];
  out->off_rsv = cl.off[39];
  out->off_sum = cl.off[40];
  out->off_cload = cl.off[44];
  out->sum_load.assign(T, 0.0);
  out->vload = 0.0;
  for (int t = 0; t < T; ++t) {
    double s = 0.0;
    for (int i = 0; i < N; ++i) s += load_p[(size_t)t * N + i];
    out->sum_load[t] = s;
    out->vload += p->dt_host[t] * p->load_value * s;
  }
  out->cload.assign((size_t)T * Lp, 0.0);
  const double* isf = p->isf_host.data();
  parallel_for(T, [&](int t) {
    const double* ld = load_p + (size_t)t * N;
    for (int l = 0; l < L; ++l) {
      const double* row = &isf[(size_t)l * Np];
      double s = 0.0;
      for (int i = 0; i < N; ++i) s += row[i] * ld[i];
      out->cload[(size_t)t * Lp + l] = s - p->rsum_host[l] * out->sum_load[t] / (double)N;
    }
  });
}

void rebase_pointers(Problem* p, void* arena) {
  const ConstLayout cl = const_layout(*p);
  unsigned char* base = static_cast<unsigned char*>(arena);
  DevProblem& dp = p->dp;
  auto I = [&](int i) { return reinterpret_cast<const int*>(base + cl.off[i]); };
  auto D = [&](int i) { return reinterpret_cast<const double*>(base + cl.off[i]); };
  dp.br_from = I(0); dp.br_to = I(1); dp.slot_fr = I(2); dp.slot_to = I(3);
  dp.br_g = D(4); dp.br_b = D(5); dp.br_bh = D(6); dp.br_smax = D(7);
  dp.ctg_smax = D(8); dp.ctg_smax2 = D(9); dp.kof = I(10); dp.brk = I(11);
  dp.bptr = I(12); dp.gptr = I(13); dp.glist = I(14); dp.vmin = D(15); dp.vmax = D(16);
  dp.gen_bus = I(17);
  dp.pmin = D(18); dp.pmax = D(19); dp.qmin = D(20); dp.qmax = D(21); dp.rmax = D(22);
  dp.ru = D(23); dp.rd = D(24); dp.rusu = D(25); dp.rdsd = D(26); dp.p0 = D(27);
  dp.u0 = D(28); dp.con = D(29); dp.csu = D(30); dp.csd = D(31); dp.cr = D(32);
  dp.seg_cost = D(33); dp.seg_size = D(34); dp.pcum = D(35);
  dp.load_p = D(36); dp.load_q = D(37); dp.dt = D(38); dp.rsv_req = D(39);
  dp.sum_load = D(40); dp.isf_gT = D(41); dp.isf_ga = D(42);
  dp.lodf_kind = lodf_kind_of(p->flags);
  dp.ctg_sum = (p->flags & QG_FLAG_CTG_SUM) ? 1 : 0;
  dp.lodf = dp.lodf_kind == kLodfF64 ? D(43) : nullptr;
  dp.lmaxh = !(p->flags & QG_FLAG_CTG_NO_SKIP) ? D(46) : nullptr;
  dp.lodf32 = dp.lodf_kind == kLodfF32 ? reinterpret_cast<const float*>(base + cl.off[43]) : nullptr;
  dp.lodf16 =
      dp.lodf_kind == kLodfBF16 ? reinterpret_cast<const uint16_t*>(base + cl.off[43]) : nullptr;
  dp.cload = D(44); dp.rsum = D(45);
  p->arena = arena;
}

DevWork carve_workspace(const Problem* p, void* ws) {
  const WorkLayout wl = work_layout(*p);
  unsigned char* base = static_cast<unsigned char*>(ws);
  auto D = [&](int i) { return reinterpret_cast<double*>(base + wl.off[i]); };
  DevWork w;
  w.params = D(0);
  w.step = reinterpret_cast<int64_t*>(base + wl.off[1]);
  w.sched = D(2);
  w.epP = D(3); w.epQ = D(4); w.bco = D(5); w.q2 = D(6);
  w.F = D(7); w.Fk = D(8); w.lamp = D(9); w.lamq = D(10); w.gdev = D(11);
  w.zpart = D(12); w.spart = D(13); w.rpart = D(14); w.qpart = D(15);
  w.smean = D(16); w.zval = D(17); w.gfT = D(18); w.qtot = D(19); w.gpdc = D(20);
  w.epGV = D(21); w.epGT = D(22); w.tpart = D(23); w.terms = D(24);
  w.drs = D(25); w.zmaxp = D(26); w.zargp = D(27); w.zsump = D(28); w.kstar = D(29);
  w.smaxp = D(30);
  w.lamg = D(31); w.lamqg = D(32); w.isfk = D(33); w.thr = D(34);
  w.zflag = base + wl.off[35];
  w.rflag = base + wl.off[36];
  w.snext = D(37);
  w.fh = D(38);
  return w;
}

// Screening buffer: act_k, act_slot, top, sel [Kp] int32; sev [Kp] double;
// key [Kp] uint64; then the gathered outage factors [Lp][cap padded to 64]
// in the problem's factor storage.  Each part 256-byte aligned.
namespace {
struct ScreenLayout {
  size_t off[7];
  size_t total;
};
ScreenLayout screen_layout(const Problem& p, int cap) {
  const size_t Kp = (size_t)p.Kp;
  const size_t ka = (size_t)round_up(cap, kCtgLanes);
  const size_t cnt[7] = {Kp * 4, Kp * 4, Kp * 4, Kp * 4, Kp * 8, Kp * 8,
                         (size_t)p.Lp * ka * lodf_elem_bytes(lodf_kind_of(p.flags))};
  ScreenLayout sl;
  size_t o = 0;
  for (int i = 0; i < 7; ++i) {
    sl.off[i] = o;
    o += (size_t)round_up((int64_t)cnt[i], kAlign);
  }
  sl.total = o;
  return sl;
}
}  // namespace

size_t screen_bytes(const Problem& p, int cap) { return screen_layout(p, cap).total; }

void carve_screen(const Problem& p, void* buf, int cap, Screen* sc) {
  const ScreenLayout sl = screen_layout(p, cap);
  unsigned char* b = static_cast<unsigned char*>(buf);
  sc->act_k = reinterpret_cast<int*>(b + sl.off[0]);
  sc->act_slot = reinterpret_cast<int*>(b + sl.off[1]);
  sc->top = reinterpret_cast<int*>(b + sl.off[2]);
  sc->sel = reinterpret_cast<int*>(b + sl.off[3]);
  sc->sev = reinterpret_cast<double*>(b + sl.off[4]);
  sc->key = reinterpret_cast<uint64_t*>(b + sl.off[5]);
  sc->lodf_act = b + sl.off[6];
  sc->bytes = sl.total;
}

}  // namespace qg
