// extern "C" entry points of qg.h: argument checks, uploads, stream handling,
// graph capture of the solve loop and error plumbing.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "qg_internal.h"

namespace qg {
const char* last_error_text();
}

struct qg_problem {
  qg::Problem p;
  hipStream_t own = nullptr;  // non-blocking stream for capture when the caller passes NULL
  bool alive = true;
};

namespace {

using qg::fail;

constexpr int kCycleMax = 128;  // longest refresh cycle captured as one graph

bool aligned(const void* ptr) { return (reinterpret_cast<uintptr_t>(ptr) % qg::kAlign) == 0; }

qg_status hip_fail(hipError_t e, const char* what) {
  return fail(QG_ERR_DEVICE, std::string(what) + ": " + hipGetErrorString(e));
}

#define HIP_TRY(call, what)                   \
  do {                                        \
    hipError_t e_ = (call);                   \
    if (e_ != hipSuccess) return hip_fail(e_, what); \
  } while (0)

qg_status check_problem(const qg_problem* pr) {
  if (!pr) return fail(QG_ERR_ARG, "null problem handle");
  if (!pr->alive) return fail(QG_ERR_STATE, "problem handle already destroyed");
  return QG_OK;
}

void drop_graph(qg::Problem& p) {
  if (p.graph_exec) {
    (void)hipGraphExecDestroy(static_cast<hipGraphExec_t>(p.graph_exec));
    p.graph_exec = nullptr;
  }
  for (auto& g : p.step_graph) {
    if (g) (void)hipGraphExecDestroy(static_cast<hipGraphExec_t>(g));
    g = nullptr;
  }
}

// Pinned staging of the schedule table and the step-timing events, created
// at a problem's first solve and kept until it is destroyed.
qg_status solve_resources(qg::Problem& p) {
  if (!p.sched_host) {
    void* h = nullptr;
    hipError_t e = hipHostMalloc(&h, 2 * (size_t)qg::kSchedCap * qg::kSchedStride * sizeof(double),
                                 hipHostMallocDefault);
    if (e != hipSuccess) return hip_fail(e, "pinned schedule table");
    p.sched_host = static_cast<double*>(h);
  }
  for (auto& ev : p.sched_ev)
    if (!ev) {
      hipEvent_t x;
      hipError_t e = hipEventCreateWithFlags(&x, hipEventDisableTiming);
      if (e != hipSuccess) return hip_fail(e, "event");
      ev = x;
    }
  for (auto& ev : p.step_ev)
    if (!ev) {
      hipEvent_t x;
      hipError_t e = hipEventCreate(&x);
      if (e != hipSuccess) return hip_fail(e, "event");
      ev = x;
    }
  return QG_OK;
}

void release_solve_resources(qg::Problem& p) {
  if (p.sched_host) (void)hipHostFree(p.sched_host);
  p.sched_host = nullptr;
  for (auto* set : {&p.sched_ev, &p.step_ev})
    for (auto& ev : *set) {
      if (ev) (void)hipEventDestroy(static_cast<hipEvent_t>(ev));
      ev = nullptr;
    }
}

// Set sizes of the screening options (Alg. 2): worst slots and slots in all.
qg_status screen_counts(const qg::Problem& p, const qg_screen_opts* o, int* n_top, int* n_act) {
  if (!o) return fail(QG_ERR_ARG, "null screening options");
  if (p.K < 1) return fail(QG_ERR_ARG, "screening needs a problem with contingencies");
  if (!(o->top_frac >= 0.0 && o->top_frac <= 1.0) || !(o->rand_frac >= 0.0 && o->rand_frac <= 1.0))
    return fail(QG_ERR_ARG, "top_frac and rand_frac must lie in [0, 1]");
  if (!std::isfinite(o->zeta)) return fail(QG_ERR_ARG, "zeta must be finite");
  if (o->refresh_every < 1) return fail(QG_ERR_ARG, "refresh_every must be >= 1");
  if (o->reserved != 0) return fail(QG_ERR_ARG, "reserved field must be 0");
  const int nt = std::min(p.K, (int)std::ceil(o->top_frac * (double)p.K));
  const int na = std::min(p.K, nt + (int)std::ceil(o->rand_frac * (double)p.K));
  if (na < 1) return fail(QG_ERR_ARG, "the options select no contingency");
  *n_top = nt;
  *n_act = na;
  return QG_OK;
}

// Evaluations score the chosen set once screening is on and a set exists.
bool screened(const qg::Problem& p) { return p.scr.on && p.scr.chosen; }

// Scratch of qg_eval_grad_noalloc: a static device array, one copy per GPU.
// In host code its name is a host-side stand-in, never a device address:
// the device address is looked up once per device with hipGetSymbolAddress
// (that device current) and only that address is passed to kernels.
static __device__ __align__(256) unsigned char scratch[QG_NOALLOC_SCRATCH];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_addr[kMaxDevices] = {};

qg_status noalloc_scratch(int dev, void** out) {
  if (dev < 0 || dev >= kMaxDevices) return fail(QG_ERR_ARG, "device index out of range");
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_addr[dev]) {
    void* ptr = nullptr;
    hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return hip_fail(e, "address of the static scratch");
    if (!ptr || !aligned(ptr)) return fail(QG_ERR_DEVICE, "static scratch is not 256-byte aligned");
    g_scratch_addr[dev] = ptr;
  }
  *out = g_scratch_addr[dev];
  return QG_OK;
}

}  // namespace

extern "C" {

const char* qg_status_string(qg_status s) {
  switch (s) {
    case QG_OK: return "ok";
    case QG_ERR_ARG: return "invalid argument";
    case QG_ERR_TOPOLOGY: return "topology error";
    case QG_ERR_SINGULAR: return "singular susceptance matrix";
    case QG_ERR_NONFINITE: return "non-finite input";
    case QG_ERR_DEVICE: return "device error";
    case QG_ERR_STATE: return "invalid state";
  }
  return "unknown status";
}

const char* qg_last_error(void) { return qg::last_error_text(); }

qg_status qg_problem_sizes(const qg_grid_desc* desc, const qg_build_opts* opts, qg_sizes* out) {
  if (!out) return fail(QG_ERR_ARG, "null output");
  qg::Problem p;
  qg_status s = qg::plan_problem(desc, opts, &p);
  if (s != QG_OK) return s;
  out->const_bytes = p.const_bytes;
  out->workspace_bytes = p.work_bytes;
  out->n_x = p.n_x;
  out->n_ctg = p.K;
  return QG_OK;
}

qg_status qg_build_problem(const qg_grid_desc* desc, const qg_build_opts* opts,
                           void* d_const_arena, size_t const_bytes, void* stream,
                           qg_problem** out) {
  if (!out) return fail(QG_ERR_ARG, "null output handle");
  if (!d_const_arena || !aligned(d_const_arena))
    return fail(QG_ERR_ARG, "constant arena must be non-null and 256-byte aligned");
  qg_problem* pr = new (std::nothrow) qg_problem();
  if (!pr) return fail(QG_ERR_ARG, "host allocation failed");
  qg_status s = qg::plan_problem(desc, opts, &pr->p);
  if (s != QG_OK) { delete pr; return s; }
  if (const_bytes < pr->p.const_bytes) {
    delete pr;
    return fail(QG_ERR_ARG, "constant arena too small: need " + std::to_string(pr->p.const_bytes));
  }
  qg::HostBuild hb;
  s = qg::build_arena(desc, opts, &pr->p, &hb);
  if (s != QG_OK) { delete pr; return s; }
  hipStream_t st = static_cast<hipStream_t>(stream);
  hipError_t e = hipMemcpyAsync(d_const_arena, hb.image.data(), hb.image.size(),
                                hipMemcpyHostToDevice, st);
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  if (e == hipSuccess) e = hipStreamCreateWithFlags(&pr->own, hipStreamNonBlocking);
  if (e != hipSuccess) { delete pr; return hip_fail(e, "upload of the constant arena"); }
  qg::rebase_pointers(&pr->p, d_const_arena);
  e = hipGetDevice(&pr->p.device);
  if (e != hipSuccess) { qg_destroy_problem(pr); return hip_fail(e, "current device"); }
  *out = pr;
  return QG_OK;
}

qg_status qg_build_image(const qg_grid_desc* desc, const qg_build_opts* opts, void* host_image,
                         size_t bytes) {
  if (!host_image) return fail(QG_ERR_ARG, "null host image");
  qg::Problem p;
  qg_status s = qg::plan_problem(desc, opts, &p);
  if (s != QG_OK) return s;
  if (bytes < p.const_bytes)
    return fail(QG_ERR_ARG, "host image too small: need " + std::to_string(p.const_bytes));
  qg::HostBuild hb;
  s = qg::build_arena(desc, opts, &p, &hb);
  if (s != QG_OK) return s;
  std::memcpy(host_image, hb.image.data(), hb.image.size());
  return QG_OK;
}

qg_status qg_update_loads(qg_problem* pr, const double* load_p, const double* load_q,
                          const double* reserve_req, void* stream) {
  qg_status s = check_problem(pr);
  if (s != QG_OK) return s;
  if (!load_p || !load_q || !reserve_req) return fail(QG_ERR_ARG, "null load array");
  qg::Problem& p = pr->p;
  const size_t TN = (size_t)p.T * p.N;
  for (size_t e = 0; e < TN; ++e)
    if (!std::isfinite(load_p[e]) || !std::isfinite(load_q[e]))
      return fail(QG_ERR_ARG, "non-finite load");
  for (int t = 0; t < p.T; ++t)
    if (!std::isfinite(reserve_req[t])) return fail(QG_ERR_ARG, "non-finite reserve requirement");
  qg::LoadBlock lb;
  qg::load_block(&p, load_p, &lb);
  hipStream_t st = static_cast<hipStream_t>(stream);
  unsigned char* base = static_cast<unsigned char*>(p.arena);
  // the stream's earlier work may still read the old values
  HIP_TRY(hipStreamSynchronize(st), "stream sync");
  HIP_TRY(hipMemcpyAsync(base + lb.off_lp, load_p, TN * sizeof(double), hipMemcpyHostToDevice,
                         st), "load upload");
  HIP_TRY(hipMemcpyAsync(base + lb.off_lq, load_q, TN * sizeof(double), hipMemcpyHostToDevice,
                         st), "load upload");
  HIP_TRY(hipMemcpyAsync(base + lb.off_rsv, reserve_req, p.T * sizeof(double),
                         hipMemcpyHostToDevice, st), "load upload");
  HIP_TRY(hipMemcpyAsync(base + lb.off_sum, lb.sum_load.data(), p.T * sizeof(double),
                         hipMemcpyHostToDevice, st), "load upload");
  HIP_TRY(hipMemcpyAsync(base + lb.off_cload, lb.cload.data(), lb.cload.size() * sizeof(double),
                         hipMemcpyHostToDevice, st), "load upload");
  HIP_TRY(hipStreamSynchronize(st), "stream sync");
  p.dp.vload = lb.vload;
  // a cached step graph holds the old consumer value among its arguments
  drop_graph(p);
  return QG_OK;
}

qg_status qg_layout_of(const qg_problem* pr, qg_layout* out) {
  qg_status s = check_problem(pr);
  if (s != QG_OK) return s;
  if (!out) return fail(QG_ERR_ARG, "null output");
  const int64_t TN = (int64_t)pr->p.T * pr->p.N, TG = (int64_t)pr->p.T * pr->p.G;
  const int64_t len[QG_NCLASS] = {TN, TN, TG, TG, TG, TG};
  int64_t o = 0;
  for (int c = 0; c < QG_NCLASS; ++c) { out->off[c] = o; out->len[c] = len[c]; o += len[c]; }
  return QG_OK;
}

qg_status qg_ctg_list(const qg_problem* pr, int32_t* out, int32_t capacity) {
  qg_status s = check_problem(pr);
  if (s != QG_OK) return s;
  if (capacity < pr->p.K || (pr->p.K > 0 && !out)) return fail(QG_ERR_ARG, "output too small");
  for (int k = 0; k < pr->p.K; ++k) out[k] = pr->p.ctg[k];
  return QG_OK;
}

qg_status qg_problem_dims(const qg_problem* pr, int32_t* d, int32_t capacity) {
  qg_status s = check_problem(pr);
  if (s != QG_OK) return s;
  if (!d || capacity < 16) return fail(QG_ERR_ARG, "dims needs 16 entries");
  const qg::Problem& p = pr->p;
  const int32_t v[19] = {p.N,  p.L,   p.G,   p.T,       p.M,       p.K,       p.Lp,
                         p.Kp, p.G16, p.G4,  p.Tp,      p.nLb,     p.nKb,     p.tile.bl,
                         p.tile.wl,   p.tile.tc, p.dp.lodf_kind, p.tile.lt, p.tile.split};
  std::memcpy(d, v, sizeof(int32_t) * (capacity < 19 ? capacity : 19));
  return QG_OK;
}

qg_status qg_screen_bytes(const qg_problem* pr, const qg_screen_opts* o, size_t* bytes) {
  qg_status s = check_problem(pr);
  if (s != QG_OK) return s;
  if (!bytes) return fail(QG_ERR_ARG, "null output");
  int nt = 0, na = 0;
  s = screen_counts(pr->p, o, &nt, &na);
  if (s != QG_OK) return s;
  *bytes = qg::screen_bytes(pr->p, na);
  return QG_OK;
}

qg_status qg_set_screening(qg_problem* pr, const qg_screen_opts* o, void* d_buf, size_t bytes,
                           void* stream) {
  (void)stream;  // no device work: the buffer is written by the first selection
  qg_status s = check_problem(pr);
  if (s != QG_OK) return s;
  qg::Problem& p = pr->p;
  if (!o) {
    p.scr = qg::Screen{};
    drop_graph(p);
    return QG_OK;
  }
  int nt = 0, na = 0;
  s = screen_counts(p, o, &nt, &na);
  if (s != QG_OK) return s;
  if (!d_buf || !aligned(d_buf)) return fail(QG_ERR_ARG, "screening buffer must be 256-byte aligned");
  const size_t need = qg::screen_bytes(p, na);
  if (bytes < need) return fail(QG_ERR_ARG, "screening buffer too small: need " + std::to_string(need));
  qg::Screen sc;
  qg::carve_screen(p, d_buf, na, &sc);
  sc.on = true;
  sc.chosen = false;
  sc.n_top = nt;
  sc.n_act = na;
  sc.cap = na;
  sc.Ka = (int)qg::round_up(na, qg::kCtgLanes);
  sc.zeta = o->zeta;
  sc.refresh = o->refresh_every;
  sc.seed = o->seed;
  p.scr = sc;
  drop_graph(p);
  return QG_OK;
}

qg_status qg_screen_refresh(qg_problem* pr, const double* d_x, const qg_homotopy* h,
                            int64_t round, void* d_workspace, void* stream) {
  qg_status s = check_problem(pr);
  if (s != QG_OK) return s;
  qg::Problem& p = pr->p;
  if (!p.scr.on) return fail(QG_ERR_STATE, "screening is off");
  if (!d_x || !h || !d_workspace) return fail(QG_ERR_ARG, "null x, homotopy or workspace");
  if (!aligned(d_x) || !aligned(d_workspace))
    return fail(QG_ERR_ARG, "device buffers must be 256-byte aligned");
  if (round < 0) return fail(QG_ERR_ARG, "round must be >= 0");
  if (!(h->eps >= 0.0) || !(h->beta >= 0.0) || !(h->rho_scale >= 0.0) || !std::isfinite(h->eps) ||
      !std::isfinite(h->beta) || !std::isfinite(h->rho_scale))
    return fail(QG_ERR_ARG, "homotopy values must be finite and non-negative");
  qg::DevWork w = qg::carve_workspace(&p, d_workspace);
  qg::EvalMode m{};
  m.schedule = 0;
  m.eps = h->eps;
  m.beta = h->beta;
  m.rho_s = h->rho_scale;
  if (p.scr.n_act != p.scr.cap) drop_graph(p);
  p.scr.n_act = p.scr.cap;
  p.scr.Ka = (int)qg::round_up(p.scr.cap, qg::kCtgLanes);
  int e = qg::launch_eval(&p, w, d_x, nullptr, nullptr, m, 0, nullptr, nullptr, stream, nullptr);
  if (e == 0) e = qg::launch_screen_select(&p, w, round, stream);
  if (e != 0) return hip_fail((hipError_t)e, "kernel launch");
  p.scr.chosen = true;
  return QG_OK;
}

qg_status qg_set_active_contingencies(qg_problem* pr, const int32_t* ks, int32_t n,
                                      void* stream) {
  qg_status s = check_problem(pr);
  if (s != QG_OK) return s;
  qg::Problem& p = pr->p;
  if (!p.scr.on) return fail(QG_ERR_STATE, "screening is off");
  if (!ks || n < 1 || n > p.scr.cap)
    return fail(QG_ERR_ARG, "need 1 <= n <= " + std::to_string(p.scr.cap) + " contingencies");
  for (int i = 0; i < n; ++i)
    if (ks[i] < 0 || ks[i] >= p.K || (i > 0 && ks[i] <= ks[i - 1]))
      return fail(QG_ERR_ARG, "positions must be strictly increasing in [0, K)");
  std::vector<int32_t> act(p.Kp, 0), slot(p.Kp, -1);
  for (int i = 0; i < n; ++i) {
    act[i] = ks[i];
    slot[ks[i]] = i;
  }
  hipStream_t st = static_cast<hipStream_t>(stream);
  HIP_TRY(hipStreamSynchronize(st), "stream sync");  // earlier steps may still read the set
  HIP_TRY(hipMemcpyAsync(p.scr.act_k, act.data(), act.size() * sizeof(int32_t),
                         hipMemcpyHostToDevice, st), "set upload");
  HIP_TRY(hipMemcpyAsync(p.scr.act_slot, slot.data(), slot.size() * sizeof(int32_t),
                         hipMemcpyHostToDevice, st), "set upload");
  if (n != p.scr.n_act) drop_graph(p);
  p.scr.n_act = n;
  p.scr.Ka = (int)qg::round_up(n, qg::kCtgLanes);
  if (qg::launch_screen_gather(&p, st) != 0) return hip_fail(hipGetLastError(), "kernel launch");
  HIP_TRY(hipStreamSynchronize(st), "stream sync");
  p.scr.chosen = true;
  return QG_OK;
}

qg_status qg_get_active_contingencies(const qg_problem* pr, int32_t* out, int32_t capacity,
                                      int32_t* n, double* sev, void* stream) {
  qg_status s = check_problem(pr);
  if (s != QG_OK) return s;
  const qg::Problem& p = pr->p;
  if (!p.scr.on || !p.scr.chosen) return fail(QG_ERR_STATE, "screening is off or no set chosen");
  if (!out || !n) return fail(QG_ERR_ARG, "null output");
  if (capacity < p.scr.n_act) return fail(QG_ERR_ARG, "output too small");
  if (sev && capacity < p.K) return fail(QG_ERR_ARG, "severities need capacity >= K");
  hipStream_t st = static_cast<hipStream_t>(stream);
  HIP_TRY(hipMemcpyAsync(out, p.scr.act_k, (size_t)p.scr.n_act * sizeof(int32_t),
                         hipMemcpyDeviceToHost, st), "set read");
  if (sev)
    HIP_TRY(hipMemcpyAsync(sev, p.scr.sev, (size_t)p.K * sizeof(double), hipMemcpyDeviceToHost, st),
            "severity read");
  HIP_TRY(hipStreamSynchronize(st), "stream sync");
  *n = p.scr.n_act;
  return QG_OK;
}

qg_status qg_set_ctg_tile(qg_problem* pr, int32_t bl, int32_t wl, int32_t tc) {
  qg_status s = check_problem(pr);
  if (s != QG_OK) return s;
  if (!(bl == 8 || bl == 16 || bl == 32) || !(wl == 1 || wl == 2 || wl == 4 || wl == 8) ||
      bl * wl < 16)
    return fail(QG_ERR_ARG, "tile must have bl in {8,16,32}, wl in {1,2,4,8}, bl*wl >= 16");
  qg::Problem& p = pr->p;
  if (tc <= 0) tc = qg::default_ctg_tc(p, wl);
  if (tc > p.T) tc = p.T;
  if (tc > qg::kCtgMaxTc) return fail(QG_ERR_ARG, "at most 8 periods per block");
  if (tc > qg::ctg_tc_cap(wl))
    return fail(QG_ERR_ARG, "too many periods per block for the LDS budget at this wl");
  qg::CtgTile t{bl, wl, tc, 1};
  t.lt = qg::default_ctg_lt(p, t);
  qg::apply_ctg_tile(&p, t);
  return QG_OK;
}

qg_status qg_set_ctg_tile_split(qg_problem* pr, int32_t wl, int32_t tcw, int32_t lt) {
  qg_status s = check_problem(pr);
  if (s != QG_OK) return s;
  if (wl < 1 || wl > 8 || tcw < 1 || tcw > qg::kCtgMaxTc || lt == 1 || lt < 0 || lt > 64)
    return fail(QG_ERR_ARG, "split tile needs wl in [1, 8], tcw in [1, 8], lt 0 or in [2, 64]");
  qg::CtgTile t{8, wl, tcw, lt};
  t.split = 1;
  if (lt == 0) t.lt = qg::default_ctg_lt(pr->p, t);
  qg::apply_ctg_tile(&pr->p, t);
  return QG_OK;
}

qg_status qg_set_ctg_ltiles(qg_problem* pr, int32_t lt) {
  qg_status s = check_problem(pr);
  if (s != QG_OK) return s;
  if (lt < 0 || lt > 64) return fail(QG_ERR_ARG, "lt must lie in [0, 64]");
  qg::Problem& p = pr->p;
  qg::CtgTile t = p.tile;
  if (t.split && lt == 1) return fail(QG_ERR_ARG, "a period-split tile needs lt >= 2");
  t.lt = lt > 0 ? lt : qg::default_ctg_lt(p, t);
  qg::apply_ctg_tile(&p, t);
  return QG_OK;
}

qg_status eval_grad_in(qg_problem* pr, const double* d_x, double* d_grad, double* d_terms,
                       const qg_homotopy* h, void* d_workspace, void* stream);

qg_status qg_eval_grad(qg_problem* pr, const double* d_x, double* d_grad, double* d_terms,
                       const qg_homotopy* h, void* d_workspace, void* stream) {
  return eval_grad_in(pr, d_x, d_grad, d_terms, h, d_workspace, stream);
}

qg_status qg_eval_grad_noalloc(qg_problem* pr, const double* d_x, double* d_grad,
                               double* d_terms, const qg_homotopy* h, void* stream) {
  qg_status s = check_problem(pr);
  if (s != QG_OK) return s;
  if (pr->p.work_bytes > QG_NOALLOC_SCRATCH)
    return fail(QG_ERR_ARG, "workspace of this problem (" + std::to_string(pr->p.work_bytes) +
                                " bytes) exceeds the static scratch of qg_eval_grad_noalloc (" +
                                std::to_string((size_t)QG_NOALLOC_SCRATCH) + " bytes)");
  int dev = -1;
  HIP_TRY(hipGetDevice(&dev), "current device");
  if (dev != pr->p.device)
    return fail(QG_ERR_ARG, "current device " + std::to_string(dev) +
                                " is not the problem's device " + std::to_string(pr->p.device));
  void* ws = nullptr;
  s = noalloc_scratch(dev, &ws);
  if (s != QG_OK) return s;
  return eval_grad_in(pr, d_x, d_grad, d_terms, h, ws, stream);
}

qg_status eval_grad_in(qg_problem* pr, const double* d_x, double* d_grad, double* d_terms,
                       const qg_homotopy* h, void* d_workspace, void* stream) {
  qg_status s = check_problem(pr);
  if (s != QG_OK) return s;
  if (!d_x || !h || !d_workspace) return fail(QG_ERR_ARG, "null x, homotopy or workspace");
  if (!aligned(d_x) || !aligned(d_workspace) || (d_grad && !aligned(d_grad)) ||
      (d_terms && !aligned(d_terms)))
    return fail(QG_ERR_ARG, "device buffers must be 256-byte aligned");
  if (!(h->eps >= 0.0) || !(h->beta >= 0.0) || !(h->rho_scale >= 0.0) || !std::isfinite(h->eps) ||
      !std::isfinite(h->beta) || !std::isfinite(h->rho_scale))
    return fail(QG_ERR_ARG, "homotopy values must be finite and non-negative");
  const qg::Problem& p = pr->p;
  qg::DevWork w = qg::carve_workspace(&p, d_workspace);
  if (p.flags & QG_FLAG_CHECK_FINITE) {
    int* flag = reinterpret_cast<int*>(w.params + 14);
    if (qg::launch_check_finite(&p, d_x, flag, stream) != 0)
      return hip_fail(hipGetLastError(), "finite check launch");
    int hflag = 0;
    HIP_TRY(hipMemcpyAsync(&hflag, flag, sizeof(int), hipMemcpyDeviceToHost,
                           static_cast<hipStream_t>(stream)), "finite check read");
    HIP_TRY(hipStreamSynchronize(static_cast<hipStream_t>(stream)), "finite check sync");
    if (hflag) return fail(QG_ERR_NONFINITE, "x holds a NaN or Inf");
  }
  qg::EvalMode m{};
  m.schedule = 0;
  m.eps = h->eps;
  m.beta = h->beta;
  m.rho_s = h->rho_scale;
  m.screened = screened(p) ? 1 : 0;
  int e = qg::launch_eval(&p, w, d_x, d_grad, d_terms, m, 0, nullptr, nullptr, stream, nullptr);
  if (e != 0) return hip_fail((hipError_t)e, "kernel launch");
  return QG_OK;
}

qg_status qg_time_stage(qg_problem* pr, const double* d_x, const qg_homotopy* h, int32_t stage,
                        int32_t reps, void* d_workspace, void* stream, double* mean_us) {
  qg_status s = check_problem(pr);
  if (s != QG_OK) return s;
  if (!d_x || !h || !d_workspace || !mean_us) return fail(QG_ERR_ARG, "null argument");
  if (!aligned(d_x) || !aligned(d_workspace))
    return fail(QG_ERR_ARG, "device buffers must be 256-byte aligned");
  if (stage < 0 || stage >= qg::kStages) return fail(QG_ERR_ARG, "stage out of range");
  if (reps < 1 || reps > 100000) return fail(QG_ERR_ARG, "reps must be in [1, 100000]");
  if (!(h->eps >= 0.0) || !(h->beta >= 0.0) || !(h->rho_scale >= 0.0) || !std::isfinite(h->eps) ||
      !std::isfinite(h->beta) || !std::isfinite(h->rho_scale))
    return fail(QG_ERR_ARG, "homotopy values must be finite and non-negative");
  const qg::Problem& p = pr->p;
  qg::DevWork w = qg::carve_workspace(&p, d_workspace);
  qg::EvalMode m{};
  m.schedule = 0;
  m.eps = h->eps;
  m.beta = h->beta;
  m.rho_s = h->rho_scale;
  m.screened = screened(p) ? 1 : 0;
  double ms = 0.0;
  int e = qg::time_stage(&p, w, d_x, m, stage, reps, stream, &ms);
  if (e != 0) return hip_fail((hipError_t)e, "stage timing");
  *mean_us = ms * 1e3;
  return QG_OK;
}

qg_status qg_adam_step(qg_problem* pr, double* d_x, double* d_m, double* d_v,
                       const double* d_grad, int64_t iter, const double lr[QG_NCLASS],
                       const qg_adam_cfg* cfg, void* stream) {
  qg_status s = check_problem(pr);
  if (s != QG_OK) return s;
  if (!d_x || !d_m || !d_v || !d_grad || !lr || !cfg)
    return fail(QG_ERR_ARG, "null argument");
  if (!aligned(d_x) || !aligned(d_m) || !aligned(d_v) || !aligned(d_grad))
    return fail(QG_ERR_ARG, "device buffers must be 256-byte aligned");
  if (iter < 1) return fail(QG_ERR_ARG, "iter is 1-based");
  if (!(cfg->beta1 >= 0.0 && cfg->beta1 < 1.0) || !(cfg->beta2 >= 0.0 && cfg->beta2 < 1.0) ||
      !(cfg->eps > 0.0))
    return fail(QG_ERR_ARG, "need 0 <= beta1, beta2 < 1 and eps > 0");
  const double bc1 = 1.0 - std::pow(cfg->beta1, (double)iter);
  const double bc2 = 1.0 - std::pow(cfg->beta2, (double)iter);
  int e = qg::launch_adam(&pr->p, d_x, d_m, d_v, d_grad, lr, bc1, bc2, cfg->beta1, cfg->beta2,
                          cfg->eps, cfg->eps_in_numerator, stream);
  if (e != 0) return hip_fail((hipError_t)e, "kernel launch");
  return QG_OK;
}

// Rows of the per-step schedule table for steps first .. first+count-1:
// eqs. (norm_t)-(step_size) indexed by the iteration i (t0 = 0, tf = n_total)
// for eps and the step sizes, linear ramps for beta and rho, and the Adam
// bias corrections.
static void fill_schedule(double* table, const qg_solve_opts* o, const qg_adam_cfg* cfg,
                          int64_t n_total, int64_t first, int count) {
  const double n = (double)n_total;
  for (int q = 0; q < count; ++q) {
    const double i = (double)(first + q);
    const double th = 2.0 * i / n - 1.0;
    const double e = std::exp(4.0 * th);
    const double sc = e / (0.6 + e);
    double* row = &table[(size_t)q * qg::kSchedStride];
    row[0] = o->eps0 * std::pow(10.0, sc * std::log10(o->epsf / o->eps0));
    row[1] = o->beta0 + (o->betaf - o->beta0) * (i / n);
    row[2] = o->rho0 + (o->rhof - o->rho0) * (i / n);
    for (int c = 0; c < QG_NCLASS; ++c)
      row[3 + c] = o->alpha0[c] * std::pow(10.0, sc * std::log10(o->alphaf[c] / o->alpha0[c]));
    row[9] = 1.0 - std::pow(cfg->beta1, i);
    row[10] = 1.0 - std::pow(cfg->beta2, i);
    row[11] = i - 1.0;  // 0-based iteration index (refresh index of screening)
  }
}

static qg_status check_solve_opts(const qg_solve_opts* o, const qg_adam_cfg* cfg) {
  if (o->n_steps < 0 || o->iter0 < 0 || o->check_every < 0)
    return fail(QG_ERR_ARG, "negative step counts");
  const int64_t n_total = o->n_total > 0 ? o->n_total : o->iter0 + o->n_steps;
  if (o->iter0 + o->n_steps > n_total) return fail(QG_ERR_ARG, "n_total below iter0 + n_steps");
  for (int c = 0; c < QG_NCLASS; ++c)
    if (!(o->alpha0[c] > 0.0) || !(o->alphaf[c] > 0.0))
      return fail(QG_ERR_ARG, "step sizes must be positive");
  if (!(o->eps0 > 0.0) || !(o->epsf > 0.0)) return fail(QG_ERR_ARG, "eps0, epsf must be positive");
  if (!(cfg->beta1 >= 0.0 && cfg->beta1 < 1.0) || !(cfg->beta2 >= 0.0 && cfg->beta2 < 1.0) ||
      !(cfg->eps > 0.0))
    return fail(QG_ERR_ARG, "need 0 <= beta1, beta2 < 1 and eps > 0");
  return QG_OK;
}

qg_status qg_solve(qg_problem* pr, double* d_x, double* d_m, double* d_v,
                   const qg_solve_opts* o, const qg_adam_cfg* cfg, qg_solve_report* rep,
                   void* d_workspace, void* stream) {
  using clock = std::chrono::steady_clock;
  const auto t_start = clock::now();
  qg_status s = check_problem(pr);
  if (s != QG_OK) return s;
  if (!d_x || !d_m || !d_v || !o || !cfg || !rep || !d_workspace)
    return fail(QG_ERR_ARG, "null argument");
  if (!aligned(d_x) || !aligned(d_m) || !aligned(d_v) || !aligned(d_workspace))
    return fail(QG_ERR_ARG, "device buffers must be 256-byte aligned");
  s = check_solve_opts(o, cfg);
  if (s != QG_OK) return s;
  if (o->profile && pr->p.scr.on)
    return fail(QG_ERR_ARG, "profile mode times the exact step: turn screening off");
  if (o->reserved != 0) return fail(QG_ERR_ARG, "reserved field must be 0");
  s = solve_resources(pr->p);
  if (s != QG_OK) return s;
  const int64_t n_total = o->n_total > 0 ? o->n_total : o->iter0 + o->n_steps;

  const qg::Problem& p = pr->p;
  const bool scr = p.scr.on;
  const int64_t R = scr ? p.scr.refresh : 0;
  qg::DevWork w = qg::carve_workspace(&p, d_workspace);
  hipStream_t user = static_cast<hipStream_t>(stream);
  hipStream_t ex = user ? user : pr->own;
  if (!user) {
    // order the internal stream after prior work on the default stream
    hipEvent_t ev;
    HIP_TRY(hipEventCreateWithFlags(&ev, hipEventDisableTiming), "event");
    HIP_TRY(hipEventRecord(ev, nullptr), "event record");
    HIP_TRY(hipStreamWaitEvent(ex, ev, 0), "stream wait");
    (void)hipEventDestroy(ev);
  }

  // the kernels read each step's homotopy and step sizes from the schedule
  // table; the captured graphs depend only on the Adam constants
  qg::EvalMode sm;
  std::memset(&sm, 0, sizeof(sm));  // memcmp below compares padding too
  sm.schedule = 1;
  sm.adam_b1 = cfg->beta1; sm.adam_b2 = cfg->beta2; sm.adam_eps = cfg->eps;
  sm.eps_in_num = cfg->eps_in_numerator;
  // screened steps (the graph holds these when screening is on); exact steps
  // with a refresh of the set in between
  qg::EvalMode sm_run = sm;
  sm_run.screened = scr ? 1 : 0;

  // The device table holds the schedule rows of up to kSchedCap consecutive
  // iterations.  A chunk of steps whose rows are already there (same
  // schedule, same workspace: a later call of the same solve) only sets the
  // step counter; otherwise the rows from its first iteration to the end of
  // the horizon (at most kSchedCap) are filled in one half of the pinned
  // staging buffer and copied on the stream.  A half is refilled only after
  // the event behind its previous copy (the copies are asynchronous).
  unsigned char skey[sizeof(pr->p.sched_key)];
  {
    std::memset(skey, 0, sizeof(skey));
    size_t at = 0;
    auto put = [&](const void* v, size_t n) { std::memcpy(skey + at, v, n); at += n; };
    const void* wsp = d_workspace;
    put(&wsp, sizeof(wsp));
    put(&n_total, sizeof(n_total));
    put(o->alpha0, sizeof(o->alpha0));
    put(o->alphaf, sizeof(o->alphaf));
    const double sc[8] = {o->eps0, o->epsf, o->beta0, o->betaf, o->rho0, o->rhof,
                          cfg->beta1, cfg->beta2};
    put(sc, sizeof(sc));
    static_assert(8 + 8 + 2 * 6 * 8 + 8 * 8 <= sizeof(skey), "schedule key size");
  }
  int half = 0;
  bool half_used[2] = {false, false};
  auto upload = [&](int64_t first, int count) -> qg_status {
    qg::Problem& pm = pr->p;
    if (pm.sched_base >= 1 && std::memcmp(skey, pm.sched_key, sizeof(skey)) == 0 &&
        first >= pm.sched_base && first + count <= pm.sched_base + pm.sched_rows) {
      const bool continues = first == pm.sched_next;
      pm.sched_next = -1;  // set again once this chunk's steps are enqueued
      if (!continues && qg::launch_set_step(&p, w, first - pm.sched_base, ex) != 0)
        return hip_fail(hipGetLastError(), "launch");
      return QG_OK;
    }
    pm.sched_next = -1;
    const int rows = (int)std::min<int64_t>(qg::kSchedCap, n_total - first + 1);
    double* table = pm.sched_host + (size_t)half * qg::kSchedCap * qg::kSchedStride;
    hipEvent_t done_ev = static_cast<hipEvent_t>(pm.sched_ev[half]);
    if (half_used[half]) HIP_TRY(hipEventSynchronize(done_ev), "event sync");
    fill_schedule(table, o, cfg, n_total, first, rows);
    pm.sched_base = -1;
    HIP_TRY(hipMemcpyAsync(w.sched, table, (size_t)rows * qg::kSchedStride * sizeof(double),
                           hipMemcpyHostToDevice, ex), "schedule upload");
    HIP_TRY(hipEventRecord(done_ev, ex), "event record");
    half_used[half] = true;
    half ^= 1;
    std::memcpy(pm.sched_key, skey, sizeof(skey));
    pm.sched_base = first;
    pm.sched_rows = rows;
    if (qg::launch_set_step(&p, w, 0, ex) != 0) return hip_fail(hipGetLastError(), "launch");
    return QG_OK;
  };

  qg::EvalMode score{};
  score.schedule = 0;
  score.eps = 0.0;
  score.beta = 1.0;
  score.rho_s = o->rhof;

  std::memset(rep, 0, sizeof(*rep));
  rep->steps_to_gap = -1;
  rep->time_to_gap_s = -1.0;

  const bool profile = o->profile != 0;
  const bool graph = o->use_graph != 0 && !profile;
  // profile: events around every kernel of up to kProfSteps queued steps,
  // read after one synchronisation, so host latency does not enter the times
  constexpr int kKernels = qg::kStages, kProfSteps = 32, kEv = kKernels + 1;
  struct Events {  // destroyed on every return path
    std::vector<hipEvent_t> v;
    ~Events() {
      for (auto& e : v)
        if (e) (void)hipEventDestroy(e);
    }
  } ev_hold;
  std::vector<hipEvent_t>& evs = ev_hold.v;
  if (profile) {
    evs.assign(kProfSteps * kEv, nullptr);
    for (auto& e : evs) HIP_TRY(hipEventCreate(&e), "event");
  }

  // plain steps replay the cached graphs of 2^i consecutive steps (the step
  // counter lives on the device): a call of n steps launches one graph per
  // set bit of n (at most 32 steps per launch), whatever n is, so calls of
  // different lengths share the same graphs.  Screening: one graph per
  // refresh cycle (the exact step, the selection and the R - 1 screened
  // steps), so the refresh adds no launch gaps
  int gsteps = 0;
  if (scr) gsteps = (R >= 2 && R <= kCycleMax && o->n_steps >= R) ? (int)R : 0;
  if (scr && pr->p.scr.n_act != pr->p.scr.cap) {
    // a smaller set given by the caller: the solve works with full-size sets,
    // chosen afresh at its first step
    pr->p.scr.chosen = false;
    pr->p.scr.n_act = pr->p.scr.cap;
    pr->p.scr.Ka = (int)qg::round_up(pr->p.scr.cap, qg::kCtgLanes);
    drop_graph(pr->p);
  }
  hipGraphExec_t gexec = nullptr;  // screening: the cycle graph, when it holds this call's steps
  bool step_graphs = false;        // plain steps: the cached 2^i-step graphs are current
  if (graph && (scr ? gsteps >= 4 : o->n_steps > 0)) {
    const void* key[5] = {d_x, d_m, d_v, d_workspace, nullptr};
    bool hit = (scr ? pr->p.graph_exec != nullptr : pr->p.step_graph[0] != nullptr) &&
               std::memcmp(key, pr->p.graph_key, sizeof(key)) == 0 &&
               (!scr || pr->p.graph_steps == gsteps);
    // the schedule constants are kernel arguments, so a different schedule
    // needs a new capture as well
    if (hit && std::memcmp(&pr->p.graph_mode, &sm_run, sizeof(sm_run)) != 0) hit = false;
    // and so is the contingency tile (grid and LDS size of the map-reduce)
    const qg::CtgTile& gt = pr->p.graph_tile;
    if (hit && (gt.bl != p.tile.bl || gt.wl != p.tile.wl || gt.tc != p.tile.tc ||
                gt.lt != p.tile.lt || gt.split != p.tile.split))
      hit = false;
    if (!hit) {
      drop_graph(pr->p);
      auto capture = [&](int nsteps, bool cycle, void** slot) -> qg_status {
        hipGraph_t g;
        hipGraphExec_t ge = nullptr;
        HIP_TRY(hipStreamBeginCapture(pr->own, hipStreamCaptureModeThreadLocal), "begin capture");
        if (cycle) {
          qg::launch_eval(&p, w, d_x, nullptr, nullptr, sm, 1, d_m, d_v, pr->own, nullptr);
          qg::launch_screen_select(&p, w, -1, pr->own);
          for (int k = 1; k < nsteps; ++k)
            qg::launch_eval(&p, w, d_x, nullptr, nullptr, sm_run, 1, d_m, d_v, pr->own, nullptr);
        } else {
          for (int k = 0; k < nsteps; ++k)
            qg::launch_eval(&p, w, d_x, nullptr, nullptr, sm_run, 1, d_m, d_v, pr->own, nullptr);
        }
        HIP_TRY(hipStreamEndCapture(pr->own, &g), "end capture");
        hipError_t e = hipGraphInstantiate(&ge, g, nullptr, nullptr, 0);
        (void)hipGraphDestroy(g);
        if (e != hipSuccess) return hip_fail(e, "graph instantiate");
        *slot = ge;
        return QG_OK;
      };
      if (scr) {
        s = capture(gsteps, true, &pr->p.graph_exec);
      } else {
        for (int i = 0; i < qg::kStepGraphs && s == QG_OK; ++i)
          s = capture(1 << i, false, &pr->p.step_graph[i]);
      }
      if (s != QG_OK) {
        drop_graph(pr->p);
        return s;
      }
      std::memcpy(pr->p.graph_key, key, sizeof(key));
      pr->p.graph_steps = scr ? gsteps : 0;
      std::memcpy(&pr->p.graph_mode, &sm_run, sizeof(sm_run));
      pr->p.graph_tile = p.tile;
    }
    if (scr) gexec = static_cast<hipGraphExec_t>(pr->p.graph_exec);
    else step_graphs = true;
  }

  // screening: steps [done0, done0 + n) of this call, the step of iteration
  // index it = iter0 + done (0-based) exact and followed by a selection when
  // it is a multiple of R or no set exists yet
  auto run_screened = [&](int64_t done0, int64_t n) -> qg_status {
    int64_t k = 0;
    while (k < n) {
      const int64_t it = o->iter0 + done0 + k;
      if (gexec && it % R == 0 && n - k >= R) {
        HIP_TRY(hipGraphLaunch(gexec, ex), "graph launch");
        pr->p.scr.chosen = true;
        k += R;
        continue;
      }
      if (it % R == 0 || !pr->p.scr.chosen) {
        pr->p.scr.n_act = pr->p.scr.cap;
        pr->p.scr.Ka = (int)qg::round_up(pr->p.scr.cap, qg::kCtgLanes);
        int e = qg::launch_eval(&p, w, d_x, nullptr, nullptr, sm, 1, d_m, d_v, ex, nullptr);
        if (e == 0) e = qg::launch_screen_select(&p, w, it / R, ex);
        if (e != 0) return hip_fail((hipError_t)e, "kernel launch");
        pr->p.scr.chosen = true;
        ++k;
        continue;
      }
      int64_t len = std::min(n - k, R - it % R);
      for (; len > 0; --len, ++k) {
        int e = qg::launch_eval(&p, w, d_x, nullptr, nullptr, sm_run, 1, d_m, d_v, ex, nullptr);
        if (e != 0) return hip_fail((hipError_t)e, "kernel launch");
      }
    }
    return QG_OK;
  };

  auto run_steps = [&](int64_t n) -> qg_status {
    int64_t left = n;
    if (step_graphs) {
      for (int i = qg::kStepGraphs - 1; i >= 0; --i) {
        const int64_t len = int64_t(1) << i;
        while (left >= len) {
          HIP_TRY(hipGraphLaunch(static_cast<hipGraphExec_t>(pr->p.step_graph[i]), ex),
                  "graph launch");
          left -= len;
        }
      }
    }
    if (profile) {
      for (int64_t k = 0; k < left;) {
        const int nb = (int)std::min<int64_t>(kProfSteps, left - k);
        for (int st = 0; st < nb; ++st) {
          int e = qg::launch_eval(&p, w, d_x, nullptr, nullptr, sm, 1, d_m, d_v, ex,
                                  reinterpret_cast<void**>(&evs[st * kEv]));
          if (e != 0) return hip_fail((hipError_t)e, "kernel launch");
        }
        HIP_TRY(hipEventSynchronize(evs[(nb - 1) * kEv + kKernels]), "event sync");
        for (int st = 0; st < nb; ++st)
          for (int q = 0; q < kKernels; ++q) {
            float ms = 0.f;
            HIP_TRY(hipEventElapsedTime(&ms, evs[st * kEv + q], evs[st * kEv + q + 1]),
                    "elapsed");
            rep->kernel_ms[q] += ms;
            rep->kernel_calls[q] += 1;
          }
        k += nb;
      }
      return QG_OK;
    }
    for (int64_t k = 0; k < left; ++k) {
      int e = qg::launch_eval(&p, w, d_x, nullptr, nullptr, sm, 1, d_m, d_v, ex, nullptr);
      if (e != 0) return hip_fail((hipError_t)e, "kernel launch");
    }
    return QG_OK;
  };

  auto eval_score = [&](double* total, double* terms) -> qg_status {
    int e = qg::launch_eval(&p, w, d_x, nullptr, nullptr, score, 0, nullptr, nullptr, ex, nullptr);
    if (e != 0) return hip_fail((hipError_t)e, "kernel launch");
    HIP_TRY(hipMemcpyAsync(terms, w.terms, QG_NTERMS * sizeof(double), hipMemcpyDeviceToHost, ex),
            "terms read");
    HIP_TRY(hipStreamSynchronize(ex), "sync");
    *total = terms[QG_T_TOTAL];
    return QG_OK;
  };

  hipEvent_t ev_steps0 = static_cast<hipEvent_t>(pr->p.step_ev[0]);
  hipEvent_t ev_steps1 = static_cast<hipEvent_t>(pr->p.step_ev[1]);
  HIP_TRY(hipEventRecord(ev_steps0, ex), "event record");
  int64_t done = 0;
  while (done < o->n_steps) {
    int64_t n = o->n_steps - done;
    if (o->check_every > 0) n = std::min(n, o->check_every - (done % o->check_every));
    n = std::min<int64_t>(n, qg::kSchedCap);
    s = upload(o->iter0 + done + 1, (int)n);
    if (s != QG_OK) return s;
    s = scr ? run_screened(done, n) : run_steps(n);
    if (s != QG_OK) return s;
    done += n;
    // every scheduled step advanced the device counter by one
    pr->p.sched_next = o->iter0 + done + 1;
    if (o->check_every > 0 && (done % o->check_every == 0) && o->z_ed > 0.0) {
      double tot, terms[QG_NTERMS];
      s = eval_score(&tot, terms);
      if (s != QG_OK) return s;
      const double ratio = -tot / o->z_ed;
      if (ratio >= o->stop_ratio) {
        rep->steps_to_gap = done;
        rep->time_to_gap_s = std::chrono::duration<double>(clock::now() - t_start).count();
        break;
      }
    }
  }
  HIP_TRY(hipEventRecord(ev_steps1, ex), "event record");
  HIP_TRY(hipStreamSynchronize(ex), "sync");
  rep->steps_done = done;
  rep->wall_s = std::chrono::duration<double>(clock::now() - t_start).count();
  {
    float ms = 0.f;
    HIP_TRY(hipEventElapsedTime(&ms, ev_steps0, ev_steps1), "elapsed");
    rep->steps_ms = ms;
  }
  if (profile) {
    for (int q = 0; q < kKernels; ++q)
      if (rep->kernel_calls[q]) rep->kernel_ms[q] /= (double)rep->kernel_calls[q];
  }
  if (o->skip_final) {
    rep->final_loss = rep->final_score = std::nan("");
    for (double& t : rep->terms) t = std::nan("");
    return QG_OK;
  }
  // objective at the last schedule point was left in the workspace terms
  double last[QG_NTERMS];
  // on the solve's own stream: a legacy-stream copy would conflict with a
  // graph capture running on another thread
  HIP_TRY(hipMemcpyAsync(last, w.terms, sizeof(last), hipMemcpyDeviceToHost, ex), "terms read");
  HIP_TRY(hipStreamSynchronize(ex), "sync");
  rep->final_loss = last[QG_T_TOTAL];
  double tot;
  s = eval_score(&tot, rep->terms);
  if (s != QG_OK) return s;
  rep->final_score = -tot;
  return QG_OK;
}

// Common checks of a batch; fills the workspaces' device views.
static qg_status check_batch(qg_problem* const* probs, int32_t n, double* const* d_x,
                             double* const* d_m, double* const* d_v, void* const* d_workspace,
                             std::vector<qg::DevWork>* w) {
  if (n < 1 || n > QG_BATCH_MAX || !probs) return fail(QG_ERR_ARG, "bad batch size or problems");
  for (int i = 0; i < n; ++i) {
    qg_status s = check_problem(probs[i]);
    if (s != QG_OK) return s;
    for (int j = 0; j < i; ++j)
      if (probs[j] == probs[i]) return fail(QG_ERR_ARG, "a problem appears twice in the batch");
    if (probs[i]->p.scr.on)
      return fail(QG_ERR_ARG, "batched solves score every contingency: turn screening off");
  }
  w->assign((size_t)n, qg::DevWork{});
  if (!d_x) return QG_OK;  // sizing only
  if (!d_m || !d_v || !d_workspace) return fail(QG_ERR_ARG, "null buffer arrays");
  for (int i = 0; i < n; ++i) {
    if (!d_x[i] || !d_m[i] || !d_v[i] || !d_workspace[i] || !aligned(d_x[i]) ||
        !aligned(d_m[i]) || !aligned(d_v[i]) || !aligned(d_workspace[i]))
      return fail(QG_ERR_ARG, "null or misaligned buffer of scenario " + std::to_string(i));
    (*w)[i] = qg::carve_workspace(&probs[i]->p, d_workspace[i]);
  }
  return QG_OK;
}

static qg::EvalMode batch_mode(const qg_adam_cfg* cfg) {
  qg::EvalMode sm;
  std::memset(&sm, 0, sizeof(sm));
  sm.schedule = 1;
  sm.adam_b1 = cfg->beta1; sm.adam_b2 = cfg->beta2; sm.adam_eps = cfg->eps;
  sm.eps_in_num = cfg->eps_in_numerator;
  return sm;
}

qg_status qg_batch_bytes(qg_problem* const* probs, int32_t n, size_t* bytes) {
  if (!bytes) return fail(QG_ERR_ARG, "null output");
  std::vector<qg::DevWork> w;
  qg_status s = check_batch(probs, n, nullptr, nullptr, nullptr, nullptr, &w);
  if (s != QG_OK) return s;
  std::vector<const qg::Problem*> prs((size_t)n);
  for (int i = 0; i < n; ++i) prs[i] = &probs[i]->p;
  std::vector<const double*> xs((size_t)n, nullptr);
  std::vector<double*> ms((size_t)n, nullptr);
  qg_adam_cfg cfg{0.9, 0.999, 1e-8, 0};
  qg::BatchPlan plan;
  std::string err;
  if (qg::plan_batch(prs.data(), w.data(), n, xs.data(), ms.data(), ms.data(), batch_mode(&cfg),
                     &plan, nullptr, &err) != 0)
    return fail(QG_ERR_ARG, err);
  *bytes = plan.bytes;
  return QG_OK;
}

qg_status qg_solve_batch(qg_problem* const* probs, int32_t n, double* const* d_x,
                         double* const* d_m, double* const* d_v, void* const* d_workspace,
                         void* d_batch, size_t batch_bytes, const qg_solve_opts* o,
                         const qg_adam_cfg* cfg, qg_solve_report* reps, void* stream) {
  using clock = std::chrono::steady_clock;
  if (!d_x || !o || !cfg || !reps) return fail(QG_ERR_ARG, "null argument");
  std::vector<qg::DevWork> w;
  qg_status s = check_batch(probs, n, d_x, d_m, d_v, d_workspace, &w);
  if (s != QG_OK) return s;
  s = check_solve_opts(o, cfg);
  if (s != QG_OK) return s;
  if (o->check_every != 0 || o->profile != 0)
    return fail(QG_ERR_ARG, "batched solves take no gap checks and no profiling");
  if (o->reserved != 0) return fail(QG_ERR_ARG, "reserved field must be 0");
  if (!d_batch || !aligned(d_batch)) return fail(QG_ERR_ARG, "batch buffer null or misaligned");
  const int64_t n_total = o->n_total > 0 ? o->n_total : o->iter0 + o->n_steps;
  hipStream_t user = static_cast<hipStream_t>(stream);
  hipStream_t ex = user ? user : probs[0]->own;
  const qg::EvalMode sm = batch_mode(cfg);

  // kernel arguments and block tables of every problem, in the batch buffer
  std::vector<const qg::Problem*> prs((size_t)n);
  std::vector<const double*> xs((size_t)n);
  for (int i = 0; i < n; ++i) {
    prs[i] = &probs[i]->p;
    xs[i] = d_x[i];
  }
  qg::BatchPlan plan;
  std::vector<unsigned char> image;
  std::string err;
  if (qg::plan_batch(prs.data(), w.data(), n, xs.data(), d_m, d_v, sm, &plan, &image, &err) != 0)
    return fail(QG_ERR_ARG, err);
  if (batch_bytes < plan.bytes)
    return fail(QG_ERR_ARG, "batch buffer too small: need " + std::to_string(plan.bytes));
  HIP_TRY(hipMemcpyAsync(d_batch, image.data(), plan.bytes, hipMemcpyHostToDevice, ex),
          "batch upload");
  HIP_TRY(hipStreamSynchronize(ex), "sync");

  // one graph of gsteps batched steps (six launches each)
  const int gsteps = (int)std::min<int64_t>(16, std::max<int64_t>(1, o->n_steps));
  hipGraphExec_t gexec = nullptr;
  hipEvent_t ev[2] = {nullptr, nullptr};
  auto cleanup = [&]() {
    if (gexec) (void)hipGraphExecDestroy(gexec);
    for (auto& e : ev)
      if (e) (void)hipEventDestroy(e);
  };
  {
    hipGraph_t g;
    hipStream_t cap = probs[0]->own;
    hipError_t e = hipStreamBeginCapture(cap, hipStreamCaptureModeThreadLocal);
    for (int k = 0; k < gsteps && e == hipSuccess; ++k)
      e = (hipError_t)qg::launch_eval_batch(plan, d_batch, cap);
    hipError_t e2 = hipStreamEndCapture(cap, &g);
    if (e == hipSuccess) e = e2;
    if (e == hipSuccess) {
      e = hipGraphInstantiate(&gexec, g, nullptr, nullptr, 0);
      (void)hipGraphDestroy(g);
    }
    if (e == hipSuccess) e = hipEventCreate(&ev[0]);
    if (e == hipSuccess) e = hipEventCreate(&ev[1]);
    if (e != hipSuccess) { cleanup(); return hip_fail(e, "batch graph capture"); }
  }

  const auto t_start = clock::now();
  std::vector<double> table((size_t)qg::kSchedCap * qg::kSchedStride, 0.0);
  for (int i = 0; i < n; ++i) {  // their tables and counters are rewritten here
    probs[i]->p.sched_base = -1;
    probs[i]->p.sched_next = -1;
  }
  hipError_t e = hipEventRecord(ev[0], ex);
  if (e != hipSuccess) { cleanup(); return hip_fail(e, "event record"); }
  int64_t done = 0;
  while (done < o->n_steps) {
    const int64_t nc = std::min<int64_t>(o->n_steps - done, qg::kSchedCap);
    fill_schedule(table.data(), o, cfg, n_total, o->iter0 + done + 1, (int)nc);
    for (int i = 0; i < n; ++i) {
      e = hipMemcpyAsync(w[i].sched, table.data(), (size_t)nc * qg::kSchedStride * sizeof(double),
                         hipMemcpyHostToDevice, ex);
      if (e == hipSuccess && qg::launch_set_step(&probs[i]->p, w[i], 0, ex) != 0)
        e = hipGetLastError();
      if (e != hipSuccess) { cleanup(); return hip_fail(e, "schedule upload"); }
    }
    int64_t left = nc;
    for (; left >= gsteps; left -= gsteps) {
      e = hipGraphLaunch(gexec, ex);
      if (e != hipSuccess) { cleanup(); return hip_fail(e, "graph launch"); }
    }
    for (; left > 0; --left)
      if (qg::launch_eval_batch(plan, d_batch, ex) != 0) {
        cleanup();
        return hip_fail(hipGetLastError(), "kernel launch");
      }
    done += nc;
  }
  e = hipEventRecord(ev[1], ex);
  if (e == hipSuccess) e = hipStreamSynchronize(ex);
  if (e != hipSuccess) { cleanup(); return hip_fail(e, "sync"); }
  const double wall = std::chrono::duration<double>(clock::now() - t_start).count();
  float steps_ms = 0.f;
  (void)hipEventElapsedTime(&steps_ms, ev[0], ev[1]);
  cleanup();
  // reports: the objective at the last schedule point and the score
  for (int i = 0; i < n; ++i) {
    qg_solve_report* r = &reps[i];
    std::memset(r, 0, sizeof(*r));
    r->steps_done = done;
    r->steps_to_gap = -1;
    r->time_to_gap_s = -1.0;
    r->wall_s = wall;
    r->steps_ms = steps_ms;
    if (o->skip_final) {
      r->final_loss = r->final_score = std::nan("");
      for (double& t : r->terms) t = std::nan("");
      continue;
    }
    double last[QG_NTERMS];
    HIP_TRY(hipMemcpyAsync(last, w[i].terms, sizeof(last), hipMemcpyDeviceToHost, ex),
            "terms read");
    HIP_TRY(hipStreamSynchronize(ex), "sync");
    r->final_loss = last[QG_T_TOTAL];
    qg::EvalMode score{};
    score.schedule = 0;
    score.eps = 0.0;
    score.beta = 1.0;
    score.rho_s = o->rhof;
    if (qg::launch_eval(&probs[i]->p, w[i], d_x[i], nullptr, nullptr, score, 0, nullptr, nullptr,
                        ex, nullptr) != 0)
      return hip_fail(hipGetLastError(), "kernel launch");
    HIP_TRY(hipMemcpyAsync(r->terms, w[i].terms, QG_NTERMS * sizeof(double),
                           hipMemcpyDeviceToHost, ex), "terms read");
    HIP_TRY(hipStreamSynchronize(ex), "sync");
    r->final_score = -r->terms[QG_T_TOTAL];
  }
  return QG_OK;
}

qg_status qg_debug_fetch(const qg_problem* pr, const void* d_workspace, const char* name,
                         void* host, size_t bytes, void* stream) {
  qg_status s = check_problem(pr);
  if (s != QG_OK) return s;
  if (!d_workspace || !name || !host) return fail(QG_ERR_ARG, "null argument");
  const qg::Problem& p = pr->p;
  qg::DevWork w = qg::carve_workspace(&p, const_cast<void*>(d_workspace));
  const size_t D = sizeof(double);
  struct Item { const char* n; const void* ptr; size_t bytes; };
  const Item items[] = {
      {"F", w.F, (size_t)p.T * p.Lp * D},       {"Fk", w.Fk, (size_t)p.T * p.Kp * D},
      {"q2", w.q2, (size_t)p.T * p.Lp * D},     {"thr", w.thr, (size_t)p.T * p.Lp * D},
      {"lamp", w.lamp, (size_t)p.T * p.N * D},  {"lamq", w.lamq, (size_t)p.T * p.N * D},
      {"zval", w.zval, (size_t)p.T * p.Kp * D}, {"gfT", w.gfT, (size_t)p.Lp * p.Tp * D},
      {"gpdc", w.gpdc, (size_t)p.nsplit * p.T * p.G16 * D},
      {"qtot", w.qtot, (size_t)p.T * p.Lp * D},
      {"params", w.params, (size_t)qg::kParams * D}, {"terms", w.terms, (size_t)QG_NTERMS * D}};
  for (const Item& it : items) {
    if (std::strcmp(it.n, name) != 0) continue;
    if (bytes > it.bytes) return fail(QG_ERR_ARG, "request larger than the array");
    hipStream_t st = static_cast<hipStream_t>(stream);
    HIP_TRY(hipMemcpyAsync(host, it.ptr, bytes, hipMemcpyDeviceToHost, st), "debug copy");
    HIP_TRY(hipStreamSynchronize(st), "sync");
    return QG_OK;
  }
  return fail(QG_ERR_ARG, std::string("unknown array ") + name);
}

void qg_destroy_problem(qg_problem* pr) {
  if (!pr) return;
  drop_graph(pr->p);
  release_solve_resources(pr->p);
  if (pr->own) (void)hipStreamDestroy(pr->own);
  pr->alive = false;
  delete pr;
}

}  // extern "C"
