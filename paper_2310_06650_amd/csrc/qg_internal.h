// Internal types shared by the host builder, the kernels and the C ABI.
#pragma once

#include <cstddef>
#include <cstdint>
#include <string>
#include <vector>

#include "qg.h"

namespace qg {

constexpr int kAlign = 256;
constexpr int kMaxT = 64;          // periods per problem (4 MFMA row tiles of 16)
constexpr int kBlock = 256;        // threads per block of the streaming kernels
constexpr int kCtgLanes = 64;      // contingencies per wavefront in the map-reduce
constexpr int kParams = 16;        // doubles in the per-step parameter block
constexpr int kCtgMaxTc = 8;            // periods per block of the contingency kernel
constexpr int kCtgLdsBytes = 64 * 1024; // LDS budget of one contingency block
constexpr int kAdjStepsPerBlock = 32;   // MFMA k-steps per block of the adjoint product
constexpr int kSchedCap = 2048;         // solve steps per uploaded schedule table
constexpr int kSchedStride = 16;        // doubles per step in the schedule table
constexpr int kStepGraphs = 6;          // cached step graphs of 1, 2, 4, ..., 32 steps

inline int64_t round_up(int64_t a, int64_t b) { return (a + b - 1) / b * b; }

// Parameter block layout (DevWork::params): the homotopy and step sizes of
// the step being evaluated.
enum ParamSlot { PB_EPS = 0, PB_BETA = 1, PB_RHO = 2, PB_ALPHA = 4, PB_BC1 = 10, PB_BC2 = 11 };

// Storage kind of the outage factors, from the build flags.
enum LodfKind { kLodfF64 = 0, kLodfF32 = 1, kLodfBF16 = 2 };
inline int lodf_kind_of(uint32_t flags) {
  return (flags & QG_FLAG_CTG_BF16) ? kLodfBF16 : (flags & QG_FLAG_CTG_FP32) ? kLodfF32 : kLodfF64;
}
inline size_t lodf_elem_bytes(int kind) { return kind == kLodfF64 ? 8 : kind == kLodfF32 ? 4 : 2; }

// Device view of the constant arena (all pointers into caller memory).
struct DevProblem {
  int N, L, G, T, M, K;
  int Lp;    // L padded to 64 (row count of the outage-factor tile space)
  int Kp;    // K padded to 64 (one wavefront of contingencies)
  int G16;   // G padded to 16 (MFMA output columns of the adjoint product)
  int G4;    // G padded to 4  (MFMA reduction depth of the flow product)
  int Tp;    // T padded to 16 (MFMA rows)
  int twoL;  // endpoint slots per period
  // branches
  const int* br_from; const int* br_to; const int* slot_fr; const int* slot_to;
  const double* br_g; const double* br_b; const double* br_bh; const double* br_smax;
  const double* ctg_smax;   // [Lp] contingency rating (1 on padding)
  const double* ctg_smax2;  // [Lp] its square
  const int* kof;           // [Lp] contingency index of a branch, -1 if none
  const int* brk;           // [Kp] outaged branch of a contingency (0 on padding)
  // buses
  const int* bptr;          // [N+1] endpoint-slot ranges (bus-sorted)
  const int* gptr;          // [N+1] generator ranges
  const int* glist;         // [G]   generators sorted by bus
  const double* vmin; const double* vmax;
  // generators
  const int* gen_bus;
  const double *pmin, *pmax, *qmin, *qmax, *rmax, *ru, *rd, *rusu, *rdsd, *p0, *u0;
  const double *con, *csu, *csd, *cr;
  const double *seg_cost, *seg_size, *pcum;   // [G*M]
  // periods
  const double* load_p; const double* load_q;  // [T*N]
  const double* dt; const double* rsv_req; const double* sum_load;  // [T]
  // sensitivities, restricted to generator buses
  const double* isf_gT;  // [G4][Lp]  ISF[l][bus(j)] - rsum[l]/N, zero padded (B of the flow product)
  const double* isf_ga;  // [Lp][G16] ISF[l][bus(j)] - rsum[l]/N (B of the adjoint product)
  const double* cload;   // [T][Lp]   sum_i ISF[l][i] load_p[t][i] - rsum[l] sum_load[t] / N
  const double* rsum;    // [Lp]      sum_i ISF[l][i]
  const double* lodf;    // [Lp][Kp]  outage factors; NaN marks (k,k) and padding
  const float* lodf32;   //           the same in FP32 (QG_FLAG_CTG_FP32)
  const uint16_t* lodf16;  //         the same in BF16 (QG_FLAG_CTG_BF16)
  int lodf_kind;         // 0 FP64, 1 FP32, 2 BF16 (one of the three pointers is set)
  const double* lmaxh;   // [Lp/4][Kp/64] max |lodf| (as stored) of each 4-branch group and
                         // 64-contingency block, NaN left out (null with QG_FLAG_CTG_NO_SKIP)
  int ctg_sum;           // 1: per-period sum over contingencies instead of max + mean
  // prices
  double c_p, c_q, c_s, c_ang, ang_max, c_rsv, rho, vload;
};

// Device view of the caller's workspace.
struct DevWork {
  double* params;      // [kParams] parameters of the step being evaluated
  int64_t* step;       // [1] index of the current step in the schedule table
  double* sched;       // [kSchedCap][kSchedStride] per-step eps, beta, rho_s, alpha[6], bc1, bc2
  double* snext;       // [kSchedStride] the schedule row of the next scheduled evaluation
  double* fh;          // [Lp/8 + 1][T][16] (+ 8 rows): per 8-branch tile and period, F and
                       // the test radii thr of branches 0-3, then of branches 4-7 (the
                       // same values as F, thr); the spare tile and rows absorb the
                       // map-reduce's prefetch
  double* epP; double* epQ;      // [T][2L] branch flows at bus-sorted endpoint slots
  double* bco;         // [9][T][L] per-branch reverse coefficients
  double* q2;          // [T][Lp]  max(q_fr^2, q_to^2)
  double* F;           // [T][Lp]  base-case DC flows
  double* Fk;          // [T][Kp]  flows of the outaged branches
  double* lamp; double* lamq;    // [T][N] balance multipliers
  double* gdev;        // [4][T][G] device-only partials of p, q, r, u
  double* zpart; double* spart;  // [nLb][T][Kp]
  double* rpart; double* qpart;  // [nKb][T][Lp]
  double* smean;       // [T][Kp]
  double* zval;        // [T][Kp]
  double* gfT;         // [Lp][Tp] dL/dF, transposed
  double* qtot;        // [T][Lp]  dL/d qmax2
  double* gpdc;        // [nsplit][T][G16] DC part of dL/dp (split-K partials)
  double* epGV; double* epGT;    // [T][2L] endpoint adjoints
  double* tpart;       // term partial sums
  double* terms;       // [QG_NTERMS] last evaluated terms
  double* drs;         // [T]       reserve-shortfall derivative, subtracted from dL/dr
  double* zmaxp;       // [T][nKc]  per-chunk worst penalty
  double* zargp;       // [T][nKc]  its contingency index
  double* zsump;       // [T][nKc]  per-chunk penalty sum
  double* kstar;       // [T]       worst contingency of the period
  double* smaxp;       // [T][nLc]  per-chunk dL/dF of the worst contingency's own branch
  double* lamg; double* lamqg;   // [T][G] balance multipliers at each generator's bus
  double* isfk;        // [T][G16]  ISF[br(k*_t)][bus(j)] - rowsum/N of the period's worst outage
  double* thr;         // [T][Lp]  test radius of the outage flows (k_ctg_pm)
  // which partials were stored (the rest are all zero and not written):
  uint8_t* zflag;      // [T][nKb_max][nLb_max] z/S partials of (t, k-block, l-block)
  uint8_t* rflag;      // [T][Lp/8][rflag_stride] R/Q partials of (t, 8 branches, k-block)
};

// Row stride of DevWork::rflag: k-blocks rounded up to 16 (16-byte loads).
inline int rflag_stride(int nKb_max) { return (nKb_max + 15) / 16 * 16; }

// Offsets of the term partial sums inside DevWork::tpart.
struct TermOffsets {
  int br, ang, dev, pen, rsv, bal, cmax, cmean, total;
};

// Tile shape of the contingency map-reduce.
struct CtgTile {
  int bl;   // branches per wavefront (8, 16 or 32)
  int wl;   // wavefronts per block, stacked along branches
  int tc;   // periods per block (the period range is split over grid.z)
  int lt;   // consecutive tiles of wl * bl branches per block (split: of 8
            // branches, shared by the block's wavefronts)
  int split = 0;  // 1: period-split blocks (bl = 8, tc periods per wavefront)
};

// Homotopy source of one evaluation.
struct EvalMode {
  int schedule;          // 0: homotopy from args, 1: from the solve schedule
  double eps, beta, rho_s;
  // schedule (mode 1)
  int64_t n_total;
  double alpha0[QG_NCLASS], alphaf[QG_NCLASS];
  double eps0, epsf, beta0, betaf, rho0, rhof;
  double adam_b1, adam_b2, adam_eps;
  int eps_in_num;
  int screened;          // 1: score only the problem's chosen contingency set
};

struct Problem;

// Contingency screening (Alg. 2): the set of contingencies scored by the
// screened steps, and its outage factors gathered into contiguous columns.
// All device arrays live in the caller's screening buffer.
struct Screen {
  bool on = false;
  bool chosen = false;       // a set has been selected or given
  int n_top = 0;             // worst-set slots
  int n_act = 0;             // contingencies scored (slots in use)
  int cap = 0;               // most slots the buffer holds
  int Ka = 0;                // n_act padded to 64: row stride of lodf_act
  double zeta = 0.0;         // severity threshold of the worst set
  int refresh = 0;           // steps between exact refresh steps in qg_solve
  uint64_t seed = 0;         // seed of the random draw
  int* act_k = nullptr;      // [Kp] slot -> contingency (0 past n_act)
  int* act_slot = nullptr;   // [Kp] contingency -> slot, -1 if not scored
  int* top = nullptr;        // [Kp] worst-set flags of the last selection
  int* sel = nullptr;        // [Kp] chosen flags of the last selection
  double* sev = nullptr;     // [Kp] severities of the last refresh
  uint64_t* key = nullptr;   // [Kp] draw keys of the last refresh
  void* lodf_act = nullptr;  // [Lp][Ka] outage factors of the slots, NaN past n_act
  size_t bytes = 0;          // bytes of the buffer in use
};
// Bytes of a screening buffer for up to cap scored contingencies, and the
// carve of one (sets the pointers of sc).
size_t screen_bytes(const Problem& p, int cap);
void carve_screen(const Problem& p, void* buf, int cap, Screen* sc);

struct Problem {
  int device = -1;  // HIP device current at build (the arena's device)
  // sizes
  int N, L, G, T, M, K;
  int Lp, Kp, G16, G4, Tp;
  int64_t n_x;
  uint32_t flags;
  std::vector<int32_t> ctg;
  // launch geometry
  int nb_br;      // blocks of the per-(t, branch) kernels
  int nb_bus;     // blocks of the per-(t, bus chunk) kernels
  int bus_chunks; // bus chunks per period
  int nb_gen;     // blocks of the per-(t, generator) final stage
  int nsplit;     // reduction splits of the adjoint product
  int nKc, nLc;   // chunks of Kp (64 wide) and Lp (256 wide)
  CtgTile tile;
  int nLb, nKb;   // partial counts of the contingency map-reduce
  int nLb_max, nKb_max;
  TermOffsets toff;
  size_t const_bytes, work_bytes;
  DevProblem dp;
  void* arena = nullptr;
  // graph cache of qg_solve: graph_exec holds one screening refresh cycle;
  // step_graph[i] holds 2^i plain steps (i < kStepGraphs), so that a solve of
  // any length replays cached graphs (n = sum of powers of two)
  void* graph_exec = nullptr;
  void* step_graph[kStepGraphs] = {};
  const void* graph_key[5] = {nullptr, nullptr, nullptr, nullptr, nullptr};
  int graph_steps = 0;
  EvalMode graph_mode{};
  CtgTile graph_tile{};   // contingency tile the cached graph was captured with
  // host data kept for load updates (same grid, new loads)
  std::vector<double> isf_host;  // [L][isf_np] injection shift factors (reference column 0)
  int isf_np = 0;
  std::vector<double> rsum_host; // [Lp] ISF row sums
  std::vector<double> dt_host;   // [T]
  double load_value = 0.0;
  Screen scr;
  // pinned host staging of the schedule table (two halves, each reused only
  // after the event recorded behind its last upload), and the events that
  // time a solve's steps; created at the first qg_solve
  double* sched_host = nullptr;
  void* sched_ev[2] = {nullptr, nullptr};
  // what the device schedule table holds: rows of iterations
  // [sched_base, sched_base + sched_rows) for the schedule sched_key (bytes
  // of the solve options and Adam constants the rows depend on, and the
  // workspace they live in); sched_base < 1 when unknown
  unsigned char sched_key[192] = {};
  int64_t sched_base = -1;
  int sched_rows = 0;
  // iteration the device step counter and the copied-ahead row point at
  // after the last scheduled step (-1: unknown); a call continuing there
  // needs no counter reset
  int64_t sched_next = -1;
  void* step_ev[2] = {nullptr, nullptr};
};

// Host build products (before upload).
struct HostBuild {
  std::vector<unsigned char> image;  // arena image
  size_t const_bytes = 0;
};

// Set the thread-local error text; returns s.
qg_status fail(qg_status s, const std::string& msg);

// Validate the description and find the contingency set.  Fills p's sizes.
qg_status plan_problem(const qg_grid_desc* d, const qg_build_opts* o, Problem* p);
// Factor, sensitivities and the arena image.
qg_status build_arena(const qg_grid_desc* d, const qg_build_opts* o, Problem* p,
                      HostBuild* hb);
void rebase_pointers(Problem* p, void* arena);
// Load-dependent parts of the arena for new loads: byte offsets and host
// values of load_p, load_q, rsv_req, sum_load and the flow constant, and the
// consumer value.  Uses the ISF kept at build.
struct LoadBlock {
  size_t off_lp, off_lq, off_rsv, off_sum, off_cload;
  std::vector<double> sum_load, cload;
  double vload;
};
void load_block(const Problem* p, const double* load_p, LoadBlock* out);
DevWork carve_workspace(const Problem* p, void* ws);
int default_ctg_tc(const Problem& p, int wl);
int default_ctg_lt(const Problem& p, const CtgTile& t);  // tiles per block for tile t
void apply_ctg_tile(Problem* p, const CtgTile& t);        // set the tile and the l-block count
CtgTile default_ctg_tile(const Problem& p);               // the tile a new problem starts with
int ctg_tc_cap(int wl);  // most periods per block the LDS budget allows

// Kernel launchers (qg_kernels.hip).  A step is kStages kernels.
constexpr int kStages = 6;
int launch_eval(const Problem* p, const DevWork& w, const double* x, double* grad,
                double* terms_out, const EvalMode& mode, int fuse_adam, double* m,
                double* v, void* stream, void** events /* nullable [QG_NKERNELS] */);
// Mean duration of one kernel of the step (0..kStages-1), launched reps times
// back to back after a full evaluation at x has produced its inputs.
int time_stage(const Problem* p, const DevWork& w, const double* x, const EvalMode& mode,
               int stage, int reps, void* stream, double* mean_ms);
int launch_adam(const Problem* p, double* x, double* m, double* v, const double* g,
                const double lr[QG_NCLASS], double bc1, double bc2, double b1,
                double b2, double eps, int eps_in_num, void* stream);
int launch_set_step(const Problem* p, const DevWork& w, int64_t value, void* stream);

// Batched step of independent problems: kStages launches for all of them.
// The caller's batch buffer holds every problem's kernel arguments and, per
// stage, a table of the launch's blocks (problem index << 22 | block of that
// problem); stage 1, the contingency map-reduce, is a persistent launch that
// takes its blocks' work items from a counter reset by stage 0.
struct BatchPlan {
  int n = 0;
  int nblk[kStages] = {};      // blocks (stage 1: work items) of each batched launch
  size_t off_args = 0;         // byte offsets into the batch buffer
  size_t off_tab[kStages] = {};
  size_t off_ctr = 0;
  size_t bytes = 0;            // size of the batch buffer
  int lodf_kind = 0;
  int pm_grid = 0;             // blocks of the persistent map-reduce
  bool skip = false;           // the map-reduce takes the skip test (FP64 factors)
};
constexpr int kBatchLocBits = 22;                  // block index bits of a table entry
constexpr int kBatchWl = 4;                        // wavefronts per map-reduce block
constexpr int kBatchTcw = 4;                       // periods per map-reduce wavefront
// Sizes, validation and (image != nullptr) the host image of a batch buffer
// for problems whose steps take x[i], m[i], v[i] and workspaces ws[i]; 0 or
// a message in *err.
int plan_batch(const Problem* const* prs, const DevWork* ws, int n, const double* const* x,
               double* const* m, double* const* v, const EvalMode& mode, BatchPlan* plan,
               std::vector<unsigned char>* image, std::string* err);
int launch_eval_batch(const BatchPlan& plan, void* d_buf, void* stream);
int launch_check_finite(const Problem* p, const double* x, int* flag, void* stream);
// Screening (qg_screen.hip): choose the set from the severities of the last
// exact evaluation (its z_tk and homotopy in the workspace), then gather its
// outage factors; or gather only, for a set uploaded by the host.  round < 0:
// the refresh index follows from the schedule row of the step just taken.
int launch_screen_select(const Problem* p, const DevWork& w, int64_t round, void* stream);
int launch_screen_gather(const Problem* p, void* stream);

}  // namespace qg
