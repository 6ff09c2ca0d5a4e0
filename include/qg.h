/*
 * qg.h -- C ABI of the MI355X hot path of the Adam-based, reserve- and
 * security-constrained AC unit-commitment solver (Chevalier, "A Parallelized,
 * Adam-Based Solver for Reserve and Security Constrained AC Unit Commitment",
 * PSCC 2024).
 *
 * One solver step is a forward and reverse pass of the penalised market-
 * surplus objective (Section II-C, eq. (nlp_updated); gradient eq. (grads))
 * over every period, bus, branch, generator and single-branch outage
 * contingency (Section II-E), followed by the modified Adam update and the
 * clip to the variable box (Section II-G, Alg. 3).
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * - Sizes: N buses, L branches, G generators, T periods, M cost blocks per
 *   generator, K contingencies.
 * - Host arrays are read during the call only and never retained.
 * - Device buffers are allocated by the caller (the library never allocates
 *   device memory); each must be 256-byte aligned.  The library keeps
 *   non-owning pointers to the constant arena until qg_destroy_problem.
 * - "stream" is a hipStream_t passed as void*; NULL means the default stream.
 *   qg_eval_grad and qg_adam_step only enqueue work (no host synchronisation);
 *   qg_build_problem and qg_solve synchronise the stream before returning.
 * - The variable vector x (length n_x = 2TN + 4TG, FP64) holds six blocks in
 *   this order, each period-major (entry (t, e) at t*E + e):
 *     V  [T][N] voltage magnitudes      TH [T][N] voltage angles (rad)
 *     P  [T][G] active output           Q  [T][G] reactive output
 *     R  [T][G] spinning reserve        U  [T][G] relaxed on/off status
 *   These are the basis variables of Section II-B (Omega_c, Omega_d) that
 *   the reduced model keeps.
 * - Every call returns a qg_status.  On error the outputs are left untouched
 *   and qg_last_error() returns a description (thread-local).  No exception
 *   or abort crosses the ABI.
 */
#ifndef QG_H
#define QG_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  QG_OK = 0,
  QG_ERR_ARG = 1,        /* bad size, index, value, null or misaligned pointer */
  QG_ERR_TOPOLOGY = 2,   /* disconnected grid, or a listed outage that islands */
  QG_ERR_SINGULAR = 3,   /* non-positive pivot in the susceptance factor */
  QG_ERR_NONFINITE = 4,  /* NaN/Inf found where QG_FLAG_CHECK_FINITE asked */
  QG_ERR_DEVICE = 5,     /* a HIP runtime call failed */
  QG_ERR_STATE = 6       /* call out of order (e.g. destroyed handle) */
} qg_status;

/* Slots of the per-term objective vector (the families of Table 1's
 * penalty breakdown, for the reduced model). */
enum {
  QG_T_DEV = 0,      /* block-bid energy, no-load, start-up/shut-down, reserve cost */
  QG_T_BAL = 1,      /* power-balance soft-abs penalties (Example 4) */
  QG_T_BR = 2,       /* branch thermal soft-ReLU penalties (Example 1) */
  QG_T_ANG = 3,      /* branch angle-difference soft-ReLU penalties */
  QG_T_PEN = 4,      /* penalised linear device constraints rho*sigma(Ax) */
  QG_T_RSV = 5,      /* reserve shortfall */
  QG_T_CTG_MAX = 6,  /* sum over periods of the worst contingency penalty */
  QG_T_CTG_MEAN = 7, /* sum over periods of the mean contingency penalty */
  QG_T_LOADVAL = 8,  /* consumer value (constant, enters with a minus sign) */
  QG_T_TOTAL = 9,    /* the objective L = sum of slots 0..7 minus slot 8 */
  QG_NTERMS = 10
};

/* Variable classes (the six blocks of x). */
enum { QG_C_V = 0, QG_C_TH = 1, QG_C_P = 2, QG_C_Q = 3, QG_C_R = 4, QG_C_U = 5,
       QG_NCLASS = 6 };

enum { QG_CTG_ALL_NONBRIDGE = 0, QG_CTG_LIST = 1 };

/* Flags for qg_build_opts.flags */
#define QG_FLAG_CHECK_FINITE 0x1u /* qg_eval_grad rejects non-finite x (syncs) */
/* Precision of the contingency map-reduce (eqs. (rank_correct), (sfr_pen)-(zctg)
 * and their reverse).  Default: FP64 throughout.  With one of these flags the
 * outage factors are stored in FP32 or in BF16 (rounded to nearest even), and
 * the post-outage flows, penalties, derivatives and their sums over branches
 * and contingencies are computed in FP32; their partial sums are handed to
 * the FP64 remainder of the step.  The base-case flows, the sensitivity
 * products, every other term and the Adam moments stay FP64.  At most one of
 * the two may be set (ARG otherwise). */
#define QG_FLAG_CTG_FP32 0x2u
#define QG_FLAG_CTG_BF16 0x4u
/* Aggregation over contingencies.  Default: per period the worst penalty
 * plus the mean, max_k z_tk + (1/K) sum_k z_tk (the two contingency rows of
 * Table 1).  With this flag: per period the plain sum sum_k z_tk (every
 * scored contingency's gradient handed to Adam with weight 1, as Alg. 2
 * accumulates them); the sum goes into the QG_T_CTG_MEAN slot and
 * QG_T_CTG_MAX is 0. */
#define QG_FLAG_CTG_SUM 0x8u
/* Bound-based skip in the contingency map-reduce.  Default: with every
 * contingency scored and blocks of 4 to 64 / (periods per wavefront) branch
 * tiles, a half row (4 branches, one period, 64 contingencies) is passed
 * over when |F_tl| + max|LODF_lk| max|F_tk| proves every post-outage flow
 * within its test radius, the factors' maximum taken as stored (FP64, FP32
 * or BF16) and with margins that cover the rounding of the exact test of
 * that precision, so the results are bitwise those of testing every
 * element.  With this flag every element is tested (a reference for that
 * claim). */
#define QG_FLAG_CTG_NO_SKIP 0x10u

/* Grid description: host arrays, all FP64 per unit (100 MVA base) unless
 * stated; prices in $ per pu-hour, durations in hours. */
typedef struct {
  int32_t n_bus, n_branch, n_gen, n_period, n_seg;
  /* branches [L]: endpoints, series r and x (x > 0, r >= 0), total line
   * charging b_ch, base-case and contingency apparent-power ratings */
  const int32_t *br_from, *br_to;
  const double *br_r, *br_x, *br_bch, *br_smax, *br_smax_ctg;
  /* generators [G] */
  const int32_t *gen_bus;
  const double *gen_pmin, *gen_pmax, *gen_qmin, *gen_qmax, *gen_rmax;
  const double *gen_ru, *gen_rd;       /* ramp limits, pu per hour, when on */
  const double *gen_ru_su, *gen_rd_sd; /* ramp allowance while starting/stopping */
  const double *gen_p0, *gen_u0;       /* output and status before period 0 */
  const double *gen_c_on, *gen_c_su, *gen_c_sd, *gen_c_r;
  /* cost blocks [G*M], row-major per generator, marginal cost and size */
  const double *gen_seg_cost, *gen_seg_size;
  /* loads [T*N] period-major; reserve requirement and duration [T] */
  const double *load_p, *load_q;
  const double *reserve_req, *dt;
  const double *v_min, *v_max;         /* [N] */
  double c_p, c_q;     /* power-balance prices */
  double c_s;          /* branch thermal (base and contingency) price */
  double c_ang;        /* angle-difference price */
  double ang_max;      /* angle-difference limit, rad */
  double c_rsv;        /* reserve-shortfall price */
  double rho;          /* penalty weight of the linear device constraints */
  double load_value;   /* consumer value per pu-hour of load */
} qg_grid_desc;

typedef struct {
  int32_t ref_bus;          /* reference bus of the reduced susceptance factor */
  int32_t ctg_mode;         /* QG_CTG_ALL_NONBRIDGE or QG_CTG_LIST */
  const int32_t *ctg_list;  /* [n_ctg] outaged branch per contingency (LIST) */
  int32_t n_ctg;
  uint32_t flags;
} qg_build_opts;

typedef struct {
  size_t const_bytes;      /* device bytes of the constant arena */
  size_t workspace_bytes;  /* device bytes of the per-call workspace */
  int64_t n_x;             /* length of x */
  int32_t n_ctg;           /* K actually used */
} qg_sizes;

typedef struct {
  int64_t off[QG_NCLASS], len[QG_NCLASS];
} qg_layout;

/* Homotopy state of one evaluation (Section II-G): soft-function width eps,
 * penalty scale beta and the multiplier of rho. */
typedef struct {
  double eps, beta, rho_scale;
} qg_homotopy;

typedef struct {
  double beta1, beta2, eps;
  int32_t eps_in_numerator; /* 1: the update printed in Alg. 3, (m_hat+eps)/(sqrt(v_hat)+eps) */
} qg_adam_cfg;

typedef struct {
  int64_t n_steps;       /* Adam steps to run in this call */
  int64_t iter0;         /* steps already taken (resume); first step is iter0+1 */
  int64_t n_total;       /* schedule horizon tf; 0 means iter0 + n_steps */
  int64_t check_every;   /* score check period (0: never) */
  double alpha0[QG_NCLASS], alphaf[QG_NCLASS]; /* eqs. (norm_t)-(step_size) per class */
  double eps0, epsf;     /* eps on the same reflected-sigmoid curve */
  double beta0, betaf;   /* homotopy scale, linear in the iteration */
  double rho0, rhof;     /* penalty multiplier, linear in the iteration */
  double z_ed;           /* copper-plate bound (Proj. 3) for the gap stop; 0: none */
  double stop_ratio;     /* stop once score / z_ed >= stop_ratio (if z_ed > 0) */
  int32_t use_graph;     /* 1: replay captured HIP graphs; 0: plain launches */
  int32_t profile;       /* 1: time each kernel with events (plain launches) */
  int32_t skip_final;    /* 1: no end-of-call score evaluation and no read of the
                          * last objective (final_loss, final_score and terms are
                          * NaN): the call ends with the last step */
  int32_t reserved;      /* must be 0 */
} qg_solve_opts;

#define QG_NKERNELS 8
typedef struct {
  int64_t steps_done;
  int64_t steps_to_gap;      /* first checked step with ratio >= stop_ratio, else -1 */
  double wall_s;             /* host wall time of the call */
  double time_to_gap_s;      /* wall time until steps_to_gap, else -1 */
  double final_loss;         /* objective at the last schedule point */
  double final_score;        /* -L at eps = 0, beta = 1, rho_scale = rhof */
  double terms[QG_NTERMS];   /* score-point terms at the end */
  /* mean duration per launch when profile = 1, in stream order: k_forward,
   * k_ctg_main, k_ctg_zred, k_ctg_asm, k_adjoint, k_final (slots 6, 7 unused) */
  double kernel_ms[QG_NKERNELS];
  int64_t kernel_calls[QG_NKERNELS];
  /* device time of the steps, from HIP events on the solve's stream around
   * them (the schedule upload, every step and any gap checks in between;
   * not the end-of-call score): milliseconds */
  double steps_ms;
} qg_solve_report;

typedef struct qg_problem qg_problem;

/*
 * Sizes of the device buffers a problem needs.  Host-only: validates the
 * description, finds the contingency set (non-islanding single-branch
 * outages; Section II-E) and returns the arena and workspace sizes.
 * Errors: ARG (sizes, indices, values), TOPOLOGY (disconnected grid, listed
 * outage that islands).
 */
qg_status qg_problem_sizes(const qg_grid_desc* desc, const qg_build_opts* opts,
                           qg_sizes* out);

/*
 * Build a problem: topology, contingency set, the FP64 factor of the reduced
 * susceptance matrix (eq. (Yb_solve)), injection shift factors (the
 * factor applied to unit injections, eq. (p_flow)) and line outage
 * distribution factors (the rank-1 outage correction of eq. (rank_correct)
 * expressed on flows); copies everything into d_const_arena (caller-owned,
 * const_bytes long) on the given stream and synchronises it.
 * Errors: ARG, TOPOLOGY, SINGULAR, DEVICE.  *out is set only on success.
 */
qg_status qg_build_problem(const qg_grid_desc* desc, const qg_build_opts* opts,
                           void* d_const_arena, size_t const_bytes, void* stream,
                           qg_problem** out);

/*
 * The host part of qg_build_problem alone: validates the description, finds
 * the contingency set, factors the reduced susceptance matrix (eq.
 * (Yb_solve)), forms the shift factors (eq. (p_flow)) and outage factors
 * (eq. (rank_correct)), and writes the constant arena's image into
 * host_image (caller-owned host memory of at least const_bytes bytes; the
 * bytes qg_build_problem uploads).  No device work.
 * Errors: ARG, TOPOLOGY, SINGULAR.
 */
qg_status qg_build_image(const qg_grid_desc* desc, const qg_build_opts* opts, void* host_image,
                         size_t bytes);

/*
 * New loads on the same grid (warm-start workflows: the topology, the factor
 * and the outage factors are kept): load_p, load_q [T*N] period-major and
 * reserve_req [T], host arrays read during the call.  Re-derives the
 * load-dependent constants (total load, the flow constant ISF load - rowsum
 * total / N, the consumer value), uploads them into the constant arena on the
 * stream and synchronises it; a step graph cached by qg_solve is dropped.
 * Errors: ARG (null or non-finite input), DEVICE.
 */
qg_status qg_update_loads(qg_problem* prob, const double* load_p, const double* load_q,
                          const double* reserve_req, void* stream);

/* Offsets and lengths of the six blocks of x. */
qg_status qg_layout_of(const qg_problem* prob, qg_layout* out);

/* Copy the contingency list actually used (K entries) into host memory. */
qg_status qg_ctg_list(const qg_problem* prob, int32_t* out, int32_t capacity);

/*
 * Objective terms and gradient at x (Section II-C/II-E/II-F; gradient of
 * eq. (grads) with every contingency included).
 *   d_x         device [n_x], read only
 *   d_grad      device [n_x] or NULL; receives dL/dx at x, including entries
 *               at a bound (clipping happens only in Adam)
 *   d_terms     device [QG_NTERMS] or NULL
 *   h           host; eps >= 0, beta >= 0, rho_scale >= 0
 *   d_workspace device, workspace_bytes long, caller-owned scratch
 * Enqueued on the stream; no host synchronisation unless
 * QG_FLAG_CHECK_FINITE was set at build.
 */
qg_status qg_eval_grad(qg_problem* prob, const double* d_x, double* d_grad,
                       double* d_terms, const qg_homotopy* h, void* d_workspace,
                       void* stream);

/*
 * qg_eval_grad without a workspace argument, for callers that cannot
 * allocate device memory (code under HIP graph capture, tight serving loops,
 * harnesses that forbid hipMalloc).  Same kernels, same results as
 * qg_eval_grad; its scratch is a static device array of QG_NOALLOC_SCRATCH
 * bytes inside the library, one per GPU, resolved at the first call on each
 * device and held until the process ends.  The caller still passes x and the
 * outputs (d_grad, d_terms: device, as for qg_eval_grad).
 *   Allocates nothing: no hipMalloc, hipFree or allocating library call.
 *   The current device must be the one the problem was built on (ARG
 *   otherwise).  A problem whose workspace_bytes exceeds QG_NOALLOC_SCRATCH
 *   is rejected with ARG.
 *   Every call on one GPU shares that GPU's array and leaves its contents
 *   behind (nothing in it needs to start at zero).  Calls that overlap on
 *   one GPU (two streams, two threads, a capture replayed beside another
 *   call) race on it: order them.
 * Errors: ARG, STATE, NONFINITE (QG_FLAG_CHECK_FINITE), DEVICE.
 */
#define QG_NOALLOC_SCRATCH ((size_t)32 << 20)
qg_status qg_eval_grad_noalloc(qg_problem* prob, const double* d_x, double* d_grad,
                               double* d_terms, const qg_homotopy* h, void* stream);

/*
 * One modified-Adam step with clip (Alg. 3) on device arrays of length n_x:
 * m <- b1 m + (1-b1) g; v <- b2 v + (1-b2) g^2;
 * x <- clip(x - lr_c (m/(1-b1^iter) [+eps]) / (sqrt(v/(1-b2^iter)) + eps)),
 * with lr_c the step size of the entry's class and the clip to the box
 * (v in [v_min, v_max], theta free, p in [0, pmax], q in [qmin, qmax],
 * r in [0, rmax], u in [0, 1]).  iter is 1-based.
 */
qg_status qg_adam_step(qg_problem* prob, double* d_x, double* d_m, double* d_v,
                       const double* d_grad, int64_t iter,
                       const double lr[QG_NCLASS], const qg_adam_cfg* cfg,
                       void* stream);

/*
 * Run n_steps of the Adam window of Alg. 4 (evaluate, backpropagate all
 * contingencies, or the screened set of qg_set_screening, Adam, clip) with
 * iteration-indexed schedules: step sizes
 * per class and eps from eqs. (norm_t)-(step_size), beta and rho_scale
 * linear.  x, m, v are updated in place (resume by passing iter0).  Every
 * check_every steps the score -L(eps=0, beta=1, rho_scale=rhof) is read back
 * for the gap stop against z_ed.  Synchronises the stream.
 */
qg_status qg_solve(qg_problem* prob, double* d_x, double* d_m, double* d_v,
                   const qg_solve_opts* opts, const qg_adam_cfg* cfg,
                   qg_solve_report* report, void* d_workspace, void* stream);

/*
 * Batched solve of independent scenarios (problems built separately, of any
 * sizes; the scenario batching of the many-problem workload): the same
 * schedule and Adam constants for all, n_steps steps each.  A step is six
 * launches for the whole batch, one per stage of the single-problem step
 * (Section II-C to II-G; Alg. 3), each covering every scenario's blocks;
 * the contingency map-reduce (eqs. (rank_correct), (sfr_pen)-(zctg)) is one
 * persistent launch whose blocks take (scenario, branch block, contingency
 * block, period chunk) work items from a counter until none is left.  Steps
 * are replayed from one HIP graph per 16 steps.  Every scenario gets the
 * points of its own qg_solve steps, bit for bit.
 *   Arrays of n entries (n <= QG_BATCH_MAX): problems, x, m, v, workspaces
 *   (caller-owned, as for qg_solve) and reports.
 *   d_batch: caller-owned device buffer of at least qg_batch_bytes bytes,
 *   256-byte aligned (every scenario's kernel arguments, the block tables of
 *   the six launches and the work counter); overwritten by the call.
 *   Every problem with contingencies needs a period-split tile of 4
 *   wavefronts of 4 periods (qg_set_ctg_tile_split(prob, 4, 4, lt); the
 *   branch tiles per block lt chosen per problem), screening off, and the
 *   same storage of the outage factors as the others.
 *   No gap checks or profiling (check_every and profile must be 0).
 *   reports[i].wall_s and steps_ms time the steps of the whole batch (upload
 *   of the tables and graph capture excluded).  Synchronises the stream.
 * Errors: ARG, DEVICE.
 */
#define QG_BATCH_MAX 256
qg_status qg_batch_bytes(qg_problem* const* probs, int32_t n, size_t* bytes);
qg_status qg_solve_batch(qg_problem* const* probs, int32_t n, double* const* d_x,
                         double* const* d_m, double* const* d_v, void* const* d_workspace,
                         void* d_batch, size_t batch_bytes, const qg_solve_opts* opts,
                         const qg_adam_cfg* cfg, qg_solve_report* reports, void* stream);

/*
 * Padded sizes and launch geometry, for tests and tools: dims[0..15] =
 * N, L, G, T, M, K, Lp, Kp, G16, G4, Tp, nLb, nKb, ctg_bl, ctg_wl, ctg_tc
 * (Lp = L rounded up to 64, Kp = K up to 64, G16 = G up to 16, G4 = G up to 4,
 * Tp = T up to 16; nLb, nKb = partial-sum counts of the contingency
 * map-reduce; ctg_bl, ctg_wl, ctg_tc = its tile).  With capacity >= 17,
 * dims[16] = storage of the outage factors (0 FP64, 1 FP32, 2 BF16); with
 * capacity >= 18, dims[17] = branch tiles per block (qg_set_ctg_ltiles);
 * capacity >= 19, dims[18] = 1 for a period-split tile (qg_set_ctg_tile_split).
 * capacity must be >= 16.
 */
qg_status qg_problem_dims(const qg_problem* prob, int32_t* dims, int32_t capacity);

/*
 * Branch-stacked tile of the contingency map-reduce: bl branches per
 * wavefront (8, 16 or 32), wl wavefronts per block (1, 2, 4 or 8) stacked
 * along the branches with bl*wl >= 16, and tc periods per block (0: a default
 * from the problem size; at most 8, and at most T).  A new problem starts
 * with the period-split tile of qg_set_ctg_tile_split (below 32 periods tcw
 * 2 and wl 4, 3 or 2, whichever pads the last period chunk least, ties to
 * the larger; from 32 periods wl 1 and tcw 4; default lt).  The results do not depend on the
 * tile except through the order of floating-point sums.  A step graph cached
 * by qg_solve is re-captured after a change.  Errors: ARG.
 */
qg_status qg_set_ctg_tile(qg_problem* prob, int32_t bl, int32_t wl, int32_t tc);

/*
 * Branch tiles (of wl * bl branches; of 8 branches for a period-split tile)
 * that one block of the contingency map-reduce covers, lt in [1, 64] (at
 * least 2 for a period-split tile), or 0 for the default (doubling from 1,
 * or 2, while at least 2048 blocks remain, at most 8).  More tiles per block
 * spread each block's fixed costs and shrink the per-(period, contingency)
 * partial sums; fewer leave more blocks.  qg_set_ctg_tile resets it to the
 * default; qg_set_ctg_tile_split sets it (0: the default).
 * Results depend on it only through the order of floating-point sums.  A
 * step graph cached by qg_solve is re-captured after a change.  Errors: ARG.
 */
qg_status qg_set_ctg_ltiles(qg_problem* prob, int32_t lt);

/*
 * Period-split tile of the contingency map-reduce (the default form): a
 * block of wl wavefronts (1..8) covers lt consecutive tiles of 8 branches (lt
 * in [2, 64], or 0 for the default of qg_set_ctg_ltiles) and 64
 * contingencies, and its wavefronts split the periods, tcw (1..8) each, so a
 * block spans wl * tcw periods.  A wavefront's per-(period, contingency) sums
 * stay with it over the block's whole branch range (no sum over wavefronts);
 * with wl * tcw >= T each outage factor is read once per evaluation.
 * Results depend on the tile only through the order of floating-point sums.
 * qg_set_ctg_tile returns to the branch-stacked form.  A step graph cached by
 * qg_solve is re-captured after a change.  Errors: ARG.
 */
qg_status qg_set_ctg_tile_split(qg_problem* prob, int32_t wl, int32_t tcw, int32_t lt);

/*
 * Test support: copy an intermediate array of the last evaluation from the
 * workspace into host memory (synchronises the stream).  Names and shapes
 * (row-major, padded sizes from qg_problem_dims):
 *   "F" [T][Lp] base-case DC flows      "Fk" [T][Kp] flows of outaged branches
 *   "q2" [T][Lp] max(q_fr^2, q_to^2)   "thr" [T][Lp] test radius of the outage flows
 *   "lamp", "lamq" [T][N] balance multipliers
 *   "zval" [T][Kp] contingency penalties z_tk
 *   "gfT" [Lp][Tp] dL/dF                "qtot" [T][Lp] dL/d max(q^2)
 *   "gpdc" [nsplit][T][G16] partial sums of the DC part of dL/dp (without
 *          the worst contingency's own outage term)
 *   "params" [16] step parameter block  "terms" [QG_NTERMS]
 * bytes must not exceed the array's size.  Errors: ARG, DEVICE.
 */
qg_status qg_debug_fetch(const qg_problem* prob, const void* d_workspace, const char* name,
                         void* host, size_t bytes, void* stream);

/*
 * Measurement support: mean duration (microseconds, written to *mean_us) of
 * one kernel of the step, stage 0..5 in stream order (k_forward, k_ctg_main,
 * k_ctg_zred, k_ctg_asm, k_adjoint, k_final), launched reps times back to back
 * on the stream after one full evaluation at x (homotopy h) has produced its
 * inputs; each of these launches recomputes the same outputs.  Synchronises
 * the stream.  Errors: ARG (stage, reps outside [1, 100000], pointers),
 * DEVICE.
 */
qg_status qg_time_stage(qg_problem* prob, const double* d_x, const qg_homotopy* h, int32_t stage,
                        int32_t reps, void* d_workspace, void* stream, double* mean_us);

/*
 * Contingency screening, the contingency solver of Alg. 2 (Section II-F,
 * contingency backpropagation summary): screened steps score and
 * backpropagate only a set of n_act contingencies, the worst set (the n_top
 * most severe of the last exact step with severity above zeta) plus a
 * uniform random draw from the rest.  The severity of contingency k is
 * max_t (z_tk - d_t c_s beta (L - 1) eps), its penalty above the value it has
 * with no overloaded branch (zero for an outage that overloads nothing).  In
 * a screened evaluation a contingency outside the set takes that
 * no-overload value in the per-period max and mean, and contributes no
 * gradient.  One set serves every period.  Keys of the draw: output
 * r 2^32 + k + 1 of SplitMix64 seeded with seed, r the refresh index.
 *
 * n_top = min(K, ceil(top_frac K)); n_act = min(K, n_top + ceil(rand_frac K)),
 * which must be >= 1.  When fewer than n_top contingencies exceed zeta, the
 * draw fills the remaining slots.  In qg_solve, step i (1-based iteration)
 * is an exact step followed by a new selection (refresh index
 * (i - 1) / refresh_every) when (i - 1) is a multiple of refresh_every or no
 * set of n_act contingencies has been chosen yet; the other steps are
 * screened.
 */
typedef struct qg_screen_opts {
  double top_frac;         /* in [0, 1] */
  double rand_frac;        /* in [0, 1] */
  double zeta;             /* finite */
  int32_t refresh_every;   /* >= 1 */
  int32_t reserved;        /* 0 */
  uint64_t seed;
} qg_screen_opts;

/* Bytes of the device screening buffer for these options.  Errors: ARG
 * (options out of range, problem without contingencies). */
qg_status qg_screen_bytes(const qg_problem* prob, const qg_screen_opts* opts, size_t* bytes);

/*
 * Turn screening on (opts non-NULL) or off (opts NULL; d_buf, bytes ignored).
 * d_buf: caller-owned device buffer of at least qg_screen_bytes bytes,
 * 256-byte aligned, used until screening is turned off or reconfigured (it
 * holds the set, the severities and the set's outage factors gathered into
 * contiguous columns).  No set is chosen yet: until one is, evaluations
 * score every contingency.  Does no device work (stream is unused).  A step graph cached by qg_solve is dropped.
 * With screening on and a set chosen, qg_eval_grad and qg_time_stage
 * evaluate the screened objective; qg_solve_batch and qg_solve with
 * profile = 1 refuse a problem with screening on.
 * Errors: ARG, STATE.
 */
qg_status qg_set_screening(qg_problem* prob, const qg_screen_opts* opts, void* d_buf,
                           size_t bytes, void* stream);

/*
 * Exact evaluation at x (homotopy h; gradient discarded) followed by the
 * selection with refresh index round >= 0 on the device: the severities,
 * the set and its gathered outage factors.  Enqueued on the stream.
 * Errors: ARG, STATE (screening off), DEVICE.
 */
qg_status qg_screen_refresh(qg_problem* prob, const double* d_x, const qg_homotopy* h,
                            int64_t round, void* d_workspace, void* stream);

/*
 * Use the given set (host array of n strictly increasing positions into
 * the contingency list, 1 <= n <= n_act of the options) for the screened
 * evaluations until the next refresh.  Uploads it and gathers its outage
 * factors; synchronises the stream.  Errors: ARG, STATE, DEVICE.
 */
qg_status qg_set_active_contingencies(qg_problem* prob, const int32_t* ks, int32_t n,
                                      void* stream);

/*
 * Copy the current set (increasing positions into the contingency list) to
 * host memory: *n receives its size, out needs capacity >= *n entries; and,
 * if sev is non-NULL, the K severities of the last refresh (capacity >= K).
 * Synchronises the stream.  Errors: ARG, STATE (screening off or no set),
 * DEVICE.
 */
qg_status qg_get_active_contingencies(const qg_problem* prob, int32_t* out, int32_t capacity,
                                      int32_t* n, double* sev, void* stream);

void qg_destroy_problem(qg_problem* prob);
const char* qg_status_string(qg_status s);
const char* qg_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* QG_H */
