/*
 * ebe.h -- C ABI of the MI355X (gfx950) library for repeated implicit time
 * stepping with a data-driven initial guess refined by block-Jacobi PCG.
 *
 * Method: Ichimura et al., "Heterogeneous computing in a strongly-connected
 * CPU-GPU environment: fast multiple time-evolution equation-based modeling
 * accelerated using data-driven approach", arXiv:2409.20380.
 *   - problem statement: solve A x^it = f^it for it = 1..nt in sequence
 *     (Sec. 2.1, Eq. general);
 *   - application: linear elastodynamics discretised with straight 10-node
 *     tetrahedra and Newmark-beta with damping (Sec. 3.1, Eq. GE:DIS and
 *     Eq. timestep);
 *   - matvec: matrix-free element-by-element product (Sec. 2.2 Eq. EBE,
 *     Sec. 3.2 Eq. eqebefem);
 *   - solver: conjugate gradient with a 3x3 block-Jacobi preconditioner
 *     (Sec. 3.2, Algorithm 1), stopped when ||r||/||f|| < tol;
 *   - predictor: x-bar = predictor(X, F, f) (Sec. 2.2, Eq. predictor), made
 *     concrete as an Adams-Bashforth 4-step estimate plus a regional
 *     least-squares map over the Adams-Bashforth errors of the past s steps
 *     (Sec. 3.2).
 *
 * Conventions
 *   - Every call returns an int status: EBE_OK (0), EBE_NOT_CONVERGED (1,
 *     results and statistics are still written) or a negative error code.
 *     The message of the last error is returned by ebe_last_error().
 *     No C++ exception crosses this boundary.
 *   - Host pointers appear only in ebe_assemble, ebe_get_regions and the
 *     3-value base acceleration; they are read during the call and may be
 *     freed afterwards.
 *   - All other vectors are caller-owned DEVICE pointers on the handle's
 *     device: contiguous float64 arrays of length 3*n_nodes, node-major with
 *     the x, y, z components interleaved (dof = 3*node + component), in the
 *     caller's node numbering.  They are borrowed for the duration of the
 *     call only.  The library permutes them into its own internal order.
 *   - The library owns all of its internal buffers and frees them in
 *     ebe_destroy.  All work is ordered on the stream given to ebe_create.
 *     Calls that fill a statistics struct synchronise that stream before
 *     returning.  A handle is not thread-safe.
 *   - Degrees of freedom flagged as fixed carry zero displacement; the
 *     operator A has identity rows and columns there (A_bc = Z A Z + I - Z,
 *     Z the free-dof mask), and every right-hand side is zeroed there.
 */
#ifndef EBE_H
#define EBE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define EBE_OK 0
#define EBE_NOT_CONVERGED 1
#define EBE_E_INVALID_ARG (-1)
#define EBE_E_HIP (-2)
#define EBE_E_NO_MEMORY (-3)
#define EBE_E_BAD_STATE (-4)
#define EBE_E_NONFINITE (-5)

/* Kinds of initial guess for the next step's increment. */
#define EBE_PRED_ZERO 0      /* x-bar = 0 */
#define EBE_PRED_AB4 1       /* Adams-Bashforth 4-step estimate (Sec. 3.2) */
#define EBE_PRED_SNAPSHOT 2  /* AB4 + regional snapshot map (Sec. 3.2) over
                                a guarded window (see ebe_predict) */
#define EBE_PRED_LEARNED 3   /* the kind-2 guess judged against the AB4
                                increment plus a node-wise network estimate of
                                its error (see "Learned predictor" below); the
                                one with the smaller initial residual is kept
                                (ties keep the kind-2 guess).  The network is
                                used from step 5 on once weights are set;
                                after 8 consecutive steps that kept the kind-2
                                guess it is evaluated only on steps divisible
                                by 16 until it wins again. */

/* Precision of the refinement.  FP64: Algorithm 1 in FP64.  FP32 / BF16: a
 * flexible outer PCG in FP64 (residual, dot products, update; Polak-Ribiere
 * beta because the preconditioner varies) whose preconditioner is an inner
 * 3x3 block-Jacobi PCG with an FP32 element-by-element matvec and FP32
 * arithmetic, its direction and preconditioned-residual vectors stored in
 * FP32 or BF16; the outer stop test is the same relative FP64 residual.  The
 * predictor's least squares stays FP64 in every mode. */
#define EBE_PREC_FP64 0
#define EBE_PREC_FP32 1
#define EBE_PREC_BF16 2

typedef struct ebe_handle ebe_handle;

typedef struct {
    double dt;              /* time increment (s) */
    double rayleigh_alpha;  /* damping C = alpha M + beta K (1/s) */
    double rayleigh_beta;   /* (s) */
    double tol;             /* relative residual tolerance of Algorithm 1 (e.g. 1e-8) */
    double drop_tol;        /* snapshot column kept only if its part orthogonal to the
                               earlier kept columns has norm >= drop_tol * its norm
                               (<= 0: 1e-6, or 1e-5 with an FP32 / BF16 inner solve) */
    double inner_tol;       /* mixed precision: relative residual target of each inner
                               solve (<= 0: 1e-2) */
    int32_t max_iter;       /* PCG iteration cap per solve (<= 0: 10000) */
    int32_t s;              /* snapshot window: number of input columns, 0..32 */
    int32_t predictor;      /* EBE_PRED_* */
    int32_t region_nodes;   /* nodes per predictor region when ebe_assemble receives no
                               region map (<= 0: 512) */
    int32_t patch_elems;    /* at most this many elements per EBE patch, 1..256 (<= 0: 256);
                               a patch closes earlier when its nodes would need more
                               LDS than two resident element workgroups per CU allow */
    int32_t chunk_iters;    /* PCG iterations enqueued between convergence checks
                               (<= 0: adaptive) */
    int32_t precision;      /* EBE_PREC_*: how Algorithm 1 is run (see below) */
    int32_t inner_iters;    /* mixed precision: inner PCG trips per outer trip at most
                               (<= 0: 12) */
    int32_t s_min;          /* snapshot map used once its window holds at least
                               min(s_min, s) column pairs (<= 0: 3; the guard below keeps
                               AB4 where the short map is worse); AB4 alone before.  The
                               window length itself stays at least max(s_min, min(8, s)),
                               the lower end of the paper's range 8 <= s <= 32 (Sec. 4,
                               Fig. 3) */
    int32_t fixed_window;   /* 0 (default): guarded window -- whenever the map is used, the
                               AB4 guess is evaluated too and kept when its initial residual
                               is strictly smaller, and the window then restarts at that step;
                               the window length adapts by probes (see "Snapshot window"
                               below); 1: the map's guess is always used, over s column
                               pairs, and the window never restarts */
    int32_t probe_every;    /* guarded window: steps with a full window between two length
                               probes (<= 0: 16) */
    int32_t probe_step;     /* guarded window: column pairs a probe adds or removes (<= 0: 8) */
    double skip_ratio;      /* guarded window: the AB4 guess is not evaluated while the map's
                               initial residual is below skip_ratio x the last evaluated AB4
                               one (0: 0.01; < 0: always evaluated) */
    double col_cost;        /* guarded window: predictor cost of one window column, in PCG
                               trips, against which the probes weigh the trips a longer window
                               saves (0: 0.08, measured on the 64x64x32-cell mesh; < 0: no
                               probes, the length stays s) */
    int32_t region_merge;   /* <= 1: the predictor's regions are the regions ebe_assemble
                               receives (or builds).  m > 1: those regions, ordered by the
                               Morton code of their centroids, are merged m at a time into
                               the regions of the snapshot map's least squares (Sec. 3.2:
                               each region has its own fit), while the given regions keep
                               ordering the nodes and so shaping the element patches: small
                               compact regions give compact patches, merged ones give each
                               fit more rows per column.  ebe_get_regions reports the
                               merged regions.  The batch (ebe_batch_*) merges each mesh's
                               regions the same way. */
    int32_t reserved[3];
} ebe_config;

typedef struct {
    int32_t iters;      /* PCG loop trips (q = A p products), the r0 product excluded */
    int32_t restarts;   /* restarts after a true-residual check failed */
    int32_t status;     /* EBE_OK or EBE_NOT_CONVERGED */
    int32_t inner_iters;  /* mixed precision: inner PCG trips summed over the solve */
    double res0;        /* ||b - A x-bar|| / ||b|| */
    double res_rec;     /* recursive residual at exit, relative */
    double res_true;    /* ||b - A x|| / ||b|| recomputed at exit */
    double bnorm;       /* ||b|| */
} ebe_solve_stats;

typedef struct {
    int32_t it;         /* index of the step just completed (1-based) */
    int32_t s_eff;      /* snapshot column pairs used by the map (0: map not used) */
    int32_t iters;
    int32_t restarts;
    int32_t status;
    int32_t inner_iters;
    double res0, res_rec, res_true, bnorm;
    int32_t learned;        /* kind 3: 1 the learned candidate was kept, 0 the snapshot
                               prediction; -1 if no candidate was evaluated this step */
    int32_t first;          /* the window held the AB errors e^first .. e^{it-1} (0: no map) */
    double res0_snapshot;   /* kind 3: ||b - A x||/||b|| of both candidates (free rows) */
    double res0_learned;
    int32_t map_kept;       /* guarded window: 1 the map's guess was kept, 0 the AB4 guess
                               (the window restarted at this step); -1 no comparison */
    int32_t skipped;        /* guarded window: 1 if the AB4 guess was not evaluated (map far ahead) */
    double res0_map;        /* guarded window: ||b - A x||/||b|| of the map's and of the */
    double res0_ab;         /* AB4 guess (free rows; 0 without a comparison or when skipped) */
    int32_t probe;          /* window length probed this step (0: none) */
    int32_t s_cap;          /* window length cap after this step */
    double res0_probe;      /* ||b - A x||/||b|| of the guess over the probed length */
} ebe_step_stats;

/* Snapshot-window state carried from step to step (checkpoint / resume). */
typedef struct {
    int32_t start;          /* first step whose AB error may enter the window (>= 1) */
    int32_t s_cap;          /* window length cap in column pairs (1..s; 0 on input: s) */
    int32_t since;          /* steps with a full window since the last length probe */
    int32_t grow_next;      /* direction of the next probe: 1 longer, 0 shorter */
    double rho_ab;          /* last evaluated initial relative residual of the AB4 guess (0: none) */
    double rate;            /* ln(res0 / res_end) / trips of the last solve, inner trips
                               of the mixed forms at 0.62 each (0: none) */
} ebe_window;

typedef struct {
    int32_t s_eff;          /* as in ebe_step_stats, for the step ebe_predict looks at */
    int32_t first;
    int32_t map_kept;       /* 1 map's guess returned, 0 AB4's, -1 no comparison */
    int32_t learned;        /* kind 3: 1 learned candidate returned, 0 not, -1 not evaluated */
    double res0;            /* ||b - A x-bar|| / ||b|| of the returned guess (free rows) */
    double res0_map, res0_ab, res0_learned;   /* candidates compared (else 0) */
    double bnorm;           /* ||b|| of the step's right-hand side */
} ebe_pred_stats;

/* Version string of the library. */
const char* ebe_version(void);

/* Create a handle on the current HIP device.  stream: a hipStream_t (may be
 * NULL for the default stream), e.g. torch.cuda.current_stream().cuda_stream.
 * Errors: INVALID_ARG (bad config), HIP. */
int ebe_create(const ebe_config* cfg, void* stream, ebe_handle** out);

/* Free every device and host resource of the handle.  NULL is accepted. */
int ebe_destroy(ebe_handle* h);

/* Message of the last error on this handle (or of the last failed create when
 * h is NULL).  Owned by the library, valid until the next call. */
const char* ebe_last_error(const ebe_handle* h);

/* Mesh and material data (Sec. 3.1): straight 10-node tetrahedra.
 *   coords  host [n_nodes][3]  node coordinates (m)
 *   conn    host [n_elems][10] node ids: 4 vertices, then the midpoints of
 *           edges (0,1),(1,2),(0,2),(0,3),(1,3),(2,3); positive orientation
 *           det[x1-x0, x2-x0, x3-x0] > 0; edge nodes must sit at the edge
 *           midpoints (geometry is taken from the vertices)
 *   elem_mat host [n_elems] material id in [0, n_mat)
 *   mat     host [n_mat][3] density rho, P velocity vp, S velocity vs;
 *           mu = rho vs^2, lambda = rho (vp^2 - 2 vs^2)
 *   fixed   host [n_nodes][3] 1 = component fixed (zero displacement)
 *   region_of_node host [n_nodes] predictor region id in [0, R), every id
 *           used, any region size (one region over the whole mesh is valid),
 *           or NULL to let the library group nodes into spatially compact
 *           regions of cfg.region_nodes nodes (query them with ebe_get_regions)
 * Builds the element patches, the internal node order, the element
 * geometry checks and the block-Jacobi inverse, and resets the state to rest
 * (u = v = a = 0, empty history, step 0).
 * Errors: INVALID_ARG (ids out of range, inverted or degenerate element,
 * misplaced edge node, node used both as vertex and edge node), NO_MEMORY, HIP. */
int ebe_assemble(ebe_handle* h, int64_t n_nodes, const double* coords, int64_t n_elems,
                 const int32_t* conn, const int32_t* elem_mat, int32_t n_mat, const double* mat,
                 const uint8_t* fixed, const int32_t* region_of_node);

/* Region id of every node (host [n_nodes]); returns the region count in *n_regions. */
int ebe_get_regions(ebe_handle* h, int32_t* region_of_node, int32_t* n_regions);

/* q = A_bc p with A = (4/dt^2 + 2 alpha/dt) M + (1 + 2 beta/dt) K (the Newmark
 * system matrix of Eq. GE:DIS with Rayleigh damping), evaluated element by
 * element (Eq. EBE) without storing any matrix. */
int ebe_apply(ebe_handle* h, const double* p, double* q);

/* q = cm * M p + ck * K p, unconstrained (no fixed-dof handling). */
int ebe_apply_mk(ebe_handle* h, double cm, double ck, const double* p, double* q);

/* z = B^{-1} r, B the 3x3 diagonal blocks of A_bc (Algorithm 1 preconditioner). */
int ebe_precond(ebe_handle* h, const double* r, double* z);

/* Right-hand side of the next step for the increment du = u^it - u^(it-1):
 *   b = f + C v + M (a + (4/dt) v) - K u,  zero on fixed dofs,
 * from the current state (u, v, a), where f = f_ext (device, may be NULL)
 * minus sum_k base_acc[k] M r_k (host [3], may be NULL; r_k the rigid unit
 * translation along axis k: the inertial load of a uniform base acceleration). */
int ebe_rhs(ebe_handle* h, const double* f_ext, const double* base_acc, double* b);

/* Initial guess of the next step's increment from the stored history
 * (Eq. predictor with the concrete predictor of Sec. 3.2 chosen by
 * cfg.predictor): exactly the guess ebe_step would start from with the same
 * f_ext (f_next, device, may be NULL) and base_acc (host [3], may be NULL),
 * whose right-hand side the guarded window and kind 3 need to compare
 * candidates.  dxbar: device [3N] out.  stats (may be NULL): window, picks and
 * initial residuals (filling it synchronises the stream).  The state is not
 * modified: a window restart implied by the comparison happens only in
 * ebe_step.
 *
 * Snapshot window (kinds 2 and 3).  Step n fits the regional map on the AB
 * errors e^first .. e^{n-1}, first = max(w, n - 1 - s_cap): inputs e^first ..
 * e^{n-2}, outputs e^{first+1} .. e^{n-1}, query e^{n-1}, s_eff = n - 1 - first
 * column pairs; w = 1 and s_cap = s at rest.  The map is used once s_eff >=
 * min(s_min, s).  Unless cfg.fixed_window:
 *   - guard: the AB4 guess is evaluated too (one more matvec) and kept when
 *     ||b - A x|| is strictly smaller; ebe_step then sets w = n, discarding the
 *     columns that span the change of regime (the start from rest, a kink of
 *     the input) that made the map lose.  The evaluation is skipped (the map
 *     kept) while the map's relative residual is below skip_ratio times the
 *     last evaluated AB4 one.
 *   - length (the paper varies s during the run to balance predictor and
 *     solver time, Sec. 3.2 and Fig. 4; on one device they add up): on the
 *     probe_every-th step with a full window (s_eff = s_cap) ebe_step also
 *     evaluates the map over s_cap - probe_step or s_cap + probe_step pairs
 *     (alternating; at least max(s_min, min(8, s)), at most s, columns after
 *     w), estimates the
 *     trips the longer of the two saves as 2 ln(rho_short / rho_long) / rate
 *     (rate = ln(res0 / res_end) / trips of the previous solve, an inner trip of
 *     the mixed-precision forms counted as 0.62 of a trip; the factor 2
 *     because a guess removes mostly slowly converging components) and moves
 *     s_cap to the probed length when that beats (or, for a shorter probe,
 *     falls below) col_cost x probe_step.  The step uses the s_cap window. */
int ebe_predict(ebe_handle* h, const double* f_next, const double* base_acc, double* dxbar,
                ebe_pred_stats* stats);

/* Algorithm 1 (or its mixed-precision form, cfg.precision): solve A_bc x = b to
 * ||b - A x|| / ||b|| < tol starting from the guess in x (overwritten with the
 * solution).  If ||b|| = 0, x = 0 with zero
 * iterations.  Returns NOT_CONVERGED when max_iter is reached, NONFINITE if a
 * scalar of the iteration is not finite. */
int ebe_refine(ebe_handle* h, const double* b, double* x, ebe_solve_stats* stats);

/* One time step: right-hand side, predictor, Algorithm 1, Newmark-beta
 * (beta = 1/4, gamma = 1/2) update of u, v, a, velocity history and snapshot
 * ring.  f_ext (device) and base_acc (host [3]) as in ebe_rhs, at the new time.
 * The call waits for the solve's stop test (the scalars are read back once
 * per chunk of trips); the final update may still be running on the handle's
 * stream when it returns, ordered before any later call.  stats may be NULL. */
int ebe_step(ebe_handle* h, const double* f_ext, const double* base_acc, ebe_step_stats* stats);

/* Checkpoint / resume.  u, v, a: device [3N] each, caller order.
 * History: vhist device [4][3N] = v^it, v^(it-1), v^(it-2), v^(it-3);
 * ring device [s+1][3N] with e^j = du^j - du_AB^j in slot (j-1) mod (s+1);
 * it = completed steps; win: host, the snapshot-window state (NULL in
 * ebe_set_history: window from step 1 at length s, no probe or AB4
 * residual history). */
int ebe_get_state(ebe_handle* h, double* u, double* v, double* a);
int ebe_set_state(ebe_handle* h, const double* u, const double* v, const double* a);
int ebe_get_history(ebe_handle* h, double* vhist, double* ring, int32_t* it, ebe_window* win);
int ebe_set_history(ebe_handle* h, const double* vhist, const double* ring, int32_t it, const ebe_window* win);

/* Block until all work enqueued on the handle's stream is done. */
int ebe_sync(ebe_handle* h);

/* Kernel timing: when enabled, every n-th launch of the element-by-element
 * PCG matvec kernel is bracketed by HIP events on the handle's stream (only
 * trips that certainly run: index + 3 below the previous solve's count).
 * ebe_kernel_time returns the number of timed launches and their mean
 * duration in milliseconds since the last reset. */
int ebe_set_kernel_timing(ebe_handle* h, int32_t every_n);
int ebe_kernel_time(ebe_handle* h, int64_t* launches, double* mean_ms);

/* Sizes used for roofline accounting of one PCG iteration: n_nodes, n_elems,
 * n_patch_nodes (sum over patches of the nodes each patch touches), patches. */
int ebe_sizes(ebe_handle* h, int64_t* n_nodes, int64_t* n_elems, int64_t* n_patch_nodes, int64_t* n_patches);

/* Changes the predictor kind (EBE_PRED_*) of later steps. */
int ebe_set_predictor(ebe_handle* h, int32_t kind);

/* Back to rest: u = v = a = 0, empty velocity history and snapshot ring,
 * it = 0.  The mesh, the network weights and the collected samples stay. */
int ebe_reset(ebe_handle* h);

/* ---- Learned predictor ---------------------------------------------------
 * Not in the paper (which mentions learned surrogates only as related work,
 * Sec. 1): an extension of the predictor of Sec. 3.2 (Eq. predictor, whose
 * guess may use the force f of the new step).  A network applied node by
 * node, 15 -> 64 -> 64 -> 3 with GELU (tanh form) after each hidden layer,
 * estimates the error of the Adams-Bashforth increment, du - du_AB (the
 * quantity the snapshot map predicts from past errors).  Inputs of node n for
 * step it: its last four displacements, encoded as u^{it-1} (divided by
 * scales[0]) and the increments u^{it-1} - u^{it-2}, u^{it-2} - u^{it-3},
 * u^{it-3} - u^{it-4} (divided by scales[1]; the same information without the
 * cancellation BF16 inputs would cause), then its external force f^{it}
 * (divided by scales[2]); the estimate is scales[3] times the output (zero on
 * fixed dofs).
 * Inference uses BF16 weights and activations with FP32 accumulation (MFMA).
 * Training (FP32 with BF16-rounded weights and inputs in the forward, Adam
 * with beta1 = 0.9, beta2 = 0.999, eps = 1e-8) minimises the mean squared
 * error between the output and (du^{it} - du_AB^{it}) / scales[3] over samples
 * collected during ebe_step (steps 5 and later).
 * Parameter vector (FP32, 5379 values): W1[64][15], b1[64], W2[64][64],
 * b2[64], W3[3][64], b3[3], row-major; layer k computes W_k h + b_k.
 * ebe_assemble drops weights and samples. */
#define EBE_MLP_IN 15
#define EBE_MLP_HIDDEN 64
#define EBE_MLP_OUT 3
#define EBE_MLP_PARAMS 5379
#define EBE_MLP_SAMPLE 18     /* floats per collected sample: 15 raw inputs, 3 raw targets */
#define EBE_MLP_SCALES 4
#define EBE_MLP_MAX_BATCH 8192

/* Sets the FP32 master weights (host [5379]) and scales (host [4], > 0);
 * resets the Adam moments and step count. */
int ebe_mlp_set(ebe_handle* h, const float* params, const float* scales);
/* Reads the FP32 master weights (host [5379] or NULL) and scales (host [4] or NULL). */
int ebe_mlp_get(ebe_handle* h, float* params, float* scales);
/* Inference kernel on given inputs: x device [n][15] (already scaled), y
 * device [n][3] (network outputs, unscaled).  With predictor kind 3,
 * ebe_predict returns the guess ebe_step would keep (the learned candidate
 * when its initial residual is the smaller). */
int ebe_mlp_forward(ebe_handle* h, int64_t n, const float* x, float* y);
/* Loss and gradient over n (1..8192) samples: x device [n][15], t device
 * [n][3] (scaled targets); grad device [5379] out; loss host out or NULL. */
int ebe_mlp_grad(ebe_handle* h, int64_t n, const float* x, const float* t, float* grad, double* loss);
/* For callers that cannot allocate device memory during a call (code under
 * HIP graph capture, tight training or serving loops, harnesses that forbid
 * allocation): the result of ebe_mlp_grad (same kernels, same gradient and
 * loss) with the training activations and partial sums in a fixed device
 * array of the library (about 13 MB per GPU, held until the process ends)
 * instead of buffers the handle allocates when n first exceeds its capacity.
 * n must be in 1..8192, the array's capacity (EBE_E_INVALID_ARG otherwise);
 * the weights must be set (EBE_E_BAD_STATE otherwise).  grad device [5379]
 * out.  loss: host out, or NULL -- then the call only enqueues kernels on the
 * handle's stream (no copy, no synchronisation).  All calls on one GPU share
 * the one array: calls that overlap in time on that GPU (other streams,
 * threads or handles) race and give wrong results. */
int ebe_mlp_grad_noalloc(ebe_handle* h, int64_t n, const float* x, const float* t, float* grad, double* loss);
/* One Adam step of the master weights with the given gradient (device [5379]). */
int ebe_mlp_adam(ebe_handle* h, const float* grad, float lr);
/* Sample collection: every later ebe_step from step 5 on appends one sample
 * per listed node (device int32 [k], caller's node ids) while `capacity`
 * samples fit.  A capacity different from the current one
 * drops the samples collected so far.  nodes NULL or k = 0 stops collecting. */
int ebe_collect(ebe_handle* h, int64_t capacity, const int32_t* nodes, int32_t k);
/* Number of collected samples; copies them to dst (device [count][18]) if not NULL. */
int ebe_samples(ebe_handle* h, int64_t* count, float* dst);
/* Sets the scales to the root mean squares of the collected inputs of each
 * group (newest displacement, increments, force) and of the targets (a zero
 * RMS gives 1); returns them in scales (host [4]) if not NULL.  A later ebe_mlp_set replaces them with the
 * scales it is given. */
int ebe_mlp_fit_scales(ebe_handle* h, float* scales);
/* `steps` Adam steps on minibatches of the collected samples: idx device
 * int64 [steps][batch], every entry in 0..count-1 (checked); loss host
 * [steps] receives each minibatch's loss, or NULL. */
int ebe_mlp_train(ebe_handle* h, int32_t steps, int32_t batch, const int64_t* idx, float lr, double* loss);

/* ---- Batched ensembles ------------------------------------------------------
 * Many cases (each its own base acceleration) on one or more meshes,
 * advanced one time step together: the paper's r-case element pass (Sec.
 * 2.2, Eq. eqmebefem; Table 2) with independent CGs per case (Algorithm 1 per
 * case: own alpha, beta, stop test and iteration count, stopped cases masked
 * out of the shared element passes).  Every case follows the single-case
 * step of ebe_step (right-hand side, AB4 + regional snapshot map, refine to
 * tol, Newmark; every case has its own guarded snapshot window, see
 * ebe_predict, at length s and with the AB4 guess evaluated on every step
 * where the map is used).  Each mesh added forms a group of n_cases cases; the group's
 * element pass works on tiles of case_tile cases (1, 2, 4 or 8) with element
 * patches of 256 / case_tile elements and `chunks` persistent workgroups per
 * tile, chosen by timing every candidate when ebe_batch_assemble is asked to
 * tune.  The PCG trips of all groups are enqueued in chunks that are captured
 * once in a hipGraph and replayed (ebe_batch_use_graph).  Only FP64 and
 * predictor kinds 0..2 are supported.  Host arrays are copied; per-case
 * vectors are device float64 [3 N] of that case's mesh in the caller's node
 * order. */
typedef struct ebe_batch ebe_batch;

typedef struct {
    int32_t iters;      /* PCG trips of this case in the last step */
    int32_t restarts;
    int32_t status;     /* EBE_OK or EBE_NOT_CONVERGED */
    int32_t s_eff;      /* snapshot column pairs of this case's map (0: not used) */
    double res0;        /* relative residual of the initial guess */
    double res_true;    /* relative true residual at exit */
    double bnorm;
    int32_t first;      /* this case's window held e^first .. e^{it-1} (0: no map) */
    int32_t map_kept;   /* guarded window: 1 map's guess kept, 0 AB4's (window restarted), -1 none */
} ebe_batch_stats;

int ebe_batch_create(const ebe_config* cfg, void* hip_stream, ebe_batch** out);
int ebe_batch_destroy(ebe_batch* b);
const char* ebe_batch_last_error(const ebe_batch* b);
/* Adds a mesh (same arrays and validation as ebe_assemble) with n_cases
 * cases; group receives its index.  Cases are numbered group by group. */
int ebe_batch_add_mesh(ebe_batch* b, int64_t n_nodes, const double* coords, int64_t n_elems, const int32_t* conn,
                       const int32_t* elem_mat, int32_t n_mat, const double* mat, const uint8_t* fixed,
                       const int32_t* region_of_node, int32_t n_cases, int32_t* group);
/* Fixes a group's case tile and workgroups per tile (used by the next
 * ebe_batch_assemble instead of tuning). */
int ebe_batch_set_group_config(ebe_batch* b, int32_t group, int32_t case_tile, int32_t chunks);
/* Builds every group (tuning the groups without a fixed configuration when
 * tune != 0), allocates the stacked state and puts every case at rest. */
int ebe_batch_assemble(ebe_batch* b, int32_t tune);
int ebe_batch_group_info(ebe_batch* b, int32_t group, int32_t* first_case, int32_t* n_cases, int64_t* n_nodes,
                         int32_t* case_tile, int32_t* chunks);
/* on = 0 enqueues the PCG trips directly; trips (even, 2..64) per chunk. */
int ebe_batch_use_graph(ebe_batch* b, int32_t on, int32_t trips);
int ebe_batch_reset(ebe_batch* b);
/* q = A_bc p for every case of a group: p, q device [n_cases][3 N]. */
int ebe_batch_apply(ebe_batch* b, int32_t group, const double* p, double* q);
/* One time step of every case: base_acc host [n_cases][3]; stats host
 * [n_cases] or NULL.  EBE_NOT_CONVERGED if any case hit max_iter. */
int ebe_batch_step(ebe_batch* b, const double* base_acc, ebe_batch_stats* stats);
int ebe_batch_get_state(ebe_batch* b, int32_t case_index, double* u, double* v, double* a);
int ebe_batch_sizes(ebe_batch* b, int32_t* n_groups, int32_t* n_cases, int64_t* total_dof);

/* The configuration in effect (defaults filled in for fields given as <= 0).
 * out: host struct written by the call.  EBE_E_INVALID_ARG if out is NULL. */
int ebe_get_config(ebe_handle* h, ebe_config* out);

#ifdef __cplusplus
}
#endif
#endif /* EBE_H */
