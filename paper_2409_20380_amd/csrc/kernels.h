// kernels.h -- launch wrappers of the gfx950 kernels (internal to the library).
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>

#include "topology.h"

namespace ebe {

// Device-side scalars of one PCG solve (Algorithm 1).  Written by workgroup 0
// of the kernel that decides them; read by later kernels and the host.
struct DevScalars {
    double rho[2];    // (z, r) of trip j, stored in slot j & 1
    double bnorm;     // ||b||
    double rr;        // ||r||^2 of the last residual tested
    double res0;      // relative residual of the initial guess
    double res_true;  // relative true residual at the last check
    int32_t done;     // 0 running, 1 converged, 2 non-finite, 3 iteration cap, 4 zero rhs
    int32_t iters;    // PCG trips taken
    int32_t restarts;
    int32_t checked;  // true residual evaluated since the loop stopped
    int32_t cycle_start;  // trip index at which the current CG cycle began (beta = 0 there)
    int32_t inner_iters;  // mixed precision: inner trips summed over the solve
    // learned predictor: squared free-row residuals of the snapshot (0) and
    // learned (1) candidates and which one was kept; not reset by a solve
    double cand_rr[2];
    int32_t cand_pick;
    int32_t pad_;
    // snapshot-map guard: squared free-row residuals of the map's guess (0)
    // and of the Adams-Bashforth guess (1); guard_pick = 1 when the latter was
    // kept (strictly smaller); not reset by a solve
    double guard_rr[2];
    int32_t guard_pick;
    int32_t guard_skip;  // 1: the AB4 guess was not evaluated (the map's residual far below the last AB4 one)
    double probe_rr;     // ||b - A x||^2 of the guess over the probed window length (free rows)
    // FP64 solve: x += alpha p is applied for two trips at once; trip j with (j - x_base) even
    // leaves its alpha in x_alpha for trip j + 1 (or the flush at the stop)
    double x_alpha;
    int32_t x_base;
    int32_t pad3_;
    double guess_rr;   // ||b - A x||^2 of the last guess evaluated by ebe_predict (free rows)
    double guess_bb;   // ||b||^2 of the same right-hand side (free rows)
};

enum { DONE_RUNNING = 0, DONE_CONVERGED = 1, DONE_NONFINITE = 2, DONE_MAXITER = 3, DONE_ZERO_RHS = 4 };

// Precision of a PCG solve: FP64 throughout, or FP32 arithmetic with the
// direction and preconditioned-residual vectors stored in FP32 or BF16.
enum { PREC_FP64 = 0, PREC_FP32 = 1, PREC_BF16 = 2 };

// 16-bit brain float storage (upper half of an IEEE binary32).
struct bf16_t {
    uint16_t bits;
};

// Device copies of the topology arrays used by the element kernels.
struct DevPatches {
    const int32_t* el_ptr;      // [Ppad+1]
    const int32_t* pn_ptr;      // [Ppad+1]
    const int32_t* nv;          // [Ppad]
    const uint32_t* nodes;      // [PN] internal node id | owner bit
    const int32_t* slot;        // [PN] output slot of each patch node
    const ElemRec* elems;       // [E]
    const double* coords;       // [N][3]
    const double* mat;          // [n_mat][3] lambda, mu, rho
    const uint8_t* fixmask;     // [N]
    int32_t n_patches_pad;
    int32_t max_pn, max_nv;
    int32_t n_mat;              // materials in `mat` (the element kernels stage them in LDS)
};

struct DevNodes {
    const int32_t* slot_ptr;    // [N+1] node n sums slots [slot_ptr[n], slot_ptr[n+1])
    const uint8_t* fixmask;     // [N]
    int64_t n;
};

constexpr int kMaxCols = 33;    // s <= 32 input columns plus the query
constexpr int kEbeWaves = 4;        // wavefronts per EBE workgroup (one patch per workgroup)
constexpr int kMaxPcgGrid = 512;    // persistent workgroups of the PCG matvec (multiple of 8)
constexpr int kMaxResGrid = 1024;   // workgroups of the node-wise reduction kernels
constexpr int kResArrays = 4;       // partial arrays per slot: (z,r), (r,r), (b,b), (z,r_prev)
struct ColPtrs {
    const double* c[kMaxCols];
};

// ---- element-by-element operator
// qbuf[pn] = sum over the patch's elements of (cm M_e + ck K_e) p_e for the
// patch's nodes; p gathered with fixed components zeroed when mask_in.
// guard: if non-NULL, the kernel runs only when a true-residual check is due.
// skip: if non-NULL, the kernel returns at once when sc->guard_skip is set.
void launch_ebe_apply(hipStream_t s, const DevPatches& P, const double* p, bool mask_in, double cm, double ck,
                      double* qbuf, const DevScalars* guard = nullptr, const DevScalars* skip = nullptr);
// PCG trip j, matvec part: stop test on the incoming residual partials, beta,
// p_cur = z + beta p_prev, qbuf = A_e p_cur and (p, A p) partials.
int pcg_ebe_grid(const DevPatches& P);
struct PcgLaunch {
    const DevPatches* P;
    int prec;            // PREC_*: compute / storage types of z, p_prev, p_cur, qbuf
    bool flexible;       // FP64 only: Polak-Ribiere beta (needs the (z, r_prev) partials)
    const void* z;
    const void* p_prev;
    void* p_cur;
    void* qbuf;
    double cm, ck;
    DevScalars* sc;
    const DevScalars* outer;   // inner solves: stop when the outer solve stopped
    const double* res_part;
    int g_res;
    double* pap_part;
    int j, max_iter;
    double tol;
};
void launch_ebe_pcg(hipStream_t s, const PcgLaunch& L);
// Right-hand side operands: M part w1 = a + c1 v - g, K part w2 = c2 v - u.
void launch_ebe_rhs(hipStream_t s, const DevPatches& P, const double* u, const double* v, const double* a,
                    double c1, double c2, double g0, double g1, double g2, double* qbuf);
// Block diagonal of cm M + ck K per patch node (6 symmetric entries).
void launch_ebe_diag(hipStream_t s, const DevPatches& P, double cm, double ck, double* qbuf6);
// Dynamic LDS of the element kernels for this topology, and the opt-in that
// lets them use more than the default 64 KiB (returns false if refused).
size_t ebe_lds_bytes(const DevPatches& P, int mode);
PatchLds ebe_patch_lds(int32_t n_mat);
bool ebe_set_lds_limit(const DevPatches& P);

// ---- node-wise kernels
void launch_combine_apply(hipStream_t s, const DevNodes& N, const double* qbuf, const double* p, int mode, double* q);
void launch_diag_finalize(hipStream_t s, const DevNodes& N, const double* qbuf6, double* binv6);
void launch_precond(hipStream_t s, const DevNodes& N, const double* binv6, const double* r, double* z);
void launch_rhs_finalize(hipStream_t s, const DevNodes& N, const double* qbuf, const double* f_ext, double* b);
// Grid of the node-wise reduction kernels (their partial-sum count).
int res_grid(int64_t n);
// mode 0: initial residual of a solve (also sets x = b on fixed dofs, resets
// the scalars); mode 1: true-residual check, runs only when due.
void launch_residual(hipStream_t s, const DevNodes& N, const double* qbuf, const double* b, const double* binv6,
                     double* x, double* r, double* z, DevScalars* sc, double* res_part, int mode);
void launch_check_finalize(hipStream_t s, DevScalars* sc, const double* res_part, int g, int j_next, double tol);
struct UpdLaunch {
    const DevNodes* N;
    int prec;
    const void* qbuf;
    const void* p;
    const void* binv;
    void* x;
    void* r;
    void* z;
    DevScalars* sc;
    const DevScalars* outer;
    const double* pap_part;
    int g_pap;
    double* res_part;
    int j;
    int32_t* inner_count;   // if set, incremented once per trip that ran
    const void* p_other;    // FP64 solve: the previous trip's direction (the pair's first half); NULL: x every trip
};
void launch_pcg_update(hipStream_t s, const UpdLaunch& L);
// At the stop of an FP64 solve (only when the true-residual check is due): the
// pending x += alpha p of the last trip, if its pair was not completed.  p_j is
// p[(par0 + j + 1) & 1] (par0: the direction buffer parity at trip 0).
void launch_flush_x(hipStream_t s, const DevNodes& N, double* x, const double* p0, const double* p1, int par0,
                    DevScalars* sc);
// Mixed precision (flexible FP64 outer PCG with an inner PCG preconditioner).
void launch_inner_init(hipStream_t s, int prec, const DevNodes& N, const double* r64, const void* binv, void* r,
                       void* e, void* z, DevScalars* outer, const double* outer_part, int j, int max_iter, double tol,
                       DevScalars* sc_in, double* in_part);
void launch_outer_z(hipStream_t s, const DevNodes& N, const void* e, const double* r, const double* r_prev, double* z,
                    const DevScalars* outer, double* part, int j);
void launch_outer_update(hipStream_t s, const DevNodes& N, const double* qbuf, const double* p, double* x, double* r,
                         double* r_prev, DevScalars* sc, const double* pap_part, int g_pap, double* part, int j);
void launch_to_f32(hipStream_t s, int64_t n, const double* in, float* out);

// ---- predictor and time integration (all lengths in dofs, 3N)
void launch_ab4(hipStream_t s, int64_t n3, double dt, const double* v1, const double* v2, const double* v3,
                const double* v4, int kind, double* dab, double* x);
constexpr int kGhStride = 32 * 32 + 32;   // per-chunk Gram [32][32] followed by X^T q [32]
// Predictor regions cut into node chunks (device arrays; see region_chunks).
struct DevChunks {
    int32_t n_regions = 0, n_chunks = 0;
    const int32_t* start = nullptr;    // [n_chunks+1] internal node ranges
    const int32_t* region = nullptr;   // [n_chunks] region of each chunk
    const int32_t* first = nullptr;    // [n_regions+1] first chunk of each region
    const int32_t* region_case = nullptr;  // batched ensembles: [n_regions] case of each region
};
// gh: [n_chunks][kGhStride] partial Grams; coef: [n_regions][32].  case_lo
// (batched ensembles, may be NULL): region r uses only the columns j >=
// case_lo[C.region_case[r]] of the window (its case's shorter window; the
// older columns get zero coefficients).
void launch_gram_solve(hipStream_t s, const ColPtrs& W, int s_eff, const DevChunks& C, double drop, double* gh,
                       double* coef, const int32_t* case_lo = nullptr);
// The partial Grams alone (gh as for launch_gram_solve).
void launch_gram(hipStream_t s, const ColPtrs& W, int s_eff, const DevChunks& C, double* gh);
// The least-squares solve alone on the partial Grams of a window of s_eff columns,
// leaving out the first lo columns in every region (the window's newest s_eff - lo).
void launch_ls_solve(hipStream_t s, int s_eff, const DevChunks& C, double drop, const double* gh, double* coef,
                     int lo);
void launch_pred_apply(hipStream_t s, const ColPtrs& W, int s_eff, const DevChunks& C, const double* coef,
                       const double* dab, double* x);
// guard (may be NULL): run only once the solve's stop flag reads converged or max_iter
void launch_newmark(hipStream_t s, int64_t n3, double dt, const double* du, const double* dab, double* u,
                    const double* v_old, double* v_new, double* a, double* ring_slot,
                    const DevScalars* guard = nullptr);
void launch_gather3(hipStream_t s, int64_t n, const int32_t* idx, const double* in, double* out);
void launch_zero(hipStream_t s, int64_t count, double* p);

// ---- batched ensembles (batch.hip): groups of r cases on one mesh, vectors
// stacked case-major [r][N][3], slots [r][PN][3]
constexpr int kMaxCaseTile = 8;
struct BEbeArgs {
    DevPatches P;
    int r;                       // cases in the group
    int64_t n3;                  // 3 N: stride between the cases of a stacked vector
    int64_t pn;                  // slots per case
    const double *in0, *in1, *in2;   // APPLY: p; PCG: z, p_prev; RHS: u, v, a
    double* p_cur;               // PCG
    double* qbuf;
    double cm, ck, c1, c2;
    const double* g;             // RHS: base acceleration per case [r][3]
    int mask_in;                 // APPLY
    DevScalars* sc;              // [r]
    const DevScalars* guard;     // APPLY: only cases with a true-residual check due
    const double* upd_part;      // update partials [2][kResArrays][r][g_upd]
    int g_upd;
    double* pap_part;            // [r][chunks]
    const int* trip;             // current trip index (device)
    int max_iter;
    double tol;
};
struct BNodeArgs {
    DevNodes N;
    int r;
    int64_t pn;
    const double* qbuf;
    const double* b;
    const double* p;
    const double* binv6;
    double *x, *r_, *z;
    DevScalars* sc;
    const double* pap_part;
    int g_pap;
    double* part;                // [2][kResArrays][r][g_upd]
    int g_upd;                   // node-wise workgroups per case (<= 256)
    const int* trip;
};
size_t bebe_lds_bytes(const DevPatches& P, int ct, int mode);
bool bebe_set_lds_limit(const DevPatches& P, int ct);
// mode: MODE_APPLY 0, MODE_PCG 1, MODE_RHS 2; grid (chunks, ceil(r / ct)), chunks a multiple of 8, <= 512
void launch_bebe(hipStream_t s, int mode, const BEbeArgs& A, int ct, int chunks);
void launch_bupdate(hipStream_t s, const BNodeArgs& A);
void launch_bresidual(hipStream_t s, const BNodeArgs& A, int mode);
void launch_bcheck_finalize(hipStream_t s, const BNodeArgs& A, double tol);
// mode 0: slot sums; 1: A_bc (fixed rows take p); 2: f + slot sums, fixed rows zero
void launch_bcombine(hipStream_t s, const BNodeArgs& A, const double* p, const double* f, double* out, int mode);
void launch_bzero_rhs_cases(hipStream_t s, const DevScalars* sc, int r, int64_t n3, double* x);
// Guarded snapshot window per case: residual partials of a guess, part [r][g_upd]; then keep
// dab in x for the cases whose AB4 residual is strictly smaller (recorded in the case scalars).
void launch_bcand_res(hipStream_t s, const BNodeArgs& A, double* part);
void launch_bguard_select(hipStream_t s, const BNodeArgs& A, const double* part_m, const double* part_a,
                          const double* dab);
void launch_set_trip(hipStream_t s, int* trip, int v);
void launch_trip_inc(hipStream_t s, int* trip);

// ---- learned node-wise predictor (mlp.hip)
constexpr int kMlpIn = 15, kMlpHid = 64, kMlpOut = 3;
constexpr int kMlpParams = kMlpHid * kMlpIn + kMlpHid + kMlpHid * kMlpHid + kMlpHid + kMlpOut * kMlpHid + kMlpOut;
constexpr int kMlpSample = kMlpIn + kMlpOut;   // one collected sample: 15 raw features + 3 raw targets
constexpr int kMlpScales = 4;                   // newest displacement, increments, force, target
// Input group of feature k: 0 displacement u^{it-1}, 1 increments, 2 force.
__host__ __device__ constexpr int mlp_group(int k) { return k < 3 ? 0 : (k < 12 ? 1 : 2); }
constexpr int kMlpMaxBatch = 8192;
// Solver state read by the in-step inference and the sample collection.
struct MlpState {
    const double* u;                              // u^{it-1}
    const double *v1, *v2, *v3, *v4;              // v^{it-1} .. v^{it-4}
    double hdt;                                   // dt / 2
    const double* msum;                           // [N] row sums of M (base-motion force)
    double g0, g1, g2;                            // base acceleration of the step
    const double* f_int;                          // extra external force (internal order) or null
    double inv_s[3];                              // 1 / scale of each input group
    double s_t;                                   // output scale
    const uint8_t* fixmask;
    const double* xs;                             // base of the candidate (Adams-Bashforth increment)
    double* xl;                                   // learned candidate xs + s_t * output (out)
};
// Training buffers (batch-major activations are stored [feature][B]).
struct MlpTrain {
    uint16_t* w;                                  // BF16 weights used by every forward
    float *wm, *m, *v;                            // FP32 master weights and Adam moments
    const float* samples;                         // collected rows of kMlpSample floats
    int64_t n_samples;
    float inv_s[3], inv_st;
    const float *x_in, *t_in;                     // explicit scaled inputs / targets (gradient checks)
    float *X, *Z1, *H1, *Z2, *H2, *dY, *dZ1, *dZ2;
    float* loss_part;
    float* grad;                                  // [kMlpParams]
};
// Row sums of M (x component of M 1) per node, from an unmasked M-only matvec.
void launch_msum(hipStream_t s, const DevNodes& N, const double* qbuf, double* msum);
// Choice between two guesses: free-row ||b - A x||^2 partials of a candidate
// (slot sums in qbuf; qbuf NULL gives ||b||^2), then keep the candidate with
// the smaller residual in x and its matvec slots in qbuf (ties keep the
// primary).  which = 0 records the result in cand_rr / cand_pick (learned
// candidate), 1 in guard_rr / guard_pick (Adams-Bashforth against the map).
// skip (may be NULL): with sc->guard_skip set, cand_res returns at once and cand_select keeps the primary.
void launch_cand_res(hipStream_t s, const DevNodes& N, const double* qbuf, const double* b, double* part,
                     const DevScalars* skip = nullptr);
void launch_cand_select(hipStream_t s, const DevNodes& N, const double* part_s, const double* part_l, double* x,
                        const double* x_alt, double* qbuf, const double* qbuf_alt, int64_t nq, DevScalars* sc,
                        int which = 0, const DevScalars* skip = nullptr);
// Guard of the snapshot map: rr_map and ||b||^2 from their partials into guard_rr[0] and
// guess_bb; guard_skip = 1 when the map's relative residual is below thresh (thresh <= 0: never).
void launch_guard_decide(hipStream_t s, const double* part_map, const double* part_bb, int g, double thresh,
                         DevScalars* sc);
// *out = sum of the g = res_grid(n) partials, in the fixed order of the solver's reductions.
void launch_sum_partials(hipStream_t s, const double* part, int g, double* out);
void launch_fill(hipStream_t s, int64_t n, double value, double* p);
void launch_mlp_infer_array(hipStream_t s, const uint16_t* w, int64_t n, const float* x, float* y);
void launch_mlp_infer_state(hipStream_t s, const uint16_t* w, const MlpState& S, int64_t n);
// Forward + backward + weight gradients (into T.grad) over B samples: rows
// idx of the collected samples when idx is set, else T.x_in / T.t_in.
void launch_mlp_grads(hipStream_t s, const MlpTrain& T, int B, const int64_t* idx);
// One Adam step (step number t >= 1) with gradient grad; if loss is set, also
// writes the loss of the last forward over B samples to loss[step].
void launch_mlp_adam(hipStream_t s, const MlpTrain& T, const float* grad, float lr, int t, int B, double* loss,
                     int step);
void launch_mlp_loss(hipStream_t s, const MlpTrain& T, int B, double* loss);
void launch_mlp_round(hipStream_t s, const float* wm, uint16_t* wb);
void launch_collect_pre(hipStream_t s, const int32_t* nodes, int k, const double* xs, double* stage);
void launch_collect_post(hipStream_t s, const MlpState& S, const int32_t* nodes, int k, const double* du,
                         const double* stage, float* out);
void launch_sample_rms(hipStream_t s, const float* samples, int64_t count, double* out4);
void launch_map_nodes(hipStream_t s, const int32_t* user, int k, const int32_t* u2i, int64_t n, int32_t* out,
                      int32_t* flag);
void launch_check_index(hipStream_t s, const int64_t* idx, int64_t m, int64_t limit, int32_t* flag);

}  // namespace ebe
