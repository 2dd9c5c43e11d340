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
    int32_t pad;
};

enum { DONE_RUNNING = 0, DONE_CONVERGED = 1, DONE_NONFINITE = 2, DONE_MAXITER = 3, DONE_ZERO_RHS = 4 };

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
struct ColPtrs {
    const double* c[kMaxCols];
};

// ---- element-by-element operator
// qbuf[pn] = sum over the patch's elements of (cm M_e + ck K_e) p_e for the
// patch's nodes; p gathered with fixed components zeroed when mask_in.
// guard: if non-NULL, the kernel runs only when a true-residual check is due.
void launch_ebe_apply(hipStream_t s, const DevPatches& P, const double* p, bool mask_in, double cm, double ck,
                      double* qbuf, const DevScalars* guard = nullptr);
// PCG trip j, matvec part: stop test on the incoming residual partials, beta,
// p_cur = z + beta p_prev, qbuf = A_e p_cur and (p, A p) partials.
int pcg_ebe_grid(const DevPatches& P);
void launch_ebe_pcg(hipStream_t s, const DevPatches& P, const double* z, const double* p_prev, double* p_cur,
                    double cm, double ck, double* qbuf, DevScalars* sc, const double* res_part, int g_res,
                    double* pap_part, int j, int max_iter, double tol);
// Right-hand side operands: M part w1 = a + c1 v - g, K part w2 = c2 v - u.
void launch_ebe_rhs(hipStream_t s, const DevPatches& P, const double* u, const double* v, const double* a,
                    double c1, double c2, double g0, double g1, double g2, double* qbuf);
// Block diagonal of cm M + ck K per patch node (6 symmetric entries).
void launch_ebe_diag(hipStream_t s, const DevPatches& P, double cm, double ck, double* qbuf6);
// Dynamic LDS of the element kernels for this topology, and the opt-in that
// lets them use more than the default 64 KiB (returns false if refused).
size_t ebe_lds_bytes(const DevPatches& P, int mode);
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
void launch_pcg_update(hipStream_t s, const DevNodes& N, const double* qbuf, const double* p, const double* binv6,
                       double* x, double* r, double* z, DevScalars* sc, const double* pap_part, int g_pap,
                       double* res_part, int j);

// ---- predictor and time integration (all lengths in dofs, 3N)
void launch_ab4(hipStream_t s, int64_t n3, double dt, const double* v1, const double* v2, const double* v3,
                const double* v4, int kind, double* dab, double* x);
constexpr int kGhStride = 32 * 32 + 32;   // per-region Gram [32][32] followed by X^T q [32]
void launch_gram_solve(hipStream_t s, const ColPtrs& W, int s_eff, int n_regions, const int32_t* region_start,
                       double drop, double* gh, double* coef);
void launch_pred_apply(hipStream_t s, const ColPtrs& W, int s_eff, int n_regions, const int32_t* region_start,
                       const double* coef, const double* dab, double* x);
void launch_newmark(hipStream_t s, int64_t n3, double dt, const double* du, const double* dab, double* u,
                    const double* v_old, double* v_new, double* a, double* ring_slot);
void launch_gather3(hipStream_t s, int64_t n, const int32_t* idx, const double* in, double* out);
void launch_zero(hipStream_t s, int64_t count, double* p);

}  // namespace ebe
