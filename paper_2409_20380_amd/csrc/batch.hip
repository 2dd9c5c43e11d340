// batch.hip -- batched ensembles: many cases (independent input waves) on one
// or more meshes advanced together.  The paper batches r cases through one
// element pass (Sec. 2.2, Eq. eqmebefem: the element data are read once for
// r right-hand sides); here a group is one mesh with r cases whose vectors
// are stacked case-major ([r][N][3]), and the element kernel maps a workgroup
// of 256 threads to (element, case) pairs: 256/CT elements x CT cases (the
// case tile CT is chosen by the autotuner).  The CT lanes of one element are
// adjacent, so they share the element's node entries and geometry loads and
// their LDS accumulator addresses are adjacent (no bank conflicts between
// them).  Every case keeps its own PCG scalars (alpha, beta, stop test,
// iteration count) -- independent CGs sharing one matvec pass -- and a case
// that has stopped is masked out of the element work.
//
// Grid-wide scalars follow the single-case design: each kernel writes one
// partial per (case, workgroup) with plain stores and the next kernel
// re-reduces the partials of its case in a fixed order.  The trip index lives
// in device memory, so a chunk of trips can be captured once in a hipGraph
// and replayed.
#include <hip/hip_runtime.h>

#include "element.h"
#include "kernels.h"

namespace ebe {

namespace {

// index of the partial of array a (0 (z,r), 1 (r,r), 2 (b,b)) of case c,
// block b, in the parity slot of trip j
__device__ __forceinline__ int64_t upd_index(int j, int a, int c, int b, int r, int g) {
    return ((int64_t)((j & 1) * kResArrays + a) * r + c) * g + b;
}

struct BSmem {
    double beta[kMaxCaseTile];
    int active[kMaxCaseTile];
    double red[kEbeWaves][kMaxCaseTile];
};

// Entries per thread per gather round: a deeper round for a single-case tile,
// where the registers allow it (3 x 256 pairs cover a 256-element patch of a
// structured mesh); the largest depth at which each case tile does not spill.
template <int CT>
constexpr int bgu() { return CT == 1 ? 3 : (CT == 2 ? 1 : 2); }

// Node entries of the first gather round of one patch, loaded one patch ahead
// (pair q = node q / CT, case q % CT).  Lanes past the patch's end load entry 0
// (in bounds) and are masked by the consumer.  Only the single-case tile
// prefetches: with CT > 1 the entries held through the element phase make the
// kernel spill, and the first round loads its entries itself.
template <int CT>
constexpr bool bprefetching() { return CT == 1; }
template <int CT>
struct BPre {
    uint32_t ent[bgu<CT>()];
};
template <int CT>
__device__ __forceinline__ void bprefetch(const DevPatches& P, int patch, BPre<CT>& f) {
    if (!bprefetching<CT>()) return;
    constexpr int NT = 64 * kEbeWaves;
    const PatchMeta m = patch_meta(P, patch);
    const int npairs = m.npn * CT;
#pragma unroll
    for (int u = 0; u < bgu<CT>(); ++u) {
        const int q = threadIdx.x + NT * u;
        f.ent[u] = ld_ro(P.nodes + (q < npairs ? m.pn0 + q / CT : 0));
    }
}

// One patch for CT cases.  Thread tid handles element tid / CT of the patch
// and case tid % CT of the tile.  pf holds this patch's first-round node
// entries and is refilled for patch `next` (if >= 0) while this patch computes.
// As in the single-case kernel, every global load of the gather is
// unconditional (inactive cases and cases past the group read case c0's
// values, lanes past the patch's end read entry 0) and unused values are
// discarded by selects, and the direction stores follow the LDS writes, so
// the compiler waits only for the loads it needs.  (Unlike the single-case
// kernel, the slots are loaded at the write-out: holding them through the
// element phase makes the case-tiled kernels spill.)  Returns this thread's
// share of (p, A p).
template <int MODE, int CT>
__device__ __forceinline__ double bebe_patch(const BEbeArgs& A, int patch, int c0, BSmem& sm, double* lds,
                                             BPre<CT>& pf, int next) {
    const DevPatches& P = A.P;
    constexpr int NT = 64 * kEbeWaves;
    constexpr int GU = bgu<CT>();
    const int tid = threadIdx.x, wave = tid >> 6;
    const int e = tid / CT, k = tid % CT;
    const PatchMeta pm_ = patch_meta(P, patch);
    const int pn0 = pm_.pn0, npn = pm_.npn, nv = pm_.nv, e0 = pm_.e0, ne = pm_.ne;
    const int stride = 3 * CT * P.max_pn;
    double* la = lds;                                       // kEbeWaves x [max_pn][CT][3]
    double* lm = la + kEbeWaves * stride;                   // [max_pn][CT][3]
    double* lk = lm + stride;                               // [max_pn][CT][3] (RHS)
    double* lx = lk + (MODE == MODE_RHS ? stride : 0);      // [max_nv][3]
    const double* lmat = lx + 3 * P.max_nv;                 // [n_mat][3]
    const int npairs = npn * CT;

    // Gather round over (node, case) pairs, case fastest.
    auto gather = [&](auto first, int qb) {
        uint32_t ent[GU];
#pragma unroll
        for (int u = 0; u < GU; ++u) {
            const int q = qb + tid + NT * u;
            const uint32_t en = (decltype(first)::value && bprefetching<CT>()) ? pf.ent[u]
                                                                                : ld_ro(P.nodes + (q < npairs ? pn0 + q / CT : 0));
            ent[u] = q < npairs ? en : 0u;
        }
        double v[GU][3], w[GU][3], a3[GU][3], xc[GU][3];
        uint8_t fm[GU];
#pragma unroll
        for (int u = 0; u < GU; ++u) {
            const int q = qb + tid + NT * u;
            const int j = q / CT, kk = q % CT;
            const int64_t g = (int64_t)(ent[u] & ~kOwnerBit);
            const int cc = c0 + kk < A.r ? c0 + kk : c0;      // a case of the group (c0 < r)
            const int64_t o = (int64_t)cc * A.n3 + 3 * g;
            const int64_t gx = (kk == 0 && j < nv) ? g : 0;
            if (MODE == MODE_APPLY) fm[u] = ld_ro(P.fixmask + g);
#pragma unroll
            for (int d = 0; d < 3; ++d) {
                v[u][d] = ld_ro(A.in0 + o + d);
                if (MODE != MODE_APPLY) w[u][d] = ld_ro(A.in1 + o + d);
                if (MODE == MODE_RHS) a3[u][d] = ld_ro(A.in2 + o + d);
                xc[u][d] = ld_ro(P.coords + 3 * gx + d);
            }
        }
        double mo[GU][3];
#pragma unroll
        for (int u = 0; u < GU; ++u) {
            const int q = qb + tid + NT * u;
            const int j = q / CT, kk = q % CT;
            const bool act = sm.active[kk] != 0;
            double m[3];
            if (MODE == MODE_APPLY) {
                const bool mask = A.mask_in != 0;
#pragma unroll
                for (int d = 0; d < 3; ++d) m[d] = (!act || (mask && ((fm[u] >> d) & 1))) ? 0.0 : v[u][d];
            } else if (MODE == MODE_PCG) {
                const double b = sm.beta[kk];
#pragma unroll
                for (int d = 0; d < 3; ++d) {
                    // p_prev is not used on the first trip of a cycle (beta = 0) nor for a stopped case
                    const double wv = (act && b != 0.0) ? w[u][d] : 0.0;
                    m[d] = act ? fma(b, wv, v[u][d]) : 0.0;
                }
            } else {   // RHS: mass operand a + c1 v - g, stiffness operand c2 v - u
                const double* gc = A.g + 3 * (act ? c0 + kk : 0);
#pragma unroll
                for (int d = 0; d < 3; ++d) {
                    m[d] = act ? fma(A.c1, w[u][d], a3[u][d]) - gc[d] : 0.0;
                    if (q < npairs) lk[(j * CT + kk) * 3 + d] = act ? fma(A.c2, w[u][d], -v[u][d]) : 0.0;
                }
            }
#pragma unroll
            for (int d = 0; d < 3; ++d) mo[u][d] = m[d];
            if (q < npairs) {
#pragma unroll
                for (int d = 0; d < 3; ++d) {
                    lm[(j * CT + kk) * 3 + d] = m[d];
#pragma unroll
                    for (int ww = 0; ww < kEbeWaves; ++ww) la[ww * stride + (j * CT + kk) * 3 + d] = 0.0;
                }
            }
            if (kk == 0 && j < nv) {
#pragma unroll
                for (int d = 0; d < 3; ++d) lx[3 * j + d] = xc[u][d];
            }
        }
        if (MODE == MODE_PCG) {
#pragma unroll
            for (int u = 0; u < GU; ++u) {
                const int q = qb + tid + NT * u;
                const int kk = q % CT;
                const int64_t g = (int64_t)(ent[u] & ~kOwnerBit);
                if (sm.active[kk] && (ent[u] & kOwnerBit)) {   // entries past the end are 0: no owner bit
                    double* pc = A.p_cur + (int64_t)(c0 + kk) * A.n3 + 3 * g;
                    pc[0] = mo[u][0]; pc[1] = mo[u][1]; pc[2] = mo[u][2];
                }
            }
        }
    };
    // this thread's element record, in flight with the node values
    const ElemRec rec = ld_ro(P.elems + (e < ne ? e0 + e : 0));
    gather(Bool<true>{}, 0);
    for (int qb = NT * GU; qb < npairs; qb += NT * GU) gather(Bool<false>{}, qb);
    bprefetch<CT>(P, next >= 0 ? next : patch, pf);   // in flight during this patch's elements
    __syncthreads();

    double pap = 0.0;
    if (e < ne && sm.active[k]) {
        double* acc = la + wave * stride;
        GeoT<double> G;
        tet_geo<double>(lx + 3 * rec.lid[0], lx + 3 * rec.lid[1], lx + 3 * rec.lid[2], lx + 3 * rec.lid[3], G);
        const double* mp = lmat + 3 * rec.mat;
        const double w = G.V * (1.0 / 20.0) * A.ck;
        const double lamV = mp[0] * w, muV = mp[1] * w;
        const double mc = (A.cm * mp[2]) * G.V * (1.0 / 420.0);
        double pm[10][3], pk[10][3];
#pragma unroll
        for (int i = 0; i < 10; ++i) {
            const int l = rec.lid[i];
#pragma unroll
            for (int d = 0; d < 3; ++d) pm[i][d] = lm[(l * CT + k) * 3 + d];
        }
        auto emit = [&](int i, double f0, double f1, double f2) {
            const int l = rec.lid[i];
            double* a = acc + (l * CT + k) * 3;
            lds_add(a, f0);
            lds_add(a + 1, f1);
            lds_add(a + 2, f2);
            if (MODE == MODE_PCG) pap = fma(pm[i][0], f0, fma(pm[i][1], f1, fma(pm[i][2], f2, pap)));
        };
        if (MODE == MODE_RHS) {
#pragma unroll
            for (int i = 0; i < 10; ++i) {
                const int l = rec.lid[i];
#pragma unroll
                for (int d = 0; d < 3; ++d) pk[i][d] = lk[(l * CT + k) * 3 + d];
            }
            element_apply_emit<double>(pm, pk, G, lamV, muV, mc, emit);
        } else {
            element_apply_emit<double>(pm, pm, G, lamV, muV, mc, emit);
        }
    }
    __syncthreads();
    // Write-out: the kEbeWaves accumulators of each (node, case) pair, summed in
    // a fixed order, go to the pair's slot.
    auto write_out = [&](int qb, int sli) {
        const int q = qb + tid;
        const int j = q / CT, kk = q % CT;
        if (q >= npairs) return;
        double s3[3];
#pragma unroll
        for (int d = 0; d < 3; ++d) {
            double t = la[(j * CT + kk) * 3 + d];
#pragma unroll
            for (int ww = 1; ww < kEbeWaves; ++ww) t += la[ww * stride + (j * CT + kk) * 3 + d];
            s3[d] = t;
        }
        if (sm.active[kk]) {
            double* qo = A.qbuf + 3 * ((int64_t)(c0 + kk) * A.pn + sli);
            qo[0] = s3[0]; qo[1] = s3[1]; qo[2] = s3[2];
        }
    };
    if constexpr (CT == 1) {
        // slots of a group of GU rounds are loaded before any is used (entry 0 past the end)
        for (int qb = 0; qb < npairs; qb += NT * GU) {
            int sl[GU];
#pragma unroll
            for (int u = 0; u < GU; ++u) {
                const int q = qb + NT * u + tid;
                sl[u] = ld_ro(P.slot + (q < npairs ? pn0 + q : 0));
            }
#pragma unroll
            for (int u = 0; u < GU; ++u) write_out(qb + NT * u, sl[u]);
        }
    } else {
        // (grouping the slot loads makes the case-tiled kernels spill)
        for (int qb = 0; qb < npairs; qb += NT)
            write_out(qb, ld_ro(P.slot + (qb + tid < npairs ? pn0 + (qb + tid) / CT : 0)));
    }
    __syncthreads();
    return pap;
}

// Sum over the lanes of one wavefront that share lane % CT; lane k < CT gets
// the sum of its case (fixed butterfly order).
template <int CT>
__device__ __forceinline__ double case_wave_sum(double v) {
#pragma unroll
    for (int o = 32; o >= CT; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

// Element pass over a chunk of patches for the case tile blockIdx.y.
// APPLY: q = A_e p (guarded cases only when A.guard is set); RHS; PCG: the
// per-case stop test on the incoming partials, beta, p = z + beta p and
// q = A p with the (p, A p) partials of each case.
template <int MODE, int CT>
__global__ __launch_bounds__(64 * kEbeWaves, 2) void k_bebe(BEbeArgs A) {
    extern __shared__ double lds[];
    __shared__ BSmem sm;
    const int tid = threadIdx.x;
    const int c0 = blockIdx.y * CT;
    if (MODE == MODE_PCG) {
        const int j = *A.trip;
        const int g = A.g_upd;
        for (int kk = 0; kk < CT; ++kk) {
            const int c = c0 + kk;
            if (c >= A.r) {
                if (tid == 0) { sm.active[kk] = 0; sm.beta[kk] = 0.0; }
                continue;
            }
            DevScalars* sc = A.sc + c;
            double zr = 0.0, rr = 0.0, bb = 0.0, unused = 0.0;
            if (tid < g) {   // the (b, b) array exists in both slots: read with the others, used on trip 0
                zr = A.upd_part[upd_index(j, 0, c, tid, A.r, g)];
                rr = A.upd_part[upd_index(j, 1, c, tid, A.r, g)];
                bb = A.upd_part[upd_index(j, 2, c, tid, A.r, g)];
            }
            block_bcast_sum4(zr, rr, bb, unused);
            if (j != 0) bb = 0.0;
            int stop = sc->done;
            double beta = 0.0;
            if (stop == DONE_RUNNING) {
                const double bnorm = (j == 0) ? sqrt(bb) : sc->bnorm;
                const double res = bnorm > 0.0 ? sqrt(rr) / bnorm : 0.0;
                if (bnorm == 0.0) stop = DONE_ZERO_RHS;
                else if (!isfinite(res) || !isfinite(zr)) stop = DONE_NONFINITE;
                else if (res < A.tol) stop = DONE_CONVERGED;
                else if (sc->iters >= A.max_iter) stop = DONE_MAXITER;
                if (stop == DONE_RUNNING && j != sc->cycle_start) {
                    beta = zr / sc->rho[(j - 1) & 1];
                    if (!isfinite(beta)) stop = DONE_NONFINITE;
                }
                if (blockIdx.x == 0 && tid == 0) {
                    if (j == 0) {
                        sc->bnorm = bnorm;
                        sc->res0 = res;
                    }
                    sc->rr = rr;
                    if (stop != DONE_RUNNING) sc->done = stop;
                    else sc->rho[j & 1] = zr;
                }
            }
            if (tid == 0) {
                sm.active[kk] = stop == DONE_RUNNING;
                sm.beta[kk] = beta;
            }
        }
    } else {
        if (tid < CT) {
            const int c = c0 + tid;
            sm.active[tid] = c < A.r && (!A.guard || check_due(A.guard + c));
            sm.beta[tid] = 0.0;
        }
    }
    __syncthreads();
    bool any = false;
#pragma unroll
    for (int kk = 0; kk < CT; ++kk) any = any || sm.active[kk];
    if (!any) {
        if (MODE == MODE_PCG && tid < CT && c0 + tid < A.r) A.pap_part[(int64_t)(c0 + tid) * gridDim.x + blockIdx.x] = 0.0;
        return;
    }
    const int nb = gridDim.x;   // multiple of 8
    const int xcd = blockIdx.x & 7, k0 = blockIdx.x >> 3, per_xcd = nb >> 3;
    const int chunk = A.P.n_patches_pad >> 3;
    double pap_acc = 0.0;
    {
        const int stride = 3 * CT * A.P.max_pn;
        stage_material_table(A.P, lds + (size_t)stride * (kEbeWaves + (MODE == MODE_RHS ? 2 : 1)) + 3 * A.P.max_nv,
                             64 * kEbeWaves);
    }
    BPre<CT> pf;
    if (k0 < chunk) bprefetch<CT>(A.P, xcd * chunk + k0, pf);
    for (int kq = k0; kq < chunk; kq += per_xcd) {
        const int kn = kq + per_xcd;
        const double pap = bebe_patch<MODE, CT>(A, xcd * chunk + kq, c0, sm, lds, pf, kn < chunk ? xcd * chunk + kn : -1);
        if (MODE == MODE_PCG) {
            const double ws = case_wave_sum<CT>(pap);
            if ((tid & 63) < CT) sm.red[tid >> 6][tid & 63] = ws;
            __syncthreads();
            if (tid < CT) pap_acc += (sm.red[0][tid] + sm.red[1][tid]) + (sm.red[2][tid] + sm.red[3][tid]);
            __syncthreads();
        }
    }
    if (MODE == MODE_PCG && tid < CT && c0 + tid < A.r)
        A.pap_part[(int64_t)(c0 + tid) * gridDim.x + blockIdx.x] = pap_acc;
}

// node range of block b of g blocks over n nodes
__device__ __forceinline__ void node_range(int64_t n, int b, int g, int64_t& lo, int64_t& hi) {
    const int64_t per = (n + g - 1) / g;
    lo = (int64_t)b * per;
    hi = lo + per < n ? lo + per : n;
}

__device__ __forceinline__ void gather_slots(const DevNodes& N, const double* q, int64_t n, double& q0, double& q1,
                                             double& q2) {
    const int k0 = N.slot_ptr[n], k1 = N.slot_ptr[n + 1];
    double s[3];
    sum_slots(q, k0, k1 - k0, s);
    q0 = s[0]; q1 = s[1]; q2 = s[2];
}

// Trip j, update part for case blockIdx.y: alpha = rho_j / (p, A p), r -= alpha q,
// x += alpha p, z = B^{-1} r, partials (z, r), (r, r) for trip j + 1.
__global__ __launch_bounds__(256) void k_bupdate(BNodeArgs A) {
    const int c = blockIdx.y;
    DevScalars* sc = A.sc + c;
    if (sc->done) return;
    const int j = *A.trip;
    double pap = lane_partials<kMaxPcgGrid / 256>(A.pap_part + (int64_t)c * A.g_pap, A.g_pap, threadIdx.x, 256);
    pap = block_bcast_sum(pap);
    const double alpha = sc->rho[j & 1] / pap;
    double v0 = 0.0, v1 = 0.0;
    if (isfinite(alpha)) {
        const int64_t off = (int64_t)c * 3 * A.N.n;
        const double* q = A.qbuf + 3 * (int64_t)c * A.pn;
        int64_t lo, hi;
        node_range(A.N.n, blockIdx.x, gridDim.x, lo, hi);
        // Every load of a node is issued before the first store (the stores to
        // x, r and z could alias the later loads as far as the compiler knows).
        for (int64_t n = lo + threadIdx.x; n < hi; n += blockDim.x) {
            const int k0 = A.N.slot_ptr[n], ns = A.N.slot_ptr[n + 1] - k0;
            const uint8_t fm = A.N.fixmask[n];
            const int64_t i = off + 3 * n;
            double rv[3], xv[3], pv[3], B[6];
#pragma unroll
            for (int d = 0; d < 3; ++d) {
                rv[d] = A.r_[i + d];
                xv[d] = A.x[i + d];
                pv[d] = A.p[i + d];
            }
#pragma unroll
            for (int t = 0; t < 6; ++t) B[t] = A.binv6[6 * n + t];
            double qv[3];
            sum_slots(q, k0, ns, qv);
            if (fm & 1) qv[0] = 0.0;
            if (fm & 2) qv[1] = 0.0;
            if (fm & 4) qv[2] = 0.0;
            const double r0 = fma(-alpha, qv[0], rv[0]), r1 = fma(-alpha, qv[1], rv[1]), r2 = fma(-alpha, qv[2], rv[2]);
            double z0, z1, z2;
            apply_binv(B, r0, r1, r2, z0, z1, z2);
            A.x[i] = fma(alpha, pv[0], xv[0]);
            A.x[i + 1] = fma(alpha, pv[1], xv[1]);
            A.x[i + 2] = fma(alpha, pv[2], xv[2]);
            A.r_[i] = r0; A.r_[i + 1] = r1; A.r_[i + 2] = r2;
            A.z[i] = z0; A.z[i + 1] = z1; A.z[i + 2] = z2;
            v0 += z0 * r0 + z1 * r1 + z2 * r2;
            v1 += r0 * r0 + r1 * r1 + r2 * r2;
        }
        if (blockIdx.x == 0 && threadIdx.x == 0) sc->iters += 1;   // trips done by this case
    } else if (blockIdx.x == 0 && threadIdx.x == 0) {
        sc->done = DONE_NONFINITE;
    }
    v0 = block_bcast_sum(v0);
    v1 = block_bcast_sum(v1);
    if (threadIdx.x == 0) {
        A.part[upd_index(j + 1, 0, c, blockIdx.x, A.r, gridDim.x)] = v0;
        A.part[upd_index(j + 1, 1, c, blockIdx.x, A.r, gridDim.x)] = v1;
    }
}

// r = b - A x from the slots, z = B^{-1} r, partials (z,r), (r,r), (b,b) in
// the parity slot of the current trip.  mode 0 (start of a solve): also
// x = b on fixed dofs and resets the case's scalars; mode 1 (true-residual
// check): cases with a check due only.
__global__ __launch_bounds__(256) void k_bresidual(BNodeArgs A, int mode) {
    const int c = blockIdx.y;
    DevScalars* sc = A.sc + c;
    if (mode == 1 && !check_due(sc)) return;
    const int j = mode == 0 ? 0 : *A.trip;
    if (mode == 0 && blockIdx.x == 0 && threadIdx.x == 0) {
        sc->done = DONE_RUNNING;
        sc->iters = 0;
        sc->restarts = 0;
        sc->checked = 0;
        sc->cycle_start = 0;
        sc->res_true = 0.0;
    }
    const int64_t off = (int64_t)c * 3 * A.N.n;
    const double* q = A.qbuf + 3 * (int64_t)c * A.pn;
    int64_t lo, hi;
    node_range(A.N.n, blockIdx.x, gridDim.x, lo, hi);
    double v0 = 0.0, v1 = 0.0, v2 = 0.0;
    // every load of a node before its first store
    for (int64_t n = lo + threadIdx.x; n < hi; n += blockDim.x) {
        const int k0 = A.N.slot_ptr[n], k1 = A.N.slot_ptr[n + 1];
        const uint8_t fm = A.N.fixmask[n];
        const int64_t i = off + 3 * n;
        const double b0 = A.b[i], b1 = A.b[i + 1], b2 = A.b[i + 2];
        double B[6], qv[3];
#pragma unroll
        for (int t = 0; t < 6; ++t) B[t] = A.binv6[6 * n + t];
        sum_slots(q, k0, k1 - k0, qv);
        if (mode == 0 && fm) {
            if (fm & 1) A.x[i] = b0;
            if (fm & 2) A.x[i + 1] = b1;
            if (fm & 4) A.x[i + 2] = b2;
        }
        const double r0 = (fm & 1) ? 0.0 : b0 - qv[0];
        const double r1 = (fm & 2) ? 0.0 : b1 - qv[1];
        const double r2 = (fm & 4) ? 0.0 : b2 - qv[2];
        double z0, z1, z2;
        apply_binv(B, r0, r1, r2, z0, z1, z2);
        A.r_[i] = r0; A.r_[i + 1] = r1; A.r_[i + 2] = r2;
        A.z[i] = z0; A.z[i + 1] = z1; A.z[i + 2] = z2;
        v0 += z0 * r0 + z1 * r1 + z2 * r2;
        v1 += r0 * r0 + r1 * r1 + r2 * r2;
        v2 += b0 * b0 + b1 * b1 + b2 * b2;
    }
    v0 = block_bcast_sum(v0);
    v1 = block_bcast_sum(v1);
    v2 = block_bcast_sum(v2);
    if (threadIdx.x == 0) {
        A.part[upd_index(j, 0, c, blockIdx.x, A.r, gridDim.x)] = v0;
        A.part[upd_index(j, 1, c, blockIdx.x, A.r, gridDim.x)] = v1;
        A.part[upd_index(j, 2, c, blockIdx.x, A.r, gridDim.x)] = v2;
    }
}

// One workgroup per case: finish the true-residual check; restart the CG
// cycle of a case whose recursive residual converged but whose true
// residual did not.
__global__ __launch_bounds__(256) void k_bcheck_finalize(BNodeArgs A, double tol) {
    const int c = blockIdx.x;
    DevScalars* sc = A.sc + c;
    if (!check_due(sc)) return;
    const int j = *A.trip;
    const double rr = block_bcast_sum(threadIdx.x < A.g_upd ? A.part[upd_index(j, 1, c, threadIdx.x, A.r, A.g_upd)]
                                                            : 0.0);
    if (threadIdx.x == 0) {
        const double res = sqrt(rr) / sc->bnorm;
        sc->res_true = res;
        sc->checked = 1;
        if (!isfinite(res)) {
            sc->done = DONE_NONFINITE;
        } else if (res >= tol && sc->done == DONE_CONVERGED) {
            sc->done = DONE_RUNNING;
            sc->checked = 0;
            sc->restarts += 1;
            sc->cycle_start = j;
        }
    }
}

// q = slot sums (mode 0) or A_bc (mode 1: fixed rows take p); b = f + slot
// sums with fixed rows zeroed (mode 2).
__global__ __launch_bounds__(256) void k_bcombine(BNodeArgs A, const double* p, const double* f, double* out,
                                                  int mode) {
    const int c = blockIdx.y;
    const int64_t off = (int64_t)c * 3 * A.N.n;
    const double* q = A.qbuf + 3 * (int64_t)c * A.pn;
    int64_t lo, hi;
    node_range(A.N.n, blockIdx.x, gridDim.x, lo, hi);
    // every load of a node (unconditional for the launch's mode) before its first store
    for (int64_t n = lo + threadIdx.x; n < hi; n += blockDim.x) {
        const int k0 = A.N.slot_ptr[n], k1 = A.N.slot_ptr[n + 1];
        const uint8_t fm = A.N.fixmask[n];
        const int64_t i = off + 3 * n;
        double pv[3] = {0.0, 0.0, 0.0}, fv[3] = {0.0, 0.0, 0.0}, s[3];
        if (mode == 1) {
#pragma unroll
            for (int d = 0; d < 3; ++d) pv[d] = p[i + d];
        }
        if (mode == 2 && f) {
#pragma unroll
            for (int d = 0; d < 3; ++d) fv[d] = f[i + d];
        }
        sum_slots(q, k0, k1 - k0, s);
#pragma unroll
        for (int d = 0; d < 3; ++d) {
            double v = s[d];
            if (mode == 1 && ((fm >> d) & 1)) v = pv[d];
            if (mode == 2) v = ((fm >> d) & 1) ? 0.0 : v + fv[d];
            out[i + d] = v;
        }
    }
}

// x = 0 for the cases that stopped on a zero right-hand side.
__global__ void k_bzero_rhs_cases(const DevScalars* sc, int64_t n3, double* x) {
    const int c = blockIdx.y;
    if (sc[c].done != DONE_ZERO_RHS) return;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n3; i += (int64_t)gridDim.x * blockDim.x)
        x[(int64_t)c * n3 + i] = 0.0;
}

// Guarded snapshot window, per case: free-row ||b - A x||^2 partials of one
// guess (its slots in A.qbuf) into part[c][g_upd].
__global__ __launch_bounds__(256) void k_bcand_res(BNodeArgs A, double* part) {
    const int c = blockIdx.y;
    const int64_t off = (int64_t)c * 3 * A.N.n;
    const double* q = A.qbuf + 3 * (int64_t)c * A.pn;
    int64_t lo, hi;
    node_range(A.N.n, blockIdx.x, gridDim.x, lo, hi);
    double v = 0.0;
    for (int64_t n = lo + threadIdx.x; n < hi; n += blockDim.x) {
        double q0, q1, q2;
        gather_slots(A.N, q, n, q0, q1, q2);
        const uint8_t fm = A.N.fixmask[n];
        const int64_t i = off + 3 * n;
        const double r0 = (fm & 1) ? 0.0 : A.b[i] - q0;
        const double r1 = (fm & 2) ? 0.0 : A.b[i + 1] - q1;
        const double r2 = (fm & 4) ? 0.0 : A.b[i + 2] - q2;
        v += r0 * r0 + r1 * r1 + r2 * r2;
    }
    v = block_bcast_sum(v);
    if (threadIdx.x == 0) part[(int64_t)c * gridDim.x + blockIdx.x] = v;
}

// Per case: the map's guess (in x, partials part_m) against the AB4 guess
// (dab, partials part_a); the AB4 guess replaces x when its residual is
// strictly smaller.  Every workgroup of a case sums the partials in the same
// order; workgroup 0 records the result in the case's scalars.
__global__ __launch_bounds__(256) void k_bguard_select(BNodeArgs A, const double* part_m, const double* part_a,
                                                       const double* dab) {
    const int c = blockIdx.y;
    const double rm = block_bcast_sum(threadIdx.x < A.g_upd ? part_m[(int64_t)c * A.g_upd + threadIdx.x] : 0.0);
    const double ra = block_bcast_sum(threadIdx.x < A.g_upd ? part_a[(int64_t)c * A.g_upd + threadIdx.x] : 0.0);
    const bool pick = ra < rm;
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        A.sc[c].guard_rr[0] = rm;
        A.sc[c].guard_rr[1] = ra;
        A.sc[c].guard_pick = pick ? 1 : 0;
    }
    if (!pick) return;
    const int64_t off = (int64_t)c * 3 * A.N.n;
    int64_t lo, hi;
    node_range(A.N.n, blockIdx.x, gridDim.x, lo, hi);
    for (int64_t i = 3 * lo + threadIdx.x; i < 3 * hi; i += blockDim.x) A.x[off + i] = dab[off + i];
}

__global__ void k_set_trip(int* trip, int v) { *trip = v; }
__global__ void k_trip_inc(int* trip) { *trip += 1; }

template <int MODE>
void launch_bebe_ct(hipStream_t s, const BEbeArgs& A, int ct, int chunks, int tiles, size_t lds) {
    const dim3 grid(chunks, tiles), block(64 * kEbeWaves);
    switch (ct) {
        case 1: hipLaunchKernelGGL((k_bebe<MODE, 1>), grid, block, lds, s, A); break;
        case 2: hipLaunchKernelGGL((k_bebe<MODE, 2>), grid, block, lds, s, A); break;
        case 4: hipLaunchKernelGGL((k_bebe<MODE, 4>), grid, block, lds, s, A); break;
        default: hipLaunchKernelGGL((k_bebe<MODE, 8>), grid, block, lds, s, A); break;
    }
}

template <int MODE>
const void* bebe_fn(int ct) {
    switch (ct) {
        case 1: return (const void*)k_bebe<MODE, 1>;
        case 2: return (const void*)k_bebe<MODE, 2>;
        case 4: return (const void*)k_bebe<MODE, 4>;
        default: return (const void*)k_bebe<MODE, 8>;
    }
}

}  // namespace

size_t bebe_lds_bytes(const DevPatches& P, int ct, int mode) {
    return sizeof(double) *
           ((size_t)3 * ct * P.max_pn * (kEbeWaves + (mode == MODE_RHS ? 2 : 1)) + 3 * P.max_nv + 3 * P.n_mat);
}

bool bebe_set_lds_limit(const DevPatches& P, int ct) {
    const size_t need = bebe_lds_bytes(P, ct, MODE_RHS);
    int dev = 0, maxlds = 0;
    if (hipGetDevice(&dev) != hipSuccess) return false;
    if (hipDeviceGetAttribute(&maxlds, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess) return false;
    // static shared (BSmem, reductions) comes on top of the dynamic part
    if (need + 1024 > (size_t)maxlds) return false;
    if (need <= 65536 - 1024) return true;
    const int v = (int)need;
    const void* fns[] = {bebe_fn<MODE_APPLY>(ct), bebe_fn<MODE_PCG>(ct), bebe_fn<MODE_RHS>(ct)};
    for (const void* f : fns)
        if (hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, v) != hipSuccess) return false;
    return true;
}

void launch_bebe(hipStream_t s, int mode, const BEbeArgs& A, int ct, int chunks) {
    const int tiles = (A.r + ct - 1) / ct;
    const size_t lds = bebe_lds_bytes(A.P, ct, mode);
    if (mode == MODE_APPLY) launch_bebe_ct<MODE_APPLY>(s, A, ct, chunks, tiles, lds);
    else if (mode == MODE_PCG) launch_bebe_ct<MODE_PCG>(s, A, ct, chunks, tiles, lds);
    else launch_bebe_ct<MODE_RHS>(s, A, ct, chunks, tiles, lds);
}

void launch_bupdate(hipStream_t s, const BNodeArgs& A) {
    hipLaunchKernelGGL(k_bupdate, dim3(A.g_upd, A.r), dim3(256), 0, s, A);
}

void launch_bresidual(hipStream_t s, const BNodeArgs& A, int mode) {
    hipLaunchKernelGGL(k_bresidual, dim3(A.g_upd, A.r), dim3(256), 0, s, A, mode);
}

void launch_bcheck_finalize(hipStream_t s, const BNodeArgs& A, double tol) {
    hipLaunchKernelGGL(k_bcheck_finalize, dim3(A.r), dim3(256), 0, s, A, tol);
}

void launch_bcombine(hipStream_t s, const BNodeArgs& A, const double* p, const double* f, double* out, int mode) {
    hipLaunchKernelGGL(k_bcombine, dim3(A.g_upd, A.r), dim3(256), 0, s, A, p, f, out, mode);
}

void launch_bzero_rhs_cases(hipStream_t s, const DevScalars* sc, int r, int64_t n3, double* x) {
    hipLaunchKernelGGL(k_bzero_rhs_cases, dim3(64, r), dim3(256), 0, s, sc, n3, x);
}

void launch_bcand_res(hipStream_t s, const BNodeArgs& A, double* part) {
    hipLaunchKernelGGL(k_bcand_res, dim3(A.g_upd, A.r), dim3(256), 0, s, A, part);
}

void launch_bguard_select(hipStream_t s, const BNodeArgs& A, const double* part_m, const double* part_a,
                          const double* dab) {
    hipLaunchKernelGGL(k_bguard_select, dim3(A.g_upd, A.r), dim3(256), 0, s, A, part_m, part_a, dab);
}

void launch_set_trip(hipStream_t s, int* trip, int v) { hipLaunchKernelGGL(k_set_trip, dim3(1), dim3(1), 0, s, trip, v); }
void launch_trip_inc(hipStream_t s, int* trip) { hipLaunchKernelGGL(k_trip_inc, dim3(1), dim3(1), 0, s, trip); }

}  // namespace ebe
