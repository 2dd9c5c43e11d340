// kernels.hip -- gfx950 kernels of the single-case element-by-element
// Newmark / PCG path.
//
// Element-by-element matvec (Eq. EBE / Eq. eqebefem):
//   q = sum_e P_e^T (cm M_e + ck K_e) P_e p
// for straight 10-node tetrahedra (element operator in element.h).  One
// workgroup of kEbeWaves wavefronts owns one patch of up to 256 elements (one
// element per thread): it gathers the patch's nodal values into LDS once,
// evaluates every element from its vertex coordinates, accumulates the
// element results into per-wave LDS accumulators (deterministic: a single
// wave issues its LDS atomics in program order), sums the accumulators in a
// fixed order and writes one 3-vector per (patch, node) slot.  Each node then
// sums its slots in patch order, so no global atomics are used and results
// are bitwise reproducible.
#include <hip/hip_runtime.h>

#include <cmath>

#include "element.h"
#include "kernels.h"

namespace ebe {

// ---------------------------------------------------------------------------
// element-by-element kernel (one wavefront per patch)
// ---------------------------------------------------------------------------

// Operands of the element kernels.  APPLY and RHS read FP64 vectors; PCG reads
// z and p_prev in the storage type S of its solve and writes p_cur in S and the
// slots in the compute type T.
struct EbeArgs {
    DevPatches P;
    const void* in0;     // APPLY: p; PCG: z; RHS: u
    const void* in1;     // PCG: p_prev; RHS: v
    const double* in2;   // RHS: a
    void* p_cur;         // PCG
    void* qbuf;
    double cm, ck;
    double c1, c2;       // RHS: w1 = a + c1 v - g, w2 = c2 v - u
    double g0, g1, g2;
    int mask_in;         // APPLY
    const DevScalars* guard;  // APPLY: run only when a true-residual check is due
    const DevScalars* skip;   // APPLY: return at once when guard_skip is set
};


// Node entries of one patch, loaded one patch ahead by the persistent matvec
// so that the index load is off the critical path: only the node values are
// loaded after it.  (The output slots and the element record are loaded with
// the patch's own node values: they are first used after the gather.  Slots
// carried from one patch to the next were copied between registers at the
// loop's back edge, which made every wave wait there for its slot stores.)
// Lanes past the patch's end load entry 0 (in bounds, also for an empty
// padding patch) and are masked by the consumer, so nothing here waits for
// the loads.
// Node entries per thread per gather round: 3 x 256 = 768 covers the patches of
// 256 elements seen on structured tetrahedral meshes (560-630 nodes); larger
// patches take more rounds.  (Four entries per thread would not fit beside the
// element's registers without spilling.)
constexpr int kGU = 3;
struct PatchPre {
    uint32_t ent[kGU];   // node entries of the first gather round (unmasked)
};

__device__ __forceinline__ void prefetch_gather(const DevPatches& P, int patch, PatchPre& f) {
    constexpr int NT = 64 * kEbeWaves;
    const int tid = threadIdx.x;
    const PatchMeta m = patch_meta(P, patch);
#pragma unroll
    for (int u = 0; u < kGU; ++u) {
        const int j = tid + NT * u;
        f.ent[u] = ld_ro(P.nodes + (j < m.npn ? m.pn0 + j : 0));
    }
}

__device__ __forceinline__ void patch_prefetch(const DevPatches& P, int patch, PatchPre& f) {
    prefetch_gather(P, patch, f);
}

// One patch on one workgroup of kEbeWaves wavefronts (one element per thread),
// compute type T, storage type S of the PCG vectors.  The waves share the
// gather of the patch's nodes into LDS; wave w adds its elements' results into
// its own LDS accumulator (a single wave issues its LDS atomics in program
// order), and the kEbeWaves accumulators are summed in a fixed order: results
// are bitwise reproducible.  pf holds this patch's index data on entry and is
// refilled for patch `next` (if >= 0) while this patch computes.
// The gather and write-out of a patch of up to kGU x 256 nodes are one
// straight-line round each; every global load in them is unconditional (lanes
// past the patch's end read a valid entry, lanes past its vertices read node
// 0's coordinates) and unused values are discarded by selects, so that the
// compiler waits for exactly the loads it needs.  Larger patches take further
// rounds.  Returns this thread's share of (p, A p) (PCG).
template <int MODE, class T, class S>
__device__ __forceinline__ double ebe_patch(const EbeArgs& A, int patch, double beta_d, double* lds, PatchPre& pf,
                                            int next) {
    const DevPatches& P = A.P;
    constexpr int NT = 64 * kEbeWaves;
    constexpr int GU = kGU;
    const int tid = threadIdx.x, wave = tid >> 6;
    const PatchMeta m = patch_meta(P, patch);
    const int pn0 = m.pn0, npn = m.npn, nv = m.nv, e0 = m.e0, ne = m.ne;
    const int stride = 3 * P.max_pn;
    const T beta = (T)beta_d;
    const bool use_in1 = MODE == MODE_RHS || (MODE == MODE_PCG && beta_d != 0.0);
    // The per-wave accumulators are FP64 in every variant: LDS FP32 atomic adds
    // were measured to stall the LDS queue (about 8x the issue wait of the FP64
    // ones), and FP64 accumulation is at least as accurate.
    double* la = lds;                                      // kEbeWaves x [max_pn][3] accumulators
    T* lm = reinterpret_cast<T*>(la + kEbeWaves * stride); // [max_pn][3] mass (or shared) operand
    T* lk = lm + stride;                                   // [max_pn][3] stiffness operand (RHS)
    T* lx = lk + (MODE == MODE_RHS ? stride : 0);          // [max_nv][3] vertex coordinates
    // [n_mat][3] material table (lambda, mu, rho), after the FP64-sized regions above
    const double* lmat = lds + (size_t)stride * (kEbeWaves + (MODE == MODE_RHS ? 2 : 1)) + 3 * P.max_nv;
    const S* in0 = static_cast<const S*>(A.in0);
    const S* in1 = static_cast<const S*>(A.in1);

    // Gather round: all loads of GU x NT node entries are issued before any is
    // consumed; the first round also issues the loads of its output slots.
    int sl0[GU];
    auto gather = [&](auto first, int jb) {
        uint32_t ent[GU];
#pragma unroll
        for (int u = 0; u < GU; ++u) {
            const int j = jb + tid + NT * u;
            const uint32_t e = decltype(first)::value ? pf.ent[u] : ld_ro(P.nodes + (j < npn ? pn0 + j : 0));
            ent[u] = j < npn ? e : 0u;
        }
        S v[GU][3], w[GU][3];
        double xc[GU][3], a3[GU][3];
#pragma unroll
        for (int u = 0; u < GU; ++u) {
            const int j = jb + tid + NT * u;
            const int64_t g = (int64_t)(ent[u] & ~kOwnerBit);
            const int64_t gx = j < nv ? g : 0;
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                v[u][c] = ld_ro(in0 + 3 * g + c);
                if (MODE != MODE_APPLY) w[u][c] = ld_ro(in1 + 3 * g + c);
                if (MODE == MODE_RHS) a3[u][c] = ld_ro(A.in2 + 3 * g + c);
                xc[u][c] = ld_ro(P.coords + 3 * gx + c);
            }
        }
        if (decltype(first)::value) {
#pragma unroll
            for (int u = 0; u < GU; ++u) {
                const int j = tid + NT * u;
                sl0[u] = ld_ro(P.slot + (j < npn ? pn0 + j : 0));
            }
        }
        // Consume every loaded value (LDS writes) before the direction stores
        // are issued: the stores are conditional, and a load consumed after a
        // conditional store would make the compiler wait for that store too.
        S sp[GU][3];
#pragma unroll
        for (int u = 0; u < GU; ++u) {
            const int j = jb + tid + NT * u;
            const int64_t g = (int64_t)(ent[u] & ~kOwnerBit);
            T v0 = from_storage<T>(v[u][0]), v1 = from_storage<T>(v[u][1]), v2 = from_storage<T>(v[u][2]);
            if (MODE == MODE_APPLY) {
                if (A.mask_in) {
                    uint8_t fm = ld_ro(P.fixmask + g);
                    if (fm & 1) v0 = T(0);
                    if (fm & 2) v1 = T(0);
                    if (fm & 4) v2 = T(0);
                }
            } else if (MODE == MODE_PCG) {
                // p = z + beta p_prev; p_prev is not used on the first trip of a cycle (beta = 0)
                const T w0 = use_in1 ? from_storage<T>(w[u][0]) : T(0);
                const T w1 = use_in1 ? from_storage<T>(w[u][1]) : T(0);
                const T w2 = use_in1 ? from_storage<T>(w[u][2]) : T(0);
                v0 = fma(beta, w0, v0);
                v1 = fma(beta, w1, v1);
                v2 = fma(beta, w2, v2);
                // the matvec uses p as stored, so that q = A p holds for the stored p
                sp[u][0] = to_storage<S>(v0); sp[u][1] = to_storage<S>(v1); sp[u][2] = to_storage<S>(v2);
                v0 = from_storage<T>(sp[u][0]); v1 = from_storage<T>(sp[u][1]); v2 = from_storage<T>(sp[u][2]);
            } else if (j < npn) {  // RHS: v = u, w = v (velocity), a3 = a
                const T u0 = v0, u1 = v1, u2 = v2;
                const T w0 = from_storage<T>(w[u][0]), w1 = from_storage<T>(w[u][1]), w2 = from_storage<T>(w[u][2]);
                v0 = fma((T)A.c1, w0, (T)a3[u][0]) - (T)A.g0;
                v1 = fma((T)A.c1, w1, (T)a3[u][1]) - (T)A.g1;
                v2 = fma((T)A.c1, w2, (T)a3[u][2]) - (T)A.g2;
                lk[3 * j] = fma((T)A.c2, w0, -u0);
                lk[3 * j + 1] = fma((T)A.c2, w1, -u1);
                lk[3 * j + 2] = fma((T)A.c2, w2, -u2);
            }
            if (j < npn) {
                lm[3 * j] = v0; lm[3 * j + 1] = v1; lm[3 * j + 2] = v2;
#pragma unroll
                for (int q = 0; q < kEbeWaves; ++q) {
                    la[q * stride + 3 * j] = 0.0; la[q * stride + 3 * j + 1] = 0.0; la[q * stride + 3 * j + 2] = 0.0;
                }
            }
            if (j < nv) {
                lx[3 * j] = (T)xc[u][0]; lx[3 * j + 1] = (T)xc[u][1]; lx[3 * j + 2] = (T)xc[u][2];
            }
        }
        if (MODE == MODE_PCG) {
            S* pc = static_cast<S*>(A.p_cur);
#pragma unroll
            for (int u = 0; u < GU; ++u) {
                const int64_t g = (int64_t)(ent[u] & ~kOwnerBit);
                if (ent[u] & kOwnerBit) {   // entries past the patch's end are 0: no owner bit
                    pc[3 * g] = sp[u][0]; pc[3 * g + 1] = sp[u][1]; pc[3 * g + 2] = sp[u][2];
                }
            }
        }
    };
    // this thread's element record and material, in flight with the node values
    const ElemRec rec = ld_ro(P.elems + (tid < ne ? e0 + tid : 0));
    gather(Bool<true>{}, 0);
    for (int jb = NT * GU; jb < npn; jb += NT * GU) gather(Bool<false>{}, jb);
    // in flight during this patch's elements; issued unconditionally (the last
    // patch re-reads its own entries) so the compiler can count the loads in flight
    prefetch_gather(P, next >= 0 ? next : patch, pf);
    __syncthreads();

    double pap = 0.0;
    if (tid < ne) {
        double* acc = la + wave * stride;
        GeoT<T> G;
        tet_geo<T>(lx + 3 * rec.lid[0], lx + 3 * rec.lid[1], lx + 3 * rec.lid[2], lx + 3 * rec.lid[3], G);
        const double* mp = lmat + 3 * rec.mat;
        const T w = G.V * T(1.0 / 20.0) * (T)A.ck;
        const T lamV = (T)mp[0] * w, muV = (T)mp[1] * w;
        const T mc = (T)(A.cm * mp[2]) * G.V * T(1.0 / 420.0);
        T pm[10][3], pk[10][3];
#pragma unroll
        for (int i = 0; i < 10; ++i) {
            const int l = rec.lid[i];
#pragma unroll
            for (int c = 0; c < 3; ++c) pm[i][c] = lm[3 * l + c];
        }
        T papT = T(0);
        auto emit = [&](int i, T f0, T f1, T f2) {
            const int l = rec.lid[i];
            lds_add(acc + 3 * l, (double)f0);
            lds_add(acc + 3 * l + 1, (double)f1);
            lds_add(acc + 3 * l + 2, (double)f2);
            if (MODE == MODE_PCG) papT = fma(pm[i][0], f0, fma(pm[i][1], f1, fma(pm[i][2], f2, papT)));
        };
        if (MODE == MODE_RHS) {
#pragma unroll
            for (int i = 0; i < 10; ++i) {
                const int l = rec.lid[i];
#pragma unroll
                for (int c = 0; c < 3; ++c) pk[i][c] = lk[3 * l + c];
            }
            element_apply_emit<T>(pm, pk, G, lamV, muV, mc, emit);
        } else {
            element_apply_emit<T>(pm, pm, G, lamV, muV, mc, emit);
        }
        pap = (double)papT;
    }
    __syncthreads();

    // Write-out round: the kEbeWaves accumulators of each patch node, summed in
    // a fixed order, go to the node's slot for this patch.
    T* qb = static_cast<T*>(A.qbuf);
    auto write_out = [&](auto first, int jb) {
#pragma unroll
        for (int u = 0; u < GU; ++u) {
            const int j = jb + tid + NT * u;
            const int sl = decltype(first)::value ? sl0[u] : ld_ro(P.slot + (j < npn ? pn0 + j : 0));
            if (j >= npn) continue;
            double q0 = la[3 * j], q1 = la[3 * j + 1], q2 = la[3 * j + 2];
#pragma unroll
            for (int q = 1; q < kEbeWaves; ++q) {
                q0 += la[q * stride + 3 * j];
                q1 += la[q * stride + 3 * j + 1];
                q2 += la[q * stride + 3 * j + 2];
            }
            T* qo = qb + 3 * (int64_t)sl;
            qo[0] = (T)q0; qo[1] = (T)q1; qo[2] = (T)q2;
        }
    };
    write_out(Bool<true>{}, 0);
    for (int jb = NT * GU; jb < npn; jb += NT * GU) write_out(Bool<false>{}, jb);
    __syncthreads();   // LDS is reused by the next patch of a persistent workgroup
    return pap;
}

// Copies the material table into LDS after the patch regions (read by the
// element phase, which follows the first gather's barrier).
template <int MODE>
__device__ __forceinline__ void stage_materials(const DevPatches& P, double* lds) {
    const int stride = 3 * P.max_pn;
    double* lmat = lds + (size_t)stride * (kEbeWaves + (MODE == MODE_RHS ? 2 : 1)) + 3 * P.max_nv;
    stage_material_table(P, lmat, 64 * kEbeWaves);
}

// Apply / right-hand side: persistent grid as in the PCG matvec (each
// workgroup walks a contiguous per-XCD range of patches, node entries loaded
// one patch ahead).
template <int MODE>
__global__ __launch_bounds__(64 * kEbeWaves, 2) void k_ebe(EbeArgs A) {
    if (MODE == MODE_APPLY && A.guard && !check_due(A.guard)) return;
    if (MODE == MODE_APPLY && A.skip && A.skip->guard_skip) return;
    extern __shared__ double lds[];
    stage_materials<MODE>(A.P, lds);
    const int xcd = blockIdx.x & 7, k0 = blockIdx.x >> 3, per_xcd_wg = gridDim.x >> 3;   // grid: multiple of 8
    const int chunk = A.P.n_patches_pad >> 3;
    PatchPre pf;
    if (k0 < chunk) patch_prefetch(A.P, xcd * chunk + k0, pf);
    for (int k = k0; k < chunk; k += per_xcd_wg) {
        const int kn = k + per_xcd_wg;
        ebe_patch<MODE, double, double>(A, xcd * chunk + k, 0.0, lds, pf, kn < chunk ? xcd * chunk + kn : -1);
    }
}

// Persistent grid of the apply / right-hand-side passes: the workgroups that
// fit on the device at once (one or two per CU by LDS), a multiple of 8.
// CU count and LDS bytes per CU of the current device, queried once per process
// (a function-local static: initialised once, also under concurrent first calls).
static void device_limits(int& cus, int& lds_cu) {
    struct Limits {
        int cus = 256, lds = 160 * 1024;
    };
    static const Limits L = [] {
        Limits v;
        int dev = 0, c = 0, l = 0;
        if (hipGetDevice(&dev) == hipSuccess &&
            hipDeviceGetAttribute(&c, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess &&
            hipDeviceGetAttribute(&l, hipDeviceAttributeMaxSharedMemoryPerMultiprocessor, dev) == hipSuccess &&
            c > 0 && l > 0) {
            v.cus = c;
            v.lds = l;
        }
        return v;
    }();
    cus = L.cus;
    lds_cu = L.lds;
}

// The patch builder's LDS limit: the element pass of the PCG loop keeps two
// workgroups per CU (its static shared memory, 200 bytes, within the reserve).
constexpr int64_t kStaticLdsReserve = 256;
PatchLds ebe_patch_lds(int32_t n_mat) {
    int cus = 0, lds_cu = 0;
    device_limits(cus, lds_cu);
    DevPatches z{};
    z.n_mat = n_mat;
    PatchLds L;
    L.fixed = (int64_t)ebe_lds_bytes(z, MODE_PCG);
    z.max_pn = 1;
    L.per_node = (int64_t)ebe_lds_bytes(z, MODE_PCG) - L.fixed;
    z.max_pn = 0;
    z.max_nv = 1;
    L.per_vertex = (int64_t)ebe_lds_bytes(z, MODE_PCG) - L.fixed;
    L.budget = lds_cu / 2 - kStaticLdsReserve;
    return L;
}

int ebe_grid(const DevPatches& P, int mode) {
    int cus = 0, lds_cu = 0;
    device_limits(cus, lds_cu);
    const size_t need = ebe_lds_bytes(P, mode);
    int per_cu = need > 0 ? (int)(lds_cu / need) : 2;
    per_cu = per_cu < 1 ? 1 : (per_cu > 2 ? 2 : per_cu);
    int g = cus * per_cu / 8 * 8;
    if (g < 8) g = 8;
    return g < P.n_patches_pad ? g : P.n_patches_pad;
}

// FP64 sizing; it also covers the FP32 operands of the low-precision variants.
size_t ebe_lds_bytes(const DevPatches& P, int mode) {
    return sizeof(double) *
           (size_t)(3 * P.max_pn * ((mode == MODE_RHS ? 2 : 1) + kEbeWaves) + 3 * P.max_nv + 3 * P.n_mat);
}

// ---------------------------------------------------------------------------
// PCG iteration kernels (Algorithm 1)
// ---------------------------------------------------------------------------
// Grid-wide scalars without atomics or device-scope fences: each kernel writes
// one partial sum per workgroup with plain stores, and every workgroup of the
// next kernel sums all partials in the same fixed order (the kernel boundary
// makes them visible), so alpha, beta and the stop test are bitwise identical
// in every workgroup.  Workgroup 0 records the scalars for later kernels and
// the host.  Partial slots (kResArrays arrays of g_res values: (z,r), (r,r),
// (b,b), (z,r_prev)) are double-buffered by trip parity.

struct PcgEbeArgs {
    EbeArgs E;
    DevScalars* sc;
    const DevScalars* outer;  // inner solves: stop as soon as the outer solve has stopped
    const double* res_part;   // slot read by trip j
    int g_res;
    double* pap_part;         // [gridDim.x] (p, A p) partials written here
    int j;                    // trip index within the solve (0-based)
    int max_iter;
    double tol;
};


// Trip j of Algorithm 1, matvec part: stop test on the incoming residual,
// beta = rho_j / rho_{j-1} (0 on the first trip of a cycle; with FLEX the
// Polak-Ribiere form (rho_j - (z_j, r_{j-1})) / rho_{j-1} of flexible CG),
// p = z + beta p, q = A p (patch slots) and the partials of (p, A p).
// Persistent grid: each workgroup walks a contiguous (per XCD) range of patches.
template <class T, class S, bool FLEX>
__global__ __launch_bounds__(64 * kEbeWaves, 2) void k_ebe_pcg(PcgEbeArgs A) {
    DevScalars* sc = A.sc;
    if (sc->done) return;
    if (A.outer && A.outer->done) return;
    extern __shared__ double lds[];
    constexpr int NT = 64 * kEbeWaves;
    const int tid = threadIdx.x;
    const int j = A.j;
    const int g = A.g_res;
    // the four partial arrays of the slot exist whether used or not: all are
    // read together and the unused sums discarded
    double zr = lane_partials<kMaxResGrid / NT>(A.res_part, g, tid, NT);
    double rr = lane_partials<kMaxResGrid / NT>(A.res_part + g, g, tid, NT);
    double bb = lane_partials<kMaxResGrid / NT>(A.res_part + 2 * g, g, tid, NT);
    double zp = lane_partials<kMaxResGrid / NT>(A.res_part + 3 * g, g, tid, NT);
    block_bcast_sum4(zr, rr, bb, zp);
    if (j != 0) bb = 0.0;
    if (!FLEX || j == sc->cycle_start) zp = 0.0;
    const double bnorm = (j == 0) ? sqrt(bb) : sc->bnorm;
    const double res = bnorm > 0.0 ? sqrt(rr) / bnorm : 0.0;
    int stop = DONE_RUNNING;
    if (bnorm == 0.0) stop = DONE_ZERO_RHS;
    else if (!isfinite(res) || !isfinite(zr)) stop = DONE_NONFINITE;
    else if (res < A.tol) stop = DONE_CONVERGED;
    else if (j >= A.max_iter) stop = DONE_MAXITER;
    double beta = 0.0;
    if (stop == DONE_RUNNING && j != sc->cycle_start) {
        beta = (zr - zp) / sc->rho[(j - 1) & 1];
        if (!isfinite(beta)) stop = DONE_NONFINITE;
    }
    if (blockIdx.x == 0 && tid == 0) {
        if (j == 0) {
            sc->bnorm = bnorm;
            sc->res0 = res;
        }
        sc->rr = rr;
        if (stop != DONE_RUNNING) {
            sc->done = stop;
            sc->iters = j;
        } else {
            sc->rho[j & 1] = zr;
            sc->iters = j + 1;
        }
    }
    if (stop != DONE_RUNNING) return;

    const int nb = gridDim.x;              // multiple of 8
    const int xcd = blockIdx.x & 7, k0 = blockIdx.x >> 3, per_xcd_wg = nb >> 3;
    const int chunk = A.E.P.n_patches_pad >> 3;
    double pap = 0.0;
    stage_materials<MODE_PCG>(A.E.P, lds);
    PatchPre pf;
    if (k0 < chunk) patch_prefetch(A.E.P, xcd * chunk + k0, pf);
    for (int k = k0; k < chunk; k += per_xcd_wg) {
        const int kn = k + per_xcd_wg;
        pap += ebe_patch<MODE_PCG, T, S>(A.E, xcd * chunk + k, beta, lds, pf, kn < chunk ? xcd * chunk + kn : -1);
    }
    pap = block_bcast_sum(pap);
    if (tid == 0) A.pap_part[blockIdx.x] = pap;
}


bool ebe_set_lds_limit(const DevPatches& P) {
    const size_t need = ebe_lds_bytes(P, MODE_RHS);
    if (need <= 65536) return true;
    int dev = 0, maxlds = 0;
    if (hipGetDevice(&dev) != hipSuccess) return false;
    if (hipDeviceGetAttribute(&maxlds, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess) return false;
    if (need > (size_t)maxlds) return false;
    const int v = (int)need;
    const void* fns[] = {(const void*)k_ebe<MODE_APPLY>, (const void*)k_ebe<MODE_RHS>,
                         (const void*)k_ebe_pcg<double, double, false>, (const void*)k_ebe_pcg<double, double, true>,
                         (const void*)k_ebe_pcg<float, float, false>, (const void*)k_ebe_pcg<float, bf16_t, false>};
    for (const void* f : fns)
        if (hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, v) != hipSuccess) return false;
    return true;
}

void launch_ebe_apply(hipStream_t s, const DevPatches& P, const double* p, bool mask_in, double cm, double ck,
                      double* qbuf, const DevScalars* guard, const DevScalars* skip) {
    EbeArgs A{};
    A.P = P; A.in0 = p; A.qbuf = qbuf; A.cm = cm; A.ck = ck; A.mask_in = mask_in ? 1 : 0;
    A.guard = guard;
    A.skip = skip;
    hipLaunchKernelGGL(k_ebe<MODE_APPLY>, dim3(ebe_grid(P, MODE_APPLY)), dim3(64 * kEbeWaves),
                       ebe_lds_bytes(P, MODE_APPLY), s, A);
}

int pcg_ebe_grid(const DevPatches& P) {
    // the resident workgroups (ebe_grid), at most kMaxPcgGrid; all multiples of 8
    const int g = ebe_grid(P, MODE_PCG);
    return g < kMaxPcgGrid ? g : kMaxPcgGrid;
}

void launch_ebe_pcg(hipStream_t s, const PcgLaunch& L) {
    PcgEbeArgs A{};
    A.E.P = *L.P; A.E.in0 = L.z; A.E.in1 = L.p_prev; A.E.p_cur = L.p_cur; A.E.qbuf = L.qbuf;
    A.E.cm = L.cm; A.E.ck = L.ck;
    A.sc = L.sc; A.outer = L.outer; A.res_part = L.res_part; A.g_res = L.g_res; A.pap_part = L.pap_part;
    A.j = L.j; A.max_iter = L.max_iter; A.tol = L.tol;
    const size_t lds = ebe_lds_bytes(*L.P, MODE_PCG);   // FP64 sizing also covers FP32 operands
    const dim3 grid(pcg_ebe_grid(*L.P)), block(64 * kEbeWaves);
    switch (L.prec) {
        case PREC_FP64:
            if (L.flexible) hipLaunchKernelGGL((k_ebe_pcg<double, double, true>), grid, block, lds, s, A);
            else hipLaunchKernelGGL((k_ebe_pcg<double, double, false>), grid, block, lds, s, A);
            break;
        case PREC_FP32: hipLaunchKernelGGL((k_ebe_pcg<float, float, false>), grid, block, lds, s, A); break;
        default: hipLaunchKernelGGL((k_ebe_pcg<float, bf16_t, false>), grid, block, lds, s, A); break;
    }
}

void launch_ebe_rhs(hipStream_t s, const DevPatches& P, const double* u, const double* v, const double* a,
                    double c1, double c2, double g0, double g1, double g2, double* qbuf) {
    EbeArgs A{};
    A.P = P; A.in0 = u; A.in1 = v; A.in2 = a; A.qbuf = qbuf; A.cm = 1.0; A.ck = 1.0;
    A.c1 = c1; A.c2 = c2; A.g0 = g0; A.g1 = g1; A.g2 = g2;
    hipLaunchKernelGGL(k_ebe<MODE_RHS>, dim3(ebe_grid(P, MODE_RHS)), dim3(64 * kEbeWaves), ebe_lds_bytes(P, MODE_RHS), s,
                       A);
}

// ---------------------------------------------------------------------------
// block diagonal of cm M + ck K (setup)
// ---------------------------------------------------------------------------
// Node-diagonal 3x3 blocks: int gradN_i (x) gradN_i is
//   vertex i:    (3/5) V g_i g_i^T            (gradN_i = (4 L_i - 1) g_i)
//   edge (i,j):  (8/5) V (g_i g_i^T + g_j g_j^T) + (4/5) V (g_i g_j^T + g_j g_i^T)
// K_ii = (lam + mu) G + mu tr(G) I; M_ii = rho V {6, 32}/420.
__global__ __launch_bounds__(64) void k_ebe_diag(DevPatches P, double cm, double ck, double* qbuf6) {
    extern __shared__ double lds[];
    const int lane = threadIdx.x;
    const int patch = xcd_remap(blockIdx.x, gridDim.x);
    const int pn0 = P.pn_ptr[patch], npn = P.pn_ptr[patch + 1] - pn0;
    const int nv = P.nv[patch];
    const int e0 = P.el_ptr[patch], ne = P.el_ptr[patch + 1] - e0;
    double* la = lds;                 // [max_pn][6]
    double* lx = la + 6 * P.max_pn;   // [max_nv][3]
    for (int j = lane; j < npn; j += 64) {
        int g = (int)(P.nodes[pn0 + j] & ~kOwnerBit);
        for (int t = 0; t < 6; ++t) la[6 * j + t] = 0.0;
        if (j < nv)
            for (int d = 0; d < 3; ++d) lx[3 * j + d] = P.coords[3 * (int64_t)g + d];
    }
    __syncthreads();
    for (int e = lane; e < ne; e += 64) {
        const ElemRec rec = P.elems[e0 + e];
        Geo Gm;
        tet_geo(lx + 3 * rec.lid[0], lx + 3 * rec.lid[1], lx + 3 * rec.lid[2], lx + 3 * rec.lid[3], Gm);
        const double* mp = P.mat + 3 * rec.mat;
        double lam = ck * mp[0], mu = ck * mp[1], rho = cm * mp[2];
        double V = Gm.V;
        constexpr int EV[6][2] = {{0, 1}, {1, 2}, {0, 2}, {0, 3}, {1, 3}, {2, 3}};
        for (int i = 0; i < 10; ++i) {
            double G[3][3];
            double mdiag;
            if (i < 4) {
                const double* g = Gm.g[i];
                for (int a = 0; a < 3; ++a)
                    for (int b = 0; b < 3; ++b) G[a][b] = 0.6 * V * g[a] * g[b];
                mdiag = rho * V * (6.0 / 420.0);
            } else {
                const double* gi = Gm.g[EV[i - 4][0]];
                const double* gj = Gm.g[EV[i - 4][1]];
                for (int a = 0; a < 3; ++a)
                    for (int b = 0; b < 3; ++b)
                        G[a][b] = 1.6 * V * (gi[a] * gi[b] + gj[a] * gj[b]) + 0.8 * V * (gi[a] * gj[b] + gj[a] * gi[b]);
                mdiag = rho * V * (32.0 / 420.0);
            }
            double tr = G[0][0] + G[1][1] + G[2][2];
            double lm = lam + mu;
            double* acc = la + 6 * rec.lid[i];
            lds_add(acc + 0, lm * G[0][0] + mu * tr + mdiag);
            lds_add(acc + 1, lm * G[1][1] + mu * tr + mdiag);
            lds_add(acc + 2, lm * G[2][2] + mu * tr + mdiag);
            lds_add(acc + 3, lm * G[0][1]);
            lds_add(acc + 4, lm * G[0][2]);
            lds_add(acc + 5, lm * G[1][2]);
        }
    }
    __syncthreads();
    for (int j = lane; j < npn; j += 64)
        for (int t = 0; t < 6; ++t) qbuf6[6 * (int64_t)P.slot[pn0 + j] + t] = la[6 * j + t];
}

void launch_ebe_diag(hipStream_t s, const DevPatches& P, double cm, double ck, double* qbuf6) {
    size_t lds = sizeof(double) * (size_t)(6 * P.max_pn + 3 * P.max_nv);
    hipLaunchKernelGGL(k_ebe_diag, dim3(P.n_patches_pad), dim3(64), lds, s, P, cm, ck, qbuf6);
}

// ---------------------------------------------------------------------------
// node-wise kernels
// ---------------------------------------------------------------------------
template <class T>
__device__ __forceinline__ void gather_q(const DevNodes& N, const T* qbuf, int64_t n, T& q0, T& q1, T& q2) {
    const int k0 = N.slot_ptr[n], k1 = N.slot_ptr[n + 1];
    T q[3];
    sum_slots(qbuf, k0, k1 - k0, q);
    q0 = q[0]; q1 = q[1]; q2 = q[2];
}

// mode 0: q = sum (no constraint handling); mode 1: A_bc (free rows: sum, fixed: identity p)
__global__ void k_combine_apply(DevNodes N, const double* qbuf, const double* p, int mode, double* q) {
    int64_t n = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (n >= N.n) return;
    double q0, q1, q2;
    gather_q(N, qbuf, n, q0, q1, q2);
    if (mode == 1) {
        uint8_t fm = N.fixmask[n];
        if (fm & 1) q0 = p[3 * n];
        if (fm & 2) q1 = p[3 * n + 1];
        if (fm & 4) q2 = p[3 * n + 2];
    }
    q[3 * n] = q0; q[3 * n + 1] = q1; q[3 * n + 2] = q2;
}

void launch_combine_apply(hipStream_t s, const DevNodes& N, const double* qbuf, const double* p, int mode, double* q) {
    int nb = (int)((N.n + 255) / 256);
    hipLaunchKernelGGL(k_combine_apply, dim3(nb), dim3(256), 0, s, N, qbuf, p, mode, q);
}

// symmetric 3x3 inverse of the constrained block Z B Z + (I - Z), then fixed
// rows/columns zeroed: z = binv r is zero on fixed dofs.
__global__ void k_diag_finalize(DevNodes N, const double* qbuf6, double* binv6) {
    int64_t n = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (n >= N.n) return;
    double b[6] = {0, 0, 0, 0, 0, 0};
    for (int k = N.slot_ptr[n]; k < N.slot_ptr[n + 1]; ++k)
        for (int t = 0; t < 6; ++t) b[t] += qbuf6[6 * (int64_t)k + t];
    uint8_t fm = N.fixmask[n];
    bool f0 = fm & 1, f1 = fm & 2, f2 = fm & 4;
    double xx = f0 ? 1.0 : b[0], yy = f1 ? 1.0 : b[1], zz = f2 ? 1.0 : b[2];
    double xy = (f0 || f1) ? 0.0 : b[3], xz = (f0 || f2) ? 0.0 : b[4], yz = (f1 || f2) ? 0.0 : b[5];
    double c00 = yy * zz - yz * yz, c01 = xz * yz - xy * zz, c02 = xy * yz - xz * yy;
    double c11 = xx * zz - xz * xz, c12 = xy * xz - xx * yz, c22 = xx * yy - xy * xy;
    double det = xx * c00 + xy * c01 + xz * c02;
    double id = 1.0 / det;
    double r[6] = {c00 * id, c11 * id, c22 * id, c01 * id, c02 * id, c12 * id};
    if (f0) { r[0] = 0; r[3] = 0; r[4] = 0; }
    if (f1) { r[1] = 0; r[3] = 0; r[5] = 0; }
    if (f2) { r[2] = 0; r[4] = 0; r[5] = 0; }
    for (int t = 0; t < 6; ++t) binv6[6 * n + t] = r[t];
}

void launch_diag_finalize(hipStream_t s, const DevNodes& N, const double* qbuf6, double* binv6) {
    int nb = (int)((N.n + 255) / 256);
    hipLaunchKernelGGL(k_diag_finalize, dim3(nb), dim3(256), 0, s, N, qbuf6, binv6);
}


// z = B^{-1} r for the constrained operator: identity on fixed dofs
__global__ void k_precond(DevNodes N, const double* binv6, const double* r, double* z) {
    int64_t n = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (n >= N.n) return;
    double z0, z1, z2;
    apply_binv(binv6 + 6 * n, r[3 * n], r[3 * n + 1], r[3 * n + 2], z0, z1, z2);
    uint8_t fm = N.fixmask[n];
    if (fm & 1) z0 = r[3 * n];
    if (fm & 2) z1 = r[3 * n + 1];
    if (fm & 4) z2 = r[3 * n + 2];
    z[3 * n] = z0; z[3 * n + 1] = z1; z[3 * n + 2] = z2;
}

void launch_precond(hipStream_t s, const DevNodes& N, const double* binv6, const double* r, double* z) {
    int nb = (int)((N.n + 255) / 256);
    hipLaunchKernelGGL(k_precond, dim3(nb), dim3(256), 0, s, N, binv6, r, z);
}

// b = (sum of patch slots) + f_ext on free dofs, 0 on fixed dofs
__global__ void k_rhs_finalize(DevNodes N, const double* qbuf, const double* f_ext, double* b) {
    int64_t n = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (n >= N.n) return;
    double q0, q1, q2;
    gather_q(N, qbuf, n, q0, q1, q2);
    if (f_ext) { q0 += f_ext[3 * n]; q1 += f_ext[3 * n + 1]; q2 += f_ext[3 * n + 2]; }
    uint8_t fm = N.fixmask[n];
    b[3 * n] = (fm & 1) ? 0.0 : q0;
    b[3 * n + 1] = (fm & 2) ? 0.0 : q1;
    b[3 * n + 2] = (fm & 4) ? 0.0 : q2;
}

void launch_rhs_finalize(hipStream_t s, const DevNodes& N, const double* qbuf, const double* f_ext, double* b) {
    int nb = (int)((N.n + 255) / 256);
    hipLaunchKernelGGL(k_rhs_finalize, dim3(nb), dim3(256), 0, s, N, qbuf, f_ext, b);
}

int res_grid(int64_t n) {
    int64_t g = (n + 255) / 256;
    return (int)(g < kMaxResGrid ? g : kMaxResGrid);
}

// r = b - A x (from the slots), z = B^{-1} r; partials of (z,r), (r,r), (b,b)
// into res_part[3][gridDim.x].  mode 0 (start of a solve): also x = b on fixed
// dofs and resets the solve scalars.  mode 1 (true-residual check): runs only
// when the check is due, the scalars are finished by k_check_finalize.
__global__ __launch_bounds__(256) void k_residual(DevNodes N, const double* qbuf, const double* b, const double* binv6,
                                                  double* x, double* r, double* z, DevScalars* sc,
                                                  double* res_part, int mode) {
    if (mode == 1 && !check_due(sc)) return;
    if (mode == 0 && blockIdx.x == 0 && threadIdx.x == 0) {
        sc->done = DONE_RUNNING;
        sc->iters = 0;
        sc->restarts = 0;
        sc->checked = 0;
        sc->cycle_start = 0;
        sc->inner_iters = 0;
        sc->res_true = 0.0;
        sc->x_base = 0;
    }
    double v0 = 0.0, v1 = 0.0, v2 = 0.0;
    // every load of a node before its first store
    for (int64_t n = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; n < N.n; n += (int64_t)gridDim.x * blockDim.x) {
        const int k0 = N.slot_ptr[n], k1 = N.slot_ptr[n + 1];
        const uint8_t fm = N.fixmask[n];
        const double b0 = b[3 * n], b1 = b[3 * n + 1], b2 = b[3 * n + 2];
        double B[6], q[3];
#pragma unroll
        for (int t = 0; t < 6; ++t) B[t] = binv6[6 * n + t];
        sum_slots(qbuf, k0, k1 - k0, q);
        if (mode == 0 && fm) {  // fixed rows of A_bc are identity: x = b there, exactly
            if (fm & 1) x[3 * n] = b0;
            if (fm & 2) x[3 * n + 1] = b1;
            if (fm & 4) x[3 * n + 2] = b2;
        }
        const double r0 = (fm & 1) ? 0.0 : b0 - q[0];
        const double r1 = (fm & 2) ? 0.0 : b1 - q[1];
        const double r2 = (fm & 4) ? 0.0 : b2 - q[2];
        double z0, z1, z2;
        apply_binv(B, r0, r1, r2, z0, z1, z2);
        r[3 * n] = r0; r[3 * n + 1] = r1; r[3 * n + 2] = r2;
        z[3 * n] = z0; z[3 * n + 1] = z1; z[3 * n + 2] = z2;
        v0 += z0 * r0 + z1 * r1 + z2 * r2;
        v1 += r0 * r0 + r1 * r1 + r2 * r2;
        v2 += b0 * b0 + b1 * b1 + b2 * b2;
    }
    v0 = block_bcast_sum(v0);
    v1 = block_bcast_sum(v1);
    v2 = block_bcast_sum(v2);
    if (threadIdx.x == 0) {
        res_part[blockIdx.x] = v0;
        res_part[gridDim.x + blockIdx.x] = v1;
        res_part[2 * gridDim.x + blockIdx.x] = v2;
    }
}

void launch_residual(hipStream_t s, const DevNodes& N, const double* qbuf, const double* b, const double* binv6,
                     double* x, double* r, double* z, DevScalars* sc, double* res_part, int mode) {
    hipLaunchKernelGGL(k_residual, dim3(res_grid(N.n)), dim3(256), 0, s, N, qbuf, b, binv6, x, r, z, sc, res_part,
                       mode);
}

// Finish the true-residual check (one workgroup): relative true residual; if
// it is not below tol after the recursive residual converged, restart the CG
// cycle from the true residual at trip j_next (beta = 0 there).
__global__ __launch_bounds__(256) void k_check_finalize(DevScalars* sc, const double* res_part, int g, int j_next,
                                                        double tol) {
    if (!check_due(sc)) return;
    double rr = lane_partials<kMaxResGrid / 256>(res_part + g, g, threadIdx.x, 256);
    rr = block_bcast_sum(rr);
    if (threadIdx.x == 0) {
        double res = sqrt(rr) / sc->bnorm;
        sc->res_true = res;
        sc->checked = 1;
        if (!isfinite(res)) {
            sc->done = DONE_NONFINITE;
        } else if (res >= tol && sc->done == DONE_CONVERGED) {
            sc->done = DONE_RUNNING;
            sc->checked = 0;
            sc->restarts += 1;
            sc->cycle_start = j_next;
            sc->x_base = j_next;   // the flush completed x: the next trip starts a new pair
        }
    }
}

void launch_check_finalize(hipStream_t s, DevScalars* sc, const double* res_part, int g, int j_next, double tol) {
    hipLaunchKernelGGL(k_check_finalize, dim3(1), dim3(256), 0, s, sc, res_part, g, j_next, tol);
}

// The node loop of the update for one x mode (XM 0: x untouched, the first
// trip of a pair; 1: x += alpha p; 2: x += alpha p + alpha_prev p_other).
// The mode is fixed per launch, so the loop has no branch around its loads:
// every load of a node is issued before the first is consumed.
template <class T, class S, int XM>
__device__ __forceinline__ void pcg_update_nodes(const DevNodes& N, const T* qbuf, const S* p, const T* binv6, T* x,
                                                 T* r, S* z, const S* p_other, T alpha, T alpha_prev, double& v0,
                                                 double& v1) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t n = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; n < N.n; n += stride) {
        const int k0 = N.slot_ptr[n], k1 = N.slot_ptr[n + 1];
        const uint8_t fm = N.fixmask[n];
        T rv[3], xv[3], pv[3], po[3], B[6];
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            rv[c] = r[3 * n + c];
            if (XM != 0) {
                xv[c] = x[3 * n + c];
                pv[c] = from_storage<T>(p[3 * n + c]);
            }
            if (XM == 2) po[c] = from_storage<T>(p_other[3 * n + c]);
        }
#pragma unroll
        for (int t = 0; t < 6; ++t) B[t] = binv6[6 * n + t];
        T q[3];
        sum_slots(qbuf, k0, k1 - k0, q);
        if (fm & 1) q[0] = T(0);
        if (fm & 2) q[1] = T(0);
        if (fm & 4) q[2] = T(0);
        const T r0 = fma(-alpha, q[0], rv[0]);
        const T r1 = fma(-alpha, q[1], rv[1]);
        const T r2 = fma(-alpha, q[2], rv[2]);
        if (XM == 2) {
            x[3 * n] = fma(alpha, pv[0], fma(alpha_prev, po[0], xv[0]));
            x[3 * n + 1] = fma(alpha, pv[1], fma(alpha_prev, po[1], xv[1]));
            x[3 * n + 2] = fma(alpha, pv[2], fma(alpha_prev, po[2], xv[2]));
        } else if (XM == 1) {
            x[3 * n] = fma(alpha, pv[0], xv[0]);
            x[3 * n + 1] = fma(alpha, pv[1], xv[1]);
            x[3 * n + 2] = fma(alpha, pv[2], xv[2]);
        }
        T z0, z1, z2;
        apply_binv(B, r0, r1, r2, z0, z1, z2);
        r[3 * n] = r0; r[3 * n + 1] = r1; r[3 * n + 2] = r2;
        const S zs0 = to_storage<S>(z0), zs1 = to_storage<S>(z1), zs2 = to_storage<S>(z2);
        z[3 * n] = zs0; z[3 * n + 1] = zs1; z[3 * n + 2] = zs2;
        // dots in FP64 with the stored z (what the next matvec reads)
        v0 += (double)from_storage<T>(zs0) * r0 + (double)from_storage<T>(zs1) * r1 + (double)from_storage<T>(zs2) * r2;
        v1 += (double)r0 * r0 + (double)r1 * r1 + (double)r2 * r2;
    }
}

// Trip j, update part: alpha = rho_j / (p, A p) from the matvec partials,
// r -= alpha q, x += alpha p, z = B^{-1} r, and partials of (z, r), (r, r)
// for trip j + 1.  Compute type T, storage type S of p and z.  Persistent
// grid-stride over nodes, one node per thread per round.
template <class T, class S>
__global__ __launch_bounds__(256) void k_pcg_update(DevNodes N, const T* qbuf, const S* p, const T* binv6, T* x, T* r,
                                                    S* z, DevScalars* sc, const DevScalars* outer,
                                                    const double* pap_part, int g_pap, double* res_part, int j,
                                                    int32_t* inner_count, const S* p_other) {
    if (sc->done) return;
    if (outer && outer->done) return;
    double pap = lane_partials<kMaxPcgGrid / 256>(pap_part, g_pap, threadIdx.x, 256);
    pap = block_bcast_sum(pap);
    const double alpha_d = sc->rho[j & 1] / pap;
    if (!isfinite(alpha_d)) {
        if (blockIdx.x == 0 && threadIdx.x == 0) sc->done = DONE_NONFINITE;
        return;
    }
    if (inner_count && blockIdx.x == 0 && threadIdx.x == 0) *inner_count += 1;
    const T alpha = (T)alpha_d;
    // paired x update: the first trip of a pair only records its alpha, the second
    // applies both (x_base is written only between solves and by the restart)
    const bool defer = p_other && ((j - sc->x_base) & 1) == 0;
    const bool pair = p_other && !defer;
    const T alpha_prev = pair ? (T)sc->x_alpha : T(0);
    if (defer && blockIdx.x == 0 && threadIdx.x == 0) sc->x_alpha = alpha_d;
    double v0 = 0.0, v1 = 0.0;
    if (defer) pcg_update_nodes<T, S, 0>(N, qbuf, p, binv6, x, r, z, p_other, alpha, alpha_prev, v0, v1);
    else if (pair) pcg_update_nodes<T, S, 2>(N, qbuf, p, binv6, x, r, z, p_other, alpha, alpha_prev, v0, v1);
    else pcg_update_nodes<T, S, 1>(N, qbuf, p, binv6, x, r, z, p_other, alpha, alpha_prev, v0, v1);
    v0 = block_bcast_sum(v0);
    v1 = block_bcast_sum(v1);
    if (threadIdx.x == 0) {
        res_part[blockIdx.x] = v0;
        res_part[gridDim.x + blockIdx.x] = v1;
    }
}

void launch_pcg_update(hipStream_t s, const UpdLaunch& L) {
    const dim3 grid(res_grid(L.N->n)), block(256);
    switch (L.prec) {
        case PREC_FP64:
            hipLaunchKernelGGL((k_pcg_update<double, double>), grid, block, 0, s, *L.N, (const double*)L.qbuf,
                               (const double*)L.p, (const double*)L.binv, (double*)L.x, (double*)L.r, (double*)L.z,
                               L.sc, L.outer, L.pap_part, L.g_pap, L.res_part, L.j, L.inner_count,
                               (const double*)L.p_other);
            break;
        case PREC_FP32:
            hipLaunchKernelGGL((k_pcg_update<float, float>), grid, block, 0, s, *L.N, (const float*)L.qbuf,
                               (const float*)L.p, (const float*)L.binv, (float*)L.x, (float*)L.r, (float*)L.z, L.sc,
                               L.outer, L.pap_part, L.g_pap, L.res_part, L.j, L.inner_count, (const float*)nullptr);
            break;
        default:
            hipLaunchKernelGGL((k_pcg_update<float, bf16_t>), grid, block, 0, s, *L.N, (const float*)L.qbuf,
                               (const bf16_t*)L.p, (const float*)L.binv, (float*)L.x, (float*)L.r, (bf16_t*)L.z,
                               L.sc, L.outer, L.pap_part, L.g_pap, L.res_part, L.j, L.inner_count,
                               (const bf16_t*)nullptr);
            break;
    }
}

// The pending half of a paired x update at the stop: the last trip j = iters - 1
// deferred its alpha p when (j - x_base) is even.
__global__ void k_flush_x(DevNodes N, double* x, const double* p0, const double* p1, int par0, DevScalars* sc) {
    if (!check_due(sc)) return;
    const int j = sc->iters - 1;
    if (j < sc->x_base || ((j - sc->x_base) & 1) != 0) return;
    const double* p = ((par0 + j + 1) & 1) ? p1 : p0;
    const double alpha = sc->x_alpha;
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < 3 * N.n) x[i] = fma(alpha, p[i], x[i]);
}

void launch_flush_x(hipStream_t s, const DevNodes& N, double* x, const double* p0, const double* p1, int par0,
                    DevScalars* sc) {
    hipLaunchKernelGGL(k_flush_x, dim3((unsigned)((3 * N.n + 255) / 256)), dim3(256), 0, s, N, x, p0, p1, par0, sc);
}

// ---------------------------------------------------------------------------
// Mixed precision: flexible FP64 outer PCG, inner FP32 / BF16-stored PCG
// ---------------------------------------------------------------------------
// Start of the inner solve for outer trip j: outer stop test on the outer
// residual partials of slot j (the remaining kernels of the trip return at
// once when it fires), then r_in = float(r), e = 0, z = B^{-1} r_in and the
// inner partials (z,r), (r,r), (r,r) into the inner slot 0.  Resets the inner
// scalars.
template <class T, class S>
__global__ __launch_bounds__(256) void k_inner_init(DevNodes N, const double* r64, const T* binv6, T* r, T* e, S* z,
                                                    DevScalars* outer, const double* outer_part, int g_out, int j,
                                                    int max_iter, double tol, DevScalars* sc_in, double* in_part) {
    if (outer->done) return;
    const int g = g_out;
    double rr = lane_partials<kMaxResGrid / 256>(outer_part + g, g, threadIdx.x, 256);
    double bb = j == 0 ? lane_partials<kMaxResGrid / 256>(outer_part + 2 * g, g, threadIdx.x, 256) : 0.0;
    rr = block_bcast_sum(rr);
    bb = block_bcast_sum(bb);
    const double bnorm = (j == 0) ? sqrt(bb) : outer->bnorm;
    const double res = bnorm > 0.0 ? sqrt(rr) / bnorm : 0.0;
    int stop = DONE_RUNNING;
    if (bnorm == 0.0) stop = DONE_ZERO_RHS;
    else if (!isfinite(res)) stop = DONE_NONFINITE;
    else if (res < tol) stop = DONE_CONVERGED;
    else if (j >= max_iter) stop = DONE_MAXITER;
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        if (stop != DONE_RUNNING) {
            outer->done = stop;
            outer->iters = j;
            outer->rr = rr;
            if (j == 0) {
                outer->bnorm = bnorm;
                outer->res0 = res;
            }
        }
        sc_in->done = DONE_RUNNING;
        sc_in->cycle_start = 0;
        sc_in->checked = 0;
    }
    if (stop != DONE_RUNNING) return;
    double v0 = 0.0, v1 = 0.0;
    for (int64_t n = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; n < N.n; n += (int64_t)gridDim.x * blockDim.x) {
        // every load unconditional and before the first store
        const uint8_t fm = N.fixmask[n];
        const double a0 = r64[3 * n], a1 = r64[3 * n + 1], a2 = r64[3 * n + 2];
        T B[6];
#pragma unroll
        for (int t = 0; t < 6; ++t) B[t] = binv6[6 * n + t];
        const T r0 = (fm & 1) ? T(0) : (T)a0;
        const T r1 = (fm & 2) ? T(0) : (T)a1;
        const T r2 = (fm & 4) ? T(0) : (T)a2;
        T z0, z1, z2;
        apply_binv(B, r0, r1, r2, z0, z1, z2);
        r[3 * n] = r0; r[3 * n + 1] = r1; r[3 * n + 2] = r2;
        e[3 * n] = T(0); e[3 * n + 1] = T(0); e[3 * n + 2] = T(0);
        const S zs0 = to_storage<S>(z0), zs1 = to_storage<S>(z1), zs2 = to_storage<S>(z2);
        z[3 * n] = zs0; z[3 * n + 1] = zs1; z[3 * n + 2] = zs2;
        v0 += (double)from_storage<T>(zs0) * r0 + (double)from_storage<T>(zs1) * r1 + (double)from_storage<T>(zs2) * r2;
        v1 += (double)r0 * r0 + (double)r1 * r1 + (double)r2 * r2;
    }
    v0 = block_bcast_sum(v0);
    v1 = block_bcast_sum(v1);
    if (threadIdx.x == 0) {
        in_part[blockIdx.x] = v0;
        in_part[gridDim.x + blockIdx.x] = v1;
        in_part[2 * gridDim.x + blockIdx.x] = v1;   // the inner right-hand side is r itself
    }
}

// Outer trip j, preconditioned residual: z = e (the inner solution, in FP64)
// and the partials (z, r), (r, r), (z, r_prev) of slot j for the flexible
// matvec kernel.
template <class T>
__global__ __launch_bounds__(256) void k_outer_z(DevNodes N, const T* e, const double* r, const double* r_prev,
                                                 double* z, const DevScalars* outer, double* part, int j) {
    if (outer->done) return;
    const bool prev = j != outer->cycle_start;
    double v0 = 0.0, v1 = 0.0, v3 = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < 3 * N.n; i += (int64_t)gridDim.x * blockDim.x) {
        const double zi = (double)e[i];
        const double ri = r[i];
        z[i] = zi;
        v0 += zi * ri;
        v1 += ri * ri;
        if (prev) v3 += zi * r_prev[i];
    }
    v0 = block_bcast_sum(v0);
    v1 = block_bcast_sum(v1);
    v3 = block_bcast_sum(v3);
    if (threadIdx.x == 0) {
        part[blockIdx.x] = v0;
        part[gridDim.x + blockIdx.x] = v1;
        part[3 * gridDim.x + blockIdx.x] = v3;
    }
}

// Outer trip j, update: alpha = rho_j / (p, A p); r_prev = r; r -= alpha q
// (fixed rows masked); x += alpha p; partials (r, r) into slot j + 1.
__global__ __launch_bounds__(256) void k_outer_update(DevNodes N, const double* qbuf, const double* p, double* x,
                                                      double* r, double* r_prev, DevScalars* sc,
                                                      const double* pap_part, int g_pap, double* part, int j) {
    if (sc->done) return;
    double pap = lane_partials<kMaxPcgGrid / 256>(pap_part, g_pap, threadIdx.x, 256);
    pap = block_bcast_sum(pap);
    const double alpha = sc->rho[j & 1] / pap;
    if (!isfinite(alpha)) {
        if (blockIdx.x == 0 && threadIdx.x == 0) sc->done = DONE_NONFINITE;
        return;
    }
    double v1 = 0.0;
    // every load of a node before its first store (the stores could alias the
    // later loads as far as the compiler knows)
    for (int64_t n = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; n < N.n; n += (int64_t)gridDim.x * blockDim.x) {
        const int k0 = N.slot_ptr[n], k1 = N.slot_ptr[n + 1];
        const uint8_t fm = N.fixmask[n];
        double ro[3], xv[3], pv[3], qq[3];
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            ro[c] = r[3 * n + c];
            xv[c] = x[3 * n + c];
            pv[c] = p[3 * n + c];
        }
        sum_slots(qbuf, k0, k1 - k0, qq);
        if (fm & 1) qq[0] = 0.0;
        if (fm & 2) qq[1] = 0.0;
        if (fm & 4) qq[2] = 0.0;
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            const double rn = fma(-alpha, qq[c], ro[c]);
            r_prev[3 * n + c] = ro[c];
            r[3 * n + c] = rn;
            x[3 * n + c] = fma(alpha, pv[c], xv[c]);
            v1 += rn * rn;
        }
    }
    v1 = block_bcast_sum(v1);
    if (threadIdx.x == 0) part[gridDim.x + blockIdx.x] = v1;
}

__global__ void k_to_f32(int64_t n, const double* in, float* out) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) out[i] = (float)in[i];
}

void launch_inner_init(hipStream_t s, int prec, const DevNodes& N, const double* r64, const void* binv, void* r,
                       void* e, void* z, DevScalars* outer, const double* outer_part, int j, int max_iter, double tol,
                       DevScalars* sc_in, double* in_part) {
    const int g = res_grid(N.n);
    if (prec == PREC_FP32)
        hipLaunchKernelGGL((k_inner_init<float, float>), dim3(g), dim3(256), 0, s, N, r64, (const float*)binv,
                           (float*)r, (float*)e, (float*)z, outer, outer_part, g, j, max_iter, tol, sc_in, in_part);
    else
        hipLaunchKernelGGL((k_inner_init<float, bf16_t>), dim3(g), dim3(256), 0, s, N, r64, (const float*)binv,
                           (float*)r, (float*)e, (bf16_t*)z, outer, outer_part, g, j, max_iter, tol, sc_in, in_part);
}

void launch_outer_z(hipStream_t s, const DevNodes& N, const void* e, const double* r, const double* r_prev, double* z,
                    const DevScalars* outer, double* part, int j) {
    hipLaunchKernelGGL((k_outer_z<float>), dim3(res_grid(N.n)), dim3(256), 0, s, N, (const float*)e, r, r_prev, z,
                       outer, part, j);
}

void launch_outer_update(hipStream_t s, const DevNodes& N, const double* qbuf, const double* p, double* x, double* r,
                         double* r_prev, DevScalars* sc, const double* pap_part, int g_pap, double* part, int j) {
    hipLaunchKernelGGL(k_outer_update, dim3(res_grid(N.n)), dim3(256), 0, s, N, qbuf, p, x, r, r_prev, sc, pap_part,
                       g_pap, part, j);
}

void launch_to_f32(hipStream_t s, int64_t n, const double* in, float* out) {
    hipLaunchKernelGGL(k_to_f32, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, n, in, out);
}

// ---------------------------------------------------------------------------
// learned-predictor support: M row sums, candidate residuals and selection
// ---------------------------------------------------------------------------
__global__ void k_msum(DevNodes N, const double* qbuf, double* msum) {
    const int64_t n = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (n >= N.n) return;
    double q0, q1, q2;
    gather_q(N, qbuf, n, q0, q1, q2);
    msum[n] = q0;
}

void launch_msum(hipStream_t s, const DevNodes& N, const double* qbuf, double* msum) {
    hipLaunchKernelGGL(k_msum, dim3((unsigned)((N.n + 255) / 256)), dim3(256), 0, s, N, qbuf, msum);
}

__global__ __launch_bounds__(256) void k_cand_res(DevNodes N, const double* qbuf, const double* b, double* part,
                                                  const DevScalars* skip) {
    if (skip && skip->guard_skip) return;
    double v = 0.0;
    for (int64_t n = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; n < N.n; n += (int64_t)gridDim.x * blockDim.x) {
        double q0 = 0.0, q1 = 0.0, q2 = 0.0;
        if (qbuf) gather_q(N, qbuf, n, q0, q1, q2);
        const uint8_t fm = N.fixmask[n];
        const double r0 = (fm & 1) ? 0.0 : b[3 * n] - q0;
        const double r1 = (fm & 2) ? 0.0 : b[3 * n + 1] - q1;
        const double r2 = (fm & 4) ? 0.0 : b[3 * n + 2] - q2;
        v += r0 * r0 + r1 * r1 + r2 * r2;
    }
    v = block_bcast_sum(v);
    if (threadIdx.x == 0) part[blockIdx.x] = v;
}

void launch_cand_res(hipStream_t s, const DevNodes& N, const double* qbuf, const double* b, double* part,
                     const DevScalars* skip) {
    hipLaunchKernelGGL(k_cand_res, dim3(res_grid(N.n)), dim3(256), 0, s, N, qbuf, b, part, skip);
}

__global__ __launch_bounds__(256) void k_cand_select(DevNodes N, const double* part_s, const double* part_l, int g,
                                                     double* x, const double* x_alt, double* qbuf,
                                                     const double* qbuf_alt, int64_t nq, DevScalars* sc, int which,
                                                     const DevScalars* skip) {
    if (skip && skip->guard_skip) {   // the alternative was not evaluated: keep the primary
        if (blockIdx.x == 0 && threadIdx.x == 0) {
            sc->guard_rr[1] = 0.0;
            sc->guard_pick = 0;
        }
        return;
    }
    double rs = lane_partials<kMaxResGrid / 256>(part_s, g, threadIdx.x, 256);
    double rl = lane_partials<kMaxResGrid / 256>(part_l, g, threadIdx.x, 256);
    rs = block_bcast_sum(rs);
    rl = block_bcast_sum(rl);
    const bool pick = rl < rs;   // NaN in the alternative keeps the primary candidate
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        double* rr = which ? sc->guard_rr : sc->cand_rr;
        rr[0] = rs;
        rr[1] = rl;
        if (which) sc->guard_pick = pick ? 1 : 0;
        else sc->cand_pick = pick ? 1 : 0;
    }
    if (!pick) return;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < 3 * N.n; i += stride) x[i] = x_alt[i];
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < nq; i += stride) qbuf[i] = qbuf_alt[i];
}

void launch_cand_select(hipStream_t s, const DevNodes& N, const double* part_s, const double* part_l, double* x,
                        const double* x_alt, double* qbuf, const double* qbuf_alt, int64_t nq, DevScalars* sc,
                        int which, const DevScalars* skip) {
    const int g = res_grid(N.n);
    hipLaunchKernelGGL(k_cand_select, dim3(g), dim3(256), 0, s, N, part_s, part_l, g, x, x_alt, qbuf, qbuf_alt, nq,
                       sc, which, skip);
}

__global__ __launch_bounds__(256) void k_guard_decide(const double* part_map, const double* part_bb, int g,
                                                      double thresh, DevScalars* sc) {
    double rm = lane_partials<kMaxResGrid / 256>(part_map, g, threadIdx.x, 256);
    double bb = lane_partials<kMaxResGrid / 256>(part_bb, g, threadIdx.x, 256);
    rm = block_bcast_sum(rm);
    bb = block_bcast_sum(bb);
    if (threadIdx.x == 0) {
        const double rho2 = bb > 0.0 ? rm / bb : rm;
        sc->guard_rr[0] = rm;
        sc->guess_bb = bb;
        sc->guard_skip = (thresh > 0.0 && rho2 < thresh * thresh) ? 1 : 0;
    }
}

void launch_guard_decide(hipStream_t s, const double* part_map, const double* part_bb, int g, double thresh,
                         DevScalars* sc) {
    hipLaunchKernelGGL(k_guard_decide, dim3(1), dim3(256), 0, s, part_map, part_bb, g, thresh, sc);
}

__global__ __launch_bounds__(256) void k_sum_partials(const double* part, int g, double* out) {
    double v = lane_partials<kMaxResGrid / 256>(part, g, threadIdx.x, 256);
    v = block_bcast_sum(v);
    if (threadIdx.x == 0) *out = v;
}

void launch_sum_partials(hipStream_t s, const double* part, int g, double* out) {
    hipLaunchKernelGGL(k_sum_partials, dim3(1), dim3(256), 0, s, part, g, out);
}

__global__ void k_fill(int64_t n, double value, double* p) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = value;
}

void launch_fill(hipStream_t s, int64_t n, double value, double* p) {
    hipLaunchKernelGGL(k_fill, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, n, value, p);
}

// ---------------------------------------------------------------------------
// predictor
// ---------------------------------------------------------------------------
// Adams-Bashforth 4-step increment: dab = dt/24 (55 v1 - 59 v2 + 37 v3 - 9 v4);
// x = dab (kind >= 1) or 0 (kind 0).
__global__ void k_ab4(int64_t n3, double dt, const double* v1, const double* v2, const double* v3, const double* v4,
                      int kind, double* dab, double* x) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n3) return;
    double w = dt * (1.0 / 24.0);
    double d = w * (55.0 * v1[i] - 59.0 * v2[i] + 37.0 * v3[i] - 9.0 * v4[i]);
    dab[i] = d;
    if (x) x[i] = kind == 0 ? 0.0 : d;
}

void launch_ab4(hipStream_t s, int64_t n3, double dt, const double* v1, const double* v2, const double* v3,
                const double* v4, int kind, double* dab, double* x) {
    int nb = (int)((n3 + 255) / 256);
    hipLaunchKernelGGL(k_ab4, dim3(nb), dim3(256), 0, s, n3, dt, v1, v2, v3, v4, kind, dab, x);
}

// Regional Gram products on FP64 MFMA (v_mfma_f64_16x16x4f64).  For the
// region's rows of W = [x_1 .. x_s, q]: X^T X from 16x16 tiles and X^T q from
// per-lane FMAs, written to gh[r] = [32][32] Gram followed by [32] X^T q.
template <int NB>
// Partial Gram of one node chunk (one workgroup): G = X^T X over the chunk's
// rows for the s_eff input columns, and X^T q for the query column s_eff.
__global__ __launch_bounds__(256) void k_gram(ColPtrs W, int s_eff, const int32_t* chunk_start, double* gh) {
    constexpr int NC = 16 * NB;
    constexpr int TR = 128;          // rows per LDS tile
    constexpr int LD = TR + 1;       // odd stride: the 16 columns read by one MFMA operand hit distinct banks
    constexpr int NT = NB * (NB + 1) / 2;
    __shared__ double tile[(NC + 1) * LD];
    __shared__ double hq[4][NC];
    double (*Gw)[NT][4][64] = reinterpret_cast<double (*)[NT][4][64]>(tile);   // reuses the tile after the loop
    static_assert(4 * NT * 4 * 64 <= (NC + 1) * LD, "per-wave tiles must fit in the staging buffer");
    const int r = blockIdx.x;
    const int64_t d0 = 3 * (int64_t)chunk_start[r], d1 = 3 * (int64_t)chunk_start[r + 1];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int col = lane & 15, krow = lane >> 4;
    const int ncols = s_eff + 1;     // X columns and the query
    __shared__ const double* colp[kMaxCols];
    if (threadIdx.x < ncols) colp[threadIdx.x] = W.c[threadIdx.x];
    const bool use0 = col < s_eff, use1 = NB == 2 && 16 + col < s_eff;
    double4_t c00 = {0, 0, 0, 0}, c01 = {0, 0, 0, 0}, c11 = {0, 0, 0, 0};
    double h0 = 0.0, h1 = 0.0;
    // staging map: thread t copies row t % TR of columns t / TR, t / TR + 2, ...
    constexpr int CPT = (NC + 2) / 2;          // columns per thread (ceil((NC + 1) / 2))
    const int srow = threadIdx.x % TR, sc0 = threadIdx.x / TR;
    __syncthreads();
    const double* sp[CPT];
#pragma unroll
    for (int k = 0; k < CPT; ++k) {
        const int c = sc0 + 2 * k;
        sp[k] = c < ncols ? colp[c] : nullptr;
    }
    // software pipeline: the next tile's loads are in flight while this tile's MFMAs run
    double v[CPT];
#pragma unroll
    for (int k = 0; k < CPT; ++k) v[k] = (sp[k] && d0 + srow < d1) ? sp[k][d0 + srow] : 0.0;
    for (int64_t base = d0; base < d1; base += TR) {
        __syncthreads();
#pragma unroll
        for (int k = 0; k < CPT; ++k)
            if (sp[k]) tile[(sc0 + 2 * k) * LD + srow] = v[k];
        __syncthreads();
        const int64_t nrow = base + TR + srow;
#pragma unroll
        for (int k = 0; k < CPT; ++k) v[k] = (sp[k] && nrow < d1) ? sp[k][nrow] : 0.0;
        // each wave owns 32 rows of the tile: 8 k-steps of 4 rows
#pragma unroll
        for (int t = 0; t < TR / 16; ++t) {
            const int rr = wave * (TR / 4) + 4 * t + krow;
            const double a0 = use0 ? tile[col * LD + rr] : 0.0;
            const double a1 = use1 ? tile[(16 + col) * LD + rr] : 0.0;
            const double q = tile[s_eff * LD + rr];
            c00 = __builtin_amdgcn_mfma_f64_16x16x4f64(a0, a0, c00, 0, 0, 0);
            if (NB == 2) {
                c01 = __builtin_amdgcn_mfma_f64_16x16x4f64(a0, a1, c01, 0, 0, 0);
                c11 = __builtin_amdgcn_mfma_f64_16x16x4f64(a1, a1, c11, 0, 0, 0);
            }
            h0 = fma(a0, q, h0);
            h1 = fma(a1, q, h1);
        }
    }
    __syncthreads();   // the staging buffer becomes Gw
    // per-wave tiles to LDS: register v of lane l holds D[l/16 + 4 v][l%16]
    for (int v = 0; v < 4; ++v) {
        Gw[wave][0][v][lane] = c00[v];
        if (NB == 2) {
            Gw[wave][1][v][lane] = c01[v];
            Gw[wave][2][v][lane] = c11[v];
        }
    }
    h0 += __shfl_xor(h0, 16, 64);
    h0 += __shfl_xor(h0, 32, 64);
    h1 += __shfl_xor(h1, 16, 64);
    h1 += __shfl_xor(h1, 32, 64);
    if (lane < 16) {
        hq[wave][lane] = h0;
        if (NB == 2) hq[wave][16 + lane] = h1;
    }
    __syncthreads();
    // sum over waves (fixed order) and store the symmetric Gram
    double* out = gh + (int64_t)r * kGhStride;
    for (int idx = threadIdx.x; idx < 4 * 64 * NT; idx += 256) {
        int t = idx / 256, rem = idx % 256, v = rem / 64, l = rem % 64;
        double sum = (Gw[0][t][v][l] + Gw[1][t][v][l]) + (Gw[2][t][v][l] + Gw[3][t][v][l]);
        int i = (l / 16) + 4 * v, j = l % 16;
        int bi = (t == 2) ? 1 : 0, bj = (t == 0) ? 0 : 1;
        out[(16 * bi + i) * 32 + 16 * bj + j] = sum;
        if (bi != bj) out[(16 * bj + j) * 32 + 16 * bi + i] = sum;
    }
    if (threadIdx.x < NC)
        out[1024 + threadIdx.x] = (hq[0][threadIdx.x] + hq[1][threadIdx.x]) + (hq[2][threadIdx.x] + hq[3][threadIdx.x]);
}

// Least-squares coefficients of one region (one 256-thread workgroup): the
// region's Gram is the sum of its chunks' partial Grams, taken by 8 streams
// (chunk c to stream (c - first) mod 8, in chunk order within a stream) and
// combined in a fixed tree; with column scaling d_j = sqrt(G_jj), Cholesky of
// the scaled Gram taken column by column in time order; a column whose
// remaining (orthogonal) part is below drop * its norm is dropped, which
// reproduces the column selection of modified Gram-Schmidt in that order.
// Then R^T y = h, R a = y, coef = a / d.
// Broadcast of lane l's value (l a compile-time constant in the unrolled loops below).
__device__ __forceinline__ double lane_value(double v, int l) {
    const int lo = __builtin_amdgcn_readlane(__double2loint(v), l);
    const int hi = __builtin_amdgcn_readlane(__double2hiint(v), l);
    return __hiloint2double(hi, lo);
}

// The sum over the chunks: the half-waves of the four waves each read every
// 8th chunk (a region of 14,000 nodes has 28 chunks: the serial sum of one
// wave waited for 28 round trips to memory).  Then every wave runs the same
// factorisation on the same sums, lane = column index; only wave 0 writes.
// Each lane keeps its column of the (scaled) Gram matrix in registers; row
// values of other columns come by readlane at unrolled, compile-time lane
// indices, so the factorisation has no LDS round trip and no barrier per
// pivot.  The column oriented Cholesky with pivot drop, the forward and the
// back substitution perform the same operations in the same order as a
// row-by-row implementation (the back substitution reads R^T from one LDS copy).
__global__ __launch_bounds__(256) void k_ls_solve(const double* gh, const int32_t* region_chunk, int s, double drop,
                                                  double* coef, const int32_t* region_case, const int32_t* case_lo,
                                                  int lo_all) {
    __shared__ double R[32][33];
    __shared__ double part[4][34][32];   // per wave: G[i][column] (i < 32), h[column], G[column][column]
    const int r = blockIdx.x, tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
    const int cl = lane & 31, stream = 2 * wave + (lane >> 5);
    // columns before lo are left out: zero in the Gram, never kept, zero coefficients
    const int lo = lo_all + (case_lo ? case_lo[region_case[r]] : 0);
    const bool ccol = cl >= lo && cl < s;
    double g[32], y = 0.0, gll = 0.0;   // g[i] = G[i][column]; gll = G[column][column]
#pragma unroll
    for (int i = 0; i < 32; ++i) g[i] = 0.0;
    for (int c = region_chunk[r] + stream; c < region_chunk[r + 1]; c += 8) {
        const double* in = gh + (int64_t)c * kGhStride;
#pragma unroll
        for (int i = 0; i < 32; ++i) g[i] += (ccol && i < s) ? in[i * 32 + cl] : 0.0;
        y += ccol ? in[1024 + cl] : 0.0;
        gll += ccol ? in[cl * 32 + cl] : 0.0;
    }
    // streams 2w and 2w + 1 (the two half-waves), then the four waves: ((w0 + w1) + (w2 + w3))
#pragma unroll
    for (int i = 0; i < 32; ++i) g[i] += __shfl_down(g[i], 32, 64);
    y += __shfl_down(y, 32, 64);
    gll += __shfl_down(gll, 32, 64);
    if (lane < 32) {
#pragma unroll
        for (int i = 0; i < 32; ++i) part[wave][i][cl] = g[i];
        part[wave][32][cl] = y;
        part[wave][33][cl] = gll;
    }
    __syncthreads();
    const bool col = lane < 32 && ccol;   // lanes 32..63 hold no column
#pragma unroll
    for (int i = 0; i < 32; ++i)
        g[i] = col ? (part[0][i][cl] + part[1][i][cl]) + (part[2][i][cl] + part[3][i][cl]) : 0.0;
    y = col ? (part[0][32][cl] + part[1][32][cl]) + (part[2][32][cl] + part[3][32][cl]) : 0.0;
    gll = col ? (part[0][33][cl] + part[1][33][cl]) + (part[2][33][cl] + part[3][33][cl]) : 0.0;
    const double dl = col ? sqrt(gll) : 0.0;
    // scaling by the column norms: G_il / (d_i d_l), h_l / d_l
#pragma unroll
    for (int i = 0; i < 32; ++i) {
        const double di = lane_value(dl, i);
        g[i] = (di > 0.0 && dl > 0.0) ? g[i] / (di * dl) : 0.0;
    }
    y = dl > 0.0 ? y / dl : 0.0;
    const double drop2 = drop * drop;
    uint32_t keep = 0;   // bit j: column j kept (uniform)
#pragma unroll
    for (int j = 0; j < 32; ++j) {
        if (j < s) {
            const double t = lane_value(g[j], j);
            const bool kj = lane_value(dl, j) > 0.0 && t >= drop2;
            const double rjj = kj ? sqrt(t) : 0.0;
            if (lane > j && col) g[j] = kj ? g[j] / rjj : 0.0;
            if (lane == j) g[j] = rjj;
            keep |= kj ? 1u << j : 0u;
            if (kj) {   // trailing update of the upper triangle, column = lane
#pragma unroll
                for (int k = j + 1; k < 32; ++k) {
                    const double gjk = lane_value(g[j], k);   // G[j][k] (row j, column k)
                    if (k < s && k <= lane && col) g[k] -= gjk * g[j];
                }
            }
        }
    }
#pragma unroll
    for (int j = 0; j < 32; ++j) {     // R^T y = h (column-oriented)
        if (j < s) {
            if (lane == j) y = ((keep >> j) & 1) ? y / g[j] : 0.0;
            const double yj = lane_value(y, j);
            if (lane > j && col) y -= g[j] * yj;
        }
    }
#pragma unroll
    for (int i = 0; i < 32; ++i)
        if (wave == 0 && lane < 32) R[i][lane] = g[i];   // R[i][l] from lane l
    __syncthreads();
#pragma unroll
    for (int j = 31; j >= 0; --j) {    // R a = y
        if (j < s) {
            if (lane == j) y = ((keep >> j) & 1) ? y / g[j] : 0.0;
            const double yj = lane_value(y, j);
            if (lane < j) y -= R[lane][j] * yj;
        }
    }
    if (wave == 0 && lane < 32) coef[32 * (int64_t)r + lane] = (col && ((keep >> lane) & 1)) ? y / dl : 0.0;
}

void launch_gram_solve(hipStream_t s, const ColPtrs& W, int s_eff, const DevChunks& C, double drop, double* gh,
                       double* coef, const int32_t* case_lo) {
    if (s_eff <= 16)
        hipLaunchKernelGGL(k_gram<1>, dim3(C.n_chunks), dim3(256), 0, s, W, s_eff, C.start, gh);
    else
        hipLaunchKernelGGL(k_gram<2>, dim3(C.n_chunks), dim3(256), 0, s, W, s_eff, C.start, gh);
    hipLaunchKernelGGL(k_ls_solve, dim3(C.n_regions), dim3(256), 0, s, gh, C.first, s_eff, drop, coef, C.region_case,
                       case_lo, 0);
}

void launch_gram(hipStream_t s, const ColPtrs& W, int s_eff, const DevChunks& C, double* gh) {
    if (s_eff <= 16)
        hipLaunchKernelGGL(k_gram<1>, dim3(C.n_chunks), dim3(256), 0, s, W, s_eff, C.start, gh);
    else
        hipLaunchKernelGGL(k_gram<2>, dim3(C.n_chunks), dim3(256), 0, s, W, s_eff, C.start, gh);
}

void launch_ls_solve(hipStream_t s, int s_eff, const DevChunks& C, double drop, const double* gh, double* coef,
                     int lo) {
    hipLaunchKernelGGL(k_ls_solve, dim3(C.n_regions), dim3(256), 0, s, gh, C.first, s_eff, drop, coef,
                       (const int32_t*)nullptr, (const int32_t*)nullptr, lo);
}

// x = dab + sum_j coef_j Y_j on each node chunk with its region's
// coefficients, Y_j = W.c[j + 1] (outputs).  (A fully unrolled variant with
// all 32 column loads of a row in flight measured slower, 228 vs 195 us.)
__global__ __launch_bounds__(256) void k_pred_apply(ColPtrs W, int s_eff, const int32_t* chunk_start,
                                                    const int32_t* chunk_region, const double* coef,
                                                    const double* dab, double* x) {
    // chunks in the reverse of the Gram pass's order: the columns that pass
    // read last are the ones still in the memory-side cache
    const int c = gridDim.x - 1 - blockIdx.x;
    const int64_t d0 = 3 * (int64_t)chunk_start[c], d1 = 3 * (int64_t)chunk_start[c + 1];
    const double* a = coef + 32 * (int64_t)chunk_region[c];
    for (int64_t i = d0 + threadIdx.x; i < d1; i += 256) {
        double t = dab[i];
#pragma unroll 8
        for (int j = 0; j < s_eff; ++j) t = fma(a[j], W.c[j + 1][i], t);
        x[i] = t;
    }
}

void launch_pred_apply(hipStream_t s, const ColPtrs& W, int s_eff, const DevChunks& C, const double* coef,
                       const double* dab, double* x) {
    hipLaunchKernelGGL(k_pred_apply, dim3(C.n_chunks), dim3(256), 0, s, W, s_eff, C.start, C.region, coef, dab, x);
}

// Newmark-beta (beta = 1/4, gamma = 1/2): u += du; v' = -v + (2/dt) du;
// a' = -a - (4/dt) v + (4/dt^2) du; AB error du - dab into the ring slot.
// With a guard, the update runs only if the solve that produced du has ended
// with a usable increment (converged, or stopped at max_iter).
__global__ void k_newmark(int64_t n3, double dt, const double* du, const double* dab, double* u, const double* v_old,
                          double* v_new, double* a, double* ring_slot, const DevScalars* guard) {
    if (guard) {
        const int d = guard->done;
        if (d != DONE_CONVERGED && d != DONE_MAXITER) return;
    }
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n3) return;
    double d = du[i], vo = v_old[i];
    u[i] += d;
    v_new[i] = fma(2.0 / dt, d, -vo);
    a[i] = fma(4.0 / (dt * dt), d, fma(-4.0 / dt, vo, -a[i]));
    if (ring_slot) ring_slot[i] = d - dab[i];
}

void launch_newmark(hipStream_t s, int64_t n3, double dt, const double* du, const double* dab, double* u,
                    const double* v_old, double* v_new, double* a, double* ring_slot, const DevScalars* guard) {
    int nb = (int)((n3 + 255) / 256);
    hipLaunchKernelGGL(k_newmark, dim3(nb), dim3(256), 0, s, n3, dt, du, dab, u, v_old, v_new, a, ring_slot, guard);
}

__global__ void k_gather3(int64_t n, const int32_t* idx, const double* in, double* out) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    int64_t j = idx[i];
    out[3 * i] = in[3 * j]; out[3 * i + 1] = in[3 * j + 1]; out[3 * i + 2] = in[3 * j + 2];
}

void launch_gather3(hipStream_t s, int64_t n, const int32_t* idx, const double* in, double* out) {
    int nb = (int)((n + 255) / 256);
    hipLaunchKernelGGL(k_gather3, dim3(nb), dim3(256), 0, s, n, idx, in, out);
}

__global__ void k_zero(int64_t n, double* p) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0.0;
}

void launch_zero(hipStream_t s, int64_t count, double* p) {
    int nb = (int)((count + 255) / 256);
    hipLaunchKernelGGL(k_zero, dim3(nb), dim3(256), 0, s, count, p);
}

}  // namespace ebe
