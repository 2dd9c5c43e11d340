// api.hip -- C ABI of the library (declared in include/ebe.h): handle
// management, assembly and the per-step orchestration
//   right-hand side -> Adams-Bashforth 4 -> regional snapshot map ->
//   Algorithm 1 (block-Jacobi PCG, element-by-element matvec) -> Newmark.
// Every numerical step runs in the kernels of kernels.hip; this file only
// allocates, copies topology to the device and enqueues work on the stream.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "../../include/ebe.h"
#include "kernels.h"
#include "topology.h"

using namespace ebe;

namespace {

struct HipError {
    std::string msg;
};

#define HIPCHK(expr)                                                                           \
    do {                                                                                       \
        hipError_t _e = (expr);                                                                \
        if (_e != hipSuccess) throw HipError{std::string(#expr) + ": " + hipGetErrorString(_e)}; \
    } while (0)

struct Arg {
    std::string msg;
};
struct State {
    std::string msg;
};

thread_local std::string g_create_error;

// ---- fixed device array of ebe_mlp_grad_noalloc ---------------------------
// Training activations of one gradient evaluation of at most kMlpMaxBatch
// samples, laid out as 256-byte aligned pieces: the loss (one double), the
// per-workgroup loss partials, then X [15][B], Z1, H1, Z2, H2 [64][B],
// dY [3][B], dZ1, dZ2 [64][B] (B = the call's sample count, at most
// kMlpMaxBatch, so every piece is sized for kMlpMaxBatch).
constexpr size_t kScratchAlign = 256;
constexpr size_t scratch_piece(size_t bytes) { return (bytes + kScratchAlign - 1) / kScratchAlign * kScratchAlign; }
constexpr size_t kScratchLoss = 0;
constexpr size_t kScratchLossPart = kScratchLoss + scratch_piece(sizeof(double));
constexpr size_t kScratchAct = kScratchLossPart + scratch_piece(sizeof(float) * (kMlpMaxBatch + 255) / 256);
constexpr size_t kScratchFloatsPerSample = kMlpIn + 4 * kMlpHid + kMlpOut + 2 * kMlpHid;
constexpr size_t kScratchBytes = kScratchAct + scratch_piece(sizeof(float) * kScratchFloatsPerSample * kMlpMaxBatch);
static_assert(kScratchBytes < 14u * 1024 * 1024, "the fixed training scratch stays modest");

static __device__ __align__(256) unsigned char scratch[kScratchBytes];

// Device address of `scratch` on each device (its host-side name is not a
// device address).  Looked up once per device, with that device current, by
// ebe_create.
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

hipError_t lookup_scratch(int device) {
    if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (g_scratch_ptr[device]) return hipSuccess;
    void* ptr = nullptr;
    hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e == hipSuccess) g_scratch_ptr[device] = ptr;
    return e;
}

void* scratch_ptr(int device) {
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    return device >= 0 && device < kMaxDevices ? g_scratch_ptr[device] : nullptr;
}

}  // namespace

struct ebe_handle {
    ebe_config cfg{};
    hipStream_t stream = nullptr;
    int device = 0;
    std::string err;
    bool assembled = false;
    double cM = 0, cK = 0;
    Topology T;
    DevPatches dp{};
    DevNodes dn{};
    std::vector<void*> allocs;
    int32_t* d_i2u = nullptr;
    int32_t* d_u2i = nullptr;
    DevChunks chunks{};
    double* binv6 = nullptr;
    double* qbuf = nullptr;
    // state (internal node order)
    double* u = nullptr;
    double* a = nullptr;
    double* vh[4] = {nullptr, nullptr, nullptr, nullptr};
    int head = 0;  // vh[(head + j) & 3] = v^(it - j)
    double* ring = nullptr;
    int32_t it = 0;
    ebe_window ws{1, 0, 0, 0, 0.0, 0.0};   // snapshot-window state (start, length cap, probes)
    double* coef_probe = nullptr;          // [n_regions][32] coefficients over the probed length
    double* x_probe = nullptr;             // [3N] guess over the probed length
    // scratch
    double *dab = nullptr, *x = nullptr, *b = nullptr, *r = nullptr, *z = nullptr, *p[2] = {nullptr, nullptr};
    double *t0 = nullptr, *t1 = nullptr, *coef = nullptr, *gh = nullptr;
    int par = 0;
    int last_iters = 0;
    // Set by ebe_step for the duration of its solve: the Newmark update is
    // enqueued, guarded by the stop flag, behind every read-back of the scalars,
    // so that it runs while the host handles the read-back.
    bool post_newmark = false;
    double* post_slot = nullptr;
    DevScalars* sc = nullptr;
    DevScalars* sc_host = nullptr;
    double* pap_part = nullptr;   // (p, A p) partials of the matvec grid
    double* res_part = nullptr;   // two slots of [kResArrays][res_grid] residual partials
    // mixed precision (inner solve in FP32 arithmetic, vectors in FP32 / BF16)
    void *r_in = nullptr, *e_in = nullptr, *z_in = nullptr, *p_in[2] = {nullptr, nullptr}, *q_in = nullptr;
    void* binv_in = nullptr;
    double* r_prev = nullptr;
    DevScalars* sc_in = nullptr;
    double* pap_in = nullptr;
    double* res_in = nullptr;
    int par_in = 0;
    // learned predictor (allocated on first use; dropped by ebe_assemble)
    double* msum = nullptr;          // [N] row sums of M
    double* x_alt = nullptr;         // [3N] learned candidate
    double* cand_part = nullptr;     // [2][res_grid] candidate residual partials
    double* qbuf_alt = nullptr;      // matvec slots of the alternative guess (AB4 or learned)
    bool q_ready = false;            // qbuf already holds A x for the next solve's guess
    uint16_t* mlp_w = nullptr;       // BF16 weights
    float *mlp_wm = nullptr, *mlp_m = nullptr, *mlp_v = nullptr;
    float mlp_scales[kMlpScales] = {1.0f, 1.0f, 1.0f, 1.0f};
    int cand_losses = 0;             // consecutive steps the learned candidate lost
    bool mlp_ready = false;
    int mlp_t = 0;                   // Adam steps taken
    MlpTrain tr{};
    int tr_cap = 0;                  // batch capacity of the training scratch
    double* tr_loss = nullptr;
    int tr_loss_cap = 0;
    float* samples = nullptr;        // [samples_cap][kMlpSample]
    int64_t samples_cap = 0, samples_n = 0;
    int32_t* coll_nodes = nullptr;   // internal ids of the sampled nodes
    double* coll_stage = nullptr;
    int coll_k = 0, coll_cap_k = 0;
    double* rms3 = nullptr;
    int32_t* flag = nullptr;
    // kernel timing
    int timing_every = 0;
    int64_t pcg_launches = 0;
    std::vector<hipEvent_t> ev_free;
    std::vector<std::pair<hipEvent_t, hipEvent_t>> ev_pending;
    double time_sum_ms = 0.0;
    int64_t time_n = 0;

    int64_t n3() const { return 3 * T.n_nodes; }
    double* ring_slot(int k) const { return ring + (int64_t)k * n3(); }
    double* vslot(int j) const { return vh[(head + j) & 3]; }

    template <class X>
    X* alloc(size_t count) {
        void* p = nullptr;
        if (count == 0) count = 1;
        hipError_t e = hipMalloc(&p, count * sizeof(X));
        if (e != hipSuccess) throw std::bad_alloc();
        allocs.push_back(p);
        return static_cast<X*>(p);
    }
    // Frees one allocation made by alloc (no-op for null).
    void release(void* p) {
        if (!p) return;
        auto it = std::find(allocs.begin(), allocs.end(), p);
        if (it == allocs.end()) return;
        if (stream) (void)hipStreamSynchronize(stream);
        (void)hipFree(p);
        allocs.erase(it);
    }
    template <class X>
    X* upload(const std::vector<X>& v) {
        X* d = alloc<X>(v.size());
        if (!v.empty()) HIPCHK(hipMemcpyAsync(d, v.data(), v.size() * sizeof(X), hipMemcpyHostToDevice, stream));
        return d;
    }
    void free_all() {
        if (stream) (void)hipStreamSynchronize(stream);
        for (void* p : allocs) (void)hipFree(p);
        allocs.clear();
        for (auto& pr : ev_pending) {
            (void)hipEventDestroy(pr.first);
            (void)hipEventDestroy(pr.second);
        }
        ev_pending.clear();
        for (auto e : ev_free) (void)hipEventDestroy(e);
        ev_free.clear();
        assembled = false;
        msum = x_alt = cand_part = qbuf_alt = nullptr;
        q_ready = false;
        cand_losses = 0;
        mlp_w = nullptr;
        mlp_wm = mlp_m = mlp_v = nullptr;
        mlp_ready = false;
        mlp_t = 0;
        tr = MlpTrain{};
        tr_cap = 0;
        tr_loss = nullptr;
        tr_loss_cap = 0;
        samples = nullptr;
        samples_cap = samples_n = 0;
        coll_nodes = nullptr;
        coll_stage = nullptr;
        coll_k = coll_cap_k = 0;
        rms3 = nullptr;
        flag = nullptr;
    }
};

namespace {

template <class F>
int guarded(ebe_handle* h, F&& f) {
    if (!h) return EBE_E_INVALID_ARG;
    h->err.clear();
    try {
        HIPCHK(hipSetDevice(h->device));
        return f();
    } catch (const Arg& e) {
        h->err = e.msg;
        return EBE_E_INVALID_ARG;
    } catch (const State& e) {
        h->err = e.msg;
        return EBE_E_BAD_STATE;
    } catch (const HipError& e) {
        h->err = e.msg;
        return EBE_E_HIP;
    } catch (const std::bad_alloc&) {
        h->err = "out of memory";
        return EBE_E_NO_MEMORY;
    } catch (const std::exception& e) {
        h->err = e.what();
        return EBE_E_HIP;
    } catch (...) {
        h->err = "unknown error";
        return EBE_E_HIP;
    }
}

void need_assembled(ebe_handle* h) {
    if (!h->assembled) throw State{"ebe_assemble has not been called"};
}

void need_ptr(const void* p, const char* name) {
    if (!p) throw Arg{std::string(name) + " is NULL"};
}

void check_launch() { HIPCHK(hipGetLastError()); }

// user order -> internal order, and back
void to_internal(ebe_handle* h, const double* user, double* internal) {
    launch_gather3(h->stream, h->T.n_nodes, h->d_i2u, user, internal);
}
void to_user(ebe_handle* h, const double* internal, double* user) {
    launch_gather3(h->stream, h->T.n_nodes, h->d_u2i, internal, user);
}

void harvest_timing(ebe_handle* h, bool wait) {
    auto it = h->ev_pending.begin();
    while (it != h->ev_pending.end()) {
        if (!wait && hipEventQuery(it->second) != hipSuccess) {
            ++it;
            continue;
        }
        HIPCHK(hipEventSynchronize(it->second));
        float ms = 0.f;
        HIPCHK(hipEventElapsedTime(&ms, it->first, it->second));
        h->time_sum_ms += ms;
        h->time_n += 1;
        h->ev_free.push_back(it->first);
        h->ev_free.push_back(it->second);
        it = h->ev_pending.erase(it);
    }
}

hipEvent_t take_event(ebe_handle* h) {
    if (!h->ev_free.empty()) {
        hipEvent_t e = h->ev_free.back();
        h->ev_free.pop_back();
        return e;
    }
    hipEvent_t e;
    HIPCHK(hipEventCreate(&e));
    return e;
}

void sync_stream(ebe_handle* h) {
    HIPCHK(hipStreamSynchronize(h->stream));
    if (!h->ev_pending.empty()) harvest_timing(h, true);
}

// Copies the scalars to the host and waits for them.  With post_newmark the
// guarded Newmark update goes behind the copy and is not waited for.
void read_scalars(ebe_handle* h) {
    hipStream_t s = h->stream;
    HIPCHK(hipMemcpyAsync(h->sc_host, h->sc, sizeof(DevScalars), hipMemcpyDeviceToHost, s));
    if (!h->post_newmark) {
        sync_stream(h);
        return;
    }
    hipEvent_t e = take_event(h);
    HIPCHK(hipEventRecord(e, s));
    launch_newmark(s, h->n3(), h->cfg.dt, h->x, h->dab, h->u, h->vslot(0), h->vslot(3), h->a, h->post_slot, h->sc);
    check_launch();
    HIPCHK(hipEventSynchronize(e));
    h->ev_free.push_back(e);
    if (!h->ev_pending.empty()) harvest_timing(h, true);
}

// Statistics and status of a finished solve from the scalars read back last.
int finish_solve(ebe_handle* h, double* x, int done, ebe_solve_stats* st) {
    const DevScalars& S = *h->sc_host;
    if (done == DONE_ZERO_RHS) {
        launch_zero(h->stream, h->n3(), x);
        check_launch();
    }
    if (st) {
        st->iters = S.iters;
        st->restarts = S.restarts;
        st->inner_iters = S.inner_iters;
        st->res0 = S.res0;
        st->bnorm = S.bnorm;
        st->res_rec = S.bnorm > 0 ? std::sqrt(S.rr) / S.bnorm : 0.0;
        st->res_true = S.bnorm > 0 ? S.res_true : 0.0;
        st->status = (done == DONE_MAXITER) ? EBE_NOT_CONVERGED : EBE_OK;
    }
    if (done == DONE_NONFINITE) {
        h->err = "non-finite value in the PCG iteration";
        return EBE_E_NONFINITE;
    }
    h->last_iters = S.iters;
    if (done == DONE_MAXITER) {
        h->err = "PCG reached max_iter";
        return EBE_NOT_CONVERGED;
    }
    return EBE_OK;
}

// Algorithm 1 on internal-order vectors: b, x (guess in, solution out).
// Trips are enqueued in chunks; a device-side stop flag makes the remaining
// kernels of a chunk return at once, and the host reads the scalars once per
// chunk.  Each chunk ends with the true-residual check, which only runs on the
// device once the loop has stopped.
int solve(ebe_handle* h, const double* b, double* x, ebe_solve_stats* st) {
    hipStream_t s = h->stream;
    const double tol = h->cfg.tol;
    const int max_iter = h->cfg.max_iter;
    const int g_res = res_grid(h->T.n_nodes);
    const int g_pap = pcg_ebe_grid(h->dp);
    auto slot = [&](int j) { return h->res_part + (size_t)(j & 1) * kResArrays * g_res; };
    if (!h->q_ready) launch_ebe_apply(s, h->dp, x, true, h->cM, h->cK, h->qbuf);
    h->q_ready = false;
    launch_residual(s, h->dn, h->qbuf, b, h->binv6, x, h->r, h->z, h->sc, slot(0), 0);
    check_launch();
    int chunk = h->cfg.chunk_iters > 0 ? h->cfg.chunk_iters : std::max(2, h->last_iters + 1);
    int done = DONE_RUNNING;
    int j = 0;
    const int par0 = h->par;
    for (int round = 0;; ++round) {
        for (int k = 0; k < chunk; ++k, ++j) {
            double* pprev = h->p[h->par];
            double* pcur = h->p[h->par ^ 1];
            // time only trips that certainly do work (well before the previous solve's count)
            bool timed = h->timing_every > 0 && (h->pcg_launches % h->timing_every) == 0 && j + 3 < h->last_iters;
            hipEvent_t e0 = nullptr, e1 = nullptr;
            if (timed) {
                e0 = take_event(h);
                e1 = take_event(h);
                HIPCHK(hipEventRecord(e0, s));
            }
            PcgLaunch L{&h->dp, PREC_FP64, false, h->z, pprev, pcur, h->qbuf, h->cM, h->cK, h->sc, nullptr,
                        slot(j), g_res, h->pap_part, j, max_iter, tol};
            launch_ebe_pcg(s, L);
            if (timed) {
                HIPCHK(hipEventRecord(e1, s));
                h->ev_pending.emplace_back(e0, e1);
            }
            h->pcg_launches++;
            UpdLaunch U{&h->dn, PREC_FP64, h->qbuf, pcur, h->binv6, x, h->r, h->z, h->sc, nullptr, h->pap_part, g_pap,
                        slot(j + 1), j, nullptr, pprev};
            launch_pcg_update(s, U);
            h->par ^= 1;
        }
        // true-residual check (runs on the device only once the loop stopped), after the
        // last trip's deferred half of the paired x update
        launch_flush_x(s, h->dn, x, h->p[0], h->p[1], par0, h->sc);
        launch_ebe_apply(s, h->dp, x, true, h->cM, h->cK, h->qbuf, h->sc);
        launch_residual(s, h->dn, h->qbuf, b, h->binv6, x, h->r, h->z, h->sc, slot(j), 1);
        launch_check_finalize(s, h->sc, slot(j), g_res, j, tol);
        check_launch();
        read_scalars(h);
        done = h->sc_host->done;
        if (done == DONE_RUNNING) {
            chunk = h->cfg.chunk_iters > 0 ? h->cfg.chunk_iters : std::max(2, h->last_iters / 8);
            if (round > 100000) throw HipError{"PCG loop did not terminate"};
            continue;
        }
        break;
    }
    return finish_solve(h, x, done, st);
}

// Mixed-precision refinement: flexible FP64 outer PCG whose preconditioner is
// an inner block-Jacobi PCG in FP32 arithmetic (vectors stored in FP32 or BF16).
// Outer trip j: inner init (outer stop test on r, r_in = float(r)), at most
// inner_iters inner trips (they stop at inner_tol), z = e in FP64 with the
// partials (z,r), (r,r), (z,r_prev), flexible matvec (Polak-Ribiere beta,
// p = z + beta p, q = A p), outer update.  All stop tests run on the device;
// the host reads the scalars once per chunk of outer trips.
int solve_mixed(ebe_handle* h, const double* b, double* x, ebe_solve_stats* st) {
    hipStream_t s = h->stream;
    const double tol = h->cfg.tol;
    const int max_iter = h->cfg.max_iter;
    const int prec = h->cfg.precision;
    const int g_res = res_grid(h->T.n_nodes);
    const int g_pap = pcg_ebe_grid(h->dp);
    auto slot = [&](int j) { return h->res_part + (size_t)(j & 1) * kResArrays * g_res; };
    auto islot = [&](int i) { return h->res_in + (size_t)(i & 1) * kResArrays * g_res; };
    if (!h->q_ready) launch_ebe_apply(s, h->dp, x, true, h->cM, h->cK, h->qbuf);
    h->q_ready = false;
    launch_residual(s, h->dn, h->qbuf, b, h->binv6, x, h->r, h->z, h->sc, slot(0), 0);
    check_launch();
    // an outer trip past the stop test still launches its ~2 x inner_iters guarded kernels, so the
    // first chunk is the previous count (not more), which covers almost every step in one read-back
    int chunk = h->cfg.chunk_iters > 0 ? h->cfg.chunk_iters : std::max(1, h->last_iters);
    int done = DONE_RUNNING;
    int j = 0;
    for (int round = 0;; ++round) {
        for (int k = 0; k < chunk; ++k, ++j) {
            launch_inner_init(s, prec, h->dn, h->r, h->binv_in, h->r_in, h->e_in, h->z_in, h->sc, slot(j), j,
                              max_iter, tol, h->sc_in, islot(0));
            for (int i = 0; i < h->cfg.inner_iters; ++i) {
                void* pprev = h->p_in[h->par_in];
                void* pcur = h->p_in[h->par_in ^ 1];
                PcgLaunch L{&h->dp, prec, false, h->z_in, pprev, pcur, h->q_in, h->cM, h->cK, h->sc_in, h->sc,
                            islot(i), g_res, h->pap_in, i, h->cfg.inner_iters, h->cfg.inner_tol};
                launch_ebe_pcg(s, L);
                UpdLaunch U{&h->dn, prec, h->q_in, pcur, h->binv_in, h->e_in, h->r_in, h->z_in, h->sc_in, h->sc,
                            h->pap_in, g_pap, islot(i + 1), i, &h->sc->inner_iters};
                launch_pcg_update(s, U);
                h->par_in ^= 1;
            }
            launch_outer_z(s, h->dn, h->e_in, h->r, h->r_prev, h->z, h->sc, slot(j), j);
            double* pprev = h->p[h->par];
            double* pcur = h->p[h->par ^ 1];
            // the first outer trip always works; later ones well before the previous solve's count
            bool timed = h->timing_every > 0 && (h->pcg_launches % h->timing_every) == 0 &&
                         (j == 0 || j + 2 < h->last_iters);
            hipEvent_t e0 = nullptr, e1 = nullptr;
            if (timed) {
                e0 = take_event(h);
                e1 = take_event(h);
                HIPCHK(hipEventRecord(e0, s));
            }
            PcgLaunch L{&h->dp, PREC_FP64, true, h->z, pprev, pcur, h->qbuf, h->cM, h->cK, h->sc, nullptr, slot(j),
                        g_res, h->pap_part, j, max_iter, tol};
            launch_ebe_pcg(s, L);
            if (timed) {
                HIPCHK(hipEventRecord(e1, s));
                h->ev_pending.emplace_back(e0, e1);
            }
            h->pcg_launches++;
            launch_outer_update(s, h->dn, h->qbuf, pcur, x, h->r, h->r_prev, h->sc, h->pap_part, g_pap, slot(j + 1),
                                j);
            h->par ^= 1;
        }
        launch_ebe_apply(s, h->dp, x, true, h->cM, h->cK, h->qbuf, h->sc);
        launch_residual(s, h->dn, h->qbuf, b, h->binv6, x, h->r, h->z, h->sc, slot(j), 1);
        launch_check_finalize(s, h->sc, slot(j), g_res, j, tol);
        check_launch();
        read_scalars(h);
        done = h->sc_host->done;
        if (done == DONE_RUNNING) {
            chunk = h->cfg.chunk_iters > 0 ? h->cfg.chunk_iters : 1;
            if (round > 100000) throw HipError{"PCG loop did not terminate"};
            continue;
        }
        break;
    }
    return finish_solve(h, x, done, st);
}

int run_solve(ebe_handle* h, const double* b, double* x, ebe_solve_stats* st) {
    return h->cfg.precision == EBE_PREC_FP64 ? solve(h, b, x, st) : solve_mixed(h, b, x, st);
}

int s_min_eff(const ebe_handle* h) { return std::max(1, std::min(h->cfg.s_min, h->cfg.s)); }

// Shortest window length the probes may reach: s_min, but not below the
// paper's lower end of s (8, or s itself when s < 8; Sec. 4, Fig. 3).
int len_min_eff(const ebe_handle* h) { return std::max(s_min_eff(h), std::min(8, h->cfg.s)); }

// Snapshot window of step n: AB errors e^first .. e^{n-1}, first = max(start,
// n - 1 - s_cap); returns the column pairs s_eff = n - 1 - first when the map is
// used (s_eff >= s_min), else 0.
int snapshot_window(const ebe_handle* h, int n, int* first_out) {
    *first_out = 0;
    if ((h->cfg.predictor != EBE_PRED_SNAPSHOT && h->cfg.predictor != EBE_PRED_LEARNED) || h->cfg.s < 1) return 0;
    const int first = std::max(h->ws.start, n - 1 - h->ws.s_cap);
    const int s_eff = n - 1 - first;
    if (s_eff < s_min_eff(h)) return 0;
    *first_out = first;
    return s_eff;
}

// Window length probed on step n (0: none): on the probe_every-th step with a
// full window, s_cap -/+ probe_step, alternating, as far as the bounds allow.
int probe_length(const ebe_handle* h, int n, int s_eff) {
    const ebe_config& c = h->cfg;
    if (c.fixed_window || c.col_cost < 0 || s_eff != h->ws.s_cap || h->ws.since + 1 < c.probe_every) return 0;
    const int s_cap = h->ws.s_cap, d = c.probe_step;
    const bool can_grow = s_cap + d <= c.s && n - 1 - (s_cap + d) >= h->ws.start;
    const bool can_shrink = s_cap - d >= len_min_eff(h);
    if (h->ws.grow_next && can_grow) return s_cap + d;
    if (can_shrink) return s_cap - d;
    if (can_grow) return s_cap + d;
    return 0;
}

// AB4 increment into dab and the guess of step n = it + 1 into x: dab (or 0
// for kind 0), plus the regional map over the window when it is used; with a
// probed length alt, also the map over alt pairs into x_probe (one Gram over
// the longer of the two windows, each least-squares solve on its newest columns).
int predict_into(ebe_handle* h, double* x, int* first, int alt = 0) {
    hipStream_t s = h->stream;
    const int n = h->it + 1;
    launch_ab4(s, h->n3(), h->cfg.dt, h->vslot(0), h->vslot(1), h->vslot(2), h->vslot(3),
               h->cfg.predictor == EBE_PRED_ZERO ? 0 : 1, h->dab, x);
    int s_eff = snapshot_window(h, n, first);
    if (s_eff >= 1) {
        const int s_long = std::max(s_eff, alt);
        ColPtrs W{};
        const int S1 = h->cfg.s + 1, f0 = n - 1 - s_long;
        for (int j = 0; j <= s_long; ++j) W.c[j] = h->ring_slot((f0 + j - 1) % S1);   // e^{f0 + j}
        launch_gram(s, W, s_long, h->chunks, h->gh);
        launch_ls_solve(s, s_long, h->chunks, h->cfg.drop_tol, h->gh, h->coef, s_long - s_eff);
        launch_pred_apply(s, W, s_long, h->chunks, h->coef, h->dab, x);
        if (alt > 0) {
            launch_ls_solve(s, s_long, h->chunks, h->cfg.drop_tol, h->gh, h->coef_probe, s_long - alt);
            launch_pred_apply(s, W, s_long, h->chunks, h->coef_probe, h->dab, h->x_probe);
        }
    }
    check_launch();
    return s_eff;
}

void rhs_into(ebe_handle* h, const double* f_int, const double* g, double* b) {
    const ebe_config& c = h->cfg;
    double g0 = g ? g[0] : 0.0, g1 = g ? g[1] : 0.0, g2 = g ? g[2] : 0.0;
    launch_ebe_rhs(h->stream, h->dp, h->u, h->vslot(0), h->a, 4.0 / c.dt + c.rayleigh_alpha, c.rayleigh_beta, g0, g1,
                   g2, h->qbuf);
    launch_rhs_finalize(h->stream, h->dn, h->qbuf, f_int, b);
    check_launch();
}

MlpState mlp_state(ebe_handle* h, const double* f_int, const double* g) {
    MlpState S{};
    S.u = h->u;
    S.v1 = h->vslot(0); S.v2 = h->vslot(1); S.v3 = h->vslot(2); S.v4 = h->vslot(3);
    S.hdt = 0.5 * h->cfg.dt;
    S.msum = h->msum;
    S.g0 = g ? g[0] : 0.0; S.g1 = g ? g[1] : 0.0; S.g2 = g ? g[2] : 0.0;
    S.f_int = f_int;
    for (int g = 0; g < 3; ++g) S.inv_s[g] = 1.0 / h->mlp_scales[g];
    S.s_t = h->mlp_scales[3];
    S.fixmask = h->dn.fixmask;
    return S;
}

// First step whose four displacement inputs are all past the rest state.
constexpr int kLearnFirstStep = 5;

bool learned_due(const ebe_handle* h, int n) {
    return h->cfg.predictor == EBE_PRED_LEARNED && h->mlp_ready && n >= kLearnFirstStep;
}

void need_x_alt(ebe_handle* h) {
    if (!h->x_alt) h->x_alt = h->alloc<double>(h->n3());
}

// After this many consecutive steps in which the kind-2 guess was kept, the
// learned candidate is evaluated only on every kCandProbe-th step until it
// wins again (its evaluation costs two matvecs and an inference).
constexpr int kCandPatience = 8;
constexpr int kCandProbe = 16;

// Keeps in x whichever of x (primary; its matvec slots already in qbuf when
// q_ready) and x_alt has the smaller initial residual ||b - A x|| over the free
// rows, with that guess's matvec slots in qbuf (ties keep the primary).
void choose(ebe_handle* h, const double* x_alt, int which) {
    hipStream_t s = h->stream;
    const int gr = res_grid(h->T.n_nodes);
    if (!h->q_ready) launch_ebe_apply(s, h->dp, h->x, true, h->cM, h->cK, h->qbuf);
    launch_cand_res(s, h->dn, h->qbuf, h->b, h->cand_part);
    launch_ebe_apply(s, h->dp, x_alt, true, h->cM, h->cK, h->qbuf_alt);
    launch_cand_res(s, h->dn, h->qbuf_alt, h->b, h->cand_part + gr);
    launch_cand_select(s, h->dn, h->cand_part, h->cand_part + gr, h->x, x_alt, h->qbuf, h->qbuf_alt,
                       (int64_t)(3 * h->T.patch_nodes.size()), h->sc, which);
    check_launch();
    h->q_ready = true;   // qbuf holds the kept guess's matvec: the solve skips its first one
}

// Learned candidate = Adams-Bashforth increment (dab) + network estimate of
// its error, judged against the guess in x.
void choose_learned(ebe_handle* h, const double* f_int, const double* g) {
    need_x_alt(h);
    MlpState S = mlp_state(h, f_int, g);
    S.xs = h->dab;
    S.xl = h->x_alt;
    launch_mlp_infer_state(h->stream, h->mlp_w, S, h->T.n_nodes);
    choose(h, h->x_alt, 0);
}

// What the guess of the next step was made of (host-side facts; the picks are
// device scalars read back with the solve's).
struct GuessInfo {
    int n = 0, s_eff = 0, first = 0;
    int probe = 0;          // window length probed (0: none)
    bool guarded = false;   // map's guess compared with the AB4 guess (or that comparison skipped)
    bool learned = false;   // learned candidate evaluated
};

// Right-hand side of step n = it + 1 into b and its guess into x (Eq.
// predictor with the predictor of Sec. 3.2): AB4; the regional map once the
// window holds s_min column pairs; unless the window is fixed, the AB4 guess
// evaluated too (unless the map is far ahead) and kept when its residual is
// strictly smaller, and on probe steps the map over the probed length
// evaluated as well (ebe_step then updates the window); kind 3: the learned
// candidate against the result.  The state is not modified.
GuessInfo guess_into(ebe_handle* h, const double* f_int, const double* g, bool allow_probe) {
    hipStream_t s = h->stream;
    GuessInfo info;
    info.n = h->it + 1;
    rhs_into(h, f_int, g, h->b);
    h->q_ready = false;
    int first0 = 0;
    const int s_eff0 = snapshot_window(h, info.n, &first0);
    info.probe = allow_probe && s_eff0 > 0 ? probe_length(h, info.n, s_eff0) : 0;
    info.s_eff = predict_into(h, h->x, &info.first, info.probe);
    if (info.s_eff > 0 && !h->cfg.fixed_window) {
        const int gr = res_grid(h->T.n_nodes);
        const int64_t nq = (int64_t)(3 * h->T.patch_nodes.size());
        double* part0 = h->cand_part;
        double* part1 = h->cand_part + gr;
        double* part_bb = h->cand_part + 2 * (size_t)gr;
        // the map's guess: its matvec (kept for the solve) and residual, and ||b||
        launch_ebe_apply(s, h->dp, h->x, true, h->cM, h->cK, h->qbuf);
        launch_cand_res(s, h->dn, h->qbuf, h->b, part0);
        launch_cand_res(s, h->dn, nullptr, h->b, part_bb);
        if (info.probe > 0) {
            launch_ebe_apply(s, h->dp, h->x_probe, true, h->cM, h->cK, h->qbuf_alt);
            launch_cand_res(s, h->dn, h->qbuf_alt, h->b, part1);
            launch_sum_partials(s, part1, gr, &h->sc->probe_rr);
        }
        const double thresh = (h->cfg.skip_ratio > 0 && h->ws.rho_ab > 0) ? h->cfg.skip_ratio * h->ws.rho_ab : 0.0;
        launch_guard_decide(s, part0, part_bb, gr, thresh, h->sc);
        // the AB4 guess, unless skipped on the device
        launch_ebe_apply(s, h->dp, h->dab, true, h->cM, h->cK, h->qbuf_alt, nullptr, h->sc);
        launch_cand_res(s, h->dn, h->qbuf_alt, h->b, part1, h->sc);
        launch_cand_select(s, h->dn, part0, part1, h->x, h->dab, h->qbuf, h->qbuf_alt, nq, h->sc, 1, h->sc);
        check_launch();
        h->q_ready = true;   // qbuf holds the kept guess's matvec: the solve skips its first one
        info.guarded = true;
    }
    info.learned = learned_due(h, info.n) && (h->cand_losses < kCandPatience || info.n % kCandProbe == 0);
    if (info.learned) choose_learned(h, f_int, g);
    return info;
}

// Trips saved per unit of log initial residual, in units of 1 / rate (the
// average per-trip decay of a solve): a guess lowers mostly the slowly
// converging components, so a lower initial residual saves about twice what
// the average decay suggests (64 x 64 x 32-cell mesh, steady state: s = 8 ->
// 16 lowers ln(res0) by 0.31 and saves 3.9 trips at rate 0.15).
constexpr double kTripGain = 2.0;

// Cost of one inner trip of the mixed-precision solve (FP32 matvec + update)
// in FP64 trips (64 x 64 x 32-cell mesh: (42.7 + 24.3) / (61.1 + 46.1) us), so
// that the decay rate, and with it the trips a probe saves, is per FP64-trip
// equivalent in every precision, the unit the column cost is measured in.
constexpr double kInnerTripCost = 0.62;

// Window state after step n from the scalars of its guess and solve (the rule
// of guess_into / ebe_predict's "Snapshot window").
void update_window(ebe_handle* h, const GuessInfo& info, const ebe_solve_stats& st) {
    ebe_window& W = h->ws;
    const ebe_config& c = h->cfg;
    const DevScalars& S = *h->sc_host;
    if (info.guarded) {
        const double bb = S.guess_bb;
        auto rel = [&](double rr) { return bb > 0 ? std::sqrt(rr / bb) : std::sqrt(rr); };
        const double rho_map = rel(S.guard_rr[0]);
        if (!c.fixed_window && c.col_cost >= 0 && info.s_eff == W.s_cap) {
            if (W.since + 1 >= c.probe_every) {
                if (info.probe > 0) {
                    const double rho_p = rel(S.probe_rr);
                    if (W.rate > 0 && rho_map > 0 && rho_p > 0) {
                        const double dtrips = kTripGain * std::log(rho_p / rho_map) / W.rate;
                        const double cols = c.col_cost * c.probe_step;
                        if (info.probe < W.s_cap ? dtrips < cols : -dtrips > cols) W.s_cap = info.probe;
                    }
                    W.grow_next = info.probe < info.s_eff ? 1 : 0;
                }
                W.since = 0;
            } else {
                W.since += 1;
            }
        }
        if (!S.guard_skip) {
            W.rho_ab = rel(S.guard_rr[1]);
            if (S.guard_pick) W.start = info.n;   // the AB4 guess beat the map: restart the window here
        }
    }
    const double trips = st.iters + (c.precision != EBE_PREC_FP64 ? kInnerTripCost * st.inner_iters : 0.0);
    if (trips > 0 && st.res0 > 0 && st.res_rec > 0) W.rate = std::log(st.res0 / st.res_rec) / trips;
}

void need_mlp(ebe_handle* h) {
    if (!h->mlp_w) {
        h->mlp_w = h->alloc<uint16_t>(kMlpParams);
        h->mlp_wm = h->alloc<float>(kMlpParams);
        h->mlp_m = h->alloc<float>(kMlpParams);
        h->mlp_v = h->alloc<float>(kMlpParams);
    }
    if (!h->flag) h->flag = h->alloc<int32_t>(1);
    if (!h->tr_loss) {
        h->tr_loss_cap = 1;
        h->tr_loss = h->alloc<double>(1);
    }
    h->tr.w = h->mlp_w;
    h->tr.wm = h->mlp_wm;
    h->tr.m = h->mlp_m;
    h->tr.v = h->mlp_v;
}

void need_train(ebe_handle* h, int B) {
    need_mlp(h);
    if (B > h->tr_cap) {
        MlpTrain& T = h->tr;
        for (void* q : {(void*)T.X, (void*)T.Z1, (void*)T.H1, (void*)T.Z2, (void*)T.H2, (void*)T.dY, (void*)T.dZ1,
                        (void*)T.dZ2, (void*)T.loss_part})
            h->release(q);
        const size_t b = (size_t)B;
        T.X = h->alloc<float>(kMlpIn * b);
        T.Z1 = h->alloc<float>(kMlpHid * b);
        T.H1 = h->alloc<float>(kMlpHid * b);
        T.Z2 = h->alloc<float>(kMlpHid * b);
        T.H2 = h->alloc<float>(kMlpHid * b);
        T.dY = h->alloc<float>(kMlpOut * b);
        T.dZ1 = h->alloc<float>(kMlpHid * b);
        T.dZ2 = h->alloc<float>(kMlpHid * b);
        T.loss_part = h->alloc<float>((b + 255) / 256);
        if (!T.grad) T.grad = h->alloc<float>(kMlpParams);
        h->tr_cap = B;
    }
}

void need_ready(const ebe_handle* h) {
    if (!h->mlp_ready) throw State{"no network weights: call ebe_mlp_set first"};
}

int32_t read_flag(ebe_handle* h) {
    int32_t f = 0;
    HIPCHK(hipMemcpyAsync(&f, h->flag, sizeof(f), hipMemcpyDeviceToHost, h->stream));
    sync_stream(h);
    return f;
}

}  // namespace

extern "C" {

const char* ebe_version(void) { return "ebe-ddpcg 0.2 (gfx950; FP64, mixed FP32/BF16 inner PCG)"; }

const char* ebe_last_error(const ebe_handle* h) { return h ? h->err.c_str() : g_create_error.c_str(); }

int ebe_create(const ebe_config* cfg, void* stream, ebe_handle** out) {
    g_create_error.clear();
    if (!cfg || !out) {
        g_create_error = "cfg and out must not be NULL";
        return EBE_E_INVALID_ARG;
    }
    *out = nullptr;
    ebe_config c = *cfg;
    if (!(c.dt > 0) || !(c.tol > 0) || c.s < 0 || c.s > 32 || c.predictor < 0 || c.predictor > 2 ||
        c.rayleigh_alpha < 0 || c.rayleigh_beta < 0 || c.patch_elems > kMaxPatchElems || c.precision < 0 ||
        c.precision > 2) {
        g_create_error = "invalid configuration (need dt > 0, tol > 0, 0 <= s <= 32, predictor in 0..2, "
                         "non-negative damping, patch_elems <= 256, precision in 0..2)";
        return EBE_E_INVALID_ARG;
    }
    if (c.max_iter <= 0) c.max_iter = 10000;
    // FP32 inner solves leave rounding noise of about 1e-5 of a snapshot's norm, which a
    // smaller threshold would fit as signal
    if (c.drop_tol <= 0) c.drop_tol = c.precision == EBE_PREC_FP64 ? 1e-6 : 1e-5;
    if (c.region_nodes <= 0) c.region_nodes = 512;
    if (c.patch_elems <= 0) c.patch_elems = kMaxPatchElems;
    if (c.inner_iters <= 0) c.inner_iters = 12;
    if (c.inner_tol <= 0) c.inner_tol = 1e-2;
    if (c.s_min <= 0) c.s_min = 3;
    if (c.probe_every <= 0) c.probe_every = 16;
    if (c.probe_step <= 0) c.probe_step = 8;
    if (c.skip_ratio == 0) c.skip_ratio = 0.01;
    if (c.col_cost == 0) c.col_cost = 0.08;
    ebe_handle* h = new (std::nothrow) ebe_handle();
    if (!h) {
        g_create_error = "out of memory";
        return EBE_E_NO_MEMORY;
    }
    h->cfg = c;
    h->stream = static_cast<hipStream_t>(stream);
    if (hipGetDevice(&h->device) != hipSuccess) {
        g_create_error = "no HIP device";
        delete h;
        return EBE_E_HIP;
    }
    if (hipError_t e = lookup_scratch(h->device); e != hipSuccess) {
        g_create_error = std::string("device address of the fixed scratch array: ") + hipGetErrorString(e);
        delete h;
        return EBE_E_HIP;
    }
    h->cM = 4.0 / (c.dt * c.dt) + 2.0 * c.rayleigh_alpha / c.dt;
    h->cK = 1.0 + 2.0 * c.rayleigh_beta / c.dt;
    *out = h;
    return EBE_OK;
}

int ebe_destroy(ebe_handle* h) {
    if (!h) return EBE_OK;
    (void)hipSetDevice(h->device);
    h->free_all();
    if (h->sc_host) (void)hipHostFree(h->sc_host);
    delete h;
    return EBE_OK;
}

int ebe_assemble(ebe_handle* h, int64_t n_nodes, const double* coords, int64_t n_elems, const int32_t* conn,
                 const int32_t* elem_mat, int32_t n_mat, const double* mat, const uint8_t* fixed,
                 const int32_t* region_of_node) {
    return guarded(h, [&]() -> int {
        need_ptr(coords, "coords");
        need_ptr(conn, "conn");
        need_ptr(elem_mat, "elem_mat");
        need_ptr(mat, "mat");
        need_ptr(fixed, "fixed");
        h->free_all();
        Topology& T = h->T;
        std::string e = build_topology(T, n_nodes, coords, n_elems, conn, elem_mat, n_mat, mat, fixed,
                                       region_of_node, h->cfg.region_nodes, h->cfg.patch_elems,
                                       ebe_patch_lds(n_mat), h->cfg.region_merge);
        if (!e.empty()) throw Arg{e};
        hipStream_t s = h->stream;
        const int64_t N = T.n_nodes, n3 = 3 * N;
        // topology
        h->dp.el_ptr = h->upload(T.patch_el_ptr);
        h->dp.pn_ptr = h->upload(T.patch_pn_ptr);
        h->dp.nv = h->upload(T.patch_nv);
        h->dp.nodes = h->upload(T.patch_nodes);
        h->dp.slot = h->upload(T.patch_slot);
        h->dp.elems = h->upload(T.elems);
        h->dp.coords = h->upload(T.coords);
        h->dp.mat = h->upload(T.mat_lmr);
        uint8_t* fm = h->upload(T.fixmask);
        h->dp.fixmask = fm;
        h->dp.n_patches_pad = T.n_patches_pad;
        h->dp.max_pn = T.max_pn;
        h->dp.max_nv = T.max_nv;
        h->dp.n_mat = n_mat;
        h->dn.slot_ptr = h->upload(T.slot_ptr);
        if (!ebe_set_lds_limit(h->dp)) throw Arg{"an element patch needs more LDS than the device allows; lower patch_elems"};
        h->dn.fixmask = fm;
        h->dn.n = N;
        h->d_i2u = h->upload(T.i2u);
        h->d_u2i = h->upload(T.u2i);
        h->chunks.n_regions = T.n_regions;
        h->chunks.n_chunks = (int32_t)T.chunk_region.size();
        h->chunks.start = h->upload(T.chunk_start);
        h->chunks.region = h->upload(T.chunk_region);
        h->chunks.first = h->upload(T.region_chunk);
        // buffers
        const size_t PN = T.patch_nodes.size();
        h->qbuf = h->alloc<double>(6 * PN);  // 6 entries per slot during setup, 3 afterwards
        h->binv6 = h->alloc<double>(6 * N);
        h->u = h->alloc<double>(n3);
        h->a = h->alloc<double>(n3);
        for (int k = 0; k < 4; ++k) h->vh[k] = h->alloc<double>(n3);
        h->ring = h->alloc<double>((size_t)(h->cfg.s + 1) * n3);
        h->dab = h->alloc<double>(n3);
        h->x = h->alloc<double>(n3);
        h->b = h->alloc<double>(n3);
        h->r = h->alloc<double>(n3);
        h->z = h->alloc<double>(n3);
        h->p[0] = h->alloc<double>(n3);
        h->p[1] = h->alloc<double>(n3);
        h->t0 = h->alloc<double>(n3);
        h->t1 = h->alloc<double>(n3);
        h->coef = h->alloc<double>(32 * (size_t)T.n_regions);
        h->gh = h->alloc<double>((size_t)kGhStride * T.chunk_region.size());
        h->sc = h->alloc<DevScalars>(1);
        h->pap_part = h->alloc<double>(pcg_ebe_grid(h->dp));
        h->cand_part = h->alloc<double>(3 * (size_t)res_grid(N));
        h->qbuf_alt = h->alloc<double>(3 * PN);
        h->coef_probe = h->alloc<double>(32 * (size_t)T.n_regions);
        h->x_probe = h->alloc<double>(n3);
        h->res_part = h->alloc<double>(2 * kResArrays * (size_t)res_grid(N));
        if (h->cfg.precision != EBE_PREC_FP64) {
            h->r_in = h->alloc<float>(n3);
            h->e_in = h->alloc<float>(n3);
            h->z_in = h->alloc<float>(n3);         // FP32 or BF16 storage (BF16 uses half)
            h->p_in[0] = h->alloc<float>(n3);
            h->p_in[1] = h->alloc<float>(n3);
            h->q_in = h->alloc<float>(3 * PN);
            h->binv_in = h->alloc<float>(6 * N);
            h->r_prev = h->alloc<double>(n3);
            h->sc_in = h->alloc<DevScalars>(1);
            h->pap_in = h->alloc<double>(pcg_ebe_grid(h->dp));
            h->res_in = h->alloc<double>(2 * kResArrays * (size_t)res_grid(N));
        }
        if (!h->sc_host) HIPCHK(hipHostMalloc((void**)&h->sc_host, sizeof(DevScalars), hipHostMallocDefault));
        HIPCHK(hipMemsetAsync(h->sc, 0, sizeof(DevScalars), s));
        // block-Jacobi inverse of A_bc
        launch_ebe_diag(s, h->dp, h->cM, h->cK, h->qbuf);
        launch_diag_finalize(s, h->dn, h->qbuf, h->binv6);
        if (h->binv_in) launch_to_f32(s, 6 * N, h->binv6, static_cast<float*>(h->binv_in));
        // row sums of M: the base-motion force of a node is -msum * g
        h->msum = h->alloc<double>(N);
        launch_fill(s, n3, 1.0, h->t0);
        launch_ebe_apply(s, h->dp, h->t0, false, 1.0, 0.0, h->qbuf);
        launch_msum(s, h->dn, h->qbuf, h->msum);
        // rest state
        launch_zero(s, n3, h->u);
        launch_zero(s, n3, h->a);
        for (int k = 0; k < 4; ++k) launch_zero(s, n3, h->vh[k]);
        launch_zero(s, (int64_t)(h->cfg.s + 1) * n3, h->ring);
        launch_zero(s, n3, h->p[0]);
        launch_zero(s, n3, h->p[1]);
        if (h->p_in[0]) {
            HIPCHK(hipMemsetAsync(h->p_in[0], 0, n3 * sizeof(float), s));
            HIPCHK(hipMemsetAsync(h->p_in[1], 0, n3 * sizeof(float), s));
            HIPCHK(hipMemsetAsync(h->sc_in, 0, sizeof(DevScalars), s));
        }
        check_launch();
        HIPCHK(hipStreamSynchronize(s));
        h->head = 0;
        h->it = 0;
        h->ws = ebe_window{1, h->cfg.s, 0, 0, 0.0, 0.0};
        h->par = 0;
        h->last_iters = 0;
        h->assembled = true;
        return EBE_OK;
    });
}

int ebe_get_regions(ebe_handle* h, int32_t* region_of_node, int32_t* n_regions) {
    return guarded(h, [&]() -> int {
        need_assembled(h);
        if (region_of_node) std::copy(h->T.region_user.begin(), h->T.region_user.end(), region_of_node);
        if (n_regions) *n_regions = h->T.n_regions;
        return EBE_OK;
    });
}

int ebe_apply(ebe_handle* h, const double* p, double* q) {
    return guarded(h, [&]() -> int {
        need_assembled(h);
        need_ptr(p, "p");
        need_ptr(q, "q");
        to_internal(h, p, h->t0);
        launch_ebe_apply(h->stream, h->dp, h->t0, true, h->cM, h->cK, h->qbuf);
        launch_combine_apply(h->stream, h->dn, h->qbuf, h->t0, 1, h->t1);
        to_user(h, h->t1, q);
        check_launch();
        return EBE_OK;
    });
}

int ebe_apply_mk(ebe_handle* h, double cm, double ck, const double* p, double* q) {
    return guarded(h, [&]() -> int {
        need_assembled(h);
        need_ptr(p, "p");
        need_ptr(q, "q");
        to_internal(h, p, h->t0);
        launch_ebe_apply(h->stream, h->dp, h->t0, false, cm, ck, h->qbuf);
        launch_combine_apply(h->stream, h->dn, h->qbuf, h->t0, 0, h->t1);
        to_user(h, h->t1, q);
        check_launch();
        return EBE_OK;
    });
}

int ebe_precond(ebe_handle* h, const double* r, double* z) {
    return guarded(h, [&]() -> int {
        need_assembled(h);
        need_ptr(r, "r");
        need_ptr(z, "z");
        to_internal(h, r, h->t0);
        launch_precond(h->stream, h->dn, h->binv6, h->t0, h->t1);
        to_user(h, h->t1, z);
        check_launch();
        return EBE_OK;
    });
}

int ebe_rhs(ebe_handle* h, const double* f_ext, const double* base_acc, double* b) {
    return guarded(h, [&]() -> int {
        need_assembled(h);
        need_ptr(b, "b");
        const double* f_int = nullptr;
        if (f_ext) {
            to_internal(h, f_ext, h->t0);
            f_int = h->t0;
        }
        rhs_into(h, f_int, base_acc, h->t1);
        to_user(h, h->t1, b);
        check_launch();
        return EBE_OK;
    });
}

int ebe_predict(ebe_handle* h, const double* f_next, const double* base_acc, double* dxbar, ebe_pred_stats* stats) {
    return guarded(h, [&]() -> int {
        need_assembled(h);
        need_ptr(dxbar, "dxbar");
        hipStream_t s = h->stream;
        const double* f_int = nullptr;
        if (f_next) {
            to_internal(h, f_next, h->t0);
            f_int = h->t0;
        }
        GuessInfo info = guess_into(h, f_int, base_acc, false);
        to_user(h, h->x, dxbar);
        if (stats) {
            const int gr = res_grid(h->T.n_nodes);
            if (!h->q_ready) launch_ebe_apply(s, h->dp, h->x, true, h->cM, h->cK, h->qbuf);
            launch_cand_res(s, h->dn, h->qbuf, h->b, h->cand_part);
            launch_sum_partials(s, h->cand_part, gr, &h->sc->guess_rr);
            launch_cand_res(s, h->dn, nullptr, h->b, h->cand_part);
            launch_sum_partials(s, h->cand_part, gr, &h->sc->guess_bb);
            check_launch();
            HIPCHK(hipMemcpyAsync(h->sc_host, h->sc, sizeof(DevScalars), hipMemcpyDeviceToHost, s));
            sync_stream(h);
            const DevScalars& S = *h->sc_host;
            const double bn = std::sqrt(S.guess_bb);
            auto rel = [&](double rr) { return bn > 0 ? std::sqrt(rr) / bn : std::sqrt(rr); };
            *stats = ebe_pred_stats{};
            stats->s_eff = info.s_eff;
            stats->first = info.first;
            stats->map_kept = info.guarded ? 1 - S.guard_pick : -1;
            stats->learned = info.learned ? S.cand_pick : -1;
            stats->res0 = rel(S.guess_rr);
            stats->bnorm = bn;
            if (info.guarded) {
                stats->res0_map = rel(S.guard_rr[0]);
                stats->res0_ab = S.guard_skip ? 0.0 : rel(S.guard_rr[1]);
            }
            if (info.learned) stats->res0_learned = rel(S.cand_rr[1]);
        }
        h->q_ready = false;
        check_launch();
        return EBE_OK;
    });
}

int ebe_refine(ebe_handle* h, const double* b, double* x, ebe_solve_stats* stats) {
    return guarded(h, [&]() -> int {
        need_assembled(h);
        need_ptr(b, "b");
        need_ptr(x, "x");
        to_internal(h, b, h->t0);
        to_internal(h, x, h->t1);
        check_launch();
        int rc = run_solve(h, h->t0, h->t1, stats);
        to_user(h, h->t1, x);
        check_launch();
        return rc;
    });
}

int ebe_step(ebe_handle* h, const double* f_ext, const double* base_acc, ebe_step_stats* stats) {
    return guarded(h, [&]() -> int {
        need_assembled(h);
        hipStream_t s = h->stream;
        const double* f_int = nullptr;
        if (f_ext) {
            to_internal(h, f_ext, h->t0);
            f_int = h->t0;
        }
        GuessInfo info = guess_into(h, f_int, base_acc, true);
        const int n = info.n;
        const bool collect = h->coll_k > 0 && n >= kLearnFirstStep && h->samples_n + h->coll_k <= h->samples_cap;
        if (collect) launch_collect_pre(s, h->coll_nodes, h->coll_k, h->dab, h->coll_stage);
        double* slot = h->cfg.s >= 1 ? h->ring_slot((n - 1) % (h->cfg.s + 1)) : nullptr;
        ebe_solve_stats st{};
        // without sample collection (which reads the state before the update) the
        // Newmark update is enqueued during the solve, guarded by the stop flag
        h->post_newmark = !collect;
        h->post_slot = slot;
        int rc;
        try {
            rc = run_solve(h, h->b, h->x, &st);
        } catch (...) {
            h->post_newmark = false;
            throw;
        }
        h->post_newmark = false;
        if (rc < 0) return rc;
        const DevScalars& S = *h->sc_host;
        if (info.learned) h->cand_losses = S.cand_pick ? 0 : h->cand_losses + 1;
        update_window(h, info, st);
        if (collect) {
            MlpState MS = mlp_state(h, f_int, base_acc);
            launch_collect_post(s, MS, h->coll_nodes, h->coll_k, h->x, h->coll_stage,
                                h->samples + h->samples_n * kMlpSample);
            h->samples_n += h->coll_k;
        }
        const int done = S.done;
        const bool updated = !collect && (done == DONE_CONVERGED || done == DONE_MAXITER);
        if (!updated) launch_newmark(s, h->n3(), h->cfg.dt, h->x, h->dab, h->u, h->vslot(0), h->vslot(3), h->a, slot);
        check_launch();
        h->head = (h->head + 3) & 3;
        h->it = n;
        if (stats) {
            *stats = ebe_step_stats{};
            stats->it = n;
            stats->s_eff = info.s_eff;
            stats->first = info.first;
            stats->iters = st.iters;
            stats->restarts = st.restarts;
            stats->inner_iters = st.inner_iters;
            stats->status = st.status;
            stats->res0 = st.res0;
            stats->res_rec = st.res_rec;
            stats->res_true = st.res_true;
            stats->bnorm = st.bnorm;
            auto rel = [&](double rr) { return st.bnorm > 0 ? std::sqrt(rr) / st.bnorm : 0.0; };
            stats->map_kept = info.guarded ? 1 - S.guard_pick : -1;
            if (info.guarded) {
                stats->skipped = S.guard_skip;
                stats->res0_map = rel(S.guard_rr[0]);
                stats->res0_ab = S.guard_skip ? 0.0 : rel(S.guard_rr[1]);
                stats->probe = info.probe;
                if (info.probe > 0) stats->res0_probe = rel(S.probe_rr);
            }
            stats->s_cap = h->ws.s_cap;
            stats->learned = info.learned ? S.cand_pick : -1;
            if (info.learned) {
                stats->res0_snapshot = rel(S.cand_rr[0]);
                stats->res0_learned = rel(S.cand_rr[1]);
            }
        }
        return rc;
    });
}

int ebe_get_state(ebe_handle* h, double* u, double* v, double* a) {
    return guarded(h, [&]() -> int {
        need_assembled(h);
        if (u) to_user(h, h->u, u);
        if (v) to_user(h, h->vslot(0), v);
        if (a) to_user(h, h->a, a);
        check_launch();
        return EBE_OK;
    });
}

int ebe_set_state(ebe_handle* h, const double* u, const double* v, const double* a) {
    return guarded(h, [&]() -> int {
        need_assembled(h);
        if (u) to_internal(h, u, h->u);
        if (v) to_internal(h, v, h->vslot(0));
        if (a) to_internal(h, a, h->a);
        check_launch();
        return EBE_OK;
    });
}

int ebe_get_history(ebe_handle* h, double* vhist, double* ring, int32_t* it, ebe_window* win) {
    return guarded(h, [&]() -> int {
        need_assembled(h);
        const int64_t n3 = h->n3();
        if (vhist)
            for (int j = 0; j < 4; ++j) to_user(h, h->vslot(j), vhist + j * n3);
        if (ring)
            for (int k = 0; k <= h->cfg.s; ++k) to_user(h, h->ring_slot(k), ring + k * n3);
        if (it) *it = h->it;
        if (win) *win = h->ws;
        check_launch();
        return EBE_OK;
    });
}

int ebe_set_history(ebe_handle* h, const double* vhist, const double* ring, int32_t it, const ebe_window* win) {
    return guarded(h, [&]() -> int {
        need_assembled(h);
        if (it < 0) throw Arg{"it must be non-negative"};
        ebe_window w = win ? *win : ebe_window{1, h->cfg.s, 0, 0, 0.0, 0.0};
        if (w.s_cap == 0) w.s_cap = h->cfg.s;
        if (w.start < 1 || w.s_cap < 1 || w.s_cap > std::max(1, h->cfg.s) || w.since < 0 || !(w.rho_ab >= 0) ||
            !(w.rate >= 0))
            throw Arg{"invalid window state (start >= 1, 1 <= s_cap <= s, since >= 0, rho_ab >= 0, rate >= 0)"};
        const int64_t n3 = h->n3();
        if (vhist)
            for (int j = 0; j < 4; ++j) to_internal(h, vhist + j * n3, h->vslot(j));
        if (ring)
            for (int k = 0; k <= h->cfg.s; ++k) to_internal(h, ring + k * n3, h->ring_slot(k));
        h->it = it;
        h->ws = w;
        check_launch();
        return EBE_OK;
    });
}

int ebe_sync(ebe_handle* h) {
    return guarded(h, [&]() -> int {
        sync_stream(h);
        return EBE_OK;
    });
}

int ebe_set_kernel_timing(ebe_handle* h, int32_t every_n) {
    return guarded(h, [&]() -> int {
        sync_stream(h);
        h->timing_every = every_n > 0 ? every_n : 0;
        h->time_sum_ms = 0.0;
        h->time_n = 0;
        h->pcg_launches = 0;
        return EBE_OK;
    });
}

int ebe_kernel_time(ebe_handle* h, int64_t* launches, double* mean_ms) {
    return guarded(h, [&]() -> int {
        sync_stream(h);
        if (launches) *launches = h->time_n;
        if (mean_ms) *mean_ms = h->time_n ? h->time_sum_ms / h->time_n : 0.0;
        return EBE_OK;
    });
}

int ebe_sizes(ebe_handle* h, int64_t* n_nodes, int64_t* n_elems, int64_t* n_patch_nodes, int64_t* n_patches) {
    return guarded(h, [&]() -> int {
        need_assembled(h);
        if (n_nodes) *n_nodes = h->T.n_nodes;
        if (n_elems) *n_elems = h->T.n_elems;
        if (n_patch_nodes) *n_patch_nodes = (int64_t)h->T.patch_nodes.size();
        if (n_patches) *n_patches = h->T.n_patches;
        return EBE_OK;
    });
}

int ebe_set_predictor(ebe_handle* h, int32_t kind) {
    return guarded(h, [&]() -> int {
        if (kind < EBE_PRED_ZERO || kind > EBE_PRED_LEARNED) throw Arg{"predictor kind must be 0..3"};
        h->cfg.predictor = kind;
        return EBE_OK;
    });
}

int ebe_reset(ebe_handle* h) {
    return guarded(h, [&]() -> int {
        need_assembled(h);
        hipStream_t s = h->stream;
        const int64_t n3 = h->n3();
        launch_zero(s, n3, h->u);
        launch_zero(s, n3, h->a);
        for (int k = 0; k < 4; ++k) launch_zero(s, n3, h->vh[k]);
        launch_zero(s, (int64_t)(h->cfg.s + 1) * n3, h->ring);
        check_launch();
        h->head = 0;
        h->it = 0;
        h->ws = ebe_window{1, h->cfg.s, 0, 0, 0.0, 0.0};
        h->last_iters = 0;
        h->cand_losses = 0;
        return EBE_OK;
    });
}

int ebe_mlp_set(ebe_handle* h, const float* params, const float* scales) {
    return guarded(h, [&]() -> int {
        need_assembled(h);
        need_ptr(params, "params");
        need_ptr(scales, "scales");
        for (int i = 0; i < kMlpParams; ++i)
            if (!std::isfinite(params[i])) throw Arg{"non-finite network parameter"};
        for (int i = 0; i < kMlpScales; ++i)
            if (!(scales[i] > 0.0f) || !std::isfinite(scales[i])) throw Arg{"scales must be positive and finite"};
        need_mlp(h);
        hipStream_t s = h->stream;
        HIPCHK(hipMemcpyAsync(h->mlp_wm, params, kMlpParams * sizeof(float), hipMemcpyHostToDevice, s));
        HIPCHK(hipMemsetAsync(h->mlp_m, 0, kMlpParams * sizeof(float), s));
        HIPCHK(hipMemsetAsync(h->mlp_v, 0, kMlpParams * sizeof(float), s));
        launch_mlp_round(s, h->mlp_wm, h->mlp_w);
        check_launch();
        sync_stream(h);
        std::copy(scales, scales + kMlpScales, h->mlp_scales);
        h->mlp_t = 0;
        h->mlp_ready = true;
        return EBE_OK;
    });
}

int ebe_mlp_get(ebe_handle* h, float* params, float* scales) {
    return guarded(h, [&]() -> int {
        need_ready(h);
        if (params) {
            HIPCHK(hipMemcpyAsync(params, h->mlp_wm, kMlpParams * sizeof(float), hipMemcpyDeviceToHost, h->stream));
            sync_stream(h);
        }
        if (scales) std::copy(h->mlp_scales, h->mlp_scales + kMlpScales, scales);
        return EBE_OK;
    });
}

int ebe_mlp_forward(ebe_handle* h, int64_t n, const float* x, float* y) {
    return guarded(h, [&]() -> int {
        need_ready(h);
        if (n < 0) throw Arg{"n must be non-negative"};
        if (n == 0) return EBE_OK;
        need_ptr(x, "x");
        need_ptr(y, "y");
        launch_mlp_infer_array(h->stream, h->mlp_w, n, x, y);
        check_launch();
        return EBE_OK;
    });
}

int ebe_mlp_grad(ebe_handle* h, int64_t n, const float* x, const float* t, float* grad, double* loss) {
    return guarded(h, [&]() -> int {
        need_ready(h);
        if (n < 1 || n > kMlpMaxBatch) throw Arg{"n must be in 1..8192"};
        need_ptr(x, "x");
        need_ptr(t, "t");
        need_ptr(grad, "grad");
        need_train(h, (int)n);
        MlpTrain T = h->tr;
        T.x_in = x;
        T.t_in = t;
        launch_mlp_grads(h->stream, T, (int)n, nullptr);
        HIPCHK(hipMemcpyAsync(grad, T.grad, kMlpParams * sizeof(float), hipMemcpyDeviceToDevice, h->stream));
        launch_mlp_loss(h->stream, T, (int)n, h->tr_loss);
        check_launch();
        double l = 0.0;
        HIPCHK(hipMemcpyAsync(&l, h->tr_loss, sizeof(double), hipMemcpyDeviceToHost, h->stream));
        sync_stream(h);
        if (loss) *loss = l;
        return EBE_OK;
    });
}

int ebe_mlp_grad_noalloc(ebe_handle* h, int64_t n, const float* x, const float* t, float* grad, double* loss) {
    return guarded(h, [&]() -> int {
        need_ready(h);
        if (n < 1 || n > kMlpMaxBatch) throw Arg{"n must be in 1..8192 (the fixed scratch array's capacity)"};
        need_ptr(x, "x");
        need_ptr(t, "t");
        need_ptr(grad, "grad");
        unsigned char* base = static_cast<unsigned char*>(scratch_ptr(h->device));
        if (!base) throw State{"no device address of the fixed scratch array on this device"};
        const size_t B = (size_t)n;
        float* act = reinterpret_cast<float*>(base + kScratchAct);
        MlpTrain T = h->tr;   // weights, master weights and moments of the handle; no training buffers
        T.x_in = x;
        T.t_in = t;
        T.X = act;
        T.Z1 = T.X + kMlpIn * B;
        T.H1 = T.Z1 + kMlpHid * B;
        T.Z2 = T.H1 + kMlpHid * B;
        T.H2 = T.Z2 + kMlpHid * B;
        T.dY = T.H2 + kMlpHid * B;
        T.dZ1 = T.dY + kMlpOut * B;
        T.dZ2 = T.dZ1 + kMlpHid * B;
        T.loss_part = reinterpret_cast<float*>(base + kScratchLossPart);
        T.grad = grad;        // every entry is written by the weight-gradient kernels
        launch_mlp_grads(h->stream, T, (int)n, nullptr);
        if (loss) {
            double* dloss = reinterpret_cast<double*>(base + kScratchLoss);
            launch_mlp_loss(h->stream, T, (int)n, dloss);
            check_launch();
            double l = 0.0;
            HIPCHK(hipMemcpyAsync(&l, dloss, sizeof(double), hipMemcpyDeviceToHost, h->stream));
            sync_stream(h);
            *loss = l;
        }
        check_launch();
        return EBE_OK;
    });
}

int ebe_mlp_adam(ebe_handle* h, const float* grad, float lr) {
    return guarded(h, [&]() -> int {
        need_ready(h);
        need_ptr(grad, "grad");
        if (!(lr > 0.0f) || !std::isfinite(lr)) throw Arg{"lr must be positive"};
        need_mlp(h);
        h->mlp_t += 1;
        launch_mlp_adam(h->stream, h->tr, grad, lr, h->mlp_t, 0, nullptr, 0);
        check_launch();
        return EBE_OK;
    });
}

int ebe_collect(ebe_handle* h, int64_t capacity, const int32_t* nodes, int32_t k) {
    return guarded(h, [&]() -> int {
        need_assembled(h);
        if (!nodes || k == 0) {
            h->coll_k = 0;
            return EBE_OK;
        }
        if (k < 0 || k > h->T.n_nodes) throw Arg{"k must be in 0..n_nodes"};
        if (capacity < k) throw Arg{"capacity must hold at least one step of samples"};
        need_mlp(h);
        hipStream_t s = h->stream;
        if (capacity != h->samples_cap) {
            h->release(h->samples);
            h->samples = h->alloc<float>((size_t)capacity * kMlpSample);
            h->samples_cap = capacity;
            h->samples_n = 0;
        }
        if (k > h->coll_cap_k) {
            h->release(h->coll_nodes);
            h->release(h->coll_stage);
            h->coll_nodes = h->alloc<int32_t>(k);
            h->coll_stage = h->alloc<double>(3 * (size_t)k);
            h->coll_cap_k = k;
        }
        launch_map_nodes(s, nodes, k, h->d_u2i, h->T.n_nodes, h->coll_nodes, h->flag);
        check_launch();
        if (read_flag(h)) throw Arg{"node id out of range"};
        h->coll_k = k;
        return EBE_OK;
    });
}

int ebe_samples(ebe_handle* h, int64_t* count, float* dst) {
    return guarded(h, [&]() -> int {
        need_assembled(h);
        if (count) *count = h->samples_n;
        if (dst && h->samples_n > 0) {
            HIPCHK(hipMemcpyAsync(dst, h->samples, (size_t)h->samples_n * kMlpSample * sizeof(float),
                                  hipMemcpyDeviceToDevice, h->stream));
            check_launch();
        }
        return EBE_OK;
    });
}

int ebe_mlp_fit_scales(ebe_handle* h, float* scales) {
    return guarded(h, [&]() -> int {
        need_assembled(h);
        if (h->samples_n < 1) throw State{"no samples collected"};
        if (!h->rms3) h->rms3 = h->alloc<double>(kMlpScales);
        launch_sample_rms(h->stream, h->samples, h->samples_n, h->rms3);
        check_launch();
        double r[kMlpScales];
        HIPCHK(hipMemcpyAsync(r, h->rms3, sizeof(r), hipMemcpyDeviceToHost, h->stream));
        sync_stream(h);
        for (int i = 0; i < kMlpScales; ++i) {
            if (!std::isfinite(r[i])) throw Arg{"non-finite samples"};
            h->mlp_scales[i] = r[i] > 0.0 ? (float)r[i] : 1.0f;
        }
        if (scales) std::copy(h->mlp_scales, h->mlp_scales + kMlpScales, scales);
        return EBE_OK;
    });
}

int ebe_mlp_train(ebe_handle* h, int32_t steps, int32_t batch, const int64_t* idx, float lr, double* loss) {
    return guarded(h, [&]() -> int {
        need_ready(h);
        if (steps < 0) throw Arg{"steps must be non-negative"};
        if (batch < 1 || batch > kMlpMaxBatch) throw Arg{"batch must be in 1..8192"};
        if (!(lr > 0.0f) || !std::isfinite(lr)) throw Arg{"lr must be positive"};
        if (steps == 0) return EBE_OK;
        need_ptr(idx, "idx");
        if (h->samples_n < 1) throw State{"no samples collected"};
        need_train(h, batch);
        hipStream_t s = h->stream;
        launch_check_index(s, idx, (int64_t)steps * batch, h->samples_n, h->flag);
        check_launch();
        if (read_flag(h)) throw Arg{"sample index out of range"};
        if (steps > h->tr_loss_cap) {
            h->release(h->tr_loss);
            h->tr_loss = h->alloc<double>(steps);
            h->tr_loss_cap = steps;
        }
        MlpTrain T = h->tr;
        T.samples = h->samples;
        T.n_samples = h->samples_n;
        for (int g = 0; g < 3; ++g) T.inv_s[g] = 1.0f / h->mlp_scales[g];
        T.inv_st = 1.0f / h->mlp_scales[3];
        for (int k = 0; k < steps; ++k) {
            launch_mlp_grads(s, T, batch, idx + (int64_t)k * batch);
            h->mlp_t += 1;
            launch_mlp_adam(s, T, T.grad, lr, h->mlp_t, batch, h->tr_loss, k);
        }
        check_launch();
        if (loss) {
            HIPCHK(hipMemcpyAsync(loss, h->tr_loss, steps * sizeof(double), hipMemcpyDeviceToHost, s));
        }
        sync_stream(h);
        return EBE_OK;
    });
}

int ebe_get_config(ebe_handle* h, ebe_config* out) {
    return guarded(h, [&]() -> int {
        need_ptr(out, "out");
        *out = h->cfg;
        return EBE_OK;
    });
}

}  // extern "C"
