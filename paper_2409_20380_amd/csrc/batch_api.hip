// batch_api.hip -- C ABI of batched ensembles (declared in include/ebe.h):
// many cases, each its own input wave, on one or more meshes, advanced one
// time step together.  Per step: right-hand sides of all cases (one batched
// element pass per mesh), Adams-Bashforth 4 and the regional snapshot map
// over the stacked vectors (the regions of every case are independent least
// squares problems), Algorithm 1 for every case with shared element passes,
// Newmark.  A chunk of PCG trips for all meshes is captured once in a
// hipGraph and replayed; the host reads the per-case scalars once per check.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "../../include/ebe.h"
#include "element.h"
#include "kernels.h"
#include "topology.h"

using namespace ebe;

namespace {

struct BErr {
    int code;
    std::string msg;
};

#define BCHK(expr)                                                                                        \
    do {                                                                                                  \
        hipError_t _e = (expr);                                                                           \
        if (_e != hipSuccess) throw BErr{EBE_E_HIP, std::string(#expr) + ": " + hipGetErrorString(_e)}; \
    } while (0)

thread_local std::string g_batch_create_error;

// Allocation list with individual release (tuning candidates are dropped).
struct Allocs {
    std::vector<void*> v;
    Allocs() = default;
    Allocs(const Allocs&) = delete;
    Allocs& operator=(const Allocs&) = delete;
    Allocs(Allocs&& o) noexcept : v(std::move(o.v)) { o.v.clear(); }
    Allocs& operator=(Allocs&& o) noexcept {
        free_all();
        v = std::move(o.v);
        o.v.clear();
        return *this;
    }
    ~Allocs() { free_all(); }
    template <class X>
    X* alloc(size_t count) {
        void* p = nullptr;
        if (count == 0) count = 1;
        if (hipMalloc(&p, count * sizeof(X)) != hipSuccess) throw BErr{EBE_E_NO_MEMORY, "device allocation failed"};
        v.push_back(p);
        return static_cast<X*>(p);
    }
    void free_all() {
        for (void* p : v) (void)hipFree(p);
        v.clear();
    }
};

struct MeshIn {
    int64_t n_nodes = 0, n_elems = 0;
    int32_t n_mat = 0, r = 0;
    std::vector<double> coords, mat;
    std::vector<int32_t> conn, elem_mat, regions;
    std::vector<uint8_t> fixed;
    bool has_regions = false;
    int ct_fixed = 0, chunks_fixed = 0;   // from ebe_batch_set_group_config (0: tune or default)
};

// One mesh with r cases: topology for the chosen case tile and launch shape.
struct Group {
    Topology T;
    Allocs topo;            // device topology of the chosen configuration
    DevPatches dp{};
    DevNodes dn{};
    int r = 0, ct = 1, chunks = 8, g_upd = 1;
    int case0 = 0;
    int64_t N = 0, PN = 0;
    int64_t dof_off = 0;    // doubles: case 0's vector in the stacked arrays
    int64_t slot_off = 0;   // doubles: case 0's slots in qbuf
    int32_t *d_i2u = nullptr, *d_u2i = nullptr;
    double* binv6 = nullptr;
    double* part = nullptr;  // update partials [2][kResArrays][r][g_upd]
    double* pap = nullptr;   // (p, A p) partials [r][chunks]
    double* cand = nullptr;  // guarded window: residual partials of the two guesses [2][r][g_upd]
};

}  // namespace

struct ebe_batch {
    ebe_config cfg{};
    hipStream_t stream = nullptr;
    int device = 0;
    std::string err;
    std::vector<MeshIn> meshes;
    std::vector<Group> groups;
    bool assembled = false;
    double cM = 0, cK = 0;
    int C = 0;
    int64_t n3 = 0, slots = 0, nodes = 0;
    Allocs mem;
    double *u = nullptr, *a = nullptr, *vh[4] = {nullptr, nullptr, nullptr, nullptr}, *ring = nullptr;
    double *dab = nullptr, *x = nullptr, *b = nullptr, *r = nullptr, *z = nullptr, *p[2] = {nullptr, nullptr};
    double *qbuf = nullptr, *t0 = nullptr, *t1 = nullptr, *coef = nullptr, *gh = nullptr, *g_dev = nullptr;
    double* g_host = nullptr;
    DevScalars* sc = nullptr;
    DevScalars* sc_host = nullptr;
    int* trip = nullptr;
    DevChunks chunks{};
    int head = 0, it = 0, par = 0, last_iters = 0;
    std::vector<int> win;          // per case: first step whose AB error may enter its snapshot window
    int32_t* lo_dev = nullptr;     // per case: first window column its regions use
    int32_t* lo_host = nullptr;    // pinned staging of lo_dev
    bool use_graph = true;
    int graph_trips = 8;
    hipGraph_t graph = nullptr;
    hipGraphExec_t gexec = nullptr;
    int graph_par = -1;
    hipStream_t cap_stream = nullptr;   // private stream the chunk graph is captured on

    double* vslot(int j) const { return vh[(head + j) & 3]; }
    double* ring_slot(int k) const { return ring + (int64_t)k * n3; }
    void drop_graph() {
        if (gexec) (void)hipGraphExecDestroy(gexec);
        if (graph) (void)hipGraphDestroy(graph);
        gexec = nullptr;
        graph = nullptr;
        graph_par = -1;
    }
    void release() {
        if (stream) (void)hipStreamSynchronize(stream);
        drop_graph();
        for (auto& g : groups) g.topo.free_all();
        groups.clear();
        mem.free_all();
        assembled = false;
    }
};

namespace {

template <class F>
int bguard(ebe_batch* b, F&& f) {
    if (!b) return EBE_E_INVALID_ARG;
    b->err.clear();
    try {
        BCHK(hipSetDevice(b->device));
        return f();
    } catch (const BErr& e) {
        b->err = e.msg;
        return e.code;
    } catch (const std::bad_alloc&) {
        b->err = "out of host memory";
        return EBE_E_NO_MEMORY;
    } catch (...) {
        b->err = "unexpected error";
        return EBE_E_HIP;
    }
}

void need_asm(const ebe_batch* b) {
    if (!b->assembled) throw BErr{EBE_E_BAD_STATE, "call ebe_batch_assemble first"};
}

void check_launch() { BCHK(hipGetLastError()); }

// Device topology of one configuration into a.
void upload_topology(Group& g, Allocs& a, hipStream_t s) {
    auto up = [&](const auto& v) {
        using X = typename std::decay_t<decltype(v)>::value_type;
        X* d = a.alloc<X>(v.size());
        if (!v.empty()) BCHK(hipMemcpyAsync(d, v.data(), v.size() * sizeof(X), hipMemcpyHostToDevice, s));
        return d;
    };
    const Topology& T = g.T;
    g.dp.el_ptr = up(T.patch_el_ptr);
    g.dp.pn_ptr = up(T.patch_pn_ptr);
    g.dp.nv = up(T.patch_nv);
    g.dp.nodes = up(T.patch_nodes);
    g.dp.slot = up(T.patch_slot);
    g.dp.elems = up(T.elems);
    g.dp.coords = up(T.coords);
    g.dp.mat = up(T.mat_lmr);
    uint8_t* fm = up(T.fixmask);
    g.dp.fixmask = fm;
    g.dp.n_patches_pad = T.n_patches_pad;
    g.dp.max_pn = T.max_pn;
    g.dp.max_nv = T.max_nv;
    g.dp.n_mat = (int32_t)(T.mat_lmr.size() / 3);
    g.dn.slot_ptr = up(T.slot_ptr);
    g.dn.fixmask = fm;
    g.dn.n = T.n_nodes;
    g.d_i2u = up(T.i2u);
    g.d_u2i = up(T.u2i);
    g.N = T.n_nodes;
    g.PN = (int64_t)T.patch_nodes.size();
}

void build_group_topology(ebe_batch* b, const MeshIn& m, Topology& T, int ct) {
    std::string e = build_topology(T, m.n_nodes, m.coords.data(), m.n_elems, m.conn.data(), m.elem_mat.data(),
                                   m.n_mat, m.mat.data(), m.fixed.data(), m.has_regions ? m.regions.data() : nullptr,
                                   b->cfg.region_nodes, kMaxPatchElems / ct, PatchLds(), b->cfg.region_merge);
    if (!e.empty()) throw BErr{EBE_E_INVALID_ARG, e};
}

int default_ct(int r) {
    int ct = 1;
    while (ct * 2 <= std::min(r, 4)) ct *= 2;
    return ct;
}

int clamp_chunks(const Group& g, int chunks) {
    int c = std::min(chunks, std::min(g.dp.n_patches_pad, kMaxPcgGrid));
    c = std::max(8, c - c % 8);
    return c;
}

int g_upd_for(int64_t n) { return (int)std::max<int64_t>(1, std::min<int64_t>(256, (n + 2047) / 2048)); }

BEbeArgs ebe_args(const ebe_batch* b, const Group& g) {
    BEbeArgs A{};
    A.P = g.dp;
    A.r = g.r;
    A.n3 = 3 * g.N;
    A.pn = g.PN;
    A.qbuf = b->qbuf + g.slot_off;
    A.cm = b->cM;
    A.ck = b->cK;
    A.sc = b->sc + g.case0;
    A.upd_part = g.part;
    A.g_upd = g.g_upd;
    A.pap_part = g.pap;
    A.trip = b->trip;
    A.max_iter = b->cfg.max_iter;
    A.tol = b->cfg.tol;
    return A;
}

BNodeArgs node_args(const ebe_batch* b, const Group& g) {
    BNodeArgs A{};
    A.N = g.dn;
    A.r = g.r;
    A.pn = g.PN;
    A.qbuf = b->qbuf + g.slot_off;
    A.b = b->b + g.dof_off;
    A.binv6 = g.binv6;
    A.x = b->x + g.dof_off;
    A.r_ = b->r + g.dof_off;
    A.z = b->z + g.dof_off;
    A.sc = b->sc + g.case0;
    A.pap_part = g.pap;
    A.g_pap = g.chunks;
    A.part = g.part;
    A.g_upd = g.g_upd;
    A.trip = b->trip;
    return A;
}

// Mean duration (ms) of the PCG-shaped element pass of one configuration.
double time_config(ebe_batch* b, Group& g, int ct, int chunks, double* p, double* q) {
    hipStream_t s = b->stream;
    BEbeArgs A{};
    A.P = g.dp;
    A.r = g.r;
    A.n3 = 3 * g.N;
    A.pn = g.PN;
    A.in0 = p;
    A.qbuf = q;
    A.cm = b->cM;
    A.ck = b->cK;
    A.mask_in = 1;
    hipEvent_t e0, e1;
    BCHK(hipEventCreate(&e0));
    BCHK(hipEventCreate(&e1));
    for (int k = 0; k < 2; ++k) launch_bebe(s, MODE_APPLY, A, ct, chunks);
    BCHK(hipEventRecord(e0, s));
    const int reps = 5;
    for (int k = 0; k < reps; ++k) launch_bebe(s, MODE_APPLY, A, ct, chunks);
    BCHK(hipEventRecord(e1, s));
    check_launch();
    BCHK(hipEventSynchronize(e1));
    float ms = 0.f;
    BCHK(hipEventElapsedTime(&ms, e0, e1));
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    return ms / reps;
}

// Choose (case tile, grid) of a group by timing its element pass.
void tune_group(ebe_batch* b, Group& g, const MeshIn& m, bool tune) {
    hipStream_t s = b->stream;
    if (!tune) {
        build_group_topology(b, m, g.T, g.ct);
        upload_topology(g, g.topo, s);
        if (!bebe_set_lds_limit(g.dp, g.ct)) throw BErr{EBE_E_INVALID_ARG, "element patch too large for LDS"};
        g.chunks = clamp_chunks(g, g.chunks);
        return;
    }
    double best = 1e300;
    int best_ct = 0, best_chunks = 0;
    for (int ct = 1; ct <= kMaxCaseTile; ct *= 2) {
        if (ct > 1 && ct / 2 >= g.r) break;   // a tile wider than the case count only idles lanes
        Group cand;
        cand.r = g.r;
        build_group_topology(b, m, cand.T, ct);
        Allocs tmp;
        upload_topology(cand, tmp, s);
        if (!bebe_set_lds_limit(cand.dp, ct)) {
            BCHK(hipStreamSynchronize(s));
            tmp.free_all();
            continue;
        }
        double* p = tmp.alloc<double>((size_t)g.r * 3 * cand.N);
        double* q = tmp.alloc<double>((size_t)g.r * 3 * cand.PN);
        BCHK(hipMemsetAsync(p, 0, (size_t)g.r * 3 * cand.N * sizeof(double), s));
        for (int chunks : {64, 128, 256, 512}) {
            const int c = clamp_chunks(cand, chunks);
            if (c != chunks && chunks != 64) continue;
            const double ms = time_config(b, cand, ct, c, p, q);
            if (ms < best) {
                best = ms;
                best_ct = ct;
                best_chunks = c;
            }
        }
        BCHK(hipStreamSynchronize(s));
        tmp.free_all();
    }
    if (!best_ct) throw BErr{EBE_E_INVALID_ARG, "no element patch configuration fits in LDS"};
    g.ct = best_ct;
    build_group_topology(b, m, g.T, g.ct);
    upload_topology(g, g.topo, s);
    (void)bebe_set_lds_limit(g.dp, g.ct);
    g.chunks = best_chunks;
}

void enqueue_trips(ebe_batch* b, int trips, hipStream_t s) {
    for (int t = 0; t < trips; ++t) {
        const int par = (b->par + t) & 1;
        for (auto& g : b->groups) {
            BEbeArgs A = ebe_args(b, g);
            A.in0 = b->z + g.dof_off;
            A.in1 = b->p[par] + g.dof_off;
            A.p_cur = b->p[par ^ 1] + g.dof_off;
            launch_bebe(s, MODE_PCG, A, g.ct, g.chunks);
        }
        for (auto& g : b->groups) {
            BNodeArgs A = node_args(b, g);
            A.p = b->p[par ^ 1] + g.dof_off;
            launch_bupdate(s, A);
        }
        launch_trip_inc(s, b->trip);
    }
}

// A chunk of trips: replayed from the captured graph when graphs are on.
// The direction buffers alternate with the trip parity, so the graph holds an
// even number of trips and always starts at parity 0.  The graph is captured
// on a private stream (the caller's stream may be the null stream, which
// cannot be captured) and launched on the caller's stream.
void run_chunk(ebe_batch* b) {
    hipStream_t s = b->stream;
    if (!b->use_graph) {
        enqueue_trips(b, b->graph_trips, s);
        b->par = (b->par + b->graph_trips) & 1;
        return;
    }
    if (!b->gexec) {
        if (!b->cap_stream) BCHK(hipStreamCreateWithFlags(&b->cap_stream, hipStreamNonBlocking));
        BCHK(hipStreamBeginCapture(b->cap_stream, hipStreamCaptureModeThreadLocal));
        enqueue_trips(b, b->graph_trips, b->cap_stream);
        hipGraph_t gr = nullptr;
        hipError_t e = hipStreamEndCapture(b->cap_stream, &gr);
        if (e != hipSuccess) throw BErr{EBE_E_HIP, std::string("graph capture: ") + hipGetErrorString(e)};
        b->graph = gr;
        BCHK(hipGraphInstantiate(&b->gexec, gr, nullptr, nullptr, 0));
    }
    BCHK(hipGraphLaunch(b->gexec, s));
}

bool case_finished(const DevScalars& S) {
    if (S.done == DONE_RUNNING) return false;
    if (S.done == DONE_CONVERGED || S.done == DONE_MAXITER) return S.checked != 0;
    return true;
}

int solve_batch(ebe_batch* b) {
    hipStream_t s = b->stream;
    launch_set_trip(s, b->trip, 0);
    b->par = 0;
    for (auto& g : b->groups) {
        BEbeArgs A = ebe_args(b, g);
        A.in0 = b->x + g.dof_off;
        A.mask_in = 1;
        launch_bebe(s, MODE_APPLY, A, g.ct, g.chunks);
        launch_bresidual(s, node_args(b, g), 0);
    }
    check_launch();
    // chunks before the first read: enough for the previous step's slowest case
    int before = std::max(1, (b->last_iters - 1) / b->graph_trips);
    int worst = 0;
    for (int round = 0;; ++round) {
        const int n = round == 0 ? before : 1;
        for (int k = 0; k < n; ++k) run_chunk(b);
        for (auto& g : b->groups) {
            BEbeArgs A = ebe_args(b, g);
            A.in0 = b->x + g.dof_off;
            A.mask_in = 1;
            A.guard = b->sc + g.case0;
            launch_bebe(s, MODE_APPLY, A, g.ct, g.chunks);
            BNodeArgs N = node_args(b, g);
            launch_bresidual(s, N, 1);
            launch_bcheck_finalize(s, N, b->cfg.tol);
        }
        check_launch();
        BCHK(hipMemcpyAsync(b->sc_host, b->sc, b->C * sizeof(DevScalars), hipMemcpyDeviceToHost, s));
        BCHK(hipStreamSynchronize(s));
        bool all = true;
        worst = 0;
        for (int c = 0; c < b->C; ++c) {
            all = all && case_finished(b->sc_host[c]);
            worst = std::max(worst, b->sc_host[c].iters);
        }
        if (all) break;
        if (round > 200000) throw BErr{EBE_E_HIP, "batched PCG loop did not terminate"};
    }
    for (auto& g : b->groups) launch_bzero_rhs_cases(s, b->sc + g.case0, g.r, 3 * g.N, b->x + g.dof_off);
    check_launch();
    b->last_iters = worst;
    int rc = EBE_OK;
    for (int c = 0; c < b->C; ++c) {
        if (b->sc_host[c].done == DONE_NONFINITE) return EBE_E_NONFINITE;
        if (b->sc_host[c].done == DONE_MAXITER) rc = EBE_NOT_CONVERGED;
    }
    return rc;
}

}  // namespace

extern "C" {

int ebe_batch_create(const ebe_config* cfg, void* stream, ebe_batch** out) {
    g_batch_create_error.clear();
    if (!cfg || !out) {
        g_batch_create_error = "null argument";
        return EBE_E_INVALID_ARG;
    }
    *out = nullptr;
    ebe_config c = *cfg;
    if (c.max_iter <= 0) c.max_iter = 10000;
    if (c.drop_tol <= 0) c.drop_tol = 1e-6;
    if (c.region_nodes <= 0) c.region_nodes = 512;
    if (c.s_min <= 0) c.s_min = 3;
    if (!(c.dt > 0) || !(c.tol > 0) || c.s < 0 || c.s > kMaxCols - 1 || c.predictor < 0 || c.predictor > 2 ||
        c.rayleigh_alpha < 0 || c.rayleigh_beta < 0 || c.precision != EBE_PREC_FP64) {
        g_batch_create_error = "invalid configuration (need dt > 0, tol > 0, 0 <= s <= 32, predictor 0..2, FP64)";
        return EBE_E_INVALID_ARG;
    }
    ebe_batch* b = new (std::nothrow) ebe_batch();
    if (!b) return EBE_E_NO_MEMORY;
    b->cfg = c;
    b->stream = static_cast<hipStream_t>(stream);
    if (hipGetDevice(&b->device) != hipSuccess) {
        delete b;
        g_batch_create_error = "no HIP device";
        return EBE_E_HIP;
    }
    b->cM = 4.0 / (c.dt * c.dt) + 2.0 * c.rayleigh_alpha / c.dt;
    b->cK = 1.0 + 2.0 * c.rayleigh_beta / c.dt;
    *out = b;
    return EBE_OK;
}

int ebe_batch_destroy(ebe_batch* b) {
    if (!b) return EBE_OK;
    (void)hipSetDevice(b->device);
    b->release();
    if (b->sc_host) (void)hipHostFree(b->sc_host);
    if (b->g_host) (void)hipHostFree(b->g_host);
    if (b->lo_host) (void)hipHostFree(b->lo_host);
    if (b->cap_stream) (void)hipStreamDestroy(b->cap_stream);
    delete b;
    return EBE_OK;
}

const char* ebe_batch_last_error(const ebe_batch* b) { return b ? b->err.c_str() : g_batch_create_error.c_str(); }

int ebe_batch_add_mesh(ebe_batch* b, int64_t n_nodes, const double* coords, int64_t n_elems, const int32_t* conn,
                       const int32_t* elem_mat, int32_t n_mat, const double* mat, const uint8_t* fixed,
                       const int32_t* region_of_node, int32_t n_cases, int32_t* group) {
    return bguard(b, [&]() -> int {
        if (!coords || !conn || !elem_mat || !mat || !fixed) throw BErr{EBE_E_INVALID_ARG, "null mesh array"};
        if (n_nodes < 1 || n_elems < 1 || n_mat < 1) throw BErr{EBE_E_INVALID_ARG, "empty mesh"};
        if (n_cases < 1) throw BErr{EBE_E_INVALID_ARG, "n_cases must be >= 1"};
        MeshIn m;
        m.n_nodes = n_nodes;
        m.n_elems = n_elems;
        m.n_mat = n_mat;
        m.r = n_cases;
        m.coords.assign(coords, coords + 3 * n_nodes);
        m.conn.assign(conn, conn + 10 * n_elems);
        m.elem_mat.assign(elem_mat, elem_mat + n_elems);
        m.mat.assign(mat, mat + 3 * n_mat);
        m.fixed.assign(fixed, fixed + 3 * n_nodes);
        if (region_of_node) {
            m.regions.assign(region_of_node, region_of_node + n_nodes);
            m.has_regions = true;
        }
        b->meshes.push_back(std::move(m));
        b->release();
        if (group) *group = (int32_t)b->meshes.size() - 1;
        return EBE_OK;
    });
}

int ebe_batch_set_group_config(ebe_batch* b, int32_t group, int32_t case_tile, int32_t chunks) {
    return bguard(b, [&]() -> int {
        if (group < 0 || group >= (int)b->meshes.size()) throw BErr{EBE_E_INVALID_ARG, "no such group"};
        if (case_tile != 1 && case_tile != 2 && case_tile != 4 && case_tile != 8)
            throw BErr{EBE_E_INVALID_ARG, "case_tile must be 1, 2, 4 or 8"};
        if (chunks < 8 || chunks > kMaxPcgGrid || chunks % 8) throw BErr{EBE_E_INVALID_ARG, "chunks: multiple of 8 in 8..512"};
        // takes effect at the next ebe_batch_assemble
        b->meshes[group].ct_fixed = case_tile;
        b->meshes[group].chunks_fixed = chunks;
        return EBE_OK;
    });
}

int ebe_batch_assemble(ebe_batch* b, int32_t tune) {
    return bguard(b, [&]() -> int {
        if (b->meshes.empty()) throw BErr{EBE_E_BAD_STATE, "no mesh added"};
        b->release();
        hipStream_t s = b->stream;
        b->groups.resize(b->meshes.size());
        int case0 = 0;
        int64_t dof = 0, slot = 0, nodes = 0;
        for (size_t i = 0; i < b->meshes.size(); ++i) {
            const MeshIn& m = b->meshes[i];
            Group& g = b->groups[i];
            g.r = m.r;
            g.ct = m.ct_fixed ? m.ct_fixed : default_ct(m.r);
            g.chunks = m.chunks_fixed ? m.chunks_fixed : 256;
            tune_group(b, g, m, tune != 0 && !m.ct_fixed);
            g.case0 = case0;
            g.dof_off = dof;
            g.slot_off = slot;
            g.g_upd = g_upd_for(g.N);
            case0 += g.r;
            dof += (int64_t)g.r * 3 * g.N;
            slot += (int64_t)g.r * 3 * g.PN;
            nodes += (int64_t)g.r * g.N;
        }
        b->C = case0;
        b->n3 = dof;
        b->slots = slot;
        b->nodes = nodes;
        Allocs& M = b->mem;
        b->u = M.alloc<double>(dof);
        b->a = M.alloc<double>(dof);
        for (int k = 0; k < 4; ++k) b->vh[k] = M.alloc<double>(dof);
        b->ring = M.alloc<double>((size_t)(b->cfg.s + 1) * dof);
        b->dab = M.alloc<double>(dof);
        b->x = M.alloc<double>(dof);
        b->b = M.alloc<double>(dof);
        b->r = M.alloc<double>(dof);
        b->z = M.alloc<double>(dof);
        b->p[0] = M.alloc<double>(dof);
        b->p[1] = M.alloc<double>(dof);
        b->t0 = M.alloc<double>(dof);
        b->t1 = M.alloc<double>(dof);
        b->qbuf = M.alloc<double>(std::max<int64_t>(slot, 1));
        b->sc = M.alloc<DevScalars>(b->C);
        b->trip = M.alloc<int>(1);
        b->g_dev = M.alloc<double>(3 * (size_t)b->C);
        if (b->sc_host) (void)hipHostFree(b->sc_host);
        if (b->g_host) (void)hipHostFree(b->g_host);
        if (b->lo_host) (void)hipHostFree(b->lo_host);
        b->sc_host = nullptr;
        b->g_host = nullptr;
        b->lo_host = nullptr;
        BCHK(hipHostMalloc((void**)&b->sc_host, b->C * sizeof(DevScalars), hipHostMallocDefault));
        BCHK(hipHostMalloc((void**)&b->g_host, 3 * b->C * sizeof(double), hipHostMallocDefault));
        BCHK(hipHostMalloc((void**)&b->lo_host, b->C * sizeof(int32_t), hipHostMallocDefault));
        b->lo_dev = M.alloc<int32_t>(b->C);
        b->win.assign(b->C, 1);
        BCHK(hipMemsetAsync(b->sc, 0, b->C * sizeof(DevScalars), s));
        // regions of every case of every group, in stacked node order, cut into
        // node chunks (the host vectors live until the stream is synchronised below)
        if (nodes > INT32_MAX) throw BErr{EBE_E_INVALID_ARG, "batch too large"};
        std::vector<int32_t> rs, cs, cr, rc, rcase;
        for (auto& g : b->groups) {
            const int64_t base = g.dof_off / 3;
            for (int c = 0; c < g.r; ++c)
                for (int k = 0; k < g.T.n_regions; ++k) {
                    rs.push_back((int32_t)(base + c * g.N + g.T.region_start[k]));
                    rcase.push_back(g.case0 + c);
                }
        }
        rs.push_back((int32_t)nodes);
        region_chunks(rs, cs, cr, rc);
        b->chunks.n_regions = (int32_t)rs.size() - 1;
        b->chunks.n_chunks = (int32_t)cr.size();
        int32_t* d_cs = M.alloc<int32_t>(cs.size());
        int32_t* d_cr = M.alloc<int32_t>(cr.size());
        int32_t* d_rc = M.alloc<int32_t>(rc.size());
        BCHK(hipMemcpyAsync(d_cs, cs.data(), cs.size() * sizeof(int32_t), hipMemcpyHostToDevice, s));
        BCHK(hipMemcpyAsync(d_cr, cr.data(), cr.size() * sizeof(int32_t), hipMemcpyHostToDevice, s));
        BCHK(hipMemcpyAsync(d_rc, rc.data(), rc.size() * sizeof(int32_t), hipMemcpyHostToDevice, s));
        int32_t* d_rcase = M.alloc<int32_t>(rcase.size());
        BCHK(hipMemcpyAsync(d_rcase, rcase.data(), rcase.size() * sizeof(int32_t), hipMemcpyHostToDevice, s));
        b->chunks.start = d_cs;
        b->chunks.region = d_cr;
        b->chunks.first = d_rc;
        b->chunks.region_case = d_rcase;
        b->coef = M.alloc<double>(32 * (size_t)b->chunks.n_regions);
        b->gh = M.alloc<double>((size_t)kGhStride * b->chunks.n_chunks);
        // per group: block-Jacobi inverse (shared by its cases) and partials
        for (auto& g : b->groups) {
            g.binv6 = M.alloc<double>(6 * g.N);
            double* q6 = M.alloc<double>(6 * g.PN);
            launch_ebe_diag(s, g.dp, b->cM, b->cK, q6);
            launch_diag_finalize(s, g.dn, q6, g.binv6);
            g.part = M.alloc<double>(2 * (size_t)kResArrays * g.r * g.g_upd);
            g.pap = M.alloc<double>((size_t)g.r * g.chunks);
            g.cand = M.alloc<double>(2 * (size_t)g.r * g.g_upd);
        }
        for (double* v : {b->u, b->a, b->vh[0], b->vh[1], b->vh[2], b->vh[3], b->p[0], b->p[1], b->x})
            launch_zero(s, dof, v);
        launch_zero(s, (int64_t)(b->cfg.s + 1) * dof, b->ring);
        check_launch();
        BCHK(hipStreamSynchronize(s));
        b->head = b->it = b->par = 0;
        b->last_iters = 0;
        b->assembled = true;
        return EBE_OK;
    });
}

int ebe_batch_group_info(ebe_batch* b, int32_t group, int32_t* first_case, int32_t* n_cases, int64_t* n_nodes,
                         int32_t* case_tile, int32_t* chunks) {
    return bguard(b, [&]() -> int {
        need_asm(b);
        if (group < 0 || group >= (int)b->groups.size()) throw BErr{EBE_E_INVALID_ARG, "no such group"};
        const Group& g = b->groups[group];
        if (first_case) *first_case = g.case0;
        if (n_cases) *n_cases = g.r;
        if (n_nodes) *n_nodes = g.N;
        if (case_tile) *case_tile = g.ct;
        if (chunks) *chunks = g.chunks;
        return EBE_OK;
    });
}

int ebe_batch_use_graph(ebe_batch* b, int32_t on, int32_t trips) {
    return bguard(b, [&]() -> int {
        if (trips < 2 || trips > 64 || trips % 2) throw BErr{EBE_E_INVALID_ARG, "trips must be even, 2..64"};
        b->drop_graph();
        b->use_graph = on != 0;
        b->graph_trips = trips;
        return EBE_OK;
    });
}

int ebe_batch_reset(ebe_batch* b) {
    return bguard(b, [&]() -> int {
        need_asm(b);
        hipStream_t s = b->stream;
        for (double* v : {b->u, b->a, b->vh[0], b->vh[1], b->vh[2], b->vh[3]}) launch_zero(s, b->n3, v);
        launch_zero(s, (int64_t)(b->cfg.s + 1) * b->n3, b->ring);
        check_launch();
        b->head = b->it = 0;
        b->last_iters = 0;
        b->win.assign(b->C, 1);
        return EBE_OK;
    });
}

int ebe_batch_apply(ebe_batch* b, int32_t group, const double* p, double* q) {
    return bguard(b, [&]() -> int {
        need_asm(b);
        if (group < 0 || group >= (int)b->groups.size()) throw BErr{EBE_E_INVALID_ARG, "no such group"};
        if (!p || !q) throw BErr{EBE_E_INVALID_ARG, "null vector"};
        hipStream_t s = b->stream;
        Group& g = b->groups[group];
        const int64_t n3 = 3 * g.N;
        for (int c = 0; c < g.r; ++c)
            launch_gather3(s, g.N, g.d_i2u, p + c * n3, b->t0 + g.dof_off + c * n3);
        BEbeArgs A = ebe_args(b, g);
        A.in0 = b->t0 + g.dof_off;
        A.mask_in = 1;
        launch_bebe(s, MODE_APPLY, A, g.ct, g.chunks);
        launch_bcombine(s, node_args(b, g), b->t0 + g.dof_off, nullptr, b->t1 + g.dof_off, 1);
        for (int c = 0; c < g.r; ++c)
            launch_gather3(s, g.N, g.d_u2i, b->t1 + g.dof_off + c * n3, q + c * n3);
        check_launch();
        return EBE_OK;
    });
}

int ebe_batch_step(ebe_batch* b, const double* base_acc, ebe_batch_stats* stats) {
    return bguard(b, [&]() -> int {
        need_asm(b);
        if (!base_acc) throw BErr{EBE_E_INVALID_ARG, "base_acc (host [n_cases][3]) required"};
        hipStream_t s = b->stream;
        const ebe_config& c = b->cfg;
        std::memcpy(b->g_host, base_acc, 3 * b->C * sizeof(double));
        BCHK(hipMemcpyAsync(b->g_dev, b->g_host, 3 * b->C * sizeof(double), hipMemcpyHostToDevice, s));
        // right-hand sides
        for (auto& g : b->groups) {
            BEbeArgs A = ebe_args(b, g);
            A.in0 = b->u + g.dof_off;
            A.in1 = b->vslot(0) + g.dof_off;
            A.in2 = b->a + g.dof_off;
            A.cm = 1.0;   // b = M w1 + K w2: plain M and K, not the system coefficients
            A.ck = 1.0;
            A.c1 = 4.0 / c.dt + c.rayleigh_alpha;
            A.c2 = c.rayleigh_beta;
            A.g = b->g_dev + 3 * g.case0;
            launch_bebe(s, MODE_RHS, A, g.ct, g.chunks);
            launch_bcombine(s, node_args(b, g), nullptr, nullptr, b->b + g.dof_off, 2);
        }
        // Adams-Bashforth 4 and the regional snapshot map over the stacked vectors; every
        // case has its own window (see ebe_step), the regions of a case use the newest
        // columns of the common window that its own window holds
        const int n = b->it + 1;
        launch_ab4(s, b->n3, c.dt, b->vslot(0), b->vslot(1), b->vslot(2), b->vslot(3),
                   c.predictor == EBE_PRED_ZERO ? 0 : 1, b->dab, b->x);
        std::vector<int> se(b->C, 0), first(b->C, 0);
        int S = 0;
        if (c.predictor == EBE_PRED_SNAPSHOT && c.s >= 1) {
            const int s_min = std::max(1, std::min(c.s_min, c.s));
            for (int k = 0; k < b->C; ++k) {
                const int f = std::max(b->win[k], n - 1 - c.s);
                if (n - 1 - f >= s_min) {
                    se[k] = n - 1 - f;
                    first[k] = f;
                    S = std::max(S, se[k]);
                }
            }
        }
        const bool guarded = S >= 1 && !c.fixed_window;
        if (S >= 1) {
            ColPtrs W{};
            const int S1 = c.s + 1, f0 = n - 1 - S;
            for (int jj = 0; jj <= S; ++jj) W.c[jj] = b->ring_slot((f0 + jj - 1) % S1);   // e^{f0 + jj}
            for (int k = 0; k < b->C; ++k) b->lo_host[k] = se[k] > 0 ? S - se[k] : S;
            BCHK(hipMemcpyAsync(b->lo_dev, b->lo_host, b->C * sizeof(int32_t), hipMemcpyHostToDevice, s));
            launch_gram_solve(s, W, S, b->chunks, c.drop_tol, b->gh, b->coef, b->lo_dev);
            launch_pred_apply(s, W, S, b->chunks, b->coef, b->dab, b->x);
            if (guarded) {
                for (auto& g : b->groups) {
                    BNodeArgs N = node_args(b, g);
                    BEbeArgs A = ebe_args(b, g);
                    A.mask_in = 1;
                    A.in0 = b->x + g.dof_off;
                    launch_bebe(s, MODE_APPLY, A, g.ct, g.chunks);
                    launch_bcand_res(s, N, g.cand);
                    A.in0 = b->dab + g.dof_off;
                    launch_bebe(s, MODE_APPLY, A, g.ct, g.chunks);
                    launch_bcand_res(s, N, g.cand + (size_t)g.r * g.g_upd);
                    launch_bguard_select(s, N, g.cand, g.cand + (size_t)g.r * g.g_upd, b->dab + g.dof_off);
                }
            }
        }
        check_launch();
        int rc = solve_batch(b);
        if (rc < 0) return rc;
        // a case whose AB4 guess beat its map restarts its window at this step
        for (int k = 0; k < b->C; ++k)
            if (guarded && se[k] > 0 && b->sc_host[k].guard_pick) b->win[k] = n;
        double* slot = c.s >= 1 ? b->ring_slot((n - 1) % (c.s + 1)) : nullptr;
        launch_newmark(s, b->n3, c.dt, b->x, b->dab, b->u, b->vslot(0), b->vslot(3), b->a, slot);
        check_launch();
        b->head = (b->head + 3) & 3;
        b->it = n;
        if (stats) {
            for (int k = 0; k < b->C; ++k) {
                const DevScalars& Sk = b->sc_host[k];
                ebe_batch_stats& o = stats[k];
                o = ebe_batch_stats{};
                o.iters = Sk.iters;
                o.restarts = Sk.restarts;
                o.status = Sk.done == DONE_MAXITER ? EBE_NOT_CONVERGED : EBE_OK;
                o.s_eff = se[k];
                o.first = first[k];
                o.map_kept = (guarded && se[k] > 0) ? 1 - Sk.guard_pick : -1;
                o.res0 = Sk.res0;
                o.res_true = Sk.bnorm > 0 ? Sk.res_true : 0.0;
                o.bnorm = Sk.bnorm;
            }
        }
        return rc;
    });
}

int ebe_batch_get_state(ebe_batch* b, int32_t case_index, double* u, double* v, double* a) {
    return bguard(b, [&]() -> int {
        need_asm(b);
        if (case_index < 0 || case_index >= b->C) throw BErr{EBE_E_INVALID_ARG, "no such case"};
        for (auto& g : b->groups) {
            if (case_index < g.case0 || case_index >= g.case0 + g.r) continue;
            const int64_t o = g.dof_off + (int64_t)(case_index - g.case0) * 3 * g.N;
            if (u) launch_gather3(b->stream, g.N, g.d_u2i, b->u + o, u);
            if (v) launch_gather3(b->stream, g.N, g.d_u2i, b->vslot(0) + o, v);
            if (a) launch_gather3(b->stream, g.N, g.d_u2i, b->a + o, a);
        }
        check_launch();
        return EBE_OK;
    });
}

int ebe_batch_sizes(ebe_batch* b, int32_t* n_groups, int32_t* n_cases, int64_t* total_dof) {
    return bguard(b, [&]() -> int {
        need_asm(b);
        if (n_groups) *n_groups = (int32_t)b->groups.size();
        if (n_cases) *n_cases = b->C;
        if (total_dof) *total_dof = b->n3;
        return EBE_OK;
    });
}

}  // extern "C"
