// topology.cpp -- host-side preprocessing of the mesh for the EBE kernels.
//
// Internal node order: nodes sorted by (region, Morton code of the position),
// so every region is one contiguous range of the state vectors and nodes that
// are close in space are close in memory.  With merging, the regions are
// taken in the Morton order of their centroids and each run of region_merge
// of them is one predictor region (contiguous too).
// Element order: by the lowest internal id among the element's vertices,
// ties broken by the Morton code of the centroid.  Consecutive runs of
// patch_elems elements form a patch (inside a patch the elements are dealt
// round-robin to the workgroup's groups of 8 lanes and the local node ids are
// spread over the LDS banks, see spread_banks); a patch is processed by one workgroup
// (one element per thread) that stages the patch's nodes in LDS.  Each patch lists its nodes
// (vertices first, so the geometry gather touches a prefix only).  Each
// (patch, node) pair writes its partial result to its own slot; the slots of a
// node are contiguous and in patch order, which fixes the summation order and
// makes results bitwise reproducible.
#include "topology.h"

#include <algorithm>
#include <array>
#include <cmath>
#include <cstdio>
#include <numeric>

namespace ebe {

static const int kEdge[6][2] = {{0, 1}, {1, 2}, {0, 2}, {0, 3}, {1, 3}, {2, 3}};

static uint64_t spread3(uint64_t x) {
    x &= 0x1fffff;
    x = (x | x << 32) & 0x1f00000000ffffull;
    x = (x | x << 16) & 0x1f0000ff0000ffull;
    x = (x | x << 8) & 0x100f00f00f00f00full;
    x = (x | x << 4) & 0x10c30c30c30c30c3ull;
    x = (x | x << 2) & 0x1249249249249249ull;
    return x;
}

namespace {
struct Box {
    double lo[3], hi[3];
    uint64_t morton(const double* p) const {
        uint64_t c = 0;
        for (int d = 0; d < 3; ++d) {
            double ext = hi[d] - lo[d];
            double t = ext > 0 ? (p[d] - lo[d]) / ext : 0.0;
            uint64_t q = (uint64_t)std::min(2097151.0, std::max(0.0, std::floor(t * 2097151.0)));
            c |= spread3(q) << d;
        }
        return c;
    }
};
}  // namespace

// Patch-local numbering against LDS bank conflicts.  The element kernels add
// each element's nodal results into a per-wavefront FP64 LDS accumulator
// indexed by the patch-local node id l (doubles 3l .. 3l+2); the same ids index
// the element's reads of the staged operand.  On gfx950 an FP64 LDS atomic is
// serviced in groups of 8 lanes over 16 bank pairs (32 four-byte banks),
// measured: lanes of one group whose doubles fall on the same bank pair are
// serialised, so the cost of one atomic instruction of one group is the
// largest number of its lanes that share a bank pair.  Double 3l + c lies on
// bank pair (3l + c) mod 16, and 3 is invertible mod 16, so the lanes of a
// group conflict exactly when their node ids agree mod 16.
//
// spread_banks() reassigns the local ids of one patch so that, for every group
// of 8 consecutive elements (the 8 lanes) and every element position i
// (the i-th node of each element, added by the same instruction), the ids are
// spread over the residues mod 16.  Ids are only exchanged between nodes of the
// same kind (vertex or edge node: vertices keep the prefix [0, nv)) inside an
// aligned block of 64 ids -- the ids one wavefront gathers and writes out in
// one instruction -- so the set of global addresses each gather and write-out
// instruction touches is unchanged.  Greedy exchanges that lower the number of
// same-residue pairs, over a few passes; deterministic.
constexpr int kLdsLaneGroup = 8;    // lanes serviced together by an FP64 LDS atomic
constexpr int kLdsBankPairs = 16;   // 8-byte bank pairs

static void spread_banks(int ne, const std::vector<std::array<int32_t, 10>>& el_local, int nv, int npn,
                         std::vector<int32_t>& newid) {
    // sets: (lane group, position); members: local node ids (pre-renumbering)
    const int ngroups = (ne + kLdsLaneGroup - 1) / kLdsLaneGroup;
    const int nsets = ngroups * 10;
    std::vector<std::vector<int32_t>> memb(npn);   // sets containing each node (with multiplicity)
    for (int e = 0; e < ne; ++e)
        for (int i = 0; i < 10; ++i) memb[el_local[e][i]].push_back((e / kLdsLaneGroup) * 10 + i);
    newid.resize(npn);
    std::iota(newid.begin(), newid.end(), 0);
    std::vector<int32_t> at(npn);                  // node at each id
    std::iota(at.begin(), at.end(), 0);
    std::vector<int32_t> cnt((size_t)nsets * kLdsBankPairs, 0);
    auto res = [&](int node) { return newid[node] % kLdsBankPairs; };
    for (int v = 0; v < npn; ++v)
        for (int s : memb[v]) cnt[(size_t)s * kLdsBankPairs + res(v)]++;
    // change of the number of same-residue pairs if node v moves from residue a to b
    auto move_delta = [&](int v, int a, int b) {
        if (a == b) return 0;
        int d = 0;
        for (int s : memb[v]) {
            const int32_t* c = &cnt[(size_t)s * kLdsBankPairs];
            d += c[b] - (c[a] - 1);
        }
        return d;
    };
    auto apply_move = [&](int v, int a, int b) {
        for (int s : memb[v]) {
            cnt[(size_t)s * kLdsBankPairs + a]--;
            cnt[(size_t)s * kLdsBankPairs + b]++;
        }
    };
    int dv[kLdsBankPairs];
    for (int pass = 0; pass < 4; ++pass) {
        bool changed = false;
        for (int v = 0; v < npn; ++v) {
            const int idv = newid[v], ra = idv % kLdsBankPairs;
            // only nodes in a conflicting set, and only residues that help v
            int worst = 0;
            for (int s : memb[v]) worst = std::max(worst, cnt[(size_t)s * kLdsBankPairs + ra]);
            if (worst <= 1) continue;
            bool any = false;
            for (int r = 0; r < kLdsBankPairs; ++r) {
                dv[r] = move_delta(v, ra, r);
                any = any || dv[r] < 0;
            }
            if (!any) continue;
            // ids v may take: same 64-block, same kind
            const int blk0 = idv / 64 * 64, blk1 = std::min(npn, blk0 + 64);
            const int lo = idv < nv ? blk0 : std::max(blk0, nv), hi = idv < nv ? std::min(blk1, nv) : blk1;
            int best = 0, best_id = -1;
            for (int idu = lo; idu < hi; ++idu) {
                const int rb = idu % kLdsBankPairs;
                if (rb == ra || dv[rb] >= 0) continue;
                const int u = at[idu];
                // exchange v (ra -> rb) and u (rb -> ra); sets holding both see both moves
                apply_move(v, ra, rb);
                const int d = dv[rb] + move_delta(u, rb, ra);
                apply_move(v, rb, ra);
                if (d < best) {
                    best = d;
                    best_id = idu;
                }
            }
            if (best_id >= 0) {
                const int u = at[best_id], rb = best_id % kLdsBankPairs;
                apply_move(v, ra, rb);
                apply_move(u, rb, ra);
                std::swap(newid[v], newid[u]);
                at[newid[v]] = v;
                at[newid[u]] = u;
                changed = true;
            }
        }
        if (!changed) break;
    }
}

template <class... A>
static std::string fmt(const char* f, A... a) {
    char buf[512];
    std::snprintf(buf, sizeof(buf), f, a...);
    return std::string(buf);
}

void region_chunks(const std::vector<int32_t>& region_start, std::vector<int32_t>& chunk_start,
                   std::vector<int32_t>& chunk_region, std::vector<int32_t>& region_chunk) {
    const int32_t R = (int32_t)region_start.size() - 1;
    chunk_start.clear();
    chunk_region.clear();
    region_chunk.assign(R + 1, 0);
    for (int32_t r = 0; r < R; ++r) {
        const int64_t a = region_start[r], len = region_start[r + 1] - a;
        const int64_t n = std::max<int64_t>(1, std::min<int64_t>(kMaxRegionChunks, (len + kChunkNodes - 1) / kChunkNodes));
        region_chunk[r] = (int32_t)chunk_start.size();
        for (int64_t k = 0; k < n; ++k) {
            chunk_start.push_back((int32_t)(a + len * k / n));
            chunk_region.push_back(r);
        }
    }
    region_chunk[R] = (int32_t)chunk_start.size();
    chunk_start.push_back(R > 0 ? region_start[R] : 0);
}

std::string build_topology(Topology& T, int64_t N, const double* X, int64_t E, const int32_t* conn,
                           const int32_t* elem_mat, int32_t n_mat, const double* mat, const uint8_t* fixed,
                           const int32_t* region_of_node, int region_nodes, int patch_elems, const PatchLds& lds, int region_merge) {
    if (N <= 0 || E <= 0) return "mesh must have nodes and elements";
    if (N >= (int64_t)1 << 31 || E >= (int64_t)1 << 31) return "mesh too large for 32-bit ids";
    if (n_mat <= 0 || n_mat > 65535) return "n_mat must be in [1, 65535]";
    if (patch_elems <= 0 || patch_elems > kMaxPatchElems) return "patch_elems must be in [1, 256]";
    T = Topology();
    T.n_nodes = N;
    T.n_elems = E;

    // ---- materials
    T.mat_lmr.resize(3 * (size_t)n_mat);
    for (int m = 0; m < n_mat; ++m) {
        double rho = mat[3 * m], vp = mat[3 * m + 1], vs = mat[3 * m + 2];
        double mu = rho * vs * vs, lam = rho * (vp * vp - 2.0 * vs * vs);
        if (!(rho > 0) || !(vs > 0) || !(lam + 2.0 * mu / 3.0 > 0) || !std::isfinite(lam))
            return fmt("material %d is not a valid isotropic elastic solid", m);
        T.mat_lmr[3 * m] = lam;
        T.mat_lmr[3 * m + 1] = mu;
        T.mat_lmr[3 * m + 2] = rho;
    }

    // ---- element validation: ids, orientation, midpoint edge nodes; vertex/edge roles
    std::vector<uint8_t> role(N, 0);  // bit0 vertex, bit1 edge
    for (int64_t e = 0; e < E; ++e) {
        const int32_t* c = conn + 10 * e;
        for (int i = 0; i < 10; ++i)
            if (c[i] < 0 || c[i] >= N) return fmt("element %lld references node %d out of range", (long long)e, c[i]);
        if (elem_mat[e] < 0 || elem_mat[e] >= n_mat) return fmt("element %lld has material %d out of range", (long long)e, elem_mat[e]);
        const double* x0 = X + 3 * (int64_t)c[0];
        double J[3][3];
        double h2 = 0;
        for (int k = 0; k < 3; ++k)
            for (int r = 0; r < 3; ++r) {
                J[r][k] = X[3 * (int64_t)c[k + 1] + r] - x0[r];
                h2 = std::max(h2, std::fabs(J[r][k]));
            }
        double det = J[0][0] * (J[1][1] * J[2][2] - J[1][2] * J[2][1]) - J[0][1] * (J[1][0] * J[2][2] - J[1][2] * J[2][0]) +
                     J[0][2] * (J[1][0] * J[2][1] - J[1][1] * J[2][0]);
        if (!(det > 1e-12 * h2 * h2 * h2)) return fmt("element %lld is inverted or degenerate", (long long)e);
        for (int m = 0; m < 6; ++m) {
            const double* xa = X + 3 * (int64_t)c[kEdge[m][0]];
            const double* xb = X + 3 * (int64_t)c[kEdge[m][1]];
            const double* xm = X + 3 * (int64_t)c[4 + m];
            for (int r = 0; r < 3; ++r)
                if (std::fabs(xm[r] - 0.5 * (xa[r] + xb[r])) > 1e-9 * h2)
                    return fmt("element %lld: edge node %d is not at its edge midpoint", (long long)e, c[4 + m]);
        }
        for (int i = 0; i < 4; ++i) role[c[i]] |= 1;
        for (int i = 4; i < 10; ++i) role[c[i]] |= 2;
    }
    for (int64_t v = 0; v < N; ++v) {
        if (role[v] == 0) return fmt("node %lld is not used by any element", (long long)v);
        if (role[v] == 3) return fmt("node %lld is a vertex of one element and an edge node of another", (long long)v);
    }

    // ---- Morton codes of nodes
    Box box;
    for (int d = 0; d < 3; ++d) { box.lo[d] = 1e300; box.hi[d] = -1e300; }
    for (int64_t v = 0; v < N; ++v)
        for (int d = 0; d < 3; ++d) {
            box.lo[d] = std::min(box.lo[d], X[3 * v + d]);
            box.hi[d] = std::max(box.hi[d], X[3 * v + d]);
        }
    std::vector<uint64_t> mort(N);
    for (int64_t v = 0; v < N; ++v) mort[v] = box.morton(X + 3 * v);

    // ---- regions
    T.region_user.assign(N, 0);
    if (region_of_node) {
        int32_t rmax = -1;
        for (int64_t v = 0; v < N; ++v) {
            if (region_of_node[v] < 0) return "region ids must be non-negative";
            rmax = std::max(rmax, region_of_node[v]);
        }
        T.n_regions = rmax + 1;
        std::vector<int64_t> cnt(T.n_regions, 0);
        for (int64_t v = 0; v < N; ++v) cnt[region_of_node[v]]++;
        for (int32_t r = 0; r < T.n_regions; ++r)
            if (cnt[r] == 0) return fmt("region %d is empty (ids must be dense)", r);
        std::copy(region_of_node, region_of_node + N, T.region_user.begin());
    } else {
        if (region_nodes <= 0) region_nodes = 512;
        std::vector<int32_t> ord(N);
        std::iota(ord.begin(), ord.end(), 0);
        std::stable_sort(ord.begin(), ord.end(), [&](int32_t a, int32_t b) { return mort[a] < mort[b]; });
        int64_t nr = (N + region_nodes - 1) / region_nodes;
        T.n_regions = (int32_t)nr;
        for (int64_t k = 0; k < N; ++k) T.region_user[ord[k]] = (int32_t)std::min<int64_t>(k / region_nodes, nr - 1);
    }

    // ---- merged predictor regions: the given regions in Morton order of
    // their centroids, region_merge at a time; rank[r] is region r's position
    // in that order (the identity without merging)
    std::vector<int64_t> rank(T.n_regions);
    std::iota(rank.begin(), rank.end(), 0);
    if (region_merge > 1 && T.n_regions > 1) {
        const int32_t R = T.n_regions;
        std::vector<double> cen(3 * (size_t)R, 0.0);
        std::vector<int64_t> cnt(R, 0);
        for (int64_t v = 0; v < N; ++v) {
            const int32_t r = T.region_user[v];
            for (int d = 0; d < 3; ++d) cen[3 * (size_t)r + d] += X[3 * v + d];
            cnt[r]++;
        }
        std::vector<uint64_t> rmort(R);
        for (int32_t r = 0; r < R; ++r) {
            for (int d = 0; d < 3; ++d) cen[3 * (size_t)r + d] /= (double)cnt[r];
            rmort[r] = box.morton(&cen[3 * (size_t)r]);
        }
        std::vector<int32_t> rord(R);
        std::iota(rord.begin(), rord.end(), 0);
        std::stable_sort(rord.begin(), rord.end(), [&](int32_t a, int32_t b) { return rmort[a] < rmort[b]; });
        for (int32_t k = 0; k < R; ++k) rank[rord[k]] = k;
    }

    // ---- internal node order: (given region in merge order, Morton)
    T.i2u.resize(N);
    std::iota(T.i2u.begin(), T.i2u.end(), 0);
    std::stable_sort(T.i2u.begin(), T.i2u.end(), [&](int32_t a, int32_t b) {
        const int64_t ra = rank[T.region_user[a]], rb = rank[T.region_user[b]];
        if (ra != rb) return ra < rb;
        return mort[a] < mort[b];
    });
    if (region_merge > 1 && T.n_regions > 1) {
        for (int64_t v = 0; v < N; ++v) T.region_user[v] = (int32_t)(rank[T.region_user[v]] / region_merge);
        T.n_regions = (int32_t)((T.n_regions + region_merge - 1) / region_merge);
    }
    T.u2i.resize(N);
    for (int64_t i = 0; i < N; ++i) T.u2i[T.i2u[i]] = (int32_t)i;
    T.region_start.assign(T.n_regions + 1, 0);
    for (int64_t v = 0; v < N; ++v) T.region_start[T.region_user[v] + 1]++;
    for (int32_t r = 0; r < T.n_regions; ++r) T.region_start[r + 1] += T.region_start[r];
    region_chunks(T.region_start, T.chunk_start, T.chunk_region, T.region_chunk);
    T.coords.resize(3 * N);
    T.fixmask.resize(N);
    for (int64_t i = 0; i < N; ++i) {
        int32_t u = T.i2u[i];
        for (int d = 0; d < 3; ++d) T.coords[3 * i + d] = X[3 * (int64_t)u + d];
        T.fixmask[i] = (uint8_t)((fixed[3 * (int64_t)u] ? 1 : 0) | (fixed[3 * (int64_t)u + 1] ? 2 : 0) |
                                 (fixed[3 * (int64_t)u + 2] ? 4 : 0));
    }

    // ---- element order
    std::vector<int32_t> eord(E);
    std::iota(eord.begin(), eord.end(), 0);
    std::vector<int32_t> ekey(E);
    std::vector<uint64_t> emort(E);
    for (int64_t e = 0; e < E; ++e) {
        const int32_t* c = conn + 10 * e;
        int32_t k = INT32_MAX;
        double cen[3] = {0, 0, 0};
        for (int i = 0; i < 4; ++i) {
            k = std::min(k, T.u2i[c[i]]);
            for (int d = 0; d < 3; ++d) cen[d] += 0.25 * X[3 * (int64_t)c[i] + d];
        }
        ekey[e] = k;
        emort[e] = box.morton(cen);
    }
    std::stable_sort(eord.begin(), eord.end(), [&](int32_t a, int32_t b) {
        if (ekey[a] != ekey[b]) return ekey[a] < ekey[b];
        return emort[a] < emort[b];
    });

    // ---- patches: cut the element order into runs of at most patch_elems
    // elements whose nodes fit the LDS budget.  The kernels size LDS by the
    // largest node count and the largest vertex count over all patches (which
    // may come from different patches), so a patch is closed once it would
    // raise that combined size past the budget.
    std::vector<int64_t> cut(1, 0);
    {
        std::vector<int64_t> mark(N, -1);   // last patch that listed the node
        int64_t npn = 0, nvx = 0, cnt = 0, max_n = 0, max_v = 0;
        for (int64_t k = 0; k < E; ++k) {
            const int32_t* c = conn + 10 * (int64_t)eord[k];
            const int64_t cur = (int64_t)cut.size() - 1;
            int64_t add_n = 0, add_v = 0;
            for (int i = 0; i < 10; ++i)
                if (mark[c[i]] != cur) { ++add_n; add_v += i < 4; }
            const bool over = lds.budget > 0 && lds.fixed + lds.per_node * std::max(max_n, npn + add_n) +
                                                        lds.per_vertex * std::max(max_v, nvx + add_v) >
                                                    lds.budget;
            if (cnt > 0 && (cnt == patch_elems || over)) {
                cut.push_back(k);
                max_n = std::max(max_n, npn);
                max_v = std::max(max_v, nvx);
                npn = nvx = cnt = 0;
                add_n = 10;
                add_v = 4;
            }
            const int64_t now = (int64_t)cut.size() - 1;
            for (int i = 0; i < 10; ++i) mark[c[i]] = now;
            npn += add_n;
            nvx += add_v;
            ++cnt;
        }
        if (E > 0) cut.push_back(E);
    }
    int64_t P = (int64_t)cut.size() - 1;
    int64_t Ppad = (P + 7) / 8 * 8;
    T.n_patches = (int32_t)P;
    T.n_patches_pad = (int32_t)Ppad;
    T.patch_el_ptr.assign(Ppad + 1, 0);
    T.patch_pn_ptr.assign(Ppad + 1, 0);
    T.patch_nv.assign(Ppad, 0);
    T.elems.resize(E);
    T.patch_nodes.clear();
    T.patch_nodes.reserve(3 * N);
    std::vector<int32_t> nodes;
    std::vector<int32_t> local(N, -1);
    std::vector<uint8_t> seen(N, 0);
    std::vector<int32_t> dealt, newid, ordered;
    std::vector<std::array<int32_t, 10>> el_local;
    for (int64_t p = 0; p < Ppad; ++p) {
        const int64_t e0 = p < P ? cut[p] : E, e1 = p < P ? cut[p + 1] : E;
        T.patch_el_ptr[p + 1] = (int32_t)e1;
        // Deal the patch's spatially sorted elements round-robin to the
        // groups of 8 lanes (kLdsLaneGroup) of the workgroup: elements that
        // share nodes (e.g. the six tetrahedra of one cell, which share the
        // cell's diagonal at the same element positions) land in different
        // lane groups, so the lanes serviced together by one LDS atomic rarely
        // add into the same address.
        const int deal = std::max(1, patch_elems / kLdsLaneGroup);
        dealt.clear();
        for (int w = 0; w < deal; ++w)
            for (int64_t k = e0 + w; k < e1; k += deal) dealt.push_back(eord[k]);
        std::copy(dealt.begin(), dealt.end(), eord.begin() + e0);
        nodes.clear();
        for (int64_t k = e0; k < e1; ++k) {
            const int32_t* c = conn + 10 * (int64_t)eord[k];
            for (int i = 0; i < 10; ++i) nodes.push_back(T.u2i[c[i]]);
        }
        std::sort(nodes.begin(), nodes.end());
        nodes.erase(std::unique(nodes.begin(), nodes.end()), nodes.end());
        // vertices first
        std::stable_partition(nodes.begin(), nodes.end(), [&](int32_t v) { return role[T.i2u[v]] == 1; });
        int nv = 0;
        for (int32_t v : nodes) nv += role[T.i2u[v]] == 1;
        if (nodes.size() > 65535) return "patch too large";
        for (size_t j = 0; j < nodes.size(); ++j) local[nodes[j]] = (int32_t)j;
        // spread the local ids over the LDS bank pairs (see spread_banks)
        el_local.resize(e1 - e0);
        for (int64_t k = e0; k < e1; ++k) {
            const int32_t* c = conn + 10 * (int64_t)eord[k];
            for (int i = 0; i < 10; ++i) el_local[k - e0][i] = local[T.u2i[c[i]]];
        }
        spread_banks((int)(e1 - e0), el_local, nv, (int)nodes.size(), newid);
        ordered.assign(nodes.size(), 0);
        for (size_t j = 0; j < nodes.size(); ++j) ordered[newid[j]] = nodes[j];
        nodes.swap(ordered);
        for (size_t j = 0; j < nodes.size(); ++j) {
            int32_t v = nodes[j];
            local[v] = (int32_t)j;
            uint32_t ent = (uint32_t)v;
            if (!seen[v]) { ent |= kOwnerBit; seen[v] = 1; }
            T.patch_nodes.push_back(ent);
        }
        for (int64_t k = e0; k < e1; ++k) {
            const int32_t* c = conn + 10 * (int64_t)eord[k];
            ElemRec& r = T.elems[k];
            for (int i = 0; i < 10; ++i) r.lid[i] = (uint16_t)local[T.u2i[c[i]]];
            r.mat = (uint16_t)elem_mat[eord[k]];
            r.pad = 0;
        }
        T.patch_nv[p] = nv;
        T.patch_pn_ptr[p + 1] = (int32_t)T.patch_nodes.size();
        T.max_pn = std::max<int32_t>(T.max_pn, (int32_t)nodes.size());
        T.max_nv = std::max(T.max_nv, nv);
    }
    if ((int64_t)T.patch_nodes.size() >= ((int64_t)1 << 31)) return "too many patch nodes";

    // ---- node-major slots (patch order within a node)
    T.slot_ptr.assign(N + 1, 0);
    for (uint32_t ent : T.patch_nodes) T.slot_ptr[(ent & ~kOwnerBit) + 1]++;
    for (int64_t v = 0; v < N; ++v) T.slot_ptr[v + 1] += T.slot_ptr[v];
    T.patch_slot.resize(T.patch_nodes.size());
    std::vector<int32_t> pos(T.slot_ptr.begin(), T.slot_ptr.end() - 1);
    for (size_t k = 0; k < T.patch_nodes.size(); ++k) T.patch_slot[k] = pos[T.patch_nodes[k] & ~kOwnerBit]++;
    for (int64_t v = 0; v < N; ++v)
        if (T.slot_ptr[v + 1] == T.slot_ptr[v]) return "internal error: node without patch";
    return std::string();
}

}  // namespace ebe
