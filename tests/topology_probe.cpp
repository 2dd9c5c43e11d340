// Test helper (not product code): exposes the host-side patch topology of the
// library's topology.cpp through a C interface, so the CPU tests can check its
// invariants.  Built by tests/test_topology.py with the host compiler.
#include <cstdint>
#include <cstring>
#include <string>
#include <vector>

#include "topology.h"

using namespace ebe;

namespace {
Topology g_T;
}

extern "C" int probe_build(int64_t nn, const double* xyz, int64_t ne, const int32_t* conn, const int32_t* em, int nm,
                           const double* mat, const uint8_t* fx, const int32_t* reg, int region_nodes,
                           int patch_elems) {
    g_T = Topology();
    std::string e = build_topology(g_T, nn, xyz, ne, conn, em, nm, mat, fx, reg, region_nodes, patch_elems);
    return e.empty() ? 0 : 1;
}

// As probe_build, with the patch LDS budget of the element kernels.
extern "C" int probe_build_lds(int64_t nn, const double* xyz, int64_t ne, const int32_t* conn, const int32_t* em,
                               int nm, const double* mat, const uint8_t* fx, const int32_t* reg, int region_nodes,
                               int patch_elems, int64_t per_node, int64_t per_vertex, int64_t fixed_bytes,
                               int64_t budget) {
    g_T = Topology();
    PatchLds lds;
    lds.per_node = per_node;
    lds.per_vertex = per_vertex;
    lds.fixed = fixed_bytes;
    lds.budget = budget;
    std::string e = build_topology(g_T, nn, xyz, ne, conn, em, nm, mat, fx, reg, region_nodes, patch_elems, lds);
    return e.empty() ? 0 : 1;
}

// As probe_build_lds, with region_merge.
extern "C" int probe_build_merge(int64_t nn, const double* xyz, int64_t ne, const int32_t* conn, const int32_t* em,
                                 int nm, const double* mat, const uint8_t* fx, const int32_t* reg, int region_nodes,
                                 int patch_elems, int64_t per_node, int64_t per_vertex, int64_t fixed_bytes,
                                 int64_t budget, int region_merge) {
    g_T = Topology();
    PatchLds lds;
    lds.per_node = per_node;
    lds.per_vertex = per_vertex;
    lds.fixed = fixed_bytes;
    lds.budget = budget;
    std::string e =
        build_topology(g_T, nn, xyz, ne, conn, em, nm, mat, fx, reg, region_nodes, patch_elems, lds, region_merge);
    return e.empty() ? 0 : 1;
}

// Predictor regions: the region of every user node [nn], the count, and the
// internal ranges region_start [n_regions + 1] (room for cap entries).
extern "C" int32_t probe_regions(int32_t* region_user, int32_t* region_start, int32_t cap) {
    std::memcpy(region_user, g_T.region_user.data(), g_T.region_user.size() * 4);
    if ((int32_t)g_T.region_start.size() <= cap)
        std::memcpy(region_start, g_T.region_start.data(), g_T.region_start.size() * 4);
    return g_T.n_regions;
}

// sizes: n_patches, n_patches_pad, PN (patch-node entries), E, max_pn, max_nv, n_slots
extern "C" void probe_sizes(int64_t* out) {
    out[0] = g_T.n_patches;
    out[1] = g_T.n_patches_pad;
    out[2] = (int64_t)g_T.patch_nodes.size();
    out[3] = (int64_t)g_T.elems.size();
    out[4] = g_T.max_pn;
    out[5] = g_T.max_nv;
    out[6] = g_T.slot_ptr.empty() ? 0 : g_T.slot_ptr.back();
}

extern "C" void probe_arrays(int32_t* el_ptr, int32_t* pn_ptr, int32_t* nv, uint32_t* nodes, int32_t* slot,
                             uint16_t* lids, int32_t* slot_ptr, int32_t* i2u) {
    std::memcpy(el_ptr, g_T.patch_el_ptr.data(), g_T.patch_el_ptr.size() * 4);
    std::memcpy(pn_ptr, g_T.patch_pn_ptr.data(), g_T.patch_pn_ptr.size() * 4);
    std::memcpy(nv, g_T.patch_nv.data(), g_T.patch_nv.size() * 4);
    std::memcpy(nodes, g_T.patch_nodes.data(), g_T.patch_nodes.size() * 4);
    std::memcpy(slot, g_T.patch_slot.data(), g_T.patch_slot.size() * 4);
    for (size_t k = 0; k < g_T.elems.size(); ++k)
        for (int i = 0; i < 10; ++i) lids[10 * k + i] = g_T.elems[k].lid[i];
    std::memcpy(slot_ptr, g_T.slot_ptr.data(), g_T.slot_ptr.size() * 4);
    std::memcpy(i2u, g_T.i2u.data(), g_T.i2u.size() * 4);
}

// Node chunks of the predictor regions given by region_start [nr + 1]; returns
// the number of chunks and fills chunk_start [C+1], chunk_region [C] and
// region_chunk [nr+1] when cap (the room in chunk_region) is large enough.
extern "C" int64_t probe_region_chunks(const int32_t* region_start, int32_t nr, int64_t cap, int32_t* chunk_start,
                                       int32_t* chunk_region, int32_t* region_chunk) {
    std::vector<int32_t> rs(region_start, region_start + nr + 1), cs, cr, rc;
    region_chunks(rs, cs, cr, rc);
    if ((int64_t)cr.size() <= cap) {
        std::memcpy(chunk_start, cs.data(), cs.size() * 4);
        std::memcpy(chunk_region, cr.data(), cr.size() * 4);
        std::memcpy(region_chunk, rc.data(), rc.size() * 4);
    }
    return (int64_t)cr.size();
}
