// topology.h -- host-side mesh preprocessing for the element-by-element
// kernels: internal node order, element patches, patch-local numbering and
// the per-node list of patch slots that the matvec writes.
#pragma once
#include <cstdint>
#include <string>
#include <vector>

namespace ebe {

// Bit set on a patch-node entry when that patch is the first (owner) patch of
// the node: the owner writes per-node values that every touching patch computes.
constexpr uint32_t kOwnerBit = 0x80000000u;
constexpr int kMaxPatchElems = 256;  // one element per thread of a 256-thread workgroup

// Element record used by the kernels: ten patch-local node indices (vertices
// first, then edges in the conn order), the material id and one pad word.
struct ElemRec {
    uint16_t lid[10];
    uint16_t mat;
    uint16_t pad;
};
static_assert(sizeof(ElemRec) == 24, "ElemRec must be 24 bytes");

struct Topology {
    int64_t n_nodes = 0, n_elems = 0;
    int32_t n_regions = 0;
    // node numbering
    std::vector<int32_t> i2u, u2i;          // internal -> user, user -> internal
    std::vector<int32_t> region_user;       // region id per user node
    std::vector<int32_t> region_start;      // [n_regions+1] internal node ranges
    std::vector<int32_t> chunk_start, chunk_region, region_chunk;   // region_chunks(region_start)
    std::vector<double> coords;             // [N][3] internal order
    std::vector<uint8_t> fixmask;           // [N] bit c = component c fixed, internal order
    // patches
    int32_t n_patches = 0, n_patches_pad = 0;   // pad = multiple of 8 (XCD count)
    std::vector<int32_t> patch_el_ptr;      // [Ppad+1] element ranges (internal element order)
    std::vector<int32_t> patch_pn_ptr;      // [Ppad+1] patch-node ranges
    std::vector<int32_t> patch_nv;          // [Ppad] number of vertex nodes (local ids < nv)
    std::vector<uint32_t> patch_nodes;      // [PN] internal node id | kOwnerBit
    std::vector<ElemRec> elems;             // [E] internal element order
    int32_t max_pn = 0, max_nv = 0;
    // Slots: every (patch, node) pair owns one 3-vector of the matvec output.
    // Slots are numbered node-major: node n owns [slot_ptr[n], slot_ptr[n+1]),
    // one per touching patch in patch order; patch_slot[pn] is the slot that
    // patch-node pn writes.
    std::vector<int32_t> slot_ptr;          // [N+1]
    std::vector<int32_t> patch_slot;        // [PN]
    // material table: lambda, mu, rho
    std::vector<double> mat_lmr;
};

// The predictor's Gram and apply passes work on node chunks of the regions, so
// that their parallelism does not depend on the region size: a region of n
// nodes is cut into min(kMaxRegionChunks, ceil(n / kChunkNodes)) chunks of
// near-equal length.  Outputs: chunk_start [C+1] internal node ranges,
// chunk_region [C] region of each chunk, region_chunk [R+1] first chunk of
// each region.  Chunks of one region are consecutive.
constexpr int kChunkNodes = 512;
constexpr int kMaxRegionChunks = 64;
void region_chunks(const std::vector<int32_t>& region_start, std::vector<int32_t>& chunk_start,
                   std::vector<int32_t>& chunk_region, std::vector<int32_t>& region_chunk);

// LDS bytes that a patch needs in the element kernels: fixed + per_node * (patch
// nodes) + per_vertex * (vertex nodes).  A patch is closed before it would
// exceed budget (budget <= 0: no limit), so that the kernels keep the number
// of resident workgroups per CU the budget was chosen for.
struct PatchLds {
    int64_t per_node = 0, per_vertex = 0, fixed = 0, budget = 0;
};

// Builds the topology; returns an empty string on success or an error message.
// Patches take consecutive elements of the spatial element order, at most
// patch_elems of them and within lds.  region_merge > 1 merges the given
// regions, in Morton order of their centroids, region_merge at a time into
// the predictor's regions (T.region_user); the given regions still order the
// nodes.
std::string build_topology(Topology& T, int64_t n_nodes, const double* coords, int64_t n_elems,
                           const int32_t* conn, const int32_t* elem_mat, int32_t n_mat, const double* mat,
                           const uint8_t* fixed, const int32_t* region_of_node, int region_nodes,
                           int patch_elems, const PatchLds& lds = PatchLds(), int region_merge = 1);

}  // namespace ebe
