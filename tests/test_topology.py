"""Host-side patch topology of the element kernels (paper_2409_20380_amd/csrc/topology.cpp), on the CPU.

The element kernels stage each patch's nodes in LDS under patch-local ids; the
ids are spread over the LDS bank pairs that an FP64 LDS atomic services
together (8 lanes, 16 bank pairs on gfx950), by exchanging ids only between
nodes of the same kind inside an aligned block of 64 ids.  These tests build
the topology through a small probe compiled from the library's own source and
check what the kernels rely on: every element appears once with its exact
nodes, vertices keep the id prefix [0, nv), ids stay in their 64-id block,
owner bits and node-major slots are consistent, and the bank conflicts of the
atomics are actually reduced.
"""
import ctypes as C
import os
import shutil
import subprocess
import tempfile
import types

import numpy as np
import pytest

from paper_2409_20380_amd import inputs

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2409_20380_amd", "csrc")
OWNER = 0x80000000


@pytest.fixture(scope="module")
def probe():
    gxx = shutil.which("g++")
    if not gxx:
        pytest.skip("no host C++ compiler")
    d = tempfile.mkdtemp(prefix="topo_probe_")
    so = os.path.join(d, "libprobe.so")
    subprocess.check_call([gxx, "-O2", "-std=c++17", "-shared", "-fPIC", "-I", CSRC,
                           os.path.join(ROOT, "tests", "topology_probe.cpp"), os.path.join(CSRC, "topology.cpp"),
                           "-o", so])
    yield C.CDLL(so)
    shutil.rmtree(d, ignore_errors=True)


def build(probe, wl, patch_elems=256, lds=None):
    mesh, em, mat, fx, regions, _ = wl.build()
    a = lambda x, t: np.ascontiguousarray(x, dtype=t)
    P = lambda x: x.ctypes.data_as(C.c_void_p)
    xyz, conn, emm, matt = a(mesh.coords, np.float64), a(mesh.conn, np.int32), a(em, np.int32), a(mat, np.float64)
    fxx, reg = a(fx, np.uint8), a(regions, np.int32)
    args = (C.c_int64(mesh.n_nodes), P(xyz), C.c_int64(len(conn)), P(conn), P(emm), C.c_int(len(matt)), P(matt),
            P(fxx), P(reg), C.c_int(512), C.c_int(patch_elems))
    if lds is None:
        rc = probe.probe_build(*args)
    else:
        rc = probe.probe_build_lds(*args, *(C.c_int64(v) for v in lds))
    assert rc == 0
    sz = np.zeros(7, np.int64)
    probe.probe_sizes(P(sz))
    npat, ppad, pn, ne, max_pn, max_nv, nslot = (int(v) for v in sz)
    el_ptr = np.zeros(ppad + 1, np.int32); pn_ptr = np.zeros(ppad + 1, np.int32); nv = np.zeros(ppad, np.int32)
    nodes = np.zeros(pn, np.uint32); slot = np.zeros(pn, np.int32); lids = np.zeros((ne, 10), np.uint16)
    slot_ptr = np.zeros(mesh.n_nodes + 1, np.int32); i2u = np.zeros(mesh.n_nodes, np.int32)
    probe.probe_arrays(P(el_ptr), P(pn_ptr), P(nv), P(nodes), P(slot), P(lids), P(slot_ptr), P(i2u))
    return dict(conn=conn, n=mesh.n_nodes, npat=npat, ppad=ppad, el_ptr=el_ptr, pn_ptr=pn_ptr, nv=nv, nodes=nodes,
                slot=slot, lids=lids, slot_ptr=slot_ptr, i2u=i2u, max_pn=max_pn, patch_elems=patch_elems)


def patches(t):
    for p in range(t["ppad"]):
        e0, e1 = t["el_ptr"][p], t["el_ptr"][p + 1]
        n0, n1 = t["pn_ptr"][p], t["pn_ptr"][p + 1]
        yield p, e0, e1, n0, n1


def bank_multiplicity(lids, lane_group=8, bank_pairs=16):
    """Mean over (group of 8 consecutive elements, element position) of the largest number of
    lanes whose accumulator double 3 l + c falls on one bank pair."""
    worst = []
    for g0 in range(0, len(lids), lane_group):
        grp = lids[g0:g0 + lane_group].astype(np.int64)
        for i in range(10):
            worst.append(np.bincount((3 * grp[:, i]) % bank_pairs, minlength=bank_pairs).max())
    return float(np.mean(worst))


class OneTet:
    """A single straight 10-node tet (vertices, then edges 01, 12, 02, 03, 13, 23): one patch of one element."""

    @staticmethod
    def build():
        v = np.array([[0.0, 0.0, 0.0], [2.5, 0.0, 0.0], [0.0, 2.5, 0.0], [0.0, 0.0, 2.5]])
        edges = [(0, 1), (1, 2), (0, 2), (0, 3), (1, 3), (2, 3)]
        coords = np.vstack([v] + [0.5 * (v[a] + v[b]) for a, b in edges])
        mesh = types.SimpleNamespace(coords=coords, conn=np.arange(10, dtype=np.int32)[None, :], n_nodes=10)
        fixed = np.zeros((10, 3), np.uint8)
        fixed[0] = 1
        return (mesh, np.zeros(1, np.int32), np.array([[1800.0, 380.0, 200.0]]), fixed, np.zeros(10, np.int32),
                None)


CASES = [(inputs.SMALL, 256), (inputs.SMALL, 64),
         (inputs.Workload("box3x5x2_ragged", cells=(3, 5, 2), nt=30, s=6, region_block=4), 256),
         (OneTet, 256), (inputs.Workload("box1x1x1", cells=(1, 1, 1), nt=1, s=1), 1)]


@pytest.mark.parametrize("wl,pe", CASES, ids=["8x8x8_256", "8x8x8_64", "3x5x2_256", "one_tet", "1x1x1_1"])
def test_patch_topology_invariants(probe, wl, pe):
    t = build(probe, wl, pe)
    conn = t["conn"]
    want = {}
    for e, row in enumerate(conn):
        want.setdefault(tuple(int(v) for v in row), []).append(e)
    seen = {}
    owners = np.zeros(t["n"], np.int64)
    patches_of = [[] for _ in range(t["n"])]
    assert t["ppad"] % 8 == 0 and t["ppad"] >= t["npat"]
    for p, e0, e1, n0, n1 in patches(t):
        assert e1 - e0 <= pe
        ent = t["nodes"][n0:n1]
        internal = (ent & ~np.uint32(OWNER)).astype(np.int64)
        npn, nv = n1 - n0, int(t["nv"][p])
        assert npn <= t["max_pn"] and len(set(internal.tolist())) == npn
        used = np.zeros(npn, bool)
        for k in range(e0, e1):
            lid = t["lids"][k].astype(np.int64)
            assert (lid < npn).all()
            assert (lid[:4] < nv).all() and (lid[4:] >= nv).all()   # vertices first
            used[lid] = True
            key = tuple(int(t["i2u"][internal[l]]) for l in lid)     # element nodes in connectivity order
            assert key in want, (p, k)
            seen[key] = seen.get(key, 0) + 1
        assert used.all()   # the patch lists exactly its elements' nodes
        for l, v in enumerate(internal):
            patches_of[v].append(p)
            if ent[l] & OWNER:
                owners[v] += 1
                assert len(patches_of[v]) == 1   # owner = first patch of the node
        # ids move only inside their aligned 64-id block (same kind): the unspread numbering is
        # vertices by internal id, then edge nodes by internal id
        order = np.concatenate([np.sort(internal[:nv]), np.sort(internal[nv:])])
        pos = {int(v): i for i, v in enumerate(order)}
        for new_id, v in enumerate(internal):
            assert pos[int(v)] // 64 == new_id // 64
    assert all(seen.get(k, 0) == len(v) for k, v in want.items()) and sum(seen.values()) == len(conn)
    assert (owners == 1).all()
    counts = np.diff(t["slot_ptr"])
    assert (counts == np.array([len(x) for x in patches_of])).all() and t["slot_ptr"][-1] == len(t["nodes"])
    for p, e0, e1, n0, n1 in patches(t):   # node-major slots in patch order
        for l in range(n0, n1):
            v = int(t["nodes"][l] & ~np.uint32(OWNER))
            assert t["slot"][l] == t["slot_ptr"][v] + patches_of[v].index(p)


def test_bank_spreading_reduces_conflicts(probe):
    """Full 256-element patches of the 8x8x8 mesh: the spread ids put the 8 lanes of an atomic on distinct
    bank pairs far more often than the plain (sorted) numbering of the same patches would."""
    t = build(probe, inputs.SMALL, 256)
    spread, plain = [], []
    for p, e0, e1, n0, n1 in patches(t):
        if e1 - e0 < 256:
            continue
        internal = (t["nodes"][n0:n1] & ~np.uint32(OWNER)).astype(np.int64)
        nv = int(t["nv"][p])
        order = np.concatenate([np.sort(internal[:nv]), np.sort(internal[nv:])])
        pos = {int(v): i for i, v in enumerate(order)}
        lids = t["lids"][e0:e1].astype(np.int64)
        plain_lids = np.vectorize(lambda l: pos[int(internal[l])])(lids)
        spread.append(bank_multiplicity(lids))
        plain.append(bank_multiplicity(plain_lids))
    assert spread, "no full patch"
    assert np.mean(spread) < 1.25, np.mean(spread)
    assert np.mean(spread) < np.mean(plain) - 0.5, (np.mean(spread), np.mean(plain))


@pytest.mark.parametrize("sizes", [[512], [513], [1], [614, 614, 615], [4096, 100, 1024 * 512 + 7], [1081665]],
                         ids=["512", "513", "1", "3x614", "mixed", "one_global"])
def test_region_chunks(probe, sizes):
    """The predictor's node chunks tile each region with consecutive ranges of near-equal length: at most
    512 nodes each, unless the region needs more than 64 chunks, then 64 equal ones."""
    rs = np.concatenate([[0], np.cumsum(sizes)]).astype(np.int32)
    P = lambda x: x.ctypes.data_as(C.c_void_p)
    probe.probe_region_chunks.restype = C.c_int64
    n = probe.probe_region_chunks(P(rs), C.c_int32(len(sizes)), C.c_int64(0), None, None, None)
    cs, cr, rc = np.zeros(n + 1, np.int32), np.zeros(n, np.int32), np.zeros(len(sizes) + 1, np.int32)
    assert probe.probe_region_chunks(P(rs), C.c_int32(len(sizes)), C.c_int64(n), P(cs), P(cr), P(rc)) == n
    assert cs[0] == 0 and cs[-1] == rs[-1] and (np.diff(cs) > 0).all()
    assert rc[0] == 0 and rc[-1] == n
    for r, size in enumerate(sizes):
        c0, c1 = rc[r], rc[r + 1]
        assert cs[c0] == rs[r] and cs[c1] == rs[r + 1]
        assert (cr[c0:c1] == r).all()
        lens = np.diff(cs[c0:c1 + 1])
        want = min(64, -(-size // 512))
        assert c1 - c0 == want
        assert lens.max() - lens.min() <= 1
        if want < 64:
            assert lens.max() <= 512


# per node, per vertex node, fixed bytes: the FP64 element pass (four wave accumulators and one operand per
# node, vertex coordinates, a two-row material table)
LDS_COEF = (120, 24, 48)


@pytest.mark.parametrize("budget", [81920, 40000, 20000])
def test_patch_lds_budget(probe, budget):
    """The kernels size LDS by the largest node count and the largest vertex count over all patches; the
    builder closes a patch before that combined size would exceed the budget.  With a budget the natural
    256-element patches fit, nothing changes."""
    per_node, per_vertex, fixed_b = LDS_COEF
    free = build(probe, inputs.SMALL, 256)
    t = build(probe, inputs.SMALL, 256, lds=(per_node, per_vertex, fixed_b, budget))
    sizes = [(n1 - n0, int(t["nv"][p])) for p, e0, e1, n0, n1 in patches(t)]
    combined = lambda sz: fixed_b + per_node * max(n for n, v in sz) + per_vertex * max(v for n, v in sz)
    assert combined(sizes) <= budget
    counts = [e1 - e0 for p, e0, e1, n0, n1 in patches(t) if e1 > e0]
    assert sum(counts) == len(t["conn"]) and max(counts) <= 256
    natural = combined([(n1 - n0, int(free["nv"][p])) for p, e0, e1, n0, n1 in patches(free)])
    if natural <= budget:
        assert t["npat"] == free["npat"] and (t["el_ptr"] == free["el_ptr"]).all()
    else:
        assert t["npat"] > free["npat"]
        # a patch is closed only when the next element would raise the combined size past the budget
        conn, i2u = t["conn"], t["i2u"]
        max_n = max_v = 0
        for p, e0, e1, n0, n1 in patches(t):
            if p + 1 >= t["npat"]:
                continue
            if e1 - e0 < 256:
                ent = t["nodes"][n0:n1] & ~np.uint32(OWNER)
                users = set(int(i2u[v]) for v in ent)
                nxt = t["lids"][e1]   # local ids of the next patch's first element, in the next patch
                m0, m1 = t["pn_ptr"][p + 1], t["pn_ptr"][p + 2]
                nxt_users = [int(i2u[int(t["nodes"][m0 + int(l)] & ~np.uint32(OWNER))]) for l in nxt]
                add = [u for u in nxt_users if u not in users]
                add_v = sum(1 for i, u in enumerate(nxt_users) if u not in users and i < 4)
                assert (fixed_b + per_node * max(max_n, n1 - n0 + len(add)) +
                        per_vertex * max(max_v, int(t["nv"][p]) + add_v)) > budget
            max_n, max_v = max(max_n, n1 - n0), max(max_v, int(t["nv"][p]))


def _morton_codes(p, lo, hi):
    """Morton codes of points p [n, 3] in the box [lo, hi] (21 bits per axis, x in the lowest bit)."""
    t = np.where(hi > lo, (p - lo) / np.where(hi > lo, hi - lo, 1.0), 0.0)
    q = np.clip(np.floor(t * 2097151.0), 0, 2097151).astype(np.uint64)
    out = np.zeros(len(p), np.uint64)
    for b in range(21):
        for d in range(3):
            out |= ((q[:, d] >> np.uint64(b)) & np.uint64(1)) << np.uint64(3 * b + d)
    return out


@pytest.mark.parametrize("merge,own", [(2, False), (3, False), (8, False), (4, True)])
def test_region_merge(probe, merge, own):
    """Merged predictor regions: the given regions (or, with no region map, the library's own regions of
    region_nodes nodes), ordered by the Morton code of their centroids, merged `merge` at a time; each
    merged region is one contiguous range of the internal order; the patches are as compact as without
    merging (the given regions still order the nodes)."""
    wl = inputs.Workload("box8x8x8_rb4", cells=(8, 8, 8), nt=1, s=1, region_block=4)
    mesh, em, mat, fx, given, _ = wl.build()
    a = lambda x, t: np.ascontiguousarray(x, dtype=t)
    P = lambda x: x.ctypes.data_as(C.c_void_p)
    xyz, conn = a(mesh.coords, np.float64), a(mesh.conn, np.int32)
    reg = None if own else P(a(given, np.int32))
    args = lambda m: (C.c_int64(mesh.n_nodes), P(xyz), C.c_int64(len(conn)), P(conn), P(a(em, np.int32)),
                      C.c_int(len(mat)), P(a(mat, np.float64)), P(a(fx, np.uint8)), reg,
                      C.c_int(128), C.c_int(256), *(C.c_int64(v) for v in (120, 24, 48, 81920)), C.c_int(m))
    if own:   # the library's own regions: Morton chunks of 128 nodes, as built without merging
        assert probe.probe_build_merge(*args(1)) == 0
        given = np.zeros(mesh.n_nodes, np.int32)
        rs0 = np.zeros(mesh.n_nodes + 2, np.int32)
        probe.probe_regions(P(given), P(rs0), C.c_int32(len(rs0)))
    R = int(given.max()) + 1
    stats = {}
    for m in (1, merge):
        assert probe.probe_build_merge(*args(m)) == 0
        ru = np.zeros(mesh.n_nodes, np.int32)
        rs = np.zeros(R + 2, np.int32)
        nr = probe.probe_regions(P(ru), P(rs), C.c_int32(R + 2))
        assert nr <= R
        sz = np.zeros(7, np.int64)
        probe.probe_sizes(P(sz))
        i2u = np.zeros(mesh.n_nodes, np.int32)
        el_ptr = np.zeros(sz[1] + 1, np.int32); pn_ptr = np.zeros(sz[1] + 1, np.int32); nv = np.zeros(sz[1], np.int32)
        nodes = np.zeros(sz[2], np.uint32); slot = np.zeros(sz[2], np.int32); lids = np.zeros((sz[3], 10), np.uint16)
        slot_ptr = np.zeros(mesh.n_nodes + 1, np.int32)
        probe.probe_arrays(P(el_ptr), P(pn_ptr), P(nv), P(nodes), P(slot), P(lids), P(slot_ptr), P(i2u))
        stats[m] = (nr, ru.copy(), rs[:nr + 1].copy(), i2u.copy(), sz[2] / mesh.n_nodes)
    nr1, ru1, _, _, slots1 = stats[1]
    assert nr1 == R and (ru1 == given).all()
    nr, ru, rs, i2u, slots = stats[merge]
    assert nr == (R + merge - 1) // merge
    # the given regions in Morton order of their centroids, merged `merge` at a time
    cen = np.array([mesh.coords[given == r].mean(0) for r in range(R)])
    lo, hi = mesh.coords.min(0), mesh.coords.max(0)
    order = np.argsort(_morton_codes(cen, lo, hi), kind="stable")
    want = np.empty(R, np.int64)
    want[order] = np.arange(R) // merge
    assert (ru == want[given]).all()
    # contiguous ranges of the internal order
    assert rs[0] == 0 and rs[-1] == mesh.n_nodes
    for r in range(nr):
        assert (ru[i2u[rs[r]:rs[r + 1]]] == r).all()
    assert slots <= 1.02 * slots1
