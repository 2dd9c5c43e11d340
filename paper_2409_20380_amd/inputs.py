"""Seeded synthetic inputs shared by the tests, the bench and the oracle runs.

This module only *generates problem data*: a layered box discretised by
second-order (10-node) tetrahedra, its material table, the fixed-bottom mask,
a partition of the nodes into predictor regions, and a band-limited random
base-acceleration record.  It holds none of the method's arithmetic (no
element integrals, no solver, no predictor): the oracle under ``oracle/`` and
the HIP library each compute everything else on their own.

Workload shapes follow the paper's application (Sec. 3.1): a horizontally
stratified elastic ground model (soft layer over stiffer layer), meshed with
quadratic tetrahedra, with the bottom fixed, driven by random waves.  The
paper's own ground models and impulse inputs are not available, so these
synthetic stand-ins are used instead.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

# Local node order of a 10-node tetrahedron used throughout the project:
# the four vertices, then the edge midpoints of edges (0,1),(1,2),(0,2),(0,3),(1,3),(2,3).
TET10_EDGES = ((0, 1), (1, 2), (0, 2), (0, 3), (1, 3), (2, 3))


# --------------------------------------------------------------------------
# Mesh
# --------------------------------------------------------------------------
def _kuhn_tets():
    """Six tetrahedra of the Kuhn (Freudenthal) split of the unit cube.

    Every tet runs from corner (0,0,0) to corner (1,1,1) along a monotone path
    of unit steps; the split is the same in every cell, so the mesh conforms.
    Vertices are returned as integer corner offsets, reordered so that each
    tet has positive orientation.
    """
    tets = []
    for perm in ((0, 1, 2), (1, 2, 0), (2, 0, 1), (0, 2, 1), (2, 1, 0), (1, 0, 2)):
        v0 = np.zeros(3, dtype=np.int64)
        v1 = v0.copy(); v1[perm[0]] = 1
        v2 = v1.copy(); v2[perm[1]] = 1
        v3 = np.ones(3, dtype=np.int64)
        verts = [v0, v1, v2, v3]
        det = np.linalg.det(np.stack([v1 - v0, v2 - v0, v3 - v0]).astype(float))
        if det < 0:
            verts = [v0, v2, v1, v3]
        tets.append(verts)
    return tets


@dataclasses.dataclass
class BoxMesh:
    nx: int
    ny: int
    nz: int
    h: float
    coords: np.ndarray      # [N,3] float64, metres; z is up, z=0 is the bottom
    conn: np.ndarray        # [E,10] int32, vertex ids then edge-midpoint ids
    lattice: np.ndarray     # [N,3] int64 index of each node on the half-cell lattice

    @property
    def n_nodes(self) -> int:
        return self.coords.shape[0]

    @property
    def n_elems(self) -> int:
        return self.conn.shape[0]


def box_mesh(nx: int, ny: int, nz: int, h: float = 2.5) -> BoxMesh:
    """nx*ny*nz cubic cells of edge h, each split into 6 straight 10-node tets.

    Nodes sit on the half-cell lattice, (2nx+1)(2ny+1)(2nz+1) of them, numbered
    x fastest, then y, then z.  Element vertices are cell corners; edge nodes
    are the lattice points halfway along each edge.
    """
    Lx, Ly, Lz = 2 * nx + 1, 2 * ny + 1, 2 * nz + 1
    ii, jj, kk = np.meshgrid(np.arange(Lx), np.arange(Ly), np.arange(Lz), indexing="ij")
    lat = np.stack([ii.ravel(order="F"), jj.ravel(order="F"), kk.ravel(order="F")], axis=1)
    # order: x fastest -> use Fortran ravel of an (x,y,z) grid
    node_id = lambda p: p[..., 0] + Lx * (p[..., 1] + Ly * p[..., 2])  # noqa: E731
    order = np.argsort(node_id(lat), kind="stable")
    lat = lat[order]
    coords = lat.astype(np.float64) * (h / 2.0)

    cx, cy, cz = np.meshgrid(np.arange(nx), np.arange(ny), np.arange(nz), indexing="ij")
    cells = np.stack([cx.ravel(order="F"), cy.ravel(order="F"), cz.ravel(order="F")], axis=1)
    cell_key = cells[:, 0] + nx * (cells[:, 1] + ny * cells[:, 2])
    cells = cells[np.argsort(cell_key, kind="stable")]

    tets = _kuhn_tets()
    conn = np.empty((cells.shape[0], 6, 10), dtype=np.int64)
    for t, verts in enumerate(tets):
        vlat = [2 * cells + 2 * v[None, :] for v in verts]      # vertex lattice coords
        ids = [node_id(v) for v in vlat]
        for m, (a, b) in enumerate(TET10_EDGES):
            ids.append(node_id((vlat[a] + vlat[b]) // 2))
        conn[:, t, :] = np.stack(ids, axis=1)
    conn = conn.reshape(-1, 10).astype(np.int32)
    return BoxMesh(nx, ny, nz, h, coords, conn, lat)


# --------------------------------------------------------------------------
# Materials, boundary, regions
# --------------------------------------------------------------------------
@dataclasses.dataclass
class Layer:
    vs: float
    rho: float
    vp_over_vs: float = 1.9

    def row(self):
        return (self.rho, self.vp_over_vs * self.vs, self.vs)


DEFAULT_LAYERS = (Layer(vs=400.0, rho=2000.0), Layer(vs=200.0, rho=1800.0))  # bottom, top


def two_layer_materials(mesh: BoxMesh, layers=DEFAULT_LAYERS):
    """Material id per element by centroid depth: lower half of the box gets
    layers[0] (bedrock-like), upper half layers[1] (sediment-like).

    Returns (elem_mat int32 [E], mat float64 [n_mat,3] with columns rho, vp, vs).
    """
    zc = mesh.coords[mesh.conn[:, :4], 2].mean(axis=1)
    z_split = 0.5 * mesh.nz * mesh.h
    elem_mat = (zc > z_split).astype(np.int32)
    mat = np.array([ly.row() for ly in layers], dtype=np.float64)
    return elem_mat, mat


def fixed_bottom(mesh: BoxMesh) -> np.ndarray:
    """uint8 [N,3]: 1 where the displacement component is fixed (z = 0 face)."""
    fixed = np.zeros((mesh.n_nodes, 3), dtype=np.uint8)
    fixed[mesh.lattice[:, 2] == 0, :] = 1
    return fixed


def _split(n: int, b: int):
    """Block boundaries of [0,n) in chunks of b, the remainder merged into the last."""
    nb = max(1, n // b)
    edges = [i * b for i in range(nb)] + [n]
    return np.asarray(edges)


def block_regions(mesh: BoxMesh, block: int = 8) -> np.ndarray:
    """Predictor regions: blocks of block^3 lattice nodes (512 for block=8).

    Returns int32 [N] region id per node; a short remainder along an axis is
    merged into the last block so no region is thin.
    """
    out = np.empty(mesh.n_nodes, dtype=np.int64)
    Ls = [2 * mesh.nx + 1, 2 * mesh.ny + 1, 2 * mesh.nz + 1]
    ids = []
    for d in range(3):
        e = _split(Ls[d], block)
        ids.append(np.searchsorted(e, mesh.lattice[:, d], side="right") - 1)
    nb = [len(_split(L, block)) - 1 for L in Ls]
    out[:] = ids[0] + nb[0] * (ids[1] + nb[1] * ids[2])
    return out.astype(np.int32)


# --------------------------------------------------------------------------
# Input wave
# --------------------------------------------------------------------------
def base_wave(seed: int, nt: int, dt: float, f_lo: float = 0.1, f_hi: float = 2.5,
              ng: int = 8192, ramp_s: float = 0.2) -> np.ndarray:
    """Seeded band-limited Gaussian base acceleration, shape [nt+1, 3] (m/s^2).

    For each component k: ng standard normals from default_rng([seed, k]),
    zero every Fourier bin outside [f_lo, f_hi] Hz, scale to unit RMS, take the
    first nt+1 samples (t = 0, dt, ...), and taper the first ramp_s seconds
    with sin^2 so the record starts from rest (g(0) = 0).
    """
    n = max(ng, nt + 1)
    out = np.empty((nt + 1, 3), dtype=np.float64)
    freqs = np.fft.rfftfreq(n, d=dt)
    band = (freqs >= f_lo) & (freqs <= f_hi)
    t = np.arange(nt + 1) * dt
    ramp = np.where(t < ramp_s, np.sin(0.5 * np.pi * np.clip(t / ramp_s, 0, 1)) ** 2, 1.0)
    for k in range(3):
        rng = np.random.default_rng([seed, k])
        w = rng.standard_normal(n)
        W = np.fft.rfft(w)
        W[~band] = 0.0
        g = np.fft.irfft(W, n=n)
        g /= math.sqrt(np.mean(g * g))
        out[:, k] = g[: nt + 1] * ramp
    return out


def surface_impulses(mesh: BoxMesh, seed: int, nt: int, dt: float, n_points: int = 284,
                     f_lo: float = 0.1, f_hi: float = 2.5, onset_s: float = 0.5, ng: int = 8192):
    """Paper-like point forces: impulses with random amplitudes and flat spectra in
    random directions at randomly chosen points of the ground surface, after which
    the body vibrates freely (the paper's application, Sec. 3.1).

    n_points distinct top-surface nodes (284 keeps the paper's 10,000 points per
    950 x 950 m of surface on a 160 x 160 m top); each gets a unit impulse
    band-passed to [f_lo, f_hi] Hz (flat amplitude spectrum in the band), centred
    at 1 s plus a uniform random onset in [0, onset_s] s and windowed by a
    Gaussian of 0.4 s standard deviation (so the pulse has decayed before t = 0
    and ends within about 3 s), times a standard-normal amplitude, along a
    uniformly random unit direction.  Returns (nodes int32 [K], force float64
    [nt + 1][K][3], t = 0, dt, ...); force 0 at t = 0 by a sin^2 taper over 0.2 s.
    """
    rng = np.random.default_rng([seed, 6007])
    top = np.where(mesh.lattice[:, 2] == 2 * mesh.nz)[0]
    k = min(n_points, top.size)
    nodes = np.sort(rng.choice(top, size=k, replace=False)).astype(np.int32)
    amp = rng.standard_normal(k)
    d = rng.standard_normal((k, 3))
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    onset = 1.0 + rng.uniform(0.0, onset_s, size=k)
    n = max(ng, nt + 1)
    freqs = np.fft.rfftfreq(n, d=dt)
    band = (freqs >= f_lo) & (freqs <= f_hi)
    t = np.arange(nt + 1) * dt
    ramp = np.where(t < 0.2, np.sin(0.5 * np.pi * np.clip(t / 0.2, 0, 1)) ** 2, 1.0)
    tt = np.arange(n) * dt
    force = np.zeros((nt + 1, k, 3))
    for p in range(k):
        spec = np.where(band, np.exp(-2j * np.pi * freqs * onset[p]), 0.0)
        pulse = np.fft.irfft(spec, n=n) * np.exp(-0.5 * ((tt - onset[p]) / 0.4) ** 2)
        pulse /= np.abs(pulse).max()
        force[:, p, :] = (amp[p] * pulse[: nt + 1] * ramp)[:, None] * d[p][None, :]
    return nodes, force


def random_vector(seed: int, n: int) -> np.ndarray:
    """Seeded standard-normal float64 vector (parity-test operand)."""
    return np.random.default_rng([seed, 7919]).standard_normal(n)


# --------------------------------------------------------------------------
# Random draws of the learned predictor (passed to the library as inputs)
# --------------------------------------------------------------------------
MLP_SHAPES = ((64, 15), (64,), (64, 64), (64,), (3, 64), (3,))


def mlp_init(seed: int, gain: float = 1.0) -> np.ndarray:
    """Glorot-uniform weights and zero biases, flattened W1, b1, W2, b2, W3, b3 (float32)."""
    rng = np.random.default_rng([seed, 4099])
    parts = []
    for shape in MLP_SHAPES:
        if len(shape) == 2:
            lim = gain * math.sqrt(6.0 / (shape[0] + shape[1]))
            parts.append(rng.uniform(-lim, lim, size=shape).ravel())
        else:
            parts.append(np.zeros(shape))
    return np.concatenate(parts).astype(np.float32)


def minibatches(seed: int, steps: int, batch: int, count: int) -> np.ndarray:
    """Sample indices [steps][batch] drawn uniformly from 0..count-1 (int64)."""
    rng = np.random.default_rng([seed, 8191])
    return rng.integers(0, count, size=(steps, batch), dtype=np.int64)


def sample_nodes(seed: int, fixed: np.ndarray, k: int) -> np.ndarray:
    """k distinct nodes with no fixed component (int32, sorted)."""
    free = np.where(fixed.reshape(-1, 3).max(axis=1) == 0)[0]
    rng = np.random.default_rng([seed, 131])
    k = min(k, free.size)
    return np.sort(rng.choice(free, size=k, replace=False)).astype(np.int32)


# --------------------------------------------------------------------------
# Workloads
# --------------------------------------------------------------------------
def rayleigh_coefficients(zeta: float, f1: float, f2: float):
    """Mass/stiffness-proportional damping giving ratio zeta at f1 and f2 (Hz)."""
    w1, w2 = 2 * math.pi * f1, 2 * math.pi * f2
    return 2 * zeta * w1 * w2 / (w1 + w2), 2 * zeta / (w1 + w2)


@dataclasses.dataclass
class Workload:
    name: str
    cells: tuple
    h: float = 2.5
    dt: float = 0.01
    nt: int = 100
    s: int = 16
    tol: float = 1e-8
    seed: int = 0
    zeta: float = 0.05
    f_band: tuple = (0.1, 2.5)
    region_block: int = 8
    region_merge: int = 1   # given regions per predictor region (the library's region_merge)

    @property
    def rayleigh(self):
        return rayleigh_coefficients(self.zeta, *self.f_band)

    def build(self):
        """Mesh, materials, mask, regions and wave for this workload."""
        mesh = box_mesh(*self.cells, h=self.h)
        elem_mat, mat = two_layer_materials(mesh)
        fixed = fixed_bottom(mesh)
        regions = block_regions(mesh, self.region_block)
        wave = base_wave(self.seed, self.nt, self.dt, *self.f_band)
        return mesh, elem_mat, mat, fixed, regions, wave


# The small case the oracle finishes in seconds, the single-GPU headline case,
# and the large mesh of the mixed-precision comparison (8.5M nodes, 25.6M dof).
SMALL = Workload("box8x8x8_p2tet_fp64", cells=(8, 8, 8), nt=100, s=16)
# learned predictor: training and test waves of the headline mesh
LEARN_TRAIN_SEEDS = tuple(range(100, 150))
LEARN_TEST_SEEDS = tuple(range(200, 232))
PLAIN = Workload("box64x64x32_p2tet_fp64", cells=(64, 64, 32), nt=1000, s=32, region_merge=27)
LARGE = Workload("box128x128x64_p2tet", cells=(128, 128, 64), nt=300, s=32, region_merge=27)
WORKLOADS = {"plain": PLAIN, "large": LARGE, "small": SMALL}
# batched ensemble: (cells, cases) per mesh; cases take seeds 1..64 in order
ENSEMBLE = (((16, 16, 8), 20), ((32, 32, 16), 24), ((48, 48, 24), 20))
ENSEMBLE_STEPS, ENSEMBLE_S = 500, 32
ENSEMBLE_REGION_MERGE = 27   # as the single-mesh workloads: runs of 27 blocks of 8^3 lattice nodes
