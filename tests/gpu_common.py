"""Shared helpers of the GPU parity tests (CPU oracle vs HIP library)."""
import math

import numpy as np

from paper_2409_20380_amd import inputs


def cm_ck(dt, aR, bR):
    """Coefficients of the Newmark system matrix A = cM M + cK K (average
    acceleration with Rayleigh damping C = aR M + bR K)."""
    return 4.0 / dt ** 2 + 2.0 * aR / dt, 1.0 + 2.0 * bR / dt


def torch_cuda():
    import torch
    assert torch.cuda.is_available(), "GPU test run without a GPU"
    return torch


def to_dev(a):
    torch = torch_cuda()
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).cuda()


def to_host(t):
    return t.detach().cpu().numpy()


def rel_max(a, b):
    return float(np.abs(a - b).max() / max(np.abs(b).max(), 1e-300))


def build_case(wl, oracle_lib, **solver_kw):
    """Mesh + oracle model + GPU solver for a workload."""
    from paper_2409_20380_amd import ebe
    mesh, em, mat, fx, regions, wave = wl.build()
    aR, bR = wl.rayleigh
    cM, cK = cm_ck(wl.dt, aR, bR)
    model = oracle_lib.Model(mesh.coords, mesh.conn, em, mat, fx, cM, cK)
    kw = dict(s=wl.s, tol=wl.tol)
    kw.update(solver_kw)
    sol = ebe.Solver(wl.dt, aR, bR, **kw)
    sol.assemble(mesh.coords, mesh.conn, em, mat, fx, regions)
    return dict(mesh=mesh, em=em, mat=mat, fx=fx, regions=regions, wave=wave, aR=aR, bR=bR, cM=cM, cK=cK,
                model=model, sol=sol, wl=wl)


def node_elements(conn, n_nodes):
    """CSR node -> elements map."""
    cnt = np.bincount(conn.ravel(), minlength=n_nodes)
    ptr = np.zeros(n_nodes + 1, dtype=np.int64)
    ptr[1:] = np.cumsum(cnt)
    order = np.argsort(conn.ravel(), kind="stable")
    elems = order // 10
    return ptr, elems


def sampled_rows(oracle_lib, mesh, em, mat, fixed, cM, cK, p, nodes):
    """Rows of A_bc p at the given nodes, from oracle element matrices one by one."""
    ptr, elems = node_elements(mesh.conn, mesh.n_nodes)
    free = (fixed == 0).astype(np.float64)           # [N,3]
    pz = p.reshape(-1, 3) * free
    out = np.zeros((len(nodes), 3))
    for t, n in enumerate(nodes):
        acc = np.zeros(3)
        for e in elems[ptr[n]:ptr[n + 1]]:
            c = mesh.conn[e]
            rho, vp, vs = mat[em[e]]
            mu = rho * vs * vs
            lam = rho * (vp * vp - 2 * vs * vs)
            Ke, Me, V = oracle_lib.element_matrices(mesh.coords[c[:4]], lam, mu, rho)
            Ae = cM * Me + cK * Ke
            loc = int(np.where(c == n)[0][0])
            acc += Ae[3 * loc:3 * loc + 3] @ pz[c].ravel()
        for k in range(3):
            out[t, k] = p.reshape(-1, 3)[n, k] if fixed[n, k] else acc[k]
    return out


def history_columns(ring, it, s):
    """Snapshot columns for step n = it+1 under the ring convention e^j in slot (j-1) mod (s+1)."""
    n = it + 1
    s_eff = min(s, n - 2)
    S1 = s + 1
    X = [ring[(n - s_eff - 1 + j - 1) % S1] for j in range(s_eff)]
    Y = [ring[(n - s_eff - 1 + j) % S1] for j in range(s_eff)]
    q = ring[(n - 2) % S1]
    return X, Y, q, s_eff


SMALL = inputs.SMALL
RAGGED = inputs.Workload("box3x5x2_ragged", cells=(3, 5, 2), nt=30, s=6, region_block=4)
# the same 8x8x8-cell lattice with 1/8 m cells (a 1 m box): a correctness-only case whose
# condition number is about 400 times that of the 2.5 m cells (hundreds of trips per step)
LITERAL = inputs.Workload("box8x8x8_h0.125", cells=(8, 8, 8), h=0.125, nt=40, s=16)
