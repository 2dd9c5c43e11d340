"""Batched ensembles on the GPU against the FP64 oracle (needs an MI355X).

Every case of a batch is checked against its own single-case oracle
trajectory: the batch shares element passes between cases but each case runs
its own CG, so each result must meet the plain path's bars (space-time
relative L2 error <= 1e-6 against the tight oracle, true residual < 1e-8 every
step, iteration counts within 2 trips of the oracle's at the same
tolerance).
"""
import numpy as np
import pytest

from paper_2409_20380_amd import inputs
from tests.gpu_common import RAGGED, SMALL, cm_ck, to_dev, to_host

pytestmark = pytest.mark.gpu

TRAJ_TOL = 1e-6


def say(*a):
    print("[gpu-case]", *a, flush=True)


def meshes():
    out = []
    for wl, r in ((SMALL, 3), (RAGGED, 5)):
        mesh, em, mat, fx, regions, _ = wl.build()
        out.append(dict(wl=wl, r=r, mesh=mesh, em=em, mat=mat, fx=fx, regions=regions))
    return out


def make_batch(ms, tune=True, tiles=None, chunks=8, **kw):
    from paper_2409_20380_amd import ebe
    wl = SMALL
    aR, bR = wl.rayleigh
    b = ebe.Batch(wl.dt, aR, bR, s=6, tol=wl.tol, **kw)
    for i, m in enumerate(ms):
        g = b.add_mesh(m["mesh"].coords, m["mesh"].conn, m["em"], m["mat"], m["fx"], m["regions"], m["r"])
        if tiles is not None:
            b.set_group_config(g, tiles[i], chunks)
    b.assemble(tune=tune)
    return b


@pytest.fixture(scope="module")
def ms():
    return meshes()


@pytest.fixture(scope="module")
def models(ms, oracle_lib):
    aR, bR = SMALL.rayleigh
    cM, cK = cm_ck(SMALL.dt, aR, bR)
    return [oracle_lib.Model(m["mesh"].coords, m["mesh"].conn, m["em"], m["mat"], m["fx"], cM, cK) for m in ms]


@pytest.mark.parametrize("ct", [1, 2, 4, 8])
def test_batch_apply_matches_oracle(ms, models, ct):
    torch = pytest.importorskip("torch")
    say("batched apply, case tile", ct)
    b = make_batch(ms, tune=False, tiles=[ct, ct])
    for gi, (m, model) in enumerate(zip(ms, models)):
        r, n3 = m["r"], model.n3
        P = np.random.default_rng([gi, ct]).standard_normal((r, n3))
        Q = to_host(b.apply(gi, to_dev(P.ravel()))).reshape(r, n3)
        for c in range(r):
            ref = model.spmv("A", P[c])
            err = np.abs(Q[c] - ref).max() / np.abs(ref).max()
            assert err < 1e-12, (gi, c, err)
        info = b.group_info(gi)
        assert info["case_tile"] == ct and info["n_cases"] == r
    b.close()


def _waves(n_cases, nt, dt, first_seed):
    return [inputs.base_wave(first_seed + c, nt, dt) for c in range(n_cases)]


def _oracle_traj(model, m, wave, nt, tol, oracle_lib, s=6):
    wl = SMALL
    aR, bR = wl.rayleigh
    # batched cases use the guarded window at length s, always evaluating AB4
    st = oracle_lib.Stepper(model, wl.dt, aR, bR, s=s, kind=2, tol=tol, regions=m["regions"], skip_ratio=0.0,
                            col_cost=0.0)
    U, its, dec = [], [], []
    for it in range(1, nt + 1):
        rec, _, _ = st.step(g=wave[it])
        U.append(st.u.copy()); its.append(rec.iters); dec.append((rec.s_eff, rec.first, rec.pick))
    return np.array(U), np.array(its), dec


def test_batch_trajectories_match_oracle(ms, models, oracle_lib):
    torch = pytest.importorskip("torch")
    nt = 30
    say("batched trajectories, tuned, steps", nt)
    b = make_batch(ms, tune=True)
    for gi in range(len(ms)):
        say("group", gi, b.group_info(gi))
    C = sum(m["r"] for m in ms)
    waves = _waves(C, nt, SMALL.dt, 1)
    U = [[] for _ in range(C)]
    dec = [[] for _ in range(C)]
    its = np.zeros((nt, C), dtype=int)
    for it in range(1, nt + 1):
        st = b.step(np.array([w[it] for w in waves]))
        for c in range(C):
            assert st[c].status == 0 and st[c].res_true < SMALL.tol, (it, c, st[c].res_true)
            its[it - 1, c] = st[c].iters
            dec[c].append((st[c].s_eff, st[c].first, st[c].map_kept))
            U[c].append(to_host(b.get_state(c)[0]))
    c = 0
    for m, model in zip(ms, models):
        for k in range(m["r"]):
            Uref, _, _ = _oracle_traj(model, m, waves[c], nt, 1e-13, oracle_lib)
            _, its8, dec8 = _oracle_traj(model, m, waves[c], nt, SMALL.tol, oracle_lib)
            err = np.linalg.norm(np.array(U[c]) - Uref) / np.linalg.norm(Uref)
            say(f"case {c}: space-time rel L2 {err:.2e}; iters {its[:, c].mean():.2f} vs oracle {its8.mean():.2f}")
            say(f"case {c}: window decisions {dec[c]}")
            assert err < TRAJ_TOL
            assert np.abs(its[:, c] - its8).max() <= 2
            # each case's guarded window takes the oracle's decisions
            assert dec[c] == dec8
            c += 1
    b.close()


def test_batch_zero_forcing_case_and_masking(ms):
    """A case with no forcing stays at rest with zero iterations while the others run."""
    torch = pytest.importorskip("torch")
    say("batched zero-forcing case")
    b = make_batch(ms[:1], tune=False, tiles=[2])
    waves = _waves(3, 12, SMALL.dt, 7)
    for it in range(1, 13):
        g = np.array([w[it] for w in waves])
        g[1] = 0.0
        st = b.step(g)
        assert st[1].iters == 0 and st[1].status == 0
        assert st[0].iters > 0 and st[2].iters > 0
    assert float(b.get_state(1)[0].abs().max()) == 0.0
    assert float(b.get_state(0)[0].abs().max()) > 0.0
    b.close()


def test_batch_graph_replays_match_eager(ms):
    """The graph-captured trips give bitwise the eager result, step after step
    (each step replays the graph several times, with eager work between)."""
    torch = pytest.importorskip("torch")
    say("graph vs eager")
    runs = []
    for graph in (False, True):
        b = make_batch(ms, tune=False, tiles=[4, 2])
        b.use_graph(graph, 4)
        C = b.n_cases
        waves = _waves(C, 15, SMALL.dt, 20)
        hist = []
        for it in range(1, 16):
            st = b.step(np.array([w[it] for w in waves]))
            hist.append(([s.iters for s in st], [to_host(b.get_state(c)[0]) for c in range(C)]))
        runs.append(hist)
        b.close()
    for (ie, ue), (ig, ug) in zip(*runs):
        assert ie == ig
        for a, c in zip(ue, ug):
            assert np.array_equal(a, c)


def test_batch_case_tiles_agree(ms):
    torch = pytest.importorskip("torch")
    say("case tiles agree")
    finals = []
    for ct in (1, 8):
        b = make_batch(ms, tune=False, tiles=[ct, ct])
        C = b.n_cases
        waves = _waves(C, 10, SMALL.dt, 30)
        for it in range(1, 11):
            b.step(np.array([w[it] for w in waves]))
        finals.append([to_host(b.get_state(c)[0]) for c in range(C)])
        b.close()
    for a, c in zip(*finals):
        assert np.linalg.norm(a - c) <= 1e-9 * np.linalg.norm(c)


def test_batch_max_iter_and_errors(ms):
    torch = pytest.importorskip("torch")
    from paper_2409_20380_amd import ebe
    say("batched max_iter and invalid input")
    b = make_batch(ms[:1], tune=False, tiles=[1], max_iter=2)
    waves = _waves(3, 5, SMALL.dt, 40)
    st = b.step(np.array([w[1] for w in waves]))
    assert all(s.status == ebe.NOT_CONVERGED and s.iters == 2 for s in st)
    with pytest.raises(ValueError):
        b.step(np.zeros((2, 3)))
    with pytest.raises(ebe.EbeError):
        b.set_group_config(0, 3, 8)
    b.close()
    with pytest.raises(ebe.EbeError):
        ebe.Batch(0.01, predictor=3)


@pytest.mark.slow
def test_full_size_batch_apply_sampled_rows(oracle_lib):
    """Largest ensemble mesh (48x48x24 cells, 20 cases) in the bench's tuned launch configuration:
    sampled rows of A p of several cases by the oracle's element matrices."""
    torch = pytest.importorskip("torch")
    from paper_2409_20380_amd import ebe
    from tests.gpu_common import sampled_rows
    cells, r = inputs.ENSEMBLE[2]
    say("full-size batched apply", cells, "cases", r)
    wl = inputs.Workload("ens_large", cells=cells, nt=2, s=inputs.ENSEMBLE_S)
    mesh, em, mat, fx, regions, _ = wl.build()
    aR, bR = wl.rayleigh
    cM, cK = cm_ck(wl.dt, aR, bR)
    b = ebe.Batch(wl.dt, aR, bR, s=wl.s, tol=wl.tol)
    b.add_mesh(mesh.coords, mesh.conn, em, mat, fx, regions, r)
    b.assemble(tune=True)
    say("tuned", b.group_info(0))
    n3 = 3 * mesh.n_nodes
    P = np.stack([inputs.random_vector(500 + c, n3) for c in range(r)])
    Q = to_host(b.apply(0, to_dev(P.ravel()))).reshape(r, n3)
    rng = np.random.default_rng(1)
    nodes = np.concatenate([rng.choice(mesh.n_nodes, 60, replace=False), [0, mesh.n_nodes - 1]])
    for c in (0, 7, r - 1):
        ref = sampled_rows(oracle_lib, mesh, em, mat, fx, cM, cK, P[c], nodes)
        q = Q[c].reshape(-1, 3)
        assert np.abs(q[nodes] - ref).max() < 1e-12 * np.abs(q).max(), c
    b.close()
