"""Parity of the HIP library against the FP64 CPU oracle (needs an MI355X).

Every case prints its name, sizes and seed before touching the GPU, so a
failing run names what it was doing.
"""
import math

import numpy as np
import pytest

from paper_2409_20380_amd import inputs
from tests.gpu_common import (LITERAL, RAGGED, SMALL, build_case, cm_ck, history_columns, rel_max, sampled_rows,
                              to_dev, to_host)

pytestmark = pytest.mark.gpu

APPLY_TOL = 1e-12      # FP64 element-by-element vs assembled BCSR, max-abs relative
TRAJ_TOL = 1e-6        # space-time relative L2 against the tight-tolerance oracle


def say(*a):
    print("[gpu-case]", *a, flush=True)


@pytest.fixture(scope="module")
def small(oracle_lib):
    say("build small workload", SMALL.cells)
    return build_case(SMALL, oracle_lib)


@pytest.fixture(scope="module")
def small_map(oracle_lib):
    """The small workload with the plain map of Sec. 3.2: no AB4 guard, window from step 1."""
    say("build small workload, fixed window", SMALL.cells)
    c = build_case(SMALL, oracle_lib, fixed_window=True, s_min=1)
    yield c
    c["sol"].close()


@pytest.fixture(scope="module")
def ragged(oracle_lib):
    say("build ragged workload", RAGGED.cells)
    return build_case(RAGGED, oracle_lib, patch_elems=17)


@pytest.fixture(scope="module")
def literal(oracle_lib):
    say("build 1 m box workload", LITERAL.cells, "h", LITERAL.h)
    return build_case(LITERAL, oracle_lib)


def test_version_and_regions(small):
    from paper_2409_20380_amd import ebe
    assert b"gfx950" in ebe.lib().ebe_version()
    reg, n = small["sol"].regions()
    np.testing.assert_array_equal(reg, small["regions"])
    assert n == small["regions"].max() + 1


@pytest.mark.parametrize("case", ["small", "ragged"])
def test_apply_matches_oracle_bcsr(case, request):
    c = request.getfixturevalue(case)
    m, sol = c["model"], c["sol"]
    for seed in (0, 1):
        say("apply", case, "seed", seed, "n3", m.n3)
        p = inputs.random_vector(seed, m.n3)
        q = to_host(sol.apply(to_dev(p)))
        assert rel_max(q, m.spmv("A", p)) < APPLY_TOL
        qm = to_host(sol.apply_mk(1.0, 0.0, to_dev(p)))
        assert rel_max(qm, m.spmv("M", p)) < APPLY_TOL
        qk = to_host(sol.apply_mk(0.0, 1.0, to_dev(p)))
        assert rel_max(qk, m.spmv("K", p)) < APPLY_TOL


def test_apply_edge_cases(small):
    m, sol = small["model"], small["sol"]
    torch = pytest.importorskip("torch")
    say("apply zeros / unit vectors")
    z = torch.zeros(m.n3, dtype=torch.float64, device="cuda")
    assert float(sol.apply(z).abs().max()) == 0.0
    for dof in (0, m.n3 // 2 + 1, m.n3 - 1):
        e = np.zeros(m.n3); e[dof] = 1.0
        assert rel_max(to_host(sol.apply(to_dev(e))), m.spmv("A", e)) < APPLY_TOL


@pytest.mark.parametrize("case", ["small", "ragged"])
def test_precond_matches_oracle(case, request):
    c = request.getfixturevalue(case)
    m, sol = c["model"], c["sol"]
    say("precond", case)
    r = inputs.random_vector(3, m.n3)
    r[c["fx"].ravel() == 1] = 0.0
    assert rel_max(to_host(sol.precond(to_dev(r))), m.precond(r)) < 1e-12


@pytest.mark.parametrize("case", ["small", "ragged"])
def test_rhs_matches_oracle(case, request):
    c = request.getfixturevalue(case)
    m, sol, wl = c["model"], c["sol"], c["wl"]
    say("rhs", case)
    n3 = m.n3
    u, v, a = (inputs.random_vector(10 + k, n3) for k in range(3))
    for vec in (u, v, a):
        vec[c["fx"].ravel() == 1] = 0.0
    f = inputs.random_vector(13, n3)
    g = np.array([0.3, -1.1, 0.7])
    u0, v0, a0 = sol.get_state()
    sol.set_state(to_dev(u), to_dev(v), to_dev(a))
    for fe, gg in ((None, g), (f, None), (f, g), (None, None)):
        b = to_host(sol.rhs(None if fe is None else to_dev(fe), gg))
        ref = m.rhs(u, v, a, wl.dt, c["aR"], c["bR"], g=gg, f_add=fe)
        assert rel_max(b, ref) < 1e-12
    sol.set_state(u0, v0, a0)


def _random_history(m, s, it, seed, fx):
    rng = np.random.default_rng(seed)
    vh = rng.standard_normal((4, m.n3))
    ring = rng.standard_normal((s + 1, m.n3))
    vh[:, fx.ravel() == 1] = 0.0
    ring[:, fx.ravel() == 1] = 0.0
    return vh, ring


@pytest.mark.parametrize("it", [0, 1, 2, 3, 9, 17, 40])
def test_predict_matches_oracle_on_identical_history(small_map, oracle_lib, it):
    small = small_map
    m, sol, wl = small["model"], small["sol"], small["wl"]
    s = wl.s
    say("predict it", it, "s", s)
    vh, ring = _random_history(m, s, it, 100 + it, small["fx"])
    vh0, ring0, it0, w0 = sol.get_history()
    sol.set_history(to_dev(vh), to_dev(ring), it)
    xg, ps = sol.predict()
    xg = to_host(xg)
    expect = oracle_lib.ab4(wl.dt, vh[0], vh[1], vh[2], vh[3])
    se = min(s, it + 1 - 2)
    if se >= 1:
        X, Y, q, se2 = history_columns(ring, it, s)
        expect = expect + oracle_lib.predict_regional(small["regions"], X, Y, q)
    assert ps.s_eff == max(se, 0) and ps.map_kept == -1
    assert rel_max(xg, expect) < 1e-10
    sol.set_history(vh0, ring0, it0, w0)


def test_one_global_region(small, oracle_lib):
    """One predictor region over the whole 8x8x8-cell mesh (4,913 nodes, cut into 10 node chunks whose
    partial Grams the least-squares kernel sums): predict on an identical history and a 30-step
    trajectory against the oracle with the same single region."""
    from paper_2409_20380_amd import ebe
    c = dict(small)
    wl, m = c["wl"], c["model"]
    c["regions"] = np.zeros(m.n3 // 3, np.int32)
    say("one global region: predict and 30-step trajectory")
    sol = ebe.Solver(wl.dt, c["aR"], c["bR"], s=wl.s, tol=wl.tol, fixed_window=True, s_min=1)
    sol.assemble(c["mesh"].coords, c["mesh"].conn, c["em"], c["mat"], c["fx"], c["regions"])
    it = 25
    vh, ring = _random_history(m, wl.s, it, 300, c["fx"])
    sol.set_history(to_dev(vh), to_dev(ring), it)
    xg, ps = sol.predict()
    X, Y, q, se = history_columns(ring, it, wl.s)
    assert ps.s_eff == se == wl.s
    expect = oracle_lib.ab4(wl.dt, vh[0], vh[1], vh[2], vh[3]) + oracle_lib.predict_regional(c["regions"], X, Y, q)
    assert rel_max(to_host(xg), expect) < 1e-10
    sol.close()
    sol = ebe.Solver(wl.dt, c["aR"], c["bR"], s=wl.s, tol=wl.tol)
    sol.assemble(c["mesh"].coords, c["mesh"].conn, c["em"], c["mat"], c["fx"], c["regions"])
    U, its, res = _gpu_run(sol, c["wave"], 30)
    Uref, _ = _oracle_run(c, oracle_lib, 1e-13, 30)
    _, its8 = _oracle_run(c, oracle_lib, wl.tol, 30)
    err = np.linalg.norm(U - Uref) / np.linalg.norm(Uref)
    say("one global region: space-time rel L2", err, "iters", its.mean(), its8.mean())
    assert err < TRAJ_TOL and (res < wl.tol).all()
    assert np.abs(its - its8).max() <= 2
    sol.close()


def test_predict_exact_recovery_in_snapshot_span(small_map):
    """Query e^{n-1} built inside span(X) per region: the prediction is Y a exactly."""
    small = small_map
    m, sol, wl = small["model"], small["sol"], small["wl"]
    s, it = wl.s, 30
    say("predict exact recovery")
    rng = np.random.default_rng(7)
    vh = np.zeros((4, m.n3))
    ring = rng.standard_normal((s + 1, m.n3))
    ring[:, small["fx"].ravel() == 1] = 0.0
    n, S1 = it + 1, s + 1
    cols = [(n - s - 1 + j - 1) % S1 for j in range(s + 1)]   # slots of e^{n-s-1} .. e^{n-1}
    dof_region = np.repeat(small["regions"], 3)
    q = np.zeros(m.n3)
    expect = np.zeros(m.n3)
    for r in range(small["regions"].max() + 1):
        sel = dof_region == r
        a = rng.standard_normal(s)
        q[sel] = sum(a[j] * ring[cols[j]][sel] for j in range(s))          # q = X a
        # outputs Y = columns 1..s; column s is q itself
        ycols = [ring[cols[j + 1]][sel] for j in range(s - 1)] + [q[sel]]
        expect[sel] = sum(a[j] * ycols[j] for j in range(s))               # Y a
    ring[cols[s]] = q
    vh0, ring0, it0, w0 = sol.get_history()
    sol.set_history(to_dev(vh), to_dev(ring), it)
    xg, _ = sol.predict()
    assert rel_max(to_host(xg), expect) < 1e-9
    sol.set_history(vh0, ring0, it0, w0)


def _window_ring(small, seed, it):
    """Random free-dof ring and the slots of the window W = [e^{n-s-1} .. e^{n-1}] of step n = it + 1."""
    m, wl = small["model"], small["wl"]
    s = wl.s
    rng = np.random.default_rng(seed)
    ring = rng.standard_normal((s + 1, m.n3))
    ring[:, small["fx"].ravel() == 1] = 0.0
    n, S1 = it + 1, s + 1
    cols = [(n - s - 1 + j - 1) % S1 for j in range(s + 1)]
    return rng, ring, cols


def _predict_on(small, ring, it):
    sol = small["sol"]
    vh0, ring0, it0, w0 = sol.get_history()
    sol.set_history(to_dev(np.zeros((4, small["model"].n3))), to_dev(ring), it)
    xg, ps = sol.predict()
    sol.set_history(vh0, ring0, it0, w0)
    return to_host(xg), ps


def test_predict_dependent_columns_match_oracle(small_map, oracle_lib):
    """Sec. 3.2's modified Gram-Schmidt with exactly dependent inputs: a duplicated
    column and a scaled copy.  Both sides drop the later copy (its orthogonal part is
    zero), so the prediction is the same least-squares map: equal to 1e-10."""
    small = small_map
    s, it = small["wl"].s, 30
    say("predict with a duplicated and a scaled column")
    rng, ring, cols = _window_ring(small, 41, it)
    ring[cols[5]] = ring[cols[2]]             # duplicate of input 2
    ring[cols[9]] = -2.5 * ring[cols[4]]      # scaled copy of input 4
    xg, ps = _predict_on(small, ring, it)
    W = [ring[c] for c in cols]
    expect = oracle_lib.predict_regional(small["regions"], W[:s], W[1:], W[s])
    assert ps.s_eff == s and np.isfinite(xg).all()
    assert rel_max(xg, expect) < 1e-10


@pytest.mark.parametrize("rho,kept", [(3e-6, True), (3e-7, False)])
def test_predict_near_dependent_column_is_a_least_squares_minimiser(small_map, rho, kept):
    """Input 6 = 3 x input 0 + a part orthogonal-ish of relative size rho, just above
    (3e-6) or below (3e-7) the drop threshold 1e-6.  Near the threshold several answers
    are correct (any minimiser over the kept columns), so the check is validity: the
    coefficients, recovered per region from the prediction (input 0 is not an output,
    so the outputs stay well conditioned), are finite, leave column 6 out when its
    part is below the threshold, and give a residual ||X_K a - q|| within 1e-9 of the
    least-squares minimum over the kept columns K (an SVD solve in FP64)."""
    small = small_map
    s, it = small["wl"].s, 30
    say("predict with a near-dependent column, rho", rho)
    rng, ring, cols = _window_ring(small, 42, it)
    dof_region = np.repeat(small["regions"], 3)
    free = small["fx"].ravel() == 0
    c6 = 3.0 * ring[cols[0]]
    for r in range(int(small["regions"].max()) + 1):
        sel = (dof_region == r) & free
        z = rng.standard_normal(sel.sum())
        c6[sel] += rho * np.linalg.norm(c6[sel]) * z / np.linalg.norm(z)
    ring[cols[6]] = c6
    xg, ps = _predict_on(small, ring, it)
    assert np.isfinite(xg).all()
    W = [ring[c] for c in cols]
    worst = 0.0
    for r in range(int(small["regions"].max()) + 1):
        sel = (dof_region == r) & free
        X = np.stack([w[sel] for w in W[:s]], axis=1)
        Y = np.stack([w[sel] for w in W[1:]], axis=1)
        q = W[s][sel]
        a, res, *_ = np.linalg.lstsq(Y, xg[sel], rcond=None)
        assert np.linalg.norm(Y @ a - xg[sel]) <= 1e-10 * np.linalg.norm(xg[sel])   # a prediction Y a
        K = [j for j in range(s) if kept or j != 6]
        if not kept:
            assert abs(a[6]) <= 1e-8 * np.abs(a).max()
        a_star, *_ = np.linalg.lstsq(X[:, K], q, rcond=None)
        r_gpu = np.linalg.norm(X[:, K] @ a[K] - q)
        r_min = np.linalg.norm(X[:, K] @ a_star - q)
        worst = max(worst, r_gpu / r_min - 1.0)
    say(f"rho {rho}: worst relative excess of the least-squares residual {worst:.2e}")
    assert worst <= 1e-9


def _oracle_at(c, oracle_lib, vh, ring, it, win, u, v, a, **kw):
    """An oracle stepper holding the given state and history."""
    wl = c["wl"]
    st = oracle_lib.Stepper(c["model"], wl.dt, c["aR"], c["bR"], s=wl.s, kind=2, tol=wl.tol, regions=c["regions"],
                            **kw)
    for k in range(4):
        st.vh[k][:] = vh[k]
    for k in range(wl.s + 1):
        st.ring[k][:] = ring[k]
    st.u[:] = u; st.v[:] = v; st.a[:] = a
    st.it.value = it
    st.ws.win = win
    return st


@pytest.mark.parametrize("it,win", [(5, 1), (9, 1), (30, 1), (30, 20), (30, 25)])
def test_predict_guarded_window_matches_oracle(small, oracle_lib, it, win):
    """Default rule (s_min 3, AB4 guard) on an identical state and history: the same
    window, the same pick and both candidates' initial residuals as the oracle's."""
    m, sol, wl = small["model"], small["sol"], small["wl"]
    say("predict guarded it", it, "win", win)
    free = small["fx"].ravel() == 0
    rng = np.random.default_rng(200 + it + win)
    vh = rng.standard_normal((4, m.n3)) * 1e-3
    ring = rng.standard_normal((wl.s + 1, m.n3)) * 1e-6
    u, v, a = (rng.standard_normal(m.n3) * sc for sc in (1e-3, 1e-2, 1e-1))
    for arr in (vh, ring):
        arr[:, ~free] = 0.0
    for arr in (u, v, a):
        arr[~free] = 0.0
    v[:] = vh[0]
    g = np.array([0.4, -0.3, 0.8])
    st = _oracle_at(small, oracle_lib, vh, ring, it, win, u, v, a)
    rec, _, guess = st.step(g=g, want_guess=True)
    s0 = sol.get_state(), sol.get_history()
    sol.set_state(to_dev(u), to_dev(v), to_dev(a))
    sol.set_history(to_dev(vh), to_dev(ring), it, win)
    xg, ps = sol.predict(base_acc=g)
    say("oracle s_eff/first/pick", rec.s_eff, rec.first, rec.pick, "res map/ab", rec.res_map, rec.res_ab)
    say("gpu    s_eff/first/pick", ps.s_eff, ps.first, ps.map_kept, "res map/ab", ps.res0_map, ps.res0_ab)
    assert (ps.s_eff, ps.first, ps.map_kept) == (rec.s_eff, rec.first, rec.pick)
    assert rel_max(to_host(xg), guess) < 1e-10
    if rec.pick >= 0:
        assert abs(ps.res0_map - rec.res_map) <= 1e-10 * rec.res_map
        assert abs(ps.res0_ab - rec.res_ab) <= 1e-10 * rec.res_ab
    assert abs(ps.res0 - rec.res0) <= 1e-10 * rec.res0
    # predict leaves the state alone: the window start is unchanged
    assert sol.get_history()[3].start == win
    (u0, v0, a0), (vh0, ring0, it0, w0) = s0
    sol.set_state(u0, v0, a0)
    sol.set_history(vh0, ring0, it0, w0)


def test_predict_guard_keeps_a_map_that_solves_the_step(oracle_lib):
    """Window e^{n-2} = e^{n-1} = e*, the exact AB error of the step (s_min 1): the
    map's guess is the solution, it is kept over AB4 and predict returns it."""
    c = build_case(SMALL, oracle_lib, s_min=1)
    m, sol, wl = c["model"], c["sol"], c["wl"]
    say("predict guard: map reproducing the solution")
    free = c["fx"].ravel() == 0
    rng = np.random.default_rng(31)
    it, n = 12, 13
    vh = rng.standard_normal((4, m.n3)) * 1e-3
    vh[:, ~free] = 0.0
    u = rng.standard_normal(m.n3) * 1e-3
    u[~free] = 0.0
    z = np.zeros(m.n3)
    g = np.array([0.3, -0.2, 0.5])
    b = m.rhs(u, vh[0], z, wl.dt, c["aR"], c["bR"], g=g)
    du_star, _ = m.pcg(b, z, tol=1e-14)
    dab = oracle_lib.ab4(wl.dt, vh[0], vh[1], vh[2], vh[3])
    e_star = np.where(free, du_star - dab, 0.0)
    ring = np.zeros((wl.s + 1, m.n3))
    for k in (n - 2, n - 1):
        ring[(k - 1) % (wl.s + 1)] = e_star
    sol.set_state(to_dev(u), to_dev(vh[0]), to_dev(z))
    sol.set_history(to_dev(vh), to_dev(ring), it, n - 2)
    xg, ps = sol.predict(base_acc=g)
    say("map/ab residuals", ps.res0_map, ps.res0_ab)
    assert ps.s_eff == 1 and ps.first == n - 2 and ps.map_kept == 1
    assert ps.res0_map < 1e-10 < ps.res0_ab and ps.res0 == ps.res0_map
    assert rel_max(to_host(xg), du_star) < 1e-9
    sol.close()


def test_refine_matches_oracle(small):
    m, sol = small["model"], small["sol"]
    say("refine random rhs")
    b = inputs.random_vector(21, m.n3)
    b[small["fx"].ravel() == 1] = 0.0
    x = to_dev(np.zeros(m.n3))
    st = sol.refine(to_dev(b), x)
    xr = to_host(x)
    assert st.status == 0 and st.res_true < 1e-8
    # residual re-evaluated with the oracle's assembled operator
    assert np.linalg.norm(b - m.spmv("A", xr)) / np.linalg.norm(b) < 1e-8
    xo, so = m.pcg(b, np.zeros(m.n3), tol=1e-8)
    assert abs(st.iters - so.iters) <= 2
    x_ref, _ = m.pcg(b, np.zeros(m.n3), tol=1e-13)
    assert np.linalg.norm(xr - x_ref) / np.linalg.norm(x_ref) < 1e-6


def test_refine_edge_cases(small):
    from paper_2409_20380_amd import ebe
    m, sol = small["model"], small["sol"]
    torch = pytest.importorskip("torch")
    say("refine edge cases")
    # zero right-hand side: x = 0, no iterations
    x = to_dev(inputs.random_vector(5, m.n3))
    st = sol.refine(torch.zeros(m.n3, dtype=torch.float64, device="cuda"), x)
    assert st.iters == 0 and float(x.abs().max()) == 0.0
    # exact guess: no iterations
    b = inputs.random_vector(22, m.n3); b[small["fx"].ravel() == 1] = 0.0
    x_ref, _ = m.pcg(b, np.zeros(m.n3), tol=1e-14)
    x = to_dev(x_ref)
    st = sol.refine(to_dev(b), x)
    assert st.iters == 0 and st.res_true < 1e-8
    # fixed rows are identity: a non-zero fixed component of b lands in x exactly
    b2 = b.copy(); fixed_dofs = np.where(small["fx"].ravel() == 1)[0]
    b2[fixed_dofs[:5]] = 3.0
    x = to_dev(np.zeros(m.n3))
    st = sol.refine(to_dev(b2), x)
    assert st.res_true < 1e-8
    np.testing.assert_array_equal(to_host(x)[fixed_dofs[:5]], 3.0)
    # non-finite guess: reported, not hidden
    xn = np.zeros(m.n3); xn[np.where(small["fx"].ravel() == 0)[0][7]] = np.nan   # a free dof
    with pytest.raises(ebe.EbeError) as ei:
        sol.refine(to_dev(b), to_dev(xn))
    assert ei.value.code == ebe.E_NONFINITE


def test_max_iter_cap_reports_not_converged(oracle_lib):
    from paper_2409_20380_amd import ebe
    say("max_iter cap")
    c = build_case(SMALL, oracle_lib, max_iter=5)
    m, sol = c["model"], c["sol"]
    b = inputs.random_vector(23, m.n3); b[c["fx"].ravel() == 1] = 0.0
    x = to_dev(np.zeros(m.n3))
    st = sol.refine(to_dev(b), x)
    assert st.status == ebe.NOT_CONVERGED and st.iters == 5 and st.res_true > 1e-8
    sol.close()


def test_invalid_inputs_are_rejected(oracle_lib):
    from paper_2409_20380_amd import ebe
    say("invalid inputs")
    mesh = inputs.box_mesh(2, 2, 2)
    em, mat = inputs.two_layer_materials(mesh)
    fx = inputs.fixed_bottom(mesh)
    sol = ebe.Solver(0.01)
    with pytest.raises(ebe.EbeError) as ei:
        sol.step(base_acc=[0, 0, 0])
    assert ei.value.code == ebe.E_BAD_STATE
    bad = mesh.conn.copy(); bad[0, [1, 2]] = bad[0, [2, 1]]          # inverted element
    with pytest.raises(ebe.EbeError) as ei:
        sol.assemble(mesh.coords, bad, em, mat, fx)
    assert ei.value.code == ebe.E_INVALID_ARG
    bad = mesh.conn.copy(); bad[0, 4] = bad[0, 9]                     # misplaced edge node
    with pytest.raises(ebe.EbeError):
        sol.assemble(mesh.coords, bad, em, mat, fx)
    bad = mesh.conn.copy(); bad[3, 0] = mesh.n_nodes                  # id out of range
    with pytest.raises(ebe.EbeError):
        sol.assemble(mesh.coords, bad, em, mat, fx)
    with pytest.raises(ebe.EbeError):
        sol.assemble(mesh.coords, mesh.conn, em + 5, mat, fx)          # material out of range
    sol.assemble(mesh.coords, mesh.conn, em, mat, fx)                  # still usable afterwards
    sol.close()
    with pytest.raises(ebe.EbeError):
        ebe.Solver(0.01, s=40)


def _oracle_run(c, oracle_lib, tol, nt, s=None, kind=2, decisions=None, **kw):
    wl = c["wl"]
    st = oracle_lib.Stepper(c["model"], wl.dt, c["aR"], c["bR"], s=wl.s if s is None else s, kind=kind, tol=tol,
                            regions=c["regions"], **kw)
    U, its = [], []
    for it in range(1, nt + 1):
        rec, _, _ = st.step(g=c["wave"][it])
        U.append(st.u.copy()); its.append(rec.iters)
        if decisions is not None:
            decisions.append((rec.s_eff, rec.first, rec.pick, rec.skipped, rec.probe, rec.s_cap))
    return np.array(U), np.array(its)


def _gpu_run(sol, wave, nt, decisions=None):
    U, its, res = [], [], []
    for it in range(1, nt + 1):
        st = sol.step(base_acc=wave[it])
        assert st.status == 0
        u, _, _ = sol.get_state()
        U.append(to_host(u)); its.append(st.iters); res.append(st.res_true)
        if decisions is not None:
            decisions.append((st.s_eff, st.first, st.map_kept, st.skipped, st.probe, st.s_cap))
    return np.array(U), np.array(its), np.array(res)


@pytest.mark.parametrize("case", ["small", "ragged", "literal"])
def test_trajectory_matches_oracle(case, request, oracle_lib):
    c = request.getfixturevalue(case)
    wl = c["wl"]
    from paper_2409_20380_amd import ebe
    say("trajectory", case, "steps", wl.nt, "s", wl.s)
    sol = ebe.Solver(wl.dt, c["aR"], c["bR"], s=wl.s, tol=wl.tol, patch_elems=c["sol"].cfg.patch_elems)
    sol.assemble(c["mesh"].coords, c["mesh"].conn, c["em"], c["mat"], c["fx"], c["regions"])
    dg, do = [], []
    U, its, res = _gpu_run(sol, c["wave"], wl.nt, dg)
    Uref, _ = _oracle_run(c, oracle_lib, 1e-13, wl.nt)
    U8, its8 = _oracle_run(c, oracle_lib, wl.tol, wl.nt, decisions=do)
    err = np.linalg.norm(U - Uref) / np.linalg.norm(Uref)
    say("space-time rel L2 vs tight oracle", err, "iters gpu/oracle", its.mean(), its8.mean())
    say("window decisions (s_eff, first, map kept, AB4 skipped, probe, length cap) gpu:", dg)
    assert err < TRAJ_TOL
    assert (res < wl.tol).all()
    # the guarded window takes the same decisions as the oracle's at the same tolerance (the 1 m
    # box's steps are not reproducible to that level, see below: its decisions are only printed)
    if case != "literal":
        assert dg == do
    if case == "literal":
        # At 1/8 m cells (condition number ~1e5) the trip count of a step is not a stable
        # quantity: the oracle itself, fed the same wave scaled by 1 + 1e-13, moves single
        # steps by up to 18 of ~330 trips while its mean moves by 0.6 %. Only the mean is
        # compared there; the trajectory and residual checks above are the same as elsewhere.
        assert abs(its.mean() - its8.mean()) <= 0.02 * its8.mean()
    else:
        assert np.abs(its - its8).max() <= 2
    if case == "small":
        # trend of the paper's Fig. 3 (not an exact pin): the data-driven predictor
        # needs fewer iterations than Adams-Bashforth alone once its window is full
        _, its_ab = _oracle_run(c, oracle_lib, wl.tol, wl.nt, kind=1)
        tail = slice(wl.nt // 2, None)
        assert its[tail].mean() < its_ab[tail].mean()
    sol.close()


def test_trajectory_with_merged_regions(small, oracle_lib):
    """Merged predictor regions (region_merge 8 over 64 given regions of 4^3 lattice nodes): every merged
    region is the union of 8 whole given regions, and the merged map the library reports is the partition
    the oracle's least squares uses; trajectory, residuals, decisions and trips as for given regions."""
    from paper_2409_20380_amd import ebe, inputs as inp
    c = small
    wl, mesh = c["wl"], c["mesh"]
    given = inp.block_regions(mesh, 4)
    R = int(given.max()) + 1
    say("trajectory with merged regions:", R, "given regions, 8 per predictor region")
    sol = ebe.Solver(wl.dt, c["aR"], c["bR"], s=wl.s, tol=wl.tol, region_merge=8)
    sol.assemble(mesh.coords, mesh.conn, c["em"], c["mat"], c["fx"], given)
    merged, nr = sol.regions()
    assert R == 64 and nr == 8
    of = [set(merged[given == r].tolist()) for r in range(R)]
    assert all(len(x) == 1 for x in of)
    assert np.bincount([next(iter(x)) for x in of], minlength=nr).tolist() == [8] * nr
    cm = dict(c, regions=merged)
    dg, do = [], []
    U, its, res = _gpu_run(sol, c["wave"], wl.nt, dg)
    Uref, _ = _oracle_run(cm, oracle_lib, 1e-13, wl.nt)
    U8, its8 = _oracle_run(cm, oracle_lib, wl.tol, wl.nt, decisions=do)
    err = np.linalg.norm(U - Uref) / np.linalg.norm(Uref)
    say("space-time rel L2 vs tight oracle", err, "iters gpu/oracle", its.mean(), its8.mean())
    assert err < TRAJ_TOL
    assert (res < wl.tol).all()
    assert dg == do
    assert np.abs(its - its8).max() <= 2
    sol.close()


def test_bitwise_determinism_and_checkpoint(small):
    from paper_2409_20380_amd import ebe
    c = small
    wl = c["wl"]
    say("determinism + checkpoint/resume")

    def fresh():
        s = ebe.Solver(wl.dt, c["aR"], c["bR"], s=wl.s, tol=wl.tol)
        s.assemble(c["mesh"].coords, c["mesh"].conn, c["em"], c["mat"], c["fx"], c["regions"])
        return s

    a, b = fresh(), fresh()
    for it in range(1, 31):
        a.step(base_acc=c["wave"][it])
        b.step(base_acc=c["wave"][it])
    ua, ub = to_host(a.get_state()[0]), to_host(b.get_state()[0])
    assert np.array_equal(ua, ub)
    # checkpoint at step 30 into a third solver, continue both to 45
    vh, ring, it, win = a.get_history()
    u, v, acc = a.get_state()
    cpt = fresh()
    cpt.set_state(u, v, acc)
    cpt.set_history(vh, ring, it, win)
    for it in range(31, 46):
        sa = a.step(base_acc=c["wave"][it])
        sc = cpt.step(base_acc=c["wave"][it])
        assert sa.iters == sc.iters
    assert np.array_equal(to_host(a.get_state()[0]), to_host(cpt.get_state()[0]))
    for s in (a, b, cpt):
        s.close()


@pytest.mark.slow
def test_full_size_apply_sampled_rows(oracle_lib):
    """Headline mesh (64x64x32 cells, 3.24M dof): sampled rows of A p by the oracle's element matrices."""
    from paper_2409_20380_amd import ebe
    wl = inputs.PLAIN
    say("full-size apply", wl.cells)
    mesh = inputs.box_mesh(*wl.cells, h=wl.h)
    em, mat = inputs.two_layer_materials(mesh)
    fx = inputs.fixed_bottom(mesh)
    regions = inputs.block_regions(mesh, wl.region_block)
    aR, bR = wl.rayleigh
    cM, cK = cm_ck(wl.dt, aR, bR)
    sol = ebe.Solver(wl.dt, aR, bR, s=wl.s, tol=wl.tol)
    sol.assemble(mesh.coords, mesh.conn, em, mat, fx, regions)
    p = inputs.random_vector(42, 3 * mesh.n_nodes)
    q = to_host(sol.apply(to_dev(p))).reshape(-1, 3)
    rng = np.random.default_rng(0)
    nodes = np.concatenate([rng.choice(mesh.n_nodes, 200, replace=False), [0, mesh.n_nodes - 1]])
    ref = sampled_rows(oracle_lib, mesh, em, mat, fx, cM, cK, p, nodes)
    assert np.abs(q[nodes] - ref).max() < APPLY_TOL * np.abs(q).max()
    # symmetry at full size: x^T A y = y^T A x
    y = inputs.random_vector(43, 3 * mesh.n_nodes)
    Ay = to_host(sol.apply(to_dev(y)))
    lhs, rhs = p @ Ay, y @ q.ravel()
    assert abs(lhs - rhs) < 1e-12 * abs(lhs) * 100
    sol.close()


def _one_tet():
    """A single straight 10-node tet (vertices, then edges 01, 12, 02, 03, 13, 23)."""
    v = np.array([[0.0, 0.0, 0.0], [2.5, 0.0, 0.0], [0.0, 2.5, 0.0], [0.0, 0.0, 2.5]])
    edges = [(0, 1), (1, 2), (0, 2), (0, 3), (1, 3), (2, 3)]
    coords = np.vstack([v] + [0.5 * (v[a] + v[b]) for a, b in edges])
    conn = np.arange(10, dtype=np.int32)[None, :]
    fixed = np.zeros((10, 3), dtype=np.uint8)
    fixed[0, :] = 1                      # one vertex held; the mass keeps A definite anyway
    fixed[1, 2] = 1
    return coords, conn, np.zeros(1, np.int32), np.array([[1800.0, 380.0, 200.0]]), fixed


def test_single_element_mesh(oracle_lib):
    """One element, one patch of one element, one region: apply and a short
    trajectory (the snapshot window never fills) against the oracle."""
    from paper_2409_20380_amd import ebe
    coords, conn, em, mat, fx = _one_tet()
    wl = SMALL
    aR, bR = wl.rayleigh
    cM, cK = cm_ck(wl.dt, aR, bR)
    regions = np.zeros(10, np.int32)
    say("single element: 10 nodes, 1 element, s 4")
    m = oracle_lib.Model(coords, conn, em, mat, fx, cM, cK)
    sol = ebe.Solver(wl.dt, aR, bR, s=4, tol=wl.tol)
    sol.assemble(coords, conn, em, mat, fx, regions)
    for seed in (0, 1):
        p = inputs.random_vector(seed, 30)
        assert rel_max(to_host(sol.apply(to_dev(p))), m.spmv("A", p)) < APPLY_TOL
    wave = inputs.base_wave(3, 12, wl.dt, *wl.f_band)
    U, its = [], []
    for it in range(1, 13):
        st = sol.step(base_acc=wave[it])
        assert st.status == 0 and st.res_true < wl.tol
        U.append(to_host(sol.get_state()[0])); its.append(st.iters)
    orc = oracle_lib.Stepper(m, wl.dt, aR, bR, s=4, kind=2, tol=1e-13, regions=regions)
    o8 = oracle_lib.Stepper(m, wl.dt, aR, bR, s=4, kind=2, tol=wl.tol, regions=regions)
    Uref, its8 = [], []
    for it in range(1, 13):
        orc.step(g=wave[it])
        rec, _, _ = o8.step(g=wave[it])
        Uref.append(orc.u.copy()); its8.append(rec.iters)
    err = np.linalg.norm(np.array(U) - np.array(Uref)) / np.linalg.norm(np.array(Uref))
    say("single element: space-time rel L2", err, "iters", its, its8)
    assert err < TRAJ_TOL
    assert np.abs(np.array(its) - np.array(its8)).max() <= 2
    sol.close()


def test_all_dofs_fixed():
    """Every dof fixed: A is the identity, every right-hand side is zero, so each
    step takes no trip and the state stays exactly at rest (zero Gram columns
    are dropped by the least-squares solve)."""
    from paper_2409_20380_amd import ebe
    mesh = inputs.box_mesh(1, 1, 1)
    em, mat = inputs.two_layer_materials(mesh)
    fx = np.ones((mesh.n_nodes, 3), dtype=np.uint8)
    wl = SMALL
    aR, bR = wl.rayleigh
    say("all dofs fixed: 1x1x1 cells,", mesh.n_nodes, "nodes")
    sol = ebe.Solver(wl.dt, aR, bR, s=4, tol=wl.tol)
    sol.assemble(mesh.coords, mesh.conn, em, mat, fx)
    p = inputs.random_vector(4, 3 * mesh.n_nodes)
    np.testing.assert_array_equal(to_host(sol.apply(to_dev(p))), p)
    wave = inputs.base_wave(5, 10, wl.dt, *wl.f_band)
    for it in range(1, 11):
        st = sol.step(base_acc=wave[it])
        assert st.status == 0 and st.iters == 0
    for vec in sol.get_state():
        assert float(vec.abs().max()) == 0.0
    sol.close()
