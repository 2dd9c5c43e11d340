"""Pins of the CPU oracle against facts fixed by the paper and by mathematics.

None of these checks re-types the oracle's formulas: each compares the
oracle with an independent route (numerical quadrature, a direct solver, a
closed-form solution, an invariant, a published table) chosen so that a
dropped term, wrong sign, wrong index or transposed operand fails one of them.
"""
import math
import os

import numpy as np
import pytest
import scipy.linalg as sla
import scipy.sparse.linalg as spla

from paper_2409_20380_amd import inputs

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


# ----------------------------------------------------------------------------
# helpers (test-side, independent of oracle.c)
# ----------------------------------------------------------------------------
def _gauss01(n):
    x, w = np.polynomial.legendre.leggauss(n)
    return 0.5 * (x + 1.0), 0.5 * w


def tet_quadrature(n=6):
    """Collapsed-coordinate (Duffy / conical product) rule on the reference
    simplex {L1,L2,L3 >= 0, L1+L2+L3 <= 1}: L1 = u, L2 = (1-u) v,
    L3 = (1-u)(1-v) w, Jacobian (1-u)^2 (1-v); Gauss-Legendre in u, v, w.
    Exact for polynomials of degree <= 2n-3 in L."""
    g, w = _gauss01(n)
    pts, wts = [], []
    for iu, u in enumerate(g):
        for iv, v in enumerate(g):
            for iw, ww in enumerate(g):
                L1 = u
                L2 = (1 - u) * v
                L3 = (1 - u) * (1 - v) * ww
                pts.append((1 - L1 - L2 - L3, L1, L2, L3))
                wts.append(w[iu] * w[iv] * w[iw] * (1 - u) ** 2 * (1 - v))
    return np.array(pts), np.array(wts)  # weights sum to 1/6


def barycentric(xv, x):
    """Barycentric coordinates of point x in tet xv by solving [X;1] L = [x;1]."""
    A = np.vstack([np.asarray(xv).T, np.ones(4)])
    return np.linalg.solve(A, np.append(x, 1.0))


def p2_shape_L(L):
    """Quadratic Lagrange basis on the tet in terms of barycentrics."""
    N = [L[i] * (2 * L[i] - 1) for i in range(4)]
    N += [4 * L[a] * L[b] for a, b in inputs.TET10_EDGES]
    return np.array(N)


def p2_grad(xv, L):
    """Physical gradients [10,3] at barycentric point L (chain rule through L)."""
    A = np.vstack([np.asarray(xv).T, np.ones(4)])
    gL = np.linalg.inv(A)[:, :3]          # dL_k/dx_a
    dNdL = np.zeros((10, 4))
    for i in range(4):
        dNdL[i, i] = 4 * L[i] - 1
    for m, (a, b) in enumerate(inputs.TET10_EDGES):
        dNdL[4 + m, a] = 4 * L[b]
        dNdL[4 + m, b] = 4 * L[a]
    return dNdL @ gL


def quadrature_element(xv, lam, mu, rho, n=6):
    pts, wts = tet_quadrature(n)
    V = signed_volume(xv)
    K = np.zeros((30, 30)); M = np.zeros((30, 30))
    for L, w in zip(pts, wts):
        N = p2_shape_L(L)
        G = p2_grad(xv, L)
        # B matrix (6 x 30), engineering strain order xx,yy,zz,yz,xz,xy
        B = np.zeros((6, 30))
        for i in range(10):
            gx, gy, gz = G[i]
            B[0, 3 * i] = gx; B[1, 3 * i + 1] = gy; B[2, 3 * i + 2] = gz
            B[3, 3 * i + 1] = gz; B[3, 3 * i + 2] = gy
            B[4, 3 * i] = gz; B[4, 3 * i + 2] = gx
            B[5, 3 * i] = gy; B[5, 3 * i + 1] = gx
        D = np.zeros((6, 6))
        D[:3, :3] = lam
        D[np.arange(3), np.arange(3)] += 2 * mu
        D[np.arange(3, 6), np.arange(3, 6)] = mu
        K += 6 * V * w * B.T @ D @ B
        Nm = np.zeros((3, 30))
        for i in range(10):
            Nm[:, 3 * i:3 * i + 3] = np.eye(3) * N[i]
        M += 6 * V * w * rho * Nm.T @ Nm
    return K, M, V


def signed_volume(xv):
    xv = np.asarray(xv)
    return np.linalg.det(np.stack([xv[1] - xv[0], xv[2] - xv[0], xv[3] - xv[0]])) / 6.0


def random_tet(rng):
    """Random well-shaped tet with positive orientation det[x1-x0, x2-x0, x3-x0] > 0."""
    while True:
        xv = rng.standard_normal((4, 3))
        if signed_volume(xv) > 0.2:
            return xv


def rigid_modes(points):
    """6 rigid-body modes (3 translations, 3 rotations) on the given points."""
    n = points.shape[0]
    R = np.zeros((3 * n, 6))
    for k in range(3):
        R[k::3, k] = 1.0
    x, y, z = points[:, 0], points[:, 1], points[:, 2]
    R[0::3, 3] = -y; R[1::3, 3] = x           # about z
    R[1::3, 4] = -z; R[2::3, 4] = y           # about x
    R[0::3, 5] = z; R[2::3, 5] = -x           # about y
    return R


def elem_points(xv):
    pts = list(xv)
    for a, b in inputs.TET10_EDGES:
        pts.append(0.5 * (xv[a] + xv[b]))
    return np.array(pts)


def small_model(oracle_lib, cells=(2, 2, 2), h=2.5, fixed=True, cM=None, cK=None, dt=0.01, aR=0.0, bR=0.0):
    mesh = inputs.box_mesh(*cells, h=h)
    em, mat = inputs.two_layer_materials(mesh)
    fx = inputs.fixed_bottom(mesh) if fixed else np.zeros((mesh.n_nodes, 3), np.uint8)
    if cM is None:
        cM = 4 / dt ** 2 + 2 * aR / dt
    if cK is None:
        cK = 1 + 2 * bR / dt
    return mesh, em, mat, fx, oracle_lib.Model(mesh.coords, mesh.conn, em, mat, fx, cM, cK)


# ----------------------------------------------------------------------------
# P1 mesh
# ----------------------------------------------------------------------------
@pytest.mark.parametrize("cells", [(1, 1, 1), (2, 3, 2), (8, 8, 8)])
def test_mesh_counts_volume_faces(cells):
    nx, ny, nz = cells
    m = inputs.box_mesh(nx, ny, nz, h=2.5)
    assert m.n_nodes == (2 * nx + 1) * (2 * ny + 1) * (2 * nz + 1)
    assert m.n_elems == 6 * nx * ny * nz
    x = m.coords[m.conn[:, :4]]
    V = np.linalg.det(np.stack([x[:, 1] - x[:, 0], x[:, 2] - x[:, 0], x[:, 3] - x[:, 0]], axis=1)) / 6
    assert V.min() > 0
    assert math.isclose(V.sum(), nx * ny * nz * 2.5 ** 3, rel_tol=1e-12)
    # edge nodes at edge midpoints
    for m_, (a, b) in enumerate(inputs.TET10_EDGES):
        np.testing.assert_allclose(m.coords[m.conn[:, 4 + m_]], 0.5 * (x[:, a] + x[:, b]), atol=1e-12)
    # every interior face shared by exactly two elements, boundary faces by one
    faces = {}
    for e in range(m.n_elems):
        for f in ((0, 1, 2), (0, 1, 3), (0, 2, 3), (1, 2, 3)):
            key = tuple(sorted(m.conn[e, list(f)]))
            faces[key] = faces.get(key, 0) + 1
    n_boundary = sum(1 for c in faces.values() if c == 1)
    assert set(faces.values()) <= {1, 2}
    assert n_boundary == 4 * (nx * ny + ny * nz + nx * nz)  # 2 triangles per boundary square


# ----------------------------------------------------------------------------
# P2, P3 element matrices
# ----------------------------------------------------------------------------
def test_test_side_shape_functions_are_the_p2_lagrange_basis():
    rng = np.random.default_rng(1)
    xv = random_tet(rng)
    pts = elem_points(xv)
    N = np.array([p2_shape_L(barycentric(xv, p)) for p in pts])
    np.testing.assert_allclose(N, np.eye(10), atol=1e-12)
    # analytic gradient vs central differences
    p = xv.mean(axis=0) + 0.05
    G = p2_grad(xv, barycentric(xv, p))
    h = 1e-6
    for a in range(3):
        dp = np.zeros(3); dp[a] = h
        fd = (p2_shape_L(barycentric(xv, p + dp)) - p2_shape_L(barycentric(xv, p - dp))) / (2 * h)
        np.testing.assert_allclose(G[:, a], fd, atol=1e-7)


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_element_matrices_match_independent_quadrature(oracle_lib, seed):
    rng = np.random.default_rng(seed)
    xv = random_tet(rng)
    lam, mu, rho = rng.uniform(0.5, 2.0, 3)
    Ke, Me, V = oracle_lib.element_matrices(xv, lam, mu, rho)
    Kq, Mq, Vq = quadrature_element(xv, lam, mu, rho)
    assert math.isclose(V, Vq, rel_tol=1e-12)
    np.testing.assert_allclose(Ke, Kq, atol=1e-12 * np.abs(Kq).max())
    np.testing.assert_allclose(Me, Mq, atol=1e-12 * np.abs(Mq).max())


def test_element_stiffness_invariants(oracle_lib):
    rng = np.random.default_rng(5)
    xv = random_tet(rng)
    Ke, Me, V = oracle_lib.element_matrices(xv, 1.3, 0.7, 1.0)
    assert np.abs(Ke - Ke.T).max() <= 1e-15 * np.abs(Ke).max() * 30
    ev = np.linalg.eigvalsh(Ke)
    scale = ev[-1]
    assert np.sum(np.abs(ev) < 1e-10 * scale) == 6        # rank 24
    assert ev.min() > -1e-10 * scale                        # PSD
    R = rigid_modes(elem_points(xv))
    assert np.abs(Ke @ R).max() < 1e-11 * scale * np.abs(R).max()


def test_element_mass_invariants_and_table(oracle_lib):
    rng = np.random.default_rng(6)
    xv = random_tet(rng)
    rho = 1.7
    Ke, Me, V = oracle_lib.element_matrices(xv, 1.0, 1.0, rho)
    assert np.linalg.eigvalsh(Me).min() > 0
    Mxx = Me[0::3, 0::3]
    assert math.isclose(Mxx.sum(), rho * V, rel_tol=1e-13)
    assert np.abs(Me[0::3, 1::3]).max() == 0.0
    table = np.loadtxt(os.path.join(GOLDEN, "p2_tet_mass_table.txt"))
    np.testing.assert_allclose(Mxx * 420 / (rho * V), table, atol=1e-11)
    # the golden table obeys the textbook rule stated in its header
    E = inputs.TET10_EDGES
    for i in range(4):
        for m_, e in enumerate(E):
            assert table[i, 4 + m_] == (-4 if i in e else -6)
    for m_, e in enumerate(E):
        for n_, f in enumerate(E):
            shared = len(set(e) & set(f))
            assert table[4 + m_, 4 + n_] == {2: 32, 1: 16, 0: 8}[shared]


# ----------------------------------------------------------------------------
# P4 assembly
# ----------------------------------------------------------------------------
def test_patch_test_linear_field_interior_forces_vanish(oracle_lib):
    # homogeneous material: a constant stress is in equilibrium everywhere
    mesh = inputs.box_mesh(3, 3, 3)
    em = np.zeros(mesh.n_elems, np.int32)
    mat = np.array([[1800.0, 500.0, 250.0]])
    mod = oracle_lib.Model(mesh.coords, mesh.conn, em, mat, np.zeros((mesh.n_nodes, 3), np.uint8), 0.0, 1.0)
    rng = np.random.default_rng(3)
    G = rng.standard_normal((3, 3)); c = rng.standard_normal(3)
    u = (mesh.coords @ G.T + c).ravel()
    f = mod.spmv("K", u).reshape(-1, 3)
    L = mesh.lattice
    interior = np.all((L > 0) & (L < np.array([6, 6, 6])), axis=1)
    scale = np.abs(mod.spmv("K", rng.standard_normal(mod.n3))).max()
    assert np.abs(f[interior]).max() < 1e-11 * scale
    assert np.abs(f[~interior]).max() > 1e-3 * scale     # boundary tractions are not zero


def test_assembled_symmetry_and_translation(oracle_lib):
    dt, aR, bR = 0.01, 0.06, 0.006
    mesh, em, mat, fx, mod = small_model(oracle_lib, cells=(2, 2, 2), fixed=False, dt=dt, aR=aR, bR=bR)
    A = mod.scipy("A")
    assert abs(A - A.T).max() <= 1e-12 * abs(A).max()
    for k in range(3):
        r = np.zeros(mod.n3); r[k::3] = 1.0
        np.testing.assert_allclose(mod.spmv("A", r), mod.cM * mod.spmv("M", r), atol=1e-9 * mod.cM)
        # total mass
        rho_v = sum(mat[em[e], 0] for e in range(mesh.n_elems)) * (2.5 ** 3 / 6)
        assert math.isclose(r @ mod.spmv("M", r), rho_v, rel_tol=1e-12)


def test_fixed_dofs_identity_and_block_jacobi(oracle_lib):
    mesh, em, mat, fx, mod = small_model(oracle_lib, cells=(2, 2, 2))
    A = mod.scipy("A").toarray()
    fixed = fx.ravel().astype(bool)
    np.testing.assert_array_equal(A[np.ix_(fixed, fixed)], np.eye(fixed.sum()))
    assert np.abs(A[np.ix_(fixed, ~fixed)]).max() == 0
    Binv = mod.binv()
    for v in range(mod.n):
        np.testing.assert_allclose(Binv[v] @ A[3 * v:3 * v + 3, 3 * v:3 * v + 3], np.eye(3), atol=1e-12)


# ----------------------------------------------------------------------------
# P5 Algorithm 1 against direct solvers
# ----------------------------------------------------------------------------
@pytest.mark.parametrize("cells", [(1, 1, 1), (2, 2, 2), (4, 4, 4)])
def test_pcg_matches_dense_direct_solve(oracle_lib, cells):
    mesh, em, mat, fx, mod = small_model(oracle_lib, cells=cells, aR=0.06, bR=0.006)
    A = mod.scipy("A").toarray()
    rng = np.random.default_rng(11)
    b = rng.standard_normal(mod.n3)
    b[fx.ravel() == 1] = 0
    x_ref = sla.cho_solve(sla.cho_factor(A), b)
    for tol in (1e-8, 1e-12):
        x, st = mod.pcg(b, np.zeros(mod.n3), tol=tol)
        assert st.status == 0 and st.res_true < tol
        kappa = np.linalg.cond(A)
        assert np.linalg.norm(x - x_ref) <= 2 * kappa * tol * np.linalg.norm(x_ref)
        assert np.linalg.norm(b - A @ x) / np.linalg.norm(b) < tol


def test_pcg_matches_sparse_lu_on_small_workload(oracle_lib):
    wl = inputs.SMALL
    mesh, em, mat, fx, regions, wave = wl.build()
    aR, bR = wl.rayleigh
    mod = oracle_lib.Model(mesh.coords, mesh.conn, em, mat, fx, 4 / wl.dt ** 2 + 2 * aR / wl.dt,
                           1 + 2 * bR / wl.dt)
    A = mod.scipy("A").tocsc()
    rng = np.random.default_rng(12)
    b = rng.standard_normal(mod.n3)
    b[fx.ravel() == 1] = 0
    x_ref = spla.splu(A).solve(b)
    x, st = mod.pcg(b, np.zeros(mod.n3), tol=1e-12)
    assert np.linalg.norm(x - x_ref) <= 1e-9 * np.linalg.norm(x_ref)
    # a guess that already solves the system: zero iterations (stop test at loop top)
    x2, st2 = mod.pcg(b, x_ref, tol=1e-8)
    assert st2.iters == 0
    # zero right-hand side: x = 0, no iterations
    x3, st3 = mod.pcg(np.zeros(mod.n3), rng.standard_normal(mod.n3), tol=1e-8)
    assert st3.iters == 0 and not x3.any()


# ----------------------------------------------------------------------------
# P6, P7 Newmark
# ----------------------------------------------------------------------------
def test_newmark_discrete_energy_balance_damped_forced(oracle_lib):
    dt, aR, bR = 0.01, 0.5, 0.002
    mesh, em, mat, fx, mod = small_model(oracle_lib, cells=(2, 2, 2), dt=dt, aR=aR, bR=bR)
    st = oracle_lib.Stepper(mod, dt, aR, bR, s=4, kind=2, tol=1e-13)
    wave = inputs.base_wave(3, 40, dt) * 50.0
    M = mod.scipy("M"); K = mod.scipy("K"); Cm = aR * M + bR * K
    zero = np.zeros(mod.n3)

    def force(g):
        return mod.rhs(zero, zero, zero, dt, aR, bR, g=g)

    def energy():
        return 0.5 * st.v @ (M @ st.v) + 0.5 * st.u @ (K @ st.u)

    E0, f0 = energy(), force(wave[0])
    for it in range(1, 41):
        u0, v0 = st.u.copy(), st.v.copy()
        rec, _, _ = st.step(g=wave[it])
        f1 = force(wave[it])
        E1 = energy()
        du = st.u - u0
        vs = st.v + v0
        expect = 0.5 * du @ (f0 + f1) - dt / 4 * vs @ (Cm @ vs)
        scale = max(abs(E1), abs(E0), 1e-300)
        assert abs((E1 - E0) - expect) <= 1e-9 * scale, (it, E1 - E0, expect)
        E0, f0 = E1, f1


def test_newmark_undamped_unforced_energy_constant(oracle_lib):
    dt = 0.01
    mesh, em, mat, fx, mod = small_model(oracle_lib, cells=(2, 2, 2), dt=dt)
    st = oracle_lib.Stepper(mod, dt, 0.0, 0.0, s=0, kind=1, tol=1e-13)
    M = mod.scipy("M").toarray(); K = mod.scipy("K").toarray()
    free = fx.ravel() == 0
    rng = np.random.default_rng(4)
    u0 = np.zeros(mod.n3); u0[free] = rng.standard_normal(free.sum()) * 1e-3
    a0 = np.zeros(mod.n3)
    a0[free] = -np.linalg.solve(M[np.ix_(free, free)], K[np.ix_(free, free)] @ u0[free])
    st.u[:] = u0; st.a[:] = a0
    E = lambda: 0.5 * st.v @ M @ st.v + 0.5 * st.u @ K @ st.u  # noqa: E731
    E0 = E()
    for _ in range(30):
        st.step()
        assert abs(E() - E0) <= 1e-9 * E0


def test_newmark_single_mode_closed_form(oracle_lib):
    dt = 0.01
    mesh, em, mat, fx, mod = small_model(oracle_lib, cells=(2, 2, 1), dt=dt)
    M = mod.scipy("M").toarray(); K = mod.scipy("K").toarray()
    free = fx.ravel() == 0
    w2, V = sla.eigh(K[np.ix_(free, free)], M[np.ix_(free, free)])
    for mode in (0, 5, len(w2) - 1):
        om = math.sqrt(w2[mode])
        phi = np.zeros(mod.n3); phi[free] = V[:, mode]
        st = oracle_lib.Stepper(mod, dt, 0.0, 0.0, s=0, kind=1, tol=1e-14)
        st.u[:] = phi; st.a[:] = -w2[mode] * phi
        theta = 2 * math.atan(om * dt / 2)
        for n in range(1, 16):
            st.step()
            np.testing.assert_allclose(st.u, math.cos(n * theta) * phi, atol=1e-9 * np.abs(phi).max())


# ----------------------------------------------------------------------------
# P9 Adams-Bashforth
# ----------------------------------------------------------------------------
def test_ab4_weights_match_paper_and_are_exact_for_cubics(oracle_lib):
    w = np.loadtxt(os.path.join(GOLDEN, "ab4_weights.txt"))
    dt = 0.37
    for j in range(4):
        vs = [np.zeros(1) for _ in range(4)]
        vs[j][0] = 1.0
        out = oracle_lib.ab4(dt, *vs)
        assert math.isclose(out[0], dt * w[j] / w[4], rel_tol=1e-15)
    assert w[:4].sum() == w[4]
    # exact integral of a cubic velocity over the next step
    rng = np.random.default_rng(0)
    c = rng.standard_normal(4)
    vel = lambda t: c[0] + c[1] * t + c[2] * t ** 2 + c[3] * t ** 3  # noqa: E731
    t0 = 1.3
    v = [np.array([vel(t0 - k * dt)]) for k in range(4)]
    exact = (np.polyval(np.polyint(c[::-1]), t0 + dt) - np.polyval(np.polyint(c[::-1]), t0))
    assert math.isclose(oracle_lib.ab4(dt, *v)[0], exact, rel_tol=1e-12)


# ----------------------------------------------------------------------------
# P8 data-driven predictor
# ----------------------------------------------------------------------------
def _region_data(seed, n_nodes=300, s=8, nreg=3):
    rng = np.random.default_rng(seed)
    regions = rng.integers(0, nreg, n_nodes).astype(np.int32)
    X = [rng.standard_normal(3 * n_nodes) for _ in range(s)]
    Y = [rng.standard_normal(3 * n_nodes) for _ in range(s)]
    x = rng.standard_normal(3 * n_nodes)
    return rng, regions, X, Y, x


def test_predictor_is_regional_least_squares(oracle_lib):
    rng, regions, X, Y, x = _region_data(0)
    out = oracle_lib.predict_regional(regions, X, Y, x)
    dof_region = np.repeat(regions, 3)
    for r in range(3):
        sel = dof_region == r
        Xr = np.stack([c[sel] for c in X], axis=1)
        Yr = np.stack([c[sel] for c in Y], axis=1)
        a, *_ = np.linalg.lstsq(Xr, x[sel], rcond=None)
        np.testing.assert_allclose(out[sel], Yr @ a, rtol=1e-10, atol=1e-12)


def test_predictor_exact_recovery_in_snapshot_span(oracle_lib):
    rng, regions, X, Y, _ = _region_data(1)
    dof_region = np.repeat(regions, 3)
    x = np.zeros_like(X[0]); expect = np.zeros_like(X[0])
    for r in range(3):
        a = rng.standard_normal(len(X))
        sel = dof_region == r
        x[sel] = sum(ai * c[sel] for ai, c in zip(a, X))
        expect[sel] = sum(ai * c[sel] for ai, c in zip(a, Y))
    out = oracle_lib.predict_regional(regions, X, Y, x)
    np.testing.assert_allclose(out, expect, rtol=1e-10, atol=1e-12)
    # Y = L X for a linear map L acting within each region: prediction = L x
    n = X[0].size
    Lmap = np.zeros((n, n))
    for r in range(3):
        sel = np.where(dof_region == r)[0]
        Lmap[np.ix_(sel, sel)] = rng.standard_normal((sel.size, sel.size)) / math.sqrt(sel.size)
    Y2 = [Lmap @ c for c in X]
    out2 = oracle_lib.predict_regional(regions, X, Y2, x)
    np.testing.assert_allclose(out2, Lmap @ x, rtol=1e-9, atol=1e-11)


def test_predictor_drops_dependent_column(oracle_lib):
    rng, regions, X, Y, x = _region_data(2, nreg=1)
    regions[:] = 0
    X2 = X[:3] + [2.0 * X[1]] + X[3:]          # a dependent copy of column 1
    Y2 = Y[:3] + [rng.standard_normal(Y[0].size)] + Y[3:]
    out = oracle_lib.predict_regional(regions, X2, Y2, x)
    ref = oracle_lib.predict_regional(regions, X, Y, x)
    assert np.isfinite(out).all()
    np.testing.assert_allclose(out, ref, rtol=1e-9, atol=1e-12)


# ----------------------------------------------------------------------------
# P10/P11 whole run on the small workload
# ----------------------------------------------------------------------------
@pytest.mark.slow
def test_predictor_does_not_change_the_answer_only_the_iterations(oracle_lib):
    wl = inputs.Workload("t", cells=(4, 4, 4), nt=40, s=8)
    mesh, em, mat, fx, regions, wave = wl.build()
    aR, bR = wl.rayleigh
    mod = oracle_lib.Model(mesh.coords, mesh.conn, em, mat, fx, 4 / wl.dt ** 2 + 2 * aR / wl.dt,
                           1 + 2 * bR / wl.dt)
    runs = {}
    for kind in (0, 1, 2):
        st = oracle_lib.Stepper(mod, wl.dt, aR, bR, s=wl.s, kind=kind, tol=1e-8, regions=regions)
        U, its = [], []
        for it in range(1, wl.nt + 1):
            rec, _, _ = st.step(g=wave[it])
            assert rec.status == 0 and rec.res_true < 1e-8
            U.append(st.u.copy()); its.append(rec.iters)
        runs[kind] = (np.array(U), np.array(its))
    ref = oracle_lib.Stepper(mod, wl.dt, aR, bR, s=0, kind=1, tol=1e-13)
    Uref = []
    for it in range(1, wl.nt + 1):
        ref.step(g=wave[it]); Uref.append(ref.u.copy())
    Uref = np.array(Uref)
    for kind in (0, 1, 2):
        err = np.linalg.norm(runs[kind][0] - Uref) / np.linalg.norm(Uref)
        assert err < 1e-6, (kind, err)
    # trend of Fig. 3: AB beats a zero guess, the data-driven predictor beats AB
    tail = slice(20, None)
    assert runs[1][1][tail].mean() < runs[0][1][tail].mean()
    assert runs[2][1][tail].mean() < runs[1][1][tail].mean()


# ----------------------------------------------------------------------------
# P8 in the time loop: which AB errors form the snapshot window of a step
# ----------------------------------------------------------------------------
def _window_case(oracle_lib, seed, s, it, win):
    """A stepper about to take step n = it + 1 whose ring holds, per region R,
    AB errors e^k = B_R z^k: inside the window the coefficients follow
    z^{k+1} = Q_R z^k (an exact one-step linear recurrence of dimension d =
    s_eff), every other slot holds unrelated vectors of the same span.  The
    map of Sec. 3.2 fitted on the right window then predicts e^n = B_R Q_R
    z^{n-1} exactly, and any other choice of inputs, outputs or query does not.
    Returns the stepper, the dofs' regions, the expected AB-error estimate and
    the window's first step."""
    mesh = inputs.box_mesh(4, 4, 4)
    em, mat = inputs.two_layer_materials(mesh)
    fx = inputs.fixed_bottom(mesh)
    dt = 0.01
    mod = oracle_lib.Model(mesh.coords, mesh.conn, em, mat, fx, 4 / dt ** 2, 1.0)
    regions = inputs.block_regions(mesh, 4)
    st = oracle_lib.Stepper(mod, dt, 0.0, 0.0, s=s, kind=2, tol=1e-8, regions=regions, s_min=1, guard=False)
    n = it + 1
    first = max(win, n - 1 - s)
    d = n - 1 - first
    rng = np.random.default_rng(seed)
    free = fx.ravel() == 0
    dof_region = np.repeat(regions, 3)
    cols = {}                                      # step k -> e^k
    expect = np.zeros(mod.n3)
    steps_in_ring = range(max(1, n - 1 - s), n)    # the s + 1 newest steps occupy every slot
    for k in steps_in_ring:
        cols[k] = np.zeros(mod.n3)
    for r in range(int(regions.max()) + 1):
        sel = np.where((dof_region == r) & free)[0]
        B = rng.standard_normal((sel.size, d))
        Q, _ = np.linalg.qr(rng.standard_normal((d, d)))
        z = rng.standard_normal(d)
        zs = {}
        for k in range(first, n):
            zs[k] = z
            z = Q @ z
        Z = np.stack([zs[k] for k in range(first, n - 1)], axis=1)
        assert np.linalg.cond(Z) < 1e4
        for k in steps_in_ring:
            c = zs[k] if k in zs else rng.standard_normal(d)
            cols[k][sel] = B @ c
        expect[sel] = B @ (Q @ zs[n - 1])
    S1 = s + 1
    for k, c in cols.items():
        st.ring[(k - 1) % S1][:] = c
    # slots of a ring that has not wrapped yet hold unrelated vectors too
    for k in range(1, S1 + 1):
        if k not in cols and n - 1 < S1:
            st.ring[(k - 1) % S1][:] = 0.0
            st.ring[(k - 1) % S1][free] = rng.standard_normal(free.sum())
    for j in range(4):
        st.vh[j][:] = 0.0
        st.vh[j][free] = 1e-3 * rng.standard_normal(free.sum())
    st.it.value = it
    st.ws.win = win
    return st, free, expect, first


@pytest.mark.parametrize("s,it,win", [
    (8, 5, 1),     # ring not full: s_eff = 4 < s
    (6, 7, 1),     # ring just full, not wrapped: s_eff = s
    (6, 20, 1),    # ring wrapped twice
    (8, 29, 25),   # window restarted at step 25: older valid-looking columns ignored
])
def test_snapshot_window_recovers_exact_recurrence(oracle_lib, s, it, win):
    st, free, expect, first = _window_case(oracle_lib, 11 + it, s, it, win)
    n = it + 1
    vh0 = [c.copy() for c in st.vh]
    ring0 = [c.copy() for c in st.ring]
    dab = oracle_lib.ab4(st.P.dt, *vh0)
    rec, du, guess = st.step(want_du=True, want_guess=True)
    assert rec.s_eff == n - 1 - first and rec.first == first
    ehat = guess - dab
    assert not guess[~free].any()
    err = np.abs(ehat[free] - expect[free]).max() / np.abs(expect).max()
    assert err < 1e-10, err
    # e^n = du - du_AB lands in slot (n - 1) mod (s + 1); the other slots are untouched
    S1 = s + 1
    for k in range(S1):
        if k == (n - 1) % S1:
            np.testing.assert_array_equal(st.ring[k], du - dab)
        else:
            np.testing.assert_array_equal(st.ring[k], ring0[k])
    assert st.it.value == n and st.ws.win == win


def test_guard_keeps_ab4_and_restarts_the_window(oracle_lib):
    # a ring of unrelated columns: the map's guess is far worse than AB4's
    st, free, expect, first = _window_case(oracle_lib, 5, 8, 29, 1)
    st.P.guard = 1
    n = 30
    dab = oracle_lib.ab4(st.P.dt, *[c.copy() for c in st.vh])
    for k in range(len(st.ring)):
        st.ring[k][free] = np.random.default_rng(k).standard_normal(free.sum())
    rec, du, guess = st.step(want_guess=True)
    xab = np.where(free, dab, 0.0)
    assert rec.pick == 0 and rec.res_ab < rec.res_map
    np.testing.assert_array_equal(guess, xab)
    assert st.ws.win == n
    # the next step has no columns left: AB4 alone, no comparison
    rec2, _, guess2 = st.step(want_guess=True)
    assert rec2.s_eff == 0 and rec2.pick == -1 and st.ws.win == n


def test_guard_keeps_a_map_that_reproduces_the_solution(oracle_lib):
    # window e^{n-2} = e^{n-1} = e*, the exact AB error of the step: the map with
    # one column pair predicts e* itself, the guess solves the system
    st, free, _, _ = _window_case(oracle_lib, 6, 4, 9, 1)
    st.P.guard = 1
    n = 10
    g = np.array([0.3, -0.2, 0.5])
    st.u[free] = 1e-4 * np.random.default_rng(1).standard_normal(free.sum())
    b = st.m.rhs(st.u, st.v, st.a, st.P.dt, 0.0, 0.0, g=g)
    du_star, _ = st.m.pcg(b, np.zeros(st.m.n3), tol=1e-14)
    dab = oracle_lib.ab4(st.P.dt, *[c.copy() for c in st.vh])
    e_star = np.where(free, du_star - dab, 0.0)
    st.P.s_min = 1
    st.ws.win = n - 2            # window e^{n-2}, e^{n-1}: one column pair
    for k in (n - 2, n - 1):
        st.ring[(k - 1) % 5][:] = e_star
    rec, _, guess = st.step(g=g, want_guess=True)
    assert rec.s_eff == 1 and rec.pick == 1 and rec.res_map < 1e-10 < rec.res_ab
    assert np.abs(guess - du_star).max() <= 1e-9 * np.abs(du_star).max()
    assert st.ws.win == n - 2


def test_map_waits_for_s_min_column_pairs(oracle_lib):
    st, free, _, _ = _window_case(oracle_lib, 7, 8, 8, 1)
    st.P.s_min = 8
    dab = oracle_lib.ab4(st.P.dt, *[c.copy() for c in st.vh])
    rec, _, guess = st.step(want_guess=True)        # step 9: 7 column pairs
    assert rec.s_eff == 0 and rec.pick == -1
    np.testing.assert_array_equal(guess, np.where(free, dab, 0.0))
    dab = oracle_lib.ab4(st.P.dt, *[c.copy() for c in st.vh])
    rec, _, guess = st.step(want_guess=True)        # step 10: 8 column pairs
    assert rec.s_eff == 8 and rec.first == 1
    assert np.abs(guess - np.where(free, dab, 0.0)).max() > 0


# ----------------------------------------------------------------------------
# Window length probes and the skipped AB4 evaluation (kind 2, guard)
# ----------------------------------------------------------------------------
def _exact_step(oracle_lib, s, it, seed):
    """A stepper about to take step n = it + 1 with a random state, and the exact AB
    error e* = du* - du_AB of that step (du* from PCG at 1e-14)."""
    mesh = inputs.box_mesh(4, 4, 4)
    em, mat = inputs.two_layer_materials(mesh)
    fx = inputs.fixed_bottom(mesh)
    dt = 0.01
    mod = oracle_lib.Model(mesh.coords, mesh.conn, em, mat, fx, 4 / dt ** 2, 1.0)
    regions = inputs.block_regions(mesh, 4)
    st = oracle_lib.Stepper(mod, dt, 0.0, 0.0, s=s, kind=2, tol=1e-8, regions=regions, s_min=4, guard=True,
                            col_cost=0.08, probe_every=1, probe_step=8)
    rng = np.random.default_rng(seed)
    free = fx.ravel() == 0
    for j in range(4):
        st.vh[j][:] = 0.0
        st.vh[j][free] = 1e-3 * rng.standard_normal(free.sum())
    st.v[:] = st.vh[0]
    st.u[free] = 1e-4 * rng.standard_normal(free.sum())
    g = np.array([0.3, -0.2, 0.5])
    b = mod.rhs(st.u, st.v, st.a, dt, 0.0, 0.0, g=g)
    du_star, _ = mod.pcg(b, np.zeros(mod.n3), tol=1e-14)
    dab = oracle_lib.ab4(dt, *[c.copy() for c in st.vh])
    e_star = np.where(free, du_star - dab, 0.0)
    st.it.value = it
    return st, rng, free, np.repeat(regions, 3), g, e_star


def _ring_predicting(st, rng, free, dof_region, n, coeffs, target):
    """Fill the window e^{n-17} .. e^{n-1} (16 inputs c_0..c_15, query q = X a with the given
    coefficients a, outputs the inputs shifted by one step) so that, per region, the map over
    all 16 pairs predicts `target` exactly: c_15 is solved for from Y a = target."""
    s, S1 = 16, len(st.ring)
    first = n - 1 - s
    a = coeffs
    cols = np.zeros((s + 1, st.m.n3))
    for r in range(int(dof_region.max()) + 1):
        sel = (dof_region == r) & free
        scale = np.linalg.norm(target[sel]) / np.sqrt(sel.sum())     # inputs of the target's size
        c = [scale * rng.standard_normal(sel.sum()) for _ in range(s)]
        # Y a = sum_{j<15} a_j c_{j+1} + a_15 q,  q = sum_{j<15} a_j c_j + a_15 c_15
        rhs = target[sel] - sum(a[j - 1] * c[j] for j in range(1, 15)) - a[15] * sum(a[j] * c[j] for j in range(15))
        c[15] = rhs / (a[14] + a[15] ** 2)
        q = sum(a[j] * c[j] for j in range(16))
        for j in range(16):
            cols[j][sel] = c[j]
        cols[16][sel] = q
    for j in range(s + 1):
        st.ring[(first + j - 1) % S1][:] = cols[j]


def test_probe_keeps_the_window_when_the_shorter_one_predicts_worse(oracle_lib):
    st, rng, free, dreg, g, e_star = _exact_step(oracle_lib, 16, 40, 71)
    n = 41
    a = rng.uniform(0.5, 1.0, 16)                  # the query needs all 16 inputs
    _ring_predicting(st, rng, free, dreg, n, a, e_star)
    st.ws.s_cap, st.ws.rate, st.ws.grow_next = 16, 0.1, 0
    rec, _, _ = st.step(g=g)
    assert rec.s_eff == 16 and rec.probe == 8 and rec.pick == 1
    assert rec.res_map < 1e-10 < rec.res_probe
    assert st.ws.s_cap == 16 and rec.s_cap == 16 and st.ws.since == 0 and st.ws.grow_next == 1


def test_probe_shortens_the_window_when_the_shorter_one_predicts_as_well(oracle_lib):
    st, rng, free, dreg, g, e_star = _exact_step(oracle_lib, 16, 40, 72)
    n = 41
    a = np.concatenate([np.zeros(8), rng.uniform(0.5, 1.0, 8)])    # only the newest 8 inputs
    miss = 1e-3 * np.abs(e_star).max() * rng.standard_normal(e_star.size) * free
    _ring_predicting(st, rng, free, dreg, n, a, e_star + miss)      # both windows predict e* + miss
    st.ws.s_cap, st.ws.rate, st.ws.grow_next = 16, 0.1, 0
    rec, _, _ = st.step(g=g)
    assert rec.probe == 8 and abs(rec.res_probe - rec.res_map) <= 1e-8 * rec.res_map
    assert st.ws.s_cap == 8


def test_probe_lengthens_the_window_when_the_longer_one_saves_trips(oracle_lib):
    st, rng, free, dreg, g, e_star = _exact_step(oracle_lib, 16, 40, 73)
    n = 41
    a = rng.uniform(0.5, 1.0, 16)
    _ring_predicting(st, rng, free, dreg, n, a, e_star)             # only the 16-pair window is exact
    st.ws.s_cap, st.ws.rate, st.ws.grow_next = 8, 0.1, 1
    rec, _, _ = st.step(g=g)
    assert rec.s_eff == 8 and rec.probe == 16 and rec.res_probe < 1e-10 < rec.res_map
    assert st.ws.s_cap == 16
    # a longer window needs its columns after the window start: none to probe, so it shortens
    st2, rng2, free2, dreg2, g2, e2 = _exact_step(oracle_lib, 16, 40, 73)
    _ring_predicting(st2, rng2, free2, dreg2, n, a, e2)
    st2.ws.s_cap, st2.ws.rate, st2.ws.grow_next, st2.ws.win = 8, 0.1, 1, n - 1 - 12
    rec2, _, _ = st2.step(g=g2)
    assert rec2.probe == 0 or rec2.probe < 8


def test_probes_keep_the_window_length_in_the_papers_range(oracle_lib):
    """The map may start from one column pair (s_min = 1), but a probe never takes the
    window below 8 pairs, the lower end of the paper's range of s: from 8 pairs with a
    probe step of 4 the probe lengthens (12), from 12 it may shorten to exactly 8."""
    for cap, expect in ((8, 12), (12, 8)):
        st, rng, free, dreg, g, e_star = _exact_step(oracle_lib, 16, 40, 74)
        st.P.s_min = 1
        st.P.probe_step = 4
        st.ws.s_cap, st.ws.rate, st.ws.grow_next = cap, 0.1, 0
        rec, _, _ = st.step(g=g)
        assert rec.s_eff == cap and rec.probe == expect


def test_guard_skips_the_ab4_evaluation_while_the_map_is_far_ahead(oracle_lib):
    st, rng, free, dreg, g, e_star = _exact_step(oracle_lib, 16, 40, 74)
    n = 41
    a = rng.uniform(0.5, 1.0, 16)
    _ring_predicting(st, rng, free, dreg, n, a, e_star)
    st.P.col_cost = 0.0                              # no probes
    st.ws.rho_ab = 1e-3                              # last AB4 residual far above the map's
    dab = oracle_lib.ab4(st.P.dt, *[c.copy() for c in st.vh])
    rec, _, guess = st.step(g=g, want_guess=True)
    assert rec.skipped == 1 and rec.pick == 1 and rec.res_ab == 0.0 and st.ws.rho_ab == 1e-3
    assert rec.res_map < 1e-10
    # the same step with a reference below the map's residual evaluates AB4 and records it
    st2, rng2, free2, dreg2, g2, e2 = _exact_step(oracle_lib, 16, 40, 74)
    _ring_predicting(st2, rng2, free2, dreg2, n, a, e2)
    st2.P.col_cost = 0.0
    st2.ws.rho_ab = 1e-14
    rec2, _, _ = st2.step(g=g2)
    assert rec2.skipped == 0 and rec2.pick == 1 and rec2.res_ab > 1e-6 and st2.ws.rho_ab == rec2.res_ab
