"""Learned node-wise predictor on the GPU against the FP64 oracle (needs an MI355X).

Inference runs on BF16 MFMA (BF16 weights, inputs and activations, FP32 accumulation);
its bound against the FP64 oracle with the same BF16 weights comes from three
BF16 roundings of layer inputs (unit roundoff 2^-9 each) and is taken as
2e-2 normwise; against an oracle that rounds the same layer inputs to BF16
the remaining differences are FP32 accumulation order and rare rounding ties
(3e-3).  Training runs in FP32 on BF16 inputs and weights: gradients within
1e-4 normwise of the FP64 oracle's, Adam steps within FP32 rounding of the
oracle's update.
"""
import numpy as np
import pytest

from oracle import mlp as omlp
from paper_2409_20380_amd import inputs
from tests.gpu_common import SMALL, build_case, history_columns, to_dev, to_host

pytestmark = pytest.mark.gpu

INFER_TOL = 2e-2
INFER_MIMIC_TOL = 3e-3
GRAD_TOL = 1e-4


def say(*a):
    print("[gpu-case]", *a, flush=True)


def nrel(a, b):
    return float(np.linalg.norm(np.asarray(a, dtype=np.float64) - b) / max(np.linalg.norm(b), 1e-300))


def bf16_params(seed, gain=1.0):
    """Seeded weights that are exactly representable in BF16 (so both sides use the same values)."""
    p = inputs.mlp_init(seed, gain).astype(np.float64)
    rng = np.random.default_rng([seed, 5])
    p = p + 0.05 * rng.standard_normal(p.size) * (p == 0)      # non-zero biases
    return omlp.bf16_round(p).astype(np.float32)


@pytest.fixture(scope="module")
def small(oracle_lib):
    say("build small workload", SMALL.cells)
    c = build_case(SMALL, oracle_lib)
    yield c
    c["sol"].close()


def _mimic_forward(params, X):
    """Oracle forward with the layer inputs rounded to BF16, as the MFMA kernel takes them."""
    W1, b1, W2, b2, W3, b3 = omlp.unpack(params)
    h = omlp.bf16_round(X)
    h = omlp.bf16_round(omlp.gelu(h @ W1.T + b1))
    h = omlp.bf16_round(omlp.gelu(h @ W2.T + b2))
    return h @ W3.T + b3


@pytest.mark.parametrize("n", [1, 17, 1000, 70001])
def test_inference_matches_oracle(small, n):
    torch = pytest.importorskip("torch")
    sol = small["sol"]
    say("mlp inference n", n)
    p = bf16_params(11)
    sol.mlp_set(p, [1.0, 1.0, 1.0, 1.0])
    X = np.random.default_rng([n, 3]).standard_normal((n, 15)).astype(np.float32)
    y = to_host(sol.mlp_forward(torch.from_numpy(X).cuda()))
    ref, _ = omlp.forward(p.astype(np.float64), X.astype(np.float64))
    e1, e2 = nrel(y, ref), nrel(y, _mimic_forward(p.astype(np.float64), X.astype(np.float64)))
    say(f"n={n}: rel error vs FP64 oracle {e1:.2e}, vs BF16-input oracle {e2:.2e}")
    assert e1 < INFER_TOL and e2 < INFER_MIMIC_TOL


def test_inference_empty_and_errors(small):
    torch = pytest.importorskip("torch")
    from paper_2409_20380_amd import ebe
    sol = small["sol"]
    say("mlp inference edge cases")
    sol.mlp_set(bf16_params(1), [1.0, 1.0, 1.0, 1.0])
    assert sol.mlp_forward(torch.zeros((0, 15), dtype=torch.float32, device="cuda")).shape == (0, 3)
    with pytest.raises(ebe.EbeError):
        sol.mlp_set(bf16_params(1), [1.0, 0.0, 1.0, 1.0])          # scales must be positive
    bad = bf16_params(1); bad[7] = np.nan
    with pytest.raises(ebe.EbeError):
        sol.mlp_set(bad, [1.0, 1.0, 1.0, 1.0])


@pytest.mark.parametrize("n", [300, 8192])
def test_gradient_matches_oracle(small, n):
    torch = pytest.importorskip("torch")
    sol = small["sol"]
    say("mlp gradient n", n)
    p = bf16_params(21)
    sol.mlp_set(p, [1.0, 1.0, 1.0, 1.0])
    rng = np.random.default_rng([n, 8])
    # inputs exactly representable in BF16: the training forward takes its inputs in BF16
    X = omlp.bf16_round(rng.standard_normal((n, 15))).astype(np.float32)
    T = rng.standard_normal((n, 3)).astype(np.float32)
    g, loss = sol.mlp_grad(torch.from_numpy(X).cuda(), torch.from_numpy(T).cuda())
    L, gref = omlp.loss_and_grad(p.astype(np.float64), X.astype(np.float64), T.astype(np.float64))
    g = to_host(g)
    bounds = [0, 960, 1024, 5120, 5184, 5376, 5379]
    errs = [nrel(g[a:b], gref[a:b]) for a, b in zip(bounds[:-1], bounds[1:])]
    say(f"n={n}: loss {loss:.6f} vs {L:.6f}; per-block gradient errors " + " ".join(f"{e:.1e}" for e in errs))
    assert abs(loss - L) <= 1e-5 * L
    assert max(errs) < GRAD_TOL


def test_adam_matches_oracle(small):
    torch = pytest.importorskip("torch")
    sol = small["sol"]
    say("adam steps")
    p = bf16_params(31)
    sol.mlp_set(p, [1.0, 1.0, 1.0, 1.0])
    w, m, v = p.astype(np.float64), np.zeros(p.size), np.zeros(p.size)
    rng = np.random.default_rng(77)
    for t in (1, 2, 3):
        g = (rng.standard_normal(p.size) * 1e-2).astype(np.float32)
        sol.mlp_adam(torch.from_numpy(g).cuda(), 1e-3)
        w, m, v = omlp.adam_step(w, m, v, g.astype(np.float64), t, 1e-3)
    wg, _ = sol.mlp_get()
    err = np.abs(wg - w).max()
    say(f"max |w_gpu - w_oracle| after 3 steps: {err:.2e} (lr 1e-3)")
    assert err < 1e-6


def test_collected_samples(small, oracle_lib):
    """Collected rows: displacements u^{it-1..it-4}, force, and du - du_AB at the sampled nodes."""
    torch = pytest.importorskip("torch")
    from paper_2409_20380_amd import ebe
    c = small
    wl, sol, m = c["wl"], c["sol"], c["model"]
    say("sample collection")
    nodes = inputs.sample_nodes(5, c["fx"], 40)
    sol.reset()
    sol.set_predictor(ebe.PRED_SNAPSHOT)
    sol.collect(20 * nodes.size, torch.from_numpy(nodes).cuda())
    hist = [np.zeros(m.n3)] * 4
    rows = []
    for it in range(1, 13):
        vh = to_host(sol.get_history()[0])
        u_prev = to_host(sol.get_state()[0])
        st = sol.step(base_acc=c["wave"][it])
        u_new = to_host(sol.get_state()[0])
        if it >= 5:
            f = m.rhs(np.zeros(m.n3), np.zeros(m.n3), np.zeros(m.n3), wl.dt, c["aR"], c["bR"], g=c["wave"][it])
            X = omlp.features([u_prev] + hist[:3], f, 1.0, 1.0, 1.0)[nodes]
            du = (u_new - u_prev).reshape(-1, 3)[nodes]
            dab = oracle_lib.ab4(wl.dt, vh[0], vh[1], vh[2], vh[3]).reshape(-1, 3)[nodes]
            rows.append(np.concatenate([X, du - dab], axis=1))
        hist = [u_prev] + hist[:3]
        assert st.status == 0
    sol.collect(0, None)
    got = to_host(sol.samples())
    expect = np.concatenate(rows)
    assert got.shape == expect.shape == (8 * nodes.size, 18)
    for a, b in ((0, 12), (12, 15), (15, 18)):
        e = nrel(got[:, a:b], expect[:, a:b])
        say(f"columns {a}..{b - 1}: rel error {e:.2e}")
        assert e < 1e-5
    with pytest.raises(ebe.EbeError):
        sol.collect(100, torch.tensor([0, m.n], dtype=torch.int32, device="cuda"))


def test_predict_learned_matches_oracle(small, oracle_lib):
    """Kind 3 guess = AB4 increment + s_t * network(features), features from the state.
    ebe_predict returns the candidate ebe_step would keep, so the history is chosen to
    make the comparison decided by the network alone: an all-zero snapshot ring makes
    the kind-2 guess the AB4 increment exactly, and with a tiny output scale s_t the
    learned candidate's residual differs from it to first order in the network output,
    so of the network and its negation (last layer's sign flipped) exactly one is kept."""
    torch = pytest.importorskip("torch")
    from paper_2409_20380_amd import ebe
    c = small
    wl, sol, m = c["wl"], c["sol"], c["model"]
    s, it = wl.s, 40
    say("predict kind 3 on identical history")
    rng = np.random.default_rng(12)
    vh = rng.standard_normal((4, m.n3)) * 1e-3
    ring = np.zeros((s + 1, m.n3))
    u = rng.standard_normal(m.n3) * 1e-2
    free = c["fx"].ravel() == 0
    vh[:, ~free] = 0.0; u[~free] = 0.0
    f = rng.standard_normal(m.n3); f[~free] = 0.0
    scales = np.array([1e-2, 1e-4, 1.0, 1e-12], dtype=np.float32)
    p = bf16_params(41, gain=0.5)
    w3 = 64 * 15 + 64 + 64 * 64 + 64      # offset of W3; W3 and b3 end the parameter vector
    sol.set_state(to_dev(u))
    sol.set_predictor(ebe.PRED_LEARNED)
    dab = oracle_lib.ab4(wl.dt, vh[0], vh[1], vh[2], vh[3])
    hdt = 0.5 * wl.dt
    us = [u]
    for q in range(3):
        us.append(us[-1] - hdt * (vh[q] + vh[q + 1]))
    X = omlp.features(us, f, float(scales[0]), float(scales[1]), float(scales[2]))
    kept = []
    for sign in (1.0, -1.0):
        ps_ = p.copy()
        ps_[w3:] *= sign
        sol.mlp_set(ps_, scales)
        sol.set_history(to_dev(vh), to_dev(ring), it)
        xl, st = sol.predict(f_next=to_dev(f))
        assert st.learned in (0, 1) and st.map_kept == 1 and st.res0_map == st.res0_ab
        kept.append(st.learned)
        if st.learned:
            corr = (to_host(xl) - dab).reshape(-1, 3)
            ref = omlp.correction(ps_.astype(np.float64), X, float(scales[3]))
            ref[c["fx"] == 1] = 0.0
            e = nrel(corr, ref)
            say(f"sign {sign:+.0f}: AB-error estimate kept, rel error vs FP64 oracle {e:.2e}")
            assert e < INFER_TOL
            assert st.res0 == st.res0_learned < st.res0_ab
        else:
            xa = np.where(free, dab, 0.0)
            assert np.abs(to_host(xl) - xa).max() <= 1e-10 * np.abs(xa).max()
    assert sorted(kept) == [0, 1]
    # steps before the fifth use the plain guess
    sol.set_history(to_dev(vh), to_dev(ring), 2)
    xl2, st2 = sol.predict(f_next=to_dev(f))
    assert st2.learned == -1
    sol.set_predictor(ebe.PRED_SNAPSHOT)
    xs2, _ = sol.predict(f_next=to_dev(f))
    assert np.array_equal(to_host(xl2), to_host(xs2))
    sol.reset()


def _kind3_trajectory(c, oracle_lib, params=None, scales=None):
    """Kind 3 (an untrained network unless params are given): per step the kept
    guess has the smaller initial residual, and the trajectory is the oracle's
    to the tolerance (the predictor changes the iteration count, not the
    answer, so the oracle reference is the tight kind-2 run).  Returns the
    number of steps that kept the learned candidate."""
    from paper_2409_20380_amd import ebe
    wl, sol = c["wl"], c["sol"]
    sol.reset()
    if params is None:
        sol.mlp_set(bf16_params(51, gain=0.2), [1e-3, 1e-4, 1e4, 1e-6])
    else:
        sol.mlp_set(params, scales)
    sol.set_predictor(ebe.PRED_LEARNED)
    U, evaluated, losses, kept = [], 0, 0, 0
    for it in range(1, 41):
        st = sol.step(base_acc=c["wave"][it])
        assert st.status == 0 and st.res_true < wl.tol
        due = it >= 5 and (losses < 8 or it % 16 == 0)      # the documented evaluation rule
        if due:
            evaluated += 1
            assert st.learned in (0, 1)
            best = min(st.res0_snapshot, st.res0_learned)
            assert abs(st.res0 - best) <= 1e-9 * best
            assert st.learned == int(st.res0_learned < st.res0_snapshot)
            losses = 0 if st.learned else losses + 1
            kept += st.learned
        else:
            assert st.learned == -1
        U.append(to_host(sol.get_state()[0]))
    assert evaluated >= 8
    orc = oracle_lib.Stepper(c["model"], wl.dt, c["aR"], c["bR"], s=wl.s, kind=2, tol=1e-13, regions=c["regions"])
    Uref = []
    for it in range(1, 41):
        orc.step(g=c["wave"][it])
        Uref.append(orc.u.copy())
    err = nrel(np.array(U), np.array(Uref))
    say(f"space-time rel L2 vs tight oracle {err:.2e}; learned candidate kept on {kept} of {evaluated} steps")
    assert err < 1e-6
    sol.set_predictor(ebe.PRED_SNAPSHOT)
    sol.reset()
    return kept


def test_learned_steps_keep_the_better_guess_and_the_answer(small, oracle_lib):
    say("kind 3 trajectory, untrained network, FP64 refine")
    _kind3_trajectory(small, oracle_lib)


def test_learned_steps_with_mixed_precision_refine(oracle_lib):
    """The learned guess composes with the FP32 inner solve: same selection rule,
    same answer to the tolerance."""
    from paper_2409_20380_amd import ebe
    say("kind 3 trajectory, untrained network, FP32 inner solve")
    c = build_case(SMALL, oracle_lib, precision=ebe.PREC_FP32)
    try:
        _kind3_trajectory(c, oracle_lib)
    finally:
        c["sol"].close()


@pytest.mark.slow
def test_full_size_inference_sampled_rows():
    """Headline mesh size (1,081,665 nodes), the size the kind-3 step runs the network at:
    sampled rows of the inference kernel against the oracle."""
    torch = pytest.importorskip("torch")
    from paper_2409_20380_amd import ebe
    say("full-size inference")
    mesh = inputs.box_mesh(2, 2, 2)
    em, mat = inputs.two_layer_materials(mesh)
    fx = inputs.fixed_bottom(mesh)
    sol = ebe.Solver(0.01)
    sol.assemble(mesh.coords, mesh.conn, em, mat, fx)
    p = bf16_params(61)
    sol.mlp_set(p, [1.0, 1.0, 1.0, 1.0])
    n = 1081665
    X = torch.randn((n, 15), dtype=torch.float32, device="cuda", generator=torch.Generator("cuda").manual_seed(5))
    Y = to_host(sol.mlp_forward(X))
    rows = np.concatenate([np.random.default_rng(2).choice(n, 2000, replace=False), [0, n - 1]])
    Xs = to_host(X)[rows].astype(np.float64)
    e = nrel(Y[rows], _mimic_forward(p.astype(np.float64), Xs))
    say(f"sampled rows: rel error vs BF16-input oracle {e:.2e}")
    assert e < INFER_MIMIC_TOL
    sol.close()


def test_trained_network_generalises(oracle_lib):
    """What training gains: on a wave the network never saw, its estimate of the
    AB4 error has a loss well below that of the zero network (no correction,
    i.e. the AB4 guess alone), after training on trajectories the solver
    generated itself with the library's own kernels."""
    torch = pytest.importorskip("torch")
    from paper_2409_20380_amd import learn
    wl = inputs.Workload(SMALL.name, cells=SMALL.cells, nt=60, s=SMALL.s)
    say("train on 4 small-mesh trajectories, evaluate on a held-out wave")
    c = build_case(wl, oracle_lib)
    sol = c["sol"]
    try:
        nodes = torch.from_numpy(inputs.sample_nodes(3, c["fx"], 1024)).cuda()
        train_seeds = inputs.LEARN_TRAIN_SEEDS[:4]
        learn.generate(sol, wl, train_seeds, 60, nodes, len(train_seeds) * 56 * nodes.numel())
        losses = learn.train(sol, 1, [(1000, 1e-3), (500, 3e-4)], 1024)
        trained, scales = sol.mlp_get()
        # held-out samples (a different capacity drops the training samples)
        learn.generate(sol, wl, inputs.LEARN_TEST_SEEDS[:1], 60, nodes, 56 * nodes.numel())
        raw = sol.samples()
        pick = torch.from_numpy(inputs.minibatches(9, 1, 8192, raw.shape[0])[0]).cuda()
        raw = raw[pick]
        div = torch.tensor([scales[0]] * 3 + [scales[1]] * 9 + [scales[2]] * 3, device="cuda")
        X = (raw[:, :15] / div).contiguous()
        T = (raw[:, 15:] / float(scales[3])).contiguous()
        _, l_trained = sol.mlp_grad(X, T)
        sol.mlp_set(np.zeros_like(trained), scales)
        _, l_zero = sol.mlp_grad(X, T)
        say(f"training loss {losses[:20].mean():.3f} -> {losses[-50:].mean():.3f}; "
            f"held-out loss trained {l_trained:.3f} vs zero network {l_zero:.3f}")
        assert losses[-50:].mean() < 0.7 * losses[:20].mean()
        assert l_trained < 0.7 * l_zero
        # the trained network drives kind-3 steps on the case's own wave (not a
        # training wave): same selection rule and the oracle's answer.  How often
        # its candidate is kept is reported, not asserted: a node-wise estimate
        # with a lower mean-square error can still leave the larger residual
        # b - A x, since the operator weights node-to-node roughness heavily.
        say("kind 3 trajectory, trained network, FP64 refine")
        _kind3_trajectory(c, oracle_lib, params=trained, scales=scales)
    finally:
        sol.close()
