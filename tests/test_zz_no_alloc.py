"""ebe_mlp_grad_noalloc (the entry point that allocates nothing) against ebe_mlp_grad
(needs an MI355X).

Both run the same kernels on the same inputs, so gradient and loss must agree
bitwise; the second pair of calls uses fewer samples than the first, so stale
contents of the fixed device array would show.  Also checked against the FP64
oracle of the network (the gradient bar of the learned-predictor tests).
"""
import numpy as np
import pytest

from oracle import mlp as omlp
from paper_2409_20380_amd import inputs
from tests.gpu_common import SMALL, build_case, to_host

pytestmark = pytest.mark.gpu

GRAD_TOL = 1e-4


def say(*a):
    print("[gpu-case]", *a, flush=True)


def _params(seed):
    p = inputs.mlp_init(seed, 1.0).astype(np.float64)
    rng = np.random.default_rng([seed, 5])
    p = p + 0.05 * rng.standard_normal(p.size) * (p == 0)
    return omlp.bf16_round(p).astype(np.float32)


def _batch(n, seed):
    rng = np.random.default_rng([n, seed])
    X = omlp.bf16_round(rng.standard_normal((n, 15))).astype(np.float32)
    T = rng.standard_normal((n, 3)).astype(np.float32)
    return X, T


@pytest.fixture(scope="module")
def case(oracle_lib):
    say("no-alloc gradient: build small workload", SMALL.cells)
    c = build_case(SMALL, oracle_lib)
    yield c
    c["sol"].close()


def test_noalloc_gradient_matches_allocating_entry_point(case):
    torch = pytest.importorskip("torch")
    from paper_2409_20380_amd import ebe
    sol = case["sol"]
    p = _params(61)
    sol.mlp_set(p, [1.0, 1.0, 1.0, 1.0])
    for n in (8192, 4096, 300):      # first the full capacity, then smaller batches
        say("no-alloc gradient n", n)
        X, T = _batch(n, 3)
        xd, td = torch.from_numpy(X).cuda(), torch.from_numpy(T).cuda()
        g_na, loss_na = sol.mlp_grad_noalloc(xd, td)
        g_ref, loss_ref = sol.mlp_grad(xd, td)
        assert np.array_equal(to_host(g_na), to_host(g_ref)), n
        assert loss_na == loss_ref
        # and the oracle of the network (FP64)
        L, gref = omlp.loss_and_grad(p.astype(np.float64), X.astype(np.float64), T.astype(np.float64))
        g = to_host(g_na).astype(np.float64)
        err = np.linalg.norm(g - gref) / np.linalg.norm(gref)
        say(f"n={n}: loss {loss_na:.6f} vs oracle {L:.6f}; gradient rel error {err:.1e}")
        assert abs(loss_na - L) <= 1e-5 * L and err < GRAD_TOL
    # without a loss pointer the call only enqueues work; same gradient
    X, T = _batch(300, 3)
    xd, td = torch.from_numpy(X).cuda(), torch.from_numpy(T).cuda()
    g2, none = sol.mlp_grad_noalloc(xd, td, want_loss=False)
    torch.cuda.synchronize()
    assert none is None and np.array_equal(to_host(g2), to_host(sol.mlp_grad(xd, td)[0]))


def test_noalloc_gradient_rejects_oversized_and_unready(case, oracle_lib):
    torch = pytest.importorskip("torch")
    from paper_2409_20380_amd import ebe
    sol = case["sol"]
    sol.mlp_set(_params(62), [1.0, 1.0, 1.0, 1.0])
    X, T = _batch(8193, 4)
    with pytest.raises(ebe.EbeError) as ei:
        sol.mlp_grad_noalloc(torch.from_numpy(X).cuda(), torch.from_numpy(T).cuda())
    assert ei.value.code == ebe.E_INVALID_ARG and "8192" in str(ei.value)
    fresh = build_case(SMALL, oracle_lib)["sol"]          # no weights set
    X, T = _batch(16, 4)
    with pytest.raises(ebe.EbeError) as ei:
        fresh.mlp_grad_noalloc(torch.from_numpy(X).cuda(), torch.from_numpy(T).cuda())
    assert ei.value.code == ebe.E_BAD_STATE
    fresh.close()
