"""Mixed precision (needs an MI355X): flexible FP64 outer PCG whose
preconditioner is an inner block-Jacobi PCG with an FP32 element-by-element
matvec (vectors in FP32, or p and z stored in BF16).  The outer residual, the
dots, the stop test and the predictor stay FP64, so every result is checked
against the FP64 oracle to the same bars as the plain path; the error of each
result against the tight oracle is printed.
"""
import numpy as np
import pytest

from paper_2409_20380_amd import inputs
from tests.gpu_common import RAGGED, SMALL, build_case, to_dev, to_host

pytestmark = pytest.mark.gpu

TRAJ_TOL = 1e-6
PRECS = {"fp32": 1, "bf16": 2}


def say(*a):
    print("[gpu-case]", *a, flush=True)


@pytest.fixture(scope="module", params=list(PRECS))
def mixed(request, oracle_lib):
    name = request.param
    say("build small workload", SMALL.cells, "precision", name)
    c = build_case(SMALL, oracle_lib, precision=PRECS[name])
    c["prec"] = name
    yield c
    c["sol"].close()


def test_refine_matches_oracle(mixed, oracle_lib):
    m, sol = mixed["model"], mixed["sol"]
    say("mixed refine random rhs", mixed["prec"])
    b = inputs.random_vector(21, m.n3)
    b[mixed["fx"].ravel() == 1] = 0.0
    x = to_dev(np.zeros(m.n3))
    st = sol.refine(to_dev(b), x)
    xr = to_host(x)
    assert st.status == 0 and st.res_true < 1e-8
    assert st.inner_iters > 0
    assert np.linalg.norm(b - m.spmv("A", xr)) / np.linalg.norm(b) < 1e-8
    x_ref, _ = m.pcg(b, np.zeros(m.n3), tol=1e-13)
    err = np.linalg.norm(xr - x_ref) / np.linalg.norm(x_ref)
    _, so = m.pcg(b, np.zeros(m.n3), tol=1e-8)
    say(f"{mixed['prec']}: rel L2 error vs tight oracle {err:.3e}; outer iters {st.iters}, inner {st.inner_iters}, "
        f"plain FP64 oracle iters {so.iters}")
    assert err < 1e-6
    # the inner solve is a stronger preconditioner than block Jacobi alone
    assert st.iters < so.iters


def test_refine_edge_cases(mixed):
    from paper_2409_20380_amd import ebe
    torch = pytest.importorskip("torch")
    m, sol = mixed["model"], mixed["sol"]
    say("mixed refine edge cases", mixed["prec"])
    x = to_dev(inputs.random_vector(5, m.n3))
    st = sol.refine(torch.zeros(m.n3, dtype=torch.float64, device="cuda"), x)
    assert st.iters == 0 and float(x.abs().max()) == 0.0
    b = inputs.random_vector(22, m.n3); b[mixed["fx"].ravel() == 1] = 0.0
    x_ref, _ = m.pcg(b, np.zeros(m.n3), tol=1e-14)
    st = sol.refine(to_dev(b), to_dev(x_ref))
    assert st.iters == 0 and st.inner_iters == 0 and st.res_true < 1e-8
    b2 = b.copy(); fixed_dofs = np.where(mixed["fx"].ravel() == 1)[0]
    b2[fixed_dofs[:5]] = 3.0
    x = to_dev(np.zeros(m.n3))
    st = sol.refine(to_dev(b2), x)
    assert st.res_true < 1e-8
    np.testing.assert_array_equal(to_host(x)[fixed_dofs[:5]], 3.0)
    xn = np.zeros(m.n3); xn[np.where(mixed["fx"].ravel() == 0)[0][7]] = np.nan
    with pytest.raises(ebe.EbeError) as ei:
        sol.refine(to_dev(b), to_dev(xn))
    assert ei.value.code == ebe.E_NONFINITE


def test_max_iter_cap(oracle_lib):
    from paper_2409_20380_amd import ebe
    say("mixed max_iter cap")
    c = build_case(SMALL, oracle_lib, max_iter=2, precision=ebe.PREC_FP32)
    m, sol = c["model"], c["sol"]
    b = inputs.random_vector(23, m.n3); b[c["fx"].ravel() == 1] = 0.0
    st = sol.refine(to_dev(b), to_dev(np.zeros(m.n3)))
    assert st.status == ebe.NOT_CONVERGED and st.iters == 2 and st.res_true > 1e-8
    sol.close()


def _oracle_traj(c, oracle_lib, tol, nt):
    wl = c["wl"]
    st = oracle_lib.Stepper(c["model"], wl.dt, c["aR"], c["bR"], s=wl.s, kind=2, tol=tol, regions=c["regions"])
    U = []
    for it in range(1, nt + 1):
        st.step(g=c["wave"][it])
        U.append(st.u.copy())
    return np.array(U)


@pytest.mark.parametrize("case", ["small", "ragged"])
@pytest.mark.parametrize("prec", list(PRECS))
def test_trajectory_matches_oracle(case, prec, oracle_lib):
    wl = SMALL if case == "small" else RAGGED
    pe = 256 if case == "small" else 17
    say("mixed trajectory", case, prec, "steps", wl.nt)
    c = build_case(wl, oracle_lib, precision=PRECS[prec], patch_elems=pe)
    sol = c["sol"]
    U, its, inner, res = [], [], [], []
    for it in range(1, wl.nt + 1):
        st = sol.step(base_acc=c["wave"][it])
        assert st.status == 0
        U.append(to_host(sol.get_state()[0])); its.append(st.iters); inner.append(st.inner_iters)
        res.append(st.res_true)
    U = np.array(U)
    Uref = _oracle_traj(c, oracle_lib, 1e-13, wl.nt)
    err = np.linalg.norm(U - Uref) / np.linalg.norm(Uref)
    step_err = np.linalg.norm(U - Uref, axis=1) / np.maximum(np.linalg.norm(Uref, axis=1), 1e-300)
    say(f"{case}/{prec}: space-time rel L2 {err:.3e}, worst step {step_err.max():.3e}; outer iters/step "
        f"{np.mean(its):.2f}, inner {np.mean(inner):.1f}; max true residual {max(res):.2e}")
    assert err < TRAJ_TOL
    assert max(res) < wl.tol
    sol.close()


def test_mixed_is_deterministic(oracle_lib):
    from paper_2409_20380_amd import ebe
    say("mixed determinism")
    a = build_case(SMALL, oracle_lib, precision=ebe.PREC_BF16)
    b = build_case(SMALL, oracle_lib, precision=ebe.PREC_BF16)
    for it in range(1, 21):
        sa = a["sol"].step(base_acc=a["wave"][it])
        sb = b["sol"].step(base_acc=b["wave"][it])
        assert (sa.iters, sa.inner_iters) == (sb.iters, sb.inner_iters)
    assert np.array_equal(to_host(a["sol"].get_state()[0]), to_host(b["sol"].get_state()[0]))
    a["sol"].close(); b["sol"].close()
