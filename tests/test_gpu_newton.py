"""Device Newton-GMRES on manufactured problems: R_F(X) = R(X) - R(X*) has the exact root X*
(drift speed C* included through the phase slot); both Jacobian precisions must reach
||R_F|| <= 1e-10 and recover X*, C*."""
import numpy as np
import pytest

import seeded_inputs as si
from oracle.solver import Problem

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def sc():
    import paper_2508_16635_amd as m
    m.load_library()
    return m


def _dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda")


@pytest.mark.parametrize("shell", [(12, 12, 4, 14, 1e-3, 78.0, 0.1), (24, 24, 4, 20, 1e-3, 78.0, 0.1)],
                         ids=["L12N14", "L24N20"])
@pytest.mark.parametrize("prec", [0, 1], ids=["fp64", "mixed"])
def test_manufactured_newton(sc, shell, prec):
    L, M, m0, N, Ek, Ra, amp = shell
    plan = sc.Plan(L, M, m0, N, Ek=Ek, Ra=Ra, Pr=1.0, dt=200.0, nvec_max=1)
    plan.factor()
    ora = Problem(L, M, m0, N, Ek=Ek, Ra=Ra, Pr=1.0, dt=200.0)
    lay = si.Layout(L, M, m0, N)
    Xs = ora.clean(si.random_state(lay, 3999, amp=(amp, amp, amp), p=2) + ora.conductive_state())
    J = si.default_phase_slot(lay, Xs)
    Cs = 0.5
    # forcing F* = -R(X*), computed by the library itself in FP64
    Fd = torch.empty(plan.n_real, dtype=torch.float64, device="cuda")
    plan.newton_residual(_dev(Xs), Cs, Fd)
    Fd.neg_()
    d = ora.clean(si.random_state(lay, 77, p=2))
    d[J] = 0.0
    X0 = Xs + 1e-3 * np.linalg.norm(Xs) * d / np.linalg.norm(d)
    xd = _dev(X0)
    C, rep = plan.newton(xd, Cs + 1e-3, J, tol=1e-10, gmres_tol=1e-10 if prec == 0 else 1e-6, restart=40,
                         max_newton=10, max_matvec=200, prec=prec, forcing=Fd)
    X = xd.cpu().numpy()
    print(f"shell L={L} N={N} prec={prec}: {rep}", flush=True)
    assert rep["converged"], rep
    assert rep["rnorm"][-1] <= 1e-10
    assert np.linalg.norm(X - Xs) <= 1e-8 * np.linalg.norm(Xs)
    assert abs(C - Cs) <= 1e-8


def test_newton_matches_oracle_trajectory(sc):
    """First Newton step from the same guess: GPU (FP64) and oracle decrements agree."""
    L, M, m0, N = 10, 10, 2, 12
    plan = sc.Plan(L, M, m0, N, Ek=1e-3, Ra=78.0, dt=200.0, nvec_max=1)
    plan.factor()
    ora = Problem(L, M, m0, N, Ek=1e-3, Ra=78.0, Pr=1.0, dt=200.0)
    lay = si.Layout(L, M, m0, N)
    X0 = ora.clean(si.random_state(lay, 5, amp=(0.05, 0.05, 0.05), p=2) + ora.conductive_state())
    J = si.default_phase_slot(lay, X0)
    from oracle.solver import newton as onewton
    Xo, Co, hist = onewton(ora, X0.copy(), 0.2, J, tol=0.0, gmres_tol=1e-12, max_newton=1)
    xd = _dev(X0)
    C, rep = plan.newton(xd, 0.2, J, tol=0.0, gmres_tol=1e-12, restart=40, max_newton=1, max_matvec=400, prec=0)
    X = xd.cpu().numpy()
    print("oracle", hist, "gpu", rep["rnorm"], flush=True)
    assert abs(rep["rnorm"][0] - hist[0]) <= 1e-12 * hist[0]
    assert np.linalg.norm(X - Xo) <= 1e-9 * np.linalg.norm(X0 - Xo)
    assert abs(C - Co) <= 1e-9 * max(1.0, abs(0.2 - Co))


@pytest.mark.parametrize("prec", [0, 1], ids=["fp64", "mixed"])
def test_newton_converges_to_the_rw4_of_the_oracle(sc, prec):
    """The converged rotating wave RW4 of the tiny shell (L = M = 16, m0 = 4, N = 16, Ek = 1e-3,
    Ra = 78; tests/golden/rw4_L16_m4_N16.npz, computed by the oracle): the device Newton-GMRES,
    started 1e-2 |X*| away with the drift speed off by 0.05, returns to the same X* and C*."""
    import os
    d = np.load(os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "rw4_L16_m4_N16.npz"),
                allow_pickle=False)
    Xs, Cs, J = d["X"], float(d["C"]), int(d["J"])
    L, M, m0, N = (int(v) for v in d["shell"])
    Ek, Pr, Ra = (float(v) for v in d["params"])
    plan = sc.Plan(L, M, m0, N, Ek=Ek, Ra=Ra, Pr=Pr, dt=200.0, nvec_max=1)
    plan.factor()
    ora = Problem(L, M, m0, N, Ek=Ek, Ra=Ra, Pr=Pr, dt=200.0)
    lay = si.Layout(L, M, m0, N)
    dd = ora.clean(si.random_state(lay, 4001, p=2))
    dd[J] = 0.0
    X0 = Xs + 1e-2 * np.linalg.norm(Xs) * dd / np.linalg.norm(dd)
    xd = _dev(X0)
    C, rep = plan.newton(xd, Cs + 0.05, J, tol=1e-12, gmres_tol=1e-12 if prec == 0 else 1e-6, restart=40,
                         max_newton=12, max_matvec=400, prec=prec)
    X = xd.cpu().numpy()
    ex, ec = np.linalg.norm(X - Xs) / np.linalg.norm(Xs), abs(C - Cs) / abs(Cs)
    print(f"RW4 prec={prec}: {rep}; |X - X*|/|X*| {ex:.2e}, |C - C*|/|C*| {ec:.2e}", flush=True)
    assert rep["converged"] and rep["rnorm"][-1] <= 1e-12
    assert ex <= 1e-10 and ec <= 1e-10


@pytest.mark.skip(reason="HIP graph capture is switched off (a captured batch call crashed the host process; "
                         "cause not found); this case uses the same capture path")
@pytest.mark.parametrize("prec", [0, 1], ids=["fp64", "mixed"])
def test_newton_with_graph_capture_equals_eager(sc, prec):
    """graph_capture: the Arnoldi chunks of GMRES are captured into HIP graphs and replayed (the
    same graphs across restart cycles and Newton steps: the drift speed is read from device
    memory); the Newton history, state and drift speed are identical to the eager launches."""
    L, M, m0, N, Ek, Ra = 12, 12, 4, 14, 1e-3, 78.0
    out = []
    for gc in (0, 1):
        plan = sc.Plan(L, M, m0, N, Ek=Ek, Ra=Ra, Pr=1.0, dt=200.0, nvec_max=1, graph_capture=gc)
        plan.factor()
        ora = Problem(L, M, m0, N, Ek=Ek, Ra=Ra, Pr=1.0, dt=200.0)
        lay = si.Layout(L, M, m0, N)
        Xs = ora.clean(si.random_state(lay, 3999, amp=(0.1, 0.1, 0.1), p=2) + ora.conductive_state())
        J = si.default_phase_slot(lay, Xs)
        Fd = torch.empty(plan.n_real, dtype=torch.float64, device="cuda")
        plan.newton_residual(_dev(Xs), 0.5, Fd)
        Fd.neg_()
        d = ora.clean(si.random_state(lay, 77, p=2))
        d[J] = 0.0
        xd = _dev(Xs + 1e-3 * np.linalg.norm(Xs) * d / np.linalg.norm(d))
        C, rep = plan.newton(xd, 0.501, J, tol=1e-10, gmres_tol=1e-10 if prec == 0 else 1e-6, restart=20,
                             max_newton=10, max_matvec=400, prec=prec, forcing=Fd)
        print(f"graph_capture={gc}: {rep}", flush=True)
        assert rep["converged"]
        out.append((xd.cpu().numpy(), C, rep))
        plan.close()
    (X0, C0, r0), (X1, C1, r1) = out
    assert r0 == r1 and C0 == C1 and np.array_equal(X0, X1)
