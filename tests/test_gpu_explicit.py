"""The explicit-Coriolis variant (Sec. 3.1: eq:expcor_e / eq:expcor_f with the force of
eq:defineFexp) on the GPU against the oracle's explicit variant, and its Newton-GMRES on the
converged rotating wave RW4 beside the implicit one (the comparison of Sec. 5)."""
import os

import numpy as np
import pytest

import seeded_inputs as si
from oracle.solver import Problem
from parity_util import FP64_BLOCK, check

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

SMALL = [(16, 16, 1, 16, 1e-3, 78.0, 200.0), (12, 12, 4, 14, 1e-3, 78.0, 200.0), (12, 12, 4, 14, 1e-3, 78.0, 1e-4)]


@pytest.fixture(scope="module")
def sc():
    import paper_2508_16635_amd as m
    m.load_library()
    return m


def _dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda")


@pytest.mark.parametrize("cfg", SMALL, ids=["L16m1", "L12m4", "L12m4-dt1e-4"])
def test_explicit_step_residual_and_jvp(sc, cfg):
    L, M, m0, N, Ek, Ra, dt = cfg
    plan = sc.Plan(L, M, m0, N, Ek=Ek, Ra=Ra, Pr=1.0, dt=dt, nvec_max=4, coriolis=sc.SC_CORIOLIS_EXPLICIT)
    plan.factor()
    ora = Problem(L, M, m0, N, Ek=Ek, Ra=Ra, Pr=1.0, dt=dt, coriolis="explicit")
    lay = si.Layout(L, M, m0, N)
    X = si.random_state(lay, 101, amp=(1e-1, 1e-1, 1e-1), p=2) + ora.conductive_state()
    C = 0.3
    xd = _dev(X)
    out = torch.empty_like(xd)
    plan.step(xd, C, out)
    check(lay, out.cpu().numpy(), ora.step(X, C), 1e-12, FP64_BLOCK, f"explicit {cfg} step")
    plan.newton_residual(xd, C, out, norm=False)
    check(lay, out.cpu().numpy(), ora.residual(X, C), 1e-12, FP64_BLOCK, f"explicit {cfg} residual")
    J = si.default_phase_slot(lay, X)
    plan.set_base(xd, C, J)
    ora.set_base(X, C, J)
    V = si.random_vectors(lay, [1001, 1002, 1003, 1004])
    vd = _dev(V)
    for prec, tol, btol in ((0, 1e-12, FP64_BLOCK), (1, 1e-6, 1e-5)):
        yd = torch.empty_like(vd)
        plan.jvp(vd, yd, prec)
        Y = yd.cpu().numpy()
        for i in range(len(V)):
            check(lay, Y[i], ora.jvp(V[i]), tol, btol, f"explicit {cfg} prec={prec} vec {i}")


def test_explicit_newton_on_rw4_needs_more_actions(sc):
    """From the same perturbed RW4, Newton-GMRES with implicit and with explicit Coriolis: both
    converge (the explicit root differs from the implicit one only by the radial truncation of
    the projected Coriolis force), and the explicit one needs more Jacobian actions."""
    d = np.load(os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "rw4_L16_m4_N16.npz"),
                allow_pickle=False)
    Xs, Cs, J = d["X"], float(d["C"]), int(d["J"])
    L, M, m0, N = (int(v) for v in d["shell"])
    Ek, Pr, Ra = (float(v) for v in d["params"])
    lay = si.Layout(L, M, m0, N)
    dd = si.random_state(lay, 4001, p=2)
    dd[lay.nonphysical_mask()] = 0.0
    dd[J] = 0.0
    X0 = Xs + 1e-2 * np.linalg.norm(Xs) * dd / np.linalg.norm(dd)
    out = {}
    for name, cor in (("implicit", sc.SC_CORIOLIS_IMPLICIT), ("explicit", sc.SC_CORIOLIS_EXPLICIT)):
        plan = sc.Plan(L, M, m0, N, Ek=Ek, Ra=Ra, Pr=Pr, dt=200.0, nvec_max=1, coriolis=cor)
        plan.factor()
        xd = _dev(X0)
        C, rep = plan.newton(xd, Cs + 0.05, J, tol=1e-10, gmres_tol=1e-10, restart=128, max_newton=10,
                             max_matvec=4000, prec=0)
        out[name] = (xd.cpu().numpy(), C, rep)
        print(f"{name}: {rep}", flush=True)
        assert rep["converged"]
        plan.close()
    Xe, Ce, repe = out["explicit"]
    Xi, Ci, repi = out["implicit"]
    ora = Problem(L, M, m0, N, Ek=Ek, Ra=Ra, Pr=Pr, dt=200.0, coriolis="explicit")
    assert np.linalg.norm(ora.residual(Xe, Ce)) <= 1e-9
    assert np.linalg.norm(Xe - Xi) <= 1e-2 * np.linalg.norm(Xi) and abs(Ce - Ci) <= 1e-2 * abs(Ci)
    assert repe["matvecs"] > 2 * repi["matvecs"]
