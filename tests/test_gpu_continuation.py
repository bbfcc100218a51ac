"""Continuation on the GPU (sc_cont_*, Sec. 3.5, 3.6, 4.2) and grid refinement (sc_interpolate,
sc_tail_ratios, Sec. 4.2) against the oracle.

* Refinement and tail ratios: the library's interpolation of a state onto a finer grid and its
  tail ratios equal the oracle's.
* Ra continuation of the rotating wave RW4 of the tiny shell (tests/golden/rw4_L16_m4_N16.npz):
  the GPU session and the oracle's continuation driver, started from the same converged point
  with the same options, produce the same branch (parameters, drift speeds, states).
* Ek continuation with refinement: every converged point of the GPU session is a root of the
  oracle's residual at its (Ek, Ra = ra_coef Ek^(-1/3), L, N), the step sizes follow eq:new_EK,
  and the refinement happens when the reported (and oracle-recomputed) tail ratio exceeds the
  threshold.
"""
import os

import numpy as np
import pytest

import seeded_inputs as si
from oracle import physics
from oracle.continuation import Continuation, step_factor
from oracle.grids import Grid
from oracle.resolution import interpolate, tail_ratios
from oracle.solver import Problem, newton

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "rw4_L16_m4_N16.npz")


@pytest.fixture(scope="module")
def sc():
    import paper_2508_16635_amd as m
    m.load_library()
    return m


@pytest.fixture(scope="module")
def rw4():
    d = np.load(GOLDEN, allow_pickle=False)
    return dict(X=d["X"], C=float(d["C"]), J=int(d["J"]))


def _dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda")


def test_interpolate_and_tail_ratios_match_the_oracle(sc):
    coarse = sc.Plan(10, 10, 2, 12, Ek=1e-3, Ra=78.0, nvec_max=1)
    fine = sc.Plan(13, 13, 2, 17, Ek=1e-3, Ra=78.0, nvec_max=1)
    lay = si.Layout(10, 10, 2, 12)
    X = si.random_state(lay, 17, p=2.0)
    y = torch.empty(fine.n_real, dtype=torch.float64, device="cuda")
    sc.interpolate(coarse, _dev(X), fine, y)
    ref = interpolate(Grid(10, 10, 2, 12), X, Grid(13, 13, 2, 17))
    e = np.abs(y.cpu().numpy() - ref).max() / np.abs(ref).max()
    print(f"interpolation max rel diff {e:.2e}", flush=True)
    assert e <= 1e-13
    back = torch.empty(coarse.n_real, dtype=torch.float64, device="cuda")
    sc.interpolate(fine, y, coarse, back)
    assert np.abs(back.cpu().numpy() - X).max() <= 1e-12 * np.abs(X).max()
    rc, rl = coarse.tail_ratios(_dev(X))
    orc, orl = tail_ratios(Grid(10, 10, 2, 12), X)
    print(f"tail ratios {rc:.6e} {rl:.6e} vs oracle {orc:.6e} {orl:.6e}", flush=True)
    assert abs(rc - orc) <= 1e-12 * orc and abs(rl - orl) <= 1e-12 * orl


def test_ra_continuation_of_rw4_matches_the_oracle(sc, rw4):
    L, M, m0, N, Ek = 16, 16, 4, 16, 1e-3
    opts = dict(n_opt=4, gamma=50.0, tol=1e-10, gmres_tol=1e-10, restart=40, max_newton=8, max_matvec=400)
    plan = sc.Plan(L, M, m0, N, Ek=Ek, Ra=78.0, dt=200.0, nvec_max=1)
    plan.factor()
    cont = sc.Continuation(plan, _dev(rw4["X"]), rw4["C"], rw4["J"], param=sc.SC_CONT_RA, prec=sc.SC_FP64, **opts)
    gpu = [cont.first]
    states = [cont.state()[0].cpu().numpy()]
    for i in range(4):
        pt = cont.step(dp_first=3.0)
        print(f"GPU point {i + 1}: {pt}", flush=True)
        assert pt["converged"]
        gpu.append(pt)
        states.append(cont.state()[0].cpu().numpy())
    cont.close()

    def solve(Ra, X, C):
        p = Problem(L, M, m0, N, Ek=Ek, Ra=Ra, Pr=1.0, dt=200.0)
        Xn, Cn, hist = newton(p, X, C, rw4["J"], tol=1e-10, gmres_tol=1e-10, restart=40, max_newton=8, max_gmres=400)
        return Xn, Cn, len(hist) - 1, hist[-1] <= 1e-10

    oc = Continuation(solve, n_opt=4, gamma=50.0)
    oc.add_point(78.0, rw4["X"], rw4["C"], gpu[0]["newton_steps"])
    for i in range(4):
        p, ok, r = oc.step(dp_first=3.0)
        assert ok
        g = gpu[i + 1]
        print(f"point {i + 1}: Ra {g['Ra']:.12f} vs {p:.12f}, C {g['C']:.12f} vs {oc.Cs[-1]:.12f}, "
              f"Newton steps {g['newton_steps']} vs {oc.iters[-1]}", flush=True)
        assert g["newton_steps"] == oc.iters[-1] and g["retries"] == r and bool(g["state_mode"]) == oc.state_mode[-1]
        assert abs(g["Ra"] - p) <= 1e-10 * p
        assert abs(g["C"] - oc.Cs[-1]) <= 1e-8 * max(1.0, abs(oc.Cs[-1]))
        assert np.linalg.norm(states[i + 1] - oc.states[-1]) <= 1e-8 * np.linalg.norm(oc.states[-1])
    # along this branch the drift slows as Ra grows (prograde towards retrograde, Sec. 2.2)
    Cs = [g["C"] for g in gpu]
    assert all(b < a for a, b in zip(Cs, Cs[1:]))


def test_ek_continuation_with_refinement(sc, rw4):
    L, M, m0, N = 16, 16, 4, 16
    ra_coef = 78.0 * 1e-3 ** (1.0 / 3.0)        # Ra = 78 at Ek = 1e-3, Ra proportional to Ek^(-1/3)
    plan = sc.Plan(L, M, m0, N, Ek=1e-3, Ra=78.0, dt=200.0, nvec_max=1)
    plan.factor()
    tol = 3e-3                                   # the tiny shell's Chebyshev tail (3.9e-3) exceeds it
    cont = sc.Continuation(plan, _dev(rw4["X"]), rw4["C"], rw4["J"], param=sc.SC_CONT_EK, n_opt=3, gamma=450.0,
                           ra_coef=ra_coef, refine_tol=tol, refine_growth=1.2, restart=60, max_matvec=600)
    pts = [cont.first]
    for i in range(3):
        pt = cont.step(dp_first=-0.05)
        print(f"Ek point {i + 1}: {pt}", flush=True)
        assert pt["converged"]
        pts.append(pt)
        X, C = cont.state()
        X = X.cpu().numpy()
        Ek, Ra, Lp, Np = pt["Ek"], pt["Ra"], pt["L"], pt["N"]
        assert abs(Ra - ra_coef * Ek ** (-1.0 / 3.0)) <= 1e-12 * Ra
        # a root of the oracle's residual at the point's parameters and resolution
        ora = Problem(Lp, Lp, m0, Np, Ek=Ek, Ra=Ra, Pr=1.0, dt=200.0)
        rn = np.linalg.norm(ora.residual(X, C))
        print(f"  oracle |R| {rn:.2e}", flush=True)
        assert rn <= 1e-9
    # refinement: first step's point had Chebyshev tail 3.9e-3 > tol on N = 16, so N grew to 20
    assert pts[1]["refined"] == 1 and pts[1]["N"] == 20 and pts[1]["L"] == 16
    assert pts[1]["cheb_ratio"] > tol and pts[1]["sh_ratio"] <= tol
    assert all(p["refined"] == 0 for p in pts[2:])
    # step sizes of eq:new_EK (no turning point here): dp_i+1 = alpha (p_i - p_i-1)
    for a, b, c in zip(pts, pts[1:], pts[2:]):
        if not c["state_mode"] and not c["retries"]:
            alpha = step_factor(3, max(b["newton_steps"], 1))
            assert abs((c["param"] - b["param"]) - alpha * (b["param"] - a["param"])) <= 1e-12
    cont.close()
