"""Paper-resolution validation (Table 1, Sec. 5): the rotating wave RW4 at Ek = 1e-3, Ra = 120,
m0 = 4, computed on the GPU at the paper's resolution, has the drift speed the paper prints.

Route: the oracle's RW4 of the tiny shell (tests/golden/rw4_L16_m4_N16.npz, Ra = 78) carried by
sc_interpolate to L = M = 47, N = 46 (N_theta = 72 Gauss-Legendre nodes, as in Table 1's
(46, 72, 32 x 4)); Newton there; continuation in Ra (sc_cont_*) past 112; Newton at Ra = 120.
The paper's discretization differs in its details (tau rows, its own grids), so agreement is to
the resolution of both, not to rounding; the paper prints five digits."""
import os

import numpy as np
import pytest

import seeded_inputs as si

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

HERE = os.path.dirname(os.path.abspath(__file__))


@pytest.fixture(scope="module")
def sc():
    import paper_2508_16635_amd as m
    m.load_library()
    return m


def _table1():
    rows = [ln.split() for ln in open(os.path.join(HERE, "golden", "table1_rw4.txt")) if ln.strip() and ln[0] != "#"]
    Ek, Ra, M, Nr, Nth, _, C = rows[0]
    return float(Ek), float(Ra), int(M), int(Nr), int(Nth), float(C)


def test_rw4_drift_speed_of_table1(sc):
    Ek, Ra, m0, Nr, Nth, C_exact = _table1()
    d = np.load(os.path.join(HERE, "golden", "rw4_L16_m4_N16.npz"), allow_pickle=False)
    L, N = 47, Nr
    tiny = sc.Plan(16, 16, m0, 16, Ek=Ek, Ra=78.0, nvec_max=1)
    big = sc.Plan(L, L, m0, N, Ek=Ek, Ra=78.0, dt=200.0, nvec_max=1)
    assert big.layout["ntheta"] == Nth
    big.factor()
    x = torch.empty(big.n_real, dtype=torch.float64, device="cuda")
    sc.interpolate(tiny, torch.from_numpy(d["X"]).cuda(), big, x)
    J = si.default_phase_slot(si.Layout(L, L, m0, N), x.cpu().numpy())
    C, rep = big.newton(x, float(d["C"]), J, tol=1e-10, gmres_tol=1e-10, restart=100, max_newton=15, max_matvec=800)
    assert rep["converged"], rep
    cont = sc.Continuation(big, x, C, J, param=sc.SC_CONT_RA, n_opt=4, gamma=50.0, restart=100, max_matvec=800)
    while True:
        pt = cont.step(dp_first=5.0)
        print(f"continuation: Ra {pt['Ra']:.4f} C {pt['C']:.8f} Newton steps {pt['newton_steps']}", flush=True)
        assert pt["converged"]
        if pt["Ra"] > 112.0:
            break
    xs, Cs = cont.state()
    cont.close()
    big.set_params(Ra, Ek, 200.0)
    Cf, rep = big.newton(xs, Cs, J, tol=1e-10, gmres_tol=1e-10, restart=100, max_newton=15, max_matvec=800)
    rc, rl = big.tail_ratios(xs)
    print(f"Ra = {Ra}: C = {Cf:.8f} (Table 1: {C_exact}); {rep}; tail ratios {rc:.1e} {rl:.1e}", flush=True)
    assert rep["converged"] and rep["rnorm"][-1] <= 1e-10
    assert rc < 1e-6 and rl < 1e-5                   # resolved (the paper's criterion is 1e-6)
    assert abs(Cf - C_exact) <= 2e-4
