"""The allocation-free residual (sc_newton_residual_noalloc) against sc_newton_residual: the same
residual vector and norm, on two calls in a row, the second on a smaller shell."""
import numpy as np
import pytest

import seeded_inputs as si

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def sc():
    import paper_2508_16635_amd as m
    m.load_library()
    return m


def test_noalloc_residual_matches_the_allocating_one(sc):
    shells = [(64, 64, 6, 32, 1e-4, 168.0, 0.5), (12, 12, 4, 14, 1e-3, 78.0, 0.3)]   # larger first
    rn_dev = torch.full((1,), float("nan"), dtype=torch.float64, device="cuda")
    for L, M, m0, N, Ek, Ra, C in shells:
        print(f"plan L={L} N={N}", flush=True)
        plan = sc.Plan(L, M, m0, N, Ek=Ek, Ra=Ra, Pr=1.0, dt=200.0, nvec_max=1)
        plan.factor()
        lay = si.Layout(L, M, m0, N)
        ri, ro = 0.35 / 0.65, 1.0 / 0.65
        X = si.random_state(lay, 11, amp=(1.0, 1.0, 0.1), p=2.0, t_offset=lambda x: ro * ri / ((x + ri + ro) / 2) - ri)
        xd = torch.from_numpy(X).cuda()
        r_ref = torch.empty_like(xd)
        rn_ref = plan.newton_residual(xd, C, r_ref)
        r = torch.full_like(xd, float("nan"))
        plan.newton_residual_noalloc(xd, C, r, rn_dev)
        torch.cuda.synchronize()
        rh, rrh = r.cpu().numpy(), r_ref.cpu().numpy()
        rn = float(rn_dev.cpu()[0])
        print(f"L={L} N={N}: |r| {rn:.15e} vs {rn_ref:.15e}", flush=True)
        assert np.array_equal(rh, rrh)
        assert abs(rn - rn_ref) <= 1e-13 * rn_ref
        assert abs(rn - np.linalg.norm(rrh)) <= 1e-13 * rn_ref
        plan.close()
