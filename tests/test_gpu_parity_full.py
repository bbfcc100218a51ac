"""GPU parity at the full shells (L=64/N=32 and L=128/N=48) and edge cases, against the FP64
oracle on sampled vectors, in the batched launch configuration the benchmark times."""
import numpy as np
import pytest

import seeded_inputs as si
from oracle.solver import Problem
from parity_util import FP64_BLOCK, check

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

# (L, M, m0, N, Ek, Ra, seed_base, amp) -- Ra = 1.2 * 6.5 Ek^(-1/3)
SHELL_C2 = (64, 64, 6, 32, 1e-4, 168.0, 201, (4.0, 4.0, 0.1))
SHELL_C3 = (128, 128, 10, 48, 1e-5, 362.0, 301, (8.0, 8.0, 0.1))


def _dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda")


def _rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


@pytest.fixture(scope="module")
def sc():
    import paper_2508_16635_amd as m
    m.load_library()
    return m


def _base(lay, ora, seed, amp):
    ri, ro = ora.g.ri, ora.g.ro
    return si.random_state(lay, seed, amp=amp, p=3.0, t_offset=lambda x: ro * ri / ((x + ri + ro) / 2) - ri)


@pytest.mark.parametrize("shell", [SHELL_C2, SHELL_C3], ids=["L64N32", "L128N48"])
def test_full_shell_jvp_batched(sc, shell):
    """nvec = 17 (a full group of 16 plus a ragged tail of 1); every vector is compared with the
    oracle one by one (global and per-(field, m) block errors), in both implicit solves of the
    mixed path (one FP64 solve, the default; the FP32 solve with one FP64 refinement pass, a
    plan of its own) and in FP64."""
    L, M, m0, N, Ek, Ra, seed, amp = shell
    nvec = 17
    plan = sc.Plan(L, M, m0, N, Ek=Ek, Ra=Ra, Pr=1.0, dt=200.0, nvec_max=nvec)
    plan.factor()
    ora = Problem(L, M, m0, N, Ek=Ek, Ra=Ra, Pr=1.0, dt=200.0)
    lay = si.Layout(L, M, m0, N)
    X = _base(lay, ora, seed, amp)
    J = si.default_phase_slot(lay, X)
    C = 0.5
    plan.set_base(_dev(X), C, J)
    ora.set_base(X, C, J)
    V = si.random_vectors(lay, range(seed * 10 + 1, seed * 10 + 1 + nvec))
    Vd = _dev(V)
    Y64 = torch.empty_like(Vd)
    Y32 = torch.empty_like(Vd)
    plan.jvp(Vd, Y64, sc.SC_FP64)
    plan.jvp(Vd, Y32, sc.SC_MIXED)
    plan2 = sc.Plan(L, M, m0, N, Ek=Ek, Ra=Ra, Pr=1.0, dt=200.0, nvec_max=nvec, mixed_solve=sc.SC_MIXED_SOLVE_FP32,
                    refine_mixed=1)
    plan2.factor()
    plan2.set_base(_dev(X), C, J)
    Y32r = torch.empty_like(Vd)
    plan2.jvp(Vd, Y32r, sc.SC_MIXED)
    torch.cuda.synchronize()
    y64, y32, y32r = Y64.cpu().numpy(), Y32.cpu().numpy(), Y32r.cpu().numpy()
    plan2.close()
    worst = {"fp64": 0.0, "mixed": 0.0, "mixed_fp32solve": 0.0}
    for i in range(nvec):
        ref = ora.jvp(V[i])
        tag = f"L={L} N={N} vec {seed * 10 + 1 + i}"
        worst["fp64"] = max(worst["fp64"], check(lay, y64[i], ref, 1e-12, FP64_BLOCK, tag + " fp64")[0])
        worst["mixed"] = max(worst["mixed"], check(lay, y32[i], ref, 1e-6, 1e-5, tag + " mixed")[0])
        worst["mixed_fp32solve"] = max(worst["mixed_fp32solve"],
                                       check(lay, y32r[i], ref, 1e-6, 1e-5, tag + " mixed fp32 solve")[0])
    print(f"L={L} N={N} worst relative error over {nvec} vectors vs the oracle: {worst}", flush=True)


@pytest.mark.parametrize("shell", [SHELL_C2, SHELL_C3], ids=["L64N32", "L128N48"])
def test_full_shell_residual(sc, shell):
    L, M, m0, N, Ek, Ra, seed, amp = shell
    plan = sc.Plan(L, M, m0, N, Ek=Ek, Ra=Ra, Pr=1.0, dt=200.0, nvec_max=1)
    plan.factor()
    ora = Problem(L, M, m0, N, Ek=Ek, Ra=Ra, Pr=1.0, dt=200.0)
    lay = si.Layout(L, M, m0, N)
    X = _base(lay, ora, seed, amp)
    Xd = _dev(X)
    R = torch.empty_like(Xd)
    rn = plan.newton_residual(Xd, 0.5, R)
    ref = ora.residual(X, 0.5)
    e = _rel(R.cpu().numpy(), ref)
    print(f"L={L} N={N} residual rel err {e:.2e}, |R| {rn:.6e} vs {np.linalg.norm(ref):.6e}", flush=True)
    assert e < 1e-12
    check(lay, R.cpu().numpy(), ref, 1e-12, FP64_BLOCK, f"L={L} N={N} residual")


def test_axisymmetric_and_odd_sizes(sc):
    """m0 > L (only m = 0, no phase slot) and odd N: FP64 jvp and step against the oracle."""
    L, M, m0, N = 7, 7, 9, 15
    plan = sc.Plan(L, M, m0, N, Ek=3e-3, Ra=50.0, Pr=0.7, dt=5.0, nvec_max=3)
    plan.factor()
    ora = Problem(L, M, m0, N, Ek=3e-3, Ra=50.0, Pr=0.7, dt=5.0)
    lay = si.Layout(L, M, m0, N)
    X = si.random_state(lay, 7, amp=(1e-1, 1e-1, 1e-1), p=2) + ora.conductive_state()
    plan.set_base(_dev(X), 0.0, -1)
    ora.set_base(X, 0.0, -1)
    V = si.random_vectors(lay, [71, 72, 73])
    Y = torch.empty((3, plan.n_real), dtype=torch.float64, device="cuda")
    plan.jvp(_dev(V), Y, sc.SC_FP64)
    y = Y.cpu().numpy()
    for i in range(3):
        check(lay, y[i], ora.jvp(V[i]), 1e-12, FP64_BLOCK, f"axisymmetric odd N vec {i}")
    out = torch.empty(plan.n_real, dtype=torch.float64, device="cuda")
    plan.step(_dev(X), 0.0, out)
    check(lay, out.cpu().numpy(), ora.step(X, 0.0), 1e-12, FP64_BLOCK, "axisymmetric odd N step")


def test_jvp_batch_limits(sc):
    L, M, m0, N = 8, 8, 2, 10
    plan = sc.Plan(L, M, m0, N, Ek=1e-3, Ra=50.0, dt=200.0, nvec_max=2)
    plan.factor()
    lay = si.Layout(L, M, m0, N)
    X = si.random_state(lay, 3)
    plan.set_base(_dev(X), 0.0, si.default_phase_slot(lay, X))
    V = torch.zeros((3, plan.n_real), dtype=torch.float64, device="cuda")
    with pytest.raises(sc.ShellConvError) as ei:
        plan.jvp(V, V.clone(), sc.SC_FP64)          # more than nvec_max
    assert ei.value.code == 1
    # a stale factor after changing Ek is refused until factor() runs again
    plan.set_params(50.0, 2e-3, 200.0)
    with pytest.raises(sc.ShellConvError) as ei:
        plan.jvp(V[:1], V[:1].clone(), sc.SC_FP64)
    assert ei.value.code == 2



def test_wide_theta_fallback_paths(sc):
    """N_theta = 258 > 256: the analysis runs on the GEMM path with the untiled output layout,
    and N_phi = 8 takes the Stockham ring in both precisions; FP64 and mixed jvp against the
    oracle."""
    L, M, m0, N = 171, 171, 80, 10
    plan = sc.Plan(L, M, m0, N, Ek=1e-3, Ra=60.0, Pr=1.0, dt=5.0, nvec_max=3)
    plan.factor()
    assert plan.layout["ntheta"] > 256
    ora = Problem(L, M, m0, N, Ek=1e-3, Ra=60.0, Pr=1.0, dt=5.0)
    lay = si.Layout(L, M, m0, N)
    X = si.random_state(lay, 5, amp=(1e-2, 1e-2, 1e-2), p=2) + ora.conductive_state()
    J = si.default_phase_slot(lay, X)
    plan.set_base(_dev(X), 0.2, J)
    ora.set_base(X, 0.2, J)
    V = si.random_vectors(lay, [11, 12, 13])
    Vd = _dev(V)
    Y64 = torch.empty_like(Vd)
    Y32 = torch.empty_like(Vd)
    plan.jvp(Vd, Y64, sc.SC_FP64)
    plan.jvp(Vd, Y32, sc.SC_MIXED)
    torch.cuda.synchronize()
    y64, y32 = Y64.cpu().numpy(), Y32.cpu().numpy()
    for i in range(3):
        ref = ora.jvp(V[i])
        check(lay, y64[i], ref, 1e-12, FP64_BLOCK, f"L={L} N_theta={plan.layout['ntheta']} vec {i} fp64")
        check(lay, y32[i], ref, 1e-6, 1e-5, f"L={L} N_theta={plan.layout['ntheta']} vec {i} mixed")


# the throughput-stress shell: Ra = 1.2 * 6.5 Ek^(-1/3)
SHELL_C5 = (255, 255, 12, 64, 3e-6, 541.0, 501, (8.0, 8.0, 0.1))


def test_stress_shell_linearization(sc):
    """L = M = 255, m0 = 12, N = 64 (N_theta = 384: batched-GEMM analysis; N_phi = 64: LDS ring
    kernel), beyond the oracle's reach: the FP64 Jacobian action equals central differences of
    the library's FP64 residual R(X, C), which is exactly quadratic in (X, C), for two step
    sizes; the mixed path agrees with the FP64 one within 1e-6 on 16 vectors."""
    L, M, m0, N, Ek, Ra, seed, amp = SHELL_C5
    print(f"plan L={L} N={N}", flush=True)
    plan = sc.Plan(L, M, m0, N, Ek=Ek, Ra=Ra, Pr=1.0, dt=200.0, nvec_max=16)
    plan.factor()
    lay = si.Layout(L, M, m0, N)
    assert lay.n_real == plan.n_real
    ri, ro = 0.35 / 0.65, 1.0 / 0.65
    X = si.random_state(lay, seed, amp=amp, p=3.0, t_offset=lambda x: ro * ri / ((x + ri + ro) / 2) - ri)
    J = si.default_phase_slot(lay, X)
    C = 0.5
    Xd = _dev(X)
    plan.set_base(Xd, C, J)
    V = _dev(si.random_vectors(lay, range(seed * 10, seed * 10 + 16)))
    Y64, Ym = torch.empty_like(V), torch.empty_like(V)
    plan.jvp(V, Y64, sc.SC_FP64)
    plan.jvp(V, Ym, sc.SC_MIXED)
    y64, ym = Y64.cpu().numpy(), Ym.cpu().numpy()
    worst = max(_rel(ym[i], y64[i]) for i in range(16))
    print(f"L={L} N={N} max mixed-vs-fp64 over 16 vectors {worst:.2e}", flush=True)
    assert worst <= 1e-6
    Rp, Rm = torch.empty_like(Xd), torch.empty_like(Xd)
    for i in (0, 15):
        v = V[i]
        c = float(v[J])
        u = v.clone()
        u[J] = 0.0
        for eps in (1.0, 1e-2):
            plan.newton_residual(Xd + eps * u, C + eps * c, Rp, norm=False)
            plan.newton_residual(Xd - eps * u, C - eps * c, Rm, norm=False)
            cd = ((Rp - Rm) / (2 * eps)).cpu().numpy()
            e = _rel(cd, y64[i])
            print(f"vector {i} eps {eps:g}: central difference vs FP64 jvp {e:.2e}", flush=True)
            assert e <= 1e-10
    plan.close()


@pytest.mark.timeout(900)
def test_stress_shell_vs_oracle(sc):
    """The stress shell against the oracle itself on one vector (the oracle's factor and one
    Jacobian action take about a minute of host time at this size)."""
    L, M, m0, N, Ek, Ra, seed, amp = SHELL_C5
    plan = sc.Plan(L, M, m0, N, Ek=Ek, Ra=Ra, Pr=1.0, dt=200.0, nvec_max=1)
    plan.factor()
    lay = si.Layout(L, M, m0, N)
    print("oracle factor at L=255, N=64", flush=True)
    ora = Problem(L, M, m0, N, Ek=Ek, Ra=Ra, Pr=1.0, dt=200.0)
    ora.factor()
    X = _base(lay, ora, seed, amp)
    J = si.default_phase_slot(lay, X)
    plan.set_base(_dev(X), 0.5, J)
    ora.set_base(X, 0.5, J)
    V = si.random_vectors(lay, [seed * 10])
    Vd = _dev(V)
    ref = ora.jvp(V[0])
    for prec, tol, btol in ((sc.SC_FP64, 1e-12, FP64_BLOCK), (sc.SC_MIXED, 1e-6, 1e-5)):
        Y = torch.empty_like(Vd)
        plan.jvp(Vd, Y, prec)
        check(lay, Y.cpu().numpy()[0], ref, tol, btol, f"L={L} N={N} vec {seed * 10} prec={prec}")
    plan.close()
