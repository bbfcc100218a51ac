"""GPU parity of libshellconv against the FP64 oracle (run on an MI355X)."""
import numpy as np
import pytest

import seeded_inputs as si
from oracle.solver import Problem
from parity_util import FP64_BLOCK, check

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

SMALL = [  # (L, M, m0, N, Ek, Ra, dt)
    (16, 16, 1, 16, 1e-3, 78.0, 200.0),
    (12, 12, 4, 14, 1e-3, 78.0, 200.0),
]


def _dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda")


def _host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


@pytest.fixture(scope="module")
def lib():
    import paper_2508_16635_amd as sc
    sc.load_library()
    return sc


def _setup(sc, cfg, nvec=4, mixed_solve=0):
    L, M, m0, N, Ek, Ra, dt = cfg
    plan = sc.Plan(L, M, m0, N, Ek=Ek, Ra=Ra, Pr=1.0, dt=dt, nvec_max=nvec, mixed_solve=mixed_solve)
    plan.factor()
    ora = Problem(L, M, m0, N, Ek=Ek, Ra=Ra, Pr=1.0, dt=dt)
    lay = si.Layout(L, M, m0, N)
    assert plan.n_real == lay.n_real == ora.n_real
    return plan, ora, lay


def _rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


@pytest.mark.parametrize("cfg", SMALL)
def test_step_and_residual_fp64(lib, cfg):
    plan, ora, lay = _setup(lib, cfg)
    X = si.random_state(lay, 101, amp=(1e-2, 1e-2, 1e-2), p=2) + ora.conductive_state()
    C = 0.3
    xd = _dev(X)
    out = torch.empty_like(xd)
    plan.step(xd, C, out)
    ref = ora.step(X, C)
    e1 = _rel(_host(out), ref)
    rn = plan.newton_residual(xd, C, out)
    R = ora.residual(X, C)
    e2 = _rel(_host(out), R)
    print(f"cfg={cfg} step rel err {e1:.2e} residual rel err {e2:.2e} |R| {rn:.6e} vs {np.linalg.norm(R):.6e}", flush=True)
    assert e1 < 1e-12
    assert e2 < 1e-12
    assert abs(rn - np.linalg.norm(R)) <= 1e-12 * np.linalg.norm(R)


def test_conductive_fixed_point(lib):
    plan, ora, lay = _setup(lib, SMALL[0])
    Xc = ora.conductive_state()
    r = torch.empty(plan.n_real, dtype=torch.float64, device="cuda")
    rn = plan.newton_residual(_dev(Xc), 0.0, r)
    print("conductive |R|", rn, flush=True)
    assert rn <= 1e-12 * np.linalg.norm(Xc)


@pytest.mark.parametrize("cfg", SMALL)
@pytest.mark.parametrize("prec,solve,tol,btol", [(0, 0, 1e-12, FP64_BLOCK), (1, 1, 1e-6, 1e-5), (1, 2, 1e-6, 1e-5)],
                         ids=["fp64", "mixed-fp64solve", "mixed-fp32solve-refined"])
def test_jvp(lib, cfg, prec, solve, tol, btol):
    plan, ora, lay = _setup(lib, cfg, mixed_solve=solve)
    X = si.random_state(lay, 101, amp=(1e-2, 1e-2, 1e-2), p=2) + ora.conductive_state()
    J = si.default_phase_slot(lay, X)
    C = 0.3
    plan.set_base(_dev(X), C, J)
    ora.set_base(X, C, J)
    V = si.random_vectors(lay, [1001, 1002, 1003, 1004])
    vd = _dev(V)
    yd = torch.empty_like(vd)
    plan.jvp(vd, yd, prec)
    Y = _host(yd)
    for i in range(len(V)):
        check(lay, Y[i], ora.jvp(V[i]), tol, btol, f"cfg={cfg} prec={prec} solve={solve} vec {i}")


# N = 52: every block spans four 16-row tiles (the largest chain-solve shape, 16 waves per
# boundary-walk workgroup); at L = 24 the chains hold 2-4 segments, so the boundary walks take
# several steps
FOUR_TILES = (24, 24, 4, 52, 1e-3, 78.0, 200.0)


@pytest.mark.parametrize("prec,solve,tol,btol", [(0, 0, 1e-12, FP64_BLOCK), (1, 1, 1e-6, 1e-5), (1, 2, 1e-6, 1e-5)],
                         ids=["fp64", "mixed-fp64solve", "mixed-fp32solve-refined"])
def test_jvp_four_row_tiles(lib, prec, solve, tol, btol):
    """17 vectors in one call (a full vector group and a one-column one) at N = 52; sampled
    actions of both groups, and one of them applied alone, against the oracle."""
    plan, ora, lay = _setup(lib, FOUR_TILES, nvec=17, mixed_solve=solve)
    X = si.random_state(lay, 111, amp=(1e-2, 1e-2, 1e-2), p=2) + ora.conductive_state()
    J = si.default_phase_slot(lay, X)
    plan.set_base(_dev(X), 0.3, J)
    ora.set_base(X, 0.3, J)
    V = si.random_vectors(lay, range(1201, 1218))
    vd = _dev(V)
    yd = torch.empty_like(vd)
    plan.jvp(vd, yd, prec)
    Y = _host(yd)
    for i in (0, 9, 16):
        ref = ora.jvp(V[i])
        check(lay, Y[i], ref, tol, btol, f"N=52 prec={prec} solve={solve} vec {i}")
        if i == 9:    # one vector per call: the vector-unit walks at four row tiles
            y1 = torch.empty_like(vd[i])
            plan.jvp(vd[i].contiguous(), y1, prec)
            check(lay, _host(y1), ref, tol, btol, f"N=52 prec={prec} solve={solve} single vec {i}")


@pytest.mark.parametrize("cfg", SMALL)
@pytest.mark.parametrize("prec,solve,tol,btol", [(0, 0, 1e-12, FP64_BLOCK), (1, 1, 1e-6, 1e-5), (1, 2, 1e-6, 1e-5)],
                         ids=["fp64", "mixed-fp64solve", "mixed-fp32solve-refined"])
def test_single_vector_jvp(lib, cfg, prec, solve, tol, btol):
    """One vector per call takes the one-right-hand-side chain solve (vector-unit walks and
    output): each action matches the oracle, and the same vectors in one batched call (the
    matrix-core walks) give the same actions up to rounding."""
    plan, ora, lay = _setup(lib, cfg, mixed_solve=solve)
    X = si.random_state(lay, 101, amp=(1e-2, 1e-2, 1e-2), p=2) + ora.conductive_state()
    J = si.default_phase_slot(lay, X)
    plan.set_base(_dev(X), 0.3, J)
    ora.set_base(X, 0.3, J)
    V = si.random_vectors(lay, [1101, 1102, 1103])
    vd = _dev(V)
    yb = torch.empty_like(vd)
    plan.jvp(vd, yb, prec)
    Yb = _host(yb)
    for i in range(len(V)):
        y1 = torch.empty_like(vd[i])
        plan.jvp(vd[i].contiguous(), y1, prec)
        Y1 = _host(y1)
        check(lay, Y1, ora.jvp(V[i]), tol, btol, f"cfg={cfg} prec={prec} solve={solve} single vec {i}")
        d = float(np.abs(Y1 - Yb[i]).max() / np.abs(Yb[i]).max())
        print(f"cfg={cfg} prec={prec} solve={solve} vec {i}: one-vector vs batched max rel {d:.2e}", flush=True)
        assert d <= 2 * tol    # both are within tol of the oracle


@pytest.mark.parametrize("cfg", SMALL)
def test_autotune_then_jvp(lib, cfg):
    """sc_autotune times every ring and analysis candidate of the shell and keeps the fastest;
    the Jacobian actions with the chosen kernels still match the oracle in both precisions."""
    plan, ora, lay = _setup(lib, cfg)
    rep = plan.autotune(nvec=4, reps=2)
    print(f"cfg={cfg} autotune {rep}", flush=True)
    assert rep["candidates"] >= 2 and rep["ms_fp32"] > 0 and rep["ms_fp64"] > 0
    assert rep["ring_fp32"] >= -3 and rep["ring_fp64"] >= -2 and rep["anal_folded"] in (0, 1)
    X = si.random_state(lay, 101, amp=(1e-2, 1e-2, 1e-2), p=2) + ora.conductive_state()
    J = si.default_phase_slot(lay, X)
    plan.set_base(_dev(X), 0.3, J)
    ora.set_base(X, 0.3, J)
    V = si.random_vectors(lay, [1001, 1002, 1003, 1004])
    vd = _dev(V)
    for prec, tol, btol in ((0, 1e-12, FP64_BLOCK), (1, 1e-6, 1e-5)):
        yd = torch.empty_like(vd)
        plan.jvp(vd, yd, prec)
        Y = _host(yd)
        for i in range(len(V)):
            check(lay, Y[i], ora.jvp(V[i]), tol, btol, f"cfg={cfg} tuned prec={prec} vec {i}")
    with pytest.raises(lib.ShellConvError) as ei:
        plan.autotune(nvec=0)
    assert ei.value.code == 1


@pytest.mark.parametrize("cfg", SMALL)
def test_every_kernel_candidate_matches_the_oracle(lib, cfg):
    """Each ring kernel (the register-transform kernel in each workgroup shape where the grid has
    one, the LDS kernel at every 2^k rings per workgroup) in both precisions, with each analysis
    kernel, forced with sc_set_kernels: every Jacobian action of a batch of 6 vectors matches the
    oracle; unavailable choices are refused."""
    plan, ora, lay = _setup(lib, cfg, nvec=6)
    X = si.random_state(lay, 101, amp=(1e-2, 1e-2, 1e-2), p=2) + ora.conductive_state()
    J = si.default_phase_slot(lay, X)
    plan.set_base(_dev(X), 0.3, J)
    ora.set_base(X, 0.3, J)
    V = si.random_vectors(lay, [1001, 1002, 1003, 1004, 1005, 1006])
    vd = _dev(V)
    refs = [ora.jvp(V[i]) for i in range(len(V))]
    default = plan.kernels()
    d32, d64, df = default["ring_fp32"], default["ring_fp64"], default["anal_folded"]

    def available(args):
        before = plan.kernels()
        try:
            plan.set_kernels(*args)
            return True
        except lib.ShellConvError as e:
            assert e.code == 1 and plan.kernels() == before      # a refused choice changes nothing
            return False

    c32 = [c for c in range(-5, 6) if available((c, d64, df))]
    c64 = [c for c in range(-5, 6) if available((d32, c, df))]
    folds = [f for f in (0, 1) if available((d32, d64, f))]
    print(f"cfg={cfg} default {default}, ring candidates fp32 {c32} fp64 {c64}, analysis {folds}", flush=True)
    assert 0 in c32 and 0 in c64 and len(c32) >= 3 and len(c64) >= 2 and 0 in folds
    # register kernels: three shapes in FP32, two in FP64, where the grid has one
    assert [c for c in c32 if c < 0] in ([], [-3, -2, -1]) and [c for c in c64 if c < 0] in ([], [-2, -1])
    ran = 0
    for f in folds:
        for prec, cands, tol, btol in ((1, c32, 1e-6, 1e-5), (0, c64, 1e-12, FP64_BLOCK)):
            for c in cands:
                args = (c, d64, f) if prec == 1 else (d32, c, f)
                plan.set_kernels(*args)
                assert plan.kernels() == dict(zip(("ring_fp32", "ring_fp64", "anal_folded"), args))
                yd = torch.empty_like(vd)
                plan.jvp(vd, yd, prec)
                Y = _host(yd)
                for i in range(len(V)):
                    check(lay, Y[i], refs[i], tol, btol, f"cfg={cfg} kernels={args} prec={prec} vec {i}")
                ran += 1
    print(f"cfg={cfg} {ran} forced (kernel, precision) combinations match the oracle", flush=True)
    with pytest.raises(lib.ShellConvError):
        plan.set_kernels(99, 0, 0)
    with pytest.raises(lib.ShellConvError):
        plan.set_kernels(0, 0, 2)


def test_state_errors(lib):
    plan, ora, lay = _setup(lib, SMALL[1])
    v = torch.zeros((1, plan.n_real), dtype=torch.float64, device="cuda")
    with pytest.raises(lib.ShellConvError) as ei:
        plan.jvp(v, v.clone(), 0)
    assert ei.value.code == 2
    with pytest.raises(lib.ShellConvError) as ei:
        plan.set_base(v[0], 0.0, 2)   # an Re slot
    assert ei.value.code == 1


# the tiny shell: L = M = 16, m0 = 1, N = 16, Ek = 1e-3, Pr = 1, Ra = 1.2 x 6.5 Ek^(-1/3) = 78
C1 = (16, 16, 1, 16, 1e-3, 78.0)


@pytest.mark.parametrize("dt", [1e-4, 200.0])
def test_c1_step_and_ten_jvps(lib, dt):
    """The tiny shell's state (conductive state plus a seeded perturbation of amplitude 1e-3,
    coefficients decaying as (l+1)^-2): one IMEX step and ten Jacobian actions (vectors
    1001..1010) at the small timestep 1e-4 and at the Newton pseudo-timestep 200."""
    L, M, m0, N, Ek, Ra = C1
    plan, ora, lay = _setup(lib, (L, M, m0, N, Ek, Ra, dt), nvec=10)
    X = si.random_state(lay, 101, amp=(1e-3, 1e-3, 1e-3), p=2) + ora.conductive_state()
    xd = _dev(X)
    out = torch.empty_like(xd)
    plan.step(xd, 0.0, out)
    check(lay, _host(out), ora.step(X, 0.0), 1e-12, FP64_BLOCK, f"C1 dt={dt} step")
    J = si.default_phase_slot(lay, X)
    plan.set_base(xd, 0.0, J)
    ora.set_base(X, 0.0, J)
    V = si.random_vectors(lay, range(1001, 1011))
    vd = _dev(V)
    for prec, tol, btol in ((0, 1e-12, FP64_BLOCK), (1, 1e-6, 1e-5)):
        yd = torch.empty_like(vd)
        plan.jvp(vd, yd, prec)
        Y = _host(yd)
        for i in range(len(V)):
            check(lay, Y[i], ora.jvp(V[i]), tol, btol, f"C1 dt={dt} prec={prec} vec {1001 + i}")


@pytest.mark.parametrize("cfg", SMALL)
def test_jvp_of_the_drift_unknown_alone(lib, cfg):
    """v = c e_J (only the phase slot set): the action is the c im M X column of Sec. 3.4,
    which is far smaller than the rest of a jvp and would hide in a mixed vector."""
    plan, ora, lay = _setup(lib, cfg)
    X = si.random_state(lay, 101, amp=(1e-1, 1e-1, 1e-1), p=2) + ora.conductive_state()
    J = si.default_phase_slot(lay, X)
    plan.set_base(_dev(X), 0.3, J)
    ora.set_base(X, 0.3, J)
    v = np.zeros((1, plan.n_real))
    v[0, J] = 0.7
    ref = ora.jvp(v[0])
    vd = _dev(v)
    for prec, tol, btol in ((0, 1e-12, FP64_BLOCK), (1, 1e-6, 1e-5)):
        yd = torch.empty_like(vd)
        plan.jvp(vd, yd, prec)
        check(lay, _host(yd)[0], ref, tol, btol, f"cfg={cfg} drift column prec={prec}")
