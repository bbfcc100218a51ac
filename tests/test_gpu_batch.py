"""Ragged batch of problems (sc_batch_jvp, one stream branch per plan): every call must reproduce
the eager per-plan jvp of the same kernels, also with eager work between calls and after a change
of base state."""
import numpy as np
import pytest

import seeded_inputs as si

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

# (L, M, m0, N, Ek, Ra, seed) -- uneven truncations and parameters
SHELLS = [(12, 12, 4, 14, 1e-3, 78.0, 401), (16, 16, 1, 16, 1e-3, 60.0, 402), (20, 20, 3, 20, 3e-4, 100.0, 403)]


@pytest.fixture(scope="module")
def sc():
    import paper_2508_16635_amd as m
    m.load_library()
    return m


def _setup(sc, nvecs):
    plans, vs, bases = [], [], []
    for (L, M, m0, N, Ek, Ra, seed), nv in zip(SHELLS, nvecs):
        print(f"plan L={L} M={M} m0={m0} N={N} nvec={nv}", flush=True)
        p = sc.Plan(L, M, m0, N, Ek=Ek, Ra=Ra, Pr=1.0, dt=200.0, nvec_max=max(nv, 1))
        p.factor()
        lay = si.Layout(L, M, m0, N)
        X = si.random_state(lay, seed, amp=(0.5, 0.5, 0.1), p=2.0)
        J = si.default_phase_slot(lay, X)
        p.set_base(torch.from_numpy(X).cuda(), 0.3, J)
        plans.append(p)
        bases.append((lay, X, J))
        vs.append(torch.from_numpy(si.random_vectors(lay, range(seed * 10, seed * 10 + nv))).cuda() if nv else None)
    torch.cuda.synchronize()
    return plans, vs, bases


def _eager(plans, vs, prec):
    out = []
    for i, (p, v) in enumerate(zip(plans, vs)):
        if v is None:
            out.append(None)
            continue
        print(f"eager jvp plan {i} prec {prec}", flush=True)
        y = torch.empty_like(v)
        p.jvp(v, y, prec)
        out.append(y)
    torch.cuda.synchronize()
    return [None if y is None else y.cpu().numpy() for y in out]


@pytest.mark.parametrize("prec", [0, 1], ids=["fp64", "mixed"])
def test_batch_matches_eager(sc, prec):
    nvecs = [3, 1, 2]
    plans, vs, bases = _setup(sc, nvecs)
    ref = _eager(plans, vs, prec)
    ys = [torch.full_like(v, float("nan")) for v in vs]
    print("batch create", flush=True)
    b = sc.Batch(plans)
    for rep in range(3):
        for y in ys:
            y.fill_(float("nan"))
        print(f"batch jvp call {rep}", flush=True)
        b.jvp(vs, ys, prec)
        torch.cuda.synchronize()
        for i, (y, r) in enumerate(zip(ys, ref)):
            err = float(np.max(np.abs(y.cpu().numpy() - r)) / np.max(np.abs(r)))
            print(f"call {rep} plan {i}: max rel diff {err:.2e}", flush=True)
            assert err <= 1e-14
        _ = _eager(plans[:1], vs[:1], 1 - prec)
    lay, X, J = bases[1]
    plans[1].set_base(torch.from_numpy(0.5 * X).cuda(), 0.1, J)
    ref2 = _eager(plans, vs, prec)
    b.jvp(vs, ys, prec)
    torch.cuda.synchronize()
    for y, r in zip(ys, ref2):
        assert float(np.max(np.abs(y.cpu().numpy() - r)) / np.max(np.abs(r))) <= 1e-14
    b.close()


def test_batch_errors(sc):
    plans, vs, _ = _setup(sc, [1, 1, 0])
    with pytest.raises(sc.ShellConvError) as ei:
        sc.Batch([plans[0], plans[0]])
    assert ei.value.code == 1
    b = sc.Batch(plans)
    ys = [None if v is None else torch.empty_like(v) for v in vs]
    plans[0].profile(True)
    with pytest.raises(sc.ShellConvError) as ei:
        b.jvp(vs, ys, 1)
    assert ei.value.code == 2
    plans[0].profile(False)
    b.jvp(vs, ys, 1)
    torch.cuda.synchronize()
    b.close()
