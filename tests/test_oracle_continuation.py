"""Pins of the oracle's continuation (Sec. 3.5, 3.6, 4.2) and grid refinement (Sec. 4.2). CPU only.

* Quadratic Lagrange prediction (eq:lagrange) is exact on a branch quadratic in the parameter,
  and its weights sum to one.
* The turning-point switch (eq:tp_detection_Ra): on a saddle-node, (mu - mu0) = sinh(x - x0)^2,
  continuation in mu goes around the fold and returns along the other branch; with the switch
  disabled every prediction leaves the branch past the fold and Newton fails.
* Refinement by zero padding (Sec. 4.2) reproduces polynomial radial profiles exactly on the
  new nodes, keeps every coarse coefficient, and a round trip fine -> coarse of a padded state
  is the identity; the tail ratios see under-resolution in either direction.
"""
import numpy as np

import seeded_inputs as si
from oracle import physics
from oracle.continuation import Continuation, lagrange_weights, step_factor
from oracle.grids import Grid, gl_nodes
from oracle.resolution import interpolate, tail_ratios


def test_lagrange_prediction_is_exact_on_quadratics():
    rng = np.random.default_rng(3)
    A, B, Cq = rng.standard_normal((3, 7))
    U = lambda p: A + B * p + Cq * p * p
    ps = [80.0, 83.5, 85.0]
    p_new = 88.2
    w = lagrange_weights(p_new, ps)
    assert abs(sum(w) - 1.0) < 1e-14
    assert abs(sum(wq * pq for wq, pq in zip(w, ps)) - p_new) < 1e-12
    pred = sum(wq * U(pq) for wq, pq in zip(w, ps))
    assert np.abs(pred - U(p_new)).max() < 1e-10 * np.abs(U(p_new)).max()
    assert step_factor(5, 5) == 1.0 and step_factor(4, 9) < 1.0 < step_factor(6, 2)


def _fold_problem(mu0=10.0, x0=3.0):
    """A saddle-node at (mu0, x0): (mu - mu0) = sinh(x - x0)^2, branches x = x0 +- asinh(sqrt(mu - mu0));
    states X = (x, 2x); Newton at fixed mu (at most 8 iterations, like a capped Newton solve)."""
    F = lambda x, mu: (mu - mu0) - np.sinh(x - x0) ** 2

    def solve(mu, X, C):
        x = X[0]
        for it in range(1, 9):
            dF = -np.sinh(2 * (x - x0))
            if dF == 0.0 or not np.isfinite(x):
                break
            x = x - F(x, mu) / dF
            if abs(F(x, mu)) < 1e-13:
                return np.array([x, 2 * x]), C, it, True
        return X, C, 8, False
    return solve


def _branch_point(mu, upper=True):
    x = 3.0 + (1 if upper else -1) * np.arcsinh(np.sqrt(mu - 10.0))
    return np.array([x, 2 * x])


def test_continuation_goes_around_a_fold():
    c = Continuation(_fold_problem(), n_opt=4, gamma=10.0)
    for mu in (11.0, 10.8):
        c.add_point(mu, _branch_point(mu), 0.0, 4)
    for _ in range(40):
        p, ok, _ = c.step()
        assert ok, p
        if c.states[-1][0] < 3.0 and c.params[-1] > 10.5:
            break
    xs = np.array([X[0] for X in c.states])
    mus = np.array(c.params)
    assert np.allclose((mus - 10.0) - np.sinh(xs - 3.0) ** 2, 0.0, atol=1e-11)
    assert xs[-1] < 3.0 and mus[-1] > 10.5, (mus, xs)       # on the other branch, moving away
    assert any(c.state_mode) and min(mus) > 10.0            # it switched, and never left the branch


def test_continuation_without_the_switch_fails_at_the_fold():
    c = Continuation(_fold_problem(), n_opt=4, gamma=1e30)
    for mu in (11.0, 10.8):
        c.add_point(mu, _branch_point(mu), 0.0, 4)
    for _ in range(40):
        p, ok, _ = c.step()
        if not ok:
            break
    assert not ok and p < 10.0            # every retry predicts past the fold: no root there


# ---------------------------------------------------------------- refinement
def _poly_state(g, seed, deg_r):
    """e, f, T per (l, m): polynomials of degree deg_r in x, real at m = 0."""
    rng = np.random.default_rng(seed)
    x = g.rad.x
    out = []
    for _ in range(3):
        lst = []
        for m in g.ms:
            nl = g.L - m + 1
            c = rng.standard_normal((nl, deg_r + 1)) + 1j * rng.standard_normal((nl, deg_r + 1))
            if m == 0:
                c = c.real + 0j
            lst.append(np.stack([np.polynomial.polynomial.polyval(x, ci) for ci in c]))
        out.append(lst)
    return out


def test_refinement_is_exact_and_keeps_the_coarse_modes():
    gc = Grid(10, 10, 2, 12)
    gf = Grid(12, 12, 2, 15)
    e, f, T = _poly_state(gc, 1, 11)
    Xc = physics.pack(gc, e, f, T)
    Xf = interpolate(gc, Xc, gf)
    ef, ff, Tf = physics.unpack(gf, Xf)
    xf = gl_nodes(gf.N)
    rng = np.random.default_rng(1)
    for flds, fine in (((e, f, T)[0], ef), ((e, f, T)[1], ff), ((e, f, T)[2], Tf)):
        for k, m in enumerate(gc.ms):
            n = gc.L - m + 1
            # the coarse profiles are degree-11 polynomials: exact on the new nodes
            ref = np.stack([np.polynomial.polynomial.polyval(xf, np.polynomial.polynomial.polyfit(gc.rad.x, p.real, 11))
                            + 1j * np.polynomial.polynomial.polyval(xf, np.polynomial.polynomial.polyfit(gc.rad.x, p.imag, 11))
                            for p in flds[k]])
            assert np.abs(fine[gf.ms.index(m)][:n] - ref).max() < 1e-11 * np.abs(ref).max()
            assert np.abs(fine[gf.ms.index(m)][n:]).max(initial=0.0) == 0.0          # new degrees are zero
        for kf, m in enumerate(gf.ms):
            if m not in gc.ms:
                assert np.abs(fine[kf]).max() == 0.0                                 # new orders are zero
    # back to the coarse grid: the identity
    assert np.abs(interpolate(gf, Xf, gc) - Xc).max() < 1e-11 * np.abs(Xc).max()


def test_tail_ratios_see_under_resolution():
    g = Grid(12, 12, 3, 16)
    lay = si.Layout(12, 12, 3, 16)
    # seeded states decay as (l+1)^-p in degree and 10^(-6 n/(N-1)) in Chebyshev degree
    X = si.random_state(lay, 5, p=8.0)
    rc, rl = tail_ratios(g, X)
    assert 1e-8 < rc < 1e-4 and 1e-11 < rl < 1e-6, (rc, rl)
    X2 = si.random_state(lay, 5, p=1.0)
    assert tail_ratios(g, X2)[1] > 10 * rl                    # slower decay in l: larger l ratio
    X3 = si.random_state(lay, 5, p=8.0, decay_k=2.0)
    assert tail_ratios(g, X3)[0] > 10 * rc                    # slower decay in n: larger n ratio
