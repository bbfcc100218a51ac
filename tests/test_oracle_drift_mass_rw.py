"""Pins of the oracle's drift term, mass operator and converged rotating wave (CPU only).

* The drift term C im M X of the co-rotating step (Sec. 3.4, eq:twdefine and the augmented
  step after it) is what a rotation of the pattern by C dt does to one step: B_C(X) and
  B_0(rot(X, C dt)) agree to O(dt^2), while a wrong sign or a missing M leaves O(dt).
* M (the operator under the time derivative, eq:expcor_e / eq:expcor_f) is the pair of curl
  projections of Ek u: projecting the synthesized velocity itself gives M_e e / Ek and
  M_f f / Ek, to the spectral accuracy of the radial grid.
* The m0 = 4 rotating wave RW4 of the tiny shell (tests/golden/rw4_L16_m4_N16.npz, written by
  tests/golden/make_rw4.py from the oracle): a root of R_C at any dt, m0-fold symmetric, and
  in the laboratory frame the plain step (C = 0) rotates it rigidly, with a first-order error
  in dt (the IMEX Euler step of eq:discrete).
"""
import os

import numpy as np
import pytest

import seeded_inputs as si
from oracle import physics
from oracle.solver import Problem

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "rw4_L16_m4_N16.npz")


def rot(g, v, phi0):
    """Pattern rotation: every g_lm multiplied by exp(i m phi0) (the field moves by -phi0)."""
    e, f, T = physics.unpack(g, v)
    r = lambda a: [a[k] * np.exp(1j * m * phi0) for k, m in enumerate(g.ms)]
    return physics.pack(g, r(e), r(f), r(T))


# ---------------------------------------------------------------- drift term
def _drift_errors(C, dts, planted=None):
    L, N, m0 = 12, 14, 2
    lay = si.Layout(L, L, m0, N)
    out = []
    for dt in dts:
        p = Problem(L, L, m0, N, Ek=1e-3, Ra=78.0, Pr=1.0, dt=dt)
        X = p.clean(si.random_state(lay, 101, amp=(1e-1, 1e-1, 1e-1), p=2) + p.conductive_state())
        B = p.step(X, C)
        if planted == "no_M":
            # the drift term written as C im X instead of C im M X: add (M - dt K)^-1 dt C im (X - M X)
            e, f, T = physics.unpack(p.g, X)
            Me, Mf, MT = p.M_apply(e, f, T)
            im = [1j * m for m in p.g.ms]
            be = [dt * C * im[k] * (e[k] - Me[k]) for k in range(len(im))]
            bf = [dt * C * im[k] * (f[k] - Mf[k]) for k in range(len(im))]
            bT = [dt * C * im[k] * (T[k] - MT[k]) for k in range(len(im))]
            p._set_bc(be, bf, bT, inhomogeneous=False)
            xe, xf, xT = p.solve(be, bf, bT)
            p._zero_nonphysical(xe, xf, xT)
            B = B + physics.pack(p.g, xe, xf, xT)
        sgn = -1.0 if planted == "sign" else 1.0
        out.append(np.linalg.norm(B - p.step(rot(p.g, X, sgn * C * dt), 0.0)))
    return np.array(out)


def test_drift_term_is_a_rotation_of_the_step():
    """||B_C(X) - B_0(rot(X, C dt))|| = O(dt^2): observed order 2 between dt = 2e-4 and 5e-5."""
    e = _drift_errors(2.0, (2e-4, 1e-4, 5e-5))
    order = np.log2(e[:-1] / e[1:])
    assert np.all(order > 1.8) and np.all(order < 2.3), order


@pytest.mark.parametrize("planted", ["sign", "no_M"])
def test_drift_pin_sees_planted_mistakes(planted):
    """A flipped sign, or C im X in place of C im M X (both planted here, in a copy of the
    oracle's step), leave an O(dt) mismatch: the pin above would fail on them."""
    e = _drift_errors(2.0, (2e-4, 1e-4, 5e-5), planted)
    order = np.log2(e[:-1] / e[1:])
    assert np.all(order < 1.3), order


# ---------------------------------------------------------------- mass operator
def _smooth_potentials(g, seed):
    """e = (1-x^2) c exp(a x), f = (1-x^2)^2 c' exp(a' x) per (l, m): analytic, independent of N,
    with the velocity boundary conditions (e = f = f' = 0 at both walls)."""
    rng = np.random.default_rng(seed)
    x = g.rad.x
    e, f, T = [], [], []
    for m in g.ms:
        nl = g.L - m + 1
        ce = rng.standard_normal((nl, 2)) @ np.array([1, 1j])
        cf = rng.standard_normal((nl, 2)) @ np.array([1, 1j])
        ae, af = rng.uniform(-1, 1, nl), rng.uniform(-1, 1, nl)
        if m == 0:
            ce, cf = ce.real + 0j, cf.real + 0j
        e.append(ce[:, None] * (1 - x * x) * np.exp(ae[:, None] * x))
        f.append(cf[:, None] * (1 - x * x) ** 2 * np.exp(af[:, None] * x))
        T.append(np.zeros((nl, g.N), complex))
    if g.ms[0] == 0:
        e[0][0] = 0
        f[0][0] = 0
    return e, f, T


def _mass_mismatch(N):
    L, m0 = 10, 2
    p = Problem(L, L, m0, N, Ek=1e-3, Ra=0.0, Pr=1.0, dt=1.0)
    e, f, T = _smooth_potentials(p.g, 5)
    F = physics.fields(p.g, physics.spectral_inputs(p.g, e, f, T))
    Ne, Nf, _ = physics.project(p.g, F["U"], 0 * F["U"][0])
    Me, Mf, _ = p.M_apply(e, f, T)
    se = max(np.abs(a).max() for a in Me) / p.Ek
    sf = max(np.abs(a).max() for a in Mf) / p.Ek
    ee = max(np.abs(Ne[k] - Me[k] / p.Ek).max() for k in range(len(Me))) / se
    ef = max(np.abs(Nf[k] - Mf[k] / p.Ek).max() for k in range(len(Mf))) / sf
    return ee, ef


def test_mass_operator_is_the_curl_projection_of_the_velocity():
    """(e_r . curl u)_lm = lambda e/r^2 = M_e e / Ek and (e_r . curl curl u)_lm = -lambda/r^2 L_l f
    = M_f f / Ek, with u synthesized from (e, f) and projected like any force: the projection
    passes 1/r factors through the dealiasing nodes, so the agreement is spectral in N."""
    errs = [_mass_mismatch(N) for N in (12, 20, 32)]
    (e12, f12), (e20, f20), (e32, f32) = errs
    assert e20 < 1e-3 * e12 and e32 < 1e-3 * e20 and e32 <= 1e-13, errs
    assert f20 < 1e-3 * f12 and f32 < 1e-3 * f20 and f32 <= 1e-12, errs


# ---------------------------------------------------------------- converged rotating wave (RW4)
@pytest.fixture(scope="module")
def rw4():
    d = np.load(GOLDEN, allow_pickle=False)
    L, M, m0, N = (int(v) for v in d["shell"])
    Ek, Pr, Ra = (float(v) for v in d["params"])
    return dict(X=d["X"], C=float(d["C"]), J=int(d["J"]), L=L, M=M, m0=m0, N=N, Ek=Ek, Pr=Pr, Ra=Ra)


def _prob(w, dt, m0=None):
    return Problem(w["L"], w["M"], w["m0"] if m0 is None else m0, w["N"], Ek=w["Ek"], Ra=w["Ra"], Pr=w["Pr"], dt=dt)


def test_rw4_is_a_root_at_any_dt(rw4):
    """R_C(X*) = 0 (eq:finalrhs: B - I = P(dt) A, whose roots do not depend on dt); a prograde
    drift at Ra = 78 (the drift changes from prograde to retrograde as Ra grows, Sec. 2.2)."""
    X, C = rw4["X"], rw4["C"]
    assert np.linalg.norm(_prob(rw4, 200.0).residual(X, C)) <= 1e-10
    p = _prob(rw4, 1e-3)
    R = p.residual(X, C)
    assert np.linalg.norm(R) <= 1e-12 * np.linalg.norm(X)
    # not the conductive state: the wave carries most of its energy in m = 4
    e, f, T = physics.unpack(p.g, X)
    assert np.abs(f[1]).max() > 0.1 * np.abs(f[0][1:]).max()
    assert C > 0


def test_rw4_is_m0_fold_symmetric(rw4):
    """Embedded in the full domain (m0 = 1), X* is still a root and the harmonics m not
    divisible by 4 stay zero under the step (to the rounding of the azimuthal transforms)."""
    ps = _prob(rw4, 200.0)
    pf = _prob(rw4, 200.0, m0=1)
    L, N = rw4["L"], rw4["N"]
    es, fs, Ts = physics.unpack(ps.g, rw4["X"])
    z = lambda m: np.zeros((L - m + 1, N), dtype=complex)
    ef, ff, Tf = [z(m) for m in pf.g.ms], [z(m) for m in pf.g.ms], [z(m) for m in pf.g.ms]
    for k, m in enumerate(ps.g.ms):
        ef[m], ff[m], Tf[m] = es[k], fs[k], Ts[k]
    Xf = physics.pack(pf.g, ef, ff, Tf)
    Rf = pf.residual(Xf, rw4["C"])
    assert np.linalg.norm(Rf) <= 1e-10
    Y = pf.step(Xf, rw4["C"])
    re, rf, rT = physics.unpack(pf.g, Y)
    for m in pf.g.ms:
        if m % 4:
            for a in (re, rf, rT):
                assert np.abs(a[m]).max() <= 1e-14 * np.abs(Y).max()


def test_rw4_rotates_rigidly_in_the_lab_frame(rw4):
    """With C = 0 the step integrates the laboratory frame: after time tau the state is
    rot(X*, -C* tau) up to the error of the first-order step, which halves with dt."""
    X, C = rw4["X"], rw4["C"]
    tau = 0.05
    errs = []
    for n in (20, 40, 80):
        dt = tau / n
        p = _prob(rw4, dt)
        Y = X.copy()
        for _ in range(n):
            Y = p.step(Y, 0.0)
        errs.append(np.linalg.norm(Y - rot(p.g, X, -C * tau)) / np.linalg.norm(X))
    errs = np.array(errs)
    order = np.log2(errs[:-1] / errs[1:])
    assert np.all(order > 0.85) and np.all(order < 1.2), (errs, order)
    assert errs[-1] < 0.05
    # the rotation is what the step does: the unrotated state is much further away
    assert np.linalg.norm(Y - X) / np.linalg.norm(X) > 10 * errs[-1]
