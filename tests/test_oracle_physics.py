"""Pins of the oracle's physics: conductive state, Coriolis form, projections, solve,
exactness of the linearization, symmetries, manufactured Newton (CPU only)."""
import numpy as np
import pytest

import seeded_inputs as si
from oracle import physics, sht
from oracle.grids import Grid, gl_nodes, nodal_to_cheb, cheb_eval
from oracle.operators import Operators, ChainSolver, chain_dense, kappa
from oracle.solver import Problem, newton


def small_problem(m0=1, dt=200.0, L=12, N=14, Ek=1e-3, Ra=78.0):
    return Problem(L, L, m0, N, Ek=Ek, Ra=Ra, Pr=1.0, dt=dt)


def base_state(p, seed=101, amp=1e-2):
    lay = si.Layout(p.g.L, p.g.M, p.g.m0, p.g.N)
    return p.clean(si.random_state(lay, seed, amp=(amp, amp, amp), p=2) + p.conductive_state())


# ---------------------------------------------------------------- P4 conductive state
@pytest.mark.parametrize("dt", [1e-4, 200.0])
def test_conductive_state_is_fixed_point(dt):
    p = small_problem(dt=dt, N=16)
    Xc = p.conductive_state()
    R = p.residual(Xc)
    assert np.linalg.norm(R) <= 1e-13 * np.linalg.norm(Xc)


@pytest.mark.parametrize("N,tol", [(16, 3e-9), (32, 1e-13)])
def test_conductive_state_matches_closed_form(N, tol):
    """T_cond = r_o r_i / r - r_i (Sec. 2.1) to the spectral accuracy of N nodes."""
    p = small_problem(N=N)
    Xc = p.conductive_state()
    _, _, T = physics.unpack(p.g, Xc)
    r = p.g.rad.r
    Tc = p.g.ro * p.g.ri / r - p.g.ri
    assert np.abs(T[0][0].real - Tc).max() < tol


# ---------------------------------------------------------------- P5 jvp at the conductive state
def test_jvp_at_conductive_state_is_spectral():
    """At U = 0, T = T_c(r): W' = 0 and Q' = -u_r dT_c/dr, a product with a radial function
    only, so the transform path must equal a formula with no angular transforms."""
    p = small_problem(m0=2, L=10, N=12)
    Xc = p.conductive_state()
    p.set_base(Xc, 0.0, -1)
    lay = si.Layout(p.g.L, p.g.M, p.g.m0, p.g.N)
    v = si.random_vectors(lay, [7])[0]
    y = p.jvp(v)
    g = p.g
    e, f, T = physics.unpack(g, p.clean(v))
    _, _, Tb = physics.unpack(g, Xc)
    dTc = (g.rad.E @ (g.rad.D @ Tb[0][0]))                    # on N_p nodes
    rp = g.rad.rp
    NT = []
    for k, lam in enumerate(physics.lam_list(g)):
        ur = lam[:, None] * (f[k] @ g.rad.E.T) / rp ** 2
        NT.append((-ur * dTc[None, :]) @ g.rad.P.T)
    Me, Mf, MT = p.M_apply(e, f, T)
    Bf = p.buoyancy(T)
    dt = p.dt
    be = [Me[k] for k in range(len(g.ms))]
    bf = [Mf[k] + dt * Bf[k] for k in range(len(g.ms))]
    bT = [MT[k] + dt * NT[k] for k in range(len(g.ms))]
    p._set_bc(be, bf, bT, inhomogeneous=False)
    xe, xf, xT = p.solve(be, bf, bT)
    p._zero_nonphysical(xe, xf, xT)
    y_ref = physics.pack(g, xe, xf, xT) - v
    assert np.linalg.norm(y - y_ref) <= 1e-12 * np.linalg.norm(y_ref)


# ---------------------------------------------------------------- P6 Coriolis forms
def _coriolis_spectral_e(g, e, f):
    """Row e of the implicit Coriolis operator, evaluated at the N_p nodes."""
    rad = g.rad
    rp = rad.rp
    out = []
    for k, m in enumerate(g.ms):
        ls = np.arange(m, g.L + 1)
        eE = e[k] @ rad.E.T
        fE = f[k] @ rad.E.T
        fDE = f[k] @ rad.D.T @ rad.E.T
        res = 2j * m * eE / rp ** 2
        for i, l in enumerate(ls):
            if i > 0:
                res[i] -= 2 / rp ** 2 * kappa(l, m) * (l / rp * fE[i - 1] - fDE[i - 1])
            if i < len(ls) - 1:
                res[i] -= 2 / rp ** 2 * kappa(l + 1, m) * (-(l + 1) / rp * fE[i + 1] - fDE[i + 1])
        out.append(res)
    return out


def _coriolis_spectral_f(g, e, f):
    rad = g.rad
    rp = rad.rp
    out = []
    for k, m in enumerate(g.ms):
        ls = np.arange(m, g.L + 1)
        lam = ls * (ls + 1.0)
        eE = e[k] @ rad.E.T
        eDE = e[k] @ rad.D.T @ rad.E.T
        LfE = f[k] @ rad.D.T @ rad.D.T @ rad.E.T - lam[:, None] * (f[k] @ rad.E.T) / rp ** 2
        res = -2j * m * LfE / rp ** 2
        for i, l in enumerate(ls):
            if i > 0:
                res[i] -= 2 / rp ** 2 * kappa(l, m) * (l / rp * eE[i - 1] - eDE[i - 1])
            if i < len(ls) - 1:
                res[i] -= 2 / rp ** 2 * kappa(l + 1, m) * (-(l + 1) / rp * eE[i + 1] - eDE[i + 1])
        out.append(res)
    return out


def _coriolis_mismatch(m0, N):
    g = Grid(14, 14, m0, N)
    lay = si.Layout(g.L, g.M, g.m0, g.N)
    v = si.random_state(lay, 11, p=1)
    p = Problem(g.L, g.M, g.m0, g.N, 1e-3, 0.0, 1.0, 1.0)
    e, f, T = physics.unpack(g, p.clean(v))
    F = physics.fields(g, physics.spectral_inputs(g, e, f, T))
    W = physics.coriolis_force(g, F)
    S, Tor = sht.vector_anal(g, W[1], W[2])
    Wr = sht.scalar_anal(g, W[0])
    rp = g.rad.rp
    ce = _coriolis_spectral_e(g, e, f)
    cf = _coriolis_spectral_f(g, e, f)
    scale_e = max(np.abs(a).max() for a in ce)
    scale_f = max(np.abs(a).max() for a in cf)
    err_e = err_f = 0.0
    for k, lam in enumerate(physics.lam_list(g)):
        pe = lam[:, None] / rp * Tor[k]
        err_e = max(err_e, np.abs(pe - ce[k]).max() / scale_e)
        pf = lam[:, None] / rp ** 2 * (Wr[k] - (rp * S[k]) @ g.rad.Dp.T)
        err_f = max(err_f, np.abs(pf - cf[k]).max() / scale_f)
    return err_e, err_f


@pytest.mark.parametrize("m0", [1, 3])
def test_coriolis_pseudospectral_equals_implicit_form(m0):
    """P6: -2 e_z x U computed on the grid and projected equals the kappa-coupled spectral
    operator of eq:impcor_e_final / eq:impcor_f_final.  e-row: pointwise in r (no radial
    derivative of analysed data), so to rounding; f-row: the projection differentiates
    r S(r), which carries 1/r factors, on the N_p nodes, so it agrees to radial truncation
    level and converges spectrally as N grows."""
    e16, f16 = _coriolis_mismatch(m0, 16)
    e24, f24 = _coriolis_mismatch(m0, 24)
    assert e16 <= 1e-12 and e24 <= 1e-12
    assert f16 <= 3e-8
    assert f24 <= 1e-10 and f24 <= 1e-2 * f16


# ---------------------------------------------------------------- P7 skew-adjointness
def test_coriolis_is_skew_adjoint():
    """P7: Coriolis does no work: Re sum_lm int r^2 [conj(e) C_e + conj(f) C_f] dr = 0 for
    fields with e = f = f' = 0 at both walls.  Fields are polynomials of degree d with
    2d <= N-1, so after the r^2 weight every term whose real part does not vanish pointwise
    is a polynomial that Clenshaw-Curtis quadrature on the N nodes integrates exactly."""
    L, N, d = 10, 20, 9
    g = Grid(L, L, 1, N)
    ops = Operators(g, 1e-3, 1.0, 1.0)
    x = g.rad.x
    rng = np.random.default_rng(5)

    def rnd(bub, deg):
        c = rng.standard_normal(deg + 1) + 1j * rng.standard_normal(deg + 1)
        return bub * np.polynomial.polynomial.polyval(x, c)

    e = [np.stack([rnd(1 - x * x, d - 2) for _ in range(m, L + 1)]) for m in g.ms]
    f = [np.stack([rnd((1 - x * x) ** 2, d - 4) for _ in range(m, L + 1)]) for m in g.ms]
    e[0][0] = 0
    f[0][0] = 0
    k = np.arange(N)
    intT = np.where(k % 2 == 0, 2.0 / (1 - k ** 2 + (k % 2 == 1)), 0.0)
    w = (intT @ nodal_to_cheb(N)) / 2 * g.rad.r ** 2             # CC weights in r, times r^2
    total, ref = 0.0, 0.0
    for kk, m in enumerate(g.ms):
        ls = np.arange(m, L + 1)
        for i, l in enumerate(ls):
            visc = np.diag(ops.Ek * l * (l + 1) / g.rad.r ** 2) @ ops.Lop(l)
            Ce = (ops.K_e_self(l, m) - visc) @ e[kk][i]
            Cf = (ops.K_f_self(l, m) + visc @ ops.Lop(l)) @ f[kk][i]
            if i > 0:
                Ce = Ce + ops.K_couple(l, m, -1) @ f[kk][i - 1]
                Cf = Cf + ops.K_couple(l, m, -1) @ e[kk][i - 1]
            if i < len(ls) - 1:
                Ce = Ce + ops.K_couple(l, m, +1) @ f[kk][i + 1]
                Cf = Cf + ops.K_couple(l, m, +1) @ e[kk][i + 1]
            term = np.conj(e[kk][i]) * Ce + np.conj(f[kk][i]) * Cf
            total += (w * term).sum().real
            ref += (np.abs(w) * np.abs(term)).sum()
    assert abs(total) < 1e-12 * ref
    # and a wrong sign on one coupling breaks it (the pin is sensitive)
    assert ref > 0


# ---------------------------------------------------------------- P11 gradients project to 0
def test_gradient_force_projects_to_zero():
    g = Grid(10, 10, 2, 12)
    rng = np.random.default_rng(4)
    rp = g.rad.rp
    # a smooth potential phi_lm(r) given on the N_p nodes as polynomials of degree < N_p
    phi = []
    for m in g.ms:
        nl = g.L - m + 1
        c = rng.standard_normal((nl, 6)) + 1j * rng.standard_normal((nl, 6))
        if m == 0:
            c = c.real + 0j
        phi.append(np.stack([np.polynomial.polynomial.polyval(rp, ci) for ci in c]))
    dphi = [a @ g.rad.Dp.T for a in phi]
    Wr = sht.scalar_synth(g, dphi)
    Wt, Wp = sht.vector_synth(g, [a / rp for a in phi], None)
    Ne, Nf, NT = physics.project(g, (Wr, Wt, Wp), 0 * Wr)
    scale = max(np.abs(a).max() for a in phi)
    for a, b in zip(Ne, Nf):
        assert np.abs(a).max() < 1e-10 * scale
        assert np.abs(b).max() < 1e-9 * scale


# ---------------------------------------------------------------- P8 chain solve vs dense
@pytest.mark.parametrize("m,cls", [(0, 0), (0, 1), (3, 0), (5, 1)])
def test_chain_solve_vs_dense(m, cls):
    g = Grid(16, 16, 1, 14)
    ops = Operators(g, 1e-4, 1.0, 200.0)
    types, Dg, Lo, Up = ops.chain_blocks(m, cls)
    A = chain_dense(Dg, Lo, Up)
    rng = np.random.default_rng(m * 10 + cls)
    x_true = rng.standard_normal((A.shape[0], 2)) + 1j * rng.standard_normal((A.shape[0], 2))
    b = A @ x_true
    sol = ChainSolver(Dg, Lo, Up, refine=2)
    x = sol.solve(b.reshape(len(Dg), g.N, 2)).reshape(-1, 2)
    # forward error bounded by the conditioning of the equilibrated system
    assert np.linalg.norm(A @ x - b) <= 1e-13 * np.linalg.norm(b)
    Ae = sol.R[:, None] * A * sol.C[None, :]
    cond = np.linalg.cond(Ae)
    assert cond < 1e6
    err = np.linalg.norm((x - x_true) / sol.C[:, None]) / np.linalg.norm(x_true / sol.C[:, None])
    assert err <= 1e-15 * cond * 100


# ---------------------------------------------------------------- P9 central FD is exact
@pytest.mark.parametrize("m0", [1, 4])
def test_central_difference_equals_jvp(m0):
    """R is quadratic in (X, C), so the central difference is exact for every eps."""
    p = small_problem(m0=m0)
    X = base_state(p)
    lay = si.Layout(p.g.L, p.g.M, p.g.m0, p.g.N)
    J = si.default_phase_slot(lay, X)
    C = 0.37
    p.set_base(X, C, J)
    v = si.random_vectors(lay, [21])[0]
    y = p.jvp(v)
    u = p.clean(v)
    c = u[J]
    u[J] = 0
    for eps in (1e-3, 1.0, 1e3):
        fd = (p.residual(X + eps * u, C + eps * c) - p.residual(X - eps * u, C - eps * c)) / (2 * eps)
        assert np.linalg.norm(fd - y) <= 1e-11 * np.linalg.norm(y), eps


def test_jvp_nonphysical_slots():
    p = small_problem(m0=1, L=6, N=10)
    X = base_state(p)
    p.set_base(X, 0.0, -1)
    lay = si.Layout(6, 6, 1, 10)
    v = si.random_state(lay, 3)
    y = p.jvp(v)
    assert np.array_equal(y[p.mask], -v[p.mask])


# ---------------------------------------------------------------- P10 symmetries
def _rotate(g, v, phi0):
    e, f, T = physics.unpack(g, v)
    rot = lambda a: [a[k] * np.exp(1j * m * phi0) for k, m in enumerate(g.ms)]
    return physics.pack(g, rot(e), rot(f), rot(T))


def test_rotation_equivariance():
    p = small_problem(m0=2)
    X = base_state(p)
    phi0 = 0.7
    R1 = _rotate(p.g, p.residual(X, 0.2), phi0)
    R2 = p.residual(_rotate(p.g, X, phi0), 0.2)
    assert np.linalg.norm(R1 - R2) <= 1e-12 * np.linalg.norm(R1)


def test_sector_equals_full_domain():
    """An m0-sector run equals the full-domain run on an m0-symmetric state."""
    L, N, m0 = 12, 12, 4
    ps = Problem(L, L, m0, N, 1e-3, 78.0, 1.0, 200.0)
    pf = Problem(L, L, 1, N, 1e-3, 78.0, 1.0, 200.0)
    Xs = base_state(ps)
    es, fs, Ts = physics.unpack(ps.g, Xs)
    # embed into the full-domain layout
    z = lambda m: np.zeros((L - m + 1, N), dtype=complex)
    ef, ff, Tf = [z(m) for m in pf.g.ms], [z(m) for m in pf.g.ms], [z(m) for m in pf.g.ms]
    for k, m in enumerate(ps.g.ms):
        ef[m], ff[m], Tf[m] = es[k], fs[k], Ts[k]
    Xf = physics.pack(pf.g, ef, ff, Tf)
    Rs = physics.unpack(ps.g, ps.residual(Xs, 0.1))
    Rf = physics.unpack(pf.g, pf.residual(Xf, 0.1))
    scale = np.linalg.norm(ps.residual(Xs, 0.1))
    for fld in range(3):
        for k, m in enumerate(ps.g.ms):
            assert np.abs(Rs[fld][k] - Rf[fld][m]).max() <= 1e-12 * scale
        for m in pf.g.ms:
            if m % m0:
                assert np.abs(Rf[fld][m]).max() <= 1e-14 * scale


def test_equatorial_parity_subspace():
    """States with T, f of even l-m and e of odd l-m stay in that subspace."""
    p = small_problem(m0=1, L=10, N=12)
    g = p.g
    X = base_state(p)
    e, f, T = physics.unpack(g, X)
    for k, m in enumerate(g.ms):
        par = (np.arange(m, g.L + 1) - m) % 2
        e[k][par == 0] = 0
        f[k][par == 1] = 0
        T[k][par == 1] = 0
    Xs = physics.pack(g, e, f, T)
    re, rf, rT = physics.unpack(g, p.residual(Xs, 0.0))
    scale = np.linalg.norm(p.residual(Xs, 0.0))
    for k, m in enumerate(g.ms):
        par = (np.arange(m, g.L + 1) - m) % 2
        assert np.abs(re[k][par == 0]).max(initial=0) <= 1e-13 * scale
        assert np.abs(rf[k][par == 1]).max(initial=0) <= 1e-13 * scale
        assert np.abs(rT[k][par == 1]).max(initial=0) <= 1e-13 * scale


# ---------------------------------------------------------------- P13 manufactured Newton
def test_manufactured_newton_converges():
    """X* seeded, F* = -R(X*): R_F(X) = R(X) - R(X*) has the exact root X*; Newton-GMRES
    from X* + delta must reach |R_F| <= 1e-10."""
    p = small_problem(m0=4, L=10, N=12, Ek=1e-3)
    Xs = base_state(p, amp=1e-1)
    lay = si.Layout(p.g.L, p.g.M, p.g.m0, p.g.N)
    J = si.default_phase_slot(lay, Xs)
    Cs = 0.5
    Fstar = -p.residual(Xs, Cs)
    d = p.clean(si.random_state(lay, 77, p=2))
    d[J] = 0
    X0 = Xs + 1e-3 * np.linalg.norm(Xs) * d / np.linalg.norm(d)
    X, C, hist = newton(p, X0, Cs + 1e-3, J, tol=1e-10, gmres_tol=1e-12, forcing=Fstar, max_newton=8)
    assert hist[-1] <= 1e-10, hist
    assert np.linalg.norm(X - Xs) <= 1e-8 * np.linalg.norm(Xs)
    assert abs(C - Cs) < 1e-8


# ---------------------------------------------------------------- advection sign (rigid rotation)
def _rigid_rotation_base(g, Om):
    """e_10 = Om r^2/sqrt(3) gives U = Om e_z x r (U_phi = Om r sin th), omega = 2 Om e_z."""
    e = [np.zeros((g.L - m + 1, g.N), dtype=complex) for m in g.ms]
    f = [a.copy() for a in e]
    T = [a.copy() for a in e]
    e[0][1] = Om * g.rad.r ** 2 / np.sqrt(3.0)
    return e, f, T


def test_temperature_advection_by_rigid_rotation():
    """U.grad T = Om d_phi T for rigid rotation, so Q_lm = -i m Om T_lm exactly (eq:temp)."""
    g = Grid(10, 10, 2, 12)
    Om = 0.7
    e, f, _ = _rigid_rotation_base(g, Om)
    lay = si.Layout(g.L, g.M, g.m0, g.N)
    _, _, T = physics.unpack(g, si.random_state(lay, 9, p=1))
    T[0] = T[0].real + 0j
    F = physics.fields(g, physics.spectral_inputs(g, e, f, T))
    W, Q = physics.nonlinear_forces(F, 1.0)
    _, _, NT = physics.project(g, W, Q)
    scale = max(np.abs(a).max() for a in T)
    for k, m in enumerate(g.ms):
        assert np.abs(NT[k] - (-1j * m * Om) * T[k]).max() <= 1e-12 * scale * max(1, m)


def test_linearized_momentum_advection_by_rigid_rotation():
    """With U = Om e_z x r: (U.grad)u + (u.grad)U = Om d_phi u + 2 Om e_z x u (components in
    the spherical basis), so the e-row projection of -Ek[(U.grad)u + (u.grad)U] equals
    Ek Om [-i m lambda e/r^2 + C_e(u)], with C_e the implicit-Coriolis e-row.  This fixes
    the sign of the rotational form W' = Ek (U x omega_u + u x Omega)."""
    g = Grid(12, 12, 3, 14)
    Om = 0.9
    Ek = 1.0
    eb, fb, Tb = _rigid_rotation_base(g, Om)
    Fb = physics.fields(g, physics.spectral_inputs(g, eb, fb, Tb))
    lay = si.Layout(g.L, g.M, g.m0, g.N)
    p = Problem(g.L, g.M, g.m0, g.N, Ek, 0.0, 1.0, 1.0)
    e, f, T = physics.unpack(g, p.clean(si.random_state(lay, 13, p=1)))
    Fu = physics.fields(g, physics.spectral_inputs(g, e, f, T))
    W, _ = physics.linearized_forces(Fb, Fu, Ek)
    _, Tor = sht.vector_anal(g, W[1], W[2])
    rp = g.rad.rp
    ce = _coriolis_spectral_e(g, e, f)
    scale = max(np.abs(a).max() for a in ce)
    for k, (m, lam) in enumerate(zip(g.ms, physics.lam_list(g))):
        lhs = lam[:, None] / rp * Tor[k]
        rhs = Ek * Om * (-1j * m * lam[:, None] * (e[k] @ g.rad.E.T) / rp ** 2 + ce[k])
        assert np.abs(lhs - rhs).max() <= 1e-12 * scale
