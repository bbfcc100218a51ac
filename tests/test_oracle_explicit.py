"""Pins of the oracle's explicit-Coriolis variant (Sec. 3.1: eq:expcor_e / eq:expcor_f with the
force of eq:defineFexp; the implicit form is Sec. 3.2).  CPU only.

Both variants discretize the same equations; they differ in where the Coriolis force is
evaluated: in the implicit operator K (kappa-coupled spectral form at the N nodes) or with the
explicit forces (-2 e_z x U on the grid, projected through the N_p dealiasing nodes).  So the
right-hand side of the continuous-time system, G(X) = K X + N(X) + C im M X, recovered from the
preconditioned residual as (M - dt K) R / dt on the interior rows, agrees between the variants to
the spectral accuracy of the radial grid; and the explicit residual is, like the implicit one,
exactly quadratic in (X, C), so central differences reproduce its Jacobian action for any step.
"""
import numpy as np
import pytest

import seeded_inputs as si
from oracle import physics
from oracle.operators import chain_matvec
from oracle.solver import Problem
from test_oracle_drift_mass_rw import _smooth_potentials


def continuous_rhs(p, X, C):
    """(M - dt K) R(X) / dt with the boundary rows zeroed: K X + N(X) + C im M X."""
    g, ops = p.g, p.ops
    e, f, T = physics.unpack(g, p.residual(X, C))
    oe, of, oT = [np.zeros_like(a) for a in e], [np.zeros_like(a) for a in f], [np.zeros_like(a) for a in T]
    for k, m in enumerate(g.ms):
        for cls in (0, 1):
            types, Dg, Lo, Up = ops.chain_blocks(m, cls)
            if not types:
                continue
            x = np.stack([(e if t == "e" else f)[k][l - m] for t, l in types])[:, :, None]
            y = chain_matvec(Dg, Lo, Up, x)[:, :, 0]
            for i, (t, l) in enumerate(types):
                y[i, ops.bc_rows(t)] = 0
                (oe if t == "e" else of)[k][l - m] = y[i]
        for i, l in enumerate(range(m, g.L + 1)):
            y = ops.A_T(l) @ T[k][i]
            y[[0, g.N - 1]] = 0
            oT[k][i] = y
    return physics.pack(g, oe, of, oT) / p.dt


def _mismatch(N, planted=False):
    L, m0 = 10, 2
    pi = Problem(L, L, m0, N, Ek=1e-3, Ra=78.0, Pr=1.0, dt=1.0)
    pe = Problem(L, L, m0, N, Ek=1e-3, Ra=78.0, Pr=1.0, dt=1.0, coriolis="explicit")
    if planted:
        # a copy of the explicit variant that forgets the Coriolis force in the explicit terms
        pe.coriolis = "none"
    e, f, T = _smooth_potentials(pi.g, 7)
    X = 0.1 * physics.pack(pi.g, e, f, T) + pi.conductive_state()
    gi, ge = continuous_rhs(pi, X, 0.3), continuous_rhs(pe, X, 0.3)
    return np.linalg.norm(gi - ge) / np.linalg.norm(gi)


def test_explicit_and_implicit_coriolis_discretize_the_same_equations():
    e12, e20, e32 = (_mismatch(N) for N in (12, 20, 32))
    assert e20 < 1e-3 * e12 and e32 < 1e-3 * e20 and e32 <= 1e-10, (e12, e20, e32)


def test_explicit_pin_sees_a_missing_coriolis_force():
    assert _mismatch(20, planted=True) > 1e-2


@pytest.mark.parametrize("m0", [1, 4])
def test_explicit_central_difference_equals_jvp(m0):
    """R of the explicit variant is quadratic in (X, C) too (the Coriolis force is linear), so
    the central difference equals the Jacobian action for every step size."""
    L, N = 12, 14
    p = Problem(L, L, m0, N, Ek=1e-3, Ra=78.0, Pr=1.0, dt=200.0, coriolis="explicit")
    lay = si.Layout(L, L, m0, N)
    X = p.clean(si.random_state(lay, 101, amp=(1e-2, 1e-2, 1e-2), p=2) + p.conductive_state())
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


def test_explicit_operator_is_block_diagonal():
    """No kappa couplings and no 2im terms remain in the explicit variant's implicit operator."""
    p = Problem(10, 10, 2, 12, Ek=1e-3, Ra=78.0, Pr=1.0, dt=200.0, coriolis="explicit")
    for m in (0, 2, 6):
        for cls in (0, 1):
            types, Dg, Lo, Up = p.ops.chain_blocks(m, cls)
            assert all(np.abs(b).max() == 0.0 for b in Lo[1:] + Up[:-1])
            assert all(np.abs(b.imag).max() == 0.0 for b in Dg)
