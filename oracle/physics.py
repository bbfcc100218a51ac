"""Potentials -> physical fields, (linearized) nonlinear terms and curl projections
(oracle; test infrastructure only).

Velocity from toroidal and poloidal potentials, U = curl(e e_r) + curl curl(f e_r) with e_r
the unit radial vector (Sec. 3.1).  For one harmonic g(r) Y_l^m, lambda = l(l+1):
   U:      U_r = lambda f/r^2,   S = f'/r,      Tor = e/r
   omega:  w_r = lambda e/r^2,   S = e'/r,      Tor = -L_l f / r,  L_l = d_rr - lambda/r^2
   grad T: d_r T,                S = T/r,       Tor = 0
(surface potentials as in sht.py).  The curl projections used by the e- and f-equations
(eq:expcor_e, eq:expcor_f):
   (e_r . curl W)_lm      = (lambda/r) Tor_lm[W_h]
   (e_r . curl curl W)_lm = (lambda/r^2) (W_r,lm - d_r (r S_lm[W_h]))
Forcing: the momentum equation (eq:Navier-Stokes) has the advection on the left, so the
explicit force is -Ek (U.grad)U - grad P + Ra T r/r_o; -Ek (U.grad)U differs from
W = Ek U x omega by a gradient, which both projections remove.  Temperature:
Q = -U.grad T (eq:temp).  Linearization about (U, T) (Sec. 3.3, replacement rules):
W' = Ek (U x omega_u + u x Omega),  Q' = -(U.grad tau + u.grad T).

Radial evaluation order: spectral inputs are formed on the N_p dealiasing nodes as
diag(r_p^-k) E D^j applied to the N nodal values; after the angular analysis every
r-factor and d_r(r S) is applied on the N_p nodes, then one projection P back to N nodes.
"""
from __future__ import annotations

import numpy as np

from . import sht
from .grids import Grid


def unpack(g: Grid, v: np.ndarray):
    """Packed real vector -> (e, f, T), each a list over k of complex [l - m, N]."""
    S = sum(g.L - m + 1 for m in g.ms)
    a = v.reshape(3, S, g.N, 2)
    c = a[..., 0] + 1j * a[..., 1]
    out = []
    for fld in range(3):
        lst, o = [], 0
        for m in g.ms:
            nl = g.L - m + 1
            lst.append(c[fld, o:o + nl].copy())
            o += nl
        out.append(lst)
    return tuple(out)


def pack(g: Grid, e, f, T) -> np.ndarray:
    parts = []
    for fld in (e, f, T):
        c = np.concatenate(fld, axis=0)
        parts.append(np.stack([c.real, c.imag], axis=-1))
    return np.stack(parts).ravel()


def lam_list(g: Grid):
    return [np.arange(m, g.L + 1) * (np.arange(m, g.L + 1) + 1.0) for m in g.ms]


def spectral_inputs(g: Grid, e, f, T):
    """The eight radial profiles at the N_p nodes that the angular synthesis needs."""
    rad = g.rad
    rp = rad.rp[None, :]
    E, D = rad.E.T, rad.D.T          # right-multiplication on [l, N] rows
    out = {k: [] for k in ("ur", "Su", "Tu", "wr", "Sw", "Tw", "dT", "ST")}
    for k, lam in enumerate(lam_list(g)):
        lm = lam[:, None]
        fE = f[k] @ E
        fDE = f[k] @ D @ E
        fDDE = f[k] @ D @ D @ E
        eE = e[k] @ E
        eDE = e[k] @ D @ E
        out["ur"].append(lm * fE / rp ** 2)
        out["Su"].append(fDE / rp)
        out["Tu"].append(eE / rp)
        out["wr"].append(lm * eE / rp ** 2)
        out["Sw"].append(eDE / rp)
        out["Tw"].append(-fDDE / rp + lm * fE / rp ** 3)
        out["dT"].append(T[k] @ D @ E)
        out["ST"].append(T[k] @ E / rp)
    return out


def fields(g: Grid, spec):
    """Physical U, omega and grad T on the [theta, phi, r_p] grid."""
    Ur = sht.scalar_synth(g, spec["ur"])
    Uth, Uph = sht.vector_synth(g, spec["Su"], spec["Tu"])
    wr = sht.scalar_synth(g, spec["wr"])
    wth, wph = sht.vector_synth(g, spec["Sw"], spec["Tw"])
    Gr = sht.scalar_synth(g, spec["dT"])
    Gth, Gph = sht.vector_synth(g, spec["ST"], None)
    return {"U": (Ur, Uth, Uph), "w": (wr, wth, wph), "G": (Gr, Gth, Gph)}


def cross(a, b):
    return (a[1] * b[2] - a[2] * b[1],
            a[2] * b[0] - a[0] * b[2],
            a[0] * b[1] - a[1] * b[0])


def dot(a, b):
    return a[0] * b[0] + a[1] * b[1] + a[2] * b[2]


def nonlinear_forces(F, Ek: float):
    """W = Ek U x omega, Q = -U . grad T."""
    W = tuple(Ek * c for c in cross(F["U"], F["w"]))
    Q = -dot(F["U"], F["G"])
    return W, Q


def linearized_forces(Fb, Fu, Ek: float):
    """W' = Ek (U x omega_u + u x Omega), Q' = -(U . grad tau + u . grad T)."""
    c1 = cross(Fb["U"], Fu["w"])
    c2 = cross(Fu["U"], Fb["w"])
    W = tuple(Ek * (a + b) for a, b in zip(c1, c2))
    Q = -(dot(Fb["U"], Fu["G"]) + dot(Fu["U"], Fb["G"]))
    return W, Q


def project(g: Grid, W, Q):
    """Angular analysis of (W, Q), then the curl projections; returns the explicit
    right-hand sides (N_e, N_f, N_T) at the N nodes (buoyancy not included)."""
    rad = g.rad
    rp = rad.rp[None, :]
    Wr = sht.scalar_anal(g, W[0])
    S, Tor = sht.vector_anal(g, W[1], W[2])
    Ql = sht.scalar_anal(g, Q)
    Ne, Nf, NT = [], [], []
    P = rad.P.T
    Dp = rad.Dp.T
    for k, lam in enumerate(lam_list(g)):
        lm = lam[:, None]
        # analysis returns [l, r_p]
        Ne.append(((lm / rp) * Tor[k]) @ P)
        Nf.append(((lm / rp ** 2) * (Wr[k] - (rp * S[k]) @ Dp)) @ P)
        NT.append(Ql[k] @ P)
    return Ne, Nf, NT


def coriolis_force(g: Grid, F):
    """-2 e_z x U on the [theta, phi, r_p] grid (used only by the Coriolis pins)."""
    ct = g.ct[:, None, None]
    st = g.st[:, None, None]
    Ur, Uth, Uph = F["U"]
    ezxU = (-st * Uph, -ct * Uph, ct * Uth + st * Ur)
    return tuple(-2.0 * c for c in ezxU)
