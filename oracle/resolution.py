"""Resolution checks and grid refinement of a packed state (oracle; test infrastructure only).

Sec. 4.2 (continuation in Ekman number and resolution): the spectral resolution grows by 20 %
whenever the ratio between the amplitude of the highest-wavenumber mode and that of the mode of
largest amplitude exceeds a threshold (1e-6) in the Chebyshev or in the spherical-harmonic modes;
the fields are then carried to the new grid by filling the new modes with zero (Fourier
interpolation, exact for the represented functions).

Readings: the Chebyshev ratio is max |a_{N-1}| / max |a_n| over every radial profile of every
field (a_n the Chebyshev coefficients of the nodal profile); the spherical-harmonic ratio is
max |X at l = L| / max |X| over every field, m and node; a ratio above the threshold means
under-resolution (the printed wording is inverted, but only this sense refines when the tail
grows).  New degrees l and new orders m are zero; each radial profile is its interpolating
polynomial evaluated at the new Gauss-Lobatto nodes (its Chebyshev series padded with zeros).
"""
from __future__ import annotations

import numpy as np

from . import physics
from .grids import Grid, cheb_eval, gl_nodes, nodal_to_cheb


def tail_ratios(g: Grid, X):
    """(Chebyshev ratio, spherical-harmonic ratio) of the packed state X."""
    e, f, T = physics.unpack(g, X)
    Cm = nodal_to_cheb(g.N)
    amax = acheb = 0.0
    xmax = xl = 0.0
    for fld in (e, f, T):
        for k, m in enumerate(g.ms):
            a = fld[k] @ Cm.T                       # [l - m, n]
            amax = max(amax, np.abs(a).max(initial=0.0))
            acheb = max(acheb, np.abs(a[:, -1]).max(initial=0.0))
            xmax = max(xmax, np.abs(fld[k]).max(initial=0.0))
            if m <= g.L:
                xl = max(xl, np.abs(fld[k][g.L - m]).max(initial=0.0))
    return acheb / amax, xl / xmax


def interpolate(g_from: Grid, X, g_to: Grid):
    """X on g_from carried to g_to (same m0; L, M, N may grow or shrink)."""
    if g_from.m0 != g_to.m0:
        raise ValueError("the sector (m0) must not change")
    e, f, T = physics.unpack(g_from, X)
    V = cheb_eval(g_from.N, gl_nodes(g_to.N)) @ nodal_to_cheb(g_from.N)     # [N_to, N_from]
    out = []
    for fld in (e, f, T):
        lst = []
        for m in g_to.ms:
            z = np.zeros((g_to.L - m + 1, g_to.N), dtype=complex)
            if m in g_from.ms:
                k = g_from.ms.index(m)
                n = min(g_from.L, g_to.L) - m + 1
                if n > 0:
                    z[:n] = fld[k][:n] @ V.T
            lst.append(z)
        out.append(lst)
    return physics.pack(g_to, *out)
