"""Spherical-harmonic synthesis and analysis by direct sums (oracle; test infrastructure only).

Real-field convention: g(theta, phi) = sum_{m >= 0} sum_l Re[g_lm Y_l^m], with Y_l^m as in
eq:Ylm_norm and m restricted to multiples of m0 (the azimuthal sector of Sec. 3.1).
Coefficient arrays are lists indexed by the m-index k, each of shape [l - m, ...].
Grid arrays have shape [theta, phi, ...].

Horizontal vectors use surface potentials (S, Tor):
   V_theta = d_theta S + (1/sin th) d_phi Tor,   V_phi = (1/sin th) d_phi S - d_theta Tor.

Synthesis: A_m(theta) = sum_l g_lm Pbar_lm(cos theta), g = sum_m Re[A_m e^{i m phi}].
Analysis:  A_m = (2 - delta_m0)/N_phi sum_k g(phi_k) e^{-i m phi_k}   (direct DFT),
           g_lm = sum_j w_j A_m(theta_j) Pbar_lm(theta_j) / (2 (2 - delta_m0)),
both exact for band-limited data given the Gauss quadrature (Sec. 3.1: SHTns with FFTW,
here replaced by plain sums).
"""
from __future__ import annotations

import numpy as np

from .grids import Grid


def _dft_matrices(g: Grid):
    """E_syn[k_phi, km] = e^{i m phi}, E_ana[km, k_phi] = (2-delta)/N_phi e^{-i m phi}."""
    ms = np.array(g.ms, dtype=float)
    ph = g.phi
    Esyn = np.exp(1j * np.outer(ph, ms))
    fac = np.where(ms == 0, 1.0, 2.0) / g.nphi
    Eana = fac[:, None] * np.exp(-1j * np.outer(ms, ph))
    return Esyn, Eana


def fourier_synth(g: Grid, Am):
    """[k][theta, ...] complex -> grid [theta, phi, ...] real: sum_m Re[A_m e^{i m phi}]."""
    Esyn, _ = _dft_matrices(g)
    A = np.stack(Am, axis=0)                      # [k, theta, ...]
    out = np.tensordot(Esyn, A, axes=([1], [0]))  # [phi, theta, ...]
    return np.moveaxis(out.real, 0, 1)


def fourier_anal(g: Grid, G):
    """grid [theta, phi, ...] real -> list over k of [theta, ...] complex."""
    _, Eana = _dft_matrices(g)
    out = np.tensordot(Eana, np.moveaxis(G, 1, 0), axes=([1], [0]))   # [k, theta, ...]
    return [out[k] for k in range(len(g.ms))]


def scalar_synth(g: Grid, c):
    Am = [np.tensordot(g.P[m].T, c[k], axes=([1], [0])) for k, m in enumerate(g.ms)]
    return fourier_synth(g, Am)


def vector_synth(g: Grid, S, T):
    """(S, Tor) coefficients -> (V_theta, V_phi) on the grid.  T may be None (gradient)."""
    Ath, Aph = [], []
    for k, m in enumerate(g.ms):
        dP, mPs = g.dP[m].T, g.mPs[m].T          # [theta, l]
        th = np.tensordot(dP, S[k], axes=([1], [0]))
        ph = 1j * np.tensordot(mPs, S[k], axes=([1], [0]))
        if T is not None:
            th = th + 1j * np.tensordot(mPs, T[k], axes=([1], [0]))
            ph = ph - np.tensordot(dP, T[k], axes=([1], [0]))
        Ath.append(th)
        Aph.append(ph)
    return fourier_synth(g, Ath), fourier_synth(g, Aph)


def scalar_anal(g: Grid, G):
    A = fourier_anal(g, G)
    out = []
    for k, m in enumerate(g.ms):
        wP = g.P[m] * g.wt[None, :]              # [l, theta]
        out.append(np.tensordot(wP, A[k], axes=([1], [0])) / (2.0 * (2.0 - (m == 0))))
    return out


def vector_anal(g: Grid, Vth, Vph):
    """(V_theta, V_phi) on the grid -> (S, Tor) coefficients (l = 0 entries set to 0)."""
    Ath, Aph = fourier_anal(g, Vth), fourier_anal(g, Vph)
    S, T = [], []
    for k, m in enumerate(g.ms):
        ls = np.arange(m, g.L + 1)
        lam = ls * (ls + 1.0)
        inv = np.where(lam > 0, 1.0 / np.where(lam > 0, lam, 1.0), 0.0) / (2.0 * (2.0 - (m == 0)))
        wdP = g.dP[m] * g.wt[None, :]
        wmPs = g.mPs[m] * g.wt[None, :]
        s = (np.tensordot(wdP, Ath[k], axes=([1], [0]))
             - 1j * np.tensordot(wmPs, Aph[k], axes=([1], [0])))
        t = (-1j * np.tensordot(wmPs, Ath[k], axes=([1], [0]))
             - np.tensordot(wdP, Aph[k], axes=([1], [0])))
        shape = (len(ls),) + (1,) * (s.ndim - 1)
        S.append(s * inv.reshape(shape))
        T.append(t * inv.reshape(shape))
    return S, T
