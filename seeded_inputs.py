"""Seeded synthetic inputs for the rotating-shell Jacobian-vector product.

This module only draws random numbers and packs them into the canonical state
layout; it holds none of the method's arithmetic (no transforms, no operators).
Both the oracle and the GPU library read what it produces.

Canonical packed layout (real float64, Re/Im interleaved):
    for field F in (e, f, T)            -- toroidal, poloidal potential, temperature
      for k in 0..K, m = k*m0, K = M // m0
        for l in m..L
          for j in 0..N-1               -- Gauss-Lobatto node x_j = cos(pi j/(N-1)); j=0 is r_out
            (Re, Im)
n_real = 2 * 3 * N * S,  S = sum_k (L - k*m0 + 1).

Radial profiles are drawn in Chebyshev space and evaluated at the nodes:
    value(x_j) = bubble(x_j) * sum_{k < N-b} c_k T_k(x_j),   T_k(x_j) = cos(pi k j/(N-1)),
with bubble = 1-x^2 (e, T: b=2) or (1-x^2)^2 (f: b=4), so the homogeneous
boundary conditions of the potentials hold exactly; c_k are complex Gaussian
(real for m = 0), scaled by amp * (l+1)^-p * 10^(-6k/(N-1)).
"""
from __future__ import annotations

import numpy as np

FIELDS = ("e", "f", "T")


class Layout:
    """Index arithmetic of the packed state (the ABI contract)."""

    def __init__(self, L: int, M: int, m0: int, N: int):
        if L < 1 or m0 < 1 or M < 0 or N < 6:
            raise ValueError("bad truncation")
        self.L, self.M, self.m0, self.N = L, M, m0, N
        self.K = min(M, L) // m0
        self.ms = [k * m0 for k in range(self.K + 1)]
        self.nl = [L - m + 1 for m in self.ms]
        self.lm_base = np.concatenate([[0], np.cumsum(self.nl)[:-1]]).astype(int)
        self.S = int(sum(self.nl))
        self.n_real = 2 * 3 * N * self.S

    def offset(self, field: int, k: int, l: int, j: int = 0) -> int:
        """Index of Re part of coefficient (field, m=k*m0, l) at node j."""
        m = self.ms[k]
        assert m <= l <= self.L
        lm = int(self.lm_base[k]) + (l - m)
        return 2 * (self.N * (field * self.S + lm) + j)

    def nonphysical_mask(self) -> np.ndarray:
        """Slots that carry no physical content: e, f at l=0 and Im parts at m=0."""
        mask = np.zeros(self.n_real, dtype=bool)
        for fld in range(3):
            for l in range(self.L + 1):
                o = self.offset(fld, 0, l)
                mask[o + 1:o + 2 * self.N:2] = True          # Im at m = 0
                if l == 0 and fld < 2:
                    mask[o:o + 2 * self.N] = True            # e_00, f_00
        return mask


def _profiles(rng, N, nprof, bubble_pow, nmodes, decay_k, real):
    """nprof radial profiles at the N Gauss-Lobatto nodes (complex)."""
    j = np.arange(N)
    x = np.cos(np.pi * j / (N - 1))
    k = np.arange(nmodes)
    Tk = np.cos(np.pi * np.outer(j, k) / (N - 1))           # T_k(x_j)
    scale = 10.0 ** (-decay_k * k / (N - 1))
    c = rng.standard_normal((nprof, nmodes))
    if not real:
        c = c + 1j * rng.standard_normal((nprof, nmodes))
    c = c * scale
    bub = (1.0 - x * x) ** bubble_pow
    return (c @ Tk.T) * bub


def random_state(lay: Layout, seed: int, amp=(1.0, 1.0, 1.0), p: float = 2.0,
                 decay_k: float = 6.0, t_offset=None) -> np.ndarray:
    """Packed random state; amp gives the (e, f, T) amplitudes.

    t_offset: optional callable r -> value added to T at l=m=0 (the caller
    passes the closed-form conductive profile when a physical base is wanted).
    """
    rng = np.random.default_rng(seed)
    out = np.zeros(lay.n_real)
    N = lay.N
    for fld, (bpow, nb) in enumerate(((1, 2), (2, 4), (1, 2))):
        for k, m in enumerate(lay.ms):
            ls = np.arange(m, lay.L + 1)
            prof = _profiles(rng, N, len(ls), bpow, N - nb, decay_k, real=(m == 0))
            prof *= (amp[fld] * (ls + 1.0) ** (-p))[:, None]
            for i, l in enumerate(ls):
                if l == 0 and fld < 2:
                    continue
                o = lay.offset(fld, k, l)
                out[o:o + 2 * N:2] = prof[i].real
                out[o + 1:o + 2 * N:2] = prof[i].imag
    if t_offset is not None:
        x = np.cos(np.pi * np.arange(N) / (N - 1))
        o = lay.offset(2, 0, 0)
        out[o:o + 2 * N:2] += t_offset(x)
    return out


def random_vectors(lay: Layout, seeds, p: float = 1.0) -> np.ndarray:
    """Unit-norm random Krylov-like vectors, one row per seed (zero on non-physical slots)."""
    mask = lay.nonphysical_mask()
    rows = []
    for s in seeds:
        v = random_state(lay, s, amp=(1.0, 1.0, 1.0), p=p)
        v[mask] = 0.0
        rows.append(v / np.linalg.norm(v))
    return np.stack(rows)


def default_phase_slot(lay: Layout, X: np.ndarray) -> int:
    """Phase slot J: Im entry of the m=m0 coefficient whose real part is largest in |.|
    over the f and T fields (the caller may pass any Im slot with m > 0)."""
    if lay.K < 1:
        raise ValueError("phase slot needs m0 <= M")
    best, bestv = -1, -1.0
    for fld in (1, 2):
        for l in range(lay.ms[1], lay.L + 1):
            o = lay.offset(fld, 1, l)
            re = np.abs(X[o:o + 2 * lay.N:2])
            j = int(np.argmax(re))
            if re[j] > bestv:
                bestv, best = re[j], o + 2 * j + 1
    return best
