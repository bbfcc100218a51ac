"""Pins of the oracle's grids, tables and transforms against textbook facts and library
routines (CPU only)."""
import math

import numpy as np
import pytest
from scipy.special import lpmv

from oracle import sht
from oracle.grids import Grid, Radial, default_grid_sizes, legendre_tables, norm_factor, shell_radii
from oracle.operators import kappa, kappa_from_paper


def test_grid_size_rules():
    # dealiasing rules; sizes of the four standard shells
    assert default_grid_sizes(16, 16, 1, 16) == (24, 26, 50)
    assert default_grid_sizes(64, 64, 6, 32) == (48, 98, 32)
    assert default_grid_sizes(128, 128, 10, 48) == (72, 194, 40)
    assert default_grid_sizes(255, 255, 12, 64) == (96, 384, 64)
    ri, ro = shell_radii(0.35)
    assert abs(ri - 7 / 13) < 1e-15 and abs(ro - 20 / 13) < 1e-15


def test_legendre_vs_scipy():
    """P3: Pbar_l^m = N_l^m P_l^m without the Condon-Shortley phase (scipy includes it)."""
    L = 40
    x = np.linspace(-0.97, 0.97, 23)
    ms = list(range(0, L + 1))
    P, dP, mPs = legendre_tables(L, ms, x)
    for m in ms:
        for l in range(m, L + 1):
            ref = (-1) ** m * lpmv(m, l, x) * norm_factor(l, m)
            scale = max(1.0, np.abs(ref).max())
            assert np.abs(P[m][l - m] - ref).max() <= 1e-12 * scale, (l, m)


def test_legendre_m0_is_legendre_polynomial():
    x = np.linspace(-1, 1, 17)[1:-1]
    P, _, _ = legendre_tables(10, [0], x)
    for l in range(11):
        c = np.zeros(l + 1)
        c[l] = 1
        assert np.allclose(P[0][l] / math.sqrt(2 * l + 1), np.polynomial.legendre.legval(x, c), atol=1e-14)
    # small-l closed forms: Pbar_1^0 = sqrt(3) cos th, Pbar_1^1 = sqrt(3) sin th
    P, _, _ = legendre_tables(2, [0, 1], x)
    assert np.allclose(P[0][1], math.sqrt(3) * x, atol=1e-15)
    assert np.allclose(P[1][0], math.sqrt(3) * np.sqrt(1 - x * x), atol=1e-15)


def test_legendre_theta_derivative_vs_finite_difference():
    L = 24
    th = np.linspace(0.2, 2.9, 11)
    h = 1e-5
    ms = [0, 1, 5, 12, 24]
    _, dP, mPs = legendre_tables(L, ms, np.cos(th))
    Pp, _, _ = legendre_tables(L, ms, np.cos(th + h))
    Pm, _, _ = legendre_tables(L, ms, np.cos(th - h))
    for m in ms:
        fd = (Pp[m] - Pm[m]) / (2 * h)
        assert np.abs(fd - dP[m]).max() < 1e-7 * max(1, np.abs(dP[m]).max())


def test_unsold_and_gram():
    """P1: addition theorem sum_m Pbar_l^m(x)^2 = 2l+1; Gauss-quadrature Gram matrix."""
    g = Grid(20, 20, 1, 8)
    for l in range(g.L + 1):
        s = sum(g.P[m][l - m] ** 2 for m in g.ms if m <= l)
        assert np.abs(s - (2 * l + 1)).max() < 1e-12 * (2 * l + 1)
    for m in g.ms:
        G = (g.P[m] * g.wt) @ g.P[m].T
        assert np.abs(G - 2 * (2 - (m == 0)) * np.eye(len(G))).max() < 1e-12


def _rand_coeffs(g, rng, shape_tail):
    out = []
    for m in g.ms:
        nl = g.L - m + 1
        c = rng.standard_normal((nl,) + shape_tail) + 1j * rng.standard_normal((nl,) + shape_tail)
        if m == 0:
            c = c.real + 0j
        out.append(c)
    return out


@pytest.mark.parametrize("L,m0", [(12, 1), (16, 4), (20, 3)])
def test_sht_roundtrip(L, m0):
    """P1: analysis o synthesis = identity on band-limited data (scalar and vector)."""
    g = Grid(L, L, m0, 8)
    rng = np.random.default_rng(1)
    c = _rand_coeffs(g, rng, (3,))
    back = sht.scalar_anal(g, sht.scalar_synth(g, c))
    for a, b in zip(c, back):
        assert np.abs(a - b).max() < 1e-12
    S = _rand_coeffs(g, rng, (3,))
    T = _rand_coeffs(g, rng, (3,))
    if g.ms[0] == 0:
        S[0][0] = 0
        T[0][0] = 0
    S2, T2 = sht.vector_anal(g, *sht.vector_synth(g, S, T))
    for a, b in zip(S + T, S2 + T2):
        assert np.abs(a - b).max() < 1e-12


def test_parseval():
    """Real-field convention: int g^2 dOmega = 4 pi sum |g_lm|^2."""
    g = Grid(10, 10, 1, 8)
    rng = np.random.default_rng(2)
    c = _rand_coeffs(g, rng, ())
    G = sht.scalar_synth(g, c)
    integral = (g.wt[:, None] * G ** 2).sum() * (2 * np.pi / g.nphi)
    assert abs(integral - 4 * np.pi * sum((abs(a) ** 2).sum() for a in c)) < 1e-11 * integral


def test_fourier_vs_numpy_fft():
    """P2: the direct DFT equals numpy's FFT; round trip on harmonics <= K."""
    g = Grid(8, 8, 2, 8)
    rng = np.random.default_rng(3)
    G = rng.standard_normal((g.nth, g.nphi))
    A = sht.fourier_anal(g, G)
    F = np.fft.rfft(G, axis=1) / g.nphi
    for k, m in enumerate(g.ms):
        assert np.abs(A[k] - (1 if m == 0 else 2) * F[:, k]).max() < 1e-14
    B = sht.fourier_synth(g, [A[k] for k in range(len(g.ms))])
    Fk = F.copy()
    Fk[:, g.K + 1:] = 0
    Gb = np.fft.irfft(Fk, n=g.nphi, axis=1) * g.nphi
    assert np.abs(B - Gb).max() < 1e-13


def test_radial_matrices():
    """Chebyshev collocation: exact on polynomials of degree N-1; P E = I; D vs monomials."""
    rad = Radial(12, 18, 7 / 13, 20 / 13)
    for deg in range(12):
        p = rad.r ** deg
        dp = deg * rad.r ** (deg - 1) if deg else 0 * rad.r
        assert np.abs(rad.D @ p - dp).max() < 1e-10 * max(1, np.abs(dp).max())
        assert np.abs(rad.E @ p - rad.rp ** deg).max() < 1e-12 * max(1, (rad.rp ** deg).max())
    assert np.abs(rad.P @ rad.E - np.eye(12)).max() < 1e-13
    # the N_p-node projection keeps the first N Chebyshev modes: exact for degree <= N-1
    q = rad.rp ** 7
    assert np.abs(rad.P @ q - rad.r ** 7).max() < 1e-12


def test_kappa_equals_printed_coefficients():
    """The compact kappa_l equals both printed neighbour coefficients of eq:impcor_e_final."""
    for m in range(0, 30):
        for l in range(max(m, 1), 60):
            assert abs(kappa(l, m) - kappa_from_paper(l, m, "lower")) < 1e-12 * max(1, kappa(l, m))
            assert abs(kappa(l + 1, m) - kappa_from_paper(l, m, "upper")) < 1e-12 * max(1, kappa(l + 1, m))


def test_gauss_legendre_moments_to_rounding():
    """Gauss quadrature with n nodes integrates x^(2k) exactly for 2k <= 2n - 1; the highest
    moments live next to the poles, so they fix the weights of the polar nodes (where the weights
    numpy's leggauss returns are off by up to 3e-11)."""
    from oracle.grids import gauss_legendre
    for n in (26, 98, 194):
        x, w, st = gauss_legendre(n)
        assert np.abs(st * st + x * x - 1).max() < 5e-16
        for k in (0, n // 2, n - 1):
            exact = 2.0 / (2 * k + 1)
            assert abs((w * x ** (2 * k)).sum() - exact) <= 1e-14 * exact, (n, k)
