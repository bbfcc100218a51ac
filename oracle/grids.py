"""Grids and tables of the spectral discretization (oracle; test infrastructure only).

Radial: Chebyshev polynomials of x = (2r - (r_o + r_i))/(r_o - r_i) (Sec. 3.1, eq:expansion),
represented by values at the N Gauss-Lobatto nodes x_j = cos(pi j/(N-1)) (collocation).
Dealiasing in r by the 3/2 rule (Sec. 3.1): products are formed on N_p = ceil(3N/2)
Gauss-Lobatto nodes.  Angular: spherical harmonics Y_l^m = N_l^m P_l^m(cos th) e^{im phi}
with N_l^m = sqrt((2 - delta_m0)(2l+1)(l-m)!/(l+m)!) (Sec. 3.2, eq:Ylm_norm), on a
Gauss-Legendre grid in theta and an equispaced grid on the sector 0 <= phi < 2 pi/m0
(Sec. 3.1, azimuthal periodicity).

Everything here is defined from the Chebyshev coefficient representation:
a nodal vector stands for its interpolating polynomial of degree N-1.
"""
from __future__ import annotations

import functools
import math
from dataclasses import dataclass, field

import numpy as np
from numpy.polynomial import chebyshev as npcheb
from numpy.polynomial import legendre as nplegendre


def shell_radii(eta: float = 0.35):
    """r_i, r_o for a gap of 1 and radius ratio eta (Sec. 2.1: r_o = 20/13, r_i = 7/13)."""
    ro = 1.0 / (1.0 - eta)
    return ro - 1.0, ro


def gl_nodes(n: int) -> np.ndarray:
    """Chebyshev-Gauss-Lobatto nodes x_j = cos(pi j/(n-1)), j = 0 at x = 1."""
    return np.cos(np.pi * np.arange(n) / (n - 1))


def nodal_to_cheb(n: int) -> np.ndarray:
    """Matrix C with a = C v: Chebyshev coefficients of the interpolant of nodal values v.

    Discrete Chebyshev transform on Gauss-Lobatto points:
      a_k = 2/((n-1) cbar_k) * sum_j v_j T_k(x_j) / cbar_j,  cbar_0 = cbar_{n-1} = 2, else 1,
    so that p(x) = sum_k a_k T_k(x) interpolates v.
    """
    j = np.arange(n)
    cbar = np.ones(n)
    cbar[0] = cbar[-1] = 2.0
    Tkj = np.cos(np.pi * np.outer(j, j) / (n - 1))            # [k, j]
    return 2.0 / (n - 1) * Tkj / cbar[:, None] / cbar[None, :]


def cheb_eval(nmodes: int, x: np.ndarray) -> np.ndarray:
    """Matrix V[i, k] = T_k(x_i), k < nmodes."""
    return npcheb.chebvander(x, nmodes - 1)


def cheb_deriv_coeffs(n: int) -> np.ndarray:
    """Matrix Dc with a' = Dc a (coefficients of d/dx of sum a_k T_k)."""
    Dc = np.zeros((n, n))
    for k in range(n):
        e = np.zeros(n)
        e[k] = 1.0
        d = npcheb.chebder(e)
        Dc[:len(d), k] = d
    return Dc


@dataclass
class Radial:
    """Radial matrices on the N collocation nodes and the N_p dealiasing nodes."""
    N: int
    Np: int
    ri: float
    ro: float
    x: np.ndarray = field(init=False)
    r: np.ndarray = field(init=False)
    xp: np.ndarray = field(init=False)
    rp: np.ndarray = field(init=False)
    D: np.ndarray = field(init=False)      # d/dr on N nodes
    Dp: np.ndarray = field(init=False)     # d/dr on N_p nodes
    E: np.ndarray = field(init=False)      # N -> N_p evaluation of the interpolant
    P: np.ndarray = field(init=False)      # N_p -> N: truncate to N Chebyshev modes, evaluate

    def __post_init__(self):
        N, Np = self.N, self.Np
        self.x = gl_nodes(N)
        self.xp = gl_nodes(Np)
        # x = (2r - (ro+ri))/(ro-ri)  =>  r = ((ro-ri) x + ro + ri)/2, d/dr = 2/(ro-ri) d/dx
        g = self.ro - self.ri
        self.r = (g * self.x + self.ro + self.ri) / 2.0
        self.rp = (g * self.xp + self.ro + self.ri) / 2.0
        C = nodal_to_cheb(N)
        Cp = nodal_to_cheb(Np)
        self.D = (2.0 / g) * cheb_eval(N, self.x) @ cheb_deriv_coeffs(N) @ C
        self.Dp = (2.0 / g) * cheb_eval(Np, self.xp) @ cheb_deriv_coeffs(Np) @ Cp
        self.E = cheb_eval(N, self.xp) @ C
        self.P = cheb_eval(N, self.x) @ Cp[:N, :]


def smooth_235(n: int) -> int:
    """Smallest integer >= n whose prime factors are 2, 3, 5."""
    n = max(n, 1)
    while True:
        k = n
        for p in (2, 3, 5):
            while k % p == 0:
                k //= p
        if k == 1:
            return n
        n += 1


def default_grid_sizes(L: int, M: int, m0: int, N: int):
    """(N_p, N_theta, N_phi) dealiasing rules for quadratic products (Sec. 3.1):
    N_p = ceil(3N/2); N_theta = smallest even >= (3L+1)/2; N_phi = smallest 2^a3^b5^c >= 3K+1."""
    K = min(M, L) // m0
    Np = (3 * N + 1) // 2
    nth = math.ceil((3 * L + 1) / 2)
    nth += nth % 2
    nphi = smooth_235(3 * K + 1)
    return Np, nth, nphi


@functools.lru_cache(maxsize=32)
def _gauss_legendre_cached(nth: int):
    return _gauss_legendre(nth)


def gauss_legendre(nth: int):
    """Copies of the cached (nodes, weights, sin(theta)) of _gauss_legendre."""
    return tuple(a.copy() for a in _gauss_legendre_cached(nth))


def _gauss_legendre(nth: int):
    """Gauss-Legendre nodes x = cos(theta) (descending, north first), weights and sin(theta).

    numpy's leggauss gives the nodes to double precision, but its weights lose up to 3e-11 of
    relative accuracy at the nodes next to the poles (where 1 - x^2 is small), which the m = 0
    analysis feels.  So each node is polished by Newton's iteration on P_n in 40-digit arithmetic
    (three-term recurrence), and w = 2 / ((1 - x^2) P_n'(x)^2) and sin(theta) = sqrt(1 - x^2) are
    evaluated there before rounding to double."""
    import mpmath
    x0, _ = nplegendre.leggauss(nth)
    x0 = x0[::-1]
    x = np.empty(nth)
    w = np.empty(nth)
    st = np.empty(nth)
    with mpmath.workdps(40):
        def pn(z):
            p0, p1 = mpmath.mpf(1), z
            for k in range(1, nth):
                p0, p1 = p1, ((2 * k + 1) * z * p1 - k * p0) / (k + 1)
            return p1, p0                      # P_n(z), P_(n-1)(z)
        for j in range((nth + 1) // 2):        # northern half; the rest by symmetry
            z = mpmath.mpf(float(x0[j]))
            for _ in range(4):
                p, q = pn(z)
                z = z - p / (nth * (z * p - q) / (z * z - 1))
            p, q = pn(z)
            dp = nth * (z * p - q) / (z * z - 1)
            x[j], w[j], st[j] = float(z), float(2 / ((1 - z * z) * dp * dp)), float(mpmath.sqrt(1 - z * z))
            x[nth - 1 - j], w[nth - 1 - j], st[nth - 1 - j] = -x[j], w[j], st[j]
    return x, w, st


def norm_factor(l: int, m: int) -> float:
    """N_l^m of eq:Ylm_norm, with the factorial ratio (l-m)!/(l+m)! (the printed
    parenthesis is garbled; this is the standard reading)."""
    lr = math.lgamma(l - m + 1) - math.lgamma(l + m + 1)
    return math.sqrt((2.0 - (m == 0)) * (2 * l + 1) * math.exp(lr))


def legendre_tables(L: int, ms, x: np.ndarray, s: np.ndarray = None):
    """Normalized associated Legendre functions Pbar_l^m = N_l^m P_l^m(x) (no Condon-Shortley
    phase), their theta-derivative and m Pbar/sin(theta), at the nodes x = cos(theta); s is
    sin(theta) (default sqrt(1 - x^2), which loses digits next to the poles).

    Returns dicts keyed by m of arrays [l - m, j].  The recursion is the textbook one
    for sqrt((2l+1)(l-m)!/(l+m)!) P_l^m (sectoral seed, then the three-term recursion
    in l); the theta-derivative uses (1-x^2) dP_l^m/dx = -l x P_l^m + (l+m) P_{l-1}^m.
    """
    if s is None:
        s = np.sqrt(1.0 - x * x)
    P, dP, mPs = {}, {}, {}
    pmm = np.ones_like(x)                       # p_0^0
    for m in range(0, max(ms) + 1):
        if m > 0:
            pmm = math.sqrt((2 * m + 1) / (2.0 * m)) * s * pmm
        if m not in ms:
            continue
        nl = L - m + 1
        p = np.zeros((nl + 1, len(x)))          # p_l^m for l = m .. L+1 (one extra)
        p[0] = pmm
        if nl >= 1:
            p[1] = math.sqrt(2 * m + 3) * x * pmm
        for i in range(2, nl + 1):
            l = m + i
            a = math.sqrt((4.0 * l * l - 1) / (l * l - m * m))
            b = math.sqrt(((l - 1.0) ** 2 - m * m) / (4.0 * (l - 1) ** 2 - 1))
            p[i] = a * (x * p[i - 1] - b * p[i - 2])
        fac = math.sqrt(2.0 - (m == 0))
        Pm = fac * p[:nl]
        # derivative: sin(th) dP/dth = l x P_l - (l+m) P_{l-1} (in unnormalized P);
        # in the normalized functions (l+m) N_l/N_{l-1} = sqrt((2l+1)(l^2-m^2)/(2l-1)).
        dPm = np.zeros_like(Pm)
        for i in range(nl):
            l = m + i
            t = l * x * Pm[i]
            if i > 0:
                t = t - math.sqrt((2 * l + 1) * (l * l - m * m) / (2.0 * l - 1)) * Pm[i - 1]
            dPm[i] = t / s
        P[m], dP[m], mPs[m] = Pm, dPm, m * Pm / s
    return P, dP, mPs


@dataclass
class Grid:
    """All discretization data for one plan (oracle side)."""
    L: int
    M: int
    m0: int
    N: int
    eta: float = 0.35
    Np: int = 0
    nth: int = 0
    nphi: int = 0

    def __post_init__(self):
        Np, nth, nphi = default_grid_sizes(self.L, self.M, self.m0, self.N)
        self.Np = self.Np or Np
        self.nth = self.nth or nth
        self.nphi = self.nphi or nphi
        self.ri, self.ro = shell_radii(self.eta)
        self.rad = Radial(self.N, self.Np, self.ri, self.ro)
        self.K = min(self.M, self.L) // self.m0
        self.ms = [k * self.m0 for k in range(self.K + 1)]
        self.ct, self.wt, self.st = gauss_legendre(self.nth)
        self.P, self.dP, self.mPs = legendre_tables(self.L, self.ms, self.ct, self.st)
        # sector grid: phi_k = 2 pi k /(m0 N_phi)
        self.phi = 2.0 * np.pi * np.arange(self.nphi) / (self.m0 * self.nphi)
