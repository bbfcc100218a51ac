"""Implicit operator of the IMEX step and its solution (oracle; test infrastructure only).

Per harmonic (l, m), lambda = l(l+1), L_l = d_rr - lambda/r^2 (eq:expcor_e/f), the
system M dX/dt = K X + N(X) with
   M_e = Ek lambda/r^2,        M_f = -Ek lambda/r^2 L_l,        M_T = 1
   K_e = Ek lambda/r^2 L_l e + (2im/r^2) e
         - (2/r^2) [kappa_l (l/r - d_r) f_{l-1} + kappa_{l+1} (-(l+1)/r - d_r) f_{l+1}]
   K_f = -Ek lambda/r^2 L_l^2 f - (2im/r^2) L_l f
         - (2/r^2) [kappa_l (l/r - d_r) e_{l-1} + kappa_{l+1} (-(l+1)/r - d_r) e_{l+1}]
   K_T = (d_rr + (2/r) d_r - lambda/r^2)/Pr
where the implicit Coriolis terms are eq:impcor_e_final / eq:impcor_f_final of Sec. 3.2 with
   kappa_l = (l-1)(l+1)(l-|m|)/(2l-1) N_{l-1}^m/N_l^m = (l^2-1) sqrt((l^2-m^2)/(4l^2-1))
(the coefficient of the l+1 neighbour, l(l+2)(l+1+|m|)/(2l+3) N_{l+1}^m/N_l^m, equals kappa_{l+1}).
M is the operator under the time derivative in eq:expcor_e/f ("the correspondence is
imperfect", Sec. 3.3); the IMEX step of eq:discrete then reads (M - dt K) X+ = M X + dt(...).
Buoyancy is explicit (it sits in F^implicit, eq:defineFimp), so the factor depends on
(dt, Ek, Pr) only.

Explicit-Coriolis variant (Sec. 3.1, eq:expcor_e / eq:expcor_f with the force of eq:defineFexp):
the Coriolis force -2 e_z x U stays in the explicit force, so K keeps only the viscous and
thermal-diffusion parts (no 2im/r^2 terms, no kappa couplings) and the matrices are block
diagonal, one N x N block per (l, m) and potential.  The chains below are then kept with zero
coupling blocks, which the banded solve handles unchanged.

Boundary conditions by row replacement (Sec. 3.1), read as collocation at the
Gauss-Lobatto nodes: e and T rows j = 0 and N-1 become Dirichlet rows; f rows 0 and N-1
become f = 0 and rows 1 and N-2 become d_r f = 0 at r_o and r_i respectively.

The coupling of e_l with f_{l+-1} splits each m into two chains (Sec. 3.2: odd-l e with
even-l f, and the complement); along l each chain is block tridiagonal with N x N
complex blocks.  T is decoupled per l.  Solves use Ruiz equilibration, LAPACK banded LU
with partial pivoting (zgbtrf) and FP64 iterative refinement.
"""
from __future__ import annotations

import math

import numpy as np
import scipy.linalg as sla
from scipy.linalg import lapack

from .grids import Grid


def kappa(l: int, m: int) -> float:
    """Coupling coefficient kappa_l of the implicit Coriolis terms (0 for l <= m or l <= 1)."""
    if l <= 1 or l <= abs(m):
        return 0.0
    return (l * l - 1.0) * math.sqrt((l * l - m * m) / (4.0 * l * l - 1.0))


def kappa_from_paper(l: int, m: int, which: str) -> float:
    """The printed coefficients, evaluated literally through N_l^m (for the pin that
    kappa equals them).  which='lower': coefficient of the l-1 neighbour in row l;
    'upper': coefficient of the l+1 neighbour in row l."""
    from .grids import norm_factor
    if which == "lower":
        if l - 1 < abs(m) or l < 1:
            return 0.0
        return (l - 1) * (l + 1) * (l - abs(m)) / (2 * l - 1) * norm_factor(l - 1, m) / norm_factor(l, m)
    return l * (l + 2) * (l + 1 + abs(m)) / (2 * l + 3) * norm_factor(l + 1, m) / norm_factor(l, m)


class Operators:
    """Blocks of M and A = M - dt K for one grid and (Ek, Pr, dt)."""

    def __init__(self, g: Grid, Ek: float, Pr: float, dt: float, coriolis: str = "implicit"):
        if coriolis not in ("implicit", "explicit"):
            raise ValueError("coriolis must be 'implicit' or 'explicit'")
        self.g, self.Ek, self.Pr, self.dt = g, Ek, Pr, dt
        self.cor = 1.0 if coriolis == "implicit" else 0.0     # weight of the Coriolis terms in K
        rad = g.rad
        self.r = rad.r
        self.D = rad.D
        self.D2 = rad.D @ rad.D
        self.I = np.eye(g.N)

    # --- pieces -----------------------------------------------------------
    def Lop(self, l):
        lam = l * (l + 1.0)
        return self.D2 - np.diag(lam / self.r ** 2)

    def M_e(self, l):
        lam = l * (l + 1.0)
        return np.diag(self.Ek * lam / self.r ** 2) + 0j

    def M_f(self, l):
        lam = l * (l + 1.0)
        return -np.diag(self.Ek * lam / self.r ** 2) @ self.Lop(l) + 0j

    def K_e_self(self, l, m):
        lam = l * (l + 1.0)
        return (np.diag(self.Ek * lam / self.r ** 2) @ self.Lop(l)
                + self.cor * np.diag(2j * m / self.r ** 2))

    def K_f_self(self, l, m):
        lam = l * (l + 1.0)
        Lo = self.Lop(l)
        return (-np.diag(self.Ek * lam / self.r ** 2) @ Lo @ Lo
                - self.cor * np.diag(2j * m / self.r ** 2) @ Lo)

    def K_couple(self, l, m, nb):
        """Coriolis coupling of row l to the neighbour l+nb (nb = -1 or +1), same form for
        e-rows (acting on f) and f-rows (acting on e)."""
        r = self.r
        if nb == -1:
            kap = kappa(l, m)
            op = np.diag(l / r) - self.D
        else:
            kap = kappa(l + 1, m)
            op = np.diag(-(l + 1.0) / r) - self.D
        return -self.cor * np.diag(2.0 / r ** 2) @ op * kap + 0j

    def A_T(self, l):
        lam = l * (l + 1.0)
        K = (self.D2 + np.diag(2.0 / self.r) @ self.D - np.diag(lam / self.r ** 2)) / self.Pr
        A = self.I - self.dt * K
        N = self.g.N
        A[0] = 0.0
        A[0, 0] = 1.0
        A[N - 1] = 0.0
        A[N - 1, N - 1] = 1.0
        return A

    # --- boundary rows ------------------------------------------------------
    def bc_rows(self, typ):
        """Rows replaced by boundary conditions, for field 'e', 'f' or 'T'."""
        N = self.g.N
        return [0, N - 1] if typ in ("e", "T") else [0, 1, N - 2, N - 1]

    def apply_bc_diag(self, A, typ):
        N = self.g.N
        A = A.copy()
        for j in self.bc_rows(typ):
            A[j] = 0.0
        if typ in ("e", "T"):
            A[0, 0] = A[N - 1, N - 1] = 1.0
        else:
            A[0, 0] = A[N - 1, N - 1] = 1.0
            A[1] = self.D[0]
            A[N - 2] = self.D[N - 1]
        return A

    def apply_bc_off(self, B, typ):
        B = B.copy()
        for j in self.bc_rows(typ):
            B[j] = 0.0
        return B

    # --- chains -----------------------------------------------------------------
    def chain_types(self, m, cls):
        """(type, l) of the unknown blocks of chain cls in {0, 1} at order m."""
        l0 = max(m, 1)
        out = []
        for l in range(l0, self.g.L + 1):
            first = "e" if cls == 0 else "f"
            other = "f" if cls == 0 else "e"
            out.append((first if (l - l0) % 2 == 0 else other, l))
        return out

    def chain_blocks(self, m, cls):
        """Diagonal, lower (row i, col i-1) and upper (row i, col i+1) blocks of A = M - dt K."""
        dt = self.dt
        types = self.chain_types(m, cls)
        Dg, Lo, Up = [], [None], []
        for i, (t, l) in enumerate(types):
            if t == "e":
                Ad = self.M_e(l) - dt * self.K_e_self(l, m)
            else:
                Ad = self.M_f(l) - dt * self.K_f_self(l, m)
            Dg.append(self.apply_bc_diag(Ad, t))
            if i > 0:
                Lo.append(self.apply_bc_off(-dt * self.K_couple(l, m, -1), t))
            if i < len(types) - 1:
                Up.append(self.apply_bc_off(-dt * self.K_couple(l, m, +1), t))
        Up.append(None)
        return types, Dg, Lo, Up


def chain_dense(Dg, Lo, Up):
    """Assemble a chain's block tridiagonal matrix densely (small sizes only)."""
    n, N = len(Dg), Dg[0].shape[0]
    A = np.zeros((n * N, n * N), dtype=complex)
    for i in range(n):
        A[i * N:(i + 1) * N, i * N:(i + 1) * N] = Dg[i]
        if i > 0:
            A[i * N:(i + 1) * N, (i - 1) * N:i * N] = Lo[i]
        if i < n - 1:
            A[i * N:(i + 1) * N, (i + 1) * N:(i + 2) * N] = Up[i]
    return A


def chain_matvec(Dg, Lo, Up, x):
    """y = A x for the block tridiagonal chain; x has shape [n, N, ncol]."""
    n = len(Dg)
    y = np.empty_like(x)
    for i in range(n):
        acc = Dg[i] @ x[i]
        if i > 0:
            acc = acc + Lo[i] @ x[i - 1]
        if i < n - 1:
            acc = acc + Up[i] @ x[i + 1]
        y[i] = acc
    return y


def ruiz(rowmax_fn, colmax_fn, n, iters=30):
    """Ruiz equilibration: returns row and column scalings (vectors of length n)."""
    R = np.ones(n)
    C = np.ones(n)
    for _ in range(iters):
        rm = rowmax_fn(R, C)
        cm = colmax_fn(R, C)
        R = R / np.sqrt(rm)
        C = C / np.sqrt(cm)
        if max(abs(rm - 1).max(), abs(cm - 1).max()) < 1e-3:
            break
    return R, C


class ChainSolver:
    """Equilibrated banded LU of one chain, with FP64 iterative refinement."""

    def __init__(self, Dg, Lo, Up, refine=2):
        self.Dg, self.Lo, self.Up, self.refine = Dg, Lo, Up, refine
        n, N = len(Dg), Dg[0].shape[0]
        self.n, self.N = n, N
        aD = [abs(b) for b in Dg]
        aL = [None] + [abs(b) for b in Lo[1:]]
        aU = [abs(b) for b in Up[:-1]] + [None]

        def rowmax(R, C):
            out = np.zeros(n * N)
            Cb = C.reshape(n, N)
            for i in range(n):
                v = (aD[i] * Cb[i][None, :]).max(1)
                if i > 0:
                    v = np.maximum(v, (aL[i] * Cb[i - 1][None, :]).max(1))
                if i < n - 1:
                    v = np.maximum(v, (aU[i] * Cb[i + 1][None, :]).max(1))
                out[i * N:(i + 1) * N] = v
            return out * R

        def colmax(R, C):
            out = np.zeros(n * N)
            Rb = R.reshape(n, N)
            for j in range(n):
                v = (aD[j] * Rb[j][:, None]).max(0)
                if j + 1 < n:
                    v = np.maximum(v, (aL[j + 1] * Rb[j + 1][:, None]).max(0))
                if j - 1 >= 0:
                    v = np.maximum(v, (aU[j - 1] * Rb[j - 1][:, None]).max(0))
                out[j * N:(j + 1) * N] = v
            return out * C

        self.R, self.C = ruiz(rowmax, colmax, n * N)
        kl = ku = 2 * N - 1
        self.kl, self.ku = kl, ku
        nn = n * N
        ab = np.zeros((2 * kl + ku + 1, nn), dtype=complex)
        Rb, Cb = self.R.reshape(n, N), self.C.reshape(n, N)

        def put(i0, j0, blk):
            ii, jj = np.meshgrid(np.arange(N) + i0, np.arange(N) + j0, indexing="ij")
            ab[kl + ku + ii - jj, jj] = blk

        for i in range(n):
            put(i * N, i * N, Rb[i][:, None] * Dg[i] * Cb[i][None, :])
            if i > 0:
                put(i * N, (i - 1) * N, Rb[i][:, None] * Lo[i] * Cb[i - 1][None, :])
            if i < n - 1:
                put(i * N, (i + 1) * N, Rb[i][:, None] * Up[i] * Cb[i + 1][None, :])
        lu, piv, info = lapack.zgbtrf(ab, kl, ku)
        if info != 0:
            raise np.linalg.LinAlgError(f"zgbtrf info={info}")
        self.lu, self.piv = lu, piv

    def _solve_once(self, b):
        """b: [n*N, ncol] complex."""
        rhs = self.R[:, None] * b
        x, info = lapack.zgbtrs(self.lu, self.kl, self.ku, rhs, self.piv)
        if info != 0:
            raise np.linalg.LinAlgError(f"zgbtrs info={info}")
        return self.C[:, None] * x

    def solve(self, b):
        """Solve A x = b for b of shape [n, N, ncol]."""
        n, N = self.n, self.N
        bb = b.reshape(n * N, -1)
        x = self._solve_once(bb)
        for _ in range(self.refine):
            r = bb - chain_matvec(self.Dg, self.Lo, self.Up, x.reshape(n, N, -1)).reshape(n * N, -1)
            x = x + self._solve_once(r)
        return x.reshape(b.shape)


class TSolver:
    """Equilibrated dense LU of the temperature block of one l, with refinement."""

    def __init__(self, A, refine=2):
        self.A, self.refine = A, refine
        aA = abs(A)
        self.R, self.C = ruiz(lambda R, C: (aA * C[None, :]).max(1) * R,
                              lambda R, C: (aA * R[:, None]).max(0) * C, A.shape[0])
        self.lu = sla.lu_factor(self.R[:, None] * A * self.C[None, :])

    def _solve_once(self, b):
        def real_solve(br):
            return self.C[:, None] * sla.lu_solve(self.lu, self.R[:, None] * br)
        if np.iscomplexobj(b):
            return real_solve(b.real) + 1j * real_solve(b.imag)
        return real_solve(b)

    def solve(self, b):
        x = self._solve_once(b)
        for _ in range(self.refine):
            x = x + self._solve_once(b - self.A @ x)
        return x
