"""Step, Newton residual, Jacobian-vector product, GMRES and Newton (oracle; test
infrastructure only).

IMEX Euler step (Sec. 3.3, eq:discrete), augmented with the drift term of a rotating wave
(Sec. 3.4, eq:twdefine and the step that follows it):
    (M - dt K) X+ = M X + dt (N(X) + C im M X),   boundary rows replaced,
so the step map is B_C(X) = X+ and the Newton residual is R = B_C(X) - X
(eq:finalrhs: B - I = P(dt) A, whose roots do not depend on dt).
Jacobian action (Sec. 3.3, eq:precond and the replacement rules; Sec. 3.4, eq:twNewton
and the phase-slot trick): for v with c = v_J and u = v with u_J = 0,
    y = (M - dt K)^-1 [M u + dt (N'_X u + C im M u + c im M X)]_homogeneous BCs  -  u.

Slots without physical content (e, f at l = 0; imaginary parts at m = 0) are set to 0 by
the step map, so R = -X and y = -v there.

coriolis="explicit" is the variant of Sec. 3.1 (eq:expcor_e / eq:expcor_f, force of
eq:defineFexp): -2 e_z x U (-2 e_z x u in the Jacobian action) joins the explicit force before
the curl projections, and the implicit operator loses its Coriolis terms (block diagonal).
The roots of R do not change, up to the radial truncation of the projected Coriolis force.
"""
from __future__ import annotations

import numpy as np

from . import physics
from .grids import Grid
from .operators import ChainSolver, Operators, TSolver


class Problem:
    def __init__(self, L, M, m0, N, Ek, Ra, Pr, dt, eta=0.35, Np=0, nth=0, nphi=0, refine=2,
                 coriolis="implicit"):
        self.g = Grid(L, M, m0, N, eta=eta, Np=Np, nth=nth, nphi=nphi)
        self.Ek, self.Ra, self.Pr, self.dt = Ek, Ra, Pr, dt
        self.refine = refine
        self.coriolis = coriolis
        self.ops = Operators(self.g, Ek, Pr, dt, coriolis=coriolis)
        self._chains = None
        self._tsol = None
        g = self.g
        S = sum(g.L - m + 1 for m in g.ms)
        self.n_real = 2 * 3 * g.N * S
        self.mask = self._nonphysical_mask()
        self.base = None

    # --- layout helpers -------------------------------------------------------
    def _nonphysical_mask(self):
        g = self.g
        e, f, T = [], [], []
        for k, m in enumerate(g.ms):
            nl = g.L - m + 1
            z = np.zeros((nl, g.N), dtype=complex)
            if m == 0:
                z += 1j                                  # Im parts at m = 0
            ze, zf = z.copy(), z.copy()
            if m == 0:
                ze[0] = 1 + 1j                           # e_00, f_00
                zf[0] = 1 + 1j
            e.append(ze)
            f.append(zf)
            T.append(z.copy())
        return physics.pack(g, e, f, T) != 0

    def clean(self, v):
        w = v.copy()
        w[self.mask] = 0.0
        return w

    # --- factorization -------------------------------------------------------------
    def factor(self):
        g, ops = self.g, self.ops
        self._chains = {}
        for k, m in enumerate(g.ms):
            for cls in (0, 1):
                types, Dg, Lo, Up = ops.chain_blocks(m, cls)
                self._chains[(k, cls)] = (types, ChainSolver(Dg, Lo, Up, refine=self.refine))
        self._tsol = [TSolver(ops.A_T(l), refine=self.refine) for l in range(g.L + 1)]

    def solve(self, be, bf, bT):
        """Solve (M - dt K) X = b, b already carrying its boundary rows."""
        if self._chains is None:
            self.factor()
        g = self.g
        xe = [np.zeros_like(a) for a in be]
        xf = [np.zeros_like(a) for a in bf]
        xT = [np.zeros_like(a) for a in bT]
        for k, m in enumerate(g.ms):
            for cls in (0, 1):
                types, sol = self._chains[(k, cls)]
                if not types:
                    continue
                rhs = np.stack([(be if t == "e" else bf)[k][l - m] for t, l in types])[:, :, None]
                x = sol.solve(rhs)[:, :, 0]
                for i, (t, l) in enumerate(types):
                    (xe if t == "e" else xf)[k][l - m] = x[i]
        for l in range(g.L + 1):
            ks = [k for k, m in enumerate(g.ms) if m <= l]
            cols = np.stack([bT[k][l - g.ms[k]] for k in ks], axis=1)     # [N, nk]
            x = self._tsol[l].solve(cols)
            for i, k in enumerate(ks):
                xT[k][l - g.ms[k]] = x[:, i]
        return xe, xf, xT

    # --- pieces of the right-hand side ------------------------------------------------
    def M_apply(self, e, f, T):
        g, ops = self.g, self.ops
        Me, Mf = [], []
        for k, m in enumerate(g.ms):
            ls = np.arange(m, g.L + 1)
            Me.append(np.stack([ops.M_e(l) @ e[k][i] for i, l in enumerate(ls)]) if len(ls) else e[k])
            Mf.append(np.stack([ops.M_f(l) @ f[k][i] for i, l in enumerate(ls)]) if len(ls) else f[k])
        return Me, Mf, [t.copy() for t in T]

    def buoyancy(self, T):
        """Ra lambda T/(r r_o): the f-equation projection of Ra T r/r_o e_r, at the N nodes."""
        g = self.g
        r = g.rad.r[None, :]
        return [self.Ra * lam[:, None] * T[k] / (r * g.ro) for k, lam in enumerate(physics.lam_list(g))]

    def _set_bc(self, be, bf, bT, inhomogeneous):
        g = self.g
        N = g.N
        for k in range(len(g.ms)):
            for a in (be[k], bT[k]):
                a[:, 0] = 0.0
                a[:, N - 1] = 0.0
            bf[k][:, [0, 1, N - 2, N - 1]] = 0.0
        if inhomogeneous:
            bT[0][0, 0] = 0.0        # T_00(r_o) = 0
            bT[0][0, N - 1] = 1.0    # T_00(r_i) = 1  (Y_0^0 = 1)

    def _zero_nonphysical(self, e, f, T):
        g = self.g
        if g.ms[0] == 0:
            e[0][0] = 0.0
            f[0][0] = 0.0
            for a in (e[0], f[0], T[0]):
                a.imag[:] = 0.0

    # --- the maps ------------------------------------------------------------------
    def step(self, X, C=0.0):
        """B_C(X): one IMEX step with drift speed C."""
        g = self.g
        e, f, T = physics.unpack(g, self.clean(X))
        F = physics.fields(g, physics.spectral_inputs(g, e, f, T))
        W, Q = physics.nonlinear_forces(F, self.Ek)
        if self.coriolis == "explicit":
            W = tuple(a + b for a, b in zip(W, physics.coriolis_force(g, F)))
        Ne, Nf, NT = physics.project(g, W, Q)
        Bf = self.buoyancy(T)
        Me, Mf, MT = self.M_apply(e, f, T)
        dt = self.dt
        im = [1j * m for m in g.ms]
        be = [Me[k] + dt * (Ne[k] + C * im[k] * Me[k]) for k in range(len(g.ms))]
        bf = [Mf[k] + dt * (Nf[k] + Bf[k] + C * im[k] * Mf[k]) for k in range(len(g.ms))]
        bT = [MT[k] + dt * (NT[k] + C * im[k] * MT[k]) for k in range(len(g.ms))]
        self._set_bc(be, bf, bT, inhomogeneous=True)
        xe, xf, xT = self.solve(be, bf, bT)
        self._zero_nonphysical(xe, xf, xT)
        return physics.pack(g, xe, xf, xT)

    def residual(self, X, C=0.0):
        return self.step(X, C) - X

    def set_base(self, X, C=0.0, J=-1):
        g = self.g
        Xc = self.clean(X)
        e, f, T = physics.unpack(g, Xc)
        F = physics.fields(g, physics.spectral_inputs(g, e, f, T))
        Me, Mf, MT = self.M_apply(e, f, T)
        self.base = dict(X=Xc, F=F, M=(Me, Mf, MT), C=C, J=J)

    def jvp(self, v):
        """(B_X - I)(u, c) with c stored in slot J (J < 0: no drift unknown)."""
        if self.base is None:
            raise RuntimeError("set_base first")
        g, b = self.g, self.base
        J = b["J"]
        u = v.copy()
        c = 0.0
        if J >= 0:
            c = u[J]
            u[J] = 0.0
        e, f, T = physics.unpack(g, self.clean(u))
        Fu = physics.fields(g, physics.spectral_inputs(g, e, f, T))
        W, Q = physics.linearized_forces(b["F"], Fu, self.Ek)
        if self.coriolis == "explicit":
            W = tuple(a + b_ for a, b_ in zip(W, physics.coriolis_force(g, Fu)))
        Ne, Nf, NT = physics.project(g, W, Q)
        Bf = self.buoyancy(T)
        Me, Mf, MT = self.M_apply(e, f, T)
        XMe, XMf, XMT = b["M"]
        dt, C = self.dt, b["C"]
        im = [1j * m for m in g.ms]
        n = len(g.ms)
        be = [Me[k] + dt * (Ne[k] + C * im[k] * Me[k] + c * im[k] * XMe[k]) for k in range(n)]
        bf = [Mf[k] + dt * (Nf[k] + Bf[k] + C * im[k] * Mf[k] + c * im[k] * XMf[k]) for k in range(n)]
        bT = [MT[k] + dt * (NT[k] + C * im[k] * MT[k] + c * im[k] * XMT[k]) for k in range(n)]
        self._set_bc(be, bf, bT, inhomogeneous=False)
        xe, xf, xT = self.solve(be, bf, bT)
        self._zero_nonphysical(xe, xf, xT)
        return physics.pack(g, xe, xf, xT) - u

    def conductive_state(self):
        """Discrete conductive state: T_00 solves the l = 0 temperature rows with
        T(r_i) = 1, T(r_o) = 0 and zero interior right-hand side; everything else 0."""
        g = self.g
        N = g.N
        A = self.ops.A_T(0)
        # interior rows of A_T(0) are I - dt K_T; use K_T itself (dt-independent root)
        K = A.copy()
        K[1:N - 1] = (self.ops.D2 + np.diag(2.0 / g.rad.r) @ self.ops.D)[1:N - 1]
        b = np.zeros(N)
        b[N - 1] = 1.0
        t = np.linalg.solve(K, b)
        X = np.zeros(self.n_real)
        # T block starts at field 2, lm index 0
        S = sum(g.L - m + 1 for m in g.ms)
        o = 2 * (g.N * (2 * S))
        X[o:o + 2 * N:2] = t
        return X


# --- Krylov / Newton -----------------------------------------------------------------------

def gmres(matvec, b, tol=1e-10, restart=40, maxiter=400, x0=None):
    """Restarted GMRES (Saad and Schultz) with modified Gram-Schmidt and Givens rotations.
    Returns (x, relative residual, number of matvecs)."""
    n = b.shape[0]
    x = np.zeros(n) if x0 is None else x0.copy()
    bn = np.linalg.norm(b)
    if bn == 0:
        return x, 0.0, 0
    nmv = 0
    r = b - matvec(x) if x0 is not None else b.copy()
    if x0 is not None:
        nmv += 1
    while True:
        beta = np.linalg.norm(r)
        if beta / bn <= tol or nmv >= maxiter:
            return x, beta / bn, nmv
        V = np.zeros((restart + 1, n))
        H = np.zeros((restart + 1, restart))
        cs, sn = np.zeros(restart), np.zeros(restart)
        g = np.zeros(restart + 1)
        g[0] = beta
        V[0] = r / beta
        j_end = 0
        for j in range(restart):
            w = matvec(V[j])
            nmv += 1
            for i in range(j + 1):
                H[i, j] = w @ V[i]
                w = w - H[i, j] * V[i]
            H[j + 1, j] = np.linalg.norm(w)
            if H[j + 1, j] > 0:
                V[j + 1] = w / H[j + 1, j]
            for i in range(j):
                t = cs[i] * H[i, j] + sn[i] * H[i + 1, j]
                H[i + 1, j] = -sn[i] * H[i, j] + cs[i] * H[i + 1, j]
                H[i, j] = t
            den = np.hypot(H[j, j], H[j + 1, j])
            cs[j], sn[j] = H[j, j] / den, H[j + 1, j] / den
            H[j, j] = den
            H[j + 1, j] = 0.0
            g[j + 1] = -sn[j] * g[j]
            g[j] = cs[j] * g[j]
            j_end = j + 1
            if abs(g[j + 1]) / bn <= tol or nmv >= maxiter:
                break
        y = np.linalg.solve(np.triu(H[:j_end, :j_end]), g[:j_end])
        x = x + V[:j_end].T @ y
        r = b - matvec(x)
        nmv += 1


def newton(prob: Problem, X, C=0.0, J=-1, tol=1e-10, gmres_tol=1e-10, restart=40,
           max_newton=20, max_gmres=400, forcing=None):
    """Newton on R_C(X) = B_C(X) - X (+ forcing), decrement subtracted (Sec. 3.3, 3.4).
    forcing: constant vector added to the residual (manufactured problems)."""
    hist = []
    for it in range(max_newton + 1):
        R = prob.residual(X, C)
        if forcing is not None:
            R = R + forcing
        rn = np.linalg.norm(R)
        hist.append(rn)
        if rn <= tol or it == max_newton:
            break
        prob.set_base(X, C, J)
        du, rel, nmv = gmres(prob.jvp, R, tol=gmres_tol, restart=restart, maxiter=max_gmres)
        if J >= 0:
            c = du[J]
            du[J] = 0.0
            C = C - c
        X = X - du
    return X, C, hist
