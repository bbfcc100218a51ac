"""Writes rw4_L16_m4_N16.npz: the m0 = 4 rotating wave (RW4) of the tiny shell, computed with the
FP64 oracle only.

RW4 is the first state to bifurcate at Ek = 1e-3 (Sec. 2.2; the paper shows it at Ra = 77 with
kinetic-energy density about 25, and the paper's own states were found by timestepping from a
cos(4 phi) perturbation).  Recipe:
  1. the shell L = M = 16, m0 = 4, N = 16, Ek = 1e-3, Pr = 1, Ra = 78 (1.2 x 6.5 Ek^(-1/3));
  2. the discrete conductive state plus the seeded perturbation of amplitude 1e-3 with
     coefficients decaying as (l+1)^-2 (seed 101);
  3. 1500 oracle IMEX steps at dt = 2e-3 (t = 3: the m = 4 wave grows and saturates);
  4. the drift speed estimated from the phase advance of one m = 4 coefficient over 50 more
     steps (a rotating wave has coefficients g_m(t) = g_m* exp(-i m C t) in the lab frame);
  5. oracle Newton-GMRES on R_C(X) = B_C(X) - X at dt = 200 with the phase slot of Sec. 3.4,
     to ||R|| <= 1e-12.
Run from the repository root:  python tests/golden/make_rw4.py
"""
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import seeded_inputs as si  # noqa: E402
from oracle.solver import Problem, newton  # noqa: E402

SHELL = dict(L=16, M=16, m0=4, N=16, Ek=1e-3, Pr=1.0, Ra=78.0)
OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "rw4_L16_m4_N16.npz")


def main():
    s = SHELL
    dt = 2e-3
    p = Problem(s["L"], s["M"], s["m0"], s["N"], Ek=s["Ek"], Ra=s["Ra"], Pr=s["Pr"], dt=dt)
    lay = si.Layout(s["L"], s["M"], s["m0"], s["N"])
    X = p.conductive_state() + p.clean(si.random_state(lay, 101, amp=(1e-3, 1e-3, 1e-3), p=2))
    for _ in range(1500):
        X = p.step(X)
    Y = X.copy()
    for _ in range(50):
        Y = p.step(Y)
    o = lay.offset(1, 1, 8, s["N"] // 3)          # f, m = 4, l = 8, an interior node
    C0 = -np.angle((Y[o] + 1j * Y[o + 1]) / (X[o] + 1j * X[o + 1])) / (s["m0"] * 50 * dt)
    pn = Problem(s["L"], s["M"], s["m0"], s["N"], Ek=s["Ek"], Ra=s["Ra"], Pr=s["Pr"], dt=200.0)
    J = si.default_phase_slot(lay, Y)
    Xs, Cs, hist = newton(pn, Y, C0, J, tol=1e-12, gmres_tol=1e-12, restart=40, max_newton=10, max_gmres=800)
    print("drift estimate", C0, "Newton history", [float(h) for h in hist], "C*", Cs, flush=True)
    if not hist[-1] <= 1e-12:
        raise SystemExit("Newton did not converge")
    np.savez(OUT, X=Xs, C=np.float64(Cs), J=np.int64(J), rnorm=np.float64(hist[-1]),
             shell=np.array([s["L"], s["M"], s["m0"], s["N"]], dtype=np.int64),
             params=np.array([s["Ek"], s["Pr"], s["Ra"]]))
    print("wrote", OUT)


if __name__ == "__main__":
    main()
