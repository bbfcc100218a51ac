"""Natural-parameter continuation with turning-point switching (oracle; test infrastructure only).

Sec. 3.5 (continuation) and Sec. 3.6 (turning points); Sec. 4.2 for the Ekman variant:
  * step control, eq:new_Ra / eq:alpha_cont: p_new = p_i + alpha (p_i - p_{i-1}) with
    alpha = (N_opt + 1) / (N_i + 1), N_i the Newton iterations of the last point;
  * prediction, eq:lagrange: the quadratic Lagrange weights (a, b, c) of the three previous
    parameter values, evaluated at p_new (so that p_new = a p_i + b p_{i-1} + c p_{i-2}), give the
    new estimate U = a U_i + b U_{i-1} + c U_{i-2};
  * turning points, eq:tp_detection_Ra: with J the index of the largest |U_i| element, when
    |(U_J,i - U_J,i-1)/U_J,i| exceeds gamma |(p_i - p_{i-1})/p_i| the component U_J becomes the
    independent variable: U_J,new = U_J,i + alpha (U_J,i - U_J,i-1), the weights are those of the
    three previous U_J values at U_J,new, and the parameter is extrapolated with them like every
    other component (eq:quad_extra_Ra).  Newton then runs at that fixed parameter with every
    component free.  The switch back happens when the test reverses.
With one point on the branch the first step is p_0 + dp_first from that point (zeroth order),
with two the prediction is linear.  A point that needed no Newton step counts as one in alpha.
The drift speed C is carried with the state and extrapolated with the same weights.

If Newton fails at the predicted point, the step is taken again from the last converged point
with alpha and gamma halved (Sec. 3.6 restarts a failed continuation with a reduced gamma), up
to max_retries times.

The driver is generic: `solve(param, X, C) -> (X, C, newton_steps, converged)` runs Newton at a
fixed parameter, so the same logic serves Ra (p = Ra) and Ek (p = log10 Ek, Sec. 4.2).
"""
from __future__ import annotations

import numpy as np


def step_factor(n_opt: int, n_last: int) -> float:
    """alpha of eq:alpha_cont."""
    return (n_opt + 1.0) / (n_last + 1.0)


def lagrange_weights(t_new, ts):
    """Weights w_q of the Lagrange interpolation polynomial through the nodes ts (1, 2 or 3 of
    them), evaluated at t_new: f(t_new) ~ sum_q w_q f(ts[q])."""
    ts = [float(t) for t in ts]
    w = []
    for q, tq in enumerate(ts):
        v = 1.0
        for r, tr in enumerate(ts):
            if r != q:
                v *= (t_new - tr) / (tq - tr)
        w.append(v)
    return w


class Continuation:
    """Branch of converged points (param, X, C), newest last."""

    def __init__(self, solve, n_opt=5, gamma=50.0, max_retries=3):
        self.solve = solve
        self.n_opt, self.gamma, self.max_retries = n_opt, gamma, max_retries
        self.params, self.states, self.Cs, self.iters = [], [], [], []
        self.state_mode = []          # per point: True if it was predicted with U_J as the variable

    def add_point(self, p, X, C, iters):
        self.params.append(float(p))
        self.states.append(np.array(X, dtype=float))
        self.Cs.append(float(C))
        self.iters.append(int(iters))
        self.state_mode.append(False)

    def turning(self, gamma):
        """eq:tp_detection_Ra on the last two points: (switch to U_J, J)."""
        X1, X0 = self.states[-1], self.states[-2]
        J = int(np.argmax(np.abs(X1)))
        dU = abs((X1[J] - X0[J]) / X1[J])
        p1, p0 = self.params[-1], self.params[-2]
        dp = abs((p1 - p0) / p1)
        return dU > gamma * dp, J

    def predict(self, scale=1.0):
        """(param, X, C) estimate of the next point and whether U_J was the variable; scale
        multiplies alpha and gamma (1 on a first attempt)."""
        n = len(self.params)
        if n < 2:
            raise ValueError("continuation needs two converged points to set its step")
        alpha = scale * step_factor(self.n_opt, max(self.iters[-1], 1))
        k = min(n, 3)
        Xs, Cs, ps = self.states[-k:], self.Cs[-k:], self.params[-k:]
        switch, J = self.turning(scale * self.gamma)
        if not switch:
            p_new = ps[-1] + alpha * (ps[-1] - ps[-2])
            w = lagrange_weights(p_new, ps)
        else:
            uj = [X[J] for X in Xs]
            u_new = uj[-1] + alpha * (uj[-1] - uj[-2])
            w = lagrange_weights(u_new, uj)
            p_new = sum(wq * pq for wq, pq in zip(w, ps))
        X = sum(wq * Xq for wq, Xq in zip(w, Xs))
        C = sum(wq * Cq for wq, Cq in zip(w, Cs))
        return p_new, X, C, switch

    def step(self, dp_first=None):
        """One continuation step; returns (param, converged, retries).  dp_first: the first
        parameter step when the branch holds a single point (halved on a retry)."""
        for r in range(self.max_retries + 1):
            if len(self.params) == 1:
                p, X, C, switch = self.params[0] + dp_first * 0.5 ** r, self.states[0], self.Cs[0], False
            else:
                p, X, C, switch = self.predict(0.5 ** r)
            Xn, Cn, its, ok = self.solve(p, X, C)
            if ok:
                self.add_point(p, Xn, Cn, its)
                self.state_mode[-1] = switch
                return p, True, r
        return p, False, r
