"""Oracle method of moving asymptotes (test infrastructure only).

Sec. "Optimisation problem": the design problem (one volume constraint) is
solved with MMA.  The algorithm is in the cited references, not in the paper's
text; this is the published method written out for m = 1 constraint, in the
form of Svanberg's MMA with the usual safeguards (the reading the HIP path
follows as well):

* asymptotes: low = x - 0.5 (xmax - xmin), upp = x + 0.5 (xmax - xmin) in the
  first two iterations; afterwards low = x - s (x_{k-1} - low_{k-1}),
  upp = x + s (upp_{k-1} - x_{k-1}) with s = 1.2 where the last two steps of
  x_j had the same sign, 0.7 where they had opposite signs, 1 otherwise;
  low clipped to [x - 10 d, x - 0.01 d], upp to [x + 0.01 d, x + 10 d],
  d = xmax - xmin;
* subproblem bounds alpha = max(xmin, low + 0.1 (x - low), x - move d),
  beta = min(xmax, upp - 0.1 (upp - x), x + move d);
* convex separable approximations of f_i, i = 0 (objective), 1 (constraint):
  p = (upp - x)^2 (1.001 max(df, 0) + 0.001 max(-df, 0) + 1e-5 / d),
  q = (x - low)^2 (0.001 max(df, 0) + 1.001 max(-df, 0) + 1e-5 / d),
  f_i ~ r_i + sum_j p_ij / (upp_j - x_j) + q_ij / (x_j - low_j);
* the subproblem min f_0~ s.t. f_1~ <= 0, alpha <= x <= beta through its
  dual: x_j(lam) minimises (p0 + lam p1) / (upp - x) + (q0 + lam q1) / (x - low)
  over [alpha_j, beta_j] in closed form; lam >= 0 is the root of
  f_1~(x(lam)) (or 0 if f_1~(x(0)) <= 0), found by doubling then 200-step
  bisection.
"""
from __future__ import annotations

import numpy as np


class MMA:
    def __init__(self, n: int, xmin: float = 0.0, xmax: float = 1.0, move: float = 0.2):
        self.n, self.xmin, self.xmax, self.move = n, xmin, xmax, move
        self.k = 0
        self.xold1 = None
        self.xold2 = None
        self.low = None
        self.upp = None

    def subproblem(self, x, f1, df0, df1):
        d = self.xmax - self.xmin
        self.k += 1
        if self.k <= 2:
            low = x - 0.5 * d
            upp = x + 0.5 * d
        else:
            zz = (x - self.xold1) * (self.xold1 - self.xold2)
            s = np.where(zz > 0, 1.2, np.where(zz < 0, 0.7, 1.0))
            low = x - s * (self.xold1 - self.low)
            upp = x + s * (self.upp - self.xold1)
            low = np.minimum(np.maximum(low, x - 10 * d), x - 0.01 * d)
            upp = np.maximum(np.minimum(upp, x + 10 * d), x + 0.01 * d)
        alpha = np.maximum(np.maximum(self.xmin, low + 0.1 * (x - low)), x - self.move * d)
        beta = np.minimum(np.minimum(self.xmax, upp - 0.1 * (upp - x)), x + self.move * d)
        ux2, xl2 = (upp - x) ** 2, (x - low) ** 2
        reg = 1e-5 / d

        def pq(df):
            pos, neg = np.maximum(df, 0.0), np.maximum(-df, 0.0)
            return ux2 * (1.001 * pos + 0.001 * neg + reg), xl2 * (0.001 * pos + 1.001 * neg + reg)

        p0, q0 = pq(df0)
        p1, q1 = pq(df1)
        r1 = f1 - np.sum(p1 / (upp - x) + q1 / (x - low))
        return dict(low=low, upp=upp, alpha=alpha, beta=beta, p0=p0, q0=q0, p1=p1, q1=q1, r1=r1)

    @staticmethod
    def x_of(sp, lam):
        P = sp["p0"] + lam * sp["p1"]
        Q = sp["q0"] + lam * sp["q1"]
        sP, sQ = np.sqrt(P), np.sqrt(Q)
        xs = (sP * sp["low"] + sQ * sp["upp"]) / (sP + sQ)
        return np.minimum(np.maximum(xs, sp["alpha"]), sp["beta"])

    @staticmethod
    def g_of(sp, x):
        return sp["r1"] + np.sum(sp["p1"] / (sp["upp"] - x) + sp["q1"] / (x - sp["low"]))

    def update(self, x, f0, df0, f1, df1):
        """One MMA iteration; returns (x_new, lam)."""
        x = np.asarray(x, dtype=np.float64)
        sp = self.subproblem(x, f1, np.asarray(df0, dtype=np.float64), np.asarray(df1, dtype=np.float64))
        if self.g_of(sp, self.x_of(sp, 0.0)) <= 0.0:
            lam = 0.0
        else:
            lo, hi = 0.0, 1.0
            while self.g_of(sp, self.x_of(sp, hi)) > 0.0 and hi < 1e30:
                lo, hi = hi, 2.0 * hi
            for _ in range(200):
                mid = 0.5 * (lo + hi)
                if mid <= lo or mid >= hi:
                    break
                if self.g_of(sp, self.x_of(sp, mid)) > 0.0:
                    lo = mid
                else:
                    hi = mid
            lam = hi
        xnew = self.x_of(sp, lam)
        self.xold2 = self.xold1
        self.xold1 = x.copy()
        self.low, self.upp = sp["low"], sp["upp"]
        return xnew, lam
