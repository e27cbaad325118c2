"""Alg. 3 (constraint optimisation on the Stiefel manifold) — oracle, FP64.

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__``).

Steps, in the paper's order (Section 3, Alg. 3 with eqs. (bb-1), (NMLS-Armijo);
stopping rules of Section 4.1):

1. C_0 = E(X_0), Q_0 = 1.
2. While ||grad E(X_k)||_F > eps:
   a. BB step: tau_{k,1} = tr(S^T S)/|tr(S^T Y)|, tau_{k,2} = |tr(S^T Y)|/tr(Y^T Y) with
      S = X_k - X_{k-1}, Y = grad E(X_k) - grad E(X_{k-1}).  The paper allows either;
      the default alternates (tau_{k,1} for odd k, tau_{k,2} for even k).  At k = 0, and
      whenever the BB value is not finite and positive, tau_0 is used (the paper only says
      an unbounded value is "reset to a finite number"); the value is clamped to
      [tau_min, tau_max].
   b. tau_k = tau_BB delta^h for the smallest h >= 0 with
      E(X_k(tau_k)) <= C_k - rho_1 tau_k ||grad E(X_k)||_F^2; after h_max reductions the
      last trial is accepted and the event counted.
   c. X_{k+1} = X_QR(tau_k) or X_WY(tau_k).  With WY, a trial point whose
      ||X^T X - I||_F exceeds reorth_tol (1e-12 in Section 4.1) is re-orthonormalised by
      Cholesky QR before its energy is evaluated.
   d. Q_{k+1} = eta Q_k + 1, C_{k+1} = (eta Q_k C_k + E(X_{k+1}))/Q_{k+1}.
   e. Stop when the mean of the last three df_k = |E_{k-1} - E_k|/(|E_{k-1}| + 1) falls
      below stagnation_tol (1e-13), or after max_iter iterations.

Parameter values the paper leaves open (rho_1, delta, eta, tau_0, bounds) take common
values from the nonmonotone-line-search literature; see ``Params``.

The optimiser is written against a small "manifold" object so that the same steps
serve the Euclidean constraint X^T X = I and the B-metric constraint X^T B X = I.
"""
from __future__ import annotations

import dataclasses
import math
from typing import Callable, List

import numpy as np

from . import stiefel


@dataclasses.dataclass
class Params:
    tau0: float = 1e-3
    rho1: float = 1e-4
    delta: float = 0.1
    eta: float = 0.85
    eps_g: float = 1e-6
    max_iter: int = 10000
    bb: str = "alt"          # "alt", "bb1", "bb2"
    retraction: str = "qr"   # "qr", "wy"
    tau_min: float = 1e-20
    tau_max: float = 1e20
    h_max: int = 20
    reorth_tol: float = 1e-12
    stagnation_tol: float = 1e-13


@dataclasses.dataclass
class Result:
    X: np.ndarray
    energy: object
    E: float
    gnorm: float
    iters: int
    nfe: int
    backtracks: int
    ls_fail: int
    reorths: int
    stop: str
    history: List[dict]


class EuclideanStiefel:
    """X^T X = I (Section 3)."""

    def grad(self, X, G):
        return stiefel.manifold_grad(X, G)

    def inner(self, A, B):
        return float(np.sum(A * B))

    def retract(self, kind, X, G, tau):
        if kind == "qr":
            return stiefel.retract_qr(X, G, tau)
        return stiefel.retract_wy(X, G, tau)

    def orth_error(self, X):
        return stiefel.orth_error(X)

    def reorth(self, X):
        return stiefel.cholqr(X)[0]


def bb_candidates(ss, sy, yy):
    """The two Barzilai-Borwein values of eq. (bb-1) from the Frobenius sums
    ss = tr(S^T S), sy = tr(S^T Y), yy = tr(Y^T Y):
    tau_{k,1} = ss / |sy|  and  tau_{k,2} = |sy| / yy  (inf where the divisor is zero)."""
    tau1 = ss / abs(sy) if sy != 0.0 else float("inf")
    tau2 = abs(sy) / yy if yy != 0.0 else float("inf")
    return tau1, tau2


def bb_step(k, ss, sy, yy, p: Params):
    """Step of iteration k: tau_0 at k = 0; otherwise tau_{k,1} (rule "bb1"), tau_{k,2}
    ("bb2") or, by default, tau_{k,1} on odd and tau_{k,2} on even k.  A value that is not
    finite and positive becomes tau_0; the result is clamped to [tau_min, tau_max]."""
    if k == 0:
        return p.tau0
    rule = p.bb
    if rule == "alt":
        rule = "bb1" if (k % 2 == 1) else "bb2"
    tau1, tau2 = bb_candidates(ss, sy, yy)
    tau = tau1 if rule == "bb1" else tau2
    if not math.isfinite(tau) or tau <= 0.0:
        tau = p.tau0
    return min(max(tau, p.tau_min), p.tau_max)


def reference_update(C, Q, E_new, eta):
    """Alg. 3's nonmonotone reference: Q_{k+1} = eta Q_k + 1,
    C_{k+1} = (eta Q_k C_k + E(X_{k+1})) / Q_{k+1}.  Returns (C_{k+1}, Q_{k+1})."""
    Qn = eta * Q + 1.0
    return (eta * Q * C + E_new) / Qn, Qn


def minimize(energy_grad: Callable, X0, params: Params = Params(), manifold=None, vh0=None,
             callback=None, keep_iterates=False):
    """Run Alg. 3 from X0.  energy_grad(X, vh_warm) -> (Energy, E_X, vh).

    callback(k, E, gnorm), if given, is called after every accepted iteration.  With
    keep_iterates the history also holds every accepted X_k (small problems only).
    """
    mf = manifold or EuclideanStiefel()
    p = params
    X = np.array(X0, dtype=np.float64)
    en, G, vh = energy_grad(X, vh0)
    E = en.total
    D = mf.grad(X, G)
    g2 = mf.inner(D, D)
    C, Q = E, 1.0
    k = 0
    nfe, backtracks, ls_fail, reorths = 1, 0, 0, 0
    ss = sy = yy = 0.0
    dfs: List[float] = []
    hist = []
    stop = "maxit"
    while True:
        if math.sqrt(g2) <= p.eps_g:
            stop = "grad"
            break
        if k >= p.max_iter:
            stop = "maxit"
            break
        tau_bb = bb_step(k, ss, sy, yy, p)
        tau1, tau2 = bb_candidates(ss, sy, yy) if k > 0 else (p.tau0, p.tau0)
        h = 0
        while True:
            tau = tau_bb * p.delta ** h
            Xt = mf.retract(p.retraction, X, G, tau)
            if p.retraction == "wy" and mf.orth_error(Xt) > p.reorth_tol:
                Xt = mf.reorth(Xt)
                reorths += 1
            ent, Gt, vht = energy_grad(Xt, vh)
            nfe += 1
            ok = ent.total <= C - p.rho1 * tau * g2
            if ok or h >= p.h_max:
                if not ok:
                    ls_fail += 1
                break
            h += 1
            backtracks += 1
        Dt = mf.grad(Xt, Gt)
        S = Xt - X
        Yd = Dt - D
        ss, sy, yy = mf.inner(S, S), mf.inner(S, Yd), mf.inner(Yd, Yd)
        Et = ent.total
        df = abs(E - Et) / (abs(E) + 1.0)
        hist.append(dict(k=k, E=E, E_new=Et, C=C, Q=Q, tau=tau, tau_bb=tau_bb, tau1=tau1,
                         tau2=tau2, h=h, g2=g2, armijo_rhs=C - p.rho1 * tau * g2))
        if keep_iterates:
            hist[-1]["X"] = X.copy()
        C, Q = reference_update(C, Q, Et, p.eta)
        X, G, D, E, en, vh = Xt, Gt, Dt, Et, ent, vht
        g2 = mf.inner(D, D)
        k += 1
        dfs.append(df)
        if callback is not None:
            callback(k, E, math.sqrt(g2))
        if len(dfs) >= 3 and (dfs[-1] + dfs[-2] + dfs[-3]) / 3.0 < p.stagnation_tol:
            stop = "stagnation"
            break
    return Result(X=X, energy=en, E=E, gnorm=math.sqrt(g2), iters=k, nfe=nfe,
                  backtracks=backtracks, ls_fail=ls_fail, reorths=reorths, stop=stop,
                  history=hist)
