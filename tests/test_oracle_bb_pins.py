"""Pins of the Barzilai-Borwein step (Section 3 eq. (bb-1)) and of the nonmonotone
reference value of Alg. 3 (Q_{k+1} = eta Q_k + 1, C_{k+1} = (eta Q_k C_k + E_{k+1})/Q_{k+1}),
checked against what the mathematics fixes rather than against a retyped formula:

* on an eigenvector s of a fixed symmetric matrix with y = A s, both BB values equal
  1/|lambda| (the step that solves the quadratic along s exactly);
* tau_{k,1} >= tau_{k,2} for every pair (Cauchy-Schwarz), with equality only for y || s;
* the default rule takes the larger value on odd k and the smaller on even k, and the sums
  it uses come from S = X_k - X_{k-1} and Y = grad E_k - grad E_{k-1};
* eta = 0 makes C_k the current energy E_k; eta = 1 makes C_k the running mean of
  E_0 .. E_k and Q_k = k + 1.

The last test plants plausible mistakes in the oracle (swapped values, a squared sum, a
wrong alternation, a wrong weight in the recursion) and checks that a pin fails for each.
"""
import math

import numpy as np
import pytest

from oracle import optm, stiefel


class _E:
    def __init__(self, total):
        self.total = total


def _quadratic_problem(n=40, p=3, seed=0):
    """E(X) = tr(X^T A X) on X^T X = I with a fixed SPD A of distinct eigenvalues."""
    rng = np.random.default_rng(seed)
    Qm, _ = np.linalg.qr(rng.standard_normal((n, n)))
    lam = np.linspace(1.0, 9.0, n) + 0.05 * rng.random(n)
    A = (Qm * lam) @ Qm.T
    A = 0.5 * (A + A.T)

    def energy_grad(X, vh=None):
        AX = A @ X
        return _E(float(np.sum(X * AX))), 2.0 * AX, None

    X0, _ = np.linalg.qr(rng.standard_normal((n, p)))
    return A, energy_grad, X0


# ---- pin checks (each raises AssertionError when its property fails) ------------------

def check_eigenvector(cand):
    rng = np.random.default_rng(1)
    Qm, _ = np.linalg.qr(rng.standard_normal((7, 7)))
    lam = np.array([0.3, 1.0, 2.5, 4.0, -1.5, 7.0, 11.0])
    A = (Qm * lam) @ Qm.T
    for j in range(7):
        s = Qm[:, j] * (0.1 + rng.random())
        y = A @ s
        t1, t2 = cand(float(s @ s), float(s @ y), float(y @ y))
        assert abs(t1 * abs(lam[j]) - 1.0) < 1e-12, (j, t1, lam[j])
        assert abs(t2 * abs(lam[j]) - 1.0) < 1e-12, (j, t2, lam[j])


def check_cauchy_schwarz(cand):
    rng = np.random.default_rng(2)
    for _ in range(50):
        s = rng.standard_normal(9)
        y = rng.standard_normal(9) + 0.3 * s
        t1, t2 = cand(float(s @ s), float(s @ y), float(y @ y))
        assert t1 > t2, (t1, t2)
    s = rng.standard_normal(5)
    t1, t2 = cand(float(s @ s), float(s @ (2.5 * s)), float((2.5 * s) @ (2.5 * s)))
    assert abs(t1 - t2) <= 1e-14 * t1


def check_run(hist, prm, energy_grad):
    """Alternation, clamping and the origin of the sums along a recorded run."""
    mf = optm.EuclideanStiefel()
    assert len(hist) >= 6
    for a, b in zip(hist[:-1], hist[1:]):
        k = b["k"]
        Xp, Xk = a["X"], b["X"]
        Dp = mf.grad(Xp, energy_grad(Xp)[1])
        Dk = mf.grad(Xk, energy_grad(Xk)[1])
        S, Y = Xk - Xp, Dk - Dp
        ss, sy, yy = float(np.sum(S * S)), float(np.sum(S * Y)), float(np.sum(Y * Y))
        assert abs(b["tau1"] - ss / abs(sy)) <= 1e-9 * b["tau1"], k
        assert abs(b["tau2"] - abs(sy) / yy) <= 1e-9 * b["tau2"], k
        assert b["tau1"] >= b["tau2"], k
        want = {"alt": b["tau1"] if k % 2 == 1 else b["tau2"], "bb1": b["tau1"],
                "bb2": b["tau2"]}[prm.bb]
        want = min(max(want, prm.tau_min), prm.tau_max)
        assert b["tau_bb"] == want, (k, b["tau_bb"], want)
    assert hist[0]["tau_bb"] == prm.tau0


def check_reference(hist, eta):
    Es = [h["E"] for h in hist]
    for i, h in enumerate(hist):
        if eta == 0.0:
            assert h["C"] == h["E"] and h["Q"] == 1.0, i
        elif eta == 1.0:
            assert h["Q"] == i + 1.0, i
            assert abs(h["C"] - math.fsum(Es[: i + 1]) / (i + 1)) <= 1e-13 * abs(h["C"]), i


def _run(bb="alt", eta=0.85, iters=12):
    _, eg, X0 = _quadratic_problem()
    prm = optm.Params(bb=bb, eta=eta, eps_g=0.0, max_iter=iters, stagnation_tol=0.0)
    res = optm.minimize(eg, X0, prm, keep_iterates=True)
    return res.history, prm, eg


# ---- the pins ---------------------------------------------------------------------------

def test_bb_values_on_an_eigenvector_are_the_inverse_eigenvalue():
    check_eigenvector(optm.bb_candidates)


def test_bb_values_are_ordered_by_cauchy_schwarz():
    check_cauchy_schwarz(optm.bb_candidates)


def test_bb_step_hand_values_fallback_and_clamp():
    prm = optm.Params(tau0=1e-3)
    # ss = 4, sy = -2, yy = 4: tau_1 = 4/2 = 2, tau_2 = 2/4 = 0.5
    assert optm.bb_step(0, 4.0, -2.0, 4.0, prm) == 1e-3
    assert optm.bb_step(1, 4.0, -2.0, 4.0, prm) == 2.0
    assert optm.bb_step(2, 4.0, -2.0, 4.0, prm) == 0.5
    assert optm.bb_step(3, 4.0, -2.0, 4.0, prm) == 2.0
    assert optm.bb_step(2, 4.0, -2.0, 4.0, optm.Params(bb="bb1")) == 2.0
    assert optm.bb_step(1, 4.0, -2.0, 4.0, optm.Params(bb="bb2")) == 0.5
    # unusable values fall back to tau_0; finite ones are clamped
    assert optm.bb_step(1, 4.0, 0.0, 4.0, prm) == 1e-3
    assert optm.bb_step(2, 4.0, 1.0, 0.0, prm) == 1e-3
    assert optm.bb_step(1, 1e30, 1.0, 1.0, prm) == prm.tau_max
    assert optm.bb_step(2, 1.0, 1e-30, 1.0, prm) == prm.tau_min


@pytest.mark.parametrize("bb", ["alt", "bb1", "bb2"])
def test_bb_alternation_and_sums_along_a_run(bb):
    check_run(*_run(bb=bb))


@pytest.mark.parametrize("eta", [0.0, 1.0])
def test_reference_value_limits(eta):
    hist, _, _ = _run(eta=eta, iters=15)
    check_reference(hist, eta)


def test_reference_update_two_steps_by_hand():
    # C_0 = 5, Q_0 = 1, eta = 0.5: Q_1 = 1.5, C_1 = (0.5*5 + 2)/1.5 = 3; Q_2 = 1.75,
    # C_2 = (0.5*1.5*3 + 1)/1.75 = 3.25/1.75
    C, Q = optm.reference_update(5.0, 1.0, 2.0, 0.5)
    assert (C, Q) == (3.0, 1.5)
    C, Q = optm.reference_update(C, Q, 1.0, 0.5)
    assert Q == 1.75 and abs(C - 3.25 / 1.75) < 1e-15


# ---- mutations planted in the oracle must fail a pin ------------------------------------

_ORIG_CAND = optm.bb_candidates
_ORIG_BB_STEP = optm.bb_step


def _swapped(ss, sy, yy):
    t1, t2 = _ORIG_CAND(ss, sy, yy)
    return t2, t1


def _inverted_tau2(ss, sy, yy):
    t1, _ = _ORIG_CAND(ss, sy, yy)
    return t1, abs(sy) / ss


def _no_abs(ss, sy, yy):
    return ss / sy, sy / yy


def _bad_alternation(k, ss, sy, yy, p):
    q = optm.Params(**{**p.__dict__, "bb": "bb1" if k % 2 == 0 else "bb2"})
    return _ORIG_BB_STEP(max(k, 1), ss, sy, yy, q) if k > 0 else p.tau0


def _bad_weight(C, Q, E, eta):
    Qn = eta * Q + 1.0
    return (eta * C + E) / Qn, Qn


def _bad_q(C, Q, E, eta):
    Qn = eta + 1.0
    return (eta * Q * C + E) / Qn, Qn


@pytest.mark.parametrize("name", ["swapped", "inverted_tau2", "no_abs", "bad_alternation",
                                  "bad_weight", "bad_q"])
def test_planted_mistakes_fail_a_pin(name, monkeypatch):
    def all_pins():
        check_eigenvector(optm.bb_candidates)
        check_cauchy_schwarz(optm.bb_candidates)
        check_run(*_run())
        for eta in (0.0, 1.0):
            check_reference(_run(eta=eta, iters=15)[0], eta)

    all_pins()  # the unmutated oracle passes every pin
    mut = {"swapped": ("bb_candidates", _swapped), "inverted_tau2": ("bb_candidates", _inverted_tau2),
           "no_abs": ("bb_candidates", _no_abs), "bad_alternation": ("bb_step", _bad_alternation),
           "bad_weight": ("reference_update", _bad_weight), "bad_q": ("reference_update", _bad_q)}
    attr, fn = mut[name]
    monkeypatch.setattr(optm, attr, fn)
    with pytest.raises((AssertionError, ZeroDivisionError, FloatingPointError)):
        all_pins()
