"""The BB sums of a QR trial formed without a pass over X_k (CPU check of the identity the
device summary uses; Section 3 eq. (bb-1) with the retraction of eq. (QR) and Alg. 2).

For a trial X_t = (X_k - tau D_k) R^{-1} with R^T R = (X_k - tau D_k)^T (X_k - tau D_k), the
step s = X_t - X_k equals X_t (I - R) - tau D_k, so with y = D_t - D_k

    <s, y>   = sum_ij (I - R)_ij (X_t^T D_t)_ij - tau <D_k, D_t> - <s, D_k>
    ||y||^2  = ||D_t||^2 - 2 <D_k, D_t> + ||D_k||^2

where ||s||^2 and <s, D_k> are the sums the retraction pass forms (it holds X_k, D_k and
X_t) and <D_k, D_t> the one the gradient pass forms (it holds D_k and D_t).  These tests
compare the assembled values with the definitions, in FP64, on a tangent direction (the
projected gradient of a quadratic energy, as Alg. 3 uses) and on a general one, over a
range of step sizes.
"""
import numpy as np
import pytest


def _orthonormal(n, p, rng):
    q, _ = np.linalg.qr(rng.standard_normal((n, p)))
    return q


def _projected(G, X):
    return G - X @ (G.T @ X)


def _qr_trial(X, D, tau):
    Y = X - tau * D
    R = np.linalg.cholesky(Y.T @ Y).T  # upper, Y^T Y = R^T R
    return np.linalg.solve(R.T, Y.T).T, R  # Y R^{-1}


def _assembled(X, D, Xt, Dt, R, tau):
    s = Xt - X
    ss = float(np.sum(s * s))          # retraction pass
    sdk = float(np.sum(s * D))         # retraction pass
    cr = float(np.sum(D * Dt))         # gradient pass
    dd = float(np.sum(Dt * Dt))        # gradient pass
    p = X.shape[1]
    sy = float(np.sum((np.eye(p) - R) * (Xt.T @ Dt))) - tau * cr - sdk
    yy = dd - 2.0 * cr + float(np.sum(D * D))
    return ss, sy, yy


@pytest.mark.parametrize("tau", [1e-3, 0.05, 0.4, 2.0])
@pytest.mark.parametrize("tangent", [True, False])
def test_bb_sums_match_definitions(tau, tangent):
    """tangent: D_k and D_t are projected gradients of a symmetric energy (X^T D = 0, as in
    Alg. 3, where the (I - R) term vanishes); otherwise general matrices, which exercise it."""
    rng = np.random.default_rng(7)
    n, p = 300, 8
    A = rng.standard_normal((n, n))
    A = A + A.T
    X = _orthonormal(n, p, rng)
    D = _projected(2.0 * A @ X, X) if tangent else rng.standard_normal((n, p))
    Xt, R = _qr_trial(X, D, tau)
    Dt = _projected(2.0 * A @ Xt, Xt) if tangent else rng.standard_normal((n, p))
    ss, sy, yy = _assembled(X, D, Xt, Dt, R, tau)
    s, y = Xt - X, Dt - D
    scale = np.linalg.norm(s) * (np.linalg.norm(Dt) + np.linalg.norm(D))
    assert ss == pytest.approx(float(np.sum(s * s)), rel=1e-13)
    assert abs(sy - float(np.sum(s * y))) <= 1e-12 * scale
    assert abs(yy - float(np.sum(y * y))) <= 1e-12 * (np.linalg.norm(Dt) + np.linalg.norm(D)) ** 2


def test_bb_sums_detect_a_wrong_factor():
    """The identity needs the factor of this trial: R^T (the lower factor) or the factor of
    another step size gives a different <s, y>.  (General matrices D_k, D_t: for projected
    gradients of a symmetric energy X_t^T D_t = 0 and the (I - R) term drops out.)"""
    rng = np.random.default_rng(3)
    n, p, tau = 200, 6, 0.3
    X = _orthonormal(n, p, rng)
    D = rng.standard_normal((n, p))
    Xt, R = _qr_trial(X, D, tau)
    Dt = rng.standard_normal((n, p))
    s, y = Xt - X, Dt - D
    exact = float(np.sum(s * y))
    _, sy_ok, _ = _assembled(X, D, Xt, Dt, R, tau)
    _, sy_lower, _ = _assembled(X, D, Xt, Dt, R.T, tau)
    _, R_other = _qr_trial(X, D, 0.5 * tau)
    _, sy_other, _ = _assembled(X, D, Xt, Dt, R_other, tau)
    assert abs(sy_ok - exact) <= 1e-10 * abs(exact)
    assert abs(sy_lower - exact) > 1e-6 * abs(exact)
    assert abs(sy_other - exact) > 1e-6 * abs(exact)
