"""Stiefel-manifold gradient and retractions (oracle, FP64).

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__``).

* Manifold gradient, Section 3 eq. (def-nablaE):  grad E = E_X - X E_X^T X.
* QR retraction, eq. (QR) with Alg. 2 (Cholesky QR): Y = X - tau grad E (eq. (def-Y)),
  Y^T Y = R^T R with R upper triangular with positive diagonal, X+ = Y R^{-1}.
  (Alg. 2 prints "Q = Y L^{-1}" for Y^T Y = L L^T; the dimensionally consistent
  reading is Q = Y L^{-T} = Y R^{-1}, which is the unique QR factor with positive
  diagonal R.)
* Cayley retraction, eq. (WY3): X+ = X - tau U (I + tau/2 V^T U)^{-1} V^T X with
  U = [E_X, X], V = [X, -E_X], the 2p x 2p system solved by LU with partial pivoting.
* The dense form eq. (WY1) and the p = 1 closed form eq. (WY-1d) are provided for
  the checks only.
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as sla


def manifold_grad(X, G):
    """grad E = G - X G^T X."""
    return G - X @ (G.T @ X)


def cholesky_upper(A):
    """Upper triangular R with R^T R = A (positive diagonal)."""
    return sla.cholesky(A, lower=False)


def cholqr(Y):
    """Alg. 2: Q = Y R^{-1} with Y^T Y = R^T R."""
    R = cholesky_upper(Y.T @ Y)
    return sla.solve_triangular(R, Y.T, trans="T", lower=False).T, R


def retract_qr(X, G, tau):
    """eq. (QR): X_QR(tau) = qr(X - tau grad E)."""
    Y = X - tau * manifold_grad(X, G)
    Q, _ = cholqr(Y)
    return Q


def retract_wy(X, G, tau):
    """eq. (WY3): X - tau U (I + tau/2 V^T U)^{-1} V^T X, U = [G, X], V = [X, -G]."""
    p = X.shape[1]
    U = np.hstack([G, X])
    V = np.hstack([X, -G])
    A = np.eye(2 * p) + 0.5 * tau * (V.T @ U)
    lu = sla.lu_factor(A)
    return X - tau * (U @ sla.lu_solve(lu, V.T @ X))


def retract_wy_dense(X, G, tau):
    """eq. (WY1): (I + tau/2 W)^{-1} (I - tau/2 W) X with W = G X^T - X G^T (n x n; tiny n only)."""
    n = X.shape[0]
    W = G @ X.T - X @ G.T
    return np.linalg.solve(np.eye(n) + 0.5 * tau * W, (np.eye(n) - 0.5 * tau * W) @ X)


def orth_error(X):
    """||X^T X - I||_F."""
    return float(np.linalg.norm(X.T @ X - np.eye(X.shape[1])))
