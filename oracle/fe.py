"""Trilinear (Q1) finite elements with the B-orthonormality constraint (oracle, FP64).

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__``).

Section 2.3 discretises with finite elements: orbitals are coefficient vectors of a
nodal basis {u_k}, the mass matrix is B_kl = int u_k u_l, and the constraint becomes
c^T B c = 1 (eq. (disOFinf)); Section 3 maps it to the unit sphere by y = B^{1/2} c
(eq. (OFDFT-y)).  For p orbitals the same substitution Y = B^{1/2} X turns
X^T B X = I into Y^T Y = I.  What is built here:

* Mesh: the interior nodes of the uniform grid (same coordinates and index order as
  the finite-difference grid), trilinear basis on the cubes of side h, zero Dirichlet
  boundary.
* With the 1D linear-element matrices K = (1/h) tridiag(-1, 2, -1) and
  M = (h/6) tridiag(1, 4, 1) (kron order z, y, x, x fastest):
      B = M (x) M (x) M,      A = K (x) M (x) M + M (x) K (x) M + M (x) M (x) K,
  so A_kl = int grad u_k . grad u_l and B_kl = int u_k u_l.
* Potential terms use nodal quadrature with weights h^3 (the paper leaves the
  quadrature open): rho_k = f sum_i X_ki^2, E_ext = h^3 sum V_ext rho,
  A V_H = 4 pi h^3 rho (weak form of the Poisson equation), E_H = (h^3/2) rho^T V_H,
  E_x = h^3 sum rho eps_x(rho).
* E = (f/2) tr(X^T A X) + E_ext + E_H + E_x + E_II, whose exact partial derivative is
      E_X = 2 f [ (1/2) A X + h^3 Diag(V_ext + V_H + v_x) X ].
* The manifold X^T B X = I is handled in the B metric, i.e. every formula of Section 3
  with Y = B^{1/2} X substituted (``BStiefel``):
      grad E = B^{-1} E_X - X (E_X^T X),       <U, W> = tr(U^T B W),
      QR:  Y = X - tau grad E,  Y^T B Y = R^T R,  X+ = Y R^{-1},
      WY:  X+ = X - tau U (I + tau/2 N)^{-1} [X^T B X; -E_X^T X],  U = [B^{-1}E_X, X],
           N = [[X^T E_X, X^T B X], [-E_X^T B^{-1} E_X, -E_X^T X]].
  With B = I all of this is the Euclidean method of Section 3.
"""
from __future__ import annotations

import math

import numpy as np
import scipy.linalg as sla
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from .fd import FDGrid, e_nuclear, v_ext_erf
from .ks import C_TF, CV, CX, Energy, eps_c_rs, pz_rs, v_c_rs


def k1d(m, h):
    """1D stiffness (1/h) tridiag(-1, 2, -1) on m interior nodes."""
    return sp.diags([-np.ones(m - 1), 2.0 * np.ones(m), -np.ones(m - 1)], [-1, 0, 1]) / h


def m1d(m, h):
    """1D consistent mass (h/6) tridiag(1, 4, 1) on m interior nodes."""
    return sp.diags([np.ones(m - 1), 4.0 * np.ones(m), np.ones(m - 1)], [-1, 0, 1]) * (h / 6.0)


def q1_matrices(nx, ny, nz, h):
    """CSR stiffness A and mass B of the Q1 elements (index g = i + nx (j + ny k))."""
    Kx, Ky, Kz = k1d(nx, h), k1d(ny, h), k1d(nz, h)
    Mx, My, Mz = m1d(nx, h), m1d(ny, h), m1d(nz, h)
    B = sp.kron(Mz, sp.kron(My, Mx, format="csr"), format="csr")
    A = (sp.kron(Kz, sp.kron(My, Mx, format="csr"), format="csr")
         + sp.kron(Mz, sp.kron(Ky, Mx, format="csr"), format="csr")
         + sp.kron(Mz, sp.kron(My, Kx, format="csr"), format="csr"))
    A, B = A.tocsr(), B.tocsr()
    for m in (A, B):
        m.sum_duplicates()
        m.eliminate_zeros()
    return A, B


def q1_generalized_eigenvalues(nx, ny, nz, h):
    """All eigenvalues of A v = lambda B v: sum over axes of (6/h^2)(1-cos t)/(2+cos t)."""
    def axis(m):
        t = np.arange(1, m + 1) * math.pi / (m + 1)
        return (6.0 / h ** 2) * (1.0 - np.cos(t)) / (2.0 + np.cos(t))
    lx, ly, lz = axis(nx), axis(ny), axis(nz)
    return (lz[:, None, None] + ly[None, :, None] + lx[None, None, :]).ravel()


class KSSystemQ1:
    """One synthetic Kohn-Sham system discretised by Q1 finite elements."""

    def __init__(self, nx, ny, nz, h, lo, p, R, Z, f=2.0, rc=0.5, ext=True, hartree=True,
                 xc=True, v_ext_override=None, hartree_tol=1e-14, hartree_maxit=20000,
                 corr=False, mu=1.0, tf=False, vext="erf", hartree_bc="zero"):
        self.grid = FDGrid(nx, ny, nz, h, lo)
        self.use_corr = bool(corr)
        # orbital-free (TFW, Section 2.2): von Weizsaecker weight mu on the stiffness term
        # and the Thomas-Fermi term C_TF int rho^{5/3} (nodal quadrature)
        self.mu = float(mu)
        self.use_tf = bool(tf)
        self.n = self.grid.n
        self.p = int(p)
        self.f = float(f)
        self.h3 = self.grid.h ** 3
        self.A, self.B = q1_matrices(nx, ny, nz, h)
        self._Blu = None  # sparse LU of B, built on the first mass solve
        R = np.asarray(R, dtype=np.float64).reshape(-1, 3)
        Z = np.asarray(Z, dtype=np.float64).ravel()
        self.use_hartree, self.use_xc = bool(hartree), bool(xc)
        if v_ext_override is not None:
            self.v_ext = np.asarray(v_ext_override, dtype=np.float64).copy()
            self.e_ii = 0.0
        elif ext and vext == "gnh":
            from .gnh import v_ext_gnh
            self.v_ext = v_ext_gnh(self.grid.coords(), R, Z)
            self.e_ii = e_nuclear(R, Z)
        elif ext:
            self.v_ext = v_ext_erf(self.grid.coords(), R, Z, float(rc))
            self.e_ii = e_nuclear(R, Z)
        else:
            self.v_ext = np.zeros(self.n)
            self.e_ii = 0.0
        self.hartree_tol = float(hartree_tol)
        self.hartree_maxit = int(hartree_maxit)
        # Hartree boundary: zero Dirichlet, or the monopole values of the electron count
        self.v_bc, self.e_bc = np.zeros(self.n), 0.0
        if hartree_bc == "monopole" and self.use_hartree:
            from .boundary import monopole_potential
            self.v_bc, self.e_bc, _ = monopole_potential(
                lambda b: self.hartree_cg(b / (4.0 * math.pi * self.h3))[0], nx, ny, nz, h,
                lo, R, Z, self.f * self.p, "q1")
        elif hartree_bc not in ("zero", "monopole"):
            raise ValueError(hartree_bc)

    def density(self, X):
        """Nodal density rho_k = f sum_i X_ki^2."""
        return self.f * np.einsum("gi,gi->g", X, X)

    def mass_solve(self, G):
        """B^{-1} G (sparse LU of B)."""
        if self._Blu is None:
            self._Blu = spla.splu(self.B.tocsc())
        return self._Blu.solve(np.asarray(G, dtype=np.float64))

    def hartree_cg(self, rho, v0=None):
        """Conjugate gradients on A v = 4 pi h^3 rho to ||r|| <= tol ||b||, warm start."""
        b = 4.0 * math.pi * self.h3 * rho
        bnorm = math.sqrt(float(b @ b))
        if bnorm == 0.0:
            return np.zeros_like(b), 0, 0.0
        x = np.zeros_like(b) if v0 is None else np.array(v0, dtype=np.float64)
        r = b - self.A @ x
        rr = float(r @ r)
        d = r.copy()
        it = 0
        while math.sqrt(rr) > self.hartree_tol * bnorm and it < self.hartree_maxit:
            q = self.A @ d
            alpha = rr / float(d @ q)
            x += alpha * d
            r -= alpha * q
            rr_new = float(r @ r)
            d = r + (rr_new / rr) * d
            rr = rr_new
            it += 1
        return x, it, math.sqrt(rr) / bnorm

    def energy_terms(self, X, vh0=None):
        h3 = self.h3
        rho = self.density(X)
        kinetic = 0.5 * self.mu * self.f * float(np.sum(X * (self.A @ X)))
        if self.use_tf:
            kinetic += h3 * C_TF * float(np.sum(rho ** (5.0 / 3.0)))
        external = h3 * float(self.v_ext @ rho)
        if self.use_hartree:
            vh, it, rel = self.hartree_cg(rho, vh0)
            hartree = 0.5 * h3 * float(rho @ vh) + h3 * float(rho @ self.v_bc) + self.e_bc
        else:
            vh, it, rel, hartree = np.zeros(self.n), 0, 0.0, 0.0
        if self.use_xc:
            vx = -CV * np.cbrt(rho)
            exc = h3 * float(rho @ (-CX * np.cbrt(rho)))
        else:
            vx, exc = np.zeros(self.n), 0.0
        if self.use_corr:
            rs = pz_rs(rho)
            vx = vx + v_c_rs(rs)
            exc += h3 * float(rho @ eps_c_rs(rs))
        if self.use_tf:
            vx = vx + (5.0 / 3.0) * C_TF * np.cbrt(rho) ** 2
        total = kinetic + external + hartree + exc + self.e_ii
        return Energy(total, kinetic, external, hartree, exc, self.e_ii, it, rel), rho, vh, vx

    def energy_grad(self, X, vh0=None):
        """Returns (Energy, E_X, V_H)."""
        en, rho, vh, vx = self.energy_terms(X, vh0)
        veff = self.v_ext + vh + self.v_bc + vx
        G = 2.0 * self.f * (0.5 * self.mu * (self.A @ X) + self.h3 * veff[:, None] * X)
        return en, G, vh

    def energy(self, X, vh0=None):
        return self.energy_terms(X, vh0)[0].total

    def hamiltonian(self, veff):
        """Sparse H = 1/2 A + h^3 Diag(veff): E_X = 2 f H X and H X = B X Lambda at a minimiser."""
        return (0.5 * self.mu * self.A + self.h3 * sp.diags(veff)).tocsr()

    def effective_potential(self, X, vh0=None):
        en, rho, vh, vx = self.energy_terms(X, vh0)
        return self.v_ext + vh + self.v_bc + vx


class BStiefel:
    """The constraint X^T B X = I in the B metric (Section 3 with Y = B^{1/2} X)."""

    def __init__(self, B, mass_solve):
        self.B = B
        self.solve = mass_solve

    def grad(self, X, G):
        return self.solve(G) - X @ (G.T @ X)

    def inner(self, U, W):
        return float(np.sum(U * (self.B @ W)))

    def cholqr(self, Y):
        R = sla.cholesky(Y.T @ (self.B @ Y), lower=False)
        return sla.solve_triangular(R, Y.T, trans="T", lower=False).T

    def retract(self, kind, X, G, tau):
        if kind == "qr":
            return self.cholqr(X - tau * self.grad(X, G))
        p = X.shape[1]
        Gt = self.solve(G)
        XBX = X.T @ (self.B @ X)
        XG = X.T @ G
        N = np.block([[XG, XBX], [-(G.T @ Gt), -XG.T]])
        rhs = np.vstack([XBX, -XG.T])
        U = np.hstack([Gt, X])
        return X - tau * (U @ np.linalg.solve(np.eye(2 * p) + 0.5 * tau * N, rhs))

    def orth_error(self, X):
        return float(np.linalg.norm(X.T @ (self.B @ X) - np.eye(X.shape[1])))

    def reorth(self, X):
        return self.cholqr(X)


def b_orthonormalize(B, X):
    """X R^{-1} with X^T B X = R^T R (start blocks for the B constraint)."""
    R = sla.cholesky(X.T @ (B @ X), lower=False)
    return sla.solve_triangular(R, X.T, trans="T", lower=False).T
