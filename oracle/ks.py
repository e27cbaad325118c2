"""Discrete Kohn-Sham energy and its partial derivative on the uniform grid (oracle, FP64).

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__``).

Definitions (Section 2.1 eq. (EKS), Section 2.3 discrete energy and eq. (partial deriv)),
with the readings needed to make the printed formulas consistent:

* Orbitals are normalised by X^T X = I, so the continuous orbital at grid point g is
  phi_i(r_g) = X_gi h^{-3/2} and integrals are h^3 times grid sums.  With occupation
  f per orbital the density is rho_g = (f/h^3) sum_i X_gi^2 (the paper's
  rho = diag(XX^T) up to this scale).
* The Hartree potential solves L V_H = 4 pi rho with L = -Laplacian_h and zero
  Dirichlet boundary (the paper's "L^dagger rho" without its 4 pi); it is computed
  by conjugate gradients started from the previous potential.
* Exchange-correlation is the Slater (Dirac) local exchange, spin unpolarised:
  eps_x(rho) = -(3/4)(3/pi)^{1/3} rho^{1/3},  v_x = d(rho eps_x)/d rho; optionally
  (``corr=True``) plus LDA correlation in the Perdew-Zunger (1981) parametrisation of the
  Ceperley-Alder electron gas, unpolarised: with r_s = (3/(4 pi rho))^{1/3},
  eps_c = gamma/(1 + beta1 sqrt(r_s) + beta2 r_s) for r_s >= 1 and
  eps_c = A ln r_s + B + C r_s ln r_s + D r_s for r_s < 1, v_c = d(rho eps_c)/d rho
  = eps_c - (r_s/3) d eps_c/d r_s.
* E = (f/2) tr(X^T L X) + h^3 sum V_ext rho + (h^3/2) rho^T V_H
      + h^3 sum rho eps_x(rho) + E_II.
* The exact partial derivative of that E is
      E_X = 2 f [ (1/2) L X + Diag(V_ext + V_H + v_x) X ],
  i.e. the paper's H(X)X with the factor 2f that its normalisation leaves implicit.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

from .fd import FDGrid, e_nuclear, v_ext_erf

CX = 0.75 * (3.0 / math.pi) ** (1.0 / 3.0)   # eps_x = -CX rho^{1/3}
CV = (3.0 / math.pi) ** (1.0 / 3.0)          # v_x  = -CV rho^{1/3}

# Thomas-Fermi kinetic energy density of Section 2.2 eq. (TFW): C_TF rho^{5/3}
C_TF = 0.3 * (3.0 * math.pi ** 2) ** (2.0 / 3.0)

# Perdew-Zunger (1981) unpolarised correlation constants
PZ_GAMMA, PZ_BETA1, PZ_BETA2 = -0.1423, 1.0529, 0.3334
PZ_A, PZ_B, PZ_C, PZ_D = 0.0311, -0.048, 0.0020, -0.0116


def pz_rs(rho):
    """Wigner-Seitz radius r_s = (3/(4 pi rho))^{1/3} (inf where rho = 0)."""
    rho = np.asarray(rho, dtype=np.float64)
    with np.errstate(divide="ignore"):
        return np.where(rho > 0.0, np.cbrt(3.0 / (4.0 * math.pi * np.where(rho > 0.0, rho, 1.0))),
                        np.inf)


def eps_c_rs(rs):
    """Correlation energy per electron as a function of r_s (both branches)."""
    rs = np.asarray(rs, dtype=np.float64)
    hi = rs < 1.0
    zero = np.isinf(rs)                 # rho = 0: no correlation energy
    r = np.where(hi | zero, 1.0, rs)    # low-density branch argument
    q = np.where(hi, rs, 1.0)           # high-density branch argument
    low = np.where(zero, 0.0, PZ_GAMMA / (1.0 + PZ_BETA1 * np.sqrt(r) + PZ_BETA2 * r))
    lnq = np.log(q)
    high = PZ_A * lnq + PZ_B + PZ_C * q * lnq + PZ_D * q
    return np.where(hi, high, low)


def v_c_rs(rs):
    """v_c = eps_c - (r_s/3) d eps_c/d r_s, the derivative written out per branch."""
    rs = np.asarray(rs, dtype=np.float64)
    hi = rs < 1.0
    zero = np.isinf(rs)
    r = np.where(hi | zero, 1.0, rs)
    q = np.where(hi, rs, 1.0)
    den = 1.0 + PZ_BETA1 * np.sqrt(r) + PZ_BETA2 * r
    low = np.where(zero, 0.0,
                   PZ_GAMMA * (1.0 + (7.0 / 6.0) * PZ_BETA1 * np.sqrt(r)
                               + (4.0 / 3.0) * PZ_BETA2 * r) / (den * den))
    lnq = np.log(q)
    high = (PZ_A * lnq + (PZ_B - PZ_A / 3.0) + (2.0 / 3.0) * PZ_C * q * lnq
            + (2.0 * PZ_D - PZ_C) / 3.0 * q)
    return np.where(hi, high, low)


@dataclasses.dataclass
class Energy:
    total: float
    kinetic: float
    external: float
    hartree: float
    xc: float
    nuclear: float
    cg_iters: int = 0
    cg_relres: float = 0.0


class KSSystemFD:
    """One synthetic Kohn-Sham system on a uniform grid.

    Arguments are plain numbers/arrays: grid (nx, ny, nz, h, lo), orbitals p,
    occupation f, nuclei R (M,3) and Z (M,), smoothing radius rc, and switches for
    the external, Hartree and exchange terms.  ``v_ext_override`` replaces the
    nuclear potential by a given grid vector (used for closed-form checks).
    """

    def __init__(self, nx, ny, nz, h, lo, p, R, Z, f=2.0, rc=0.5, ext=True, hartree=True,
                 xc=True, v_ext_override=None, hartree_tol=1e-14, hartree_maxit=20000,
                 corr=False, mu=1.0, tf=False, vext="erf", hartree_bc="zero"):
        self.grid = FDGrid(nx, ny, nz, h, lo)
        self.n = self.grid.n
        self.p = int(p)
        self.f = float(f)
        self.R = np.asarray(R, dtype=np.float64).reshape(-1, 3)
        self.Z = np.asarray(Z, dtype=np.float64).ravel()
        self.rc = float(rc)
        self.use_ext, self.use_hartree, self.use_xc = bool(ext), bool(hartree), bool(xc)
        self.use_corr = bool(corr)
        # orbital-free (TFW, Section 2.2): von Weizsaecker weight mu on the kinetic term and
        # the Thomas-Fermi term C_TF int rho^{5/3}
        self.mu = float(mu)
        self.use_tf = bool(tf)
        if v_ext_override is not None:
            self.v_ext = np.asarray(v_ext_override, dtype=np.float64).copy()
            self.e_ii = 0.0
        elif self.use_ext and vext == "gnh":
            from .gnh import v_ext_gnh
            self.v_ext = v_ext_gnh(self.grid.coords(), self.R, self.Z)
            self.e_ii = e_nuclear(self.R, self.Z)
        elif self.use_ext:
            self.v_ext = v_ext_erf(self.grid.coords(), self.R, self.Z, self.rc)
            self.e_ii = e_nuclear(self.R, self.Z)
        else:
            self.v_ext = np.zeros(self.n)
            self.e_ii = 0.0
        self.hartree_tol = float(hartree_tol)
        self.hartree_maxit = int(hartree_maxit)
        # Hartree boundary: zero Dirichlet, or the monopole values of the electron count
        # (oracle/boundary.py): a fixed potential v_bc and an energy constant e_bc
        self.v_bc, self.e_bc = np.zeros(self.n), 0.0
        if hartree_bc == "monopole" and self.use_hartree:
            from .boundary import monopole_potential
            self.v_bc, self.e_bc, _ = monopole_potential(
                lambda b: self.hartree_cg(b / (4.0 * math.pi))[0], nx, ny, nz, h, lo,
                self.R, self.Z, self.f * self.p, "fd7")
        elif hartree_bc not in ("zero", "monopole"):
            raise ValueError(hartree_bc)

    # -- density (Section 2.3: rho(X) = diag(X X^T)) --------------------------------------
    def density(self, X):
        return (self.f / self.grid.dV) * np.einsum("gi,gi->g", X, X)

    # -- Hartree: L V_H = 4 pi rho by CG, warm start --------------------------------------
    def hartree_cg(self, rho, v0=None):
        """Conjugate gradients on L v = 4 pi rho, stopped when ||r||_2 <= tol ||4 pi rho||_2."""
        b = 4.0 * math.pi * rho
        bnorm = math.sqrt(float(b @ b))
        x = np.zeros_like(b) if v0 is None else np.array(v0, dtype=np.float64)
        if bnorm == 0.0:
            return np.zeros_like(b), 0, 0.0
        r = b - self.grid.lap(x)
        rr = float(r @ r)
        d = r.copy()
        it = 0
        while math.sqrt(rr) > self.hartree_tol * bnorm and it < self.hartree_maxit:
            q = self.grid.lap(d)
            alpha = rr / float(d @ q)
            x += alpha * d
            r -= alpha * q
            rr_new = float(r @ r)
            d = r + (rr_new / rr) * d
            rr = rr_new
            it += 1
        return x, it, math.sqrt(rr) / bnorm

    # -- Slater exchange ------------------------------------------------------------------
    @staticmethod
    def eps_x(rho):
        return -CX * np.cbrt(rho)

    @staticmethod
    def v_x(rho):
        return -CV * np.cbrt(rho)

    @staticmethod
    def eps_c(rho):
        return eps_c_rs(pz_rs(rho))

    @staticmethod
    def v_c(rho):
        return v_c_rs(pz_rs(rho))

    # -- energy and gradient ----------------------------------------------------------------
    def energy_terms(self, X, vh0=None):
        """Returns (Energy, rho, V_H, v_x)."""
        dV = self.grid.dV
        rho = self.density(X)
        kinetic = 0.5 * self.mu * self.f * float(np.sum(X * self.grid.lap(X)))
        if self.use_tf:
            kinetic += dV * C_TF * float(np.sum(rho ** (5.0 / 3.0)))
        external = dV * float(self.v_ext @ rho)
        if self.use_hartree:
            vh, it, rel = self.hartree_cg(rho, vh0)
            hartree = 0.5 * dV * float(rho @ vh) + dV * float(rho @ self.v_bc) + self.e_bc
        else:
            vh, it, rel, hartree = np.zeros(self.n), 0, 0.0, 0.0
        if self.use_xc:
            vx = self.v_x(rho)
            exc = dV * float(rho @ self.eps_x(rho))
        else:
            vx, exc = np.zeros(self.n), 0.0
        if self.use_corr:
            vx = vx + self.v_c(rho)
            exc += dV * float(rho @ self.eps_c(rho))
        if self.use_tf:
            vx = vx + (5.0 / 3.0) * C_TF * np.cbrt(rho) ** 2
        total = kinetic + external + hartree + exc + self.e_ii
        return Energy(total, kinetic, external, hartree, exc, self.e_ii, it, rel), rho, vh, vx

    def energy_grad(self, X, vh0=None):
        """Returns (Energy, G = E_X, V_H)."""
        en, rho, vh, vx = self.energy_terms(X, vh0)
        veff = self.v_ext + vh + self.v_bc + vx
        G = 2.0 * self.f * (0.5 * self.mu * self.grid.lap(X) + veff[:, None] * X)
        return en, G, vh

    def energy(self, X, vh0=None):
        return self.energy_terms(X, vh0)[0].total

    def hamiltonian_apply(self, X, veff):
        """H X with H = mu/2 L + Diag(veff)  (no 2f factor)."""
        return 0.5 * self.mu * self.grid.lap(X) + veff[:, None] * X

    def effective_potential(self, X, vh0=None):
        en, rho, vh, vx = self.energy_terms(X, vh0)
        return self.v_ext + vh + self.v_bc + vx
