"""Uniform-grid finite-difference discretisation (oracle, FP64).

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__``).

Readings of the paper used here:

* Section 2.3 calls L "an approximation to the Laplacian" but uses it with a
  kinetic energy of +1/2 tr(X^T L X); the only reading with a positive kinetic
  energy is L = -Laplacian_h, i.e. (Lu)_g = (6 u_g - sum of the 6 neighbours)/h^2,
  with u = 0 outside the interior grid (zero Dirichlet boundary).
* The external potential of the synthetic systems is the Coulomb potential of
  point charges smoothed by erf with radius r_c (the paper's pseudopotentials
  are not available); the nuclear repulsion E_II of eq. (EKS) is the bare
  Coulomb sum over pairs.
"""
from __future__ import annotations

import math

import numpy as np
from scipy.special import erf


class FDGrid:
    """Interior grid nx*ny*nz with spacing h; point (i,j,k) at lo + (i+1, j+1, k+1) h.

    Linear index g = i + nx*(j + ny*k); numpy arrays of grid values are reshaped to
    (nz, ny, nx) so that x is the fastest axis.
    """

    def __init__(self, nx, ny, nz, h, lo):
        self.nx, self.ny, self.nz = int(nx), int(ny), int(nz)
        self.h = float(h)
        self.lo = tuple(float(v) for v in lo)
        self.n = self.nx * self.ny * self.nz
        self.dV = self.h ** 3

    def coords(self):
        """(n, 3) coordinates of the interior points in linear-index order."""
        x = self.lo[0] + (np.arange(self.nx) + 1) * self.h
        y = self.lo[1] + (np.arange(self.ny) + 1) * self.h
        z = self.lo[2] + (np.arange(self.nz) + 1) * self.h
        Zc, Yc, Xc = np.meshgrid(z, y, x, indexing="ij")
        return np.stack([Xc.ravel(), Yc.ravel(), Zc.ravel()], axis=1)

    def lap(self, U):
        """L U with L = -Laplacian_h (7 points, zero Dirichlet).  U: (n,) or (n, p)."""
        vec = U.ndim == 1
        p = 1 if vec else U.shape[1]
        u = U.reshape(self.nz, self.ny, self.nx, p)
        out = 6.0 * u
        out[:, :, 1:, :] -= u[:, :, :-1, :]
        out[:, :, :-1, :] -= u[:, :, 1:, :]
        out[:, 1:, :, :] -= u[:, :-1, :, :]
        out[:, :-1, :, :] -= u[:, 1:, :, :]
        out[1:, :, :, :] -= u[:-1, :, :, :]
        out[:-1, :, :, :] -= u[1:, :, :, :]
        out /= self.h ** 2
        return out.reshape(U.shape)

    def lap_eigenvalues_1d(self, m):
        """Eigenvalues of the 1D Dirichlet second-difference matrix (2 - 2cos)/h^2 on m points."""
        k = np.arange(1, m + 1)
        return (2.0 - 2.0 * np.cos(k * math.pi / (m + 1))) / self.h ** 2


def v_ext_erf(coords, R, Z, rc):
    """V_ext(r) = sum_a -Z_a erf(|r-R_a|/r_c)/|r-R_a|  (limit -Z_a 2/(sqrt(pi) r_c) at r = R_a)."""
    v = np.zeros(coords.shape[0])
    for a in range(R.shape[0]):
        d = np.sqrt(((coords - R[a]) ** 2).sum(axis=1))
        small = d < 1e-6
        dd = np.where(small, 1.0, d)
        term = erf(dd / rc) / dd
        # Taylor expansion of erf(d/rc)/d about d = 0
        term = np.where(small, (2.0 / (math.sqrt(math.pi) * rc)) * (1.0 - d * d / (3.0 * rc * rc)), term)
        v -= Z[a] * term
    return v


def e_nuclear(R, Z):
    """E_II = 1/2 sum_{i != j} Z_i Z_j / |R_i - R_j| (eq. (EKS))."""
    e = 0.0
    for a in range(R.shape[0]):
        for b in range(a + 1, R.shape[0]):
            e += Z[a] * Z[b] / math.sqrt(float(((R[a] - R[b]) ** 2).sum()))
    return e
