"""Monopole boundary values for the Hartree potential of a finite cluster (oracle, FP64).

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__``).

The Hartree problem of Section 2.3 is posed on a box.  With a zero Dirichlet boundary the
box acts as a grounded conductor, which lowers the Hartree energy of a charged electron
cloud by roughly Q^2/(2R) -- for an aluminium cluster of hundreds of atoms far more than
its binding energy.  The free-space potential is V_0 + H, where V_0 is the zero-boundary
solution and H the harmonic function that takes the free-space values on the boundary.
To the monopole order those values are Q/|r_b - c| for the electron count Q and a centre c.
For a fixed Q (the constraint fixes the charge) the kernel k(r, r') = w(r) + w(r') - w(c),
with w the harmonic extension of 1/|r_b - c|, is the symmetric first-order form of the
boundary part of the Green's function, and it gives

    E_H = (1/2) int rho V_0 + Q int rho w - (1/2) Q^2 w(c),
    dE_H/drho = V_0 + Q w,

so the correction is a fixed potential V_bc = Q w added to the Hartree potential and a
constant -(1/2) Q V_bc(c) in the energy.  Both are computed once per system.

Discrete forms.  7-point grid: L w = b with b_g = sum over the face neighbours of g that lie
on the boundary layer (index -1 or N) of g(r_b)/h^2.  Q1 elements: A w = b with
b_k = -sum over boundary neighbours j of A_kj g(r_j) (edge neighbours h/6, corner
neighbours h/12, face neighbours 0).  V_bc(c) is the trilinear interpolation of the nodal
values at c.
"""
from __future__ import annotations

import itertools
import math

import numpy as np


def centre_of_charge(R, Z, lo, dims, h):
    """Nuclear-charge centre sum Z R / sum Z, or the box centre without nuclei."""
    R = np.asarray(R, dtype=np.float64).reshape(-1, 3)
    Z = np.asarray(Z, dtype=np.float64).ravel()
    if R.shape[0] == 0 or Z.sum() == 0.0:
        return np.array([lo[d] + 0.5 * (dims[d] + 1) * h for d in range(3)])
    return (Z[:, None] * R).sum(axis=0) / Z.sum()


def _coords(idx, lo, h):
    return lo + (np.asarray(idx, dtype=np.float64) + 1.0) * h


def boundary_rhs(nx, ny, nz, h, lo, Q, c, disc="fd7"):
    """Right-hand side b of the interior system for the boundary values Q/|r_b - c|."""
    lo = np.asarray(lo, dtype=np.float64)
    c = np.asarray(c, dtype=np.float64)
    dims = (nx, ny, nz)
    b = np.zeros((nz, ny, nx))

    def g(ix, iy, iz):
        r = _coords((ix, iy, iz), lo, h)
        return Q / float(np.linalg.norm(r - c))

    if disc == "fd7":
        offs = [(1, 0, 0), (-1, 0, 0), (0, 1, 0), (0, -1, 0), (0, 0, 1), (0, 0, -1)]
        weights = {o: 1.0 / h ** 2 for o in offs}
    else:
        offs, weights = [], {}
        for o in itertools.product((-1, 0, 1), repeat=3):
            cls = sum(1 for v in o if v != 0)
            if cls == 2:
                offs.append(o)
                weights[o] = h / 6.0
            elif cls == 3:
                offs.append(o)
                weights[o] = h / 12.0
    # only nodes next to the boundary have boundary neighbours
    for k in range(nz):
        for j in range(ny):
            for i in range(nx):
                if 0 < i < nx - 1 and 0 < j < ny - 1 and 0 < k < nz - 1:
                    continue
                acc = 0.0
                for o in offs:
                    a, bb, cc = i + o[0], j + o[1], k + o[2]
                    inside = 0 <= a < nx and 0 <= bb < ny and 0 <= cc < nz
                    if inside:
                        continue
                    acc += weights[o] * g(a, bb, cc)
                b[k, j, i] = acc
    del dims
    return b.ravel()


def point_value(w, nx, ny, nz, h, lo, c, Q, c_bc):
    """Trilinear interpolation at c of the nodal field w, with the boundary values
    Q/|r_b - c_bc| on the boundary layer."""
    lo = np.asarray(lo, dtype=np.float64)
    u = (np.asarray(c, dtype=np.float64) - lo) / h - 1.0  # fractional node index
    base = np.floor(u).astype(int)
    t = u - base
    W = np.asarray(w).reshape(nz, ny, nx)

    def val(i, j, k):
        if 0 <= i < nx and 0 <= j < ny and 0 <= k < nz:
            return float(W[k, j, i])
        r = _coords((i, j, k), lo, h)
        return Q / float(np.linalg.norm(r - np.asarray(c_bc)))

    out = 0.0
    for di, dj, dk in itertools.product((0, 1), repeat=3):
        wt = (t[0] if di else 1 - t[0]) * (t[1] if dj else 1 - t[1]) * (t[2] if dk else 1 - t[2])
        out += wt * val(base[0] + di, base[1] + dj, base[2] + dk)
    return out


def monopole_potential(solve, nx, ny, nz, h, lo, R, Z, Q, disc="fd7"):
    """(V_bc, E constant) for the electron count Q: V_bc = Q w solves the interior system
    with the boundary values Q/|r_b - c| (``solve(b)`` returns the solution of the
    discrete Laplace problem for the right-hand side b), E constant = -(1/2) Q V_bc(c)."""
    c = centre_of_charge(R, Z, lo, (nx, ny, nz), h)
    b = boundary_rhs(nx, ny, nz, h, lo, Q, c, disc)
    v = solve(b)
    vc = point_value(v, nx, ny, nz, h, lo, c, Q, c)
    return v, -0.5 * Q * vc, c


def gaussian_self_energy(Q, sigma):
    """Coulomb self-energy of a spherical Gaussian charge: Q^2 / (2 sqrt(pi) sigma)."""
    return Q * Q / (2.0 * math.sqrt(math.pi) * sigma)
