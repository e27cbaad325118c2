"""Alg. 4 with uniform refinement (coarse-to-fine warm start) — oracle, FP64.

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__``).

Alg. 4 solves the discrete problem on a sequence of meshes, each level started from the
solution of the next coarser one carried over to the finer mesh.  Marking by an a
posteriori error estimator is not part of this build: every level refines the previous
one uniformly, the variant of Table 5.

Nested meshes.  A level with N interior nodes per axis and spacing h on a box whose first
node sits at lo + h refines to 2N + 1 nodes with spacing h/2 on the same box, so coarse
node i is fine node 2i + 1 and every even fine index lies half-way between two coarse
nodes (index -1 and N being the zero boundary).

Carrying a block over (``prolong``).  Trilinear interpolation of the nodal values.  For Q1
elements this is exact: the coarse finite-element function is an element of the finer
space, so it is the same function (the same B- and A-products).  For the 7-point grid the
interpolated values are rescaled by (h_f/h_c)^{3/2} = 2^{-3/2}, the change of
phi = X h^{-3/2} (Section 2.3 normalisation), and the block is orthonormalised by
Cholesky QR (Alg. 2), in the B metric for elements.
"""
from __future__ import annotations

import math

import numpy as np

from . import optm, stiefel


def _axis_weights(N):
    """(2N+1) x N matrix of the 1D linear interpolation between nested levels."""
    P = np.zeros((2 * N + 1, N))
    for i in range(N):
        P[2 * i + 1, i] = 1.0          # coarse node i itself
        P[2 * i, i] += 0.5             # half-way to the node (or boundary) before it
        P[2 * i + 2, i] += 0.5         # half-way to the node (or boundary) after it
    return P


def prolong(X, nx, ny, nz):
    """Trilinear interpolation of the columns of X from (nx, ny, nz) interior nodes to the
    nested (2nx+1, 2ny+1, 2nz+1) mesh; node index g = i + nx (j + ny k)."""
    X = np.asarray(X, dtype=np.float64)
    p = X.shape[1]
    Px, Py, Pz = _axis_weights(nx), _axis_weights(ny), _axis_weights(nz)
    out = np.empty(((2 * nx + 1) * (2 * ny + 1) * (2 * nz + 1), p))
    for c in range(p):
        u = X[:, c].reshape(nz, ny, nx)
        u = np.einsum("ai,kji->kja", Px, u)
        u = np.einsum("bj,kja->kba", Py, u)
        u = np.einsum("ck,kba->cba", Pz, u)
        out[:, c] = u.ravel()
    return out


def carry_over(X, coarse_spec, disc, B_fine=None):
    """The start of the next level: prolongation, the FD rescaling, Cholesky QR (in the B
    metric for elements)."""
    Xf = prolong(X, coarse_spec.nx, coarse_spec.ny, coarse_spec.nz)
    if disc == "q1":
        R = np.linalg.cholesky(Xf.T @ (B_fine @ Xf)).T
        return np.linalg.solve(R.T, Xf.T).T
    Xf *= 2.0 ** -1.5
    return stiefel.cholqr(Xf)[0]


def solve_levels(systems, specs, X0, params, manifolds=None):
    """Alg. 4 (uniform refinement): Alg. 3 on level 0 from X0, then on every finer level
    from the carried-over solution of the level before.  Returns the per-level results."""
    out = []
    X = X0
    for lev, (sysk, spec) in enumerate(zip(systems, specs)):
        if lev > 0:
            X = carry_over(out[-1].X, specs[lev - 1], spec.disc,
                           getattr(sysk, "B", None))
        mf = manifolds[lev] if manifolds else None
        res = optm.minimize(sysk.energy_grad, X, params, manifold=mf)
        out.append(res)
    return out


def refine_check(coarse, fine):
    """True when fine is the uniform refinement of coarse (same box, half the spacing)."""
    return (fine.nx == 2 * coarse.nx + 1 and fine.ny == 2 * coarse.ny + 1
            and fine.nz == 2 * coarse.nz + 1 and abs(2.0 * fine.h - coarse.h) <= 1e-12 * coarse.h
            and all(abs(a - b) <= 1e-12 * max(1.0, abs(a)) for a, b in zip(coarse.lo, fine.lo))
            and math.isclose(coarse.f, fine.f) and coarse.p == fine.p)
