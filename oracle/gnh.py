"""Goodwin-Needs-Heine local pseudopotential (oracle, FP64).

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__``).

The external potential of the paper's orbital-free experiments (Section 4.2): for a nucleus
with Z valence electrons at distance r,

    V(r) = -(2/pi) int_0^inf  sin(r t)/(r t) [ (Z - A R_p) cos(R_p t) + A sin(R_p t)/t ]
                              exp(-(t/R_c)^6) dt,

with R_p = 1.15, R_c = 3.5 and A = 0.1107 bohr units.  The paper prints the integral without
the leading minus sign; without it the potential would tend to +Z/r far from the nucleus
(both terms have closed forms there, Z - A R_p and A R_p, divided by r), so the electron-ion
attraction is its negative, -Z/r far away.

The integral is evaluated here by composite Gauss-Legendre quadrature on t in [0, 8]
(exp(-(8/3.5)^6) < 1e-61), 128 panels of 32 nodes; the nodes come from numpy's Legendre
routine.  At r = 0 the sinc factor is 1.
"""
from __future__ import annotations

import math

import numpy as np

GNH_RP, GNH_RC, GNH_A = 1.15, 3.5, 0.1107
T_MAX = 8.0


def _nodes(panels=128, per=32, tmax=T_MAX):
    x, w = np.polynomial.legendre.leggauss(per)
    edges = np.linspace(0.0, tmax, panels + 1)
    mid = 0.5 * (edges[:-1] + edges[1:])
    half = 0.5 * (edges[1:] - edges[:-1])
    t = (mid[:, None] + half[:, None] * x[None, :]).ravel()
    wt = (half[:, None] * w[None, :]).ravel()
    return t, wt


def gnh_radial(r, Z, panels=128, per=32):
    """V(r) of one nucleus of valence Z at distances r (any shape)."""
    r = np.asarray(r, dtype=np.float64)
    t, w = _nodes(panels, per)
    f = ((Z - GNH_A * GNH_RP) * np.cos(GNH_RP * t) + GNH_A * np.sin(GNH_RP * t) / t) \
        * np.exp(-(t / GNH_RC) ** 6)
    flat = r.ravel()
    out = np.empty_like(flat)
    for a in range(0, flat.size, 4096):
        rr = flat[a:a + 4096]
        rt = np.outer(rr, t)
        sinc = np.where(rt > 0.0, np.sin(rt) / np.where(rt > 0.0, rt, 1.0), 1.0)
        out[a:a + 4096] = -(2.0 / math.pi) * (sinc * f[None, :]) @ w
    return out.reshape(r.shape)


def v_ext_gnh(coords, R, Z):
    """Sum over nuclei of the GNH potential at the points coords (n, 3)."""
    v = np.zeros(coords.shape[0])
    for a in range(R.shape[0]):
        d = np.sqrt(((coords - R[a]) ** 2).sum(axis=1))
        v += gnh_radial(d, float(Z[a]))
    return v
