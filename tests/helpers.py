"""Shared test helpers: build oracle systems from the seeded specs."""
import numpy as np

from oracle.ks import KSSystemFD


def oracle_fd(spec, **kw):
    args = dict(f=spec.f, rc=spec.rc, ext=spec.ext, hartree=spec.hartree, xc=spec.xc)
    args.update(kw)
    return KSSystemFD(spec.nx, spec.ny, spec.nz, spec.h, spec.lo, spec.p, spec.R, spec.Z, **args)


def box_energy_closed_form(nx, ny, nz, h, p, f=2.0):
    """(f/2) * sum of the p smallest eigenvalues of -Laplacian_h with zero Dirichlet boundary.

    Each eigenvalue is a sum over axes of (2 - 2 cos(k pi/(m+1)))/h^2, k = 1..m.
    """
    ev = []
    for m in (nx, ny, nz):
        k = np.arange(1, m + 1)
        ev.append((2.0 - 2.0 * np.cos(k * np.pi / (m + 1))) / h ** 2)
    lam = (ev[0][None, None, :] + ev[1][None, :, None] + ev[2][:, None, None]).ravel()
    lam.sort()
    return 0.5 * f * float(lam[:p].sum()), lam


def oracle_q1(spec, **kw):
    from oracle.fe import KSSystemQ1
    args = dict(f=spec.f, rc=spec.rc, ext=spec.ext, hartree=spec.hartree, xc=spec.xc)
    args.update(kw)
    return KSSystemQ1(spec.nx, spec.ny, spec.nz, spec.h, spec.lo, spec.p, spec.R, spec.Z, **args)
