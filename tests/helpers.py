"""Shared test helpers: build oracle systems from the seeded specs."""
import numpy as np

from oracle.ks import KSSystemFD


def oracle_fd(spec, **kw):
    args = dict(f=spec.f, rc=spec.rc, ext=spec.ext, hartree=spec.hartree, xc=spec.xc,
                corr=spec.corr, mu=spec.mu, tf=spec.tf, vext=spec.vext,
                hartree_bc=spec.hartree_bc)
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
    args = dict(f=spec.f, rc=spec.rc, ext=spec.ext, hartree=spec.hartree, xc=spec.xc,
                corr=spec.corr, mu=spec.mu, tf=spec.tf, vext=spec.vext,
                hartree_bc=spec.hartree_bc)
    args.update(kw)
    return KSSystemQ1(spec.nx, spec.ny, spec.nz, spec.h, spec.lo, spec.p, spec.R, spec.Z, **args)


# Systems with blocks wider than 64 columns (the 128 x 128-tile wide kernels and, with
# KS_PREC_MIXED_BF16, the bf16 X^T G): (N, p, nuclei, seed) on [-8, 8]^3.
WIDE = {80: (14, 80, 4, 5), 130: (16, 130, 6, 5)}


def wide_spec(p):
    from paper_1308_2864_amd import synth
    N, pp, M, seed = WIDE[p]
    return synth.make_system(N, N, N, 16.0 / (N + 1), pp, M, seed=seed, cfg="c5",
                             lo=(-8.0,) * 3, margin=3.0, zrange=(1, 4))
