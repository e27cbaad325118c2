"""Seeded synthetic inputs for the Kohn-Sham Stiefel minimisation.

This module only draws numbers: grid geometry, nuclei (positions and charges),
the random orthonormal starting block X0 and the arrival times of the serving
stream.  It contains none of the method's arithmetic (no potential, energy,
gradient or retraction), so both the GPU path and the CPU oracle can take their
inputs from it without sharing any computation.

The paper's systems (molecules with Troullier-Martins pseudopotentials, Section 4)
cannot be rebuilt here.  The synthetic systems below stand in for them: a
uniform real-space grid with zero Dirichlet boundary (Section 2.3), point-like
nuclei whose Coulomb potential is smoothed by erf (radius r_c), occupation f = 2
per orbital, and an orthonormalised Gaussian random start in place of the LCAO
guess (Section 4.1).

Workloads (grid side N, spacing h, orbitals p, nuclei M, charges Z):

* ``c1``  box [-8,8]^3, N=24 (h=16/25), p=4, M=2, Z=2, R ~ U[-3,3]^3.
* ``c2``  N=64, h=0.3, p=32, M=16, Z in {1..4}, min spacing 1.5 bohr.
* ``c3``  Q1 finite elements, 96^3 interior nodes, h=0.3, p=128, M=64.
* ``c4``  N=128, h=0.3, p=512, M=256, Z in {1..6}.
* ``c5``  serving stream: 512 requests, N in {16,24,32,40,48} on [-8,8]^3,
          p in [2,32], M in [1,16], Z in {1..4}, Poisson arrivals.
"""
from __future__ import annotations

import dataclasses
from typing import List, Optional

import numpy as np

__all__ = [
    "SystemSpec",
    "make_config",
    "make_system",
    "make_x0",
    "make_random_block",
    "make_serving_stream",
    "rng_for",
]

# config ids used in SeedSequence entropy
_CFG_ID = {"c1": 1, "c2": 2, "c3": 3, "c4": 4, "c5": 5, "small": 100}


@dataclasses.dataclass
class SystemSpec:
    """Geometry and physics switches of one synthetic system.

    Grid point (i, j, k), 0-based over the interior, sits at
    ``lo + ((i+1) h, (j+1) h, (k+1) h)`` and has linear index
    ``g = i + nx*(j + ny*k)`` (x fastest).
    """

    nx: int
    ny: int
    nz: int
    h: float
    lo: tuple
    p: int
    R: np.ndarray  # (M, 3) float64
    Z: np.ndarray  # (M,) float64
    f: float = 2.0
    rc: float = 0.5
    disc: str = "fd7"  # "fd7" finite differences, "q1" trilinear finite elements
    ext: bool = True
    hartree: bool = True
    xc: bool = True
    corr: bool = False  # LDA correlation (Perdew-Zunger) on top of the exchange
    tf: bool = False    # Thomas-Fermi kinetic term (orbital-free TFW with p = 1)
    mu: float = 1.0     # weight of the kinetic (von Weizsaecker) term
    vext: str = "erf"   # nuclear potential: "erf" (smoothed Coulomb) or "gnh" (pseudopotential)
    hartree_bc: str = "zero"  # Hartree boundary: "zero" Dirichlet or "monopole" values
    name: str = ""

    @property
    def n(self) -> int:
        return self.nx * self.ny * self.nz

    @property
    def M(self) -> int:
        return int(self.R.shape[0])

    def copy(self, **kw) -> "SystemSpec":
        return dataclasses.replace(self, **kw)


def rng_for(cfg: str, seed: int, stream: int = 0) -> np.random.Generator:
    """Generator seeded from (config id, seed, stream)."""
    return np.random.default_rng(np.random.SeedSequence([_CFG_ID.get(cfg, 999), int(seed), int(stream)]))


def _nuclei(rng, M, lo_box, hi_box, zmin, zmax, min_spacing, fixed_z=None):
    R = np.zeros((M, 3))
    placed = 0
    tries = 0
    while placed < M:
        tries += 1
        if tries > 200000:
            raise RuntimeError("could not place nuclei with the requested spacing")
        c = rng.uniform(lo_box, hi_box, size=3)
        if min_spacing > 0 and placed > 0:
            d = np.sqrt(((R[:placed] - c) ** 2).sum(axis=1))
            if d.min() < min_spacing:
                continue
        R[placed] = c
        placed += 1
    if fixed_z is not None:
        Z = np.full(M, float(fixed_z))
    else:
        Z = rng.integers(zmin, zmax + 1, size=M).astype(np.float64)
    return R, Z


def make_system(nx, ny, nz, h, p, M, *, seed=0, cfg="small", lo=None, zrange=(1, 4),
                fixed_z=None, min_spacing=1.5, margin=None, f=2.0, rc=0.5,
                disc="fd7", name="") -> SystemSpec:
    """A system on an nx*ny*nz interior grid with box centred at the origin."""
    L = np.array([nx + 1, ny + 1, nz + 1], dtype=np.float64) * h
    if lo is None:
        lo = tuple((-L / 2.0).tolist())
    lo = tuple(float(v) for v in lo)
    hi = np.array(lo) + L
    if margin is None:
        margin = min(5.0, 0.25 * float(L.min()))
    rng = rng_for(cfg, seed, 0)
    R, Z = _nuclei(rng, M, np.array(lo) + margin, hi - margin, zrange[0], zrange[1],
                   min_spacing, fixed_z)
    return SystemSpec(nx=nx, ny=ny, nz=nz, h=float(h), lo=lo, p=int(p), R=R, Z=Z, f=f, rc=rc,
                      disc=disc, name=name or f"{cfg}-{nx}x{ny}x{nz}-p{p}")


def make_config(cfg: str, seed: int = 0) -> SystemSpec:
    """The named synthetic workloads (see module docstring)."""
    if cfg == "c1":
        rng = rng_for("c1", seed, 0)
        R, Z = _nuclei(rng, 2, -3.0, 3.0, 2, 2, 0.0, fixed_z=2)
        h = 16.0 / 25.0
        return SystemSpec(nx=24, ny=24, nz=24, h=h, lo=(-8.0, -8.0, -8.0), p=4, R=R, Z=Z,
                          name="c1-fd-24^3-p4")
    if cfg == "c2":
        return make_system(64, 64, 64, 0.3, 32, 16, seed=seed, cfg="c2", zrange=(1, 4),
                           margin=5.0, name="c2-fd-64^3-p32")
    if cfg == "c3":
        return make_system(96, 96, 96, 0.3, 128, 64, seed=seed, cfg="c3", zrange=(1, 4),
                           margin=5.0, disc="q1", name="c3-q1-96^3-p128")
    if cfg == "c4":
        return make_system(128, 128, 128, 0.3, 512, 256, seed=seed, cfg="c4", zrange=(1, 6),
                           margin=5.0, name="c4-fd-128^3-p512")
    raise ValueError(f"unknown config {cfg!r}")


def make_random_block(n, p, seed=0, cfg="small", stream=1) -> np.ndarray:
    """An n x p block of N(0,1) entries (not orthonormalised)."""
    rng = rng_for(cfg, seed, stream)
    return rng.standard_normal((n, p))


def make_x0(spec: SystemSpec, seed=0, cfg: Optional[str] = None, stream=1) -> np.ndarray:
    """Starting block: N(0,1) entries, then the Q factor of a thin Householder QR.

    Returned as an (n, p) float64 array in grid-major layout (row g = grid point).
    """
    cfg = cfg or (spec.name.split("-")[0] if spec.name else "small")
    A = make_random_block(spec.n, spec.p, seed=seed, cfg=cfg, stream=stream)
    Q, _ = np.linalg.qr(A, mode="reduced")
    return np.ascontiguousarray(Q)


# ---- orbital-free workloads ------------------------------------------------------------
AL_LATTICE = 7.559  # bohr, the aluminium cell of the paper's orbital-free experiments
AL_VALENCE = 3.0


def al_cluster(cells: int, a: float = AL_LATTICE) -> np.ndarray:
    """(M, 3) positions of an fcc aluminium cluster of cells^3 unit cells, surface sites
    included: the points (i, j, k) a/2 with i + j + k even and 0 <= i, j, k <= 2 cells,
    centred at the origin (14 atoms for 1 cell, 365 for 4, 1688 for 7)."""
    idx = np.arange(2 * cells + 1)
    I, J, K = np.meshgrid(idx, idx, idx, indexing="ij")
    keep = (I + J + K) % 2 == 0
    R = np.stack([I[keep], J[keep], K[keep]], axis=1).astype(np.float64) * (0.5 * a)
    return R - 0.5 * cells * a


def make_ofdft(cells: int, N: int, margin: float = 4.0, mu: float = 1.0,
               disc: str = "q1", hartree_bc: str = "zero") -> SystemSpec:
    """Orbital-free TFW system (p = 1) of an fcc Al cluster in a cube with margin bohr of
    vacuum on each side, N interior nodes per axis; GNH nuclei of valence 3, LDA exchange
    and correlation, occupation = number of valence electrons."""
    R = al_cluster(cells)
    M = R.shape[0]
    L = cells * AL_LATTICE + 2.0 * margin
    h = L / (N + 1)
    return SystemSpec(nx=N, ny=N, nz=N, h=h, lo=(-0.5 * L,) * 3, p=1, R=R,
                      Z=np.full(M, AL_VALENCE), f=AL_VALENCE * M, disc=disc, corr=True,
                      tf=True, mu=mu, vext="gnh", hartree_bc=hartree_bc,
                      name=f"of-al{M}-{N}^3")


def refine_spec(spec: SystemSpec) -> SystemSpec:
    """The uniform refinement of a system: same box and nuclei, half the spacing,
    2N + 1 interior nodes per axis (coarse node i is fine node 2i + 1)."""
    return spec.copy(nx=2 * spec.nx + 1, ny=2 * spec.ny + 1, nz=2 * spec.nz + 1,
                     h=0.5 * spec.h, name=f"{spec.name}/2")


def refine_levels(spec: SystemSpec, levels: int) -> List[SystemSpec]:
    """spec and its levels - 1 successive uniform refinements, coarsest first."""
    out = [spec]
    for _ in range(levels - 1):
        out.append(refine_spec(out[-1]))
    return out


def make_atomic_guess(spec: SystemSpec, width: float = 1.5) -> np.ndarray:
    """(n, 1) start for p = 1: the square root of a superposition of Gaussians of the given
    width at the nuclei (positive everywhere; normalised by the solver)."""
    g = np.arange(spec.nx) + 1
    x = spec.lo[0] + g * spec.h
    y = spec.lo[1] + (np.arange(spec.ny) + 1) * spec.h
    z = spec.lo[2] + (np.arange(spec.nz) + 1) * spec.h
    Zc, Yc, Xc = np.meshgrid(z, y, x, indexing="ij")
    dens = np.zeros(Xc.shape)
    for a in range(spec.R.shape[0]):
        r2 = (Xc - spec.R[a, 0]) ** 2 + (Yc - spec.R[a, 1]) ** 2 + (Zc - spec.R[a, 2]) ** 2
        dens += np.exp(-r2 / width ** 2)
    return np.ascontiguousarray(np.sqrt(dens).reshape(-1, 1))


@dataclasses.dataclass
class Request:
    rid: int
    arrival: float  # seconds after stream start
    spec: SystemSpec
    seed: int


def make_serving_stream(n_req=512, rate=1.0, seed=0, sides=(16, 24, 32, 40, 48),
                        p_range=(2, 32), m_range=(1, 16)) -> List[Request]:
    """Requests with exponential inter-arrival times (rate per second)."""
    rng = rng_for("c5", seed, 0)
    out = []
    t = 0.0
    for r in range(n_req):
        t += float(rng.exponential(1.0 / rate)) if rate > 0 else 0.0
        N = int(rng.choice(sides))
        p = int(rng.integers(p_range[0], p_range[1] + 1))
        M = int(rng.integers(m_range[0], m_range[1] + 1))
        h = 16.0 / (N + 1)
        spec = make_system(N, N, N, h, p, M, seed=seed * 100000 + r, cfg="c5",
                           lo=(-8.0, -8.0, -8.0), zrange=(1, 4), margin=3.0,
                           name=f"c5-r{r}-{N}^3-p{p}")
        out.append(Request(rid=r, arrival=t, spec=spec, seed=seed * 100000 + r))
    return out
