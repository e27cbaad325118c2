"""The orbital-free (TFW) model on the GPU against the oracle: Section 2.2 eqs. (TFW),
(OFeng), (OFinf) as the p = 1 case of the orbital minimisation (occupation = number of
electrons, rho = N phi^2, von Weizsaecker weight mu), Section 3 eqs. (OFDFT-y), (WY-1d),
and the GNH pseudopotential of Section 4.2 on fcc aluminium clusters.

* the GNH external potential at every grid node (finite differences and Q1 elements);
* energy terms, E_x and grad E at a fixed x;
* Alg. 3 to the Section 4.1 rule with both retractions: the finite-difference runs against
  oracle runs made here, the Q1 run against tests/golden/oracle_ofdft_q1.txt (written by
  tests/golden/make_golden.py from oracle/ only; the oracle takes minutes there).
"""
import math
import os

import numpy as np
import pytest

from oracle import fe, optm, stiefel
from paper_1308_2864_amd import synth
from tests.helpers import oracle_fd, oracle_q1

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
GOLD = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def ks():
    from paper_1308_2864_amd import ks as _ks
    return _ks


def dev(a):
    return torch.tensor(np.ascontiguousarray(a), dtype=torch.float64, device="cuda")


def host(t):
    return t.detach().cpu().numpy().astype(np.float64)


TERMS = ["kinetic", "external", "hartree", "xc", "nuclear", "total"]


def _guess(spec, orc_B=None):
    x = synth.make_atomic_guess(spec)
    nrm = math.sqrt(float(x[:, 0] @ (orc_B @ x[:, 0]))) if orc_B is not None else \
        float(np.linalg.norm(x))
    return x / nrm


@pytest.mark.parametrize("disc", ["fd7", "q1"])
def test_gnh_potential_matches_oracle(disc):
    K = ks()
    spec = synth.make_ofdft(1, 19, margin=2.5, disc=disc)
    print(f"# gnh {disc} n={spec.n}", flush=True)
    s = K.system_from_spec(spec)
    v = torch.zeros(spec.n, dtype=torch.float64, device="cuda")
    s.ks_get_potentials(v_ext=v)
    orc = oracle_fd(spec) if disc == "fd7" else oracle_q1(spec)
    ref = orc.v_ext
    # cubic interpolation of the tabulated radial integrals (step 1/2000 bohr)
    assert np.max(np.abs(host(v) - ref)) <= 1e-10
    s.close()


@pytest.mark.parametrize("solver", ["cg", "pcg_fd"])
@pytest.mark.parametrize("disc", ["fd7", "q1"])
def test_ofdft_energy_grad_matches_oracle(disc, solver):
    K = ks()
    spec = synth.make_ofdft(1, 15, margin=2.5, disc=disc)
    print(f"# ofdft energy {disc} {solver}", flush=True)
    s = K.system_from_spec(spec, hartree_solver=K.KS_HARTREE_CG if solver == "cg"
                           else K.KS_HARTREE_PCG_FD, hartree_tol=1e-14)
    orc = oracle_fd(spec) if disc == "fd7" else oracle_q1(spec)
    x = _guess(spec, orc.B if disc == "q1" else None)
    # a perturbed, still positive start: not a critical point
    x = x * (1.0 + 0.1 * np.sin(np.arange(spec.n) * 0.37)[:, None])
    x = x / (math.sqrt(float(x[:, 0] @ (orc.B @ x[:, 0]))) if disc == "q1"
             else float(np.linalg.norm(x)))
    X = dev(x)
    G = torch.zeros_like(X)
    D = torch.zeros_like(X)
    e = s.ks_energy_grad(X, G, D)
    en, Gr, _ = orc.energy_grad(x)
    if disc == "q1":
        Dr = fe.BStiefel(orc.B, orc.mass_solve).grad(x, Gr)
    else:
        Dr = stiefel.manifold_grad(x, Gr)
    for t in TERMS:
        a, b = getattr(e, t), float(getattr(en, t))
        assert abs(a - b) <= 1e-10 * max(1.0, abs(en.total)), (t, a, b)
    assert np.max(np.abs(host(G) - Gr)) <= 1e-9 * np.max(np.abs(Gr))
    assert np.max(np.abs(host(D) - Dr)) <= 1e-9 * np.max(np.abs(Dr))
    # the Thomas-Fermi term is in the kinetic energy: positive and above the vW part
    en_vw = (oracle_fd if disc == "fd7" else oracle_q1)(spec.copy(tf=False)).energy_terms(x)[0]
    assert e.kinetic > en_vw.kinetic > 0.0
    s.close()


@pytest.mark.parametrize("kind", ["qr", "wy"])
def test_ofdft_minimize_fd_matches_oracle(kind):
    """Al14 on the 7-point grid (h = 0.698), the unit sphere: same energy as the oracle's
    run to 1e-10 relative and the same one-signed ground state."""
    K = ks()
    spec = synth.make_ofdft(1, 17, margin=2.5, disc="fd7")
    print(f"# ofdft minimize fd {kind}", flush=True)
    orc = oracle_fd(spec)
    x0 = _guess(spec)
    ref = optm.minimize(orc.energy_grad, x0, optm.Params(eps_g=1e-8, stagnation_tol=0.0,
                                                         max_iter=3000, retraction=kind))
    assert ref.stop == "grad"
    s = K.system_from_spec(spec, hartree_tol=1e-14)
    X = dev(x0)
    r = s.ks_minimize(X, K.ks_default_params(eps_g=1e-8, stagnation_tol=0.0, max_iter=3000,
                                             retraction=K.KS_WY if kind == "wy" else K.KS_QR))
    print(f"OFDFT fd {kind}: gpu E={r.energy:.12f} ({r.iters} it) oracle E={ref.E:.12f} "
          f"({ref.iters} it)", flush=True)
    assert r.stop_reason == K.KS_STOP_GRAD
    assert abs(r.energy - ref.E) <= 1e-10 * abs(ref.E)
    xg = host(X)[:, 0]
    xr = ref.X[:, 0]
    assert np.all(xg > 0) or np.all(xg < 0)
    assert np.linalg.norm(np.abs(xg) - np.abs(xr)) <= 1e-6
    assert abs(np.linalg.norm(xg) - 1.0) < 1e-12
    s.close()


def _golden(name):
    vals = {}
    for line in open(os.path.join(GOLD, name)):
        if "=" in line and not line.startswith("#"):
            k, v = line.split("=")
            vals[k.strip()] = float(v)
    return vals


@pytest.mark.parametrize("kind", ["qr", "wy"])
def test_ofdft_minimize_q1_matches_golden(kind):
    """Al14 on Q1 elements (h = 0.377, inside the mesh bound of the nodal quadrature), the
    B-sphere x^T B x = 1: the converged energy equals the oracle's to 1e-10 relative, the
    ground state has one sign and its nodal charge h^3 sum rho is the oracle's."""
    K = ks()
    g = _golden("oracle_ofdft_q1.txt")
    spec = synth.make_ofdft(1, int(g["N"]), margin=g["margin"], disc="q1")
    print(f"# ofdft minimize q1 {kind} n={spec.n}", flush=True)
    s = K.system_from_spec(spec, hartree_tol=1e-14)
    X0 = dev(synth.make_atomic_guess(spec))
    X = X0.clone()
    r = s.ks_minimize(X, K.ks_default_params(eps_g=1e-8, stagnation_tol=0.0, max_iter=3000,
                                             retraction=K.KS_WY if kind == "wy" else K.KS_QR))
    print(f"OFDFT q1 {kind}: gpu E={r.energy:.12f} ({r.iters} it) oracle E={g['E']:.12f}",
          flush=True)
    assert r.stop_reason == K.KS_STOP_GRAD
    assert abs(r.energy - g["E"]) <= 1e-10 * abs(g["E"])
    xg = host(X)[:, 0]
    assert np.all(xg > 0) or np.all(xg < 0)
    rho = torch.zeros(spec.n, dtype=torch.float64, device="cuda")
    s.ks_density(X, rho)
    assert abs(spec.h ** 3 * float(rho.sum()) - g["charge"]) <= 1e-6 * g["charge"]
    s.close()


@pytest.mark.parametrize("disc", ["fd7", "q1"])
def test_monopole_boundary_energy_grad_matches_oracle(disc):
    """KS_HBC_MONOPOLE: the boundary potential V_bc (formed once at creation with the
    system's Hartree solver), its energy terms and the gradient against the oracle."""
    K = ks()
    spec = synth.make_ofdft(1, 15, margin=2.5, disc=disc, hartree_bc="monopole")
    print(f"# monopole energy {disc}", flush=True)
    s = K.system_from_spec(spec, hartree_solver=K.KS_HARTREE_PCG_FD, hartree_tol=1e-14)
    orc = oracle_fd(spec) if disc == "fd7" else oracle_q1(spec)
    x = _guess(spec, orc.B if disc == "q1" else None)
    X = dev(x)
    G = torch.zeros_like(X)
    e = s.ks_energy_grad(X, G)
    en, Gr, _ = orc.energy_grad(x)
    for t in TERMS:
        a, b = getattr(e, t), float(getattr(en, t))
        assert abs(a - b) <= 1e-10 * max(1.0, abs(en.total)), (t, a, b)
    assert np.max(np.abs(host(G) - Gr)) <= 1e-9 * np.max(np.abs(Gr))
    # V_eff includes the boundary potential
    veff = torch.zeros(spec.n, dtype=torch.float64, device="cuda")
    s.ks_get_potentials(v_eff=veff)
    assert np.max(np.abs(host(veff) - orc.effective_potential(x))) <= 1e-9 * \
        np.max(np.abs(orc.effective_potential(x)))
    s.close()


def test_monopole_kohn_sham_system_matches_oracle():
    """The boundary option on a Kohn-Sham system (p = 5, erf nuclei, plain CG)."""
    K = ks()
    spec = synth.make_system(17, 13, 11, 0.55, 5, 3, seed=25, zrange=(1, 4), margin=1.5,
                             min_spacing=1.0).copy(hartree_bc="monopole")
    s = K.system_from_spec(spec, hartree_solver=K.KS_HARTREE_CG, hartree_tol=1e-14)
    X0 = synth.make_x0(spec, 2)
    X = dev(X0)
    G = torch.zeros_like(X)
    e = s.ks_energy_grad(X, G)
    orc = oracle_fd(spec)
    en, Gr, _ = orc.energy_grad(X0)
    for t in TERMS:
        a, b = getattr(e, t), float(getattr(en, t))
        assert abs(a - b) <= 1e-10 * max(1.0, abs(en.total)), (t, a, b)
    assert np.max(np.abs(host(G) - Gr)) <= 1e-9 * np.max(np.abs(Gr))
    s.close()


@pytest.mark.parametrize("kind", ["qr", "wy"])
def test_ofdft_minimize_fd_monopole_matches_oracle(kind):
    """Al14 with the monopole boundary: the converged energy (about -1.7 Ha per atom, the
    scale of one atom's energy) equals the oracle's to 1e-10 relative."""
    K = ks()
    spec = synth.make_ofdft(1, 17, margin=2.5, disc="fd7", hartree_bc="monopole")
    orc = oracle_fd(spec)
    x0 = _guess(spec)
    ref = optm.minimize(orc.energy_grad, x0, optm.Params(eps_g=1e-8, stagnation_tol=0.0,
                                                         max_iter=3000, retraction=kind))
    assert ref.stop == "grad"
    s = K.system_from_spec(spec, hartree_tol=1e-14)
    X = dev(x0)
    r = s.ks_minimize(X, K.ks_default_params(eps_g=1e-8, stagnation_tol=0.0, max_iter=3000,
                                             retraction=K.KS_WY if kind == "wy" else K.KS_QR))
    print(f"OFDFT monopole {kind}: gpu E={r.energy:.12f} ({r.iters} it) oracle E={ref.E:.12f}"
          f" ({ref.iters} it), {r.energy / spec.M:.4f} Ha/atom", flush=True)
    assert r.stop_reason == K.KS_STOP_GRAD
    assert abs(r.energy - ref.E) <= 1e-10 * abs(ref.E)
    assert -2.5 < r.energy / spec.M < -1.0
    s.close()
