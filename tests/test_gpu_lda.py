"""LDA correlation (KS_TERM_CORR, Perdew-Zunger 1981) on the GPU against the oracle: the
energy terms, E_X and grad E at fixed blocks (finite differences and Q1 elements, both
Hartree solvers), and a converged minimisation with the full LDA."""
import math

import numpy as np
import pytest

from oracle import optm, stiefel
from oracle.fe import BStiefel
from paper_1308_2864_amd import synth
from tests.helpers import oracle_fd, oracle_q1

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def ks():
    from paper_1308_2864_amd import ks as _ks
    return _ks


def dev(a, dtype=torch.float64):
    return torch.tensor(np.ascontiguousarray(a), dtype=dtype, device="cuda")


def host(t):
    return t.detach().cpu().numpy().astype(np.float64)


def _spec(nx=17, ny=13, nz=11, p=5, seed=0, **kw):
    return synth.make_system(nx, ny, nz, 0.55, p, 3, seed=seed, zrange=(1, 4), margin=1.5,
                             min_spacing=1.0, **kw).copy(corr=True)


TERMS = ["kinetic", "external", "hartree", "xc", "nuclear", "total"]


@pytest.mark.parametrize("solver", ["cg", "pcg_fd"])
@pytest.mark.parametrize("p", [1, 5, 32, 70])
def test_fd_energy_grad_with_correlation(p, solver):
    K = ks()
    spec = _spec(p=p, seed=20 + p)
    sysg = K.system_from_spec(spec, hartree_solver=K.KS_HARTREE_CG if solver == "cg"
                              else K.KS_HARTREE_PCG_FD)
    X = synth.make_x0(spec, 2)
    G = torch.zeros((spec.n, p), dtype=torch.float64, device="cuda")
    D = torch.zeros_like(G)
    e = sysg.ks_energy_grad(dev(X), G, D)
    orc = oracle_fd(spec)
    assert orc.use_corr
    en, Gr, _ = orc.energy_grad(X)
    Dr = stiefel.manifold_grad(X, Gr)
    for t in TERMS:
        a, b = getattr(e, t), float(getattr(en, t))
        assert abs(a - b) <= 1e-10 * max(abs(b), 1e-3), (t, a, b)
    assert np.max(np.abs(host(G) - Gr)) <= 1e-9 * np.max(np.abs(Gr))
    assert np.max(np.abs(host(D) - Dr)) <= 1e-9 * np.max(np.abs(Gr))
    # correlation changed the exchange-correlation energy by a negative amount
    en0 = oracle_fd(spec.copy(corr=False)).energy_terms(X)[0]
    assert e.xc < en0.xc


@pytest.mark.parametrize("p", [3, 20])
def test_q1_energy_grad_with_correlation(p):
    K = ks()
    spec = _spec(p=p, seed=40 + p).copy(disc="q1")
    sysg = K.system_from_spec(spec, hartree_solver=K.KS_HARTREE_PCG_FD)
    orc = oracle_q1(spec)
    # a B-orthonormal block
    X0 = synth.make_x0(spec, 2)
    R = np.linalg.cholesky(X0.T @ (orc.B @ X0)).T
    X = np.linalg.solve(R.T, X0.T).T
    Xd = dev(X)
    G = torch.zeros_like(Xd)
    D = torch.zeros_like(Xd)
    e = sysg.ks_energy_grad(Xd, G, D)
    en, Gr, _ = orc.energy_grad(X)
    mf = BStiefel(orc.B, orc.mass_solve)
    Dr = mf.grad(X, Gr)
    for t in TERMS:
        a, b = getattr(e, t), float(getattr(en, t))
        assert abs(a - b) <= 1e-10 * max(1.0, abs(en.total)), (t, a, b)
    assert np.max(np.abs(host(G) - Gr)) <= 1e-9 * np.max(np.abs(Gr))
    assert np.max(np.abs(host(D) - Dr)) <= 1e-9 * np.max(np.abs(Dr))
    assert abs(e.grad_norm - math.sqrt(mf.inner(Dr, Dr))) <= 1e-9 * e.grad_norm


def test_minimize_full_lda_matches_oracle():
    K = ks()
    spec = synth.make_system(12, 12, 12, 0.6, 4, 2, seed=0, zrange=(2, 3), margin=2.0,
                             min_spacing=1.0).copy(corr=True)
    X0 = synth.make_x0(spec, 1)
    sysg = K.system_from_spec(spec, hartree_tol=1e-14)
    X = dev(X0)
    r = sysg.ks_minimize(X, K.ks_default_params(eps_g=1e-7, stagnation_tol=0.0, max_iter=4000))
    orc = oracle_fd(spec)
    ref = optm.minimize(orc.energy_grad, X0, optm.Params(eps_g=1e-7, stagnation_tol=0.0,
                                                         max_iter=4000))
    print(f"LDA: gpu E={r.energy:.12f} ({r.iters} it) oracle E={ref.E:.12f} ({ref.iters} it)")
    assert ref.stop == "grad" and r.stop_reason == K.KS_STOP_GRAD
    assert abs(r.energy - ref.E) <= 1e-10 * abs(ref.E)
    Xg = host(X)
    assert np.linalg.norm(Xg @ Xg.T - ref.X @ ref.X.T) <= 1e-5
    # the full-LDA minimum lies below the exchange-only one reached from the same start
    ref_x = optm.minimize(oracle_fd(spec.copy(corr=False)).energy_grad, X0,
                          optm.Params(eps_g=1e-6, max_iter=4000))
    assert ref.E < ref_x.E
