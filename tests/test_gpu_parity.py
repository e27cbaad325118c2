"""Parity of the HIP path (through the C ABI) against the FP64 CPU oracle.

Tolerances (FP64 on both sides; derivations in the design notes):
* density, Hamiltonian apply, Gram blocks: rounding only, 1e-13 relative;
* Hartree potential: both CG solves stop at a relative residual <= 1e-13 (GPU) and
  <= 1e-14 (oracle), so the potentials agree to kappa(L) * 1e-13 ~ 1e-10 relative;
  tested at 1e-9;
* energy terms at a fixed X: 1e-10 relative; G and grad E: 1e-9 of max |G|;
* retractions at fixed (X, G, tau): 1e-11 absolute (entries are O(1));
* converged minimisations: energy 1e-10 relative, occupied subspace ||XX^T - YY^T||_F
  <= 1e-6 (both runs to ||grad E|| <= 1e-8 with a spectral gap > 0.05).
"""
import math
import os

import numpy as np
import pytest

from oracle import optm, stiefel
from paper_1308_2864_amd import synth
from tests.helpers import box_energy_closed_form, oracle_fd

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def ks():
    from paper_1308_2864_amd import ks as _ks
    return _ks


def dev(a):
    return torch.tensor(np.ascontiguousarray(a), dtype=torch.float64, device="cuda")


def host(t):
    return t.detach().cpu().numpy()


def spec_small(nx=17, ny=13, nz=11, p=5, M=3, seed=0, h=0.55, margin=1.5, **kw):
    return synth.make_system(nx, ny, nz, h, p, M, seed=seed, zrange=(1, 3), margin=margin,
                             min_spacing=1.0, **kw)


def _dst_poisson(nx, ny, nz, h, b):
    import scipy.fft
    B = b.reshape(nz, ny, nx)
    Bh = scipy.fft.dstn(B, type=1)
    lam = [(2 - 2 * np.cos(np.arange(1, m + 1) * np.pi / (m + 1))) / h ** 2 for m in (nx, ny, nz)]
    Vh = Bh / (lam[2][:, None, None] + lam[1][None, :, None] + lam[0][None, None, :])
    return scipy.fft.idstn(Vh, type=1).ravel()


# ------------------------------------------------------------------------------------------
# step-level parity
# ------------------------------------------------------------------------------------------

@pytest.mark.parametrize("p", [1, 4, 5, 16, 20, 32, 37, 64])
def test_gram_blocks(p):
    spec = spec_small(9, 7, 5, p=p, seed=p)
    sysg = ks().system_from_spec(spec)
    rng = np.random.default_rng(p)
    A = rng.standard_normal((spec.n, p))
    B = rng.standard_normal((spec.n, p))
    out = torch.zeros(3 * p * p, dtype=torch.float64, device="cuda")
    sysg.ks_gram(dev(A), dev(B), out)
    got = host(out).reshape(3, p, p)
    for g, ref in zip(got, (A.T @ A, A.T @ B, B.T @ B)):
        assert np.max(np.abs(g - ref)) <= 1e-13 * np.max(np.abs(ref)) * math.sqrt(spec.n)


@pytest.mark.parametrize("p", [80, 97, 130, 257])
def test_gram_blocks_wide(p):
    """More than 64 columns: one launch forms the products on 128 x 128 output tiles over
    row chunks (ragged last tile; odd p takes element loads; n = 1320 rows)."""
    spec = spec_small(12, 11, 10, p=p, seed=p)
    sysg = ks().system_from_spec(spec)
    rng = np.random.default_rng(p)
    A = rng.standard_normal((spec.n, p))
    B = rng.standard_normal((spec.n, p))
    out = torch.zeros(3 * p * p, dtype=torch.float64, device="cuda")
    sysg.ks_gram(dev(A), dev(B), out)
    got = host(out).reshape(3, p, p)
    for g, ref in zip(got, (A.T @ A, A.T @ B, B.T @ B)):
        assert np.max(np.abs(g - ref)) <= 1e-13 * np.max(np.abs(ref)) * math.sqrt(spec.n)


def test_gram_blocks_large_n_ragged():
    spec = spec_small(64, 33, 31, p=32, seed=3)
    sysg = ks().system_from_spec(spec)
    X = synth.make_x0(spec, 3)
    G = synth.make_random_block(spec.n, 32, seed=4)
    out = torch.zeros(3 * 32 * 32, dtype=torch.float64, device="cuda")
    sysg.ks_gram(dev(X), dev(G), out)
    got = host(out).reshape(3, 32, 32)
    assert np.max(np.abs(got[0] - np.eye(32))) < 1e-13
    assert np.max(np.abs(got[1] - X.T @ G)) < 1e-12 * np.max(np.abs(X.T @ G)) * 10
    assert np.max(np.abs(got[2] - G.T @ G)) < 1e-12 * np.max(np.abs(G.T @ G)) * 10


def test_density():
    spec = spec_small(p=7)
    sysg = ks().system_from_spec(spec)
    X = synth.make_x0(spec, 1)
    rho = torch.zeros(spec.n, dtype=torch.float64, device="cuda")
    sysg.ks_density(dev(X), rho)
    ref = oracle_fd(spec).density(X)
    assert np.max(np.abs(host(rho) - ref)) <= 1e-14 * np.max(ref)


@pytest.mark.parametrize("solver", ["cg", "pcg_fd"])
@pytest.mark.parametrize("shape", [(17, 13, 11), (32, 32, 32), (5, 40, 3), (70, 9, 66),
                                   (128, 120, 20)])
def test_hartree_solve(shape, solver):
    nx, ny, nz = shape
    K = ks()
    spec = spec_small(nx, ny, nz, p=2, seed=2, M=1, margin=0.3)
    sysg = K.system_from_spec(spec, hartree_solver=K.KS_HARTREE_CG if solver == "cg"
                              else K.KS_HARTREE_PCG_FD)
    rho = np.abs(synth.make_random_block(spec.n, 1, seed=9)[:, 0])
    exact = _dst_poisson(nx, ny, nz, spec.h, 4 * math.pi * rho)
    vh = torch.zeros(spec.n, dtype=torch.float64, device="cuda")
    it, rel = sysg.ks_hartree_solve(dev(rho), vh, warm=False)
    assert rel <= 1e-13 and it > 0
    assert np.max(np.abs(host(vh) - exact)) <= 1e-9 * np.max(np.abs(exact))
    orc = oracle_fd(spec)
    v_orc, _, _ = orc.hartree_cg(rho)
    assert np.max(np.abs(host(vh) - v_orc)) <= 1e-9 * np.max(np.abs(exact))
    if solver == "pcg_fd":
        assert it <= 3  # the preconditioner is the exact inverse
    # warm start from the converged potential
    it2, _ = sysg.ks_hartree_solve(dev(rho), vh, warm=True)
    assert it2 <= 3


def test_hartree_zero_density():
    spec = spec_small(p=2)
    sysg = ks().system_from_spec(spec)
    vh = torch.ones(spec.n, dtype=torch.float64, device="cuda")
    it, rel = sysg.ks_hartree_solve(torch.zeros(spec.n, dtype=torch.float64, device="cuda"), vh,
                                    warm=True)
    assert it == 0 and float(vh.abs().max()) == 0.0


@pytest.mark.parametrize("p,ld", [(5, 0), (32, 0), (6, 9)])
def test_apply_hamiltonian(p, ld):
    spec = spec_small(p=p, seed=p)
    sysg = ks().system_from_spec(spec, ld=ld)
    ldx = ld or p
    X = synth.make_random_block(spec.n, p, seed=5)
    veff = synth.make_random_block(spec.n, 1, seed=6)[:, 0]
    Xp = np.zeros((spec.n, ldx))
    Xp[:, :p] = X
    Y = torch.full((spec.n, ldx), 7.0, dtype=torch.float64, device="cuda")
    sysg.ks_apply_hamiltonian(dev(Xp), Y, dev(veff))
    ref = oracle_fd(spec).hamiltonian_apply(X, veff)
    got = host(Y)
    assert np.max(np.abs(got[:, :p] - ref)) <= 1e-13 * np.max(np.abs(ref))
    assert np.all(got[:, p:] == 7.0)  # padding untouched


def test_potentials_setup():
    spec = spec_small(p=3, M=4, seed=8)
    sysg = ks().system_from_spec(spec)
    v = torch.zeros(spec.n, dtype=torch.float64, device="cuda")
    sysg.ks_get_potentials(v_ext=v)
    ref = oracle_fd(spec).v_ext
    assert np.max(np.abs(host(v) - ref)) <= 1e-14 * np.max(np.abs(ref))


# ------------------------------------------------------------------------------------------
# energy and gradient at a fixed X
# ------------------------------------------------------------------------------------------

TERMS = ["kinetic", "external", "hartree", "xc", "nuclear", "total"]


def _compare_energy_grad(spec, X, ld=0, solver=0):
    K = ks()
    sysg = K.system_from_spec(spec, ld=ld, hartree_solver=solver)
    p = spec.p
    ldx = ld or p
    Xp = np.zeros((spec.n, ldx))
    Xp[:, :p] = X
    G = torch.zeros((spec.n, ldx), dtype=torch.float64, device="cuda")
    D = torch.zeros((spec.n, ldx), dtype=torch.float64, device="cuda")
    e = sysg.ks_energy_grad(dev(Xp), G, D)
    orc = oracle_fd(spec)
    en, Gr, _ = orc.energy_grad(X)
    Dr = stiefel.manifold_grad(X, Gr)
    for t in TERMS:
        a, b = getattr(e, t), float(getattr(en, t))
        assert abs(a - b) <= 1e-10 * max(abs(b), 1e-3), (t, a, b)
    gG, gD = host(G)[:, :p], host(D)[:, :p]
    assert np.max(np.abs(gG - Gr)) <= 1e-9 * np.max(np.abs(Gr))
    assert np.max(np.abs(gD - Dr)) <= 1e-9 * np.max(np.abs(Gr))
    assert abs(e.grad_norm - np.linalg.norm(Dr)) <= 1e-9 * np.linalg.norm(Gr)
    assert abs(e.orth_error - stiefel.orth_error(X)) < 1e-12
    assert e.hartree_relres <= 1e-13 or not spec.hartree
    return sysg, e


@pytest.mark.parametrize("case", ["all", "no_hartree", "no_xc", "ext_only", "p1", "p37"])
def test_energy_grad_small(case):
    kw = dict(all={}, no_hartree=dict(hartree=False), no_xc=dict(xc=False),
              ext_only=dict(hartree=False, xc=False), p1={}, p37={})[case]
    p = dict(p1=1, p37=37).get(case, 5)
    spec = spec_small(p=p, seed=11).copy(**kw)
    X = synth.make_x0(spec, 2)
    _compare_energy_grad(spec, X)


def test_energy_grad_pcg_fd():
    spec = spec_small(20, 17, 15, p=6, seed=14)
    _compare_energy_grad(spec, synth.make_x0(spec, 3), solver=ks().KS_HARTREE_PCG_FD)


def test_energy_grad_c2_pcg_fd():
    spec = synth.make_config("c2", 0)
    _compare_energy_grad(spec, synth.make_x0(spec, 0), solver=ks().KS_HARTREE_PCG_FD)


def test_energy_grad_padded_ld():
    spec = spec_small(p=6, seed=12)
    _compare_energy_grad(spec, synth.make_x0(spec, 3), ld=8)


def test_energy_grad_c1():
    spec = synth.make_config("c1", 0)
    _compare_energy_grad(spec, synth.make_x0(spec, 0))


def test_energy_grad_c2():
    """Full-size FP64 workload (64^3 grid, p = 32): the evaluation at the seeded start."""
    spec = synth.make_config("c2", 0)
    _compare_energy_grad(spec, synth.make_x0(spec, 0))


def test_energy_grad_is_deterministic():
    spec = spec_small(32, 24, 20, p=20, seed=13)
    X = dev(synth.make_x0(spec, 4))
    sysg = ks().system_from_spec(spec)
    out = []
    for _ in range(2):
        G = torch.zeros_like(X)
        sysg.ks_hartree_solve(torch.zeros(spec.n, dtype=torch.float64, device="cuda"),
                              torch.zeros(spec.n, dtype=torch.float64, device="cuda"))
        e = sysg.ks_energy_grad(X, G)
        out.append((e.total, host(G)))
    # same warm start each time is not guaranteed (V_H is kept), so compare G to 1e-12 and
    # a repeated call from the same state bitwise
    sys2 = ks().system_from_spec(spec)
    G1 = torch.zeros_like(X)
    G2 = torch.zeros_like(X)
    e1 = sys2.ks_energy_grad(X, G1)
    sys3 = ks().system_from_spec(spec)
    e2 = sys3.ks_energy_grad(X, G2)
    assert e1.total == e2.total
    assert torch.equal(G1, G2)


def test_energy_grad_nonfinite_input():
    K = ks()
    spec = spec_small(p=3)
    sysg = K.system_from_spec(spec)
    X = synth.make_x0(spec, 1)
    X[5, 1] = np.nan
    with pytest.raises(K.KSError) as ei:
        sysg.ks_energy_grad(dev(X))
    assert ei.value.code == K.KS_E_NONFINITE


# ------------------------------------------------------------------------------------------
# retractions at fixed (X, G, tau)
# ------------------------------------------------------------------------------------------

@pytest.mark.parametrize("kind", ["qr", "wy"])
@pytest.mark.parametrize("p", [1, 5, 17, 29, 32])
def test_retract(kind, p):
    K = ks()
    spec = spec_small(p=p, seed=20 + p)
    sysg = K.system_from_spec(spec)
    X = synth.make_x0(spec, 5)
    orc = oracle_fd(spec)
    _, G, _ = orc.energy_grad(X)
    for tau in (1e-3, 0.05):
        out = torch.zeros((spec.n, p), dtype=torch.float64, device="cuda")
        sysg.ks_retract(dev(X), dev(G), tau, K.KS_QR if kind == "qr" else K.KS_WY, out)
        ref = stiefel.retract_qr(X, G, tau) if kind == "qr" else stiefel.retract_wy(X, G, tau)
        assert np.max(np.abs(host(out) - ref)) <= 1e-11, (kind, p, tau)


@pytest.mark.parametrize("kind", ["qr", "wy"])
@pytest.mark.parametrize("p", [80, 97, 130])
def test_retract_wide(kind, p):
    """More than 64 columns: the persistent combine forms 128-row x 128-column output tiles
    over weight slabs of 16 contraction rows (n = 1320: a ragged last row tile; odd p takes
    element loads); the density follows from the finished block."""
    K = ks()
    spec = spec_small(12, 11, 10, p=p, seed=40 + p)
    sysg = K.system_from_spec(spec)
    X = synth.make_x0(spec, 5)
    orc = oracle_fd(spec)
    _, G, _ = orc.energy_grad(X)
    for tau in (1e-3, 0.05):
        out = torch.zeros((spec.n, p), dtype=torch.float64, device="cuda")
        sysg.ks_retract(dev(X), dev(G), tau, K.KS_QR if kind == "qr" else K.KS_WY, out)
        ref = stiefel.retract_qr(X, G, tau) if kind == "qr" else stiefel.retract_wy(X, G, tau)
        assert np.max(np.abs(host(out) - ref)) <= 1e-11, (kind, p, tau)


@pytest.mark.parametrize("kind,p,shape", [("qr", 200, (12, 11, 10)), ("wy", 200, (12, 11, 10)),
                                          ("qr", 512, (16, 16, 16))])
def test_retract_wide_factor_in_global_memory(kind, p, shape):
    """Factors too large for LDS (the p x p Cholesky above p = 138, the 2p x 2p LU above
    p = 64) work in the global scratch area; p = 512 is the widest block the library takes."""
    K = ks()
    spec = spec_small(*shape, p=p, seed=7 + p)
    sysg = K.system_from_spec(spec)
    X = synth.make_x0(spec, 6)
    orc = oracle_fd(spec)
    _, G, _ = orc.energy_grad(X)
    tau = 1e-3
    out = torch.zeros((spec.n, p), dtype=torch.float64, device="cuda")
    sysg.ks_retract(dev(X), dev(G), tau, K.KS_QR if kind == "qr" else K.KS_WY, out)
    ref = stiefel.retract_qr(X, G, tau) if kind == "qr" else stiefel.retract_wy(X, G, tau)
    assert np.max(np.abs(host(out) - ref)) <= 1e-10 * np.max(np.abs(ref)), (kind, p)
    Y = host(out)
    assert np.max(np.abs(Y.T @ Y - np.eye(p))) < 1e-11


@pytest.mark.parametrize("p", [3, 24])
def test_retract_rank_deficient_reports_cholesky_breakdown(p):
    K = ks()
    spec = spec_small(p=p)
    sysg = K.system_from_spec(spec)
    X = synth.make_x0(spec, 5)
    X[:, p - 1] = X[:, 1]
    G = np.zeros_like(X)
    out = torch.zeros_like(dev(X))
    with pytest.raises(K.KSError) as ei:
        sysg.ks_retract(dev(X), dev(G), 0.0, K.KS_QR, out)
    assert ei.value.code == K.KS_E_NOT_SPD


def test_retract_nonfinite_wy_system():
    K = ks()
    spec = spec_small(p=3)
    sysg = K.system_from_spec(spec)
    X = synth.make_x0(spec, 5)
    G = np.ones_like(X)
    G[0, 0] = np.inf
    out = torch.zeros_like(dev(X))
    with pytest.raises(K.KSError) as ei:
        sysg.ks_retract(dev(X), dev(G), 0.1, K.KS_WY, out)
    assert ei.value.code in (K.KS_E_SINGULAR, K.KS_E_NONFINITE)


def test_retract_rejects_aliasing():
    K = ks()
    spec = spec_small(p=3)
    sysg = K.system_from_spec(spec)
    X = dev(synth.make_x0(spec, 5))
    with pytest.raises(K.KSError) as ei:
        sysg.ks_retract(X, X.clone(), 0.1, K.KS_QR, X)
    assert ei.value.code == K.KS_E_INVAL


# ------------------------------------------------------------------------------------------
# Alg. 3 end to end
# ------------------------------------------------------------------------------------------

def _run_both(spec, seed, kind, eps=1e-8, max_iter=4000, solver=0):
    K = ks()
    X0 = synth.make_x0(spec, seed)
    sysg = K.system_from_spec(spec, hartree_solver=solver)
    X = dev(X0)
    prm = K.ks_default_params(eps_g=eps, stagnation_tol=0.0, max_iter=max_iter,
                              retraction=K.KS_QR if kind == "qr" else K.KS_WY)
    r = sysg.ks_minimize(X, prm)
    orc = oracle_fd(spec)
    ref = optm.minimize(orc.energy_grad, X0, optm.Params(eps_g=eps, stagnation_tol=0.0,
                                                         max_iter=max_iter, retraction=kind))
    return r, host(X), ref, sysg


@pytest.mark.parametrize("kind", ["qr", "wy"])
def test_minimize_matches_oracle(kind):
    K = ks()
    spec = synth.make_system(12, 12, 12, 0.6, 4, 2, seed=0, zrange=(2, 3), margin=2.0,
                             min_spacing=1.0)
    r, X, ref, _ = _run_both(spec, 1, kind)
    # 1e-8 sits near the rounding floor of the Armijo test (about sqrt(eps |E| / tau));
    # a run whose rounding leaves it stalled just above stops at max_iter instead
    assert ref.stop == "grad" and r.grad_norm <= 5e-8
    assert abs(r.energy - ref.E) <= 1e-10 * abs(ref.E)
    assert np.linalg.norm(X @ X.T - ref.X @ ref.X.T) <= 1e-6
    assert r.terms.orth_error < 1e-12


@pytest.mark.parametrize("kind", ["qr", "wy"])
def test_minimize_matches_oracle_pcg_fd(kind):
    K = ks()
    spec = synth.make_system(13, 12, 11, 0.6, 4, 2, seed=3, zrange=(2, 3), margin=2.0,
                             min_spacing=1.0)
    r, X, ref, _ = _run_both(spec, 2, kind, solver=K.KS_HARTREE_PCG_FD)
    assert ref.stop == "grad" and r.grad_norm <= 5e-8
    assert abs(r.energy - ref.E) <= 1e-10 * abs(ref.E)
    assert np.linalg.norm(X @ X.T - ref.X @ ref.X.T) <= 1e-6


@pytest.mark.parametrize("kind", ["qr", "wy"])
def test_minimize_p32_first_steps_match_oracle(kind):
    """p = 32 (c2's width): the Hamiltonian pass forms X^T X and X^T G itself (QR), the
    gradient combine forms D^T D (X^T D = X^T G + (X^T X) W from the reduced blocks) and the
    BB sums come without a pass over X_k (Section 3 eq. (bb-1) through the QR factor of the
    trial); eight steps of Alg. 3 from the same start follow the oracle's eight steps (the
    trajectories agree to rounding this early)."""
    K = ks()
    spec = synth.make_system(16, 14, 12, 0.6, 32, 6, seed=4, zrange=(2, 4), margin=1.5,
                             min_spacing=1.0)
    X0 = synth.make_x0(spec, 5)
    sysg = K.system_from_spec(spec, hartree_solver=K.KS_HARTREE_PCG_FD)
    X = dev(X0)
    r = sysg.ks_minimize(X, K.ks_default_params(eps_g=1e-12, stagnation_tol=0.0, max_iter=8,
                                                retraction=K.KS_QR if kind == "qr" else K.KS_WY))
    orc = oracle_fd(spec)
    ref = optm.minimize(orc.energy_grad, X0, optm.Params(eps_g=1e-12, stagnation_tol=0.0,
                                                         max_iter=8, retraction=kind))
    assert r.iters == ref.iters == 8 and r.nfe == ref.nfe
    assert abs(r.energy - ref.E) <= 1e-12 * abs(ref.E)
    assert abs(r.grad_norm - ref.gnorm) <= 1e-8 * ref.gnorm
    assert np.max(np.abs(host(X) - ref.X)) <= 1e-9
    assert r.terms.orth_error < 1e-12


@pytest.mark.parametrize("p", [13, 24])
def test_minimize_ragged_p_first_steps_match_oracle(p):
    """Widths that leave padded columns in the last 16-column tile (p_p = 16 and 32): the
    QR trial's BB sums from the retraction and gradient passes and the factor R, and X^T D
    formed from the reduced blocks, with the padded rows and columns of R, W and the Gram
    blocks zero; six steps of Alg. 3 follow the oracle's six steps."""
    K = ks()
    spec = synth.make_system(14, 13, 12, 0.6, p, 5, seed=11, zrange=(2, 4), margin=1.5,
                             min_spacing=1.0)
    X0 = synth.make_x0(spec, 3)
    sysg = K.system_from_spec(spec, hartree_solver=K.KS_HARTREE_PCG_FD)
    X = dev(X0)
    r = sysg.ks_minimize(X, K.ks_default_params(eps_g=1e-12, stagnation_tol=0.0, max_iter=6,
                                                retraction=K.KS_QR))
    orc = oracle_fd(spec)
    ref = optm.minimize(orc.energy_grad, X0, optm.Params(eps_g=1e-12, stagnation_tol=0.0,
                                                         max_iter=6, retraction="qr"))
    print(f"p={p}: gpu E={r.energy:.15f} nfe={r.nfe}, oracle E={ref.E:.15f} nfe={ref.nfe}",
          flush=True)
    assert r.iters == ref.iters == 6 and r.nfe == ref.nfe
    assert abs(r.energy - ref.E) <= 1e-12 * abs(ref.E)
    assert abs(r.grad_norm - ref.gnorm) <= 1e-8 * ref.gnorm
    assert np.max(np.abs(host(X) - ref.X)) <= 1e-9
    assert r.terms.orth_error < 1e-12


@pytest.mark.parametrize("kind", ["qr", "wy"])
def test_minimize_wide_p_first_steps_match_oracle(kind):
    """p = 100 (one ragged 128-column tile of the wide kernels): six steps of Alg. 3 against
    the oracle's six steps (wide Gram and combine, the one-workgroup factorisations for
    p > 64)."""
    K = ks()
    spec = synth.make_system(14, 13, 12, 0.6, 100, 8, seed=6, zrange=(2, 4), margin=1.5,
                             min_spacing=1.0)
    X0 = synth.make_x0(spec, 7)
    sysg = K.system_from_spec(spec, hartree_solver=K.KS_HARTREE_PCG_FD)
    X = dev(X0)
    r = sysg.ks_minimize(X, K.ks_default_params(eps_g=1e-12, stagnation_tol=0.0, max_iter=6,
                                                retraction=K.KS_QR if kind == "qr" else K.KS_WY))
    orc = oracle_fd(spec)
    ref = optm.minimize(orc.energy_grad, X0, optm.Params(eps_g=1e-12, stagnation_tol=0.0,
                                                         max_iter=6, retraction=kind))
    assert r.iters == ref.iters == 6 and r.nfe == ref.nfe
    assert abs(r.energy - ref.E) <= 1e-12 * abs(ref.E)
    assert abs(r.grad_norm - ref.gnorm) <= 1e-8 * ref.gnorm
    assert np.max(np.abs(host(X) - ref.X)) <= 1e-9
    assert r.terms.orth_error < 1e-12


def test_minimize_p512_first_steps_match_oracle():
    """p = 512, the widest block (four 128-column tiles; the factor in global memory):
    three steps of Alg. 3 against the oracle's three on a 16^3 grid."""
    K = ks()
    spec = synth.make_system(16, 16, 16, 0.6, 512, 8, seed=9, zrange=(2, 4), margin=1.5,
                             min_spacing=1.0)
    X0 = synth.make_x0(spec, 8)
    sysg = K.system_from_spec(spec, hartree_solver=K.KS_HARTREE_PCG_FD)
    X = dev(X0)
    r = sysg.ks_minimize(X, K.ks_default_params(eps_g=1e-12, stagnation_tol=0.0, max_iter=3))
    orc = oracle_fd(spec)
    ref = optm.minimize(orc.energy_grad, X0, optm.Params(eps_g=1e-12, stagnation_tol=0.0,
                                                         max_iter=3))
    assert r.iters == ref.iters == 3 and r.nfe == ref.nfe
    assert abs(r.energy - ref.E) <= 1e-12 * abs(ref.E)
    assert abs(r.grad_norm - ref.gnorm) <= 1e-8 * ref.gnorm
    assert np.max(np.abs(host(X) - ref.X)) <= 1e-9
    assert r.terms.orth_error < 1e-11


@pytest.mark.parametrize("solver", ["cg", "pcg_fd"])
def test_minimize_wide_planes_first_steps_match_oracle(solver):
    """128 x 120 x 20 (planes of the widest transform, S_x read from L2): three steps of
    Alg. 3 against the oracle's three, with the plain CG solver and with the fast
    diagonalisation (whose exact steps meet the 1e-13 residual test on this grid)."""
    K = ks()
    spec = synth.make_system(128, 120, 20, 0.3, 4, 3, seed=4, zrange=(1, 3), margin=1.5,
                             min_spacing=1.0)
    X0 = synth.make_x0(spec, 2)
    sysg = K.system_from_spec(spec, hartree_solver=K.KS_HARTREE_CG if solver == "cg"
                              else K.KS_HARTREE_PCG_FD,
                              **({"hartree_tol": 1e-14} if solver == "cg" else {}))
    X = dev(X0)
    r = sysg.ks_minimize(X, K.ks_default_params(eps_g=1e-12, stagnation_tol=0.0, max_iter=3))
    orc = oracle_fd(spec)
    ref = optm.minimize(orc.energy_grad, X0, optm.Params(eps_g=1e-12, stagnation_tol=0.0,
                                                         max_iter=3))
    assert r.iters == ref.iters == 3 and r.nfe == ref.nfe
    assert abs(r.energy - ref.E) <= 1e-10 * abs(ref.E)
    assert abs(r.grad_norm - ref.gnorm) <= 1e-7 * ref.gnorm
    assert np.max(np.abs(host(X) - ref.X)) <= 1e-8


def test_minimize_with_backtracking_matches_oracle():
    """A first step far too long (tau0 = 20) is rejected and backtracked: the next trial's QR
    factor, queued before the host has read the judgement, must then take the current
    point's Gram blocks.  Eight steps against the oracle's eight, backtracks included."""
    K = ks()
    spec = synth.make_system(17, 13, 11, 0.55, 5, 3, seed=21, zrange=(1, 3), margin=1.5,
                             min_spacing=1.0)
    X0 = synth.make_x0(spec, 3)
    sysg = K.system_from_spec(spec, hartree_solver=K.KS_HARTREE_PCG_FD)
    X = dev(X0)
    r = sysg.ks_minimize(X, K.ks_default_params(tau0=20.0, eps_g=1e-12, stagnation_tol=0.0,
                                                max_iter=8))
    orc = oracle_fd(spec)
    ref = optm.minimize(orc.energy_grad, X0, optm.Params(tau0=20.0, eps_g=1e-12,
                                                         stagnation_tol=0.0, max_iter=8))
    assert ref.backtracks >= 1
    assert (r.iters, r.nfe, r.backtracks) == (ref.iters, ref.nfe, ref.backtracks)
    assert abs(r.energy - ref.E) <= 1e-12 * abs(ref.E)
    assert np.max(np.abs(host(X) - ref.X)) <= 1e-9


def test_minimize_ragged_p5():
    K = ks()
    spec = spec_small(15, 12, 10, p=5, M=2, seed=31, h=0.6)
    r, X, ref, _ = _run_both(spec, 2, "qr", eps=1e-7)
    assert r.stop_reason == K.KS_STOP_GRAD
    assert abs(r.energy - ref.E) <= 1e-10 * abs(ref.E)


def test_minimize_box_closed_form_c1_grid():
    """V = 0, no Hartree, no exchange: the minimum is the closed-form eigenvalue sum."""
    K = ks()
    spec = synth.make_config("c1", 0).copy(ext=False, hartree=False, xc=False)
    sysg = K.system_from_spec(spec)
    X = dev(synth.make_x0(spec, 0))
    r = sysg.ks_minimize(X, K.ks_default_params(eps_g=1e-9, stagnation_tol=0.0))
    expect, _ = box_energy_closed_form(24, 24, 24, spec.h, 4)
    assert r.stop_reason == K.KS_STOP_GRAD
    assert abs(r.energy - expect) <= 1e-11 * expect


def _golden(name):
    vals = {}
    path = os.path.join(GOLDEN, name)
    if not os.path.exists(path):
        return None
    for line in open(path):
        line = line.split("#", 1)[0].strip()
        if line:
            k, v = line.split("=")
            vals[k.strip()] = float(v)
    return vals


@pytest.mark.parametrize("kind,solver", [("qr", 0), ("wy", 0), ("qr", 1)])
def test_minimize_c1_matches_oracle_reference(kind, solver):
    """Config c1 (24^3, p = 4, 2 nuclei Z = 2): converged energy vs the stored oracle run."""
    K = ks()
    gold = _golden("oracle_c1_s0_qr.txt")
    if gold is None:
        pytest.skip("oracle reference for c1 not generated")
    spec = synth.make_config("c1", 0)
    # The plain CG solve runs to the oracle's tolerance (1e-14): at the library default of
    # 1e-13 its warm-started V_H carries energy noise that puts the stall floor of the
    # gradient (sqrt(noise / tau)) above 1e-7, so Alg. 3 would stop on max_iter.
    sysg = K.system_from_spec(spec, hartree_solver=solver,
                              **({"hartree_tol": 1e-14} if solver == 0 else {}))
    X = dev(synth.make_x0(spec, 0))
    # the oracle needs 1549 iterations; a run stalled at the rounding floor (below) stops
    # on max_iter
    r = sysg.ks_minimize(X, K.ks_default_params(
        eps_g=1e-7, stagnation_tol=0.0, max_iter=5000,
        retraction=K.KS_QR if kind == "qr" else K.KS_WY), check=False)
    print(f"c1 {kind}: stop={K.STOP_NAMES[r.stop_reason]} it={r.iters} nfe={r.nfe} "
          f"|grad|={r.grad_norm:.2e} E={r.energy:.14f} E_ref={gold['E']:.14f}", flush=True)
    # 1e-7 lies near the rounding floor of the Armijo test on c1, about sqrt(eps |E| / tau):
    # 3e-8 .. 2e-7 on QR trajectories, and up to about 1e-6 on WY ones, whose last steps
    # can shrink to tau ~ 1e-3.  A run may stall just above 1e-7; its energy must still
    # agree with the oracle's.
    floor = 3e-7 if kind == "qr" else 2e-6
    assert r.stop_reason == K.KS_STOP_GRAD or (r.stop_reason == K.KS_STOP_MAXIT and
                                               r.grad_norm <= floor)
    assert abs(r.energy - gold["E"]) <= 1e-10 * abs(gold["E"])
    # The occupied subspace of c1 is ill-determined at ||grad E|| = 1e-7 (gap ~8e-3 Ha and a
    # softer nonlinear Hessian), so compare what is unique -- the energy above and the
    # occupied Ritz values -- and check that the GPU point is a stationary point of the same
    # kind as the oracle's: every occupied Ritz value is an eigenvalue of its own H(rho).
    # (From this seed Alg. 3 -- oracle and GPU alike -- ends at a stationary point that
    # occupies levels 1, 2, 3 and 5 of H(rho); the theory of Alg. 3 promises stationarity,
    # not the aufbau occupation.)
    import scipy.sparse.linalg as spla
    Xref = np.load(os.path.join(GOLDEN, "oracle_c1_s0_qr_X.npy"))
    Xg = host(X)
    orc = oracle_fd(spec)

    def ritz_and_resid(Xa):
        veff = orc.effective_potential(Xa)
        HX = orc.hamiltonian_apply(Xa, veff)
        T = Xa.T @ HX
        return np.linalg.eigvalsh(0.5 * (T + T.T)), np.linalg.norm(HX - Xa @ T), veff

    rg, resid, veff = ritz_and_resid(Xg)
    rr, _, _ = ritz_and_resid(Xref)
    assert resid <= 1.01 * r.grad_norm / (2 * spec.f) + 1e-12
    assert np.max(np.abs(rg - rr)) <= 1e-7
    # lowest p + 3 eigenvalues of H(rho(X_gpu)) by Lanczos (scipy eigsh, ARPACK)
    op = spla.LinearOperator((orc.n, orc.n), dtype=float,
                             matmat=lambda V: orc.hamiltonian_apply(V, veff),
                             matvec=lambda v: orc.hamiltonian_apply(v.reshape(-1, 1), veff).ravel())
    w = np.sort(spla.eigsh(op, k=Xg.shape[1] + 3, which="SA", tol=1e-12)[0])
    for lam in rg:
        assert np.min(np.abs(w - lam)) <= 1e-6


def test_minimize_stop_rules():
    K = ks()
    spec = spec_small(p=3, seed=40)
    sysg = K.system_from_spec(spec)
    X0 = synth.make_x0(spec, 1)
    X = dev(X0)
    r = sysg.ks_minimize(X, K.ks_default_params(max_iter=5, stagnation_tol=0.0))
    assert r.code == K.KS_E_NOT_CONVERGED and r.iters == 5 and r.stop_reason == K.KS_STOP_MAXIT
    X = dev(X0)
    r = sysg.ks_minimize(X, K.ks_default_params(eps_g=1e6))
    assert r.code == K.KS_OK and r.iters == 0 and r.stop_reason == K.KS_STOP_GRAD
    assert torch.equal(X, dev(X0))
    X = dev(X0)
    r = sysg.ks_minimize(X, K.ks_default_params(eps_g=0.0, stagnation_tol=1e-13, max_iter=5000))
    assert r.stop_reason == K.KS_STOP_STAGNATION


def test_minimize_forced_line_search_exhaustion():
    """rho_1 close to 1 makes Armijo fail; after h_max reductions the trial is accepted."""
    K = ks()
    spec = spec_small(p=3, seed=41)
    sysg = K.system_from_spec(spec)
    X = dev(synth.make_x0(spec, 1))
    r = sysg.ks_minimize(X, K.ks_default_params(rho1=0.999999, h_max=2, max_iter=6,
                                                stagnation_tol=0.0))
    assert r.iters == 6 and r.backtracks >= 2


# ------------------------------------------------------------------------------------------
# FP32 storage mode: X, G, D stored in float, every product accumulated in FP64
# ------------------------------------------------------------------------------------------

def devf(a):
    return torch.tensor(np.ascontiguousarray(a), dtype=torch.float32, device="cuda")


@pytest.mark.parametrize("p", [6, 100])
def test_fp32_energy_grad_matches_oracle_on_rounded_input(p):
    """Energies are computed in FP64 from the FP32 data, so they match the oracle applied to
    the FP32-rounded X to FP64 accuracy; G and grad E are rounded to FP32 on store.  p = 100
    takes the wide Gram and combine kernels in FP32 storage."""
    K = ks()
    spec = spec_small(p=p, seed=50)
    X = synth.make_x0(spec, 4).astype(np.float32)
    Xd = X.astype(np.float64)
    sysg = K.system_from_spec(spec, precision=K.KS_PREC_FP32)
    G = torch.zeros((spec.n, spec.p), dtype=torch.float32, device="cuda")
    D = torch.zeros_like(G)
    e = sysg.ks_energy_grad(devf(X), G, D)
    orc = oracle_fd(spec)
    en, Gr, _ = orc.energy_grad(Xd)
    Dr = stiefel.manifold_grad(Xd, Gr)
    for t in TERMS:
        a, b = getattr(e, t), float(getattr(en, t))
        assert abs(a - b) <= 1e-10 * max(abs(b), 1e-3), (t, a, b)
    assert np.max(np.abs(host(G) - Gr)) <= 2e-7 * np.max(np.abs(Gr))
    # D is formed in FP64 from the FP32 G (already rounded) and rounded once more
    assert np.max(np.abs(host(D) - Dr)) <= 5e-7 * np.max(np.abs(Gr))
    assert abs(e.orth_error - stiefel.orth_error(Xd)) < 1e-12


@pytest.mark.parametrize("kind", ["qr", "wy"])
@pytest.mark.parametrize("p", [5, 100])
def test_fp32_retract_matches_oracle_on_rounded_input(kind, p):
    K = ks()
    spec = spec_small(p=p, seed=51)
    X = synth.make_x0(spec, 5).astype(np.float32)
    orc = oracle_fd(spec)
    _, G, _ = orc.energy_grad(X.astype(np.float64))
    G = G.astype(np.float32)
    sysg = K.system_from_spec(spec, precision=K.KS_PREC_FP32)
    out = torch.zeros((spec.n, spec.p), dtype=torch.float32, device="cuda")
    tau = 0.05
    sysg.ks_retract(devf(X), devf(G), tau, K.KS_QR if kind == "qr" else K.KS_WY, out)
    Xd, Gd = X.astype(np.float64), G.astype(np.float64)
    ref = stiefel.retract_qr(Xd, Gd, tau) if kind == "qr" else stiefel.retract_wy(Xd, Gd, tau)
    assert np.max(np.abs(host(out) - ref)) <= 2e-7 * np.max(np.abs(ref))


def test_fp32_wide_p_first_steps_track_oracle():
    """FP32 storage at p = 100 (wide kernels, X^T D as a Gram pass of the stored D): four
    steps of Alg. 3 from the float-rounded start stay within the float rounding of the FP64
    oracle's four steps (each retraction rounds X to float: ~6e-8 relative)."""
    K = ks()
    spec = synth.make_system(14, 13, 12, 0.6, 100, 8, seed=6, zrange=(2, 4), margin=1.5,
                             min_spacing=1.0)
    X0 = synth.make_x0(spec, 7).astype(np.float32)
    sysg = K.system_from_spec(spec, hartree_solver=K.KS_HARTREE_PCG_FD,
                              precision=K.KS_PREC_FP32)
    X = devf(X0)
    r = sysg.ks_minimize(X, K.ks_default_params(eps_g=1e-12, stagnation_tol=0.0, max_iter=4))
    orc = oracle_fd(spec)
    ref = optm.minimize(orc.energy_grad, X0.astype(np.float64),
                        optm.Params(eps_g=1e-12, stagnation_tol=0.0, max_iter=4))
    assert r.iters == ref.iters == 4
    assert abs(r.energy - ref.E) <= 1e-7 * abs(ref.E)
    assert abs(r.grad_norm - ref.gnorm) <= 1e-6 * ref.gnorm
    assert np.max(np.abs(host(X) - ref.X)) <= 1e-5
    assert r.terms.orth_error < 1e-5


def test_fp32_minimize_reaches_fp64_energy():
    """The FP32-storage run ends within 1e-6 Ha of the FP64 oracle minimum."""
    K = ks()
    spec = synth.make_system(12, 12, 12, 0.6, 4, 2, seed=0, zrange=(2, 3), margin=2.0,
                             min_spacing=1.0)
    X0 = synth.make_x0(spec, 1)
    sysg = K.system_from_spec(spec, precision=K.KS_PREC_FP32, hartree_solver=K.KS_HARTREE_PCG_FD)
    X = devf(X0)
    r = sysg.ks_minimize(X, K.ks_default_params(max_iter=4000))
    orc = oracle_fd(spec)
    ref = optm.minimize(orc.energy_grad, X0, optm.Params(eps_g=1e-8, stagnation_tol=0.0,
                                                         max_iter=4000))
    assert r.stop_reason in (K.KS_STOP_GRAD, K.KS_STOP_STAGNATION)
    assert abs(r.energy - ref.E) <= 1e-6
    assert r.terms.orth_error < 1e-5


def test_minimize_c2_matches_oracle_reference():
    """Config c2 (64^3, p = 32, 16 nuclei, FP64) with the Section 4.1 stopping rules.  Both
    runs stop by the stagnation test at ||grad E|| ~ 5e-5, where the energy is fixed only
    to about ||grad E||^2 / curvature: the stopped energies agree to 1e-9 relative.  The
    1e-10 bar is held by the tighter run below."""
    K = ks()
    gold = _golden("oracle_c2_s0_qr.txt")
    if gold is None:
        pytest.skip("oracle reference for c2 not generated")
    spec = synth.make_config("c2", 0)
    sysg = K.system_from_spec(spec, hartree_solver=K.KS_HARTREE_PCG_FD)
    X = dev(synth.make_x0(spec, 0))
    r = sysg.ks_minimize(X, K.ks_default_params())
    assert r.stop_reason in (K.KS_STOP_GRAD, K.KS_STOP_STAGNATION)
    assert abs(r.energy - gold["E"]) <= 1e-9 * abs(gold["E"])
    assert r.terms.orth_error < 1e-12


def test_minimize_c2_matches_tight_oracle_reference():
    """Config c2 run further (||grad E|| <= 5e-6, stagnation test at 1e-16) on both sides:
    the energies agree to 1e-10 relative."""
    K = ks()
    gold = _golden("oracle_c2_s0_qr_tight.txt")
    if gold is None:
        pytest.skip("tight oracle reference for c2 not generated")
    spec = synth.make_config("c2", 0)
    sysg = K.system_from_spec(spec, hartree_solver=K.KS_HARTREE_PCG_FD)
    X = dev(synth.make_x0(spec, 0))
    r = sysg.ks_minimize(X, K.ks_default_params(eps_g=5e-6, stagnation_tol=1e-16,
                                                max_iter=20000))
    assert r.stop_reason in (K.KS_STOP_GRAD, K.KS_STOP_STAGNATION)
    assert abs(r.energy - gold["E"]) <= 1e-10 * abs(gold["E"])
    assert r.terms.orth_error < 1e-12

def test_c2_occupied_subspace_gap_gated():
    """The c2 occupied subspace (Section 2.3, eq. (disKS)), gated by the spectral gap.  The
    oracle reference (tests/golden/oracle_c2_s0_subspace.txt) stops at ||grad E|| = 3.5e-6
    and stores the gap lambda_(p+1) - lambda_p = 8.9e-4 Ha of H(rho*), the Ritz values of
    X^T H X and V^T X X^T V for two seeded unit vectors V.  By the Davis-Kahan sin-theta
    theorem a block with residual R = H X - X (X^T H X) spans the invariant subspace P* to
    ||sin theta||_F <= ||R||_F / (gap - ||R||_F), and ||X X^T - P*||_F = sqrt(2) of that.
    At the oracle's stop that is ~1e-3, so the GPU runs on to ||grad E|| <= 1e-9, where the
    bound falls below the 1e-6 of ||X X^T - Y Y^T||_F; against the oracle:
    * the energy to 1e-10 relative (second order in the subspace error on both sides);
    * V^T (P_gpu - P_oracle) V: for unit V drawn independently of the problem each entry
      has spread ||P_gpu - P_oracle||_F / n, so it stays within 5 sqrt(2) (||R_gpu||_F +
      ||R_oracle||_F) / (gap n), with ||R_oracle||_F = ||grad E|| / (2 f) from the stored
      gradient norm;
    * the Ritz values to 1e-5: each lies within its run's residual of an eigenvalue of its
      own H(rho), and the two densities differ at first order in the oracle's subspace error
      (measured 3e-6)."""
    K = ks()
    gold = _golden("oracle_c2_s0_subspace.txt")
    if gold is None:
        pytest.skip("c2 subspace reference not generated")
    spec = synth.make_config("c2", 0)
    p, n = spec.p, spec.n
    sysg = K.system_from_spec(spec, hartree_solver=K.KS_HARTREE_PCG_FD, hartree_tol=1e-14)
    X = dev(synth.make_x0(spec, 0))
    r = sysg.ks_minimize(X, K.ks_default_params(eps_g=1e-9, stagnation_tol=0.0,
                                                max_iter=20000), check=False)
    Y = torch.empty_like(X)
    sysg.ks_apply_hamiltonian(X, Y)
    sysg.close()
    Xh, Yh = host(X), host(Y)
    T = Xh.T @ Yh
    T = 0.5 * (T + T.T)
    theta = np.linalg.eigvalsh(T)
    R = np.linalg.norm(Yh - Xh @ T)
    gap = gold["gap"]
    dk = R / (gap - R)
    V = np.random.default_rng(123).standard_normal((n, 2))
    V /= np.linalg.norm(V, axis=0)
    XV = Xh.T @ V
    vpv = XV.T @ XV
    vpv_o = np.array([[gold["vpv_00"], gold["vpv_01"]], [gold["vpv_10"], gold["vpv_11"]]])
    ritz_o = np.array([gold[f"ritz_{i}"] for i in range(p)])
    r_orc = gold["gnorm"] / (2 * spec.f)
    vbar = 5 * math.sqrt(2) * (R + r_orc) / (gap * n)
    print(f"c2 subspace: {r.iters} it, |grad| {r.grad_norm:.2e}, ||R||_F {R:.2e}, "
          f"Davis-Kahan ||sin theta||_F <= {dk:.2e}; dE {r.energy - gold['E']:.2e}; "
          f"max dRitz {np.max(np.abs(theta - ritz_o)):.2e}; max dVPV "
          f"{np.max(np.abs(vpv - vpv_o)):.2e} (bar {vbar:.2e})", flush=True)
    assert r.stop_reason == K.KS_STOP_GRAD
    assert math.sqrt(2) * dk <= 1e-6
    assert abs(r.energy - gold["E"]) <= 1e-10 * abs(gold["E"])
    assert np.max(np.abs(vpv - vpv_o)) <= vbar
    assert np.max(np.abs(theta - ritz_o)) <= 1e-5
    assert r.terms.orth_error < 1e-12


@pytest.mark.parametrize("p", [80, 130])
def test_bf16_gram_matches_rounded_oracle(p):
    """KS_PREC_MIXED_BF16 forms A^T B (X^T G) of blocks wider than 64 columns on the bf16
    matrix cores; A^T A and B^T B stay as in FP32 storage (exact products, FP64 sums).
    Against the exact FP64 Gram of the bf16-rounded operands the only
    difference is the fp32 accumulation of each wavefront's rows: at most m fp32 roundings
    of a partial sum bounded by sum |a b|, m <= 1024 rows per chain at every size the
    library chunks, so |err| <= (m + 16) 2^-24 (|A|^T |B|) elementwise.  Ragged p (two and
    three 64-column sub-blocks) and a row count that is not a multiple of 16."""
    from oracle import precision
    K = ks()
    spec = spec_small(13, 11, 10, p=p, seed=70 + p)
    sysg = K.system_from_spec(spec, precision=K.KS_PREC_MIXED_BF16)
    rng = np.random.default_rng(p)
    A = rng.standard_normal((spec.n, p)).astype(np.float32)
    B = rng.standard_normal((spec.n, p)).astype(np.float32)
    out = torch.zeros(3 * p * p, dtype=torch.float64, device="cuda")
    sysg.ks_gram(devf(A), devf(B), out)
    got = host(out).reshape(3, p, p)
    ref = precision.gram_blocks_bf16(A, B)
    Ar, Br = np.abs(precision.round_bf16(A)), np.abs(precision.round_bf16(B))
    bound = ((1024 + 16) * 2.0**-24) * np.stack([Ar.T @ Ar, Ar.T @ Br, Br.T @ Br])
    A64, B64 = A.astype(np.float64), B.astype(np.float64)
    f32ref = np.stack([A64.T @ A64, A64.T @ B64, B64.T @ B64])
    assert np.all(np.abs(got[1] - ref[1]) <= bound[1])
    # the operands were rounded: the float products differ by far more than the bound
    assert np.mean(np.abs(got[1] - ref[1])) < 1e-2 * np.mean(np.abs(got[1] - f32ref[1]))
    # A^T A and B^T B from the float operands, summed in FP64
    for k in (0, 2):
        assert np.max(np.abs(got[k] - f32ref[k])) <= 1e-12 * np.max(np.abs(f32ref[k]))
    sysg.close()
