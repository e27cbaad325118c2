"""Pins of the finite-element (Q1, B-metric) oracle.

Each test checks the oracle against something other than itself: an element-by-element
assembly with Gauss quadrature, the closed-form generalized eigenvalues of the tensor
product matrices, an eigen-decomposition by sine transforms, the Euclidean oracle run on
the transformed variables Y = B^{1/2} X, finite differences, and a dense generalized
eigensolver at the minimiser.
"""
import itertools
import math

import numpy as np
import pytest
import scipy.fft
import scipy.linalg as sla

from oracle import optm
from oracle.fe import (BStiefel, KSSystemQ1, b_orthonormalize, q1_generalized_eigenvalues,
                       q1_matrices)
from paper_1308_2864_amd import synth
from tests.helpers import oracle_q1


def _element_assembly(nx, ny, nz, h):
    """Dense A, B by looping over the cubes of the full mesh (interior + boundary nodes)
    with the trilinear shape functions and 2-point Gauss quadrature per axis (exact for
    these polynomial integrands), then dropping the boundary rows and columns."""
    fx, fy, fz = nx + 2, ny + 2, nz + 2
    N = fx * fy * fz
    A = np.zeros((N, N))
    B = np.zeros((N, N))
    gp = [0.5 - 0.5 / math.sqrt(3.0), 0.5 + 0.5 / math.sqrt(3.0)]
    corners = list(itertools.product((0, 1), repeat=3))  # (cx, cy, cz)

    def shape(c, s, t, u):
        vals = [(1 - s) if c[0] == 0 else s, (1 - t) if c[1] == 0 else t,
                (1 - u) if c[2] == 0 else u]
        ds = [(-1.0 if c[0] == 0 else 1.0), (-1.0 if c[1] == 0 else 1.0),
              (-1.0 if c[2] == 0 else 1.0)]
        phi = vals[0] * vals[1] * vals[2]
        grad = np.array([ds[0] * vals[1] * vals[2], vals[0] * ds[1] * vals[2],
                         vals[0] * vals[1] * ds[2]]) / h
        return phi, grad

    for ez, ey, ex in itertools.product(range(fz - 1), range(fy - 1), range(fx - 1)):
        idx = [(ex + c[0]) + fx * ((ey + c[1]) + fy * (ez + c[2])) for c in corners]
        for s, t, u in itertools.product(gp, gp, gp):
            w = (h ** 3) / 8.0
            ev = [shape(c, s, t, u) for c in corners]
            for a in range(8):
                for b in range(8):
                    B[idx[a], idx[b]] += w * ev[a][0] * ev[b][0]
                    A[idx[a], idx[b]] += w * float(ev[a][1] @ ev[b][1])
    inner = [i + fx * (j + fy * k) for k in range(1, nz + 1) for j in range(1, ny + 1)
             for i in range(1, nx + 1)]
    return A[np.ix_(inner, inner)], B[np.ix_(inner, inner)]


def test_q1_matrices_match_element_assembly():
    nx, ny, nz, h = 3, 4, 2, 0.7
    A, B = q1_matrices(nx, ny, nz, h)
    Ae, Be = _element_assembly(nx, ny, nz, h)
    assert np.max(np.abs(A.toarray() - Ae)) < 1e-13 * np.max(np.abs(Ae))
    assert np.max(np.abs(B.toarray() - Be)) < 1e-13 * np.max(np.abs(Be))
    # 27-point stencils.  On the uniform cube mesh the face couplings of A cancel exactly
    # (-16h/36 + 2 * 8h/36), leaving centre 8h/3, edges -h/6 and corners -h/12; B has
    # centre 8h^3/27, faces 2h^3/27, edges h^3/54 and corners h^3/216.
    A2, B2 = q1_matrices(5, 5, 5, h)
    mid = 2 + 5 * (2 + 5 * 2)
    assert A2[mid].nnz == 21 and B2[mid].nnz == 27
    ra, rb = A2[mid].toarray().reshape(5, 5, 5)[1:4, 1:4, 1:4], \
        B2[mid].toarray().reshape(5, 5, 5)[1:4, 1:4, 1:4]
    for (c, e, f) in itertools.product(range(3), repeat=3):
        k = abs(c - 1) + abs(e - 1) + abs(f - 1)
        assert abs(ra[c, e, f] - [8 * h / 3, 0.0, -h / 6, -h / 12][k]) < 1e-14
        assert abs(rb[c, e, f] - [8 * h ** 3 / 27, 2 * h ** 3 / 27, h ** 3 / 54,
                                  h ** 3 / 216][k]) < 1e-15


def test_q1_generalized_eigenvalues_closed_form():
    nx, ny, nz, h = 5, 4, 3, 0.4
    A, B = q1_matrices(nx, ny, nz, h)
    w = sla.eigh(A.toarray(), B.toarray(), eigvals_only=True)
    ref = np.sort(q1_generalized_eigenvalues(nx, ny, nz, h))
    assert np.max(np.abs(w - ref)) < 1e-11 * ref.max()


def _sine_basis(m):
    """Orthonormal DST-I matrix and the eigenvalues of K and M on m interior nodes."""
    j = np.arange(1, m + 1)
    S = math.sqrt(2.0 / (m + 1)) * np.sin(np.outer(j, j) * math.pi / (m + 1))
    return S


def test_mass_solve_and_hartree_match_sine_diagonalisation():
    """B^{-1} and A^{-1} in the sine basis: B = S3 diag(mu x mu x mu) S3 and
    A = S3 diag(lk mu mu + mu lk mu + mu mu lk) S3 with 1D eigenvalues
    lk = (2/h)(1 - cos t), mu = (h/3)(2 + cos t)."""
    nx, ny, nz, h = 7, 6, 5, 0.45
    spec = synth.make_system(nx, ny, nz, h, 2, 2, seed=3, zrange=(1, 2), min_spacing=0.5,
                             margin=0.8)
    sysk = oracle_q1(spec)
    rng = np.random.default_rng(5)
    b = rng.standard_normal(sysk.n)

    def axis(m):
        t = np.arange(1, m + 1) * math.pi / (m + 1)
        return (2.0 / h) * (1 - np.cos(t)), (h / 3.0) * (2 + np.cos(t))

    (kx, mx), (ky, my), (kz, mz) = axis(nx), axis(ny), axis(nz)
    bh = scipy.fft.dstn(b.reshape(nz, ny, nx), type=1, norm="ortho")
    mu = mz[:, None, None] * my[None, :, None] * mx[None, None, :]
    den = (kz[:, None, None] * my[None, :, None] * mx[None, None, :]
           + mz[:, None, None] * ky[None, :, None] * mx[None, None, :]
           + mz[:, None, None] * my[None, :, None] * kx[None, None, :])
    binv = scipy.fft.idstn(bh / mu, type=1, norm="ortho").ravel()
    assert np.max(np.abs(sysk.mass_solve(b) - binv)) < 1e-12 * np.max(np.abs(binv))
    rho = np.abs(b)
    vh, it, rel = sysk.hartree_cg(rho)
    rhs = 4 * math.pi * h ** 3 * rho
    ref = scipy.fft.idstn(scipy.fft.dstn(rhs.reshape(nz, ny, nx), type=1, norm="ortho") / den,
                          type=1, norm="ortho").ravel()
    assert rel <= 1e-14
    assert np.max(np.abs(vh - ref)) < 1e-11 * np.max(np.abs(ref))


def test_q1_box_minimum():
    """V = 0, no Hartree, no exchange: min (f/2) tr(X^T A X) over X^T B X = I is (f/2) times
    the sum of the p smallest closed-form generalized eigenvalues."""
    nx, ny, nz, h, p = 8, 7, 6, 0.6, 4
    spec = synth.make_system(nx, ny, nz, h, p, 0, seed=1).copy(ext=False, hartree=False,
                                                                xc=False, disc="q1")
    sysk = oracle_q1(spec)
    lam = np.sort(q1_generalized_eigenvalues(nx, ny, nz, h))
    assert lam[p] - lam[p - 1] > 0.05
    expect = 0.5 * spec.f * lam[:p].sum()
    mf = BStiefel(sysk.B, sysk.mass_solve)
    X0 = b_orthonormalize(sysk.B, synth.make_x0(spec, 2))
    for kind in ("qr", "wy"):
        res = optm.minimize(sysk.energy_grad, X0, optm.Params(eps_g=1e-9, stagnation_tol=0.0,
                                                              retraction=kind, max_iter=5000),
                            manifold=mf)
        assert res.stop == "grad", kind
        assert abs(res.E - expect) < 1e-11 * expect, kind
        assert mf.orth_error(res.X) < 1e-12


def _tiny_fe(seed=2, m=6, p=2):
    spec = synth.make_system(m, m - 1, m - 1, 0.7, p, 2, seed=seed, zrange=(1, 2),
                             min_spacing=0.8, margin=0.9).copy(disc="q1")
    return spec, oracle_q1(spec)


@pytest.mark.parametrize("kind", ["qr", "wy"])
def test_b_metric_iteration_equals_euclidean_iteration_in_y(kind):
    """The B-metric formulas are Section 3 with Y = B^{1/2} X substituted: Alg. 3 run on
    E(B^{-1/2} Y) with the Euclidean oracle (dense B^{1/2} from eigh) takes the same steps
    and reaches the same energies as the B-metric oracle on X."""
    spec, sysk = _tiny_fe()
    w, V = np.linalg.eigh(sysk.B.toarray())
    Bh = (V * np.sqrt(w)) @ V.T
    Bmh = (V / np.sqrt(w)) @ V.T
    X0 = b_orthonormalize(sysk.B, synth.make_x0(spec, 4))
    prm = optm.Params(max_iter=25, retraction=kind, eps_g=0.0, stagnation_tol=0.0)

    def eg_y(Y, vh0):
        en, G, vh = sysk.energy_grad(Bmh @ Y, vh0)
        return en, Bmh @ G, vh

    rx = optm.minimize(sysk.energy_grad, X0, prm, manifold=BStiefel(sysk.B, sysk.mass_solve))
    ry = optm.minimize(eg_y, Bh @ X0, prm)
    assert rx.iters == ry.iters == 25
    for hx, hy in zip(rx.history, ry.history):
        assert abs(hx["E"] - hy["E"]) <= 1e-10 * abs(hy["E"])
        assert abs(hx["tau"] - hy["tau"]) <= 1e-6 * hy["tau"]
        assert hx["h"] == hy["h"]
    assert np.max(np.abs(rx.X - Bmh @ ry.X)) < 1e-8


def test_q1_gradient_matches_central_differences():
    spec, sysk = _tiny_fe(p=3)
    X = b_orthonormalize(sysk.B, synth.make_x0(spec, 7))
    _, G, _ = sysk.energy_grad(X)
    rng = np.random.default_rng(12)
    for _ in range(3):
        D = rng.standard_normal(X.shape)
        eps = 1e-5
        fd = (sysk.energy(X + eps * D) - sysk.energy(X - eps * D)) / (2 * eps)
        an = float(np.sum(G * D))
        assert abs(fd - an) < 1e-7 * max(1.0, abs(an))


def test_q1_converged_point_is_generalized_ks_stationary_and_aufbau():
    """At the minimiser H(rho*) X = B X Lambda, and X spans the B-orthonormal eigenvectors
    of the p smallest generalized eigenvalues of (H(rho*), B) (cosines of the principal
    angles in the B inner product all equal 1)."""
    spec, sysk = _tiny_fe(seed=2, m=6, p=2)
    mf = BStiefel(sysk.B, sysk.mass_solve)
    X0 = b_orthonormalize(sysk.B, synth.make_x0(spec, 4))
    res = optm.minimize(sysk.energy_grad, X0, optm.Params(eps_g=1e-9, stagnation_tol=0.0,
                                                          max_iter=6000), manifold=mf)
    assert res.stop == "grad"
    X = res.X
    H = sysk.hamiltonian(sysk.effective_potential(X)).toarray()
    Bd = sysk.B.toarray()
    HX = H @ X
    lam_x = X.T @ HX
    assert np.linalg.norm(HX - Bd @ X @ lam_x) < 1e-8
    w, V = sla.eigh(H, Bd)
    assert w[spec.p] - w[spec.p - 1] > 0.1
    cos = np.linalg.svd(X.T @ Bd @ V[:, :spec.p], compute_uv=False)
    assert np.min(cos) > 1 - 1e-10
    assert np.allclose(np.sort(np.linalg.eigvalsh(0.5 * (lam_x + lam_x.T))), w[:spec.p],
                       atol=1e-9)
