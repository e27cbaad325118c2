"""Pins of the oracle's Alg. 4 with uniform refinement (oracle/refine.py) against what the
mathematics fixes:

* nested Q1 spaces: the prolongation of a coarse block is the same finite-element
  function, so its mass and stiffness Gram matrices X^T B X and X^T A X are unchanged on
  the fine mesh (a wrong weight, index or boundary treatment changes them);
* nested grids: coarse node i sits at fine node 2i + 1 (the same point of the box);
* on the 7-point grid, the carried-over lowest box mode is orthonormal and its Rayleigh
  quotient lies within the O(h^2) discretisation gap of the fine lowest eigenvalue;
* Alg. 4 ends where a direct solve on the finest level ends (the orbital-free ground state
  is unique), in fewer finest-level iterations.
"""
import math

import numpy as np

from oracle import fe, optm, refine, stiefel
from paper_1308_2864_amd import synth
from tests.helpers import oracle_fd


def test_q1_prolongation_is_the_same_function():
    nx, ny, nz, h, p = 5, 4, 6, 0.7, 3
    rng = np.random.default_rng(11)
    Xc = rng.standard_normal((nx * ny * nz, p))
    Xf = refine.prolong(Xc, nx, ny, nz)
    Ac, Bc = fe.q1_matrices(nx, ny, nz, h)
    Af, Bf = fe.q1_matrices(2 * nx + 1, 2 * ny + 1, 2 * nz + 1, h / 2)
    for Mc, Mf in ((Bc, Bf), (Ac, Af)):
        gc = Xc.T @ (Mc @ Xc)
        gf = Xf.T @ (Mf @ Xf)
        assert np.max(np.abs(gf - gc)) <= 1e-12 * np.max(np.abs(gc))


def test_nested_nodes_coincide():
    spec = synth.make_system(6, 5, 4, 0.8, 2, 1, seed=0)
    fine = synth.refine_spec(spec)
    assert refine.refine_check(spec, fine)
    lo = np.array(spec.lo)
    for i, j, k in ((0, 0, 0), (5, 4, 3), (2, 3, 1)):
        pc = lo + (np.array([i, j, k]) + 1) * spec.h
        pf = lo + (2 * np.array([i, j, k]) + 2) * fine.h
        assert np.allclose(pc, pf, rtol=0, atol=1e-14)
    Xc = np.random.default_rng(1).standard_normal((spec.n, 2))
    Xf = refine.prolong(Xc, spec.nx, spec.ny, spec.nz).reshape(fine.nz, fine.ny, fine.nx, 2)
    assert np.array_equal(Xf[1::2, 1::2, 1::2], Xc.reshape(spec.nz, spec.ny, spec.nx, 2))


def test_fd_carry_over_of_the_box_ground_state():
    N, h = 7, 1.0
    spec = synth.make_system(N, N, N, h, 1, 0, seed=0).copy(ext=False, hartree=False, xc=False)
    k = np.arange(1, N + 1)
    s1 = np.sin(k * math.pi / (N + 1))
    x = np.einsum("k,j,i->kji", s1, s1, s1).reshape(-1, 1)
    x /= np.linalg.norm(x)
    fine = synth.refine_spec(spec)
    xf = refine.carry_over(x, spec, "fd7")
    assert stiefel.orth_error(xf) < 1e-14
    orc = oracle_fd(fine)
    lam_f = 3 * (2 - 2 * math.cos(math.pi / (fine.nx + 1))) / fine.h ** 2
    lam_c = 3 * (2 - 2 * math.cos(math.pi / (N + 1))) / h ** 2
    rq = float(xf[:, 0] @ orc.hamiltonian_apply(xf, np.zeros(fine.n))[:, 0]) * 2.0
    assert lam_f < rq < lam_f + 2 * abs(lam_c - lam_f)


def test_levels_end_at_the_direct_solution():
    specs = synth.refine_levels(synth.make_ofdft(1, 4, margin=2.5, disc="fd7"), 3)
    assert [s.nx for s in specs] == [4, 9, 19]
    systems = [oracle_fd(s) for s in specs]
    prm = optm.Params(eps_g=1e-8, stagnation_tol=0.0, max_iter=3000)
    x0 = synth.make_atomic_guess(specs[0])
    res = refine.solve_levels(systems, specs, x0 / np.linalg.norm(x0), prm)
    assert all(r.stop == "grad" for r in res)
    xd = synth.make_atomic_guess(specs[-1])
    direct = optm.minimize(systems[-1].energy_grad, xd / np.linalg.norm(xd), prm)
    assert direct.stop == "grad"
    assert abs(res[-1].E - direct.E) <= 1e-10 * abs(direct.E)
    assert res[-1].iters < direct.iters
    # energies decrease with refinement toward the converged value here
    assert np.all(np.abs(res[-1].X[:, 0]) > 0)
