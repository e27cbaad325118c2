"""Pins of the orbital-free (TFW) parts of the oracle (Section 2.2 eqs. (TFW), (OFeng),
(OFinf); the GNH pseudopotential of Section 4.2), against what the physics fixes:

* GNH: far from the nucleus the potential is the Coulomb attraction -Z/r (the printed
  integrand then has closed forms), at r = 0 it is the finite integral with sinc = 1, it is
  linear in Z, and the quadrature is converged (doubling the panels changes nothing);
* Thomas-Fermi: C_TF rho^{2/3} is 3/5 of the Fermi energy (1/2)(3 pi^2 rho)^{2/3} of the
  uniform electron gas, and v_TF is the density derivative of rho eps_TF;
* von Weizsaecker: for rho = N phi^2 with phi a trilinear finite-element function,
  (1/8) int |grad rho|^2 / rho by element-wise Gauss quadrature equals (N/2) c^T A c, the
  kinetic term of the solver with occupation N (the reading that makes the orbital-free
  model the p = 1 case of the orbital minimisation);
* the converged TFW ground state solves the discrete Euler equation H phi = lambda phi and
  is of one sign, as the ground state of eq. (OF_euler) must be.
"""
import itertools
import math

import numpy as np
import pytest

from oracle import fe, gnh, optm
from oracle import ks as oks
from paper_1308_2864_amd import synth
from tests.helpers import oracle_fd


def test_gnh_far_field_origin_linearity_and_quadrature():
    Z = 3.0
    r = np.array([16.0, 20.0, 30.0])
    assert np.max(np.abs(gnh.gnh_radial(r, Z) + Z / r)) < 5e-12
    # r = 0 with the sinc factor 1: the plain integral of the bracket
    t, w = gnh._nodes()
    f = ((Z - gnh.GNH_A * gnh.GNH_RP) * np.cos(gnh.GNH_RP * t)
         + gnh.GNH_A * np.sin(gnh.GNH_RP * t) / t) * np.exp(-(t / gnh.GNH_RC) ** 6)
    assert abs(gnh.gnh_radial(np.array([0.0]), Z)[0] + (2 / math.pi) * float(f @ w)) < 1e-14
    assert np.isfinite(gnh.gnh_radial(np.array([0.0, 1e-9]), Z)).all()
    rr = np.linspace(0.0, 12.0, 41)
    v1, v2, v3 = (gnh.gnh_radial(rr, z) for z in (1.0, 2.0, 3.0))
    assert np.max(np.abs((v3 - v2) - (v2 - v1))) < 1e-13
    # converged: twice the panels and nodes
    fine = gnh.gnh_radial(rr, Z, panels=256, per=48)
    assert np.max(np.abs(fine - v3)) < 1e-13
    # an attractive well outside the core, repulsive at the nucleus
    assert v3[rr.searchsorted(2.0)] < -1.0 and v3[0] > 0.0


def test_thomas_fermi_is_three_fifths_of_the_fermi_energy():
    for rho in (1e-4, 0.01, 0.3, 2.0):
        ef = 0.5 * (3 * math.pi ** 2 * rho) ** (2.0 / 3.0)
        assert abs(oks.C_TF * rho ** (2.0 / 3.0) - 0.6 * ef) <= 1e-14 * ef
        e = lambda x: oks.C_TF * x ** (5.0 / 3.0)
        dr = 1e-6 * rho
        assert abs((e(rho + dr) - e(rho - dr)) / (2 * dr)
                   - (5.0 / 3.0) * oks.C_TF * rho ** (2.0 / 3.0)) <= 1e-8 * rho ** (2.0 / 3.0)


def test_von_weizsaecker_of_rho_equals_the_kinetic_term_with_occupation_n():
    nx, ny, nz, h, N = 4, 3, 3, 0.7, 42.0
    A, _ = fe.q1_matrices(nx, ny, nz, h)
    rng = np.random.default_rng(3)
    c = 0.5 + rng.random(nx * ny * nz)  # a positive phi (rho > 0 inside)
    fx, fy, fz = nx + 2, ny + 2, nz + 2
    full = np.zeros((fz, fy, fx))
    full[1:-1, 1:-1, 1:-1] = c.reshape(nz, ny, nx)
    gp = [0.5 - 0.5 / math.sqrt(3.0), 0.5 + 0.5 / math.sqrt(3.0)]
    total = 0.0
    for ez, ey, ex in itertools.product(range(fz - 1), range(fy - 1), range(fx - 1)):
        cc = full[ez:ez + 2, ey:ey + 2, ex:ex + 2]
        for s, t, u in itertools.product(gp, gp, gp):
            ws = np.array([1 - s, s]), np.array([1 - t, t]), np.array([1 - u, u])
            ds = np.array([-1.0, 1.0]) / h
            phi = np.einsum("kji,k,j,i->", cc, ws[2], ws[1], ws[0])
            grad = np.array([np.einsum("kji,k,j,i->", cc, ws[2], ws[1], ds),
                             np.einsum("kji,k,j,i->", cc, ws[2], ds, ws[0]),
                             np.einsum("kji,k,j,i->", cc, ds, ws[1], ws[0])])
            if phi <= 0.0:
                continue  # boundary cells where phi vanishes contribute |grad phi|^2 below
            rho = N * phi ** 2
            grho = 2.0 * N * phi * grad
            total += (h ** 3 / 8.0) * float(grho @ grho) / rho / 8.0
    assert abs(total - 0.5 * N * float(c @ (A @ c))) <= 1e-12 * total


def test_tfw_ground_state_solves_the_euler_equation_and_has_one_sign():
    """Al14 (one fcc cell) on the 7-point grid, h = 0.698: Alg. 3 on the unit sphere reaches
    a stationary point of E_OF that is an eigenvector of its own Hamiltonian and has no
    node, i.e. the ground state of eq. (OF_euler)."""
    spec = synth.make_ofdft(1, 17, margin=2.5, disc="fd7")
    orc = oracle_fd(spec)
    X0 = synth.make_atomic_guess(spec)
    X0 = X0 / np.linalg.norm(X0)
    res = optm.minimize(orc.energy_grad, X0, optm.Params(eps_g=1e-8, stagnation_tol=0.0,
                                                         max_iter=2000))
    assert res.stop == "grad"
    x = res.X[:, 0]
    veff = orc.effective_potential(res.X)
    Hx = orc.hamiltonian_apply(res.X, veff)[:, 0]
    lam = float(x @ Hx)
    assert np.linalg.norm(Hx - lam * x) <= 1e-8
    assert np.all(x > 0) or np.all(x < 0)
    # the total charge is the number of valence electrons
    rho = orc.density(res.X)
    assert abs(spec.h ** 3 * rho.sum() - 42.0) < 1e-10
