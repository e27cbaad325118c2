"""Pins of the LDA correlation in the oracle (Perdew-Zunger 1981 parametrisation of the
Ceperley-Alder unpolarised electron gas; the functional of Section 2.1 eq. (EKS) with the
"LDA" of Section 4).  They check what the functional fixes, not a retyped formula:

* v_c is the density derivative of rho eps_c (central differences in rho, both branches);
* the two branches meet at r_s = 1 (to the rounding of the published constants);
* the high-density branch tends to A ln r_s + B as r_s -> 0;
* the low-density branch decays like gamma/(beta2 r_s), and rho = 0 gives no energy;
* in a KS energy, turning correlation on adds exactly h^3 sum rho eps_c, and the gradient
  E_X still matches central differences of the total energy.
"""
import math

import numpy as np

from oracle import ks as oks
from paper_1308_2864_amd import synth
from tests.helpers import oracle_fd


def test_vc_is_the_density_derivative_of_rho_eps_c():
    for rho in (1e-6, 1e-3, 0.05, 0.2387, 0.25, 1.0, 40.0):
        h = 1e-6 * rho
        f = lambda r: r * oks.KSSystemFD.eps_c(np.array([r]))[0]
        fd = (f(rho + h) - f(rho - h)) / (2 * h)
        vc = oks.KSSystemFD.v_c(np.array([rho]))[0]
        assert abs(fd - vc) <= 1e-7 * abs(vc), (rho, fd, vc)


def test_branches_meet_at_rs_one():
    lo = oks.eps_c_rs(np.array([1.0 - 1e-12]))[0]
    hi = oks.eps_c_rs(np.array([1.0]))[0]
    assert abs(lo - hi) < 5e-5
    vlo = oks.v_c_rs(np.array([1.0 - 1e-12]))[0]
    vhi = oks.v_c_rs(np.array([1.0]))[0]
    assert abs(vlo - vhi) < 5e-5
    # the value itself is the electron-gas correlation energy at r_s = 1 (about -0.06 Ha)
    assert -0.0600 < hi < -0.0592


def test_high_density_limit():
    for rs in (1e-4, 1e-6, 1e-8):
        e = oks.eps_c_rs(np.array([rs]))[0]
        lead = oks.PZ_A * math.log(rs) + oks.PZ_B
        assert abs(e - lead) <= 0.02 * rs * abs(math.log(rs)) + 0.02 * rs


def test_low_density_decay_and_zero_density():
    for rs in (1e4, 1e6):
        e = oks.eps_c_rs(np.array([rs]))[0]
        assert abs(e * rs * oks.PZ_BETA2 / oks.PZ_GAMMA - 1.0) < 0.05
    assert oks.KSSystemFD.eps_c(np.array([0.0]))[0] == 0.0
    assert oks.KSSystemFD.v_c(np.array([0.0]))[0] == 0.0


def _spec():
    return synth.make_system(10, 9, 8, 0.7, 3, 2, seed=3, zrange=(2, 3), margin=1.5,
                             min_spacing=1.0)


def test_correlation_energy_term_and_gradient():
    spec = _spec()
    X = synth.make_x0(spec, 0)
    a = oracle_fd(spec)
    b = oracle_fd(spec, corr=True)
    ea, rho, _, _ = a.energy_terms(X)
    eb = b.energy_terms(X)[0]
    ec = a.grid.dV * float(rho @ oks.KSSystemFD.eps_c(rho))
    assert ec < 0.0
    assert abs((eb.xc - ea.xc) - ec) <= 1e-12 * abs(ec)
    assert abs((eb.total - ea.total) - ec) <= 1e-12 * abs(eb.total)
    # E_X of the energy with correlation against central differences
    _, G, _ = b.energy_grad(X)
    rng = np.random.default_rng(4)
    for _ in range(3):
        V = rng.standard_normal(X.shape)
        eps = 1e-5
        fd = (b.energy(X + eps * V) - b.energy(X - eps * V)) / (2 * eps)
        an = float(np.sum(G * V))
        assert abs(fd - an) <= 1e-7 * abs(an)
