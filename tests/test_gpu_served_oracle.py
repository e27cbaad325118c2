"""Batched and served runs against the oracle, not only against lone GPU runs: a system of
the serving mix (16^3 grid on [-8, 8]^3, p = 6, two nuclei) converged to the Section 4.1
gradient rule inside a lockstep batch (ks_minimize_batch, next to two other systems) and as
a request of the continuous-batching server, each against the FP64 oracle's Alg. 3 run of
the same start at 1e-10 relative in energy."""
import numpy as np
import pytest

from oracle import optm
from paper_1308_2864_amd import synth
from tests.helpers import oracle_fd

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

EPS_G = 1e-7


def ks():
    from paper_1308_2864_amd import ks as _ks
    return _ks


def _spec(N=16, p=6, M=2, seed=11):
    return synth.make_system(N, N, N, 16.0 / (N + 1), p, M, seed=seed, cfg="c5",
                             lo=(-8.0,) * 3, margin=3.0, zrange=(1, 4))


@pytest.fixture(scope="module")
def reference():
    spec = _spec()
    X0 = synth.make_x0(spec, 1)
    ref = optm.minimize(oracle_fd(spec).energy_grad, X0,
                        optm.Params(eps_g=EPS_G, stagnation_tol=0.0, max_iter=6000))
    assert ref.stop == "grad"
    return spec, X0, ref


def _params(K):
    return K.ks_default_params(eps_g=EPS_G, stagnation_tol=0.0, max_iter=6000)


def test_batched_system_matches_oracle(reference):
    K = ks()
    spec, X0, ref = reference
    others = [_spec(20, 9, 3, 12), _spec(18, 4, 1, 13)]
    systems, blocks = [], []
    for sp, x in [(spec, X0)] + [(o, synth.make_x0(o, 1)) for o in others]:
        systems.append(K.system_from_spec(sp, hartree_solver=K.KS_HARTREE_PCG_FD,
                                          hartree_tol=1e-14))
        blocks.append(torch.tensor(x, dtype=torch.float64, device="cuda"))
    res, codes = K.ks_minimize_batch(systems, blocks, _params(K))
    r = res[0]
    print(f"batched: E={r.energy:.13f} ({r.iters} it) oracle E={ref.E:.13f} ({ref.iters} it)",
          flush=True)
    assert codes[0] == K.KS_OK and r.stop_reason == K.KS_STOP_GRAD
    assert abs(r.energy - ref.E) <= 1e-10 * abs(ref.E)
    for s in systems:
        s.close()


def test_served_request_matches_oracle(reference):
    K = ks()
    spec, X0, ref = reference
    desc = K.desc_from_spec(spec, hartree_solver=K.KS_HARTREE_PCG_FD, hartree_tol=1e-14)
    sv = K.KSServer(K.ks_request_bytes(desc) * 2, 4, batched=True)
    sv.ks_server_submit(7, desc, X0, _params(K), want_X=True)
    sv.ks_server_wait_idle()
    done = {c["id"]: c for c in sv.ks_server_poll()}
    sv.close()
    c = done[7]
    r = c["result"]
    print(f"served: E={r.energy:.13f} ({r.iters} it) oracle E={ref.E:.13f}", flush=True)
    assert c["status"] == K.KS_OK and r.stop_reason == K.KS_STOP_GRAD
    assert abs(r.energy - ref.E) <= 1e-10 * abs(ref.E)
    # the returned block spans the oracle's occupied subspace up to the convergence level
    X = np.asarray(c["X"], dtype=np.float64)
    assert np.linalg.norm(X.T @ X - np.eye(spec.p)) < 1e-12
